// HIP kernels (gfx950) of the MPO-TEBD step.
//
// Complex numbers are double2 (x = re, y = im), interleaved in memory.
// Site tensors A[l][a][r] are row-major; the two-site block theta and the
// SVD work matrix X are column-major.
#include "lmpo_internal.h"

namespace lmpo {

namespace {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ void cfma(cplx<T> &acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 dconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ void dfma(double2 &acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
__device__ __forceinline__ void dfma_cj(double2 &acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

inline void check_launch() { (void)hipGetLastError(); }

}  // namespace

// ---------------------------------------------------------------------------
// Two-site contraction with the gate (north_star steps "contract the two-site
// block" and "apply the propagator"):
//   M[(l,s),(t,r)] = sum_m A_k[l][s][m] A_{k+1}[m][t][r]
//   theta[(l,s'),(t',r)] = sum_{s,t} G[(s' t'),(s t)] M[(l,s),(t,r)]
// A workgroup owns 16 values of l and 16 of r, i.e. a 64 x 64 tile of M with
// all four s and all four t, so the 16x16 gate is applied in the epilogue
// from LDS.  T is the arithmetic type (double, or float for the FP32
// contraction form: operands rounded to FP32, FP32 accumulation).
// Output: trans = 0 -> X = theta, column-major, ld = 4 chl;
//         trans = 1 -> X = theta^H, column-major, ld = 4 chr.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void contract_body(double2 *const *sites, const int *dims, int N, int k,
                                              const double2 *__restrict__ G, double2 *__restrict__ X,
                                              const int bx, const int by) {
  using C2 = cplx<T>;
  const int chl = (k == 0) ? 1 : dims[k - 1], chm = dims[k], chr = (k + 1 == N - 1) ? 1 : dims[k + 1];
  const int trans = (4 * chl >= 4 * chr) ? 0 : 1;
  if (by * 16 >= chl || bx * 16 >= chr) return;
  const double2 *__restrict__ Ak = sites[k];
  const double2 *__restrict__ Ak1 = sites[k + 1];
  __shared__ C2 As[16][64];
  __shared__ C2 Bs[16][64];
  __shared__ C2 Ms[64][65];
  __shared__ C2 Gs[16][16];
  const int t = threadIdx.x;
  const int l0 = by * 16, r0 = bx * 16;
  const int ty = t / 16, tx = t % 16;
  const int R = 4 * chl;
  {
    double2 g = G[t];
    Gs[t / 16][t % 16] = C2{(T)g.x, (T)g.y};
  }
  C2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = C2{0, 0};
  for (int m0 = 0; m0 < chm; m0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = t + 256 * q;
      int row = e / 16, kk = e % 16;
      int gr = l0 * 4 + row, gm = m0 + kk;
      double2 v = make_double2(0, 0);
      if (gr < R && gm < chm) v = Ak[(size_t)gr * chm + gm];
      As[kk][row] = C2{(T)v.x, (T)v.y};
      int kb = e / 64, j = e % 64;
      int gmb = m0 + kb, r = r0 + (j % 16);
      double2 w = make_double2(0, 0);
      if (gmb < chm && r < chr) w = Ak1[(size_t)gmb * 4 * chr + (j / 16) * chr + r];
      Bs[kb][j] = C2{(T)w.x, (T)w.y};
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      C2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cfma(acc[i][j], a[i], b[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) Ms[ty * 4 + i][tx * 4 + j] = acc[i][j];
  __syncthreads();
  // epilogue: thread -> (l, r); 16 outputs (s', t')
  const int li = t / 16, ri = t % 16;
  const int l = l0 + li, r = r0 + ri;
  if (l >= chl || r >= chr) return;
  C2 m[16];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) m[4 * s + tt] = Ms[li * 4 + s][tt * 16 + ri];
#pragma unroll
  for (int o = 0; o < 16; ++o) {
    C2 out{0, 0};
#pragma unroll
    for (int q = 0; q < 16; ++q) cfma(out, Gs[o][q], m[q]);
    const int sp = o / 4, tp = o % 4;
    const size_t row = (size_t)l * 4 + sp, col = (size_t)tp * chr + r;
    if (trans == 0)
      X[row + col * (size_t)(4 * chl)] = make_double2((double)out.x, (double)out.y);
    else
      X[col + row * (size_t)(4 * chr)] = make_double2((double)out.x, -(double)out.y);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void contract_gate_kernel(double2 *const *sites, const int *dims, int N, int k,
                                                            const double2 *__restrict__ G,
                                                            double2 *__restrict__ X) {
  contract_body<T>(sites, dims, N, k, G, X, blockIdx.x, blockIdx.y);
}

// Batched form: job blockIdx.z of a device array of independent contractions.
template <typename T>
__global__ __launch_bounds__(256) void contract_gate_batched_kernel(const ContractJob *__restrict__ jobs) {
  const ContractJob j = jobs[blockIdx.z];
  contract_body<T>(j.sites, j.dims, j.N, j.k, j.G, j.X, blockIdx.x, blockIdx.y);
}

void launch_contract_gate(hipStream_t s, int precision, double2 *const *sites, const int *dims, int N, int k,
                          int cap_l, int cap_r, const double2 *G, double2 *X) {
  dim3 grid((cap_r + 15) / 16, (cap_l + 15) / 16);
  if (precision == LMPO_FP32_CONTRACT)
    hipLaunchKernelGGL(contract_gate_kernel<float>, grid, dim3(256), 0, s, sites, dims, N, k, G, X);
  else
    hipLaunchKernelGGL(contract_gate_kernel<double>, grid, dim3(256), 0, s, sites, dims, N, k, G, X);
  check_launch();
}

void launch_contract_batched(hipStream_t s, int precision, const ContractJob *d_jobs, int n_jobs, int cap_l,
                             int cap_r) {
  if (n_jobs <= 0) return;
  dim3 grid((cap_r + 15) / 16, (cap_l + 15) / 16, n_jobs);
  if (precision == LMPO_FP32_CONTRACT)
    hipLaunchKernelGGL(contract_gate_batched_kernel<float>, grid, dim3(256), 0, s, d_jobs);
  else
    hipLaunchKernelGGL(contract_gate_batched_kernel<double>, grid, dim3(256), 0, s, d_jobs);
  check_launch();
}

// ---------------------------------------------------------------------------
// Contractions with product covectors (trace and Pauli observables).
// In the basis P_a = sigma^a/sqrt(2): Tr(P_a) = sqrt(2) delta_{a,1} and
// Tr(sigma^b P_a) = sqrt(2) delta_{ab}, so tr(rho) is the product of the
// sqrt(2) A_i[:, 1, :] slices and <sigma^a_i> replaces slice i by index a
// (Sec. 2.3, Eqs. mu and 2Qdef; Sec. 2.4 trace).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void site_dims(const int *dims, int N, int i, int &cl, int &cr) {
  cl = (i == 0) ? 1 : dims[i - 1];
  cr = (i == N - 1) ? 1 : dims[i];
}

// v_out[r] = sqrt(2) sum_l v_in[l] A[l][a][r]  (block-wide, v in LDS)
__device__ void env_step_right(const double2 *__restrict__ A, int cl, int cr, int a, const double2 *vin,
                               double2 *vout) {
  const double s2 = 1.4142135623730951;
  for (int r = threadIdx.x; r < cr; r += blockDim.x) {
    double2 acc = make_double2(0, 0);
    const double2 *col = A + (size_t)a * cr + r;
    for (int l = 0; l < cl; ++l) dfma(acc, vin[l], col[(size_t)l * 4 * cr]);
    vout[r] = make_double2(acc.x * s2, acc.y * s2);
  }
}
// v_out[l] = sqrt(2) sum_r A[l][a][r] v_in[r]
__device__ void env_step_left(const double2 *__restrict__ A, int cl, int cr, int a, const double2 *vin,
                              double2 *vout) {
  const double s2 = 1.4142135623730951;
  for (int l = threadIdx.x; l < cl; l += blockDim.x) {
    double2 acc = make_double2(0, 0);
    const double2 *row = A + (size_t)l * 4 * cr + (size_t)a * cr;
    for (int r = 0; r < cr; ++r) dfma(acc, row[r], vin[r]);
    vout[l] = make_double2(acc.x * s2, acc.y * s2);
  }
}

__global__ __launch_bounds__(256) void trace_kernel(double2 *const *sites, const int *dims, int N,
                                                    double2 *out) {
  extern __shared__ double2 buf[];
  int cap = 1;
  for (int i = 0; i < N - 1; ++i) cap = dims[i] > cap ? dims[i] : cap;
  double2 *v0 = buf, *v1 = buf + cap;
  if (threadIdx.x == 0) v0[0] = make_double2(1.0, 0.0);
  __syncthreads();
  for (int i = 0; i < N; ++i) {
    int cl, cr;
    site_dims(dims, N, i, cl, cr);
    env_step_right(sites[i], cl, cr, 0, v0, v1);
    __syncthreads();
    double2 *tmp = v0;
    v0 = v1;
    v1 = tmp;
  }
  if (threadIdx.x == 0) out[0] = v0[0];
}

void launch_trace(hipStream_t s, double2 *const *sites, const int *dims, int N, double2 *out) {
  hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(256), 2 * kMaxDim * sizeof(double2), s, sites, dims, N, out);
  check_launch();
}

// envL[i] = contraction of sites < i with the identity covector (length chi_{i-1}),
// envR[i] = contraction of sites > i (length chi_i); stride cap.
__global__ __launch_bounds__(256) void env_all_kernel(double2 *const *sites, const int *dims, int N, int cap,
                                                      double2 *envL, double2 *envR) {
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) envL[0] = make_double2(1.0, 0.0);
    __syncthreads();
    for (int i = 0; i < N - 1; ++i) {
      int cl, cr;
      site_dims(dims, N, i, cl, cr);
      env_step_right(sites[i], cl, cr, 0, envL + (size_t)i * cap, envL + (size_t)(i + 1) * cap);
      __syncthreads();
    }
  } else {
    if (threadIdx.x == 0) envR[(size_t)(N - 1) * cap] = make_double2(1.0, 0.0);
    __syncthreads();
    for (int i = N - 1; i > 0; --i) {
      int cl, cr;
      site_dims(dims, N, i, cl, cr);
      env_step_left(sites[i], cl, cr, 0, envR + (size_t)i * cap, envR + (size_t)(i - 1) * cap);
      __syncthreads();
    }
  }
}

void launch_env_all(hipStream_t s, double2 *const *sites, const int *dims, int N, int cap, double2 *envL,
                    double2 *envR) {
  hipLaunchKernelGGL(env_all_kernel, dim3(2), dim3(256), 0, s, sites, dims, N, cap, envL, envR);
  check_launch();
}

// Request q: req[4q..4q+3] = (i, a, j, b); j < 0 for a 1Q observable.  Output
// out[q] = numerator contraction (not yet divided by the trace).
__global__ __launch_bounds__(256) void measure_kernel(double2 *const *sites, const int *dims, int N, int cap,
                                                      const double2 *__restrict__ envL,
                                                      const double2 *__restrict__ envR, const int *req,
                                                      double2 *out) {
  extern __shared__ double2 buf[];
  double2 *v0 = buf, *v1 = buf + cap;
  __shared__ double2 red[256];
  const int q = blockIdx.x;
  const int i = req[4 * q], a = req[4 * q + 1], j = req[4 * q + 2], b = req[4 * q + 3];
  int cl, cr;
  site_dims(dims, N, i, cl, cr);
  for (int l = threadIdx.x; l < cl; l += blockDim.x) v0[l] = envL[(size_t)i * cap + l];
  __syncthreads();
  env_step_right(sites[i], cl, cr, a, v0, v1);
  __syncthreads();
  int last = i;
  if (j >= 0) {
    for (int k = i + 1; k <= j; ++k) {
      double2 *tmp = v0;
      v0 = v1;
      v1 = tmp;
      int kl, kr;
      site_dims(dims, N, k, kl, kr);
      env_step_right(sites[k], kl, kr, (k == j) ? b : 0, v0, v1);
      __syncthreads();
    }
    last = j;
  }
  int ll, lr;
  site_dims(dims, N, last, ll, lr);
  double2 acc = make_double2(0, 0);
  for (int r = threadIdx.x; r < lr; r += blockDim.x) dfma(acc, v1[r], envR[(size_t)last * cap + r]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = dadd(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q] = red[0];
}

void launch_measure(hipStream_t s, double2 *const *sites, const int *dims, int N, int cap, const double2 *envL,
                    const double2 *envR, int n, const int *req, double2 *out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(measure_kernel, dim3(n), dim3(256), 2 * cap * sizeof(double2), s, sites, dims, N, cap, envL,
                     envR, req, out);
  check_launch();
}

// A_site <- A_site / tr
__global__ void scale_site_kernel(double2 *const *sites, const int *dims, int N, int site, const double2 *tr) {
  int cl, cr;
  site_dims(dims, N, site, cl, cr);
  const size_t n = (size_t)cl * 4 * cr;
  const double2 z = tr[0];
  const double d = z.x * z.x + z.y * z.y;
  const double2 inv = make_double2(z.x / d, -z.y / d);
  double2 *A = sites[site];
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    A[e] = dmul(A[e], inv);
}

void launch_scale_site(hipStream_t s, double2 *const *sites, const int *dims, int N, int site, const double2 *tr) {
  hipLaunchKernelGGL(scale_site_kernel, dim3(256), dim3(256), 0, s, sites, dims, N, site, tr);
  check_launch();
}

}  // namespace lmpo
