// HIP kernels (gfx950) of the MPO-TEBD step.
//
// Complex numbers are double2 (x = re, y = im), interleaved in memory.
// Site tensors A[l][a][r] are row-major; the two-site block theta and the
// SVD work matrix X are column-major.
#include "contract_tile.h"
#include "lmpo_internal.h"

namespace lmpo {

namespace {

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

template <typename T, bool kReal>
__global__ __launch_bounds__(256) void contract_gate_kernel(double2 *const *sites, const int *dims, int N, int k,
                                                            const double2 *__restrict__ G,
                                                            double2 *__restrict__ X) {
  __shared__ ContractLds<T> lds;
  contract_tile<T, kReal>(lds, sites, dims, N, k, G, X, blockIdx.x, blockIdx.y);
}

void launch_contract_gate(hipStream_t s, int precision, double2 *const *sites, const int *dims, int N, int k,
                          int cap_l, int cap_r, const double2 *G, double2 *X) {
  dim3 grid((cap_r + 15) / 16, (cap_l + 15) / 16);
  if (precision == LMPO_FP32_CONTRACT)
    hipLaunchKernelGGL((contract_gate_kernel<float, false>), grid, dim3(256), 0, s, sites, dims, N, k, G, X);
  else if (precision == LMPO_FP64_REAL)
    hipLaunchKernelGGL((contract_gate_kernel<double, true>), grid, dim3(256), 0, s, sites, dims, N, k, G, X);
  else
    hipLaunchKernelGGL((contract_gate_kernel<double, false>), grid, dim3(256), 0, s, sites, dims, N, k, G, X);
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
  const double2 tr = chain_trace(sites, dims, N, buf, buf + kMaxDim / 4);
  if (threadIdx.x == 0) out[0] = tr;
}

void launch_trace(hipStream_t s, double2 *const *sites, const int *dims, int N, double2 *out) {
  hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(256), 2 * (kMaxDim / 4) * sizeof(double2), s, sites, dims, N, out);
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
  const double2 inv = zinv_exact(tr[0]);
  double2 *A = sites[site];
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    A[e] = zmul_exact(A[e], inv);
}

// out[0] = sum |A_site|^2 by one workgroup (fixed summation order).
__global__ __launch_bounds__(256) void norm2_site_kernel(double2 *const *sites, const int *dims, int N, int site,
                                                         double *out) {
  __shared__ double red[256];
  int cl, cr;
  site_dims(dims, N, site, cl, cr);
  const size_t n = (size_t)cl * 4 * cr;
  const double2 *A = sites[site];
  double acc = 0.0;
  for (size_t e = threadIdx.x; e < n; e += 256) acc = fma(A[e].x, A[e].x, fma(A[e].y, A[e].y, acc));
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

void launch_norm2_site(hipStream_t s, double2 *const *sites, const int *dims, int N, int site, double *out) {
  hipLaunchKernelGGL(norm2_site_kernel, dim3(1), dim3(256), 0, s, sites, dims, N, site, out);
  check_launch();
}

void launch_scale_site(hipStream_t s, double2 *const *sites, const int *dims, int N, int site, const double2 *tr) {
  hipLaunchKernelGGL(scale_site_kernel, dim3(256), dim3(256), 0, s, sites, dims, N, site, tr);
  check_launch();
}

// ---------------------------------------------------------------------------
// Hermitian part rho -> (rho + rho^+) / 2 (the solver's force_rho_hermitian_step,
// Sec. 6).  The basis operators P_a are Hermitian, so rho^+ has the complex
// conjugate coefficients; the sum is the MPS whose site k is the direct sum of
// A_k and conj(A_k) (bond dims doubled: block diagonal inside the chain, a row
// of two blocks on the first site, a column on the last), the first site
// carrying the factor 1/2.  src is a copy of site k taken before the call;
// dims are the bond dims before doubling.
// ---------------------------------------------------------------------------
__global__ void hermitian_sum_site_kernel(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                          const int *dims, int N, int k) {
  int cl, cr;
  site_dims(dims, N, k, cl, cr);
  const bool first = (k == 0), last = (k == N - 1);
  const int nl = first ? 1 : 2 * cl, nr = last ? 1 : 2 * cr;
  const double f = first ? 0.5 : 1.0;
  const size_t n = (size_t)nl * 4 * nr;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % nr), a = (int)((e / nr) % 4), l = (int)(e / ((size_t)4 * nr));
    const int hl = first ? 0 : l / cl, hr = last ? 0 : r / cr;  // copy (0: rho, 1: rho^+) of each index
    double2 out = make_double2(0.0, 0.0);
    if (first || last || hl == hr) {
      const int copy = first ? hr : hl;
      const double2 v = src[(size_t)(l - hl * cl) * 4 * cr + (size_t)a * cr + (r - hr * cr)];
      out = make_double2(f * v.x, copy ? -f * v.y : f * v.y);
    }
    dst[e] = out;
  }
}

__global__ void double_dims_kernel(int *dims, int n) {
  for (int b = threadIdx.x; b < n; b += blockDim.x) dims[b] *= 2;
}

void launch_hermitian_sum_site(hipStream_t s, const double2 *src, double2 *dst, const int *dims, int N, int k) {
  hipLaunchKernelGGL(hermitian_sum_site_kernel, dim3(256), dim3(256), 0, s, src, dst, dims, N, k);
  check_launch();
}

void launch_double_dims(hipStream_t s, int *dims, int n) {
  hipLaunchKernelGGL(double_dims_kernel, dim3(1), dim3(64), 0, s, dims, n);
  check_launch();
}

// ---------------------------------------------------------------------------
// FP64 matrix-core throughput probe (the measured counterpart of the FP64
// peak the rooflines are quoted against): every wavefront issues `iters`
// rounds of eight independent v_mfma_f64_16x16x4f64 (16 x 16 x 4 multiply-adds,
// 2048 flops each) on register operands, enough chains to cover the
// instruction latency; one store per lane keeps the results live.
// ---------------------------------------------------------------------------
typedef double probe_f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void mfma_f64_probe_kernel(int iters, double seed, double *out) {
  const double a = seed + 1e-3 * threadIdx.x, b = seed - 1e-3 * threadIdx.x;
  probe_f64x4 acc[8];
  for (int i = 0; i < 8; ++i) acc[i] = probe_f64x4{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double sum = 0.0;
  for (int i = 0; i < 8; ++i) sum += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = sum;
}

void launch_mfma_f64_probe(hipStream_t s, int blocks, int iters, double *out) {
  hipLaunchKernelGGL(mfma_f64_probe_kernel, dim3(blocks), dim3(256), 0, s, iters, 0.5, out);
  check_launch();
}

}  // namespace lmpo
