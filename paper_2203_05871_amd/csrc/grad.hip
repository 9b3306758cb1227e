// HIP kernels (gfx950) of the adjoint gradient: contractions of the state MPS
// with the co-state MPS (bilinear: coefficients are paired without complex
// conjugation), the two-site transition density, and the accumulation of
// each gate's contribution tr(K Gamma) into the parameter gradient.
//
// Complex numbers are double2 (x = re, y = im).
#include "lmpo_internal.h"

namespace lmpo {

namespace {

__device__ __forceinline__ void zfma(double2 &acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

constexpr int kBM = 32, kBN = 32, kBK = 16;

}  // namespace

// C(m, n) = sum_k A(m, k) B(k, n) for batch z, every operand addressed by its
// own element strides (any transposition or slice of a row-major tensor).
// 256 threads own a 32 x 32 tile of C, 2 x 2 elements each; A and B pass
// through LDS in k-chunks of 16.  Reads outside [0, M) x [0, K) and
// [0, K) x [0, N) are replaced by zeros, so the grid may cover more than C.
__global__ __launch_bounds__(256) void zgemm_kernel(ZgemmArgs g) {
  __shared__ double2 As[kBK][kBM + 1];
  __shared__ double2 Bs[kBK][kBN + 1];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN, z = blockIdx.z;
  const double2 *A = g.A + (long long)z * g.sab;
  const double2 *B = g.B + (long long)z * g.sbb;
  double2 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < g.K; k0 += kBK) {
    for (int e = tid; e < kBK * kBM; e += 256) {
      const int kk = e / kBM, mm = e % kBM;
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < g.M && k < g.K) ? A[(long long)m * g.sam + (long long)k * g.sak] : make_double2(0.0, 0.0);
    }
    for (int e = tid; e < kBK * kBN; e += 256) {
      const int kk = e / kBN, nn = e % kBN;
      const int n = n0 + nn, k = k0 + kk;
      Bs[kk][nn] = (n < g.N && k < g.K) ? B[(long long)k * g.sbk + (long long)n * g.sbn] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kBK; ++kk) {
      const double2 a0 = As[kk][ty], a1 = As[kk][ty + 16];
      const double2 b0 = Bs[kk][tx], b1 = Bs[kk][tx + 16];
      zfma(acc[0][0], a0, b0);
      zfma(acc[0][1], a0, b1);
      zfma(acc[1][0], a1, b0);
      zfma(acc[1][1], a1, b1);
    }
    __syncthreads();
  }
  double2 *C = g.C + (long long)z * g.scb;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const int m = m0 + ty + 16 * i, n = n0 + tx + 16 * j;
      if (m < g.M && n < g.N) C[(long long)m * g.scm + (long long)n * g.scn] = acc[i][j];
    }
}

void launch_zgemm(hipStream_t s, const ZgemmArgs &g, int batch) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return;
  dim3 grid((g.N + kBN - 1) / kBN, (g.M + kBM - 1) / kBM, batch);
  hipLaunchKernelGGL(zgemm_kernel, grid, dim3(256), 0, s, g);
  (void)hipGetLastError();
}

// gam[(c d) * 16 + (a b)] = sum_{p, q} E[a][p][c][q] Fr[d][p][b][q] with p <
// pm (co-state bond) and q < qm (state bond): one workgroup per output, a
// fixed-order reduction (results do not depend on timing).
__global__ __launch_bounds__(256) void transition_reduce_kernel(const double2 *__restrict__ E,
                                                                const double2 *__restrict__ Fr, int pm, int qm,
                                                                double2 *__restrict__ gam) {
  __shared__ double2 red[256];
  const int out = blockIdx.x;
  const int x = out / 16, y = out % 16;
  const int c = x / 4, d = x % 4, a = y / 4, b = y % 4;
  const long long n = (long long)pm * qm;
  double2 acc = make_double2(0.0, 0.0);
  for (long long e = threadIdx.x; e < n; e += 256) {
    const int p = (int)(e / qm), q = (int)(e % qm);
    const double2 u = E[(((long long)a * pm + p) * 4 + c) * qm + q];
    const double2 v = Fr[(((long long)d * pm + p) * 4 + b) * qm + q];
    zfma(acc, u, v);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = zadd(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) gam[out] = red[0];
}

void launch_transition_reduce(hipStream_t s, const double2 *E, const double2 *Fr, int pm, int qm, double2 *gam) {
  hipLaunchKernelGGL(transition_reduce_kernel, dim3(256), dim3(256), 0, s, E, Fr, pm, qm, gam);
  (void)hipGetLastError();
}

// grad[pidx[j]] += scale * sum_{y, x} K[j][y][x] gam[x][y] for the nk
// parameters j of one gate (K: [nk][16][16], row = output index).  One
// workgroup per parameter; workgroups write distinct entries.
__global__ __launch_bounds__(256) void grad_accumulate_kernel(const double2 *__restrict__ K, const int *pidx,
                                                              const double2 *__restrict__ gam, double2 scale,
                                                              double2 *grad) {
  __shared__ double2 red[256];
  const int j = blockIdx.x, e = threadIdx.x;
  const int y = e / 16, x = e % 16;
  double2 acc = make_double2(0.0, 0.0);
  zfma(acc, K[(size_t)j * 256 + e], gam[x * 16 + y]);
  red[e] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (e < off) red[e] = zadd(red[e], red[e + off]);
    __syncthreads();
  }
  if (e == 0) {
    const int t = pidx[j];
    if (t >= 0) {
      double2 v = make_double2(0.0, 0.0);
      zfma(v, scale, red[0]);
      grad[t] = zadd(grad[t], v);
    }
  }
}

void launch_grad_accumulate(hipStream_t s, const double2 *K, const int *pidx, int nk, const double2 *gam,
                            double2 scale, double2 *grad) {
  hipLaunchKernelGGL(grad_accumulate_kernel, dim3(nk), dim3(256), 0, s, K, pidx, gam, scale, grad);
  (void)hipGetLastError();
}

// Site k of the MPS sum A + B (the co-state plus an output's source): A from a
// copy of the site (bond dims `dims`, before the sum), B with bond kb; the
// sum's site is a row [A B] on the first site, a column [A; B] on the last,
// block-diagonal inside.  Grid-stride over the summed site.
__global__ void mps_sum_site_kernel(const double2 *__restrict__ A, const double2 *__restrict__ B,
                                    double2 *__restrict__ dst, const int *dims, int N, int k, int kb) {
  const int cl = k == 0 ? 1 : dims[k - 1], cr = k == N - 1 ? 1 : dims[k];
  const bool first = k == 0, last = k == N - 1;
  const int bl = first ? 1 : kb, br = last ? 1 : kb;
  const int nl = first ? 1 : cl + kb, nr = last ? 1 : cr + kb;
  const size_t n = (size_t)nl * 4 * nr;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % nr), a = (int)((e / nr) % 4), l = (int)(e / ((size_t)4 * nr));
    double2 v = make_double2(0.0, 0.0);
    const bool la = first || l < cl, ra = last || r < cr;  // index inside A's block
    if (la && ra) {
      v = A[((size_t)l * 4 + a) * cr + r];
    } else if (!la && !ra) {
      v = B[((size_t)(l - cl) * 4 + a) * br + (r - cr)];
    } else if (first && !ra) {
      v = B[((size_t)a) * br + (r - cr)];
    } else if (last && !la) {
      v = B[((size_t)(l - cl) * 4 + a) * br];
    }
    (void)bl;
    dst[e] = v;
  }
}

// Site k right after an identity gate on bond (k - 1, k) swept left to right
// holds diag(s) V^dagger: rows are the bond index, each of length 4 chr, and
// with every site to its right right-orthonormal row i has norm s_i.  With
// p_i = s_i^2 / W, W = sum s^2 and S = -sum p ln p (the OSEE across the bond,
// into *out), dS/ds_i = (2 s_i / W)(-ln p_i - S): scaling row i by that over
// s_i, (2 / W)(-ln p_i - S), makes the site the right factor of
// U diag(dS/ds) V^dagger.  Rows of zero weight are left zero.  out[1] =
// sum_i (dS/ds_i)^2: zero when the co-state is (a single weight, or equal
// weights).  One workgroup; rows <= kOseeRows (checked on the host).
__global__ __launch_bounds__(256) void osee_costate_kernel(double2 *const *sites, const int *dims, int N, int k,
                                                           double *out) {
  __shared__ double nrm[kOseeRows];
  __shared__ double red[256];
  const int rows = dims[k - 1], len = 4 * (k == N - 1 ? 1 : dims[k]);
  double2 *A = sites[k];
  auto reduce = [&](double v) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
  };
  for (int i = 0; i < rows; ++i) {
    double acc = 0.0;
    for (int e = threadIdx.x; e < len; e += 256) {
      const double2 v = A[(size_t)i * len + e];
      acc = fma(v.x, v.x, fma(v.y, v.y, acc));
    }
    const double r = reduce(acc);
    if (threadIdx.x == 0) nrm[i] = r;
  }
  __syncthreads();
  double w = 0.0;
  for (int i = threadIdx.x; i < rows; i += 256) w += nrm[i];
  const double W = reduce(w);
  double h = 0.0;
  for (int i = threadIdx.x; i < rows; i += 256) {
    const double p = nrm[i] / W;
    if (p > 0.0) h -= p * log(p);
  }
  const double S = reduce(h);
  double q = 0.0;
  for (int i = threadIdx.x; i < rows; i += 256) {
    const double p = nrm[i] / W;
    const double f = p > 0.0 ? (2.0 / W) * (-log(p) - S) : 0.0;
    q = fma(nrm[i] * f, f, q);
  }
  const double G2 = reduce(q);
  for (size_t e = threadIdx.x; e < (size_t)rows * len; e += 256) {
    const double p = nrm[e / len] / W;
    const double f = p > 0.0 ? (2.0 / W) * (-log(p) - S) : 0.0;
    A[e] = make_double2(A[e].x * f, A[e].y * f);
  }
  if (threadIdx.x == 0) {
    out[0] = S;
    out[1] = G2;
  }
}

void launch_osee_costate(hipStream_t s, double2 *const *sites, const int *dims, int N, int k, double *out) {
  hipLaunchKernelGGL(osee_costate_kernel, dim3(1), dim3(256), 0, s, sites, dims, N, k, out);
  (void)hipGetLastError();
}

__global__ void add_dims_kernel(int *dims, int n, int add) {
  for (int b = threadIdx.x; b < n; b += blockDim.x) dims[b] += add;
}

void launch_mps_sum_site(hipStream_t s, const double2 *A, const double2 *B, double2 *dst, const int *dims, int N,
                         int k, int kb) {
  hipLaunchKernelGGL(mps_sum_site_kernel, dim3(256), dim3(256), 0, s, A, B, dst, dims, N, k, kb);
  (void)hipGetLastError();
}

void launch_add_dims(hipStream_t s, int *dims, int n, int add) {
  hipLaunchKernelGGL(add_dims_kernel, dim3(1), dim3(64), 0, s, dims, n, add);
  (void)hipGetLastError();
}

}  // namespace lmpo
