// Two-site contraction tile shared by the single-chain and batched kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace lmpo {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ void cfma(cplx<T> &acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

// Bond dimension read that bypasses stale cache lines (dims are rewritten by
// other workgroups inside persistent kernels).
__device__ __forceinline__ int ld_dim(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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
struct ContractLds {
  cplx<T> As[16][64];
  cplx<T> Bs[16][64];
  cplx<T> Ms[64][65];
  cplx<T> Gs[16][16];
};

// One 16 (l) x 16 (r) output tile (bx, by) of the contraction on bond k, run by
// one workgroup of 256 threads; tiles outside the current dims return at once.
// dims may change between launches, so they are read with device-scope loads.
template <typename T>
__device__ __forceinline__ void contract_tile(ContractLds<T> &lds, double2 *const *sites, const int *dims, int N,
                                              int k, const double2 *__restrict__ G, double2 *__restrict__ X,
                                              const int bx, const int by) {
  using C2 = cplx<T>;
  const int chl = (k == 0) ? 1 : ld_dim(dims + k - 1), chm = ld_dim(dims + k),
            chr = (k + 1 == N - 1) ? 1 : ld_dim(dims + k + 1);
  const int trans = (4 * chl >= 4 * chr) ? 0 : 1;
  if (by * 16 >= chl || bx * 16 >= chr) return;
  const double2 *__restrict__ Ak = sites[k];
  const double2 *__restrict__ Ak1 = sites[k + 1];
  auto &As = lds.As;
  auto &Bs = lds.Bs;
  auto &Ms = lds.Ms;
  auto &Gs = lds.Gs;
  __syncthreads();  // the previous tile of this workgroup may still read Gs / Ms
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

// ---------------------------------------------------------------------------
// Trace and rescaling shared by the single-chain kernels and the batched
// layer kernel (explicit fma, so both give the same bits).
// In the basis P_a = sigma^a / sqrt(2), Tr P_a = sqrt(2) delta_{a0}.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 zmul_exact(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ void zfma_exact(double2 &acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

// v_out[r] = sqrt(2) sum_l v_in[l] A[l][a][r], by one workgroup (v in LDS).
__device__ __forceinline__ void env_step_right(const double2 *__restrict__ A, int cl, int cr, int a,
                                               const double2 *vin, double2 *vout) {
  const double s2 = 1.4142135623730951;
  for (int r = threadIdx.x; r < cr; r += blockDim.x) {
    double2 acc = make_double2(0, 0);
    const double2 *col = A + (size_t)a * cr + r;
    for (int l = 0; l < cl; ++l) zfma_exact(acc, vin[l], col[(size_t)l * 4 * cr]);
    vout[r] = make_double2(acc.x * s2, acc.y * s2);
  }
}

// tr(rho) by one workgroup; v0, v1 hold at least max bond dim entries.
__device__ __forceinline__ double2 chain_trace(double2 *const *sites, const int *dims, int N, double2 *v0,
                                               double2 *v1) {
  if (threadIdx.x == 0) v0[0] = make_double2(1.0, 0.0);
  __syncthreads();
  for (int i = 0; i < N; ++i) {
    const int cl = i == 0 ? 1 : ld_dim(dims + i - 1), cr = i == N - 1 ? 1 : ld_dim(dims + i);
    env_step_right(sites[i], cl, cr, 0, v0, v1);
    __syncthreads();
    double2 *t = v0;
    v0 = v1;
    v1 = t;
  }
  return v0[0];
}

// 1 / z for the rescaling rho -> rho / tr(rho).
__device__ __forceinline__ double2 zinv_exact(double2 z) {
  const double d = fma(z.x, z.x, z.y * z.y);
  return make_double2(z.x / d, -z.y / d);
}

}  // namespace lmpo
