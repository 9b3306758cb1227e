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
// Two-site contraction with the gate (forming the two-site block and applying
// the propagator to it):
//   M[(l,s),(t,r)] = sum_m A_k[l][s][m] A_{k+1}[m][t][r]
//   theta[(l,s'),(t',r)] = sum_{s,t} G[(s' t'),(s t)] M[(l,s),(t,r)]
// A workgroup owns 16 values of l and 16 of r, i.e. a 64 x 64 tile of M with
// all four s and all four t (a complex GEMM on the matrix cores, real-split),
// so the 16x16 gate is applied in the epilogue from LDS.  T is the arithmetic type (double, or float for the FP32
// contraction form: operands rounded to FP32, FP32 accumulation).  kReal: the
// real-arithmetic form (every operand has zero imaginary part in the Pauli
// basis), one real product instead of four and a zero imaginary output.
// Output: trans = 0 -> X = theta, column-major, ld = 4 chl;
//         trans = 1 -> X = theta^H, column-major, ld = 4 chr.
// ---------------------------------------------------------------------------
// Matrix-core step D += A B on 16 x 16 x 4 tiles: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16].  The accumulator rows a lane holds differ by type:
// FP64 (v_mfma_f64_16x16x4f64) D[l / 16 + 4 r][l % 16], FP32
// (v_mfma_f32_16x16x4f32) D[4 (l / 16) + r][l % 16], r = 0..3.
template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  typedef double type __attribute__((ext_vector_type(4)));
  __device__ static int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct MfmaAcc<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  __device__ static int row(int lk, int r) { return 4 * lk + r; }
};
template <typename T>
__device__ __forceinline__ typename MfmaAcc<T>::type mfma_step(T a, T b, typename MfmaAcc<T>::type c);
template <>
__device__ __forceinline__ MfmaAcc<double>::type mfma_step<double>(double a, double b, MfmaAcc<double>::type c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ MfmaAcc<float>::type mfma_step<float>(float a, float b, MfmaAcc<float>::type c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

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
template <typename T, bool kReal = false>
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
  const int R = 4 * chl;
  {
    double2 g = G[t];
    Gs[t / 16][t % 16] = C2{(T)g.x, (T)g.y};
  }
  // M tile (64 x 64) on the matrix cores: wave w owns rows [16 w, 16 w + 16)
  // as four 16 x 16 sub-tiles; complex products as four real MFMAs.
  const int lane = t & 63, wave = t >> 6, lr = lane & 15, lk = lane >> 4;
  using V4 = typename MfmaAcc<T>::type;
  V4 re[4], im[4];
#pragma unroll
  for (int st = 0; st < 4; ++st) re[st] = im[st] = V4{0, 0, 0, 0};
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
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
      const C2 a = As[k0 + lk][16 * wave + lr];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const C2 b = Bs[k0 + lk][16 * st + lr];
        re[st] = mfma_step<T>(a.x, b.x, re[st]);
        if (!kReal) {
          re[st] = mfma_step<T>(-a.y, b.y, re[st]);
          im[st] = mfma_step<T>(a.x, b.y, im[st]);
          im[st] = mfma_step<T>(a.y, b.x, im[st]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int r = 0; r < 4; ++r) Ms[16 * wave + MfmaAcc<T>::row(lk, r)][16 * st + lr] = C2{re[st][r], im[st][r]};
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
    for (int q = 0; q < 16; ++q) {
      if (kReal)
        out.x = fma(Gs[o][q].x, m[q].x, out.x);
      else
        cfma(out, Gs[o][q], m[q]);
    }
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
