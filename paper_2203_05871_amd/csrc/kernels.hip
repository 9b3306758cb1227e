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
__global__ __launch_bounds__(256) void contract_gate_kernel(const double2 *__restrict__ Ak,
                                                            const double2 *__restrict__ Ak1,
                                                            const double2 *__restrict__ G, int chl,
                                                            int chm, int chr,
                                                            double2 *__restrict__ X, int trans) {
  using C2 = cplx<T>;
  __shared__ C2 As[16][64];
  __shared__ C2 Bs[16][64];
  __shared__ C2 Ms[64][65];
  __shared__ C2 Gs[16][16];
  const int t = threadIdx.x;
  const int l0 = blockIdx.y * 16, r0 = blockIdx.x * 16;
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

void launch_contract_gate(hipStream_t s, int precision, const double2 *Ak, const double2 *Ak1,
                          const double2 *G, int chl, int chm, int chr, double2 *X, int trans) {
  dim3 grid((chr + 15) / 16, (chl + 15) / 16);
  if (precision == LMPO_FP32_CONTRACT)
    hipLaunchKernelGGL(contract_gate_kernel<float>, grid, dim3(256), 0, s, Ak, Ak1, G, chl, chm, chr, X,
                       trans);
  else
    hipLaunchKernelGGL(contract_gate_kernel<double>, grid, dim3(256), 0, s, Ak, Ak1, G, chl, chm, chr, X,
                       trans);
  check_launch();
}

// ---------------------------------------------------------------------------
// Block one-sided Jacobi SVD (Hestenes): X (R x C, column-major) is driven to
// mutually orthogonal columns by unitary column rotations, accumulated in V:
// X_0 V = X_final = U diag(sigma).  Columns form blocks of JB; in every round
// of a sweep the blocks are paired by a round-robin tournament and each pair's
// JP x JP Gram matrix is diagonalised by two-sided cyclic Jacobi in LDS; the
// resulting JP x JP unitary W is then applied to the pair's columns of X and V.
// A pair is skipped when all its off-diagonal Gram entries satisfy
// |g_pq| <= tol sqrt(g_pp g_qq); a sweep with no active pair has converged.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pair_blocks(int round, int p, int nbp, int &bi, int &bj) {
  const int m = nbp - 1;
  if (p == 0) {
    bi = m;
    bj = round;
  } else {
    bi = (round + p) % m;
    bj = (round - p + m) % m;
  }
}

__global__ __launch_bounds__(256) void jac_pair_kernel(const double2 *__restrict__ X, int ldx, int R,
                                                       int C, int round, int nbp, double tol,
                                                       double2 *__restrict__ Wout,
                                                       int *__restrict__ active,
                                                       int *__restrict__ counter) {
  __shared__ double2 tile[64][JP + 1];
  __shared__ double2 G[2][JP][JP + 1];
  __shared__ double2 W[2][JP][JP + 1];
  __shared__ int col[JP];
  __shared__ int partner[JP];
  __shared__ double2 alpha[JP], beta[JP];
  __shared__ int rotated[JP];
  const int t = threadIdx.x;
  const int p = blockIdx.x;
  int bi, bj;
  pair_blocks(round, p, nbp, bi, bj);
  if (t < JP) {
    int c = (t < JB) ? bi * JB + t : bj * JB + (t - JB);
    col[t] = (c < C) ? c : -1;
  }
  __syncthreads();
  const int a = t / JP, b = t % JP;
  double2 acc = make_double2(0, 0);
  for (int r0 = 0; r0 < R; r0 += 64) {
    for (int e = t; e < 64 * JP; e += 256) {
      int c = e / 64, i = e % 64;
      double2 v = make_double2(0, 0);
      if (col[c] >= 0 && r0 + i < R) v = X[(size_t)(r0 + i) + (size_t)col[c] * ldx];
      tile[i][c] = v;
    }
    __syncthreads();
#pragma unroll 8
    for (int i = 0; i < 64; ++i) dfma_cj(acc, tile[i][a], tile[i][b]);
    __syncthreads();
  }
  if (a == b) acc.y = 0.0;
  G[0][a][b] = acc;
  W[0][a][b] = make_double2(a == b ? 1.0 : 0.0, 0.0);
  __syncthreads();
  // is any off-diagonal entry above the threshold?
  int need = 0;
  if (a < b) {
    double d = sqrt(G[0][a][a].x * G[0][b][b].x);
    double m = sqrt(acc.x * acc.x + acc.y * acc.y);
    need = m > tol * d;
  }
  need = __syncthreads_or(need);
  if (!need) {
    if (t == 0) active[p] = 0;
    return;
  }
  int cur = 0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    int any = 0;
    for (int step = 0; step < JP - 1; ++step) {
      if (t < JP / 2) {
        int pp, qq;
        if (t == 0) {
          pp = JP - 1;
          qq = step;
        } else {
          pp = (step + t) % (JP - 1);
          qq = (step - t + JP - 1) % (JP - 1);
        }
        double app = G[cur][pp][pp].x, aqq = G[cur][qq][qq].x;
        double2 c = G[cur][pp][qq];
        double mc = sqrt(c.x * c.x + c.y * c.y);
        partner[pp] = qq;
        partner[qq] = pp;
        if (mc > tol * sqrt(app * aqq) && mc > 0.0) {
          double zeta = (aqq - app) / (2.0 * mc);
          double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double cs = 1.0 / sqrt(1.0 + tt * tt), sn = tt * cs;
          double2 ph = make_double2(c.x / mc, -c.y / mc);  // e^{-i phi}
          alpha[pp] = make_double2(cs, 0.0);
          beta[pp] = make_double2(-sn * ph.x, -sn * ph.y);
          alpha[qq] = make_double2(cs * ph.x, cs * ph.y);
          beta[qq] = make_double2(sn, 0.0);
          rotated[pp] = rotated[qq] = 1;
        } else {
          alpha[pp] = alpha[qq] = make_double2(1.0, 0.0);
          beta[pp] = beta[qq] = make_double2(0.0, 0.0);
          rotated[pp] = rotated[qq] = 0;
        }
      }
      __syncthreads();
      const int pa = partner[a], pb = partner[b];
      const int nxt = cur ^ 1;
      // G' = J^H G J, W' = W J
      double2 gj_a = dadd(dmul(G[cur][a][b], alpha[b]), dmul(G[cur][a][pb], beta[b]));
      double2 gj_pa = dadd(dmul(G[cur][pa][b], alpha[b]), dmul(G[cur][pa][pb], beta[b]));
      double2 g = dadd(dmul(dconj(alpha[a]), gj_a), dmul(dconj(beta[a]), gj_pa));
      if (a == b) g.y = 0.0;
      if (pa == b && rotated[a]) g = make_double2(0.0, 0.0);
      G[nxt][a][b] = g;
      W[nxt][a][b] = dadd(dmul(W[cur][a][b], alpha[b]), dmul(W[cur][a][pb], beta[b]));
      any |= rotated[0] | rotated[1] | rotated[2] | rotated[3] | rotated[4] | rotated[5] |
             rotated[6] | rotated[7] | rotated[8] | rotated[9] | rotated[10] | rotated[11] |
             rotated[12] | rotated[13] | rotated[14] | rotated[15];
      __syncthreads();
      cur = nxt;
    }
    if (!any) break;
  }
  Wout[(size_t)p * JP * JP + a * JP + b] = W[cur][a][b];
  if (t == 0) {
    active[p] = 1;
    atomicAdd(counter, 1);
  }
}

__device__ __forceinline__ void apply_pair_rotation(double2 *M, int ld, int rows, int r0,
                                                    const double2 (*W)[JP], const int *col) {
  const int t = threadIdx.x;
  const int i = r0 + (t % 64);
  const int g = t / 64;
  double2 x[JP];
#pragma unroll
  for (int c = 0; c < JP; ++c)
    x[c] = (i < rows && col[c] >= 0) ? M[(size_t)i + (size_t)col[c] * ld] : make_double2(0, 0);
  double2 out[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    out[j] = make_double2(0, 0);
#pragma unroll
    for (int c = 0; c < JP; ++c) dfma(out[j], x[c], W[c][g * 4 + j]);
  }
  __syncthreads();
  if (i < rows) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int cc = col[g * 4 + j];
      if (cc >= 0) M[(size_t)i + (size_t)cc * ld] = out[j];
    }
  }
}

__global__ __launch_bounds__(256) void jac_update_kernel(double2 *__restrict__ X, int ldx, int R,
                                                         double2 *__restrict__ V, int ldv, int C,
                                                         int round, int nbp,
                                                         const double2 *__restrict__ Win,
                                                         const int *__restrict__ active) {
  __shared__ double2 W[JP][JP];
  __shared__ int col[JP];
  const int p = blockIdx.x;
  if (!active[p]) return;
  const int t = threadIdx.x;
  int bi, bj;
  pair_blocks(round, p, nbp, bi, bj);
  if (t < JP) {
    int c = (t < JB) ? bi * JB + t : bj * JB + (t - JB);
    col[t] = (c < C) ? c : -1;
  }
  W[t / JP][t % JP] = Win[(size_t)p * JP * JP + t];
  __syncthreads();
  const int r0 = blockIdx.y * 64;
  if (r0 < R) apply_pair_rotation(X, ldx, R, r0, W, col);
  if (r0 < C) apply_pair_rotation(V, ldv, C, r0, W, col);
}

void launch_jacobi_round(hipStream_t s, double2 *X, int ldx, int R, double2 *V, int ldv, int C, int round,
                         int nbp, double tol, double2 *W, int *active, int *counter) {
  const int np = nbp / 2;
  hipLaunchKernelGGL(jac_pair_kernel, dim3(np), dim3(256), 0, s, X, ldx, R, C, round, nbp, tol, W, active,
                     counter);
  const int rows = R > C ? R : C;
  hipLaunchKernelGGL(jac_update_kernel, dim3(np, (rows + 63) / 64), dim3(256), 0, s, X, ldx, R, V, ldv, C,
                     round, nbp, W, active);
  check_launch();
}

__global__ void identity_kernel(double2 *V, int ldv, int C) {
  size_t n = (size_t)C * C;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    int i = e % C, j = e / C;
    V[(size_t)i + (size_t)j * ldv] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
}

void launch_identity(hipStream_t s, double2 *V, int ldv, int C) {
  size_t n = (size_t)C * C;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(identity_kernel, dim3(blocks), dim3(256), 0, s, V, ldv, C);
  check_launch();
}

__global__ __launch_bounds__(64) void colnorm_kernel(const double2 *__restrict__ X, int ldx, int R,
                                                     double *__restrict__ sig) {
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < R; i += 64) {
    double2 v = X[(size_t)i + (size_t)j * ldx];
    acc = fma(v.x, v.x, fma(v.y, v.y, acc));
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (threadIdx.x == 0) sig[j] = sqrt(acc);
}

void launch_colnorm(hipStream_t s, const double2 *X, int ldx, int R, int C, double *sig) {
  hipLaunchKernelGGL(colnorm_kernel, dim3(C), dim3(64), 0, s, X, ldx, R, sig);
  check_launch();
}

// ---------------------------------------------------------------------------
// Truncation select (App. B: the more severe of cut_off_rho and max_dim_rho):
// sort sigma descending (ties by column index), W = sum sigma^2,
// k_c = smallest k >= 1 with sum_{j >= k} sigma_j^2 <= cutoff W,
// k = min(chi_max, k_c, #nonzero), k >= 1.  hop = 1 keeps every nonzero value.
// One workgroup of 1024 threads, bitonic sort in LDS over <= kMaxDim entries.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void select_kernel(const double *__restrict__ sig, int C, int chi_max,
                                                      double cutoff, int hop, int *__restrict__ perm,
                                                      double *__restrict__ sorted, int *__restrict__ kept,
                                                      int *__restrict__ dims_slot, double *__restrict__ disc,
                                                      int *__restrict__ err) {
  __shared__ double key[kMaxDim];
  __shared__ int idx[kMaxDim];
  __shared__ double tail[kMaxDim + 1];
  __shared__ int cnt_above, cnt_nz, bad;
  const int t = threadIdx.x;
  int n2 = 2;
  while (n2 < C) n2 <<= 1;
  if (t == 0) {
    cnt_above = 0;
    cnt_nz = 0;
    bad = 0;
  }
  __syncthreads();
  for (int e = t; e < n2; e += 1024) {
    double v = (e < C) ? sig[e] : -1.0;
    if (e < C && !(v >= 0.0 && v < INFINITY)) atomicOr(&bad, 1);
    key[e] = v;
    idx[e] = e;
  }
  __syncthreads();
  // bitonic sort: descending key, ascending index on ties
  for (int size = 2; size <= n2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int e = t; e < n2; e += 1024) {
        int partner = e ^ stride;
        if (partner > e) {
          bool desc = ((e & size) == 0);
          double ka = key[e], kb = key[partner];
          int ia = idx[e], ib = idx[partner];
          // "a before b" in the final order
          bool a_first = (ka > kb) || (ka == kb && ia < ib);
          bool swap = desc ? !a_first : a_first;
          if (swap) {
            key[e] = kb;
            key[partner] = ka;
            idx[e] = ib;
            idx[partner] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
  // suffix sums of sigma^2 (tail[k] = sum_{j >= k})
  for (int e = t; e < n2; e += 1024) tail[e] = (e < C) ? key[e] * key[e] : 0.0;
  if (t == 0) tail[n2] = 0.0;
  __syncthreads();
  for (int off = 1; off < n2; off <<= 1) {
    double v[kMaxDim / 1024];
    int q = 0;
    for (int e = t; e < n2; e += 1024, ++q) v[q] = (e + off < n2) ? tail[e + off] : 0.0;
    __syncthreads();
    q = 0;
    for (int e = t; e < n2; e += 1024, ++q) tail[e] += v[q];
    __syncthreads();
  }
  const double W = tail[0];
  for (int e = t; e < C; e += 1024) {
    if (e >= 1 && tail[e] > cutoff * W) atomicAdd(&cnt_above, 1);
    if (key[e] > 0.0) atomicAdd(&cnt_nz, 1);
    perm[e] = idx[e];
    sorted[e] = key[e];
  }
  __syncthreads();
  if (t == 0) {
    int k;
    if (hop) {
      k = cnt_nz;
    } else {
      int kc = 1 + cnt_above;
      k = kc < chi_max ? kc : chi_max;
      if (k > cnt_nz) k = cnt_nz;
    }
    if (k < 1) k = 1;
    if (bad || !(W > 0.0)) *err = 1;
    *kept = k;
    if (dims_slot) *dims_slot = k;
    if (!hop && W > 0.0) *disc += tail[k] / W;
  }
}

void launch_select(hipStream_t s, const double *sig, int C, int chi_max, double cutoff, int hop, int *perm,
                   double *sorted, int *kept, int *dims_slot, double *disc, int *err) {
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(1024), 0, s, sig, C, chi_max, cutoff, hop, perm, sorted,
                     kept, dims_slot, disc, err);
  check_launch();
}

// ---------------------------------------------------------------------------
// Canonical update after a gate: theta = U S V^H truncated to k.
// ascending:  A_k <- U,   A_{k+1} <- S V^H   (centre moves right)
// descending: A_k <- U S, A_{k+1} <- V^H
// trans = 0: X = theta (U S = X columns, V from Jacobi);
// trans = 1: X = theta^H, so theta's left vectors are V's columns and its right
// vectors are X's columns / sigma.
// ---------------------------------------------------------------------------
__global__ void canon_kernel(const double2 *__restrict__ X, int ldx, const double2 *__restrict__ V, int ldv,
                             const int *__restrict__ perm, const double *__restrict__ sorted,
                             const int *__restrict__ kept, double2 *__restrict__ Ak,
                             double2 *__restrict__ Ak1, int chl, int chr, int trans, int asc) {
  const int k = *kept;
  const size_t na = (size_t)4 * chl * k, nbb = (size_t)k * 4 * chr;
  const size_t n = na > nbb ? na : nbb;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    if (e < na) {
      const int i = e / k, al = e % k;
      const int pc = perm[al];
      const double sg = sorted[al];
      double2 u;
      if (trans == 0) {
        double2 x = X[(size_t)i + (size_t)pc * ldx];
        u = make_double2(x.x / sg, x.y / sg);
      } else {
        u = V[(size_t)i + (size_t)pc * ldv];
      }
      if (!asc) u = make_double2(u.x * sg, u.y * sg);
      Ak[e] = u;
    }
    if (e < nbb) {
      const int al = e / (4 * chr), j = e % (4 * chr);
      const int pc = perm[al];
      const double sg = sorted[al];
      double2 v;  // right singular vector component (not yet conjugated)
      if (trans == 0) {
        v = V[(size_t)j + (size_t)pc * ldv];
      } else {
        double2 x = X[(size_t)j + (size_t)pc * ldx];
        v = make_double2(x.x / sg, x.y / sg);
      }
      if (asc) v = make_double2(v.x * sg, v.y * sg);
      Ak1[e] = dconj(v);
    }
  }
}

void launch_canon(hipStream_t s, const double2 *X, int ldx, const double2 *V, int ldv, const int *perm,
                  const double *sorted, const int *kept, double2 *Ak, double2 *Ak1, int chl, int chr, int trans,
                  int asc, int kmax) {
  size_t n = (size_t)4 * (chl > chr ? chl : chr) * kmax;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(canon_kernel, dim3(blocks), dim3(256), 0, s, X, ldx, V, ldv, perm, sorted, kept, Ak, Ak1,
                     chl, chr, trans, asc);
  check_launch();
}

// ---------------------------------------------------------------------------
// Orthogonality-centre hop (exact; no truncation beyond exact zeros).
// Right hop of the centre from site c to c+1: X = A_c as (4 chl x chm);
//   X V = U S  =>  A_c <- U,  A_{c+1} <- (S V^H) A_{c+1}.
// Left hop from c to c-1: X = A_c^H as (4 chr x chm);
//   A_c = V S U^H  =>  A_c <- U^H,  A_{c-1} <- A_{c-1} (V S).
// ---------------------------------------------------------------------------
__global__ void hop_load_kernel(const double2 *__restrict__ A, int rows, int cols, double2 *__restrict__ X,
                                int ct) {
  size_t n = (size_t)rows * cols;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    int i = e / cols, j = e % cols;
    double2 a = A[e];
    if (!ct)
      X[(size_t)i + (size_t)j * rows] = a;
    else
      X[(size_t)j + (size_t)i * cols] = dconj(a);
  }
}

void launch_hop_load(hipStream_t s, const double2 *A, int rows, int cols, double2 *X, int ct) {
  size_t n = (size_t)rows * cols;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(hop_load_kernel, dim3(blocks), dim3(256), 0, s, A, rows, cols, X, ct);
  check_launch();
}

// right = 1: A_c[i][al] = X[i][perm al] / s (R x k); Z[al][m] = s conj(V[m][perm al]) (k x C)
// right = 0: A_c[al][j] = conj(X[j][perm al]) / s (k x R); Z[m][al] = V[m][perm al] s (C x k)
__global__ void hop_write_kernel(const double2 *__restrict__ X, int ldx, const double2 *__restrict__ V, int ldv,
                                 const int *__restrict__ perm, const double *__restrict__ sorted, int k,
                                 double2 *__restrict__ Ac, double2 *__restrict__ Z, int R, int C, int right) {
  const size_t na = (size_t)R * k, nz = (size_t)k * C;
  const size_t n = na > nz ? na : nz;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    if (e < na) {
      int i, al;
      if (right) {
        i = e / k;
        al = e % k;
      } else {
        al = e / R;
        i = e % R;
      }
      const double sg = sorted[al];
      double2 x = X[(size_t)i + (size_t)perm[al] * ldx];
      x = make_double2(x.x / sg, x.y / sg);
      Ac[e] = right ? x : dconj(x);
    }
    if (e < nz) {
      int al, m;
      if (right) {
        al = e / C;
        m = e % C;
      } else {
        m = e / k;
        al = e % k;
      }
      const double sg = sorted[al];
      double2 v = V[(size_t)m + (size_t)perm[al] * ldv];
      v = make_double2(v.x * sg, v.y * sg);
      Z[e] = right ? dconj(v) : v;
    }
  }
}

void launch_hop_write(hipStream_t s, const double2 *X, int ldx, const double2 *V, int ldv, const int *perm,
                      const double *sorted, int k, double2 *Ac, double2 *Z, int R, int C, int right) {
  size_t n = (size_t)(R > C ? R : C) * k;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(hop_write_kernel, dim3(blocks), dim3(256), 0, s, X, ldx, V, ldv, perm, sorted, k, Ac, Z, R,
                     C, right);
  check_launch();
}

// Plain complex FP64 GEMM, row-major: Cm[M x N] = A[M x K] B[K x N].
__global__ __launch_bounds__(256) void zgemm_kernel(int M, int N, int K, const double2 *__restrict__ A, int lda,
                                                    const double2 *__restrict__ B, int ldb,
                                                    double2 *__restrict__ Cm, int ldc) {
  __shared__ double2 As[16][64];
  __shared__ double2 Bs[16][64];
  const int t = threadIdx.x;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int ty = t / 16, tx = t % 16;
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0, 0);
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = t + 256 * q;
      int row = e / 16, kk = e % 16;
      As[kk][row] = (i0 + row < M && k0 + kk < K) ? A[(size_t)(i0 + row) * lda + k0 + kk] : make_double2(0, 0);
      int kb = e / 64, j = e % 64;
      Bs[kb][j] = (k0 + kb < K && j0 + j < N) ? B[(size_t)(k0 + kb) * ldb + j0 + j] : make_double2(0, 0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      double2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) dfma(acc[i][j], a[i], b[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int r = i0 + ty * 4 + i, c = j0 + tx + 16 * j;
      if (r < M && c < N) Cm[(size_t)r * ldc + c] = acc[i][j];
    }
}

void launch_zgemm(hipStream_t s, int M, int N, int K, const double2 *A, int lda, const double2 *B, int ldb,
                  double2 *Cm, int ldc) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL(zgemm_kernel, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, Cm, ldc);
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
