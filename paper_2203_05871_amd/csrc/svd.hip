// Persistent, device-driven truncated SVD for one two-site block or one
// orthogonality-centre hop (gfx950).
//
// One cooperative launch performs, with grid barriers between phases:
//   (hop only) load X from the site tensor
//   V <- I
//   sweeps of block one-sided Jacobi until a sweep applies no rotation
//   column norms sigma_j = ||x_j||
//   sort + truncation select (workgroup 0)
//   gate: canonical update of A_k, A_{k+1};  hop: A_c <- Q, neighbour <- R * neighbour
// All problem sizes come from the bond-dimension array in device memory, so a
// whole Trotter step is enqueued without any host synchronisation.
//
// Jacobi (Hestenes) on X (R x C, column-major, R >= C): X V = U diag(sigma).
// Columns form blocks of JB; each round pairs the blocks by a round-robin
// tournament.  Per pair, the JP x JP Gram matrix G = X_p^H X_p is diagonalised
// by cyclic two-sided Jacobi in LDS (W unitary, G W = W diag), then X_p <- X_p W
// and V_p <- V_p W.  A pair is skipped when every off-diagonal entry satisfies
// |g_pq| <= tol sqrt(g_pp g_qq): the columns are then orthogonal to working
// accuracy relative to their own norms, which gives small singular values
// to high relative accuracy.
#include <cstdlib>

#include "contract_tile.h"
#include "householder.h"
#include "lmpo_internal.h"
#include "rsi.h"

namespace lmpo {

namespace {

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ void zfma(double2 &acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ void zfma_cj(double2 &acc, double2 a, double2 b) {  // acc += conj(a) b
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

constexpr int NT = 256;  // threads per workgroup
constexpr int kInnerSweeps = 1;
constexpr int kHopCholMin = 64;  // smallest bond a centre hop moves by Cholesky QR
constexpr int kRsiMaxIters = 40;  // subspace iterations before the full SVD takes over

// Hierarchical grid barrier: 8 group counters (one per workgroup residue mod 8,
// i.e. per XCD under the default round-robin dispatch) and a top counter; all
// counters are monotonic (barrier n waits for n * members arrivals).
struct Barrier {
  unsigned *grp;  // [8 * 32] (one 128-byte line per group)
  unsigned *top;
  unsigned *flag;
  int *err;       // set to 2 if a wait ever exceeds its spin limit
  unsigned G;     // workgroups taking part
  unsigned rank;  // this workgroup's index among them
  unsigned phase;
  // Every thread's global writes before the barrier are visible to every
  // workgroup after it: the workgroup barrier orders this block's stores,
  // thread 0 publishes them device-wide (agent-scope fence) and, after the
  // wait, acquires the other blocks' stores for the whole workgroup.
  __device__ void sync() {
    if (G == 1u) {
      // one workgroup: its own barrier orders its plain global traffic, and
      // the device-scope fence orders that against the atomics, which are
      // performed beyond the L2 that holds the plain stores
      __syncthreads();
      if (threadIdx.x == 0) __threadfence();
      __syncthreads();
      ++phase;
      return;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      const unsigned target = ++phase;
      const unsigned g = rank & 7u;
      const unsigned ngrp = G < 8u ? G : 8u;
      const unsigned members = (G - g + 7u) / 8u;
      unsigned old = atomicAdd(&grp[g * 32], 1u);
      if (old == target * members - 1u) {
        unsigned t = atomicAdd(top, 1u);
        if (t == target * ngrp - 1u) __hip_atomic_store(flag, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      // bounded wait: a co-resident grid always completes; the limit (seconds)
      // only guarantees that every wave exits if residency were ever violated.
      // The flag is polled with relaxed loads and acquired once by the fence
      // below: an acquiring load invalidates the XCD's L2 at every poll,
      // which starves the workgroups still working on that XCD.
      unsigned spins = 0;
      while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1u << 25)) {
          atomicOr(err, 2);
          break;
        }
      }
      __threadfence();
    } else {
      ++phase;
    }
    __syncthreads();
  }
};

// 1/sqrt(x) from the hardware estimate plus Newton steps (to ~1 ulp; x > 0
// normal).
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y * fma(-0.5 * x * y, y, 1.5);
}

// LDS ordering among the lanes of one wavefront: its LDS operations execute in
// order, so a compiler fence plus a wait for outstanding LDS traffic suffices.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Dataflow order between Jacobi rounds: every column block belongs to exactly
// one pair per round, so a pair of round r needs only its two blocks as the
// pairs of round r - 1 left them.  ver[b] counts the rounds that have
// finished with block b (monotonic within a launch); a pair waits until both
// of its blocks reach `need`, works, and publishes need + 1 for both.  The
// fences are those of the grid barrier (agent-scope release before the
// publishing store; relaxed polling, then an acquire fence after the wait);
// the wait is bounded like the barrier's and skipped once an error has been
// flagged.
__device__ __forceinline__ void wait_blocks(unsigned *va, unsigned *vb, unsigned need, int *err) {
  if (threadIdx.x == 0) {
    unsigned spins = 0;
    while (__hip_atomic_load(va, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need ||
           __hip_atomic_load(vb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 25)) {  // the grid barrier's bound
        atomicOr(err, 2);
        break;
      }
    }
    __threadfence();
  }
  __syncthreads();
}
// Call after a __syncthreads() that follows the block's writes.
__device__ __forceinline__ void publish_blocks(unsigned *va, unsigned *vb, unsigned v) {
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_store(va, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(vb, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

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

// Partner of index i in step `step` of the round-robin over JP indices.
__device__ __forceinline__ int inner_partner(int i, int step) {
  const int m = JP - 1;
  if (i == m) return step;
  if (i == step) return m;
  // i = (step + t) % m  <->  partner = (step - t) % m
  int t = (i - step + m) % m;
  return (step - t + m) % m;
}

constexpr int kChunk = 512;  // rows of a column pair staged in LDS at once
struct SharedPair {
  double2 xs[kChunk][JP + 1];
  double2 G[2][JP][JP + 1];
  double2 W[2][JP][JP + 1];
  int col[JP];
};
struct SharedSelect {
  double key[kMaxDim];
  int idx[kMaxDim];
  double tail[kMaxDim + 1];
  int cnt_above, cnt_nz, bad;
};
struct SharedGemm {
  double2 As[16][64];
  double2 Bs[16][64];
};
union SharedAll {
  SharedPair pair;
  SharedSelect sel;
  SharedGemm gemm;
  SharedQR qr;
  rsi::SharedGemm rg;
  rsi::SharedChol rc;
  double red[NT];
};
static_assert(NT == NT_QR, "the Householder helpers assume the SVD workgroup size");

// Stage rows [r0, r0 + n) of the pair's columns of M into LDS (xs[i][c]).
// All global loads of a thread are issued before any LDS store, so their
// latencies overlap instead of adding up.
__device__ __forceinline__ void stage_rows(SharedPair &s, const double2 *__restrict__ M, int ld, int r0, int n) {
  constexpr int kRows = kChunk / NT;  // rows per thread and column
  double2 buf[JP][kRows];
#pragma unroll
  for (int c = 0; c < JP; ++c)
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int i = threadIdx.x + k * NT;
      buf[c][k] = (i < n && s.col[c] >= 0) ? rsi::gld(M, (size_t)(r0 + i) + (size_t)s.col[c] * ld) : make_double2(0, 0);
    }
#pragma unroll
  for (int c = 0; c < JP; ++c)
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int i = threadIdx.x + k * NT;
      if (i < n) s.xs[i][c] = buf[c][k];
    }
}

// MFMA helpers: v_mfma_f64_16x16x4f64 computes D(16x16) += A(16x4) B(4x16).
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; it holds
// D[l / 16 + 4 r][l % 16] in register r (rows interleaved by 4, unlike the
// f32 16x16x4 form; checked on gfx950).  Complex products are split into four
// real MFMAs.
typedef double d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// M[r0 + i][col[c]] <- sum_q xs[i][q] W[q][c] for the staged rows (n rows),
// one 16-row block per wave and step.  kReal: every operand is real (the
// real-arithmetic form), one real MFMA per step and a zero imaginary part.
template <bool kReal>
__device__ __forceinline__ void rotate_staged(SharedPair &s, const double2 (*W)[JP + 1], double2 *__restrict__ M,
                                              int ld, int r0, int n) {
  static_assert(JP == 16, "MFMA tiling assumes 16 columns per pair");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  double2 w[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) w[kk] = W[4 * kk + lk][lr];
  const int cj = s.col[lr];
  for (int i0 = wave * 16; i0 < n; i0 += 64) {
    d4 yr = {0, 0, 0, 0}, yi = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int row = i0 + lr;
      const double2 x = (row < n) ? s.xs[row][4 * kk + lk] : make_double2(0, 0);
      yr = mfma64(x.x, w[kk].x, yr);
      if (!kReal) {
        yr = mfma64(-x.y, w[kk].y, yr);
        yi = mfma64(x.x, w[kk].y, yi);
        yi = mfma64(x.y, w[kk].x, yi);
      }
    }
    if (cj >= 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + lk + 4 * r;
        if (row < n) rsi::gst(M, (size_t)(r0 + row) + (size_t)cj * ld, make_double2(yr[r], yi[r]));
      }
    }
  }
}

// One Jacobi pair: Gram of the JP columns, one cyclic sweep of two-sided
// Jacobi on it (W), then X_p <- X_p W and V_p <- V_p W.  The same workgroup
// does all of it, so a round needs a single grid barrier.  Returns whether the
// pair was rotated (some off-diagonal above threshold).  kReal: the columns are
// real (real-arithmetic form): real Gram, real rotations, real products.
template <bool kReal>
__device__ __forceinline__ bool pair_work(SharedPair &s, double2 *__restrict__ X, int ldx, int R, double2 *__restrict__ Wout,
                          int C, int bi, int bj, double tol, const int *__restrict__ cmap, unsigned long long *tp) {
  const int t = threadIdx.x;
  unsigned long long tm = wall_clock64();
  auto mark = [&](int slot) {
    if (tp && t == 0) {
      unsigned long long now = wall_clock64();
      tp[slot] += now - tm;
      tm = now;
    }
  };
  if (t < JP) {
    int c = (t < JB) ? bi * JB + t : bj * JB + (t - JB);
    s.col[t] = (c < C) ? cmap[c] : -1;
  }
  __syncthreads();
  const int a = t / JP, b = t % JP;
  // G = X_p^H X_p with MFMA: A[i][k] = conj(X[k][i]) and B[k][j] = X[k][j] take
  // the same element per lane; each wave covers every fourth 4-row step.
  {
    const int lane = t & 63, wave = t >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    d4 gr = {0, 0, 0, 0}, gi = {0, 0, 0, 0};
    for (int r0 = 0; r0 < R; r0 += kChunk) {
      const int n = min(kChunk, R - r0);
      stage_rows(s, X, ldx, r0, n);
      __syncthreads();
      for (int k0 = wave * 4; k0 < n; k0 += 16) {
        const int row = k0 + lk;
        const double2 x = (row < n) ? s.xs[row][lr] : make_double2(0, 0);
        gr = mfma64(x.x, x.x, gr);
        if (!kReal) {
          gr = mfma64(x.y, x.y, gr);
          gi = mfma64(x.x, x.y, gi);
          gi = mfma64(-x.y, x.x, gi);
        }
      }
      if (r0 + kChunk < R) __syncthreads();
    }
    // reduce the four waves' partial Grams through LDS: wave w writes its
    // partial to scratch slot w (G[0], G[1], W[0], W[1]), one barrier, sum
    double2 (*part)[JP + 1] = (wave == 0) ? s.G[0] : (wave == 1) ? s.G[1] : (wave == 2) ? s.W[0] : s.W[1];
#pragma unroll
    for (int r = 0; r < 4; ++r) part[lk + 4 * r][lr] = make_double2(gr[r], gi[r]);
    __syncthreads();
  }
  double2 acc = zadd(zadd(s.G[0][a][b], s.G[1][a][b]), zadd(s.W[0][a][b], s.W[1][a][b]));
  __syncthreads();
  if (a == b) acc.y = 0.0;
  s.G[0][a][b] = acc;
  s.W[0][a][b] = make_double2(a == b ? 1.0 : 0.0, 0.0);
  __syncthreads();
  int need = 0;
  if (a < b) {
    double d = sqrt(s.G[0][a][a].x * s.G[0][b][b].x);
    double m = sqrt(acc.x * acc.x + acc.y * acc.y);
    need = m > tol * d;
  }
  need = __syncthreads_or(need);
  mark(8);
  if (tp && t == 0) {
    tp[13] += 1;
    tp[14] += need ? 1 : 0;
  }
  if (!need) return false;
  // One cyclic sweep over the JP x JP Gram per round: the pair need not be
  // diagonalised exactly, later rounds recompute its Gram from the columns
  // (the outer sweep count is the same as with a fully converged inner solve).
  // Each thread (a, b) computes the two rotations it needs (those of a's and
  // b's pairs) itself, so a step costs one workgroup barrier.
  int cur = 0;
  const double tol2 = tol * tol;
  // rotation of pair (p, q), p < q, that zeroes g_pq: columns
  // x_p' = cs x_p + s x_q, x_q' = cs x_q - conj(s) x_p with cs real,
  // s = tau cs, cs = 1 / sqrt(1 + |tau|^2) and the small root
  // tau = 2 conj(g_pq) / D, D = d + sgn(d) sqrt(d^2 + 4 |g_pq|^2), d = g_pp - g_qq;
  // with q = 1 / sqrt(D^2 + 4 |g_pq|^2) that is cs = |D| q, s = 2 sgn(d) conj(g_pq) q
  // (two reciprocal square roots, no division).
  // Returns false (identity) when g_pq is below the threshold.
  auto rotation = [&](int p, int q, double &cs, double2 &sc) {
    const double app = s.G[cur][p][p].x, aqq = s.G[cur][q][q].x;
    const double2 c = s.G[cur][p][q];
    const double mc2 = fma(c.x, c.x, c.y * c.y);
    if (!(mc2 > tol2 * (app * aqq) && mc2 > 1e-290)) {  // (normal range for the rsq estimates)
      cs = 1.0;
      sc = make_double2(0.0, 0.0);
      return false;
    }
    const double d = app - aqq;
    const double r2 = fma(d, d, 4.0 * mc2);
    const double r = r2 * rsq_nr(r2);
    const double D = d + copysign(r, d);
    const double iq = rsq_nr(fma(D, D, 4.0 * mc2));
    cs = fabs(D) * iq;
    const double f = copysign(2.0 * iq, d);
    sc = make_double2(f * c.x, -f * c.y);
    return true;
  };
  // complex products, or real ones in the real-arithmetic form
  auto mul = [](double2 x, double2 y) { return kReal ? make_double2(x.x * y.x, 0.0) : zmul(x, y); };
  auto cmul_conj = [](double2 x, double2 y) {  // conj(x) y
    return kReal ? make_double2(x.x * y.x, 0.0) : zmul(zconj(x), y);
  };
  for (int sweep = 0; sweep < kInnerSweeps; ++sweep) {
    for (int step = 0; step < JP - 1; ++step) {
      const int pa = inner_partner(a, step), pb = inner_partner(b, step);
      double cs_a, cs_b;
      double2 s_a, s_b;
      const bool rot_a = rotation(min(a, pa), max(a, pa), cs_a, s_a);
      rotation(min(b, pb), max(b, pb), cs_b, s_b);
      // column b of J: J[b][b] = cs, J[pb][b] = s (b the lower index) or -conj(s)
      const double2 al_a = make_double2(cs_a, 0.0), al_b = make_double2(cs_b, 0.0);
      const double2 be_a = a < pa ? s_a : make_double2(-s_a.x, s_a.y);
      const double2 be_b = b < pb ? s_b : make_double2(-s_b.x, s_b.y);
      const int nxt = cur ^ 1;
      const double2 gj_a = zadd(mul(s.G[cur][a][b], al_b), mul(s.G[cur][a][pb], be_b));
      const double2 gj_pa = zadd(mul(s.G[cur][pa][b], al_b), mul(s.G[cur][pa][pb], be_b));
      double2 g = zadd(cmul_conj(al_a, gj_a), cmul_conj(be_a, gj_pa));
      if (a == b) g.y = 0.0;
      if (pa == b && rot_a) g = make_double2(0.0, 0.0);
      s.G[nxt][a][b] = g;
      s.W[nxt][a][b] = zadd(mul(s.W[cur][a][b], al_b), mul(s.W[cur][a][pb], be_b));
      __syncthreads();
      cur = nxt;
    }
  }
  mark(9);
  const double2(*W)[JP + 1] = s.W[cur];
  // X_p <- X_p W (rows still staged when R fits one chunk)
  // (the Gram pass left the last chunk of rows staged: rotate it first, then
  // stage the others again)
  const int rlast = ((R - 1) / kChunk) * kChunk;
  rotate_staged<kReal>(s, W, X, ldx, rlast, R - rlast);
  for (int r0 = 0; r0 < rlast; r0 += kChunk) {
    __syncthreads();
    stage_rows(s, X, ldx, r0, kChunk);
    __syncthreads();
    rotate_staged<kReal>(s, W, X, ldx, r0, kChunk);
  }
  // record W for the row-parallel update of V after the sweep
  rsi::gst(Wout, t, W[t / JP][t % JP]);
  __syncthreads();
  mark(10);
  return true;
}

// V <- V W_1 W_2 ... over one sweep's rounds (kReal: real V and W).  The rows of V transform
// independently, so workgroups take row blocks of V into LDS and apply every
// recorded pair rotation of the sweep in round order; no grid barrier needed.
template <bool kReal>
__device__ __forceinline__ void sweep_update_v(SharedPair &s, double2 *__restrict__ V, int ldv, int C, int nbp,
                               const double2 *__restrict__ Wsw, const int *__restrict__ act, int G,
                               const int *__restrict__ cmap, int rank) {
  const int npairs = nbp / 2;
  double2 *vs = &s.xs[0][0];  // h rows x C columns, row-major, h * C <= kChunk * (JP + 1)
  int h = (kChunk * (JP + 1)) / C;
  h = h >= 16 ? 16 : (h >= 8 ? 8 : 4);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  for (int r0 = rank * h; r0 < C; r0 += G * h) {
    const int nr = min(h, C - r0);
    __syncthreads();
    for (int e = threadIdx.x; e < h * C; e += NT) {
      const int i = e / C, c = e - i * C;
      vs[e] = (i < nr) ? rsi::gld(V, (size_t)(r0 + i) + (size_t)c * ldv) : make_double2(0, 0);
    }
    __syncthreads();
    for (int round = 0; round < nbp - 1; ++round) {
      for (int p = wave; p < npairs; p += 4) {
        if (!act[round * npairs + p]) continue;
        int bi, bj;
        pair_blocks(round, p, nbp, bi, bj);
        const double2 *W = Wsw + (size_t)(round * npairs + p) * JP * JP;
        int cq[4];
        double2 w[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int q = 4 * kk + lk;
          const int c = (q < JB) ? bi * JB + q : bj * JB + (q - JB);
          cq[kk] = c < C ? cmap[c] : -1;
          w[kk] = rsi::gld(W, q * JP + lr);
        }
        const int cj0 = (lr < JB) ? bi * JB + lr : bj * JB + (lr - JB);
        const int cj = cj0 < C ? cmap[cj0] : -1;
        d4 yr = {0, 0, 0, 0}, yi = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double2 x = (lr < h && cq[kk] >= 0) ? vs[lr * C + cq[kk]] : make_double2(0, 0);
          yr = mfma64(x.x, w[kk].x, yr);
          if (!kReal) {
            yr = mfma64(-x.y, w[kk].y, yr);
            yi = mfma64(x.x, w[kk].y, yi);
            yi = mfma64(x.y, w[kk].x, yi);
          }
        }
        if (cj >= 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = lk + 4 * r;
            if (row < h) vs[row * C + cj] = make_double2(yr[r], yi[r]);
          }
        }
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < nr * C; e += NT) {
      const int i = e / C, c = e - i * C;
      rsi::gst(V, (size_t)(r0 + i) + (size_t)c * ldv, vs[e]);
    }
  }
}

// cmap[0..C) = physical columns sorted by decreasing squared norm (ties by
// index); cmap[C..n) = identity (padding columns).
__device__ void order_columns(SharedSelect &s, const double *__restrict__ nrm, int C, int n, int *__restrict__ cmap) {
  const int t = threadIdx.x;
  int n2 = 2;
  while (n2 < C) n2 <<= 1;
  for (int e = t; e < n2; e += NT) {
    s.key[e] = (e < C) ? nrm[e] : -1.0;
    s.idx[e] = e;
  }
  __syncthreads();
  for (int size = 2; size <= n2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int e = t; e < n2; e += NT) {
        int partner = e ^ stride;
        if (partner > e) {
          bool desc = ((e & size) == 0);
          double ka = s.key[e], kb = s.key[partner];
          int ia = s.idx[e], ib = s.idx[partner];
          bool a_first = (ka > kb) || (ka == kb && ia < ib);
          if (desc ? !a_first : a_first) {
            s.key[e] = kb;
            s.key[partner] = ka;
            s.idx[e] = ib;
            s.idx[partner] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int e = t; e < n; e += NT) cmap[e] = (e < C) ? s.idx[e] : e;
  __syncthreads();
}

// Neighbouring singular values closer than kTie times the larger one form one
// multiplet at the truncation cut (block_select).
constexpr double kTie = 1e-4;

// Sort the C values sig (descending, ties by index) into sorted / perm and
// choose the kept count (a5).  extra: squared weight of singular values not
// listed (those beyond a subspace), added to every tail sum.  With
// disc_pending set, the discarded fraction goes there and neither *disc nor
// *dims_slot is touched (the caller commits them once the result is accepted).
__device__ void block_select(SharedSelect &s, const double *__restrict__ sig, int C, int chi_max, double cutoff,
                             int hop, int *__restrict__ perm, double *__restrict__ sorted, int *__restrict__ kept,
                             int *__restrict__ dims_slot, double *__restrict__ disc, int *__restrict__ err,
                             double extra = 0.0, double *__restrict__ disc_pending = nullptr) {
  const int t = threadIdx.x;
  int n2 = 2;
  while (n2 < C) n2 <<= 1;
  if (t == 0) {
    s.cnt_above = 0;
    s.cnt_nz = 0;
    s.bad = 0;
  }
  __syncthreads();
  for (int e = t; e < n2; e += NT) {
    double v = (e < C) ? sig[e] : -1.0;
    if (e < C && !(v >= 0.0 && v < INFINITY)) atomicOr(&s.bad, 1);
    s.key[e] = v;
    s.idx[e] = e;
  }
  __syncthreads();
  for (int size = 2; size <= n2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int e = t; e < n2; e += NT) {
        int partner = e ^ stride;
        if (partner > e) {
          bool desc = ((e & size) == 0);
          double ka = s.key[e], kb = s.key[partner];
          int ia = s.idx[e], ib = s.idx[partner];
          bool a_first = (ka > kb) || (ka == kb && ia < ib);
          if (desc ? !a_first : a_first) {
            s.key[e] = kb;
            s.key[partner] = ka;
            s.idx[e] = ib;
            s.idx[partner] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int e = t; e < n2; e += NT) s.tail[e] = (e < C) ? s.key[e] * s.key[e] : 0.0;
  if (t == 0) s.tail[n2] = 0.0;
  __syncthreads();
  for (int off = 1; off < n2; off <<= 1) {
    double v[kMaxDim / NT];
    int q = 0;
    for (int e = t; e < n2; e += NT, ++q) v[q] = (e + off < n2) ? s.tail[e + off] : 0.0;
    __syncthreads();
    q = 0;
    for (int e = t; e < n2; e += NT, ++q) s.tail[e] += v[q];
    __syncthreads();
  }
  if (extra != 0.0) {
    for (int e = t; e <= n2; e += NT) s.tail[e] += extra;
    __syncthreads();
  }
  const double W = s.tail[0];
  for (int e = t; e < C; e += NT) {
    if (e >= 1 && s.tail[e] > cutoff * W) atomicAdd(&s.cnt_above, 1);
    if (s.key[e] > 0.0) atomicAdd(&s.cnt_nz, 1);
    perm[e] = s.idx[e];
    sorted[e] = s.key[e];
  }
  __syncthreads();
  if (t == 0) {
    int k;
    if (hop) {
      k = s.cnt_nz;
    } else {
      // k = min(chi_max, k_c) over the nonzero values, then moved off a
      // multiplet: neighbours closer than kTie times the larger are one
      // multiplet and the cut never splits it (which of its vectors to keep
      // is not determined); a cut set by the cutoff moves past the multiplet
      // while chi_max allows, otherwise in front of it
      const int nz = s.cnt_nz;
      const int kc = 1 + s.cnt_above;
      k = kc < chi_max ? kc : chi_max;
      if (k > nz) k = nz;
      if (k < 1) k = 1;
      auto tie = [&](int q) { return q < nz && s.key[q - 1] - s.key[q] <= kTie * s.key[q - 1]; };
      const int kmax = chi_max < nz ? chi_max : nz;
      if (k == kc)
        while (k < kmax && tie(k)) ++k;
      while (k > 1 && tie(k)) --k;
    }
    if (k < 1) k = 1;
    if (s.bad || !(W > 0.0)) *err = 1;
    *kept = k;
    if (disc_pending) {
      *disc_pending = W > 0.0 ? s.tail[k] / W : 0.0;
    } else {
      *dims_slot = k;
      if (!hop && W > 0.0) *disc += s.tail[k] / W;
    }
  }
  __syncthreads();
}

// Phase timers of the first workgroup (thread 0 only; null when not profiling).
struct Laps {
  unsigned long long *tp;
  unsigned long long tmark;
  __device__ void lap(int slot) {
    if (tp) {
      const unsigned long long now = wall_clock64();
      tp[slot] += now - tmark;
      tmark = now;
    }
  }
};

}  // namespace



// Column norms (root) or squared norms of the rows x C matrix M (ld), one
// column per workgroup at a time, with a fixed-order reduction.
__device__ void col_norms(SharedAll &sh, const double2 *M, int ld, int rows, int C, double *out, bool root, int rank,
                          int G) {
  for (int j = rank; j < C; j += G) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < rows; i += NT) {
      double2 v = rsi::gld(M, (size_t)i + (size_t)j * ld);
      acc = fma(v.x, v.x, fma(v.y, v.y, acc));
    }
    sh.red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) sh.red[threadIdx.x] += sh.red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = root ? sqrt(sh.red[0]) : sh.red[0];
    __syncthreads();
  }
}

// Block one-sided Jacobi on Y (C x C, ld C) until a sweep rotates no pair
// (or the sweep limit).  On entry the caller's workgroups have written Y, the
// identity into V (C x C, ld C) and zeros into sweep_cnt (the first grid
// barrier inside orders those writes).  On return (behind a barrier) Y holds
// Y W and V the accumulated W.  Returns the number of sweeps.
template <bool kReal>
__device__ __noinline__ int jacobi_run(const SvdLaunch &a, Barrier &bar, SharedAll &sh, Laps &laps, double2 *Y, int C) {
  const unsigned rank = bar.rank;
  const int G = (int)bar.G;
  const int ldy = C, ldv = C;
  int nbp = (C + JB - 1) / JB;
  nbp += nbp & 1;
  if (nbp < 2) nbp = 2;
  const int npairs = nbp / 2;
  // Workgroups [0, np) do the pair rounds, ordered block by block (see
  // wait_blocks); the others (nv of them) apply the previous sweep's rotations
  // to V meanwhile, so the V update leaves the critical path.  The block
  // versions live in the second barrier block and are cleared here (every
  // workgroup has left its previous use behind a full barrier).
  const int np = G < npairs ? G : npairs, nv = G - np;
  static_assert(kMaxDim / JB + 2 <= (int)kBarBlock, "block versions must fit the barrier block");
  unsigned *ver = a.bar + kBarBlock;
  if (rank == 0)
    for (int b = threadIdx.x; b < nbp; b += NT) ver[b] = 0u;
  bar.sync();
  const double tol = a.tol_factor * sqrt((double)C) * 2.220446049250313e-16;
  int sweeps = 0, pending = -1;  // pending: active sweep whose V update is outstanding
  const size_t wsw_stride = (size_t)(nbp - 1) * npairs;  // pair slots per sweep
  const size_t cmap_stride = (size_t)nbp * JB;
  auto update_v = [&](int sw, int workers, int me) {
    sweep_update_v<kReal>(sh.pair, a.V, ldv, C, nbp, a.W + (size_t)(sw & 1) * wsw_stride * JP * JP,
                          a.act + (size_t)(sw & 1) * wsw_stride, workers, a.cmap + (sw & 1) * cmap_stride, me);
  };
  for (int sweep = 0; sweep < a.max_sweeps; ++sweep) {
    double2 *Wsw = a.W + (size_t)(sweep & 1) * wsw_stride * JP * JP;
    int *act = a.act + (size_t)(sweep & 1) * wsw_stride;
    int *cmap = a.cmap + (sweep & 1) * cmap_stride;
    // order the columns by decreasing norm for this sweep (blocks then hold
    // columns of similar size, which speeds up convergence on graded spectra)
    col_norms(sh, Y, ldy, C, C, a.cnorm, false, (int)rank, G);
    bar.sync();
    if (rank == 0) order_columns(sh.sel, a.cnorm, C, nbp * JB, cmap);
    bar.sync();
    if ((int)rank < np) {
      const unsigned base = (unsigned)sweep * (unsigned)(nbp - 1);  // every block's version at the sweep's start
      for (int round = 0; round < nbp - 1; ++round) {
        for (int p = rank; p < npairs; p += np) {
          int bi, bj;
          pair_blocks(round, p, nbp, bi, bj);
          if (np > 1) wait_blocks(ver + bi, ver + bj, base + round, a.err);
          laps.lap(2);
          const size_t slot = (size_t)round * npairs + p;
          unsigned long long *tp = (a.tprof && rank == 0) ? a.tprof : nullptr;
          const bool active = pair_work<kReal>(sh.pair, Y, ldy, C, Wsw + slot * JP * JP, C, bi, bj, tol, cmap, tp);
          if (threadIdx.x == 0) {
            act[slot] = active ? 1 : 0;
            if (active) atomicAdd(&a.sweep_cnt[sweep], 1);
          }
          __syncthreads();
          if (np > 1) publish_blocks(ver + bi, ver + bj, base + round + 1);
          laps.lap(1);
        }
      }
    } else if (pending >= 0) {
      update_v(pending, nv, rank - np);
    }
    bar.sync();
    sweeps = sweep + 1;
    const bool converged =
        __hip_atomic_load(&a.sweep_cnt[sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    if (nv == 0) {
      if (converged) break;
      update_v(sweep, G, rank);
      laps.lap(11);
    } else {
      pending = converged ? -1 : sweep;
      if (converged) break;
    }
  }
  if (pending >= 0) update_v(pending, G, rank);  // the sweep limit was reached while rotating
  bar.sync();
  return sweeps;
}

// Width of the subspace for the truncated SVD of a gate block with C columns
// whose bond held chm before the gate (0: run the full SVD).
__device__ __forceinline__ int rsi_width(const SvdLaunch &a, int C, int chm) {
  if (a.rsi_pmax <= 0 || C < a.rsi_min_cols) return 0;
  const int keep = min(a.chi_max, chm + a.rsi_grow);  // the kept vectors the bond is expected to need
  int want = (keep + a.rsi_margin + 15) & ~15;
  if (want > a.rsi_pmax) {
    // a capped subspace must still hold them and the 16 beyond the cut that
    // acceptance asks for, else the attempt could only fail
    if (a.rsi_pmax < keep + 16) return 0;
    want = a.rsi_pmax;
  }
  if (4 * want > 3 * C) return 0;
  return want;
}

// Mout <- M L^{-H} with L the Cholesky factor of M^H M (M, Mout: rows x p,
// ld rows; Mout may not be M): one Cholesky QR pass.  The Gram matrix is
// formed in kGramSplit partial sums by all workgroups and summed by all,
// workgroup 0 factors it, L^{-1} is formed by column blocks and the product
// with it is a GEMM.
// near_identity > 0: the pass is a repeat, and its Gram matrix must lie
// within that distance of the identity (max entry of the lower triangle),
// which bounds the loss of orthogonality of the result to a few units of
// round-off (Yamamoto, Nakatsukasa, Yanagisawa & Fukaya, ETNA 44 (2015) 306).
// False (on every workgroup) when the factorisation broke down or the check
// failed; a.rsi_flag[0] is then set.
template <bool kReal>
__device__ __noinline__ bool cholqr_pass(const SvdLaunch &a, Barrier &bar, SharedAll &sh, const double2 *M,
                                         double2 *Mout, int rows, int p, double2 *L, int rank, int G,
                                         double near_identity = 0.0) {
  // phase timers of the first workgroup: [26] Gram, [27] Cholesky, [28] L^{-1} and the product
  Laps laps{a.tprof && rank == 0 && threadIdx.x == 0 ? a.tprof : nullptr, (unsigned long long)wall_clock64()};
  const size_t gstride = (size_t)p * p;
  if (rank == 0 && threadIdx.x == 0)
    __hip_atomic_store((unsigned long long *)&a.rsi_scal[3], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  rsi::gemm<kReal>(sh.rg, p, p, rows, M, rows, 1, M, rows, 0, nullptr, nullptr, a.Gr, p, true, rank, G,
                   rsi::kGramSplit, gstride);
  bar.sync();
  laps.lap(26);
  if (laps.tp) laps.tp[15] += 1;  // Cholesky-QR passes
  // the partial sums, added into the first (lower triangle) by all
  // workgroups; on a repeat pass also the largest deviation from the identity
  // (a max over non-negative values, exact in any order: the bit patterns
  // order like the values, NaN above all)
  double dev = 0.0;
  for (size_t e = (size_t)rank * NT + threadIdx.x; e < gstride; e += (size_t)G * NT) {
    const int i = (int)(e % p), j = (int)(e / p);
    if (i >= j) {
      double2 g = a.Gr[e];
      for (int sp = 1; sp < rsi::kGramSplit; ++sp) {
        const double2 h = a.Gr[e + sp * gstride];
        g.x += h.x;
        g.y += h.y;
      }
      a.Gr[e] = g;
      const double d = fabs(g.x - (i == j ? 1.0 : 0.0)) + fabs(g.y);
      dev = d <= dev ? dev : d;
    }
  }
  if (near_identity > 0.0) {
    sh.red[threadIdx.x] = dev;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) {
        const double o = sh.red[threadIdx.x + off];
        sh.red[threadIdx.x] = o <= sh.red[threadIdx.x] ? sh.red[threadIdx.x] : o;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0)
      atomicMax((unsigned long long *)&a.rsi_scal[3], (unsigned long long)__double_as_longlong(sh.red[0]));
    __syncthreads();
  }
  bar.sync();
  if (rank == 0) {
    bool ok = true;
    if (near_identity > 0.0)
      ok = __longlong_as_double((long long)__hip_atomic_load((unsigned long long *)&a.rsi_scal[3], __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) <= near_identity;
    if (ok) ok = rsi::cholesky<kReal>(sh.rc, p, a.Gr, 1, 0, L, a.Ldi, laps.tp);
    if (threadIdx.x == 0 && !ok) a.rsi_flag[0] = 1;
  }
  bar.sync();
  laps.lap(27);
  if (__hip_atomic_load(&a.rsi_flag[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
  rsi::tri_inverse<kReal>(sh.rc, p, L, a.Ldi, a.Li, rank, G);
  bar.sync();
  // Mout = M (L^{-1})^H
  rsi::gemm<kReal>(sh.rg, rows, p, p, M, rows, 0, a.Li, p, 1, nullptr, nullptr, Mout, rows, false, rank, G);
  bar.sync();
  laps.lap(28);
  return true;
}

// C = op(A) B (M x N, inner K; C contiguous, ld M), then a grid barrier.
// Products with few 64 x 64 output tiles and a long inner dimension (the
// products with the gate block) cut the inner dimension into up to four
// ranges, so that more workgroups take part: the partial products go to the
// Gram scratch and are summed in a fixed order afterwards.  The cut depends
// on the shape alone, never on the number of workgroups.
template <bool kReal>
__device__ void split_gemm(const SvdLaunch &a, Barrier &bar, SharedAll &sh, int M, int N, int K,
                           const double2 *A, int lda, int opa, const double2 *B, double2 *C, int rank, int G) {
  const int tiles = ((M + rsi::kTile - 1) / rsi::kTile) * ((N + rsi::kTile - 1) / rsi::kTile);
  int ks = tiles > 0 ? min(4, max(1, 256 / tiles)) : 1;
  if (K < 256) ks = 1;
  const size_t mn = (size_t)M * N, cap = (size_t)rsi::kGramSplit * a.rsi_pmax * a.rsi_pmax;
  while (ks > 1 && (size_t)ks * mn > cap) --ks;
  if (ks == 1) {
    rsi::gemm<kReal>(sh.rg, M, N, K, A, lda, opa, B, K, 0, nullptr, nullptr, C, M, false, rank, G);
    bar.sync();
    return;
  }
  rsi::gemm<kReal>(sh.rg, M, N, K, A, lda, opa, B, K, 0, nullptr, nullptr, a.Gr, M, false, rank, G, ks, mn);
  bar.sync();
  for (size_t e = (size_t)rank * NT + threadIdx.x; e < mn; e += (size_t)G * NT) {
    double2 v = rsi::gld(a.Gr, e);
    for (int s = 1; s < ks; ++s) {
      const double2 w = rsi::gld(a.Gr, e + s * mn);
      v.x += w.x;
      v.y += w.y;
    }
    rsi::gst(C, e, v);
  }
  bar.sync();
}

// The subspace result is not used: count it and let the full SVD run.
__device__ __forceinline__ bool rsi_reject(const SvdLaunch &a, int rank) {
  if (rank == 0 && threadIdx.x == 0 && a.stats) a.stats[6] += 1;
  return false;
}

// Truncated SVD of the gate block X (R x C, R >= C) by subspace iteration
// with Rayleigh-Ritz (Halko, Martinsson & Tropp, SIAM Rev. 53 (2011) 217,
// Alg. 4.4 with Cholesky-QR orthonormalisation): from a random C x p start,
// alternate Z = orth(X V), V = orth(X^H Z); then X V = Q T (Cholesky QR
// twice), one-sided Jacobi on T^H gives T = W S U^H, and X ~ (Q W) S (V U)^H
// on the subspace.  The kept Ritz triplets are accepted when every residual
// ||X^H u_j - s_j v_j|| is below rsi_tol s_1; else, once, the iteration goes
// on for as many steps as the residual's rate of decrease needs, and if that
// fails too the full SVD takes over (X is never modified here).  Squared weight outside
// the subspace, ||X||^2 - sum_j s_j^2, joins the tail sums of the truncation
// rule.  Returns true when the gate is complete (canonical update written).
template <bool kReal>
__device__ __noinline__ bool rsi_gate(const SvdLaunch &a, Barrier &bar, SharedAll &sh, Laps &laps, int R, int C, int trans,
                         int chl, int chr, int p) {
  const int rank = (int)bar.rank, G = (int)bar.G;
  const size_t gtid = (size_t)rank * NT + threadIdx.x, gstride = (size_t)G * NT;
  const double2 *X = a.X;
  const int ldx = R;
  // the basis, its image and a scratch matrix rotate through three buffers
  double2 *Vc = a.Vr, *Zc = a.Zr, *Wk = a.Wk;
  auto swap2 = [](double2 *&x, double2 *&y) {
    double2 *t = x;
    x = y;
    y = t;
  };
  // squared column norms of X (for its Frobenius norm), random start, flags
  col_norms(sh, X, ldx, R, C, a.cnorm, false, rank, G);
  for (size_t e = gtid; e < (size_t)C * p; e += gstride)
    Vc[e] = make_double2(rsi::hash_uniform((unsigned)(e % C), (unsigned)(e / C), 0u), 0.0);
  if (gtid < 4) a.rsi_flag[gtid] = 0;
  bar.sync();
  if (rank == 0) {
    // fixed-order sum of the column norms
    double w = 0.0;
    for (int j = threadIdx.x; j < C; j += NT) w += a.cnorm[j];
    sh.red[threadIdx.x] = w;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) sh.red[threadIdx.x] += sh.red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.rsi_scal[0] = sh.red[0];
  }
  laps.lap(20);
  int iters = a.rsi_iters, done = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    for (; done < iters; ++done) {
      split_gemm<kReal>(a, bar, sh, R, p, C, X, ldx, 0, Vc, Zc, rank, G);
      if (!cholqr_pass<kReal>(a, bar, sh, Zc, Wk, R, p, a.L1, rank, G)) return rsi_reject(a, rank);
      swap2(Zc, Wk);
      split_gemm<kReal>(a, bar, sh, C, p, R, X, ldx, 1, Zc, Vc, rank, G);
      if (!cholqr_pass<kReal>(a, bar, sh, Vc, Wk, C, p, a.L1, rank, G)) return rsi_reject(a, rank);
      swap2(Vc, Wk);
    }
    laps.lap(21);
    // V orthonormal to working accuracy, then X V = Q T with T^H = L1 L2
    if (!cholqr_pass<kReal>(a, bar, sh, Vc, Wk, C, p, a.L1, rank, G, 0.5)) return rsi_reject(a, rank);
    swap2(Vc, Wk);
    split_gemm<kReal>(a, bar, sh, R, p, C, X, ldx, 0, Vc, Zc, rank, G);
    if (!cholqr_pass<kReal>(a, bar, sh, Zc, Wk, R, p, a.L1, rank, G)) return rsi_reject(a, rank);
    if (!cholqr_pass<kReal>(a, bar, sh, Wk, Zc, R, p, a.L2, rank, G, 0.5)) return rsi_reject(a, rank);
    laps.lap(22);
    // Jacobi on Y = T^H = L1 L2 (p x p), V = I
    rsi::gemm<kReal>(sh.rg, p, p, p, a.L1, p, 0, a.L2, p, 0, nullptr, nullptr, a.Y, p, false, rank, G);
    for (size_t e = gtid; e < (size_t)p * p; e += gstride)
      a.V[e] = make_double2((e % p) == (e / p) ? 1.0 : 0.0, 0.0);
    if (gtid < (size_t)a.max_sweeps) a.sweep_cnt[gtid] = 0;
    const int sweeps = jacobi_run<kReal>(a, bar, sh, laps, a.Y, p);
    laps.lap(23);
    col_norms(sh, a.Y, p, p, p, a.sig, true, rank, G);
    bar.sync();
    if (rank == 0) {
      // weight outside the subspace joins every tail sum
      double w = 0.0;
      for (int j = threadIdx.x; j < p; j += NT) w += a.sig[j] * a.sig[j];
      sh.red[threadIdx.x] = w;
      __syncthreads();
      for (int off = NT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh.red[threadIdx.x] += sh.red[threadIdx.x + off];
        __syncthreads();
      }
      const double extra = fmax(0.0, a.rsi_scal[0] - sh.red[0]);
      __syncthreads();
      if (threadIdx.x == 0 && a.stats) {
        a.stats[0] = sweeps;
        a.stats[1] = p;
        a.stats[2] = R;
      }
      block_select(sh.sel, a.sig, p, a.chi_max, a.cutoff, 0, a.perm, a.sorted, a.kept, nullptr, a.disc,
                   a.rsi_flag + 1, extra, a.rsi_scal + 1);
    }
    bar.sync();
    const int k = __hip_atomic_load(a.kept, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // left vectors Q W(:, perm), right vectors V Y(:, perm) / s
    rsi::gemm<kReal>(sh.rg, R, k, p, Zc, R, 0, a.V, p, 0, a.perm, nullptr, a.Lb, R, false, rank, G);
    rsi::gemm<kReal>(sh.rg, C, k, p, Vc, C, 0, a.Y, p, 0, a.perm, nullptr, a.Rb, C, false, rank, G);
    bar.sync();
    for (size_t e = gtid; e < (size_t)C * k; e += gstride) {
      const double inv = 1.0 / a.sorted[e / C];
      a.Rb[e] = make_double2(a.Rb[e].x * inv, a.Rb[e].y * inv);
    }
    bar.sync();
    // residuals X^H u_j - s_j v_j of the kept triplets
    split_gemm<kReal>(a, bar, sh, C, k, R, X, ldx, 1, a.Lb, a.Res, rank, G);
    for (int j = rank; j < k; j += G) {
      const double sg = a.sorted[j];
      double acc = 0.0;
      for (int i = threadIdx.x; i < C; i += NT) {
        const double2 r = a.Res[(size_t)i + (size_t)j * C], v = a.Rb[(size_t)i + (size_t)j * C];
        const double dx = r.x - sg * v.x, dy = r.y - sg * v.y;
        acc = fma(dx, dx, fma(dy, dy, acc));
      }
      sh.red[threadIdx.x] = acc;
      __syncthreads();
      for (int off = NT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh.red[threadIdx.x] += sh.red[threadIdx.x + off];
        __syncthreads();
      }
      if (threadIdx.x == 0) a.cnorm[j] = sqrt(sh.red[0]);
      __syncthreads();
    }
    bar.sync();
    if (rank == 0) {
      double r = 0.0;
      for (int j = threadIdx.x; j < k; j += NT) r = fmax(r, a.cnorm[j]);
      sh.red[threadIdx.x] = r;
      __syncthreads();
      for (int off = NT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh.red[threadIdx.x] = fmax(sh.red[threadIdx.x], sh.red[threadIdx.x + off]);
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        const double res = sh.red[0], bound = a.rsi_tol * a.sorted[0];
        a.rsi_scal[2] = res;
        // decision of this attempt (every workgroup reads its own slot, so no
        // slot is ever reset while another workgroup may still read it):
        // 0 accepted (small residuals, room in the subspace beyond the cut);
        // n > 0: run n more iterations (the residual has been falling by the
        // factor f = res^(1/done) per iteration from about 1 at the random
        // start: n iterations reach the bound); -1: hand over to the full SVD
        int verdict;
        if (a.rsi_flag[1] == 0 && res <= bound && k + 16 <= p) {
          verdict = 0;
        } else if (attempt == 0 && a.rsi_flag[1] == 0 && k + 16 <= p && res > 0.0 && bound > 0.0) {
          const double f = fmin(0.95, fmax(1e-6, pow(res / a.sorted[0], 1.0 / done)));
          const int more = (int)ceil(log(bound / res) / log(f)) + 1;
          verdict = (more >= 1 && done + more <= kRsiMaxIters) ? more : -1;
        } else {
          verdict = -1;
        }
        a.rsi_flag[2 + attempt] = verdict;
      }
    }
    bar.sync();
    laps.lap(24);
    const int verdict = __hip_atomic_load(&a.rsi_flag[2 + attempt], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (verdict == 0) {
      // ---- accepted: commit the bond dimension and discarded weight, canonical update ----
      if (rank == 0 && threadIdx.x == 0) {
        a.dims[a.k] = k;
        *a.disc += a.rsi_scal[1];
        if (a.stats) {
          a.stats[3] += 1;
          a.stats[4] += sweeps;
          a.stats[5] += 1;
          a.stats[7] += done;
        }
        if (a.alg_flops) {
          const double rr = R, cc = C;
          *a.alg_flops += (a.real ? 1.0 : 4.0) * (14.0 * rr * cc * cc + 8.0 * cc * cc * cc);
        }
      }
      double2 *Ak = a.sites[a.k], *Ak1 = a.sites[a.k + 1];
      const size_t na = (size_t)4 * chl * k, nb2 = (size_t)k * 4 * chr;
      const size_t n = na > nb2 ? na : nb2;
      for (size_t e = gtid; e < n; e += gstride) {
        if (e < na) {
          const int i = e / k, al = e % k;
          const double sg = a.sorted[al];
          double2 u = trans == 0 ? a.Lb[(size_t)i + (size_t)al * R] : a.Rb[(size_t)i + (size_t)al * C];
          if (!a.asc) u = make_double2(u.x * sg, u.y * sg);
          Ak[e] = u;
        }
        if (e < nb2) {
          const int al = e / (4 * chr), j = e % (4 * chr);
          const double sg = a.sorted[al];
          double2 v = trans == 0 ? a.Rb[(size_t)j + (size_t)al * C] : a.Lb[(size_t)j + (size_t)al * R];
          if (a.asc) v = make_double2(v.x * sg, v.y * sg);
          Ak1[e] = zconj(v);
        }
      }
      laps.lap(6);
      return true;
    }
    // rejected: more iterations from the present subspace, or give up
    if (verdict < 0) break;
    iters += verdict;
  }
  if (rank == 0 && threadIdx.x == 0 && a.stats) a.stats[6] += 1;
  return false;
}

// The whole truncated SVD / centre hop, run by G cooperating workgroups
// (group-local barriers only, so independent problems can share one launch).
//
// Gate (mode 0), on the R x C block X (R >= C; X = theta, or theta^H when
// that is taller): the columns are ordered by decreasing norm (P), X P = Q R
// by blocked Householder QR, and one-sided block Jacobi runs on Y = R^H
// (C x C): Y W = U_Y diag(sigma).  Then X = (Q W) diag(sigma) (P U_Y)^H, so
// the left vectors of X are Q W and the right ones P U_Y.  Jacobi on the
// triangular factor of a norm-ordered QR needs far fewer sweeps than on X
// itself for graded spectra (Drmac & Veselic, 2008).
// Hop (modes 1, 2): A_c = Q R (right) or A_c^H = Q R (left) by the same QR;
// the centre site takes Q (or Q^H) and the neighbour absorbs R (or R^H).
template <bool kReal>
__device__ __forceinline__ void svd_body(const SvdLaunch &a, Barrier &bar, SharedAll &sh) {
  const unsigned rank = bar.rank, G_ = bar.G;
  // phase timers (workgroup 0, thread 0): 0 setup + QR, 1 pair Gram+eig, 2 wait
  // after a round, 5 norms+select, 6 epilogue, 7 launches, 11 V update
  const unsigned long long cyc0 = clock64();
  Laps laps{a.tprof && rank == 0 && threadIdx.x == 0 ? a.tprof : nullptr, (unsigned long long)wall_clock64()};
  const bool prof = laps.tp != nullptr;
  auto lap = [&](int slot) { laps.lap(slot); };
  if (prof) a.tprof[7] += 1;
  const int G = (int)G_;
  const size_t gtid = (size_t)rank * NT + threadIdx.x, gstride = (size_t)G * NT;
  const int N = a.N;
  auto dimL = [&](int s) { return s == 0 ? 1 : ld_dim(a.dims + s - 1); };
  auto dimR = [&](int s) { return s == N - 1 ? 1 : ld_dim(a.dims + s); };
  // ---- problem shape (read before any bond dimension is rewritten) ----
  int R, C, trans = 0, chl = 1, chm = 1, chr = 1, site = a.k;
  if (a.mode == 0) {
    chl = dimL(a.k);
    chm = ld_dim(a.dims + a.k);  // the bond's dimension before the gate
    chr = dimR(a.k + 1);
    const int r = 4 * chl, c = 4 * chr;
    trans = r >= c ? 0 : 1;
    R = trans ? c : r;
    C = trans ? r : c;
  } else if (a.mode == 1) {
    chl = dimL(site);
    chm = ld_dim(a.dims + site);
    chr = dimR(site + 1);  // right dim of the neighbour
    R = 4 * chl;
    C = chm;
  } else if (a.mode == 3) {
    // spectrum of site k as a (4 chl) x chr matrix (or its adjoint when wider)
    chl = dimL(site);
    chr = dimR(site);
    const int r = 4 * chl, c = chr;
    trans = r >= c ? 0 : 1;
    R = trans ? c : r;
    C = trans ? r : c;
  } else {
    chm = ld_dim(a.dims + site - 1);
    chr = dimR(site);
    chl = dimL(site - 1);  // left dim of the neighbour
    R = 4 * chr;
    C = chm;
  }
  const int ldx = R;
  // ---- hop: load X from the site tensor; gate: order the columns ----
  auto load_hop = [&]() {
    const double2 *A = a.sites[site];
    if (a.mode == 1) {
      for (size_t e = gtid; e < (size_t)R * C; e += gstride) {
        int i = e / C, j = e % C;
        a.X[(size_t)i + (size_t)j * ldx] = A[e];
      }
    } else {  // A: chm x (4 chr)
      for (size_t e = gtid; e < (size_t)R * C; e += gstride) {
        int i = e / R, j = e % R;  // A[i][j], i < chm, j < 4 chr
        a.X[(size_t)j + (size_t)i * ldx] = zconj(A[e]);
      }
    }
  };
  // hops by Cholesky QR (twice) where it applies; false: Householder QR below
  bool hop_chol = false;
  if (a.mode == 1 || a.mode == 2) {
    load_hop();
    if (a.rsi_pmax > 0 && a.rsi_min_cols > 0 && C >= kHopCholMin && C <= a.rsi_pmax && R >= C) {
      if (rank == 0 && threadIdx.x == 0) a.rsi_flag[0] = 0;
      bar.sync();  // X, written by every workgroup, is read by every workgroup below
      hop_chol = cholqr_pass<kReal>(a, bar, sh, a.X, a.Wk, R, C, a.L1, (int)rank, G) &&
                 cholqr_pass<kReal>(a, bar, sh, a.Wk, a.X, R, C, a.L2, (int)rank, G, 0.5);
      if (hop_chol) {
        // X = Q (L1 L2)^H: Y = L1 L2 (its adjoint is the R factor), Lb = Q
        rsi::gemm<kReal>(sh.rg, C, C, C, a.L1, C, 0, a.L2, C, 0, nullptr, nullptr, a.Y, C, false, (int)rank, G);
        for (size_t e = gtid; e < (size_t)R * C; e += gstride) a.Lb[e] = a.X[e];
      } else {
        load_hop();
      }
      bar.sync();
      lap(25);
    }
  } else if (a.mode == 3) {
    const double2 *A = a.sites[site];  // (4 chl) x chr, row-major
    for (size_t e = gtid; e < (size_t)R * C; e += gstride) {
      const int i = e / chr, j = e % chr;
      if (trans == 0)
        a.X[(size_t)i + (size_t)j * ldx] = A[e];
      else
        a.X[(size_t)j + (size_t)i * ldx] = zconj(A[e]);
    }
  }
  if (a.mode == 0) {
    // wide blocks: the truncated SVD on a subspace (falls back to the full
    // SVD below when its result is not accepted)
    const int p = rsi_width(a, C, chm);
    if (p > 0 && rsi_gate<kReal>(a, bar, sh, laps, R, C, trans, chl, chr, p)) {
      if (prof) a.tprof[12] += clock64() - cyc0;
      return;
    }
  }
  if (a.mode == 0 || a.mode == 3) {
    col_norms(sh, a.X, ldx, R, C, a.cnorm, false, (int)rank, G);
    bar.sync();
    if (rank == 0) order_columns(sh.sel, a.cnorm, C, C, a.qmap);
  } else if (!hop_chol) {
    for (size_t e = gtid; e < (size_t)C; e += gstride) a.qmap[e] = (int)e;
  }
  if (!hop_chol) bar.sync();
  lap(16);
  // ---- blocked Householder QR of X P, with look-ahead: workgroup 0 applies
  // panel p to the first 16-column task (which holds panel p + 1) and factors
  // panel p + 1 at once, while the others apply panel p to the remaining tasks;
  // one barrier per panel ----
  const int nq = R < C ? R : C, nbw = qr_panel_width(R);
  auto Tpan = [&](int p) { return a.Tq + (size_t)p * kQrNbMax * kQrNbMax; };
  if (nq > 0 && !hop_chol) {
    if (rank == 0) qr_panel(sh.qr, a.X, ldx, a.qmap, R, 0, min(nbw, nq), Tpan(0));
    lap(17);
    bar.sync();
    lap(2);
  }
  for (int j0 = 0, p = 0; j0 < nq && !hop_chol; j0 += nbw, ++p) {
    const int nb = min(nbw, nq - j0);
    const int c0 = j0 + nb, ntail = C - c0, ntask = (ntail + 15) / 16;
    if (ntail <= 0) break;
    auto apply_tasks = [&](int first, int stride) {
      for (int task = first; task < ntask; task += stride)
        qr_apply_panel(sh.qr, R - j0, nb, true, a.X, ldx, j0, a.qmap + c0 + task * 16, 0,
                       min(16, ntail - task * 16));
    };
    if (rank == 0) {
      qr_load_panel(sh.qr, a.X, ldx, a.qmap, R, j0, nb, Tpan(p));
      apply_tasks(0, ntask);  // task 0 only
      lap(18);
      if (c0 < nq) {
        qr_panel(sh.qr, a.X, ldx, a.qmap, R, c0, min(nbw, nq - c0), Tpan(p + 1));
        lap(17);
      }
      if (G == 1 && ntask > 1) {
        qr_load_panel(sh.qr, a.X, ldx, a.qmap, R, j0, nb, Tpan(p));
        apply_tasks(1, 1);
        lap(18);
      }
    } else if ((int)rank < ntask) {
      qr_load_panel(sh.qr, a.X, ldx, a.qmap, R, j0, nb, Tpan(p));
      apply_tasks((int)rank, G - 1);
    }
    bar.sync();
    lap(2);
  }
  // Q Y for the columns of Lb (R rows, ncol columns): panels in reverse
  // order, each workgroup on its own column tasks (no barrier needed).  Up to
  // 512 rows a task of 8 columns stays in the upper half of the panel buffer
  // for all panels (only the reflectors stream in); beyond, 16-column tasks
  // are read and written per panel.
  auto apply_q = [&](int ncol) {
    constexpr int kTileCols = 8;
    if (R <= 64 * kQyRows) {
      // up to 1024 rows: one wavefront per column, rows in registers
      qr_form_qy_waves(sh.qr, a.X, ldx, a.qmap, R, nq, nbw, a.Tq, a.Lb, ncol, (int)rank, G);
    } else if (R * kQrNbMax <= kQrPanelElems / 2) {
      double2 *tile = sh.qr.P + kQrPanelElems / 2;  // R x kTileCols, column-major
      const int ntask = (ncol + kTileCols - 1) / kTileCols;
      for (int task = rank; task < ntask; task += G) {
        const int c0 = task * kTileCols, nc = min(kTileCols, ncol - c0);
        __syncthreads();
        for (int e = threadIdx.x; e < R * kTileCols; e += NT) {
          const int i = e % R, j = e / R;
          tile[e] = j < nc ? a.Lb[(size_t)i + (size_t)(c0 + j) * R] : make_double2(0, 0);
        }
        for (int j0 = ((nq - 1) / nbw) * nbw, p = (nq - 1) / nbw; j0 >= 0; j0 -= nbw, --p) {
          const int nb = min(nbw, nq - j0);
          qr_load_panel(sh.qr, a.X, ldx, a.qmap, R, j0, nb, a.Tq + (size_t)p * kQrNbMax * kQrNbMax);
          qr_apply_panel(sh.qr, R - j0, nb, false, tile, R, j0, nullptr, 0, nc);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < R * nc; e += NT) {
          const int i = e % R, j = e / R;
          a.Lb[(size_t)i + (size_t)(c0 + j) * R] = tile[e];
        }
      }
    } else {
      const int ntask = (ncol + 15) / 16;
      for (int task = rank; task < ntask; task += G) {
        for (int j0 = ((nq - 1) / nbw) * nbw, p = (nq - 1) / nbw; j0 >= 0; j0 -= nbw, --p) {
          const int nb = min(nbw, nq - j0);
          qr_load_panel(sh.qr, a.X, ldx, a.qmap, R, j0, nb, a.Tq + (size_t)p * kQrNbMax * kQrNbMax);
          qr_apply_panel(sh.qr, R - j0, nb, false, a.Lb, R, j0, nullptr, task * 16, min(16, ncol - task * 16));
        }
      }
    }
    lap(19);
  };
  lap(0);
  if (a.mode == 1 || a.mode == 2) {
    // ---- hop: explicit thin Q, then A_c <- Q (or Q^H), neighbour <- R A (or A R^H) ----
    const int k = nq;
    if (!hop_chol) {
      for (size_t e = gtid; e < (size_t)R * k; e += gstride) {
        const int i = e % R, jj = e / R;
        a.Lb[e] = make_double2(i == jj ? 1.0 : 0.0, 0.0);
      }
      bar.sync();
      apply_q(k);
    }
    int *dslot = (a.mode == 2) ? a.dims + (site - 1) : a.dims + site;
    if (rank == 0 && threadIdx.x == 0) {
      if (a.alg_flops) {
        // declared cost of a thin QR with Q formed: 4 R n^2 - 4 n^3 / 3 real flops, n = min(R, C),
        // four times that for complex operands
        const double rr = R, cc = k;
        *a.alg_flops += (a.real ? 1.0 : 4.0) * (4.0 * rr * cc * cc - 4.0 / 3.0 * cc * cc * cc);
      }
      if (a.stats) {
        a.stats[0] = 0;
        a.stats[1] = C;
        a.stats[2] = R;
        a.stats[5] += 1;
      }
      *a.kept = k;
    }
    bar.sync();
    if (rank == 0 && threadIdx.x == 0) *dslot = k;
    const bool right = a.mode == 1;
    double2 *Ac = a.sites[site];
    {
      const size_t na = (size_t)R * k, nz = (size_t)k * C;
      const size_t n = na > nz ? na : nz;
      for (size_t e = gtid; e < n; e += gstride) {
        if (e < na) {
          int i, al;
          if (right) {
            i = e / k;
            al = e % k;
          } else {
            al = e / R;
            i = e % R;
          }
          const double2 q = a.Lb[(size_t)i + (size_t)al * R];
          Ac[e] = right ? q : zconj(q);
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
          // R[al][m]: Householder R in the upper triangle of X, or conj(Y[m][al])
          const double2 r = m < al ? make_double2(0, 0)
                            : hop_chol ? zconj(a.Y[(size_t)m + (size_t)al * C])
                                       : a.X[(size_t)al + (size_t)m * ldx];
          a.Z[e] = right ? r : zconj(r);
        }
      }
    }
    bar.sync();
    // neighbour update: right: T = Z (k x C) * A_{c+1} (C x 4 chr);  left: T = A_{c-1} (4 chl x C) * Z (C x k)
    const double2 *Am = right ? a.Z : a.sites[site - 1];
    const double2 *Bm = right ? a.sites[site + 1] : a.Z;
    const int M = right ? k : 4 * chl, Nn = right ? 4 * chr : k, K = C;
    const int lda = K, ldb = Nn;
    const int tiles_m = (M + 63) / 64, tiles_n = (Nn + 63) / 64;
    for (int tile = rank; tile < tiles_m * tiles_n; tile += G) {
      const int i0 = (tile / tiles_n) * 64, j0 = (tile % tiles_n) * 64;
      const int t = threadIdx.x, ty = t / 16, tx = t % 16;
      double2 acc[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0, 0);
      for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int e = t + NT * q;
          int row = e / 16, kk = e % 16;
          sh.gemm.As[kk][row] =
              (i0 + row < M && k0 + kk < K) ? Am[(size_t)(i0 + row) * lda + k0 + kk] : make_double2(0, 0);
          int kb = e / 64, j = e % 64;
          sh.gemm.Bs[kb][j] = (k0 + kb < K && j0 + j < Nn) ? Bm[(size_t)(k0 + kb) * ldb + j0 + j] : make_double2(0, 0);
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
          double2 av[4], bv[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) av[i] = sh.gemm.As[kk][ty * 4 + i];
#pragma unroll
          for (int j = 0; j < 4; ++j) bv[j] = sh.gemm.Bs[kk][tx + 16 * j];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) zfma(acc[i][j], av[i], bv[j]);
        }
        __syncthreads();
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          int r = i0 + ty * 4 + i, c = j0 + tx + 16 * j;
          if (r < M && c < Nn) a.T[(size_t)r * Nn + c] = acc[i][j];
        }
    }
    bar.sync();
    double2 *dst = right ? a.sites[site + 1] : a.sites[site - 1];
    for (size_t e = gtid; e < (size_t)M * Nn; e += gstride) dst[e] = a.T[e];
    lap(6);
    if (prof) a.tprof[12] += clock64() - cyc0;
    return;
  }
  // ---- gate: Y = R^H (C x C, lower triangular), V = I ----
  double2 *Y = a.Y;
  const int ldy = C, ldv = C;
  for (size_t e = gtid; e < (size_t)C * C; e += gstride) {
    const int i = e % C, j = e / C;
    Y[e] = i >= j ? zconj(a.X[(size_t)j + (size_t)a.qmap[i] * ldx]) : make_double2(0, 0);
    a.V[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  if (gtid < (size_t)a.max_sweeps) a.sweep_cnt[gtid] = 0;
  const int sweeps = jacobi_run<kReal>(a, bar, sh, laps, Y, C);
  if (a.mode == 3) {
    // ---- spectrum only: OSEE = -sum p ln p, p = sigma^2 / sum sigma^2 (no state change) ----
    col_norms(sh, Y, ldy, C, C, a.sig, false, (int)rank, G);
    bar.sync();
    if (rank == 0) {
      double w = 0.0;
      for (int j = threadIdx.x; j < C; j += NT) w += a.sig[j];
      sh.red[threadIdx.x] = w;
      __syncthreads();
      for (int off = NT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh.red[threadIdx.x] += sh.red[threadIdx.x + off];
        __syncthreads();
      }
      const double W = sh.red[0];
      __syncthreads();
      double h = 0.0;
      for (int j = threadIdx.x; j < C; j += NT) {
        const double p = a.sig[j] / W;
        if (p > 0.0) h -= p * log(p);
      }
      sh.red[threadIdx.x] = h;
      __syncthreads();
      for (int off = NT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh.red[threadIdx.x] += sh.red[threadIdx.x + off];
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        a.aux[0] = sh.red[0];
        a.aux[1] = W;
        if (!(W > 0.0) || !(sh.red[0] >= 0.0)) atomicOr(a.err, 1);
      }
    }
    lap(5);
    if (prof) a.tprof[12] += clock64() - cyc0;
    return;
  }
  // ---- singular values, truncation select; inverse of the QR column order ----
  col_norms(sh, Y, ldy, C, C, a.sig, true, (int)rank, G);
  for (size_t e = gtid; e < (size_t)C; e += gstride) a.qinv[a.qmap[e]] = (int)e;
  bar.sync();
  int *dslot = a.dims + site;
  if (rank == 0) {
    if (threadIdx.x == 0 && a.alg_flops) {
      // declared cost of a thin SVD of an R x C block (R >= C): 14 R C^2 + 8 C^3
      // real flops (Golub & Van Loan, Golub-Reinsch count), four times that for
      // complex operands
      const double rr = R, cc = C;
      *a.alg_flops += (a.real ? 1.0 : 4.0) * (14.0 * rr * cc * cc + 8.0 * cc * cc * cc);
    }
    if (threadIdx.x == 0 && a.stats) {
      a.stats[0] = sweeps;
      a.stats[1] = C;
      a.stats[2] = R;
      a.stats[4] += sweeps;
      a.stats[5] += 1;
    }
    block_select(sh.sel, a.sig, C, a.chi_max, a.cutoff, 0, a.perm, a.sorted, a.kept, dslot, a.disc, a.err);
  }
  bar.sync();
  lap(5);
  const int k = __hip_atomic_load(a.kept, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // ---- left vectors of X: Lb = Q [W(:, perm(0:k)); 0] ----
  for (size_t e = gtid; e < (size_t)R * k; e += gstride) {
    const int i = e % R, al = e / R;
    a.Lb[e] = i < C ? a.V[(size_t)i + (size_t)a.perm[al] * ldv] : make_double2(0, 0);
  }
  bar.sync();
  apply_q(k);
  bar.sync();
  // ---- canonical update: theta = U S V^H; ascending A_k <- U, A_{k+1} <- S V^H;
  // descending A_k <- U S, A_{k+1} <- V^H.  Left vectors of X: Lb; right
  // vectors of X: row r is row qinv[r] of Y W / sigma.  X = theta^H swaps them.
  double2 *Ak = a.sites[a.k], *Ak1 = a.sites[a.k + 1];
  const size_t na = (size_t)4 * chl * k, nb2 = (size_t)k * 4 * chr;
  const size_t n = na > nb2 ? na : nb2;
  for (size_t e = gtid; e < n; e += gstride) {
    if (e < na) {
      const int i = e / k, al = e % k;
      const double sg = a.sorted[al];
      double2 u;
      if (trans == 0) {
        u = a.Lb[(size_t)i + (size_t)al * R];
      } else {
        const double2 y = Y[(size_t)a.qinv[i] + (size_t)a.perm[al] * ldy];
        u = make_double2(y.x / sg, y.y / sg);
      }
      if (!a.asc) u = make_double2(u.x * sg, u.y * sg);
      Ak[e] = u;
    }
    if (e < nb2) {
      const int al = e / (4 * chr), j = e % (4 * chr);
      const double sg = a.sorted[al];
      double2 v;
      if (trans == 0) {
        const double2 y = Y[(size_t)a.qinv[j] + (size_t)a.perm[al] * ldy];
        v = make_double2(y.x / sg, y.y / sg);
      } else {
        v = a.Lb[(size_t)j + (size_t)al * R];
      }
      if (a.asc) v = make_double2(v.x * sg, v.y * sg);
      Ak1[e] = zconj(v);
    }
  }
  lap(6);
  if (prof) a.tprof[12] += clock64() - cyc0;
}

// Columns of the launch's QR / Jacobi problem, from the current bond dims (the
// shape svd_body derives).
__device__ int svd_cols(const SvdLaunch &a) {
  const int N = a.N, k = a.k;
  auto dimL = [&](int s) { return s == 0 ? 1 : ld_dim(a.dims + s - 1); };
  auto dimR = [&](int s) { return s == N - 1 ? 1 : ld_dim(a.dims + s); };
  switch (a.mode) {
    case 0: return min(4 * dimL(k), 4 * dimR(k + 1));
    case 1: return ld_dim(a.dims + k);
    case 3: return min(4 * dimL(k), dimR(k));
    default: return ld_dim(a.dims + k - 1);
  }
}

// The host launches the grid its bond capacities could need; every workgroup
// computes the same effective count from the actual dims, and the surplus
// leaves before touching the barrier (whose member count is the effective one).
// kReal selects the real-arithmetic form (a separate instantiation, so the
// complex kernel carries none of it).
template <bool kReal>
__global__ __launch_bounds__(NT) void svd_persistent_kernel(SvdLaunch a) {
  __shared__ SharedAll sh;
  const unsigned want = (unsigned)svd_workgroups(svd_cols(a));
  const unsigned G = gridDim.x < want ? gridDim.x : want;
  if (blockIdx.x >= G) return;
  Barrier bar{a.bar, a.bar + 8 * 32, a.bar + 8 * 32 + 32, a.err, G, blockIdx.x, 0u};
  svd_body<kReal>(a, bar, sh);
}

// A batch may mix real-form and complex chains: one out-of-line call site
// serves both instantiations.
__device__ __noinline__ void svd_body_any(const SvdLaunch &a, Barrier &bar, SharedAll &sh) {
  if (a.real)
    svd_body<true>(a, bar, sh);
  else
    svd_body<false>(a, bar, sh);
}

// ---------------------------------------------------------------------------
// Batched form: one cooperative launch runs one Trotter layer of many chains.
// Workgroup b serves chain block_group[b] as member block_rank[b] of its
// group_size[g] workgroups; the group walks the layer's gates in order, each
// preceded by the centre hops that bring the orthogonality centre onto the
// bond, as the single-chain executor does (the same device code per op).
// The layer of chain g is the global layer L n_g + j (L = 3, 6 or 7 layers
// per step, n_g = its step count); it runs ascending when that index is even,
// i.e. when step_parity[g] + local_step + j is even (the host passes zeros
// for both when L is even).  Bonds b =
// parity, parity + 2, ... < N - 1 get the gate in table slot `slot`.
// ---------------------------------------------------------------------------
union SharedBatch {
  SharedAll all;
  ContractLds<double> cd;
  ContractLds<float> cf;
  double2 env[2][kMaxDim / 4];
};

__global__ __launch_bounds__(NT) void batch_layer_kernel(const BatchChain *__restrict__ chains,
                                                         const int *__restrict__ block_group,
                                                         const int *__restrict__ block_rank,
                                                         const int *__restrict__ group_size, int local_step,
                                                         int j, int parity, int slot, int last_layer) {
  __shared__ SharedBatch sh;
  const int g = block_group[blockIdx.x];
  const unsigned rank = block_rank[blockIdx.x], G = group_size[g];
  // the chain's launch record lives in LDS (mode, k, asc change per op)
  __shared__ SvdLaunch L;
  if (threadIdx.x == 0) L = chains[g].L;
  __syncthreads();
  const double2 *gates = chains[g].gates;
  int *centre_p = chains[g].centre;
  const int precision = chains[g].precision;
  Barrier bar{L.bar, L.bar + 8 * 32, L.bar + 8 * 32 + 32, L.err, G, rank, 0u};
  const int N = L.N;
  const int asc = ((chains[g].step_parity + local_step + j) & 1) == 0;
  int centre = ld_dim(centre_p);
  const int nbonds = parity > N - 2 ? 0 : (N - 2 - parity) / 2 + 1;
  // ops in order: for each bond of the layer, the hops that bring the centre
  // onto it, then the gate; one svd_body call site serves both kinds
  int q = 0;
  while (q < nbonds) {
    const int b = asc ? parity + 2 * q : parity + 2 * (nbonds - 1 - q);
    const int target = centre <= b ? b : b + 1;
    const bool gate = centre == target;
    if (gate) {
      const double2 *Gt = gates + ((size_t)b * kGateSlots + slot) * 256;
      const int chl = b == 0 ? 1 : ld_dim(L.dims + b - 1), chr = b + 1 == N - 1 ? 1 : ld_dim(L.dims + b + 1);
      const int tx = (chr + 15) / 16, ntiles = tx * ((chl + 15) / 16);
      for (int t = rank; t < ntiles; t += G) {
        if (precision == LMPO_FP32_CONTRACT)
          contract_tile<float>(sh.cf, L.sites, L.dims, N, b, Gt, L.X, t % tx, t / tx);
        else if (precision == LMPO_FP64_REAL)
          contract_tile<double, true>(sh.cd, L.sites, L.dims, N, b, Gt, L.X, t % tx, t / tx);
        else
          contract_tile<double>(sh.cd, L.sites, L.dims, N, b, Gt, L.X, t % tx, t / tx);
      }
    }
    if (threadIdx.x == 0) {
      L.mode = gate ? 0 : (centre < target ? 1 : 2);
      L.k = gate ? b : centre;
      L.asc = gate ? asc : 0;
    }
    bar.sync();
    svd_body_any(L, bar, sh.all);
    bar.sync();
    if (gate) {
      centre = asc ? b + 1 : b;
      ++q;
    } else {
      centre += centre < target ? 1 : -1;
    }
  }
  if (last_layer && chains[g].force_trace) {
    // rho <- rho / tr(rho): trace by the first workgroup, scaling of the
    // centre site by all, with the single-chain kernels' arithmetic
    if (rank == 0) {
      const double2 tr = chain_trace(L.sites, L.dims, N, sh.env[0], sh.env[1]);
      if (threadIdx.x == 0) *chains[g].tr = tr;
    }
    bar.sync();
    const double2 inv = zinv_exact(chains[g].tr[0]);
    const int cl = centre == 0 ? 1 : ld_dim(L.dims + centre - 1), cr = centre == N - 1 ? 1 : ld_dim(L.dims + centre);
    double2 *A = L.sites[centre];
    const size_t n = (size_t)cl * 4 * cr;
    for (size_t e = (size_t)rank * NT + threadIdx.x; e < n; e += (size_t)G * NT) A[e] = zmul_exact(A[e], inv);
  }
  if (rank == 0) {
    if (threadIdx.x == 0) *centre_p = centre;
    if (chains[g].dims_out)
      for (int i = threadIdx.x; i < N - 1; i += NT) chains[g].dims_out[i] = ld_dim(L.dims + i);
  }
}

static int g_grid = 0;

int svd_grid_size() {
  if (g_grid) return g_grid;
  int dev = 0, cus = 0, occ = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, svd_persistent_kernel<false>, NT, 0);
  if (cus <= 0) cus = 1;
  if (occ <= 0) occ = 1;
  g_grid = cus;  // one workgroup per compute unit
  if (g_grid > cus * occ) g_grid = cus * occ;
  return g_grid;
}

// The persistent kernels need every workgroup of their grid resident at once
// (they meet at grid barriers).  The grids are sized to the co-resident
// capacity (one workgroup per compute unit), and by default the launch is
// cooperative, so that the runtime guarantees residency.  With the environment
// variable LMPO_PLAIN_LAUNCH=1 the same grid goes through an ordinary launch:
// rocprofv3's counter collection intercepts ordinary dispatches only (its
// --pmc mode fails inside hipLaunchCooperativeKernel).  On an otherwise idle
// device the grid is then resident as well; should it not be, the bounded
// waits of the grid barrier end the kernel with an error instead of a hang.
static bool plain_launch() {
  static const bool plain = [] {
    const char *v = std::getenv("LMPO_PLAIN_LAUNCH");
    return v && v[0] == '1';
  }();
  return plain;
}

static hipError_t launch_persistent(const void *fn, int grid, void **args, hipStream_t s) {
  if (plain_launch()) return hipLaunchKernel(fn, dim3(grid), dim3(NT), args, 0, s);
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(NT), args, 0, s);
}

hipError_t launch_svd_persistent(hipStream_t s, const SvdLaunch &L, int grid) {
  hipError_t e = hipMemsetAsync(L.bar, 0, kBarWords * sizeof(unsigned), s);
  if (e != hipSuccess) return e;
  SvdLaunch a = L;
  void *args[] = {&a};
  const void *fn = L.real ? reinterpret_cast<const void *>(svd_persistent_kernel<true>)
                         : reinterpret_cast<const void *>(svd_persistent_kernel<false>);
  return launch_persistent(fn, grid, args, s);
}

int batch_grid_size() {
  int dev = 0, cus = 0, occ = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_layer_kernel, NT, 0);
  if (cus <= 0) cus = 1;
  if (occ <= 0) occ = 1;
  return cus * occ;
}

hipError_t launch_batch_layer(hipStream_t s, const BatchChain *d_chains, const int *d_block_group,
                              const int *d_block_rank, const int *d_group_size, int total_blocks, unsigned *bar_base,
                              size_t bar_words, int local_step, int j, int parity, int slot, int last_layer) {
  hipError_t e = hipMemsetAsync(bar_base, 0, bar_words * sizeof(unsigned), s);
  if (e != hipSuccess) return e;
  void *args[] = {(void *)&d_chains, (void *)&d_block_group, (void *)&d_block_rank, (void *)&d_group_size,
                  &local_step, &j, &parity, &slot, &last_layer};
  return launch_persistent(reinterpret_cast<const void *>(batch_layer_kernel), total_blocks, args, s);
}

}  // namespace lmpo
