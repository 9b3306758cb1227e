// Building blocks of the subspace-iteration truncated SVD (gfx950): complex
// FP64 GEMM tiles on the matrix cores, a Cholesky factorisation and a
// row-parallel triangular solve (Cholesky QR), and a counter-based random
// start.  All are device functions run by the workgroups of a persistent
// launch between grid barriers; every result is independent of the number
// of workgroups (tiles and rows are computed whole by one workgroup, in a
// fixed order).
#pragma once

#include <hip/hip_runtime.h>

namespace lmpo {
namespace rsi {

typedef double d4v __attribute__((ext_vector_type(4)));

// Global-memory accesses with the address space stated, so that callees that
// receive generic pointers still issue global (not flat) loads and stores.
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const dv2 gcv2;
typedef __attribute__((address_space(1))) dv2 gv2;
__device__ __forceinline__ double2 gld(const double2 *p, size_t i) {
  const dv2 v = ((gcv2 *)p)[i];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void gst(double2 *p, size_t i, double2 v) { ((gv2 *)p)[i] = dv2{v.x, v.y}; }
__device__ __forceinline__ d4v mma(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// LDS ordering among the lanes of one wavefront (its LDS operations execute
// in order): compiler fence plus a wait for outstanding LDS traffic.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kTile = 64;   // output tile side of the GEMM (one workgroup)
constexpr int kKc = 16;     // inner dimension per LDS stage
constexpr int kPanel = 16;  // Cholesky / inverse block width
constexpr int kGramSplit = 8;  // inner-dimension split of the Gram matrices

struct SharedGemm {
  double2 As[2][kKc][kTile + 1];  // op(A)[m][k] stored as [k][m], two stages
  double2 Bs[2][kKc][kTile + 1];  // op(B)[k][n] stored as [k][n]
};
// Cholesky and the triangular inverse work on subspaces of at most kMaxP vectors.
constexpr int kMaxP = 384;
constexpr int kNT = 256;  // threads per workgroup
struct SharedChol {
  double2 P[kPanel][kMaxP];          // Cholesky: the block column, P[c][i]; inverse: M's block column
  double2 part[4][kPanel][kPanel];   // per-wave partial products
  double2 Ld[kPanel][kPanel + 1];    // diagonal block of the factor
  double2 Mi[kPanel][kPanel + 1];    // its inverse (or a 16 x 16 right-hand side)
  int fail;
  int next;  // next row block of the look-ahead update
};

// Operand access: op 0 = as stored (column-major, element (i, j) at
// M[i + j ld]), op 1 = conjugate transpose (element (i, j) = conj(M[j + i ld])).
__device__ __forceinline__ double2 ld_op(const double2 *__restrict__ M, int ld, int op, int i, int j) {
  if (op == 0) return gld(M, (size_t)i + (size_t)j * ld);
  const double2 v = gld(M, (size_t)j + (size_t)i * ld);
  return make_double2(v.x, -v.y);
}

// C = op_a(A) op_b(B) (M x N, inner K), C column-major with ld ldc.
// bcol (op_b = 0 only): logical column n of B is physical column bcol[n].
// cscale: output column n is multiplied by cscale[n].  lower_only: only tiles
// touching the lower triangle (the Gram matrices feeding Cholesky).
// ksplit > 1: the inner dimension is cut into ksplit ranges and range s
// writes its partial product to C + s * cstride (the reader sums them).
// 64 x 64 output tiles, each wavefront a 32 x 32 quarter (2 x 2 blocks of
// 16 x 16 on the matrix cores); operands staged through LDS 16 deep, the next
// stage's global loads issued before the present stage's products.  Tasks
// rank, rank + G, ... of this workgroup; no barrier inside.
template <bool kReal>
__device__ void gemm(SharedGemm &sh, int M, int N, int K, const double2 *__restrict__ A, int lda, int opa,
                     const double2 *__restrict__ B, int ldb, int opb, const int *__restrict__ bcol,
                     const double *__restrict__ cscale, double2 *__restrict__ C, int ldc, bool lower_only, int rank,
                     int G, int ksplit = 1, size_t cstride = 0) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int mo = 32 * (wave & 1), no = 32 * (wave >> 1);
  const int tm = (M + kTile - 1) / kTile, tn = (N + kTile - 1) / kTile;
  const int kper = ((K + ksplit - 1) / ksplit + kKc - 1) / kKc * kKc;
  for (int task = rank; task < tm * tn * ksplit; task += G) {
    const int tile = task / ksplit, ks = task % ksplit;
    const int i0 = (tile % tm) * kTile, j0 = (tile / tm) * kTile;
    if (lower_only && i0 + kTile <= j0) continue;
    const int kb = ks * kper, ke = min(K, kb + kper);
    // complex products with three real MFMAs (Gauss): t1 = a.x b.x, t2 = a.y b.y,
    // t3 = (a.x + a.y)(b.x + b.y); real part t1 - t2, imaginary t3 - t1 - t2
    d4v t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) t1[x][y] = t2[x][y] = t3[x][y] = d4v{0, 0, 0, 0};
    if (ke <= kb) {
      // an empty inner range (split beyond K): zero partial product
      double2 *Cs = C + (size_t)ks * cstride;
      for (int e = t; e < kTile * kTile; e += 256) {
        const int m = i0 + (e & 63), n = j0 + (e >> 6);
        if (m < M && n < N) Cs[(size_t)m + (size_t)n * ldc] = make_double2(0, 0);
      }
      continue;
    }
    // global -> registers for the stage starting at k0: every load is issued
    // (indices clamped into the operand) and out-of-range values are zeroed
    // afterwards, so that no branch forces the loads to complete early
    // (raw values are masked only when they are stashed, after the products
    // of the present stage, so that no wait for them comes earlier)
    double2 ra[4], rb[4];
    bool oka[4], okb[4];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int m, k;
        if (opa == 0) {
          m = t & 63;
          k = (t >> 6) + 4 * q;
        } else {
          k = t & 15;
          m = (t >> 4) + 16 * q;
        }
        oka[q] = i0 + m < M && k0 + k < ke;
        ra[q] = ld_op(A, lda, opa, min(i0 + m, M - 1), min(k0 + k, ke - 1));
        int n;
        if (opb == 0) {
          k = t & 15;
          n = (t >> 4) + 16 * q;
        } else {
          n = t & 63;
          k = (t >> 6) + 4 * q;
        }
        okb[q] = j0 + n < N && k0 + k < ke;
        const int nn = min(j0 + n, N - 1);
        rb[q] = ld_op(B, ldb, opb, min(k0 + k, ke - 1), bcol ? bcol[nn] : nn);
      }
    };
    auto stash = [&](int buf) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 va = oka[q] ? ra[q] : make_double2(0, 0);
        const double2 vb = okb[q] ? rb[q] : make_double2(0, 0);
        if (opa == 0)
          sh.As[buf][(t >> 6) + 4 * q][t & 63] = va;
        else
          sh.As[buf][t & 15][(t >> 4) + 16 * q] = va;
        if (opb == 0)
          sh.Bs[buf][t & 15][(t >> 4) + 16 * q] = vb;
        else
          sh.Bs[buf][(t >> 6) + 4 * q][t & 63] = vb;
      }
    };
    __syncthreads();  // the previous task may still read both stages
    fetch(kb);
    stash(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += kKc) {
      const bool more = k0 + kKc < ke;
      if (more) fetch(k0 + kKc);
#pragma unroll
      for (int kk = 0; kk < kKc; kk += 4) {
        double2 a[2], b[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) a[x] = sh.As[buf][kk + lk][mo + 16 * x + lr];
#pragma unroll
        for (int y = 0; y < 2; ++y) b[y] = sh.Bs[buf][kk + lk][no + 16 * y + lr];
        double sa[2], sb[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) sa[x] = a[x].x + a[x].y;
#pragma unroll
        for (int y = 0; y < 2; ++y) sb[y] = b[y].x + b[y].y;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            t1[x][y] = mma(a[x].x, b[y].x, t1[x][y]);
            if (!kReal) {
              t2[x][y] = mma(a[x].y, b[y].y, t2[x][y]);
              t3[x][y] = mma(sa[x], sb[y], t3[x][y]);
            }
          }
      }
      if (more) {
        stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
      }
    }
    // lane holds D[lk + 4 r][lr] of each 16 x 16 block
    double2 *Cs = C + (size_t)ks * cstride;
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int n = j0 + no + 16 * y + lr;
      if (n < N) {
        const double sc = cscale ? cscale[n] : 1.0;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = i0 + mo + 16 * x + lk + 4 * r;
            if (m < M) {
              const double re = kReal ? t1[x][y][r] : t1[x][y][r] - t2[x][y][r];
              const double im = kReal ? 0.0 : t3[x][y][r] - t1[x][y][r] - t2[x][y][r];
              gst(Cs, (size_t)m + (size_t)n * ldc, make_double2(re * sc, im * sc));
            }
          }
      }
    }
  }
}

__device__ __forceinline__ double rdlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wavefront 0: Cholesky factor L_d of the nb x nb diagonal block P[c][r]
// (r, c < nb, lower part; identity beyond nb) and its inverse M_d.  Lane l
// holds row r = l % 16 of the columns q, q + 4, q + 8, q + 12 (q = l / 16) of
// both.  Step c finishes column c of L_d (right-looking, the column then
// broadcast through LDS for the update of the columns right of it) and row
// c of M_d (forward substitution: that row broadcast likewise for the rows
// below it), so the two run side by side in 16 steps.  L_d goes to sh.Ld,
// M_d to sh.Mi and to Ldinv[j0 / 16].  Sets sh.fail when a pivot is not
// positive and finite.
template <bool kReal>
__device__ __noinline__ void factor_diag_block(SharedChol &sh, int nb, int j0, int p,
                                                  double2 *__restrict__ Ldinv) {
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
  double xr[4], xi[4], mr[4], mi[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = q + 4 * t;
    const double2 v = (r < nb && c <= r) ? sh.P[c][r] : make_double2(0, 0);
    xr[t] = v.x;
    xi[t] = kReal ? 0.0 : v.y;
    mr[t] = c == r ? 1.0 : 0.0;
    mi[t] = 0.0;
  }
  double2 *cbuf = &sh.part[0][0][0];  // column c of L_d (two buffers of 16)
  double2 *rbuf = &sh.part[1][0][0];  // row c of M_d
#pragma unroll
  for (int c = 0; c < kPanel; ++c) {
    const int cq = c & 3, ct = c >> 2;
    const double dd = rdlane(xr[ct], c + 16 * cq);
    const bool good = dd > 0.0 && dd < INFINITY;
    if (c < nb && lane == 0 && !good) sh.fail = 1;
    const double d = (c < nb && good) ? sqrt(dd) : 1.0;
    const double inv = 1.0 / d;
    double2 *cb = cbuf + 16 * (c & 1), *rb = rbuf + 16 * (c & 1);
    if (q == cq) {
      if (r > c) {
        xr[ct] *= inv;
        xi[ct] = kReal ? 0.0 : xi[ct] * inv;
      } else {
        xr[ct] = r == c ? d : 0.0;
        xi[ct] = 0.0;
      }
      cb[r] = make_double2(xr[ct], xi[ct]);
    }
    if (r == c) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        mr[t] *= inv;
        mi[t] *= inv;
        rb[q + 4 * t] = make_double2(mr[t], mi[t]);
      }
    }
    wave_lds_sync();
    if (c + 1 < kPanel) {
      const double2 lrc = cb[r];  // L[r][c]
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int s = q + 4 * t;
        if (s > c) {
          // L: column s -= L[r][c] conj(L[s][c])
          const double2 y = cb[s];
          xr[t] -= lrc.x * y.x + lrc.y * y.y;
          if (!kReal) xi[t] -= lrc.y * y.x - lrc.x * y.y;
        }
      }
      if (r > c) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          // M: row r -= L[r][c] M[c][j]
          const double2 m = rb[q + 4 * t];
          mr[t] -= lrc.x * m.x - lrc.y * m.y;
          if (!kReal) mi[t] -= lrc.x * m.y + lrc.y * m.x;
        }
      }
    }
  }
  double2 *Dst = Ldinv + (size_t)(j0 / kPanel) * kPanel * kPanel;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = q + 4 * t;
    sh.Ld[r][c] = c <= r ? make_double2(xr[t], xi[t]) : make_double2(0, 0);
    const double2 v = make_double2(mr[t], kReal ? 0.0 : mi[t]);
    sh.Mi[r][c] = v;
    gst(Dst, r + c * kPanel, v);
  }
}

// Cholesky factorisation G = L L^H of the Hermitian p x p matrix G (the sum
// of nsplit partial matrices G + s * gstride; lower triangle read,
// column-major, ld p) by one workgroup: L (ld p) receives the factor with
// zeros above the diagonal.  Left-looking in blocks of 16 columns with one
// block of look-ahead: while wavefront 0 factors the diagonal block of panel
// n and inverts it (factor_diag_block), the wavefronts (wavefront 0 once done,
// row blocks handed out through an LDS counter) bring panel n + 1 up to date
// against every finished column but panel n's, on the matrix cores (operands
// straight from the cache, the next four inner steps loaded while the present
// four are multiplied; complex products as three real MFMAs), and leave
// G - that sum in L's columns of panel n + 1; then the rows below panel n's
// diagonal block are that block's inverse applied on the matrix cores, and
// panel n + 1 takes panel n's columns as its last update step into LDS.
// Ldinv receives the inverses of the diagonal blocks (16 x 16 each,
// column-major).  Returns false when a pivot is not positive and finite.
template <bool kReal>
__device__ bool cholesky(SharedChol &sh, int p, const double2 *__restrict__ Gm, int nsplit, size_t gstride,
                         double2 *__restrict__ L, double2 *__restrict__ Ldinv, unsigned long long *tp = nullptr) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  if (t == 0) {
    sh.fail = 0;
    sh.next = 0;
  }
  // phase timers (thread 0, when tp is set): [29] diagonal block beside the
  // next panel's update, [30] the next panel's last update step, [31] rows below
  unsigned long long tm = tp && t == 0 ? (unsigned long long)wall_clock64() : 0ull;
  auto lap = [&](int slot) {
    if (tp && t == 0) {
      const unsigned long long now = wall_clock64();
      tp[slot] += now - tm;
      tm = now;
    }
  };
  auto gsum = [&](size_t off) {
    double2 g = gld(Gm, off);
    for (int sp = 1; sp < nsplit; ++sp) {
      const double2 h = gld(Gm, off + sp * gstride);
      g.x += h.x;
      g.y += h.y;
    }
    return g;
  };
  // t += L[jn + 16 blk + lr][k] conj(L[jn + lr][k]) over k in [klo, khi)
  // (khi - klo a multiple of 16); lane ends with rows lk + 4 r, column lr
  auto accumulate = [&](int jn, int blk, int klo, int khi, d4v &t1, d4v &t2, d4v &t3) {
    const int iac = min(jn + 16 * blk + lr, p - 1), ibc = min(jn + lr, p - 1);
    double2 a[4], b[4], an[4], bn[4];
    auto load = [&](int k0, double2 *ax, double2 *bx) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = min(k0 + 4 * q + lk, p - 1);
        ax[q] = gld(L, (size_t)iac + (size_t)k * p);
        bx[q] = gld(L, (size_t)ibc + (size_t)k * p);
      }
    };
    auto step = [&](const double2 *ax, const double2 *bx) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        t1 = mma(ax[q].x, bx[q].x, t1);
        if (!kReal) {
          t2 = mma(ax[q].y, bx[q].y, t2);
          t3 = mma(ax[q].x + ax[q].y, bx[q].x - bx[q].y, t3);
        }
      }
    };
    load(klo, a, b);
    int k0 = klo;
    for (; k0 + 16 < khi; k0 += 32) {
      load(k0 + 16, an, bn);
      step(a, b);
      load(k0 + 32, a, b);
      step(an, bn);
    }
    if (k0 < khi) step(a, b);
  };
  auto value = [&](const d4v &t1, const d4v &t2, const d4v &t3, int r, double2 g) {
    return kReal ? make_double2(g.x - t1[r], 0.0)
                 : make_double2(g.x - (t1[r] + t2[r]), g.y - (t3[r] - t1[r] + t2[r]));
  };
  // panel 0 is G itself
  {
    const int nb0 = min(kPanel, p);
    for (int blk = wave; 16 * blk < p; blk += 4) {
      if (lr < nb0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * blk + lk + 4 * r;
          if (i < p) sh.P[lr][i] = gsum((size_t)i + (size_t)lr * p);
        }
      }
    }
  }
  __syncthreads();
  for (int j0 = 0; j0 < p; j0 += kPanel) {
    const int nb = min(kPanel, p - j0), rows = p - j0;
    const int j1 = j0 + kPanel, rows1 = p - j1, nb1 = min(kPanel, rows1);
    // wavefront 0 factors the diagonal block while the others (and wavefront 0
    // once done) bring the next panel up to date with every finished column
    // but this panel's, leaving G - that sum in L's next-panel columns
    if (wave == 0) factor_diag_block<kReal>(sh, nb, j0, p, Ldinv);
    if (rows1 > 0) {
      for (;;) {
        int bk = 0;
        if (lane == 0) bk = atomicAdd(&sh.next, 1);
        bk = __builtin_amdgcn_readfirstlane(bk);
        if (16 * bk >= rows1) break;
        d4v t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
        if (j0 > 0) accumulate(j1, bk, 0, j0, t1, t2, t3);
        if (lr < nb1) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * bk + lk + 4 * r;
            if (i < rows1) {
              const size_t off = (size_t)(j1 + i) + (size_t)(j1 + lr) * p;
              gst(L, off, value(t1, t2, t3, r, gsum(off)));
            }
          }
        }
      }
    }
    __syncthreads();
    lap(29);
    // rows below the diagonal block: L[j0 + 16 + i][j0 + c] = sum_k P[k][16 + i] conj(Mi[c][k])
    for (int blk = wave; 16 + 16 * blk < rows; blk += 4) {
      const int i0 = 16 + 16 * blk;
      d4v t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < kPanel; kk += 4) {
        const int k = kk + lk;
        const double2 a = (i0 + lr < rows && k < nb) ? sh.P[k][i0 + lr] : make_double2(0, 0);
        const double2 m = (lr < nb && k < nb) ? sh.Mi[lr][k] : make_double2(0, 0);
        const double2 b = make_double2(m.x, -m.y);
        t1 = mma(a.x, b.x, t1);
        if (!kReal) {
          t2 = mma(a.y, b.y, t2);
          t3 = mma(a.x + a.y, b.x + b.y, t3);
        }
      }
      if (lr < nb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + lk + 4 * r;
          if (i < rows)
            gst(L, (size_t)(j0 + i) + (size_t)(j0 + lr) * p,
                kReal ? make_double2(t1[r], 0.0) : make_double2(t1[r] - t2[r], t3[r] - t1[r] - t2[r]));
        }
      }
    }
    for (int e = t; e < nb * (j0 + nb); e += kNT) {
      const int c = e / (j0 + nb), i = e % (j0 + nb);
      double2 v = make_double2(0, 0);
      if (i >= j0 + c) v = sh.Ld[i - j0][c];
      gst(L, (size_t)i + (size_t)(j0 + c) * p, v);
    }
    __syncthreads();
    lap(31);
    // the next panel's last step: this panel's columns
    if (rows1 > 0) {
      for (int blk = wave; 16 * blk < rows1; blk += 4) {
        d4v t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
        accumulate(j1, blk, j0, j1, t1, t2, t3);
        if (lr < nb1) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * blk + lk + 4 * r;
            if (i < rows1) sh.P[lr][i] = value(t1, t2, t3, r, gld(L, (size_t)(j1 + i) + (size_t)(j1 + lr) * p));
          }
        }
      }
    }
    if (t == 0) sh.next = 0;
    __syncthreads();
    lap(30);
  }
  return sh.fail == 0;
}

// M = L^{-1} for the lower triangular L (p x p, ld p; M likewise, zeros
// above the diagonal), given the inverses of L's 16 x 16 diagonal blocks
// (Ldinv, from the factorisation).  Column blocks of 16 are independent
// (L M_J = E_J); workgroup rank takes blocks rank, rank + G, ...  Inside a
// block, forward substitution by 16-row blocks: M[I][J] = L_II^{-1} (delta_IJ
// - sum_{J <= K < I} L[I][K] M[K][J]), the sum on the matrix cores (the four
// wavefronts split the inner range, partial products summed in LDS) and the
// product with L_II^{-1} by wavefront 0.  No barrier inside.
template <bool kReal>
__device__ void tri_inverse(SharedChol &sh, int p, const double2 *__restrict__ L, const double2 *__restrict__ Ldinv,
                            double2 *__restrict__ Mi, int rank, int G) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nblk = (p + kPanel - 1) / kPanel;
  for (int J = rank; J < nblk; J += G) {
    const int J0 = J * kPanel, nj = min(kPanel, p - J0);
    // sh.P[c][i]: M[J0 + i][J0 + c]
    for (int I = J; I < nblk; ++I) {
      const int I0 = I * kPanel, ni = min(kPanel, p - I0);
      // wavefront 0's operand of the last product, L_II^{-1}, loaded now so
      // that its latency overlaps the partial products
      double2 dv[4];
      if (wave == 0) {
        const double2 *Di = Ldinv + (size_t)I * kPanel * kPanel;
#pragma unroll
        for (int q = 0; q < 4; ++q) dv[q] = gld(Di, lr + (4 * q + lk) * kPanel);
      }
      __syncthreads();
      if (I > J) {
        // complex products with three real MFMAs (Gauss): real t1 - t2,
        // imaginary t3 - t1 - t2
        d4v t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
        // wave w takes the 16-wide inner slices w, w + 4, ... (four steps of
        // four, their loads issued together)
        for (int k0 = J0 + 16 * wave; k0 < I0; k0 += 64) {
          // (a clamped row only feeds rows of the partial product that are
          // masked when the right-hand side is formed)
          double2 a[4];
          const int ic = min(I0 + lr, p - 1);
#pragma unroll
          for (int q = 0; q < 4; ++q) a[q] = gld(L, (size_t)ic + (size_t)(k0 + 4 * q + lk) * p);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double2 b = sh.P[lr][k0 + 4 * q + lk - J0];  // B[lk][lr] = M[k][J0 + lr]
            t1 = mma(a[q].x, b.x, t1);
            if (!kReal) {
              t2 = mma(a[q].y, b.y, t2);
              t3 = mma(a[q].x + a[q].y, b.x + b.y, t3);
            }
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
          sh.part[wave][lk + 4 * r][lr] = kReal ? make_double2(t1[r], 0.0)
                                                : make_double2(t1[r] - t2[r], t3[r] - t1[r] - t2[r]);
        __syncthreads();
      }
      {
        // right-hand side delta_IJ - sum into sh.Ld (row r, column c)
        const int r = t & 15, c = t >> 4;
        double2 v = make_double2(I == J && r == c && r < ni ? 1.0 : 0.0, 0.0);
        if (I > J) {
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            v.x -= sh.part[w][r][c].x;
            v.y -= sh.part[w][r][c].y;
          }
        }
        sh.Ld[r][c] = (r < ni && c < nj) ? v : make_double2(0, 0);
      }
      __syncthreads();
      if (wave == 0) {
        // M[I][J] = L_II^{-1} rhs
        d4v t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = 4 * q + lk;
          const double2 a = (lr < ni && k < ni) ? dv[q] : make_double2(0, 0);  // A[lr][lk]
          const double2 b = sh.Ld[k][lr];                                      // B[lk][lr]
          t1 = mma(a.x, b.x, t1);
          if (!kReal) {
            t2 = mma(a.y, b.y, t2);
            t3 = mma(a.x + a.y, b.x + b.y, t3);
          }
        }
        if (lr < nj) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = lk + 4 * r;
            if (row < ni)
              sh.P[lr][I0 - J0 + row] = kReal ? make_double2(t1[r], 0.0)
                                              : make_double2(t1[r] - t2[r], t3[r] - t1[r] - t2[r]);
          }
        }
      }
    }
    __syncthreads();
    for (int e = t; e < nj * p; e += kNT) {
      const int c = e / p, i = e % p;
      gst(Mi, (size_t)i + (size_t)(J0 + c) * p, i >= J0 ? sh.P[c][i - J0] : make_double2(0, 0));
    }
  }
}

// Counter-based uniform deviate in [-1, 1) from (i, j, seed): the 64-bit
// finaliser of SplitMix64 (Steele, Lea & Flood, 2014) applied to the packed
// index, top 53 bits as the fraction.
__device__ __forceinline__ double hash_uniform(unsigned i, unsigned j, unsigned seed) {
  unsigned long long z = ((unsigned long long)i << 32 | j) + 0x9e3779b97f4a7c15ULL * (seed + 1ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

}  // namespace rsi
}  // namespace lmpo
