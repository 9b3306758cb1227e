// Blocked Householder QR for the persistent SVD kernel (gfx950).
//
// A = Q R for a complex R x C matrix held column-major in global memory,
// logical column j at physical column qmap[j] (the caller's pivoting order).
// Each reflector is Hermitian and unitary, H = I - tau v v^H with real tau and
// v(leading) = 1: for a column x with leading entry alpha = |alpha| e^{i phi},
// H x = -e^{i phi} ||x|| e_1 (the sign choice that avoids cancellation; the
// diagonal of R is therefore complex).  Reflectors are grouped in panels of nb
// and kept in compact WY form, H_1 ... H_nb = I - V T V^H with T upper
// triangular (Schreiber & Van Loan, 1989).  A panel is factored by one
// workgroup with the panel in LDS; the trailing columns are updated with
// A <- (I - V T^H V^H) A by all workgroups, 16 columns per task.  The same
// panel update with T (not T^H), applied panel by panel in reverse order,
// forms Q Y.
#pragma once

#include <hip/hip_runtime.h>

namespace lmpo {

constexpr int NT_QR = 256;            // threads per workgroup
constexpr int kQrNbMax = 8;           // reflectors per panel: 8 up to 1024 rows, 4 beyond
constexpr int kQrPanelElems = 8192;   // panel elements held in LDS (rows x width)

struct SharedQR {
  double2 P[kQrPanelElems];           // panel (factor) or reflectors (update), column-major, ld = m
  double2 T[kQrNbMax][kQrNbMax];      // the panel's T
  double2 Wt[kQrNbMax][17];           // T^H (V^H Y) or T (V^H Y) of one 16-column task
  double2 red[4][kQrNbMax];           // per-wave partial sums
  double sred[4];
};

namespace qr {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ void cfma(double2 &acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ void cfmac(double2 &acc, double2 a, double2 b) {  // acc += conj(a) b
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// Lane exchange within rows of 16 lanes through DPP (no LDS round trip).
template <int kCtrl>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), kCtrl, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over each row of 16 lanes, the same bits in every lane of the row:
// pairs (quad_perm 1,0,3,2), quads (2,3,0,1), half rows (row_half_mirror),
// rows (row_mirror).
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  v += dpp_mov<0x140>(v);
  return v;
}

__device__ __forceinline__ double lane_read(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of the wave, the same bits in every lane.
__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

}  // namespace qr

// Panel width for an R-row matrix (the panel of R x width elements fits in LDS).
__device__ __host__ inline int qr_panel_width(int R) { return R <= 1024 ? 8 : 4; }

// 1/x and sqrt(x) from the hardware estimates plus Newton steps (x > 0 normal).
__device__ __forceinline__ double qr_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  return y * fma(-x, y, 2.0);
}
__device__ __forceinline__ double qr_sqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return x * y;
}

// Factor logical columns [j0, j0 + nb) of A (rows j0 .. R-1) with this
// workgroup: on return those columns of X hold R's entries on and above the
// diagonal and the reflectors below it; Tg (nb x nb, row-major) holds T.
// Per column c, with x = a_c below the diagonal and v = (1, x r), r the
// reflector's scale: every quantity the column needs comes from one
// workgroup reduction over the unscaled x, ||x||^2, d_q = x^H a_q (later
// columns q) and e_j = v_j^H x (earlier reflectors j), since
// w_q = v^H a_q = conj(r) d_q + a_q[c] and z_j = v_j^H v = r e_j + conj(v_j[c]);
// then one pass scales x and updates the later columns.  Two workgroup
// barriers per column.
__device__ __noinline__ void qr_panel(SharedQR &s, double2 *__restrict__ X, int ldx, const int *__restrict__ qmap, int R, int j0,
                         int nb, double2 *__restrict__ Tg) {
  using namespace qr;
  const int m = R - j0, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  __syncthreads();  // the panel's columns may just have been written by other threads of this workgroup
  for (int c = 0; c < nb; ++c) {
    const double2 *col = X + (size_t)qmap[j0 + c] * ldx + j0;
    for (int i = t; i < m; i += NT_QR) s.P[c * m + i] = col[i];
  }
  if (t < kQrNbMax * kQrNbMax) s.T[t / kQrNbMax][t % kQrNbMax] = make_double2(0, 0);
  __syncthreads();
  const int nd = nb - 1;
  for (int c = 0; c < nb; ++c) {
    double2 *pc = s.P + c * m;
    // row c of the panel: written before the last barrier, rewritten after the next one
    const double2 al = pc[c];
    double2 rowc[kQrNbMax];
#pragma unroll
    for (int q = 0; q < kQrNbMax; ++q)
      if (q < nd) rowc[q] = s.P[(q < c ? q : q + 1) * m + c];
    double ss = 0.0;
    double2 acc[kQrNbMax];
#pragma unroll
    for (int q = 0; q < kQrNbMax; ++q) acc[q] = make_double2(0, 0);
    for (int i = c + 1 + t; i < m; i += NT_QR) {
      const double2 x = pc[i];
      ss = fma(x.x, x.x, fma(x.y, x.y, ss));
#pragma unroll
      for (int q = 0; q < kQrNbMax; ++q) {
        if (q < nd) {
          const int cq = q < c ? q : q + 1;
          const double2 e = s.P[cq * m + i];
          if (cq < c)
            cfmac(acc[q], e, x);  // e_j: conj(v_j[i]) x_i
          else
            cfmac(acc[q], x, e);  // d_q: conj(x_i) a_q[i]
        }
      }
    }
    // workgroup sums: DPP inside the waves, then the four waves in a fixed order
    ss = wave_sum(ss);
#pragma unroll
    for (int q = 0; q < kQrNbMax; ++q) {
      if (q < nd) {
        acc[q].x = wave_sum(acc[q].x);
        acc[q].y = wave_sum(acc[q].y);
      }
    }
    if (lane == 0) {
      s.sred[wave] = ss;
#pragma unroll
      for (int q = 0; q < kQrNbMax; ++q)
        if (q < nd) s.red[wave][q] = acc[q];
    }
    __syncthreads();
    ss = (s.sred[0] + s.sred[1]) + (s.sred[2] + s.sred[3]);
#pragma unroll
    for (int q = 0; q < kQrNbMax; ++q) {
      if (q < nd) {
        const double2 a = s.red[0][q], b = s.red[1][q], cc = s.red[2][q], d = s.red[3][q];
        acc[q] = make_double2((a.x + b.x) + (cc.x + d.x), (a.y + b.y) + (cc.y + d.y));
      }
    }
    double tau = 0.0;
    double2 beta = al, rinv = make_double2(0, 0);
    if (ss > 1e-290) {  // (normal range for the estimates; smaller columns are left as they are)
      const double a2 = fma(al.x, al.x, al.y * al.y);
      const double nrm = qr_sqrt(a2 + ss);
      const double aa = a2 > 1e-290 ? qr_sqrt(a2) : 0.0;
      const double iaa = aa > 0.0 ? qr_rcp(aa) : 0.0;
      const double2 ph = aa > 0.0 ? make_double2(al.x * iaa, al.y * iaa) : make_double2(1.0, 0.0);
      const double d = aa + nrm;
      tau = d * qr_rcp(nrm);
      beta = make_double2(-ph.x * nrm, -ph.y * nrm);
      const double id = qr_rcp(d);
      rinv = make_double2(ph.x * id, -ph.y * id);  // 1 / (e^{i phi} (|alpha| + ||x||))
    }
    // w_q (later columns) and z_j (earlier reflectors), uniform over the workgroup
#pragma unroll
    for (int q = 0; q < kQrNbMax; ++q) {
      if (q < nd) {
        if (q < c) {
          const double2 u = cmul(rinv, acc[q]);
          acc[q] = make_double2(u.x + rowc[q].x, u.y - rowc[q].y);  // r e_j + conj(v_j[c])
        } else {
          const double2 u = cmulc(rinv, acc[q]);
          acc[q] = make_double2(u.x + rowc[q].x, u.y + rowc[q].y);  // conj(r) d_q + a_q[c]
        }
      }
    }
    if (tau != 0.0) {
      for (int i = c + t; i < m; i += NT_QR) {
        double2 v = make_double2(1.0, 0.0);
        if (i > c) {
          v = cmul(pc[i], rinv);
          pc[i] = v;
        }
#pragma unroll
        for (int q = 0; q < kQrNbMax; ++q) {
          if (q < nd && q >= c) {  // column q + 1
            const double2 u = cmul(v, make_double2(tau * acc[q].x, tau * acc[q].y));
            double2 *pq = s.P + (q + 1) * m;
            pq[i] = make_double2(pq[i].x - u.x, pq[i].y - u.y);
          }
        }
      }
    }
    if (t == 0) pc[c] = beta;
    // T(0:c, c) = -tau T(0:c, 0:c) z (row r by thread r), T(c, c) = tau
    if (t < c) {
      double2 a = make_double2(0, 0);
#pragma unroll
      for (int j = 0; j < kQrNbMax; ++j)
        if (j >= t && j < c) cfma(a, s.T[t][j], acc[j]);
      s.T[t][c] = make_double2(-tau * a.x, -tau * a.y);
    } else if (t == c) {
      s.T[c][c] = make_double2(tau, 0.0);
    }
    __syncthreads();
  }
  for (int c = 0; c < nb; ++c) {
    double2 *col = X + (size_t)qmap[j0 + c] * ldx + j0;
    for (int i = t; i < m; i += NT_QR) col[i] = s.P[c * m + i];
  }
  if (t < nb * nb) Tg[t] = s.T[t / nb][t % nb];
  __syncthreads();
}

// Load the reflectors of the panel at logical columns [j0, j0 + nb) (rows
// j0 .. R-1, unit diagonal, zeros above) and its T into LDS.
__device__ __noinline__ void qr_load_panel(SharedQR &s, const double2 *__restrict__ X, int ldx, const int *__restrict__ qmap, int R,
                              int j0, int nb, const double2 *__restrict__ Tg) {
  const int m = R - j0, t = threadIdx.x;
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    const double2 *col = X + (size_t)qmap[j0 + c] * ldx + j0;
    for (int i = t; i < m; i += NT_QR)
      s.P[c * m + i] = i < c ? make_double2(0, 0) : (i == c ? make_double2(1.0, 0.0) : col[i]);
  }
  if (t < nb * nb) s.T[t / nb][t % nb] = Tg[t];
  __syncthreads();
}

// Y[row0 + i][cols] <- (I - V M V^H) Y for the 16 (or fewer) columns
// cols[0 .. ncols) of Y (col0 + 0 .. ncols when cols is null), rows i < m, with M = T^H (adjoint = true, the
// factorisation) or T (forming Q).  V and T from qr_load_panel.  Column c of
// Y is at Y + ycol(c) * ldy.  Thread (j = t / 16, g = t % 16) works on column
// j, rows g, g + 16, ... (coalesced); the reduction over g stays in the wave.
__device__ __noinline__ void qr_apply_panel(SharedQR &s, int m, int nb, bool adjoint, double2 *__restrict__ Y, int ldy, int row0,
                               const int *cols, int col0, int ncols) {
  using namespace qr;
  const int t = threadIdx.x, j = t >> 4, g = t & 15;
  double2 *ycol = (j < ncols) ? Y + (size_t)(cols ? cols[j] : col0 + j) * ldy + row0 : nullptr;
  double2 acc[kQrNbMax];
#pragma unroll
  for (int q = 0; q < kQrNbMax; ++q) acc[q] = make_double2(0, 0);
  if (ycol) {
    for (int i = g; i < m; i += 16) {
      const double2 y = ycol[i];
#pragma unroll
      for (int q = 0; q < kQrNbMax; ++q)
        if (q < nb) cfmac(acc[q], s.P[q * m + i], y);
    }
  }
#pragma unroll
  for (int q = 0; q < kQrNbMax; ++q) {
    acc[q].x = row16_sum(acc[q].x);  // the 16 lanes of column j form one DPP row
    acc[q].y = row16_sum(acc[q].y);
  }
  __syncthreads();
  if (g == 0 && j < 16) {
    // Wt[:, j] = M (V^H y_j); q unrolled so that acc stays in registers
    for (int r = 0; r < nb; ++r) {
      double2 a = make_double2(0, 0);
#pragma unroll
      for (int q = 0; q < kQrNbMax; ++q) {
        if (q < nb) {
          if (adjoint) {
            if (q <= r) cfmac(a, s.T[q][r], acc[q]);  // (T^H)[r][q] = conj(T[q][r]), upper T
          } else {
            if (q >= r) cfma(a, s.T[r][q], acc[q]);
          }
        }
      }
      s.Wt[r][j] = a;
    }
  }
  __syncthreads();
  if (ycol) {
    for (int i = g; i < m; i += 16) {
      double2 y = ycol[i];
#pragma unroll
      for (int q = 0; q < kQrNbMax; ++q) {
        if (q < nb) {
          const double2 u = cmul(s.P[q * m + i], s.Wt[q][j]);
          y.x -= u.x;
          y.y -= u.y;
        }
      }
      ycol[i] = y;
    }
  }
}

// Q Y for columns [0, ncol) of Y (R <= 64 kQyRows rows, column-major, ld R),
// Q = H_1 ... H_nq from the factored panels (reflectors below the diagonal of
// X at physical columns qmap[.], T of panel p at Tq + p * kQrNbMax^2).  The
// workgroup takes four columns at a time (columns 4 rank + w, + 4 G, ...), one
// per wavefront; lane l keeps rows l, l + 64, ... of its column in registers
// through every panel (applied in reverse order, Y <- (I - V T V^H) Y), while
// the workgroup stages each panel's reflectors and T in LDS once for its four
// columns.  Each column's arithmetic is the same whatever the number of
// workgroups.
constexpr int kQyRows = 16;
__device__ __noinline__ void qr_form_qy_waves(SharedQR &s, const double2 *__restrict__ X, int ldx,
                                              const int *__restrict__ qmap, int R, int nq, int nbw,
                                              const double2 *__restrict__ Tq, double2 *__restrict__ Y, int ncol,
                                              int rank, int G) {
  using namespace qr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int npan = (nq + nbw - 1) / nbw;
  for (int c0 = 4 * rank; c0 < ncol; c0 += 4 * G) {
    const int c = c0 + wave;
    const bool active = c < ncol;
    double2 y[kQyRows];
    double2 *yc = Y + (size_t)(active ? c : 0) * R;
#pragma unroll
    for (int r = 0; r < kQyRows; ++r) {
      const int i = lane + 64 * r;
      y[r] = (active && i < R) ? yc[i] : make_double2(0, 0);
    }
    for (int p = npan - 1; p >= 0; --p) {
      const int j0 = p * nbw, nb = min(nbw, nq - j0), m = R - j0;
      qr_load_panel(s, X, ldx, qmap, R, j0, nb, Tq + (size_t)p * kQrNbMax * kQrNbMax);
      if (active) {
        // w = V^H y over rows >= j0 (the staged panel holds the unit diagonal and zeros above it)
        double2 w[kQrNbMax];
#pragma unroll
        for (int q = 0; q < kQrNbMax; ++q) w[q] = make_double2(0, 0);
#pragma unroll
        for (int r = 0; r < kQyRows; ++r) {
          const int i = lane + 64 * r - j0;
          if (i >= 0 && i < m) {
#pragma unroll
            for (int q = 0; q < kQrNbMax; ++q)
              if (q < nb) cfmac(w[q], s.P[q * m + i], y[r]);
          }
        }
#pragma unroll
        for (int q = 0; q < kQrNbMax; ++q) {
          w[q].x = wave_sum(w[q].x);
          w[q].y = wave_sum(w[q].y);
        }
        double2 u[kQrNbMax];
#pragma unroll
        for (int rr = 0; rr < kQrNbMax; ++rr) {
          double2 a = make_double2(0, 0);
#pragma unroll
          for (int q = 0; q < kQrNbMax; ++q)
            if (rr < nb && q < nb && q >= rr) cfma(a, s.T[rr][q], w[q]);
          u[rr] = a;
        }
#pragma unroll
        for (int r = 0; r < kQyRows; ++r) {
          const int i = lane + 64 * r - j0;
          if (i >= 0 && i < m) {
#pragma unroll
            for (int q = 0; q < kQrNbMax; ++q) {
              if (q < nb) {
                const double2 t = cmul(s.P[q * m + i], u[q]);
                y[r].x -= t.x;
                y[r].y -= t.y;
              }
            }
          }
        }
      }
    }
    if (active) {
#pragma unroll
      for (int r = 0; r < kQyRows; ++r) {
        const int i = lane + 64 * r;
        if (i < R) yc[i] = y[r];
      }
    }
  }
  __syncthreads();
}

}  // namespace lmpo
