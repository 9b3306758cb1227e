// Host-side model: per-bond Lindblad generators in the normalised Pauli basis
// and their exponentials (FP64).
//
// The Lindbladian of Eq. (dtrho), with H of Eq. (H0), K of Eq. (K_def) (one
// term J (s+ s- + s- s+) + Jz/2 sz sz per coupled pair) and the dissipators
// Eqs. (D0) (jump s+ = |0><1|, relaxation to s^z = +1), (D1) (jump s-) and
// (D2) (jump s^z), is split into bond terms L_b; on-site terms of a site are
// shared equally among the bonds that touch it, so that sum_b L_b = L.
//
// L_b is a superoperator on two qubits.  In the orthonormal basis
// B_ab = P_a (x) P_b, P_a = sigma^a / sqrt(2), a in (1, x, y, z) (the basis of
// Eq. (mpo_def) normalised), its matrix is
//     (L_b)[ab][cd] = Tr( B_ab L_b[B_cd] ),
// which we evaluate literally by applying L_b to each basis operator.  The
// propagator exp(x L_b) uses Pade-13 scaling and squaring (N. J. Higham,
// "The scaling and squaring method for the matrix exponential revisited",
// SIAM J. Matrix Anal. Appl. 26 (2005) 1179-1193).
#include "lmpo_internal.h"

#include <cmath>
#include <cstring>

namespace lmpo {

namespace {

using C = std::complex<double>;

struct M2 {  // 2x2 complex
  C a[2][2];
};
struct M4 {  // 4x4 complex, index 2*k_i + k_j for two qubits
  C a[4][4];
};

M2 pauli2(int which) {
  M2 m{};
  switch (which) {
    case 0: m.a[0][0] = 1; m.a[1][1] = 1; break;                  // 1
    case 1: m.a[0][1] = 1; m.a[1][0] = 1; break;                  // sigma^x
    case 2: m.a[0][1] = C(0, -1); m.a[1][0] = C(0, 1); break;     // sigma^y
    case 3: m.a[0][0] = 1; m.a[1][1] = -1; break;                 // sigma^z
  }
  return m;
}

M2 sigma_plus() {  // (sigma^x + i sigma^y)/2 = |0><1|
  M2 m{};
  m.a[0][1] = 1;
  return m;
}
M2 sigma_minus() {
  M2 m{};
  m.a[1][0] = 1;
  return m;
}

M2 scale(const M2 &x, C f) {
  M2 r = x;
  for (auto &row : r.a)
    for (auto &v : row) v *= f;
  return r;
}
M2 add(const M2 &x, const M2 &y) {
  M2 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r.a[i][j] = x.a[i][j] + y.a[i][j];
  return r;
}

M4 kron(const M2 &x, const M2 &y) {
  M4 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 2; ++l) r.a[2 * i + k][2 * j + l] = x.a[i][j] * y.a[k][l];
  return r;
}
M4 zero4() { return M4{}; }
M4 add4(const M4 &x, const M4 &y) {
  M4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) r.a[i][j] = x.a[i][j] + y.a[i][j];
  return r;
}
M4 scale4(const M4 &x, C f) {
  M4 r = x;
  for (auto &row : r.a)
    for (auto &v : row) v *= f;
  return r;
}
M4 mul4(const M4 &x, const M4 &y) {
  M4 r{};
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 4; ++j) r.a[i][j] += x.a[i][k] * y.a[k][j];
  return r;
}
M4 dagger4(const M4 &x) {
  M4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) r.a[i][j] = std::conj(x.a[j][i]);
  return r;
}
C trace4(const M4 &x) { return x.a[0][0] + x.a[1][1] + x.a[2][2] + x.a[3][3]; }

M2 onsite_h(const ModelHost &m, int s, double w) {
  M2 h = scale(pauli2(1), 0.5 * w * m.hx[s]);
  h = add(h, scale(pauli2(2), 0.5 * w * m.hy[s]));
  h = add(h, scale(pauli2(3), 0.5 * w * m.hz[s]));
  return h;
}

// Apply the bond Lindbladian to the two-qubit operator E.
M4 apply_lindblad(const M4 &H, const std::vector<M4> &jumps, const M4 &E) {
  M4 out = scale4(add4(mul4(H, E), scale4(mul4(E, H), -1.0)), C(0, -1));
  for (const M4 &L : jumps) {
    M4 Ld = dagger4(L);
    M4 LdL = mul4(Ld, L);
    out = add4(out, mul4(mul4(L, E), Ld));
    out = add4(out, scale4(add4(mul4(LdL, E), mul4(E, LdL)), -0.5));
  }
  return out;
}

// ---- dense complex n x n helpers for the Pade approximant ----
void matmul(int n, const C *a, const C *b, C *c) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      C acc = 0;
      for (int k = 0; k < n; ++k) acc += a[i * n + k] * b[k * n + j];
      c[i * n + j] = acc;
    }
}

// Solve A X = B (n x n, column count n) by Gaussian elimination with partial pivoting.
bool solve(int n, std::vector<C> A, std::vector<C> &B) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    double best = std::abs(A[col * n + col]);
    for (int r = col + 1; r < n; ++r)
      if (std::abs(A[r * n + col]) > best) {
        best = std::abs(A[r * n + col]);
        piv = r;
      }
    if (best == 0.0) return false;
    if (piv != col)
      for (int j = 0; j < n; ++j) {
        std::swap(A[col * n + j], A[piv * n + j]);
        std::swap(B[col * n + j], B[piv * n + j]);
      }
    C inv = 1.0 / A[col * n + col];
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      C f = A[r * n + col] * inv;
      if (f == C(0)) continue;
      for (int j = 0; j < n; ++j) {
        A[r * n + j] -= f * A[col * n + j];
        B[r * n + j] -= f * B[col * n + j];
      }
    }
  }
  for (int r = 0; r < n; ++r) {
    C inv = 1.0 / A[r * n + r];
    for (int j = 0; j < n; ++j) B[r * n + j] *= inv;
  }
  return true;
}

}  // namespace

// exp(A) for a dense n x n complex matrix (row-major), Pade-13 with scaling
// and squaring (Higham 2005, Algorithm 2.3 with m = 13 always).
bool expm_pade13(int n, const std::complex<double> *Ain, std::complex<double> *out) {
  static const double b[14] = {64764752532480000.0, 32382376266240000.0, 7771770303897600.0,
                               1187353796428800.0,  129060195264000.0,   10559470521600.0,
                               670442572800.0,      33522128640.0,       1323241920.0,
                               40840800.0,          960960.0,            16380.0,
                               182.0,               1.0};
  const double theta13 = 5.371920351148152;
  double norm1 = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += std::abs(Ain[i * n + j]);
    norm1 = std::max(norm1, s);
  }
  int sq = 0;
  if (norm1 > theta13) sq = (int)std::ceil(std::log2(norm1 / theta13));
  const double f = std::ldexp(1.0, -sq);
  const size_t nn = (size_t)n * n;
  std::vector<C> A(nn), A2(nn), A4(nn), A6(nn), T(nn), U(nn), V(nn), I(nn, C(0));
  for (size_t i = 0; i < nn; ++i) A[i] = Ain[i] * f;
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  matmul(n, A.data(), A.data(), A2.data());
  matmul(n, A2.data(), A2.data(), A4.data());
  matmul(n, A4.data(), A2.data(), A6.data());
  // U = A [A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I]
  for (size_t i = 0; i < nn; ++i) T[i] = b[13] * A6[i] + b[11] * A4[i] + b[9] * A2[i];
  matmul(n, A6.data(), T.data(), U.data());
  for (size_t i = 0; i < nn; ++i) U[i] += b[7] * A6[i] + b[5] * A4[i] + b[3] * A2[i] + b[1] * I[i];
  matmul(n, A.data(), U.data(), T.data());
  U = T;
  // V = A6 (b12 A6 + b10 A4 + b8 A2) + b6 A6 + b4 A4 + b2 A2 + b0 I
  for (size_t i = 0; i < nn; ++i) T[i] = b[12] * A6[i] + b[10] * A4[i] + b[8] * A2[i];
  matmul(n, A6.data(), T.data(), V.data());
  for (size_t i = 0; i < nn; ++i) V[i] += b[6] * A6[i] + b[4] * A4[i] + b[2] * A2[i] + b[0] * I[i];
  std::vector<C> P(nn), Q(nn);
  for (size_t i = 0; i < nn; ++i) {
    P[i] = V[i] + U[i];
    Q[i] = V[i] - U[i];
  }
  if (!solve(n, Q, P)) return false;  // P <- Q^{-1} P = r13(A)
  for (int s = 0; s < sq; ++s) {
    matmul(n, P.data(), P.data(), T.data());
    P.swap(T);
  }
  for (size_t i = 0; i < nn; ++i) out[i] = P[i];
  return true;
}

// 16x16 generator of bond b in the basis B_ab = P_a (x) P_b (index 4a + b).
void bond_generator_pauli(const ModelHost &m, int bond, std::complex<double> *Lout) {
  const int i = m.bonds[2 * bond], j = m.bonds[2 * bond + 1];
  const double wi = 1.0 / m.degree[i], wj = 1.0 / m.degree[j];
  const M2 I2 = pauli2(0), Z = pauli2(3), Sp = sigma_plus(), Sm = sigma_minus();
  M4 H = scale4(add4(kron(Sp, Sm), kron(Sm, Sp)), m.J[bond]);
  H = add4(H, scale4(kron(Z, Z), 0.5 * m.Jz[bond]));
  H = add4(H, kron(onsite_h(m, i, wi), I2));
  H = add4(H, kron(I2, onsite_h(m, j, wj)));
  std::vector<M4> jumps;
  auto site_jumps = [&](int s, double w, bool left) {
    const double rates[3] = {m.g0[s], m.g1[s], m.g2[s]};
    const M2 ops[3] = {Sp, Sm, Z};
    for (int r = 0; r < 3; ++r) {
      if (rates[r] == 0.0) continue;
      M2 op = scale(ops[r], std::sqrt(w * rates[r]));
      jumps.push_back(left ? kron(op, I2) : kron(I2, op));
    }
  };
  site_jumps(i, wi, true);
  site_jumps(j, wj, false);
  const double inv_sqrt2 = 1.0 / std::sqrt(2.0);
  M4 basis[16];
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 4; ++c)
      basis[4 * a + c] = kron(scale(pauli2(a), inv_sqrt2), scale(pauli2(c), inv_sqrt2));
  for (int col = 0; col < 16; ++col) {
    M4 image = apply_lindblad(H, jumps, basis[col]);
    for (int row = 0; row < 16; ++row) Lout[row * 16 + col] = trace4(mul4(basis[row], image));
  }
}

void unitary_channel_pauli(const std::complex<double> *U, std::complex<double> *G) {
  M4 u;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) u.a[r][c] = U[4 * r + c];
  const M4 ud = dagger4(u);
  const double inv_sqrt2 = 1.0 / std::sqrt(2.0);
  M4 basis[16];
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 4; ++c)
      basis[4 * a + c] = kron(scale(pauli2(a), inv_sqrt2), scale(pauli2(c), inv_sqrt2));
  for (int col = 0; col < 16; ++col) {
    const M4 image = mul4(mul4(u, basis[col]), ud);
    for (int row = 0; row < 16; ++row) G[row * 16 + col] = trace4(mul4(basis[row], image));
  }
}

void swap_pauli(std::complex<double> *G) {
  for (int e = 0; e < 256; ++e) G[e] = 0.0;
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 4; ++c) G[(4 * c + a) * 16 + (4 * a + c)] = 1.0;
}

}  // namespace lmpo
