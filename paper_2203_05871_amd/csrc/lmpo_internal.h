// Internal declarations shared by the host executor and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <string>
#include <vector>

#include "../../include/lmpo.h"

namespace lmpo {

// Model parameters copied from the caller (Sec. 2.1 of the paper).
struct ModelHost {
  int N = 0, nb = 0;
  std::vector<int> bonds;  // [nb][2]
  std::vector<double> J, Jz, hx, hy, hz, g0, g1, g2;
  std::vector<int> degree;  // bonds touching each site
};

bool expm_pade13(int n, const std::complex<double> *A, std::complex<double> *out);
void bond_generator_pauli(const ModelHost &m, int bond, std::complex<double> *L);
// 16x16 superoperators in the Pauli-product basis B_ab = P_a (x) P_b (index 4a + b):
// rho -> U rho U^+ for a two-qubit unitary U (row-major 4x4, basis |k_i k_j>,
// index 2 k_i + k_j), and the exchange of the two sites.
void unitary_channel_pauli(const std::complex<double> *U, std::complex<double> *G);
void swap_pauli(std::complex<double> *G);

// Block one-sided Jacobi: columns are processed in blocks of JB, two blocks
// (JP columns) per workgroup and round.
constexpr int JB = 8;
constexpr int JP = 2 * JB;
constexpr int kMaxDim = 2048;  // largest block side (4 chi) the sort handles
constexpr int kOseeRows = kMaxDim / 4;  // largest bond the OSEE co-state kernel takes
constexpr int kGateSlots = 12;  // gates per bond: the time fractions of orders 2, 3 and 4

// Workgroups that serve one persistent SVD or hop whose Jacobi/QR works on C
// columns: one per Jacobi pair of a round, and from 4 pairs up as many again
// to update V behind the rounds.  The host sizes launches from the bond
// capacities; the kernel trims itself to this count from the actual dims.
__host__ __device__ inline int svd_workgroups(int C) {
  int nbp = (C + JB - 1) / JB;
  nbp += nbp & 1;
  const int npairs = nbp / 2 > 1 ? nbp / 2 : 1;
  return npairs >= 4 ? 2 * npairs : npairs;
}

// ---- kernel launchers (kernels.hip, svd.hip) ----
void launch_contract_gate(hipStream_t s, int precision, double2 *const *sites, const int *dims, int N, int k,
                          int cap_l, int cap_r, const double2 *G, double2 *X);

// One persistent cooperative launch: mode 0 = truncated SVD + canonical update
// of the two-site block on bond k (X filled by the contraction); mode 1/2 =
// exact centre hop right/left from site k; mode 3 = singular values of site k
// as a (4 chi_l) x chi_r matrix and their entropy (no change of the state).
struct SvdLaunch {
  int mode, k, N, asc, chi_max, max_sweeps;
  int real;  // real-arithmetic form: every operand has zero imaginary part
  double cutoff, tol_factor;
  double2 *const *sites;
  int *dims;
  double2 *X, *V, *W, *Z, *T;
  double2 *Y;   // C x C Jacobi matrix (R^H of the QR)
  double2 *Lb;  // left vectors of X, or the hop's explicit Q (R x k)
  double2 *Tq;  // T factors of the QR panels, kQrNbMax^2 each
  int *qmap;    // QR column order (logical -> physical column of X)
  int *qinv;    // its inverse
  double *aux;  // mode 3 results: (entropy, total squared weight)
  int *act;
  int *cmap;
  double *cnorm;
  int *sweep_cnt;
  double *sig, *sorted;
  int *perm, *kept, *err, *stats;
  double *disc;
  unsigned *bar;
  unsigned long long *tprof;
  double *alg_flops;
  // Subspace-iteration truncated SVD of wide gate blocks (mode 0): used when
  // the block has at least rsi_min_cols columns and the subspace (the bond's
  // present dimension plus rsi_grow, at most chi_max, plus rsi_margin; at most
  // rsi_pmax) is at most 3/4 of them; rsi_pmax = 0 switches it off.
  int rsi_pmax, rsi_margin, rsi_grow, rsi_iters, rsi_min_cols;
  double rsi_tol;    // accepted Ritz residual, relative to the largest singular value
  double2 *Vr;       // max(R) x pmax: basis of the right subspace
  double2 *Zr;       // max(R) x pmax: its image, then the orthonormal left factor Q
  double2 *Wk;       // max(R) x pmax: scratch (the three rotate)
  double2 *Gr;       // kGramSplit partial pmax x pmax Gram matrices
  double2 *L1, *L2;  // pmax x pmax Cholesky factors
  double2 *Li;       // pmax x pmax inverse of a Cholesky factor
  double2 *Ldi;      // inverses of its 16 x 16 diagonal blocks (pmax / 16 of them)
  double2 *Rb;       // C x pmax: right singular vectors (kept columns)
  double2 *Res;      // C x pmax: residual scratch
  double *rsi_scal;  // [0] squared Frobenius norm of the block, [1] pending discarded fraction, [2] residual,
                     // [3] deviation of a repeat Gram matrix from the identity
  int *rsi_flag;     // [0] Cholesky breakdown, [1] result rejected
};
int svd_grid_size();
hipError_t launch_svd_persistent(hipStream_t s, const SvdLaunch &L, int grid);
// Batched form: one chain of a batch as seen by the per-layer kernel.
struct BatchChain {
  SvdLaunch L;           // the chain's buffers (mode, k, asc set per op); L.bar is its barrier block
  const double2 *gates;  // [nb][kGateSlots][256]
  int *centre;           // orthogonality centre, kept on the device between layers
  double2 *tr;           // trace scratch
  int *dims_out;         // copy of the bond dims after each layer (or null)
  int precision;
  int force_trace;       // renormalise after the step's last layer
  int step_parity;       // parity of the chain's step count at local step 0
};
int batch_grid_size();
// One cooperative launch running layer j of local step `local_step` of every
// chain: workgroup b serves chain block_group[b] as its member block_rank[b]
// of group_size[chain].  bar_base[0 .. bar_words) (all barrier blocks) is
// zeroed first.
hipError_t launch_batch_layer(hipStream_t s, const BatchChain *d_chains, const int *d_block_group,
                              const int *d_block_rank, const int *d_group_size, int total_blocks, unsigned *bar_base,
                              size_t bar_words, int local_step, int j, int parity, int slot, int last_layer);
constexpr size_t kBarBlock = 8 * 32 + 64;   // one grid barrier: 8 group counters, top, flag
constexpr size_t kBarWords = 2 * kBarBlock;  // a problem's grid barrier and its Jacobi block versions

void launch_trace(hipStream_t s, double2 *const *sites, const int *dims, int N, double2 *out);
void launch_env_all(hipStream_t s, double2 *const *sites, const int *dims, int N, int cap,
                    double2 *envL, double2 *envR);
void launch_measure(hipStream_t s, double2 *const *sites, const int *dims, int N, int cap,
                    const double2 *envL, const double2 *envR, int n, const int *req, double2 *out);
void launch_norm2_site(hipStream_t s, double2 *const *sites, const int *dims, int N, int site, double *out);
void launch_scale_site(hipStream_t s, double2 *const *sites, const int *dims, int N, int site,
                       const double2 *tr);
void launch_hermitian_sum_site(hipStream_t s, const double2 *src, double2 *dst, const int *dims, int N, int k);
void launch_double_dims(hipStream_t s, int *dims, int n);

// FP64 matrix-core probe: blocks x 256 threads, each wavefront 8 x iters MFMAs
// of 2048 flops; out holds blocks * 256 doubles.
void launch_mfma_f64_probe(hipStream_t s, int blocks, int iters, double *out);

// ---- adjoint gradient (grad.hip) ----
// C(m, n) = sum_k A(m, k) B(k, n) per batch z; element (m, k) of A at
// A[m * sam + k * sak + z * sab], likewise for B and C.
struct ZgemmArgs {
  int M, N, K;
  const double2 *A;
  long long sam, sak, sab;
  const double2 *B;
  long long sbk, sbn, sbb;
  double2 *C;
  long long scm, scn, scb;
};
void launch_zgemm(hipStream_t s, const ZgemmArgs &g, int batch);
void launch_transition_reduce(hipStream_t s, const double2 *E, const double2 *Fr, int pm, int qm, double2 *gam);
void launch_grad_accumulate(hipStream_t s, const double2 *K, const int *pidx, int nk, const double2 *gam,
                            double2 scale, double2 *grad);
// Site k of A + B (A: a copy of the site before the sum, bond dims `dims`;
// B: bond kb) into dst; then add_dims raises every bond by kb.
void launch_mps_sum_site(hipStream_t s, const double2 *A, const double2 *B, double2 *dst, const int *dims, int N,
                         int k, int kb);
void launch_add_dims(hipStream_t s, int *dims, int n, int add);
void launch_osee_costate(hipStream_t s, double2 *const *sites, const int *dims, int N, int k, double *out);

}  // namespace lmpo
