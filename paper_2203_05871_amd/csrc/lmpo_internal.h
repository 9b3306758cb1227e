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

// Block one-sided Jacobi: columns are processed in blocks of JB, two blocks
// (JP columns) per workgroup and round.
constexpr int JB = 8;
constexpr int JP = 2 * JB;
constexpr int kMaxDim = 2048;  // largest block side (4 chi) the sort handles

// ---- kernel launchers (kernels.hip) ----
void launch_contract_gate(hipStream_t s, int precision, const double2 *Ak, const double2 *Ak1,
                          const double2 *G, int chl, int chm, int chr, double2 *X, int trans);
void launch_jacobi_round(hipStream_t s, double2 *X, int ldx, int R, double2 *V, int ldv, int C,
                         int round, int nbp, double tol, double2 *W, int *active, int *counter);
void launch_identity(hipStream_t s, double2 *V, int ldv, int C);
void launch_colnorm(hipStream_t s, const double2 *X, int ldx, int R, int C, double *sig);
void launch_select(hipStream_t s, const double *sig, int C, int chi_max, double cutoff, int hop,
                   int *perm, double *sorted, int *kept, int *dims_slot, double *disc, int *err);
void launch_canon(hipStream_t s, const double2 *X, int ldx, const double2 *V, int ldv,
                  const int *perm, const double *sorted, const int *kept, double2 *Ak,
                  double2 *Ak1, int chl, int chr, int trans, int asc, int kmax);
void launch_hop_load(hipStream_t s, const double2 *A, int rows, int cols, double2 *X, int ct);
void launch_hop_write(hipStream_t s, const double2 *X, int ldx, const double2 *V, int ldv,
                      const int *perm, const double *sorted, int k, double2 *Ac, double2 *Z,
                      int R, int C, int right);
void launch_zgemm(hipStream_t s, int M, int N, int K, const double2 *A, int lda, const double2 *B,
                  int ldb, double2 *Cm, int ldc);
void launch_trace(hipStream_t s, double2 *const *sites, const int *dims, int N, double2 *out);
void launch_env_all(hipStream_t s, double2 *const *sites, const int *dims, int N, int cap,
                    double2 *envL, double2 *envR);
void launch_measure(hipStream_t s, double2 *const *sites, const int *dims, int N, int cap,
                    const double2 *envL, const double2 *envR, int n, const int *req, double2 *out);
void launch_scale_site(hipStream_t s, double2 *const *sites, const int *dims, int N, int site,
                       const double2 *tr);

}  // namespace lmpo
