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

// ---- kernel launchers (kernels.hip, svd.hip) ----
// One two-site contraction (for the batched launch).
struct ContractJob {
  double2 *const *sites;
  const int *dims;
  int N, k;
  const double2 *G;
  double2 *X;
};
void launch_contract_batched(hipStream_t s, int precision, const ContractJob *d_jobs, int n_jobs, int cap_l,
                             int cap_r);
void launch_contract_gate(hipStream_t s, int precision, double2 *const *sites, const int *dims, int N, int k,
                          int cap_l, int cap_r, const double2 *G, double2 *X);

// One persistent cooperative launch: mode 0 = truncated SVD + canonical update
// of the two-site block on bond k (X filled by the contraction); mode 1/2 =
// exact centre hop right/left from site k.
struct SvdLaunch {
  int mode, k, N, asc, chi_max, max_sweeps;
  double cutoff, tol_factor;
  double2 *const *sites;
  int *dims;
  double2 *X, *V, *W, *Z, *T;
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
};
int svd_grid_size();
hipError_t launch_svd_persistent(hipStream_t s, const SvdLaunch &L, int grid);
// One cooperative launch over many independent SvdLaunch problems (device
// array d_args); workgroup b serves problem d_block_group[b].  The callers
// zero every participating problem's barrier block beforehand.
hipError_t launch_svd_batched(hipStream_t s, const SvdLaunch *d_args, const int *d_block_group,
                              const int *d_group_first, int total_blocks);

void launch_trace(hipStream_t s, double2 *const *sites, const int *dims, int N, double2 *out);
void launch_env_all(hipStream_t s, double2 *const *sites, const int *dims, int N, int cap,
                    double2 *envL, double2 *envR);
void launch_measure(hipStream_t s, double2 *const *sites, const int *dims, int N, int cap,
                    const double2 *envL, const double2 *envR, int n, const int *req, double2 *out);
void launch_scale_site(hipStream_t s, double2 *const *sites, const int *dims, int N, int site,
                       const double2 *tr);

}  // namespace lmpo
