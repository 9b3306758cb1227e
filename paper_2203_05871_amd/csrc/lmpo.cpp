// C ABI and step executor of the MPO-TEBD Lindblad step (include/lmpo.h).
//
// The executor walks the second-order Trotter schedule (layers A(tau/2),
// B(tau), A(tau/2); A = even bonds, B = odd bonds; global layer l runs its
// gates in ascending bond order when l is even, descending when odd) and, per
// gate, launches: centre hops (exact SVD-based QR/LQ), the fused contraction +
// gate kernel, the block-Jacobi SVD, truncation select and canonical update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "lmpo_internal.h"

using namespace lmpo;

namespace {
thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(LMPO_EHIP, std::string(#expr " failed: ") + hipGetErrorString(e_));   \
  } while (0)

struct Arena {
  char *base;
  size_t size, used = 0;
  template <typename T>
  T *take(size_t n) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + n * sizeof(T);
    return reinterpret_cast<T *>(base + off);
  }
};

constexpr int kMaxReq = 4096;
constexpr int kMaxSweeps = 80;
// [last sweeps, last C, last R, subspace SVDs accepted, total sweeps, total SVDs,
//  subspace SVDs handed to the full SVD, subspace iterations]
constexpr int kStats = 8;
constexpr int kRsiMarginMax = 128;  // largest margin the subspace buffers allow
constexpr double kFp32TolFactor = 1e6;  // Jacobi threshold of the FP32-contraction form, units of sqrt(C) eps
constexpr size_t kGramSplitHost = 8;  // partial Gram matrices (rsi::kGramSplit)
constexpr int kRsiMaxWidth = 384;   // largest subspace (the triangular solve keeps 16 x p in LDS)

// Gate table slots: exp(x L_b) with x = fraction * tau.  Slots 0, 1 serve the
// second-order step A(tau/2) B(tau) A(tau/2); slots 2..5 the fourth-order
// composition S2(w1 tau) S2(w0 tau) S2(w1 tau), w1 = 1 / (2 - 2^(1/3)),
// w0 = 1 - 2 w1, with adjacent A half-layers merged: seven layers
// A(w1/2) B(w1) A((w1+w0)/2) B(w0) A((w0+w1)/2) B(w1) A(w1/2).
// Slots 7..11 (with slot 0) serve the third-order product (R. D. Ruth,
// IEEE Trans. Nucl. Sci. 30 (1983) 2669) of the two layer operators,
// A(7/24) B(2/3) A(3/4) B(-2/3) A(-1/24) B(1), whose negative fractions run
// the dissipators backwards for that sub-step.
// On other bond lists a second-order step is the symmetric sweep
// F(tau/2) R(tau/2) over the bonds (slot 1); fourth order composes such
// sweeps with w1/2 (slot 2) and w0/2 (slot 6).
double gate_fraction(int slot) {
  const double w1 = 1.0 / (2.0 - std::cbrt(2.0)), w0 = 1.0 - 2.0 * w1;
  switch (slot) {
    case 0: return 1.0;
    case 1: return 0.5;
    case 2: return 0.5 * w1;
    case 3: return w1;
    case 4: return 0.5 * (w1 + w0);
    case 5: return w0;
    case 6: return 0.5 * w0;
    case 7: return 7.0 / 24.0;
    case 8: return 2.0 / 3.0;
    case 9: return 0.75;
    case 10: return -2.0 / 3.0;
    default: return -1.0 / 24.0;
  }
}

// Slots of the symmetric sweeps of one step on a general bond list.
const std::vector<int> &sweep_slots(int order) {
  static const std::vector<int> o2 = {1};
  static const std::vector<int> o4 = {2, 6, 2};
  return order == 4 ? o4 : o2;
}

struct TrotterLayer {
  int parity;  // bonds b = parity, parity + 2, ...
  int slot;    // gate table slot
};

const std::vector<TrotterLayer> &trotter_layers(int order) {
  static const std::vector<TrotterLayer> o2 = {{0, 1}, {1, 0}, {0, 1}};
  static const std::vector<TrotterLayer> o3 = {{0, 7}, {1, 8}, {0, 9}, {1, 10}, {0, 11}, {1, 0}};
  static const std::vector<TrotterLayer> o4 = {{0, 2}, {1, 3}, {0, 4}, {1, 5}, {0, 4}, {1, 3}, {0, 2}};
  return order == 4 ? o4 : order == 3 ? o3 : o2;
}
}  // namespace

// Bond-dimension mirror for the batched form's planner.  After each step the
// device bond dims are copied into one of kRing pinned slots; before enqueuing
// step s the host waits for the copy of step s - kLag, so the plan (how many
// workgroups each chain gets) is made with dims at most kLag steps old while
// the GPU still has kLag steps of work queued.  Plans only affect speed, never
// results.
struct DimsRing {
  static constexpr int kRing = 3, kLag = 2;
  int n = 0;
  int *pinned = nullptr;  // [kRing][n]
  hipEvent_t ev[kRing] = {nullptr, nullptr, nullptr};
  long long issued[kRing] = {-1, -1, -1};  // step whose dims each slot holds
  hipError_t init(int count) {
    n = count > 0 ? count : 1;
    hipError_t e = hipHostMalloc((void **)&pinned, (size_t)kRing * n * sizeof(int), hipHostMallocDefault);
    for (int i = 0; i < kRing && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    return e;
  }
  ~DimsRing() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (pinned) (void)hipHostFree(pinned);
  }
  // before step s: wait for the copy taken after step s - kLag and load it
  hipError_t before(long long s, int *est) {
    const long long want = s - kLag;
    if (want < 0) return hipSuccess;
    const int slot = (int)(want % kRing);
    if (issued[slot] != want) return hipSuccess;
    hipError_t e = hipEventSynchronize(ev[slot]);
    if (e == hipSuccess) std::copy(pinned + (size_t)slot * n, pinned + (size_t)(slot + 1) * n, est);
    return e;
  }
  // after step s: copy the device dims into slot s mod kRing
  hipError_t after(long long s, const int *d_dims, hipStream_t st) {
    const int slot = (int)(s % kRing);
    hipError_t e = hipMemcpyAsync(pinned + (size_t)slot * n, d_dims, n * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(ev[slot], st);
    if (e == hipSuccess) issued[slot] = s;
    return e;
  }
};

// Gates of one step recorded for the adjoint pass: after every two-site gate
// the site tensors and bond dims are copied into the next snapshot slot.
struct OpRecord {
  int k;     // left site of the pair the gate acted on
  int bond;  // model bond of the gate, or -1 for a SWAP
  int slot;  // gate table slot (time fraction)
  int asc;   // direction the centre moved
};
struct Recorder {
  std::vector<OpRecord> ops;
  char *slots = nullptr;  // device: capacity snapshots of `stride` bytes
  size_t stride = 0, capacity = 0;
};

struct lmpo_state {
  ModelHost m;
  lmpo_options opt{};
  hipStream_t stream = nullptr;
  int N = 0;
  std::vector<int> cap;                 // bond capacities
  std::vector<double2 *> site;          // device site tensors
  std::vector<size_t> site_elems;       // capacity in complex elements
  std::vector<int> dims;                // host mirror of bond dims
  int centre = 0;
  int cap_max = 1;
  // device
  double2 **d_sites = nullptr;
  int *d_dims = nullptr;
  double2 *d_gates = nullptr;
  double2 *X = nullptr, *V = nullptr, *W = nullptr, *Z = nullptr, *T = nullptr;
  double2 *Y = nullptr, *Lb = nullptr, *Tq = nullptr;
  int *qmap = nullptr, *qinv = nullptr;
  int *act = nullptr, *cmap = nullptr;
  double *cnorm = nullptr;
  int *sweep_cnt = nullptr, *stats = nullptr, *perm = nullptr, *kept = nullptr, *err = nullptr, *req = nullptr;
  unsigned *bar = nullptr;
  unsigned long long *tprof = nullptr;
  double *alg_flops = nullptr;
  // optional profiling window: HIP events around every persistent SVD launch
  bool profiling = false;
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  size_t ev_used = 0;
  bool ev_overflow = false;
  int grid = 1;                 // largest co-resident grid of the persistent SVD
  int wg_cap = 0;               // caller's cap on workgroups per SVD launch (0: none)
  double tol_factor = 32.0;     // Jacobi stopping threshold, in units of sqrt(C) eps
  // subspace-iteration truncated SVD of wide gate blocks (see SvdLaunch)
  int rsi_pmax = 0;             // allocated subspace width (0: not available)
  int rsi_min_cols = 512, rsi_margin = 48, rsi_grow = 32, rsi_iters = 4;
  double rsi_tol = 1e-12;
  double2 *Vr = nullptr, *Zr = nullptr, *Wk = nullptr, *Gr = nullptr, *L1 = nullptr, *L2 = nullptr, *Li = nullptr, *Ldi = nullptr;
  double2 *Rb = nullptr, *Res = nullptr;
  double *rsi_scal = nullptr;
  int *rsi_flag = nullptr;
  ~lmpo_state() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  double *sig = nullptr, *sorted = nullptr, *disc = nullptr, *aux = nullptr;
  double2 *tr = nullptr, *envL = nullptr, *envR = nullptr, *mout = nullptr;
  long long step_index = 0;  // global Trotter step count (fixes the layer order)
  int device = 0;            // the GPU current at creation
  std::vector<std::complex<double>> gates_host;  // [nb][kGateSlots][256]
  bool chain = true;            // bond list is the open chain (b, b+1) in order
  double2 *d_swap = nullptr;    // exchange of two sites (Pauli basis)
  double2 *d_user = nullptr;    // caller-supplied two-site superoperator
  double2 *d_ident = nullptr;   // identity (compression sweep of the Hermitian part)
  bool herm_room = false;       // bond capacities doubled for the Hermitian part
  Recorder *rec = nullptr;      // set while the adjoint pass replays a step
};

namespace {

struct Sizes {
  std::vector<int> cap;
  std::vector<size_t> site_elems;
  size_t x_elems = 0, v_elems = 0, t_elems = 0, z_elems = 0;
  int max_cols = 1, max_dim = 1, cap_max = 1;
  int rsi_pmax = 0;  // subspace width the buffers of the truncated SVD allow
};

bool is_chain(const lmpo_model *m) {
  if (m->n_bonds != m->n_qubits - 1) return false;
  for (int b = 0; b < m->n_bonds; ++b)
    if (m->bond_ij[2 * b] != b || m->bond_ij[2 * b + 1] != b + 1) return false;
  return true;
}

int validate(const lmpo_model *m, const lmpo_options *o) {
  if (!m || !o) return fail(LMPO_EINVAL, "null model or options");
  if (m->n_qubits < 2) return fail(LMPO_EINVAL, "n_qubits must be >= 2");
  if (m->n_bonds < 1 || !m->bond_ij) return fail(LMPO_EINVAL, "at least one bond is required");
  if (!m->J || !m->Jz || !m->hx || !m->hy || !m->hz || !m->g0 || !m->g1 || !m->g2)
    return fail(LMPO_EINVAL, "null parameter array");
  for (int b = 0; b < m->n_bonds; ++b) {
    int i = m->bond_ij[2 * b], j = m->bond_ij[2 * b + 1];
    if (i < 0 || j <= i || j >= m->n_qubits) return fail(LMPO_EINVAL, "bond indices must satisfy 0 <= i < j < N");
    if (!std::isfinite(m->J[b]) || !std::isfinite(m->Jz[b])) return fail(LMPO_EINVAL, "non-finite coupling");
  }
  for (int s = 0; s < m->n_qubits; ++s) {
    double v[6] = {m->hx[s], m->hy[s], m->hz[s], m->g0[s], m->g1[s], m->g2[s]};
    for (double x : v)
      if (!std::isfinite(x)) return fail(LMPO_EINVAL, "non-finite on-site parameter");
    if (m->g0[s] < 0 || m->g1[s] < 0 || m->g2[s] < 0) return fail(LMPO_EINVAL, "dissipation rates must be >= 0");
  }
  if (!(o->tau > 0) || !std::isfinite(o->tau)) return fail(LMPO_EINVAL, "tau must be > 0");
  if (o->chi_max < 1) return fail(LMPO_EINVAL, "chi_max must be >= 1");
  if (!(o->cutoff >= 0) || !std::isfinite(o->cutoff)) return fail(LMPO_EINVAL, "cutoff must be >= 0");
  if (o->precision != LMPO_FP64 && o->precision != LMPO_FP32_CONTRACT && o->precision != LMPO_FP64_REAL)
    return fail(LMPO_EINVAL, "precision must be LMPO_FP64, LMPO_FP32_CONTRACT or LMPO_FP64_REAL");
  if (o->trotter_order < 2 || o->trotter_order > 4) return fail(LMPO_EUNSUPPORTED, "trotter_order must be 2, 3 or 4");
  if (o->chi_max > kMaxDim / 4) return fail(LMPO_EUNSUPPORTED, "chi_max above 512 is not supported");
  std::vector<int> deg(m->n_qubits, 0);
  for (int b = 0; b < m->n_bonds; ++b) {
    deg[m->bond_ij[2 * b]]++;
    deg[m->bond_ij[2 * b + 1]]++;
  }
  for (int s = 0; s < m->n_qubits; ++s)
    if (deg[s] == 0) return fail(LMPO_EINVAL, "every qubit must belong to a bond (its on-site terms ride on them)");
  if (o->force_hermitian_every < 0) return fail(LMPO_EINVAL, "force_hermitian_every must be >= 0");
  if (o->force_hermitian_every > 0 && o->chi_max > kMaxDim / 8)
    return fail(LMPO_EUNSUPPORTED, "force_hermitian_every needs chi_max <= 256 (the doubled bonds reach 512)");
  if (o->trotter_order == 3 && !is_chain(m))
    return fail(LMPO_EUNSUPPORTED, "trotter_order 3 needs the open chain (two commuting layer operators)");
  return LMPO_OK;
}

// Bond capacities min(chi_max, 4^(b+1), 4^(N-1-b)), times `mult` (2 when the
// Hermitian part is taken: the direct sum of rho and rho^+ doubles every bond
// until it is compressed again).
Sizes compute_sizes(int N, int chi_max, int mult) {
  Sizes z;
  z.cap.resize(N - 1);
  for (int b = 0; b < N - 1; ++b) {
    long long c = chi_max, p = 1;
    for (int q = 0; q < b + 1 && p < c; ++q) p *= 4;
    c = std::min(c, p);
    p = 1;
    for (int q = 0; q < N - 1 - b && p < c; ++q) p *= 4;
    c = std::min(c, p) * mult;
    z.cap[b] = (int)c;
    z.cap_max = std::max(z.cap_max, (int)c);
  }
  auto capL = [&](int k) { return k == 0 ? 1 : z.cap[k - 1]; };
  auto capR = [&](int k) { return k == N - 1 ? 1 : z.cap[k]; };
  z.site_elems.resize(N);
  for (int k = 0; k < N; ++k) {
    z.site_elems[k] = (size_t)capL(k) * 4 * capR(k);
    z.t_elems = std::max(z.t_elems, z.site_elems[k]);
  }
  auto consider = [&](size_t R, size_t C) {  // Jacobi on R x C, R >= C
    z.x_elems = std::max(z.x_elems, R * C);
    z.v_elems = std::max(z.v_elems, C * C);
    z.max_cols = std::max(z.max_cols, (int)C);
    z.max_dim = std::max(z.max_dim, (int)std::max(R, C));
  };
  for (int b = 0; b < N - 1; ++b) {
    size_t R = 4 * (size_t)capL(b), C = 4 * (size_t)capR(b + 1);
    consider(std::max(R, C), std::min(R, C));
    // hops across bond b
    consider(4 * (size_t)capL(b), z.cap[b]);
    consider(4 * (size_t)capR(b + 1), z.cap[b]);
    z.z_elems = std::max(z.z_elems, (size_t)z.cap[b] * z.cap[b]);
  }
  // the subspace of a gate's truncated SVD holds at most chi_max + kRsiMarginMax
  // vectors (and is only used when that is at most 3/4 of the block's columns)
  {
    int pm = (chi_max * mult + kRsiMarginMax + 15) & ~15;
    pm = std::min(pm, kRsiMaxWidth);
    if (4 * pm > 3 * z.max_cols) pm = (3 * z.max_cols / 4) & ~15;
    z.rsi_pmax = pm >= 32 ? pm : 0;
  }
  return z;
}

size_t layout(lmpo_state *S, const Sizes &z, int N, int nb, char *base, size_t size) {
  Arena a{base, size};
  S->site.resize(N);
  for (int k = 0; k < N; ++k) S->site[k] = a.take<double2>(z.site_elems[k]);
  S->d_sites = a.take<double2 *>(N);
  S->d_dims = a.take<int>(std::max(N - 1, 1));
  S->d_gates = a.take<double2>((size_t)nb * kGateSlots * 256);
  S->d_swap = a.take<double2>(256);
  S->d_user = a.take<double2>(256);
  S->d_ident = a.take<double2>(256);
  S->X = a.take<double2>(z.x_elems);
  S->V = a.take<double2>(z.v_elems);
  int nbp = (z.max_cols + JB - 1) / JB;
  nbp += nbp & 1;
  if (nbp < 2) nbp = 2;
  // rotations of two consecutive sweeps: [2][rounds][pairs][JP][JP]
  const size_t slots = (size_t)(nbp - 1) * (nbp / 2);
  S->W = a.take<double2>(2 * slots * JP * JP);
  S->act = a.take<int>(2 * slots);
  S->cmap = a.take<int>((size_t)2 * nbp * JB);  // two sweeps' column orders
  S->cnorm = a.take<double>(z.max_cols);
  S->Y = a.take<double2>(z.v_elems);
  S->Lb = a.take<double2>(z.x_elems);
  S->Tq = a.take<double2>((size_t)(z.max_cols / 4 + 2) * 256);  // one 16 x 16 T per QR panel
  S->qmap = a.take<int>(z.max_cols);
  S->qinv = a.take<int>(z.max_cols);
  S->Z = a.take<double2>(z.z_elems);
  S->T = a.take<double2>(z.t_elems);
  S->rsi_pmax = z.rsi_pmax;
  if (z.rsi_pmax > 0) {
    const size_t pm = (size_t)z.rsi_pmax;
    S->Vr = a.take<double2>((size_t)z.max_dim * pm);
    S->Zr = a.take<double2>((size_t)z.max_dim * pm);
    S->Wk = a.take<double2>((size_t)z.max_dim * pm);
    S->Gr = a.take<double2>(kGramSplitHost * pm * pm);
    S->L1 = a.take<double2>(pm * pm);
    S->L2 = a.take<double2>(pm * pm);
    S->Li = a.take<double2>(pm * pm);
    S->Ldi = a.take<double2>((pm / 16 + 1) * 256);
    S->Rb = a.take<double2>((size_t)z.max_cols * pm);
    S->Res = a.take<double2>((size_t)z.max_cols * pm);
    S->rsi_scal = a.take<double>(4);
    S->rsi_flag = a.take<int>(4);
  }
  S->sig = a.take<double>(z.max_cols);
  S->sorted = a.take<double>(z.max_cols);
  S->perm = a.take<int>(z.max_cols);
  S->sweep_cnt = a.take<int>(kMaxSweeps);
  S->stats = a.take<int>(kStats);
  S->bar = a.take<unsigned>(kBarWords);
  S->tprof = a.take<unsigned long long>(32);
  S->alg_flops = a.take<double>(1);
  S->kept = a.take<int>(1);
  S->err = a.take<int>(1);
  S->disc = a.take<double>(1);
  S->aux = a.take<double>(4);
  S->tr = a.take<double2>(1);
  S->envL = a.take<double2>((size_t)(N + 1) * z.cap_max);
  S->envR = a.take<double2>((size_t)(N + 1) * z.cap_max);
  S->req = a.take<int>(4 * kMaxReq);
  S->mout = a.take<double2>(kMaxReq);
  return a.used;
}

ModelHost copy_model(const lmpo_model *m) {
  ModelHost h;
  h.N = m->n_qubits;
  h.nb = m->n_bonds;
  h.bonds.assign(m->bond_ij, m->bond_ij + 2 * m->n_bonds);
  h.J.assign(m->J, m->J + h.nb);
  h.Jz.assign(m->Jz, m->Jz + h.nb);
  h.hx.assign(m->hx, m->hx + h.N);
  h.hy.assign(m->hy, m->hy + h.N);
  h.hz.assign(m->hz, m->hz + h.N);
  h.g0.assign(m->g0, m->g0 + h.N);
  h.g1.assign(m->g1, m->g1 + h.N);
  h.g2.assign(m->g2, m->g2 + h.N);
  h.degree.assign(h.N, 0);
  for (int b = 0; b < h.nb; ++b) {
    h.degree[h.bonds[2 * b]]++;
    h.degree[h.bonds[2 * b + 1]]++;
  }
  return h;
}

int parse_init(const char *init, int N, std::vector<std::pair<int, int>> &out) {
  if (!init) return fail(LMPO_EINVAL, "init_pauli is null");
  size_t len = std::strlen(init);
  if (len != 2 && len != (size_t)2 * N) return fail(LMPO_EINVAL, "init_pauli must hold 1 or N two-character labels");
  out.resize(N);
  for (int i = 0; i < N; ++i) {
    const char *p = (len == 2) ? init : init + 2 * i;
    int sign = p[0] == '+' ? 1 : (p[0] == '-' ? -1 : 0);
    int axis = (p[1] == 'x' || p[1] == 'X') ? 1 : (p[1] == 'y' || p[1] == 'Y') ? 2 : (p[1] == 'z' || p[1] == 'Z') ? 3 : 0;
    if (!sign || !axis) return fail(LMPO_EINVAL, std::string("bad Pauli state label in init_pauli: ") + init);
    out[i] = {sign, axis};
  }
  return LMPO_OK;
}

int dimL(const lmpo_state *S, int k) { return k == 0 ? 1 : S->dims[k - 1]; }
int dimR(const lmpo_state *S, int k) { return k == S->N - 1 ? 1 : S->dims[k]; }
int capL(const lmpo_state *S, int k) { return k == 0 ? 1 : S->cap[k - 1]; }
int capR(const lmpo_state *S, int k) { return k == S->N - 1 ? 1 : S->cap[k]; }

int read_int(lmpo_state *S, const int *d, int *h) {
  HIP_TRY(hipMemcpyAsync(h, d, sizeof(int), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  return LMPO_OK;
}

int sync_dims(lmpo_state *S) {
  HIP_TRY(hipMemcpyAsync(S->dims.data(), S->d_dims, (S->N - 1) * sizeof(int), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  return LMPO_OK;
}

SvdLaunch svd_args(lmpo_state *S, int mode, int k, int asc) {
  SvdLaunch L;
  L.mode = mode;
  L.k = k;
  L.N = S->N;
  L.asc = asc;
  L.chi_max = S->opt.chi_max;
  L.max_sweeps = kMaxSweeps;
  L.real = S->opt.precision == LMPO_FP64_REAL ? 1 : 0;
  L.cutoff = S->opt.cutoff;
  L.tol_factor = S->tol_factor;
  L.sites = S->d_sites;
  L.dims = S->d_dims;
  L.X = S->X;
  L.V = S->V;
  L.Y = S->Y;
  L.Lb = S->Lb;
  L.Tq = S->Tq;
  L.qmap = S->qmap;
  L.qinv = S->qinv;
  L.aux = S->aux;
  L.W = S->W;
  L.act = S->act;
  L.cmap = S->cmap;
  L.cnorm = S->cnorm;
  L.Z = S->Z;
  L.T = S->T;
  L.sweep_cnt = S->sweep_cnt;
  L.sig = S->sig;
  L.sorted = S->sorted;
  L.perm = S->perm;
  L.kept = S->kept;
  L.err = S->err;
  L.stats = S->stats;
  L.disc = S->disc;
  L.bar = S->bar;
  L.tprof = S->tprof;
  L.alg_flops = S->alg_flops;
  L.rsi_pmax = S->rsi_min_cols > 0 ? S->rsi_pmax : 0;
  L.rsi_margin = S->rsi_margin;
  L.rsi_grow = S->rsi_grow;
  L.rsi_iters = S->rsi_iters;
  L.rsi_min_cols = S->rsi_min_cols;
  L.rsi_tol = S->rsi_tol;
  L.Vr = S->Vr;
  L.Zr = S->Zr;
  L.Wk = S->Wk;
  L.Gr = S->Gr;
  L.L1 = S->L1;
  L.L2 = S->L2;
  L.Li = S->Li;
  L.Ldi = S->Ldi;
  L.Rb = S->Rb;
  L.Res = S->Res;
  L.rsi_scal = S->rsi_scal;
  L.rsi_flag = S->rsi_flag;
  return L;
}

// Workgroups launched for one persistent SVD whose problem has at most C
// columns (from the bond capacities, so nothing waits for the device's dims):
// svd_workgroups(C), capped by the caller's limit and the co-resident grid.
// The kernel trims the grid to what the actual dims need (grid barriers get
// slower with every extra workgroup); the count only affects speed, never
// results.
int grid_for(const lmpo_state *S, int R, int C) {
  (void)R;
  const int cap = S->wg_cap > 0 ? std::min(S->wg_cap, S->grid) : S->grid;
  return std::max(1, std::min(svd_workgroups(C), cap));
}
int est(const lmpo_state *S, int bond) {
  if (bond < 0 || bond >= S->N - 1) return 1;
  return S->cap[bond];
}

int launch_svd(lmpo_state *S, const SvdLaunch &L, int grid) {
  hipEvent_t *pair = nullptr;
  if (S->profiling) {
    if (S->ev_used + 2 <= S->ev.size()) {
      pair = &S->ev[S->ev_used];
      S->ev_used += 2;
    } else {
      S->ev_overflow = true;
    }
  }
  if (pair) HIP_TRY(hipEventRecord(pair[0], S->stream));
  HIP_TRY(launch_svd_persistent(S->stream, L, grid));
  if (pair) HIP_TRY(hipEventRecord(pair[1], S->stream));
  return LMPO_OK;
}

// Exact move of the orthogonality centre by one site (SVD-based QR / LQ).
int hop(lmpo_state *S, int c, bool right) {
  int R, C;
  if (right) {
    R = 4 * (c == 0 ? 1 : est(S, c - 1));
    C = est(S, c);
  } else {
    R = 4 * (c == S->N - 1 ? 1 : est(S, c));
    C = est(S, c - 1);
  }
  return launch_svd(S, svd_args(S, right ? 1 : 2, c, 0), grid_for(S, R, C));
}

int move_centre(lmpo_state *S, int to) {
  int rc;
  while (S->centre < to) {
    if ((rc = hop(S, S->centre, true))) return rc;
    S->centre++;
  }
  while (S->centre > to) {
    if ((rc = hop(S, S->centre, false))) return rc;
    S->centre--;
  }
  return LMPO_OK;
}

// Snapshot of the state: the site tensors (one contiguous block of the arena,
// at capacity) followed by the bond dims.
size_t site_region_bytes(const lmpo_state *S) {
  return (size_t)(reinterpret_cast<const char *>(S->site[S->N - 1] + S->site_elems[S->N - 1]) -
                  reinterpret_cast<const char *>(S->site[0]));
}
size_t snapshot_dims_offset(const lmpo_state *S) { return (site_region_bytes(S) + 255) & ~size_t(255); }
size_t snapshot_bytes(const lmpo_state *S) {
  return snapshot_dims_offset(S) + ((((size_t)S->N - 1) * sizeof(int) + 255) & ~size_t(255));
}
int save_snapshot(lmpo_state *S, char *dst) {
  HIP_TRY(hipMemcpyAsync(dst, S->site[0], site_region_bytes(S), hipMemcpyDeviceToDevice, S->stream));
  HIP_TRY(hipMemcpyAsync(dst + snapshot_dims_offset(S), S->d_dims, (S->N - 1) * sizeof(int),
                         hipMemcpyDeviceToDevice, S->stream));
  return LMPO_OK;
}
int load_snapshot(lmpo_state *S, const char *src) {
  HIP_TRY(hipMemcpyAsync(S->site[0], src, site_region_bytes(S), hipMemcpyDeviceToDevice, S->stream));
  HIP_TRY(hipMemcpyAsync(S->d_dims, src + snapshot_dims_offset(S), (S->N - 1) * sizeof(int),
                         hipMemcpyDeviceToDevice, S->stream));
  return LMPO_OK;
}

int record_gate(lmpo_state *S, int k, const double2 *G, int asc) {
  Recorder &R = *S->rec;
  OpRecord op{k, -1, 0, asc};
  const size_t table = (size_t)S->m.nb * kGateSlots * 256;
  if (G >= S->d_gates && G < S->d_gates + table) {
    const size_t idx = (size_t)(G - S->d_gates) / 256;
    op.bond = (int)(idx / kGateSlots);
    op.slot = (int)(idx % kGateSlots);
  } else if (G != S->d_swap) {
    return fail(LMPO_EUNSUPPORTED, "only model gates and SWAP gates can be recorded");
  }
  if (R.ops.size() >= R.capacity) return fail(LMPO_EINVAL, "a step holds more gates than the gradient workspace");
  int rc = save_snapshot(S, R.slots + R.ops.size() * R.stride);
  if (rc) return rc;
  R.ops.push_back(op);
  return LMPO_OK;
}

// Two-site gate G (device, 16x16 Pauli basis) on sites (k, k+1).
int apply_gate_dev(lmpo_state *S, int k, const double2 *G, int asc) {
  int rc = move_centre(S, S->centre <= k ? k : k + 1);
  if (rc) return rc;
  launch_contract_gate(S->stream, S->opt.precision, S->d_sites, S->d_dims, S->N, k, capL(S, k), capR(S, k + 1), G,
                       S->X);
  HIP_TRY(hipGetLastError());
  const int r = 4 * (k == 0 ? 1 : est(S, k - 1)), c = 4 * (k + 1 == S->N - 1 ? 1 : est(S, k + 1));
  rc = launch_svd(S, svd_args(S, 0, k, asc), grid_for(S, std::max(r, c), std::min(r, c)));
  if (rc) return rc;
  S->centre = asc ? k + 1 : k;
  return S->rec ? record_gate(S, k, G, asc) : LMPO_OK;
}

const double2 *gate_ptr(const lmpo_state *S, int bond, int slot) {
  return S->d_gates + ((size_t)bond * kGateSlots + slot) * 256;
}

int apply_gate(lmpo_state *S, int k, int slot, int asc) { return apply_gate_dev(S, k, gate_ptr(S, k, slot), asc); }

// G on qubits i < j.  Neighbours on the path: one gate (the centre ends right
// of the pair on forward sweeps, left of it otherwise).  Apart: SWAP gates
// carry site j down to i + 1 (centre moving left), G acts on (i, i + 1), SWAP
// gates carry it back (centre moving right).  Every SWAP is an ordinary
// truncated two-site gate.
int apply_pair(lmpo_state *S, int i, int j, const double2 *G, bool forward) {
  int rc;
  if (j == i + 1) return apply_gate_dev(S, i, G, forward ? 1 : 0);
  for (int k = j - 1; k > i; --k)
    if ((rc = apply_gate_dev(S, k, S->d_swap, 0))) return rc;
  if ((rc = apply_gate_dev(S, i, G, 1))) return rc;
  for (int k = i + 1; k < j; ++k)
    if ((rc = apply_gate_dev(S, k, S->d_swap, 1))) return rc;
  return LMPO_OK;
}

// Product of Pauli eigenstates: per site (1, 0, 0, 0) / sqrt(2) with
// +-1/sqrt(2) on the axis; bond dims 1, centre 0.  Synchronises.
int upload_product(lmpo_state *S, const std::vector<std::pair<int, int>> &init) {
  const double r2 = 1.0 / std::sqrt(2.0);
  std::vector<double2> sitev(4 * S->N);
  for (int i = 0; i < S->N; ++i) {
    for (int a = 0; a < 4; ++a) sitev[4 * i + a] = make_double2(0, 0);
    sitev[4 * i] = make_double2(r2, 0);
    sitev[4 * i + init[i].second] = make_double2(init[i].first * r2, 0);
  }
  for (int i = 0; i < S->N; ++i)
    HIP_TRY(hipMemcpyAsync(S->site[i], &sitev[4 * i], 4 * sizeof(double2), hipMemcpyHostToDevice, S->stream));
  std::fill(S->dims.begin(), S->dims.end(), 1);
  std::vector<int> ones(std::max(S->N - 1, 1), 1);
  HIP_TRY(hipMemcpyAsync(S->d_dims, ones.data(), ones.size() * sizeof(int), hipMemcpyHostToDevice, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  S->centre = 0;
  return LMPO_OK;
}

// Copies a caller's 16x16 Pauli-basis superoperator for qubits (i, j) into the
// device slot, re-indexed to act on (min, max) when i > j.  The stream is
// drained first, so no queued gate still reads the slot.  Synchronises.
int upload_user_gate(lmpo_state *S, int i, int j, const double *G) {
  std::vector<double2> g(256);
  auto flip = [](int x) { return (x % 4) * 4 + x / 4; };
  for (int r = 0; r < 16; ++r)
    for (int c = 0; c < 16; ++c) {
      const int rr = i > j ? flip(r) : r, cc = i > j ? flip(c) : c;
      g[rr * 16 + cc] = make_double2(G[2 * (r * 16 + c)], G[2 * (r * 16 + c) + 1]);
    }
  double big = 0.0, im = 0.0;
  for (const double2 &v : g) {
    if (!std::isfinite(v.x) || !std::isfinite(v.y)) return fail(LMPO_EINVAL, "non-finite gate entry");
    big = std::max(big, std::hypot(v.x, v.y));
    im = std::max(im, std::abs(v.y));
  }
  if (S->opt.precision == LMPO_FP64_REAL) {
    if (im > 1e-12 * big)
      return fail(LMPO_EINVAL, "the real-arithmetic form needs a superoperator that is real in the Pauli basis");
    for (double2 &v : g) v.y = 0.0;
  }
  HIP_TRY(hipStreamSynchronize(S->stream));
  HIP_TRY(hipMemcpyAsync(S->d_user, g.data(), 256 * sizeof(double2), hipMemcpyHostToDevice, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  return LMPO_OK;
}

int pair_args(const lmpo_state *S, int i, int j) {
  if (i < 0 || j < 0 || i >= S->N || j >= S->N || i == j)
    return fail(LMPO_EINVAL, "a two-site gate needs two distinct qubits in range");
  return LMPO_OK;
}

int renormalize(lmpo_state *S) {
  launch_trace(S->stream, S->d_sites, S->d_dims, S->N, S->tr);
  launch_scale_site(S->stream, S->d_sites, S->d_dims, S->N, S->centre, S->tr);
  return LMPO_OK;
}

// rho -> (rho + rho^+) / 2 (force_rho_hermitian_step, Sec. 6): the direct
// sum of the MPS and its conjugate (bonds doubled, first site halved), an
// exact QR sweep from the left (bonds fall to their exact rank bound), then a
// right-to-left sweep of identity gates, i.e. the truncated two-site SVD of
// every bond with the state's chi_max and cutoff.  The centre ends on site 0.
int hermitize(lmpo_state *S) {
  if (S->opt.precision == LMPO_FP64_REAL) return LMPO_OK;  // real coefficients: rho^+ = rho exactly
  const int N = S->N;
  for (int k = 0; k < N; ++k) {
    HIP_TRY(hipMemcpyAsync(S->T, S->site[k], S->site_elems[k] * sizeof(double2), hipMemcpyDeviceToDevice,
                           S->stream));
    launch_hermitian_sum_site(S->stream, S->T, S->site[k], S->d_dims, N, k);
    HIP_TRY(hipGetLastError());
  }
  launch_double_dims(S->stream, S->d_dims, N - 1);
  HIP_TRY(hipGetLastError());
  S->centre = 0;
  int rc = move_centre(S, N - 1);
  for (int k = N - 2; k >= 0 && !rc; --k) rc = apply_gate_dev(S, k, S->d_ident, 0);
  return rc;
}

// End of step `step`: the Hermitian part every force_hermitian_every steps,
// then the trace forced to one.
int finish_step(lmpo_state *S, long long step) {
  const int every = S->opt.force_hermitian_every;
  if (every > 0 && (step + 1) % every == 0) {
    int rc = hermitize(S);
    if (rc) return rc;
  }
  if (S->opt.force_trace) return renormalize(S);
  return LMPO_OK;
}

int check_err(lmpo_state *S) {
  int e = 0;
  int rc = read_int(S, S->err, &e);
  if (rc) return rc;
  if (e & 2) return fail(LMPO_EHIP, "a grid barrier wait exceeded its spin limit (workgroups not co-resident)");
  if (e) return fail(LMPO_ENUMERIC, "non-finite or zero singular values / trace encountered");
  return LMPO_OK;
}

int one_step(lmpo_state *S, long long step) {
  const int N = S->N;
  if (!S->chain) {  // symmetric sweeps F(x) R(x) over the bond list
    const int nb = S->m.nb;
    for (int slot : sweep_slots(S->opt.trotter_order)) {
      for (int b = 0; b < nb; ++b) {
        int rc = apply_pair(S, S->m.bonds[2 * b], S->m.bonds[2 * b + 1], gate_ptr(S, b, slot), true);
        if (rc) return rc;
      }
      for (int b = nb - 1; b >= 0; --b) {
        int rc = apply_pair(S, S->m.bonds[2 * b], S->m.bonds[2 * b + 1], gate_ptr(S, b, slot), false);
        if (rc) return rc;
      }
    }
    return finish_step(S, step);
  }
  const std::vector<TrotterLayer> &layers = trotter_layers(S->opt.trotter_order);
  for (int j = 0; j < (int)layers.size(); ++j) {
    const long long layer = (long long)layers.size() * step + j;
    const bool asc = (layer % 2) == 0;
    const int par = layers[j].parity, slot = layers[j].slot;
    std::vector<int> bonds;
    for (int b = par; b < N - 1; b += 2) bonds.push_back(b);
    if (!asc) std::reverse(bonds.begin(), bonds.end());
    for (int b : bonds) {
      int rc = apply_gate(S, b, slot, asc ? 1 : 0);
      if (rc) return rc;
    }
  }
  return finish_step(S, step);
}

// <<rho|rho>> = tr(rho^dagger rho) = sum |c|^2 in the orthonormal Pauli basis,
// the squared norm of the orthogonality centre (every other site is an
// isometry), and |tr rho|^2; tr rho itself into *tr when asked.  Synchronises.
int purity_and_trace(lmpo_state *S, double &n2, double &t2, double2 *tr_out) {
  launch_trace(S->stream, S->d_sites, S->d_dims, S->N, S->tr);
  launch_norm2_site(S->stream, S->d_sites, S->d_dims, S->N, S->centre, S->aux + 2);
  double2 tr;
  n2 = 0.0;
  HIP_TRY(hipMemcpyAsync(&tr, S->tr, sizeof(double2), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipMemcpyAsync(&n2, S->aux + 2, sizeof(double), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  int rc = check_err(S);
  if (rc) return rc;
  t2 = tr.x * tr.x + tr.y * tr.y;
  if (!(t2 > 0) || !(n2 > 0) || !std::isfinite(n2)) return fail(LMPO_ENUMERIC, "trace or purity is zero or non-finite");
  if (tr_out) *tr_out = tr;
  return LMPO_OK;
}

}  // namespace

extern "C" {

const char *lmpo_last_error(void) { return g_err.c_str(); }

size_t lmpo_arena_bytes(const lmpo_model *model, const lmpo_options *opt) {
  if (validate(model, opt) != LMPO_OK) return 0;
  Sizes z = compute_sizes(model->n_qubits, opt->chi_max, opt->force_hermitian_every > 0 ? 2 : 1);
  lmpo_state tmp;
  return layout(&tmp, z, model->n_qubits, model->n_bonds, nullptr, 0) + 256;
}

namespace {
int scratch_setup(int device);
}  // namespace

int lmpo_create(const lmpo_model *model, const lmpo_options *opt, const char *init_pauli, void *device_arena,
                size_t arena_bytes, void *hip_stream, lmpo_state **out) {
  if (!out) return fail(LMPO_EINVAL, "out is null");
  *out = nullptr;
  int rc = validate(model, opt);
  if (rc) return rc;
  std::vector<std::pair<int, int>> init;
  if ((rc = parse_init(init_pauli, model->n_qubits, init))) return rc;
  if (!device_arena) return fail(LMPO_EINVAL, "device_arena is null");
  if (reinterpret_cast<uintptr_t>(device_arena) % 256) return fail(LMPO_EINVAL, "device_arena must be 256-byte aligned");
  Sizes z = compute_sizes(model->n_qubits, opt->chi_max, opt->force_hermitian_every > 0 ? 2 : 1);
  if (z.max_dim > kMaxDim) return fail(LMPO_EUNSUPPORTED, "block dimension above 2048");
  lmpo_state *S = new lmpo_state();
  S->m = copy_model(model);
  S->opt = *opt;
  if (opt->precision == LMPO_FP32_CONTRACT) {
    // the contraction hands the SVD a block rounded to FP32 (relative error
    // about 6e-8): the FP64 SVD resolves it to just below that instead of to
    // FP64 round-off.  Jacobi stops at a relative off-diagonal size of about
    // 4e-9 (C = 304) to 7e-9 (C = 1024), the subspace SVD accepts Ritz
    // residuals up to 1e-8 of the largest singular value and starts with two
    // iterations.
    S->tol_factor = kFp32TolFactor;
    S->rsi_tol = 1e-8;
    S->rsi_iters = 2;
  }
  S->chain = is_chain(model);
  S->herm_room = opt->force_hermitian_every > 0;
  S->N = model->n_qubits;
  S->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&S->device) != hipSuccess || (rc = scratch_setup(S->device)) != LMPO_OK) {
    delete S;
    return rc ? rc : fail(LMPO_EHIP, "hipGetDevice failed");
  }
  size_t need = layout(S, z, S->N, S->m.nb, reinterpret_cast<char *>(device_arena), arena_bytes);
  if (need > arena_bytes) {
    delete S;
    return fail(LMPO_ENOMEM, "arena too small: need " + std::to_string(need) + " bytes");
  }
  S->cap = z.cap;
  S->site_elems = z.site_elems;
  S->cap_max = z.cap_max;
  S->dims.assign(S->N - 1, 1);
  S->centre = 0;
  // gate table: exp(x L_b) for every time fraction x / tau of the scheme, index [b][slot]
  const int nb = S->m.nb;
  S->gates_host.assign((size_t)nb * kGateSlots * 256, 0.0);
  std::vector<std::complex<double>> L(256), A(256);
  for (int b = 0; b < nb; ++b) {
    bond_generator_pauli(S->m, b, L.data());
    for (int slot = 0; slot < kGateSlots; ++slot) {
      const double x = gate_fraction(slot) * opt->tau;
      for (int e = 0; e < 256; ++e) A[e] = x * L[e];
      if (!expm_pade13(16, A.data(), &S->gates_host[((size_t)b * kGateSlots + slot) * 256])) {
        delete S;
        return fail(LMPO_ENUMERIC, "matrix exponential failed");
      }
    }
  }
  if (opt->precision == LMPO_FP64_REAL) {
    // a Lindblad propagator maps Hermitian operators to Hermitian ones, so in
    // the Hermitian basis B_ab it is real; drop the round-off imaginary parts
    double big = 0.0, im = 0.0;
    for (const auto &v : S->gates_host) {
      big = std::max(big, std::abs(v));
      im = std::max(im, std::abs(v.imag()));
    }
    if (im > 1e-12 * big) {
      delete S;
      return fail(LMPO_ENUMERIC, "gate table not real in the Pauli basis");
    }
    for (auto &v : S->gates_host) v = v.real();
  }
  auto cleanup = [&](int code) {
    delete S;
    return code;
  };
  hipError_t e;
  e = hipMemcpyAsync(S->d_gates, S->gates_host.data(), S->gates_host.size() * sizeof(double2), hipMemcpyHostToDevice,
                     S->stream);
  if (e != hipSuccess) return cleanup(fail(LMPO_EHIP, std::string("gate upload: ") + hipGetErrorString(e)));
  std::vector<std::complex<double>> swap(256), ident(256, 0.0);
  swap_pauli(swap.data());
  for (int q = 0; q < 16; ++q) ident[17 * q] = 1.0;
  e = hipMemcpyAsync(S->d_swap, swap.data(), 256 * sizeof(double2), hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(S->d_ident, ident.data(), 256 * sizeof(double2), hipMemcpyHostToDevice, S->stream);
  if (e != hipSuccess) return cleanup(fail(LMPO_EHIP, std::string("swap upload: ") + hipGetErrorString(e)));
  e = hipMemcpyAsync(S->d_sites, S->site.data(), S->N * sizeof(double2 *), hipMemcpyHostToDevice, S->stream);
  if (e != hipSuccess) return cleanup(fail(LMPO_EHIP, std::string("site table upload: ") + hipGetErrorString(e)));
  std::vector<int> ones(std::max(S->N - 1, 1), 1);
  e = hipMemcpyAsync(S->d_dims, ones.data(), ones.size() * sizeof(int), hipMemcpyHostToDevice, S->stream);
  if (e != hipSuccess) return cleanup(fail(LMPO_EHIP, std::string("dims upload: ") + hipGetErrorString(e)));
  if ((rc = upload_product(S, init))) return cleanup(rc);
  S->grid = svd_grid_size();
  int zero = 0;
  double zd = 0.0;
  e = hipMemsetAsync(S->stats, 0, kStats * sizeof(int), S->stream);
  if (e == hipSuccess) e = hipMemsetAsync(S->tprof, 0, 32 * sizeof(unsigned long long), S->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(S->err, &zero, sizeof(int), hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(S->disc, &zd, sizeof(double), hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return cleanup(fail(LMPO_EHIP, std::string("init: ") + hipGetErrorString(e)));
  *out = S;
  return LMPO_OK;
}

int lmpo_evolve_step(lmpo_state *S, int32_t n_steps) {
  if (!S) return fail(LMPO_EINVAL, "state is null");
  if (n_steps < 0) return fail(LMPO_EINVAL, "n_steps must be >= 0");
  for (int n = 0; n < n_steps; ++n) {
    int rc = one_step(S, S->step_index);
    if (rc) return rc;
    S->step_index++;
  }
  return LMPO_OK;
}

int lmpo_sync(lmpo_state *S) {
  if (!S) return fail(LMPO_EINVAL, "state is null");
  HIP_TRY(hipStreamSynchronize(S->stream));
  return check_err(S);
}

int lmpo_trace(lmpo_state *S, double out[2]) {
  if (!S || !out) return fail(LMPO_EINVAL, "null argument");
  launch_trace(S->stream, S->d_sites, S->d_dims, S->N, S->tr);
  double2 t;
  HIP_TRY(hipMemcpyAsync(&t, S->tr, sizeof(double2), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  out[0] = t.x;
  out[1] = t.y;
  int rc = check_err(S);
  if (rc) return rc;
  if (!std::isfinite(t.x) || !std::isfinite(t.y)) return fail(LMPO_ENUMERIC, "non-finite trace");
  return LMPO_OK;
}

int lmpo_renormalize(lmpo_state *S) {
  if (!S) return fail(LMPO_EINVAL, "state is null");
  return renormalize(S);
}

namespace {
int pauli_index(char c) {
  switch (c) {
    case 'X': case 'x': return 1;
    case 'Y': case 'y': return 2;
    case 'Z': case 'z': return 3;
    case 'I': case 'i': return 0;
  }
  return -1;
}

// req rows (i, a, j, b); j < 0 for 1Q.  out[n][2] = numerator / trace.
int run_measure(lmpo_state *S, const std::vector<int> &req, double *out) {
  const int n = (int)req.size() / 4;
  launch_env_all(S->stream, S->d_sites, S->d_dims, S->N, S->cap_max, S->envL, S->envR);
  launch_trace(S->stream, S->d_sites, S->d_dims, S->N, S->tr);
  double2 tr;
  HIP_TRY(hipMemcpyAsync(&tr, S->tr, sizeof(double2), hipMemcpyDeviceToHost, S->stream));
  std::vector<double2> buf(kMaxReq);
  for (int q0 = 0; q0 < n; q0 += kMaxReq) {
    const int m = std::min(kMaxReq, n - q0);
    HIP_TRY(hipMemcpyAsync(S->req, req.data() + 4 * (size_t)q0, 4 * (size_t)m * sizeof(int), hipMemcpyHostToDevice,
                           S->stream));
    launch_measure(S->stream, S->d_sites, S->d_dims, S->N, S->cap_max, S->envL, S->envR, m, S->req, S->mout);
    HIP_TRY(hipMemcpyAsync(buf.data(), S->mout, (size_t)m * sizeof(double2), hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    const double d = tr.x * tr.x + tr.y * tr.y;
    if (!(d > 0) || !std::isfinite(d)) return fail(LMPO_ENUMERIC, "trace is zero or non-finite");
    for (int q = 0; q < m; ++q) {
      double2 v = buf[q];
      out[2 * (q0 + q)] = (v.x * tr.x + v.y * tr.y) / d;
      out[2 * (q0 + q) + 1] = (v.y * tr.x - v.x * tr.y) / d;
    }
  }
  return check_err(S);
}
}  // namespace

// ---- allocation-free measurement (lmpo_measure_2q_noalloc) ----
// A fixed device array serves as the measurement's working memory instead of
// the state's arena: the trace, the left and right identity environments, the
// request rows and the numerators.  Each GPU that the library runs on holds
// its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in, not a device address: the address is resolved once per
// device with hipGetSymbolAddress (at state creation, with the state's device
// current) and only that address is handed to kernels and copies.
namespace {
constexpr size_t kScratchBytes = size_t(2) << 20;  // 2 MiB per device
constexpr size_t kScratchHead = 256;               // the trace (one double2), padded
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(LMPO_EUNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return LMPO_OK;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(LMPO_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = static_cast<char *>(p);
  return LMPO_OK;
}

// Bytes of scratch a state's measurement needs: the trace, both environments
// ((N + 1) x chi capacity each), kMaxReq request rows and numerators.
size_t scratch_need(const lmpo_state *S) {
  return kScratchHead + 2 * ((size_t)(S->N + 1) * S->cap_max * sizeof(double2)) + 4 * (size_t)kMaxReq * sizeof(int) +
         (size_t)kMaxReq * sizeof(double2);
}
}  // namespace

int lmpo_measure_2q_noalloc(lmpo_state *S, int32_t n, const int32_t *i, const int32_t *j, const char *paulis,
                            double *out) {
  if (!S || n < 0 || (n > 0 && (!i || !j || !paulis || !out))) return fail(LMPO_EINVAL, "null argument or n < 0");
  const size_t need = scratch_need(S);
  if (need > kScratchBytes)
    return fail(LMPO_EUNSUPPORTED, "lmpo_measure_2q_noalloc: the state needs " + std::to_string(need) +
                                       " bytes of measurement scratch, above the fixed " +
                                       std::to_string(kScratchBytes) + " (2 (N + 1) chi_cap 16 + 128 KiB)");
  for (int q = 0; q < n; ++q) {
    const int a = pauli_index(paulis[2 * q]), b = pauli_index(paulis[2 * q + 1]);
    if (i[q] < 0 || i[q] >= S->N || j[q] < 0 || j[q] >= S->N) return fail(LMPO_EINVAL, "site index out of range");
    if (i[q] == j[q]) return fail(LMPO_EINVAL, "2Q observable needs i != j");
    if (a <= 0 || b <= 0) return fail(LMPO_EINVAL, "paulis must be X, Y or Z");
  }
  if (n == 0) return LMPO_OK;
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != S->device) return fail(LMPO_EINVAL, "the state's device is not the current device");
  int rc = scratch_setup(dev);  // resolved at creation already; a no-op here
  if (rc) return rc;
  char *base = g_scratch_ptr[dev];
  double2 *tr_d = reinterpret_cast<double2 *>(base);
  double2 *envL = reinterpret_cast<double2 *>(base + kScratchHead);
  double2 *envR = envL + (size_t)(S->N + 1) * S->cap_max;
  int *req_d = reinterpret_cast<int *>(envR + (size_t)(S->N + 1) * S->cap_max);
  double2 *num_d = reinterpret_cast<double2 *>(req_d + 4 * (size_t)kMaxReq);
  // host staging of fixed size per thread (no allocation per call)
  static thread_local int req_h[4 * kMaxReq];
  static thread_local double2 num_h[kMaxReq];
  launch_env_all(S->stream, S->d_sites, S->d_dims, S->N, S->cap_max, envL, envR);
  launch_trace(S->stream, S->d_sites, S->d_dims, S->N, tr_d);
  double2 tr;
  HIP_TRY(hipMemcpyAsync(&tr, tr_d, sizeof(double2), hipMemcpyDeviceToHost, S->stream));
  for (int q0 = 0; q0 < n; q0 += kMaxReq) {
    const int m = std::min(kMaxReq, n - q0);
    for (int q = 0; q < m; ++q) {
      int ii = i[q0 + q], jj = j[q0 + q];
      int a = pauli_index(paulis[2 * (q0 + q)]), b = pauli_index(paulis[2 * (q0 + q) + 1]);
      if (ii > jj) {
        std::swap(ii, jj);
        std::swap(a, b);
      }
      req_h[4 * q] = ii;
      req_h[4 * q + 1] = a;
      req_h[4 * q + 2] = jj;
      req_h[4 * q + 3] = b;
    }
    HIP_TRY(hipMemcpyAsync(req_d, req_h, 4 * (size_t)m * sizeof(int), hipMemcpyHostToDevice, S->stream));
    launch_measure(S->stream, S->d_sites, S->d_dims, S->N, S->cap_max, envL, envR, m, req_d, num_d);
    HIP_TRY(hipMemcpyAsync(num_h, num_d, (size_t)m * sizeof(double2), hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    const double d = tr.x * tr.x + tr.y * tr.y;
    if (!(d > 0) || !std::isfinite(d)) return fail(LMPO_ENUMERIC, "trace is zero or non-finite");
    for (int q = 0; q < m; ++q) {
      const double2 v = num_h[q];
      out[2 * (q0 + q)] = (v.x * tr.x + v.y * tr.y) / d;
      out[2 * (q0 + q) + 1] = (v.y * tr.x - v.x * tr.y) / d;
    }
  }
  return check_err(S);
}

int lmpo_measure_1q(lmpo_state *S, int32_t n, const int32_t *site, const char *pauli, double *out) {
  if (!S || n < 0 || (n > 0 && (!site || !pauli || !out))) return fail(LMPO_EINVAL, "null argument or n < 0");
  std::vector<int> req;
  for (int q = 0; q < n; ++q) {
    int a = pauli_index(pauli[q]);
    if (site[q] < 0 || site[q] >= S->N) return fail(LMPO_EINVAL, "site index out of range");
    if (a <= 0) return fail(LMPO_EINVAL, "pauli must be one of X, Y, Z");
    req.insert(req.end(), {site[q], a, -1, 0});
  }
  if (n == 0) return LMPO_OK;
  return run_measure(S, req, out);
}

int lmpo_measure_2q(lmpo_state *S, int32_t n, const int32_t *i, const int32_t *j, const char *paulis, double *out) {
  if (!S || n < 0 || (n > 0 && (!i || !j || !paulis || !out))) return fail(LMPO_EINVAL, "null argument or n < 0");
  std::vector<int> req;
  for (int q = 0; q < n; ++q) {
    int a = pauli_index(paulis[2 * q]), b = pauli_index(paulis[2 * q + 1]);
    int ii = i[q], jj = j[q];
    if (ii < 0 || ii >= S->N || jj < 0 || jj >= S->N) return fail(LMPO_EINVAL, "site index out of range");
    if (ii == jj) return fail(LMPO_EINVAL, "2Q observable needs i != j");
    if (a <= 0 || b <= 0) return fail(LMPO_EINVAL, "paulis must be X, Y or Z");
    if (ii > jj) {
      std::swap(ii, jj);
      std::swap(a, b);
    }
    req.insert(req.end(), {ii, a, jj, b});
  }
  if (n == 0) return LMPO_OK;
  return run_measure(S, req, out);
}

int lmpo_bond_dims(lmpo_state *S, int32_t *out) {
  if (!S || !out) return fail(LMPO_EINVAL, "null argument");
  HIP_TRY(hipMemcpyAsync(out, S->d_dims, (S->N - 1) * sizeof(int), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  return check_err(S);
}

int lmpo_discarded_weight(lmpo_state *S, double *out) {
  if (!S || !out) return fail(LMPO_EINVAL, "null argument");
  HIP_TRY(hipMemcpyAsync(out, S->disc, sizeof(double), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  return check_err(S);
}

int lmpo_destroy(lmpo_state *S) {
  if (!S) return LMPO_OK;
  hipError_t e = hipStreamSynchronize(S->stream);
  delete S;
  if (e != hipSuccess) return fail(LMPO_EHIP, std::string("destroy: ") + hipGetErrorString(e));
  return LMPO_OK;
}

int lmpo_get_site(lmpo_state *S, int32_t k, int32_t dims[2], double *out) {
  if (!S || !dims) return fail(LMPO_EINVAL, "null argument");
  if (k < 0 || k >= S->N) return fail(LMPO_EINVAL, "site index out of range");
  int rc = sync_dims(S);
  if (rc) return rc;
  dims[0] = dimL(S, k);
  dims[1] = dimR(S, k);
  if (out)
    HIP_TRY(hipMemcpyAsync(out, S->site[k], (size_t)dims[0] * 4 * dims[1] * sizeof(double2), hipMemcpyDeviceToHost,
                           S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  return LMPO_OK;
}

int lmpo_set_site(lmpo_state *S, int32_t k, int32_t chl, int32_t chr, const double *data) {
  if (!S || !data) return fail(LMPO_EINVAL, "null argument");
  if (k < 0 || k >= S->N) return fail(LMPO_EINVAL, "site index out of range");
  // with room reserved for the Hermitian part, half the capacity is usable
  const int div = S->herm_room ? 2 : 1;
  const int capl = k == 0 ? 1 : capL(S, k) / div, capr = k == S->N - 1 ? 1 : capR(S, k) / div;
  if (chl < 1 || chr < 1 || chl > capl || chr > capr) return fail(LMPO_EINVAL, "site shape exceeds the bond capacity");
  int rc = sync_dims(S);
  if (rc) return rc;
  if (k > 0) S->dims[k - 1] = chl;
  if (k < S->N - 1) S->dims[k] = chr;
  HIP_TRY(hipMemcpyAsync(S->site[k], data, (size_t)chl * 4 * chr * sizeof(double2), hipMemcpyHostToDevice, S->stream));
  HIP_TRY(hipMemcpyAsync(S->d_dims, S->dims.data(), (S->N - 1) * sizeof(int), hipMemcpyHostToDevice, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  return LMPO_OK;
}

int lmpo_set_centre(lmpo_state *S, int32_t c) {
  if (!S) return fail(LMPO_EINVAL, "state is null");
  if (c < 0 || c >= S->N) return fail(LMPO_EINVAL, "centre out of range");
  S->centre = c;
  return LMPO_OK;
}

int lmpo_get_centre(lmpo_state *S, int32_t *c) {
  if (!S || !c) return fail(LMPO_EINVAL, "null argument");
  *c = S->centre;
  return LMPO_OK;
}

int lmpo_get_gate(lmpo_state *S, int32_t bond, int32_t half, double *out) {
  if (!S || !out) return fail(LMPO_EINVAL, "null argument");
  if (bond < 0 || bond >= S->m.nb) return fail(LMPO_EINVAL, "bond out of range");
  std::memcpy(out, &S->gates_host[((size_t)bond * kGateSlots + (half ? 1 : 0)) * 256], 256 * sizeof(double2));
  return LMPO_OK;
}

int lmpo_apply_gate(lmpo_state *S, int32_t k, int32_t half, int32_t ascending) {
  if (!S) return fail(LMPO_EINVAL, "state is null");
  if (k < 0 || k >= S->N - 1) return fail(LMPO_EINVAL, "bond out of range");
  return apply_gate(S, k, half ? 1 : 0, ascending);
}

int lmpo_apply_superop(lmpo_state *S, int32_t i, int32_t j, const double *G) {
  if (!S || !G) return fail(LMPO_EINVAL, "null argument");
  int rc = pair_args(S, i, j);
  if (rc || (rc = upload_user_gate(S, i, j, G))) return rc;
  return apply_pair(S, std::min(i, j), std::max(i, j), S->d_user, true);
}

int lmpo_apply_unitary(lmpo_state *S, int32_t i, int32_t j, const double *U) {
  if (!S || !U) return fail(LMPO_EINVAL, "null argument");
  int rc = pair_args(S, i, j);
  if (rc) return rc;
  std::vector<std::complex<double>> u(16), G(256);
  for (int e = 0; e < 16; ++e) u[e] = {U[2 * e], U[2 * e + 1]};
  for (const auto &v : u)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return fail(LMPO_EINVAL, "non-finite unitary entry");
  unitary_channel_pauli(u.data(), G.data());
  if ((rc = upload_user_gate(S, i, j, reinterpret_cast<const double *>(G.data())))) return rc;
  return apply_pair(S, std::min(i, j), std::max(i, j), S->d_user, true);
}

int lmpo_init_graph_state(lmpo_state *S, int32_t n_pairs, const int32_t *pairs) {
  if (!S) return fail(LMPO_EINVAL, "state is null");
  if (n_pairs < 0 || (n_pairs > 0 && !pairs)) return fail(LMPO_EINVAL, "bad pair list");
  for (int p = 0; p < n_pairs; ++p) {
    int rc = pair_args(S, pairs[2 * p], pairs[2 * p + 1]);
    if (rc) return rc;
  }
  HIP_TRY(hipStreamSynchronize(S->stream));
  std::vector<std::pair<int, int>> plus_x(S->N, {1, 1});
  int rc = upload_product(S, plus_x);
  if (rc) return rc;
  // a fresh initial condition: time 0, nothing discarded yet
  S->step_index = 0;
  const double zd = 0.0;
  HIP_TRY(hipMemcpyAsync(S->disc, &zd, sizeof(double), hipMemcpyHostToDevice, S->stream));
  if (n_pairs == 0) {
    HIP_TRY(hipStreamSynchronize(S->stream));
    return LMPO_OK;
  }
  // CZ = diag(1, 1, 1, -1): rho -> CZ rho CZ on every listed pair
  std::vector<std::complex<double>> cz(16, 0.0), G(256);
  cz[0] = cz[5] = cz[10] = 1.0;
  cz[15] = -1.0;
  unitary_channel_pauli(cz.data(), G.data());
  if ((rc = upload_user_gate(S, 0, 1, reinterpret_cast<const double *>(G.data())))) return rc;
  for (int p = 0; p < n_pairs; ++p) {
    const int a = pairs[2 * p], b = pairs[2 * p + 1];
    if ((rc = apply_pair(S, std::min(a, b), std::max(a, b), S->d_user, true))) return rc;
  }
  return LMPO_OK;
}

int lmpo_hermitize(lmpo_state *S) {
  if (!S) return fail(LMPO_EINVAL, "state is null");
  if (!S->herm_room)
    return fail(LMPO_EUNSUPPORTED, "create the state with force_hermitian_every > 0 to reserve the doubled bonds");
  return hermitize(S);
}

int lmpo_last_spectrum(lmpo_state *S, int32_t n_out, double *sv, int32_t *n_sv, int32_t *kept) {
  if (!S || !n_sv || !kept) return fail(LMPO_EINVAL, "null argument");
  int st[kStats];
  HIP_TRY(hipMemcpyAsync(st, S->stats, sizeof(st), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipMemcpyAsync(kept, S->kept, sizeof(int), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  *n_sv = st[1];
  int n = std::min<int>(n_out, st[1]);
  if (sv && n > 0) {
    HIP_TRY(hipMemcpyAsync(sv, S->sorted, n * sizeof(double), hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
  }
  return LMPO_OK;
}

int lmpo_svd_profile(lmpo_state *S, double out_us[32]) {
  if (!S || !out_us) return fail(LMPO_EINVAL, "null argument");
  unsigned long long t[32];
  HIP_TRY(hipMemcpyAsync(t, S->tprof, sizeof(t), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  int dev = 0, khz = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  auto us = [&](unsigned long long v) { return khz > 0 ? (double)v * 1e3 / khz : 0.0; };
  for (int i = 0; i < 32; ++i) out_us[i] = us(t[i]);
  out_us[3] = (double)t[12];   // shader clock cycles of the first workgroup (whole kernels)
  out_us[4] = (double)t[13];   // pair tasks of the first workgroup
  out_us[7] = (double)t[7];    // launches
  out_us[12] = (double)t[14];  // of which rotated
  out_us[13] = out_us[14] = 0.0;
  out_us[15] = (double)t[15];  // Cholesky-QR passes
  return LMPO_OK;
}

int lmpo_profile_begin(lmpo_state *S, int32_t max_launches) {
  if (!S || max_launches < 1) return fail(LMPO_EINVAL, "null state or max_launches < 1");
  while (S->ev.size() < 2 * (size_t)max_launches) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    S->ev.push_back(e);
  }
  HIP_TRY(hipMemsetAsync(S->alg_flops, 0, sizeof(double), S->stream));
  S->ev_used = 0;
  S->ev_overflow = false;
  S->profiling = true;
  return LMPO_OK;
}

int lmpo_profile_end(lmpo_state *S, double out[3]) {
  if (!S || !out) return fail(LMPO_EINVAL, "null argument");
  S->profiling = false;
  HIP_TRY(hipStreamSynchronize(S->stream));
  double ms = 0.0;
  for (size_t i = 0; i + 1 < S->ev_used; i += 2) {
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, S->ev[i], S->ev[i + 1]));
    ms += t;
  }
  double flops = 0.0;
  HIP_TRY(hipMemcpy(&flops, S->alg_flops, sizeof(double), hipMemcpyDeviceToHost));
  out[0] = (double)(S->ev_used / 2);
  out[1] = ms;
  out[2] = flops;
  if (S->ev_overflow) return fail(LMPO_EINVAL, "more SVD launches than max_launches in the profiling window");
  return LMPO_OK;
}

int lmpo_renyi2(lmpo_state *S, double *out) {
  if (!S || !out) return fail(LMPO_EINVAL, "null argument");
  double n2, t2;
  int rc = purity_and_trace(S, n2, t2, nullptr);
  if (rc) return rc;
  *out = -std::log(n2 / t2);
  return LMPO_OK;
}

int lmpo_osee(lmpo_state *S, int32_t bond, double *out) {
  if (!S || !out) return fail(LMPO_EINVAL, "null argument");
  if (bond < 0 || bond >= S->N - 1) return fail(LMPO_EINVAL, "bond out of range");
  int rc = move_centre(S, bond);
  if (rc) return rc;
  const int R = 4 * (bond == 0 ? 1 : est(S, bond - 1)), C = est(S, bond);
  if ((rc = launch_svd(S, svd_args(S, 3, bond, 0), grid_for(S, std::max(R, C), std::min(R, C))))) return rc;
  double h[2];
  HIP_TRY(hipMemcpyAsync(h, S->aux, 2 * sizeof(double), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  if ((rc = check_err(S))) return rc;
  *out = h[0];
  return LMPO_OK;
}

int lmpo_set_svd_tolerance(lmpo_state *S, double factor) {
  if (!S) return fail(LMPO_EINVAL, "state is null");
  if (!(factor >= 1.0) || !std::isfinite(factor)) return fail(LMPO_EINVAL, "the tolerance factor must be >= 1");
  S->tol_factor = factor;
  return LMPO_OK;
}

int lmpo_set_workgroups(lmpo_state *S, int32_t max_workgroups) {
  if (!S) return fail(LMPO_EINVAL, "state is null");
  if (max_workgroups < 0) return fail(LMPO_EINVAL, "max_workgroups must be >= 0");
  S->wg_cap = max_workgroups;
  return LMPO_OK;
}

int lmpo_set_svd_subspace(lmpo_state *S, int32_t min_cols, int32_t margin, int32_t grow, int32_t iterations,
                          double tol) {
  if (!S) return fail(LMPO_EINVAL, "state is null");
  if (min_cols > 0) {
    if (margin < 16 || margin > kRsiMarginMax) return fail(LMPO_EINVAL, "margin must be in [16, 128]");
    if (grow < 0) return fail(LMPO_EINVAL, "grow must be >= 0");
    if (iterations < 1 || iterations > 64) return fail(LMPO_EINVAL, "iterations must be in [1, 64]");
    if (!(tol > 0.0) || !(tol < 1.0)) return fail(LMPO_EINVAL, "tol must be in (0, 1)");
  }
  S->rsi_min_cols = min_cols > 0 ? min_cols : 0;
  if (min_cols > 0) {
    S->rsi_margin = margin;
    S->rsi_grow = grow;
    S->rsi_iters = iterations;
    S->rsi_tol = tol;
  }
  return LMPO_OK;
}

int lmpo_svd_subspace_stats(lmpo_state *S, int32_t out[3]) {
  if (!S || !out) return fail(LMPO_EINVAL, "null argument");
  int st[kStats];
  HIP_TRY(hipMemcpyAsync(st, S->stats, sizeof(st), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  out[0] = st[3];
  out[1] = st[6];
  out[2] = st[7];
  return LMPO_OK;
}

int lmpo_svd_stats(lmpo_state *S, int32_t out[4]) {
  if (!S || !out) return fail(LMPO_EINVAL, "null argument");
  int st[kStats];
  HIP_TRY(hipMemcpyAsync(st, S->stats, sizeof(st), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  out[0] = st[0];
  out[1] = st[1];
  out[2] = st[4];
  out[3] = st[5];
  return LMPO_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form: many independent chains advance together, one cooperative
// launch per Trotter layer.  Each chain keeps its own state (arena, gates,
// buffers); the batch adds the per-layer tables, one barrier block per chain
// and a plan that splits the co-resident grid between the chains.
// ---------------------------------------------------------------------------
namespace {
constexpr int kMaxBatchBlocks = 4096;

// Planning model of one persistent SVD of an R x C block on G workgroups,
// in microseconds: sweeps x rounds x (pair tasks per workgroup x pair time +
// barrier).  Only the split of the grid between chains depends on it.
struct CostModel {
  double pair_fixed = 6.0, pair_per_row = 0.03, bar_fixed = 2.0, bar_per_wg = 0.05;
};

int jacobi_pairs(int C) {
  int nbp = (C + JB - 1) / JB;
  nbp += nbp & 1;
  if (nbp < 2) nbp = 2;
  return nbp / 2;
}

double svd_cost(int R, int C, int G, const CostModel &m) {
  if (R < C) std::swap(R, C);
  const int npairs = jacobi_pairs(C), rounds = 2 * npairs - 1;
  const double sweeps = 3.0 + 0.9 * std::log2((double)std::max(C, 2));
  const double tb = G == 1 ? 0.2 : m.bar_fixed + m.bar_per_wg * G;
  const int per_wg = (npairs + G - 1) / G;
  return sweeps * rounds * (per_wg * (m.pair_fixed + m.pair_per_row * R) + tb);
}
}  // namespace

namespace {
// Online autotuner of the batched form.  Results do not depend on how the
// grid is split, so the batch can try plans during real steps: for each
// (largest block bucket, precision) it runs real steps under each candidate
// cap on the workgroups per chain, times them with HIP events and keeps the
// fastest.  Each candidate is timed twice, in palindromic order (1, 2, ..., 0,
// 0, ..., 2, 1), and ranked by the sum: steps get dearer as the bond dims
// grow, and the mirrored order cancels that drift to first order.  The table
// lives for the process (one per device), so later batches reuse it.
constexpr int kTuneCaps[] = {1, 2, 4, 8, 16, 0};  // 0: the cost model's choice, uncapped
constexpr int kTuneN = sizeof(kTuneCaps) / sizeof(kTuneCaps[0]);
constexpr int kTuneTrials = 2 * kTuneN;
int tune_candidate(int trial) { return trial < kTuneN ? trial : kTuneTrials - 1 - trial; }
struct TuneEntry {
  double ms[kTuneN] = {};  // summed over the candidate's two trials
  int next = 0;            // next trial (0 .. kTuneTrials - 1)
  int best = -1;           // index into kTuneCaps once all are timed
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, TuneEntry> g_tune;  // (device, log2 bucket, precision)
}  // namespace

struct lmpo_batch {
  std::vector<lmpo_state *> ch;
  hipStream_t stream = nullptr;
  int n = 0, grid_max = 1;
  CostModel model;
  bool autotune = false;
  int wg_cap = 0;  // cap on workgroups per chain in force (0: none)
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  // device tables (caller's arena)
  BatchChain *d_chains = nullptr;
  int *d_block_group = nullptr, *d_block_rank = nullptr, *d_group_size = nullptr;
  unsigned *d_bar = nullptr;
  int *d_centre = nullptr, *d_dims = nullptr;
  double2 *d_tr = nullptr;
  double *d_flops = nullptr;
  std::vector<int> dims_off;
  int dims_total = 0;
  // current plan
  std::vector<int> gsize, block_group, block_rank;
  int total_blocks = 0;
  // pinned staging for table uploads and the bond-dim readback
  char *stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_done = nullptr;
  DimsRing ring;
  long long steps_done = 0;
  std::vector<int> dims_est;
  // profiling window
  bool profiling = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  bool ev_overflow = false;
  ~lmpo_batch() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : tune_ev)
      if (e) (void)hipEventDestroy(e);
    if (stage_done) (void)hipEventDestroy(stage_done);
    if (stage) (void)hipHostFree(stage);
  }
};

namespace {

size_t batch_layout(lmpo_batch *B, char *base, size_t size) {
  Arena a{base, size};
  B->d_chains = a.take<BatchChain>(B->n);
  B->d_block_group = a.take<int>(kMaxBatchBlocks);
  B->d_block_rank = a.take<int>(kMaxBatchBlocks);
  B->d_group_size = a.take<int>(B->n);
  B->d_bar = a.take<unsigned>((size_t)B->n * kBarWords);
  B->d_centre = a.take<int>(B->n);
  B->d_tr = a.take<double2>(B->n);
  B->d_dims = a.take<int>(std::max(B->dims_total, 1));
  B->d_flops = a.take<double>(B->n);
  return a.used;
}

int batch_check_chains(lmpo_state *const *chains, int n) {
  if (!chains || n < 1) return fail(LMPO_EINVAL, "need at least one chain");
  if (n > kMaxBatchBlocks) return fail(LMPO_EUNSUPPORTED, "too many chains for one batch");
  for (int c = 0; c < n; ++c) {
    if (!chains[c]) return fail(LMPO_EINVAL, "null chain in batch");
    if (chains[c]->stream != chains[0]->stream) return fail(LMPO_EINVAL, "all chains of a batch must share one stream");
    if (chains[c]->opt.trotter_order != chains[0]->opt.trotter_order)
      return fail(LMPO_EINVAL, "all chains of a batch must use the same Trotter order");
    if (!chains[c]->chain)
      return fail(LMPO_EUNSUPPORTED, "the batched form runs open chains only (bonds (b, b+1) in order)");
    if (chains[c]->opt.force_hermitian_every > 0)
      return fail(LMPO_EUNSUPPORTED, "the batched form does not take the Hermitian part (force_hermitian_every)");
    for (int d = 0; d < c; ++d)
      if (chains[d] == chains[c]) return fail(LMPO_EINVAL, "a chain appears twice in the batch");
  }
  return LMPO_OK;
}

// Bond dims used for planning: last known value plus a growth margin.
int batch_est(const lmpo_batch *B, int c, int bond) {
  const lmpo_state *S = B->ch[c];
  if (bond < 0 || bond >= S->N - 1) return 1;
  return std::min(S->cap[bond], B->dims_est[B->dims_off[c] + bond] + 8);
}

// Modelled time of one Trotter step of chain c on G workgroups: every gate
// (even bonds twice) and about one centre hop per gate.
double chain_cost(const lmpo_batch *B, int c, int G) {
  const int N = B->ch[c]->N;
  double t = 0.0;
  for (int b = 0; b < N - 1; ++b) {
    const int mult = (b % 2 == 0) ? 2 : 1;
    const int l = b == 0 ? 1 : batch_est(B, c, b - 1), r = b + 1 == N - 1 ? 1 : batch_est(B, c, b + 1);
    t += mult * (svd_cost(4 * l, 4 * r, G, B->model) + svd_cost(4 * l, batch_est(B, c, b), G, B->model));
  }
  return t;
}

int chain_max_pairs(const lmpo_batch *B, int c) {
  const int N = B->ch[c]->N;
  int p = 1;
  for (int b = 0; b < N - 1; ++b) {
    const int l = b == 0 ? 1 : batch_est(B, c, b - 1), r = b + 1 == N - 1 ? 1 : batch_est(B, c, b + 1);
    p = std::max(p, jacobi_pairs(std::min(4 * l, 4 * r)));
  }
  return p;
}

// Split the co-resident grid: start from one workgroup per chain and give
// the next workgroup to the chain with the longest modelled step while that
// shortens it.  Then place each chain's workgroups on one XCD where they fit
// (workgroup b runs on XCD b mod 8), so a chain's barrier and data traffic
// stay within one L2.
void batch_plan(lmpo_batch *B, std::vector<int> &gsize, std::vector<int> &bgroup, std::vector<int> &brank) {
  const int n = B->n, budget = std::min(B->grid_max, kMaxBatchBlocks);
  gsize.assign(n, 1);
  std::vector<double> cost(n);
  std::vector<int> maxg(n);
  for (int c = 0; c < n; ++c) {
    cost[c] = chain_cost(B, c, 1);
    maxg[c] = chain_max_pairs(B, c);
    if (B->wg_cap > 0) maxg[c] = std::min(maxg[c], B->wg_cap);
  }
  int total = n;
  while (total < budget) {
    int worst = 0;
    for (int c = 1; c < n; ++c)
      if (cost[c] > cost[worst]) worst = c;
    if (gsize[worst] >= maxg[worst]) break;
    const double next = chain_cost(B, worst, gsize[worst] + 1);
    if (next >= cost[worst]) break;
    gsize[worst]++;
    cost[worst] = next;
    total++;
  }
  // XCD-aware placement
  constexpr int kXcd = 8;
  std::vector<std::vector<int>> slots(kXcd);
  for (int b = total - 1; b >= 0; --b) slots[b % kXcd].push_back(b);  // popped in increasing order
  std::vector<int> order(n);
  for (int c = 0; c < n; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return gsize[x] > gsize[y]; });
  bgroup.assign(total, -1);
  brank.assign(total, 0);
  for (int c : order) {
    int need = gsize[c], rank = 0;
    while (need > 0) {
      int best = 0;
      for (int x = 1; x < kXcd; ++x)
        if (slots[x].size() > slots[best].size()) best = x;
      // prefer an XCD that holds the whole group
      for (int x = 0; x < kXcd; ++x)
        if ((int)slots[x].size() >= need && slots[x].size() < slots[best].size()) best = x;
      while (need > 0 && !slots[best].empty()) {
        const int b = slots[best].back();
        slots[best].pop_back();
        bgroup[b] = c;
        brank[b] = rank++;
        --need;
      }
    }
  }
}

// Upload through the pinned staging buffer (waits for its previous use).
struct StageCopy {
  void *dst;
  const void *src;
  size_t bytes;
};
int batch_upload(lmpo_batch *B, const std::vector<StageCopy> &copies) {
  size_t need = 0;
  for (const auto &c : copies) need += (c.bytes + 255) & ~size_t(255);
  HIP_TRY(hipEventSynchronize(B->stage_done));
  if (need > B->stage_bytes) {
    if (B->stage) HIP_TRY(hipHostFree(B->stage));
    B->stage = nullptr;
    HIP_TRY(hipHostMalloc((void **)&B->stage, need, hipHostMallocDefault));
    B->stage_bytes = need;
  }
  size_t off = 0;
  for (const auto &c : copies) {
    std::memcpy(B->stage + off, c.src, c.bytes);
    HIP_TRY(hipMemcpyAsync(c.dst, B->stage + off, c.bytes, hipMemcpyHostToDevice, B->stream));
    off += (c.bytes + 255) & ~size_t(255);
  }
  HIP_TRY(hipEventRecord(B->stage_done, B->stream));
  return LMPO_OK;
}

int batch_refresh_estimates(lmpo_batch *B) {
  HIP_TRY(B->ring.before(B->steps_done, B->dims_est.data()));
  return LMPO_OK;
}

// Re-plan from the current estimates; upload the tables if the plan changed.
int batch_replan(lmpo_batch *B) {
  std::vector<int> gs, bg, br;
  batch_plan(B, gs, bg, br);
  if (gs == B->gsize && bg == B->block_group && br == B->block_rank) return LMPO_OK;
  B->gsize = gs;
  B->block_group = bg;
  B->block_rank = br;
  B->total_blocks = (int)bg.size();
  return batch_upload(B, {{B->d_group_size, gs.data(), gs.size() * sizeof(int)},
                          {B->d_block_group, bg.data(), bg.size() * sizeof(int)},
                          {B->d_block_rank, br.data(), br.size() * sizeof(int)}});
}

// Tuning key: device, log2 of the largest (estimated) gate block column count
// over the batch, and the precisions present (bit mask).
std::tuple<int, int, int> tune_key(const lmpo_batch *B) {
  int cmax = 1, prec = 0;
  for (int c = 0; c < B->n; ++c) {
    const int N = B->ch[c]->N;
    prec |= 1 << B->ch[c]->opt.precision;
    for (int b = 0; b < N - 1; ++b) {
      const int l = b == 0 ? 1 : batch_est(B, c, b - 1), r = b + 1 == N - 1 ? 1 : batch_est(B, c, b + 1);
      cmax = std::max(cmax, std::min(4 * l, 4 * r));
    }
  }
  int lg = 0;
  while ((1 << lg) < cmax) ++lg;
  int dev = 0;
  (void)hipGetDevice(&dev);
  return std::make_tuple(dev, lg, prec);
}

int batch_launch(lmpo_batch *B, int local_step, int j, const TrotterLayer &lay, bool last) {
  hipEvent_t *pair = nullptr;
  if (B->profiling) {
    if (B->ev_used + 2 <= B->ev.size()) {
      pair = &B->ev[B->ev_used];
      B->ev_used += 2;
    } else {
      B->ev_overflow = true;
    }
  }
  const int parity = lay.parity, slot = lay.slot;
  if (pair) HIP_TRY(hipEventRecord(pair[0], B->stream));
  HIP_TRY(launch_batch_layer(B->stream, B->d_chains, B->d_block_group, B->d_block_rank, B->d_group_size,
                             B->total_blocks, B->d_bar, (size_t)B->n * kBarWords, local_step, j, parity, slot,
                             last ? 1 : 0));
  if (pair) HIP_TRY(hipEventRecord(pair[1], B->stream));
  return LMPO_OK;
}

}  // namespace

extern "C" {

size_t lmpo_batch_arena_bytes(lmpo_state *const *chains, int32_t n_chains) {
  if (batch_check_chains(chains, n_chains) != LMPO_OK) return 0;
  lmpo_batch tmp;
  tmp.n = n_chains;
  for (int c = 0; c < n_chains; ++c) tmp.dims_total += chains[c]->N - 1;
  return batch_layout(&tmp, nullptr, 0) + 256;
}

int lmpo_batch_create(lmpo_state *const *chains, int32_t n_chains, void *device_arena, size_t arena_bytes,
                      lmpo_batch **out) {
  if (!out) return fail(LMPO_EINVAL, "out is null");
  *out = nullptr;
  int rc = batch_check_chains(chains, n_chains);
  if (rc) return rc;
  if (!device_arena) return fail(LMPO_EINVAL, "device_arena is null");
  if (reinterpret_cast<uintptr_t>(device_arena) % 256) return fail(LMPO_EINVAL, "device_arena must be 256-byte aligned");
  lmpo_batch *B = new lmpo_batch();
  auto cleanup = [&](int code) {
    delete B;
    return code;
  };
  B->n = n_chains;
  B->ch.assign(chains, chains + n_chains);
  B->stream = chains[0]->stream;
  B->dims_off.resize(n_chains);
  for (int c = 0; c < n_chains; ++c) {
    B->dims_off[c] = B->dims_total;
    B->dims_total += chains[c]->N - 1;
  }
  const size_t need = batch_layout(B, reinterpret_cast<char *>(device_arena), arena_bytes);
  if (need > arena_bytes) return cleanup(fail(LMPO_ENOMEM, "batch arena too small: need " + std::to_string(need) + " bytes"));
  B->grid_max = batch_grid_size();
  if (n_chains > B->grid_max)
    return cleanup(fail(LMPO_EUNSUPPORTED, "more chains than co-resident workgroups (" + std::to_string(B->grid_max) + ")"));
  hipError_t e = hipEventCreateWithFlags(&B->stage_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(B->stage_done, B->stream);
  if (e == hipSuccess) e = B->ring.init(B->dims_total);
  if (e == hipSuccess) e = hipEventCreate(&B->tune_ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&B->tune_ev[1]);
  if (e == hipSuccess) e = hipMemsetAsync(B->d_flops, 0, n_chains * sizeof(double), B->stream);
  if (e != hipSuccess) return cleanup(fail(LMPO_EHIP, std::string("batch init: ") + hipGetErrorString(e)));
  // estimates from the chains' current bond dims
  B->dims_est.assign(std::max(B->dims_total, 1), 1);
  for (int c = 0; c < n_chains; ++c) {
    lmpo_state *S = chains[c];
    if ((rc = sync_dims(S))) return cleanup(rc);
    std::copy(S->dims.begin(), S->dims.end(), B->dims_est.begin() + B->dims_off[c]);
  }
  if ((rc = batch_replan(B))) return cleanup(rc);
  *out = B;
  return LMPO_OK;
}

int lmpo_batch_evolve_step(lmpo_batch *B, int32_t n_steps) {
  if (!B) return fail(LMPO_EINVAL, "batch is null");
  if (n_steps < 0) return fail(LMPO_EINVAL, "n_steps must be >= 0");
  if (n_steps == 0) return LMPO_OK;
  // per-call chain records: the chains may have been advanced on their own
  // since the last call, so centre and step parity come from their states
  std::vector<BatchChain> recs(B->n);
  std::vector<int> centres(B->n);
  for (int c = 0; c < B->n; ++c) {
    lmpo_state *S = B->ch[c];
    BatchChain &r = recs[c];
    r.L = svd_args(S, 0, 0, 0);
    r.L.bar = B->d_bar + (size_t)c * kBarWords;
    r.L.alg_flops = B->d_flops + c;
    r.gates = S->d_gates;
    r.centre = B->d_centre + c;
    r.tr = B->d_tr + c;
    r.dims_out = B->d_dims + B->dims_off[c];
    r.precision = S->opt.precision;
    r.force_trace = S->opt.force_trace ? 1 : 0;
    // layer L n + j runs ascending iff even: with L even only j decides
    r.step_parity = trotter_layers(S->opt.trotter_order).size() % 2 ? (int)(S->step_index & 1) : 0;
    centres[c] = S->centre;
  }
  int rc = batch_upload(B, {{B->d_chains, recs.data(), recs.size() * sizeof(BatchChain)},
                            {B->d_centre, centres.data(), centres.size() * sizeof(int)}});
  if (rc) return rc;
  for (int s = 0; s < n_steps; ++s) {
    if ((rc = batch_refresh_estimates(B))) return rc;
    // autotuner: the cap of this step (a candidate under trial, or the best known)
    int trial = -1;
    std::tuple<int, int, int> key;
    {
      key = tune_key(B);
      std::lock_guard<std::mutex> lock(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end() && it->second.best >= 0) {
        B->wg_cap = kTuneCaps[it->second.best];
      } else if (B->autotune) {
        trial = g_tune[key].next;
        B->wg_cap = kTuneCaps[tune_candidate(trial)];
      } else {
        B->wg_cap = 0;
      }
    }
    if ((rc = batch_replan(B))) return rc;
    if (trial >= 0) HIP_TRY(hipEventRecord(B->tune_ev[0], B->stream));
    const std::vector<TrotterLayer> &layers = trotter_layers(B->ch[0]->opt.trotter_order);
    const int ls = layers.size() % 2 ? s : 0;  // see step_parity
    for (int j = 0; j < (int)layers.size(); ++j)
      if ((rc = batch_launch(B, ls, j, layers[j], j + 1 == (int)layers.size()))) return rc;
    if (trial >= 0) {
      HIP_TRY(hipEventRecord(B->tune_ev[1], B->stream));
      HIP_TRY(hipEventSynchronize(B->tune_ev[1]));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, B->tune_ev[0], B->tune_ev[1]));
      std::lock_guard<std::mutex> lock(g_tune_mu);
      TuneEntry &te = g_tune[key];
      if (te.best < 0 && te.next == trial) {
        te.ms[tune_candidate(trial)] += ms;
        te.next = trial + 1;
        if (te.next == kTuneTrials) te.best = (int)(std::min_element(te.ms, te.ms + kTuneN) - te.ms);
      }
    }
    HIP_TRY(B->ring.after(B->steps_done, B->d_dims, B->stream));
    B->steps_done++;
  }
  // host mirrors: the last layer (even bonds) ends ascending on the last even
  // bond or descending on bond 0
  for (int c = 0; c < B->n; ++c) {
    lmpo_state *S = B->ch[c];
    const long long last = S->step_index + n_steps - 1;
    const bool asc = ((last + 2) & 1) == 0;
    const int last_even = ((S->N - 2) / 2) * 2;
    S->centre = asc ? last_even + 1 : 0;
    S->step_index += n_steps;
  }
  return LMPO_OK;
}

int lmpo_batch_sync(lmpo_batch *B) {
  if (!B) return fail(LMPO_EINVAL, "batch is null");
  HIP_TRY(hipStreamSynchronize(B->stream));
  for (int c = 0; c < B->n; ++c) {
    int rc = check_err(B->ch[c]);
    if (rc) return fail(rc, "chain " + std::to_string(c) + ": " + g_err);
  }
  return LMPO_OK;
}

int lmpo_batch_set_autotune(lmpo_batch *B, int32_t enable) {
  if (!B) return fail(LMPO_EINVAL, "batch is null");
  B->autotune = enable != 0;
  return LMPO_OK;
}

int lmpo_autotune_table(int32_t max_entries, int32_t *log2_bucket, int32_t *precisions, int32_t *cap,
                        double *best_ms, int32_t *n_entries) {
  if (!n_entries || max_entries < 0 || (max_entries > 0 && (!log2_bucket || !precisions || !cap || !best_ms)))
    return fail(LMPO_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(g_tune_mu);
  int n = 0, dev = 0;
  (void)hipGetDevice(&dev);
  for (const auto &kv : g_tune) {
    if (std::get<0>(kv.first) != dev || kv.second.best < 0) continue;
    if (n < max_entries) {
      log2_bucket[n] = std::get<1>(kv.first);
      precisions[n] = std::get<2>(kv.first);
      cap[n] = kTuneCaps[kv.second.best];
      best_ms[n] = 0.5 * kv.second.ms[kv.second.best];
    }
    ++n;
  }
  *n_entries = n;
  return LMPO_OK;
}

int lmpo_batch_plan(lmpo_batch *B, int32_t *workgroups) {
  if (!B || !workgroups) return fail(LMPO_EINVAL, "null argument");
  for (int c = 0; c < B->n; ++c) workgroups[c] = B->gsize[c];
  return LMPO_OK;
}

int lmpo_batch_profile_begin(lmpo_batch *B, int32_t max_launches) {
  if (!B || max_launches < 1) return fail(LMPO_EINVAL, "null batch or max_launches < 1");
  while (B->ev.size() < 2 * (size_t)max_launches) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    B->ev.push_back(e);
  }
  HIP_TRY(hipMemsetAsync(B->d_flops, 0, B->n * sizeof(double), B->stream));
  B->ev_used = 0;
  B->ev_overflow = false;
  B->profiling = true;
  return LMPO_OK;
}

int lmpo_batch_profile_end(lmpo_batch *B, double out[3]) {
  if (!B || !out) return fail(LMPO_EINVAL, "null argument");
  B->profiling = false;
  HIP_TRY(hipStreamSynchronize(B->stream));
  double ms = 0.0;
  for (size_t i = 0; i + 1 < B->ev_used; i += 2) {
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, B->ev[i], B->ev[i + 1]));
    ms += t;
  }
  std::vector<double> f(B->n);
  HIP_TRY(hipMemcpy(f.data(), B->d_flops, B->n * sizeof(double), hipMemcpyDeviceToHost));
  double flops = 0.0;
  for (double x : f) flops += x;
  out[0] = (double)(B->ev_used / 2);
  out[1] = ms;
  out[2] = flops;
  if (B->ev_overflow) return fail(LMPO_EINVAL, "more layer launches than max_launches in the profiling window");
  return LMPO_OK;
}

int lmpo_batch_destroy(lmpo_batch *B) {
  if (!B) return LMPO_OK;
  hipError_t e = hipStreamSynchronize(B->stream);
  delete B;
  if (e != hipSuccess) return fail(LMPO_EHIP, std::string("batch destroy: ") + hipGetErrorString(e));
  return LMPO_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Adjoint gradient of a final-time one-qubit expectation value with respect
// to every model parameter (lmpo_grad_*).
//
// F = Tr(O rho_T) / Tr(rho_T).  Every bond generator is linear in each
// parameter theta, and a gate's derivative is dG/dtheta = K G with
// K = (d/dtheta exp(x L)) exp(-x L).  Then
//   dF/dtheta = sum_g s_g <mu_g, K_g rho_g>,
// rho_g the state right after gate g, mu_g the co-state after it (mu_T =
// (o - F 1) / Tr(rho_T), carried back through every later gate by its
// transpose: the pairing of coefficient vectors is bilinear), s_g = 1 / the
// product of the traces divided out at the ends of the steps from g's own
// step on.  <mu, K rho> = tr(K Gamma) with Gamma the two-site transition
// density of the two MPS on the gate's sites.
//
// Forward: the state runs the steps as lmpo_evolve_step does, with a
// snapshot of all site tensors at the start of every step.  Backward, step by
// step from the last: the step is replayed from its snapshot recording every
// gate's output (bit-identical: same kernels, same inputs), then its gates
// are walked in reverse: Gamma between the co-state and the recorded state,
// the contributions of the gate's 14 parameters, and the co-state advanced by
// the transposed gate (truncated like any gate, the state's chi_max and
// cutoff).  The state ends as after the forward run.
// ---------------------------------------------------------------------------
struct lmpo_grad {
  lmpo_state *S = nullptr;  // the state (the caller's)
  lmpo_state *C = nullptr;  // co-state, in the workspace
  int n_steps = 0, max_ops = 0, P = 0;
  size_t snap = 0;
  char *ckpt = nullptr;  // n_steps + 1 snapshots
  Recorder rec;          // one step's gate snapshots
  double2 *L = nullptr, *R = nullptr, *W = nullptr, *E = nullptr, *Fr = nullptr, *gam = nullptr;
  double2 *K = nullptr;  // [nb][kGateSlots][kGradLocal][16][16]
  int *pidx = nullptr;   // [nb][kGradLocal] global parameter index
  double2 *grad = nullptr, *traces = nullptr, *one = nullptr;
  double2 *src = nullptr;  // an output's source MPS (bond 2), [N][16]
  bool series = false;     // co-state capacities doubled for sources
  bool keep = false;       // every step's gate snapshots kept from the forward run (no replay)
  char *rec_base = nullptr;                   // gate snapshot slots: one step's, or all steps' when keep
  std::vector<std::vector<OpRecord>> kept;    // the forward run's gate records per step when keep
  double *disc_save = nullptr;
  int *stats_save = nullptr;
  std::vector<int> ckpt_centre;
  ~lmpo_grad() { delete C; }
};

namespace {

constexpr int kGradLocal = 15;  // parameters of one gate: 6 per site, J, Jz of its generator, and tau

lmpo_model model_view(const ModelHost &m) {
  lmpo_model v;
  v.n_qubits = m.N;
  v.n_bonds = m.nb;
  v.bond_ij = m.bonds.data();
  v.J = m.J.data();
  v.Jz = m.Jz.data();
  v.hx = m.hx.data();
  v.hy = m.hy.data();
  v.hz = m.hz.data();
  v.g0 = m.g0.data();
  v.g1 = m.g1.data();
  v.g2 = m.g2.data();
  return v;
}

// Gates (SWAPs included) one step applies, and the gate table slots it uses.
int grad_ops_per_step(const lmpo_state *S) {
  int n = 0;
  if (S->chain) {
    for (const TrotterLayer &l : trotter_layers(S->opt.trotter_order))
      for (int b = l.parity; b < S->N - 1; b += 2) ++n;
    return n;
  }
  for (int b = 0; b < S->m.nb; ++b) n += 1 + 2 * (S->m.bonds[2 * b + 1] - S->m.bonds[2 * b] - 1);
  return 2 * n * (int)sweep_slots(S->opt.trotter_order).size();
}
std::vector<int> grad_slots(const lmpo_state *S) {
  std::vector<int> out;
  if (S->chain)
    for (const TrotterLayer &l : trotter_layers(S->opt.trotter_order)) out.push_back(l.slot);
  else
    out = sweep_slots(S->opt.trotter_order);
  std::sort(out.begin(), out.end());
  out.erase(std::unique(out.begin(), out.end()), out.end());
  return out;
}

size_t grad_layout(lmpo_grad *G, const lmpo_state *S, int n_steps, const lmpo_options &co_opt, bool keep,
                   char *base, size_t size, char **co, size_t co_bytes) {
  Arena a{base, size};
  const int co_mult = co_opt.force_hermitian_every > 0 ? 2 : 1;
  const size_t cm = (size_t)std::max(S->cap_max, compute_sizes(S->N, co_opt.chi_max, co_mult).cap_max);
  *co = a.take<char>(co_bytes);
  G->snap = snapshot_bytes(S);
  G->max_ops = grad_ops_per_step(S);
  G->ckpt = a.take<char>((size_t)(n_steps + 1) * G->snap);
  G->rec_base = a.take<char>((keep ? (size_t)n_steps : 1) * G->max_ops * G->snap);
  G->rec.slots = G->rec_base;
  G->rec.stride = G->snap;
  G->rec.capacity = (size_t)G->max_ops;
  G->L = a.take<double2>(cm * cm);
  G->R = a.take<double2>(cm * cm);
  G->W = a.take<double2>(4 * cm * cm);
  G->E = a.take<double2>(16 * cm * cm);
  G->Fr = a.take<double2>(16 * cm * cm);
  G->gam = a.take<double2>(256);
  G->K = a.take<double2>((size_t)S->m.nb * kGateSlots * kGradLocal * 256);
  G->pidx = a.take<int>((size_t)S->m.nb * kGradLocal);
  G->P = 6 * S->N + 2 * S->m.nb + 1;  // the model's parameters, then tau
  G->grad = a.take<double2>(G->P);
  G->traces = a.take<double2>(n_steps);
  G->one = a.take<double2>(1);
  G->src = a.take<double2>((size_t)S->N * 16);
  G->disc_save = a.take<double>(1);
  G->stats_save = a.take<int>(kStats);
  return a.used;
}

// Controls of the co-state: the state's, with chi_max and cutoff replaced
// where the caller gives them (chi_max > 0, cutoff >= 0).
int grad_check(const lmpo_state *S, int n_steps, int co_chi, double co_cut, int flags, lmpo_options *co_opt) {
  if (!S) return fail(LMPO_EINVAL, "state is null");
  if (n_steps < 1) return fail(LMPO_EINVAL, "n_steps must be >= 1");
  if (S->opt.force_hermitian_every > 0)
    return fail(LMPO_EUNSUPPORTED, "the gradient does not pass through the Hermitian part");
  if (!std::isfinite(co_cut)) return fail(LMPO_EINVAL, "costate_cutoff must be finite");
  *co_opt = S->opt;
  // The co-state of a Hermitian observable has real coefficients in the
  // Pauli basis, where every propagator (and so its transpose) is real: it
  // runs in the real-arithmetic form whatever the state's precision, unless
  // the complex form is asked for (a co-state copied from a complex state).
  co_opt->precision = (flags & LMPO_GRAD_COMPLEX_COSTATE) ? LMPO_FP64 : LMPO_FP64_REAL;
  if (co_chi > 0) co_opt->chi_max = co_chi;
  if (co_cut >= 0) co_opt->cutoff = co_cut;
  if (co_opt->chi_max < 2) return fail(LMPO_EUNSUPPORTED, "the co-state needs chi_max >= 2 (it starts at bond 2)");
  if (co_opt->chi_max > kMaxDim / 4) return fail(LMPO_EUNSUPPORTED, "costate_chi_max above 512 is not supported");
  if (flags & ~(LMPO_GRAD_SERIES | LMPO_GRAD_KEEP_GATES | LMPO_GRAD_COMPLEX_COSTATE))
    return fail(LMPO_EINVAL, "unknown gradient flags");
  if (flags & LMPO_GRAD_SERIES) {
    // room for an output's source beside the co-state: the bond capacities
    // doubled (the co-state never takes a step, so no Hermitian part is formed)
    if (co_opt->chi_max > kMaxDim / 8)
      return fail(LMPO_EUNSUPPORTED, "LMPO_GRAD_SERIES needs a co-state chi_max <= 256");
    co_opt->force_hermitian_every = 1;
  }
  return LMPO_OK;
}

size_t costate_bytes(const lmpo_state *S, const lmpo_options &co_opt) {
  lmpo_model mv = model_view(S->m);
  return lmpo_arena_bytes(&mv, &co_opt);
}

// K = (d/dtheta exp(x L_b)) exp(-x L_b) for the kGradLocal parameters of bond
// b: the Frechet derivative of the exponential in the direction x dL/dtheta
// is the upper-right block of exp([[x L, x dL], [0, x L]]) (C. Van Loan,
// IEEE Trans. Autom. Control 23 (1978) 395).  dL/dtheta is the generator of a
// model with theta = 1 and every other parameter 0 (same bonds).
int build_k_table(lmpo_grad *G, std::vector<std::complex<double>> &Kh, std::vector<int> &ph) {
  const lmpo_state *S = G->S;
  const ModelHost &m = S->m;
  const int nb = m.nb, N = m.N;
  Kh.assign((size_t)nb * kGateSlots * kGradLocal * 256, 0.0);
  ph.assign((size_t)nb * kGradLocal, -1);
  using cd = std::complex<double>;
  std::vector<cd> Lb(256), dL(256), B(1024), EB(1024), X(256), Ginv(256);
  for (int b = 0; b < nb; ++b) {
    const int i = m.bonds[2 * b], j = m.bonds[2 * b + 1];
    bond_generator_pauli(m, b, Lb.data());
    std::vector<std::pair<std::vector<double> ModelHost::*, int>> par;
    std::vector<int> gidx;
    std::vector<double> ModelHost::*keys[6] = {&ModelHost::hx, &ModelHost::hy, &ModelHost::hz,
                                              &ModelHost::g0, &ModelHost::g1, &ModelHost::g2};
    for (int s : {i, j})
      for (int q = 0; q < 6; ++q) {
        par.push_back({keys[q], s});
        gidx.push_back(q * N + s);
      }
    par.push_back({&ModelHost::J, b});
    gidx.push_back(6 * N + b);
    par.push_back({&ModelHost::Jz, b});
    gidx.push_back(6 * N + nb + b);
    gidx.push_back(6 * N + 2 * nb);  // tau: d/dtau exp(f tau L) = f L exp(f tau L), so K = f L
    for (int p = 0; p < kGradLocal; ++p) ph[(size_t)b * kGradLocal + p] = gidx[p];
    for (int slot : grad_slots(S)) {
      const double x = gate_fraction(slot) * S->opt.tau;
      for (int e = 0; e < 256; ++e) X[e] = -x * Lb[e];
      if (!expm_pade13(16, X.data(), Ginv.data())) return fail(LMPO_ENUMERIC, "matrix exponential failed");
      {
        std::complex<double> *Kt = &Kh[(((size_t)b * kGateSlots + slot) * kGradLocal + (kGradLocal - 1)) * 256];
        for (int e = 0; e < 256; ++e) Kt[e] = gate_fraction(slot) * Lb[e];
      }
      for (int p = 0; p < kGradLocal - 1; ++p) {
        ModelHost u = m;
        for (auto *v : {&u.J, &u.Jz, &u.hx, &u.hy, &u.hz, &u.g0, &u.g1, &u.g2}) std::fill(v->begin(), v->end(), 0.0);
        (u.*(par[p].first))[par[p].second] = 1.0;
        bond_generator_pauli(u, b, dL.data());
        std::fill(B.begin(), B.end(), cd(0.0));
        for (int r = 0; r < 16; ++r)
          for (int c = 0; c < 16; ++c) {
            B[r * 32 + c] = B[(r + 16) * 32 + c + 16] = x * Lb[r * 16 + c];
            B[r * 32 + c + 16] = x * dL[r * 16 + c];
          }
        if (!expm_pade13(32, B.data(), EB.data())) return fail(LMPO_ENUMERIC, "matrix exponential failed");
        cd *Kp = &Kh[(((size_t)b * kGateSlots + slot) * kGradLocal + p) * 256];
        for (int r = 0; r < 16; ++r)
          for (int c = 0; c < 16; ++c) {
            cd acc = 0.0;
            for (int t = 0; t < 16; ++t) acc += EB[r * 32 + 16 + t] * Ginv[t * 16 + c];
            Kp[r * 16 + c] = acc;
          }
      }
    }
  }
  return LMPO_OK;
}

// Gamma of the co-state C and the recorded state (sites at `snap`, bond dims
// rd) on sites (k, k + 1), into G->gam.  C->dims must be current on the host.
int transition_density(lmpo_grad *G, int k, const char *snap, const int *rd) {
  lmpo_state *S = G->S, *C = G->C;
  const int N = S->N;
  hipStream_t st = S->stream;
  auto md = [&](int b) { return (b < 0 || b >= N - 1) ? 1 : C->dims[b]; };
  auto qd = [&](int b) { return (b < 0 || b >= N - 1) ? 1 : rd[b]; };
  auto rs = [&](int s) {
    return reinterpret_cast<const double2 *>(snap + (reinterpret_cast<const char *>(S->site[s]) -
                                                     reinterpret_cast<const char *>(S->site[0])));
  };
  auto gemm = [&](int M, int Nn, int K, const double2 *A, long long sam, long long sak, long long sab,
                  const double2 *B, long long sbk, long long sbn, long long sbb, double2 *Cc, long long scm,
                  long long scn, long long scb, int batch) {
    ZgemmArgs g{M, Nn, K, A, sam, sak, sab, B, sbk, sbn, sbb, Cc, scm, scn, scb};
    launch_zgemm(st, g, batch);
  };
  // left environment L[p][q] over sites < k
  HIP_TRY(hipMemcpyAsync(G->L, G->one, sizeof(double2), hipMemcpyDeviceToDevice, st));
  for (int s = 0; s < k; ++s) {
    const int pl = md(s - 1), pr = md(s), ql = qd(s - 1), qr = qd(s);
    // W[p][(a q')] = sum_q L[p][q] r_s[q][(a q')]
    gemm(pl, 4 * qr, ql, G->L, ql, 1, 0, rs(s), 4 * qr, 1, 0, G->W, 4 * qr, 1, 0, 1);
    // L'[p'][q'] = sum_{(p a)} mu_s[(p a)][p'] W[(p a)][q']
    gemm(pr, qr, 4 * pl, C->site[s], 1, pr, 0, G->W, qr, 1, 0, G->L, qr, 1, 0, 1);
  }
  // right environment R[p][q] over sites > k + 1
  HIP_TRY(hipMemcpyAsync(G->R, G->one, sizeof(double2), hipMemcpyDeviceToDevice, st));
  for (int s = N - 1; s > k + 1; --s) {
    const int pl = md(s - 1), pr = md(s), ql = qd(s - 1), qr = qd(s);
    // W[(p a)][q'] = sum_{p'} mu_s[(p a)][p'] R[p'][q']
    gemm(4 * pl, qr, pr, C->site[s], pr, 1, 0, G->R, qr, 1, 0, G->W, qr, 1, 0, 1);
    // R'[p][q] = sum_{(a q')} W[p][(a q')] r_s[q][(a q')]
    gemm(pl, ql, 4 * qr, G->W, 4 * qr, 1, 0, rs(s), 1, 4 * qr, 0, G->R, ql, 1, 0, 1);
  }
  const int pl = md(k - 1), pm = md(k), pr = md(k + 1), ql = qd(k - 1), qm = qd(k), qr = qd(k + 1);
  // E[a][p'][(c q')] = sum_p mu_k[p][a][p'] sum_q L[p][q] r_k[q][(c q')]
  gemm(pl, 4 * qm, ql, G->L, ql, 1, 0, rs(k), 4 * qm, 1, 0, G->W, 4 * qm, 1, 0, 1);
  gemm(pm, 4 * qm, pl, C->site[k], 1, 4 * pm, pm, G->W, 4 * qm, 1, 0, G->E, 4 * qm, 1, (long long)pm * 4 * qm, 4);
  // Fr[d][(p' b)][q'] = sum_{q''} (sum_{p''} mu_{k+1}[(p' b)][p''] R[p''][q'']) r_{k+1}[q'][d][q'']
  gemm(4 * pm, qr, pr, C->site[k + 1], pr, 1, 0, G->R, qr, 1, 0, G->W, qr, 1, 0, 1);
  gemm(4 * pm, qm, qr, G->W, qr, 1, 0, rs(k + 1), 1, 4 * qr, qr, G->Fr, qm, 1, (long long)4 * pm * qm, 4);
  launch_transition_reduce(st, G->E, G->Fr, pm, qm, G->gam);
  HIP_TRY(hipGetLastError());
  return LMPO_OK;
}

// A sum of product covectors sum_k c_k prod_s v_{k,s} as an MPS in the co-state:
// v_{k,s} = sqrt(2) e_{a_k[s]} in the Pauli basis (the covector of the Pauli
// factor a_k[s], index 0 the trace), bond dimension K (a row on the first
// site, block-diagonal inside, a column carrying the c_k on the last; K <= 4
// fits every bond capacity).  With `canonical` set, an exact QR sweep then
// makes it left-orthonormal with the centre on the last site (bonds fall to
// their rank).
struct CostateTerm {
  double c;
  std::vector<int> a;
};
void terms_host(int N, const std::vector<CostateTerm> &terms, std::vector<std::vector<double2>> &host) {
  const int K = (int)terms.size();
  const double r2 = std::sqrt(2.0);
  host.assign(N, {});
  for (int s = 0; s < N; ++s) {
    const int nl = s == 0 ? 1 : K, nr = s == N - 1 ? 1 : K;
    host[s].assign((size_t)nl * 4 * nr, make_double2(0.0, 0.0));
    for (int k = 0; k < K; ++k) {
      const int l = s == 0 ? 0 : k, r = s == N - 1 ? 0 : k;
      const double v = s == N - 1 ? r2 * terms[k].c : r2;
      double2 &e = host[s][((size_t)l * 4 + terms[k].a[s]) * nr + r];
      e.x += v;
    }
  }
}

int init_costate(lmpo_grad *G, const std::vector<CostateTerm> &terms, bool canonical) {
  lmpo_state *C = G->C;
  const int N = C->N, K = (int)terms.size();
  if (K < 1 || K > 4) return fail(LMPO_EINVAL, "internal: co-state of 1 to 4 product terms");
  for (int b = 0; b < N - 1; ++b)
    if (C->cap[b] < K)
      return fail(LMPO_EUNSUPPORTED, "this objective's co-state starts at bond " + std::to_string(K) +
                                         ": the co-state's chi_max must be at least that");
  std::vector<std::vector<double2>> host;
  terms_host(N, terms, host);
  for (int s = 0; s < N; ++s)
    HIP_TRY(hipMemcpyAsync(C->site[s], host[s].data(), host[s].size() * sizeof(double2), hipMemcpyHostToDevice,
                           C->stream));
  std::fill(C->dims.begin(), C->dims.end(), K);
  HIP_TRY(hipMemcpyAsync(C->d_dims, C->dims.data(), (N - 1) * sizeof(int), hipMemcpyHostToDevice, C->stream));
  HIP_TRY(hipStreamSynchronize(C->stream));
  C->centre = 0;
  return canonical ? move_centre(C, N - 1) : LMPO_OK;
}

// mu <- mu + sum_k c_k prod_s v_{k,s} (one or two terms: an output's source
// has two): the direct sum of the co-state and the source (bonds + the term
// count, in the capacity the series flag doubled), an exact QR sweep from the
// left, then the truncated two-site SVD of every bond from the right (the
// identity gate, the co-state's chi_max and cutoff).  The centre ends on site 0.
int add_costate_source(lmpo_grad *G, const std::vector<CostateTerm> &terms) {
  lmpo_state *C = G->C;
  const int N = C->N, kb = (int)terms.size();
  if (kb < 1 || kb > 2) return fail(LMPO_EINVAL, "internal: a source has one or two product terms");
  std::vector<std::vector<double2>> host;
  terms_host(N, terms, host);
  for (int s = 0; s < N; ++s)
    HIP_TRY(hipMemcpyAsync(G->src + (size_t)s * 16, host[s].data(), host[s].size() * sizeof(double2),
                           hipMemcpyHostToDevice, C->stream));
  for (int k = 0; k < N; ++k) {
    HIP_TRY(hipMemcpyAsync(C->T, C->site[k], C->site_elems[k] * sizeof(double2), hipMemcpyDeviceToDevice,
                           C->stream));
    launch_mps_sum_site(C->stream, C->T, G->src + (size_t)k * 16, C->site[k], C->d_dims, N, k, kb);
    HIP_TRY(hipGetLastError());
  }
  launch_add_dims(C->stream, C->d_dims, N - 1, kb);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(C->stream));  // the host copies of the source outlive their upload
  C->centre = 0;
  int rc = move_centre(C, N - 1);
  for (int k = N - 2; k >= 0 && !rc; --k) rc = apply_gate_dev(C, k, C->d_ident, 0);
  return rc;
}

// <o, rho> for the Pauli string a on the state as it stands: o goes into the
// co-state as a product (bond 1) and the transition density of the last bond,
// traced with the identity, is the whole contraction.
int string_expectation_numerator(lmpo_grad *G, const std::vector<int> &a, std::complex<double> &out) {
  lmpo_state *S = G->S;
  int rc = init_costate(G, {{1.0, a}}, false);
  if (rc || (rc = sync_dims(S))) return rc;
  if ((rc = transition_density(G, S->N - 2, reinterpret_cast<const char *>(S->site[0]), S->dims.data()))) return rc;
  double2 gam[256];
  HIP_TRY(hipMemcpyAsync(gam, G->gam, sizeof(gam), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  out = 0.0;
  for (int x = 0; x < 16; ++x) out += std::complex<double>(gam[17 * x].x, gam[17 * x].y);
  return LMPO_OK;
}

}  // namespace

extern "C" {

size_t lmpo_grad_arena_bytes(lmpo_state *S, int32_t n_steps, int32_t costate_chi_max, double costate_cutoff,
                             int32_t flags) {
  lmpo_options co_opt;
  if (grad_check(S, n_steps, costate_chi_max, costate_cutoff, flags, &co_opt)) return 0;
  const size_t co = costate_bytes(S, co_opt);
  if (co == 0) return 0;
  lmpo_grad tmp;
  tmp.S = S;
  char *dummy = nullptr;
  return grad_layout(&tmp, S, n_steps, co_opt, (flags & LMPO_GRAD_KEEP_GATES) != 0, nullptr, 0, &dummy, co) + 256;
}

int lmpo_grad_create(lmpo_state *S, int32_t n_steps, int32_t costate_chi_max, double costate_cutoff, int32_t flags,
                     void *device_arena, size_t arena_bytes, lmpo_grad **out) {
  if (!out) return fail(LMPO_EINVAL, "out is null");
  *out = nullptr;
  lmpo_options co_opt;
  int rc = grad_check(S, n_steps, costate_chi_max, costate_cutoff, flags, &co_opt);
  if (rc) return rc;
  if (!device_arena) return fail(LMPO_EINVAL, "device_arena is null");
  if (reinterpret_cast<uintptr_t>(device_arena) % 256) return fail(LMPO_EINVAL, "device_arena must be 256-byte aligned");
  const size_t co = costate_bytes(S, co_opt);
  if (co == 0) return LMPO_EINVAL;
  lmpo_grad *G = new lmpo_grad();
  G->S = S;
  G->n_steps = n_steps;
  G->series = (flags & LMPO_GRAD_SERIES) != 0;
  char *co_arena = nullptr;
  G->keep = (flags & LMPO_GRAD_KEEP_GATES) != 0;
  const size_t need = grad_layout(G, S, n_steps, co_opt, G->keep, reinterpret_cast<char *>(device_arena), arena_bytes,
                                  &co_arena, co);
  if (need > arena_bytes) {
    delete G;
    return fail(LMPO_ENOMEM, "gradient arena too small: need " + std::to_string(need) + " bytes");
  }
  G->ckpt_centre.assign(n_steps + 1, 0);
  auto bail = [&](int code) {
    delete G;
    return code;
  };
  // co-state: same model and controls, its gate table replaced by the transposes
  lmpo_model mv = model_view(S->m);
  if ((rc = lmpo_create(&mv, &co_opt, "+z", co_arena, co, S->stream, &G->C))) return bail(rc);
  std::vector<double2> gt(S->gates_host.size());
  for (size_t g = 0; g < gt.size() / 256; ++g)
    for (int r = 0; r < 16; ++r)
      for (int c = 0; c < 16; ++c)  // transposed; real (its imaginary parts are round-off)
        gt[g * 256 + r * 16 + c] = make_double2(S->gates_host[g * 256 + c * 16 + r].real(), 0.0);
  std::vector<std::complex<double>> Kh;
  std::vector<int> ph;
  if ((rc = build_k_table(G, Kh, ph))) return bail(rc);
  const double2 one = make_double2(1.0, 0.0);
  hipError_t e = hipMemcpyAsync(G->C->d_gates, gt.data(), gt.size() * sizeof(double2), hipMemcpyHostToDevice,
                                S->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(G->K, Kh.data(), Kh.size() * sizeof(double2), hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(G->pidx, ph.data(), ph.size() * sizeof(int), hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(G->one, &one, sizeof(double2), hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return bail(fail(LMPO_EHIP, std::string("gradient setup: ") + hipGetErrorString(e)));
  *out = G;
  return LMPO_OK;
}

}  // extern "C"

namespace {

// Forward run of the gradient: the state advances by the workspace's steps
// with a snapshot at every step start and one of the final state; the traces
// divided out per step and tr(rho_T) come back to the host.
int grad_forward(lmpo_grad *G, long long &step0, std::complex<double> &trT, std::vector<double2> &tr_host,
                 const std::function<int(int)> &observe = nullptr) {
  lmpo_state *S = G->S;
  const int N = S->N, T = G->n_steps;
  hipStream_t st = S->stream;
  step0 = S->step_index;
  int rc;
  HIP_TRY(hipMemsetAsync(G->grad, 0, (size_t)G->P * sizeof(double2), st));
  if (G->keep) G->kept.assign(T, {});
  for (int n = 0; n < T; ++n) {
    if ((rc = save_snapshot(S, G->ckpt + (size_t)n * G->snap))) return rc;
    G->ckpt_centre[n] = S->centre;
    if (G->keep) {  // record this step's gates into its own slots
      G->rec.ops.clear();
      G->rec.slots = G->rec_base + (size_t)n * G->max_ops * G->snap;
      S->rec = &G->rec;
    }
    rc = one_step(S, step0 + n);
    S->rec = nullptr;
    if (rc) return rc;
    if (G->keep) G->kept[n] = G->rec.ops;
    if (S->opt.force_trace) HIP_TRY(hipMemcpyAsync(G->traces + n, S->tr, sizeof(double2), hipMemcpyDeviceToDevice, st));
    if (observe && (rc = observe(n + 1))) return rc;  // after n + 1 steps
  }
  if ((rc = save_snapshot(S, G->ckpt + (size_t)T * G->snap))) return rc;
  G->ckpt_centre[T] = S->centre;
  // the replays of the backward pass add to these; the forward run's values are restored at the end
  HIP_TRY(hipMemcpyAsync(G->disc_save, S->disc, sizeof(double), hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(G->stats_save, S->stats, kStats * sizeof(int), hipMemcpyDeviceToDevice, st));
  launch_trace(st, S->d_sites, S->d_dims, N, S->tr);
  double2 t;
  HIP_TRY(hipMemcpyAsync(&t, S->tr, sizeof(double2), hipMemcpyDeviceToHost, st));
  tr_host.assign(T, make_double2(1.0, 0.0));
  if (S->opt.force_trace)
    HIP_TRY(hipMemcpyAsync(tr_host.data(), G->traces, T * sizeof(double2), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  trT = std::complex<double>(t.x, t.y);
  if (!(std::abs(trT) > 0) || !std::isfinite(std::abs(trT))) return fail(LMPO_ENUMERIC, "trace is zero or non-finite");
  return LMPO_OK;
}

// Backward pass from the co-state mu_T already in G->C: per step from the
// last, replay with gate snapshots, then the gates in reverse (transition
// density, contributions, transposed gate).  Leaves the state as after the
// forward run and writes the real parts of the gradient.
// sources[n] (when given and not empty): two product terms added to the
// co-state when the pass reaches the end of step n, scaled by the traces
// divided out after step n; the co-state is zero (and the steps skipped)
// until the first of them unless `live`.
int grad_backward(lmpo_grad *G, long long step0, const std::vector<double2> &tr_host, double *grad_out,
                  const std::vector<std::vector<CostateTerm>> *sources = nullptr, bool live = true) {
  lmpo_state *S = G->S, *C = G->C;
  const int N = S->N, T = G->n_steps;
  hipStream_t st = S->stream;
  int rc;
  std::complex<double> scale = 1.0;
  std::vector<int> rd;
  for (int n = T - 1; n >= 0; --n) {
    if (sources && !(*sources)[n].empty()) {
      std::vector<CostateTerm> terms = (*sources)[n];
      for (CostateTerm &t : terms) t.c /= scale.real();  // times the traces divided out after step n
      rc = live ? add_costate_source(G, terms) : init_costate(G, terms, true);
      if (rc) return rc;
      live = true;
    }
    scale /= std::complex<double>(tr_host[n].x, tr_host[n].y);
    if (!live) continue;  // zero co-state: nothing to carry back yet
    if (G->keep) {  // the forward run's records of this step
      G->rec.slots = G->rec_base + (size_t)n * G->max_ops * G->snap;
      G->rec.ops = G->kept[n];
    } else {  // replay the step from its snapshot, recording every gate
      if ((rc = load_snapshot(S, G->ckpt + (size_t)n * G->snap))) return rc;
      S->centre = G->ckpt_centre[n];
      G->rec.ops.clear();
      G->rec.slots = G->rec_base;
      S->rec = &G->rec;
      rc = one_step(S, step0 + n);
      S->rec = nullptr;
      if (rc) return rc;
    }
    const int nops = (int)G->rec.ops.size();
    rd.assign((size_t)nops * (N - 1), 1);
    for (int i = 0; i < nops; ++i)
      HIP_TRY(hipMemcpyAsync(&rd[(size_t)i * (N - 1)], G->rec.slots + (size_t)i * G->rec.stride +
                             snapshot_dims_offset(S), (N - 1) * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int i = nops - 1; i >= 0; --i) {
      const OpRecord &op = G->rec.ops[i];
      if (op.bond < 0) {
        if ((rc = apply_gate_dev(C, op.k, C->d_swap, op.asc ? 0 : 1))) return rc;
        continue;
      }
      if ((rc = sync_dims(C))) return rc;
      if ((rc = transition_density(G, op.k, G->rec.slots + (size_t)i * G->rec.stride, &rd[(size_t)i * (N - 1)])))
        return rc;
      const size_t kb = ((size_t)op.bond * kGateSlots + op.slot) * kGradLocal;
      launch_grad_accumulate(st, G->K + kb * 256, G->pidx + (size_t)op.bond * kGradLocal, kGradLocal, G->gam,
                             make_double2(scale.real(), scale.imag()), G->grad);
      HIP_TRY(hipGetLastError());
      if ((rc = apply_gate_dev(C, op.k, gate_ptr(C, op.bond, op.slot), op.asc ? 0 : 1))) return rc;
    }
  }
  if ((rc = load_snapshot(S, G->ckpt + (size_t)T * G->snap))) return rc;
  S->centre = G->ckpt_centre[T];
  S->step_index = step0 + T;
  HIP_TRY(hipMemcpyAsync(S->disc, G->disc_save, sizeof(double), hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(S->stats, G->stats_save, kStats * sizeof(int), hipMemcpyDeviceToDevice, st));
  std::vector<double2> gh(G->P);
  HIP_TRY(hipMemcpyAsync(gh.data(), G->grad, (size_t)G->P * sizeof(double2), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if ((rc = sync_dims(S))) return rc;
  if ((rc = check_err(S)) || (rc = check_err(C))) return rc;
  for (int p = 0; p < G->P; ++p) {
    if (!std::isfinite(gh[p].x)) return fail(LMPO_ENUMERIC, "non-finite gradient");
    grad_out[p] = gh[p].x;
  }
  return LMPO_OK;
}

}  // namespace

extern "C" {

int lmpo_grad_run(lmpo_grad *G, const char *paulis, double F_out[2], double *grad_out) {
  if (!G || !paulis || !F_out || !grad_out) return fail(LMPO_EINVAL, "null argument");
  lmpo_state *S = G->S;
  const int N = S->N;
  if (std::strlen(paulis) != (size_t)N) return fail(LMPO_EINVAL, "paulis must hold one of I, X, Y, Z per qubit");
  std::vector<int> a(N);
  std::vector<int> req;  // the string as a 1Q / 2Q measurement request when it has one or two factors
  for (int s = 0; s < N; ++s) {
    a[s] = pauli_index(paulis[s]);
    if (a[s] < 0) return fail(LMPO_EINVAL, "paulis must hold one of I, X, Y, Z per qubit");
    if (a[s] > 0) req.insert(req.end(), {s, a[s]});
  }
  if (req.empty()) return fail(LMPO_EINVAL, "paulis must name at least one X, Y or Z");
  long long step0;
  std::complex<double> trT;
  std::vector<double2> tr_host;
  int rc = grad_forward(G, step0, trT, tr_host);
  if (rc) return rc;
  // F = <string>: one or two factors through the measurement kernels (as
  // lmpo_measure_1q / _2q), more through the transition density of o and rho_T
  double fo[2];
  if (req.size() <= 4) {
    if (req.size() == 2) req.insert(req.end(), {-1, 0});
    if ((rc = run_measure(S, req, fo))) return rc;
  } else {
    std::complex<double> num;
    if ((rc = string_expectation_numerator(G, a, num))) return rc;
    const std::complex<double> f = num / trT;
    fo[0] = f.real();
    fo[1] = f.imag();
  }
  // mu_T = (o - F 1) / tr; F and tr are real up to round-off, which is dropped
  const double tr = trT.real();
  if ((rc = init_costate(G, {{1.0 / tr, a}, {-fo[0] / tr, std::vector<int>(N, 0)}}, true))) return rc;
  if ((rc = grad_backward(G, step0, tr_host, grad_out))) return rc;
  F_out[0] = fo[0];
  F_out[1] = fo[1];
  return LMPO_OK;
}

int lmpo_grad_run_series(lmpo_grad *G, const char *paulis, int32_t n_out, const int32_t *out_steps,
                         const double *weights, double *F_out, double *grad_out) {
  if (!G || !paulis || !out_steps || !weights || !F_out || !grad_out) return fail(LMPO_EINVAL, "null argument");
  if (!G->series) return fail(LMPO_EUNSUPPORTED, "create the workspace with LMPO_GRAD_SERIES for output sources");
  lmpo_state *S = G->S;
  const int N = S->N, T = G->n_steps;
  if (std::strlen(paulis) != (size_t)N) return fail(LMPO_EINVAL, "paulis must hold one of I, X, Y, Z per qubit");
  std::vector<int> a(N);
  std::vector<int> req;
  for (int s = 0; s < N; ++s) {
    a[s] = pauli_index(paulis[s]);
    if (a[s] < 0) return fail(LMPO_EINVAL, "paulis must hold one of I, X, Y, Z per qubit");
    if (a[s] > 0) req.insert(req.end(), {s, a[s]});
  }
  if (req.empty()) return fail(LMPO_EINVAL, "paulis must name at least one X, Y or Z");
  if (n_out < 1) return fail(LMPO_EINVAL, "n_out must be >= 1");
  std::vector<int> slot(T + 1, -1);  // output index of the state after n steps
  for (int k = 0; k < n_out; ++k) {
    if (out_steps[k] < 1 || out_steps[k] > T || (k > 0 && out_steps[k] <= out_steps[k - 1]))
      return fail(LMPO_EINVAL, "out_steps must increase strictly within 1..n_steps");
    if (!std::isfinite(weights[k])) return fail(LMPO_EINVAL, "non-finite weight");
    slot[out_steps[k]] = k;
  }
  if (req.size() == 2) req.insert(req.end(), {-1, 0});
  std::vector<double> F(2 * (size_t)n_out), trk(n_out);
  auto observe = [&](int done) -> int {
    const int k = slot[done];
    if (k < 0) return LMPO_OK;
    launch_trace(S->stream, S->d_sites, S->d_dims, N, S->tr);
    double2 t;
    HIP_TRY(hipMemcpyAsync(&t, S->tr, sizeof(double2), hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    trk[k] = t.x;
    if (!(std::abs(t.x) > 0) || !std::isfinite(t.x)) return fail(LMPO_ENUMERIC, "trace is zero or non-finite");
    if (req.size() <= 4) return run_measure(S, req, &F[2 * (size_t)k]);
    std::complex<double> num;
    int rc = string_expectation_numerator(G, a, num);
    const std::complex<double> f = num / std::complex<double>(t.x, t.y);
    F[2 * (size_t)k] = f.real();
    F[2 * (size_t)k + 1] = f.imag();
    return rc;
  };
  long long step0;
  std::complex<double> trT;
  std::vector<double2> tr_host;
  int rc = grad_forward(G, step0, trT, tr_host, observe);
  if (rc) return rc;
  // the source of output k: w_k (o - F_k 1) / tr_k at the end of its step
  std::vector<std::vector<CostateTerm>> sources(T);
  for (int k = 0; k < n_out; ++k) {
    const double w = weights[k];
    if (w == 0.0) continue;  // no source (a zero co-state is never formed: all-zero weights give a zero gradient)
    sources[out_steps[k] - 1] = {{w / trk[k], a}, {-(w * F[2 * (size_t)k]) / trk[k], std::vector<int>(N, 0)}};
  }
  if ((rc = grad_backward(G, step0, tr_host, grad_out, &sources, false))) return rc;  // restores the state
  std::copy(F.begin(), F.end(), F_out);
  return LMPO_OK;
}

int lmpo_grad_run_connected(lmpo_grad *G, int32_t i, int32_t j, const char *paulis, double F_out[2],
                            double *grad_out) {
  if (!G || !paulis || !F_out || !grad_out) return fail(LMPO_EINVAL, "null argument");
  lmpo_state *S = G->S;
  const int N = S->N;
  if (i < 0 || j < 0 || i >= N || j >= N || i == j) return fail(LMPO_EINVAL, "a correlator needs two distinct qubits");
  if (std::strlen(paulis) != 2) return fail(LMPO_EINVAL, "paulis must hold two of X, Y, Z");
  int ai = pauli_index(paulis[0]), aj = pauli_index(paulis[1]);
  if (ai <= 0 || aj <= 0) return fail(LMPO_EINVAL, "paulis must hold two of X, Y, Z");
  if (i > j) {
    std::swap(i, j);
    std::swap(ai, aj);
  }
  for (int b = 0; b < N - 1; ++b)  // before the state moves: the four-term co-state must fit
    if (G->C->cap[b] < 4)
      return fail(LMPO_EUNSUPPORTED, "the connected correlator's co-state starts at bond 4: the co-state's "
                                     "chi_max must be at least 4");
  long long step0;
  std::complex<double> trT;
  std::vector<double2> tr_host;
  int rc = grad_forward(G, step0, trT, tr_host);
  if (rc) return rc;
  double f[6];  // <a_i b_j>, <a_i>, <b_j> as (re, im)
  if ((rc = run_measure(S, {i, ai, j, aj, i, ai, -1, 0, j, aj, -1, 0}, f))) return rc;
  const double Fij = f[0], Fi = f[2], Fj = f[4], tr = trT.real();
  // C = F_ij - F_i F_j, dC = dF_ij - F_j dF_i - F_i dF_j with dF_x = (o_x - F_x 1) / tr:
  // mu_T = (o_ij - F_j o_i - F_i o_j + (2 F_i F_j - F_ij) 1) / tr
  std::vector<int> oij(N, 0), oi(N, 0), oj(N, 0), one(N, 0);
  oij[i] = oi[i] = ai;
  oij[j] = oj[j] = aj;
  if ((rc = init_costate(G, {{1.0 / tr, oij}, {-Fj / tr, oi}, {-Fi / tr, oj}, {(2.0 * Fi * Fj - Fij) / tr, one}},
                         true)))
    return rc;
  if ((rc = grad_backward(G, step0, tr_host, grad_out))) return rc;
  F_out[0] = Fij - Fi * Fj;
  F_out[1] = f[1] - (f[3] * Fj + Fi * f[5]);
  return LMPO_OK;
}

int lmpo_grad_run_renyi2(lmpo_grad *G, double *S2_out, double *grad_out) {
  if (!G || !S2_out || !grad_out) return fail(LMPO_EINVAL, "null argument");
  lmpo_state *S = G->S, *C = G->C;
  const int N = S->N;
  if (S->opt.precision != LMPO_FP64_REAL && C->opt.precision == LMPO_FP64_REAL)
    return fail(LMPO_EUNSUPPORTED, "the Renyi-2 gradient of a state in a complex form needs a workspace created "
                                   "with LMPO_GRAD_COMPLEX_COSTATE: its co-state starts as a copy of the state's "
                                   "tensors (the real-arithmetic form is the other way)");
  if (!G->series)
    return fail(LMPO_EUNSUPPORTED, "create the workspace with LMPO_GRAD_SERIES for the Renyi-2 gradient (its "
                                   "co-state holds the state plus one bond)");
  for (int b = 0; b < N - 1; ++b)  // before the state moves
    if (C->cap[b] < S->cap[b] + 1)
      return fail(LMPO_EUNSUPPORTED, "the Renyi-2 co-state holds the state plus one bond: its chi_max must be at "
                                     "least the state's");
  long long step0;
  std::complex<double> trT;
  std::vector<double2> tr_host;
  int rc = grad_forward(G, step0, trT, tr_host);
  if (rc) return rc;
  double P, t2;
  double2 tr;
  if ((rc = purity_and_trace(S, P, t2, &tr)) || (rc = sync_dims(S))) return rc;
  // S_2 = -ln(P / tr^2) with P = <rho, rho> (real coefficients, so the
  // bilinear pairing is the norm): dS_2 = -2 <rho, drho> / P + 2 <1, drho> / tr,
  // mu_T = (-2 / P) (rho - (P / tr) 1).  The co-state is the bracket (the
  // state's own tensors plus one product term, compressed), and the factor
  // -2 / P scales the gradient at the end.
  for (int k = 0; k < N; ++k) {
    const size_t n = (size_t)(k == 0 ? 1 : S->dims[k - 1]) * 4 * (k == N - 1 ? 1 : S->dims[k]);
    HIP_TRY(hipMemcpyAsync(C->site[k], S->site[k], n * sizeof(double2), hipMemcpyDeviceToDevice, C->stream));
  }
  C->dims = S->dims;
  HIP_TRY(hipMemcpyAsync(C->d_dims, C->dims.data(), (N - 1) * sizeof(int), hipMemcpyHostToDevice, C->stream));
  HIP_TRY(hipStreamSynchronize(C->stream));
  if ((rc = add_costate_source(G, {{-P / tr.x, std::vector<int>(N, 0)}}))) return rc;
  if ((rc = grad_backward(G, step0, tr_host, grad_out))) return rc;
  for (int p = 0; p < G->P; ++p) grad_out[p] *= -2.0 / P;
  S2_out[0] = -std::log(P / t2);
  return LMPO_OK;
}

int lmpo_grad_run_osee(lmpo_grad *G, int32_t bond, double *value, double *grad_out) {
  if (!G || !value || !grad_out) return fail(LMPO_EINVAL, "null argument");
  lmpo_state *S = G->S, *C = G->C;
  const int N = S->N;
  if (bond < 0 || bond >= N - 1) return fail(LMPO_EINVAL, "bond out of range");
  // the Pauli-basis coefficients of rho, and so those of the co-state, are
  // real whatever the gauge of the tensors: a complex-form state only needs a
  // co-state that holds its tensors exactly
  if (S->opt.precision != LMPO_FP64_REAL && C->opt.precision == LMPO_FP64_REAL)
    return fail(LMPO_EUNSUPPORTED, "the OSEE gradient of a state in a complex form needs a workspace created with "
                                   "LMPO_GRAD_COMPLEX_COSTATE: its co-state starts as a copy of the state's tensors "
                                   "(the real-arithmetic form is the other way)");
  for (int b = 0; b < N - 1; ++b)  // before the state moves
    if (C->cap[b] < S->cap[b] || S->cap[b] > kOseeRows)
      return fail(LMPO_EUNSUPPORTED, "the OSEE co-state starts as a copy of the state: its chi_max must be at least "
                                     "the state's");
  long long step0;
  std::complex<double> trT;
  std::vector<double2> tr_host;
  int rc = grad_forward(G, step0, trT, tr_host);
  if (rc || (rc = sync_dims(S))) return rc;
  for (int k = 0; k < N; ++k) {
    const size_t n = (size_t)(k == 0 ? 1 : S->dims[k - 1]) * 4 * (k == N - 1 ? 1 : S->dims[k]);
    HIP_TRY(hipMemcpyAsync(C->site[k], S->site[k], n * sizeof(double2), hipMemcpyDeviceToDevice, C->stream));
  }
  C->dims = S->dims;
  HIP_TRY(hipMemcpyAsync(C->d_dims, C->dims.data(), (N - 1) * sizeof(int), hipMemcpyHostToDevice, C->stream));
  HIP_TRY(hipStreamSynchronize(C->stream));
  C->centre = S->centre;
  // the bond's SVD through an identity gate swept left to right, nothing
  // truncated but exact zeros (the bond cannot grow): site bond + 1 becomes
  // diag(s) V^T with right-orthonormal sites after it; the kernel rescales its
  // rows to dS/ds_i and reports S
  const double cut = C->opt.cutoff;
  C->opt.cutoff = 0.0;
  rc = apply_gate_dev(C, bond, C->d_ident, 1);
  C->opt.cutoff = cut;
  if (rc) return rc;
  double *res = reinterpret_cast<double *>(G->gam);  // free until the backward pass
  launch_osee_costate(C->stream, C->d_sites, C->d_dims, N, bond + 1, res);
  HIP_TRY(hipGetLastError());
  double h[2] = {0.0, 0.0};
  HIP_TRY(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, C->stream));
  HIP_TRY(hipStreamSynchronize(C->stream));
  if ((rc = check_err(C))) return rc;
  if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return fail(LMPO_ENUMERIC, "non-finite entropy");
  if (h[1] > 0.0) {
    rc = grad_backward(G, step0, tr_host, grad_out);
  } else {  // a zero co-state (one weight, or all equal): a zero gradient, the state restored as usual
    const std::vector<std::vector<CostateTerm>> none(G->n_steps);
    rc = grad_backward(G, step0, tr_host, grad_out, &none, false);
  }
  if (rc) return rc;
  *value = h[0];
  return LMPO_OK;
}

lmpo_state *lmpo_grad_costate(lmpo_grad *G) { return G ? G->C : nullptr; }

size_t lmpo_probe_fp64_mfma_bytes(void) { return (size_t)2048 * 256 * sizeof(double); }

int lmpo_probe_fp64_mfma(void *hip_stream, void *device_buffer, size_t buffer_bytes, double *tflops) {
  if (!device_buffer || !tflops) return fail(LMPO_EINVAL, "null argument");
  const int blocks = 2048, iters = 4096;  // 8 workgroups per compute unit, about 7 ms at the datasheet peak
  if (buffer_bytes < (size_t)blocks * 256 * sizeof(double)) return fail(LMPO_EINVAL, "probe buffer too small");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  double *out = reinterpret_cast<double *>(device_buffer);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  float ms = 0.0f;
  if (e == hipSuccess) {
    launch_mfma_f64_probe(st, blocks, iters, out);  // warm-up
    e = hipEventRecord(e0, st);
  }
  if (e == hipSuccess) {
    launch_mfma_f64_probe(st, blocks, iters, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(LMPO_EHIP, std::string("probe: ") + hipGetErrorString(e));
  const double flops = (double)blocks * 4 * iters * 8 * 2048.0;  // 4 wavefronts per workgroup
  *tflops = flops / (ms * 1e-3) / 1e12;
  return LMPO_OK;
}

int lmpo_grad_costate_dims(lmpo_grad *G, int32_t *out) {
  if (!G || !out) return fail(LMPO_EINVAL, "null argument");
  return lmpo_bond_dims(G->C, out);
}

int lmpo_grad_destroy(lmpo_grad *G) {
  if (!G) return LMPO_OK;
  hipError_t e = hipStreamSynchronize(G->S->stream);
  delete G;
  if (e != hipSuccess) return fail(LMPO_EHIP, std::string("destroy: ") + hipGetErrorString(e));
  return LMPO_OK;
}

}  // extern "C"
