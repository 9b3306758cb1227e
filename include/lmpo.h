/*
 * lmpo.h -- C ABI of an MI355X (gfx950) library that evolves the vectorised
 * density matrix |rho>> of N qubits, stored as a matrix product state with
 * local dimension 4, under the Lindblad master equation of
 *   H. Landa and G. Misguich, "Nonlocal correlations in noisy multiqubit
 *   systems simulated using matrix product operators", arXiv:2203.05871:
 *   Eq. (dtrho) with the Hamiltonian Eq. (H0), interactions Eq. (K_def) and
 *   the dissipators Eqs. (D0), (D1), (D2); state format Eq. (mpo_def), App. A.
 *
 * One call of lmpo_evolve_step performs second-order Trotter steps made of
 * two-site propagators exp(x L_b), each followed by a truncated SVD that keeps
 * the more severe of a discarded-weight cutoff and a maximal bond dimension
 * (App. B, parameters cut_off_rho / max_dim_rho of Sec. 6), with the trace
 * forced to one after every step (b_force_rho_trace, Sec. 6).  The cut never
 * splits a multiplet of singular values (neighbours closer than 1e-4 times the
 * larger; the paper does not say which vectors of a degenerate multiplet to
 * keep, and any choice is an SVD): a cut set by the cutoff moves past the
 * multiplet while chi_max allows, otherwise in front of it.
 *
 * Conventions
 *  - All functions return 0 (LMPO_OK) or a negative error code; a message is
 *    then available from lmpo_last_error() (thread-local, valid until the
 *    next call on the same thread).
 *  - Host pointers are read during the call only; the library keeps copies.
 *  - Device memory: the caller owns one device buffer (the "arena") of at
 *    least lmpo_arena_bytes() bytes, 256-byte aligned, that must outlive the
 *    state.  The library never allocates or frees device memory.
 *  - Streams: every device operation of a state is enqueued on the
 *    hipStream_t given at creation (NULL = the default stream).  Calls that
 *    return host values (trace, measure, bond dims, weights, sync)
 *    synchronise that stream.  A state must be used from one host thread at a
 *    time; distinct states are independent.
 *  - Storage in the arena: site k holds A_k[l][a][r] (row-major, complex
 *    double interleaved re/im) in the normalised Pauli basis a = (1, x, y, z),
 *    P_a = sigma^a / sqrt(2), i.e. rho = sum c_{a_1..a_N} P_{a_1} x ... x P_{a_N}
 *    (Eq. mpo_def with orthonormal basis operators).
 */
#ifndef LMPO_H
#define LMPO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LMPO_OK = 0,
  LMPO_EINVAL = -1,       /* invalid or missing argument (the paper's solver stops with an error there, Sec. 6) */
  LMPO_ENOMEM = -2,       /* arena too small */
  LMPO_EHIP = -3,         /* HIP runtime error; the message carries its name */
  LMPO_ENUMERIC = -4,     /* NaN/Inf in a singular value or observable, or tr(rho) = 0 */
  LMPO_EUNSUPPORTED = -5  /* valid input this version does not handle */
};

/* LMPO_FP64_REAL: the real-arithmetic form.  In the Hermitian Pauli basis every
 * Lindblad propagator, SWAP, unitary channel and Pauli / graph initial state is
 * real, so the coefficients stay real: contractions, Gram matrices, Jacobi
 * rotations and V updates run in real FP64 (one product per complex four),
 * the storage keeps its complex layout with zero imaginary parts, and rho is
 * Hermitian by construction (Hermitisation is a no-op). */
enum { LMPO_FP64 = 0, LMPO_FP32_CONTRACT = 1, LMPO_FP64_REAL = 2 };

/* Model parameters (Sec. 2.1).  bond_ij lists the coupled pairs (i, j), i < j;
 * each bond contributes J (s+_i s-_j + s-_i s+_j) + (1/2) Jz s^z_i s^z_j
 * (Eq. K_def read as one term per unordered pair).  Qubit indices are
 * positions along the MPS path (Sec. 2.3), so a pair may be several sites
 * apart (a ladder or plaquette folded onto the path); every qubit must belong
 * to at least one bond, whose generators carry its on-site terms (shared
 * equally among its bonds).  Per-site arrays have
 * length n_qubits: h_x, h_y, h_z of Eq. (H0) and the rates g0, g1, g2 of
 * Eqs. (D0) (relaxation to s^z = +1), (D1) (to s^z = -1), (D2) (dephasing). */
typedef struct {
  int32_t n_qubits;
  int32_t n_bonds;
  const int32_t *bond_ij; /* [n_bonds][2] */
  const double *J;        /* [n_bonds] */
  const double *Jz;       /* [n_bonds] */
  const double *hx, *hy, *hz;   /* [n_qubits] */
  const double *g0, *g1, *g2;   /* [n_qubits], >= 0 */
} lmpo_model;

/* Numerical controls of the solver (Sec. 6). */
typedef struct {
  double tau;            /* time step, > 0 */
  int32_t trotter_order; /* 2; 3 (open chain only): the product A(7/24) B(2/3) A(3/4) B(-2/3)
                            A(-1/24) B(1) of the even (A) and odd (B) bond layers (R. D. Ruth,
                            1983); or 4: the symmetric triple product S2(w1 t) S2(w0 t) S2(w1 t),
                            w1 = 1/(2 - 2^(1/3)), w0 = 1 - 2 w1 (7 layers).  Others:
                            LMPO_EUNSUPPORTED */
  int32_t chi_max;       /* max_dim_rho, >= 1 */
  double cutoff;         /* cut_off_rho: largest discarded squared Schmidt weight,
                            relative to the block's total; >= 0 (a multiplet at the
                            cut is kept whole when chi_max allows) */
  int32_t precision;     /* LMPO_FP64, LMPO_FP32_CONTRACT (two-site contractions
                            in FP32 with FP32 accumulation, SVD/truncation/trace FP64),
                            or LMPO_FP64_REAL (real arithmetic, see above) */
  int32_t force_trace;   /* 1: rho -> rho / tr(rho) after every step */
  int32_t force_hermitian_every; /* force_rho_hermitian_step: k >= 1 replaces rho by
                            (rho + rho^+)/2 after every k-th step (before the trace is
                            forced), 0 never.  k >= 1 doubles the bond capacities (arena
                            about 4x) and needs chi_max <= 256 */
} lmpo_options;

typedef struct lmpo_state lmpo_state;

/* Bytes of device memory a state of this model/options needs (0 on invalid
 * input; lmpo_last_error() then says why). */
size_t lmpo_arena_bytes(const lmpo_model *model, const lmpo_options *opt);

/* Create a state in the Pauli product state init_pauli (Sec. 2.2): either one
 * label such as "+z" for all qubits or n_qubits labels concatenated ("+z-x+y..."),
 * sign then axis x|y|z.  Builds the gate table exp(x L_b) for every time
 * fraction x/tau the schedule uses, on the host in FP64, and uploads it.
 * hip_stream is a hipStream_t (NULL for the default stream). */
int lmpo_create(const lmpo_model *model, const lmpo_options *opt, const char *init_pauli,
                void *device_arena, size_t arena_bytes, void *hip_stream, lmpo_state **out);

/* Enqueue n_steps >= 0 Trotter steps.  Open chain (bond b = (b, b+1) for
 * b = 0..N-2, in that order): layers A(tau/2) B(tau) A(tau/2) over even bonds
 * (A) and odd bonds (B) (orders 3 and 4: the six or seven layers of the
 * composition; layer L n + j of step n runs ascending in k iff even).  Any
 * other bond list: the symmetric sweep F(tau/2) R(tau/2), F applying
 * exp(tau/2 L_b) for b = 0, 1, ..., R the same factors in reverse order (order
 * 4: S2(w1 tau) S2(w0 tau) S2(w1 tau) of such sweeps); a pair (i, j) with
 * j > i + 1 is applied by SWAP gates carrying site j to i + 1, the propagator
 * on (i, i + 1), and SWAP gates carrying it back.  Each gate (SWAPs included)
 * moves the orthogonality centre onto its two sites (exact), applies the
 * 16 x 16 superoperator to the two-site block, truncates by SVD and restores
 * canonical form; then rho -> rho / tr(rho) if force_trace.  The step is the
 * gate-by-gate (TEBD) form of the Trotter product of App. B; the truncation
 * rule is the more severe of cut_off_rho and max_dim_rho (App. B, Sec. 6). */
int lmpo_evolve_step(lmpo_state *s, int32_t n_steps);

/* tr(rho) (Sec. 2.4) as (re, im); synchronises. */
int lmpo_trace(lmpo_state *s, double out_re_im[2]);

/* rho -> rho / tr(rho) (complex division; the trace forcing of Sec. 6,
 * b_force_rho_trace); asynchronous. */
int lmpo_renormalize(lmpo_state *s);

/* <sigma^a_i> = Tr(rho sigma^a_i) / Tr(rho) (Eq. mu) for n requests:
 * site[n], pauli[n] in 'X','Y','Z'; out[n][2] = (re, im).  Synchronises. */
int lmpo_measure_1q(lmpo_state *s, int32_t n, const int32_t *site, const char *pauli, double *out);

/* <sigma^a_i sigma^b_j> / Tr(rho) (Eq. 2Qdef), i != j, paulis[n][2] = (a, b)
 * for (i[k], j[k]); out[n][2] = (re, im).  Synchronises. */
int lmpo_measure_2q(lmpo_state *s, int32_t n, const int32_t *i, const int32_t *j,
                    const char *paulis, double *out);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lmpo_measure_2q with
 * the same arguments, results and kernels, but whose working memory (the
 * trace, the two identity environments of (N + 1) x chi_cap complex entries
 * each, the request rows and the numerators) lives in a fixed 2 MiB device
 * array of the library (one per GPU, held until the process ends) instead of
 * the state's arena.  It calls no hipMalloc / hipFree.  A state needing more
 * than 2 MiB, i.e. 2 (N + 1) chi_cap * 16 bytes + 128 KiB (chi_cap the largest
 * bond capacity), gives LMPO_EUNSUPPORTED before anything runs.  Every call on
 * one GPU shares that array and leaves its contents behind: calls that overlap
 * in time on one GPU (several host threads or streams) race and must be
 * serialised by the caller.  The state's device must be current.
 * Synchronises. */
int lmpo_measure_2q_noalloc(lmpo_state *s, int32_t n, const int32_t *i, const int32_t *j,
                            const char *paulis, double *out);

/* Second Renyi entropy S_2 = -ln tr(rho^2) (Eq. S_2, Sec. 2.4), evaluated as
 * -ln( <<rho|rho>> / |tr rho|^2 ): <<rho|rho>> = tr(rho^dagger rho) is the squared
 * norm of the orthogonality centre (the state is kept in mixed-canonical form)
 * and equals tr(rho^2) for Hermitian rho.  Synchronises. */
int lmpo_renyi2(lmpo_state *s, double *out);

/* Operator-space entanglement entropy across bond (bond, bond+1) (Eq. OSEE,
 * Sec. 2.4): the von Neumann entropy of the normalised Schmidt weights
 * s_j^2 / sum s^2 of |rho>>.  Moves the orthogonality centre onto site `bond`
 * (exact hops; the state is unchanged) and takes the singular values of that
 * site on the GPU.  Synchronises. */
int lmpo_osee(lmpo_state *s, int32_t bond, double *out);

/* Current bond dimensions chi_0..chi_{N-2}; synchronises. */
int lmpo_bond_dims(lmpo_state *s, int32_t *out);

/* Sum over all truncations so far of (discarded squared weight / total squared
 * weight) of the two-site block; synchronises. */
int lmpo_discarded_weight(lmpo_state *s, double *out);

/* Wait for the state's queued work and report deferred numerical errors. */
int lmpo_sync(lmpo_state *s);

/* Release host-side resources (the arena stays the caller's). */
int lmpo_destroy(lmpo_state *s);

const char *lmpo_last_error(void);

/* ---- inspection and kernel-level entry points (used by parity tests) ---- */

/* Site tensor k in the Pauli basis: writes dims[0..1] = (chi_l, chi_r) and, if
 * out is non-NULL, chi_l*4*chi_r complex values (interleaved, [l][a][r]).
 * Synchronises.  lmpo_set_site replaces it (shapes must fit the capacity, half
 * of it when force_hermitian_every > 0, and
 * match the neighbours' bonds); the caller states where the orthogonality
 * centre is (the library assumes sites < centre left-orthonormal and
 * > centre right-orthonormal). */
int lmpo_get_site(lmpo_state *s, int32_t k, int32_t dims[2], double *out);
int lmpo_set_site(lmpo_state *s, int32_t k, int32_t chi_l, int32_t chi_r, const double *data);
int lmpo_set_centre(lmpo_state *s, int32_t centre);
int lmpo_get_centre(lmpo_state *s, int32_t *centre);

/* Gate table entry exp(x L_b) in the Pauli basis, x = tau/2 (half = 1) or tau
 * (half = 0): 16x16 complex row-major over (a_i a_j) x (a_i' a_j'). */
int lmpo_get_gate(lmpo_state *s, int32_t bond, int32_t half, double *out);

/* One gate on bond k (k, k+1) with the chosen propagator, as inside a step:
 * centre move, contraction, truncated SVD, canonical update (ascending: centre
 * ends on k+1; descending: on k).  Asynchronous. */
int lmpo_apply_gate(lmpo_state *s, int32_t k, int32_t half, int32_t ascending);

/* A caller's two-site superoperator G on qubits i != j, applied like one gate
 * of a step (SWAP network when |i - j| > 1, truncation by the state's chi_max
 * and cutoff).  G: 16x16 complex (interleaved re/im, row-major) in the Pauli
 * basis P_{a_i} (x) P_{a_j}, index 4 a_i + a_j, acting on (qubit i, qubit j) in
 * that order.  Non-finite entries: LMPO_EINVAL; in the real-arithmetic form an
 * entry with an imaginary part above 1e-12 of the largest entry is
 * LMPO_EINVAL too (smaller ones are dropped).  Drains the stream before
 * copying G to the device, then enqueues the gate asynchronously. */
int lmpo_apply_superop(lmpo_state *s, int32_t i, int32_t j, const double *G);

/* The channel rho -> U rho U^+ of a two-qubit unitary U on qubits (i, j), as
 * lmpo_apply_superop.  U: 4x4 complex (interleaved, row-major) in the basis
 * |k_i k_j>, index 2 k_i + k_j, with |0> the s^z = +1 state.  Unitarity is
 * not checked. */
int lmpo_apply_unitary(lmpo_state *s, int32_t i, int32_t j, const double *U);

/* Restart from the graph state of Eq. (graph_state): every qubit in |+x>,
 * then CZ applied to each of the n_pairs pairs (pairs[2p], pairs[2p+1]) in
 * order, through the SWAP network when apart.  The bond dims grow as the CZ
 * gates require (truncated by chi_max / cutoff like any gate; cutoff 0 keeps
 * round-off singular values).  Resets the step count (time 0) and the
 * discarded weight.  Synchronises at entry; the gates run asynchronously. */
int lmpo_init_graph_state(lmpo_state *s, int32_t n_pairs, const int32_t *pairs);

/* rho -> (rho + rho^+)/2 now (Sec. 6, force_rho_hermitian_step).  In the
 * Hermitian Pauli basis rho^+ has the conjugate coefficients, so the sum is
 * the direct sum of the MPS and its complex conjugate (bond dims doubled,
 * factor 1/2 on site 0); it is made left-orthonormal by exact QR from the
 * left and compressed by the truncated two-site SVD of every bond from the
 * right (chi_max, cutoff; the discarded weight counts).  The centre ends on
 * site 0; the trace is not renormalised.  Requires a state created with
 * force_hermitian_every > 0 (LMPO_EUNSUPPORTED otherwise).  Asynchronous. */
int lmpo_hermitize(lmpo_state *s);

/* Singular values of the last two-site block, sorted descending (n_out
 * entries at most), and its kept rank; synchronises. */
int lmpo_last_spectrum(lmpo_state *s, int32_t n_out, double *sv, int32_t *n_sv, int32_t *kept);

/* Cap on the workgroups that serve one SVD or centre hop of this state (0:
 * automatic, one per Jacobi pair of the block, at most the co-resident grid).
 * Results do not depend on it; it exists for tuning and for tests of that. */
int lmpo_set_workgroups(lmpo_state *s, int32_t max_workgroups);

/* Stopping threshold of this state's block Jacobi SVDs: a column pair counts
 * as orthogonal when |g_pq| <= factor sqrt(C) eps sqrt(g_pp g_qq) (C columns,
 * eps the FP64 unit round-off); default 32, factor >= 1.  A larger factor ends
 * the sweeps earlier at the price of singular vectors accurate to about that
 * threshold: meant for the gradient's co-state (lmpo_grad_costate), whose
 * truncation is usually far coarser than the round-off. */
int lmpo_set_svd_tolerance(lmpo_state *s, double factor);

/* Truncated SVD of wide two-site blocks on a subspace (App. B, Sec. 6: only
 * the kept singular triplets, at most max_dim_rho of them, and the discarded
 * weight enter the step).  A gate block with at least min_cols columns is
 * decomposed by subspace iteration: p = min(chi_max, chi + grow) + margin
 * vectors (chi the bond's dimension before the gate, p rounded up to 16, at
 * most 3/4 of the columns and at most 384; a block whose min(chi_max, chi +
 * grow) + 16 exceeds 384 takes the full SVD), `iterations` multiplications by the block and
 * its adjoint with Cholesky-QR orthonormalisation, then the exact SVD of the
 * block restricted to the subspace (Rayleigh-Ritz, block Jacobi on a p x p
 * factor).  The kept triplets are accepted when each residual
 * ||theta^H u_j - s_j v_j|| is at most tol * s_1 and at least 16 vectors lie
 * beyond the cut; else the iteration continues once, for as many steps as
 * the residual's observed rate of decrease needs to reach the bound (40 in
 * all at most), and if that still fails the full SVD of the block is taken
 * instead.  The squared weight outside the subspace, ||theta||_F^2 -
 * sum_j s_j^2, counts as discarded.  Defaults: min_cols 512, margin 48, grow
 * 32, iterations 4, tol 1e-12 (the FP32-contraction form: iterations 2, tol
 * 1e-8, below the FP32 rounding of its block); min_cols <= 0 turns it off
 * (every block then takes the full SVD).  margin must lie in [16, 128],
 * iterations in [1, 64], tol in (0, 1). */
int lmpo_set_svd_subspace(lmpo_state *s, int32_t min_cols, int32_t margin, int32_t grow, int32_t iterations,
                          double tol);

/* Counters of the subspace SVD since creation: out = (blocks accepted, blocks
 * handed to the full SVD, subspace iterations of the accepted blocks);
 * synchronises. */
int lmpo_svd_subspace_stats(lmpo_state *s, int32_t out[3]);

/* Jacobi statistics: out = (sweeps of the last SVD, its column count,
 * total sweeps so far, total SVDs so far, hops included); synchronises. */
int lmpo_svd_stats(lmpo_state *s, int32_t out[4]);

/* Accumulated time of the persistent SVD phases seen by its first workgroup,
 * microseconds: [0] setup, [1] Jacobi pair work, [2] barrier wait, [5] norms +
 * select, [6] epilogue; inside the pair work [8] Gram, [9] eigen sweep, [10] X
 * update, [11] V update; [16] column order, [17] QR panels, [18] QR trailing
 * updates, [19] forming Q Y; subspace SVD: [20] set-up, [21] iterations,
 * [22] final Cholesky QR, [23] Rayleigh-Ritz outside its Jacobi phases,
 * [24] vectors and residual check, [25] hops by Cholesky QR, and inside
 * every Cholesky-QR pass [26] Gram matrix, [27] the sum of its parts and
 * the Cholesky factorisation (inside it [29] diagonal blocks with the next
 * panel's update beside them, [30] the next panel's last update step, [31]
 * rows below), [28] inverse factor and product.  Counts: [3] shader clock
 * cycles, [4] pair tasks, [7] launches, [12] pair tasks that rotated, [15]
 * Cholesky-QR passes.  out_us has 32 entries.  Synchronises. */
int lmpo_svd_profile(lmpo_state *s, double out_us[32]);

/* Profiling window for the persistent SVD kernel (one launch per truncated
 * SVD or centre hop).  Between begin and end, HIP events bracket every such
 * launch on the state's stream (at most max_launches; more is an error at
 * end) and each launch adds its declared flop count to a device counter:
 * 4 (14 R C^2 + 8 C^3) for the thin SVD of a gate's R x C block (R >= C;
 * Golub & Van Loan), 4 (4 R n^2 - 4 n^3 / 3) for a hop's thin QR with Q formed
 * (n = min(R, C)).  end synchronises and returns out = (launches, summed
 * kernel milliseconds, summed declared flops). */
int lmpo_profile_begin(lmpo_state *s, int32_t max_launches);
int lmpo_profile_end(lmpo_state *s, double out[3]);

/* ---- batched form: many independent chains in one launch per layer ----
 *
 * A batch groups existing states (each from lmpo_create, all on the same
 * stream, possibly of different N, models, chi_max, cutoff and precision) and
 * advances them together: every Trotter layer of every chain runs in one
 * cooperative launch in which each chain is served by its own group of
 * workgroups that walks the chain's gates (and centre hops) in the same order
 * and with the same arithmetic as lmpo_evolve_step, so each chain's result is
 * the one lmpo_evolve_step gives.  The co-resident grid is split between the
 * chains by a cost model of the Jacobi SVD (more workgroups to chains with
 * larger bond dimensions), and a chain's workgroups are placed on one XCD
 * where they fit.
 *
 * The chains stay owned by the caller and usable through the single-chain
 * calls (measure, trace, bond dims, ...) after lmpo_batch_sync; they must not
 * be destroyed before the batch.  The batch needs a second device arena of
 * lmpo_batch_arena_bytes() bytes (256-byte aligned, caller-owned).  At most
 * one workgroup per compute unit per chain is available: n_chains above the
 * co-resident grid gives LMPO_EUNSUPPORTED. */
typedef struct lmpo_batch lmpo_batch;

size_t lmpo_batch_arena_bytes(lmpo_state *const *chains, int32_t n_chains);
int lmpo_batch_create(lmpo_state *const *chains, int32_t n_chains, void *device_arena, size_t arena_bytes,
                      lmpo_batch **out);

/* Enqueue n_steps Trotter steps of every chain (asynchronous).  Each chain
 * continues from its own step count and centre, as lmpo_evolve_step would. */
int lmpo_batch_evolve_step(lmpo_batch *b, int32_t n_steps);

/* Wait for the batch's work; reports the first chain with a deferred error. */
int lmpo_batch_sync(lmpo_batch *b);

/* Online autotuner (off by default).  Results do not depend on how the grid
 * is split between chains, so with autotuning on, the batch times two steps
 * under each candidate cap on the workgroups per chain (1, 2, 4, 8, 16, none),
 * in palindromic order so that the growth of the steps' cost cancels, for
 * every (largest block size bucket, precision) it meets, with HIP events
 * (those steps synchronise), and then keeps the fastest.  The table is
 * process-wide per device, so later batches reuse it; a batch with tuning off
 * still uses entries that exist. */
int lmpo_batch_set_autotune(lmpo_batch *b, int32_t enable);

/* The tuned entries of the current device: log2 of the block column bucket,
 * precision bit mask (1 << LMPO_FP64 | 1 << LMPO_FP32_CONTRACT), chosen cap
 * (0 = none) and its mean step time in ms; at most max_entries written, the count
 * in *n_entries. */
int lmpo_autotune_table(int32_t max_entries, int32_t *log2_bucket, int32_t *precisions, int32_t *cap,
                        double *best_ms, int32_t *n_entries);

/* Workgroups per chain in the current plan (n_chains entries). */
int lmpo_batch_plan(lmpo_batch *b, int32_t *workgroups);

/* Profiling window over the per-layer launches, as lmpo_profile_begin/_end:
 * out = (launches, summed kernel milliseconds, summed declared SVD flops of
 * all chains). */
int lmpo_batch_profile_begin(lmpo_batch *b, int32_t max_launches);
int lmpo_batch_profile_end(lmpo_batch *b, double out[3]);

int lmpo_batch_destroy(lmpo_batch *b);

/* ---- Parameter gradients (adjoint form) ----------------------------------
 * Derivatives of a final-time expectation value F = Tr(O rho_T) / Tr(rho_T),
 * O a Pauli string (sigma^a_i of Eq. mu, the correlators of Eq. 2Qdef, or any
 * longer product), with respect to every model parameter, by the adjoint
 * (co-state) method.  Every bond generator L_b is linear in each parameter
 * theta, and the derivative of the gate exp(x L_b) is K exp(x L_b) with K =
 * (d/dtheta exp(x L_b)) exp(-x L_b), so the derivative of the Trotter product
 * is sum over gates g of s_g <mu_g, K_g rho_g>: rho_g the state after gate g,
 * mu_g the co-state after it (mu_T = (o - F 1)/Tr(rho_T), o and 1 the
 * covectors of O and of the trace, both products, carried back by the transposed
 * gates, SWAP gates included), s_g the inverse product of the traces divided
 * out at the ends of the steps from g's own step on, and <mu, K rho> the trace
 * of K with the two-site transition density of the two MPS.  The co-state is
 * an MPS truncated by the same rule as the state, with the state's chi_max and
 * cutoff unless the caller gives its own (a backward-evolved local observable
 * spreads faster than a weakly driven state, so its bonds can be the larger
 * cost).  Without truncation the result is the exact derivative of the
 * Trotter product; with it, an approximation to the truncation error of the
 * two passes (this is not a derivative of the truncated SVD).
 *
 * A workspace serves one state and a fixed number of steps.  It holds the
 * co-state (a state of the same model and controls, its gate table
 * transposed, in the real-arithmetic form: the co-state of a Hermitian
 * observable is real in the Pauli basis, as every propagator is), a snapshot of the state at the start of every step, the gate
 * outputs of one step (the step is replayed from its snapshot during the
 * backward pass) and the environments; lmpo_grad_arena_bytes gives its size
 * (device memory, 256-byte aligned, caller-owned, bounded by (n_steps + 1 +
 * gates per step) site blocks at capacity).  Not supported (LMPO_EUNSUPPORTED):
 * force_hermitian_every > 0, chi_max < 2. */
typedef struct lmpo_grad lmpo_grad;

/* Workspace flags.  LMPO_GRAD_SERIES: room for lmpo_grad_run_series, whose
 * outputs enter the co-state as sources (its bond capacities doubled, arena
 * about 4x, co-state chi_max <= 256).  LMPO_GRAD_KEEP_GATES: the forward run
 * keeps every step's gate snapshots (n_steps times the gate slots of one step:
 * tens of GB at chi 128 over 40 steps), so the backward pass replays nothing
 * (one forward run less; same results).  LMPO_GRAD_COMPLEX_COSTATE: the co-state
 * in the complex FP64 form instead of the real-arithmetic one (about four
 * times the co-state's SVD flops; the same gradient to round-off), which the
 * Renyi-2 and OSEE gradients of a state in a complex form need. */
enum { LMPO_GRAD_SERIES = 1, LMPO_GRAD_KEEP_GATES = 2, LMPO_GRAD_COMPLEX_COSTATE = 4 };

/* Device bytes of the workspace for n_steps >= 1 steps of s (0 on invalid
 * input).  costate_chi_max <= 0 and costate_cutoff < 0 take the state's
 * values; the co-state's chi_max must be 2..512.  flags: 0 or a combination
 * of LMPO_GRAD_SERIES and LMPO_GRAD_KEEP_GATES. */
size_t lmpo_grad_arena_bytes(lmpo_state *s, int32_t n_steps, int32_t costate_chi_max, double costate_cutoff,
                             int32_t flags);

/* Builds the workspace: creates the co-state in it, transposes its gate table,
 * and tabulates K for every bond, used time fraction and parameter on the host
 * (the Frechet derivative of the exponential as the upper-right block of the
 * exponential of [[x L, x dL], [0, x L]]).  Synchronises.  The state must
 * outlive the workspace. */
int lmpo_grad_create(lmpo_state *s, int32_t n_steps, int32_t costate_chi_max, double costate_cutoff, int32_t flags,
                     void *device_arena, size_t arena_bytes, lmpo_grad **out);

/* Advances the state by the workspace's n_steps exactly as lmpo_evolve_step
 * would (same results; the discarded weight and the statistics count the
 * forward run only) and returns F = <O>(T) as (re, im) and grad_out[p] =
 * d Re F / d theta_p for the 6 n_qubits + 2 n_bonds parameters in the order
 * hx[0..N-1], hy, hz, g0, g1, g2, J[0..n_bonds-1], Jz, followed by d Re F /
 * d tau (6 n_qubits + 2 n_bonds + 1 entries; the gate exp(f tau L) has
 * derivative f L exp(f tau L), and sum_theta theta dF/dtheta = tau dF/dtau
 * since F depends on the parameters only through tau theta).  paulis: the string O,
 * n_qubits characters of I, X, Y, Z (qubit 0 first), at least one not I.  F
 * of one or two factors equals lmpo_measure_1q / _2q on the final state bit
 * for bit.  Synchronises (once per co-state gate).  Arguments are checked
 * before the state moves; after an error met later (LMPO_EHIP, LMPO_ENUMERIC)
 * the state's tensors are unspecified. */
int lmpo_grad_run(lmpo_grad *g, const char *paulis, double F[2], double *grad_out);

/* As lmpo_grad_run for J = sum_k weights[k] Re <O>(t_k), t_k the state after
 * out_steps[k] steps (n_out >= 1 entries, strictly increasing within
 * 1..n_steps): the time series the paper's observables are.  F_out[k] =
 * <O>(t_k) as (re, im) ([n_out][2]), grad_out = dJ/dtheta.  When the backward
 * pass reaches the end of step out_steps[k], the co-state gains that output's
 * source w_k (o - F_k 1) / tr_k (times the traces divided out after it): the
 * direct sum of the co-state and the bond-2 source, compressed like the
 * Hermitian part (exact QR from the left, truncated identity gates from the
 * right, the co-state's chi_max and cutoff).  Before the last output the
 * co-state is zero and the steps after it are skipped; outputs of weight 0
 * add nothing (all weights 0: the values alone, a zero gradient).  Needs a workspace
 * created with LMPO_GRAD_SERIES (LMPO_EUNSUPPORTED otherwise).  A single output
 * at n_steps with weight 1 gives lmpo_grad_run's result bit for bit. */
int lmpo_grad_run_series(lmpo_grad *g, const char *paulis, int32_t n_out, const int32_t *out_steps,
                         const double *weights, double *F_out, double *grad_out);

/* As lmpo_grad_run for the connected correlator C = <a_i b_j> - <a_i><b_j>
 * (the paper's connected two-qubit function) with paulis = "ab" (two of X,
 * Y, Z) on qubits i != j: one backward pass whose co-state is the gradient
 * of C at T, mu_T = (o_ij - F_j o_i - F_i o_j + (2 F_i F_j - F_ij) 1) / tr
 * (F_x the three expectations at T).  F = C as (re, im).  That co-state
 * starts at bond 4: a co-state chi_max below 4 is LMPO_EUNSUPPORTED, checked
 * before the state moves. */
int lmpo_grad_run_connected(lmpo_grad *g, int32_t i, int32_t j, const char *paulis, double F[2], double *grad_out);

/* As lmpo_grad_run for the second Renyi entropy S_2 = -ln(tr rho^2 / (tr rho)^2)
 * at T (Eq. S_2, Sec. 2.4; the value lmpo_renyi2 reports): S2[0] = S_2,
 * grad_out = dS_2/dtheta.  In the Pauli basis tr rho^2 = <rho, rho> = P, so the
 * co-state is mu_T = (-2 / P)(rho_T - (P / tr) 1): the state's own tensors
 * plus one product term (bonds + 1), compressed as an output's source is
 * (the co-state's chi_max and cutoff), the factor applied to the gradient.
 * The copy is exact when state and co-state share a number format: needs the
 * state in the real-arithmetic form (LMPO_FP64_REAL) or a workspace created
 * with LMPO_GRAD_COMPLEX_COSTATE, and LMPO_GRAD_SERIES, and a co-state chi_max
 * at least the state's: LMPO_EUNSUPPORTED otherwise, checked before the state
 * moves. */
int lmpo_grad_run_renyi2(lmpo_grad *g, double S2[1], double *grad_out);

/* As lmpo_grad_run for the operator-space entanglement entropy across bond
 * (bond, bond + 1) at T (Eq. OSEE; the value lmpo_osee reports): value[0] =
 * S = -sum p ln p with p = s^2 / sum s^2 over the bond's singular values s,
 * grad_out = dS/dtheta.  With dS/ds_i = (2 s_i / W)(-ln p_i - S), W = sum s^2,
 * the co-state is the state with the bond's matrix U diag(s) V^T replaced by
 * U diag(dS/ds) V^T: the state's tensors copied at T, an identity gate on the
 * bond with cutoff 0 (every nonzero singular value kept), and its right factor
 * rescaled row by row (with complex tensors the row norms are still the s_i and
 * the co-state's coefficients stay real).  When every dS/ds_i is zero (a single
 * nonzero weight, or equal weights) the gradient is zero and no backward pass
 * runs.  Needs the state in the
 * real-arithmetic form (LMPO_FP64_REAL) or a workspace created with
 * LMPO_GRAD_COMPLEX_COSTATE, and a co-state chi_max at least the state's:
 * LMPO_EUNSUPPORTED otherwise, checked before the state moves; a bond outside
 * 0..n_qubits-2 is LMPO_EINVAL. */
int lmpo_grad_run_osee(lmpo_grad *g, int32_t bond, double value[1], double *grad_out);

/* Bond dims of the co-state (n_qubits - 1 entries): after a run, those of
 * mu at time 0, the end of the backward pass.  Synchronises. */
int lmpo_grad_costate_dims(lmpo_grad *g, int32_t *out);

/* The co-state as a state handle (owned by the workspace; NULL for a NULL
 * workspace), for inspection only: lmpo_bond_dims, lmpo_svd_stats and the
 * profiling window lmpo_profile_begin / lmpo_profile_end around a run.
 * Evolving or modifying it changes the next run's result. */
lmpo_state *lmpo_grad_costate(lmpo_grad *g);

int lmpo_grad_destroy(lmpo_grad *g);

/* ---- Measured peak ---------------------------------------------------------
 * FP64 matrix-core throughput of the device, the measured counterpart of the
 * datasheet peak the rooflines use: 2048 workgroups of four wavefronts, each
 * issuing 8 x 4096 independent v_mfma_f64_16x16x4f64 (2048 flops each) on
 * register operands; the second of two launches is timed with HIP events on
 * hip_stream.  device_buffer (caller-owned, at least
 * lmpo_probe_fp64_mfma_bytes() bytes) receives one value per thread.
 * Synchronises. */
size_t lmpo_probe_fp64_mfma_bytes(void);
int lmpo_probe_fp64_mfma(void *hip_stream, void *device_buffer, size_t buffer_bytes, double *tflops);

#ifdef __cplusplus
}
#endif
#endif /* LMPO_H */
