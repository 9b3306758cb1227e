"""Parameter gradients of a final-time expectation value by the adjoint
(co-state) method on the MPS (oracle, FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package header).

Also d/dtau of the same objectives: a gate exp(f tau L) has derivative
f L exp(f tau L), so its K is f L (no Frechet derivative needed); since F
depends on the parameters only through tau theta, sum_theta theta dF/dtheta =
tau dF/dtau exactly.

Objective: F = Tr(O rho_T) / Tr(rho_T) with O a Pauli string (sigma^a on one
qubit as in Eq. mu, a correlator as in Eq. 2Qdef, or a longer product), or the
connected correlator <a_i b_j> - <a_i><b_j>, after T Trotter steps from a
fixed initial state; or a weighted sum of a string's expectations at several
output steps (each output's gradient enters the co-state as a source when the
backward pass reaches its step, added to the co-state MPS by a direct sum
compressed like the Hermitian part: QR from the left, truncated identity gates
from the right); or the second Renyi entropy S_2 (Eq. S_2) or the
operator-space entanglement entropy across a bond (Eq. OSEE) at T, whose
co-states are built from rho_T itself (costate_renyi2, costate_osee: each
pinned against central differences of the dense entropy along a Hermitian
direction).  Every objective is unchanged when rho_T is scaled, which is
what lets the traces divided out enter only through s_g below.  Parameters: every
entry of hx, hy, hz, g0, g1, g2 (per qubit) and J, Jz (per bond) of the model
of Sec. 2.1.  Each bond generator L_b is linear in every one of them (the
Hamiltonian enters through a commutator, each rate multiplies its dissipator),
so dL_b/dtheta is the generator of the same bond with theta = 1 and all other
parameters 0, with the same sharing of the on-site terms among the bonds.

Derivative of the Trotter product (gates G_g = exp(x_g L_b(g)), the step's
division by the trace at its end): F does not change when rho_T is scaled, and
each gate's derivative is dG/dtheta = K G with K = (dG/dtheta) G^{-1}, so

    dF/dtheta = sum_g  s_g  < mu_g , K_g rho_g >

  rho_g  the state right after gate g (as computed: divided by the traces of
         the steps before),
  mu_g   the co-state right after gate g: mu_T = (o - F 1) / Tr(rho_T), with o
         and 1 the covectors of O and of the trace, carried backwards by
         mu <- G^T mu through every later gate (SWAP gates included); <., .>
         is the bilinear pairing sum_x mu_x rho_x of coefficient vectors, so
         the transpose (not the adjoint) is the backward map,
  s_g    1 / (product of the traces t_m divided out at the ends of steps m
         from the gate's own step to the last; 1 without trace forcing),
  K_g    the Frechet derivative of the exponential at x L in the direction
         x dL/dtheta (SciPy), times exp(-x L), on the gate's two sites.

< mu, K rho > only involves the two sites the gate acted on: it is
tr(K Gamma) with the transition density Gamma[(c d), (a b)] = the sum over
every other index of rho[..c d..] mu[..a b..].

On the MPS, rho_g is the forward TEBD state after gate g (every snapshot kept)
and mu_g the co-state MPS (bond dimension 2 at time T, brought to canonical
form by an exact QR sweep) after the truncated two-site gates G^T, applied
in reverse order with the state's chi_max and cutoff or the co-state's own.  Without truncation this
is exactly the derivative of the Trotter product (pinned against central
differences of the dense Trotter evolution).  With truncation it approximates
that derivative to the truncation error of both passes; it is not the
derivative of the truncated map itself (no differentiation of the truncated
SVD).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import model as lm
from . import tebd

SITE_KEYS = ("hx", "hy", "hz", "g0", "g1", "g2")
BOND_KEYS = ("J", "Jz")


def parameter_list(model):
    """[(key, index)] in the order hx[0..N-1], hy, hz, g0, g1, g2, J[0..nb-1], Jz."""
    N, nb = model["N"], len(model["bonds"])
    return [(k, s) for k in SITE_KEYS for s in range(N)] + [(k, b) for k in BOND_KEYS for b in range(nb)]


def unit_model(model, key, index):
    """The model with parameter (key, index) = 1 and every other parameter 0."""
    out = dict(model)
    for k in SITE_KEYS + BOND_KEYS:
        out[k] = np.zeros(len(model[k]))
    out[key][index] = 1.0
    return out


def generator_derivative(model, b, key, index):
    """dL_b / dtheta (16 x 16, site-major computational basis)."""
    return lm.bond_generator(unit_model(model, key, index), b)


def bond_parameters(model, b):
    """Parameters that bond b's generator depends on."""
    i, j = (int(x) for x in model["bonds"][b])
    return [(k, s) for s in (i, j) for k in SITE_KEYS] + [("J", b), ("Jz", b)]


def k_matrix(L, dL, x):
    """(d/dtheta exp(x L)) exp(-x L) for dL/dtheta = dL."""
    _, D = scipy.linalg.expm_frechet(x * L, x * dL)
    return D @ scipy.linalg.expm(-x * L)


def transition_density(mu, rho, k):
    """Gamma[(c d), (a b)] on sites (k, k + 1): rho's local indices (c, d)
    and mu's (a, b), every other index of the two MPS contracted pairwise."""
    N = len(mu)
    L = np.ones((1, 1), dtype=np.complex128)
    for s in range(k):
        L = np.einsum("pq,pam,qan->mn", L, mu[s], rho[s], optimize=True)
    R = np.ones((1, 1), dtype=np.complex128)
    for s in range(N - 1, k + 1, -1):
        R = np.einsum("map,naq,pq->mn", mu[s], rho[s], R, optimize=True)
    g = np.einsum("pq,pam,mbr,qcn,nds,rs->cdab", L, mu[k], mu[k + 1], rho[k], rho[k + 1], R, optimize=True)
    return g.reshape(16, 16)


def _record_one(model, tau, n, chi_max, cutoff, order, force_trace, mps, gates=None):
    """Step n of tebd.evolve on mps, recording every two-site gate: returns
    (mps, [(site k, bond or None for a SWAP, fraction of tau, ascending?, copy
    of all site tensors)], trace divided out at the step's end)."""
    N = model["N"]
    gates = gates if gates is not None else tebd.gate_tables(model, tau, order)
    P = lm.swap_gate()
    bonds = np.asarray(model["bonds"])
    ops = []

    def gate(k, G, asc, b, frac):
        mps.apply_gate(k, G, chi_max, cutoff, asc)
        ops.append((k, b, frac, asc, [a.copy() for a in mps.A]))

    if tebd.is_chain(model):
        for k, frac, asc in tebd.step_schedule(N, n, order):
            gate(k, gates[(k, frac)], asc, k, frac)
    else:
        for b, frac, fwd in tebd.sweep_schedule(model, order):
            i, j = int(bonds[b, 0]), int(bonds[b, 1])
            if j == i + 1:
                gate(i, gates[(b, frac)], fwd, b, frac)
                continue
            for k in range(j - 1, i, -1):
                gate(k, P, False, None, None)
            gate(i, gates[(b, frac)], True, b, frac)
            for k in range(i + 1, j):
                gate(k, P, True, None, None)
    return mps, ops, (mps.renormalize() if force_trace else 1.0)


def forward_record(model, tau, steps, chi_max, cutoff, init, order=2, force_trace=True):
    """The TEBD run of tebd.evolve, keeping after every two-site gate the
    record (site k, bond or None for a SWAP, fraction of tau, ascending?,
    copy of all site tensors), and the trace divided out at each step's end.
    Returns (final MPS, [records of step n], [trace of step n])."""
    mps = tebd.MPS.product(init, model["N"])
    gates = tebd.gate_tables(model, tau, order)
    records, traces = [], []
    for n in range(steps):
        _, ops, t = _record_one(model, tau, n, chi_max, cutoff, order, force_trace, mps, gates)
        records.append(ops)
        traces.append(t)
    return mps, records, traces


def costate(N, site, pauli, F, tr):
    """MPS of mu_T = (o - F 1) / tr for O = sigma^pauli on `site`."""
    return costate_string(N, {site: pauli}, F, tr)


def costate_string(N, ops, F, tr):
    """MPS of mu_T = (o - F 1) / tr for the Pauli string O = prod_s ops[s]
    ({site: 'X' | 'Y' | 'Z'})."""
    return costate_terms(N, [(1.0 / tr, ops), (-F / tr, {})])


def costate_terms(N, terms):
    """MPS of sum_k c_k prod_s o_{k,s} for terms [(c_k, {site: pauli})] (the
    trace covector on every site not named): bond dimension K (a row on the
    first site, block-diagonal inside, a column carrying the c_k on the last),
    then left-orthonormal by QR with the centre on the last site."""
    K = len(terms)
    cov = [[tebd.covector(lm.PAULI[ops[s]]) if s in ops else tebd.E_ID for s in range(N)] for _, ops in terms]
    A = []
    for s in range(N):
        nl, nr = (1 if s == 0 else K), (1 if s == N - 1 else K)
        t = np.zeros((nl, 4, nr), dtype=np.complex128)
        for k, (c, _) in enumerate(terms):
            t[0 if s == 0 else k, :, 0 if s == N - 1 else k] += (c if s == N - 1 else 1.0) * cov[k][s]
        A.append(t)
    mu = tebd.MPS(A, 0)
    mu.move_centre(N - 1)
    return mu


def add_compress(mu, src, chi_mu, cut_mu):
    """mu + src as an MPS: the direct sum of the two (bonds added, a row on the
    first site, block-diagonal inside, a column on the last), made
    left-orthonormal by QR from the left, then compressed from the right by the
    truncated two-site SVD of every bond (the identity gate, usual rule).  The
    centre ends on site 0."""
    N = mu.N
    A = []
    for k, (a, b) in enumerate(zip(mu.A, src.A)):
        if k == 0:
            t = np.concatenate([a, b], axis=2)
        elif k == N - 1:
            t = np.concatenate([a, b], axis=0)
        else:
            t = np.zeros((a.shape[0] + b.shape[0], 4, a.shape[2] + b.shape[2]), dtype=np.complex128)
            t[:a.shape[0], :, :a.shape[2]] = a
            t[a.shape[0]:, :, a.shape[2]:] = b
        A.append(t)
    out = tebd.MPS(A, 0)
    out.move_centre(N - 1)
    ident = np.eye(16, dtype=np.complex128)
    for k in range(N - 2, -1, -1):
        out.apply_gate(k, ident, chi_mu, cut_mu, False)
    return out


def backward(model, tau, records, traces, mu, chi_mu, cut_mu, order=2, sources=None):
    """The co-state pass: {key: complex array of dF/dtheta} for the co-state
    mu = mu_T (module header), which it advances back to time 0.  sources:
    {step n: source MPS} added when the pass reaches the end of step n (0-based),
    each weighted by the traces divided out after that step; mu may then be
    None (zero) until the first source."""
    gates = tebd.gate_tables(model, tau, order)
    P = lm.swap_gate()
    grads = {k: np.zeros(len(model[k]), dtype=np.complex128) for k in SITE_KEYS + BOND_KEYS}
    grads["tau"] = np.zeros(1, dtype=np.complex128)  # the gate exp(f tau L) has d/dtau = f L exp(f tau L)
    kcache = {}
    scale = 1.0
    for n in reversed(range(len(records))):
        if sources and n in sources:
            src = sources[n]
            src.A[-1] = src.A[-1] / scale  # the traces divided out after step n
            mu = src if mu is None else add_compress(mu, src, chi_mu, cut_mu)
        scale = scale / traces[n]
        if mu is None:
            continue
        for k, b, frac, asc, snap in reversed(records[n]):
            if b is None:
                mu.apply_gate(k, P.T, chi_mu, cut_mu, not asc)
                continue
            Gam = transition_density(mu.A, snap, k)
            for key, idx in bond_parameters(model, b):
                ck = (b, frac, key, idx)
                if ck not in kcache:
                    kcache[ck] = k_matrix(lm.bond_generator(model, b), generator_derivative(model, b, key, idx),
                                          frac * tau)
                grads[key][idx] += scale * np.sum(kcache[ck] * Gam.T)
            grads["tau"][0] += scale * frac * np.sum(lm.bond_generator(model, b) * Gam.T)
            mu.apply_gate(k, gates[(b, frac)].T, chi_mu, cut_mu, not asc)
    return grads


def gradient(model, tau, steps, chi_max, cutoff, init, site, pauli, order=2, force_trace=True,
             costate_chi_max=None, costate_cutoff=None, paulis=None):
    """(F, {key: complex array of dF/dtheta}, final MPS) for O = sigma^pauli
    on `site`, or for the Pauli string `paulis` (one of I, X, Y, Z per qubit)
    when given (module header).  The co-state is truncated with chi_max and
    cutoff unless costate_chi_max / costate_cutoff are given."""
    if paulis is not None:
        ops = {s: p for s, p in enumerate(paulis.upper()) if p != "I"}
    else:
        ops = {site: pauli.upper()}
    chi_mu = chi_max if costate_chi_max is None else costate_chi_max
    cut_mu = cutoff if costate_cutoff is None else costate_cutoff
    mps, records, traces = forward_record(model, tau, steps, chi_max, cutoff, init, order, force_trace)
    F = mps.expect({s: lm.PAULI[p] for s, p in ops.items()})
    mu = costate_string(model["N"], ops, F, mps.trace())
    return F, backward(model, tau, records, traces, mu, chi_mu, cut_mu, order), mps


def gradient_series(model, tau, steps, chi_max, cutoff, init, paulis, out_steps, weights, order=2,
                    force_trace=True, costate_chi_max=None, costate_cutoff=None):
    """(F_k array, {key: dJ/dtheta}, final MPS) for J = sum_k w_k F_k, F_k the
    Pauli string's expectation after out_steps[k] steps (1 <= out_steps[k] <=
    steps, increasing).  The gradient of F_k is carried back from the end of
    its step: the co-state gains the source w_k (o - F_k 1) / tr_k there."""
    ops = {s: p for s, p in enumerate(paulis.upper()) if p != "I"}
    chi_mu = chi_max if costate_chi_max is None else costate_chi_max
    cut_mu = cutoff if costate_cutoff is None else costate_cutoff
    N = model["N"]
    Fk, trk = {}, {}
    want = set(int(s) for s in out_steps)

    def observe(n_done, mps):
        if n_done in want:
            Fk[n_done] = mps.expect({s: lm.PAULI[p] for s, p in ops.items()})
            trk[n_done] = mps.trace()

    mps = tebd.MPS.product(init, N)
    gates = tebd.gate_tables(model, tau, order)
    records, traces = [], []
    # the recording forward pass, one step at a time so that the outputs can be read
    for n in range(steps):
        _, r1, t1 = _record_one(model, tau, n, chi_max, cutoff, order, force_trace, mps, gates)
        records.append(r1)
        traces.append(t1)
        observe(n + 1, mps)
    sources = {s - 1: costate_string(N, ops, Fk[s], trk[s]) for s in want}
    for s, w in zip(out_steps, weights):
        sources[int(s) - 1].A[-1] = sources[int(s) - 1].A[-1] * w
    grads = backward(model, tau, records, traces, None, chi_mu, cut_mu, order, sources)
    return np.array([Fk[int(s)] for s in out_steps]), grads, mps


def costate_renyi2(mps, chi_mu, cut_mu):
    """The gradient of S_2 = -ln(tr rho^2 / (tr rho)^2) (Eq. S_2) at the MPS rho as
    a covector: tr rho^2 = sum rho[k, b] rho[b, k], so the covector of its
    derivative is 2 rho with every site's (ket, bra) pair exchanged, and
    mu = -2 rho^swap / tr rho^2 + 2 . 1 / tr rho, an MPS sum (rho's bonds + 1)
    compressed like any source."""
    N = mps.N
    t2, tr = mps.tr_rho2(), mps.trace()
    swap = np.array([0, 2, 1, 3])
    rho_sw = tebd.MPS([a[:, swap, :].copy() for a in mps.A], 0)
    rho_sw.A[-1] = rho_sw.A[-1] * (-2.0 / t2)
    return add_compress(rho_sw, costate_terms(N, [(2.0 / tr, {})]), chi_mu, cut_mu)


def gradient_renyi2(model, tau, steps, chi_max, cutoff, init, order=2, force_trace=True, costate_chi_max=None,
                    costate_cutoff=None):
    """(S_2, {key: dS_2/dtheta}, final MPS) for S_2 at T (Eq. S_2): the co-state
    pass from costate_renyi2 of the final state."""
    chi_mu = chi_max if costate_chi_max is None else costate_chi_max
    cut_mu = cutoff if costate_cutoff is None else costate_cutoff
    mps, records, traces = forward_record(model, tau, steps, chi_max, cutoff, init, order, force_trace)
    S2 = -np.log(mps.tr_rho2() / mps.trace() ** 2)
    mu = costate_renyi2(mps, chi_mu, cut_mu)
    return S2, backward(model, tau, records, traces, mu, chi_mu, cut_mu, order), mps


def costate_osee(mps, bond):
    """(OSEE, mu): the operator-space entanglement entropy across (bond, bond + 1)
    (Eq. OSEE) at the MPS rho and its gradient as a covector.  With the centre
    on site `bond`, the site's matrix is M = U diag(s) V^dagger, p = s^2 / W with
    W = sum s^2, S = -sum p ln p, and dS/ds_i = (2 s_i / W)(-ln p_i - S).  Along
    a Hermitian direction ds_i = Re <u_i v_i^dagger, dM> (Frobenius): for
    Hermitian rho this is the bilinear pairing with the complex conjugate, so mu
    is the conjugate of the MPS with M replaced by U diag(dS/ds) V^dagger.
    Nothing is truncated."""
    c = tebd.MPS([a.copy() for a in mps.A], mps.centre)
    c.move_centre(bond)
    l, _, r = c.A[bond].shape
    U, s, Vh = np.linalg.svd(c.A[bond].reshape(l * 4, r), full_matrices=False)
    W = np.sum(s ** 2)
    p = s ** 2 / W
    nz = p > 0
    S = float(-np.sum(p[nz] * np.log(p[nz])))
    g = np.zeros_like(s)
    g[nz] = 2.0 * s[nz] / W * (-np.log(p[nz]) - S)
    c.A[bond] = ((U * g) @ Vh).reshape(l, 4, r)
    return S, tebd.MPS([np.conj(a) for a in c.A], bond)


def gradient_osee(model, tau, steps, chi_max, cutoff, init, bond, order=2, force_trace=True, costate_chi_max=None,
                  costate_cutoff=None):
    """(OSEE, {key: dOSEE/dtheta}, final MPS) across (bond, bond + 1) at T: the
    co-state pass from costate_osee of the final state."""
    chi_mu = chi_max if costate_chi_max is None else costate_chi_max
    cut_mu = cutoff if costate_cutoff is None else costate_cutoff
    mps, records, traces = forward_record(model, tau, steps, chi_max, cutoff, init, order, force_trace)
    S, mu = costate_osee(mps, bond)
    return S, backward(model, tau, records, traces, mu, chi_mu, cut_mu, order), mps


def gradient_connected(model, tau, steps, chi_max, cutoff, init, i, j, paulis="ZZ", order=2, force_trace=True,
                       costate_chi_max=None, costate_cutoff=None):
    """(C, {key: dC/dtheta}, final MPS) for the connected correlator
    C = <a_i b_j> - <a_i><b_j>: its gradient at T is
    (o_ij - F_j o_i - F_i o_j + (2 F_i F_j - F_ij) 1) / tr, the co-state."""
    a, b = paulis.upper()
    chi_mu = chi_max if costate_chi_max is None else costate_chi_max
    cut_mu = cutoff if costate_cutoff is None else costate_cutoff
    mps, records, traces = forward_record(model, tau, steps, chi_max, cutoff, init, order, force_trace)
    Fij = mps.expect({i: lm.PAULI[a], j: lm.PAULI[b]})
    Fi, Fj = mps.expect({i: lm.PAULI[a]}), mps.expect({j: lm.PAULI[b]})
    tr = mps.trace()
    mu = costate_terms(model["N"], [(1.0 / tr, {i: a, j: b}), (-Fj / tr, {i: a}), (-Fi / tr, {j: b}),
                                    ((2.0 * Fi * Fj - Fij) / tr, {})])
    return Fij - Fi * Fj, backward(model, tau, records, traces, mu, chi_mu, cut_mu, order), mps


def flatten(model, grads):
    """Gradient dict -> array in parameter_list order."""
    return np.array([grads[k][i] for k, i in parameter_list(model)])
