"""MPS-TEBD of the vectorised density matrix |rho>> (oracle, FP64, CPU).

State (Eq. mpo_def, App. A): rho is stored as an MPS with local dimension 4,
site tensors A[k] of shape (chi_left, 4, chi_right); the local index is the
computational (ket, bra) pair 2*ket + bra of the site.

One Trotter step of size tau, second order (the default):
    layers  A(tau/2), B(tau), A(tau/2)
    A = bonds (k, k+1) with k even, B = k odd (chain)
Fourth order (the paper's trotter_order = 4, Sec. 6; the composition is not
printed there, the symmetric triple product of second-order steps is used):
    S4(tau) = S2(w1 tau) S2(w0 tau) S2(w1 tau),
    w1 = 1 / (2 - 2^(1/3)), w0 = 1 - 2 w1,
with the two adjacent A half-layers merged (A layers commute), i.e. seven
layers A(w1/2) B(w1) A((w1+w0)/2) B(w0) A((w0+w1)/2) B(w1) A(w1/2) (times tau).
Third order (trotter_order = 3, chain only): the non-symmetric product of the
two layer operators A(7/24) B(2/3) A(3/4) B(-2/3) A(-1/24) B(1) (R. D. Ruth,
IEEE Trans. Nucl. Sci. 30 (1983) 2669); negative fractions run the dissipators
backwards for that sub-step.
Global layer l = L*step + j (L layers per step); gates of layer l run in
ascending k when l is even, descending when l is odd.
Per gate (bond k): bring the orthogonality centre onto (k, k+1); form the
two-site block theta = G (A_k A_{k+1}) as a (4 chi_l) x (4 chi_r) matrix;
full SVD (LAPACK); keep k' = min(chi_max, k_c) singular triplets, where k_c is
the smallest k' >= 1 whose discarded squared weight sum_{j > k'} s_j^2 is at
most cutoff * sum_j s_j^2 (App. B: the more severe of cut_off_rho and
max_dim_rho), except that a multiplet of (near-)equal singular values is never
split by the cut (see truncation_rank).  An ascending gate leaves A_k = U, A_{k+1} = S V^+ (centre moves
right), a descending one A_k = U S, A_{k+1} = V^+.  Singular values are not
rescaled.  After each step, when trace forcing is on, rho -> rho / tr(rho)
with the complex trace (App. B, b_force_rho_trace).

Other geometries (Sec. 2.3: the MPS follows a path through the qubits, so a
coupled pair may sit several sites apart along it, e.g. the zigzag ladder of
the plaquette appendix).  When the bond list is not the open chain in order,
a step is the symmetric sweep over the bond list
    S2(tau) = F(tau/2) R(tau/2),
F applying exp(tau/2 L_b) for b = 0, 1, ..., R the same factors in reverse
order; fourth order composes S2(w1 tau) S2(w0 tau) S2(w1 tau) without merging.
A bond (i, j) with j > i + 1 is applied by carrying site j down to i + 1 with
SWAP gates on (j-1, j), ..., (i+1, i+2) (each a two-site gate with the same
truncation rule), applying G on (i, i+1) and carrying it back up.
"""
from __future__ import annotations

import numpy as np

from . import model as lm

# local covectors: Tr(O rho_site) = sum_{k,b} O[b, k] rho[k, b]
def covector(O):
    return np.asarray(O).T.reshape(4)


E_ID = covector(lm.I2)


def pauli_state_vector(label):
    """vec of |psi><psi| for a Pauli eigenstate '+z', '-x', ... (Sec. 2.2)."""
    if len(label) != 2 or label[0] not in "+-" or label[1] not in "xyzXYZ":
        raise ValueError(f"bad Pauli state label {label!r}")
    sign = 1.0 if label[0] == "+" else -1.0
    op = lm.PAULI[label[1].upper()]
    rho = 0.5 * (lm.I2 + sign * op)
    return rho.reshape(4).astype(np.complex128)


def init_labels(init, N):
    if isinstance(init, str):
        return [init] * N
    init = list(init)
    if len(init) != N:
        raise ValueError("init must be one label or N labels")
    return init


def chain_layers(N):
    A = list(range(0, N - 1, 2))
    B = list(range(1, N - 1, 2))
    return A, B


def trotter_layers(order=2):
    """[(bond parity, fraction of tau)] of one step (see the module header)."""
    if order == 2:
        return [(0, 0.5), (1, 1.0), (0, 0.5)]
    if order == 3:
        return [(0, 7.0 / 24.0), (1, 2.0 / 3.0), (0, 0.75), (1, -2.0 / 3.0), (0, -1.0 / 24.0), (1, 1.0)]
    if order == 4:
        w1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
        w0 = 1.0 - 2.0 * w1
        return [(0, 0.5 * w1), (1, w1), (0, 0.5 * (w1 + w0)), (1, w0), (0, 0.5 * (w1 + w0)), (1, w1),
                (0, 0.5 * w1)]
    raise ValueError("trotter order must be 2, 3 or 4")


def step_schedule(N, step, order=2):
    """[(bond k, fraction of tau, ascending?)] for one chain step."""
    layers = chain_layers(N)
    lay = trotter_layers(order)
    out = []
    for j, (parity, frac) in enumerate(lay):
        asc = (len(lay) * step + j) % 2 == 0
        bonds = layers[parity]
        for k in (bonds if asc else bonds[::-1]):
            out.append((k, frac, asc))
    return out


def is_chain(model):
    """True when the bond list is the open chain (k, k+1), k = 0..N-2, in order."""
    bonds = np.asarray(model["bonds"])
    N = model["N"]
    return (len(bonds) == N - 1 and bool(np.all(bonds[:, 0] == np.arange(N - 1)))
            and bool(np.all(bonds[:, 1] == np.arange(1, N))))


def sweep_fractions(order=2):
    """Fractions x of tau of the symmetric sweeps F(x) R(x) of one step on a
    general bond list (see the module header)."""
    if order == 2:
        return [0.5]
    if order == 4:
        w1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
        w0 = 1.0 - 2.0 * w1
        return [0.5 * w1, 0.5 * w0, 0.5 * w1]
    raise ValueError("on a general bond list the trotter order must be 2 or 4")


def sweep_schedule(model, order=2):
    """[(bond b, fraction of tau, forward?)] of one step on a general bond list."""
    nb = len(model["bonds"])
    out = []
    for x in sweep_fractions(order):
        out += [(b, x, True) for b in range(nb)]
        out += [(b, x, False) for b in reversed(range(nb))]
    return out


TIE = 1e-4  # neighbouring singular values closer than TIE times the larger form one multiplet


def truncation_rank(s, chi_max, cutoff):
    """k' = min(chi_max, k_c); s sorted descending (App. B), adjusted so that
    the cut does not split a multiplet.

    App. B and Sec. 6 bound the discarded weight (cut_off_rho) and the bond
    dimension (max_dim_rho) but do not say which singular vectors of a
    degenerate multiplet straddling the cut are kept; any basis of the
    multiplet is a valid SVD, so splitting it leaves the truncated state
    undetermined (two backward-stable SVDs then disagree by about the
    multiplet's singular value).  Reading: neighbours with s_q - s_{q+1} <=
    TIE * s_q tie (a split of a pair that close moves the kept subspace by
    about eps s_1 / (s_q - s_{q+1}) under round-off, i.e. the truncated state
    by eps s_1 s_q / (s_q - s_{q+1})); when the cutoff set the cut, it moves
    past the multiplet
    while chi_max allows (discarding less than the cutoff permits), otherwise
    it moves in front of the multiplet (keeping fewer than chi_max).  Exact
    zeros never join a multiplet and are always discarded; k' >= 1.

    Returns (k', discarded squared weight, total squared weight)."""
    s = np.asarray(s, dtype=np.float64)
    w = s ** 2
    W = float(np.sum(w))
    r = len(s)
    # tail[k] = sum_{j >= k} w_j  (weight discarded when k values are kept)
    tail = np.zeros(r + 1)
    tail[:r] = np.cumsum(w[::-1])[::-1]
    kc = r
    for k in range(1, r + 1):
        if tail[k] <= cutoff * W:
            kc = k
            break
    nz = int(np.count_nonzero(s > 0))
    k = max(1, min(int(chi_max), kc, nz))

    def tie(q):  # the q-th and (q+1)-th values (1-based) tie; both nonzero
        return q < nz and s[q - 1] - s[q] <= TIE * s[q - 1]

    if k == kc:
        while k < min(int(chi_max), nz) and tie(k):
            k += 1
    while k > 1 and tie(k):
        k -= 1
    return k, float(tail[k]), W


class MPS:
    def __init__(self, tensors, centre=0):
        self.A = [np.array(t, dtype=np.complex128) for t in tensors]
        self.centre = centre
        self.discarded = 0.0  # cumulative relative discarded weight
        self.last_spectra = {}

    @property
    def N(self):
        return len(self.A)

    @classmethod
    def product(cls, init, N):
        labels = init_labels(init, N)
        return cls([pauli_state_vector(l).reshape(1, 4, 1) for l in labels], 0)

    def bond_dims(self):
        return [self.A[k].shape[2] for k in range(self.N - 1)]

    # -- orthogonality centre (exact QR moves; the state is unchanged) --
    def _shift_right(self, k):
        a = self.A[k]
        cl, _, cr = a.shape
        q, r = np.linalg.qr(a.reshape(cl * 4, cr))
        self.A[k] = q.reshape(cl, 4, q.shape[1])
        self.A[k + 1] = np.tensordot(r, self.A[k + 1], axes=(1, 0))

    def _shift_left(self, k):
        a = self.A[k]
        cl, _, cr = a.shape
        q, r = np.linalg.qr(a.reshape(cl, 4 * cr).T)  # a = r^T q^T
        self.A[k] = q.T.reshape(q.shape[1], 4, cr)
        self.A[k - 1] = np.tensordot(self.A[k - 1], r.T, axes=(2, 0))

    def move_centre(self, to):
        while self.centre < to:
            self._shift_right(self.centre)
            self.centre += 1
        while self.centre > to:
            self._shift_left(self.centre)
            self.centre -= 1

    # -- two-site gate --
    def two_site_block(self, k, G):
        """theta[(l,s'),(t',r)] = sum_{s,t} G[(s't'),(st)] sum_m A_k[l,s,m] A_{k+1}[m,t,r]."""
        M = np.einsum("lsm,mtr->lstr", self.A[k], self.A[k + 1])
        th = np.einsum("abst,lstr->labr", G.reshape(4, 4, 4, 4), M)
        cl, cr = self.A[k].shape[0], self.A[k + 1].shape[2]
        return th.reshape(cl * 4, 4 * cr)

    def apply_gate(self, k, G, chi_max, cutoff, ascending=True):
        if self.centre <= k:
            self.move_centre(k)
        else:
            self.move_centre(k + 1)
        cl, cr = self.A[k].shape[0], self.A[k + 1].shape[2]
        th = self.two_site_block(k, G)
        u, s, vh = np.linalg.svd(th, full_matrices=False)
        kk, disc, W = truncation_rank(s, chi_max, cutoff)
        self.last_spectra[k] = s.copy()
        if W > 0:
            self.discarded += disc / W
        u, s_k, vh = u[:, :kk], s[:kk], vh[:kk, :]
        if ascending:
            self.A[k] = u.reshape(cl, 4, kk)
            self.A[k + 1] = (s_k[:, None] * vh).reshape(kk, 4, cr)
            self.centre = k + 1
        else:
            self.A[k] = (u * s_k[None, :]).reshape(cl, 4, kk)
            self.A[k + 1] = vh.reshape(kk, 4, cr)
            self.centre = k
        return kk, s

    def apply_pair_gate(self, i, j, G, chi_max, cutoff, forward=True):
        """G (16 x 16, acting on (site i, site j)) on a pair i < j.  Adjacent:
        one gate, the centre ends right of the pair on forward sweeps and left
        of it otherwise.  Apart: SWAPs carry site j to i + 1 (centre moving
        left), G on (i, i + 1), SWAPs carry it back (centre moving right)."""
        if j == i + 1:
            self.apply_gate(i, G, chi_max, cutoff, forward)
            return
        P = lm.swap_gate()
        for k in range(j - 1, i, -1):
            self.apply_gate(k, P, chi_max, cutoff, False)
        self.apply_gate(i, G, chi_max, cutoff, True)
        for k in range(i + 1, j):
            self.apply_gate(k, P, chi_max, cutoff, True)

    # -- Hermitian part (Sec. 6, force_rho_hermitian_step) --
    def hermitize(self, chi_max, cutoff):
        """rho -> (rho + rho^+)/2.  rho^+ has site tensors conj(A_k) with the
        site's ket and bra exchanged; the sum is the MPS of the direct sums of
        the two (bonds doubled, 1/2 on the first site), made left-orthonormal
        by QR from the left, then compressed from the right by the truncated
        two-site SVD of every bond (the identity gate, usual rule).  The
        centre ends on site 0."""
        N = self.N
        swap = np.array([0, 2, 1, 3])  # local (ket, bra) -> (bra, ket)
        B = []
        for k, A in enumerate(self.A):
            D = np.conj(A[:, swap, :])
            cl, _, cr = A.shape
            if N == 1:
                T = A + D
            elif k == 0:
                T = np.concatenate([A, D], axis=2)
            elif k == N - 1:
                T = np.concatenate([A, D], axis=0)
            else:
                T = np.zeros((2 * cl, 4, 2 * cr), dtype=np.complex128)
                T[:cl, :, :cr] = A
                T[cl:, :, cr:] = D
            B.append(0.5 * T if k == 0 else T)
        self.A = B
        self.centre = 0
        self.move_centre(N - 1)
        ident = np.eye(16, dtype=np.complex128)
        for k in range(N - 2, -1, -1):
            self.apply_gate(k, ident, chi_max, cutoff, False)

    # -- contractions with product covectors --
    def contract(self, covectors):
        """sum over all indices of prod_k covectors[k] . A_k (a scalar)."""
        v = np.ones(1, dtype=np.complex128)
        for k, c in enumerate(covectors):
            v = v @ np.tensordot(self.A[k], c, axes=(1, 0))
        return complex(v[0])

    def trace(self):
        return self.contract([E_ID] * self.N)

    def renormalize(self):
        tr = self.trace()
        self.A[self.centre] = self.A[self.centre] / tr
        return tr

    def expect(self, ops):
        """<prod_i O_i> = Tr(rho prod_i O_i) / Tr(rho); ops = {site: 2x2}."""
        cov = [covector(ops[k]) if k in ops else E_ID for k in range(self.N)]
        return self.contract(cov) / self.trace()

    # -- global characteristics (Sec. 2.4) --
    def tr_rho2(self):
        """tr(rho^2) = sum rho[k, b] rho[b, k]: each site's (ket, bra) index
        of one copy meets the swapped index of the other."""
        swap = np.array([0, 2, 1, 3])  # 2*ket + bra -> 2*bra + ket
        env = np.ones((1, 1), dtype=np.complex128)
        for A in self.A:
            # env'[r, r'] = sum_{l, l', s} env[l, l'] A[l, s, r] A[l', swap(s), r']
            t = np.tensordot(env, A, axes=(0, 0))              # (l', s, r)
            env = np.tensordot(t, A[:, swap, :], axes=((0, 1), (0, 1)))  # (r, r')
        return complex(env[0, 0])

    def renyi2(self):
        """S_2 = -ln tr(rho^2) (Eq. S_2), for rho normalised to unit trace."""
        return float(-np.log((self.tr_rho2() / self.trace() ** 2).real))

    def osee(self, bond):
        """OSEE of |rho>> across bond (bond, bond + 1) (Eq. OSEE): von Neumann
        entropy of the normalised Schmidt weights s^2 / sum s^2, obtained from
        the SVD of the orthogonality centre placed on site `bond`."""
        self.move_centre(bond)
        A = self.A[bond]
        s = np.linalg.svd(A.reshape(A.shape[0] * 4, A.shape[2]), compute_uv=False)
        p = s ** 2 / np.sum(s ** 2)
        p = p[p > 0]
        return float(-np.sum(p * np.log(p)))


def gate_tables(model, tau, order=2):
    """{(bond, fraction): G} for every fraction of tau the scheme uses."""
    out = {}
    if is_chain(model):
        fracs = sorted({f for _, f in trotter_layers(order)})
    else:
        fracs = sorted(set(sweep_fractions(order)))
    for b in range(len(model["bonds"])):
        for frac in fracs:
            out[(b, frac)] = lm.bond_gate(model, b, frac * tau)
    return out


def evolve(mps, model, tau, steps, chi_max, cutoff, force_trace=True, gates=None,
           observer=None, first_step=0, order=2, hermitian_every=0):
    """Run `steps` Trotter steps; observer(step_done, mps) after each step.
    The open chain in order takes the layered schedule, any other bond list
    the symmetric bond-list sweep (module header).  With hermitian_every = k
    >= 1, rho -> (rho + rho^+)/2 ends every k-th step (global count), before
    the trace is forced."""
    chain = is_chain(model)
    if gates is None:
        gates = gate_tables(model, tau, order)
    bonds = np.asarray(model["bonds"])
    for n in range(first_step, first_step + steps):
        if chain:
            for k, frac, asc in step_schedule(mps.N, n, order):
                mps.apply_gate(k, gates[(k, frac)], chi_max, cutoff, asc)
        else:
            for b, frac, fwd in sweep_schedule(model, order):
                i, j = int(bonds[b, 0]), int(bonds[b, 1])
                mps.apply_pair_gate(i, j, gates[(b, frac)], chi_max, cutoff, fwd)
        if hermitian_every and (n + 1) % hermitian_every == 0:
            mps.hermitize(chi_max, cutoff)
        if force_trace:
            mps.renormalize()
        if observer is not None:
            observer(n + 1, mps)
    return mps


def zz_observables(mps):
    """<sz_i> for all i and <sz_i sz_j> for i < j (real parts, complex kept)."""
    N = mps.N
    z1 = np.array([mps.expect({i: lm.SZ}) for i in range(N)])
    z2 = np.array([mps.expect({i: lm.SZ, j: lm.SZ}) for i in range(N) for j in range(i + 1, N)])
    return z1, z2


def connected(mps, i, j, a="Z", b="Z"):
    """<s^a_i s^b_j> - <s^a_i><s^b_j> (the connected correlator)."""
    Oa, Ob = lm.PAULI[a], lm.PAULI[b]
    return mps.expect({i: Oa, j: Ob}) - mps.expect({i: Oa}) * mps.expect({j: Ob})


# -- basis conversion to the normalised Pauli basis P_a = sigma^a / sqrt(2),
#    a in (1, x, y, z) (Eq. mpo_def with orthonormal basis operators) --
def pauli_basis_matrix():
    """T[a, 2k+b] with c_a = Tr(P_a rho) = sum_{k,b} T[a, 2k+b] rho[k, b]."""
    T = np.zeros((4, 4), dtype=np.complex128)
    for a, key in enumerate("IXYZ"):
        T[a] = covector(lm.PAULI[key] / np.sqrt(2.0))
    return T


def to_pauli(tensors):
    T = pauli_basis_matrix()
    return [np.einsum("as,lsr->lar", T, A) for A in tensors]


def from_pauli(tensors):
    Ti = np.linalg.inv(pauli_basis_matrix())
    return [np.einsum("as,lsr->lar", Ti, A) for A in tensors]


def gate_to_pauli(G):
    T = pauli_basis_matrix()
    TT = np.kron(T, T)
    return TT @ G @ np.linalg.inv(TT)


# -- graph-state initial condition (Eq. graph_state) --
def cz_channel():
    """Superoperator of rho -> CZ rho CZ on two sites (site-major order)."""
    return lm.unitary_channel(np.diag([1.0, 1.0, 1.0, -1.0]).astype(np.complex128))


def graph_state(N, pairs, chi_max, cutoff):
    """|psi0><psi0| with psi0 = prod_{(j,k) in V} CZ[j,k] prod_i |+x_i>: the
    product of +x states, then the CZ channel on every listed pair in order
    (a pair apart along the path goes through the SWAP network)."""
    mps = MPS.product("+x", N)
    G = cz_channel()
    for a, b in pairs:
        i, j = (int(a), int(b)) if a < b else (int(b), int(a))
        if not (0 <= i < j < N):
            raise ValueError("graph pairs need two distinct sites in range")
        mps.apply_pair_gate(i, j, G, chi_max, cutoff, True)
    return mps
