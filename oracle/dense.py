"""Brute-force references on the full 4^N vector |rho>> (oracle, small N).

* dense Trotter: the same gates and schedule as the MPS, no truncation;
* dense exact:   exp(t L) |rho0>> for the full Liouvillian L = sum_b L_b
  (sparse, scipy.sparse.linalg.expm_multiply), the brute-force comparison
  the paper uses for N up to ~10 (Sec. 3.2, App. B).
Site-major ordering: index (k_0 b_0)(k_1 b_1)...(k_{N-1} b_{N-1}).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import model as lm
from . import tebd


def product_vector(init, N):
    labels = tebd.init_labels(init, N)
    v = np.ones(1, dtype=np.complex128)
    for l in labels:
        v = np.kron(v, tebd.pauli_state_vector(l))
    return v


def apply_two_site(v, G, i, j, N):
    """Apply a 16x16 two-site superoperator on sites i < j of the 4^N vector."""
    t = v.reshape((4,) * N)
    g = G.reshape(4, 4, 4, 4)
    t = np.tensordot(g, t, axes=([2, 3], [i, j]))  # new axes (i, j) first
    t = np.moveaxis(t, [0, 1], [i, j])
    return t.reshape(-1)


def trotter_evolve(v, model, tau, steps, gates=None, first_step=0, observer=None,
                   force_trace=True, order=2):
    """The MPS schedule on the full vector; a bond (i, j) apart along the path
    acts on sites i and j directly (no SWAP network)."""
    N = model["N"]
    chain = tebd.is_chain(model)
    bonds = np.asarray(model["bonds"])
    if gates is None:
        gates = tebd.gate_tables(model, tau, order)
    for n in range(first_step, first_step + steps):
        if chain:
            for k, frac, _ in tebd.step_schedule(N, n, order):
                v = apply_two_site(v, gates[(k, frac)], k, k + 1, N)
        else:
            for b, frac, _ in tebd.sweep_schedule(model, order):
                v = apply_two_site(v, gates[(b, frac)], int(bonds[b, 0]), int(bonds[b, 1]), N)
        if force_trace:
            v = v / trace(v, N)
        if observer is not None:
            observer(n + 1, v)
    return v


def liouvillian(model):
    """Sparse 4^N x 4^N matrix of the full Liouvillian sum_b L_b."""
    N = model["N"]
    dim = 4 ** N
    L = sp.csr_matrix((dim, dim), dtype=np.complex128)
    for b, (i, j) in enumerate(model["bonds"]):
        Lb = lm.bond_generator(model, b)
        i, j = int(i), int(j)
        if j == i + 1:
            term = sp.kron(sp.kron(sp.identity(4 ** i), sp.csr_matrix(Lb)),
                           sp.identity(4 ** (N - j - 1)))
        else:  # non-adjacent bond: build column by column
            cols = []
            for c in range(dim):
                e = np.zeros(dim, dtype=np.complex128)
                e[c] = 1.0
                cols.append(sp.csr_matrix(apply_two_site(e, Lb, i, j, N)).T)
            term = sp.hstack(cols)
        L = L + sp.csr_matrix(term)
    return L.tocsr()


def exact_evolve(v0, model, times):
    """[exp(t L) v0 for t in times] (times equally spaced from 0)."""
    L = liouvillian(model)
    times = np.asarray(times, dtype=np.float64)
    out = spla.expm_multiply(L, v0, start=float(times[0]), stop=float(times[-1]),
                             num=len(times), endpoint=True)
    return np.asarray(out)


def contract(v, covectors):
    t = v.reshape((4,) * len(covectors))
    for c in covectors:
        t = np.tensordot(c, t, axes=(0, 0))
    return complex(t)


def trace(v, N):
    return contract(v, [tebd.E_ID] * N)


def expect(v, N, ops):
    cov = [tebd.covector(ops[k]) if k in ops else tebd.E_ID for k in range(N)]
    return contract(v, cov) / trace(v, N)


def zz_observables(v, N):
    z1 = np.array([expect(v, N, {i: lm.SZ}) for i in range(N)])
    z2 = np.array([expect(v, N, {i: lm.SZ, j: lm.SZ}) for i in range(N) for j in range(i + 1, N)])
    return z1, z2


def to_matrix(v, N):
    """rho as a 2^N x 2^N matrix (rows: kets, columns: bras)."""
    t = v.reshape((2, 2) * N)  # k0 b0 k1 b1 ...
    perm = [2 * s for s in range(N)] + [2 * s + 1 for s in range(N)]
    return t.transpose(perm).reshape(2 ** N, 2 ** N)


def mps_to_vector(tensors):
    v = np.ones((1, 1), dtype=np.complex128)
    for A in tensors:
        v = np.tensordot(v, A, axes=(1, 0)).reshape(-1, A.shape[2])
    return v.reshape(-1)


def renyi2(v, N):
    """S_2 = -ln tr(rho^2) from the dense matrix (Eq. S_2), unit-trace normalised."""
    rho = to_matrix(v, N)
    rho = rho / np.trace(rho)
    return float(-np.log(np.trace(rho @ rho).real))


def osee(v, N, bond):
    """OSEE of |rho>> across bond (bond, bond + 1) (Eq. OSEE): entropy of the
    normalised squared singular values of the coefficient vector reshaped as
    (sites 0..bond) x (sites bond+1..N-1)."""
    s = np.linalg.svd(v.reshape(4 ** (bond + 1), 4 ** (N - bond - 1)), compute_uv=False)
    p = s ** 2 / np.sum(s ** 2)
    p = p[p > 0]
    return float(-np.sum(p * np.log(p)))


def graph_state_vector(N, pairs):
    """|psi><psi| for the graph state of Eq. (graph_state), from its closed
    form psi(x) = 2^(-N/2) (-1)^(sum over pairs of x_j x_k), x_i in {0, 1}."""
    x = (np.arange(2 ** N)[:, None] >> (N - 1 - np.arange(N))[None, :]) & 1
    phase = np.zeros(2 ** N, dtype=np.int64)
    for a, b in pairs:
        phase += x[:, a] * x[:, b]
    psi = (1.0 - 2.0 * (phase % 2)) / np.sqrt(2.0 ** N)
    rho = np.outer(psi, psi.conj()).astype(np.complex128)
    # rows k_0..k_{N-1}, columns b_0..b_{N-1} -> site-major (k_0 b_0)(k_1 b_1)...
    t = rho.reshape((2,) * (2 * N))
    perm = [q for s in range(N) for q in (s, N + s)]
    return t.transpose(perm).reshape(-1)


def adjoint(v, N):
    """|rho^+>> from |rho>> (rho^+[k, b] = conj(rho[b, k]) on every site)."""
    t = np.conj(v).reshape((2, 2) * N)
    perm = [q for s in range(N) for q in (2 * s + 1, 2 * s)]
    return t.transpose(perm).reshape(-1)
