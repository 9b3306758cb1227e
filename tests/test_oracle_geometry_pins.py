"""Pins of the oracle's general-geometry step (bonds apart along the MPS path,
Sec. 2.3), its unitary-channel gates and the graph-state initial condition
(Eq. graph_state), against brute force and closed forms."""
import numpy as np
import pytest

import workloads
from oracle import dense
from oracle import model as lm
from oracle import tebd


def random_unitary(n, seed):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


def random_state_mps(N, seed, chi=4):
    """A generic (non-Hermitian, non-product) MPS with small bonds."""
    rng = np.random.default_rng(seed)
    dims = [1] + [min(chi, 4 ** (k + 1), 4 ** (N - k - 1)) for k in range(N - 1)] + [1]
    A = [rng.standard_normal((dims[k], 4, dims[k + 1])) + 1j * rng.standard_normal((dims[k], 4, dims[k + 1]))
         for k in range(N)]
    mps = tebd.MPS(A, centre=0)
    mps.move_centre(N - 1)  # canonical form, as every gate assumes
    return mps


@pytest.mark.parametrize("i,j", [(0, 2), (1, 4), (0, 4), (2, 3)])
def test_swap_network_equals_direct_long_range_gate(i, j):
    """The SWAP route of a pair gate equals the gate applied to sites i, j of the
    full vector directly (no truncation), whatever the gate."""
    N = 5
    rng = np.random.default_rng(i * 10 + j)
    G = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    mps = random_state_mps(N, 3)
    v0 = dense.mps_to_vector(mps.A)
    mps.apply_pair_gate(i, j, G, 4 ** 3, 0.0, True)
    ref = dense.apply_two_site(v0, G, i, j, N)
    assert np.abs(dense.mps_to_vector(mps.A) - ref).max() < 1e-12 * np.abs(ref).max()


def test_swap_gate_exchanges_sites():
    """SWAP on (k, k+1) exchanges the two sites' reduced states of a product."""
    mps = tebd.MPS.product(["+x", "-y", "+z"], 3)
    mps.apply_gate(1, lm.swap_gate(), 16, 0.0, True)
    assert abs(mps.expect({1: lm.SZ}) - 1.0) < 1e-14
    assert abs(mps.expect({2: lm.SY}) + 1.0) < 1e-14
    assert abs(mps.expect({0: lm.SX}) - 1.0) < 1e-14


def test_unitary_channel_superoperator():
    """rho -> U rho U^+: trace preserving, unital, and on a product operator it
    equals conjugating the 4 x 4 matrix directly."""
    U = random_unitary(4, 5)
    G = lm.unitary_channel(U)
    rng = np.random.default_rng(1)
    r1 = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    r2 = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    v = np.kron(r1.reshape(4), r2.reshape(4))  # site-major (k1 b1)(k2 b2)
    out = (G @ v).reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)
    ref = U @ np.kron(r1, r2) @ U.conj().T
    assert np.abs(out - ref).max() < 1e-13
    e = np.kron(tebd.E_ID, tebd.E_ID)
    assert np.abs(e @ G - e).max() < 1e-13  # trace preserving
    ident = np.kron(np.eye(2).reshape(4), np.eye(2).reshape(4))
    assert np.abs(G @ ident - ident).max() < 1e-13  # unital


def test_cz_channel_is_diagonal_sign_pattern():
    """CZ rho CZ flips the sign of rho[k, b] when exactly one of k, b has both
    qubits in |1>."""
    G = tebd.cz_channel()
    assert np.abs(G - np.diag(np.diag(G))).max() == 0
    d = np.diag(G).real.reshape(2, 2, 2, 2)  # k1 b1 k2 b2
    for k1, b1, k2, b2 in np.ndindex(2, 2, 2, 2):
        sign = (-1) ** ((k1 & k2) + (b1 & b2))
        assert d[k1, b1, k2, b2] == sign


GRAPHS = [
    (5, [(0, 1), (1, 2), (2, 3), (3, 4)]),          # chain (cluster state)
    (5, [(0, 2), (0, 4), (1, 3), (2, 3)]),          # pairs apart along the path
    (6, [(0, 5), (1, 2), (2, 4), (0, 3), (3, 4)]),  # with a cycle
]


@pytest.mark.parametrize("N,pairs", GRAPHS)
def test_graph_state_closed_form_and_stabilisers(N, pairs):
    """The MPS graph state equals the closed-form amplitudes (-1)^(sum x_j x_k),
    is pure, and every stabiliser X_a prod_{b ~ a} Z_b has expectation 1."""
    mps = tebd.graph_state(N, pairs, 256, 0.0)
    v = dense.mps_to_vector(mps.A)
    ref = dense.graph_state_vector(N, pairs)
    assert np.abs(v - ref).max() < 1e-13
    assert abs(mps.tr_rho2() - 1.0) < 1e-12
    for a in range(N):
        ops = {a: lm.SX}
        for p, q in pairs:
            for u, w in ((p, q), (q, p)):
                if u == a:
                    ops[w] = lm.SZ @ ops.get(w, lm.I2)
        assert abs(mps.expect(ops) - 1.0) < 1e-12
        if any(a in e for e in pairs):
            assert abs(mps.expect({a: lm.SX})) < 1e-12


def test_graph_state_chain_bond_dimension():
    """A chain graph state has Schmidt rank 2 across every cut, so its density
    matrix has operator rank 4 (with the cutoff removing round-off)."""
    mps = tebd.graph_state(7, [(k, k + 1) for k in range(6)], 64, 1e-14)
    assert mps.bond_dims() == [4] * 6


def ladder_small():
    return workloads.ladder_model(n_rungs=3)  # N = 6, legs (s, s+2)


@pytest.mark.parametrize("order", [2, 4])
def test_general_sweep_tebd_equals_dense_trotter(order):
    """Ladder (bonds apart along the path) without truncation: the MPS with its
    SWAP network equals the dense product of the same factors applied to
    sites i, j directly."""
    m = ladder_small()
    assert not tebd.is_chain(m)
    mps = tebd.MPS.product("+z", m["N"])
    tebd.evolve(mps, m, 0.05, 4, 4 ** 3, 0.0, order=order)
    v = dense.trotter_evolve(dense.product_vector("+z", m["N"]), m, 0.05, 4, order=order)
    assert np.abs(dense.mps_to_vector(mps.A) - v).max() < 1e-12


@pytest.mark.parametrize("order,ratio", [(2, 4.0), (4, 16.0)])
def test_general_sweep_order_against_exact(order, ratio):
    """Halving tau divides the gap to exp(t L) by 2^order on a graph with a
    cycle and bonds apart along the path."""
    m = workloads.random_model(5, 11, bonds=[(0, 1), (0, 2), (1, 3), (2, 3), (3, 4), (2, 4)])
    v0 = dense.product_vector("+x", 5)
    T = 0.4
    exact = dense.exact_evolve(v0, m, [0.0, T])[-1]
    errs = []
    for n in (4, 8):
        v = dense.trotter_evolve(v0, m, T / n, n, order=order, force_trace=False)
        errs.append(np.abs(v - exact).max())
    assert errs[1] < errs[0]
    assert abs(errs[0] / errs[1] / ratio - 1.0) < 0.15, errs


def test_chain_in_another_order_takes_the_sweep():
    """The same chain with its bonds listed in reverse is a general bond list;
    both schedules are second order and agree to O(tau^2)."""
    m = workloads.jittered_chain(5, 2)
    r = dict(m)
    r["bonds"] = m["bonds"][::-1].copy()
    r["J"] = m["J"][::-1].copy()
    r["Jz"] = m["Jz"][::-1].copy()
    assert tebd.is_chain(m) and not tebd.is_chain(r)
    v0 = dense.product_vector("+x", 5)
    a = dense.trotter_evolve(v0, m, 0.01, 10)
    b = dense.trotter_evolve(v0, r, 0.01, 10)
    assert 0 < np.abs(a - b).max() < 1e-3
