"""Pins of the oracle's fourth-order Trotter scheme and of the global
characteristics S_2 (Eq. S_2) and OSEE (Eq. OSEE), Sec. 2.4."""
import numpy as np

import workloads
from oracle import dense
from oracle import model as lm
from oracle import tebd


def test_trotter_fourth_order_against_exact():
    """Halving tau divides the error of the composed scheme by ~16 (order 4),
    and it is far below the second-order error at the same tau."""
    m = workloads.random_model(4, 7)
    N = m["N"]
    v0 = dense.product_vector("+x", N)
    T = 0.8
    ex = dense.exact_evolve(v0, m, [0.0, T])[-1]
    b1, b2 = dense.zz_observables(ex, N)
    errs = {}
    for order in (2, 4):
        errs[order] = []
        for tau in (0.2, 0.1):
            vt = dense.trotter_evolve(v0.copy(), m, tau, int(round(T / tau)), order=order)
            a1, a2 = dense.zz_observables(vt, N)
            errs[order].append(max(np.abs(a1 - b1).max(), np.abs(a2 - b2).max()))
    r4 = errs[4][0] / errs[4][1]
    assert 12.0 < r4 < 20.0, r4
    assert errs[4][1] < 0.05 * errs[2][1]


def test_fourth_order_tebd_equals_dense_without_truncation():
    m = workloads.random_model(5, 2)
    mps = tebd.MPS.product("-y", 5)
    tebd.evolve(mps, m, 0.07, 4, 1024, 0.0, order=4)
    v = dense.trotter_evolve(dense.product_vector("-y", 5), m, 0.07, 4, order=4)
    for ops in ({0: lm.SZ}, {2: lm.SX, 4: lm.SY}, {1: lm.SZ, 3: lm.SZ}):
        assert abs(mps.expect(ops) - dense.expect(v, 5, ops)) < 1e-13


def test_fourth_order_schedule_weights():
    lay = tebd.trotter_layers(4)
    assert len(lay) == 7
    # each parity class sums to the full step; layers alternate parity
    assert abs(sum(f for p, f in lay if p == 0) - 1.0) < 1e-15
    assert abs(sum(f for p, f in lay if p == 1) - 1.0) < 1e-15
    assert [p for p, _ in lay] == [0, 1, 0, 1, 0, 1, 0]
    w1 = lay[1][1]
    assert abs(2 * w1 ** 3 + (1 - 2 * w1) ** 3) < 1e-14  # third-order condition of the triple product


def mixed_product_mps(rs):
    """MPS of the product of single-qubit states (I + r . sigma) / 2."""
    A = []
    for r in rs:
        rho = 0.5 * (np.eye(2) + r[0] * lm.SX + r[1] * lm.SY + r[2] * lm.SZ)
        A.append(rho.reshape(4).reshape(1, 4, 1).astype(np.complex128))
    return tebd.MPS(A, 0)


def test_renyi2_of_mixed_product_states():
    """S_2 is additive over a product, with tr rho^2 = (1 + |r|^2) / 2 per qubit;
    the r_y components make a transposed contraction fail."""
    rng = np.random.default_rng(3)
    rs = []
    for _ in range(5):
        r = rng.normal(size=3)
        rs.append(r / np.linalg.norm(r) * rng.uniform(0.1, 0.9))
    mps = mixed_product_mps(rs)
    want = sum(-np.log((1 + np.dot(r, r)) / 2) for r in rs)
    assert abs(mps.renyi2() - want) < 1e-13
    v = dense.mps_to_vector(mps.A)
    assert abs(dense.renyi2(v, 5) - want) < 1e-13
    assert abs(tebd.MPS.product("+y", 4).renyi2()) < 1e-14  # pure product state


def test_osee_pure_state_is_twice_von_neumann():
    """For rho = |psi><psi| the OSEE of a cut is twice the entanglement
    entropy of psi (stated with Eq. OSEE)."""
    rng = np.random.default_rng(4)
    N = 4
    psi = rng.normal(size=2 ** N) + 1j * rng.normal(size=2 ** N)
    psi /= np.linalg.norm(psi)
    rho = np.outer(psi, psi.conj())
    # vec with per-site (ket, bra) pairs: t[k0..k3, b0..b3] -> (k0 b0 k1 b1 ...)
    t = rho.reshape((2,) * (2 * N)).transpose([0, 4, 1, 5, 2, 6, 3, 7])
    v = t.reshape(-1)
    for bond in range(N - 1):
        nA = bond + 1
        rA = np.einsum("ij,kj->ik", psi.reshape(2 ** nA, -1), psi.reshape(2 ** nA, -1).conj())
        ev = np.linalg.eigvalsh(rA)
        ev = ev[ev > 1e-15]
        svn = float(-np.sum(ev * np.log(ev)))
        assert abs(dense.osee(v, N, bond) - 2 * svn) < 1e-12


def test_osee_product_zero_and_mps_matches_dense():
    assert abs(mixed_product_mps([[0.1, 0.2, 0.3], [0.0, -0.5, 0.1], [0.3, 0.3, 0.3]]).osee(1)) < 1e-14
    m = workloads.random_model(5, 5)
    mps = tebd.MPS.product("+x", 5)
    tebd.evolve(mps, m, 0.1, 6, 1024, 0.0)
    v = dense.trotter_evolve(dense.product_vector("+x", 5), m, 0.1, 6)
    for bond in range(4):
        assert abs(mps.osee(bond) - dense.osee(v, 5, bond)) < 1e-12
    assert abs(mps.renyi2() - dense.renyi2(v, 5)) < 1e-12


def test_trotter_third_order_against_exact():
    """Order 3 (chain): halving tau divides the error by ~8, and it sits below
    the second-order error at the same tau."""
    m = workloads.random_model(4, 7)
    N = m["N"]
    v0 = dense.product_vector("+x", N)
    T = 0.8
    ex = dense.exact_evolve(v0, m, [0.0, T])[-1]
    errs = {}
    for order in (2, 3):
        errs[order] = []
        for tau in (0.1, 0.05):
            vt = dense.trotter_evolve(v0.copy(), m, tau, int(round(T / tau)), order=order, force_trace=False)
            errs[order].append(np.abs(vt - ex).max())
    r3 = errs[3][0] / errs[3][1]
    assert 6.5 < r3 < 9.5, r3
    assert errs[3][1] < 0.5 * errs[2][1]


def test_third_order_schedule_and_tebd_equals_dense():
    lay = tebd.trotter_layers(3)
    assert [p for p, _ in lay] == [0, 1, 0, 1, 0, 1]
    assert abs(sum(f for p, f in lay if p == 0) - 1.0) < 1e-15
    assert abs(sum(f for p, f in lay if p == 1) - 1.0) < 1e-15
    # six layers: step n's layer j is ascending iff j is even, for every n
    s0, s1 = tebd.step_schedule(6, 0, 3), tebd.step_schedule(6, 1, 3)
    assert s0 == s1
    m = workloads.random_model(5, 4)
    mps = tebd.MPS.product("+x", 5)
    tebd.evolve(mps, m, 0.07, 3, 1024, 0.0, order=3)
    v = dense.trotter_evolve(dense.product_vector("+x", 5), m, 0.07, 3, order=3)
    for ops in ({0: lm.SZ}, {2: lm.SX, 4: lm.SY}, {1: lm.SZ, 3: lm.SZ}):
        assert abs(mps.expect(ops) - dense.expect(v, 5, ops)) < 1e-13


def nonhermitian_mps(N, seed, chi=4):
    """A generic MPS (not Hermitian), in canonical form with centre N-1."""
    rng = np.random.default_rng(seed)
    dims = [1] + [min(chi, 4 ** (k + 1), 4 ** (N - k - 1)) for k in range(N - 1)] + [1]
    A = [rng.standard_normal((dims[k], 4, dims[k + 1])) + 1j * rng.standard_normal((dims[k], 4, dims[k + 1]))
         for k in range(N)]
    mps = tebd.MPS(A, centre=0)
    mps.move_centre(N - 1)
    return mps


def test_adjoint_vector_is_the_matrix_adjoint():
    rng = np.random.default_rng(3)
    v = rng.standard_normal(4 ** 3) + 1j * rng.standard_normal(4 ** 3)
    M = dense.to_matrix(v, 3)
    assert np.abs(dense.to_matrix(dense.adjoint(v, 3), 3) - M.conj().T).max() == 0


def test_hermitize_equals_dense_hermitian_part():
    """Without truncation the MPS result is (rho + rho^+)/2 of the full vector,
    whose matrix is Hermitian; the trace becomes Re tr(rho)."""
    N = 5
    mps = nonhermitian_mps(N, 1)
    v = dense.mps_to_vector(mps.A)
    tr = mps.trace()
    mps.hermitize(4 ** 3, 1e-14)  # the cutoff drops the round-off tail of the rank-8 sum
    h = dense.mps_to_vector(mps.A)
    ref = 0.5 * (v + dense.adjoint(v, N))
    assert np.abs(h - ref).max() < 1e-12 * np.abs(ref).max()
    M = dense.to_matrix(h, N)
    assert np.abs(M - M.conj().T).max() < 1e-12 * np.abs(M).max()
    assert abs(mps.trace() - tr.real) < 1e-12 * abs(tr)
    assert mps.centre == 0
    assert max(mps.bond_dims()) <= 2 * 4


def test_hermitize_keeps_a_hermitian_state():
    """An evolved (Hermitian) state is unchanged, and the compression returns
    the bond dims to their exact ranks (the doubled copies are dependent)."""
    m = workloads.random_model(5, 3)
    mps = tebd.MPS.product("+x", 5)
    tebd.evolve(mps, m, 0.05, 3, 1024, 1e-13)
    v = dense.mps_to_vector(mps.A)
    dims = mps.bond_dims()
    mps.hermitize(1024, 1e-13)
    assert np.abs(dense.mps_to_vector(mps.A) - v).max() < 1e-12
    assert mps.bond_dims() == dims


def test_evolve_with_hermitian_every_matches_dense():
    """Second-order steps with the Hermitian part taken every 2nd step, no
    truncation, against the same sequence on the full vector."""
    m = workloads.random_model(4, 8)
    N = 4
    mps = nonhermitian_mps(N, 2)
    v = dense.mps_to_vector(mps.A)
    v = v / dense.trace(v, N)
    tebd.evolve(mps, m, 0.05, 4, 1024, 0.0, hermitian_every=2)
    gates = tebd.gate_tables(m, 0.05)
    for n in range(4):
        v = dense.trotter_evolve(v, m, 0.05, 1, gates=gates, first_step=n, force_trace=False)
        if (n + 1) % 2 == 0:
            v = 0.5 * (v + dense.adjoint(v, N))
        v = v / dense.trace(v, N)
    assert np.abs(dense.mps_to_vector(mps.A) - v).max() < 1e-12
