"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test targets a plausible mistake: a sign of a field or of a coupling, the
direction of a jump operator, a missing 1/2, a wrong degree weight, a wrong
vectorisation transpose, a wrong Trotter order, a wrong truncation rule.
"""
import os

import numpy as np
import pytest

import workloads
from oracle import closed_forms as cf
from oracle import dense
from oracle import model as lm
from oracle import tebd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def bloch_vector(v):
    """(x, y, z) of a one-site vectorised rho."""
    return np.array([np.real(tebd.covector(lm.PAULI[k]) @ v) for k in "XYZ"])


def test_single_site_generator_matches_bloch_equations():
    rng = np.random.default_rng(1)
    for _ in range(5):
        hx, hy, hz = rng.uniform(-2, 2, 3)
        g0, g1, g2 = rng.uniform(0, 0.5, 3)
        m = {"hx": [hx], "hy": [hy], "hz": [hz], "g0": [g0], "g1": [g1], "g2": [g2]}
        L = lm.single_site_generator(m, 0)
        r0 = rng.standard_normal(3)
        r0 /= np.linalg.norm(r0)
        v0 = 0.5 * (lm.I2 + r0[0] * lm.SX + r0[1] * lm.SY + r0[2] * lm.SZ).reshape(4)
        for t in (0.3, 1.7):
            import scipy.linalg
            v = scipy.linalg.expm(t * L) @ v0
            np.testing.assert_allclose(bloch_vector(v), cf.bloch_evolve(r0, t, hx, hy, hz, g0, g1, g2),
                                       atol=1e-13)


def test_bloch_steady_state_golden_and_tebd():
    """J = 0: each site follows its own Bloch equations; the driven edge
    relaxes to the optical-Bloch steady state (golden file)."""
    data = np.loadtxt(os.path.join(GOLDEN, "bloch_steady_driven_qubit.txt"))
    np.testing.assert_allclose(cf.bloch_steady_state(1.0, 0.0, 0.1, 0.05), data, atol=1e-15)
    m, _ = workloads.chain6_exact()
    m["J"][:] = 0.0
    m["N"] = 3
    m["bonds"] = m["bonds"][:2]
    m["J"] = m["J"][:2]
    m["Jz"] = m["Jz"][:2]
    for k in ("hx", "hy", "hz", "g0", "g1", "g2"):
        m[k] = m[k][:3]
    mps = tebd.MPS.product("+z", 3)
    tebd.evolve(mps, m, 0.25, 800, 4, 0.0)  # t = 200 >> 1/G1
    r = np.array([np.real(mps.expect({0: lm.PAULI[k]})) for k in "XYZ"])
    np.testing.assert_allclose(r, data, atol=1e-10)
    assert mps.bond_dims() == [1, 1]


def test_rabi_oscillation_sign():
    """Unitary drive of a single site from +z: z = cos(Omega t), y = -sin(Omega t)."""
    m = workloads.chain_model(3, 0.0, 0.0, 1.3, 0.0, 0.0)
    mps = tebd.MPS.product("+z", 3)
    tau = 0.1
    for n in range(10):
        tebd.evolve(mps, m, tau, 1, 4, 0.0, first_step=n)
        t = (n + 1) * tau
        assert abs(mps.expect({0: lm.SZ}) - np.cos(1.3 * t)) < 1e-12
        assert abs(mps.expect({0: lm.SY}) + np.sin(1.3 * t)) < 1e-12
        assert abs(mps.expect({0: lm.SX})) < 1e-12


def test_gate_properties():
    m = workloads.random_model(4, 3)
    e = np.kron(tebd.E_ID, tebd.E_ID)
    for b in range(3):
        G = lm.bond_gate(m, b, 0.07)
        np.testing.assert_allclose(e @ G, e, atol=1e-14)  # trace preserving
        np.testing.assert_allclose(G @ G, lm.bond_gate(m, b, 0.14), atol=1e-13)
        Gp = tebd.gate_to_pauli(G)
        assert np.abs(Gp.imag).max() < 1e-14  # real in the Pauli basis
    # J = Jz = 0: the bond gate factorises into weighted one-site exponentials
    m["J"][:] = 0.0
    m["Jz"][:] = 0.0
    import scipy.linalg
    deg = lm.site_degrees(m)
    G = lm.bond_gate(m, 1, 0.3)
    Gi = scipy.linalg.expm(0.3 / deg[1] * lm.single_site_generator(m, 1))
    Gj = scipy.linalg.expm(0.3 / deg[2] * lm.single_site_generator(m, 2))
    np.testing.assert_allclose(G, np.kron(Gi, Gj), atol=1e-13)


def test_sum_of_bond_generators_is_full_liouvillian():
    """Independent construction of the full Lindbladian on 2^N x 2^N matrices."""
    m = workloads.random_model(3, 5)
    N = 3
    Lsum = dense.liouvillian(m).toarray()

    def embed(op, site):
        mats = [lm.I2] * N
        mats[site] = op
        out = np.ones((1, 1))
        for x in mats:
            out = np.kron(out, x)
        return out

    H = sum(0.5 * (m["hx"][s] * embed(lm.SX, s) + m["hy"][s] * embed(lm.SY, s) + m["hz"][s] * embed(lm.SZ, s))
            for s in range(N))
    for b, (i, j) in enumerate(m["bonds"]):
        H = H + m["J"][b] * (embed(lm.SP, i) @ embed(lm.SM, j) + embed(lm.SM, i) @ embed(lm.SP, j))
        H = H + 0.5 * m["Jz"][b] * embed(lm.SZ, i) @ embed(lm.SZ, j)
    jumps = []
    for s in range(N):
        jumps += [np.sqrt(m["g0"][s]) * embed(lm.SP, s), np.sqrt(m["g1"][s]) * embed(lm.SM, s),
                  np.sqrt(m["g2"][s]) * embed(lm.SZ, s)]
    rng = np.random.default_rng(0)
    X = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    LX = -1j * (H @ X - X @ H)
    for Lk in jumps:
        LX = LX + Lk @ X @ Lk.conj().T - 0.5 * (Lk.conj().T @ Lk @ X + X @ Lk.conj().T @ Lk)
    # X as a site-major vector: entries X[k0k1k2, b0b1b2] -> (k0 b0)(k1 b1)(k2 b2)
    vx = X.reshape(2, 2, 2, 2, 2, 2).transpose(0, 3, 1, 4, 2, 5).reshape(-1)
    got = dense.to_matrix(Lsum @ vx, N)
    np.testing.assert_allclose(got, LX, atol=1e-12)


def test_tebd_equals_dense_trotter_without_truncation():
    m = workloads.random_model(5, 7)
    N = 5
    mps = tebd.MPS.product(["+z", "-x", "+y", "-z", "+x"], N)
    v = dense.product_vector(["+z", "-x", "+y", "-z", "+x"], N)
    gates = tebd.gate_tables(m, 0.05)
    for n in range(6):
        tebd.evolve(mps, m, 0.05, 1, 16, 0.0, gates=gates, first_step=n)
        v = dense.trotter_evolve(v, m, 0.05, 1, gates=gates, first_step=n)
    np.testing.assert_allclose(dense.mps_to_vector(mps.A), v, atol=1e-13)
    for ops in ({1: lm.SX}, {0: lm.SZ, 4: lm.SY}, {2: lm.SX, 3: lm.SZ}):
        assert abs(mps.expect(ops) - dense.expect(v, N, ops)) < 1e-13
    assert mps.bond_dims() == [4, 16, 16, 4]  # 4^floor(N/2) cap (App. B)


def test_trotter_second_order_against_exact():
    m, run = workloads.chain6_exact()
    N = m["N"]
    v0 = dense.product_vector("+z", N)
    T = 1.0
    ex = dense.exact_evolve(v0, m, [0.0, T])[-1]
    errs = []
    for tau in (0.1, 0.05, 0.025):
        vt = dense.trotter_evolve(v0.copy(), m, tau, int(round(T / tau)))
        a1, a2 = dense.zz_observables(vt, N)
        b1, b2 = dense.zz_observables(ex, N)
        errs.append(max(np.abs(a1 - b1).max(), np.abs(a2 - b2).max()))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5
    assert errs[2] < 3e-5


def test_chain6_oracle_close_to_exact():
    """The exact 6-site chain (tau = 0.01, T = 1, chi = 64 = 4^3): MPS-TEBD is within the
    O(tau^2) Trotter error of the exact Lindblad evolution."""
    m, run = workloads.chain6_exact()
    N = m["N"]
    mps = tebd.MPS.product("+z", N)
    tebd.evolve(mps, m, run["tau"], 100, run["chi_max"], run["cutoff"])
    ex = dense.exact_evolve(dense.product_vector("+z", N), m, [0.0, 1.0])[-1]
    a1, a2 = tebd.zz_observables(mps)
    b1, b2 = dense.zz_observables(ex, N)
    err = max(np.abs(a1 - b1).max(), np.abs(a2 - b2).max())
    # second-order Trotter error: 1.8e-5 at tau = 0.025 scales to ~3e-6 at 0.01
    assert 1e-7 < err < 6e-6


def one_excitation_run(m, site0, tau, steps):
    N = m["N"]
    labels = ["+z"] * N
    labels[site0] = "-z"
    mps = tebd.MPS.product(labels, N)
    z1, z2 = [], []

    def obs(n, s):
        a, b = tebd.zz_observables(s)
        z1.append(a)
        z2.append(b)

    tebd.evolve(mps, m, tau, steps, 64, 0.0, observer=obs)
    return np.real(np.array(z1)), np.real(np.array(z2)), mps


def test_one_excitation_sector_closed_form():
    """Omega = 0, Jz = 0, non-uniform J, h_z, g0, g2 (quasi-free XY chain)."""
    rng = np.random.default_rng(11)
    N = 7
    m = workloads.chain_model(N, rng.uniform(0.5, 1.5, N - 1), rng.uniform(-1, 1, N), 0.0, 0.1, 0.03)
    m["g0"] = rng.uniform(0.05, 0.2, N)
    m["g2"] = rng.uniform(0.0, 0.1, N)
    T = 1.0
    errs = []
    for tau in (0.05, 0.025):
        steps = int(round(T / tau))
        z1, z2, _ = one_excitation_run(m, 2, tau, steps)
        e1, e2 = cf.one_excitation(m, 2, [tau * (n + 1) for n in range(steps)])
        errs.append(max(np.abs(z1 - e1).max(), np.abs(z2 - e2).max()))
    assert errs[1] < 2e-4
    assert 3.0 < errs[0] / errs[1] < 5.0  # Trotter error, second order


def test_one_excitation_long_chain():
    """N = 20: bond dimensions stay small and the closed form holds."""
    N = 20
    m = workloads.chain_model(N, 1.0, workloads.alternating(N, 0.7), 0.0, 0.1, 0.05)
    labels = ["+z"] * N
    labels[9] = "-z"
    mps = tebd.MPS.product(labels, N)
    tebd.evolve(mps, m, 0.01, 60, 64, 1e-20)  # drops round-off singular values only
    e1, e2 = cf.one_excitation(m, 9, [0.6])
    z1 = np.real([mps.expect({i: lm.SZ}) for i in range(N)])
    assert np.abs(z1 - e1[0]).max() < 2e-5
    pairs = [(i, j) for i in range(N) for j in range(i + 1, N)]
    for i, j in ((8, 9), (9, 10), (7, 11), (0, 19)):
        z2 = np.real(mps.expect({i: lm.SZ, j: lm.SZ}))
        assert abs(z2 - e2[0][pairs.index((i, j))]) < 2e-5
    # operator Schmidt rank across a cut <= 2 + 2 rank(P[left, right]): small
    assert max(mps.bond_dims()) <= 16


def test_delta_zero_symmetry_survives_truncation():
    """h_z = h_y = Jz = 0 and h_x only on even sites: <sx_even> = <sy_odd> = 0
    exactly (the x-projection of the driven qubit stays 0, Sec. 3.2), also with
    truncation, because the symmetry is a sign flip per site in the Pauli basis."""
    N = 8
    m = workloads.chain_model(N, 1.0, 0.0, 1.0, 0.1, 0.05)
    m["hx"][4] = 0.6
    mps = tebd.MPS.product("+z", N)
    tebd.evolve(mps, m, 0.05, 30, 6, 1e-12)
    assert max(mps.bond_dims()) == 6  # truncation active
    assert mps.discarded > 1e-8
    for i in range(N):
        O = lm.SX if i % 2 == 0 else lm.SY
        assert abs(mps.expect({i: O})) < 1e-13
    assert abs(mps.expect({0: lm.SY})) > 1e-2


def test_trace_and_hermiticity_invariants():
    m, run = workloads.chain6_exact()
    N = 6
    v = dense.product_vector("+z", N)
    v = dense.trotter_evolve(v, m, 0.05, 20, force_trace=False)
    assert abs(dense.trace(v, N) - 1) < 1e-13
    rho = dense.to_matrix(v, N)
    assert np.abs(rho - rho.conj().T).max() < 1e-14
    # truncated MPS: Hermitian to round-off (observables real), trace drifts
    mps = tebd.MPS.product("+x", N)
    tebd.evolve(mps, m, 0.05, 20, 8, 1e-10, force_trace=False)
    assert mps.discarded > 0
    rho = dense.to_matrix(dense.mps_to_vector(mps.A), N)
    assert np.abs(rho - rho.conj().T).max() < 1e-13
    assert abs(np.imag(mps.expect({2: lm.SX, 3: lm.SY}))) < 1e-13


@pytest.mark.parametrize("s,chi,cut,k", [
    ([3.0, 2.0, 1.0], 5, 0.0, 3),
    ([3.0, 2.0, 1.0], 2, 0.0, 2),
    ([3.0, 2.0, 0.0, 0.0], 9, 0.0, 2),            # exact zeros are discarded
    ([1.0, 1e-3, 1e-6], 9, 2e-6, 1),              # tail 1e-6 + 1e-12 <= 2e-6 W
    ([1.0, 1e-3, 1e-6], 9, 1e-7, 2),
    ([1.0, 1e-3, 1e-6], 9, 1e-13, 3),
    ([1.0, 0.5], 9, 0.25, 1),                     # tail 0.25 <= 0.25 * 1.25
    ([1.0, 0.5], 9, 0.19, 2),                     # tail 0.25 >  0.19 * 1.25
])
def test_truncation_rule_brute_force(s, chi, cut, k):
    """Spectra without ties: the plain rule of App. B."""
    s = np.array(s)
    got, disc, W = tebd.truncation_rank(s, chi, cut)
    # brute force: smallest kk >= 1 whose discarded weight is within the cutoff
    w = s ** 2
    kc = next(kk for kk in range(1, len(s) + 1) if w[kk:].sum() <= cut * w.sum())
    assert got == min(chi, kc)
    assert disc == pytest.approx(w[got:].sum())
    assert W == pytest.approx(w.sum())
    assert got == k


@pytest.mark.parametrize("s,chi,cut,k", [
    ([1.0, 0.5, 0.5, 0.1], 2, 0.0, 1),            # chi_max cuts the pair 0.5, 0.5: drop it whole
    ([1.0, 0.5, 0.5, 0.1], 3, 0.0, 3),            # the pair fits under chi_max: no change
    ([1.0, 0.5, 0.5, 0.5, 0.1], 2, 0.0, 1),       # a triplet
    ([1.0, 0.5, 0.5, 0.5, 0.1], 3, 0.0, 1),
    ([1.0, 0.3, 0.3, 1e-4], 9, 0.05, 3),          # the cutoff alone keeps one of the pair: keep both
    ([1.0, 0.3, 0.3, 1e-4], 2, 0.05, 1),          # ... unless chi_max forbids: drop both
    ([1.0, 0.3, 0.3 - 2e-5, 1e-4], 2, 0.05, 1),   # within 1e-4 of 0.3: a multiplet, dropped whole
    ([1.0, 0.3, 0.3 - 5e-5, 1e-4], 2, 0.05, 2),   # 5e-5 / 0.3 > 1e-4 apart: two values, the plain rule
    ([1.0, 1e-12, 5e-13, 0.0], 2, 0.0, 2),        # values far below s_1 tie only relative to themselves
    ([1.0, 1.0, 0.2], 1, 0.0, 1),                 # the multiplet holds s_1: k stays >= 1
    ([1e-20, 1e-20, 0.0], 1, 0.0, 1),
    ([2.0, 1e-12, 0.0, 0.0], 9, 0.0, 2),          # tiny nonzero vs exact zero: no tie, zeros dropped
])
def test_truncation_rule_never_splits_a_multiplet(s, chi, cut, k):
    """Spectra with ties at the cut, against a brute force over every k:
    among the ks that do not split a multiplet (the k-th and (k+1)-th values
    not within 1e-4 of the k-th, exact zeros excluded) and keep at most chi_max, the
    smallest whose discarded weight is within the cutoff if one exists, else
    the largest (chi_max decides)."""
    s = np.array(s)
    got, disc, W = tebd.truncation_rank(s, chi, cut)
    w = s ** 2
    nz = int(np.count_nonzero(s))

    def splits(kk):
        return kk < nz and s[kk - 1] - s[kk] <= 1e-4 * s[kk - 1]

    ok = [kk for kk in range(1, nz + 1) if kk <= chi and not splits(kk)]
    within = [kk for kk in ok if w[kk:].sum() <= cut * w.sum()]
    want = min(within) if within else (max(ok) if ok else 1)
    assert got == want == k
    assert disc == pytest.approx(w[got:].sum(), abs=1e-300)


def test_truncated_converges_to_dense_as_chi_grows():
    m = workloads.jittered_chain(6, 0)
    N = 6
    v = dense.trotter_evolve(dense.product_vector("+x", N), m, 0.05, 20)
    b1, b2 = dense.zz_observables(v, N)
    errs = []
    for chi in (4, 16, 64):
        mps = tebd.MPS.product("+x", N)
        tebd.evolve(mps, m, 0.05, 20, chi, 0.0)
        a1, a2 = tebd.zz_observables(mps)
        errs.append(max(np.abs(a1 - b1).max(), np.abs(a2 - b2).max()))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-12


def test_pauli_basis_conversion_roundtrip():
    m = workloads.random_model(4, 9)
    mps = tebd.MPS.product("+x", 4)
    tebd.evolve(mps, m, 0.1, 3, 16, 0.0)
    back = tebd.from_pauli(tebd.to_pauli(mps.A))
    for a, b in zip(back, mps.A):
        np.testing.assert_allclose(a, b, atol=1e-15)
    # product state +z in the Pauli basis: (1, 0, 0, 1) / sqrt(2) per site
    p = tebd.to_pauli(tebd.MPS.product("+z", 2).A)[0].reshape(4)
    np.testing.assert_allclose(p, np.array([1, 0, 0, 1]) / np.sqrt(2), atol=1e-15)


def one_excitation_coherence_errors(N=6, tau=0.01, steps=50):
    """Max deviation of XX+YY and XY-YX on all pairs from 4 Re/-4 Im P_jk."""
    rng = np.random.default_rng(4)
    m = workloads.chain_model(N, rng.uniform(0.5, 1.5, N - 1), rng.uniform(-1, 1, N), 0.0, 0.1, 0.03)
    labels = ["+z"] * N
    labels[1] = "-z"
    mps = tebd.MPS.product(labels, N)
    tebd.evolve(mps, m, tau, steps, 64, 1e-20)
    P = cf.one_excitation_P(m, 1, tau * steps)
    err = 0.0
    for i in range(N):
        for j in range(i + 1, N):
            xx = mps.expect({i: lm.SX, j: lm.SX}) + mps.expect({i: lm.SY, j: lm.SY})
            xy = mps.expect({i: lm.SX, j: lm.SY}) - mps.expect({i: lm.SY, j: lm.SX})
            err = max(err, abs(xx - 4 * P[i, j].real), abs(xy + 4 * P[i, j].imag))
    return err


def test_one_excitation_coherences_fix_signs():
    """Coherences P_jk are sensitive to the signs of J and h_z and to the
    (ket, bra) vectorisation convention, which <sz> alone cannot see."""
    assert one_excitation_coherence_errors() < 1e-4  # second-order Trotter error at tau = 0.01


# ---- planted mistakes: each must be caught by one of the pins above ----

def _plant(monkeypatch, what):
    if what == "jump_direction":      # D0 with sigma^- instead of sigma^+
        monkeypatch.setattr(lm, "SP", lm.SM.copy())
    elif what == "J_sign":
        orig = lm.bond_generator

        def flipped(model, b):
            m = dict(model)
            m["J"] = -np.asarray(model["J"])
            return orig(m, b)
        monkeypatch.setattr(lm, "bond_generator", flipped)
    elif what == "hz_sign":
        orig_h = lm.onsite_hamiltonian
        monkeypatch.setattr(lm, "onsite_hamiltonian",
                            lambda model, s: orig_h(model, s) - model["hz"][s] * lm.SZ)
    elif what == "dissipator_transpose":   # L rho L^T instead of L rho L^+
        monkeypatch.setattr(lm, "superop", lambda A, B: np.kron(A, B))
    elif what == "degree_weight":
        monkeypatch.setattr(lm, "site_degrees", lambda model: np.ones(model["N"], dtype=np.int64))


@pytest.mark.parametrize("what", ["jump_direction", "J_sign", "hz_sign", "dissipator_transpose",
                                  "degree_weight"])
def test_planted_mistakes_are_caught(monkeypatch, what):
    _plant(monkeypatch, what)
    caught = []
    data = np.loadtxt(os.path.join(GOLDEN, "bloch_steady_driven_qubit.txt"))
    m = workloads.chain_model(3, 0.0, 0.0, 1.0, 0.1, 0.05)
    mps = tebd.MPS.product("+z", 3)
    tebd.evolve(mps, m, 0.25, 400, 4, 0.0)
    r = np.array([np.real(mps.expect({0: lm.PAULI[k]})) for k in "XYZ"])
    caught.append(np.abs(r - data).max() > 1e-6)
    caught.append(one_excitation_coherence_errors(N=5, steps=30) > 1e-3)
    assert any(caught), what
