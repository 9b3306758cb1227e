"""Pins of the oracle's adjoint gradient (oracle/adjoint.py) against what does
not depend on it: central differences of the dense Trotter evolution (the same
product of gates on the full 4^N vector, no MPS), brute-force contractions of
the full vectors, and central differences of the matrix exponential."""
import numpy as np
import pytest
import scipy.linalg

from oracle import adjoint, dense, tebd
from oracle import model as lm


def rich_chain(N, seed):
    """Every parameter nonzero, so that a dropped term shows."""
    rng = np.random.default_rng(seed)
    nb = N - 1
    return {
        "N": N,
        "bonds": np.array([[b, b + 1] for b in range(nb)]),
        "J": rng.uniform(0.5, 1.5, nb), "Jz": rng.uniform(-0.8, 0.8, nb),
        "hx": rng.uniform(-1, 1, N), "hy": rng.uniform(-1, 1, N), "hz": rng.uniform(-2, 2, N),
        "g0": rng.uniform(0.05, 0.3, N), "g1": rng.uniform(0.02, 0.2, N), "g2": rng.uniform(0.02, 0.2, N),
    }


def rich_graph(N, bonds, seed):
    m = rich_chain(N, seed)
    rng = np.random.default_rng(seed + 1)
    nb = len(bonds)
    m["bonds"] = np.asarray(bonds)
    m["J"], m["Jz"] = rng.uniform(0.5, 1.5, nb), rng.uniform(-0.8, 0.8, nb)
    return m


def dense_expectation(model, tau, steps, init, site, pauli, order=2, force_trace=True):
    N = model["N"]
    v = dense.product_vector(init, N)
    v = dense.trotter_evolve(v, model, tau, steps, order=order, force_trace=force_trace)
    return dense.expect(v, N, {site: lm.PAULI[pauli]})


def dense_fd_gradient(model, tau, steps, init, site, pauli, order=2, force_trace=True, h=1e-6):
    out = []
    for key, idx in adjoint.parameter_list(model):
        vals = []
        for sgn in (1.0, -1.0):
            m = {k: (np.array(v, dtype=float) if k in adjoint.SITE_KEYS + adjoint.BOND_KEYS else v)
                 for k, v in model.items()}
            m[key][idx] += sgn * h
            vals.append(dense_expectation(m, tau, steps, init, site, pauli, order, force_trace))
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out)


def test_forward_record_is_the_tebd_run():
    """The recording forward pass performs exactly tebd.evolve's gates."""
    m = rich_chain(5, 1)
    mps, records, traces = adjoint.forward_record(m, 0.1, 3, 6, 1e-8, "+x")
    ref = tebd.MPS.product("+x", 5)
    tebd.evolve(ref, m, 0.1, 3, 6, 1e-8)
    for a, b in zip(mps.A, ref.A):
        assert np.array_equal(a, b)
    assert len(records) == 3 and all(len(r) == 6 for r in records)  # A, B, A: 2 + 2 + 2 gates on 5 sites
    assert np.allclose(traces, 1.0, atol=1e-2)  # truncation alone moves the trace


def test_forward_record_swap_network_is_the_tebd_run():
    m = rich_graph(4, [[0, 1], [0, 2], [1, 3], [2, 3]], 2)
    mps, records, _ = adjoint.forward_record(m, 0.1, 2, 16, 0.0, "+x")
    ref = tebd.MPS.product("+x", 4)
    tebd.evolve(ref, m, 0.1, 2, 16, 0.0)
    for a, b in zip(mps.A, ref.A):
        assert np.array_equal(a, b)
    # per step: F and R sweeps over 4 bonds, the two bonds apart taking 2 SWAPs each
    assert len(records[0]) == 2 * (4 + 2 * 2)
    assert sum(r[1] is None for r in records[0]) == 8


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_transition_density_brute_force(k):
    """tr(K Gamma) equals <mu, K rho> on the full vectors, for random MPS and K."""
    rng = np.random.default_rng(k)
    N = 5
    dims = [1, 3, 4, 5, 2, 1]
    mk = lambda d: [rng.standard_normal((d[s], 4, d[s + 1])) + 1j * rng.standard_normal((d[s], 4, d[s + 1]))
                    for s in range(N)]
    mu, rho = mk(dims), mk([1, 2, 6, 3, 4, 1])
    K = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    Gam = adjoint.transition_density(mu, rho, k)
    got = np.sum(K * Gam.T)
    ref = np.dot(dense.mps_to_vector(mu), dense.apply_two_site(dense.mps_to_vector(rho), K, k, k + 1, N))
    assert abs(got - ref) <= 1e-12 * abs(ref)


def test_k_matrix_against_central_differences_of_expm():
    m = rich_chain(3, 4)
    L = lm.bond_generator(m, 0)
    for key, idx in [("hz", 0), ("g0", 1), ("J", 0), ("hy", 1)]:
        dL = adjoint.generator_derivative(m, 0, key, idx)
        x, h = 0.07, 1e-5
        fd = (scipy.linalg.expm(x * (L + h * dL)) - scipy.linalg.expm(x * (L - h * dL))) / (2 * h)
        K = adjoint.k_matrix(L, dL, x)
        assert np.abs(K @ scipy.linalg.expm(x * L) - fd).max() < 1e-9


def test_generator_is_linear_in_every_parameter():
    """The unit-model derivative reproduces L_b exactly as sum theta dL/dtheta."""
    m = rich_graph(4, [[0, 1], [0, 2], [1, 3], [2, 3]], 5)
    for b in range(4):
        acc = sum(m[k][i] * adjoint.generator_derivative(m, b, k, i) for k, i in adjoint.bond_parameters(m, b))
        assert np.abs(acc - lm.bond_generator(m, b)).max() < 1e-12


@pytest.mark.parametrize("site,pauli,force", [(1, "Z", True), (2, "X", True), (0, "Y", False)])
def test_exact_chain_gradient_equals_dense_trotter_derivative(site, pauli, force):
    """No truncation (chi = 4^2 on 4 sites, cutoff 0): every one of the 30
    derivatives equals central differences of the dense Trotter product."""
    m = rich_chain(4, 7)
    tau, steps = 0.1, 3
    F, g, _ = adjoint.gradient(m, tau, steps, 16, 0.0, "+x", site, pauli, force_trace=force)
    assert abs(F - dense_expectation(m, tau, steps, "+x", site, pauli, force_trace=force)) < 1e-12
    got = adjoint.flatten(m, g)
    ref = dense_fd_gradient(m, tau, steps, "+x", site, pauli, force_trace=force)
    assert np.abs(got.imag).max() < 1e-12
    assert np.abs(got - ref).max() < 1e-8, np.abs(got - ref).max()


def test_exact_plaquette_gradient_equals_dense_trotter_derivative():
    """A 2 x 2 plaquette on the zigzag path: two of the four bonds go through
    the SWAP network, whose transposes the co-state passes back through."""
    m = rich_graph(4, [[0, 1], [0, 2], [1, 3], [2, 3]], 8)
    tau, steps = 0.1, 2
    F, g, _ = adjoint.gradient(m, tau, steps, 16, 0.0, "+z", 3, "X")
    got = adjoint.flatten(m, g)
    ref = dense_fd_gradient(m, tau, steps, "+z", 3, "X")
    assert np.abs(got - ref).max() < 1e-8, np.abs(got - ref).max()


def test_exact_fourth_order_gradient_equals_dense_trotter_derivative():
    m = rich_chain(3, 9)
    F, g, _ = adjoint.gradient(m, 0.15, 2, 16, 0.0, "+y", 0, "Z", order=4)
    got = adjoint.flatten(m, g)
    ref = dense_fd_gradient(m, 0.15, 2, "+y", 0, "Z", order=4)
    assert np.abs(got - ref).max() < 1e-8, np.abs(got - ref).max()


def test_truncated_gradient_approaches_the_dense_derivative():
    """With truncation the co-state gradient approximates the Trotter
    derivative; the error falls as chi grows and vanishes at the exact chi."""
    m = rich_chain(6, 11)
    tau, steps = 0.1, 4
    ref = dense_fd_gradient(m, tau, steps, "+x", 2, "Z")
    errs = []
    for chi in (4, 8, 16, 64):
        _, g, _ = adjoint.gradient(m, tau, steps, chi, 0.0, "+x", 2, "Z")
        errs.append(np.abs(adjoint.flatten(m, g) - ref).max())
    assert errs[-1] < 1e-8
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[1] < 0.05 * np.abs(ref).max()


@pytest.mark.parametrize("N,site,pauli", [(2, 0, "X"), (4, 2, "Z"), (5, 4, "Y")])
def test_costate_brute_force(N, site, pauli):
    """<mu_T, v> = (Tr(O v) - F Tr(v)) / tr for any vector v (the F 1 term
    contributes nothing to exact trace-preserving dynamics, so it is pinned
    here on its own), and the QR sweep leaves sites 0..N-2 left-orthonormal."""
    rng = np.random.default_rng(N)
    F, tr = 0.3 - 0.2j, 0.9 + 0.1j
    mu = adjoint.costate(N, site, pauli, F, tr)
    v = rng.standard_normal(4 ** N) + 1j * rng.standard_normal(4 ** N)
    ops = {site: lm.PAULI[pauli]}
    cov_o = [tebd.covector(ops[k]) if k in ops else tebd.E_ID for k in range(N)]
    ref = (dense.contract(v, cov_o) - F * dense.contract(v, [tebd.E_ID] * N)) / tr
    got = np.dot(dense.mps_to_vector(mu.A), v)
    assert abs(got - ref) <= 1e-12 * abs(ref)
    for A in mu.A[:-1]:
        M = A.reshape(-1, A.shape[2])
        assert np.abs(M.conj().T @ M - np.eye(M.shape[1])).max() < 1e-12


def dense_string_expectation(model, tau, steps, init, paulis, order=2):
    N = model["N"]
    v = dense.trotter_evolve(dense.product_vector(init, N), model, tau, steps, order=order)
    return dense.expect(v, N, {s: lm.PAULI[p] for s, p in enumerate(paulis) if p != "I"})


@pytest.mark.parametrize("paulis", ["ZIZI", "XYIZ"])
def test_exact_string_gradient_equals_dense_trotter_derivative(paulis):
    """Correlators and longer Pauli strings: the co-state starts from the product
    covector of the string; every derivative against dense central differences."""
    m = rich_chain(4, 13)
    tau, steps, h = 0.1, 3, 1e-6
    F, g, _ = adjoint.gradient(m, tau, steps, 16, 0.0, "+x", None, None, paulis=paulis)
    assert abs(F - dense_string_expectation(m, tau, steps, "+x", paulis)) < 1e-12
    got = adjoint.flatten(m, g)
    ref = []
    for key, idx in adjoint.parameter_list(m):
        vals = []
        for sgn in (1.0, -1.0):
            mm = {k: (np.array(v, dtype=float) if k in adjoint.SITE_KEYS + adjoint.BOND_KEYS else v)
                  for k, v in m.items()}
            mm[key][idx] += sgn * h
            vals.append(dense_string_expectation(mm, tau, steps, "+x", paulis))
        ref.append((vals[0] - vals[1]) / (2 * h))
    assert np.abs(got - np.array(ref)).max() < 1e-8


def test_costate_string_brute_force():
    N, F, tr = 4, 0.1 + 0.05j, 1.2
    ops = {0: "X", 2: "Y", 3: "Z"}
    mu = adjoint.costate_string(N, ops, F, tr)
    v = np.random.default_rng(3).standard_normal(4 ** N) + 0j
    cov = [tebd.covector(lm.PAULI[ops[k]]) if k in ops else tebd.E_ID for k in range(N)]
    ref = (dense.contract(v, cov) - F * dense.contract(v, [tebd.E_ID] * N)) / tr
    assert abs(np.dot(dense.mps_to_vector(mu.A), v) - ref) <= 1e-12 * abs(ref)


def test_exact_connected_correlator_gradient_equals_dense_trotter_derivative():
    """<Z_0 X_3> - <Z_0><X_3>: the four-term co-state against dense central differences."""
    m = rich_chain(4, 17)
    tau, steps, h = 0.1, 3, 1e-6

    def dense_C(model):
        N = model["N"]
        v = dense.trotter_evolve(dense.product_vector("+x", N), model, tau, steps)
        return (dense.expect(v, N, {0: lm.SZ, 3: lm.SX})
                - dense.expect(v, N, {0: lm.SZ}) * dense.expect(v, N, {3: lm.SX}))

    C, g, _ = adjoint.gradient_connected(m, tau, steps, 16, 0.0, "+x", 0, 3, "ZX")
    assert abs(C - dense_C(m)) < 1e-12
    ref = []
    for key, idx in adjoint.parameter_list(m):
        vals = []
        for sgn in (1.0, -1.0):
            mm = {k: (np.array(v, dtype=float) if k in adjoint.SITE_KEYS + adjoint.BOND_KEYS else v)
                  for k, v in m.items()}
            mm[key][idx] += sgn * h
            vals.append(dense_C(mm))
        ref.append((vals[0] - vals[1]) / (2 * h))
    assert np.abs(adjoint.flatten(m, g) - np.array(ref)).max() < 1e-8


def test_costate_terms_brute_force():
    N = 5
    terms = [(0.7, {1: "Z", 4: "X"}), (-0.2, {1: "Z"}), (0.3, {4: "X"}), (1.1, {})]
    mu = adjoint.costate_terms(N, terms)
    v = np.random.default_rng(4).standard_normal(4 ** N) + 1j * np.random.default_rng(5).standard_normal(4 ** N)
    ref = 0.0
    for c, ops in terms:
        ref += c * dense.contract(v, [tebd.covector(lm.PAULI[ops[k]]) if k in ops else tebd.E_ID
                                      for k in range(N)])
    assert abs(np.dot(dense.mps_to_vector(mu.A), v) - ref) <= 1e-12 * abs(ref)


def test_series_gradient_equals_dense_trotter_derivative():
    """J = sum_k w_k <X_1 Z_2>(t_k) over three output steps: the co-state gains a
    source at each; every derivative against dense central differences of J."""
    m = rich_chain(4, 23)
    tau, steps, h = 0.1, 4, 1e-6
    outs, ws = [1, 3, 4], [0.5, -1.2, 2.0]

    def dense_J(model):
        N = model["N"]
        v = dense.product_vector("+x", N)
        J = 0.0
        for n in range(steps):
            v = dense.trotter_evolve(v, model, tau, 1, first_step=n)
            if n + 1 in outs:
                J += ws[outs.index(n + 1)] * dense.expect(v, N, {1: lm.SX, 2: lm.SZ})
        return J

    F, g, _ = adjoint.gradient_series(m, tau, steps, 16, 0.0, "+x", "IXZI", outs, ws)
    assert abs(np.dot(ws, F) - dense_J(m)) < 1e-12
    ref = []
    for key, idx in adjoint.parameter_list(m):
        vals = []
        for sgn in (1.0, -1.0):
            mm = {k: (np.array(v, dtype=float) if k in adjoint.SITE_KEYS + adjoint.BOND_KEYS else v)
                  for k, v in m.items()}
            mm[key][idx] += sgn * h
            vals.append(dense_J(mm))
        ref.append((vals[0] - vals[1]) / (2 * h))
    assert np.abs(adjoint.flatten(m, g) - np.array(ref)).max() < 1e-8


def test_series_with_one_final_output_is_the_plain_gradient():
    m = rich_chain(5, 24)
    F1, g1, _ = adjoint.gradient(m, 0.1, 3, 8, 1e-10, "+x", None, None, paulis="IZIII")
    F2, g2, _ = adjoint.gradient_series(m, 0.1, 3, 8, 1e-10, "+x", "IZIII", [3], [1.0])
    assert F2[0] == F1
    assert np.array_equal(adjoint.flatten(m, g1), adjoint.flatten(m, g2))


def test_add_compress_is_the_sum_without_truncation():
    rng = np.random.default_rng(25)
    N = 5
    mk = lambda d: tebd.MPS([rng.standard_normal((d[s], 4, d[s + 1])) + 1j * rng.standard_normal((d[s], 4, d[s + 1]))
                             for s in range(N)], 0)
    a, b = mk([1, 3, 4, 5, 2, 1]), mk([1, 2, 2, 2, 2, 1])
    ref = dense.mps_to_vector(a.A) + dense.mps_to_vector(b.A)
    out = adjoint.add_compress(a, b, 64, 0.0)
    assert np.abs(dense.mps_to_vector(out.A) - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("steps", [1, 3])
def test_two_qubit_gradient_equals_dense_trotter_derivative(steps):
    """The smallest system: one bond, no environments on either side."""
    m = rich_chain(2, 31)
    F, g, _ = adjoint.gradient(m, 0.2, steps, 4, 0.0, "+y", 1, "X")
    got = adjoint.flatten(m, g)
    ref = dense_fd_gradient(m, 0.2, steps, "+y", 1, "X")
    assert np.abs(got - ref).max() < 1e-8


def test_exact_third_order_gradient_equals_dense_trotter_derivative():
    """Order 3 (negative time fractions: gates that run the dissipators backwards)."""
    m = rich_chain(4, 35)
    F, g, _ = adjoint.gradient(m, 0.1, 2, 16, 0.0, "+x", 2, "Y", order=3)
    got = adjoint.flatten(m, g)
    ref = dense_fd_gradient(m, 0.1, 2, "+x", 2, "Y", order=3)
    assert np.abs(got - ref).max() < 1e-8, np.abs(got - ref).max()


def test_tau_derivative_and_scaling_identity():
    """d F / d tau against central differences of the dense Trotter product in
    tau, and sum_theta theta dF/dtheta = tau dF/dtau (F depends on tau theta)."""
    m = rich_chain(4, 38)
    tau, steps, h = 0.1, 3, 1e-6
    F, g, _ = adjoint.gradient(m, tau, steps, 16, 0.0, "+x", 1, "Z")
    fd = (dense_expectation(m, tau + h, steps, "+x", 1, "Z") - dense_expectation(m, tau - h, steps, "+x", 1, "Z")) / (2 * h)
    assert abs(g["tau"][0] - fd) < 1e-8
    lhs = sum(m[k][i] * g[k][i] for k, i in adjoint.parameter_list(m))
    assert abs(lhs - tau * g["tau"][0]) < 1e-12 * max(1.0, abs(lhs))


def test_renyi2_gradient_equals_dense_trotter_derivative():
    """dS_2/dtheta (Eq. S_2): co-state from rho itself; against dense differences of
    S_2 computed from the density matrix."""
    m = rich_chain(4, 39)
    tau, steps, h = 0.1, 3, 1e-6

    def dense_S2(model):
        v = dense.trotter_evolve(dense.product_vector("+x", 4), model, tau, steps)
        return dense.renyi2(v, 4)

    S2, g, _ = adjoint.gradient_renyi2(m, tau, steps, 16, 0.0, "+x")
    assert abs(S2 - dense_S2(m)) < 1e-12
    ref = []
    for key, idx in adjoint.parameter_list(m):
        vals = []
        for sgn in (1.0, -1.0):
            mm = {k: (np.array(v, dtype=float) if k in adjoint.SITE_KEYS + adjoint.BOND_KEYS else v)
                  for k, v in m.items()}
            mm[key][idx] += sgn * h
            vals.append(dense_S2(mm))
        ref.append((vals[0] - vals[1]) / (2 * h))
    assert np.abs(adjoint.flatten(m, g) - np.array(ref)).max() < 1e-8


def test_renyi2_costate_brute_force():
    """<mu, v> = the derivative of S_2 at rho along v (central differences of the
    dense S_2 of rho + eps v), v Hermitian with nonzero trace: the trace term,
    which exact trace-preserving dynamics never sees, is pinned here."""
    m = rich_chain(3, 46)
    mps, _, _ = adjoint.forward_record(m, 0.1, 2, 64, 0.0, "+x")
    mu = adjoint.costate_renyi2(mps, 64, 0.0)
    r = dense.mps_to_vector(mps.A)
    rng = np.random.default_rng(46)
    v = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    v = 0.5 * (v + dense.adjoint(v, 3))
    assert abs(dense.trace(v, 3)) > 0.1
    eps = 1e-6
    ref = (dense.renyi2(r + eps * v, 3) - dense.renyi2(r - eps * v, 3)) / (2 * eps)
    got = np.dot(dense.mps_to_vector(mu.A), v)
    assert abs(got.imag) < 1e-10
    assert abs(got.real - ref) < 1e-7 * max(1.0, abs(ref))


@pytest.mark.parametrize("bond", [0, 1, 2])
def test_osee_costate_brute_force(bond):
    """<mu, v> = the derivative of the OSEE (Eq. OSEE) at rho along a Hermitian v:
    central differences of the dense OSEE (the SVD of the full vector)."""
    m = rich_chain(4, 47)
    mps, _, _ = adjoint.forward_record(m, 0.1, 3, 64, 0.0, "+x")
    S, mu = adjoint.costate_osee(mps, bond)
    r = dense.mps_to_vector(mps.A)
    assert abs(S - dense.osee(r, 4, bond)) < 1e-12
    rng = np.random.default_rng(bond)
    v = rng.standard_normal(256) + 1j * rng.standard_normal(256)
    v = 0.5 * (v + dense.adjoint(v, 4))
    v = v / np.linalg.norm(v) * np.linalg.norm(r)
    f = lambda e: dense.osee(r + e * v, 4, bond)  # noqa: E731
    eps = 1e-4  # fourth-order central stencil: the smallest weights (p ~ 1e-8) bend S fast
    ref = (8.0 * (f(eps) - f(-eps)) - (f(2 * eps) - f(-2 * eps))) / (12 * eps)
    got = np.dot(dense.mps_to_vector(mu.A), v)
    assert abs(got.imag) < 1e-9
    assert abs(got.real - ref) < 1e-8 * max(1.0, abs(ref))


@pytest.mark.parametrize("bond", [0, 1, 2])
def test_osee_gradient_equals_dense_trotter_derivative(bond):
    """dOSEE/dtheta across each bond of a 4-qubit chain against dense
    differences of the OSEE of the dense Trotter evolution."""
    m = rich_chain(4, 48)
    tau, steps, h = 0.1, 3, 1e-6

    def dense_osee(model):
        v = dense.trotter_evolve(dense.product_vector("+x", 4), model, tau, steps)
        return dense.osee(v, 4, bond)

    S, g, _ = adjoint.gradient_osee(m, tau, steps, 16, 0.0, "+x", bond)
    assert abs(S - dense_osee(m)) < 1e-12
    ref = []
    for key, idx in adjoint.parameter_list(m):
        vals = []
        for sgn in (1.0, -1.0):
            mm = {k: (np.array(v, dtype=float) if k in adjoint.SITE_KEYS + adjoint.BOND_KEYS else v)
                  for k, v in m.items()}
            mm[key][idx] += sgn * h
            vals.append(dense_osee(mm))
        ref.append((vals[0] - vals[1]) / (2 * h))
    assert np.abs(adjoint.flatten(m, g) - np.array(ref)).max() < 1e-7


@pytest.mark.parametrize("objective", ["renyi2", "osee"])
def test_truncated_entropy_gradient_approaches_the_dense_derivative(objective):
    """S_2 and the OSEE across bond (2, 3) of a 6-qubit chain: with truncation
    the co-state gradient approximates the dense Trotter derivative, the error
    falls as chi grows and vanishes at the exact chi (measured 1e-2 .. 7e-10
    for S_2, 3e-3 .. 4e-10 for the OSEE)."""
    m = rich_chain(6, 11)
    tau, steps, h = 0.1, 4, 1e-6

    def f(model):
        v = dense.trotter_evolve(dense.product_vector("+x", 6), model, tau, steps)
        return dense.renyi2(v, 6) if objective == "renyi2" else dense.osee(v, 6, 2)

    ref = []
    for key, idx in adjoint.parameter_list(m):
        vals = []
        for sgn in (1.0, -1.0):
            mm = {k: (np.array(v, dtype=float) if k in adjoint.SITE_KEYS + adjoint.BOND_KEYS else v)
                  for k, v in m.items()}
            mm[key][idx] += sgn * h
            vals.append(f(mm))
        ref.append((vals[0] - vals[1]) / (2 * h))
    ref = np.array(ref)
    errs = []
    for chi in (4, 8, 16, 64):
        if objective == "renyi2":
            _, g, _ = adjoint.gradient_renyi2(m, tau, steps, chi, 0.0, "+x")
        else:
            _, g, _ = adjoint.gradient_osee(m, tau, steps, chi, 0.0, "+x", 2)
        errs.append(np.abs(adjoint.flatten(m, g) - ref).max())
    assert errs[-1] < 1e-8
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[1] < 0.05 * np.abs(ref).max()
