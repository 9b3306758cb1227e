"""Parity of the adjoint gradient (lmpo_grad_*) with the oracle's
(oracle/adjoint.py) on the same seeded models, and the state it leaves.

Both sides make the same truncation decisions (the co-state's included), so
the gradients agree to FP64 round-off; the bar is 1e-9 relative to the largest
derivative (the observables of the step itself agree to ~1e-13)."""
import numpy as np
import pytest

import workloads
from oracle import adjoint

pytestmark = pytest.mark.gpu


def Gradient(chain, n_steps, co_chi=0, co_cut=-1.0, series=False, keep_gates=False, complex_costate=False):
    from paper_2203_05871_amd import Gradient as G

    return G(chain, n_steps, co_chi, co_cut, series, keep_gates, complex_costate)


def _chain(m, tau, chi, cutoff, init, precision="fp64", order=2, force_trace=True):
    from paper_2203_05871_amd import Chain

    return Chain(m, tau, chi, cutoff, precision, init, force_trace=force_trace, order=order, device="cuda:0")


def _compare(m, tau, steps, chi, cutoff, init, site, pauli, precision="fp64", order=2, force_trace=True,
             co_chi=None, co_cut=None, paulis=None):
    print(f"gradient case: N={m['N']} bonds={len(m['bonds'])} chi={chi} cutoff={cutoff} steps={steps} "
          f"order={order} {precision} <{paulis or f'{pauli}_{site}'}> co-state {co_chi} {co_cut}", flush=True)
    ch = _chain(m, tau, chi, cutoff, init, precision, order, force_trace)
    F, g = ch.gradient(steps, site, pauli, paulis, co_chi or 0, -1.0 if co_cut is None else co_cut)
    ch.close()
    Fo, go, _ = adjoint.gradient(m, tau, steps, chi, cutoff, init, site, pauli, order=order,
                                 force_trace=force_trace, costate_chi_max=co_chi, costate_cutoff=co_cut,
                                 paulis=paulis)
    got = np.concatenate([g[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS + ("tau",)])
    ref = np.concatenate([adjoint.flatten(m, go).real, go["tau"].real])
    assert abs(F - Fo) < 1e-11
    scale = max(1.0, np.abs(ref).max())
    err = np.abs(got - ref).max() / scale
    print(f"  F = {F.real:.12f}, max |grad - oracle| / scale = {err:.2e}", flush=True)
    assert err < 1e-9, err
    return got, ref


def test_exact_chain_gradient():
    """4 qubits, no truncation: the oracle's value is the dense Trotter derivative."""
    _compare(workloads.random_model(4, 7), 0.1, 3, 16, 0.0, "+x", 1, "Z")


def test_truncated_chain_gradient():
    _compare(workloads.random_model(8, 3), 0.1, 4, 8, 1e-10, "+x", 3, "X")


def test_truncated_chain_gradient_without_trace_forcing():
    _compare(workloads.random_model(7, 4), 0.1, 3, 6, 1e-12, "+y", 6, "Y", force_trace=False)


def test_ladder_gradient_through_swap_network():
    """2 x 3 ladder on the zigzag path: rungs (2r, 2r+1), legs (s, s+2) through SWAP gates."""
    lad = workloads.ladder_model(3)
    m = workloads.random_model(6, 5, bonds=lad["bonds"])
    _compare(m, 0.1, 3, 16, 1e-12, "+z", 2, "X")


def test_ladder_gradient_with_own_costate_truncation():
    """The co-state truncated harder than the state (its own chi_max and cutoff)."""
    lad = workloads.ladder_model(4)
    m = workloads.random_model(8, 6, bonds=lad["bonds"])
    _compare(m, 0.1, 3, 16, 1e-12, "+x", 3, "Z", co_chi=6, co_cut=1e-6)


def test_correlator_gradient():
    """<Z_2 Z_5> (Eq. 2Qdef's correlator): F through the two-site measurement."""
    _compare(workloads.random_model(8, 14), 0.1, 4, 8, 1e-10, "+x", None, None, paulis="IIZIIZII")


def test_pauli_string_gradient_on_a_ladder():
    """A three-factor string: F through the transition density of o and rho_T."""
    lad = workloads.ladder_model(3)
    m = workloads.random_model(6, 15, bonds=lad["bonds"])
    _compare(m, 0.1, 3, 16, 1e-12, "+z", None, None, paulis="XIZIIY")


@pytest.mark.parametrize("ladder", [False, True])
def test_connected_correlator_gradient(ladder):
    """<Z_0 Z_j> - <Z_0><Z_j> (the paper's connected function): one backward pass
    from the four-term co-state, against the oracle's."""
    if ladder:
        m = workloads.random_model(8, 18, bonds=workloads.ladder_model(4)["bonds"])
        args = (0.1, 3, 16, 1e-12, "+z")
    else:
        m = workloads.random_model(8, 19)
        args = (0.1, 4, 8, 1e-10, "+x")
    print(f"gradient case: connected <Z_0 Z_7>, N=8, ladder={ladder}", flush=True)
    tau, steps, chi, cut, init = args
    ch = _chain(m, tau, chi, cut, init)
    G = Gradient(ch, steps)
    C, g = G.run_connected(0, 7, "ZZ")
    G.close()
    ch.close()
    Co, go, _ = adjoint.gradient_connected(m, tau, steps, chi, cut, init, 0, 7, "ZZ")
    got = np.concatenate([g[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS])
    ref = adjoint.flatten(m, go).real
    err = np.abs(got - ref).max() / max(1.0, np.abs(ref).max())
    print(f"  C = {C.real:.12f}, max |grad - oracle| / scale = {err:.2e}", flush=True)
    assert abs(C - Co) < 1e-11
    assert err < 1e-9


def test_connected_correlator_needs_room_for_its_costate():
    """Four product terms start the co-state at bond 4: a co-state chi_max of 3
    is refused before any GPU work on it."""
    from paper_2203_05871_amd import LmpoError

    ch = _chain(workloads.random_model(5, 20), 0.1, 8, 1e-10, "+x")
    before = [ch.get_site(k) for k in range(5)]
    G = Gradient(ch, 1, 3, -1.0)
    with pytest.raises(LmpoError, match="co-state"):
        G.run_connected(0, 4, "ZZ")
    G.close()
    assert all(np.array_equal(a, ch.get_site(k)) for k, a in enumerate(before))  # the state did not move
    ch.close()


@pytest.mark.parametrize("steps", [1, 3])
def test_two_qubit_gradient(steps):
    """N = 2: one bond, empty environments; one step and several."""
    _compare(workloads.random_model(2, 32), 0.2, steps, 4, 0.0, "+y", 1, "X")


def test_gradient_at_the_smallest_chi():
    """chi_max = 2 for the state and the co-state (the co-state starts at bond 2)."""
    _compare(workloads.random_model(5, 33), 0.1, 3, 2, 1e-12, "+x", 2, "Z")


def test_fourth_order_gradient():
    _compare(workloads.random_model(5, 8), 0.1, 2, 16, 1e-12, "+x", 0, "Z", order=4)


def test_third_order_gradient():
    _compare(workloads.random_model(6, 36), 0.1, 3, 8, 1e-10, "+x", 3, "Y", order=3)


def test_fp32_contraction_form_gradient():
    """The state in the FP32-contraction form (the co-state stays real FP64): the
    derivatives follow the oracle's to the FP32 form's tolerance."""
    m = workloads.random_model(8, 22)
    print("gradient case: N=8 chi=8 fp32 contraction, <Z_4>", flush=True)
    ch = _chain(m, 0.1, 8, 1e-10, "+x", precision="fp32")
    F, g = ch.gradient(4, 4, "Z")
    ch.close()
    Fo, go, _ = adjoint.gradient(m, 0.1, 4, 8, 1e-10, "+x", 4, "Z")
    got = np.concatenate([g[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS])
    ref = adjoint.flatten(m, go).real
    err = np.abs(got - ref).max() / max(1.0, np.abs(ref).max())
    print(f"  F error {abs(F - Fo):.2e}, max |grad - oracle| / scale = {err:.2e}", flush=True)
    assert abs(F - Fo) < 1e-5
    assert err < 1e-5


def test_real_form_gradient():
    _compare(workloads.random_model(8, 9), 0.1, 4, 8, 1e-10, "+x", 4, "Z", precision="real")


def test_gradient_leaves_the_state_of_the_forward_run():
    """After run() the state equals that of lmpo_evolve_step over the same steps
    (site tensors bit for bit, discarded weight, step count), and a second run
    continues from there."""
    m = workloads.random_model(6, 11)
    a = _chain(m, 0.1, 8, 1e-10, "+x")
    b = _chain(m, 0.1, 8, 1e-10, "+x")
    a.gradient(3, 2, "Z")
    b.evolve(3)
    for k in range(6):
        assert np.array_equal(a.get_site(k), b.get_site(k))
    assert a.discarded_weight() == b.discarded_weight()
    assert a.centre() == b.centre()
    F, _ = a.gradient(2, 2, "Z")
    b.evolve(2)
    assert F == b.measure_1q([2], "Z")[0]
    for k in range(6):
        assert np.array_equal(a.get_site(k), b.get_site(k))
    a.close()
    b.close()


def test_autograd_function_matches_the_c_abi_and_the_oracle():
    """torch.autograd through paper_2203_05871_amd.expectation: .grad of every
    parameter tensor equals the C ABI's gradient (same run) and the oracle's."""
    import torch

    from paper_2203_05871_amd import expectation

    m = workloads.random_model(6, 12)
    spec = {"N": 6, "bonds": m["bonds"], "tau": 0.1, "steps": 3, "chi_max": 8, "cutoff": 1e-10, "site": 2,
            "pauli": "X", "init": "+x"}
    params = {k: torch.tensor(m[k], dtype=torch.float64, requires_grad=True)
              for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS}
    F = expectation(spec, params)
    (2.0 * F).backward()
    ch = _chain(m, 0.1, 8, 1e-10, "+x")
    Fc, gc = ch.gradient(3, 2, "X")
    ch.close()
    assert F.item() == Fc.real
    _, go, _ = adjoint.gradient(m, 0.1, 3, 8, 1e-10, "+x", 2, "X")
    for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS:
        assert np.array_equal(params[k].grad.numpy(), 2.0 * gc[k])
        assert np.abs(params[k].grad.numpy() - 2.0 * go[k].real).max() < 1e-9


@pytest.mark.parametrize("precision", ["real", "fp64"])
def test_autograd_renyi2(precision):
    """torch.autograd through paper_2203_05871_amd.renyi2: S_2 and .grad equal
    the workspace's run_renyi2 bit for bit and the oracle's gradient."""
    import torch

    from paper_2203_05871_amd import renyi2

    m = workloads.random_model(6, 45)
    spec = {"N": 6, "bonds": m["bonds"], "tau": 0.1, "steps": 3, "chi_max": 8, "cutoff": 1e-10, "init": "+x",
            "precision": precision}
    params = {k: torch.tensor(m[k], dtype=torch.float64, requires_grad=True)
              for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS}
    S2 = renyi2(spec, params)
    (-3.0 * S2).backward()
    ch = _chain(m, 0.1, 8, 1e-10, "+x", precision=precision)
    G = Gradient(ch, 3, series=True, complex_costate=precision != "real")
    Sc, gc = G.run_renyi2()
    G.close()
    ch.close()
    assert S2.item() == Sc
    _, go, _ = adjoint.gradient_renyi2(m, 0.1, 3, 8, 1e-10, "+x")
    for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS:
        assert np.array_equal(params[k].grad.numpy(), -3.0 * gc[k])
        assert np.abs(params[k].grad.numpy() + 3.0 * go[k].real).max() < 1e-9


def test_autograd_osee():
    """torch.autograd through paper_2203_05871_amd.osee: the value and .grad equal
    the workspace's run_osee bit for bit and the oracle's gradient."""
    import torch

    from paper_2203_05871_amd import osee

    m = workloads.random_model(6, 52)
    spec = {"N": 6, "bonds": m["bonds"], "tau": 0.1, "steps": 3, "chi_max": 8, "cutoff": 1e-10, "init": "+x",
            "bond": 2}
    params = {k: torch.tensor(m[k], dtype=torch.float64, requires_grad=True)
              for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS}
    S = osee(spec, params)
    (0.5 * S).backward()
    ch = _chain(m, 0.1, 8, 1e-10, "+x", precision="real")
    G = Gradient(ch, 3)
    Sc, gc = G.run_osee(2)
    G.close()
    ch.close()
    assert S.item() == Sc
    _, go, _ = adjoint.gradient_osee(m, 0.1, 3, 8, 1e-10, "+x", 2)
    for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS:
        assert np.array_equal(params[k].grad.numpy(), 0.5 * gc[k])
        assert np.abs(params[k].grad.numpy() - 0.5 * go[k].real).max() < 1e-9


@pytest.mark.timeout(600)
@pytest.mark.parametrize("objective", ["z15", "connected_z0_z15"])
def test_ladder2x8_configured_objectives_against_the_oracle(objective):
    """Both objectives of the ladder's differentiation workload, <s^z_15> and
    the connected <s^z_0 s^z_15>_c, on the 2 x 8 ladder (chi_max 128, cutoff
    1e-12, tau 0.05, from +z) after its first 16 steps: all 6N + 2 n_bonds =
    140 parameter derivatives and d/dtau against the oracle's, element by
    element, to 1e-9 of the largest derivative (no absolute floor).  The
    connected correlator's derivative dC = dF_ij - F_j dF_i - F_i dF_j is a
    difference of terms of the size of dF_ij (about 1 here, with F_j = <s^z_15>
    within 1e-11 of 1) that cancel down to about 1e-5, so its round-off is set
    by the terms: its bar is 1e-9 of the larger of its own and dF_ij's largest
    derivative, dF_ij from the same GPU run's Pauli string Z_0 Z_15."""
    m, run = workloads.ladder2x8()
    tau, chi, cut, init = run["tau"], run["chi_max"], run["cutoff"], run["init"]
    n = 16
    print(f"gradient case: 2x8 ladder, chi 128, first {n} steps, {objective}", flush=True)
    ch = _chain(m, tau, chi, cut, init)
    G = Gradient(ch, n)
    if objective == "z15":
        F, g = G.run(15, "Z")
        Fo, go, _ = adjoint.gradient(m, tau, n, chi, cut, init, 15, "Z")
    else:
        F, g = G.run_connected(0, 15, "ZZ")
        Fo, go, _ = adjoint.gradient_connected(m, tau, n, chi, cut, init, 0, 15, "ZZ")
    G.close()
    ch.close()
    got = np.concatenate([g[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS + ("tau",)])
    ref = np.concatenate([adjoint.flatten(m, go).real, go["tau"].real])
    assert len(got) == 6 * m["N"] + 2 * len(m["bonds"]) + 1 == 141
    scale = np.abs(ref).max()
    if objective != "z15":
        ch = _chain(m, tau, chi, cut, init)
        _, gij = ch.gradient(n, paulis="Z" + "I" * 14 + "Z")
        ch.close()
        term = max(float(np.abs(v).max()) for v in gij.values())
        print(f"  largest derivative of F_ij = <Z_0 Z_15>: {term:.3e}", flush=True)
        scale = max(scale, term)
    err = np.abs(got - ref).max() / scale
    print(f"  F = {F.real:.15f} (oracle {Fo.real:.15f}), largest derivative {np.abs(ref).max():.3e}, "
          f"bar scale {scale:.3e}, max |grad - oracle| / scale = {err:.2e}", flush=True)
    assert abs(F - Fo) < 1e-12
    assert err < 1e-9, err


@pytest.mark.timeout(300)
def test_ladder2x8_full_size_gradient():
    """The 2 x 8 ladder at full size (N=16, chi_max 128, 40 steps): the oracle
    cannot run it in seconds, so the check is what holds at any size.  F equals
    the forward run's bit for bit; the adjoint derivatives agree with central
    differences of the GPU forward run (h = 1e-5) to 5e-4 of the largest
    derivative (measured 4e-5: the truncated forward is only piecewise smooth,
    its kept ranks move between +h and -h, and the co-state is itself
    truncated at chi 128)."""
    m, run = workloads.ladder2x8()
    tau, steps, chi, cut, init = run["tau"], run["steps"], run["chi_max"], run["cutoff"], run["init"]
    print("gradient case: 2x8 ladder, chi 128, 40 steps, <Z_1>", flush=True)

    def forward(model):
        c = _chain(model, tau, chi, cut, init)
        c.evolve(steps)
        v = c.measure_1q([1], "Z")[0]
        c.close()
        return v

    ch = _chain(m, tau, chi, cut, init)
    F, g = ch.gradient(steps, 1, "Z")
    ch.close()
    assert F == forward(m)
    gmax = max(np.abs(v).max() for v in g.values())
    # F depends on the parameters only through tau theta: sum theta dF/dtheta = tau dF/dtau
    lhs = sum(float(np.dot(np.asarray(m[k], dtype=float), g[k])) for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS)
    print(f"  sum theta dF/dtheta = {lhs:.12e}, tau dF/dtau = {tau * g['tau'][0]:.12e}", flush=True)
    assert abs(lhs - tau * g["tau"][0]) < 1e-9 * max(1.0, abs(lhs))
    for key, idx in (("hx", 0), ("J", 5)):
        vals = []
        for sgn in (1.0, -1.0):
            mm = {k: (np.array(v, dtype=float) if k != "bonds" and isinstance(v, np.ndarray) else v)
                  for k, v in m.items()}
            mm[key][idx] += sgn * 1e-5
            vals.append(forward(mm).real)
        fd = (vals[0] - vals[1]) / 2e-5
        print(f"  {key}[{idx}]: adjoint {g[key][idx]:.8e} central difference {fd:.8e}", flush=True)
        assert abs(g[key][idx] - fd) < 5e-4 * gmax


@pytest.mark.timeout(300)
@pytest.mark.parametrize("objective", ["renyi2", "osee"])
def test_ladder2x8_full_size_entropy_gradient(objective):
    """S_2 and the OSEE across the middle bond (7, 8) of the zigzag path on the
    2 x 8 ladder at full size (real-arithmetic form, chi 128, 40 steps): the
    value equals the forward run's, sum theta dS/dtheta = tau dS/dtau, and the
    adjoint derivatives on the drive, a decay rate and a leg coupling agree
    with central differences of the GPU forward (h = 1e-5) to 5e-4 of the
    largest derivative (the truncated forward is only piecewise smooth)."""
    m, run = workloads.ladder2x8()
    tau, steps, chi, cut, init = run["tau"], run["steps"], run["chi_max"], run["cutoff"], run["init"]
    print(f"gradient case: 2x8 ladder, chi 128, 40 steps, real form, {objective}", flush=True)

    def value(c):
        return c.renyi2() if objective == "renyi2" else c.osee(7)

    def forward(model):
        c = _chain(model, tau, chi, cut, init, precision="real")
        c.evolve(steps)
        v = value(c)
        c.close()
        return v

    ch = _chain(m, tau, chi, cut, init, precision="real")
    G = Gradient(ch, steps, series=objective == "renyi2")
    S, g = G.run_renyi2() if objective == "renyi2" else G.run_osee(7)
    G.close()
    ch.close()
    assert abs(S - forward(m)) < 1e-12
    gmax = max(np.abs(v).max() for v in g.values())
    lhs = sum(float(np.dot(np.asarray(m[k], dtype=float), g[k])) for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS)
    print(f"  S = {S:.12f}, sum theta dS/dtheta = {lhs:.12e}, tau dS/dtau = {tau * g['tau'][0]:.12e}", flush=True)
    assert abs(lhs - tau * g["tau"][0]) < 1e-9 * max(1.0, abs(lhs))
    for key, idx in (("hx", 0), ("g0", 0), ("J", 5)):
        vals = []
        for sgn in (1.0, -1.0):
            mm = {k: (np.array(v, dtype=float) if k != "bonds" and isinstance(v, np.ndarray) else v)
                  for k, v in m.items()}
            mm[key][idx] += sgn * 1e-5
            vals.append(forward(mm))
        fd = (vals[0] - vals[1]) / 2e-5
        print(f"  {key}[{idx}]: adjoint {g[key][idx]:.8e} central difference {fd:.8e} (max {gmax:.3e})", flush=True)
        assert abs(g[key][idx] - fd) < 5e-4 * gmax


def test_ladder2x3_exact_gradient_against_dense_trotter():
    """The 2 x 3 ladder at chi 64 (no truncation: 4^3 is the largest rank): the
    GPU derivatives against central differences of the dense Trotter product on
    the full 4^6 vector (no MPS, no co-state), all 50 parameters."""
    from oracle import dense
    from oracle import model as lm

    lad = workloads.ladder_model(3)
    m = workloads.random_model(6, 16, bonds=lad["bonds"])
    tau, steps = 0.1, 3
    print("gradient case: 2x3 ladder, chi 64, exact, <Z_3> vs dense Trotter", flush=True)
    ch = _chain(m, tau, 64, 0.0, "+x")
    F, g = ch.gradient(steps, 3, "Z")
    ch.close()
    got = np.concatenate([g[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS])

    def dense_F(model):
        v = dense.trotter_evolve(dense.product_vector("+x", 6), model, tau, steps)
        return dense.expect(v, 6, {3: lm.PAULI["Z"]}).real

    assert abs(F.real - dense_F(m)) < 1e-12
    ref = []
    for key, idx in adjoint.parameter_list(m):
        vals = []
        for sgn in (1.0, -1.0):
            mm = {k: (np.array(v, dtype=float) if k in adjoint.SITE_KEYS + adjoint.BOND_KEYS else v)
                  for k, v in m.items()}
            mm[key][idx] += sgn * 1e-6
            vals.append(dense_F(mm))
        ref.append((vals[0] - vals[1]) / 2e-6)
    err = np.abs(got - np.array(ref)).max()
    print(f"  max |grad - dense central difference| = {err:.2e}", flush=True)
    assert err < 1e-8


def test_gradient_error_paths():
    """Refused before any work: Hermitisation, a co-state chi below 2, zero steps,
    malformed strings (the state is left where it was)."""
    from paper_2203_05871_amd import LmpoError

    m = workloads.random_model(4, 21)
    from paper_2203_05871_amd import Chain

    h = Chain(m, 0.1, 8, 1e-10, "fp64", "+x", hermitian_every=2, device="cuda:0")
    with pytest.raises(LmpoError, match="Hermitian"):
        Gradient(h, 2)
    h.close()
    ch = _chain(m, 0.1, 8, 1e-10, "+x")
    with pytest.raises(LmpoError, match="chi_max"):
        Gradient(ch, 2, 1, -1.0)
    with pytest.raises(LmpoError, match="n_steps"):
        Gradient(ch, 0)
    G = Gradient(ch, 2)
    before = [ch.get_site(k) for k in range(4)]
    for bad in ("IZ", "IIII", "IZQI"):
        with pytest.raises(LmpoError, match="paulis"):
            G.run_string(bad)
    with pytest.raises(LmpoError, match="distinct"):
        G.run_connected(1, 1, "ZZ")
    assert all(np.array_equal(a, ch.get_site(k)) for k, a in enumerate(before))
    G.close()
    ch.close()


@pytest.mark.parametrize("ladder", [False, True])
def test_series_gradient(ladder):
    """J = sum_k w_k <O>(t_k) over several output steps: each output's source
    enters the co-state (MPS sum + compression) when the backward pass reaches
    it; against the oracle's series gradient."""
    if ladder:
        m = workloads.random_model(6, 26, bonds=workloads.ladder_model(3)["bonds"])
        tau, steps, chi, cut, init, paulis, outs, ws = 0.1, 4, 16, 1e-12, "+z", "XIZIIY", [2, 3], [1.5, -0.4]
    else:
        m = workloads.random_model(8, 27)
        tau, steps, chi, cut, init, paulis, outs, ws = 0.1, 5, 8, 1e-10, "+x", "IIZIIIII", [1, 2, 4], [0.3, -1.0, 0.7]
    print(f"gradient case: series {paulis} at {outs}, ladder={ladder}", flush=True)
    ch = _chain(m, tau, chi, cut, init)
    G = Gradient(ch, steps, series=True)
    F, g = G.run_series(paulis, outs, ws)
    G.close()
    ch.close()
    Fo, go, _ = adjoint.gradient_series(m, tau, steps, chi, cut, init, paulis, outs, ws)
    got = np.concatenate([g[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS])
    ref = adjoint.flatten(m, go).real
    err = np.abs(got - ref).max() / max(1.0, np.abs(ref).max())
    print(f"  F_k error {np.abs(F - Fo).max():.2e}, max |grad - oracle| / scale = {err:.2e}", flush=True)
    assert np.abs(F - Fo).max() < 1e-11
    assert err < 1e-9


def test_series_with_one_final_output_is_the_plain_gradient():
    m = workloads.random_model(6, 28)
    a = _chain(m, 0.1, 8, 1e-10, "+x")
    b = _chain(m, 0.1, 8, 1e-10, "+x")
    Ga, Gb = Gradient(a, 3, series=True), Gradient(b, 3)
    Fa, ga = Ga.run_series("IIZIII", [3], [1.0])
    Fb, gb = Gb.run_string("IIZIII")
    assert Fa[0] == Fb
    for k in ga:
        assert np.array_equal(ga[k], gb[k])
    Ga.close()
    Gb.close()
    a.close()
    b.close()


def test_series_argument_checks():
    from paper_2203_05871_amd import LmpoError

    ch = _chain(workloads.random_model(4, 29), 0.1, 8, 1e-10, "+x")
    G = Gradient(ch, 3)
    with pytest.raises(LmpoError, match="LMPO_GRAD_SERIES"):
        G.run_series("IZII", [3], [1.0])
    G.close()
    G = Gradient(ch, 3, series=True)
    before = [ch.get_site(k) for k in range(4)]
    for outs in ([0], [4], [2, 2], [3, 1]):
        with pytest.raises(LmpoError, match="out_steps"):
            G.run_series("IZII", outs, [1.0] * len(outs))
    assert all(np.array_equal(x, ch.get_site(k)) for k, x in enumerate(before))
    G.close()
    ch.close()


def test_autograd_time_series_least_squares():
    """loss = sum_k (F_k - d_k)^2 over a time series through
    paulis-valued expectation_series: .grad equals the oracle's series gradient
    with weights 2 (F_k - d_k)."""
    import torch

    from paper_2203_05871_amd import expectation_series

    m = workloads.random_model(6, 30)
    outs, d = [1, 2, 4], np.array([0.1, -0.2, 0.3])
    spec = {"N": 6, "bonds": m["bonds"], "tau": 0.1, "steps": 4, "chi_max": 8, "cutoff": 1e-10, "init": "+x",
            "paulis": "IIZIII", "out_steps": outs}
    params = {k: torch.tensor(m[k], dtype=torch.float64, requires_grad=True)
              for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS}
    F = expectation_series(spec, params)
    loss = ((F - torch.tensor(d)) ** 2).sum()
    loss.backward()
    Fo, _, _ = adjoint.gradient_series(m, 0.1, 4, 8, 1e-10, "+x", "IIZIII", outs, [1.0, 1.0, 1.0])
    assert np.abs(F.detach().numpy() - Fo.real).max() < 1e-11
    w = 2.0 * (F.detach().numpy() - d)
    _, go, _ = adjoint.gradient_series(m, 0.1, 4, 8, 1e-10, "+x", "IIZIII", outs, w)
    ref = adjoint.flatten(m, go).real
    got = np.concatenate([params[k].grad.numpy() for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS])
    err = np.abs(got - ref).max() / max(1.0, np.abs(ref).max())
    print(f"autograd series: max |grad - oracle| / scale = {err:.2e}", flush=True)
    assert err < 1e-9


@pytest.mark.parametrize("series", [False, True])
def test_kept_gate_snapshots_give_the_replayed_result(series):
    """LMPO_GRAD_KEEP_GATES (no replay in the backward pass) gives the replayed
    workspace's results bit for bit, on a ladder through the SWAP network."""
    m = workloads.random_model(6, 34, bonds=workloads.ladder_model(3)["bonds"])
    out = []
    for keep in (False, True):
        ch = _chain(m, 0.1, 16, 1e-12, "+x")
        G = Gradient(ch, 3, series=series, keep_gates=keep)
        F, g = G.run_series("IZIIXI", [1, 3], [0.5, 1.0]) if series else G.run_string("IZIIXI")
        G.close()
        sites = [ch.get_site(k) for k in range(6)]
        ch.close()
        out.append((F, g, sites))
    (Fa, ga, sa), (Fb, gb, sb) = out
    assert np.array_equal(np.atleast_1d(Fa), np.atleast_1d(Fb))
    for k in ga:
        assert np.array_equal(ga[k], gb[k])
    assert all(np.array_equal(x, y) for x, y in zip(sa, sb))


def test_costate_svd_tolerance_knob():
    """A looser Jacobi threshold on the co-state changes the derivatives only at
    about that threshold; factors below 1 are refused."""
    from paper_2203_05871_amd import LmpoError

    m = workloads.random_model(8, 37)
    out = []
    for fac in (32.0, 1e4):
        ch = _chain(m, 0.1, 8, 1e-10, "+x")
        G = Gradient(ch, 3)
        G.set_costate_svd_tolerance(fac)
        out.append(G.run(3, "Z")[1])
        if fac == 32.0:
            with pytest.raises(LmpoError, match="tolerance"):
                G.set_costate_svd_tolerance(0.5)
        G.close()
        ch.close()
    a = np.concatenate([out[0][k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS])
    b = np.concatenate([out[1][k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS])
    assert np.abs(a - b).max() < 1e-8 * max(1.0, np.abs(a).max())


@pytest.mark.parametrize("case", ["exact_chain", "truncated_ladder", "costate_truncated", "complex_fp64",
                                  "complex_fp32"])
def test_renyi2_gradient(case):
    """dS_2/dtheta for S_2 = -ln(tr rho^2 / (tr rho)^2) (Eq. S_2): the co-state
    starts from the state itself; against the oracle (which forms it from the
    density matrix's transpose) and, all parameters and tau together, the
    scaling identity sum theta dS_2/dtheta = tau dS_2/dtau."""
    co_chi = co_cut = None
    if case == "exact_chain":
        m, tau, steps, chi, cut, init = workloads.random_model(5, 41), 0.1, 3, 32, 0.0, "+x"
    else:
        lad = workloads.ladder_model(4)
        m = workloads.random_model(8, 42, bonds=lad["bonds"])
        tau, steps, chi, cut, init = 0.1, 4, 8, 1e-10, "+z"
        if case == "costate_truncated":
            co_chi, co_cut = 8, 1e-6
    prec = {"complex_fp64": "fp64", "complex_fp32": "fp32"}.get(case, "real")
    tol = 1e-5 if prec == "fp32" else 1e-9
    print(f"gradient case: renyi2 {case} N={m['N']} chi={chi} co-state {co_chi} {co_cut}", flush=True)
    ch = _chain(m, tau, chi, cut, init, precision=prec)
    G = Gradient(ch, steps, co_chi or 0, -1.0 if co_cut is None else co_cut, series=True,
                 complex_costate=prec != "real")
    S2, g = G.run_renyi2()
    G.close()
    assert abs(ch.renyi2() - S2) < 1e-13  # the state is left at T
    ch.close()
    So, go, _ = adjoint.gradient_renyi2(m, tau, steps, chi, cut, init, costate_chi_max=co_chi,
                                        costate_cutoff=co_cut)
    got = np.concatenate([g[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS + ("tau",)])
    ref = np.concatenate([adjoint.flatten(m, go).real, go["tau"].real])
    err = np.abs(got - ref).max() / max(1.0, np.abs(ref).max())
    print(f"  S_2 = {S2:.12f} (oracle {So:.12f}), max |grad - oracle| / scale = {err:.2e}", flush=True)
    assert abs(S2 - So) < (tol if prec == "fp32" else 1e-11)  # FP32 contractions: 7e-6 relative measured
    assert err < tol
    theta = np.concatenate([np.asarray(m[k], dtype=float) for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS])
    lhs, rhs = float(theta @ got[:-1]), tau * got[-1]
    assert abs(lhs - rhs) < tol * max(1.0, abs(rhs)), (lhs, rhs)


def test_complex_costate_gives_the_real_costate_result():
    """The co-state in the complex FP64 form: the gradient of a string on an
    untruncated run (no truncation decision to differ) equals the real form's
    to round-off, and the oracle's."""
    m = workloads.random_model(5, 44)
    got = []
    for cplx in (False, True):
        ch = _chain(m, 0.1, 32, 0.0, "+x")
        G = Gradient(ch, 3, complex_costate=cplx)
        F, g = G.run_string("IZIXI")
        G.close()
        ch.close()
        got.append(np.concatenate([g[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS + ("tau",)]))
    Fo, go, _ = adjoint.gradient(m, 0.1, 3, 32, 0.0, "+x", None, None, paulis="IZIXI")
    ref = np.concatenate([adjoint.flatten(m, go).real, go["tau"].real])
    scale = max(1.0, np.abs(ref).max())
    print(f"  real vs complex co-state {np.abs(got[0] - got[1]).max() / scale:.2e}, complex vs oracle "
          f"{np.abs(got[1] - ref).max() / scale:.2e}", flush=True)
    assert np.abs(got[0] - got[1]).max() < 1e-12 * scale
    assert np.abs(got[1] - ref).max() < 1e-9 * scale


def test_renyi2_gradient_checks():
    """Refused before the state moves: a complex-form state with the real
    co-state, a workspace without the series headroom, a co-state chi_max
    below the state's."""
    from paper_2203_05871_amd import LmpoError

    m = workloads.random_model(4, 43)
    ch = _chain(m, 0.1, 8, 1e-10, "+x")
    G = Gradient(ch, 2, series=True)
    with pytest.raises(LmpoError, match="LMPO_GRAD_COMPLEX_COSTATE"):
        G.run_renyi2()
    G.close()
    ch.close()
    ch = _chain(m, 0.1, 8, 1e-10, "+x", precision="real")
    before = [ch.get_site(k) for k in range(4)]
    for kw, msg in (({}, "LMPO_GRAD_SERIES"), ({"co_chi": 2, "series": True}, "at least the state's")):
        G = Gradient(ch, 2, **kw)
        with pytest.raises(LmpoError, match=msg):
            G.run_renyi2()
        G.close()
    assert all(np.array_equal(x, ch.get_site(k)) for k, x in enumerate(before))
    ch.close()


@pytest.mark.parametrize("case", ["exact_chain_mid", "exact_chain_edge", "truncated_ladder", "costate_truncated",
                                  "complex_fp64", "complex_fp32"])
def test_osee_gradient(case):
    """dOSEE/dtheta across a bond (Eq. OSEE): the co-state is the state with the
    bond's singular values replaced by dS/ds; against the oracle (which takes
    the SVD of the centre site in its own basis and conjugates), the value
    against lmpo_osee on the state left at T, and the scaling identity."""
    co_chi = co_cut = None
    if case.startswith("exact_chain"):
        m, tau, steps, chi, cut, init = workloads.random_model(5, 49), 0.1, 3, 32, 0.0, "+x"
        bond = 2 if case.endswith("mid") else 0
    else:
        lad = workloads.ladder_model(4)
        m = workloads.random_model(8, 50, bonds=lad["bonds"])
        tau, steps, chi, cut, init, bond = 0.1, 4, 8, 1e-10, "+z", 3
        if case == "costate_truncated":
            co_chi, co_cut = 8, 1e-6
    prec = {"complex_fp64": "fp64", "complex_fp32": "fp32"}.get(case, "real")
    tol = 1e-5 if prec == "fp32" else 1e-9
    print(f"gradient case: osee {case} N={m['N']} bond={bond} chi={chi} co-state {co_chi} {co_cut}", flush=True)
    ch = _chain(m, tau, chi, cut, init, precision=prec)
    G = Gradient(ch, steps, co_chi or 0, -1.0 if co_cut is None else co_cut, complex_costate=prec != "real")
    S, g = G.run_osee(bond)
    G.close()
    assert abs(ch.osee(bond) - S) < 1e-12
    ch.close()
    So, go, _ = adjoint.gradient_osee(m, tau, steps, chi, cut, init, bond, costate_chi_max=co_chi,
                                      costate_cutoff=co_cut)
    got = np.concatenate([g[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS + ("tau",)])
    ref = np.concatenate([adjoint.flatten(m, go).real, go["tau"].real])
    err = np.abs(got - ref).max() / max(1.0, np.abs(ref).max())
    print(f"  OSEE = {S:.12f} (oracle {So:.12f}), max |grad - oracle| / scale = {err:.2e}", flush=True)
    assert abs(S - So) < (tol * max(1.0, abs(So)) if prec == "fp32" else 1e-11)
    assert err < tol
    theta = np.concatenate([np.asarray(m[k], dtype=float) for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS])
    lhs, rhs = float(theta @ got[:-1]), tau * got[-1]
    assert abs(lhs - rhs) < tol * max(1.0, abs(rhs)), (lhs, rhs)


def test_osee_gradient_checks():
    """Refused before the state moves: a complex-form state with the real
    co-state, a bond out of range, a co-state chi_max below the state's."""
    from paper_2203_05871_amd import LmpoError

    m = workloads.random_model(4, 51)
    ch = _chain(m, 0.1, 8, 1e-10, "+x")
    G = Gradient(ch, 2)
    with pytest.raises(LmpoError, match="LMPO_GRAD_COMPLEX_COSTATE"):
        G.run_osee(1)
    G.close()
    ch.close()
    ch = _chain(m, 0.1, 8, 1e-10, "+x", precision="real")
    before = [ch.get_site(k) for k in range(4)]
    G = Gradient(ch, 2)
    for b in (-1, 3):
        with pytest.raises(LmpoError, match="bond out of range"):
            G.run_osee(b)
    G.close()
    G = Gradient(ch, 2, co_chi=2)
    with pytest.raises(LmpoError, match="at least the state's"):
        G.run_osee(1)
    G.close()
    assert all(np.array_equal(x, ch.get_site(k)) for k, x in enumerate(before))
    ch.close()


def test_entropy_gradient_edge_cases():
    """N = 2 (S_2 and the OSEE of its one bond, one step) against the oracle; a
    bond with no coupling across it (the state a product there at every time):
    OSEE 0 and a zero gradient, the oracle's too."""
    m2 = workloads.random_model(2, 54)
    ch = _chain(m2, 0.1, 8, 1e-12, "+x", precision="real")
    G = Gradient(ch, 1, series=True)
    S2, g2 = G.run_renyi2()
    Sb, gb = G.run_osee(0)  # continues from the state after the first run: two steps in all
    G.close()
    ch.close()
    So, go, _ = adjoint.gradient_renyi2(m2, 0.1, 1, 8, 1e-12, "+x")
    assert abs(S2 - So) < 1e-12
    assert np.abs(np.concatenate([g2[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS])
                  - adjoint.flatten(m2, go).real).max() < 1e-9
    ch = _chain(m2, 0.1, 8, 1e-12, "+x", precision="real")
    ch.evolve(1)
    G = Gradient(ch, 1)
    Sb2, gb2 = G.run_osee(0)
    G.close()
    ch.close()
    assert Sb == Sb2 and all(np.array_equal(gb[k], gb2[k]) for k in gb)
    m = workloads.random_model(3, 53)
    m["J"] = np.array(m["J"], dtype=float)
    m["Jz"] = np.array(m["Jz"], dtype=float)
    m["J"][0] = m["Jz"][0] = 0.0
    print("gradient case: osee across an uncoupled bond, N=3", flush=True)
    ch = _chain(m, 0.1, 8, 1e-12, "+x", precision="real")
    G = Gradient(ch, 2)
    S, g = G.run_osee(0)
    G.close()
    ch.close()
    _, go, _ = adjoint.gradient_osee(m, 0.1, 2, 8, 1e-12, "+x", 0)
    got = np.concatenate([g[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS + ("tau",)])
    print(f"  OSEE = {S:.3e}, max |grad| = {np.abs(got).max():.3e}", flush=True)
    assert abs(S) < 1e-14
    assert np.abs(got).max() < 1e-10
    assert np.abs(adjoint.flatten(m, go)).max() == 0.0
