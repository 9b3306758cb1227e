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


def _chain(m, tau, chi, cutoff, init, precision="fp64", order=2, force_trace=True):
    from paper_2203_05871_amd import Chain

    return Chain(m, tau, chi, cutoff, precision, init, force_trace=force_trace, order=order, device="cuda:0")


def _compare(m, tau, steps, chi, cutoff, init, site, pauli, precision="fp64", order=2, force_trace=True,
             co_chi=None, co_cut=None):
    print(f"gradient case: N={m['N']} bonds={len(m['bonds'])} chi={chi} cutoff={cutoff} steps={steps} "
          f"order={order} {precision} <{pauli}_{site}> co-state {co_chi} {co_cut}", flush=True)
    ch = _chain(m, tau, chi, cutoff, init, precision, order, force_trace)
    F, g = ch.gradient(steps, site, pauli, co_chi or 0, -1.0 if co_cut is None else co_cut)
    ch.close()
    Fo, go, _ = adjoint.gradient(m, tau, steps, chi, cutoff, init, site, pauli, order=order,
                                 force_trace=force_trace, costate_chi_max=co_chi, costate_cutoff=co_cut)
    got = np.concatenate([g[k] for k in adjoint.SITE_KEYS + adjoint.BOND_KEYS])
    ref = adjoint.flatten(m, go).real
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


def test_fourth_order_gradient():
    _compare(workloads.random_model(5, 8), 0.1, 2, 16, 1e-12, "+x", 0, "Z", order=4)


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
