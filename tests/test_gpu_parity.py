"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Bar: observables within 1e-10 on the FP64 path and 1e-5 on the FP32-contraction
path, at equal chi_max and cutoff; bond dimensions identical where the
spectrum has a clear gap at the cut.
"""
import numpy as np
import pytest

import workloads
from oracle import tebd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_05871_amd import Chain, load_library

    load_library()
    return Chain


def run_both(Chain, m, run, steps, precision="fp64", every=1, observables=None):
    """Evolve GPU and oracle side by side; return max |delta obs| and dims."""
    N = m["N"]
    ch = Chain(m, run["tau"], run["chi_max"], run["cutoff"], precision, run["init"])
    ref = tebd.MPS.product(run["init"], N)
    gates = tebd.gate_tables(m, run["tau"])
    worst = 0.0
    for n in range(0, steps, every):
        k = min(every, steps - n)
        ch.evolve(k)
        tebd.evolve(ref, m, run["tau"], k, run["chi_max"], run["cutoff"], gates=gates, first_step=n)
        z1, z2 = ch.zz_observables()
        r1, r2 = tebd.zz_observables(ref)
        worst = max(worst, np.abs(z1 - r1).max(), np.abs(z2 - r2).max())
        print(f"step {n + k}: max|dz|={worst:.2e} dims={ch.bond_dims()}", flush=True)
    return worst, ch, ref


def test_gate_table_matches_oracle(lib):
    m = workloads.random_model(4, 3)
    ch = lib(m, 0.07, 16, 0.0)
    for b in range(3):
        for half in (0, 1):
            G = ch.gate(b, half)
            ref = tebd.gate_to_pauli(__import__("oracle.model", fromlist=["x"]).bond_gate(m, b, 0.07 * (0.5 if half else 1.0)))
            np.testing.assert_allclose(G, ref, atol=1e-14)
    ch.close()


def test_initial_state_observables(lib):
    m = workloads.random_model(5, 1)
    ch = lib(m, 0.05, 16, 0.0, init="+x-y+z-x+y")
    x = ch.measure_1q([0, 1, 2, 3, 4], "XYZXY")
    np.testing.assert_allclose(x, [1, -1, 1, -1, 1], atol=1e-15)
    assert abs(ch.trace() - 1) < 1e-15
    zz = ch.measure_2q([0], [2], ["XZ"])
    np.testing.assert_allclose(zz, [1.0], atol=1e-15)
    ch.close()


def test_chain6_exact_parity_fp64(lib):
    """N=6, chi=64 (exact), tau=0.01, 100 steps, all <sz_i> and <sz_i sz_j>."""
    m, run = workloads.chain6_exact()
    worst, ch, ref = run_both(lib, m, run, run["steps"], every=10)
    assert worst < 1e-10
    assert ch.bond_dims() == ref.bond_dims()
    assert abs(ch.trace() - 1) < 1e-12
    ch.close()


def test_random_model_no_truncation(lib):
    """Every term of the model switched on (h_y, J_z, g1), mixed initial state."""
    m = workloads.random_model(5, 7)
    run = {"tau": 0.05, "chi_max": 16, "cutoff": 0.0, "init": ["+z", "-x", "+y", "-z", "+x"]}
    worst, ch, _ = run_both(lib, m, run, 12, every=4)
    assert worst < 1e-10
    ch.close()


def test_truncated_parity_fp64(lib):
    """chi_max binds (chi=12 < 4^4) with cutoff 1e-12 on a jittered chain."""
    m = workloads.jittered_chain(8, 0)
    run = {"tau": 0.05, "chi_max": 12, "cutoff": 1e-12, "init": "+x"}
    worst, ch, ref = run_both(lib, m, run, 20, every=5)
    assert max(ch.bond_dims()) == 12
    assert ch.bond_dims() == ref.bond_dims()
    assert worst < 1e-10
    assert abs(ch.discarded_weight() - ref.discarded) < 1e-10 * max(1.0, ref.discarded)
    ch.close()


def test_fp32_contraction_parity(lib):
    m = workloads.jittered_chain(8, 0)
    run = {"tau": 0.05, "chi_max": 12, "cutoff": 1e-12, "init": "+x"}
    worst, ch, _ = run_both(lib, m, run, 20, precision="fp32", every=10)
    assert worst < 1e-5
    ch.close()
