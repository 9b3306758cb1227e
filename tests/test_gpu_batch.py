"""GPU parity of the batched form (lmpo_batch_*): many uneven chains advanced
together, one cooperative launch per Trotter layer.

Every chain of a batch runs the same device code per op as the single-chain
executor, so its state after the batch must equal, bit for bit, the state the
single-chain path gives for the same steps; a few chains are also compared
with the FP64 oracle.
"""
import numpy as np
import pytest

import workloads
from oracle import model as lm
from oracle import tebd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_05871_amd as p

    p.load_library()
    return p


def snapshot(ch):
    """All site tensors (Pauli basis) and bond dims of a chain."""
    dims = ch.bond_dims()
    return dims, [ch.get_site(k) for k in range(ch.N)]


def assert_same_state(a, b):
    da, sa = snapshot(a)
    db, sb = snapshot(b)
    assert da == db
    for x, y in zip(sa, sb):
        assert x.shape == y.shape
        assert np.array_equal(x, y), np.abs(x - y).max()


def observables(ch):
    N = ch.N
    z = ch.measure_1q(np.arange(N), "Z")
    x = ch.measure_1q(np.arange(N), "X")
    zz = ch.measure_2q(np.arange(N - 1), np.arange(1, N), "ZZ")
    return np.concatenate([z, x, zz])


def oracle_observables(mps, N):
    z = [mps.expect({i: lm.SZ}) for i in range(N)]
    x = [mps.expect({i: lm.SX}) for i in range(N)]
    zz = [mps.expect({i: lm.SZ, i + 1: lm.SZ}) for i in range(N - 1)]
    return np.array(z + x + zz)


def uneven_models():
    """Five chains of different length and parameters (N = 4 .. 11)."""
    out = []
    for N, seed in ((6, 1), (4, 2), (9, 3), (7, 4), (11, 5)):
        out.append(workloads.random_model(N, seed) if seed % 2 else workloads.jittered_chain(N, seed))
    return out


def test_batch_matches_single_chain_bitwise(lib):
    models = uneven_models()
    chis = [16, 8, 24, 12, 20]
    inits = ["+x", "+z", "-y", "+x", "+z"]
    batch_chains = [lib.Chain(m, 0.05, c, 1e-12, "fp64", s) for m, c, s in zip(models, chis, inits)]
    single = [lib.Chain(m, 0.05, c, 1e-12, "fp64", s) for m, c, s in zip(models, chis, inits)]
    b = lib.Batch(batch_chains)
    b.evolve(7)
    b.sync()
    plan = b.plan()
    assert len(plan) == 5 and plan.min() >= 1
    for ch in single:
        ch.evolve(7)
        ch.sync()
    for x, y in zip(batch_chains, single):
        assert x.centre() == y.centre()
        assert_same_state(x, y)
    b.close()
    for ch in batch_chains + single:
        ch.close()


def test_batch_matches_oracle(lib):
    models = uneven_models()[:3]
    chains = [lib.Chain(m, 0.05, 32, 1e-12, "fp64", "+x") for m in models]
    b = lib.Batch(chains)
    b.evolve(6)
    b.sync()
    for m, ch in zip(models, chains):
        ref = tebd.MPS.product("+x", m["N"])
        tebd.evolve(ref, m, 0.05, 6, 32, 1e-12)
        assert ch.bond_dims() == ref.bond_dims()
        err = np.abs(observables(ch) - oracle_observables(ref, m["N"])).max()
        assert err < 1e-10, err
        assert abs(ch.trace() - 1.0) < 1e-12
    b.close()
    for ch in chains:
        ch.close()


def test_batch_continues_single_chain_steps(lib):
    """A chain stepped alone (odd step count: descending first layer) and then
    in a batch equals the same number of single-chain steps; a second batch
    call continues the first."""
    m1, m2 = workloads.jittered_chain(8, 7), workloads.jittered_chain(5, 8)
    a1, a2 = lib.Chain(m1, 0.05, 16, 1e-12, "fp64", "+x"), lib.Chain(m2, 0.05, 16, 1e-12, "fp64", "+x")
    r1, r2 = lib.Chain(m1, 0.05, 16, 1e-12, "fp64", "+x"), lib.Chain(m2, 0.05, 16, 1e-12, "fp64", "+x")
    a1.evolve(1)
    b = lib.Batch([a1, a2])
    b.evolve(2)
    b.evolve(1)
    b.sync()
    r1.evolve(4)
    r2.evolve(3)
    assert_same_state(a1, r1)
    assert_same_state(a2, r2)
    assert a1.centre() == r1.centre() and a2.centre() == r2.centre()
    # and the single-chain path continues the batch's result
    a1.evolve(1)
    r1.evolve(1)
    assert_same_state(a1, r1)
    b.close()
    for ch in (a1, a2, r1, r2):
        ch.close()


def test_batch_mixed_precision(lib):
    """FP32-contraction and FP64 chains in one batch; each equals its own
    single-chain run, and the FP32 one stays within 1e-5 of the FP64 one."""
    m = workloads.jittered_chain(10, 3)
    c64, c32 = lib.Chain(m, 0.05, 24, 1e-12, "fp64", "+x"), lib.Chain(m, 0.05, 24, 1e-12, "fp32", "+x")
    s32 = lib.Chain(m, 0.05, 24, 1e-12, "fp32", "+x")
    b = lib.Batch([c64, c32])
    b.evolve(5)
    b.sync()
    s32.evolve(5)
    assert_same_state(c32, s32)
    assert np.abs(observables(c32) - observables(c64)).max() < 1e-5
    b.close()
    for ch in (c64, c32, s32):
        ch.close()


def test_batch_64_chains_full_size_sampled(lib):
    """The 64-chain batching workload (N in [8, 24], chi_max = 64, cutoff
    1e-12) over all 40 configured steps in the launch configuration the
    benchmark times: the chains of the largest and smallest N, the first and
    the last chain equal their single-chain runs bit for bit, and the same four
    chains match the FP64 oracle (<s^z>, <s^x> of every qubit and <s^z s^z> of
    every neighbour pair, 1e-10)."""
    models, run = workloads.chains64_uneven()
    chains = [lib.Chain(m, run["tau"], run["chi_max"], run["cutoff"], "fp64", run["init"]) for m in models]
    b = lib.Batch(chains)
    steps = run["steps"]
    b.evolve(steps)
    b.sync()
    plan = b.plan()
    assert plan.sum() >= len(models)
    Ns = [m["N"] for m in models]
    sample = sorted({int(np.argmax(Ns)), int(np.argmin(Ns)), 0, 63})
    print(f"chains {sample}, N {[Ns[c] for c in sample]}, {steps} steps", flush=True)
    for c in sample:
        ref = lib.Chain(models[c], run["tau"], run["chi_max"], run["cutoff"], "fp64", run["init"])
        ref.evolve(steps)
        assert_same_state(chains[c], ref)
        ref.close()
        mps = tebd.MPS.product(run["init"], Ns[c])
        tebd.evolve(mps, models[c], run["tau"], steps, run["chi_max"], run["cutoff"])
        err = np.abs(observables(chains[c]) - oracle_observables(mps, Ns[c])).max()
        print(f"chain {c} (N={Ns[c]}): max |obs - oracle| = {err:.2e}, dims {chains[c].bond_dims()}", flush=True)
        assert err < 1e-10
        assert chains[c].bond_dims() == mps.bond_dims()
    b.close()
    for ch in chains:
        ch.close()


def test_batch_errors(lib):
    import torch

    from paper_2203_05871_amd import LmpoError

    m = workloads.jittered_chain(5, 0)
    a = lib.Chain(m, 0.05, 8, 0.0, "fp64", "+z")
    with pytest.raises(LmpoError, match="twice"):
        lib.Batch([a, a])
    s = torch.cuda.Stream()
    c = lib.Chain(m, 0.05, 8, 0.0, "fp64", "+z", stream=s)
    with pytest.raises(LmpoError, match="stream"):
        lib.Batch([a, c])
    with pytest.raises(LmpoError):
        lib.Batch([])
    a.close()
    c.close()


def test_batch_autotune_keeps_results(lib):
    """Autotuning tries several workgroup caps during real steps: the state is
    the same bits as without tuning, and the tuned entries are recorded."""
    models = uneven_models()
    # chi_max = 8 saturates within a few steps, so the block-size bucket settles
    # and its twelve trial steps (two per candidate) complete within the run
    a = [lib.Chain(m, 0.05, 8, 1e-12, "fp64", "+x") for m in models]
    r = [lib.Chain(m, 0.05, 8, 1e-12, "fp64", "+x") for m in models]
    ba = lib.Batch(a)
    ba.set_autotune(True)
    ba.evolve(20)
    ba.sync()
    for ch in r:
        ch.evolve(20)
        ch.sync()
    for x, y in zip(a, r):
        assert_same_state(x, y)
    table = lib.Batch.tuning_table()
    assert len(table) >= 1
    assert all(cap in (0, 1, 2, 4, 8, 16) and ms > 0 for _, _, cap, ms in table)
    ba.close()
    for ch in a + r:
        ch.close()
