"""GPU parity of general geometries (bonds apart along the MPS path, Sec. 2.3)
through the SWAP network, of caller-supplied two-site gates, and of the
graph-state initial condition (Eq. graph_state), against the FP64 oracle."""
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


def obs(ch, N):
    ii, jj = np.triu_indices(N, 1)
    return np.concatenate([ch.measure_1q(np.arange(N), "Z"), ch.measure_1q(np.arange(N), "X"),
                           ch.measure_1q(np.arange(N), "Y"), ch.measure_2q(ii, jj, "ZZ"),
                           ch.measure_2q(ii, jj, "XZ")])


def oracle_obs(mps, N):
    ii, jj = np.triu_indices(N, 1)
    one = [mps.expect({i: op}) for op in (lm.SZ, lm.SX, lm.SY) for i in range(N)]
    zz = [mps.expect({i: lm.SZ, j: lm.SZ}) for i, j in zip(ii, jj)]
    xz = [mps.expect({i: lm.SX, j: lm.SZ}) for i, j in zip(ii, jj)]
    return np.array(one + zz + xz)


def random_unitary(n, seed):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


@pytest.mark.parametrize("order", [2, 4])
def test_ladder_truncated_matches_oracle(lib, order):
    """2 x 4 ladder from +x (chi_max = 24 binds), every step's SWAPs truncated."""
    m = workloads.ladder_model(4)
    N = m["N"]
    ch = lib.Chain(m, 0.05, 24, 1e-12, "fp64", "+x", order=order)
    ref = tebd.MPS.product("+x", N)
    for n in range(0, 4, 2):
        ch.evolve(2)
        tebd.evolve(ref, m, 0.05, 2, 24, 1e-12, first_step=n, order=order)
        assert ch.bond_dims() == ref.bond_dims()
        assert np.abs(obs(ch, N) - oracle_obs(ref, N)).max() < 1e-10
    assert max(ch.bond_dims()) == 24
    assert abs(ch.trace() - 1.0) < 1e-12
    ch.close()


def test_graph_with_cycle_and_long_bonds(lib):
    """A random model on a graph with a cycle and pairs 2 and 3 sites apart."""
    bonds = [(0, 1), (0, 3), (1, 2), (2, 4), (3, 4), (1, 4), (4, 5)]
    m = workloads.random_model(6, 21, bonds=bonds)
    ch = lib.Chain(m, 0.04, 64, 1e-12, "fp64", ["+x", "-z", "+y", "+z", "-x", "+z"])
    ref = tebd.MPS.product(["+x", "-z", "+y", "+z", "-x", "+z"], 6)
    ch.evolve(3)
    tebd.evolve(ref, m, 0.04, 3, 64, 1e-12)
    assert ch.bond_dims() == ref.bond_dims()
    assert np.abs(obs(ch, 6) - oracle_obs(ref, 6)).max() < 1e-10
    ch.close()


def test_ladder2x8_full_run(lib):
    """The 2 x 8 ladder workload in full (N = 16, chi_max = 128, cutoff 1e-12,
    40 steps from +z), in the FP64 and FP32-contraction forms."""
    m, run = workloads.ladder2x8()
    N = m["N"]
    ch = lib.Chain(m, run["tau"], run["chi_max"], run["cutoff"], "fp64", run["init"])
    c32 = lib.Chain(m, run["tau"], run["chi_max"], run["cutoff"], "fp32", run["init"])
    ref = tebd.MPS.product(run["init"], N)
    ch.evolve(run["steps"])
    c32.evolve(run["steps"])
    tebd.evolve(ref, m, run["tau"], run["steps"], run["chi_max"], run["cutoff"])
    assert ch.bond_dims() == ref.bond_dims()
    o = obs(ch, N)
    assert np.abs(o - oracle_obs(ref, N)).max() < 1e-10
    assert np.abs(obs(c32, N) - o).max() < 1e-5
    ch.close()
    c32.close()


def test_ladder2x8_truncating_sampled(lib):
    """The same ladder from +x with chi_max = 32, which binds from the second
    step: three steps against the oracle."""
    m, run = workloads.ladder2x8()
    N = m["N"]
    ch = lib.Chain(m, run["tau"], 32, run["cutoff"], "fp64", "+x")
    ref = tebd.MPS.product("+x", N)
    ch.evolve(3)
    tebd.evolve(ref, m, run["tau"], 3, 32, run["cutoff"])
    assert ch.bond_dims() == ref.bond_dims()
    assert max(ch.bond_dims()) == 32
    assert np.abs(obs(ch, N) - oracle_obs(ref, N)).max() < 1e-10
    ch.close()


@pytest.mark.parametrize("i,j", [(1, 4), (4, 1), (2, 3)])
def test_unitary_and_superop_gates(lib, i, j):
    """A random two-qubit unitary channel and a random superoperator on an
    evolved chain, on neighbours and on qubits apart in either order."""
    m = workloads.jittered_chain(6, 5)
    ch = lib.Chain(m, 0.05, 64, 1e-12, "fp64", "+x")
    ref = tebd.MPS.product("+x", 6)
    ch.evolve(2)
    tebd.evolve(ref, m, 0.05, 2, 64, 1e-12)
    U = random_unitary(4, 10 * i + j)
    ch.apply_unitary(i, j, U)
    Gu = lm.unitary_channel(U)
    rng = np.random.default_rng(i + j)
    Gc = np.eye(16) + 0.3 * (rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16)))
    ch.apply_superop(i, j, tebd.gate_to_pauli(Gc))
    P = lm.swap_gate()
    lo, hi = min(i, j), max(i, j)
    for G in (Gu, Gc):
        ref.apply_pair_gate(lo, hi, G if i < j else P @ G @ P, 64, 1e-12, True)
    assert ch.bond_dims() == ref.bond_dims()
    tr = ref.trace()
    assert abs(ch.trace() - tr) < 1e-10 * abs(tr)
    assert np.abs(obs(ch, 6) - oracle_obs(ref, 6)).max() < 1e-10
    ch.close()


@pytest.mark.parametrize("pairs", [[(k, k + 1) for k in range(6)], [(0, 3), (1, 5), (2, 3), (4, 6), (0, 6)]])
def test_graph_state(lib, pairs):
    """The graph state equals the oracle's, is pure (S_2 = 0), and its
    two-body stabilisers hold; evolution from it matches the oracle."""
    m = workloads.jittered_chain(7, 2)
    ch = lib.Chain(m, 0.05, 64, 1e-12, "fp64", "+z")
    ch.evolve(1)  # the restart must discard this
    ch.init_graph_state(pairs)
    ref = tebd.graph_state(7, pairs, 64, 1e-12)
    assert ch.bond_dims() == ref.bond_dims()
    assert np.abs(obs(ch, 7) - oracle_obs(ref, 7)).max() < 1e-12
    assert abs(ch.renyi2()) < 1e-12
    nbrs = {a: [b for p in pairs for a2, b in (p, p[::-1]) if a2 == a] for a in range(7)}
    for a, nb in nbrs.items():
        if len(nb) == 1:  # X_a Z_b for a vertex with one neighbour
            assert abs(ch.measure_2q([a], [nb[0]], "XZ")[0] - 1.0) < 1e-12
        assert abs(ch.measure_1q([a], "X")[0]) < 1e-12
    ch.evolve(3)
    tebd.evolve(ref, m, 0.05, 3, 64, 1e-12)
    assert ch.bond_dims() == ref.bond_dims()
    assert np.abs(obs(ch, 7) - oracle_obs(ref, 7)).max() < 1e-10
    ch.close()


def test_errors_and_batch_rejects_general_bonds(lib):
    m = workloads.ladder_model(3)
    ch = lib.Chain(m, 0.05, 16, 1e-12, "fp64", "+z")
    with pytest.raises(lib.LmpoError, match="distinct"):
        ch.apply_unitary(2, 2, np.eye(4))
    with pytest.raises(lib.LmpoError, match="distinct"):
        ch.init_graph_state([(0, 6)])
    G = np.eye(16, dtype=np.complex128)
    G[3, 3] = np.nan
    with pytest.raises(lib.LmpoError, match="non-finite"):
        ch.apply_superop(0, 1, G)
    with pytest.raises(lib.LmpoError, match="open chains"):
        lib.Batch([ch])
    ch.close()
