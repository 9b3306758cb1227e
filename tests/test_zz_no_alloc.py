"""The allocation-free measurement entry point (lmpo_measure_2q_noalloc)
against lmpo_measure_2q, through the C ABI: the same kernels on the same
state, so the results agree bit for bit; two calls in a row, the second on a
smaller state with fewer requests, so that the shared device array is reused
with a different layout; and the size limit."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_05871_amd as p

    p.load_library()
    return p


def both(ch, i, j, paulis):
    ref = ch.measure_2q(i, j, paulis)
    got = ch.measure_2q_noalloc(i, j, paulis)
    return ref, got


def test_noalloc_measure_matches_the_arena_measure_twice(lib):
    rng = np.random.default_rng(3)
    m, run = workloads.chain30_jittered("+x")
    big = lib.Chain(m, run["tau"], 64, run["cutoff"], "fp64", "+x")
    big.evolve(8)
    ii, jj = np.triu_indices(30, 1)
    paulis = ["".join(rng.choice(list("XYZ"), 2)) for _ in ii]
    print(f"call 1: N=30, chi {max(big.bond_dims())}, {len(ii)} requests", flush=True)
    ref, got = both(big, ii, jj, paulis)
    assert np.array_equal(ref, got), np.abs(ref - got).max()
    # reversed pairs (i > j) take the swapped request, as in the arena version
    ref, got = both(big, jj[:7], ii[:7], paulis[:7])
    assert np.array_equal(ref, got)
    small_m = workloads.jittered_chain(6, 1)
    small = lib.Chain(small_m, 0.05, 16, 0.0, "fp64", "+y")
    small.evolve(5)
    print(f"call 2: N=6, chi {max(small.bond_dims())}, 4 requests", flush=True)
    ref, got = both(small, [0, 1, 5, 2], [3, 4, 0, 3], ["ZZ", "XY", "ZX", "YY"])
    assert np.array_equal(ref, got), np.abs(ref - got).max()
    # and the first state again after the second used the array
    ref, got = both(big, ii[:50], jj[:50], paulis[:50])
    assert np.array_equal(ref, got)
    big.close()
    small.close()


def test_noalloc_measure_argument_checks(lib):
    from paper_2203_05871_amd import LmpoError

    m = workloads.jittered_chain(5, 0)
    ch = lib.Chain(m, 0.05, 8, 0.0, "fp64", "+z")
    with pytest.raises(LmpoError, match="i != j"):
        ch.measure_2q_noalloc([1], [1], ["ZZ"])
    with pytest.raises(LmpoError, match="range"):
        ch.measure_2q_noalloc([0], [7], ["ZZ"])
    with pytest.raises(LmpoError, match="X, Y or Z"):
        ch.measure_2q_noalloc([0], [1], ["ZQ"])
    assert len(ch.measure_2q_noalloc([], [], [])) == 0
    ch.close()


def test_noalloc_measure_rejects_states_beyond_its_array(lib):
    """2 (N + 1) chi_cap 16 bytes + 128 KiB above 2 MiB: N = 241 at chi_cap 256."""
    from paper_2203_05871_amd import LmpoError

    m = workloads.jittered_chain(241, 0)
    ch = lib.Chain(m, 0.05, 256, 1e-10, "fp64", "+z")
    with pytest.raises(LmpoError, match="2 MiB|2097152"):
        ch.measure_2q_noalloc([0], [1], ["ZZ"])
    # the arena version serves the same state
    assert abs(ch.measure_2q([0], [1], ["ZZ"])[0] - 1.0) < 1e-12
    ch.close()
