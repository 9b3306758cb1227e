"""GPU parity of the paper features next to the step: the third- and
fourth-order Trotter schemes (Sec. 6, trotter_order), the second Renyi entropy
(Eq. S_2) and the operator-space entanglement entropy (Eq. OSEE), against the
FP64 oracle."""
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
    return np.concatenate([ch.measure_1q(np.arange(N), "Z"), ch.measure_1q(np.arange(N), "X"),
                           ch.measure_2q(np.arange(N - 1), np.arange(1, N), "ZZ")])


def oracle_obs(mps, N):
    z = [mps.expect({i: lm.SZ}) for i in range(N)]
    x = [mps.expect({i: lm.SX}) for i in range(N)]
    zz = [mps.expect({i: lm.SZ, i + 1: lm.SZ}) for i in range(N - 1)]
    return np.array(z + x + zz)


@pytest.mark.parametrize("order", [3, 4])
def test_higher_order_exact_chain(lib, order):
    """N = 6 at chi = 64 = 4^3 (no truncation), every model term on, 12 steps."""
    m = workloads.random_model(6, 9)
    ch = lib.Chain(m, 0.05, 64, 0.0, "fp64", "+x", order=order)
    ref = tebd.MPS.product("+x", 6)
    for n in range(0, 12, 4):
        ch.evolve(4)
        tebd.evolve(ref, m, 0.05, 4, 64, 0.0, first_step=n, order=order)
        assert np.abs(obs(ch, 6) - oracle_obs(ref, 6)).max() < 1e-10
    assert ch.bond_dims() == ref.bond_dims()
    ch.close()


@pytest.mark.parametrize("order", [3, 4])
def test_higher_order_truncated(lib, order):
    """Jittered chain N = 10, chi_max = 12 binding, cutoff 1e-12, 8 steps."""
    m = workloads.jittered_chain(10, 4)
    ch = lib.Chain(m, 0.05, 12, 1e-12, "fp64", "+x", order=order)
    ref = tebd.MPS.product("+x", 10)
    ch.evolve(8)
    tebd.evolve(ref, m, 0.05, 8, 12, 1e-12, order=order)
    assert ch.bond_dims() == ref.bond_dims()
    assert max(ch.bond_dims()) == 12
    assert np.abs(obs(ch, 10) - oracle_obs(ref, 10)).max() < 1e-10
    ch.close()


@pytest.mark.parametrize("order", [3, 4])
def test_higher_order_batch_equals_single(lib, order):
    """A batch continues chains already stepped alone (odd step count), so the
    per-chain layer directions must follow each chain's own step count."""
    ms = [workloads.jittered_chain(7, 1), workloads.random_model(5, 2)]
    b_chains = [lib.Chain(m, 0.05, 16, 1e-12, "fp64", "+x", order=order) for m in ms]
    singles = [lib.Chain(m, 0.05, 16, 1e-12, "fp64", "+x", order=order) for m in ms]
    b_chains[0].evolve(1)
    singles[0].evolve(1)
    b = lib.Batch(b_chains)
    b.evolve(3)
    b.sync()
    for x, y in zip(b_chains, singles):
        y.evolve(3)
        assert x.bond_dims() == y.bond_dims()
        for k in range(x.N):
            assert np.array_equal(x.get_site(k), y.get_site(k))
    b.close()
    with pytest.raises(lib.LmpoError, match="Trotter order"):
        lib.Batch([b_chains[0], lib.Chain(ms[0], 0.05, 16, 1e-12, "fp64", "+x", order=2)])
    for c in b_chains + singles:
        c.close()


def test_renyi2_and_osee_parity(lib):
    """S_2 and the OSEE of every bond after truncated evolution; evolution
    continues to agree after the OSEE has moved the orthogonality centre."""
    m = workloads.jittered_chain(9, 6)
    ch = lib.Chain(m, 0.05, 20, 1e-12, "fp64", "+x")
    ref = tebd.MPS.product("+x", 9)
    assert abs(ch.renyi2() - ref.renyi2()) < 1e-12
    assert abs(ch.osee(4)) < 1e-12  # product state
    ch.evolve(6)
    tebd.evolve(ref, m, 0.05, 6, 20, 1e-12)
    assert abs(ch.renyi2() - ref.renyi2()) < 1e-10
    for bond in (4, 0, 7, 2):
        g, r = ch.osee(bond), ref.osee(bond)
        assert abs(g - r) < 1e-10, (bond, g, r)
        assert g > 0
    ch.evolve(3)
    tebd.evolve(ref, m, 0.05, 3, 20, 1e-12, first_step=6)
    assert ch.bond_dims() == ref.bond_dims()
    assert np.abs(obs(ch, 9) - oracle_obs(ref, 9)).max() < 1e-10
    assert abs(ch.renyi2() - ref.renyi2()) < 1e-10
    ch.close()


def test_osee_wide_centre_site(lib):
    """A centre site wider than tall (chi_r > 4 chi_l: an injected state with a
    non-minimal bond) takes the adjoint branch; the hop away from it compresses
    the bond to its rank exactly as the oracle's QR does."""
    from test_gpu_fullsize import random_canonical_mps

    dims = [2, 16, 16, 16, 4]  # N = 6; site 1 is 2 x 4 x 16, an 8 x 16 matrix
    m = workloads.jittered_chain(6, 3)
    A = random_canonical_mps(dims, 1, 8)
    ch = lib.Chain(m, 0.05, 64, 0.0, "fp64", "+z")
    for k, t in enumerate(A):
        ch.set_site(k, t)
    ch.set_centre(1)
    ref = tebd.MPS(tebd.from_pauli(A), centre=1)
    for bond in (1, 2, 4, 0):
        g, r = ch.osee(bond), ref.osee(bond)
        assert abs(g - r) < 1e-10, (bond, g, r)
    assert ch.bond_dims() == ref.bond_dims()
    ch.close()


def test_hermitize_non_hermitian_state(lib):
    """A non-Hermitian-preserving superoperator makes rho non-Hermitian; the
    Hermitian part then matches the oracle's, and observables become real."""
    m = workloads.jittered_chain(7, 3)
    ch = lib.Chain(m, 0.05, 32, 1e-12, "fp64", "+x", hermitian_every=1000)
    ref = tebd.MPS.product("+x", 7)
    ch.evolve(3)
    tebd.evolve(ref, m, 0.05, 3, 32, 1e-12)
    rng = np.random.default_rng(4)
    Gc = np.eye(16) + 0.2 * (rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16)))
    ch.apply_superop(1, 3, tebd.gate_to_pauli(Gc))
    ref.apply_pair_gate(1, 3, Gc, 32, 1e-12, True)
    assert np.abs(obs(ch, 7).imag).max() > 1e-3  # no longer Hermitian
    ch.hermitize()
    ref.hermitize(32, 1e-12)
    assert ch.bond_dims() == ref.bond_dims()
    assert ch.centre() == 0
    o = obs(ch, 7)
    assert np.abs(o - oracle_obs(ref, 7)).max() < 1e-10
    assert np.abs(o.imag).max() < 1e-12
    tr = ref.trace()
    assert abs(ch.trace() - tr) < 1e-12 * abs(tr) and abs(tr.imag) < 1e-14
    ch.close()


@pytest.mark.parametrize("ladder", [False, True])
def test_evolution_with_hermitian_every(lib, ladder):
    """The Hermitian part every 2nd step inside the evolution (chain and
    ladder, truncating), FP64 against the oracle, FP32 form within 1e-5."""
    m = workloads.ladder_model(4) if ladder else workloads.jittered_chain(9, 1)
    N = m["N"]
    ch = lib.Chain(m, 0.05, 16, 1e-12, "fp64", "+x", hermitian_every=2)
    c32 = lib.Chain(m, 0.05, 16, 1e-12, "fp32", "+x", hermitian_every=2)
    ref = tebd.MPS.product("+x", N)
    ch.evolve(5)
    c32.evolve(5)
    tebd.evolve(ref, m, 0.05, 5, 16, 1e-12, hermitian_every=2)
    assert ch.bond_dims() == ref.bond_dims()
    assert max(ch.bond_dims()) == 16
    o = obs(ch, N)
    assert np.abs(o - oracle_obs(ref, N)).max() < 1e-10
    assert np.abs(obs(c32, N) - o).max() < 1e-5
    ch.close()
    c32.close()


def test_hermitize_errors(lib):
    m = workloads.jittered_chain(5, 0)
    plain = lib.Chain(m, 0.05, 8, 0.0, "fp64", "+z")
    with pytest.raises(lib.LmpoError, match="force_hermitian_every"):
        plain.hermitize()
    roomy = lib.Chain(m, 0.05, 8, 0.0, "fp64", "+z", hermitian_every=3)
    with pytest.raises(lib.LmpoError, match="Hermitian"):
        lib.Batch([roomy])
    with pytest.raises(lib.LmpoError, match="capacity"):
        roomy.set_site(2, np.zeros((16, 4, 8)))  # bond capacity 16 reserved, 8 usable
    with pytest.raises(lib.LmpoError, match="chi_max <= 256"):
        lib.Chain(m, 0.05, 300, 0.0, "fp64", "+z", hermitian_every=1)
    plain.close()
    roomy.close()
