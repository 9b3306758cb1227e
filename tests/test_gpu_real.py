"""GPU parity of the real-arithmetic Pauli-basis form (LMPO_FP64_REAL): in the
Hermitian Pauli basis every propagator and Pauli / graph initial state is
real, so the real form must reproduce the complex FP64 path and the oracle,
with imaginary parts exactly zero."""
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
                           ch.measure_1q(np.arange(N), "Y"), ch.measure_2q(ii, jj, "ZZ")])


def oracle_obs(mps, N):
    ii, jj = np.triu_indices(N, 1)
    one = [mps.expect({i: op}) for op in (lm.SZ, lm.SX, lm.SY) for i in range(N)]
    return np.array(one + [mps.expect({i: lm.SZ, j: lm.SZ}) for i, j in zip(ii, jj)])


def all_real(ch):
    return all(np.all(ch.get_site(k).imag == 0) for k in range(ch.N))


def test_real_form_equals_complex_fp64_truncated(lib):
    m = workloads.jittered_chain(10, 3)
    r = lib.Chain(m, 0.05, 24, 1e-12, "real", "+x")
    c = lib.Chain(m, 0.05, 24, 1e-12, "fp64", "+x")
    r.evolve(8)
    c.evolve(8)
    assert r.bond_dims() == c.bond_dims() and max(r.bond_dims()) == 24
    assert np.abs(obs(r, 10) - obs(c, 10)).max() < 1e-12
    assert all_real(r)
    assert np.abs(obs(r, 10).imag).max() == 0
    r.close()
    c.close()


@pytest.mark.parametrize("order", [2, 3, 4])
def test_real_form_against_oracle(lib, order):
    """Every model term switched on (h_y, g1, Jz included), no truncation."""
    m = workloads.random_model(6, 9)
    ch = lib.Chain(m, 0.05, 64, 0.0, "real", "-y", order=order)
    ref = tebd.MPS.product("-y", 6)
    ch.evolve(6)
    tebd.evolve(ref, m, 0.05, 6, 64, 0.0, order=order)
    assert np.abs(obs(ch, 6) - oracle_obs(ref, 6)).max() < 1e-10
    assert all_real(ch)
    ch.close()


def test_real_form_chain6_exact(lib):
    m, run = workloads.chain6_exact()
    ch = lib.Chain(m, run["tau"], run["chi_max"], run["cutoff"], "real", run["init"])
    ref = tebd.MPS.product(run["init"], m["N"])
    ch.evolve(run["steps"])
    tebd.evolve(ref, m, run["tau"], run["steps"], run["chi_max"], run["cutoff"])
    assert np.abs(obs(ch, 6) - oracle_obs(ref, 6)).max() < 1e-10
    ch.close()


def test_real_form_ladder_graph_state_and_gates(lib):
    """SWAP network, graph state and a real unitary channel (a rotation about
    y, real in the computational basis) in the real form."""
    m = workloads.ladder_model(3)
    ch = lib.Chain(m, 0.05, 32, 1e-12, "real", "+z")
    ref_c = lib.Chain(m, 0.05, 32, 1e-12, "fp64", "+z")
    pairs = [(0, 1), (1, 3), (2, 5)]
    ch.init_graph_state(pairs)
    ref_c.init_graph_state(pairs)
    ref = tebd.graph_state(6, pairs, 32, 1e-12)
    th = 0.3
    ry = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    U = np.kron(ry, ry)
    for x in (ch, ref_c):
        x.apply_unitary(1, 4, U)
        x.evolve(3)
    ref.apply_pair_gate(1, 4, lm.unitary_channel(U), 32, 1e-12, True)
    tebd.evolve(ref, m, 0.05, 3, 32, 1e-12)
    assert ch.bond_dims() == ref.bond_dims() == ref_c.bond_dims()
    assert np.abs(obs(ch, 6) - oracle_obs(ref, 6)).max() < 1e-10
    assert np.abs(obs(ch, 6) - obs(ref_c, 6)).max() < 1e-12
    assert all_real(ch)
    ch.close()
    ref_c.close()


def test_real_form_full_size_gate(lib):
    """A 1024 x 1024 block between two chi = 256 bonds of a real injected
    state (N = 10), one gate, against the oracle."""
    from test_gpu_fullsize import random_canonical_mps

    dims = [4, 16, 64, 256, 256, 256, 64, 16, 4]
    A = [t.real.astype(np.complex128) for t in random_canonical_mps(dims, 4, 3)]
    # bring the real parts back to canonical form around site 4 (QR sweeps from
    # both ends keep a real Pauli-basis state real)
    ref = tebd.MPS(tebd.from_pauli(A), centre=9)
    ref.move_centre(0)
    ref.move_centre(4)
    A = tebd.to_pauli(ref.A)
    assert max(np.abs(t.imag).max() for t in A) < 1e-12
    A = [t.real.astype(np.complex128) for t in A]
    m = workloads.jittered_chain(10, 3)
    ch = lib.Chain(m, 0.05, 256, 1e-10, "real", "+z")
    for k, t in enumerate(A):
        ch.set_site(k, t)
    ch.set_centre(4)
    ch.apply_gate(4, True, True)
    sv, kept = ch.last_spectrum()
    ref = tebd.MPS(tebd.from_pauli(A), centre=4)
    kk, s = ref.apply_gate(4, lm.bond_gate(m, 4, 0.025), 256, 1e-10, True)
    assert kept == kk
    assert np.abs(sv[:kk] - s[:kk]).max() < 1e-10 * s[0]
    assert np.abs(obs(ch, 10) - oracle_obs(ref, 10)).max() < 1e-10
    ch.close()


def test_real_batch(lib):
    """A batch of real-form chains equals their single-chain runs bit for
    bit, also beside a complex chain in the same batch."""
    ms = [workloads.jittered_chain(7, 1), workloads.jittered_chain(9, 2)]
    b_ch = [lib.Chain(m, 0.05, 16, 1e-12, "real", "+x") for m in ms] + [lib.Chain(ms[0], 0.05, 16, 1e-12, "fp64", "+x")]
    single = [lib.Chain(m, 0.05, 16, 1e-12, "real", "+x") for m in ms]
    b = lib.Batch(b_ch)
    b.evolve(5)
    b.sync()
    for x, y in zip(b_ch, single):
        y.evolve(5)
        assert x.bond_dims() == y.bond_dims()
        for k in range(x.N):
            assert np.array_equal(x.get_site(k), y.get_site(k))
    assert np.abs(obs(b_ch[0], 7) - obs(b_ch[2], 7)).max() < 1e-12
    b.close()
    for c in b_ch + single:
        c.close()


def test_real_form_rules(lib):
    m = workloads.jittered_chain(5, 0)
    ch = lib.Chain(m, 0.05, 16, 1e-12, "real", "+x", hermitian_every=1)
    ch.evolve(2)
    before = [ch.get_site(k) for k in range(5)]
    ch.hermitize()  # rho is Hermitian by construction: nothing to do
    assert all(np.array_equal(a, ch.get_site(k)) for k, a in enumerate(before))
    G = np.eye(16, dtype=np.complex128)
    G[1, 2] = 0.1j
    with pytest.raises(lib.LmpoError, match="real"):
        ch.apply_superop(0, 1, G)
    ch.close()
