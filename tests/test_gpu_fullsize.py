"""GPU parity at full size and on edge cases, through the C ABI.

Full size: a random canonical MPS at chi = 256 is injected (N = 10, so the
middle gate sees a 1024 x 1024 two-site block, as in the chi = 256 chain);
one gate is applied on the GPU and by the oracle; the singular values, the
kept rank and the observables after the gate must agree.
"""
import numpy as np
import pytest

import workloads
from oracle import model as lm
from oracle import tebd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Chain():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_05871_amd import Chain, load_library

    load_library()
    return Chain


def random_canonical_mps(dims, centre, seed, centre_decay=0.0):
    """Pauli-basis site tensors with bond dims `dims`: sites < centre left-,
    sites > centre right-orthonormal, the centre Gaussian (singular values
    reshaped to decay as exp(-decay j) when decay > 0)."""
    rng = np.random.default_rng(seed)
    N = len(dims) + 1
    A = []
    for k in range(N):
        cl = 1 if k == 0 else dims[k - 1]
        cr = 1 if k == N - 1 else dims[k]
        t = rng.standard_normal((cl, 4, cr)) + 1j * rng.standard_normal((cl, 4, cr))
        if k < centre:
            q, _ = np.linalg.qr(t.reshape(cl * 4, cr))
            t = q.reshape(cl, 4, cr)
        elif k > centre:
            q, _ = np.linalg.qr(t.reshape(cl, 4 * cr).T)
            t = q.T.reshape(cl, 4, cr)
        elif centre_decay > 0:
            u, s, vh = np.linalg.svd(t.reshape(cl * 4, cr), full_matrices=False)
            s = np.exp(-centre_decay * np.arange(len(s)))
            t = ((u * s) @ vh).reshape(cl, 4, cr)
        A.append(t)
    return A


def inject(ch, A, centre):
    """Write the site tensors and declare the centre."""
    for k, t in enumerate(A):
        ch.set_site(k, t)
    ch.set_centre(centre)


def one_gate_parity(Chain, dims, bond, chi_max, cutoff, seed, decay=0.0, asc=True, half=True, tau=0.05,
                    subspace=True):
    N = len(dims) + 1
    m = workloads.jittered_chain(N, seed)
    A = random_canonical_mps(dims, bond, seed, decay)
    ch = Chain(m, tau, chi_max, cutoff, "fp64", "+z")
    if not subspace:
        ch.set_svd_subspace(min_cols=0)
    inject(ch, A, bond)
    ch.apply_gate(bond, half, asc)
    sv, kept = ch.last_spectrum()
    ref = tebd.MPS(tebd.from_pauli(A), centre=bond)
    G = lm.bond_gate(m, bond, (0.5 if half else 1.0) * tau)
    kk, s = ref.apply_gate(bond, G, chi_max, cutoff, asc)
    return ch, ref, sv, kept, kk, s


@pytest.mark.parametrize("subspace", [False, True])
@pytest.mark.parametrize("decay", [0.0, 0.02])
def test_full_size_gate_1024(Chain, decay, subspace):
    """One gate on a 1024 x 1024 block, by the full SVD (all 1024 singular
    values) and by the subspace SVD with its defaults (the Ritz values of its
    p = min(256, 256 + 32) + 48 = 304 vectors)."""
    dims = [4, 16, 64, 256, 256, 256, 64, 16, 4]  # N = 10; bond 4 joins two chi = 256 bonds
    print(f"case: 1024 x 1024 gate, decay {decay}, subspace {subspace}", flush=True)
    ch, ref, sv, kept, kk, s = one_gate_parity(Chain, dims, 4, 256, 1e-10, 3, decay, subspace=subspace)
    assert len(s) == 1024
    assert kept == kk
    acc, fell, _ = ch.svd_subspace_stats()
    if subspace and decay == 0.0:
        # a Gaussian centre: the gate block has a gap at the bond's 256
        assert (acc, fell) == (1, 0) and len(sv) == 304
    if subspace and acc:
        # the kept Ritz values; the first discarded one (a Ritz value from
        # below, accurate to the residual of its unconverged vector) loosely
        np.testing.assert_allclose(sv[:kept], s[:kept], rtol=1e-10, atol=1e-13 * s[0])
        assert s[kept] * (1 - 1e-2) <= sv[kept] <= s[kept] * (1 + 1e-12)
    else:
        assert len(sv) == 1024
        assert acc == 0
        # singular values: relative agreement where they carry weight
        big = s > 1e-12 * s[0]
        np.testing.assert_allclose(sv[big], s[big], rtol=1e-10, atol=1e-13 * s[0])
    assert ch.bond_dims() == ref.bond_dims()
    for i in (0, 3, 4, 5, 9):
        g = ch.measure_1q([i], "Z")[0]
        r = ref.expect({i: lm.SZ})
        assert abs(g - r) < 1e-10, (i, g, r)
    g = ch.measure_2q([2], [7], ["XY"])[0]
    assert abs(g - ref.expect({2: lm.SX, 7: lm.SY})) < 1e-10
    ch.close()


@pytest.mark.parametrize("asc", [True, False])
def test_ragged_gate_both_directions(Chain, asc):
    """Bond dims that are not multiples of any tile: 37, 53, 29."""
    dims = [4, 16, 37, 53, 29, 16, 4]  # N = 8
    ch, ref, sv, kept, kk, s = one_gate_parity(Chain, dims, 3, 64, 1e-12, 5, 0.05, asc=asc)
    assert kept == kk
    big = s > 1e-12 * s[0]
    np.testing.assert_allclose(sv[big], s[big], rtol=1e-10, atol=1e-13 * s[0])
    for i in range(8):
        assert abs(ch.measure_1q([i], "Z")[0] - ref.expect({i: lm.SZ})) < 1e-10
    # the next gate needs a centre hop (and it is exact)
    nb = 5 if asc else 1
    G = lm.bond_gate(ch_model(8, 5), nb, 0.05)
    ref.apply_gate(nb, G, 64, 1e-12, asc)
    ch.apply_gate(nb, 0, asc)
    for i in range(8):
        assert abs(ch.measure_1q([i], "X")[0] - ref.expect({i: lm.SX})) < 1e-10
    ch.close()


def ch_model(N, seed):
    return workloads.jittered_chain(N, seed)


def test_chain20_full_run(Chain):
    """The 20-site chain workload in full (chi_max = 128, cutoff 1e-12, tau =
    0.05, 100 steps from +z): every 10 steps all <sz_i> and <sz_i sz_j> (i < j)
    and the bond dims against the oracle."""
    m, run = workloads.chain20_jittered()
    ch = Chain(m, run["tau"], run["chi_max"], run["cutoff"], "fp64", run["init"])
    ref = tebd.MPS.product(run["init"], m["N"])
    gates = tebd.gate_tables(m, run["tau"])
    for n in range(0, run["steps"], 10):
        ch.evolve(10)
        tebd.evolve(ref, m, run["tau"], 10, run["chi_max"], run["cutoff"], gates=gates, first_step=n)
        z1, z2 = ch.zz_observables()
        r1, r2 = tebd.zz_observables(ref)
        assert max(np.abs(z1 - r1).max(), np.abs(z2 - r2).max()) < 1e-10, n
        assert ch.bond_dims() == ref.bond_dims(), n
    ch.close()


def test_determinism(Chain):
    """Two identical runs are bitwise equal (no races in LDS / grid phases)."""
    m = workloads.jittered_chain(10, 2)
    outs = []
    for _ in range(2):
        ch = Chain(m, 0.05, 24, 1e-12, "fp64", "+x")
        ch.evolve(8)
        outs.append(np.concatenate([ch.measure_1q(np.arange(10), "X"), ch.measure_1q(np.arange(10), "Z")]))
        dims = ch.bond_dims()
        ch.close()
    assert np.array_equal(outs[0], outs[1])
    assert max(dims) == 24


def test_result_independent_of_workgroups(Chain):
    """The same gate (a 212 x 164 block: 11 Jacobi pairs per round, 11 QR
    update tasks) and the same steps with 1, 2, 5 and automatic workgroups per
    SVD give the same bits."""
    dims = [4, 16, 53, 64, 41, 16, 4]  # N = 8; bond 3 joins 53 and 41 (block 212 x 164)
    m = workloads.jittered_chain(8, 11)
    A = random_canonical_mps(dims, 3, 11, 0.05)
    outs = []
    for wg in (1, 2, 5, 0):
        ch = Chain(m, 0.05, 64, 1e-12, "fp64", "+z")
        inject(ch, A, 3)
        ch.set_workgroups(wg)
        ch.apply_gate(3, True, True)
        ch.apply_gate(5, False, True)
        ch.evolve(2)
        outs.append([ch.get_site(k) for k in range(8)] + [np.array(ch.bond_dims())])
        ch.close()
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.array_equal(x, y), np.abs(x - y).max()


def test_two_site_chain_and_chi_one(Chain):
    """N = 2 (a single bond) and chi_max = 1 (product-state truncation)."""
    m = workloads.random_model(2, 4)
    ch = Chain(m, 0.1, 4, 0.0, "fp64", "-y")
    ref = tebd.MPS.product("-y", 2)
    ch.evolve(5)
    tebd.evolve(ref, m, 0.1, 5, 4, 0.0)
    for i in range(2):
        for P, O in (("X", lm.SX), ("Y", lm.SY), ("Z", lm.SZ)):
            assert abs(ch.measure_1q([i], P)[0] - ref.expect({i: O})) < 1e-12
    ch.close()
    m = workloads.jittered_chain(6, 1)
    ch = Chain(m, 0.05, 1, 0.0, "fp64", "+x")
    ref = tebd.MPS.product("+x", 6)
    ch.evolve(3)
    tebd.evolve(ref, m, 0.05, 3, 1, 0.0)
    assert ch.bond_dims() == [1] * 5
    z = ch.measure_1q(np.arange(6), "Z")
    assert np.abs(z - [ref.expect({i: lm.SZ}) for i in range(6)]).max() < 1e-12
    ch.close()


def test_error_paths(Chain):
    from paper_2203_05871_amd import LmpoError

    m = workloads.jittered_chain(5, 0)
    with pytest.raises(LmpoError, match="Pauli"):
        Chain(m, 0.05, 8, 0.0, "fp64", "+q")
    ch = Chain(m, 0.05, 8, 0.0, "fp64", "+z")
    with pytest.raises(LmpoError, match="i != j"):
        ch.measure_2q([1], [1], ["ZZ"])
    with pytest.raises(LmpoError, match="range"):
        ch.measure_1q([7], "Z")
    with pytest.raises(LmpoError, match="X, Y, Z"):
        ch.measure_1q([0], "Q")
    ch.close()


@pytest.mark.timeout(400)
def test_chain30_full_run_parity(Chain):
    """The 30-site benchmark chain (chi_max = 256, cutoff 1e-10, tau = 0.05,
    +x, 50 steps) in the launch configuration the benchmark times: after every
    step of the run the bond dims, and at the end every <sz_i> and
    <sz_i sz_j> (i < j), FP64 against the oracle; the FP32-contraction form
    within 1e-5 of FP64."""
    m, run = workloads.chain30_jittered()
    N = m["N"]
    ch = Chain(m, run["tau"], run["chi_max"], run["cutoff"], "fp64", run["init"])
    c32 = Chain(m, run["tau"], run["chi_max"], run["cutoff"], "fp32", run["init"])
    ref = tebd.MPS.product(run["init"], N)
    for n in range(run["steps"]):
        ch.evolve(1)
        tebd.evolve(ref, m, run["tau"], 1, run["chi_max"], run["cutoff"], first_step=n)
        assert ch.bond_dims() == ref.bond_dims(), n
    c32.evolve(run["steps"])
    z1, z2 = ch.zz_observables()
    r1, r2 = tebd.zz_observables(ref)
    assert max(np.abs(z1 - r1).max(), np.abs(z2 - r2).max()) < 1e-10
    f1, f2 = c32.zz_observables()
    assert max(np.abs(f1 - z1).max(), np.abs(f2 - z2).max()) < 1e-5
    assert abs(ch.trace() - 1.0) < 1e-12
    ch.close()
    c32.close()


@pytest.mark.timeout(400)
def test_chain30_fp32_against_fp64_where_chi256_binds(Chain):
    """The 30-site benchmark chain where chi_max = 256 binds on every interior
    bond (cutoff 0: four steps from +x fill the bonds, 1024 x 1024 blocks in
    the bulk); from that one state the FP32-contraction form and the FP64 form
    each run two more steps: every <sz_i> and <sz_i sz_j> within 1e-5, the bond
    dims identical."""
    m, run = workloads.chain30_jittered()
    N = m["N"]
    print("case: N=30 chain, chi 256, cutoff 0, 4 steps then 2 per form", flush=True)
    ch = Chain(m, run["tau"], run["chi_max"], 0.0, "fp64", run["init"])
    ch.evolve(4)
    dims = ch.bond_dims()
    assert dims[3:-3] == [256] * (N - 7), dims
    sites = [ch.get_site(k) for k in range(N)]
    centre = ch.centre()
    ch.close()
    out = {}
    for prec in ("fp64", "fp32"):
        c = Chain(m, run["tau"], run["chi_max"], 0.0, prec, run["init"])
        inject(c, sites, centre)
        c.evolve(2)
        out[prec] = (c.zz_observables(), c.bond_dims())
        c.close()
    (z1, z2), d64 = out["fp64"]
    (f1, f2), d32 = out["fp32"]
    err = max(np.abs(f1 - z1).max(), np.abs(f2 - z2).max())
    print(f"  max |obs fp32 - fp64| = {err:.2e}", flush=True)
    assert d32 == d64
    assert err < 1e-5
