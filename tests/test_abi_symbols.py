"""CPU checks of the C ABI: the library loads and exports every declared symbol."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lmpo.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lmpo_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_core_entry_points():
    syms = declared_symbols()
    for s in ("lmpo_create", "lmpo_evolve_step", "lmpo_trace", "lmpo_renormalize", "lmpo_measure_1q",
              "lmpo_measure_2q", "lmpo_destroy", "lmpo_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2203_05871_amd import lmpo

    lib = ctypes.CDLL(lmpo.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(lmpo.EXPORTS) == declared_symbols()


def test_arena_size_and_argument_errors_on_host():
    """lmpo_arena_bytes validates on the host without touching a GPU."""
    import workloads
    from paper_2203_05871_amd import lmpo

    m, run = workloads.chain30_jittered()
    n = lmpo.arena_bytes(m, run["tau"], run["chi_max"], run["cutoff"])
    # 30 sites at chi=256 dominate: at least 28 * 256*4*256 complex doubles
    assert n > 28 * 256 * 4 * 256 * 16
    assert n < 2 << 30
    import pytest
    with pytest.raises(lmpo.LmpoError, match="tau"):
        lmpo.arena_bytes(m, -1.0, 16)
    with pytest.raises(lmpo.LmpoError, match="chi_max"):
        lmpo.arena_bytes(m, 0.1, 0)
    with pytest.raises(lmpo.LmpoError, match="cutoff"):
        lmpo.arena_bytes(m, 0.1, 8, cutoff=-1)
    with pytest.raises(lmpo.LmpoError, match="trotter_order"):
        lmpo.arena_bytes(m, 0.1, 8, order=5)
    assert lmpo.arena_bytes(m, 0.1, 8, order=3) > 0
    with pytest.raises(lmpo.LmpoError, match="trotter_order 3"):
        lmpo.arena_bytes(workloads.ladder_model(3), 0.1, 8, order=3)
    bad = dict(m)
    bad["g0"] = -m["g0"]
    with pytest.raises(lmpo.LmpoError, match="rates"):
        lmpo.arena_bytes(bad, 0.1, 8)
    lad = workloads.ladder_model(3)
    assert lmpo.arena_bytes(lad, 0.1, 8) > 0  # bonds apart along the path are accepted
    lone = dict(lad)
    lone["bonds"] = lad["bonds"][lad["bonds"].max(axis=1) < 5]  # qubit 5 in no bond
    lone["J"], lone["Jz"] = lad["J"][: len(lone["bonds"])], lad["Jz"][: len(lone["bonds"])]
    with pytest.raises(lmpo.LmpoError, match="belong to a bond"):
        lmpo.arena_bytes(lone, 0.1, 8)


def test_gradient_entry_points_reject_bad_arguments_on_host():
    """The gradient workspace calls validate their arguments before any GPU work."""
    from paper_2203_05871_amd import lmpo

    lib = lmpo.load_library()
    assert lib.lmpo_grad_arena_bytes(None, 4, 0, -1.0, 0) == 0
    assert b"state is null" in lib.lmpo_last_error()
    out = ctypes.c_void_p()
    assert lib.lmpo_grad_create(None, 4, 0, -1.0, 0, None, 0, ctypes.byref(out)) == -1
    assert lib.lmpo_grad_run_series(None, b"IZ", 1, None, None, None, None) == -1
    assert lib.lmpo_grad_costate_dims(None, None) == -1
    assert lib.lmpo_grad_costate(None) is None
    assert lib.lmpo_grad_run_connected(None, 0, 1, b"ZZ", None, None) == -1
    assert lib.lmpo_grad_run_renyi2(None, None, None) == -1
    assert lib.lmpo_grad_run_osee(None, 0, None, None) == -1
    assert lib.lmpo_probe_fp64_mfma_bytes() == 2048 * 256 * 8
    assert lib.lmpo_probe_fp64_mfma(None, None, 0, None) == -1
    assert lib.lmpo_set_svd_tolerance(None, 32.0) == -1
    assert lib.lmpo_grad_run(None, b"IZ", None, None) == -1
    assert lib.lmpo_grad_destroy(None) == 0


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message before any GPU work."""
    import subprocess
    import sys

    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert out.returncode != 0 and "one GPU" in out.stderr
