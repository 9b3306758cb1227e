"""Thin Python binding of the lmpo C ABI (include/lmpo.h).

Argument marshalling only: every step of the evolution runs in the HIP
library.  PyTorch supplies the device arena (a uint8 tensor on the GPU) and
the stream; the library never allocates device memory.  If the compiled
library is missing, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblmpo.so")

LMPO_FP64 = 0
LMPO_FP32_CONTRACT = 1
LMPO_FP64_REAL = 2

_ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENUMERIC", -5: "EUNSUPPORTED"}


class LmpoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lmpo error {code} ({_ERRORS.get(code, '?')}): {msg}")
        self.code = code


class _Model(ctypes.Structure):
    _fields_ = [
        ("n_qubits", ctypes.c_int32),
        ("n_bonds", ctypes.c_int32),
        ("bond_ij", ctypes.POINTER(ctypes.c_int32)),
        ("J", ctypes.POINTER(ctypes.c_double)),
        ("Jz", ctypes.POINTER(ctypes.c_double)),
        ("hx", ctypes.POINTER(ctypes.c_double)),
        ("hy", ctypes.POINTER(ctypes.c_double)),
        ("hz", ctypes.POINTER(ctypes.c_double)),
        ("g0", ctypes.POINTER(ctypes.c_double)),
        ("g1", ctypes.POINTER(ctypes.c_double)),
        ("g2", ctypes.POINTER(ctypes.c_double)),
    ]


class _Options(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double),
        ("trotter_order", ctypes.c_int32),
        ("chi_max", ctypes.c_int32),
        ("cutoff", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("force_trace", ctypes.c_int32),
        ("force_hermitian_every", ctypes.c_int32),
    ]


_lib = None

EXPORTS = [
    "lmpo_arena_bytes", "lmpo_create", "lmpo_evolve_step", "lmpo_trace", "lmpo_renormalize",
    "lmpo_measure_1q", "lmpo_measure_2q", "lmpo_measure_2q_noalloc", "lmpo_bond_dims", "lmpo_discarded_weight", "lmpo_sync",
    "lmpo_destroy", "lmpo_last_error", "lmpo_get_site", "lmpo_set_site", "lmpo_set_centre",
    "lmpo_get_centre", "lmpo_get_gate", "lmpo_apply_gate", "lmpo_last_spectrum", "lmpo_svd_stats",
    "lmpo_svd_profile", "lmpo_profile_begin", "lmpo_profile_end", "lmpo_set_workgroups", "lmpo_set_svd_tolerance",
    "lmpo_set_svd_subspace", "lmpo_svd_subspace_stats",
    "lmpo_renyi2", "lmpo_osee", "lmpo_apply_superop", "lmpo_apply_unitary", "lmpo_init_graph_state",
    "lmpo_hermitize",
    "lmpo_batch_arena_bytes", "lmpo_batch_create", "lmpo_batch_evolve_step", "lmpo_batch_sync",
    "lmpo_batch_plan", "lmpo_batch_profile_begin", "lmpo_batch_profile_end", "lmpo_batch_destroy",
    "lmpo_batch_set_autotune", "lmpo_autotune_table",
    "lmpo_grad_arena_bytes", "lmpo_grad_create", "lmpo_grad_run", "lmpo_grad_costate_dims", "lmpo_grad_costate", "lmpo_grad_run_connected", "lmpo_grad_run_series",
    "lmpo_grad_run_renyi2", "lmpo_grad_run_osee",
    "lmpo_probe_fp64_mfma_bytes", "lmpo_probe_fp64_mfma",
    "lmpo_grad_destroy",
]


def load_library(path: str = LIB_PATH):
    """Load the compiled library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, dbl = ctypes.c_int32, ctypes.c_double
    pi32 = ctypes.POINTER(ctypes.c_int32)
    pdbl = ctypes.POINTER(ctypes.c_double)
    sig = {
        "lmpo_arena_bytes": (ctypes.c_size_t, [ctypes.POINTER(_Model), ctypes.POINTER(_Options)]),
        "lmpo_create": (ctypes.c_int, [ctypes.POINTER(_Model), ctypes.POINTER(_Options), ctypes.c_char_p, P,
                                       ctypes.c_size_t, P, ctypes.POINTER(P)]),
        "lmpo_evolve_step": (ctypes.c_int, [P, i32]),
        "lmpo_trace": (ctypes.c_int, [P, pdbl]),
        "lmpo_renormalize": (ctypes.c_int, [P]),
        "lmpo_measure_1q": (ctypes.c_int, [P, i32, pi32, ctypes.c_char_p, pdbl]),
        "lmpo_measure_2q": (ctypes.c_int, [P, i32, pi32, pi32, ctypes.c_char_p, pdbl]),
        "lmpo_measure_2q_noalloc": (ctypes.c_int, [P, i32, pi32, pi32, ctypes.c_char_p, pdbl]),
        "lmpo_bond_dims": (ctypes.c_int, [P, pi32]),
        "lmpo_discarded_weight": (ctypes.c_int, [P, pdbl]),
        "lmpo_sync": (ctypes.c_int, [P]),
        "lmpo_destroy": (ctypes.c_int, [P]),
        "lmpo_last_error": (ctypes.c_char_p, []),
        "lmpo_get_site": (ctypes.c_int, [P, i32, pi32, pdbl]),
        "lmpo_set_site": (ctypes.c_int, [P, i32, i32, i32, pdbl]),
        "lmpo_set_centre": (ctypes.c_int, [P, i32]),
        "lmpo_get_centre": (ctypes.c_int, [P, pi32]),
        "lmpo_get_gate": (ctypes.c_int, [P, i32, i32, pdbl]),
        "lmpo_apply_gate": (ctypes.c_int, [P, i32, i32, i32]),
        "lmpo_last_spectrum": (ctypes.c_int, [P, i32, pdbl, pi32, pi32]),
        "lmpo_svd_stats": (ctypes.c_int, [P, pi32]),
        "lmpo_svd_profile": (ctypes.c_int, [P, pdbl]),
        "lmpo_profile_begin": (ctypes.c_int, [P, i32]),
        "lmpo_profile_end": (ctypes.c_int, [P, pdbl]),
        "lmpo_set_workgroups": (ctypes.c_int, [P, i32]),
        "lmpo_set_svd_tolerance": (ctypes.c_int, [P, dbl]),
        "lmpo_set_svd_subspace": (ctypes.c_int, [P, i32, i32, i32, i32, dbl]),
        "lmpo_svd_subspace_stats": (ctypes.c_int, [P, pi32]),
        "lmpo_renyi2": (ctypes.c_int, [P, pdbl]),
        "lmpo_osee": (ctypes.c_int, [P, i32, pdbl]),
        "lmpo_apply_superop": (ctypes.c_int, [P, i32, i32, pdbl]),
        "lmpo_apply_unitary": (ctypes.c_int, [P, i32, i32, pdbl]),
        "lmpo_init_graph_state": (ctypes.c_int, [P, i32, pi32]),
        "lmpo_hermitize": (ctypes.c_int, [P]),
        "lmpo_batch_arena_bytes": (ctypes.c_size_t, [ctypes.POINTER(P), i32]),
        "lmpo_batch_create": (ctypes.c_int, [ctypes.POINTER(P), i32, P, ctypes.c_size_t, ctypes.POINTER(P)]),
        "lmpo_batch_evolve_step": (ctypes.c_int, [P, i32]),
        "lmpo_batch_sync": (ctypes.c_int, [P]),
        "lmpo_batch_plan": (ctypes.c_int, [P, pi32]),
        "lmpo_batch_profile_begin": (ctypes.c_int, [P, i32]),
        "lmpo_batch_profile_end": (ctypes.c_int, [P, pdbl]),
        "lmpo_batch_destroy": (ctypes.c_int, [P]),
        "lmpo_batch_set_autotune": (ctypes.c_int, [P, i32]),
        "lmpo_autotune_table": (ctypes.c_int, [i32, pi32, pi32, pi32, pdbl, pi32]),
        "lmpo_grad_arena_bytes": (ctypes.c_size_t, [P, i32, i32, dbl, i32]),
        "lmpo_grad_create": (ctypes.c_int, [P, i32, i32, dbl, i32, P, ctypes.c_size_t, ctypes.POINTER(P)]),
        "lmpo_grad_run_series": (ctypes.c_int, [P, ctypes.c_char_p, i32, pi32, pdbl, pdbl, pdbl]),
        "lmpo_grad_costate_dims": (ctypes.c_int, [P, pi32]),
        "lmpo_grad_costate": (P, [P]),
        "lmpo_grad_run_renyi2": (ctypes.c_int, [P, pdbl, pdbl]),
        "lmpo_grad_run_osee": (ctypes.c_int, [P, i32, pdbl, pdbl]),
        "lmpo_grad_run_connected": (ctypes.c_int, [P, i32, i32, ctypes.c_char_p, pdbl, pdbl]),
        "lmpo_probe_fp64_mfma_bytes": (ctypes.c_size_t, []),
        "lmpo_probe_fp64_mfma": (ctypes.c_int, [P, P, ctypes.c_size_t, pdbl]),
        "lmpo_grad_run": (ctypes.c_int, [P, ctypes.c_char_p, pdbl, pdbl]),
        "lmpo_grad_destroy": (ctypes.c_int, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise LmpoError(rc, _lib.lmpo_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class _ModelArrays:
    """Keeps the contiguous host arrays alive while the C struct points at them."""

    def __init__(self, model):
        N = int(model["N"])
        self.bonds = np.ascontiguousarray(np.asarray(model["bonds"], dtype=np.int32).reshape(-1, 2))
        nb = len(self.bonds)
        f = lambda k, n: np.ascontiguousarray(np.broadcast_to(np.asarray(model.get(k, 0.0), dtype=np.float64), (n,)))
        self.arrs = {k: f(k, nb) for k in ("J", "Jz")}
        self.arrs.update({k: f(k, N) for k in ("hx", "hy", "hz", "g0", "g1", "g2")})
        self.struct = _Model(N, nb, _iptr(self.bonds), *[_dptr(self.arrs[k]) for k in
                                                          ("J", "Jz", "hx", "hy", "hz", "g0", "g1", "g2")])


def _options(tau, chi_max, cutoff, precision, force_trace, order=2, hermitian_every=0):
    prec = {"fp64": LMPO_FP64, "fp32": LMPO_FP32_CONTRACT, "real": LMPO_FP64_REAL}.get(precision, precision)
    return _Options(float(tau), int(order), int(chi_max), float(cutoff), int(prec), int(bool(force_trace)),
                    int(hermitian_every))


def arena_bytes(model, tau, chi_max, cutoff=0.0, precision="fp64", force_trace=True, order=2, hermitian_every=0):
    lib = load_library()
    m = _ModelArrays(model)
    o = _options(tau, chi_max, cutoff, precision, force_trace, order, hermitian_every)
    n = lib.lmpo_arena_bytes(ctypes.byref(m.struct), ctypes.byref(o))
    if n == 0:
        raise LmpoError(-1, lib.lmpo_last_error().decode())
    return int(n)


def _init_string(init, N):
    if isinstance(init, str):
        return init.encode()
    labels = list(init)
    if len(labels) != N:
        raise ValueError("init must be one label or N labels")
    return "".join(labels).encode()


class Chain:
    """One qubit chain's vectorised density matrix on the GPU."""

    def __init__(self, model, tau, chi_max, cutoff=0.0, precision="fp64", init="+z", force_trace=True,
                 order=2, device="cuda:0", stream=None, hermitian_every=0):
        import torch

        lib = load_library()
        self.N = int(model["N"])
        self._m = _ModelArrays(model)
        self._o = _options(tau, chi_max, cutoff, precision, force_trace, order, hermitian_every)
        n = lib.lmpo_arena_bytes(ctypes.byref(self._m.struct), ctypes.byref(self._o))
        if n == 0:
            raise LmpoError(-1, lib.lmpo_last_error().decode())
        self.arena = torch.empty(n + 256, dtype=torch.uint8, device=device)
        base = self.arena.data_ptr()
        off = (-base) % 256
        self._stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        _check(lib.lmpo_create(ctypes.byref(self._m.struct), ctypes.byref(self._o), _init_string(init, self.N),
                               ctypes.c_void_p(base + off), ctypes.c_size_t(n), ctypes.c_void_p(self._stream.cuda_stream),
                               ctypes.byref(h)))
        self._h = h
        self._lib = lib

    # -- evolution --
    def evolve(self, n_steps=1):
        _check(self._lib.lmpo_evolve_step(self._h, int(n_steps)))

    def renormalize(self):
        _check(self._lib.lmpo_renormalize(self._h))

    def sync(self):
        _check(self._lib.lmpo_sync(self._h))

    def apply_gate(self, k, half, ascending):
        _check(self._lib.lmpo_apply_gate(self._h, int(k), int(bool(half)), int(bool(ascending))))

    def apply_superop(self, i, j, G):
        """16x16 superoperator (Pauli basis, index 4 a_i + a_j) on qubits (i, j)."""
        G = np.asarray(G, dtype=np.complex128).reshape(16, 16)
        buf = np.ascontiguousarray(np.stack([G.real, G.imag], axis=-1).reshape(-1))
        _check(self._lib.lmpo_apply_superop(self._h, int(i), int(j), _dptr(buf)))

    def apply_unitary(self, i, j, U):
        """rho -> U rho U^+ for a 4x4 unitary on qubits (i, j), basis |k_i k_j>."""
        U = np.asarray(U, dtype=np.complex128).reshape(4, 4)
        buf = np.ascontiguousarray(np.stack([U.real, U.imag], axis=-1).reshape(-1))
        _check(self._lib.lmpo_apply_unitary(self._h, int(i), int(j), _dptr(buf)))

    def hermitize(self):
        """rho -> (rho + rho^+)/2 now (needs hermitian_every > 0 at creation)."""
        _check(self._lib.lmpo_hermitize(self._h))

    def init_graph_state(self, pairs):
        """Restart from the graph state of Eq. (graph_state) on the given pairs."""
        p = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        _check(self._lib.lmpo_init_graph_state(self._h, len(p), _iptr(p)))

    # -- readouts --
    def trace(self):
        out = np.zeros(2)
        _check(self._lib.lmpo_trace(self._h, _dptr(out)))
        return complex(out[0], out[1])

    def measure_1q(self, sites, paulis):
        sites = np.ascontiguousarray(sites, dtype=np.int32)
        if isinstance(paulis, str) and len(paulis) == 1:
            paulis = paulis * len(sites)
        p = "".join(paulis).encode()
        out = np.zeros((len(sites), 2))
        _check(self._lib.lmpo_measure_1q(self._h, len(sites), _iptr(sites), p, _dptr(out)))
        return out[:, 0] + 1j * out[:, 1]

    def measure_2q(self, i, j, paulis):
        i = np.ascontiguousarray(i, dtype=np.int32)
        j = np.ascontiguousarray(j, dtype=np.int32)
        if isinstance(paulis, str) and len(paulis) == 2:
            paulis = [paulis] * len(i)
        p = "".join(paulis).encode()
        out = np.zeros((len(i), 2))
        _check(self._lib.lmpo_measure_2q(self._h, len(i), _iptr(i), _iptr(j), p, _dptr(out)))
        return out[:, 0] + 1j * out[:, 1]

    def measure_2q_noalloc(self, i, j, paulis):
        """measure_2q through lmpo_measure_2q_noalloc (working memory in the
        library's fixed device array instead of the arena)."""
        i = np.ascontiguousarray(i, dtype=np.int32)
        j = np.ascontiguousarray(j, dtype=np.int32)
        if isinstance(paulis, str) and len(paulis) == 2:
            paulis = [paulis] * len(i)
        p = "".join(paulis).encode()
        out = np.zeros((len(i), 2))
        _check(self._lib.lmpo_measure_2q_noalloc(self._h, len(i), _iptr(i), _iptr(j), p, _dptr(out)))
        return out[:, 0] + 1j * out[:, 1]

    def zz_observables(self):
        """<sz_i> (all i) and <sz_i sz_j> (all i < j), as complex arrays."""
        N = self.N
        z1 = self.measure_1q(np.arange(N), "Z")
        ii, jj = np.triu_indices(N, 1)
        z2 = self.measure_2q(ii, jj, "ZZ")
        return z1, z2

    def renyi2(self):
        """S_2 = -ln tr(rho^2) (Eq. S_2)."""
        out = np.zeros(1)
        _check(self._lib.lmpo_renyi2(self._h, _dptr(out)))
        return float(out[0])

    def osee(self, bond):
        """Operator-space entanglement entropy across bond (bond, bond+1) (Eq. OSEE)."""
        out = np.zeros(1)
        _check(self._lib.lmpo_osee(self._h, int(bond), _dptr(out)))
        return float(out[0])

    def bond_dims(self):
        out = np.zeros(self.N - 1, dtype=np.int32)
        _check(self._lib.lmpo_bond_dims(self._h, _iptr(out)))
        return out.tolist()

    def discarded_weight(self):
        out = np.zeros(1)
        _check(self._lib.lmpo_discarded_weight(self._h, _dptr(out)))
        return float(out[0])

    def get_site(self, k):
        dims = np.zeros(2, dtype=np.int32)
        _check(self._lib.lmpo_get_site(self._h, int(k), _iptr(dims), None))
        buf = np.zeros(int(dims[0]) * 4 * int(dims[1]) * 2)
        _check(self._lib.lmpo_get_site(self._h, int(k), _iptr(dims), _dptr(buf)))
        return (buf[0::2] + 1j * buf[1::2]).reshape(int(dims[0]), 4, int(dims[1]))

    def set_site(self, k, A):
        A = np.asarray(A, dtype=np.complex128)
        buf = np.ascontiguousarray(np.stack([A.real, A.imag], axis=-1).reshape(-1))
        _check(self._lib.lmpo_set_site(self._h, int(k), A.shape[0], A.shape[2], _dptr(buf)))

    def set_centre(self, c):
        _check(self._lib.lmpo_set_centre(self._h, int(c)))

    def centre(self):
        out = np.zeros(1, dtype=np.int32)
        _check(self._lib.lmpo_get_centre(self._h, _iptr(out)))
        return int(out[0])

    def gate(self, bond, half):
        buf = np.zeros(512)
        _check(self._lib.lmpo_get_gate(self._h, int(bond), int(bool(half)), _dptr(buf)))
        return (buf[0::2] + 1j * buf[1::2]).reshape(16, 16)

    def last_spectrum(self, n=4096):
        sv = np.zeros(n)
        nsv = np.zeros(1, dtype=np.int32)
        kept = np.zeros(1, dtype=np.int32)
        _check(self._lib.lmpo_last_spectrum(self._h, n, _dptr(sv), _iptr(nsv), _iptr(kept)))
        return sv[: int(nsv[0])], int(kept[0])

    def svd_stats(self):
        """(last sweeps, last column count, total sweeps, total SVDs incl. hops)."""
        out = np.zeros(4, dtype=np.int32)
        _check(self._lib.lmpo_svd_stats(self._h, _iptr(out)))
        return tuple(int(x) for x in out)

    def svd_profile(self):
        """Accumulated microseconds per persistent-SVD phase (first workgroup)."""
        out = np.zeros(32)
        _check(self._lib.lmpo_svd_profile(self._h, _dptr(out)))
        names = ["setup", "pairs", "wait", "cycles", "tasks", "select", "epilogue", "launches", "gram", "eig",
                 "upd_x", "upd_v", "rotated", "-", "-", "cholqr_passes", "order", "qr_panel", "qr_update", "form_q",
                 "sub_setup", "sub_iterations", "sub_final_cholqr", "sub_rr_rest", "sub_vectors", "hop_cholqr",
                 "cholqr_gram", "cholqr_cholesky", "cholqr_solve", "chol_diag_lookahead", "chol_last_step",
                 "chol_rows"]
        return dict(zip(names, out.tolist()))

    def profile_begin(self, max_launches=20000):
        _check(self._lib.lmpo_profile_begin(self._h, int(max_launches)))

    def set_workgroups(self, max_workgroups):
        """Cap the workgroups per SVD launch (0: automatic); results do not depend on it."""
        _check(self._lib.lmpo_set_workgroups(self._h, int(max_workgroups)))

    def set_svd_tolerance(self, factor):
        """Jacobi stopping threshold in units of sqrt(C) eps (default 32)."""
        _check(self._lib.lmpo_set_svd_tolerance(self._h, float(factor)))

    def set_svd_subspace(self, min_cols=512, margin=48, grow=32, iterations=4, tol=1e-12):
        """Truncated SVD of gate blocks with at least min_cols columns on a
        subspace (min_cols <= 0: every block takes the full SVD)."""
        _check(self._lib.lmpo_set_svd_subspace(self._h, int(min_cols), int(margin), int(grow), int(iterations),
                                               float(tol)))

    def svd_subspace_stats(self):
        """(subspace SVDs accepted, handed to the full SVD, iterations of the accepted ones)."""
        out = np.zeros(3, dtype=np.int32)
        _check(self._lib.lmpo_svd_subspace_stats(self._h, _iptr(out)))
        return tuple(int(x) for x in out)

    def profile_end(self):
        """(SVD launches, summed kernel ms from HIP events, summed declared flops)."""
        out = np.zeros(3)
        _check(self._lib.lmpo_profile_end(self._h, _dptr(out)))
        return int(out[0]), float(out[1]), float(out[2])

    def gradient(self, n_steps, site=None, pauli=None, paulis=None, costate_chi_max=0, costate_cutoff=-1.0):
        """Advance n_steps and return (F, {key: dF/dtheta}) for F = <sigma^pauli_site>,
        or for the Pauli string `paulis` (one of I, X, Y, Z per qubit), at the end
        (lmpo_grad_run); keys hx, hy, hz, g0, g1, g2 (per qubit), J, Jz (per bond) and
        tau (one entry).
        The co-state takes the chain's chi_max / cutoff unless given."""
        g = Gradient(self, n_steps, costate_chi_max, costate_cutoff)
        try:
            return g.run_string(paulis) if paulis is not None else g.run(site, pauli)
        finally:
            g.close()

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.lmpo_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def measured_fp64_mfma_peak(device="cuda:0"):
    """FP64 matrix-core TFLOP/s measured by lmpo_probe_fp64_mfma on the current stream."""
    import torch

    lib = load_library()
    n = lib.lmpo_probe_fp64_mfma_bytes()
    buf = torch.empty(n, dtype=torch.uint8, device=device)
    out = np.zeros(1)
    _check(lib.lmpo_probe_fp64_mfma(ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream),
                                    ctypes.c_void_p(buf.data_ptr()), ctypes.c_size_t(n), _dptr(out)))
    return float(out[0])


GRAD_SITE_KEYS = ("hx", "hy", "hz", "g0", "g1", "g2")
GRAD_BOND_KEYS = ("J", "Jz")


class Gradient:
    """Adjoint-gradient workspace of one chain for a fixed number of steps
    (lmpo_grad_*).  Each run() advances the chain by those steps.  series:
    room for run_series; keep_gates: every step's gate snapshots kept from the
    forward run (no replay in the backward pass, much more device memory);
    complex_costate: the co-state in the complex FP64 form (run_renyi2 and
    run_osee of a complex-form chain need it)."""

    def __init__(self, chain, n_steps, costate_chi_max=0, costate_cutoff=-1.0, series=False, keep_gates=False,
                 complex_costate=False):
        import torch

        lib = load_library()
        self.chain, self.n_steps = chain, int(n_steps)
        co = (int(costate_chi_max), float(costate_cutoff), (1 if series else 0) | (2 if keep_gates else 0)
              | (4 if complex_costate else 0))
        n = lib.lmpo_grad_arena_bytes(chain._h, self.n_steps, *co)
        if n == 0:
            raise LmpoError(-1, lib.lmpo_last_error().decode())
        self.arena = torch.empty(n + 256, dtype=torch.uint8, device=chain.arena.device)
        base = self.arena.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        _check(lib.lmpo_grad_create(chain._h, self.n_steps, *co, ctypes.c_void_p(base + off), ctypes.c_size_t(n),
                                    ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.n_bonds = len(chain._m.bonds)

    def run(self, site, pauli):
        """run_string for sigma^pauli on one qubit."""
        s = ["I"] * self.chain.N
        s[int(site)] = pauli.upper()
        return self.run_string("".join(s))

    def run_string(self, paulis):
        """(F, {key: dF/dtheta}) for the Pauli string (one of I, X, Y, Z per qubit)."""
        F = np.zeros(2)
        g = np.zeros(6 * self.chain.N + 2 * self.n_bonds + 1)
        _check(self._lib.lmpo_grad_run(self._h, paulis.upper().encode(), _dptr(F), _dptr(g)))
        return self._unpack(F, g)

    def run_series(self, paulis, out_steps, weights):
        """(F_k array, {key: dJ/dtheta}) for J = sum_k w_k Re <paulis> after out_steps[k]
        steps (needs series=True at creation)."""
        outs = np.ascontiguousarray(out_steps, dtype=np.int32)
        w = np.ascontiguousarray(weights, dtype=np.float64)
        if len(w) != len(outs):
            raise ValueError("one weight per output step")
        F = np.zeros((len(outs), 2))
        g = np.zeros(6 * self.chain.N + 2 * self.n_bonds + 1)
        _check(self._lib.lmpo_grad_run_series(self._h, paulis.upper().encode(), len(outs), _iptr(outs), _dptr(w),
                                              _dptr(F), _dptr(g)))
        _, out = self._unpack(np.zeros(2), g)
        return F[:, 0] + 1j * F[:, 1], out

    def run_connected(self, i, j, paulis="ZZ"):
        """(C, {key: dC/dtheta}) for the connected correlator <a_i b_j> - <a_i><b_j>."""
        F = np.zeros(2)
        g = np.zeros(6 * self.chain.N + 2 * self.n_bonds + 1)
        _check(self._lib.lmpo_grad_run_connected(self._h, int(i), int(j), paulis.upper().encode(), _dptr(F),
                                                 _dptr(g)))
        return self._unpack(F, g)

    def run_renyi2(self):
        """(S_2, {key: dS_2/dtheta}) for the second Renyi entropy at T (needs
        series=True at creation, and the real-arithmetic form or complex_costate=True)."""
        S2 = np.zeros(1)
        g = np.zeros(6 * self.chain.N + 2 * self.n_bonds + 1)
        _check(self._lib.lmpo_grad_run_renyi2(self._h, _dptr(S2), _dptr(g)))
        _, out = self._unpack(np.zeros(2), g)
        return float(S2[0]), out

    def run_osee(self, bond):
        """(OSEE, {key: dOSEE/dtheta}) across bond (bond, bond + 1) at T (needs
        the real-arithmetic form or complex_costate=True)."""
        h = np.zeros(1)
        g = np.zeros(6 * self.chain.N + 2 * self.n_bonds + 1)
        _check(self._lib.lmpo_grad_run_osee(self._h, int(bond), _dptr(h), _dptr(g)))
        _, out = self._unpack(np.zeros(2), g)
        return float(h[0]), out

    def _unpack(self, F, g):
        N, nb = self.chain.N, self.n_bonds
        out = {k: g[q * N:(q + 1) * N].copy() for q, k in enumerate(GRAD_SITE_KEYS)}
        out["J"] = g[6 * N:6 * N + nb].copy()
        out["Jz"] = g[6 * N + nb:6 * N + 2 * nb].copy()
        out["tau"] = g[6 * N + 2 * nb:].copy()
        return complex(F[0], F[1]), out

    def costate_profile_begin(self, max_launches=20000):
        """HIP events around every co-state SVD launch of the next run()."""
        _check(self._lib.lmpo_profile_begin(self._lib.lmpo_grad_costate(self._h), int(max_launches)))

    def costate_profile_end(self):
        """(co-state SVD launches, summed kernel ms, summed declared flops)."""
        out = np.zeros(3)
        _check(self._lib.lmpo_profile_end(self._lib.lmpo_grad_costate(self._h), _dptr(out)))
        return int(out[0]), float(out[1]), float(out[2])

    def set_costate_svd_tolerance(self, factor):
        """The co-state's Jacobi stopping threshold (lmpo_set_svd_tolerance on it)."""
        _check(self._lib.lmpo_set_svd_tolerance(self._lib.lmpo_grad_costate(self._h), float(factor)))

    def costate_dims(self):
        """Bond dims of the co-state (after run(): at time 0)."""
        out = np.zeros(self.chain.N - 1, dtype=np.int32)
        _check(self._lib.lmpo_grad_costate_dims(self._h, _iptr(out)))
        return out.tolist()

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.lmpo_grad_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many chains advanced together, one cooperative launch per Trotter layer
    (lmpo_batch_*).  The chains stay usable for readouts after sync(); they
    must share one stream and outlive the batch."""

    def __init__(self, chains, device="cuda:0"):
        import torch

        lib = load_library()
        self.chains = list(chains)
        arr = (ctypes.c_void_p * len(self.chains))(*[c._h.value for c in self.chains])
        self._arr = arr
        n = lib.lmpo_batch_arena_bytes(arr, len(self.chains))
        if n == 0:
            raise LmpoError(-1, lib.lmpo_last_error().decode())
        self.arena = torch.empty(n + 256, dtype=torch.uint8, device=device)
        base = self.arena.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        _check(lib.lmpo_batch_create(arr, len(self.chains), ctypes.c_void_p(base + off), ctypes.c_size_t(n),
                                     ctypes.byref(h)))
        self._h = h
        self._lib = lib

    def evolve(self, n_steps=1):
        _check(self._lib.lmpo_batch_evolve_step(self._h, int(n_steps)))

    def sync(self):
        _check(self._lib.lmpo_batch_sync(self._h))

    def set_autotune(self, enable=True):
        _check(self._lib.lmpo_batch_set_autotune(self._h, int(bool(enable))))

    @staticmethod
    def tuning_table():
        """[(log2 block bucket, precision mask, cap, best ms)] tuned so far on this device."""
        lib = load_library()
        n = np.zeros(1, dtype=np.int32)
        _check(lib.lmpo_autotune_table(0, None, None, None, None, _iptr(n)))
        m = int(n[0])
        if m == 0:
            return []
        b, p, c = (np.zeros(m, dtype=np.int32) for _ in range(3))
        ms = np.zeros(m)
        _check(lib.lmpo_autotune_table(m, _iptr(b), _iptr(p), _iptr(c), _dptr(ms), _iptr(n)))
        return [(int(b[i]), int(p[i]), int(c[i]), float(ms[i])) for i in range(m)]

    def plan(self):
        """Workgroups per chain in the current launch plan."""
        out = np.zeros(len(self.chains), dtype=np.int32)
        _check(self._lib.lmpo_batch_plan(self._h, _iptr(out)))
        return out

    def profile_begin(self, max_launches=20000):
        _check(self._lib.lmpo_batch_profile_begin(self._h, int(max_launches)))

    def profile_end(self):
        """(layer launches, summed kernel ms from HIP events, summed declared SVD flops)."""
        out = np.zeros(3)
        _check(self._lib.lmpo_batch_profile_end(self._h, _dptr(out)))
        return int(out[0]), float(out[1]), float(out[2])

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.lmpo_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _expectation_function():
    import torch

    class ExpectationFn(torch.autograd.Function):
        """F = Re <sigma^pauli_site>(T) as a differentiable function of the model
        parameters: the forward pass runs lmpo_grad_run (state forward, co-state
        backward) and keeps the gradient, the backward pass scales it."""

        @staticmethod
        def forward(ctx, spec, *params):
            model = {"N": spec["N"], "bonds": spec["bonds"]}
            for key, t in zip(GRAD_SITE_KEYS + GRAD_BOND_KEYS, params):
                model[key] = t.detach().to("cpu", torch.float64).numpy().reshape(-1)
            ch = Chain(model, spec["tau"], spec["chi_max"], spec.get("cutoff", 0.0), spec.get("precision", "fp64"),
                       spec.get("init", "+z"), force_trace=spec.get("force_trace", True),
                       order=spec.get("order", 2), device=spec.get("device", "cuda:0"))
            try:
                F, g = ch.gradient(spec["steps"], spec.get("site"), spec.get("pauli"), spec.get("paulis"),
                                   spec.get("costate_chi_max", 0), spec.get("costate_cutoff", -1.0))
            finally:
                ch.close()
            grads = [torch.as_tensor(g[k], dtype=p.dtype, device=p.device).reshape(p.shape)
                     for k, p in zip(GRAD_SITE_KEYS + GRAD_BOND_KEYS, params)]
            ctx.save_for_backward(*grads)
            return torch.tensor(F.real, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gout):
            return (None,) + tuple(gout.to(g.dtype) * g for g in ctx.saved_tensors)

    return ExpectationFn


def _series_function():
    import torch

    def run(spec, params, weights):
        model = {"N": spec["N"], "bonds": spec["bonds"]}
        for key, t in zip(GRAD_SITE_KEYS + GRAD_BOND_KEYS, params):
            model[key] = t.detach().to("cpu", torch.float64).numpy().reshape(-1)
        ch = Chain(model, spec["tau"], spec["chi_max"], spec.get("cutoff", 0.0), spec.get("precision", "fp64"),
                   spec.get("init", "+z"), force_trace=spec.get("force_trace", True), order=spec.get("order", 2),
                   device=spec.get("device", "cuda:0"))
        try:
            G = Gradient(ch, spec["steps"], spec.get("costate_chi_max", 0), spec.get("costate_cutoff", -1.0), True)
            try:
                return G.run_series(spec["paulis"], spec["out_steps"], weights)
            finally:
                G.close()
        finally:
            ch.close()

    class ExpectationSeriesFn(torch.autograd.Function):
        """F_k = Re <paulis> after spec["out_steps"][k] steps, as a vector-valued
        differentiable function of the model parameters: the forward pass is a
        series run with zero weights (values only), the backward pass one series
        gradient whose weights are the incoming gradients."""

        @staticmethod
        def forward(ctx, spec, *params):
            F, _ = run(spec, params, np.zeros(len(spec["out_steps"])))
            ctx.spec = spec
            ctx.save_for_backward(*params)
            return torch.as_tensor(F.real, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gout):
            params = ctx.saved_tensors
            _, g = run(ctx.spec, params, gout.detach().to("cpu", torch.float64).numpy())
            return (None,) + tuple(torch.as_tensor(g[k], dtype=p.dtype, device=p.device).reshape(p.shape)
                                   for k, p in zip(GRAD_SITE_KEYS + GRAD_BOND_KEYS, params))

    return ExpectationSeriesFn


def _entropy_function(kind):
    import torch

    class EntropyFn(torch.autograd.Function):
        """S_2(T) = -ln(tr rho^2 / (tr rho)^2) (kind "renyi2") or the OSEE across
        spec["bond"] (kind "osee") as a differentiable function of the model
        parameters: the forward pass runs lmpo_grad_run_renyi2 (the complex
        co-state for a complex-form chain) or lmpo_grad_run_osee and keeps the
        gradient, the backward pass scales it."""

        @staticmethod
        def forward(ctx, spec, *params):
            model = {"N": spec["N"], "bonds": spec["bonds"]}
            for key, t in zip(GRAD_SITE_KEYS + GRAD_BOND_KEYS, params):
                model[key] = t.detach().to("cpu", torch.float64).numpy().reshape(-1)
            prec = spec.get("precision", "real")
            ch = Chain(model, spec["tau"], spec["chi_max"], spec.get("cutoff", 0.0), prec, spec.get("init", "+z"),
                       force_trace=spec.get("force_trace", True), order=spec.get("order", 2),
                       device=spec.get("device", "cuda:0"))
            try:
                G = Gradient(ch, spec["steps"], spec.get("costate_chi_max", 0), spec.get("costate_cutoff", -1.0),
                             series=kind == "renyi2", complex_costate=prec != "real")
                try:
                    S2, g = G.run_renyi2() if kind == "renyi2" else G.run_osee(spec["bond"])
                finally:
                    G.close()
            finally:
                ch.close()
            grads = [torch.as_tensor(g[k], dtype=p.dtype, device=p.device).reshape(p.shape)
                     for k, p in zip(GRAD_SITE_KEYS + GRAD_BOND_KEYS, params)]
            ctx.save_for_backward(*grads)
            return torch.tensor(S2, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gout):
            return (None,) + tuple(gout.to(g.dtype) * g for g in ctx.saved_tensors)

    return EntropyFn


_EXPECTATION_FN = None
_SERIES_FN = None
_ENTROPY_FN = {}


def renyi2(spec, params):
    """Differentiable S_2 = -ln(tr rho^2 / (tr rho)^2) after spec["steps"] steps
    (Eq. S_2); spec as for expectation() without the observable (precision
    "real" by default), params likewise."""
    if "renyi2" not in _ENTROPY_FN:
        _ENTROPY_FN["renyi2"] = _entropy_function("renyi2")
    return _ENTROPY_FN["renyi2"].apply(spec, *[params[k] for k in GRAD_SITE_KEYS + GRAD_BOND_KEYS])


def osee(spec, params):
    """Differentiable OSEE across bond spec["bond"] (bond, bond + 1) after
    spec["steps"] steps (Eq. OSEE); spec as for renyi2(), params likewise."""
    if "osee" not in _ENTROPY_FN:
        _ENTROPY_FN["osee"] = _entropy_function("osee")
    return _ENTROPY_FN["osee"].apply(spec, *[params[k] for k in GRAD_SITE_KEYS + GRAD_BOND_KEYS])


def expectation_series(spec, params):
    """Differentiable vector F_k = Re <spec["paulis"]> after spec["out_steps"][k]
    steps (strictly increasing, at most spec["steps"]); otherwise as
    expectation().  The backward pass costs one series gradient."""
    global _SERIES_FN
    if _SERIES_FN is None:
        _SERIES_FN = _series_function()
    return _SERIES_FN.apply(spec, *[params[k] for k in GRAD_SITE_KEYS + GRAD_BOND_KEYS])


def expectation(spec, params):
    """Differentiable F = Re <sigma^pauli_site> after spec["steps"] steps.

    spec: N, bonds, tau, steps, chi_max, site and pauli (or a Pauli string
    paulis) and optionally cutoff,
    precision, init, force_trace, order, costate_chi_max, costate_cutoff,
    device.  params: tensors hx, hy, hz, g0, g1, g2 (length N) and J, Jz
    (length n_bonds); the result's backward fills their .grad."""
    global _EXPECTATION_FN
    if _EXPECTATION_FN is None:
        _EXPECTATION_FN = _expectation_function()
    return _EXPECTATION_FN.apply(spec, *[params[k] for k in GRAD_SITE_KEYS + GRAD_BOND_KEYS])
