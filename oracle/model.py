"""Lindbladian of the qubit model, split into two-site generators (oracle).

Computational basis: sigma^z = diag(1, -1), |0> is the sigma^z = +1 state.
Ladder operators sigma^+- = (sigma^x +- i sigma^y)/2 (Sec. 2.1), so
sigma^+ = |0><1|.

Vectorisation: a one-qubit operator rho[k, b] maps to the 4-vector index
2*k + b (row-major).  Then vec(A rho B) = (A kron B^T) vec(rho).

Per-bond generator (Eq. dtrho with (H0), (K_def), (D0)-(D2)):
  H_b = J_b (s+_i s-_j + s-_i s+_j) + (1/2) Jz_b sz_i sz_j
        + sum_{s in b} w_s (1/2)(hx_s sx + hy_s sy + hz_s sz)_s
  jump operators  sqrt(w_s g0_s) s+_s,  sqrt(w_s g1_s) s-_s,  sqrt(w_s g2_s) sz_s
  w_s = 1 / (number of bonds touching site s)
so that the sum of all bond generators is the full Liouvillian.  K_def sums
over i != j; it is read here as one term per unordered coupled pair (the
nearest-neighbour form of Eq. K_drive).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

I2 = np.eye(2, dtype=np.complex128)
SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
SP = (SX + 1j * SY) / 2  # |0><1|
SM = (SX - 1j * SY) / 2  # |1><0|
PAULI = {"I": I2, "X": SX, "Y": SY, "Z": SZ}


def superop(A, B):
    """Matrix of rho -> A rho B on row-major vec(rho)."""
    return np.kron(A, B.T)


def lindblad_superop(H, jumps):
    """Matrix of rho -> -i[H, rho] + sum_k (L rho L^+ - 1/2 {L^+ L, rho})."""
    d = H.shape[0]
    Id = np.eye(d, dtype=np.complex128)
    L = -1j * (superop(H, Id) - superop(Id, H))
    for Lk in jumps:
        LdL = Lk.conj().T @ Lk
        L = L + superop(Lk, Lk.conj().T) - 0.5 * superop(LdL, Id) - 0.5 * superop(Id, LdL)
    return L


def site_degrees(model):
    deg = np.zeros(model["N"], dtype=np.int64)
    for i, j in model["bonds"]:
        deg[i] += 1
        deg[j] += 1
    return deg


def onsite_hamiltonian(model, s):
    return 0.5 * (model["hx"][s] * SX + model["hy"][s] * SY + model["hz"][s] * SZ)


def onsite_jumps(model, s, weight=1.0):
    out = []
    for rate, op in ((model["g0"][s], SP), (model["g1"][s], SM), (model["g2"][s], SZ)):
        if rate != 0.0:
            out.append(np.sqrt(weight * rate) * op)
    return out


def single_site_generator(model, s):
    """4x4 generator of the on-site part of site s alone (weight 1)."""
    return lindblad_superop(onsite_hamiltonian(model, s), onsite_jumps(model, s))


def _two_site_to_site_major(L16):
    """Reorder a 16x16 superoperator from (k_i k_j, b_i b_j) vec order to the
    site-major MPS order (k_i b_i, k_j b_j) on both sides."""
    T = L16.reshape(2, 2, 2, 2, 2, 2, 2, 2)  # ki kj bi bj ; ki' kj' bi' bj'
    T = T.transpose(0, 2, 1, 3, 4, 6, 5, 7)
    return T.reshape(16, 16)


def bond_generator(model, b):
    """16x16 generator L_b of bond b in site-major order (k_i b_i, k_j b_j)."""
    i, j = (int(x) for x in model["bonds"][b])
    deg = site_degrees(model)
    wi, wj = 1.0 / deg[i], 1.0 / deg[j]
    H = model["J"][b] * (np.kron(SP, SM) + np.kron(SM, SP))
    H = H + 0.5 * model["Jz"][b] * np.kron(SZ, SZ)
    H = H + wi * np.kron(onsite_hamiltonian(model, i), I2)
    H = H + wj * np.kron(I2, onsite_hamiltonian(model, j))
    jumps = [np.kron(L, I2) for L in onsite_jumps(model, i, wi)]
    jumps += [np.kron(I2, L) for L in onsite_jumps(model, j, wj)]
    return _two_site_to_site_major(lindblad_superop(H, jumps))


def bond_gate(model, b, x):
    """Two-site propagator exp(x L_b), Pade scaling-and-squaring (SciPy)."""
    return scipy.linalg.expm(x * bond_generator(model, b))


def unitary_channel(U):
    """Superoperator of rho -> U rho U^+ for a two-qubit unitary U (basis
    |k_i k_j>, index 2 k_i + k_j), in site-major order (k_i b_i, k_j b_j)."""
    U = np.asarray(U, dtype=np.complex128)
    return _two_site_to_site_major(superop(U, U.conj().T))


def swap_gate():
    """Superoperator that exchanges two sites' (ket, bra) pairs."""
    P = np.zeros((16, 16))
    for a in range(4):
        for c in range(4):
            P[c * 4 + a, a * 4 + c] = 1.0
    return P.astype(np.complex128)


def validate(model):
    """Parameter checks that mirror the solver's input rules (Sec. 6)."""
    N = model["N"]
    if N < 2:
        raise ValueError("N must be >= 2")
    bonds = np.asarray(model["bonds"])
    if bonds.ndim != 2 or bonds.shape[1] != 2:
        raise ValueError("bonds must be [n_bonds, 2]")
    for i, j in bonds:
        if not (0 <= i < j < N):
            raise ValueError("bond indices must satisfy 0 <= i < j < N")
    if np.any(site_degrees(model) == 0):
        raise ValueError("every site must belong to a bond")
    for key in ("g0", "g1", "g2"):
        if np.any(np.asarray(model[key]) < 0):
            raise ValueError(f"{key} must be >= 0")
