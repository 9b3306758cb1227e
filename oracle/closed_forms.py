"""Closed forms used to pin the oracle (textbook results, no MPS involved).

1. Single qubit (Eqs. H0, D0-D2 for one site): with rho = (1 + x sx + y sy + z sz)/2
   the Bloch vector r = (x, y, z) obeys dr/dt = h x r (precession for
   H = h.sigma/2) plus relaxation:
       dx/dt = -G2 x - hz y + hy z
       dy/dt =  hz x - G2 y - hx z
       dz/dt = (g0 - g1) - hy x + hx y - G1 z
   G1 = g0 + g1 (D0 pumps towards z = +1, D1 towards z = -1), G2 = G1/2 + 2 g2.
   Steady state for hx = Omega, hy = 0, hz = Delta, g1 = 0 (optical Bloch):
       D = G1 (G2^2 + Delta^2) + Omega^2 G2
       x = Delta Omega G1 / D,  y = -Omega G1 G2 / D,  z = G1 (G2^2 + Delta^2) / D.
2. One-excitation sector of the XY chain with Omega = 0, Jz = 0 (the quasi-free
   case of Sec. 2.1): starting from one flipped qubit, the one-body matrix
   P_jk = <j| rho |k> obeys
       dP/dt = -i [M, P] - (g0_j + g0_k)/2 P_jk - 2 (g2_j + g2_k)(1 - delta_jk) P_jk
   with M = -diag(hz) + J on the bond off-diagonals, and
       <sz_j> = 1 - 2 P_jj,   <sz_j sz_k> = 1 - 2 (P_jj + P_kk)  (j != k).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def bloch_generator(hx, hy, hz, g0, g1, g2):
    """4x4 affine generator acting on (1, x, y, z)."""
    G1 = g0 + g1
    G2 = G1 / 2 + 2 * g2
    return np.array([
        [0.0, 0.0, 0.0, 0.0],
        [0.0, -G2, -hz, hy],
        [0.0, hz, -G2, -hx],
        [g0 - g1, -hy, hx, -G1],
    ])


def bloch_evolve(r0, t, hx, hy, hz, g0, g1, g2):
    M = bloch_generator(hx, hy, hz, g0, g1, g2)
    v = scipy.linalg.expm(t * M) @ np.concatenate([[1.0], r0])
    return v[1:]


def bloch_steady_state(omega, delta, g0, g2):
    G1 = g0
    G2 = G1 / 2 + 2 * g2
    D = G1 * (G2 ** 2 + delta ** 2) + omega ** 2 * G2
    return np.array([delta * omega * G1 / D, -omega * G1 * G2 / D, G1 * (G2 ** 2 + delta ** 2) / D])


def one_excitation(model, site0, times):
    """(<sz_j>, <sz_j sz_k>) at each time, starting with qubit site0 flipped."""
    N = model["N"]
    M = np.diag(-np.asarray(model["hz"], dtype=np.complex128))
    for b, (i, j) in enumerate(model["bonds"]):
        M[i, j] += model["J"][b]
        M[j, i] += model["J"][b]
    g0 = np.asarray(model["g0"])
    g2 = np.asarray(model["g2"])
    decay = 0.5 * (g0[:, None] + g0[None, :]) + 2 * (g2[:, None] + g2[None, :]) * (1 - np.eye(N))
    # vec(P) row-major: d vec(P)/dt = (-i (M kron 1 - 1 kron M^T) - diag(decay)) vec(P)
    Id = np.eye(N)
    K = -1j * (np.kron(M, Id) - np.kron(Id, M.T)) - np.diag(decay.reshape(-1))
    P0 = np.zeros((N, N), dtype=np.complex128)
    P0[site0, site0] = 1.0
    z1s, z2s = [], []
    for t in times:
        P = (scipy.linalg.expm(t * K) @ P0.reshape(-1)).reshape(N, N)
        d = np.real(np.diag(P))
        z1s.append(1 - 2 * d)
        z2s.append(np.array([1 - 2 * (d[i] + d[j]) for i in range(N) for j in range(i + 1, N)]))
    return np.array(z1s), np.array(z2s)


def one_excitation_P(model, site0, t):
    """The one-body matrix P_jk(t) = <j| rho(t) |k> of the one-excitation sector;
    <sx_j sx_k + sy_j sy_k> = 4 Re P_jk and <sx_j sy_k - sy_j sx_k> = -4 Im P_jk."""
    N = model["N"]
    M = np.diag(-np.asarray(model["hz"], dtype=np.complex128))
    for b, (i, j) in enumerate(model["bonds"]):
        M[i, j] += model["J"][b]
        M[j, i] += model["J"][b]
    g0 = np.asarray(model["g0"])
    g2 = np.asarray(model["g2"])
    decay = 0.5 * (g0[:, None] + g0[None, :]) + 2 * (g2[:, None] + g2[None, :]) * (1 - np.eye(N))
    Id = np.eye(N)
    K = -1j * (np.kron(M, Id) - np.kron(Id, M.T)) - np.diag(decay.reshape(-1))
    P0 = np.zeros((N, N), dtype=np.complex128)
    P0[site0, site0] = 1.0
    return (scipy.linalg.expm(t * K) @ P0.reshape(-1)).reshape(N, N)
