"""Seeded synthetic workloads: driven-dissipative qubit chains of the model of
Eqs. (H0), (K_def), (D0)-(D2) of Landa & Misguich, arXiv:2203.05871.

This module only *draws parameters*: it holds no arithmetic of the method (no
generators, no gates, no contractions).  Both the FP64 oracle and the HIP path
consume the same dictionaries, so that their inputs are identical bit for bit.

A model dictionary has the keys
    N      number of qubits
    bonds  int32 array [n_bonds, 2], coupled pairs (i, j) with i < j
    J, Jz  float64 [n_bonds], flip-flop and Ising couplings of Eq. (K_def),
           one term per unordered bond
    hx, hy, hz, g0, g1, g2   float64 [N], on-site fields of Eq. (H0) and the
           rates of the three dissipators Eqs. (D0), (D1), (D2)
and a run dictionary has
    tau, steps, chi_max, cutoff, init ("+z", "-x", ... or a list of N such)

The driven-edge setup follows Sec. 3.1 (Eq. h_xi_hz_i): qubit 0 carries the
drive h_x = Omega, and h_z alternates 0 / Delta with the driven site at 0.
"""
from __future__ import annotations

import numpy as np


def chain_model(N, J, hz, hx0, g0, g2, g1=0.0, Jz=0.0):
    """Open chain with nearest-neighbour bonds (i, i+1)."""
    N = int(N)
    bonds = np.stack([np.arange(N - 1), np.arange(1, N)], axis=1).astype(np.int32)
    nb = N - 1
    hx = np.zeros(N)
    hx[0] = hx0
    return {
        "N": N,
        "bonds": bonds,
        "J": np.broadcast_to(np.asarray(J, dtype=np.float64), (nb,)).copy(),
        "Jz": np.broadcast_to(np.asarray(Jz, dtype=np.float64), (nb,)).copy(),
        "hx": hx,
        "hy": np.zeros(N),
        "hz": np.broadcast_to(np.asarray(hz, dtype=np.float64), (N,)).copy(),
        "g0": np.full(N, float(g0)),
        "g1": np.full(N, float(g1)),
        "g2": np.full(N, float(g2)),
    }


def alternating(N, delta):
    """h_z = Delta * (i mod 2): the driven site 0 sits at 0 detuning."""
    return float(delta) * (np.arange(N) % 2)


def chain6_exact():
    """N=6 chain, chi_max=64 = 4^3 (exact, no truncation), tau=0.01, 100 steps."""
    m = chain_model(6, 1.0, alternating(6, 5.0), 1.0, 0.1, 0.05)
    run = {"tau": 0.01, "steps": 100, "chi_max": 64, "cutoff": 0.0, "init": "+z"}
    return m, run


def jittered_chain(N, seed=0):
    """Alternating 0/5 detunings plus N(0, 0.1^2) jitter, then J ~ U[0.8, 1.2].

    Draw order: first the N detuning jitters, then the N-1 couplings."""
    rng = np.random.default_rng(seed)
    hz = alternating(N, 5.0) + 0.1 * rng.standard_normal(N)
    J = rng.uniform(0.8, 1.2, N - 1)
    return chain_model(N, J, hz, 1.0, 0.1, 0.05)


def chain20_jittered():
    """N=20 jittered chain, chi_max=128, cutoff 1e-12, tau=0.05, 100 steps."""
    m = jittered_chain(20, 0)
    run = {"tau": 0.05, "steps": 100, "chi_max": 128, "cutoff": 1e-12, "init": "+z"}
    return m, run


def chain30_jittered(init="+x"):
    """N=30 jittered chain, chi_max=256, cutoff 1e-10, tau=0.05, 50 steps.

    init "+x" (a global quench) makes chi=256 bind in the bulk; "+z" is the
    edge-driven variant in which most of the chain stays near product."""
    m = jittered_chain(30, 0)
    run = {"tau": 0.05, "steps": 50, "chi_max": 256, "cutoff": 1e-10, "init": init}
    return m, run


def chains64_uneven(n_chains=64, seed=0):
    """Independent chains: per chain, in order, N ~ U{8..24}, Omega ~ U[0.5, 2],
    Delta ~ U[2, 8]; J=1, g0=0.1, g2=0.05; chi_max=64, cutoff 1e-12."""
    rng = np.random.default_rng(seed)
    chains = []
    for _ in range(n_chains):
        N = int(rng.integers(8, 25))
        omega = float(rng.uniform(0.5, 2.0))
        delta = float(rng.uniform(2.0, 8.0))
        chains.append(chain_model(N, 1.0, alternating(N, delta), omega, 0.1, 0.05))
    run = {"tau": 0.05, "steps": 40, "chi_max": 64, "cutoff": 1e-12, "init": "+z"}
    return chains, run


def ladder_model(n_rungs=8, J=1.0, delta=5.0, omega=1.0, g0=0.1, g2=0.05):
    """2 x n_rungs ladder on the zigzag path s = 2r + l (rung r, leg l).

    Rungs (2r, 2r+1) and legs (s, s+2); h_z is a checkerboard Delta*((r+l) mod 2)."""
    N = 2 * n_rungs
    bonds = [(2 * r, 2 * r + 1) for r in range(n_rungs)]
    bonds += [(s, s + 2) for s in range(N - 2)]
    bonds = np.array(sorted(bonds), dtype=np.int32)
    r = np.arange(N) // 2
    leg = np.arange(N) % 2
    hx = np.zeros(N)
    hx[0] = omega
    return {
        "N": N,
        "bonds": bonds,
        "J": np.full(len(bonds), float(J)),
        "Jz": np.zeros(len(bonds)),
        "hx": hx,
        "hy": np.zeros(N),
        "hz": float(delta) * ((r + leg) % 2),
        "g0": np.full(N, float(g0)),
        "g1": np.zeros(N),
        "g2": np.full(N, float(g2)),
    }


def ladder2x8():
    """2 x 8 ladder (N = 16, 8 rungs, 14 legs two sites apart on the path),
    chi_max = 128, cutoff 1e-12, tau = 0.05, 40 steps, init +z."""
    m = ladder_model(8)
    run = {"tau": 0.05, "steps": 40, "chi_max": 128, "cutoff": 1e-12, "init": "+z"}
    return m, run


def random_model(N, seed, bonds=None, zz=True, all_fields=True):
    """A generic model with every term switched on (for coverage tests)."""
    rng = np.random.default_rng(seed)
    if bonds is None:
        bonds = np.stack([np.arange(N - 1), np.arange(1, N)], axis=1)
    bonds = np.asarray(bonds, dtype=np.int32)
    nb = len(bonds)
    u = lambda lo, hi, n: rng.uniform(lo, hi, n)
    return {
        "N": int(N),
        "bonds": bonds,
        "J": u(0.5, 1.5, nb),
        "Jz": u(-0.5, 0.5, nb) if zz else np.zeros(nb),
        "hx": u(-1, 1, N) if all_fields else np.zeros(N),
        "hy": u(-1, 1, N) if all_fields else np.zeros(N),
        "hz": u(-2, 2, N),
        "g0": u(0.0, 0.2, N),
        "g1": u(0.0, 0.1, N) if all_fields else np.zeros(N),
        "g2": u(0.0, 0.1, N),
    }


def random_block(m, n, seed, decay=0.0):
    """Seeded complex Gaussian m x n matrix; with decay > 0 its singular values
    are reshaped to fall off as exp(-decay * j) (for truncation tests)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    if decay > 0.0:
        q1, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
        q2, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        k = min(m, n)
        s = np.exp(-decay * np.arange(k))
        a = (q1[:, :k] * s) @ q2[:k, :]
    return a
