"""Seeded synthetic inputs shared by the HIP path's tests, the oracle's tests and the bench.

This module holds no step of the method: only workload parameters, seeded random states and
the synthetic quasi-particle-weight table that stands in for the paper's self-energy-derived
Z (whose values the paper does not print). It imports nothing from the HIP binding or from
the oracle.

Workloads (square lattice, t = 1, t' = 0, mu = 0, i.e. half filling with perfect nesting as
in Sec. 3 of the paper; initial condition V = U; stop when max|V| > 20 t; T_end = 0.01 t):

  C1  N=16,  L=32,  U=2,   RK4 with 200 steps in ln T, no Z feedback, FP64
  C2  N=48,  L=128, U=3,   Dormand-Prince in ln T, synthetic Z table, FP32 loop integrals
  C3  N=96,  L=256, U=3,   Dormand-Prince, no Z, BF16 operands with FP32 accumulation
  C4  64 flows, U in {1.0,1.5,...,4.5} x T0_i = 0.5*4^(i/7), N=48, L=128, FP32, ragged
  C5  16 flows, U_i = 1 + 3i/15, N=128, L=512, synthetic Z (per-flow U), BF16 contraction
  shells  energy-shell patching as in the paper's 224-patch runs: 7 shells x 32 sectors,
      L=128, U=3, Dormand-Prince, no Z, FP32
"""
from __future__ import annotations

import math

import numpy as np

SEED = 20050827

WORKLOADS = {
    "C1": dict(N=16, L=32, U=[2.0], T0=[1.0], T_end=0.01, integrator="rk4", n_steps=200,
               z=False, precision="fp64"),
    "C2": dict(N=48, L=128, U=[3.0], T0=[1.0], T_end=0.01, integrator="rk45", n_steps=200,
               z=True, precision="fp32"),
    "C3": dict(N=96, L=256, U=[3.0], T0=[1.0], T_end=0.01, integrator="rk45", n_steps=200,
               z=False, precision="bf16"),
    "C4": dict(N=48, L=128,
               U=[1.0 + 0.5 * u for u in range(8) for _ in range(8)],
               T0=[0.5 * 4.0 ** (i / 7.0) for _ in range(8) for i in range(8)],
               T_end=0.01, integrator="rk45", n_steps=200, z=False, precision="fp32"),
    "C5": dict(N=128, L=512, U=[1.0 + 3.0 * i / 15.0 for i in range(16)], T0=[1.0] * 16,
               T_end=0.01, integrator="rk45", n_steps=200, z=True, precision="bf16"),
    "shells": dict(N=224, n_shells=7, L=128, U=[3.0], T0=[1.0], T_end=0.01, integrator="rk45",
                   n_steps=200, z=False, precision="fp32"),
}


def workload(name: str) -> dict:
    w = dict(WORKLOADS[name])
    w["name"] = name
    return w


def constant_state(N: int, U: float) -> np.ndarray:
    """s0: the initial condition V = U."""
    return np.full((N, N, N), float(U), np.float64)


def noisy_state(N: int, U: float, seed: int = SEED, rel: float = 0.1) -> np.ndarray:
    """s1: V = U (1 + rel * eps), eps ~ N(0, 1), seeded."""
    rng = np.random.default_rng(seed)
    return float(U) * (1.0 + rel * rng.standard_normal((N, N, N)))


def random_state(N: int, seed: int = SEED, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((N, N, N))


def sample_indices(N: int, n: int, seed: int = SEED) -> np.ndarray:
    """n random output indices (a, b, c), always including the corners."""
    rng = np.random.default_rng(seed)
    abc = rng.integers(0, N, size=(n, 3)).astype(np.int32)
    abc[0] = (0, 0, 0)
    if n > 1:
        abc[1] = (N - 1, N - 1, N - 1)
    return abc


def sector_centres(N: int) -> np.ndarray:
    """Angles of the patch centres (theta_off + 2 pi a / N)."""
    off = 0.0 if (N == 1 or N % 8 == 0) else math.pi / N
    return off + 2.0 * math.pi * np.arange(N) / N


def synthetic_z_table(N: int, U: float, T0: float, T_end: float, lam: float = 0.02,
                      eta: float = 0.1, n_nodes: int = 33):
    """Synthetic per-patch quasi-particle weights on n_nodes ln T nodes over [T_end, T0]:

        Z_a(T) = 1 / (1 + lam U^2 (1 + eta cos 4 theta_a) (1 + ln(T0/T) / (2 ln(T0/T_end))))

    Nearly angle independent and slowly decreasing along the flow (the paper reports Z that
    varies little along the Fermi surface, Sec. 3.2), between 0.77 and 0.86 at U = 3.
    Returns (lnT nodes ascending [n_nodes], table [n_nodes, N])."""
    lnT = np.linspace(math.log(T_end), math.log(T0), n_nodes)
    th = sector_centres(N)
    frac = np.log(T0 / np.exp(lnT)) / math.log(T0 / T_end)
    table = 1.0 / (1.0 + lam * U * U * (1.0 + eta * np.cos(4.0 * th))[None, :] *
                   (1.0 + 0.5 * frac)[:, None])
    return lnT, np.ascontiguousarray(table)
