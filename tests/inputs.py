"""Seeded synthetic inputs shared by the oracle and the GPU side of the tests.

This module holds no arithmetic of the method: it only draws random grids,
particle states and parameter sets from numpy's PCG64 with fixed seeds.
"""
from __future__ import annotations

import math

import numpy as np

MTORR = 133.322368e-3   # Pa per mTorr
F_RF = 13.56e6


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def random_nodes(L, N, seed, max_ratio=1.8):
    """N+1 increasing nodes on [0, L] with neighbouring cells within max_ratio."""
    g = rng(seed)
    h = np.empty(N)
    h[0] = 1.0
    for j in range(1, N):
        h[j] = h[j - 1] * math.exp(g.uniform(-math.log(max_ratio), math.log(max_ratio)))
        h[j] = min(max(h[j], 0.25), 4.0)
    nodes = np.concatenate([[0.0], np.cumsum(h)])
    nodes *= L / nodes[-1]
    nodes[-1] = L
    return nodes


def unique_ids(n, seed):
    g = rng(seed)
    ids = g.integers(0, 2 ** 63, size=2 * n + 16, dtype=np.int64).astype(np.uint64)
    ids = np.unique(ids)
    g.shuffle(ids)
    return ids[:n].copy()


def particles_fp64(n, L, vscale, seed, k=0, knext_spread=8):
    """Positions uniform on [0, L), Gaussian velocities of rms ``vscale`` per
    component, unique 63-bit ids, candidate steps in [k, k + knext_spread)."""
    g = rng(seed)
    x = g.uniform(0.0, L, size=n)
    x = np.minimum(x, np.nextafter(L, 0.0))
    v = g.normal(0.0, vscale, size=(3, n))
    knext = g.integers(k, k + knext_spread, size=n).astype(np.int64)
    return dict(x=x, vx=v[0].copy(), vy=v[1].copy(), vz=v[2].copy(),
                id=unique_ids(n, seed + 1), knext=knext)


def particles_fp32(n, N, vscale, seed, k=0, knext_spread=8):
    """Cells uniform on [0, N), offsets uniform on [0, 1) in float32, float32
    Gaussian velocities, unique ids, candidate steps in [k, k + knext_spread)."""
    g = rng(seed)
    cell = g.integers(0, N, size=n).astype(np.int32)
    off = g.uniform(0.0, 1.0, size=n).astype(np.float32)
    off = np.minimum(off, np.nextafter(np.float32(1.0), np.float32(0.0)))
    v = g.normal(0.0, vscale, size=(3, n)).astype(np.float32)
    knext = g.integers(k, k + knext_spread, size=n).astype(np.int64)
    return dict(cell=cell, off=off, vx=v[0].copy(), vy=v[1].copy(), vz=v[2].copy(),
                id=unique_ids(n, seed + 1), knext=knext)


def small_discharge(**over):
    """A small argon CCP (the 128-cell, 2.5 cm, 200 V, 50 mTorr case at reduced
    particle count) used by the parity tests."""
    cfg = dict(n_cells=128, bc=0, nodes=None, gap_m=0.025, v_rf=200.0, f_rf=F_RF, phase=0.0,
               p_pa=50.0 * MTORR, t_gas_k=300.0, n0_m3=1e15, te_ev=2.0, ti_ev=0.026,
               n_per_species=12800, weight_m2=0.0, dt_s=1.0 / (400 * F_RF), gather=0,
               precision=0, gamma_see=0.1, t_see_ev=2.0, seed=1, n_species=2, collisions=1,
               pullback=0, nu_max_e=0.0, nu_max_i=0.0, avg_start=0, avg_every=0, eedf_every=0,
               eedf_bins=200, eedf_emax_ev=50.0, eedf_width_m=1e-3)
    cfg.update(over)
    return cfg
