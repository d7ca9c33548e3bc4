"""Synthetic workloads (argon RF-CCP discharges) as configuration dictionaries.

The paper's runs are helium with tabulated cross sections (Table 1), which are
not available here; these argon discharges with analytic cross sections stand
in for them, at the sizes of the five benchmark workloads:

1. ``small``     128 uniform cells over 2.5 cm, 100 + 100 particles per cell,
                 200 V, 50 mTorr, dt = T_RF/400, FP64, EC or MC gather.
2. ``resolved``  512 uniform cells over 3.0 cm, 512 particles per cell per
                 species at 3e15 m^-3, 300 V, 30 mTorr, dt = T_RF/800; the
                 ``coarse`` variant has 64 cells and the same particle count.
3. ``large``     the paper's 0.3 m gap (Table 1) on a 2048-cell refined grid
                 (max/min cell ratio 8, buffers of about 5 cm as in Section 3c),
                 32 M electrons + 32 M ions at 7e15 m^-3 and 2.585 eV, 400 V,
                 20 mTorr, dt = T_RF/1000, FP32 state, sort every 20 steps.
4. ``sweep``     256 independent discharges with random grids (64-1024 cells),
                 particle counts (5e4-2e6, log-uniform), voltages, pressures and
                 time steps, drawn from seed 13092.
5. ``stream``    a Poisson-arrival request trace (mean 20/s, seed 13093) of
                 discharges with 64-2048 cells and 1e5-8e6 particles, run for
                 50-500 RF cycles each.
"""
from __future__ import annotations

import math

import numpy as np

F_RF = 13.56e6
T_RF = 1.0 / F_RF
MTORR = 133.322368e-3  # Pa


def base(**over):
    cfg = dict(n_cells=128, bc=0, nodes=None, gap_m=0.025, v_rf=200.0, f_rf=F_RF, phase=0.0,
               p_pa=50.0 * MTORR, t_gas_k=300.0, n0_m3=1e15, te_ev=2.0, ti_ev=0.026,
               n_per_species=12800, capacity=0, weight_m2=0.0, dt_s=T_RF / 400, gather=0,
               precision=0, gamma_see=0.1, t_see_ev=2.0, seed=1, sort_interval=50, n_species=2,
               collisions=1, pullback=0, nu_max_e=0.0, nu_max_i=0.0, avg_start=0, avg_every=0,
               eedf_every=0, eedf_bins=200, eedf_emax_ev=50.0, eedf_width_m=1e-3, k_stop=0,
               growth_limit=0.0, moments=0)
    cfg.update(over)
    return cfg


def small(gather=0, seed=1, precision=0, **over):
    """Workload 1: 128 cells, 25.6 k particles, 2000 steps of T_RF/400."""
    return base(gather=gather, seed=seed, precision=precision, **over)


SMALL_STEPS = 2000


def resolved(precision=1, n_cells=512, seed=2, **over):
    """Workload 2: 512 cells (or 64), 262 144 particles per species."""
    return base(n_cells=n_cells, gap_m=0.03, n0_m3=3e15, v_rf=300.0, p_pa=30.0 * MTORR,
                n_per_species=262144, dt_s=T_RF / 800, precision=precision, seed=seed,
                sort_interval=20, **over)


RESOLVED_STEPS = 16000


def large_grid_nodes(L=0.3):
    """2048 cells: 818 of L/4912 at each electrode (about 5 cm), one cell each of
    2x and 4x that width, and 408 cells of 8x in the centre (rules of Section 3c)."""
    d = L / 4912.0
    sizes = [1] * 818 + [2, 4] + [8] * 408 + [4, 2] + [1] * 818
    units = np.concatenate([[0], np.cumsum(sizes)])
    nodes = units.astype(np.float64) * d
    nodes[-1] = L
    return nodes


def large(n_per_species=32_000_000, precision=1, seed=3, **over):
    """Workload 3: 0.3 m gap, 2048 refined cells, 32 M + 32 M particles, FP32 state."""
    return base(n_cells=2048, nodes=large_grid_nodes(), gap_m=0.3, n0_m3=7e15, te_ev=2.585,
                v_rf=400.0, p_pa=20.0 * MTORR, n_per_species=n_per_species,
                capacity=int(n_per_species * 1.25) + 65536, dt_s=T_RF / 1000,
                precision=precision, seed=seed, sort_interval=20, **over)


LARGE_STEPS = 5000


def large_rebalanced(n_per_species=32_000_000, precision=1, seed=3, every=1000, **over):
    """Workload 3 with particle rebalancing (Section 3d): the target count per
    cell is the initial count of the narrowest cells (n_per_species / 4912),
    so the sheath keeps its particles per cell while the 8x wider centre cells
    are merged toward the same count; a pass runs every ``every`` steps."""
    ppc = max(1, int(round(n_per_species / 4912.0)))
    return large(n_per_species=n_per_species, precision=precision, seed=seed, rebalance_ppc=ppc,
                 rebalance_every=every, **over)


def sweep(n=256, master_seed=13092, precision=1, scale=1.0):
    """Workload 4: n independent discharges drawn from a master seed."""
    g = np.random.Generator(np.random.PCG64(master_seed))
    out = []
    for i in range(n):
        cells = int(g.integers(64, 1025))
        npart = int(math.exp(g.uniform(math.log(5e4), math.log(2e6))) * scale)
        per = max(256, npart // 2)
        v = float(g.uniform(100.0, 500.0))
        p = float(g.uniform(10.0, 100.0))
        div = int(g.integers(400, 1001))
        out.append(base(n_cells=cells, gap_m=0.025, n0_m3=1e15, v_rf=v, p_pa=p * MTORR,
                        n_per_species=per, dt_s=T_RF / div, precision=precision,
                        seed=master_seed + i, sort_interval=20))
    return out


def stream(n=256, master_seed=13093, rate=20.0, precision=1, scale=1.0, cycles=(50, 500),
           headroom=8):
    """Workload 5: (arrival time, config, steps) of n requests.

    A served discharge starts at 1e15 m^-3 and, at high pressure and voltage,
    ionises its way to a density several times higher over its hundreds of RF
    cycles; each request's particle capacity is ``headroom`` times its initial
    count, so that such growth fits (a request that still outgrows it ends
    with PIC_ECAPACITY)."""
    g = np.random.Generator(np.random.PCG64(master_seed))
    t = 0.0
    out = []
    for i in range(n):
        t += float(g.exponential(1.0 / rate))
        cells = int(g.integers(64, 2049))
        npart = int(math.exp(g.uniform(math.log(1e5), math.log(8e6))) * scale)
        per = max(256, npart // 2)
        v = float(g.uniform(100.0, 500.0))
        p = float(g.uniform(10.0, 100.0))
        div = int(g.integers(400, 1001))
        ncyc = int(g.integers(cycles[0], cycles[1] + 1))
        steps = ncyc * div
        cfg = base(n_cells=cells, gap_m=0.025, n0_m3=1e15, v_rf=v, p_pa=p * MTORR,
                   n_per_species=per, capacity=headroom * per + 4096, dt_s=T_RF / div,
                   precision=precision, seed=master_seed + i,
                   sort_interval=20, avg_every=1, avg_start=max(0, steps - 10 * div),
                   eedf_every=max(1, div // 10), k_stop=steps)
        out.append((t, cfg, steps))
    return out
