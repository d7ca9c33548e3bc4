"""Helpers shared by the GPU parity tests: moving one seeded state into both the
oracle and the HIP library, and comparing particle sets by id."""
from __future__ import annotations

import numpy as np

from oracle import physics as ph
from oracle.pic import FP32, FP64, Species
from oracle.sim import Sim


def oracle_species(state, s, prec):
    kw = dict(s=s, prec=prec, vx=np.array(state["vx"]), vy=np.array(state["vy"]),
              vz=np.array(state["vz"]), id=np.array(state["id"], dtype=np.uint64),
              knext=np.array(state["knext"], dtype=np.int64))
    if prec == FP64:
        kw["x"] = np.array(state["x"], dtype=np.float64)
        for f in ("vx", "vy", "vz"):
            kw[f] = kw[f].astype(np.float64)
    else:
        kw["cell"] = np.array(state["cell"], dtype=np.int32)
        kw["off"] = np.array(state["off"], dtype=np.float32)
        for f in ("vx", "vy", "vz"):
            kw[f] = kw[f].astype(np.float32)
    return Species(**kw)


def oracle_from_states(cfg, states, k):
    prec = int(cfg["precision"])
    sps = [oracle_species(st, s, prec) for s, st in enumerate(states)]
    return Sim(cfg, species=sps, k=k)


def gpu_from_states(cfg, states, k, Context):
    ctx = Context([cfg])
    for s, st in enumerate(states):
        ctx.set_state(0, s, st)
    ctx.set_step(0, k)
    return ctx


def species_dict(sp):
    d = dict(vx=sp.vx, vy=sp.vy, vz=sp.vz, id=sp.id, knext=sp.knext)
    if sp.prec == FP64:
        d["x"] = sp.x
    else:
        d["cell"] = sp.cell
        d["off"] = sp.off
    return d


def by_id(d):
    o = np.argsort(d["id"], kind="stable")
    return {k: np.asarray(v)[o] for k, v in d.items()}


def positions(d, grid):
    if "x" in d:
        return np.asarray(d["x"], dtype=np.float64)
    return grid.position(d["cell"], d["off"])


def compare_species(gpu, ref, grid, rel_x, rel_v, vscale, max_flips):
    """Match by id; count particles present on one side only or outside the
    tolerance (branch flips).  Returns a dict of statistics; asserts the flip
    count and the agreement of everything else."""
    g = by_id(gpu)
    r = by_id(ref)
    common, gi, ri = np.intersect1d(g["id"], r["id"], return_indices=True)
    only = (len(g["id"]) - len(common)) + (len(r["id"]) - len(common))
    xg = positions({k: v[gi] for k, v in g.items()}, grid)
    xr = positions({k: v[ri] for k, v in r.items()}, grid)
    dx = np.abs(xg - xr)
    dv = np.zeros(len(common))
    for f in ("vx", "vy", "vz"):
        dv = np.maximum(dv, np.abs(g[f][gi].astype(np.float64) - r[f][ri].astype(np.float64)))
    bad_x = dx > rel_x * grid.L
    bad_v = dv > rel_v * vscale
    bad_k = g["knext"][gi].astype(np.int64) != np.minimum(r["knext"][ri], 2 ** 31 - 1)
    bad = bad_x | bad_v | bad_k
    flips = only + int(bad.sum())
    stats = dict(n_gpu=len(g["id"]), n_ref=len(r["id"]), common=len(common), only=only,
                 bad_x=int(bad_x.sum()), bad_v=int(bad_v.sum()), bad_k=int(bad_k.sum()),
                 max_dx=float(dx.max()) if len(dx) else 0.0,
                 max_dv=float(dv[~bad].max()) if (~bad).any() else 0.0)
    assert flips <= max_flips, stats
    return stats


def normwise(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def vscale_of(state, s, E_max, qmdt_abs):
    v = np.abs(np.asarray(state["vx"], dtype=np.float64))
    return float(v.max()) + qmdt_abs * E_max + 1.0


def qmdt_abs(cfg, s):
    q, m = ph.SPECIES[s]
    return abs(q / m * cfg["dt_s"])
