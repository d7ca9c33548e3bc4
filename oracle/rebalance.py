"""Particle rebalancing on non-uniform grids, toward a constant number of
particles per cell (Section 3d names it as the way to turn the smaller cell
count of a refined grid into a speed-up; the paper gives no algorithm).

Test infrastructure only (see ``oracle/__init__.py``).

Readings (the builder's design; the paper is silent):

* Weights.  A particle of weight class c (0-7) carries the weight W 2^(c-4).
  Powers of two keep the fixed-point deposit exact: the deposit adds the
  particle's S1 weights shifted by c - 4 + u, in units of W 2^-u (u = 4 for
  a rebalanced discharge).  The FP32 state form only.
* When.  On demand, between steps, on the state (x^k, v^{k-1/2}) at step k.
* Which cells.  Per species, with n_j the particles in cell j and P the
  target: cells with n_j > 2P merge, cells with 0 < n_j < P/2 split.
* Merge.  In a merging cell the particles of class c < 7 are grouped by
  (class, velocity bin floor(vx / dv)), each group taken in increasing id
  order, and every full quadruple (ids a < b < c < d) becomes two particles
  of class c + 1 at the quadruple's mean offset, with velocities
  v_mean +- delta e: delta^2 = <|v|^2> - |v_mean|^2 and e the unit vector of
  v_d - v_a (else v_c - v_b, else x).  Weight is conserved exactly, momentum
  and kinetic energy up to rounding.  The two keep the ids and candidate steps
  of a and b; c and d are removed.
* Split.  In a splitting cell every particle of class c > 0 becomes two of
  class c - 1 at the same position and velocity: itself, and a child whose id
  is Philox words 0-1 of (key = parent id, counter = (k, TAG_SPLIT | s << 8,
  seed)) and whose first candidate step is drawn as for a particle created at
  step k (base k).
* Velocity bins.  dv = rebalance_dv_e / rebalance_dv_i, or 0.25 sqrt(e T / m)
  with the configuration's initial temperature of the species; bin indices
  are clipped to [-128, 127].
"""
from __future__ import annotations

import math

import numpy as np

from . import physics as ph
from .pic import FP64, Species, WC_UNIT, draw, ids_from_words, next_candidate

TAG_SPLIT = 8
WC_MAX = 7


def default_dv(cfg, s):
    """Velocity bin width of species s (m/s)."""
    given = float(cfg["rebalance_dv_e"] if s == 0 else cfg["rebalance_dv_i"])
    if given > 0.0:
        return given
    t = float(cfg["te_ev"] if s == 0 else cfg["ti_ev"])
    m = ph.SPECIES[s][1]
    return 0.25 * math.sqrt(max(t, 1e-6) * ph.QE / m)


def velocity_bin(vx, dv):
    return np.clip(np.floor(np.asarray(vx, dtype=np.float64) / dv), -128, 127).astype(np.int64)


def merge_quadruples(v, off):
    """v: (4, 3, M) FP64 velocities of M quadruples in id order; off: (4, M)
    FP64 offsets.  Returns (va, vb) (3, M) FP64 and the mean offset as FP32."""
    S = ((v[0] + v[1]) + v[2]) + v[3]
    vbar = S * 0.25
    e = [(v[i][0] * v[i][0] + v[i][1] * v[i][1]) + v[i][2] * v[i][2] for i in range(4)]
    E2 = ((e[0] + e[1]) + e[2]) + e[3]
    d2 = E2 * 0.25 - ((vbar[0] * vbar[0] + vbar[1] * vbar[1]) + vbar[2] * vbar[2])
    delta = np.sqrt(np.maximum(d2, 0.0))
    d = v[3] - v[0]
    n2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    alt = v[2] - v[1]
    n2b = (alt[0] * alt[0] + alt[1] * alt[1]) + alt[2] * alt[2]
    use_alt = n2 == 0.0
    d = np.where(use_alt, alt, d)
    n2 = np.where(use_alt, n2b, n2)
    none = n2 == 0.0
    d = np.where(none, np.array([[1.0], [0.0], [0.0]]), d)
    n2 = np.where(none, 1.0, n2)
    nn = np.sqrt(n2)
    u = d / nn
    va = vbar + delta * u
    vb = vbar - delta * u
    ob = ((((off[0] + off[1]) + off[2]) + off[3]) * 0.25).astype(np.float32)
    ob = np.minimum(ob, np.nextafter(np.float32(1.0), np.float32(0.0)))
    return va, vb, ob


def rebalance_species(sp: Species, N, P, dv, k, seed, nudt):
    """One species' particles after a rebalancing pass (a new Species) and
    the numbers of merges and splits."""
    assert sp.prec != FP64, "rebalancing needs the FP32 state form"
    cell = sp.cell.astype(np.int64)
    wc = sp.classes().astype(np.int64).copy()
    n = np.bincount(cell, minlength=N)
    merge_c = n > 2 * P
    split_c = (n > 0) & (2 * n < P)
    vx = sp.vx.astype(np.float32).copy()
    vy = sp.vy.astype(np.float32).copy()
    vz = sp.vz.astype(np.float32).copy()
    off = sp.off.astype(np.float32).copy()
    keep = np.ones(sp.n, dtype=bool)
    # merges
    elig = np.nonzero(merge_c[cell] & (wc < WC_MAX))[0]
    vb = velocity_bin(vx[elig], dv)
    order = elig[np.lexsort((sp.id[elig], vb, wc[elig], cell[elig]))]
    vbo = velocity_bin(vx[order], dv)
    key = (cell[order] * 8 + wc[order]) * 256 + (vbo + 128)
    n_merge = 0
    if len(order):
        head = np.r_[True, key[1:] != key[:-1]]
        gid = np.cumsum(head) - 1
        gstart = np.nonzero(head)[0]
        gsize = np.diff(np.r_[gstart, len(order)])
        pos = np.arange(len(order)) - gstart[gid]
        lead = np.nonzero((pos % 4 == 0) & (pos + 4 <= gsize[gid]))[0]
        q = [order[lead + i] for i in range(4)]
        n_merge = len(lead)
        if n_merge:
            v = np.array([[vx[qi].astype(np.float64), vy[qi].astype(np.float64), vz[qi].astype(np.float64)]
                          for qi in q])
            o = np.array([off[qi].astype(np.float64) for qi in q])
            va, vbb, ob = merge_quadruples(v, o)
            for dst, vv in ((q[0], va), (q[1], vbb)):
                vx[dst] = vv[0].astype(np.float32)
                vy[dst] = vv[1].astype(np.float32)
                vz[dst] = vv[2].astype(np.float32)
                off[dst] = ob
                wc[dst] += 1
            keep[q[2]] = False
            keep[q[3]] = False
    # splits
    parents = np.nonzero(split_c[cell] & (wc > 0))[0]
    wc[parents] -= 1
    out = Species(s=sp.s, prec=sp.prec, vx=vx, vy=vy, vz=vz, id=sp.id.copy(), knext=sp.knext.copy(),
                  cell=sp.cell.copy(), off=off, wc=wc.astype(np.uint8))
    children = None
    if len(parents):
        c0, c1, _, _ = draw(sp.id[parents], k, TAG_SPLIT, sp.s, seed)
        cid = ids_from_words(c0, c1)
        children = Species(s=sp.s, prec=sp.prec, vx=vx[parents].copy(), vy=vy[parents].copy(),
                           vz=vz[parents].copy(), id=cid, knext=next_candidate(cid, k - 1, sp.s, seed, nudt),
                           cell=sp.cell[parents].copy(), off=off[parents].copy(),
                           wc=wc[parents].astype(np.uint8))
    out = out.subset(keep)
    return out.append(children), n_merge, len(parents)


def rebalance(sim):
    """Rebalance every species of an oracle Sim in place; returns
    [(merges, splits) per species]."""
    P = int(sim.cfg["rebalance_ppc"])
    assert P > 0, "rebalance_ppc must be set"
    out = []
    for s in range(sim.nsp):
        sp, nm, ns = rebalance_species(sim.sp[s], sim.grid.N, P, default_dv(sim.cfg, s), sim.k,
                                       sim.seed, sim.nudt[s])
        sim.sp[s] = sp
        out.append((nm, ns))
    return out
