"""Pins of the oracle's gather and leapfrog push (Eqs 6-9) in both state forms."""
import math

import numpy as np
import pytest

import inputs
from oracle import physics as ph
from oracle.pic import (BC_PERIODIC, FP32, FP64, Grid, Species, push_fp32, to_fp32_state)
from oracle.sim import Sim


def single_particle_sim(prec, uniform, species_index, x0, v0, V=200.0, L=0.025, N=64):
    nodes = None if uniform else inputs.random_nodes(L, N, seed=21)
    cfg = inputs.small_discharge(n_cells=N, nodes=nodes, gap_m=L, v_rf=V, f_rf=0.0,
                                 phase=math.pi / 2, weight_m2=1e-20, collisions=0, n_species=2,
                                 precision=prec, gamma_see=0.0)
    g = Grid.make(L, N, nodes)
    one = np.array([x0])
    sps = []
    for s in range(2):
        n = 1 if s == species_index else 0
        kw = dict(s=s, prec=prec, vx=np.full(n, v0), vy=np.zeros(n), vz=np.zeros(n),
                  id=np.arange(n, dtype=np.uint64), knext=np.full(n, 2 ** 31 - 1, dtype=np.int64))
        if prec == FP64:
            kw["x"] = one[:n].copy()
        else:
            c, o = to_fp32_state(g, one[:n])
            kw.update(cell=c, off=o)
            for f in ("vx", "vy", "vz"):
                kw[f] = kw[f].astype(np.float32)
        sps.append(Species(**kw))
    return Sim(cfg, species=sps)


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("uniform", [True, False])
@pytest.mark.parametrize("s", [0, 1])
def test_single_particle_in_uniform_field(prec, uniform, s):
    """a = q V / (m L): v^{k-1/2} = v^{-1/2} + k a dt and
    x^k = x^0 + k dt v^{-1/2} + a dt^2 k (k+1)/2, until absorption."""
    L = 0.025
    V = 200.0 if s == 0 else 2000.0
    q, m = ph.SPECIES[s]
    a = q * (V / L) / m
    dt = 1.0 / (400 * 13.56e6)
    x0 = 0.3 * L
    v0 = 2e5 if s == 0 else 3e3
    sim = single_particle_sim(prec, uniform, s, x0, v0, V=V, L=L)
    tol = 1e-10 if prec == FP64 else 2e-5
    absorbed_at = None
    for k in range(1, 4000):
        sim.step()
        xe = x0 + k * dt * v0 + a * dt * dt * k * (k + 1) / 2
        ve = v0 + k * a * dt
        if sim.sp[s].n == 0:
            absorbed_at = k
            assert xe < 0 or xe >= L or min(abs(xe), abs(xe - L)) < 10 * tol * L
            break
        assert abs(sim.positions(s)[0] - xe) <= tol * L
        # FP32 rounding of v accumulates at most one ulp per step.
        tol_v = tol if prec == FP64 else max(tol, k * 1.2e-7)
        assert abs(float(sim.sp[s].vx[0]) - ve) <= tol_v * (abs(v0) + abs(a * dt) * k)
        assert 0.0 <= xe < L or min(abs(xe), abs(xe - L)) < 10 * tol * L
    assert absorbed_at is not None
    assert sim.absorbed[s].sum() == 1


def walk_reference(g, cell, off, vx, dt):
    """Exact FP64 new position of an FP32-state particle."""
    return g.position(cell, off) + vx.astype(np.float64) * dt


@pytest.mark.parametrize("uniform", [True, False])
def test_fp32_walk_tracks_exact_position(uniform):
    L, N = 0.03, 96
    nodes = None if uniform else inputs.random_nodes(L, N, seed=22)
    g = Grid.make(L, N, nodes)
    dt = 1e-10
    st = inputs.particles_fp32(20000, N, 3e6, seed=23)   # up to ~10 cells per step
    sp = Species(s=0, prec=FP32, vx=st["vx"], vy=st["vy"], vz=st["vz"], id=st["id"],
                 knext=st["knext"], cell=st["cell"], off=st["off"])
    tables = g.walk_tables(dt)
    E32 = np.zeros(N, dtype=np.float32)
    vx, cell, off, wall = push_fp32(g, sp, E32, 0, np.float32(0.0), tables)
    exact = walk_reference(g, st["cell"], st["off"], st["vx"], dt)
    inside = (exact >= 0) & (exact < L)
    live = wall == 0
    hmax = float(np.max(g.h))
    # Away from the walls the walk keeps the particle and lands within FP32 error.
    far = inside & (exact > 1e-4 * L) & (exact < L * (1 - 1e-4))
    assert np.all(live[far])
    err = np.abs(g.position(cell[far], off[far]) - exact[far])
    assert err.max() < 1e-5 * hmax
    assert np.all(wall[(exact < -1e-4 * L)] == -1)
    assert np.all(wall[(exact > L * (1 + 1e-4))] == 1)
    assert np.all((off[live] >= 0) & (off[live] < 1))


def closed_form_uniform_walk(sig):
    """Uniform-grid shortcut: M = floor(sigma), sigma - M in one FP32 op, and a
    final carry when the result rounds to 1.  Bit-identical to the walk."""
    m = np.floor(sig)
    out = (sig - m).astype(np.float32)
    shift = m.astype(np.int64)
    carry = out >= np.float32(1.0)
    out[carry] = np.float32(0.0)
    shift[carry] += 1
    return shift, out


def test_uniform_closed_form_at_the_electrodes_equals_walk_bitwise():
    """A bounded grid: the closed form leaves at the left electrode when
    cell + floor(sigma) < 0, before the carry (a left move from x = 0 smaller
    than half an FP32 ulp rounds sigma + 1 up to 1, but the cell-by-cell walk
    has already left the grid), and at the right one when the carried cell
    reaches N."""
    N = 64
    g = Grid.make(1.0, N)
    tiny = [-1e-30, -2.0 ** -30, -2.0 ** -26, -2.0 ** -25, -3 * 2.0 ** -26, -2.0 ** -24, -0.5, -1.0,
            -1.5, 0.0, 2.0 ** -25, 0.5, 1.0 - 2 ** -24]
    cells, sigs = [], []
    for c in (0, 1, 2, N - 2, N - 1):
        for t in tiny:
            for o in (0.0, 2.0 ** -24, 1.0 - 2 ** -24):
                cells.append(c)
                sigs.append(np.float32(o) + np.float32(t))
    sig = np.array(sigs, dtype=np.float32)
    cell0 = np.array(cells, dtype=np.int32)
    n = len(sig)
    sp = Species(s=0, prec=FP32, vx=np.zeros(n, np.float32), vy=np.zeros(n, np.float32),
                 vz=np.zeros(n, np.float32), id=np.arange(n, dtype=np.uint64),
                 knext=np.zeros(n, np.int64), cell=cell0, off=sig)
    dtoh, rf, rb = g.walk_tables(0.0)
    _, cell, off, wall = push_fp32(g, sp, np.zeros(N, np.float32), 0, np.float32(0.0), (dtoh, rf, rb))
    m = np.floor(sig)
    jj = cell0.astype(np.int64) + m.astype(np.int64)
    out = (sig - m).astype(np.float32)
    left = jj < 0
    carry = ~left & (out >= np.float32(1.0))
    out[carry] = np.float32(0.0)
    jj[carry] += 1
    right = ~left & (jj >= N)
    assert np.array_equal(wall == -1, left) and np.array_equal(wall == 1, right)
    live = wall == 0
    assert np.array_equal(cell[live].astype(np.int64), jj[live])
    assert np.array_equal(off[live].view(np.uint32), out[live].view(np.uint32))
    # the case that needs the order: x = 0 moving left by less than half an ulp
    k = np.nonzero((cell0 == 0) & (sig < 0) & (sig > -2.0 ** -25))[0]
    assert len(k) and np.all(wall[k] == -1)


def test_uniform_closed_form_equals_walk_bitwise():
    g = Grid.make(1.0, 10 ** 6)  # large enough that nobody leaves
    r = inputs.rng(24)
    sig = np.concatenate([
        r.uniform(-40, 40, 200000), -(10.0 ** r.uniform(-12, 0, 20000)),
        np.arange(-30, 31, dtype=np.float64), np.array([-1e-30, -2.0 ** -24, 0.0, 1.0 - 2 ** -24]),
    ]).astype(np.float32)
    n = len(sig)
    cell0 = np.full(n, 500000, dtype=np.int32)
    sp = Species(s=0, prec=FP32, vx=np.zeros(n, np.float32), vy=np.zeros(n, np.float32),
                 vz=np.zeros(n, np.float32), id=np.arange(n, dtype=np.uint64),
                 knext=np.zeros(n, np.int64), cell=cell0, off=sig)
    # With zero field and dt/h = 0 the walk starts from sigma = off exactly.
    dtoh, rf, rb = g.walk_tables(0.0)
    _, cell, off, wall = push_fp32(g, sp, np.zeros(g.N, np.float32), 0, np.float32(0.0),
                                   (dtoh, rf, rb))
    shift, out = closed_form_uniform_walk(sig)
    assert np.array_equal(cell.astype(np.int64) - 500000, shift)
    assert np.array_equal(off.view(np.uint32), out.view(np.uint32))


def test_ec_gather_takes_field_of_cell_on_the_right_of_a_node():
    L, N = 1.0, 4
    cfg = inputs.small_discharge(n_cells=N, gap_m=L, collisions=0, weight_m2=1e-20)
    g = Grid.make(L, N)
    E = np.array([1.0, 2.0, 3.0, 4.0])
    sp = Species(s=1, prec=FP64, vx=np.zeros(1), vy=np.zeros(1), vz=np.zeros(1),
                 id=np.zeros(1, np.uint64), knext=np.zeros(1, np.int64), x=np.array([0.5]))
    from oracle.pic import gather_fp64
    assert gather_fp64(g, sp.x, E, 0)[0] == 3.0
    En = np.array([0.0, 1.0, 2.0, 3.0, 4.0])
    assert gather_fp64(g, np.array([0.625]), En, 1)[0] == pytest.approx(2.5)


def test_periodic_wrap_fp64_and_fp32():
    L, N = 0.01, 20
    g = Grid.make(L, N, bc=BC_PERIODIC)
    x = np.array([0.001, 0.009])
    vx = np.array([-3e7, 2e7])
    dt = 1e-10   # moves -3 mm and +2 mm
    from oracle.pic import push_fp64
    sp = Species(s=1, prec=FP64, vx=vx, vy=np.zeros(2), vz=np.zeros(2),
                 id=np.arange(2, dtype=np.uint64), knext=np.zeros(2, np.int64), x=x)
    _, xn, wall = push_fp64(g, sp, np.zeros(N), 0, 0.0, dt)
    assert np.all(wall == 0)
    assert np.allclose(xn, [0.008, 0.001], atol=1e-15)
    c, o = to_fp32_state(g, x)
    sp32 = Species(s=1, prec=FP32, vx=vx.astype(np.float32), vy=np.zeros(2, np.float32),
                   vz=np.zeros(2, np.float32), id=np.arange(2, dtype=np.uint64),
                   knext=np.zeros(2, np.int64), cell=c, off=o)
    _, cell, off, wall = push_fp32(g, sp32, np.zeros(N, np.float32), 0, np.float32(0.0),
                                   g.walk_tables(dt))
    assert np.all(wall == 0)
    assert np.allclose(g.position(cell, off), [0.008, 0.001], atol=1e-9)


def collapsed_walk(cell, sig, rf, rb, runs_lo, runs_hi, N):
    """Run-collapsed form of the FP32 walk (what the GPU kernel executes):
    inside a run of equal cells m steps become one FP32 operation."""
    one = np.float32(1.0)
    j = int(cell)
    s = np.float32(sig)
    while s < 0:
        lo = runs_lo[j]
        if lo < j:
            m = np.float32(-np.floor(s))
            avail = j - lo
            if m <= avail:
                j -= int(m)
                s = np.float32(s + m)
                continue
            s = np.float32(s + np.float32(avail))
            j = lo
        j -= 1
        if j < 0:
            return j, s, -1
        s = np.float32(one + np.float32(s * rb[j]))
    while s >= one:
        hi = runs_hi[j]
        if hi > j:
            m = np.float32(np.floor(s))
            avail = hi - j
            if m <= avail:
                j += int(m)
                s = np.float32(s - m)
                continue
            s = np.float32(s - np.float32(avail))
            j = hi
        s = np.float32(np.float32(s - one) * rf[j])
        j += 1
        if j >= N:
            return j, s, 1
    return j, s, 0


def test_run_collapsed_walk_equals_cell_walk_bitwise():
    """The refined grid of Section 3c consists of long runs of equal cells;
    collapsing the unit-ratio steps of a run must not change a single bit."""
    from oracle.grid import refined_nodes
    L = 0.03
    nodes = refined_nodes(L, L / 1024, L / 128, 0.004)
    N = len(nodes) - 1
    g = Grid.make(L, N, nodes)
    dtoh, rf, rb = g.walk_tables(1e-10)
    lo = np.zeros(N, int)
    hi = np.zeros(N, int)
    j = 0
    while j < N:
        e = j
        while e + 1 < N and rf[e] == 1.0 and rb[e] == 1.0:
            e += 1
        lo[j:e + 1] = j
        hi[j:e + 1] = e
        j = e + 1
    assert (hi - lo).max() > 50
    r = inputs.rng(25)
    n = 20000
    cell = r.integers(0, N, n).astype(np.int32)
    sig = np.concatenate([r.uniform(-300, 300, n - 2000), -(10.0 ** r.uniform(-10, 0, 1000)),
                          r.uniform(0.999, 1.0, 1000)]).astype(np.float32)
    sp = Species(s=0, prec=FP32, vx=np.zeros(n, np.float32), vy=np.zeros(n, np.float32),
                 vz=np.zeros(n, np.float32), id=np.arange(n, dtype=np.uint64),
                 knext=np.zeros(n, np.int64), cell=cell, off=sig)
    zero = np.zeros(N, np.float32)
    _, c1, o1, w1 = push_fp32(g, sp, zero, 0, np.float32(0.0), (zero, rf, rb))
    for i in range(n):
        jj, ss, ww = collapsed_walk(cell[i], sig[i], rf, rb, lo, hi, N)
        assert ww == w1[i]
        if ww == 0:
            assert jj == c1[i] and np.float32(ss).view(np.uint32) == o1[i].view(np.uint32), i


def test_in_run_single_step_equals_cell_walk_bitwise():
    """A move that stays inside the run of equal cells around the start cell is
    sigma - floor(sigma) in one FP32 operation (with a carry when a left move
    rounds up to 1); the GPU kernel takes this shortcut before walking."""
    from oracle.grid import refined_nodes
    L = 0.03
    nodes = refined_nodes(L, L / 1024, L / 128, 0.004)
    N = len(nodes) - 1
    g = Grid.make(L, N, nodes)
    _, rf, rb = g.walk_tables(1e-10)
    lo = np.zeros(N, int)
    hi = np.zeros(N, int)
    j = 0
    while j < N:
        e = j
        while e + 1 < N and rf[e] == 1.0 and rb[e] == 1.0:
            e += 1
        lo[j:e + 1] = j
        hi[j:e + 1] = e
        j = e + 1
    r = inputs.rng(26)
    n = 30000
    cell = r.integers(0, N, n).astype(np.int32)
    sig = np.concatenate([r.uniform(-40, 40, n - 3000), -(10.0 ** r.uniform(-12, 0, 2000)),
                          r.uniform(-1.0, 2.0, 1000)]).astype(np.float32)
    sp = Species(s=0, prec=FP32, vx=np.zeros(n, np.float32), vy=np.zeros(n, np.float32),
                 vz=np.zeros(n, np.float32), id=np.arange(n, dtype=np.uint64),
                 knext=np.zeros(n, np.int64), cell=cell, off=sig)
    zero = np.zeros(N, np.float32)
    _, c1, o1, w1 = push_fp32(g, sp, zero, 0, np.float32(0.0), (zero, rf, rb))
    used = 0
    for i in range(n):
        s = np.float32(sig[i])
        j0 = int(cell[i])
        if s < 0 or s >= 1:
            m = np.float32(np.floor(s))
            jm = j0 + int(m)
            if lo[j0] <= jm <= hi[j0]:
                s2 = np.float32(s - m)
                if s2 >= np.float32(1.0):
                    s2 = np.float32(0.0)
                    jm += 1
                used += 1
                assert w1[i] == 0 and c1[i] == jm and s2.view(np.uint32) == o1[i].view(np.uint32), i
    assert used > n // 2
