"""GPU against the oracle on what the benchmark runs and on crafted edge cases:
the library's own null-collision bounds, the stability monitors and energy
tallies of pic_diagnostics, single steps from states placed exactly on the
branch points of the push (nodes, offsets one ulp below 1, sub-ulp moves,
the last position below L, walks across several runs of a refined grid), and
impact histograms after one step with many wall crossings.

Every case states its seed and shape before it touches the GPU.
"""
import math
import sys

import numpy as np
import pytest

import inputs
from gpu_common import compare_species, gpu_from_states, oracle_from_states, species_dict
from oracle import physics as ph
from oracle.grid import refined_nodes
from oracle.pic import Grid
from oracle.sim import Sim

pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps
K0 = 37


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def Context():
    from paper_2308_13092_amd import Context as C
    return C


# -- the library's own null-collision bounds ---------------------------------
@pytest.mark.parametrize("p_mtorr,v_rf,t_gas", [(50.0, 200.0, 300.0), (20.0, 400.0, 300.0),
                                                (10.0, 100.0, 350.0), (100.0, 500.0, 280.0)])
def test_library_nu_max_equals_the_oracle(gpu, p_mtorr, v_rf, t_gas):
    """With nu_max_e = nu_max_i = 0 (the benchmark's configurations) the
    library computes the bounds on its host: the same doubles as the oracle's
    to a few ulps (both scan 200001 log-spaced energies)."""
    note("nu_max", p_mtorr, v_rf, t_gas)
    cfg = inputs.small_discharge(n_per_species=1000, p_pa=p_mtorr * inputs.MTORR, v_rf=v_rf,
                                 t_gas_k=t_gas, nu_max_e=0.0, nu_max_i=0.0)
    ctx = Context()([cfg])
    nu = ctx.diagnostics()["nu_max"]
    n_g = ph.gas_density(cfg["p_pa"], t_gas)
    assert abs(nu[0] / ph.nu_max_electron(n_g) - 1) <= 4 * EPS
    assert abs(nu[1] / ph.nu_max_ion(n_g, v_rf, t_gas) - 1) <= 4 * EPS
    ctx.close()


# -- stability monitors and energy tallies -----------------------------------
def discharge_cfg(prec, kind, n, **over):
    L, N = 0.025, 128
    nodes, bc = None, 0
    if kind == "refined":
        nodes = refined_nodes(L, L / 512, L / 64, 0.004)
        N = len(nodes) - 1
    elif kind == "periodic":
        bc = 1
    n_g = ph.gas_density(50 * inputs.MTORR, 300.0)
    cfg = inputs.small_discharge(precision=prec, nodes=nodes, bc=bc, n_per_species=n, n_cells=N,
                                 nu_max_e=ph.nu_max_electron(n_g),
                                 nu_max_i=ph.nu_max_ion(n_g, 200.0, 300.0), gamma_see=0.3,
                                 sort_interval=0)
    cfg.update(over)
    return cfg


def near_wall_states(cfg, seed, n, ve=3.0e6, vi=3.0e4, bands=(0.2, 0.001)):
    """Particles within a band (a fraction of the gap; electrons, ions) of
    either electrode, hot enough that many of them cross a wall in one step."""
    prec = cfg["precision"]
    L = cfg["gap_m"] if cfg["nodes"] is None else float(cfg["nodes"][-1])
    g = Grid.make(L, cfg["n_cells"], cfg["nodes"], cfg["bc"])
    out = []
    for s, vs in ((0, ve), (1, vi)):
        r = inputs.rng(seed + 10 * s)
        st = inputs.particles_fp64(n, L, vs, seed + 10 * s, k=K0)
        u = r.uniform(0.0, bands[s] * L, size=n)
        x = np.where(r.random(n) < 0.5, u, L - u)
        x = np.minimum(np.maximum(x, 0.0), np.nextafter(L, 0.0))
        st["x"] = x
        if prec == 1:
            from oracle.pic import to_fp32_state
            cell, off = to_fp32_state(g, x)
            st = dict(cell=cell, off=off, vx=st["vx"].astype(np.float32),
                      vy=st["vy"].astype(np.float32), vz=st["vz"].astype(np.float32), id=st["id"],
                      knext=st["knext"])
        out.append(st)
    return out


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", ["uniform", "refined"])
def test_monitors_and_energy_tallies_against_oracle(gpu, prec, kind):
    """One step from identical state: the stability monitors of Section 1
    (Eqs 1a-1c) and the kinetic and absorbed energies of pic_diagnostics
    against the oracle's.  The library sums energies in fixed point, so the
    bars are its rounding: 2^-21 eV per particle for the kinetic energy,
    2^-17 eV per absorbed particle for the wall energies."""
    n = 50_003
    note("monitors", prec, kind, n)
    cfg = discharge_cfg(prec, kind, n)
    states = near_wall_states(cfg, seed=91, n=n)
    ref = oracle_from_states(cfg, states, K0)
    ctx = gpu_from_states(cfg, states, K0, Context())
    ctx.step(1)
    ref.step()
    d = ctx.diagnostics()
    for s in range(2):   # identical particle sets (no branch flips)
        st = compare_species(ctx.get_state(0, s), species_dict(ref.sp[s]), ref.grid, 1e-5, 1e-5, 1e7,
                             max_flips=0)
        note("species", s, st)
    m = ref.monitors()
    assert d["ne_max_m3"] == pytest.approx(m["ne_max_m3"], rel=4 * EPS)
    assert d["wpe_dt_max"] == pytest.approx(m["wpe_dt_max"], rel=8 * EPS)
    rel_v = 4 * EPS if prec == 1 else 1e-12
    assert d["vmax_dt_over_dxmin"] == pytest.approx(m["vmax_dt_over_dxmin"], rel=rel_v)
    # T_e from the fixed-point kinetic sum: |dT| <= 2/3 2^-21 eV; lambda ~ sqrt(T)
    rel_l = 0.5 * (2.0 / 3.0) * 2.0 ** -21 / m["te_ev"] + 1e-12
    assert d["lambda_de_over_dxmin"] == pytest.approx(m["lambda_de_over_dxmin"], rel=rel_l)
    for s in range(2):
        n_s = ref.sp[s].n
        ke = ref.kinetic_energy(s)
        bar = n_s * 2.0 ** -21 * ref.W * ph.QE * (1 + 1e-9) + 1e-12 * ke
        assert abs(d["kinetic_j_m2"][s] - ke) <= bar, (s, d["kinetic_j_m2"][s], ke, bar)
        for w in range(2):
            na = int(ref.absorbed[s, w])
            assert int(d["absorbed"][s][w]) == na
            ea = float(ref.absorbed_energy_ev[s, w])
            assert abs(d["absorbed_energy_ev"][s][w] - ea) <= na * 2.0 ** -17 + 1e-12 * ea, (s, w)
            note("absorbed", s, w, na, d["absorbed_energy_ev"][s][w], ea)
    assert ref.absorbed.sum() > 1000


# -- impact histograms, exactly ----------------------------------------------
def edge_counts(ref, nb, na, emax):
    """Absorbed particles of the last oracle step whose energy or angle bin
    lies within 1e-9 of a bin edge (there the device's and the host's last
    ulp of acos, or of the FP64 state, may pick the other bin), per
    (species, wall)."""
    out = np.zeros((2, 2), dtype=np.int64)
    for s, w, en, vx, v2 in ref.last_absorbed:
        fe = en * (nb / emax)
        c = np.ones_like(v2)
        pos = v2 > 0.0
        c[pos] = np.minimum(1.0, np.abs(vx[pos]) / np.sqrt(v2[pos]))
        fa = np.degrees(np.arccos(c)) * (na / 90.0)
        near = (np.abs(fe - np.round(fe)) < 1e-9 * np.maximum(1.0, fe)) | \
               (np.abs(fa - np.round(fa)) < 1e-9 * np.maximum(1.0, fa))
        out[s, w] += int(near.sum())
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_impact_histograms_after_one_step_are_exact(gpu, prec):
    """Energy and angle histograms of the particles absorbed in one step from
    identical state, with thousands of wall crossings: bin for bin equal to
    the oracle's, except particles within 1e-9 of a bin edge (counted, and
    there are normally none)."""
    n, nb, na, emax = 50_003, 100, 45, 200.0
    note("impacts one step", prec, n)
    cfg = discharge_cfg(prec, "uniform", n, avg_every=1, impact_bins=nb, impact_angle_bins=na,
                        impact_emax_ev=emax)
    states = near_wall_states(cfg, seed=17, n=n)
    ref = oracle_from_states(cfg, states, K0)
    ctx = gpu_from_states(cfg, states, K0, Context())
    ctx.step(1)
    ref.step()
    d = ctx.diagnostics()
    edges = edge_counts(ref, nb, na, emax)
    total = 0
    for s in range(2):
        for w in range(2):
            h = ctx.impacts(0, s, w)
            assert int(d["absorbed"][s][w]) == int(ref.absorbed[s, w])
            de = int(np.abs(h["energy"] - ref.impact_e[s, w]).sum())
            da = int(np.abs(h["angle"] - ref.impact_a[s, w]).sum())
            note("impact", s, w, int(ref.absorbed[s, w]), "diff", de, da, "edges", int(edges[s, w]))
            assert de <= 2 * edges[s, w] and da <= 2 * edges[s, w]
            total += int(ref.absorbed[s, w])
    assert total > 2000


# -- crafted branch points of the push ----------------------------------------
def grid_of(cfg):
    L = cfg["gap_m"] if cfg["nodes"] is None else float(cfg["nodes"][-1])
    return Grid.make(L, cfg["n_cells"], cfg["nodes"], cfg["bc"])


def edge_state_fp32(g, dt, seed):
    """FP32 form: offsets 0, one ulp above 0, 1/2, one and two ulps below 1, in
    the end cells, interior cells and the cells where the width changes;
    moves of 0, +-2^-26, +-2^-25, +-3 2^-26, +-2^-24 and +-2^-23 cell widths
    (sub-ulp, tie and one-ulp moves), and long walks of 1 to 60 cells either
    way."""
    N = g.N
    r = inputs.rng(seed)
    change = np.nonzero(np.abs(np.diff(g.h)) > 0)[0]
    cells = sorted(set([0, 1, 2, N // 2, N - 3, N - 2, N - 1] + list(change) + list(change + 1)))
    offs = [0.0, 2.0 ** -24, 0.5, 1.0 - 2.0 ** -24, 1.0 - 2.0 ** -23]
    moves = [0.0] + [sgn * t for t in (2.0 ** -26, 2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -24, 2.0 ** -23)
                     for sgn in (1, -1)]
    c, o, v = [], [], []
    for j in cells:
        for off in offs:
            for mv in moves:
                c.append(j)
                o.append(off)
                v.append(mv * g.h[j] / dt)
        for _ in range(24):
            c.append(j)
            o.append(float(np.float32(r.random())))
            v.append(float(r.choice([-1, 1]) * r.uniform(1.0, 60.0) * g.h[j] / dt))
    cell = np.array(c, dtype=np.int32)
    off = np.array(o, dtype=np.float32)
    off = np.minimum(off, np.nextafter(np.float32(1.0), np.float32(0.0)))
    return cell, off, np.array(v, dtype=np.float32)


def edge_state_fp64(g, dt, seed):
    """FP64 form: exactly on nodes, one ulp either side of a node, 0, the last
    double below L, cell middles; moves of 0, +-1/4, +-1/2, +-3/4 and +-1 ulp
    of the position and long moves of 1 to 60 cell widths."""
    r = inputs.rng(seed)
    N, L = g.N, g.L
    change = np.nonzero(np.abs(np.diff(g.h)) > 0)[0]
    cells = sorted(set([0, 1, 2, N // 2, N - 3, N - 2, N - 1] + list(change) + list(change + 1)))
    xs = [0.0, np.nextafter(L, 0.0)]
    for j in cells:
        xn = g.nodes[j]
        xs += [xn, np.nextafter(xn, L), xn + 0.5 * g.h[j]]
        if j > 0:
            xs.append(np.nextafter(xn, 0.0))
    x, v = [], []
    for x0 in xs:
        ulp = np.spacing(max(x0, 1e-300))
        for mv in (0.0, 0.25, -0.25, 0.5, -0.5, 0.75, -0.75, 1.0, -1.0):
            x.append(x0)
            v.append(mv * ulp / dt)
        j = min(int(np.searchsorted(g.nodes, x0, side="right")) - 1, N - 1)
        for _ in range(8):
            x.append(x0)
            v.append(float(r.choice([-1, 1]) * r.uniform(1.0, 60.0) * g.h[j] / dt))
    return np.array(x, dtype=np.float64), np.array(v, dtype=np.float64)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", ["uniform", "refined", "periodic"])
def test_single_step_at_the_branch_points_of_the_push(gpu, prec, kind):
    """Electrons and ions at the same crafted positions (so the charge, and with
    no drive the field, is exactly zero on both sides and every move is the
    one given): after one step the FP32 form equals the oracle bitwise (cell,
    offset, velocity) and the FP64 form to the last bit of x + v dt, with the
    same particles absorbed at each wall."""
    note("branch points", prec, kind)
    cfg = discharge_cfg(prec, kind, 1000, v_rf=0.0, collisions=0, gamma_see=0.0)
    g = grid_of(cfg)
    dt = cfg["dt_s"]
    states = []
    ids = inputs.unique_ids(200_000, seed=5)
    if prec == 1:
        cell, off, ve = edge_state_fp32(g, dt, seed=3)
        n = len(cell)
        for s in range(2):
            vs = ve if s == 0 else (ve[::-1].copy() / np.float32(50.0))
            z = np.zeros(n, np.float32)
            states.append(dict(cell=cell, off=off, vx=vs, vy=z, vz=z, id=ids[s * n:(s + 1) * n],
                               knext=np.full(n, 2 ** 31 - 1, np.int64)))
    else:
        x, ve = edge_state_fp64(g, dt, seed=3)
        n = len(x)
        for s in range(2):
            vs = ve if s == 0 else ve[::-1] / 50.0
            z = np.zeros(n)
            states.append(dict(x=x, vx=vs, vy=z, vz=z, id=ids[s * n:(s + 1) * n],
                               knext=np.full(n, 2 ** 31 - 1, np.int64)))
    cfg["n_per_species"] = n
    note("particles per species", n)
    ref = oracle_from_states(cfg, states, K0)
    ctx = gpu_from_states(cfg, states, K0, Context())
    ctx.step(1)
    ref.step()
    assert np.all(ref.E == 0.0)
    f = ctx.fields()
    assert np.all(f["E"] == 0.0)
    d = ctx.diagnostics()
    for s in range(2):
        gs = ctx.get_state(0, s)
        rs = species_dict(ref.sp[s])
        og, orr = np.argsort(gs["id"]), np.argsort(rs["id"])
        assert np.array_equal(gs["id"][og], rs["id"][orr]), s
        keys = ("cell", "off", "vx") if prec == 1 else ("x", "vx")
        for key in keys:
            a = np.asarray(gs[key])[og]
            b = np.asarray(rs[key])[orr].astype(a.dtype)
            bad = np.nonzero(a != b)[0]
            assert len(bad) == 0, (s, key, a[bad[:5]], b[bad[:5]])
        for w in range(2):
            assert int(d["absorbed"][s][w]) == int(ref.absorbed[s, w]), (s, w)
        note("species", s, "kept", len(gs["id"]), "absorbed", ref.absorbed[s].tolist())
    if kind != "periodic":
        assert ref.absorbed.sum() > 0
