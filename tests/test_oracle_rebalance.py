"""Pins of the oracle's particle rebalancing (merge and split toward a constant
number of particles per cell on non-uniform grids, Section 3d): hand values
of one merge, exact charge, momentum and energy to rounding, the bound on
how far a merge moves node charge, exact deposits through splits,
independence of the storage order, and cell counts that settle within a
factor of two of the target on a refined grid."""
import math

import numpy as np
import pytest

import inputs
from oracle import physics as ph
from oracle.grid import refined_nodes
from oracle.pic import FP32, Species, WC_UNIT, deposit_species, Grid
from oracle.rebalance import default_dv, merge_quadruples, rebalance_species, velocity_bin
from oracle.sim import Sim


def test_one_merge_by_hand():
    """Four particles with velocities (1,0,0), (3,0,0), (0,2,0), (0,-2,0): mean
    (1,0,0), <|v|^2> = (1 + 9 + 4 + 4)/4 = 4.5, delta^2 = 4.5 - 1 = 3.5; e is
    the unit vector of v_d - v_a = (-1,-2,0)/sqrt(5)."""
    v = np.array([[[1.0], [0.0], [0.0]], [[3.0], [0.0], [0.0]], [[0.0], [2.0], [0.0]],
                  [[0.0], [-2.0], [0.0]]])
    off = np.array([[0.125], [0.25], [0.5], [0.625]])
    va, vb, ob = merge_quadruples(v, off)
    d = math.sqrt(3.5)
    e = np.array([-1.0, -2.0, 0.0]) / math.sqrt(5.0)
    assert np.allclose(va[:, 0], np.array([1.0, 0.0, 0.0]) + d * e, rtol=0, atol=1e-15)
    assert np.allclose(vb[:, 0], np.array([1.0, 0.0, 0.0]) - d * e, rtol=0, atol=1e-15)
    assert ob[0] == np.float32(0.375)
    # weight 4 -> 2 x 2: momentum and energy
    assert np.allclose(2 * (va + vb)[:, 0], v.sum(axis=0)[:, 0], atol=1e-14)
    e_before = sum(float((v[i] ** 2).sum()) for i in range(4))
    e_after = 2 * float((va ** 2).sum() + (vb ** 2).sum())
    assert e_after == pytest.approx(e_before, rel=1e-15)


def test_equal_velocities_merge_without_spread():
    v = np.tile(np.array([[2.0], [-1.0], [0.5]]), (4, 1, 1))
    va, vb, _ = merge_quadruples(v, np.full((4, 1), 0.5))
    assert np.array_equal(va, v[0]) and np.array_equal(vb, v[0])


def cell_state(n, N, seed, vt=6e5):
    r = inputs.rng(seed)
    cell = r.integers(0, N, n).astype(np.int32)
    off = r.uniform(0, 1, n).astype(np.float32)
    off = np.minimum(off, np.nextafter(np.float32(1), np.float32(0)))
    v = r.normal(0, vt, (3, n)).astype(np.float32)
    return Species(s=0, prec=FP32, vx=v[0], vy=v[1], vz=v[2], id=inputs.unique_ids(n, seed + 1),
                   knext=r.integers(0, 100, n).astype(np.int64), cell=cell, off=off,
                   wc=np.full(n, WC_UNIT, np.uint8))


def moments(sp, N):
    """Per cell: weight (in units W 2^-4), momentum and energy sums (FP64)."""
    w = np.ldexp(1.0, sp.classes().astype(np.int64))
    cell = sp.cell.astype(np.int64)
    v = np.array([sp.vx, sp.vy, sp.vz], dtype=np.float64)
    M = np.zeros(N)
    P = np.zeros((3, N))
    E = np.zeros(N)
    np.add.at(M, cell, w)
    for c in range(3):
        np.add.at(P[c], cell, w * v[c])
    np.add.at(E, cell, w * (v * v).sum(axis=0))
    return M, P, E


def test_merge_conserves_charge_momentum_energy_per_cell():
    N = 16
    sp = cell_state(20000, N, seed=3)
    dv = 1.5e5
    M0, P0, E0 = moments(sp, N)
    g = Grid.make(0.01, N)
    A0 = deposit_species(g, sp, u=4)
    out, nm, ns = rebalance_species(sp, N, 200, dv, k=10, seed=9, nudt=0.01)
    assert nm > 2000 and ns == 0
    M1, P1, E1 = moments(out, N)
    assert np.array_equal(M0, M1)                        # weight, exactly
    A1 = deposit_species(g, out, u=4)
    assert A0.sum() == A1.sum()                          # total charge, exactly
    vmax = float(np.max(np.abs([sp.vx, sp.vy, sp.vz])))
    # momentum and energy: the FP32 rounding of the stored velocities only
    assert np.max(np.abs(P1 - P0)) <= 2 ** -23 * vmax * M0.max()
    assert np.max(np.abs(E1 / E0 - 1)) <= 2 ** -22
    # node charge moves only by the FP32 rounding of the mean offsets:
    # at most 2^(c+1) x 2^-25 x 2^32 per merge touching the node
    merges_per_node = np.zeros(N + 1)
    before = np.bincount(sp.cell, minlength=N)
    after = np.bincount(out.cell, minlength=N)
    m_cell = (before - after) / 2
    merges_per_node[:-1] += m_cell
    merges_per_node[1:] += m_cell
    bound = merges_per_node * 2.0 ** (WC_UNIT + 1 + 7)
    assert np.all(np.abs(A1 - A0) <= bound)


def test_merged_particles_keep_the_first_two_ids_and_candidacies():
    N = 4
    sp = cell_state(4000, N, seed=5)
    sp.vx = np.abs(sp.vx)
    out, nm, _ = rebalance_species(sp, N, 100, 1e9, k=0, seed=1, nudt=0.0)   # one velocity bin
    # every group (cell, class) of n particles keeps n - 2 floor(n/4) of them
    assert out.n == sp.n - 2 * nm
    kept = set(out.id.tolist())
    for c in range(N):
        ids = np.sort(sp.id[sp.cell == c])
        q = len(ids) // 4
        for i in range(q):
            a, b, cc, d = ids[4 * i: 4 * i + 4]
            assert a in kept and b in kept and cc not in kept and d not in kept
    k0 = dict(zip(sp.id.tolist(), sp.knext.tolist()))
    assert all(k0[i] == k for i, k in zip(out.id.tolist(), out.knext.tolist()))


def test_split_keeps_the_deposit_exactly():
    N = 8
    sp = cell_state(40, N, seed=7)
    g = Grid.make(0.01, N)
    A0 = deposit_species(g, sp, u=4)
    out, nm, ns = rebalance_species(sp, N, 100, 1.5e5, k=33, seed=2, nudt=0.05)
    assert nm == 0 and ns == 40 and out.n == 80
    assert np.array_equal(deposit_species(g, out, u=4), A0)
    assert np.all(out.classes() == WC_UNIT - 1)
    # children: first candidacy at step 33 or later, new ids
    children = out.subset(~np.isin(out.id, sp.id))
    assert children.n == 40 and np.all(children.knext >= 33)
    assert len(np.unique(out.id)) == 80


def test_result_does_not_depend_on_storage_order():
    N = 8
    sp = cell_state(6000, N, seed=11)
    a, _, _ = rebalance_species(sp, N, 300, 2e5, k=4, seed=3, nudt=0.02)
    perm = inputs.rng(12).permutation(sp.n)
    b, _, _ = rebalance_species(sp.subset(perm), N, 300, 2e5, k=4, seed=3, nudt=0.02)
    oa, ob = np.argsort(a.id), np.argsort(b.id)
    for f in ("vx", "vy", "vz", "off", "cell", "knext", "wc"):
        assert np.array_equal(getattr(a, f)[oa], getattr(b, f)[ob]), f


def test_counts_settle_near_the_target_on_a_refined_grid():
    """Uniform density on a refined grid (cells of 1 to 8 units) starts with
    particle counts proportional to the cell widths (199 to 1945 per cell
    here); rebalancing brings every cell within a factor of two of the target
    and then leaves the state as it is."""
    L = 0.025
    nodes = refined_nodes(L, L / 512, L / 64, 0.004)
    N = len(nodes) - 1
    cfg = inputs.small_discharge(nodes=nodes, n_cells=N, precision=1, n_per_species=120_000,
                                 rebalance_ppc=400, collisions=0)
    sim = Sim(cfg)
    n0 = np.bincount(sim.sp[0].cell, minlength=N)
    assert n0.max() > 4 * n0.min()
    for _ in range(2):
        sim.rebalance()
    n1 = np.bincount(sim.sp[0].cell, minlength=N)
    assert n1.max() <= 2 * 400 and n1.min() >= 200
    assert n1.std() / n1.mean() < n0.std() / n0.mean() / 2
    assert sim.rebalance() == [(0, 0), (0, 0)]      # settled: nothing more to do
    # the total weight (charge) is exactly that of the initial load
    w = np.ldexp(1.0, sim.sp[0].classes().astype(np.int64) - 4).sum()
    assert w == 120_000


def test_default_bin_widths():
    cfg = dict(rebalance_dv_e=0.0, rebalance_dv_i=0.0, te_ev=2.0, ti_ev=0.026)
    assert default_dv(cfg, 0) == pytest.approx(0.25 * math.sqrt(2.0 * ph.QE / ph.ME))
    assert default_dv(dict(cfg, rebalance_dv_e=1e5), 0) == 1e5
    assert velocity_bin(np.array([-1e12, -0.5, 0.0, 0.5, 1e12]), 1.0).tolist() == [-128, -1, 0, 0, 127]


def test_a_particle_of_double_weight_counts_as_two():
    """Every weighted quantity of the oracle -- deposit, field, kinetic energy,
    absorbed energy, impact and EEDF histograms, velocity moments -- gives a
    particle of class 5 (weight 2W) exactly what two copies of class 4 give."""
    N, n = 64, 3000
    base = dict(n_cells=N, precision=1, n_per_species=n, rebalance_ppc=100, collisions=0, gamma_see=0.0,
                avg_every=1, eedf_every=1, eedf_width_m=0.01, moments=1, impact_bins=40,
                impact_angle_bins=18, impact_emax_ev=100.0, v_rf=150.0)
    cfg = inputs.small_discharge(**base)
    sps = [cell_state(n, N, seed=21 + s) for s in range(2)]
    for s, sp in enumerate(sps):
        sp.s = s
        if s == 1:
            sp.vx = sp.vx / np.float32(200.0)
            sp.vy = sp.vy / np.float32(200.0)
            sp.vz = sp.vz / np.float32(200.0)
    heavy = [sp.subset(np.arange(sp.n)) for sp in sps]
    for sp in heavy:
        sp.wc = np.full(sp.n, 5, np.uint8)
    twins = [sp.append(Species(s=sp.s, prec=FP32, vx=sp.vx, vy=sp.vy, vz=sp.vz,
                               id=sp.id + np.uint64(1 << 62), knext=sp.knext, cell=sp.cell, off=sp.off,
                               wc=sp.wc)) for sp in sps]
    a = Sim(cfg, species=heavy, k=5)
    b = Sim(cfg, species=twins, k=5)
    for _ in range(3):
        a.step()
        b.step()
    assert np.array_equal(a.A[0], b.A[0]) and np.array_equal(a.A[1], b.A[1])
    assert np.array_equal(a.phi, b.phi)
    for s in range(2):
        assert a.kinetic_energy(s) == pytest.approx(b.kinetic_energy(s), rel=1e-13)
        assert np.allclose(a.absorbed_energy_ev[s], b.absorbed_energy_ev[s], rtol=1e-13)
        assert np.array_equal(a.impact_e[s], b.impact_e[s]) and np.array_equal(a.impact_a[s], b.impact_a[s])
        ma, mb = a.moments(s), b.moments(s)
        for key in ma:
            assert np.allclose(ma[key], mb[key], rtol=1e-12, atol=0), key
    assert np.array_equal(a.eedf, b.eedf) and a.eedf.sum() > 0
    assert a.absorbed.sum() > 0 and 2 * a.absorbed.sum() == b.absorbed.sum()
