"""Particle rebalancing (pic_rebalance) and weighted particles against the
oracle through the C ABI.

* One rebalancing pass from identical state: every particle (cell, offset,
  velocity, weight class, id, candidacy) bitwise equal to the oracle's, merges
  and splits counted alike, the deposit's total charge unchanged exactly.
* A step of a state of mixed weight classes: deposit bitwise, particles
  bitwise, kinetic and absorbed energies within the fixed-point rounding.
* A run that rebalances every 10 steps stays equal to the oracle.
Every case states its seed and shape before it touches the GPU.
"""
import sys

import numpy as np
import pytest

import inputs
from gpu_common import compare_species, gpu_from_states, oracle_from_states, species_dict
from oracle import physics as ph
from oracle.grid import refined_nodes
from oracle.sim import Sim

pytestmark = pytest.mark.gpu

K0 = 41


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def rb_cfg(n=60_000, ppc=300, **over):
    L = 0.025
    nodes = refined_nodes(L, L / 512, L / 64, 0.004)
    n_g = ph.gas_density(50 * inputs.MTORR, 300.0)
    cfg = inputs.small_discharge(precision=1, nodes=nodes, n_cells=len(nodes) - 1, n_per_species=n,
                                 nu_max_e=ph.nu_max_electron(n_g), nu_max_i=ph.nu_max_ion(n_g, 200.0, 300.0),
                                 gamma_see=0.3, sort_interval=0, rebalance_ppc=ppc, capacity=3 * n)
    cfg.update(over)
    return cfg


def states_of(ctx):
    return [ctx.get_state(0, s) for s in range(2)]


def same_by_id(g, r, keys=("cell", "off", "vx", "vy", "vz", "wc", "knext")):
    og, orr = np.argsort(g["id"]), np.argsort(r["id"])
    assert np.array_equal(g["id"][og], r["id"][orr]), (len(g["id"]), len(r["id"]))
    for key in keys:
        a = np.asarray(g[key])[og]
        b = np.asarray(r[key])[orr].astype(a.dtype)
        bad = np.nonzero(a != b)[0]
        assert len(bad) == 0, (key, len(bad), a[bad[:4]], b[bad[:4]])


def rdict(sp):
    d = species_dict(sp)
    d["wc"] = sp.classes()
    return d


@pytest.mark.parametrize("seed", [3, 8])
def test_rebalance_pass_equals_the_oracle(gpu, seed):
    from paper_2308_13092_amd import Context
    cfg = rb_cfg(seed=seed)
    note("rebalance pass", seed, cfg["n_per_species"], cfg["n_cells"])
    ctx = Context([cfg])
    ctx.step(3)
    st = states_of(ctx)
    d0 = ctx.diagnostics()
    ref = oracle_from_states(cfg, st, int(d0["step"]))
    for s in range(2):
        ref.sp[s].wc = st[s]["wc"].copy()
    ctx.rebalance()
    counts = ref.rebalance()
    d1 = ctx.diagnostics()
    note("merges/splits", counts, list(d1["merges"]), list(d1["splits"]))
    for s in range(2):
        assert (int(d1["merges"][s]), int(d1["splits"][s])) == counts[s]
        same_by_id(ctx.get_state(0, s), rdict(ref.sp[s]))
    assert counts[0][0] > 1000 and counts[0][1] > 100
    # charge: the deposit of the rebalanced state has the same total
    ctx.deposit()
    d2 = ctx.diagnostics()
    assert list(d2["deposit_total"]) == list(d0["deposit_total"])
    A = ref.deposit()
    f = ctx.fields()
    assert np.array_equal(f["A_e"], A[0]) and np.array_equal(f["A_i"], A[1])


def test_step_of_mixed_weight_classes(gpu):
    from paper_2308_13092_amd import Context
    cfg = rb_cfg(n=50_003, avg_every=1, impact_bins=60, impact_angle_bins=30, impact_emax_ev=150.0,
                 eedf_every=1, eedf_width_m=0.004, moments=1)
    note("mixed classes", cfg["n_per_species"])
    N = cfg["n_cells"]
    states = []
    for s, vs in ((0, 1.5e6), (1, 2.0e4)):
        st = inputs.particles_fp32(cfg["n_per_species"], N, vs, seed=61 + s, k=K0)
        st["wc"] = inputs.rng(70 + s).integers(2, 7, cfg["n_per_species"]).astype(np.uint8)
        states.append(st)
    ref = oracle_from_states(cfg, states, K0)
    for s in range(2):
        ref.sp[s].wc = states[s]["wc"].copy()
    ctx = gpu_from_states(cfg, states, K0, Context)
    ctx.step(1)
    ref.step()
    m = ref.monitors()                # of the last solve (the deposit before the step)
    f = ctx.fields()
    A = ref.deposit()                 # the deposit of the state after the step
    assert np.array_equal(f["A_e"], A[0]) and np.array_equal(f["A_i"], A[1])
    d = ctx.diagnostics()
    for s in range(2):
        stats = compare_species(ctx.get_state(0, s), species_dict(ref.sp[s]), ref.grid, 1e-5, 1e-5, 1e7,
                                max_flips=0)
        note("species", s, stats)
        g = ctx.get_state(0, s)
        og, orr = np.argsort(g["id"]), np.argsort(ref.sp[s].id)
        assert np.array_equal(g["wc"][og], ref.sp[s].classes()[orr])
        ke = ref.kinetic_energy(s)
        n_w = float(np.ldexp(1.0, ref.sp[s].classes().astype(np.int64)).sum())
        assert abs(d["kinetic_j_m2"][s] - ke) <= n_w * 2.0 ** -21 * ref.W_unit * ph.QE + 1e-12 * ke
        for w in range(2):
            assert int(d["absorbed"][s][w]) == int(ref.absorbed[s, w])
            h = ctx.impacts(0, s, w)
            assert np.array_equal(h["energy"], ref.impact_e[s, w]) and np.array_equal(h["angle"], ref.impact_a[s, w])
        # velocity moments and power: FP64 sums in another order
        mg, mr = ctx.moments(0, s), ref.moments(s)
        for key in mr:
            scale = max(float(np.max(np.abs(mr[key]))), 1e-300)
            assert np.max(np.abs(mg[key] - mr[key])) <= 1e-9 * scale, key
    assert np.array_equal(ctx.profiles()["eedf"], ref.eedf) and ref.eedf.sum() > 0
    assert d["ne_max_m3"] == pytest.approx(m["ne_max_m3"], rel=1e-15)
    assert d["lambda_de_over_dxmin"] == pytest.approx(m["lambda_de_over_dxmin"], rel=1e-6)


def test_run_with_rebalancing_every_10_steps(gpu):
    """pic_step rebalances after every 10th step: the state before each pass,
    the counts of the pass and the state after it follow the oracle."""
    from paper_2308_13092_amd import Context
    cfg = rb_cfg(n=30_000, ppc=200, rebalance_every=10, sort_interval=7)
    note("rebalanced run", cfg["n_per_species"])
    ctx = Context([cfg])
    ref = Sim(cfg)
    merges = np.zeros(2, np.int64)
    splits = np.zeros(2, np.int64)

    def compare(stage):
        for s in range(2):
            stats = compare_species(ctx.get_state(0, s), species_dict(ref.sp[s]), ref.grid, 1e-5, 1e-5, 1e7,
                                    max_flips=3)
            note(stage, "species", s, stats)

    for block in range(3):
        ctx.step(9)
        ref.run(9)
        compare("block %d before" % block)
        ctx.step(1)
        ref.run(1)
        counts = ref.rebalance()
        d = ctx.diagnostics()
        for s in range(2):
            merges[s] += counts[s][0]
            splits[s] += counts[s][1]
        note("block", block, counts, list(d["merges"]), list(d["splits"]))
        assert list(d["merges"]) == list(merges) and list(d["splits"]) == list(splits)
        compare("block %d after" % block)
    d = ctx.diagnostics()
    assert d["step"] == 30 and d["merges"][0] > 0
    for s in range(2):
        # charge: the deposit holds every particle's weight exactly (units W/16 x 2^-32)
        g = ctx.get_state(0, s)
        assert d["deposit_total"][s] == int((np.int64(1) << g["wc"].astype(np.int64)).sum()) * 2 ** 32


def test_rebalancing_of_a_served_slot(gpu):
    """A discharge admitted into an empty slot (as the server does) with a
    rebalancing cadence: pic_step rebalances it at that cadence, and it ends
    as the same discharge in a context of its own."""
    from paper_2308_13092_amd import Context
    from paper_2308_13092_amd._lib import PIC_OK, slot_bytes
    from paper_2308_13092_amd.configs import base
    cfg = rb_cfg(n=20_000, ppc=150, rebalance_every=6, sort_interval=5)
    note("served slot rebalancing", cfg["n_per_species"])
    served = Context([base(n_cells=0, precision=1)] * 3, pool_bytes=slot_bytes(cfg))
    assert served.slot_reset(1, cfg) == PIC_OK
    alone = Context([cfg])
    served.step(13)
    alone.step(13)
    ds, da = served.diagnostics(1), alone.diagnostics(0)
    assert int(ds["merges"][0]) > 0 and list(ds["merges"]) == list(da["merges"])
    assert list(ds["splits"]) == list(da["splits"])
    for s in range(2):
        same_by_id(served.get_state(1, s), alone.get_state(0, s), keys=("cell", "off", "vx", "vy", "vz", "wc", "knext"))
