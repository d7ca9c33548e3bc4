"""Batched discharges, graph replay, the autotuner and the served mix, each
against the same discharges run alone (GPU).

Every discharge's result depends only on its own configuration: the deposit
is an exact integer sum, the field solve is per instance, and each particle
draws from its own Philox stream.  So these comparisons are bitwise (particle
sets compared by id, storage order being unspecified).
"""
import sys

import numpy as np
import pytest

import inputs
from oracle import physics as ph

pytestmark = pytest.mark.gpu


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def Context():
    from paper_2308_13092_amd import Context as C
    return C


def mixed_configs(prec, n_scale=1.0):
    """Six discharges of different sizes, grids, gathers and drives, and one
    empty slot."""
    from oracle.grid import refined_nodes
    L = 0.025
    out = []
    specs = [
        dict(n_cells=64, gather=0, v_rf=150.0, p=30.0, div=400, n=4_000),
        dict(n_cells=200, gather=1, v_rf=300.0, p=80.0, div=700, n=12_001),
        dict(nodes=inputs.random_nodes(L, 96, seed=3), gather=0, v_rf=250.0, p=50.0, div=500, n=7_777),
        dict(nodes=refined_nodes(L, L / 512, L / 64, 0.004), gather=0, v_rf=400.0, p=20.0, div=1000,
             n=20_000),
        None,
        dict(n_cells=1024, gather=1, v_rf=100.0, p=100.0, div=900, n=9_000),
        dict(n_cells=128, gather=0, v_rf=500.0, p=10.0, div=400, n=2_500),
    ]
    for i, s in enumerate(specs):
        if s is None:
            out.append(inputs.small_discharge(n_cells=0, precision=prec))
            continue
        n_g = ph.gas_density(s["p"] * inputs.MTORR, 300.0)
        cfg = inputs.small_discharge(
            precision=prec, gather=s["gather"], n_per_species=int(s["n"] * n_scale),
            v_rf=s["v_rf"], p_pa=s["p"] * inputs.MTORR, dt_s=1.0 / (13.56e6 * s["div"]),
            nu_max_e=ph.nu_max_electron(n_g), nu_max_i=ph.nu_max_ion(n_g, 2 * s["v_rf"], 300.0),
            gamma_see=0.2, seed=100 + i, sort_interval=10, avg_every=1, eedf_every=7,
            nodes=s.get("nodes"), n_cells=s.get("n_cells", 0) if s.get("nodes") is None else 0)
        if s.get("nodes") is not None:
            cfg["n_cells"] = len(s["nodes"]) - 1
        out.append(cfg)
    return out


def sorted_state(ctx, inst, s):
    st = ctx.get_state(inst, s)
    o = np.argsort(st["id"], kind="stable")
    return {k: v[o] for k, v in st.items()}


def assert_same_instance(a, ia, b, ib, nsp=2):
    for s in range(nsp):
        sa, sb = sorted_state(a, ia, s), sorted_state(b, ib, s)
        assert len(sa["id"]) == len(sb["id"]), (ia, s)
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), (ia, s, k)
    da, db = a.diagnostics(ia), b.diagnostics(ib)
    for k in ("step", "n_live", "absorbed", "see_emitted", "ionisations", "excitations", "elastic",
              "charge_exchange", "candidates", "particle_steps", "deposit_total", "eedf_samples"):
        assert np.array_equal(np.asarray(da[k]), np.asarray(db[k])), (ia, k)
    pa, pb = a.profiles(ia), b.profiles(ib)
    for k in ("ne", "ni", "phi", "eedf"):
        assert np.array_equal(pa[k], pb[k]), (ia, k)
    fa, fb = a.fields(ia), b.fields(ib)
    for k in ("A_e", "A_i", "phi", "E"):
        assert np.array_equal(fa[k], fb[k]), (ia, k)


def test_large_batch_equals_alone(gpu):
    """Six discharges scaled to 35 M particles in all: the batch sorts and
    drains with the large-batch grids (a sort scatter of 128 workgroups per
    CU beside a count of 16, a drain of eight times the resident
    workgroups), each discharge alone with the ordinary ones.  A sort falls
    inside the 12 steps; every discharge ends bitwise as it does alone."""
    cfgs = mixed_configs(1, n_scale=320.0)
    total = sum(2 * c["n_per_species"] for c in cfgs if c["n_cells"] > 0)
    note("large batch vs alone", total, [c["n_per_species"] for c in cfgs])
    assert total >= 32 << 20
    steps = 12
    batch = Context()(cfgs)
    batch.step(steps)
    for i, cfg in enumerate(cfgs):
        if cfg["n_cells"] == 0:
            continue
        alone = Context()([cfg])
        alone.step(steps)
        assert_same_instance(batch, i, alone, 0)
        alone.close()
    batch.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_alone(gpu, prec):
    cfgs = mixed_configs(prec)
    note("batch vs alone", prec, [c["n_cells"] for c in cfgs])
    steps = 45
    batch = Context()(cfgs)
    batch.step(steps)
    for i, cfg in enumerate(cfgs):
        if cfg["n_cells"] == 0:
            continue
        note("alone", i)
        alone = Context()([cfg])
        alone.step(steps)
        assert_same_instance(batch, i, alone, 0)
        alone.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replay_equals_eager_launches(gpu, prec):
    cfgs = [c for c in mixed_configs(prec) if c["n_cells"] > 0][:4]
    note("graph vs eager", prec)
    a, b = Context()(cfgs), Context()(cfgs)
    a.set_tuning(use_graph=1)
    b.set_tuning(use_graph=0)
    for n in (1, 9, 30):       # crosses sorts at steps 10, 20, 30, 40
        a.step(n)
        b.step(n)
    for i in range(len(cfgs)):
        assert_same_instance(a, i, b, i)


@pytest.mark.parametrize("use_graph", [1, 0])
def test_kernel_timing_changes_nothing(gpu, use_graph):
    """Timed steps (eager launches with HIP events around the kernels, also
    when graphs are on) give the untimed graph results bitwise.  Over 60 steps
    the streaming pass is timed 15 times (every 4th step), the sort 3 times,
    the field and the drain on steps 0, 16, 32 and 48."""
    cfgs = [c for c in mixed_configs(1) if c["n_cells"] > 0][:3]
    note("timing", use_graph)
    a, b = Context()(cfgs), Context()(cfgs)
    a.set_tuning(use_graph=use_graph, sort_interval=20)
    b.set_tuning(use_graph=1, sort_interval=20)
    a.kernel_times(True)
    a.step(60)
    kt = a.kernel_times(False)
    b.step(60)
    assert kt["particle_launches"] == 15 and kt["field_launches"] == 4
    assert kt["drain_launches"] == 4 and kt["sort_launches"] == 3
    assert kt["particle_ms"] > 0 and kt["field_ms"] > 0 and kt["drain_ms"] > 0 and kt["sort_ms"] > 0
    for i in range(len(cfgs)):
        assert_same_instance(a, i, b, i)


@pytest.mark.parametrize("prec", [0, 1])
def test_chained_steps_equal_single_steps(gpu, prec):
    """Within one multi-step call a step's close runs in the next step's field
    launch; one-step calls close every step with its own kernel.  Both give
    the same state bitwise, across sorts (every 7 steps here)."""
    cfgs = [c for c in mixed_configs(prec) if c["n_cells"] > 0][:4]
    note("chained vs single", prec)
    a, b = Context()(cfgs), Context()(cfgs)
    for ctx in (a, b):
        ctx.set_tuning(use_graph=0, sort_interval=7)
    a.step(23)
    for _ in range(23):
        b.step(1)
    for i in range(len(cfgs)):
        assert_same_instance(a, i, b, i)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("block,bpc", [(256, 1), (1024, 0), (512, 5)])
def test_launch_shape_does_not_change_results(gpu, block, bpc, prec):
    """Small tiles split every species over several workgroups."""
    cfgs = [c for c in mixed_configs(prec) if c["n_cells"] > 0][:3]
    note("launch shape", block, bpc, prec)
    a, b = Context()(cfgs), Context()(cfgs)
    b.set_tuning(block=block, blocks_per_cu=bpc, sort_interval=7)
    a.step(33)
    b.step(33)
    for i in range(len(cfgs)):
        assert_same_instance(a, i, b, i)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("block", [256, 1024])
def test_inline_drain_equals_the_drain_kernel(gpu, prec, block):
    """Small contexts drain collisions and absorptions inside the fused
    particle kernel (pic_tuning.inline_drain = 0 chooses it by size, 1 forces
    it); with 2 they launch k_drain.  The same discharges end bitwise equal
    either way: states by id, counters, profiles, deposits and fields."""
    cfgs = [c for c in mixed_configs(prec) if c["n_cells"] > 0][:4]
    note("inline drain vs drain kernel", prec, block, [c["n_per_species"] for c in cfgs])
    a, b = Context()(cfgs), Context()(cfgs)
    assert a.tuning()["inline_drain"] == 0
    b.set_tuning(block=block, inline_drain=2)
    a.step(37)
    b.step(37)
    for i in range(len(cfgs)):
        assert_same_instance(a, i, b, i)
    d = [a.diagnostics(i) for i in range(len(cfgs))]
    # the drained paths were exercised: collisions and absorption
    assert sum(int(x["elastic"]) for x in d) > 0
    assert sum(int(np.sum(x["absorbed"])) for x in d) > 0


def test_autotuner_keeps_results_and_picks_a_valid_setting(gpu):
    from paper_2308_13092_amd.autotune import autotune
    cfgs = [c for c in mixed_configs(1, n_scale=0.5) if c["n_cells"] > 0][:3]
    note("autotune")
    a, b = Context()(cfgs), Context()(cfgs)
    chosen, table = autotune(a, steps=10, blocks=(256, 1024), blocks_per_cu=(0, 2),
                             sort_intervals=(5, 10))
    assert chosen["block"] in (256, 1024) and chosen["sort_interval"] in (5, 10)
    assert chosen["use_graph"] in (0, 1)
    assert all(a.tuning()[key] == v for key, v in chosen.items())
    assert all(sec > 0 for _, sec in table)
    k = int(a.diagnostics(0)["step"])
    b.step(k)
    for i in range(len(cfgs)):
        assert_same_instance(a, i, b, i)


def test_served_mix_equals_alone(gpu):
    """Continuous batching: requests admitted while others run, through slot
    reuse and a pool that holds only some of them at once; each result equals
    the same discharge run alone."""
    from paper_2308_13092_amd import slot_bytes
    from paper_2308_13092_amd.serve import GpuBackend, Server
    cfgs = [c for c in mixed_configs(1) if c["n_cells"] > 0]
    steps = [120, 40, 200, 80, 60, 150]
    trace = []
    for i, (cfg, n) in enumerate(zip(cfgs, steps)):
        cfg = dict(cfg, k_stop=n, avg_start=n // 2)
        trace.append((0.002 * i, cfg, n))
    sizes = [slot_bytes(c) for _, c, _ in trace]
    pool = int(sum(sorted(sizes)[-3:]) * 1.05)       # room for about three at once
    note("serve", sizes, pool)
    be = GpuBackend(n_slots=3, pool_bytes=pool, precision=1)
    srv = Server(be, n_slots=3, chunk_max=25)
    reqs = srv.run(trace)
    assert all(r.status == "done" for r in reqs), [r.status for r in reqs]
    overlapped = any(r2.admitted < r1.done and r2.admitted > r1.admitted
                     for r1 in reqs for r2 in reqs if r1 is not r2)
    assert overlapped
    for r in reqs:
        note("alone", r.rid)
        alone = Context()([r.cfg])
        alone.step(r.steps + 5)     # k_stop holds it at its last step
        d = alone.diagnostics(0)
        assert d["step"] == r.steps
        p = alone.profiles(0)
        for k in ("ne", "ni", "phi", "eedf"):
            assert np.array_equal(p[k], r.result[k]), (r.rid, k)
        assert r.result["particle_steps"] == d["particle_steps"]
        alone.close()
    be.close()
