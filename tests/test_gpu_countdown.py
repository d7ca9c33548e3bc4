"""The FP32 form's collision candidacy (a 16-bit offset from the slot's
epoch step in each particle's hot word, with the far flag and the knext array
for candidacies beyond its range or overdue) against the oracle's absolute
candidate steps.

A periodic electron box at very low pressure (waits of ~1e8 steps) is set to
candidacies spread around the offset's range, set_step moves it to k0, it is
advanced 2^16 - 9 steps on the GPU with no configured sort (the epoch is
re-expressed by the sorts forced every 16384 steps), and then the oracle and
the GPU advance together: every candidacy happens at its step, every far
particle keeps its candidacy, and the state matches the oracle's by id.
"""
import sys

import numpy as np
import pytest

import inputs
from gpu_common import compare_species, oracle_from_states, species_dict

pytestmark = pytest.mark.gpu

CNT_MAX = 2 ** 16 - 1
K0 = 100
INT32_MAX = 2 ** 31 - 1


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_countdown_across_its_range(gpu):
    from paper_2308_13092_amd import Context
    offsets = [0, 1, 5, CNT_MAX - 9, CNT_MAX - 3, CNT_MAX - 1, CNT_MAX, CNT_MAX + 1, CNT_MAX + 3,
               CNT_MAX + 9, 2 * CNT_MAX + 7, 3_000_000]
    reps = 24
    kn = np.array([K0 + o for o in offsets] * reps + [50] * reps + [INT32_MAX] * reps, dtype=np.int64)
    n = len(kn)
    cfg = inputs.small_discharge(n_cells=16, bc=1, gap_m=0.004, n_species=1, precision=1,
                                 n_per_species=n, p_pa=1e-6, v_rf=0.0, gamma_see=0.0,
                                 sort_interval=0, te_ev=1.0)
    st = inputs.particles_fp32(n, 16, 4.0e5, seed=77)
    st["knext"] = kn
    note("countdown", n, "particles", offsets)
    ctx = Context([cfg])
    ctx.set_state(0, 0, st)
    ctx.set_step(0, K0)
    g0 = ctx.get_state(0, 0)
    o = np.argsort(g0["id"])
    os_ = np.argsort(st["id"])
    assert np.array_equal(g0["knext"][o].astype(np.int64), kn[os_])   # exact, past and far included
    n_steps = CNT_MAX - 9
    ctx.step(n_steps)
    k1 = K0 + n_steps
    d = ctx.diagnostics()
    assert d["step"] == k1
    g1 = ctx.get_state(0, 0)
    # candidacies before k1 happened (once each: their next waits are ~1e8 steps)
    due = kn[os_] < k1
    assert d["candidates"][0] == int(due.sum())
    o1 = np.argsort(g1["id"])
    kept = g1["knext"][o1].astype(np.int64)
    assert np.array_equal(kept[~due], kn[os_][~due])
    assert np.all(kept[due] >= k1)
    note("at", k1, "candidates", int(d["candidates"][0]))
    # the oracle and the GPU together from there
    ref = oracle_from_states(cfg, [g1], k1)
    ctx2 = Context([cfg])
    ctx2.set_state(0, 0, g1)
    ctx2.set_step(0, k1)
    for step in range(20):
        ctx.step(1)
        ctx2.step(1)
        ref.step()
    for c in (ctx, ctx2):
        stats = compare_species(c.get_state(0, 0), species_dict(ref.sp[0]), ref.grid, 1e-5, 1e-5, 1e7,
                                max_flips=0)
        note("species", stats)
        assert c.diagnostics()["candidates"][0] - (d["candidates"][0] if c is ctx else 0) == \
            ref.mcc[0].candidates
    assert ref.mcc[0].candidates == int(((kn >= k1) & (kn < k1 + 20)).sum())
    ctx.close()
    ctx2.close()


def test_split_calls_re_express_like_pic_step(gpu):
    """With no configured sort, pic_step and the split calls (pic_deposit,
    pic_poisson, pic_gather_push, pic_mcc) both re-express the candidacy
    offsets after 16384 steps (a forced sort): the two runs end bitwise
    equal by id, every candidacy before the end happened once, and the
    others, near and far, decode to the steps they were given."""
    from paper_2308_13092_amd import Context
    n_steps = 16384 + 30
    reps = 16
    offsets = [0, 1, 100, 16383, 16384, 16385, n_steps - 1, n_steps, n_steps + 5, CNT_MAX - 1, CNT_MAX,
               CNT_MAX + 16384, CNT_MAX + 16390, 2 * CNT_MAX + 3]
    kn = np.array([K0 + o for o in offsets] * reps + [INT32_MAX] * reps, dtype=np.int64)
    n = len(kn)
    cfg = inputs.small_discharge(n_cells=16, bc=1, gap_m=0.004, n_species=1, precision=1,
                                 n_per_species=n, p_pa=1e-6, v_rf=0.0, gamma_see=0.0,
                                 sort_interval=0, te_ev=1.0)
    st = inputs.particles_fp32(n, 16, 4.0e5, seed=78)
    st["knext"] = kn
    note("split calls re-express", n, "particles", n_steps, "steps")
    ctxs = []
    for _ in range(2):
        c = Context([cfg])
        c.set_state(0, 0, st)
        c.set_step(0, K0)
        ctxs.append(c)
    a, b = ctxs
    a.step(n_steps)
    for _ in range(n_steps):
        b.deposit()
        b.poisson()
        b.gather_push()
        b.mcc()
    k1 = K0 + n_steps
    os_ = np.argsort(st["id"])
    due = kn[os_] < k1
    for c in (a, b):
        d = c.diagnostics()
        assert d["step"] == k1
        assert d["candidates"][0] == int(due.sum())
        g = c.get_state(0, 0)
        o = np.argsort(g["id"])
        kept = g["knext"][o].astype(np.int64)
        assert np.array_equal(kept[~due], kn[os_][~due])
        assert np.all(kept[due] >= k1)
    ga, gb = a.get_state(0, 0), b.get_state(0, 0)
    oa, ob = np.argsort(ga["id"]), np.argsort(gb["id"])
    for key in ga:
        assert np.array_equal(ga[key][oa], gb[key][ob]), key
    a.close()
    b.close()
