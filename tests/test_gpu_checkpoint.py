"""Checkpoint and resume through the C ABI: a run stopped, saved, loaded into
a fresh context (or from a batch slot into a context of its own) and
continued ends bit for bit as the uninterrupted run -- particles by id,
counters, energies, averaged profiles, EEDF and impact histograms; the
velocity moments, FP64 sums whose order varies from run to run, to 1e-12."""
import sys

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

DIAG_KEYS = ["step", "status", "n_samples", "eedf_samples", "n_live", "deposit_total", "kinetic_j_m2",
             "field_j_m2", "absorbed", "absorbed_energy_ev", "see_emitted", "ionisations", "excitations",
             "elastic", "charge_exchange", "candidates", "bound_violations", "particle_steps", "ne_max_m3"]


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def run_cfg(prec, **over):
    cfg = inputs.small_discharge(precision=prec, n_per_species=40_000, nodes=inputs.random_nodes(0.025, 128, 3),
                                 gamma_see=0.3, sort_interval=7, avg_every=1, eedf_every=5, moments=1,
                                 impact_bins=50, impact_angle_bins=30, impact_emax_ev=100.0, seed=41,
                                 v_rf=300.0)
    cfg.update(over)
    return cfg


def same_run(a, ia, b, ib, cfg):
    da, db = a.diagnostics(ia), b.diagnostics(ib)
    for k in DIAG_KEYS:
        assert np.array_equal(np.asarray(da[k]), np.asarray(db[k])), k
    for s in range(2):
        ga, gb = a.get_state(ia, s), b.get_state(ib, s)
        oa, ob = np.argsort(ga["id"]), np.argsort(gb["id"])
        for key in ga:
            assert np.array_equal(ga[key][oa], gb[key][ob]), (s, key)
        for w in range(2):
            ha, hb = a.impacts(ia, s, w), b.impacts(ib, s, w)
            assert np.array_equal(ha["energy"], hb["energy"]) and np.array_equal(ha["angle"], hb["angle"])
        ma, mb = a.moments(ia, s), b.moments(ib, s)
        for key in ma:
            d = np.max(np.abs(ma[key] - mb[key])) / max(np.max(np.abs(mb[key])), 1e-300)
            assert d <= 1e-12, (s, key, d)
    pa, pb = a.profiles(ia), b.profiles(ib)
    for key in pa:
        assert np.array_equal(pa[key], pb[key]), key
    return da


@pytest.mark.parametrize("prec", [0, 1])
def test_resume_equals_uninterrupted_run(gpu, prec):
    from paper_2308_13092_amd import Context
    cfg = run_cfg(prec)
    note("checkpoint", prec, cfg["n_per_species"])
    a = Context([cfg])
    a.step(30)
    ck = a.checkpoint(0)
    note("checkpoint bytes", len(ck))
    a.step(25)
    b = Context([cfg])
    b.step(3)                      # a different state, overwritten by the load
    b.restore(0, ck)
    b.step(25)
    d = same_run(a, 0, b, 0, cfg)
    assert d["step"] == 55 and d["n_samples"] == 55 and d["ionisations"] > 0
    a.close()
    b.close()


def test_resume_from_a_batch_slot(gpu):
    """A checkpoint of one discharge of a batch continues in a context of its
    own as it does in the batch."""
    from paper_2308_13092_amd import Context
    cfg = run_cfg(1)
    other = run_cfg(1, seed=5, nodes=None, n_per_species=20_000)
    note("checkpoint from batch")
    batch = Context([other, cfg])
    batch.step(21)
    ck = batch.checkpoint(1)
    single = Context([cfg])
    single.restore(0, ck)
    batch.step(16)
    single.step(16)
    same_run(batch, 1, single, 0, cfg)
    batch.close()
    single.close()


def test_checkpoint_of_another_configuration_is_refused(gpu):
    from paper_2308_13092_amd import Context, PicError
    from paper_2308_13092_amd._lib import PIC_EINVAL
    note("checkpoint refused")
    a = Context([run_cfg(1)])
    a.step(2)
    ck = a.checkpoint(0)
    b = Context([run_cfg(1, seed=42)])
    before = b.get_state(0, 0)
    with pytest.raises(PicError) as e:
        b.restore(0, ck)
    assert e.value.status == PIC_EINVAL
    with pytest.raises(PicError):
        b.restore(0, ck[: len(ck) // 2])
    after = b.get_state(0, 0)
    assert np.array_equal(np.sort(before["id"]), np.sort(after["id"]))
    a.close()
    b.close()


def test_resume_across_the_forced_re_expression(gpu):
    """FP32 state with no configured sort: the checkpoint is taken 4 steps
    before the sort that re-expresses the candidacy offsets (after 16384
    steps) and restored into a fresh context, whose own forced sort comes
    16384 steps later; both runs end bit for bit alike.  A periodic electron
    box below the ionisation threshold keeps its extent without sorts."""
    from paper_2308_13092_amd import Context
    cfg = inputs.small_discharge(n_cells=16, bc=1, gap_m=0.004, n_species=1, precision=1,
                                 n_per_species=8_000, p_pa=0.05, v_rf=0.0, gamma_see=0.0,
                                 sort_interval=0, te_ev=1.0, seed=43)
    note("checkpoint across the forced re-expression")
    a = Context([cfg])
    a.step(16380)
    ck = a.checkpoint(0)
    a.step(12)
    b = Context([cfg])
    b.restore(0, ck)
    b.step(12)
    da, db = a.diagnostics(0), b.diagnostics(0)
    for key in ("step", "status", "n_live", "deposit_total", "kinetic_j_m2", "field_j_m2", "candidates",
                "elastic", "excitations", "ionisations", "particle_steps"):
        assert np.array_equal(np.asarray(da[key]), np.asarray(db[key])), key
    assert da["step"] == 16392 and da["candidates"][0] > 1000 and da["status"] == 0
    ga, gb = a.get_state(0, 0), b.get_state(0, 0)
    oa, ob = np.argsort(ga["id"]), np.argsort(gb["id"])
    for key in ga:
        assert np.array_equal(ga[key][oa], gb[key][ob]), key
    a.close()
    b.close()
