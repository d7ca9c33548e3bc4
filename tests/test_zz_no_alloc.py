"""The entry point for callers that cannot allocate (pic_diagnostics_noalloc)
against pic_diagnostics, through the C ABI: two calls in a row, the second
over fewer instances, each record equal to the per-instance call's."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS_EXACT = ["step", "status", "n_samples", "eedf_samples", "n_live", "extent", "deposit_total",
                "kinetic_j_m2", "field_j_m2", "absorbed", "absorbed_energy_ev", "see_emitted",
                "ionisations", "excitations", "elastic", "charge_exchange", "candidates",
                "bound_violations", "particle_steps", "ne_max_m3", "wpe_dt_max", "vmax_dt_over_dxmin",
                "lambda_de_over_dxmin", "nu_max"]


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def same(a, b):
    for k in FIELDS_EXACT:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (k, a[k], b[k])


def test_noalloc_diagnostics_equal_the_per_instance_call(gpu):
    from paper_2308_13092_amd import Context, PicError, configs
    from paper_2308_13092_amd._lib import PIC_EINVAL
    cfgs = [configs.small(n_per_species=30_000, precision=1, seed=3, gamma_see=0.2),
            configs.small(n_per_species=5_000, precision=1, seed=4, n_cells=64, avg_every=1),
            configs.small(n_per_species=60_000, precision=1, seed=5, v_rf=350.0)]
    note("noalloc diagnostics", [c["n_per_species"] for c in cfgs])
    ctx = Context(cfgs)
    ctx.step(12)
    first = ctx.diagnostics_noalloc([0, 1, 2])
    for i, d in enumerate(first):
        same(d, ctx.diagnostics(i))
        assert d["n_live"].sum() > 0 and d["deposit_total"][0] == d["n_live"][0] * 2 ** 32
    ctx.step(7)
    second = ctx.diagnostics_noalloc([1])      # fewer instances than the call before
    assert len(second) == 1
    same(second[0], ctx.diagnostics(1))
    assert second[0]["step"] == first[1]["step"] + 7
    # out-of-range sizes are rejected before any work
    for n_bad in (0, 513):
        with pytest.raises(PicError) as e:
            ctx.diagnostics_noalloc([0] * n_bad)
        assert e.value.status == PIC_EINVAL
    ctx.close()
