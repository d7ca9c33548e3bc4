"""RF-averaged profiles over seed ensembles: the HIP path against the oracle.

The oracle's ensemble (32 seeds, EC and MC gathers, FP64) is stored under
``tests/golden/`` by ``make_ensemble.py``, which calls only ``oracle/``.  Here
64 further seeds of the same discharge run on the GPU, in one batched context
per precision, and the ensemble means of n_e, n_i and phi must agree within 3 %
in the L2 norm; the EEDF is compared as a normalised distribution over the bins
where the oracle ensemble holds at least 100 counts.  The seeds differ between
the two sides, so the comparison is between two samples of one distribution.
"""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_ensemble as ens  # noqa: E402

pytestmark = pytest.mark.gpu

GPU_SEEDS = list(range(1000, 1064))
TOL = 0.03


def golden(name):
    with open(os.path.join(HERE, "golden", f"ensemble_small_{name}.json")) as f:
        return json.load(f)


def l2rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", [0, 1])
def test_profiles_match_oracle_ensemble(gpu, prec):
    from paper_2308_13092_amd import Context
    cfgs = [ens.ensemble_config(g, s, precision=prec) for g in (0, 1) for s in GPU_SEEDS]
    print("[case] ensemble", prec, len(cfgs), flush=True)
    ctx = Context(cfgs)
    ctx.step(ens.STEPS + 10)          # k_stop holds each discharge at its last step
    ns = len(GPU_SEEDS)
    report = {}
    for g, name in ((0, "ec"), (1, "mc")):
        ref = golden(name)
        n_ref = len(ref["seeds"])
        prof = [ctx.profiles(g * ns + i) for i in range(ns)]
        for i in range(ns):
            d = ctx.diagnostics(g * ns + i)
            assert d["step"] == ens.STEPS and d["status"] == 0
        for key in ("ne", "ni", "phi"):
            a = np.mean([p[key] for p in prof], axis=0)
            b = np.array(ref["profiles"][key]["mean"])
            report[(name, key)] = l2rel(a, b)
        a = np.sum([p["eedf"] for p in prof], axis=0).astype(np.float64)
        b = np.array(ref["profiles"]["eedf"]["mean"]) * n_ref
        m = b >= 100
        assert m.sum() >= 20
        pa, pb = a / a.sum(), b / b.sum()
        report[(name, "eedf")] = l2rel(pa[m], pb[m])
    print("[ensemble L2]", {f"{k[0]}.{k[1]}": round(v, 4) for k, v in report.items()}, flush=True)
    bad = {k: v for k, v in report.items() if not v <= TOL}
    assert not bad, bad
