"""GPU parity: the HIP library, called through its C ABI, against the oracle.

Every case states its seed and shape before it touches the GPU.
"""
import math
import sys

import numpy as np
import pytest

import inputs
from gpu_common import (compare_species, gpu_from_states, normwise, oracle_from_states,
                        qmdt_abs, species_dict)
from oracle import physics as ph
from oracle.pic import Grid
from oracle.sim import Sim

pytestmark = pytest.mark.gpu

N_PART = 50_003          # not a multiple of the tile size: exercises the ragged tail
K0 = 37


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def Context():
    from paper_2308_13092_amd import Context as C
    return C


def case_cfg(prec, kind, gather=0, n=N_PART, **over):
    L, N = 0.025, 128
    nodes = None
    bc = 0
    if kind == "nonuniform":
        nodes = inputs.random_nodes(L, N, seed=11)
    elif kind == "refined":
        from oracle.grid import refined_nodes
        nodes = refined_nodes(L, L / 512, L / 64, 0.004)
        N = len(nodes) - 1
    elif kind == "periodic":
        bc = 1
    n_g = ph.gas_density(50 * inputs.MTORR, 300.0)
    cfg = inputs.small_discharge(precision=prec, gather=gather, nodes=nodes, bc=bc, n_per_species=n,
                                 n_cells=N,
                                 nu_max_e=ph.nu_max_electron(n_g), nu_max_i=ph.nu_max_ion(n_g, 200.0, 300.0),
                                 gamma_see=0.3, sort_interval=0)
    cfg.update(over)
    return cfg


def field_tol(kind, ref):
    """Normwise tolerance on E.  Eq (5) forms E by differencing phi, so the
    oracle's own E carries ~eps |phi| / h of rounding; on fine cells that term
    exceeds 1e-12 |E| and is added (64 ulps of phi).  Periodic: the
    neutralising background makes the net charge a small difference of large
    sums, and both solves carry ~1e-12 of rounding."""
    if kind == "periodic":
        return 1e-9
    cond = 64 * np.finfo(float).eps * np.max(np.abs(ref.phi)) / (np.min(ref.grid.h) * np.max(np.abs(ref.E)))
    return 1e-12 + cond


def case_states(cfg, seed=5, ve=1.0e6):
    prec = cfg["precision"]
    L = cfg["gap_m"] if cfg["nodes"] is None else float(cfg["nodes"][-1])
    N = cfg["n_cells"]
    out = []
    for s, vs in ((0, ve), (1, 2.0e3)):
        if prec == 0:
            st = inputs.particles_fp64(cfg["n_per_species"], L, vs, seed + 10 * s, k=K0)
        else:
            st = inputs.particles_fp32(cfg["n_per_species"], N, vs, seed + 10 * s, k=K0)
        out.append(st)
    return out


KINDS = ["uniform", "nonuniform", "refined", "periodic"]
# (grid kind, gather): EC and MC on every grid, second-order EC on uniform ones
KIND_GATHER = [(k, g) for k in KINDS for g in (0, 1)] + [("uniform", 2), ("periodic", 2)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,gather", [(k, 0) for k in KINDS] + [("uniform", 2), ("periodic", 2)])
def test_deposit_is_bit_exact(gpu, prec, kind, gather):
    note("deposit", prec, kind, gather, N_PART)
    cfg = case_cfg(prec, kind, gather=gather)
    states = case_states(cfg)
    ctx = gpu_from_states(cfg, states, K0, Context())
    ctx.deposit()
    f = ctx.fields()
    ref = oracle_from_states(cfg, states, K0)
    A = ref.deposit()
    assert np.array_equal(f["A_e"], A[0])
    assert np.array_equal(f["A_i"], A[1])
    d = ctx.diagnostics()
    assert list(d["deposit_total"]) == [N_PART * 2 ** 32, N_PART * 2 ** 32]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,gather", KIND_GATHER)
def test_poisson_and_field(gpu, prec, kind, gather):
    note("poisson", prec, kind, gather)
    cfg = case_cfg(prec, kind, gather=gather)
    states = case_states(cfg)
    ctx = gpu_from_states(cfg, states, K0, Context())
    ctx.deposit()
    ctx.poisson()
    f = ctx.fields()
    ref = oracle_from_states(cfg, states, K0)
    ref.deposit()
    ref.solve()
    tol = 1e-12 if kind != "periodic" else 1e-9
    assert normwise(f["phi"], ref.phi) <= tol
    assert normwise(f["E"], ref.E) <= field_tol(kind, ref)
    assert np.max(np.abs(f["E32"] - ref.E.astype(np.float32))) <= 1e-6 * np.max(np.abs(ref.E))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,gather", KIND_GATHER)
@pytest.mark.parametrize("path", ["fused", "separate"])
def test_single_step(gpu, prec, kind, gather, path):
    note("single step", prec, kind, gather, path)
    cfg = case_cfg(prec, kind, gather=gather)
    states = case_states(cfg)
    ref = oracle_from_states(cfg, states, K0)
    ctx = gpu_from_states(cfg, states, K0, Context())
    if path == "fused":
        ctx.step(1)
    else:
        ctx.deposit()
        ctx.poisson()
        ctx.gather_push()
        ctx.mcc()
    ref.step()
    f = ctx.fields()
    tol = 1e-12 if kind != "periodic" else 1e-9
    tol_e = field_tol(kind, ref)
    assert normwise(f["phi"], ref.phi) <= tol
    assert normwise(f["E"], ref.E) <= tol_e
    rel = max(1e-12, tol_e) if prec == 0 else 1e-5
    emax = float(np.max(np.abs(ref.E)))
    for s in range(2):
        g = ctx.get_state(0, s)
        r = species_dict(ref.sp[s])
        vs = float(np.max(np.abs(np.asarray(states[s]["vx"], dtype=np.float64)))) + \
            qmdt_abs(cfg, s) * emax
        stats = compare_species(g, r, ref.grid, rel, rel, vs, max_flips=3 + len(r["id"]) // 20000)
        note("species", s, stats)
    d = ctx.diagnostics()
    assert d["step"] == K0 + 1
    for s in range(2):
        assert d["absorbed"][s].sum() == ref.absorbed[s].sum()
    assert d["see_emitted"] == ref.see_emitted
    assert d["ionisations"] == ref.mcc[0].ionisation
    assert d["candidates"][0] == ref.mcc[0].candidates
    assert d["candidates"][1] == ref.mcc[1].candidates
    assert d["charge_exchange"] == ref.mcc[1].cx
    assert d["bound_violations"] == 0


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", ["uniform", "nonuniform"])
def test_initial_load(gpu, prec, kind):
    note("init", prec, kind)
    cfg = case_cfg(prec, kind, n=20_001)
    ctx = Context()([cfg])
    ref = Sim(cfg)
    for s in range(2):
        g = ctx.get_state(0, s)
        r = species_dict(ref.sp[s])
        vs = float(np.max(np.abs(r["vx"])))
        compare_species(g, r, ref.grid, 1e-14 if prec == 0 else 1e-7, 1e-13, vs, max_flips=0)
    f = ctx.fields()
    A = ref.deposit()
    assert np.array_equal(f["A_e"], A[0]) and np.array_equal(f["A_i"], A[1])


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,gather", [("uniform", 0), ("periodic", 0), ("uniform", 2), ("periodic", 2)])
def test_next_deposit_includes_new_particles(gpu, prec, kind, gather):
    """The fused step deposits x^{k+1} of every particle, ionisation products
    and secondary electrons included, straight into the next step's grid
    (products of cells 0 and N-1 touch the end nodes, which a periodic box
    shares).  Hot electrons make ionisations frequent.  With no branch flips
    the FP32 form's deposit is bit-exact; the FP64 form's positions agree to
    rounding, so a node's sum may differ by a unit for a particle whose
    weight rounds the other way."""
    note("next deposit", prec, kind, gather)
    cfg = case_cfg(prec, kind, gather=gather)
    states = case_states(cfg, ve=3.0e6)
    ref = oracle_from_states(cfg, states, K0)
    ctx = gpu_from_states(cfg, states, K0, Context())
    ctx.step(1)
    ref.step()
    assert ref.mcc[0].ionisation > 200
    for s in range(2):
        st = compare_species(ctx.get_state(0, s), species_dict(ref.sp[s]), ref.grid, 1e-5, 1e-5,
                             1e7, max_flips=0)
        note("species", s, st)
    f = ctx.fields()
    A = ref.deposit()
    n = len(A[0]) if kind != "periodic" else len(A[0]) - 1
    for key, a in (("A_e", A[0]), ("A_i", A[1])):
        d = np.abs(f[key].astype(np.int64) - a)
        if prec == 1:
            assert np.array_equal(f[key], a), (key, int(d.max()))
        else:
            assert d.max() <= 8, (key, int(d.max()))
        assert int(f[key][:n].sum()) == int(a[:n].sum())


@pytest.mark.parametrize("prec", [0, 1])
def test_fused_equals_separate_calls_bitwise(gpu, prec):
    note("fused vs separate", prec)
    cfg = case_cfg(prec, "nonuniform", n=30_000)
    a = Context()([cfg])
    b = Context()([cfg])
    a.step(20)
    for _ in range(20):
        b.deposit()
        b.poisson()
        b.gather_push()
        b.mcc()
    for s in range(2):
        ga, gb = a.get_state(0, s), b.get_state(0, s)
        oa, ob = np.argsort(ga["id"]), np.argsort(gb["id"])
        for k in ga:
            assert np.array_equal(ga[k][oa], gb[k][ob]), k


@pytest.mark.parametrize("prec", [0, 1])
def test_sort_interval_does_not_change_results(gpu, prec):
    note("sort invariance", prec)
    outs = []
    for S in (1, 7, 0):
        cfg = case_cfg(prec, "nonuniform", n=30_000, sort_interval=S)
        c = Context()([cfg])
        c.step(30)
        outs.append([c.get_state(0, s) for s in range(2)])
        d = c.diagnostics()
        for s in range(2):   # dead and new particles since the last sort stay in the extent
            assert d["extent"][s] >= d["n_live"][s] == len(outs[-1][s]["id"]), (S, s)
    for s in range(2):
        ref = outs[0][s]
        o0 = np.argsort(ref["id"])
        for other in outs[1:]:
            o1 = np.argsort(other[s]["id"])
            for k in ref:
                assert np.array_equal(ref[k][o0], other[s][k][o1]), (s, k)


@pytest.mark.parametrize("prec", [0, 1])
def test_sort_keeps_every_particle_in_cell_order(gpu, prec):
    """An explicit sort after unsorted steps (particles moved, some absorbed,
    products appended): every live particle is kept once with its values
    bitwise, the absorbed ones are dropped, and the storage order is by
    cell."""
    note("sort keeps particles", prec)
    cfg = case_cfg(prec, "nonuniform", n=200_000)
    c = Context()([cfg])
    c.step(9)
    before = [c.get_state(0, s) for s in range(2)]
    c.sort()
    after = [c.get_state(0, s) for s in range(2)]
    d = c.diagnostics()
    nodes = np.asarray(cfg["nodes"], dtype=np.float64)
    for s in range(2):
        a, b = before[s], after[s]
        assert len(b["id"]) == len(a["id"]) == d["n_live"][s] == d["extent"][s]
        assert len(np.unique(b["id"])) == len(b["id"])
        oa, ob = np.argsort(a["id"]), np.argsort(b["id"])
        for k in a:
            assert np.array_equal(a[k][oa], b[k][ob]), (s, k)
        cells = b["cell"] if "cell" in b else np.searchsorted(nodes, b["x"], side="right") - 1
        assert np.all(np.diff(cells) >= 0), s


@pytest.mark.parametrize("prec", [0, 1])
def test_run_twice_identical_and_charge_exact(gpu, prec):
    note("run twice", prec)
    cfg = case_cfg(prec, "uniform", n=30_000, sort_interval=5, avg_every=1, eedf_every=10)
    runs = []
    for _ in range(2):
        c = Context()([cfg])
        c.step(40)
        runs.append((c.diagnostics(), c.profiles(), [c.get_state(0, s) for s in range(2)]))
    (d0, p0, s0), (d1, p1, s1) = runs
    for k in ("n_live", "kinetic_j_m2", "absorbed", "particle_steps", "ionisations", "field_j_m2"):
        assert np.array_equal(np.asarray(d0[k]), np.asarray(d1[k])), k
    for k in ("ne", "ni", "phi", "eedf"):
        assert np.array_equal(p0[k], p1[k]), k
    assert list(d0["deposit_total"]) == [int(n) * 2 ** 32 for n in d0["n_live"]]


def test_diagnostics_against_oracle(gpu):
    note("diagnostics")
    cfg = case_cfg(0, "uniform", n=20_000)
    ctx = Context()([cfg])
    ref = Sim(cfg)
    ctx.step(5)
    ref.run(5)
    d = ctx.diagnostics()
    for s in range(2):
        assert d["n_live"][s] == ref.sp[s].n
        assert d["kinetic_j_m2"][s] == pytest.approx(ref.kinetic_energy(s), rel=1e-6)
    assert d["field_j_m2"] == pytest.approx(ref.field_energy, rel=1e-9)
    assert d["particle_steps"] > 0


@pytest.mark.parametrize("prec", [0, 1])
def test_impact_distributions_against_oracle(gpu, prec):
    """Energy and angle histograms of absorbed particles over 30 steps from the
    same initial load: totals equal the absorbed counts on both sides, and the
    histograms agree up to particles whose bin depends on the last ulp of acos
    (or whose trajectories the field's rounding has moved apart)."""
    note("impacts", prec)
    cfg = case_cfg(prec, "uniform", n=20_000, avg_every=1, impact_bins=100, impact_angle_bins=45,
                   impact_emax_ev=200.0)
    ctx = Context()([cfg])
    ref = Sim(cfg)
    ctx.step(30)
    ref.run(30)
    d = ctx.diagnostics()
    for s in range(2):
        for w in range(2):
            h = ctx.impacts(0, s, w)
            assert h["energy"].sum() == d["absorbed"][s][w]
            assert h["angle"].sum() == d["absorbed"][s][w]
            tot = max(int(ref.absorbed[s, w]), 1)
            assert abs(int(d["absorbed"][s][w]) - int(ref.absorbed[s, w])) <= 2 + tot // 100
            de = np.abs(h["energy"] - ref.impact_e[s, w]).sum()
            da = np.abs(h["angle"] - ref.impact_a[s, w]).sum()
            note("impact", s, w, int(ref.absorbed[s, w]), int(de), int(da))
            assert de <= 4 + tot // 50 and da <= 4 + tot // 50


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,gather", [(k, g) for k in ("uniform", "refined", "periodic") for g in (0, 1)]
                         + [("uniform", 2), ("periodic", 2)])
def test_moments_against_oracle(gpu, prec, kind, gather):
    """Averaged velocity moments and power after one step from identical
    state (sampled before the push): FP64 sums in different orders."""
    note("moments", prec, kind, gather)
    cfg = case_cfg(prec, kind, gather=gather, avg_every=1, moments=1)
    states = case_states(cfg)
    ref = oracle_from_states(cfg, states, K0)
    ctx = gpu_from_states(cfg, states, K0, Context())
    ctx.step(1)
    ref.step()
    for s in range(2):
        g = ctx.moments(0, s)
        r = ref.moments(s)
        for key in ("ux", "tx", "power"):
            assert normwise(g[key], r[key]) <= 1e-10, (s, key, normwise(g[key], r[key]))


def test_moments_are_opt_in(gpu):
    """Without moments = 1 nothing is accumulated and pic_moments says so;
    the step itself is unchanged."""
    import paper_2308_13092_amd._lib as L
    note("moments off")
    cfg = case_cfg(1, "uniform", avg_every=1)
    states = case_states(cfg)
    a = gpu_from_states(cfg, states, K0, Context())
    b = gpu_from_states(dict(cfg, moments=1), states, K0, Context())
    a.step(3)
    b.step(3)
    with pytest.raises(L.PicError) as e:
        a.moments(0, 0)
    assert e.value.status == L.PIC_ESTATE
    for s in range(2):
        sa, sb = a.get_state(0, s), b.get_state(0, s)
        oa, ob = np.argsort(sa["id"]), np.argsort(sb["id"])   # storage order is unspecified
        for key in sa:
            assert np.array_equal(sa[key][oa], sb[key][ob]), (s, key)
