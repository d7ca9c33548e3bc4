"""Error paths of the library and physics checks run directly on the GPU path.

Device errors are forced from the host through the inputs (no kernel is made
to fault): an ionising burst that outgrows a tight capacity, a particle whose
move leaves a periodic box by far more than one period, a growth limit just
above 1.  Each freezes its own discharge only; a neighbour in the same batch
ends bitwise as it does alone.
"""
import math
import sys

import numpy as np
import pytest

import inputs
from oracle import physics as ph

pytestmark = pytest.mark.gpu


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def lib():
    import paper_2308_13092_amd._lib as L
    return L


def hot_electrons(n, L, ev, seed, prec):
    """n electrons of energy ev in seeded isotropic directions, uniform in [0, L)."""
    g = inputs.rng(seed)
    x = g.uniform(0.0, L, n)
    mu = g.uniform(-1.0, 1.0, n)
    phi = g.uniform(0.0, 2 * math.pi, n)
    v = math.sqrt(2.0 * ev * ph.QE / ph.ME)
    s = np.sqrt(1.0 - mu * mu)
    vel = [v * mu, v * s * np.cos(phi), v * s * np.sin(phi)]
    st = dict(id=inputs.unique_ids(n, seed + 1), knext=np.zeros(n, np.int64))
    return _with_position(st, x, vel, L, 128, prec)


def cold_ions(n, L, seed, prec):
    g = inputs.rng(seed)
    x = g.uniform(0.0, L, n)
    vel = [g.normal(0.0, 250.0, n) for _ in range(3)]
    st = dict(id=inputs.unique_ids(n, seed + 1) | np.uint64(1 << 63), knext=np.full(n, 10 ** 6))
    return _with_position(st, x, vel, L, 128, prec)


def _with_position(st, x, vel, L, N, prec):
    if prec == 0:
        st["x"] = x
        st.update(vx=vel[0], vy=vel[1], vz=vel[2])
    else:
        s = x / (L / N)
        cell = np.minimum(np.floor(s), N - 1).astype(np.int32)
        off = np.clip((s - cell).astype(np.float32), 0.0, np.nextafter(np.float32(1), np.float32(0)))
        st.update(cell=cell, off=off, vx=vel[0].astype(np.float32), vy=vel[1].astype(np.float32),
                  vz=vel[2].astype(np.float32))
    return st


def burst_cfg(prec, n, **over):
    p = 100.0 * inputs.MTORR
    n_g = ph.gas_density(p, 300.0)
    cfg = inputs.small_discharge(precision=prec, n_per_species=n, p_pa=p, capacity=n,
                                 nu_max_e=ph.nu_max_electron(n_g), nu_max_i=ph.nu_max_ion(n_g, 200.0, 300.0))
    cfg.update(over)
    return cfg


def quiet_cfg(prec):
    return inputs.small_discharge(precision=prec, n_per_species=5000, seed=9)


def load_burst(ctx, inst, prec, n):
    ctx.set_state(inst, 0, hot_electrons(n, 0.025, 60.0, 21, prec))
    ctx.set_state(inst, 1, cold_ions(n, 0.025, 22, prec))


def same_as_alone(batch, i, cfg):
    from paper_2308_13092_amd import Context
    alone = Context([cfg])
    k = int(batch.diagnostics(i)["step"])
    alone.step(k)
    for s in range(2):
        a, b = batch.get_state(i, s), alone.get_state(0, s)
        oa, ob = np.argsort(a["id"]), np.argsort(b["id"])
        for key in a:
            assert np.array_equal(a[key][oa], b[key][ob]), (s, key)
    alone.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_capacity_overflow_freezes_only_its_discharge(gpu, prec):
    L = lib()
    n = 4096                                   # a multiple of 64: capacity is exactly n
    cfgs = [burst_cfg(prec, n), quiet_cfg(prec)]
    note("capacity", prec)
    ctx = L.Context(cfgs)
    load_burst(ctx, 0, prec, n)
    ctx.step(12)
    d = ctx.diagnostics(0, allow_error=True)
    assert d["return_status"] == L.PIC_ECAPACITY
    assert d["step"] < 12                      # frozen at the step that overflowed
    assert max(d["extent"]) <= n
    with pytest.raises(L.PicError):
        ctx.diagnostics(0)
    st = ctx.get_state(0, 0)                   # the frozen state stays readable
    assert len(st["id"]) <= n
    d1 = ctx.diagnostics(1)
    assert d1["step"] == 12
    same_as_alone(ctx, 1, cfgs[1])


@pytest.mark.parametrize("prec", [0, 1])
def test_growth_limit(gpu, prec):
    L = lib()
    n = 4096
    cfg = burst_cfg(prec, n, capacity=8 * n, growth_limit=1.02)
    note("growth", prec)
    ctx = L.Context([cfg])
    load_burst(ctx, 0, prec, n)
    ctx.step(20)
    d = ctx.diagnostics(0, allow_error=True)
    assert d["return_status"] == L.PIC_EGROWTH
    assert d["n_live"][0] > 1.02 * n
    assert d["step"] < 20


@pytest.mark.parametrize("prec", [0, 1])
def test_runaway_particle_in_a_periodic_box(gpu, prec):
    L = lib()
    N, Lx = 128, 0.025
    cfgs = [inputs.small_discharge(precision=prec, bc=1, v_rf=0.0, n_per_species=2000, collisions=0,
                                   n_species=1),
            quiet_cfg(prec)]
    note("nonfinite", prec)
    ctx = L.Context(cfgs)
    st = ctx.get_state(0, 0)
    st["vx"] = st["vx"].copy()
    st["vx"][17] = 1e30                       # finite, but crosses ~1e19 periods in one step
    ctx.set_state(0, 0, st)
    ctx.step(5)
    d = ctx.diagnostics(0, allow_error=True)
    assert d["return_status"] == L.PIC_ENONFINITE
    assert d["step"] == 1
    assert ctx.diagnostics(1)["step"] == 5
    same_as_alone(ctx, 1, cfgs[1])


@pytest.mark.parametrize("prec", [0, 1])
def test_argument_errors_leave_the_context_usable(gpu, prec):
    L = lib()
    cfg = quiet_cfg(prec)
    ctx = L.Context([cfg])
    st = ctx.get_state(0, 0)
    bad = {k: v.copy() for k, v in st.items()}
    if prec == 0:
        bad["x"][3] = 0.025                    # x must lie in [0, L)
    else:
        bad["off"][3] = 1.0                    # offsets in [0, 1)
    with pytest.raises(L.PicError) as e:
        ctx.set_state(0, 0, bad)
    assert e.value.status == L.PIC_EINVAL
    bad = {k: v.copy() for k, v in st.items()}
    bad["vy"][0] = np.nan
    with pytest.raises(L.PicError) as e:
        ctx.set_state(0, 0, bad)
    assert e.value.status == L.PIC_EINVAL
    big = {k: np.concatenate([v] * 3) for k, v in st.items()}
    with pytest.raises(L.PicError) as e:
        ctx.set_state(0, 0, big)
    assert e.value.status == L.PIC_ECAPACITY
    with pytest.raises(L.PicError) as e:
        ctx.diagnostics(3)
    assert e.value.status == L.PIC_EINVAL
    with pytest.raises(L.PicError) as e:
        ctx.set_tuning(block=128)
    assert e.value.status == L.PIC_EINVAL
    with pytest.raises(L.PicError) as e:
        ctx.slot_reset(0, dict(cfg, precision=1 - prec))
    assert e.value.status == L.PIC_EINVAL
    ctx.set_state(0, 0, st)                    # a valid state: the deposit is now stale
    with pytest.raises(L.PicError) as e:
        ctx.poisson()
    assert e.value.status == L.PIC_ESTATE
    ctx.deposit()
    ctx.poisson()
    ctx.step(3)
    assert ctx.diagnostics(0)["step"] == 3


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gather", [0, 1, 2])
def test_cold_plasma_frequency_on_the_gpu(gpu, prec, gather):
    """Periodic box, cold electrons at cell centres displaced by
    0.01 dx sin(2 pi x/L), neutralising background: the charge perturbation
    oscillates at (2/dt) asin(w_pe dt/2) (leapfrog dispersion)."""
    L = lib()
    N, ppc, n0, wdt, Lx = 128, 8, 1e15, 0.1, 0.01
    wpe = math.sqrt(n0 * ph.QE ** 2 / (ph.EPS0 * ph.ME))
    dx = Lx / N
    n = N * ppc
    x0 = (np.arange(n) + 0.5) * (Lx / n)
    x = x0 + 0.01 * dx * np.sin(2 * math.pi * x0 / Lx)
    z = np.zeros(n)
    st = _with_position(dict(id=np.arange(n, dtype=np.uint64), knext=np.full(n, 2 ** 31 - 1)),
                        x, [z, z.copy(), z.copy()], Lx, N, prec)
    cfg = inputs.small_discharge(n_cells=N, bc=1, gap_m=Lx, v_rf=0.0, n0_m3=n0, n_per_species=n,
                                 dt_s=wdt / wpe, gather=gather, n_species=1, collisions=0,
                                 precision=prec)
    note("cold plasma", prec, gather)
    ctx = L.Context([cfg])
    ctx.set_state(0, 0, st)
    ctx.deposit()
    basis = np.cos(2 * math.pi * (np.arange(N) * dx) / Lx)
    amp = []
    for _ in range(int(round(8 * 2 * math.pi / wdt))):
        ctx.step(1)
        amp.append(float(np.sum(ctx.fields(0)["A_e"][:N].astype(np.float64) * basis)))
    s = np.asarray(amp) - np.mean(amp)
    idx = np.nonzero(np.signbit(s[:-1]) != np.signbit(s[1:]))[0]
    t = [(i + s[i] / (s[i] - s[i + 1])) * cfg["dt_s"] for i in idx]
    w = math.pi * (len(t) - 1) / (t[-1] - t[0])
    expect = (2 / cfg["dt_s"]) * math.asin(wdt / 2)
    assert abs(w / expect - 1) < 0.005, (w, expect)
