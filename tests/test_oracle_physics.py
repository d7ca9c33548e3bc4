"""Pins of the oracle's gas physics and stability monitors against values fixed
outside the oracle: calculus (the peak of ln(x)/x), a bounded minimiser,
the stated peaks and summed-rate maximum of the synthetic argon cross
sections, textbook plasma constants (NRL formulary: omega_pe = 5.64e4 n^1/2
rad/s and lambda_D = 743 (T/n)^1/2 cm, n in cm^-3, T in eV), hand values on
crafted states, and energy conservation of the oracle's own push.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import inputs
from oracle import physics as ph
from oracle.pic import FP64, Grid, Species, push_fp64
from oracle.sim import Sim


# -- cross sections ----------------------------------------------------------
def test_elastic_cross_section_hand_values():
    # 1e-19 m^2 at rest, half of it at 20 eV, a third at 40 eV
    assert ph.sigma_el(0.0) == 1.0e-19
    assert ph.sigma_el(20.0) == pytest.approx(0.5e-19, rel=1e-15)
    assert ph.sigma_el(40.0) == pytest.approx(1.0e-19 / 3.0, rel=1e-15)


@pytest.mark.parametrize("fn,thr,amp,peak_ev,peak_sigma", [
    (ph.sigma_ex, 11.5, 2.7e-20, 31.0, 9.9e-21),     # stated: 9.9e-21 m^2 near 31 eV
    (ph.sigma_iz, 15.76, 7.6e-20, 43.0, 2.8e-20),    # stated: 2.8e-20 m^2 near 43 eV
])
def test_inelastic_cross_sections_thresholds_and_peaks(fn, thr, amp, peak_ev, peak_sigma):
    # zero at and below the threshold, positive just above it
    below = fn(np.array([0.0, 1.0, thr * 0.999, thr]))
    assert np.all(below == 0.0)
    assert fn(np.array([thr * (1 + 1e-9)]))[0] > 0.0
    # ln(x)/x peaks at x = e with value 1/e: the maximum of the oracle's
    # function, found by a bounded minimiser, sits at thr * e with amp / e
    res = minimize_scalar(lambda e: -float(fn(np.array([e]))[0]), bounds=(thr * 1.01, 10 * thr),
                          method="bounded", options=dict(xatol=1e-9))
    assert res.x == pytest.approx(thr * math.e, rel=1e-4)
    assert -res.fun == pytest.approx(amp / math.e, rel=1e-9)
    # and agrees with the stated peak location and value to their two digits
    assert abs(res.x - peak_ev) < 0.5
    assert abs(-res.fun / peak_sigma - 1) < 0.01
    # decays on both sides of the peak
    lo = fn(np.linspace(thr * 1.001, res.x * 0.999, 200))
    hi = fn(np.linspace(res.x * 1.001, 1e5, 2000))
    assert np.all(np.diff(lo) > 0) and np.all(np.diff(hi) < 0)


def rate(eps):
    """Summed electron collision rate coefficient sum_p sigma_p(eps) v(eps) (m^3/s)."""
    eps = np.atleast_1d(np.asarray(eps, dtype=np.float64))
    v = np.sqrt(2.0 * eps * ph.QE / ph.ME)
    return (ph.sigma_el(eps) + ph.sigma_ex(eps) + ph.sigma_iz(eps)) * v


def test_summed_rate_maximum_and_decay():
    """Stated: max over energy of sum sigma v = 2.77e-13 m^3/s near 64 eV, and
    the sum decays above that."""
    res = minimize_scalar(lambda e: -float(rate(e)[0]), bounds=(20.0, 300.0), method="bounded",
                          options=dict(xatol=1e-8))
    top, at = -res.fun, res.x
    assert abs(top / 2.77e-13 - 1) < 0.005
    assert 60.0 < at < 68.0
    tail = rate(np.geomspace(at * 1.0001, 1e7, 4000))
    assert np.all(np.diff(tail) < 0)
    # below the peak the rate stays under it everywhere on a fine scan
    assert np.all(rate(np.geomspace(1e-6, at, 20000)) <= top * (1 + 1e-12))


@pytest.mark.parametrize("p_mtorr", [10.0, 20.0, 50.0, 100.0])
def test_electron_bound_covers_every_energy(p_mtorr):
    n_g = ph.gas_density(p_mtorr * inputs.MTORR, 300.0)
    nu = ph.nu_max_electron(n_g)
    res = minimize_scalar(lambda e: -float(rate(e)[0]), bounds=(20.0, 300.0), method="bounded",
                          options=dict(xatol=1e-8))
    top = -res.fun
    # the oracle's log scan finds the continuous maximum to a few parts in 1e8
    assert nu / (1.02 * n_g * top) == pytest.approx(1.0, abs=1e-7)
    eps = np.concatenate([np.geomspace(1e-8, 1e9, 200000), np.linspace(50, 80, 30001)])
    assert np.all(n_g * rate(eps) < nu)


def test_gas_density_hand_value():
    # 20 mTorr at 300 K: 2.66645 Pa / (1.380649e-23 J/K * 300 K) = 6.4377e20 m^-3
    assert ph.gas_density(20.0 * inputs.MTORR, 300.0) == pytest.approx(6.4377e20, rel=2e-5)


def test_ion_bound_hand_value():
    """20 mTorr, 300 K, V0 = 400 V: g_max = 62 165 m/s (an Ar+ ion that fell
    through 2 V0 = 800 V) + 6 x 249.88 m/s (thermal) = 63 664 m/s, so
    nu_max,i = 6.4377e20 m^-3 x 5e-19 m^2 x 63 664 m/s = 2.0492e7 1/s."""
    n_g = ph.gas_density(20.0 * inputs.MTORR, 300.0)
    assert ph.nu_max_ion(n_g, 400.0, 300.0) == pytest.approx(2.0492e7, rel=1e-4)
    assert ph.nu_max_ion(n_g, -400.0, 300.0) == ph.nu_max_ion(n_g, 400.0, 300.0)


def test_ion_bound_is_the_speed_gained_through_twice_the_drive():
    """The first term of g_max is the speed of an Ar+ ion that starts at rest
    and falls through a potential drop of 2 V0 (the peak-to-peak drive): the
    oracle's leapfrog push of one ion across a uniform field of that drop
    reaches the wall with that speed."""
    V0, L, N = 400.0, 0.01, 64
    g = Grid.make(L, N)
    E = np.full(N, 2 * V0 / L)
    dt = 1e-9
    qmdt = (ph.QE / ph.M_AR) * dt
    sp = Species(s=1, prec=FP64, vx=np.zeros(1), vy=np.zeros(1), vz=np.zeros(1),
                 id=np.zeros(1, np.uint64), knext=np.zeros(1, np.int64), x=np.zeros(1))
    for _ in range(100000):
        vx, x, wall = push_fp64(g, sp, E, 0, qmdt, dt)
        if wall[0] != 0:
            break
        sp.vx, sp.x = vx, x
    assert wall[0] == 1
    # leapfrog: the last half-step velocity lies within a*dt of the exact one
    n_g = ph.gas_density(20.0 * inputs.MTORR, 300.0)
    g_th = 6.0 * math.sqrt(ph.KB * 300.0 / ph.M_AR)
    g_fall = ph.nu_max_ion(n_g, V0, 300.0) / (n_g * ph.SIGMA_CX) - g_th
    assert abs(vx[0] - g_fall) < qmdt * E[0] * 1.01


# -- stability monitors (Section 1, Eqs 1a-1c) -------------------------------
def crafted(n_e, cell, v_e, N=100, L=0.01, dt=1e-10, W=1e12):
    """n_e electrons at the centre of `cell` with velocity (v_e, 0, 0), no ions,
    uniform grid, no drive: the deposit and monitors follow by hand."""
    z = np.zeros(n_e)
    x = np.full(n_e, (cell + 0.5) * (L / N))
    sp = Species(s=0, prec=FP64, vx=np.full(n_e, v_e), vy=z.copy(), vz=z.copy(),
                 id=np.arange(n_e, dtype=np.uint64), knext=np.full(n_e, 2 ** 31 - 1, np.int64), x=x)
    cfg = inputs.small_discharge(n_cells=N, gap_m=L, v_rf=0.0, dt_s=dt, n_species=1, collisions=0,
                                 weight_m2=W, n_per_species=n_e, bc=0)
    sim = Sim(cfg, species=[sp])
    sim.deposit()
    sim.solve()
    return sim


def test_density_maximum_hand_value():
    # 10 electrons at a cell centre put half their weight on each of its nodes:
    # n = 10 * 1e12 * 0.5 / 1e-4 m = 5e16 m^-3 at both nodes
    sim = crafted(10, 40, 0.0)
    assert sim.monitors()["ne_max_m3"] == pytest.approx(5e16, rel=1e-14)
    # at the first cell the left node is an electrode node of volume dx/2
    sim = crafted(10, 0, 0.0)
    assert sim.monitors()["ne_max_m3"] == pytest.approx(1e17, rel=1e-14)


def test_plasma_frequency_matches_the_textbook():
    # n = 5e16 m^-3 = 5e10 cm^-3: omega_pe = 5.64e4 * sqrt(5e10) rad/s
    sim = crafted(10, 40, 0.0, dt=2e-11)
    w = 5.64e4 * math.sqrt(5e10)
    assert sim.monitors()["wpe_dt_max"] == pytest.approx(w * 2e-11, rel=1e-3)


def test_debye_length_matches_the_textbook():
    """Electrons of 3 eV each (|v|^2 = 6 eV * 2e/m along x): T_e = 2/3 * 3 = 2 eV;
    lambda_D = 743 sqrt(2 / 5e10) cm at n = 5e16 m^-3."""
    v = math.sqrt(ph.TWO_QE_OVER_ME * 3.0)
    sim = crafted(10, 40, v)
    m = sim.monitors()
    assert m["te_ev"] == pytest.approx(2.0, rel=1e-14)
    lam = 743.0 * math.sqrt(2.0 / 5e10) * 1e-2
    assert m["lambda_de_over_dxmin"] == pytest.approx(lam / 1e-4, rel=1e-3)


def test_courant_monitor_hand_value():
    # fastest electron 2e6 m/s (in either direction), dt = 1e-10 s, dx = 1e-4 m: 2.0
    sim = crafted(3, 10, -2.0e6)
    sim.sp[0].vx[1] = 1.0e6
    assert sim.monitors()["vmax_dt_over_dxmin"] == pytest.approx(2.0, rel=1e-14)


def test_plasma_frequency_monitor_matches_the_measured_oscillation():
    """The monitor's omega_pe dt, formed from the deposit, against the
    frequency the cold plasma actually oscillates at (leapfrog dispersion
    omega = (2/dt) asin(omega_pe dt / 2)): a pin through the dynamics."""
    from test_oracle_loop import cold_plasma, measured_frequency
    wdt = 0.1
    sim, wpe = cold_plasma(wdt, 0)
    N, L, dt = sim.grid.N, sim.L, sim.dt
    basis = np.cos(2 * math.pi * sim.grid.nodes[:N] / L)
    amp, mons = [], []
    for _ in range(int(round(6 * 2 * math.pi / wdt))):
        sim.step()
        amp.append(float(np.sum(sim.Q[:N] * basis)))
        mons.append(sim.monitors()["wpe_dt_max"])
    w = measured_frequency(amp, dt)
    wdt_measured = 2 * math.sin(w * dt / 2)
    # the displaced plasma's densest node is at most a few per cent above n0
    assert min(mons) == pytest.approx(wdt_measured, rel=0.01)
    assert max(mons) < wdt_measured * 1.05


def test_absorbed_energy_is_the_kinetic_energy_brought_to_the_wall():
    """One electron 1 um from the right electrode moving out at 3 eV (with a
    negligible weight, so no field acts): one absorption at the right wall
    carrying exactly 3 eV (the push leaves vx unchanged)."""
    L, N = 0.01, 100
    v = math.sqrt(ph.TWO_QE_OVER_ME * 3.0)
    sp = Species(s=0, prec=FP64, vx=np.array([v]), vy=np.zeros(1), vz=np.zeros(1),
                 id=np.zeros(1, np.uint64), knext=np.full(1, 2 ** 31 - 1, np.int64),
                 x=np.array([L - 1e-6]))
    cfg = inputs.small_discharge(n_cells=N, gap_m=L, v_rf=0.0, dt_s=1e-10, n_species=1,
                                 collisions=0, weight_m2=1e-30, n_per_species=1)
    sim = Sim(cfg, species=[sp])
    sim.step()
    assert sim.absorbed[0].tolist() == [0, 1]
    assert sim.absorbed_energy_ev[0, 1] == pytest.approx(3.0, rel=1e-12)
    assert sim.absorbed_energy_ev[0, 0] == 0.0
    assert len(sim.last_absorbed) == 1 and sim.last_absorbed[0][:2] == (0, 1)
