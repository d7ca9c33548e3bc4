"""Pins of the oracle's impact distributions (energy and angle at the walls of
absorbed particles, the ion-impact data of Section 3a)."""
import math

import numpy as np
import pytest

import inputs
from oracle import physics as ph
from oracle.pic import FP64, Species
from oracle.sim import Sim, impact_bins


def beam(E_ev, theta_deg, n=5, x0=1e-6):
    """n electrons just inside x = 0 moving into the left wall with kinetic
    energy E_ev at angle theta_deg to the wall normal."""
    v = math.sqrt(2.0 * E_ev * ph.QE / ph.ME)
    th = math.radians(theta_deg)
    z = np.zeros(n)
    return Species(s=0, prec=FP64, x=np.full(n, x0), vx=np.full(n, -v * math.cos(th)),
                   vy=np.full(n, v * math.sin(th)), vz=z.copy(), id=np.arange(n, dtype=np.uint64),
                   knext=np.full(n, 2 ** 31 - 1, np.int64))


@pytest.mark.parametrize("E_ev,theta,nb,na,emax", [(123.4, 30.5, 200, 90, 1000.0),
                                                   (7.9, 71.2, 50, 18, 20.0),
                                                   (45.0, 3.3, 100, 45, 40.0)])
def test_beam_lands_in_its_bins(E_ev, theta, nb, na, emax):
    cfg = inputs.small_discharge(v_rf=0.0, collisions=0, n_species=1, bc=0, weight_m2=1e-9,
                                 avg_every=1, impact_bins=nb, impact_angle_bins=na, impact_emax_ev=emax)
    sp = beam(E_ev, theta)
    sim = Sim(cfg, species=[sp])
    sim.step()
    assert sim.absorbed[0, 0] == sp.n
    e = sim.impact_e[0, 0]
    a = sim.impact_a[0, 0]
    eb = int(E_ev * nb / emax) if E_ev < emax else nb
    ab = int(theta * na / 90.0)
    assert e[eb] == sp.n and e.sum() == sp.n
    assert a[ab] == sp.n and a.sum() == sp.n
    assert sim.impact_e[0, 1].sum() == 0


def test_energy_overflow_and_grazing_angle():
    be, ba = impact_bins(np.array([999.9, 1000.0, 5e4]), np.array([1.0, 0.0, 1e-300]),
                         np.array([1.0, 1.0, 1.0]), 200, 90, 1000.0)
    assert list(be) == [199, 200, 200]
    assert list(ba) == [0, 89, 89]           # theta = 90 degrees goes to the last bin


def test_vectorised_bins_match_a_scalar_loop():
    g = np.random.default_rng(4)
    en = g.exponential(60.0, 2000)
    vx = g.normal(0.0, 1e5, 2000)
    v2 = vx * vx + g.normal(0.0, 1e5, 2000) ** 2
    be, ba = impact_bins(en, vx, v2, 120, 30, 300.0)
    for i in range(0, 2000, 7):
        f = math.floor(en[i] * (120 / 300.0))
        assert be[i] == (f if f < 120 else 120)
        c = min(1.0, abs(vx[i]) / math.sqrt(v2[i]))
        assert ba[i] == min(math.floor(math.acos(c) * (180.0 / math.pi) * (30 / 90.0)), 29)


@pytest.mark.slow
def test_histogram_totals_equal_absorbed_counts():
    n_g = ph.gas_density(50 * inputs.MTORR, 300.0)
    cfg = inputs.small_discharge(n_per_species=3000, avg_every=1, gamma_see=0.2,
                                 nu_max_e=ph.nu_max_electron(n_g), nu_max_i=ph.nu_max_ion(n_g, 200.0, 300.0))
    sim = Sim(cfg)
    sim.run(150)
    for s in range(2):
        for w in range(2):
            assert sim.impact_e[s, w].sum() == sim.absorbed[s, w]
            assert sim.impact_a[s, w].sum() == sim.absorbed[s, w]
    assert sim.absorbed[0].sum() > 0
