"""Pins of the oracle's averaged velocity moments and power (Section 3a)."""
import math

import numpy as np
import pytest

import inputs
from oracle import physics as ph
from oracle.pic import FP64, Species
from oracle.sim import Sim


def sp_at(s, x, vx, vy=None):
    n = len(x)
    z = np.zeros(n)
    return Species(s=s, prec=FP64, x=np.asarray(x, float), vx=np.asarray(vx, float),
                   vy=z.copy() if vy is None else np.asarray(vy, float), vz=z.copy(),
                   id=np.arange(n, dtype=np.uint64) + 1000 * s, knext=np.full(n, 2 ** 31 - 1, np.int64))


def test_two_particles_on_a_node_give_their_mean_and_spread():
    u, a = 2.0e5, 3.0e5
    cfg = inputs.small_discharge(n_cells=8, gap_m=8.0, bc=1, n_species=1, v_rf=0.0, collisions=0,
                                 weight_m2=1e-9, avg_every=1, moments=1)
    sim = Sim(cfg, species=[sp_at(0, [3.0, 3.0], [u - a, u + a])])
    sim.step()
    m = sim.moments(0)
    assert m["ux"][3] == pytest.approx(u, rel=1e-15)
    assert m["tx"][3] == pytest.approx(ph.ME / ph.QE * a * a, rel=1e-12)
    others = [n for n in range(9) if n != 3]
    assert np.all(m["ux"][others] == 0.0) and np.all(m["tx"][others] == 0.0)


def test_power_in_a_uniform_field():
    """Drive at its peak (phase pi/2) and negligible charge: E = V/L in every
    cell; the power density of one particle in cell j is q W vx E / h."""
    V, L, N = 100.0, 0.08, 16
    W = 1e-3
    cfg = inputs.small_discharge(n_cells=N, gap_m=L, v_rf=V, phase=math.pi / 2, collisions=0,
                                 weight_m2=W, avg_every=1, moments=1)
    ve, vi = 3.0e5, -2.0e3
    sim = Sim(cfg, species=[sp_at(0, [0.0123], [ve]), sp_at(1, [0.0567], [vi])])
    sim.step()
    E0 = V / L   # phi falls from V at x = 0 to 0 at x = L
    h = L / N
    pe = sim.moments(0)["power"]
    pi_ = sim.moments(1)["power"]
    je, ji = int(0.0123 / h), int(0.0567 / h)
    assert pe[je] == pytest.approx(-ph.QE * W * ve * E0 / h, rel=1e-9)
    assert pi_[ji] == pytest.approx(ph.QE * W * vi * E0 / h, rel=1e-9)
    assert np.count_nonzero(pe) == 1 and np.count_nonzero(pi_) == 1


@pytest.mark.slow
def test_drifting_maxwellian():
    g = np.random.default_rng(3)
    n, L, N = 200_000, 0.02, 16
    u, T = 4.0e4, 3.0
    sig = math.sqrt(T * ph.QE / ph.ME)
    x = g.uniform(0.0, L, n)
    vx = u + sig * g.standard_normal(n)
    cfg = inputs.small_discharge(n_cells=N, gap_m=L, bc=1, n_species=1, v_rf=0.0, collisions=0,
                                 n0_m3=1e6, avg_every=1, moments=1)
    sim = Sim(cfg, species=[sp_at(0, x, vx)])
    sim.step()
    m = sim.moments(0)
    per_node = n / N
    assert np.all(np.abs(m["ux"] - u) < 5 * sig / math.sqrt(per_node))
    assert np.all(np.abs(m["tx"] / T - 1.0) < 5 * math.sqrt(2.0 / per_node))
