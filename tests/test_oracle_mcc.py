"""Pins of the oracle's null-collision Monte Carlo step (argon, analytic cross sections)."""
import math

import numpy as np
import pytest

import inputs
from oracle import physics as ph
from oracle.pic import (INT32_MAX, MccCounts, collide_electrons, collide_ions, emit_secondaries,
                        Grid, FP64, init_species, next_candidate)
from oracle.sim import Sim

NG = ph.gas_density(50 * inputs.MTORR, 300.0)


def test_candidate_counts_are_binomial():
    """Waiting-time candidates: each step a particle is a candidate with
    probability P = 1 - exp(-nu_max dt), independently of its history."""
    n, nudt = 20000, 0.05
    P = 1 - math.exp(-nudt)
    ids = inputs.unique_ids(n, seed=1)
    kn = next_candidate(ids, -1, 0, 77, nudt)     # first candidate step >= 0
    counts = []
    for k in range(200):
        c = kn == k
        counts.append(int(c.sum()))
        kn[c] = next_candidate(ids[c], k, 0, 77, nudt)
    counts = np.array(counts)
    assert abs(counts.mean() - n * P) < 5 * math.sqrt(n * P * (1 - P) / len(counts))
    assert abs(counts.var() / (n * P * (1 - P)) - 1) < 0.35
    assert np.all(kn >= 200)


def test_collisions_off_never_candidate():
    ids = inputs.unique_ids(10, seed=2)
    assert np.all(next_candidate(ids, 5, 0, 1, 0.0) == INT32_MAX)


def mono(eps_ev, n, seed):
    g = inputs.rng(seed)
    d = g.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0)
    s = math.sqrt(ph.TWO_QE_OVER_ME * eps_ev)
    return s * d[0], s * d[1], s * d[2]


@pytest.mark.parametrize("eps", [5.0, 30.0, 80.0])
def test_process_selection_frequencies(eps):
    n = 60000
    vx, vy, vz = mono(eps, n, seed=3)
    nu_max = ph.nu_max_electron(NG)
    cnt = MccCounts()
    ids = inputs.unique_ids(n, seed=4)
    collide_electrons(vx, vy, vz, ids, 10, 5, NG, nu_max, cnt)
    v = math.sqrt(ph.TWO_QE_OVER_ME * eps)
    p = np.array([float(NG * ph.sigma_el(eps) * v), float(NG * ph.sigma_ex(np.array([eps]))[0] * v),
                  float(NG * ph.sigma_iz(np.array([eps]))[0] * v)]) / nu_max
    got = np.array([cnt.elastic, cnt.excitation, cnt.ionisation])
    for k in range(3):
        sd = math.sqrt(n * p[k] * (1 - p[k])) + 1
        assert abs(got[k] - n * p[k]) < 5 * sd
    assert cnt.bound_violations == 0


def energy(vx, vy, vz):
    return ph.HALF_ME_OVER_QE * ((vx * vx + vy * vy) + vz * vz)


def test_energy_bookkeeping_and_isotropy():
    n = 100000
    eps0 = 60.0
    vx, vy, vz = mono(eps0, n, seed=6)
    ids = inputs.unique_ids(n, seed=7)
    nu_max = ph.nu_max_electron(NG)
    cnt = MccCounts()
    nvx, nvy, nvz, iz, ej = collide_electrons(vx, vy, vz, ids, 3, 11, NG, nu_max, cnt)
    e1 = energy(nvx, nvy, nvz)
    changed = (nvx != vx) | (nvy != vy) | (nvz != vz)
    lost = eps0 - e1
    # Excitation loses 11.5 eV; ionisation 15.76 eV shared equally with the ejected electron.
    exc = np.isclose(lost, ph.E_EXC, rtol=1e-9)
    assert exc.sum() == cnt.excitation
    e_ej = energy(*ej)
    assert np.allclose(e1[iz] + e_ej, eps0 - ph.E_ION, rtol=1e-9)
    assert np.allclose(e1[iz], e_ej, rtol=1e-9)
    # Elastic: the loss matches (2 m/M)(1 - cos chi) measured from the two directions.
    el = changed & ~exc & ~iz
    assert el.sum() == cnt.elastic
    cos_chi = (vx[el] * nvx[el] + vy[el] * nvy[el] + vz[el] * nvz[el]) / (
        np.sqrt(energy(vx[el], vy[el], vz[el]) * e1[el]) / ph.HALF_ME_OVER_QE)
    assert np.allclose(lost[el] / eps0, ph.TWO_ME_OVER_M * (1 - cos_chi), rtol=1e-6, atol=1e-12)
    frac = lost[el] / eps0
    assert abs(frac.mean() / ph.TWO_ME_OVER_M - 1) < 0.05
    # New directions are isotropic: <cos> = 0, <cos^2> = 1/3 for each axis.
    d = np.stack([nvx[changed], nvy[changed], nvz[changed]])
    d /= np.linalg.norm(d, axis=0)
    m = d.shape[1]
    for ax in range(3):
        assert abs(d[ax].mean()) < 5 / math.sqrt(3 * m)
        assert abs((d[ax] ** 2).mean() - 1 / 3) < 0.01


def test_charge_exchange_relaxes_to_gas_maxwellian():
    n = 40000
    g = inputs.rng(8)
    vti_hot = math.sqrt(ph.QE * 1.0 / ph.M_AR)      # 1 eV ions
    vx, vy, vz = (g.normal(0, vti_hot, n) for _ in range(3))
    vx = vx + 3 * vti_hot
    vti = math.sqrt(ph.KB * 300.0 / ph.M_AR)
    nu_max = NG * ph.SIGMA_CX * 12 * vti_hot
    ids = inputs.unique_ids(n, seed=9)
    cnt = MccCounts()
    for k in range(400):
        vx, vy, vz = collide_ions(vx, vy, vz, ids, k, 3, NG, nu_max, vti, cnt)
    assert cnt.bound_violations == 0
    for v in (vx, vy, vz):
        assert abs(v.mean()) < 5 * vti / math.sqrt(n)
        assert abs(v.var() / vti ** 2 - 1) < 0.05


def test_secondary_emission():
    L = 0.025
    g = Grid.make(L, 64)
    n = 50000
    ids = inputs.unique_ids(n, seed=10)
    walls = np.where(np.arange(n) % 2 == 0, -1, 1)
    dt = 1e-10
    sp = emit_secondaries(g, ids, walls, 7, 99, 0.1, 2.0, dt, FP64, 0.01)
    frac = sp.n / n
    assert abs(frac - 0.1) < 5 * math.sqrt(0.1 * 0.9 / n)
    vt = math.sqrt(2.0 * ph.QE / ph.ME)
    left = sp.x < L / 2
    assert np.all(sp.vx[left] > 0) and np.all(sp.vx[~left] < 0)
    # |vx| is Rayleigh(v_t): mean v_t sqrt(pi/2); vy, vz Maxwellian.
    assert abs(np.abs(sp.vx).mean() / (vt * math.sqrt(math.pi / 2)) - 1) < 0.03
    assert abs(sp.vy.var() / vt ** 2 - 1) < 0.06
    assert np.all(sp.x[left] <= np.abs(sp.vx[left]) * dt)
    assert np.all(L - sp.x[~left] <= np.abs(sp.vx[~left]) * dt * (1 + 1e-12))
    assert np.all(sp.knext >= 8)
    assert len(np.unique(sp.id)) == sp.n


def test_initial_load_statistics():
    L, N, n = 0.025, 128, 200000
    g = Grid.make(L, N)
    sp = init_species(g, 0, n, 2.0, ph.ME, 5, FP64, 0.02)
    assert np.all((sp.x >= 0) & (sp.x < L))
    hist, _ = np.histogram(sp.x, bins=50, range=(0, L))
    chi2 = float(np.sum((hist - n / 50) ** 2 / (n / 50)))
    assert chi2 < 49 + 6 * math.sqrt(98)
    vt = math.sqrt(2.0 * ph.QE / ph.ME)
    for v in (sp.vx, sp.vy, sp.vz):
        assert abs(v.var() / vt ** 2 - 1) < 0.02
    # First candidate step: floor(Exp / nudt), mean ~ 1/nudt - 1/2.
    assert abs(sp.knext.mean() - (1 / 0.02 - 0.5)) < 5 * (1 / 0.02) / math.sqrt(n)


def test_ionisation_creates_one_pair_and_counts_balance():
    cfg = inputs.small_discharge(n_per_species=3000, v_rf=400.0, gamma_see=0.3, seed=4)
    sim = Sim(cfg)
    for _ in range(60):
        ne, ni = sim.sp[0].n, sim.sp[1].n
        a0 = sim.absorbed.copy()
        see0, cr0, iz0 = sim.see_emitted, sim.created, sim.mcc[0].ionisation
        sim.step()
        dabs = sim.absorbed - a0
        dsee, dcr = sim.see_emitted - see0, sim.created - cr0
        assert dcr == sim.mcc[0].ionisation - iz0
        assert sim.sp[0].n == ne - dabs[0].sum() + dsee + dcr
        assert sim.sp[1].n == ni - dabs[1].sum() + dcr
        for sp in sim.sp:
            assert int(sim.A[sp.s].sum()) >= 0
        total = [int(a.sum()) for a in sim.deposit()]
        assert total == [sim.sp[0].n * 2 ** 32, sim.sp[1].n * 2 ** 32]
    assert sim.created > 0 and sim.see_emitted > 0
    allids = np.concatenate([sim.sp[0].id, sim.sp[1].id])
    assert len(np.unique(sim.sp[0].id)) == sim.sp[0].n
    assert len(np.unique(sim.sp[1].id)) == sim.sp[1].n
    assert allids.size > 0
