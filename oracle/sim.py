"""The oracle's time loop: one discharge advanced step by step in FP64.

Test infrastructure only (see ``oracle/__init__.py``).

``Sim.step`` follows the loop of Section 2a in its order: deposit x^k (Eqs
2-3), solve Poisson at t_k (Eq 4), form the field (Eq 5, or the centred MC
field), gather and push (Eqs 6-9) with absorption at the electrodes and
secondary emission, then collide with the gas and advance k.  The RF-averaged
moments of Section 3a (density and potential every ``avg_every`` steps, the
central EEDF every ``eedf_every`` steps) accumulate along the way.

Configuration keys mirror the C ``pic_config`` structure; enumerations use the
same integers (bc 0 Dirichlet-RF / 1 periodic, gather 0 EC / 1 MC, precision
0 FP64 / 1 FP32-state).
"""
from __future__ import annotations

import math

import numpy as np

from . import physics as ph
from .pic import (BC_PERIODIC, FP64, GATHER_EC, GATHER_EC2, TAG_CHILD, TWO_M32, Grid, MccCounts,
                  Species, collide_electrons, collide_ions, deposit_species, draw, emit_secondaries,
                  field_ec, field_ec2, field_mc, fold_s2, gas_velocity, gather_fp32, gather_fp64,
                  ids_from_words, init_species, locate, next_candidate, node_charge, poisson,
                  push_fp32, push_fp64, s2_gather_index, weight_shift)

DEFAULTS = dict(
    n_cells=128, bc=0, nodes=None, gap_m=0.025, v_rf=200.0, f_rf=13.56e6, phase=0.0,
    p_pa=50.0 * 133.322368 / 1000.0, t_gas_k=300.0, n0_m3=1e15, te_ev=2.0, ti_ev=0.026,
    n_per_species=12800, weight_m2=0.0, dt_s=1.0 / (400 * 13.56e6), gather=0, precision=0,
    gamma_see=0.0, t_see_ev=2.0, seed=1, n_species=2, collisions=1, pullback=0,
    nu_max_e=0.0, nu_max_i=0.0, avg_start=0, avg_every=0, eedf_every=0, eedf_bins=200,
    eedf_emax_ev=50.0, eedf_width_m=1e-3, impact_bins=0, impact_angle_bins=0, impact_emax_ev=0.0,
    moments=0, rebalance_ppc=0, rebalance_dv_e=0.0, rebalance_dv_i=0.0,
)


def impact_bins(en, vx, v2, nb, na, emax):
    """Histogram bins of absorbed particles (the ion-impact energy and angle
    data of Section 3a): energy E in eV binned as floor(E * nb / emax) with one
    overflow bin nb; angle to the wall normal theta = acos(|vx| / |v|) in
    degrees, binned as floor(theta * na / 90), theta = 90 in the last bin."""
    fe = np.floor(en * (nb / emax))
    be = np.where(fe < nb, fe, nb).astype(np.int64)
    cth = np.ones_like(v2)
    pos = v2 > 0.0
    cth[pos] = np.minimum(1.0, np.abs(vx[pos]) / np.sqrt(v2[pos]))
    th = np.arccos(cth) * (180.0 / math.pi)
    ba = np.minimum(np.floor(th * (na / 90.0)).astype(np.int64), na - 1)
    return be, ba


def resolve(cfg):
    c = dict(DEFAULTS)
    c.update(cfg or {})
    return c


class Sim:
    def __init__(self, cfg, species=None, k=0):
        """``species``: optional list of ``Species`` to start from (else the
        seeded Maxwellian load); ``k``: the step index of that state."""
        c = resolve(cfg)
        self.cfg = c
        self.grid = Grid.make(c["gap_m"], int(c["n_cells"]), c["nodes"], int(c["bc"]))
        g = self.grid
        self.L = g.L
        self.dt = float(c["dt_s"])
        self.prec = int(c["precision"])
        self.gather = int(c["gather"])
        if self.gather == GATHER_EC2 and not g.uniform:
            raise ValueError("second-order EC needs a uniform grid")
        self.nsp = int(c["n_species"])
        W = float(c["weight_m2"])
        if W == 0.0:
            W = c["n0_m3"] * g.L / c["n_per_species"]
        self.W = W
        # With rebalancing, weights are W 2^(c-4) for classes c = 0..7 and
        # deposits and weighted sums are kept in units of W 2^-4.
        self.u = 4 if int(c["rebalance_ppc"]) > 0 else 0
        self.W_unit = W * 2.0 ** -self.u
        self.n_g = ph.gas_density(c["p_pa"], c["t_gas_k"])
        nu_e = float(c["nu_max_e"]) or ph.nu_max_electron(self.n_g)
        nu_i = float(c["nu_max_i"]) or ph.nu_max_ion(self.n_g, c["v_rf"], c["t_gas_k"])
        self.nu_max = [nu_e, nu_i]
        on = bool(c["collisions"])
        self.nudt = [nu_e * self.dt if on else 0.0, nu_i * self.dt if on else 0.0]
        self.q = [ph.SPECIES[s][0] for s in range(2)]
        self.m = [ph.SPECIES[s][1] for s in range(2)]
        self.qmdt = [(self.q[s] / self.m[s]) * self.dt for s in range(2)]
        self.qW = [self.q[s] * self.W_unit for s in range(2)]
        self.vti = math.sqrt(ph.KB * c["t_gas_k"] / ph.M_AR)
        self.seed = int(c["seed"])
        if self.prec != FP64:
            self.qmdt32 = [np.float32(v) for v in self.qmdt]
            self.tables = g.walk_tables(self.dt)
        self.k = int(k)
        N = g.N
        self.acc_A = [np.zeros(N + 1) for _ in range(2)]
        self.acc_phi = np.zeros(N + 1)
        # velocity moments (nodes) and power (cells) of the averaged steps
        self.acc_m1 = [np.zeros(N + 1) for _ in range(2)]
        self.acc_m2 = [np.zeros(N + 1) for _ in range(2)]
        self.acc_p = [np.zeros(N) for _ in range(2)]
        self.n_samples = 0
        self.eedf = np.zeros(int(c["eedf_bins"]), dtype=np.int64)
        self.eedf_samples = 0
        self.absorbed = np.zeros((2, 2), dtype=np.int64)      # [species][wall: 0 left, 1 right]
        self.absorbed_energy_ev = np.zeros((2, 2))
        # the particles absorbed in the last step: (species, wall, energy eV, vx, |v|^2)
        self.last_absorbed = []
        # impact distributions [species][wall]: energy (bins + overflow), angle
        self.imp_nb = int(c["impact_bins"] or 200)
        self.imp_na = int(c["impact_angle_bins"] or 90)
        self.imp_emax = float(c["impact_emax_ev"] or 1000.0)
        self.impact_e = np.zeros((2, 2, self.imp_nb + 1), dtype=np.int64)
        self.impact_a = np.zeros((2, 2, self.imp_na), dtype=np.int64)
        self.see_emitted = 0
        self.created = 0
        self.mcc = [MccCounts(), MccCounts()]
        self.field_energy = 0.0
        self.phi = None
        self.E = None
        self.Q = None
        self.A = None
        if species is None:
            T = [c["te_ev"], c["ti_ev"]]
            self.sp = [init_species(g, s, int(c["n_per_species"]), T[s], self.m[s], self.seed,
                                    self.prec, self.nudt[s]) for s in range(self.nsp)]
            if c["pullback"]:
                self._pullback()
        else:
            self.sp = list(species)

    # -- deposit, field solve, field ----------------------------------------
    def deposit(self):
        self.A = [deposit_species(self.grid, sp, self.gather, self.u) for sp in self.sp]
        return self.A

    def solve(self):
        c = self.cfg
        self.Q = node_charge(self.A, self.qW[:self.nsp])
        t = self.k * self.dt
        self.phi = poisson(self.grid, self.Q, t, c["v_rf"], c["f_rf"], c["phase"])
        self.E_cell = field_ec(self.grid, self.phi)
        if self.gather == GATHER_EC:
            self.E = self.E_cell
        elif self.gather == GATHER_EC2:
            self.E = field_ec2(self.grid, self.phi)
        else:
            self.E = field_mc(self.grid, self.phi, self.Q)
        self.field_energy = 0.5 * ph.EPS0 * float(np.sum(self.grid.h * self.E_cell * self.E_cell))
        if self.prec != FP64:
            self.E32 = self.E.astype(np.float32)
        return self.phi

    def _pullback(self):
        """v^{-1/2} = v^0 - (q/m) E^0 dt / 2 (switch; off by default)."""
        self.deposit()
        self.solve()
        for sp in self.sp:
            hq = 0.5 * self.qmdt[sp.s]
            if self.prec == FP64:
                e = gather_fp64(self.grid, sp.x, self.E, self.gather)
                sp.vx = sp.vx - hq * e
            else:
                e = gather_fp32(sp.cell, sp.off, self.E32, self.gather)
                sp.vx = sp.vx - np.float32(hq) * e

    def _accumulate(self):
        c = self.cfg
        k = self.k
        if c["avg_every"] > 0 and k >= c["avg_start"] and (k - c["avg_start"]) % c["avg_every"] == 0:
            for s in range(self.nsp):
                self.acc_A[s] += self.A[s].astype(np.float64)
                if c["moments"]:
                    self._accumulate_moments(s)
            self.acc_phi += self.phi
            self.n_samples += 1

    def _accumulate_moments(self, s):
        """Section 3a moments from x^k, v^{k-1/2} and E^k: sum w vx and
        sum w vx^2 at the nodes with the deposit's shape (linear weights
        w = 1 - xi, xi; for second-order EC the quadratic spline, in FP64),
        and per cell sum vx E(x) with the gathered field."""
        sp = self.sp[s]
        if sp.n == 0:
            return
        if self.prec == FP64:
            j, xi = locate(self.grid, sp.x)
        else:
            j = sp.cell.astype(np.int64)
            xi = sp.off.astype(np.float64)
        vx = sp.vx.astype(np.float64)
        f = np.ldexp(1.0, weight_shift(sp, self.u))     # the particle's weight in units W 2^-u
        E = self.E
        if self.gather == GATHER_EC2:
            up = xi >= 0.5
            n = j + up.astype(np.int64)
            a = np.where(up, 1.5 - xi, 0.5 - xi)
            b = np.where(up, xi - 0.5, 0.5 + xi)
            wl = 0.5 * (a * a)
            wr = 0.5 * (b * b)
            wc = 1.0 - wl - wr
            for idx, w in ((fold_s2(self.grid, n - 1), wl), (n, wc), (fold_s2(self.grid, n + 1), wr)):
                np.add.at(self.acc_m1[s], idx, (f * w) * vx)
                np.add.at(self.acc_m2[s], idx, (f * w) * (vx * vx))
            m, t = s2_gather_index(j, xi)
            e = (1.0 - t) * E[m] + t * E[m + 1]
        else:
            w0, w1 = 1.0 - xi, xi
            np.add.at(self.acc_m1[s], j, (f * w0) * vx)
            np.add.at(self.acc_m1[s], j + 1, (f * w1) * vx)
            np.add.at(self.acc_m2[s], j, (f * w0) * (vx * vx))
            np.add.at(self.acc_m2[s], j + 1, (f * w1) * (vx * vx))
            e = E[j] if self.gather == GATHER_EC else (1.0 - xi) * E[j] + xi * E[j + 1]
        np.add.at(self.acc_p[s], j, f * (vx * e))

    def moments(self, s):
        """Mean x-velocity (m/s) and x-temperature (eV) at the nodes, power
        density (W/m^3) per cell: ratios of the averaged sums."""
        g = self.grid
        N = g.N
        m1 = self.acc_m1[s].copy()
        m2 = self.acc_m2[s].copy()
        if g.bc == BC_PERIODIC:          # node N is node 0
            m1[0] += m1[N]
            m1[N] = m1[0]
            m2[0] += m2[N]
            m2[N] = m2[0]
        w = self.acc_A[s] * TWO_M32
        ok = w > 0
        ux = np.zeros(N + 1)
        tx = np.zeros(N + 1)
        ux[ok] = m1[ok] / w[ok]
        tx[ok] = (self.m[s] / ph.QE) * (m2[ok] / w[ok] - ux[ok] * ux[ok])
        power = (self.qW[s] * self.acc_p[s]) / (g.h * max(self.n_samples, 1))
        return dict(ux=ux, tx=tx, power=power)

    def _eedf_due(self):
        c = self.cfg
        k = self.k
        return c["eedf_every"] > 0 and k >= c["avg_start"] and (k - c["avg_start"]) % c["eedf_every"] == 0

    def _sample_eedf(self, x, vx, vy, vz, sh):
        """Central EEDF sample; a particle counts its weight in units W 2^-u
        (2^sh; 1 without rebalancing)."""
        c = self.cfg
        centre = 0.5 * self.L
        half = 0.5 * c["eedf_width_m"]
        m = np.abs(x - centre) < half
        v2 = (vx[m] * vx[m] + vy[m] * vy[m]) + vz[m] * vz[m]
        eps = ph.HALF_ME_OVER_QE * v2
        de = c["eedf_emax_ev"] / c["eedf_bins"]
        b = np.floor(eps / de)
        keep = b < c["eedf_bins"]
        np.add.at(self.eedf, b[keep].astype(np.int64), np.int64(1) << sh[m][keep])
        self.eedf_samples += 1

    # -- one full step ------------------------------------------------------
    def step(self):
        c = self.cfg
        g = self.grid
        k = self.k
        self.deposit()
        self.solve()
        self._accumulate()
        eedf_due = self._eedf_due()

        survivors = []
        see_new = None
        self.last_absorbed = []
        for sp in self.sp:
            s = sp.s
            if self.prec == FP64:
                vx, x, wall = push_fp64(g, sp, self.E, self.gather, self.qmdt[s], self.dt)
                moved = Species(s=s, prec=FP64, vx=vx, vy=sp.vy, vz=sp.vz, id=sp.id,
                                knext=sp.knext, x=x, wc=sp.wc)
            else:
                vx, cell, off, wall = push_fp32(g, sp, self.E32, self.gather, self.qmdt32[s],
                                                self.tables)
                moved = Species(s=s, prec=sp.prec, vx=vx, vy=sp.vy, vz=sp.vz, id=sp.id,
                                knext=sp.knext, cell=cell, off=off, wc=sp.wc)
            gone = wall != 0
            sh = weight_shift(moved, self.u)
            if gone.any():
                for wi, wv in ((0, -1), (1, 1)):
                    mw = wall == wv
                    self.absorbed[s, wi] += int(mw.sum())
                    vxa = moved.vx[mw].astype(np.float64)
                    vya = moved.vy[mw].astype(np.float64)
                    vza = moved.vz[mw].astype(np.float64)
                    v2 = (vxa * vxa + vya * vya) + vza * vza
                    en = (0.5 * self.m[s] / ph.QE) * v2
                    # energies and histogram counts carry the particle's weight
                    # (units W 2^-u)
                    fw = np.ldexp(1.0, sh[mw])
                    self.absorbed_energy_ev[s, wi] += float(np.sum(fw * en))
                    if len(en):
                        self.last_absorbed.append((s, wi, en, vxa, v2))
                    if c["avg_every"] > 0 and k >= c["avg_start"] and len(en):
                        be, ba = impact_bins(en, vxa, v2, self.imp_nb, self.imp_na, self.imp_emax)
                        np.add.at(self.impact_e[s, wi], be, np.int64(1) << sh[mw])
                        np.add.at(self.impact_a[s, wi], ba, np.int64(1) << sh[mw])
                if s == 1 and self.nsp > 1:
                    see_new = emit_secondaries(g, moved.id[gone], wall[gone], k, self.seed,
                                               c["gamma_see"], c["t_see_ev"], self.dt, self.prec,
                                               self.nudt[0],
                                               ion_wc=None if moved.wc is None else moved.wc[gone])
                    if see_new is not None:
                        self.see_emitted += see_new.n
            live = moved.subset(~gone)
            if s == 0 and eedf_due:
                if self.prec == FP64:
                    xs = live.x
                else:
                    xs = g.position(live.cell, live.off)
                self._sample_eedf(xs, live.vx.astype(np.float64), live.vy.astype(np.float64),
                                  live.vz.astype(np.float64), weight_shift(live, self.u))
            survivors.append(live)

        new_e, new_i = [], []
        for idx, sp in enumerate(survivors):
            s = sp.s
            if self.nudt[s] <= 0.0:
                continue
            cand = sp.knext <= k
            if not cand.any():
                continue
            ci = np.nonzero(cand)[0]
            ids = sp.id[ci]
            vx = sp.vx[ci].astype(np.float64)
            vy = sp.vy[ci].astype(np.float64)
            vz = sp.vz[ci].astype(np.float64)
            if s == 0:
                nvx, nvy, nvz, iz, ej = collide_electrons(vx, vy, vz, ids, k, self.seed, self.n_g,
                                                          self.nu_max[0], self.mcc[0])
                if iz.any() and self.nsp > 1:
                    pid = ids[iz]
                    c0, c1, c2, c3 = draw(pid, k, TAG_CHILD, 0, self.seed)
                    eid = ids_from_words(c0, c1)
                    iid = ids_from_words(c2, c3)
                    gx, gy, gz = gas_velocity(pid, k, 0, self.seed, self.vti)
                    pos = {}
                    if self.prec == FP64:
                        pos["x"] = sp.x[ci][iz]
                    else:
                        pos["cell"] = sp.cell[ci][iz]
                        pos["off"] = sp.off[ci][iz]
                    cast = (lambda a: a) if self.prec == FP64 else (lambda a: a.astype(np.float32))
                    if sp.wc is not None:     # the pair carries the primary's weight
                        pos["wc"] = sp.wc[ci][iz]
                    new_e.append(Species(s=0, prec=self.prec, vx=cast(ej[0]), vy=cast(ej[1]),
                                         vz=cast(ej[2]), id=eid,
                                         knext=next_candidate(eid, k, 0, self.seed, self.nudt[0]),
                                         **{kk: v.copy() for kk, v in pos.items()}))
                    new_i.append(Species(s=1, prec=self.prec, vx=cast(gx), vy=cast(gy),
                                         vz=cast(gz), id=iid,
                                         knext=next_candidate(iid, k, 1, self.seed, self.nudt[1]),
                                         **{kk: v.copy() for kk, v in pos.items()}))
                    self.created += int(iz.sum())
            else:
                nvx, nvy, nvz = collide_ions(vx, vy, vz, ids, k, self.seed, self.n_g,
                                             self.nu_max[1], self.vti, self.mcc[1])
            if self.prec == FP64:
                sp.vx[ci], sp.vy[ci], sp.vz[ci] = nvx, nvy, nvz
            else:
                sp.vx[ci] = nvx.astype(np.float32)
                sp.vy[ci] = nvy.astype(np.float32)
                sp.vz[ci] = nvz.astype(np.float32)
            sp.knext[ci] = next_candidate(ids, k, s, self.seed, self.nudt[s])

        if see_new is not None:
            survivors[0] = survivors[0].append(see_new)
        for ne in new_e:
            survivors[0] = survivors[0].append(ne)
        for ni in new_i:
            survivors[1] = survivors[1].append(ni)
        self.sp = survivors
        self.k = k + 1

    def run(self, n):
        for _ in range(n):
            self.step()

    # -- diagnostics ----------------------------------------------------------
    def kinetic_energy(self, s):
        """sum_i W_i (m/2) |v_i|^2 per unit area (J/m^2), W_i the particle's weight."""
        sp = self.sp[s]
        vx = sp.vx.astype(np.float64)
        vy = sp.vy.astype(np.float64)
        vz = sp.vz.astype(np.float64)
        f = np.ldexp(1.0, weight_shift(sp, self.u))
        return self.W_unit * (0.5 * self.m[s]) * float(np.sum(f * ((vx * vx + vy * vy) + vz * vz)))

    def monitors(self):
        """The three stability conditions of Section 1 (Eqs 1a-1c), in the
        form Section 3a quotes them for a steady state:

        * ne_max: the largest electron density over the nodes of the last
          solve, n_e,n = W A_e,n 2^-32 / V_n (the deposit of x^k);
        * wpe_dt_max = omega_pe,max dt with omega_pe^2 = n_e,max e^2 / (eps0 m_e)
          (condition 1b);
        * vmax_dt_over_dxmin = max |vx| dt / min h over the electrons of the
          current state (condition 1c; the fastest particle against the
          smallest cell);
        * lambda_de_over_dxmin = lambda_De,min / min h with
          lambda_De,min = sqrt(eps0 T_e / (n_e,max e)), T_e (in volts) taken as
          2/3 of the electrons' mean kinetic energy in eV (condition 1a; a
          reading: the paper does not say which temperature it uses).
        """
        g = self.grid
        A_e = np.asarray(self.A[0], dtype=np.float64)
        ne = ((A_e * self.W_unit) * TWO_M32) / g.V
        ne_max = float(ne.max())
        wpe = math.sqrt(ne_max * ph.QE * ph.QE / (ph.EPS0 * ph.ME))
        sp = self.sp[0]
        hmin = float(np.min(g.h))
        vmax = float(np.max(np.abs(sp.vx.astype(np.float64)))) if sp.n else 0.0
        vx = sp.vx.astype(np.float64)
        vy = sp.vy.astype(np.float64)
        vz = sp.vz.astype(np.float64)
        f = np.ldexp(1.0, weight_shift(sp, self.u))      # weighted mean over the electrons
        mean_ev = float(np.sum(f * (ph.HALF_ME_OVER_QE * ((vx * vx + vy * vy) + vz * vz))) / np.sum(f)) \
            if sp.n else 0.0
        te = 2.0 * mean_ev / 3.0
        lde = math.sqrt(ph.EPS0 * te / (ne_max * ph.QE)) if ne_max > 0 else 0.0
        return dict(ne_max_m3=ne_max, wpe_dt_max=wpe * self.dt,
                    vmax_dt_over_dxmin=vmax * self.dt / hmin, lambda_de_over_dxmin=lde / hmin,
                    te_ev=te)

    def rebalance(self):
        """Merge and split particles toward rebalance_ppc per cell (Section 3d;
        see oracle/rebalance.py); returns [(merges, splits) per species]."""
        from .rebalance import rebalance
        return rebalance(self)

    def positions(self, s):
        sp = self.sp[s]
        if self.prec == FP64:
            return sp.x
        return self.grid.position(sp.cell, sp.off)

    def profiles(self):
        """RF-averaged electron and ion densities (m^-3), potential (V), EEDF counts."""
        n = max(self.n_samples, 1)
        scale = self.W_unit * TWO_M32
        dens = [(self.acc_A[s] * scale) / (self.grid.V * n) for s in range(2)]
        return dict(ne=dens[0], ni=dens[1], phi=self.acc_phi / n, eedf=self.eedf.copy(),
                    n_samples=self.n_samples, eedf_samples=self.eedf_samples)
