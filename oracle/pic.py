"""Plain FP64 reference of one EC-PIC / MC-PIC time step (1D3V, argon).

Test infrastructure only (see ``oracle/__init__.py``).

Each function states the passage of the paper it follows.  Where the paper is
silent the reading taken is stated in the docstring; the readings are:

* Geometry.  N cells, nodes x_0 = 0 < ... < x_N = L, cell j = [x_j, x_{j+1})
  of width h_j.  Eq (4) calls the Dirichlet nodes phi_0 and phi_{N+1}; here the
  ends are nodes 0 and N.  The left electrode is the powered one,
  phi_0(t_k) = V0 sin(2 pi f t_k + phase) with t_k = k dt, and phi_N = 0.
* Deposit (Eqs 2-3).  The S1 weights are formed in 32-bit fixed point and
  summed in int64 so the charge is exact and order independent: with xi the
  fractional position in the cell, w1 = rint(xi 2^32) (half-to-even) and
  w0 = 2^32 - w1 go to nodes j and j+1.  A particle on a node belongs to the
  cell on its right (S0 of Eq 7 is 1 on [0, 1)).  The node charge per area is
  Q_n = sum_s q_s W A_{s,n} 2^-32.
* Poisson (Eq 4), generalised to a non-uniform grid in its finite-volume
  form (phi_{n+1}-phi_n)/h_n - (phi_n-phi_{n-1})/h_{n-1} = -Q_n/eps0, which
  divided by dx is Eq 4 on a uniform grid.  Solved by the Thomas algorithm
  (the "LU decomposition" of Section 2).
* EC field (Eq 5) on cells, E_j = -(phi_{j+1}-phi_j)/h_j; EC gather (Eqs 6-7)
  gives a particle the field of its cell.
* MC field: centred differences at nodes (Section 1), with the Dirichlet end
  nodes closed by Gauss's law on the half cell; MC gather uses S1 (Eq 3).
* Leapfrog (Eqs 8-9).  The initial velocity is used as v^{-1/2} unless the
  pull-back switch is set.
* Collisions (Sections 2 and 2a): null collisions after the push,
  with the candidate steps drawn as exponential waiting times (equivalent in
  law to a per-step test with probability 1 - exp(-nu_max dt)).
* Secondary emission (not in the paper): an absorbed ion emits an electron at
  the same wall with probability gamma.
* FP32-state form: the particle keeps an int32 cell and an FP32 offset; the
  push moves it by an FP32 cell walk whose operation order is fixed below.
* Second-order EC (Section 2a: the gather shape one order below the deposit
  shape), uniform grids only: quadratic-spline (S2) deposit to the nearest
  node and its two neighbours, linear (S1) gather of the cell-centred field.
  Deposit weights that fall beyond a Dirichlet end go to the electrode node;
  the matching gather sees a zero field half a cell outside each electrode.
  A periodic grid wraps both.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import physics as ph
from .philox import philox4x32, u32, u52

TWO32 = 4294967296.0
TWO_M32 = 2.0 ** -32
INT32_MAX = 2 ** 31 - 1
TWO_PI = 2.0 * math.pi

BC_DIRICHLET, BC_PERIODIC = 0, 1
WC_UNIT = 4          # weight class of weight W (classes 0-7: W 2^(c-4))
GATHER_EC, GATHER_MC, GATHER_EC2 = 0, 1, 2
FP64, FP32 = 0, 1

# Philox counter tags (counter word 1 = tag | species << 8).
TAG_COLL, TAG_EJECT, TAG_GAS, TAG_SEE, TAG_CHILD, TAG_SEE_POS, TAG_SKIP = 0, 1, 2, 3, 4, 5, 7
TAG_INIT0, TAG_INIT1 = 0xF0, 0xF1


# ---------------------------------------------------------------------------
# Random draws
# ---------------------------------------------------------------------------
def draw(ids, k, tag, species, seed):
    """Philox4x32-10 block with key = id and counter = (k, tag | species<<8, seed)."""
    ids = np.asarray(ids, dtype=np.uint64)
    seed = int(seed)
    return philox4x32(np.uint64(k & 0xFFFFFFFF), np.uint64(tag | (species << 8)),
                      np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF),
                      ids & np.uint64(0xFFFFFFFF), ids >> np.uint64(32))


def box_muller(ua, ub):
    """Two standard normals from two uniforms in (0, 1)."""
    r = np.sqrt(-2.0 * np.log(ua))
    a = TWO_PI * ub
    return r * np.cos(a), r * np.sin(a)


def next_candidate(ids, k, species, seed, nudt):
    """First candidate step after step k: k + 1 + floor(-ln u / (nu_max dt)).

    With collisions off (nudt == 0) the particle is never a candidate.
    """
    ids = np.asarray(ids, dtype=np.uint64)
    if nudt <= 0.0:
        return np.full(ids.shape, INT32_MAX, dtype=np.int64)
    r0, r1, _, _ = draw(ids, k, TAG_SKIP, species, seed)
    return _geometric(k + 1, u52(r0, r1), nudt)


def _geometric(base, u, nudt):
    g = np.floor(-np.log(u) / nudt)
    g = np.minimum(g, float(INT32_MAX))
    out = np.minimum(base + g, float(INT32_MAX))
    return out.astype(np.int64)


def ids_from_words(lo, hi):
    return np.asarray(lo, dtype=np.uint64) | (np.asarray(hi, dtype=np.uint64) << np.uint64(32))


# ---------------------------------------------------------------------------
# Grid
# ---------------------------------------------------------------------------
@dataclass
class Grid:
    """Cells j = [x_j, x_{j+1}); ``uniform`` grids use dx = L / N exactly."""
    L: float
    N: int
    bc: int
    uniform: bool
    dx: float
    nodes: np.ndarray   # (N+1,)
    h: np.ndarray       # (N,)
    V: np.ndarray       # (N+1,) control-volume widths of the nodes

    @staticmethod
    def make(L, N, nodes=None, bc=BC_DIRICHLET):
        if nodes is None:
            dx = L / N
            h = np.full(N, dx)
            nd = np.arange(N + 1, dtype=np.float64) * dx
            uniform = True
        else:
            nd = np.asarray(nodes, dtype=np.float64).copy()
            assert nd.shape == (N + 1,)
            h = nd[1:] - nd[:-1]
            dx = 0.0
            uniform = False
            L = float(nd[-1])
        V = np.empty(N + 1)
        V[1:N] = (h[:-1] + h[1:]) / 2.0
        if bc == BC_PERIODIC:
            V[0] = (h[N - 1] + h[0]) / 2.0
            V[N] = V[0]
        else:
            V[0] = h[0] / 2.0
            V[N] = h[N - 1] / 2.0
        return Grid(L=L, N=N, bc=bc, uniform=uniform, dx=dx, nodes=nd, h=h, V=V)

    # FP32 walk tables (per cell): Delta t / h_j and neighbour ratios.
    def walk_tables(self, dt):
        N = self.N
        if self.uniform:
            dtoh = np.full(N, np.float32(dt / self.dx), dtype=np.float32)
            rf = np.ones(N, dtype=np.float32)
            rb = np.ones(N, dtype=np.float32)
        else:
            h = self.h
            nxt = np.roll(h, -1)                 # h_{(j+1) mod N}
            dtoh = (dt / h).astype(np.float32)
            rf = (h / nxt).astype(np.float32)    # leaving cell j forward
            rb = (nxt / h).astype(np.float32)    # entering cell j from j+1
        return dtoh, rf, rb

    def position(self, cell, off):
        """FP64 position of an FP32-state particle: x_j + off h_j."""
        cell = np.asarray(cell, dtype=np.int64)
        off = np.asarray(off, dtype=np.float32).astype(np.float64)
        if self.uniform:
            return cell.astype(np.float64) * self.dx + off * self.dx
        return self.nodes[cell] + off * self.h[cell]


def locate(grid: Grid, x):
    """(j, xi) for FP64 positions x in [0, L) -- the deposit contract.

    Uniform grid: s = x / dx, j = floor(s), xi = s - j.  Non-uniform grid:
    j = max{n : x_n <= x}, xi = (x - x_j) / h_j.  xi is clipped to [0, 1]; j to
    [0, N-1].
    """
    x = np.asarray(x, dtype=np.float64)
    N = grid.N
    if grid.uniform:
        s = x / grid.dx
        jf = np.floor(s)
        j = jf.astype(np.int64)
        over = j >= N
        j[over] = N - 1
        xi = s - j.astype(np.float64)
    else:
        j = np.searchsorted(grid.nodes, x, side="right").astype(np.int64) - 1
        j = np.clip(j, 0, N - 1)
        xi = (x - grid.nodes[j]) / grid.h[j]
    xi = np.clip(xi, 0.0, 1.0)
    return j, xi


def to_fp32_state(grid: Grid, x):
    """(cell int32, off float32) of FP64 positions: off = (float) xi; an offset
    that rounds up to 1 moves to the next cell (or, in the last cell of a
    bounded grid, stays below 1)."""
    j, xi = locate(grid, x)
    off = xi.astype(np.float32)
    up = off >= np.float32(1.0)
    if up.any():
        last = up & (j + 1 >= grid.N)
        mid = up & ~last
        j[mid] += 1
        off[mid] = np.float32(0.0)
        if grid.bc == BC_PERIODIC:
            j[last] = 0
            off[last] = np.float32(0.0)
        else:
            off[last] = np.nextafter(np.float32(1.0), np.float32(0.0))
    return j.astype(np.int32), off


# ---------------------------------------------------------------------------
# Species state
# ---------------------------------------------------------------------------
@dataclass
class Species:
    """Live particles of one species (the oracle keeps no dead slots)."""
    s: int                    # 0 electrons, 1 ions
    prec: int
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    id: np.ndarray            # uint64
    knext: np.ndarray         # int64, first step at which the particle is a collision candidate
    x: np.ndarray = None      # FP64 form
    cell: np.ndarray = None   # FP32 form
    off: np.ndarray = None
    wc: np.ndarray = None     # weight class c (uint8): weight W 2^(c-4); None = all 4

    @property
    def n(self):
        return int(self.id.shape[0])

    def classes(self):
        """Weight class of every particle (4, weight W, unless set)."""
        if self.wc is None:
            return np.full(self.n, WC_UNIT, dtype=np.uint8)
        return self.wc

    def subset(self, m):
        kw = dict(s=self.s, prec=self.prec, vx=self.vx[m], vy=self.vy[m], vz=self.vz[m],
                  id=self.id[m], knext=self.knext[m])
        if self.prec == FP64:
            kw["x"] = self.x[m]
        else:
            kw["cell"] = self.cell[m]
            kw["off"] = self.off[m]
        if self.wc is not None:
            kw["wc"] = self.wc[m]
        return Species(**kw)

    def append(self, other: "Species"):
        if other is None or other.n == 0:
            return self
        kw = dict(s=self.s, prec=self.prec)
        for f in ("vx", "vy", "vz", "id", "knext") + (("x",) if self.prec == FP64 else ("cell", "off")):
            kw[f] = np.concatenate([getattr(self, f), getattr(other, f)])
        if self.wc is not None or other.wc is not None:
            kw["wc"] = np.concatenate([self.classes(), other.classes()])
        return Species(**kw)

    def order_by_id(self):
        return self.subset(np.argsort(self.id, kind="stable"))


# ---------------------------------------------------------------------------
# Step 1: charge deposit (Eqs 2-3)
# ---------------------------------------------------------------------------
def weights(xi):
    """Fixed-point S1 weights: w1 = rint(xi 2^32), w0 = 2^32 - w1 (int64)."""
    w1 = np.rint(np.asarray(xi, dtype=np.float64) * TWO32).astype(np.int64)
    w0 = (np.int64(1) << np.int64(32)) - w1
    return w0, w1


def weights_s2(j, xi):
    """Fixed-point quadratic-spline (S2) weights of a particle at (j, xi).

    The particle's nearest node is n = j (xi < 1/2) or j + 1, at signed
    distance d = xi or xi - 1 cells.  The spline gives nodes n-1, n, n+1 the
    weights (1/2 - d)^2/2, 3/4 - d^2, (1/2 + d)^2/2.  With a = 1/2 - d and
    b = 1/2 + d formed in FP64 (a = 1/2 - xi or 3/2 - xi, b = 1/2 + xi or
    xi - 1/2), wl = rint(a a 2^31), wr = rint(b b 2^31) (half-to-even) and
    wc = 2^32 - wl - wr, so the three sum to 2^32 exactly.
    Returns (n, wl, wc, wr).
    """
    j = np.asarray(j, dtype=np.int64)
    xi = np.asarray(xi, dtype=np.float64)
    up = xi >= 0.5
    n = j + up.astype(np.int64)
    a = np.where(up, 1.5 - xi, 0.5 - xi)
    b = np.where(up, xi - 0.5, 0.5 + xi)
    wl = np.rint((a * a) * 2147483648.0).astype(np.int64)
    wr = np.rint((b * b) * 2147483648.0).astype(np.int64)
    wc = (np.int64(1) << np.int64(32)) - wl - wr
    return n, wl, wc, wr


def fold_s2(grid: Grid, m):
    """Node index of an S2 weight at node m in [-1, N+1]: beyond a Dirichlet
    end it goes to the electrode node; a periodic grid wraps it."""
    N = grid.N
    m = np.asarray(m, dtype=np.int64).copy()
    if grid.bc == BC_PERIODIC:
        m[m < 0] += N
        m[m > N] -= N
    else:
        m = np.clip(m, 0, N)
    return m


def weight_shift(sp: Species, u):
    """Per particle, the power of two of its weight in the deposit's unit
    W 2^-u: c - 4 + u (0 for every particle without rebalancing, u = 0)."""
    return sp.classes().astype(np.int64) - WC_UNIT + int(u)


def deposit_species(grid: Grid, sp: Species, gather=GATHER_EC, u=0):
    """A_{s,n} = sum over particles of the weights of node n (int64, exact):
    S1 for EC and MC, S2 for second-order EC; a particle of weight class c
    adds its weights times 2^(c - 4 + u), in units of W 2^-u 2^-32."""
    A = np.zeros(grid.N + 1, dtype=np.int64)
    if sp.n == 0:
        return A
    if sp.prec == FP64:
        j, xi = locate(grid, sp.x)
    else:
        j = sp.cell.astype(np.int64)
        xi = sp.off.astype(np.float64)
    sh = weight_shift(sp, u)
    if gather == GATHER_EC2:
        n, wl, wc, wr = weights_s2(j, xi)
        np.add.at(A, fold_s2(grid, n - 1), wl << sh)
        np.add.at(A, n, wc << sh)
        np.add.at(A, fold_s2(grid, n + 1), wr << sh)
    else:
        w0, w1 = weights(xi)
        np.add.at(A, j, w0 << sh)
        np.add.at(A, j + 1, w1 << sh)
    if grid.bc == BC_PERIODIC:
        A[0] += A[grid.N]
        A[grid.N] = A[0]
    return A


def node_charge(A_list, qW_list):
    """Q_n = sum_s (q_s W_s A_{s,n}) 2^-32, per unit area (C/m^2)."""
    Q = None
    for A, qW in zip(A_list, qW_list):
        term = (qW * A.astype(np.float64)) * TWO_M32
        Q = term if Q is None else Q + term
    return Q


def density(grid: Grid, Q):
    """rho_n = Q_n / V_n (Eq 2 on a uniform grid)."""
    return Q / grid.V


# ---------------------------------------------------------------------------
# Step 2: Poisson (Eq 4), Thomas algorithm
# ---------------------------------------------------------------------------
def thomas(a, b, c, d):
    """Solve a_i u_{i-1} + b_i u_i + c_i u_{i+1} = d_i (a_0 and c_{n-1} unused)."""
    n = len(d)
    cp = [0.0] * n
    dp = [0.0] * n
    cp[0] = c[0] / b[0]
    dp[0] = d[0] / b[0]
    for i in range(1, n):
        m = b[i] - a[i] * cp[i - 1]
        cp[i] = c[i] / m
        dp[i] = (d[i] - a[i] * dp[i - 1]) / m
    u = [0.0] * n
    u[n - 1] = dp[n - 1]
    for i in range(n - 2, -1, -1):
        u[i] = dp[i] - cp[i] * u[i + 1]
    return u


def poisson_dirichlet(grid: Grid, Q, phi0, phiN=0.0):
    """phi with phi_0, phi_N given and, for n = 1..N-1,
    (phi_{n+1}-phi_n)/h_n - (phi_n-phi_{n-1})/h_{n-1} = -Q_n/eps0."""
    N = grid.N
    h = [float(v) for v in grid.h]
    phi = np.empty(N + 1)
    phi[0] = phi0
    phi[N] = phiN
    if N < 2:
        return phi
    a, b, c, d = [], [], [], []
    for n in range(1, N):
        an = 1.0 / h[n - 1]
        cn = 1.0 / h[n]
        a.append(an)
        c.append(cn)
        b.append(-(an + cn))
        d.append(-float(Q[n]) / ph.EPS0)
    d[0] -= a[0] * phi0
    d[-1] -= c[-1] * phiN
    phi[1:N] = thomas(a, b, c, d)
    return phi


def neutralise(grid: Grid, Q):
    """Periodic domain: subtract the uniform background (sum Q / L) V_n."""
    N = grid.N
    Qp = Q.copy()
    total = float(np.sum(Q[:N]))
    Qp[:N] = Q[:N] - (total / grid.L) * grid.V[:N]
    Qp[N] = Qp[0]
    return Qp


def poisson(grid: Grid, Q, t, v_rf, f_rf, phase):
    """Dirichlet: phi_0 = V0 sin(2 pi f t + phase), phi_N = 0.  Periodic: the
    neutralised charge with the gauge phi_0 = phi_N = 0 (node N is node 0)."""
    if grid.bc == BC_PERIODIC:
        return poisson_dirichlet(grid, neutralise(grid, Q), 0.0, 0.0)
    phi0 = v_rf * math.sin(TWO_PI * f_rf * t + phase)
    return poisson_dirichlet(grid, Q, phi0, 0.0)


# ---------------------------------------------------------------------------
# Step 3: field
# ---------------------------------------------------------------------------
def field_ec(grid: Grid, phi):
    """Eq (5): E_j = -(phi_{j+1} - phi_j) / h_j, one value per cell."""
    return -(phi[1:] - phi[:-1]) / grid.h


def field_mc(grid: Grid, phi, Q):
    """Centred nodal field E_n = -(phi_{n+1} - phi_{n-1}) / (h_{n-1} + h_n).

    Dirichlet end nodes: Gauss's law on the half cell,
    E_0 = -(phi_1 - phi_0)/h_0 - Q_0/eps0 and E_N = -(phi_N - phi_{N-1})/h_{N-1} + Q_N/eps0.
    Periodic: node 0 uses cells N-1 and 0; E_N = E_0.
    """
    N = grid.N
    h = grid.h
    E = np.empty(N + 1)
    E[1:N] = -(phi[2:] - phi[:-2]) / (h[:-1] + h[1:])
    if grid.bc == BC_PERIODIC:
        E[0] = -(phi[1] - phi[N - 1]) / (h[N - 1] + h[0])
        E[N] = E[0]
    else:
        E[0] = -(phi[1] - phi[0]) / h[0] - Q[0] / ph.EPS0
        E[N] = -(phi[N] - phi[N - 1]) / h[N - 1] + Q[N] / ph.EPS0
    return E


def field_ec2(grid: Grid, phi):
    """Gather table of second-order EC: the cell fields E_j of Eq (5) at the
    cell centres, with one ghost centre outside each end, N + 2 values
    G[m] = E_{m-1}.  The ghosts follow from the folded S2 deposit (the
    particle's energy sum_n S2_n(x) phi_n with the outside weight on the
    electrode node is that of a ghost node at the electrode's potential):
    zero field at a Dirichlet end, the wrapped cell in a periodic box."""
    E = field_ec(grid, phi)
    N = grid.N
    G = np.zeros(N + 2)
    G[1:N + 1] = E
    if grid.bc == BC_PERIODIC:
        G[0] = E[N - 1]
        G[N + 1] = E[0]
    return G


# ---------------------------------------------------------------------------
# Steps 4-5: gather and leapfrog push (Eqs 6-9)
# ---------------------------------------------------------------------------
def s2_gather_index(j, xi):
    """Second-order EC gather of a particle at (j, xi): linear between the
    two cell centres around it, table entries m and m + 1 (G[m] = E_{m-1}),
    m = j with t = xi + 1/2 when xi < 1/2, else m = j + 1 with t = xi - 1/2."""
    up = xi >= 0.5
    m = j + up.astype(np.int64)
    t = np.where(up, xi - 0.5, xi + 0.5)
    return m, t


def gather_fp64(grid: Grid, x, E, gather):
    j, xi = locate(grid, x)
    if gather == GATHER_EC:
        return E[j]
    if gather == GATHER_EC2:
        m, t = s2_gather_index(j, xi)
        return (1.0 - t) * E[m] + t * E[m + 1]
    return (1.0 - xi) * E[j] + xi * E[j + 1]


def gather_fp32(cell, off, E32, gather):
    """FP32 gather: EC takes E32[cell]; MC forms ((1 - off) E_j) + (off E_{j+1})
    in FP32; second-order EC forms t = off + 1/2 or off - 1/2 in FP32, then
    ((1 - t) G_m) + (t G_{m+1})."""
    j = cell.astype(np.int64)
    if gather == GATHER_EC:
        return E32[j]
    one = np.float32(1.0)
    if gather == GATHER_EC2:
        half = np.float32(0.5)
        up = off >= half
        m = j + up.astype(np.int64)
        t = np.where(up, off - half, off + half).astype(np.float32)
        return ((one - t) * E32[m]) + (t * E32[m + 1])
    a = (one - off) * E32[j]
    b = off * E32[j + 1]
    return a + b


def push_fp64(grid: Grid, sp: Species, E, gather, qmdt, dt):
    """vx += (q/m) E_i dt (Eq 8), x += vx dt (Eq 9); returns (vx, x, wall) with
    wall = -1 (absorbed at x < 0), +1 (absorbed at x >= L) or 0."""
    e = gather_fp64(grid, sp.x, E, gather)
    vx = sp.vx + qmdt * e
    x = sp.x + vx * dt
    wall = np.zeros(sp.n, dtype=np.int8)
    L = grid.L
    if grid.bc == BC_PERIODIC:
        while True:
            m = x < 0.0
            if not m.any():
                break
            x[m] = x[m] + L
        while True:
            m = x >= L
            if not m.any():
                break
            x[m] = x[m] - L
    else:
        wall[x < 0.0] = -1
        wall[x >= L] = 1
    return vx, x, wall


def push_fp32(grid: Grid, sp: Species, E32, gather, qmdt32, tables):
    """FP32-state push.  In FP32 arithmetic, in this order:

    vx' = vx + qmdt * e;  sigma = off + vx' * (dt/h_j);
    while sigma < 0:  j -= 1 (leave/wrap), sigma = 1 + sigma * (h_{j+1}/h_j);
    while sigma >= 1: sigma = (sigma - 1) * (h_j/h_{j+1}), j += 1 (leave/wrap).
    The walk stops when the particle leaves a bounded grid.  Returns
    (vx, cell, off, wall).
    """
    dtoh, rf, rb = tables
    N = grid.N
    periodic = grid.bc == BC_PERIODIC
    one = np.float32(1.0)
    e = gather_fp32(sp.cell, sp.off, E32, gather)
    vx = sp.vx + qmdt32 * e
    j = sp.cell.astype(np.int64).copy()
    sig = sp.off + vx * dtoh[j]
    wall = np.zeros(sp.n, dtype=np.int8)

    m = sig < 0
    while m.any():
        j[m] -= 1
        out = m & (j < 0)
        if periodic:
            j[out] += N
        else:
            wall[out] = -1
            m &= ~out
        idx = np.nonzero(m)[0]
        t = sig[idx] * rb[j[idx]]
        sig[idx] = one + t
        m[idx] = sig[idx] < 0

    m = (sig >= one) & (wall == 0)
    while m.any():
        idx = np.nonzero(m)[0]
        sig[idx] = (sig[idx] - one) * rf[j[idx]]
        j[idx] += 1
        out = m & (j >= N)
        if periodic:
            j[out] -= N
        else:
            wall[out] = 1
            m &= ~out
        m &= sig >= one
    return vx, j.astype(np.int32), sig, wall


# ---------------------------------------------------------------------------
# Secondary electron emission at the electrodes (not in the paper)
# ---------------------------------------------------------------------------
def emit_secondaries(grid: Grid, ion_ids, walls, k, seed, gamma, t_see_ev, dt, prec, nudt_e,
                     ion_wc=None):
    """Each absorbed ion emits one electron at its wall with probability gamma.

    |vx| = v_t sqrt(-2 ln u) (flux-weighted half Maxwellian), vy, vz Maxwellian,
    v_t = sqrt(e T_see / m_e); the electron starts at wall +- |vx| dt u' moving
    into the gap; an emission whose start point would lie outside [0, L) is dropped.
    """
    if gamma <= 0.0 or len(ion_ids) == 0:
        return None
    ion_ids = np.asarray(ion_ids, dtype=np.uint64)
    r0, r1, r2, r3 = draw(ion_ids, k, TAG_SEE, 1, seed)
    emit = u32(r0) < gamma
    p0, p1, p2, _ = draw(ion_ids, k, TAG_SEE_POS, 1, seed)
    vt = math.sqrt(t_see_ev * ph.QE / ph.ME)
    vxm = vt * np.sqrt(-2.0 * np.log(u32(r1)))
    zy, zz = box_muller(u32(r2), u32(r3))
    d = (vxm * dt) * u32(p0)
    left = np.asarray(walls) < 0
    x = np.where(left, d, grid.L - d)
    vx = np.where(left, vxm, -vxm)
    ok = emit & (x >= 0.0) & (x < grid.L)
    if not ok.any():
        return None
    ids = ids_from_words(p1[ok], p2[ok])
    sp = Species(s=0, prec=prec, vx=vx[ok], vy=vt * zy[ok], vz=vt * zz[ok], id=ids,
                 knext=next_candidate(ids, k, 0, seed, nudt_e))
    if ion_wc is not None:
        sp.wc = np.asarray(ion_wc)[ok]     # the electron carries the ion's weight
    if prec == FP64:
        sp.x = x[ok]
    else:
        sp.cell, sp.off = to_fp32_state(grid, x[ok])
        sp.vx = sp.vx.astype(np.float32)
        sp.vy = sp.vy.astype(np.float32)
        sp.vz = sp.vz.astype(np.float32)
    return sp


# ---------------------------------------------------------------------------
# Step 6: Monte-Carlo collisions (null collision, after the push)
# ---------------------------------------------------------------------------
def iso_dir(ua, ub):
    """Unit vector uniform on the sphere: cos = 1 - 2 ua about x, azimuth 2 pi ub."""
    ct = 1.0 - 2.0 * ua
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    a = TWO_PI * ub
    return ct, st * np.cos(a), st * np.sin(a)


@dataclass
class MccCounts:
    candidates: int = 0
    elastic: int = 0
    excitation: int = 0
    ionisation: int = 0
    cx: int = 0
    bound_violations: int = 0


def collide_electrons(vx, vy, vz, ids, k, seed, n_g, nu_max, counts: MccCounts):
    """Electron-argon null collision for candidate particles (FP64 arrays).

    R = u1 nu_max selects elastic (R < nu_el), excitation (R < nu_el + nu_ex),
    ionisation (R < nu_el + nu_ex + nu_iz) or a null event.  The scattered
    direction is isotropic; elastic scattering loses the fraction
    (2 m_e / M)(1 - cos chi) of the energy, excitation 11.5 eV; ionisation
    removes 15.76 eV and shares the rest equally between the primary and an
    ejected electron of independent isotropic direction, and creates an Ar+
    with a gas-temperature Maxwellian velocity (filled in by the caller).
    Returns new (vx, vy, vz), the ionising mask, and the ejected velocities.
    """
    r0, r1, r2, _ = draw(ids, k, TAG_COLL, 0, seed)
    u1, u2, u3 = u32(r0), u32(r1), u32(r2)
    v2 = (vx * vx + vy * vy) + vz * vz
    speed = np.sqrt(v2)
    eps = ph.HALF_ME_OVER_QE * v2
    nu_el = (n_g * ph.sigma_el(eps)) * speed
    nu_ex = (n_g * ph.sigma_ex(eps)) * speed
    nu_iz = (n_g * ph.sigma_iz(eps)) * speed
    s_el_ex = nu_el + nu_ex
    s_all = s_el_ex + nu_iz
    R = u1 * nu_max
    el = R < nu_el
    ex = ~el & (R < s_el_ex)
    iz = ~el & ~ex & (R < s_all)
    counts.candidates += int(len(ids))
    counts.elastic += int(el.sum())
    counts.excitation += int(ex.sum())
    counts.ionisation += int(iz.sum())
    counts.bound_violations += int((s_all > nu_max).sum())

    dx, dy, dz = iso_dir(u2, u3)
    new_speed = speed.copy()
    if el.any():
        cos_chi = ((vx[el] * dx[el] + vy[el] * dy[el]) + vz[el] * dz[el]) / speed[el]
        f = 1.0 - ph.TWO_ME_OVER_M * (1.0 - cos_chi)
        new_speed[el] = speed[el] * np.sqrt(f)
    if ex.any():
        new_speed[ex] = np.sqrt((eps[ex] - ph.E_EXC) * ph.TWO_QE_OVER_ME)
    if iz.any():
        new_speed[iz] = np.sqrt((0.5 * (eps[iz] - ph.E_ION)) * ph.TWO_QE_OVER_ME)
    hit = el | ex | iz
    nvx = np.where(hit, new_speed * dx, vx)
    nvy = np.where(hit, new_speed * dy, vy)
    nvz = np.where(hit, new_speed * dz, vz)

    ej = None
    if iz.any():
        q0, q1, _, _ = draw(ids[iz], k, TAG_EJECT, 0, seed)
        ex2, ey2, ez2 = iso_dir(u32(q0), u32(q1))
        s = new_speed[iz]
        ej = (s * ex2, s * ey2, s * ez2)
    return nvx, nvy, nvz, iz, ej


def gas_velocity(ids, k, species, seed, vti):
    """Three Maxwellian components at the gas temperature from one Philox block."""
    g0, g1, g2, g3 = draw(ids, k, TAG_GAS, species, seed)
    z0, z1 = box_muller(u32(g0), u32(g1))
    z2, _ = box_muller(u32(g2), u32(g3))
    return vti * z0, vti * z1, vti * z2


def collide_ions(vx, vy, vz, ids, k, seed, n_g, nu_max, vti, counts: MccCounts):
    """Ion-argon charge exchange: the ion takes the velocity v_g of a gas atom
    drawn from the gas Maxwellian when u1 nu_max < n_g sigma_cx |v - v_g|."""
    r0, _, _, _ = draw(ids, k, TAG_COLL, 1, seed)
    u1 = u32(r0)
    gx, gy, gz = gas_velocity(ids, k, 1, seed, vti)
    ddx, ddy, ddz = vx - gx, vy - gy, vz - gz
    g = np.sqrt((ddx * ddx + ddy * ddy) + ddz * ddz)
    nu = (n_g * ph.SIGMA_CX) * g
    cx = (u1 * nu_max) < nu
    counts.candidates += int(len(ids))
    counts.cx += int(cx.sum())
    counts.bound_violations += int((nu > nu_max).sum())
    return np.where(cx, gx, vx), np.where(cx, gy, vy), np.where(cx, gz, vz)


# ---------------------------------------------------------------------------
# Initial load (Section 2b: uniform density, Maxwellian velocities)
# ---------------------------------------------------------------------------
def init_species(grid: Grid, s, n, T_ev, mass, seed, prec, nudt):
    """Particle i of species s: id = i; x = u L from 52 uniform bits; v from
    Box-Muller normals scaled by sqrt(e T / m); first candidate step from a
    geometric draw.  All draws come from two Philox blocks at k = 0."""
    ids = np.arange(n, dtype=np.uint64)
    r0, r1, r2, r3 = draw(ids, 0, TAG_INIT0, s, seed)
    q0, q1, q2, q3 = draw(ids, 0, TAG_INIT1, s, seed)
    L = grid.L
    x = u52(r0, r1) * L
    top = np.nextafter(L, 0.0)
    x = np.minimum(x, top)
    z0, z1 = box_muller(u32(r2), u32(r3))
    z2, _ = box_muller(u32(q0), u32(q1))
    vt = math.sqrt(T_ev * ph.QE / mass)
    vx, vy, vz = vt * z0, vt * z1, vt * z2
    if nudt > 0.0:
        knext = _geometric(0, u52(q2, q3), nudt)
    else:
        knext = np.full(n, INT32_MAX, dtype=np.int64)
    sp = Species(s=s, prec=prec, vx=vx, vy=vy, vz=vz, id=ids, knext=knext)
    if prec == FP64:
        sp.x = x
    else:
        sp.cell, sp.off = to_fp32_state(grid, x)
        sp.vx = vx.astype(np.float32)
        sp.vy = vy.astype(np.float32)
        sp.vz = vz.astype(np.float32)
    return sp
