"""Pins of the oracle's second-order energy-conserving scheme: quadratic-spline
(S2) deposit and linear (S1) gather of the cell-centred field (Section 2a: the
gather shape one order below the deposit shape).

The spline is written out here from its textbook definition, independently of
the oracle's branch form; the gather is pinned to the deposit by energy
consistency: q times the gathered field is minus the derivative of the
particle's potential energy sum_n S2_n(x) phi_n (with the deposit's treatment
of the ends).
"""
import math

import numpy as np
import pytest

import inputs
from oracle.pic import (BC_DIRICHLET, BC_PERIODIC, FP32, FP64, GATHER_EC2, Grid, Species,
                        deposit_species, field_ec2, gather_fp32, gather_fp64, to_fp32_state,
                        weights_s2)
from oracle.sim import Sim

TWO32 = 2 ** 32


def s2(u):
    """Quadratic B-spline of unit width: 3/4 - u^2 for |u| <= 1/2,
    (3/2 - |u|)^2 / 2 for 1/2 <= |u| <= 3/2, else 0."""
    u = np.abs(np.asarray(u, dtype=np.float64))
    return np.where(u <= 0.5, 0.75 - u * u, np.where(u <= 1.5, 0.5 * (1.5 - u) ** 2, 0.0))


def spline_weights(grid, x):
    """Exact (real) S2 weight of every node for positions x: nodes -1..N+1 of
    the extended grid, the outside ones moved as the reading states (onto the
    electrode node, or wrapped)."""
    N, dx = grid.N, grid.dx
    s = np.asarray(x, dtype=np.float64) / dx
    W = np.zeros((len(s), N + 1))
    for m in range(-1, N + 2):
        w = s2(s - m)
        if grid.bc == BC_PERIODIC:
            n = m % N
        else:
            n = min(max(m, 0), N)
        W[:, n] += w
    if grid.bc == BC_PERIODIC:
        W[:, N] = 0.0          # node N is node 0
    return W


def one(grid, x):
    return Species(s=0, prec=FP64, vx=np.zeros(len(x)), vy=np.zeros(len(x)), vz=np.zeros(len(x)),
                   id=np.arange(len(x), dtype=np.uint64), knext=np.zeros(len(x), np.int64),
                   x=np.asarray(x, dtype=np.float64))


def test_hand_values_of_the_weights():
    # on a node: 1/8, 3/4, 1/8 of the charge
    n, wl, wc, wr = weights_s2(np.array([3]), np.array([0.0]))
    assert (n[0], wl[0], wc[0], wr[0]) == (3, 2 ** 29, 3 * 2 ** 30, 2 ** 29)
    # a quarter cell right of node 3: 1/32, 11/16, 9/32
    n, wl, wc, wr = weights_s2(np.array([3]), np.array([0.25]))
    assert (n[0], wl[0], wc[0], wr[0]) == (3, 2 ** 27, 22 * 2 ** 27, 9 * 2 ** 27)
    # at a cell centre the nearest node is the right one: half each on j, j+1
    n, wl, wc, wr = weights_s2(np.array([3]), np.array([0.5]))
    assert (n[0], wl[0], wc[0], wr[0]) == (4, 2 ** 31, 2 ** 31, 0)
    # just left of the centre: node j with the same split (continuity)
    n, wl, wc, wr = weights_s2(np.array([3]), np.array([np.nextafter(0.5, 0.0)]))
    assert n[0] == 3 and wl[0] == 0 and wc[0] == 2 ** 31 and wr[0] == 2 ** 31


@pytest.mark.parametrize("bc", [BC_DIRICHLET, BC_PERIODIC])
def test_deposit_against_the_spline_definition(bc):
    """Brute force: every node's fixed-point sum is within one unit per
    touching particle of sum_i S2(x_n - x_i) 2^32, and the total is exact."""
    g = Grid.make(0.02, 16, None, bc)
    rng = inputs.rng(5)
    x = np.concatenate([rng.uniform(0, g.L, 3000), [0.0, 0.3 * g.dx, g.L - 0.2 * g.dx,
                                                    5 * g.dx, 5.5 * g.dx]])
    A = deposit_species(g, one(g, x), GATHER_EC2)
    W = spline_weights(g, x)
    exact = W.sum(axis=0) * TWO32
    touching = (W > 0).sum(axis=0)
    nodes = g.N if bc == BC_PERIODIC else g.N + 1
    assert np.all(np.abs(A[:nodes] - exact[:nodes]) <= touching[:nodes])
    assert int(A[:nodes].sum()) == len(x) * TWO32
    if bc == BC_PERIODIC:
        assert A[g.N] == A[0]


@pytest.mark.parametrize("bc", [BC_DIRICHLET, BC_PERIODIC])
def test_gather_is_minus_the_gradient_of_the_particle_energy(bc):
    """q E(x) = -d/dx sum_n S2_n(x) phi_n for a fixed random potential: the
    gathered field is the one that conserves energy with this deposit,
    including the half cells next to the ends."""
    g = Grid.make(0.02, 12, None, bc)
    rng = inputs.rng(8)
    phi = rng.normal(0.0, 50.0, g.N + 1)
    if bc == BC_PERIODIC:
        phi[g.N] = phi[0]
    G = field_ec2(g, phi)
    x = np.concatenate([rng.uniform(0.0, g.L, 400), [1e-3 * g.dx, 0.49 * g.dx, 0.51 * g.dx,
                                                     g.L - 0.3 * g.dx, 4.5 * g.dx]])
    h = 1e-6 * g.dx
    xp, xm = x + h, x - h
    if bc == BC_PERIODIC:
        xm = np.mod(xm, g.L)
        xp = np.mod(xp, g.L)
    else:
        xm = np.maximum(xm, 0.0)
    dphi = (spline_weights(g, xp) @ phi - spline_weights(g, xm) @ phi) / (xp - xm)
    e = gather_fp64(g, x, G, GATHER_EC2)
    scale = np.max(np.abs(G))
    assert np.max(np.abs(e + dphi)) < 1e-6 * scale
    # the FP32 form gathers the same field to FP32 rounding
    cell, off = to_fp32_state(g, x)
    e32 = gather_fp32(cell, off, G.astype(np.float32), GATHER_EC2)
    assert np.max(np.abs(e32.astype(np.float64) - e)) < 1e-5 * scale


def test_uniform_field_is_gathered_exactly():
    """A linear potential gives E = V/L in every cell and at every position
    at least half a cell from the electrodes.  Closer to an electrode the
    ghost field is zero, so the gathered field falls linearly to half of V/L
    at the wall."""
    g = Grid.make(0.02, 10, None, BC_DIRICHLET)
    V = 100.0
    phi = V * (1.0 - g.nodes / g.L)
    G = field_ec2(g, phi)
    x = np.linspace(0.0, g.L, 1001)[:-1]
    e = gather_fp64(g, x, G, GATHER_EC2)
    inner = (x >= 0.5 * g.dx) & (x <= g.L - 0.5 * g.dx)
    assert np.allclose(e[inner], V / g.L, rtol=1e-12)
    assert math.isclose(e[0], 0.5 * V / g.L, rel_tol=1e-12)


def test_second_order_ec_needs_a_uniform_grid():
    from oracle.grid import refined_nodes
    nodes = refined_nodes(0.025, 0.025 / 256, 0.025 / 32, 0.004)
    with pytest.raises(ValueError):
        Sim(inputs.small_discharge(nodes=nodes, n_cells=len(nodes) - 1, gather=GATHER_EC2))


def test_fp32_form_tracks_fp64_form_for_one_step():
    cfg = inputs.small_discharge(n_per_species=4000, seed=4, precision=FP32, gamma_see=0.0,
                                 gather=GATHER_EC2)
    s32 = Sim(cfg)
    s32.run(3)
    sps64 = [Species(s=sp.s, prec=FP64, vx=sp.vx.astype(np.float64), vy=sp.vy.astype(np.float64),
                     vz=sp.vz.astype(np.float64), id=sp.id.copy(), knext=sp.knext.copy(),
                     x=s32.grid.position(sp.cell, sp.off)) for sp in s32.sp]
    s64 = Sim(dict(cfg, precision=FP64), species=sps64, k=s32.k)
    s32.deposit()
    s64.deposit()
    for a, b in zip(s32.A, s64.A):
        # the same positions (FP32 widened exactly): charge equal to rounding
        assert np.max(np.abs(a - b)) <= 2 * 4000
    s32.step()
    s64.step()
    assert np.max(np.abs(s32.phi - s64.phi)) < 1e-5 * np.max(np.abs(s64.phi))
