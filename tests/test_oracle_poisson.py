"""Pins of the oracle's Poisson solve (Eq 4) and fields (Eq 5, MC centred field)."""
import math

import numpy as np
import pytest
import scipy.linalg

import inputs
from oracle import physics as ph
from oracle.pic import (BC_PERIODIC, Grid, field_ec, field_mc, poisson, poisson_dirichlet)

EPS0 = ph.EPS0


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("uniform", [True, False])
def test_uniform_charge_between_plates(uniform):
    """phi = phi0 (1 - x/L) + rho0 x (L - x) / (2 eps0) is exact at the nodes:
    the stencil is exact for quadratics and linear FEM is nodally exact."""
    L, N, phi0, rho0 = 0.025, 64, 150.0, 3e-4
    g = Grid.make(L, N, None if uniform else inputs.random_nodes(L, N, seed=1))
    x = g.nodes
    Q = rho0 * g.V
    phi = poisson_dirichlet(g, Q, phi0)
    exact = phi0 * (1 - x / L) + rho0 * x * (L - x) / (2 * EPS0)
    assert rel(phi, exact) < 1e-12
    # EC cell field equals the exact field at cell mid-points (quadratic phi).
    xm = 0.5 * (x[1:] + x[:-1])
    e_exact = phi0 / L - rho0 * (L - 2 * xm) / (2 * EPS0)
    assert rel(field_ec(g, phi), e_exact) < 1e-9
    # MC end nodes: the half-cell Gauss law gives the exact wall fields.
    E = field_mc(g, phi, Q)
    assert E[0] == pytest.approx(phi0 / L - rho0 * L / (2 * EPS0), rel=1e-9)
    assert E[N] == pytest.approx(phi0 / L + rho0 * L / (2 * EPS0), rel=1e-9)


def test_linear_charge_on_random_grid_is_nodally_exact():
    L, N = 0.03, 64
    g = Grid.make(L, N, inputs.random_nodes(L, N, seed=2))
    a, b = 2e-4, -5e-3
    x, h = g.nodes, g.h
    # Exact FEM load of rho = a + b x against the hat function of node n.
    Q = (a + b * x) * g.V
    Q[1:N] += b * (h[1:] ** 2 - h[:-1] ** 2) / 6.0
    phi0 = -80.0
    phi = poisson_dirichlet(g, Q, phi0)
    # phi'' = -(a + b x)/eps0 with phi(0) = phi0, phi(L) = 0.
    part = -(a * x ** 2 / 2 + b * x ** 3 / 6) / EPS0
    pL = -(a * L ** 2 / 2 + b * L ** 3 / 6) / EPS0
    exact = part + phi0 + (0.0 - phi0 - pL) * x / L
    assert rel(phi, exact) < 1e-11


def test_discrete_eigenmode():
    L, N, m, r0 = 0.02, 128, 3, 1e-5
    g = Grid.make(L, N)
    dx = L / N
    x = g.nodes
    Q = r0 * np.sin(math.pi * m * x / L) * dx
    phi = poisson_dirichlet(g, Q, 0.0)
    exact = r0 * dx ** 2 / (EPS0 * (2 - 2 * math.cos(math.pi * m * dx / L))) * np.sin(math.pi * m * x / L)
    assert rel(phi, exact) < 1e-11


def test_matches_scipy_banded_on_random_grid():
    L, N = 0.3, 2048
    g = Grid.make(L, N, inputs.random_nodes(L, N, seed=3))
    Q = inputs.rng(4).normal(0, 1e-7, N + 1)
    phi0 = 321.0
    phi = poisson_dirichlet(g, Q, phi0)
    h = g.h
    n = N - 1
    ab = np.zeros((3, n))
    ab[0, 1:] = 1 / h[1:N - 1]
    ab[1, :] = -(1 / h[:N - 1] + 1 / h[1:])
    ab[2, :-1] = 1 / h[1:N - 1]
    rhs = -Q[1:N] / EPS0
    rhs[0] -= phi0 / h[0]
    ref = scipy.linalg.solve_banded((1, 1), ab, rhs)
    assert rel(phi[1:N], ref) < 1e-12


def test_periodic_matches_fft():
    L, N = 0.05, 256
    g = Grid.make(L, N, bc=BC_PERIODIC)
    dx = L / N
    Q = inputs.rng(5).normal(0, 1e-8, N + 1)
    Q[N] = Q[0]
    phi = poisson(g, Q, 0.0, 0.0, 0.0, 0.0)
    q = Q[:N] - Q[:N].mean()
    k = np.arange(N)
    lam = (2 - 2 * np.cos(2 * np.pi * k / N)) / dx ** 2
    qh = np.fft.fft(q / dx / EPS0)
    ph_ = np.zeros_like(qh)
    ph_[1:] = qh[1:] / lam[1:]
    ref = np.real(np.fft.ifft(ph_))
    ref -= ref[0]
    assert rel(phi[:N], ref) < 1e-10
    assert phi[N] == 0.0 and phi[0] == 0.0


def test_rf_potential_at_left_electrode():
    g = Grid.make(0.025, 32)
    f, v0, dt = 13.56e6, 200.0, 1 / (400 * 13.56e6)
    phi = poisson(g, np.zeros(33), 37 * dt, v0, f, 0.0)
    assert phi[0] == pytest.approx(v0 * math.sin(2 * math.pi * 37 / 400), rel=1e-12)
    assert phi[-1] == 0.0
    assert np.allclose(np.diff(phi), np.diff(phi)[0], rtol=1e-9)


def test_linear_potential_gives_constant_field_on_any_grid():
    L, N = 0.025, 40
    g = Grid.make(L, N, inputs.random_nodes(L, N, seed=6))
    phi = 300.0 * (1 - g.nodes / L)
    assert np.allclose(field_ec(g, phi), 300.0 / L, rtol=1e-9)
    assert np.allclose(field_mc(g, phi, np.zeros(N + 1)), 300.0 / L, rtol=1e-9)


def test_field_energy_summation_by_parts():
    """With grounded ends, (1/2) sum Q_n phi_n = (eps0/2) sum h_j E_j^2."""
    L, N = 0.02, 50
    g = Grid.make(L, N, inputs.random_nodes(L, N, seed=7))
    Q = inputs.rng(8).normal(0, 1e-8, N + 1)
    phi = poisson_dirichlet(g, Q, 0.0)
    E = field_ec(g, phi)
    assert 0.5 * np.sum(Q[1:N] * phi[1:N]) == pytest.approx(0.5 * EPS0 * np.sum(g.h * E * E), rel=1e-10)
