"""Pins of the oracle's charge deposit (Eqs 2-3)."""
import numpy as np
import pytest

import inputs
from oracle import physics as ph
from oracle.pic import (BC_DIRICHLET, BC_PERIODIC, FP32, FP64, Grid, Species, deposit_species,
                        locate, node_charge, to_fp32_state, weights)

TWO32 = 2 ** 32


def sp64(x):
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    z = np.zeros(n)
    return Species(s=0, prec=FP64, vx=z, vy=z, vz=z, id=np.arange(n, dtype=np.uint64),
                   knext=np.zeros(n, dtype=np.int64), x=x)


def sp32(cell, off):
    n = len(cell)
    z = np.zeros(n, dtype=np.float32)
    return Species(s=0, prec=FP32, vx=z, vy=z, vz=z, id=np.arange(n, dtype=np.uint64),
                   knext=np.zeros(n, dtype=np.int64), cell=np.asarray(cell, dtype=np.int32),
                   off=np.asarray(off, dtype=np.float32))


def test_hand_values_uniform():
    g = Grid.make(1.0, 4)
    A = deposit_species(g, sp64([0.0625]))          # xi = 0.25 in cell 0
    assert list(A) == [3 * TWO32 // 4, TWO32 // 4, 0, 0, 0]
    A = deposit_species(g, sp64([0.75]))            # exactly on node 3: belongs to cell 3
    assert list(A) == [0, 0, 0, TWO32, 0]
    A = deposit_species(g, sp64([0.125, 0.375, 0.875]))   # three cell centres
    assert list(A) == [TWO32 // 2, TWO32 // 2 + TWO32 // 2, TWO32 // 2, TWO32 // 2, TWO32 // 2]


def test_rint_is_half_even():
    w0, w1 = weights(np.array([2.0 ** -33, 3 * 2.0 ** -33, 0.5, 0.0, 1.0]))
    assert list(w1) == [0, 2, TWO32 // 2, 0, TWO32]
    assert list(w0 + w1) == [TWO32] * 5


@pytest.mark.parametrize("uniform", [True, False])
@pytest.mark.parametrize("bc", [BC_DIRICHLET, BC_PERIODIC])
def test_total_charge_exact(uniform, bc):
    L, N = 0.03, 37
    nodes = None if uniform else inputs.random_nodes(L, N, seed=4)
    g = Grid.make(L, N, nodes, bc)
    st = inputs.particles_fp64(5000, L, 1.0, seed=5)
    A = deposit_species(g, sp64(st["x"]))
    total = int(A[:N].sum()) if bc == BC_PERIODIC else int(A.sum())
    assert total == 5000 * TWO32


def test_fp32_total_charge_exact():
    st = inputs.particles_fp32(4000, 50, 1.0, seed=6)
    A = deposit_species(Grid.make(0.02, 50), sp32(st["cell"], st["off"]))
    assert int(A.sum()) == 4000 * TWO32


def s1(t):
    """Eq (3): the linear shape function."""
    t = np.asarray(t)
    return np.where((t >= -1) & (t < 0), 1 + t, np.where((t >= 0) & (t <= 1), 1 - t, 0.0))


def test_uniform_density_matches_eq2_by_brute_force():
    L, N = 0.025, 16
    g = Grid.make(L, N)
    dx = L / N
    st = inputs.particles_fp64(300, L, 1.0, seed=7)
    W = 1e9
    A = deposit_species(g, sp64(st["x"]))
    Q = node_charge([A], [-ph.QE * W])
    rho = Q / g.V
    xn = np.arange(N + 1) * dx
    rho_eq2 = (1.0 / dx) * (-ph.QE * W) * s1((st["x"][None, :] - xn[:, None]) / dx).sum(axis=1)
    touching = (np.abs(st["x"][None, :] - xn[:, None]) < dx).sum(axis=1)
    bound = touching * ph.QE * W * 2.0 ** -33 / dx + 1e-12 * np.abs(rho_eq2).max()
    assert np.all(np.abs(rho[1:N] - rho_eq2[1:N]) <= bound[1:N])


def test_nonuniform_charge_matches_hat_functions():
    L, N = 0.02, 23
    nodes = inputs.random_nodes(L, N, seed=8)
    g = Grid.make(L, N, nodes)
    st = inputs.particles_fp64(400, L, 1.0, seed=9)
    A = deposit_species(g, sp64(st["x"]))
    W = 2e9
    Q = node_charge([A], [ph.QE * W])
    X = st["x"]
    Qb = np.zeros(N + 1)
    for n in range(N + 1):
        s = np.zeros_like(X)
        if n > 0:
            m = (X >= nodes[n - 1]) & (X < nodes[n])
            s[m] = (X[m] - nodes[n - 1]) / (nodes[n] - nodes[n - 1])
        if n < N:
            m = (X >= nodes[n]) & (X < nodes[n + 1])
            s[m] = (nodes[n + 1] - X[m]) / (nodes[n + 1] - nodes[n])
        Qb[n] = ph.QE * W * s.sum()
    assert np.allclose(Q, Qb, rtol=0, atol=ph.QE * W * 400 * 2.0 ** -32 * 2)


def test_periodic_fold_puts_last_cell_weight_on_node_zero():
    g = Grid.make(1.0, 4, bc=BC_PERIODIC)
    A = deposit_species(g, sp64([0.875]))    # centre of the last cell
    assert A[0] == TWO32 // 2 and A[3] == TWO32 // 2 and A[4] == A[0]


def test_locate_agrees_between_uniform_and_explicit_nodes():
    L, N = 0.025, 64
    gu = Grid.make(L, N)
    gn = Grid.make(L, N, np.arange(N + 1) * (L / N))
    x = inputs.particles_fp64(3000, L, 1.0, seed=10)["x"]
    ju, xu = locate(gu, x)
    jn, xn = locate(gn, x)
    same = ju == jn
    assert same.mean() > 0.999
    assert np.allclose(xu[same], xn[same], atol=1e-12)


def test_fp32_state_conversion_keeps_offsets_in_unit_interval():
    L, N = 0.3, 100
    g = Grid.make(L, N)
    x = np.concatenate([inputs.particles_fp64(2000, L, 1.0, seed=11)["x"],
                        np.arange(N) * (L / N), [np.nextafter(L, 0.0)]])
    cell, off = to_fp32_state(g, x)
    assert np.all((off >= 0) & (off < 1)) and np.all((cell >= 0) & (cell < N))
    back = g.position(cell, off)
    assert np.allclose(back, x, atol=L / N * 1e-7)
