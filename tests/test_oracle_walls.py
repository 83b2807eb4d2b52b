"""Walls of the thermal Couette flow (Section 4.1) on the oracle.

The paper gives the flow and its steady solution but not its wall
treatment; the reading is diffuse reflection (the ghost beyond each wall
re-emits equilibria of the wall state scaled to the mass it absorbed).
What the paper and kinetic theory fix:
  * a fluid at rest between walls at rest at its temperature is a fixed
    point, and no mass crosses a wall (mass conserved to round-off);
  * the steady thermal Couette flow: u_y(x) exactly linear, the walls where
    it extrapolates to the wall velocities (within a fraction of a cell of
    the ghost nodes), and the temperature profile a parabola of curvature
    -mu U_w^2 / (2 k L^2) (the paper's solution T = T_w + mu U_w^2 / (2 k)
    (x/L)(1 - x/L)) at the paper's Prandtl numbers 0.6, 1.2, 4.9 and Mach
    number 0.8 (bar 5 %; the temperature jumps at the walls, a kinetic
    slip effect, leave the curvature alone).
"""
import numpy as np
import pytest

import oracle
from oracle import thermo as th

A, B, R, CV = 3.0 / 49.0, 2.0 / 21.0, 1.0, 2.5
RHOC, TC, _ = th.critical(A, B, R)


def test_rest_between_resting_walls_is_a_fixed_point():
    shape = (14, 3, 4)
    T0 = 1.1 * TC
    p = oracle.Params(3, shape, bc=(2, 0, 0), walls=(((0, 0, 0), T0), ((0, 0, 0), T0)))
    N = p.N
    f, g = oracle.init(p, np.full(N, 3.1), np.zeros(3 * N), np.full(N, T0))
    f1, g1 = oracle.run(p, f, g, 7)
    assert np.max(np.abs(f1 - f)) <= 1e-13 * 3.1
    assert np.max(np.abs(g1 - g)) <= 1e-13 * np.abs(g).max()


def test_walls_conserve_mass():
    shape = (20, 6)
    p = oracle.Params(2, shape, bc=(2, 0, 0), walls=(((0.0, -0.05), 0.9 * TC), ((0.0, 0.1), 1.3 * TC)))
    N = p.N
    rng = np.random.default_rng(5)
    rho = RHOC * (1 + 0.05 * rng.uniform(-1, 1, N))
    u = 0.05 * rng.uniform(-1, 1, 2 * N)
    f, g = oracle.init(p, rho, u, np.full(N, 1.1 * TC))
    f1, _ = oracle.run(p, f, g, 50)
    assert abs(f1.sum() - f.sum()) <= 1e-13 * f.sum()


@pytest.mark.parametrize("Pr", [0.6, 1.2, 4.9])
def test_thermal_couette_steady_profile(Pr):
    nx = 32
    rho0, Tw = RHOC, 1.1 * TC
    Uw = 0.8 * np.sqrt(th.cs2(rho0, Tw, A, B, R, CV))
    mu = 0.2
    k = mu * th.cp(rho0, Tw, A, B, R, CV) / Pr
    p = oracle.Params(2, (nx, 1), bc=(2, 0, 0), mu=mu, eta=mu, k=k, kappa=0.0,
                      walls=(((0.0, 0.0), Tw), ((0.0, Uw), Tw)))
    # start from the paper's solution on walls at the ghost nodes
    xi = (np.arange(nx) + 1.0) / (nx + 1.0)
    uy = Uw * xi
    T = Tw + mu * Uw ** 2 / (2 * k) * xi * (1 - xi)
    f, g = oracle.init(p, np.full(nx, rho0), np.concatenate([np.zeros(nx), uy]), T)
    m0 = f.sum()
    f, g = oracle.run(p, f, g, 30000)
    fl = oracle.fields(p, f, g)
    assert abs(f.sum() - m0) <= 1e-12 * m0
    x = np.arange(nx)
    u = fl["u"][nx:]
    c = np.polyfit(x, u, 1)
    assert np.abs(np.polyval(c, x) - u).max() <= 1e-6 * Uw
    xlo, xhi = -c[1] / c[0], (Uw - c[1]) / c[0]
    assert abs(xlo + 1.0) < 0.2 and abs(xhi - nx) < 0.2
    L = xhi - xlo
    curv = np.polyfit(x, fl["T"], 2)[0]
    assert curv == pytest.approx(-mu * Uw ** 2 / (2 * k * L * L), rel=0.05)
