"""Pins of the oracle's equilibria against what the paper fixes.

* Moments of f^eq and g^eq: the table of equilibrium moments in Appendix A
  (zeroth, first and second moments; off-diagonal third moments of f^eq,
  which the first-neighbour lattice reproduces exactly).
* The operator moments prod_a O_a^{k_a} E (eqs. Egen, Oa): recomputed here
  symbolically with sympy, an independent route to the same definition.
* The product-form factor Psi (eq. phi): zeroth, first and second moments
  over c in {-1, 0, 1} equal 1, xi and zeta.
"""
import itertools

import numpy as np
import pytest
import sympy as sp

import oracle


def _states(D, n=6, seed=1):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        rho = rng.uniform(0.5, 8.0)
        u = rng.uniform(-0.3, 0.3, D)
        theta = rng.uniform(0.02, 0.2)
        e = rng.uniform(-0.2, 0.8)
        yield rho, u, theta, e


@pytest.mark.parametrize("D", [2, 3])
def test_feq_moments_table(D):
    c = oracle.velocities(D).astype(np.float64)
    for rho, u, theta, _ in _states(D):
        f = oracle.feq(D, rho, u, theta)
        P = rho * theta  # theta = P / rho (eq. theta)
        assert np.isclose(f.sum(), rho, rtol=1e-14, atol=0)
        np.testing.assert_allclose(c.T @ f, rho * u, rtol=1e-13, atol=1e-15)
        for a in range(D):
            for b in range(D):
                m2 = np.sum(c[:, a] * c[:, b] * f)
                ref = rho * u[a] * u[b] + (P if a == b else 0.0)
                assert abs(m2 - ref) <= 1e-13 * rho
        # third moments with at most two equal indices (c^3 = c on the lattice
        # spoils only the all-equal diagonal)
        for a, b, g in itertools.product(range(D), repeat=3):
            if a == b == g:
                continue
            m3 = np.sum(c[:, a] * c[:, b] * c[:, g] * f)
            d = lambda i, j: 1.0 if i == j else 0.0
            ref = rho * u[a] * u[b] * u[g] + P * (u[a] * d(b, g) + u[b] * d(a, g) + u[g] * d(a, b))
            assert abs(m3 - ref) <= 1e-13 * rho


@pytest.mark.parametrize("D", [2, 3])
def test_geq_moments_table(D):
    c = oracle.velocities(D).astype(np.float64)
    for rho, u, theta, e in _states(D, seed=2):
        g = oracle.geq(D, rho, u, e, theta)
        E = e + 0.5 * np.dot(u, u)
        P = rho * theta
        scale = rho * (abs(E) + theta + 1.0)
        assert abs(g.sum() - rho * E) <= 1e-13 * scale
        np.testing.assert_allclose(c.T @ g, rho * (E + P / rho) * u, rtol=0, atol=1e-13 * scale)
        for a in range(D):
            for b in range(D):
                m2 = np.sum(c[:, a] * c[:, b] * g)
                ref = rho * u[a] * u[b] * (E + 2 * P / rho) + (P * (E + P / rho) if a == b else 0.0)
                assert abs(m2 - ref) <= 1e-13 * scale


@pytest.mark.parametrize("D", [2, 3])
def test_operator_moments_symbolic(D):
    """prod_a O_a^{k_a} E with O_a = theta d/du_a + u_a, by sympy."""
    us = sp.symbols("ux uy uz")[:D]
    th, e = sp.symbols("theta e")
    E = e + sum(x ** 2 for x in us) / 2

    def O(expr, a):
        return th * sp.diff(expr, us[a]) + us[a] * expr

    exprs = {}
    for k in itertools.product(range(3), repeat=D):
        ex = E
        for a in range(D):
            for _ in range(k[a]):
                ex = O(ex, a)
        exprs[k] = sp.lambdify((*us, th, e), sp.expand(ex))
    for rho, u, theta, ee in _states(D, n=4, seed=3):
        M = oracle.operator_moments(D, u, ee, theta)
        for k, fn in exprs.items():
            kk = k[0] + 3 * k[1] + (9 * k[2] if D == 3 else 0)
            ref = fn(*u, theta, ee)
            assert abs(M[kk] - ref) <= 1e-14 * (1 + abs(ref))


def test_psi_moments():
    """sum_c Psi = 1, sum_c c Psi = xi, sum_c c^2 Psi = zeta (eq. phi)."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        rho, xi, zeta = 1.0, rng.uniform(-1, 1), rng.uniform(0, 1)
        f = oracle.feq(2, rho, np.array([xi, 0.0]), zeta - xi * xi)
        # with u_y = 0 and theta = zeta - xi^2 the y-factor has moments (1, 0, theta)
        c = oracle.velocities(2).astype(np.float64)
        fx = np.array([f[c[:, 0] == v].sum() for v in (-1, 0, 1)])
        cx = np.array([-1.0, 0.0, 1.0])
        assert np.isclose(fx.sum(), 1.0, rtol=0, atol=1e-15)
        assert np.isclose((cx * fx).sum(), xi, rtol=0, atol=1e-15)
        assert np.isclose((cx * cx * fx).sum(), zeta, rtol=0, atol=1e-15)


@pytest.mark.parametrize("D", [2, 3])
def test_geq_reduces_to_feq_weighting_at_rest(D):
    """At u = 0 the operator form gives g^eq_i = f^eq_i (e - D theta/2 + |c_i|^2/2 ...):
    checked through the continuous-model relation of eq. geq_cont restricted to
    the lattice's first three moments: sum g = rho e, sum c_a^2 g = rho theta (e + theta)."""
    c = oracle.velocities(D).astype(np.float64)
    rho, theta, e = 2.0, 0.1, 0.3
    g = oracle.geq(D, rho, np.zeros(D), e, theta)
    assert np.isclose(g.sum(), rho * e, rtol=1e-15)
    for a in range(D):
        assert np.isclose(np.sum(c[:, a] ** 2 * g), rho * theta * (e + theta), rtol=1e-14)
