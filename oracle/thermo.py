"""Van der Waals thermodynamics in FP64 (arXiv 2510.14712, Section 2 and 4).

TEST INFRASTRUCTURE ONLY (part of the oracle; see ``oracle/__init__.py``).

Everything here is per unit mass, lattice units, with the van der Waals
equation of state P = rho R T / (1 - b rho) - a rho^2 (eq. Pvdw) and the
caloric relation de = c_v dT - a drho (eq. de_vdW), integrated with the
reference e = c_v T - a rho.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize


# -- critical point (the a, b definitions after eq. Pvdw, solved for rho_c, T_c, P_c)
def critical(a, b, R=1.0):
    """rho_c = 1/(3b), T_c = 8a/(27 R b), P_c = a/(27 b^2)."""
    return 1.0 / (3.0 * b), 8.0 * a / (27.0 * R * b), a / (27.0 * b * b)


def pressure(rho, T, a, b, R=1.0):
    """eq. Pvdw."""
    return rho * R * T / (1.0 - b * rho) - a * rho * rho


def energy(rho, T, a, cv):
    """Specific internal energy from eq. de_vdW: e = c_v T - a rho."""
    return cv * T - a * rho


def temperature(rho, e, a, cv):
    """Explicit caloric inversion, eq. lbm_temp with E - u^2/2 = e."""
    return (e + a * rho) / cv


def cs2(rho, T, a, b, R, cv):
    """Adiabatic sound speed squared, eq. vdW_speed_of_sound."""
    return R * T * (1.0 + R / cv) / (1.0 - b * rho) ** 2 - 2.0 * a * rho


def dPdrho_T(rho, T, a, b, R=1.0):
    return R * T / (1.0 - b * rho) ** 2 - 2.0 * a * rho


def cp(rho, T, a, b, R, cv):
    """Isobaric specific heat for van der Waals, eq. cpvdW."""
    return cv + R * R * T / (R * T - 2.0 * a * rho * (1.0 - b * rho) ** 2)


def enthalpy(rho, T, a, b, R, cv):
    """h = e + P / rho (eq. enthalpy)."""
    return energy(rho, T, a, cv) + pressure(rho, T, a, b, R) / rho


def gibbs(rho, T, a, b, R=1.0):
    """Specific Gibbs energy up to a function of T alone:
    g = -R T ln(1/rho - b) - a rho + P / rho (Helmholtz f = -RT ln(v-b) - a/v)."""
    return -R * T * np.log(1.0 / rho - b) - a * rho + pressure(rho, T, a, b, R) / rho


def spinodal(T, a, b, R=1.0):
    """Densities where (dP/drho)_T = 0 (requires T < T_c)."""
    f = lambda r: dPdrho_T(r, T, a, b, R)
    rc = 1.0 / (3.0 * b)
    lo = optimize.brentq(f, 1e-12, rc)
    hi = optimize.brentq(f, rc, (1.0 - 1e-12) / b)
    return lo, hi


def _volume_roots(P, T, a, b, R):
    # P v^3 - (P b + R T) v^2 + a v - a b = 0  (eq. Pvdw times v^2 (v - b))
    r = np.roots([P, -(P * b + R * T), a, -a * b])
    r = np.sort(r[np.abs(r.imag) < 1e-9].real)
    r = r[r > b]
    return r[0], r[-1]


def maxwell(T, a, b, R=1.0):
    """Coexisting (rho_liquid, rho_vapour, P_sat) by Maxwell's equal-area rule:
    int_{v_l}^{v_v} (P(v) - P_sat) dv = 0 with P(v_l) = P(v_v) = P_sat."""
    rho_lo, rho_hi = spinodal(T, a, b, R)
    P_max = pressure(rho_lo, T, a, b, R)   # local maximum (vapour spinodal)
    P_min = pressure(rho_hi, T, a, b, R)   # local minimum (liquid spinodal)
    lo = max(P_min, 1e-14 * abs(P_max)) * (1 + 1e-12)
    hi = P_max * (1 - 1e-12)

    def area(P):
        vl, vv = _volume_roots(P, T, a, b, R)
        integral = R * T * math.log((vv - b) / (vl - b)) + a / vv - a / vl
        return integral - P * (vv - vl)

    P_sat = optimize.brentq(area, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    vl, vv = _volume_roots(P_sat, T, a, b, R)
    return 1.0 / vl, 1.0 / vv, P_sat


def rankine_hugoniot(rho1, T1, Ma, a, b, R, cv):
    """Post-shock state behind a shock entering fluid 1 at rest.

    Shock speed u_s = Ma c_s(rho1, T1).  In the shock frame (w = u_s - u)
    mass, momentum and total enthalpy are continuous:
      rho1 w1 = rho2 w2,  P1 + rho1 w1^2 = P2 + rho2 w2^2,
      h1 + w1^2/2 = h2 + w2^2/2.
    Returns (rho2, T2, u2, P2, u_s) with u2 the lab-frame velocity behind it.
    """
    us = Ma * math.sqrt(cs2(rho1, T1, a, b, R, cv))
    P1 = pressure(rho1, T1, a, b, R)
    h1 = enthalpy(rho1, T1, a, b, R, cv)
    m = rho1 * us

    def res(x):
        rho2, T2 = x
        w2 = m / rho2
        return [P1 + m * us - pressure(rho2, T2, a, b, R) - m * w2,
                h1 + 0.5 * us * us - enthalpy(rho2, T2, a, b, R, cv) - 0.5 * w2 * w2]

    # ideal-gas estimate as the starting point
    g = 1.0 + R / cv
    r_ratio = (g + 1) * Ma * Ma / ((g - 1) * Ma * Ma + 2)
    p_ratio = 1 + 2 * g / (g + 1) * (Ma * Ma - 1)
    x0 = [rho1 * r_ratio, T1 * p_ratio / r_ratio]
    sol = optimize.fsolve(res, x0, xtol=1e-13, full_output=True)
    rho2, T2 = sol[0]
    if max(abs(v) for v in res([rho2, T2])) > 1e-12:
        raise RuntimeError("Rankine-Hugoniot solve did not converge")
    u2 = us * (1.0 - rho1 / rho2)
    return rho2, T2, u2, pressure(rho2, T2, a, b, R), us


def fundamental_derivative(rho, T, a, b, R, cv):
    """Gamma = 1 + (rho/c) (dc/drho)_s (eq. Gamma, its definition),
    evaluated by differentiating c along an isentrope numerically."""
    # isentrope of van der Waals: T (1/rho - b)^(R/cv) = const (from eq. ds_vdW)
    s_const = T * (1.0 / rho - b) ** (R / cv)

    def c_on_isentrope(r):
        Ti = s_const / (1.0 / r - b) ** (R / cv)
        return math.sqrt(cs2(r, Ti, a, b, R, cv))

    hstep = 1e-5 * rho
    dc = (c_on_isentrope(rho + hstep) - c_on_isentrope(rho - hstep)) / (2 * hstep)
    return 1.0 + rho / c_on_isentrope(rho) * dc


def fundamental_derivative_vdw(rho, P, a, b, R, cv):
    """Closed form of Gamma(P, rho) for van der Waals with constant c_v
    (Section 4.3, the expression after eq. Gamma).  The printed denominator
    reads 2 (R/c_v + 1) (P + a rho^2) / (1/rho - b) - 4 a rho^4, whose two
    terms differ in dimension by a density; differentiating the isentrope
    P + a rho^2 = K (1/rho - b)^-(1 + R/c_v) twice gives the first term with
    one more factor rho, which this function restores (it then reduces to
    (gamma + 1)/2 for the ideal gas and agrees with the definition)."""
    g = R / cv + 1.0
    v = 1.0 / rho
    Pa = P + a * rho * rho
    num = g * (g + 1.0) * Pa / (v - b) ** 2 - 6.0 * a * rho ** 4
    den = 2.0 * g * rho * Pa / (v - b) - 4.0 * a * rho ** 4
    return num / den


# -- exact Riemann solution of the ideal-gas Euler equations (gamma-law gas)
def riemann_star(rhoL, uL, pL, rhoR, uR, pR, gamma):
    """Star-region pressure and velocity of the ideal-gas Riemann problem
    (pressure function of the two non-linear waves, solved by Brent's method)."""
    cL = math.sqrt(gamma * pL / rhoL)
    cR = math.sqrt(gamma * pR / rhoR)

    def fk(p, rho, pk, ck):
        if p > pk:  # shock
            A = 2.0 / ((gamma + 1) * rho)
            B = (gamma - 1) / (gamma + 1) * pk
            return (p - pk) * math.sqrt(A / (p + B))
        # rarefaction
        return 2 * ck / (gamma - 1) * ((p / pk) ** ((gamma - 1) / (2 * gamma)) - 1)

    F = lambda p: fk(p, rhoL, pL, cL) + fk(p, rhoR, pR, cR) + (uR - uL)
    p_star = optimize.brentq(F, 1e-12, 100 * max(pL, pR), xtol=1e-15, rtol=1e-15)
    u_star = 0.5 * (uL + uR) + 0.5 * (fk(p_star, rhoR, pR, cR) - fk(p_star, rhoL, pL, cL))
    return p_star, u_star


def riemann_sample(rhoL, uL, pL, rhoR, uR, pR, gamma, xi):
    """Exact self-similar solution (rho, u, p) at xi = (x - x0)/t."""
    p_s, u_s = riemann_star(rhoL, uL, pL, rhoR, uR, pR, gamma)
    cL = math.sqrt(gamma * pL / rhoL)
    cR = math.sqrt(gamma * pR / rhoR)
    g = gamma
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    out = np.zeros((3, xi.size))
    for n, s in enumerate(xi):
        if s <= u_s:  # left of contact
            if p_s > pL:
                rho_s = rhoL * ((p_s / pL + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p_s / pL + 1))
                S = uL - cL * math.sqrt((g + 1) / (2 * g) * p_s / pL + (g - 1) / (2 * g))
                out[:, n] = (rhoL, uL, pL) if s < S else (rho_s, u_s, p_s)
            else:
                rho_s = rhoL * (p_s / pL) ** (1 / g)
                c_s = cL * (p_s / pL) ** ((g - 1) / (2 * g))
                head, tail = uL - cL, u_s - c_s
                if s < head:
                    out[:, n] = (rhoL, uL, pL)
                elif s > tail:
                    out[:, n] = (rho_s, u_s, p_s)
                else:
                    fac = 2 / (g + 1) + (g - 1) / ((g + 1) * cL) * (uL - s)
                    out[:, n] = (rhoL * fac ** (2 / (g - 1)),
                                 2 / (g + 1) * (cL + (g - 1) / 2 * uL + s),
                                 pL * fac ** (2 * g / (g - 1)))
        else:  # right of contact
            if p_s > pR:
                rho_s = rhoR * ((p_s / pR + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p_s / pR + 1))
                S = uR + cR * math.sqrt((g + 1) / (2 * g) * p_s / pR + (g - 1) / (2 * g))
                out[:, n] = (rho_s, u_s, p_s) if s < S else (rhoR, uR, pR)
            else:
                rho_s = rhoR * (p_s / pR) ** (1 / g)
                c_s = cR * (p_s / pR) ** ((g - 1) / (2 * g))
                head, tail = uR + cR, u_s + c_s
                if s > head:
                    out[:, n] = (rhoR, uR, pR)
                elif s < tail:
                    out[:, n] = (rho_s, u_s, p_s)
                else:
                    fac = 2 / (g + 1) - (g - 1) / ((g + 1) * cR) * (uR - s)
                    out[:, n] = (rhoR * fac ** (2 / (g - 1)),
                                 2 / (g + 1) * (-cR + (g - 1) / 2 * uR + s),
                                 pR * fac ** (2 * g / (g - 1)))
    return out
