"""Physics pins of the full oracle scheme (Section 4 of the paper).

Each test runs the oracle on a small pseudo-1-D lattice and compares a
measured quantity with a closed form the paper states:
  * shear-wave decay rate k^2 mu/rho (Section 4.1, shear dissipation), with
    and without a mean flow (Galilean invariance);
  * acoustic (normal-mode) energy decay exp(-k^2 sigma t),
    sigma = 2(D-1)/D mu/rho + eta/rho + k/(rho c_p)(c_p/c_v - 1)
    (Section 4.1, normal-mode dissipation), with and without a mean flow
    along the wave -- this exercises the Galilean correction Phi and the
    bulk-viscosity shift alpha;
  * thermal decay rate k^2 k_th/(rho c_p) at uniform pressure (Section 4.1,
    thermal conductivity) -- this exercises the heat-flux correction q^c;
  * sound speed of a weak pressure front against eq. vdW_speed_of_sound on
    both saturated branches (Section 4.1, speed of sound);
  * coexistence densities of a liquid slab against Maxwell's rule
    (Section 4.2);
  * the ideal-gas Riemann problem (a = b = 0) against the exact solution;
  * a D3Q27 run uniform in z equals the D2Q9 run after summing over c_z when
    the bulk viscosities are chosen so that alpha (eq. corr_bulk) agrees.
"""
import numpy as np
import pytest

import oracle
from oracle import thermo as th
from paper_2510_14712_amd import inputs

A, B, R, CV = 3.0 / 49.0, 2.0 / 21.0, 1.0, 2.5
RHOC, TC, PC = th.critical(A, B, R)


def _mode_amp(v, nx, k=1):
    """|Fourier coefficient| of a 1-D profile at wavenumber index k."""
    return np.abs(np.fft.rfft(v)[k]) * 2 / nx


def _fit_rate(t, y):
    return -np.polyfit(t, np.log(y), 1)[0]


@pytest.mark.parametrize("U", [(0.0, 0.0), (0.0, 0.1), (0.15, 0.0)])
def test_shear_wave_decay(U):
    nx = 32
    p = oracle.Params(2, (nx, 1), mu=0.05, eta=0.05)
    rho0, T0 = RHOC, 1.1 * TC
    x = np.arange(nx)
    k = 2 * np.pi / nx
    ux = np.full(nx, U[0])
    uy = U[1] + 1e-3 * np.sin(k * x)
    f, g = oracle.init(p, np.full(nx, rho0), np.concatenate([ux, uy]), np.full(nx, T0))
    f, g = oracle.run(p, f, g, 50)
    ts, amps = [], []
    for s in range(6):
        f, g = oracle.run(p, f, g, 100)
        fl = oracle.fields(p, f, g)
        ts.append(50 + 100 * (s + 1))
        amps.append(_mode_amp(fl["u"][nx:], nx))
    nu = _fit_rate(np.array(ts), np.array(amps)) / k ** 2
    assert abs(nu / (p.mu / rho0) - 1) < 0.02


def _isentropic_wave(nx, rho0, T0, eps):
    """Density sin perturbation with T on the van der Waals isentrope
    T (1/rho - b)^(R/c_v) = const (from eq. ds_vdW)."""
    x = np.arange(nx)
    rho = rho0 * (1 + eps * np.sin(2 * np.pi * x / nx))
    T = T0 * ((1 / rho0 - B) / (1 / rho - B)) ** (R / CV)
    return rho, T


@pytest.mark.parametrize("Ux", [0.0, 0.1])
def test_normal_mode_dissipation(Ux):
    nx = 48
    mu, eta = 0.03, 0.04
    p = oracle.Params(2, (nx, 1), mu=mu, eta=eta)
    rho0, T0 = RHOC, 1.2 * TC
    rho, T = _isentropic_wave(nx, rho0, T0, 1e-4)
    u = np.concatenate([np.full(nx, Ux), np.zeros(nx)])
    f, g = oracle.init(p, rho, u, T)
    c2 = th.cs2(rho0, T0, A, B, R, CV)
    cp = th.cp(rho0, T0, A, B, R, CV)
    ts, es = [], []
    per = 2
    for s in range(60):
        f, g = oracle.run(p, f, g, per)
        fl = oracle.fields(p, f, g)
        du = fl["u"][:nx] - Ux
        dr = fl["rho"] - rho0
        es.append(0.5 * np.sum(rho0 * (du ** 2 + fl["u"][nx:] ** 2) + dr ** 2 * c2 / rho0))
        ts.append(per * (s + 1))
    ts, es = np.array(ts), np.array(es)
    k = 2 * np.pi / nx
    sigma = _fit_rate(ts[10:], es[10:]) / k ** 2
    sigma_ref = 2 * (2 - 1) / 2 * mu / rho0 + eta / rho0 + p.k / (rho0 * cp) * (cp / CV - 1)
    assert abs(sigma / sigma_ref - 1) < 0.04


@pytest.mark.parametrize("Ux", [0.0, 0.1])
def test_thermal_decay(Ux):
    """Uniform pressure, density wave: T decays at k^2 k_th/(rho c_p).
    With k_th != mu c_p this separates the Fourier flux (q^c present) from the
    enthalpy-gradient flux the BGK part alone would give (Section 3.1 remark 3)."""
    nx = 64
    kth, mu = 0.2, 0.05
    p = oracle.Params(2, (nx, 1), mu=mu, eta=mu, k=kth)
    rho0, T0 = 2.0, 1.5 * TC
    cp = th.cp(rho0, T0, A, B, R, CV)
    assert abs(mu * cp / kth - 1) > 0.15
    P0 = th.pressure(rho0, T0, A, B, R)
    x = np.arange(nx)
    rho = rho0 * (1 + 1e-3 * np.sin(2 * np.pi * x / nx))
    T = (P0 + A * rho ** 2) * (1 - B * rho) / (rho * R)  # T(rho, P0) from eq. Pvdw
    u = np.concatenate([np.full(nx, Ux), np.zeros(nx)])
    f, g = oracle.init(p, rho, u, T)
    k = 2 * np.pi / nx
    tau = int(1.0 / (k * k * kth / (rho0 * cp)))
    f, g = oracle.run(p, f, g, tau // 4)
    ts, amps = [], []
    for s in range(8):
        f, g = oracle.run(p, f, g, tau // 8)
        fl = oracle.fields(p, f, g)
        ts.append(tau // 4 + tau // 8 * (s + 1))
        amps.append(_mode_amp(fl["T"] - fl["T"].mean(), nx))
    D_th = _fit_rate(np.array(ts), np.array(amps)) / k ** 2
    assert abs(D_th / (kth / (rho0 * cp)) - 1) < 0.01


@pytest.mark.parametrize("branch", ["vapour", "liquid"])
def test_sound_speed_saturated(branch):
    Tr = 0.9
    rl, rv, _ = th.maxwell(Tr * TC, A, B, R)
    rho0 = rl if branch == "liquid" else rv
    T0 = Tr * TC
    nx = 400
    p = oracle.Params(2, (nx, 1), bc=(1, 0, 0), mu=0.02, eta=0.02, kappa=0.0)
    x = np.arange(nx)
    # weak isentropic step: pressure front pair, density jump eps
    eps = 2e-3
    rho = np.where(x < nx // 2, rho0, rho0 * (1 + eps))
    T = T0 * ((1 / rho0 - B) / (1 / rho - B)) ** (R / CV)
    f, g = oracle.init(p, rho, np.zeros(2 * nx), T)
    c = np.sqrt(th.cs2(rho0, T0, A, B, R, CV))

    def front(fl):
        # left-moving front: position where the density crosses the mean of
        # the two plateaus on the left half
        d = fl["rho"][: nx // 2 + 5]
        lo, hi = rho0, rho0 * (1 + eps / 2)
        mid = 0.5 * (lo + hi)
        i = np.nonzero(d > mid)[0][0]
        return i - 1 + (mid - d[i - 1]) / (d[i] - d[i - 1])

    t1, t2 = 60, 160
    f, g = oracle.run(p, f, g, t1)
    x1 = front(oracle.fields(p, f, g))
    f, g = oracle.run(p, f, g, t2 - t1)
    x2 = front(oracle.fields(p, f, g))
    speed = (x1 - x2) / (t2 - t1)
    assert abs(speed / c - 1) < 0.01


def test_coexistence_maxwell():
    Tr = 0.9
    rl, rv, _ = th.maxwell(Tr * TC, A, B, R)
    nx = 160
    p = oracle.Params(2, (nx, 1), mu=0.05, eta=0.05, kappa=0.02)
    x = np.arange(nx)
    r = np.abs(x - nx / 2 + 0.5)
    rho = 0.5 * (rl + rv) + 0.5 * (rl - rv) * np.tanh(2 * (40 - r) / 4.0)
    f, g = oracle.init(p, rho, np.zeros(2 * nx), np.full(nx, Tr * TC))
    f, g = oracle.run(p, f, g, 6000)
    fl = oracle.fields(p, f, g)
    # both bulk phases at (nearly) one temperature; compare with Maxwell there
    T_l, T_v = fl["T"][nx // 2], fl["T"][0]
    assert abs(T_l / T_v - 1) < 2e-3
    rl_t, _, _ = th.maxwell(T_l, A, B, R)
    _, rv_t, _ = th.maxwell(T_v, A, B, R)
    assert abs(fl["rho"][nx // 2] / rl_t - 1) < 0.01
    assert abs(fl["rho"][0] / rv_t - 1) < 0.01


def test_ideal_gas_riemann():
    nx = 512
    p = oracle.Params(2, (nx, 1), bc=(1, 0, 0), a=0.0, b=0.0, mu=0.02, eta=0.02, kappa=0.0,
                      k=0.02 * (CV + R))
    T0 = 0.9 * TC
    rho, u, T = inputs.shock_tube((nx, 1), 3.15, 1.05, T0)
    f, g = oracle.init(p, rho, u, T)
    t = 200
    f, g = oracle.run(p, f, g, t)
    fl = oracle.fields(p, f, g)
    gamma = 1 + R / CV
    xc = np.arange(nx) + 0.5 - nx / 2
    ex = th.riemann_sample(3.15, 0, 3.15 * T0, 1.05, 0, 1.05 * T0, gamma, xc / t)
    err = np.abs(fl["rho"] - ex[0]).sum() / np.abs(3.15 - 1.05) / nx
    assert err < 0.01
    p_star, u_star = th.riemann_star(3.15, 0, 3.15 * T0, 1.05, 0, 1.05 * T0, gamma)
    # plateau between the rarefaction tail and the shock: pressure and velocity
    i0 = nx // 2 + int(0.3 * u_star * t)
    i1 = nx // 2 + int(0.8 * u_star * t)
    assert abs(np.mean(fl["P"][i0:i1]) / p_star - 1) < 0.01
    assert abs(np.mean(fl["u"][:nx][i0:i1]) / u_star - 1) < 0.02


def test_d3q27_z_uniform_equals_d2q9():
    shape2 = (12, 10)
    nz = 3
    mu, eta2 = 0.05, 0.05
    eta3 = eta2 - mu / 3.0  # equal alpha: (D+2)/D - eta/mu agrees for D = 2, 3
    p2 = oracle.Params(2, shape2, mu=mu, eta=eta2)
    p3 = oracle.Params(3, shape2 + (nz,), mu=mu, eta=eta3)
    rho, u, T = inputs.random_state(2, shape2, 31, RHOC, 1.1 * TC, drho=0.03, du=0.06, dT=0.02)
    N2 = rho.size
    rho3, T3 = np.tile(rho, nz), np.tile(T, nz)
    u3 = np.concatenate([np.tile(u[:N2], nz), np.tile(u[N2:], nz), np.zeros(N2 * nz)])
    f2, g2 = oracle.run(p2, *oracle.init(p2, rho, u, T), 20)
    f3, g3 = oracle.run(p3, *oracle.init(p3, rho3, u3, T3), 20)
    c3 = oracle.velocities(3)
    c2 = oracle.velocities(2)
    F3 = f3.reshape(27, nz, N2)[:, 0]
    G3 = g3.reshape(27, nz, N2)[:, 0]
    for i in range(9):
        sel = (c3[:, 0] == c2[i, 0]) & (c3[:, 1] == c2[i, 1])
        np.testing.assert_allclose(F3[sel].sum(0), f2.reshape(9, N2)[i], rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(G3[sel].sum(0), g2.reshape(9, N2)[i], rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("side", ["positive", "negative", "dead_zone"])
def test_upwind_orientation_of_phi(axis, side):
    """Phi_aa = -(1/rho) d_a Lambda_a with the difference biased by sgn(u_a)
    (Section 3.2, the upwind formula after eq. correction): u_a > 0 takes
    the backward difference Lambda(x) - Lambda(x - e_a), u_a < 0 the forward
    difference Lambda(x + e_a) - Lambda(x), |u_a| inside the dead zone the
    central average.  Uniform density and temperature (so F = 0 and theta
    is uniform), u_a linear along the axis (a sine inside the dead zone):
    Lambda_a = rho u^3 + 3 rho u (theta - 1/3) is then non-linear there, and
    the three differences differ by far more than the tolerance.  Lambda is computed here from the imposed
    u and the van der Waals theta, not taken from the oracle."""
    n = 24
    shape = [3, 3, 3]
    shape[axis] = n
    bc = [0, 0, 0]
    bc[axis] = 1
    p = oracle.Params(3, tuple(shape), bc=tuple(bc))
    N = int(np.prod(shape))
    coords = inputs.grid(tuple(shape))
    s = coords[axis].astype(np.float64)
    rho0, T0 = RHOC, 1.1 * TC
    if side == "dead_zone":
        ua = 7e-7 * np.sin(2 * np.pi * s / n)  # |u| < 1e-6, the dead zone
    else:
        ua = (0.05 + 0.01 * s) * (1.0 if side == "positive" else -1.0)
    u = np.zeros(3 * N)
    u[axis * N:(axis + 1) * N] = ua
    f, g = oracle.init(p, np.full(N, rho0), u, np.full(N, T0))
    _, _, fl = oracle.collide(p, f, g)
    theta = th.pressure(rho0, T0, A, B, R) / rho0
    lam = rho0 * ua ** 3 + 3.0 * rho0 * ua * (theta - 1.0 / 3.0)
    phi = fl["Phi"][axis * N:(axis + 1) * N]
    stride = [1, shape[0], shape[0] * shape[1]][axis]
    inner = [c for c in range(N) if 0 < coords[axis][c] < n - 1]
    back = np.array([lam[c] - lam[c - stride] for c in inner])
    fwd = np.array([lam[c + stride] - lam[c] for c in inner])
    expect = {"positive": back, "negative": fwd, "dead_zone": 0.5 * (back + fwd)}[side]
    got = -phi[inner] * rho0
    scale = np.abs(expect).max()
    assert np.abs(got - expect).max() <= 1e-9 * scale + 1e-15  # + round-off of u from the moments
    # the test can tell the orientations apart
    assert np.abs(back - fwd).max() > 1e-2 * scale
    # the other axes carry no correction (u is zero along them)
    for b in range(3):
        if b != axis:
            assert np.abs(fl["Phi"][b * N:(b + 1) * N]).max() <= 1e-13
