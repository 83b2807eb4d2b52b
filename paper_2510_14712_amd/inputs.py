"""Seeded synthetic initial conditions (rho, u, T) for the lattice Boltzmann step.

This module holds no arithmetic of the method itself: it only draws seeded
random numbers and lays out piecewise-constant, tanh-interface, Taylor-Green
and smooth-noise fields from state constants it is given.  Thermodynamic
states that need the equation of state (Maxwell coexistence densities,
Rankine-Hugoniot post-shock states, sound speeds) are read from
``workload_states.json``, a table written once by a script that evaluates
them in FP64 (``oracle/make_workload_states.py``).

Layout of every returned field: numpy float64, C order, cell index
idx = x + nx (y + ny z); vector fields are (D, N) flattened component-major.
"""
from __future__ import annotations

import json
import os

import numpy as np

_STATES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workload_states.json")


def states() -> dict:
    with open(_STATES) as fh:
        return json.load(fh)


def physics(st: dict, workload: str | None = None) -> dict:
    """Lattice-unit constants (a, b, R, cv, mu, eta, k, kappa) of a workload:
    the shared constants, with the transport coefficients a workload entry
    gives in place of the shared ones."""
    kw = {k: st["constants"][k] for k in ("a", "b", "R", "cv", "mu", "eta", "k", "kappa")}
    if workload is not None:
        for k in ("cv", "mu", "eta", "k"):
            if k in st[workload]:
                kw[k] = st[workload][k]
    return kw


def grid(shape):
    """Integer coordinate arrays (x, y[, z]) of a lattice, x fastest."""
    if len(shape) == 2:
        nx, ny = shape
        y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        return x.reshape(-1), y.reshape(-1)
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def smooth_noise(shape, seed, modes=3, amp=1.0):
    """Sum of random low-wavenumber Fourier modes, periodic, max |value| <= amp."""
    rng = np.random.default_rng(seed)
    coords = grid(shape)
    out = np.zeros(coords[0].size)
    for _ in range(modes):
        phase = rng.uniform(0, 2 * np.pi)
        arg = phase
        for ax, c in enumerate(coords):
            k = rng.integers(0, 3)
            arg = arg + 2 * np.pi * k * c / shape[ax]
        out += rng.uniform(-1, 1) * np.cos(arg)
    return amp * out / max(modes, 1)


def random_state(D, shape, seed, rho0, T0, drho=0.02, du=0.05, dT=0.02, white=0.0):
    """Smooth random (rho, u, T) around (rho0, 0, T0): relative density and
    temperature perturbations drho, dT, velocity amplitude du; optional white
    noise of relative amplitude ``white`` on the density (exercises every
    stencil entry)."""
    N = int(np.prod(shape))
    rho = rho0 * (1.0 + smooth_noise(shape, seed, amp=drho))
    if white:
        rho *= 1.0 + white * np.random.default_rng(seed + 1000).uniform(-1, 1, N)
    u = np.concatenate([smooth_noise(shape, seed + 10 + a, amp=du) for a in range(D)])
    T = T0 * (1.0 + smooth_noise(shape, seed + 20, amp=dT))
    return rho, u, T


def shock_tube(shape, rho_left, rho_right, T, x_split=None, T_right=None):
    """Piecewise-constant Riemann data at rest: rho = rho_left (and T) for
    x < x_split, rho_right (and T_right, default T) beyond."""
    coords = grid(shape)
    x = coords[0]
    xs = shape[0] // 2 if x_split is None else x_split
    rho = np.where(x < xs, rho_left, rho_right).astype(np.float64)
    u = np.zeros(len(shape) * x.size)
    Tf = np.where(x < xs, float(T), float(T if T_right is None else T_right)).astype(np.float64)
    return rho, u, Tf


def shock_drop(shape, centre, radius, width, rho_liquid, rho_vapour, T1,
               x_shock, rho2, T2, u2):
    """Liquid drop (2-D disc or 3-D sphere) with a tanh interface of the given
    width in coexisting vapour; the region x < x_shock holds the post-shock
    state (rho2, T2, u2 along +x)."""
    coords = grid(shape)
    D = len(shape)
    r = np.sqrt(sum((c - centre[a]) ** 2 for a, c in enumerate(coords)).astype(np.float64))
    rho = 0.5 * (rho_liquid + rho_vapour) + 0.5 * (rho_liquid - rho_vapour) * np.tanh(2.0 * (radius - r) / width)
    T = np.full(r.size, float(T1))
    u = np.zeros(D * r.size)
    post = coords[0] < x_shock
    rho[post] = rho2
    T[post] = T2
    u[: r.size][post] = u2
    return rho, u, T


def taylor_green(shape, seed, rho0, T0, U0, noise=0.01):
    """3-D Taylor-Green vortex u = U0 (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0),
    k = 2 pi / n per axis, uniform T0, density rho0 (1 + noise xi), xi ~ U[-1, 1]
    drawn by numpy's PCG64 with the given seed in C order [z][y][x]."""
    nx, ny, nz = shape
    x, y, z = grid(shape)
    kx, ky, kz = 2 * np.pi * x / nx, 2 * np.pi * y / ny, 2 * np.pi * z / nz
    ux = U0 * np.sin(kx) * np.cos(ky) * np.cos(kz)
    uy = -U0 * np.cos(kx) * np.sin(ky) * np.cos(kz)
    uz = np.zeros_like(ux)
    xi = np.random.default_rng(seed).uniform(-1.0, 1.0, x.size)
    rho = rho0 * (1.0 + noise * xi)
    return rho, np.concatenate([ux, uy, uz]), np.full(x.size, float(T0))


def mlp_samples(n, seed, rho_range, T_range):
    """Uniform (rho, T) samples for surrogate training / evaluation."""
    rng = np.random.default_rng(seed)
    return rng.uniform(*rho_range, n), rng.uniform(*T_range, n)


def mlp_params(seed, scale=1.0):
    """Random MLP parameters (Glorot-uniform) in the flat layout
    W1[64x2], b1[64], W2[64x64], b2[64], W3[3x64], b3[3] (4547 values)."""
    rng = np.random.default_rng(seed)

    def glorot(fan_out, fan_in):
        lim = scale * np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, fan_out * fan_in)

    return np.concatenate([glorot(64, 2), np.zeros(64), glorot(64, 64), np.zeros(64),
                           glorot(3, 64), np.zeros(3)])
