"""FP64 CPU oracle of the non-ideal compressible DDF lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, obviously-correct
implementation written from arXiv 2510.14712 (Section 3.2 and the flowchart
figure closing it; thermodynamics of Section 2; experiments of Section 4).
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the GPU library.

Modules:
  * this package: ctypes binding of ``liblbm_oracle.so`` (the C step).
  * ``oracle.thermo``: van der Waals thermodynamics, Maxwell construction,
    Rankine-Hugoniot states and the exact ideal-gas Riemann solution.
  * ``oracle.mlp``: FP64 reference of the MLP equation-of-state surrogate
    (forward, backward, Adam step) and the FP32 -> BF16/FP16 encoders.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbm_oracle.so")
_SRC = os.path.join(_HERE, "lbm_oracle.c")


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("bc", ctypes.c_int * 3),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
                ("cv", ctypes.c_double), ("mu", ctypes.c_double), ("eta", ctypes.c_double),
                ("k", ctypes.c_double), ("kappa", ctypes.c_double), ("upwind_eps", ctypes.c_double),
                ("sc_cmu", ctypes.c_double), ("sc_ceta", ctypes.c_double), ("sc_ck", ctypes.c_double),
                ("eos", ctypes.c_int), ("pr_m", ctypes.c_double), ("pr_Tc", ctypes.c_double),
                ("pr_c0", ctypes.c_double), ("pr_c1", ctypes.c_double),
                ("wall_u", (ctypes.c_double * 3) * 2), ("wall_T", ctypes.c_double * 2)]


_DP = ctypes.POINTER(ctypes.c_double)


class _Fields(ctypes.Structure):
    _fields_ = [(n, _DP) for n in ("rho", "u", "E", "T", "P", "theta", "h", "cs2",
                                    "F", "Lambda", "lap", "Phi", "mu_num", "eta_num", "k_num")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        PP = ctypes.POINTER(_Params)
        L.oracle_init.argtypes = [PP, _DP, _DP, _DP, _DP, _DP]
        L.oracle_fields_eval.argtypes = [PP, _DP, _DP, ctypes.POINTER(_Fields)]
        L.oracle_collide.argtypes = [PP, _DP, _DP, _DP, _DP, ctypes.POINTER(_Fields)]
        L.oracle_stream.argtypes = [PP, _DP, _DP, _DP, _DP]
        L.oracle_run.argtypes = [PP, _DP, _DP, ctypes.c_int]
        L.oracle_feq.argtypes = [ctypes.c_int, ctypes.c_double, _DP, ctypes.c_double, _DP]
        L.oracle_feq.restype = None
        L.oracle_geq.argtypes = [ctypes.c_int, ctypes.c_double, _DP, ctypes.c_double,
                                 ctypes.c_double, _DP]
        L.oracle_geq.restype = None
        L.oracle_operator_moments.argtypes = [ctypes.c_int, _DP, ctypes.c_double,
                                              ctypes.c_double, _DP]
        L.oracle_operator_moments.restype = None
        for fn in ("oracle_init", "oracle_fields_eval", "oracle_collide", "oracle_stream",
                   "oracle_run", "oracle_num_threads"):
            getattr(L, fn).restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        L.oracle_eos.argtypes = [PP, ctypes.c_double, ctypes.c_double, _DP]
        L.oracle_eos.restype = None
        L.oracle_temperature.argtypes = [PP, ctypes.c_double, ctypes.c_double, _DP]
        L.oracle_temperature.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


# |u| at or below this takes the central average in the upwind-biased
# derivative of the Galilean correction (the tie sgn(0) = 0 widened to a
# round-off dead zone)
UPWIND_EPS = 1e-6


def num_vel(D: int) -> int:
    return 9 if D == 2 else 27


def velocities(D: int) -> np.ndarray:
    """c_i for i = (c_x+1) + 3(c_y+1) [+ 9(c_z+1)] (eq. D3Q27c ordering)."""
    Q = num_vel(D)
    c = np.zeros((Q, D), dtype=np.int64)
    for i in range(Q):
        c[i, 0] = i % 3 - 1
        c[i, 1] = (i // 3) % 3 - 1
        if D == 3:
            c[i, 2] = i // 9 - 1
    return c


class Params:
    """Lattice and physical parameters (lattice units)."""

    def __init__(self, D, shape, bc=(0, 0, 0), a=3.0 / 49.0, b=2.0 / 21.0, R=1.0, cv=2.5,
                 mu=0.05, eta=0.05, k=None, kappa=0.01, upwind_eps=UPWIND_EPS, sc=(0.0, 0.0, 0.0), pr=None,
                 walls=None):
        nx, ny = shape[0], shape[1]
        nz = shape[2] if D == 3 else 1
        self.D, self.nx, self.ny, self.nz = D, nx, ny, nz
        self.bc = tuple(bc)
        self.a, self.b, self.R, self.cv = a, b, R, cv
        self.mu, self.eta = mu, eta
        self.k = mu * (cv + R) if k is None else k
        self.kappa = kappa
        self.upwind_eps = upwind_eps
        # shock-capturing coefficients (C_mu, C_eta, C_k) of Section 4.4; zeros: off
        self.sc = tuple(float(v) for v in sc)
        # walls (bc 2 on x): ((u_lo, T_lo), (u_hi, T_hi)) with u a D-vector
        self.walls = walls
        # Peng-Robinson: dict(m, Tc, c0, c1) with a, b, R its constants; None: van der Waals
        self.pr = dict(pr) if pr is not None else None
        if self.pr is not None:
            self.k = mu * (self.pr["c0"] + R) if k is None else k

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    @property
    def Q(self):
        return num_vel(self.D)

    def c_struct(self):
        s = _Params()
        s.D, s.nx, s.ny, s.nz = self.D, self.nx, self.ny, self.nz
        for i in range(3):
            s.bc[i] = int(self.bc[i])
        s.a, s.b, s.R, s.cv = self.a, self.b, self.R, self.cv
        s.mu, s.eta, s.k, s.kappa = self.mu, self.eta, self.k, self.kappa
        s.upwind_eps = self.upwind_eps
        s.sc_cmu, s.sc_ceta, s.sc_ck = self.sc
        if self.walls is not None:
            for side, (uw, Tw) in enumerate(self.walls):
                for a, v in enumerate(uw):
                    s.wall_u[side][a] = float(v)
                s.wall_T[side] = float(Tw)
        if self.pr is not None:
            s.eos = 1
            s.pr_m, s.pr_Tc, s.pr_c0, s.pr_c1 = (float(self.pr[k]) for k in ("m", "Tc", "c0", "c1"))
        return s


def init(p: Params, rho, u, T):
    """f = f^eq, g = g^eq from (rho, u, T) fields (flowchart: initialise)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
    assert rho.size == p.N and u.size == p.D * p.N and T.size == p.N
    f = np.zeros(p.Q * p.N)
    g = np.zeros(p.Q * p.N)
    rc = lib().oracle_init(ctypes.byref(p.c_struct()), _ptr(rho), _ptr(u), _ptr(T),
                           _ptr(f), _ptr(g))
    if rc != 0:
        raise ValueError(f"oracle_init failed ({rc})")
    return f, g


def _alloc_fields(p: Params):
    N, D = p.N, p.D
    arrs = {n: np.zeros(N) for n in ("rho", "E", "T", "P", "theta", "h", "cs2", "lap", "mu_num", "eta_num",
                                      "k_num")}
    for n in ("u", "F", "Lambda", "Phi"):
        arrs[n] = np.zeros(D * N)
    s = _Fields()
    for n, a in arrs.items():
        setattr(s, n, _ptr(a))
    return arrs, s


def fields(p: Params, f, g):
    """Macroscopic fields of the state (rho, u, E, T, P, theta, h, cs2, F, ...,
    and the shock-capturing numerical transport mu_num, eta_num, k_num)."""
    arrs, s = _alloc_fields(p)
    rc = lib().oracle_fields_eval(ctypes.byref(p.c_struct()), _ptr(f), _ptr(g), ctypes.byref(s))
    if rc != 0:
        raise ValueError("oracle_fields_eval failed")
    return arrs


def collide(p: Params, f, g):
    """Post-collision populations at each cell (no streaming) and the fields
    used, with the upwind Galilean correction Phi_aa of each cell."""
    fp = np.zeros_like(f)
    gp = np.zeros_like(g)
    arrs, s = _alloc_fields(p)
    rc = lib().oracle_collide(ctypes.byref(p.c_struct()), _ptr(f), _ptr(g), _ptr(fp), _ptr(gp),
                              ctypes.byref(s))
    if rc != 0:
        raise ValueError("oracle_collide failed")
    return fp, gp, arrs


def stream(p: Params, fpost, gpost):
    f = np.zeros_like(fpost)
    g = np.zeros_like(gpost)
    rc = lib().oracle_stream(ctypes.byref(p.c_struct()), _ptr(fpost), _ptr(gpost), _ptr(f), _ptr(g))
    if rc != 0:
        raise ValueError("oracle_stream failed")
    return f, g


def run(p: Params, f, g, nsteps: int):
    """Advance (f, g) by nsteps full steps; returns new arrays."""
    f = np.array(f, dtype=np.float64, copy=True)
    g = np.array(g, dtype=np.float64, copy=True)
    rc = lib().oracle_run(ctypes.byref(p.c_struct()), _ptr(f), _ptr(g), int(nsteps))
    if rc != 0:
        raise ValueError("oracle_run failed")
    return f, g


def feq(D, rho, u, theta):
    out = np.zeros(num_vel(D))
    uu = np.ascontiguousarray(u, dtype=np.float64)
    lib().oracle_feq(D, float(rho), _ptr(uu), float(theta), _ptr(out))
    return out


def geq(D, rho, u, e, theta):
    out = np.zeros(num_vel(D))
    uu = np.ascontiguousarray(u, dtype=np.float64)
    lib().oracle_geq(D, float(rho), _ptr(uu), float(e), float(theta), _ptr(out))
    return out


def operator_moments(D, u, e, theta):
    out = np.zeros(27)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    lib().oracle_operator_moments(D, _ptr(uu), float(e), float(theta), _ptr(out))
    return out[: 3 ** D]


def eos(p: Params, rho: float, T: float) -> dict:
    """The parameters' equation of state at (rho, T): P, e, c_v, c_s^2, (dP/dT)_rho."""
    out = np.zeros(5)
    lib().oracle_eos(ctypes.byref(p.c_struct()), float(rho), float(T), _ptr(out))
    return dict(zip(("P", "e", "cv", "cs2", "dPdT"), out))


def temperature(p: Params, rho: float, e: float):
    """Caloric inversion T(rho, e) and the Newton iterations it took (0 when
    explicit, -1 when not converged)."""
    t = ctypes.c_double()
    it = lib().oracle_temperature(ctypes.byref(p.c_struct()), float(rho), float(e), ctypes.byref(t))
    return t.value, it


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's loops over cells (OpenMP)."""
    lib().oracle_set_num_threads(int(n))
