"""Write ``paper_2510_14712_amd/workload_states.json``: the thermodynamic
states and constants of the five synthetic workloads, evaluated in FP64 by
the oracle's thermodynamics (Maxwell construction, Rankine-Hugoniot states,
sound speeds).  Run:  python -m oracle.make_workload_states

The workloads stand in for the paper's experiments (its shock tubes and
shock-liquid-column runs compare with external data that is not used here):
  1 D2Q9 512x4 van der Waals shock tube, FP64 (+ ideal-gas variant a = b = 0)
  2 D2Q9 2048x1024 shock-drop at T = 0.85 T_c, FP32
  3 D3Q27 256^3 near-critical Taylor-Green vortex, FP32
  4 D3Q27 384x256x256 shock-drop, surrogate EOS vs plain FP32
  5 D3Q27 512^3 Taylor-Green, BF16/FP16 deviation storage + surrogate EOS
Transport and capillarity constants are not given with the workloads; the
values below are the readings taken (lattice units): mu = eta = 0.05,
k = mu (c_v + R) (unit Prandtl number in the ideal limit), kappa = 0.01,
c_v = R / 0.4 (the nitrogen ratio R/c_v = 0.4 of the paper's Table 1).  The
512^3 Taylor-Green workload takes mu = eta = 0.1 (its entry's "mu", "eta",
"k"): at 0.05 (lattice Reynolds number about 1,370) that flow diverges after
about 350 of its 2000 steps; 0.1 halves the Reynolds number to that of the
256^3 workload at 0.05, which runs its 5000 steps.
"""
from __future__ import annotations

import json
import math
import os

from . import thermo as th

A, B, R = 3.0 / 49.0, 2.0 / 21.0, 1.0
CV = R / 0.4
MU = ETA = 0.05
K_TH = MU * (CV + R)
KAPPA = 0.01


def build():
    rc, Tc, Pc = th.critical(A, B, R)
    phys = dict(a=A, b=B, R=R, cv=CV, mu=MU, eta=ETA, k=K_TH, kappa=KAPPA)
    out = {"constants": phys, "critical": dict(rho=rc, T=Tc, P=Pc)}

    out["shock_tube_2d"] = dict(lattice=2, shape=[512, 4], bc=[1, 0, 0], steps=1000,
                                rho_left=0.9 * rc, rho_right=0.3 * rc, T=0.9 * Tc,
                                ideal=dict(a=0.0, b=0.0, kappa=0.0))

    T1 = 0.85 * Tc
    rl, rv, Ps = th.maxwell(T1, A, B, R)
    rho2, T2, u2, P2, us = th.rankine_hugoniot(rv, T1, 1.47, A, B, R, CV)
    drop = dict(T1=T1, rho_liquid=rl, rho_vapour=rv, P_sat=Ps, Ma=1.47, shock_speed=us,
                rho2=rho2, T2=T2, u2=u2, P2=P2, width=4.0)
    out["shock_drop_2d"] = dict(lattice=2, shape=[2048, 1024], bc=[1, 0, 0], steps=20000,
                                centre=[600, 512], radius=100, x_shock=200, **drop)
    out["shock_drop_3d"] = dict(lattice=3, shape=[384, 256, 256], bc=[1, 0, 0], steps=2000,
                                centre=[160, 128, 128], radius=48, x_shock=64, **drop,
                                mlp_tol=1e-6,
                                mlp_box=dict(rho=[0.05 * rc, 2.5 * rc], T=[0.8 * Tc, 1.5 * Tc]),
                                mlp_samples=1_000_000, mlp_seed=4)
    Ttgv = 1.1 * Tc
    cs = math.sqrt(th.cs2(rc, Ttgv, A, B, R, CV))
    out["tgv_3d_256"] = dict(lattice=3, shape=[256, 256, 256], bc=[0, 0, 0], steps=5000,
                             rho0=rc, T0=Ttgv, U0=0.5 * cs, cs=cs, noise=0.01, seed=3)
    out["tgv_3d_512"] = dict(lattice=3, shape=[512, 512, 512], bc=[0, 0, 0], steps=2000,
                             rho0=rc, T0=Ttgv, U0=0.5 * cs, cs=cs, noise=0.01, seed=5,
                             mu=2 * MU, eta=2 * ETA, k=2 * MU * (CV + R),
                             mlp_box=dict(rho=[0.05 * rc, 2.5 * rc], T=[0.8 * Tc, 1.5 * Tc]))
    # The paper's non-ideal shock tubes I-III (Section 4.3.1, its table of
    # cases): reduced states (P_r, rho_r) left / right of the mid-point and
    # R / c_v per case, on this van der Waals fluid in lattice units; 1000
    # cells along x (zero-gradient ends) as the paper's dx = L_x / 1000; run to
    # the times of its figures, t = t_r L_x sqrt(rho_c / P_c) with t_r = 0.45,
    # 0.2, 0.15 (readings: transport mu = eta = 0.05, k = mu (c_v + R),
    # kappa = 0.01 in lattice units; the paper's own are not given).
    cases = {"I": (0.0125, (1.09, 0.879), (0.885, 0.562), 0.45), "II": (0.329, (1.6077, 1.01), (0.8957, 0.594), 0.2),
             "III": (0.0125, (3.00, 1.818), (0.575, 0.275), 0.15)}
    for name, (rcv, (PLr, rLr), (PRr, rRr), tr) in cases.items():
        rl, rr = rLr * rc, rRr * rc
        TL = (PLr * Pc + A * rl * rl) * (1.0 - B * rl) / (rl * R)  # eq. Pvdw solved for T
        TR = (PRr * Pc + A * rr * rr) * (1.0 - B * rr) / (rr * R)
        cvc = R / rcv
        out["shock_tube_" + name] = dict(lattice=2, shape=[1000, 4], bc=[1, 0, 0], R_over_cv=rcv, cv=cvc,
                                         rho_left=rl, T_left=TL, rho_right=rr, T_right=TR, t_reduced=tr,
                                         steps=int(round(tr * 1000 * math.sqrt(rc / Pc))), mu=MU, eta=ETA,
                                         k=MU * (cvc + R))
    # Peng-Robinson fluid for the iterative caloric inversion (Section 3.2,
    # after eq. lbm_temp): Peng & Robinson's published coefficients
    # a = 0.45724 R^2 Tc^2 / Pc, b = 0.07780 R Tc / Pc and
    # m = 0.37464 + 1.54226 omega - 0.26992 omega^2, here with the van der
    # Waals fluid's T_c, P_c = Z_c rho_c R T_c at Z_c = 0.3074 and rho_c = 3.5
    # (so both fluids share the critical state), acentric factor omega = 0.2,
    # and a temperature-dependent ideal-gas heat capacity c_v0 = c0 + c1 T
    # with c0 = 2.0, c1 = 5.0 (readings: the paper names the equation of state
    # only).
    om = 0.2
    Pc_pr = 0.3074 * rc * R * Tc
    out["peng_robinson"] = dict(a=0.45724 * R * R * Tc * Tc / Pc_pr, b=0.07780 * R * Tc / Pc_pr, R=R,
                                m=0.37464 + 1.54226 * om - 0.26992 * om * om, Tc=Tc, Pc=Pc_pr, rho_c=rc,
                                c0=2.0, c1=5.0, omega=om, Zc=0.3074)
    return out


def main():
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2510_14712_amd", "workload_states.json")
    with open(path, "w") as fh:
        json.dump(build(), fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
