"""Write ``tests/golden/tgv64_mu0.1_2000.npz``: the FP64 oracle's fields after
2000 steps of the D3Q27 near-critical Taylor-Green vortex on a 64^3 periodic
lattice, the error reference of the 512^3 reduced-precision workload (same
recipe and lattice-unit parameters, reduced size).

Recipe (seeded; ``paper_2510_14712_amd/inputs.py`` draws the inputs and holds
none of the method's arithmetic): rho = rho_c (1 + 0.01 xi), xi ~ U[-1, 1]
(numpy PCG64, seed 5, C order [z][y][x]); u = U0 (sin kx cos ky cos kz,
-cos kx sin ky cos kz, 0), k = 2 pi / 64, U0 = c_s(rho_c, 1.1 T_c) / 2; T =
1.1 T_c.  Van der Waals a = 3/49, b = 2/21, R = 1, c_v = 2.5, kappa = 0.01;
mu = eta = 0.1 and k = mu (c_v + R): the viscosity at which the 512^3 flow
runs its 2000 steps.

Only ``oracle/`` computes the stored values.  Fields are stored as float32
(rho, u_x, u_y, u_z, T), far below the error bars they serve.  Run:
    python -m oracle.make_tgv64_reference            (about 15 min on 8 threads)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "tests", "golden", "tgv64_mu0.1_2000.npz")
SHAPE = (64, 64, 64)
STEPS = 2000
MU = 0.1
SEED = 5


def params():
    import oracle
    from paper_2510_14712_amd import inputs
    c = inputs.states()["constants"]
    return oracle.Params(3, SHAPE, a=c["a"], b=c["b"], R=c["R"], cv=c["cv"], mu=MU, eta=MU,
                         k=MU * (c["cv"] + c["R"]), kappa=c["kappa"])


def initial_state():
    from paper_2510_14712_amd import inputs
    st = inputs.states()
    t = st["tgv_3d_512"]
    return inputs.taylor_green(SHAPE, SEED, t["rho0"], t["T0"], t["U0"], t["noise"])


def main():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import oracle
    p = params()
    rho, u, T = initial_state()
    f, g = oracle.init(p, rho, u, T)
    t0 = time.time()
    for k in range(STEPS // 100):
        f, g = oracle.run(p, f, g, 100)
        print(f"step {100 * (k + 1)}  {time.time() - t0:.0f} s", flush=True)
    fl = oracle.fields(p, f, g)
    np.savez_compressed(OUT, rho=fl["rho"].astype(np.float32), u=fl["u"].astype(np.float32),
                        T=fl["T"].astype(np.float32), steps=np.int64(STEPS), mu=np.float64(MU),
                        seed=np.int64(SEED), shape=np.array(SHAPE, dtype=np.int64))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
