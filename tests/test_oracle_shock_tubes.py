"""The paper's non-ideal shock tubes I-III (Section 4.3.1) on the oracle.

The reference solutions the paper compares with are external data and not
used, so the profiles themselves are unpinned; what the paper prints and
the theory of non-classical gas dynamics fix is checked:
  * the largest Mach number reached, |u| / c_s over the domain and the run,
    is printed in the paper's table of numerical parameters: 0.45 (case I)
    and 0.196 (case II) -- scale-free numbers, so they hold in lattice units
    (bars 3 %);
  * case I lies at negative fundamental derivative Gamma (the text of
    Section 4.3.1; here all cells but the few inside the rarefaction front,
    whose intermediate states touch Gamma > 0): its rarefaction travels as a
    steep front and its
    compression as a spread-out fan -- the reverse of the classical case II
    (Gamma > 0 throughout), whose rarefaction is a fan and compression a
    shock;
  * case III starts classical on the dense side (Gamma > 1) and crosses
    Gamma < 0 in the middle of the tube; it stays finite over its run.
Lattice: 1000 cells along x (the paper's dx = L_x / 1000), zero-gradient
ends; constants from workload_states.json (van der Waals a = 3/49, b = 2/21,
R = 1, R/c_v per case, mu = eta = 0.05, kappa = 0.01).
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import thermo as th
from paper_2510_14712_amd import inputs

ST = inputs.states()
with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as _fh:
    GOLD = json.load(_fh)["shock_tube_cases"]


def _run(case, every=0):
    c = ST["shock_tube_" + case]
    shape = (c["shape"][0], 1)
    kw = inputs.physics(ST, "shock_tube_" + case)
    p = oracle.Params(2, shape, bc=tuple(c["bc"]), **kw)
    rho, u, T = inputs.shock_tube(shape, c["rho_left"], c["rho_right"], c["T_left"], T_right=c["T_right"])
    f, g = oracle.init(p, rho, u, T)
    mach = 0.0
    done = 0
    while done < c["steps"]:
        n = min(every or c["steps"], c["steps"] - done)
        f, g = oracle.run(p, f, g, n)
        done += n
        fl = oracle.fields(p, f, g)
        ok = fl["cs2"] > 0
        mach = max(mach, float(np.max(np.abs(fl["u"][: p.N][ok]) / np.sqrt(fl["cs2"][ok]))))
    return p, fl, mach


def _steepness(r):
    """Largest density step between neighbouring cells in the left and right
    halves of the tube."""
    d = np.abs(np.diff(r))
    n = r.size // 2
    return d[:n].max(), d[n:].max()


@pytest.mark.parametrize("case", ["I", "II"])
def test_peak_mach_number_matches_paper(case):
    _, fl, mach = _run(case, every=50)
    assert np.isfinite(fl["rho"]).all()
    assert mach == pytest.approx(GOLD[case]["max_ma"], rel=0.03)


def test_nonclassical_case_I_reverses_the_classical_wave_structure():
    _, fl1, _ = _run("I")
    _, fl2, _ = _run("II")
    left1, right1 = _steepness(fl1["rho"])
    left2, right2 = _steepness(fl2["rho"])
    # case I (Gamma < 0): rarefaction (left) steep, compression (right) a fan
    assert left1 > 3.0 * right1
    # case II (Gamma > 0): rarefaction a fan, compression a shock
    assert right2 > 10.0 * left2
    # Gamma < 0 over case I at the final time, but for the few cells inside
    # the rarefaction front (whose intermediate states touch Gamma > 0)
    c = ST["shock_tube_I"]
    G = np.array([th.fundamental_derivative_vdw(r, P, ST["constants"]["a"], ST["constants"]["b"], 1.0, c["cv"])
                  for r, P in zip(fl1["rho"], fl1["P"])])
    assert np.mean(G < 0) >= 0.98


def test_case_III_crosses_negative_gamma_and_stays_finite():
    p, fl, _ = _run("III")
    assert np.isfinite(fl["rho"]).all()
    c = ST["shock_tube_III"]
    a, b = ST["constants"]["a"], ST["constants"]["b"]
    G = np.array([th.fundamental_derivative_vdw(r, P, a, b, 1.0, c["cv"]) for r, P in zip(fl["rho"], fl["P"])])
    assert G[:100].min() > 1.0
    assert G.min() < 0.0
