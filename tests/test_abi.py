"""Host-side checks of the C ABI (no GPU needed): the built library loads,
exports every function declared in include/lbm.h, and rejects invalid
parameters before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2510_14712_amd import lbm
    L = lbm.load()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_library_is_not_a_cpu_fallback():
    from paper_2510_14712_amd import lbm
    data = open(lbm.LIB_PATH, "rb").read()
    assert b"amdgcn" in data or b"gfx950" in data  # device code object present


def _params(**over):
    from paper_2510_14712_amd import lbm
    p = lbm._Params()
    p.lattice, p.nx, p.ny, p.nz = 3, 8, 8, 8
    p.a, p.b, p.R, p.cv, p.mu, p.eta, p.k, p.kappa = 3 / 49, 2 / 21, 1.0, 2.5, 0.05, 0.05, 0.175, 0.01
    p.storage, p.eos = 1, 0
    for k, v in over.items():
        if k == "bc":
            for i in range(3):
                p.bc[i] = v[i]
        else:
            setattr(p, k, v)
    return p


@pytest.mark.parametrize("over", [
    dict(lattice=4), dict(nx=0), dict(lattice=2, nz=2), dict(bc=(2, 0, 0)), dict(storage=7),
    dict(eos=3), dict(cv=0.0), dict(mu=-1.0), dict(storage=2, ref_rho=0.0, ref_T=0.2),
    dict(storage=0, eos=1), dict(ny=70000), dict(upwind_eps=-1.0), dict(zsegments=-1), dict(zsegments=9),
    dict(check_every=-1),
])
def test_invalid_parameters_rejected(over):
    from paper_2510_14712_amd import lbm
    L = lbm.load()
    h = ctypes.c_void_p()
    assert L.lbm_create(ctypes.byref(_params(**over)), ctypes.byref(h)) == lbm.LBM_EINVAL
    assert not h.value


def test_null_handles_rejected():
    from paper_2510_14712_amd import lbm
    L = lbm.load()
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_init(None, None, None, None) == lbm.LBM_EINVAL
    assert L.lbm_create(None, None) == lbm.LBM_EINVAL
    assert L.lbm_codec_encode(9, None, None, None, 10, None) == lbm.LBM_EINVAL
    assert L.lbm_codec_encode(2, None, None, None, 0, None) == lbm.LBM_OK
    assert lbm.strerror(-5) == "non-finite value in the state"
    assert lbm.strerror(-4) == "state left the admissible set"
    # the Adam step checks its arguments before any launch
    assert L.lbm_mlp_adam(None, None, None, None, 1, ctypes.c_float(1e-3), None) == lbm.LBM_EINVAL
