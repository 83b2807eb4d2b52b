"""ctypes binding of ``liblbm_hip.so`` (C ABI in ``include/lbm.h``).

Argument marshalling only: every step of the method runs in the HIP kernels.
Device arrays are torch CUDA tensors (PyTorch supplies device memory and the
stream); host numpy inputs are copied to the device first.  A missing or
unloadable library raises immediately -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_hip.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ENAN, LBM_ESTATE = 0, -1, -2, -3, -4, -5, -6
STORAGE = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
EOS = {"vdw": 0, "mlp": 1, "pr": 2, "pr_prev": 3, "pr_mlp": 4}
MLP_BF16, MLP_F32, MLP_BF16_L1 = 0, 1, 2
MLP_NPARAMS, MLP_NNORM = 4547, 10
# dead zone of the upwind switch: |u| at or below takes the central average
UPWIND_EPS = 1e-6


class LbmError(RuntimeError):
    def __init__(self, status, what):
        detail = load().lbm_last_error().decode() if status in (LBM_EDEVICE, LBM_ENOMEM) else ""
        super().__init__(f"{what}: {strerror(status)} ({status}) {detail}".rstrip())
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("bc", ctypes.c_int * 3),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double), ("cv", ctypes.c_double),
                ("mu", ctypes.c_double), ("eta", ctypes.c_double), ("k", ctypes.c_double),
                ("kappa", ctypes.c_double),
                ("storage", ctypes.c_int), ("eos", ctypes.c_int), ("mlp_tol", ctypes.c_double),
                ("ref_rho", ctypes.c_double), ("ref_T", ctypes.c_double), ("stream", ctypes.c_void_p),
                ("upwind_eps", ctypes.c_double), ("zsegments", ctypes.c_int), ("check_every", ctypes.c_int),
                ("pr_m", ctypes.c_double), ("pr_Tc", ctypes.c_double), ("pr_c0", ctypes.c_double),
                ("pr_c1", ctypes.c_double),
                ("wall_u", (ctypes.c_double * 3) * 2), ("wall_T", ctypes.c_double * 2),
                ("sc_cmu", ctypes.c_double), ("sc_ceta", ctypes.c_double), ("sc_ck", ctypes.c_double)]


_lib = None
_VP, _DP, _FP = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)


def load():
    """Load the HIP library (raises if it has not been built).

    torch is imported first: its bundled HIP runtime (soname libamdhip64.so.7)
    is then the one the library binds to, so the process holds a single HIP
    runtime; loading the library first would pull in a second copy."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime before the library, see above)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    PP = ctypes.POINTER(_Params)
    sig = {
        "lbm_create": ([PP, ctypes.POINTER(_VP)], ctypes.c_int),
        "lbm_destroy": ([_VP], None),
        "lbm_init": ([_VP, _VP, _VP, _VP], ctypes.c_int),
        "lbm_step": ([_VP, ctypes.c_int], ctypes.c_int),
        "lbm_moments": ([_VP, _VP, _VP, _VP, _VP], ctypes.c_int),
        "lbm_get_populations": ([_VP, _VP, _VP], ctypes.c_int),
        "lbm_set_populations": ([_VP, _VP, _VP], ctypes.c_int),
        "lbm_conservation": ([_VP, _DP], ctypes.c_int),
        "lbm_synchronize": ([_VP], ctypes.c_int),
        "lbm_bytes_per_cell": ([_VP], ctypes.c_double),
        "lbm_step_timed": ([_VP, ctypes.c_int, _DP, ctypes.c_int], ctypes.c_int),
        "lbm_kernel_name": ([_VP, ctypes.c_int], ctypes.c_char_p),
        "lbm_is_fused": ([_VP], ctypes.c_int),
        "lbm_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "lbm_last_error": ([], ctypes.c_char_p),
        "lbm_mlp_train": ([PP, _DP, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                           ctypes.c_int, _FP, _FP, _DP], ctypes.c_int),
        "lbm_mlp_set": ([_VP, _FP, _FP], ctypes.c_int),
        "lbm_mlp_stats": ([_VP, _DP], ctypes.c_int),
        "lbm_eos_stats": ([_VP, _DP, _DP], ctypes.c_int),
        "lbm_mlp_forward": ([_VP, _VP, _VP, _VP, ctypes.c_int, ctypes.c_int, _VP], ctypes.c_int),
        "lbm_mlp_loss_grad": ([_VP, _VP, _VP, ctypes.c_int, _VP, _VP, ctypes.c_int, _VP], ctypes.c_int),
        "lbm_mlp_loss_grad_noalloc": ([_VP, _VP, _VP, ctypes.c_int, _VP, _VP, ctypes.c_int, _VP], ctypes.c_int),
        "lbm_mlp_adam": ([_VP, _VP, _VP, _VP, ctypes.c_int, ctypes.c_float, _VP], ctypes.c_int),
        "lbm_hbm_probe": ([ctypes.c_int, _VP, _VP, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _VP, _DP],
                          ctypes.c_int),
        "lbm_codec_encode": ([ctypes.c_int, _VP, _VP, _VP, ctypes.c_int64, _VP], ctypes.c_int),
        "lbm_codec_decode": ([ctypes.c_int, _VP, _VP, _VP, ctypes.c_int64, _VP], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def strerror(status: int) -> str:
    return load().lbm_strerror(int(status)).decode()


def _check(status, what):
    if status != LBM_OK:
        raise LbmError(status, what)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(arr, dtype, n=None):
    """Contiguous CUDA tensor of the given torch dtype (copies host arrays)."""
    torch = _torch()
    if isinstance(arr, torch.Tensor):
        t = arr.to(device="cuda", dtype=dtype).contiguous()
    else:
        t = torch.as_tensor(np.ascontiguousarray(arr)).to(device="cuda", dtype=dtype).contiguous()
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} values, got {t.numel()}")
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Lattice:
    """One lattice Boltzmann context (lbm_create ... lbm_destroy)."""

    def __init__(self, lattice, shape, bc=(0, 0, 0), a=3.0 / 49.0, b=2.0 / 21.0, R=1.0, cv=2.5, mu=0.05,
                 eta=0.05, k=None, kappa=0.01, storage="f32", eos="vdw", mlp_tol=1e-6, ref_rho=0.0, ref_T=0.0,
                 stream=None, upwind_eps=UPWIND_EPS, zsegments=0, check_every=0, sc=(0.0, 0.0, 0.0), pr=None,
                 walls=None):
        L = load()
        self.D = int(lattice)
        nx, ny = int(shape[0]), int(shape[1])
        nz = int(shape[2]) if self.D == 3 else 1
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        self.Q = 9 if self.D == 2 else 27
        p = _Params()
        p.lattice, p.nx, p.ny, p.nz = self.D, nx, ny, nz
        for i in range(3):
            p.bc[i] = int(bc[i])
        p.a, p.b, p.R, p.cv = a, b, R, cv
        p.mu, p.eta = mu, eta
        p.k = mu * (cv + R) if k is None else k
        p.kappa = kappa
        p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        p.eos = EOS[eos] if isinstance(eos, str) else int(eos)
        p.mlp_tol = mlp_tol
        p.ref_rho, p.ref_T = ref_rho, ref_T
        p.upwind_eps = upwind_eps
        p.zsegments = int(zsegments)
        p.check_every = int(check_every)
        p.sc_cmu, p.sc_ceta, p.sc_ck = (float(v) for v in sc)  # shock capturing (C_mu, C_eta, C_k)
        if walls is not None:  # bc[0] = 2: ((u_lo, T_lo), (u_hi, T_hi)) of the x walls
            for side, (uw, Tw) in enumerate(walls):
                for a, v in enumerate(uw):
                    p.wall_u[side][a] = float(v)
                p.wall_T[side] = float(Tw)
        if pr is not None:  # Peng-Robinson constants dict(m, Tc, c0, c1); a, b, R above
            p.pr_m, p.pr_Tc, p.pr_c0, p.pr_c1 = (float(pr[k]) for k in ("m", "Tc", "c0", "c1"))
        self._stream = stream
        p.stream = _stream_ptr(stream).value if _torch().cuda.is_available() else None
        self.params = p
        h = _VP()
        _check(L.lbm_create(ctypes.byref(p), ctypes.byref(h)), "lbm_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the ABI calls -----------------------------------------------------
    def init(self, rho, u, T):
        torch = _torch()
        r = _dev(rho, torch.float64, self.N)
        uu = _dev(u, torch.float64, self.D * self.N)
        t = _dev(T, torch.float64, self.N)
        _check(load().lbm_init(self._h, _ptr(r), _ptr(uu), _ptr(t)), "lbm_init")
        self._keep = (r, uu, t)  # alive until the stream has consumed them
        return self

    def step(self, n=1):
        _check(load().lbm_step(self._h, int(n)), "lbm_step")
        return self

    def step_timed(self, n):
        """Average per-launch duration (ms) of each kernel of the step over n steps."""
        out = (ctypes.c_double * 8)()
        _check(load().lbm_step_timed(self._h, int(n), out, 8), "lbm_step_timed")
        names = [load().lbm_kernel_name(self._h, k).decode() for k in range(8)]
        return {nm: out[k] for k, nm in enumerate(names) if nm}

    @property
    def fused(self):
        return bool(load().lbm_is_fused(self._h))

    def moments(self):
        torch = _torch()
        out = {k: torch.empty(self.N * (self.D if k == "u" else 1), dtype=torch.float64, device="cuda")
               for k in ("rho", "u", "T", "P")}
        _check(load().lbm_moments(self._h, _ptr(out["rho"]), _ptr(out["u"]), _ptr(out["T"]), _ptr(out["P"])),
               "lbm_moments")
        return out

    def get_populations(self):
        torch = _torch()
        f = torch.empty(self.Q * self.N, dtype=torch.float64, device="cuda")
        g = torch.empty_like(f)
        _check(load().lbm_get_populations(self._h, _ptr(f), _ptr(g)), "lbm_get_populations")
        return f, g

    def set_populations(self, f, g):
        torch = _torch()
        ft = _dev(f, torch.float64, self.Q * self.N)
        gt = _dev(g, torch.float64, self.Q * self.N)
        _check(load().lbm_set_populations(self._h, _ptr(ft), _ptr(gt)), "lbm_set_populations")
        self._keep = (ft, gt)
        return self

    def conservation(self, raise_on_nan=True):
        """[sum rho, sum rho u (D), sum g, non-finite cells, inadmissible cells];
        raises on LBM_ENAN / LBM_EUNSTABLE unless raise_on_nan is False."""
        out = (ctypes.c_double * 8)()
        rc = load().lbm_conservation(self._h, out)
        if rc != LBM_OK and (rc not in (LBM_ENAN, LBM_EUNSTABLE) or raise_on_nan):
            _check(rc, "lbm_conservation")
        return np.array(out[: self.D + 4])

    def synchronize(self):
        _check(load().lbm_synchronize(self._h), "lbm_synchronize")

    @property
    def bytes_per_cell(self):
        return load().lbm_bytes_per_cell(self._h)

    def mlp_set(self, params, norm):
        p = np.ascontiguousarray(params, dtype=np.float32)
        n = np.ascontiguousarray(norm, dtype=np.float32)
        assert p.size == MLP_NPARAMS and n.size == MLP_NNORM
        _check(load().lbm_mlp_set(self._h, p.ctypes.data_as(_FP), n.ctypes.data_as(_FP)), "lbm_mlp_set")

    def mlp_stats(self):
        v = ctypes.c_double()
        _check(load().lbm_mlp_stats(self._h, ctypes.byref(v)), "lbm_mlp_stats")
        return v.value

    def eos_stats(self):
        """(fallback fraction, mean Newton iterations per cell) since the last call."""
        fb, it = ctypes.c_double(), ctypes.c_double()
        _check(load().lbm_eos_stats(self._h, ctypes.byref(fb), ctypes.byref(it)), "lbm_eos_stats")
        return fb.value, it.value


def mlp_train(box, n_samples, seed, epochs, batch, lr, params0, precision=MLP_BF16, a=3.0 / 49.0, b=2.0 / 21.0,
              R=1.0, cv=2.5, pr=None):
    """lbm_mlp_train: returns (params[4547], norm[10], final_loss).  pr:
    Peng-Robinson constants dict(m, Tc, c0, c1) to train on that equation of
    state (a, b, R then its constants), else van der Waals."""
    p = _Params()
    p.lattice, p.nx, p.ny, p.nz = 2, 1, 1, 1
    p.a, p.b, p.R, p.cv = a, b, R, cv
    p.mu = 1.0
    if pr is not None:
        p.eos = EOS["pr_mlp"]
        p.pr_m, p.pr_Tc, p.pr_c0, p.pr_c1 = (float(pr[k]) for k in ("m", "Tc", "c0", "c1"))
    bx = np.ascontiguousarray(box, dtype=np.float64)
    prm = np.ascontiguousarray(params0, dtype=np.float32).copy()
    norm = np.zeros(MLP_NNORM, dtype=np.float32)
    loss = ctypes.c_double()
    _check(load().lbm_mlp_train(ctypes.byref(p), bx.ctypes.data_as(_DP), int(n_samples), int(seed), int(epochs),
                                int(batch), float(lr), int(precision), prm.ctypes.data_as(_FP),
                                norm.ctypes.data_as(_FP), ctypes.byref(loss)), "lbm_mlp_train")
    return prm, norm, loss.value


def mlp_forward(params, norm, x, precision=MLP_BF16, stream=None):
    torch = _torch()
    pt = _dev(params, torch.float32, MLP_NPARAMS)
    nt = _dev(norm, torch.float32, MLP_NNORM)
    xt = _dev(x, torch.float32)
    B = xt.numel() // 2
    y = torch.empty(3 * B, dtype=torch.float32, device="cuda")
    _check(load().lbm_mlp_forward(_ptr(pt), _ptr(nt), _ptr(xt), _ptr(y), B, int(precision), _stream_ptr(stream)),
           "lbm_mlp_forward")
    return y.view(B, 3)


def mlp_loss_grad(params, xn, tn, precision=MLP_BF16, stream=None):
    torch = _torch()
    pt = _dev(params, torch.float32, MLP_NPARAMS)
    xt = _dev(xn, torch.float32)
    tt = _dev(tn, torch.float32)
    B = xt.numel() // 2
    grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(load().lbm_mlp_loss_grad(_ptr(pt), _ptr(xt), _ptr(tt), B, _ptr(grad), _ptr(loss), int(precision),
                                    _stream_ptr(stream)), "lbm_mlp_loss_grad")
    return loss, grad


def mlp_loss_grad_noalloc(params, xn, tn, precision=MLP_BF16, stream=None, out=None):
    """lbm_mlp_loss_grad_noalloc: the library allocates nothing; `out` =
    (loss[1], grad[4547]) float32 CUDA tensors to fill, else new ones."""
    torch = _torch()
    pt = _dev(params, torch.float32, MLP_NPARAMS)
    xt = _dev(xn, torch.float32)
    tt = _dev(tn, torch.float32)
    B = xt.numel() // 2
    if out is None:
        out = (torch.empty(1, dtype=torch.float32, device="cuda"),
               torch.empty(MLP_NPARAMS, dtype=torch.float32, device="cuda"))
    loss, grad = out
    _check(load().lbm_mlp_loss_grad_noalloc(_ptr(pt), _ptr(xt), _ptr(tt), B, _ptr(grad), _ptr(loss), int(precision),
                                            _stream_ptr(stream)), "lbm_mlp_loss_grad_noalloc")
    return loss, grad


def mlp_adam(params, grad, m, v, t, lr, stream=None):
    """lbm_mlp_adam on CUDA float32 tensors of 4547 values (updated in place)."""
    for a in (params, grad, m, v):
        assert a.is_cuda and a.dtype == _torch().float32 and a.is_contiguous() and a.numel() == MLP_NPARAMS
    _check(load().lbm_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t), float(lr), _stream_ptr(stream)),
           "lbm_mlp_adam")


def hbm_probe(kind, src, dst, blocks_per_cu, iters=10, stream=None):
    """lbm_hbm_probe on CUDA tensors: average ms per launch of the read (0),
    write (1) or copy (2) probe over dst's bytes."""
    ms = ctypes.c_double()
    nbytes = dst.numel() * dst.element_size()
    _check(load().lbm_hbm_probe(int(kind), _ptr(src), _ptr(dst), nbytes, int(blocks_per_cu), int(iters),
                                _stream_ptr(stream), ctypes.byref(ms)), "lbm_hbm_probe")
    return ms.value


def codec_encode(kind, x, ref, stream=None):
    torch = _torch()
    xt = _dev(x, torch.float32)
    rt = _dev(ref, torch.float32, xt.numel())
    out = torch.empty(xt.numel(), dtype=torch.int16, device="cuda")
    _check(load().lbm_codec_encode(STORAGE[kind], _ptr(xt), _ptr(rt), _ptr(out), xt.numel(), _stream_ptr(stream)),
           "lbm_codec_encode")
    return out


def codec_decode(kind, code, ref, stream=None):
    torch = _torch()
    ct = _dev(code, torch.int16)
    rt = _dev(ref, torch.float32, ct.numel())
    out = torch.empty(ct.numel(), dtype=torch.float32, device="cuda")
    _check(load().lbm_codec_decode(STORAGE[kind], _ptr(ct), _ptr(rt), _ptr(out), ct.numel(), _stream_ptr(stream)),
           "lbm_codec_decode")
    return out
