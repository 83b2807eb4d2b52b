"""Throughput of the fused stream-collide step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload tgv512]

Workload (default): the D3Q27 near-critical Taylor-Green vortex on a 512^3
periodic lattice (rho_c, 1.1 T_c, Mach 0.5, 1 % seeded density noise), run in
the two forms the metric compares on the same steps:
  * plain: FP32 populations, FP32 arithmetic, explicit van der Waals EOS;
  * surrogate: BF16 deviation storage, FP32 arithmetic, MLP EOS (BF16 MFMA)
    with residual check and FP64 Newton fallback, FP64 conservation sums.
`value` is the surrogate form's MLUPS (the full hot path); the plain form's
figures are reported beside it, and those of BF16 storage with the explicit
EOS (what the surrogate pass costs).  Inputs are synthetic and resident in
HBM before the timed region; the timed region is K steps bracketed by device
synchronisation.  One JSON line is printed.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# sources of the fused step; the measured HBM traffic in profiles/ is reported
# only while these are unchanged since the counters were taken
KERNEL_SOURCES = ("lbm_fused.hpp", "lbm_kernels.hpp", "lbm_device.hpp", "lbm_mlp_device.hpp", "lbm_capi.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_fused_tgv512_hbm_traffic.md")


def strip_comments(text):
    """C++ source without its comments and blank lines (an edit of a comment
    leaves the kernels, and so the measured traffic, as they were)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = []
    for line in text.split("\n"):
        i = line.find("//")
        if i >= 0:
            line = line[:i]
        line = line.rstrip()
        if line:
            out.append(line)
    return "\n".join(out)


def kernel_source_hash(read=None):
    """Hash of the fused step's sources, comments stripped; `read(name)` gives
    a file's text (default: the working tree)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        if read is None:
            with open(os.path.join(ROOT, "paper_2510_14712_amd", "csrc", name)) as fh:
                text = fh.read()
        else:
            text = read(name)
        h.update(strip_comments(text).encode())
    return h.hexdigest()[:16]


def measured_traffic(form):
    """HBM bytes per launch of the fused kernel of `form` from the committed
    FETCH_SIZE / WRITE_SIZE summary (scaled by the plain-copy calibration), or
    None when the summary is missing or the kernel sources changed since."""
    try:
        with open(TRAFFIC_SUMMARY) as fh:
            for line in fh:
                if line.startswith("traffic-json:"):
                    rec = json.loads(line[len("traffic-json:"):])
                    if rec.get("source_hash") == kernel_source_hash() and form in rec.get("forms", {}):
                        return rec["forms"][form]
    except OSError:
        pass
    return None


def _p(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name, st):
    from paper_2510_14712_amd import inputs
    if name in ("tgv512", "tgv256"):
        c = st["tgv_3d_512" if name == "tgv512" else "tgv_3d_256"]
        shape = tuple(c["shape"])
        rho, u, T = inputs.taylor_green(shape, c["seed"], c["rho0"], c["T0"], c["U0"], c["noise"])
        desc = (f"D3Q27 near-critical Taylor-Green vortex {shape[0]}x{shape[1]}x{shape[2]} periodic, "
                f"rho_c, 1.1 T_c, Mach 0.5, 1% noise (seed {c['seed']})")
        return shape, (0, 0, 0), (rho, u, T), (c["rho0"], c["T0"]), desc
    if name == "drop3d":
        c = st["shock_drop_3d"]
        shape = tuple(c["shape"])
        rho, u, T = inputs.shock_drop(shape, c["centre"], c["radius"], c["width"], c["rho_liquid"],
                                      c["rho_vapour"], c["T1"], c["x_shock"], c["rho2"], c["T2"], c["u2"])
        desc = (f"D3Q27 shock-drop {shape[0]}x{shape[1]}x{shape[2]}, sphere R {c['radius']}, Ma 1.47, "
                f"T = 0.85 T_c")
        return shape, tuple(c["bc"]), (rho, u, T), (c["rho_vapour"], c["T1"]), desc
    raise SystemExit(f"unknown workload {name}")


def train_surrogate(st, lbm):
    c = st["shock_drop_3d"]
    box = [c["mlp_box"]["rho"][0], c["mlp_box"]["rho"][1], c["mlp_box"]["T"][0], c["mlp_box"]["T"][1]]
    from paper_2510_14712_amd import inputs
    k = st["constants"]
    p0 = inputs.mlp_params(c["mlp_seed"]).astype(np.float32)
    t0 = time.perf_counter()
    params, norm, loss = lbm.mlp_train(box, c["mlp_samples"], c["mlp_seed"], 40, 8192, 3e-3, p0,
                                       a=k["a"], b=k["b"], R=k["R"], cv=k["cv"])
    return params, norm, loss, time.perf_counter() - t0


def time_form(lbm, torch, shape, bc, fields, ref, kw, storage, eos, steps, warmup, mlp=None):
    rho, u, T = fields
    N = int(np.prod(shape))
    lat = lbm.Lattice(3, shape, bc=bc, storage=storage, eos=eos, mlp_tol=1e-6, ref_rho=ref[0], ref_T=ref[1], **kw)
    try:
        if mlp is not None:
            lat.mlp_set(mlp[0], mlp[1])
        lat.init(rho, u, T)
        lat.step(warmup)
        lat.synchronize()
        if eos == "mlp":
            lat.mlp_stats()  # reset the fallback counters
        # the timed region: K steps with HIP events around every launch on the
        # library's stream (per-kernel average durations of these same steps)
        lat.synchronize()
        t0 = time.perf_counter()
        kt = lat.step_timed(steps)
        lat.synchronize()
        dt = time.perf_counter() - t0
        sums = lat.conservation(raise_on_nan=False)
        fb = lat.mlp_stats() if eos == "mlp" else None
        bpc = lat.bytes_per_cell
    finally:
        lat.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    # sums: [mass, momentum (3), sum g, non-finite cells, inadmissible cells]
    return dict(seconds=dt, mlups=N * steps / dt / 1e6, ms_per_step=1e3 * dt / steps, bytes_per_cell=bpc,
                kernel_ms=kt, finite=bool(sums[5] == 0), admissible=bool(sums[6] == 0), fallback_fraction=fb,
                mass=float(sums[0]))


def cpu_baseline(st, seconds_target=12.0):
    """The FP64 oracle on the host's cores: a 64^3 sample of the benchmark's
    workload (same recipe and constants), timed with every host thread and
    with one."""
    import oracle
    from paper_2510_14712_amd import inputs
    c = st["tgv_3d_512"]
    shape = (64, 64, 64)
    rho, u, T = inputs.taylor_green(shape, c["seed"], c["rho0"], c["T0"], c["U0"], c["noise"])
    p = oracle.Params(3, shape, **inputs.physics(st, "tgv_3d_512"))
    f0, g0 = oracle.init(p, rho, u, T)

    def timed(threads):
        oracle.set_num_threads(threads)
        t0 = time.perf_counter()
        f, g = oracle.run(p, f0, g0, 1)
        one = time.perf_counter() - t0
        n = max(1, int(seconds_target / max(one, 1e-3)))
        t0 = time.perf_counter()
        oracle.run(p, f, g, n)
        dt = time.perf_counter() - t0
        return p.N * n / dt / 1e6, n, dt

    ncores = oracle.num_threads()  # the OpenMP default: OMP_NUM_THREADS, else the host's cores
    mt, n, dt = timed(ncores)
    threads = oracle.num_threads()
    st1, n1, dt1 = timed(1)
    oracle.set_num_threads(ncores)
    return {"value": round(mt, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, D3Q27 Taylor-Green 64^3 (the workload's recipe and constants), {n} steps in "
                      f"{dt:.1f} s on {threads} threads; 1 thread: {n1} steps in {dt1:.1f} s",
            "single_thread": {"value": round(st1, 4), "unit": "MLUPS", "cores": 1}}


def hbm_probe(lbm, torch):
    """Ceiling of the access pattern-free HBM streams on this GPU: GB/s of the
    library's read / write / copy probes (16-byte accesses, non-temporal
    hint) per workgroups-per-CU setting, and of the runtime's device copy."""
    nbytes = 4 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {"bytes": nbytes, "probes": {}}
    for kind, name, moved in ((0, "read", 1), (1, "write", 1), (2, "copy", 2)):
        row = {}
        for bpc in (1, 2, 4, 8, 16, 32):
            ms = lbm.hbm_probe(kind, src, dst, bpc, iters=10)
            row[bpc] = round(moved * nbytes / (ms * 1e-3) / 1e9, 1)
        out["probes"][name] = row
        _p(f"{name}: GB/s by workgroups per CU {row}")
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    dst.copy_(src)
    t0.record()
    for _ in range(10):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    out["runtime_copy_gbs"] = round(2 * nbytes / (t0.elapsed_time(t1) / 10 * 1e-3) / 1e9, 1)
    out["peak_gbs"] = HBM_PEAK_GBS
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="tgv512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="plain,bf16vdw,surrogate,f16surrogate", help="comma list of forms to time")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="only measure the HBM ceiling: read, write and copy probes over 4 GiB, "
                         "workgroups per compute unit swept, beside the runtime's copy")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        torch.cuda.set_device(0)
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "launches": 3}), flush=True)
        return
    from paper_2510_14712_amd import inputs, lbm
    lbm.load()
    torch.cuda.set_device(0)
    if args.hbm_probe:
        hbm_probe(lbm, torch)
        return
    st = inputs.states()
    wl = {"tgv512": "tgv_3d_512", "tgv256": "tgv_3d_256", "drop3d": "shock_drop_3d"}[args.workload]
    kw = inputs.physics(st, wl)
    shape, bc, fields, ref, desc = workload(args.workload, st)
    N = int(np.prod(shape))

    forms = args.forms.split(",")
    plain = bvdw = surr = f16s = None
    # the value form first, on a device whose memory no earlier form has
    # fragmented (a form timed after others' large allocations and frees ran
    # its fused kernel up to 6 % slower)
    if "surrogate" in forms:
        _p("training the surrogate EOS on the GPU")
        params, norm, loss, t_train = train_surrogate(st, lbm)
        _p(f"  loss {loss:.3e} in {t_train:.1f} s")
        _p("surrogate + BF16 deviation form")
        surr = time_form(lbm, torch, shape, bc, fields, ref, kw, "bf16", "mlp", args.steps, args.warmup,
                         mlp=(params, norm))
        _p(f"  {surr['mlups']:.0f} MLUPS, kernels {surr['kernel_ms']}, fallback {surr['fallback_fraction']}")
    if "f16surrogate" in forms and surr is not None:
        _p("surrogate + FP16 deviation form")
        f16s = time_form(lbm, torch, shape, bc, fields, ref, kw, "f16", "mlp", args.steps, args.warmup,
                         mlp=(params, norm))
        _p(f"  {f16s['mlups']:.0f} MLUPS, kernels {f16s['kernel_ms']}, fallback {f16s['fallback_fraction']}")
    if "plain" in forms:
        _p(f"plain FP32 form on {shape}")
        plain = time_form(lbm, torch, shape, bc, fields, ref, kw, "f32", "vdw", args.steps, args.warmup)
        _p(f"  {plain['mlups']:.0f} MLUPS, kernels {plain['kernel_ms']}")
    if "bf16vdw" in forms:
        _p("BF16 deviation form, explicit van der Waals EOS")
        bvdw = time_form(lbm, torch, shape, bc, fields, ref, kw, "bf16", "vdw", args.steps, args.warmup)
        _p(f"  {bvdw['mlups']:.0f} MLUPS, kernels {bvdw['kernel_ms']}")
    if surr is None or plain is None:
        print(json.dumps({"forms": {"plain_fp32": plain, "bf16_vdw": bvdw, "surrogate_bf16": surr}}), flush=True)
        return

    def roof(form, name):
        kms = form["kernel_ms"]
        dom = max(kms, key=kms.get)
        bytes_launch = form["bytes_per_cell"] * N
        achieved = bytes_launch / (kms[dom] * 1e-3) / 1e9
        tr = measured_traffic(name)
        return dom, {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if tr is None else tr["bytes_per_launch"],
                     "traffic_bytes_per_cell": None if tr is None else round(tr["bytes_per_launch"] / N, 1),
                     "algorithmic_bytes_per_cell": form["bytes_per_cell"]}

    dom, rl = roof(surr, "surrogate_bf16")
    line = {
        "metric": "MLUPS & % HBM peak, D3Q27 fused step: plain FP32 vs surrogate-EOS/BF16 form",
        "value": round(surr["mlups"], 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(surr["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16-storage/f32", "data": "synthetic",
        "config": {"workload": desc, "form": "BF16 deviation storage + MLP EOS (BF16 MFMA) + Newton fallback",
                   "cells": N},
        "roofline": dict(rl, kernel=dom),
        "forms": {
            "plain_fp32": {"mlups": round(plain["mlups"], 1), "ms_per_step": round(plain["ms_per_step"], 4),
                           "step_hbm_frac": round(plain["bytes_per_cell"] * plain["mlups"] * 1e6 / 1e9
                                                  / HBM_PEAK_GBS, 4),
                           "kernel_ms": plain["kernel_ms"], "finite": plain["finite"],
                           "roofline": roof(plain, "plain_fp32")[1]},
            "surrogate_bf16": {"mlups": round(surr["mlups"], 1), "ms_per_step": round(surr["ms_per_step"], 4),
                               "step_hbm_frac": round(surr["bytes_per_cell"] * surr["mlups"] * 1e6 / 1e9
                                                      / HBM_PEAK_GBS, 4),
                               "kernel_ms": surr["kernel_ms"], "finite": surr["finite"],
                               "fallback_fraction": surr["fallback_fraction"], "mlp_train_s": round(t_train, 2),
                               "mlp_loss": loss, "admissible": surr["admissible"]},
        },
    }
    if bvdw is not None:
        line["forms"]["bf16_vdw"] = {
            "mlups": round(bvdw["mlups"], 1), "ms_per_step": round(bvdw["ms_per_step"], 4),
            "step_hbm_frac": round(bvdw["bytes_per_cell"] * bvdw["mlups"] * 1e6 / 1e9 / HBM_PEAK_GBS, 4),
            "kernel_ms": bvdw["kernel_ms"], "finite": bvdw["finite"], "roofline": roof(bvdw, "bf16_vdw")[1]}
    if f16s is not None:
        line["forms"]["surrogate_f16"] = {
            "mlups": round(f16s["mlups"], 1), "ms_per_step": round(f16s["ms_per_step"], 4),
            "kernel_ms": f16s["kernel_ms"], "finite": f16s["finite"], "fallback_fraction": f16s["fallback_fraction"],
            "admissible": f16s["admissible"]}
    if not args.no_cpu_baseline:
        _p("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(st)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
