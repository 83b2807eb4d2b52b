"""Host-side logic of bench.py (no GPU): the kernel-source hash that decides
whether the committed HBM-traffic record still describes the kernels, and the
one-GPU contract of the command line."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _read(name):
    with open(os.path.join(ROOT, "paper_2510_14712_amd", "csrc", name)) as fh:
        return fh.read()


def test_comment_edits_keep_the_hash_code_edits_change_it():
    base = bench.kernel_source_hash(_read)
    assert base == bench.kernel_source_hash()
    first = bench.KERNEL_SOURCES[0]

    def commented(name):
        t = _read(name)
        return t + "\n// a note\n/* and a block\n   comment */\n\n" if name == first else t

    def edited(name):
        t = _read(name)
        return t + "\nstatic const int extra_constant = 1;\n" if name == first else t

    assert bench.kernel_source_hash(commented) == base
    assert bench.kernel_source_hash(edited) != base


def test_strip_comments():
    src = "int a = 1; // one\n/* two\n three */ int b = 2;\n\n   // only a comment\nint c;"
    assert bench.strip_comments(src) == "int a = 1;\n int b = 2;\nint c;"


def test_traffic_record_parses():
    # the committed record is well formed and names the four forms it covers
    with open(bench.TRAFFIC_SUMMARY) as fh:
        lines = [l for l in fh if l.startswith("traffic-json:")]
    assert len(lines) == 1
    rec = json.loads(lines[0][len("traffic-json:"):])
    assert rec["kernel"] == "k_fused" and len(rec["source_hash"]) == 16
    for form in ("plain_fp32", "surrogate_bf16", "bf16_vdw"):
        f = rec["forms"][form]
        assert f["bytes_per_cell"] >= f["algorithmic_bytes_per_cell"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in out["error"]
