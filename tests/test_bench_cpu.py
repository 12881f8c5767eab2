"""The benchmark's contract on the host (no GPU): the one-GPU rule and the roofline model
computed from the committed rocprofv3 counters."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""   # no JSON line for a configuration that is not measured


def test_roofline_model():
    """frac = achieved / peak with achieved = ops per set x sets / time; the HBM traffic is
    2 x FETCH_SIZE + WRITE_SIZE (KiB) of the committed counters when they were taken with the
    current kernel sources, and absent otherwise."""
    sets, ms = 8.41e8, 5.2
    out = bench.roofline("batch4096", sets, ms, "k_small", 1.7e9)
    assert out["bound"] == "alu" and out["unit"] == "TOP/s"
    assert out["achieved"] == pytest.approx(bench.MODEL_OPS_PER_SET * sets / (ms * 1e-3) / 1e12)
    assert out["frac"] == pytest.approx(out["achieved"] / out["peak"])
    with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
        rec = json.load(f)["batch4096"]
    if rec["sources_sha256"] == bench.sources_sha256("batch4096"):
        assert out["traffic"] == pytest.approx(1024.0 * (2.0 * rec["fetch_kib"] + rec["write_kib"]))
        assert out["measured"]["memory_side_atomics"] == rec["tcc_ea0_atomic"]
    else:
        assert out["traffic"] is None and "note" in out
    # an unknown workload has no counters: traffic stays unmeasured
    other = bench.roofline("no-such-workload", sets, ms, "k", 1.0)
    assert other["traffic"] is None


def test_counter_keys_cover_every_workload_with_a_profile():
    """Every workload with committed counters names the kernel sources its key covers."""
    with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
        recs = json.load(f)
    for name, rec in recs.items():
        assert name in bench.COUNTER_SOURCES, name
        assert len(rec["sources_sha256"]) == 64
        for key in ("fetch_kib", "write_kib", "valu_insts", "tcc_ea0_atomic", "command"):
            assert key in rec, (name, key)
