"""Host side of the benchmark (no GPU): the roofline arithmetic of the bench
line, the committed hardware-counter summaries it reads (present, parsable,
for the kernel whose source they name), and the refusal of more than one
GPU."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_summaries_parse(bench):
    for name, spec in bench.KERNELS.items():
        rec = bench.read_traffic(spec["traffic_file"])
        assert rec is not None, spec["traffic_file"]
        assert rec["kernel"] == name
        assert len(rec["source_sha"]) == 16
        assert float(rec["fetch_bytes_per_unit"]) > 0 and float(rec["write_bytes_per_unit"]) > 0
        if "valu_file" in spec:
            v = bench.read_traffic(spec["valu_file"])
            assert v["kernel"] == name and len(v["source_sha"]) == 16
            assert float(v["valu_quad_cycles_per_unit"]) > 0
    for mode, name in bench.DOMINANT.items():
        assert name in bench.KERNELS, mode


def test_headline_counters_are_current(bench):
    """The summaries of the headline step's dominant kernel were taken on the
    kernel's present source (else the line would report their figures null)."""
    name = bench.DOMINANT[0]
    sha = bench.kernel_source_sha(name)
    spec = bench.KERNELS[name]
    assert bench.read_traffic(spec["traffic_file"])["source_sha"] == sha
    assert bench.read_traffic(spec["valu_file"])["source_sha"] == sha


def test_roofline_arithmetic(bench):
    name = bench.DOMINANT[0]
    spec = bench.KERNELS[name]
    launches, units_per_launch, us = 10, 3000, 250.0
    r = bench.dominant_roofline(name, launches, launches * units_per_launch, launches * us * 1e-3)
    limb = 8 << bench.LOGN
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(units_per_launch * limb)
    assert r["achieved"] == pytest.approx(units_per_launch * limb / (us * 1e-6) / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / spec["peak"])
    rec = bench.read_traffic(spec["traffic_file"])
    per = float(rec["fetch_bytes_per_unit"]) + float(rec["write_bytes_per_unit"])
    assert r["traffic"] == pytest.approx(per * units_per_launch)
    v = bench.read_traffic(spec["valu_file"])
    slots = 1024 * us * 1e-6 * 2.4e9 / 4
    assert r["valu"]["issue_frac"] == pytest.approx(float(v["valu_quad_cycles_per_unit"]) * units_per_launch / slots)
    assert bench.dominant_roofline(name, 0, 0, 0.0) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode != 0
    assert "--gpus 1" in p.stderr + p.stdout
