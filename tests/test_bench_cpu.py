"""Host-side checks of bench.py: the counter figures it reports (HBM traffic,
MFMA busy share, executed MFMA flops) are recorded in profiles/ for the
current contraction sources of both workloads, the recorded kernel trace
agrees with the roofline figures next to it, and a request for more than one
GPU is refused before anything touches a device."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("w", ["ceal", "lih"])
def test_counter_figures_recorded_for_current_sources(w):
    tag = "contract_f64_%s_cell" % w
    traffic, = bench.recorded(tag + "_hbm_traffic.md", "traffic_bytes_per_launch")
    busy, executed = bench.recorded(tag + "_mfma_counters.md", "mfma_busy_frac", "mfma_executed_flops_per_launch")
    assert traffic is not None and busy is not None and executed is not None, \
        "profiles/%s_*.md were measured on other kernel sources" % tag
    assert 0.0 < busy < 1.0
    assert traffic > 0 and executed > 0


@pytest.mark.parametrize("w", ["ceal", "lih"])
def test_kernel_trace_roofline_line(w):
    """The trace summary's roofline line is its algorithmic flop over its
    contraction time, against the FP64 peak."""
    txt = open(os.path.join(ROOT, "profiles", "contract_f64_%s_cell_kernel_trace.md" % w)).read()
    m = re.search(r"([0-9.]+e\+[0-9]+) algorithmic flop .*? / ([0-9.]+) ms\s*= ([0-9.]+) TFLOP/s = ([0-9.]+) of",
                  txt, re.S)
    assert m, "no roofline line"
    flop, ms, tf, frac = (float(x) for x in m.groups())
    assert abs(flop / (ms * 1e-3) / 1e12 - tf) < 0.06
    assert abs(tf / bench.PEAK["fp64"] - frac) < 2e-3


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 1" in r.stderr
