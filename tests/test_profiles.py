"""The committed profiler summaries describe the kernels the library runs by default: the kernel trace holds the
template instance of the residual conv the benchmark's roofline names, and the HBM-traffic record covers the
library's default tile variant.  Host-side checks of text files only."""
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_02912_amd", "csrc")
PROF = os.path.join(ROOT, "profiles")


def _default_variant():
    src = open(os.path.join(CSRC, "internal.h")).read()
    return int(re.search(r"constexpr int CONV_DEFAULT_VARIANT = (\d+);", src).group(1))


def _ring_case(variant):
    """Template arguments (M, NW, G, OCC, NBUF, SCHED, STG, ALG) of a ring-kernel variant."""
    src = open(os.path.join(CSRC, "k_conv.hip")).read()
    m = re.search(r"NRX_RING_CASE\(%d,\s*([0-9,\s]+)\)" % variant, src)
    assert m, f"variant {variant} is not a ring-kernel case"
    return [int(x) for x in m.group(1).split(",")]


def test_kernel_trace_holds_the_default_residual_conv():
    args = _ring_case(_default_variant())
    name = "conv3x3_ring_kernel<unsigned short, 2, " + ", ".join(str(a) for a in args) + ">"   # EPI_RESID = 2
    txt = open(os.path.join(PROF, "nrx_forward_bf16_m273_kernel_stats.txt")).read()
    assert f"BF16 conv_b = {name}" in txt
    rows = [l for l in txt.splitlines() if l.startswith(name)]
    assert len(rows) == 1
    calls, avg_us = int(rows[0].split()[-4]), float(rows[0].split()[-3])
    assert calls > 0 and avg_us > 0.0
    # the stated fraction of the BF16 peak follows from the row's average: 294,912 FLOP x 5,870,592 rows
    frac = 294912 * 5870592 / (avg_us * 1e-6) / 2.5e15
    assert f"{frac:.3f} of 2.5 PFLOP/s" in txt


def test_traffic_record_covers_the_default_variant():
    d = json.load(open(os.path.join(PROF, "conv_b_bf16_m273_traffic.json")))
    v = str(_default_variant())
    assert v in d["hbm_bytes_per_launch"]
    # measured traffic is at least the algorithmic bytes (a in, residual in, h out: 768 B per row)
    assert d["algorithmic_bytes_per_launch"] == 768 * 5870592
    assert d["hbm_bytes_per_launch"][v] >= d["algorithmic_bytes_per_launch"]
    for src in d["sources"]:
        assert os.path.exists(os.path.join(ROOT, src))


def test_every_summary_names_its_command():
    for f in sorted(os.listdir(PROF)):
        if f.endswith(".txt"):
            txt = open(os.path.join(PROF, f)).read()
            assert "rocprofv3" in txt and "--" in txt, f
