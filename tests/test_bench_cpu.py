"""Host-side checks of the benchmark's accounting (no GPU): which profiled
kernel instantiation stands for a phase, the algorithmic bytes of the two
contact searches, and the counter summaries' guard by kernel source."""
import hashlib
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_is_picks_the_half_search_force_instantiation():
    assert bench.kernel_is("k_force<float, 8>", "k_force", "float")
    assert bench.kernel_is("k_force<double, 16>", "k_force", "double")
    # the full search's force kernel (no list slots) is not the headline's
    assert not bench.kernel_is("k_force<float, 0>", "k_force", "float")
    assert not bench.kernel_is("k_force<double, 8>", "k_force", "float")
    assert not bench.kernel_is("k_force_thread<float>", "k_force", "float")
    assert bench.kernel_is("k_detect_half<8, false>", "k_detect_half", "float")
    assert not bench.kernel_is("k_detect<8, false>", "k_detect_half", "float")


def test_kernel_bytes_of_the_two_searches():
    n, m, mo = 1000, 300, 250
    # half search: records 48, cell bounds 8, per contact list entry 8 and
    # counter 4; its force kernel adds the counter read and reset and, per
    # contact, the entry read and the partner index written
    assert bench.kernel_bytes("detect", n, m, mo, False, 20) == 56 * n + 12 * m
    assert bench.kernel_bytes("detect", n, m, mo, False, 20, half=False) == 48 * n + 4 * m
    full = bench.kernel_bytes("force", n, m, mo, False, 20, half=False)
    half = bench.kernel_bytes("force", n, m, mo, False, 20)
    assert full == 184 * n + 36 * m + 28 * mo
    assert half - full == 8 * n + 12 * m
    # the radix sort's input: key and index instead of the key before the
    # step, and the old cell's bound read
    radix = bench.kernel_bytes("force", n, m, mo, False, 20, half=False, merge=False)
    assert radix - full == 8 * n
    assert bench.kernel_bytes("force", n, m, mo, True, 20, force_out=True, half=False) == full + 48 * n


def test_counter_summaries_match_the_kernel_source_or_are_ignored():
    src = os.path.join(ROOT, "paper_1503_03553_amd", "csrc", "dem_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for name in ("hbm_traffic_dilute_1m.json", "valu_dilute_1m.json"):
        path = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(path):
            # no counter summary: the figures it would give are null
            if name.startswith("hbm"):
                assert bench.measured_traffic("k_force", "float") is None
            else:
                assert bench.valu_insts("force", "float") is None
            continue
        rec = json.load(open(path))
        if rec["kernels_source_sha256"] == sha:
            continue
        # a stale summary is never used
        if name.startswith("hbm"):
            assert bench.measured_traffic("k_force", "float") is None
        else:
            assert bench.valu_insts("force", "float") is None
    traffic = bench.measured_traffic("k_force", "float")
    if traffic is not None and os.path.exists(os.path.join(ROOT, "profiles",
                                                           "hbm_traffic_dilute_1m.json")):
        rec = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic_dilute_1m.json")))
        key = [k for k in rec["per_launch_bytes"] if bench.kernel_is(k, "k_force", "float")]
        assert len(key) == 1 and traffic == rec["per_launch_bytes"][key[0]]


def test_method_bytes_count_the_method_not_the_implementation():
    n, m, mo = 1000, 300, 250
    # contact search: record 28, cell ranges 8, row 4, partner index 4 per contact
    assert bench.method_bytes("detect", n, m, mo, False, 20) == 40 * n + 4 * m
    # history match + contact law + sums + integration + hashing in one pass:
    # 176 per particle, 4 + 28 per contact, 28 per old contact; F/T only when stored
    assert bench.method_bytes("force", n, m, mo, False, 20) == 176 * n + 32 * m + 28 * mo
    assert bench.method_bytes("force", n, m, mo, True, 20, force_out=True) == \
        (176 + 48) * n + 32 * m + 28 * mo
    # the implementation moves more than the method needs in both kernels
    for ph in ("detect", "force"):
        assert bench.kernel_bytes(ph, n, m, mo, False, 20) > bench.method_bytes(ph, n, m, mo,
                                                                                False, 20)
    # the kernels move positions only: their own counts are below the
    # method's 168 for the gather into cell order (after the merge sort the
    # placement writes the FP32 records and the reorder only the bounds)
    assert bench.method_bytes("reorder", n, m, mo, False, 20, merge=False) == 68 * n
    assert bench.method_bytes("reorder", n, m, mo, False, 20) == 12 * n
    assert bench.method_bytes("sort", n, m, mo, False, 20) == 60 * n
    assert bench.method_bytes("sort", n, m, mo, False, 20) + \
        bench.method_bytes("reorder", n, m, mo, False, 20) < 168 * n
    rows = bench.phase_rows({"detect": (0.05, 1), "force": (0.07, 1)}, n, m, mo, False, 20)
    c = bench.contact_kernels_of(rows)
    assert c["bytes_per_step"] == 40 * n + 4 * m + 176 * n + 32 * m + 28 * mo
    assert abs(c["us_per_step"] - 120.0) < 1e-9
    r = bench.roofline_of(rows)
    assert r["kernel"] == "k_force" and r["overhead_bytes_per_launch"] == \
        bench.kernel_bytes("force", n, m, mo, False, 20) - r["bytes_per_launch"]
