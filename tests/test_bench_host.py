"""Host logic of bench.py (no GPU): how the grouped solves partition the systems, and
that the roofline traffic recorded with the counters is used only for the kernel
source it was measured on."""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def systems(fields=4, masses=5):
    # (solver, rhs, seed, mass) in the benchmark's order: field-major
    return [(None, None, 2000 + f, 0.1 * k) for f in range(fields) for k in range(masses)]


def test_groups_hold_one_mass_each():
    syss = systems()
    parts = bench.group_parts(syss, bench.GROUPS)
    assert len(parts) == bench.GROUPS and all(len(p) == bench.GROUP_SIZE for p in parts)
    assert sorted(j for p in parts for j in p) == list(range(len(syss)))
    for p in parts:
        assert len({syss[j][3] for j in p}) == 1  # one mass per group
        assert len({syss[j][2] for j in p}) == len(p)  # every field once


def test_groups_cover_every_system_for_any_count():
    syss = systems()
    for ng in range(1, len(syss) + 1):
        parts = bench.group_parts(syss, ng)
        sizes = [len(p) for p in parts]
        assert len(parts) == ng and max(sizes) - min(sizes) <= 1
        assert sorted(j for p in parts for j in p) == list(range(len(syss)))
        # ranks (position in the field's mass list) never decrease along the groups
        flat = [j % 5 for p in parts for j in p]
        assert flat == sorted(flat)


def test_traffic_is_tied_to_the_kernel_source(tmp_path):
    good = bench.measured_traffic(bench.COUNTERS_MD_GROUP)
    assert good is not None and good > 0
    text = open(bench.COUNTERS_MD_GROUP).read()
    stale = tmp_path / "stale.md"
    stale.write_text(text.replace("kernel_source_sha256 = ", "kernel_source_sha256 = 0"))
    assert bench.measured_traffic(str(stale)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md")) is None
