"""The benchmark's bookkeeping (CPU only): committed counter traffic is used
only for the sources and kernel choice it was measured with, and the tuning
cache holds well-formed choices."""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    import bench as b
    return b


def test_traffic_needs_matching_choice(bench):
    """Each traffic summary matches its own choice line and no other choice."""
    for wl, n in (("cavity", 1024), ("cavity", 2048), ("powerlaw", 2048)):
        path = os.path.join(ROOT, "profiles", f"fused_step_{wl}{n}_traffic.md")
        txt = open(path).read()
        line = [ln for ln in txt.splitlines() if ln.startswith("choice:")][0]
        v, tw, pf, sx, sy = line.split(":", 1)[1].split()
        choice = (int(v), int(tw), int(pf), float(sx), float(sy))
        got = bench.measured_traffic(wl, n, choice)
        sha = [ln for ln in txt.splitlines() if ln.startswith("kernel_sha:")][0].split()[1]
        if sha != bench.kernel_sha():
            assert got is None      # the sources changed since the counters were taken
            continue
        assert got is not None and got > 2 * 80 * n * n    # above the algorithmic bytes
        assert bench.measured_traffic(wl, n, (choice[0], choice[1], 3 if choice[2] == 2 else 2) + choice[3:]) is None
        assert bench.measured_traffic(wl, n, choice[:3] + (choice[3] + 0.5, choice[4])) is None
        assert bench.measured_traffic(wl, n, None) is None
    assert bench.measured_traffic("taylor-green", 777, (1, 64, 2, 1.0, 1.0)) is None


def test_digest_covers_the_step_sources(bench, tmp_path, monkeypatch):
    """Changing any of the step's sources changes the digest."""
    import shutil
    files = tuple(bench.step_sources())
    assert "mdf_fused_impl.hpp" in files and "mdf_fused_w256p.hip" in files and "mdf_api.hip" in files
    d = tmp_path / "csrc"
    d.mkdir()
    for f in files:
        shutil.copy(os.path.join(bench.CSRC, f), d / f)
    monkeypatch.setattr(bench, "CSRC", str(d))
    base = bench.kernel_sha()
    for f in files:
        p = d / f
        old = p.read_bytes()
        p.write_bytes(old + b"\n")
        assert bench.kernel_sha() != base, f
        p.write_bytes(old)
    assert bench.kernel_sha() == base


def test_tuning_cache_entries_are_valid():
    cache = json.load(open(os.path.join(ROOT, "paper_2306_08216_amd", "tuning_mi355x.json")))
    assert cache
    for key, entry in cache.items():
        ch = entry["choice"]
        if "count" in entry:
            v, pf, rounds, tw = ch          # batch: (variant, prefetch, rounds, tile_w)
            assert key.startswith(f"{entry['count']}x-")
            assert v in (1, 2) and pf in (2, 3) and 1 <= rounds <= 8 and tw in (64, 128, 256)
            assert not (tw == 256 and pf != 2) and not (v == 2 and tw != 64)
        else:
            v, tw, pf, sx, sy = ch          # single run: (variant, tile_w, prefetch, x scale, y scale)
            assert key.startswith(f"{entry['nx']}x{entry['ny']}-")
            assert v in (1, 2) and tw in (64, 128, 256) and pf in (2, 3)
            assert not (v == 2 and tw != 64)
            assert 0.0 <= sx <= 10.0 and 0.0 <= sy <= 10.0
