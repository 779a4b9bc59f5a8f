"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/mdf.h declares, and rejects bad parameters before touching
the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdf_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2306_08216_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmdf.so is not built (run __graft_entry__.build())")
    _lib.lib()
    return _lib


def test_exports_every_declared_symbol(L):
    names = _declared("mdf.h")
    assert "mdf_init" in names and "mdf_step" in names and "mdf_moments" in names and "mdf_derived" in names
    raw = C.CDLL(L.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing
    # the binding wraps every declared call under the same name
    assert set(names) <= set(L.SIGNATURES), set(names) - set(L.SIGNATURES)


def _params(L, **kw):
    from paper_2306_08216_amd import problems as P
    from paper_2306_08216_amd.solver import params_of
    keep = []
    prob = P.taylor_green(16)
    for k, v in kw.items():
        setattr(prob, k, v)
    return params_of(prob, keep), keep


def test_workspace_size_and_validation(L):
    p, keep = _params(L)
    n = L.mdf_workspace_size(p)
    assert n >= 4 * 10 * 16 * 16 * 8
    for bad in (dict(nu=0.0), dict(cfl=-1.0), dict(eta=1.5), dict(nx=4), dict(pl_n=2.0),
                dict(pl_n=0.5, nu_min=0.0, nu_max=1.0), dict(inv_dx_x=np.ones(16), dx_min=0.0),
                dict(force_harmonic=2), dict(force_harmonic=True, force_omega=float("nan")),
                dict(force_harmonic=True, force_phase=float("inf")),
                dict(metric=np.ones((4, 16, 16)), dx_min=0.0),
                dict(metric=np.ones((4, 16, 16)), dx_min=0.1, inv_dx_x=np.ones(16)),
                dict(mass_source=np.zeros((16, 16)), pl_n=0.5, nu_min=1e-3, nu_max=1.0)):
        p, keep = _params(L, **bad)
        assert L.mdf_workspace_size(p) == 0, bad
    # a mass source adds one plane of nx*ny values
    p, keep = _params(L, mass_source=np.zeros((16, 16)))
    assert L.mdf_workspace_size(p) == n + 16 * 16 * 8


def test_init_rejects_bad_input_without_device_work(L):
    p, keep = _params(L, nu=-1.0)
    out = C.c_void_p()
    s = L.lib().mdf_init(C.byref(p), 1, 1, 1, 256, 1 << 30, None, C.byref(out))
    assert s == L.MDF_EINVAL and out.value is None
    assert "nu" in L.mdf_last_error(None)
    p, keep = _params(L)
    s = L.lib().mdf_init(C.byref(p), 1, 1, 1, 256, 16, None, C.byref(out))   # workspace too small
    assert s == L.MDF_EINVAL and "workspace" in L.mdf_last_error(None)
    s = L.lib().mdf_init(C.byref(p), 1, 1, 1, 257, 1 << 30, None, C.byref(out))  # misaligned
    assert s == L.MDF_EINVAL and "aligned" in L.mdf_last_error(None)


def test_null_context_calls(L):
    lib = L.lib()
    assert lib.mdf_step(None, 1) == L.MDF_EINVAL
    assert lib.mdf_moments(None, None, None, None) == L.MDF_EINVAL
    assert lib.mdf_derived(None, None, 1) == L.MDF_EINVAL
    assert lib.mdf_set_kernel(None, 1, 0, 0, 0) == L.MDF_EINVAL
    assert lib.mdf_dt(None) == 0.0 and lib.mdf_steps(None) == 0
    lib.mdf_destroy(None)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2306_08216_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()


@pytest.mark.parametrize("n,bc,variant,tile_w", [(1024, 1, 2, 64), (1024, 1, 1, 64), (2048, 1, 1, 64),
                                                 (1024, 0, 2, 64), (100, 1, 1, 128), (37, 0, 1, 64),
                                                 (4099, 1, 2, 64), (2048, 1, 1, 128), (2048, 1, 1, 256),
                                                 (300, 1, 1, 256), (5, 1, 1, 64), (5, 0, 2, 64),
                                                 (6, 1, 1, 256), (9, 0, 1, 128)])
def test_balanced_partition_covers_every_row_once(L, n, bc, variant, tile_w):
    """The launch plan of the fused step: every (strip, row) exactly once, at
    most one round of workgroups, and wall segments no taller than interior
    ones (their rows cost more)."""
    p, keep = _params(L, nx=n, ny=n + 3, bc_x=bc, bc_y=bc)
    slots = 1024
    segs = L.mdf_plan_segments(p, variant, tile_w, slots)
    assert segs
    tw = 64 if variant == 2 else tile_w
    nstrips = -(-n // (tw - 8))
    assert len(segs) <= max(slots, nstrips)
    cover = {}
    for s, y0, y1 in segs:
        assert 0 <= s < nstrips and 0 <= y0 < y1 <= n + 3
        cover.setdefault(s, []).append((y0, y1))
    assert sorted(cover) == list(range(nstrips))
    for s, iv in cover.items():
        iv.sort()
        assert iv[0][0] == 0 and iv[-1][1] == n + 3
        assert all(a[1] == b[0] for a, b in zip(iv, iv[1:]))   # contiguous, no overlap
    if bc and nstrips > 2 and n >= 1024:
        h_int = max(y1 - y0 for s, y0, y1 in segs if 0 < s < nstrips - 1)
        h_wall = max(y1 - y0 for s, y0, y1 in segs if s == 0)
        assert h_wall < h_int


def test_plan_rejects_bad_arguments(L):
    p, keep = _params(L)
    assert L.mdf_plan_segments(p, 0, 64, 1024) == []
    assert L.mdf_plan_segments(p, 1, 96, 1024) == []
    assert L.mdf_plan_segments(p, 1, 64, 0) == []


def test_batch_validation_without_device_work(L):
    from paper_2306_08216_amd import problems as P
    from paper_2306_08216_amd.solver import params_of
    keep = []
    good = [params_of(P.taylor_green(n), keep) for n in (16, 40, 64)]
    arr = (L.mdf_params * 3)(*good)
    n = L.mdf_batch_workspace_size(arr, 3)
    assert n >= 3 * sum(10 * ((m + 15) // 16 * 16) * m * 8 for m in (16, 40, 64))
    assert L.mdf_batch_workspace_size(arr, 0) == 0
    bad_wall = (L.mdf_params * 2)(good[0], params_of(P.cavity(32), keep))
    assert L.mdf_batch_workspace_size(bad_wall, 2) == 0
    mapped = P.taylor_green(32)
    mapped.inv_dx_x, mapped.dx_min = np.ones(32), 0.1
    assert L.mdf_batch_workspace_size((L.mdf_params * 2)(good[0], params_of(mapped, keep)), 2) == 0
    pl = P.taylor_green(32)
    pl.pl_n, pl.nu_min, pl.nu_max = 0.5, 1e-4, 1e-1
    assert L.mdf_batch_workspace_size((L.mdf_params * 2)(good[0], params_of(pl, keep)), 2) == 0
    osc = P.taylor_green(32)
    osc.fx, osc.force_harmonic, osc.force_omega = 1e-4, True, 0.3
    assert L.mdf_batch_workspace_size((L.mdf_params * 2)(good[0], params_of(osc, keep)), 2) == 0
    warped = P.warped_taylor_green(32)
    assert L.mdf_batch_workspace_size((L.mdf_params * 2)(good[0], params_of(warped, keep)), 2) == 0
    src = P.divergent_flow(32)
    src.force_x = src.force_y = None
    assert L.mdf_batch_workspace_size((L.mdf_params * 2)(good[0], params_of(src, keep)), 2) == 0
    out = C.c_void_p()
    arrp = (C.c_void_p * 3)()
    s = L.lib().mdf_batch_init(arr, 3, arrp, arrp, arrp, None, 0, None, C.byref(out))
    assert s == L.MDF_EINVAL and out.value is None
    assert L.lib().mdf_batch_step(None, 1) == L.MDF_EINVAL
    assert L.lib().mdf_batch_set_kernel(None, 1, 64, 2, 1) == L.MDF_EINVAL
    L.lib().mdf_batch_destroy(None)


@pytest.mark.parametrize("nx,ny,bc", [(32768, 6, 0), (32768, 5, 1), (6, 32768, 1), (5, 32768, 0)])
@pytest.mark.parametrize("variant,tile_w", [(1, 64), (1, 256), (2, 64)])
def test_partition_at_maximum_extent(L, nx, ny, bc, variant, tile_w):
    """The launch plan at the largest extent the boundary accepts on one axis:
    every (strip, row) exactly once, within the segment table."""
    p, keep = _params(L, nx=nx, ny=ny, bc_x=bc, bc_y=bc)
    segs = L.mdf_plan_segments(p, variant, tile_w, 1024)
    assert segs and len(segs) <= 4096
    nstrips = -(-nx // (tile_w - 8))
    cover = {}
    for s, y0, y1 in segs:
        assert 0 <= s < nstrips and 0 <= y0 < y1 <= ny
        cover.setdefault(s, []).append((y0, y1))
    assert sorted(cover) == list(range(nstrips))
    for iv in cover.values():
        iv.sort()
        assert iv[0][0] == 0 and iv[-1][1] == ny and all(a[1] == b[0] for a, b in zip(iv, iv[1:]))
