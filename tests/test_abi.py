"""CPU tests of the C ABI: symbols, host-side plan logic and argument checks (no GPU calls)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1911_01353_amd as J
from paper_1911_01353_amd import _lib
from oracle.grid import Grid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(jerk_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = J.load()
    names = _declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    assert set(names) <= set(_lib.SIGNATURES)


def test_status_strings_and_version():
    assert _lib.status_str(0) == "JERK_OK"
    assert _lib.status_str(-2) == "JERK_ENOMEM"
    assert J.version().startswith("jerk-mi355x")


@pytest.mark.parametrize("zmax,wmax", [(20, 60), (100, 300), (200, 600), (50, 150), (0, 0), (7, 45)])
def test_plan_lattice_matches_oracle(zmax, wmax):
    p = J.Plan(4096, zmax, wmax, 2.0, 20.0)
    g = Grid(zmax, wmax, 2.0, 20.0)
    info = p.info()
    assert (info["n_z"], info["n_w"], info["n_templates"]) == (g.n_z, g.n_w, g.n_templates)
    ts = range(g.n_templates) if g.n_templates < 500 else np.linspace(0, g.n_templates - 1, 400).astype(int)
    for t in ts:
        zb, w, h, grp, slot = p.template(int(t))
        assert (zb, w, h) == g.params(int(t))
    assert info["max_taps"] == 2 * int(g.half_widths().max())


def test_groups_partition_templates_by_width():
    p = J.Plan(1 << 20, 200, 600, 2.0, 20.0, path="auto")
    members = p.members()
    assert sorted(members.tolist()) == list(range(p.info()["n_templates"]))
    prev = 0
    for gi, g in enumerate(p.groups()):
        assert g["taps"] % 16 == 0 and g["taps"] > prev
        prev = g["taps"]
        ms = members[g["first_member"]:g["first_member"] + g["n_members"]]
        assert np.all(np.diff(ms) > 0)
        for t in ms[:: max(1, len(ms) // 7)]:
            zb, w, h, grp, slot = p.template(int(t))
            assert grp == gi and g["taps"] - 16 < 2 * h <= g["taps"]
        # AUTO: narrow groups on the MFMA path, wide ones on the FFT path
        assert g["path"] == (J.PATH_GEMM_SPLIT_BF16 if g["taps"] <= 96 else J.PATH_FFT_FP32)


def test_default_templates_per_block_follows_the_launch_size():
    """Plan default: per group the largest of 64, 32, 16, 8 templates per block whose launch over
    the whole group has at least 4096 workgroups at the plan's nbins, else 4 (explicit values win)."""
    for n, z, w in ((1 << 22, 200, 600), (1 << 20, 100, 300), (1 << 15, 20, 60), (9001, 40, 120)):
        p = J.Plan(n, z, w, 2.0, 20.0, path="fft")
        for g in p.groups():
            U = g["seg_len"] - g["taps"] + 1
            n_seg = -(-n // U)
            want = next((t for t in (64, 32, 16, 8) if n_seg * -(-g["n_members"] // t) >= 4096), 4)
            assert g["templates_per_block"] == want, (n, g)
        p.close()
    assert {g["templates_per_block"] for g in J.Plan(1 << 22, 200, 600, 2.0, 20.0, path="fft").groups()} == {64}
    assert {g["templates_per_block"] for g in J.Plan(1 << 15, 20, 60, 2.0, 20.0, path="fft").groups()} == {4}
    fixed = J.Plan(1 << 22, 200, 600, 2.0, 20.0, path="fft", templates_per_block=16)
    assert {g["templates_per_block"] for g in fixed.groups()} == {16}


def test_bank_layout_grows_with_overrides():
    p = J.Plan(1 << 16, 20, 60, 2.0, 20.0, path="fft")
    b0 = p.info()["bank_bytes"]
    p.set_group(0, 4096, 4, "fft", 8)
    assert p.info()["bank_bytes"] > b0
    g0 = p.group(0)
    assert (g0["seg_len"], g0["templates_per_block"], g0["fft_ept"]) == (4096, 4, 8)


@pytest.mark.parametrize("kwargs,status", [
    (dict(dz=0.0), J.JERK_EINVAL),
    (dict(dw=-1.0), J.JERK_EINVAL),
    (dict(numbetween=4), J.JERK_EINVAL),
    (dict(seg_len=3000), J.JERK_EINVAL),
    (dict(seg_len=512, zmax=200, wmax=600), J.JERK_EINVAL),  # segment too short for the widest group
    (dict(margin=-1), J.JERK_EINVAL),
    (dict(path=7), J.JERK_EINVAL),
    (dict(path="split_bf16", zmax=400, wmax=1800), -6),   # wider than the MFMA kernels accept
])
def test_plan_argument_errors(kwargs, status):
    args = dict(nbins=1024, zmax=20, wmax=60, dz=2.0, dw=20.0)
    args.update(kwargs)
    with pytest.raises(J.JerkError) as ei:
        J.Plan(**args)
    assert ei.value.status == status
    assert J.load().jerk_last_error().decode()


def test_search_argument_errors_are_synchronous():
    """Bad arguments are rejected before anything touches a device."""
    lib = J.load()
    p = J.Plan(1024, 20, 60)
    fake = C.c_void_p(0x100000)  # never dereferenced: validation fails first
    null = C.c_void_p(0)
    # ld too small
    assert lib.jerk_search(p.handle, fake, fake, 1024, fake, 100, 0, 1, null, 0, null) == J.JERK_EINVAL
    # template range outside the plan
    assert lib.jerk_search(p.handle, fake, fake, 1024, fake, 2048, 0, 148, null, 0, null) == J.JERK_EINVAL
    assert lib.jerk_search(p.handle, fake, fake, 1024, fake, 2048, 5, 4, null, 0, null) == J.JERK_EINVAL
    # NULL pointers
    assert lib.jerk_search(p.handle, null, fake, 1024, fake, 2048, 0, 1, null, 0, null) == J.JERK_EINVAL
    # bank too small
    assert lib.jerk_templates_build(p.handle, fake, 16, null) == J.JERK_ENOMEM
    # NULL plan everywhere
    assert lib.jerk_plan_info(None, None) == J.JERK_EINVAL


def test_batch_argument_errors_without_gpu():
    lib = J.load()
    fake = C.c_void_p(0x100000)
    null = C.c_void_p(0)
    item = (J._lib.BatchItem * 1)()
    item[0].spec = 0x100000
    item[0].nbins = 4096
    item[0].plane = 0x200000
    item[0].ld = 8192
    auto = J.Plan(4096, 20, 60, path="auto")   # MFMA groups: not batchable
    assert lib.jerk_batch_search(auto.handle, fake, item, 1, 0, 147, fake, 1 << 20, 0, null) == J.JERK_EINVAL
    fft = J.Plan(4096, 20, 60, path="fft", seg_len=1024)
    need = lib.jerk_batch_workspace_bytes(fft.handle, 1)
    assert need > 0
    assert lib.jerk_batch_search(fft.handle, fake, item, 1, 0, 147, fake, need - 1, 0, null) == J.JERK_ENOMEM
    assert lib.jerk_batch_search(fft.handle, fake, item, 1, 0, 147, fake, need, 7, null) == J.JERK_EINVAL
    item[0].ld = 100
    assert lib.jerk_batch_search(fft.handle, fake, item, 1, 0, 147, fake, need, 0, null) == J.JERK_EINVAL
    # one key per FFT segment of the narrowest-output (widest) group
    assert fft.keys_per_row(4096) == -(-4096 // (1024 - 64 + 1))


def test_candidate_entry_points_validate_on_the_host():
    """Argument errors and empty slabs are decided before any device call."""
    import ctypes as C
    from paper_1911_01353_amd import _lib
    lib = _lib.load()
    one = C.c_void_p(1)
    assert lib.jerk_stats_workspace_bytes(0, 100) == 0
    assert lib.jerk_stats_workspace_bytes(3, 0) == 0
    assert lib.jerk_stats_workspace_bytes(4, 1 << 23) >= 4 * 24
    assert lib.jerk_plane_stats(None, 10, 0, 10, None, None, 0, None) == _lib.JERK_OK
    assert lib.jerk_plane_stats(one, 5, 2, 10, one, one, 1 << 20, None) == _lib.JERK_EINVAL
    assert lib.jerk_plane_stats(None, 10, 2, 10, one, one, 1 << 20, None) == _lib.JERK_EINVAL
    f = lib.jerk_find_candidates
    assert f(None, 10, 0, 10, None, 3.0, None, 0, None, 10, None, None) == _lib.JERK_OK
    assert f(one, 10, 2, 10, one, float("nan"), None, 0, one, 10, one, None) == _lib.JERK_EINVAL
    assert f(one, 10, 2, 10, one, 3.0, None, 0, None, 10, one, None) == _lib.JERK_EINVAL
    assert f(one, 10, 2, 10, one, 3.0, None, -1, one, 10, one, None) == _lib.JERK_EINVAL
    assert f(one, 1 << 32, 2, 1 << 32, one, 3.0, None, 0, one, 10, one, None) == _lib.JERK_EINVAL
    assert f(one, 10, 2, 10, one, 3.0, None, 0, one, -1, one, None) == _lib.JERK_EINVAL


def test_spectrum_entry_point_validates_on_the_host():
    import ctypes as C
    from paper_1911_01353_amd import _lib
    lib = _lib.load()
    one = C.c_void_p(256)
    assert lib.jerk_spectrum_workspace_bytes(1 << 23) >= (1 << 22) * 32
    for bad in (0, 2, 3, 6, 1000):
        assert lib.jerk_spectrum_workspace_bytes(bad) == 0
    assert lib.jerk_spectrum_prepare(one, 1000, one, one, 1 << 30, None) == _lib.JERK_EUNSUPPORTED
    assert lib.jerk_spectrum_prepare(one, 2, one, one, 1 << 30, None) == _lib.JERK_EINVAL
    assert lib.jerk_spectrum_prepare(None, 1024, one, one, 1 << 30, None) == _lib.JERK_EINVAL
    assert lib.jerk_spectrum_prepare(C.c_void_p(260), 1024, one, one, 1 << 30, None) == _lib.JERK_EINVAL
    assert lib.jerk_spectrum_prepare(one, 1024, one, one, 16, None) == _lib.JERK_ENOMEM


def test_harmonic_shape_matches_the_oracle_and_validates():
    import ctypes as C
    from paper_1911_01353_amd import _lib
    from oracle import Grid
    from oracle.harmonics import fundamental_shape
    for zmax, wmax, n_r, H in [(200.0, 600.0, 1 << 23, 2), (200.0, 600.0, 1 << 23, 3), (20.0, 60.0, 65536, 4),
                               (24.0, 80.0, 8192, 4), (50.0, 150.0, 1000, 1), (6.0, 0.0, 17, 8)]:
        plan = J.Plan(1024, zmax, wmax, 2.0, 20.0, path="fft")
        assert plan.harmonic_shape(n_r, H) == fundamental_shape(Grid(zmax, wmax, 2.0, 20.0), n_r, H)
        plan.close()
    plan = J.Plan(1024, 21.0, 60.0, 2.0, 20.0, path="fft")
    lib = _lib.load()
    a, b, c = C.c_int32(), C.c_int32(), C.c_int64()
    assert lib.jerk_harmonic_shape(plan.handle, 100, 2, C.byref(a), C.byref(b), C.byref(c)) == _lib.JERK_EUNSUPPORTED
    plan.close()
    plan = J.Plan(1024, 20.0, 60.0, 2.0, 20.0, path="fft")
    assert lib.jerk_harmonic_shape(plan.handle, 100, 0, C.byref(a), C.byref(b), C.byref(c)) == _lib.JERK_EINVAL
    assert lib.jerk_harmonic_shape(plan.handle, 100, 65, C.byref(a), C.byref(b), C.byref(c)) == _lib.JERK_EINVAL
    one = C.c_void_p(256)
    assert lib.jerk_harmonic_sum(plan.handle, None, 100, 100, 2, one, 100, None) == _lib.JERK_EINVAL
    assert lib.jerk_harmonic_sum(plan.handle, one, 99, 100, 2, one, 100, None) == _lib.JERK_EINVAL
    assert lib.jerk_harmonic_sum(plan.handle, one, 100, 100, 2, one, 49, None) == _lib.JERK_EINVAL
    plan.close()


def test_search_candidates_validates_on_the_host():
    """Argument, path and workspace errors of the fused search are decided before any device call."""
    import ctypes as C
    from paper_1911_01353_amd import _lib
    lib = _lib.load()
    one = C.c_void_p(1)
    plan = J.Plan(4096, 20.0, 60.0, 2.0, 20.0, path="fft")
    T = plan.info()["n_templates"]
    wsb = lib.jerk_search_candidates_workspace_bytes
    assert wsb(None, 4096, 0, T, 2.7, 0) == 0
    assert wsb(plan.handle, 0, 0, T, 2.7, 0) == 0
    assert wsb(plan.handle, 4096, 0, T + 1, 2.7, 0) == 0
    assert wsb(plan.handle, 4096, 0, T, 2.7, -1) == 0
    assert wsb(plan.handle, 4096, 0, T, float("nan"), 0) == 0
    small = wsb(plan.handle, 4096, 0, T, 50.0, 0)
    assert small > 0
    assert wsb(plan.handle, 4096, 0, T, 0.0, 0) > small           # a low level stages more
    assert wsb(plan.handle, 4096, 0, T, 50.0, 1000) > wsb(plan.handle, 4096, 0, T, 50.0, 1) > 0  # slots per tile
    assert wsb(plan.handle, 1 << 20, 0, T, 50.0, 0) > small
    f = lib.jerk_search_candidates

    def call(p=plan.handle, bank=one, spec=one, n=4096, tb=0, te=T, k=2.0, pre=2.7, staged=0, out=one, cap=10,
             count=one, ws=one, wsn=1 << 40):
        return f(p, bank, spec, n, tb, te, k, pre, staged, None, out, cap, count, ws, wsn, None)

    assert call(tb=5, te=5, bank=None, spec=None, out=None, count=None, ws=None) == _lib.JERK_OK
    assert call(p=None) == _lib.JERK_EINVAL
    assert call(tb=-1) == _lib.JERK_EINVAL and call(te=T + 1) == _lib.JERK_EINVAL
    assert call(n=0) == _lib.JERK_EINVAL and call(n=1 << 31) == _lib.JERK_EINVAL
    assert call(k=float("nan")) == _lib.JERK_EINVAL and call(pre=float("inf")) == _lib.JERK_EINVAL
    assert call(staged=-1) == _lib.JERK_EINVAL and call(cap=-1) == _lib.JERK_EINVAL
    assert call(out=None) == _lib.JERK_EINVAL and call(count=None) == _lib.JERK_EINVAL
    assert call(wsn=16) == _lib.JERK_ENOMEM
    mfma = J.Plan(4096, 20.0, 60.0, 2.0, 20.0, path="split_bf16")
    Tm = mfma.info()["n_templates"]
    slab = wsb(mfma.handle, 4096, 0, Tm, 2.7, 0)
    biggest = max(g["n_members"] for g in mfma.groups())
    assert slab >= biggest * 2 * 4096 * 4     # MFMA groups go through a plane slab (a whole group fits)
    assert call(p=mfma.handle, te=Tm, wsn=slab - 1) == _lib.JERK_ENOMEM


def test_plain_c_caller_is_built():
    """The C caller of the GPU tests links against the library and rejects bad arguments before
    any device call."""
    import subprocess
    demo = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "jerk_demo")
    assert os.path.exists(demo), "tests/c_abi/jerk_demo is missing: build the library first"
    r = subprocess.run([demo], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage" in r.stderr


def test_oversized_search_is_refused_before_anything_is_queued():
    """A spectrum so long that a width group's FFT tiles exceed one launch: EINVAL from the
    host-side check, before any group is queued (no device call is made here)."""
    import ctypes as C
    from paper_1911_01353_amd import _lib
    lib = _lib.load()
    one = C.c_void_p(8)
    plan = J.Plan(4096, 200.0, 600.0, 2.0, 20.0, path="fft")
    T = plan.info()["n_templates"]
    n = 1 << 36
    assert lib.jerk_search(plan.handle, one, one, n, one, 2 * n, 0, T, None, 0, None) == _lib.JERK_EINVAL
    assert "too large" in lib.jerk_last_error().decode()


def test_search_peaks_validates_on_the_host():
    import ctypes as C
    from paper_1911_01353_amd import _lib
    lib = _lib.load()
    one = C.c_void_p(8)
    plan = J.Plan(4096, 20.0, 60.0, 2.0, 20.0, path="auto")
    T = plan.info()["n_templates"]
    assert lib.jerk_search_peaks_workspace_bytes(plan.handle, 0, T) == 8 * T
    assert lib.jerk_search_peaks_workspace_bytes(plan.handle, 0, T + 1) == 0
    f = lib.jerk_search_peaks
    assert f(plan.handle, None, None, 4096, 3, 3, None, None, 0, None) == _lib.JERK_OK
    assert f(None, one, one, 4096, 0, T, one, one, 8 * T, None) == _lib.JERK_EINVAL
    assert f(plan.handle, one, one, 0, 0, T, one, one, 8 * T, None) == _lib.JERK_EINVAL
    assert f(plan.handle, one, one, 4096, 0, T, None, one, 8 * T, None) == _lib.JERK_EINVAL
    assert f(plan.handle, one, C.c_void_p(12), 4096, 0, T, one, one, 8 * T, None) == _lib.JERK_EINVAL
    assert f(plan.handle, one, one, 4096, 0, T, one, one, 8 * T - 1, None) == _lib.JERK_ENOMEM


def test_batch_search_candidates_validates_on_the_host():
    import ctypes as C
    from paper_1911_01353_amd import _lib
    lib = _lib.load()
    plan = J.Plan(4096, 20.0, 60.0, 2.0, 20.0, path="fft")
    T = plan.info()["n_templates"]
    items = (_lib.BatchCandItem * 2)()
    for i, n in enumerate((4096, 1 << 16)):
        items[i].spec, items[i].nbins, items[i].out, items[i].capacity, items[i].count = 8, n, 8, 10, 8
    one = lib.jerk_search_candidates_workspace_bytes(plan.handle, 1 << 16, 0, T, 2.7, 0)
    assert lib.jerk_batch_search_candidates_workspace_bytes(plan.handle, items, 2, 0, T, 2.7, 0) == one
    f = lib.jerk_batch_search_candidates
    ws = C.c_void_p(8)
    assert f(plan.handle, ws, items, 0, 0, T, 2.0, 2.7, 0, ws, 0, None) == _lib.JERK_OK
    assert f(None, ws, items, 2, 0, T, 2.0, 2.7, 0, ws, one, None) == _lib.JERK_EINVAL
    assert f(plan.handle, ws, None, 2, 0, T, 2.0, 2.7, 0, ws, one, None) == _lib.JERK_EINVAL
    items[1].nbins = 0
    assert f(plan.handle, ws, items, 2, 0, T, 2.0, 2.7, 0, ws, one, None) == _lib.JERK_EINVAL
    items[1].nbins = 1 << 16
    items[1].count = None
    assert f(plan.handle, ws, items, 2, 0, T, 2.0, 2.7, 0, ws, one, None) == _lib.JERK_EINVAL
    items[1].count = 8
    # the second item needs more than the first: a workspace sized for the first is refused up front
    small = lib.jerk_search_candidates_workspace_bytes(plan.handle, 4096, 0, T, 2.7, 0)
    assert f(plan.handle, ws, items, 2, 0, T, 2.0, 2.7, 0, ws, small, None) == _lib.JERK_ENOMEM


STRUCTS = {
    "PlanDesc": "jerk_plan_desc", "PlanInfo": "jerk_plan_info_t", "GroupInfo": "jerk_group_info_t",
    "BatchItem": "jerk_batch_item", "BatchCandItem": "jerk_batch_cand_item", "Peak": "jerk_peak",
    "ServeDesc": "jerk_serve_desc", "Request": "jerk_request", "Top": "jerk_top", "Result": "jerk_result",
    "ServeStats": "jerk_serve_stats",
}


def test_binding_struct_layouts_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets of its C struct."""
    import shutil
    import subprocess

    from paper_1911_01353_amd import _lib

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(shutil.which("hipcc") or "/opt/rocm/bin/hipcc")))
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "jerk.h"', "int main(void) {"]
    for py, c in STRUCTS.items():
        lines.append(f'  printf("{py} size %zu\\n", sizeof({c}));')
        for f, _ in getattr(_lib, py)._fields_:
            lines.append(f'  printf("{py} {f} %zu\\n", offsetof({c}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", inc, "-I", os.path.join(rocm, "include"),
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    got = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    want = []
    for py in STRUCTS:
        cls = getattr(_lib, py)
        want.append(f"{py} size {C.sizeof(cls)}")
        want += [f"{py} {f} {getattr(cls, f).offset}" for f, _ in cls._fields_]
    assert got[:-1] == want
