"""The C-ABI library loads and exports every function include/fhv.h declares;
host-side argument checks reject bad calls before anything is launched.
No compute call is made, so these run without a GPU."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fhv.h")


def declared() -> list[str]:
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(fhv_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def F():
    from paper_2211_15460_amd import fhv
    if not os.path.exists(fhv.LIB_PATH):
        pytest.fail("libfhv.so is not built")
    fhv.lib()
    return fhv


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("fhv_capture", "fhv_compact", "fhv_splat", "fhv_create", "fhv_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported(F):
    out = subprocess.run(["nm", "-D", "--defined-only", F.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    for n in declared():
        assert n in exported, n
        getattr(F.lib(), n)
    assert set(F.EXPORTS) <= set(declared())


def test_library_links_only_the_hip_runtime(F):
    out = subprocess.run(["readelf", "-d", F.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    needed = re.findall(r"\[(.*?)\]", "\n".join(ln for ln in out.splitlines() if "NEEDED" in ln))
    assert any(n.startswith("libamdhip64") for n in needed)
    assert not any("torch" in n or "c10" in n or "python" in n for n in needed)


def test_status_strings(F):
    L = F.lib()
    assert L.fhv_status_str(0) == b"ok"
    assert L.fhv_status_str(-1) == b"invalid argument"
    assert L.fhv_status_str(-2) == b"workspace too small"
    assert L.fhv_status_str(1001) == b"HIP runtime error"


def test_workspace_queries(F):
    L = F.lib()
    d = F.desc(F.FHV_PPFL, 128, 128)
    assert L.fhv_capture_workspace(C.byref(d), 64) >= 64 * 128
    assert L.fhv_capture_workspace(C.byref(d), 0) > 0
    assert L.fhv_compact_workspace(C.byref(d), 1 << 18) >= 16 << 18
    p = F.desc(F.FHV_POFL, levels=9)
    assert L.fhv_compact_workspace(C.byref(p), 1000) >= 8 ** 9 // 8
    for bad in (F.desc(7, 1, 1), F.desc(F.FHV_PPFL, 0, 5), F.desc(F.FHV_PPFL, 20000, 5),
                F.desc(F.FHV_POFL, levels=0), F.desc(F.FHV_POFL, levels=12)):
        assert L.fhv_capture_workspace(C.byref(bad), 10) == 0
        assert L.fhv_compact_workspace(C.byref(bad), 10) == 0


def test_bad_arguments_rejected_before_launch(F):
    L = F.lib()
    d = F.desc(F.FHV_PPFL, 8, 8)
    m = F.Mesh_(None, None, None, None, 0, 0)
    ls = F.Lists_(None, 64, None, 0, None, None)
    assert L.fhv_capture(None, C.byref(m), C.byref(d), C.byref(ls), None, 0, None) == -1
    assert L.fhv_compact(None, C.byref(ls), C.byref(d), None, None, 0, None) == -1
    assert L.fhv_splat(None, None, C.byref(d), None, 0, None, None, None, None, None, 0, None) == -1
    assert L.fhv_create(None, 0) == -1


def test_batch_workspace_shapes(F):
    bm = F.BatchMesh_(None, None, None, None, None, 1000, 5000, 4, 9)
    bv = F.BatchViews_(None, 8, 1280, 720, 1)
    assert L_ws(F, bm, bv, 1 << 20) > (1 << 20) * 16
    for bad_m, bad_v in (((0, 9), (8, 1280, 720, 1)), ((4, 0), (8, 1280, 720, 1)), ((4, 12), (8, 1280, 720, 1)),
                         ((1 << 20, 9), (8, 1280, 720, 1)), ((4, 9), (0, 1280, 720, 1)),
                         ((4, 9), (33, 1280, 720, 1)), ((4, 9), (8, 0, 720, 1)), ((4, 9), (8, 1280, 720, 0)),
                         ((4, 9), (8, 1280, 720, 65))):
        m = F.BatchMesh_(None, None, None, None, None, 1000, 5000, *bad_m)
        v = F.BatchViews_(None, *bad_v)
        assert L_ws(F, m, v, 1000) == 0


def L_ws(F, m, v, cap):
    return F.lib().fhv_batch_workspace(C.byref(m), C.byref(v), cap)


def test_probe_rejects_missing_context(F):
    L = F.lib()
    assert L.fhv_probe(None, 0, None, 4096, 128, 1, None) == -1
