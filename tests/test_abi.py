"""Host-side checks of the C ABI (no GPU needed).

  * the library loads and exports every function declared in include/md.h;
  * the ctypes mirrors of the md_* structures have the C layout (sizes and
    field offsets printed by a host-only program compiled against md.h);
  * argument validation returns the documented status codes before any launch.
"""

import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "md.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


@pytest.fixture(scope="module")
def A():
    from paper_1012_2677_amd import _abi

    _abi.lib()
    return _abi


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(md_\w+)\s*\(", text, re.M)))


def test_constants_match_headers(A):
    # every integer #define of the headers that the binding mirrors has the
    # header's value
    text = "".join(open(h).read() for h in HEADERS)
    seen = 0
    for name, expr in re.findall(r"^#define\s+(MD_\w+)\s+(\S[^/\n]*?)\s*(?:/\*.*)?$", text, re.M):
        expr = re.sub(r"\((?:u?int\d+_t|size_t)\)", "", expr)
        if not re.fullmatch(r"[-()\d\s<]+", expr):
            continue
        if hasattr(A, name):
            assert getattr(A, name) == eval(expr), name
            seen += 1
    assert seen >= 15


def test_exports_every_declared_symbol(A):
    names = declared_functions()
    assert len(names) >= 12
    lib = A.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(A.EXPORTED) == names


LAYOUT_PROG = r"""
#include <cstdio>
#include <cstddef>
#include "md.h"
#define OFF(T, f) std::printf(#T "." #f " %zu\n", offsetof(T, f))
int main() {
  std::printf("md_params %zu\n", sizeof(md_params));
  std::printf("md_cells %zu\n", sizeof(md_cells));
  std::printf("md_pairlist %zu\n", sizeof(md_pairlist));
  std::printf("md_timers %zu\n", sizeof(md_timers));
  std::printf("md_state %zu\n", sizeof(md_state));
  OFF(md_params, precision); OFF(md_params, resort_every); OFF(md_params, dt);
  OFF(md_cells, cell_of); OFF(md_cells, order);
  OFF(md_pairlist, cell_stride); OFF(md_pairlist, status); OFF(md_pairlist, tiled); OFF(md_pairlist, half);
  OFF(md_state, cells); OFF(md_state, list); OFF(md_state, energy); OFF(md_state, ws_bytes);
  OFF(md_state, timers); OFF(md_state, step); OFF(md_state, phase); OFF(md_state, list_valid);
  OFF(md_params, list_layout); OFF(md_params, tile_cells); OFF(md_state, list_tiled); OFF(md_state, tile_stage);
  OFF(md_state, tile_cells); OFF(md_params, step_run); OFF(md_params, build_waves);
  return 0;
}
"""


def test_struct_layout_matches_header(A):
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.cpp")
        exe = os.path.join(d, "layout")
        open(src, "w").write(LAYOUT_PROG)
        subprocess.run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                        "-I", "/opt/rocm/include", src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    got = {k: int(v) for k, v in got.items()}
    assert got["md_params"] == C.sizeof(A.MdParams)
    assert got["md_cells"] == C.sizeof(A.MdCells)
    assert got["md_pairlist"] == C.sizeof(A.MdPairlist)
    assert got["md_timers"] == C.sizeof(A.MdTimers)
    assert got["md_state"] == C.sizeof(A.MdState)
    for key, val in got.items():
        if "." in key:
            struct, field = key.split(".")
            cls = {"md_params": A.MdParams, "md_cells": A.MdCells, "md_pairlist": A.MdPairlist,
                   "md_state": A.MdState}[struct]
            assert getattr(cls, field).offset == val, key


def _params(A, n=4000, L=20.0, **kw):
    from paper_1012_2677_amd.engine import make_params

    return make_params(n, L, **kw)


def test_cell_dims_and_workspace(A):
    p = _params(A)
    assert A.md_cell_dims(p) == (7, 7, 7)
    assert A.md_workspace_bytes(p) > 4000 * 4
    p = _params(A, n=32_000_000, L=400.0)
    assert A.md_cell_dims(p) == (142, 142, 142)


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), -1), (dict(n=1 << 27), -1), (dict(L=8.0), -2), (dict(L=3000.0), -2),
    (dict(rc=3.0, rs=2.8), -1), (dict(eps=-1.0), -1), (dict(precision=7), -1),
    (dict(list_layout=3), -1), (dict(tile_cells=-1), -1), (dict(tile_cells=1024), -1),
    (dict(step_run=-1), -1), (dict(step_run=65), -1), (dict(build_waves=-1), -1), (dict(build_waves=3), -1),
])
def test_validation_codes(A, kw, code):
    fields = ("list_layout", "tile_cells", "step_run", "build_waves")
    p = _params(A, **{k: v for k, v in kw.items() if k != "precision" and k not in fields})
    if kw.get("precision") == 7:
        p.precision = 7
    for f in fields:
        if f in kw:
            setattr(p, f, kw[f])
    with pytest.raises(A.MdError) as e:
        A.md_cell_dims(p)
    assert e.value.code == code
    assert A.last_error()
    assert A.md_workspace_bytes(p) == 0


def test_null_pointers_rejected_before_launch(A):
    p = _params(A)
    cells = A.MdCells()
    with pytest.raises(A.MdError) as e:
        A.md_bin_cells(p, None, cells, None, 0, None)
    assert e.value.code == A.MD_ERR_ARG
    with pytest.raises(A.MdError) as e:
        A.md_bin_cells(p, 1 << 20, cells, None, 0, None)
    assert e.value.code == A.MD_ERR_ARG
    plist = A.MdPairlist()
    with pytest.raises(A.MdError) as e:
        A.md_forces(p, 1 << 20, cells, plist, 1 << 20, None, None, 0, None)
    assert e.value.code == A.MD_ERR_ARG
    state = A.MdState()
    with pytest.raises(A.MdError) as e:
        A.md_step(p, state, 10, 0, None, None)
    assert e.value.code == A.MD_ERR_ARG


def test_half_layout_accepted(A):
    p = _params(A, list_layout="half")
    assert p.list_layout == A.MD_LIST_HALF
    assert A.md_cell_dims(p) == (7, 7, 7)


def test_tiled_list_rejected_by_standalone_passes(A):
    # a state's tiled list holds tile offsets, not slots: the standalone
    # passes refuse it before any launch; the same list marked as slot
    # entries gets past the list check and fails on the workspace size
    p = _params(A)
    fake = 1 << 20  # never dereferenced: validation fails first
    cells = A.MdCells()
    for k, m in enumerate(A.md_cell_dims(p)):
        cells.ncell[k] = m
    cells.cell_of = cells.cell_xyz = cells.count = cells.start = cells.order = fake
    plist = A.MdPairlist()
    plist.offsets = plist.counts = plist.nbr = plist.status = fake
    plist.cell_stride = 64
    plist.capacity = 64 * 7 * 7 * 7
    calls = [
        lambda: A.md_forces(p, fake, cells, plist, fake, None, fake, 16, None),
        lambda: A.md_hvp(p, fake, cells, plist, fake, fake, None, fake, 16, None),
        lambda: A.md_param_grad(p, fake, cells, plist, fake, fake, 16, None),
        lambda: A.md_adjoint_kick(p, fake, cells, plist, fake, fake + 64, None, [0.0] * 5, fake, fake, 16, None),
    ]
    for tiled, code in ((1, A.MD_ERR_ARG), (0, A.MD_ERR_WORKSPACE)):
        plist.tiled = tiled
        for call in calls:
            with pytest.raises(A.MdError) as e:
                call()
            assert e.value.code == code, (tiled, e.value)
    # a half list: the force pass takes it, the Hessian and adjoint passes do not
    plist.half = 1
    for k, call in enumerate(calls):
        with pytest.raises(A.MdError) as e:
            call()
        assert e.value.code == (A.MD_ERR_WORKSPACE if k == 0 else A.MD_ERR_ARG), (k, e.value)


def test_workspace_too_small(A):
    p = _params(A)
    cells = A.MdCells()
    fake = 1 << 20  # never dereferenced: validation fails first
    cells.cell_of = cells.cell_xyz = cells.count = cells.start = cells.order = fake
    with pytest.raises(A.MdError) as e:
        A.md_bin_cells(p, fake, cells, fake, 16, None)
    assert e.value.code == A.MD_ERR_WORKSPACE


def test_hbm_probe_rejects_bad_arguments(A):
    # host-side validation: nothing is launched, so fake pointers are never used
    fake = 1 << 20
    for kind, a, b, c, nbytes, reps in ((7, fake, fake, fake, 64, 1), (-1, fake, fake, fake, 64, 1),
                                        (A.MD_PROBE_COPY, fake, None, None, 64, 1),
                                        (A.MD_PROBE_TRIAD, fake, fake, None, 64, 1),
                                        (A.MD_PROBE_READ, fake, fake, None, 65, 1),
                                        (A.MD_PROBE_READ, None, fake, None, 64, 1),
                                        (A.MD_PROBE_READ, fake, fake, None, 64, 0)):
        with pytest.raises(A.MdError) as e:
            A.md_hbm_probe(kind, a, b, c, nbytes, reps, None)
        assert e.value.code == A.MD_ERR_ARG, (kind, nbytes, reps)
