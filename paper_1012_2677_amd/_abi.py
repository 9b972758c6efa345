"""ctypes binding of the C ABI declared in include/md.h (argument marshalling only).

Every function here has the name of the C entry point it calls and takes raw
device pointers (ints) plus the ctypes structures below; it raises MdError on a
non-OK status.  Loading fails loudly when the HIP library has not been built:
there is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmd355.so")

MD_OK = 0
MD_ERR_ARG = -1
MD_ERR_BOX = -2
MD_ERR_CAPACITY = -3
MD_ERR_NONFINITE = -4
MD_ERR_HIP = -5
MD_ERR_WORKSPACE = -6

MD_FP64 = 0
MD_MIXED = 1
MD_MAX_N = 1 << 27

MD_LIST_AUTO = 0
MD_LIST_SLOTS = 1
MD_LIST_HALF = 2
MD_REBUILD_HALF_SKIN = 0
MD_REBUILD_DUTC_LDC = 1
MD_STEP_RUN_MAX = 64
MD_BUILD_AUTO, MD_BUILD_CELL_WAVES, MD_BUILD_TILE_WAVES = 0, 1, 2
MD_BUILD_TILE_MIN = 32768

MD_T_FORCE, MD_T_INTEGRATE, MD_T_BIN, MD_T_RESORT, MD_T_BUILD, MD_T_REDUCE, MD_T_CHECK, MD_T_COUNT = range(8)
TIMER_NAMES = ["force", "integrate", "bin", "resort", "build", "reduce", "check"]

EXPORTED = ["md_cell_dims", "md_workspace_bytes", "md_pack_positions", "md_bin_cells", "md_resort", "md_build_pairlist",
            "md_forces", "md_prepare", "md_step", "md_energy", "md_hvp", "md_adjoint_kick", "md_param_grad",
            "md_ldc_check", "md_last_error", "md_hbm_probe", "md_forces_noalloc", "md_step_record"]
MD_NOALLOC_MAX_N = 1 << 20

MD_PROBE_READ, MD_PROBE_COPY, MD_PROBE_TRIAD, MD_PROBE_NT = 0, 1, 2, 4


class MdError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: status {code}: {msg}")
        self.code = code


class MdParams(C.Structure):
    _fields_ = [("n", C.c_int64), ("box", C.c_double * 3), ("eps", C.c_double), ("sigma", C.c_double),
                ("rc", C.c_double), ("rs", C.c_double), ("dt", C.c_double), ("precision", C.c_int32),
                ("resort_every", C.c_int32), ("rebuild_rule", C.c_int32), ("ldc_max", C.c_int32),
                ("list_layout", C.c_int32), ("tile_cells", C.c_int32), ("step_run", C.c_int32),
                ("build_waves", C.c_int32)]


class MdCells(C.Structure):
    _fields_ = [("ncell", C.c_int32 * 3), ("sorted", C.c_int32), ("cell_of", C.c_void_p),
                ("cell_xyz", C.c_void_p), ("count", C.c_void_p), ("start", C.c_void_p),
                ("order", C.c_void_p)]


class MdPairlist(C.Structure):
    _fields_ = [("offsets", C.c_void_p), ("counts", C.c_void_p), ("nbr", C.c_void_p),
                ("cell_stride", C.c_int64), ("capacity", C.c_int64), ("status", C.c_void_p),
                ("tiled", C.c_int32), ("half", C.c_int32)]


class MdTimers(C.Structure):
    _fields_ = [("ms", C.c_double * MD_T_COUNT), ("launches", C.c_int64 * MD_T_COUNT)]


class MdState(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("vel", C.c_void_p), ("force", C.c_void_p), ("pos_ref", C.c_void_p),
                ("pos32", C.c_void_p), ("pos32_alt", C.c_void_p), ("id", C.c_void_p), ("pos_alt", C.c_void_p), ("vel_alt", C.c_void_p),
                ("id_alt", C.c_void_p), ("cells", MdCells), ("list", MdPairlist), ("energy", C.c_void_p),
                ("flags", C.c_void_p), ("host_scratch", C.c_void_p), ("ws", C.c_void_p),
                ("ws_bytes", C.c_size_t), ("timers", C.POINTER(MdTimers)), ("step", C.c_int64),
                ("rebuilds", C.c_int64), ("resorts", C.c_int64), ("phase", C.c_int32),
                ("list_valid", C.c_int32), ("dutc_buffer", C.c_double), ("ldc_checks", C.c_int64),
                ("ldc_kept", C.c_int64), ("list_tiled", C.c_int32), ("tile_stage", C.c_int32),
                ("tile_cells", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def lib():
    """Load libmd355.so (built by paper_1012_2677_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    sig = {
        "md_cell_dims": (C.c_int, [P(MdParams), P(C.c_int32)]),
        "md_workspace_bytes": (C.c_size_t, [P(MdParams)]),
        "md_pack_positions": (C.c_int, [P(MdParams), vp, vp, vp]),
        "md_bin_cells": (C.c_int, [P(MdParams), vp, P(MdCells), vp, C.c_size_t, vp]),
        "md_resort": (C.c_int, [P(MdParams), P(MdState), vp]),
        "md_build_pairlist": (C.c_int, [P(MdParams), vp, P(MdCells), P(MdPairlist), vp, C.c_size_t, vp]),
        "md_forces": (C.c_int, [P(MdParams), vp, P(MdCells), P(MdPairlist), vp, vp, vp, C.c_size_t, vp]),
        "md_prepare": (C.c_int, [P(MdParams), P(MdState), vp]),
        "md_step": (C.c_int, [P(MdParams), P(MdState), C.c_int64, C.c_int64, vp, vp]),
        "md_step_record": (C.c_int, [P(MdParams), P(MdState), C.c_int64, C.c_int64, vp, vp, P(C.c_int32), vp]),
        "md_energy": (C.c_int, [P(MdParams), P(MdState), vp, vp]),
        "md_hvp": (C.c_int, [P(MdParams), vp, P(MdCells), P(MdPairlist), vp, vp, vp, vp, C.c_size_t, vp]),
        "md_adjoint_kick": (C.c_int, [P(MdParams), vp, P(MdCells), P(MdPairlist), vp, vp, vp,
                                      P(C.c_double), vp, vp, C.c_size_t, vp]),
        "md_param_grad": (C.c_int, [P(MdParams), vp, P(MdCells), P(MdPairlist), vp, vp, C.c_size_t, vp]),
        "md_ldc_check": (C.c_int, [P(MdParams), vp, vp, P(C.c_int32), P(C.c_int64), P(C.c_double), vp,
                                   C.c_size_t, vp]),
        "md_last_error": (C.c_char_p, []),
        "md_hbm_probe": (C.c_int, [C.c_int32, vp, vp, vp, C.c_size_t, C.c_int32, P(C.c_float), vp]),
        "md_forces_noalloc": (C.c_int, [P(MdParams), vp, P(MdCells), P(MdPairlist), vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    m = lib().md_last_error()
    return m.decode() if m else ""


def _check(code: int, where: str) -> int:
    if code != MD_OK:
        raise MdError(code, where, last_error())
    return code


# ---- entry points (same names as the C ABI) ---------------------------------

def md_cell_dims(params: MdParams):
    nc = (C.c_int32 * 3)()
    _check(lib().md_cell_dims(C.byref(params), nc), "md_cell_dims")
    return tuple(int(x) for x in nc)


def md_workspace_bytes(params: MdParams) -> int:
    return int(lib().md_workspace_bytes(C.byref(params)))


def md_pack_positions(params, q, pos, stream):
    return _check(lib().md_pack_positions(C.byref(params), q, pos, stream), "md_pack_positions")


def md_bin_cells(params, pos, cells, ws, ws_bytes, stream):
    return _check(lib().md_bin_cells(C.byref(params), pos, C.byref(cells), ws, ws_bytes, stream), "md_bin_cells")


def md_resort(params, state, stream):
    return _check(lib().md_resort(C.byref(params), C.byref(state), stream), "md_resort")


def md_build_pairlist(params, pos, cells, plist, ws, ws_bytes, stream):
    return _check(lib().md_build_pairlist(C.byref(params), pos, C.byref(cells), C.byref(plist), ws, ws_bytes,
                                          stream), "md_build_pairlist")


def md_forces(params, pos, cells, plist, force, pe_w, ws, ws_bytes, stream):
    return _check(lib().md_forces(C.byref(params), pos, C.byref(cells), C.byref(plist), force, pe_w, ws,
                                  ws_bytes, stream), "md_forces")


def md_forces_noalloc(params, pos, cells, plist, force, pe_w, stream):
    return _check(lib().md_forces_noalloc(C.byref(params), pos, C.byref(cells), C.byref(plist), force, pe_w,
                                          stream), "md_forces_noalloc")


def md_prepare(params, state, stream):
    return _check(lib().md_prepare(C.byref(params), C.byref(state), stream), "md_prepare")


def md_step(params, state, nsteps, sample_every, energy_log, stream):
    return _check(lib().md_step(C.byref(params), C.byref(state), nsteps, sample_every, energy_log, stream),
                  "md_step")


def md_step_record(params, state, nsteps, sample_every, energy_log, traj, built, stream):
    """built: a ctypes int32 array of nsteps (host)."""
    return _check(lib().md_step_record(C.byref(params), C.byref(state), nsteps, sample_every, energy_log, traj,
                                       built, stream), "md_step_record")


def md_energy(params, state, out, stream):
    return _check(lib().md_energy(C.byref(params), C.byref(state), out, stream), "md_energy")


def md_hvp(params, pos, cells, plist, u, Hu, dparam, ws, ws_bytes, stream):
    return _check(lib().md_hvp(C.byref(params), pos, C.byref(cells), C.byref(plist), u, Hu, dparam, ws,
                               ws_bytes, stream), "md_hvp")


def md_adjoint_kick(params, pos, cells, plist, u, out, u_out, coef, acc, ws, ws_bytes, stream):
    c5 = (C.c_double * 5)(*[float(x) for x in coef])
    return _check(lib().md_adjoint_kick(C.byref(params), pos, C.byref(cells), C.byref(plist), u, out, u_out, c5,
                                        acc, ws, ws_bytes, stream), "md_adjoint_kick")


def md_param_grad(params, pos, cells, plist, dU, ws, ws_bytes, stream):
    return _check(lib().md_param_grad(C.byref(params), pos, C.byref(cells), C.byref(plist), dU, ws, ws_bytes,
                                      stream), "md_param_grad")


def md_ldc_check(params, pos, pos_ref, ws, ws_bytes, stream):
    """(valid, members, max squared displacement) of the large-displacement check."""
    valid, members, dmax2 = C.c_int32(0), C.c_int64(0), C.c_double(0.0)
    _check(lib().md_ldc_check(C.byref(params), pos, pos_ref, C.byref(valid), C.byref(members), C.byref(dmax2),
                              ws, ws_bytes, stream), "md_ldc_check")
    return bool(valid.value), int(members.value), float(dmax2.value)


def md_hbm_probe(kind, a, b, c, nbytes, reps, stream) -> float:
    """Shortest of reps launches of a streaming probe kernel, in ms (md_probe.h)."""
    ms = C.c_float(0.0)
    _check(lib().md_hbm_probe(int(kind), a, b, c, int(nbytes), int(reps), C.byref(ms), stream), "md_hbm_probe")
    return float(ms.value)
