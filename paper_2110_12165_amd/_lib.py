"""ctypes declarations mirroring include/hmat.h."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmat.so")

HMAT_OK = 0
STATUS = {0: "HMAT_OK", -1: "HMAT_EINVAL", -2: "HMAT_ENOMEM", -3: "HMAT_EDEVICE",
          -4: "HMAT_ESTATE", -5: "HMAT_EUNSUPPORTED"}
PREC = {"f64": 0, "f32": 1}
KERNEL = {"plain": 0, "split": 1, "persistent": 2, "auto": 3}
KERNEL_NAME = {v: k for k, v in KERNEL.items()}
MM_MODE = {"x3": 2, "x6": 3}
GF_FS_RECT_COPLANAR = 1
GF_FS_TRIANGLE = 2


class HmatMesh(C.Structure):
    _fields_ = [("n", C.c_int64), ("nvert", C.c_int32), ("verts", C.POINTER(C.c_double)),
                ("slip_dir", C.POINTER(C.c_double))]


class HmatGreen(C.Structure):
    _fields_ = [("kind", C.c_int32), ("component", C.c_int32), ("mu", C.c_double), ("nu", C.c_double)]


class HmatOpts(C.Structure):
    _fields_ = [("aca_eps", C.c_double), ("eta", C.c_double), ("leaf", C.c_int32), ("lattice", C.c_int32),
                ("max_rank", C.c_int32), ("prec", C.c_int32), ("kernel", C.c_int32), ("n_threads", C.c_int32),
                ("wg_waves", C.c_int32), ("unit_kib", C.c_int32), ("wg_waves_p1", C.c_int32),
                ("max_nrhs", C.c_int32), ("transpose", C.c_int32), ("build_device", C.c_int32),
                ("mm_groups", C.c_int32)]


class HmatStats(C.Structure):
    _fields_ = [(name, C.c_int64) for name in (
        "n", "n_dense", "n_lr", "dense_entries", "lr_entries", "max_rank", "sum_rank", "n_leaves",
        "tree_depth", "device_bytes", "factor_bytes", "alg_bytes", "n_units_p1", "n_units_p2")] + [
        ("prec", C.c_int32), ("kernel", C.c_int32), ("wg_waves", C.c_int32), ("lattice", C.c_int32),
        ("wg_waves_p1", C.c_int32), ("mm_groups", C.c_int32)]


class HmatHostBlocks(C.Structure):
    _fields_ = [("n", C.c_int64), ("nblocks", C.c_int64), ("nvalues", C.c_int64),
                ("perm", C.POINTER(C.c_int32)), ("desc", C.POINTER(C.c_int64)),
                ("off", C.POINTER(C.c_int64)), ("values", C.POINTER(C.c_double))]


class HmatProfile(C.Structure):
    _fields_ = [("n_launches", C.c_int32), ("reps", C.c_int32), ("ms", C.c_double * 2), ("ms_product", C.c_double),
                ("alg_bytes", C.c_int64 * 2)]


class RsParams(C.Structure):
    _fields_ = [("n", C.c_int64), ("V0", C.c_double), ("f0", C.c_double), ("eta_rad", C.c_double),
                ("V_pl", C.c_double), ("a", C.c_void_p), ("b", C.c_void_p), ("dc", C.c_void_p)]


class RsRk45State(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("eps_rk", C.c_double), ("last_err", C.c_double),
                ("accepted", C.c_int64), ("rejected", C.c_int64)]


class RsRk45Timing(C.Structure):
    _fields_ = [("product_ms", C.c_double), ("attempt_ms", C.c_double), ("attempts", C.c_int64)]


class RsEnsParams(C.Structure):
    _fields_ = [("n", C.c_int64), ("members", C.c_int32), ("mode", C.c_int32), ("V0", C.c_double),
                ("f0", C.c_double), ("eta_rad", C.c_double), ("V_pl", C.c_double), ("a", C.c_void_p),
                ("b", C.c_void_p), ("dc", C.c_void_p)]


class RsEnsState(C.Structure):
    _fields_ = [("eps_rk", C.c_double), ("t", C.c_double * 64), ("dt", C.c_double * 64),
                ("last_err", C.c_double * 64), ("accepted", C.c_int64 * 64), ("rejected", C.c_int64 * 64)]


# Symbols declared in include/hmat.h, with their ctypes signatures.
SIGNATURES = {
    "hmat_default_opts": (None, [C.POINTER(HmatOpts)]),
    "hmat_build": (C.c_int, [C.POINTER(HmatMesh), C.POINTER(HmatGreen), C.POINTER(HmatOpts), C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    "hmat_build_host": (C.c_int, [C.POINTER(HmatMesh), C.POINTER(HmatGreen), C.POINTER(HmatOpts),
                                  C.POINTER(C.c_void_p)]),
    "hmat_import": (C.c_int, [C.POINTER(HmatHostBlocks), C.POINTER(HmatOpts), C.c_void_p, C.POINTER(C.c_void_p)]),
    "hmat_export": (C.c_int, [C.c_void_p, C.POINTER(HmatHostBlocks)]),
    "hmat_matvec": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_double, C.c_double,
                              C.c_void_p]),
    "hmat_matvec_T": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_double, C.c_double,
                                C.c_void_p]),
    "hmat_matmat": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int64, C.c_double,
                              C.c_double, C.c_int32, C.c_void_p]),
    "hmat_info": (C.c_int, [C.c_void_p, C.POINTER(HmatStats)]),
    "hmat_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "hmat_profile": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(HmatProfile)]),
    "rs_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RsParams), C.c_void_p, C.c_void_p, C.c_void_p,
                         C.c_void_p]),
    "rs_rk45_workspace_bytes": (C.c_int64, [C.c_int64]),
    "rs_rk45_attempt": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RsParams), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(RsRk45State), C.c_int32, C.c_void_p]),
    "rs_rk45_run": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RsParams), C.c_void_p, C.c_void_p, C.c_void_p,
                              C.POINTER(RsRk45State), C.c_int64, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]),
    "rs_rk45_run_timed": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RsParams), C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.POINTER(RsRk45State), C.c_int64, C.c_int64, C.c_void_p, C.c_int32,
                                    C.c_void_p, C.POINTER(RsRk45Timing)]),
    "rs_rk45_replay": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RsParams), C.c_void_p, C.c_void_p,
                                 C.POINTER(C.c_double), C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "rs_rk45_replay_noalloc_max_n": (C.c_int64, []),
    "rs_rk45_replay_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RsParams), C.c_void_p, C.c_void_p,
                                         C.POINTER(C.c_double), C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "hmat_check": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rs_rk45_adjoint_workspace_bytes": (C.c_int64, [C.c_int64, C.c_int64]),
    "rs_rk45_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RsParams), C.c_void_p, C.c_int64,
                                  C.POINTER(C.c_double), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_int64, C.c_void_p]),
    "rs_rk45_step": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RsParams), C.c_void_p, C.c_void_p, C.c_void_p,
                               C.POINTER(RsRk45State), C.c_int32, C.c_void_p]),
    "rs_ens_workspace_bytes": (C.c_int64, [C.c_int64, C.c_int32]),
    "rs_ens_rk45_run": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RsEnsParams), C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.POINTER(RsEnsState), C.c_int64, C.c_int64, C.c_int32, C.c_void_p]),
    "hmat_kernel_entries": (C.c_int, [C.POINTER(HmatMesh), C.POINTER(HmatGreen), C.c_int64,
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "hmat_destroy": (None, [C.c_void_p]),
    "hmat_last_error": (C.c_char_p, []),
}

_lib = None


def load():
    """Load libhmat.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2110_12165_amd.build` "
                          "(or __graft_entry__.build()) first")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class HmatError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def check(status):
    if status != HMAT_OK:
        raise HmatError(status, load().hmat_last_error().decode(errors="replace"))
