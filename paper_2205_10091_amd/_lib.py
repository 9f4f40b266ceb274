"""ctypes declarations of the C ABI in include/tcx.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtcx.so")


class TcxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


STATUS = {0: "TC_OK", 1: "TC_ERR_INVALID_ARG", 2: "TC_ERR_UNSUPPORTED",
          3: "TC_ERR_OUT_OF_MEMORY", 4: "TC_ERR_TOO_LARGE", 5: "TC_ERR_DEVICE",
          6: "TC_ERR_BUSY", 7: "TC_ERR_STATE"}
TC_OK, TC_ERR_INVALID_ARG, TC_ERR_UNSUPPORTED, TC_ERR_OUT_OF_MEMORY, \
    TC_ERR_TOO_LARGE, TC_ERR_DEVICE, TC_ERR_BUSY, TC_ERR_STATE = range(8)

GATE_KIND = {"h": 0, "x": 1, "y": 2, "z": 3, "s": 4, "sqrt_x": 5, "sqrt_y": 6,
             "sqrt_w": 7, "rx": 8, "ry": 9, "rz": 10, "u1": 11, "cnot": 12,
             "cz": 13, "rzz": 14, "rxx": 15, "ryy": 16, "fsim": 17, "u2": 18,
             "depol": 19, "rswitch": 20}


class Gate(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q", C.c_int32 * 2),
                ("param", C.c_int32 * 2), ("fixed", C.c_double * 2),
                ("matrix", C.POINTER(C.c_double))]


class Circuit(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_params", C.c_int32),
                ("n_gates", C.c_int32), ("gates", C.POINTER(Gate))]


class Observable(C.Structure):
    _fields_ = [("kind", C.c_int32), ("bits", C.POINTER(C.c_uint8)),
                ("n_terms", C.c_int32), ("structures", C.POINTER(C.c_uint8)),
                ("weights", C.POINTER(C.c_double)), ("mpo_bonds", C.POINTER(C.c_int32)),
                ("mpo", C.POINTER(C.c_double))]


class BuildOpts(C.Structure):
    _fields_ = [("split_2q", C.c_int32), ("lightcone", C.c_int32),
                ("absorb_1q", C.c_int32)]


class NetworkInfo(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_params", C.c_int32),
                ("n_terms", C.c_int32), ("max_leaves", C.c_int32),
                ("total_leaves", C.c_int64)]


class PathOpts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_trials", C.c_int32),
                ("score", C.c_int32), ("temperature", C.c_double),
                ("reconf_k", C.c_int32), ("max_depth", C.c_int32)]


class PathStats(C.Structure):
    _fields_ = [("log10_flops", C.c_double), ("log2_write", C.c_double),
                ("log2_size", C.c_double), ("flops", C.c_double),
                ("write", C.c_double), ("size", C.c_double),
                ("n_steps", C.c_int32), ("max_depth", C.c_int32)]


class PlanOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("batch", C.c_int32),
                ("want_grad", C.c_int32), ("device", C.c_int32),
                ("mem_budget_bytes", C.c_uint64), ("stream", C.c_void_p),
                ("gemm_min_k", C.c_int32), ("checkpoint_every", C.c_int32),
                ("gemm_min_macs", C.c_uint64), ("exec_mode", C.c_int32),
                ("tile_mode", C.c_int32), ("qgt", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("flops", C.c_double), ("alg_bytes", C.c_double),
                ("grad_flops", C.c_double), ("grad_alg_bytes", C.c_double),
                ("workspace_bytes", C.c_uint64),
                ("peak_tensor_bytes", C.c_uint64),
                ("n_nodes", C.c_int32), ("n_levels", C.c_int32),
                ("n_gemm_nodes", C.c_int32), ("n_launches", C.c_int32),
                ("n_grad_launches", C.c_int32), ("batch", C.c_int32),
                ("n_params", C.c_int32), ("n_terms", C.c_int32),
                ("checkpoint_every", C.c_int32), ("exec_mode", C.c_int32),
                ("n_split_nodes", C.c_int32), ("n_split_sums", C.c_int32),
                ("n_wide_nodes", C.c_int32), ("n_term_groups", C.c_int32),
                ("n_qgt_rows", C.c_int32)]


class ServeOpts(C.Structure):
    _fields_ = [("device", C.c_int32), ("pool_bytes", C.c_uint64),
                ("max_request_bytes", C.c_uint64), ("max_active", C.c_int32),
                ("path_trials", C.c_int32), ("stream", C.c_void_p),
                ("max_request_flops", C.c_double)]


class ServeResult(C.Structure):
    _fields_ = [("id", C.c_int64), ("value", C.c_double),
                ("value_im", C.c_double), ("submit_to_done_s", C.c_double),
                ("want_grad", C.c_int32), ("status", C.c_int32),
                ("plan_s", C.c_double), ("admit_to_done_s", C.c_double)]


VP = C.c_void_p
PVP = C.POINTER(C.c_void_p)
I32P = C.POINTER(C.c_int32)
I64P = C.POINTER(C.c_int64)
F32P = C.POINTER(C.c_float)
F64P = C.POINTER(C.c_double)

# (name, restype, argtypes): every symbol the header declares
SIGNATURES = [
    ("tc_status_string", C.c_char_p, [C.c_int]),
    ("tc_last_error", C.c_char_p, []),
    ("tc_version", C.c_int32, []),
    ("tc_build_network", C.c_int, [C.POINTER(Circuit), C.POINTER(Observable),
                                   C.POINTER(BuildOpts), PVP]),
    ("tc_network_free", None, [VP]),
    ("tc_network_info_get", C.c_int, [VP, C.POINTER(NetworkInfo)]),
    ("tc_network_term_leaves", C.c_int, [VP, C.c_int32, I32P, I32P, I32P,
                                         I32P, I32P, I32P, I32P]),
    ("tc_greedy_path", C.c_int, [VP, C.POINTER(PathOpts), PVP]),
    ("tc_path_replace_term", C.c_int, [VP, C.c_int32, I32P, C.c_int32]),
    ("tc_path_free", None, [VP]),
    ("tc_slice", C.c_int, [VP, VP, C.c_int32, C.c_int32, PVP, PVP, I32P]),
    ("tc_path_stats_get", C.c_int, [VP, C.c_int32, C.POINTER(PathStats)]),
    ("tc_path_term_pairs", C.c_int, [VP, C.c_int32, I32P, I32P]),
    ("tc_plan_create", C.c_int, [VP, VP, C.POINTER(PlanOpts), PVP]),
    ("tc_plan_free", None, [VP]),
    ("tc_plan_info_get", C.c_int, [VP, C.POINTER(PlanInfo)]),
    ("tc_plan_bind", C.c_int, [VP, VP, C.c_uint64]),
    ("tc_contract", C.c_int, [VP, VP, F64P]),
    ("tc_contract_grad", C.c_int, [VP, VP, F64P, F64P]),
    ("tc_contract_device", C.c_int, [VP, VP, VP]),
    ("tc_contract_grad_device", C.c_int, [VP, VP, VP, VP]),
    ("tc_contract_grad_device_noalloc", C.c_int, [VP, VP, VP, VP]),
    ("tc_contract_qgt", C.c_int, [VP, VP, F64P]),
    ("tc_plan_profile", C.c_int, [VP, VP, C.c_int32, C.c_int32, C.c_int32, I32P,
                                  I32P, F64P, F64P, F64P]),
    ("tc_serve_create", C.c_int, [C.POINTER(ServeOpts), PVP]),
    ("tc_serve_submit", C.c_int, [VP, C.POINTER(Circuit), C.POINTER(Observable),
                                  F32P, C.c_int32, I64P]),
    ("tc_serve_step", C.c_int, [VP, I32P]),
    ("tc_serve_result_get", C.c_int, [VP, C.c_int64, C.POINTER(ServeResult),
                                      F64P]),
    ("tc_serve_free", None, [VP]),
]

_lib = None


def load(path: str = LIB_PATH, strict: bool = True):
    """Load the shared library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    # One HIP runtime per process: torch's bundled libamdhip64 carries the
    # same SONAME as the system one, so loading torch first makes this
    # library bind to it instead of starting a second runtime (which would
    # find no device) and lets torch tensors and this library share memory
    # and streams.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name, None)
        if fn is None:
            if strict:
                raise ImportError(f"{path} does not export {name}")
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != TC_OK:
        msg = _lib.tc_last_error().decode() if _lib is not None else ""
        raise TcxError(status, msg)
