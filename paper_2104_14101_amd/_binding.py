"""ctypes binding of libaes.so (include/aes.h).  Argument marshalling only.

Loading fails loudly (ImportError) when the library has not been built: there is no CPU
fallback.
"""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_uint64, c_void_p

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libaes.so")

AES_OK, AES_ERR_INVALID_ARG, AES_ERR_NOT_SPD, AES_ERR_NONFINITE, AES_ERR_MAX_ITER, AES_ERR_HIP, AES_ERR_OOM, \
    AES_ERR_NOT_IMPLEMENTED = range(8)
STATUS_NAMES = {0: "ok", 1: "invalid_arg", 2: "not_spd", 3: "nonfinite", 4: "max_iter", 5: "hip_error", 6: "oom",
                7: "not_implemented"}
METHODS = {"pcg": 0, "ihs": 1, "cg": 2, "polyak": 3}
SKETCHES = {"srht": 0, "gauss": 1, "sjlt": 2, "srht_reuse": 3, "srht_nested": 4}
PRECISIONS = {"fp64": 0, "mixed": 1, "mixed_fp32": 2}
STOPS = {"xrel": 0, "dtilde_rel": 1, "fixed": 2, "remark": 3}


class TraceEntry(ctypes.Structure):
    _fields_ = [("t", c_int64), ("m", c_int64), ("k", c_int64), ("log_ratio", c_double), ("threshold", c_double),
                ("accept", c_int32), ("pad_", c_int32), ("dtilde", c_double), ("time_ms", c_double)]


class Options(ctypes.Structure):
    _fields_ = [("method", c_int32), ("sketch", c_int32), ("precision", c_int32), ("stop", c_int32),
                ("rho", c_double), ("m_init", c_int64), ("m_max", c_int64), ("max_iter", c_int64),
                ("seed", c_uint64), ("problem", c_int32), ("adaptive", c_int32), ("force_reject_at", c_int64),
                ("inner_tol", c_double), ("max_refine", c_int32), ("trace_cap", c_int32),
                ("trace", POINTER(TraceEntry)), ("x0", c_void_p), ("profile", c_int32), ("keep_fp32_copy", c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", c_int64), ("attempts", c_int64), ("final_m", c_int64), ("resketches", c_int64),
                ("a_passes", c_int64), ("refine_sweeps", c_int64), ("trace_len", c_int64),
                ("dtilde_final", c_double), ("time_sketch_ms", c_double), ("time_total_ms", c_double),
                ("m_cap_reached", c_int32), ("status", c_int32), ("time_hv_ms", c_double), ("hv_launches", c_int64)]

    def as_dict(self):
        out = {f[0]: getattr(self, f[0]) for f in self._fields_}
        out["status"] = STATUS_NAMES.get(self.status, str(self.status))
        return out


class Problem(ctypes.Structure):
    _fields_ = [("n", c_int64), ("d", c_int64), ("c", c_int64), ("A", c_void_p), ("lda", c_int64), ("b", c_void_p),
                ("ldb", c_int64), ("nu", c_double), ("lam", c_void_p), ("x", c_void_p), ("ldx", c_int64)]


_PROTOS = {
    "aes_create": (c_int, [POINTER(c_void_p), c_int]),
    "aes_destroy": (c_int, [c_void_p]),
    "aes_last_error": (c_char_p, [c_void_p]),
    "aes_default_options": (None, [POINTER(Options)]),
    "aes_solve": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_double,
                          c_void_p, c_double, POINTER(Options), c_void_p, c_int64, POINTER(Info)]),
    "aes_solve_dual": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                               c_double, c_void_p, c_double, POINTER(Options), c_void_p, c_int64, POINTER(Info)]),
    "aes_solve_direct": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                                 c_double, c_void_p, c_void_p, c_int64]),
    "aes_solve_batched": (c_int, [c_void_p, c_void_p, c_int64, POINTER(Problem), c_double, POINTER(Options),
                                  POINTER(Info)]),
    "aes_solve_keep": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                               c_double, c_void_p, c_double, POINTER(Options), c_void_p, c_int64, POINTER(Info),
                               POINTER(c_void_p)]),
    "aes_adjoint_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_void_p, POINTER(Info)]),
    "aes_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double)]),
    "aes_ctx_free": (None, [c_void_p]),
    "aes_hv": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_int64, c_double, c_void_p, c_void_p, c_void_p,
                       c_void_p]),
    "aes_hv_noalloc": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_int64, c_double, c_void_p, c_void_p,
                               c_void_p, c_void_p]),
    "aes_residual": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                             c_double, c_void_p, c_void_p, c_int64, c_void_p, c_int64]),
    "aes_tune_hp": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int64, c_int, c_int, c_int64,
                            c_int, POINTER(c_double)]),
    "aes_hv_multi": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int64, c_double, c_void_p,
                             c_void_p, c_void_p, c_int]),
    "aes_sketch": (c_int, [c_void_p, c_void_p, c_int, c_int64, c_int64, c_void_p, c_int64, c_int64, c_uint64, c_int32,
                           c_int64, c_void_p]),
    "aes_factor": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
    "aes_precond_apply": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_double, c_void_p,
                                  c_void_p, c_void_p]),
}

_lib = None


def load():
    """Load libaes.so and set the prototypes (raises ImportError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2104_14101_amd.build` "
                          "(the library has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_functions():
    """Names of the functions declared in include/aes.h."""
    import re

    hdr = os.path.join(os.path.dirname(_HERE), "include", "aes.h")
    text = open(hdr).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aes_[a-z_]+)\s*\(", text)))


class AesError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
