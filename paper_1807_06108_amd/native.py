"""ctypes binding of libmppi_jump.so (the C ABI of include/mppi_jump.h).

Argument marshalling only: every step of an iteration runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmppi_jump.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mppi_jump.h")


def _int_literal(text):
    """Value of an integer macro body: a literal or "(a << b)"."""
    t = text.strip().strip("()").strip()
    if "<<" in t:
        a, b = t.split("<<")
        return int(a.strip(), 0) << int(b.strip(), 0)
    return int(t, 0)


def _header_constants():
    consts = {}
    for name, val in re.findall(r"^#define\s+(MPPI_\w+)\s+([^/\n]+)", open(HEADER).read(), re.M):
        try:
            consts[name] = _int_literal(val)
        except ValueError:
            pass
    return consts


C = _header_constants()

MPPI_OK = C["MPPI_OK"]
ITEM = {k[len("MPPI_ITEM_"):]: v for k, v in C.items() if k.startswith("MPPI_ITEM_")}
MAX_LEVELS = C["MPPI_JUMP_MAX_LEVELS"]


class Config(ctypes.Structure):
    """Mirror of mppi_jump_config."""
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("dynamics", ctypes.c_int32),
        ("K", ctypes.c_int32), ("T", ctypes.c_int32),
        ("dt", ctypes.c_float), ("lambda_", ctypes.c_float),
        ("alpha", ctypes.c_float), ("c", ctypes.c_float), ("nu", ctypes.c_float),
        ("count_law", ctypes.c_int32), ("cost_form", ctypes.c_int32),
        ("debug_dump", ctypes.c_int32),
        ("sigma", ctypes.c_float * 4), ("sigma_J", ctypes.c_float * 4),
        ("u_init", ctypes.c_float * 4), ("R", ctypes.c_float * 4),
        ("Q", ctypes.c_float * 12), ("Qf", ctypes.c_float * 12),
        ("x_goal", ctypes.c_float * 12), ("params", ctypes.c_float * 12),
        ("crash_penalty", ctypes.c_float), ("schedule", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("controller_id", ctypes.c_uint64),
        ("start_iteration", ctypes.c_uint64),
        ("full_sigma", ctypes.c_int32), ("sigma_L", ctypes.c_float * 16),
        ("sample_offset", ctypes.c_int32), ("mark_law", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    """Mirror of mppi_jump_stats."""
    _fields_ = [("rho", ctypes.c_double), ("eta", ctypes.c_double),
                ("status", ctypes.c_int32), ("n_finite", ctypes.c_int32),
                ("iteration", ctypes.c_uint64)]


def make_config(cfg):
    """Config structure from a configuration dict (keys as in the C struct)."""
    c = Config()
    c.abi_version = C["MPPI_JUMP_ABI_VERSION"]
    for name, ctype in Config._fields_:
        key = "lambda" if name == "lambda_" else name
        if name == "abi_version" or key not in cfg:
            continue
        v = cfg[key]
        if hasattr(ctype, "_length_"):
            arr = getattr(c, name)
            vals = list(v)
            if len(vals) > ctype._length_:
                raise ValueError("%s has more than %d entries" % (key, ctype._length_))
            for i, x in enumerate(vals):
                arr[i] = x
        else:
            setattr(c, name, v)
    return c


class MppiError(RuntimeError):
    def __init__(self, code, detail):
        super().__init__("mppi_jump error %d (%s): %s" % (code, strerror(code), detail))
        self.code = code


_lib = None

_PROTOS = {
    "mppi_jump_abi_version": (ctypes.c_int, []),
    "mppi_jump_dims": (ctypes.c_int, [ctypes.c_int32] + [ctypes.POINTER(ctypes.c_int32)] * 3),
    "mppi_jump_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)]),
    "mppi_jump_count_thresholds": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_uint64)]),
    "mppi_jump_init": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "mppi_jump_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "mppi_jump_control_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                              ctypes.c_void_p, ctypes.c_void_p]),
    "mppi_jump_control_step_static": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.c_void_p,
                                                     ctypes.c_void_p, ctypes.c_int32,
                                                     ctypes.c_void_p, ctypes.c_void_p]),
    "mppi_jump_rollout": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mppi_jump_update": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mppi_jump_shift": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mppi_jump_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.c_void_p]),
    "mppi_jump_set": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.c_void_p]),
    "mppi_jump_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "mppi_jump_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "mppi_jump_last_error": (ctypes.c_char_p, []),
    "mppi_jump_plant_step": (ctypes.c_int, [ctypes.c_void_p] * 5),
    "mppi_jump_plant_step_force": (ctypes.c_int, [ctypes.c_void_p] * 6),
    "mppi_jump_batch_scratch_bytes": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                                     ctypes.POINTER(ctypes.c_size_t)]),
    "mppi_jump_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p),
                                              ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                              ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                              ctypes.POINTER(ctypes.c_void_p)]),
    "mppi_jump_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_void_p]),
    "mppi_jump_batch_set_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "mppi_jump_batch_u0": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "mppi_jump_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "mppi_jump_pool_bytes": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "mppi_jump_pool_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p,
                                             ctypes.POINTER(ctypes.c_void_p)]),
    "mppi_jump_pool_tick": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_void_p]),
    "mppi_jump_pool_replace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "mppi_jump_pool_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "mppi_jump_pool_results": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.POINTER(ctypes.c_int32)]),
    "mppi_jump_pool_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "mppi_jump_philox": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "mppi_jump_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "mppi_jump_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_int64)]),
}


def use_library(path):
    """Load the library from `path` instead (the phase-profiling build);
    only before the first load."""
    global LIB_PATH
    if _lib is not None and path != LIB_PATH:
        raise RuntimeError("the library is already loaded from %s" % LIB_PATH)
    LIB_PATH = path


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built; run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(code):
    return lib().mppi_jump_strerror(code).decode()


def check(rc):
    if rc != MPPI_OK:
        raise MppiError(rc, lib().mppi_jump_last_error().decode())
    return rc


def dims(dynamics):
    n, m, q = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().mppi_jump_dims(dynamics, ctypes.byref(n), ctypes.byref(m), ctypes.byref(q)))
    return n.value, m.value, q.value


def workspace_bytes(cfg):
    c = make_config(cfg)
    b = ctypes.c_size_t()
    check(lib().mppi_jump_workspace_bytes(ctypes.byref(c), ctypes.byref(b)))
    return b.value


def count_thresholds(cfg):
    c = make_config(cfg)
    out = (ctypes.c_uint64 * MAX_LEVELS)()
    check(lib().mppi_jump_count_thresholds(ctypes.byref(c), out))
    return list(out)
