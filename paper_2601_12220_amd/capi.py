"""ctypes binding of include/bes.h: the same names, argument marshalling only.

Loading fails loudly when libbes.so is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbes.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bes.h")

# status codes
BES_OK = 0
BES_W_NOTFOUND = 1
BES_E_INVALID = -1
BES_E_UNSUPPORTED = -2
BES_E_HIP = -3
BES_E_NOMEM = -4
BES_E_BUFFER = -5
BES_E_STATE = -6

# dtypes (DtypeRank)
BES_INT8, BES_INT32, BES_INT64, BES_FLOAT16 = 1, 2, 3, 4
BES_FLOAT32, BES_FLOAT64, BES_COMPLEX64, BES_COMPLEX128 = 5, 6, 7, 8
DTYPE_CODE = {"int8": 1, "int32": 2, "int64": 3, "float16": 4, "float32": 5,
              "float64": 6, "complex64": 7, "complex128": 8}

# operand kinds and unary ops
BES_ARRAY, BES_VIEW, BES_ELEMENTWISE, BES_TET_JACOBIAN, BES_EXPR = 0, 1, 2, 3, 4
OP_CODE = {"id": 0, "sin": 1, "cos": 2, "square": 3}

# templates
BES_T_AUTO, BES_T_FEM_STREAM, BES_T_GENERIC, BES_T_MFMA = 0, 1, 2, 3
TEMPLATE_NAME = {0: "auto", 1: "fem_stream", 2: "generic", 3: "mfma", 4: "gett"}

BES_MAX_DIM = 8
BES_MAX_SRC = 2


class bes_operand(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("ndim", ctypes.c_int32),
        ("nsrc", ctypes.c_int32),
        ("shape", ctypes.c_int64 * BES_MAX_DIM),
        ("src_offset", ctypes.c_int64 * BES_MAX_SRC),
        ("src_strides", (ctypes.c_int64 * BES_MAX_DIM) * BES_MAX_SRC),
        ("op", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
    ]


class bes_config(ctypes.Structure):
    _fields_ = [("template_id", ctypes.c_int32), ("p", ctypes.c_int32 * 6)]


_lib = None


class BesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bes error {code}: {msg}")
        self.code = code


def load():
    """Load libbes.so (built by paper_2601_12220_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2601_12220_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    PP = ctypes.POINTER(ctypes.c_void_p)
    i32 = ctypes.c_int32
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    sz = ctypes.c_size_t
    szp = ctypes.POINTER(ctypes.c_size_t)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    cp = ctypes.c_char_p
    sig = {
        "bes_ctx_create": ([PP, cp], i32),
        "bes_ctx_destroy": ([P], None),
        "bes_register": ([P, cp, i32, i32, i32, ctypes.POINTER(bes_operand), i32p, PP], i32),
        "bes_plan_destroy": ([P], None),
        "bes_plan_key": ([P, ctypes.c_char_p, sz, szp], i32),
        "bes_plan_canonical": ([P, ctypes.c_char_p, sz, szp], i32),
        "bes_plan_maps": ([P, i32p, i32p, i32p, ctypes.c_char_p, i32p], i32),
        "bes_plan_graph": ([P, i32, i32p, u8p, i32p], i32),
        "bes_check_compliance": ([i32, u8p, i32p], i32),
        "bes_canonical_labeling": ([i32, u8p, i32p, i32p], i32),
        "bes_plan_lookup": ([P, P, cp], i32),
        "bes_plan_get_config": ([P, ctypes.POINTER(bes_config)], i32),
        "bes_plan_set_config": ([P, ctypes.POINTER(bes_config)], i32),
        "bes_db_record": ([P, cp, cp, ctypes.POINTER(bes_config), ctypes.c_double], i32),
        "bes_ctx_stats": ([P, i64p, i64p], i32),
        "bes_launch": ([P, PP, PP, P], i32),
        "bes_plan_set_timing": ([P, P, P], i32),
        "bes_batch_create": ([P, PP, i32, PP], i32),
        "bes_batch_launch": ([P, ctypes.POINTER(PP), ctypes.POINTER(PP), P], i32),
        "bes_batch_destroy": ([P], None),
        "bes_batch_bind": ([P, ctypes.POINTER(PP), ctypes.POINTER(PP), P], i32),
        "bes_batch_replay": ([P, P], i32),
        "bes_adjoint": ([P, P, i32, PP, i32p], i32),
        "bes_plan_set_output": ([P, i32, ctypes.c_int64, i64p, i32], i32),
        "bes_fill_zero": ([P, ctypes.c_int64, i32, P], i32),
        "bes_launch_noalloc": ([P, PP, PP, P], i32),
        "bes_identify": ([P, P, i32p, i32p, i32p, ctypes.c_char_p], i32),
        "bes_register_expr": ([P, cp, i32, i32, i32, ctypes.POINTER(bes_operand), i32p,
                               ctypes.POINTER(ctypes.c_char_p), PP], i32),
        "bes_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def header_symbols():
    """Function names declared in include/bes.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bes_[a-z_]+)\s*\(", text)))


def last_error() -> str:
    return load().bes_last_error().decode()


def check(rc: int, what: str = "") -> int:
    """Raise on a negative status; return warnings (> 0) unchanged."""
    if rc < 0:
        raise BesError(rc, f"{what}: {last_error()}" if what else last_error())
    return rc


# Thin wrappers with the C names ------------------------------------------------

def bes_ctx_create(path: str | None = None):
    h = ctypes.c_void_p()
    check(load().bes_ctx_create(ctypes.byref(h), path.encode() if path else None), "bes_ctx_create")
    return h


def bes_ctx_destroy(h):
    load().bes_ctx_destroy(h)


def bes_register(ctx, notation: str, b: int, n: int, args, table, exprs=None):
    """args: list of bes_operand; table: flat b*n ints; exprs: per argument the
    body of an expression operand or None.  Returns (plan, status)."""
    arr = (bes_operand * len(args))(*args)
    tab = (ctypes.c_int32 * len(table))(*table)
    h = ctypes.c_void_p()
    if exprs is not None and any(x is not None for x in exprs):
        bodies = (ctypes.c_char_p * len(args))(*[x.encode() if x is not None else None
                                                   for x in exprs])
        rc = load().bes_register_expr(ctx, notation.encode(), b, n, len(args), arr, tab,
                                      bodies, ctypes.byref(h))
        check(rc, "bes_register_expr")
    else:
        rc = load().bes_register(ctx, notation.encode(), b, n, len(args), arr, tab,
                                 ctypes.byref(h))
        check(rc, "bes_register")
    return h, rc


def bes_plan_destroy(h):
    load().bes_plan_destroy(h)


def _string(fn, h):
    n = ctypes.c_size_t()
    rc = fn(h, None, 0, ctypes.byref(n))
    if rc not in (BES_OK, BES_E_BUFFER):
        check(rc)
    buf = ctypes.create_string_buffer(n.value + 1)
    check(fn(h, buf, n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


def bes_plan_key(h) -> str:
    return _string(load().bes_plan_key, h)


def bes_plan_canonical(h) -> str:
    return _string(load().bes_plan_canonical, h)


def bes_plan_maps(h, b: int, n: int, n_args: int):
    mm = (ctypes.c_int32 * b)()
    pm = (ctypes.c_int32 * n)()
    am = (ctypes.c_int32 * n_args)()
    im = ctypes.create_string_buffer(27)
    ni = ctypes.c_int32()
    check(load().bes_plan_maps(h, mm, pm, am, im, ctypes.byref(ni)), "bes_plan_maps")
    return list(mm), list(pm), list(am), im.raw[:ni.value].decode()


def bes_plan_graph(h, which: int = 0):
    import numpy as np
    n = ctypes.c_int32()
    check(load().bes_plan_graph(h, which, ctypes.byref(n), None, None))
    adj = np.zeros((n.value, n.value), dtype=np.uint8)
    col = np.zeros(n.value, dtype=np.int32)
    check(load().bes_plan_graph(h, which, ctypes.byref(n),
                                adj.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return adj, col


def bes_check_compliance(adj, colors) -> int:
    import numpy as np
    adj = np.ascontiguousarray(adj, dtype=np.uint8)
    col = np.ascontiguousarray(colors, dtype=np.int32)
    return load().bes_check_compliance(len(col), adj.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                       col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))


def bes_canonical_labeling(adj, colors):
    import numpy as np
    adj = np.ascontiguousarray(adj, dtype=np.uint8)
    col = np.ascontiguousarray(colors, dtype=np.int32)
    lab = np.zeros(len(col), dtype=np.int32)
    check(load().bes_canonical_labeling(len(col), adj.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                        col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return lab


def bes_plan_lookup(ctx, h, arch: str = "gfx950") -> int:
    return check(load().bes_plan_lookup(ctx, h, arch.encode()), "bes_plan_lookup")


def bes_plan_get_config(h) -> bes_config:
    c = bes_config()
    check(load().bes_plan_get_config(h, ctypes.byref(c)))
    return c


def bes_plan_set_config(h, cfg: bes_config) -> None:
    check(load().bes_plan_set_config(h, ctypes.byref(cfg)), "bes_plan_set_config")


def bes_db_record(ctx, key: str, arch: str, cfg: bes_config, seconds: float) -> None:
    check(load().bes_db_record(ctx, key.encode(), arch.encode(), ctypes.byref(cfg), seconds),
          "bes_db_record")


def bes_ctx_stats(ctx):
    h, m = ctypes.c_int64(), ctypes.c_int64()
    check(load().bes_ctx_stats(ctx, ctypes.byref(h), ctypes.byref(m)))
    return h.value, m.value


def _ptrs(ptrs):
    return (ctypes.c_void_p * max(1, len(ptrs)))(*[int(p) for p in ptrs])


def bes_plan_set_timing(h, start_event: int, stop_event: int) -> None:
    check(load().bes_plan_set_timing(h, ctypes.c_void_p(start_event or None),
                                     ctypes.c_void_p(stop_event or None)), "bes_plan_set_timing")


def bes_launch(h, src_ptrs, out_ptrs, stream: int = 0) -> None:
    check(load().bes_launch(h, _ptrs(src_ptrs), _ptrs(out_ptrs), ctypes.c_void_p(stream)),
          "bes_launch")


def bes_launch_noalloc(h, src_ptrs, out_ptrs, stream: int = 0) -> None:
    check(load().bes_launch_noalloc(h, _ptrs(src_ptrs), _ptrs(out_ptrs), ctypes.c_void_p(stream)),
          "bes_launch_noalloc")


def bes_batch_create(ctx, plans):
    arr = (ctypes.c_void_p * len(plans))(*[p.value for p in plans])
    h = ctypes.c_void_p()
    check(load().bes_batch_create(ctx, arr, len(plans), ctypes.byref(h)), "bes_batch_create")
    return h


def _flat_lists(lists):
    """One uint64 buffer holding every list back to back, and an array of
    the lists' start addresses (the void *const *const * the C side reads).
    Returns (array of starts as POINTER(POINTER(c_void_p)), keep-alive)."""
    sizes = [max(1, len(l)) for l in lists]
    buf = (ctypes.c_uint64 * max(1, sum(sizes)))()
    base = ctypes.addressof(buf)
    starts = []
    off = 0
    for l, n in zip(lists, sizes):
        starts.append(base + 8 * off)
        if l:
            buf[off:off + len(l)] = [int(p) for p in l]
        off += n
    arr = (ctypes.c_uint64 * max(1, len(starts)))(*starts)
    PP = ctypes.POINTER(ctypes.c_void_p)
    return ctypes.cast(arr, ctypes.POINTER(PP)), (buf, arr)


def _ptr_lists(src_lists, out_lists):
    sarr, ks = _flat_lists(src_lists)
    oarr, ko = _flat_lists(out_lists)
    return sarr, oarr, (ks, ko)


def bes_batch_launch(h, src_lists, out_lists, stream: int = 0, _keep=None) -> None:
    sarr, oarr, _ = _ptr_lists(src_lists, out_lists)
    check(load().bes_batch_launch(h, sarr, oarr, ctypes.c_void_p(stream)), "bes_batch_launch")


def bes_batch_bind(h, src_lists, out_lists, stream: int = 0) -> None:
    sarr, oarr, _ = _ptr_lists(src_lists, out_lists)
    check(load().bes_batch_bind(h, sarr, oarr, ctypes.c_void_p(stream)), "bes_batch_bind")


def bes_batch_replay(h, stream: int = 0) -> None:
    check(load().bes_batch_replay(h, ctypes.c_void_p(stream)), "bes_batch_replay")


def bes_batch_destroy(h) -> None:
    load().bes_batch_destroy(h)


def bes_adjoint(ctx, fwd, pos: int):
    h = ctypes.c_void_p()
    n = ctypes.c_int32()
    rc = load().bes_adjoint(ctx, fwd, pos, ctypes.byref(h), ctypes.byref(n))
    check(rc, "bes_adjoint")
    return h, n.value, rc


def bes_plan_set_output(h, slot: int, offset: int = 0, strides=None, accumulate: bool = False):
    st = None
    if strides is not None:
        st = (ctypes.c_int64 * max(1, len(strides)))(*[int(v) for v in strides])
    check(load().bes_plan_set_output(h, slot, int(offset), st, 1 if accumulate else 0),
          "bes_plan_set_output")


def bes_fill_zero(ptr: int, n: int, dtype: int, stream: int = 0) -> None:
    check(load().bes_fill_zero(ctypes.c_void_p(ptr), int(n), dtype, ctypes.c_void_p(stream)),
          "bes_fill_zero")


def bes_identify(ref, raised, b: int, n: int, n_args: int):
    """(member_map, pos_map, arg_map, index_map) from the reference plan's names
    to the raised plan's (index_map: dict reference letter -> raised letter)."""
    mm = (ctypes.c_int32 * max(1, b))()
    pm = (ctypes.c_int32 * max(1, n))()
    am = (ctypes.c_int32 * max(1, n_args))()
    im = ctypes.create_string_buffer(b"\0" * 27, 27)
    check(load().bes_identify(ref, raised, mm, pm, am, im), "bes_identify")
    raw = im.raw[:26]
    imap = {chr(ord("a") + x): chr(raw[x]) for x in range(26) if raw[x] != 0}
    return list(mm)[:b], list(pm)[:n], list(am)[:n_args], imap
