"""Oracle for batched einsums: plain, slow, obviously correct CPU code.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  It
shares no code with the HIP library (``paper_2601_12220_amd``) and imports
nothing from it; the two meet only through seeded inputs and through results
that the tests compare.

Contents
--------
* :func:`einsum` / :func:`batched_einsum` -- FP64 loop nest of Eq. (1)
  (Section "Einstein Notation"), applied per member of a batched einsum
  (Definition "Batched Einstein Summation").  Implemented in ``einsum_ref.c``.
* :func:`einsum_at` -- selected output elements, for outputs too large to
  evaluate whole.
* :func:`einsum_grad` -- gradient of <G, R> w.r.t. one operand, written as the
  derivative of a multilinear form (a plain loop over every index assignment).
* :mod:`oracle.functional` -- FP64 materialization of functional operands
  (Definition "Functional Batched Einstein Summation").
* :mod:`oracle.brute` -- brute-force isomorphism test and normal form
  (Definitions "Einsum Isomorphism", "Batched einsum Isomorphism" and
  "Canonicalization of a batched einsum").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "einsum_ref.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the C loop nest with gcc (OpenMP over output elements)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99",
           "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int)
    i64p = ctypes.POINTER(ctypes.c_longlong)
    dpp = ctypes.POINTER(ctypes.c_void_p)
    dp = ctypes.c_void_p
    lib.oracle_einsum.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int, i32p,
                                  i64p, dpp, dp]
    lib.oracle_einsum_at.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int,
                                     i32p, i64p, dpp, ctypes.c_longlong, i64p, dp]
    lib.oracle_einsum_grad.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int,
                                       i32p, i64p, dpp, dp, ctypes.c_int, dp]
    lib.oracle_einsum_grad_at.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int,
                                          i32p, i64p, dpp, dp, ctypes.c_int,
                                          ctypes.c_longlong, i64p, dp]
    for f in (lib.oracle_einsum, lib.oracle_einsum_at, lib.oracle_einsum_grad,
              lib.oracle_einsum_grad_at):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# Notation (grammar of Listings "Grammar for an index" / "index list")
# ---------------------------------------------------------------------------

def parse(notation: str):
    """'ij,ej->ei' -> ([[8, 9], [4, 9]], [4, 8]).  Letters a..z only."""
    if "->" not in notation:
        raise ValueError("notation needs '->'")
    lhs, rhs = notation.split("->")
    ins = lhs.split(",")
    for s in ins + [rhs]:
        for ch in s:
            if not ("a" <= ch <= "z"):
                raise ValueError(f"bad index {ch!r}")
    return [[ord(c) - 97 for c in s] for s in ins], [ord(c) - 97 for c in rhs]


def _extents(ins, arrays):
    ext = [0] * 26
    seen = [False] * 26
    for labels, arr in zip(ins, arrays):
        if arr.ndim != len(labels):
            raise ValueError("operand rank does not match its index list")
        for L, s in zip(labels, arr.shape):
            if seen[L] and ext[L] != s:
                raise ValueError("inconsistent extent for an index")
            ext[L] = s
            seen[L] = True
    return ext


def _marshal(notation, arrays):
    ins, out = parse(notation)
    if len(ins) != len(arrays):
        raise ValueError("operand count does not match notation")
    arrs = [np.array(a, dtype=np.float64, order="C") for a in arrays]
    ext = _extents(ins, arrs)
    ndim = (ctypes.c_int * len(ins))(*[len(x) for x in ins])
    flat = [L for x in ins for L in x]
    labels = (ctypes.c_int * max(1, len(flat)))(*flat)
    outl = (ctypes.c_int * max(1, len(out)))(*out)
    extc = (ctypes.c_longlong * 26)(*ext)
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    shape = tuple(ext[L] for L in out)
    return ins, out, arrs, ndim, labels, outl, extc, ptrs, shape


def einsum(notation: str, *arrays) -> np.ndarray:
    """FP64 evaluation of one einsum by the plain loop nest of Eq. (1)."""
    lib = _load()
    ins, out, arrs, ndim, labels, outl, extc, ptrs, shape = _marshal(notation, arrays)
    res = np.empty(shape, dtype=np.float64)
    rc = lib.oracle_einsum(len(ins), ndim, labels, len(out), outl, extc, ptrs,
                           res.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected notation {notation!r}")
    return res


def einsum_at(notation: str, arrays, flat_positions) -> np.ndarray:
    """Output elements at the given flat row-major positions only."""
    lib = _load()
    ins, out, arrs, ndim, labels, outl, extc, ptrs, shape = _marshal(notation, arrays)
    where = np.ascontiguousarray(flat_positions, dtype=np.int64)
    vals = np.empty(where.shape, dtype=np.float64)
    rc = lib.oracle_einsum_at(len(ins), ndim, labels, len(out), outl, extc, ptrs,
                              where.size,
                              where.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                              vals.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected notation {notation!r}")
    return vals


def einsum_grad(notation: str, arrays, G, wrt: int) -> np.ndarray:
    """d<G, R>/d arrays[wrt] for R = einsum(notation, *arrays)."""
    lib = _load()
    ins, out, arrs, ndim, labels, outl, extc, ptrs, shape = _marshal(notation, arrays)
    g = np.array(G, dtype=np.float64, order="C")
    if g.shape != shape:
        raise ValueError("G must have the output's shape")
    dA = np.empty(arrs[wrt].shape, dtype=np.float64)
    rc = lib.oracle_einsum_grad(len(ins), ndim, labels, len(out), outl, extc,
                                ptrs, g.ctypes.data, wrt, dA.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected notation {notation!r}")
    return dA


def einsum_grad_at(notation: str, arrays, G, wrt: int, flat_positions) -> np.ndarray:
    """Entries of d<G, R>/d arrays[wrt] at flat row-major positions of that
    operand (its index letters must be distinct)."""
    lib = _load()
    ins, out, arrs, ndim, labels, outl, extc, ptrs, shape = _marshal(notation, arrays)
    g = np.array(G, dtype=np.float64, order="C")
    if g.shape != shape:
        raise ValueError("G must have the output's shape")
    where = np.ascontiguousarray(flat_positions, dtype=np.int64)
    vals = np.empty(where.shape, dtype=np.float64)
    rc = lib.oracle_einsum_grad_at(len(ins), ndim, labels, len(out), outl, extc, ptrs,
                                   g.ctypes.data, wrt, where.size,
                                   where.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                                   vals.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected notation {notation!r} for wrt={wrt}")
    return vals


def batched_einsum(notation: str, table, arrays: dict):
    """Batched einsum: member i evaluates the notation on the arguments named
    in row i of ``table`` (a b x n list of names keyed into ``arrays``)."""
    return [einsum(notation, *[arrays[name] for name in row]) for row in table]


def threads_used() -> int:
    """OpenMP threads the C loop nest runs with (OMP_NUM_THREADS or cores)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


__all__ = ["build", "parse", "einsum", "einsum_at", "einsum_grad",
           "batched_einsum", "threads_used"]

if __name__ == "__main__":  # pragma: no cover
    print(build(), file=sys.stderr)
