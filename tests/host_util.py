"""Helpers shared by the host-logic tests (CPU) and the GPU tests.

Registration goes through the library's C ABI; expected values come from the
oracle only.
"""
from __future__ import annotations

import numpy as np

from paper_2601_12220_amd import Context, make_operand

SHORT = {"f64": "float64", "f32": "float32", "i8": "int8", "i32": "int32", "i64": "int64",
         "f16": "float16", "c64": "complex64", "c128": "complex128"}


def register_structure(ctx: Context, notation, table, shapes, dtypes="float64"):
    """Register a batched einsum given by structure only (dense arrays)."""
    names = sorted({a for row in table for a in row})
    if isinstance(dtypes, str):
        dtypes = {a: dtypes for a in names}
    ops = {a: (make_operand(shapes[a], dtypes[a]), [a]) for a in names}
    return ctx.register(notation, table, ops, arg_order=names)


def parse_key(key: str):
    """Key string -> (notation, table of names A_k, shapes, dtypes)."""
    parts = key.split(";")
    fields = {}
    rest = []
    for p in parts:
        if p.startswith(("b=", "n=", "ext=", "dt=")):
            k, v = p.split("=", 1)
            fields[k] = v
        else:
            rest.append(p)
    notation, tab = rest
    ext = [int(x) for x in fields["ext"].split(",")] if fields["ext"] else []
    dts = [SHORT[x] for x in fields["dt"].split(",")]
    rows = [[f"A_{int(a)}" for a in r.split(",")] for r in tab.split("/")]
    ins = notation.split("->")[0].split(",")
    shapes = {}
    for row in rows:
        for j, a in enumerate(row):
            shapes[a] = tuple(ext[ord(c) - 97] for c in ins[j])
    dtypes = {f"A_{k}": d for k, d in enumerate(dts)}
    return notation, rows, shapes, dtypes


def brute_spec(notation, table, shapes, dtypes="float64"):
    from oracle import brute
    return brute.make(notation, table, shapes, dtypes)
