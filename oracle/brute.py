"""Brute-force isomorphism and normal form of batched einsums.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Pure Python, exponential
in b and n; meant for the tiny specs of the tests.

* :func:`isomorphism` follows Definitions "Einsum Isomorphism" and "Batched
  einsum Isomorphism" literally: it tries every member bijection sigma^i and
  every operand-position bijection sigma^j; once those two are fixed, the
  index map sigma^I and the argument map sigma^A are forced position by
  position, and the definition's conditions (equal index lists under sigma^I,
  equal arguments under sigma^A, equal shapes and dtypes) are checked.
* :func:`normal_form` is a second, independent route to the same equivalence:
  for every (sigma^i, sigma^j) it renames indices and arguments by first
  occurrence, serializes the result as an integer tuple, and keeps the
  lexicographic minimum.  For a fixed member and position order, naming by
  first occurrence is the unique representative under renaming, so two specs
  have equal normal forms exactly when some (sigma^i, sigma^j) and renaming make
  them equal -- the isomorphism of the definition (a canonicalization function
  in the sense of Definition "Canonicalization of a batched einsum").
* :func:`check_maps` verifies a given substitution (as printed in the paper's
  examples) against the definition.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations
from typing import Dict, Optional, Sequence, Tuple

# DtypeRank of the induced-graph construction (Appendix B.1, dtype ranks).
DTYPE_RANK = {"int8": 1, "int32": 2, "int64": 3, "float16": 4, "float32": 5,
              "float64": 6, "complex64": 7, "complex128": 8}


@dataclass(frozen=True)
class BSpec:
    """(b, n, I_out, (I_in^j), ((A^{i,j}))) plus shapes and dtypes of args."""
    out: str
    ins: Tuple[str, ...]
    table: Tuple[Tuple[str, ...], ...]
    shapes: Tuple[Tuple[str, Tuple[int, ...]], ...]
    dtypes: Tuple[Tuple[str, str], ...]

    @property
    def b(self) -> int:
        return len(self.table)

    @property
    def n(self) -> int:
        return len(self.ins)

    def shape(self, a: str) -> Tuple[int, ...]:
        return dict(self.shapes)[a]

    def dtype(self, a: str) -> str:
        return dict(self.dtypes)[a]


def make(notation: str, table: Sequence[Sequence[str]], shapes: Dict[str, Sequence[int]],
         dtypes: Dict[str, str] | str = "float64") -> BSpec:
    lhs, rhs = notation.split("->")
    ins = tuple(lhs.split(","))
    tab = tuple(tuple(r) for r in table)
    used = sorted({a for r in tab for a in r})
    if isinstance(dtypes, str):
        dtypes = {a: dtypes for a in used}
    spec = BSpec(rhs, ins, tab,
                 tuple((a, tuple(int(s) for s in shapes[a])) for a in used),
                 tuple((a, dtypes[a]) for a in used))
    validate(spec)
    return spec


def validate(spec: BSpec) -> Dict[str, int]:
    """Soundness conditions of Eq. (1) for every member, plus one extent per
    index across the whole batch.  Returns the extent of every index."""
    ext: Dict[str, int] = {}
    for row in spec.table:
        if len(row) != spec.n:
            raise ValueError("table row length differs from n")
        for j, a in enumerate(row):
            shp = spec.shape(a)
            if len(shp) != len(spec.ins[j]):
                raise ValueError("rank mismatch")
            for ch, s in zip(spec.ins[j], shp):
                if ext.setdefault(ch, s) != s:
                    raise ValueError("inconsistent extent")
    if len(set(spec.out)) != len(spec.out):
        raise ValueError("repeated output index")
    for ch in spec.out:
        if ch not in ext:
            raise ValueError("output index not in any input")
    return ext


def isomorphism(e1: BSpec, e2: BSpec):
    """Return (sigma_i, sigma_j, sigma_I, sigma_A) with e1 ~ e2, or None.

    Convention of the definitions: sigma_i, sigma_j map positions of e1 to
    positions of e2 (0-based); sigma_I maps e2 index names to e1 names and
    sigma_A maps e2 argument names to e1 names.
    """
    if (e1.b, e1.n, len(e1.out)) != (e2.b, e2.n, len(e2.out)):
        return None
    all1 = set(e1.out).union(*e1.ins)
    all2 = set(e2.out).union(*e2.ins)
    if len(all1) != len(all2):
        return None
    for si in permutations(range(e1.b)):
        for sj in permutations(range(e1.n)):
            m = check_maps(e1, e2, si, sj)
            if m is not None:
                return (si, sj) + m
    return None


def _extend(mp: dict, inv: dict, k, v) -> bool:
    if k in mp:
        return mp[k] == v
    if v in inv:
        return False
    mp[k] = v
    inv[v] = k
    return True


def check_maps(e1: BSpec, e2: BSpec, si, sj, sigma_I=None, sigma_A=None):
    """Check the definition for fixed sigma^i, sigma^j.  When sigma_I /
    sigma_A are given they must be consistent with the forced maps.  Returns
    the (sigma_I, sigma_A) maps or None."""
    sI: dict = {}
    sIinv: dict = {}
    sA: dict = {}
    sAinv: dict = {}
    for d in range(len(e1.out)):
        if not _extend(sI, sIinv, e2.out[d], e1.out[d]):
            return None
    for j in range(e1.n):
        l1, l2 = e1.ins[j], e2.ins[sj[j]]
        if len(l1) != len(l2):
            return None
        for d in range(len(l1)):
            if not _extend(sI, sIinv, l2[d], l1[d]):
                return None
    for i in range(e1.b):
        for j in range(e1.n):
            a1 = e1.table[i][j]
            a2 = e2.table[si[i]][sj[j]]
            if not _extend(sA, sAinv, a2, a1):
                return None
            if e1.shape(a1) != e2.shape(a2) or e1.dtype(a1) != e2.dtype(a2):
                return None
    if sigma_I is not None and any(sigma_I.get(k) != v for k, v in sI.items()):
        return None
    if sigma_A is not None and any(sigma_A.get(k) != v for k, v in sA.items()):
        return None
    return sI, sA


def _serialize(spec: BSpec, ext, si, sj):
    ins = [spec.ins[sj[j]] for j in range(spec.n)]
    tab = [[spec.table[si[i]][sj[j]] for j in range(spec.n)] for i in range(spec.b)]
    order: Dict[str, int] = {}
    for ch in spec.out + "".join(ins):
        order.setdefault(ch, len(order))
    args: Dict[str, int] = {}
    for row in tab:
        for a in row:
            args.setdefault(a, len(args))
    idx_by_ord = sorted(order, key=order.get)
    arg_by_ord = sorted(args, key=args.get)
    return (spec.b, spec.n,
            tuple(order[c] for c in spec.out),
            tuple(tuple(order[c] for c in s) for s in ins),
            tuple(ext[c] for c in idx_by_ord),
            tuple(tuple(args[a] for a in row) for row in tab),
            tuple(DTYPE_RANK[spec.dtype(a)] for a in arg_by_ord))


def normal_form(spec: BSpec):
    """Lexicographic minimum over sigma^i x sigma^j of first-occurrence forms."""
    ext = validate(spec)
    best = None
    for si in permutations(range(spec.b)):
        for sj in permutations(range(spec.n)):
            t = _serialize(spec, ext, si, sj)
            if best is None or t < best:
                best = t
    return best


def normal_form_cost(spec: BSpec) -> int:
    """Number of (sigma^i, sigma^j) pairs the brute force visits."""
    from math import factorial
    return factorial(spec.b) * factorial(spec.n)


def normal_form_spec(spec: BSpec) -> BSpec:
    """The normal form written back as a batched einsum (indices a, b, ...,
    arguments A_0, A_1, ...) -- convenient for printing and re-checking."""
    b, n, out, ins, ext, tab, dts = normal_form(spec)
    letters = "abcdefghijklmnopqrstuvwxyz"
    names = [f"A_{k}" for k in range(len(dts))]
    inv_rank = {v: k for k, v in DTYPE_RANK.items()}
    shapes = {}
    for j in range(n):
        for i in range(b):
            shapes[names[tab[i][j]]] = tuple(ext[c] for c in ins[j])
    return BSpec("".join(letters[c] for c in out),
                 tuple("".join(letters[c] for c in s) for s in ins),
                 tuple(tuple(names[a] for a in row) for row in tab),
                 tuple((a, shapes[a]) for a in names),
                 tuple((names[k], inv_rank[dts[k]]) for k in range(len(dts))))
