"""Seeded synthetic inputs for batched-einsum workloads.

This module only draws random numbers and describes operands; it holds none of
the method's arithmetic (no canonicalization, no contraction, no functional
operand evaluation).  Both the oracle-side tests and the HIP path consume what
it produces, so both see bit-identical inputs.

Every random tensor is drawn in FP64 on the CPU from
``torch.Generator().manual_seed(2601_12220 + 100 * config + k)`` and then
rounded once to the workload's compute dtype.

Operand kinds (what the library calls functional operands):

* ``array``        M(A)[idx] = S0[idx]  (dense row-major buffer)
* ``view``         M(A)[idx] = S0[offset + sum idx_k * strides_k]
* ``elementwise``  M(A)[idx] = alpha * op(S0[idx]) + beta (+ S1[idx])
* ``tet_jacobian`` M(A)[e, x, r] from vertex coordinates S0[e, 4, 3]
* ``expr``         M(A)[idx] = body(S0[idx], S1[idx]) for an expression body
"""
from __future__ import annotations

import random
import string
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional, Sequence, Tuple

import torch

SEED_BASE = 2601_12220


def gen(config: int, k: int) -> torch.Generator:
    return torch.Generator().manual_seed(SEED_BASE + 100 * config + k)


@dataclass
class Operand:
    name: str
    shape: Tuple[int, ...]
    dtype: str                       # "float32" | "float64"
    kind: str = "array"              # array | view | elementwise | tet_jacobian
    sources: Tuple[str, ...] = ()    # buffer names
    offset: int = 0                  # view: element offset into sources[0]
    strides: Optional[Tuple[int, ...]] = None  # view / elementwise strides
    op: str = "id"                   # elementwise: id | sin | cos | square
    alpha: float = 1.0
    beta: float = 0.0
    expr: Optional[str] = None       # expr: body over s0, s1 (e.g. "3*cos(s0)+5")


@dataclass
class Workload:
    name: str
    notation: str
    table: List[List[str]]
    operands: Dict[str, Operand]
    buffers: Dict[str, torch.Tensor]   # CPU tensors in the compute dtype
    dtype: str
    info: Dict[str, object] = field(default_factory=dict)

    @property
    def b(self) -> int:
        return len(self.table)

    @property
    def n(self) -> int:
        return len(self.table[0])

    def out_shape(self) -> Tuple[int, ...]:
        lhs, rhs = self.notation.split("->")
        ext = {}
        for labels, a in zip(lhs.split(","), self.table[0]):
            for ch, s in zip(labels, self.operands[a].shape):
                ext[ch] = s
        return tuple(ext[ch] for ch in rhs)


def _tdtype(dtype: str):
    return {"float32": torch.float32, "float64": torch.float64}[dtype]


def _normal(config, k, shape, dtype):
    return torch.randn(*shape, generator=gen(config, k), dtype=torch.float64).to(_tdtype(dtype))


def _uniform(config, k, shape, lo, hi, dtype):
    x = torch.rand(*shape, generator=gen(config, k), dtype=torch.float64)
    return (lo + (hi - lo) * x).to(_tdtype(dtype))


def _dense(name, t, dtype):
    return Operand(name, tuple(t.shape), dtype, "array", (name,))


# ---------------------------------------------------------------------------
# Config 1: tiny FEM-style batch 'ij,ej->ei', b = 3, shared u[e=64, j=10]
# ---------------------------------------------------------------------------

def config1(e: int = 64, nj: int = 10, dtype: str = "float64") -> Workload:
    bufs = {"u": _normal(1, 0, (e, nj), dtype)}
    for m in range(3):
        bufs[f"D{m}"] = _uniform(1, 1 + m, (nj, nj), -1.0, 1.0, dtype)
    ops = {k: _dense(k, v, dtype) for k, v in bufs.items()}
    return Workload("fem_matvec_b3", "ij,ej->ei",
                    [["D0", "u"], ["D1", "u"], ["D2", "u"]], ops, bufs, dtype,
                    {"e": e, "nj": nj})


# ---------------------------------------------------------------------------
# Config 2: out_x[e,i] = sum_{r,j} J[e,x,r] D[r,i,j] u[e,j], x = 0..2
# ---------------------------------------------------------------------------

def fem_jacobian(config, k, e, dtype):
    """J[e,3,3]: diagonal U[0.5,1.5], off-diagonal U[-0.1,0.1]."""
    diag = _uniform(config, k, (e, 3, 3), 0.5, 1.5, "float64")
    off = _uniform(config, k + 50, (e, 3, 3), -0.1, 0.1, "float64")
    eye = torch.eye(3, dtype=torch.bool).expand(e, 3, 3)
    return torch.where(eye, diag, off).to(_tdtype(dtype))


def config2(e: int = 1 << 20, ni: int = 20, dtype: str = "float64") -> Workload:
    bufs = {"J": fem_jacobian(2, 0, e, dtype),
            "D": _uniform(2, 1, (3, ni, ni), -1.0, 1.0, dtype),
            "u": _normal(2, 2, (e, ni), dtype)}
    ops = {"D": _dense("D", bufs["D"], dtype), "u": _dense("u", bufs["u"], dtype)}
    for x in range(3):
        ops[f"J{x}"] = Operand(f"J{x}", (e, 3), dtype, "view", ("J",),
                               offset=3 * x, strides=(9, 1))
    return Workload("fem_grad_p3", "er,rij,ej->ei",
                    [["J0", "D", "u"], ["J1", "D", "u"], ["J2", "D", "u"]],
                    ops, bufs, dtype, {"e": e, "ni": ni})


# ---------------------------------------------------------------------------
# Config 3: functional operands 'rij,exr,ej->exi', b = 4, P4 (i = j = 35)
# ---------------------------------------------------------------------------

def config3(e: int = 1 << 19, ni: int = 35, dtype: str = "float64") -> Workload:
    bufs = {"V": _uniform(3, 0, (e, 4, 3), 0.0, 1.0, dtype),
            "D": _uniform(3, 1, (3, ni, ni), -1.0, 1.0, dtype)}
    ops = {"D": _dense("D", bufs["D"], dtype),
           "J": Operand("J", (e, 3, 3), dtype, "tet_jacobian", ("V",))}
    table = []
    for k in range(4):
        bufs[f"a{k}"] = _normal(3, 2 + 2 * k, (e, ni), dtype)
        bufs[f"b{k}"] = _normal(3, 3 + 2 * k, (e, ni), dtype)
        ops[f"u{k}"] = Operand(f"u{k}", (e, ni), dtype, "elementwise",
                               (f"a{k}", f"b{k}"), op="sin")
        table.append(["D", "J", f"u{k}"])
    return Workload("fem_grad_functional_p4", "rij,exr,ej->exi", table, ops,
                    bufs, dtype, {"e": e, "ni": ni})


# ---------------------------------------------------------------------------
# The other two DG-FEM classes at the paper's shapes (P1..P4, e = 10^5, a
# sweep over b), as their kernel-pattern listings index the arrays:
#   face mass        y_k[e,i] = sum_{f,j} J[f,e] M[i,f,j] F_k[f,e,j]
#                    'fe,ifj,fej->ei'; f = 4 faces, j = face DOFs
#   local divergence y_k[e,i] = sum_{x,r,j} J[x,r,e] D[r,i,j] U_k[x,e,j]
#                    'xre,rij,xej->ei'; U_k holds the three components of a
#                    vector field as planes U_k[x] of one buffer
# ---------------------------------------------------------------------------

VOLUME_DOFS = {1: 4, 2: 10, 3: 20, 4: 35}     # P_k tetrahedron
FACE_DOFS = {1: 3, 2: 6, 3: 10, 4: 15}        # P_k triangle


def face_mass(p: int = 3, e: int = 100_000, b: int = 1, dtype: str = "float64") -> Workload:
    ni, nj = VOLUME_DOFS[p], FACE_DOFS[p]
    bufs = {"J": _uniform(6, 0, (4, e), 0.5, 1.5, dtype),
            "M": _uniform(6, 1, (ni, 4, nj), -1.0, 1.0, dtype)}
    ops = {"J": _dense("J", bufs["J"], dtype), "M": _dense("M", bufs["M"], dtype)}
    table = []
    for k in range(b):
        bufs[f"F{k}"] = _normal(6, 2 + k, (4, e, nj), dtype)
        ops[f"F{k}"] = _dense(f"F{k}", bufs[f"F{k}"], dtype)
        table.append(["J", "M", f"F{k}"])
    return Workload(f"face_mass_p{p}", "fe,ifj,fej->ei", table, ops, bufs, dtype,
                    {"e": e, "ni": ni, "nj": nj, "p": p})


def local_divergence(p: int = 3, e: int = 100_000, b: int = 1,
                     dtype: str = "float64") -> Workload:
    n = VOLUME_DOFS[p]
    jac = fem_jacobian(7, 0, e, "float64")             # [e, x, r]
    bufs = {"J": jac.permute(1, 2, 0).contiguous().to(_tdtype(dtype)),   # [x, r, e]
            "D": _uniform(7, 1, (3, n, n), -1.0, 1.0, dtype)}
    ops = {"J": _dense("J", bufs["J"], dtype), "D": _dense("D", bufs["D"], dtype)}
    table = []
    for k in range(b):
        bufs[f"U{k}"] = _normal(7, 2 + k, (3, e, n), dtype)
        ops[f"U{k}"] = _dense(f"U{k}", bufs[f"U{k}"], dtype)
        table.append(["J", "D", f"U{k}"])
    return Workload(f"local_div_p{p}", "xre,rij,xej->ei", table, ops, bufs, dtype,
                    {"e": e, "ni": n, "nj": n, "p": p})


# ---------------------------------------------------------------------------
# Binary contractions with affine operands (alpha_1 A + beta_1)(alpha_2 B +
# beta_2), the extension of the TCCG suite in Section "TCCG Benchmark suite
# with Unmaterialized Operands".  The suite itself is not available here: a
# seeded generator draws contractions of the same kind -- 1-3 free indices
# per operand, 1-3 contracted indices, operand and output axes in random
# orders (the transpositions that make them tensor contractions rather than
# GEMMs), extents multiples of 8, the largest tensor of 2^20 - 2^24 elements
# -- with FP64 data and runtime scalars.
# ---------------------------------------------------------------------------

TCCG_EXTENTS = (8, 16, 24, 32, 48, 64, 72, 96)


def tccg_like(case: int, dtype: str = "float64", affine: bool = True,
              max_elems: int = 1 << 24, min_elems: int = 1 << 20) -> Workload:
    rng = random.Random(SEED_BASE + 800 + case)
    while True:
        na, nb, nk = rng.randint(1, 3), rng.randint(1, 3), rng.randint(1, 3)
        if na + nb + nk > 6:
            continue
        letters = rng.sample(string.ascii_lowercase[:12], na + nb + nk)
        fa, fb, kk = letters[:na], letters[na:na + nb], letters[na + nb:]
        ext = {c: rng.choice(TCCG_EXTENTS) for c in letters}
        size = lambda ls: _prod(ext[c] for c in ls)    # noqa: E731
        big = max(size(fa + kk), size(kk + fb), size(fa + fb))
        if min_elems <= big <= max_elems:
            break
    A = fa + kk
    B = kk + fb
    rng.shuffle(A)
    rng.shuffle(B)
    out = fa + fb
    rng.shuffle(out)
    notation = "".join(A) + "," + "".join(B) + "->" + "".join(out)
    bufs = {"A": _normal(8, 2 * case, tuple(ext[c] for c in A), dtype),
            "B": _normal(8, 2 * case + 1, tuple(ext[c] for c in B), dtype)}
    ops = {}
    for nm in ("A", "B"):
        shape = tuple(bufs[nm].shape)
        if affine:
            alpha = round(rng.uniform(0.5, 2.0), 3)
            beta = round(rng.uniform(-1.0, 1.0), 3)
            ops[nm + "x"] = Operand(nm + "x", shape, dtype, "elementwise", (nm,),
                                    op="id", alpha=alpha, beta=beta)
        else:
            ops[nm + "x"] = Operand(nm + "x", shape, dtype, "array", (nm,))
    return Workload(f"tccg_like_{case}", notation, [["Ax", "Bx"]], ops, bufs, dtype,
                    {"ext": ext, "free_a": na, "free_b": nb, "contracted": nk})


# ---------------------------------------------------------------------------
# Config 5: dense pair sharing T: 'abij,cdab->cdij' rows (T, V), (T, W')
# with W'[c,d,a,b] = W[a,b,c,d] a permuted view.
# ---------------------------------------------------------------------------

def config5(a: int = 64, i: int = 32, dtype: str = "float32") -> Workload:
    bufs = {"T": _normal(5, 0, (a, a, i, i), dtype),
            "V": _normal(5, 1, (a, a, a, a), dtype),
            "W": _normal(5, 2, (a, a, a, a), dtype)}
    a2, a3 = a * a, a * a * a
    ops = {"T": _dense("T", bufs["T"], dtype), "V": _dense("V", bufs["V"], dtype),
           "Wp": Operand("Wp", (a, a, a, a), dtype, "view", ("W",), offset=0,
                         strides=(a, 1, a3, a2))}
    return Workload("dense_pair_shared_T", "abij,cdab->cdij",
                    [["T", "V"], ["T", "Wp"]], ops, bufs, dtype, {"a": a, "i": i})


# ---------------------------------------------------------------------------
# Config 4: 256 random batched einsums of uneven shapes, 25 % variants
# ---------------------------------------------------------------------------

EXTENTS = (4, 8, 16, 32, 64)


def _random_structure(rng: random.Random):
    while True:
        n = rng.randint(2, 4)
        m = rng.randint(3, 6)
        letters = rng.sample(string.ascii_lowercase, m)
        ins = []
        for _ in range(n):
            ins.append("".join(rng.sample(letters, rng.randint(1, min(3, m)))))
        used = set("".join(ins))
        missing = [c for c in letters if c not in used]
        for c in missing:           # every index appears in some operand
            j = rng.randrange(n)
            if len(ins[j]) < 3:
                ins[j] += c
            else:
                ins[j] = ins[j][:-1] + c
        used = sorted(set("".join(ins)))
        if len(used) < 3:
            continue
        out = "".join(rng.sample(used, rng.randint(1, min(3, len(used)))))
        for _ in range(64):
            ext = {c: rng.choice(EXTENTS) for c in used}
            space = 1
            for c in used:
                space *= ext[c]
            big = max(_prod(ext[c] for c in s) for s in ins)
            if space <= (1 << 21) and big <= (1 << 20):
                return n, ins, out, ext
        # extents could not be made to fit: draw a new structure


def _prod(xs):
    p = 1
    for x in xs:
        p *= x
    return p


def random_batched(rng: random.Random, tag: str):
    """A random batched einsum structure: (notation, table, shapes)."""
    n, ins, out, ext = _random_structure(rng)
    b = rng.randint(1, 8)
    names = []
    table = []
    for i in range(b):
        row = []
        for j in range(n):
            if i > 0 and rng.random() < 0.5:
                row.append(table[0][j])
            else:
                nm = f"{tag}a{len(names)}"
                names.append(nm)
                row.append(nm)
        table.append(row)
    shapes = {}
    for row in table:
        for j, nm in enumerate(row):
            shapes[nm] = tuple(ext[c] for c in ins[j])
    return ",".join(ins) + "->" + out, table, shapes


def variant_of(rng: random.Random, notation: str, table, shapes, tag: str):
    """Random index renaming, member and position permutation and argument
    renaming of a batched einsum.  Returns the new structure and the maps
    used: (notation, table, shapes, member_perm, pos_perm, index_map, arg_map)."""
    lhs, rhs = notation.split("->")
    ins = lhs.split(",")
    b, n = len(table), len(ins)
    used = sorted(set("".join(ins)))
    fresh = rng.sample(string.ascii_lowercase, len(used))
    imap = dict(zip(used, fresh))
    pi = list(range(b))
    rng.shuffle(pi)
    pj = list(range(n))
    rng.shuffle(pj)
    old_args = []
    for row in table:
        for a in row:
            if a not in old_args:
                old_args.append(a)
    perm_names = old_args[:]
    rng.shuffle(perm_names)
    amap = {a: f"{tag}v{k}" for k, a in enumerate(perm_names)}
    new_ins = ["".join(imap[c] for c in ins[pj[j]]) for j in range(n)]
    new_out = "".join(imap[c] for c in rhs)
    new_table = [[amap[table[pi[i]][pj[j]]] for j in range(n)] for i in range(b)]
    new_shapes = {amap[a]: shapes[a] for a in old_args}
    return (",".join(new_ins) + "->" + new_out, new_table, new_shapes, pi, pj,
            imap, amap)


def config4(count: int = 256, n_variants: int = 64, dtype: str = "float32",
            seed_k: int = 0):
    """``count`` batched einsums; ``n_variants`` of them (at random positions)
    are renamed/permuted copies of earlier ones.  Returns a list of
    Workload objects; ``info['variant_of']`` names the original's position."""
    rng = random.Random(SEED_BASE + 400 + seed_k)
    positions = sorted(rng.sample(range(1, count), n_variants))
    structures = []
    for p in range(count):
        tag = f"w{p}_"
        if p in positions:
            src = rng.choice([q for q in range(p) if q not in positions] or [0])
            nota, tab, shp = structures[src][:3]
            v = variant_of(rng, nota, tab, shp, tag)
            structures.append((v[0], v[1], v[2], src))
        else:
            nota, tab, shp = random_batched(rng, tag)
            structures.append((nota, tab, shp, None))
    out = []
    for p, (nota, tab, shp, src) in enumerate(structures):
        bufs = {}
        ops = {}
        for k, nm in enumerate(sorted(shp)):
            bufs[nm] = _normal(4, 1000 * p + k + 1, shp[nm], dtype)
            ops[nm] = _dense(nm, bufs[nm], dtype)
        out.append(Workload(f"random_{p}", nota, tab, ops, bufs, dtype,
                            {"variant_of": src}))
    return out


# ---------------------------------------------------------------------------
# Small specs used by the canonicalization tests (structure only)
# ---------------------------------------------------------------------------

def spec_structure(w: Workload):
    """(notation, table, shapes, dtypes) of a workload, for key tests."""
    shapes = {k: o.shape for k, o in w.operands.items()}
    dtypes = {k: o.dtype for k, o in w.operands.items()}
    return w.notation, w.table, shapes, dtypes
