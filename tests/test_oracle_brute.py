"""Pins of the brute-force isomorphism and normal form (CPU only).

The two brute-force routines take different routes (forced maps checked
against the definitions, versus first-occurrence serialization); they are
checked against each other, against the substitution maps printed in the
paper's examples, and against the invariances the definitions require.
"""
import random
import string
from itertools import permutations

import pytest

from oracle import brute


def _spec(d, dtype="float64", default_extent=None):
    shapes = d.get("shapes")
    if shapes is None:
        shapes = {}
        lhs = d["notation"].split("->")[0].split(",")
        for row in d["table"]:
            for j, a in enumerate(row):
                shapes[a] = tuple(default_extent for _ in lhs[j])
    return brute.make(d["notation"], d["table"], shapes, d.get("dtype", dtype))


def test_fig1_pair_and_printed_substitution(paper_examples):
    ex = paper_examples["fig1_sameish"]
    e1, e2 = _spec(ex["e1"], default_extent=3), _spec(ex["e2"], default_extent=3)
    assert brute.isomorphism(e1, e2) is not None
    assert brute.normal_form(e1) == brute.normal_form(e2)
    sub = ex["subst_e1_to_e2"]
    # the caption maps e1 names to e2 names; the definition's maps go e2 -> e1
    sI = {v: k for k, v in sub["indices"].items()}
    sA = {v: k for k, v in sub["args"].items()}
    si = [sub["members"][str(i + 1)] - 1 for i in range(3)]
    ok = [sj for sj in permutations(range(3))
          if brute.check_maps(e1, e2, si, sj, sI, sA) is not None]
    assert ok, "printed substitution does not satisfy the definition"


def test_isomorphic_einsums_example(paper_examples):
    ex = paper_examples["isomorphic_einsums"]
    e1, e2 = _spec(ex["e1"]), _spec(ex["e2"])
    sj = [ex["sigma_j"][str(j + 1)] - 1 for j in range(2)]
    assert brute.check_maps(e1, e2, [0], sj, ex["sigma_I"], ex["sigma_A"]) is not None
    assert brute.normal_form(e1) == brute.normal_form(e2)


def test_isomorphic_batched_example(paper_examples):
    ex = paper_examples["isomorphic_batched"]
    e1, e2 = _spec(ex["e1"]), _spec(ex["e2"])
    si = [ex["sigma_i"][str(i + 1)] - 1 for i in range(2)]
    sj = [ex["sigma_j"][str(j + 1)] - 1 for j in range(4)]
    assert brute.check_maps(e1, e2, si, sj, ex["sigma_I"], ex["sigma_A"]) is not None
    assert brute.normal_form(e1) == brute.normal_form(e2)
    # near miss: un-share B in row 2 (a fresh argument E takes its place)
    d = dict(ex["e1"])
    d["table"] = [["A", "B", "C", "D"], ["A", "B", "C", "E"]]
    d["shapes"] = dict(d["shapes"], E=[5, 10])
    near = _spec(d)
    assert brute.isomorphism(near, e2) is None
    assert brute.normal_form(near) != brute.normal_form(e2)


def test_canonical_example_pair(paper_examples):
    ex = paper_examples["canonical_example"]
    e1, e2 = _spec(ex["e1"]), _spec(ex["e2"])
    assert brute.normal_form(e1) == brute.normal_form(e2)
    # the paper's canonical form is itself a member of the class
    c = ex["canonical"]
    canon = brute.make(",".join(c["ins"]) + "->" + c["out"], c["table"], c["shapes"], c["dtype"])
    assert brute.isomorphism(canon, e1) is not None


def test_wrong_maps_are_rejected(paper_examples):
    ex = paper_examples["isomorphic_einsums"]
    e1, e2 = _spec(ex["e1"]), _spec(ex["e2"])
    # identity operand order cannot work: shapes (10,4) vs (4,10) differ
    assert brute.check_maps(e1, e2, [0], [0, 1]) is None
    bad_I = dict(ex["sigma_I"], p="j", q="i")
    assert brute.check_maps(e1, e2, [0], [1, 0], bad_I, ex["sigma_A"]) is None


# ---------------------------------------------------------------------------
# Randomized agreement between the two brute-force routes
# ---------------------------------------------------------------------------

def _random_spec(rng):
    n = rng.randint(1, 3)
    m = rng.randint(1, 4)
    letters = rng.sample(string.ascii_lowercase[:8], m)
    ins = ["".join(rng.choice(letters) for _ in range(rng.randint(1, 2))) for _ in range(n)]
    used = sorted(set("".join(ins)))
    out = "".join(rng.sample(used, rng.randint(0, min(2, len(used)))))
    ext = {c: rng.choice([2, 3]) for c in used}
    b = rng.randint(1, 3)
    table, pool = [], []
    for i in range(b):
        row = []
        for j in range(n):
            cands = [a for a in pool if a[1] == ins[j]]
            if cands and rng.random() < 0.5:
                row.append(rng.choice(cands)[0])
            else:
                nm = f"X{len(pool)}"
                pool.append((nm, ins[j]))
                row.append(nm)
        table.append(row)
    shapes = {nm: tuple(ext[c] for c in lab) for nm, lab in pool}
    dts = {nm: rng.choice(["float64", "float64", "float32"]) for nm, _ in pool}
    return brute.make(",".join(ins) + "->" + out, table, shapes, dts)


def _random_variant(rng, spec):
    b, n = spec.b, spec.n
    used = sorted(set(spec.out).union(*spec.ins))
    fresh = rng.sample(string.ascii_lowercase, len(used))
    imap = dict(zip(used, fresh))
    pi = list(range(b)); rng.shuffle(pi)
    pj = list(range(n)); rng.shuffle(pj)
    args = sorted({a for r in spec.table for a in r})
    names = [f"Y{k}" for k in range(len(args))]
    rng.shuffle(names)
    amap = dict(zip(args, names))
    ins = ["".join(imap[c] for c in spec.ins[pj[j]]) for j in range(n)]
    table = [[amap[spec.table[pi[i]][pj[j]]] for j in range(n)] for i in range(b)]
    shapes = {amap[a]: spec.shape(a) for a in args}
    dts = {amap[a]: spec.dtype(a) for a in args}
    return brute.make(",".join(ins) + "->" + "".join(imap[c] for c in spec.out),
                      table, shapes, dts)


def test_variants_share_normal_form():
    rng = random.Random(7)
    for _ in range(60):
        s = _random_spec(rng)
        nf = brute.normal_form(s)
        for _ in range(4):
            v = _random_variant(rng, s)
            assert brute.normal_form(v) == nf
            assert brute.isomorphism(s, v) is not None


def test_normal_form_equality_iff_isomorphic():
    rng = random.Random(11)
    specs = [_random_spec(rng) for _ in range(70)]
    # add near misses of the first few: swap axes of one operand, change one extent
    for s in specs[:20]:
        specs.append(_random_variant(rng, s))
    for i in range(len(specs)):
        for j in range(i + 1, len(specs)):
            a, b = specs[i], specs[j]
            same_nf = brute.normal_form(a) == brute.normal_form(b)
            iso = brute.isomorphism(a, b) is not None
            assert same_nf == iso, (a, b)


def test_normal_form_spec_round_trip():
    rng = random.Random(3)
    for _ in range(30):
        s = _random_spec(rng)
        c = brute.normal_form_spec(s)
        assert brute.isomorphism(c, s) is not None
        assert brute.normal_form(c) == brute.normal_form(s)
        assert brute.normal_form_spec(c) == c   # idempotent
