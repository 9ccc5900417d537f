"""Pins of the oracle's loop-nest evaluator and gradient (CPU only).

Each check ties the oracle to something other than itself: numpy's einsum or
matmul (library routines for special cases), the paper's worked examples,
closed forms (the GEMM gradient) and central finite differences.
"""
import numpy as np
import pytest

import oracle
from oracle import functional as F

RNG = np.random.default_rng(12220)


def _rand(*shape):
    return RNG.standard_normal(shape)


@pytest.mark.parametrize("notation,shapes", [
    ("ij,ej->ei", [(10, 10), (64, 10)]),
    ("er,rij,ej->ei", [(7, 3), (3, 5, 5), (7, 5)]),
    ("rij,exr,ej->exi", [(3, 4, 4), (6, 3, 3), (6, 4)]),
    ("abij,cdab->cdij", [(3, 2, 4, 2), (2, 3, 3, 2)]),
    ("ijk,ik,ij,ij->i", [(5, 4, 3), (5, 3), (5, 4), (5, 4)]),
    ("ij,ij->", [(4, 5), (4, 5)]),
    ("ii->i", [(6, 6)]),
    ("iij,j->i", [(3, 3, 4), (4,)]),
    ("ab,bc,cd,de->ae", [(2, 3), (3, 4), (4, 2), (2, 3)]),
    ("i,j->ij", [(4,), (5,)]),
    ("xre,rij,xej->ei", [(3, 3, 5), (3, 4, 4), (3, 5, 4)]),
])
def test_matches_numpy_einsum(notation, shapes):
    ops = [_rand(*s) for s in shapes]
    got = oracle.einsum(notation, *ops)
    ref = np.einsum(notation, *ops)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_zero_extent_gives_zero_fill():
    # Shape allows 0 and an empty sum is 0 (Definition of a multidimensional
    # array; Eq. (1)).
    A = np.zeros((3, 0))
    B = np.zeros((0, 4))
    got = oracle.einsum("ik,kj->ij", A, B)
    assert got.shape == (3, 4) and np.all(got == 0.0)


def test_invalid_notations_rejected():
    with pytest.raises(ValueError):
        oracle.einsum("ij,jk->ii", _rand(2, 3), _rand(3, 2))   # repeated output index
    with pytest.raises(ValueError):
        oracle.einsum("ij->ik", _rand(2, 3))                   # output index not in inputs
    with pytest.raises(ValueError):
        oracle.einsum("ij,jk->ik", _rand(2, 3), _rand(4, 2))   # inconsistent extent


def test_config1_is_a_gemm():
    # R_b[e,i] = sum_j D_b[i,j] u[e,j] = (u @ D_b^T)[e,i]
    u = _rand(64, 10)
    for _ in range(3):
        D = RNG.uniform(-1, 1, (10, 10))
        np.testing.assert_allclose(oracle.einsum("ij,ej->ei", D, u), u @ D.T,
                                   rtol=1e-13, atol=1e-13)


def test_dense_pair_is_a_gemm_after_reshape():
    # 'abij,cdab->cdij' is C[(cd),(ij)] = V[(cd),(ab)] @ T[(ab),(ij)]
    a, i = 3, 2
    T = _rand(a, a, i, i)
    V = _rand(a, a, a, a)
    got = oracle.einsum("abij,cdab->cdij", T, V)
    ref = (V.reshape(a * a, a * a) @ T.reshape(a * a, i * i)).reshape(a, a, i, i)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_batched_example(paper_examples):
    # Example 'Batched einsum': R1 = A B C, R2 = B C D (10 x 10 each).
    ex = paper_examples["batched_example"]
    arrs = {k: _rand(*s) for k, s in ex["shapes"].items()}
    R = oracle.batched_einsum(ex["notation"], ex["table"], arrs)
    np.testing.assert_allclose(R[0], arrs["A"] @ arrs["B"] @ arrs["C"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(R[1], arrs["B"] @ arrs["C"] @ arrs["D"], rtol=1e-12, atol=1e-12)


def test_functional_retrieval_listing(paper_examples):
    # Listing 'Computational scientist's view': u = P*P, v = 3 cos(Q) + 5,
    # w = sin(R); y1[i0] = sum_i1 u v, y2[i0] = sum_i1 u w, i0 < 96, i1 < 4.
    ex = paper_examples["functional_retrieval"]
    n0, n1 = ex["domain"]["i0"], ex["domain"]["i1"]
    P, Q, R = _rand(n0, n1), _rand(n1), _rand(n1)
    U = F.elementwise(P, "square")
    Vq = F.elementwise(Q, "cos", 3.0, 5.0)
    Wr = F.elementwise(R, "sin")
    y = oracle.batched_einsum("ij,j->i", [["U", "V"], ["U", "W"]],
                              {"U": U, "V": Vq, "W": Wr})
    # the generated OpenCL listing written out with numpy
    p = P * P
    y1 = (p * (3 * np.cos(Q) + 5)).sum(axis=1)
    y2 = (p * np.sin(R)).sum(axis=1)
    np.testing.assert_allclose(y[0], y1, rtol=1e-13)
    np.testing.assert_allclose(y[1], y2, rtol=1e-13)


def test_tet_jacobian_maps_reference_vertices():
    # The affine map sends reference vertex 0 to v0 and unit vector r to
    # v_{r+1}: x(e_r) - x(0) = J e_r = v_{r+1} - v_0.
    V = RNG.uniform(0, 1, (5, 4, 3))
    J = F.tet_jacobian(V)
    for r in range(3):
        xi = np.zeros(3)
        xi[r] = 1.0
        np.testing.assert_allclose(J @ xi, V[:, r + 1, :] - V[:, 0, :], rtol=0, atol=0)
    # volume of the tetrahedron = |det J| / 6 (a closed form for the unit
    # reference simplex)
    e0 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    np.testing.assert_allclose(np.linalg.det(F.tet_jacobian(e0[None]))[0], 1.0)


def test_strided_view_matches_numpy_view():
    W = _rand(3, 4, 5, 6)
    got = F.strided_view(W, (5, 6, 3, 4), (6, 1, 120, 30), 0)
    np.testing.assert_array_equal(got, W.transpose(2, 3, 0, 1))
    J = _rand(7, 3, 3)
    for x in range(3):
        np.testing.assert_array_equal(F.strided_view(J, (7, 3), (9, 1), 3 * x), J[:, x, :])


def test_einsum_at_matches_full():
    A, B = _rand(6, 5), _rand(5, 7)
    full = oracle.einsum("ik,kj->ij", A, B)
    pos = np.array([0, 3, 17, 41])
    np.testing.assert_allclose(oracle.einsum_at("ik,kj->ij", [A, B], pos), full.ravel()[pos],
                               rtol=0, atol=0)


def test_grad_closed_form_gemm():
    # R = A B, <G, R> has dA = G B^T and dB = A^T G.
    A, B, G = _rand(4, 3), _rand(3, 5), _rand(4, 5)
    np.testing.assert_allclose(oracle.einsum_grad("ik,kj->ij", [A, B], G, 0), G @ B.T, rtol=1e-13)
    np.testing.assert_allclose(oracle.einsum_grad("ik,kj->ij", [A, B], G, 1), A.T @ G, rtol=1e-13)


@pytest.mark.parametrize("notation,shapes", [
    ("abij,cdab->cdij", [(2, 2, 3, 2), (2, 3, 2, 2)]),
    ("rij,exr,ej->exi", [(2, 3, 3), (2, 2, 2), (2, 3)]),
    ("ii,i->i", [(3, 3), (3,)]),
    ("ij,ij->", [(3, 4), (3, 4)]),
])
def test_grad_central_differences(notation, shapes):
    ops = [_rand(*s) for s in shapes]
    R = oracle.einsum(notation, *ops)
    G = _rand(*R.shape) if R.ndim else np.array(RNG.standard_normal())
    h = 1e-6
    for k in range(len(ops)):
        g = oracle.einsum_grad(notation, ops, G, k)
        fd = np.zeros_like(ops[k])
        # repeated labels read only the diagonal, so only those entries move
        for idx in np.ndindex(ops[k].shape):
            p = [o.copy() for o in ops]
            m = [o.copy() for o in ops]
            p[k][idx] += h
            m[k][idx] -= h
            fd[idx] = (np.sum(G * oracle.einsum(notation, *p)) -
                       np.sum(G * oracle.einsum(notation, *m))) / (2 * h)
        np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("notation,shapes", [
    ("abij,cdab->cdij", [(2, 3, 2, 2), (3, 2, 2, 3)]),
    ("er,rij,ej->ei", [(5, 3), (3, 4, 4), (5, 4)]),
])
def test_grad_at_matches_full_grad(notation, shapes):
    ops = [_rand(*s) for s in shapes]
    R = oracle.einsum(notation, *ops)
    G = _rand(*R.shape)
    for k in range(len(ops)):
        full = oracle.einsum_grad(notation, ops, G, k)
        pos = np.arange(full.size)
        np.testing.assert_allclose(oracle.einsum_grad_at(notation, ops, G, k, pos),
                                   full.ravel(), rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------------------
# Element-wise functional operands with a second source (Definition
# "Functional Batched Einstein Summation": an argument is replaced by a
# function of its index tuple; here alpha * op(S0[idx]) + beta + S1[idx]).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("op,args,values", [
    # arguments at which the function value is fixed by the mathematics and
    # exactly representable (sin pi/2 = 1 and cos pi = -1 round exactly in
    # FP64; the squares are exact binary fractions)
    ("sin", [0.0, np.pi / 2, -np.pi / 2, np.pi / 6], [0.0, 1.0, -1.0, 0.5]),
    ("cos", [0.0, np.pi, 2 * np.pi, np.pi / 3], [1.0, -1.0, 1.0, 0.5]),
    ("square", [0.0, 3.0, -0.5, 1.5], [0.0, 9.0, 0.25, 2.25]),
    ("id", [0.0, 3.0, -0.5, 1.5], [0.0, 3.0, -0.5, 1.5]),
])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (2.0, 0.5), (-3.0, 1.25)])
def test_elementwise_two_sources_known_values(op, args, values, alpha, beta):
    # b is chosen so that every plausible mis-wiring gives another value:
    # dropping b, adding it inside alpha*op(.) (alpha != 1), applying op to
    # it, or swapping the two sources.
    a = np.array(args)
    b = np.array([0.25, -1.5, 2.0, 0.75])
    got = F.elementwise(a, op, alpha, beta, b)
    want = alpha * np.array(values) + beta + b
    # pi/6 and pi/3 are rounded arguments: the values hold within a few ulp
    np.testing.assert_allclose(got, want, rtol=0, atol=4e-15)
    # the single-source form is the same without b
    np.testing.assert_allclose(F.elementwise(a, op, alpha, beta), want - b, rtol=0, atol=4e-15)


def test_elementwise_second_source_is_added_outside_alpha():
    # alpha * op(a) + beta + b with a = 0 under sin: the value is beta + b
    # whatever alpha is; alpha * (op(a) + b) + beta would give beta + alpha b.
    a = np.zeros(3)
    b = np.array([1.0, -2.0, 4.0])
    for alpha in (2.0, -1.0, 10.0):
        np.testing.assert_array_equal(F.elementwise(a, "sin", alpha, 0.5, b), 0.5 + b)


def test_functional_p4_batch_against_hand_materialized_numpy():
    # A tiny instance of the functional P4 batch 'rij,exr,ej->exi' built by
    # the seeded workload generator, evaluated along the oracle's own path
    # (operand materialization, then the loop nest), against numpy.einsum on
    # operands materialized by hand from their definitions:
    #   u_k[e, j] = sin(a_k[e, j]) + b_k[e, j]
    #   J[e, x, r] = V[e, r + 1, x] - V[e, 0, x]   (affine tetrahedron map)
    import workloads
    from tests.gpu_util import oracle_full
    w = workloads.config3(e=9, ni=5)
    got = oracle_full(w)
    V = w.buffers["V"].numpy()
    J = np.transpose(V[:, 1:, :] - V[:, :1, :], (0, 2, 1))
    D = w.buffers["D"].numpy()
    for k in range(4):
        u = np.sin(w.buffers[f"a{k}"].numpy()) + w.buffers[f"b{k}"].numpy()
        ref = np.einsum("rij,exr,ej->exi", D, J, u)
        np.testing.assert_allclose(got[k], ref, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------------------
# The face-mass and local-divergence classes (Section "Batched einsums in
# DG-FEM Operators"; kernel patterns in Appendix "DG-FEM Batched Einsum Kernel
# Patterns"): the oracle's loop nest on their notations against the listings'
# semantics written per element with numpy matrix-vector products.
# ---------------------------------------------------------------------------

def test_face_mass_against_listing_semantics():
    import workloads
    w = workloads.face_mass(p=2, e=9, b=3)
    vals = {k: v.numpy() for k, v in w.buffers.items()}
    got = oracle.batched_einsum(w.notation, w.table, {a: vals[a] for a in w.operands})
    J, M = vals["J"], vals["M"]
    for k, row in enumerate(w.table):
        F_ = vals[row[2]]
        ref = np.zeros((9, M.shape[0]))
        for e in range(9):
            for f in range(4):                 # y[e] += J[f,e] * M[:,f,:] @ F[f,e,:]
                ref[e] += J[f, e] * (M[:, f, :] @ F_[f, e, :])
        np.testing.assert_allclose(got[k], ref, rtol=1e-13, atol=1e-13)


def test_local_divergence_against_listing_semantics():
    import workloads
    w = workloads.local_divergence(p=1, e=7, b=2)
    vals = {k: v.numpy() for k, v in w.buffers.items()}
    got = oracle.batched_einsum(w.notation, w.table, {a: vals[a] for a in w.operands})
    J, D = vals["J"], vals["D"]
    for k, row in enumerate(w.table):
        U = vals[row[2]]
        ref = np.zeros((7, D.shape[1]))
        for e in range(7):
            for x in range(3):                 # component x of the vector field
                for r in range(3):
                    ref[e] += J[x, r, e] * (D[r] @ U[x, e, :])
        np.testing.assert_allclose(got[k], ref, rtol=1e-13, atol=1e-13)


def test_local_divergence_of_a_constant_field_is_zero():
    # D with zero row sums differentiates constants to zero: with every
    # component of the field constant in j, the divergence vanishes exactly
    # up to rounding, for any geometry J
    import workloads
    w = workloads.local_divergence(p=1, e=5, b=1)
    vals = {k: v.numpy().copy() for k, v in w.buffers.items()}
    D = vals["D"]
    D -= D.mean(axis=2, keepdims=True)        # rows sum to zero
    U = np.broadcast_to(RNG.standard_normal((3, 5, 1)), (3, 5, 4)).copy()
    vals["U0"] = U
    got = oracle.batched_einsum(w.notation, w.table, vals)
    assert np.abs(got[0]).max() < 1e-13


def test_affine_binary_contraction_against_numpy():
    # (alpha_1 A + beta_1)(alpha_2 B + beta_2) contracted: the oracle on the
    # functional operands against numpy.einsum on hand-materialized ones
    import workloads
    from tests.gpu_util import oracle_full
    w = workloads.tccg_like(3, min_elems=1 << 8, max_elems=1 << 12)
    A, B = w.buffers["A"].numpy(), w.buffers["B"].numpy()
    oa, ob = w.operands["Ax"], w.operands["Bx"]
    ref = np.einsum(w.notation, oa.alpha * A + oa.beta, ob.alpha * B + ob.beta)
    np.testing.assert_allclose(oracle_full(w)[0], ref, rtol=1e-12, atol=1e-12)
