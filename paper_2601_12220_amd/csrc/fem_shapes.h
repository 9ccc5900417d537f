// Extents (NI, NJ, NR, NX) for which the FEM-stream template is compiled:
// the local-gradient class of DG-FEM operators on P1..P4 tetrahedra
// (i = j in {4, 10, 20, 35}, x = r = 3; Section "Batched einsums in DG-FEM
// Operators"), the same with one output component per member (x absent),
// and plain element-wise mat-vecs (r and x absent).
#pragma once

#ifndef BES_FEM_SHAPES
#define BES_FEM_SHAPES(X)                                                  \
  X(4, 4, 1, 1) X(10, 10, 1, 1) X(20, 20, 1, 1) X(35, 35, 1, 1)            \
  X(4, 4, 3, 1) X(10, 10, 3, 1) X(20, 20, 3, 1) X(35, 35, 3, 1)            \
  X(4, 4, 3, 3) X(10, 10, 3, 3) X(20, 20, 3, 3) X(35, 35, 3, 3)
#endif

inline bool fem_shape_compiled(bool /*f64*/, int ni, int nj, int nr, int nx) {
#define BES_FEM_MATCH(a, b, c, d) \
  if (ni == (a) && nj == (b) && nr == (c) && nx == (d)) return true;
  BES_FEM_SHAPES(BES_FEM_MATCH)
#undef BES_FEM_MATCH
  return false;
}

// Extents (NI, NJ, NC, NX, DIAG) of the FEM-stream "apply" class: face mass
// on P1..P4 tetrahedra (i volume DOFs 4/10/20/35, j face DOFs 3/6/10/15,
// f = 4 faces; the geometry term is diagonal in the face) and local
// divergence (i = j volume DOFs, r = x = 3).
#ifndef BES_FEM_APPLY_SHAPES
#define BES_FEM_APPLY_SHAPES(X)                                            \
  X(4, 3, 4, 4, true) X(10, 6, 4, 4, true) X(20, 10, 4, 4, true)           \
  X(35, 15, 4, 4, true)                                                    \
  X(4, 4, 3, 3, false) X(10, 10, 3, 3, false) X(20, 20, 3, 3, false)       \
  X(35, 35, 3, 3, false)
#endif

inline bool fem_apply_shape_listed(int ni, int nj, int nc, int nx, bool diag) {
#define BES_FEM_APPLY_MATCH(a, b, c, d, g) \
  if (ni == (a) && nj == (b) && nc == (c) && nx == (d) && diag == (g)) return true;
  BES_FEM_APPLY_SHAPES(BES_FEM_APPLY_MATCH)
#undef BES_FEM_APPLY_MATCH
  return false;
}
