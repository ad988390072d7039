"""Degree-of-freedom counts of the macro-element HDG spaces (Sec. 2.2 spaces;
Tables 1, 3, 7, 8, 10).  Test infrastructure (oracle).

Simplicial macros of m elements per edge at degree p carry C0 P_p nodes of the
m-refined simplex: n_simplex(mp) = C(mp + d, d); each macro face carries C0 P_p
trace nodes of the m-refined triangle: C(mp + d - 1, d - 1).  The local
unknowns are u and q: ns (1 + d) values per node.
"""
from math import comb


def simplex_counts(n_macros, n_faces, m, p, d=3):
    ns = d + 2
    per_macro = comb(m * p + d, d) * ns * (1 + d)
    per_face = comb(m * p + d - 1, d - 1) * ns
    return n_macros * per_macro, n_faces * per_face, per_macro


def refined_cube_faces(level):
    """Faces of the cube split into 12 tetrahedra and refined `level` times
    (each tet into 8, each boundary triangle into 4): interior I and boundary
    Bd faces satisfy 2 I + Bd = 4 N_tets."""
    n_tets = 12 * 8 ** level
    bd = 12 * 4 ** level
    return n_tets, (4 * n_tets + bd) // 2


def box_counts(mesh):
    """(local total, global, local per macro) for a box-macro mesh: u and q at
    the prod(m_k p + 1) C0 nodes, traces at the C0 nodes of each macro face."""
    ns = mesh.dim + 2
    loc = [mesh.macro_n_nodes(i) * ns * (1 + mesh.dim) for i in range(mesh.n_macros)]
    return sum(loc), mesh.n_glob, loc
