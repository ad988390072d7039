"""Pins of the nested (third-layer) condensation of the oracle: the closed-form
count of the internal-face traces of a block, the skeleton size, the
reduction to the element system for one-element blocks, and the nested
solve against the direct solve of the whole element-level system (the
elimination is exact, so the two agree to rounding)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from cases import small_case
from oracle import nested
from oracle.mesh import box_mesh

DIRK_DII = 1.0 / 0.435866521508459


def _element_system(dim, n_elem, p, periodic, state="tgv", supg=False):
    S, q, u, uh, uD = small_case(dim=dim, n_elem=n_elem, m=1, p=p, periodic=periodic, state=state,
                                 supg=supg, noise=1e-2)
    dt = 0.1
    lin = S.linearize(q, u, uh, w=-DIRK_DII * u, dt=dt, dii=DIRK_DII)
    cond = S.condense(lin, "B")
    return S, lin, cond


def test_internal_trace_count_closed_form_and_counted():
    # 3^3 blocks of p = 2 hexes: 54 internal faces x 9 nodes x 5 components
    assert nested.internal_trace_dofs(3, 3, 2) == 2430
    for dim, n, M, p in [(3, 6, 3, 2), (2, 6, 3, 3), (2, 4, 2, 1)]:
        mesh = box_mesh(dim, n, 1, p, periodic=True)
        B = nested.Blocks(mesh, M)
        for g in range(B.n_blocks):
            nI = B.face_dofs(B.internal[g]).size
            assert nI == nested.internal_trace_dofs(dim, M, p)
            # each block face holds M^(d-1) element faces
            assert len(B.boundary[g]) == 2 * dim * M ** (dim - 1)
        # the skeleton is what the blocks do not eliminate
        assert B.n_skel == mesh.n_glob - sum(B.face_dofs(B.internal[g]).size for g in range(B.n_blocks))


@pytest.mark.parametrize("dim,n_elem,p,M,periodic,state", [
    (2, 4, 2, 2, True, "tgv"),
    (2, 6, 1, 3, False, "shear"),
    (3, 4, 1, 2, True, "tgv"),
])
def test_nested_solve_equals_direct_solve(dim, n_elem, p, M, periodic, state):
    S, lin, cond = _element_system(dim, n_elem, p, periodic, state)
    A, b = S.assemble(cond)
    x_ref = S.solve_direct(A, b)
    B = nested.Blocks(S.mesh, M)
    nc = nested.condense(B, cond)
    As, bs = nested.assemble(B, nc)
    xs = spla.splu(As.tocsc()).solve(bs)
    x = nested.recover_traces(B, nc, xs)
    assert np.abs(x - x_ref).max() / np.abs(x_ref).max() < 1e-10
    # and the element unknowns recovered from them
    dq, du = S.backsolve(lin, cond, x)
    dq_r, du_r = S.backsolve(lin, cond, x_ref)
    assert np.abs(du - du_r).max() / np.abs(du_r).max() < 1e-10


def test_one_element_blocks_are_the_element_system():
    S, lin, cond = _element_system(2, 4, 2, True)
    A, b = S.assemble(cond)
    B = nested.Blocks(S.mesh, 1)
    assert B.n_skel == S.mesh.n_glob and all(len(f) == 0 for f in B.internal)
    nc = nested.condense(B, cond)
    As, bs = nested.assemble(B, nc)
    # skeleton order = global face order when nothing is eliminated
    assert np.abs((As - A).toarray()).max() <= 1e-12 * np.abs(A.toarray()).max()
    assert np.abs(bs - b).max() <= 1e-12 * np.abs(b).max()


def test_block_schur_complement_is_the_global_elimination():
    """A-hat^G of one block equals eliminating that block's internal traces
    from the globally assembled system (rows and columns of its boundary
    faces, with only this block's elements assembled)."""
    S, lin, cond = _element_system(2, 4, 2, True)
    B = nested.Blocks(S.mesh, 2)
    g = 1
    A, b, nI = B.local_system(cond, g)
    nc = nested.condense(B, cond)[g]
    # dense elimination by Gauss-Jordan on the assembled block system
    n = A.shape[0]
    Aug = np.concatenate([A, b[:, None]], axis=1)
    for j in range(nI):
        piv = j + int(np.argmax(np.abs(Aug[j:nI, j])))
        Aug[[j, piv]] = Aug[[piv, j]]
        Aug[j] /= Aug[j, j]
        for r in range(n):
            if r != j:
                Aug[r] -= Aug[r, j] * Aug[j]
    assert np.abs(Aug[nI:, nI:n] - nc["Ahat"]).max() <= 1e-10 * np.abs(nc["Ahat"]).max()
    assert np.abs(Aug[nI:, n] - nc["bhat"]).max() <= 1e-10 * np.abs(nc["bhat"]).max()
