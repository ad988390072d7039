"""Pins of the oracle's reference element, time integrator and DOF counting
against closed forms and the paper's tables."""
import numpy as np
import pytest
from oracle.basis import gll_nodes, gauss_rule, lagrange
from oracle import dirk, counts
from oracle.mesh import box_mesh


def test_gll_closed_forms():
    assert np.allclose(gll_nodes(1), [-1, 1])
    assert np.allclose(gll_nodes(2), [-1, 0, 1])
    assert np.allclose(gll_nodes(3), [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1])
    r = np.sqrt(3.0 / 7.0)
    assert np.allclose(gll_nodes(4), [-1, -r, 0, r, 1])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_exactness(n):
    x, w = gauss_rule(n)
    for deg in range(2 * n):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(w @ x ** deg - exact) < 1e-14
    # and fails at degree 2n (not exact)
    assert abs(w @ x ** (2 * n) - 2.0 / (2 * n + 1)) > 1e-6


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lagrange_properties(p):
    g = gll_nodes(p)
    xs = np.linspace(-1, 1, 13)
    V, D = lagrange(g, xs)
    assert np.allclose(V.sum(axis=1), 1.0)          # partition of unity
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-12)
    Vn, _ = lagrange(g, g)
    assert np.allclose(Vn, np.eye(p + 1))           # cardinality
    # derivative of the interpolant of x^p is p x^(p-1)
    assert np.allclose(D @ g ** p, p * xs ** (p - 1))


def test_p1_mass_matrix():
    from oracle.discretization import MacroClass, mass_matrix
    h = 0.3
    mc = MacroClass(2, [1, 1], 1, [h, 1.0])
    M = mass_matrix(mc)
    M1 = h / 6 * np.array([[2, 1], [1, 2]])
    assert np.allclose(M, np.kron(1.0 / 6 * np.array([[2, 1], [1, 2]]), M1))


def test_dirk33_order_conditions():
    A, b, c = dirk.dirk33()
    a = A[0, 0]
    assert abs(6 * a ** 3 - 18 * a ** 2 + 9 * a - 1) < 1e-14
    assert abs(a - 0.435866521508459) < 1e-12
    assert abs(b.sum() - 1) < 1e-14
    assert abs(b @ c - 0.5) < 1e-14
    assert abs(b @ c ** 2 - 1 / 3) < 1e-14
    assert abs(b @ (A @ c) - 1 / 6) < 1e-14
    assert abs(c[-1] - 1) < 1e-15 and np.allclose(A[-1], b)   # stiffly accurate


def test_dirk33_third_order_on_linear_ode():
    """Stage equations in the form of eq. (C242) for y' = lam y, update (C241)."""
    lam = -1.3
    A, b, c = dirk.dirk33()
    Ai = np.linalg.inv(A)
    errs = []
    for nsteps in (10, 20, 40):
        dt = 1.0 / nsteps
        y = np.array([1.0])
        for _ in range(nsteps):
            st = []
            for i in range(3):
                # (d_ii y_i + w)/dt = lam y_i,  w = stage_history
                w = dirk.stage_history(Ai, i, y, st)
                yi = -w / (Ai[i, i] - lam * dt)
                st.append(yi)
            y = dirk.update(Ai, b, y, st)
        errs.append(abs(y[0] - np.exp(lam)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.85), rates


def test_paper_dof_tables_simplicial():
    # Table 1: 768 tets, p = 3, m = 1, 2, 4 (12, 96, 768 macros = refinement levels 0, 1, 2)
    expect = {1: (307200, 81600, 400), 2: (161280, 30240, 1680), 4: (109200, 13650, 9100)}
    for m, lev in ((1, 2), (2, 1), (4, 0)):
        n_macros, n_faces = counts.refined_cube_faces(lev)
        assert counts.simplex_counts(n_macros, n_faces, m, 3) == expect[m]
    # Table 3 (12 macros, refinement level 0), (m,p) with mp = 8
    for m, p in ((2, 4), (4, 2), (8, 1)):
        assert counts.simplex_counts(12, 30, m, p) == (39600, 6750, 3300)
    # Tables 8 and 10: periodic Taylor-Green meshes, every face shared: 2 N faces
    for n, loc, glob in ((1592, 5253600, 716400), (10143, 33471900, 4564350),
                         (495, 1633500, 222750), (955, 3151500, 429750)):
        assert counts.simplex_counts(n, 2 * n, 4, 2)[:2] == (loc, glob)
    # Table 7: sphere, local dofs for m = 1 (139,272 tets) and m = 2 (17,409 macros)
    assert counts.simplex_counts(139272, 0, 1, 3)[0] == 55708800
    assert counts.simplex_counts(17409, 0, 2, 3)[0] == 29247120
    assert counts.simplex_counts(0, 35800, 2, 3)[1] == 5012000


def test_box_mesh_counts():
    m2 = box_mesh(2, 16, 4, 2)
    assert (m2.n_macros, m2.n_faces, m2.n_glob) == (16, 40, 1440)
    m3 = box_mesh(3, 24, 3, 2, periodic=True)
    tot, glob, loc = counts.box_counts(m3)
    assert (m3.n_macros, m3.n_faces, glob) == (512, 1536, 376320)
    assert loc[0] == 343 * 5 * 4
