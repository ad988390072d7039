"""Pins of the oracle's learned coarse correction (coarse restriction and
prolongation, network, loss gradients, Adam) against closed forms, exact
reproduction properties and finite differences."""
import math

import numpy as np
import pytest

from oracle import learned as Ld
from oracle.mesh import box_mesh


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gll_weights_integrate_monomials(p):
    from oracle.basis import gll_nodes
    x = gll_nodes(p)
    w = Ld.gll_weights(p)
    for k in range(2 * p):  # exact up to degree 2p - 1
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-13


def test_composite_weights():
    pos, wt = Ld.composite_1d(3, 2)
    assert pos[0] == 0.0 and abs(pos[-1] - 1.0) < 1e-15
    assert abs(wt.sum() - 1.0) < 1e-14
    # integral of s^3 over [0, 1] (degree 3 = 2p - 1: exact)
    assert abs(np.sum(wt * pos ** 3) - 0.25) < 1e-14


def _face_param(mesh, f):
    fc = mesh.faces[f]
    tn_m = [(n - 1) // mesh.p for n in fc["tn"]]
    return [Ld.composite_1d(m, mesh.p)[0] for m in tn_m]


def test_restriction_of_s_squared_is_its_best_linear_fit():
    # on [0, 1] the L2-best linear approximation of s^2 is s - 1/6: nodal
    # values -1/6 at s = 0 and 5/6 at s = 1 (the GLL rule is exact for the
    # degree-3 integrands at p = 2)
    M = box_mesh(2, 4, 2, 2, periodic=True)
    v = np.zeros(M.n_glob)
    for f in range(M.n_faces):
        (s,) = _face_param(M, f)
        nn = len(s)
        for c in range(M.ns):
            v[M.face_offset[f] + c * nn:M.face_offset[f] + (c + 1) * nn] = (c + 1) * s ** 2
    X = Ld.coarse_restrict(M, v)
    nq = 2
    for i in range(M.n_macros):
        for lf in range(4):
            for c in range(M.ns):
                coef = X[i, (lf * M.ns + c) * nq:(lf * M.ns + c + 1) * nq]
                assert np.allclose(coef, (c + 1) * np.array([-1.0 / 6.0, 5.0 / 6.0]), atol=1e-13)


@pytest.mark.parametrize("dim,n,m,p,per", [(2, 6, 3, 2, False), (3, 4, 2, 2, True), (3, 4, 2, 1, False)])
def test_multilinear_fields_are_reproduced(dim, n, m, p, per):
    """R_c reproduces the corner values of a multilinear face field and
    P_c R_c is the identity on such fields."""
    M = box_mesh(dim, n, m, p, periodic=per)
    rng = np.random.default_rng(3)
    corners = rng.standard_normal((M.n_faces, M.ns, 2 ** (dim - 1)))
    v = np.zeros(M.n_glob)
    for f in range(M.n_faces):
        par = _face_param(M, f)
        if dim == 2:
            s = par[0]
            basis = np.stack([1 - s, s], axis=1)
        else:
            s, t = par
            S, T = np.tile(s, len(t)), np.repeat(t, len(s))
            basis = np.stack([(1 - S) * (1 - T), S * (1 - T), (1 - S) * T, S * T], axis=1)
        nn = basis.shape[0]
        for c in range(M.ns):
            v[M.face_offset[f] + c * nn:M.face_offset[f] + (c + 1) * nn] = basis @ corners[f, c]
    X = Ld.coarse_restrict(M, v)
    nq = 2 ** (dim - 1)
    for i in range(M.n_macros):
        for lf in range(2 * dim):
            f = M.macro_faces[i, lf]
            got = X[i, lf * M.ns * nq:(lf + 1) * M.ns * nq].reshape(M.ns, nq)
            assert np.allclose(got, corners[f], atol=1e-12)
    assert np.allclose(Ld.coarse_prolong(M, X), v, atol=1e-12)


def test_forward_hand_example_and_homogeneity():
    P = dict(W1=np.array([[1.0, 0.0]]), b1=np.array([0.0]), W2=np.array([[2.0]]), b2=np.array([0.5]))
    X = np.array([[3.0, 4.0]])
    tanh06 = 0.5370495669980353  # tanh(0.6)
    assert abs(Ld.forward(P, X)[0, 0] - 5.0 * (2.0 * tanh06 + 0.5)) < 1e-14
    rng = np.random.default_rng(0)
    Q = Ld.init_params(6, 8, 5, rng)
    Q["b1"] = rng.standard_normal(8)
    Q["b2"] = rng.standard_normal(5)
    Xr = rng.standard_normal((4, 6))
    assert np.allclose(Ld.forward(Q, 3.5 * Xr), 3.5 * Ld.forward(Q, Xr), rtol=1e-13, atol=0)
    assert np.all(Ld.forward(Q, np.zeros((2, 6))) == 0.0)


def test_loss_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    n_in, n_h, n_out = 7, 9, 5
    P = Ld.init_params(n_in, n_h, n_out, rng)
    P["b1"] = 0.1 * rng.standard_normal(n_h)
    P["b2"] = 0.1 * rng.standard_normal(n_out)
    X = rng.standard_normal((6, n_in))
    T = rng.standard_normal((6, n_out))
    loss, G = Ld.loss_and_grads(P, X, T)
    g = Ld.flat(G)
    v = Ld.flat(P)
    h = 1e-6
    for j in rng.choice(v.size, 40, replace=False):
        vp, vm = v.copy(), v.copy()
        vp[j] += h
        vm[j] -= h
        lp, _ = Ld.loss_and_grads(Ld.unflat(vp, n_in, n_h, n_out), X, T)
        lm, _ = Ld.loss_and_grads(Ld.unflat(vm, n_in, n_h, n_out), X, T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[j]) <= 1e-7 * max(1.0, abs(g[j])), (j, fd, g[j])


def test_loss_is_zero_on_own_output():
    rng = np.random.default_rng(2)
    P = Ld.init_params(4, 6, 3, rng)
    X = rng.standard_normal((5, 4))
    loss, G = Ld.loss_and_grads(P, X, Ld.forward(P, X))
    assert loss < 1e-28
    assert np.abs(Ld.flat(G)).max() < 1e-14


def test_adam_first_step_is_signed_lr():
    P = dict(W1=np.array([[1.0, -2.0]]), b1=np.array([0.5]), W2=np.array([[3.0]]), b2=np.array([0.0]))
    G = dict(W1=np.array([[0.3, -4.0]]), b1=np.array([-0.01]), W2=np.array([[2.0]]), b2=np.array([1e-3]))
    M = {k: np.zeros_like(v) for k, v in P.items()}
    V = {k: np.zeros_like(v) for k, v in P.items()}
    P0 = {k: v.copy() for k, v in P.items()}
    lr, eps = 1e-3, 1e-8
    Ld.adam_step(P, G, M, V, 1, lr=lr, eps=eps)
    for k in P:
        expect = P0[k] - lr * G[k] / (np.abs(G[k]) + eps)
        assert np.allclose(P[k], expect, rtol=0, atol=1e-15)


def test_zero_rows_carry_no_loss_gradient_of_the_input_layer():
    """A row with x = 0 is normalised to x~ = 0, t~ = 0: it adds (b-term)^2 to
    the loss and nothing to the gradient of W1."""
    rng = np.random.default_rng(6)
    P = Ld.init_params(3, 4, 2, rng)
    X = np.zeros((1, 3))
    T = rng.standard_normal((1, 2))
    P["b2"] = np.array([0.5, -1.0])
    loss, G = Ld.loss_and_grads(P, X, T)
    h0 = np.tanh(P["b1"])
    y0 = P["W2"] @ h0 + P["b2"]
    assert abs(loss - np.mean(y0 ** 2)) < 1e-15
    assert np.all(G["W1"] == 0.0)


def test_neighbour_features_hand_example_and_shared_faces():
    """2 x 3 macros, periodic in x only: the blocks are the right macros'
    coefficients (checked against macro indices by hand), zero across the
    Dirichlet walls, and the coefficients of a shared face agree from both
    sides (the same face field restricted twice)."""
    mesh = box_mesh(2, [4, 6], [2, 2], 2, periodic=[True, False])
    assert mesh.n_macros == 6
    F = Ld.n_features(2)
    X = np.arange(mesh.n_macros * F, dtype=float).reshape(mesh.n_macros, F) + 1.0
    Xe = Ld.neighbour_features(mesh, X)
    assert Xe.shape == (6, 5 * F)
    # macro (s0, s1) = s0 + 2 s1; local faces (x-low, x-high, y-low, y-high)
    expect = {0: [1, 1, -1, 2], 1: [0, 0, -1, 3], 2: [3, 3, 0, 4], 5: [4, 4, 3, -1]}
    for i, nbs in expect.items():
        assert np.array_equal(Xe[i, :F], X[i])
        for lf, j in enumerate(nbs):
            blk = Xe[i, (1 + lf) * F:(2 + lf) * F]
            assert np.array_equal(blk, X[j] if j >= 0 else np.zeros(F)), (i, lf)
    # a smooth field: both sides restrict a shared face to the same coefficients
    rng = np.random.default_rng(3)
    v = rng.standard_normal(mesh.n_glob)
    Xr = Ld.coarse_restrict(mesh, v)
    Xe = Ld.neighbour_features(mesh, Xr)
    ns, nq = mesh.ns, 2
    for i in range(mesh.n_macros):
        for lf in range(4):
            j = Ld.neighbour_of(mesh, i, lf)
            if j < 0:
                continue
            opp = lf ^ 1
            own = Xr[i, lf * ns * nq:(lf + 1) * ns * nq]
            theirs = Xe[i, (1 + lf) * F + opp * ns * nq:(1 + lf) * F + (opp + 1) * ns * nq]
            assert np.array_equal(own, theirs)
