"""Pins of the oracle's residuals (eq. C38), Jacobian blocks (eq. C312) and
their invariants."""
import numpy as np
import pytest
from oracle.discretization import macro_residual, macro_jacobian, split_blocks
from cases import small_case


@pytest.mark.parametrize("dim,supg", [(2, False), (2, True), (3, True)])
def test_free_stream_preservation(dim, supg):
    """A uniform state with q = 0 and u-hat = u is an exact discrete steady
    state on a periodic box: R_Q = R_U = 0 and the summed trace residual is 0."""
    S, q, u, uh, _ = small_case(dim=dim, n_elem=4, m=2, p=2, supg=supg)
    ns = dim + 2
    st = np.array([1.1, 0.05, -0.03, 0.02, 0.0][:ns])
    st[-1] = 1 / (1.4 * 0.4) + 0.5 * (st[1:dim + 1] ** 2).sum() / st[0]
    u = np.tile(np.repeat(st, S.cls(0).N), S.mesh.n_macros)
    uh = np.concatenate([np.repeat(st, S.mesh.faces[f]["n_nodes"]) for f in range(S.mesh.n_faces)])
    q = np.zeros(S.q_off[-1])
    dii = 2.0
    RQ, RU, RB = S.residual(q, u, uh, w=-dii * u, dt=0.3, dii=dii)
    assert abs(RQ).max() < 1e-14 and abs(RU).max() < 1e-14 and abs(RB).max() < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_equation_exact_for_linear_fields(dim):
    """Eq. (C38a) reproduces q = grad u exactly for a linear field with
    u-hat equal to the trace of u: R_Q = 0."""
    S, q, u, uh, _ = small_case(dim=dim, n_elem=4, m=2, p=2, periodic=False, state="shear")
    M = S.mesh
    ns = dim + 2
    # a physical linear state (rho > 0 and pressure > 0 on the unit box)
    A = 0.1 * np.random.default_rng(3).standard_normal((ns, dim))
    c0 = np.array([1.0] + list(0.05 * np.random.default_rng(4).standard_normal(dim)) + [2.5])
    lin = lambda X: (c0[:, None] + A @ X.T)
    u = np.concatenate([lin(M.macro_node_coords(i)).reshape(-1) for i in range(M.n_macros)])
    uh = np.concatenate([lin(M.face_node_coords(f)).reshape(-1) for f in range(M.n_faces)])
    q = np.concatenate([np.repeat(A.T[:, :, None], S.cls(i).N, axis=2).reshape(-1) for i in range(M.n_macros)])
    RQ, RU, RB = S.residual(q, u, uh)
    assert abs(RQ).max() < 1e-13
    assert np.all(np.isfinite(RU)) and np.all(np.isfinite(RB))


@pytest.mark.parametrize("supg", [False, True])
def test_macro_conservation_identity(supg):
    """sum_a R_U[c,a] - sum_j R_Uhat^(i)[c,j] = (time term, 1) for every macro and
    component: the volume and SUPG terms vanish against sum_a phi_a = 1 and the
    face fluxes cancel because sum_a phi_a = sum_j mu_j = 1 on the boundary."""
    S, q, u, uh, _ = small_case(dim=2, n_elem=4, m=2, p=2, supg=supg, noise=1e-2)
    dt, dii = 0.2, 2.3
    w = -dii * u * 0.97
    for i in range(S.mesh.n_macros):
        mc = S.cls(i)
        qi, ui, bi, wi = S.local(i, q, u, uh, w)
        rq, ru, rb = macro_residual(mc, S.ph, qi[None], ui[None], bi[None], w=wi[None], dt=dt, dii=dii, supg=supg)
        sb = np.zeros(mc.ns)
        for lf in range(2 * mc.dim):
            off, nf = mc.nf_off[lf], mc.nf_nodes[lf]
            sb += rb[0, off:off + mc.ns * nf].reshape(mc.ns, nf).sum(axis=1)
        from oracle.discretization import mass_matrix
        Mm = mass_matrix(mc)
        time = (Mm.sum(axis=0)[None, :] * (dii * ui + wi)).sum(axis=1) / dt
        assert np.allclose(ru[0].sum(axis=1) - sb, time, atol=1e-13)


def test_complex_step_matches_finite_differences():
    S, q, u, uh, _ = small_case(dim=2, n_elem=4, m=2, p=2, supg=True, noise=1e-2)
    i = 3
    mc = S.cls(i)
    qi, ui, bi, _ = S.local(i, q, u, uh, None)
    kw = dict(dt=0.25, dii=1.7, supg=True, w=(-1.7 * ui)[None])
    J, _ = macro_jacobian(mc, S.ph, qi[None], ui[None], bi[None], **kw)
    x0 = np.concatenate([qi.reshape(-1), ui.reshape(-1), bi])
    rng = np.random.default_rng(0)

    def R(x):
        rq, ru, rb = macro_residual(mc, S.ph, x[:mc.n_q].reshape(1, mc.dim, mc.ns, mc.N),
                                    x[mc.n_q:mc.n_q + mc.n_u].reshape(1, mc.ns, mc.N),
                                    x[None, mc.n_q + mc.n_u:], **kw)
        return np.concatenate([rq.reshape(-1), ru.reshape(-1), rb.reshape(-1)])

    # frozen coefficients (lambda_max, SUPG A and tau) depend on u and u-hat only;
    # the residual is linear in q, so FD in q directions agrees to rounding.
    dirs = rng.standard_normal((3, x0.size))
    dirs[:, mc.n_q:] = 0.0
    errs = []
    for eps in (1e-4, 5e-5):
        e = max(np.abs((R(x0 + eps * v) - R(x0 - eps * v)) / (2 * eps) - J[0] @ v).max() for v in dirs)
        errs.append(e)
    assert max(errs) < 1e-8


def test_complex_step_all_columns_with_frozen_coefficients():
    """With SUPG off and u-hat = trace of u on every face (so lambda_max enters
    only multiplied by u - u-hat = 0), the frozen Jacobian is the exact one:
    central FD agrees to O(eps^2) in every column."""
    S, q, u, uh, _ = small_case(dim=2, n_elem=4, m=2, p=2, supg=False, noise=0.0)
    i = 0
    mc = S.cls(i)
    qi, ui, bi, _ = S.local(i, q, u, uh, None)
    kw = dict(dt=0.25, dii=1.7, w=(-1.5 * ui)[None])
    J, _ = macro_jacobian(mc, S.ph, qi[None], ui[None], bi[None], **kw)
    x0 = np.concatenate([qi.reshape(-1), ui.reshape(-1), bi])

    def R(x):
        rq, ru, rb = macro_residual(mc, S.ph, x[:mc.n_q].reshape(1, mc.dim, mc.ns, mc.N),
                                    x[mc.n_q:mc.n_q + mc.n_u].reshape(1, mc.ns, mc.N),
                                    x[None, mc.n_q + mc.n_u:], **kw)
        return np.concatenate([rq.reshape(-1), ru.reshape(-1), rb.reshape(-1)])

    rng = np.random.default_rng(1)
    for v in rng.standard_normal((3, x0.size)):
        v[mc.n_q:] *= 1e-3      # keep u - u-hat tiny so lambda_max variation is O(eps * 1e-3)
        eps = 1e-5
        fd = (R(x0 + eps * v) - R(x0 - eps * v)) / (2 * eps)
        assert np.abs(fd - J[0] @ v).max() < 1e-7


def test_geometric_q_blocks():
    """A_qq, A_qu, A_q-uhat are state independent (eq. C38a is linear):
    I (x) M, I (x) B_k and -(I (x) E_k), with A_{q_k q_k} = M (the paper's
    diag(J) M for the affine box)."""
    S, q, u, uh, _ = small_case(dim=3, n_elem=2, m=1, p=2, periodic=True, supg=False)
    lin = S.linearize(q, u, uh, dt=0.5, dii=2.0, macros=[0])
    blk = lin[0]["blk"]
    Aqq, Aqu, Aqb = S.geo(S.mclass[0])["qblk"]
    assert abs(blk["A_qq"] - Aqq).max() < 1e-13
    assert abs(blk["A_qu"] - Aqu).max() < 1e-13
    assert abs(blk["A_qb"] - Aqb).max() < 1e-13
