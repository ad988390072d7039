"""Pins of the oracle's trace residual R_Uhat (eq. C38c): face conservation
and the boundary operator.
  * A linear state with u-hat equal to the trace of u and q its exact
    gradient is continuous across every interior face, so the two one-sided
    normal fluxes cancel node by node and the summed R_Uhat vanishes there,
    while each side alone does not (a wrong normal sign or a one-sided term
    breaks this).
  * Summed over the trace basis (sum_j mu_j = 1), the trace residual of a
    macro side equals the normal-flux integral that also enters the macro's
    own residual: for every macro and component, sum_a R_U[c, a] minus the
    summed trace residual of its sides is the time term (the volume and SUPG
    terms vanish against sum_a phi_a = 1).  Over a periodic mesh the summed
    R_Uhat then equals the summed R_U minus the time terms, so a trace
    residual that loses or doubles a side's flux fails.
  * On a full-state Dirichlet face (survey reading A9) R_Uhat = M_f (u-hat -
    u_D) per component, with the face mass matrix M_f rebuilt here from GLL
    Lagrange polynomials and a high-order Gauss rule."""
import numpy as np
import pytest
from numpy.polynomial import legendre as L

from oracle.discretization import macro_residual, mass_matrix
from cases import small_case


def _gll(p):
    inner = L.legroots(L.legder([0] * p + [1])) if p > 1 else np.array([])
    return np.concatenate([[-1.0], np.sort(inner), [1.0]])


def _lagrange_1d_mass(p, m, h):
    """Mass matrix of the C0 degree-p Lagrange basis on GLL nodes over m
    elements of length h (one tangential direction of a macro face)."""
    x = _gll(p)
    g, w = L.leggauss(2 * p + 4)
    V = np.zeros((g.size, p + 1))
    for a in range(p + 1):
        others = [x[b] for b in range(p + 1) if b != a]
        V[:, a] = np.prod([(g - xb) / (x[a] - xb) for xb in others], axis=0) if others else 1.0
    Me = (V * (w * h / 2)[:, None]).T @ V
    n = m * p + 1
    M = np.zeros((n, n))
    for e in range(m):
        M[e * p:e * p + p + 1, e * p:e * p + p + 1] += Me
    return M


def _linear_state(S, dim):
    rng = np.random.default_rng(3)
    ns = dim + 2
    c0 = np.array([1.0] + [0.05] * dim + [2.5])
    A = 0.1 * rng.standard_normal((ns, dim))
    f = lambda X: c0[:, None] + A @ X.T
    M = S.mesh
    u = np.concatenate([f(M.macro_node_coords(i)).reshape(-1) for i in range(M.n_macros)])
    uh = np.concatenate([f(M.face_node_coords(fc)).reshape(-1) for fc in range(M.n_faces)])
    q = np.concatenate([np.repeat(A.T[:, :, None], S.cls(i).N, axis=2).reshape(-1) for i in range(M.n_macros)])
    return q, u, uh


@pytest.mark.parametrize("dim,p,supg", [(2, 2, False), (2, 3, True), (3, 1, True)])
def test_interior_faces_conserve_for_a_continuous_linear_state(dim, p, supg):
    S, _, _, _, _ = small_case(dim=dim, n_elem=4 if dim == 2 else 2, m=2 if dim == 2 else 1, p=p,
                               periodic=False, state="shear", mach=0.2, supg=supg)
    q, u, uh = _linear_state(S, dim)
    RQ, RU, RB = S.residual(q, u, uh)
    assert np.all(np.isfinite(RU))
    M = S.mesh
    one_sided = np.zeros(M.n_glob)
    for i in range(M.n_macros):
        qi, ui, bi, _ = S.local(i, q, u, uh, None)
        _, _, rb = macro_residual(S.cls(i), S.ph, qi[None], ui[None], bi[None], **S._kw(i, None, np.inf, 1.0))
        idx = M.macro_trace_index(i)
        # one side of each face only: the minus side
        for lf in range(2 * dim):
            f = M.macro_faces[i, lf]
            if M.faces[f]["minus"] == i and not M.face_is_boundary(f):
                off = sum(M.face_ndof[M.macro_faces[i, l]] for l in range(lf))
                one_sided[M.face_offset[f]:M.face_offset[f] + M.face_ndof[f]] = rb[0, off:off + M.face_ndof[f]]
    interior = np.concatenate([M.face_offset[f] + np.arange(M.face_ndof[f])
                               for f in range(M.n_faces) if not M.face_is_boundary(f)])
    scale = np.abs(one_sided[interior]).max()
    assert scale > 1e-3
    assert np.abs(RB[interior]).max() < 1e-13 * max(scale, 1.0)


@pytest.mark.parametrize("supg", [False, True])
def test_summed_trace_residual_balances_summed_macro_residual(supg):
    S, q, u, uh, _ = small_case(dim=2, n_elem=6, m=3, p=2, periodic=True, supg=supg, noise=2e-2)
    dt, dii = 0.25, 2.1
    w = -dii * u * 0.95
    RQ, RU, RB = S.residual(q, u, uh, w=w, dt=dt, dii=dii)
    ns = S.mesh.ns
    sum_u = np.zeros(ns)
    time = np.zeros(ns)
    for i in range(S.mesh.n_macros):
        mc = S.cls(i)
        sum_u += RU[S.u_off[i]:S.u_off[i + 1]].reshape(ns, mc.N).sum(axis=1)
        wts = mass_matrix(mc).sum(axis=0)
        ui = u[S.u_off[i]:S.u_off[i + 1]].reshape(ns, mc.N)
        wi = w[S.u_off[i]:S.u_off[i + 1]].reshape(ns, mc.N)
        time += (wts[None, :] * (dii * ui + wi)).sum(axis=1) / dt
    sum_b = np.zeros(ns)
    for f in range(S.mesh.n_faces):
        nn = S.mesh.faces[f]["n_nodes"]
        sum_b += RB[S.mesh.face_offset[f]:S.mesh.face_offset[f] + ns * nn].reshape(ns, nn).sum(axis=1)
    # the trace residual is not zero for this noisy state: the balance is not trivial
    assert np.abs(sum_b).max() > 1e-6
    assert np.allclose(sum_u - sum_b, time, rtol=0, atol=1e-12 * max(1.0, np.abs(time).max()))


@pytest.mark.parametrize("dim,p,m", [(2, 2, 2), (2, 3, 3), (3, 2, 1)])
def test_dirichlet_face_rows_are_face_mass_times_jump(dim, p, m):
    S, q, u, uh, uD = small_case(dim=dim, n_elem=2 * m, m=m, p=p, periodic=False, state="shear", mach=0.2,
                                 noise=1e-2)
    RQ, RU, RB = S.residual(q, u, uh)
    M = S.mesh
    ns = M.ns
    checked = 0
    for f in range(M.n_faces):
        if not M.face_is_boundary(f):
            continue
        fc = M.faces[f]
        mass = np.ones((1, 1))
        for j, t in enumerate(fc["tang"]):
            mt = M.seg_len[t][fc["grid"][t]]
            mass = np.kron(_lagrange_1d_mass(p, mt, M.h[t]), mass)   # first tangential axis fastest
        sl = slice(M.face_offset[f], M.face_offset[f] + M.face_ndof[f])
        jump = (uh[sl] - uD[sl]).reshape(ns, -1)
        ref = (mass @ jump.T).T.reshape(-1)
        assert np.abs(RB[sl] - ref).max() < 1e-13 * max(1.0, np.abs(ref).max()), f
        checked += 1
    assert checked > 0
