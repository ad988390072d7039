"""Pins of the oracle with a polynomial degree per macro (mixed degrees): the
trace on a face between degrees p+ and p- has degree max(p+, p-), which
contains both sides' traces.  Counts in closed form, the exact discrete
states of the uniform-degree mesh (free stream, linear fields), the
per-macro conservation identity, and the condensation routes against the
direct solve of the whole block system."""
import numpy as np
import pytest

from cases import small_case
from oracle.discretization import macro_residual, mass_matrix
from test_oracle_solvers import _full_system

# 2 x 2 macros of 2 x 2 elements (2D), 2 x 1 x 2 macros of one element (3D)
MIXED = {
    "2d_per": dict(dim=2, n_elem=4, m=2, p=2, periodic=True, macro_p=[1, 3, 2, 1]),
    "2d_per_supg": dict(dim=2, n_elem=4, m=2, p=2, periodic=True, supg=True, macro_p=[2, 1, 3, 2]),
    "2d_dir": dict(dim=2, n_elem=4, m=2, p=2, periodic=False, state="shear", macro_p=[3, 1, 1, 2]),
    "3d_per": dict(dim=3, seg=[[1, 1], [2], [1, 1]], p=1, periodic=True, macro_p=[1, 2, 2, 1]),
}


def _case(name, **kw):
    c = dict(MIXED[name])
    c.update(kw)
    return small_case(**c)


@pytest.mark.parametrize("name", list(MIXED))
def test_trace_degree_and_dof_counts(name):
    S, q, u, uh, _ = _case(name)
    M = S.mesh
    d, ns = M.dim, M.ns
    assert M.mixed
    n_glob = 0
    for f, fc in enumerate(M.faces):
        sides = [M.macro_deg(i) for i in (fc["minus"], fc["plus"]) if i >= 0]
        assert fc["deg"] == max(sides)
        tn = [int(M.seg_len[j][fc["grid"][j]]) * fc["deg"] + 1 for j in fc["tang"]]
        assert M.face_ndof[f] == ns * int(np.prod(tn))
        n_glob += M.face_ndof[f]
    assert M.n_glob == n_glob == uh.size
    for i in range(M.n_macros):
        mc = S.cls(i)
        assert mc.n_u == ns * int(np.prod([m * M.macro_deg(i) + 1 for m in M.macro_m(i)]))
        # the class's local faces carry exactly the mesh faces' trace nodes
        for lf in range(2 * d):
            f = M.macro_faces[i, lf]
            assert mc.face_deg[lf] == M.face_deg(f)
            assert ns * mc.nf_nodes[lf] == M.face_ndof[f]
            assert mc.Tf[lf] == (M.face_deg(f) + 1) ** (d - 1)
    assert S.u_off[-1] == u.size
    # a face between degrees 1 and 3 (2D periodic case): 2 sub-faces x 3 + 1 nodes
    if name == "2d_per":
        degs = sorted({fc["deg"] for fc in M.faces})
        assert degs == [2, 3]


@pytest.mark.parametrize("name", ["2d_per", "3d_per"])
def test_free_stream_preserved(name):
    """A uniform state with q = 0 and u-hat = u is an exact discrete steady
    state across faces of different trace degree: R_Q = R_U = R_Uhat = 0."""
    S, q, u, uh, _ = _case(name)
    M = S.mesh
    d = M.dim
    st = np.array([1.1, 0.05, -0.03, 0.02, 0.0][:d + 2])
    st[-1] = 1 / (1.4 * 0.4) + 0.5 * (st[1:d + 1] ** 2).sum() / st[0]
    u = np.concatenate([np.repeat(st, S.cls(i).N) for i in range(M.n_macros)])
    uh = np.concatenate([np.repeat(st, M.faces[f]["n_nodes"]) for f in range(M.n_faces)])
    q = np.zeros(S.q_off[-1])
    RQ, RU, RB = S.residual(q, u, uh)
    assert abs(RQ).max() < 1e-14 and abs(RU).max() < 1e-14 and abs(RB).max() < 1e-14
    dii = 2.0
    RQ, RU, RB = S.residual(q, u, uh, w=-dii * u, dt=0.3, dii=dii)
    assert abs(RQ).max() < 1e-14 and abs(RU).max() < 1e-14 and abs(RB).max() < 1e-14


@pytest.mark.parametrize("name", ["2d_dir", "3d_per"])
def test_gradient_equation_exact_for_linear_fields(name):
    """Eq. (C38a) reproduces q = grad u exactly for a linear field (in every
    degree's space) with u-hat its trace: R_Q = 0 also on the faces whose
    trace degree exceeds a side's degree."""
    S, q, u, uh, _ = _case(name, periodic=False, state="shear")
    M = S.mesh
    ns = M.dim + 2
    A = 0.1 * np.random.default_rng(3).standard_normal((ns, M.dim))
    c0 = np.array([1.0] + list(0.05 * np.random.default_rng(4).standard_normal(M.dim)) + [2.5])
    lin = lambda X: (c0[:, None] + A @ X.T)
    u = np.concatenate([lin(M.macro_node_coords(i)).reshape(-1) for i in range(M.n_macros)])
    uh = np.concatenate([lin(M.face_node_coords(f)).reshape(-1) for f in range(M.n_faces)])
    q = np.concatenate([np.repeat(A.T[:, :, None], S.cls(i).N, axis=2).reshape(-1) for i in range(M.n_macros)])
    RQ, RU, RB = S.residual(q, u, uh)
    assert abs(RQ).max() < 1e-13


@pytest.mark.parametrize("name", ["2d_per", "3d_per"])
def test_macro_conservation_identity(name):
    """sum_a R_U[c,a] - sum_j R_Uhat^(i)[c,j] = (time term, 1) per macro and
    component, also where the trace basis has a higher degree than the
    macro (it is still a partition of unity on the face)."""
    S, q, u, uh, _ = _case(name, noise=1e-2)
    dt, dii = 0.2, 2.3
    w = -dii * u * 0.97
    for i in range(S.mesh.n_macros):
        mc = S.cls(i)
        qi, ui, bi, wi = S.local(i, q, u, uh, w)
        assert mc.T > min(mc.Tf) or len(set(mc.face_deg)) == 1
        rq, ru, rb = macro_residual(mc, S.ph, qi[None], ui[None], bi[None], w=wi[None], dt=dt, dii=dii)
        sb = np.zeros(mc.ns)
        for lf in range(2 * mc.dim):
            off, nf = mc.nf_off[lf], mc.nf_nodes[lf]
            sb += rb[0, off:off + mc.ns * nf].reshape(mc.ns, nf).sum(axis=1)
        Mm = mass_matrix(mc)
        time = (Mm.sum(axis=0)[None, :] * (dii * ui + wi)).sum(axis=1) / dt
        assert np.allclose(ru[0].sum(axis=1) - sb, time, atol=1e-13)


@pytest.mark.parametrize("name", list(MIXED))
def test_condensation_routes_and_brute_force(name):
    """Route A (C47) == route B (ASC2) == direct solve of the full block system
    (C312) on a mixed-degree mesh; Algorithm 2 == the explicit A-hat^{T_i};
    the recovery Csc4 gives the full-system solution."""
    S, q, u, uh, uD = _case(name)
    w = -1.9 * u
    lin = S.linearize(q, u, uh, w=w, dt=0.3, dii=1.9)
    cB, cA = S.condense(lin, "B"), S.condense(lin, "A")
    for i in lin:
        sc = abs(cA[i]["Ahat"]).max()
        assert abs(cB[i]["Ahat"] - cA[i]["Ahat"]).max() < 1e-12 * sc
        assert abs(cB[i]["bhat"] - cA[i]["bhat"]).max() < 1e-12 * max(1.0, abs(cA[i]["bhat"]).max())
    A, b = S.assemble(cB)
    xr = np.random.default_rng(5).standard_normal(S.mesh.n_glob)
    assert abs(S.apply_alg2(lin, cB, xr) - A @ xr).max() < 1e-12 * abs(A @ xr).max()
    x = S.solve_direct(A, b)
    dq, du = S.backsolve(lin, cB, x)
    J, R = _full_system(S, lin)
    sol = np.linalg.solve(J, -R)
    nq, nu = S.q_off[-1], S.u_off[-1]
    ref = np.abs(sol).max()
    assert abs(sol[nq + nu:] - x).max() < 1e-10 * ref
    assert abs(sol[nq:nq + nu] - du).max() < 1e-10 * ref
    assert abs(sol[:nq] - dq).max() < 1e-10 * ref


@pytest.mark.parametrize("name", ["2d_per", "3d_per"])
def test_geometric_q_blocks(name):
    """A_qq, A_qu, A_q-uhat of eq. (C38a) from the mass, gradient and face
    matrices (faces of a higher trace degree included) equal the
    complex-step blocks of every macro."""
    S, q, u, uh, _ = _case(name)
    lin = S.linearize(q, u, uh, dt=0.5, dii=2.0)
    for i, L in lin.items():
        blk = L["blk"]
        Aqq, Aqu, Aqb = S.geo(S.mclass[i])["qblk"]
        assert abs(blk["A_qq"] - Aqq).max() < 1e-13
        assert abs(blk["A_qu"] - Aqu).max() < 1e-13
        assert abs(blk["A_qb"] - Aqb).max() < 1e-13


@pytest.mark.slow
def test_couette_convergence_on_mixed_degrees():
    """Steady Couette flow (Sec. 5.1) on a checkerboard of p = 2 and p = 3
    macros (m = 2), exact Dirichlet trace: v_1 converges at the rate of the
    lower degree, p_min + 1 = 3 (2.86, 2.95 on 4 -> 8 -> 16); rho and rho E at
    about p_min = 2 (2.08, 2.05), below the uniform p = 2 mesh's 2.8 on the
    same levels (measured: the same with a trace of the smaller degree on
    the mixed faces, so the face degree choice is not the cause)."""
    from oracle import newton, couette
    from oracle.mesh import box_mesh
    from oracle.physics import Phys
    from oracle.system import System
    ph = Phys(Re=1.0, Mach=0.15)
    errs = []
    for ne in (4, 8, 16):
        nseg = ne // 2
        mp = [(2, 3)[(a + b) % 2] for b in range(nseg) for a in range(nseg)]
        M = box_mesh(2, ne, 2, 3, macro_p=mp)
        uD = np.concatenate([couette.exact_u(M.face_node_coords(f).T, ph).reshape(-1) for f in range(M.n_faces)])
        S = System(M, ph, source=lambda X: couette.source(X, ph), uD=uD)
        u = np.concatenate([couette.exact_u(M.macro_node_coords(i).T, ph).reshape(-1) for i in range(M.n_macros)])
        q = np.concatenate([couette.exact_q(M.macro_node_coords(i).T, ph).reshape(-1) for i in range(M.n_macros)])
        q2, u2, uh2, info = newton.newton_solve(S, q, u, uD.copy(), abs_tol=1e-12, rel_tol=1e-13)
        assert info["res_hist"][-1] < 1e-11
        errs.append(couette.l2_errors(S, u2, ph))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])          # columns: rho, v_1, rho E
    assert rates[-1][1] > 3 - 0.2, rates
    assert np.all(rates[-1] > 2 - 0.15), rates
