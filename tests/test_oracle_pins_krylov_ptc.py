"""Pins of the oracle's Krylov solvers, face-block preconditioner and
pseudo-transient continuation against definitions computed another way:
  * GMRES (Sec. 4.2, inner solver): the iterate minimises the preconditioned
    residual over the Krylov space, computed here from an explicit Krylov
    matrix, a Householder QR and a dense least-squares solve;
  * FGMRES (Sec. 4.2, outer solver): one cycle minimises the true residual
    over x0 + P K_k(A P, r0), computed the same way;
  * the preconditioner (Sec. 4.2): A_uhat-uhat of the assembled full system
    (eq. C312) is block diagonal by face, and the oracle's preconditioner is
    the inverse of that block diagonal;
  * PTC with SER (Sec. 3.1, eq. C31222, ratio as in the survey's reading):
    the continuation adds M / dtau to A_uu only, reaches the same steady
    state as plain Newton, and its dtau sequence telescopes to
    tau_init ||R_U^0|| / ||R_U^m|| below the cap."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import krylov, newton, couette
from oracle.discretization import mass_matrix
from oracle.mesh import box_mesh
from oracle.physics import Phys
from oracle.system import System
from cases import small_case


def _krylov_basis(op, r0, k):
    K = np.zeros((r0.size, k))
    K[:, 0] = r0
    for j in range(1, k):
        K[:, j] = op(K[:, j - 1])
    Q, _ = np.linalg.qr(K)          # Householder; independent of the Arnoldi process
    return Q


def _random_system(n=60, seed=0):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    Mi = np.diag(1.0 / (1.0 + rng.random(n)))
    return A, Mi, rng.standard_normal(n)


@pytest.mark.parametrize("steps", [1, 3, 6])
def test_gmres_left_fixed_is_the_krylov_minimiser(steps):
    A, Mi, v = _random_system()
    z = krylov.gmres_left_fixed(lambda x: A @ x, lambda x: Mi @ x, v, steps)
    r0 = Mi @ v
    Q = _krylov_basis(lambda x: Mi @ (A @ x), r0, steps)
    y = np.linalg.lstsq(Mi @ A @ Q, r0, rcond=None)[0]
    zr = Q @ y
    assert np.linalg.norm(z - zr) < 1e-11 * np.linalg.norm(zr)
    # a right-preconditioned minimiser would be a different vector
    Qr = _krylov_basis(lambda x: A @ (Mi @ x), v, steps)
    zr_right = Mi @ Qr @ np.linalg.lstsq(A @ Mi @ Qr, v, rcond=None)[0]
    assert np.linalg.norm(z - zr_right) > 1e-6 * np.linalg.norm(zr)


@pytest.mark.parametrize("k", [2, 5])
def test_fgmres_cycle_is_the_true_residual_minimiser(k):
    A, Mi, b = _random_system(seed=1)
    x0 = np.random.default_rng(2).standard_normal(b.size) * 0.1
    P = lambda v: Mi @ v
    x, info = krylov.fgmres(lambda v: A @ v, b, x0=x0, precond=P, restart=k, rtol=1e-300, max_outer=k)
    assert info["its"] == k
    r0 = b - A @ x0
    Q = _krylov_basis(lambda v: A @ (Mi @ v), r0, k)
    Zb = Mi @ Q
    xr = x0 + Zb @ np.linalg.lstsq(A @ Zb, r0, rcond=None)[0]
    assert np.linalg.norm(x - xr) < 1e-11 * np.linalg.norm(xr)
    assert abs(info["res"] - np.linalg.norm(b - A @ xr)) < 1e-10 * np.linalg.norm(b)


def _assembled_Abb(S, lin):
    """A_uhat-uhat of the full system, assembled by scattering each macro's
    trace rows and columns through its global trace indices."""
    n = S.mesh.n_glob
    A = np.zeros((n, n))
    for i, L in lin.items():
        idx = S.mesh.macro_trace_index(i)
        rr, cc = np.meshgrid(idx, idx, indexing="ij")
        np.add.at(A, (rr, cc), L["blk"]["A_bb"])   # repeated indices accumulate
    return A


@pytest.mark.parametrize("kw", [dict(dim=2, n_elem=4, m=2, p=2, periodic=True, supg=True),
                                dict(dim=2, n_elem=2, m=2, p=2, periodic=True),
                                dict(dim=2, n_elem=6, m=3, p=1, periodic=False, state="shear"),
                                dict(dim=3, n_elem=2, m=1, p=2, periodic=True)])
def test_face_block_preconditioner_inverts_block_diagonal_of_Abb(kw):
    S, q, u, uh, _ = small_case(**kw)
    lin = S.linearize(q, u, uh, w=-2.0 * u, dt=0.3, dii=2.0)
    A = _assembled_Abb(S, lin)
    m = S.mesh
    mask = np.zeros_like(A, dtype=bool)
    for f in range(m.n_faces):
        sl = slice(m.face_offset[f], m.face_offset[f] + m.face_ndof[f])
        mask[sl, sl] = True
    # each face's trace rows couple only that face's traces (both sides summed)
    assert np.abs(A[~mask]).max() == 0.0
    assert np.abs(A[mask]).max() > 0.0
    # both sides contribute: on an interior face the block is the sum of two
    # one-sided blocks, not either of them
    v = np.random.default_rng(7).standard_normal(m.n_glob)
    Minv = newton.face_block_precond(S, lin)
    z = Minv(v)
    ref = np.linalg.solve(A, v)     # A is block diagonal, so this is the block-diagonal inverse
    assert np.linalg.norm(z - ref) < 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(A @ z - v) < 1e-12 * np.linalg.norm(v) * np.linalg.cond(A)


def test_ptc_term_is_mass_over_dtau_on_A_uu_only():
    S, q, u, uh, _ = small_case(dim=2, n_elem=4, m=2, p=2, periodic=True)
    w = -2.0 * u
    l0 = S.linearize(q, u, uh, w=w, dt=0.3, dii=2.0, macros=[1])[1]
    dtau = 0.37
    l1 = S.linearize(q, u, uh, w=w, dt=0.3, dii=2.0, dtau=dtau, macros=[1])[1]
    mc = S.cls(1)
    for k in l0["blk"]:
        d = l1["blk"][k] - l0["blk"][k]
        if k != "A_uu":
            assert np.abs(d).max() == 0.0, k
    d = l1["blk"]["A_uu"] - l0["blk"]["A_uu"]
    # (phi_b, phi_a)/dtau per component: symmetric, component-diagonal, and
    # summing to the macro's area per component (sum_a phi_a = 1)
    assert np.allclose(d, d.T, atol=1e-15)
    area = np.prod([mc.m[k] * mc.h[k] for k in range(mc.dim)])
    for c in range(mc.ns):
        for c2 in range(mc.ns):
            blk = d[c * mc.N:(c + 1) * mc.N, c2 * mc.N:(c2 + 1) * mc.N]
            if c == c2:
                assert abs(blk.sum() * dtau - area) < 1e-12 * area
            else:
                assert np.abs(blk).max() == 0.0
    # residuals are unchanged (the continuation modifies only the Jacobian)
    for k in ("RQ", "RU", "RB"):
        assert np.array_equal(l0[k], l1[k])


@pytest.mark.slow
def test_ptc_ser_reaches_the_newton_solution_with_telescoping_dtau():
    ph = Phys(Re=1.0, Mach=0.15)
    M = box_mesh(2, 4, 2, 2)
    uD = np.concatenate([couette.exact_u(M.face_node_coords(f).T, ph).reshape(-1) for f in range(M.n_faces)])
    S = System(M, ph, source=lambda X: couette.source(X, ph), uD=uD)
    u = np.concatenate([couette.exact_u(M.macro_node_coords(i).T, ph).reshape(-1) for i in range(M.n_macros)])
    # a start far from the solution: density and energy perturbed by 5%
    rng = np.random.default_rng(11)
    u0 = u * (1.0 + 0.05 * rng.uniform(-1, 1, u.size))
    q0 = np.zeros(S.q_off[-1])
    ref = newton.newton_solve(S, q0, u0, uD.copy(), abs_tol=1e-12, rel_tol=1e-13)
    tau0 = 0.05
    out = newton.newton_solve(S, q0, u0, uD.copy(), ptc=True, tau_init=tau0, abs_tol=1e-12, rel_tol=1e-13,
                              max_it=40)
    assert out[3]["res_hist"][-1] < 1e-11
    assert np.abs(out[1] - ref[1]).max() < 1e-10 * np.abs(ref[1]).max()
    assert np.abs(out[2] - ref[2]).max() < 1e-10 * np.abs(ref[2]).max()
    # dtau_m = tau0 ||R_U^0|| / ||R_U^m|| (product of the SER ratios) below the cap
    qs, us, uhs = q0.copy(), u0.copy(), uD.copy()
    RU0 = np.linalg.norm(S.residual(qs, us, uhs)[1])
    dt = out[3]["dtau_hist"]
    assert dt[0] == tau0
    # rerun the iteration step by step to read ||R_U^m||
    hist = newton.newton_solve(S, q0, u0, uD.copy(), ptc=True, tau_init=tau0, abs_tol=0.0, rel_tol=0.0,
                               max_it=3)
    assert len(hist[3]["dtau_hist"]) == 3
    for m_ in range(1, 3):
        part = newton.newton_solve(S, q0, u0, uD.copy(), ptc=True, tau_init=tau0, abs_tol=0.0, rel_tol=0.0,
                                   max_it=m_)
        RUm = np.linalg.norm(S.residual(part[0], part[1], part[2])[1])
        expect = min(tau0 * RU0 / RUm, 1e8)
        assert abs(hist[3]["dtau_hist"][m_] - expect) < 1e-12 * expect
    # the continuation takes more steps than plain Newton from this start and
    # the pseudo-time step grows as the residual falls
    assert len(dt) > ref[3]["its"]
    assert dt[-1] > 100 * dt[0]
