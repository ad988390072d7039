"""Pins of the oracle's condensation (eq. C47 vs AP12/ASC2), Algorithm 2, the
Krylov solvers, the local recovery (Csc4) and the Couette convergence rates."""
import numpy as np
import pytest
from oracle import krylov, newton, couette
from oracle.mesh import box_mesh
from oracle.physics import Phys
from oracle.system import System
from cases import small_case


def _full_system(S, lin):
    nq, nu, ng = S.q_off[-1], S.u_off[-1], S.mesh.n_glob
    n = nq + nu + ng
    J = np.zeros((n, n)); R = np.zeros(n)
    for i, L in lin.items():
        qi = np.arange(S.q_off[i], S.q_off[i + 1])
        ui = nq + np.arange(S.u_off[i], S.u_off[i + 1])
        bi = nq + nu + S.mesh.macro_trace_index(i)
        idx = dict(q=qi, u=ui, b=bi)
        for r in "qub":
            for c in "qub":
                # np.add.at: a macro can see one face from both sides (a single
                # periodic macro), so trace indices repeat and must accumulate
                rr, cc = np.meshgrid(idx[r], idx[c], indexing="ij")
                np.add.at(J, (rr, cc), L["blk"][f"A_{r}{c}"])
        R[qi] += L["RQ"]; R[ui] += L["RU"]; np.add.at(R, bi, L["RB"])
    return J, R


CASES = [dict(dim=2, n_elem=4, m=2, p=2, periodic=True, supg=True),
         # one periodic macro: each of its faces is its own neighbour
         dict(dim=2, n_elem=2, m=2, p=2, periodic=True),
         # standard HDG (one element per macro) at p = 1
         dict(dim=3, n_elem=2, m=1, p=1, periodic=True),
         dict(dim=2, n_elem=6, m=[3, 2], p=1, periodic=False, state="shear", supg=True),
         dict(dim=3, n_elem=2, m=1, p=2, periodic=True, supg=False)]


@pytest.mark.parametrize("kw", CASES)
def test_condensation_routes_and_brute_force(kw):
    """Route A (C47) == route B (ASC2) == direct solve of the full block system
    (C312); Algorithm 2 == the explicit A-hat^{T_i}; the recovery Csc4 gives the
    full-system solution."""
    kw = dict(kw)
    m = kw.pop("m")
    if isinstance(m, list):
        S, q, u, uh, uD = small_case(seg=[[m[0]] * 2, [m[1]] * 3], **{k: v for k, v in kw.items() if k != "n_elem"})
    else:
        S, q, u, uh, uD = small_case(m=m, **kw)
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
    dqa, dua = S.backsolve(lin, cA, x)
    J, R = _full_system(S, lin)
    sol = np.linalg.solve(J, -R)
    nq, nu = S.q_off[-1], S.u_off[-1]
    ref = np.abs(sol).max()
    assert abs(sol[nq + nu:] - x).max() < 1e-10 * ref
    assert abs(sol[nq:nq + nu] - du).max() < 1e-10 * ref
    assert abs(sol[:nq] - dq).max() < 1e-10 * ref
    assert abs(dua - du).max() < 1e-10 * ref
    res = J @ np.concatenate([dq, du, x]) + R
    assert np.linalg.norm(res) < 1e-12 * np.linalg.norm(R)


def test_fgmres_matches_direct_and_sc_equals_sl_iterations():
    S, q, u, uh, uD = small_case(dim=2, n_elem=8, m=2, p=2, supg=True)
    lin = S.linearize(q, u, uh, w=-2.0 * u, dt=0.2, dii=2.0)
    cB, cA = S.condense(lin, "B"), S.condense(lin, "A")
    A, b = S.assemble(cB)
    Aa, ba = S.assemble(cA)
    x_ref = S.solve_direct(A, b)
    Minv = newton.face_block_precond(S, lin)
    infos = []
    for AA, bb in ((A, b), (Aa, ba)):
        Aop = lambda v, AA=AA: AA @ v
        P = lambda v, Aop=Aop: krylov.gmres_left_fixed(Aop, Minv, v, 5)
        x, info = krylov.fgmres(Aop, bb, precond=P, restart=30, rtol=1e-13)
        assert info["converged"]
        assert np.linalg.norm(x - x_ref) < 1e-9 * np.linalg.norm(x_ref)
        infos.append(info["its"])
    # second-layer and standard condensation give the same operator: same iterations
    assert infos[0] == infos[1]
    # an exact preconditioner makes FGMRES converge in one iteration
    import scipy.sparse.linalg as spla
    lu = spla.splu(A.tocsc())
    x, info = krylov.fgmres(lambda v: A @ v, b, precond=lu.solve, rtol=1e-12)
    assert info["its"] == 1 and info["converged"]


def test_couette_source_x1_momentum_matches_printed_entry():
    ph = Phys(Re=1.0, Mach=0.15)
    x2 = np.linspace(0, 1, 7)
    X = np.stack([0.3 + 0 * x2, x2])
    s = couette.source(X, ph)
    expect = -(ph.mu * ph.Mach / ph.Re_c) * (2 + x2) / (1 + x2) ** 2
    assert np.allclose(s[1], expect, rtol=1e-12, atol=1e-15)
    assert np.allclose(s[0], 0, atol=1e-15) and np.allclose(s[2], 0, atol=1e-15)


COUETTE_LEVELS = {1: (8, 16, 32), 2: (8, 16, 32), 3: (4, 8, 16), 4: (4, 8, 16), 5: (4, 8, 16)}
# how far below p + 1 the energy (and every variable) may stay on the finest pair
COUETTE_SLACK = {1: (0.45, 0.5), 2: (0.2, 0.5), 3: (0.45, 0.5), 4: (0.45, 0.5), 5: (0.7, 0.7)}


@pytest.mark.slow
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_couette_optimal_convergence(p):
    """Steady Couette flow with the exact Dirichlet trace, m = 2 (Sec. 5.1):
    L2 errors of v_1 converge at the optimal rate p + 1 at every degree
    (finest pair 1.92 / 2.93 / 3.91 / 4.86 / 5.86 at p = 1 to 5).  The energy
    rho E reaches p + 1 at p = 2 (2.97) and approaches it from below at p = 1
    (1.58, 1.61 on these pairs; 1.63 on 32 -> 64), p = 3 (3.60, 3.59) and
    p = 4 (4.39, 4.66); at p = 5 it stays at 5.35-5.37 (errors near 1e-12 on
    the finest mesh).  rho alone (a purely convected variable) stays between
    p + 1/2 and p + 1 up to p = 4 (5.37 at p = 5).  The paper reads p + 1
    for velocity and energy off plots on tetrahedra (p = 1 to 5); the bounds
    below are what this discretisation reaches on these meshes.  The
    library's kernels stop at p = 3; the oracle takes any degree."""
    ph = Phys(Re=1.0, Mach=0.15)
    errs = []
    for ne in COUETTE_LEVELS[p]:
        M = box_mesh(2, ne, 2, p)
        uD = np.concatenate([couette.exact_u(M.face_node_coords(f).T, ph).reshape(-1) for f in range(M.n_faces)])
        S = System(M, ph, source=lambda X: couette.source(X, ph), uD=uD)
        u = np.concatenate([couette.exact_u(M.macro_node_coords(i).T, ph).reshape(-1) for i in range(M.n_macros)])
        q = np.concatenate([couette.exact_q(M.macro_node_coords(i).T, ph).reshape(-1) for i in range(M.n_macros)])
        q2, u2, uh2, info = newton.newton_solve(S, q, u, uD.copy(), abs_tol=1e-12, rel_tol=1e-13)
        assert info["res_hist"][-1] < 1e-11
        errs.append(couette.l2_errors(S, u2, ph))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])          # columns: rho, v_1, rho E
    assert rates[-1][1] > p + 1 - 0.2, rates
    assert rates[-1][2] > p + 1 - COUETTE_SLACK[p][0], rates
    assert np.all(rates[-1] > p + 1 - COUETTE_SLACK[p][1]), rates
    assert rates[-1][2] >= rates[0][2] - 0.05, rates


def test_newton_quadratic_convergence():
    """Steady Couette Newton iterations with the complex-step Jacobian converge
    quadratically (Sec. 3.1)."""
    ph = Phys(Re=1.0, Mach=0.15)
    M = box_mesh(2, 4, 2, 2)
    uD = np.concatenate([couette.exact_u(M.face_node_coords(f).T, ph).reshape(-1) for f in range(M.n_faces)])
    S = System(M, ph, source=lambda X: couette.source(X, ph), uD=uD)
    u = np.concatenate([couette.exact_u(M.macro_node_coords(i).T, ph).reshape(-1) for i in range(M.n_macros)])
    q = np.zeros(S.q_off[-1])
    _, _, _, info = newton.newton_solve(S, q, u, uD.copy(), abs_tol=1e-13, rel_tol=1e-14, linear="fgmres",
                                        krylov_opts=dict(rtol=1e-13))
    h = info["res_hist"]
    assert h[-1] < 1e-12
    assert h[2] < 10 * h[1] ** 2 / h[0] + 1e-13


def test_dirk_step_conserves_mass_momentum_energy():
    """On a periodic box the HDG scheme is conservative: the trace equation
    makes the two one-sided face fluxes cancel, the volume and SUPG terms
    vanish against sum_a phi_a = 1, so each stage conserves the integral of
    every conserved variable (Sec. 2.3; checked across a full DIRK step)."""
    from oracle.newton import dirk_step
    from oracle.discretization import mass_matrix
    S, q, u, uh, uD = small_case(dim=2, n_elem=4, m=2, p=2, periodic=True, supg=True, noise=1e-2)
    mc = S.cls(0)
    wts = mass_matrix(mc).sum(axis=0)

    def totals(uu):
        return sum((uu[S.u_off[i]:S.u_off[i + 1]].reshape(mc.ns, mc.N) * wts).sum(axis=1)
                   for i in range(S.mesh.n_macros))

    t0 = totals(u)
    q1, u1, uh1, infos = dirk_step(S, q, u, uh, 0.4, newton_kw=dict(abs_tol=1e-13, rel_tol=1e-13, max_it=15))
    t1 = totals(u1)
    assert np.abs(u1 - u).max() > 1e-5           # the state moved
    assert np.allclose(t1, t0, rtol=0, atol=1e-11), (t0, t1)
