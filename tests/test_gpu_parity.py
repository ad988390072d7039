"""Parity of every hot-path stage of the HIP library against the CPU oracle
(called through the C ABI).  Element-by-element comparisons at FP64
rounding level; the solve is compared at stagnation tolerance."""
import math

import numpy as np
import pytest

from gpu_common import make_pair, to_dev, say, gpu_available

pytestmark = pytest.mark.gpu

CASES = {
    "2d_per_p2": dict(dim=2, n_elem=4, m=2, p=2, periodic=True),
    "2d_dir_p1": dict(dim=2, n_elem=6, m=3, p=1, periodic=False, state="shear", mach=0.2),
    "2d_dir_p3": dict(dim=2, n_elem=4, m=2, p=3, periodic=False, state="shear", mach=0.2),
    "C1_2d_16x16_m4_p2": dict(dim=2, n_elem=16, m=4, p=2, periodic=False, state="shear", mach=0.2, Re=100.0),
    "3d_per_p2": dict(dim=3, n_elem=4, m=2, p=2, periodic=True),
    "3d_dir_p1": dict(dim=3, n_elem=4, m=2, p=1, periodic=False, state="shear", mach=0.2),
    "3d_per_p3": dict(dim=3, n_elem=2, m=1, p=3, periodic=True),
    "3d_dir_p3_2x1x1": dict(dim=3, seg=[[2], [1, 1], [1, 1]], p=3, periodic=False, state="shear", mach=0.2),
    # SUPG on (frozen A_k and tau; strong residual in group form)
    "2d_dir_p2_supg": dict(dim=2, n_elem=6, m=3, p=2, periodic=False, state="shear", mach=0.2, supg=True),
    "2d_per_p3_supg": dict(dim=2, n_elem=4, m=2, p=3, periodic=True, supg=True),
    "3d_per_p2_supg": dict(dim=3, n_elem=4, m=2, p=2, periodic=True, supg=True),
    "3d_per_p3_supg": dict(dim=3, n_elem=2, m=1, p=3, periodic=True, supg=True),
    # macros of different sizes in one mesh (several classes in one launch)
    "2d_dir_uneven_p2": dict(dim=2, seg=[[2, 3], [3, 2]], p=2, periodic=False, state="shear", mach=0.2),
    "3d_per_uneven_p2": dict(dim=3, seg=[[2, 3], [3, 2], [2, 2]], p=2, periodic=True),
    # one class too large for the grouped formation beside seven small ones
    "3d_per_uneven_p2_split_form": dict(dim=3, seg=[[4, 1], [4, 1], [2, 1]], p=2, periodic=True),
    "3d_dir_uneven_p1_supg": dict(dim=3, seg=[[1, 2], [2, 1], [2, 2]], p=1, periodic=False, state="shear",
                                  mach=0.2, supg=True),
    # degenerate meshes: one periodic macro (each face is its own neighbour),
    # standard HDG with one element per macro at p = 1
    "2d_per_single_macro_p2": dict(dim=2, n_elem=2, m=2, p=2, periodic=True),
    "3d_per_m1_p1": dict(dim=3, n_elem=2, m=1, p=1, periodic=True),
}


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _close(a, b, tol, what):
    r = _rel(a, b)
    assert r < tol, f"{what}: rel err {r:.3e} >= {tol:.0e}"


@pytest.fixture(scope="module")
def pairs():
    return {}


def _get(pairs, name):
    if name not in pairs:
        say(f"[setup] {name}")
        case = dict(CASES[name])
        supg = case.pop("supg", False)
        S, inp, ctx = make_pair(case, supg=supg)
        d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
        nrm = ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
        macros = list(range(S.mesh.n_macros)) if S.mesh.n_macros <= 16 else [0, 5, S.mesh.n_macros - 1]
        lin = S.linearize(inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"], macros=macros)
        cond = S.condense(lin, "B")
        pairs[name] = (S, inp, ctx, d, nrm, lin, cond)
    return pairs[name]


@pytest.mark.parametrize("name", list(CASES))
def test_residuals(pairs, name):
    S, inp, ctx, d, nrm, lin, cond = _get(pairs, name)
    say(f"[residuals] {name}")
    RQ, RU, RB = S.residual(inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"])
    rq, ru, rb = (t.cpu().numpy() for t in ctx.get_residuals())
    # residual entries are sums of O(h^d) terms that cancel down to the size of
    # the noise in the state: compare at 1e-10 of the result (about 1e-13 of
    # the individual terms)
    _close(rq, RQ, 1e-10, "R_Q")
    _close(ru, RU, 1e-10, "R_U")
    _close(rb, RB, 1e-10, "R_Uhat")
    assert np.allclose(nrm, [np.linalg.norm(RQ), np.linalg.norm(RU), np.linalg.norm(RB)], rtol=1e-10)


@pytest.mark.parametrize("name", list(CASES))
def test_formed_blocks(pairs, name):
    """[[S, -C, f], [D, E, g]] of eq. ASC2 against the oracle's dense algebra."""
    S, inp, ctx, d, nrm, lin, cond = _get(pairs, name)
    say(f"[formed] {name}")
    for i in lin:
        blk = lin[i]["blk"]
        Qi = S.geo(S.mclass[i])["Qi"]
        c = cond[i]
        nu = S.cls(i).n_u
        W = ctx.get_formed(i)
        E = blk["A_bb"] - blk["A_bq"] @ Qi @ blk["A_qb"]
        g = -lin[i]["RB"] + blk["A_bq"] @ Qi @ lin[i]["RQ"]
        ref_top = np.hstack([c["S"], -c["right"], c["f"][:, None]])
        ref_bot = np.hstack([c["left"], E, g[:, None]])
        scale = np.abs(ref_top).max()
        e1 = np.abs(W[:nu] - ref_top).max() / scale
        e2 = np.abs(W[nu:] - ref_bot).max() / max(scale, np.abs(ref_bot).max())
        assert e1 < 1e-12 and e2 < 1e-12, f"macro {i}: top {e1:.3e} bottom {e2:.3e}"


@pytest.mark.parametrize("name", list(CASES))
def test_condensed_and_apply_and_solve(pairs, name):
    S, inp, ctx, d, nrm, lin, cond = _get(pairs, name)
    import torch
    say(f"[condense] {name}")
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat)
    for i in lin:
        A_i, b_i = ctx.get_condensed(i)
        _close(A_i, cond[i]["Ahat"], 1e-10, f"Ahat macro {i}")
        _close(b_i, cond[i]["bhat"], 1e-10, f"bhat macro {i}")
    if len(lin) < S.mesh.n_macros:
        return  # global checks need every macro in the oracle
    A, b = S.assemble(cond)
    _close(bhat.cpu().numpy(), b, 1e-10, "assembled bhat")
    say(f"[apply] {name}")
    x = np.random.default_rng(7).standard_normal(ctx.n_glob)
    y = torch.zeros_like(bhat)
    ctx.apply_global(to_dev(x), y)
    _close(y.cpu().numpy(), A @ x, 1e-12, "A-hat x")
    say(f"[fgmres] {name}")
    x_ref = S.solve_direct(A, b)
    xg = torch.zeros_like(bhat)
    # run to rtol 1e-13 (near stagnation): the error is bounded by
    # kappa(A-hat) * 1e-13 plus the rounding of the operator, well inside 1e-10
    # for these small condensed systems
    info = ctx.fgmres_solve(bhat, xg, rtol=1e-13, restart=30, max_outer=400, inner_its=5)
    assert info["converged"], info
    _close(xg.cpu().numpy(), x_ref, 1e-10, "FGMRES solution")
    say(f"[backsolve] {name}")
    dq = torch.zeros(ctx.n_q_tot, dtype=torch.float64, device="cuda")
    du = torch.zeros(ctx.n_u_tot, dtype=torch.float64, device="cuda")
    ctx.local_backsolve(to_dev(x_ref), dq, du)
    dq_o, du_o = S.backsolve(lin, cond, x_ref)
    _close(du.cpu().numpy(), du_o, 1e-10, "dU")
    _close(dq.cpu().numpy(), dq_o, 1e-10, "dQ")


def _assembled(pairs, name):
    import torch
    S, inp, ctx, d, nrm, lin, cond = _get(pairs, name)
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat)
    A, b = S.assemble(cond)
    return S, ctx, lin, A, b, bhat


@pytest.mark.parametrize("name", list(CASES))
def test_precond_apply_matches_oracle(pairs, name):
    """The preconditioner of Sec. 4.2 element by element: the inverse face
    blocks of A_uhat-uhat alone (inner_its = 0), and inner GMRES with 5 steps
    left-preconditioned by them, against the oracle's face_block_precond and
    gmres_left_fixed on the assembled A-hat."""
    import torch
    from oracle import krylov, newton
    S, ctx, lin, A, b, bhat = _assembled(pairs, name)
    say(f"[precond] {name}")
    v = np.random.default_rng(21).standard_normal(ctx.n_glob)
    Minv = newton.face_block_precond(S, lin)
    z = torch.zeros_like(bhat)
    ctx.precond_apply(to_dev(v), z, 0)
    _close(z.cpu().numpy(), Minv(v), 1e-11, "face-block inverse")
    ctx.precond_apply(to_dev(v), z, 5)
    ref = krylov.gmres_left_fixed(lambda x: A @ x, Minv, v, 5)
    _close(z.cpu().numpy(), ref, 1e-9, "inner GMRES(5)")


@pytest.mark.parametrize("name", list(CASES))
def test_outer_iterations_match_oracle(pairs, name):
    """Outer FGMRES iterations to rtol 1e-8 on the same A-hat and b-hat with the
    same multi-level preconditioner: the library and the oracle's fgmres agree
    to one iteration."""
    import torch
    from oracle import krylov, newton
    S, ctx, lin, A, b, bhat = _assembled(pairs, name)
    say(f"[iterations] {name}")
    Minv = newton.face_block_precond(S, lin)
    P = lambda v: krylov.gmres_left_fixed(lambda x: A @ x, Minv, v, 5)
    xo, io = krylov.fgmres(lambda v: A @ v, b, precond=P, restart=30, rtol=1e-8, max_outer=400)
    xg = torch.zeros_like(bhat)
    ig = ctx.fgmres_solve(bhat, xg, rtol=1e-8, restart=30, max_outer=400, inner_its=5)
    say(f"[iterations] {name}: library {ig['outer_its']}, oracle {io['its']}")
    assert io["converged"] and ig["converged"]
    assert abs(ig["outer_its"] - io["its"]) <= 1, (ig["outer_its"], io["its"])


@pytest.mark.parametrize("name", ["3d_per_p2", "3d_per_uneven_p2", "2d_dir_p3"])
def test_apply_is_bitwise_repeatable(pairs, name):
    """The global apply sums each face's contributions in a fixed order: the
    same x gives the same bits on every call, also after applies to other
    vectors in between."""
    import torch
    S, ctx, lin, A, b, bhat = _assembled(pairs, name)
    say(f"[repeat] {name}")
    x = to_dev(np.random.default_rng(31).standard_normal(ctx.n_glob))
    x2 = to_dev(np.random.default_rng(32).standard_normal(ctx.n_glob))
    y1, y2, y3 = (torch.zeros_like(bhat) for _ in range(3))
    ctx.apply_global(x, y1)
    ctx.apply_global(x2, y3)
    ctx.apply_global(x, y2)
    assert torch.equal(y1, y2)
    assert not torch.equal(y1, y3)
