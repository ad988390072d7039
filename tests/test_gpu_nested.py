"""Nested (third-layer) condensation on the GPU against the oracle: the block
systems A-hat^G, b-hat^G of every block, element by element, and the
skeleton solve built from the GPU's blocks against the oracle's direct solve
of the whole element-level system."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gpu_common import make_pair, to_dev, say

pytestmark = pytest.mark.gpu

CASES = {
    "2d_per_p2_M2": (dict(dim=2, n_elem=4, m=1, p=2, periodic=True), 2),
    "2d_dir_p1_M3": (dict(dim=2, n_elem=6, m=1, p=1, periodic=False, state="shear"), 3),
    "3d_per_p1_M2": (dict(dim=3, n_elem=4, m=1, p=1, periodic=True), 2),
    "3d_per_p2_M3": (dict(dim=3, n_elem=6, m=1, p=2, periodic=True), 3),
}


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


@pytest.mark.parametrize("name", list(CASES))
def test_nested_blocks_match_oracle(name):
    import torch
    from oracle import nested
    from paper_2402_11361_amd.hdg import HDG_FP64
    case, M = CASES[name]
    say(f"[nested] {name}: oracle element system")
    S, inp, ctx = make_pair(case)
    lin = S.linearize(inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"])
    cond = S.condense(lin, "B")
    B = nested.Blocks(S.mesh, M)
    nc = nested.condense(B, cond)
    say(f"[nested] {name}: GPU linearise, condense, nested condense")
    d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat, HDG_FP64)
    nb, nI, nB = ctx.nested_dims(M)
    assert nb == B.n_blocks and nI == B.face_dofs(B.internal[0]).size and nB == B.face_dofs(B.boundary[0]).size
    if case["dim"] == 3 and case["p"] == 2 and M == 3:
        assert nI == nested.internal_trace_dofs(3, 3, 2) == 2430
    Ag = torch.zeros(nb * nB * nB, dtype=torch.float64, device="cuda")
    bg = torch.zeros(nb * nB, dtype=torch.float64, device="cuda")
    ctx.condense_nested(M, Ag, bg)
    Ag = Ag.cpu().numpy().reshape(nb, nB, nB)
    bg = bg.cpu().numpy().reshape(nb, nB)
    ea = max(_rel(Ag[g], nc[g]["Ahat"]) for g in range(nb))
    eb = max(_rel(bg[g], nc[g]["bhat"]) for g in range(nb))
    say(f"[nested] {name}: {nb} blocks, n_I {nI}, n_B {nB}: A-hat^G {ea:.2e}, b-hat^G {eb:.2e}")
    assert ea < 1e-10 and eb < 1e-10
    # the skeleton system from the GPU's blocks solves the element system
    gpu_blocks = [dict(Ahat=Ag[g], bhat=bg[g]) for g in range(nb)]
    As, bs = nested.assemble(B, gpu_blocks)
    xs = spla.splu(As.tocsc()).solve(bs)
    A, b = S.assemble(cond)
    x_ref = S.solve_direct(A, b)
    skel = np.concatenate([S.mesh.face_offset[f] + np.arange(S.mesh.face_ndof[f]) for f in B.skeleton])
    assert _rel(xs, x_ref[skel]) < 1e-9
    # the skeleton solve and the recovery of the internal traces on the GPU
    x = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    info = ctx.nested_solve(M, x, rtol=1e-13, restart=30, max_outer=400, inner_its=5)
    ex = _rel(x.cpu().numpy(), x_ref)
    dq = torch.zeros(ctx.n_q_tot, dtype=torch.float64, device="cuda")
    du = torch.zeros(ctx.n_u_tot, dtype=torch.float64, device="cuda")
    ctx.local_backsolve(x, dq, du)
    dq_o, du_o = S.backsolve(lin, cond, x_ref)
    eu, eq = _rel(du.cpu().numpy(), du_o), _rel(dq.cpu().numpy(), dq_o)
    say(f"[nested] {name}: skeleton FGMRES {info['outer_its']} outer / {info['inner_its']} inner, "
        f"traces {ex:.2e}, dU {eu:.2e}, dQ {eq:.2e}")
    assert info["converged"] and ex < 1e-10 and eu < 1e-10 and eq < 1e-10
    # a second call with the same block size reuses the plan
    ctx.condense_nested(M, torch.zeros(nb * nB * nB, dtype=torch.float64, device="cuda"),
                        torch.zeros(nb * nB, dtype=torch.float64, device="cuda"))
    ctx.close()


def test_nested_needs_condensation_and_a_fitting_mesh():
    import torch
    from paper_2402_11361_amd.hdg import HdgError, HDG_FP64
    S, inp, ctx = make_pair(dict(dim=2, n_elem=4, m=1, p=1, periodic=True))
    nb, nI, nB = ctx.nested_dims(2)
    Ag = torch.zeros(nb * nB * nB, dtype=torch.float64, device="cuda")
    bg = torch.zeros(nb * nB, dtype=torch.float64, device="cuda")
    with pytest.raises(HdgError, match="EINVAL"):
        ctx.condense_nested(2, Ag, bg)  # no condensation yet
    with pytest.raises(HdgError, match="EINVAL"):
        ctx.nested_solve(2, torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda"))  # no nested condensation
    with pytest.raises(HdgError, match="EINVAL"):
        ctx.nested_dims(3)  # 4 elements per axis
    d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    ctx.condense(torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda"), HDG_FP64)
    ctx.condense_nested(2, Ag, bg)
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    with pytest.raises(HdgError, match="EINVAL"):
        ctx.condense_nested(2, Ag, bg)  # the linearisation changed the element blocks
    ctx.close()
    S2, _, ctx2 = make_pair(dict(dim=2, n_elem=4, m=2, p=1, periodic=True))
    with pytest.raises(HdgError, match="EUNSUPPORTED"):
        ctx2.nested_dims(1)  # macros of two elements per axis
    ctx2.close()


def test_dirk_step_through_the_nested_path_matches_oracle():
    """One DIRK(3,3) step whose Newton steps all go through the nested path
    (element condensation, block condensation, skeleton FGMRES, internal
    traces, element recovery) against the oracle's time step, which solves
    the element system directly: the nested path is an exact reformulation."""
    from oracle.newton import dirk_step
    from paper_2402_11361_amd.driver import StageDriver
    case = dict(dim=2, n_elem=4, m=1, p=2, periodic=True, mach=0.1, Re=100.0)
    say(f"[nested driver] {case}")
    S, inp, ctx = make_pair(case)
    drv = StageDriver(ctx, rtol=1e-13, newton_abs=1e-12, newton_rel=1e-12, max_newton=12, nested_block=2)
    q, u, uh = to_dev(inp["q"]), to_dev(inp["u"]), to_dev(inp["uh"])
    infos = drv.step(q, u, uh, inp["dt"])
    qo, uo, uho, _ = dirk_step(S, inp["q"], inp["u"], inp["uh"], inp["dt"],
                               newton_kw=dict(abs_tol=1e-12, rel_tol=1e-12, max_it=12))
    for st in infos:
        assert st["res_hist"][-1] < 1e-11, st["res_hist"]
    du = _rel(u.cpu().numpy(), uo)
    duh = _rel(uh.cpu().numpy(), uho)
    say(f"[nested driver] u {du:.2e}, u-hat {duh:.2e}")
    assert du < 1e-10 and duh < 1e-10
    assert np.abs(uo - inp["u"]).max() > 1e-6
    ctx.close()
