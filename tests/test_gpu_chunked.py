"""Chunked condensation (macros formed and eliminated in consecutive ranges
through one buffer, condensed blocks kept compact, S re-factored range by
range in the recovery) against the CPU oracle and the unchunked path."""
import numpy as np
import pytest

from gpu_common import make_pair, to_dev, say

pytestmark = pytest.mark.gpu

# (mesh, macros per chunk, chunk slots of W, factor store (macros, precision) or None)
CASES = {
    # 8 macros in chunks of 2, 3, 3 (the first chunk takes the remainder)
    "3d_per_p2_chunk3": (dict(dim=3, n_elem=4, m=2, p=2, periodic=True), 3, 1, None),
    # 4 macro shapes; chunks of 2 hold macros of different classes
    "3d_per_uneven_p2_chunk2": (dict(dim=3, seg=[[2, 3], [3, 2], [2, 2]], p=2, periodic=True), 2, 1, None),
    # boundary faces; single-macro chunks
    "2d_dir_p3_chunk1": (dict(dim=2, n_elem=4, m=2, p=3, periodic=False, state="shear", mach=0.2), 1, 1, None),
    # two slots: chunk j + 1 formed beside the elimination of chunk j; the
    # recovery starts from the last two chunks and forms the other two again
    "3d_per_p2_chunk2_2slots": (dict(dim=3, n_elem=4, m=2, p=2, periodic=True), 2, 2, None),
    # two slots, several classes per chunk, chunks of 2, 3, 3 in slots 0, 1, 0
    # (the recovery forms the first chunk again)
    "3d_per_uneven_p2_chunk3_2slots": (dict(dim=3, seg=[[2, 3], [3, 2], [2, 3]], p=2, periodic=True), 3, 2, None),
    # factor store: chunks 0 and 1 from FP32 copies of their factors, chunk 2
    # formed again, chunk 3 from W
    "3d_per_p2_chunk2_store32": (dict(dim=3, n_elem=4, m=2, p=2, periodic=True), 2, 1, (4, "fp32")),
    # FP64 store of chunks 0 to 2 over several classes, chunk 3 from W
    "3d_per_uneven_p2_chunk2_store64": (dict(dim=3, seg=[[2, 3], [3, 2], [2, 2]], p=2, periodic=True), 2, 1,
                                        (8, "fp64")),
    # two slots and a store: chunk 0 stored, chunk 1 formed again, 2 and 3 from W
    "2d_dir_p3_chunk1_2slots_store32": (dict(dim=2, n_elem=4, m=2, p=3, periodic=False, state="shear", mach=0.2), 1, 2,
                                        (1, "fp32")),
}
STORED = {"3d_per_p2_chunk2_store32": 4, "3d_per_uneven_p2_chunk2_store64": 6, "2d_dir_p3_chunk1_2slots_store32": 1}

TOL32 = 5e-4


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def pairs():
    return {}


def _get(pairs, name):
    if name not in pairs:
        from paper_2402_11361_amd.hdg import HDG_FP32, HDG_FP64
        case, per, slots, store = CASES[name]
        say(f"[chunked setup] {name}")
        S, inp, ctx = make_pair(case)
        ctx.set_chunking(per)
        ctx.set_chunk_buffers(slots)
        if store:
            kept = ctx.set_factor_store(store[0], HDG_FP32 if store[1] == "fp32" else HDG_FP64)
            assert kept == STORED[name], kept
        ctx.bind_workspace()
        d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
        ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
        lin = S.linearize(inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"])
        cond = S.condense(lin, "B")
        pairs[name] = (S, inp, ctx, d, lin, cond)
    return pairs[name]


@pytest.mark.parametrize("name", list(CASES))
def test_chunked_fp64_matches_oracle(pairs, name):
    import torch
    S, inp, ctx, d, lin, cond = _get(pairs, name)
    say(f"[chunked fp64] {name}")
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat)
    for i in lin:
        A_i, b_i = ctx.get_condensed(i)
        assert _rel(A_i, cond[i]["Ahat"]) < 1e-10, f"Ahat macro {i}"
        assert _rel(b_i, cond[i]["bhat"]) < 1e-10, f"bhat macro {i}"
    A, b = S.assemble(cond)
    assert _rel(bhat.cpu().numpy(), b) < 1e-10
    x = np.random.default_rng(7).standard_normal(ctx.n_glob)
    y = torch.zeros_like(bhat)
    ctx.apply_global(to_dev(x), y)
    assert _rel(y.cpu().numpy(), A @ x) < 1e-12
    x_ref = S.solve_direct(A, b)
    xg = torch.zeros_like(bhat)
    info = ctx.fgmres_solve(bhat, xg, rtol=1e-13, restart=30, max_outer=400, inner_its=5)
    assert info["converged"], info
    assert _rel(xg.cpu().numpy(), x_ref) < 1e-10
    dq = torch.zeros(ctx.n_q_tot, dtype=torch.float64, device="cuda")
    du = torch.zeros(ctx.n_u_tot, dtype=torch.float64, device="cuda")
    ctx.local_backsolve(to_dev(x_ref), dq, du)
    dq_o, du_o = S.backsolve(lin, cond, x_ref)
    edu, edq = _rel(du.cpu().numpy(), du_o), _rel(dq.cpu().numpy(), dq_o)
    say(f"[chunked fp64] {name}: dU {edu:.2e} dQ {edq:.2e}")
    assert edu < 1e-10 and edq < 1e-10
    # the chunk condensed last was recovered from its elimination left in W;
    # a second recovery (W then holds recovery forms), and one after the
    # inspection of a formed matrix wrote W, form every chunk again
    for redo in ("second recovery", "after get_formed"):
        if redo == "after get_formed":
            ctx.condense(bhat)
            ctx.get_formed(0)
        dq.zero_()
        du.zero_()
        ctx.local_backsolve(to_dev(x_ref), dq, du)
        edu, edq = _rel(du.cpu().numpy(), du_o), _rel(dq.cpu().numpy(), dq_o)
        say(f"[chunked fp64] {name}, {redo}: dU {edu:.2e} dQ {edq:.2e}")
        assert edu < 1e-10 and edq < 1e-10
    # an FP32 inner operator needs an FP32 condensation when chunked
    from paper_2402_11361_amd.hdg import HDG_FP32, HdgError
    with pytest.raises(HdgError, match="EUNSUPPORTED"):
        ctx.fgmres_solve(bhat, xg, rtol=1e-8, inner_prec=HDG_FP32)


@pytest.mark.parametrize("name", list(CASES))
def test_chunked_fp32_matches_oracle(pairs, name):
    import torch
    from paper_2402_11361_amd.hdg import HDG_FP32
    S, inp, ctx, d, lin, cond = _get(pairs, name)
    say(f"[chunked fp32] {name}")
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat, HDG_FP32)
    ea = max(_rel(ctx.get_condensed(i)[0], cond[i]["Ahat"]) for i in lin)
    eb = max(_rel(ctx.get_condensed(i)[1], cond[i]["bhat"]) for i in lin)
    A, b = S.assemble(cond)
    eB = _rel(bhat.cpu().numpy(), b)
    say(f"[chunked fp32] {name}: A-hat {ea:.2e} b-hat {eb:.2e} assembled {eB:.2e}")
    assert 1e-10 < ea < TOL32 and eb < TOL32 and eB < TOL32
    x = np.random.default_rng(7).standard_normal(ctx.n_glob)
    y = torch.zeros_like(bhat)
    ctx.apply_global(to_dev(x), y)
    assert _rel(y.cpu().numpy(), A @ x) < TOL32
    # FP32 inner operator on the FP32 condensation
    xg = torch.zeros_like(bhat)
    info = ctx.fgmres_solve(bhat, xg, rtol=1e-10, restart=30, max_outer=400, inner_its=5, inner_prec=HDG_FP32)
    assert info["converged"], info
    x_ref = S.solve_direct(A, b)
    dq = torch.zeros(ctx.n_q_tot, dtype=torch.float64, device="cuda")
    du = torch.zeros(ctx.n_u_tot, dtype=torch.float64, device="cuda")
    ctx.local_backsolve(to_dev(x_ref), dq, du)
    dq_o, du_o = S.backsolve(lin, cond, x_ref)
    # refined in FP64 against the u-rows' residual (FP32 factors only precondition it)
    assert _rel(du.cpu().numpy(), du_o) < 1e-10 and _rel(dq.cpu().numpy(), dq_o) < 1e-10
    # the last chunk from the condensation's factors above; every chunk formed again here
    dq.zero_()
    du.zero_()
    ctx.local_backsolve(to_dev(x_ref), dq, du)
    assert _rel(du.cpu().numpy(), du_o) < 1e-10 and _rel(dq.cpu().numpy(), dq_o) < 1e-10


def test_chunked_formed_matrix_of_a_middle_chunk(pairs):
    S, inp, ctx, d, lin, cond = _get(pairs, "3d_per_p2_chunk3")
    i = 4  # second chunk
    say(f"[chunked formed] macro {i}")
    blk = lin[i]["blk"]
    Qi = S.geo(S.mclass[i])["Qi"]
    c = cond[i]
    nu = S.cls(i).n_u
    W = ctx.get_formed(i)
    E = blk["A_bb"] - blk["A_bq"] @ Qi @ blk["A_qb"]
    g = -lin[i]["RB"] + blk["A_bq"] @ Qi @ lin[i]["RQ"]
    ref = np.vstack([np.hstack([c["S"], -c["right"], c["f"][:, None]]), np.hstack([c["left"], E, g[:, None]])])
    assert np.abs(W - ref).max() / np.abs(ref).max() < 1e-12


def test_chunked_newton_refines_fp32_to_oracle():
    """FP32 chunked condensation inside the Newton stage solve reaches the
    oracle's FP64 stage solution."""
    from oracle.newton import newton_solve
    from paper_2402_11361_amd.driver import StageDriver
    from paper_2402_11361_amd.hdg import HDG_FP32
    case, per, _, _ = CASES["3d_per_uneven_p2_chunk2"]
    say("[chunked newton] 3d_per_uneven_p2 chunks of 2, FP32")
    S, inp, ctx = make_pair(case)
    ctx.set_chunking(per)
    ctx.bind_workspace()
    qo, uo, uho, _ = newton_solve(S, inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"],
                                  abs_tol=1e-12, rel_tol=1e-12, max_it=12)
    drv = StageDriver(ctx, rtol=1e-10, newton_abs=1e-12, newton_rel=1e-12, max_newton=12, condense_prec=HDG_FP32)
    q, u, uh = to_dev(inp["q"]), to_dev(inp["u"]), to_dev(inp["uh"])
    res = drv.solve_stage(q, u, uh, to_dev(inp["w"]), inp["dt"], inp["dii"])
    assert res["res_hist"][-1] < 1e-11
    eu, euh, eq = _rel(u.cpu().numpy(), uo), _rel(uh.cpu().numpy(), uho), _rel(q.cpu().numpy(), qo)
    say(f"[chunked newton] u {eu:.2e} uhat {euh:.2e} q {eq:.2e}")
    assert eu < 1e-8 and euh < 1e-8 and eq < 1e-8


def test_chunked_newton_with_factor_store_matches_oracle():
    """FP64 chunked condensation with an FP32 factor store inside the Newton
    stage solve: every linearisation invalidates the store and the next
    condensation refills it; the stage solution is the oracle's."""
    from oracle.newton import newton_solve
    from paper_2402_11361_amd.driver import StageDriver
    from paper_2402_11361_amd.hdg import HDG_FP32
    case, per, _, _ = CASES["3d_per_p2_chunk2_store32"]
    say("[chunked newton] 3d_per_p2 chunks of 2, FP64 with an FP32 factor store of 4 macros")
    S, inp, ctx = make_pair(case)
    ctx.set_chunking(per)
    assert ctx.set_factor_store(4, HDG_FP32) == 4
    ctx.bind_workspace()
    qo, uo, uho, _ = newton_solve(S, inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"],
                                  abs_tol=1e-12, rel_tol=1e-12, max_it=12)
    drv = StageDriver(ctx, rtol=1e-12, newton_abs=1e-12, newton_rel=1e-12, max_newton=12)
    q, u, uh = to_dev(inp["q"]), to_dev(inp["u"]), to_dev(inp["uh"])
    res = drv.solve_stage(q, u, uh, to_dev(inp["w"]), inp["dt"], inp["dii"])
    assert res["res_hist"][-1] < 1e-11
    eu, euh, eq = _rel(u.cpu().numpy(), uo), _rel(uh.cpu().numpy(), uho), _rel(q.cpu().numpy(), qo)
    say(f"[chunked newton store] u {eu:.2e} uhat {euh:.2e} q {eq:.2e}")
    assert eu < 1e-10 and euh < 1e-10 and eq < 1e-10


def test_progress_lines_name_every_chunk(capfd):
    """hdg_set_progress: one line per finished chunk of the condensation and
    of the recovery (stored chunks together, the resident chunk none)."""
    import torch
    from paper_2402_11361_amd.hdg import HDG_FP32
    case, per, _, _ = CASES["3d_per_p2_chunk2_store32"]
    say("[chunked progress] 3d_per_p2 chunks of 2, store of 4")
    S, inp, ctx = make_pair(case)
    ctx.set_chunking(per)
    ctx.set_factor_store(4, HDG_FP32)
    ctx.bind_workspace()
    ctx.set_progress(True)
    d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat)
    dq = torch.zeros(ctx.n_q_tot, dtype=torch.float64, device="cuda")
    du = torch.zeros(ctx.n_u_tot, dtype=torch.float64, device="cuda")
    ctx.local_backsolve(bhat, dq, du)
    torch.cuda.synchronize()
    err = capfd.readouterr().err
    for j in range(1, 5):
        assert f"[hdg] condensation: chunk {j} of 4 done" in err, err
    assert "[hdg] recovery: stored chunks 2 of 4 done" in err, err
    assert "[hdg] recovery: chunk 3 of 4 done" in err, err
    assert "[hdg] recovery: chunk 4 of 4 done" not in err  # left in W by the condensation
    ctx.set_progress(False)
    ctx.condense(bhat)
    torch.cuda.synchronize()
    assert "[hdg]" not in capfd.readouterr().err
    ctx.close()
