"""Parity at the full 24^3 Taylor-Green workload (512 macros of 3^3 elements,
p = 2): oracle blocks for sampled macros, and properties that hold at any
size for the whole system (FGMRES true residual, Newton reduction)."""
import gc
import math

import numpy as np
import pytest

from gpu_common import to_dev, say

pytestmark = pytest.mark.gpu


def test_tgv24_sampled_macros_and_global_properties():
    import torch
    from oracle.mesh import box_mesh
    from oracle.physics import Phys
    from oracle.system import System
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.hdg import Context, mesh_spec_box
    cfg = dict(inputs.CONFIGS["tgv24_m3_p2"])
    say("[fullsize] building oracle mesh and inputs")
    M = box_mesh(3, cfg["n_elem"], cfg["m"], cfg["p"], lo=cfg["lo"], hi=cfg["hi"], periodic=True)
    S = System(M, Phys(Re=cfg["Re"], Mach=cfg["mach"]))
    mc = [M.macro_node_coords(i) for i in range(M.n_macros)]
    fc = [M.face_node_coords(f) for f in range(M.n_faces)]
    u, q, uh = inputs.make_state(cfg, mc, fc, seed=0)
    dii = 1.0 / 0.435866521508459
    dt = inputs.cfl_dt(cfg)
    w = -dii * u
    spec = mesh_spec_box(3, cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], True)
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"])
    ctx.bind_workspace()
    # the library's node coordinates are the oracle's
    mx, fx = ctx.node_coords()
    assert np.abs(mx - np.concatenate(mc)).max() < 1e-13
    assert np.abs(fx - np.concatenate(fc)).max() < 1e-13
    d = dict(q=to_dev(q), u=to_dev(u), uh=to_dev(uh), w=to_dev(w))
    say("[fullsize] GPU linearise")
    nrm = ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], dt, dii)
    sample = [0, 137, 511]
    say("[fullsize] oracle linearise of sampled macros")
    lin = S.linearize(q, u, uh, w=w, dt=dt, dii=dii, macros=sample)
    cond = S.condense(lin, "B")
    rq, ru, rb = (t.cpu().numpy() for t in ctx.get_residuals())
    for i in sample:
        L = lin[i]
        sl = slice(S.u_off[i], S.u_off[i + 1])
        assert np.abs(ru[sl] - L["RU"]).max() < 1e-10 * np.abs(L["RU"]).max()
        assert np.abs(rq[S.q_off[i]:S.q_off[i + 1]] - L["RQ"]).max() < 1e-10 * np.abs(L["RQ"]).max()
        W = ctx.get_formed(i)
        c = cond[i]
        nu = S.cls(i).n_u
        ref_top = np.hstack([c["S"], -c["right"], c["f"][:, None]])
        assert np.abs(W[:nu] - ref_top).max() < 1e-12 * np.abs(ref_top).max()
    say("[fullsize] GPU condense")
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat)
    for i in sample:
        A_i, b_i = ctx.get_condensed(i)
        assert np.abs(A_i - cond[i]["Ahat"]).max() < 1e-10 * np.abs(cond[i]["Ahat"]).max()
        assert np.abs(b_i - cond[i]["bhat"]).max() < 1e-10 * np.abs(cond[i]["bhat"]).max()
    say("[fullsize] GPU FGMRES")
    x = torch.zeros_like(bhat)
    info = ctx.fgmres_solve(bhat, x, rtol=1e-10, restart=30, max_outer=400, inner_its=5)
    assert info["converged"]
    y = torch.zeros_like(bhat)
    ctx.apply_global(x, y)
    rel = float(torch.linalg.norm(bhat - y) / torch.linalg.norm(bhat))
    assert rel <= 1.01e-10, rel
    say("[fullsize] recovery + Newton update")
    dq = torch.zeros_like(d["q"]); du = torch.zeros_like(d["u"])
    ctx.local_backsolve(x, dq, du)
    ctx.axpy(1.0, dq, d["q"]); ctx.axpy(1.0, du, d["u"]); ctx.axpy(1.0, x, d["uh"])
    nrm2 = ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], dt, dii)
    r0, r1 = math.sqrt((nrm ** 2).sum()), math.sqrt((nrm2 ** 2).sum())
    say(f"[fullsize] Newton residual {r0:.3e} -> {r1:.3e}")
    assert r1 < 1e-2 * r0


def _setup_tgv(name):
    """Oracle System, seeded state and a library context for a Taylor-Green
    workload of inputs.CONFIGS, condensed in chunks sized to the free device
    memory."""
    import torch
    from oracle.mesh import box_mesh
    from oracle.physics import Phys
    from oracle.system import System
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.hdg import Context, mesh_spec_box
    cfg = dict(inputs.CONFIGS[name])
    say(f"[fullsize {name}] oracle mesh and inputs")
    M = box_mesh(3, cfg["n_elem"], cfg["m"], cfg["p"], lo=cfg["lo"], hi=cfg["hi"], periodic=True)
    S = System(M, Phys(Re=cfg["Re"], Mach=cfg["mach"]))
    mc = [M.macro_node_coords(i) for i in range(M.n_macros)]
    fc = [M.face_node_coords(f) for f in range(M.n_faces)]
    u, q, uh = inputs.make_state(cfg, mc, fc, seed=0)
    dii = 1.0 / 0.435866521508459
    dt = inputs.cfl_dt(cfg)
    w = -dii * u
    spec = mesh_spec_box(3, cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], True)
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"])
    gc.collect()  # earlier tests' workspaces back to the device
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    per = ctx.fit_chunking(free - (8 << 30))
    say(f"[fullsize {name}] {ctx.n_macros} macros, {per} per chunk, workspace {ctx.workspace_bytes / 1e9:.1f} GB")
    ctx.bind_workspace()
    d = dict(q=to_dev(q), u=to_dev(u), uh=to_dev(uh), w=to_dev(w))
    return S, ctx, dict(q=q, u=u, uh=uh, w=w, dt=dt, dii=dii), d, per


def _solve_recover_and_check_newton(ctx, d, inp, nrm, rtol, inner_prec):
    import torch
    bhat = ctx._bhat
    x = torch.zeros_like(bhat)
    info = ctx.fgmres_solve(bhat, x, rtol=rtol, restart=30, max_outer=400, inner_its=5, inner_prec=inner_prec)
    assert info["converged"], info
    y = torch.zeros_like(bhat)
    ctx.apply_global(x, y)
    rel = float(torch.linalg.norm(bhat - y) / torch.linalg.norm(bhat))
    say(f"[fullsize] FGMRES {info['outer_its']} outer, true residual {rel:.2e}")
    assert rel <= 1.01 * rtol, rel
    dq = torch.zeros_like(d["q"]); du = torch.zeros_like(d["u"])
    ctx.local_backsolve(x, dq, du)
    ctx.axpy(1.0, dq, d["q"]); ctx.axpy(1.0, du, d["u"]); ctx.axpy(1.0, x, d["uh"])
    nrm2 = ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    r0, r1 = math.sqrt((nrm ** 2).sum()), math.sqrt((nrm2 ** 2).sum())
    say(f"[fullsize] Newton residual {r0:.3e} -> {r1:.3e}")
    assert r1 < 1e-2 * r0


def test_tgv48_m4_p2_chunked_sampled_macros_and_global_properties():
    """48^3, 4^3-element macros (1728), p = 2, FP64: the augmented matrices
    (510 GB) do not fit, so the condensation runs in chunks."""
    import torch
    S, ctx, inp, d, per = _setup_tgv("tgv48_m4_p2")
    assert 0 < per < ctx.n_macros
    say("[fullsize tgv48] GPU linearise")
    nrm = ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    sample = [0, 1000]
    say("[fullsize tgv48] oracle linearise of sampled macros")
    lin = S.linearize(inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"], macros=sample)
    cond = S.condense(lin, "B")
    rq, ru, rb = (t.cpu().numpy() for t in ctx.get_residuals())
    for i in sample:
        L = lin[i]
        assert np.abs(ru[S.u_off[i]:S.u_off[i + 1]] - L["RU"]).max() < 1e-10 * np.abs(L["RU"]).max()
        assert np.abs(rq[S.q_off[i]:S.q_off[i + 1]] - L["RQ"]).max() < 1e-10 * np.abs(L["RQ"]).max()
    say("[fullsize tgv48] GPU condense (chunked, FP64)")
    ctx._bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(ctx._bhat)
    for i in sample:
        A_i, b_i = ctx.get_condensed(i)
        ea = np.abs(A_i - cond[i]["Ahat"]).max() / np.abs(cond[i]["Ahat"]).max()
        eb = np.abs(b_i - cond[i]["bhat"]).max() / np.abs(cond[i]["bhat"]).max()
        say(f"[fullsize tgv48] macro {i}: A-hat {ea:.2e} b-hat {eb:.2e}")
        assert ea < 1e-10 and eb < 1e-10
    from paper_2402_11361_amd.hdg import HDG_FP64
    _solve_recover_and_check_newton(ctx, d, inp, nrm, 1e-8, HDG_FP64)
    ctx.close()


def test_tgv32_m4_p3_chunked_fp32_residuals_and_global_properties():
    """32^3, 4^3-element macros (512), p = 3 (n_u = 10985 per macro), FP32
    chunked condensation: residuals of sampled macros against the oracle
    (its Jacobian of one such macro takes minutes on the CPU), then the
    FGMRES true residual and the Newton reduction, which hold only if the
    condensed operator is the Jacobian of the residual."""
    import torch
    from paper_2402_11361_amd.hdg import HDG_FP32
    S, ctx, inp, d, per = _setup_tgv("tgv32_m4_p3")
    say("[fullsize tgv32 p3] GPU linearise")
    nrm = ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    sample = [0, 300, 511]
    res = S.macro_residuals(inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"], macros=sample)
    rq, ru, rb = (t.cpu().numpy() for t in ctx.get_residuals())
    for i in sample:
        RQ_i, RU_i, _ = res[i]
        assert np.abs(ru[S.u_off[i]:S.u_off[i + 1]] - RU_i).max() < 1e-10 * np.abs(RU_i).max()
        assert np.abs(rq[S.q_off[i]:S.q_off[i + 1]] - RQ_i).max() < 1e-10 * np.abs(RQ_i).max()
    say("[fullsize tgv32 p3] GPU condense (chunked, FP32)")
    ctx._bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(ctx._bhat, HDG_FP32)
    _solve_recover_and_check_newton(ctx, d, inp, nrm, 1e-8, HDG_FP32)
    ctx.close()
