"""First-layer (standard) static condensation on the GPU against the
oracle's route A (eq. C47: the local matrix of q and u factored at once)
and against the library's second layer: same condensed blocks, solution
and recovery."""
import numpy as np
import pytest

from gpu_common import make_pair, to_dev, say

pytestmark = pytest.mark.gpu

CASES = {
    "3d_per_p2": (dict(dim=3, n_elem=4, m=2, p=2, periodic=True), 3),
    "2d_dir_p3": (dict(dim=2, n_elem=4, m=2, p=3, periodic=False, state="shear", mach=0.2), 2),
}


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", list(CASES))
def test_first_layer_matches_route_a_and_second_layer(name):
    import torch
    case, per = CASES[name]
    say(f"[first layer] {name}")
    S, inp, ctx = make_pair(case)
    ctx.set_chunking(per)
    ctx.bind_workspace()
    d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    lin = S.linearize(inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"])
    cond_a = S.condense(lin, "A")
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense_first_layer(bhat)
    first = {}
    for i in lin:
        A_i, b_i = ctx.get_condensed(i)
        first[i] = (A_i, b_i)
        assert _rel(A_i, cond_a[i]["Ahat"]) < 1e-10, f"Ahat macro {i}"
        assert _rel(b_i, cond_a[i]["bhat"]) < 1e-10, f"bhat macro {i}"
    A, b = S.assemble(cond_a)
    assert _rel(bhat.cpu().numpy(), b) < 1e-10
    x = np.random.default_rng(7).standard_normal(ctx.n_glob)
    y = torch.zeros_like(bhat)
    ctx.apply_global(to_dev(x), y)
    assert _rel(y.cpu().numpy(), A @ x) < 1e-12
    x_ref = S.solve_direct(A, b)
    xg = torch.zeros_like(bhat)
    info = ctx.fgmres_solve(bhat, xg, rtol=1e-13, restart=30, max_outer=400, inner_its=5)
    assert info["converged"] and _rel(xg.cpu().numpy(), x_ref) < 1e-10
    dq = torch.zeros(ctx.n_q_tot, dtype=torch.float64, device="cuda")
    du = torch.zeros(ctx.n_u_tot, dtype=torch.float64, device="cuda")
    ctx.local_backsolve(to_dev(x_ref), dq, du)
    dq_o, du_o = S.backsolve(lin, S.condense(lin, "B"), x_ref)
    assert _rel(du.cpu().numpy(), du_o) < 1e-10 and _rel(dq.cpu().numpy(), dq_o) < 1e-10
    # the second layer gives the same blocks
    b2 = torch.zeros_like(bhat)
    ctx.condense(b2)
    ea = max(_rel(ctx.get_condensed(i)[0], first[i][0]) for i in lin)
    say(f"[first layer] {name}: first vs second layer A-hat {ea:.2e}")
    assert ea < 1e-10 and _rel(b2.cpu().numpy(), bhat.cpu().numpy()) < 1e-10


def test_first_layer_needs_chunking():
    import torch
    from paper_2402_11361_amd.hdg import HdgError
    S, inp, ctx = make_pair(CASES["3d_per_p2"][0])
    b = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    with pytest.raises(HdgError, match="EUNSUPPORTED"):
        ctx.condense_first_layer(b)


def test_first_layer_tgv24_sampled_macros():
    """The 24^3 workload in two chunks: first-layer blocks of sampled macros
    against the oracle's route A, then the same blocks from the second layer
    (pivot order 6860: the 24-row panel instance)."""
    import torch
    from oracle.mesh import box_mesh
    from oracle.physics import Phys
    from oracle.system import System
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.hdg import Context, mesh_spec_box
    cfg = dict(inputs.CONFIGS["tgv24_m3_p2"])
    say("[first layer tgv24] oracle mesh and inputs")
    M = box_mesh(3, cfg["n_elem"], cfg["m"], cfg["p"], lo=cfg["lo"], hi=cfg["hi"], periodic=True)
    S = System(M, Phys(Re=cfg["Re"], Mach=cfg["mach"]))
    mc = [M.macro_node_coords(i) for i in range(M.n_macros)]
    fc = [M.face_node_coords(f) for f in range(M.n_faces)]
    u, q, uh = inputs.make_state(cfg, mc, fc, seed=0)
    dii = 1.0 / 0.435866521508459
    dt = inputs.cfl_dt(cfg)
    w = -dii * u
    ctx = Context.from_mesh_spec(mesh_spec_box(3, cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], True),
                                 Re=cfg["Re"], Mach=cfg["mach"])
    ctx.set_chunking((ctx.n_macros + 1) // 2)
    ctx.bind_workspace()
    ctx.linearize_stage(to_dev(q), to_dev(u), to_dev(uh), to_dev(w), dt, dii)
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    say("[first layer tgv24] GPU first-layer condensation")
    ctx.condense_first_layer(bhat)
    sample = [0, 511]
    first = {i: ctx.get_condensed(i) for i in sample}
    say("[first layer tgv24] oracle route A of sampled macros")
    lin = S.linearize(q, u, uh, w=w, dt=dt, dii=dii, macros=sample)
    cond = S.condense(lin, "A")
    for i in sample:
        ea, eb = _rel(first[i][0], cond[i]["Ahat"]), _rel(first[i][1], cond[i]["bhat"])
        say(f"[first layer tgv24] macro {i}: A-hat {ea:.2e} b-hat {eb:.2e}")
        assert ea < 1e-10 and eb < 1e-10
    b1 = bhat.clone()
    ctx.condense(bhat)
    for i in sample:
        assert _rel(ctx.get_condensed(i)[0], first[i][0]) < 1e-10
    assert _rel(b1.cpu().numpy(), bhat.cpu().numpy()) < 1e-10
    ctx.close()
