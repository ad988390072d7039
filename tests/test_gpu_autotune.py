"""The elimination autotuner: launch shapes picked per macro class and
precision by timing, cached in a text file, and condensation results that
still match the oracle with the chosen shapes."""
import numpy as np
import pytest

from gpu_common import make_pair, to_dev, say

pytestmark = pytest.mark.gpu

CASE = dict(dim=3, seg=[[2, 3], [3, 2], [2, 2]], p=2, periodic=True)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_autotune_caches_and_keeps_parity(tmp_path):
    import torch
    from paper_2402_11361_amd.hdg import HDG_FP32, HDG_FP64, HdgError
    say("[autotune] uneven 3D p=2")
    S, inp, ctx = make_pair(CASE)
    with pytest.raises(HdgError, match="linearisation"):
        ctx.autotune(HDG_FP64)
    d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    ncl = ctx.class_count()
    assert ncl == 4
    cache = tmp_path / "lu_tuning.txt"
    assert ctx.autotune(HDG_FP64, cache) == ncl
    lines = cache.read_text().splitlines()
    assert len(lines) == ncl
    for k, line in enumerate(lines):
        f = line.split()
        assert f[2] == "fp64" and int(f[9]) in (8, 16, 32, 64, 128, 256) and int(f[10]) in (0, 1, 2) and int(f[11]) in (0, 1)
        assert ctx.tuning(k, HDG_FP64) == (int(f[9]), int(f[10]), int(f[11]))
    # the cache answers a second call without timing
    assert ctx.autotune(HDG_FP64, cache) == 0
    assert ctx.autotune(HDG_FP32, cache) == ncl
    assert len(cache.read_text().splitlines()) == 2 * ncl
    say("[autotune] tuned: " + ", ".join(f"{ctx.tuning(k, HDG_FP64)}/{ctx.tuning(k, HDG_FP32)}" for k in range(ncl)))
    # condensation with the chosen shapes
    lin = S.linearize(inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"])
    cond = S.condense(lin, "B")
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat, HDG_FP64)
    for i in lin:
        A_i, b_i = ctx.get_condensed(i)
        assert _rel(A_i, cond[i]["Ahat"]) < 1e-10 and _rel(b_i, cond[i]["bhat"]) < 1e-10
    A, b = S.assemble(cond)
    assert _rel(bhat.cpu().numpy(), b) < 1e-10
    ctx.condense(bhat, HDG_FP32)
    ea = max(_rel(ctx.get_condensed(i)[0], cond[i]["Ahat"]) for i in lin)
    say(f"[autotune] FP32 A-hat {ea:.2e}")
    assert ea < 5e-4


@pytest.mark.parametrize("case", [dict(dim=3, n_elem=4, m=2, p=2, periodic=True), CASE])
@pytest.mark.parametrize("shape", [(16, 1, 1), (64, 0, 1), (8, 1, 0), (16, 2, 1), (32, 2, 0)])
def test_forced_launch_shapes_keep_parity(case, shape):
    """Every launch shape the autotuner may pick (the look-ahead stream and
    tournament pivoting included) gives the oracle's condensed blocks and
    recovery."""
    import torch
    from paper_2402_11361_amd.hdg import HDG_FP64
    say(f"[shapes] {shape}")
    S, inp, ctx = make_pair(case)
    for k in range(ctx.class_count()):
        ctx.set_tuning(k, HDG_FP64, *shape)
        assert ctx.tuning(k, HDG_FP64) == shape
    d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    lin = S.linearize(inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"])
    cond = S.condense(lin, "B")
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat, HDG_FP64)
    for i in lin:
        A_i, b_i = ctx.get_condensed(i)
        assert _rel(A_i, cond[i]["Ahat"]) < 1e-10 and _rel(b_i, cond[i]["bhat"]) < 1e-10
    # recovery re-uses the factors
    A, b = S.assemble(cond)
    x_ref = S.solve_direct(A, b)
    dq = torch.zeros(ctx.n_q_tot, dtype=torch.float64, device="cuda")
    du = torch.zeros(ctx.n_u_tot, dtype=torch.float64, device="cuda")
    ctx.local_backsolve(to_dev(x_ref), dq, du)
    dq_o, du_o = S.backsolve(lin, cond, x_ref)
    assert _rel(du.cpu().numpy(), du_o) < 1e-10 and _rel(dq.cpu().numpy(), dq_o) < 1e-10
