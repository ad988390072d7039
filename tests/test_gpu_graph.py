"""Device-resident FGMRES steps replayed from HIP graphs against the
host-controlled FGMRES on the same condensed operator: same iteration counts
and the same solution, on every replay of the cached graphs, with eager
library work and synchronisations between the replays."""
import numpy as np
import pytest

from gpu_common import make_pair, to_dev, say

pytestmark = pytest.mark.gpu


def _setup(case, prec):
    import torch
    S, inp, ctx = make_pair(case)
    d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat, prec)
    return ctx, bhat


@pytest.mark.parametrize("prec,restart,k,inner", [(0, 30, 10, 5), (1, 30, 10, 5), (0, 12, 5, 3), (0, 20, 7, 0)])
def test_graph_fgmres_matches_host_fgmres(prec, restart, k, inner):
    import torch
    say(f"[graph] prec {prec} restart {restart} graph_steps {k} inner {inner}")
    ctx, bhat = _setup(dict(dim=3, n_elem=4, m=2, p=2, periodic=True), prec)
    xh = torch.zeros_like(bhat)
    ih = ctx.fgmres_solve(bhat, xh, rtol=1e-11, restart=restart, inner_its=inner, max_outer=400)
    assert ih["converged"]
    y = torch.empty_like(bhat)
    for rep in range(3):
        xg = torch.zeros_like(bhat)
        ig = ctx.fgmres_solve(bhat, xg, rtol=1e-11, restart=restart, inner_its=inner, max_outer=400, graph_steps=k)
        e = float((xg - xh).norm() / xh.norm())
        say(f"[graph] replay {rep}: outer its host {ih['outer_its']} graph {ig['outer_its']}, rel diff {e:.2e}, "
            f"{ih['ms']:.1f} ms vs {ig['ms']:.1f} ms")
        assert ig["converged"]
        assert abs(ig["outer_its"] - ih["outer_its"]) <= 1
        assert e < 1e-9
        # eager library work and a synchronisation between replays
        ctx.apply_global(xg, y)
        torch.cuda.synchronize()


def test_graph_respects_max_outer_and_reports_noconv():
    import torch
    say("[graph] max_outer inside a graph batch")
    ctx, bhat = _setup(dict(dim=3, n_elem=4, m=2, p=2, periodic=True), 0)
    xh = torch.zeros_like(bhat)
    ih = ctx.fgmres_solve(bhat, xh, rtol=1e-14, restart=30, inner_its=2, max_outer=7, allow_noconv=True)
    xg = torch.zeros_like(bhat)
    ig = ctx.fgmres_solve(bhat, xg, rtol=1e-14, restart=30, inner_its=2, max_outer=7, allow_noconv=True,
                          graph_steps=5)
    assert not ih["converged"] and not ig["converged"]
    assert ih["outer_its"] == 7 and ig["outer_its"] == 7
    assert float((xg - xh).norm() / xh.norm()) < 1e-10
