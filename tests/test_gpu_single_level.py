"""Single-level GMRES (the face-block inverse of A_uh,uh as the only
preconditioner, no inner GMRES) against the oracle's direct solve, and its
iteration count against the multi-level method (Sec. 4.2, Table 2: the
multi-level preconditioner needs fewer outer iterations)."""
import numpy as np
import pytest

from gpu_common import make_pair, to_dev, say

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("graph_steps", [0, 10])
def test_single_level_solution_and_iterations(graph_steps):
    import torch
    case = dict(dim=3, n_elem=4, m=2, p=2, periodic=True)
    say(f"[single level] graph_steps {graph_steps}")
    S, inp, ctx = make_pair(case)
    d = {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in inp.items()}
    ctx.linearize_stage(d["q"], d["u"], d["uh"], d["w"], inp["dt"], inp["dii"])
    lin = S.linearize(inp["q"], inp["u"], inp["uh"], w=inp["w"], dt=inp["dt"], dii=inp["dii"])
    cond = S.condense(lin, "B")
    A, b = S.assemble(cond)
    x_ref = S.solve_direct(A, b)
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    ctx.condense(bhat)
    its = {}
    for inner in (0, 5):
        x = torch.zeros_like(bhat)
        info = ctx.fgmres_solve(bhat, x, rtol=1e-12, restart=30, max_outer=3000, inner_its=inner,
                                graph_steps=graph_steps)
        assert info["converged"], info
        assert _rel(x.cpu().numpy(), x_ref) < 1e-8
        its[inner] = info["outer_its"]
    say(f"[single level] outer iterations: single-level {its[0]}, multi-level {its[5]}")
    assert its[0] > its[5]
