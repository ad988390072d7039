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
