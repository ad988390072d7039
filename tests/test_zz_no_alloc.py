"""The flow-diagnostics entry point that allocates nothing
(hdg_flow_diagnostics_noalloc, static device scratch) against the workspace
entry point hdg_flow_diagnostics: the same kernels, so the same bits, on two
calls in a row, the second on a smaller mesh."""
import numpy as np
import pytest

from gpu_common import make_pair, to_dev, say

pytestmark = pytest.mark.gpu

CASES = [("3d_per_p2_larger", dict(dim=3, n_elem=6, m=3, p=2, periodic=True)),
         ("3d_per_uneven_p2_smaller", dict(dim=3, seg=[[2, 1], [1, 2], [2, 1]], p=2, periodic=True))]


def test_noalloc_matches_workspace_entry_twice():
    pairs = []
    for name, case in CASES:
        S, inp, ctx = make_pair(case)
        pairs.append((name, S, inp, ctx))
    for name, S, inp, ctx in pairs:
        say(f"[no-alloc] {name}: n_u_tot={ctx.n_u_tot}")
        q, u = to_dev(inp["q"]), to_dev(inp["u"])
        got = ctx.flow_diagnostics_noalloc(q, u)
        ref = ctx.flow_diagnostics(q, u)
        assert got == ref, (name, got, ref)
        assert np.all(np.isfinite(got)) and got[2] > 0
        # the scratch keeps the last call's contents: a repeat gives the same bits
        assert ctx.flow_diagnostics_noalloc(q, u) == ref


def test_noalloc_needs_no_workspace():
    from oracle.diagnostics import flow_diagnostics
    from oracle.mesh import box_mesh
    from oracle.physics import Phys
    from oracle.system import System
    from paper_2402_11361_amd.hdg import Context, mesh_spec_box
    from paper_2402_11361_amd import inputs
    say("[no-alloc] context without a workspace")
    M = box_mesh(3, 4, 2, 2, lo=-np.pi, hi=np.pi, periodic=True)
    ctx = Context.from_mesh_spec(mesh_spec_box(3, 4, 2, 2, -np.pi, np.pi, True), Re=100.0, Mach=0.1)
    cfg = dict(state="tgv", mach=0.1, noise=0.0)
    mc = [M.macro_node_coords(i) for i in range(M.n_macros)]
    fc = [M.face_node_coords(f) for f in range(M.n_faces)]
    u, q, _ = inputs.make_state(cfg, mc, fc, seed=0)
    got = ctx.flow_diagnostics_noalloc(to_dev(q), to_dev(u))
    ref = flow_diagnostics(System(M, Phys(Re=100.0, Mach=0.1)), q, u)
    for g, r in zip(got, ref):
        assert abs(g - r) <= 1e-12 * abs(r), (got, ref)
