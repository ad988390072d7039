"""Small seeded problems shared by the oracle tests and the GPU parity tests."""
import numpy as np
from oracle.mesh import box_mesh, Mesh
from oracle.physics import Phys
from oracle.system import System
from paper_2402_11361_amd import inputs


def small_case(dim=2, n_elem=4, m=2, p=2, periodic=True, state="tgv", mach=0.1, Re=100.0,
               noise=1e-3, supg=False, seed=0, lo=None, hi=None, seg=None, macro_p=None):
    """A small mesh with a seeded state; returns (System, q, u, uhat, uD).
    macro_p: optional degree per macro (mixed degrees, oracle only)."""
    if lo is None:
        lo, hi = ((-np.pi, np.pi) if state == "tgv" else (0.0, 1.0))
    if seg is None:
        M = box_mesh(dim, n_elem, m, p, lo=lo, hi=hi, periodic=periodic, macro_p=macro_p)
    else:
        per = [periodic] * dim if np.isscalar(periodic) else periodic
        M = Mesh(dim, [sum(s) for s in seg], [lo] * dim, [hi] * dim, per, seg, p, macro_p)
    cfg = dict(state=state, mach=mach, noise=noise)
    mc = [M.macro_node_coords(i) for i in range(M.n_macros)]
    fc = [M.face_node_coords(f) for f in range(M.n_faces)]
    u, q, uh = inputs.make_state(cfg, mc, fc, seed=seed)
    uD = inputs.exact_trace(cfg, fc)
    S = System(M, Phys(Re=Re, Mach=mach), supg=supg, uD=uD)
    return S, q, u, uh, uD
