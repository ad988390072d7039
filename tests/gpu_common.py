"""Helpers shared by the GPU tests: build the oracle case and the matching
library context on the same mesh and seeded inputs."""
import math
import sys

import numpy as np

from cases import small_case
from oracle import dirk


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def mesh_spec_from(S):
    M = S.mesh
    if M.mixed:
        raise ValueError("the library takes one degree per mesh; mixed degrees are an oracle-only case")
    return dict(dim=M.dim, n_elem=M.n_elem, lo=M.lo, hi=M.hi, periodic=M.periodic,
                seg_len=[list(s) for s in M.seg_len], p=M.p)


def make_pair(case, supg=False):
    """(oracle System, inputs dict, library Context with bound workspace)."""
    import torch
    from paper_2402_11361_amd.hdg import Context
    kw = dict(case)
    S, q, u, uh, uD = small_case(supg=supg, **kw)
    ph = S.ph
    has_bnd = any(S.mesh.face_is_boundary(f) for f in range(S.mesh.n_faces))
    ctx = Context.from_mesh_spec(mesh_spec_from(S), gamma=ph.gamma, Pr=ph.Pr, Re=ph.Re, Mach=ph.Mach,
                                 supg=supg, bc_state=uD if has_bnd else None)
    ctx.bind_workspace()
    A, b, c = dirk.dirk33()
    dii = 1.0 / A[0, 0]
    h = (S.mesh.hi[0] - S.mesh.lo[0]) / S.mesh.n_elem[0]
    dt = h / (ph.Mach * (S.mesh.p + 1))
    w = -dii * u * (1.0 - 1e-3)
    inp = dict(q=q, u=u, uh=uh, w=w, dt=dt, dii=dii)
    return S, inp, ctx


def to_dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()
