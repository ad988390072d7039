"""Newton / pseudo-transient continuation for one nonlinear stage (Sec. 3.1).
Test infrastructure (oracle).

Readings: the SER update of eq. (C31222) is printed with the residual ratio
inverted; used as dtau^{m+1} = min(dtau^m ||R_U^m|| / ||R_U^{m+1}||, tau_max)
with the Euclidean norm of the residual vector, tau_init = 1, tau_max = 1e8;
stop when ||R_F||_2 <= max(abs_tol, rel_tol ||R_F^0||_2).
"""
import numpy as np
from . import krylov


def face_block_precond(S, lin):
    blocks = S.face_blocks_Abb(lin)
    inv = [np.linalg.inv(B) for B in blocks]
    offs = S.mesh.face_offset
    nd = S.mesh.face_ndof

    def Minv(v):
        out = np.empty_like(v)
        for f, Bi in enumerate(inv):
            out[offs[f]:offs[f] + nd[f]] = Bi @ v[offs[f]:offs[f] + nd[f]]
        return out
    return Minv


def newton_solve(S, q, u, uhat, w=None, dt=np.inf, dii=1.0, ptc=False, tau_init=1.0, tau_max=1e8,
                 abs_tol=1e-10, rel_tol=1e-8, max_it=20, linear="direct", krylov_opts=None):
    """Solve R(q, u, uhat) = 0 for one stage.  Returns (q, u, uhat, info)."""
    q, u, uhat = q.copy(), u.copy(), uhat.copy()
    hist, dtaus = [], []
    dtau = tau_init if ptc else np.inf
    RQ, RU, RB = S.residual(q, u, uhat, w, dt, dii)
    r0 = np.sqrt(RQ @ RQ + RU @ RU + RB @ RB)
    rU_prev = np.linalg.norm(RU)
    for it in range(max_it):
        rn = np.sqrt(RQ @ RQ + RU @ RU + RB @ RB)
        hist.append(rn)
        if rn <= max(abs_tol, rel_tol * r0):
            break
        lin = S.linearize(q, u, uhat, w, dt, dii, dtau)
        dtaus.append(dtau)
        cond = S.condense(lin, "B")
        A, b = S.assemble(cond)
        if linear == "direct":
            x = S.solve_direct(A, b)
        else:
            ko = dict(restart=30, rtol=1e-10, inner=5)
            ko.update(krylov_opts or {})
            Minv = face_block_precond(S, lin)
            Aop = lambda v: A @ v
            P = lambda v: krylov.gmres_left_fixed(Aop, Minv, v, ko["inner"])
            x, _ = krylov.fgmres(Aop, b, precond=P, restart=ko["restart"], rtol=ko["rtol"])
        dq, du = S.backsolve(lin, cond, x)
        q, u, uhat = q + dq, u + du, uhat + x
        RQ, RU, RB = S.residual(q, u, uhat, w, dt, dii)
        if ptc:
            rU = np.linalg.norm(RU)
            dtau = min(dtau * rU_prev / max(rU, 1e-300), tau_max)
            rU_prev = rU
    return q, u, uhat, dict(res_hist=hist, its=len(hist) - 1, dtau_hist=dtaus)


def dirk_step(S, q, u, uhat, dt, newton_kw=None):
    """One step of the DIRK(3,3) scheme (eq. C242 stages, eq. C241 update) with
    a Newton solve per stage; returns (q, u, uhat, infos)."""
    from . import dirk
    A, b, c = dirk.dirk33()
    Ai = np.linalg.inv(A)
    u_n = u.copy()
    stages, infos = [], []
    kw = dict(newton_kw or {})
    for i in range(3):
        w = dirk.stage_history(Ai, i, u_n, stages)
        q, u, uhat, info = newton_solve(S, q, u, uhat, w=w, dt=dt, dii=Ai[i, i], **kw)
        stages.append(u.copy())
        infos.append(info)
    u = dirk.update(Ai, b, u_n, stages)
    return q, u, uhat, infos
