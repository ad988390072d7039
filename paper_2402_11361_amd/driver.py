"""Time stepping driver: DIRK(3,3) stages, each solved by Newton's method with
optional pseudo-transient continuation (paper Sec. 2.4, Sec. 3.1, Algorithm 1).

Host-side control only: every vector update and every solve goes through the
C ABI (hdg_linearize_stage, hdg_condense, hdg_fgmres_solve or the nested
hdg_condense_nested + hdg_nested_solve, hdg_local_backsolve, hdg_axpy);
torch provides the device buffers.

Time integrator: Alexander's three-stage L-stable SDIRK, alpha the root in
(0, 1) of 6a^3 - 18a^2 + 9a - 1, stiffly accurate (c_3 = 1, b = last row of
A), so u^{n+1} is the last stage (the post-processing solve of eq. C243 is
not needed, remark after eq. C243).  Stage i uses the discrete derivative
(d_ii u + w)/dt with d = A^{-1} and w = sum_{j<i} d_ij (u^{n,j} - u^n) - d_ii u^n
(eq. C242).

Pseudo-transient continuation (eq. C31222, ratio read as ||R_U^m|| /
||R_U^{m+1}||): dtau^0 = tau_init, dtau^{m+1} = min(dtau^m ||R_U^m|| /
||R_U^{m+1}||, tau_max); it adds M/dtau to A_uu.
"""
import math

import numpy as np

from .hdg import HDG_FP64


def alexander_dirk33():
    """Butcher table (A, b, c) of Alexander's 3-stage SDIRK."""
    f = lambda a: ((6.0 * a - 18.0) * a + 9.0) * a - 1.0
    fp = lambda a: (18.0 * a - 36.0) * a + 9.0
    a = 0.4358665215
    for _ in range(50):  # Newton on the cubic, started inside (0.4, 0.5)
        a -= f(a) / fp(a)
    A = np.array([[a, 0.0, 0.0],
                  [(1.0 - a) / 2.0, a, 0.0],
                  [(-6.0 * a * a + 16.0 * a - 1.0) / 4.0, (6.0 * a * a - 20.0 * a + 5.0) / 4.0, a]])
    return A, A[2].copy(), A.sum(axis=1)


class StageDriver:
    """Newton solves of DIRK stages on one library context."""

    def __init__(self, ctx, rtol=1e-8, restart=30, inner_its=5, max_outer=300, newton_abs=1e-10, newton_rel=1e-8,
                 max_newton=20, inner_prec=HDG_FP64, condense_prec=HDG_FP64, mark=None, use_learned=False,
                 graph_steps=0, nested_block=0):
        """nested_block > 0 (one element per macro, FP64): every Newton step
        goes through the nested path, hdg_condense_nested with blocks of that
        many elements per axis and hdg_nested_solve on the block skeleton."""
        import torch
        self.ctx = ctx
        self.nested_block = int(nested_block)
        # optional callback mark(phase) at phase boundaries ("linearize", "condense",
        # "fgmres", "backsolve"), e.g. to record stream events
        self.mark = mark if mark is not None else (lambda phase: None)
        self.t = torch
        self.kry = dict(rtol=rtol, restart=restart, inner_its=inner_its, max_outer=max_outer, inner_prec=inner_prec,
                        use_learned=use_learned, graph_steps=graph_steps)
        self.newton_abs, self.newton_rel, self.max_newton = newton_abs, newton_rel, max_newton
        self.condense_prec = condense_prec
        dev = dict(dtype=torch.float64, device="cuda")
        self.bhat = torch.zeros(ctx.n_glob, **dev)
        self.x = torch.zeros(ctx.n_glob, **dev)
        self.dq = torch.zeros(ctx.n_q_tot, **dev)
        self.du = torch.zeros(ctx.n_u_tot, **dev)
        self.A, self.b, self.c = alexander_dirk33()
        self.Ainv = np.linalg.inv(self.A)
        self.nested_A = self.nested_b = None  # the block systems (output of hdg_condense_nested)

    def solve_stage(self, q, u, uh, w, dt, dii, ptc=False, tau_init=1.0, tau_max=1e8):
        """Newton iterations on (q, u, uh) in place until ||R_F|| <= max(abs, rel ||R_F^0||)."""
        ctx = self.ctx
        dtau = tau_init if ptc else math.inf
        hist, krylov, dtaus = [], [], []
        rU_prev = None
        r0 = None
        mark = self.mark
        for it in range(self.max_newton + 1):
            mark("linearize")
            nrm = ctx.linearize_stage(q, u, uh, w, dt, dii, dtau)
            rn = float(np.sqrt(np.sum(nrm ** 2)))
            hist.append(rn)
            if r0 is None:
                r0 = rn
            if ptc and rU_prev is not None:
                dtau = min(dtau * rU_prev / max(nrm[1], 1e-300), tau_max)
                nrm = ctx.linearize_stage(q, u, uh, w, dt, dii, dtau)
            rU_prev = nrm[1]
            if rn <= max(self.newton_abs, self.newton_rel * r0) or it == self.max_newton:
                break
            dtaus.append(dtau)
            mark("condense")
            ctx.condense(self.bhat, self.condense_prec)
            mark("fgmres")
            self.x.zero_()
            if self.nested_block > 0:
                if self.nested_A is None:
                    nb, _, nB = ctx.nested_dims(self.nested_block)
                    self.nested_A = self.t.empty(nb * nB * nB, dtype=self.t.float64, device="cuda")
                    self.nested_b = self.t.empty(nb * nB, dtype=self.t.float64, device="cuda")
                ctx.condense_nested(self.nested_block, self.nested_A, self.nested_b)
                krylov.append(ctx.nested_solve(self.nested_block, self.x, rtol=self.kry["rtol"],
                                               restart=self.kry["restart"], max_outer=self.kry["max_outer"],
                                               inner_its=self.kry["inner_its"]))
            else:
                krylov.append(ctx.fgmres_solve(self.bhat, self.x, **self.kry))
            mark("backsolve")
            ctx.local_backsolve(self.x, self.dq, self.du)
            ctx.axpy(1.0, self.dq, q)
            ctx.axpy(1.0, self.du, u)
            ctx.axpy(1.0, self.x, uh)
        mark("end")
        return dict(newton_its=len(hist) - 1, res_hist=hist, krylov=krylov, dtau_hist=dtaus)

    def step(self, q, u, uh, dt):
        """One DIRK(3,3) time step in place; returns per-stage infos."""
        t = self.t
        ctx = self.ctx
        u_n = u.clone()
        stages = []
        w = t.empty_like(u)
        infos = []
        for i in range(3):
            # w = -d_ii u^n + sum_{j<i} d_ij (u^{n,j} - u^n)
            w.zero_()
            ctx.axpy(-self.Ainv[i, i], u_n, w)
            for j in range(i):
                ctx.axpy(self.Ainv[i, j], stages[j], w)
                ctx.axpy(-self.Ainv[i, j], u_n, w)
            infos.append(self.solve_stage(q, u, uh, w, dt, self.Ainv[i, i]))
            stages.append(u.clone())
        # stiffly accurate: u^{n+1} = u^{n,3} (already in u)
        return infos
