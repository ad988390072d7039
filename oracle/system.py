"""Whole-mesh oracle: linearisation of all macros, condensation, assembly of
the global trace system (eq. C44), direct and Krylov solves, local recovery
and the Newton update (Sec. 3.1, Algorithms 1 and 2).  Test infrastructure.

Global layouts: u = concatenation over macros of [comp][node]; q likewise of
[dir][comp][node]; u-hat = [face][comp][facenode] (see mesh.py).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from .discretization import (MacroClass, macro_residual, macro_jacobian, split_blocks,
                             mass_matrix, grad_matrices, face_matrices)
from . import condense as cd


class System:
    def __init__(self, mesh, phys, supg=False, source=None, uD=None):
        self.mesh = mesh
        self.ph = phys
        self.supg = supg
        self.source = source
        self.uD = uD                      # global trace vector of Dirichlet data (or None)
        d = mesh.dim
        self.classes = {}
        self.mclass = []
        for i in range(mesh.n_macros):
            # shape; with mixed degrees also the macro's degree and its faces' trace degrees
            key = tuple(mesh.macro_m(i))
            if mesh.mixed:
                key = key + (mesh.macro_deg(i),) + tuple(mesh.macro_face_degs(i))
            if key not in self.classes:
                if mesh.mixed:
                    self.classes[key] = MacroClass(d, list(key[:d]), key[d], mesh.h, face_deg=list(key[d + 1:]))
                else:
                    self.classes[key] = MacroClass(d, list(key), mesh.p, mesh.h)
            self.mclass.append(key)
        nu = [self.cls(i).n_u for i in range(mesh.n_macros)]
        nq = [self.cls(i).n_q for i in range(mesh.n_macros)]
        self.u_off = np.concatenate([[0], np.cumsum(nu)]).astype(int)
        self.q_off = np.concatenate([[0], np.cumsum(nq)]).astype(int)
        self.bnd = np.array([[mesh.face_is_boundary(mesh.macro_faces[i, lf]) for lf in range(2 * d)]
                             for i in range(mesh.n_macros)])
        self._geo = {}

    def cls(self, i):
        return self.classes[self.mclass[i]]

    def geo(self, key):
        """Mass, gradient and face matrices of a macro class (independent of
        the state)."""
        if key not in self._geo:
            mc = self.classes[key]
            M = mass_matrix(mc)
            Bk = grad_matrices(mc)
            Ek = face_matrices(mc)
            self._geo[key] = dict(M=M, Bk=Bk, Ek=Ek, Qi=cd.qinv(mc, M),
                                  qblk=cd.geometric_qblocks(mc, M, Bk, Ek))
        return self._geo[key]

    def origin(self, i):
        s = self.mesh.macro_seg(i)
        return np.array([self.mesh.lo[k] + self.mesh.seg_start[k][s[k]] * self.mesh.h[k]
                         for k in range(self.mesh.dim)])

    def local(self, i, q, u, uhat, w):
        mc = self.cls(i)
        qi = q[self.q_off[i]:self.q_off[i + 1]].reshape(mc.dim, mc.ns, mc.N)
        ui = u[self.u_off[i]:self.u_off[i + 1]].reshape(mc.ns, mc.N)
        bi = uhat[self.mesh.macro_trace_index(i)]
        wi = None if w is None else w[self.u_off[i]:self.u_off[i + 1]].reshape(mc.ns, mc.N)
        return qi, ui, bi, wi

    def _kw(self, i, w_i, dt, dii):
        kw = dict(dt=dt, dii=dii, supg=self.supg)
        if w_i is not None:
            kw["w"] = w_i[None]
        if self.bnd[i].any():
            kw["bnd"] = self.bnd[i][None]
            kw["uD"] = (self.uD[self.mesh.macro_trace_index(i)] if self.uD is not None
                        else np.zeros(self.cls(i).n_b))[None]
        if self.source is not None:
            kw["source"] = self.source
            kw["origin"] = self.origin(i)[None]
        return kw

    # ---- residuals ----------------------------------------------------
    def residual(self, q, u, uhat, w=None, dt=np.inf, dii=1.0):
        """Global residual vectors (R_Q, R_U, R_Uhat); R_Uhat sums both sides."""
        RQ = np.zeros_like(q)
        RU = np.zeros_like(u)
        RB = np.zeros(self.mesh.n_glob)
        for i in range(self.mesh.n_macros):
            mc = self.cls(i)
            qi, ui, bi, wi = self.local(i, q, u, uhat, w)
            rq, ru, rb = macro_residual(mc, self.ph, qi[None], ui[None], bi[None], **self._kw(i, wi, dt, dii))
            RQ[self.q_off[i]:self.q_off[i + 1]] = rq.reshape(-1)
            RU[self.u_off[i]:self.u_off[i + 1]] = ru.reshape(-1)
            np.add.at(RB, self.mesh.macro_trace_index(i), rb.reshape(-1))
        return RQ, RU, RB

    def macro_residuals(self, q, u, uhat, w=None, dt=np.inf, dii=1.0, macros=()):
        """Per-macro residual pieces {i: (R_Q^(i), R_U^(i), R_Uhat^(i))} of the
        listed macros (R_Uhat^(i): this macro's side of its faces)."""
        out = {}
        for i in macros:
            mc = self.cls(i)
            qi, ui, bi, wi = self.local(i, q, u, uhat, w)
            rq, ru, rb = macro_residual(mc, self.ph, qi[None], ui[None], bi[None], **self._kw(i, wi, dt, dii))
            out[i] = (rq.reshape(-1), ru.reshape(-1), rb.reshape(-1))
        return out

    # ---- linearisation --------------------------------------------------
    def linearize(self, q, u, uhat, w=None, dt=np.inf, dii=1.0, dtau=np.inf, macros=None):
        """Per-macro Jacobian blocks (eq. C312) and residuals.  Pseudo-time
        continuation adds M/dtau to A_uu."""
        out = {}
        macros = range(self.mesh.n_macros) if macros is None else macros
        for i in macros:
            mc = self.cls(i)
            qi, ui, bi, wi = self.local(i, q, u, uhat, w)
            J, (rq, ru, rb) = macro_jacobian(mc, self.ph, qi[None], ui[None], bi[None],
                                             **self._kw(i, wi, dt, dii))
            blk = split_blocks(mc, J[0])
            if np.isfinite(dtau):
                blk["A_uu"] = blk["A_uu"] + np.kron(np.eye(mc.ns), self.geo(self.mclass[i])["M"]) / dtau
            out[i] = dict(blk=blk, RQ=rq.reshape(-1), RU=ru.reshape(-1), RB=rb.reshape(-1))
        return out

    # ---- condensation ---------------------------------------------------
    def condense(self, lin, route="B"):
        out = {}
        for i, L in lin.items():
            g = self.geo(self.mclass[i])
            if route == "B":
                out[i] = cd.route_b(L["blk"], L["RQ"], L["RU"], L["RB"], g["Qi"])
            else:
                out[i] = cd.route_a(L["blk"], L["RQ"], L["RU"], L["RB"])
        return out

    def assemble(self, cond):
        """A-hat = sum_i P_i^T A-hat^{T_i} P_i (sparse) and b-hat (eq. C44,
        Algorithm 1 assembly)."""
        rows, cols, vals = [], [], []
        b = np.zeros(self.mesh.n_glob)
        for i, C in cond.items():
            idx = self.mesh.macro_trace_index(i)
            rows.append(np.repeat(idx, idx.size))
            cols.append(np.tile(idx, idx.size))
            vals.append(C["Ahat"].reshape(-1))
            np.add.at(b, idx, C["bhat"])
        n = self.mesh.n_glob
        A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
        return A, b

    def apply_alg2(self, lin, cond, x):
        """Matrix-free y = A-hat x following Algorithm 2 literally."""
        y = np.zeros(self.mesh.n_glob)
        for i, L in lin.items():
            idx = self.mesh.macro_trace_index(i)
            y4 = cd.alg2_apply_local(L["blk"], cond[i], self.geo(self.mclass[i])["Qi"], x[idx])
            np.add.at(y, idx, y4)
        return y

    def backsolve(self, lin, cond, x):
        """dQ, dU for every macro from the trace increment x (eq. Csc4)."""
        dq = np.zeros(self.q_off[-1])
        du = np.zeros(self.u_off[-1])
        for i, L in lin.items():
            idx = self.mesh.macro_trace_index(i)
            Qi = self.geo(self.mclass[i])["Qi"]
            if "left" in cond[i]:
                dQ, dU = cd.backsolve_b(L["blk"], cond[i], Qi, L["RQ"], x[idx])
            else:
                dQ, dU = cd.backsolve_a(L["blk"], cond[i], L["RQ"], L["RU"], x[idx])
            dq[self.q_off[i]:self.q_off[i + 1]] = dQ
            du[self.u_off[i]:self.u_off[i + 1]] = dU
        return dq, du

    def face_blocks_Abb(self, lin):
        """Per-face blocks of A_uhat-uhat summed over the (one or two) macro
        sides: the preconditioner blocks of Sec. 4.2."""
        m = self.mesh
        blocks = [np.zeros((m.face_ndof[f], m.face_ndof[f])) for f in range(m.n_faces)]
        for i, L in lin.items():
            mc = self.cls(i)
            off = 0
            for lf in range(2 * m.dim):
                f = m.macro_faces[i, lf]
                nf = m.face_ndof[f]
                blocks[f] += L["blk"]["A_bb"][off:off + nf, off:off + nf]
                off += nf
        return blocks

    def solve_direct(self, A, b):
        return spla.splu(A.tocsc()).solve(b)
