"""Macro-element HDG residuals (eq. C38a-c / C242) and their Jacobian blocks
(eq. C312) for one macro-element at a time.  Test infrastructure (oracle).

Per macro T_i (u, q continuous inside, u-hat on the macro boundary), with
test functions set to the nodal basis phi_a of the C0 macro space and the
trace basis mu_j of each macro face:

  R_Q[k,c,a] = (q_kc, phi_a) + (u_c, d_k phi_a) - <uhat_c n_k, phi_a>        (C38a)
  R_U[c,a]   = (dt_u_c, phi_a) - sum_k (F_kc + G_kc, d_k phi_a)
               + <fhat_c, phi_a> + SUPG[c,a] - (s_c, phi_a)                 (C38b)
  R_Uhat^(i)[c,j] = <fhat_c, mu_j>  on interior faces,                      (C38c)
                    <uhat_c - uD_c, mu_j> on Dirichlet boundary faces
  fhat = F(uhat).n + G(uhat, q).n + S (u - uhat),  S = lambda_max I + S_vis   (numerical flux)

Element-interior faces carry no terms because u and q are C0 inside a macro.
The discrete time derivative of a DIRK stage (eq. C242) is written
dt_u = (d_ii u + w) / dt with w = sum_{j<i} d_ij (u^{n,j} - u^n) - d_ii u^n;
dt = inf means steady (no time term).

With a degree per macro (mixed degrees; this oracle only), a macro's face
whose trace degree exceeds the macro's (a neighbour of higher degree) is
integrated with its own Gauss rule (MacroClass).

Readings (the paper defers these to its references; parity unpinned against
the paper, fixed here and in the HIP library by convention):
  * lambda_max = |v.n| + c of the trace state, frozen in the Jacobian;
  * SUPG: strong residual R = dt_u + sum_k d_k F_k^I + sum_k d_k G_k^I - s with
    F^I, G^I the nodal interpolants of the fluxes (group form); test operator
    (A_k d_k w) with A_k = dF_k/du at the quadrature state; scalar
    tau = ((2 d_ii/dt)^2 + (2 (|v|+c) p/h)^2 + (4 mu p^2/(Re_c rho h^2))^2)^(-1/2),
    h = smallest element edge; A_k and tau frozen in the Jacobian;
  * Dirichlet boundary operator B-hat = uhat - uD (weak, face mass);
  * pseudo-time continuation adds M/dtau to A_uu only.

The Jacobian is computed by complex-step differentiation of these residuals
(J[:, c] = Im R(x + i h e_c) / h, h = 1e-30), independently of the analytic
derivatives used by the HIP library.
"""
import numpy as np
from functools import partial
from .basis import gll_nodes, gauss_rule, lagrange
from . import physics as phy

_ein = partial(np.einsum, optimize=True)


class MacroClass:
    """Reference tables for all macros of one shape (m per axis, p, h per axis)
    and trace degrees of its 2d local faces (face_deg, default p each).

    A face of trace degree pf > p (a neighbour of higher degree) carries
    Tf = (pf + 1)^(d-1) trace nodes per sub-face and its own Gauss rule of
    max(p, pf) + 2 points per direction; the per-element face arrays are
    padded to the largest Tf (T), the padding inactive (Tf and the trace
    basis Psi's zero columns mark it)."""

    def __init__(self, dim, m, p, h, nq=None, face_deg=None):
        self.dim = d = dim
        self.m = list(m)
        self.p = p
        self.face_deg = [p] * (2 * d) if face_deg is None else [int(v) for v in face_deg]
        self.h = list(h)
        self.ns = d + 2
        self.nq1 = nq if nq is not None else p + 2
        self.n1 = [mk * p + 1 for mk in self.m]
        self.N = int(np.prod(self.n1))
        g = gll_nodes(p)
        xq, wq = gauss_rule(self.nq1)
        V1, D1 = lagrange(g, xq)
        Vend, _ = lagrange(g, [-1.0, 1.0])
        A1 = p + 1
        self.A = A1 ** d              # nodes per element
        self.Q = self.nq1 ** d        # volume quadrature points per element
        # local node / qp multi-indices (axis 0 fastest)
        aidx = np.array(np.unravel_index(np.arange(self.A), [A1] * d, order="F")).T
        qidx = np.array(np.unravel_index(np.arange(self.Q), [self.nq1] * d, order="F")).T
        Phi = np.ones((self.Q, self.A))
        dPhi = np.ones((d, self.Q, self.A))
        W = np.ones(self.Q)
        for k in range(d):
            Phi *= V1[qidx[:, k]][:, aidx[:, k]]
            W *= wq[qidx[:, k]] * self.h[k] / 2.0
            for j in range(d):
                if j == k:
                    dPhi[k] *= (2.0 / self.h[k]) * D1[qidx[:, j]][:, aidx[:, j]]
                else:
                    dPhi[k] *= V1[qidx[:, j]][:, aidx[:, j]]
        self.Phi, self.dPhi, self.W = Phi, dPhi, W
        self.xq_ref = np.stack([(xq[qidx[:, k]] + 1.0) / 2.0 for k in range(d)], axis=1)  # in [0,1]
        # elements
        self.E = int(np.prod(self.m))
        eidx = np.array(np.unravel_index(np.arange(self.E), self.m, order="F")).T
        self.eidx = eidx
        self.elem_nodes = np.zeros((self.E, self.A), dtype=int)
        for e in range(self.E):
            gidx = eidx[e][None, :] * p + aidx  # [A, d]
            self.elem_nodes[e] = np.ravel_multi_index(gidx.T, self.n1, order="F")
        # macro faces: 2d local faces, sub-faces, face quadrature
        self.nf_nodes = []   # trace nodes per local face
        self.face_sub = []   # per local face: list of (element, trace node ids [Tf], padded to T with 0)
        self.Tf = [(pf + 1) ** (d - 1) for pf in self.face_deg]
        self.T = max(self.Tf)
        self.Fq = self.nq1 ** (d - 1)
        self.face_tabs = []
        for lf in range(2 * d):
            k, s = divmod(lf, 2)
            tang = [j for j in range(d) if j != k]
            pf = self.face_deg[lf]
            tn = [mk * pf + 1 for mk in (self.m[j] for j in tang)]
            self.nf_nodes.append(int(np.prod(tn)))
            if pf == p:
                nqf, xqf, wqf, V1f, Vt = self.nq1, xq, wq, V1, V1
            else:
                nqf = max(p, pf) + 2
                xqf, wqf = gauss_rule(nqf)
                V1f, _ = lagrange(g, xqf)
                Vt, _ = lagrange(gll_nodes(pf), xqf)
            Fq = nqf ** (d - 1)
            fq = np.array(np.unravel_index(np.arange(Fq), [nqf] * (d - 1), order="F")).T
            tt = np.array(np.unravel_index(np.arange(self.Tf[lf]), [pf + 1] * (d - 1), order="F")).T
            # volume basis and trace basis at the face quadrature points
            PhiF = np.ones((Fq, self.A))
            Psi = np.ones((Fq, self.Tf[lf]))
            WF = np.ones(Fq)
            for j in range(d):
                if j == k:
                    PhiF *= Vend[s][aidx[:, j]][None, :]
                else:
                    t = tang.index(j)
                    PhiF *= V1f[fq[:, t]][:, aidx[:, j]]
                    Psi *= Vt[fq[:, t]][:, tt[:, t]]
                    WF *= wqf[fq[:, t]] * self.h[j] / 2.0
            if self.Tf[lf] < self.T:
                Psi = np.concatenate([Psi, np.zeros((Fq, self.T - self.Tf[lf]))], axis=1)
            nvec = np.zeros(d); nvec[k] = -1.0 if s == 0 else 1.0
            fqref = np.zeros((Fq, d))
            for j in range(d):
                if j == k:
                    fqref[:, j] = 0.0 if s == 0 else 1.0
                else:
                    fqref[:, j] = (xqf[fq[:, tang.index(j)]] + 1.0) / 2.0
            subs = []
            for e in range(self.E):
                if eidx[e][k] != (0 if s == 0 else self.m[k] - 1):
                    continue
                tid = []
                for r in range(self.Tf[lf]):
                    tcoord = [eidx[e][tang[t]] * pf + tt[r, t] for t in range(d - 1)]
                    tid.append(np.ravel_multi_index(tcoord, tn, order="F") if d == 3 else tcoord[0])
                tid += [0] * (self.T - self.Tf[lf])
                subs.append((e, np.array(tid, dtype=int)))
            self.face_sub.append(subs)
            self.face_tabs.append(dict(PhiF=PhiF, Psi=Psi, WF=WF, n=nvec, k=k, s=s, xref=fqref))
        self.nf_off = np.concatenate([[0], np.cumsum(self.nf_nodes)[:-1]]) * self.ns
        self.n_u = self.ns * self.N
        self.n_q = d * self.ns * self.N
        self.n_b = self.ns * int(sum(self.nf_nodes))


def _tau_supg(uq_real, ph, p, hmin, dii, dt):
    rho, v, E, P = phy.primitives(uq_real, ph)
    d = uq_real.shape[0] - 2
    vn = np.sqrt(sum(v[j] ** 2 for j in range(d)))
    c = np.sqrt(ph.gamma * P / rho)
    t_time = (2.0 * dii / dt) ** 2 if np.isfinite(dt) else 0.0
    t_adv = (2.0 * (vn + c) * p / hmin) ** 2
    t_vis = (4.0 * ph.mu * p * p / (ph.Re_c * rho * hmin * hmin)) ** 2
    return (t_time + t_adv + t_vis) ** -0.5


def element_residual(mc, ph, ue, qe, ube, face_on, we=None, dt=np.inf, dii=1.0,
                     is_bnd=None, uDe=None, supg=False, src=None):
    """Contributions of single elements to the macro residuals.

    ue [X, ns, A], qe [X, d, ns, A], ube [X, 2d, ns, T] (trace on the element's
    sub-face of each local macro face), face_on [X, 2d] (1 where that element
    face lies on the macro boundary), we [X, ns, A], is_bnd [X, 2d] (Dirichlet),
    uDe like ube, src [X, ns, Q] source at the volume quadrature points.
    Returns RQe [X, d, ns, A], RUe [X, ns, A], RBe [X, 2d, ns, T]."""
    d, ns = mc.dim, mc.ns
    X = ue.shape[0]
    steady = not np.isfinite(dt)
    W = mc.W
    uq = _ein("qa,xca->cxq", mc.Phi, ue)                 # [ns, X, Q]
    qq = _ein("qa,xkca->kcxq", mc.Phi, qe)               # [d, ns, X, Q]
    F = phy.flux_inviscid(uq, ph)
    G = phy.flux_viscous(uq, qq, ph)
    RQe = _ein("q,qa,kcxq->xkca", W, mc.Phi, qq) + _ein("q,kqa,cxq->xkca", W, mc.dPhi, uq)
    RUe = -_ein("q,kqa,kcxq->xca", W, mc.dPhi, F + G)
    if not steady:
        wq = _ein("qa,xca->cxq", mc.Phi, we) if we is not None else 0.0
        tt = (dii * uq + wq) / dt
        RUe = RUe + _ein("q,qa,cxq->xca", W, mc.Phi, tt)
    if src is not None:
        RUe = RUe - _ein("q,qa,xcq->xca", W, mc.Phi, src)
    if supg:
        Fn = phy.flux_inviscid(np.moveaxis(ue, 1, 0), ph)                  # [d, ns, X, A]
        Gn = phy.flux_viscous(np.moveaxis(ue, 1, 0), np.moveaxis(qe, [1, 2], [0, 1]), ph)
        Rs = _ein("kqa,kcxa->cxq", mc.dPhi, Fn + Gn)
        if not steady:
            Rs = Rs + tt
        if src is not None:
            Rs = Rs - np.moveaxis(src, 1, 0)
        ur = np.real(uq)
        Ak = phy.inviscid_jacobian(ur, ph)                                 # [d, ns, ns, X, Q]
        tau = _tau_supg(ur, ph, mc.p, min(mc.h), dii, dt)                  # [X, Q]
        AtR = _ein("kycxq,xq,yxq->kcxq", Ak, tau, Rs)
        RUe = RUe + _ein("q,kqa,kcxq->xca", W, mc.dPhi, AtR)
    RBe = np.zeros((X, 2 * d, ns, mc.T), dtype=RUe.dtype)
    svis = phy.s_vis_diag(d, ph)
    for lf in range(2 * d):
        tab = mc.face_tabs[lf]
        k, n = tab["k"], tab["n"]
        on = face_on[:, lf].astype(float)
        if not on.any():
            continue
        WF = tab["WF"]
        uf = _ein("fa,xca->cxf", tab["PhiF"], ue)
        qf = _ein("fa,xkca->kcxf", tab["PhiF"], qe)
        uhf = _ein("ft,xct->cxf", tab["Psi"], ube[:, lf])
        Fh = phy.flux_inviscid(uhf, ph)
        Gh = phy.flux_viscous(uhf, qf, ph)
        lam = phy.lambda_max(uhf, n, ph)
        fn = sum((Fh[j] + Gh[j]) * n[j] for j in range(d)) + (lam[None] + svis[:, None, None]) * (uf - uhf)
        RUe = RUe + on[:, None, None] * _ein("f,fa,cxf->xca", WF, tab["PhiF"], fn)
        RQe[:, k] = RQe[:, k] - on[:, None, None] * _ein("f,fa,cxf->xca", WF, tab["PhiF"], uhf) * n[k]
        rb = _ein("f,ft,cxf->xct", WF, tab["Psi"], fn)
        if is_bnd is not None and np.any(is_bnd[:, lf]):
            uDq = _ein("ft,xct->cxf", tab["Psi"], uDe[:, lf])
            rbd = _ein("f,ft,cxf->xct", WF, tab["Psi"], uhf - uDq)
            rb = np.where(np.asarray(is_bnd[:, lf], bool)[:, None, None], rbd, rb)
        RBe[:, lf] = on[:, None, None] * rb
    return RQe, RUe, RBe


class _ElemMaps:
    """Index maps between element-local dofs and macro dofs for class mc."""

    def __init__(self, mc):
        d, ns, A, T, N = mc.dim, mc.ns, mc.A, mc.T, mc.N
        E = mc.E
        self.face_on = np.zeros((E, 2 * d))
        self.tid = np.zeros((E, 2 * d, T), dtype=int)
        for lf in range(2 * d):
            for (e, tid) in mc.face_sub[lf]:
                self.face_on[e, lf] = 1.0
                self.tid[e, lf] = tid
        en = mc.elem_nodes
        # element dof order: q[k,c,a], u[c,a], ub[lf,c,t]; macro dof order: q, u, ub
        qmap = (np.arange(d)[None, :, None, None] * ns * N + np.arange(ns)[None, None, :, None] * N
                + en[:, None, None, :])                                             # [E, d, ns, A]
        umap = mc.n_q + np.arange(ns)[None, :, None] * N + en[:, None, :]          # [E, ns, A]
        bmap = np.zeros((E, 2 * d, ns, T), dtype=int)
        for lf in range(2 * d):
            bmap[:, lf] = (mc.n_q + mc.n_u + mc.nf_off[lf] + np.arange(ns)[None, :, None] * mc.nf_nodes[lf]
                           + self.tid[:, lf][:, None, :])
        self.dof = np.concatenate([qmap.reshape(E, -1), umap.reshape(E, -1), bmap.reshape(E, -1)], axis=1)
        # trace dofs of a face on the macro boundary, without the padding past Tf
        fa = np.zeros((E, 2 * d, ns, T), dtype=bool)
        for lf in range(2 * d):
            fa[:, lf, :, :mc.Tf[lf]] = self.face_on[:, lf][:, None, None] > 0
        self.active = np.concatenate([np.ones((E, d * ns * A + ns * A), dtype=bool), fa.reshape(E, -1)], axis=1)
        self.ne = self.dof.shape[1]


def _maps(mc):
    if not hasattr(mc, "_emaps"):
        mc._emaps = _ElemMaps(mc)
    return mc._emaps


def _gather_elements(mc, q, u, ub, w, bnd, uD, origin, source):
    """Element-local arrays for a batch of macros (flattened to X = B*E)."""
    em = _maps(mc)
    d, ns, A, T, E = mc.dim, mc.ns, mc.A, mc.T, mc.E
    B = u.shape[0]
    en = mc.elem_nodes
    ue = np.moveaxis(u[:, :, en], 2, 1).reshape(B * E, ns, A)
    qe = np.moveaxis(q[:, :, :, en], 3, 1).reshape(B * E, d, ns, A)
    ube = np.zeros((B, E, 2 * d, ns, T), dtype=ub.dtype)
    uDe = None if uD is None else np.zeros((B, E, 2 * d, ns, T))
    for lf in range(2 * d):
        off, nf = mc.nf_off[lf], mc.nf_nodes[lf]
        ubf = ub[:, off:off + ns * nf].reshape(B, ns, nf)
        ube[:, :, lf] = np.moveaxis(ubf[:, :, em.tid[:, lf]], 2, 1)
        if uD is not None:
            uDf = uD[:, off:off + ns * nf].reshape(B, ns, nf)
            uDe[:, :, lf] = np.moveaxis(uDf[:, :, em.tid[:, lf]], 2, 1)
    ube = ube.reshape(B * E, 2 * d, ns, T)
    if uDe is not None:
        uDe = uDe.reshape(B * E, 2 * d, ns, T)
    we = None if w is None else np.moveaxis(w[:, :, en], 2, 1).reshape(B * E, ns, A)
    face_on = np.tile(em.face_on, (B, 1))
    is_bnd = None
    if bnd is not None:
        is_bnd = (np.asarray(bnd, bool)[:, None, :] & em.face_on[None].astype(bool)).reshape(B * E, 2 * d)
    src = None
    if source is not None:
        xq = origin[:, None, None, :] + (mc.eidx[None, :, None, :] + mc.xq_ref[None, None, :, :]) * np.array(mc.h)
        src = np.moveaxis(source(np.moveaxis(xq, -1, 0)), 0, 2).reshape(B * E, ns, mc.Q)
    return ue, qe, ube, we, face_on, is_bnd, uDe, src


def macro_residual(mc, ph, q, u, ub, w=None, dt=np.inf, dii=1.0, bnd=None, uD=None,
                   supg=False, source=None, origin=None):
    """Residuals (R_Q [B,d,ns,N], R_U [B,ns,N], R_Ub [B,n_b]) of a batch of macros
    of class mc: element contributions assembled into macro vectors.
    bnd [B, 2d] marks Dirichlet local faces, uD [B, n_b] their data, origin
    [B, d] the macro low corner (for the source term only)."""
    em = _maps(mc)
    B = u.shape[0]
    E = mc.E
    ue, qe, ube, we, face_on, is_bnd, uDe, src = _gather_elements(mc, q, u, ub, w, bnd, uD, origin, source)
    RQe, RUe, RBe = element_residual(mc, ph, ue, qe, ube, face_on, we, dt, dii, is_bnd, uDe, supg, src)
    Re = np.concatenate([RQe.reshape(B, E, -1), RUe.reshape(B, E, -1), RBe.reshape(B, E, -1)], axis=2)
    R = np.zeros((B, mc.n_q + mc.n_u + mc.n_b), dtype=Re.dtype)
    for e in range(E):
        act = em.active[e]
        np.add.at(R, (slice(None), em.dof[e][act]), Re[:, e][:, act])
    return (R[:, :mc.n_q].reshape(B, mc.dim, mc.ns, mc.N),
            R[:, mc.n_q:mc.n_q + mc.n_u].reshape(B, mc.ns, mc.N),
            R[:, mc.n_q + mc.n_u:])


def macro_jacobian(mc, ph, q, u, ub, w=None, dt=np.inf, dii=1.0, bnd=None, uD=None,
                   supg=False, source=None, origin=None, chunk=128):
    """Complex-step Jacobian of the assembled macro residual w.r.t. (q, u, ub):
    each element contribution is differentiated w.r.t. its own dofs
    (J_e[:, c] = Im R_e(x_e + i h e_c) / h, h = 1e-30) and the element
    Jacobians are assembled.  Returns J [B, n, n] in (q, u, ub) order and the
    real residuals."""
    em = _maps(mc)
    d, ns, A, T, E = mc.dim, mc.ns, mc.A, mc.T, mc.E
    B = u.shape[0]
    ue, qe, ube, we, face_on, is_bnd, uDe, src = _gather_elements(mc, q, u, ub, w, bnd, uD, origin, source)
    X = B * E
    nQ, nU = d * ns * A, ns * A
    x0 = np.concatenate([qe.reshape(X, -1), ue.reshape(X, -1), ube.reshape(X, -1)], axis=1)
    ne = x0.shape[1]
    h = 1e-30
    Je = np.zeros((X, ne, ne))

    def rep(a, C):
        return None if a is None else np.tile(a, (C,) + (1,) * (a.ndim - 1))

    for c0 in range(0, ne, chunk):
        cols = np.arange(c0, min(ne, c0 + chunk))
        C = cols.size
        Xc = np.repeat(x0[None].astype(complex), C, axis=0)
        Xc[np.arange(C), :, cols] += 1j * h
        Xc = Xc.reshape(C * X, ne)
        RQe, RUe, RBe = element_residual(
            mc, ph, Xc[:, nQ:nQ + nU].reshape(C * X, ns, A), Xc[:, :nQ].reshape(C * X, d, ns, A),
            Xc[:, nQ + nU:].reshape(C * X, 2 * d, ns, T), rep(face_on, C), rep(we, C), dt, dii,
            rep(is_bnd, C), rep(uDe, C), supg, rep(src, C))
        R = np.concatenate([RQe.reshape(C * X, -1), RUe.reshape(C * X, -1), RBe.reshape(C * X, -1)], axis=1)
        Je[:, :, cols] = np.transpose(R.reshape(C, X, ne).imag / h, (1, 2, 0))
    Je = Je.reshape(B, E, ne, ne)
    n = mc.n_q + mc.n_u + mc.n_b
    J = np.zeros((B, n, n))
    for e in range(E):
        act = em.active[e]
        dof = em.dof[e][act]
        J[:, dof[:, None], dof[None, :]] += Je[:, e][:, act][:, :, act]
    Rr = macro_residual(mc, ph, q, u, ub, w, dt, dii, bnd, uD, supg, source, origin)
    return J, tuple(np.real(r) for r in Rr)


def split_blocks(mc, J):
    """Split a macro Jacobian into the nine blocks of eq. (C312)."""
    nq, nu = mc.n_q, mc.n_u
    s = [slice(0, nq), slice(nq, nq + nu), slice(nq + nu, None)]
    names = ["q", "u", "b"]
    return {f"A_{names[r]}{names[c]}": J[..., s[r], s[c]] for r in range(3) for c in range(3)}


def mass_matrix(mc):
    """Assembled C0 macro mass matrix M[a,b] = (phi_a, phi_b) (dense, N x N)."""
    M = np.zeros((mc.N, mc.N))
    Me = _ein("q,qa,qb->ab", mc.W, mc.Phi, mc.Phi)
    for e in range(mc.E):
        M[np.ix_(mc.elem_nodes[e], mc.elem_nodes[e])] += Me
    return M


def face_mass(mc, lf):
    """Trace mass matrix <mu_i, mu_j> on local face lf (dense)."""
    tab = mc.face_tabs[lf]
    nf, tf = mc.nf_nodes[lf], mc.Tf[lf]
    Mf = np.zeros((nf, nf))
    Me = _ein("f,fs,ft->st", tab["WF"], tab["Psi"], tab["Psi"])[:tf, :tf]
    for (e, tid) in mc.face_sub[lf]:
        Mf[np.ix_(tid[:tf], tid[:tf])] += Me
    return Mf


def grad_matrices(mc):
    """B_k[a, b] = (phi_b, d_k phi_a) over the macro (dense, N x N each)."""
    out = []
    for k in range(mc.dim):
        Bk = np.zeros((mc.N, mc.N))
        Be = _ein("q,qa,qb->ab", mc.W, mc.dPhi[k], mc.Phi)
        for e in range(mc.E):
            Bk[np.ix_(mc.elem_nodes[e], mc.elem_nodes[e])] += Be
        out.append(Bk)
    return out


def face_matrices(mc):
    """E_k[a, j] = <mu_j n_k, phi_a> over the macro boundary; columns are the
    trace nodes of the 2d local faces in local order (node level, N x sum nf)."""
    nf_tot = int(sum(mc.nf_nodes))
    out = [np.zeros((mc.N, nf_tot)) for _ in range(mc.dim)]
    col = 0
    for lf in range(2 * mc.dim):
        tab = mc.face_tabs[lf]
        tf = mc.Tf[lf]
        Ee = _ein("f,fa,ft->at", tab["WF"], tab["PhiF"], tab["Psi"])[:, :tf]
        for (e, tid) in mc.face_sub[lf]:
            for k in range(mc.dim):
                out[k][np.ix_(mc.elem_nodes[e], col + tid[:tf])] += Ee * tab["n"][k]
        col += mc.nf_nodes[lf]
    return out
