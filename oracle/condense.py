"""Static condensation of the macro-local Newton system.  Test infrastructure
(oracle).

Route A (standard static condensation, eq. C46/C47): dense A_local =
[[A_qq, A_qu], [A_uq, A_uu]] factored with LU.
Route B (second-layer static condensation, eq. AP12/ASC2/Csc4): A_qq inverted
block by block through the macro mass matrix (A_{q_k q_k} = M, so
A_qq^{-1} = I (x) M^{-1}), the Schur complement S = A_uu - A_uq A_qq^{-1} A_qu
factored with LU and never inverted (remark after Csc4).
Algorithm 2 applies A-hat^{T_i} matrix-free through S^{-1} solves.
"""
import numpy as np
import scipy.linalg as sla


def geometric_qblocks(mc, M, Bk, Ek):
    """The state-independent blocks of eq. (C38a) for one macro:
    A_qq = I_{d ns} (x) M, A_qu[k] = I_ns (x) B_k (B_k[a,b] = (phi_b, d_k phi_a)),
    A_qb[k] = -(I_ns (x) E_k) (E_k[a,j] = <mu_j n_k, phi_a>)."""
    d, ns, N = mc.dim, mc.ns, mc.N
    I = np.eye(ns)
    Aqq = np.kron(np.eye(d * ns), M)
    Aqu = np.concatenate([np.kron(I, Bk[k]) for k in range(d)], axis=0)
    Aqb = np.concatenate([-_kron_comp(mc, Ek[k]) for k in range(d)], axis=0)
    return Aqq, Aqu, Aqb


def _kron_comp(mc, Ek):
    """Expand a node-level face matrix E [N, sum_f nf] to component-level
    [ns N, n_b] with the local trace layout (faces, each [comp][facenode])."""
    ns, N = mc.ns, mc.N
    out = np.zeros((ns * N, mc.n_b))
    col = 0
    for lf, nf in enumerate(mc.nf_nodes):
        off = mc.nf_off[lf]
        for c in range(ns):
            out[c * N:(c + 1) * N, off + c * nf: off + (c + 1) * nf] = Ek[:, col:col + nf]
        col += nf
    return out


def qinv(mc, M):
    """A_qq^{-1} = I_{d ns} (x) M^{-1} (paper: inverse of A_{q_k q_k} from the
    reference mass matrix; exact here since each macro is an affine box)."""
    Mi = np.linalg.inv(M)
    return np.kron(np.eye(mc.dim * mc.ns), Mi)


def route_b(blk, RQ, RU, RB, Qi):
    """Second-layer condensation (eq. ASC2a/b) of one macro.  Returns
    A-hat^{T_i}, b-hat^{T_i} and the pieces needed by Algorithm 2 and Csc4."""
    Aqq, Aqu, Aqb = blk["A_qq"], blk["A_qu"], blk["A_qb"]
    Auq, Auu, Aub = blk["A_uq"], blk["A_uu"], blk["A_ub"]
    Abq, Abu, Abb = blk["A_bq"], blk["A_bu"], blk["A_bb"]
    S = Auu - Auq @ Qi @ Aqu
    lu = sla.lu_factor(S)
    left = Abu - Abq @ Qi @ Aqu                    # (A_uhat u - A_uhat q A_qq^-1 A_qu)
    right = -Aub + Auq @ Qi @ Aqb                  # (-A_u uhat + A_uq A_qq^-1 A_q uhat)
    Ahat = left @ sla.lu_solve(lu, right) + (Abb - Abq @ Qi @ Aqb)
    f = -RU + Auq @ Qi @ RQ
    bhat = -left @ sla.lu_solve(lu, f) + (-RB + Abq @ Qi @ RQ)
    return dict(Ahat=Ahat, bhat=bhat, S=S, lu=lu, left=left, right=right, f=f)


def route_a(blk, RQ, RU, RB):
    """Standard static condensation (eq. C47a/b) with a dense LU of A_local."""
    Aloc = np.block([[blk["A_qq"], blk["A_qu"]], [blk["A_uq"], blk["A_uu"]]])
    lu = sla.lu_factor(Aloc)
    Bc = np.concatenate([blk["A_qb"], blk["A_ub"]], axis=0)
    Rr = np.concatenate([blk["A_bq"], blk["A_bu"]], axis=1)
    Ahat = blk["A_bb"] - Rr @ sla.lu_solve(lu, Bc)
    bhat = -RB + Rr @ sla.lu_solve(lu, np.concatenate([RQ, RU]))
    return dict(Ahat=Ahat, bhat=bhat, lu=lu)


def alg2_apply_local(blk, rb, Qi, x):
    """Steps 1-4 of Algorithm 2 for one macro: y4 = A-hat^{T_i} x without
    forming A-hat^{T_i}; S^{-1} is applied by LU back-substitution."""
    Aqu, Aqb = blk["A_qu"], blk["A_qb"]
    Auq, Aub = blk["A_uq"], blk["A_ub"]
    Abq, Abu, Abb = blk["A_bq"], blk["A_bu"], blk["A_bb"]
    y1 = -Aub @ x + Auq @ (Qi @ (Aqb @ x))
    y2 = sla.lu_solve(rb["lu"], y1)
    y3 = Abu @ y2 - Abq @ (Qi @ (Aqu @ y2))
    y4 = y3 + (Abb @ x - Abq @ (Qi @ (Aqb @ x)))
    return y4


def backsolve_b(blk, rb, Qi, RQ, x):
    """Local recovery, eq. (Csc4a) for dU first, then (Csc4b) for dQ (the
    printed Algorithm 1 lists dQ before dU although dQ needs dU)."""
    dU = sla.lu_solve(rb["lu"], rb["f"] + rb["right"] @ x)
    dQ = Qi @ (-RQ - blk["A_qu"] @ dU - blk["A_qb"] @ x)
    return dQ, dU


def backsolve_a(blk, ra, RQ, RU, x):
    """Local recovery through A_local (eq. C46)."""
    rhs = -np.concatenate([RQ, RU]) - np.concatenate([blk["A_qb"], blk["A_ub"]], axis=0) @ x
    sol = sla.lu_solve(ra["lu"], rhs)
    nq = blk["A_qq"].shape[0]
    return sol[:nq], sol[nq:]
