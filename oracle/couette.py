"""Compressible Couette flow with a source (Sec. 5.1, eq. CF0 and the source
that follows it).  Test infrastructure (oracle).

Reading (the printed temperature and source are garbled and free-stream
scaled): in acoustic units v_1 = M x_2 log(1 + x_2), other velocities 0,
P = 1/gamma, T = alpha + x_2 (beta - alpha) + (gamma-1)/(2 gamma) Pr x_2 (1-x_2),
rho = gamma P / T, alpha = 0.8, beta = 0.85.  The source is
s = div(F + G) of the exact fields, evaluated by a complex-step derivative in
x_2 of the exact fluxes (the exact gradients are written out by hand).  Its
x_1-momentum entry equals -(mu M / Re_c) (2 + x_2)/(1 + x_2)^2, the printed
entry with the acoustic scaling factor.
"""
import numpy as np
from . import physics as phy

ALPHA, BETA = 0.8, 0.85


def _fields(x2, ph):
    g, Pr, M = ph.gamma, ph.Pr, ph.Mach
    cT = (g - 1.0) / (2.0 * g) * Pr
    T = ALPHA + x2 * (BETA - ALPHA) + cT * x2 * (1.0 - x2)
    dT = (BETA - ALPHA) + cT * (1.0 - 2.0 * x2)
    P = 1.0 / g
    rho = g * P / T
    drho = -g * P * dT / T ** 2
    v1 = M * x2 * np.log(1.0 + x2)
    dv1 = M * (np.log(1.0 + x2) + x2 / (1.0 + x2))
    rE = P / (g - 1.0) + 0.5 * rho * v1 * v1
    drE = 0.5 * drho * v1 * v1 + rho * v1 * dv1
    return rho, drho, v1, dv1, rE, drE


def exact_u(X, ph):
    """Conserved state at points X [d, ...] (components on axis 0)."""
    d = X.shape[0]
    rho, _, v1, _, rE, _ = _fields(X[1], ph)
    z = np.zeros_like(rho)
    comps = [rho, rho * v1] + [z] * (d - 1) + [rE]
    return np.stack(comps)


def exact_q(X, ph):
    """grad u, q[k] = d_k u, shape [d, ns, ...]."""
    d = X.shape[0]
    rho, drho, v1, dv1, rE, drE = _fields(X[1], ph)
    z = np.zeros_like(rho)
    q = np.zeros((d, d + 2) + rho.shape, dtype=np.result_type(rho, 1.0))
    q[1] = np.stack([drho, drho * v1 + rho * dv1] + [z] * (d - 1) + [drE])
    return q


def source(X, ph):
    """s = sum_k d_k (F_k + G_k) of the exact solution at points X [d, ...]."""
    h = 1e-30
    Xc = X.astype(complex)
    Xc[1] = Xc[1] + 1j * h
    u = exact_u(Xc, ph)
    q = exact_q(Xc, ph)
    F = phy.flux_inviscid(u, ph)
    G = phy.flux_viscous(u, q, ph)
    return (F[1] + G[1]).imag / h


def l2_errors(S, u, ph):
    """L2(Omega) errors of rho, v_1 and rhoE of the nodal state u against the
    exact solution, with the element quadrature."""
    err = np.zeros(3)
    for i in range(S.mesh.n_macros):
        mc = S.cls(i)
        ui = u[S.u_off[i]:S.u_off[i + 1]].reshape(mc.ns, mc.N)
        org = S.origin(i)
        for e in range(mc.E):
            uq = mc.Phi @ ui[:, mc.elem_nodes[e]].T                      # [Q, ns]
            xq = org[None, :] + (mc.eidx[e][None, :] + mc.xq_ref) * np.array(mc.h)
            ue = exact_u(xq.T, ph).T
            dv = uq[:, 1] / uq[:, 0] - ue[:, 1] / ue[:, 0]
            err += np.array([mc.W @ (uq[:, 0] - ue[:, 0]) ** 2, mc.W @ dv ** 2,
                             mc.W @ (uq[:, -1] - ue[:, -1]) ** 2])
    return np.sqrt(err)
