"""Flow diagnostics of the Taylor-Green study (Sec. 5.3, eq. C5321).
Test infrastructure (oracle): plain numpy over the elements of each macro.

  E_k = (1 / |Omega|) int 1/2 rho |v|^2 dOmega            (volume-averaged kinetic energy)
  eps = 2 mu_eff / |Omega| int rho |omega|^2 / 2 dOmega   (eq. C5321), omega = curl v

with v = m / rho and the velocity gradient from q = grad u by the chain rule,
d_k v_j = (q_k[m_j] - v_j q_k[rho]) / rho.  In two dimensions omega is the
scalar d_x v_y - d_y v_x.  mu_eff = mu / Re_c is the viscosity of the
library's acoustic scaling (see physics.py).  Readings: the paper writes the
dynamic viscosity and keeps rho inside the integral (exact for incompressible
flow, approximate at low Mach number); the velocity gradient is that of the
method's gradient variable q, not the derivative of the u polynomial.  The
integrals use the element quadrature of the discretisation (Gauss-Legendre,
p + 2 points per direction).
"""
import numpy as np


def flow_diagnostics(S, q, u):
    """(E_k, eps, |Omega|) of the state (q, u) in the global layouts of
    system.py: u = [macro][comp][node], q = [macro][dir][comp][node]."""
    ph = S.ph
    mu_eff = ph.mu / ph.Re_c
    ke = ens = vol = 0.0
    for i in range(S.mesh.n_macros):
        mc = S.cls(i)
        d, ns, N = mc.dim, mc.ns, mc.N
        ui = u[S.u_off[i]:S.u_off[i + 1]].reshape(ns, N)
        qi = q[S.q_off[i]:S.q_off[i + 1]].reshape(d, ns, N)
        # values at the quadrature points of every element: [.., E, Q]
        uq = ui[:, mc.elem_nodes] @ mc.Phi.T
        qq = qi[:, :, mc.elem_nodes] @ mc.Phi.T
        rho = uq[0]
        v = uq[1:d + 1] / rho
        dv = [[(qq[k, j + 1] - v[j] * qq[k, 0]) / rho for k in range(d)] for j in range(d)]
        if d == 3:
            om2 = ((dv[2][1] - dv[1][2]) ** 2 + (dv[0][2] - dv[2][0]) ** 2 + (dv[1][0] - dv[0][1]) ** 2)
        else:
            om2 = (dv[1][0] - dv[0][1]) ** 2
        W = mc.W[None, :]
        ke += float(np.sum(W * 0.5 * rho * np.sum(v * v, axis=0)))
        ens += float(np.sum(W * 0.5 * rho * om2))
        vol += float(np.sum(np.broadcast_to(W, rho.shape)))
    return ke / vol, 2.0 * mu_eff * ens / vol, vol
