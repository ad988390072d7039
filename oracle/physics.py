"""Compressible Navier-Stokes fluxes in the compact form of eq. (C4)-(C6).
Test infrastructure (oracle).  All functions are complex-safe (used with the
complex-step derivative) except those documented as frozen coefficients.

Reading of the nondimensionalisation (the paper mixes acoustic and
free-stream scalings, Sec. 2.1): acoustic scaling throughout, rho_inf = 1,
c_inf = 1, mu = 1,
    P   = (gamma-1) (rhoE - |m|^2 / (2 rho)),     gamma P = rho T,
    tau = (1/Re_c) (grad v + grad v^T - (2/d) div v I)     (lambda = -2/d),
    phi = -(1 / (Re_c Pr (gamma-1))) grad T,
with Re_c = Re / M_inf the acoustic Reynolds number.
u = (rho, m_1..m_d, rhoE), components on axis 0; q = grad u with q[k] = d_k u.
"""
import numpy as np


class Phys:
    def __init__(self, gamma=1.4, Pr=0.71, Re=100.0, Mach=0.1, mu=1.0):
        self.gamma = float(gamma)
        self.Pr = float(Pr)
        self.Re = float(Re)
        self.Mach = float(Mach)
        self.mu = float(mu)
        self.Re_c = self.Re / self.Mach

    @property
    def kappa_eff(self):
        """Heat-flux coefficient mu / (Re_c Pr (gamma-1))."""
        return self.mu / (self.Re_c * self.Pr * (self.gamma - 1.0))


def primitives(u, ph):
    d = u.shape[0] - 2
    rho = u[0]
    v = u[1:d + 1] / rho
    E = u[d + 1] / rho
    P = (ph.gamma - 1.0) * (u[d + 1] - 0.5 * rho * sum(v[j] * v[j] for j in range(d)))
    return rho, v, E, P


def flux_inviscid(u, ph):
    """F[k, c] = k-th column of F(u) = [rho v, rho v (x) v + P I, rho v H], eq. (C5)."""
    d = u.shape[0] - 2
    rho, v, E, P = primitives(u, ph)
    F = np.zeros((d, d + 2) + u.shape[1:], dtype=np.result_type(u, 1.0))
    for k in range(d):
        F[k, 0] = u[k + 1]
        for j in range(d):
            F[k, j + 1] = u[j + 1] * v[k] + (P if j == k else 0.0)
        F[k, d + 1] = (u[d + 1] + P) * v[k]
    return F


def flux_viscous(u, q, ph):
    """G[k, c] = -[0, tau_{.k}, (tau v)_k - phi_k], eq. (C5)/(C6), with gradients
    of primitives obtained from q = grad u by the chain rule."""
    d = u.shape[0] - 2
    rho, v, E, P = primitives(u, ph)
    # gradients: dv[j][k] = d_k v_j, dE[k], dT[k]
    dv = [[(q[k, j + 1] - v[j] * q[k, 0]) / rho for k in range(d)] for j in range(d)]
    dE = [(q[k, d + 1] - E * q[k, 0]) / rho for k in range(d)]
    g = ph.gamma
    dT = [g * (g - 1.0) * (dE[k] - sum(v[j] * dv[j][k] for j in range(d))) for k in range(d)]
    div = sum(dv[j][j] for j in range(d))
    lam = -2.0 / d
    c_mu = ph.mu / ph.Re_c
    tau = [[c_mu * (dv[j][k] + dv[k][j] + (lam * div if j == k else 0.0)) for k in range(d)]
           for j in range(d)]
    G = np.zeros((d, d + 2) + u.shape[1:], dtype=np.result_type(u, q, 1.0))
    kap = ph.kappa_eff
    for k in range(d):
        for j in range(d):
            G[k, j + 1] = -tau[j][k]
        # -( (tau v)_k - phi_k ) with phi = -kap grad T
        G[k, d + 1] = -(sum(tau[k][j] * v[j] for j in range(d)) + kap * dT[k])
    return G


def lambda_max(uh, n, ph):
    """Largest |eigenvalue| of d(F.n)/du at the trace state: |v.n| + c.
    Frozen coefficient: evaluated on the real part only."""
    uh = np.real(uh)
    d = uh.shape[0] - 2
    rho, v, E, P = primitives(uh, ph)
    vn = sum(v[k] * n[k] for k in range(d))
    c = np.sqrt(ph.gamma * P / rho)
    return np.abs(vn) + c


def s_vis_diag(d, ph):
    """Viscous stabilisation S_vis = (1/Re_c) diag(0, 1..1, 1/((gamma-1) Pr)).
    Reading of the printed S_vis (free-stream scaled) in acoustic scaling;
    parity unpinned against the paper (any positive S is consistent)."""
    s = np.zeros(d + 2)
    s[1:d + 1] = 1.0 / ph.Re_c
    s[d + 1] = 1.0 / (ph.Re_c * (ph.gamma - 1.0) * ph.Pr)
    return s


def inviscid_jacobian(u_real, ph):
    """A_k = dF_k/du at a real state (complex step on a real input), shape
    [d, ns, ns, ...].  Used only as a frozen SUPG coefficient."""
    u_real = np.real(u_real).astype(float)
    ns = u_real.shape[0]
    d = ns - 2
    h = 1e-30
    A = np.zeros((d, ns, ns) + u_real.shape[1:])
    for c in range(ns):
        up = u_real.astype(complex)
        up[c] = up[c] + 1j * h
        F = flux_inviscid(up, ph)
        A[:, :, c] = F.imag / h
    return A
