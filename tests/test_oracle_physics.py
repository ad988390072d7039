"""Pins of the oracle's flux functions (eq. C5/C6) against mathematics and the
paper's nondimensionalisation (Sec. 2.1 scaling table)."""
import numpy as np
import pytest
from oracle import physics as phy

RNG = np.random.default_rng(1234)


def _state(d, rng):
    rho = 1.0 + 0.3 * rng.random()
    v = 0.3 * (rng.random(d) - 0.5)
    P = 0.7 + 0.2 * rng.random()
    u = np.zeros(d + 2)
    u[0] = rho
    u[1:d + 1] = rho * v
    u[d + 1] = P / 0.4 + 0.5 * rho * v @ v
    return u, rho, v, P


@pytest.mark.parametrize("d", [2, 3])
def test_inviscid_jacobian_eigenvalues(d):
    ph = phy.Phys()
    u, rho, v, P = _state(d, RNG)
    A = phy.inviscid_jacobian(u, ph)
    n = RNG.standard_normal(d); n /= np.linalg.norm(n)
    An = sum(A[k] * n[k] for k in range(d))
    ev = np.sort(np.linalg.eigvals(An).real)
    c = np.sqrt(1.4 * P / rho)
    vn = v @ n
    assert np.allclose(ev, np.sort([vn - c] + [vn] * d + [vn + c]), atol=1e-12)
    lam = phy.lambda_max(u, n, ph)
    assert abs(lam - (abs(vn) + c)) < 1e-14


@pytest.mark.parametrize("d", [2, 3])
def test_euler_flux_homogeneity(d):
    """F_k(u) = (dF_k/du) u (Euler fluxes are homogeneous of degree one)."""
    ph = phy.Phys()
    u, *_ = _state(d, RNG)
    A = phy.inviscid_jacobian(u, ph)
    F = phy.flux_inviscid(u, ph)
    for k in range(d):
        assert np.allclose(A[k] @ u, F[k], atol=1e-13)


def _grad_state(d, rng, v_grad):
    u, rho, v, P = _state(d, rng)
    # q = grad u for fields with the given velocity gradient, constant rho, P
    q = np.zeros((d, d + 2))
    for k in range(d):
        q[k, 1:d + 1] = rho * v_grad[:, k]
        q[k, d + 1] = rho * (v @ v_grad[:, k])
    return u, q, rho, v


@pytest.mark.parametrize("d", [2, 3])
def test_viscous_stress_invariants(d):
    ph = phy.Phys(Re=50.0, Mach=0.2)
    # rigid rotation: antisymmetric velocity gradient -> no viscous stress
    Wm = RNG.standard_normal((d, d)); Wm = Wm - Wm.T
    u, q, rho, v = _grad_state(d, RNG, Wm)
    G = phy.flux_viscous(u, q, ph)
    assert np.allclose(G[:, 1:d + 1], 0.0, atol=1e-15)
    # uniform dilation: trace-free stress (Stokes, lambda = -2/d) -> zero
    u, q, rho, v = _grad_state(d, RNG, 0.7 * np.eye(d))
    G = phy.flux_viscous(u, q, ph)
    assert np.allclose(G[:, 1:d + 1], 0.0, atol=1e-15)
    # simple shear dv1/dx2 = s: tau_12 = mu s / Re_c and G_{2, mom1} = -tau_12
    s = 0.37
    Lg = np.zeros((d, d)); Lg[0, 1] = s
    u, q, rho, v = _grad_state(d, RNG, Lg)
    G = phy.flux_viscous(u, q, ph)
    assert abs(G[1, 1] + ph.mu * s / ph.Re_c) < 1e-15
    assert abs(G[0, 2] + ph.mu * s / ph.Re_c) < 1e-15


@pytest.mark.parametrize("d", [2, 3])
def test_viscous_flux_matches_dimensional_physics(d):
    """Dimensional stress and Fourier heat flux (eq. with tau*, phi*), scaled by
    the paper's reference quantities, equal the nondimensional G (reading of
    the acoustic scaling)."""
    gamma, Rg, T_inf, rho_inf, X0, mu_inf, Pr = 1.4, 287.0, 300.0, 1.2, 2.0, 1.8e-5, 0.71
    c_inf = np.sqrt(gamma * Rg * T_inf)
    cp = gamma * Rg / (gamma - 1.0)
    cv = Rg / (gamma - 1.0)
    kappa = cp * mu_inf / Pr
    Re_c = rho_inf * c_inf * X0 / mu_inf
    Mach = 0.3
    ph = phy.Phys(gamma=gamma, Pr=Pr, Re=Re_c * Mach, Mach=Mach)
    rng = np.random.default_rng(7)
    x0 = rng.random(d)
    g_rho, g_T = rng.standard_normal(d) * 0.1, rng.standard_normal(d) * 5.0
    g_v = rng.standard_normal((d, d)) * 20.0
    rho0, T0, v0 = 1.1, 310.0, rng.standard_normal(d) * 30.0

    def dim_fields(x):  # linear dimensional fields around x0
        dx = x - x0
        rho = rho0 + g_rho @ dx
        v = v0 + g_v @ dx
        T = T0 + g_T @ dx
        return rho, v, T

    def nondim_u(xs):  # xs = nondimensional coordinates (complex allowed)
        rho, v, T = dim_fields(xs * X0)
        E = cv * T + 0.5 * (v @ v)
        return np.concatenate([[rho / rho_inf], rho * v / (rho_inf * c_inf), [rho * E / (rho_inf * c_inf ** 2)]])

    xs0 = x0 / X0
    u = nondim_u(xs0.astype(complex)).real
    q = np.zeros((d, d + 2))
    for k in range(d):
        xc = xs0.astype(complex); xc[k] += 1e-30j
        q[k] = nondim_u(xc).imag / 1e-30
    G = phy.flux_viscous(u, q, ph)
    rho, v, T = dim_fields(x0)
    tau = mu_inf * (g_v + g_v.T - (2.0 / d) * np.trace(g_v) * np.eye(d))
    phi = -kappa * g_T
    for k in range(d):
        assert np.allclose(G[k, 1:d + 1], -tau[:, k] / (rho_inf * c_inf ** 2), rtol=1e-10, atol=1e-14)
        assert np.isclose(G[k, d + 1], -(tau[k] @ v - phi[k]) / (rho_inf * c_inf ** 3), rtol=1e-10)
    # equation of state: gamma P = rho T in nondimensional variables
    rho_, v_, E_, P_ = phy.primitives(u, ph)
    assert np.isclose(gamma * P_, rho_ * (T / T_inf), rtol=1e-12)
