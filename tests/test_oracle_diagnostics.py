"""Pins of the oracle's flow diagnostics (Sec. 5.3, eq. C5321): exact
integrals of polynomial fields the discretisation represents exactly, and the
closed forms of the Taylor-Green initial field."""
import numpy as np
import pytest

from oracle.diagnostics import flow_diagnostics
from oracle.mesh import box_mesh
from oracle.physics import Phys
from oracle.system import System
from paper_2402_11361_amd.inputs import state_gradient, tgv_state


def _state(M, fn, **kw):
    X = [M.macro_node_coords(i) for i in range(M.n_macros)]
    u = np.concatenate([fn(x.T, **kw).reshape(-1) for x in X])
    q = np.concatenate([state_gradient(fn, x.T, **kw).reshape(-1) for x in X])
    return q, u


# rho = 1 + c x and a velocity whose momentum is of degree <= 2 per axis, on
# the unit box: p = 2 interpolates u and q exactly and the p + 2 point rule
# integrates rho |v|^2 and rho |omega|^2 exactly
A_, B_, C_, E_, F_ = 0.3, -0.7, 0.4, 0.2, 0.5


def _poly3(X):
    x, y, z = X
    rho = 1.0 + C_ * x
    v = [A_ * y + E_ * z, B_ * x, F_ * x]
    return np.stack([rho, rho * v[0], rho * v[1], rho * v[2], 2.0 + 0.0 * x])


def _poly2(X):
    x, y = X
    rho = 1.0 + C_ * x
    v = [A_ * y, B_ * x]
    return np.stack([rho, rho * v[0], rho * v[1], 2.0 + 0.0 * x])


def test_polynomial_field_3d_exact():
    M = box_mesh(3, 4, 2, 2, lo=0.0, hi=1.0, periodic=False)
    S = System(M, Phys(Re=100.0, Mach=0.1))
    q, u = _state(M, _poly3)
    ek, eps, vol = flow_diagnostics(S, q, u)
    mu = S.ph.mu / S.ph.Re_c
    # moments of the unit box: <y^2> = 1/3, <yz> = 1/4, <x y^2> = 1/6, <x yz> = 1/8, <x^3> = 1/4
    ek_ref = 0.5 * (A_ ** 2 / 3 + A_ * E_ / 2 + E_ ** 2 / 3 + (B_ ** 2 + F_ ** 2) / 3
                    + C_ * (A_ ** 2 / 6 + A_ * E_ / 4 + E_ ** 2 / 6 + (B_ ** 2 + F_ ** 2) / 4))
    # omega = (0, e - f, b - a) everywhere, weighted by <1 + c x> = 1 + c/2
    eps_ref = mu * ((E_ - F_) ** 2 + (B_ - A_) ** 2) * (1.0 + C_ / 2)
    assert abs(vol - 1.0) < 1e-14
    assert abs(ek - ek_ref) < 1e-13 * ek_ref
    assert abs(eps - eps_ref) < 1e-13 * eps_ref


def test_polynomial_field_2d_exact():
    M = box_mesh(2, 4, 2, 2, lo=0.0, hi=1.0, periodic=False)
    S = System(M, Phys(Re=50.0, Mach=0.2))
    q, u = _state(M, _poly2)
    ek, eps, vol = flow_diagnostics(S, q, u)
    mu = S.ph.mu / S.ph.Re_c
    ek_ref = 0.5 * (A_ ** 2 / 3 + B_ ** 2 / 3 + C_ * (A_ ** 2 / 6 + B_ ** 2 / 4))
    eps_ref = mu * (B_ - A_) ** 2 * (1.0 + C_ / 2)
    assert abs(vol - 1.0) < 1e-14
    assert abs(ek - ek_ref) < 1e-13 * ek_ref
    assert abs(eps - eps_ref) < 1e-13 * eps_ref


def _tgv(n, m, p, mach=0.1, Re=100.0):
    M = box_mesh(3, n, m, p, lo=-np.pi, hi=np.pi, periodic=True)
    S = System(M, Phys(Re=Re, Mach=mach))
    q, u = _state(M, tgv_state, mach=mach)
    ek, eps, vol = flow_diagnostics(S, q, u)
    mu, g, V0 = S.ph.mu / S.ph.Re_c, S.ph.gamma, mach
    # closed forms of the initial field with rho = gamma P: the density
    # variation drops out of <rho |v|^2> and lowers <rho |omega|^2> by
    # 5 gamma V0^2 / 64 against 3/4
    return ek, eps, vol, V0 ** 2 / 8.0, mu * V0 ** 2 * (0.75 - 5.0 * g * V0 ** 2 / 64.0), mu * V0 ** 2 * 0.75


def test_taylor_green_initial_closed_forms():
    ek, eps, vol, ek_ref, eps_ref, eps_rho1 = _tgv(8, 4, 3)
    assert abs(vol - (2 * np.pi) ** 3) < 1e-12 * vol
    e1, e2 = abs(ek - ek_ref) / ek_ref, abs(eps - eps_ref) / eps_ref
    assert e1 < 3e-5 and e2 < 3e-5, (e1, e2)
    # the density weighting is resolved: the constant-density value is off
    assert abs(eps - eps_rho1) / eps_ref > 30 * e2


@pytest.mark.parametrize("p", [2, 3])
def test_taylor_green_converges_under_refinement(p):
    r8 = _tgv(8, 4, p)
    r16 = _tgv(16, 4, p)
    for k, ref in ((0, 3), (1, 4)):
        err8 = abs(r8[k] - r8[ref]) / r8[ref]
        err16 = abs(r16[k] - r16[ref]) / r16[ref]
        assert err16 < err8 / 10, (p, k, err8, err16)
