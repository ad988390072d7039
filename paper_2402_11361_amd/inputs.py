"""Seeded synthetic inputs: flow states evaluated at caller-supplied points,
and seeded noise.  Shared by the tests, the smoke check and the benchmark.
Holds none of the discretisation's arithmetic: only the initial fields of the
paper's workloads (Taylor-Green vortex, eq. TGV0; a linear shear layer) in
conserved variables (rho, rho v, rho E) with gamma P = rho T, and their exact
gradients by a complex-step derivative of those fields.
"""
import numpy as np

GAMMA = 1.4


def _conserved(rho, v, P, gamma=GAMMA):
    ke = 0.5 * rho * sum(vk * vk for vk in v)
    return np.stack([rho] + [rho * vk for vk in v] + [P / (gamma - 1.0) + ke])


def tgv_state(X, mach=0.1, gamma=GAMMA):
    """Taylor-Green vortex at t = 0 (L = 1, rho0 = 1, P0 = 1/gamma, V0 = mach,
    isothermal P/rho = P0/rho0).  X [d, ...] -> u [d+2, ...]."""
    d = X.shape[0]
    V0, P0 = mach, 1.0 / gamma
    x, y = X[0], X[1]
    if d == 3:
        z = X[2]
        v = [V0 * np.sin(x) * np.cos(y) * np.cos(z), -V0 * np.cos(x) * np.sin(y) * np.cos(z), 0.0 * x]
        P = P0 + V0 * V0 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    else:
        v = [V0 * np.sin(x) * np.cos(y), -V0 * np.cos(x) * np.sin(y)]
        P = P0 + V0 * V0 / 4.0 * (np.cos(2 * x) + np.cos(2 * y))
    rho = P / P0
    return _conserved(rho, v, P, gamma)


def shear_state(X, mach=0.2, gamma=GAMMA):
    """Linear shear: rho = 1, v = (mach * y, 0[, 0]), T = 1 (P = 1/gamma)."""
    d = X.shape[0]
    v = [mach * X[1]] + [0.0 * X[0]] * (d - 1)
    return _conserved(1.0 + 0.0 * X[0], v, 1.0 / gamma + 0.0 * X[0], gamma)


def state_gradient(fn, X, **kw):
    """q[k] = d u / d x_k of a field function, by complex step (exact)."""
    d = X.shape[0]
    out = []
    for k in range(d):
        Xc = X.astype(complex)
        Xc[k] = Xc[k] + 1e-30j
        out.append(fn(Xc, **kw).imag / 1e-30)
    return np.stack(out)


def noise(seed, shape, amp):
    """Uniform U(-amp, amp) noise from numpy's PCG64 generator."""
    rng = np.random.default_rng(seed)
    return amp * rng.uniform(-1.0, 1.0, size=shape)


# Workloads (mesh, physics, solver tolerance), named by state, mesh, macro size and degree.
CONFIGS = {
    "shear16_m4_p2": dict(dim=2, n_elem=16, m=4, p=2, lo=0.0, hi=1.0, periodic=False, state="shear",
               mach=0.2, Re=100.0, noise=1e-3, rtol=1e-10),
    "tgv24_m3_p2": dict(dim=3, n_elem=24, m=3, p=2, lo=-np.pi, hi=np.pi, periodic=True, state="tgv",
               mach=0.1, Re=1600.0, noise=1e-4, rtol=1e-8),
    "tgv32_m4_p3": dict(dim=3, n_elem=32, m=4, p=3, lo=-np.pi, hi=np.pi, periodic=True, state="tgv",
               mach=0.1, Re=1600.0, noise=1e-4, rtol=1e-8),
    "tgv48_m4_p2": dict(dim=3, n_elem=48, m=4, p=2, lo=-np.pi, hi=np.pi, periodic=True, state="tgv",
               mach=0.1, Re=1600.0, noise=1e-4, rtol=1e-8),
    # the Re = 100 Taylor-Green run of the m-versus-p comparison (Sec. 5.3):
    # 6 macros per axis and m p = 6, so both have N_eff = (6 (m p + 1))^3 = 42^3
    # and the same n_u and n_b per macro; clean initial field
    "tgv_re100_m3_p2": dict(dim=3, n_elem=18, m=3, p=2, lo=-np.pi, hi=np.pi, periodic=True, state="tgv",
               mach=0.1, Re=100.0, noise=0.0, rtol=1e-8),
    "tgv_re100_m2_p3": dict(dim=3, n_elem=12, m=2, p=3, lo=-np.pi, hi=np.pi, periodic=True, state="tgv",
               mach=0.1, Re=100.0, noise=0.0, rtol=1e-8),
    # macros of uneven sizes: every axis of the 32^3 mesh cut into seeded
    # segments of 2, 3 or 4 elements (one degree for the whole mesh)
    "tgv32_uneven_p2": dict(dim=3, n_elem=32, m=None, parts=(2, 3, 4), seg_seed=3, p=2, lo=-np.pi, hi=np.pi, periodic=True,
               state="tgv", mach=0.1, Re=1600.0, noise=1e-4, rtol=1e-8),
}


def random_segments(n, parts, seed):
    """Seeded cut of n elements into consecutive segments whose lengths are
    drawn uniformly from `parts` among the choices that leave a remainder
    that can still be cut (the last piece closes exactly)."""
    rng = np.random.default_rng(seed)
    out, left = [], n
    small = min(parts)

    def ok(r):
        return r == 0 or any(r - x == 0 or (r - x >= small and ok_cache(r - x)) for x in parts)

    memo = {}

    def ok_cache(r):
        if r not in memo:
            memo[r] = ok(r)
        return memo[r]

    while left > 0:
        choices = [x for x in parts if x <= left and ok_cache(left - x)]
        x = int(rng.choice(choices))
        out.append(x)
        left -= x
    return out


def segments(cfg):
    """Per-axis segment lengths of a workload (uniform m, or seeded parts)."""
    d, n = cfg["dim"], cfg["n_elem"]
    if cfg.get("m"):
        return [[cfg["m"]] * (n // cfg["m"]) for _ in range(d)]
    return [random_segments(n, cfg["parts"], cfg["seg_seed"] + k) for k in range(d)]


def cfl_dt(cfg, cfl=1.0):
    """Time step dt = CFL h / (V0 (p + 1)) (Sec. 5.3)."""
    h = (cfg["hi"] - cfg["lo"]) / cfg["n_elem"]
    return cfl * h / (cfg["mach"] * (cfg["p"] + 1))


def make_state(cfg, macro_coords, face_coords, q_seed_offset=1000, seed=0):
    """Nodal u (list per macro, [ns, N] flattened), q (gradient + noise) and
    trace u-hat (state + independent noise) for a workload.

    macro_coords: list of [N_i, d] node coordinates per macro; face_coords:
    list of [n_f, d] trace-node coordinates per face.  Returns flat arrays
    (u, q, uhat) in the library's layouts."""
    fn = tgv_state if cfg["state"] == "tgv" else shear_state
    kw = dict(mach=cfg["mach"])
    u = np.concatenate([fn(X.T, **kw).reshape(-1) for X in macro_coords])
    q = np.concatenate([state_gradient(fn, X.T, **kw).reshape(-1) for X in macro_coords])
    uh = np.concatenate([fn(X.T, **kw).reshape(-1) for X in face_coords])
    a = cfg["noise"]
    u = u + noise(seed, u.shape, a)
    uh = uh + noise(seed + 1, uh.shape, a)
    q = q + noise(seed + q_seed_offset, q.shape, a)
    return u, q, uh


def exact_trace(cfg, face_coords):
    fn = tgv_state if cfg["state"] == "tgv" else shear_state
    return np.concatenate([fn(X.T, mach=cfg["mach"]).reshape(-1) for X in face_coords])
