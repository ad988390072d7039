"""Learned coarse correction for the FGMRES preconditioner: plain FP64
definitions of the coarse restriction and prolongation, the two-layer network,
its loss and gradients, and the Adam update.  Test infrastructure (oracle).

The paper has no learned component; FGMRES (Sec. 4.2) accepts a
preconditioner that changes from step to step, which is what admits this
stage.  Definitions used here:

* Coarse restriction R_c: for every macro and each of its 2d faces and n_s
  components, the discrete L2 projection of the face field onto the
  multilinear functions of the face's tangential coordinates (2 functions in
  2D, 4 in 3D), with the tangential coordinates scaled to [0, 1] over the
  face and the composite Gauss-Lobatto quadrature of the face nodes as inner
  product.  Feature order: [local face][component][coarse function], i.e.
  2d * n_s * 2^(d-1) features per macro (120 in 3D, 32 in 2D).
* Coarse prolongation P_c: the coarse functions evaluated at the face nodes;
  a face receives the mean over the macros that own it (two, or one on the
  domain boundary).
* Neighbour features: a macro's coefficients followed by those of the macro
  across each local face (zeros on the domain boundary), (1 + 2d) times the
  per-macro count, as an input that reaches beyond the macro.
* Network: y = W2 tanh(W1 x~ + b1) + b2 applied to x~ = x / ||x||_2 and
  rescaled by ||x||_2 (homogeneous of degree one in x); x = 0 maps to 0.
* Loss on a batch (x_b, t_b): mean over the batch and the outputs of
  (W2 tanh(W1 x~_b + b1) + b2 - t~_b)^2 with t~_b = t_b / ||x_b||, i.e. in
  normalised units; a row with x_b = 0 (which the network maps to 0 whatever
  its weights) is normalised to x~_b = 0 and t~_b = 0.
* Adam (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
  p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
import numpy as np
from numpy.polynomial import legendre as L

from .basis import gll_nodes


def gll_weights(p):
    """Weights of the (p+1)-point Gauss-Lobatto rule on [-1, 1]:
    2 / (p (p+1) P_p(x_j)^2)."""
    x = gll_nodes(p)
    c = np.zeros(p + 1)
    c[p] = 1.0
    return 2.0 / (p * (p + 1) * L.legval(x, c) ** 2)


def composite_1d(m, p):
    """Node positions in [0, 1] and composite GLL weights of m elements of
    degree p (shared end nodes get the sum of both weights)."""
    x = gll_nodes(p)
    w = gll_weights(p)
    n = m * p + 1
    pos = np.zeros(n)
    wt = np.zeros(n)
    for e in range(m):
        for a in range(p + 1):
            pos[e * p + a] = (e + (x[a] + 1.0) / 2.0) / m
            wt[e * p + a] += w[a] / (2.0 * m)
    return pos, wt


def coarse_basis(tn_m, p):
    """(Phi [n_nodes, 2^(d-1)], weights [n_nodes]) on a face whose tangential
    axes carry tn_m elements (lower axis fastest in the node order)."""
    if len(tn_m) == 1:
        s, ws = composite_1d(tn_m[0], p)
        Phi = np.stack([1.0 - s, s], axis=1)
        return Phi, ws
    s, ws = composite_1d(tn_m[0], p)
    t, wt = composite_1d(tn_m[1], p)
    S = np.tile(s, len(t))
    T = np.repeat(t, len(s))
    W = np.tile(ws, len(t)) * np.repeat(wt, len(s))
    Phi = np.stack([(1 - S) * (1 - T), S * (1 - T), (1 - S) * T, S * T], axis=1)
    return Phi, W


def _face_ops(mesh, f):
    fc = mesh.faces[f]
    deg = fc["deg"]  # the face's trace degree (the mesh degree unless degrees are mixed)
    tn_m = [(n - 1) // deg for n in fc["tn"]]
    return coarse_basis(tn_m, deg)


def n_features(dim):
    return 2 * dim * (dim + 2) * 2 ** (dim - 1)


def coarse_restrict(mesh, v):
    """X [n_macros, n_features] = R_c v."""
    d, ns = mesh.dim, mesh.ns
    nq = 2 ** (d - 1)
    X = np.zeros((mesh.n_macros, n_features(d)))
    for i in range(mesh.n_macros):
        for lf in range(2 * d):
            f = mesh.macro_faces[i, lf]
            Phi, W = _face_ops(mesh, f)
            G = Phi.T @ (W[:, None] * Phi)
            nn = Phi.shape[0]
            seg = v[mesh.face_offset[f]:mesh.face_offset[f] + ns * nn].reshape(ns, nn)
            coef = np.linalg.solve(G, (Phi * W[:, None]).T @ seg.T)  # [nq, ns]
            X[i, (lf * ns) * nq:(lf * ns + ns) * nq] = coef.T.reshape(-1)
    return X


def coarse_prolong(mesh, Y):
    """z [n_glob] = P_c Y (mean over the macros that own each face)."""
    d, ns = mesh.dim, mesh.ns
    nq = 2 ** (d - 1)
    z = np.zeros(mesh.n_glob)
    for f in range(mesh.n_faces):
        fc = mesh.faces[f]
        Phi, _ = _face_ops(mesh, f)
        sides = []
        if fc["minus"] >= 0:
            sides.append((fc["minus"], 2 * fc["axis"] + 1))
        if fc["plus"] >= 0:
            sides.append((fc["plus"], 2 * fc["axis"]))
        acc = np.zeros((ns, Phi.shape[0]))
        for i, lf in sides:
            coef = Y[i, (lf * ns) * nq:(lf * ns + ns) * nq].reshape(ns, nq)
            acc += coef @ Phi.T
        acc /= len(sides)
        z[mesh.face_offset[f]:mesh.face_offset[f] + ns * Phi.shape[0]] = acc.reshape(-1)
    return z


def neighbour_of(mesh, i, lf):
    """The macro across local face lf of macro i, or -1 on the domain boundary."""
    fc = mesh.faces[mesh.macro_faces[i, lf]]
    return fc["plus"] if lf % 2 == 1 else fc["minus"]


def neighbour_features(mesh, X):
    """Xe [n_macros, (1 + 2d) n_features]: a macro's own coarse coefficients,
    then those of the macro across each of its local faces in order (zeros
    where the face is on the domain boundary), so that the network sees the
    coarse state of the face neighbours as well."""
    d = mesh.dim
    F = X.shape[1]
    Xe = np.zeros((mesh.n_macros, (1 + 2 * d) * F))
    for i in range(mesh.n_macros):
        Xe[i, :F] = X[i]
        for lf in range(2 * d):
            j = neighbour_of(mesh, i, lf)
            if j >= 0:
                Xe[i, (1 + lf) * F:(2 + lf) * F] = X[j]
    return Xe


# ---- network ---------------------------------------------------------------

def init_params(n_in, n_hidden, n_out, rng):
    """Glorot-uniform weights, zero biases."""
    a1 = np.sqrt(6.0 / (n_in + n_hidden))
    a2 = np.sqrt(6.0 / (n_hidden + n_out))
    return dict(W1=rng.uniform(-a1, a1, (n_hidden, n_in)), b1=np.zeros(n_hidden),
                W2=rng.uniform(-a2, a2, (n_out, n_hidden)), b2=np.zeros(n_out))


def _norms(X):
    return np.sqrt(np.sum(X * X, axis=1))


def forward(P, X):
    """Network output in physical units: ||x|| (W2 tanh(W1 x/||x|| + b1) + b2)."""
    s = _norms(X)
    safe = np.where(s > 0, s, 1.0)
    H = np.tanh((X / safe[:, None]) @ P["W1"].T + P["b1"])
    Y = H @ P["W2"].T + P["b2"]
    return np.where(s[:, None] > 0, Y * s[:, None], 0.0)


def loss_and_grads(P, X, T):
    """Mean squared error in normalised units and its gradient (plain chain
    rule through the two layers)."""
    s = _norms(X)
    inv = np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0)
    Xn = X * inv[:, None]
    Tn = T * inv[:, None]
    Z = Xn @ P["W1"].T + P["b1"]
    H = np.tanh(Z)
    Y = H @ P["W2"].T + P["b2"]
    R = Y - Tn
    B, n_out = R.shape
    loss = float(np.sum(R * R) / (B * n_out))
    dY = 2.0 * R / (B * n_out)
    g = dict(W2=dY.T @ H, b2=dY.sum(axis=0))
    dZ = (dY @ P["W2"]) * (1.0 - H * H)
    g["W1"] = dZ.T @ Xn
    g["b1"] = dZ.sum(axis=0)
    return loss, g


def adam_step(P, G, M, V, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place (t counts from 1)."""
    for k in P:
        M[k] = beta1 * M[k] + (1.0 - beta1) * G[k]
        V[k] = beta2 * V[k] + (1.0 - beta2) * G[k] ** 2
        mh = M[k] / (1.0 - beta1 ** t)
        vh = V[k] / (1.0 - beta2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)


def flat(P):
    """Parameters in the order W1 [h][in], b1 [h], W2 [out][h], b2 [out]."""
    return np.concatenate([P["W1"].ravel(), P["b1"], P["W2"].ravel(), P["b2"]])


def unflat(v, n_in, n_hidden, n_out):
    o = 0
    W1 = v[o:o + n_hidden * n_in].reshape(n_hidden, n_in); o += n_hidden * n_in
    b1 = v[o:o + n_hidden]; o += n_hidden
    W2 = v[o:o + n_out * n_hidden].reshape(n_out, n_hidden); o += n_out * n_hidden
    b2 = v[o:o + n_out]
    return dict(W1=W1.copy(), b1=b1.copy(), W2=W2.copy(), b2=b2.copy())
