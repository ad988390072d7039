"""1D reference element: Gauss-Lobatto-Legendre nodes, Gauss-Legendre rule,
Lagrange basis.  Test infrastructure (oracle).

The paper (Sec. 2.2, finite element spaces) uses degree-p Lagrange polynomials
but names no nodal set and no quadrature.  Readings used here:
  * nodes: the p+1 Gauss-Lobatto-Legendre points on [-1, 1];
  * quadrature: Gauss-Legendre with p+2 points per direction.
"""
import numpy as np
from numpy.polynomial import legendre as L


def gll_nodes(p):
    """GLL points: -1, the roots of P_p'(x), +1 (ascending)."""
    if p < 1:
        raise ValueError("p >= 1 required")
    cP = np.zeros(p + 1)
    cP[p] = 1.0
    inner = L.legroots(L.legder(cP)) if p > 1 else np.zeros(0)
    x = np.concatenate([[-1.0], np.sort(inner.real), [1.0]])
    # polish interior roots of P_p' with Newton steps
    d1 = L.legder(cP)
    d2 = L.legder(cP, 2)
    for _ in range(4):
        xi = x[1:-1]
        if xi.size:
            x[1:-1] = xi - L.legval(xi, d1) / L.legval(xi, d2)
    return x


def gauss_rule(n):
    """n-point Gauss-Legendre rule on [-1, 1]."""
    return L.leggauss(n)


def lagrange(nodes, x):
    """Values V[i, j] = l_j(x_i) and derivatives D[i, j] = l_j'(x_i) of the
    Lagrange polynomials through `nodes`, at points `x` (plain product form)."""
    nodes = np.asarray(nodes, dtype=float)
    x = np.atleast_1d(np.asarray(x, dtype=float))
    n = nodes.size
    V = np.ones((x.size, n))
    D = np.zeros((x.size, n))
    for j in range(n):
        den = 1.0
        for m in range(n):
            if m != j:
                den *= nodes[j] - nodes[m]
        for i, xi in enumerate(x):
            prod = 1.0
            for m in range(n):
                if m != j:
                    prod *= xi - nodes[m]
            V[i, j] = prod / den
            s = 0.0
            for l in range(n):
                if l == j:
                    continue
                t = 1.0
                for m in range(n):
                    if m != j and m != l:
                        t *= xi - nodes[m]
                s += t
            D[i, j] = s / den
    return V, D
