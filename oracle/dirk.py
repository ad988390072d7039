"""Time integration (Sec. 2.4): the three-stage L-stable SDIRK of Alexander,
the stage history of eq. (C242) and the update of eq. (C241).  Test
infrastructure (oracle).

The paper names DIRK(3,3) but prints no coefficients.  Reading: Alexander's
method with alpha the root in (0, 1) of 6a^3 - 18a^2 + 9a - 1 = 0, i.e.
alpha = 0.4358665215..., c = (alpha, (1+alpha)/2, 1), a21 = (1-alpha)/2,
b = (a31, a32, a33) = (-(6a^2-16a+1)/4, (6a^2-20a+5)/4, alpha); stiffly
accurate (c_s = 1) as the remark after eq. (C243) requires.
The printed update (C241) is garbled; read as
u^{n+1} = (1 - sum_j e_j) u^n + sum_j e_j u^{n,j}, e_j = sum_i b_i d_ij,
which for a stiffly accurate method gives u^{n+1} = u^{n,s}.
"""
import numpy as np


def alexander_alpha():
    # bisection on 6a^3 - 18a^2 + 9a - 1 in the bracket [0.4, 0.5]
    f = lambda a: 6 * a ** 3 - 18 * a ** 2 + 9 * a - 1
    lo, hi = 0.4, 0.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(lo) * f(mid) <= 0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def dirk33():
    a = alexander_alpha()
    A = np.array([[a, 0.0, 0.0],
                  [(1 - a) / 2, a, 0.0],
                  [-(6 * a * a - 16 * a + 1) / 4, (6 * a * a - 20 * a + 5) / 4, a]])
    b = A[2].copy()
    c = A.sum(axis=1)
    return A, b, c


def stage_history(Ainv, i, u_n, stages):
    """w of the discrete time derivative (d_ii u + w)/dt for stage i (eq. C242):
    w = sum_{j<i} d_ij (u^{n,j} - u^n) - d_ii u^n."""
    w = -Ainv[i, i] * u_n
    for j in range(i):
        w = w + Ainv[i, j] * (stages[j] - u_n)
    return w


def update(Ainv, b, u_n, stages):
    e = b @ Ainv
    return (1.0 - e.sum()) * u_n + sum(e[j] * stages[j] for j in range(len(stages)))
