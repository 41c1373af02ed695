"""Quadrature weights for the log-singular Nystrom matrix (oracle side).

Kapur-Rokhlin 6th order (Sec. 2.3).  The paper modifies the trapezoid weights near
the diagonal: the self point gets R_0 = 0 and the points at index distance
1 <= j <= 6 get R_j = 1 + gamma_j + gamma_{-j}, with the gammas taken from a table
that is not reproduced in the paper.  We derive the symmetric corrections
g_j = gamma_j + gamma_{-j} ourselves.  For f(s) = phi(s) ln|s| + psi(s) with
phi, psi smooth and periodic, the punctured trapezoid sum h * sum_{j != 0} f(jh)
differs from the integral by (generalized Euler-Maclaurin / zeta-function
expansion)

    -h psi(0) + h phi(0) ln(2 pi / h) - 2 sum_{p>=1} zeta'(-2p) h^{2p+1} phi^{(2p)}(0)/(2p)!

so adding h sum_{m=1..6} g_m [f(mh) + f(-mh)] cancels the terms up to p = 2 iff

    sum_m g_m m^{2p}        = 1/2 delta_{p0}                (p = 0, 1, 2)
    sum_m g_m ln m          = -1/2 ln(2 pi)                 (p = 0)
    sum_m g_m m^{2p} ln m   = zeta'(-2p)                    (p = 1, 2)

a 6x6 linear system solved here in 50-digit arithmetic.  The resulting rule is
6th order (errors O(h^7 ln h)).

Kress (spectral log split; used for the small star workload): the weights of the
product trapezoid rule for integrals of ln(4 sin^2((t - tau)/2)) f(tau).
"""
from __future__ import annotations

import math

import mpmath
import numpy as np


def kr6_corrections(dps: int = 50):
    """Symmetric Kapur-Rokhlin corrections g_1..g_6 (R_m = 1 + g_m), see module doc."""
    with mpmath.workdps(dps):
        ms = [mpmath.mpf(m) for m in range(1, 7)]
        rows, rhs = [], []
        for p in range(3):
            rows.append([m ** (2 * p) for m in ms])
            rhs.append(mpmath.mpf(1) / 2 if p == 0 else mpmath.mpf(0))
        for p in range(3):
            rows.append([m ** (2 * p) * mpmath.log(m) for m in ms])
            if p == 0:
                rhs.append(-mpmath.log(2 * mpmath.pi) / 2)
            else:
                rhs.append(mpmath.zeta(-2 * p, derivative=1))
        g = mpmath.lu_solve(mpmath.matrix(rows), mpmath.matrix(rhs))
        return np.array([float(g[i]) for i in range(6)])


def kr6_band(N: int) -> np.ndarray:
    """Weight multipliers R_m, m = 0..N-1, for index offset m = (i - j) mod N (Sec. 2.3):
    R_0 = 0, R_m = R_{N-m} = 1 + g_m for 1 <= m <= 6, and 1 otherwise."""
    if N < 13:
        raise ValueError("KR6 needs N >= 13")
    g = kr6_corrections()
    R = np.ones(N)
    R[0] = 0.0
    for m in range(1, 7):
        R[m] = 1.0 + g[m - 1]
        R[N - m] = 1.0 + g[m - 1]
    return R


def kress_log_weights(N: int) -> np.ndarray:
    """Kress weights R^{(n)}(t_i - t_j) as a function of the offset m = i - j (mod N), N = 2n.

    R^{(n)}(t) = -(2 pi / n) sum_{k=1}^{n-1} cos(k t)/k - (pi / n^2) cos(n t),  t = 2 pi m / N.
    These integrate trigonometric polynomials of degree <= n times ln(4 sin^2((t-tau)/2))
    exactly (Colton & Kress, Inverse Acoustic and EM Scattering Theory, Sec. 3.5)."""
    if N % 2:
        raise ValueError("Kress quadrature needs even N")
    n = N // 2
    t = 2.0 * math.pi * np.arange(N) / N
    k = np.arange(1, n)
    R = -(2.0 * math.pi / n) * (np.cos(np.outer(t, k)) / k).sum(axis=1)
    R -= (math.pi / n ** 2) * np.cos(n * t)
    return R
