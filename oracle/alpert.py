"""Alpert's hybrid Gauss-trapezoidal end correction for the logarithmic singularity of A (oracle side).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).

Sec. 2.3 names Alpert's rule as a local-correction alternative to Kapur-Rokhlin.  Where Kapur-Rokhlin
changes the weights of grid nodes next to the singular point, Alpert's rule removes the grid nodes
closer than a h to the target and puts m nodes t_i +- x_j h (0 < x_j < a) with weights h w_j on each
side, off the grid.  For a 2 pi-periodic integrand F(t_i + s) = phi(s) ln|s| + psi(s) (phi, psi
smooth):

    int F ~ h sum_{|k| >= a} F(t_i + k h) + h sum_j w_j [F(t_i + x_j h) + F(t_i - x_j h)].

Conditions (written here from the generalized Euler-Maclaurin expansion of the punctured trapezoid
rule, whose error on |s|^p ln|s| is h^{p+1} [2 zeta(-p) ln h - 2 zeta'(-p)]): for p = 0, 2, ..., 2m-2,
    sum_j w_j x_j^p        = sum_{k=1}^{a-1} k^p - zeta(-p)          (ln h terms, and the smooth part)
    sum_j w_j x_j^p ln x_j = sum_{k=1}^{a-1} k^p ln k + zeta'(-p)
(zeta(0) = -1/2, zeta(-p) = 0 for even p > 0, zeta'(0) = -ln(2 pi)/2,
zeta'(-2q) = (-1)^q (2q)! zeta(2q+1) / (2 (2 pi)^{2q})).  Odd p vanish by the symmetry of the nodes.
The 2m equations in the 2m unknowns x_j, w_j are solved by Newton's method in 50-digit arithmetic
from x_j = a (j + 1/2) / m, w_j = (a - 1/2) / m, each step halved until every node stays positive.
The rule is exact for phi, psi polynomials of degree < 2m: error O(h^{2m+1} ln h).  Default m = 5,
a = 6 (the smallest a whose solution has every node in (0, a) and positive weights at m = 5).

Off-grid values: the density at t_i + u h (u = +-x_j) is the Lagrange interpolant of the NL grid
values at offsets floor(u) - NL/2 + 1 .. floor(u) + NL/2 (NL = 12), so A gains the entries
A[i, i + o] += h w_j K(y_i, z(t_i + u h), n(t_i + u h)) |z'(t_i + u h)| L_o(u); the geometry there
is the curve's own (this oracle evaluates the analytic curve; the GPU library interpolates its node
positions with the same stencil and differentiates the interpolant for the normal and the speed).
"""
from __future__ import annotations

import math
from functools import lru_cache

import mpmath as mp
import numpy as np

from . import nystrom

M_DEFAULT, A_DEFAULT, NL = 5, 6, 12


def zeta_minus(p):
    """zeta(-p) for even p >= 0."""
    return mp.mpf(-0.5) if p == 0 else mp.mpf(0)


def zeta_prime_minus(p):
    """zeta'(-p) for even p >= 0 (closed forms via the functional equation)."""
    if p == 0:
        return -mp.log(2 * mp.pi) / 2
    q = p // 2
    return (-1) ** q * mp.factorial(2 * q) * mp.zeta(2 * q + 1) / (2 * (2 * mp.pi) ** (2 * q))


@lru_cache(maxsize=None)
def rule(m=M_DEFAULT, a=A_DEFAULT, dps=50):
    """Nodes x (m,) and weights w (m,) of the corrected rule (module docstring), as float64."""
    with mp.workdps(dps):
        A, B = [], []
        for q in range(m):
            p = 2 * q
            A.append(sum(mp.mpf(k) ** p for k in range(1, a)) - zeta_minus(p))
            B.append(sum(mp.mpf(k) ** p * mp.log(k) for k in range(1, a)) + zeta_prime_minus(p))
        x = [mp.mpf(a) * (j + mp.mpf(1) / 2) / m for j in range(m)]
        w = [(mp.mpf(a) - mp.mpf(1) / 2) / m for _ in range(m)]
        tol = mp.mpf(10) ** (-(dps - 8))
        for _ in range(200):
            F, J = [], []
            for q in range(m):
                p = 2 * q
                F.append(sum(w[j] * x[j] ** p for j in range(m)) - A[q])
                J.append([x[j] ** p for j in range(m)] + [w[j] * p * x[j] ** (p - 1) if p else mp.mpf(0) for j in range(m)])
            for q in range(m):
                p = 2 * q
                F.append(sum(w[j] * x[j] ** p * mp.log(x[j]) for j in range(m)) - B[q])
                J.append([x[j] ** p * mp.log(x[j]) for j in range(m)] +
                         [w[j] * x[j] ** (p - 1) * (p * mp.log(x[j]) + 1) for j in range(m)])
            res = mp.norm(mp.matrix(F))
            if res < tol:
                break
            d = mp.lu_solve(mp.matrix(J), mp.matrix(F))
            lam = mp.mpf(1)
            for _ in range(60):
                xn = [x[j] - lam * d[m + j] for j in range(m)]
                if all(v > 0 for v in xn):
                    break
                lam /= 2
            w = [w[j] - lam * d[j] for j in range(m)]
            x = xn
        else:
            raise RuntimeError("Alpert rule: Newton did not converge")
        order = sorted(range(m), key=lambda j: x[j])
        return (np.array([float(x[j]) for j in order]), np.array([float(w[j]) for j in order]))


def lagrange(u, nl=NL):
    """Offsets o (nl,) and Lagrange weights L (nl,) interpolating at u from the grid offsets
    floor(u) - nl/2 + 1 .. floor(u) + nl/2."""
    f = math.floor(u)
    o = np.arange(f - nl // 2 + 1, f + nl // 2 + 1)
    L = np.ones(nl)
    for r in range(nl):
        for q in range(nl):
            if q != r:
                L[r] *= (u - o[q]) / (o[r] - o[q])
    return o, L


def matrix_alpert(disc: nystrom.Discretization, omega: float, curve, m=M_DEFAULT, a=A_DEFAULT) -> np.ndarray:
    """A = I/2 + D - i omega S with Alpert's correction (module docstring); ``curve`` gives the
    geometry at the off-grid nodes."""
    N = disc.N
    h = 2 * math.pi / N
    x, wq = rule(m, a)
    idx = np.arange(N)
    K = nystrom.kernel(omega, disc.x, disc.x, disc.nrm)
    dist = np.abs(idx[:, None] - idx[None, :])
    dist = np.minimum(dist, N - dist)
    A = np.where(dist >= a, K, 0.0) * disc.w[None, :]
    for j in range(m):
        for sg in (1.0, -1.0):
            u = sg * x[j]
            t = disc.t + u * h
            z, dz, _ = curve.sample(t)
            sp = np.hypot(dz[:, 0], dz[:, 1])
            nr = np.stack([dz[:, 1], -dz[:, 0]], axis=1) / sp[:, None]
            # kernel from the off-grid source z(t_i + u h) to the target y_i, one per row
            dx = disc.x[:, 0] - z[:, 0]
            dy = disc.x[:, 1] - z[:, 1]
            r = np.hypot(dx, dy)
            nd = (nr[:, 0] * dx + nr[:, 1] * dy) / r
            from scipy.special import hankel1
            kv = 1j * omega / 4.0 * hankel1(1, omega * r) * nd + omega / 4.0 * hankel1(0, omega * r)
            o, L = lagrange(u)
            for oo, ll in zip(o, L):
                A[idx, (idx + oo) % N] += h * wq[j] * kv * sp * ll
    A[idx, idx] += 0.5
    return A


def matrix_alpert_rows(disc: nystrom.Discretization, omega: float, curve, rows, m=M_DEFAULT, a=A_DEFAULT) -> np.ndarray:
    """Rows ``rows`` of ``matrix_alpert``, evaluated without forming the others."""
    from scipy.special import hankel1
    N = disc.N
    h = 2 * math.pi / N
    rows = np.asarray(rows, dtype=np.int64).reshape(-1)
    x, wq = rule(m, a)
    idx = np.arange(N)
    R = np.arange(len(rows))
    with np.errstate(divide="ignore", invalid="ignore"):
        K = nystrom.kernel(omega, disc.x[rows], disc.x, disc.nrm)
    dist = np.abs(rows[:, None] - idx[None, :])
    dist = np.minimum(dist, N - dist)
    A = np.where(dist >= a, K, 0.0) * disc.w[None, :]
    for j in range(m):
        for sg in (1.0, -1.0):
            u = sg * x[j]
            z, dz, _ = curve.sample(disc.t[rows] + u * h)
            sp = np.hypot(dz[:, 0], dz[:, 1])
            nr = np.stack([dz[:, 1], -dz[:, 0]], axis=1) / sp[:, None]
            dx = disc.x[rows, 0] - z[:, 0]
            dy = disc.x[rows, 1] - z[:, 1]
            r = np.hypot(dx, dy)
            nd = (nr[:, 0] * dx + nr[:, 1] * dy) / r
            kv = 1j * omega / 4.0 * hankel1(1, omega * r) * nd + omega / 4.0 * hankel1(0, omega * r)
            o, L = lagrange(u)
            for oo, ll in zip(o, L):
                A[R, (rows + oo) % N] += h * wq[j] * kv * sp * ll
    A[R, rows] += 0.5
    return A

