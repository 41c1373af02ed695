"""Periodizing scheme and the bordered quasi-periodic system (oracle side).

Follows Sec. 2.2-2.4 and Sec. 3.1: the representation of Eq. 2.14 (Eq. 2.20 with
P neighbour images), the blocks B (Eq. 2.16), C (Eq. 2.17, and C~ of Sec. 2.4), Q
(Eq. 2.18), the Sommerfeld-contour quadrature of Sec. 2.3, and the dense solve of
the bordered system (Eq. 2.19 / 2.21).

Readings of silent, ambiguous or misprinted passages (each checked numerically by
the tests through the flux balance, the two Bragg extractions, and P=0 vs P=1):
* Contour (Sec. 2.3 gives only "tanh-shaped, height O(1), trapezoid in Re k with
  spacing h, cut at K, M = 2K/h"):  t_m = -K + (m - 1/2) h, m = 1..M,
  k_m = t_m - i a tanh(t_m / b), quadrature weight h k'(t_m) with
  k'(t) = 1 - i (a/b) sech^2(t/b); s_m = sqrt(omega^2 - k_m^2) on the principal
  branch (Im s >= 0 on the whole contour since it runs through the 2nd and 4th
  quadrants).  Defaults a = b = 1, h = 0.1, K = sqrt(omega^2 + (37/g)^2) with
  g = (P + 1/2) d - max|x| the distance from a wall to the nearest image that the
  wall densities must represent.
* Q (Eq. 2.18): taking the Fourier coefficients of the wall potentials of Eq. 2.14
  on L and R from inside the cell gives, with E = e^{i s d}, a(+/-) = alpha +/- 1/alpha,
      Q = [[ i E a(-)/(2 s),     1 - E a(+)/2 ],
           [ -1 + E a(+)/2,      i E s a(-)/2 ]]
  i.e. the printed identity blocks belong off the diagonal, as [[0, I], [-I, 0]]
  (rows ordered [f; f_n], unknowns [mu; nu]).
* C~ (Sec. 2.4): the telescoped wall sum gives
      C~ = alpha^P C_L[dOmega + P d] - alpha^{-(P+1)} C_R[dOmega - P d]
  (equivalently C_L[dOmega - (P+1) d] in the second term); the printed
  "R, dOmega - (P+1) d" does not reduce to Eq. 2.17 at P = 0.
* Block solve (Eq. 3.1): eliminating eta from [A B; C Q][eta; xi] = [b; 0] gives
  xi = -(Q - C A^{-1} B)^{-1} C A^{-1} b,  eta = A^{-1} b - A^{-1} B xi
  (the printed first line lacks the factor -C).
* Bragg amplitudes: besides the sampling of Remark 2.2, the amplitudes follow from
  eta alone through the quasi-periodic Green's function
  sum_j alpha^j G(x - j d, y) = (i / 2d) sum_n e^{i kappa_n x} e^{i k_n |y|} / k_n.
* Flux error (Remark 6.1): the cited formula is not reproduced; energy balance of
  the Rayleigh-Bloch expansions (Eqs. 2.5-2.6) with unit incident amplitude gives
      eps = | sum_prop k_n |c_n|^2 + sum_{prop, n != 0} k_n |d_n|^2 + k_0 |d_0 + e^{i k_0 y0}|^2 - k_0 | / k_0
  (absolute imbalance in units of the incident flux).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import nystrom


@dataclass
class Contour:
    k: np.ndarray   # nodes k_m (complex, M)
    wk: np.ndarray  # quadrature weights h k'(t_m) (complex, M)
    s: np.ndarray   # sqrt(omega^2 - k_m^2), principal branch


def contour(omega: float, M: int | None = None, K: float | None = None, h: float = 0.1,
            a: float = 1.0, b: float = 1.0, gap: float | None = None) -> Contour:
    """Sommerfeld contour quadrature (Sec. 2.3; shape read as in the module docstring)."""
    if K is None:
        if gap is None:
            raise ValueError("need K or gap")
        K = math.sqrt(omega ** 2 + (37.0 / gap) ** 2)
    if M is None:
        M = int(math.ceil(2.0 * K / h))
        h = 2.0 * K / M
    else:
        h = 2.0 * K / M
    t = -K + (np.arange(1, M + 1) - 0.5) * h
    k = t - 1j * a * np.tanh(t / b)
    wk = h * (1.0 - 1j * (a / b) / np.cosh(t / b) ** 2)
    s = np.sqrt(omega ** 2 - k ** 2 + 0j)
    return Contour(k, wk, s)


def default_contour(disc, omega, period, P=0, h=0.1):
    gap = (P + 0.5) * period - float(np.max(np.abs(disc.x[:, 0])))
    return contour(omega, gap=gap, h=h)


def wall_B(disc, omega, period, ct: Contour):
    """B_L, B_R (N x 2M): the Fourier wall potentials of Eqs. 2.12-2.13 evaluated on dOmega,
    so that B(alpha) = B_L + alpha B_R (Eq. 2.16), columns ordered [mu; nu]."""
    out = []
    for xw in (-period / 2.0, period / 2.0):
        dx = disc.x[:, 0][:, None] - xw
        y = disc.x[:, 1][:, None]
        e = ct.wk[None, :] * np.exp(1j * ct.k[None, :] * y) * np.exp(1j * ct.s[None, :] * np.abs(dx))
        BS = 0.5j * e / ct.s[None, :]
        BD = 0.5 * np.sign(dx) * e
        out.append(np.hstack([BS, BD]))
    return out[0], out[1]


def wall_C(disc, omega, period, ct: Contour, shift: float = 0.0):
    """C_L, C_R (2M x N): the maps S^, D^, D*^, T^ of Sec. 2.2 from a density on
    dOmega + shift e_1 to Fourier data on the walls, combined as in Eq. 2.17:
    rows [value (D^ - i omega S^); x-derivative (T^ - i omega D*^)], with the
    Nystrom weights w_j.  C(alpha) = C_L - alpha^{-1} C_R."""
    out = []
    xs = disc.x[:, 0] + shift
    for xw in (-period / 2.0, period / 2.0):
        dx = xs[None, :] - xw
        sg = np.sign(dx)
        k = ct.k[:, None]
        s = ct.s[:, None]
        E = np.exp(-1j * k * disc.x[None, :, 1]) * np.exp(1j * s * np.abs(dx)) / (4.0 * math.pi)
        nx = disc.nrm[None, :, 0]
        ny = disc.nrm[None, :, 1]
        val = E * (-sg * nx + (k / s) * ny) + omega * E / s
        der = 1j * E * (s * nx - k * sg * ny) - 1j * omega * E * sg
        out.append(np.vstack([val, der]) * disc.w[None, :])
    return out[0], out[1]


def wall_Q(omega, period, alpha, ct: Contour):
    """Q(alpha), 2M x 2M with four diagonal blocks (Eq. 2.18, corrected as in the module doc)."""
    E = np.exp(1j * ct.s * period)
    ap = alpha + 1.0 / alpha
    am = alpha - 1.0 / alpha
    return np.block([[np.diag(1j * E * am / (2 * ct.s)), np.diag(1.0 - E * ap / 2)],
                     [np.diag(-1.0 + E * ap / 2), np.diag(1j * E * ct.s * am / 2)]])


def incident(disc, omega, theta):
    """Right-hand side b = -u^i on dOmega, u^i = exp(i k.x), k = omega (cos th, sin th) (Eq. 1.1)."""
    th = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    kx = omega * np.cos(th)
    ky = omega * np.sin(th)
    return -np.exp(1j * (np.outer(disc.x[:, 0], kx) + np.outer(disc.x[:, 1], ky)))


def bloch_phase(omega, period, theta):
    return np.exp(1j * omega * period * math.cos(theta))


@dataclass
class QPSystem:
    A: np.ndarray       # A~ (with neighbour images when P > 0)
    B: np.ndarray
    C: np.ndarray
    Q: np.ndarray
    alpha: complex


def assemble(disc, omega, period, alpha, ct: Contour, P: int = 0, quad: str = "kr6", A0=None):
    """Blocks of the bordered system (Eq. 2.19 for P = 0, Eq. 2.21 for P > 0)."""
    A = nystrom.matrix(disc, omega, quad) if A0 is None else A0.copy()
    for j in range(-P, P + 1):
        if j != 0:
            A = A + alpha ** j * nystrom.neighbour_matrix(disc, omega, j * period)
    BL, BR = wall_B(disc, omega, period, ct)
    B = BL + alpha * BR
    CLp, _ = wall_C(disc, omega, period, ct, shift=P * period)
    _, CRm = wall_C(disc, omega, period, ct, shift=-P * period)
    C = alpha ** P * CLp - alpha ** (-(P + 1)) * CRm
    Q = wall_Q(omega, period, alpha, ct)
    return QPSystem(A, B, C, Q, alpha)


def solve_bordered(sys: QPSystem, b: np.ndarray):
    """Dense LU of the full (N + 2M) square system [[A, B], [C, Q]] [eta; xi] = [b; 0]."""
    N = sys.A.shape[0]
    big = np.block([[sys.A, sys.B], [sys.C, sys.Q]])
    rhs = np.vstack([b, np.zeros((sys.Q.shape[0], b.shape[1]), dtype=complex)])
    sol = sla.lu_solve(sla.lu_factor(big), rhs)
    return sol[:N], sol[N:]


def solve_schur(sys: QPSystem, b: np.ndarray):
    """Block elimination of Eq. 3.1 (corrected sign), with one LU of A."""
    lu = sla.lu_factor(sys.A)
    AiB = sla.lu_solve(lu, sys.B)
    Aib = sla.lu_solve(lu, b)
    S = sys.Q - sys.C @ AiB
    xi = -np.linalg.solve(S, sys.C @ Aib)
    eta = Aib - AiB @ xi
    return eta, xi


def bragg_orders(omega, period, theta, extra=0):
    """Orders n with kappa_n = kappa + 2 pi n / d and k_n = sqrt(omega^2 - kappa_n^2) (Im >= 0):
    all propagating orders plus ``extra`` evanescent ones on each side."""
    kap = omega * math.cos(theta)
    nlo = math.ceil((-omega - kap) * period / (2 * math.pi)) - extra
    nhi = math.floor((omega - kap) * period / (2 * math.pi)) + extra
    n = np.arange(nlo, nhi + 1)
    kn_x = kap + 2 * math.pi * n / period
    kn = np.sqrt(omega ** 2 - kn_x ** 2 + 0j)
    return n, kn_x, kn


def bragg_lattice(disc, omega, period, theta, eta, y0):
    """Bragg amplitudes c_n (above, Eq. 2.5) and d_n (below, Eq. 2.6) of the scattered field
    from eta alone, via the quasi-periodic Green's function (module doc)."""
    n, kx, kn = bragg_orders(omega, period, theta)
    x, y = disc.x[:, 0], disc.x[:, 1]
    nx, ny = disc.nrm[:, 0], disc.nrm[:, 1]
    wq = disc.w * eta
    pre = 1j * np.exp(1j * kn * y0) / (2 * period * kn)
    eu = np.exp(-1j * (np.outer(kx, x) + np.outer(kn, y)))
    ed = np.exp(-1j * (np.outer(kx, x) - np.outer(kn, y)))
    fu = -1j * (np.outer(kx, nx) + np.outer(kn, ny)) - 1j * omega
    fd = 1j * (-np.outer(kx, nx) + np.outer(kn, ny)) - 1j * omega
    c = pre * ((eu * fu) @ wq)
    dd = pre * ((ed * fd) @ wq)
    return n, kn, c, dd


def field(disc, omega, period, alpha, ct: Contour, eta, xi, pts, P=0):
    """Scattered field u of Eq. 2.14 (Eq. 2.20 for P > 0) at points inside the unit cell,
    away from dOmega: obstacle potentials plus the wall potentials of Eqs. 2.12-2.13."""
    u = np.zeros(len(pts), dtype=complex)
    for j in range(-P, P + 1):
        src = disc.x + np.array([j * period, 0.0])
        K = nystrom.kernel(omega, pts, src, disc.nrm) * disc.w[None, :]
        u += alpha ** j * (K @ eta)
    M = len(ct.k)
    mu, nu = xi[:M], xi[M:]
    for xw, fac in ((-period / 2.0, 1.0), (period / 2.0, alpha)):
        dx = pts[:, 0][:, None] - xw
        e = ct.wk[None, :] * np.exp(1j * ct.k[None, :] * pts[:, 1][:, None]) \
            * np.exp(1j * ct.s[None, :] * np.abs(dx))
        u += fac * ((0.5j * e / ct.s[None, :]) @ mu + (0.5 * np.sign(dx) * e) @ nu)
    return u


def bragg_sampled(disc, omega, period, alpha, ct, theta, eta, xi, y0, ns=128, P=0):
    """Bragg amplitudes by sampling u of Eq. 2.14 on y = +/- y0 and a DFT (Remarks 2.2, 2.3)."""
    n, kx, kn = bragg_orders(omega, period, theta)
    xl = -period / 2 + (np.arange(ns) + 0.5) * period / ns
    up = field(disc, omega, period, alpha, ct, eta, xi, np.stack([xl, np.full(ns, y0)], 1), P)
    dn = field(disc, omega, period, alpha, ct, eta, xi, np.stack([xl, np.full(ns, -y0)], 1), P)
    F = np.exp(-1j * np.outer(kx, xl)) / ns
    return n, kn, F @ up, F @ dn


def flux_error(omega, theta, n, kn, c, d, y0):
    """Energy-balance error of Remark 6.1 (formula derived in the module doc)."""
    prop = np.abs(kn.imag) < 1e-14
    k0 = omega * abs(math.sin(theta))
    i0 = int(np.nonzero(n == 0)[0][0])
    out = np.sum(kn.real[prop] * np.abs(c[prop]) ** 2)
    dd = d.copy()
    dd[i0] = d[i0] + np.exp(1j * k0 * y0)
    out += np.sum(kn.real[prop] * np.abs(dd[prop]) ** 2)
    return abs(out - k0) / k0


def default_y0(disc):
    return float(np.max(np.abs(disc.x[:, 1]))) + 0.5


def solve_qp(curve_or_disc, N, omega, period, thetas, P=0, quad="kr6", h=0.1, method="bordered",
             A0=None):
    """Full oracle solve for every angle: returns dict of eta (N,q), xi (2M,q), Bragg, flux."""
    disc = curve_or_disc if isinstance(curve_or_disc, nystrom.Discretization) \
        else nystrom.Discretization(curve_or_disc, N)
    ct = default_contour(disc, omega, period, P=P, h=h)
    A = nystrom.matrix(disc, omega, quad) if A0 is None else A0
    y0 = default_y0(disc)
    thetas = np.atleast_1d(thetas)
    etas, xis, flux, braggs = [], [], [], []
    for th in thetas:
        al = bloch_phase(omega, period, th)
        sysm = assemble(disc, omega, period, al, ct, P=P, quad=quad, A0=A)
        b = incident(disc, omega, th)
        eta, xi = (solve_bordered if method == "bordered" else solve_schur)(sysm, b)
        eta, xi = eta[:, 0], xi[:, 0]
        nn, kn, c, d = bragg_lattice(disc, omega, period, th, eta, y0)
        etas.append(eta)
        xis.append(xi)
        braggs.append((nn, kn, c, d))
        flux.append(flux_error(omega, th, nn, kn, c, d, y0))
    return dict(disc=disc, contour=ct, y0=y0, eta=np.array(etas).T, xi=np.array(xis).T,
                bragg=braggs, flux=np.array(flux))
