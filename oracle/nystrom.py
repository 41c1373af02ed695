"""Dense Nystrom discretization of the isolated-obstacle operator (oracle side).

A = I/2 + D - i omega S  (Sec. 2.2, below Eq. 2.15), with the layer potentials of
Eqs. 2.7-2.8 and the free-space Green's function G(x) = (i/4) H0(omega |x|) of
Eq. 2.9, discretized on the periodic trapezoid rule of Sec. 2.3 with nodes
y_j = z(2 pi j / N) and weights w_j = (2 pi / N) |z'(t_j)|.

Readings (the paper is silent on these):
* The parameterization is counter-clockwise and the normal is the outward one,
  n = (z2', -z1') / |z'|; the obstacle interior is Omega.
* Kernel of A off the diagonal, with r = |x - y|:
      K(x, y, n_y) = dG/dn_y - i omega G
                   = (i omega / 4) H1(omega r) n_y.(x - y) / r + (omega / 4) H0(omega r).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import hankel1, jv

from . import quadrature

EULER_GAMMA = 0.57721566490153286060651209008240243


class Discretization:
    """Trapezoid-rule samples of a closed curve (Sec. 2.3)."""

    def __init__(self, curve, N: int):
        self.N = int(N)
        self.t = 2.0 * math.pi * np.arange(self.N) / self.N
        z, dz, d2z = curve.sample(self.t)
        self.x = z
        self.dz = dz
        self.d2z = d2z
        self.speed = np.hypot(dz[:, 0], dz[:, 1])
        self.w = (2.0 * math.pi / self.N) * self.speed
        self.nrm = np.stack([dz[:, 1], -dz[:, 0]], axis=1) / self.speed[:, None]
        # signed curvature of a counter-clockwise curve
        self.kappa = (dz[:, 0] * d2z[:, 1] - dz[:, 1] * d2z[:, 0]) / self.speed ** 3


def kernel(omega, tx, sy, sn):
    """K(x, y, n_y) of the module docstring for target array tx (m,2) and sources sy, sn (n,2).
    Returns the (m, n) complex matrix; entries with r = 0 are NaN (never used)."""
    dx = tx[:, None, 0] - sy[None, :, 0]
    dy = tx[:, None, 1] - sy[None, :, 1]
    r = np.hypot(dx, dy)
    with np.errstate(invalid="ignore", divide="ignore"):
        ndot = (sn[None, :, 0] * dx + sn[None, :, 1] * dy) / r
        val = 1j * omega / 4.0 * hankel1(1, omega * r) * ndot + omega / 4.0 * hankel1(0, omega * r)
    return val


def green(omega, tx, sy):
    """G(x - y) = (i/4) H0(omega |x - y|), Eq. 2.9."""
    r = np.hypot(tx[:, None, 0] - sy[None, :, 0], tx[:, None, 1] - sy[None, :, 1])
    return 0.25j * hankel1(0, omega * r)


def matrix_kr6(disc: Discretization, omega: float) -> np.ndarray:
    """A with Kapur-Rokhlin weights (Sec. 2.3): A_ij = delta_ij/2 + R_{(i-j) mod N} K(y_i, y_j, n_j) w_j."""
    N = disc.N
    R = quadrature.kr6_band(N)
    idx = np.arange(N)
    Rm = R[(idx[:, None] - idx[None, :]) % N]
    K = kernel(omega, disc.x, disc.x, disc.nrm)
    K[idx, idx] = 0.0
    A = Rm * K * disc.w[None, :]
    A[idx, idx] += 0.5
    return A


def matrix_kr6_rows(disc: Discretization, omega: float, rows) -> np.ndarray:
    """Rows ``rows`` of the Kapur-Rokhlin matrix of ``matrix_kr6`` (Sec. 2.3), evaluated without
    forming the other rows: A[r, j] = delta_rj/2 + R_{(r-j) mod N} K(y_r, y_j, n_j) w_j."""
    N = disc.N
    rows = np.asarray(rows, dtype=np.int64).reshape(-1)
    R = quadrature.kr6_band(N)
    idx = np.arange(N)
    K = kernel(omega, disc.x[rows], disc.x, disc.nrm)
    same = rows[:, None] == idx[None, :]
    K[same] = 0.0
    A = R[(rows[:, None] - idx[None, :]) % N] * K * disc.w[None, :]
    A[np.arange(len(rows)), rows] += 0.5
    return A


def matrix_kress(disc: Discretization, omega: float) -> np.ndarray:
    """A with Kress' spectral log-split quadrature (Colton & Kress, Sec. 3.5), N = 2n.

    Writing (A - I/2) eta(t) = int_0^{2pi} [L(t,tau) - i omega M(t,tau)] eta(tau) dtau with
      M = (i/4) H0(omega r) |z'(tau)|,
      L = (i omega / 4) H1(omega r) c / r,   c = z2'(tau)(z1(t)-z1(tau)) - z1'(tau)(z2(t)-z2(tau)),
    the log parts are M1 = -(1/4pi) J0(omega r)|z'(tau)|, L1 = -(omega/4pi) J1(omega r) c / r,
    and M2 = M - M1 ln(4 sin^2((t-tau)/2)), L2 = L - L1 ln(...), with diagonal limits
      M2(t,t) = [i/4 - C_E/(2pi) - ln(omega |z'(t)|/2)/(2pi)] |z'(t)|,
      L2(t,t) = (z2' z1'' - z1' z2'') / (4 pi |z'|^2),   L1(t,t) = 0,  M1(t,t) = -|z'(t)|/(4pi).
    Then A = I/2 + R o (L1 - i omega M1) + (pi/n) (L2 - i omega M2)."""
    N = disc.N
    n = N // 2
    t = disc.t
    idx = np.arange(N)
    off = idx[:, None] != idx[None, :]
    x1 = disc.x[:, 0][:, None] - disc.x[:, 0][None, :]
    x2 = disc.x[:, 1][:, None] - disc.x[:, 1][None, :]
    r = np.hypot(x1, x2)
    rs = np.where(off, r, 1.0)
    s_tau = disc.speed[None, :]
    c = disc.dz[None, :, 1] * x1 - disc.dz[None, :, 0] * x2
    H0 = np.where(off, hankel1(0, omega * rs), 0.0)
    H1 = np.where(off, hankel1(1, omega * rs), 0.0)
    J0 = np.where(off, jv(0, omega * rs), 1.0)
    J1 = np.where(off, jv(1, omega * rs), 0.0)
    M = 0.25j * H0 * s_tau
    L = 0.25j * omega * H1 * c / rs
    M1 = -J0 * s_tau / (4.0 * math.pi)
    L1 = np.where(off, -omega / (4.0 * math.pi) * J1 * c / rs, 0.0)
    dt = t[:, None] - t[None, :]
    lg = np.log(np.where(off, 4.0 * np.sin(dt / 2.0) ** 2, 1.0))
    M2 = np.where(off, M - M1 * lg, 0.0)
    L2 = np.where(off, L - L1 * lg, 0.0)
    s = disc.speed
    M2[idx, idx] = (0.25j - EULER_GAMMA / (2 * math.pi) - np.log(omega * s / 2.0) / (2 * math.pi)) * s
    L2[idx, idx] = (disc.dz[:, 1] * disc.d2z[:, 0] - disc.dz[:, 0] * disc.d2z[:, 1]) / (4 * math.pi * s ** 2)
    Rk = quadrature.kress_log_weights(N)[(idx[:, None] - idx[None, :]) % N]
    A = Rk * (L1 - 1j * omega * M1) + (math.pi / n) * (L2 - 1j * omega * M2)
    A[idx, idx] += 0.5
    return A


def matrix(disc: Discretization, omega: float, quad: str = "kr6") -> np.ndarray:
    if quad == "kr6":
        return matrix_kr6(disc, omega)
    if quad == "kress":
        return matrix_kress(disc, omega)
    raise ValueError(quad)


def neighbour_matrix(disc: Discretization, omega: float, shift: float) -> np.ndarray:
    """A_j of Sec. 2.4: the plain trapezoid discretization of D - i omega S from the
    translated copy dOmega + shift e_1 (sources) to dOmega (targets)."""
    src = disc.x + np.array([shift, 0.0])
    return kernel(omega, disc.x, src, disc.nrm) * disc.w[None, :]


def neighbour_rows(disc: Discretization, omega: float, shift: float, rows) -> np.ndarray:
    """Rows ``rows`` of ``neighbour_matrix`` (Sec. 2.4), evaluated without forming the others."""
    rows = np.asarray(rows, dtype=np.int64).reshape(-1)
    src = disc.x + np.array([shift, 0.0])
    return kernel(omega, disc.x[rows], src, disc.nrm) * disc.w[None, :]


def potential(disc: Discretization, omega: float, eta: np.ndarray, targets: np.ndarray) -> np.ndarray:
    """(D - i omega S) eta at off-surface targets (plain trapezoid; targets well away
    from the curve).  eta may be (N,) or (N, q)."""
    K = kernel(omega, targets, disc.x, disc.nrm) * disc.w[None, :]
    return K @ eta


def circle_eigenvalue(omega: float, R: float, n: int) -> complex:
    """Eigenvalue of A = I/2 + D - i omega S on the circle of radius R for the Fourier mode
    e^{i n t}: lambda_n = (pi omega R / 2) H_n(omega R) [J_n(omega R) + i J_n'(omega R)].
    From the addition theorem G = (i/4) sum_m J_m(omega r<) H_m(omega r>) e^{im(theta-phi)}
    and the exterior jump relation of the double layer."""
    kR = omega * R
    Jn = jv(n, kR)
    dJn = 0.5 * (jv(n - 1, kR) - jv(n + 1, kR))
    return math.pi * kR / 2.0 * hankel1(n, kR) * (Jn + 1j * dJn)
