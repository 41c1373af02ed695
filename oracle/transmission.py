"""Transmission problem of Sec. 5 (oracle side).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).

Sec. 5 replaces the Dirichlet condition by index n inside the obstacle (wavenumber n omega in
Omega, omega outside) and the matching conditions of Eqs. 5.3-5.4, and solves it through a pair of
densities eta = [sigma; tau] on dOmega that generate potentials on both sides, interlaced node by
node.  The paper defers the full recipe to another work; the formulation written out here is the
plain Mueller-type one that its text describes (readings, each checked by the tests):

* Representation.  With G_k = (i/4) H0(k r), S_k and D_k the single and double layers of
  Eqs. 2.7-2.8 at wavenumber k, k0 = omega, k1 = n omega:
      outside:  u+ = D_{k0} tau + S_{k0} sigma  (+ neighbour images and wall potentials, Sec. 2.2)
      inside:   u- = D_{k1} tau + S_{k1} sigma  (the interior field is the obstacle's own).
  The jump relations (outward normal) give on dOmega
      u+ - u-       = tau + (D0 - D1) tau + (S0 - S1) sigma
      u+_n - u-_n   = -sigma + (T0 - T1) tau + (D0* - D1*) sigma,
  T_k = d^2 G_k / dn_x dn_y, D_k* = dG_k/dn_x.  Eqs. 5.3-5.4 set these to -u^i and -u^i_n.  The
  second row is taken with the opposite sign, so that the operator is I plus a compact 2 x 2
  kernel (the hypersingular parts of T0 and T1 cancel in the difference).
* Unknown order: node by node, [tau_1; sigma_1; tau_2; sigma_2; ...] (row 2i: value jump at node
  i, row 2i + 1: minus the normal-derivative jump); the paper's [sigma; tau] naming of the pair is
  a label, the interlacing is what matters.
* Normalization: with kb = max(omega, n omega) the single layer carries the factor kb,
  u = D_k tau + kb S_k sigma, and the normal-derivative row is divided by kb.  In the far field
  D ~ k G, S ~ G, T ~ k^2 G and D* ~ k G, so every block of the operator is then of the size
  kb G: the interpolative decompositions of the fast solver, whose tolerance is relative to the
  largest entries, resolve both rows and both densities alike (without it the error grows like
  tol kb^2).  The jumps become tau + (D0 - D1) tau + kb (S0 - S1) sigma = -u^i and
  sigma - (T0 - T1) tau / kb - (D0* - D1*) sigma = u^i_n / kb.
* Quadrature: every one of the four difference kernels has the form phi(s) ln|s| + psi(s) with
  phi, psi smooth (the log part of G0 - G1 is O(r^2 ln r), and T0 - T1 keeps only a log
  singularity), so the Kapur-Rokhlin weights of Sec. 2.3 (R_0 = 0, R_m = 1 + g_m) apply to all four.
* Periodizing blocks: the wall potentials and neighbour images belong to the exterior field
  only.  B's rows are [value; minus normal derivative] of the wall potentials at the nodes;
  C's columns are the wall data of D_{k0} (tau) and S_{k0} (sigma) separately (the Dirichlet
  C of Eq. 2.17 is their combination D - i omega S); Q is unchanged (Sec. 5.2).
* Bragg amplitudes from eta through the quasi-periodic Green's function, as for the Dirichlet
  case, with the tau and sigma parts of the far-field weights separated.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
from scipy.special import hankel1

from . import nystrom, periodic, quadrature


def kbar(omega: float, index: float) -> float:
    """The normalization wavenumber kb = max(omega, n omega) of the module docstring."""
    return max(omega, index * omega)


def kernels(k0: float, k1: float, tx, tn, sy, sn):
    """The four difference kernels of the module docstring at targets tx (normals tn) and sources
    sy (normals sn): returns (K_vt, K_vs, K_nt, K_ns) = (D0 - D1, kb (S0 - S1), -(T0 - T1) / kb,
    -(D0* - D1*)), kb = max(k0, k1), unweighted, each (m, n).  Entries with r = 0 are NaN (never used)."""
    dx = tx[:, None, 0] - sy[None, :, 0]
    dy = tx[:, None, 1] - sy[None, :, 1]
    r = np.hypot(dx, dy)
    with np.errstate(invalid="ignore", divide="ignore"):
        a = (tn[:, None, 0] * dx + tn[:, None, 1] * dy) / r   # n_x . (x - y) / r
        b = (sn[None, :, 0] * dx + sn[None, :, 1] * dy) / r   # n_y . (x - y) / r
        nn = tn[:, None, 0] * sn[None, :, 0] + tn[:, None, 1] * sn[None, :, 1]
        out = []
        for k in (k0, k1):
            h0 = hankel1(0, k * r)
            h1 = hankel1(1, k * r)
            G = 0.25j * h0
            dGy = 0.25j * k * h1 * b            # dG/dn_y
            dGx = -0.25j * k * h1 * a           # dG/dn_x
            T = 0.25j * (k * k * h0 * a * b + (k * h1 / r) * (nn - 2.0 * a * b))
            out.append((dGy, G, T, dGx))
    (d0, s0, t0, x0), (d1, s1, t1, x1) = out
    kb = max(k0, k1)
    return d0 - d1, kb * (s0 - s1), -(t0 - t1) / kb, -(x0 - x1)


def exterior_kernels(k0: float, kb: float, tx, tn, sy, sn):
    """The exterior field's rows alone: (dG/dn_y, kb G, -T / kb, -dG/dn_x) at wavenumber k0 (the
    images of Sec. 2.4 and the walls contribute to u+ only)."""
    dx = tx[:, None, 0] - sy[None, :, 0]
    dy = tx[:, None, 1] - sy[None, :, 1]
    r = np.hypot(dx, dy)
    a = (tn[:, None, 0] * dx + tn[:, None, 1] * dy) / r
    b = (sn[None, :, 0] * dx + sn[None, :, 1] * dy) / r
    nn = tn[:, None, 0] * sn[None, :, 0] + tn[:, None, 1] * sn[None, :, 1]
    h0 = hankel1(0, k0 * r)
    h1 = hankel1(1, k0 * r)
    T = 0.25j * (k0 * k0 * h0 * a * b + (k0 * h1 / r) * (nn - 2.0 * a * b))
    return 0.25j * k0 * h1 * b, kb * 0.25j * h0, -T / kb, 0.25j * k0 * h1 * a


def interlace(Kvt, Kvs, Knt, Kns):
    """[[Kvt, Kvs], [Knt, Kns]] blocks -> one matrix with rows and columns node by node."""
    m, n = Kvt.shape
    A = np.empty((2 * m, 2 * n), dtype=complex)
    A[0::2, 0::2] = Kvt
    A[0::2, 1::2] = Kvs
    A[1::2, 0::2] = Knt
    A[1::2, 1::2] = Kns
    return A


def matrix(disc: nystrom.Discretization, omega: float, index: float) -> np.ndarray:
    """The 2N x 2N interlaced operator I + K with Kapur-Rokhlin weights on all four blocks
    (module docstring; Sec. 5.3 for the order of the unknowns)."""
    N = disc.N
    R = quadrature.kr6_band(N)
    idx = np.arange(N)
    Rm = R[(idx[:, None] - idx[None, :]) % N] * disc.w[None, :]
    blocks = kernels(omega, index * omega, disc.x, disc.nrm, disc.x, disc.nrm)
    out = []
    for K in blocks:
        K = K.copy()
        K[idx, idx] = 0.0  # R_0 = 0
        out.append(Rm * K)
    return interlace(*out) + np.eye(2 * N)


def matrix_rows(disc: nystrom.Discretization, omega: float, index: float, rows) -> np.ndarray:
    """Rows ``rows`` (indices into the 2N interlaced unknowns) of ``matrix``, without forming the
    others."""
    N = disc.N
    rows = np.asarray(rows, dtype=np.int64).reshape(-1)
    nodes = rows // 2
    R = quadrature.kr6_band(N)
    idx = np.arange(N)
    Rm = R[(nodes[:, None] - idx[None, :]) % N] * disc.w[None, :]
    blocks = kernels(omega, index * omega, disc.x[nodes], disc.nrm[nodes], disc.x, disc.nrm)
    out = np.zeros((len(rows), 2 * N), dtype=complex)
    same = nodes[:, None] == idx[None, :]
    for q, K in enumerate(blocks):
        K = np.where(same, 0.0, K)
        comp_r, comp_c = divmod(q, 2)
        sel = (rows % 2) == comp_r
        out[sel, comp_c::2] = (Rm * K)[sel]
    out[np.arange(len(rows)), rows] += 1.0
    return out


def neighbour_matrix(disc: nystrom.Discretization, omega: float, index: float, shift: float) -> np.ndarray:
    """A_j of Sec. 2.4 for the exterior field: plain trapezoid rule from the copy dOmega + shift e_1."""
    src = disc.x + np.array([shift, 0.0])
    blocks = exterior_kernels(omega, kbar(omega, index), disc.x, disc.nrm, src, disc.nrm)
    return interlace(*[K * disc.w[None, :] for K in blocks])


def neighbour_rows(disc: nystrom.Discretization, omega: float, index: float, shift: float, rows) -> np.ndarray:
    """Rows ``rows`` of ``neighbour_matrix``."""
    rows = np.asarray(rows, dtype=np.int64).reshape(-1)
    nodes = rows // 2
    src = disc.x + np.array([shift, 0.0])
    blocks = exterior_kernels(omega, kbar(omega, index), disc.x[nodes], disc.nrm[nodes], src, disc.nrm)
    out = np.zeros((len(rows), 2 * disc.N), dtype=complex)
    for q, K in enumerate(blocks):
        comp_r, comp_c = divmod(q, 2)
        sel = (rows % 2) == comp_r
        out[sel, comp_c::2] = (K * disc.w[None, :])[sel]
    return out


def rhs_from_jumps(f, g, kb):
    """Right-hand side for prescribed jumps u+ - u- = f, u+_n - u-_n = g (rows [f; -g / kb] interlaced)."""
    f = np.asarray(f)
    g = np.asarray(g)
    out = np.empty((2 * f.shape[0],) + f.shape[1:], dtype=complex)
    out[0::2] = f
    out[1::2] = -g / kb
    return out


def incident(disc: nystrom.Discretization, omega: float, index: float, theta):
    """Eqs. 5.3-5.4 with u^i = exp(i k.x): jumps -u^i and -u^i_n, interlaced (N x q -> 2N x q)."""
    th = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    kx = omega * np.cos(th)
    ky = omega * np.sin(th)
    ui = np.exp(1j * (np.outer(disc.x[:, 0], kx) + np.outer(disc.x[:, 1], ky)))
    dn = 1j * (np.outer(disc.nrm[:, 0], kx) + np.outer(disc.nrm[:, 1], ky)) * ui
    return rhs_from_jumps(-ui, -dn, kbar(omega, index))


def potential(disc: nystrom.Discretization, k: float, kb: float, eta: np.ndarray, targets: np.ndarray,
              shift: float = 0.0) -> np.ndarray:
    """D_k tau + kb S_k sigma from the copy dOmega + shift e_1 at off-surface targets (plain trapezoid;
    targets away from that copy)."""
    dx = targets[:, None, 0] - (disc.x[None, :, 0] + shift)
    dy = targets[:, None, 1] - disc.x[None, :, 1]
    r = np.hypot(dx, dy)
    b = (disc.nrm[None, :, 0] * dx + disc.nrm[None, :, 1] * dy) / r
    D = 0.25j * k * hankel1(1, k * r) * b * disc.w[None, :]
    S = 0.25j * hankel1(0, k * r) * disc.w[None, :]
    return D @ eta[0::2] + kb * (S @ eta[1::2])


def wall_B(disc, omega, index, period, ct: periodic.Contour):
    """B_L, B_R (2N x 2M): the wall potentials of Eqs. 2.12-2.13 on dOmega, rows [value; minus the
    normal derivative over kb] interlaced, columns [mu; nu]."""
    kb = kbar(omega, index)
    out = []
    nx, ny = disc.nrm[:, 0][:, None], disc.nrm[:, 1][:, None]
    for xw in (-period / 2.0, period / 2.0):
        dx = disc.x[:, 0][:, None] - xw
        y = disc.x[:, 1][:, None]
        sg = np.sign(dx)
        e = ct.wk[None, :] * np.exp(1j * ct.k[None, :] * y) * np.exp(1j * ct.s[None, :] * np.abs(dx))
        de = 1j * (ct.s[None, :] * sg * nx + ct.k[None, :] * ny) * e   # d e / dn
        BS, BD = 0.5j * e / ct.s[None, :], 0.5 * sg * e
        dBS, dBD = 0.5j * de / ct.s[None, :], 0.5 * sg * de
        B = np.empty((2 * disc.N, 2 * len(ct.k)), dtype=complex)
        B[0::2] = np.hstack([BS, BD])
        B[1::2] = -np.hstack([dBS, dBD]) / kb
        out.append(B)
    return out[0], out[1]


def wall_C(disc, omega, index, period, ct: periodic.Contour, shift: float = 0.0):
    """C_L, C_R (2M x 2N): the wall data (value rows, x-derivative rows) of D_{k0} tau (even
    columns) and kb S_{k0} sigma (odd columns) from the density on dOmega + shift e_1, as in Eq. 2.17."""
    kb = kbar(omega, index)
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
        valD = E * (-sg * nx + (k / s) * ny)
        derD = 1j * E * (s * nx - k * sg * ny)
        valS = 1j * E / s
        derS = E * sg
        C = np.empty((2 * len(ct.k), 2 * disc.N), dtype=complex)
        C[:, 0::2] = np.vstack([valD, derD]) * disc.w[None, :]
        C[:, 1::2] = kb * np.vstack([valS, derS]) * disc.w[None, :]
        out.append(C)
    return out[0], out[1]


def assemble(disc, omega, index, period, alpha, ct: periodic.Contour, P: int = 0, A0=None):
    """Blocks of the bordered system (Eq. 2.19, Eq. 2.21 with P images) for the transmission case."""
    A = matrix(disc, omega, index) if A0 is None else A0.copy()
    for j in range(-P, P + 1):
        if j != 0:
            A = A + alpha ** j * neighbour_matrix(disc, omega, index, j * period)
    BL, BR = wall_B(disc, omega, index, period, ct)
    CLp, _ = wall_C(disc, omega, index, period, ct, shift=P * period)
    _, CRm = wall_C(disc, omega, index, period, ct, shift=-P * period)
    C = alpha ** P * CLp - alpha ** (-(P + 1)) * CRm
    return periodic.QPSystem(A, BL + alpha * BR, C, periodic.wall_Q(omega, period, alpha, ct), alpha)


def bragg_lattice(disc, omega, index, period, theta, eta, y0):
    """Bragg amplitudes above (c_n) and below (d_n) from eta alone (module docstring)."""
    n, kx, kn = periodic.bragg_orders(omega, period, theta)
    x, y = disc.x[:, 0], disc.x[:, 1]
    nx, ny = disc.nrm[:, 0], disc.nrm[:, 1]
    wt, ws = disc.w * eta[0::2], kbar(omega, index) * disc.w * eta[1::2]
    pre = 1j * np.exp(1j * kn * y0) / (2 * period * kn)
    eu = np.exp(-1j * (np.outer(kx, x) + np.outer(kn, y)))
    ed = np.exp(-1j * (np.outer(kx, x) - np.outer(kn, y)))
    c = pre * ((eu * (-1j * (np.outer(kx, nx) + np.outer(kn, ny)))) @ wt + eu @ ws)
    d = pre * ((ed * (1j * (-np.outer(kx, nx) + np.outer(kn, ny)))) @ wt + ed @ ws)
    return n, kn, c, d


def field(disc, omega, index, period, alpha, ct: periodic.Contour, eta, xi, pts, P=0):
    """Scattered exterior field in the unit cell away from dOmega: images plus wall potentials."""
    u = np.zeros(len(pts), dtype=complex)
    for j in range(-P, P + 1):
        u += alpha ** j * potential(disc, omega, kbar(omega, index), eta, pts, shift=j * period)
    M = len(ct.k)
    mu, nu = xi[:M], xi[M:]
    for xw, fac in ((-period / 2.0, 1.0), (period / 2.0, alpha)):
        dx = pts[:, 0][:, None] - xw
        e = ct.wk[None, :] * np.exp(1j * ct.k[None, :] * pts[:, 1][:, None]) * np.exp(1j * ct.s[None, :] * np.abs(dx))
        u += fac * ((0.5j * e / ct.s[None, :]) @ mu + (0.5 * np.sign(dx) * e) @ nu)
    return u


def bragg_sampled(disc, omega, index, period, alpha, ct, theta, eta, xi, y0, ns=128, P=0):
    """Bragg amplitudes by sampling the exterior field on y = +-y0 and a DFT (Remarks 2.2-2.3)."""
    n, kx, kn = periodic.bragg_orders(omega, period, theta)
    xl = -period / 2 + (np.arange(ns) + 0.5) * period / ns
    up = field(disc, omega, index, period, alpha, ct, eta, xi, np.stack([xl, np.full(ns, y0)], 1), P)
    dn = field(disc, omega, index, period, alpha, ct, eta, xi, np.stack([xl, np.full(ns, -y0)], 1), P)
    F = np.exp(-1j * np.outer(kx, xl)) / ns
    return n, kn, F @ up, F @ dn


def solve_qp(curve_or_disc, N, omega, index, period, thetas, P=0, h=0.1, A0=None):
    """Dense bordered solve of the transmission grating for every angle (Sec. 5 with Sec. 2-3):
    eta (2N, q) interlaced, xi (2M, q), Bragg amplitudes and flux errors."""
    disc = curve_or_disc if isinstance(curve_or_disc, nystrom.Discretization) \
        else nystrom.Discretization(curve_or_disc, N)
    ct = periodic.default_contour(disc, omega, period, P=P, h=h)
    A = matrix(disc, omega, index) if A0 is None else A0
    y0 = periodic.default_y0(disc)
    etas, xis, braggs, flux = [], [], [], []
    for th in np.atleast_1d(thetas):
        al = periodic.bloch_phase(omega, period, th)
        sysm = assemble(disc, omega, index, period, al, ct, P=P, A0=A)
        eta, xi = periodic.solve_bordered(sysm, incident(disc, omega, index, th))
        eta, xi = eta[:, 0], xi[:, 0]
        nn, kn, c, d = bragg_lattice(disc, omega, index, period, th, eta, y0)
        etas.append(eta)
        xis.append(xi)
        braggs.append((nn, kn, c, d))
        flux.append(periodic.flux_error(omega, th, nn, kn, c, d, y0))
    return dict(disc=disc, contour=ct, y0=y0, eta=np.array(etas).T, xi=np.array(xis).T,
                bragg=braggs, flux=np.array(flux))


def solve_isolated(disc, omega, index, rhs):
    """Dense LU of the isolated-obstacle system (Sec. 5.3) for interlaced right-hand sides."""
    return sla.lu_solve(sla.lu_factor(matrix(disc, omega, index)), rhs)
