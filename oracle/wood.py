"""Robustness at and near Wood's anomalies (Sec. 2.4, second improvement) -- oracle side.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).

The wall densities mu^, nu^ of Eq. 2.14 are meromorphic in the Fourier variable k with poles at
+-k_n (k_n = sqrt(omega^2 - kappa_n^2), kappa_n = kappa + 2 pi n / d).  As an angle approaches a
Wood's anomaly some k_n -> 0, the poles +-k_n close in on the Sommerfeld contour where it crosses
the origin, and its trapezoid rule loses accuracy.  The paper's fix (details deferred to its
reference on the periodizing scheme): move the contour by an O(1) real amount so that it stays
far from every pole, add one unknown coefficient for the Rayleigh-Bloch wave of each order whose
pole the contour crossed, and add one row per such order stating that the field carries no
incoming radiation in that order, evaluated from the representation as in Remark 2.3.

Readings (the paper gives the idea, not the formulas):
* Displaced contour: k(t) = t - i a tanh((t - delta) / b), t = -K + (m - 1/2) h, m = 1..M (the same
  t-grid as the undisplaced contour of ``periodic.contour``), weight h k'(t), s = sqrt(omega^2 - k^2)
  on the principal branch.  It crosses the real axis at k = delta instead of 0; for delta > 0 it
  passes above the poles +k_n with 0 <= k_n < delta and +i|k_n| with |k_n| < a tanh(delta / b),
  which the undisplaced contour passes below, and on the same side of every other pole.
* Why one unknown per crossed order: deforming the contour across the pole k_n adds 2 pi i times
  the residue of the wall integrands.  The residue (r_mu, r_nu) of the true densities lies in the
  null space of Q(k_n) (Eq. 2.18), because C eta + Q (mu^; nu^) = 0 holds identically in k and
  C eta has no pole there.  With s(k_n) = |kappa_n| and e^{i kappa_n d} = alpha that null space
  is r_nu = i r_mu / s, and then the residue terms of the left and right walls combine into one
  quasi-periodic plane wave, phi_n = exp(i (kappa_n x + k_n y)) (up-going, or decaying upward for
  an evanescent order).  phi_n satisfies the wall conditions by itself, so it enters only the
  obstacle rows: A eta + B xi + sum_n a_n phi_n = b.
* Radiation row of a crossed order n: below the obstacle the n-th Fourier coefficient of the field
  is U_n(y) = A+ e^{i k_n y} + A- e^{-i k_n y}; the up-going (incoming from below, or growing
  downward) part A+ vanishes iff i k_n U_n(-y0) + U_n'(-y0) = 0.  U_n and U_n' are taken, as in
  Remark 2.3, from samples of the representation and of its y-derivative at ns equispaced points
  x_l = -d/2 + (l + 1/2) d / ns on y = -y0 and a discrete Fourier transform, with ns large enough
  that the aliases of every propagating order decay by e^-37 between the line and the obstacle
  (``default_samples``).  At an exact anomaly (k_n = 0) the row states U_n'(-y0) = 0 (no linearly
  growing term).
* Choice of delta: the value in [0.25, 3] (step 0.05) that keeps every pole +-k_n of the angle's
  orders farthest from the real axis of the contour's parameter plane (the trapezoid rule in t loses
  about exp(-2 pi dist / h)); the displaced contour's t-range is that of the undisplaced one (the
  shift moves only the crossing of the real axis).
* Bragg amplitudes from the solution: eta is the physical density (unchanged by the displacement),
  so the lattice sum of ``periodic.bragg_lattice`` applies to every order with k_n != 0; the flux
  balance of Remark 6.1 gives a grazing order (k_n = 0) zero weight.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
from scipy.special import hankel1

from . import nystrom
from . import periodic


def displaced_contour(omega, K, h, a=1.0, b=1.0, delta=0.0, M=None) -> periodic.Contour:
    """The Sommerfeld contour of ``periodic.contour`` with its real-axis crossing moved to delta."""
    if M is None:
        M = int(math.ceil(2.0 * K / h))
    h = 2.0 * K / M
    t = -K + (np.arange(1, M + 1) - 0.5) * h
    k = t - 1j * a * np.tanh((t - delta) / b)
    wk = h * (1.0 - 1j * (a / b) / np.cosh((t - delta) / b) ** 2)
    s = np.sqrt(omega ** 2 - k ** 2 + 0j)
    return periodic.Contour(k, wk, s)


def _contour_im_at(re, a, b, delta):
    """Imaginary part of the contour where its real part is ``re`` (Re k(t) = t)."""
    return -a * np.tanh((re - delta) / b)


def orders(omega, period, theta, extra=3):
    """All orders whose |k_n| is below omega plus ``extra`` on each side: (n, kappa_n, k_n)."""
    return periodic.bragg_orders(omega, period, theta, extra=extra)


def crossed_orders(omega, period, theta, delta, a=1.0, b=1.0):
    """Orders n whose pole +k_n the contour displaced by delta passes above (the undisplaced contour
    passes below it).  Raises if some pole -k_n changes side (not produced by delta >= 0)."""
    n, kx, kn = orders(omega, period, theta)
    out = []
    for j in range(len(n)):
        p = kn[j]
        ip = _contour_im_at(p.real, a, b, delta)
        im0 = _contour_im_at(p.real, a, b, 0.0)
        # the pole +k_n belongs above the contour: undisplaced it is (or, at k_n = 0, it sits on it)
        if p.imag < ip and p.imag >= im0 - 1e-15:
            out.append(j)
        q = -p
        if q.imag > _contour_im_at(q.real, a, b, delta) + 1e-15:
            raise ValueError("the displaced contour crossed a pole -k_n")
    return [(int(n[j]), float(kx[j]), complex(kn[j])) for j in out]


def pole_distance(omega, period, theta, delta, K, a=1.0, b=1.0):
    """Smallest distance of the poles +-k_n from the real axis of the contour's parameter plane:
    |Im t*| for the t* with k(t*) = pole (Newton from t = Re pole), which sets the error of the
    trapezoid rule in t (about exp(-2 pi |Im t*| / h))."""
    _, _, kn = orders(omega, period, theta)
    poles = np.concatenate([kn, -kn])
    poles = poles[np.abs(poles.real) <= K]
    best = np.inf
    for p in poles:
        t = complex(p.real)
        for _ in range(60):
            th_ = np.tanh((t - delta) / b)
            f = t - 1j * a * th_ - p
            fp = 1.0 - 1j * (a / b) * (1.0 - th_ * th_)
            dt = f / fp
            t -= dt
            if abs(dt) < 1e-15:
                break
        best = min(best, abs(t.imag))
    return float(best)


def choose_delta(omega, period, theta, K, a=1.0, b=1.0):
    """The shift in [0.25, 3] (step 0.05) whose contour keeps every pole farthest from the real
    axis of its parameter plane (smallest shift on ties)."""
    best, bd = 0.25, -1.0
    for dl in np.arange(0.25, 3.0 + 1e-9, 0.05):
        dist = pole_distance(omega, period, theta, dl, K, a, b)
        if dist > bd + 1e-12:
            best, bd = float(dl), dist
    return best


def kernel_dy(omega, tx, sy, sn):
    """d/dx2 of K(x, y, n_y) of ``nystrom.kernel`` with respect to the target's second coordinate.
    With d = x - y, r = |d|, nd = n.d, H1'(z) = H0(z) - H1(z)/z:
      dK/dx2 = (i omega / 4) [ (omega H1'(omega r) / r - H1(omega r) / r^2) (d2 / r) nd + H1(omega r) n2 / r ]
               - (omega^2 / 4) H1(omega r) d2 / r."""
    dx = tx[:, None, 0] - sy[None, :, 0]
    dy = tx[:, None, 1] - sy[None, :, 1]
    r = np.hypot(dx, dy)
    z = omega * r
    H0 = hankel1(0, z)
    H1 = hankel1(1, z)
    dH1 = H0 - H1 / z
    nd = sn[None, :, 0] * dx + sn[None, :, 1] * dy
    return (0.25j * omega * ((omega * dH1 / r - H1 / r ** 2) * (dy / r) * nd + H1 * sn[None, :, 1] / r)
            - 0.25 * omega ** 2 * H1 * dy / r)


def sample_points(period, ns, y):
    xl = -period / 2.0 + (np.arange(ns) + 0.5) * period / ns
    return np.stack([xl, np.full(ns, y)], axis=1)


def default_samples(disc, omega, period, y0):
    """Samples of the radiation rows' Fourier coefficients: at least 64, and enough that the alias
    kappa_n + 2 pi ns / d of every propagating order decays by e^-37 over the gap g between y = -y0
    and the obstacle: 2 pi ns / d - omega >= sqrt(omega^2 + (37 / g)^2)."""
    g = y0 - float(np.max(np.abs(disc.x[:, 1])))
    return max(64, int(math.ceil((omega + math.sqrt(omega ** 2 + (37.0 / g) ** 2)) * period / (2 * math.pi))))


def radiation_rows(disc, omega, period, alpha, ct, crossed, y0, ns=64, P=0):
    """Rows (c x N for eta, c x 2M for xi) of the radiation conditions of the crossed orders:
    row . [eta; xi] = i k_n U_n(-y0) + U_n'(-y0) of the representation of Eq. 2.14 (Eq. 2.20 with P
    neighbour images), U_n from ns samples on y = -y0 (Remark 2.3)."""
    pts = sample_points(period, ns, -y0)
    xl = pts[:, 0]
    N = disc.N
    M = len(ct.k)
    Re = np.zeros((len(crossed), N), complex)
    Rx = np.zeros((len(crossed), 2 * M), complex)
    for r, (n, kx, kn) in enumerate(crossed):
        f = np.exp(-1j * kx * xl) / ns                   # DFT weights of order n
        for j in range(-P, P + 1):
            src = disc.x + np.array([j * period, 0.0])
            Kv = nystrom.kernel(omega, pts, src, disc.nrm)
            Kd = kernel_dy(omega, pts, src, disc.nrm)
            Re[r] += alpha ** j * (f @ (1j * kn * Kv + Kd)) * disc.w
        for xw, fac, sg in ((-period / 2.0, 1.0, 1.0), (period / 2.0, alpha, -1.0)):
            e = ct.wk[None, :] * np.exp(1j * ct.k[None, :] * (-y0)) * np.exp(1j * ct.s[None, :] * np.abs(xl[:, None] - xw))
            dy = 1j * kn + 1j * ct.k[None, :]             # i k_n + d/dy of e^{i k y}
            Rx[r, :M] += fac * (f @ (0.5j * e / ct.s[None, :] * dy))
            Rx[r, M:] += fac * (f @ (0.5 * sg * e * dy))
    return Re, Rx


def plane_waves(disc, crossed):
    """phi_n = exp(i (kappa_n x + k_n y)) at the nodes (N x c)."""
    x, y = disc.x[:, 0], disc.x[:, 1]
    return np.stack([np.exp(1j * (kx * x + kn * y)) for (n, kx, kn) in crossed], axis=1) if crossed \
        else np.zeros((disc.N, 0), complex)


def radiation_of_waves(crossed, y0):
    """The radiation rows applied to the added waves: i k_n U_n + U_n' of phi_m at y = -y0 is
    2 i k_n e^{-i k_n y0} for m = n and 0 otherwise (orders differ by whole periods, and the ns-point
    DFT separates them when ns exceeds twice the order difference)."""
    return np.diag([2j * kn * np.exp(-1j * kn * y0) for (n, kx, kn) in crossed]).astype(complex)


def solve_wood(disc, omega, period, theta, P=0, quad="kr6", h=0.1, a=1.0, b=1.0, delta=None, ns=None, A0=None,
               crossed=None, y0=None):
    """Dense LU of the bordered system on the displaced contour with the added waves and radiation
    rows: [[A~, B, Phi], [C~, Q, 0], [R_eta, R_xi, R_phi]] [eta; xi; a] = [b; 0; 0]."""
    al = periodic.bloch_phase(omega, period, theta)
    gap = (P + 0.5) * period - float(np.max(np.abs(disc.x[:, 0])))
    K = math.sqrt(omega ** 2 + (37.0 / gap) ** 2)
    if delta is None:
        delta = choose_delta(omega, period, theta, K, a, b)
    ct = displaced_contour(omega, K, h, a, b, delta)
    if crossed is None:
        crossed = crossed_orders(omega, period, theta, delta, a, b)
    if y0 is None:
        y0 = periodic.default_y0(disc)
    if ns is None:
        ns = default_samples(disc, omega, period, y0)
    sysm = periodic.assemble(disc, omega, period, al, ct, P=P, quad=quad, A0=A0)
    Phi = plane_waves(disc, crossed)
    Re, Rx = radiation_rows(disc, omega, period, al, ct, crossed, y0, ns, P)
    Rp = radiation_of_waves(crossed, y0)
    N, M2, c = disc.N, 2 * len(ct.k), len(crossed)
    big = np.block([[sysm.A, sysm.B, Phi], [sysm.C, sysm.Q, np.zeros((M2, c))], [Re, Rx, Rp]])
    rhs = np.zeros((N + M2 + c, 1), complex)
    rhs[:N] = periodic.incident(disc, omega, theta)
    sol = sla.lu_solve(sla.lu_factor(big), rhs)[:, 0]
    return dict(eta=sol[:N], xi=sol[N:N + M2], a=sol[N + M2:], contour=ct, delta=delta, crossed=crossed, y0=y0,
                alpha=al)


def bragg_and_flux(disc, omega, period, theta, eta, y0, k_zero=1e-9):
    """Lattice-sum Bragg amplitudes (``periodic.bragg_lattice``) and the flux error of Remark 6.1.
    A grazing order (|k_n| <= k_zero) carries no flux: its amplitudes are reported as NaN and it is
    left out of the balance."""
    with np.errstate(divide="ignore", invalid="ignore"):
        n, kn, c, d = periodic.bragg_lattice(disc, omega, period, theta, eta, y0)
    keep = np.abs(kn) > k_zero
    c = np.where(keep, c, np.nan)
    d = np.where(keep, d, np.nan)
    eps = periodic.flux_error(omega, theta, n[keep], kn[keep], c[keep], d[keep], y0)
    return n, kn, c, d, eps
