"""Checks of a computed solution at sizes where the dense oracle does not fit (oracle side).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).

At N = 1e5 the dense Nystrom matrix needs 160 GB, so a solution (eta, xi) of the bordered
system of Eq. 2.19 is judged by sampled rows of its residual

    r1 = A~ eta + B xi - b     (rows of the obstacle block: Sec. 2.2, discretized as in Sec. 2.3)
    r2 = C eta + Q xi          (every wall row: Eqs. 2.17-2.18 on the Sommerfeld contour)

with exact dense rows of A (``nystrom.matrix_kr6_rows``), B and b on the sampled nodes and all of
C and Q (accumulated over node chunks), and by the energy balance of Remark 6.1.  The residual is
relative to |b|, with the sampled obstacle rows scaled up to all N rows; it is a residual of the
bordered system, not a forward error.
"""
from __future__ import annotations

import math

import numpy as np

from . import alpert
from . import nystrom
from . import periodic
from . import transmission


class RowSubset:
    """The nodes ``rows`` of a discretization (for B, b and C restricted to them)."""

    def __init__(self, disc: nystrom.Discretization, rows):
        rows = np.asarray(rows)
        self.N = len(rows)
        self.x = disc.x[rows]
        self.nrm = disc.nrm[rows]
        self.w = disc.w[rows]


def bordered_residual(curve, N, omega, period, thetas, eta, xi, flux=None, n_rows=48, n_ang=8, chunk=4000,
                      seed=7, angles=None, P=0, h=0.1, quad="kr6"):
    """Sampled relative residual of the bordered system (KR6 or, with quad="alpert", Alpert quadrature; Eq. 2.19, or Eq. 2.21 with
    P = 1 neighbour images: A~ = A + alpha A_1 + alpha^-1 A_-1 and C~ of Sec. 2.4) for the solutions
    eta (N x n) and xi (2M x n) of the angles ``thetas`` (n), M from the default contour of spacing h.

    n_rows obstacle rows and n_ang angles are drawn from rng(seed) (or ``angles`` given).
    Returns dict(sampled_rel_residual = max over the sampled angles of
    sqrt(|r1|^2 N / n_rows + |r2|^2) / |b|, flux_err_max over every angle when ``flux`` is given,
    rows_sampled, angles_sampled)."""
    disc = nystrom.Discretization(curve, N)
    if P not in (0, 1):
        raise ValueError("P must be 0 or 1")
    ct = periodic.default_contour(disc, omega, period, P=P, h=h)
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(N, n_rows, replace=False))
    angs = np.asarray(angles) if angles is not None else rng.choice(len(thetas), n_ang, replace=False)
    if quad not in ("kr6", "alpert"):
        raise ValueError("quad must be 'kr6' or 'alpert'")
    Arows = (nystrom.matrix_kr6_rows(disc, omega, rows) if quad == "kr6"
             else alpert.matrix_alpert_rows(disc, omega, curve, rows))
    Anb = {j: nystrom.neighbour_rows(disc, omega, j * period, rows) for j in ((-1, 1) if P else ())}
    sub = RowSubset(disc, rows)
    BL, BR = periodic.wall_B(sub, omega, period, ct)
    eta_s = eta[:, angs]
    CLe = 0
    CRe = 0
    for c0 in range(0, N, chunk):
        sl = np.arange(c0, min(N, c0 + chunk))
        CL, _ = periodic.wall_C(RowSubset(disc, sl), omega, period, ct, shift=P * period)
        _, CR = periodic.wall_C(RowSubset(disc, sl), omega, period, ct, shift=-P * period)
        CLe = CLe + CL @ eta_s[sl]
        CRe = CRe + CR @ eta_s[sl]
    worst = 0.0
    for q, a in enumerate(angs):
        th = thetas[a]
        al = periodic.bloch_phase(omega, period, th)
        x = xi[:, a]
        b = periodic.incident(sub, omega, th)[:, 0]
        At = Arows + sum(al ** j * Anb[j] for j in Anb)
        r1 = At @ eta_s[:, q] + (BL + al * BR) @ x - b
        r2 = al ** P * CLe[:, q] - al ** (-(P + 1)) * CRe[:, q] + periodic.wall_Q(omega, period, al, ct) @ x
        bn = np.linalg.norm(periodic.incident(disc, omega, th))
        worst = max(worst, math.sqrt(np.sum(np.abs(r1) ** 2) * N / n_rows + np.sum(np.abs(r2) ** 2)) / bn)
    out = {"sampled_rel_residual": float(worst), "rows_sampled": int(n_rows), "angles_sampled": int(len(angs))}
    if flux is not None:
        out["flux_err_max"] = float(np.max(flux))
    return out


def bordered_residual_tr(curve, N, omega, index, period, thetas, eta, xi, flux=None, n_rows=48, n_ang=8, chunk=4000,
                         seed=7, angles=None, P=0, h=0.1):
    """The same sampled residual for the transmission problem of Sec. 5 (``transmission``): eta is
    2N x n, interlaced; n_rows nodes are drawn and both of their rows (value and normal-derivative
    jumps) are checked, with A~ = A + alpha A_1 + alpha^-1 A_-1 for P = 1 (exterior field only)."""
    disc = nystrom.Discretization(curve, N)
    if P not in (0, 1):
        raise ValueError("P must be 0 or 1")
    ct = periodic.default_contour(disc, omega, period, P=P, h=h)
    rng = np.random.default_rng(seed)
    nodes = np.sort(rng.choice(N, n_rows, replace=False))
    rows = np.stack([2 * nodes, 2 * nodes + 1], axis=1).ravel()
    angs = np.asarray(angles) if angles is not None else rng.choice(len(thetas), min(n_ang, len(thetas)), replace=False)
    Arows = transmission.matrix_rows(disc, omega, index, rows)
    Anb = {j: transmission.neighbour_rows(disc, omega, index, j * period, rows) for j in ((-1, 1) if P else ())}
    sub = RowSubset(disc, nodes)
    BL, BR = transmission.wall_B(sub, omega, index, period, ct)
    eta_s = eta[:, angs]
    CLe = 0
    CRe = 0
    for c0 in range(0, N, chunk):
        sl = np.arange(c0, min(N, c0 + chunk))
        us = np.stack([2 * sl, 2 * sl + 1], axis=1).ravel()
        CL, _ = transmission.wall_C(RowSubset(disc, sl), omega, index, period, ct, shift=P * period)
        _, CR = transmission.wall_C(RowSubset(disc, sl), omega, index, period, ct, shift=-P * period)
        CLe = CLe + CL @ eta_s[us]
        CRe = CRe + CR @ eta_s[us]
    worst = 0.0
    for q, a in enumerate(angs):
        th = thetas[a]
        al = periodic.bloch_phase(omega, period, th)
        x = xi[:, a]
        b = transmission.incident(sub, omega, index, th)[:, 0]
        At = Arows + sum(al ** j * Anb[j] for j in Anb)
        r1 = At @ eta_s[:, q] + (BL + al * BR) @ x - b
        r2 = al ** P * CLe[:, q] - al ** (-(P + 1)) * CRe[:, q] + periodic.wall_Q(omega, period, al, ct) @ x
        bn = np.linalg.norm(transmission.incident(disc, omega, index, th))
        worst = max(worst, math.sqrt(np.sum(np.abs(r1) ** 2) * N / n_rows + np.sum(np.abs(r2) ** 2)) / bn)
    out = {"sampled_rel_residual": float(worst), "rows_sampled": int(2 * n_rows), "angles_sampled": int(len(angs))}
    if flux is not None:
        out["flux_err_max"] = float(np.max(flux))
    return out
