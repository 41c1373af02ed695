"""Pins of the Wood's-anomaly scheme of the oracle (Sec. 2.4, second improvement), CPU only.

What fixes the answer independently of the scheme:
* Away from anomalies the undisplaced scheme is accurate; displacing the contour across a pole
  (propagating or evanescent order) and adding the wave and the radiation row must reproduce its
  solution to rounding.  A wrong added wave (the down-going one) or a radiation row on the wrong
  side (no incoming from above) breaks this (planted mistakes below).
* At the exact anomaly theta = -arccos(1 - 2 pi / (omega d)) (the angle of the paper's Sec. 6.2)
  and next to it, energy is conserved (Remark 6.1), where the undisplaced scheme loses it.
* The solution is continuous through the anomaly, with the square-root rate of k_n.
* Reflection reciprocity between Bloch phases alpha and 1/alpha holds to rounding at the anomaly
  and next to it.
* The y-derivative of the kernel matches finite differences.
"""
import math

import numpy as np
import pytest

import qpinputs
from oracle import nystrom as ny
from oracle import periodic as pq
from oracle import wood

N, OM, D = 400, 10.0, 2 * math.pi
TH_WOOD = -math.acos(1 - 2 * math.pi / (OM * D))


@pytest.fixture(scope="module")
def star():
    disc = ny.Discretization(qpinputs.star(), N)
    return disc, ny.matrix(disc, OM, "kress")


def _undisplaced(disc, A, th, h=0.05):
    return pq.solve_qp(disc, N, OM, D, [th], quad="kress", A0=A, h=h)["eta"][:, 0]


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_kernel_y_derivative_matches_finite_differences():
    rng = np.random.default_rng(2)
    tx = rng.uniform(-2, 2, (5, 2)) + np.array([0.0, -4.0])
    sy = rng.uniform(-1, 1, (7, 2))
    sn = rng.standard_normal((7, 2))
    sn /= np.linalg.norm(sn, axis=1)[:, None]
    h = 1e-5
    e = np.array([0.0, h])
    fd = (ny.kernel(OM, tx + e, sy, sn) - ny.kernel(OM, tx - e, sy, sn)) / (2 * h)
    an = wood.kernel_dy(OM, tx, sy, sn)
    assert np.abs(fd - an).max() < 1e-7 * np.abs(an).max()


@pytest.mark.parametrize("case", ["propagating", "evanescent"])
def test_displaced_contour_reproduces_undisplaced_solution(star, case):
    disc, A = star
    if case == "propagating":
        th, delta = -math.pi / 5, 2.0                 # crosses k_{-18} = 1.34
    else:
        # kappa_1 = omega + 0.02: the evanescent order |k_1| = 0.63 lies under tanh(delta) = 0.96
        th, delta = -math.acos((OM + 0.02 - 1.0) / OM), 2.0
    cr = wood.crossed_orders(OM, D, th, delta)
    assert len(cr) >= 1
    if case == "evanescent":
        assert any(abs(k.real) < 1e-12 and k.imag > 0 for (_, _, k) in cr)
    r = wood.solve_wood(disc, OM, D, th, quad="kress", A0=A, delta=delta, h=0.05)
    assert _rel(r["eta"], _undisplaced(disc, A, th)) < 1e-12
    assert np.all(np.abs(r["a"]) > 1e-6)          # the added waves are really used


def test_planted_down_going_wave_breaks_agreement(star, monkeypatch):
    disc, A = star
    th = -math.pi / 5
    ref = _undisplaced(disc, A, th)
    x, y = disc.x[:, 0], disc.x[:, 1]
    monkeypatch.setattr(wood, "plane_waves", lambda d_, cr: np.stack(
        [np.exp(1j * (kx * x - kn * y)) for (n, kx, kn) in cr], axis=1))
    r = wood.solve_wood(disc, OM, D, th, quad="kress", A0=A, delta=2.0, h=0.05)
    assert _rel(r["eta"], ref) > 1e-6


def test_planted_radiation_row_above_breaks_agreement(star, monkeypatch):
    disc, A = star
    th = -math.pi / 5
    ref = _undisplaced(disc, A, th)
    orig = wood.radiation_rows
    monkeypatch.setattr(wood, "radiation_rows", lambda d_, om, p, al, ct, cr, y0, ns=64, P=0:
                        orig(d_, om, p, al, ct, cr, -y0, ns, P))
    r = wood.solve_wood(disc, OM, D, th, quad="kress", A0=A, delta=2.0, h=0.05)
    assert _rel(r["eta"], ref) > 1e-6


def test_exact_wood_angle_conserves_energy(star):
    disc, A = star
    _, _, kn = pq.bragg_orders(OM, D, TH_WOOD)
    assert np.min(np.abs(kn)) < 1e-6                 # a grazing order exists
    r = wood.solve_wood(disc, OM, D, TH_WOOD, quad="kress", A0=A)
    assert len(r["crossed"]) >= 1
    n, kn, c, d, eps = wood.bragg_and_flux(disc, OM, D, TH_WOOD, r["eta"], r["y0"])
    assert eps < 1e-12
    # the contour's own convergence: half the spacing gives the same solution
    r2 = wood.solve_wood(disc, OM, D, TH_WOOD, quad="kress", A0=A, h=0.05)
    assert _rel(r["eta"], r2["eta"]) < 1e-12


def test_near_wood_displaced_conserves_energy_where_undisplaced_fails(star):
    disc, A = star
    th = TH_WOOD + 1e-3                               # smallest |k_n| about 0.3
    und = pq.solve_qp(disc, N, OM, D, [th], quad="kress", A0=A)
    assert und["flux"][0] > 1e-9
    r = wood.solve_wood(disc, OM, D, th, quad="kress", A0=A)
    assert wood.bragg_and_flux(disc, OM, D, th, r["eta"], r["y0"])[4] < 1e-12


def test_continuity_through_the_anomaly(star):
    """|eta(theta_W + e) - eta(theta_W)| shrinks like sqrt(e) (k_n ~ sqrt(e))."""
    disc, A = star
    r0 = wood.solve_wood(disc, OM, D, TH_WOOD, quad="kress", A0=A)["eta"]
    d1 = _rel(wood.solve_wood(disc, OM, D, TH_WOOD + 1e-4, quad="kress", A0=A)["eta"], r0)
    d2 = _rel(wood.solve_wood(disc, OM, D, TH_WOOD + 1e-6, quad="kress", A0=A)["eta"], r0)
    assert d2 < d1 < 0.5
    assert 5.0 < d1 / d2 < 20.0                        # 100x smaller step, about 10x closer


@pytest.mark.parametrize("offset", [0.0, 1e-3])
def test_reciprocity_at_and_next_to_the_anomaly(star, offset):
    """Reflection reciprocity k_p^a c_p^a = k_p^b c_p^b (amplitudes referred to y = 0) between an
    angle a at (or next to) the anomaly and the angle b whose incidence reverses a's order p = -1;
    b then sits at the mirrored anomaly.  Both are solved on their displaced contours, and the
    relation holds to rounding (the derivation is in test_oracle_reciprocity.py)."""
    disc, A = star
    tha, p = TH_WOOD + offset, -1
    kap = OM * math.cos(tha) + 2 * math.pi * p / D
    thb = -math.acos(-kap / OM)
    vals = []
    for th in (tha, thb):
        r = wood.solve_wood(disc, OM, D, th, quad="kress", A0=A)
        n, kn, c, d, eps = wood.bragg_and_flux(disc, OM, D, th, r["eta"], r["y0"])
        i = int(np.nonzero(n == p)[0][0])
        vals.append(kn[i] * c[i] * np.exp(-1j * kn[i] * r["y0"]))
    assert abs(vals[0] - vals[1]) < 1e-12 * abs(vals[0])
