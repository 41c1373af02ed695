"""Reciprocity of the grating's reflection coefficients, a pin of both oracles that the energy
balance cannot give (it sees only moduli, this sees phases and the Bloch-phase dependence).

Take two solutions of the same problem (Sec. 2 for the Dirichlet obstacle, Sec. 5 for the
transmission one): a with incidence kappa_a = omega cos(theta_a), and b with incidence
kappa_b = -(kappa_a + 2 pi p / d), the reverse of a's reflected order p.  Their Bloch phases are
alpha and 1 / alpha, so u_a u_b is periodic and Green's second identity over one period cell of the
strip |y| < Y loses its wall terms.  On the obstacle it loses its boundary term: u = 0 there, or u
and its normal derivative are continuous into one interior medium shared by both fields.  Below the
grating only down-going waves meet, and their Wronskians vanish.  Above it, the incident wave of each
field meets the reflected order p of the other.  With the amplitudes c_n of the reflected orders
(Eq. 2.5) referred to y = 0, that leaves k_p^a c_p^a = k_p^b c_p^b, k_n the vertical wavenumber
of order n.  The oracle's amplitudes are referred to y = y0, hence the factors exp(-i k_n y0).

The paper's d = 1 star grating of Sec. 6.1 with P = 1 images (theta_a = -pi/5, p = -1): the
relation holds to the discretization's error, which falls at the quadrature's order.
"""
import math

import numpy as np
import pytest

import qpinputs
from oracle import periodic as pq
from oracle import transmission as tr


def _reciprocity_gap(solve, omega, period, theta_a, p):
    kap = omega * math.cos(theta_a) + 2 * math.pi * p / period
    theta_b = -math.acos(-kap / omega)
    r = solve([theta_a, theta_b])
    vals = []
    for q in range(2):
        n, kn, c, _ = r["bragg"][q]
        i = int(np.nonzero(n == p)[0][0])
        assert abs(kn[i].imag) == 0.0  # a propagating order
        vals.append(kn[i] * c[i] * np.exp(-1j * kn[i] * r["y0"]))
    return abs(vals[0] - vals[1]) / abs(vals[0])


@pytest.mark.parametrize("problem", ["dirichlet", "transmission"])
def test_reflection_reciprocity_on_the_d1_grating(problem):
    wl = qpinputs.workload("star_d1")

    def solver(N):
        if problem == "dirichlet":
            return lambda ths: pq.solve_qp(wl.curve, N, wl.omega, wl.period, ths, P=1)
        return lambda ths: tr.solve_qp(wl.curve, N, wl.omega, 1.5, wl.period, ths, P=1)

    g = [_reciprocity_gap(solver(N), wl.omega, wl.period, -math.pi / 5, -1) for N in (256, 512)]
    assert g[1] < (1e-7 if problem == "dirichlet" else 2e-6), g
    assert math.log2(g[0] / g[1]) > 5.0, g


def test_planted_phase_error_passes_energy_balance_but_breaks_reciprocity(monkeypatch):
    """Amplitudes referred to the wrong height (-y0 instead of y0) keep every modulus, so the energy
    balance still holds, while reciprocity fails."""
    wl = qpinputs.workload("star_d1")
    orig = pq.bragg_lattice

    def shifted(disc, omega, period, theta, eta, y0):
        n, kn, c, d = orig(disc, omega, period, theta, eta, y0)
        return n, kn, c * np.exp(-2j * kn * y0), d

    solve = lambda ths: pq.solve_qp(wl.curve, 512, wl.omega, wl.period, ths, P=1)
    ok = _reciprocity_gap(solve, wl.omega, wl.period, -math.pi / 5, -1)
    monkeypatch.setattr(pq, "bragg_lattice", shifted)
    r = solve([-math.pi / 5])
    bad = _reciprocity_gap(solve, wl.omega, wl.period, -math.pi / 5, -1)
    assert r["flux"][0] < 1e-6 and ok < 1e-7
    assert bad > 1e-2


@pytest.mark.parametrize("quad", ["kress", "alpert"])
def test_reflection_reciprocity_with_high_order_quadratures(quad):
    """Kress's spectral rule meets the relation to rounding at N = 128; Alpert's hybrid rule to
    about 5e-13 at N = 256 (Dirichlet, the same grating and angles)."""
    from oracle import alpert
    from oracle import nystrom as ny
    wl = qpinputs.workload("star_d1")
    N = 128 if quad == "kress" else 256
    disc = ny.Discretization(wl.curve, N)
    A0 = ny.matrix(disc, wl.omega, "kress") if quad == "kress" else alpert.matrix_alpert(disc, wl.omega, wl.curve)
    solve = lambda ths: pq.solve_qp(disc, N, wl.omega, wl.period, ths, P=1, A0=A0)
    g = _reciprocity_gap(solve, wl.omega, wl.period, -math.pi / 5, -1)
    assert g < (1e-12 if quad == "kress" else 5e-12), g
