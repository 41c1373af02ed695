"""Pins of the transmission oracle (Sec. 5) against what the mathematics fixes, not against itself:

* the four difference kernels (with the normalization kb = max(omega, n omega)) and the exterior
  rows against central differences of G_k = (i/4) H0(k r);
* an exact solution of the isolated matching problem: a radiating point source at wavenumber
  omega from inside Omega and a regular field at n omega from a source outside, whose jumps are
  the data; the represented fields reproduce both sources at the discretization's order (this pins
  the jump signs, the 2 x 2 blocks, the interlacing and the Kapur-Rokhlin weights of all four);
* index n = 1: the obstacle is invisible, the operator is the identity and every Bragg amplitude
  vanishes (this pins the incident data, the exterior representation and C against each other);
* energy balance (Remark 6.1) on the paper's d = 1 grating at index 1.5, converging at the
  quadrature's order (this pins B, Q and the Bragg formula);
* P = 0 and P = 1 give the same density (pins the exterior-only images and C~);
* Bragg amplitudes sampled from the field (through xi) equal the lattice sums (eta only);
* planted mistakes (a flipped sign in B's derivative rows, swapped columns of C) break the pins.
"""
import math

import numpy as np
import pytest
from scipy.special import hankel1

import qpinputs
from oracle import nystrom, periodic
from oracle import transmission as tr

OM, IDX = 10.0, 1.5


def _g(k, x, y):
    return 0.25j * hankel1(0, k * math.hypot(x[0] - y[0], x[1] - y[1]))


def test_kernels_match_finite_differences():
    x, y = np.array([0.3, -0.2]), np.array([-0.15, 0.4])
    nx = np.array([math.cos(0.7), math.sin(0.7)])
    ny = np.array([math.cos(2.1), math.sin(2.1)])
    hd = 1e-4
    want = []
    for k in (OM, IDX * OM):
        def g(a, b):
            return _g(k, a, b)
        dgy = (g(x, y + hd * ny) - g(x, y - hd * ny)) / (2 * hd)
        dgx = (g(x + hd * nx, y) - g(x - hd * nx, y)) / (2 * hd)
        T = (g(x + hd * nx, y + hd * ny) - g(x + hd * nx, y - hd * ny)
             - g(x - hd * nx, y + hd * ny) + g(x - hd * nx, y - hd * ny)) / (4 * hd * hd)
        want.append((dgy, g(x, y), T, dgx))
    (d0, s0, t0, x0), (d1, s1, t1, x1) = want
    kb = IDX * OM
    got = tr.kernels(OM, IDX * OM, x[None], nx[None], y[None], ny[None])
    for a, b in zip(got, (d0 - d1, kb * (s0 - s1), -(t0 - t1) / kb, -(x0 - x1))):
        assert abs(a[0, 0] - b) < 1e-6 * max(1.0, abs(b))
    # the exterior rows alone (images and walls)
    got = tr.exterior_kernels(OM, kb, x[None], nx[None], y[None], ny[None])
    for a, b in zip(got, (d0, kb * s0, -t0 / kb, -x0)):
        assert abs(a[0, 0] - b) < 1e-6 * max(1.0, abs(b))


def _point_source_error(N):
    cur = qpinputs.star(1.0, 0.3, 5)
    d = nystrom.Discretization(cur, N)
    zi, zo = np.array([0.1, 0.2]), np.array([2.0, 1.5])
    k1 = IDX * OM

    def G(k, x, z):
        return 0.25j * hankel1(0, k * np.hypot(x[:, 0] - z[0], x[:, 1] - z[1]))

    def dG(k, x, nr, z):
        dx = x - z
        r = np.hypot(dx[:, 0], dx[:, 1])
        return -0.25j * k * hankel1(1, k * r) * (nr[:, 0] * dx[:, 0] + nr[:, 1] * dx[:, 1]) / r

    f = G(OM, d.x, zi) - G(k1, d.x, zo)
    g = dG(OM, d.x, d.nrm, zi) - dG(k1, d.x, d.nrm, zo)
    kb = tr.kbar(OM, IDX)
    eta = tr.solve_isolated(d, OM, IDX, tr.rhs_from_jumps(f, g, kb))
    te = np.array([[1.8, -1.2], [-2.5, 0.3], [0.0, 1.9]])
    ti = np.array([[0.2, -0.1], [-0.3, 0.25], [0.4, 0.4]])
    ee = np.abs(tr.potential(d, OM, kb, eta, te) - G(OM, te, zi)).max()
    ei = np.abs(tr.potential(d, k1, kb, eta, ti) - G(k1, ti, zo)).max()
    return max(ee, ei)


def test_point_sources_reproduced_at_sixth_order():
    e4, e8 = _point_source_error(400), _point_source_error(800)
    assert e8 < 2e-6
    assert math.log2(e4 / e8) > 5.0


def test_index_one_is_invisible():
    d = nystrom.Discretization(qpinputs.star(1.0, 0.3, 5), 200)
    A = tr.matrix(d, OM, 1.0)
    assert np.abs(A - np.eye(2 * d.N)).max() < 1e-14
    r = tr.solve_qp(d, 200, OM, 1.0, 2 * math.pi, [-math.pi / 5, -1.1], P=0)
    for (_, _, c, dd) in r["bragg"]:
        assert np.abs(c).max() < 1e-9 and np.abs(dd).max() < 1e-9


def test_flux_balance_converges_on_the_d1_grating():
    wl = qpinputs.workload("star_d1")
    f = [tr.solve_qp(wl.curve, N, wl.omega, IDX, wl.period, wl.thetas, P=1)["flux"][0] for N in (400, 800)]
    assert f[1] < 1e-7
    assert math.log2(f[0] / f[1]) > 5.0


@pytest.fixture(scope="module")
def star2pi():
    d = nystrom.Discretization(qpinputs.star(1.0, 0.3, 5), 240)
    ths = [-math.pi / 5, -1.2]
    return d, ths, tr.solve_qp(d, 240, OM, IDX, 2 * math.pi, ths, P=0), tr.solve_qp(d, 240, OM, IDX, 2 * math.pi, ths, P=1)


def test_P0_equals_P1(star2pi):
    _, _, r0, r1 = star2pi
    assert np.abs(r0["eta"] - r1["eta"]).max() / np.abs(r0["eta"]).max() < 1e-11


def test_bragg_sampled_equals_lattice(star2pi):
    d, ths, r0, _ = star2pi
    for q, th in enumerate(ths):
        al = periodic.bloch_phase(OM, 2 * math.pi, th)
        _, _, c, dd = r0["bragg"][q]
        _, _, cs, ds = tr.bragg_sampled(d, OM, IDX, 2 * math.pi, al, r0["contour"], th, r0["eta"][:, q], r0["xi"][:, q],
                                        r0["y0"])
        assert np.abs(cs - c).max() < 1e-12 and np.abs(ds - dd).max() < 1e-12


def test_rows_agree_with_matrices():
    d = nystrom.Discretization(qpinputs.star(1.0, 0.3, 5), 60)
    rows = np.array([0, 1, 7, 64, 119, 118])
    assert np.array_equal(tr.matrix_rows(d, OM, IDX, rows), tr.matrix(d, OM, IDX)[rows])
    assert np.array_equal(tr.neighbour_rows(d, OM, IDX, 2.5, rows), tr.neighbour_matrix(d, OM, IDX, 2.5)[rows])


def test_planted_mistakes_break_the_pins(monkeypatch):
    wl = qpinputs.workload("star_d1")
    ok = tr.solve_qp(wl.curve, 300, wl.omega, IDX, wl.period, wl.thetas, P=1)["flux"][0]
    orig_B, orig_C = tr.wall_B, tr.wall_C

    def bad_B(*a, **k):
        BL, BR = orig_B(*a, **k)
        BL, BR = BL.copy(), BR.copy()
        BL[1::2] *= -1
        BR[1::2] *= -1
        return BL, BR

    monkeypatch.setattr(tr, "wall_B", bad_B)
    fb = tr.solve_qp(wl.curve, 300, wl.omega, IDX, wl.period, wl.thetas, P=1)["flux"][0]
    monkeypatch.setattr(tr, "wall_B", orig_B)

    def bad_C(*a, **k):
        return tuple(np.ascontiguousarray(C.reshape(C.shape[0], -1, 2)[:, :, ::-1].reshape(C.shape)) for C in orig_C(*a, **k))

    monkeypatch.setattr(tr, "wall_C", bad_C)
    fc = tr.solve_qp(wl.curve, 300, wl.omega, IDX, wl.period, wl.thetas, P=1)["flux"][0]
    assert ok < 1e-5
    assert fb > 1e3 * ok and fc > 1e3 * ok
