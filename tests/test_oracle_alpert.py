"""Pins of the oracle's Alpert-corrected quadrature (Sec. 2.3, the alternative to Kapur-Rokhlin)
against what the mathematics fixes: a closed-form logarithmic integral and its convergence order,
the closed-form spectrum of the circle (order of the whole Nystrom matrix), an exterior point
source, and planted mistakes in the correction's conditions."""
import math

import numpy as np
import pytest

import qpinputs
from oracle import alpert as al
from oracle import nystrom as ny
from oracle import periodic as pq


def _closed(N, mm, x, w, a):
    """Corrected rule for int_0^{2pi} [ln(4 sin^2(t/2)) + 1] cos(m t) dt = -2 pi / m, singular at t = 0."""
    h = 2 * math.pi / N
    k = np.arange(N)
    k = np.where(k > N // 2, k - N, k)
    keep = np.abs(k) >= a
    f = lambda tt: (np.log(4 * np.sin(tt / 2) ** 2) + 1.0) * np.cos(mm * tt)
    v = h * np.sum(f(k[keep] * h))
    for j in range(len(x)):
        v += h * w[j] * (f(x[j] * h) + f(-x[j] * h))
    return v


def test_rule_nodes_inside_and_weights_positive():
    x, w = al.rule()
    assert np.all(x > 0) and np.all(x < al.A_DEFAULT) and np.all(w > 0)
    assert np.all(np.diff(x) > 0)


@pytest.mark.parametrize("mm", [1, 3])
def test_closed_form_log_integral_order(mm):
    x, w = al.rule()
    errs = [abs(_closed(N, mm, x, w, al.A_DEFAULT) + 2 * math.pi / mm) for N in (32, 64)]
    assert math.log2(errs[0] / errs[1]) > 10.0          # O(h^11 ln h)
    assert abs(_closed(128, mm, x, w, al.A_DEFAULT) + 2 * math.pi / mm) < 1e-12


def test_circle_spectrum_order():
    """A e^{int} = lambda_n e^{int} on the circle (closed form); the Alpert-corrected matrix reaches
    it at order about 10 (KR6: about 6)."""
    c = qpinputs.circle(1.0)
    errs = []
    for N in (128, 256):
        disc = ny.Discretization(c, N)
        A = al.matrix_alpert(disc, 10.0, c)
        e = 0.0
        for n in (0, 3, 7):
            v = np.exp(1j * n * disc.t)
            e = max(e, np.abs(A @ v - ny.circle_eigenvalue(10.0, 1.0, n) * v).max())
        errs.append(e)
    assert errs[1] < 1e-9
    assert math.log2(errs[0] / errs[1]) > 9.0


def test_point_source_exterior_field_star():
    """u = G(x - x_s) with x_s inside the star solves the exterior Dirichlet problem; the combined
    field solution eta of A eta = u|_boundary reproduces it outside.  The Alpert-corrected solve
    converges at order about 10 (400 -> 800 nodes) and beats KR6 by orders of magnitude."""
    c = qpinputs.star()
    om = 10.0
    xs = np.array([[0.3 * math.cos(0.4), 0.3 * math.sin(0.4)]])
    tgt = np.array([[2.5, 0.5], [-2.0, 1.7], [0.3, -2.8]])
    exact = ny.green(om, tgt, xs)[:, 0]
    errs = {}
    for N in (400, 800):
        disc = ny.Discretization(c, N)
        f = ny.green(om, disc.x, xs)[:, 0]
        for name, A in (("alpert", al.matrix_alpert(disc, om, c)), ("kr6", ny.matrix_kr6(disc, om))):
            eta = np.linalg.solve(A, f)
            errs[name, N] = np.abs(ny.potential(disc, om, eta, tgt) - exact).max() / np.abs(exact).max()
    assert errs["alpert", 800] < 1e-11
    assert math.log2(errs["alpert", 400] / errs["alpert", 800]) > 9.0
    assert errs["alpert", 400] < 1e-3 * errs["kr6", 400]


@pytest.mark.parametrize("plant", ["sign of zeta'(-2q)", "zeta(0) dropped"])
def test_planted_mistakes_break_the_rule(monkeypatch, plant):
    """Plausible slips in the conditions: the alternating sign of zeta'(-2q) lost, or the zeta(0)
    term of the p = 0 moment dropped.  Either the equations lose their solution or the rule misses
    the closed-form integral by far more than its error."""
    if plant.startswith("sign"):
        orig = al.zeta_prime_minus
        monkeypatch.setattr(al, "zeta_prime_minus", lambda p: orig(p) if p == 0 else abs(orig(p)))
    else:
        monkeypatch.setattr(al, "zeta_minus", lambda p: 0)
    try:
        x, w = al.rule.__wrapped__(al.M_DEFAULT, al.A_DEFAULT, 30)
    except (RuntimeError, ZeroDivisionError):
        return
    err = abs(_closed(128, 3, x, w, al.A_DEFAULT) + 2 * math.pi / 3)
    assert err > 1e-6


def test_alpert_qp_solution_flux_balance():
    """The quasi-periodic solve with the Alpert-corrected A conserves energy (Remark 6.1)."""
    wl = qpinputs.workload("star")
    disc = ny.Discretization(wl.curve, 800)
    A = al.matrix_alpert(disc, wl.omega, wl.curve)
    r = pq.solve_qp(disc, 800, wl.omega, wl.period, wl.thetas, A0=A)
    assert r["flux"][0] < 1e-11


def test_alpert_rows_equal_full_matrix_rows():
    c = qpinputs.wavy(130102, 20, 0.3)
    disc = ny.Discretization(c, 200)
    A = al.matrix_alpert(disc, 20.0, c)
    rows = np.array([0, 1, 5, 100, 198, 199])
    assert np.array_equal(al.matrix_alpert_rows(disc, 20.0, c, rows), A[rows])


def test_residual_checker_alpert_rows():
    """The sampled residual with Alpert rows is at rounding level for the oracle's own Alpert solution,
    and far from it for the KR6 solution of the same problem (the two discretizations differ)."""
    from oracle import checks
    c = qpinputs.star()
    N, om, d = 400, 10.0, 2 * math.pi
    th = np.array([-0.7, -1.1])
    disc = ny.Discretization(c, N)
    r = pq.solve_qp(disc, N, om, d, th, A0=al.matrix_alpert(disc, om, c))
    v = checks.bordered_residual(c, N, om, d, th, r["eta"], r["xi"], n_rows=30, n_ang=2, chunk=100, quad="alpert")
    assert v["sampled_rel_residual"] < 1e-12
    r6 = pq.solve_qp(c, N, om, d, th, quad="kr6")
    v6 = checks.bordered_residual(c, N, om, d, th, r6["eta"], r6["xi"], n_rows=30, n_ang=2, chunk=100, quad="alpert")
    assert v6["sampled_rel_residual"] > 1e-8

