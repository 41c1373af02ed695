"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: closed-form
integrals, the closed-form spectrum of the circle, exact exterior solutions, and
invariants of the scattering problem (energy balance, two independent Bragg
extractions, the P = 0 / P = 1 representations, two solution routes).  The
planted-mistake tests show that a plausible misprint (the printed Q of Eq. 2.18,
the printed C~ of Sec. 2.4, missing end corrections) fails these pins.
"""
import math

import numpy as np
import pytest

import qpinputs
from oracle import nystrom as ny
from oracle import periodic as pq
from oracle import quadrature as qd


# ---------------------------------------------------------------- quadrature

def test_kr6_sum_rule_and_sign_pattern():
    g = qd.kr6_corrections()
    assert abs(g.sum() - 0.5) < 1e-13
    assert list(np.sign(g)) == [1, -1, 1, -1, 1, -1]


def _kr6_integral(f_log, f_smooth, N):
    """Corrected punctured trapezoid for int_0^{2pi} [f_log(t) ln(4 sin^2(t/2)) + f_smooth(t)] dt,
    singular node at t = 0 (Sec. 2.3 rule)."""
    R = qd.kr6_band(N)
    t = 2 * math.pi * np.arange(N) / N
    tt = t.copy()
    tt[0] = 1.0
    vals = f_log(t) * np.log(4 * np.sin(tt / 2) ** 2) + f_smooth(t)
    vals[0] = 0.0
    return (2 * math.pi / N) * np.sum(R * vals)


@pytest.mark.parametrize("m", [1, 3])
def test_kr6_closed_form_log_integral(m):
    # int_0^{2pi} ln(4 sin^2(t/2)) cos(m t) dt = -2 pi / m  and  int cos(mt) = 0.
    exact = -2 * math.pi / m
    errs = []
    for N in (64, 128, 256):
        v = _kr6_integral(lambda t: np.cos(m * t), lambda t: np.cos(m * t), N)
        errs.append(abs(v - exact))
    assert errs[-1] < 1e-7
    order = math.log2(errs[0] / errs[1])
    assert order > 6.0


def test_kress_weights_exact_on_trig_polynomials():
    N = 64
    n = N // 2
    R = qd.kress_log_weights(N)
    t = 2 * math.pi * np.arange(N) / N
    for m in (0, 1, 5, n - 1):
        f = np.cos(m * t)
        # sum_j R(t_0 - t_j) f(t_j) = int ln(4 sin^2((0 - tau)/2)) cos(m tau) d tau
        approx = np.sum(R[(0 - np.arange(N)) % N] * f)
        exact = 0.0 if m == 0 else -2 * math.pi / m
        assert abs(approx - exact) < 1e-12


# ---------------------------------------------------------------- the matrix A

@pytest.mark.parametrize("modes", [[0, 1, 4, 9, -6]])
def test_kress_matrix_circle_spectrum(modes):
    om, R = 10.0, 1.0
    d = ny.Discretization(qpinputs.circle(R), 160)
    A = ny.matrix(d, om, "kress")
    for n in modes:
        v = np.exp(1j * n * d.t)
        lam = ny.circle_eigenvalue(om, R, n)
        assert np.abs(A @ v - lam * v).max() < 1e-13 * max(1.0, abs(lam))


def test_kr6_matrix_circle_spectrum_order():
    om, R = 10.0, 1.3
    errs = []
    for N in (200, 400):
        d = ny.Discretization(qpinputs.circle(R), N)
        A = ny.matrix(d, om, "kr6")
        e = 0.0
        for n in (0, 3, 11):
            v = np.exp(1j * n * d.t)
            e = max(e, np.abs(A @ v - ny.circle_eigenvalue(om, R, n) * v).max())
        errs.append(e)
    assert errs[1] < 2e-4
    assert math.log2(errs[0] / errs[1]) > 5.5


def test_circle_eigenvalue_closed_form_vs_direct_quadrature():
    """The closed form itself against brute-force quadrature of the off-diagonal kernel
    with a log-free smooth part (mode 0 on a circle, many points, Kress)."""
    om, R = 7.0, 0.8
    d = ny.Discretization(qpinputs.circle(R), 400)
    A = ny.matrix(d, om, "kress")
    lam_num = (A @ np.ones(d.N))[0]
    assert abs(lam_num - ny.circle_eigenvalue(om, R, 0)) < 1e-12


def _point_source_error(curve, N, om, quad):
    d = ny.Discretization(curve, N)
    A = ny.matrix(d, om, quad)
    ts = 0.4
    r0 = curve.radius(ts)[0]
    src = np.array([[0.3 * r0 * math.cos(ts), 0.3 * r0 * math.sin(ts)]])
    f = ny.green(om, d.x, src)[:, 0]
    eta = np.linalg.solve(A, f)
    tg = np.array([[2.5, 0.3], [-1.0, 2.2], [0.4, -2.4]])
    u = ny.potential(d, om, eta, tg)
    ue = ny.green(om, tg, src)[:, 0]
    return np.abs(u - ue).max() / np.abs(ue).max()


def test_point_source_kress_star():
    assert _point_source_error(qpinputs.star(), 200, 10.0, "kress") < 1e-12


def test_point_source_kr6_star():
    assert _point_source_error(qpinputs.star(), 800, 10.0, "kr6") < 2e-5


# ---------------------------------------------------------------- quasi-periodic system

@pytest.fixture(scope="module")
def star_qp():
    wl = qpinputs.workload("star")
    r = pq.solve_qp(wl.curve, 400, wl.omega, wl.period, wl.thetas, quad="kress")
    return wl, r


def test_flux_balance(star_qp):
    wl, r = star_qp
    assert r["flux"][0] < 1e-12


def test_bragg_sampled_vs_lattice(star_qp):
    wl, r = star_qp
    th = wl.thetas[0]
    al = pq.bloch_phase(wl.omega, wl.period, th)
    n, kn, c, d = r["bragg"][0]
    _, _, c2, d2 = pq.bragg_sampled(r["disc"], wl.omega, wl.period, al, r["contour"], th,
                                    r["eta"][:, 0], r["xi"][:, 0], r["y0"])
    assert np.abs(c - c2).max() < 1e-12
    assert np.abs(d - d2).max() < 1e-12


def test_schur_route_matches_bordered_lu(star_qp):
    wl, r = star_qp
    th = wl.thetas[0]
    al = pq.bloch_phase(wl.omega, wl.period, th)
    s = pq.assemble(r["disc"], wl.omega, wl.period, al, r["contour"], quad="kress")
    eta, xi = pq.solve_schur(s, pq.incident(r["disc"], wl.omega, th))
    assert np.abs(eta[:, 0] - r["eta"][:, 0]).max() < 1e-12 * np.abs(r["eta"]).max()


def test_neighbour_images_same_solution(star_qp):
    wl, r = star_qp
    r1 = pq.solve_qp(r["disc"], 400, wl.omega, wl.period, wl.thetas, quad="kress", P=1)
    assert np.abs(r1["eta"] - r["eta"]).max() < 1e-12 * np.abs(r["eta"]).max()
    assert r1["flux"][0] < 1e-12


def test_contour_self_convergence(star_qp):
    wl, r = star_qp
    r2 = pq.solve_qp(r["disc"], 400, wl.omega, wl.period, wl.thetas, quad="kress", h=0.05)
    assert np.abs(r2["eta"] - r["eta"]).max() < 1e-12 * np.abs(r["eta"]).max()


# ---------------------------------------------------------------- planted mistakes

def test_planted_printed_Q_fails_flux(star_qp, monkeypatch):
    wl, r = star_qp

    def printed_Q(omega, period, alpha, ct):
        E = np.exp(1j * ct.s * period)
        ap, am = alpha + 1 / alpha, alpha - 1 / alpha
        I = np.eye(len(ct.s))
        return np.block([[I + np.diag(1j * E * am / (2 * ct.s)), np.diag(-E * ap / 2)],
                         [np.diag(E * ap / 2), I + np.diag(1j * E * ct.s * am / 2)]])

    monkeypatch.setattr(pq, "wall_Q", printed_Q)
    rb = pq.solve_qp(r["disc"], 400, wl.omega, wl.period, wl.thetas, quad="kress")
    assert rb["flux"][0] > 1e-3


def test_planted_printed_Ctilde_fails_P1(star_qp, monkeypatch):
    wl, r = star_qp
    orig = pq.wall_C

    def printed(disc, omega, period, ct, shift=0.0):
        # the printed second term uses R at dOmega - (P+1) d instead of -P d
        if shift < 0:
            shift = shift - period
        return orig(disc, omega, period, ct, shift)

    monkeypatch.setattr(pq, "wall_C", printed)
    r1 = pq.solve_qp(r["disc"], 400, wl.omega, wl.period, wl.thetas, quad="kress", P=1)
    assert np.abs(r1["eta"] - r["eta"]).max() > 1e-4 * np.abs(r["eta"]).max()


def test_planted_missing_end_correction_fails_circle(monkeypatch):
    monkeypatch.setattr(qd, "kr6_corrections", lambda dps=50: np.zeros(6))
    d = ny.Discretization(qpinputs.circle(1.0), 400)
    A = ny.matrix(d, 10.0, "kr6")
    v = np.ones(d.N)
    assert np.abs(A @ v - ny.circle_eigenvalue(10.0, 1.0, 0) * v).max() > 1e-3


# ---------------------------------------------------------------- row blocks and the residual checker

def test_kr6_rows_equal_full_matrix_rows():
    c = qpinputs.wavy(130102, 20, 0.3)
    disc = ny.Discretization(c, 400)
    A = ny.matrix_kr6(disc, 40.0)
    rows = np.array([0, 1, 7, 199, 398, 399])
    assert np.array_equal(ny.matrix_kr6_rows(disc, 40.0, rows), A[rows])


def test_neighbour_rows_equal_full_matrix_rows():
    c = qpinputs.star(0.35, 0.105, 3)
    disc = ny.Discretization(c, 300)
    rows = np.array([0, 5, 150, 299])
    for sh in (1.0, -1.0):
        assert np.array_equal(ny.neighbour_rows(disc, 10.0, sh, rows), ny.neighbour_matrix(disc, 10.0, sh)[rows])


def test_residual_checker_with_neighbour_images():
    """P = 1 (the d = 1 grating of Sec. 6.1): the dense solution's sampled residual is at rounding
    level, and a relative change of 1e-6 in one density value shows."""
    from oracle import checks
    wl = qpinputs.workload("star_d1")
    N, th = 300, np.array([-math.pi / 5, -1.2])
    r = pq.solve_qp(wl.curve, N, wl.omega, wl.period, th, P=1)
    v = checks.bordered_residual(wl.curve, N, wl.omega, wl.period, th, r["eta"], r["xi"], n_rows=30, n_ang=2,
                                 chunk=100, P=1)
    assert v["sampled_rel_residual"] < 1e-12
    eta = r["eta"].copy()
    eta[40, :] *= 1.0 + 1e-6
    v = checks.bordered_residual(wl.curve, N, wl.omega, wl.period, th, eta, r["xi"], n_rows=30, n_ang=2,
                                 chunk=100, P=1)
    assert v["sampled_rel_residual"] > 1e-10


@pytest.fixture(scope="module")
def wavy_kr6_qp():
    """A KR6 solution at N = 600 of a rough obstacle, for the residual checker."""
    from oracle import checks  # noqa: F401
    c = qpinputs.wavy(130103, 40, 0.2)
    N, om, d = 600, 12.0, 2 * math.pi
    th = np.array([-0.7, -1.1, -1.3])
    r = pq.solve_qp(c, N, om, d, th, quad="kr6")
    return c, N, om, d, th, r


def test_residual_checker_small_for_the_exact_solution(wavy_kr6_qp):
    from oracle import checks
    c, N, om, d, th, r = wavy_kr6_qp
    v = checks.bordered_residual(c, N, om, d, th, r["eta"], r["xi"], r["flux"], n_rows=40, n_ang=3, chunk=250)
    assert v["sampled_rel_residual"] < 1e-12
    assert v["angles_sampled"] == 3


def test_residual_checker_sees_planted_errors(wavy_kr6_qp):
    """A perturbation of one obstacle density value or of one wall density value shows in the
    sampled residual at about its own size (all wall rows are checked; the obstacle column of a
    perturbed node reaches every row through the kernel)."""
    from oracle import checks
    c, N, om, d, th, r = wavy_kr6_qp
    scale = np.linalg.norm(pq.incident(ny.Discretization(c, N), om, th[0]))
    for which in ("eta", "xi"):
        eta, xi = r["eta"].copy(), r["xi"].copy()
        (eta if which == "eta" else xi)[17, :] += 1e-6 * scale
        v = checks.bordered_residual(c, N, om, d, th, eta, xi, n_rows=40, n_ang=3, chunk=250)
        assert v["sampled_rel_residual"] > 1e-9, which
