"""Pins of the oracle on the paper's own grating of Sec. 6.1 (star r = 0.35 + 0.105 cos 3t, period
d = 1), where the neighbour images come within 0.25 of the obstacle and the scheme needs the P = 1
images of Sec. 2.4: the density eta is the same for P = 1 and P = 2 (both represent the one
quasi-periodic field; a slip in the image sums or in C~ breaks the agreement), and the flux balance
of Remark 6.1 converges at the quadrature's order."""
import math

import numpy as np

import qpinputs
from oracle import periodic as pq


def test_star_d1_P1_equals_P2():
    wl = qpinputs.workload("star_d1")
    r1 = pq.solve_qp(wl.curve, 300, wl.omega, wl.period, wl.thetas, P=1)
    r2 = pq.solve_qp(wl.curve, 300, wl.omega, wl.period, wl.thetas, P=2)
    e = np.abs(r1["eta"] - r2["eta"]).max() / np.abs(r2["eta"]).max()
    assert e < 1e-11


def test_star_d1_flux_converges():
    wl = qpinputs.workload("star_d1")
    f = [pq.solve_qp(wl.curve, N, wl.omega, wl.period, wl.thetas, P=1)["flux"][0] for N in (300, 600)]
    assert f[1] < 1e-6
    assert math.log2(f[0] / f[1]) > 5.0


def test_star_d1_coarser_contour_agrees():
    """At this grating's wall-to-image gap (about 1.05) the contour spacing 0.2 (M = 368) gives the
    density of spacing 0.1 (M = 736) to 1e-12: the benchmark's solve of this workload uses it."""
    wl = qpinputs.workload("star_d1")
    r1 = pq.solve_qp(wl.curve, 300, wl.omega, wl.period, wl.thetas, P=1, h=0.1)
    r2 = pq.solve_qp(wl.curve, 300, wl.omega, wl.period, wl.thetas, P=1, h=0.2)
    assert len(r2["contour"].k) == 368
    assert np.abs(r1["eta"] - r2["eta"]).max() / np.abs(r1["eta"]).max() < 1e-12
