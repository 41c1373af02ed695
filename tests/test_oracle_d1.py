"""Pins of the oracle on the paper's own grating of Sec. 6.1 (star r = 0.35 + 0.105 cos 3t, period
d = 1), where the neighbour images come within 0.25 of the obstacle and the scheme needs the P = 1
images of Sec. 2.4: the density eta is the same for P = 1 and P = 2 (both represent the one
quasi-periodic field; a slip in the image sums or in C~ breaks the agreement), the flux balance
of Remark 6.1 converges at the quadrature's order, and the neighbour interaction has the rank the
paper reports for this grating (fixture tests/golden/neighbour_rank_d1.txt)."""
import math
import os

import numpy as np

import qpinputs
from oracle import nystrom as ny
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


def _golden(name):
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_neighbour_interaction_rank_matches_the_paper():
    """The interaction of the obstacle with its two neighbours (the image blocks A_{+1}, A_{-1} side by
    side) has numerical rank at the paper's precision between 3/4 of, and at most, the ID rank the paper
    reports for this grating.  A neighbour at 2d instead of d gives about 25, one at 0.9 d about 63."""
    g = _golden("neighbour_rank_d1.txt")
    wl = qpinputs.workload("star_d1")
    assert (wl.omega, wl.period) == (g["omega"], g["period"])
    disc = ny.Discretization(wl.curve, 400)
    M = np.hstack([ny.neighbour_matrix(disc, wl.omega, wl.period), ny.neighbour_matrix(disc, wl.omega, -wl.period)])
    s = np.linalg.svd(M, compute_uv=False)
    rank = int((s > g["precision"] * s[0]).sum())
    assert 0.75 * g["neighbour_rank"] <= rank <= g["neighbour_rank"], rank
