"""Degenerate and boundary inputs through the C ABI on the GPU: empty right-hand-side and angle
sets, angles close to grazing on both sides of the normal, and one handle serving several
periods (the compressed inverse belongs to the isolated obstacle, the period only to the
periodizing step).  Bar: the oracle's dense solution to relative 1e-10 (2-norm and largest
entry)."""
import math

import numpy as np
import pytest

import qpinputs
from oracle import nystrom as ny
from oracle import periodic as pq
from paper_1301_1247_amd.geometry import discretize

pytestmark = pytest.mark.gpu


def _cmp(g, r):
    return max(np.linalg.norm(g - r) / np.linalg.norm(r), np.abs(g - r).max() / np.abs(r).max())


@pytest.fixture(scope="module")
def star():
    wl = qpinputs.workload("star")
    nodes, w, nrm, kap = discretize(wl.curve, wl.N)
    return wl, (nodes, w, nrm, kap)


def test_empty_inputs(gpu_lib, star):
    import torch
    wl, (nodes, w, nrm, kap) = star
    N = wl.N
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-12, quad="kress", leaf_size=50, curvature=kap)
    z = np.zeros((N, 0), dtype=np.complex128)
    assert h.apply(z).shape == (N, 0)
    assert h.forward(z).shape == (N, 0)
    r = h.qp_solve_many(wl.period, np.zeros(0))
    assert r["eta"].shape == (N, 0) and r["flux"].shape == (0,)
    # device pointers, and the apply that allocates nothing
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    hd = gpu_lib.Handle(t(nodes), t(w), t(nrm), wl.omega, 1e-12, device=True, leaf_size=50)
    e = torch.zeros((0, N), dtype=torch.complex128, device="cuda")
    assert tuple(hd.apply(e).shape) == (0, N)
    assert tuple(hd.apply_noalloc(e).shape) == (0, N)
    rd = hd.qp_solve_many(wl.period, t(np.zeros(0)))
    assert tuple(rd["eta"].shape) == (0, N)


def test_near_grazing_both_sides(gpu_lib, star):
    """|sin theta| = 0.1 at omega = 10 (k_0 = 1, above the Wood threshold), once with the incident
    wave travelling right and once travelling left."""
    wl, (nodes, w, nrm, kap) = star
    th = np.array([-math.asin(0.1), -math.pi + math.asin(0.1)])
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-12, quad="kress", leaf_size=50, curvature=kap)
    res = h.qp_solve_many(wl.period, th)
    ref = pq.solve_qp(wl.curve, wl.N, wl.omega, wl.period, th, quad="kress")
    for a in range(len(th)):
        assert _cmp(res["eta"][:, a], ref["eta"][:, a]) < 1e-10, a
        assert _cmp(res["xi"][:, a], ref["xi"][:, a]) < 1e-10, a
        assert abs(res["flux"][a] - ref["flux"][a]) < 1e-10


def test_one_handle_several_periods(gpu_lib, star):
    wl, (nodes, w, nrm, kap) = star
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-12, quad="kress", leaf_size=50, curvature=kap)
    disc = ny.Discretization(wl.curve, wl.N)
    A = ny.matrix(disc, wl.omega, "kress")
    for d, th in ((2 * math.pi, -0.9), (7.0, -1.3), (2 * math.pi, -0.6)):
        res = h.qp_solve_many(d, np.array([th]))
        ref = pq.solve_qp(disc, wl.N, wl.omega, d, np.array([th]), quad="kress", A0=A)
        assert _cmp(res["eta"][:, 0], ref["eta"][:, 0]) < 1e-10, d
        assert _cmp(res["xi"][:, 0], ref["xi"][:, 0]) < 1e-10, d
