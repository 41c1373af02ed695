"""Alpert-corrected Nystrom matrix on the GPU (Sec. 2.3's named alternative to Kapur-Rokhlin) against
the oracle (oracle/alpert.py), through the C ABI.  The library interpolates the off-grid geometry from
its node arrays (12-point Lagrange), the oracle evaluates the analytic curve: entries agree to the
O(h^12) interpolation error, solutions to the 1e-10 bar."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import qpinputs
from oracle import alpert as al
from oracle import nystrom as ny
from oracle import periodic as pq
from paper_1301_1247_amd.geometry import discretize

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_alpert_entries_match_oracle(gpu_lib):
    c = qpinputs.star()
    N, om = 400, 10.0
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, quad="alpert", leaf_size=50)
    A = al.matrix_alpert(ny.Discretization(c, N), om, c)
    rng = np.random.default_rng(9)
    rows = np.concatenate([rng.integers(0, N, 300), np.arange(N), np.arange(N)])
    off = np.concatenate([rng.integers(-15, 16, 300), np.full(N, 11), np.full(N, -11)])
    cols = (rows + off) % N
    rows = np.concatenate([rows, rng.integers(0, N, 200)])
    cols = np.concatenate([cols, rng.integers(0, N, 200)])
    g = h.matrix_entries(rows, cols)
    assert np.abs(g - A[rows, cols]).max() < 2e-12 * np.abs(A).max()


def test_alpert_inverse_vs_dense(gpu_lib):
    c = qpinputs.wavy(130102, 20, 0.3)
    N, om = 2000, 40.0
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, quad="alpert")
    A = al.matrix_alpert(ny.Discretization(c, N), om, c)
    rng = np.random.default_rng(4)
    B = rng.standard_normal((N, 4)) + 1j * rng.standard_normal((N, 4))
    Xe = sla.solve(A, B)
    assert _rel(h.apply(B, refine=2), Xe) < 1e-10
    assert _rel(h.forward(Xe), A @ Xe) < 1e-10


def test_alpert_qp_solve_star(gpu_lib):
    wl = qpinputs.workload("star")
    N = 800
    nodes, w, nrm, _ = discretize(wl.curve, N)
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-12, quad="alpert", leaf_size=50)
    th = np.array([wl.thetas[0], -1.1, -0.3])
    res = h.qp_solve_many(wl.period, th)
    disc = ny.Discretization(wl.curve, N)
    ref = pq.solve_qp(disc, N, wl.omega, wl.period, th, A0=al.matrix_alpert(disc, wl.omega, wl.curve))
    for a in range(len(th)):
        assert _rel(res["eta"][:, a], ref["eta"][:, a]) < 1e-10
        assert _rel(res["xi"][:, a], ref["xi"][:, a]) < 1e-10
        assert abs(res["flux"][a] - ref["flux"][a]) < 1e-10
    assert res["flux"].max() < 1e-11


def test_alpert_circle_closed_form_through_gpu(gpu_lib):
    """A^{-1} e^{int} = e^{int} / lambda_n on the circle, to the rule's accuracy at N = 256 (the
    discretization error grows with the mode: about 4e-12, 2e-11, 2e-10 for n = 0, 3, 7)."""
    c = qpinputs.circle(1.0)
    N, om = 256, 10.0
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-13, quad="alpert", leaf_size=32)
    t = 2 * math.pi * np.arange(N) / N
    for n, bar in ((0, 1e-10), (3, 1e-10), (7, 1e-9)):
        v = np.exp(1j * n * t)
        x = h.apply(v, refine=2)
        assert np.abs(x - v / ny.circle_eigenvalue(om, 1.0, n)).max() < bar * np.abs(x).max()


def test_alpert_full_size_sampled_residual(gpu_lib):
    """The benchmark's workload (N = 1e5, omega = 60, 200 angles, compressed walls, rank predictor,
    deferred root) with Alpert's quadrature: sampled rows of the bordered residual against the
    oracle's Alpert rows, and the energy balance of every angle."""
    import torch
    from oracle import checks
    wl = qpinputs.workload("wavy40")
    nodes, w, nrm, _ = discretize(wl.curve, wl.N)
    t = lambda a: torch.from_numpy(a).to("cuda")
    c = 0.5 * (nodes.max(0) + nodes.min(0))
    far = 0.9 * (0.5 * wl.period - abs(c[0]))
    h = gpu_lib.Handle(t(nodes), t(w), t(nrm), wl.omega, 1e-13, quad="alpert", leaf_size=64, device=True,
                       far_radius=far, rank_predictor=True, defer_root=True)
    res = h.qp_solve_many(wl.period, t(wl.thetas), compress_walls=1)
    v = checks.bordered_residual(wl.curve, wl.N, wl.omega, wl.period, wl.thetas, res["eta"].T.cpu().numpy(),
                                 res["xi"].T.cpu().numpy(), res["flux"], n_rows=32, n_ang=8, quad="alpert")
    print(f"alpert N=1e5 {v}", flush=True)
    assert v["sampled_rel_residual"] < 1e-10
    assert v["flux_err_max"] < 1e-8
