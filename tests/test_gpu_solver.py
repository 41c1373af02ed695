"""End-to-end parity of the GPU solver with the CPU oracle, through the C ABI.

Bar (floating point): relative error <= 1e-10 of every solution against the oracle's dense
LU solution, the target stated for the solver.  The compressed inverse alone is an
approximation to the requested tolerance amplified by the conditioning of the reduced
systems, so bare applies are held to a looser bound and refinement recovers 1e-10.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import qpinputs
from oracle import nystrom as ny
from oracle import periodic as pq
from paper_1301_1247_amd.geometry import discretize

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def wavy_small():
    c = qpinputs.wavy(130102, 20, 0.3)
    N, om = 2000, 40.0
    disc = ny.Discretization(c, N)
    A = ny.matrix(disc, om, "kr6")
    return c, N, om, disc, A, sla.lu_factor(A)


def test_hbs_inverse_and_forward_vs_dense(gpu_lib, wavy_small):
    c, N, om, disc, A, lu = wavy_small
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((N, 7)) + 1j * rng.standard_normal((N, 7))
    Xe = sla.lu_solve(lu, B)
    X0 = h.apply(B)
    assert _rel(X0, Xe) < 1e-7
    X1 = h.apply(B, refine=2)
    assert _rel(X1, Xe) < 1e-10
    F = h.forward(Xe)
    assert _rel(F, A @ Xe) < 1e-10
    # batch consistency: columns applied one at a time give the same result
    for j in (0, 6):
        xj = h.apply(B[:, j])
        assert np.abs(xj - X0[:, j]).max() <= 1e-12 * np.abs(X0[:, j]).max()
    s = h.stats()
    assert s.levels >= 4 and 0 < s.max_rank <= 2048


def test_hbs_fp32_preconditioner_refines_to_fp64(gpu_lib, wavy_small):
    """complex64 inverse factors as a preconditioner: the bare apply is single-precision
    accurate, FP64 refinement against the forward operator recovers the 1e-10 bar."""
    c, N, om, disc, A, lu = wavy_small
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, precision="fp32")
    rng = np.random.default_rng(6)
    B = rng.standard_normal((N, 5)) + 1j * rng.standard_normal((N, 5))
    Xe = sla.lu_solve(lu, B)
    e0 = _rel(h.apply(B), Xe)
    assert 1e-9 < e0 < 1e-3
    assert _rel(h.apply(B, refine=5), Xe) < 1e-10
    assert _rel(h.forward(Xe), A @ Xe) < 1e-10


@pytest.mark.parametrize("N", [130, 131, 777])
def test_hbs_ragged_and_minimal_sizes(gpu_lib, N):
    c = qpinputs.star()
    om = 10.0
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, leaf_size=64 if N < 200 else 50)
    A = ny.matrix(ny.Discretization(c, N), om, "kr6")
    b = np.exp(1j * np.arange(N) * 0.37)
    assert _rel(h.apply(b, refine=2), np.linalg.solve(A, b)) < 1e-10


def test_kress_exact_inverse_vs_dense(gpu_lib):
    c = qpinputs.star()
    N, om = 800, 10.0
    nodes, w, nrm, kap = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, quad="kress", leaf_size=50, curvature=kap)
    A = ny.matrix(ny.Discretization(c, N), om, "kress")
    rng = np.random.default_rng(3)
    b = rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3))
    assert _rel(h.apply(b, refine=2), np.linalg.solve(A, b)) < 1e-10


def test_circle_closed_form_through_gpu(gpu_lib):
    """A^{-1} e^{i n t} = e^{i n t} / lambda_n on the circle, to the quadrature's accuracy (Kress)."""
    c = qpinputs.circle(1.0)
    N, om = 256, 10.0
    nodes, w, nrm, kap = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-13, quad="kress", leaf_size=32, curvature=kap)
    t = 2 * math.pi * np.arange(N) / N
    for n in (0, 3, 17):
        v = np.exp(1j * n * t)
        x = h.apply(v, refine=2)
        assert np.abs(x - v / ny.circle_eigenvalue(om, 1.0, n)).max() < 1e-11 * np.abs(x).max()


def _oracle_qp(curve, N, om, d, thetas, quad):
    r = pq.solve_qp(curve, N, om, d, thetas, quad=quad)
    return r


def _check_qp(res, ref, nth):
    eta, xi = res["eta"], res["xi"]
    for a in range(nth):
        assert _rel(eta[:, a], ref["eta"][:, a]) < 1e-10, a
        assert _rel(xi[:, a], ref["xi"][:, a]) < 1e-10, a
        n, kn, c, d = ref["bragg"][a]
        maxm = res["maxmodes"]
        nlo, nm = res["nlo"][a], res["nmodes"][a]
        assert nlo == n[0] and nm == len(n)
        cg = res["bragg"][:nm, a]
        dg = res["bragg"][maxm:maxm + nm, a]
        scale = max(np.abs(c).max(), np.abs(d).max())
        assert np.abs(cg - c).max() < 1e-10 * scale
        assert np.abs(dg - d).max() < 1e-10 * scale
        assert abs(res["flux"][a] - ref["flux"][a]) < 1e-10


def test_qp_star_kress_parity(gpu_lib):
    wl = qpinputs.workload("star")
    nodes, w, nrm, kap = discretize(wl.curve, wl.N)
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-12, quad="kress", leaf_size=50, curvature=kap)
    res = h.qp_solve_many(wl.period, wl.thetas)
    ref = _oracle_qp(wl.curve, wl.N, wl.omega, wl.period, wl.thetas, "kress")
    assert res["M"] == len(ref["contour"].k)
    _check_qp(res, ref, len(wl.thetas))
    assert res["flux"][0] < 1e-12
    st = h.stats()
    assert st.refine_residual < 1e-12


def test_qp_wavy_kr6_parity_shared_and_distinct_phases(gpu_lib, wavy_small):
    c, N, om, disc, A, lu = wavy_small
    d = 2 * math.pi
    # two angles sharing a Bloch phase, plus two distinct ones
    c1 = 0.31   # min_n |k_n| > 5 for both angles of the shared phase (away from Wood's anomalies)
    c2 = c1 + 2 * math.pi / (om * d)
    thetas = np.array([-math.acos(c1), -1.1, -math.acos(c2), -0.45])
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12)
    res = h.qp_solve_many(d, thetas)
    ref = pq.solve_qp(disc, N, om, d, thetas, quad="kr6", A0=A)
    _check_qp(res, ref, len(thetas))


@pytest.mark.parametrize("walls", ["dense", "compressed"])
def test_qp_wavy_kr6_parity_bragg_group_basis(gpu_lib, wavy_small, walls):
    """Five angles on one Bloch phase take the shared basis of diffraction orders (groups of four
    or more: one batched product for all their Bragg amplitudes), a sixth angle the direct sums."""
    c, N, om, disc, A, lu = wavy_small
    d = 2 * math.pi
    c1 = 0.31  # the shared phase keeps the diffraction orders of c1, away from Wood's anomalies
    thetas = np.array([-math.acos(c1 + m * 2 * math.pi / (om * d)) for m in range(5)] + [-0.45])
    nodes, w, nrm, _ = discretize(c, N)
    kw = {}
    if walls == "compressed":
        c0 = 0.5 * (nodes.max(0) + nodes.min(0))
        kw["far_radius"] = 0.9 * (0.5 * d - abs(c0[0]))
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, **kw)
    res = h.qp_solve_many(d, thetas, compress_walls=1 if walls == "compressed" else -1)
    assert h.stats().walls_compressed == (walls == "compressed")
    ref = pq.solve_qp(disc, N, om, d, thetas, quad="kr6", A0=A)
    _check_qp(res, ref, len(thetas))


def test_qp_wavy_kr6_parity_fp32_preconditioner(gpu_lib, wavy_small):
    c, N, om, disc, A, lu = wavy_small
    d = 2 * math.pi
    thetas = np.array([-math.acos(0.31), -1.1, -0.45])
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, precision="fp32")
    res = h.qp_solve_many(d, thetas, refine_max_iter=6)
    ref = pq.solve_qp(disc, N, om, d, thetas, quad="kr6", A0=A)
    _check_qp(res, ref, len(thetas))
    assert h.stats().refine_residual < 1e-12


def test_qp_solve_alpha_mismatch_and_wood(gpu_lib):
    wl = qpinputs.workload("star")
    nodes, w, nrm, kap = discretize(wl.curve, wl.N)
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-10, quad="kress", leaf_size=50, curvature=kap)
    with pytest.raises(gpu_lib.HBSError) as e:
        h.qp_solve_many(wl.period, np.array([-0.6]), alpha=1.0 + 0j)
    assert e.value.code == -8
    # Wood's anomaly: kappa + n = +-omega for d = 2 pi, i.e. cos(theta) = (omega - 1)/omega
    th = -math.acos((wl.omega - 1.0) / wl.omega)
    with pytest.raises(gpu_lib.HBSError) as e:
        h.qp_solve_many(wl.period, np.array([th]), wood=-1)
    assert e.value.code == -9


def _far_radius(nodes, d):
    c = 0.5 * (nodes.max(0) + nodes.min(0))
    robs = np.hypot(*(nodes - c).T).max()
    return 0.9 * (d - robs)


def test_qp_neighbour_images_P1_star_kress(gpu_lib):
    wl = qpinputs.workload("star")
    nodes, w, nrm, kap = discretize(wl.curve, wl.N)
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-12, quad="kress", leaf_size=50, curvature=kap,
                       far_radius=_far_radius(nodes, wl.period))
    res = h.qp_solve_many(wl.period, wl.thetas, P=1)
    ref = pq.solve_qp(wl.curve, wl.N, wl.omega, wl.period, wl.thetas, quad="kress", P=1)
    assert res["M"] == len(ref["contour"].k)
    _check_qp(res, ref, len(wl.thetas))
    # P = 0 and P = 1 represent the same scattered field
    res0 = h.qp_solve_many(wl.period, wl.thetas, P=0)
    assert _rel(res["eta"][:, 0], res0["eta"][:, 0]) < 1e-10


def test_qp_neighbour_images_P1_wavy_kr6(gpu_lib, wavy_small):
    c, N, om, disc, A, lu = wavy_small
    d = 2 * math.pi
    thetas = np.array([-1.1, -0.45, -math.acos(0.31), -math.acos(0.31 + 1 / 40)])
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, far_radius=_far_radius(nodes, d))
    res = h.qp_solve_many(d, thetas, P=1)
    ref = pq.solve_qp(disc, N, om, d, thetas, quad="kr6", P=1, A0=A)
    _check_qp(res, ref, len(thetas))
    assert h.stats().refine_residual < 1e-12


def _far_walls(nodes, d):
    """far_radius for which the walls x = +-d/2 lie outside the far-field circle."""
    c = 0.5 * (nodes.max(0) + nodes.min(0))
    return 0.9 * (0.5 * d - abs(c[0]))


@pytest.mark.parametrize("P", [0, 1])
def test_qp_wavy_kr6_parity_compressed_walls(gpu_lib, wavy_small, P):
    """B and C through the root skeletons (B = U B(J,:), C = C(:,J) U^T): same solution as the
    dense oracle to the 1e-10 bar, for both the plain and the neighbour-image formulation."""
    c, N, om, disc, A, lu = wavy_small
    d = 2 * math.pi
    thetas = np.array([-1.1, -0.45, -math.acos(0.31), -math.acos(0.31 + 1 / 40)])
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, far_radius=_far_walls(nodes, d))
    res = h.qp_solve_many(d, thetas, P=P, compress_walls=1)
    assert h.stats().walls_compressed == 1
    ref = pq.solve_qp(disc, N, om, d, thetas, quad="kr6", P=P, A0=A)
    _check_qp(res, ref, len(thetas))
    assert h.stats().refine_residual < 1e-12
    # the uncompressed path on the same handle agrees
    res_u = h.qp_solve_many(d, thetas, P=P, compress_walls=-1)
    assert h.stats().walls_compressed == 0
    assert _rel(res_u["eta"], res["eta"]) < 1e-10
    # compressed solve refined against the uncompressed wall blocks
    res_x = h.qp_solve_many(d, thetas, P=P, compress_walls=2)
    assert h.stats().walls_compressed == 2
    _check_qp(res_x, ref, len(thetas))
    assert _rel(res_x["eta"], res_u["eta"]) < 1e-10


@pytest.mark.parametrize("P", [0, 1])
def test_root_over_level2_skeletons(gpu_lib, wavy_small, P):
    """root_level = 2: level 1 left uncompressed (P = I), the root holds the level-2 skeletons;
    the compressed inverse, the forward operator and the quasi-periodic solve keep the 1e-10 bar."""
    c, N, om, disc, A, lu = wavy_small
    d = 2 * math.pi
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, far_radius=_far_walls(nodes, d), root_level=2)
    h1 = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, far_radius=_far_walls(nodes, d), root_level=1)
    st, st1 = h.stats(), h1.stats()
    assert st.root_level == 2 and st1.root_level == 1
    k, lv = h.rank_features()[1], h.rank_features()[2]
    k1 = h1.rank_features()[1]
    assert st.root_size == k1[lv == 2].sum() and st1.root_size == k1[lv == 1].sum()
    rng = np.random.default_rng(8)
    b = rng.standard_normal((N, 2)) + 1j * rng.standard_normal((N, 2))
    xe = sla.lu_solve(lu, b)
    assert _rel(h.apply(b, refine=2), xe) < 1e-10
    assert _rel(h.forward(xe), A @ xe) < 1e-10
    thetas = np.array([-1.1, -math.acos(0.31), -math.acos(0.31 + 1 / 40)])
    res = h.qp_solve_many(d, thetas, P=P, compress_walls=1)
    ref = pq.solve_qp(disc, N, om, d, thetas, quad="kr6", P=P, A0=A)
    _check_qp(res, ref, len(thetas))


def test_qp_star_kress_compressed_walls(gpu_lib):
    wl = qpinputs.workload("star")
    nodes, w, nrm, kap = discretize(wl.curve, wl.N)
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-12, quad="kress", leaf_size=50, curvature=kap,
                       far_radius=_far_walls(nodes, wl.period))
    res = h.qp_solve_many(wl.period, wl.thetas)      # compress_walls = 0: taken when valid
    assert h.stats().walls_compressed == 1
    ref = _oracle_qp(wl.curve, wl.N, wl.omega, wl.period, wl.thetas, "kress")
    _check_qp(res, ref, len(wl.thetas))


def test_qp_compressed_walls_needs_far_circle_inside_cell(gpu_lib):
    wl = qpinputs.workload("star")
    nodes, w, nrm, kap = discretize(wl.curve, wl.N)
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-10, quad="kress", leaf_size=50, curvature=kap)
    with pytest.raises(gpu_lib.HBSError) as e:
        h.qp_solve_many(wl.period, wl.thetas, compress_walls=1)
    assert e.value.code == -1
    h2 = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-10, quad="kress", leaf_size=50, curvature=kap,
                        far_radius=_far_radius(nodes, wl.period))   # reaches beyond the walls
    with pytest.raises(gpu_lib.HBSError) as e:
        h2.qp_solve_many(wl.period, wl.thetas, compress_walls=1)
    assert e.value.code == -1
    h2.qp_solve_many(wl.period, wl.thetas)            # falls back to the uncompressed walls
    assert h2.stats().walls_compressed == 0


def test_qp_P1_needs_far_field_skeletons(gpu_lib):
    wl = qpinputs.workload("star")
    nodes, w, nrm, kap = discretize(wl.curve, wl.N)
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-10, quad="kress", leaf_size=50, curvature=kap)
    with pytest.raises(gpu_lib.HBSError) as e:
        h.qp_solve_many(wl.period, wl.thetas, P=1)
    assert e.value.code == -1


def test_graph_captured_applies_replay_exactly(gpu_lib, wavy_small):
    """hbs_opts.graph: the apply is captured into a HIP graph and replayed; every replay, with
    eager work of other handles in between, gives the result of the uncaptured apply."""
    import torch
    c, N, om, disc, A, lu = wavy_small
    nodes, w, nrm, _ = discretize(c, N)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)
    hg = gpu_lib.Handle(t(nodes), t(w), t(nrm), om, 1e-12, device=True, graph=True)
    h0 = gpu_lib.Handle(t(nodes), t(w), t(nrm), om, 1e-12, device=True)
    rng = np.random.default_rng(9)
    b = torch.from_numpy(rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))).to(dev)
    out = torch.empty_like(b)
    ref = h0.apply(b)
    for it in range(4):
        for inverse in (True, False):
            fn = gpu_lib._lib.hbs_apply if inverse else gpu_lib._lib.hbs_forward
            args = (hg._h, gpu_lib._ptr(b), 3, gpu_lib._ptr(out)) + ((0,) if inverse else ())
            assert fn(*args) == 0
            torch.cuda.synchronize()
            expect = ref if inverse else h0.forward(b)
            assert torch.equal(out, expect), (it, inverse)
        h0.apply(b[:1])   # eager work between the replays
    st = hg.stats()
    assert st.graph_captures == 2 and st.graph_replays == 6
    # refinement inside qp_solve replays its forward and inverse applies
    d = 2 * math.pi
    thetas = np.array([-1.1, -0.45])
    kw = dict(refine_max_iter=3, refine_tol=1e-300)
    r1 = hg.qp_solve_many(d, t(thetas), **kw)
    r0 = h0.qp_solve_many(d, t(thetas), **kw)
    assert torch.equal(r1["eta"], r0["eta"])
    assert hg.stats().graph_replays > 6
