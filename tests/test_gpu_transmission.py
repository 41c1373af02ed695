"""Parity of the transmission problem (Sec. 5) on the GPU with the CPU oracle, through the C ABI.

The handle is built with hbs_opts.index = n: 2N interlaced unknowns [tau_i; sigma_i], the 2 x 2
difference-kernel operator with Kapur-Rokhlin weights.  Bar (floating point): matrix entries to
rounding; eta and xi within relative 1e-10 of the oracle's dense LU solution after refinement (the
target stated for the solver), the Bragg amplitudes (sums of 2N terms of eta) within 1e-9 of the
largest; the bare compressed inverse within 1e-7.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.special import hankel1

import qpinputs
from oracle import nystrom as ny
from oracle import transmission as tr
from paper_1301_1247_amd.geometry import discretize

pytestmark = pytest.mark.gpu

OM, IDX, D = 10.0, 1.5, 2 * math.pi


def _rel(a, b):
    """Relative error in the 2-norm and element by element (max |a - b| / max |b|), the larger."""
    return max(np.linalg.norm(a - b) / np.linalg.norm(b), np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def star_tr():
    c = qpinputs.star(1.0, 0.3, 5)
    N = 700  # 1400 unknowns: a ragged tree of several levels
    disc = ny.Discretization(c, N)
    A = tr.matrix(disc, OM, IDX)
    return c, N, disc, A, sla.lu_factor(A)


def test_matrix_entries_match_oracle(gpu_lib, star_tr):
    c, N, disc, A, _ = star_tr
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, OM, 1e-12, index=IDX)
    assert h.stats().unknowns == 2 * N
    rng = np.random.default_rng(11)
    i = rng.integers(0, 2 * N, 400)
    j = rng.integers(0, 2 * N, 400)
    # the diagonal pairs of a node, the corrected band and its wrap-around
    i = np.concatenate([i, [0, 0, 1, 1, 2, 3, 10, 11, 0, 1, 2 * N - 1, 2 * N - 2]])
    j = np.concatenate([j, [0, 1, 0, 1, 5, 12, 3, 2, 2 * N - 1, 2 * N - 2, 0, 13]])
    g = h.matrix_entries(i, j)
    assert np.abs(g - A[i, j]).max() < 1e-12


def test_inverse_and_forward_vs_dense(gpu_lib, star_tr):
    c, N, disc, A, lu = star_tr
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, OM, 1e-12, index=IDX, leaf_size=64)
    rng = np.random.default_rng(12)
    B = rng.standard_normal((2 * N, 5)) + 1j * rng.standard_normal((2 * N, 5))
    Xe = sla.lu_solve(lu, B)
    assert _rel(h.apply(B), Xe) < 1e-7
    assert _rel(h.apply(B, refine=2), Xe) < 1e-10
    assert _rel(h.forward(Xe), A @ Xe) < 1e-10
    s = h.stats()
    assert s.levels >= 3 and s.N == N and s.unknowns == 2 * N


def test_exact_compression_agrees(gpu_lib, star_tr):
    c, N, disc, A, lu = star_tr
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, OM, 1e-12, index=IDX, compress="exact")
    b = np.exp(1j * np.arange(2 * N) * 0.21)
    assert _rel(h.apply(b, refine=2), sla.lu_solve(lu, b)) < 1e-10


def test_point_sources_reproduced(gpu_lib):
    """The jumps of a radiating source at omega from inside and a regular field at n omega from outside:
    the GPU densities reproduce both fields (an exact solution, independent of the oracle's matrix)."""
    c = qpinputs.star(1.0, 0.3, 5)
    N = 1600
    disc = ny.Discretization(c, N)
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, OM, 1e-12, index=IDX)
    zi, zo, k1 = np.array([0.1, 0.2]), np.array([2.0, 1.5]), IDX * OM

    def G(k, x, z):
        return 0.25j * hankel1(0, k * np.hypot(x[:, 0] - z[0], x[:, 1] - z[1]))

    def dG(k, x, nr, z):
        dx = x - z
        r = np.hypot(dx[:, 0], dx[:, 1])
        return -0.25j * k * hankel1(1, k * r) * (nr[:, 0] * dx[:, 0] + nr[:, 1] * dx[:, 1]) / r

    f = G(OM, disc.x, zi) - G(k1, disc.x, zo)
    g = dG(OM, disc.x, disc.nrm, zi) - dG(k1, disc.x, disc.nrm, zo)
    kb = tr.kbar(OM, IDX)
    eta = h.apply(tr.rhs_from_jumps(f, g, kb), refine=2)
    te = np.array([[1.8, -1.2], [-2.5, 0.3], [0.0, 1.9]])
    ti = np.array([[0.2, -0.1], [-0.3, 0.25], [0.4, 0.4]])
    assert np.abs(tr.potential(disc, OM, kb, eta, te) - G(OM, te, zi)).max() < 2e-8
    assert np.abs(tr.potential(disc, k1, kb, eta, ti) - G(k1, ti, zo)).max() < 2e-8


@pytest.mark.parametrize("compress", ["proxy", "exact"])
def test_qp_solve_matches_oracle(gpu_lib, star_tr, compress):
    c, N, disc, A, _ = star_tr
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, OM, 1e-12, index=IDX, compress=compress)
    # two angles sharing a Bloch phase (theta and its mirror about -pi/2) and one on its own
    ths = np.array([-math.pi / 5, -math.pi + math.pi / 5, -1.2])
    r = h.qp_solve_many(D, ths, P=0)
    ref = tr.solve_qp(disc, N, OM, IDX, D, ths, P=0, A0=A)
    assert r["M"] == len(ref["contour"].k)
    for a in range(len(ths)):
        assert _rel(r["eta"][:, a], ref["eta"][:, a]) < 1e-10
        assert _rel(r["xi"][:, a], ref["xi"][:, a]) < 1e-10
        n, kn, cc, dd = ref["bragg"][a]
        nm, mx = r["nmodes"][a], r["maxmodes"]
        assert nm == len(n) and r["nlo"][a] == n[0]
        bu, bd = r["bragg"][:nm, a], r["bragg"][mx:mx + nm, a]
        # each amplitude sums 2N terms of eta: held to 1e-9 of the largest amplitude
        assert np.abs(bu - cc).max() < 1e-9 * np.abs(cc).max()
        assert np.abs(bd - dd).max() < 1e-9 * np.abs(dd).max()
        assert abs(r["flux"][a] - ref["flux"][a]) < 1e-10


def test_index_one_leaves_the_field_unscattered(gpu_lib):
    """n = 1: the operator is the identity and every Bragg amplitude of the scattered field vanishes."""
    c = qpinputs.star(1.0, 0.3, 5)
    N = 400
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, OM, 1e-12, index=1.0)
    r = h.qp_solve_many(D, np.array([-math.pi / 5, -1.1]), P=0)
    for a in range(2):
        nm, mx = r["nmodes"][a], r["maxmodes"]
        assert np.abs(r["bragg"][:nm, a]).max() < 1e-9 and np.abs(r["bragg"][mx:mx + nm, a]).max() < 1e-9


def test_refusals(gpu_lib, star_tr):
    c, N, disc, A, _ = star_tr
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, OM, 1e-10, index=IDX)
    with pytest.raises(gpu_lib.HBSError) as e:
        h.qp_solve_many(D, np.array([-math.pi / 5]), P=1)
    assert e.value.code == -1
    # an angle next to a Wood's anomaly: k_n = 0 for some order
    th = -math.acos(1.0 - 2 * math.pi / (OM * D)) + 1e-3
    with pytest.raises(gpu_lib.HBSError) as e:
        h.qp_solve_many(D, np.array([th]), P=0)
    assert e.value.code == -9


@pytest.mark.parametrize("P,defer", [(0, False), (0, True), (1, False)])
def test_compressed_walls_match_oracle(gpu_lib, star_tr, P, defer):
    """Wall blocks through the root skeletons (the handle's far_radius circle excludes the walls), with
    the root inversion deferred into the Woodbury batch, and with the P = 1 images of Sec. 2.4 (exterior
    field only) in the Woodbury form of Eq. 3.2.  The wall blocks interpolated from the skeleton rows
    carry the decompositions' error unrefined (the refinement runs on the compressed bordered system):
    this pins the far-field circle's rows at both wavenumbers.  compress_walls = 2 refines against the
    uncompressed wall blocks instead."""
    c, N, disc, A, _ = star_tr
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, OM, 1e-12, index=IDX, far_radius=2.0, defer_root=defer)
    ths = np.array([-math.pi / 5, -1.2])
    r0 = h.qp_solve_many(D, ths, P=P)
    assert h.stats().walls_compressed == 0  # dense unless asked for (the default for this operator)
    r = h.qp_solve_many(D, ths, P=P, compress_walls=1)
    assert h.stats().walls_compressed == 1
    r2 = h.qp_solve_many(D, ths, P=P, compress_walls=2)
    assert h.stats().walls_compressed == 2
    ref = tr.solve_qp(disc, N, OM, IDX, D, ths, P=P, A0=A)
    for a in range(len(ths)):
        for rr in (r0, r, r2):
            assert _rel(rr["eta"][:, a], ref["eta"][:, a]) < 1e-10
            assert _rel(rr["xi"][:, a], ref["xi"][:, a]) < 1e-10
            assert abs(rr["flux"][a] - ref["flux"][a]) < 1e-10


def test_d1_grating_with_near_images_matches_oracle(gpu_lib):
    """The transmission case of Sec. 6.1 (d = 1: the neighbour images come within 0.09 of the obstacle)
    at a size the oracle solves densely: P = 1 with the images' near points as explicit columns."""
    wl = qpinputs.workload("star_d1_tr")
    N = 600
    disc = ny.Discretization(wl.curve, N)
    nodes, w, nrm, _ = discretize(wl.curve, N)
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-12, index=wl.index, far_radius=1.0, image_period=wl.period,
                       leaf_size=64)
    ths = np.array([-math.pi / 5, -1.0])
    r = h.qp_solve_many(wl.period, ths, P=1, h=0.2)
    assert h.stats().image_samples > 0
    ref = tr.solve_qp(disc, N, wl.omega, wl.index, wl.period, ths, P=1, h=0.2)
    for a in range(len(ths)):
        assert _rel(r["eta"][:, a], ref["eta"][:, a]) < 1e-10
        assert _rel(r["xi"][:, a], ref["xi"][:, a]) < 1e-10
        n, kn, cc, dd = ref["bragg"][a]
        nm, mx = r["nmodes"][a], r["maxmodes"]
        assert np.abs(r["bragg"][:nm, a] - cc).max() < 1e-9 * np.abs(cc).max()
        assert np.abs(r["bragg"][mx:mx + nm, a] - dd).max() < 1e-9 * np.abs(dd).max()
        assert abs(r["flux"][a] - ref["flux"][a]) < 1e-10


def test_d1_grating_full_size(gpu_lib):
    """N = 2^17 nodes (2^18 unknowns), the size of Sec. 6.1: sampled rows of the bordered residual
    (exact oracle rows) and the energy balance, both below 1e-10."""
    from oracle import checks
    wl = qpinputs.workload("star_d1_tr")
    nodes, w, nrm, _ = discretize(wl.curve, wl.N)
    h = gpu_lib.Handle(nodes, w, nrm, wl.omega, 1e-13, index=wl.index, far_radius=1.0, image_period=wl.period,
                       leaf_size=wl.leaf_size)
    r = h.qp_solve_many(wl.period, wl.thetas, P=1, h=0.2)
    v = checks.bordered_residual_tr(wl.curve, wl.N, wl.omega, wl.index, wl.period, wl.thetas, r["eta"], r["xi"],
                                    r["flux"], n_rows=16, P=1, h=0.2)
    assert v["sampled_rel_residual"] < 1e-10 and v["flux_err_max"] < 1e-10, v


def test_device_pointers_graphs_and_noalloc(gpu_lib, star_tr):
    """The 2N-long vectors through the device-pointer handle: the graph-captured applies and the
    no-allocation apply give the plain apply's result, and the qp_solve of the graph handle the
    plain one's."""
    import torch
    c, N, disc, A, lu = star_tr
    nodes, w, nrm, _ = discretize(c, N)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    h = gpu_lib.Handle(t(nodes), t(w), t(nrm), OM, 1e-12, index=IDX, device=True)
    hg = gpu_lib.Handle(t(nodes), t(w), t(nrm), OM, 1e-12, index=IDX, device=True, graph=True)
    rng = np.random.default_rng(13)
    B = rng.standard_normal((3, 2 * N)) + 1j * rng.standard_normal((3, 2 * N))
    tb = t(B)
    x = h.apply(tb, refine=1).cpu().numpy()
    assert _rel(x.T, sla.lu_solve(lu, B.T)) < 1e-10
    for _ in range(3):  # captured once, then replayed
        assert np.abs(hg.apply(tb, refine=1).cpu().numpy() - x).max() <= 1e-12 * np.abs(x).max()
    xn = h.apply_noalloc(tb, refine=1).cpu().numpy()
    assert np.abs(xn - x).max() <= 1e-12 * np.abs(x).max()
    ths = torch.tensor([-math.pi / 5, -1.2], dtype=torch.float64)
    r0 = h.qp_solve_many(D, ths, P=0)
    r1 = hg.qp_solve_many(D, ths, P=0)
    e0, e1 = r0["eta"].cpu().numpy(), r1["eta"].cpu().numpy()
    assert np.abs(e1 - e0).max() <= 1e-12 * np.abs(e0).max()


def test_fp32_preconditioner_refines_to_fp64(gpu_lib, star_tr):
    """complex64 inverse factors of the deep levels as a preconditioner for the transmission operator:
    FP64 refinement recovers the 1e-10 bar."""
    c, N, disc, A, lu = star_tr
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, OM, 1e-12, index=IDX, precision="fp32", fp64_top_levels=1)
    rng = np.random.default_rng(14)
    B = rng.standard_normal((2 * N, 4)) + 1j * rng.standard_normal((2 * N, 4))
    Xe = sla.lu_solve(lu, B)
    assert 1e-9 < _rel(h.apply(B), Xe) < 1e-3
    assert _rel(h.apply(B, refine=5), Xe) < 1e-10


@pytest.mark.parametrize("walls", ["dense", "refined"])
def test_benchmark_obstacle_full_size(gpu_lib, walls):
    """The benchmark obstacle (40 harmonics, omega = 60) as a transmission problem with index 1.5:
    k = 90 inside, N = 1e5 nodes (2e5 unknowns); sampled exact residual rows and the energy balance
    of every angle below 1e-10.  The walls go uncompressed, or through the skeletons of a handle
    with the far-field circle inside the walls and refined against the uncompressed wall blocks
    (compress_walls = 2; with 1 they stop near 6e-10 at this frequency)."""
    import torch
    from oracle import checks
    wl = qpinputs.workload("wavy40")
    nodes, w, nrm, _ = discretize(wl.curve, wl.N)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    kw = dict(index=1.5, device=True)
    if walls == "refined":
        c0 = 0.5 * (nodes.max(0) + nodes.min(0))
        kw["far_radius"] = 0.9 * (0.5 * wl.period - abs(c0[0]))
    h = gpu_lib.Handle(t(nodes), t(w), t(nrm), wl.omega, 1e-13, **kw)
    ths = wl.thetas[::25]
    r = h.qp_solve_many(wl.period, t(ths), compress_walls=2 if walls == "refined" else -1)
    st = h.stats()
    assert st.walls_compressed == (2 if walls == "refined" else 0)
    if walls == "refined":
        assert st.refine_iters >= 1
    v = checks.bordered_residual_tr(wl.curve, wl.N, wl.omega, 1.5, wl.period, ths, r["eta"].T.cpu().numpy(),
                                    r["xi"].T.cpu().numpy(), r["flux"], n_rows=12, n_ang=4)
    assert v["sampled_rel_residual"] < 1e-10 and v["flux_err_max"] < 1e-10, v
