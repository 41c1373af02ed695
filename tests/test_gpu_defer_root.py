"""hbs_opts.defer_root: the root matrix's inversion leaves hbs_build and runs in the first call that
needs it: batched with the Woodbury capacitance inversions inside qp_solve on compressed walls
(where Cq = Q^{-1} C~_J and K2 = (R - B_J Cq)^{-1} replace the forms that need R^{-1}), inverted on
entry elsewhere.  Bar: the dense oracle's 1e-10 (2-norm and largest entry); against the same handle
built without deferral, applies agree to 1e-13 (the same inversion kernel on the same matrix)."""
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
def wavy():
    c = qpinputs.wavy(130102, 20, 0.3)
    N, om, d = 2000, 40.0, 2 * math.pi
    disc = ny.Discretization(c, N)
    A = ny.matrix(disc, om, "kr6")
    nodes, w, nrm, _ = discretize(c, N)
    cen = 0.5 * (nodes.max(0) + nodes.min(0))
    far = 0.9 * (0.5 * d - abs(cen[0]))
    return c, N, om, d, disc, A, (nodes, w, nrm), far


def test_deferred_root_qp_matches_oracle(gpu_lib, wavy):
    """At the benchmark's ID tolerance 1e-13: with 1e-12 the angle -0.2 (the worst conditioned
    here) lands at 0.9e-10 to 1.1e-10 of the oracle with or without the deferral, by the draw of
    the sketches, too close to the bar for a largest-entry check."""
    c, N, om, d, disc, A, g, far = wavy
    thetas = np.array([-1.1, -0.45, -math.acos(0.31), -math.acos(0.31 + 1 / 40), -0.2])
    h = gpu_lib.Handle(*g, om, 1e-13, far_radius=far, defer_root=True)
    res = h.qp_solve_many(d, thetas, compress_walls=1)
    assert h.stats().walls_compressed == 1
    ref = pq.solve_qp(disc, N, om, d, thetas, quad="kr6", A0=A)
    for a in range(len(thetas)):
        assert _cmp(res["eta"][:, a], ref["eta"][:, a]) < 1e-10, a
        assert _cmp(res["xi"][:, a], ref["xi"][:, a]) < 1e-10, a
        assert abs(res["flux"][a] - ref["flux"][a]) < 1e-10
    # a second solve on the same handle uses the inverse the first one formed
    res2 = h.qp_solve_many(d, thetas[:2], compress_walls=1)
    assert _cmp(res2["eta"][:, 0], ref["eta"][:, 0]) < 1e-10


def test_deferred_root_apply_equals_eager(gpu_lib, wavy):
    c, N, om, d, disc, A, g, far = wavy
    rng = np.random.default_rng(11)
    B = rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3))
    h0 = gpu_lib.Handle(*g, om, 1e-12, far_radius=far)
    x0 = h0.apply(B)
    # inverted on entry to the apply
    h1 = gpu_lib.Handle(*g, om, 1e-12, far_radius=far, defer_root=True)
    x1 = h1.apply(B)
    assert np.abs(x1 - x0).max() <= 1e-13 * np.abs(x0).max()
    # inverted in the qp_solve batch, then used by the apply
    h2 = gpu_lib.Handle(*g, om, 1e-12, far_radius=far, defer_root=True)
    h2.qp_solve_many(d, np.array([-0.7]), compress_walls=1)
    x2 = h2.apply(B)
    assert np.abs(x2 - x0).max() <= 1e-13 * np.abs(x0).max()


def test_deferred_root_uncompressed_walls_and_wood(gpu_lib, wavy):
    """Paths that do not batch it (dense walls; a Wood's-anomaly angle) invert the root on entry."""
    c, N, om, d, disc, A, g, far = wavy
    th = np.array([-0.45, -math.acos(1 - 2 * math.pi / (om * d))])
    h0 = gpu_lib.Handle(*g, om, 1e-12, far_radius=far)
    h1 = gpu_lib.Handle(*g, om, 1e-12, far_radius=far, defer_root=True)
    for cw in (1, -1):
        r0 = h0.qp_solve_many(d, th, compress_walls=cw)
        r1 = h1.qp_solve_many(d, th, compress_walls=cw)
        for a in range(len(th)):
            assert _cmp(r1["eta"][:, a], r0["eta"][:, a]) < 1e-12, (cw, a)


def test_deferred_root_noalloc(gpu_lib, wavy):
    """hbs_apply_noalloc on a handle whose root is still to be inverted: the inversion's workspace
    comes from the static scratch as well."""
    import torch
    c, N, om, d, disc, A, g, far = wavy
    t = lambda a: torch.from_numpy(a).to("cuda")
    h0 = gpu_lib.Handle(*(t(a) for a in g), om, 1e-12, device=True)
    h1 = gpu_lib.Handle(*(t(a) for a in g), om, 1e-12, device=True, defer_root=True)
    gen = torch.Generator(device="cpu").manual_seed(5)
    b = torch.complex(torch.randn((2, N), generator=gen, dtype=torch.float64),
                      torch.randn((2, N), generator=gen, dtype=torch.float64)).to("cuda")
    cached = gpu_lib.pool_cached_bytes()
    x1 = h1.apply_noalloc(b)
    assert gpu_lib.pool_cached_bytes() == cached
    x0 = h0.apply(b)
    x1, x0 = x1.cpu().numpy(), x0.cpu().numpy()
    assert np.abs(x1 - x0).max() <= 1e-13 * np.abs(x0).max()
