"""Rank predictor on the GPU: the MLP kernels against the float64 oracle (forward, pinball-loss
gradient, training), the features exported by a build, and builds whose sketches are sized by
the predictor (accuracy unchanged, the fallback path, smaller sketches)."""
import numpy as np
import pytest
import scipy.linalg as sla

import qpinputs
from oracle import nystrom as ny
from oracle import rank_mlp as rm
from paper_1301_1247_amd.geometry import discretize

pytestmark = pytest.mark.gpu


def _problem(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 16)) * 1.5 + 0.5
    p = rm.init(x, seed)
    t = rm.forward(p, x) + rng.standard_normal(n)
    return p, x, t


def test_mlp_forward_matches_oracle(gpu_lib):
    p, x, _ = _problem(0, 1000)
    y = gpu_lib.mlp_forward(p.astype(np.float32), x.astype(np.float32))
    ref = rm.forward(p.astype(np.float32).astype(float), x.astype(np.float32).astype(float))
    assert np.abs(y - ref).max() <= 2e-5 * (1 + np.abs(ref).max())


def test_mlp_gradient_matches_oracle(gpu_lib):
    p, x, t = _problem(1, 777)
    p32, x32, t32 = (a.astype(np.float32) for a in (p, x, t))
    g, loss = gpu_lib.mlp_grad(p32, x32, t32, tau=0.9)
    g_ref = rm.grad(p32.astype(float), x32.astype(float), t32.astype(float), 0.9)
    l_ref = rm.loss(p32.astype(float), x32.astype(float), t32.astype(float), 0.9)
    assert loss == pytest.approx(l_ref, rel=1e-5)
    assert np.abs(g - g_ref).max() <= 1e-4 * np.abs(g_ref).max()
    assert np.all(g[:32] == 0)


def test_mlp_training_lowers_the_loss(gpu_lib):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3000, 16))
    teacher = rm.init(x, 7)
    t = rm.forward(teacher, x)
    p0 = rm.init(x, 3).astype(np.float32)
    p1, hist = gpu_lib.mlp_train(p0, x, t, tau=0.9, steps=400, lr=3e-3)
    assert hist[0] == pytest.approx(rm.loss(p0.astype(float), x.astype(np.float32).astype(float), t.astype(np.float32), 0.9)
                                    / len(t), rel=1e-4)
    l1 = rm.loss(p1.astype(float), x, t, 0.9) / len(t)
    assert l1 < 0.25 * hist[0]
    assert np.array_equal(p1[:32], p0[:32])   # the normalisation is not trained


@pytest.fixture(scope="module")
def wavy_case():
    c = qpinputs.wavy(130102, 20, 0.3)
    N, om = 2000, 40.0
    A = ny.matrix(ny.Discretization(c, N), om, "kr6")
    return c, N, om, sla.lu_factor(A)


def test_rank_features_of_a_build(gpu_lib, wavy_case):
    c, N, om, _ = wavy_case
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12)
    f, k, lv, pr = h.rank_features()
    L = h.stats().levels
    assert f.shape == (2 ** (L + 1) - 2, 16) and np.isfinite(f).all()
    assert (k >= 1).all() and lv.min() == 1 and lv.max() == L
    assert np.all(pr == 0)
    leaves = lv == L
    assert np.allclose(2 ** f[leaves, 0], N / 2 ** L, rtol=0.05)   # log2 n at the leaves
    assert np.all(f[leaves, 15] == 0)                              # no children below the leaves


def test_rank_features_geometry_matches_numpy(gpu_lib, wavy_case):
    """Arc length and max / mean |curvature| of every box (computed on the GPU for all levels in one
    launch) against numpy on the node data: the turning angle of the normals between a node's two
    neighbours over the arc length between them."""
    c, N, om, _ = wavy_case
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12)
    f, _, lv, _ = h.rank_features()
    a, cn = np.roll(np.arange(N), 1), np.roll(np.arange(N), -1)
    cr = nrm[a, 0] * nrm[cn, 1] - nrm[a, 1] * nrm[cn, 0]
    dt = nrm[a, 0] * nrm[cn, 0] + nrm[a, 1] * nrm[cn, 1]
    kabs = np.abs(np.arctan2(cr, dt)) / (0.5 * w[a] + w + 0.5 * w[cn])
    L = h.stats().levels
    row = 0
    for l in range(L, 0, -1):
        nb = 2 ** l
        for b in range(nb):
            lo, hi = b * N // nb, (b + 1) * N // nb
            rad = f[row, 3] / om
            assert f[row, 2] == pytest.approx(om * w[lo:hi].sum(), rel=1e-5)
            assert f[row, 8] == pytest.approx(kabs[lo:hi].max() * rad, rel=1e-5, abs=1e-6)
            assert f[row, 9] == pytest.approx(kabs[lo:hi].mean() * rad, rel=1e-5, abs=1e-6)
            row += 1
    assert row == len(lv)


def _default_model(gpu_lib):
    try:
        return gpu_lib.rank_model_default()
    except gpu_lib.HBSError:
        pytest.skip("library built without a rank model (run paper_1301_1247_amd.train_rank_mlp)")


def test_predictor_with_oversized_prediction_reproduces_the_worst_case_build(gpu_lib, wavy_case):
    """A model predicting an enormous rank sizes every sketch at the worst case 2n + 8: the build is
    then exactly the one without the predictor (same sketches, same CPQR ranks)."""
    c, N, om, _ = wavy_case
    nodes, w, nrm, _ = discretize(c, N)
    d = rm.unpack(np.zeros(rm.N_PARAM))
    d["sd"] = np.ones(16)
    d["b3"] = 20.0
    big = rm.pack(d).astype(np.float32)
    h0 = gpu_lib.Handle(nodes, w, nrm, om, 1e-12)
    h1 = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, rank_predictor=True, rank_model=big, root_level=1)
    assert np.array_equal(h0.rank_features()[1], h1.rank_features()[1])
    assert h1.stats().rank_fallbacks == 0
    assert h1.stats().sketch_bytes_max == h0.stats().sketch_bytes_max
    # with the level-1 ranks predicted at n, the automatic choice leaves level 1 uncompressed
    h2 = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, rank_predictor=True, rank_model=big)
    assert h2.stats().root_level == 2 and h0.stats().root_level == 1


def test_predicted_sketches_keep_the_accuracy(gpu_lib, wavy_case):
    c, N, om, lu = wavy_case
    _default_model(gpu_lib)
    nodes, w, nrm, _ = discretize(c, N)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3))
    xe = sla.lu_solve(lu, b)
    h0 = gpu_lib.Handle(nodes, w, nrm, om, 1e-12)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, rank_predictor=True)
    x = h.apply(b, refine=2)
    assert np.linalg.norm(x - xe) / np.linalg.norm(xe) < 1e-10
    s, s0 = h.stats(), h0.stats()
    assert s.sketch_bytes_max < s0.sketch_bytes_max and s.cpqr_work < s0.cpqr_work
    _, k, _, kp = h.rank_features()
    assert np.all(kp > 0)
    # ranks agree with the worst-case build's to within the randomness of the sketches
    k0 = h0.rank_features()[1]
    assert np.abs(k.astype(int) - k0).max() <= max(4, int(0.05 * k0.max()))


def test_under_predicted_sketches_fall_back(gpu_lib, wavy_case):
    c, N, om, lu = wavy_case
    _default_model(gpu_lib)
    nodes, w, nrm, _ = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-12, rank_predictor=True, rank_scale=0.05)
    assert h.stats().rank_fallbacks > 0
    rng = np.random.default_rng(6)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    xe = sla.lu_solve(lu, b)
    assert np.linalg.norm(h.apply(b, refine=2) - xe) / np.linalg.norm(xe) < 1e-10


@pytest.mark.parametrize("steps", [1, 2, 3])
def test_mlp_adam_steps_match_oracle(gpu_lib, steps):
    """qps_mlp_train against the oracle's Adam (mean pinball loss, zero initial moments), entry by
    entry.  Data with targets away from the predictions (no sample near the loss's kink).  An
    entry whose oracle gradient comes within 1e-4 of zero at some step is held to the bound
    lr * steps that any Adam step obeys (its sign is decided by rounding there); every other
    entry to 1e-2 lr + float rounding of the parameter."""
    rng = np.random.default_rng(11)
    n = 500
    x = (rng.standard_normal((n, 16)) * 1.5 + 0.5).astype(np.float32)
    p0 = rm.init(x.astype(float), 4).astype(np.float32)
    y = rm.forward(p0.astype(float), x.astype(float))
    t = (y + np.where(rng.random(n) < 0.5, -1.0, 1.0) * rng.uniform(0.5, 2.0, n)).astype(np.float32)
    lr = 1e-3
    p_gpu, hist = gpu_lib.mlp_train(p0, x, t, tau=0.9, steps=steps, lr=lr)
    xd, td = x.astype(float), t.astype(float)
    p_ref, hist_ref = rm.train(p0.astype(float), xd, td, 0.9, steps, lr)
    # the oracle's gradients along its own path, for the near-zero mask
    pp = p0.astype(float)
    m = np.zeros_like(pp)
    v = np.zeros_like(pp)
    gmin = np.full(pp.size, np.inf)
    for it in range(1, steps + 1):
        g = rm.grad(pp, xd, td, 0.9) / n
        gmin = np.minimum(gmin, np.abs(g))
        pp, m, v = rm.adam_step(pp, g, m, v, it, lr)
    assert np.array_equal(pp, p_ref)
    assert np.abs(hist - hist_ref).max() <= 1e-5 * np.abs(hist_ref).max()
    assert np.array_equal(p_gpu[:32], p0[:32])
    d = np.abs(p_gpu.astype(float) - p_ref)
    # float32 gradients sum 500 samples (absolute error ~1e-7): an entry of |g| > 1e-4 is off by
    # < 1e-3 relative, which moves a later Adam step (m / sqrt(v)) by about that fraction of lr;
    # a wrong moment rate or bias correction moves it by O(lr)
    firm = gmin > 1e-4
    assert firm[32:].mean() > 0.8
    assert d[firm].max() <= 1e-2 * lr + 4e-7 * np.abs(p_ref[firm]).max()
    assert d.max() <= lr * steps * 1.001 + 1e-6
