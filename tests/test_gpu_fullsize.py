"""Parity at the full workload sizes.

* N = 1e4 (omega = 40, the 20-harmonic obstacle): the oracle's dense Nystrom matrix and its
  LU fit the host, so the GPU solution is compared element by element with the exact dense
  block solve (bar: relative error 1e-10, both as a 2-norm per angle and as the largest entry
  error over the largest entry).  The angle set mixes the workload's random angles, four angles
  sharing one Bloch phase, angles just above the Wood's-anomaly refusal threshold (smallest
  |k_n| between 0.76 and 0.9, on the propagating and on the evanescent side) and a near-grazing
  angle (|sin theta| = 0.05).  One case runs exactly the benchmark's options: rank predictor on,
  automatic root level, compressed walls, ID tolerance 1e-13, leaves of 64, refinement off.
* N = 1e5 (omega = 60, 200 angles on 4 Bloch phases, the benchmark's launch configuration):
  the dense oracle does not fit; sampled rows of the bordered-system residual are evaluated
  by the oracle's checker on 8 angles, together with the energy balance of every angle.
"""
import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest
import scipy.linalg as sla

import qpinputs
from oracle import checks
from oracle import nystrom as ny
from oracle import periodic as pq
from paper_1301_1247_amd.geometry import discretize

pytestmark = pytest.mark.gpu

_G = {}


def _rows(r0):
    disc, om, N = _G["disc"], _G["om"], _G["N"]
    return r0, ny.matrix_kr6_rows(disc, om, np.arange(r0, min(N, r0 + 250)))


def _dense_kr6(disc, om):
    N = disc.N
    _G.update(disc=disc, om=om, N=N)
    A = np.empty((N, N), complex)
    with ProcessPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        for r0, blk in ex.map(_rows, range(0, N, 250)):
            A[r0:r0 + blk.shape[0]] = blk
    return A


def _far_walls(nodes, d):
    c = 0.5 * (nodes.max(0) + nodes.min(0))
    return 0.9 * (0.5 * d - abs(c[0]))


def _min_kn(om, d, th):
    _, _, kn = pq.bragg_orders(om, d, th, extra=2)
    return float(np.min(np.abs(kn)))


def _wood_side_angle(om, d, kmin, evanescent, offset):
    """An angle in (-pi, 0) whose closest Bragg order has |k_n| = kmin: kappa_n = -sqrt(om^2 -+ kmin^2)
    for the order n = -offset, i.e. kappa = kappa_n + 2 pi offset / d."""
    kx = math.sqrt(om * om + kmin * kmin) if evanescent else math.sqrt(om * om - kmin * kmin)
    kap = -kx + 2 * math.pi * offset / d
    return -math.acos(kap / om)


def _angles_wavy20(wl):
    om, d = wl.omega, wl.period
    th = list(wl.thetas[::6])                                             # 17 random angles
    th += list(qpinputs.shared_phase_angles(om, d, n_phase=4, per_phase=50)[[18, 23, 28, 33]])  # one phase
    th += [_wood_side_angle(om, d, 0.78, False, 37), _wood_side_angle(om, d, 0.85, True, 22)]
    th += [-math.asin(0.05)]                                              # near-grazing
    th = np.array(th)
    kmins = [_min_kn(om, d, t) for t in th]
    assert min(kmins) >= 0.76 and sorted(kmins)[1] <= 0.9
    return th


@pytest.fixture(scope="module")
def wavy20_ref():
    wl = qpinputs.workload("wavy20")
    N, om, d = wl.N, wl.omega, wl.period
    disc = ny.Discretization(wl.curve, N)
    A = _dense_kr6(disc, om)
    lu = sla.lu_factor(A)
    del A
    th = _angles_wavy20(wl)
    ct = pq.default_contour(disc, om, d)
    BL, BR = pq.wall_B(disc, om, d, ct)
    CL, CR = pq.wall_C(disc, om, d, ct)
    XL, XR = sla.lu_solve(lu, BL), sla.lu_solve(lu, BR)
    # the four alpha-free products of the Schur complement (exact algebra of Eq. 3.1)
    LL, LR, RL, RR = CL @ XL, CL @ XR, CR @ XL, CR @ XR
    Xb = sla.lu_solve(lu, pq.incident(disc, om, th))
    y0 = pq.default_y0(disc)
    ref = []
    for a, t in enumerate(th):
        al = pq.bloch_phase(om, d, t)
        S = pq.wall_Q(om, d, al, ct) - (LL + al * LR - RL / al - RR)
        xb = Xb[:, a:a + 1]
        xi = -np.linalg.solve(S, (CL - CR / al) @ xb)
        eta = (xb - (XL + al * XR) @ xi)[:, 0]
        n, kn, c, dd = pq.bragg_lattice(disc, om, d, t, eta, y0)
        ref.append((eta, xi[:, 0], n, np.concatenate([c, dd])))
    return wl, th, ref


def _check_against_ref(res, ref, bar=1e-10):
    worst = {}
    for a, (eta, xi, n, cd) in enumerate(ref):
        g_eta, g_xi = res["eta"][:, a], res["xi"][:, a]
        nm = int(res["nmodes"][a])
        assert nm == len(n) and int(res["nlo"][a]) == int(n[0])
        mx = res["bragg"].shape[0] // 2   # c_n in rows [0, maxmodes), d_n in [maxmodes, 2 maxmodes)
        g_cd = np.concatenate([res["bragg"][:nm, a], res["bragg"][mx:mx + nm, a]])
        for name, g, r in (("eta", g_eta, eta), ("xi", g_xi, xi), ("bragg", g_cd, cd)):
            e2 = np.linalg.norm(g - r) / np.linalg.norm(r)
            einf = np.abs(g - r).max() / np.abs(r).max()
            worst[name] = max(worst.get(name, 0.0), e2, einf)
            assert e2 < bar and einf < bar, (name, a, e2, einf)
    return worst


@pytest.mark.parametrize("walls", ["dense", "compressed"])
def test_qp_wavy20_full_size_vs_dense_oracle(gpu_lib, wavy20_ref, walls):
    wl, th, ref = wavy20_ref
    N, om, d = wl.N, wl.omega, wl.period
    nodes, w, nrm, _ = discretize(wl.curve, N)
    far = _far_walls(nodes, d) if walls == "compressed" else 0.0
    h = gpu_lib.Handle(nodes, w, nrm, om, 1e-13, leaf_size=wl.leaf_size, far_radius=far)
    res = h.qp_solve_many(d, th, compress_walls=1 if walls == "compressed" else -1)
    assert h.stats().walls_compressed == (walls == "compressed")
    _check_against_ref(res, ref)
    assert res["flux"].max() < 1e-8   # physics accuracy of the N = 1e4 discretization


@pytest.mark.parametrize("root_level", [0, 2])
def test_qp_wavy20_benchmark_options_vs_dense_oracle(gpu_lib, wavy20_ref, root_level):
    """The benchmark's exact option set at the largest size the dense oracle reaches: rank
    predictor on, root level automatic (and forced to 2), root inversion deferred into the solve,
    compressed walls, tol 1e-13, leaves of 64, device pointers on the torch stream, and no
    refinement step (the solution straight from the compressed inverse and the Schur step)."""
    import torch
    wl, th, ref = wavy20_ref
    N, om, d = wl.N, wl.omega, wl.period
    nodes, w, nrm, _ = discretize(wl.curve, N)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    h = gpu_lib.Handle(t(nodes), t(w), t(nrm), om, 1e-13, leaf_size=64, device=True,
                       far_radius=_far_walls(nodes, d), rank_predictor=True, root_level=root_level, defer_root=True)
    r = h.qp_solve_many(d, t(th), compress_walls=1, refine_max_iter=-1)
    st = h.stats()
    assert st.walls_compressed == 1 and st.refine_iters == 0
    assert st.rank_fallbacks >= 0 and st.root_level in ((1, 2) if root_level == 0 else (2,))
    res = {"eta": r["eta"].T.cpu().numpy(), "xi": r["xi"].T.cpu().numpy(), "bragg": r["bragg"].T.cpu().numpy(),
           "nlo": r["nlo"], "nmodes": r["nmodes"]}
    worst = _check_against_ref(res, ref)
    print(f"root_level={st.root_level} fallbacks={st.rank_fallbacks} worst={worst}", flush=True)


@pytest.mark.parametrize("walls,predictor", [("dense", False), ("compressed", False), ("compressed", True)])
def test_qp_wavy40_full_size_sampled_residual(gpu_lib, walls, predictor):
    import torch
    wl = qpinputs.workload("wavy40")
    nodes, w, nrm, _ = discretize(wl.curve, wl.N)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)
    far = _far_walls(nodes, wl.period) if walls == "compressed" else 0.0
    h = gpu_lib.Handle(t(nodes), t(w), t(nrm), wl.omega, 1e-13, leaf_size=wl.leaf_size, device=True, far_radius=far,
                       rank_predictor=predictor, defer_root=predictor)
    res = h.qp_solve_many(wl.period, t(wl.thetas), compress_walls=1 if walls == "compressed" else -1,
                          refine_max_iter=-1 if predictor else 0)
    st = h.stats()
    assert st.walls_compressed == (walls == "compressed")
    assert st.levels == 11 and st.refine_residual < 1e-12
    eta = res["eta"].T.cpu().numpy()
    xi = res["xi"].T.cpu().numpy()
    v = checks.bordered_residual(wl.curve, wl.N, wl.omega, wl.period, wl.thetas, eta, xi, res["flux"],
                                 n_rows=32, n_ang=8)
    print(f"walls={walls} predictor={predictor} fallbacks={st.rank_fallbacks} {v}", flush=True)
    assert v["sampled_rel_residual"] < 1e-10
    assert v["flux_err_max"] < 1e-8
