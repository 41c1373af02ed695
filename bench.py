"""Benchmark: incident-angle solves per second of the full hot path on one MI355X.

One step = hbs_build (recursive skeletonization of the N x N Nystrom matrix) + qp_solve_many
over every incident angle of the workload (one application of A^{-1} to the wall and incident
columns, the Schur step per Bloch phase, refinement check, Bragg amplitudes), with the geometry
already resident in HBM.  value = angles per second over the timed steps.

Default workload "wavy40": seeded 40-harmonic obstacle, N = 1e5, omega = 60, d = 2 pi, 200 angles
on 4 shared Bloch phases, rank predictor on, complex128.

Also reported on the same JSON line:
* kernel_families: summed HIP-event time per kernel family over the timed steps (events recorded on
  the stream each launch is issued on), its share, and the achieved rate against the family's
  roofline; `roofline` is the family with the largest time, `rooflines` every family above 5%;
* variants: the same workload without the rank predictor, with the complex64 preconditioner, and
  with Alpert's quadrature instead of Kapur-Rokhlin's (verified against Alpert rows);
* c5: the 64-obstacle batch with a predictor trained on 48 obstacles, held-out rate with and without
  the predictor;
* paper_grating: the paper's own d = 1 star grating (Sec. 6.1) at N = 2^17 with P = 1, build and solve
  times beside the paper's laptop figures;
* wood_sweep: the benchmark obstacle under the angle sweep of Sec. 6.2 (200 angles, 21 Bloch phases,
  exact Wood's anomalies included);
* verify: sampled residual rows of the bordered system of the timed solution (oracle checker, CPU)
  and the energy balance; a failed check voids `value`;
* cpu_baseline: the oracle (dense Nystrom + LU) timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "incident-angle solves/sec at N=1e5, rel err<=1e-10; HBS build time (s)"
FP64_PEAK = 78.6      # TFLOP/s: FP64 MFMA and FP64 vector (MI355X, dense)
FP32_MFMA_PEAK = 157.3
CSRC = os.path.join(ROOT, "paper_1301_1247_amd", "csrc")

# kernel family -> (kernels, bound, peak TFLOP/s, source whose counters the traffic file belongs to)
FAMILIES = {
    "zgemm": ("k_gemm<double, *, *>", "mfma", FP64_PEAK, "gemm.hip"),
    "zinv": ("k_gj_step<double>", "alu", FP64_PEAK, "kernels_build.hip"),
    "cpqr": ("k_cpqr<*>, k_cpqrm_*", "alu", FP64_PEAK, "kernels_build.hip"),
    "sketch": ("k_sketch", "alu", FP64_PEAK, "kernels_build.hip"),
    "assemble": ("k_eval_blocks, k_proxy, k_gen_B, k_gen_C", "alu", FP64_PEAK, "kernels_build.hip"),
    "bragg": ("k_bragg_basis, k_bragg", "alu", FP64_PEAK, "kernels_qp.hip"),
    "cgemm": ("k_gemm<float, *, *>", "mfma", FP32_MFMA_PEAK, "gemm.hip"),
    "cinv": ("k_gj_step<float>", "alu", 157.3, "kernels_build.hip"),
}
WORK = {
    "zgemm": "8 m n k flops per complex product",
    "cgemm": "8 m n k flops per complex product",
    "zinv": "8 n^3 flops per n x n Gauss-Jordan inversion, over its 16-column panel launches",
    "cinv": "8 n^3 flops per n x n Gauss-Jordan inversion",
    "cpqr": "16 s n k flops per box (s x n sketch, rank k)",
    "sketch": "8 s m n flops per box (s sketch rows, m x n compression matrix)",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(family, workload):
    """HBM bytes per launch of the family's kernel from the committed rocprofv3 counter runs
    (profiles/<family>_<workload>_traffic.txt: FETCH_SIZE and WRITE_SIZE per dispatch, KiB, scaled
    by the factors a plain copy of known size gives), or None when the kernel's source has changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{family}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(CSRC, FAMILIES[family][3])
    if kv.get("source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return 1024.0 * (float(kv["fetch_kib_per_launch"]) * float(kv["fetch_factor"]) +
                     float(kv["write_kib_per_launch"]) * float(kv["write_factor"]))


def cpu_baseline(wl, n_sample=4000, q_sample=4):
    """The oracle, as it stands, on a bounded sample of the workload: the same obstacle, frequency,
    period and one angle of each Bloch phase, at N = n_sample (dense Nystrom assembly, then for every
    angle the bordered system by one LU of A and the Schur complement of Eq. 3.1).  The rate is the
    one measured at that N; the cube-law estimate at the workload's N is given beside it, labelled."""
    from threadpoolctl import threadpool_info
    from oracle import nystrom as ny
    from oracle import periodic as pq

    disc = ny.Discretization(wl.curve, n_sample)
    per = len(wl.thetas) // 4
    th = wl.thetas[::per][:q_sample]
    t0 = time.perf_counter()
    r = pq.solve_qp(disc, n_sample, wl.omega, wl.period, th, quad=wl.quad, method="schur")
    t = time.perf_counter() - t0
    Ms = len(r["contour"].k)
    threads = sum(x.get("num_threads", 0) for x in threadpool_info() if x.get("user_api") == "blas") or os.cpu_count()
    est = (q_sample / t) / (((wl.N + 2 * Ms) / (n_sample + 2 * Ms)) ** 3)
    return {"value": q_sample / t, "unit": "angles/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{wl.name} obstacle, omega={wl.omega}, d=2pi at N={n_sample} (the workload has N={wl.N}), "
                      f"{q_sample} angles (one per Bloch phase), dense assembly + one LU and Schur solve per angle: "
                      f"{t:.1f} s measured",
            "estimate_at_workload_N": {"value": est, "unit": "angles/s",
                                       "how": "measured rate scaled by ((N+2M)/(Ns+2M))^3 (dense LU cost); "
                                              "an estimate, not a measurement"}}


def verify(wl, res, n_rows=48, n_ang=8, quad="kr6"):
    """Sampled rows of the bordered-system residual of the timed solution, by the oracle's checker
    (exact dense rows of A in the solve's quadrature and of B, all rows of C and Q), plus the flux
    error of every angle."""
    from oracle import checks
    v = checks.bordered_residual(wl.curve, wl.N, wl.omega, wl.period, wl.thetas, res["eta"], res["xi"],
                                 res["flux"], n_rows=n_rows, n_ang=n_ang, quad=quad)
    v["kind"] = "sampled residual of the bordered system (Eq. 2.19) relative to |b|, not a forward error"
    v["ok"] = bool(v["sampled_rel_residual"] <= 1e-10 and v["flux_err_max"] <= 1e-8)
    return v


def family_table(B, steps, cpqr_flops_step):
    """Per kernel family: summed event time, launches, algorithmic flops, rate and roofline fraction."""
    fams = {}
    for fam in FAMILIES:
        p = B.profile_read(fam)
        if p["launches"] == 0:
            continue
        flops = p["flops"]
        if fam == "cpqr":
            flops = cpqr_flops_step * steps
        if fam in ("assemble", "bragg"):
            flops = 0.0
        kernels, bound, peak, _ = FAMILIES[fam]
        ach = flops / (p["ms"] * 1e-3) / 1e12 if p["ms"] > 0 and flops > 0 else None
        fams[fam] = {"kernels": kernels, "ms_per_step": p["ms"] / steps, "launches_per_step": p["launches"] / steps,
                     "avg_launch_ms": p["ms"] / p["launches"], "flops_per_launch": flops / p["launches"] if flops else None,
                     "achieved": ach, "peak": peak, "unit": "TFLOP/s", "bound": bound,
                     "frac": ach / peak if ach is not None else None, "work": WORK.get(fam)}
    tot = sum(f["ms_per_step"] for f in fams.values())
    for f in fams.values():
        f["share"] = f["ms_per_step"] / tot if tot > 0 else 0.0
    return fams


def run_steps(B, torch, wl, t_nodes, t_w, t_nrm, t_th, kw, tol, cw, steps, warmup, profile=False):
    def step():
        h = B.Handle(t_nodes, t_w, t_nrm, wl.omega, tol, **kw)
        res = h.qp_solve_many(wl.period, t_th, compress_walls=cw)
        return h, res

    for i in range(warmup):
        h, res = step()
        log(f"warmup {i}: build {h.stats().build_seconds:.3f} s, refine residual {h.stats().refine_residual:.2e}")
        del h, res
    torch.cuda.synchronize()
    if profile:
        B.profile_enable(True)
    builds = []
    t0 = time.perf_counter()
    for i in range(steps):
        h, res = step()
        builds.append(h.stats().build_seconds)
        if i < steps - 1:
            del h, res
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    return h, res, t, builds


def host_solution(res):
    return {"eta": res["eta"].T.cpu().numpy(), "xi": res["xi"].T.cpu().numpy(), "flux": res["flux"]}


def c5_batch(B, torch, steps=3):
    """The 64-obstacle batch: even obstacles from the 20-harmonic family (a_k ~ U(0, 0.3/k)), odd ones
    from the 40-harmonic family (a_k ~ U(0, 0.2/k)); N = rng.integers(2000, 50001) rounded to even,
    omega ~ U[10, 80], seeds 1301500 + i, 50 angles each away from Wood's anomalies.  A predictor is
    trained on the features and CPQR ranks of obstacles i < 48 (built without it) on the GPU; the
    16 held out are then built and solved with and without it, angles/s over the held-out set."""
    import numpy as np
    import qpinputs
    from paper_1301_1247_amd import train_rank_mlp as tr
    from paper_1301_1247_amd.geometry import discretize

    members = qpinputs.c5_batch()
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    geo = []
    for m in members:
        nodes, w, nrm, _ = discretize(m["curve"], m["N"])
        c0 = 0.5 * (nodes.max(0) + nodes.min(0))
        far = 0.9 * (0.5 * m["period"] - abs(c0[0]))
        geo.append((t(nodes), t(w), t(nrm), t(m["thetas"]), far))
    # training data: every box of the 48 training obstacles, built without the predictor
    feats, ranks = [], []
    t0 = time.perf_counter()
    for m, g in zip(members[:48], geo[:48]):
        h = B.Handle(g[0], g[1], g[2], m["omega"], m["tol"], device=True, far_radius=g[4])
        f, k, lv, _ = h.rank_features()
        feats.append(f)
        ranks.append(k)
        del h
    x = np.concatenate(feats)
    y = np.log(np.maximum(np.concatenate(ranks), 1)).astype(np.float32)
    p0 = tr.initial_params(x, seed=1301)
    p1, hist = B.mlp_train(p0, x, y, tau=0.9, steps=3000, lr=3e-3)
    t_train = time.perf_counter() - t0
    held = list(zip(members[48:], geo[48:]))

    def rate(predictor):
        nang = 0
        fallbacks = 0
        flux = 0.0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            for m, g in held:
                h = B.Handle(g[0], g[1], g[2], m["omega"], m["tol"], device=True, far_radius=g[4],
                             rank_predictor=predictor, rank_model=p1 if predictor else None)
                r = h.qp_solve_many(m["period"], g[3], compress_walls=1)
                nang += len(m["thetas"])
                fallbacks += h.stats().rank_fallbacks
                flux = max(flux, float(np.max(r["flux"])))
                del h, r
        torch.cuda.synchronize()
        return nang / (time.perf_counter() - t1), fallbacks / steps, flux

    rate(True)   # warm-up
    rate(False)
    on, fb, flux_on = rate(True)
    off, _, flux_off = rate(False)
    cov, ratio = [], []
    for m, g in held:
        h = B.Handle(g[0], g[1], g[2], m["omega"], m["tol"], device=True, far_radius=g[4], rank_predictor=True,
                     rank_model=p1)
        f, k, lv, pr = h.rank_features()
        top = lv > 1
        cov.append(float((pr[top] >= k[top]).mean()))
        ratio.append(float(np.mean(pr[top] / np.maximum(k[top], 1))))
        del h
    return {"obstacles": len(members), "train": 48, "held_out": len(held), "angles_each": 50,
            "angles_per_s_predictor": on, "angles_per_s_no_predictor": off, "speedup": on / off,
            "rank_fallbacks_per_pass": fb, "held_out_rank_coverage": float(np.mean(cov)),
            "held_out_mean_predicted_over_actual": float(np.mean(ratio)),
            "train_boxes": int(len(y)), "train_seconds_incl_builds": t_train,
            "train_loss_first_last": [float(hist[0]), float(hist[-1])],
            "flux_err_max": max(flux_on, flux_off),
            "note": "flux of the low-N / high-omega members measures their discretization, not the solver"}


def grating(B, torch, steps=3, warmup=1):
    """The paper's own scaling workload of Sec. 6.1: star r = 0.35 + 0.105 cos 3t in a grating of period
    d = 1, omega = 10, theta = -pi/5, N = 2^17, P = 1 neighbour images (their near points inside the
    proxy circles are explicit columns), contour spacing 0.2 (the paper keeps M = 90 here).  Build and one-angle solve timed separately; the paper's
    figures for this workload on its laptop are quoted as context, not as a target."""
    import numpy as np
    import qpinputs
    from oracle import checks
    from paper_1301_1247_amd.geometry import discretize

    wl = qpinputs.workload("star_d1")
    nodes, w, nrm, _ = discretize(wl.curve, wl.N)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    tn, tw, tr, tth = t(nodes), t(w), t(nrm), t(wl.thetas)
    kw = dict(device=True, leaf_size=wl.leaf_size, far_radius=1.0, image_period=wl.period)
    # contour spacing 0.2 (M = 368): at this gap the oracle's solution moves by 2e-14 from spacing 0.1
    hc = 0.2
    tb, ts = [], []
    for i in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = B.Handle(tn, tw, tr, wl.omega, 1e-12, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = h.qp_solve_many(wl.period, tth, P=1, h=hc)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if i >= warmup:
            tb.append(t1 - t0)
            ts.append(t2 - t1)
        if i < warmup + steps - 1:
            del h, res
    st = h.stats()
    v = checks.bordered_residual(wl.curve, wl.N, wl.omega, wl.period, wl.thetas, res["eta"].T.cpu().numpy(),
                                 res["xi"].T.cpu().numpy(), res["flux"], n_rows=48, n_ang=1, P=1, h=hc)
    ok = v["sampled_rel_residual"] < 1e-10 and v["flux_err_max"] < 1e-10
    build, solve = float(np.median(tb)), float(np.median(ts))
    return {"workload": "star r=0.35+0.105cos3t, d=1, omega=10, theta=-pi/5, N=2^17, P=1, tol 1e-12, "
                        "contour spacing 0.2",
            "build_seconds": build, "solve_seconds": solve, "angles_per_s": 1.0 / solve if ok else None,
            "angles_per_s_incl_build": 1.0 / (build + solve) if ok else None,
            "root_size": st.root_size, "levels": st.levels, "image_samples": st.image_samples,
            "contour_M": st.contour_M, "refine_iters": st.refine_iters, "verify": dict(v, ok=bool(ok)),
            "paper_context": {"precompute_s": 114.0, "block_solve_s": 32.0, "neighbour_rank": 58,
                              "hardware": "Intel i5-2540M laptop, 2 cores, MATLAB (Sec. 6.1)"}}


def grating_tr(B, torch, steps=3, warmup=1):
    """The transmission case of Sec. 6.1: the same d = 1 star grating with refractive index 1.5 inside
    the obstacle (Sec. 5), N = 2^17 nodes = 2^18 interlaced unknowns, P = 1 with the images' near points
    as explicit columns, contour spacing 0.2, tol 1e-13.  Build and one-angle solve timed separately;
    checked by sampled exact rows of the bordered residual and by the energy balance."""
    import numpy as np
    import qpinputs
    from oracle import checks
    from paper_1301_1247_amd.geometry import discretize

    wl = qpinputs.workload("star_d1_tr")
    nodes, w, nrm, _ = discretize(wl.curve, wl.N)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    tn, tw, tr, tth = t(nodes), t(w), t(nrm), t(wl.thetas)
    kw = dict(device=True, leaf_size=wl.leaf_size, far_radius=1.0, image_period=wl.period, index=wl.index)
    hc, tol = 0.2, 1e-13
    tb, ts = [], []
    for i in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = B.Handle(tn, tw, tr, wl.omega, tol, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = h.qp_solve_many(wl.period, tth, P=1, h=hc)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if i >= warmup:
            tb.append(t1 - t0)
            ts.append(t2 - t1)
        if i < warmup + steps - 1:
            del h, res
    st = h.stats()
    v = checks.bordered_residual_tr(wl.curve, wl.N, wl.omega, wl.index, wl.period, wl.thetas,
                                    res["eta"].T.cpu().numpy(), res["xi"].T.cpu().numpy(), res["flux"], n_rows=16,
                                    n_ang=1, P=1, h=hc)
    ok = v["sampled_rel_residual"] < 1e-10 and v["flux_err_max"] < 1e-10
    build, solve = float(np.median(tb)), float(np.median(ts))
    return {"workload": "transmission, index 1.5: star r=0.35+0.105cos3t, d=1, omega=10, theta=-pi/5, N=2^17 "
                        "(2^18 unknowns), P=1, tol 1e-13, contour spacing 0.2",
            "build_seconds": build, "solve_seconds": solve, "angles_per_s": 1.0 / solve if ok else None,
            "angles_per_s_incl_build": 1.0 / (build + solve) if ok else None,
            "root_size": st.root_size, "levels": st.levels, "max_rank": st.max_rank,
            "contour_M": st.contour_M, "refine_iters": st.refine_iters, "verify": dict(v, ok=bool(ok)),
            "paper_context": {"hardware": "Intel i5-2540M laptop, 2 cores, MATLAB (Sec. 6.1); its transmission "
                                          "timings are given in a figure only"}}


def wood_sweep(B, torch, wl, t_nodes, t_w, t_nrm, kw, tol, cw, steps=2, warmup=1):
    """The wavy40 obstacle under the angle sweep of Sec. 6.2: 200 angles, cos(theta) spaced by
    2 pi / (21 omega d) from grazing, 21 Bloch phases; the phase alpha = 1 holds exact Wood's
    anomalies (some k_n = 0) and its neighbours near ones, solved on the displaced contour with the
    added Rayleigh-Bloch waves.  Build + solve per step like the headline.  Checked by the energy
    balance of every angle and by sampled residual rows for 8 angles off the displaced contour."""
    import numpy as np
    import qpinputs
    from oracle import checks

    th = qpinputs.wood_sweep_angles(wl.omega, wl.period)
    t_th = torch.from_numpy(th).to("cuda")
    h, res, t, builds = run_steps(B, torch, wl, t_nodes, t_w, t_nrm, t_th, kw, tol, cw, steps, warmup)
    st = h.stats()
    sol = host_solution(res)
    kap = wl.omega * np.cos(th)
    kn = [np.sqrt(np.abs(wl.omega ** 2 - (k + 2 * np.pi * np.arange(-80, 81) / wl.period) ** 2)).min() for k in kap]
    plain = np.nonzero(np.array(kn) >= 1.5)[0]   # well clear of the 0.75 switch: undisplaced contour
    pick = plain[np.linspace(0, len(plain) - 1, 8).astype(int)]
    v = checks.bordered_residual(wl.curve, wl.N, wl.omega, wl.period, th, sol["eta"], sol["xi"], sol["flux"],
                                 n_rows=32, angles=pick)
    ok = v["sampled_rel_residual"] <= 1e-10 and v["flux_err_max"] <= 1e-8
    return {"workload": f"{wl.name} obstacle, {len(th)} angles, cos(theta) step 2 pi/(21 omega d) from grazing",
            "angles": int(len(th)), "value": len(th) * steps / t if ok else None, "unit": "angles/s",
            "ms_per_step": 1000.0 * t / steps, "wood_angles": st.wood_angles, "wood_orders": st.wood_orders,
            "exact_anomalies": int(sum(1 for x in kn if x < 1e-5)), "verify": dict(v, ok=bool(ok))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="wavy40")
    ap.add_argument("--tol", type=float, default=1e-13)
    ap.add_argument("--walls", choices=("compressed", "dense"), default="compressed",
                    help="compressed: wall blocks through the root skeletons (needs the far-field circle)")
    ap.add_argument("--rank-predictor", choices=("on", "off"), default="on",
                    help="size each box's sketch from the MLP rank prediction (off: worst case 2n + 8)")
    ap.add_argument("--precision", choices=("fp64", "fp32"), default="fp64",
                    help="fp32: complex64 inverse factors as a preconditioner, FP64 refinement")
    ap.add_argument("--defer-root", choices=("on", "off"), default="on",
                    help="on: the root matrix is inverted in the first solve, batched with its capacitance inversions")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the no-predictor and fp32 rates")
    ap.add_argument("--no-c5", action="store_true", help="skip the 64-obstacle batch")
    ap.add_argument("--no-grating", action="store_true", help="skip the paper's d = 1 star grating at N = 2^17")
    ap.add_argument("--no-wood", action="store_true", help="skip the angle sweep through Wood's anomalies")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU (asked for --gpus {args.gpus}); splitting the angles and "
              "Bloch phases over GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    # the library's device-memory cache: each step builds a new handle, and the transmission legs'
    # handle and solve hold up to 84 GB, beyond the 64 GiB default (they would allocate and free it
    # every step); 160 GiB (172 GB) leaves about 115 GB of the 288 for the live handle and torch
    os.environ.setdefault("QPS_POOL_MAX_GB", "160")
    import numpy as np
    import torch

    import qpinputs
    from paper_1301_1247_amd import binding as B
    from paper_1301_1247_amd.geometry import discretize

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    wl = qpinputs.workload(args.workload)
    nodes, w, nrm, kap = discretize(wl.curve, wl.N)
    dev = torch.device("cuda:0")
    t_nodes = torch.from_numpy(nodes).to(dev)
    t_w = torch.from_numpy(w).to(dev)
    t_nrm = torch.from_numpy(nrm).to(dev)
    t_kap = torch.from_numpy(kap).to(dev)
    t_th = torch.from_numpy(wl.thetas).to(dev)
    stream = torch.cuda.current_stream()
    nang = len(wl.thetas)
    base_kw = dict(quad=wl.quad, leaf_size=wl.leaf_size, curvature=t_kap if wl.quad == "kress" else None, device=True,
                   stream=stream.cuda_stream)
    if args.walls == "compressed":
        # far-field circle about the bounding-box centre that stays inside the unit cell's walls
        c0 = 0.5 * (nodes.max(0) + nodes.min(0))
        base_kw["far_radius"] = 0.9 * (0.5 * wl.period - abs(c0[0]))
    cw = 1 if args.walls == "compressed" else -1
    # the root inversion runs in the solve's batch of capacitance inversions (build_seconds leaves it out)
    base_kw["defer_root"] = args.defer_root == "on"
    kw = dict(base_kw, precision=args.precision, rank_predictor=args.rank_predictor == "on")

    h, res, t, builds = run_steps(B, torch, wl, t_nodes, t_w, t_nrm, t_th, kw, args.tol, cw, args.steps, args.warmup,
                                  profile=True)
    st = h.stats()
    fams = family_table(B, args.steps, 16.0 * st.cpqr_work)
    B.profile_enable(False)
    log(f"timed {args.steps} steps in {t:.3f} s")
    ms = 1000.0 * t / args.steps
    value = nang * args.steps / t
    # the dominant family and every family above 5% of the summed kernel time
    dom = max(fams, key=lambda f: fams[f]["ms_per_step"])
    rl = {}
    for fam, f in sorted(fams.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        if f["share"] >= 0.05 and f["achieved"] is not None:
            rl[fam] = {"kernel": f["kernels"], "bound": f["bound"], "achieved": f["achieved"], "peak": f["peak"],
                       "unit": "TFLOP/s", "frac": f["frac"], "share": f["share"], "avg_launch_ms": f["avg_launch_ms"],
                       "flops_per_launch": f["flops_per_launch"], "work": f["work"]}
    d = fams[dom]
    roofline = {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": "TFLOP/s",
                "frac": d["frac"], "traffic": measured_traffic(dom, wl.name) if wl.name == "wavy40" else None,
                "kernel": d["kernels"], "family": dom, "share_of_kernel_time": d["share"],
                "avg_launch_ms": d["avg_launch_ms"], "flops_per_launch": d["flops_per_launch"],
                "launches_per_step": d["launches_per_step"], "work": d["work"],
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "angles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if args.precision == "fp64" else "c64+c128",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: seeded obstacle, N={wl.N}, omega={wl.omega}, d=2pi, "
                               f"{nang} angles, tol={args.tol:g}, KR6 + proxy compression, {args.precision} factors, "
                               f"{args.walls} walls, rank predictor {args.rank_predictor}",
                   "N": wl.N, "omega": wl.omega, "angles": nang, "contour_M": st.contour_M,
                   "walls": args.walls, "precision": args.precision, "rank_predictor": args.rank_predictor,
                   "defer_root": args.defer_root},
        "build_seconds": float(np.median(builds)),
        "build_seconds_note": ("hbs_build without the root inversion (defer_root: it runs inside the solve)"
                               if args.defer_root == "on" else "hbs_build including the root inversion"),
        "levels": st.levels, "max_rank": st.max_rank, "root_size": st.root_size, "root_level": st.root_level,
        "refine_iters": st.refine_iters, "refine_residual": st.refine_residual,
        "rank_fallbacks": st.rank_fallbacks, "sketch_bytes_max": st.sketch_bytes_max,
        "roofline": roofline,
        "rooflines": rl,
        "kernel_families": fams,
    }
    if not args.no_verify:
        out["verify"] = verify(wl, host_solution(res))
        if not out["verify"]["ok"]:
            out["invalid"] = "the timed solution failed the residual / energy check: value withheld"
            out["value"] = None
    del h, res
    if not args.no_variants and args.precision == "fp64" and args.rank_predictor == "on":
        variants = {}
        for name, vkw in (("no_rank_predictor", dict(kw, rank_predictor=False)),
                          ("fp32_preconditioner", dict(kw, precision="fp32")),
                          ("alpert_quadrature", dict(kw, quad="alpert"))):
            hv, rv, tv, bv = run_steps(B, torch, wl, t_nodes, t_w, t_nrm, t_th, vkw, args.tol, cw, 3, 1)
            sv = hv.stats()
            vr = {"value": nang * 3 / tv, "unit": "angles/s", "ms_per_step": 1000.0 * tv / 3,
                  "build_seconds": float(np.median(bv)), "refine_iters": sv.refine_iters,
                  "refine_residual": sv.refine_residual, "root_level": sv.root_level}
            if not args.no_verify:
                vr["verify"] = verify(wl, host_solution(rv), quad=vkw.get("quad", "kr6"))
                if not vr["verify"]["ok"]:
                    vr["value"] = None
            variants[name] = vr
            del hv, rv
        # the transmission problem (Sec. 5, index 1.5 inside the obstacle: 2N interlaced unknowns) on
        # the same obstacle and angles, with the rank model (trained on Dirichlet boxes) off.  Its wall
        # blocks go uncompressed, or through the skeletons with the refinement's residual taking them
        # uncompressed (compress_walls = 2: through the skeletons alone they stop near 6e-10 here)
        c0 = 0.5 * (nodes.max(0) + nodes.min(0))
        for name, cwt in (("transmission_index_1.5", -1), ("transmission_index_1.5_refined_walls", 2)):
            tkw = dict(kw, rank_predictor=False, index=1.5)
            if cwt == 2:
                tkw["far_radius"] = 0.9 * (0.5 * wl.period - abs(c0[0]))
            hv, rv, tv, bv = run_steps(B, torch, wl, t_nodes, t_w, t_nrm, t_th, tkw, args.tol, cwt, 3, 1)
            sv = hv.stats()
            vr = {"value": nang * 3 / tv, "unit": "angles/s", "ms_per_step": 1000.0 * tv / 3,
                  "build_seconds": float(np.median(bv)), "unknowns": sv.unknowns, "max_rank": sv.max_rank,
                  "refine_iters": sv.refine_iters, "refine_residual": sv.refine_residual,
                  "walls": "dense" if cwt < 0 else "compressed, refined against the dense blocks",
                  "walls_compressed": sv.walls_compressed}
            if not args.no_verify:
                from oracle import checks
                hs = host_solution(rv)
                v = checks.bordered_residual_tr(wl.curve, wl.N, wl.omega, 1.5, wl.period, wl.thetas, hs["eta"],
                                                hs["xi"], hs["flux"], n_rows=16, n_ang=4)
                v["ok"] = bool(v["sampled_rel_residual"] <= 1e-10 and v["flux_err_max"] <= 1e-8
                               and sv.walls_compressed == (0 if cwt < 0 else 2))
                vr["verify"] = v
                if not v["ok"]:
                    vr["value"] = None
            variants[name] = vr
            del hv, rv
        out["variants"] = variants
    if not args.no_c5 and args.workload == "wavy40":
        out["c5"] = c5_batch(B, torch)
    if not args.no_grating and args.workload == "wavy40":
        out["paper_grating"] = grating(B, torch)
        out["paper_grating_transmission"] = grating_tr(B, torch)
    if not args.no_wood and args.workload == "wavy40":
        out["wood_sweep"] = wood_sweep(B, torch, wl, t_nodes, t_w, t_nrm, kw, args.tol, cw)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
