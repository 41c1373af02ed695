"""Benchmark: incident-angle solves per second of the full hot path on one MI355X.

One step = hbs_build (recursive skeletonization of the N x N Nystrom matrix) + qp_solve_many
over every incident angle of the workload (one application of A^{-1} to [B_L | B_R | b...],
alpha-free Schur products, per-alpha Schur inversions, refinement, Bragg amplitudes), with the
geometry already resident in HBM.  value = angles per second over the timed steps.

Default workload "wavy40": seeded 40-harmonic obstacle, N = 1e5, omega = 60, d = 2 pi,
200 angles on 4 shared Bloch phases.

Also reported: the roofline of the dominant kernel (the complex FP64 MFMA GEMM) from HIP events
on the library's stream, the oracle timed on the host cores on a bounded sample, and a
verification of the timed solution (sampled residual rows of the bordered system evaluated by
the oracle's kernels, and the energy balance).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "incident-angle solves/sec at N=1e5, rel err<=1e-10; HBS build time (s)"
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "k_gemm_wavy40_N1e5_traffic.txt")
GEMM_SRC = os.path.join(HERE, "paper_1301_1247_amd", "csrc", "gemm.hip")
GEMM_TABLE = os.path.join(HERE, "paper_1301_1247_amd", "gemm_tune_default.json")


def measured_traffic():
    """HBM bytes per complex128 GEMM launch (k_gemm<double, *, *>, every tile configuration) from the
    committed rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE per dispatch, KiB, scaled by the
    factors a plain copy of known size gives), or None when the GEMM source or its tuning table
    has changed since the counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(open(GEMM_SRC, "rb").read()).hexdigest()
    if kv.get("source_sha256") != sha:
        return None
    # the tile configurations (and so the operand re-reads) follow the embedded tuning table
    tsha = hashlib.sha256(open(GEMM_TABLE, "rb").read()).hexdigest() if os.path.exists(GEMM_TABLE) else "none"
    if kv.get("table_sha256") != tsha:
        return None
    return 1024.0 * (float(kv["fetch_kib_per_launch"]) * float(kv["fetch_factor"]) +
                     float(kv["write_kib_per_launch"]) * float(kv["write_factor"]))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(wl, n_sample=2000, q_sample=2):
    """The oracle (dense Nystrom + bordered LU per angle) on a bounded sample of the workload:
    the same obstacle, frequency, period and first angles at N = n_sample; the per-angle time is
    scaled to the workload's N by the O((N + 2M)^3) cost of the dense LU that dominates it."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import nystrom as ny
    from oracle import periodic as pq

    disc = ny.Discretization(wl.curve, n_sample)
    th = wl.thetas[:q_sample]
    t0 = time.perf_counter()
    r = pq.solve_qp(disc, n_sample, wl.omega, wl.period, th, quad=wl.quad)
    t = time.perf_counter() - t0
    Ms = len(r["contour"].k)
    dfull = ny.Discretization(wl.curve, 2000)  # only for the contour size of the workload
    Mf = len(pq.default_contour(dfull, wl.omega, wl.period).k)
    scale = ((wl.N + 2 * Mf) / (n_sample + 2 * Ms)) ** 3
    per_angle_full = t / q_sample * scale
    threads = sum(x.get("num_threads", 0) for x in threadpool_info() if x.get("user_api") == "blas") or os.cpu_count()
    return {"value": 1.0 / per_angle_full, "unit": "angles/s", "cores": int(threads), "kind": "oracle",
            "sample": f"N={n_sample}, {q_sample} angles of the same workload in {t:.1f} s "
                      f"({q_sample / t:.3g} angles/s at that N); scaled by ((N+2M)/(Ns+2Ms))^3 = {scale:.3g} "
                      f"to N={wl.N}, M={Mf}"}


def verify(wl, res, n_rows=48, n_ang=8):
    """Sampled rows of the bordered-system residual of the timed solution, by the oracle's
    checker (exact dense rows of A and B, all rows of C and Q), plus the flux error of every angle."""
    from oracle import checks
    return checks.bordered_residual(wl.curve, wl.N, wl.omega, wl.period, wl.thetas, res["eta"], res["xi"],
                                    res["flux"], n_rows=n_rows, n_ang=n_ang)


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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the sharding design is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)

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
    kw = dict(quad=wl.quad, leaf_size=wl.leaf_size, curvature=t_kap if wl.quad == "kress" else None, device=True,
              stream=stream.cuda_stream, precision=args.precision, rank_predictor=args.rank_predictor == "on")
    if args.walls == "compressed":
        # far-field circle about the bounding-box centre that stays inside the unit cell's walls
        c0 = 0.5 * (nodes.max(0) + nodes.min(0))
        kw["far_radius"] = 0.9 * (0.5 * wl.period - abs(c0[0]))
    cw = 1 if args.walls == "compressed" else -1
    fam, peak = ("zgemm", FP64_PEAK_TFLOPS) if args.precision == "fp64" else ("cgemm", FP32_PEAK_TFLOPS)

    def step():
        h = B.Handle(t_nodes, t_w, t_nrm, wl.omega, args.tol, **kw)
        res = h.qp_solve_many(wl.period, t_th, compress_walls=cw)
        return h, res

    for i in range(args.warmup):
        h, res = step()
        log(f"warmup {i}: build {h.stats().build_seconds:.3f} s, refine residual {h.stats().refine_residual:.2e}")
        del h, res
    torch.cuda.synchronize()
    B.profile_enable(True)
    builds = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        h, res = step()
        builds.append(h.stats().build_seconds)
        if i < args.steps - 1:
            del h, res
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    prof = B.profile_read(fam)
    B.profile_enable(False)
    st = h.stats()
    log(f"timed {args.steps} steps in {t:.3f} s; {fam} {prof}")
    ms = 1000.0 * t / args.steps
    value = nang * args.steps / t
    achieved = prof["flops"] / (prof["ms"] * 1e-3) / 1e12 if prof["ms"] > 0 else 0.0
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
                               f"{args.walls} walls",
                   "N": wl.N, "omega": wl.omega, "angles": nang, "contour_M": st.contour_M,
                   "walls": args.walls, "precision": args.precision, "rank_predictor": args.rank_predictor},
        "build_seconds": float(np.median(builds)),
        "levels": st.levels, "max_rank": st.max_rank, "root_size": st.root_size,
        "refine_iters": st.refine_iters, "refine_residual": st.refine_residual,
        "rank_fallbacks": st.rank_fallbacks, "sketch_bytes_max": st.sketch_bytes_max,
        "roofline": {"bound": "mfma", "kernel": ("k_gemm<double, *, *> (complex FP64 MFMA GEMM, tuned tiles)" if fam == "zgemm"
                                                 else "k_gemm<float> (complex FP32 MFMA GEMM)"),
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic() if fam == "zgemm" and wl.name == "wavy40" else None,
                     "traffic_unit": "bytes per launch", "launches": prof["launches"],
                     "avg_launch_ms": prof["ms"] / max(1, prof["launches"]),
                     "flops_per_launch": prof["flops"] / max(1, prof["launches"])},
    }
    if not args.no_verify:
        res_h = {"eta": res["eta"].T.cpu().numpy(), "xi": res["xi"].T.cpu().numpy(), "flux": res["flux"]}
        out["verify"] = verify(wl, res_h)
    del h, res
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
