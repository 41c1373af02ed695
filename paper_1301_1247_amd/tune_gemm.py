"""Sweep the batched GEMM's tile configurations on the GPU and write the tuning table
(gemm_tune_default.json) that the library embeds.

    python -m paper_1301_1247_amd.tune_gemm [--workload wavy40] [--reps 3] [--out PATH]

Runs the solver's own launches: for each precision (complex128 factors, and complex64 factors
with complex128 refinement) one warm-up step, then, for every tile configuration in turn, --reps
steps of hbs_build + qp_solve_many on the seeded workload with that configuration forced on every
GEMM launch; each launch is timed with HIP events under its shape class (precision and
ceil(log2) of the largest m, n, k and of the entry count).  A class takes the configuration with
the least summed time when it beats configuration 0 (64 x 64 tiles) by more than --margin;
otherwise it is left out of the table and keeps configuration 0.  All configurations give
bitwise equal results, so the table changes run time only.  Rebuild the library afterwards
(paper_1301_1247_amd/build.py) to embed the new table.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "gemm_tune_default.json")


def _setup(workload):
    import torch

    import qpinputs
    from paper_1301_1247_amd.geometry import discretize

    wl = qpinputs.workload(workload)
    nodes, w, nrm, kap = discretize(wl.curve, wl.N)
    dev = torch.device("cuda:0")
    t = dict(nodes=torch.from_numpy(nodes).to(dev), w=torch.from_numpy(w).to(dev),
             nrm=torch.from_numpy(nrm).to(dev), kap=torch.from_numpy(kap).to(dev),
             th=torch.from_numpy(wl.thetas).to(dev))
    c0 = 0.5 * (nodes.max(0) + nodes.min(0))
    far = 0.9 * (0.5 * wl.period - abs(c0[0]))
    return wl, t, far


def sweep(workload="wavy40", reps=3, precisions=("fp64", "fp32"), tol=1e-13, log=print):
    """{precision: {cfg: {key: (ms, launches)}}} summed over reps steps per configuration."""
    import torch

    from paper_1301_1247_amd import binding as B

    wl, t, far = _setup(workload)
    stream = torch.cuda.current_stream()
    out = {}
    for prec in precisions:
        kw = dict(quad=wl.quad, leaf_size=wl.leaf_size, curvature=t["kap"] if wl.quad == "kress" else None,
                  device=True, stream=stream.cuda_stream, precision=prec, rank_predictor=True, far_radius=far)

        def step():
            h = B.Handle(t["nodes"], t["w"], t["nrm"], wl.omega, tol, **kw)
            h.qp_solve_many(wl.period, t["th"], compress_walls=1)
            h.free()

        step()
        torch.cuda.synchronize()
        out[prec] = {}
        for cfg in sorted(B.GEMM_CONFIGS):
            B.gemm_tune_begin(cfg)
            try:
                t0 = time.perf_counter()
                for _ in range(reps):
                    step()
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
            finally:
                times = B.gemm_tune_end()
            out[prec][cfg] = times
            tot = sum(v[0] for v in times.values())
            log(f"{prec} cfg {cfg} {B.GEMM_CONFIGS[cfg]}: {len(times)} classes, GEMM {tot / reps:.2f} ms/step, "
                f"wall {1e3 * wall / reps:.1f} ms/step")
    return wl, out


def choose(times_by_cfg, margin=0.03):
    """{key: cfg} for the classes whose fastest configuration beats configuration 0 by > margin,
    and per-class records (times under every configuration)."""
    keys = sorted(set().union(*[set(v) for v in times_by_cfg.values()]))
    table, rows = {}, []
    for k in keys:
        ms = {c: times_by_cfg[c][k][0] for c in times_by_cfg if k in times_by_cfg[c]}
        la = max(times_by_cfg[c][k][1] for c in times_by_cfg if k in times_by_cfg[c])
        best = min(ms, key=ms.get)
        cfg = best if 0 in ms and ms[best] < (1.0 - margin) * ms[0] else 0
        if cfg != 0:
            table[k] = cfg
        rows.append(dict(key=k, cfg=cfg, launches=la, ms={str(c): round(v, 5) for c, v in sorted(ms.items())}))
    return table, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="wavy40")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--margin", type=float, default=0.03)
    ap.add_argument("--precisions", default="fp64,fp32")
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()

    import torch

    from paper_1301_1247_amd import binding as B

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    wl, res = sweep(args.workload, args.reps, tuple(args.precisions.split(",")), log=log)
    # a class met in several runs (the complex128 levels of the complex64 run) sums its times
    merged = {}
    for by_cfg in res.values():
        for cfg, times in by_cfg.items():
            m = merged.setdefault(cfg, {})
            for k, (ms, la) in times.items():
                t0, l0 = m.get(k, (0.0, 0))
                m[k] = (t0 + ms, l0 + la)
    table, rows = choose(merged, args.margin)
    summary = {}
    for prec, by_cfg in res.items():
        base = sum(v[0] for v in by_cfg[0].values()) / args.reps
        tuned = sum(by_cfg[table.get(k, 0)][k][0] for k in by_cfg[0]) / args.reps
        summary[prec] = dict(gemm_ms_per_step_cfg0=round(base, 4), gemm_ms_per_step_tuned=round(tuned, 4))
        log(f"{prec}: GEMM {base:.2f} ms/step with 64 x 64 tiles, {tuned:.2f} ms/step with the table")
    doc = {
        "device": torch.cuda.get_device_name(0),
        "workload": f"{wl.name}: N={wl.N}, omega={wl.omega}, {len(wl.thetas)} angles, hbs_build + qp_solve_many",
        "reps": args.reps,
        "margin": args.margin,
        "configs": {str(c): list(v) for c, v in B.GEMM_CONFIGS.items()},
        "key": "complex64 << 24 | ceil log2 m << 18 | ceil log2 n << 12 | ceil log2 k << 6 | ceil log2 count",
        "summary": summary,
        "table": [dict(key=k, cfg=c) for k, c in sorted(table.items())],
        "classes": rows,
    }
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(json.dumps({"out": args.out, "entries": len(table), "summary": summary}), flush=True)


if __name__ == "__main__":
    main()
