"""Fit the library's built-in rank predictor (rank_mlp_default.json) on the GPU.

    python -m paper_1301_1247_amd.train_rank_mlp [--out PATH] [--steps N]

Builds the seeded training obstacles of ``qpinputs.rank_training_set`` with the predictor off,
collects every box's 16 features and the rank its column-pivoted QR chose, and fits the MLP to
log(rank) with the pinball loss at tau = 0.9 (the model errs toward over-prediction, and a box
whose sketch still turns out too short is redone at full size by the build).  Training, the
forward and backward passes and the Adam steps run in the library's HIP kernels.  The last 8
obstacles are held out; their coverage (fraction of boxes needing no fallback) and the mean
over-prediction are written next to the parameters.  Rebuild the library afterwards
(paper_1301_1247_amd/build.py) to embed the new model.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

import qpinputs
from paper_1301_1247_amd import binding as B
from paper_1301_1247_amd.geometry import discretize

HERE = os.path.dirname(os.path.abspath(__file__))
FEATURES = ["log2 n", "level / L", "omega * arc length", "omega * box radius", "omega * proxy radius",
            "near points / n", "proxy points / 100", "log10 tol", "max |curvature| * radius",
            "mean |curvature| * radius", "omega * gap to non-adjacent near boxes", "omega / 100",
            "chord / arc length", "bounding-box aspect ratio", "omega * far-field radius (0 if none)",
            "log2(1 + sum of the children's ranks)"]


def collect(cfgs, period=2 * math.pi, log=print):
    xs, ks = [], []
    for i, c in enumerate(cfgs):
        nodes, w, nrm, _ = discretize(c["curve"], c["N"])
        far = 0.0
        if c["far"]:
            c0 = 0.5 * (nodes.max(0) + nodes.min(0))
            far = 0.9 * (0.5 * period - abs(c0[0]))
        h = B.Handle(nodes, w, nrm, c["omega"], c["tol"], leaf_size=64, far_radius=far)
        f, k, _, _ = h.rank_features()
        h.free()
        xs.append(f)
        ks.append(k)
        log(f"  obstacle {i}: N={c['N']} omega={c['omega']:.1f} tol={c['tol']:g} far={c['far']} boxes={len(k)} "
            f"max rank={k.max()}")
    return np.concatenate(xs), np.concatenate(ks)


def init_params(x, seed=0):
    rng = np.random.default_rng(seed)
    mu = x.mean(0)
    sd = x.std(0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    parts = [mu, sd, rng.standard_normal((64, 16)).ravel() / 4.0, np.zeros(64),
             rng.standard_normal((64, 64)).ravel() / 8.0, np.zeros(64), rng.standard_normal(64) / 8.0, np.zeros(1)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == B.rank_model_size()
    return p


initial_params = init_params


def coverage(params, x, k, margin=8.0):
    """Fraction of boxes whose rank stays below the predicted sketch (1.25 k^ + 16) minus the margin."""
    kp = np.exp(B.mlp_forward(params, x).astype(np.float64))
    ok = k < np.ceil(1.25 * kp) + 16.0 - margin
    return float(ok.mean()), float(np.mean(kp / np.maximum(k, 1)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "rank_mlp_default.json"))
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--tau", type=float, default=0.9)
    args = ap.parse_args()
    cfgs = qpinputs.rank_training_set()
    t0 = time.time()
    x_tr, k_tr = collect(cfgs[:56])
    x_va, k_va = collect(cfgs[56:])
    print(f"collected {len(k_tr)} training and {len(k_va)} validation boxes in {time.time() - t0:.1f} s", flush=True)
    t = np.log(np.maximum(k_tr, 1)).astype(np.float32)
    p = init_params(x_tr)
    t0 = time.time()
    p, h1 = B.mlp_train(p, x_tr, t, tau=args.tau, steps=args.steps, lr=3e-3)
    p, h2 = B.mlp_train(p, x_tr, t, tau=args.tau, steps=args.steps // 2, lr=5e-4)
    print(f"trained in {time.time() - t0:.1f} s: mean pinball loss {h1[0]:.4f} -> {h1[-1]:.4f} -> {h2[-1]:.4f}", flush=True)
    cov_tr, over_tr = coverage(p, x_tr, k_tr)
    cov_va, over_va = coverage(p, x_va, k_va)
    print(f"coverage train {cov_tr:.4f} (mean k^/k {over_tr:.3f}), validation {cov_va:.4f} (mean k^/k {over_va:.3f})")
    with open(args.out, "w") as f:
        json.dump({"params": [float(v) for v in p], "features": FEATURES, "tau": args.tau,
                   "train": {"boxes": int(len(k_tr)), "obstacles": 56, "coverage": cov_tr, "mean_over": over_tr,
                             "final_loss": float(h2[-1])},
                   "validation": {"boxes": int(len(k_va)), "obstacles": 8, "coverage": cov_va, "mean_over": over_va}},
                  f)
    print(f"wrote {args.out}")


if __name__ == "__main__":
    main()
