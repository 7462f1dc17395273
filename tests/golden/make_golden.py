"""Write the stored oracle fingerprints of the full-size workloads.

Calls only the FP64 CPU oracle and the seeded input generators.  For a workload
it stores, per DFC block, the iteration count, rank and final residuals of the
oracle, the products Z w for two seeded probe vectors w, Z at 512 seeded
positions, ||Z||_F, ||S||_F and the segmentation labels -- enough to check a
full-size GPU solve element by element where the oracle can compute it once.

    python tests/golden/make_golden.py 2 [3 ...]
    python tests/golden/make_golden.py 4b1      # block 1 of workload 4 only
    python tests/golden/make_golden.py 5g       # workload 5: the oracle gradient
    python tests/golden/make_golden.py 2l       # workload 2, footnote variant (local dictionaries)

Workload 4 is too large for the oracle's DFC run (40 blocks, n = 20000); its
fingerprint covers the first block, solved as one LRR problem with the whole M
as dictionary (Eq. 2), in the push-through form of the Z-step.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1304_5583_amd.datagen import make_config  # noqa: E402


def probes(n: int, seed: int = 4242):
    rng = np.random.default_rng(seed)
    W = rng.standard_normal((n, 2))
    idx = rng.integers(0, n, size=(512, 2))
    return W, idx


def block_fingerprint(cfg: int, block: int):
    p = make_config(cfg)
    cols = p.perm[p.offsets[block - 1]:p.offsets[block]]
    X = p.M[:, cols]
    t0 = time.time()
    r = oracle.lrr_alm(X, p.M, p.lam, oracle.ALMOptions(solve_form="pushthrough"))
    el = time.time() - t0
    rng = np.random.default_rng(4243)
    W = rng.standard_normal((X.shape[1], 2))
    idx = np.stack([rng.integers(0, p.n, 512), rng.integers(0, X.shape[1], 512)], axis=1)
    out = {
        "workload": p.name, "config": cfg, "block": block, "m": p.m, "n": p.n, "l": int(X.shape[1]),
        "lam": p.lam, "oracle_seconds": el, "iters": r.iters, "rank": r.rank, "res1": r.res1,
        "res2": r.res2, "Zw": (r.Z @ W).T.tolist(), "probe_idx": idx.tolist(),
        "Z_at": [float(r.Z[i, j]) for i, j in idx], "Z_fro": float(np.linalg.norm(r.Z)),
        "E_fro": float(np.linalg.norm(r.E)), "s_top": r.s[:8].tolist(),
    }
    path = os.path.join(HERE, f"workload{cfg}_block{block}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"workload {cfg} block {block}: {el:.1f}s iters={r.iters} rank={r.rank} -> {path}", flush=True)


def gradient_fingerprint(cfg: int):
    """Unrolled DFC-LRR (fixed iteration count) and the oracle's reverse sweep for
    L = ||W o |Z| ||_F^2: dL/dlambda, ||dL/dM||_F, dL/dM at 512 seeded positions
    and <dL/dM, D> for six seeded directions D with i.i.d. standard normal
    entries (the first two as drawn before, four more after them)."""
    from oracle import adjoint as adj
    p = make_config(cfg)
    W = p.extra["W"]
    opts = oracle.ALMOptions(fixed_iters=p.extra["fixed_iters"])
    t0 = time.time()
    tapes = adj.dfc_forward(p.M, p.lam, p.perm, p.offsets, opts)
    Z = adj.dfc_combine(tapes, p.perm)[0]
    L = float(np.sum((W * Z) ** 2))
    Mbar, lambar = adj.dfc_backward(tapes, p.perm, p.offsets, 2.0 * W ** 2 * Z)
    el = time.time() - t0
    rng = np.random.default_rng(4244)
    idx = np.stack([rng.integers(0, p.m, 512), rng.integers(0, p.n, 512)], axis=1)
    D = rng.standard_normal((2, p.m, p.n))
    D_more = rng.standard_normal((4, p.m, p.n))
    Wp, _ = probes(p.n)
    out = {
        "workload": p.name, "config": cfg, "m": p.m, "n": p.n, "t": p.t, "lam": p.lam,
        "fixed_iters": opts.fixed_iters, "oracle_seconds": el, "loss": L, "dlam": lambar,
        "dM_fro": float(np.linalg.norm(Mbar)), "probe_idx": idx.tolist(),
        "dM_at": [float(Mbar[i, j]) for i, j in idx],
        "dM_dir": [float(np.sum(Mbar * D[i])) for i in range(2)] +
                  [float(np.sum(Mbar * D_more[i])) for i in range(4)],
        "Zw": (Z @ Wp).T.tolist(), "Z_fro": float(np.linalg.norm(Z)),
    }
    path = os.path.join(HERE, f"workload{cfg}_gradient_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"workload {cfg} gradient: {el:.1f}s L={L:.6e} dlam={lambar:.6e} -> {path}", flush=True)


def local_fingerprint(cfg: int):
    """The footnote variant of Section 2.2 on a workload: every block its own
    dictionary, combine = best rank-k approximation of diag(J_1..J_t) with the
    default k = max_i rank(J_i)."""
    p = make_config(cfg)
    t0 = time.time()
    d = oracle.dfc_lrr_local(p.M, p.lam, p.perm, p.offsets)
    el = time.time() - t0
    W, idx = probes(p.n)
    out = {
        "workload": p.name, "variant": "local", "config": cfg, "m": p.m, "n": p.n, "t": p.t, "lam": p.lam,
        "oracle_seconds": el, "combine_rank": d.combine_rank,
        "iters": [b.iters for b in d.blocks], "rank": [b.rank for b in d.blocks],
        "Zw": (d.Z @ W).T.tolist(), "probe_idx": idx.tolist(),
        "Z_at": [float(d.Z[i, j]) for i, j in idx],
        "Z_fro": float(np.linalg.norm(d.Z)), "S_fro": float(np.linalg.norm(d.S)),
    }
    path = os.path.join(HERE, f"workload{cfg}_local_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"workload {cfg} local: {el:.1f}s iters={out['iters']} rank={out['rank']} k={d.combine_rank} -> {path}",
          flush=True)


def main(cfgs):
    for cfg in cfgs:
        if cfg == "5g":
            gradient_fingerprint(5)
            continue
        if isinstance(cfg, str) and cfg.endswith("l"):
            local_fingerprint(int(cfg[:-1]))
            continue
        if isinstance(cfg, str):
            c, b = cfg.split("b")
            block_fingerprint(int(c), int(b))
            continue
        p = make_config(cfg)
        t0 = time.time()
        d = oracle.dfc_lrr(p.M, p.lam, p.perm, p.offsets)
        el = time.time() - t0
        W, idx = probes(p.n)
        k = p.extra["k"]
        labels = oracle.segment(d.Z, k)
        out = {
            "workload": p.name, "config": cfg, "m": p.m, "n": p.n, "t": p.t, "lam": p.lam,
            "oracle_seconds": el,
            "iters": [b.iters for b in d.blocks], "rank": [b.rank for b in d.blocks],
            "res1": [b.res1 for b in d.blocks], "res2": [b.res2 for b in d.blocks],
            "Zw": (d.Z @ W).T.tolist(), "probe_idx": idx.tolist(),
            "Z_at": [float(d.Z[i, j]) for i, j in idx],
            "Z_fro": float(np.linalg.norm(d.Z)), "S_fro": float(np.linalg.norm(d.S)),
            # Section 4.1.2 clusters every point (no outlier removal)
            "labels": labels.tolist(),
            # segmentation with the rank cut above the reduced forms' error level
            "labels_rank_tol_1e-3": oracle.segment(d.Z, k, rank_tol=1e-3).tolist(),
            "accuracy": oracle.segmentation_accuracy(labels, np.where(p.outliers, -1, p.labels)),
            # ||S[:, j]|| / ||M[:, j]||, the quantity the outlier flags threshold
            "S_ratio": (np.linalg.norm(d.S, axis=0) / np.linalg.norm(p.M, axis=0)).tolist(),
        }
        path = os.path.join(HERE, f"workload{cfg}_oracle.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"workload {cfg}: {el:.1f}s iters={out['iters']} rank={out['rank']} -> {path}", flush=True)


if __name__ == "__main__":
    main([a if ("b" in a or "g" in a or "l" in a) else int(a) for a in sys.argv[1:]] or [2])
