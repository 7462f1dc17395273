"""Write the stored oracle fingerprints of the full-size workloads.

Calls only the FP64 CPU oracle and the seeded input generators.  For a workload
it stores, per DFC block, the iteration count, rank and final residuals of the
oracle, the products Z w for two seeded probe vectors w, Z at 512 seeded
positions, ||Z||_F, ||S||_F and the segmentation labels -- enough to check a
full-size GPU solve element by element where the oracle can compute it once.

    python tests/golden/make_golden.py 2 [3 ...]
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


def main(cfgs):
    for cfg in cfgs:
        p = make_config(cfg)
        t0 = time.time()
        d = oracle.dfc_lrr(p.M, p.lam, p.perm, p.offsets)
        el = time.time() - t0
        W, idx = probes(p.n)
        k = p.extra["k"]
        labels = oracle.segment(d.Z, k, p.outliers)
        out = {
            "workload": p.name, "config": cfg, "m": p.m, "n": p.n, "t": p.t, "lam": p.lam,
            "oracle_seconds": el,
            "iters": [b.iters for b in d.blocks], "rank": [b.rank for b in d.blocks],
            "res1": [b.res1 for b in d.blocks], "res2": [b.res2 for b in d.blocks],
            "Zw": (d.Z @ W).T.tolist(), "probe_idx": idx.tolist(),
            "Z_at": [float(d.Z[i, j]) for i, j in idx],
            "Z_fro": float(np.linalg.norm(d.Z)), "S_fro": float(np.linalg.norm(d.S)),
            "labels": labels.tolist(),
            "accuracy": oracle.segmentation_accuracy(labels, p.labels),
        }
        path = os.path.join(HERE, f"workload{cfg}_oracle.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"workload {cfg}: {el:.1f}s iters={out['iters']} rank={out['rank']} -> {path}", flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [2])
