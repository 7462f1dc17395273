"""Autotuner of the solver's launch schedule.

For a problem shape it times the schedule choices the library exposes -- the
Jacobi block width of the eigensolver (16 or 32 indices: the tile shape of its
pair and apply kernels), replaying each iteration's Z- and E-step launches from
a HIP graph or launching them one by one, the spacing of the host's
convergence checks, and full versus reduced coordinates -- and keeps the
fastest candidate that reproduces the default schedule's iterates (identical
per-block iteration counts, relative difference of Z at most 1e-8).  The
result is a table the C library reads (lrr_tune_load; solves with opts.tune =
1 use the entry for their shape):

    python -m paper_1304_5583_amd.autotune --workloads 2 3 4 [--out FILE]

Every timing runs the HIP library; nothing here computes the method.
"""
from __future__ import annotations

import argparse
import itertools
import os
import sys
import time

import numpy as np

from . import binding as B

HEADER = "# m n t maxl precision eig_block use_graph check_every coords\n"


def candidates(n: int, m: int):
    coords = (B.LRR_COORDS_FULL, B.LRR_COORDS_REDUCED) if n >= m else (B.LRR_COORDS_FULL,)
    for eb, g, ce, co in itertools.product((16, 32), (1, 0), (1, 4), coords):
        yield dict(eig_block=eb, use_graph=g, check_every=ce, coords=co)


def _solve(Mt, Zt, lam, perm, offsets, ctx, precision, sched):
    import torch
    o = B.lrr_opts_default(precision=precision, **sched)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info = B.dfc_lrr_solve(Mt, lam, perm, offsets, opts=o, ctx=ctx, want_S=False, Zt=Zt)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, info


def tune(Mt, lam, perm, offsets, precision: int = 0, reps: int = 2, ctx=None, log=None):
    """Returns (entry, rows): the table entry (a dict) and the timing of every
    candidate (seconds, or None when it did not reproduce the default's iterates)."""
    import torch
    n, m = Mt.shape
    ctx = ctx or B.get_context(Mt.device.index or 0)
    Zt = torch.empty((n, n), dtype=torch.float64, device=Mt.device)
    default = dict(eig_block=16, use_graph=1, check_every=1, coords=B.LRR_COORDS_AUTO)
    _solve(Mt, Zt, lam, perm, offsets, ctx, precision, default)
    _, ref_info = _solve(Mt, Zt, lam, perm, offsets, ctx, precision, default)
    Zref = Zt.clone()
    rows = []
    for sched in candidates(n, m):
        _solve(Mt, Zt, lam, perm, offsets, ctx, precision, sched)       # warm-up (workspace, graphs)
        ts = []
        for _ in range(reps):
            t, info = _solve(Mt, Zt, lam, perm, offsets, ctx, precision, sched)
            ts.append(t)
        diff = (torch.linalg.norm(Zt - Zref) / torch.linalg.norm(Zref)).item()
        same = np.array_equal(info.iters, ref_info.iters) and diff <= 1e-8
        rows.append((sched, min(ts) if same else None, diff))
        if log:
            log(f"  {sched} {min(ts) * 1e3:.1f} ms diff {diff:.1e}{'' if same else ' (rejected)'}")
    ok = [r for r in rows if r[1] is not None]
    best = min(ok, key=lambda r: r[1])[0]
    maxl = int(np.max(np.diff(offsets)))
    entry = dict(m=m, n=n, t=len(offsets) - 1, maxl=maxl, precision=precision, **best)
    del Zt, Zref
    return entry, rows


def write_table(path: str, entries):
    with open(path, "w") as f:
        f.write(HEADER)
        for e in entries:
            f.write(f"{e['m']} {e['n']} {e['t']} {e['maxl']} {e['precision']} {e['eig_block']} "
                    f"{e['use_graph']} {e['check_every']} {e['coords']}\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workloads", type=int, nargs="+", default=[2, 3, 4])
    ap.add_argument("--out", default=B.TUNE_TABLE)
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args(argv)
    import torch
    from .datagen import make_config
    entries = []
    for wl in args.workloads:
        p = make_config(wl)
        Mt = B.to_device_colmajor(p.M, "cuda:0")
        print(f"workload {wl} ({p.name})", flush=True)
        entry, _ = tune(Mt, p.lam, p.perm, p.offsets, reps=args.reps, log=lambda s: print(s, flush=True))
        print(f"  -> {entry}", flush=True)
        entries.append(entry)
        del Mt
        torch.cuda.empty_cache()
    write_table(args.out, entries)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
