#!/usr/bin/env python3
"""DFC-LRR benchmark on one MI355X.

A step is one complete ``dfc_lrr_solve`` (Algorithm 1: D-step gather,
factorisation of I + M M^T, all t blocks iterated to tolerance in batched
launches, column-projection combine).  The default workload is the one the
mixed-precision comparison is defined on: m = 512, n = 20000, t = 40 blocks of
500 (100 rank-20 subspaces, 10% replaced columns), timed in the FP64 plain form;
the BF16x3 and FP32 forms are timed the same way and reported with their error
against the FP64 form's Z.  The input is resident in HBM before every timed
region, and no per-kernel timing runs inside the headline region.

Per-kernel roofline figures come from a separate profiled region (one FP64
solve, every launch bracketed by HIP events on the solve's stream): for the
matrix products the algorithmic flops of each launch (2 M N K summed over the
blocks it covers, from the host's descriptors) against the FP64 matrix peak, for
the column kernels their algorithmic HBM bytes against 8 TB/s.

Prints one JSON line.  The FP64 CPU oracle is timed on a bounded sample of the
same workload (block 1, a few ALM iterations, scaled by the block-iterations of
the full solve) and, single-threaded, on block 1 of the n = 2000 workload.
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

METRIC = "DFC-LRR solves/sec + ALM iters/sec at stated err vs FP64 plain form, 1 GPU"
PEAK = {"mfma_f64": 78.6, "hbm": 8000.0, "alu_f64": 78.6}   # TFLOP/s, GB/s, TFLOP/s
HBM_KERNELS = ("k_estep", "k_update_Z", "k_form_QT", "k_form_Y", "k_zstep_fused")


def prof_table(B, ctx):
    import ctypes as C
    lib = B.load_library()
    lib.lrr_prof_count.argtypes = [C.c_void_p]
    lib.lrr_prof_count.restype = C.c_int
    lib.lrr_prof_entry.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                                   C.POINTER(C.c_longlong), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    rows = []
    for i in range(lib.lrr_prof_count(ctx.handle)):
        nm, ms, nl, fl, by = C.c_char_p(), C.c_double(), C.c_longlong(), C.c_double(), C.c_double()
        lib.lrr_prof_entry(ctx.handle, i, C.byref(nm), C.byref(ms), C.byref(nl), C.byref(fl), C.byref(by))
        rows.append(dict(name=nm.value.decode(), ms=ms.value, launches=nl.value, flops=fl.value,
                         bytes=by.value))
    return sorted(rows, key=lambda r: -r["ms"])


def prof_enable(B, ctx, on, only=None):
    """Per-kernel HIP-event timing on the solve's stream (every launch, or only
    the kernels whose name starts with `only`).  Enabling clears the table."""
    import ctypes as C
    lib = B.load_library()
    lib.lrr_prof_enable.argtypes = [C.c_void_p, C.c_int]
    lib.lrr_prof_enable.restype = C.c_int
    lib.lrr_prof_filter.argtypes = [C.c_void_p, C.c_char_p]
    lib.lrr_prof_filter.restype = C.c_int
    lib.lrr_prof_filter(ctx.handle, only.encode() if only else None)
    lib.lrr_prof_enable(ctx.handle, int(on))


def roofline_of(row, traffic=None):
    """Roofline entry of one kernel from its event-timed launches: matrix
    products by their algorithmic flops against the FP64 matrix peak, column
    kernels by their algorithmic HBM bytes against 8 TB/s."""
    avg_ms = row["ms"] / max(row["launches"], 1)
    base = {"kernel": row["name"], "launches": row["launches"], "avg_launch_us": round(avg_ms * 1e3, 2)}
    if row["flops"] > 0:
        per = row["flops"] / row["launches"]
        ach = per / (avg_ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK["mfma_f64"], "unit": "TFLOP/s",
                "frac": round(ach / PEAK["mfma_f64"], 4), "traffic": traffic,
                "algorithmic_per_launch": per, **base}
    if row["bytes"] > 0:
        per = row["bytes"] / row["launches"]
        ach = per / (avg_ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK["hbm"], "unit": "GB/s",
                "frac": round(ach / PEAK["hbm"], 4), "traffic": traffic,
                "algorithmic_per_launch": per, **base}
    return None


def lib_digest(B):
    h = hashlib.sha256()
    with open(B.LIB_PATH, "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(path, digest):
    """HBM bytes per dispatch from counter runs of this very library build
    (a JSON map kernel -> bytes, with the library digest it was taken on)."""
    if not path or not os.path.exists(path):
        return {}
    tr = json.load(open(path))
    if tr.get("_lib") != digest:
        print(f"bench: counter file {path} is from another library build; traffic not reported",
              file=sys.stderr)
        return {}
    return tr


def lib_kernel_name(rocprof_name):
    """The library's timing-table name of a kernel from its rocprof name
    ("void lrr::(anonymous namespace)::k_dgemm<64, false, false, false>(...)"
    -> "k_dgemm<false, false>"); None for kernels outside the roofline set."""
    import re
    n = re.sub(r"^void ", "", rocprof_name).replace("(anonymous namespace)::", "")
    n = re.sub(r"\(.*$", "", n)
    n = n.split("::")[-1]
    m = re.match(r"k_dgemm<(\d+), (true|false), (true|false), (true|false)>", n)
    if m:
        return "k_dgemm_sym" if m.group(4) == "true" else f"k_dgemm<{m.group(2)}, {m.group(3)}>"
    base = re.sub(r"<.*$", "", n)
    base = {"k_update_Z_w": "k_update_Z", "k_estep_w": "k_estep", "k_form_Y_w": "k_form_Y"}.get(base, base)
    return base if base in HBM_KERNELS or base.startswith("k_") else None


def traffic_from_pmc(fetch_csv, write_csv, out_path, digest):
    """HBM bytes per dispatch from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE; KiB per dispatch, summed over the rows of a dispatch), each
    scaled by what the same counter reads for the 512 MiB device copy that
    --calib-copy adds (the copy's last dispatch), averaged per kernel name."""
    import csv
    from collections import defaultdict

    def per_dispatch(path, counter):
        vals, names = defaultdict(float), {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            vals[d] += float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
        return vals, names

    fv, fn = per_dispatch(fetch_csv, "FETCH_SIZE")
    wv, wn = per_dispatch(write_csv, "WRITE_SIZE")
    copy_kib = 512 * 1024.0
    fcopy = [fv[d] for d in fv if "copyBuffer" in fn[d] and fv[d] > 0.25 * copy_kib]
    wcopy = [wv[d] for d in wv if "copyBuffer" in wn[d] and wv[d] > 0.25 * copy_kib]
    if not fcopy or not wcopy:
        raise SystemExit("no 512 MiB calibration copy in the counter runs (run bench.py with --calib-copy)")
    fscale, wscale = copy_kib / fcopy[-1], copy_kib / wcopy[-1]
    acc = defaultdict(lambda: [0.0, 0.0, 0, 0])
    for d, v in fv.items():
        k = lib_kernel_name(fn[d])
        if k:
            acc[k][0] += v * fscale * 1024.0
            acc[k][2] += 1
    for d, v in wv.items():
        k = lib_kernel_name(wn[d])
        if k:
            acc[k][1] += v * wscale * 1024.0
            acc[k][3] += 1
    out = {"_lib": digest, "_scale": {"fetch": fscale, "write": wscale},
           "_source": "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, one FP64 solve each, scaled by a 512 MiB copy"}
    for k, (fb, wb, nf, nw) in sorted(acc.items()):
        if nf and nw:
            out[k] = round(fb / nf + wb / nw)
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"bench: wrote {out_path} ({len(out) - 3} kernels, scale fetch {fscale:.3f} write {wscale:.3f})",
          file=sys.stderr)


def workload_name(p, precision):
    return p.name.rsplit("-", 1)[0] + "-" + precision


def oracle_error(p, Zt):
    """Relative error of the GPU's Z against the stored FP64 oracle fingerprint:
    the probes Z w of the whole Z (workloads with a DFC fingerprint), or of the
    first block's columns (workload 4, whose fingerprint is block 1 solved as
    one LRR problem; the combine leaves block 1's columns as its J)."""
    import numpy as np
    cfg = p.extra.get("config")
    g4 = os.path.join(ROOT, "tests", "golden", "workload4_block1_oracle.json")
    gd = os.path.join(ROOT, "tests", "golden", f"workload{cfg}_oracle.json")
    if p.n == 20000 and os.path.exists(g4):
        g = json.load(open(g4))
        cols = p.perm[p.offsets[0]:p.offsets[1]]
        Zb = Zt.index_select(0, __import__("torch").as_tensor(cols, device=Zt.device).long()).cpu().numpy().T
        rng = np.random.default_rng(4243)
        W = rng.standard_normal((len(cols), 2))
        Zw = (Zb @ W).T
        ref = np.array(g["Zw"])
        return {"err_vs_oracle": float(np.linalg.norm(Zw - ref) / np.linalg.norm(ref)),
                "oracle_scope": "block 1 (Z w probes)", "oracle_iters_block1": g["iters"]}
    if cfg in (2, 3) and os.path.exists(gd):
        g = json.load(open(gd))
        Z = Zt.cpu().numpy().T
        rng = np.random.default_rng(4242)
        W = rng.standard_normal((p.n, 2))
        Zw = (Z @ W).T
        ref = np.array(g["Zw"])
        return {"err_vs_oracle": float(np.linalg.norm(Zw - ref) / np.linalg.norm(ref)),
                "oracle_scope": "all blocks (Z w probes)", "oracle_iters_per_block": g["iters"]}
    return {"err_vs_oracle": None}


def cpu_baseline(p, total_block_iters, target_s, single_thread_s):
    """The FP64 oracle on bounded samples: block 1 of the benchmark workload for
    as many ALM iterations as fit in about target_s seconds (push-through Z-step
    when n >> m, as the oracle's workload-4 fingerprint), scaled to solves/s by
    the block-iterations of the full solve; and block 1 of the n = 2000 workload
    on one thread (the paper's simulations ran on a single core)."""
    from threadpoolctl import threadpool_limits
    import oracle
    from paper_1304_5583_amd.datagen import make_config
    cores = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        cores = min(cores, int(env))
    form = "pushthrough" if p.n >= 4 * p.m else "literal"

    def sample(q, limit, seconds):
        X = q.M[:, q.perm[q.offsets[0]:q.offsets[1]]]
        with threadpool_limits(limits=limit):
            t0 = time.perf_counter()
            oracle.lrr_alm(X, q.M, q.lam, oracle.ALMOptions(fixed_iters=1, solve_form=form))
            per_it = time.perf_counter() - t0
            n_it = int(max(2, min(400, seconds / max(per_it, 1e-6))))
            t0 = time.perf_counter()
            oracle.lrr_alm(X, q.M, q.lam, oracle.ALMOptions(fixed_iters=n_it, solve_form=form))
            el = time.perf_counter() - t0
        return n_it, el, X.shape[1]

    n_it, el, l = sample(p, cores, target_s)
    rate = n_it / el
    out = {"value": rate / total_block_iters, "unit": "solves/s", "cores": cores, "kind": "oracle",
           "sample": f"{n_it} ALM iterations of block 1 (m={p.m}, n={p.n}, l={l}, {form} Z-step) in "
                     f"{el:.1f}s = {rate:.4f} block-iterations/s, divided by the {total_block_iters} "
                     f"block-iterations of the GPU's full solve (extrapolated)",
           "block_iters_per_s": rate}
    if single_thread_s > 0:
        q = make_config(2)
        form = "literal"
        n1, e1, l1 = sample(q, 1, single_thread_s)
        out["single_thread_workload2"] = {
            "block_iters_per_s": n1 / e1, "cores": 1,
            "sample": f"{n1} ALM iterations of block 1 of {q.name} (l={l1}, literal Z-step) in {e1:.1f}s"}
    return out


def timed_solves(B, torch, p, Mt, Zt, ctx, opts, steps):
    """`steps` solves after one untimed one, no per-kernel timing; returns
    seconds per solve, the last info and the totals of batched and per-block
    iterations."""
    B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=opts, ctx=ctx, want_S=False, Zt=Zt)
    torch.cuda.synchronize()
    bi = ki = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        _, _, info = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=opts, ctx=ctx, want_S=False, Zt=Zt)
        bi += info.batch_iters
        ki += int(info.iters.sum())
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, info, bi, ki


def device_loop(B, torch, p, Mt, Zref, ctx, schedule, steps):
    """The same FP64 solve with every J-step decision on the device and one
    graph per ALM iteration (use_graph = 2: one host synchronisation per
    check_every iterations): solves/s and bitwise equality with the
    host-driven solve's Z."""
    sched = schedule if isinstance(schedule, dict) else {}
    o = B.lrr_opts_default(use_graph=2, eig_block=sched.get("eig_block", 0),
                           check_every=sched.get("check_every", 0), coords=sched.get("coords", 0))
    Zt = torch.empty_like(Zref)
    sec, info, bi, _ = timed_solves(B, torch, p, Mt, Zt, ctx, o, steps)
    out = {"use_graph": 2, "check_every": int(o.check_every) or None, "steps": steps, "solves_per_s": 1.0 / sec,
           "ms_per_solve": 1e3 * sec, "host_syncs": "one per check_every iterations",
           "bitwise_equal_to_host_driven": bool(torch.equal(Zt, Zref))}
    print(f"bench: device-driven J-step {p.name}: {1e3 * sec:.1f} ms/solve "
          f"bitwise={out['bitwise_equal_to_host_driven']}", file=sys.stderr, flush=True)
    del Zt
    return out


def precision_forms(B, torch, p, Mt, Z64t, ctx, opts_of, steps, sec64):
    """The reduced-precision forms on the benchmark workload, timed like the
    headline: solves/s, speed-up over the FP64 form, relative Frobenius error of
    Z against the FP64 form's Z, iteration counts."""
    out = {}
    Zt = torch.empty_like(Z64t)
    for name, prec in (("mixed_bf16x3", B.LRR_MIXED_BF16), ("fp32", B.LRR_FP32)):
        sec, info, bi, ki = timed_solves(B, torch, p, Mt, Zt, ctx, opts_of(prec), steps)
        err = (torch.linalg.norm(Zt - Z64t) / torch.linalg.norm(Z64t)).item()
        out[name] = {"solves_per_s": 1.0 / sec, "ms_per_solve": 1e3 * sec, "steps": steps,
                     "speedup_vs_fp64": sec64 / sec, "err_vs_fp64_plain": err,
                     "alm_iters_per_s": bi / (sec * steps), "alm_block_iters_per_s": ki / (sec * steps),
                     "iters_range": [int(info.iters.min()), int(info.iters.max())]}
        print(f"bench: {name}: {1e3 * sec:.1f} ms/solve err_vs_fp64={err:.2e}", file=sys.stderr, flush=True)
    del Zt
    return out


def profiled_solve(B, torch, p, Mt, Zt, ctx, opts):
    """One FP64 solve with every launch bracketed by HIP events: the per-kernel
    table and the roofline entries of the matrix products and column kernels."""
    prof_enable(B, ctx, 1)
    B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=opts, ctx=ctx, want_S=False, Zt=Zt)
    torch.cuda.synchronize()
    rows = prof_table(B, ctx)
    prof_enable(B, ctx, 0)
    total = sum(r["ms"] for r in rows)
    for r in rows[:16]:
        rf = roofline_of(r)
        rate = f"{rf['achieved']} {rf['unit']} ({rf['frac']:.3f})" if rf else "-"
        print(f"bench:   {r['name']:30s} {r['ms']:9.2f} ms {r['launches']:6d} launches "
              f"avg {r['ms'] / max(r['launches'], 1) * 1e3:8.1f} us  {rate}", file=sys.stderr)
    return rows, total


def _accuracy(pred, truth):
    """Section 4.1.2 segmentation accuracy: each cluster takes the majority true
    label of its points; mean over classes of the fraction labelled correctly
    (points labelled -1 on either side are skipped)."""
    import numpy as np
    keep = (pred >= 0) & (truth >= 0)
    pred, truth = pred[keep], truth[keep]
    vote = {c: np.bincount(truth[pred == c]).argmax() for c in np.unique(pred)}
    mapped = np.array([vote[c] for c in pred])
    return float(np.mean([np.mean(mapped[truth == g] == g) for g in np.unique(truth)]))


def segmentation(B, torch, p, Zt, ctx, golden=None, reps=3, St=None, Mt=None, delta=0.5):
    """Section 4.1.2 labels from the solve's Z on the GPU (lrr_segment, every
    point clustered, range sketch with the largest block width as rank bound):
    time per call, the embedding's products with the affinity, the accuracy over
    the generator's clean points and, with a stored oracle record, label
    equality.  With the solve's S: the outlier columns the method flags
    (||S_j|| > delta ||M_j||, lrr_outlier_flags) against the generator's."""
    import numpy as np
    k = p.extra["k"]
    bound = int(np.diff(p.offsets).max())
    lab, info = B.lrr_segment(Zt, k, None, rank_bound=bound, ctx=ctx)   # sizes the workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lab, info = B.lrr_segment(Zt, k, None, rank_bound=bound, ctx=ctx)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    got = lab.cpu().numpy()
    out = {"ms": ms, "k": k, "n_keep": info["n_keep"], "rank": info["rank"], "sketch": info["sketch"],
           "embed_products": info["embed_iters"], "embed_resid": info["embed_resid"],
           "theta_k": info["theta_k"], "theta_k1": info["theta_k1"], "kmeans_iters": info["kmeans_iters"],
           "exclude": "none (every point clustered)",
           "accuracy_vs_truth_clean_points": _accuracy(got, np.where(p.outliers, -1, p.labels))}
    if golden is not None and "labels" in golden and "S_ratio" in golden:
        out["labels_equal_oracle"] = got.tolist() == golden["labels"]
    if St is not None:
        flags, cnt = B.lrr_outlier_flags(Mt, St, delta, ctx=ctx)
        f = flags.cpu().numpy()
        out["outlier_flags_from_S"] = {"delta": delta, "flagged": cnt, "generator_outliers": int(p.outliers.sum()),
                                       "flagged_and_generator": int((f & p.outliers).sum())}
    print(f"bench: segmentation {p.name}: {ms:.1f} ms products {info['embed_iters']}", file=sys.stderr, flush=True)
    return out


def other_workload(B, torch, ctx, cfg, steps, tuned):
    """FP64 solves/s and the error against the stored oracle fingerprint on
    another workload (context for the headline)."""
    from paper_1304_5583_amd.datagen import make_config
    p = make_config(cfg)
    dev = torch.device("cuda:0")
    Mt = B.to_device_colmajor(p.M, dev)
    Zt = torch.empty((p.n, p.n), dtype=torch.float64, device=dev)
    opts = B.lrr_opts_default(tune=1) if tuned else B.lrr_opts_default()
    sec, info, bi, ki = timed_solves(B, torch, p, Mt, Zt, ctx, opts, steps)
    out = {"workload": workload_name(p, "fp64"), "m": p.m, "n": p.n, "t": p.t, "steps": steps,
           "solves_per_s": 1.0 / sec, "ms_per_solve": 1e3 * sec, "alm_iters_per_s": bi / (sec * steps),
           "alm_block_iters_per_s": ki / (sec * steps), "iters_per_block": info.iters.tolist()}
    out.update(oracle_error(p, Zt))
    print(f"bench: {p.name}: {1e3 * sec:.1f} ms/solve err_vs_oracle={out['err_vs_oracle']}", file=sys.stderr,
          flush=True)
    sched = tuned_schedule(B.TUNE_TABLE, p) if tuned else None
    out["device_loop"] = device_loop(B, torch, p, Mt, Zt, ctx, sched, steps)
    gpath = os.path.join(ROOT, "tests", "golden", f"workload{cfg}_oracle.json")
    golden = json.load(open(gpath)) if os.path.exists(gpath) else None
    _, St, _ = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=opts, ctx=ctx, want_S=True, Zt=Zt)
    out["segmentation"] = segmentation(B, torch, p, Zt, ctx, golden, reps=1, St=St, Mt=Mt)
    del St
    if cfg == 2:
        out["local_variant"] = local_variant(B, torch, p, Mt, ctx)
        out["slr_graph"] = slr_graph(B, torch, p, Mt, Zt, ctx)
    del Zt, Mt
    torch.cuda.empty_cache()
    return out


def local_variant(B, torch, p, Mt, ctx, reps=3):
    """The footnote variant of Section 2.2 on the same workload (every block its
    own dictionary, truncated-SVD combine): solves/s and the error against the
    stored oracle fingerprint."""
    import numpy as np
    Zt = torch.empty((p.n, p.n), dtype=torch.float64, device=Mt.device)
    B.dfc_lrr_solve_local(Mt, p.lam, p.perm, p.offsets, ctx=ctx, want_S=False, Zt=Zt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, _, info = B.dfc_lrr_solve_local(Mt, p.lam, p.perm, p.offsets, ctx=ctx, want_S=False, Zt=Zt)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    out = {"solves_per_s": 1.0 / el, "ms_per_solve": 1e3 * el, "iters_per_block": info.iters.tolist(),
           "rank_per_block": info.rank.tolist(), "combine_rank": info.combine_rank}
    gpath = os.path.join(ROOT, "tests", "golden", "workload2_local_oracle.json")
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        rng = np.random.default_rng(4242)
        W = rng.standard_normal((p.n, 2))
        Zw = (Zt.cpu().numpy().T @ W).T
        out["err_vs_oracle"] = float(np.linalg.norm(Zw - np.array(g["Zw"])) / np.linalg.norm(np.array(g["Zw"])))
    print(f"bench: local variant {p.name}: {1e3 * el:.1f} ms/solve", file=sys.stderr, flush=True)
    del Zt
    return out


def slr_graph(B, torch, p, Mt, Zt, ctx, nk=500, alpha=0.05, reps=3):
    """Section 4.2.2 SLR-graph on the solve's Z with the paper's settings
    (n_k = 500 neighbours, alpha = 0.05): time per call and Lasso statistics."""
    B.lrr_slr_graph(Mt, Zt, nk, alpha, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        nbr, w, obj, info = B.lrr_slr_graph(Mt, Zt, nk, alpha, ctx=ctx)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    out = {"ms": ms, "nk": nk, "alpha": alpha, "max_steps": info["max_steps"], "max_kkt": info["max_kkt"],
           "not_converged": info["not_converged"], "large_support": info["large_support"],
           "max_support": info["max_support"], "edges_per_sample": float((w > 0).sum().item()) / p.n}
    print(f"bench: SLR-graph {p.name}: {ms:.1f} ms", file=sys.stderr, flush=True)
    return out


def workload5_adjoint(B, torch, ctx):
    """Workload 5: FP32 forward of 200 unrolled iterations with checkpoints every
    20 and the reverse sweep for L = ||W o |Z| ||_F^2; times both and compares
    dL/dlambda with the stored oracle gradient."""
    from paper_1304_5583_amd.datagen import make_config
    p = make_config(5)
    dev = torch.device("cuda:0")
    Mt = B.to_device_colmajor(p.M, dev)
    Wt = torch.from_numpy(p.extra["W"].T.copy()).to(dev)
    opts = B.lrr_opts_default(precision=B.LRR_FP32, fixed_iters=p.extra["fixed_iters"],
                              checkpoint_every=p.extra["checkpoint_every"], save_for_backward=1)
    res = {}
    for rep in range(2):    # the first pass allocates the record
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Zt, _, _ = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=opts, ctx=ctx, want_S=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dlam, dMt = B.dfc_lrr_backward(2.0 * Wt ** 2 * Zt, ctx=ctx, m=p.m)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res = {"forward_ms": 1e3 * (t1 - t0), "backward_ms": 1e3 * (t2 - t1), "dlambda": dlam}
    gpath = os.path.join(ROOT, "tests", "golden", "workload5_gradient_oracle.json")
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        res["dlambda_oracle"] = g["dlam"]
        res["dlambda_rel_err"] = abs(dlam - g["dlam"]) / abs(g["dlam"])
    res.update({"workload": p.name, "precision": "fp32 forward, fp64 reverse", "iters": p.extra["fixed_iters"],
                "checkpoint_every": p.extra["checkpoint_every"]})
    print(f"bench: workload 5 adjoint: forward {res['forward_ms']:.1f} ms backward {res['backward_ms']:.1f} ms",
          file=sys.stderr, flush=True)
    del Mt, Wt
    torch.cuda.empty_cache()
    return res


def tuned_schedule(path, p, precision=0):
    """The schedule-table entry a tuned solve of workload p uses (None: no entry)."""
    maxl = int(max(p.offsets[i + 1] - p.offsets[i] for i in range(p.t)))
    for line in open(path):
        f = line.split("#")[0].split()
        if len(f) == 9 and [int(x) for x in f[:5]] == [p.m, p.n, p.t, maxl, precision]:
            return dict(zip(("eig_block", "use_graph", "check_every", "coords"), (int(x) for x in f[5:])))
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=4, help="workload number (default 4)")
    ap.add_argument("--form-steps", type=int, default=0,
                    help="timed solves per reduced-precision form (default: steps, at most 10)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-single-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="ignore the autotuned schedule table")
    ap.add_argument("--no-forms", action="store_true", help="skip the reduced-precision forms")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip segmentation, the other workloads and the workload-5 adjoint")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_counters.json"),
                    help="HBM bytes per dispatch from counter runs of this library build")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 512 MiB device copy (reference for HBM counters)")
    ap.add_argument("--traffic-from-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write --traffic from two rocprofv3 counter-collection files and exit")
    ap.add_argument("--slr-only", action="store_true",
                    help="after the warmup solves, time only the SLR-graph on the solve's Z (one JSON line of "
                         "its statistics; for profiling that step)")
    args = ap.parse_args()
    if args.traffic_from_pmc:
        from paper_1304_5583_amd import binding as B
        traffic_from_pmc(args.traffic_from_pmc[0], args.traffic_from_pmc[1], args.traffic, lib_digest(B))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the DFC blocks would "
              f"shard across GPUs with no communication until the combine, which this build does "
              f"not implement.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1304_5583_amd import binding as B
    from paper_1304_5583_amd.datagen import make_config

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    p = make_config(args.workload)
    print(f"bench: workload {p.name} m={p.m} n={p.n} t={p.t} lam={p.lam}", file=sys.stderr, flush=True)
    Mt = B.to_device_colmajor(p.M, dev)
    Zt = torch.empty((p.n, p.n), dtype=torch.float64, device=dev)
    ctx = B.get_context(0)
    tuned = not args.no_tune and os.path.exists(B.TUNE_TABLE)
    if tuned:
        B.lrr_tune_load(B.TUNE_TABLE, ctx=ctx)

    def opts_of(prec):
        return B.lrr_opts_default(precision=prec, tune=1) if tuned else B.lrr_opts_default(precision=prec)

    schedule = (tuned_schedule(B.TUNE_TABLE, p) if tuned else None) or "default"
    print(f"bench: schedule {schedule}", file=sys.stderr, flush=True)
    opts = opts_of(B.LRR_FP64)

    for i in range(args.warmup):
        _, _, info = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=opts, ctx=ctx, want_S=False, Zt=Zt)
        torch.cuda.synchronize()
        print(f"bench: warmup {i} batch_iters={info.batch_iters}", file=sys.stderr, flush=True)
    if args.slr_only:
        if args.warmup == 0:
            B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=opts, ctx=ctx, want_S=False, Zt=Zt)
        out = slr_graph(B, torch, p, Mt, Zt, ctx, reps=1)
        out["workload"] = workload_name(p, "fp64")
        print(json.dumps(out), flush=True)
        return
    # headline region: the FP64 plain form, no per-kernel timing
    batch_iters = block_iters = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, _, info = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=opts, ctx=ctx, want_S=False, Zt=Zt)
        batch_iters += info.batch_iters
        block_iters += int(info.iters.sum())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sec64 = elapsed / args.steps
    print(f"bench: {args.steps} FP64 solves in {elapsed:.3f}s", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload_name(p, "fp64"), "m": p.m, "n": p.n, "t": p.t, "lambda": p.lam,
                   "tol": p.tol, "precision": "fp64", "mu0": opts.mu0, "rho": opts.rho, "mu_max": opts.mu_max,
                   "schedule": schedule},
        "alm_iters_per_s": batch_iters / elapsed,
        "alm_block_iters_per_s": block_iters / elapsed,
        "iters_per_block_range": [int(info.iters.min()), int(info.iters.max())],
        "rank_per_block_range": [int(info.rank.min()), int(info.rank.max())],
        "err_vs_fp64_plain": 0.0,
    }
    line.update(oracle_error(p, Zt))
    if not args.no_extras:
        line["device_loop"] = device_loop(B, torch, p, Mt, Zt, ctx, schedule, min(args.steps, 5))
    if not args.no_forms:
        fs = args.form_steps or min(args.steps, 10)
        line["forms"] = precision_forms(B, torch, p, Mt, Zt, ctx, opts_of, fs, sec64)

    # profiled region: every launch of one FP64 solve between HIP events
    rows, total = profiled_solve(B, torch, p, Mt, Zt, ctx, opts)
    digest = lib_digest(B)
    traffic = load_traffic(args.traffic, digest)
    entries = [e for e in (roofline_of(r, traffic.get(r["name"])) for r in rows) if e is not None]
    mfma = [e for e in entries if e["bound"] == "mfma"]
    hbm = [e for e in entries if e["bound"] == "hbm" and e["kernel"] in HBM_KERNELS]
    dominant = max(mfma, key=lambda e: e["avg_launch_us"] * e["launches"]) if mfma else entries[0]
    line["roofline"] = dominant
    line["roofline_hbm"] = hbm
    line["roofline_mfma_all"] = mfma
    line["kernels_profiled_solve"] = [{"name": r["name"], "ms": round(r["ms"], 3), "launches": r["launches"],
                                       "share": round(r["ms"] / total, 4)} for r in rows[:12]]
    line["lib"] = digest
    if args.calib_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)   # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("bench: calibration copy 512 MiB x 3 done", file=sys.stderr, flush=True)
        del src, dst

    if not args.no_extras:
        golden = None
        gpath = os.path.join(ROOT, "tests", "golden", f"workload{args.workload}_oracle.json")
        if os.path.exists(gpath):
            golden = json.load(open(gpath))
        _, St, _ = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=opts, ctx=ctx, want_S=True, Zt=Zt)
        line["segmentation"] = segmentation(B, torch, p, Zt, ctx, golden, reps=1 if p.n > 8192 else 3,
                                            St=St, Mt=Mt)
        del St
        line["slr_graph"] = slr_graph(B, torch, p, Mt, Zt, ctx, reps=1 if p.n > 8192 else 3)
        del Zt, Mt
        torch.cuda.empty_cache()
        line["other_workloads"] = [other_workload(B, torch, ctx, c, 5 if c == 2 else 3, tuned)
                                   for c in (2, 3) if c != args.workload]
        line["workload5_adjoint"] = workload5_adjoint(B, torch, ctx)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, int(info.iters.sum()), args.cpu_seconds, args.cpu_single_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
