#!/usr/bin/env python3
"""Benchmark of the Kronecker-product SVD hot path on one MI355X.

Workload (the n = 512 configuration): a rotated Gaussian PSF (sigma = (2, 1),
30 degrees) on the full 1023 x 1023 offset grid of a 512 x 512 image, zero
boundary conditions, so R(A) is 262144 x 262144 (never stored). One step is the
rank-20 KP-SVD of R(A) both ways the paper gives, in single precision:
  * EGKB (Algorithm 1), k = 20 enlarged to k_p = 40, full reorthogonalization;
  * RSVD (Algorithm 2), k = 20, oversampling 10, 2 power iterations;
each including the small FP64 SVD and the Kronecker factors. The PSF, start
vector and sketch are already on the device (Philox streams); the timed region
moves no input over PCIe.

value = algorithmic flops of the step (the paper's dense cost model:
4 N^2 k_p for EGKB, (4q + 4) N^2 k_p for RSVD, N = n^2) / wall time.
The roofline object is the dominant kernel, the generated-tile block product
(FP32 MFMA), timed with hipEvents around its launches on the call's stream.
The CPU baseline times the oracle's dense product of R(A) on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_FP32_PEAK_TFLOPS = 157.3     # MI355X dense FP32 matrix peak

# HBM bytes per launch of the FP32 block kernel (R X, 30 columns, n = 512) from
# rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a plain copy of known size
# (profiles/rmat_products_n512_hbm_counters.md), valid while the kernel source
# is the one the counters were taken on.
BLOCK_TRAFFIC_BYTES = 1.150e9
BLOCK_TRAFFIC_SRC_SHA1 = "df16919a8da03f62f9cb73e4d69c20d8bed8e3a8"
BLOCK16_TRAFFIC_BYTES = 2.10e8
# template arguments <TJ, JB, CB> of the FP32 block kernel per autotuner variant
BLOCK_VARIANT_TEMPLATE = {0: "16,1,2,false,64", 1: "16,2,2,false,64", 2: "8,1,2,false,64",
                          3: "8,1,1,false,64", 4: "16,1,2,false,128", 5: "16,2,2,false,128",
                          6: "8,1,2,false,128", 7: "8,1,1,false,128", 8: "16,1,2,false,192",
                          9: "16,2,2,false,192", 10: "8,1,2,false,192", 11: "8,1,1,false,192",
                          12: "16,1,2,false,176", 13: "16,2,2,false,176", 14: "8,1,2,false,176",
                          15: "8,1,1,false,176"}
BLOCK16_VARIANT_TEMPLATE = {0: "32,4,2", 1: "16,4,2", 2: "32,2,2", 3: "16,2,2", 4: "16,1,2",
                            5: "64,4,2", 6: "64,8,2"}
BLOCK16_TRAFFIC_SRC_SHA1 = "5a1fa497d43ed0c66b378fccc7483a2fd36397ef"


def counted_traffic(src, sha, value):
    """The counter-derived traffic, or None once the kernel source changed."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "paper_2410_00233_amd", "csrc", src), "rb") as f:
            return value if hashlib.sha1(f.read()).hexdigest() == sha else None
    except OSError:
        return None
MFMA_BF16_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 matrix peak
HBM_PEAK_GBS = 8000.0


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(n, ncols, target_s):
    """Oracle dense product R X on the first rows of R (the oracle as it stands:
    generated row blocks of R(A) times X with NumPy/BLAS, FP64)."""
    import numpy as np

    import workloads as wl
    from oracle import operator as op
    P, cu, cv = wl.gaussian_psf(n)
    N = n * n
    X = wl.gaussian_block(N, ncols, seed=wl.SEED_START + 7)
    cols = np.arange(N)
    chunk = 256
    rows_done = 0
    t0 = time.perf_counter()
    while True:
        rows = np.arange(rows_done, rows_done + chunk)
        _ = op.rmat_entries(P, cu, cv, n, rows, cols) @ X
        rows_done += chunk
        el = time.perf_counter() - t0
        if el >= target_s or rows_done >= N:
            break
    flops = 2.0 * rows_done * N * ncols
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    return dict(value=flops / el / 1e12, unit="TFLOP/s", cores=int(cores), kind="oracle",
                sample=f"dense R(A) X in FP64, first {rows_done} of {N} rows, {ncols} columns, "
                       f"n={n} rotated Gaussian; {el:.1f} s")


def bench_batched(ctx, count):
    """Mixed batch: `count` RSVD KP-SVDs (FP32, q = 2, p = 10, rank 10..30) of
    n in {128, 192, 256, 384, 512} with Gaussian / motion / disk PSFs, through
    kp_svd_batched, against the same problems as single calls one after another."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_2410_00233_amd import api, flops
    mix = wl.batched_mix(count)
    probs = []
    for d in mix:
        blur = api.Blur(d["P"], d["cu"], d["cv"], d["n"], on_device=True)
        o = api.Context.rsvd_opts(d["k"], d["p"], 2, prec="f32", seed=d["seed"])
        probs.append((blur, "rsvd", o, d["k"]))
    fl = sum(flops.rsvd(d["n"], d["k"], d["p"], 2) for d in mix)
    # workers warm and every image size tuned before the timed run (the one-by-one
    # run below comes after it and so finds everything tuned too)
    first = {}
    for pr, d in zip(probs, mix):
        first.setdefault(d["n"], pr)
    ctx.kp_svd_batched(list(first.values()))
    torch.cuda.synchronize()
    log("batched: timed run")
    t0 = time.perf_counter()
    facs, status = ctx.kp_svd_batched(probs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batched: {1e3 * t_batch:.0f} ms; the same problems one by one")
    t0 = time.perf_counter()
    solo = []
    for (blur, _, o, kc) in probs:
        solo.append(ctx.kp_svd_rsvd(blur, o.k, o.p, o.q, prec="f32", seed=o.seed))
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    same = all(np.array_equal(f.sigma[:f.k], g.sigma[:g.k]) for f, g in zip(facs, solo))
    sizes = [d["n"] for d in mix]
    return {
        "workload": f"{count} RSVD KP-SVDs (FP32, p=10, q=2, rank 10-30), n in "
                    "{128,192,256,384,512}, Gaussian/motion/disk PSFs, 4 worker streams",
        "problems": count, "n_hist": {str(v): sizes.count(v) for v in sorted(set(sizes))},
        "flops": fl, "batched_ms": round(1e3 * t_batch, 2), "solo_sum_ms": round(1e3 * t_solo, 2),
        "batched_tflops": round(fl / t_batch / 1e12, 3), "solo_tflops": round(fl / t_solo / 1e12, 3),
        "speedup_vs_solo": round(t_solo / t_batch, 3),
        "sigma_equal_to_solo": bool(same),
        "statuses_ok": bool(all(s_ in (0, 100) for s_ in status)),
    }


def bench_paper_settings(ctx):
    """The paper's two other KP-SVD settings with R(A) generated from the PSF:
    n = 100 (7 x 7 speckle-like PSF, zero BC, k = 5, p = 2) and n = 200 (11 x 11,
    zero BC, k = 16, p = 4); EGKB(SP) with full reorthogonalization and
    RSVD(SP) with q = 1, FP32, median of 5 calls. The paper's times are quoted
    as context (Matlab on an Apple M2 Max CPU, with its own PSFs)."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_2410_00233_amd import api
    out = {}
    for n, half, k, p, paper in ((100, 4, 5, 2, "Table 4: EGKB(SP) 0.14 s, RSVD(SP) 0.22 s"),
                                 (200, 6, 16, 4, "Table 8: EGKB(SP) 4.37 s, RSVD(SP) 3.94 s")):
        P, cu, cv = wl.speckle_psf(half, seed=wl.SEED_PSF + 900 + n)
        blur = api.Blur(P, cu, cv, n, on_device=True)
        res = {"workload": f"n={n}, {P.shape[0]}x{P.shape[1]} speckle-like PSF, zero BC, "
                           f"k={k}, p={p}, FP32, R(A) generated"}
        for name, fn in (("egkb_sp_ms", lambda: ctx.kp_svd_gkb(blur, k, p, prec="f32", seed=1)),
                         ("rsvd_sp_ms", lambda: ctx.kp_svd_rsvd(blur, k, p, 1, prec="f32",
                                                               seed=2))):
            fn()
            times = []
            for _ in range(5):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                times.append(1e3 * (time.perf_counter() - t0))
            res[name] = round(float(np.median(times)), 3)
        res["paper_context"] = paper + " (Matlab, Apple M2 Max CPU, its own speckle PSFs)"
        out[f"n{n}"] = res
    return out


def bench_paper_pipeline(ctx, n=128):
    """The paper's own pipeline on its "Medium" setting (n = 128, reflexive
    boundary conditions, a 15 x 15 speckle-like PSF, k = 8, p = 4): explicit A,
    reorder to R(A), EGKB(SP) and RSVD(SP, q = 1) over the stored R, then
    isotropic split Bregman with the Kronecker factors and with A itself."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_2410_00233_amd import api
    P, cu, cv = wl.speckle_psf(8, seed=wl.SEED_PSF + 900)      # 15 x 15 support
    blur = api.Blur(P, cu, cv, n, on_device=True, bc="reflexive")
    out = {"workload": f"n={n}, reflexive BC, 15x15 speckle-like PSF, rank 8 (p=4), "
                       "R(A) stored in HBM (FP32 for the KP-SVD, FP64 A for SB); the "
                       "KP-SVDs also with R(A) generated from the PSF"}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, 1e3 * (time.perf_counter() - t0)

    A32, out["build_A_ms"] = timed(lambda: ctx.kp_blur_matrix(blur, prec="f32"))
    R32, _ = timed(lambda: ctx.kp_rmat_reorder(n, A32))
    R32, out["reorder_ms"] = timed(lambda: ctx.kp_rmat_reorder(n, A32, R=R32))
    ctx.kp_svd_gkb(None, 8, 4, prec="f32", seed=1, stored=(n, R32))
    fg, out["egkb_sp_ms"] = timed(lambda: ctx.kp_svd_gkb(None, 8, 4, prec="f32", seed=1,
                                                          stored=(n, R32)))
    ctx.kp_svd_rsvd(None, 8, 4, 1, prec="f32", seed=2, stored=(n, R32))
    fr, out["rsvd_sp_ms"] = timed(lambda: ctx.kp_svd_rsvd(None, 8, 4, 1, prec="f32", seed=2,
                                                           stored=(n, R32)))
    out["sigma_egkb_vs_rsvd_max_diff_over_sigma1"] = float(
        np.abs(fg.sigma[:8] - fr.sigma[:8]).max() / fr.sigma[0])
    # the same KP-SVDs with R(A) generated from the PSF (reflexive terms; no A,
    # no reorder, no stored R)
    ctx.kp_svd_gkb(blur, 8, 4, prec="f32", seed=1)
    fgg, out["egkb_sp_generated_ms"] = timed(lambda: ctx.kp_svd_gkb(blur, 8, 4, prec="f32",
                                                                     seed=1))
    ctx.kp_svd_rsvd(blur, 8, 4, 1, prec="f32", seed=2)
    frg, out["rsvd_sp_generated_ms"] = timed(lambda: ctx.kp_svd_rsvd(blur, 8, 4, 1, prec="f32",
                                                                      seed=2))
    out["sigma_generated_vs_stored_max_diff_over_sigma1"] = float(max(
        np.abs(fgg.sigma[:8] - fg.sigma[:8]).max(), np.abs(frg.sigma[:8] - fr.sigma[:8]).max())
        / fr.sigma[0])
    del A32, R32
    A64 = ctx.kp_blur_matrix(blur, prec="f64")
    x_true = wl.rectangles_image(n, seed=wl.SEED_IMAGE + 900)
    xv = torch.tensor(x_true.flatten(order="F"), dtype=torch.float64, device="cuda")
    bv = ctx.kp_rmat_apply_stored(n, A64, xv).cpu().numpy()
    b = wl.add_noise(bv.reshape((n, n), order="F"), 0.01, seed=wl.SEED_NOISE + 900)
    b_dev = torch.tensor(b, dtype=torch.float64, device="cuda")
    lam = 0.115
    kw = dict(L_max=50, I_max=100, tau_sb=1e-3, tau_cgls=1e-4)
    fk = ctx.kp_svd_rsvd(None, 8, 4, 1, prec="f64", seed=2,
                         stored=(n, ctx.kp_rmat_reorder(n, A64)))
    (xk, sk), out["sb_iso_kp_ms"] = timed(lambda: ctx.sb_solve_iso(fk, b_dev, lam, lam ** 2 / 2, **kw))
    (xa, sa), out["sb_iso_direct_ms"] = timed(
        lambda: ctx.sb_solve_iso_direct(n, A64, b_dev, lam, lam ** 2 / 2, **kw))
    out["sb_kp_iterations"] = [int(sk["l_end"]), int(sk["iota_total"])]
    out["sb_direct_iterations"] = [int(sa["l_end"]), int(sa["iota_total"])]
    out["sb_speedup_kp_vs_direct"] = round(out["sb_iso_direct_ms"] / out["sb_iso_kp_ms"], 2)
    out["sb_kp_relative_error"] = round(float(np.linalg.norm(xk.cpu().numpy() - x_true)
                                              / np.linalg.norm(x_true)), 4)
    out["sb_direct_relative_error"] = round(float(np.linalg.norm(xa.cpu().numpy() - x_true)
                                                  / np.linalg.norm(x_true)), 4)
    out["paper_context"] = ("Table 5 (satellite, n=128, Medium, reflexive, Apple M2 Max CPU): "
                            "R(A) 2.04 s, EGKB(SP) 0.51 s, RSVD(SP) 0.72 s")
    for k_ in list(out):
        if k_.endswith("_ms"):
            out[k_] = round(out[k_], 3)
    return out


def bench_serving(ctx, count, rate, sizes):
    """Open-loop serving: Poisson arrivals at `rate`/s, n drawn 4:3:2:1 over
    `sizes`, 16 recurring PSFs, iso/aniso 50/50, split Bregman 50 outer
    iterations with CGLS tau 1e-4 (I_max 100), rank-20 FP32 RSVD factors kept
    per PSF. The factor cache is warmed first (the cold misses are reported
    separately); latency = completion - scheduled arrival."""
    import threading

    import numpy as np
    import torch

    import workloads as wl
    from paper_2410_00233_amd import api
    weights = (4, 3, 2, 1)[:len(sizes)]
    stream = wl.serving_stream(count, rate, sizes=sizes, weights=weights)
    kw = dict(method="rsvd", k=20, p=10, q=2, prec="f32", seed=11, lam=0.115,
              beta=0.115 ** 2 / 2.0, L_max=50, I_max=100, tau_sb=0.0, tau_cgls=1e-4)
    blurs, imgs = {}, {}
    for i, r in enumerate(stream):
        key = (r["psf_id"], r["n"])
        if key not in blurs:
            P, cu, cv = wl.serving_psf(r["psf_id"], r["n"])
            blurs[key] = api.Blur(P, cu, cv, r["n"])
        x_true = wl.rectangles_image(r["n"], seed=wl.SEED_IMAGE + 100 + i)
        P = blurs[key].P
        b = wl.add_noise(wl.blur_zero_bc(P, blurs[key].cu, blurs[key].cv, x_true), 0.01,
                         seed=wl.SEED_NOISE + 100 + i)
        imgs[i] = torch.tensor(b, dtype=torch.float64, device="cuda")
    log(f"serving: inputs ready ({len(blurs)} PSF/size pairs); warming the factor cache")
    srv = api.Server(ctx, slots=4)
    # warm the factor cache: one cheap solve per (PSF, n) computes its factors
    cold = {}
    warm_kw = dict(kw, L_max=1, I_max=1)
    for (pid, nn), blur in blurs.items():
        b = imgs[next(i for i, r in enumerate(stream) if (r["psf_id"], r["n"]) == (pid, nn))]
        x = torch.empty_like(b)
        res = srv.wait(srv.submit(blur, b, x, psf_key=1 + pid, **warm_kw))
        cold.setdefault(str(nn), []).append(res["factor_ms"])
    outs = {i: torch.empty_like(imgs[i]) for i in imgs}
    tickets = {}
    t_sub = {}
    t0 = time.perf_counter()

    def submitter():
        for i, r in enumerate(stream):
            dt = t0 + r["t"] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            key = (r["psf_id"], r["n"])
            t_sub[i] = time.perf_counter()
            tickets[i] = srv.submit(blurs[key], imgs[i], outs[i], psf_key=1 + r["psf_id"],
                                    iso=r["iso"], **kw)

    log("serving: open-loop run")
    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    res = {}
    for i, t in tickets.items():
        res[i] = srv.wait(t)
        log(f"serving: request {i} (n={stream[i]['n']}) done, {res[i]['total_ms']:.0f} ms")
    t_end = time.perf_counter()
    lat = np.array([(t_sub[i] - (t0 + stream[i]["t"])) * 1e3 + res[i]["total_ms"]
                    for i in range(count)])
    per_n = {}
    for i, r in enumerate(stream):
        per_n.setdefault(str(r["n"]), []).append(lat[i])
    st = srv.stats()
    srv.close()
    return {
        "workload": f"{count} requests, Poisson {rate}/s, n in {list(sizes)} weighted "
                    f"{list(weights)}, 16 recurring PSFs (Gaussian/motion/disk), iso/aniso 50/50, "
                    "SB 50 outer iterations, CGLS tau 1e-4 (I_max 100), rank-20 FP32 RSVD factors "
                    "cached per PSF, 4 slots",
        "p50_ms": round(float(np.percentile(lat, 50)), 2),
        "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "solves_per_s": round(count / (t_end - t0), 3),
        "per_n_p50_ms": {k_: round(float(np.percentile(v, 50)), 2) for k_, v in per_n.items()},
        "per_n_count": {k_: len(v) for k_, v in per_n.items()},
        "mean_solve_ms": round(float(np.mean([r["solve_ms"] for r in res.values()])), 2),
        "mean_queue_ms": round(float(np.mean([r["queue_ms"] for r in res.values()])), 2),
        "cache_hits": int(sum(r["cache_hit"] for r in res.values())),
        "cold_factor_ms_p50_per_n": {k_: round(float(np.median(v)), 1) for k_, v in cold.items()},
        "peak_concurrent": int(st["peak_running"]),
        "iota_total_mean": round(float(np.mean([r["iota_total"] for r in res.values()])), 1),
        "all_ok": bool(all(r["status"] == 0 for r in res.values())),
    }


def nonzero_fractions(P, cu, cv, n):
    """Fractions of the rows, columns and entries of R(A) that are nonzero for
    the PSF rounded to FP32 (R[i+nj, r+nc] = P[cu+r-c, cv+i-j]; the offset d of
    a row or column occurs n - |d| times). Every product still multiplies the
    whole dense R(A): these numbers say how much of that work meets zeros."""
    import numpy as np
    P32 = np.asarray(P, dtype=np.float32) != 0
    off = np.arange(-(n - 1), n)
    w = (n - np.abs(off)).astype(np.float64)
    sub = np.zeros((2 * n - 1, 2 * n - 1), dtype=bool)       # [e (u offset), d (v offset)]
    uu = cu + off
    vv = cv + off
    ok_u = (uu >= 0) & (uu < P.shape[0])
    ok_v = (vv >= 0) & (vv < P.shape[1])
    sub[np.ix_(ok_u, ok_v)] = P32[np.ix_(uu[ok_u], vv[ok_v])]
    N2 = float(n) ** 2
    rows = float(w[sub.any(axis=0)].sum() / N2)
    cols = float(w[sub.any(axis=1)].sum() / N2)
    ents = float((w[:, None] * w[None, :])[sub].sum() / N2 ** 2)
    return {"rows": round(rows, 5), "cols": round(cols, 5), "entries": round(ents, 6)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--sb-solves", type=int, default=5)
    ap.add_argument("--batched", type=int, default=64,
                    help="problems in the batched KP-SVD run (0 skips it)")
    ap.add_argument("--serve", type=int, default=24,
                    help="requests in the serving run (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=2.0,
                    help="offered Poisson arrival rate of the serving run (requests/s)")
    ap.add_argument("--serve-sizes", type=str, default="128,256,512,1024")
    ap.add_argument("--serve-sweep", type=str, default="",
                    help="comma-separated offered rates (req/s): run the serving workload at "
                         "each (sizes 128,256,512; --serve requests each) and report them")
    ap.add_argument("--gkb-block", type=int, default=20,
                    help="block size b of the timed block Golub-Kahan run")
    ap.add_argument("--no-paper-pipeline", action="store_true",
                    help="skip the explicit-matrix run on the paper's n = 128 setting")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the KP-SVD path is built and timed on a single "
              "MI355X (multi-GPU sharding is designed but not built); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as wl
    from paper_2410_00233_amd import api, flops

    n = args.n
    k, p_gkb, p_rsvd, q = 20, 20, 10, 2
    P, cu, cv = wl.gaussian_psf(n)
    nz = nonzero_fractions(P, cu, cv, n)
    blur = api.Blur(P, cu, cv, n, on_device=True)
    ctx = api.Context(0)
    f_gkb = flops.egkb(n, k, p_gkb)
    f_rsvd = flops.rsvd(n, k, p_rsvd, q)
    comp = {"egkb_ms": [], "rsvd_ms": []}

    def step(record):
        t0 = time.perf_counter()
        fg = ctx.kp_svd_gkb(blur, k, p_gkb, prec="f32", reorth=1, seed=1, factor_prec="f64")
        t1 = time.perf_counter()
        fr = ctx.kp_svd_rsvd(blur, k, p_rsvd, q, prec="f32", seed=2, factor_prec="f64")
        t2 = time.perf_counter()
        if record:
            comp["egkb_ms"].append(1e3 * (t1 - t0))
            comp["rsvd_ms"].append(1e3 * (t2 - t1))
        return fg, fr

    log(f"KP-SVD step at n={n}: {args.warmup} warm-up + {args.steps} timed")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    ctx.kp_prof_read(reset=True)
    ctx.kp_prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fg, fr = step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.kp_prof_enable(False)
    prof = ctx.kp_prof_read(reset=True)
    ms_step = 1e3 * (t1 - t0) / args.steps
    value = (f_gkb + f_rsvd) / (ms_step * 1e-3) / 1e12

    log(f"step {ms_step:.1f} ms ({value:.1f} TFLOP/s); block GKB (b = {args.gkb_block})")
    # the block form of Algorithm 1 on the same workload and k_p: its products
    # with B and B^T are block products of b columns on the MFMA kernel
    b_blk = args.gkb_block
    nb_blk = -(-(k + p_gkb) // b_blk)
    f_blk = flops.egkb(n, k, nb_blk * b_blk - k)
    fblk = ctx.kp_svd_gkb(blur, k, p_gkb, prec="f32", seed=1, factor_prec="f64", block=b_blk)
    tblk = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        fblk = ctx.kp_svd_gkb(blur, k, p_gkb, prec="f32", seed=1, factor_prec="f64", block=b_blk)
        tblk.append(1e3 * (time.perf_counter() - ta))
    blk_ms = float(np.median(tblk))
    blk_diff = float(np.abs(fblk.sigma[:k] - fg.sigma[:k]).max() / fg.sigma[0])

    log("reflexive boundary conditions (four generated terms)")
    blur_r = blur.with_bc("reflexive")
    ctx.kp_svd_rsvd(blur_r, k, p_rsvd, q, prec="f32", seed=2, factor_prec="f64")
    trf = []
    for _ in range(max(1, args.steps // 2)):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        frr = ctx.kp_svd_rsvd(blur_r, k, p_rsvd, q, prec="f32", seed=2, factor_prec="f64")
        trf.append(1e3 * (time.perf_counter() - ta))
    refl_ms = float(np.median(trf))
    refl_diff = float(np.abs(frr.sigma[:k] - fr.sigma[:k]).max() / fr.sigma[0])

    log("support compaction (same results, zero tiles skipped)")
    blur_c = blur.with_bc(compact=True)
    ctx.kp_svd_rsvd(blur_c, k, p_rsvd, q, prec="f32", seed=2, factor_prec="f64")
    tcp = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        frc = ctx.kp_svd_rsvd(blur_c, k, p_rsvd, q, prec="f32", seed=2, factor_prec="f64")
        tcp.append(1e3 * (time.perf_counter() - ta))
    comp_ms = float(np.median(tcp))
    comp_same = bool(np.array_equal(frc.sigma[:k], fr.sigma[:k]))
    ctx.kp_svd_gkb(blur_c, k, p_gkb, prec="f32", reorth=1, seed=1, factor_prec="f64")
    tcg = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        fgc = ctx.kp_svd_gkb(blur_c, k, p_gkb, prec="f32", reorth=1, seed=1, factor_prec="f64")
        tcg.append(1e3 * (time.perf_counter() - ta))
    compg_ms = float(np.median(tcg))
    compg_same = bool(np.array_equal(fgc.sigma[:k], fg.sigma[:k]))

    log("BF16 + refinement RSVD")
    # the reduced-precision variant: RSVD with BF16 block products + refinement
    # (refine = 2: the refinement product from split FP16 MFMA products; the
    # refine = 1 variant with an FP32 product is timed beside it)
    f_ref = flops.rmat_product(n, k)
    ctx.kp_svd_rsvd(blur, k, p_rsvd, q, prec="bf16", refine=2, seed=2, factor_prec="f64")
    torch.cuda.synchronize()
    ctx.kp_prof_enable(True)
    tb = []
    for _ in range(args.steps):
        ta = time.perf_counter()
        fb = ctx.kp_svd_rsvd(blur, k, p_rsvd, q, prec="bf16", refine=2, seed=2, factor_prec="f64")
        tb.append(1e3 * (time.perf_counter() - ta))
    ctx.kp_prof_enable(False)
    prof16 = ctx.kp_prof_read(reset=True)
    tb1 = []
    for _ in range(args.steps):
        ta = time.perf_counter()
        fb1 = ctx.kp_svd_rsvd(blur, k, p_rsvd, q, prec="bf16", refine=1, seed=2, factor_prec="f64")
        tb1.append(1e3 * (time.perf_counter() - ta))
    b16 = prof16["block16"]
    avg16 = b16["ms"] / max(b16["launches"], 1)
    ach16 = (b16["flops"] / max(b16["launches"], 1)) / (avg16 * 1e-3) / 1e12
    bf_ms = float(np.median(tb))
    bf1_ms = float(np.median(tb1))
    sig_diff = float(np.abs(fb.sigma[:k] - fr.sigma[:k]).max() / fr.sigma[0])
    sig_diff1 = float(np.abs(fb1.sigma[:k] - fr.sigma[:k]).max() / fr.sigma[0])

    log("split Bregman latency at n=256")
    ns = 256
    Ps, cus, cvs, xs_true, bs_true, bs = wl.deblur_problem(ns, "gaussian", 0.01, 0)
    blur_s = api.Blur(Ps, cus, cvs, ns, on_device=True)
    fs = ctx.kp_svd_rsvd(blur_s, k, p_rsvd, q, prec="f32", seed=3, factor_prec="f64")
    b_dev = torch.tensor(bs, dtype=torch.float64, device="cuda")
    lam, gam = 0.115, 2.0
    lat, st = [], None
    for rep in range(1 + args.sb_solves):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        xs, st = ctx.sb_solve_iso(fs, b_dev, lam, lam * lam / gam, L_max=50, I_max=100,
                                  tau_cgls=1e-4)
        torch.cuda.synchronize()
        if rep > 0:
            lat.append(1e3 * (time.perf_counter() - ta))
    x_np = xs.cpu().numpy()
    re_sb = float(np.linalg.norm(x_np - xs_true) / np.linalg.norm(xs_true))

    blk = prof["block"]
    avg_blk_ms = blk["ms"] / max(blk["launches"], 1)
    flops_blk = blk["flops"] / max(blk["launches"], 1)
    achieved = flops_blk / (avg_blk_ms * 1e-3) / 1e12
    gv = prof["gemv"]
    avg_gv_ms = gv["ms"] / max(gv["launches"], 1)
    gemv_tflops = (gv["flops"] / max(gv["launches"], 1)) / (avg_gv_ms * 1e-3) / 1e12

    tune = ctx.kp_tune_report()
    v32 = next((t["variant"] for t in tune if t["op"] == "block32" and t["n"] == n and t["a"] == 4), None)
    v16 = next((t["variant"] for t in tune if t["op"] == "block16" and t["n"] == n), None)
    line = {
        "metric": "KP-SVD time & TFLOP/s at n=512 (FP32 vs BF16+refine); p50/p99 solve latency",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"rank-{k} KP-SVD of R(A), n={n} (R(A) {n*n}x{n*n}), rotated Gaussian PSF "
                        f"sigma=(2,1) 30deg on the full offset grid, zero BC; step = EGKB "
                        f"(k_p={k+p_gkb}, full reorth) + RSVD (p={p_rsvd}, q={q}), FP32",
            "n": n, "rank": k, "egkb_kp": k + p_gkb, "rsvd_p": p_rsvd, "rsvd_q": q,
            "flops_per_step": f_gkb + f_rsvd,
            "rmat_nonzero_fractions_fp32": nz,
        },
        "components": {
            "step_ms_p10": round(float(np.percentile(np.add(comp["egkb_ms"], comp["rsvd_ms"]), 10)), 3),
            "step_ms_p50": round(float(np.percentile(np.add(comp["egkb_ms"], comp["rsvd_ms"]), 50)), 3),
            "step_ms_p90": round(float(np.percentile(np.add(comp["egkb_ms"], comp["rsvd_ms"]), 90)), 3),
            "egkb_ms": round(float(np.median(comp["egkb_ms"])), 3),
            "rsvd_ms": round(float(np.median(comp["rsvd_ms"])), 3),
            "egkb_tflops": round(f_gkb / (np.median(comp["egkb_ms"]) * 1e-3) / 1e12, 3),
            "rsvd_tflops": round(f_rsvd / (np.median(comp["rsvd_ms"]) * 1e-3) / 1e12, 3),
            "gemv_kernel_avg_ms": round(avg_gv_ms, 4),
            "gemv_kernel_tflops": round(gemv_tflops, 3),
            "egkb_block_b": b_blk,
            "egkb_block_kp": nb_blk * b_blk,
            "egkb_block_ms": round(blk_ms, 3),
            "egkb_block_tflops": round(f_blk / (blk_ms * 1e-3) / 1e12, 3),
            "egkb_block_speedup_vs_egkb": round(float(np.median(comp["egkb_ms"])) / blk_ms, 3),
            "egkb_block_breakdowns": len(fblk.breakdowns),
            "egkb_block_max_sigma_diff_vs_egkb_over_sigma1": blk_diff,
            "rsvd_compact_ms": round(comp_ms, 3),
            "rsvd_compact_speedup_vs_dense": round(float(np.median(comp["rsvd_ms"])) / comp_ms, 3),
            "rsvd_compact_sigma_bitwise_equal_to_dense": comp_same,
            "egkb_compact_ms": round(compg_ms, 3),
            "egkb_compact_speedup_vs_dense": round(float(np.median(comp["egkb_ms"])) / compg_ms, 3),
            "egkb_compact_sigma_bitwise_equal_to_dense": compg_same,
            "rsvd_reflexive_ms": round(refl_ms, 3),
            "rsvd_reflexive_tflops_algorithmic": round(f_rsvd / (refl_ms * 1e-3) / 1e12, 3),
            "rsvd_reflexive_tflops_executed": round(4 * f_rsvd / (refl_ms * 1e-3) / 1e12, 3),
            "rsvd_reflexive_max_sigma_diff_vs_zero_bc_over_sigma1": refl_diff,
            "sigma_egkb_top3": [float(x) for x in fg.sigma[:3]],
            "sigma_rsvd_top3": [float(x) for x in fr.sigma[:3]],
            "rsvd_bf16_refine_ms": round(bf_ms, 3),
            "rsvd_bf16_refine_tflops": round((f_rsvd + f_ref) / (bf_ms * 1e-3) / 1e12, 3),
            "rsvd_bf16_refine_speedup_vs_fp32": round(float(np.median(comp["rsvd_ms"])) / bf_ms, 3),
            "rsvd_bf16_refine_max_sigma_diff_vs_fp32_over_sigma1": sig_diff,
            "rsvd_bf16_refine_product": "split FP16 (three FP16 MFMA products of two-term splits)",
            "rsvd_bf16_refine_fp32_product_ms": round(bf1_ms, 3),
            "rsvd_bf16_refine_fp32_product_max_sigma_diff_vs_fp32_over_sigma1": sig_diff1,
        },
        "sb_solve_n256": {
            "kind": "isotropic split Bregman, 50 outer iterations, CGLS tau 1e-4 (I_max 100), "
                    "k = 20 factors, rectangles image + 1% noise, FP64",
            "solves": len(lat), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "iota_total": int(st["iota_total"]), "l_end": int(st["l_end"]),
            "relative_error": round(re_sb, 4),
            "cgls_tflops": round(st["iota_total"] * flops.cgls_iteration_kp(ns, k)
                                 / (float(np.percentile(lat, 50)) * 1e-3) / 1e12, 3),
        },
        "roofline_bf16": {
            "kernel": f"rmat_block16_kernel<bf16,{BLOCK16_VARIANT_TEMPLATE.get(v16, '?')}> "
                      "(generated-tile R(A) X, BF16 MFMA 16x16x32, FP32 accumulate)",
            "bound": "mfma", "achieved": round(ach16, 3), "peak": MFMA_BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach16 / MFMA_BF16_PEAK_TFLOPS, 4),
            "avg_launch_ms": round(avg16, 4), "launches": int(b16["launches"]),
            "traffic": counted_traffic("rmat_block16.hip", BLOCK16_TRAFFIC_SRC_SHA1,
                                       BLOCK16_TRAFFIC_BYTES) if n == 512 else None,
        },
        "roofline": {
            "kernel": f"rmat_block_kernel<float,{BLOCK_VARIANT_TEMPLATE.get(v32, '?')}> "
                      "(generated-tile R(A) X, FP32 MFMA 16x16x4)",
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": MFMA_FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / MFMA_FP32_PEAK_TFLOPS, 4),
            "traffic": counted_traffic("rmat_block.hip", BLOCK_TRAFFIC_SRC_SHA1,
                                       BLOCK_TRAFFIC_BYTES) if n == 512 else None,
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
            "avg_launch_ms": round(avg_blk_ms, 4),
            "launches": int(blk["launches"]),
            "flops_per_launch": flops_blk,
        },
    }
    if args.batched > 0:
        log(f"batched KP-SVD, {args.batched} problems")
        line["batched"] = bench_batched(ctx, args.batched)
    if args.serve_sweep:
        sweep = {}
        for rate in [float(r) for r in args.serve_sweep.split(",") if r]:
            log(f"serving sweep: {args.serve} requests at {rate}/s")
            r_ = bench_serving(ctx, args.serve, rate, (128, 256, 512))
            sweep[str(rate)] = {k_: r_[k_] for k_ in ("p50_ms", "p99_ms", "solves_per_s",
                                                      "mean_queue_ms", "mean_solve_ms",
                                                      "per_n_p50_ms", "all_ok")}
        line["serving_sweep"] = {"workload": f"{args.serve} requests per rate, n in "
                                             "[128, 256, 512] weighted [4, 3, 2], otherwise as "
                                             "the serving run", "rates": sweep}
    if args.serve > 0:
        sizes = tuple(int(v) for v in args.serve_sizes.split(","))
        log(f"serving, {args.serve} requests at {args.serve_rate}/s")
        line["serving"] = bench_serving(ctx, args.serve, args.serve_rate, sizes)
    if not args.no_paper_pipeline:
        log("explicit-matrix pipeline at n=128 (reflexive BC)")
        line["paper_pipeline_n128"] = bench_paper_pipeline(ctx)
        log("the paper's n=100 and n=200 KP-SVD settings")
        line["paper_settings"] = bench_paper_settings(ctx)
    line["autotune"] = ctx.kp_tune_report()
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(n, k + p_rsvd, args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
