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

Beside the headline the line carries: the block form of Algorithm 1, reflexive
boundary conditions and support compaction on the same workload; the BF16 +
refinement RSVD with its own roofline object; the defocus disk r = 8 at n = 512;
the n = 256 isotropic split Bregman latency; the 64-problem batched KP-SVD; the
serving stream (Poisson arrivals at the configured 200/s, n in 128..1024) and a
sweep of offered rates; the paper's explicit-matrix pipeline at n = 128; the
autotuner's choices. The CPU leg runs the oracle on the host cores: its dense
product R X in FP32 / FP64 with all threads and with one (cpu_baseline), and
its own runs of the timed configurations on the same start vectors and
sketches, from which the accuracy object takes each GPU result's sigma error
against the same-algorithm FP64 oracle and ||A - A_k|| / ||A|| against the
exact optimum.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --profile-products   (the rocprofv3 counter workload)
       python bench.py --profile-qr         (the same for the Householder TSQR)
       python bench.py --profile-fft        (the same for the FFT blur products)
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
BLOCK_TRAFFIC_BYTES = 1.149e9
BLOCK_TRAFFIC_SRC_SHA1 = "8437c6e328e38f76a1c577556af9242481da709b"
BLOCK16_TRAFFIC_BYTES = 2.10e8
# template arguments <TJ, JB, CB> of the FP32 block kernel per autotuner variant
BLOCK_VARIANT_TEMPLATE = {0: "16,1,2,false,64", 1: "16,2,2,false,64", 2: "8,1,2,false,64",
                          3: "8,1,1,false,64", 4: "16,1,2,false,128", 5: "16,2,2,false,128",
                          6: "8,1,2,false,128", 7: "8,1,1,false,128", 8: "16,1,2,false,192",
                          9: "16,2,2,false,192", 10: "8,1,2,false,192", 11: "8,1,1,false,192",
                          12: "16,1,2,false,176", 13: "16,2,2,false,176", 14: "8,1,2,false,176",
                          15: "8,1,1,false,176", 16: "12,1,2,false,176", 17: "12,1,2,false,128"}
BLOCK16_VARIANT_TEMPLATE = {0: "32,4,2,false", 1: "16,4,2,false", 2: "32,2,2,false",
                            3: "16,2,2,false", 4: "16,1,2,false", 5: "64,4,2,false",
                            6: "64,8,2,false"}
BLOCK16_TRAFFIC_SRC_SHA1 = "1d396a6114ec7c6b99b29d64d45dd0385a11f690"


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


def _cpu_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_dense_timings(n, ncols, run_s):
    """O-dense: the oracle's dense product R X (every n x n block of R(A) read
    as a window of the PSF and multiplied with BLAS: the same 2 N^2 flops per
    column as the GPU kernel), in FP32 and FP64, with all BLAS threads and with
    one, each the median of 3 runs over a bounded sample of block rows sized to
    about run_s seconds."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as wl
    from oracle import operator as op
    P, cu, cv = wl.gaussian_psf(n)
    N = n * n
    X = wl.gaussian_block(N, ncols, seed=wl.SEED_START + 7)
    all_threads = _cpu_threads()
    out = {}
    for dt in (np.float32, np.float64):
        for threads in (all_threads, 1):
            with threadpool_limits(limits=threads):
                t0 = time.perf_counter()
                op.rmat_window_apply(P, cu, cv, n, X, blocks=range(1), dtype=dt)
                per_block = time.perf_counter() - t0
                nb = int(min(n, max(1, run_s / max(per_block, 1e-6))))
                times = []
                for _ in range(3):
                    t0 = time.perf_counter()
                    op.rmat_window_apply(P, cu, cv, n, X, blocks=range(nb), dtype=dt)
                    times.append(time.perf_counter() - t0)
            el = float(np.median(times))
            flops = 2.0 * nb * n * N * ncols
            key = f"{np.dtype(dt).name}_{'all' if threads > 1 else '1'}_threads"
            out[key] = {"tflops": flops / el / 1e12, "threads": threads, "block_rows": nb,
                        "rows": nb * n, "median_s": round(el, 3),
                        "full_product_s_extrapolated": round(el * n / nb, 1)}
    return out


def cpu_baseline_leg(n, k, p_rsvd, q, cases, run_s):
    """The oracle on the host cores: O-dense product timings (the reported
    baseline), and the oracle's own runs of the timed configurations on the
    same start vectors / sketches as the GPU (O-struct: R applied through its
    offset structure, a different algorithm for the products, so its time is not
    comparable with the dense GPU products). The latter give the accuracy of each
    GPU result: sigma against the same-algorithm FP64 oracle (normwise, / sigma_1)
    and ||A - A_k||_F / ||A||_F of the GPU's factors beside the oracle's and the
    exact optimum (the truncated SVD of R(A))."""
    import numpy as np

    from oracle import kpsvd, metrics, operator as op, philox
    dense = cpu_dense_timings(n, k + p_rsvd, run_s)
    main = dense["float32_all_threads"]
    base = {"value": main["tflops"], "unit": "TFLOP/s", "cores": main["threads"],
            "kind": "oracle",
            "sample": f"O-dense: R(A) X in FP32 with R's n x n blocks read as PSF windows and "
                      f"multiplied with BLAS, n={n} rotated Gaussian, {k + p_rsvd} columns, "
                      f"block rows 0..{main['block_rows'] - 1} ({main['rows']} of {n * n} rows), "
                      f"median of 3 ({main['median_s']} s each); the other precisions / "
                      "thread counts under cpu_dense",
            "dense": dense}
    acc = {}
    struct = {}
    for c in cases:
        P, cu, cv, nn = c["P"], c["cu"], c["cv"], c["n"]
        N = nn * nn
        R = lambda X, P=P, cu=cu, cv=cv, nn=nn: op.rmat_struct_apply(P, cu, cv, nn, X)
        Rt = lambda X, P=P, cu=cu, cv=cv, nn=nn: op.rmat_struct_apply(P, cu, cv, nn, X,
                                                                      transpose=True)
        t0 = time.perf_counter()
        if c["method"] == "gkb":
            y = philox.normals(N, c["seed"], 0).astype(np.float32).astype(np.float64)
            ref = kpsvd.egkb(R, Rt, y, c["k"], c["p"], reorth="full", seed=c["seed"],
                             force_breakdown=set(c["breakdowns"]))
        else:
            F = np.stack([philox.normals(N, c["seed"], 0x40000000 + col)
                          for col in range(c["k"] + c["p"])], axis=1)
            F = F.astype(np.float32).astype(np.float64)
            ref = kpsvd.rsvd(R, Rt, F, c["k"], c["q"])
            if c["refine"]:
                ref = kpsvd.refine(R, ref["V"])
        t_oracle = time.perf_counter() - t0
        t0 = time.perf_counter()
        s_ex = op.exact_kpsvd(P, cu, cv, nn, c["k"])[0]
        t_exact = time.perf_counter() - t0
        r2 = op.rmat_fro_norm2(P, cu, cv, nn)
        kk = c["k"]
        sg = np.asarray(c["sigma"][:kk])
        U = np.stack([c["Ax"][t].flatten(order="F") / sg[t] if sg[t] > 0 else np.zeros(N)
                      for t in range(kk)], axis=1)
        V = np.stack([c["Ay"][t].flatten(order="F") for t in range(kk)], axis=1)
        s1 = ref["sigma"][0]
        ds = np.abs(sg - ref["sigma"][:kk])
        big = ref["sigma"][:kk] >= 1e-2 * s1
        acc[c["name"]] = {
            "sigma_err_vs_same_alg_fp64_oracle_over_sigma1": float(ds.max() / s1),
            "gate": c["gate"],
            "pass": bool(ds.max() / s1 <= c["gate"]),
            "sigma_rel_err_componentwise_max_for_sigma_ge_1e-2_sigma1":
                float((ds[big] / ref["sigma"][:kk][big]).max()),
            "kp_rel_err_gpu": metrics.kp_rel_error(P, cu, cv, nn, sg, U, V),
            "kp_rel_err_oracle": metrics.kp_rel_error(P, cu, cv, nn, ref["sigma"], ref["U"],
                                                      ref["V"]),
            "kp_rel_err_optimum": float(np.sqrt(max(0.0, 1.0 - np.sum(s_ex ** 2) / r2))),
            "sigma_err_vs_exact_over_sigma1": float(np.abs(sg - s_ex).max() / s_ex[0]),
        }
        struct[c["name"]] = {"oracle_s": round(t_oracle, 2), "exact_s": round(t_exact, 2)}
    base["o_struct"] = {"kind": "structure-exploiting oracle (R applied through its offset "
                                "structure, O(n^2) per column): a different algorithm for the "
                                "products, not comparable with the dense GPU rate",
                        "threads": _cpu_threads(), "runs": struct}
    return base, acc


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


def bench_sb_batched(ctx, count):
    """Mixed batch of `count` isotropic split Bregman solves (FP64, k = 10..20
    factors from FP32 RSVD, 50 outer x up to 100 CGLS iterations, CGLS tau 1e-4)
    of n in {64, 128, 192, 256} through sb_solve_batched, against the same
    solves as single calls one after another."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_2410_00233_amd import api, flops
    mix = wl.batched_mix(count, sizes=(64, 128, 192, 256), ranks=(10, 20),
                         seed=wl.SEED_PSF + 900)
    lam = 0.115
    probs = []
    for i, d in enumerate(mix):
        blur = api.Blur(d["P"], d["cu"], d["cv"], d["n"], on_device=True)
        f = ctx.kp_svd_rsvd(blur, d["k"], d["p"], 2, prec="f32", seed=d["seed"])
        x_true = wl.rectangles_image(d["n"], seed=wl.SEED_IMAGE + i)
        b = wl.add_noise(wl.blur_zero_bc(d["P"], d["cu"], d["cv"], x_true), 0.01,
                         seed=wl.SEED_NOISE + i)
        probs.append(dict(f=f, b=torch.tensor(b, dtype=torch.float64, device="cuda"), iso=True,
                          lam=lam, beta=lam * lam / 2.0, L_max=50, I_max=100, tau_cgls=1e-4))
    # every (n, k) apply tuned and the workers warm before the timed run
    first = {}
    for pr, d in zip(probs, mix):
        first.setdefault((d["n"], d["k"]), dict(pr, L_max=1, I_max=8))
    ctx.sb_solve_batched(list(first.values()))
    torch.cuda.synchronize()
    log("batched SB: timed run")
    t0 = time.perf_counter()
    xs, stats, status = ctx.sb_solve_batched(probs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batched SB: {1e3 * t_batch:.0f} ms; the same solves one by one")
    t0 = time.perf_counter()
    solo = [ctx.sb_solve_iso(p["f"], p["b"], p["lam"], p["beta"], L_max=50, I_max=100,
                             tau_cgls=1e-4) for p in probs]
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    same = all(torch.equal(x, y[0]) for x, y in zip(xs, solo))
    fl = sum(st["iota_total"] * flops.cgls_iteration_kp(d["n"], d["k"])
             for st, d in zip(stats, mix))
    sizes = [d["n"] for d in mix]
    return {
        "workload": f"{count} isotropic split Bregman solves (FP64, 50 outer x <= 100 CGLS, "
                    "CGLS tau 1e-4, k 10-20), n in {64,128,192,256}, Gaussian/motion/disk PSFs, "
                    "rectangles image + 1% noise, 4 worker streams",
        "problems": count, "n_hist": {str(v): sizes.count(v) for v in sorted(set(sizes))},
        "cgls_iterations": int(sum(st["iota_total"] for st in stats)),
        "batched_ms": round(1e3 * t_batch, 2), "solo_sum_ms": round(1e3 * t_solo, 2),
        "batched_cgls_tflops": round(fl / t_batch / 1e12, 3),
        "speedup_vs_solo": round(t_solo / t_batch, 3),
        "x_equal_to_solo": bool(same),
        "statuses_ok": bool(all(s_ in (0, 100) for s_ in status)),
    }


def bench_paper_pipeline(ctx, n=128):
    """The paper's own pipeline on its "Medium" setting (n = 128, reflexive
    boundary conditions, a 15 x 15 speckle-like PSF, k = 8, p = 4): explicit A,
    reorder to R(A), EGKB(SP) and RSVD(SP, q = 1) over the stored R, then
    isotropic split Bregman with the Kronecker factors and with A itself
    (stored, and through FFT products)."""
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
    ctx.sb_solve_iso_fft(blur, b_dev, lam, lam ** 2 / 2, L_max=1, I_max=1)
    (xf, sf), out["sb_iso_fft_ms"] = timed(
        lambda: ctx.sb_solve_iso_fft(blur, b_dev, lam, lam ** 2 / 2, **kw))
    out["sb_kp_iterations"] = [int(sk["l_end"]), int(sk["iota_total"])]
    out["sb_fft_iterations"] = [int(sf["l_end"]), int(sf["iota_total"])]
    out["sb_direct_iterations"] = [int(sa["l_end"]), int(sa["iota_total"])]
    out["sb_speedup_kp_vs_direct"] = round(out["sb_iso_direct_ms"] / out["sb_iso_kp_ms"], 2)
    out["sb_speedup_kp_vs_fft"] = round(out["sb_iso_fft_ms"] / out["sb_iso_kp_ms"], 2)
    out["sb_fft_relative_error"] = round(float(np.linalg.norm(xf.cpu().numpy() - x_true)
                                               / np.linalg.norm(x_true)), 4)
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


def bench_sb_fft(ctx, sizes=(256, 512), solves=2):
    """Split Bregman with A itself through FFT products (sb_solve_iso_fft)
    beside the same solve with rank-20 Kronecker factors (sb_solve_iso), on
    the same deblurring problem per n (Gaussian PSF on the full offset grid,
    1 % noise, 50 outer iterations, CGLS tau 1e-4): median wall time of
    `solves` solves after one untimed solve, CGLS iterations, restoration
    error."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_2410_00233_amd import api
    out = {"kind": "isotropic split Bregman, A through 2-D FFTs (zero BC) vs rank-20 A_k "
                   "(FP32 RSVD factors), 50 outer iterations, CGLS tau 1e-4 (I_max 100), FP64"}
    for n in sizes:
        P, cu, cv, x_true, _, b = wl.deblur_problem(n, "gaussian", 0.01, 0)
        blur = api.Blur(P, cu, cv, n, on_device=True)
        bd = torch.tensor(b, dtype=torch.float64, device="cuda")
        f = ctx.kp_svd_rsvd(blur, 20, 10, 2, prec="f32", seed=3, factor_prec="f64")
        row = {}
        for name, fn in (("fft", lambda: ctx.sb_solve_iso_fft(blur, bd, 0.115, 0.115 ** 2 / 2,
                                                              L_max=50, I_max=100, tau_cgls=1e-4)),
                         ("kp", lambda: ctx.sb_solve_iso(f, bd, 0.115, 0.115 ** 2 / 2, L_max=50,
                                                         I_max=100, tau_cgls=1e-4))):
            ts = []
            for rep in range(1 + solves):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, st = fn()
                torch.cuda.synchronize()
                if rep > 0:
                    ts.append(1e3 * (time.perf_counter() - t0))
            ms = float(np.median(ts))
            row[f"{name}_ms"] = round(ms, 2)
            row[f"{name}_iota_total"] = int(st["iota_total"])
            row[f"{name}_us_per_cgls_iteration"] = round(1e3 * ms / max(st["iota_total"], 1), 2)
            row[f"{name}_relative_error"] = round(
                float(np.linalg.norm(x.cpu().numpy() - x_true) / np.linalg.norm(x_true)), 4)
        row["fft_speedup_vs_kp"] = round(row["kp_ms"] / row["fft_ms"], 3)
        out[f"n{n}"] = row
    return out


def bench_serving(srv, count, rate, sizes, warmed):
    """Open-loop serving on the server `srv`: Poisson arrivals at `rate`/s, n
    drawn 4:3:2:1 over `sizes`, 16 recurring PSFs, iso/aniso 50/50, split
    Bregman 50 outer iterations with CGLS tau 1e-4 (I_max 100), rank-20 FP32
    RSVD factors kept per PSF. Factor sets not resident yet are computed first
    by one cheap solve each (their cold time is reported; `warmed` remembers
    them across calls); latency = completion - scheduled arrival."""
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
    cold = {}
    warm_kw = dict(kw, L_max=1, I_max=1)
    for (pid, nn), blur in blurs.items():
        if (pid, nn) in warmed:
            continue
        b = imgs[next(i for i, r in enumerate(stream) if (r["psf_id"], r["n"]) == (pid, nn))]
        x = torch.empty_like(b)
        res = srv.wait(srv.submit(blur, b, x, psf_key=1 + pid, **warm_kw))
        warmed[(pid, nn)] = res["factor_ms"]
        cold.setdefault(str(nn), []).append(res["factor_ms"])
    log(f"serving at {rate}/s: {count} requests, {len(blurs)} PSF/size pairs resident")
    outs = {i: torch.empty_like(imgs[i]) for i in imgs}
    tickets = {}
    t_sub = {}
    st0 = srv.stats()
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

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    res = {}
    for i, t in tickets.items():
        res[i] = srv.wait(t)
    t_end = time.perf_counter()
    lat = np.array([(t_sub[i] - (t0 + stream[i]["t"])) * 1e3 + res[i]["total_ms"]
                    for i in range(count)])
    per_n = {}
    for i, r in enumerate(stream):
        per_n.setdefault(str(r["n"]), []).append(lat[i])
    st = srv.stats()
    out = {
        "offered_per_s": rate,
        "requests": count,
        "p50_ms": round(float(np.percentile(lat, 50)), 2),
        "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "solves_per_s": round(count / (t_end - t0), 3),
        "per_n_p50_ms": {k_: round(float(np.percentile(v, 50)), 2) for k_, v in per_n.items()},
        "per_n_p99_ms": {k_: round(float(np.percentile(v, 99)), 2) for k_, v in per_n.items()},
        "per_n_count": {k_: len(v) for k_, v in per_n.items()},
        "mean_solve_ms": round(float(np.mean([r["solve_ms"] for r in res.values()])), 2),
        "mean_queue_ms": round(float(np.mean([r["queue_ms"] for r in res.values()])), 2),
        "cache_hits": int(sum(r["cache_hit"] for r in res.values())),
        "peak_concurrent": int(st["peak_running"]),
        "iota_total_mean": round(float(np.mean([r["iota_total"] for r in res.values()])), 1),
        "all_ok": bool(all(r["status"] == 0 for r in res.values())),
    }
    if cold:
        out["cold_factor_ms_p50_per_n"] = {k_: round(float(np.median(v)), 1)
                                           for k_, v in cold.items()}
    del st0
    return out


def profile_products():
    """Workload of the rocprofv3 counter passes (run under
    ``rocprofv3 --pmc <counters> -- python3 bench.py --profile-products``): in one
    process, a plain copy of 256 MiB FP32 (``torch.mul(x, 1.0, out=y)``: reads
    and writes 256 MiB; the calibration kernel for FETCH_SIZE / WRITE_SIZE), then
    through the library at n = 512 on the rotated Gaussian PSF (PSF in HBM) the
    FP32 block product R X with 30 columns, the FP32 matrix-vector product R x
    and the BF16 block product R X with 30 columns, then at n = 256 with k = 20
    random FP64 factors the Kronecker apply (both directions) and an isotropic
    split Bregman solve of 1 outer x 10 CGLS iterations. The first launches of
    each tuned kernel at a new shape are the autotuner's samples; the measured
    launches follow them."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_2410_00233_amd import api
    n = 512
    x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    ctx = api.Context(0)
    P, cu, cv = wl.gaussian_psf(n)
    blur = api.Blur(P, cu, cv, n, on_device=True)
    X = torch.randn(30, n * n, dtype=torch.float32, device="cuda")
    ctx.kp_rmat_apply(blur, X, prec="f32")
    v = torch.randn(n * n, dtype=torch.float32, device="cuda")
    ctx.kp_rmat_apply(blur, v, prec="f32")
    Xb = torch.randn(30, n * n, dtype=torch.float32, device="cuda")
    ctx.kp_rmat_apply(blur, Xb, prec="bf16")
    ns, k = 256, 20
    rng = np.random.default_rng(5)
    f = api.Factors.from_arrays(rng.standard_normal((k, ns, ns)), rng.standard_normal((k, ns, ns)))
    Z = torch.rand(ns, ns, dtype=torch.float64, device="cuda")
    ctx.kp_apply(f, Z)
    ctx.kp_apply(f, Z, transpose=True)
    ctx.sb_solve_iso(f, Z, 0.115, 0.0066, L_max=1, I_max=10)
    torch.cuda.synchronize()
    ctx.close()
    print("done", flush=True)
    return 0


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


def profile_qr():
    """Workload of the rocprofv3 counter pass over the Householder TSQR: two FP32
    RSVDs (p = 10, q = 2, rank 20) at n = 512 on the rotated Gaussian PSF, each
    with five 262144 x 30 QRs (the first RSVD also runs the autotuner's
    samples of the block products)."""
    import torch

    import workloads as wl
    from paper_2410_00233_amd import api
    n = 512
    ctx = api.Context(0)
    P, cu, cv = wl.gaussian_psf(n)
    blur = api.Blur(P, cu, cv, n, on_device=True)
    for _ in range(2):
        ctx.kp_svd_rsvd(blur, 20, 10, 2, prec="f32", seed=2)
    torch.cuda.synchronize()
    ctx.close()
    print("done", flush=True)
    return 0


def profile_fft():
    """Workload of the rocprofv3 passes over the FFT blur products: at n = 512
    (Gaussian PSF on the full 1023 x 1023 offset grid, zero BC: M1 = M2 =
    2048) ten A X and ten A^T X, each call planning afresh (twiddles and the
    PSF spectrum: one row and one column pass over the PSF's rows)."""
    import torch

    import workloads as wl
    from paper_2410_00233_amd import api
    n = 512
    ctx = api.Context(0)
    P, cu, cv = wl.gaussian_psf(n)
    blur = api.Blur(P, cu, cv, n, on_device=True)
    X = torch.randn(n, n, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    for tr in (False, True):
        for _ in range(10):
            ctx.kp_blur_apply(blur, X, transpose=tr, Y=Y)
    torch.cuda.synchronize()
    ctx.close()
    print("done", flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=1.0,
                    help="seconds per timed run of the CPU dense product (3 runs per "
                         "precision and thread count)")
    ap.add_argument("--sb-solves", type=int, default=5)
    ap.add_argument("--sb-fft-solves", type=int, default=2,
                    help="timed solves per method and size in the FFT split Bregman section "
                         "(0 skips it)")
    ap.add_argument("--batched", type=int, default=64,
                    help="problems in the batched KP-SVD run (0 skips it)")
    ap.add_argument("--sb-batched", type=int, default=16,
                    help="solves in the batched split Bregman run (0 skips it)")
    ap.add_argument("--serve", type=int, default=32,
                    help="requests in the serving run (0 skips serving)")
    ap.add_argument("--serve-rate", type=float, default=200.0,
                    help="offered Poisson arrival rate of the serving run (requests/s)")
    ap.add_argument("--serve-sizes", type=str, default="128,256,512,1024")
    ap.add_argument("--serve-sweep", type=str, default="1,5,20",
                    help="comma-separated offered rates (req/s) run before the serving run, "
                         "--sweep-requests requests each")
    ap.add_argument("--sweep-requests", type=int, default=12)
    ap.add_argument("--profile-products", action="store_true",
                    help="only launch the products that the rocprofv3 counter passes measure "
                         "(a copy of known size for calibration, the n=512 FP32 / BF16 block "
                         "and FP32 matrix-vector products, the n=256 Kronecker apply and a few "
                         "CGLS iterations) and exit")
    ap.add_argument("--profile-fft", action="store_true",
                    help="run only the rocprofv3 workload of the FFT blur products and exit")
    ap.add_argument("--profile-qr", action="store_true",
                    help="only run two FP32 RSVDs at n=512 (the workload of the TSQR "
                         "counter pass) and exit")
    ap.add_argument("--gkb-block", type=int, default=16,
                    help="block size b of the timed block Golub-Kahan run (16: one MFMA "
                         "column block, so no padded columns; k_p = b ceil(40 / b))")
    ap.add_argument("--no-paper-pipeline", action="store_true",
                    help="skip the explicit-matrix run on the paper's n = 128 setting")
    args = ap.parse_args()
    if args.profile_products:
        sys.exit(profile_products())
    if args.profile_qr:
        sys.exit(profile_qr())
    if args.profile_fft:
        sys.exit(profile_fft())
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
    # the block form of Algorithm 1 on the same workload, k_p = b ceil(k_p / b)
    # (48 at b = 16): its products with B and B^T are block products of b
    # columns on the MFMA kernel (b = 16 fills one 16-column MFMA block; b = 20
    # would pad every product to 32 columns)
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

    log("BF16 + refinement RSVD; split-FP16 (f16x3) RSVD")
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
    # every product with R or R^T as three FP16 MFMA products of two-term splits
    ctx.kp_svd_rsvd(blur, k, p_rsvd, q, prec="f16x3", seed=2, factor_prec="f64")
    t3 = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        f3 = ctx.kp_svd_rsvd(blur, k, p_rsvd, q, prec="f16x3", seed=2, factor_prec="f64")
        torch.cuda.synchronize()
        t3.append(1e3 * (time.perf_counter() - ta))
    cases = []

    def case(name, blur_, f, method, seed, refine=0, prec="f32", gate=1e-5, pp=None):
        cases.append(dict(name=name, P=blur_.P, cu=blur_.cu, cv=blur_.cv, n=blur_.n,
                          method=method, seed=seed, k=k, p=pp if pp is not None else
                          (p_gkb if method == "gkb" else p_rsvd), q=q, refine=refine,
                          prec=prec, gate=gate, sigma=f.sigma[:k].copy(),
                          Ax=f.Ax[:k].cpu().numpy(), Ay=f.Ay[:k].cpu().numpy(),
                          breakdowns=list(getattr(f, "breakdowns", []))))

    case("gaussian_egkb_fp32", blur, fg, "gkb", 1)
    case("gaussian_rsvd_fp32", blur, fr, "rsvd", 2)
    case("gaussian_rsvd_bf16_refine", blur, fb, "rsvd", 2, refine=2, prec="bf16", gate=1e-4)
    case("gaussian_rsvd_f16x3", blur, f3, "rsvd", 2, prec="f16x3")
    b16 = prof16["block16"]
    avg16 = b16["ms"] / max(b16["launches"], 1)
    ach16 = (b16["flops"] / max(b16["launches"], 1)) / (avg16 * 1e-3) / 1e12
    bf_ms = float(np.median(tb))
    bf1_ms = float(np.median(tb1))
    sig_diff = float(np.abs(fb.sigma[:k] - fr.sigma[:k]).max() / fr.sigma[0])
    sig_diff1 = float(np.abs(fb1.sigma[:k] - fr.sigma[:k]).max() / fr.sigma[0])
    f3_ms = float(np.median(t3))
    sig_diff3 = float(np.abs(f3.sigma[:k] - fr.sigma[:k]).max() / fr.sigma[0])

    log("defocus disk r=8 at n=512 (FP32 EGKB and RSVD, BF16 + refinement RSVD)")
    Pd, cud, cvd = wl.disk_psf(n, 8.0)
    blur_d = api.Blur(Pd, cud, cvd, n, on_device=True)
    disk = {"workload": f"disk r=8 PSF on the full {2 * n - 1}x{2 * n - 1} offset grid, n={n}, "
                        "zero BC, rank 20; same step as the Gaussian",
            "rmat_nonzero_fractions_fp32": nonzero_fractions(Pd, cud, cvd, n)}
    for name, fn in (("egkb_fp32", lambda: ctx.kp_svd_gkb(blur_d, k, p_gkb, prec="f32", reorth=1,
                                                          seed=1, factor_prec="f64")),
                     ("rsvd_fp32", lambda: ctx.kp_svd_rsvd(blur_d, k, p_rsvd, q, prec="f32",
                                                           seed=2, factor_prec="f64")),
                     ("rsvd_bf16_refine", lambda: ctx.kp_svd_rsvd(blur_d, k, p_rsvd, q,
                                                                  prec="bf16", refine=2, seed=2,
                                                                  factor_prec="f64"))):
        fd = fn()
        td = []
        for _ in range(max(3, args.steps // 2)):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            fd = fn()
            torch.cuda.synchronize()
            td.append(1e3 * (time.perf_counter() - ta))
        fl = (f_gkb if name.startswith("egkb") else f_rsvd) + (f_ref if "refine" in name else 0)
        disk[name + "_ms"] = round(float(np.median(td)), 3)
        disk[name + "_tflops"] = round(fl / (np.median(td) * 1e-3) / 1e12, 3)
        case("disk_" + name, blur_d, fd, "gkb" if name.startswith("egkb") else "rsvd",
             1 if name.startswith("egkb") else 2, refine=2 if "refine" in name else 0,
             prec="bf16" if "bf16" in name else "f32", gate=1e-4 if "bf16" in name else 1e-5)
    log("speckle-like PSF at n=512 (accuracy of FP32 and BF16 + refinement RSVD)")
    Psp, cusp, cvsp = wl.speckle_psf(n, seed=wl.SEED_PSF + 2)
    blur_sp = api.Blur(Psp, cusp, cvsp, n, on_device=True)
    case("speckle_rsvd_fp32", blur_sp,
         ctx.kp_svd_rsvd(blur_sp, k, p_rsvd, q, prec="f32", seed=2, factor_prec="f64"), "rsvd", 2)
    case("speckle_rsvd_bf16_refine", blur_sp,
         ctx.kp_svd_rsvd(blur_sp, k, p_rsvd, q, prec="bf16", refine=2, seed=2, factor_prec="f64"),
         "rsvd", 2, refine=2, prec="bf16", gate=1e-4)
    case("speckle_rsvd_f16x3", blur_sp,
         ctx.kp_svd_rsvd(blur_sp, k, p_rsvd, q, prec="f16x3", seed=2, factor_prec="f64"),
         "rsvd", 2, prec="f16x3")

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
    log("split Bregman with A through FFTs at n=256, 512")
    sb_fft = bench_sb_fft(ctx, solves=args.sb_fft_solves) if args.sb_fft_solves > 0 else None

    blk = prof["block"]
    avg_blk_ms = blk["ms"] / max(blk["launches"], 1)
    flops_blk = blk["flops"] / max(blk["launches"], 1)
    achieved = flops_blk / (avg_blk_ms * 1e-3) / 1e12
    gv = prof["gemv"]
    avg_gv_ms = gv["ms"] / max(gv["launches"], 1)
    gemv_tflops = (gv["flops"] / max(gv["launches"], 1)) / (avg_gv_ms * 1e-3) / 1e12

    tune = ctx.kp_tune_report()
    v32 = next((t["variant"] for t in tune if t["op"] == "block32" and t["n"] == n and t["a"] == 4), None)
    v16 = next((t["variant"] for t in tune if t["op"] == "block16" and t["n"] == n
                and t["a"] == 2), None)   # element type KP_BF16
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
            "rsvd_f16x3_ms": round(f3_ms, 3),
            "rsvd_f16x3_tflops_algorithmic": round(f_rsvd / (f3_ms * 1e-3) / 1e12, 3),
            "rsvd_f16x3_speedup_vs_fp32": round(float(np.median(comp["rsvd_ms"])) / f3_ms, 3),
            "rsvd_f16x3_max_sigma_diff_vs_fp32_over_sigma1": sig_diff3,
        },
        "disk_r8_n512": disk,
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
        "sb_fft": sb_fft,
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
    if args.sb_batched > 0:
        log(f"batched split Bregman, {args.sb_batched} solves")
        line["sb_batched"] = bench_sb_batched(ctx, args.sb_batched)
    if args.serve > 0:
        sizes = tuple(int(v) for v in args.serve_sizes.split(","))
        srv = api.Server(ctx, slots=4)
        warmed = {}
        rates = [float(r) for r in args.serve_sweep.split(",") if r]
        row = ("requests", "p50_ms", "p99_ms", "solves_per_s", "mean_queue_ms", "mean_solve_ms",
               "per_n_p50_ms", "all_ok")
        sweep = {}
        for rate in rates:
            r_ = bench_serving(srv, args.sweep_requests, rate, sizes, warmed)
            sweep[str(rate)] = {k_: r_[k_] for k_ in row}
        serving = bench_serving(srv, args.serve, args.serve_rate, sizes, warmed)
        sweep[str(args.serve_rate)] = {k_: serving[k_] for k_ in row}
        srv.close()
        serving["workload"] = (
            f"Poisson stream at {args.serve_rate}/s (the configured rate), first {args.serve} "
            f"requests; n in {list(sizes)} weighted {[4, 3, 2, 1][:len(sizes)]}, 16 recurring "
            "PSFs (Gaussian/motion/disk) with rank-20 FP32 RSVD factors resident, iso/aniso 50/50, "
            "SB 50 outer iterations, CGLS tau 1e-4 (I_max 100), HBM-budget admission, 4 slots")
        serving["cold_factor_ms_p50_per_n"] = {
            str(nn): round(float(np.median([v for (pid, m), v in warmed.items() if m == nn])), 1)
            for nn in sorted({m for (_, m) in warmed})}
        line["serving"] = serving
        line["serving_sweep"] = {
            "workload": f"the same stream (same sizes, PSFs and images) offered at each rate, "
                        f"first {args.sweep_requests} requests per rate; the configured rate's "
                        f"row is the serving run ({args.serve} requests)",
            "rates": sweep}
    if not args.no_paper_pipeline:
        log("explicit-matrix pipeline at n=128 (reflexive BC)")
        line["paper_pipeline_n128"] = bench_paper_pipeline(ctx)
    line["autotune"] = ctx.kp_tune_report()
    if not args.no_cpu_baseline:
        log("CPU oracle leg: dense product timings, and the oracle's runs of the timed "
            "configurations for their accuracy")
        line["cpu_baseline"], line["accuracy"] = cpu_baseline_leg(n, k, p_rsvd, q, cases,
                                                                  args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
