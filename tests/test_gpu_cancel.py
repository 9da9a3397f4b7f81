"""Cancellation: kp_cancel on a context, kp_server_cancel on a request.

Every case forces the cancellation from the host (a flag the library checks
between launches); no kernel is interrupted. After a cancelled call the same
context gives the same bits as before.
"""
import threading
import time

import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu


def test_pending_cancel_stops_the_next_call_once(ctx):
    from paper_2410_00233_amd import api
    from paper_2410_00233_amd import _lib as L
    n = 48
    P, cu, cv = wl.gaussian_psf(n)
    blur = api.Blur(P, cu, cv, n)
    ref = ctx.kp_svd_gkb(blur, 6, 6, prec="f32", seed=3)
    for call in (lambda: ctx.kp_svd_gkb(blur, 6, 6, prec="f32", seed=3),
                 lambda: ctx.kp_svd_gkb(blur, 6, 6, prec="f32", seed=3, block=4),
                 lambda: ctx.kp_svd_rsvd(blur, 6, 6, 1, prec="f32", seed=3)):
        ctx.kp_cancel()
        with pytest.raises(api.KPError) as ei:
            call()
        assert ei.value.status == L.KP_E_CANCELLED
    # consumed: the next call runs, with the same bits as before
    again = ctx.kp_svd_gkb(blur, 6, 6, prec="f32", seed=3)
    assert np.array_equal(again.sigma[:6], ref.sigma[:6])
    f = api.Factors.from_arrays(ref.Ax[:6].cpu().numpy(), ref.Ay[:6].cpu().numpy())
    b = torch.rand(n, n, dtype=torch.float64, device="cuda")
    x0, _ = ctx.sb_solve_iso(f, b, 0.115, 0.0066, L_max=3, I_max=20)
    ctx.kp_cancel()
    with pytest.raises(api.KPError) as ei:
        ctx.sb_solve_iso(f, b, 0.115, 0.0066, L_max=3, I_max=20)
    assert ei.value.status == L.KP_E_CANCELLED
    x1, _ = ctx.sb_solve_iso(f, b, 0.115, 0.0066, L_max=3, I_max=20)
    assert torch.equal(x0, x1)


def test_cancel_from_another_thread():
    """A long Algorithm 1 run (n = 512, 60 Lanczos steps) cancelled while it
    runs: it stops early with KP_E_CANCELLED."""
    from paper_2410_00233_amd import api
    from paper_2410_00233_amd import _lib as L
    n = 512
    P, cu, cv = wl.gaussian_psf(n)
    blur = api.Blur(P, cu, cv, n, on_device=True)
    c = api.Context(0)
    try:
        c.kp_svd_gkb(blur, 4, 4, prec="f32", seed=1)          # warm (grids, workspace)
        torch.cuda.synchronize()
        timer = threading.Timer(0.03, c.kp_cancel)
        t0 = time.perf_counter()
        timer.start()
        with pytest.raises(api.KPError) as ei:
            c.kp_svd_gkb(blur, 20, 40, prec="f32", seed=1)
        el = time.perf_counter() - t0
        timer.join()
        assert ei.value.status == L.KP_E_CANCELLED
        torch.cuda.synchronize()
        full0 = time.perf_counter()
        c.kp_svd_gkb(blur, 20, 40, prec="f32", seed=1)
        torch.cuda.synchronize()
        full = time.perf_counter() - full0
        assert el < full
    finally:
        c.close()


def test_batched_cancel_marks_unstarted_problems():
    from paper_2410_00233_amd import api
    from paper_2410_00233_amd import _lib as L
    c = api.Context(0)
    try:
        probs = []
        for i, n in enumerate((32, 40, 48)):
            P, cu, cv = wl.gaussian_psf(n)
            probs.append((api.Blur(P, cu, cv, n), "rsvd",
                          api.Context.rsvd_opts(5, 3, 1, prec="f32", seed=i), 5))
        ref, _ = c.kp_svd_batched(probs)
        c.kp_cancel()
        with pytest.raises(api.KPError) as ei:
            c.kp_svd_batched(probs)
        assert ei.value.status == L.KP_E_CANCELLED
        again, st = c.kp_svd_batched(probs)
        assert st == [L.KP_OK] * 3
        for f, g in zip(ref, again):
            assert np.array_equal(f.sigma[:5], g.sigma[:5])
    finally:
        c.close()


def test_batched_sb_cancel_marks_unstarted_problems():
    from paper_2410_00233_amd import api
    from paper_2410_00233_amd import _lib as L
    c = api.Context(0)
    try:
        rng = np.random.default_rng(7)
        probs = []
        for i, (n, k) in enumerate(((32, 3), (40, 4), (48, 5))):
            f = api.Factors.from_arrays(rng.standard_normal((k, n, n)),
                                        rng.standard_normal((k, n, n)))
            b = torch.tensor(rng.standard_normal((n, n)), dtype=torch.float64, device="cuda")
            probs.append(dict(f=f, b=b, iso=i % 2 == 0, lam=0.115, beta=0.0066, L_max=3,
                              I_max=16))
        ref, _, st = c.sb_solve_batched(probs)
        assert st == [L.KP_OK] * 3
        c.kp_cancel()
        with pytest.raises(api.KPError) as ei:
            c.sb_solve_batched(probs)
        assert ei.value.status == L.KP_E_CANCELLED
        again, _, st = c.sb_solve_batched(probs)
        torch.cuda.synchronize()
        assert st == [L.KP_OK] * 3
        for x, y in zip(ref, again):
            assert torch.equal(x, y)
    finally:
        c.close()

def test_server_cancel_queued_and_running(ctx):
    from paper_2410_00233_amd import api
    from paper_2410_00233_amd import _lib as L
    srv = api.Server(ctx, slots=1)
    try:
        reqs = []
        for i, n in enumerate((384, 64, 64)):
            P, cu, cv = wl.gaussian_psf(n)
            x_true = wl.rectangles_image(n, seed=wl.SEED_IMAGE + i)
            b = wl.add_noise(wl.blur_zero_bc(P, cu, cv, x_true), 0.01, seed=wl.SEED_NOISE + i)
            bd = torch.tensor(b, dtype=torch.float64, device="cuda")
            reqs.append((api.Blur(P, cu, cv, n), bd, torch.empty_like(bd)))
        kw = dict(method="rsvd", k=10, p=5, q=2, prec="f32", seed=4, L_max=30, I_max=50)
        t0 = srv.submit(*reqs[0], psf_key=901, **kw)        # long: cold factors at n = 384
        t1 = srv.submit(*reqs[1], psf_key=902, **kw)        # queued behind it
        t2 = srv.submit(*reqs[2], psf_key=903, **kw)
        srv.cancel(t1)
        r1 = srv.wait(t1)
        assert r1["status"] == L.KP_E_CANCELLED and r1["solve_ms"] == 0.0
        time.sleep(0.05)
        srv.cancel(t0)
        r0 = srv.wait(t0)
        r2 = srv.wait(t2)
        assert r0["status"] in (L.KP_E_CANCELLED, L.KP_OK)   # OK only if it had finished
        assert r2["status"] == L.KP_OK
        # the request that ran after the cancellations equals the single calls
        P, cu, cv = wl.gaussian_psf(64)
        f = ctx.kp_svd_rsvd(reqs[2][0], 10, 5, 2, prec="f32", seed=4)
        x, _ = ctx.sb_solve_iso(f, reqs[2][1], 0.115, 0.0066, L_max=30, I_max=50,
                                tau_cgls=1e-4)
        assert torch.equal(x, reqs[2][2])
        with pytest.raises(api.KPError):
            srv.cancel(987654321)
    finally:
        srv.close()
