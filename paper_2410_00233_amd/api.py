"""Python binding over the C ABI (include/kpsb.h), same entry-point names.

Argument marshalling only: inputs are NumPy arrays (host) or torch tensors
(device); torch provides device memory and the current stream. Every step of
the computation runs in libkpsb.so. If the library is missing this raises: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L

PREC = {"f64": L.KP_F64, "f32": L.KP_F32, "bf16": L.KP_BF16, "f16": L.KP_F16,
        "f16x3": L.KP_F16X3}


class KPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


BC = {"zero": L.KP_BC_ZERO, "reflexive": L.KP_BC_REFLEXIVE, "periodic": L.KP_BC_PERIODIC}


class Blur:
    """PSF P (pu x pv, u vertical) with centre (cu, cv) acting on n x n images
    with boundary conditions bc ("zero", "reflexive" or "periodic").

    P is a NumPy array (host) or, with on_device=True, copied once into a device
    tensor so that calls read it from HBM."""

    def __init__(self, P, cu, cv, n, on_device=False, bc="zero", compact=False):
        self.P = np.ascontiguousarray(P, dtype=np.float64)
        self.cu, self.cv, self.n = int(cu), int(cv), int(n)
        self.bc = bc
        self.compact = bool(compact)
        self.on_device = bool(on_device)
        if on_device:
            torch = _torch()
            self.Pd = torch.tensor(self.P, dtype=torch.float64, device="cuda")
            ptr = C.cast(C.c_void_p(self.Pd.data_ptr()), C.POINTER(C.c_double))
        else:
            ptr = self.P.ctypes.data_as(C.POINTER(C.c_double))
        self.s = L.kp_blur(self.n, ptr, self.P.shape[0], self.P.shape[1], self.cu, self.cv,
                           int(on_device), BC[bc], int(compact))

    def with_bc(self, bc=None, compact=None):
        """The same PSF (sharing its memory) with other boundary conditions
        and/or another compaction setting."""
        other = Blur.__new__(Blur)
        other.__dict__.update(self.__dict__)
        other.bc = self.bc if bc is None else bc
        other.compact = self.compact if compact is None else bool(compact)
        other.s = L.kp_blur(self.s.n, self.s.psf, self.s.pu, self.s.pv, self.s.cu, self.s.cv,
                            self.s.psf_on_device, BC[other.bc], int(other.compact))
        return other


class Factors:
    """Device Kronecker factors (k x n x n each) plus host sigma."""

    def __init__(self, n, k_cap, prec="f64", device="cuda"):
        torch = _torch()
        dt = torch.float64 if prec == "f64" else torch.float32
        self.n, self.k_cap, self.prec = n, k_cap, prec
        self.Ax = torch.zeros((k_cap, n, n), dtype=dt, device=device)
        self.Ay = torch.zeros((k_cap, n, n), dtype=dt, device=device)
        self.sigma = np.zeros(k_cap)
        self.diag = L.kp_diag()
        self.diag.cap = 0
        self.s = L.kp_factors(n, k_cap, 0, self.sigma.ctypes.data_as(C.POINTER(C.c_double)),
                              self.Ax.data_ptr(), self.Ay.data_ptr(), PREC[prec],
                              C.pointer(self.diag))
        self.status = L.KP_OK

    @property
    def k(self):
        return self.s.k

    @classmethod
    def from_arrays(cls, Ax, Ay, sigma=None):
        """Device FP64 factors from host arrays (k x n x n each)."""
        torch = _torch()
        k, n, _ = Ax.shape
        f = cls(n, k, "f64")
        f.Ax.copy_(torch.as_tensor(np.ascontiguousarray(Ax, dtype=np.float64)))
        f.Ay.copy_(torch.as_tensor(np.ascontiguousarray(Ay, dtype=np.float64)))
        if sigma is not None:
            f.sigma[:k] = sigma
        f.s.k = k
        return f


class Context:
    def __init__(self, device=0, hbm_budget=0):
        self.lib = L.load()
        h = C.c_void_p()
        st = self.lib.kp_ctx_create(int(device), C.c_size_t(hbm_budget), C.byref(h))
        if st != L.KP_OK:
            raise KPError(st, "kp_ctx_create failed")
        self.h = h

    def close(self):
        if self.h:
            self.lib.kp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=(L.KP_OK,)):
        if st not in allow:
            raise KPError(st, self.lib.kp_last_error(self.h).decode())
        return st

    def kp_cancel(self):
        """Stops the call in progress on this context (callable from any thread)."""
        self._check(self.lib.kp_cancel(self.h))

    def kp_ctx_workspace(self):
        """Bytes of device workspace the context holds."""
        held = C.c_size_t()
        self._check(self.lib.kp_ctx_workspace(self.h, C.byref(held)))
        return int(held.value)

    # ---- autotuner ------------------------------------------------------------
    def kp_tune_report(self):
        """Chosen launch variants and measured candidate costs (list of dicts)."""
        import json
        buf = C.create_string_buffer(1 << 16)
        self._check(self.lib.kp_tune_report(buf, len(buf)))
        return json.loads(buf.value.decode())

    # ---- tracing ------------------------------------------------------------
    def kp_prof_enable(self, enable=True):
        self._check(self.lib.kp_prof_enable(self.h, int(enable)))

    def kp_prof_read(self, reset=True):
        """Per class ("block", "gemv", "apply"): summed ms, launches, flops."""
        pr = L.kp_prof()
        self._check(self.lib.kp_prof_read(self.h, C.byref(pr), int(reset)))
        return {name: dict(ms=pr.ms[i], launches=pr.launches[i], flops=pr.flops[i])
                for i, name in enumerate(("block", "gemv", "apply", "block16"))}

    # ---- entry points (names follow the C ABI) ----------------------------
    def kp_rmat_apply(self, blur: Blur, X, transpose=False, prec="f32", Y=None):
        """X: device tensor (n^2,) or (ncols, n^2) -- i.e. an n^2 x ncols
        column-major block; Y has the same shape."""
        torch = _torch()
        assert X.is_contiguous() and X.shape[-1] == blur.n * blur.n
        ncols = 1 if X.dim() == 1 else X.shape[0]
        if Y is None:
            Y = torch.empty_like(X)
        self._check(self.lib.kp_rmat_apply(self.h, C.byref(blur.s), int(transpose), PREC[prec],
                                           ncols, _ptr(X), _ptr(Y), _stream()))
        return Y

    def kp_rmat_apply_noalloc(self, blur: Blur, X, transpose=False, prec="f32", Y=None):
        """kp_rmat_apply with every workspace buffer taken from the library's static
        device scratch (no device allocation by the library)."""
        torch = _torch()
        assert X.is_contiguous() and X.shape[-1] == blur.n * blur.n
        ncols = 1 if X.dim() == 1 else X.shape[0]
        if Y is None:
            Y = torch.empty_like(X)
        self._check(self.lib.kp_rmat_apply_noalloc(self.h, C.byref(blur.s), int(transpose),
                                                   PREC[prec], ncols, _ptr(X), _ptr(Y),
                                                   _stream()))
        return Y

    def kp_svd_gkb(self, blur: Blur, k, p, *, k_min=0, auto_k=False, tau=0.0,
                   literal_init=False, reorth=1, prec="f32", seed=0, y0=None, bd_rel=0.0,
                   factor_prec="f64", k_cap=None, bases=False, stored=None, block=0):
        """stored=(n, R): the KP-SVD of a stored R (device tensor N x N, the
        element type given by prec) instead of the blur's generated R.
        block=b >= 1: block Golub-Kahan bidiagonalization with b start vectors
        (y0 then an N x b array); breakdowns are reported as ("u" | "v", m)."""
        torch = _torch()
        n = blur.n if stored is None else stored[0]
        f = Factors(n, k_cap or k, factor_prec)
        y0a = None
        if y0 is not None:
            y0a = np.asarray(y0, dtype=np.float64)
            y0a = np.ascontiguousarray(y0a.T if y0a.ndim == 2 else y0a)   # columns contiguous
        o = L.kp_gkb_opts(k, p, k_min, int(auto_k), tau, int(literal_init), reorth, PREC[prec],
                          seed, None if y0a is None else y0a.ctypes.data_as(C.POINTER(C.c_double)),
                          bd_rel, block)
        cap = k + p + 2
        alpha = np.zeros(cap)
        t = np.zeros(cap)
        f.diag.cap = cap
        f.diag.alpha = alpha.ctypes.data_as(C.POINTER(C.c_double))
        f.diag.t = t.ctypes.data_as(C.POINTER(C.c_double))
        S = Q = None
        if block >= 1:
            nu_cols = (-(-(k + p) // block) + 1) * block
            nv_cols = nu_cols - block
        else:
            nu_cols, nv_cols = k + p + 1, k + p
        if bases:
            dt = torch.float32 if prec == "f32" else torch.float64
            S = torch.zeros((nu_cols, n * n), dtype=dt, device="cuda")
            Q = torch.zeros((nv_cols, n * n), dtype=dt, device="cuda")
            f.diag.basis_u = S.data_ptr()
            f.diag.basis_v = Q.data_ptr()
        if stored is None:
            st = self.lib.kp_svd_gkb(self.h, C.byref(blur.s), C.byref(o), C.byref(f.s), _stream())
        else:
            st = self.lib.kp_svd_gkb_stored(self.h, n, _ptr(stored[1]), C.byref(o), C.byref(f.s),
                                            _stream())
        st = self._check(st, allow=(L.KP_OK, L.KP_W_BREAKDOWN))
        f.status = st
        kp = f.diag.kp
        f.alpha = alpha[:kp].copy()
        f.t = t[:kp + 1].copy()
        names = ("u", "v") if block >= 1 else ("s", "q")
        f.breakdowns = [(names[f.diag.break_side[i]], f.diag.break_step[i])
                        for i in range(min(f.diag.nbreak, 128))]
        f.ms = f.diag.ms_total
        if bases:
            f.S = S[:kp + block] if block >= 1 else S[:kp + 1]
            f.Q = Q[:kp]
        return f

    @staticmethod
    def gkb_opts(k, p, *, k_min=0, auto_k=False, tau=0.0, literal_init=False, reorth=1,
                 prec="f32", seed=0, y0=None, bd_rel=0.0, block=0):
        """kp_gkb_opts; a host start vector (block: n^2 x b column-major array)
        y0 must outlive the call using it."""
        ptr = None if y0 is None else y0.ctypes.data_as(C.POINTER(C.c_double))
        return L.kp_gkb_opts(k, p, k_min, int(auto_k), tau, int(literal_init), reorth,
                             PREC[prec], seed, ptr, bd_rel, block)

    @staticmethod
    def rsvd_opts(k, p, q, *, prec="f32", refine=False, seed=0, F=None):
        ptr = None if F is None else F.ctypes.data_as(C.POINTER(C.c_double))
        return L.kp_rsvd_opts(k, p, q, PREC[prec], int(refine), seed, ptr)

    def kp_svd_batched(self, problems, nworkers=0, factor_prec="f64"):
        """problems: list of (Blur, "gkb" | "rsvd", opts struct, k_cap). Returns
        (list of Factors, list of per-problem statuses)."""
        m = len(problems)
        blurs = (L.kp_blur * m)(*[p[0].s for p in problems])
        meth = (C.c_int32 * m)(*[L.KP_METHOD_GKB if p[1] == "gkb" else L.KP_METHOD_RSVD
                                 for p in problems])
        opts = [p[2] for p in problems]
        optp = (C.c_void_p * m)(*[C.cast(C.pointer(o), C.c_void_p) for o in opts])
        facs = [Factors(p[0].n, p[3], factor_prec) for p in problems]
        outs = (L.kp_factors * m)(*[f.s for f in facs])
        status = (C.c_int * m)()
        self._check(self.lib.kp_svd_batched(self.h, m, blurs, meth, optp, outs, status,
                                            int(nworkers), _stream()),
                    allow=(L.KP_OK, L.KP_W_BREAKDOWN))
        for i, f in enumerate(facs):
            f.s.k = outs[i].k
            f.status = status[i]
        return facs, list(status)

    def kp_svd_rsvd(self, blur: Blur, k, p, q, *, prec="f32", refine=False, seed=0, F=None,
                    factor_prec="f64", k_cap=None, bases=False, stored=None):
        """stored=(n, R) as in kp_svd_gkb."""
        torch = _torch()
        n = blur.n if stored is None else stored[0]
        f = Factors(n, k_cap or k, factor_prec)
        Fa = None if F is None else np.asfortranarray(F, dtype=np.float64)
        o = L.kp_rsvd_opts(k, p, q, PREC[prec], int(refine), seed,
                           None if Fa is None else Fa.ctypes.data_as(C.POINTER(C.c_double)))
        Y = None
        if bases:
            dt = torch.float64 if prec == "f64" else torch.float32
            Y = torch.zeros((k + p, n * n), dtype=dt, device="cuda")
            f.diag.basis_u = Y.data_ptr()
        if stored is None:
            st = self.lib.kp_svd_rsvd(self.h, C.byref(blur.s), C.byref(o), C.byref(f.s), _stream())
        else:
            st = self.lib.kp_svd_rsvd_stored(self.h, n, _ptr(stored[1]), C.byref(o), C.byref(f.s),
                                             _stream())
        f.status = self._check(st)
        f.ms = f.diag.ms_total
        if bases:
            f.Y = Y
        return f

    def kp_blur_matrix(self, blur: Blur, bc=None, prec="f64", A=None):
        """Explicit blur matrix (device N x N) with the blur's boundary
        conditions (or bc, if given)."""
        torch = _torch()
        if bc is not None and bc != blur.bc:
            blur = blur.with_bc(bc)
        N = blur.n * blur.n
        if A is None:
            A = torch.empty((N, N), dtype=torch.float64 if prec == "f64" else torch.float32,
                            device="cuda")
        self._check(self.lib.kp_blur_matrix(self.h, C.byref(blur.s), PREC[prec], _ptr(A),
                                            _stream()))
        return A

    def kp_rmat_reorder(self, n, A, R=None):
        """R(A) from a stored blur matrix A (device tensor N x N, FP32 or FP64)."""
        torch = _torch()
        if R is None:
            R = torch.empty_like(A)
        prec = "f64" if A.dtype == torch.float64 else "f32"
        self._check(self.lib.kp_rmat_reorder(self.h, int(n), PREC[prec], _ptr(A), _ptr(R),
                                             _stream()))
        return R

    def kp_rmat_apply_stored(self, n, R, X, transpose=False, Y=None):
        torch = _torch()
        if Y is None:
            Y = torch.empty_like(X)
        prec = "f64" if R.dtype == torch.float64 else "f32"
        ncols = 1 if X.dim() == 1 else X.shape[0]
        self._check(self.lib.kp_rmat_apply_stored(self.h, int(n), PREC[prec], _ptr(R),
                                                  int(transpose), ncols, _ptr(X), _ptr(Y),
                                                  _stream()))
        return Y

    def sb_solve_aniso_direct(self, n, A, b, lam, beta, L_max=50, I_max=100, tau_sb=0.0,
                              tau_cgls=0.0, x=None):
        return self._sb_direct(self.lib.sb_solve_aniso_direct, n, A, b, lam, beta, L_max, I_max,
                               tau_sb, tau_cgls, x)

    def sb_solve_iso_direct(self, n, A, b, lam, beta, L_max=50, I_max=100, tau_sb=0.0,
                            tau_cgls=0.0, x=None):
        return self._sb_direct(self.lib.sb_solve_iso_direct, n, A, b, lam, beta, L_max, I_max,
                               tau_sb, tau_cgls, x)

    def _sb_direct(self, fn, n, A, b, lam, beta, L_max, I_max, tau_sb, tau_cgls, x):
        torch = _torch()
        if x is None:
            x = torch.empty_like(b)
        o = L.sb_opts(lam, beta, L_max, I_max, tau_sb, tau_cgls)
        st = L.sb_stats()
        self._check(fn(self.h, int(n), _ptr(A), _ptr(b), C.byref(o), _ptr(x), C.byref(st),
                       _stream()))
        return x, dict(l_end=st.l_end, iota_total=st.iota_total, rc_sb=st.rc_sb,
                       graph_replays=st.graph_replays)

    def kp_blur_apply(self, blur: Blur, X, transpose=False, Y=None):
        """A X or A^T X (device n x n FP64 images) through FFTs of the image
        extended by the blur's boundary conditions."""
        torch = _torch()
        if Y is None:
            Y = torch.empty_like(X)
        self._check(self.lib.kp_blur_apply(self.h, C.byref(blur.s), int(transpose), _ptr(X),
                                           _ptr(Y), _stream()))
        return Y

    def sb_solve_aniso_fft(self, blur: Blur, b, lam, beta, L_max=50, I_max=100, tau_sb=0.0,
                           tau_cgls=0.0, x=None):
        return self._sb_fft(self.lib.sb_solve_aniso_fft, blur, b, lam, beta, L_max, I_max,
                            tau_sb, tau_cgls, x)

    def sb_solve_iso_fft(self, blur: Blur, b, lam, beta, L_max=50, I_max=100, tau_sb=0.0,
                         tau_cgls=0.0, x=None):
        return self._sb_fft(self.lib.sb_solve_iso_fft, blur, b, lam, beta, L_max, I_max,
                            tau_sb, tau_cgls, x)

    def _sb_fft(self, fn, blur, b, lam, beta, L_max, I_max, tau_sb, tau_cgls, x):
        torch = _torch()
        if x is None:
            x = torch.empty_like(b)
        o = L.sb_opts(lam, beta, L_max, I_max, tau_sb, tau_cgls)
        st = L.sb_stats()
        self._check(fn(self.h, C.byref(blur.s), _ptr(b), C.byref(o), _ptr(x), C.byref(st),
                       _stream()))
        return x, dict(l_end=st.l_end, iota_total=st.iota_total, rc_sb=st.rc_sb,
                       graph_replays=st.graph_replays)

    def kp_apply(self, f: Factors, X, transpose=False, Y=None):
        torch = _torch()
        if Y is None:
            Y = torch.empty_like(X)
        self._check(self.lib.kp_apply(self.h, C.byref(f.s), int(transpose), _ptr(X), _ptr(Y),
                                      _stream()))
        return Y

    def _sb(self, fn, f, b, lam, beta, L_max, I_max, tau_sb, tau_cgls, x):
        torch = _torch()
        if x is None:
            x = torch.empty_like(b)
        o = L.sb_opts(lam, beta, L_max, I_max, tau_sb, tau_cgls)
        st = L.sb_stats()
        self._check(fn(self.h, C.byref(f.s), _ptr(b), C.byref(o), _ptr(x), C.byref(st),
                       _stream()))
        return x, dict(l_end=st.l_end, iota_total=st.iota_total, rc_sb=st.rc_sb,
                       graph_replays=st.graph_replays)

    def sb_solve_aniso(self, f, b, lam, beta, L_max=50, I_max=100, tau_sb=0.0, tau_cgls=0.0,
                       x=None):
        return self._sb(self.lib.sb_solve_aniso, f, b, lam, beta, L_max, I_max, tau_sb,
                        tau_cgls, x)

    def sb_solve_iso(self, f, b, lam, beta, L_max=50, I_max=100, tau_sb=0.0, tau_cgls=0.0,
                     x=None):
        return self._sb(self.lib.sb_solve_iso, f, b, lam, beta, L_max, I_max, tau_sb,
                        tau_cgls, x)

    def sb_solve_batched(self, problems, nworkers=0):
        """problems: list of dicts with keys f (Factors), b (device image),
        iso (bool), lam, beta and optionally L_max, I_max, tau_sb, tau_cgls, x.
        Returns (list of x, list of stats dicts, list of statuses)."""
        torch = _torch()
        m = len(problems)
        xs = [p.get("x") if p.get("x") is not None else torch.empty_like(p["b"])
              for p in problems]
        arr = (L.sb_problem * m)()
        for i, p in enumerate(problems):
            arr[i].f = C.pointer(p["f"].s)
            arr[i].b = _ptr(p["b"])
            arr[i].x = _ptr(xs[i])
            arr[i].opts = L.sb_opts(p["lam"], p["beta"], p.get("L_max", 50), p.get("I_max", 100),
                                    p.get("tau_sb", 0.0), p.get("tau_cgls", 0.0))
            arr[i].iso = int(bool(p["iso"]))
        st = (L.sb_stats * m)()
        status = (C.c_int * m)()
        self._check(self.lib.sb_solve_batched(self.h, m, arr, st, status, int(nworkers),
                                              _stream()),
                    allow=(L.KP_OK, L.KP_W_BREAKDOWN))
        stats = [dict(l_end=s.l_end, iota_total=s.iota_total, rc_sb=s.rc_sb,
                      graph_replays=s.graph_replays) for s in st]
        return xs, stats, list(status)


class Server:
    """The request server (kp_server_*): submit() is non-blocking, wait()
    returns the per-request result. Device images b and x, and host PSF arrays,
    must stay alive until wait() has returned for their ticket."""

    def __init__(self, ctx: Context, slots=0, hbm_budget=0, max_pending=0, cache_entries=0):
        self.ctx, self.lib = ctx, ctx.lib
        cfg = L.kp_server_cfg(int(slots), C.c_size_t(hbm_budget), int(max_pending),
                              int(cache_entries))
        h = C.c_void_p()
        ctx._check(self.lib.kp_server_create(ctx.h, C.byref(cfg), C.byref(h)))
        self.h = h
        self._keep = {}

    @staticmethod
    def request(blur: Blur, b=None, x=None, *, psf_key=0, method="rsvd", k=20, p=10, q=2,
                prec="f32", refine=False, seed=0, k_cap=None, iso=True, lam=0.115,
                beta=0.0066, L_max=50, I_max=100, tau_sb=0.0, tau_cgls=1e-4, gkb=None,
                rsvd=None):
        """The kp_request of a solve (b, x: device images, or None for a size query)."""
        req = L.kp_request()
        req.psf_key = psf_key
        req.blur = blur.s
        req.method = L.KP_METHOD_GKB if method == "gkb" else L.KP_METHOD_RSVD
        req.gkb = gkb if gkb is not None else Context.gkb_opts(k, p, prec=prec, seed=seed)
        req.rsvd = rsvd if rsvd is not None else Context.rsvd_opts(k, p, q, prec=prec,
                                                                  refine=refine, seed=seed)
        req.k_cap = k_cap or k
        req.iso = int(iso)
        req.sb = L.sb_opts(lam, beta, L_max, I_max, tau_sb, tau_cgls)
        req.b = b.data_ptr() if b is not None else None
        req.x = x.data_ptr() if x is not None else None
        return req

    @staticmethod
    def footprint(blur: Blur, **kw):
        """kp_request_footprint: (solve workspace, KP-SVD workspace, factor set) bytes."""
        out = (C.c_size_t * 3)()
        st = L.load().kp_request_footprint(C.byref(Server.request(blur, **kw)), out)
        if st != L.KP_OK:
            raise KPError(st, "kp_request_footprint failed")
        return tuple(int(v) for v in out)

    def submit(self, blur: Blur, b, x, **kw):
        req = Server.request(blur, b, x, **kw)
        # the server's streams read b: it must be complete before submit
        _torch().cuda.current_stream().synchronize()
        t = C.c_uint64()
        st = self.lib.kp_server_submit(self.h, C.byref(req), C.byref(t))
        if st != L.KP_OK:
            raise KPError(st, self.lib.kp_last_error(self.ctx.h).decode())
        self._keep[t.value] = (blur, b, x)
        return t.value

    def cancel(self, ticket):
        """kp_server_cancel: the request completes with KP_E_CANCELLED unless it
        has finished already; collect it with wait() as usual."""
        st = self.lib.kp_server_cancel(self.h, C.c_uint64(ticket))
        if st != L.KP_OK:
            raise KPError(st, self.lib.kp_last_error(self.ctx.h).decode())

    def wait(self, ticket, timeout=-1.0):
        r = L.kp_result()
        st = self.lib.kp_server_wait(self.h, C.c_uint64(ticket), float(timeout), C.byref(r))
        if st == L.KP_E_TIMEOUT:
            return None
        if st != L.KP_OK:
            raise KPError(st, self.lib.kp_last_error(self.ctx.h).decode())
        self._keep.pop(ticket, None)
        return dict(status=r.status, l_end=r.stats.l_end, iota_total=r.stats.iota_total,
                    rc_sb=r.stats.rc_sb, k=r.k, cache_hit=bool(r.cache_hit),
                    queue_ms=r.queue_ms, factor_ms=r.factor_ms, solve_ms=r.solve_ms,
                    total_ms=r.total_ms, msg=r.msg.decode())

    def stats(self):
        out = (C.c_int64 * 8)()
        self.lib.kp_server_stats(self.h, out)
        names = ("submitted", "completed", "hits", "misses", "evictions", "bypasses",
                 "peak_running", "resident")
        return dict(zip(names, list(out)))

    def close(self):
        if self.h:
            self.lib.kp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
