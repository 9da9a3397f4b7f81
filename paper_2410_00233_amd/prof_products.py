"""Workload for hardware-counter passes over the generated-tile products.

Run under ``rocprofv3 --pmc <counters> -- python3 -m paper_2410_00233_amd.prof_products``
from the repository root. In one process it launches:

* a plain copy of 256 MiB FP32 (``torch.mul(x, 1.0, out=y)``: reads 256 MiB and
  writes 256 MiB), the calibration kernel for FETCH_SIZE / WRITE_SIZE;
* through the library at n = 512 on the rotated Gaussian PSF (PSF in HBM): the
  FP32 block product R X with 30 columns, the FP32 matrix-vector product R x
  and the BF16 block product R X with 30 columns. The first launches of each
  block kernel are the autotuner's samples; the product launch follows them.
"""
import sys

import torch

import workloads as wl
from paper_2410_00233_amd import api


def main():
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
    torch.cuda.synchronize()
    print("done", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
