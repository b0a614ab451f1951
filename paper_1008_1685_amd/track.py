"""Test electrons in a given plane wave (pic_track): the single-particle
tests of the paper's Section 3 on the GPU.  Argument marshalling only."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N

SCHEMES = {"leapfrog": N.PIC_TRACK_LEAPFROG, "rk4": N.PIC_TRACK_RK4}
RR = {"off": N.PIC_RR_OFF, "reduced": N.PIC_RR_REDUCED, "full": N.PIC_RR_FULL}


def track(x, u, a_y, a_z=0.0, psi=0.0, dt=0.01, steps=1, t0=0.0, scheme="leapfrog", rr="reduced",
          precision="fp64", lambda_um=0.8, device="cuda"):
    """Advance electrons at positions x (n,) with momenta u (n, 3) by
    ``steps`` steps; returns (x, u) as float64 numpy arrays.  For the
    leapfrog scheme u is the half-step momentum u^{-1/2}."""
    import torch

    lib = N.load()
    x = torch.as_tensor(np.asarray(x, np.float64).reshape(-1), device=device).contiguous()
    u = np.asarray(u, np.float64).reshape(-1, 3)
    cols = [torch.as_tensor(u[:, k].copy(), device=device).contiguous() for k in range(3)]
    w = N.PicWave(float(a_y), float(a_z), float(psi))
    prec = N.PIC_FP32 if precision == "fp32" else N.PIC_FP64
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    N.check(lib.pic_track(C.byref(w), SCHEMES[scheme], RR[rr], prec, float(lambda_um), float(dt),
                          float(t0), int(steps), int(x.numel()), C.c_void_p(x.data_ptr()),
                          *[C.c_void_p(c.data_ptr()) for c in cols], st), "pic_track")
    torch.cuda.synchronize()
    return x.cpu().numpy(), np.stack([c.cpu().numpy() for c in cols], 1)
