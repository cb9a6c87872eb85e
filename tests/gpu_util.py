"""Shared helpers of the GPU parity tests (marshalling only)."""
import numpy as np
import torch


def normwise(a, ref):
    """max |a - ref| / max |ref| (per component)."""
    s = np.abs(ref).max()
    return np.abs(a - ref).max() / (s if s > 0 else 1.0)


def gpu_smooth(ctx, prob, dtype, variant, sweeps, vx0=None, vy0=None, p=None, **opts):
    from paper_2509_19061_amd import api, fields
    dp = fields.DeviceProblem(prob, dtype)
    vx, vy = dp.velocity(vx0, vy0)
    pt = None if p is None else dp.field(p)
    api.smooth(ctx, dtype, dp.grid, vx, vy, pt, dp.eta_c, dp.eta_n, dp.fx, dp.fy, sweeps, variant, **opts)
    torch.cuda.synchronize()
    return dp.get_vx(vx), dp.get_vy(vy)


def as_dtype(a, dtype):
    """Round a float64 array through the storage type."""
    return torch.from_numpy(np.asarray(a, np.float64)).to(dtype).to(torch.float64).numpy()
