"""Helpers shared by the GPU parity tests (device transfer, tolerances)."""
import math

import numpy as np

U64 = 2.0 ** -53


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a, dtype="f64"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32 if dtype == "f32" else np.float64))
    return t.to(dev())


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def kappa2(a, b, c, n):
    """2-norm condition number from the closed-form spectrum (t1 t-1 > 0), else
    the dominance bound -- the same quantity the tolerances are derived from."""
    if a * c > 0:
        s = math.copysign(math.sqrt(a * c), c)
        k = np.arange(1, n + 1)
        lam = b + 2 * s * np.cos(k * math.pi / (n + 1))
        return float(np.max(np.abs(lam)) / np.min(np.abs(lam)))
    off = abs(a) + abs(c)
    return (abs(b) + off) / (abs(b) - off) if abs(b) > off else float("inf")


def tol_f64(a, b, c, n):
    """1e-12, or 4 u cond(T) for ill-conditioned systems where no double
    algorithm can do better."""
    return max(1e-12, 4 * U64 * kappa2(a, b, c, n))


def tol_f32(a, b, c, n):
    """Plain float: 2e-5 at dominance ratio >= 1.25 (cond <= 9)."""
    return max(2e-5, 8 * 2.0 ** -24 * kappa2(a, b, c, n))
