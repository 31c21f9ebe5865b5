"""Tolerance helpers for GPU-vs-oracle parity.

A weighted sum y = sum_k w_k v_k evaluated in binary32 is accurate relative to
sum_k |w_k| |v_k| (the magnitude), not to |y|: with signed inputs y can cancel to ~0.
Parity of floating-point stages is therefore checked elementwise as
    |y - r| <= tol * mag + floor,
with mag the oracle's magnitude of the same computation, and the normwise relative error is
reported beside it.
"""
import numpy as np
import torch


def to_np(t):
    if isinstance(t, torch.Tensor):
        return t.detach().float().cpu().double().numpy() if t.dtype == torch.bfloat16 else t.detach().cpu().double().numpy()
    return np.asarray(t, dtype=np.float64)


def assert_mag_close(y, r, mag, tol, floor=1e-30, what=""):
    y, r, mag = to_np(y), to_np(r), to_np(mag)
    err = np.abs(y - r)
    bound = tol * mag + floor
    bad = err > bound
    if bad.any():
        i = np.argmax(err / bound)
        raise AssertionError(f"{what}: {bad.sum()} / {bad.size} elements exceed tol {tol}; worst "
                             f"err {err.flat[i]:.3e} at mag {mag.flat[i]:.3e} (y={y.flat[i]:.6e}, "
                             f"r={r.flat[i]:.6e}); normwise {rel_norm(y, r):.3e}")


def rel_norm(y, r):
    y, r = to_np(y), to_np(r)
    return float(np.linalg.norm(y - r) / max(np.linalg.norm(r), 1e-300))

