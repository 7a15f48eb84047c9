"""Helpers for the GPU parity tests: device setup and the parity metric."""
import sys

import numpy as np


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def parity_errors(y_gpu, y_ref, floor=1e-12):
    """Relative error where |y_ref| >= floor, absolute error elsewhere (the parity gate)."""
    big = np.abs(y_ref) >= floor
    rel = np.zeros_like(y_ref)
    rel[big] = np.abs(y_gpu[big] - y_ref[big]) / np.abs(y_ref[big])
    absd = np.where(big, 0.0, np.abs(y_gpu - y_ref))
    return rel, absd, big


def assert_parity(y_gpu, y_ref, rel_tol=1e-4, floor=1e-12, what=""):
    rel, absd, big = parity_errors(y_gpu, y_ref, floor)
    worst = float(rel.max()) if rel.size else 0.0
    worst_abs = float(absd.max()) if absd.size else 0.0
    log(f"parity {what}: max rel {worst:.3e} (bar {rel_tol:g}), max abs below floor {worst_abs:.3e}")
    assert worst <= rel_tol, (what, worst)
    assert worst_abs <= floor, (what, worst_abs)
