"""Helpers for the GPU parity tests: device transfer, error metrics, progress lines."""
import sys

import numpy as np
import torch

# Parity bars (relative, normalised by the oracle's norm over the compared set)
TOL_FP64 = 1e-12
TOL_FP32C = 1e-5


def step(msg: str) -> None:
    """Name the case before each GPU step (flushed, so a crash still shows it)."""
    print(f"[gpu-step] {msg}", file=sys.stderr, flush=True)


def dev(a, dtype=None, device="cuda:0"):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device)


def host(t):
    return t.detach().cpu().numpy()


def nrel(got, want):
    got, want = np.asarray(got), np.asarray(want)
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300))


def maxrel(got, want):
    got, want = np.asarray(got), np.asarray(want)
    return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300))


def special_q(qmax, n_axis=4):
    """Q = 0, points on each axis, and along the (1,1,1) diagonal."""
    out = [[0.0, 0.0, 0.0]]
    for k in range(3):
        for s in np.linspace(-qmax, qmax, n_axis):
            e = [0.0, 0.0, 0.0]
            e[k] = s
            out.append(e)
    for s in np.linspace(-qmax, qmax, n_axis):
        out.append([s, s, s])
    return np.array(out)
