"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys

import numpy as np


def announce(msg: str):
    """Name the case before GPU work so a failing run says which one it was."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def wrapped(d):
    return np.angle(np.exp(1j * np.asarray(d, dtype=np.float64)))


def cuda_ok() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
