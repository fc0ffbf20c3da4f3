"""Shared helpers for the GPU parity tests (not collected by pytest)."""
import sys

import numpy as np
import torch

DEV = torch.device("cuda:0")


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64 if not np.iscomplexobj(a) else np.complex128)
    b = np.asarray(b, dtype=np.float64 if not np.iscomplexobj(b) else np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def cosine(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.real(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b)))
