"""Helpers for the GPU parity tests (no method arithmetic)."""
import numpy as np
import torch


def cuda(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dtype)


def host(t):
    return t.detach().cpu().numpy()


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
