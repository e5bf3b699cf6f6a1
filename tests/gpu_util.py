"""Helpers of the GPU tests: device arrays and relative norms."""

import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def banner(*args):
    """Names the case before a GPU step, flushed, so a run that dies is traceable."""
    print("[gpu-case]", *args, flush=True)
