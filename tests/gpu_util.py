"""Helpers shared by the GPU tests: moving arrays between numpy and the device."""
import numpy as np
import torch


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def solver(**kw):
    from paper_1309_7128_amd.solver import Solver

    return Solver(**kw)


def announce(*what):
    """Name the case before the device work starts (flushed, so a crash still shows it)."""
    print("CASE", *what, flush=True)
