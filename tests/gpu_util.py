"""Helpers for the GPU tests: device placement and oracle comparisons."""
import sys

import numpy as np
import torch


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
