"""Helpers of the GPU parity tests: run the HIP path and the oracle on the
same seeded inputs and compare element by element."""
import sys

import numpy as np
import torch

from oracle.oracle import Oracle
from paper_2604_09984_amd import ugks


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def max_rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    m = np.abs(b).max()
    return np.abs(a - b).max() / (m if m > 0 else 1.0)


def both(case, prec=ugks.F64, poses=None):
    o = Oracle(case)
    s = ugks.Solver(case, prec)
    if poses is not None:
        o.set_poses(poses)
        s.set_poses(poses)
    return o, s


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().to(torch.float64).cpu().numpy()
