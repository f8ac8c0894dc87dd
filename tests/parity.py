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


def cell_max_rel(a, b, rows=None):
    """Max over cells of max |a - b| / max |b| within the cell's row (its
    velocities or conservative values): a bound that an error confined to a
    few cells (walls, overset fringe) cannot hide in, as it can in a global
    norm.  rows: an optional mask of the cells to compare."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if rows is not None:
        a, b = a[rows], b[rows]
    a = a.reshape(len(a), -1)
    b = b.reshape(len(b), -1)
    if len(b) == 0:
        return 0.0
    m = np.abs(b).max(axis=1)
    d = np.abs(a - b).max(axis=1)
    return float((d / np.where(m > 0, m, 1.0)).max())


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
