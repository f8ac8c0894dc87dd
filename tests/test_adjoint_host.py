"""Host bookkeeping of the differentiable driver (CPU): the block and side
of every face in the library's face numbering, and the wall weights' sides,
checked against the oracle's structured face ids."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2604_09984_amd import adjoint, workloads as wl


@pytest.mark.parametrize("case", [wl.cavity(5, 6), wl.cylinder(ni=12, nj=5, nvx=8),
                                  wl.overset_cylinder(ni_bg=16, nb=12, njb=6, nv=6), wl.sod_1d(12, 9)],
                         ids=["cavity", "cylinder", "overset", "sod1d"])
def test_face_blocks_match_oracle_face_ids(case):
    o = Oracle(case)
    blk, dr, fi, fj = o.face_ids()
    idx = o.product_face_index()
    fb, fs = adjoint.face_blocks(case)
    assert len(fb) == len(fs) >= o.nface
    assert np.array_equal(fb[idx], blk)
    for f in range(o.nface):
        B = case.blocks[blk[f]]
        if dr[f] == 0:
            want = 0 if fi[f] == 0 else (1 if fi[f] == B.ni else -1)
        else:
            want = 2 if fj[f] == 0 else (3 if fj[f] == B.nj else -1)
        assert fs[idx[f]] == want
