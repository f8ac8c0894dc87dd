"""ugks_flux_noalloc (the flux with its scratch in the library's static device
array, for callers that cannot allocate) through the C ABI against
ugks_flux: bit-identical divergence, face macro flux and wall output on two
calls in a row, the second on a smaller case, and a case above the array's
size rejected before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2604_09984_amd import ugks, workloads as wl
from tests.parity import dev, host, say

pytestmark = pytest.mark.gpu


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _both(case, prec):
    s = ugks.Solver(case, prec)
    h, b, W = wl.synthetic_f(case, amp=0.02)
    hd, bd, Wd = dev(h, s.dtype), dev(b, s.dtype), dev(W)
    qd = s.heatflux(hd, bd, Wd)
    dts, _ = s.timesteps()
    Dh, Db, F, wall = s.flux(dts, hd, bd, Wd, qd)
    torch.cuda.synchronize()
    Dh2, Db2 = s.empty_f(), s.empty_f()
    F2, wall2 = s.zeros_face(case.nw), s.zeros_face(case.nw + 1)
    # stale contents from the earlier call must not leak into this one
    F2.fill_(7.0)
    wall2.fill_(-3.0)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = ugks.lib().ugks_flux_noalloc(s.ctx, float(dts), _p(hd), _p(bd), _p(Wd), _p(qd), _p(Dh2), _p(Db2), _p(F2),
                                      _p(wall2), st)
    assert rc == 0, ugks.lib().ugks_last_error().decode()
    torch.cuda.synchronize()
    for a, c in ((Dh, Dh2), (Db, Db2), (F, F2), (wall, wall2)):
        assert torch.equal(a, c)
    # F NULL: the face macro flux lives in the static array too
    Dh3, Db3 = s.empty_f(), s.empty_f()
    rc = ugks.lib().ugks_flux_noalloc(s.ctx, float(dts), _p(hd), _p(bd), _p(Wd), _p(qd), _p(Dh3), _p(Db3), None,
                                      None, st)
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(Dh, Dh3) and torch.equal(Db, Db3)
    s.close()


@pytest.mark.parametrize("prec", [ugks.F64, ugks.F32])
def test_noalloc_flux_matches_flux(prec):
    say("no-alloc flux: cylinder 128 x 64, 48 x 48 velocities, then a small cavity")
    _both(wl.cylinder(ni=128, nj=64, nvx=48), prec)
    _both(wl.cavity(12, 16, kn=0.1, lid=0.5), prec)


def test_noalloc_flux_rejects_cases_above_the_array():
    case = wl.cylinder(ni=128, nj=64, nvx=100)
    s = ugks.Solver(case, ugks.F64)
    h = s.empty_f()
    W, q = s.zeros_w(), s.zeros_q()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = ugks.lib().ugks_flux_noalloc(s.ctx, 0.01, _p(h), _p(h), _p(W), _p(q), _p(h), _p(h), None, None, st)
    assert rc == -2
    assert "static array" in ugks.lib().ugks_last_error().decode()
    s.close()
