"""The HIP path at the block sizes the sweeps accept, and their rejection
just beyond (through the C ABI, FP64, against the oracle):

- a channel block of 511 rows, the largest nj: the micro sweep's LDS
  (hand-off values and staged records of every row for a chunk of two
  velocities at two rows per thread) holds 8 (24 + 40 nj) bytes, within
  160 KiB up to 511 rows;
- a block periodic in j with 256 columns, the largest ni for a j-periodic
  block (its seam couplings staged in LDS);
- 512 rows and a 257-column j-periodic block are refused with
  UGKS_E_UNSUPPORTED.

Steps 1-2 and three inner iterations: relative L2 <= 1e-10 and per cell
max |f - f_oracle| / max |f_oracle| <= 1e-12 over the field cells."""
import numpy as np
import pytest

from paper_2604_09984_amd import ugks, workloads as wl
from tests.parity import both, cell_max_rel, dev, host, rel_l2, say

pytestmark = pytest.mark.gpu


def _steps(case, n_inner=3):
    o, s = both(case)
    h, b, W = wl.synthetic_f(case, amp=0.02)
    q = o.heatflux(h, b, W)
    dts, dtp = o.timesteps()
    dt = case.dt if case.dt is not None else case.dt_over_dts * dts
    hd, bd, Wd, qd = dev(h), dev(b), dev(W), dev(q)
    Wn = W.copy()
    Sh, Sb, Fn = o.begin_step(dt, dts, h, b, W, q)
    for _ in range(n_inner):
        o.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn)
    Wnd = Wd.clone()
    Shd, Sbd, Fnd = s.begin_step(dt, hd, bd, Wd, qd)
    s.step(dt, n_inner, hd, bd, Wd, Wnd, qd, Shd, Sbd, Fnd)
    f = o.types() == 1
    hh, bb, WW = host(hd), host(bd), host(Wd)
    e = (rel_l2(hh[f], h[f]), rel_l2(bb[f], b[f]), rel_l2(WW[f], W[f]))
    c = max(cell_max_rel(hh, h, f), cell_max_rel(bb, b, f), cell_max_rel(WW, W, f))
    s.close()
    return e, c


@pytest.mark.parametrize("mk,name", [(lambda: wl.channel(3, 511, 6), "channel_511_rows"),
                                     (lambda: wl.periodic_box(2, 256, 3, 6), "j_periodic_256_columns")],
                         ids=["nj511", "periodic_j_ni256"])
def test_largest_blocks(mk, name):
    case = mk()
    e, c = _steps(case)
    say(name, "h b W", e, "per-cell max rel", c)
    assert max(e) <= 1e-10 and c <= 1e-12


@pytest.mark.parametrize("mk", [lambda: wl.channel(3, 512, 6), lambda: wl.periodic_box(2, 257, 3, 6)],
                         ids=["nj512", "periodic_j_ni257"])
def test_blocks_beyond_the_limits_are_refused(mk):
    with pytest.raises(ugks.UgksError, match="error -6"):
        ugks.Solver(mk(), ugks.F64)
