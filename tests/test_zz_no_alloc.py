"""The allocation-free diagnostics entry point against tc_get_diag.

tc_get_diag_noalloc keeps its partial sums in the library's static device
array and reduces them on the device with the same arithmetic as the host
reduction of tc_get_diag, so the two agree bit for bit.  Two calls in a row
on different contexts, the second with a smaller grid, share that array.
"""
import ctypes

import numpy as np
import pytest

import tc_inputs

pytestmark = pytest.mark.gpu


def _diag(S, fn):
    out = np.full(8, -1.0)
    st = fn(S.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert st == 0, S.lib.tc_last_error(S.ctx).decode()
    return out


@pytest.mark.parametrize("order", [("medium", "small"), ("small", "medium")])
def test_noalloc_diag_matches_tc_get_diag(order):
    import torch
    from paper_1311_2481_amd import Solver
    first = None
    for name in order:
        cfg = tc_inputs.CONFIGS[name]
        S = Solver(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt)
        print(f"[no-alloc diag] {name}: n_r={cfg.n_r} {cfg.m_theta}x{cfg.m_z}", flush=True)
        u = tc_inputs.initial_state(S.radial_nodes(), cfg, device="cuda")
        S.set_state(u)
        S.step(2)
        torch.cuda.synchronize()
        want = _diag(S, S.lib.tc_get_diag)
        got = _diag(S, S.lib.tc_get_diag_noalloc)
        again = _diag(S, S.lib.tc_get_diag_noalloc)
        np.testing.assert_array_equal(got, want)
        np.testing.assert_array_equal(again, want)
        assert got[5] == 2 and np.all(np.isfinite(got))
        if first is not None:
            # the other context's values are not left behind
            assert not np.array_equal(got, first)
        first = got
        S.close()
