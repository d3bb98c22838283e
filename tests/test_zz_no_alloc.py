"""The allocation-free diagnostics entry point (rrmhd_diagnostics_noalloc):
through the C-ABI, its results against rrmhd_diagnostics on the same state,
bit for bit (same kernels, same reduction order), on two calls in a row, the
second on a smaller grid, and the first made before the handle's own
diagnostics workspace was ever allocated."""
import math

import numpy as np
import pytest

from paper_2602_14667_amd import inputs
from test_gpu_parity import dev, note, rrmhd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pair(s):
    a = s.diagnostics_noalloc()
    b = s.diagnostics()
    c = s.diagnostics_noalloc()
    assert a == b == c, (a, b, c)
    return a


def test_noalloc_matches_diagnostics_two_calls_shrinking():
    R = rrmhd()
    note("noalloc diagnostics: 300 x 260 periodic f32")
    u, b = inputs.random_modes(300, 260, 0.04, seed=11)
    s = R.Solver(300, 260, 0.53, 0.57)
    s.init(dev(u), dev(b))
    s.step(7)
    big = _pair(s)
    assert all(math.isfinite(v) and v > 0 for v in big)
    s.close()
    note("noalloc diagnostics: 40 x 24 walls + force f16")
    h = inputs.Hartmann(nx=40, ny=24, tau_f=0.8, tau_m=0.75, G=1e-4, Ha=4.0)
    u, b = inputs.random_modes(40, 24, 0.03, seed=4)
    b[1] += h.B0
    s = R.Solver(40, 24, h.tau_f, h.tau_m, storage="f16", walls=True,
                 force=(h.G, 0.0), b_wall=(0.0, h.B0))
    s.init(dev(u), dev(b))
    s.step(5)
    small = _pair(s)
    assert all(math.isfinite(v) for v in small)
    assert small != big
    s.close()


def test_noalloc_single_buffer_and_nonfinite():
    R = rrmhd()
    note("noalloc diagnostics: single buffer, odd step count; non-finite state")
    u, b = inputs.random_modes(64, 48, 0.04, seed=2)
    s = R.Solver(64, 48, 0.6, 0.6, storage="f32", inplace=True)
    s.init(dev(u), dev(b))
    s.step(3)
    _pair(s)
    s.close()
    u[0, 5, 7] = np.nan
    s = R.Solver(64, 48, 0.6, 0.6)
    s.init(dev(u), dev(b))
    rc_ref, ref = s.diagnostics_rc()
    assert rc_ref == R.ENONFINITE
    vals = s.diagnostics_noalloc(allow_nonfinite=True)
    assert all(math.isnan(v) for v in vals) and all(math.isnan(v) for v in ref)
    s.close()
