"""The 8192^2 decaying-turbulence configuration over its 10,000-step horizon
(tau = 0.52): FP32 storage stays finite and its energies evolve smoothly;
the FP16 codecs track FP32's energies while finite, and both turn
non-finite before the horizon (between steps 6000 and 6500 when measured),
a stated miss kept as strict expected failures."""
import math

import pytest

from paper_2602_14667_amd import inputs
from test_gpu_parity import note, rrmhd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, TAU, HORIZON, EVERY = 8192, 0.52, 10_000, 500
_series = {}


def energy_series(storage):
    """(step, E_kin, E_mag, max div b) every 500 steps up to the horizon or the
    first non-finite diagnostic."""
    if storage not in _series:
        R = rrmhd()
        u, b = inputs.turbulence(N, 0.04)
        s = R.Solver(N, N, TAU, TAU, storage=storage)
        s.init(torch.from_numpy(u).cuda(), torch.from_numpy(b).cuda())
        del u, b
        out = []
        while s.step_count < HORIZON:
            s.step(EVERY)
            ek, em, dv = s.diagnostics(allow_nonfinite=True)
            out.append((s.step_count, ek, em, dv))
            note(f"  {storage} step {s.step_count}: E_kin {ek:.6e} E_mag {em:.6e} div b {dv:.3e}")
            if not all(math.isfinite(v) for v in (ek, em, dv)):
                break
        s.close()
        torch.cuda.empty_cache()
        _series[storage] = out
    return _series[storage]


def test_c3_fp32_horizon_and_fp16_tracking():
    note("C3 8192^2 over 10,000 steps: FP32, then FP16 codecs")
    f32 = energy_series("f32")
    assert len(f32) == HORIZON // EVERY and f32[-1][0] == HORIZON
    assert all(math.isfinite(v) for r in f32 for v in r[1:])
    # decaying kinetic energy, growing magnetic energy (dynamo-like exchange)
    assert f32[-1][1] < f32[0][1] and f32[-1][2] > f32[0][2]
    for storage in ("f16", "f16sr"):
        s16 = energy_series(storage)
        for (k, ek, em, _), (k2, ek2, em2, _) in zip(f32, s16):
            assert k == k2
            if k > 4000:
                break
            assert abs(ek2 / ek - 1) < 3e-3 and abs(em2 / em - 1) < 3e-3, (storage, k)


@pytest.mark.xfail(strict=True, reason="FP16 storage (round to nearest or stochastic) turns "
                   "non-finite before step 10,000 at tau = 0.52 (measured between 6000 and 6500)")
@pytest.mark.parametrize("storage", ["f16", "f16sr"])
def test_c3_fp16_finite_over_horizon(storage):
    s16 = energy_series(storage)
    assert s16[-1][0] == HORIZON and all(math.isfinite(v) for v in s16[-1][1:])
