"""GPU end-to-end test of the learned-closure pipeline at a reduced size:
fine runs -> filtered samples -> FP32 training (a-priori warm start, then the
one-step solver-in-the-loop objective) -> coarse runs with and
without the closure -> spectral judge against the filtered fine run.  The
gain of the trained closure over the plain coarse run is reported; the test
asserts that training lowers the loss, that the closure run stays finite,
and that both coarse runs are judged against the same reference."""
import math

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_closure_pipeline_small():
    from paper_2602_14667_amd import closure_pipeline as cp, rrmhd
    rrmhd.lib()
    print("[gpu] closure pipeline 256 -> 64", flush=True)
    res = cp.pipeline(n_f=256, factor=4, tau_f=0.54, fine_steps=4000, snaps=4,
                      train_seeds=range(3), val_seeds=[3], test_seeds=[20],
                      train_steps=300, onestep_steps=300, batch=16384, lr=1e-3,
                      n_times=4, log=lambda m: print("[gpu]  ", m, flush=True))
    hist = res["train_loss"]
    assert hist[-1][1] < hist[0][1]
    # the one-step training lowers its objective below the uncorrected step
    ob = res["onestep_objective"]
    assert ob["final"] < ob["no_closure"]
    t = res["tests"][0]
    for side in ("plain", "closure"):
        w = t[side]
        assert math.isfinite(w["eps_spec"]) and math.isfinite(w["ekin_err"])
    print(f"[gpu]   eps_spec plain {t['plain']['eps_spec']:.4f} closure "
          f"{t['closure']['eps_spec']:.4f}; fallback {t['fallback_at']}", flush=True)
