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


def test_spectral_error_budget_of_the_plain_coarse_run():
    """Where the plain coarse run's spectral error comes from, on the full
    protocol's grids (2048^2 fine -> 512^2 coarse, tau_f 0.56, seed 20, the
    judge's five comparison times):
    * the flow is deterministic over the horizon: a fine run from the same
      initial condition with every velocity value moved by up to 1e-4
      differs from it by eps_spec < 1e-2 at every time, so the coarse
      run's error is model error, not lost predictability;
    * the plain coarse run meets the 5 % bar at the first comparison time;
    * in the compared shells near k = N_c/4 the magnetic part of E(k) is
      several times the kinetic part, so eps_spec there is mostly the
      magnetic field's, which a closure of the fluid's a_1^(2) reaches only
      through the velocity;
    * the coarse relaxation time of the acoustic scaling is the best of
      tau_c and tau_c +- 0.001 at the first time (the spectrum's high shells
      move by more than the bar for a 7 % change of viscosity)."""
    import numpy as np
    from paper_2602_14667_amd import closure_pipeline as cp, inputs, rrmhd, spectral
    rrmhd.lib()
    n_f, factor, tau_f, seed = 2048, 4, 0.56, 20
    n_c = n_f // factor
    tc = cp.tau_coarse(tau_f, factor)
    cks = [16000 * (k + 1) // 5 for k in range(5)]
    K = n_c // 4
    print("[gpu] spectral error budget 2048 -> 512, seed 20", flush=True)

    def fine(u, b):
        s = rrmhd.Solver(n_f, n_f, tau_f, tau_f)
        s.init(cp._dev(u), cp._dev(b))
        out = {}
        for c in cks:
            s.step(factor * c - s.step_count)
            _, uu, bb = s.moments()
            out[c] = spectral.kinetic_magnetic_spectra(
                spectral.box_filter(uu.cpu().numpy(), factor),
                spectral.box_filter(bb.cpu().numpy(), factor))
        s.close()
        return out

    def coarse(tau, steps):
        uc, bc = cp.coarse_fields(n_f, factor, seed)
        s = rrmhd.Solver(n_c, n_c, tau, tau)
        s.init(cp._dev(uc), cp._dev(bc))
        out = {}
        for c in steps:
            s.step(c - s.step_count)
            _, uu, bb = s.moments()
            out[c] = spectral.kinetic_magnetic_spectra(uu.cpu().numpy(), bb.cpu().numpy())
        s.close()
        return out

    u, b = cp.fine_fields(n_f, seed)
    ref = fine(u, b)
    r = inputs.counter_uniform(120, 7, np.arange(u.size, dtype=np.uint64)).reshape(u.shape)
    alt = fine(u + 1e-4 * (2 * r - 1), b)
    for c in cks:
        e = spectral.eps_spec(sum(alt[c]), sum(ref[c]), K)
        print(f"[gpu]   perturbed fine run, step {c}: eps_spec {e:.2e}", flush=True)
        assert e < 1e-2
    plain = coarse(tc, cks)
    for c in cks:
        (ek, em), (rk, rm) = plain[c], ref[c]
        print(f"[gpu]   plain coarse step {c}: eps_spec {spectral.eps_spec(ek + em, rk + rm, K):.4f} "
              f"(kinetic {spectral.eps_spec(ek, rk, K):.4f}, magnetic "
              f"{spectral.eps_spec(em, rm, K):.4f}); E_b/E_u at k = {K}: {rm[K] / rk[K]:.2f}",
              flush=True)
        assert rm[K] / rk[K] > 2.0
    first = cks[0]
    eps = {}
    for tau in (tc - 0.001, tc, tc + 0.001):
        run = plain if tau == tc else coarse(tau, [first])
        eps[tau] = spectral.eps_spec(sum(run[first]), sum(ref[first]), K)
    print(f"[gpu]   eps_spec at step {first} for tau_c - 0.001, tau_c, tau_c + 0.001: "
          f"{[round(v, 4) for v in eps.values()]}", flush=True)
    assert eps[tc] <= 0.05
    assert eps[tc] < eps[tc - 0.001] and eps[tc] < eps[tc + 0.001]


def test_best_velocity_bound_of_a_fluid_only_closure(capsys):
    """No correction of the fluid's a_1^(2) brings the coarse run within the
    5 % spectral bar (full protocol, test seeds 20-23): with the filtered fine
    velocity imposed after every coarse step (the best velocity any fluid
    closure could give it), the kinetic spectrum and both energies are
    reproduced, yet the magnetic field evolved on the coarse grid leaves the
    worst-time eps_spec above 0.05 on every test seed.  The same bound is
    below the plain coarse run's worst eps_spec on every seed, so it is the
    room a fluid-only closure has."""
    from paper_2602_14667_amd import closure_pipeline as cp, rrmhd
    rrmhd.lib()

    def log(m):
        with capsys.disabled():
            print("[gpu]  ", m, flush=True)

    log("best-velocity bound, full protocol 2048 -> 512, test seeds 20-23")
    n_f, factor, tau_f = 2048, 4, 0.56
    n_c = n_f // factor
    tc = cp.tau_coarse(tau_f, factor)
    cks = [16000 * (k + 1) // 5 for k in range(5)]
    kmax = n_c // 4
    for sd in (20, 21, 22, 23):
        run, ref, parts = cp.velocity_bound_run(n_f, tau_f, factor, sd, cks)
        rows, worst = cp.judge(run, ref, kmax)
        uc, bc = cp.coarse_fields(n_f, factor, sd)
        plain, _, _ = cp.spectra_run(n_c, tc, uc, bc, cks)
        _, wp = cp.judge(plain, ref, kmax)
        log(f"seed {sd}: bound eps_spec {[round(r['eps_spec'], 4) for r in rows]}, magnetic "
            f"{[round(parts[c]['magnetic'], 4) for c in cks]}, kinetic max "
            f"{max(parts[c]['kinetic'] for c in cks):.1e}; plain worst {wp['eps_spec']:.4f}")
        assert max(parts[c]["kinetic"] for c in cks) < 1e-3
        assert worst["ekin_err"] < 1e-3 and worst["emag_err"] < 5e-3
        assert worst["eps_spec"] > 0.05
        assert worst["eps_spec"] < wp["eps_spec"]


@pytest.mark.xfail(strict=True, reason=(
    "measured on the full protocol (2048^2 -> 512^2, tau_f 0.56, 16 training seeds, "
    "alpha 0.01 from the validation seeds): the closure lowers the worst-time eps_spec on "
    "test seeds 21, 22, 23 (0.092 vs 0.108, 0.179 vs 0.207, 0.086 vs 0.106) but raises it "
    "on seed 20 (0.161 vs 0.121)"))
def test_closure_gain_on_held_out_seeds(capsys):
    """The learned closure against the plain coarse run on the held-out test
    seeds 20-23, full protocol: the closure run's spectral error (eps_spec,
    worst over the five comparison times) must be lower than the plain run's
    on every test seed."""
    from paper_2602_14667_amd import closure_pipeline as cp, rrmhd
    rrmhd.lib()

    def log(m):
        with capsys.disabled():
            print("[gpu]  ", m, flush=True)

    log("closure gain on held-out seeds: full protocol 2048 -> 512")
    res = cp.pipeline(n_f=2048, factor=4, tau_f=0.56, fine_steps=64000, snaps=8,
                      train_seeds=range(16), val_seeds=range(16, 20),
                      test_seeds=range(20, 24), train_steps=3000, onestep_steps=2000,
                      batch=65536, log=log)
    gains = {t["seed"]: (t["plain"]["eps_spec"], t["closure"]["eps_spec"]) for t in res["tests"]}
    log(f"eps_spec (plain, closure) per test seed: {gains}")
    for sd, (p, c) in gains.items():
        assert c < p, (sd, p, c)
