"""GPU tests of the learned closure's inference: BF16-MFMA network against
the FP64 oracle network, zero network = plain step (bitwise), and the fused
step with a non-trivial network against the oracle with the same network."""
import numpy as np
import pytest

import oracle
from paper_2602_14667_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def R():
    from paper_2602_14667_amd import rrmhd
    rrmhd.lib()
    return rrmhd


def init_params(rng, gain=1.0):
    """He-style random parameters (fan-in scaled), float64."""
    p = np.zeros(oracle.NPARAM)
    p[0:512] = rng.standard_normal(512) * gain / np.sqrt(8)
    p[512:576] = 0.1 * rng.standard_normal(64)
    p[576:4672] = rng.standard_normal(4096) * gain / np.sqrt(64)
    p[4672:4736] = 0.1 * rng.standard_normal(64)
    p[4736:4928] = rng.standard_normal(192) / np.sqrt(64)
    p[4928:4931] = 0.1 * rng.standard_normal(3)
    return p


def features(rng, n):
    x = np.empty((n, 8))
    x[:, 0] = 1 + 0.01 * rng.standard_normal(n)
    x[:, 1:5] = 0.04 * rng.standard_normal((n, 4))
    x[:, 5:8] = 1e-4 * rng.standard_normal((n, 3))
    return x


def norm_of(x, so=(1e-4, 1e-4, 1e-4)):
    return np.concatenate([x.mean(0), x.std(0), np.asarray(so)])


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 70000])
def test_network_inference_vs_fp64(n):
    note(f"closure eval n={n}")
    rr = R()
    rng = np.random.default_rng(n)
    p = init_params(rng)
    x = features(rng, n)
    nm = norm_of(features(rng, 4096))
    # the oracle sees exactly the FP32 values the GPU reads
    p32, nm32, x32 = (a.astype(np.float32).astype(np.float64) for a in (p, nm, x))
    ref = oracle.mlp_forward(p32, nm32, x32)
    got = rr.closure_eval(dev32(p), dev32(nm), dev32(x)).cpu().numpy()
    e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    note(f"  BF16 MFMA vs FP64: rel L2 {e:.3e}")
    assert e < 2e-2


def test_zero_network_is_bitwise_plain():
    note("zero closure = plain")
    rr = R()
    n = 96
    u, b = inputs.turbulence(n, 0.04)
    a = rr.Solver(n, n, 0.51, 0.52)
    a.init(torch.from_numpy(u).cuda(), torch.from_numpy(b).cuda())
    a.step(20)
    c = rr.Solver(n, n, 0.51, 0.52)
    c.init(torch.from_numpy(u).cuda(), torch.from_numpy(b).cuda())
    c.closure_set(dev32(np.zeros(4931)), dev32(norm_of(features(np.random.default_rng(1), 100))))
    c.closure_enable(True)
    c.step(20)
    for x, y in zip(a.moments(), c.moments()):
        assert torch.equal(x, y)
    a.close(); c.close()


@pytest.mark.parametrize("shape", [(64, 64), (100, 37)])
def test_fused_closure_step_vs_oracle(shape):
    """A network whose correction is of the order of a_1^(2) itself; after 10
    steps the GPU fields match the oracle-with-closure fields, and the
    closure's effect (closure minus plain) agrees to BF16 accuracy."""
    nx, ny = shape
    note(f"fused closure step {nx}x{ny}")
    rr = R()
    rng = np.random.default_rng(3)
    u, b = inputs.random_modes(nx, ny, 0.05, seed=11)
    p = init_params(rng)
    nm = norm_of(features(rng, 4096), so=(2e-4, 1e-4, 2e-4))
    p32, nm32 = (a.astype(np.float32).astype(np.float64) for a in (p, nm))
    tf, tm, steps = 0.52, 0.55, 10
    o_plain = oracle.Oracle(nx, ny, tf, tm); o_plain.init(u, b); o_plain.step(steps)
    o_cl = oracle.Oracle(nx, ny, tf, tm); o_cl.set_closure(p32, nm32); o_cl.init(u, b)
    o_cl.step(steps)
    s = rr.Solver(nx, ny, tf, tm)
    s.init(torch.from_numpy(u).cuda(), torch.from_numpy(b).cuda())
    s.closure_set(dev32(p), dev32(nm))
    s.closure_enable(True)
    s.step(steps)
    got = [t.cpu().numpy() for t in s.moments()]
    s.close()
    ref = o_cl.moments()
    pl = o_plain.moments()
    for k, (g, r, q) in enumerate(zip(got, ref, pl)):
        e = np.linalg.norm(g - r) / np.linalg.norm(r)
        eff = np.linalg.norm(r - q)
        de = np.linalg.norm((g - q) - (r - q)) / max(eff, 1e-300)
        note(f"  field {k}: rel L2 {e:.3e}, closure effect {eff:.3e}, "
             f"effect error {de:.3e}")
        # BF16 network: the closure's effect carries a few 1e-3 relative
        # error per step (inference test above); the fields inherit it in
        # proportion to the effect's size
        assert de < 5e-2
        assert e < 5e-2 * eff / np.linalg.norm(r) + 1e-6


def test_runtime_fallback_to_plain():
    """A closure whose weights are scaled by 1e6 drives the state non-finite
    within its first chunk of steps: the run reloads the last checkpoint
    (here the initial state), turns the closure off, reports the step, and
    from then on is the plain run, bit for bit."""
    from paper_2602_14667_amd import closure_pipeline as cp
    note("closure runtime fallback")
    rng = np.random.default_rng(3)
    p = init_params(rng) * 1e6
    nm = norm_of(features(rng, 4096))
    n = 64
    u, b = inputs.turbulence(n, 0.04)
    cps = [500, 1500]
    plain, _, fb0 = cp.spectra_run(n, 0.56, u, b, cps, fallback_every=500)
    got, _, fb = cp.spectra_run(n, 0.56, u, b, cps, params=dev32(p), norm=dev32(nm),
                                fallback_every=500)
    note(f"  fell back at step {fb}")
    assert fb0 is None and fb == 500
    for c in cps:
        assert np.array_equal(got[c][0], plain[c][0])
        assert got[c][1] == plain[c][1] and got[c][2] == plain[c][2]


def _bf16_values(bits):
    """Float64 values of uint16 BF16 bit patterns."""
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _round_to_bf16(v):
    """Correctly rounded BF16 bit patterns (nearest, ties to even) of float64
    values, by comparing the two BF16 neighbours found by truncating the
    FP32 conversion toward zero and stepping one unit up."""
    f = v.astype(np.float32)
    u = f.view(np.uint32)
    lo = (u >> 16).astype(np.uint32)
    hi = lo + 1
    with np.errstate(invalid="ignore"):
        dl = np.abs(_bf16_values(lo.astype(np.uint16)) - v)
        dh = np.abs(_bf16_values(hi.astype(np.uint16)) - v)
        pick_hi = (dh < dl) | ((dh == dl) & (hi % 2 == 0))
    out = np.where(pick_hi, hi, lo).astype(np.uint16)
    nan = np.isnan(v)
    out[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return out


def test_gelu_table_is_correctly_rounded():
    """Every entry of the inference's GELU table is the tanh-form GELU of its
    BF16 argument, evaluated in FP64 here by numpy and rounded to the nearest
    BF16 (ties to even); infinities and NaN propagate as the formula does
    (+inf -> +inf, -inf -> NaN, NaN -> NaN).  The reference uses the form
    z / (1 + exp(-2 v)) of z/2 (1 + tanh v), which avoids the cancellation of
    1 + tanh v for large negative z, where the tanh form itself carries a
    relative error of a few per cent in FP64."""
    rr = R()
    tab = rr.closure_gelu_table().cpu().numpy().view(np.uint16)
    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    with np.errstate(invalid="ignore", over="ignore"):
        z = _bf16_values(bits)
        v = np.sqrt(2.0 / np.pi) * (z + 0.044715 * z ** 3)
        g = z / (1.0 + np.exp(-2.0 * v))
        # the two forms agree wherever 1 + tanh v does not cancel
        t = 0.5 * z * (1.0 + np.tanh(v))
        ok = np.isfinite(t) & (z > -2.0)
        assert np.allclose(g[ok], t[ok], rtol=1e-12, atol=1e-300)
        want = _round_to_bf16(g)
    with np.errstate(invalid="ignore"):
        got_v, want_v = _bf16_values(tab), _bf16_values(want)
    both_nan = np.isnan(got_v) & np.isnan(want_v)
    mism = ~both_nan & (tab != want)
    note(f"  GELU table: {int(mism.sum())} mismatching entries of 65536")
    assert not mism.any(), np.nonzero(mism)[0][:10]
    # spot values: GELU(0) = 0, GELU(1) = 0.8412 -> BF16 0.84375, large z -> z
    assert tab[0] == 0
    assert abs(_bf16_values(tab[[0x3f80]])[0] - 0.8411920) < 4e-3
    assert tab[0x4300] == 0x4300  # GELU(128) = 128
