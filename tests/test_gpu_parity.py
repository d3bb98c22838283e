"""GPU parity: the HIP library (through its C-ABI) against the FP64 oracle.

Every input is generated on the host by the seeded generators and handed to
both sides; no oracle input or expected value comes from the HIP path.
Error measure (per field, over the whole grid): rel L2 = ||x - x_ref|| /
||x_ref|| for rho, u_x, u_y, b_x, b_y.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2602_14667_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "bx", "by")


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def rrmhd():
    from paper_2602_14667_amd import rrmhd as R
    R.lib()
    return R


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def split(rho, u, b):
    return dict(rho=rho, ux=u[0], uy=u[1], bx=b[0], by=b[1])


def rel_errors(got, ref):
    out = {}
    for k in FIELDS:
        den = np.linalg.norm(ref[k])
        out[k] = np.linalg.norm(got[k] - ref[k]) / (den if den > 0 else 1.0)
    return out


def gpu_moments(s):
    rho, u, b = s.moments()
    torch.cuda.synchronize()
    return split(rho.cpu().numpy(), u.cpu().numpy(), b.cpu().numpy())


def run_pair(nx, ny, u, b, tau_f, tau_m, checkpoints, storage="f32",
             walls=False, force=(0.0, 0.0), b_wall=(0.0, 0.0),
             initial_norm=False, equilibrium="algorithm"):
    """Run GPU and oracle side by side; per-field rel L2 at each checkpoint.

    With initial_norm the error of a field is divided by the larger of its
    current and initial norms: on small or strongly damped grids a component
    can decay towards zero, and a ratio to a vanishing norm says nothing about
    the arithmetic."""
    R = rrmhd()
    s = R.Solver(nx, ny, tau_f, tau_m, storage=storage, walls=walls,
                 force=force, b_wall=b_wall, equilibrium=equilibrium)
    s.init(dev(u), dev(b))
    o = oracle.Oracle(nx, ny, tau_f, tau_m, walls=walls, force=force,
                      b_wall=b_wall,
                      option=(oracle.FEQ_SERIES_FULL if equilibrium == "full_maxwell"
                              else oracle.FEQ_ALGORITHM))
    o.init(u, b)
    ref0 = split(*o.moments())
    errs = []
    for n in checkpoints:
        s.step(n - s.step_count)
        o.step(n - o.step_count)
        got, ref = gpu_moments(s), split(*o.moments())
        e = rel_errors(got, ref)
        if initial_norm:
            for k in FIELDS:
                den = max(np.linalg.norm(ref[k]), np.linalg.norm(ref0[k]))
                e[k] = np.linalg.norm(got[k] - ref[k]) / den
        errs.append(e)
    s.close()
    return errs


def worst(errs, fields=FIELDS):
    return max(e[k] for e in errs for k in fields)


# ---------------------------------------------------------------------------
# Single node through the public API: a 1 x 1 periodic grid makes streaming
# the identity, so one step is exactly one collision.
# ---------------------------------------------------------------------------
W = np.array([4 / 9, 1 / 36, 1 / 9, 1 / 36, 1 / 9, 1 / 36, 1 / 9, 1 / 36,
              1 / 9])


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("taus", [(0.51, 0.57), (0.9, 0.6), (0.5005, 0.5005)])
def test_single_node_collision(seed, taus):
    note(f"single node seed={seed} taus={taus}")
    R = rrmhd()
    rng = np.random.default_rng(seed)
    u0 = 0.1 * rng.standard_normal(2)
    b0 = 0.1 * rng.standard_normal(2)
    feq, geq = oracle.node_equilibrium(1.0 + 0.02 * rng.standard_normal(),
                                       u0, b0)
    d32 = ((feq - W) + 0.02 * feq * rng.standard_normal(9)).astype(np.float32)
    g32 = (geq + 0.002 * rng.standard_normal(10)).astype(np.float32)
    f64 = W + d32.astype(np.float64)
    g64 = g32.astype(np.float64)
    fs, gs, _ = oracle.node_collide(f64, g64, 1 / taus[0], 1 / taus[1])
    s = R.Solver(1, 1, *taus)
    state = torch.from_numpy(np.concatenate([d32, g32])).cuda()
    s.load_state(state, 0)
    s.step(1)
    out = torch.empty_like(state)
    s.save_state(out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = np.concatenate([fs - W, gs])
    scale = np.abs(ref).max()
    assert np.max(np.abs(got - ref)) < 1e-6 * scale + 1e-12, (got - ref)
    s.close()


# ---------------------------------------------------------------------------
# Orszag-Tang 64^2, 1000 steps (the FP64 reference configuration)
# ---------------------------------------------------------------------------
def c1_inputs():
    return inputs.orszag_tang(64, 0.05, 0.05, perturb=1e-4, seed=0)


def test_c1_fp32_storage_per_field():
    note("C1 OT 64^2 fp32 storage 1000 steps")
    u, b = c1_inputs()
    errs = run_pair(64, 64, u, b, 0.56, 0.56, list(range(100, 1001, 100)))
    for k in FIELDS:
        e = max(x[k] for x in errs)
        note(f"  {k}: max rel L2 over t = {e:.3e}")
        assert e <= 1e-6, (k, e)


def c1_fp16_errors():
    u, b = c1_inputs()
    return run_pair(64, 64, u, b, 0.56, 0.56, list(range(100, 1001, 100)),
                    storage="f16")


def test_c1_fp16_storage_within_arithmetic_bound():
    """RNE FP16 storage of f - w: each stored value carries a relative error
    up to 2^-11; over 1000 steps the field error accumulates to a few 1e-3
    (the bound used here is 1e-2)."""
    note("C1 OT 64^2 fp16 storage 1000 steps")
    errs = c1_fp16_errors()
    for k in FIELDS:
        note(f"  {k}: max rel L2 over t = {max(x[k] for x in errs):.3e}")
    assert worst(errs) < 1e-2


@pytest.mark.xfail(reason="prescribed RNE FP16 codec measured above the 1e-3 "
                          "per-field target on this flow", strict=False)
def test_c1_fp16_storage_target():
    errs = c1_fp16_errors()
    assert worst(errs, ("ux", "uy", "bx", "by")) <= 1e-3


# ---------------------------------------------------------------------------
# Ragged shapes, several tiles, edge cases
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(67, 45), (300, 7), (257, 3), (1, 37),
                                   (40, 1), (3, 5), (2, 2), (512, 33)])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_ragged_shapes(shape, storage):
    nx, ny = shape
    note(f"ragged {nx}x{ny} {storage}")
    u, b = inputs.random_modes(nx, ny, 0.06, seed=nx * 131 + ny)
    errs = run_pair(nx, ny, u, b, 0.53, 0.58, [1, 7, 30], storage=storage,
                    initial_norm=True)
    tol = 1e-6 if storage == "f32" else 1e-2
    assert worst(errs) < tol, errs


def test_elementwise_fp32_after_few_steps():
    """Element by element on a 130 x 97 grid after 5 steps."""
    note("elementwise 130x97")
    nx, ny = 130, 97
    u, b = inputs.random_modes(nx, ny, 0.08, seed=5)
    R = rrmhd()
    s = R.Solver(nx, ny, 0.52, 0.55)
    s.init(dev(u), dev(b))
    s.step(5)
    got = gpu_moments(s)
    o = oracle.Oracle(nx, ny, 0.52, 0.55); o.init(u, b); o.step(5)
    ref = split(*o.moments())
    for k in FIELDS:
        scale = np.abs(ref[k]).max() if k != "rho" else 1.0
        assert np.max(np.abs(got[k] - ref[k])) < 1e-6 * scale, k
    s.close()


def test_zero_steps_returns_initial_fields():
    note("zero steps")
    u, b = inputs.random_modes(33, 20, 0.05, seed=9)
    R = rrmhd()
    s = R.Solver(33, 20, 0.6, 0.6)
    s.init(dev(u), dev(b))
    got = gpu_moments(s)
    assert np.max(np.abs(got["rho"] - 1)) < 1e-7
    assert np.max(np.abs(got["ux"] - u[0])) < 1e-8
    assert np.max(np.abs(got["bx"] - b[0])) < 1e-8
    s.close()


def test_uniform_state_fixed_point():
    note("uniform fixed point")
    n = 64
    u = np.zeros((2, n, n)); u[0] = 0.04; u[1] = -0.03
    b = np.zeros((2, n, n)); b[0] = 0.02; b[1] = 0.05
    R = rrmhd()
    s = R.Solver(n, n, 0.55, 0.6)
    s.init(dev(u), dev(b))
    s.step(200)
    got = gpu_moments(s)
    assert np.max(np.abs(got["ux"] - 0.04)) < 1e-7
    assert np.max(np.abs(got["by"] - 0.05)) < 1e-7
    s.close()


# ---------------------------------------------------------------------------
# Diagnostics and invariants (FP64 reductions on the GPU)
# ---------------------------------------------------------------------------
def test_diagnostics_match_oracle():
    note("diagnostics C1 500 steps")
    u, b = c1_inputs()
    R = rrmhd()
    s = R.Solver(64, 64, 0.56, 0.56)
    s.init(dev(u), dev(b))
    o = oracle.Oracle(64, 64, 0.56, 0.56); o.init(u, b)
    for n in (0, 500):
        s.step(n - s.step_count); o.step(n - o.step_count)
        ek, em, dv = s.diagnostics()
        rk, rm, rd = o.diagnostics()
        assert abs(ek / rk - 1) < 2e-6 and abs(em / rm - 1) < 2e-6
        # div b is a difference of b values O(0.05): its absolute error is the
        # stencil (norm 2) applied to the field error, <= 1e-6 * max |b|
        assert abs(dv - rd) < 2e-6 * 0.05
    inv0 = o.invariants()
    inv = s.invariants()
    assert abs(inv[0] - inv0[0]) < 64 * 64 * 1e-7
    # deterministic reduction order: repeated calls agree bitwise
    assert s.diagnostics() == s.diagnostics()
    s.close()


def test_mass_and_momentum_conservation_fp32():
    note("conservation 128^2 2000 steps")
    n = 128
    u, b = inputs.turbulence(n, 0.04)
    R = rrmhd()
    s = R.Solver(n, n, 0.51, 0.51)
    s.init(dev(u), dev(b))
    inv0 = s.invariants()
    s.step(2000)
    inv1 = s.invariants()
    # per-node drift of the FP32 state (round-off, no bias)
    assert abs(inv1[0] - inv0[0]) / (n * n) < 1e-6
    for k in range(1, 5):
        assert abs(inv1[k] - inv0[k]) / (n * n) < 1e-6
    s.close()


def test_nonfinite_state_is_reported():
    note("non-finite detection")
    R = rrmhd()
    u, b = inputs.random_modes(16, 16, 0.05, seed=1)
    u[0, 3, 4] = np.nan
    s = R.Solver(16, 16, 0.6, 0.6)
    s.init(dev(u), dev(b))
    rc, vals = s.diagnostics_rc()
    assert rc == R.ENONFINITE
    assert all(math.isnan(v) for v in vals)
    s.close()


# ---------------------------------------------------------------------------
# Walls + forcing
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_walls_and_force_small(storage):
    """Walls, anti-bounce-back and the body force on a 9 x 24 channel with a
    random initial field: per-field rel L2 against the oracle at 1, 10 and 300
    steps.  FP32 storage: <= 1e-6 (the FP32 storage model of the oracle stays
    within 2e-8 here)."""
    note(f"walls+force 9x24 {storage}")
    h = inputs.Hartmann(nx=9, ny=24, tau_f=0.8, tau_m=0.75, G=1e-5, Ha=4.0)
    u, b = inputs.random_modes(9, 24, 0.01, seed=4)
    b[1] += h.B0
    errs = run_pair(9, 24, u, b, h.tau_f, h.tau_m, [1, 10, 300],
                    storage=storage, walls=True, force=(h.G, 0.0),
                    b_wall=(0.0, h.B0), initial_norm=True)
    for k in FIELDS:
        note(f"  {k}: {[float('%.2e' % e[k]) for e in errs]}")
    tol = 1e-6 if storage == "f32" else 1e-2
    assert worst(errs) < tol, errs


def c2_solver(R, h, storage="f32"):
    return R.Solver(h.nx, h.ny, h.tau_f, h.tau_m, storage=storage, walls=True,
                    force=(h.G, 0.0), b_wall=(0.0, h.B0))


C2_FIELDS = ("ux", "bx", "by")


def column_errors(got, ref_cols):
    """Per-field rel L2 of the GPU's column 0 against 1-D oracle columns; the
    GPU's columns must be identical to each other (x-invariant run)."""
    out = {}
    for k in C2_FIELDS:
        assert np.max(np.abs(got[k] - got[k][:, :1])) == 0.0, k
        col = np.asarray(ref_cols[k])
        out[k] = float(np.linalg.norm(got[k][:, 0] - col) / np.linalg.norm(col))
    return out


def test_hartmann_c2_transient_vs_oracle_columns():
    """512 x 256 channel from rest, 20000 steps: every GPU column against the
    oracle's x-invariant 1 x 256 column, per field.

    The bar is the oracle's own FP32 storage model (FP64 steps, state rounded
    to FP32 storage after each step) run alongside: the GPU's forced step
    computes in FP64 and rounds only on storage, so its error must be of the
    model's size (<= 3x it; the model gives 1.6e-6 for u_x, 1.3e-6 for
    b_x).  North_star's 1e-6 lies below that storage floor for u_x and is
    kept as a non-strict expected failure."""
    note("C2 512x256 20000 steps vs oracle 1x256")
    h = inputs.hartmann_c2()
    u, b = h.initial_fields()
    R = rrmhd()
    s = c2_solver(R, h)
    s.init(dev(u), dev(b))
    s.step(20000)
    got = gpu_moments(s)
    s.close()
    kw = dict(walls=True, force=(h.G, 0.0), b_wall=(0.0, h.B0))
    o = oracle.Oracle(1, h.ny, h.tau_f, h.tau_m, **kw)
    m = oracle.Oracle(1, h.ny, h.tau_f, h.tau_m, **kw)
    o.init(u[:, :, :1], b[:, :, :1])
    m.init(u[:, :, :1], b[:, :, :1])
    m.round_state_f32()
    o.step(20000)
    m.step_rounded_f32(20000)
    ref = {k: v[:, 0] for k, v in split(*o.moments()).items()}
    mod = {k: v[:, 0] for k, v in split(*m.moments()).items()}
    e = column_errors(got, ref)
    floor = {k: float(np.linalg.norm(mod[k] - ref[k]) / np.linalg.norm(ref[k]))
             for k in C2_FIELDS}
    note(f"  GPU vs oracle: {e}")
    note(f"  FP32 storage model vs oracle: {floor}")
    for k in C2_FIELDS:
        assert e[k] < 3.0 * floor[k] + 1e-7, (k, e[k], floor[k])


@pytest.mark.xfail(strict=False, reason="FP32 storage floor of the forced channel "
                   "(1.6e-6 for u_x at 20000 steps) lies above 1e-6")
def test_hartmann_c2_transient_fp32_target():
    h = inputs.hartmann_c2()
    u, b = h.initial_fields()
    R = rrmhd()
    s = c2_solver(R, h)
    s.init(dev(u), dev(b))
    s.step(20000)
    got = gpu_moments(s)
    s.close()
    o = oracle.Oracle(1, h.ny, h.tau_f, h.tau_m, walls=True, force=(h.G, 0.0),
                      b_wall=(0.0, h.B0))
    o.init(u[:, :, :1], b[:, :, :1])
    o.step(20000)
    e = column_errors(got, {k: v[:, 0] for k, v in split(*o.moments()).items()})
    note(f"  C2 transient per field: {e}")
    assert max(e.values()) <= 1e-6


def hartmann_closed_form(h, y):
    return h.profile(y)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_hartmann_c2_steady_state(storage):
    """512 x 256 Hartmann channel started from the closed-form profile and run
    400,000 steps (1.5 e-foldings of the slowest mode) on the GPU, against
    the closed form (<= 1e-3 for FP32 storage) and, like for like, against the
    FP64 oracle run from the same profile for the same steps (stored in
    tests/golden by a script that calls only the oracle).  FP32 storage: per
    field within 3x of the oracle's FP32 storage model at the same step (the
    model: 1.1e-6 for u_x, 2.8e-6 for b_x)."""
    import json
    import os
    fx = os.path.join(os.path.dirname(__file__), "golden",
                      "hartmann_c2_oracle.json")
    with open(fx) as fh:
        gold = json.load(fh)
    note(f"C2 steady state {storage}")
    h = inputs.hartmann_c2()
    assert gold["steps"] == 400_000 and gold["start"] == "closed form"
    y = np.arange(h.ny)
    ue, be = hartmann_closed_form(h, y)
    u = np.zeros((2, h.ny, h.nx)); u[0] = ue[:, None]
    b = np.zeros((2, h.ny, h.nx)); b[0] = be[:, None]; b[1] = h.B0
    R = rrmhd()
    s = c2_solver(R, h, storage)
    s.init(dev(u), dev(b))
    s.step(gold["steps"])
    got = gpu_moments(s)
    s.close()
    e = column_errors(got, gold["fp64"])
    gu, gb = got["ux"][:, 0], got["bx"][:, 0]
    eu = np.linalg.norm(gu - ue) / np.linalg.norm(ue)
    eb = np.linalg.norm(gb - be) / np.linalg.norm(be)
    note(f"  vs closed form: u {eu:.3e}  b_x {eb:.3e}")
    note(f"  vs FP64 oracle, same start and steps: {e}")
    if storage == "f32":
        assert eu < 1e-3 and eb < 1e-3
        for k in C2_FIELDS:
            ref, mod = np.array(gold["fp64"][k]), np.array(gold["fp32_storage"][k])
            floor = np.linalg.norm(mod - ref) / np.linalg.norm(ref)
            note(f"  {k}: model {floor:.3e}")
            assert e[k] < 3.0 * floor + 1e-7, (k, e[k], floor)
    else:
        # FP16 storage holds the profile only to its own rounding
        assert eu < 5e-3 and eb < 5e-3
        assert max(e.values()) < 1e-2


# ---------------------------------------------------------------------------
# Full size: 8192^2 turbulence in the benchmark's launch configuration,
# sampled nodes against the oracle run on (2k+1)^2 patches (after k steps a
# node depends only on nodes within distance k).
# ---------------------------------------------------------------------------
def sample_nodes(n, count, seed):
    idx = inputs.counter_u64(seed, 55, np.arange(2 * count)) % np.uint64(n)
    pts = list(zip(idx[:count].astype(int), idx[count:].astype(int)))
    pts += [(0, 0), (n - 1, 0), (0, n - 1), (n - 1, n - 1), (n // 2, 0)]
    return pts


def patch_oracle(u, b, x, y, k, tau_f, tau_m):
    n = u.shape[1]
    ys = (np.arange(y - k, y + k + 1)) % n
    xs = (np.arange(x - k, x + k + 1)) % n
    pu = u[:, ys][:, :, xs]
    pb = b[:, ys][:, :, xs]
    o = oracle.Oracle(2 * k + 1, 2 * k + 1, tau_f, tau_m)
    o.init(pu, pb)
    o.step(k)
    rho, uu, bb = o.moments()
    return np.array([rho[k, k], uu[0, k, k], uu[1, k, k], bb[0, k, k],
                     bb[1, k, k]])


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("k,count", [(3, 150), (100, 40)])
def test_full_size_8192_sampled(storage, k, count):
    """150 sampled nodes (plus corners and an edge node) after 3 steps, and
    40 after 100 steps (oracle patches of 201^2 nodes)."""
    n, tau = 8192, 0.51
    note(f"full size {n}^2 {storage}, {k} steps, sampled")
    u, b = inputs.turbulence(n, 0.04)
    R = rrmhd()
    s = R.Solver(n, n, tau, tau, storage=storage)
    s.init(dev(u), dev(b))
    s.step(k)
    rho, uu, bb = s.moments()
    pts = sample_nodes(n, count, seed=3)
    xs = torch.tensor([p[0] for p in pts], device="cuda")
    ys = torch.tensor([p[1] for p in pts], device="cuda")
    got = torch.stack([rho[ys, xs], uu[0, ys, xs], uu[1, ys, xs],
                       bb[0, ys, xs], bb[1, ys, xs]], 1).cpu().numpy()
    s.close()
    del rho, uu, bb
    torch.cuda.empty_cache()
    ref = np.array([patch_oracle(u, b, x, y, k, tau, tau) for x, y in pts])
    # per-field rel L2 over the sampled nodes (the per-field measure of the
    # precision targets, estimated on the sample), and the largest single
    # error in units of the field's rms scale
    rel = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
    scale = np.array([1.0, 0.04, 0.04, 0.04, 0.04])
    err = np.max(np.abs(got - ref) / scale, axis=0)
    note(f"  sampled rel L2 per field: {rel}")
    note(f"  max |err| / field scale: {err}")
    if storage == "f32":
        assert np.all(rel < 1e-6), rel
        assert np.all(err < 2e-6), err
    else:
        tol = 3e-3 if k < 10 else 1e-2
        assert np.all(err < tol), err


# ---------------------------------------------------------------------------
# Checkpoint / resume
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage", ["f32", "f16", "f16sr"])
def test_save_load_resume_bitwise(storage):
    note(f"resume {storage}")
    R = rrmhd()
    n = 96
    u, b = inputs.turbulence(n, 0.04)
    a = R.Solver(n, n, 0.52, 0.55, storage=storage)
    a.init(dev(u), dev(b))
    a.step(40)
    buf = torch.empty(a.state_bytes(), dtype=torch.uint8, device="cuda")
    a.save_state(buf)
    a.step(40)
    ra = gpu_moments(a)
    c = R.Solver(n, n, 0.52, 0.55, storage=storage)
    c.load_state(buf, 40)
    c.step(40)
    rc = gpu_moments(c)
    assert c.step_count == 80
    for k in FIELDS:
        assert np.array_equal(ra[k], rc[k])
    a.close(); c.close()


# ---------------------------------------------------------------------------
# Launch shapes: results do not depend on them (bitwise)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("shape", [(130, 66), (129, 40), (2, 5), (256, 17)])
def test_launch_shapes_bitwise(storage, shape):
    """Every launch shape and flag (tile shape, rows per thread, XCD order,
    non-temporal loads/stores, two nodes per thread for FP16 storage on even
    nx) gives the default shape's state bit for bit; odd nx and tiny grids
    exercise the periodic seam of the two-node update (nx = 2: both seams in
    one word) and its fallback."""
    nx, ny = shape
    note(f"launch shapes {storage} {nx}x{ny}")
    R = rrmhd()
    u, b = inputs.random_modes(nx, ny, 0.03, seed=11)
    ref = R.Solver(nx, ny, 0.53, 0.57, storage=storage)
    ref.init(dev(u), dev(b))
    ref.step(9)
    r = gpu_moments(ref)
    ref.close()
    for bx, by, ry, xcd, nt in ((64, 4, 1, 0, 0), (32, 2, 3, 1, 1), (256, 1, 1, 2, 3),
                                (128, 1, 1, 0, 5), (64, 2, 2, 2, 7), (16, 16, 1, 0, 4),
                                (1, 1, 1, 0, 5), (32, 2, 2, 1, 5)):
        s = R.Solver(nx, ny, 0.53, 0.57, storage=storage)
        s.set_launch(bx, by, ry, xcd, nt)
        s.init(dev(u), dev(b))
        s.step(9)
        g = gpu_moments(s)
        s.close()
        for k in FIELDS:
            assert np.array_equal(g[k], r[k]), (bx, by, ry, xcd, nt, k)


# ---------------------------------------------------------------------------
# Near tau = 1/2: the method's own instability, reproduced step for step
# ---------------------------------------------------------------------------
def test_near_half_tau_instability_tracks_oracle():
    """At tau_f = tau_m = 0.5003 the seeded turbulence field on 256^2 has a
    lattice Reynolds number (rms u * N / nu) near 1e5 and the scheme itself
    is unstable: in the FP64 oracle max|div b| grows by about a factor 300
    between steps 100 and 300 and the state is non-finite by step 800.  The
    FP32 GPU path follows the same growth (fields within the FP32 bar while
    the unstable mode is small, div b within 1e-3 relative) and turns
    non-finite too, so the loss of stability at small relaxation times is
    the method's (the collision with nu = c_s^2 (tau - 1/2), Sec. 2), not
    the kernel's."""
    note("near-half tau instability 256^2 tau 0.5003")
    R = rrmhd()
    n, tau = 256, 0.5003
    u, b = inputs.turbulence(n, 0.04)
    s = R.Solver(n, n, tau, tau, storage="f32")
    s.init(dev(u), dev(b))
    o = oracle.Oracle(n, n, tau, tau)
    o.init(u, b)
    divs = []
    for k, field_tol in ((100, 2e-6), (200, 4e-6), (300, 4e-5)):
        s.step(k - s.step_count)
        o.step(k - o.step_count)
        ek, em, dv = s.diagnostics()
        rek, rem, rdv = o.diagnostics()
        e = rel_errors(gpu_moments(s), split(*o.moments()))
        note(f"step {k}: div b {dv:.4e} vs {rdv:.4e}; "
             + " ".join(f"{f} {e[f]:.2e}" for f in FIELDS))
        assert max(e.values()) < field_tol, (k, e)
        assert abs(ek / rek - 1) < 1e-6 and abs(em / rem - 1) < 1e-6
        if k > 100:
            assert abs(dv / rdv - 1) < 1e-3, (k, dv, rdv)
        divs.append(rdv)
    assert divs[2] / divs[0] > 50
    s.step(800 - s.step_count)
    o.step(800 - o.step_count)
    rc, _ = s.diagnostics_rc()
    assert rc == R.ENONFINITE
    assert not all(math.isfinite(v) for v in o.diagnostics())
    s.close()


def hartmann_run(h, nx, storage, u, b, checkpoints):
    """x-averaged rel L2 of u_x and b_x against the closed form, and the
    largest spread of u_x across x, at each checkpoint."""
    R = rrmhd()
    ue, be = hartmann_closed_form(h, np.arange(h.ny))
    s = R.Solver(nx, h.ny, h.tau_f, h.tau_m, storage=storage, walls=True,
                 force=(h.G, 0.0), b_wall=(0.0, h.B0))
    s.init(dev(u), dev(b))
    out = []
    for n in checkpoints:
        s.step(n - s.step_count)
        g = gpu_moments(s)
        gu, gb = g["ux"].mean(1), g["bx"].mean(1)
        out.append((np.linalg.norm(gu - ue) / np.linalg.norm(ue),
                    np.linalg.norm(gb - be) / np.linalg.norm(be),
                    float(g["ux"].std(1).max())))
    s.close()
    return out


def test_hartmann_c2_long_wave_instability_fp32():
    """The C2 channel started from the closed-form profile plus a random
    perturbation of 1e-5 in u, FP32 storage: on the 512-wide channel the
    spread of u_x across x grows by about 10x per 5e4 steps (a mode of
    wavelength >= 256 in x is unstable), on a 64-wide channel it stays at the
    perturbation's level.  Runs started x-invariant keep every column
    identical, bit for bit, and never excite the mode; the noise of
    stochastic rounding does."""
    note("C2 long-wave instability, FP32, nx 512 and 64")
    h = inputs.hartmann_c2()
    ue, be = hartmann_closed_form(h, np.arange(h.ny))
    spread = {}
    for nx in (512, 64):
        rng = np.random.default_rng(5)
        u = np.zeros((2, h.ny, nx)); u[0] = ue[:, None]
        u += 1e-5 * rng.standard_normal(u.shape)
        b = np.zeros((2, h.ny, nx)); b[0] = be[:, None]; b[1] = h.B0
        spread[nx] = [r[2] for r in hartmann_run(h, nx, "f32", u, b, [50_000, 200_000])]
        note(f"  nx {nx}: spread of u_x across x at 5e4 / 2e5 steps {spread[nx]}")
    assert spread[512][1] > 100 * spread[512][0]
    assert spread[64][1] < 1e-5


@pytest.mark.parametrize("storage", ["f16sr", "f16"])
def test_hartmann_from_rest_fp16_narrow(storage):
    """FP16 storage from rest on an 8-wide section of the C2 channel (the
    same profile in y; every x-mode decays).  Round-to-nearest rounds every
    per-step increment of the body force away and the state freezes far
    from the profile; stochastic rounding keeps the increments on average
    and the x-averaged profile converges to within its noise (a few 1e-3)
    of the closed form."""
    h = inputs.hartmann_c2()
    nx = 8
    note(f"C2 from rest, {nx}x{h.ny}, {storage}")
    u = np.zeros((2, h.ny, nx))
    b = np.zeros((2, h.ny, nx)); b[1] = h.B0
    if storage == "f16sr":
        res = hartmann_run(h, nx, storage, u, b, [500_000])
        note(f"  rel L2 u {res[0][0]:.3e}  b_x {res[0][1]:.3e}")
        assert res[0][0] < 1e-2 and res[0][1] < 1e-2
    else:
        res = hartmann_run(h, nx, storage, u, b, [100_000])
        note(f"  rel L2 u {res[0][0]:.3e}  b_x {res[0][1]:.3e} (frozen)")
        assert res[0][0] > 0.5


# ---------------------------------------------------------------------------
# FP16 storage with stochastic rounding (optional codec variant)
# ---------------------------------------------------------------------------
def test_c1_fp16_stochastic_rounding_per_field():
    """Orszag-Tang 64^2, 1000 steps: the stochastically rounded FP16 codec
    against the FP64 oracle, next to the prescribed round-to-nearest-even
    codec on the same case.  Stochastic rounding removes the systematic part
    of the per-step rounding, so its accumulated error is expected to be the
    smaller of the two; both stay within the FP16 arithmetic bound."""
    note("C1 OT 64^2 fp16 stochastic rounding")
    u, b = c1_inputs()
    cps = list(range(100, 1001, 100))
    sr = run_pair(64, 64, u, b, 0.56, 0.56, cps, storage="f16sr")
    rne = run_pair(64, 64, u, b, 0.56, 0.56, cps, storage="f16")
    for k in FIELDS:
        note(f"  {k}: SR {max(e[k] for e in sr):.3e}  RNE {max(e[k] for e in rne):.3e}")
    assert worst(sr) < 1e-2
    assert worst(sr, ("ux", "uy", "bx", "by")) < worst(rne, ("ux", "uy", "bx", "by"))


@pytest.mark.parametrize("shape", [(130, 66), (129, 40), (132, 40), (4, 5), (520, 12)])
def test_stochastic_rounding_is_reproducible_and_shape_independent(shape):
    """The random bits are a hash of (step, node, plane): two runs, and runs
    with other launch shapes (one, two and four nodes per thread) and either
    layout, give the same state bit for bit."""
    nx, ny = shape
    R = rrmhd()
    u, b = inputs.random_modes(nx, ny, 0.03, seed=11)
    ref = None
    for bx, by, ry, xcd, nt, layout in (
            (0, 0, 0, 0, 0, "default"), (64, 4, 1, 0, 0, "default"), (32, 2, 3, 1, 1, "default"),
            (256, 1, 1, 2, 3, "default"), (128, 1, 1, 2, 9, "default"), (64, 2, 1, 2, 5, "default"),
            (64, 4, 1, 0, 13, "default"), (32, 8, 1, 0, 9, "default"), (128, 1, 1, 0, 9, "planar"),
            (64, 2, 1, 2, 5, "planar"), (0, 0, 0, 0, 0, "default")):
        s = R.Solver(nx, ny, 0.53, 0.57, storage="f16sr", layout=layout)
        if bx:
            s.set_launch(bx, by, ry, xcd, nt)
        s.init(dev(u), dev(b))
        s.step(9)
        g = gpu_moments(s)
        s.close()
        if ref is None:
            ref = g
        for k in FIELDS:
            assert np.array_equal(g[k], ref[k]), (bx, by, nt, layout, k)
    # the rounding is not round-to-nearest: the result differs from the codec
    s = R.Solver(nx, ny, 0.53, 0.57, storage="f16")
    s.init(dev(u), dev(b))
    s.step(9)
    g = gpu_moments(s)
    s.close()
    assert any(not np.array_equal(g[k], ref[k]) for k in FIELDS)


def test_stochastic_rounding_walls_force_parity():
    note("walls+force 9x24 f16sr")
    h = inputs.Hartmann(nx=9, ny=24, tau_f=0.8, tau_m=0.75, G=1e-4, Ha=4.0)
    u, b = inputs.random_modes(9, 24, 0.03, seed=4)
    b[1] += h.B0
    errs = run_pair(9, 24, u, b, h.tau_f, h.tau_m, [1, 10, 100], storage="f16sr",
                    walls=True, force=(h.G, 0.0), b_wall=(0.0, h.B0), initial_norm=True)
    assert worst(errs) < 1e-2, errs


def test_stochastic_rounding_keeps_small_increments():
    """A uniform flow (u = (0.05, 0.03), b = (0.02, 0.01)) driven by a body
    force too small to move any FP16 population by half a step: with
    round-to-nearest every increment is rounded away (the flow stagnates);
    with stochastic rounding the increments survive on average, and the mean
    momentum gained over k steps is k times the force (Guo forcing conserves
    mass and adds rho G per step), as with FP32 storage.  The mean field is
    conserved by the induction collision and stays put within the rounding
    noise.  FP32 storage: the forced step computes in FP64 and rounds only on
    storage, so the gain is exact to the storage rounding (the oracle's FP32
    storage model of this single-node state gains 1 - 1.7e-6 of k G; bar
    1e-4, where FP32 arithmetic lost 0.2 % of the force)."""
    R = rrmhd()
    n, k, G = 128, 200, 1e-6
    u = np.zeros((2, n, n))
    u[0], u[1] = 0.05, 0.03
    b = np.zeros((2, n, n))
    b[0], b[1] = 0.02, 0.01
    gain, drift = {}, {}
    for storage in ("f32", "f16", "f16sr"):
        s = R.Solver(n, n, 0.6, 0.6, storage=storage, force=(G, 0.0))
        s.init(dev(u), dev(b))
        m0 = gpu_moments(s)
        s.step(k)
        m1 = gpu_moments(s)
        s.close()
        gain[storage] = float(np.mean(m1["rho"] * m1["ux"]) - np.mean(m0["rho"] * m0["ux"]))
        drift[storage] = max(abs(float(np.mean(m1[f]) - np.mean(m0[f]))) for f in ("bx", "by"))
        note(f"  {storage}: momentum gain / (k G) = {gain[storage] / (k * G):.4f}, "
             f"mean-field drift {drift[storage]:.2e}")
    assert abs(gain["f32"] / (k * G) - 1) < 1e-4
    assert abs(gain["f16sr"] / (k * G) - 1) < 0.1
    assert abs(gain["f16"]) < 0.5 * k * G
    assert drift["f16sr"] < 2e-6


def test_stochastic_rounding_refusals():
    R = rrmhd()
    s = R.Solver(32, 32, 0.56, 0.56, storage="f16sr")
    assert R.lib().rrmhd_set_graph_chunk(s._h, 4) == R.EINVAL
    assert R.lib().rrmhd_set_equilibrium(s._h, R.FEQ_FULL_MAXWELL) == R.EINVAL
    s.close()
