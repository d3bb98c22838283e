"""Single-buffer (in-place) streaming on the GPU: a handle created with
RRMHD_STORE_INPLACE holds one population buffer and alternates two step
forms (pull + push into the opposite slots; own swapped slots + local
store).  The per-node arithmetic is that of the two-buffer step, so the two
are compared bit for bit, at odd and even step counts (the two layouts), with
walls and forcing, across launch shapes (one, two and four nodes per
thread, both layouts), through save/resume, checkpoint files and the
autotuner; plus the per-field bar against the FP64 oracle and the memory
held."""
import numpy as np
import pytest

import oracle
from paper_2602_14667_amd import inputs
from test_gpu_parity import FIELDS, dev, gpu_moments, note, rrmhd, run_pair, split

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pair(nx, ny, tau_f, tau_m, storage, **kw):
    R = rrmhd()
    return (R.Solver(nx, ny, tau_f, tau_m, storage=storage, **kw),
            R.Solver(nx, ny, tau_f, tau_m, storage=storage, inplace=True, **kw))


def assert_same(a, b, where):
    ga, gb = gpu_moments(a), gpu_moments(b)
    for k in FIELDS:
        assert np.array_equal(ga[k], gb[k]), (where, k)


@pytest.mark.parametrize("storage", ["f32", "f16", "f16sr"])
@pytest.mark.parametrize("shape", [(130, 66), (67, 45), (1, 37), (40, 1), (2, 2), (3, 5),
                                   (512, 33)])
def test_inplace_bitwise_periodic(storage, shape):
    nx, ny = shape
    note(f"in-place periodic {nx}x{ny} {storage}")
    u, b = inputs.random_modes(nx, ny, 0.05, seed=nx * 7 + ny)
    two, one = pair(nx, ny, 0.53, 0.57, storage)
    for s in (two, one):
        s.init(dev(u), dev(b))
    assert_same(two, one, 0)
    for k in (1, 2, 7, 10):
        two.step(k - two.step_count)
        one.step(k - one.step_count)
        assert_same(two, one, k)
    two.close(); one.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "f16sr"])
@pytest.mark.parametrize("shape", [(9, 24), (64, 17), (5, 2)])
def test_inplace_bitwise_walls_force(storage, shape):
    nx, ny = shape
    note(f"in-place walls+force {nx}x{ny} {storage}")
    h = inputs.Hartmann(nx=nx, ny=ny, tau_f=0.8, tau_m=0.75, G=1e-4, Ha=4.0)
    u, b = inputs.random_modes(nx, ny, 0.03, seed=4)
    b[1] += h.B0
    kw = dict(walls=True, force=(h.G, 0.0), b_wall=(0.0, h.B0))
    two, one = pair(nx, ny, h.tau_f, h.tau_m, storage, **kw)
    for s in (two, one):
        s.init(dev(u), dev(b))
    for k in (1, 2, 5, 30, 31):
        two.step(k - two.step_count)
        one.step(k - one.step_count)
        assert_same(two, one, k)
        assert two.diagnostics() == one.diagnostics()
    two.close(); one.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_inplace_diagnostics_fields_invariants(storage):
    note(f"in-place diagnostics {storage}")
    n = 96
    u, b = inputs.turbulence(n, 0.04)
    two, one = pair(n, n, 0.52, 0.55, storage)
    for s in (two, one):
        s.init(dev(u), dev(b))
    for k in (3, 8):
        two.step(k - two.step_count)
        one.step(k - one.step_count)
        assert two.diagnostics() == one.diagnostics()
        assert np.array_equal(two.invariants(), one.invariants())
        ja, wa = two.current_vorticity()
        jb, wb = one.current_vorticity()
        assert torch.equal(ja, jb) and torch.equal(wa, wb)
    two.close(); one.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "f16sr"])
def test_inplace_save_resume(storage):
    """A state saved at an odd step count (swapped layout) is returned in the
    usual layout: resumed on a two-buffer or a single-buffer handle it
    continues bit for bit."""
    note(f"in-place save/resume {storage}")
    R = rrmhd()
    n = 80
    u, b = inputs.turbulence(n, 0.04)
    ref = R.Solver(n, n, 0.52, 0.55, storage=storage)
    one = R.Solver(n, n, 0.52, 0.55, storage=storage, inplace=True)
    for s in (ref, one):
        s.init(dev(u), dev(b))
        s.step(13)
    buf = torch.empty(one.state_bytes(), dtype=torch.uint8, device="cuda")
    one.save_state(buf)
    buf2 = torch.empty_like(buf)
    ref.save_state(buf2)
    torch.cuda.synchronize()
    assert torch.equal(buf, buf2)
    ref.step(20)
    for inplace in (False, True):
        c = R.Solver(n, n, 0.52, 0.55, storage=storage, inplace=inplace)
        c.load_state(buf, 13)
        c.step(20)
        assert c.step_count == 33
        assert_same(ref, c, ("resume", inplace))
        c.close()
    ref.close(); one.close()


def test_inplace_c1_oracle_per_field():
    """Orszag-Tang 64^2 (u0 = b0 = 0.05, perturbed u, tau 0.56), 1000 steps
    on one buffer, per-field rel L2 against the FP64 oracle every 100 steps
    and at odd counts: the FP32 bar of 1e-6."""
    note("in-place C1 vs oracle")
    R = rrmhd()
    u, b = inputs.orszag_tang(64, 0.05, 0.05, perturb=1e-4, seed=0)
    s = R.Solver(64, 64, 0.56, 0.56, inplace=True)
    s.init(dev(u), dev(b))
    o = oracle.Oracle(64, 64, 0.56, 0.56)
    o.init(u, b)
    worst = 0.0
    for k in list(range(100, 1001, 100)) + [1001]:
        s.step(k - s.step_count)
        o.step(k - o.step_count)
        got, ref = gpu_moments(s), split(*o.moments())
        for f in FIELDS:
            worst = max(worst, np.linalg.norm(got[f] - ref[f]) / np.linalg.norm(ref[f]))
    note(f"  worst per-field rel L2 {worst:.3e}")
    assert worst <= 1e-6
    s.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "f16sr"])
def test_inplace_launch_shapes_bitwise(storage):
    note(f"in-place launch shapes {storage}")
    R = rrmhd()
    nx, ny = 130, 66
    u, b = inputs.random_modes(nx, ny, 0.03, seed=11)
    ref = R.Solver(nx, ny, 0.53, 0.57, storage=storage)
    ref.init(dev(u), dev(b))
    ref.step(9)
    r = gpu_moments(ref)
    ref.close()
    for bx, by, ry, xcd, nt in ((64, 4, 1, 0, 0), (32, 2, 3, 1, 1), (256, 1, 1, 2, 3),
                                (128, 1, 1, 0, 5), (16, 16, 1, 0, 4), (1, 1, 1, 0, 5)):
        s = R.Solver(nx, ny, 0.53, 0.57, storage=storage, inplace=True)
        s.set_launch(bx, by, ry, xcd, nt)
        s.init(dev(u), dev(b))
        s.step(9)
        g = gpu_moments(s)
        s.close()
        for k in FIELDS:
            assert np.array_equal(g[k], r[k]), (bx, by, ry, xcd, nt, k)


MULTI_SHAPES = [(128, 2, 1, 2, 5), (128, 1, 1, 2, 9), (64, 4, 1, 0, 5), (32, 8, 1, 0, 5),
                (16, 16, 1, 0, 9), (64, 1, 2, 1, 13), (128, 1, 1, 0, 4)]


@pytest.mark.parametrize("layout", ["default", "planar"])
@pytest.mark.parametrize("storage", ["f32", "f16", "f16sr"])
@pytest.mark.parametrize("size", [(4, 5), (8, 3), (12, 7), (2, 3), (130, 66), (520, 18), (67, 9)])
def test_inplace_multi_node_bitwise(layout, storage, size):
    """Single-buffer steps with two or four nodes per thread (whole-row
    wavefronts), one node per thread in mixed-row wavefronts and plain
    stores, on both layouts: the two-buffer state bit for bit at odd and even
    step counts; sizes with the periodic seam in the first and last word."""
    nx, ny = size
    note(f"in-place multi-node {nx}x{ny} {storage} {layout}")
    R = rrmhd()
    u, b = inputs.random_modes(nx, ny, 0.05, seed=5 * nx + ny)
    ref = R.Solver(nx, ny, 0.53, 0.57, storage=storage)
    ref.init(dev(u), dev(b))
    for shape in MULTI_SHAPES:
        s = R.Solver(nx, ny, 0.53, 0.57, storage=storage, inplace=True, layout=layout)
        s.set_launch(*shape)
        s.init(dev(u), dev(b))
        if ref.step_count:
            ref.close()
            ref = R.Solver(nx, ny, 0.53, 0.57, storage=storage)
            ref.init(dev(u), dev(b))
        for k in (1, 2, 5, 6):
            ref.step(k - ref.step_count)
            s.step(k - s.step_count)
            assert_same(ref, s, (shape, k))
        s.close()
    ref.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_inplace_multi_forcing_and_default_shape(storage):
    """Forcing on the multi-node single-buffer path at 1024 x 512 (the
    default launch shape for FP16 storage, a two-node shape for FP32): 21
    steps equal the two-buffer run."""
    n, m = 1024, 512
    note(f"in-place multi-node default shape, forcing, {storage}")
    u, b = inputs.random_modes(n, m, 0.04, seed=21)
    two, one = pair(n, m, 0.52, 0.55, storage, force=(1e-5, -2e-6))
    if storage == "f32":  # one node per thread by default
        assert one.get_launch() == (128, 1, 1, 2, 1)
        one.set_launch(64, 4, 1, 2, 5)
    else:
        assert one.get_launch() == (64, 2, 1, 2, 5)
    for s in (two, one):
        s.init(dev(u), dev(b))
        s.step(21)
    assert_same(two, one, "forced")
    two.close(); one.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "f16sr"])
def test_inplace_rows_checkpoint_at_odd_step(storage, tmp_path):
    """A row-interleaved single-buffer handle saved to a file between the two
    step forms (odd step count) and resumed on a two-buffer handle and on
    planar handles continues bit for bit."""
    note(f"in-place rows checkpoint at odd step {storage}")
    R = rrmhd()
    nx, ny = 88, 30
    u, b = inputs.random_modes(nx, ny, 0.05, seed=17)
    ref = R.Solver(nx, ny, 0.53, 0.56, storage=storage)
    one = R.Solver(nx, ny, 0.53, 0.56, storage=storage, inplace=True)
    for s in (ref, one):
        s.init(dev(u), dev(b))
        s.step(7)
    path = str(tmp_path / "odd.rrmhd")
    one.save(path)
    ref.step(6)
    for kw in (dict(), dict(layout="planar"), dict(inplace=True, layout="planar")):
        c = R.Solver(nx, ny, 0.53, 0.56, storage=storage, **kw)
        c.load(path)
        c.step(6)
        assert_same(ref, c, ("odd-step file", kw))
        c.close()
    ref.close(); one.close()


def test_inplace_autotune_keeps_state(tmp_path):
    note("in-place autotune")
    n = 256
    u, b = inputs.turbulence(n, 0.04)
    two, one = pair(n, n, 0.52, 0.55, "f32")
    for s in (two, one):
        s.init(dev(u), dev(b))
        s.step(5)
    res = one.autotune(str(tmp_path / "tune.json"), trials=4)
    assert res["ms"] > 0
    assert one.step_count == 5
    assert_same(two, one, "after autotune")
    two.step(6); one.step(6)
    assert_same(two, one, "after autotune + 6")
    two.close(); one.close()


def test_inplace_holds_one_buffer():
    """The device memory a handle takes: a single-buffer handle takes half
    the population bytes of a two-buffer one (4096^2, FP32: 1.27 GB vs
    2.55 GB)."""
    R = rrmhd()
    n = 4096
    torch.cuda.synchronize()
    taken = []
    for inplace in (False, True):
        free0 = torch.cuda.mem_get_info()[0]
        s = R.Solver(n, n, 0.52, 0.55, inplace=inplace)
        torch.cuda.synchronize()
        taken.append(free0 - torch.cuda.mem_get_info()[0])
        s.close()
        torch.cuda.synchronize()
    state = n * n * 19 * 4
    note(f"  device bytes taken: two buffers {taken[0]}, one buffer {taken[1]} "
         f"(one state = {state})")
    assert abs(taken[0] - 2 * state) < 0.02 * state
    assert abs(taken[1] - state) < 0.02 * state


def test_inplace_rejects_closure_and_equilibrium_ablation():
    R = rrmhd()
    s = R.Solver(32, 32, 0.56, 0.56, inplace=True)
    params = torch.zeros(4931, dtype=torch.float32, device="cuda")
    norm = torch.ones(19, dtype=torch.float32, device="cuda")
    s.closure_set(params, norm)
    assert R.lib().rrmhd_closure_enable(s._h, 1) == R.EINVAL
    assert R.lib().rrmhd_set_equilibrium(s._h, R.FEQ_FULL_MAXWELL) == R.EINVAL
    s.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_inplace_full_size_8192_bitwise(storage):
    """8192^2 turbulence, 3 steps on one buffer against the two-buffer
    bench configuration: every node's moments identical."""
    note(f"in-place 8192^2 {storage}")
    R = rrmhd()
    n = 8192
    u, b = inputs.turbulence(n, 0.04)
    out = []
    for inplace in (False, True):
        s = R.Solver(n, n, 0.51, 0.51, storage=storage, inplace=inplace)
        s.init(dev(u), dev(b))
        s.step(3)
        rho, uu, bb = s.moments()
        out.append((rho, uu, bb))
        s.close()
    for x, y in zip(*out):
        assert torch.equal(x, y)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_inplace_walls_plain_stores_bitwise(storage):
    """Walls and forcing with plain (not non-temporal) stores and another
    tile shape: still the two-buffer state bit for bit."""
    note(f"in-place walls, plain stores {storage}")
    nx, ny = 33, 20
    h = inputs.Hartmann(nx=nx, ny=ny, tau_f=0.7, tau_m=0.65, G=1e-4, Ha=3.0)
    u, b = inputs.random_modes(nx, ny, 0.03, seed=8)
    b[1] += h.B0
    kw = dict(walls=True, force=(h.G, 0.0), b_wall=(0.0, h.B0))
    two, one = pair(nx, ny, h.tau_f, h.tau_m, storage, **kw)
    one.set_launch(16, 4, 2, 1, 0)
    for s in (two, one):
        s.init(dev(u), dev(b))
    for k in (3, 8):
        two.step(k - two.step_count)
        one.step(k - one.step_count)
        assert_same(two, one, k)
    two.close(); one.close()


def test_inplace_scaled_f16_codec_bitwise():
    """FP16 storage with a codec scale S = 4 (the scaled codec): the single
    buffer still evolves as the two-buffer handle with the same scale."""
    note("in-place f16 codec scale 4")
    n = 48
    u, b = inputs.turbulence(n, 0.04)
    two, one = pair(n, n, 0.53, 0.56, "f16", codec_scale=4.0)
    for s in (two, one):
        s.init(dev(u), dev(b))
    for k in (5, 12):
        two.step(k - two.step_count)
        one.step(k - one.step_count)
        assert_same(two, one, k)
    two.close(); one.close()
