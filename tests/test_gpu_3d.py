"""GPU parity of the three-dimensional extension (D3Q27 fluid, D3Q7 magnetic
lattice) against the FP64 three-dimensional oracle, through the C-ABI:
ragged and degenerate boxes, a turbulence field, diagnostics, conservation,
launch shapes (bitwise) and sampled nodes of a full-size box."""
import numpy as np
import pytest

import oracle
from paper_2602_14667_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "uz", "bx", "by", "bz")


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def rrmhd():
    from paper_2602_14667_amd import rrmhd as R
    R.lib()
    return R


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def split(rho, u, b):
    return dict(rho=rho, ux=u[0], uy=u[1], uz=u[2], bx=b[0], by=b[1], bz=b[2])


def gpu_fields(s):
    rho, u, b = s.moments()
    torch.cuda.synchronize()
    return split(rho.cpu().numpy(), u.cpu().numpy(), b.cpu().numpy())


def run_pair(shape, u, b, tau_f, tau_m, checkpoints, storage="f32"):
    """Per-field error at each checkpoint, divided by the larger of the
    field's current and initial norms."""
    nx, ny, nz = shape
    R = rrmhd()
    s = R.Solver3D(nx, ny, nz, tau_f, tau_m, storage=storage)
    s.init(dev(u), dev(b))
    o = oracle.Oracle3D(nx, ny, nz, tau_f, tau_m)
    o.init(u, b)
    ref0 = split(*o.moments())
    errs = []
    for n in checkpoints:
        s.step(n - s.step_count)
        o.step(n - o.step_count)
        got, ref = gpu_fields(s), split(*o.moments())
        e = {}
        for k in FIELDS:
            den = max(np.linalg.norm(ref[k]), np.linalg.norm(ref0[k]), 1e-300)
            e[k] = np.linalg.norm(got[k] - ref[k]) / den
        errs.append(e)
    s.close()
    return errs


def worst(errs):
    return max(e[k] for e in errs for k in FIELDS)


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("shape", [(7, 5, 3), (16, 8, 4), (1, 1, 9), (12, 1, 1), (2, 2, 2),
                                   (1, 1, 1), (70, 3, 2)])
def test_3d_ragged_boxes(storage, shape):
    note(f"3D ragged {shape} {storage}")
    u, b = inputs.random_modes3d(*shape, 0.04, seed=sum(shape) * 7)
    errs = run_pair(shape, u, b, 0.56, 0.6, [1, 5, 20], storage)
    for k in FIELDS:
        note(f"  {k}: {[float('%.2e' % e[k]) for e in errs]}")
    assert worst(errs) < (1e-6 if storage == "f32" else 1e-2), errs


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_3d_turbulence_per_field(storage):
    """24^3 random-phase turbulence (rms 0.04), tau 0.52 / 0.55, 100 steps,
    per-field rel L2 against the oracle every 25 steps."""
    note(f"3D turbulence 24^3 {storage}")
    n = 24
    u, b = inputs.turbulence3d(n, 0.04)
    errs = run_pair((n, n, n), u, b, 0.52, 0.55, [25, 50, 75, 100], storage)
    for k in FIELDS:
        note(f"  {k}: max rel L2 over t = {max(e[k] for e in errs):.3e}")
    assert worst(errs) < (1e-6 if storage == "f32" else 1e-2)


def test_3d_diagnostics_and_invariants():
    note("3D diagnostics")
    R = rrmhd()
    n = 16
    u, b = inputs.turbulence3d(n, 0.04)
    s = R.Solver3D(n, n, n, 0.55, 0.6)
    s.init(dev(u), dev(b))
    o = oracle.Oracle3D(n, n, n, 0.55, 0.6)
    o.init(u, b)
    inv0 = np.array(s.invariants())
    s.step(30)
    o.step(30)
    got, ref = s.diagnostics(), o.diagnostics()
    note(f"  gpu {got} oracle {ref}")
    assert abs(got[0] / ref[0] - 1) < 1e-6 and abs(got[1] / ref[1] - 1) < 1e-6
    assert abs(got[2] / ref[2] - 1) < 1e-4
    inv = np.array(s.invariants())
    ref_inv = o.invariants()
    assert abs(inv[0] - ref_inv[0]) < 1e-9 * n ** 3
    assert np.allclose(inv[1:], ref_inv[1:], rtol=0, atol=1e-9 * n ** 3)
    # FP32 storage: mass, momentum and sum b move only by rounding
    assert np.allclose(inv, inv0, rtol=0, atol=2e-6 * n ** 3)
    s.close()


@pytest.mark.parametrize("inplace", [False, True])
@pytest.mark.parametrize("shape", [(37, 11, 5), (40, 70, 9)])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_3d_launch_shapes_bitwise(storage, shape, inplace):
    """Launch shapes and both tile orders (the XCD-local one reorders every
    full run of 64 workgroups: the 40 x 70 x 9 box has several) give the same
    state bit for bit, with one buffer or two."""
    note(f"3D launch shapes {storage} {shape} inplace={inplace}")
    R = rrmhd()
    u, b = inputs.random_modes3d(*shape, 0.03, seed=9)
    out = []
    for bx, by, xcd in ((0, 0, -1), (64, 4, 0), (64, 4, 1), (32, 8, 1), (16, 16, 0), (16, 16, 1),
                        (128, 2, 1), (1, 1, 0), (256, 1, 1)):
        s = R.Solver3D(*shape, 0.54, 0.58, storage=storage, inplace=inplace)
        if bx:
            s.set_launch(bx, by, xcd)
        s.init(dev(u), dev(b))
        s.step(7)
        out.append(gpu_fields(s))
        s.close()
    for g in out[1:]:
        for k in FIELDS:
            assert np.array_equal(g[k], out[0][k]), k


def test_3d_uniform_state_is_fixed():
    R = rrmhd()
    shape = (8, 6, 4)
    u = np.zeros((3, 4, 6, 8)) + np.array([0.03, -0.02, 0.01])[:, None, None, None]
    b = np.zeros_like(u) + np.array([0.02, 0.01, -0.03])[:, None, None, None]
    s = R.Solver3D(*shape, 0.6, 0.7)
    s.init(dev(u), dev(b))
    s.step(10)
    g = gpu_fields(s)
    assert np.allclose(g["rho"], 1, atol=2e-7)
    assert np.allclose(np.stack([g["ux"], g["uy"], g["uz"]]), u, atol=1e-8)
    assert np.allclose(np.stack([g["bx"], g["by"], g["bz"]]), b, atol=1e-8)
    s.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_3d_full_size_sampled(storage):
    """256^3 turbulence, 3 steps, 40 sampled nodes (plus corners) against the
    oracle on 7^3 patches (after k steps a node depends only on nodes within
    distance k in each direction)."""
    n, k, tau = 256, 3, 0.52
    note(f"3D full size {n}^3 {storage}")
    R = rrmhd()
    u, b = inputs.turbulence3d(n, 0.04)
    s = R.Solver3D(n, n, n, tau, tau, storage=storage)
    s.init(dev(u), dev(b))
    s.step(k)
    rho, uu, bb = s.moments()
    idx = inputs.counter_u64(5, 77, np.arange(120)) % np.uint64(n)
    pts = [tuple(int(v) for v in idx[3 * i:3 * i + 3]) for i in range(40)]
    pts += [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 0)]
    got = []
    for x, y, z in pts:
        got.append([float(rho[z, y, x])] + [float(uu[a, z, y, x]) for a in range(3)]
                   + [float(bb[a, z, y, x]) for a in range(3)])
    got = np.array(got)
    s.close()
    del rho, uu, bb
    torch.cuda.empty_cache()
    ref = []
    w = 2 * k + 1
    for x, y, z in pts:
        zs, ys, xs = [(np.arange(c - k, c + k + 1)) % n for c in (z, y, x)]
        pu = u[:, zs][:, :, ys][:, :, :, xs]
        pb = b[:, zs][:, :, ys][:, :, :, xs]
        o = oracle.Oracle3D(w, w, w, tau, tau)
        o.init(pu, pb)
        o.step(k)
        r, ou, ob = o.moments()
        ref.append([r[k, k, k]] + [ou[a, k, k, k] for a in range(3)] + [ob[a, k, k, k] for a in range(3)])
    ref = np.array(ref)
    scale = np.array([1.0] + [0.04] * 6)
    err = np.max(np.abs(got - ref) / scale, axis=0)
    note(f"  max |err| / field scale: {err}")
    assert np.all(err < (1e-6 if storage == "f32" else 3e-3)), err


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("shape", [(7, 5, 3), (1, 1, 9), (2, 2, 2), (1, 1, 1), (37, 11, 5)])
def test_3d_inplace_bitwise(storage, shape):
    """One buffer, alternating step forms: the moments and diagnostics equal
    the two-buffer handle's bit for bit at odd and even step counts."""
    note(f"3D in-place {shape} {storage}")
    R = rrmhd()
    u, b = inputs.random_modes3d(*shape, 0.04, seed=sum(shape) + 3)
    two = R.Solver3D(*shape, 0.55, 0.6, storage=storage)
    one = R.Solver3D(*shape, 0.55, 0.6, storage=storage, inplace=True)
    for s in (two, one):
        s.init(dev(u), dev(b))
    for k in (1, 2, 5, 6):
        two.step(k - two.step_count)
        one.step(k - one.step_count)
        ga, gb = gpu_fields(two), gpu_fields(one)
        for f in FIELDS:
            assert np.array_equal(ga[f], gb[f]), (k, f)
        assert two.diagnostics() == one.diagnostics()
    two.close(); one.close()


def test_3d_inplace_holds_one_buffer():
    R = rrmhd()
    n = 192
    torch.cuda.synchronize()
    taken = []
    for inplace in (False, True):
        free0 = torch.cuda.mem_get_info()[0]
        s = R.Solver3D(n, n, n, 0.55, 0.6, inplace=inplace)
        torch.cuda.synchronize()
        taken.append(free0 - torch.cuda.mem_get_info()[0])
        s.close()
        torch.cuda.synchronize()
    state = n ** 3 * 48 * 4
    note(f"  device bytes: two buffers {taken[0]}, one buffer {taken[1]} (state {state})")
    assert abs(taken[0] - 2 * state) < 0.02 * state
    assert abs(taken[1] - state) < 0.02 * state
