"""Kernel coverage through the debug poison mode: with the destination
buffer filled with NaN before every step, every step path still gives the
unpoisoned run's state bit for bit, and the diagnostics stay finite, so each
step writes every stored value of every node (no node, plane or tile edge
left unwritten)."""
import numpy as np
import pytest

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


def state(s):
    rho, u, b = s.moments()
    torch.cuda.synchronize()
    r, u, b = rho.cpu().numpy(), u.cpu().numpy(), b.cpu().numpy()
    return dict(rho=r, ux=u[0], uy=u[1], bx=b[0], by=b[1])


def run(R, nx, ny, storage, steps, poison, launch=None, graph=0, **kw):
    u, b = inputs.random_modes(nx, ny, 0.04, seed=nx + ny)
    if kw.get("walls"):
        b[1] += 0.01
    s = R.Solver(nx, ny, 0.53, 0.57, storage=storage, **kw)
    if launch:
        s.set_launch(*launch)
    if graph:
        s.set_graph_chunk(graph)
    s.set_debug_poison(poison)
    s.init(dev(u), dev(b))
    s.step(steps)
    out = state(s)
    d = s.diagnostics()
    s.close()
    return out, d


@pytest.mark.parametrize("storage", ["f32", "f16", "f16sr"])
@pytest.mark.parametrize("shape", [(130, 66), (67, 45), (2, 3), (1, 7), (512, 9)])
@pytest.mark.parametrize("launch", [None, (64, 4, 1, 0, 0), (32, 2, 3, 1, 1), (16, 16, 1, 0, 5),
                                    (1, 1, 1, 0, 5)])
def test_poisoned_destination_is_fully_written(storage, shape, launch):
    R = rrmhd()
    nx, ny = shape
    a, da = run(R, nx, ny, storage, 5, False, launch)
    p, dp = run(R, nx, ny, storage, 5, True, launch)
    for k in FIELDS:
        assert np.array_equal(a[k], p[k]), k
    assert da == dp and all(np.isfinite(v) for v in dp)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_poison_walls_and_force(storage):
    R = rrmhd()
    kw = dict(walls=True, force=(1e-5, 0.0), b_wall=(0.0, 0.01))
    for shape in ((9, 24), (130, 33)):
        a, _ = run(R, *shape, storage, 6, False, **kw)
        p, dp = run(R, *shape, storage, 6, True, **kw)
        for k in FIELDS:
            assert np.array_equal(a[k], p[k]), (shape, k)
        assert all(np.isfinite(v) for v in dp)


def test_poison_graph_replay():
    R = rrmhd()
    a, _ = run(R, 96, 40, "f32", 12, False, graph=4)
    p, _ = run(R, 96, 40, "f32", 12, True, graph=4)
    for k in FIELDS:
        assert np.array_equal(a[k], p[k]), k


def test_poison_closure_step():
    note("poison + closure")
    R = rrmhd()
    rng = np.random.default_rng(2)
    params = np.zeros(4931)
    params[:512] = 0.3 * rng.standard_normal(512)
    params[576:4672] = 0.1 * rng.standard_normal(4096)
    params[4736:4928] = 0.1 * rng.standard_normal(192)
    norm = np.concatenate([[1.0, 0, 0, 0, 0, 0, 0, 0], [0.01, 0.04, 0.04, 0.04, 0.04, 1e-4, 1e-4, 1e-4],
                           [1e-5, 1e-5, 1e-5]])
    out = []
    for poison in (False, True):
        u, b = inputs.random_modes(100, 37, 0.04, seed=3)
        s = R.Solver(100, 37, 0.53, 0.57)
        s.closure_set(torch.tensor(params, dtype=torch.float32, device="cuda"),
                      torch.tensor(norm, dtype=torch.float32, device="cuda"))
        s.closure_enable(True)
        s.set_debug_poison(poison)
        s.init(dev(u), dev(b))
        s.step(5)
        out.append(state(s))
        s.close()
    for k in FIELDS:
        assert np.array_equal(out[0][k], out[1][k]), k


def test_poison_refused_for_single_buffer():
    R = rrmhd()
    s = R.Solver(32, 32, 0.56, 0.56, inplace=True)
    assert R.lib().rrmhd_set_debug_poison(s._h, 1) == R.EINVAL
    assert R.lib().rrmhd_set_debug_poison(s._h, 0) == R.OK
    s.close()


def run3(R, shape, storage, poison, launch=None):
    u, b = inputs.random_modes3d(*shape, 0.04, seed=sum(shape))
    s = R.Solver3D(*shape, 0.55, 0.6, storage=storage)
    if launch:
        s.set_launch(*launch)
    s.set_debug_poison(poison)
    s.init(dev(u), dev(b))
    s.step(4)
    rho, uu, bb = s.moments()
    torch.cuda.synchronize()
    out = [rho.cpu().numpy(), uu.cpu().numpy(), bb.cpu().numpy()]
    d = s.diagnostics()
    s.close()
    return out, d


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("shape", [(7, 5, 3), (37, 11, 5), (1, 1, 1), (2, 2, 2), (130, 3, 2)])
@pytest.mark.parametrize("launch", [None, (64, 4), (16, 16), (1, 1)])
def test_3d_poisoned_destination_is_fully_written(storage, shape, launch):
    R = rrmhd()
    a, da = run3(R, shape, storage, False, launch)
    p, dp = run3(R, shape, storage, True, launch)
    for x, y in zip(a, p):
        assert np.array_equal(x, y)
    assert da == dp and all(np.isfinite(v) for v in dp)


def test_3d_poison_refused_for_single_buffer():
    R = rrmhd()
    s = R.Solver3D(8, 8, 8, 0.56, 0.56, inplace=True)
    assert R.lib().rrmhd3d_set_debug_poison(s._h, 1) == R.EINVAL
    s.close()
