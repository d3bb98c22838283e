"""Graph replay of the single-domain step (rrmhd_set_graph_chunk): runs of
chunk steps captured once into a hipGraph and replayed.  Every replay is
checked bit for bit against plain launches of the same steps, with eager
work (moments, diagnostics) and synchronisations between replays."""
import numpy as np
import pytest

from paper_2602_14667_amd import inputs
from test_gpu_parity import FIELDS, dev, gpu_moments, note, rrmhd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def same(a, b, where):
    ga, gb = gpu_moments(a), gpu_moments(b)
    for k in FIELDS:
        assert np.array_equal(ga[k], gb[k]), (where, k)


def drive(ref, g, plan):
    for n in plan:
        ref.step(n)
        g.step(n)
        same(ref, g, (n, g.step_count))
        assert ref.step_count == g.step_count
        ref.diagnostics(allow_nonfinite=True)
        g.diagnostics(allow_nonfinite=True)


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("chunk", [10, 7])
def test_graph_periodic_bitwise(storage, chunk):
    note(f"graph periodic {storage} chunk {chunk}")
    R = rrmhd()
    n = 96
    u, b = inputs.turbulence(n, 0.04)
    ref = R.Solver(n, n, 0.52, 0.55, storage=storage)
    g = R.Solver(n, n, 0.52, 0.55, storage=storage)
    g.set_graph_chunk(chunk)
    for s in (ref, g):
        s.init(dev(u), dev(b))
    drive(ref, g, [25, 3, 31, chunk, 2 * chunk + 1])
    ref.close(); g.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_graph_walls_force_bitwise(storage):
    note(f"graph walls+force {storage}")
    R = rrmhd()
    h = inputs.Hartmann(nx=17, ny=24, tau_f=0.8, tau_m=0.75, G=1e-4, Ha=4.0)
    u, b = inputs.random_modes(17, 24, 0.03, seed=4)
    b[1] += h.B0
    kw = dict(walls=True, force=(h.G, 0.0), b_wall=(0.0, h.B0), storage=storage)
    ref = R.Solver(17, 24, h.tau_f, h.tau_m, **kw)
    g = R.Solver(17, 24, h.tau_f, h.tau_m, **kw)
    g.set_graph_chunk(5)
    for s in (ref, g):
        s.init(dev(u), dev(b))
    drive(ref, g, [12, 5, 9])
    ref.close(); g.close()


@pytest.mark.parametrize("chunk", [6, 5])
def test_graph_inplace_bitwise(chunk):
    """Single-buffer handle: graphs per starting phase, odd and even chunks."""
    note(f"graph in-place chunk {chunk}")
    R = rrmhd()
    n = 80
    u, b = inputs.turbulence(n, 0.04)
    ref = R.Solver(n, n, 0.52, 0.55)
    g = R.Solver(n, n, 0.52, 0.55, inplace=True)
    g.set_graph_chunk(chunk)
    for s in (ref, g):
        s.init(dev(u), dev(b))
    drive(ref, g, [chunk, 1, chunk + 2, 3 * chunk])
    ref.close(); g.close()


def test_graph_closure_and_new_parameters():
    """The closure step in a graph; new parameters are read by the existing
    graph; turning the closure off drops it."""
    note("graph closure")
    R = rrmhd()
    n = 64
    u, b = inputs.turbulence(n, 0.04)
    rng = np.random.default_rng(3)

    def params(scale):
        p = np.zeros(4931, dtype=np.float32)
        p[:4931 - 3] = scale * rng.standard_normal(4931 - 3) / 8
        return torch.from_numpy(p).cuda()

    # mu[8], sigma[8], sigma_out[3]
    norm = torch.tensor([1.0, 0, 0, 0, 0, 0, 0, 0] + [0.01, 0.04, 0.04, 0.04, 0.04, 0.01, 0.01,
                        0.01] + [1e-4, 1e-4, 1e-4], dtype=torch.float32, device="cuda")
    ref = R.Solver(n, n, 0.55, 0.58)
    g = R.Solver(n, n, 0.55, 0.58)
    g.set_graph_chunk(8)
    p1 = params(1.0)
    for s in (ref, g):
        s.init(dev(u), dev(b))
        s.closure_set(p1, norm)
        s.closure_enable(True)
    drive(ref, g, [16, 3])
    p2 = params(2.0)
    for s in (ref, g):
        s.closure_set(p2, norm)
    drive(ref, g, [8, 9])
    for s in (ref, g):
        s.closure_enable(False)
    drive(ref, g, [16])
    ref.close(); g.close()


def test_graph_dropped_on_launch_shape_change():
    note("graph + set_launch")
    R = rrmhd()
    n = 72
    u, b = inputs.turbulence(n, 0.04)
    ref = R.Solver(n, n, 0.53, 0.56)
    g = R.Solver(n, n, 0.53, 0.56)
    g.set_graph_chunk(4)
    for s in (ref, g):
        s.init(dev(u), dev(b))
    drive(ref, g, [8])
    g.set_launch(32, 4, 2, 1, 0)
    drive(ref, g, [8, 5])
    g.set_graph_chunk(0)
    drive(ref, g, [4])
    ref.close(); g.close()
