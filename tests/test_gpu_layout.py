"""The two population layouts on the GPU: periodic two-buffer handles keep
their 19 planes row-interleaved by default (each grid row holds its 19 plane
rows side by side), RRMHD_STORE_PLANAR keeps planes of [ny][nx].  The layout
changes addresses only, so a run in one layout equals the same run in the
other bit for bit: the step in every storage and launch shape (the FP32 and
FP16 two-node and the FP16 four-node updates, whole-row and mixed-row
wavefronts), forcing, the equilibrium ablation, the closure step, graph
replay, moments, diagnostics, the current and vorticity fields, the imposed
fluid state, state copies and checkpoint files moved between the layouts and
a single-buffer handle."""
import numpy as np
import pytest

from paper_2602_14667_amd import inputs
from test_gpu_parity import FIELDS, dev, gpu_moments, note, rrmhd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def both(nx, ny, tau_f, tau_m, storage="f32", **kw):
    R = rrmhd()
    return (R.Solver(nx, ny, tau_f, tau_m, storage=storage, **kw),
            R.Solver(nx, ny, tau_f, tau_m, storage=storage, layout="planar", **kw))


def assert_same(a, b, where):
    ga, gb = gpu_moments(a), gpu_moments(b)
    for k in FIELDS:
        assert np.array_equal(ga[k], gb[k]), (where, k)


SHAPES = [(128, 2, 1, 0, 5), (128, 1, 1, 0, 5), (64, 4, 1, 2, 5), (32, 8, 1, 0, 5),
          (128, 2, 1, 0, 1), (32, 8, 1, 0, 1), (16, 16, 2, 1, 1), (256, 1, 1, 0, 7),
          (128, 1, 1, 0, 9), (64, 2, 2, 2, 9), (32, 4, 1, 0, 13), (64, 1, 1, 0, 11)]


@pytest.mark.parametrize("storage", ["f32", "f16", "f16sr"])
@pytest.mark.parametrize("size", [(130, 67), (64, 48), (2, 3), (1, 1), (520, 18), (67, 2), (4, 5), (8, 3), (12, 7)])
def test_layouts_bitwise_across_shapes(storage, size):
    nx, ny = size
    note(f"layouts {nx}x{ny} {storage}")
    u, b = inputs.random_modes(nx, ny, 0.05, seed=3 * nx + ny)
    rows, planar = both(nx, ny, 0.53, 0.57, storage)
    for s in (rows, planar):
        s.init(dev(u), dev(b))
    assert_same(rows, planar, "init")
    for k, shape in enumerate(SHAPES):
        rows.set_launch(*shape)
        planar.set_launch(*SHAPES[-1 - k])  # the planar kernels in other shapes
        rows.step(3)
        planar.step(3)
        assert_same(rows, planar, shape)
    ra, pa = rows.diagnostics(), planar.diagnostics()
    assert ra == pa
    rows.close()
    planar.close()


def test_layouts_default_shapes_at_size():
    """The default launches at 1024 x 512 (two nodes per thread in FP32
    storage, four in FP16), forcing included, over 20 steps."""
    n, m = 1024, 512
    u, b = inputs.random_modes(n, m, 0.04, seed=9)
    for storage in ("f32", "f16"):
        for force in ((0.0, 0.0), (1e-5, -2e-6)):
            note(f"layouts default shape {storage} force {force}")
            rows, planar = both(n, m, 0.52, 0.55, storage, force=force)
            assert rows.get_launch()[4] == (5 if storage == "f32" else 9)
            for s in (rows, planar):
                s.init(dev(u), dev(b))
                s.step(20)
            assert_same(rows, planar, (storage, force))
            rows.close()
            planar.close()


def test_layouts_equilibrium_ablation_and_graphs():
    nx, ny = 96, 40
    u, b = inputs.random_modes(nx, ny, 0.05, seed=4)
    note("layouts: equilibrium ablation, graph replay")
    rows, planar = both(nx, ny, 0.54, 0.56, "f32", equilibrium="full_maxwell")
    rows.set_graph_chunk(5)
    for s in (rows, planar):
        s.init(dev(u), dev(b))
        s.step(23)
    assert_same(rows, planar, "ablation")
    rows.close()
    planar.close()


def test_layouts_closure_step():
    from test_gpu_closure import dev32, features, init_params, norm_of
    import oracle  # noqa: F401  (the parameter layout of the network)
    note("layouts: closure step")
    nx, ny = 100, 34
    u, b = inputs.random_modes(nx, ny, 0.05, seed=6)
    rng = np.random.default_rng(6)
    p = dev32(init_params(rng))
    nm = dev32(norm_of(features(rng, 4096)))
    for storage in ("f32", "f16"):
        rows, planar = both(nx, ny, 0.55, 0.55, storage)
        for s in (rows, planar):
            s.init(dev(u), dev(b))
            s.closure_set(p, nm)
            s.closure_enable(True)
            s.step(9)
        assert_same(rows, planar, ("closure", storage))
        rows.close()
        planar.close()


def test_layouts_fields_and_imposed_state():
    note("layouts: current/vorticity fields, imposed fluid state")
    nx, ny = 72, 30
    u, b = inputs.random_modes(nx, ny, 0.05, seed=8)
    rows, planar = both(nx, ny, 0.55, 0.6)
    for s in (rows, planar):
        s.init(dev(u), dev(b))
        s.step(4)
    for a, c in zip(rows.current_vorticity(), planar.current_vorticity()):
        assert torch.equal(a, c)
    rho = dev(1.0 + 0.01 * np.cos(np.arange(nx) * 0.3)[None, :] * np.ones((ny, 1)))
    j = dev(0.02 * np.stack([np.sin(np.arange(ny) * 0.2)[:, None] * np.ones((1, nx)),
                             np.cos(np.arange(nx) * 0.1)[None, :] * np.ones((ny, 1))]))
    _, _, bb = rows.moments()
    for s in (rows, planar):
        s.impose_fluid(rho, j, bb)
        s.step(3)
    assert_same(rows, planar, "imposed")
    rows.close()
    planar.close()


def test_layouts_state_copies_and_checkpoints(tmp_path):
    """A row-interleaved state saved (device copy and checkpoint file) and
    loaded into a planar handle and a single-buffer handle, and back; every
    continuation equals the uninterrupted run."""
    R = rrmhd()
    nx, ny = 90, 52
    note("layouts: state copies and checkpoint files")
    u, b = inputs.random_modes(nx, ny, 0.05, seed=10)
    for storage in ("f32", "f16"):
        ref = R.Solver(nx, ny, 0.53, 0.56, storage=storage)
        ref.init(dev(u), dev(b))
        ref.step(6)
        buf = torch.empty(ref.state_bytes(), dtype=torch.uint8, device="cuda")
        ref.save_state(buf)
        path = str(tmp_path / f"ck_{storage}.rrmhd")
        ref.save(path)
        ref.step(5)
        targets = [R.Solver(nx, ny, 0.53, 0.56, storage=storage, layout="planar"),
                   R.Solver(nx, ny, 0.53, 0.56, storage=storage, inplace=True),
                   R.Solver(nx, ny, 0.53, 0.56, storage=storage)]
        for t in targets:
            t.load_state(buf, 6)
            t.step(5)
            assert_same(ref, t, ("state copy", storage))
            t.load(path)
            t.step(5)
            assert_same(ref, t, ("checkpoint", storage))
        # planar -> row-interleaved through a file
        p2 = str(tmp_path / f"ck2_{storage}.rrmhd")
        targets[0].load(path)
        targets[0].save(p2)
        back = targets[2]
        back.load(p2)
        back.step(5)
        assert_same(ref, back, ("planar file into rows", storage))
        for t in targets:
            t.close()
        ref.close()


def test_layouts_poison_coverage():
    """The debug poison mode on a row-interleaved handle: the NaN fill of the
    destination buffer (gaps between plane rows included) never reaches the
    state, in both storages and with the two-node and one-node updates."""
    note("layouts: poison coverage")
    nx, ny = 98, 21
    u, b = inputs.random_modes(nx, ny, 0.05, seed=12)
    for storage in ("f32", "f16"):
        for shape in ((128, 2, 1, 0, 5), (32, 8, 1, 0, 1)):
            rows, planar = both(nx, ny, 0.53, 0.57, storage)
            rows.set_debug_poison(True)
            rows.set_launch(*shape)
            for s in (rows, planar):
                s.init(dev(u), dev(b))
                s.step(7)
            assert_same(rows, planar, ("poison", storage, shape))
            assert all(np.isfinite(v) for v in rows.diagnostics())
            rows.close()
            planar.close()
