"""GPU tests of the batched ensemble (one persistent launch per step over
many uneven periodic domains): bitwise equality with standalone runs, with
the hipGraph path and across tile shapes; sampled domains against the FP64
oracle."""
import numpy as np
import pytest

import oracle
from paper_2602_14667_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = [(64, 64), (96, 96), (128, 128), (40, 72), (33, 17), (256, 32)]
TAUS_F = [0.51, 0.55, 0.6, 0.52, 0.58, 0.503]
TAUS_M = [0.53, 0.51, 0.57, 0.6, 0.52, 0.59]


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def R():
    from paper_2602_14667_amd import rrmhd
    rrmhd.lib()
    return rrmhd


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def fields(d, nx, ny):
    return inputs.random_modes(nx, ny, 0.05, seed=77 + d)


def moments_np(t3):
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in t3]


def make_batch(storage="f32"):
    rr = R()
    b = rr.Batch(SHAPES, TAUS_F, TAUS_M, storage=storage)
    for d, (nx, ny) in enumerate(SHAPES):
        u, bf = fields(d, nx, ny)
        b.init(d, dev(u), dev(bf))
    return b


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batch_equals_standalone_bitwise(storage):
    note(f"batch vs standalone {storage}")
    rr = R()
    b = make_batch(storage)
    b.step(25)
    for d, (nx, ny) in enumerate(SHAPES):
        s = rr.Solver(nx, ny, TAUS_F[d], TAUS_M[d], storage=storage)
        u, bf = fields(d, nx, ny)
        s.init(dev(u), dev(bf))
        s.step(25)
        got = moments_np(b.moments(d))
        ref = moments_np(s.moments())
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), d
        s.close()
    b.close()


def test_batch_graph_and_tile_shape_bitwise():
    note("batch graph chunks and tile shapes")
    a = make_batch()
    a.step(30)
    ref = [moments_np(a.moments(d)) for d in range(len(SHAPES))]
    a.close()
    # (graph chunk, tile width, workgroups, tiles per dynamic fetch); the
    # dynamic cases run many launches in a row (the counters must return to
    # zero after each) inside and outside captured graphs
    for chunk, bx, grid, fetch in ((10, 0, 0, 0), (4, 32, 0, 0), (7, 256, 300, 0),
                                   (0, 64, 17, 0), (0, 0, -1, 0), (10, 0, 64, 1),
                                   (7, 32, 5, 4), (0, 128, -1, 3), (4, 64, 2048, 1)):
        b = make_batch()
        b.set_shape(-1, bx=bx, grid=grid)
        b.set_fetch(fetch)
        b.set_graph_chunk(chunk)
        b.step(13)
        b.step(17)
        for d in range(len(SHAPES)):
            got = moments_np(b.moments(d))
            for g, r in zip(got, ref[d]):
                assert np.array_equal(g, r), (chunk, bx, grid, fetch, d)
        assert b.info()["steps"] == 30
        b.close()


def per_field_errors(got, ref):
    """rel L2 per field (rho, u_x, u_y, b_x, b_y) of (rho, u, b) triples."""
    g = [got[0], got[1][0], got[1][1], got[2][0], got[2][1]]
    r = [ref[0], ref[1][0], ref[1][1], ref[2][0], ref[2][1]]
    names = ("rho", "ux", "uy", "bx", "by")
    return {n: float(np.linalg.norm(a - c) / np.linalg.norm(c)) for n, a, c in zip(names, g, r)}


def test_batch_domains_against_oracle():
    note("batch vs oracle")
    b = make_batch()
    b.step(40)
    for d in (1, 3, 4):
        nx, ny = SHAPES[d]
        u, bf = fields(d, nx, ny)
        o = oracle.Oracle(nx, ny, TAUS_F[d], TAUS_M[d])
        o.init(u, bf)
        o.step(40)
        ref = o.moments()
        got = moments_np(b.moments(d))
        for k, e in per_field_errors(got, ref).items():
            assert e < 1e-6, (d, k, e)
        ek, em, dv = b.diagnostics(d)
        rk, rm, rd = o.diagnostics()
        assert abs(ek / rk - 1) < 2e-6 and abs(em / rm - 1) < 2e-6
    b.close()


def test_batch_full_ensemble_sampled():
    """The 256-domain ensemble (sides 64..1024, tau in [0.501, 0.6], OT or
    turbulence), 20 steps in 2 graph chunks; sampled domains bitwise equal to
    standalone runs and small ones against the oracle."""
    rr = R()
    doms = inputs.batch_domains(256, seed=0)
    shapes = [(x["side"], x["side"]) for x in doms]
    note(f"full ensemble: {sum(a * b for a, b in shapes)} nodes")
    b = rr.Batch(shapes, [x["tau_f"] for x in doms], [x["tau_m"] for x in doms])
    for d, x in enumerate(doms):
        u, bf = inputs.batch_fields(x)
        b.init(d, dev(u), dev(bf))
    b.set_graph_chunk(10)
    b.step(20)
    torch.cuda.synchronize()
    picks = sorted(range(256), key=lambda d: shapes[d][0])
    for d in (picks[0], picks[1], picks[128], picks[-1]):
        x = doms[d]
        u, bf = inputs.batch_fields(x)
        s = rr.Solver(x["side"], x["side"], x["tau_f"], x["tau_m"])
        s.init(dev(u), dev(bf))
        s.step(20)
        got = moments_np(b.moments(d))
        ref = moments_np(s.moments())
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), d
        s.close()
        if x["side"] <= 128:
            o = oracle.Oracle(x["side"], x["side"], x["tau_f"], x["tau_m"])
            o.init(u, bf)
            o.step(20)
            for k, e in per_field_errors(got, o.moments()).items():
                assert e < 1e-6, (d, k, e)
    b.close()


def test_autotune_preserves_state_and_caches(tmp_path):
    note("autotune single domain")
    rr = R()
    n = 256
    u, bf = inputs.turbulence(n, 0.04)
    a = rr.Solver(n, n, 0.52, 0.55)
    a.init(dev(u), dev(bf))
    a.step(10)
    cache = str(tmp_path / "tune.json")
    best = a.autotune(cache, trials=5)
    assert best["bx"] * best["by"] <= 256 and best["ms"] > 0
    assert a.step_count == 10
    a.step(10)
    got = moments_np(a.moments())
    c = rr.Solver(n, n, 0.52, 0.55)
    c.init(dev(u), dev(bf))
    c.step(20)
    ref = moments_np(c.moments())
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)
    import json
    with open(cache) as fh:
        entries = json.load(fh)
    # periodic two-buffer handles keep row-interleaved planes: their own key
    assert any(k.endswith(f"/step_rows/{n}x{n}/f32") for k in entries)
    # a second handle takes the cached entry
    again = c.autotune(cache, trials=5)
    assert (again["bx"], again["by"], again["xcd"]) == (best["bx"], best["by"],
                                                        best["xcd"])
    # tuning before init leaves the handle uninitialised
    e = rr.Solver(96, 64, 0.6, 0.6)
    e.autotune(None, trials=3)
    with pytest.raises(RuntimeError):
        e.step(1)
    a.close(); c.close(); e.close()


def test_batch_autotune_preserves_state(tmp_path):
    note("autotune batch")
    b = make_batch()
    b.step(12)
    b.autotune(str(tmp_path / "tune.json"), trials=3)
    assert b.info()["steps"] == 12
    b.step(8)
    a = make_batch()
    a.step(20)
    for d in range(len(SHAPES)):
        for g, r in zip(moments_np(b.moments(d)), moments_np(a.moments(d))):
            assert np.array_equal(g, r), d
    a.close(); b.close()


def test_environment_overrides(tmp_path, monkeypatch):
    """RRMHD_TILE replaces the default launch shape at create (results stay
    bitwise those of the default shape), RRMHD_DEBUG_POISON turns the poison
    mode on, and RRMHD_AUTOTUNE_CACHE is the cache file of an autotune call
    that passes none."""
    rr = R()
    from test_gpu_parity import dev, gpu_moments
    note("environment overrides")
    n = 96
    u, b = inputs.random_modes(n, n, 0.04, seed=5)
    ref = rr.Solver(n, n, 0.55, 0.6)
    default_shape = ref.get_launch()
    ref.init(dev(u), dev(b))
    ref.step(12)
    want = gpu_moments(ref)
    ref.close()
    monkeypatch.setenv("RRMHD_TILE", "64x4")
    monkeypatch.setenv("RRMHD_DEBUG_POISON", "1")
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("RRMHD_AUTOTUNE_CACHE", str(cache))
    s = rr.Solver(n, n, 0.55, 0.6)
    assert s.get_launch()[:3] == (64, 4, 1) and s.get_launch() != default_shape
    s.init(dev(u), dev(b))
    s.step(12)
    got = gpu_moments(s)
    for k in want:
        assert np.array_equal(got[k], want[k]), k
    s.autotune(None, trials=2)
    assert cache.exists() and "step" in cache.read_text()
    s.close()
