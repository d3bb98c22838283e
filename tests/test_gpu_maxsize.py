"""The largest two-dimensional grids the library accepts: 32768 x 32767
nodes in FP32 storage and 46340 x 46340 in FP16 (each plane just under
4 GiB, the limit of the 32-bit in-plane byte offsets; 163 GB of populations
in two buffers; FP16 runs the two-node kernel).  After three
steps, sampled nodes, including the last nodes of the grid at the top of the
offset range, match the FP64 oracle run on 7 x 7 patches around them (after
k steps a node depends only on nodes within distance k).  The fields are
built on the device; the test is skipped when the card has less free memory
than it needs."""
import math

import numpy as np
import pytest

import oracle
from paper_2602_14667_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K, TAU, A = 3, 0.52, 0.04


def fields_np(xs, ys, NX, NY):
    """u, b of the test at node coordinates (arrays of x and y indices)."""
    x = 2 * math.pi * xs / NX
    y = 2 * math.pi * ys / NY
    u = np.stack([-A * np.sin(y) + 0.01 * np.cos(3 * x + y), A * np.sin(x) + 0.01 * np.sin(2 * y)])
    b = np.stack([-A * np.sin(y), A * np.sin(2 * x) + 0.01 * np.cos(x - 2 * y)])
    return u, b


@pytest.mark.parametrize("storage,NX,NY,need_gib,tol", [("f32", 32768, 32767, 215, 1e-6),
                                                      ("f16", 46340, 46340, 245, 3e-3)])
def test_largest_grid_sampled(storage, NX, NY, need_gib, tol):
    from paper_2602_14667_amd import rrmhd as R
    R.lib()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < need_gib * 2 ** 30:
        pytest.skip(f"needs ~{need_gib} GiB of free device memory, {free / 2 ** 30:.0f} GiB free")
    print(f"[gpu] largest {storage} grid {NX}x{NY}", flush=True)
    s = R.Solver(NX, NY, TAU, TAU, storage=storage)
    X = (torch.arange(NX, dtype=torch.float64, device="cuda") * (2 * math.pi / NX))[None, :]
    ys = torch.arange(NY, dtype=torch.float64, device="cuda") * (2 * math.pi / NY)
    u = torch.empty((2, NY, NX), dtype=torch.float64, device="cuda")
    b = torch.empty_like(u)
    for r0 in range(0, NY, 2048):  # row chunks keep the temporaries small
        Y = ys[r0:r0 + 2048, None]
        u[0, r0:r0 + 2048] = -A * torch.sin(Y) + 0.01 * torch.cos(3 * X + Y)
        u[1, r0:r0 + 2048] = A * torch.sin(X) + 0.01 * torch.sin(2 * Y)
        b[0, r0:r0 + 2048] = -A * torch.sin(Y) + 0.0 * X
        b[1, r0:r0 + 2048] = A * torch.sin(2 * X) + 0.01 * torch.cos(X - 2 * Y)
    s.init(u, b)
    del u, b, X, Y, ys
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    s.step(K)
    rho, uu, bb = s.moments()
    idx = inputs.counter_u64(11, 5, np.arange(60))
    pts = [(int(idx[2 * i] % NX), int(idx[2 * i + 1] % NY)) for i in range(30)]
    pts += [(0, 0), (NX - 1, NY - 1), (NX - 1, 0), (0, NY - 1), (NX - 2, NY - 1)]
    got = np.array([[float(rho[y, x])] + [float(uu[a, y, x]) for a in range(2)]
                    + [float(bb[a, y, x]) for a in range(2)] for x, y in pts])
    s.close()
    del rho, uu, bb
    torch.cuda.empty_cache()
    w = 2 * K + 1
    ref = []
    for x, y in pts:
        px = (np.arange(x - K, x + K + 1) % NX)[None, :].repeat(w, 0)
        py = (np.arange(y - K, y + K + 1) % NY)[:, None].repeat(w, 1)
        pu, pb = fields_np(px, py, NX, NY)
        o = oracle.Oracle(w, w, TAU, TAU)
        o.init(pu, pb)
        o.step(K)
        r, ou, ob = o.moments()
        o.close()
        ref.append([r[K, K], ou[0, K, K], ou[1, K, K], ob[0, K, K], ob[1, K, K]])
    ref = np.array(ref)
    err = np.max(np.abs(got - ref) / np.array([1.0, A, A, A, A]), axis=0)
    print(f"[gpu]   max |err| / field scale: {err}", flush=True)
    assert np.all(err < tol), err


def abc_np(xs, ys, zs, n, m):
    """ABC field with m wavelengths per side at node indices, vector rms A."""
    x, y, z = (2 * math.pi * v / n for v in (xs, ys, zs))
    s = A / math.sqrt(3.0)
    return np.stack([s * (np.sin(m * z) + np.cos(m * y)), s * (np.sin(m * x) + np.cos(m * z)),
                     s * (np.sin(m * y) + np.cos(m * x))])


@pytest.mark.parametrize("storage,tol", [("f32", 1e-6), ("f16", 3e-3)])
def test_3d_single_buffer_960_sampled(storage, tol):
    """The three-dimensional single-buffer handle on a 960^3 box (885 M
    nodes; 170 GB of FP32 populations in one buffer), ABC flow and field
    built on the device: after three steps (the handle between its two step
    forms), sampled nodes match the FP64 oracle on 7^3 patches."""
    from paper_2602_14667_amd import rrmhd as R
    R.lib()
    n = 960
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    need = 215 if storage == "f32" else 150
    if free < need * 2 ** 30:
        pytest.skip(f"needs ~{need} GiB of free device memory, {free / 2 ** 30:.0f} GiB free")
    print(f"[gpu] 3D single buffer {n}^3 {storage}", flush=True)
    s = R.Solver3D(n, n, n, TAU, TAU, storage=storage, inplace=True)
    x = torch.arange(n, dtype=torch.float64, device="cuda") * (2 * math.pi / n)
    sc = A / math.sqrt(3.0)

    def field(m):
        f = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda")
        sm, cm = torch.sin(m * x), torch.cos(m * x)
        f[0] = sc * (sm[:, None, None] + cm[None, :, None])   # sin z + cos y
        f[1] = sc * (sm[None, None, :] + cm[:, None, None])   # sin x + cos z
        f[2] = sc * (sm[None, :, None] + cm[None, None, :])   # sin y + cos x
        return f

    u = field(1)
    b = field(2)
    s.init(u, b)
    del u, b
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    s.step(K)
    rho, uu, bb = s.moments()
    idx = inputs.counter_u64(13, 9, np.arange(60))
    pts = [tuple(int(v) % n for v in idx[3 * i:3 * i + 3]) for i in range(20)]
    pts += [(0, 0, 0), (n - 1, n - 1, n - 1), (n - 1, 0, n - 1)]
    got = np.array([[float(rho[z, y, x_])] + [float(uu[a, z, y, x_]) for a in range(3)]
                    + [float(bb[a, z, y, x_]) for a in range(3)] for x_, y, z in pts])
    s.close()
    del rho, uu, bb
    torch.cuda.empty_cache()
    w = 2 * K + 1
    ref = []
    for x_, y, z in pts:
        ax = np.arange(-K, K + 1)
        Z, Y, X = np.meshgrid((z + ax) % n, (y + ax) % n, (x_ + ax) % n, indexing="ij")
        o = oracle.Oracle3D(w, w, w, TAU, TAU)
        o.init(abc_np(X, Y, Z, n, 1), abc_np(X, Y, Z, n, 2))
        o.step(K)
        r, ou, ob = o.moments()
        o.close()
        ref.append([r[K, K, K]] + [ou[a, K, K, K] for a in range(3)] + [ob[a, K, K, K] for a in range(3)])
    err = np.max(np.abs(got - np.array(ref)) / np.array([1.0] + [A] * 6), axis=0)
    print(f"[gpu]   max |err| / field scale: {err}", flush=True)
    assert np.all(err < tol), err
