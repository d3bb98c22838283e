"""Handles on a stream other than torch's current one: the binding orders the
handle's stream after torch's current stream before a call that reads caller
tensors, keeps those tensors alive for the handle's stream, and makes torch's
current stream wait for results.  Results equal those of a handle on the
current stream, bit for bit."""
import numpy as np
import pytest

from paper_2602_14667_amd import inputs
from test_gpu_parity import FIELDS, gpu_moments, note, rrmhd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _fields_on_current_stream(u, b):
    """Inputs produced by work on torch's current stream just before use."""
    ut = torch.zeros(u.shape, dtype=torch.float64, device="cuda")
    bt = torch.zeros(b.shape, dtype=torch.float64, device="cuda")
    ut.add_(torch.from_numpy(u).cuda())
    bt.add_(torch.from_numpy(b).cuda())
    return ut, bt


def test_solver_on_side_stream_bitwise():
    note("solver on a non-current stream")
    R = rrmhd()
    nx, ny = 200, 120
    u, b = inputs.random_modes(nx, ny, 0.04, seed=9)
    ref = R.Solver(nx, ny, 0.55, 0.6)
    ut, bt = _fields_on_current_stream(u, b)
    ref.init(ut, bt)
    ref.step(30)
    want = gpu_moments(ref)
    ref.close()
    side = torch.cuda.Stream()
    s = R.Solver(nx, ny, 0.55, 0.6, stream=side)
    ut, bt = _fields_on_current_stream(u, b)
    s.init(ut, bt)
    del ut, bt  # released to the allocator while the side stream may still read them
    junk = torch.full((4, ny, nx), float("nan"), dtype=torch.float64, device="cuda")
    s.step(30)
    rho, uu, bb = s.moments()
    got = {"rho": rho.cpu().numpy(), "ux": uu[0].cpu().numpy(), "uy": uu[1].cpu().numpy(),
           "bx": bb[0].cpu().numpy(), "by": bb[1].cpu().numpy()}
    for k in FIELDS:
        assert np.array_equal(got[k], want[k]), k
    jz, wz = s.current_vorticity()
    assert torch.isfinite(jz).all() and torch.isfinite(wz).all()
    s.close()
    del junk


def test_batch_on_side_stream_bitwise():
    note("batch on a non-current stream")
    R = rrmhd()
    shapes = [(64, 64), (96, 40)]
    fields = [inputs.random_modes(nx, ny, 0.04, seed=20 + d) for d, (nx, ny) in enumerate(shapes)]
    out = []
    for stream in (None, torch.cuda.Stream()):
        bt = R.Batch(shapes, [0.55, 0.6], [0.6, 0.57], stream=stream)
        for d, (u, b) in enumerate(fields):
            ut, btf = _fields_on_current_stream(u, b)
            bt.init(d, ut, btf)
            del ut, btf
        bt.step(20)
        out.append([[t.cpu().numpy() for t in bt.moments(d)] for d in range(len(shapes))])
        bt.close()
    for d in range(len(shapes)):
        for a, c in zip(out[0][d], out[1][d]):
            assert np.array_equal(a, c), d
