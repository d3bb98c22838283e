"""ctypes binding of ``librrmhd.so`` (declared in include/rrmhd.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides device memory (FP64 CUDA/HIP tensors) and the stream.  The
library is loaded on first use; if it is missing the binding raises, there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librrmhd.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ESTATE, EIO = 0, -1, -2, -3, -4, -5, -6
STORE_F32, STORE_F16, STORE_INPLACE, STORE_PLANAR = 0, 1, 0x100, 0x200
STORE_F16_SR = 2
BC_PERIODIC, BC_WALLS_Y = 0, 1
FEQ_ALGORITHM, FEQ_FULL_MAXWELL = 0, 1

EXPORTED = [
    "rrmhd_create", "rrmhd_init", "rrmhd_step", "rrmhd_moments",
    "rrmhd_diagnostics", "rrmhd_diagnostics_noalloc", "rrmhd_invariants", "rrmhd_step_count",
    "rrmhd_state_bytes", "rrmhd_save_state", "rrmhd_load_state", "rrmhd_save", "rrmhd_load",
    "rrmhd_set_launch", "rrmhd_get_launch", "rrmhd_set_stream", "rrmhd_set_equilibrium", "rrmhd_set_graph_chunk",
    "rrmhd_set_debug_poison",
    "rrmhd_destroy", "rrmhd_strerror",
    "rrmhd_last_error_detail", "rrmhd_bandwidth_probe", "rrmhd_sr_encode",
    "rrmhd_batch_create", "rrmhd_batch_init", "rrmhd_batch_step",
    "rrmhd_batch_set_graph_chunk", "rrmhd_batch_set_shape", "rrmhd_batch_set_fetch",
    "rrmhd_batch_moments", "rrmhd_batch_diagnostics", "rrmhd_batch_info",
    "rrmhd_batch_destroy", "rrmhd_batch_last_error_detail",
    "rrmhd_autotune", "rrmhd_batch_autotune",
    "rrmhd_closure_set", "rrmhd_closure_enable", "rrmhd_closure_eval",
    "rrmhd_closure_gelu_table",
    "rrmhd_train_samples", "rrmhd_train_box_filter", "rrmhd_train_impose_fluid",
    "rrmhd_train_create", "rrmhd_train_loss_grad",
    "rrmhd_train_onestep_samples", "rrmhd_train_onestep_loss_grad",
    "rrmhd_train_adam", "rrmhd_train_destroy", "rrmhd_train_last_error_detail",
    "rrmhd_current_vorticity",
    "rrmhd3d_create", "rrmhd3d_init", "rrmhd3d_step", "rrmhd3d_step_count",
    "rrmhd3d_moments", "rrmhd3d_diagnostics", "rrmhd3d_invariants",
    "rrmhd3d_set_launch", "rrmhd3d_destroy", "rrmhd3d_save", "rrmhd3d_load", "rrmhd3d_set_debug_poison",
]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("codec_scale", ctypes.c_float)]


class BC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("force", ctypes.c_double * 2),
                ("b_wall", ctypes.c_double * 2)]


class RRMHDError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        L = lib()
        msg = L.rrmhd_strerror(code).decode()
        det = L.rrmhd_last_error_detail().decode()
        super().__init__(f"{where}: {msg} ({code})" + (f" [{det}]" if det and
                                                      code in (EDEVICE, EIO) else ""))


_lib = None


def lib():
    """Load librrmhd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library not built: {LIB_PATH} is missing "
                "(run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p
        L.rrmhd_create.argtypes = [ctypes.POINTER(Grid), ctypes.c_double,
                                   ctypes.c_double, ctypes.POINTER(BC), vp,
                                   ctypes.POINTER(vp)]
        L.rrmhd_init.argtypes = [vp, dp, dp]
        L.rrmhd_step.argtypes = [vp, i64]
        L.rrmhd_moments.argtypes = [vp, dp, dp, dp]
        L.rrmhd_diagnostics.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]
        L.rrmhd_diagnostics_noalloc.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double)]
        L.rrmhd_invariants.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.rrmhd_step_count.argtypes = [vp, ctypes.POINTER(i64)]
        L.rrmhd_state_bytes.argtypes = [vp]
        L.rrmhd_state_bytes.restype = i64
        L.rrmhd_save_state.argtypes = [vp, vp, i64]
        L.rrmhd_load_state.argtypes = [vp, vp, i64, i64]
        L.rrmhd_save.argtypes = [vp, ctypes.c_char_p]
        L.rrmhd_set_debug_poison.argtypes = [vp, ctypes.c_int]
        L.rrmhd3d_save.argtypes = [vp, ctypes.c_char_p]
        L.rrmhd3d_load.argtypes = [vp, ctypes.c_char_p]
        L.rrmhd3d_set_debug_poison.argtypes = [vp, ctypes.c_int]
        L.rrmhd_load.argtypes = [vp, ctypes.c_char_p]
        L.rrmhd_set_stream.argtypes = [vp, vp]
        ci = ctypes.c_int
        L.rrmhd_set_launch.argtypes = [vp, ci, ci, ci, ci, ci]
        ip = ctypes.POINTER(ci)
        L.rrmhd_get_launch.argtypes = [vp, ip, ip, ip, ip, ip]
        L.rrmhd_set_equilibrium.argtypes = [vp, ci]
        L.rrmhd_set_graph_chunk.argtypes = [vp, ci]
        L.rrmhd3d_create.argtypes = [ci, ci, ci, ci, ctypes.c_double, ctypes.c_double, vp,
                                     ctypes.POINTER(vp)]
        L.rrmhd3d_init.argtypes = [vp, dp, dp]
        L.rrmhd3d_step.argtypes = [vp, i64]
        L.rrmhd3d_step_count.argtypes = [vp, ctypes.POINTER(i64)]
        L.rrmhd3d_moments.argtypes = [vp, dp, dp, dp]
        L.rrmhd3d_diagnostics.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]
        L.rrmhd3d_invariants.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.rrmhd3d_set_launch.argtypes = [vp, ci, ci, ci]
        L.rrmhd3d_destroy.argtypes = [vp]
        L.rrmhd_destroy.argtypes = [vp]
        L.rrmhd_bandwidth_probe.argtypes = [vp, vp, i64, vp]
        L.rrmhd_sr_encode.argtypes = [vp, vp, vp, i64, vp]
        dbl = ctypes.POINTER(ctypes.c_double)
        L.rrmhd_batch_create.argtypes = [ci, ctypes.POINTER(Grid), dbl, dbl, ci,
                                         vp, ctypes.POINTER(vp)]
        L.rrmhd_batch_init.argtypes = [vp, ci, dp, dp]
        L.rrmhd_batch_step.argtypes = [vp, i64]
        L.rrmhd_batch_set_graph_chunk.argtypes = [vp, ci]
        L.rrmhd_batch_set_shape.argtypes = [vp, ci, ci, ci, ci]
        L.rrmhd_batch_set_fetch.argtypes = [vp, ci]
        L.rrmhd_batch_moments.argtypes = [vp, ci, dp, dp, dp]
        L.rrmhd_batch_diagnostics.argtypes = [vp, ci, dbl, dbl, dbl]
        L.rrmhd_batch_info.argtypes = [vp, ctypes.POINTER(i64),
                                       ctypes.POINTER(i64),
                                       ctypes.POINTER(ci), ctypes.POINTER(ci)]
        L.rrmhd_batch_destroy.argtypes = [vp]
        L.rrmhd_batch_last_error_detail.argtypes = []
        L.rrmhd_batch_last_error_detail.restype = ctypes.c_char_p
        ip = ctypes.POINTER(ci)
        L.rrmhd_autotune.argtypes = [vp, ctypes.c_char_p, ci, ip, ip, ip, dbl]
        L.rrmhd_batch_autotune.argtypes = [vp, ctypes.c_char_p, ci]
        L.rrmhd_closure_set.argtypes = [vp, vp, vp]
        L.rrmhd_closure_enable.argtypes = [vp, ci]
        L.rrmhd_closure_eval.argtypes = [vp, vp, vp, i64, vp, vp]
        L.rrmhd_closure_gelu_table.argtypes = [vp, vp]
        L.rrmhd_train_samples.argtypes = [vp, vp, vp, ci, ci, ctypes.c_double,
                                          vp, vp, vp, vp]
        L.rrmhd_train_box_filter.argtypes = [vp, vp, vp, ci, ci, vp, vp]
        L.rrmhd_train_impose_fluid.argtypes = [vp, dp, dp, dp]
        L.rrmhd_train_create.argtypes = [i64, vp, ctypes.POINTER(vp)]
        L.rrmhd_train_loss_grad.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp]
        L.rrmhd_train_onestep_samples.argtypes = [vp, vp, vp, vp, vp, vp, ci, ci,
                                                  ctypes.c_double, vp, vp, vp, vp,
                                                  vp]
        L.rrmhd_train_onestep_loss_grad.argtypes = [vp, vp, vp, vp, vp, ci, ci,
                                                    ctypes.c_double,
                                                    ctypes.c_double, ci, vp, vp]
        fl = ctypes.c_float
        L.rrmhd_train_adam.argtypes = [vp, vp, vp, vp, vp, fl, fl, fl, fl, ci]
        L.rrmhd_train_destroy.argtypes = [vp]
        L.rrmhd_current_vorticity.argtypes = [vp, dp, dp]
        L.rrmhd_train_last_error_detail.argtypes = []
        L.rrmhd_train_last_error_detail.restype = ctypes.c_char_p
        L.rrmhd_strerror.argtypes = [ctypes.c_int]
        L.rrmhd_strerror.restype = ctypes.c_char_p
        L.rrmhd_last_error_detail.argtypes = []
        L.rrmhd_last_error_detail.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("rrmhd_strerror", "rrmhd_last_error_detail",
                            "rrmhd_state_bytes",
                            "rrmhd_batch_last_error_detail",
                            "rrmhd_train_last_error_detail"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc, where):
    if rc != OK:
        raise RRMHDError(rc, where)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _own_stream(stream):
    """The torch stream a handle is created on (torch's current one if None)."""
    import torch
    return torch.cuda.current_stream() if stream is None else stream


def _before(stream):
    """Before a call that reads or writes caller tensors: the handle's stream
    waits for torch's current stream, where those tensors were produced."""
    import torch
    cur = torch.cuda.current_stream(stream.device)
    if cur != stream:
        stream.wait_stream(cur)


def _after(stream, *tensors):
    """After such a call: the caching allocator keeps the tensors until the
    handle's stream is done with them, and torch's current stream waits for
    the handle's stream before the caller uses the results."""
    import torch
    cur = torch.cuda.current_stream(stream.device)
    if cur != stream:
        for t in tensors:
            if t is not None:
                t.record_stream(stream)
        cur.wait_stream(stream)


def _dev_f64(t, shape, name):
    import torch
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{name} must be a contiguous float64 device tensor "
                         f"of shape {shape}")
    return ctypes.c_void_p(t.data_ptr())


def _dev_f32(t, shape, name):
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
            and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{name} must be a contiguous float32 device tensor "
                         f"of shape {shape}")
    return ctypes.c_void_p(t.data_ptr())


def closure_gelu_table(stream=None):
    """The inference's GELU table as an int16 device tensor [65536] holding
    BF16 bit patterns: entry v is GELU of the BF16 value with pattern v."""
    import torch
    t = torch.empty(65536, dtype=torch.int16, device="cuda")
    _check(lib().rrmhd_closure_gelu_table(ctypes.c_void_p(t.data_ptr()),
                                          _stream_handle(stream)), "rrmhd_closure_gelu_table")
    return t


def closure_eval(params, norm, x, stream=None):
    """Network outputs y[n][3] for features x[n][8] (FP32 device tensors),
    BF16 MFMA arithmetic as in the fused step."""
    import torch
    n = x.shape[0]
    y = torch.empty((n, 3), dtype=torch.float32, device=x.device)
    _check(lib().rrmhd_closure_eval(_dev_f32(params, (4931,), "params"),
                                    _dev_f32(norm, (19,), "norm"),
                                    _dev_f32(x, (n, 8), "x"), int(n),
                                    _dev_f32(y, (n, 3), "y"),
                                    _stream_handle(stream)), "rrmhd_closure_eval")
    return y


class Solver:
    """One lattice on the current device.

    storage: "f32", "f16" (populations stored as offsets f - w) or "f16sr"
    (FP16 with stochastically rounded step stores).
    walls: half-way bounce-back walls in y (periodic x); force: body force
    per unit mass; b_wall: field imposed by the magnetic walls.
    equilibrium: "algorithm" (the method's) or "full_maxwell" (ablation with
    the u.M cross terms of the third and fourth orders).
    inplace: one population buffer instead of two (single-buffer streaming).
    layout: "default" (row-interleaved planes for periodic handles) or
    "planar" (planes of [ny][nx]); results are the same.
    """

    def __init__(self, nx, ny, tau_f, tau_m, storage="f32", walls=False,
                 force=(0.0, 0.0), b_wall=(0.0, 0.0), codec_scale=0.0,
                 stream=None, equilibrium="algorithm", inplace=False, layout="default"):
        L = lib()
        self.nx, self.ny = int(nx), int(ny)
        self.storage = storage
        self._stream = _own_stream(stream)
        kind = {"f32": STORE_F32, "f16": STORE_F16, "f16sr": STORE_F16_SR}[storage]
        if layout not in ("default", "planar"):
            raise ValueError(f"layout must be 'default' or 'planar', not {layout!r}")
        flags = (STORE_INPLACE if inplace else 0) | (STORE_PLANAR if layout == "planar" else 0)
        g = Grid(self.nx, self.ny, kind | flags, float(codec_scale))
        bc = BC(BC_WALLS_Y if walls else BC_PERIODIC,
                (ctypes.c_double * 2)(*force), (ctypes.c_double * 2)(*b_wall))
        h = ctypes.c_void_p()
        _check(L.rrmhd_create(ctypes.byref(g), float(tau_f), float(tau_m),
                              ctypes.byref(bc), _stream_handle(self._stream),
                              ctypes.byref(h)), "rrmhd_create")
        self._h = h
        if equilibrium != "algorithm":
            self.set_equilibrium(equilibrium)

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _check(lib().rrmhd_destroy(self._h), "rrmhd_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- calls ---------------------------------------------------------------
    def init(self, u, b):
        shp = (2, self.ny, self.nx)
        _before(self._stream)
        _check(lib().rrmhd_init(self._h, _dev_f64(u, shp, "u"),
                                _dev_f64(b, shp, "b")), "rrmhd_init")
        _after(self._stream, u, b)

    def step(self, n=1):
        _check(lib().rrmhd_step(self._h, int(n)), "rrmhd_step")

    def moments(self, rho=None, u=None, b=None):
        """Fill (or allocate) FP64 device tensors rho, u, b."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        if rho is None:
            rho = torch.empty((self.ny, self.nx), dtype=torch.float64, device=dev)
        if u is None:
            u = torch.empty((2, self.ny, self.nx), dtype=torch.float64, device=dev)
        if b is None:
            b = torch.empty((2, self.ny, self.nx), dtype=torch.float64, device=dev)
        _before(self._stream)
        _check(lib().rrmhd_moments(
            self._h, _dev_f64(rho, (self.ny, self.nx), "rho"),
            _dev_f64(u, (2, self.ny, self.nx), "u"),
            _dev_f64(b, (2, self.ny, self.nx), "b")), "rrmhd_moments")
        _after(self._stream, rho, u, b)
        return rho, u, b

    def impose_fluid(self, rho, j, b):
        """Replace the fluid populations by the equilibrium of the given FP64
        device fields rho [ny][nx], momentum j and b [2][ny][nx] (periodic,
        two buffers); the magnetic populations are kept."""
        _before(self._stream)
        _check(lib().rrmhd_train_impose_fluid(
            self._h, _dev_f64(rho, (self.ny, self.nx), "rho"),
            _dev_f64(j, (2, self.ny, self.nx), "j"),
            _dev_f64(b, (2, self.ny, self.nx), "b")), "rrmhd_train_impose_fluid")
        _after(self._stream, rho, j, b)

    def current_vorticity(self):
        """(j_z, w_z) FP64 device tensors [ny][nx]."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        jz = torch.empty((self.ny, self.nx), dtype=torch.float64, device=dev)
        wz = torch.empty((self.ny, self.nx), dtype=torch.float64, device=dev)
        _before(self._stream)
        _check(lib().rrmhd_current_vorticity(self._h, ctypes.c_void_p(jz.data_ptr()),
                                             ctypes.c_void_p(wz.data_ptr())),
               "rrmhd_current_vorticity")
        _after(self._stream, jz, wz)
        return jz, wz

    def diagnostics(self, allow_nonfinite=False):
        ek, em, dv = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = lib().rrmhd_diagnostics(self._h, ctypes.byref(ek),
                                     ctypes.byref(em), ctypes.byref(dv))
        if not (allow_nonfinite and rc == ENONFINITE):
            _check(rc, "rrmhd_diagnostics")
        return ek.value, em.value, dv.value

    def diagnostics_noalloc(self, allow_nonfinite=False):
        """rrmhd_diagnostics_noalloc: the same results with the library's
        static per-device workspace instead of an allocated one."""
        ek, em, dv = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = lib().rrmhd_diagnostics_noalloc(self._h, ctypes.byref(ek),
                                             ctypes.byref(em), ctypes.byref(dv))
        if not (allow_nonfinite and rc == ENONFINITE):
            _check(rc, "rrmhd_diagnostics_noalloc")
        return ek.value, em.value, dv.value

    def diagnostics_rc(self):
        ek, em, dv = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = lib().rrmhd_diagnostics(self._h, ctypes.byref(ek),
                                     ctypes.byref(em), ctypes.byref(dv))
        return rc, (ek.value, em.value, dv.value)

    def invariants(self):
        out = (ctypes.c_double * 5)()
        _check(lib().rrmhd_invariants(self._h, out), "rrmhd_invariants")
        return list(out)

    @property
    def step_count(self):
        v = ctypes.c_int64()
        _check(lib().rrmhd_step_count(self._h, ctypes.byref(v)),
               "rrmhd_step_count")
        return v.value

    def state_bytes(self):
        return int(lib().rrmhd_state_bytes(self._h))

    def save_state(self, dst):
        _before(self._stream)
        _check(lib().rrmhd_save_state(self._h, ctypes.c_void_p(dst.data_ptr()),
                                      dst.numel() * dst.element_size()),
               "rrmhd_save_state")
        _after(self._stream, dst)

    def load_state(self, src, step_count):
        _before(self._stream)
        _check(lib().rrmhd_load_state(self._h, ctypes.c_void_p(src.data_ptr()),
                                      src.numel() * src.element_size(),
                                      int(step_count)), "rrmhd_load_state")
        _after(self._stream, src)

    def run(self, n, every, log=None):
        """Advance n steps, taking the diagnostics and invariants after every
        `every` steps (and after the last).  Returns the records; with `log`
        (a path, appended to, or an open text file) each record is also
        written as one JSON line.  Non-finite values are recorded as null."""
        import json
        import math

        def fin(v):
            return v if math.isfinite(v) else None

        own = isinstance(log, (str, bytes, os.PathLike))
        fh = open(log, "a") if own else log
        recs = []
        try:
            left = int(n)
            while left > 0:
                k = min(int(every), left)
                self.step(k)
                left -= k
                ek, em, dv = self.diagnostics(allow_nonfinite=True)
                inv = self.invariants()
                rec = {"step": self.step_count, "E_kin": fin(ek), "E_mag": fin(em),
                       "max_div_b": fin(dv), "mass": fin(inv[0]),
                       "momentum": [fin(inv[1]), fin(inv[2])],
                       "sum_b": [fin(inv[3]), fin(inv[4])]}
                recs.append(rec)
                if fh is not None:
                    fh.write(json.dumps(rec) + "\n")
                    fh.flush()
        finally:
            if own:
                fh.close()
        return recs

    def set_debug_poison(self, on=True):
        """NaN-fill the destination buffer before every step (debug)."""
        _check(lib().rrmhd_set_debug_poison(self._h, int(bool(on))), "rrmhd_set_debug_poison")

    def save(self, path):
        """Write a checkpoint file (header + state); synchronous."""
        _check(lib().rrmhd_save(self._h, os.fsencode(path)), "rrmhd_save")

    def load(self, path):
        """Read a checkpoint file written by save() into this handle (same
        grid, storage, relaxation times, boundary conditions)."""
        _check(lib().rrmhd_load(self._h, os.fsencode(path)), "rrmhd_load")

    def get_launch(self):
        """(bx, by, ry, xcd, nt) of the step kernel's current launch shape."""
        v = [ctypes.c_int() for _ in range(5)]
        _check(lib().rrmhd_get_launch(self._h, *[ctypes.byref(x) for x in v]),
               "rrmhd_get_launch")
        return tuple(x.value for x in v)

    def set_launch(self, bx, by, ry=1, xcd=1, nt=0):
        _check(lib().rrmhd_set_launch(self._h, int(bx), int(by), int(ry),
                                      int(xcd), int(nt)), "rrmhd_set_launch")

    def autotune(self, cache_path=None, trials=10):
        """Time candidate launch shapes and keep the fastest (state kept)."""
        bx, by, xcd = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        ms = ctypes.c_double()
        _check(lib().rrmhd_autotune(
            self._h, cache_path.encode() if cache_path else None, int(trials),
            ctypes.byref(bx), ctypes.byref(by), ctypes.byref(xcd),
            ctypes.byref(ms)), "rrmhd_autotune")
        return dict(bx=bx.value, by=by.value, xcd=xcd.value, ms=ms.value)

    def closure_set(self, params, norm):
        """Install closure parameters (FP32 device tensors of 4931 and 19
        values); params=None disables the closure."""
        if params is None:
            _check(lib().rrmhd_closure_set(self._h, None, None), "rrmhd_closure_set")
            return
        _check(lib().rrmhd_closure_set(self._h, _dev_f32(params, (4931,), "params"),
                                       _dev_f32(norm, (19,), "norm")),
               "rrmhd_closure_set")

    def closure_enable(self, on=True):
        _check(lib().rrmhd_closure_enable(self._h, int(bool(on))),
               "rrmhd_closure_enable")

    def set_graph_chunk(self, chunk):
        """Replay runs of `chunk` steps as captured hipGraphs (0: off)."""
        _check(lib().rrmhd_set_graph_chunk(self._h, int(chunk)), "rrmhd_set_graph_chunk")

    def set_equilibrium(self, kind):
        """"algorithm" or "full_maxwell"; applies to later init and steps."""
        k = {"algorithm": FEQ_ALGORITHM, "full_maxwell": FEQ_FULL_MAXWELL}[kind]
        _check(lib().rrmhd_set_equilibrium(self._h, k), "rrmhd_set_equilibrium")

    def set_stream(self, stream):
        self._stream = _own_stream(stream)
        _check(lib().rrmhd_set_stream(self._h, _stream_handle(self._stream)),
               "rrmhd_set_stream")


class Solver3D:
    """Periodic nx x ny x nz box of the three-dimensional extension (D3Q27
    fluid, D3Q7 magnetic lattice) on the current device.  Fields are FP64
    device tensors [3][nz][ny][nx]."""

    def __init__(self, nx, ny, nz, tau_f, tau_m, storage="f32", stream=None, inplace=False):
        L = lib()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self._stream = _own_stream(stream)
        h = ctypes.c_void_p()
        kind = STORE_F16 if storage == "f16" else STORE_F32
        _check(L.rrmhd3d_create(self.nx, self.ny, self.nz,
                                kind | (STORE_INPLACE if inplace else 0),
                                float(tau_f), float(tau_m), _stream_handle(self._stream),
                                ctypes.byref(h)), "rrmhd3d_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().rrmhd3d_destroy(self._h), "rrmhd3d_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, u, b):
        shp = (3, self.nz, self.ny, self.nx)
        _before(self._stream)
        _check(lib().rrmhd3d_init(self._h, _dev_f64(u, shp, "u"), _dev_f64(b, shp, "b")),
               "rrmhd3d_init")
        _after(self._stream, u, b)

    def step(self, n=1):
        _check(lib().rrmhd3d_step(self._h, int(n)), "rrmhd3d_step")

    @property
    def step_count(self):
        v = ctypes.c_int64()
        _check(lib().rrmhd3d_step_count(self._h, ctypes.byref(v)), "rrmhd3d_step_count")
        return v.value

    def moments(self):
        import torch
        shp = (self.nz, self.ny, self.nx)
        rho = torch.empty(shp, dtype=torch.float64, device="cuda")
        u = torch.empty((3,) + shp, dtype=torch.float64, device="cuda")
        b = torch.empty((3,) + shp, dtype=torch.float64, device="cuda")
        _before(self._stream)
        _check(lib().rrmhd3d_moments(self._h, _dev_f64(rho, shp, "rho"),
                                     _dev_f64(u, (3,) + shp, "u"), _dev_f64(b, (3,) + shp, "b")),
               "rrmhd3d_moments")
        _after(self._stream, rho, u, b)
        return rho, u, b

    def diagnostics(self, allow_nonfinite=False):
        ek, em, dv = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = lib().rrmhd3d_diagnostics(self._h, ctypes.byref(ek), ctypes.byref(em),
                                       ctypes.byref(dv))
        if not (allow_nonfinite and rc == ENONFINITE):
            _check(rc, "rrmhd3d_diagnostics")
        return ek.value, em.value, dv.value

    def invariants(self):
        out = (ctypes.c_double * 7)()
        _check(lib().rrmhd3d_invariants(self._h, out), "rrmhd3d_invariants")
        return list(out)

    def set_launch(self, bx, by, xcd=-1):
        """bx x by threads per workgroup; xcd 1 / 0: XCD-local or plain tile
        order, -1 keeps the current one."""
        _check(lib().rrmhd3d_set_launch(self._h, int(bx), int(by), int(xcd)),
               "rrmhd3d_set_launch")

    def save(self, path):
        """Write a checkpoint file (header + state); synchronous."""
        _check(lib().rrmhd3d_save(self._h, os.fsencode(path)), "rrmhd3d_save")

    def load(self, path):
        """Read a checkpoint file written by save() into this handle."""
        _check(lib().rrmhd3d_load(self._h, os.fsencode(path)), "rrmhd3d_load")

    def set_debug_poison(self, on=True):
        """NaN-fill the destination buffer before every step (debug)."""
        _check(lib().rrmhd3d_set_debug_poison(self._h, int(bool(on))), "rrmhd3d_set_debug_poison")


def sr_encode(x, r, stream=None):
    """The stochastically rounding FP16 encode of the storage codec: x float32
    and r uint32 (as int32 bits) device tensors of one shape; returns the FP16
    bit patterns as an int16 tensor."""
    import torch
    if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
        raise ValueError("x must be a contiguous float32 device tensor")
    if not (r.is_cuda and r.dtype == torch.int32 and r.is_contiguous() and r.shape == x.shape):
        raise ValueError("r must be a contiguous int32 device tensor shaped like x")
    out = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _check(lib().rrmhd_sr_encode(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(r.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), x.numel(),
                                 _stream_handle(stream)), "rrmhd_sr_encode")
    return out


def bandwidth_probe(dst, src, stream=None):
    """Plain device copy of src into dst (torch tensors, equal byte sizes)."""
    nb = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() >= nb
    _check(lib().rrmhd_bandwidth_probe(ctypes.c_void_p(dst.data_ptr()),
                                       ctypes.c_void_p(src.data_ptr()), nb,
                                       _stream_handle(stream)),
           "rrmhd_bandwidth_probe")


class Batch:
    """Ensemble of independent periodic domains stepped by one persistent
    launch per step.  sides: list of (nx, ny); taus: lists tau_f, tau_m."""

    def __init__(self, shapes, tau_f, tau_m, storage="f32", stream=None):
        L = lib()
        n = len(shapes)
        self.shapes = [(int(a), int(b)) for a, b in shapes]
        grids = (Grid * n)(*[Grid(a, b, 0, 0.0) for a, b in self.shapes])
        tf = (ctypes.c_double * n)(*map(float, tau_f))
        tm = (ctypes.c_double * n)(*map(float, tau_m))
        h = ctypes.c_void_p()
        self._stream = _own_stream(stream)
        rc = L.rrmhd_batch_create(n, grids, tf, tm,
                                  STORE_F16 if storage == "f16" else STORE_F32,
                                  _stream_handle(self._stream), ctypes.byref(h))
        if rc != OK:
            raise RuntimeError(f"rrmhd_batch_create: {rc} "
                               f"{L.rrmhd_batch_last_error_detail().decode()}")
        self._h = h
        self.n = n

    def _chk(self, rc, where):
        if rc != OK:
            det = lib().rrmhd_batch_last_error_detail().decode()
            raise RuntimeError(f"{where}: {lib().rrmhd_strerror(rc).decode()} "
                               f"({rc}) {det}")

    def close(self):
        if getattr(self, "_h", None):
            self._chk(lib().rrmhd_batch_destroy(self._h), "rrmhd_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, d, u, b):
        nx, ny = self.shapes[d]
        shp = (2, ny, nx)
        _before(self._stream)
        self._chk(lib().rrmhd_batch_init(self._h, int(d), _dev_f64(u, shp, "u"),
                                         _dev_f64(b, shp, "b")),
                  "rrmhd_batch_init")
        _after(self._stream, u, b)

    def step(self, n=1):
        self._chk(lib().rrmhd_batch_step(self._h, int(n)), "rrmhd_batch_step")

    def set_graph_chunk(self, chunk):
        self._chk(lib().rrmhd_batch_set_graph_chunk(self._h, int(chunk)),
                  "rrmhd_batch_set_graph_chunk")

    def set_shape(self, d=-1, bx=0, grid=0, nt=-1):
        self._chk(lib().rrmhd_batch_set_shape(self._h, int(d), int(bx),
                                              int(grid), int(nt)),
                  "rrmhd_batch_set_shape")

    def set_fetch(self, tiles_per_fetch):
        self._chk(lib().rrmhd_batch_set_fetch(self._h, int(tiles_per_fetch)),
                  "rrmhd_batch_set_fetch")

    def moments(self, d):
        import torch
        nx, ny = self.shapes[d]
        dev = torch.device("cuda", torch.cuda.current_device())
        rho = torch.empty((ny, nx), dtype=torch.float64, device=dev)
        u = torch.empty((2, ny, nx), dtype=torch.float64, device=dev)
        b = torch.empty((2, ny, nx), dtype=torch.float64, device=dev)
        _before(self._stream)
        self._chk(lib().rrmhd_batch_moments(
            self._h, int(d), ctypes.c_void_p(rho.data_ptr()),
            ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(b.data_ptr())),
            "rrmhd_batch_moments")
        _after(self._stream, rho, u, b)
        return rho, u, b

    def diagnostics(self, d):
        ek, em, dv = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._chk(lib().rrmhd_batch_diagnostics(self._h, int(d), ctypes.byref(ek),
                                                ctypes.byref(em),
                                                ctypes.byref(dv)),
                  "rrmhd_batch_diagnostics")
        return ek.value, em.value, dv.value

    def autotune(self, cache_path=None, trials=5):
        self._chk(lib().rrmhd_batch_autotune(
            self._h, cache_path.encode() if cache_path else None, int(trials)),
            "rrmhd_batch_autotune")

    def info(self):
        nodes, steps = ctypes.c_int64(), ctypes.c_int64()
        nt, grid = ctypes.c_int(), ctypes.c_int()
        self._chk(lib().rrmhd_batch_info(self._h, ctypes.byref(nodes),
                                         ctypes.byref(steps), ctypes.byref(nt),
                                         ctypes.byref(grid)), "rrmhd_batch_info")
        return dict(nodes=nodes.value, steps=steps.value, tiles=nt.value,
                    grid=grid.value)


def _ptr_t(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def train_samples(rho, u, b, factor, tau_c, stream=None):
    """Coarse training samples (x[Nc][8], target[Nc][3], FP32 device) from
    fine FP64 device moments rho[nf][nf], u, b [2][nf][nf]."""
    import torch
    nf = rho.shape[0]
    nc = nf // factor
    dev = rho.device
    work = torch.empty(10 * nc * nc, dtype=torch.float64, device=dev)
    x = torch.empty((nc * nc, 8), dtype=torch.float32, device=dev)
    t = torch.empty((nc * nc, 3), dtype=torch.float32, device=dev)
    _check(lib().rrmhd_train_samples(_ptr_t(rho), _ptr_t(u), _ptr_t(b), nf,
                                     int(factor), float(tau_c), _ptr_t(work),
                                     _ptr_t(x), _ptr_t(t),
                                     _stream_handle(stream)),
           "rrmhd_train_samples")
    return x, t


def train_box_filter(rho, u, b, factor, out=None, stream=None):
    """Block means over factor x factor of the fine FP64 device moments:
    [10][nc][nc] FP64 (rho, rho u_x, rho u_y, b_x, b_y, rho u u (xx, xy,
    yy), M(b) (xx, xy))."""
    import torch
    nf = rho.shape[0]
    nc = nf // factor
    if out is None:
        out = torch.empty((10, nc, nc), dtype=torch.float64, device=rho.device)
    _dev_f64(out, (10, nc, nc), "out")
    _check(lib().rrmhd_train_box_filter(_ptr_t(rho), _ptr_t(u), _ptr_t(b), nf, int(factor),
                                        _ptr_t(out), _stream_handle(stream)),
           "rrmhd_train_box_filter")
    return out


def train_onestep_samples(m0, m1, factor, tau_c, stream=None):
    """One-step objective data from fine FP64 device moments m0 = (rho, u, b)
    at t and m1 at t + factor: (x[Nc][8] FP32, r0[Nc][2] FP32, den[1] FP64),
    all on the device."""
    import torch
    rho0, u0, b0 = m0
    rho1, u1, b1 = m1
    nf = rho0.shape[0]
    nc = nf // factor
    dev = rho0.device
    work = torch.empty(29 * nc * nc, dtype=torch.float64, device=dev)
    x = torch.empty((nc * nc, 8), dtype=torch.float32, device=dev)
    r0 = torch.empty((nc * nc, 2), dtype=torch.float32, device=dev)
    den = torch.empty(1, dtype=torch.float64, device=dev)
    _check(lib().rrmhd_train_onestep_samples(
        _ptr_t(rho0), _ptr_t(u0), _ptr_t(b0), _ptr_t(rho1), _ptr_t(u1),
        _ptr_t(b1), nf, int(factor), float(tau_c), _ptr_t(work), _ptr_t(x),
        _ptr_t(r0), _ptr_t(den), _stream_handle(stream)),
        "rrmhd_train_onestep_samples")
    return x, r0, den


class Trainer:
    """FP32 training kernels of the closure network."""

    def __init__(self, max_batch, stream=None):
        h = ctypes.c_void_p()
        _check(lib().rrmhd_train_create(int(max_batch), _stream_handle(stream),
                                        ctypes.byref(h)), "rrmhd_train_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().rrmhd_train_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def loss_grad(self, params, norm, x, target, grad, loss=None):
        _check(lib().rrmhd_train_loss_grad(self._h, _ptr_t(params), _ptr_t(norm),
                                           _ptr_t(x), _ptr_t(target),
                                           int(x.shape[0]), _ptr_t(grad),
                                           _ptr_t(loss)),
               "rrmhd_train_loss_grad")

    def onestep_loss_grad(self, params, norm, x, r0, nsnap, nc, tau_c, den,
                          grad, loss=None, feedback=False):
        _check(lib().rrmhd_train_onestep_loss_grad(
            self._h, _ptr_t(params), _ptr_t(norm), _ptr_t(x), _ptr_t(r0),
            int(nsnap), int(nc), float(tau_c), float(den), int(bool(feedback)),
            _ptr_t(grad), _ptr_t(loss)), "rrmhd_train_onestep_loss_grad")

    def adam(self, params, m, v, grad, lr, step, beta1=0.9, beta2=0.999,
             eps=1e-8):
        _check(lib().rrmhd_train_adam(self._h, _ptr_t(params), _ptr_t(m),
                                      _ptr_t(v), _ptr_t(grad), float(lr),
                                      float(beta1), float(beta2), float(eps),
                                      int(step)), "rrmhd_train_adam")
