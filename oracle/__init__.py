"""Plain FP64 CPU oracle for the recursive regularised LB-MHD step.

TEST INFRASTRUCTURE ONLY: this package may be imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``.  The
product path (the HIP library and its binding) never imports or calls it, and
the two share no code.

The arithmetic lives in ``rrmhd_oracle.c`` (plain C, FP64, OpenMP over rows);
this module only compiles it with gcc and marshals numpy arrays through ctypes.
Every function cites the passage of the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rrmhd_oracle.c")
_SRC3 = os.path.join(_HERE, "rrmhd3d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC_REF = os.path.join(_HERE, "rrmhd_ref.c")
_LIB_REF = os.path.join(_HERE, "librrmhd_ref.so")

FEQ_ALGORITHM = 0  # equilibrium of the algorithm (Maxwell stress at 2nd order)
FEQ_SERIES_FULL = 1  # full Hermite series incl. the u.M cross terms (ablation)

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``, and the
    boundary's C-ABI over it (host pointers) into ``oracle/librrmhd_ref.so``."""
    flags = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall",
             "-Wno-unused-function"]
    for lib_path, srcs in ((_LIB, [_SRC, _SRC3]), (_LIB_REF, [_SRC, _SRC_REF])):
        if force or not os.path.exists(lib_path):
            tmp = lib_path + ".tmp"
            subprocess.run(flags + srcs + ["-o", tmp, "-lm"], check=True)
            os.replace(tmp, lib_path)
    return _LIB


_ref = None


def ref_lib():
    """The boundary's entry points (rrmhd_create, _init, _step, _moments,
    _diagnostics, _invariants, _step_count, _destroy, _strerror) over the
    oracle, with host pointers; the caller sets argument types."""
    global _ref
    if _ref is None:
        if not os.path.exists(_LIB_REF):
            build()
        _ref = ctypes.CDLL(_LIB_REF)
    return _ref


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_int]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_init.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.orc_step_count.restype = ctypes.c_long
        L.orc_step_count.argtypes = [ctypes.c_void_p]
        L.orc_moments.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_diagnostics.argtypes = [ctypes.c_void_p, _dp]
        L.orc_invariants.argtypes = [ctypes.c_void_p, _dp]
        L.orc_current_vorticity.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_get_state.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_round_state_f32.argtypes = [ctypes.c_void_p]
        L.orc_step_rounded_f32.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.orc_set_state.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_hermite.restype = ctypes.c_double
        L.orc_hermite.argtypes = [ctypes.c_int, _ip, ctypes.c_int]
        L.orc_node_equilibrium.argtypes = [ctypes.c_double, _dp, _dp,
                                           ctypes.c_int, _dp, _dp]
        L.orc_node_feq_series.argtypes = [ctypes.c_double, _dp, _dp,
                                          ctypes.c_int, _dp]
        L.orc_node_collide.argtypes = [_dp, _dp, ctypes.c_double,
                                       ctypes.c_double, _dp, ctypes.c_int,
                                       _dp, _dp, _dp]
        L.orc3d_create.restype = ctypes.c_void_p
        L.orc3d_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_double, ctypes.c_double]
        L.orc3d_destroy.argtypes = [ctypes.c_void_p]
        L.orc3d_init.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc3d_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.orc3d_step_count.restype = ctypes.c_long
        L.orc3d_step_count.argtypes = [ctypes.c_void_p]
        L.orc3d_moments.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc3d_diagnostics.argtypes = [ctypes.c_void_p, _dp]
        L.orc3d_invariants.argtypes = [ctypes.c_void_p, _dp]
        L.orc3d_hermite.restype = ctypes.c_double
        L.orc3d_hermite.argtypes = [ctypes.c_int, _ip, ctypes.c_int]
        L.orc3d_lattice.argtypes = [_ip, _dp]
        L.orc3d_aux_size.restype = ctypes.c_int
        L.orc3d_node_equilibrium.argtypes = [ctypes.c_double, _dp, _dp, _dp, _dp]
        L.orc3d_node_collide.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                         _dp, _dp, _dp]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_closure_nparams.restype = ctypes.c_int
        L.orc_set_closure.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_set_closure.restype = ctypes.c_int
        L.orc_mlp_forward.argtypes = [_dp, _dp, _dp, ctypes.c_int, _dp]
        L.orc_mlp_loss_grad.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int, _dp]
        L.orc_mlp_loss_grad.restype = ctypes.c_double
        L.orc_adam_step.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int]
        L.orc_train_samples.argtypes = [_dp, _dp, _dp, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.orc_mlp_vjp.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int, _dp]
        L.orc_onestep_objective.restype = ctypes.c_double
        L.orc_onestep_objective.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp,
                                            ctypes.c_int, ctypes.c_int,
                                            ctypes.c_double, _dp, _dp, _dp, _dp,
                                            _dp]
        L.orc_mlp_vjp_input.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int, _dp]
        L.orc_onestep_adjoint.argtypes = [_dp, ctypes.c_int, ctypes.c_double,
                                          _dp, _dp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def threads() -> int:
    """OpenMP threads the oracle's grid loops use."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP thread count of later grid loops (timing only)."""
    lib().orc_set_threads(int(n))


def hermite(n: int, idx, i: int) -> float:
    """Hermite tensor component H^(n)_{i, idx} from its definition."""
    arr = (ctypes.c_int * max(n, 1))(*idx)
    return float(lib().orc_hermite(n, arr, i))


def node_equilibrium(rho, u, b, option=FEQ_ALGORITHM):
    """(f_eq[9], g_eq[10]) of one node; g_eq is ordered [j][component]."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    feq = np.zeros(9)
    geq = np.zeros(10)
    lib().orc_node_equilibrium(float(rho), _ptr(u), _ptr(b), option,
                               _ptr(feq), _ptr(geq))
    return feq, geq


def node_feq_series(rho, u, b, full=False):
    u = np.ascontiguousarray(u, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    feq = np.zeros(9)
    lib().orc_node_feq_series(float(rho), _ptr(u), _ptr(b), int(bool(full)),
                              _ptr(feq))
    return feq


def node_collide(f, g, omega, omega_m, G=(0.0, 0.0), option=FEQ_ALGORITHM):
    """Collide one node.  Returns (f*[9], g*[10], aux dict)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(10)
    G = np.ascontiguousarray(G, dtype=np.float64)
    fs = np.zeros(9)
    gs = np.zeros(10)
    aux = np.zeros(63)
    lib().orc_node_collide(_ptr(f), _ptr(g), float(omega), float(omega_m),
                           _ptr(G), option, _ptr(fs), _ptr(gs), _ptr(aux))
    names = [("rho", 1), ("u", 2), ("b", 2), ("a1", 2), ("a2", 4), ("a3", 8),
             ("a4", 16), ("feq", 9), ("geq", 10), ("fneq_reg", 9)]
    d, k = {}, 0
    for nm, sz in names:
        d[nm] = aux[k:k + sz].copy() if sz > 1 else float(aux[k])
        k += sz
    d["a2"] = d["a2"].reshape(2, 2)
    d["a3"] = d["a3"].reshape(2, 2, 2)
    d["a4"] = d["a4"].reshape(2, 2, 2, 2)
    return fs, gs, d


# ---- learned closure (project addition) -----------------------------------
NPARAM = 4931   # W1[64][8], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]
NNORM = 19      # mu[8], sigma[8], sigma_out[3]


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def mlp_forward(params, norm, x):
    """Network output y[n][3] (normalised units) for features x[n][8]."""
    params, norm, x = _f64(params), _f64(norm), _f64(x)
    assert params.size == NPARAM and norm.size == NNORM and x.shape[-1] == 8
    n = x.shape[0]
    y = np.zeros((n, 3))
    lib().orc_mlp_forward(_ptr(params), _ptr(norm), _ptr(x), n, _ptr(y))
    return y


def mlp_loss_grad(params, norm, x, t):
    """(MSE loss, gradient[4931]) for features x[n][8], targets t[n][3]."""
    params, norm, x, t = _f64(params), _f64(norm), _f64(x), _f64(t)
    g = np.zeros(NPARAM)
    loss = lib().orc_mlp_loss_grad(_ptr(params), _ptr(norm), _ptr(x), _ptr(t),
                                   x.shape[0], _ptr(g))
    return float(loss), g


def adam_step(params, m, v, grad, lr=1e-3, beta1=0.9, beta2=0.999,
              eps=1e-8, t=1):
    """In-place Adam update of params, m, v (float64 arrays)."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    grad = _f64(grad)
    lib().orc_adam_step(_ptr(params), _ptr(m), _ptr(v), _ptr(grad),
                        params.size, lr, beta1, beta2, eps, int(t))


def train_samples(rho, u, b, factor, tau_c):
    """Closure training samples (x[Nc][8], t[Nc][3]) from fine moments."""
    rho, u, b = _f64(rho), _f64(u), _f64(b)
    nf = rho.shape[0]
    nc = nf // factor
    x = np.zeros((nc * nc, 8))
    t = np.zeros((nc * nc, 3))
    lib().orc_train_samples(_ptr(rho), _ptr(u), _ptr(b), nf, int(factor),
                            float(tau_c), _ptr(x), _ptr(t))
    return x, t


def mlp_vjp(params, norm, x, dy):
    """Gradient of sum_s dy[s] . y(x_s) with respect to the parameters."""
    params, norm, x, dy = _f64(params), _f64(norm), _f64(x), _f64(dy)
    g = np.zeros(NPARAM)
    lib().orc_mlp_vjp(_ptr(params), _ptr(norm), _ptr(x), _ptr(dy), x.shape[0],
                      _ptr(g))
    return g


def onestep_objective(m0, m1, factor, tau_c, delta=None, q=None):
    """One-step solver-in-the-loop objective of the closure.

    m0, m1: fine moments (rho, u, b) at t and t + factor.  delta: [Nc][3]
    correction of a_1^(2) per coarse node (None: zero).  q: [Nc][3] extra
    non-equilibrium of the restart (None: zero).  Returns (L, resid [Nc][2],
    x [Nc][8] restart features, den)."""
    rho0, u0, b0 = map(_f64, m0)
    rho1, u1, b1 = map(_f64, m1)
    nf = rho0.shape[0]
    nc = nf // factor
    resid = np.zeros((nc * nc, 2))
    x = np.zeros((nc * nc, 8))
    den = np.zeros(1)
    d = None if delta is None else _f64(delta)
    qq = None if q is None else _f64(q)
    for a in (d, qq):
        if a is not None:
            assert a.shape == (nc * nc, 3)
    L = lib().orc_onestep_objective(_ptr(rho0), _ptr(u0), _ptr(b0), _ptr(rho1),
                                    _ptr(u1), _ptr(b1), nf, int(factor),
                                    float(tau_c), _ptr(qq), _ptr(d), _ptr(resid),
                                    _ptr(x), _ptr(den))
    return float(L), resid, x, float(den[0])


def onestep_adjoint(x, nc, tau_c, w):
    """Transpose of the linear map delta -> coarse momentum, applied to w[Nc][2]."""
    x, w = _f64(x), _f64(w)
    out = np.zeros((nc * nc, 3))
    lib().orc_onestep_adjoint(_ptr(x), int(nc), float(tau_c), _ptr(w), _ptr(out))
    return out


def mlp_vjp_input(params, norm, x, dy):
    """Gradient of sum_s dy[s] . y(x_s) with respect to the raw inputs x."""
    params, norm, x, dy = _f64(params), _f64(norm), _f64(x), _f64(dy)
    gx = np.zeros_like(x)
    lib().orc_mlp_vjp_input(_ptr(params), _ptr(norm), _ptr(x), _ptr(dy),
                            x.shape[0], _ptr(gx))
    return gx


def onestep_loss_grad(params, norm, m0, m1, factor, tau_c, feedback=False):
    """(L, dL/dparams) of the one-step objective with delta = sigma_out * y(x),
    x the restart features: MLP forward, the objective, its adjoint, MLP
    reverse mode.

    feedback=True: the restart also carries the closure's own steady
    response q = (tau_c - 1) D0, D0 = sigma_out * y(x_CE) (a correction D
    added every step settles at a non-equilibrium (tau - 1) D), and the
    step's correction is evaluated on the features of that restart, as a
    closure run sees them; the gradient runs through both evaluations."""
    params, norm = _f64(params), _f64(norm)
    nc = np.asarray(m0[0]).shape[0] // factor
    so = norm[16:19]
    _, _, x0, _ = onestep_objective(m0, m1, factor, tau_c)
    if not feedback:
        delta = mlp_forward(params, norm, x0) * so
        L, resid, _, den = onestep_objective(m0, m1, factor, tau_c, delta)
        g_delta = onestep_adjoint(x0, nc, tau_c, resid) * (2.0 / den)
        return L, mlp_vjp(params, norm, x0, g_delta * so)
    q = (tau_c - 1.0) * mlp_forward(params, norm, x0) * so
    _, _, x1, _ = onestep_objective(m0, m1, factor, tau_c, q=q)
    d1 = mlp_forward(params, norm, x1) * so
    L, resid, _, den = onestep_objective(m0, m1, factor, tau_c, d1, q=q)
    # the post-collision populations see E = q + d1
    gE = onestep_adjoint(x1, nc, tau_c, resid) * (2.0 / den)
    g1 = mlp_vjp(params, norm, x1, gE * so)
    gq = gE + mlp_vjp_input(params, norm, x1, gE * so)[:, 5:8]
    g0 = mlp_vjp(params, norm, x0, (tau_c - 1.0) * gq * so)
    return L, g1 + g0


class Oracle:
    """FP64 grid solver: state = pre-collision populations.

    ``walls`` puts half-way bounce-back walls at y = -1/2 and ny - 1/2 (x stays
    periodic); ``force`` is the body force per unit mass; ``b_wall`` is the
    field the magnetic anti-bounce-back imposes at the walls.
    """

    def __init__(self, nx, ny, tau_f, tau_m, walls=False, force=(0.0, 0.0),
                 b_wall=(0.0, 0.0), option=FEQ_ALGORITHM):
        self.nx, self.ny = int(nx), int(ny)
        self._h = lib().orc_create(self.nx, self.ny, float(tau_f),
                                   float(tau_m), int(bool(walls)),
                                   float(force[0]), float(force[1]),
                                   float(b_wall[0]), float(b_wall[1]),
                                   int(option))
        if not self._h:
            raise ValueError("oracle: invalid grid or relaxation times")

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, u, b):
        u = np.ascontiguousarray(u, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        assert u.shape == (2, self.ny, self.nx) and b.shape == u.shape
        lib().orc_init(self._h, _ptr(u), _ptr(b))

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    def step_rounded_f32(self, n=1):
        """n FP64 steps, each followed by rounding the stored state (f - w
        and g) to FP32: the storage-precision model of FP32 storage."""
        lib().orc_step_rounded_f32(self._h, int(n))

    def round_state_f32(self):
        lib().orc_round_state_f32(self._h)

    @property
    def step_count(self):
        return int(lib().orc_step_count(self._h))

    def moments(self):
        rho = np.zeros((self.ny, self.nx))
        u = np.zeros((2, self.ny, self.nx))
        b = np.zeros((2, self.ny, self.nx))
        lib().orc_moments(self._h, _ptr(rho), _ptr(u), _ptr(b))
        return rho, u, b

    def diagnostics(self):
        out = np.zeros(3)
        lib().orc_diagnostics(self._h, _ptr(out))
        return float(out[0]), float(out[1]), float(out[2])

    def invariants(self):
        out = np.zeros(5)
        lib().orc_invariants(self._h, _ptr(out))
        return out

    def current_vorticity(self):
        jz = np.zeros((self.ny, self.nx))
        wz = np.zeros((self.ny, self.nx))
        lib().orc_current_vorticity(self._h, _ptr(jz), _ptr(wz))
        return jz, wz

    def get_state(self):
        f = np.zeros((9, self.ny, self.nx))
        g = np.zeros((5, 2, self.ny, self.nx))
        lib().orc_get_state(self._h, _ptr(f), _ptr(g))
        return f, g

    def set_closure(self, params, norm):
        """Install the learned closure (None removes it)."""
        if params is None:
            lib().orc_set_closure(self._h, None, None)
            return
        params, norm = _f64(params), _f64(norm)
        assert params.size == NPARAM and norm.size == NNORM
        if lib().orc_set_closure(self._h, _ptr(params), _ptr(norm)) != 0:
            raise MemoryError("oracle closure")

    def set_state(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        assert g.shape == (5, 2, self.ny, self.nx)
        lib().orc_set_state(self._h, _ptr(f), _ptr(g))


# ---- three-dimensional extension (D3Q27 fluid, D3Q7 magnetic lattice) -------
def lattice3d():
    """(c[27][3], w[27]) in the oracle's velocity order
    i = 9 (c_x + 1) + 3 (c_y + 1) + (c_z + 1)."""
    c = np.zeros(81, dtype=np.int32)
    w = np.zeros(27)
    lib().orc3d_lattice(c.ctypes.data_as(_ip), _ptr(w))
    return c.reshape(27, 3).astype(int), w


MAG3D_E = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0],
                    [0, 0, 1], [0, 0, -1]])
MAG3D_PSI = np.array([0.25] + [0.125] * 6)


def hermite3d(n: int, idx, i: int) -> float:
    arr = (ctypes.c_int * max(n, 1))(*idx)
    return float(lib().orc3d_hermite(n, arr, i))


def node_equilibrium3d(rho, u, b):
    """(f_eq[27], g_eq[7][3]) of one node."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    feq = np.zeros(27)
    geq = np.zeros(21)
    lib().orc3d_node_equilibrium(float(rho), _ptr(u), _ptr(b), _ptr(feq), _ptr(geq))
    return feq, geq.reshape(7, 3)


def node_collide3d(f, g, omega, omega_m):
    """Collide one node.  Returns (f*[27], g*[7][3], aux dict with rho, u,
    b, the full tensors a2..a6, feq, geq, fneq_reg)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(21)
    fs = np.zeros(27)
    gs = np.zeros(21)
    aux = np.zeros(int(lib().orc3d_aux_size()))
    lib().orc3d_node_collide(_ptr(f), _ptr(g), float(omega), float(omega_m), _ptr(fs),
                             _ptr(gs), _ptr(aux))
    names = [("rho", 1), ("u", 3), ("b", 3), ("a2", 9), ("a3", 27), ("a4", 81),
             ("a5", 243), ("a6", 729), ("feq", 27), ("geq", 21), ("fneq_reg", 27)]
    d, k = {}, 0
    for nm, sz in names:
        d[nm] = aux[k:k + sz].copy() if sz > 1 else float(aux[k])
        k += sz
    for n in range(2, 7):
        d[f"a{n}"] = d[f"a{n}"].reshape((3,) * n)
    d["geq"] = d["geq"].reshape(7, 3)
    return fs, gs.reshape(7, 3), d


class Oracle3D:
    """FP64 three-dimensional periodic grid; state = pre-collision
    populations; fields are [3][nz][ny][nx] (rho [nz][ny][nx])."""

    def __init__(self, nx, ny, nz, tau_f, tau_m):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self._h = lib().orc3d_create(self.nx, self.ny, self.nz, float(tau_f), float(tau_m))
        if not self._h:
            raise ValueError("oracle: invalid grid or relaxation times")

    def close(self):
        if self._h:
            lib().orc3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, u, b):
        u = np.ascontiguousarray(u, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        assert u.shape == (3, self.nz, self.ny, self.nx) and b.shape == u.shape
        lib().orc3d_init(self._h, _ptr(u), _ptr(b))

    def step(self, n=1):
        lib().orc3d_step(self._h, int(n))

    @property
    def step_count(self):
        return int(lib().orc3d_step_count(self._h))

    def moments(self):
        shp = (self.nz, self.ny, self.nx)
        rho = np.zeros(shp)
        u = np.zeros((3,) + shp)
        b = np.zeros((3,) + shp)
        lib().orc3d_moments(self._h, _ptr(rho), _ptr(u), _ptr(b))
        return rho, u, b

    def diagnostics(self):
        out = np.zeros(3)
        lib().orc3d_diagnostics(self._h, _ptr(out))
        return float(out[0]), float(out[1]), float(out[2])

    def invariants(self):
        out = np.zeros(7)
        lib().orc3d_invariants(self._h, _ptr(out))
        return out
