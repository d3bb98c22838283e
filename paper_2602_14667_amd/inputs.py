"""Seeded synthetic inputs (initial fields and run configurations).

This module holds no arithmetic of the lattice Boltzmann method: it only
produces the macroscopic fields (u, b) handed to ``rrmhd_init`` and the
parameters of the workloads.  Tests feed the very same arrays to the HIP
library and to the CPU oracle.

Random numbers come from one counter-based generator: the SplitMix64 output
function of Steele, Lea & Flood (OOPSLA 2014) applied to a (seed, stream,
index) counter, so a value never depends on the order in which others are
drawn.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def counter_u64(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    """SplitMix64 value for each (seed, stream, index)."""
    idx = np.asarray(index, dtype=np.uint64)
    key = _mix64(np.array([seed], dtype=np.uint64) + _GOLDEN)
    key = _mix64(key ^ np.uint64(stream))
    with np.errstate(over="ignore"):
        z = key + (idx + np.uint64(1)) * _GOLDEN
    return _mix64(z)


def counter_uniform(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) with 53 random bits."""
    z = counter_u64(seed, stream, index)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# --------------------------------------------------------------------------
# Orszag-Tang vortex (Sec. III, Eq. OT_initial)
# --------------------------------------------------------------------------
def orszag_tang(n: int, u0: float, b0: float, perturb: float = 0.0,
                seed: int = 0):
    """Orszag-Tang fields on an n x n periodic grid, nodes x_k = 2 pi k / n.

    u = u0 (-sin y, sin x), b = b0 (-sin y, sin 2x).  ``perturb`` adds
    i.i.d. U[-perturb, perturb) to each velocity component at every node
    (streams 0 and 1 of ``seed``); b is not perturbed.  Returns float64 arrays
    u, b of shape [2][n][n] (component, y, x).
    """
    k = 2.0 * np.pi * np.arange(n) / n
    X, Y = np.meshgrid(k, k, indexing="xy")
    u = np.stack([-u0 * np.sin(Y), u0 * np.sin(X)])
    b = np.stack([-b0 * np.sin(Y), b0 * np.sin(2.0 * X)])
    if perturb:
        idx = np.arange(n * n)
        for c in range(2):
            r = counter_uniform(seed, c, idx).reshape(n, n)
            u[c] += perturb * (2.0 * r - 1.0)
    return np.ascontiguousarray(u), np.ascontiguousarray(b)


def orszag_tang_paper(n: int, re: float = 200.0 * np.pi):
    """Orszag-Tang in the paper's unit mapping (Sec. III): lattice amplitude
    0.2/pi at n = 128 with diffusive scaling 128/n, tau for Reynolds number
    re (Re = 200 pi in the low-Re case, 2500 and 5000 in the turbulent
    cases) and Pr_m = 1, and the step count of one physical time unit.
    """
    ut = 0.2 / np.pi * 128.0 / n
    nu_phys = 2.0 * 2.0 * np.pi / re  # Re = u0 L / nu, u0 = 2, L = 2 pi
    dx = 2.0 * np.pi / n
    dt = dx * ut / 2.0  # lattice speed ut <-> physical speed 2
    nu_lat = nu_phys * dt / dx ** 2
    tau = nu_lat * 3.0 + 0.5  # nu = c_s^2 (tau - 1/2)
    u, b = orszag_tang(n, ut, ut)
    return dict(u=u, b=b, tau=tau, steps_per_unit=1.0 / dt,
                scale=2.0 / ut / dx)


# --------------------------------------------------------------------------
# Random-phase decaying MHD turbulence
# --------------------------------------------------------------------------
TURB_KMAX = 16  # modes with |kappa_x|, |kappa_y| <= 16 are drawn


def _turb_modes(seed: int):
    K = TURB_KMAX
    ky, kx = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1),
                         indexing="ij")
    k = np.hypot(kx, ky)
    E = np.where(k > 0, k ** 4 * np.exp(-2.0 * (k / 4.0) ** 2), 0.0)
    amp = np.where(k > 0, np.sqrt(E / (np.pi * np.maximum(k, 1.0) ** 3)), 0.0)
    idx = ((ky + K) * (2 * K + 1) + (kx + K)).ravel()
    theta = 2.0 * np.pi * counter_uniform(seed, 7, idx).reshape(k.shape)
    c = amp * np.exp(1j * theta)
    # Hermitian symmetry: c(-kappa) = conj(c(kappa)); the upper half plane
    # (ky > 0, or ky == 0 and kx > 0) carries the drawn phases.
    upper = (ky > 0) | ((ky == 0) & (kx > 0))
    c = np.where(upper, c, 0.0)
    c = c + np.conj(c[::-1, ::-1])
    return kx, ky, c


def _field_from_stream(n: int, seed: int):
    """(d_y psi, -d_x psi) on an n x n grid for the drawn stream function.

    The field has only |kappa_x|, |kappa_y| <= TURB_KMAX modes, so it is
    synthesised separably: v(y, x) = Re[Ey C Ex^T] with Ey[y, ky] =
    exp(i ky 2 pi y / n), which costs O(n^2 K) instead of a full n x n FFT.
    """
    kx, ky, c = _turb_modes(seed)
    K = TURB_KMAX
    keep = (np.abs(kx) < n / 2.0) & (np.abs(ky) < n / 2.0)
    c = np.where(keep, c, 0.0)
    k1 = np.arange(-K, K + 1)
    ph = np.exp(1j * 2.0 * np.pi * np.outer(np.arange(n), k1) / n)  # [n, 2K+1]
    pr, pi = np.ascontiguousarray(ph.real), np.ascontiguousarray(ph.imag)
    out = []
    for spec in (1j * ky * c, -1j * kx * c):  # rows: ky, cols: kx
        t = spec @ ph.T                        # [2K+1 (ky), n (x)]
        v = pr @ np.ascontiguousarray(t.real)  # Re[Ey t]
        v -= pi @ np.ascontiguousarray(t.imag)
        out.append(v)
    # vector rms from Parseval in kappa space (identical on every grid)
    ms = float(np.sum(np.abs(c) ** 2 * (kx ** 2 + ky ** 2)))
    return np.stack(out), math.sqrt(ms)


def turbulence(n: int, rms: float = 0.04, seed_psi: int = 1,
               seed_a: int = 2):
    """Decaying 2D MHD turbulence: random-phase stream function psi and flux
    function A with E(k) ~ k^4 exp(-2 (k/4)^2), u = (d_y psi, -d_x psi),
    b = (d_y A, -d_x A), both rescaled to vector rms ``rms``.  The same
    kappa-space field is sampled on any n.  Returns u, b [2][n][n] float64.
    """
    u, su = _field_from_stream(n, seed_psi)
    b, sb = _field_from_stream(n, seed_a)
    return (np.ascontiguousarray(u * (rms / su)),
            np.ascontiguousarray(b * (rms / sb)))


def random_modes(nx: int, ny: int, amp: float, seed: int, kmax: int = 3):
    """Smooth periodic test fields on a rectangular grid: each component of u
    and b is a sum of Fourier modes |k| <= kmax with counter-based random
    coefficients, scaled to max |component| ~ amp.  Returns u, b [2][ny][nx].
    """
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    fields = []
    stream = 20
    for _ in range(4):
        f = np.zeros((ny, nx))
        for kx_ in range(-kmax, kmax + 1):
            for ky_ in range(0, kmax + 1):
                r = counter_uniform(seed, stream, np.arange(2))
                stream += 1
                f += (r[0] - 0.5) * np.cos(2 * np.pi * (kx_ * x / nx + ky_ * y / ny)
                                           + 2 * np.pi * r[1])
        m = np.abs(f).max()
        fields.append(f * (amp / m if m > 0 else 0.0))
    u = np.stack(fields[:2])
    b = np.stack(fields[2:])
    return np.ascontiguousarray(u), np.ascontiguousarray(b)


# --------------------------------------------------------------------------
# Hartmann channel (walls in y, periodic x, body force in x)
# --------------------------------------------------------------------------
@dataclass
class Hartmann:
    nx: int
    ny: int
    tau_f: float
    tau_m: float
    G: float
    Ha: float

    @property
    def nu(self):
        return (self.tau_f - 0.5) / 3.0

    @property
    def eta(self):
        return (self.tau_m - 0.5) / 3.0

    @property
    def a(self):
        """Half width: walls half-way at y = -1/2 and ny - 1/2."""
        return self.ny / 2.0

    @property
    def B0(self):
        return self.Ha * math.sqrt(self.nu * self.eta) / self.a

    def initial_fields(self):
        u = np.zeros((2, self.ny, self.nx))
        b = np.zeros((2, self.ny, self.nx))
        b[1] = self.B0
        return u, b

    def profile(self, y):
        """Steady analytic solution of the incompressible MHD system for this
        channel (insulating walls at distance a from the centre): u_x(y) and
        b_x(y) at node rows y, the reference of the convergence runs."""
        a, Ha, B0 = self.a, self.Ha, self.B0
        yp = np.asarray(y, dtype=np.float64) - (self.ny - 1) / 2.0
        u = (self.G * a * a / (self.nu * Ha)) * (math.cosh(Ha) - np.cosh(Ha * yp / a)) \
            / math.sinh(Ha)
        bx = (self.G * a / B0) * (np.sinh(Ha * yp / a) / math.sinh(Ha) - yp / a)
        return u, bx


def hartmann_c2() -> Hartmann:
    """512 x 256 Hartmann channel: G = 1e-6, Ha = 10, tau_f 0.6, tau_m 0.55."""
    return Hartmann(nx=512, ny=256, tau_f=0.6, tau_m=0.55, G=1e-6, Ha=10.0)


# --------------------------------------------------------------------------
# Batched ensemble of uneven domains
# --------------------------------------------------------------------------
BATCH_SIDES = tuple(range(64, 1025, 32))


def batch_domains(n_domains: int = 256, seed: int = 0):
    """Square domains with side drawn uniformly from {64, 96, ..., 1024},
    tau_f and tau_m uniform in [0.501, 0.6], and kind 'ot' or 'turb' by a
    fair coin.  Returns a list of dicts (side, tau_f, tau_m, kind, seed)."""
    d = np.arange(n_domains)
    side_u = counter_uniform(seed, 100, d)
    tf_u = counter_uniform(seed, 101, d)
    tm_u = counter_uniform(seed, 102, d)
    kind_u = counter_uniform(seed, 103, d)
    sides = np.array(BATCH_SIDES)
    out = []
    for k in range(n_domains):
        out.append(dict(
            side=int(sides[min(int(side_u[k] * len(sides)), len(sides) - 1)]),
            tau_f=0.501 + 0.099 * float(tf_u[k]),
            tau_m=0.501 + 0.099 * float(tm_u[k]),
            kind="ot" if kind_u[k] < 0.5 else "turb",
            seed=1000 + 2 * k))
    return out


def batch_fields(dom: dict):
    """Initial fields of one batched domain."""
    s = dom["side"]
    if dom["kind"] == "ot":
        return orszag_tang(s, 0.05, 0.05, perturb=1e-4, seed=dom["seed"])
    return turbulence(s, 0.04, seed_psi=dom["seed"], seed_a=dom["seed"] + 1)


# --------------------------------------------------------------------------
# Three-dimensional fields (the three-dimensional extension)
# --------------------------------------------------------------------------
TURB3D_KMAX = 12


def _gauss(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    """Standard normal values from two counter streams (Box-Muller)."""
    u1 = counter_uniform(seed, stream, index)
    u2 = counter_uniform(seed, stream + 1, index)
    return np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * np.pi * u2)


def _solenoidal3d(n: int, seed: int):
    """u = curl A on an n^3 grid for a random vector potential A with the
    modes |kappa| <= TURB3D_KMAX, |A(kappa)| ~ sqrt(E(k) / 4 pi) / k^2 and
    E(k) ~ k^4 exp(-2 (k/4)^2), so that the shell spectrum of u follows
    E(k); real by Hermitian symmetry (irfftn).  Returns u [3][n][n][n]
    (component, z, y, x) with unit vector rms."""
    K = min(TURB3D_KMAX, n // 2 - 1) if n > 2 else 0
    kz = np.fft.fftfreq(n, 1.0 / n)[:, None, None]
    ky = np.fft.fftfreq(n, 1.0 / n)[None, :, None]
    kx = np.arange(n // 2 + 1, dtype=float)[None, None, :]
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    keep = (kk > 0) & (kk <= K)
    E = np.where(keep, kk ** 4 * np.exp(-2.0 * (kk / 4.0) ** 2), 0.0)
    amp = np.where(keep, np.sqrt(E / (4.0 * np.pi)) / np.maximum(kk, 1.0) ** 2, 0.0)
    shape = amp.shape
    # a counter index per (component, kappa) that does not depend on n
    kzi = np.rint(np.broadcast_to(kz, shape)).astype(np.int64) + 64
    kyi = np.rint(np.broadcast_to(ky, shape)).astype(np.int64) + 64
    kxi = np.rint(np.broadcast_to(kx, shape)).astype(np.int64)
    base = ((kzi * 129 + kyi) * 129 + kxi).astype(np.uint64)
    A = []
    for comp in range(3):
        idx = base + np.uint64(comp * 129 ** 3)
        re = _gauss(seed, 11, idx.ravel()).reshape(shape)
        im = _gauss(seed, 13, idx.ravel()).reshape(shape)
        A.append(amp * (re + 1j * im))
    ik = (1j * kx, 1j * ky, 1j * kz)
    uh = (ik[1] * A[2] - ik[2] * A[1], ik[2] * A[0] - ik[0] * A[2], ik[0] * A[1] - ik[1] * A[0])
    u = np.stack([np.fft.irfftn(c, s=(n, n, n), axes=(0, 1, 2)) for c in uh])
    rms = math.sqrt(float(np.mean(np.sum(u * u, axis=0))))
    return u / (rms if rms > 0 else 1.0)


def turbulence3d(n: int, rms: float = 0.04, seed_u: int = 101, seed_b: int = 102):
    """Decaying 3D MHD turbulence on a periodic n^3 box: divergence-free
    random-phase u and b with shell spectrum ~ k^4 exp(-2 (k/4)^2) (modes
    |kappa| <= 12), each rescaled to vector rms ``rms``.  Returns u, b
    [3][n][n][n] float64 (component, z, y, x)."""
    u = rms * _solenoidal3d(n, seed_u)
    b = rms * _solenoidal3d(n, seed_b)
    return np.ascontiguousarray(u), np.ascontiguousarray(b)


def random_modes3d(nx: int, ny: int, nz: int, amp: float, seed: int, kmax: int = 2):
    """Smooth periodic test fields on a box: each component of u and b is a
    sum of Fourier modes with |k_a| <= kmax and counter-based random
    coefficients, scaled to max |component| ~ amp.  Returns u, b
    [3][nz][ny][nx]."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = []
    stream = 40
    for _ in range(6):
        f = np.zeros((nz, ny, nx))
        for k3 in itertools.product(range(-kmax, kmax + 1), repeat=3):
            if k3 == (0, 0, 0):
                continue
            r = counter_uniform(seed, stream, np.arange(2, dtype=np.uint64))
            stream += 1
            ph = 2 * np.pi * (k3[0] * x / nx + k3[1] * y / ny + k3[2] * z / nz)
            f += (r[0] - 0.5) * np.cos(ph + 2 * np.pi * r[1])
        m = np.abs(f).max()
        out.append(f * (amp / m) if m > 0 else f)
    return np.stack(out[:3]), np.stack(out[3:])
