"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check is a closed form
derived independently of the oracle's generic-tensor code (D1Q3 product form
of the equilibrium, hand-expanded Maxwell and recursion terms, exact-rational
single-node collision), a moment identity the method is built to satisfy, a
conservation law or symmetry, an analytic decay rate, or a value the paper
prints.  CPU only.
"""
from fractions import Fraction as Fr
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2602_14667_amd import inputs

# D2Q9 / D2Q5 as printed in Sec. II.A (used only to take moments here)
CX = np.array([0, -1, -1, -1, 0, 1, 1, 1, 0])
CY = np.array([0, 1, 0, -1, -1, -1, 0, 1, 1])
EX = np.array([0, -1, 0, 1, 0])
EY = np.array([0, 0, -1, 0, 1])
RNG = np.random.default_rng(12345)


def weights():
    feq, _ = oracle.node_equilibrium(1.0, [0.0, 0.0], [0.0, 0.0])
    return feq


def H(idx, i):
    return oracle.hermite(len(idx), idx, i)


def Hvec(idx):
    return np.array([H(idx, i) for i in range(9)])


# --------------------------------------------------------------------------
# Lattice and Hermite basis
# --------------------------------------------------------------------------
def test_weights_and_isotropy():
    w = weights()
    assert np.allclose(w, [4 / 9, 1 / 36, 1 / 9, 1 / 36, 1 / 9, 1 / 36, 1 / 9,
                           1 / 36, 1 / 9], rtol=0, atol=1e-16)
    assert abs(w.sum() - 1) < 1e-15
    cs2 = 1 / 3
    assert abs((w * CX * CX).sum() - cs2) < 1e-15
    assert abs((w * CX * CY).sum()) < 1e-15
    assert abs((w * CX ** 4).sum() - 3 * cs2 ** 2) < 1e-15
    assert abs((w * CX ** 2 * CY ** 2).sum() - cs2 ** 2) < 1e-15


def test_hermite_gram_matrix_norms():
    """The nine D2Q9 Hermite polynomials are w-orthogonal with norms
    1, 1/3, 1/3, 2/9, 1/9, 2/9, 2/27, 2/27, 4/81."""
    w = weights()
    basis = [(), (0,), (1,), (0, 0), (0, 1), (1, 1), (0, 0, 1), (0, 1, 1),
             (0, 0, 1, 1)]
    V = np.array([Hvec(b) if b else np.ones(9) for b in basis])
    G = (V * w) @ V.T
    expect = np.diag([1, 1 / 3, 1 / 3, 2 / 9, 1 / 9, 2 / 9, 2 / 27, 2 / 27,
                      4 / 81])
    assert np.allclose(G, expect, rtol=0, atol=1e-15)


def test_hermite_values_and_aliasing():
    """H_xx = c_x^2 - 1/3, H_xy = c_x c_y, H_xxy = c_y (c_x^2 - 1/3),
    H_xxyy = (c_x^2 - 1/3)(c_y^2 - 1/3); on D2Q9 H_xxx = H_xxxy = 0 and
    H_xxxx = -H_xx."""
    assert np.allclose(Hvec((0, 0)), CX ** 2 - 1 / 3, atol=1e-16)
    assert np.allclose(Hvec((1, 1)), CY ** 2 - 1 / 3, atol=1e-16)
    assert np.allclose(Hvec((0, 1)), CX * CY, atol=1e-16)
    assert np.allclose(Hvec((0, 0, 1)), CY * (CX ** 2 - 1 / 3), atol=1e-16)
    assert np.allclose(Hvec((0, 1, 1)), CX * (CY ** 2 - 1 / 3), atol=1e-16)
    assert np.allclose(Hvec((0, 0, 1, 1)),
                       (CX ** 2 - 1 / 3) * (CY ** 2 - 1 / 3), atol=1e-16)
    assert np.allclose(Hvec((0, 0, 0)), 0, atol=1e-16)
    assert np.allclose(Hvec((0, 0, 0, 1)), 0, atol=1e-16)
    assert np.allclose(Hvec((0, 0, 0, 0)), -Hvec((0, 0)), atol=1e-16)
    # full index symmetry of the fourth-order tensor
    for perm in [(0, 1, 0, 1), (1, 0, 1, 0), (1, 1, 0, 0), (0, 1, 1, 0)]:
        assert np.allclose(Hvec(perm), Hvec((0, 0, 1, 1)), atol=1e-16)


# --------------------------------------------------------------------------
# Equilibria (algorithm task 2)
# --------------------------------------------------------------------------
def phi(c, u):
    """D1Q3 equilibrium factor: phi(0,u) = 2/3 - u^2,
    phi(+-1,u) = 1/6 +- u/2 + u^2/2."""
    return np.where(c == 0, 2 / 3 - u * u, 1 / 6 + c * u / 2 + u * u / 2)


@pytest.mark.parametrize("trial", range(5))
def test_feq_is_d1q3_product_without_field(trial):
    rho = 1 + 0.1 * RNG.standard_normal()
    u = 0.1 * RNG.standard_normal(2)
    feq, _ = oracle.node_equilibrium(rho, u, [0.0, 0.0])
    expect = rho * phi(CX, u[0]) * phi(CY, u[1])
    assert np.allclose(feq, expect, rtol=0, atol=2e-16)


@pytest.mark.parametrize("trial", range(5))
def test_maxwell_term_closed_form(trial):
    rho = 1 + 0.1 * RNG.standard_normal()
    u = 0.1 * RNG.standard_normal(2)
    b = 0.1 * RNG.standard_normal(2)
    f1, _ = oracle.node_equilibrium(rho, u, b)
    f0, _ = oracle.node_equilibrium(rho, u, [0.0, 0.0])
    bx, by = b
    expect = np.zeros(9)
    expect[[2, 6]] = 0.25 * (by * by - bx * bx)
    expect[[4, 8]] = 0.25 * (bx * bx - by * by)
    diag = [1, 3, 5, 7]
    expect[diag] = -CX[diag] * CY[diag] * bx * by / 4
    assert np.allclose(f1 - f0, expect, rtol=0, atol=2e-16)


@pytest.mark.parametrize("trial", range(5))
def test_feq_hermite_moments(trial):
    """Moments of f_eq: rho, rho u, rho uu + M, rho ux^2 uy, rho ux uy^2,
    rho ux^2 uy^2."""
    rho = 1 + 0.1 * RNG.standard_normal()
    u = 0.1 * RNG.standard_normal(2)
    b = 0.1 * RNG.standard_normal(2)
    feq, _ = oracle.node_equilibrium(rho, u, b)
    M = 0.5 * (b @ b) * np.eye(2) - np.outer(b, b)
    tol = 1e-15
    assert abs(feq.sum() - rho) < tol
    assert abs((feq * CX).sum() - rho * u[0]) < tol
    assert abs((feq * CY).sum() - rho * u[1]) < tol
    for a in range(2):
        for c in range(2):
            m = (feq * Hvec((a, c))).sum()
            assert abs(m - (rho * u[a] * u[c] + M[a, c])) < tol
    assert abs((feq * Hvec((0, 0, 1))).sum() - rho * u[0] ** 2 * u[1]) < tol
    assert abs((feq * Hvec((0, 1, 1))).sum() - rho * u[0] * u[1] ** 2) < tol
    assert abs((feq * Hvec((0, 0, 1, 1))).sum()
               - rho * u[0] ** 2 * u[1] ** 2) < tol


def test_feq_algorithm_equals_hermite_series():
    """The algorithm's f_eq equals w_i sum_n a0:H/(n! cs^2n) with the Maxwell
    tensor at second order only (the equivalence of the two forms)."""
    for _ in range(5):
        rho = 1 + 0.1 * RNG.standard_normal()
        u = 0.1 * RNG.standard_normal(2)
        b = 0.1 * RNG.standard_normal(2)
        f1, _ = oracle.node_equilibrium(rho, u, b)
        f2 = oracle.node_feq_series(rho, u, b, full=False)
        assert np.allclose(f1, f2, rtol=0, atol=1e-16)


@pytest.mark.parametrize("trial", range(5))
def test_full_series_adds_cross_terms_only(trial):
    """The equilibrium with the u.M cross terms of Eq. eq:a0_4 (the ablation
    of the reading that the algorithm keeps M at second order only) has the
    same moments up to second order, and its third and fourth supported
    Hermite moments are the hand-expanded components
      xxy:  rho ux^2 uy + uy Mxx + 2 ux Mxy,
      xyy:  rho ux uy^2 + ux Myy + 2 uy Mxy,
      xxyy: rho ux^2 uy^2 + ux^2 Myy + uy^2 Mxx + 4 ux uy Mxy."""
    rho = 1 + 0.1 * RNG.standard_normal()
    u = 0.1 * RNG.standard_normal(2)
    b = 0.1 * RNG.standard_normal(2)
    M = 0.5 * (b @ b) * np.eye(2) - np.outer(b, b)
    ux, uy = u
    for fB in (oracle.node_feq_series(rho, u, b, full=True),
               oracle.node_equilibrium(rho, u, b, option=oracle.FEQ_SERIES_FULL)[0]):
        tol = 1e-15
        assert abs(fB.sum() - rho) < tol
        assert abs((fB * CX).sum() - rho * ux) < tol
        assert abs((fB * CY).sum() - rho * uy) < tol
        for a in range(2):
            for c in range(2):
                m = (fB * Hvec((a, c))).sum()
                assert abs(m - (rho * u[a] * u[c] + M[a, c])) < tol
        assert abs((fB * Hvec((0, 0, 1))).sum()
                   - (rho * ux ** 2 * uy + uy * M[0, 0] + 2 * ux * M[0, 1])) < tol
        assert abs((fB * Hvec((0, 1, 1))).sum()
                   - (rho * ux * uy ** 2 + ux * M[1, 1] + 2 * uy * M[0, 1])) < tol
        assert abs((fB * Hvec((0, 0, 1, 1))).sum()
                   - (rho * ux ** 2 * uy ** 2 + ux ** 2 * M[1, 1]
                      + uy ** 2 * M[0, 0] + 4 * ux * uy * M[0, 1])) < tol


def test_full_series_difference_size():
    """B - A at |u_a| = |b_a| = 0.05 per component is of order 1e-4 (the size
    quoted for the difference of the two readings), and vanishes at b = 0:
    without a field both equilibria are the hydrodynamic one (Sec. II)."""
    u, b = np.array([0.05, 0.05]), np.array([0.05, -0.05])
    fA, _ = oracle.node_equilibrium(1.0, u, b)
    fB, _ = oracle.node_equilibrium(1.0, u, b, option=oracle.FEQ_SERIES_FULL)
    d = np.abs(fB - fA).max()
    assert 1e-5 < d < 3e-4
    fA0, _ = oracle.node_equilibrium(1.0, u, [0.0, 0.0])
    fB0, _ = oracle.node_equilibrium(1.0, u, [0.0, 0.0], option=oracle.FEQ_SERIES_FULL)
    assert np.allclose(fA0, fB0, rtol=0, atol=1e-16)  # product vs series order


def test_full_series_grid_conserves_and_reduces_without_field():
    """The grid run with the full-series equilibrium conserves mass,
    momentum and sum b on a periodic grid, and with b = 0 follows the
    algorithm's run to round-off."""
    n = 16
    u, b = inputs.random_modes(n, n, 0.04, seed=5)
    o = oracle.Oracle(n, n, 0.56, 0.58, option=oracle.FEQ_SERIES_FULL)
    o.init(u, b)
    inv0 = o.invariants()
    o.step(50)
    assert np.allclose(o.invariants(), inv0, rtol=0, atol=1e-12)
    z = np.zeros_like(b)
    oA = oracle.Oracle(n, n, 0.56, 0.58)
    oB = oracle.Oracle(n, n, 0.56, 0.58, option=oracle.FEQ_SERIES_FULL)
    oA.init(u, z)
    oB.init(u, z)
    oA.step(50)
    oB.step(50)
    for xa, xb in zip(oA.moments(), oB.moments()):
        assert np.allclose(xa, xb, rtol=0, atol=1e-15)


@pytest.mark.parametrize("trial", range(5))
def test_geq_moments(trial):
    """sum g_eq = b; sum e_a g_eq,b = u_a b_b - u_b b_a (the sign the
    induction equation needs); sum e_a e_c g_eq,b = b_b delta_ac / 3."""
    u = 0.1 * RNG.standard_normal(2)
    b = 0.1 * RNG.standard_normal(2)
    _, geq = oracle.node_equilibrium(1.0, u, b)
    g = geq.reshape(5, 2)
    E = [EX, EY]
    assert np.allclose(g.sum(0), b, atol=1e-16)
    for a in range(2):
        for bb in range(2):
            assert abs((E[a] * g[:, bb]).sum()
                       - (u[a] * b[bb] - u[bb] * b[a])) < 1e-16
            for c in range(2):
                assert abs((E[a] * E[c] * g[:, bb]).sum()
                           - b[bb] * (a == c) / 3) < 1e-16


# --------------------------------------------------------------------------
# Non-equilibrium coefficients, reconstruction, collision (tasks 3-5)
# --------------------------------------------------------------------------
def random_node(amp=0.01):
    u0 = 0.08 * RNG.standard_normal(2)
    b0 = 0.08 * RNG.standard_normal(2)
    feq, geq = oracle.node_equilibrium(1.0 + 0.05 * RNG.standard_normal(),
                                       u0, b0)
    f = feq + amp * RNG.standard_normal(9) * feq
    g = geq + amp * 0.1 * RNG.standard_normal(10)
    return f, g


@pytest.mark.parametrize("trial", range(5))
def test_a1_and_recursion_closed_forms(trial):
    f, g = random_node()
    _, _, A = oracle.node_collide(f, g, 1 / 0.56, 1 / 0.56)
    rho, u, b = A["rho"], A["u"], A["b"]
    M = 0.5 * (b @ b) * np.eye(2) - np.outer(b, b)
    a = A["a2"]
    tol = 2e-16
    assert abs(a[0, 0] - ((f * CX * CX).sum() - rho / 3 - rho * u[0] ** 2
                          - M[0, 0])) < tol
    assert abs(a[0, 1] - ((f * CX * CY).sum() - rho * u[0] * u[1]
                          - M[0, 1])) < tol
    assert abs(a[1, 1] - ((f * CY * CY).sum() - rho / 3 - rho * u[1] ** 2
                          - M[1, 1])) < tol
    a3, a4 = A["a3"], A["a4"]
    assert abs(a3[0, 0, 1] - (2 * u[0] * a[0, 1] + u[1] * a[0, 0])) < tol
    assert abs(a3[0, 1, 1] - (2 * u[1] * a[0, 1] + u[0] * a[1, 1])) < tol
    assert abs(a4[0, 0, 1, 1] - (u[0] ** 2 * a[1, 1] + u[1] ** 2 * a[0, 0]
                                 + 4 * u[0] * u[1] * a[0, 1])) < tol
    # the aliased components the support mask drops
    assert abs(a3[0, 0, 0] - 3 * u[0] * a[0, 0]) < tol
    assert abs(a4[0, 0, 0, 0] - 6 * u[0] ** 2 * a[0, 0]) < tol


@pytest.mark.parametrize("trial", range(5))
def test_regularised_moments(trial):
    """f_neq,reg has zero mass and momentum and returns a1^(2), a1_xxy,
    a1_xyy and a1_xxyy as its Hermite moments."""
    f, g = random_node()
    _, _, A = oracle.node_collide(f, g, 1 / 0.56, 1 / 0.56)
    fr = A["fneq_reg"]
    tol = 1e-17
    assert abs(fr.sum()) < tol
    assert abs((fr * CX).sum()) < tol and abs((fr * CY).sum()) < tol
    for a in range(2):
        for c in range(2):
            assert abs((fr * Hvec((a, c))).sum() - A["a2"][a, c]) < tol
    assert abs((fr * Hvec((0, 0, 1))).sum() - A["a3"][0, 0, 1]) < tol
    assert abs((fr * Hvec((0, 1, 1))).sum() - A["a3"][0, 1, 1]) < tol
    assert abs((fr * Hvec((0, 0, 1, 1))).sum() - A["a4"][0, 0, 1, 1]) < tol


@pytest.mark.parametrize("trial", range(5))
def test_post_collision_moments(trial):
    f, g = random_node()
    om, omm = 1 / 0.53, 1 / 0.61
    fs, gs, A = oracle.node_collide(f, g, om, omm)
    rho, u, b = A["rho"], A["u"], A["b"]
    M = 0.5 * (b @ b) * np.eye(2) - np.outer(b, b)
    tol = 1e-15
    assert abs(fs.sum() - rho) < tol
    assert abs((fs * CX).sum() - rho * u[0]) < tol
    assert abs((fs * CY).sum() - rho * u[1]) < tol
    for a in range(2):
        for c in range(2):
            assert abs((fs * Hvec((a, c))).sum()
                       - (rho * u[a] * u[c] + M[a, c]
                          + (1 - om) * A["a2"][a, c])) < tol
    assert np.allclose(gs.reshape(5, 2).sum(0), b, atol=1e-16)


def _frac(p, q=1):
    return Fr(p, q)


def _exact_equilibria(rho, ux, uy, bx, by, K=_frac):
    """f_eq (D1Q3 product form + hand-expanded Maxwell term) and g_eq of one
    node; K(p, q) makes the constant p/q in the arithmetic in use."""
    def ph(c, v):
        return K(2, 3) - v * v if c == 0 else K(1, 6) + c * v / 2 + v * v / 2

    feq = []
    for i in range(9):
        cx, cy = int(CX[i]), int(CY[i])
        m = K(0)
        if i in (2, 6):
            m = (by * by - bx * bx) / 4
        elif i in (4, 8):
            m = (bx * bx - by * by) / 4
        elif i != 0:
            m = -cx * cy * bx * by / 4
        feq.append(rho * ph(cx, ux) * ph(cy, uy) + m)
    E = ux * by - uy * bx
    psi = [K(1, 3)] + [K(1, 6)] * 4
    geq = []
    for j in range(5):
        geq.append(psi[j] * (bx - 3 * int(EY[j]) * E))
        geq.append(psi[j] * (by + 3 * int(EX[j]) * E))
    return feq, geq


def _exact_collide_k(f, g, om, omm, K=_frac):
    """Single-node collision from the hand expansion in the arithmetic of K:
    closed-form a1, closed-form recursion, reconstruction with 9/2, 27/2 and
    81/4.  f, g, om, omm are already numbers of that arithmetic."""
    t = K(1, 3)
    rho = sum(f)
    ux = sum(fi * c for fi, c in zip(f, CX)) / rho
    uy = sum(fi * c for fi, c in zip(f, CY)) / rho
    bx = sum(g[0::2])
    by = sum(g[1::2])
    W = [K(4, 9), K(1, 36), K(1, 9), K(1, 36), K(1, 9), K(1, 36),
         K(1, 9), K(1, 36), K(1, 9)]
    feq, geq = _exact_equilibria(rho, ux, uy, bx, by, K)
    Mxx = (by * by - bx * bx) / 2
    Myy = -Mxx
    Mxy = -bx * by
    axx = sum(fi * int(c) * int(c) for fi, c in zip(f, CX)) - rho * t - rho * ux * ux - Mxx
    ayy = sum(fi * int(c) * int(c) for fi, c in zip(f, CY)) - rho * t - rho * uy * uy - Myy
    axy = sum(fi * int(a) * int(c) for fi, a, c in zip(f, CX, CY)) - rho * ux * uy - Mxy
    axxy = 2 * ux * axy + uy * axx
    axyy = 2 * uy * axy + ux * ayy
    axxyy = ux * ux * ayy + uy * uy * axx + 4 * ux * uy * axy
    fs = []
    for i in range(9):
        cx, cy = int(CX[i]), int(CY[i])
        hxx, hyy, hxy = cx * cx - t, cy * cy - t, K(cx * cy)
        r = (K(9, 2) * (hxx * axx + 2 * hxy * axy + hyy * ayy)
             + K(27, 2) * (cy * hxx * axxy + cx * hyy * axyy)
             + K(81, 4) * hxx * hyy * axxyy)
        fs.append(feq[i] + (1 - om) * W[i] * r)
    gs = [geq[k] + (1 - omm) * (g[k] - geq[k]) for k in range(10)]
    return fs, gs


def _exact_collide(f, g, omega, omega_m):
    """Single-node collision in exact rational arithmetic."""
    fs, gs = _exact_collide_k([Fr(x) for x in f], [Fr(x) for x in g], Fr(omega), Fr(omega_m))
    return [float(x) for x in fs], [float(x) for x in gs]


@pytest.mark.parametrize("trial", range(4))
def test_collision_exact_rational(trial):
    f, g = random_node(0.03)
    om, omm = 1 / 0.51, 1 / 0.57
    fs, gs, _ = oracle.node_collide(f, g, om, omm)
    efs, egs = _exact_collide(f, g, om, omm)
    assert np.allclose(fs, efs, rtol=0, atol=1e-15)
    assert np.allclose(gs, egs, rtol=0, atol=1e-16)


def _grid_run_hand(u, b, tau_f, tau_m, steps, K, num):
    """Whole periodic grid from the hand expansion: equilibrium
    initialisation at rho = 1, then collide and push-stream (f*_i(x) moves to
    x + c_i, g*_j(x) to x + e_j), in the arithmetic of K (constants) and num
    (float inputs, converted exactly).  Returns the pre-collision moments
    (rho, u, b) after each step as floats."""
    ny, nx = u.shape[1:]
    om, omm = 1 / num(tau_f), 1 / num(tau_m)
    F = [[None] * nx for _ in range(ny)]
    G = [[None] * nx for _ in range(ny)]
    for y in range(ny):
        for x in range(nx):
            F[y][x], G[y][x] = _exact_equilibria(K(1), num(u[0, y, x]), num(u[1, y, x]),
                                                 num(b[0, y, x]), num(b[1, y, x]), K)
    out = []
    for _ in range(steps):
        Fn = [[[None] * 9 for _ in range(nx)] for _ in range(ny)]
        Gn = [[[None] * 10 for _ in range(nx)] for _ in range(ny)]
        for y in range(ny):
            for x in range(nx):
                fs, gs = _exact_collide_k(F[y][x], G[y][x], om, omm, K)
                for i in range(9):
                    Fn[(y + int(CY[i])) % ny][(x + int(CX[i])) % nx][i] = fs[i]
                for j in range(5):
                    yy, xx = (y + int(EY[j])) % ny, (x + int(EX[j])) % nx
                    Gn[yy][xx][2 * j] = gs[2 * j]
                    Gn[yy][xx][2 * j + 1] = gs[2 * j + 1]
        F, G = Fn, Gn
        rho = np.zeros((ny, nx)); uu = np.zeros((2, ny, nx)); bb = np.zeros((2, ny, nx))
        for y in range(ny):
            for x in range(nx):
                f, g = F[y][x], G[y][x]
                r = sum(f)
                rho[y, x] = float(r)
                uu[0, y, x] = float(sum(fi * int(c) for fi, c in zip(f, CX)) / r)
                uu[1, y, x] = float(sum(fi * int(c) for fi, c in zip(f, CY)) / r)
                bb[0, y, x] = float(sum(g[0::2]))
                bb[1, y, x] = float(sum(g[1::2]))
        out.append((rho, uu, bb))
    return out


@pytest.mark.parametrize("shape,steps", [((3, 3), 5), ((5, 4), 5), ((1, 1), 3), ((2, 1), 3)])
def test_tiny_grid_high_precision(shape, steps):
    """Tiny periodic grids, 1 to 5 steps: the oracle (generic Hermite
    tensors, FP64) against the hand expansion run in 50-digit decimal
    arithmetic, field by field."""
    from decimal import Decimal, localcontext
    nx, ny = shape
    rng = np.random.default_rng(nx * 10 + ny)
    u = 0.05 * rng.standard_normal((2, ny, nx))
    b = 0.05 * rng.standard_normal((2, ny, nx))
    with localcontext() as ctx:
        ctx.prec = 50
        ref = _grid_run_hand(u, b, 0.53, 0.57, steps, lambda p, q=1: Decimal(p) / Decimal(q),
                             lambda v: Decimal(float(v)))
    o = oracle.Oracle(nx, ny, 0.53, 0.57)
    o.init(u, b)
    for k in range(steps):
        o.step(1)
        rho, uu, bb = o.moments()
        r_rho, r_u, r_b = ref[k]
        assert np.max(np.abs(rho - r_rho)) < 1e-14, k
        assert np.max(np.abs(uu - r_u)) < 1e-15, k
        assert np.max(np.abs(bb - r_b)) < 1e-15, k
    o.close()


def test_tiny_grid_decimal_equals_exact():
    """The 50-digit run of the hand expansion equals the exact-rational one
    on a 3 x 3 grid over 2 steps (to far below FP64 resolution)."""
    from decimal import Decimal, localcontext
    rng = np.random.default_rng(7)
    u = 0.05 * rng.standard_normal((2, 3, 3))
    b = 0.05 * rng.standard_normal((2, 3, 3))
    exact = _grid_run_hand(u, b, 0.53, 0.57, 2, _frac, Fr)
    with localcontext() as ctx:
        ctx.prec = 50
        dec = _grid_run_hand(u, b, 0.53, 0.57, 2, lambda p, q=1: Decimal(p) / Decimal(q),
                             lambda v: Decimal(float(v)))
    for (a0, a1, a2), (b0, b1, b2) in zip(exact, dec):
        assert np.array_equal(a0, b0) and np.array_equal(a1, b1) and np.array_equal(a2, b2)


# --------------------------------------------------------------------------
# Whole-grid properties
# --------------------------------------------------------------------------
def test_conservation_periodic():
    n = 24
    u, b = inputs.orszag_tang(n, 0.05, 0.05, perturb=1e-3, seed=3)
    o = oracle.Oracle(n, n, 0.52, 0.58)
    o.init(u, b)
    inv0 = o.invariants()
    o.step(60)
    inv1 = o.invariants()
    assert abs(inv1[0] - inv0[0]) < 1e-12 * n * n
    assert np.all(np.abs(inv1[1:] - inv0[1:]) < 1e-14 * n * n)


def test_uniform_state_is_fixed_point():
    n = 6
    u = np.zeros((2, n, n)); u[0] = 0.03; u[1] = -0.02
    b = np.zeros((2, n, n)); b[0] = 0.04; b[1] = 0.01
    o = oracle.Oracle(n, n, 0.55, 0.6)
    o.init(u, b)
    f0, g0 = o.get_state()
    o.step(10)
    f1, g1 = o.get_state()
    # an exact fixed point; only round-off may move it
    assert np.allclose(f1, f0, rtol=0, atol=2e-15)
    assert np.allclose(g1, g0, rtol=0, atol=2e-16)


def test_zero_steps_returns_initial_fields():
    u, b = inputs.orszag_tang(16, 0.05, 0.05, perturb=1e-4)
    o = oracle.Oracle(16, 16, 0.56, 0.56)
    o.init(u, b)
    rho, uu, bb = o.moments()
    assert np.allclose(rho, 1.0, atol=1e-16)
    assert np.allclose(uu, u, atol=1e-17) and np.allclose(bb, b, atol=1e-17)


def test_translation_equivariance():
    n = 16
    u, b = inputs.turbulence(n, 0.04)
    sh = (3, -5)
    o1 = oracle.Oracle(n, n, 0.53, 0.57); o1.init(u, b); o1.step(12)
    u2 = np.roll(u, sh, axis=(1, 2)); b2 = np.roll(b, sh, axis=(1, 2))
    o2 = oracle.Oracle(n, n, 0.53, 0.57); o2.init(u2, b2); o2.step(12)
    r1, v1, c1 = o1.moments(); r2, v2, c2 = o2.moments()
    assert np.allclose(np.roll(v1, sh, axis=(1, 2)), v2, rtol=0, atol=1e-16)
    assert np.allclose(np.roll(c1, sh, axis=(1, 2)), c2, rtol=0, atol=1e-16)


def _rot90(v):
    """Rotate a vector field [2][y][x] by +90 degrees about node (0,0):
    new(x', y') = R old(R^-1 x'), R (vx, vy) = (-vy, vx)."""
    n = v.shape[1]
    out = np.empty_like(v)
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    sx, sy = yy % n, (-xx) % n  # R^-1 (x', y') = (y', -x')
    out[0] = -v[1][sy, sx]
    out[1] = v[0][sy, sx]
    return out


def _reflect_x(v):
    """Mirror x -> -x: (vx, vy)(x, y) -> (-vx, vy)(-x, y)."""
    n = v.shape[2]
    idx = (-np.arange(n)) % n
    out = v[:, :, idx].copy()
    out[0] *= -1
    return out


@pytest.mark.parametrize("op", [_rot90, _reflect_x])
def test_d4_equivariance(op):
    n = 16
    u, b = inputs.turbulence(n, 0.05, seed_psi=5, seed_a=6)
    o1 = oracle.Oracle(n, n, 0.52, 0.6); o1.init(u, b); o1.step(15)
    o2 = oracle.Oracle(n, n, 0.52, 0.6); o2.init(op(u), op(b)); o2.step(15)
    _, v1, c1 = o1.moments(); _, v2, c2 = o2.moments()
    # equal up to round-off (the rotated sums run in another order)
    assert np.allclose(op(v1), v2, rtol=0, atol=2e-15)
    assert np.allclose(op(c1), c2, rtol=0, atol=2e-15)


def test_point_symmetry_unperturbed_ot():
    """The unperturbed Orszag-Tang fields are odd about node (0,0) and stay
    so: (u, b)(-x) = -(u, b)(x)."""
    n = 32
    u, b = inputs.orszag_tang(n, 0.05, 0.05)
    o = oracle.Oracle(n, n, 0.56, 0.56); o.init(u, b); o.step(40)
    _, v, c = o.moments()
    idx = (-np.arange(n)) % n
    for fld in (v, c):
        assert np.allclose(fld[:, idx][:, :, idx], -fld, rtol=0, atol=1e-15)


def test_no_field_keeps_magnetic_populations_zero():
    """M = 0: with b = 0 the magnetic populations stay exactly zero and the
    fluid evolves as hydrodynamic RR."""
    n = 12
    u, _ = inputs.turbulence(n, 0.05)
    b = np.zeros_like(u)
    o = oracle.Oracle(n, n, 0.55, 0.55); o.init(u, b); o.step(10)
    _, g = o.get_state()
    assert np.all(g == 0.0)


# --------------------------------------------------------------------------
# Analytic rates (transport coefficients nu = cs^2 (tau - 1/2) etc.)
# --------------------------------------------------------------------------
def _amp(field, k, axis_coord):
    s = np.sin(k * axis_coord)
    return 2.0 * np.mean(field * s)


@pytest.mark.parametrize("tau", [0.56, 0.8])
def test_shear_wave_decay(tau):
    N, A, T = 64, 1e-3, 400
    k = 2 * np.pi / N
    y = np.arange(N)
    u = np.zeros((2, N, 1)); u[0, :, 0] = A * np.sin(k * y)
    b = np.zeros((2, N, 1))
    o = oracle.Oracle(1, N, tau, 0.6); o.init(u, b)
    # measure between two times so that the start-up transient of the
    # equilibrium initialisation drops out
    o.step(100)
    a1 = _amp(o.moments()[1][0, :, 0], k, y)
    o.step(T)
    a2 = _amp(o.moments()[1][0, :, 0], k, y)
    nu = (tau - 0.5) / 3
    rate = -math.log(a2 / a1) / T
    assert abs(rate / (nu * k * k) - 1) < 0.01


@pytest.mark.parametrize("tau_m", [0.55, 0.9])
def test_magnetic_diffusion_decay(tau_m):
    N, A, T = 64, 1e-3, 400
    k = 2 * np.pi / N
    y = np.arange(N)
    u = np.zeros((2, N, 1))
    b = np.zeros((2, N, 1)); b[0, :, 0] = A * np.sin(k * y)
    o = oracle.Oracle(1, N, 0.6, tau_m); o.init(u, b)
    o.step(100)
    a1 = _amp(o.moments()[2][0, :, 0], k, y)
    o.step(T)
    a2 = _amp(o.moments()[2][0, :, 0], k, y)
    eta = (tau_m - 0.5) / 3
    rate = -math.log(a2 / a1) / T
    assert abs(rate / (eta * k * k) - 1) < 0.01


def test_alfven_wave_equal_diffusivities():
    """z+ = u_y + b_y travels in -x at speed B0 and decays as exp(-nu k^2 t)."""
    N, A, B0, tau = 128, 1e-4, 0.05, 0.56
    k = 2 * np.pi / N
    x = np.arange(N)
    u = np.zeros((2, 1, N)); u[1, 0] = A * np.sin(k * x)
    b = np.zeros((2, 1, N)); b[0] = B0; b[1, 0] = A * np.sin(k * x)
    T = 600
    o = oracle.Oracle(N, 1, tau, tau); o.init(u, b); o.step(T)
    _, v, c = o.moments()
    zp = v[1, 0] + c[1, 0]
    zhat = np.fft.fft(zp)[1] / N  # coefficient of exp(i k x)
    z0 = 2 * A / 2j  # 2A sin(kx) -> coefficient 2A/(2i)
    ratio = zhat / z0
    nu = (tau - 0.5) / 3
    assert abs(-math.log(abs(ratio)) / T / (nu * k * k) - 1) < 0.01
    # sin(k(x + B0 t)): phase advances by +k B0 t
    phase = np.angle(ratio)
    assert abs(phase / (k * B0 * T) - 1) < 0.01


def test_alfven_wave_unequal_diffusivities():
    """Modes obey l^2 + (nu+eta) k^2 l + nu eta k^4 + B0^2 k^2 = 0: envelope
    decay (nu+eta) k^2 / 2, frequency sqrt(B0^2 k^2 - (nu-eta)^2 k^4 / 4)."""
    N, A, B0, tf, tm = 128, 1e-4, 0.05, 0.6, 0.55
    k = 2 * np.pi / N
    x = np.arange(N)
    u = np.zeros((2, 1, N)); u[1, 0] = A * np.sin(k * x)
    b = np.zeros((2, 1, N)); b[0] = B0
    nu, eta = (tf - 0.5) / 3, (tm - 0.5) / 3
    o = oracle.Oracle(N, 1, tf, tm); o.init(u, b)
    ts, uh = [], []
    for _ in range(60):
        o.step(20)
        _, v, _ = o.moments()
        ts.append(o.step_count)
        uh.append(np.fft.fft(v[1, 0])[1] / N)
    ts = np.array(ts, float); uh = np.array(uh)
    # u_y's k-mode with u(0) = A, b(0) = 0:
    # e^{-gamma t} [cos(w t) + (eta - nu) k^2 / (2 w) sin(w t)]
    gamma = (nu + eta) * k * k / 2
    w = math.sqrt(B0 ** 2 * k ** 2 - (nu - eta) ** 2 * k ** 4 / 4)
    amp = np.abs(uh) / (A / 2)
    model = np.exp(-gamma * ts) * np.abs(np.cos(w * ts) + (eta - nu) * k * k
                                         / (2 * w) * np.sin(w * ts))
    assert np.max(np.abs(amp - model)) < 0.01


def test_forced_box_exact_momentum_growth():
    n = 8
    G = 1e-5
    u = np.zeros((2, n, n)); b = np.zeros((2, n, n))
    o = oracle.Oracle(n, n, 0.6, 0.6, force=(G, 0.0)); o.init(u, b)
    m0 = o.invariants()
    o.step(50)
    m1 = o.invariants()
    assert abs((m1[1] - m0[1]) - 50 * G * n * n) < 1e-16 * n * n * 50
    assert abs(m1[0] - m0[0]) < 1e-12  # round-off on a sum of 64 masses


# --------------------------------------------------------------------------
# Hartmann channel (walls + forcing) against its closed form
# --------------------------------------------------------------------------
def hartmann_closed_form(h, y):
    """Steady u(y'), b_x(y') of 0 = G + nu u'' + B0 b_x', 0 = B0 u' + eta b_x''
    with no-slip insulating walls at y' = +-a."""
    a, Ha, B0 = h.a, h.Ha, h.B0
    yp = y - (h.ny - 1) / 2.0
    u = (h.G * a * a / (h.nu * Ha)) * (math.cosh(Ha) - np.cosh(Ha * yp / a)) \
        / math.sinh(Ha)
    bx = (h.G * a / B0) * (np.sinh(Ha * yp / a) / math.sinh(Ha) - yp / a)
    return u, bx


def run_hartmann_oracle(h, tol_change=1e-12, chunk=2000, max_steps=10 ** 7):
    o = oracle.Oracle(1, h.ny, h.tau_f, h.tau_m, walls=True, force=(h.G, 0.0),
                      b_wall=(0.0, h.B0))
    u, b = h.initial_fields()
    o.init(u[:, :, :1], b[:, :, :1])
    _, prev, _ = o.moments()
    while o.step_count < max_steps:
        o.step(chunk)
        _, v, c = o.moments()
        if np.max(np.abs(v - prev)) < tol_change * chunk / 1e4:
            break
        prev = v
    return o, v[0, :, 0], c[0, :, 0]


def test_hartmann_closed_form_small():
    """Ha = 4 channel with fast transport: second-order convergence to the
    closed form between ny = 32 and ny = 64."""
    errs = []
    for ny in (32, 64):
        h = inputs.Hartmann(nx=1, ny=ny, tau_f=0.8, tau_m=0.75, G=1e-6 * 4096
                            / ny ** 2, Ha=4.0)
        o, u, bx = run_hartmann_oracle(h)
        ue, be = hartmann_closed_form(h, np.arange(ny))
        errs.append((np.linalg.norm(u - ue) / np.linalg.norm(ue),
                     np.linalg.norm(bx - be) / np.linalg.norm(be)))
    (eu1, eb1), (eu2, eb2) = errs
    assert eu2 < 3e-3 and eb2 < 3e-3
    assert eu1 / eu2 > 3.0 and eb1 / eb2 > 3.0


@pytest.mark.slow
def test_hartmann_c2_closed_form():
    """The 512 x 256 Hartmann configuration (run on its x-invariant 1 x 256
    column): rel L2 <= 1e-3 for u and b_x against the closed form."""
    h = inputs.hartmann_c2()
    h.nx = 1
    o, u, bx = run_hartmann_oracle(h, chunk=20000)
    ue, be = hartmann_closed_form(h, np.arange(h.ny))
    assert np.linalg.norm(u - ue) / np.linalg.norm(ue) < 1e-3
    assert np.linalg.norm(bx - be) / np.linalg.norm(be) < 1e-3


# --------------------------------------------------------------------------
# Values the paper prints (Tables 1-3, RR column, N = 128)
# --------------------------------------------------------------------------
def test_paper_tables_low_re_n128():
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "ot_lowre_rr_n128.json")) as fh:
        gold = json.load(fh)
    p = inputs.orszag_tang_paper(128)
    o = oracle.Oracle(128, 128, p["tau"], p["tau"])
    o.init(p["u"], p["b"])
    for t in ("0.5", "1.0"):
        o.step(int(round(float(t) * p["steps_per_unit"])) - o.step_count)
        jz, wz = o.current_vorticity()
        jmax = np.abs(jz).max() * p["scale"]
        wmax = np.abs(wz).max() * p["scale"]
        assert abs(jmax / gold["j_max"][t] - 1) < 0.03, (t, jmax)
        assert abs(wmax / gold["omega_max"][t] - 1) < 0.03, (t, wmax)
        if t == "1.0":
            divb = o.diagnostics()[2] * p["scale"]
            assert abs(divb / gold["max_div_b"][t] - 1) < 0.01, divb


def test_ot_initial_energies():
    """Unperturbed OT at t = 0: E_kin = E_mag = u0^2 / 2."""
    u, b = inputs.orszag_tang(64, 0.05, 0.05)
    o = oracle.Oracle(64, 64, 0.56, 0.56); o.init(u, b)
    ek, em, _ = o.diagnostics()
    assert abs(ek - 0.05 ** 2 / 2) < 1e-15 and abs(em - 0.05 ** 2 / 2) < 1e-15


# --------------------------------------------------------------------------
# Current density and vorticity fields: sign and magnitude
# --------------------------------------------------------------------------
def _wavenumbers(n):
    k = 2 * np.pi * np.fft.fftfreq(n)
    return k[None, :], k[:, None]


def _curl_spectral(vx, vy):
    """d_x v_y - d_y v_x of a periodic field, exact for its Fourier modes."""
    kx, ky = _wavenumbers(vx.shape[0])
    return np.real(np.fft.ifft2(1j * kx * np.fft.fft2(vy) - 1j * ky * np.fft.fft2(vx)))


def _curl_isotropic_spectral(vx, vy):
    """The same curl with the isotropic lattice gradient of Sec. III.  Its
    Fourier symbol follows from summing w_i c_i e^(i k.c_i) / c_s^2 over the
    nine D2Q9 velocities: d_x -> i sin(k_x) (2 + cos k_y) / 3, and likewise
    for d_y.  Applied here by FFT, not by the stencil."""
    kx, ky = _wavenumbers(vx.shape[0])
    dx = 1j * np.sin(kx) * (2 + np.cos(ky)) / 3
    dy = 1j * np.sin(ky) * (2 + np.cos(kx)) / 3
    return np.real(np.fft.ifft2(dx * np.fft.fft2(vy) - dy * np.fft.fft2(vx)))


def test_vorticity_is_isotropic_curl_of_u():
    """omega_z = d_x u_y - d_y u_x with the isotropic gradient, on a field
    whose u_x also varies in x and u_y in y (so swapped or sign-flipped
    derivatives cannot pass): at step 0, where u is the initial field, and
    after 30 steps against the curl of the oracle's own u."""
    n = 48
    k = 2 * np.pi / n
    x = np.arange(n)[None, :] * np.ones((n, 1))
    y = np.arange(n)[:, None] * np.ones((1, n))
    u = np.zeros((2, n, n))
    u[0] = 0.02 * np.sin(k * y + 0.4) + 0.01 * np.sin(k * x)
    u[1] = 0.04 * np.sin(2 * k * x + 1.0) + 0.01 * np.cos(k * y)
    b = np.zeros((2, n, n))
    b[0] = 0.01 * np.cos(k * x + 0.2)
    b[1] = 0.01 * np.sin(k * y)
    o = oracle.Oracle(n, n, 0.6, 0.7)
    o.init(u, b)
    _, wz = o.current_vorticity()
    ref = _curl_isotropic_spectral(u[0], u[1])
    assert np.abs(wz - ref).max() < 1e-15 * np.abs(ref).max() * 100
    # the exact symbol: single modes scale by sin(k)/k against the continuum
    w_cont = 0.04 * 2 * k * np.cos(2 * k * x + 1.0) - 0.02 * k * np.cos(k * y + 0.4)
    w_lat = 0.04 * np.sin(2 * k) * np.cos(2 * k * x + 1.0) - 0.02 * np.sin(k) * np.cos(k * y + 0.4)
    assert np.abs(wz - w_lat).max() < 1e-16 * 100
    assert np.sum(wz * w_cont) > 0.99 * np.linalg.norm(wz) * np.linalg.norm(w_cont)
    o.step(30)
    _, uu, _ = o.moments()
    _, wz = o.current_vorticity()
    ref = _curl_isotropic_spectral(uu[0], uu[1])
    assert np.abs(wz - ref).max() < 1e-13 * np.abs(ref).max()


def test_current_from_populations_is_curl_of_b():
    """j_z from the magnetic non-equilibrium (Eq. current) against the
    spectral curl d_x b_y - d_y b_x of the oracle's own b, for a weak field at
    rest (u stays O(b^2), so the electric-field term of the Chapman-Enskog
    expansion drops out).  The two agree in sign everywhere that matters and
    in magnitude to O(k^2): the relative error falls 4x per doubling of N."""
    errs = []
    for n in (32, 64):
        k = 2 * np.pi / n
        x = np.arange(n)[None, :] * np.ones((n, 1))
        y = np.arange(n)[:, None] * np.ones((1, n))
        b0 = 1e-3
        b = np.zeros((2, n, n))
        b[0] = b0 * (np.sin(k * y + 0.3) + 0.5 * np.cos(k * x))
        b[1] = 2 * b0 * np.sin(k * x + 1.1) + 0.3 * b0 * np.sin(k * y)
        o = oracle.Oracle(n, n, 0.6, 0.7)
        o.init(np.zeros((2, n, n)), b)
        o.step(40)  # the populations' own transient has decayed by (0.43)^40
        _, _, bb = o.moments()
        jz, _ = o.current_vorticity()
        ref = _curl_spectral(bb[0], bb[1])
        cos = np.sum(jz * ref) / (np.linalg.norm(jz) * np.linalg.norm(ref))
        assert cos > 0.9999
        errs.append(np.linalg.norm(jz - ref) / np.linalg.norm(ref))
    assert errs[0] < 5e-3 and errs[1] < 1.5e-3
    assert 3.5 < errs[0] / errs[1] < 4.5
