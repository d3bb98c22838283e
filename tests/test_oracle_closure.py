"""Pins of the oracle's learned-closure pieces (CPU): GELU in its tanh form,
reverse-mode gradients against central finite differences, the first Adam
step's closed form, and that a zero network leaves the method unchanged."""
import math

import numpy as np
import pytest

import oracle
from paper_2602_14667_amd import inputs

RNG = np.random.default_rng(7)


def random_params(scale=0.3):
    return scale * RNG.standard_normal(oracle.NPARAM)


def random_norm():
    mu = 0.01 * RNG.standard_normal(8)
    sig = 0.5 + RNG.random(8)
    so = 0.1 + RNG.random(3)
    return np.concatenate([mu, sig, so])


def gelu_erf(z):
    return 0.5 * z * (1 + math.erf(z / math.sqrt(2)))


def one_unit_net(w, b):
    """A network whose output is y0 = GELU(w * xhat_0 + b) exactly."""
    p = np.zeros(oracle.NPARAM)
    p[0] = w            # W1[0][0]
    p[512] = b          # b1[0]
    p[512 + 64 + 0] = 1.0   # W2[0][0]: z2_0 = h1_0
    # y0 = W3[0][0] * GELU(z2_0)
    p[512 + 64 + 4096 + 64 + 0] = 1.0
    return p


def test_gelu_tanh_form_values():
    """GELU(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))): compare a
    one-unit network with the formula evaluated here, and with the erf form
    within the known approximation error (< 1e-3)."""
    norm = np.concatenate([np.zeros(8), np.ones(8), np.ones(3)])
    for z in (-3.0, -1.0, -0.2, 0.0, 0.5, 1.0, 2.5):
        # feed z through the first layer (w = 1, b = 0) and a second GELU:
        p = one_unit_net(1.0, 0.0)
        x = np.zeros((1, 8)); x[0, 0] = z
        y = oracle.mlp_forward(p, norm, x)[0, 0]
        g1 = 0.5 * z * (1 + math.tanh(math.sqrt(2 / math.pi) * (z + 0.044715 * z ** 3)))
        g2 = 0.5 * g1 * (1 + math.tanh(math.sqrt(2 / math.pi) * (g1 + 0.044715 * g1 ** 3)))
        assert abs(y - g2) < 1e-15
        assert abs(g1 - gelu_erf(z)) < 1e-3


def test_gradient_against_central_differences():
    p = random_params()
    norm = random_norm()
    x = 0.05 * RNG.standard_normal((6, 8)); x[:, 0] += 1.0
    t = RNG.standard_normal((6, 3))
    loss, g = oracle.mlp_loss_grad(p, norm, x, t)
    idx = np.concatenate([np.arange(0, 8), [512, 513], 576 + np.arange(5),
                          4672 + np.arange(3), 4736 + np.arange(3),
                          RNG.integers(0, oracle.NPARAM, 30)])
    h = 1e-6
    for k in idx:
        pp = p.copy(); pp[k] += h
        pm = p.copy(); pm[k] -= h
        fd = (oracle.mlp_loss_grad(pp, norm, x, t)[0]
              - oracle.mlp_loss_grad(pm, norm, x, t)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_loss_is_mean_squared_error():
    p = random_params()
    norm = random_norm()
    x = RNG.standard_normal((5, 8))
    t = RNG.standard_normal((5, 3))
    y = oracle.mlp_forward(p, norm, x)
    loss, _ = oracle.mlp_loss_grad(p, norm, x, t)
    assert abs(loss - np.sum((y - t) ** 2) / 5) < 1e-12


def test_adam_first_step_closed_form():
    """At t = 1, m_hat = g and v_hat = g^2, so the step is -lr g/(|g| + eps)."""
    n = 50
    p0 = RNG.standard_normal(n)
    g = RNG.standard_normal(n)
    p = p0.copy(); m = np.zeros(n); v = np.zeros(n)
    oracle.adam_step(p, m, v, g, lr=1e-3, t=1)
    assert np.allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_bias_correction():
    """With a constant gradient the bias-corrected moments stay g and g^2:
    every step moves by lr g / (|g| + eps)."""
    n = 4
    g = np.array([0.5, -2.0, 1e-3, 3.0])
    p = np.zeros(n); m = np.zeros(n); v = np.zeros(n)
    for t in range(1, 6):
        oracle.adam_step(p, m, v, g, lr=0.01, t=t)
    assert np.allclose(p, -5 * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_zero_network_is_the_plain_method():
    n = 12
    u, b = inputs.turbulence(n, 0.05)
    a = oracle.Oracle(n, n, 0.52, 0.57); a.init(u, b); a.step(8)
    c = oracle.Oracle(n, n, 0.52, 0.57); c.init(u, b)
    c.set_closure(np.zeros(oracle.NPARAM), random_norm())
    c.step(8)
    fa, ga = a.get_state(); fc, gc = c.get_state()
    assert np.array_equal(fa, fc) and np.array_equal(ga, gc)


def test_closure_shifts_a2_by_the_network_output():
    """A network with only output biases adds sigma_out * b3 to a_1^(2):
    post-collision second moments move by (1 - omega) sigma_out b3."""
    p = np.zeros(oracle.NPARAM)
    b3 = np.array([0.3, -0.2, 0.5])
    p[-3:] = b3
    norm = np.concatenate([np.zeros(8), np.ones(8), [1e-4, 2e-4, 3e-4]])
    delta = norm[-3:] * b3
    n = 4
    u, b = inputs.random_modes(n, n, 0.05, seed=3)
    a = oracle.Oracle(n, n, 0.55, 0.6); a.init(u, b)
    c = oracle.Oracle(n, n, 0.55, 0.6); c.init(u, b); c.set_closure(p, norm)
    fa, _ = a.get_state()
    om = 1 / 0.55
    CX = np.array([0, -1, -1, -1, 0, 1, 1, 1, 0])
    CY = np.array([0, 1, 0, -1, -1, -1, 0, 1, 1])
    for y in range(n):
        for x in range(n):
            f = fa[:, y, x]
            g = np.zeros(10)
            fs0, _, _ = oracle.node_collide(f, g, om, 1 / 0.6)
            # closure via a 1x1 grid with the same node
            o = oracle.Oracle(1, 1, 0.55, 0.6); o.set_closure(p, norm)
            o.set_state(f.reshape(9, 1, 1), g.reshape(5, 2, 1, 1)); o.step(1)
            fs1 = o.get_state()[0][:, 0, 0]
            d = fs1 - fs0
            assert abs(d.sum()) < 1e-15
            assert abs((d * CX * CX).sum() - (1 - om) * delta[0]) < 1e-15
            assert abs((d * CX * CY).sum() - (1 - om) * delta[1]) < 1e-15
            assert abs((d * CY * CY).sum() - (1 - om) * delta[2]) < 1e-15


def test_train_samples_closed_forms():
    """Uniform fine fields: no subgrid stress, zero gradient features.
    A fine field that is constant on each 2x2 block: filtering loses
    nothing, so tau_sgs = 0 as well; a linear shear u_x = s y gives
    a_CE_xy = -rho c_s^2 tau_c s exactly (isotropic gradient of a linear
    field is exact), up to the periodic seam rows."""
    nf, fac, tau_c = 16, 2, 0.52
    rho = np.ones((nf, nf)) * 1.01
    u = np.zeros((2, nf, nf)); u[0] = 0.03; u[1] = -0.01
    b = np.zeros((2, nf, nf)); b[0] = 0.02; b[1] = 0.04
    x, t = oracle.train_samples(rho, u, b, fac, tau_c)
    assert np.allclose(x[:, 0], 1.01) and np.allclose(x[:, 1], 0.03)
    assert np.allclose(x[:, 5:], 0, atol=1e-17) and np.allclose(t, 0, atol=1e-17)
    blk = np.kron(np.random.default_rng(1).standard_normal((nf // 2, nf // 2)),
                  np.ones((2, 2)))
    u2 = np.stack([0.01 * blk, 0.02 * blk]); b2 = np.stack([0.01 * blk, -blk * 0.01])
    _, t2 = oracle.train_samples(np.ones((nf, nf)), u2, b2, fac, tau_c)
    assert np.allclose(t2, 0, atol=1e-17)
    s = 1e-3
    yy = np.arange(nf)[:, None] * np.ones((1, nf))
    u3 = np.zeros((2, nf, nf)); u3[0] = s * yy
    x3, _ = oracle.train_samples(np.ones((nf, nf)), u3, np.zeros((2, nf, nf)), 1, tau_c)
    inner = x3.reshape(nf, nf, 8)[1:-1, :, 6]
    assert np.allclose(inner, -tau_c / 3 * s, rtol=1e-12)


def test_train_samples_subgrid_stress_of_unresolved_shear():
    """A fine field alternating +-v within each block has a zero filtered
    velocity, so tau_sgs_xx = <rho u_x^2> = v^2 and the target is
    v^2 / (tau_c - 1)."""
    nf, fac, tau_c, v = 8, 2, 0.51, 0.02
    u = np.zeros((2, nf, nf))
    u[0] = v * np.where((np.arange(nf)[None, :] % 2) == 0, 1.0, -1.0)
    x, t = oracle.train_samples(np.ones((nf, nf)), u, np.zeros((2, nf, nf)), fac, tau_c)
    assert np.allclose(x[:, 1], 0, atol=1e-18)
    assert np.allclose(t[:, 0], v * v / (tau_c - 1)) and np.allclose(t[:, 1:], 0)


# ---- one-step solver-in-the-loop objective ---------------------------------

def _fine_pair(nf, tau_f, fac, steps, seed=1):
    """Fine moments at t = steps and t + fac from the oracle's own run of a
    random-phase turbulence field."""
    u, b = inputs.turbulence(nf, 0.04, seed_psi=2 * seed + 1, seed_a=2 * seed + 2)
    o = oracle.Oracle(nf, nf, tau_f, tau_f)
    o.init(u, b)
    o.step(steps)
    m0 = o.moments()
    o.step(fac)
    m1 = o.moments()
    o.close()
    return m0, m1


@pytest.fixture(scope="module")
def fine_pair():
    fac, tf = 4, 0.8
    m0, m1 = _fine_pair(32, tf, fac, 40)
    return m0, m1, fac, 0.5 + (tf - 0.5) / fac


def test_onestep_restart_reproduces_the_filtered_fields(fine_pair):
    """The restart state's moments and a_1^(2) (computed from its
    populations) equal the filtered fields and the Chapman-Enskog estimate of
    the a-priori sample builder: f_neq,reg carries no mass or momentum and
    returns its a_1^(2) exactly (reconstruction invariants)."""
    m0, m1, fac, tc = fine_pair
    _, _, x, _ = oracle.onestep_objective(m0, m1, fac, tc)
    xs, _ = oracle.train_samples(m0[0], m0[1], m0[2], fac, tc)
    scale = np.abs(xs).max(axis=0)
    assert np.all(np.abs(x - xs).max(axis=0) <= 1e-13 * scale + 1e-300)


def test_onestep_adjoint_dot_product(fine_pair):
    """<J v, w> = <v, J^T w> for the linear part J of delta -> momentum,
    J v taken as resid(v) - resid(0) (the map is affine)."""
    m0, m1, fac, tc = fine_pair
    nc = m0[0].shape[0] // fac
    rng = np.random.default_rng(3)
    _, r0, x, _ = oracle.onestep_objective(m0, m1, fac, tc)
    for _ in range(3):
        v = 1e-4 * rng.standard_normal((nc * nc, 3))
        w = rng.standard_normal((nc * nc, 2))
        _, rv, _, _ = oracle.onestep_objective(m0, m1, fac, tc, v)
        lhs = np.sum((rv - r0) * w)
        rhs = np.sum(v * oracle.onestep_adjoint(x, nc, tc, w))
        assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_onestep_adjoint_is_a_local_push(fine_pair):
    """A unit momentum residual at one node X reaches only delta at X - c_i
    (the pull of one step), i.e. J^T is the transpose stencil."""
    m0, m1, fac, tc = fine_pair
    nc = m0[0].shape[0] // fac
    _, _, x, _ = oracle.onestep_objective(m0, m1, fac, tc)
    w = np.zeros((nc * nc, 2))
    X = (3, 5)
    w[X[1] * nc + X[0], 0] = 1.0
    g = oracle.onestep_adjoint(x, nc, tc, w).reshape(nc, nc, 3)
    nz = {(int(cx), int(cy)) for cy, cx in zip(*np.nonzero(np.abs(g).sum(axis=2)))}
    allowed = {((X[0] - dx) % nc, (X[1] - dy) % nc) for dx in (-1, 0, 1) for dy in (-1, 0, 1)
               if dx != 0}  # c_x = 0 carries no x momentum
    assert nz and nz <= allowed


def test_onestep_gradient_against_central_differences(fine_pair):
    """dL/d delta = (2 / den) J^T resid against central differences of L
    (quadratic in delta, so central differences are exact up to rounding)."""
    m0, m1, fac, tc = fine_pair
    nc = m0[0].shape[0] // fac
    rng = np.random.default_rng(4)
    v = 1e-4 * rng.standard_normal((nc * nc, 3))
    _, rv, x, den = oracle.onestep_objective(m0, m1, fac, tc, v)
    g = oracle.onestep_adjoint(x, nc, tc, rv) * (2.0 / den)
    for k, c in ((5, 0), (17, 1), (40, 2), (63, 1)):
        h = 1e-6
        vp, vm = v.copy(), v.copy()
        vp[k, c] += h
        vm[k, c] -= h
        fd = (oracle.onestep_objective(m0, m1, fac, tc, vp)[0]
              - oracle.onestep_objective(m0, m1, fac, tc, vm)[0]) / (2 * h)
        assert abs(fd - g[k, c]) <= 1e-6 * abs(g[k, c])


def test_mlp_vjp_against_central_differences():
    p = random_params()
    norm = random_norm()
    x = 0.05 * RNG.standard_normal((5, 8)); x[:, 0] += 1.0
    dy = RNG.standard_normal((5, 3))
    g = oracle.mlp_vjp(p, norm, x, dy)
    for k in (3, 600, 2000, 4700, 4930):
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (np.sum(dy * oracle.mlp_forward(pp, norm, x))
              - np.sum(dy * oracle.mlp_forward(pm, norm, x))) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k]))


def test_onestep_parameter_gradient_against_central_differences(fine_pair):
    """The composed chain (network, objective, adjoint, reverse mode) against
    central differences of L(params) evaluated through the solver step."""
    m0, m1, fac, tc = fine_pair
    p = 0.3 * np.random.default_rng(5).standard_normal(oracle.NPARAM)
    norm = np.concatenate([[1.0, 0, 0, 0, 0, 0, 0, 0], [0.01, 0.02, 0.02, 0.02, 0.02,
                                                        2e-3, 2e-3, 2e-3], [1e-4] * 3])
    L, g = oracle.onestep_loss_grad(p, norm, m0, m1, fac, tc)
    _, _, x, _ = oracle.onestep_objective(m0, m1, fac, tc)

    def L_of(q):
        d = oracle.mlp_forward(q, norm, x) * norm[16:19]
        return oracle.onestep_objective(m0, m1, fac, tc, d)[0]

    assert abs(L_of(p) - L) <= 1e-14 * L
    for k in (7, 530, 1500, 4680, 4929):
        h = 1e-5
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (L_of(pp) - L_of(pm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-5 * max(abs(g[k]), 1e-3 * np.abs(g).max())


def test_onestep_restart_of_a_resolved_shear_wave_converges():
    """Physical pin of the restart: for a viscous shear wave the one coarse
    step from the Chapman-Enskog restart reproduces the filtered fine
    momentum change over fac fine steps up to the discretisation error, which
    falls at second order in the coarse spacing (L is its square: about 16x
    per halving).  A restart without the non-equilibrium part, or with its
    sign flipped, leaves an O(1) error that does not converge."""
    fac, tf = 4, 0.8
    tc = 0.5 + (tf - 0.5) / fac
    Ls = []
    for nf in (64, 128):
        yy = np.arange(nf)
        u = np.zeros((2, nf, nf))
        u[0] = 0.01 * np.sin(2 * np.pi * yy / nf)[:, None]
        b = np.zeros((2, nf, nf))
        o = oracle.Oracle(nf, nf, tf, tf)
        o.init(u, b)
        o.step(300 * (nf // 64) ** 2)
        m0 = o.moments()
        o.step(fac)
        m1 = o.moments()
        o.close()
        Ls.append(oracle.onestep_objective(m0, m1, fac, tc)[0])
    assert Ls[1] < 5e-3
    assert Ls[0] / Ls[1] > 10.0


def test_mlp_input_gradient_against_central_differences():
    p = random_params()
    norm = random_norm()
    x = 0.05 * RNG.standard_normal((4, 8)); x[:, 0] += 1.0
    dy = RNG.standard_normal((4, 3))
    gx = oracle.mlp_vjp_input(p, norm, x, dy)
    for s in range(4):
        for k in range(8):
            h = 1e-6
            xp, xm = x.copy(), x.copy()
            xp[s, k] += h
            xm[s, k] -= h
            fd = (np.sum(dy * oracle.mlp_forward(p, norm, xp))
                  - np.sum(dy * oracle.mlp_forward(p, norm, xm))) / (2 * h)
            assert abs(fd - gx[s, k]) <= 1e-6 * max(1.0, abs(gx[s, k]))


def test_onestep_restart_carries_the_extra_non_equilibrium(fine_pair):
    """With q added to the restart's a_CE, the restart's a_1^(2) (from its
    populations) is a_CE + q, and its rho, u, b are unchanged."""
    m0, m1, fac, tc = fine_pair
    nc = m0[0].shape[0] // fac
    q = 1e-4 * np.random.default_rng(8).standard_normal((nc * nc, 3))
    _, _, x0, _ = oracle.onestep_objective(m0, m1, fac, tc)
    _, _, x1, _ = oracle.onestep_objective(m0, m1, fac, tc, q=q)
    assert np.max(np.abs(x1[:, :5] - x0[:, :5])) < 1e-15
    assert np.max(np.abs(x1[:, 5:] - x0[:, 5:] - q)) < 1e-15


def test_onestep_feedback_gradient_against_central_differences(fine_pair):
    """Feedback form of the objective (restart with the closure's steady
    response (tau_c - 1) D0, correction evaluated on that restart's
    features): the composed gradient through both network evaluations
    against central differences through the solver."""
    m0, m1, fac, tc = fine_pair
    p = 0.3 * np.random.default_rng(9).standard_normal(oracle.NPARAM)
    norm = np.concatenate([[1.0, 0, 0, 0, 0, 0, 0, 0], [0.01, 0.02, 0.02, 0.02, 0.02,
                                                        2e-3, 2e-3, 2e-3], [3e-4] * 3])
    so = norm[16:19]
    L, g = oracle.onestep_loss_grad(p, norm, m0, m1, fac, tc, feedback=True)
    _, _, x0, _ = oracle.onestep_objective(m0, m1, fac, tc)

    def L_of(w):
        q = (tc - 1.0) * oracle.mlp_forward(w, norm, x0) * so
        _, _, x1, _ = oracle.onestep_objective(m0, m1, fac, tc, q=q)
        d1 = oracle.mlp_forward(w, norm, x1) * so
        return oracle.onestep_objective(m0, m1, fac, tc, d1, q=q)[0]

    assert abs(L_of(p) - L) <= 1e-14 * L
    for k in (7, 300, 530, 1500, 4680, 4929):
        h = 1e-5
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (L_of(pp) - L_of(pm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-5 * max(abs(g[k]), 1e-3 * np.abs(g).max())


def test_onestep_feedback_with_a_silent_network_is_the_plain_objective(fine_pair):
    m0, m1, fac, tc = fine_pair
    p = 0.3 * np.random.default_rng(10).standard_normal(oracle.NPARAM)
    p[4736:] = 0.0
    norm = random_norm()
    L0 = oracle.onestep_objective(m0, m1, fac, tc)[0]
    L, g = oracle.onestep_loss_grad(p, norm, m0, m1, fac, tc, feedback=True)
    assert abs(L - L0) <= 1e-15 * L0
    assert np.all(g[:4736] == 0.0)
