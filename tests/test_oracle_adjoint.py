"""Pins of the oracle's discrete adjoint (CPU).

The adjoint is checked against its definition: transposes satisfy
<A x, y> = <x, A^T y> (the rhs is quadratic in U, so its central difference
is its exact linearisation up to rounding), and parameter gradients of the
whole objective J = sum_n dt F_x(U^n, t^n) match central finite differences
of the forward oracle.
"""
import numpy as np
import pytest

from paper_1912_05371_amd import cases, inputs


BS, NG, L = 16, 4, 4.0


def plate_grid(orc, jtop=3, clip=0, sponge=False):
    lev, ix, iy, iz = cases.plate_grid(L, 2, jtop)
    prm = cases.plate_params(jtop + 1, BS, L, clip=clip)
    prm["w"] = 0.05  # wide layer: many points carry d chi / d alpha
    if sponge:
        prm.update(sponge=1, l_sp=0.4, c_sp=5e-3, u_inf=(0.3, -0.2, 0.1), p_inf=0.05)
    g = orc.Grid(BS, NG, L, 2, jtop + 1, lev, ix, iy, iz)
    return g, prm


def test_rhs_adjoint_dot_product(orc):
    g, prm = plate_grid(orc, sponge=True)
    rng = np.random.default_rng(0)
    U = rng.standard_normal((g.nb, 4, g.P, g.P, g.P))
    D = rng.standard_normal(U.shape)
    V = rng.standard_normal(U.shape)
    eps = 1e-3
    t = 0.13
    fd = (g.rhs(prm, t, U + eps * D) - g.rhs(prm, t, U - eps * D)) / (2 * eps)
    I = slice(g.ng, g.ng + g.bs)
    lhs = np.sum(fd[..., I, I, I] * V[..., I, I, I])
    Ub = np.zeros_like(U)
    th = [0.0, 0.0, 0.0]
    g.rhs_adj(prm, t, U, V, Ub, th)
    rhs = np.sum(D * Ub)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_sync_adjoint_dot_product(orc):
    for seed in range(2):
        lev, ix, iy, iz = inputs.random_balanced_leaves(40 + seed, 1, 3, 60)
        g = orc.Grid(16, 4, 1.0, 1, 3, lev, ix, iy, iz)
        rng = np.random.default_rng(seed)
        X = rng.standard_normal((g.nb, 4, g.P, g.P, g.P))
        Y = rng.standard_normal(X.shape)
        SX = X.copy()
        g.sync(SX)
        Z = Y.copy()
        g.sync_adj(Z)
        I = slice(g.ng, g.ng + g.bs)
        lhs = np.sum(SX * Y)
        rhs = np.sum(X[..., I, I, I] * Z[..., I, I, I])
        assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(SX * Y))
        # ghosts of the adjoint are consumed
        ghost = Z.copy()
        ghost[..., I, I, I] = 0.0
        assert not ghost.any()


def test_rhs_parameter_derivatives(orc):
    g, prm = plate_grid(orc)
    rng = np.random.default_rng(1)
    U = 0.5 * rng.standard_normal((g.nb, 4, g.P, g.P, g.P))
    V = rng.standard_normal(U.shape)
    n3 = g.bs ** 3
    dus = 0.1 * rng.standard_normal((g.nb, 3, n3))
    t = 0.21
    I = slice(g.ng, g.ng + g.bs)
    th = [0.0, 0.0, 0.0]
    dusbar = np.zeros_like(dus)
    g.rhs_adj(prm, t, U, V, np.zeros_like(U), th, dusbar, dus)
    for k, name in enumerate(["amp", "freq", "phase"]):
        h = 1e-6
        pp, pm = dict(prm), dict(prm)
        pp[name] += h
        pm[name] -= h
        fd = (g.rhs(pp, t, U, dus) - g.rhs(pm, t, U, dus)) / (2 * h)
        ref = np.sum(fd[..., I, I, I] * V[..., I, I, I])
        assert abs(th[k] - ref) <= 1e-6 * abs(ref) + 1e-9, (name, th[k], ref)
    D = rng.standard_normal(dus.shape)
    e = 1e-4
    fd = (g.rhs(prm, t, U, dus + e * D) - g.rhs(prm, t, U, dus - e * D)) / (2 * e)
    ref = np.sum(fd[..., I, I, I] * V[..., I, I, I])
    assert abs(np.sum(dusbar * D) - ref) <= 1e-10 * abs(ref)


@pytest.fixture(scope="module")
def adj_case(orc):
    g, prm = plate_grid(orc)
    rng = np.random.default_rng(2)
    noise = cases.smooth_noise(7, g.bs, g.L, g.lev, g.ix, g.iy, g.iz, amp=0.2)
    U0 = inputs.pack([noise[0], noise[1], noise[2], 0 * noise[3]], g.bs, g.ng)
    dus = 0.05 * rng.standard_normal((g.nb, 3, g.bs ** 3))
    dt = 2e-4
    nsteps = 2
    J, dth, dusbar, lam0 = g.objective_grad(prm, U0, dt, nsteps, dus)
    return g, prm, U0, dus, dt, nsteps, J, dth, dusbar, lam0


def test_objective_gradient_theta_matches_fd(adj_case):
    g, prm, U0, dus, dt, nsteps, J, dth, dusbar, lam0 = adj_case
    assert abs(J) > 0
    for k, name in enumerate(["amp", "freq", "phase"]):
        h = 1e-4
        pp, pm = dict(prm), dict(prm)
        pp[name] += h
        pm[name] -= h
        Jp = g.objective(pp, U0, dt, nsteps, dus)[0]
        Jm = g.objective(pm, U0, dt, nsteps, dus)[0]
        fd = (Jp - Jm) / (2 * h)
        assert abs(dth[k] - fd) <= 1e-6 * abs(fd), (name, dth[k], fd)


def test_objective_gradient_dus_and_state_match_fd(adj_case):
    g, prm, U0, dus, dt, nsteps, J, dth, dusbar, lam0 = adj_case
    rng = np.random.default_rng(3)
    D = rng.standard_normal(dus.shape)
    h = 1e-4
    Jp = g.objective(prm, U0, dt, nsteps, dus + h * D)[0]
    Jm = g.objective(prm, U0, dt, nsteps, dus - h * D)[0]
    fd = (Jp - Jm) / (2 * h)
    assert abs(np.sum(dusbar * D) - fd) <= 1e-6 * abs(fd)
    E = np.zeros_like(U0)
    I = slice(g.ng, g.ng + g.bs)
    E[..., I, I, I] = rng.standard_normal(E[..., I, I, I].shape)
    Jp = g.objective(prm, U0 + h * E, dt, nsteps, dus)[0]
    Jm = g.objective(prm, U0 - h * E, dt, nsteps, dus)[0]
    fd = (Jp - Jm) / (2 * h)
    assert abs(np.sum(lam0[..., I, I, I] * E[..., I, I, I]) - fd) <= 1e-6 * abs(fd)
