"""Pins of the two-dimensional oracle (the model of Sec. 2.1 with D = 2) on
the CPU.

- The three-vortex initial velocity (input generator) has the paper's
  vorticity minus its mean and no divergence, both checked spectrally.
- The rhs of the three-vortex field converges with order 4 to the rhs
  evaluated spectrally on a much finer lattice (Sec. 2.3; the paper's
  equidistant runs of this case converge with slope 4.04).
- Ghost synchronisation on a uniform grid is the periodic wrap, bit for bit;
  on a two-level grid it reproduces per-axis cubics (DD4 is exact for them,
  Sec. 3.1); details vanish for cubics and equal 9 h^4 for x^4.
- On a quadtree extruded along z into an octree, with fields independent of
  z and w = 0, every 2D routine (sync, rhs, RK4 step, dt, details,
  refinement, coarsening) agrees with the 3D oracle, which is pinned by its
  own tests: a dropped term, a swapped index or a wrong weight in the 2D code
  fails here.
- RK4 amplification of the dashpot term, the time-step closed form, a
  hand-built flag table, refine-then-coarsen identity, grid validation.
"""
import math

import numpy as np
import pytest

from paper_1912_05371_amd import cases, inputs


def grid2(orc, bs, ng, L, jmin, jmax, lev, ix, iy):
    return orc.Grid2D(bs, ng, L, jmin, jmax, lev, ix, iy)


def uniform2(orc, J, bs=16, ng=4, L=2 * math.pi):
    lev, ix, iy = inputs.uniform_leaves2(J)
    return grid2(orc, bs, ng, L, J, J, lev, ix, iy)


def fill_fn(g, f):
    """Padded state (nb, 3, P, P) with f(c, x, y) at every point, ghosts too."""
    U = g.zeros()
    r = np.arange(-g.ng, g.bs + g.ng)
    for b in range(g.nb):
        h = g.L / ((1 << int(g.lev[b])) * g.bs)
        yy, xx = np.meshgrid((g.iy[b] * g.bs + r) * h, (g.ix[b] * g.bs + r) * h, indexing="ij")
        for c in range(3):
            U[b, c] = f(c, xx, yy)
    return U


# ---------------------------------------------------------------- input
def test_three_vortex_velocity_has_the_paper_vorticity():
    N, L = 256, 2 * math.pi
    u, v = inputs.three_vortex_velocity(N, L)
    w = inputs.three_vortex_vorticity(N, L)
    k = np.fft.fftfreq(N, d=L / N) * 2 * math.pi
    KX, KY = k[None, :], k[:, None]
    curl = np.real(np.fft.ifft2(1j * KX * np.fft.fft2(v) - 1j * KY * np.fft.fft2(u)))
    div = np.real(np.fft.ifft2(1j * KX * np.fft.fft2(u) + 1j * KY * np.fft.fft2(v)))
    assert np.max(np.abs(curl - (w - w.mean()))) < 1e-10 * np.max(np.abs(w))
    assert np.max(np.abs(div)) < 1e-12
    # circulation 1.5 in total, so the mean vorticity is small but not zero
    assert w.mean() * L * L == pytest.approx(1.5, rel=1e-6)
    # the strongest vortex core: peak vorticity Gamma / (pi a^2) = pi
    assert np.max(w) == pytest.approx(math.pi, rel=0.05)


# ---------------------------------------------------------------- rhs order
def _spectral_rhs(u, v, L, prm):
    N = u.shape[0]
    k = np.fft.fftfreq(N, d=L / N) * 2 * math.pi
    KX, KY = k[None, :], k[:, None]

    def dx(f):
        return np.real(np.fft.ifft2(1j * KX * np.fft.fft2(f)))

    def dy(f):
        return np.real(np.fft.ifft2(1j * KY * np.fft.fft2(f)))

    def lap(f):
        return np.real(np.fft.ifft2(-(KX ** 2 + KY ** 2) * np.fft.fft2(f)))

    ru = -(u * dx(u) + v * dy(u)) + prm["nu"] * lap(u)
    rv = -(u * dx(v) + v * dy(v)) + prm["nu"] * lap(v)
    rp = -prm["c0"] ** 2 * (dx(u) + dy(v))
    return ru, rv, rp


def test_rhs_fourth_order_against_spectral(orc):
    # the three vortices at (2^J 16)^2 points, J = 4, 5, 6, p = 0; the
    # reference is the same continuous rhs evaluated spectrally at 2048^2.
    # Scales: the largest velocity rhs for u and v, C0^2 max|du/dx| for p
    # (the field is divergence-free, so the exact dp/dt vanishes)
    prm = cases.params(nu=5e-3, c0=10.0, c_gamma=1.0)
    L = 2 * math.pi
    Nref = 2048
    u, v = inputs.three_vortex_velocity(Nref, L)
    ref = _spectral_rhs(u, v, L, prm)
    k = np.fft.fftfreq(Nref, d=L / Nref) * 2 * math.pi
    ux = np.real(np.fft.ifft2(1j * k[None, :] * np.fft.fft2(u)))
    scale = [max(np.max(np.abs(ref[0])), np.max(np.abs(ref[1])))] * 2 + \
        [prm["c0"] ** 2 * np.max(np.abs(ux))]
    errs = []
    for J in (4, 5, 6):
        g = uniform2(orc, J)
        fl = [inputs.sample2(u, 16, g.lev, g.ix, g.iy), inputs.sample2(v, 16, g.lev, g.ix, g.iy),
              np.zeros((g.nb, 16, 16))]
        U = inputs.pack2(fl, 16, 4)
        g.sync(U)
        R = inputs.interior2(g.rhs(prm, U), 16, 4)
        e = 0.0
        for c in range(3):
            rs = inputs.sample2(ref[c], 16, g.lev, g.ix, g.iy)
            e = max(e, np.max(np.abs(R[:, c] - rs)) / scale[c])
        errs.append(e)
    s1, s2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert 3.7 < s1 < 4.4 and 3.8 < s2 < 4.3, (errs, s1, s2)


# ---------------------------------------------------------------- sync
def test_sync_uniform_is_periodic_wrap(orc):
    g = uniform2(orc, 2)
    n = 4 * g.bs
    rng = np.random.default_rng(1)
    glob = rng.standard_normal((3, n, n))
    U = g.zeros()
    r = np.arange(-g.ng, g.bs + g.ng)
    exp = []
    for b in range(g.nb):
        yy, xx = np.meshgrid((g.iy[b] * g.bs + r) % n, (g.ix[b] * g.bs + r) % n, indexing="ij")
        full = glob[:, yy, xx]
        exp.append(full)
        U[b][:, g.ng:-g.ng, g.ng:-g.ng] = full[:, g.ng:-g.ng, g.ng:-g.ng]
    g.sync(U)
    for b in range(g.nb):
        assert np.array_equal(U[b], exp[b])


def _two_level2(orc, bs=16, ng=4):
    lev, ix, iy = inputs.uniform_leaves2(2)
    ls = inputs.LeafSet2(zip(lev, ix, iy), 2)
    ls.refine((2, 1, 1))
    ls.refine((2, 2, 1))
    l, x, y = ls.arrays()
    return grid2(orc, bs, ng, 1.0, 2, 3, l, x, y)


def test_sync_two_level_reproduces_cubics(orc):
    g = _two_level2(orc)
    assert set(np.unique(g.lev)) == {2, 3}

    def f(c, x, y):
        return (c + 1) * (1.0 + x - 2 * y ** 3 + x ** 2 * y ** 3 - 0.5 * x ** 3 * y + y ** 2)

    E = fill_fn(g, f)
    U = E.copy()
    ng = g.ng
    U[..., :ng, :] = U[..., -ng:, :] = U[..., :, :ng] = U[..., :, -ng:] = np.nan
    g.sync(U)
    checked = 0
    for b in range(g.nb):
        lo = np.array([g.ix[b], g.iy[b]]) / (1 << int(g.lev[b]))
        if np.any(lo < 0.2) or np.any(lo > 0.6):
            continue  # ghosts that wrap around the periodic domain
        assert np.max(np.abs(U[b] - E[b])) < 1e-13
        checked += 1
    assert checked >= 6


def test_details_cubic_zero_quartic_9h4(orc):
    g = _two_level2(orc)
    U = fill_fn(g, lambda c, x, y: (1 + x * y + x ** 3 * y ** 2 - y ** 3) * (c + 1))
    assert np.max(g.details(U)) < 1e-12
    U = fill_fn(g, lambda c, x, y: x ** 4 if c == 0 else 0.0 * x)
    N = np.max(np.abs(inputs.interior2(U, 16, 4)[:, 0]))
    h = 1.0 / ((1 << g.lev.astype(np.int64)) * 16)
    assert np.allclose(g.details(U), 9 * h ** 4 / N, rtol=1e-6, atol=0)


# ---------------------------------------------------------------- against 3D
def _extrude(lev, ix, iy):
    """Each quadtree leaf (J, x, y) becomes the 2^J octree leaves (J, x, y, z)."""
    L3 = [(int(J), int(x), int(y), z) for J, x, y in zip(lev, ix, iy) for z in range(1 << int(J))]
    return inputs._sorted(L3)


def _lift3(g2, U2, g3):
    """3D state of z-independent fields: (u, v, 0, p) from the 2D (u, v, p)."""
    pos = {(int(J), int(x), int(y)): b for b, (J, x, y) in enumerate(zip(g2.lev, g2.ix, g2.iy))}
    P = g3.P
    U3 = np.zeros((g3.nb, 4, P, P, P))
    for b3 in range(g3.nb):
        b2 = pos[(int(g3.lev[b3]), int(g3.ix[b3]), int(g3.iy[b3]))]
        for c2, c3 in ((0, 0), (1, 1), (2, 3)):
            U3[b3, c3] = U2[b2, c2][None, :, :]
    return U3, pos


@pytest.fixture(scope="module")
def extruded(orc):
    lev, ix, iy = inputs.random_balanced_leaves2(1, 2, 4, 30)
    assert len(set(lev.tolist())) == 3
    g2 = grid2(orc, 16, 4, 1.0, 2, 5, lev, ix, iy)
    l3, x3, y3, z3 = _extrude(g2.lev, g2.ix, g2.iy)
    g3 = orc.Grid(16, 4, 1.0, 2, 5, l3, x3, y3, z3)
    rng = np.random.default_rng(8)
    # a smooth periodic field plus noise, so every stencil tap matters
    U2 = fill_fn(g2, lambda c, x, y: np.sin(2 * math.pi * (x + c * y)) + 0.3 * np.cos(
        4 * math.pi * y + c))
    U2[:, :, 4:-4, 4:-4] += 1e-2 * rng.standard_normal((g2.nb, 3, 16, 16))
    return g2, g3, U2


def _compare(g2, g3, U2, U3, pos, interior_only, tol):
    scale = max(np.max(np.abs(U2)), 1e-300)
    err = 0.0
    for b3 in range(g3.nb):
        b2 = pos[(int(g3.lev[b3]), int(g3.ix[b3]), int(g3.iy[b3]))]
        for c2, c3 in ((0, 0), (1, 1), (2, 3)):
            a = U3[b3, c3]
            if interior_only:
                a = a[4:-4, 4:-4, 4:-4]
                ref = U2[b2, c2][None, 4:-4, 4:-4]
            else:
                ref = U2[b2, c2][None]
            err = max(err, np.max(np.abs(a - ref)))
    assert err <= tol * scale, err / scale


def test_2d_sync_equals_3d_extruded(orc, extruded):
    g2, g3, U2 = extruded
    A = U2.copy()
    g2.sync(A)
    U3, pos = _lift3(g2, U2, g3)
    g3.sync(U3)
    _compare(g2, g3, A, U3, pos, False, 16 * np.finfo(float).eps)
    assert np.max(np.abs(U3[:, 2])) == 0.0


def test_2d_rhs_rk4_dt_equal_3d_extruded(orc, extruded):
    g2, g3, U2 = extruded
    prm = cases.params(nu=2e-3, c0=3.0, c_gamma=0.7, cfl=0.5)
    A = U2.copy()
    g2.sync(A)
    U3, pos = _lift3(g2, A, g3)
    g3.sync(U3)
    R2 = g2.rhs(prm, A)
    R3 = g3.rhs(prm, 0.0, U3)
    _compare(g2, g3, R2, R3, pos, True, 1e-13)
    assert g2.dt(prm, A) == pytest.approx(g3.dt(prm, U3), rel=1e-15)
    dt = 0.5 * g2.dt(prm, A)
    B = U2.copy()
    g2.rk4_step(prm, dt, B)
    U3, _ = _lift3(g2, U2, g3)
    g3.rk4_step(prm, 0.0, dt, U3)
    _compare(g2, g3, B, U3, pos, True, 1e-13)


def test_2d_details_and_adaptation_equal_3d_extruded(orc, extruded):
    g2, g3, U2 = extruded
    A = U2.copy()
    g2.sync(A)
    U3, pos = _lift3(g2, A, g3)
    g3.sync(U3)
    d2 = g2.details(A)
    d3, _ = g3.details(None, 0.0, U3)
    for b3 in range(g3.nb):
        b2 = pos[(int(g3.lev[b3]), int(g3.ix[b3]), int(g3.iy[b3]))]
        assert d3[b3] == pytest.approx(d2[b2], rel=1e-12, abs=1e-15)
    # refine all: the children of the 2D refinement are the extruded 3D ones
    h2, R2 = g2.refine_all(A)
    h3, R3 = g3.refine_all(U3)
    l3, x3, y3, z3 = _extrude(h2.lev, h2.ix, h2.iy)
    assert sorted(zip(h3.lev, h3.ix, h3.iy, h3.iz)) == sorted(zip(l3, x3, y3, z3))
    pos2 = {(int(J), int(x), int(y)): b for b, (J, x, y) in enumerate(zip(h2.lev, h2.ix, h2.iy))}
    _compare(h2, h3, R2, R3, pos2, True, 16 * np.finfo(float).eps)
    # coarsen every family back
    h2.sync(R2)
    h3.sync(R3)
    f2 = np.ones(h2.nb, np.int8)
    f3 = np.ones(h3.nb, np.int8)
    c2, C2 = h2.coarsen(f2, R2)
    c3, C3 = h3.coarsen(f3, R3)
    l3, x3, y3, z3 = _extrude(c2.lev, c2.ix, c2.iy)
    assert sorted(zip(c3.lev, c3.ix, c3.iy, c3.iz)) == sorted(zip(l3, x3, y3, z3))
    posc = {(int(J), int(x), int(y)): b for b, (J, x, y) in enumerate(zip(c2.lev, c2.ix, c2.iy))}
    _compare(c2, c3, C2, C3, posc, True, 16 * np.finfo(float).eps)


# ---------------------------------------------------------------- RK4, dt
def test_rk4_dashpot_amplification(orc):
    g = uniform2(orc, 1, L=1.0)
    U = fill_fn(g, lambda c, x, y: (0.3, -0.7, 2.0)[c] + 0.0 * x)
    cg, dt = 3.0, 0.02
    prm = cases.params(nu=0.0, c0=5.0, c_gamma=cg)
    g.rk4_step(prm, dt, U)
    R = lambda z: 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    I = inputs.interior2(U, 16, 4)
    assert np.all(I[:, 0] == 0.3) and np.all(I[:, 1] == -0.7)
    assert np.max(np.abs(I[:, 2] - 2.0 * R(-cg * dt))) < 1e-15


def test_dt_closed_form(orc):
    g = uniform2(orc, 2)
    U = fill_fn(g, lambda c, x, y: (0.6, 0.8, 0.0)[c] + 0.0 * x)  # |u| = 1
    h = 2 * math.pi / 64
    prm = cases.params(nu=1e-3, c0=10.0, cfl=0.5)
    assert g.dt(prm, U) == pytest.approx(0.5 * h / (1 + math.sqrt(101)), rel=1e-15)
    prm = cases.params(nu=10.0, c0=10.0, cfl=0.5)
    assert g.dt(prm, U) == pytest.approx(0.25 * h * h / 10.0, rel=1e-15)


# ---------------------------------------------------------------- flags, adaptation
def test_flags_table(orc):
    lev, ix, iy = inputs.random_balanced_leaves2(2, 2, 4, 80)
    assert set(np.unique(lev)) == {2, 3, 4}
    g = grid2(orc, 16, 4, 1.0, 2, 4, lev, ix, iy)
    table = {2: [(0.0, 0)], 3: [(5e-4, 1), (1e-3, 0), (2e-3, 0)], 4: [(5e-4, 1), (0.5, 0)]}
    for dealias in (False, True):
        dm = np.zeros(g.nb)
        exp = np.zeros(g.nb, np.int8)
        for b in range(g.nb):
            rows = table[int(g.lev[b])]
            dm[b], exp[b] = rows[b % len(rows)]
            if dealias and g.lev[b] == 4:
                exp[b] = 1
        assert np.array_equal(g.flags(dm, 1e-3, dealias), exp)


def test_refine_then_coarsen_is_identity(orc):
    # R after P is the identity (Sec. 3.1).  Merging is Jacobi over the
    # current leaves and respects grading, so the finest families merge first:
    # repeat, flagging every block that is not an original leaf.
    lev, ix, iy = inputs.random_balanced_leaves2(6, 1, 3, 25)
    g = grid2(orc, 16, 4, 1.0, 1, 4, lev, ix, iy)
    rng = np.random.default_rng(4)
    U = g.zeros()
    U[:, :, 4:-4, 4:-4] = rng.standard_normal((g.nb, 3, 16, 16))
    g.sync(U)
    h, V = g.refine_all(U)
    assert h.nb == 4 * g.nb
    orig = {(int(J), int(x), int(y)): b for b, (J, x, y) in enumerate(zip(g.lev, g.ix, g.iy))}
    for _ in range(4):
        fl = np.array([0 if (int(J), int(x), int(y)) in orig else 1
                       for J, x, y in zip(h.lev, h.ix, h.iy)], np.int8)
        if not fl.any():
            break
        h.sync(V)
        h, V = h.coarsen(fl, V)
    assert h.nb == g.nb
    for b in range(h.nb):
        q = orig[(int(h.lev[b]), int(h.ix[b]), int(h.iy[b]))]
        assert np.array_equal(V[b][:, 4:-4, 4:-4], U[q][:, 4:-4, 4:-4])


def test_grid_validation(orc):
    lev, ix, iy = inputs.uniform_leaves2(1)
    with pytest.raises(orc.OracleError) as e:
        grid2(orc, 16, 4, 1.0, 1, 2, lev[:-1], ix[:-1], iy[:-1])  # gap
    assert e.value.code == -2
    with pytest.raises(orc.OracleError) as e:
        grid2(orc, 16, 4, 1.0, 1, 2, np.r_[lev, 1], np.r_[ix, 0], np.r_[iy, 0])  # repeat
    assert e.value.code == -2
    ls = inputs.LeafSet2(zip(lev, ix, iy), 1)
    ls.s.discard((1, 0, 0))
    ls.s.update({(2, 0, 0), (2, 1, 0), (2, 0, 1)})
    ls.s.update({(3, 2, 2), (3, 3, 2), (3, 2, 3), (3, 3, 3)})  # level 3 next to level 1
    l, x, y = ls.arrays()
    with pytest.raises(orc.OracleError) as e:
        grid2(orc, 16, 4, 1.0, 1, 3, l, x, y)
    assert e.value.code == -3
    with pytest.raises(orc.OracleError) as e:
        grid2(orc, 12, 4, 1.0, 1, 2, lev, ix, iy)  # bs < 2 (ng + 3)
    assert e.value.code == -1
