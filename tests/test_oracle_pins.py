"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Every test here runs on the CPU.  None of them re-types the oracle's formula:
each compares it with a closed form, an invariant, a value printed in the
paper (or in the work it cites, tests/golden/constants.json), or a brute-force
evaluation written independently below.  A plausible slip in the oracle (a
wrong sign, a dropped term, a transposed index, a wrong weight) fails at
least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from paper_1912_05371_amd import cases, inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "constants.json")))


def grid_of(orc, c):
    return orc.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, c.lev, c.ix, c.iy, c.iz)


def uniform_case(J, bs=16, ng=4, L=2 * math.pi):
    lev, ix, iy, iz = inputs.uniform_leaves(J)
    return cases.Case("u", bs, ng, L, J, J, lev, ix, iy, iz, cases.params())


# ---------------------------------------------------------------- Tam-Webb
def test_tam_webb_matches_published_and_constraints(orc):
    a = orc.tam_webb()
    ref = np.array(GOLD["tam_webb_a"]["value"])
    assert np.max(np.abs(a - ref)) < 1e-12
    m = np.arange(1, 4)
    assert abs(2 * np.sum(m * a) - 1.0) < 1e-15          # consistency
    assert abs(np.sum(m ** 3 * a)) < 1e-15                # 4th order


def test_tam_webb_is_least_squares_optimum(orc):
    a = orc.tam_webb()
    # 40-digit quadrature of the optimum: the oracle must agree to 1 ulp
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    f0 = lambda e: mpmath.mpf(4) / 3 * mpmath.sin(e) - mpmath.sin(2 * e) / 6 - e
    f1 = lambda e: 10 * mpmath.sin(e) - 8 * mpmath.sin(2 * e) + 2 * mpmath.sin(3 * e)
    X = mpmath.mpf("1.1")
    t = -mpmath.quad(lambda e: f0(e) * f1(e), [0, X]) / mpmath.quad(lambda e: f1(e) ** 2, [0, X])
    exact = [mpmath.mpf(2) / 3 + 5 * t, -mpmath.mpf(1) / 12 - 4 * t, t]
    for v, e in zip(a, exact):
        assert abs(v - float(e)) <= np.spacing(abs(float(e)))

    def obj(t):
        b = np.array([2 / 3 + 5 * t, -1 / 12 - 4 * t, t])
        f = lambda e: (2 * np.sum(b * np.sin(np.arange(1, 4) * e)) - e) ** 2
        return integrate.quad(f, 0.0, 1.1, epsabs=1e-15, epsrel=1e-13)[0]

    t = a[2]
    d = 1e-5
    # derivative of the quadratic objective vanishes at the oracle's t
    g = (obj(t + d) - obj(t - d)) / (2 * d)
    curv = (obj(t + d) - 2 * obj(t) + obj(t - d)) / d ** 2
    assert abs(g / curv) < 1e-8


# ---------------------------------------------------------------- treecode
def test_treecode_digits(orc):
    # level 2, block (3,0,1): level-1 digit = xbit1 + 2 ybit1 + 4 zbit1 = 1,
    # level-2 digit = 1 + 4 = 5  -> octal 15 = 13
    assert orc.treecode_encode(2, 3, 0, 1) == 0o15
    rng = np.random.default_rng(0)
    for _ in range(200):
        J = int(rng.integers(0, 19))
        x, y, z = (int(v) for v in rng.integers(0, 1 << J, 3)) if J else (0, 0, 0)
        assert orc.treecode_decode(orc.treecode_encode(J, x, y, z), J) == (x, y, z)


# ---------------------------------------------------------------- grid
def test_grid_validation_errors(orc):
    lev, ix, iy, iz = inputs.uniform_leaves(1)
    g = orc.Grid(16, 4, 1.0, 1, 3, lev, ix, iy, iz)
    assert g.nb == 8 and g.is_balanced()
    with pytest.raises(orc.OracleError) as e:   # missing a leaf: not a tiling
        orc.Grid(16, 4, 1.0, 1, 3, lev[:-1], ix[:-1], iy[:-1], iz[:-1])
    assert e.value.code == -2
    with pytest.raises(orc.OracleError) as e:   # duplicate leaf
        orc.Grid(16, 4, 1.0, 1, 3, np.r_[lev, 1], np.r_[ix, 0], np.r_[iy, 0], np.r_[iz, 0])
    assert e.value.code == -2
    with pytest.raises(orc.OracleError) as e:   # odd block size
        orc.Grid(15, 4, 1.0, 1, 3, lev, ix, iy, iz)
    assert e.value.code == -1
    with pytest.raises(orc.OracleError) as e:   # too small for the stencils
        orc.Grid(12, 4, 1.0, 1, 3, lev, ix, iy, iz)
    assert e.value.code == -1
    # level-1 block next to level-3 blocks: not 2:1 graded
    ls = inputs.LeafSet(zip(lev, ix, iy, iz), 1)
    ls.s.discard((1, 0, 0, 0))
    for c in range(8):
        ls.s.add((2, c & 1, c >> 1 & 1, c >> 2 & 1))
    ls.s.discard((2, 1, 1, 1))
    for c in range(8):
        ls.s.add((3, 2 + (c & 1), 2 + (c >> 1 & 1), 2 + (c >> 2 & 1)))
    l2, x2, y2, z2 = ls.arrays()
    with pytest.raises(orc.OracleError) as e:
        orc.Grid(16, 4, 1.0, 1, 3, l2, x2, y2, z2)
    assert e.value.code == -3


def test_random_tree_is_balanced_and_tiles(orc):
    lev, ix, iy, iz = inputs.random_balanced_leaves(7, 1, 4, 300)
    g = orc.Grid(16, 4, 1.0, 1, 4, lev, ix, iy, iz)
    assert g.is_balanced()
    assert np.sum(8.0 ** (-lev.astype(float))) == pytest.approx(1.0, abs=1e-15)


# ---------------------------------------------------------------- sync
def test_sync_uniform_equals_periodic_wrap(orc):
    c = cases.taylor_green()
    g = grid_of(orc, c)
    rng = np.random.default_rng(1)
    n = 4 * c.bs
    glob = rng.standard_normal((4, n, n, n))
    U = np.zeros((g.nb, 4, c.P, c.P, c.P))
    for b in range(g.nb):
        ox, oy, oz = g.ix[b] * c.bs, g.iy[b] * c.bs, g.iz[b] * c.bs
        r = np.arange(-c.ng, c.bs + c.ng)
        zz, yy, xx = np.meshgrid((oz + r) % n, (oy + r) % n, (ox + r) % n, indexing="ij")
        full = glob[:, zz, yy, xx]
        U[b, :, c.ng:-c.ng, c.ng:-c.ng, c.ng:-c.ng] = full[:, c.ng:-c.ng, c.ng:-c.ng,
                                                           c.ng:-c.ng]
        if b == 0:
            expect0 = full.copy()
    g.sync(U)
    assert np.array_equal(U[0], expect0)
    for b in range(g.nb):
        ox, oy, oz = g.ix[b] * c.bs, g.iy[b] * c.bs, g.iz[b] * c.bs
        r = np.arange(-c.ng, c.bs + c.ng)
        zz, yy, xx = np.meshgrid((oz + r) % n, (oy + r) % n, (ox + r) % n, indexing="ij")
        assert np.array_equal(U[b], glob[:, zz, yy, xx])


def _two_level_grid(orc, bs=16, ng=4):
    # level 2 with one level-2 block refined -> level 3 (away from the wrap)
    lev, ix, iy, iz = inputs.uniform_leaves(2)
    ls = inputs.LeafSet(zip(lev, ix, iy, iz), 2)
    ls.refine((2, 1, 1, 1))
    ls.refine((2, 2, 1, 1))
    l, x, y, z = ls.arrays()
    return orc.Grid(bs, ng, 1.0, 2, 3, l, x, y, z)


def test_sync_two_level_reproduces_cubic(orc):
    g = _two_level_grid(orc)
    bs, ng, P = g.bs, g.ng, g.P

    def f(x, y, z):  # degree <= 3 in each variable
        return 1.0 + x - 2 * y ** 3 + x ** 2 * y * z ** 3 - 0.5 * x ** 3 * y ** 2 + z ** 2

    U = np.zeros((g.nb, 4, P, P, P))
    pos = {}
    for b in range(g.nb):
        h = 1.0 / ((1 << g.lev[b]) * bs)
        r = np.arange(-ng, bs + ng)
        zz, yy, xx = np.meshgrid((g.iz[b] * bs + r) * h, (g.iy[b] * bs + r) * h,
                                 (g.ix[b] * bs + r) * h, indexing="ij")
        pos[b] = (xx, yy, zz)
        for c in range(4):
            U[b, c, ng:-ng, ng:-ng, ng:-ng] = (c + 1) * f(xx, yy, zz)[ng:-ng, ng:-ng, ng:-ng]
    g.sync(U)
    checked = 0
    for b in range(g.nb):
        xx, yy, zz = pos[b]
        # only blocks whose ghost sources never wrap: the fine blocks and the
        # coarse blocks around them lie well inside [0.125, 0.875]
        lo = np.array([g.ix[b], g.iy[b], g.iz[b]]) / (1 << g.lev[b])
        if np.any(lo < 0.2) or np.any(lo > 0.6):
            continue
        for c in range(4):
            assert np.max(np.abs(U[b, c] - (c + 1) * f(xx, yy, zz))) < 1e-13
        checked += 1
    assert checked >= 8


def _bruteforce_ghost(leaves, bs, J, G, vals):
    """Independent ghost evaluation: scan all leaves for the owner of a point
    given on the level-J lattice; DD4 weights from the golden constants."""
    w = GOLD["dd4_weights"]["value"]
    offs = GOLD["dd4_weights"]["offsets_fine"]
    top = max(l[0] for l in leaves)

    def owner_value(K, p):  # point p on the level-K lattice
        n = (1 << K) * bs
        p = [q % n for q in p]
        for (lv, x, y, z), blk in zip(leaves, range(len(leaves))):
            s = (bs << top) >> lv  # box size in level-`top` units
            pr = [(q * (1 << top)) // (1 << K) if K <= top else None for q in p]
            o = (x * s, y * s, z * s)
            if all(o[d] <= pr[d] < o[d] + s for d in range(3)):
                # local index at level lv
                num = [pr[d] - o[d] for d in range(3)]
                unit = 1 << (top - lv)
                if any(v % unit for v in num):
                    return None, lv
                loc = [v // unit for v in num]
                return vals(blk, loc), lv
        raise AssertionError("no owner")

    v, lv = owner_value(J, G)
    if v is not None:
        return v
    assert lv == J - 1
    axes = []
    for d in range(3):
        if G[d] % 2 == 0:
            axes.append([(G[d] // 2, 1.0)])
        else:
            axes.append([((G[d] + o) // 2, wt) for o, wt in zip(offs, w)])
    tot = 0.0
    for cz, wz in axes[2]:
        for cy, wy in axes[1]:
            for cx, wx in axes[0]:
                sv, slv = owner_value(J - 1, (cx, cy, cz))
                assert sv is not None
                tot += wz * wy * wx * sv
    return tot


def test_sync_bruteforce_tiny_random_grids(orc):
    rng = np.random.default_rng(3)
    for trial in range(2):
        lev, ix, iy, iz = inputs.random_balanced_leaves(100 + trial, 1, 3, 40)
        bs, ng = 14, 4
        g = orc.Grid(bs, ng, 1.0, 1, 3, lev, ix, iy, iz)
        P = g.P
        U = rng.standard_normal((g.nb, 4, P, P, P))
        V = U.copy()
        g.sync(V)
        leaves = list(zip(g.lev.tolist(), g.ix.tolist(), g.iy.tolist(), g.iz.tolist()))

        def vals(blk, loc, c=0):
            return U[blk, c, loc[2] + ng, loc[1] + ng, loc[0] + ng]

        # sample ghost points of blocks that have a coarser neighbour
        pts = 0
        for b in rng.permutation(g.nb)[:12]:
            J = int(g.lev[b])
            for _ in range(25):
                while True:
                    i, j, k = (int(v) for v in rng.integers(-ng, bs + ng, 3))
                    if not (0 <= i < bs and 0 <= j < bs and 0 <= k < bs):
                        break
                G = (int(g.ix[b]) * bs + i, int(g.iy[b]) * bs + j, int(g.iz[b]) * bs + k)
                ref = _bruteforce_ghost(leaves, bs, J, G, vals)
                assert V[b, 0, k + ng, j + ng, i + ng] == pytest.approx(ref, abs=1e-13)
                pts += 1
        assert pts == 300


# ---------------------------------------------------------------- rhs
def _modified_wavenumbers(orc, k, h):
    a = orc.tam_webb()
    kb = 2 * np.sum(a * np.sin(np.arange(1, 4) * k * h)) / h
    k2 = (8.0 / 3.0 * math.cos(k * h) - math.cos(2 * k * h) / 6.0 - 2.5) / h ** 2  # D2 e^{ikx}/e^{ikx}
    return kb, k2


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_rhs_pressure_gradient_modified_wavenumber(orc, axis):
    c = uniform_case(2)
    g = grid_of(orc, c)
    x, y, z = c.coords()
    q = (x, y, z)[axis]
    k = 3
    zero = np.zeros_like(x)
    U = inputs.pack([zero, zero, zero, np.sin(k * q)], c.bs, c.ng)
    g.sync(U)
    prm = cases.params(nu=0.0, c0=7.0, c_gamma=0.3)
    R = inputs.interior(g.rhs(prm, 0.0, U), c.bs, c.ng)
    h = c.L / (4 * c.bs)
    kb, _ = _modified_wavenumbers(orc, k, h)
    for d in range(3):
        exp = -kb * np.cos(k * q) if d == axis else 0.0
        assert np.max(np.abs(R[:, d] - exp)) < 1e-12
    assert np.max(np.abs(R[:, 3] + 0.3 * np.sin(k * q))) < 1e-13


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_rhs_viscous_and_divergence(orc, axis):
    # u_c = sin(k x_axis) with c != axis: no convection, pure diffusion along axis
    c = uniform_case(2)
    g = grid_of(orc, c)
    x, y, z = c.coords()
    q = (x, y, z)[axis]
    comp = (axis + 1) % 3
    k = 2
    f = [np.zeros_like(x) for _ in range(4)]
    f[comp] = np.sin(k * q)
    U = inputs.pack(f, c.bs, c.ng)
    g.sync(U)
    nu = 0.37
    prm = cases.params(nu=nu, c0=5.0, c_gamma=0.0)
    R = inputs.interior(g.rhs(prm, 0.0, U), c.bs, c.ng)
    h = c.L / (4 * c.bs)
    _, k2 = _modified_wavenumbers(orc, k, h)
    assert np.max(np.abs(R[:, comp] - nu * k2 * np.sin(k * q))) < 1e-12
    assert np.max(np.abs(R[:, 3])) < 1e-12  # divergence free
    # now u_axis = sin(k x_axis): divergence = kb cos(k q)
    f = [np.zeros_like(x) for _ in range(4)]
    f[axis] = np.sin(k * q)
    U = inputs.pack(f, c.bs, c.ng)
    g.sync(U)
    R = inputs.interior(g.rhs(cases.params(nu=0.0, c0=5.0, c_gamma=0.0), 0.0, U), c.bs, c.ng)
    kb, _ = _modified_wavenumbers(orc, k, h)
    assert np.max(np.abs(R[:, 3] + 25.0 * kb * np.cos(k * q))) < 1e-11
    # advective term u d/dx u = sin(kq) kb cos(kq)
    assert np.max(np.abs(R[:, axis] + np.sin(k * q) * kb * np.cos(k * q))) < 1e-12


def test_rhs_taylor_green_closed_form(orc):
    c = cases.taylor_green()
    g = grid_of(orc, c)
    U = c.padded()
    g.sync(U)
    R = inputs.interior(g.rhs(c.params, 0.0, U), c.bs, c.ng)
    x, y, z = c.coords()
    h = c.L / 64
    kb, k2 = _modified_wavenumbers(orc, 1, h)
    nu = c.params["nu"]
    u, v = np.sin(x) * np.cos(y) * np.cos(z), -np.cos(x) * np.sin(y) * np.cos(z)
    du = -kb * np.sin(x) * np.cos(x) * np.cos(z) ** 2 + 3 * nu * k2 * u
    dv = -kb * np.sin(y) * np.cos(y) * np.cos(z) ** 2 + 3 * nu * k2 * v
    assert np.max(np.abs(R[:, 0] - du)) < 1e-13
    assert np.max(np.abs(R[:, 1] - dv)) < 1e-13
    assert np.max(np.abs(R[:, 2])) < 1e-13
    assert np.max(np.abs(R[:, 3])) < 1e-11   # C0^2 (kb - kb) cos cos cos = 0


def test_rhs_fourth_order_convergence(orc):
    errs = []
    for J in (1, 2, 3):
        c = uniform_case(J, bs=16)
        g = grid_of(orc, c)
        x, y, z = c.coords()
        u, v = np.sin(x) * np.cos(y) * np.cos(z), -np.cos(x) * np.sin(y) * np.cos(z)
        U = inputs.pack([u, v, np.zeros_like(u), np.cos(x + 2 * y)], c.bs, c.ng)
        g.sync(U)
        nu = 0.05
        R = inputs.interior(g.rhs(cases.params(nu=nu, c0=1.0, c_gamma=0.0), 0.0, U), c.bs, c.ng)
        exact_u = -np.sin(x) * np.cos(x) * np.cos(z) ** 2 + np.sin(x + 2 * y) - 3 * nu * u
        errs.append(np.max(np.abs(R[:, 0] - exact_u)))
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 3.7 < slopes[1] < 4.3, (errs, slopes)


def test_pressure_sum_follows_dashpot(orc):
    c = uniform_case(2)
    g = grid_of(orc, c)
    fl = inputs.fourier_fields(5, c.bs, c.L, c.lev, c.ix, c.iy, c.iz, nmodes=6, kmax=3)
    U = inputs.pack(fl, c.bs, c.ng)
    g.sync(U)
    cg = 0.7
    R = inputs.interior(g.rhs(cases.params(nu=0.01, c0=9.0, c_gamma=cg), 0.0, U), c.bs, c.ng)
    P = inputs.interior(U, c.bs, c.ng)[:, 3]
    assert abs(np.sum(R[:, 3]) + cg * np.sum(P)) < 1e-10 * np.sum(np.abs(R[:, 3]))


# ---------------------------------------------------------------- RK4, dt
def _full_solid_params(**kw):
    # a sphere of radius 100 covers the whole domain: chi == 1 exactly
    return cases.params(mask=1, sph_c=(0.5, 0.5, 0.5), sph_r=100.0, w=0.01, **kw)


def test_rk4_amplification_factor(orc):
    c = uniform_case(1, L=1.0)
    g = grid_of(orc, c)
    one = np.ones((g.nb, c.bs, c.bs, c.bs))
    U = inputs.pack([0.3 * one, -1.2 * one, 2.0 * one, 5.0 * one], c.bs, c.ng)
    ce, cg, dt = 0.02, 3.0, 0.013
    prm = _full_solid_params(c_eta=ce, c_gamma=cg, nu=0.1, c0=4.0)
    g.rk4_step(prm, 0.0, dt, U)
    R = lambda z: 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    I = inputs.interior(U, c.bs, c.ng)
    for comp, v0 in enumerate((0.3, -1.2, 2.0)):
        assert np.max(np.abs(I[:, comp] - v0 * R(-dt / ce))) < 1e-15
    assert np.max(np.abs(I[:, 3] - 5.0 * R(-cg * dt))) < 1e-14


def test_rk4_sponge_relaxation(orc):
    c = uniform_case(1, L=1.0)
    g = grid_of(orc, c)
    one = np.ones((g.nb, c.bs, c.bs, c.bs))
    U = inputs.pack([0.0 * one, one, 0.0 * one, 2.0 * one], c.bs, c.ng)
    csp, dt = 0.05, 0.01
    prm = cases.params(sponge=1, l_sp=0.6, c_sp=csp, u_inf=(1.0, 0.0, -0.5), p_inf=0.25,
                       c_gamma=0.0, nu=0.0)
    g.rk4_step(prm, 0.0, dt, U)
    R = lambda z: 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    I = inputs.interior(U, c.bs, c.ng)
    f = R(-dt / csp)
    for comp, (v0, vi) in enumerate(((0.0, 1.0), (1.0, 0.0), (0.0, -0.5), (2.0, 0.25))):
        assert np.max(np.abs(I[:, comp] - (vi + (v0 - vi) * f))) < 1e-14


def test_dt_taylor_green_closed_form(orc):
    c = cases.taylor_green()
    g = grid_of(orc, c)
    dt = g.dt(c.params, c.padded())
    exp = 0.5 * (2 * math.pi / 64) / (1 + math.sqrt(1 + 100))
    assert dt == pytest.approx(exp, rel=1e-14)
    assert dt == pytest.approx(4.44235e-3, rel=1e-5)


def test_rk4_time_order(orc):
    # Taylor-Green, two steps of dt/2 vs one of dt vs a fine reference
    c = cases.taylor_green()
    g = grid_of(orc, c)
    U0 = c.padded()
    prm = dict(c.params)

    def run(n, T):
        U = U0.copy()
        for s in range(n):
            g.rk4_step(prm, s * T / n, T / n, U)
        return inputs.interior(U, c.bs, c.ng)

    T = 0.08
    ref = run(32, T)
    e1 = np.max(np.abs(run(2, T) - ref))
    e2 = np.max(np.abs(run(4, T) - ref))
    assert 3.6 < math.log2(e1 / e2) < 4.4


# ---------------------------------------------------------------- diagnostics
def test_force_and_energy_closed_form(orc):
    c = uniform_case(1, L=1.0)
    g = grid_of(orc, c)
    one = np.ones((g.nb, c.bs, c.bs, c.bs))
    U = inputs.pack([0.5 * one, -0.25 * one, 1.0 * one, 3.0 * one], c.bs, c.ng)
    prm = _full_solid_params(c_eta=1e-3)
    d = g.diagnostics(prm, 0.0, U)
    assert d[0] == pytest.approx(math.sqrt(0.25 + 0.0625 + 1.0), rel=1e-15)
    assert list(d[1:5]) == pytest.approx([0.5, 0.25, 1.0, 3.0], rel=1e-15)
    assert list(d[5:8]) == pytest.approx([500.0, -250.0, 1000.0], rel=1e-12)
    assert d[8] == pytest.approx(0.5 * (0.25 + 0.0625 + 1.0), rel=1e-12)


def test_plate_solid_velocity_is_rigid_rotation(orc):
    # u_s against the closed form of a rigid rotation about the y axis through
    # the leading edge, alpha-dot e_y x (x - x_le); that chi rotates the same
    # way is pinned in test_oracle_pins_model.py
    c = uniform_case(1, L=4.0)
    g = grid_of(orc, c)
    prm = cases.plate_params(5)
    t = 0.137
    chi, us = g.mask(prm, t)
    x, y, z = (a.reshape(g.nb, -1) for a in c.coords())
    adot = 0.8 * 2 * math.pi * math.cos(2 * math.pi * t)
    assert np.max(np.abs(us[:, 0] - adot * (z - 2.0))) < 1e-13
    assert np.max(np.abs(us[:, 1])) == 0.0
    assert np.max(np.abs(us[:, 2] + adot * (x - 2.0))) < 1e-13
    assert chi.max() <= 1.0 and chi.min() >= 0.0


# ---------------------------------------------------------------- details
def _fill_poly(g, f):
    bs, ng, P = g.bs, g.ng, g.P
    U = np.zeros((g.nb, 4, P, P, P))
    for b in range(g.nb):
        h = g.L / ((1 << g.lev[b]) * bs)
        r = np.arange(-ng, bs + ng)
        zz, yy, xx = np.meshgrid((g.iz[b] * bs + r) * h, (g.iy[b] * bs + r) * h,
                                 (g.ix[b] * bs + r) * h, indexing="ij")
        for c in range(4):
            U[b, c] = f(c, xx, yy, zz)
    return U


def test_details_vanish_for_cubics(orc):
    lev, ix, iy, iz = inputs.uniform_leaves(1)
    g = orc.Grid(16, 4, 1.0, 1, 1, lev, ix, iy, iz)
    U = _fill_poly(g, lambda c, x, y, z: 1 + c * x ** 3 * y ** 2 - z ** 3 * x + y ** 3 * z ** 3)
    dmax, mr = g.details(None, 0.0, U)
    assert np.max(dmax) < 1e-14
    assert np.all(mr == 0.0)


def test_details_quartic_is_9h4(orc):
    lev, ix, iy, iz = inputs.uniform_leaves(1)
    g = orc.Grid(16, 4, 1.0, 1, 1, lev, ix, iy, iz)
    h = 1.0 / 32
    U = _fill_poly(g, lambda c, x, y, z: (x if c == 0 else (y if c == 1 else z)) ** 4
                   if c < 3 else np.zeros_like(x))
    dmax, _ = g.details(None, 0.0, U)
    # component norms: max x^4 over interiors of the whole grid = (31 h)^4
    norm = (31 * h) ** 4
    assert np.allclose(dmax, 9 * h ** 4 / norm, rtol=1e-9, atol=0)


# ---------------------------------------------------------------- filtering
def test_filter_quartic_closed_form(orc):
    # Removing the details of u = x^4 subtracts the cubic interpolation error
    # (x+3h)(x+h)(x-h)(x-3h) at x = 0, i.e. 9 h^4, at every point whose x
    # index is odd, whatever the parity in y and z; points with an even x
    # index keep their value.  A cubic is reproduced, zeros stay zero.
    lev, ix, iy, iz = inputs.uniform_leaves(1)
    g = orc.Grid(16, 4, 1.0, 1, 1, lev, ix, iy, iz)
    h = 1.0 / 32
    U = _fill_poly(g, lambda c, x, y, z: x ** 4 if c == 0 else
                   ((y ** 3 - 2 * z * x * y + x ** 2) if c == 1 else 0 * x))
    F = U.copy()
    g.filter(-1, F)
    I = slice(g.ng, g.ng + g.bs)
    odd_x = (np.arange(g.bs) % 2 == 1)[None, None, :]
    d0 = (U[:, 0, I, I, I] - F[:, 0, I, I, I])
    assert np.max(np.abs(np.where(odd_x, d0 - 9 * h ** 4, d0))) < 1e-14
    assert np.max(np.abs(U[:, 1, I, I, I] - F[:, 1, I, I, I])) < 1e-14
    assert np.all(F[:, 2:] == 0.0)


def test_filter_keeps_even_points_is_idempotent_and_selects_level(orc):
    lev, ix, iy, iz = inputs.random_balanced_leaves(11, 1, 3, 60)
    g = orc.Grid(16, 4, 1.0, 1, 3, lev, ix, iy, iz)
    rng = np.random.default_rng(5)
    U = rng.standard_normal((g.nb, 4, g.P, g.P, g.P))
    g.sync(U)
    F = U.copy()
    g.filter(-1, F)
    ng, bs = g.ng, g.bs
    I = slice(ng, ng + bs)
    E = slice(ng, ng + bs, 2)
    # points with three even indices and every ghost point are untouched
    assert np.array_equal(F[:, :, E, E, E], U[:, :, E, E, E])
    ghost = np.ones((g.P, g.P, g.P), bool)
    ghost[I, I, I] = False
    assert np.array_equal(F[:, :, ghost], U[:, :, ghost])
    # odd points did change (random data has details)
    assert np.max(np.abs(F[:, :, I, I, I] - U[:, :, I, I, I])) > 1e-3
    # the predictions read only even points: a second pass changes nothing
    F2 = F.copy()
    g.filter(-1, F2)
    assert np.array_equal(F2, F)
    # one level only: those blocks as in the full pass, the others untouched
    J = int(g.lev.max())
    FJ = U.copy()
    g.filter(J, FJ)
    sel = np.asarray(g.lev) == J
    assert 0 < sel.sum() < g.nb
    assert np.array_equal(FJ[sel], F[sel])
    assert np.array_equal(FJ[~sel], U[~sel])


# ---------------------------------------------------------------- CDF 4/4 lifting
def test_lifted_lowpass_taps(orc):
    # CDF 2/2: the paper's lifted low-pass for linear interpolation (Sec. 3.2,
    # printed with garbled signs; read as the 5-tap filter whose taps sum to 1)
    t2 = orc.lift_lowpass(2)
    assert np.array_equal(t2, np.array([0, 0, 0, 0, -1, 2, 6, 2, -1, 0, 0, 0, 0]) / 8)
    # CDF 4/4: the lifting steps expanded by hand (predict (-1, 9, 9, -1)/16,
    # update (-1, 9, 9, -1)/32)
    t4 = orc.lift_lowpass(4)
    assert np.array_equal(t4, np.array([-1, 0, 18, -16, -63, 144, 348, 144, -63, -16, 18, 0,
                                        -1]) / 512)
    # M vanishing moments of the lifted primal wavelet <=> the low-pass keeps
    # the mean and has an M-fold zero at the Nyquist frequency:
    # sum (-1)^n n^p h_n = 0 for p < M, and not for p = M
    n = np.arange(-6, 7)
    for t, M in ((t2, 2), (t4, 4)):
        assert abs(t.sum() - 1.0) < 1e-15
        for p in range(M):
            assert abs(np.sum((-1.0) ** n * n ** p * t)) < 1e-13
        assert abs(np.sum((-1.0) ** n * n ** M * t)) > 1e-3


def _one_refined_block(bs=24, ng=6):
    """Uniform level 1 with block (0,0,0) split into its 8 children."""
    leaves = [(1, x, y, z) for z in range(2) for y in range(2) for x in range(2) if (x, y, z) != (0, 0, 0)]
    leaves += [(2, x, y, z) for z in range(2) for y in range(2) for x in range(2)]
    lev = np.array([l[0] for l in leaves], np.int32)
    ix, iy, iz = (np.array([l[d] for l in leaves], np.int64) for d in (1, 2, 3))
    return lev, ix, iy, iz


def test_cdf44_sync_quartic_closed_form(orc):
    # u = x^4: the details along x are 9 h^4 at every odd point, so the lifted
    # restriction adds (-1 + 9 + 9 - 1)/32 * 9 h^4 = 4.5 h^4 (h the fine
    # spacing) to the decimated value; the y and z passes see a function
    # constant along them.  Checked at ghost points of the coarse block next
    # to the children whose 13-point stencils stay inside a child's interior.
    lev, ix, iy, iz = _one_refined_block()
    g4 = orc.Grid(24, 6, 1.0, 1, 2, lev, ix, iy, iz)
    g0 = orc.Grid(24, 6, 1.0, 1, 2, lev, ix, iy, iz)
    g4.set_wavelet(1)
    U = _fill_poly(g4, lambda c, x, y, z: x ** 4 if c == 0 else 0 * x)
    U0 = U.copy()
    g4.sync(U)
    g0.sync(U0)
    b = [i for i in range(g4.nb) if (g4.lev[i], g4.ix[i], g4.iy[i], g4.iz[i]) == (1, 1, 0, 0)][0]
    ng, bs = 6, 24
    hf = 1.0 / 96
    js = [j for j in range(bs) if 3 <= j <= 8 or 15 <= j <= 20]
    n = 0
    for d in range(4, 7):
        x = 0.5 - d / 48
        for j in js:
            for k in js:
                v4 = U[b, 0, k + ng, j + ng, -d + ng]
                v0 = U0[b, 0, k + ng, j + ng, -d + ng]
                assert abs(v0 - x ** 4) < 1e-16
                assert abs(v4 - (x ** 4 + 4.5 * hf ** 4)) < 1e-15
                n += 1
    assert n == 3 * len(js) ** 2
    # other ghost points whose owner is not finer are untouched by the lifting
    assert np.array_equal(U[[i for i in range(g4.nb) if g4.lev[i] == 2]],
                          U0[[i for i in range(g4.nb) if g4.lev[i] == 2]])


def test_cdf44_sync_cubic_equals_decimation(orc):
    lev, ix, iy, iz = _one_refined_block()
    g4 = orc.Grid(24, 6, 1.0, 1, 2, lev, ix, iy, iz)
    g0 = orc.Grid(24, 6, 1.0, 1, 2, lev, ix, iy, iz)
    g4.set_wavelet(1)
    f = lambda c, x, y, z: 1 + (c + 1) * x ** 3 - y ** 2 * z + 0.5 * x * y * z ** 2
    U = _fill_poly(g4, f)
    U0 = U.copy()
    g4.sync(U)
    g0.sync(U0)
    # the -x ghost layers of the coarse block next to the children, at
    # tangential positions whose stencils stay off the periodic wrap (where a
    # polynomial jumps); every depth 1..6
    b = [i for i in range(g4.nb) if (g4.lev[i], g4.ix[i], g4.iy[i], g4.iz[i]) == (1, 1, 0, 0)][0]
    js = np.array([j for j in range(24) if 3 <= j <= 8 or 15 <= j <= 20]) + 6
    G4 = U[b][:, js][:, :, js][:, :, :, 0:6]
    G0 = U0[b][:, js][:, :, js][:, :, :, 0:6]
    assert np.max(np.abs(G4 - G0)) < 1e-14
    with pytest.raises(ValueError):
        orc.Grid(24, 4, 1.0, 1, 2, lev, ix, iy, iz).set_wavelet(1)


def test_cdf44_coarsen_quartic_closed_form(orc):
    lev, ix, iy, iz = _one_refined_block()
    g = orc.Grid(24, 6, 1.0, 1, 2, lev, ix, iy, iz)
    g.set_wavelet(1)
    U = _fill_poly(g, lambda c, x, y, z: x ** 4 if c == 0 else 0 * x)  # analytic ghosts
    flags = (np.asarray(g.lev) == 2).astype(np.int8)
    g2, U2 = g.coarsen(flags, U)
    assert g2.nb == 8
    p = [i for i in range(g2.nb) if (g2.ix[i], g2.iy[i], g2.iz[i]) == (0, 0, 0)][0]
    x = (np.arange(24) / 48.0)[None, None, :]
    I = slice(6, 30)
    assert np.max(np.abs(U2[p, 0, I, I, I] - (x ** 4 + 4.5 / 96 ** 4))) < 1e-15
    assert np.all(U2[p, 1:, I, I, I] == 0.0)


def test_cdf44_refine_then_coarsen_is_identity(orc):
    # the lifted restriction inverts the DD4 prediction: all details of a
    # predicted field vanish, so the update adds nothing
    lev, ix, iy, iz = inputs.uniform_leaves(1)
    g = orc.Grid(24, 6, 1.0, 1, 2, lev, ix, iy, iz)
    g.set_wavelet(1)
    rng = np.random.default_rng(8)
    U = rng.standard_normal((g.nb, 4, g.P, g.P, g.P))
    g.sync(U)
    g2, U2 = g.refine_all(U)
    g2.sync(U2)
    g3, U3 = g2.coarsen(np.ones(g2.nb, np.int8), U2)
    assert g3.nb == g.nb
    I = slice(6, 30)
    assert np.max(np.abs(U3[:, :, I, I, I] - U[:, :, I, I, I])) < 1e-13


# ---------------------------------------------------------------- adaptation
def test_refine_then_coarsen_is_identity(orc):
    lev, ix, iy, iz = inputs.random_balanced_leaves(4, 1, 3, 50)
    g = orc.Grid(16, 4, 1.0, 1, 4, lev, ix, iy, iz)
    rng = np.random.default_rng(4)
    U = rng.standard_normal((g.nb, 4, g.P, g.P, g.P))
    g.sync(U)
    g2, U2 = g.refine_all(U)
    assert g2.nb == int(np.sum(np.where(g.lev < 4, 8, 1)))
    assert g2.is_balanced()
    # merging is Jacobi over the current leaves and respects grading, so the
    # finest families merge first; repeat, flagging every block that is not
    # an original leaf, until the original leaf set is back.
    orig = {(l, x, y, z): b for b, (l, x, y, z) in enumerate(zip(g.lev, g.ix, g.iy, g.iz))}
    gc, Uc = g2, U2
    for _ in range(4):
        fl = np.array([0 if (l, x, y, z) in orig else 1
                       for l, x, y, z in zip(gc.lev, gc.ix, gc.iy, gc.iz)], np.int8)
        if not fl.any():
            break
        gc, Uc = gc.coarsen(fl, Uc)
    assert gc.nb == g.nb
    for b in range(gc.nb):
        ob = orig[(gc.lev[b], gc.ix[b], gc.iy[b], gc.iz[b])]
        assert np.array_equal(inputs.interior(Uc[b], 16, 4), inputs.interior(U[ob], 16, 4))


def test_refinement_reproduces_cubic(orc):
    lev, ix, iy, iz = inputs.uniform_leaves(1)
    g = orc.Grid(16, 4, 1.0, 1, 2, lev, ix, iy, iz)
    f = lambda c, x, y, z: 2 - x ** 3 + c * y ** 2 * z + x * y * z ** 3
    U = _fill_poly(g, f)
    g2, U2 = g.refine_all(U)
    V = _fill_poly(g2, f)
    assert np.max(np.abs(inputs.interior(U2, 16, 4) - inputs.interior(V, 16, 4))) < 1e-14


def test_coarsening_respects_grading(orc):
    # a fine cluster next to a mergeable group: the group must not merge if
    # its parent would touch blocks two levels finer
    lev, ix, iy, iz = inputs.uniform_leaves(1)
    ls = inputs.LeafSet(zip(lev, ix, iy, iz), 1)
    ls.refine((1, 0, 0, 0))
    ls.refine((2, 1, 0, 0))      # level 3 next to level-2 sisters
    l, x, y, z = ls.arrays()
    g = orc.Grid(16, 4, 1.0, 1, 3, l, x, y, z)
    U = np.zeros((g.nb, 4, g.P, g.P, g.P))
    flags = np.where(g.lev == 2, 1, 0).astype(np.int8)
    g2, _ = g.coarsen(flags, U)
    # the level-2 family under (1,0,0,0) holds the refined (2,1,0,0) -> no merge
    assert g2.nb == g.nb
    flags = np.where(g.lev == 3, 1, 0).astype(np.int8)
    g3, _ = g.coarsen(flags, U)
    assert g3.nb == g.nb - 7 and g3.is_balanced()
    # now the level-2 blocks may merge into (1,0,0,0)
    g4, _ = g3.coarsen(np.where(g3.lev == 2, 1, 0).astype(np.int8),
                       np.zeros((g3.nb, 4, g.P, g.P, g.P)))
    assert g4.nb == 8 and np.all(g4.lev == 1)
