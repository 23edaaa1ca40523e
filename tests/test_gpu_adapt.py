"""GPU parity of the adaptation rows: wavelet details and coarsening flags,
refine-all, one coarsening pass, and the refine -> evolve -> coarsen step on
the rotating-plate case, against the FP64 oracle through the C ABI.

Adaptive runs use flag replay: the GPU follows the oracle's coarsening flags
(mapped by treecode), so both sides visit the same grids; the GPU's own flags
are computed as well and the number of disagreements is reported (exact
agreement is required in FP64, where both sides take the decision from the
same FP64 details up to rounding).
"""
import numpy as np
import pytest

from paper_1912_05371_amd import cases, inputs, wacm

from gpu_util import from_pool, log, rel_err, slot_map, to_pool

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def plate_small(clip=1):
    c = cases.plate_adaptive(jmin=2, jmax=4, jstart=3)
    c.params = cases.plate_params(4, c.bs, c.L, clip=clip)
    return c


def octree16():
    return cases.random_octree(bs=16, ng=4, target=200, j0=1, jmax=3, seed=11)


CASES = {"sphere": cases.sphere_two_level, "octree16": octree16, "plate": plate_small}


def build(orc, c, prec=wacm.F64, capacity=None):
    og = orc.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, c.lev, c.ix, c.iy, c.iz)
    gg = wacm.Grid.from_case(c, dtype=prec, capacity=capacity or 9 * c.nb + 64)
    return og, gg


def put(gg, og, U, pool=None):
    """Oracle state (oracle block order) into the GPU pool at the GPU slots."""
    if pool is None:
        pool = gg.pool()
    slots = slot_map(gg, og)
    pool[torch.as_tensor(slots, device="cuda")] = torch.from_numpy(U).to(
        device="cuda", dtype=gg.torch_dtype())
    return pool


def active_index(gg, og):
    slots, codes, levels = gg.info()
    pos = {(int(l), int(c)): i for i, (c, l) in enumerate(zip(codes, levels))}
    return np.array([pos[(int(og.lev[b]), wacm.treecode_encode(og.lev[b], og.ix[b], og.iy[b],
                                                                og.iz[b]))]
                     for b in range(og.nb)])


def same_leaves(gg, og):
    slots, codes, levels = gg.info()
    a = sorted(zip(levels.tolist(), codes.tolist()))
    b = sorted((int(l), wacm.treecode_encode(l, x, y, z))
               for l, x, y, z in zip(og.lev, og.ix, og.iy, og.iz))
    return a == b


@pytest.mark.parametrize("name", list(CASES))
def test_threshold_matches_oracle(orc, name):
    log(f"threshold {name}")
    c = CASES[name]()
    og, gg = build(orc, c)
    U = c.padded()
    rng = np.random.default_rng(5)
    # smooth state plus a few sharp spots so that details spread over decades
    U[..., c.ng:-c.ng, c.ng:-c.ng, c.ng:-c.ng] += 1e-3 * rng.standard_normal(
        (og.nb, 4, c.bs, c.bs, c.bs)) * (rng.uniform(size=(og.nb, 1, 1, 1, 1)) < 0.2)
    t = 0.07
    og.sync(U)
    dm_o, mr_o = og.details(c.params, t, U)
    eps = float(np.median(dm_o))  # a threshold inside the spread of details
    fl_o = og.flags(dm_o, mr_o, eps, True)
    pool = put(gg, og, U)
    gg.sync_ghosts(pool)
    nb = gg.nb
    dmax = torch.zeros(nb, dtype=torch.float64, device="cuda")
    mr = torch.zeros(nb, dtype=torch.float64, device="cuda")
    fl = torch.zeros(nb, dtype=torch.int8, device="cuda")
    gg.threshold_blocks(c.params, t, pool, eps, True, dmax, mr, fl)
    torch.cuda.synchronize()
    ai = active_index(gg, og)
    dm_g, mr_g, fl_g = dmax.cpu().numpy()[ai], mr.cpu().numpy()[ai], fl.cpu().numpy()[ai]
    e = np.max(np.abs(dm_g - dm_o) / np.maximum(dm_o, 1e-300))
    log(f"  details rel err {e:.2e}; mask-range max diff {np.max(np.abs(mr_g - mr_o)):.2e}; "
        f"flags set {int(fl_o.sum())}/{og.nb}, disagreements {int(np.sum(fl_g != fl_o))}")
    assert e < 1e-10
    assert np.max(np.abs(mr_g - mr_o)) < 1e-12
    assert np.array_equal((mr_g > 0), (mr_o > 0))
    assert np.array_equal(fl_g, fl_o)


@pytest.mark.parametrize("name", ["octree16", "plate"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_filter_matches_oracle(orc, name, prec):
    c = CASES[name]()
    og, gg = build(orc, c, wacm.F64 if prec == "f64" else wacm.F32)
    U = c.padded()
    og.sync(U)
    J = int(np.max(og.lev))
    for level in (-1, J):
        log(f"filter {name} {prec} level {level}")
        pool = put(gg, og, U)
        gg.filter_blocks(pool, level)
        Uo = U.copy()
        og.filter(level, Uo)
        Ug = from_pool(pool, slot_map(gg, og))
        e = rel_err(Ug, Uo, c.bs, c.ng)
        log(f"  interior rel err {e:.2e}")
        # FP64: separable vs tensor-sum rounding; FP32: the input's rounding
        assert e < (1e-14 if prec == "f64" else 1e-6)
        if prec == "f64" and level == J:
            keep = np.asarray(og.lev) != J
            assert np.array_equal(Ug[keep], U[keep])


@pytest.mark.parametrize("name", ["octree16", "plate"])
def test_refine_all_matches_oracle(orc, name):
    log(f"refine_all {name}")
    c = CASES[name]()
    og, gg = build(orc, c)
    U = c.padded()
    pool = put(gg, og, U)
    nb_new = gg.adapt(wacm.REFINE_ALL, pool)
    Uo = U.copy()
    og.sync(Uo)
    og2, Uo2 = og.refine_all(Uo)
    assert nb_new == og2.nb and same_leaves(gg, og2)
    Ug = from_pool(pool, slot_map(gg, og2))
    e = rel_err(Ug, Uo2, c.bs, c.ng)
    log(f"  {og.nb} -> {og2.nb} blocks, interior rel err {e:.2e}")
    assert e < 1e-14


def test_coarsen_pass_matches_oracle(orc):
    log("coarsen octree16")
    c = octree16()
    og, gg = build(orc, c)
    U = c.padded()
    rng = np.random.default_rng(3)
    flags_o = (rng.uniform(size=og.nb) < 0.7).astype(np.int8)
    og2, Uo2 = og.coarsen(flags_o, U)
    pool = put(gg, og, U)
    ai = active_index(gg, og)
    flags_g = np.zeros(og.nb, np.int8)
    flags_g[ai] = flags_o
    nb_new = gg.adapt(wacm.COARSEN, pool, flags_g)
    log(f"  {og.nb} -> {og2.nb} blocks")
    assert og2.nb < og.nb
    assert nb_new == og2.nb and same_leaves(gg, og2)
    Ug = from_pool(pool, slot_map(gg, og2))
    I = slice(c.ng, c.ng + c.bs)
    assert np.array_equal(Ug[..., I, I, I], Uo2[..., I, I, I])


def test_capacity_error_leaves_grid_unchanged(orc):
    c = octree16()
    og, gg = build(orc, c, capacity=c.nb + 7)
    pool = gg.pool()
    before = gg.info()
    with pytest.raises(wacm.WacmError) as e:
        gg.adapt(wacm.REFINE_ALL, pool)
    assert e.value.code == wacm.E_CAPACITY
    after = gg.info()
    assert all(np.array_equal(a, b) for a, b in zip(before, after))


def adaptive_step_oracle(og, U, prm, t, eps, dealias):
    """Sec. 3.5: refine all, one RK4 step, coarsen until no block merges.
    Returns the new grid, state, dt and the flag lists used by each pass."""
    og.sync(U)
    g1, U1 = og.refine_all(U)
    dt = g1.dt(prm, U1)
    g1.rk4_step(prm, t, dt, U1)
    passes = []
    while True:
        g1.sync(U1)
        dm, mr = g1.details(prm, t + dt, U1)
        fl = g1.flags(dm, mr, eps, dealias)
        n_new = g1.coarsen_count(fl)
        if n_new == g1.nb:
            break
        passes.append((g1, fl))
        g1, U1 = g1.coarsen(fl, U1)
    return g1, U1, dt, passes


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adaptive_plate_replay(orc, prec):
    """Refine -> evolve -> coarsen (Sec. 3.5) on the rotating plate, 2 steps,
    each from the oracle's state; GPU follows the oracle's flags."""
    log(f"adaptive plate {prec}")
    c = plate_small()
    eps, dealias = c.extra["eps"], c.extra["dealias"]
    og = orc.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, c.lev, c.ix, c.iy, c.iz)
    U = c.padded()
    t = 0.0
    dtype = wacm.F64 if prec == "f64" else wacm.F32
    for step in range(2):
        og_n, U_n, dt, passes = adaptive_step_oracle(og, U.copy(), c.params, t, eps, dealias)
        # GPU from the same start grid and state
        lev, ix, iy, iz = og.lev, og.ix, og.iy, og.iz
        codes = [wacm.treecode_encode(l, x, y, z) for l, x, y, z in zip(lev, ix, iy, iz)]
        gg = wacm.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, codes, lev, dtype, capacity=12 * og.nb)
        Uin = U.astype(np.float32).astype(np.float64) if prec == "f32" else U
        pool = put(gg, og, Uin)
        gg.adapt(wacm.REFINE_ALL, pool)
        work = gg.work()
        t_dev = torch.tensor([t], dtype=torch.float64, device="cuda")
        dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
        gg.rk4_step(c.params, t_dev, dt_dev, pool, work, dt_mode=wacm.DT_FIXED)
        disagree = 0
        for g_o, fl_o in passes:
            assert same_leaves(gg, g_o)
            gg.sync_ghosts(pool)
            nb = gg.nb
            dmax = torch.zeros(nb, dtype=torch.float64, device="cuda")
            mr = torch.zeros(nb, dtype=torch.float64, device="cuda")
            fl = torch.zeros(nb, dtype=torch.int8, device="cuda")
            gg.threshold_blocks(c.params, t + dt, pool, eps, dealias, dmax, mr, fl)
            ai = active_index(gg, g_o)
            own = fl.cpu().numpy()[ai]
            disagree += int(np.sum(own != fl_o))
            flags_g = np.zeros(nb, np.int8)
            flags_g[ai] = fl_o
            gg.adapt(wacm.COARSEN, pool, flags_g)
        assert same_leaves(gg, og_n)
        Ug = from_pool(pool, slot_map(gg, og_n))
        e = rel_err(Ug, U_n, c.bs, c.ng)
        log(f"  step {step}: {og.nb} -> refine -> {len(passes)} merge passes -> {og_n.nb} blocks;"
            f" state rel err {e:.2e}; own-flag disagreements {disagree}")
        assert e < (1e-12 if prec == "f64" else 1e-5)
        if prec == "f64":
            assert disagree == 0
        og, U, t = og_n, U_n, t + dt
        del gg


def test_adaptive_driver_matches_oracle(orc):
    """adaptive.adaptive_step (the ABI calls of Sec. 3.5 in sequence, with the
    GPU's own coarsening flags) against the oracle's adaptive step, 2 steps of
    the rotating plate in FP64: same leaves and states to 1e-12."""
    from paper_1912_05371_amd.adaptive import adaptive_step
    c = plate_small()
    eps, dealias = c.extra["eps"], c.extra["dealias"]
    log(f"adaptive driver, plate {c.nb} blocks")
    og = orc.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, c.lev, c.ix, c.iy, c.iz)
    U = c.padded()
    gg = wacm.Grid.from_case(c, dtype=wacm.F64, capacity=12 * c.nb + 64)
    pool = put(gg, og, U)
    work = gg.work()
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = 0.0
    for step in range(2):
        og, U, dt, passes = adaptive_step_oracle(og, U, c.params, t, eps, dealias)
        t += dt
        timings = {}
        merged = adaptive_step(gg, c.params, pool, work, t_dev, dt_dev, eps, dealias,
                               timings=timings)["merged_passes"]
        assert same_leaves(gg, og)
        e = rel_err(from_pool(pool, slot_map(gg, og)), U, c.bs, c.ng)
        log(f"  step {step}: {og.nb} blocks, {merged} merging passes (oracle {len(passes)}), "
            f"state rel err {e:.2e}, dt {float(dt_dev.item()):.6e} vs {dt:.6e}; "
            f"{ {k: round(v['wall'], 2) for k, v in timings.items()} } ms")
        assert merged == len(passes)
        assert e < 1e-12
        assert abs(float(t_dev.item()) - t) <= 1e-12 * t
        # every phase split into host and device time that add up to its wall time
        for rec in timings.values():
            assert rec["host"] >= 0.0 and rec["device"] >= 0.0
            assert abs(rec["host"] + rec["device"] - rec["wall"]) <= 1e-9 * max(rec["wall"], 1.0)
        host_ms, dev_ms = gg.adapt_timing()
        assert host_ms > 0.0 and dev_ms >= 0.0


@pytest.fixture(scope="module")
def c3_oracle_steps(orc):
    """The rotating plate as configured (levels 2..6, bs 16, eps 1e-3,
    dealiasing; start grid refined to level 5 around the plate): two adaptive
    steps of the oracle, with their coarsening passes."""
    c = cases.plate_adaptive()
    assert (c.jmin, c.jmax) == (2, 6)
    eps, dealias = c.extra["eps"], c.extra["dealias"]
    og = orc.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, c.lev, c.ix, c.iy, c.iz)
    U = c.padded()
    steps, t = [], 0.0
    for _ in range(2):
        og_n, U_n, dt, passes = adaptive_step_oracle(og, U.copy(), c.params, t, eps, dealias)
        steps.append((og, U, t, og_n, U_n, dt, passes))
        og, U, t = og_n, U_n, t + dt
    return c, steps


def test_plate_c3_driver_matches_oracle(c3_oracle_steps):
    """adaptive.adaptive_step on the configured rotating-plate case (its own
    FP64 flags) against the oracle's first two adaptive steps: the same leaves
    after every step, the state to 1e-12 and the same time."""
    from paper_1912_05371_amd.adaptive import adaptive_step
    c, steps = c3_oracle_steps
    eps, dealias = c.extra["eps"], c.extra["dealias"]
    og0 = steps[0][0]
    gg = wacm.Grid.from_case(c, dtype=wacm.F64, capacity=10 * c.nb + 64)
    pool = put(gg, og0, steps[0][1])
    work = gg.work()
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    for k, (og, U, t, og_n, U_n, dt, passes) in enumerate(steps):
        r = adaptive_step(gg, c.params, pool, work, t_dev, dt_dev, eps, dealias)
        assert same_leaves(gg, og_n)
        e = rel_err(from_pool(pool, slot_map(gg, og_n)), U_n, c.bs, c.ng)
        log(f"  C3 step {k}: {og.nb} -> {r['refined']} -> {og_n.nb} blocks, "
            f"{r['merged_passes']} merging passes (oracle {len(passes)}), rel err {e:.2e}, "
            f"dt {float(dt_dev.item()):.6e} vs {dt:.6e}")
        assert r["merged_passes"] == len(passes)
        assert e < 1e-12
        assert abs(float(t_dev.item()) - (t + dt)) <= 1e-12 * (t + dt)


def test_plate_c3_fp32_replay_matches_oracle(c3_oracle_steps):
    """FP32 on the configured rotating-plate case, each step from the oracle's
    state rounded to FP32 and following the oracle's flags: 1e-5 relative."""
    c, steps = c3_oracle_steps
    eps, dealias = c.extra["eps"], c.extra["dealias"]
    for k, (og, U, t, og_n, U_n, dt, passes) in enumerate(steps):
        codes = [wacm.treecode_encode(l, x, y, z) for l, x, y, z in
                 zip(og.lev, og.ix, og.iy, og.iz)]
        gg = wacm.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, codes, og.lev, wacm.F32,
                       capacity=10 * og.nb + 64)
        pool = put(gg, og, U.astype(np.float32).astype(np.float64))
        gg.adapt(wacm.REFINE_ALL, pool)
        work = gg.work()
        t_dev = torch.tensor([t], dtype=torch.float64, device="cuda")
        dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
        gg.rk4_step(c.params, t_dev, dt_dev, pool, work, dt_mode=wacm.DT_FIXED)
        disagree = 0
        for g_o, fl_o in passes:
            assert same_leaves(gg, g_o)
            gg.sync_ghosts(pool)
            nb = gg.nb
            dmax = torch.zeros(nb, dtype=torch.float64, device="cuda")
            mr = torch.zeros(nb, dtype=torch.float64, device="cuda")
            fl = torch.zeros(nb, dtype=torch.int8, device="cuda")
            gg.threshold_blocks(c.params, t + dt, pool, eps, dealias, dmax, mr, fl)
            ai = active_index(gg, g_o)
            disagree += int(np.sum(fl.cpu().numpy()[ai] != fl_o))
            flags_g = np.zeros(nb, np.int8)
            flags_g[ai] = fl_o
            gg.adapt(wacm.COARSEN, pool, flags_g)
        assert same_leaves(gg, og_n)
        e = rel_err(from_pool(pool, slot_map(gg, og_n)), U_n, c.bs, c.ng)
        log(f"  C3 FP32 step {k}: rel err {e:.2e}, own-flag disagreements {disagree}")
        assert e < 1e-5
        del gg, pool, work
        torch.cuda.empty_cache()


@pytest.mark.parametrize("which", ["plate", "oct24", "oct32"])
@pytest.mark.parametrize("prec", [wacm.F64, wacm.F32])
def test_lattice_sync_matches_full_sync(which, prec):
    """wacm_sync_ghosts_lattice writes exactly the ghost points of the even
    lattice within 3 of each block, with the values wacm_sync_ghosts gives
    them, and leaves every other point alone; thresholding after it gives
    bitwise the results it gives after the full sync."""
    if which == "plate":
        c = cases.plate_adaptive()
        eps, dealias = 1e-3, True
    else:
        bs, ng, target, seed = (24, 4, 1500, 8) if which == "oct24" else (32, 5, 300, 9)
        c = cases.random_octree(bs=bs, ng=ng, target=target, j0=2, jmax=5, seed=seed,
                                with_fields=False)
        rng = np.random.default_rng(seed)
        c.fields = [rng.standard_normal((c.nb, bs, bs, bs)) for _ in range(4)]
        eps, dealias = 1.0, which == "oct32"
    log(f"lattice sync, {which} {c.nb} blocks, dtype {prec}")
    g = wacm.Grid.from_case(c, dtype=prec)
    U0 = to_pool(g, c.padded(fill=7.0), fill=7.0)
    A, B = U0.clone(), U0.clone()
    g.sync_ghosts(A)
    g.sync_ghosts_lattice(B)
    torch.cuda.synchronize()
    bs, ng, P = c.bs, c.ng, c.bs + 2 * c.ng
    q = np.arange(P) - ng
    lat = (q % 2 == 0) & (q >= -2) & (q <= bs + 2)
    inner = (q >= 0) & (q < bs)
    L3 = lat[:, None, None] & lat[None, :, None] & lat[None, None, :]
    I3 = inner[:, None, None] & inner[None, :, None] & inner[None, None, :]
    sel = torch.as_tensor(L3 & ~I3, device="cuda")
    a, b, u0 = A[:c.nb], B[:c.nb], U0[:c.nb]
    assert torch.equal(b[:, :, sel], a[:, :, sel])
    assert torch.equal(b[:, :, ~sel], u0[:, :, ~sel])
    n = g.nb
    out = []
    for V in (A, B):
        dm = torch.empty(n, dtype=torch.float64, device="cuda")
        mr = torch.empty_like(dm)
        fl = torch.empty(n, dtype=torch.int8, device="cuda")
        g.threshold_blocks(c.params, 0.05, V, eps, dealias, dm, mr, fl)
        out.append((dm, mr, fl))
    torch.cuda.synchronize()
    for x, y in zip(*out):
        assert torch.equal(x, y)
