"""GPU parity of the CDF 4/4 lifted restriction (Sec. 3.2) against the FP64
oracle through the C ABI: the two-phase ghost synchronisation (ghost layers
included in the comparison), a coarsening pass whose parents are lifted
restrictions of their children, and refine-all (whose own synchronisation
uses the lifted ghost values).  Grid: a seeded random 2:1 octree with bs 24
and 6 ghost layers (the lifted stencil reaches 6 fine points)."""
import numpy as np
import pytest

from paper_1912_05371_amd import cases, wacm

from gpu_util import from_pool, log, rel_err, slot_map

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def octree24():
    return cases.random_octree(bs=24, ng=6, target=120, j0=1, jmax=3, seed=21)


def build(orc, c, prec=wacm.F64):
    og = orc.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, c.lev, c.ix, c.iy, c.iz)
    og.set_wavelet(1)
    gg = wacm.Grid.from_case(c, dtype=prec, capacity=9 * c.nb + 64)
    gg.set_wavelet(wacm.CDF44)
    assert gg.get_wavelet() == wacm.CDF44
    return og, gg


def put(gg, og, U):
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


@pytest.mark.parametrize("prec,bs", [("f64", 24), ("f32", 24), ("f64", 32)])
def test_cdf44_sync_matches_oracle(orc, prec, bs):
    c = octree24() if bs == 24 else cases.random_octree(bs=32, ng=6, target=60, j0=1, jmax=3,
                                                         seed=23)
    log(f"CDF 4/4 sync, bs {bs}, {c.nb} blocks, {prec}")
    og, gg = build(orc, c, wacm.F64 if prec == "f64" else wacm.F32)
    U = c.padded()
    pool = put(gg, og, U)
    gg.sync_ghosts(pool)
    Uo = U.copy()
    og.sync(Uo)
    Ug = from_pool(pool, slot_map(gg, og))
    e = float(np.max(np.abs(Ug - Uo)) / np.max(np.abs(Uo)))
    # how many ghost values the lifting changed (so the test covers it)
    U0 = U.copy()
    orc.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, c.lev, c.ix, c.iy, c.iz).sync(U0)
    nl = int(np.sum(np.abs(Uo - U0) > 1e-12))
    log(f"  whole padded arrays rel err {e:.2e}; {nl} values differ from CDF 4/0")
    assert nl > 1000
    assert e < (1e-13 if prec == "f64" else 1e-5)


def test_cdf44_coarsen_pass_matches_oracle(orc):
    c = octree24()
    og, gg = build(orc, c)
    U = c.padded()
    og.sync(U)
    flags_o = (np.asarray(og.lev) == c.jmax).astype(np.int8)  # every finest family
    og2, Uo2 = og.coarsen(flags_o, U)
    pool = put(gg, og, U)
    ai = active_index(gg, og)
    flags_g = np.zeros(og.nb, np.int8)
    flags_g[ai] = flags_o
    nb_new = gg.adapt(wacm.COARSEN, pool, flags_g)
    log(f"CDF 4/4 coarsen: {og.nb} -> {og2.nb} blocks")
    assert og2.nb < og.nb
    assert nb_new == og2.nb and same_leaves(gg, og2)
    Ug = from_pool(pool, slot_map(gg, og2))
    e = rel_err(Ug, Uo2, c.bs, c.ng)
    log(f"  interior rel err {e:.2e}")
    assert e < 1e-13


def test_cdf44_refine_all_matches_oracle(orc):
    c = octree24()
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
    log(f"CDF 4/4 refine_all: {og.nb} -> {og2.nb} blocks, interior rel err {e:.2e}")
    assert e < 1e-13


def test_cdf44_needs_six_ghost_layers_and_guards():
    c = cases.random_octree(bs=24, ng=4, target=40, j0=1, jmax=2, seed=5)
    g = wacm.Grid.from_case(c, dtype=wacm.F64)
    with pytest.raises(wacm.WacmError):
        g.set_wavelet(wacm.CDF44)
    assert g.get_wavelet() == wacm.CDF40
    c6 = octree24()
    g6 = wacm.Grid.from_case(c6, dtype=wacm.F64)
    g6.set_wavelet(wacm.CDF44)
    pool = g6.pool()
    with pytest.raises(wacm.WacmError):
        g6.filter_blocks(pool, -1)
    g6.set_wavelet(wacm.CDF40)
    g6.filter_blocks(pool, -1)


@pytest.mark.parametrize("prec,bs", [("f64", 24), ("f32", 24), ("f64", 32)])
def test_cdf44_rk4_step_matches_oracle(orc, prec, bs):
    """RK4 steps with the lifted ghosts: each step from the oracle's state with
    the oracle's CFL time step (per-step gate), then two free-running steps
    with the device's own CFL step against two oracle steps."""
    c = octree24() if bs == 24 else cases.random_octree(bs=32, ng=6, target=80, j0=1, jmax=3,
                                                         seed=23)
    og, gg = build(orc, c, wacm.F64 if prec == "f64" else wacm.F32)
    U = c.padded()
    work = gg.work()
    t = 0.0
    worst = 0.0
    for n in range(2):
        dt = og.dt(c.params, U)
        Uin = U.astype(np.float32).astype(np.float64) if prec == "f32" else U
        pool = put(gg, og, Uin)
        t_dev = torch.tensor([t], dtype=torch.float64, device="cuda")
        dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
        gg.rk4_step(c.params, t_dev, dt_dev, pool, work, dt_mode=wacm.DT_FIXED)
        og.rk4_step(c.params, t, dt, U)
        torch.cuda.synchronize()
        e = rel_err(from_pool(pool, slot_map(gg, og)), U, c.bs, c.ng)
        worst = max(worst, e)
        t += dt
        assert abs(float(t_dev.item()) - t) <= 1e-15 * t
    log(f"CDF 4/4 RK4 {prec} bs {bs} ({c.nb} blocks): worst per-step rel err {worst:.2e}")
    assert worst < (1e-12 if prec == "f64" else 1e-5)
    if prec == "f64":
        # n steps in one call = n single calls, bitwise; CFL time step on the device
        U0 = c.padded()
        A = put(gg, og, U0)
        B = A.clone()
        ta, dta = (torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(2))
        tb, dtb = (torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(2))
        gg.rk4_steps(c.params, ta, dta, A, work, 2, dt_mode=wacm.DT_CFL)
        # the rhs of this path follows the stage-kernel schedule: tiles of 8
        # rows and the work counters give the same state bitwise
        gg.set_schedule(tile_rows=8, wg_per_cu=2, xcd_map=2, prefetch=1, nontemporal=0)
        for _ in range(2):
            gg.rk4_step(c.params, tb, dtb, B, work, dt_mode=wacm.DT_CFL)
        torch.cuda.synchronize()
        I = slice(c.ng, c.ng + c.bs)
        assert torch.equal(A[..., I, I, I], B[..., I, I, I]) and ta.item() == tb.item()
        Uo = U0.copy()
        to = 0.0
        for _ in range(2):
            dto = og.dt(c.params, Uo)
            og.rk4_step(c.params, to, dto, Uo)
            to += dto
        e = rel_err(from_pool(A, slot_map(gg, og)), Uo, c.bs, c.ng)
        log(f"  2 free CFL steps: rel err {e:.2e}, t {ta.item():.6e} vs {to:.6e}")
        assert e < 1e-12 and abs(ta.item() - to) <= 1e-12 * to


def test_cdf44_adaptive_driver_matches_oracle(orc):
    """adaptive.adaptive_step on a CDF 4/4 grid (lifted ghosts in every sync,
    lifted parents in every merge, the GPU's own flags) against the oracle's
    adaptive step: same leaves, states to 1e-12, two steps."""
    from paper_1912_05371_amd.adaptive import adaptive_step
    from test_gpu_adapt import adaptive_step_oracle
    c = octree24()
    eps, dealias = 1e-2, True
    og, gg = build(orc, c)
    gg.close()
    gg = wacm.Grid.from_case(c, dtype=wacm.F64, capacity=12 * c.nb + 64)
    gg.set_wavelet(wacm.CDF44)
    U = c.padded()
    pool = put(gg, og, U)
    work = gg.work()
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = 0.0
    for step in range(2):
        og, U, dt, passes = adaptive_step_oracle(og, U, c.params, t, eps, dealias)
        t += dt
        merged = adaptive_step(gg, c.params, pool, work, t_dev, dt_dev, eps, dealias)[
            "merged_passes"]
        assert same_leaves(gg, og)
        e = rel_err(from_pool(pool, slot_map(gg, og)), U, c.bs, c.ng)
        log(f"CDF 4/4 adaptive step {step}: {og.nb} blocks, {merged} merging passes "
            f"(oracle {len(passes)}), state rel err {e:.2e}")
        assert merged == len(passes) and merged > 0
        assert e < 1e-12
        assert abs(float(t_dev.item()) - t) <= 1e-12 * t


def test_cdf44_uniform_grid_is_cdf40(orc):
    """No ghost point has a finer owner on a uniform grid: the lifted phase has
    no work and the sync equals the CDF 4/0 one bitwise."""
    c = cases.random_octree(bs=24, ng=6, target=8, j0=1, jmax=1, seed=2)
    assert c.nb == 8
    g = wacm.Grid.from_case(c, dtype=wacm.F64)
    U = c.padded()
    A = g.pool()
    A[: c.nb].copy_(torch.from_numpy(U))
    B = A.clone()
    g.sync_ghosts(A)
    g.set_wavelet(wacm.CDF44)
    g.sync_ghosts(B)
    torch.cuda.synchronize()
    assert torch.equal(A, B)


@pytest.mark.parametrize("prec", [wacm.F64, wacm.F32])
def test_cdf44_rk4_graph_replay_matches_eager(prec):
    """The lifted step keeps t and dt on the device and launches no copy,
    memset or synchronisation: a captured wacm_rk4_step (CFL time step)
    replayed three times, with eager work and synchronisation between the
    replays, equals eager steps from the same states bitwise."""
    c = cases.random_octree(bs=24, ng=6, target=300, j0=2, jmax=4, seed=23)
    g = wacm.Grid.from_case(c, dtype=prec, capacity=c.nb + 8)
    g.set_wavelet(wacm.CDF44)
    log(f"CDF 4/4 graph replay, {c.nb} blocks, dtype {prec}")
    U0 = g.pool()
    U0[:c.nb] = torch.from_numpy(c.padded()).to("cuda", g.torch_dtype())
    pool = U0.clone()
    work = g.work()
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    p = wacm.make_params(c.params)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        g.rk4_step(None, t_dev, dt_dev, pool, work, dt_mode=wacm.DT_CFL, _p=p)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.rk4_step(None, t_dev, dt_dev, pool, work, dt_mode=wacm.DT_CFL, _p=p)
    torch.cuda.synchronize()
    state = U0.clone()
    for rep in range(3):
        ref = state.clone()
        te = torch.zeros(1, dtype=torch.float64, device="cuda")
        de = torch.zeros(1, dtype=torch.float64, device="cuda")
        g.rk4_step(None, te, de, ref, work, dt_mode=wacm.DT_CFL, _p=p)
        torch.cuda.synchronize()
        pool.copy_(state)
        t_dev.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(pool, ref), f"replay {rep} differs from eager"
        assert float(t_dev.item()) == float(te.item()) == float(de.item())
        state = ref
        _ = (state * 2.0).sum().item()
