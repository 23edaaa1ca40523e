"""The benchmark workload at its full size -- a seeded random 2:1-balanced
periodic octree of 20028 blocks of 24^3 points (levels 3-7), 4 ghost layers,
random-Fourier velocity and pressure -- in the launch configuration bench.py
times (one wacm_rk4_steps call, tiles of 8 rows, CFL time step on the
device).  The oracle needs minutes and ~100 GB of host memory for one step
at this size, so these checks use properties that hold at any size:

- the fast path (face-halo kernel + fused stage kernel, x-split registers,
  U^n recovered in stage 2, CFL maximum fused into stage 4, state kept in a
  register between the steps of a call) against classical RK4 assembled in
  torch from the ABI's own wacm_sync_ghosts and wacm_rhs_acm (which are
  pinned to the oracle at small sizes): 1e-12 relative over interiors, FP64;
- n steps in one call = n single-step calls, bitwise;
- every stage-kernel schedule gives the same state, bitwise;
- the FP32 path against the FP64 one after one step: 1e-5 relative.

Each runs the schedules bench.py times: the ones shipped for this workload
in tuned_schedules.json (FP64 and FP32).  A C4-shaped octree small enough
for the oracle (3011 blocks of 24^3, levels 3-7 with uneven counts) is
compared with the oracle directly under those schedules.
"""
import json
import os

import numpy as np
import pytest

from paper_1912_05371_amd import autotune, cases, inputs, wacm

from gpu_util import log, rel_err, to_pool

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEED = 12345
OTHER_SCHEDULE = dict(tile_rows=8, wg_per_cu=2, xcd_map=0, prefetch=1, nontemporal=1)


def shipped(dtype_name):
    """The schedule shipped for the benchmark workload (the one bench.py's
    tuner loads), matched on everything but the device name."""
    with open(autotune.SHIPPED) as f:
        data = json.load(f)
    tail = f"|{dtype_name}|bs24|ng4|nb20028|"
    hits = [v["schedule"] for k, v in data.items() if tail in k]
    assert len(hits) == 1, f"no shipped {dtype_name} schedule for the benchmark workload"
    return dict(hits[0])


@pytest.fixture(scope="module")
def full():
    c = cases.random_octree(bs=24, ng=4, target=20000, j0=3, jmax=7, seed=SEED,
                            with_fields=False)
    log(f"full-size octree: {c.nb} blocks")
    return c


def filled(g, c):
    pool = g.pool()
    modes = inputs.fourier_modes(SEED, 4, 16, 8, 1.0 / 16.0)
    inputs.fourier_fill_device(pool, modes, c.bs, c.ng, c.L, c.lev, c.ix, c.iy, c.iz,
                               np.arange(c.nb))
    return pool


def interior(U, c):
    g = c.ng
    return U[:c.nb, :, g:g + c.bs, g:g + c.bs, g:g + c.bs]


def rel(a, b, c):
    ai, bi = interior(a, c), interior(b, c)
    return float((ai - bi).abs().max() / bi.abs().max())


def scalars():
    return (torch.zeros(1, dtype=torch.float64, device="cuda"),
            torch.zeros(1, dtype=torch.float64, device="cuda"))


def test_fullsize_fast_path_matches_assembled_rk4(full):
    c = full
    g = wacm.Grid.from_case(c, dtype=wacm.F64)
    sched = shipped("f64")
    g.set_schedule(**sched)
    got = g.get_schedule()
    assert {k: got[k] for k in sched} == sched
    U0 = filled(g, c)
    A = U0.clone()
    work = g.work()
    t, dt = scalars()
    g.rk4_steps(c.params, t, dt, A, work, 2, dt_mode=wacm.DT_CFL)
    torch.cuda.synchronize()
    del work
    torch.cuda.empty_cache()
    # classical RK4 from the ABI's stand-alone sync and rhs
    B = U0.clone()
    del U0
    Y = torch.empty_like(B)
    K = torch.empty_like(B)
    acc = torch.empty_like(B)
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    tt = 0.0
    for _ in range(2):
        g.compute_dt(c.params, B, dtd)
        h = float(dtd.item())
        Y.copy_(B)
        g.sync_ghosts(Y)
        g.rhs_acm(c.params, tt, Y, K)
        torch.add(B, K, alpha=h / 6, out=acc)
        torch.add(B, K, alpha=h / 2, out=Y)
        g.sync_ghosts(Y)
        g.rhs_acm(c.params, tt + h / 2, Y, K)
        acc.add_(K, alpha=h / 3)
        torch.add(B, K, alpha=h / 2, out=Y)
        g.sync_ghosts(Y)
        g.rhs_acm(c.params, tt + h / 2, Y, K)
        acc.add_(K, alpha=h / 3)
        torch.add(B, K, alpha=h, out=Y)
        g.sync_ghosts(Y)
        g.rhs_acm(c.params, tt + h, Y, K)
        torch.add(acc, K, alpha=h / 6, out=B)
        tt += h
    torch.cuda.synchronize()
    e = rel(A, B, c)
    log(f"  2 steps: fast path vs assembled RK4 rel err {e:.2e}; t {t.item():.6e} vs {tt:.6e}")
    assert e < 1e-12
    assert abs(t.item() - tt) <= 1e-12 * tt


def test_fullsize_multi_step_call_and_schedules_bitwise(full):
    c = full
    g = wacm.Grid.from_case(c, dtype=wacm.F64)
    U0 = filled(g, c)
    work = g.work()
    g.set_schedule(**shipped("f64"))
    A = U0.clone()
    t, dt = scalars()
    g.rk4_steps(c.params, t, dt, A, work, 2, dt_mode=wacm.DT_CFL)
    for sched in (shipped("f64"), shipped("f32"), dict(OTHER_SCHEDULE),
                  dict(tile_rows=0, wg_per_cu=0, xcd_map=1, prefetch=0, nontemporal=0),
                  dict(tile_rows=8, wg_per_cu=0, xcd_map=2, prefetch=0, nontemporal=1)):
        g.set_schedule(**sched)
        B = U0.clone()
        t2, dt2 = scalars()
        for _ in range(2):
            g.rk4_step(c.params, t2, dt2, B, work, dt_mode=wacm.DT_CFL)
        torch.cuda.synchronize()
        same = torch.equal(interior(A, c), interior(B, c))
        log(f"  schedule {sched}: 2 single steps == one 2-step call: {same}")
        assert same and t.item() == t2.item() and dt.item() == dt2.item()
        del B


def test_fullsize_fp32_against_fp64(full):
    c = full
    g64 = wacm.Grid.from_case(c, dtype=wacm.F64)
    g32 = wacm.Grid.from_case(c, dtype=wacm.F32)
    g64.set_schedule(**shipped("f64"))
    g32.set_schedule(**shipped("f32"))
    U64 = filled(g64, c)
    U32 = U64.float()
    w64 = g64.work()
    t, dt = scalars()
    g64.rk4_steps(c.params, t, dt, U64, w64, 1, dt_mode=wacm.DT_CFL)
    torch.cuda.synchronize()
    del w64
    torch.cuda.empty_cache()
    w32 = g32.work()
    t3, dt3 = scalars()
    g32.rk4_steps(c.params, t3, dt3, U32, w32, 1, dt_mode=wacm.DT_CFL)
    torch.cuda.synchronize()
    e = rel(U32.double(), U64, c)
    log(f"  one step FP32 vs FP64: rel err {e:.2e}; dt {dt3.item():.9e} vs {dt.item():.9e}")
    assert e < 1e-5
    assert abs(dt3.item() - dt.item()) <= 1e-6 * dt.item()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_c4_shaped_octree_matches_oracle(orc, prec):
    """3011 blocks of 24^3 (levels 3..7: 295, 1631, 809, 244, 32), the
    benchmark's field recipe, one CFL step with the shipped schedule of the
    precision, against the oracle's step from the same input: 1e-12 (FP64)
    or 1e-5 (FP32, input rounded to FP32) relative over interiors, and the
    same time step."""
    c = cases.random_octree(bs=24, ng=4, target=3000, j0=3, jmax=7, seed=7)
    levels = np.bincount(c.lev, minlength=8)[3:8].tolist()
    log(f"c4-shaped octree {prec}: {c.nb} blocks, levels 3..7 {levels}")
    assert c.nb == 3011 and min(levels) > 0
    og = orc.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, c.lev, c.ix, c.iy, c.iz)
    U = c.padded()
    if prec == "f32":
        U = U.astype(np.float32).astype(np.float64)
    dto = og.dt(c.params, U)
    Uo = U.copy()
    og.rk4_step(c.params, 0.0, dto, Uo)
    g = wacm.Grid.from_case(c, dtype=wacm.F64 if prec == "f64" else wacm.F32)
    g.set_schedule(**shipped(prec))
    pool = to_pool(g, U)
    work = g.work()
    t, dt = scalars()
    g.rk4_steps(c.params, t, dt, pool, work, 1, dt_mode=wacm.DT_CFL)
    torch.cuda.synchronize()
    Ug = pool[:c.nb].double().cpu().numpy()
    e = rel_err(Ug, Uo, c.bs, c.ng)
    tol = 1e-12 if prec == "f64" else 1e-5
    log(f"  one step vs oracle: rel err {e:.2e} (tol {tol:g}); dt {dt.item():.9e} vs {dto:.9e}")
    assert e < tol
    assert abs(dt.item() - dto) <= (1e-14 if prec == "f64" else 1e-6) * dto
