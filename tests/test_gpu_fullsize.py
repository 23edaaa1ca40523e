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
"""
import numpy as np
import pytest

from paper_1912_05371_amd import cases, inputs, wacm

from gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEED = 12345
BENCH_SCHEDULE = dict(tile_rows=8, wg_per_cu=2, xcd_map=0, prefetch=1, nontemporal=1)


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
    g.set_schedule(**BENCH_SCHEDULE)
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
    g.set_schedule(**BENCH_SCHEDULE)
    A = U0.clone()
    t, dt = scalars()
    g.rk4_steps(c.params, t, dt, A, work, 2, dt_mode=wacm.DT_CFL)
    for sched in (dict(BENCH_SCHEDULE), dict(tile_rows=0, wg_per_cu=0, xcd_map=1, prefetch=0,
                                              nontemporal=0),
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
