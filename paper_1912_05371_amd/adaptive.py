"""One adaptive time step of the wavelet-adaptive method (Sec. 3.5) over the
C ABI: refine every block below Jmax, advance one RK4 step on the refined
grid, then coarsen until no family merges -- each pass synchronises the ghost
nodes the details read, thresholds the wavelet details of every block (Sec.
3.1, 3.3-3.4) and merges the flagged sister groups (Sec. 3.5).  All
arithmetic runs in libwacm; this module only sequences the calls and carries
the per-pass flags from the device to the host call of wacm_adapt.
"""
from __future__ import annotations

import time

from . import wacm


def adaptive_step(grid: wacm.Grid, params: dict, U, work, t_dev, dt_dev, eps: float,
                  dealias: bool = True, dt_mode: int = wacm.DT_CFL, timings: dict | None = None,
                  max_passes: int = 64) -> dict:
    """Refine all, one RK4 step (dt from the CFL rule on the refined grid, or
    read from dt_dev), coarsen until no merge.  Returns {"refined": blocks
    after refinement, "merged_passes": coarsening passes that merged blocks,
    "blocks": blocks at the end}.  U and work are the grid's pool and
    work buffer (capacity must hold the refined grid: wacm_adapt raises
    WACM_E_CAPACITY and leaves the grid unchanged otherwise).  With `timings`
    (a dict), each phase is synchronised and its milliseconds accumulated into
    timings[phase] = {"wall", "host", "device"}: for the adaptation calls the
    library's own split (host: leaf lists, merge decisions, tables and their
    upload; device: its kernels), for the others the device time between two
    stream events around the call and the rest of the wall time as host."""
    import torch

    def phase(name, fn, adapt=False):
        if timings is None:
            return fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        if adapt:
            dev = grid.adapt_timing()[1]
        else:
            dev = min(e0.elapsed_time(e1), wall)
        rec = timings.setdefault(name, {"wall": 0.0, "host": 0.0, "device": 0.0})
        rec["wall"] += wall
        rec["device"] += dev
        rec["host"] += wall - dev
        return r

    p = wacm.make_params(params)
    refined = phase("refine_all", lambda: grid.adapt(wacm.REFINE_ALL, U), adapt=True)
    phase("rk4_step", lambda: grid.rk4_step(None, t_dev, dt_dev, U, work, dt_mode=dt_mode, _p=p))
    t = float(t_dev.item())
    merged = 0
    for _ in range(max_passes):
        n = grid.nb
        dmax = torch.empty(n, dtype=torch.float64, device=U.device)
        mrange = torch.empty(n, dtype=torch.float64, device=U.device)
        flags = torch.empty(n, dtype=torch.int8, device=U.device)
        # the thresholding reads only the even lattice's ghosts
        phase("sync_ghosts", lambda: grid.sync_ghosts_lattice(U))
        phase("threshold_blocks",
              lambda: grid.threshold_blocks(params, t, U, eps, dealias, dmax, mrange, flags))
        host_flags = phase("flags_to_host", lambda: flags.cpu().numpy())
        n_new = phase("coarsen", lambda: grid.adapt(wacm.COARSEN, U, host_flags), adapt=True)
        if n_new == n:
            break
        merged += 1
    return {"refined": refined, "merged_passes": merged, "blocks": grid.nb}


def filtered_steps(grid: wacm.Grid, params: dict, U, work, t_dev, dt_dev, nsteps: int,
                   level: int = -1, dt_mode: int = wacm.DT_CFL) -> None:
    """`nsteps` RK4 steps on a fixed grid, each followed by wavelet filtering:
    ghost synchronisation, then the details of the blocks of `level` (every
    block if < 0) are removed (the results section's filtering at the finest
    level, which stabilises equidistant runs).  All arithmetic runs in
    libwacm."""
    p = wacm.make_params(params)
    for _ in range(nsteps):
        grid.rk4_step(None, t_dev, dt_dev, U, work, dt_mode=dt_mode, _p=p)
        grid.sync_ghosts(U)
        grid.filter_blocks(U, level)
