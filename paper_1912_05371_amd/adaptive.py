"""One adaptive time step of the wavelet-adaptive method (Sec. 3.5) over the
C ABI: refine every block below Jmax, advance one RK4 step on the refined
grid, then coarsen until no family merges -- each pass synchronises the ghost
nodes, thresholds the wavelet details of every block (Sec. 3.1, 3.3-3.4) and
merges the flagged sister groups (Sec. 3.5).  All arithmetic runs in libwacm;
this module only sequences the calls and carries the per-pass flags from the
device to the host call of wacm_adapt.
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
    (a dict), host wall milliseconds per phase are accumulated into it, each
    phase synchronised."""
    import torch

    def phase(name, fn):
        if timings is None:
            return fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        timings[name] = timings.get(name, 0.0) + (time.perf_counter() - t0) * 1e3
        return r

    p = wacm.make_params(params)
    refined = phase("refine_all", lambda: grid.adapt(wacm.REFINE_ALL, U))
    phase("rk4_step", lambda: grid.rk4_step(None, t_dev, dt_dev, U, work, dt_mode=dt_mode, _p=p))
    t = float(t_dev.item())
    merged = 0
    for _ in range(max_passes):
        n = grid.nb
        dmax = torch.empty(n, dtype=torch.float64, device=U.device)
        mrange = torch.empty(n, dtype=torch.float64, device=U.device)
        flags = torch.empty(n, dtype=torch.int8, device=U.device)
        phase("sync_ghosts", lambda: grid.sync_ghosts(U))
        phase("threshold_blocks",
              lambda: grid.threshold_blocks(params, t, U, eps, dealias, dmax, mrange, flags))
        host_flags = flags.cpu().numpy()
        n_new = phase("coarsen", lambda: grid.adapt(wacm.COARSEN, U, host_flags))
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
