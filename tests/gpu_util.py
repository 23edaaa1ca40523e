"""Helpers shared by the GPU parity tests: build the same grid on both sides
and move states between the oracle (numpy, oracle block order = leaf order)
and the HIP pool (torch, pool slot i = leaf i at creation)."""
import sys

import numpy as np

from paper_1912_05371_amd import wacm


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_pair(orc, case, dtype=wacm.F64, capacity=None):
    og = orc.Grid(case.bs, case.ng, case.L, case.jmin, case.jmax, case.lev, case.ix, case.iy,
                  case.iz)
    gg = wacm.Grid.from_case(case, dtype=dtype, capacity=capacity)
    return og, gg


def to_pool(gg, U_np, fill=0.0):
    """numpy (nb,4,P,P,P) float64 -> pool tensor (capacity,...) on the GPU; slot i = block i."""
    import torch
    pool = torch.full((gg.capacity, 4, gg.P, gg.P, gg.P), fill, dtype=gg.torch_dtype(),
                      device="cuda")
    pool[:U_np.shape[0]] = torch.from_numpy(U_np).to(device="cuda", dtype=gg.torch_dtype())
    return pool


def from_pool(pool, slots):
    return pool[slots.tolist()].double().cpu().numpy()


def rel_err(a, b, bs, ng):
    ai = a[..., ng:ng + bs, ng:ng + bs, ng:ng + bs]
    bi = b[..., ng:ng + bs, ng:ng + bs, ng:ng + bs]
    return float(np.max(np.abs(ai - bi)) / max(np.max(np.abs(bi)), 1e-300))


def slot_map(gg, og):
    """For each oracle block, the pool slot holding the same leaf on the GPU side."""
    slots, codes, levels = gg.info()
    key = {(int(l), int(c)): int(s) for s, c, l in zip(slots, codes, levels)}
    out = []
    for b in range(og.nb):
        c = wacm.treecode_encode(og.lev[b], og.ix[b], og.iy[b], og.iz[b])
        out.append(key[(int(og.lev[b]), c)])
    return np.array(out)
