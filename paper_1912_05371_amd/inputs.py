"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module produces leaf sets (levels and block indices of 2:1-balanced
periodic octrees) and initial fields sampled at grid points.  It holds none of
the method's arithmetic (no derivatives, no wavelet prediction, no mask, no
time stepping): only grid geometry, random numbers and closed-form initial
conditions.  Block positions follow the non-redundant reading of the paper's
nested dyadic grids (Sec. 3.1): level J has 2^J blocks per axis and the
interior point i of block b sits at x = (b bs + i) L / (2^J bs).

Leaves are returned in Morton order (level-1 octal digit most significant,
digit = xbit + 2 ybit + 4 zbit, Sec. 4.1), which keeps neighbours close in
memory.
"""
from __future__ import annotations

import math

import numpy as np

REF = 20


def morton_key(lev, ix, iy, iz) -> np.ndarray:
    lev = np.asarray(lev, np.int64)
    ix, iy, iz = (np.asarray(a, np.int64) for a in (ix, iy, iz))
    key = np.zeros(lev.shape, np.uint64)
    for b in range(REF):
        sh = REF - 1 - b  # bit of the coordinate scaled to the reference level
        xs = (ix << (REF - lev)) >> sh & 1
        ys = (iy << (REF - lev)) >> sh & 1
        zs = (iz << (REF - lev)) >> sh & 1
        key = (key << np.uint64(3)) | (xs + 2 * ys + 4 * zs).astype(np.uint64)
    return key


def _sorted(leaves):
    lev = np.array([l[0] for l in leaves], np.int32)
    ix = np.array([l[1] for l in leaves], np.int64)
    iy = np.array([l[2] for l in leaves], np.int64)
    iz = np.array([l[3] for l in leaves], np.int64)
    order = np.argsort(morton_key(lev, ix, iy, iz), kind="stable")
    return lev[order], ix[order], iy[order], iz[order]


def uniform_leaves(J: int):
    n = 1 << J
    return _sorted([(J, x, y, z) for z in range(n) for y in range(n) for x in range(n)])


# --------------------------------------------------------------------------
# Leaf dictionaries with 26-neighbour 2:1 balancing (grid generation only).
# --------------------------------------------------------------------------
class LeafSet:
    """Mutable set of leaves {(lev, x, y, z)} of a periodic octree."""

    def __init__(self, leaves, jmin: int):
        self.s = set((int(a), int(b), int(c), int(d)) for a, b, c, d in leaves)
        self.jmin = jmin

    def leaf_covering(self, J, x, y, z):
        """Leaf of level <= J containing the level-J box (x,y,z) (wrapped), or None."""
        n = 1 << J
        x, y, z = x % n, y % n, z % n
        for K in range(J, self.jmin - 1, -1):
            s = J - K
            key = (K, x >> s, y >> s, z >> s)
            if key in self.s:
                return key
        return None

    def refine(self, leaf, created=None):
        """Split a leaf into 8 children, first refining coarser neighbours.
        New leaves are added to `created` if given."""
        J, x, y, z = leaf
        if leaf not in self.s:
            return
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dx == dy == dz == 0:
                        continue
                    nb = self.leaf_covering(J, x + dx, y + dy, z + dz)
                    if nb is not None and nb[0] < J:
                        self.refine(nb, created)
        self.s.discard(leaf)
        for c in range(8):
            ch = (J + 1, 2 * x + (c & 1), 2 * y + (c >> 1 & 1), 2 * z + (c >> 2 & 1))
            self.s.add(ch)
            if created is not None:
                created.add(ch)

    def arrays(self):
        return _sorted(sorted(self.s))


def random_balanced_leaves(seed: int, j0: int, jmax: int, target: int):
    """Refine random leaves of level < jmax from a uniform level-j0 grid, keeping
    the tree 2:1 balanced over 26 neighbours, until at least `target` leaves.
    Candidates are drawn uniformly from a list of every leaf ever created below
    jmax (leaves that were refined in the meantime are skipped)."""
    rng = np.random.default_rng(seed)
    n0 = 1 << j0
    ls = LeafSet([(j0, x, y, z) for z in range(n0) for y in range(n0) for x in range(n0)], j0)
    cand = sorted(ls.s) if j0 < jmax else []
    while len(ls.s) < target and cand:
        k = int(rng.integers(len(cand)))
        pick = cand[k]
        if pick not in ls.s:
            cand[k] = cand[-1]
            cand.pop()
            continue
        created = set()
        ls.refine(pick, created=created)
        cand[k] = cand[-1]
        cand.pop()
        cand.extend(sorted(l for l in created if l[0] < jmax))
    return ls.arrays()


def ball_leaves(L: float, j0: int, centre, radius: float):
    """Level j0 everywhere, level j0+1 in every level-j0 block meeting the open
    ball |x - centre| < radius."""
    n = 1 << j0
    w = L / n
    leaves = []
    c = np.asarray(centre, float)
    for z in range(n):
        for y in range(n):
            for x in range(n):
                lo = np.array([x, y, z]) * w
                hi = lo + w
                d = np.sqrt(np.sum(np.maximum(0.0, np.maximum(lo - c, c - hi)) ** 2))
                if d < radius:
                    for k in range(8):
                        leaves.append((j0 + 1, 2 * x + (k & 1), 2 * y + (k >> 1 & 1),
                                       2 * z + (k >> 2 & 1)))
                else:
                    leaves.append((j0, x, y, z))
    return _sorted(leaves)


def box_refined_leaves(L: float, jmin: int, jtop: int, lo, hi):
    """Refine every block meeting the axis-aligned box [lo, hi] up to level jtop,
    with 2:1 balancing, starting from a uniform level-jmin grid."""
    n0 = 1 << jmin
    ls = LeafSet([(jmin, x, y, z) for z in range(n0) for y in range(n0) for x in range(n0)],
                 jmin)
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)

    def meets(leaf):
        J, x, y, z = leaf
        w = L / (1 << J)
        blo = np.array([x, y, z]) * w
        return bool(np.all(blo + w >= lo) and np.all(blo <= hi))

    todo = sorted(l for l in ls.s if l[0] < jtop and meets(l))
    while todo:
        nxt = []
        for leaf in todo:
            if leaf in ls.s:
                created = set()
                ls.refine(leaf, created=created)
                nxt.extend(l for l in created if l[0] < jtop and meets(l))
        todo = sorted(set(nxt))
    return ls.arrays()


# --------------------------------------------------------------------------
# Sampling fields at interior points.
# --------------------------------------------------------------------------
def interior_coords(bs: int, L: float, lev, ix, iy, iz):
    """x, y, z of interior points, each of shape (nb, bs, bs, bs) in (z, y, x) order."""
    lev = np.asarray(lev)
    h = L / ((2.0 ** lev) * bs)
    i = np.arange(bs, dtype=np.float64)
    X = ((np.asarray(ix, np.float64)[:, None] * bs + i[None, :]) * h[:, None])
    Y = ((np.asarray(iy, np.float64)[:, None] * bs + i[None, :]) * h[:, None])
    Z = ((np.asarray(iz, np.float64)[:, None] * bs + i[None, :]) * h[:, None])
    nb = len(lev)
    x = np.broadcast_to(X[:, None, None, :], (nb, bs, bs, bs))
    y = np.broadcast_to(Y[:, None, :, None], (nb, bs, bs, bs))
    z = np.broadcast_to(Z[:, :, None, None], (nb, bs, bs, bs))
    return x, y, z


def pack(fields, bs: int, ng: int, fill: float = 0.0) -> np.ndarray:
    """Place 4 interior fields of shape (nb, bs, bs, bs) into a padded pool
    (nb, 4, P, P, P); ghost points get `fill`."""
    nb = fields[0].shape[0]
    P = bs + 2 * ng
    U = np.full((nb, 4, P, P, P), fill, np.float64)
    for c in range(4):
        U[:, c, ng:ng + bs, ng:ng + bs, ng:ng + bs] = fields[c]
    return U


def interior(U: np.ndarray, bs: int, ng: int) -> np.ndarray:
    return U[..., ng:ng + bs, ng:ng + bs, ng:ng + bs]


def taylor_green(x, y, z):
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    p = np.zeros_like(u)
    return [u, v, w, p]


def fourier_modes(seed: int, nfields: int = 4, nmodes: int = 16, kmax: int = 8,
                  amp: float = 1.0 / 16.0, kmin: int = 1) -> np.ndarray:
    """Per field `nmodes` modes (kx, ky, kz, a, phi): integer k with
    kmin <= |k|_inf <= kmax, a ~ amp U(-1,1), phi ~ U(0, 2 pi)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((nfields, nmodes, 5))
    for f in range(nfields):
        m = 0
        while m < nmodes:
            k = rng.integers(-kmax, kmax + 1, size=3)
            if np.max(np.abs(k)) < kmin:
                continue
            out[f, m, :3] = k
            out[f, m, 3] = amp * rng.uniform(-1.0, 1.0)
            out[f, m, 4] = rng.uniform(0.0, 2.0 * math.pi)
            m += 1
    return out


def fourier_eval(modes_f: np.ndarray, x, y, z, L: float):
    """sum_m a_m cos(2 pi/L (k . x) + phi_m) for one field's modes."""
    s = 2.0 * math.pi / L
    out = np.zeros(np.shape(x))
    for kx, ky, kz, a, ph in modes_f:
        out += a * np.cos(s * (kx * x + ky * y + kz * z) + ph)
    return out


def fourier_fields(seed: int, bs: int, L: float, lev, ix, iy, iz, nmodes=16, kmax=8,
                   amp=1.0 / 16.0):
    modes = fourier_modes(seed, 4, nmodes, kmax, amp)
    x, y, z = interior_coords(bs, L, lev, ix, iy, iz)
    return [fourier_eval(modes[c], x, y, z, L) for c in range(4)]


def fourier_fill_device(pool, modes: np.ndarray, bs: int, ng: int, L: float, lev, ix, iy, iz,
                        slots, chunk: int = 512):
    """Fill the interiors of `pool` (a torch tensor (cap, 4, P, P, P) on the GPU)
    with the same sum of cosines as fourier_eval, evaluated in float64 on the
    device block by block (for workloads too large to build on the host)."""
    import torch
    dev = pool.device
    s = 2.0 * math.pi / L
    md = torch.as_tensor(modes, dtype=torch.float64, device=dev)
    i = torch.arange(bs, dtype=torch.float64, device=dev)
    lev_t = torch.as_tensor(np.asarray(lev), dtype=torch.float64, device=dev)
    h_all = L / (torch.pow(2.0, lev_t) * bs)
    ixt = torch.as_tensor(np.asarray(ix), dtype=torch.float64, device=dev)
    iyt = torch.as_tensor(np.asarray(iy), dtype=torch.float64, device=dev)
    izt = torch.as_tensor(np.asarray(iz), dtype=torch.float64, device=dev)
    slots_t = torch.as_tensor(np.asarray(slots), dtype=torch.long, device=dev)
    nb = len(slots)
    for b0 in range(0, nb, chunk):
        b1 = min(nb, b0 + chunk)
        h = h_all[b0:b1, None]
        X = (ixt[b0:b1, None] * bs + i[None, :]) * h
        Y = (iyt[b0:b1, None] * bs + i[None, :]) * h
        Z = (izt[b0:b1, None] * bs + i[None, :]) * h
        n = b1 - b0
        for c in range(md.shape[0]):
            acc = torch.zeros((n, bs, bs, bs), dtype=torch.float64, device=dev)
            for kx, ky, kz, a, ph in md[c].tolist():
                acc += a * torch.cos(s * (kx * X[:, None, None, :] + ky * Y[:, None, :, None]
                                          + kz * Z[:, :, None, None]) + ph)
            pool[slots_t[b0:b1], c, ng:ng + bs, ng:ng + bs, ng:ng + bs] = acc.to(pool.dtype)


# --------------------------------------------------------------------------
# Two dimensions: quadtree leaves (level, ix, iy) of the periodic square
# [0, L)^2, square blocks, the same non-redundant positions.  Leaves are
# ordered like the octree's with iz = 0 (x bit below y bit per level); the
# library takes the treecode of (ix, iy, 0).
# --------------------------------------------------------------------------
def _sorted2(leaves):
    lev = np.array([l[0] for l in leaves], np.int32)
    ix = np.array([l[1] for l in leaves], np.int64)
    iy = np.array([l[2] for l in leaves], np.int64)
    order = np.argsort(morton_key(lev, ix, iy, np.zeros_like(ix)), kind="stable")
    return lev[order], ix[order], iy[order]


def uniform_leaves2(J: int):
    n = 1 << J
    return _sorted2([(J, x, y) for y in range(n) for x in range(n)])


class LeafSet2:
    """Mutable set of quadtree leaves {(lev, x, y)} with 8-neighbour 2:1
    balancing on refinement (grid generation only)."""

    def __init__(self, leaves, jmin: int):
        self.s = set((int(a), int(b), int(c)) for a, b, c in leaves)
        self.jmin = jmin

    def leaf_covering(self, J, x, y):
        n = 1 << J
        x, y = x % n, y % n
        for K in range(J, self.jmin - 1, -1):
            key = (K, x >> (J - K), y >> (J - K))
            if key in self.s:
                return key
        return None

    def refine(self, leaf, created=None):
        J, x, y = leaf
        if leaf not in self.s:
            return
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == dy == 0:
                    continue
                nb = self.leaf_covering(J, x + dx, y + dy)
                if nb is not None and nb[0] < J:
                    self.refine(nb, created)
        self.s.discard(leaf)
        for c in range(4):
            ch = (J + 1, 2 * x + (c & 1), 2 * y + (c >> 1))
            self.s.add(ch)
            if created is not None:
                created.add(ch)

    def arrays(self):
        return _sorted2(sorted(self.s))


def random_balanced_leaves2(seed: int, j0: int, jmax: int, target: int):
    """Random 2:1-balanced quadtree: refine uniformly drawn leaves below jmax
    of a uniform level-j0 grid until at least `target` leaves."""
    rng = np.random.default_rng(seed)
    n0 = 1 << j0
    ls = LeafSet2([(j0, x, y) for y in range(n0) for x in range(n0)], j0)
    cand = sorted(ls.s) if j0 < jmax else []
    while len(ls.s) < target and cand:
        k = int(rng.integers(len(cand)))
        pick = cand[k]
        cand[k] = cand[-1]
        cand.pop()
        if pick not in ls.s:
            continue
        created = set()
        ls.refine(pick, created=created)
        cand.extend(sorted(l for l in created if l[0] < jmax))
    return ls.arrays()


def disc_refined_leaves2(L: float, jmin: int, jtop: int, centres, radius: float):
    """Every block meeting one of the discs |x - c| < radius (periodic) is
    refined up to level jtop, with 2:1 balancing, from a uniform level-jmin
    grid (geometry only)."""
    n0 = 1 << jmin
    ls = LeafSet2([(jmin, x, y) for y in range(n0) for x in range(n0)], jmin)
    cs = np.asarray(centres, float)

    def meets(leaf):
        J, x, y = leaf
        w = L / (1 << J)
        lo = np.array([x, y]) * w
        for c in cs:
            for sx in (-L, 0.0, L):
                for sy in (-L, 0.0, L):
                    cc = c + np.array([sx, sy])
                    d = np.sqrt(np.sum(np.maximum(0.0, np.maximum(lo - cc, cc - lo - w)) ** 2))
                    if d < radius:
                        return True
        return False

    todo = sorted(l for l in ls.s if l[0] < jtop and meets(l))
    while todo:
        nxt = []
        for leaf in todo:
            if leaf in ls.s:
                created = set()
                ls.refine(leaf, created=created)
                nxt.extend(l for l in created if l[0] < jtop and meets(l))
        todo = sorted(set(nxt))
    return ls.arrays()


# the three Gaussian vortices of the results section (periodic [0, 2 pi)^2):
# circulations, centres, core size a = 1/pi
THREE_VORTICES = dict(gamma=(1.0, 1.0, -0.5),
                      centres=((0.75 * math.pi, math.pi), (1.25 * math.pi, math.pi),
                               (1.25 * math.pi, 1.25 * math.pi)),
                      a=1.0 / math.pi)


def three_vortex_vorticity(N: int, L: float = 2.0 * math.pi, images: int = 2):
    """omega = sum_i Gamma_i / (pi a^2) exp(-|x - x_i|^2 / a^2) on the N x N
    lattice (array [y, x]), with periodic images of each Gaussian."""
    tv = THREE_VORTICES
    a = tv["a"]
    x = np.arange(N) * (L / N)
    X, Y = x[None, :], x[:, None]
    w = np.zeros((N, N))
    for g, (cx, cy) in zip(tv["gamma"], tv["centres"]):
        for sx in range(-images, images + 1):
            for sy in range(-images, images + 1):
                r2 = (X - cx - sx * L) ** 2 + (Y - cy - sy * L) ** 2
                w += g / (math.pi * a * a) * np.exp(-r2 / (a * a))
    return w


def three_vortex_velocity(N: int, L: float = 2.0 * math.pi):
    """Initial velocity of the three vortices on the N x N lattice (arrays
    [y, x]): the periodic field whose vorticity dv/dx - du/dy is omega minus
    its mean (a periodic velocity carries no net circulation), built from the
    streamfunction psi with -lap psi = omega - mean, u = dpsi/dy, v = -dpsi/dx,
    evaluated by FFT.  This only constructs the initial condition; the method
    itself differentiates with finite differences."""
    w = three_vortex_vorticity(N, L)
    k = np.fft.fftfreq(N, d=L / N) * 2.0 * math.pi
    KX, KY = k[None, :], k[:, None]
    k2 = KX ** 2 + KY ** 2
    wh = np.fft.fft2(w)
    k2[0, 0] = 1.0
    ph = wh / k2
    ph[0, 0] = 0.0
    u = np.real(np.fft.ifft2(1j * KY * ph))
    v = np.real(np.fft.ifft2(-1j * KX * ph))
    return u, v


def sample2(field: np.ndarray, bs: int, lev, ix, iy) -> np.ndarray:
    """Values of a lattice field (N x N, array [y, x], N = 2^J bs for some J
    at least every level) at the interior points of each block: (nb, bs, bs)
    in (y, x) order."""
    N = field.shape[0]
    out = np.zeros((len(lev), bs, bs))
    i = np.arange(bs)
    for b, (J, x, y) in enumerate(zip(lev, ix, iy)):
        st = N // ((1 << int(J)) * bs)
        assert st * (1 << int(J)) * bs == N
        gx = (int(x) * bs + i) * st
        gy = (int(y) * bs + i) * st
        out[b] = field[np.ix_(gy, gx)]
    return out


def pack2(fields, bs: int, ng: int, fill: float = 0.0) -> np.ndarray:
    """3 interior fields (nb, bs, bs) into a padded 2D pool (nb, 3, P, P)."""
    nb = fields[0].shape[0]
    P = bs + 2 * ng
    U = np.full((nb, 3, P, P), fill, np.float64)
    for c in range(3):
        U[:, c, ng:ng + bs, ng:ng + bs] = fields[c]
    return U


def interior2(U: np.ndarray, bs: int, ng: int) -> np.ndarray:
    return U[..., ng:ng + bs, ng:ng + bs]
