"""Workload definitions: grids, parameters and initial fields.

Each case names its sizes and the physical parameters of the penalized
artificial-compressibility model (Sec. 2.1-2.2).  Parameters are plain dicts
with the keys of the C parameter struct; both the HIP binding and the oracle
consume them.

Cases (all synthetic, seed 12345):

* ``taylor_green``  -- [0,2pi]^3 periodic, uniform level 2 (64 blocks, bs 16,
  ng 4), Taylor-Green velocity, nu 1e-2, C0 10, C_gamma 1, no mask, CFL 0.5.
* ``sphere_two_level`` -- [0,4]^3, level 3 with level 4 in every level-3 block
  meeting the ball |x-(1,2,2)| < 0.6 (736 blocks), sphere R 0.25 smoothed over
  1.5 h_4, C_eta 1e-3, binary sponge 0.5 on all faces, C_sp = L_sp/(C0 tau),
  tau 20, u_inf (1,0,0), nu 1e-2, C0 20, C_gamma 0, uniform inflow start.
* ``plate_adaptive`` -- [0,4]^3, levels 2..6, bs 16, eps 1e-3, dealiasing,
  rotating plate 1.0 x 0.25 x 0.02 about its leading edge at (2,2,2) with
  alpha = 0.8 sin(2 pi t); C_eta 1e-3, nu 2e-3, C0 20, C_gamma 1; smooth seeded
  velocity noise of amplitude 1e-3.
* ``random_octree`` -- [0,2pi]^3, bs 24, ng 4, seeded random 2:1 octree,
  levels 3..7, >= 20000 blocks; 16 random Fourier modes per field (k <= 8);
  nu 1e-2, C0 20, C_gamma 1, no mask, CFL 0.5.  Throughput workload.
* ``plate_adjoint`` -- the plate on a frozen grid, levels 2..5, bs 16.
* ``three_vortices`` (two dimensions) -- [0, 2pi)^2 periodic, three Gaussian
  vortices (circulations 1, 1, -1/2, core 1/pi, centres (0.75, 1) pi,
  (1.25, 1) pi, (1.25, 1.25) pi), nu 5e-5, C0 10, C_gamma 1, p = 0; on a
  uniform level (equidistant runs) or on a quadtree refined around the
  vortex cores (adaptive runs).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import inputs

SEED = 12345

BASE_PARAMS = dict(
    nu=1e-2, c0=10.0, c_gamma=1.0, c_eta=1e-3, c_sp=1.0, l_sp=0.0, u_inf=(0.0, 0.0, 0.0),
    p_inf=0.0, mask=0, sponge=0, clip=0, w=1.0, sph_c=(0.0, 0.0, 0.0), sph_r=0.0,
    x_le=(0.0, 0.0, 0.0), lo=(0.0, 0.0, 0.0), hi=(0.0, 0.0, 0.0), amp=0.0, freq=0.0, phase=0.0,
    cfl=0.5, cfl_eta=1.0, cfl_nu=0.25,
)


def params(**kw) -> dict:
    p = dict(BASE_PARAMS)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(k)
        p[k] = v
    return p


@dataclass
class Case:
    name: str
    bs: int
    ng: int
    L: float
    jmin: int
    jmax: int
    lev: np.ndarray
    ix: np.ndarray
    iy: np.ndarray
    iz: np.ndarray
    params: dict
    fields: list = field(default_factory=list)  # 4 arrays (nb, bs, bs, bs)
    steps: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def nb(self) -> int:
        return len(self.lev)

    @property
    def P(self) -> int:
        return self.bs + 2 * self.ng

    def padded(self, fill: float = 0.0) -> np.ndarray:
        return inputs.pack(self.fields, self.bs, self.ng, fill)

    def coords(self):
        return inputs.interior_coords(self.bs, self.L, self.lev, self.ix, self.iy, self.iz)


def taylor_green(bs: int = 16, ng: int = 4, J: int = 2) -> Case:
    L = 2.0 * math.pi
    lev, ix, iy, iz = inputs.uniform_leaves(J)
    x, y, z = inputs.interior_coords(bs, L, lev, ix, iy, iz)
    prm = params(nu=1e-2, c0=10.0, c_gamma=1.0, cfl=0.5)
    return Case("taylor_green", bs, ng, L, J, J, lev, ix, iy, iz, prm,
                inputs.taylor_green(x, y, z), steps=10)


def sphere_two_level(bs: int = 16, ng: int = 4) -> Case:
    L = 4.0
    lev, ix, iy, iz = inputs.ball_leaves(L, 3, (1.0, 2.0, 2.0), 0.6)
    h4 = L / (16 * bs)
    c0, l_sp, tau = 20.0, 0.5, 20.0
    prm = params(nu=1e-2, c0=c0, c_gamma=0.0, c_eta=1e-3, mask=1, w=1.5 * h4,
                 sph_c=(1.0, 2.0, 2.0), sph_r=0.25, sponge=1, l_sp=l_sp,
                 c_sp=l_sp / (c0 * tau), u_inf=(1.0, 0.0, 0.0), p_inf=0.0, cfl=0.5)
    nb = len(lev)
    one = np.ones((nb, bs, bs, bs))
    zero = np.zeros((nb, bs, bs, bs))
    return Case("sphere_two_level", bs, ng, L, 3, 4, lev, ix, iy, iz, prm,
                [one, zero.copy(), zero.copy(), zero.copy()], steps=20)


def plate_params(jmax: int, bs: int = 16, L: float = 4.0, clip: int = 1) -> dict:
    hmax = L / ((1 << jmax) * bs)
    return params(nu=2e-3, c0=20.0, c_gamma=1.0, c_eta=1e-3, mask=2, clip=clip, w=1.5 * hmax,
                  x_le=(2.0, 2.0, 2.0), lo=(0.0, -0.5, -0.01), hi=(0.25, 0.5, 0.01),
                  amp=0.8, freq=1.0, phase=0.0, cfl=0.5)


def plate_grid(L: float, jmin: int, jtop: int):
    # every block meeting the sphere of radius 0.3 around the plate's swept
    # region (leading edge at (2,2,2), chord 0.25 rotating by up to 0.8 rad)
    # is refined to jtop; a box bound of that region is used.
    lo = (2.0 - 0.3, 2.0 - 0.55, 2.0 - 0.3)
    hi = (2.0 + 0.3, 2.0 + 0.55, 2.0 + 0.3)
    return inputs.box_refined_leaves(L, jmin, jtop, lo, hi)


def smooth_noise(seed: int, bs, L, lev, ix, iy, iz, amp=1e-3, kmax=4):
    modes = inputs.fourier_modes(seed, 4, 16, kmax, 1.0)
    x, y, z = inputs.interior_coords(bs, L, lev, ix, iy, iz)
    out = []
    for c in range(4):
        f = inputs.fourier_eval(modes[c], x, y, z, L)
        m = np.max(np.abs(f)) if f.size else 1.0
        out.append(amp * f / (m if m > 0 else 1.0))
    return out


def plate_adaptive(bs: int = 16, ng: int = 4, jmin: int = 2, jmax: int = 6,
                   jstart: int | None = None) -> Case:
    L = 4.0
    jtop = jmax - 1 if jstart is None else jstart
    lev, ix, iy, iz = plate_grid(L, jmin, jtop)
    prm = plate_params(jmax, bs, L, clip=1)
    noise = smooth_noise(SEED, bs, L, lev, ix, iy, iz)
    noise[3] = np.zeros_like(noise[3])
    return Case("plate_adaptive", bs, ng, L, jmin, jmax, lev, ix, iy, iz, prm, noise,
                steps=200, extra=dict(eps=1e-3, dealias=True))


def random_octree(bs: int = 24, ng: int = 4, target: int = 20000, j0: int = 3, jmax: int = 7,
                  seed: int = SEED, with_fields: bool = True) -> Case:
    L = 2.0 * math.pi
    lev, ix, iy, iz = inputs.random_balanced_leaves(seed, j0, jmax, target)
    prm = params(nu=1e-2, c0=20.0, c_gamma=1.0, cfl=0.5)
    flds = inputs.fourier_fields(seed, bs, L, lev, ix, iy, iz) if with_fields else []
    return Case("random_octree", bs, ng, L, j0, jmax, lev, ix, iy, iz, prm, flds, steps=50)


def plate_adjoint(bs: int = 16, ng: int = 4) -> Case:
    L = 4.0
    lev, ix, iy, iz = plate_grid(L, 2, 5)
    prm = plate_params(5, bs, L, clip=0)
    noise = smooth_noise(SEED, bs, L, lev, ix, iy, iz)
    noise[3] = np.zeros_like(noise[3])
    return Case("plate_adjoint", bs, ng, L, 2, 5, lev, ix, iy, iz, prm, noise, steps=100)


@dataclass
class Case2:
    """A two-dimensional case: quadtree leaves and 3 interior fields (u, v, p)
    of shape (nb, bs, bs)."""
    name: str
    bs: int
    ng: int
    L: float
    jmin: int
    jmax: int
    lev: np.ndarray
    ix: np.ndarray
    iy: np.ndarray
    params: dict
    fields: list = field(default_factory=list)
    steps: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def nb(self) -> int:
        return len(self.lev)

    @property
    def P(self) -> int:
        return self.bs + 2 * self.ng

    def padded(self, fill: float = 0.0) -> np.ndarray:
        return inputs.pack2(self.fields, self.bs, self.ng, fill)


def three_vortex_params() -> dict:
    return params(nu=5e-5, c0=10.0, c_gamma=1.0, cfl=0.5)


def _three_vortex_fields(bs, lev, ix, iy, jtop):
    N = (1 << jtop) * bs
    u, v = inputs.three_vortex_velocity(N)
    return [inputs.sample2(u, bs, lev, ix, iy), inputs.sample2(v, bs, lev, ix, iy),
            np.zeros((len(lev), bs, bs))]


def three_vortices(bs: int = 16, ng: int = 4, J: int = 4) -> Case2:
    """Equidistant: uniform level J ((2^J bs)^2 points)."""
    lev, ix, iy = inputs.uniform_leaves2(J)
    return Case2("three_vortices", bs, ng, 2.0 * math.pi, J, J, lev, ix, iy,
                 three_vortex_params(), _three_vortex_fields(bs, lev, ix, iy, J), steps=10)


def three_vortices_adaptive(bs: int = 16, ng: int = 4, jmin: int = 2, jmax: int = 6,
                            jstart: int | None = None, radius: float = 1.0) -> Case2:
    """Adaptive: every block within `radius` of a vortex centre refined to
    jstart (default jmax - 1), 2:1 balanced; eps 1e-3, dealiasing."""
    jtop = jmax - 1 if jstart is None else jstart
    lev, ix, iy = inputs.disc_refined_leaves2(2.0 * math.pi, jmin, jtop,
                                              inputs.THREE_VORTICES["centres"], radius)
    return Case2("three_vortices_adaptive", bs, ng, 2.0 * math.pi, jmin, jmax, lev, ix, iy,
                 three_vortex_params(), _three_vortex_fields(bs, lev, ix, iy, jmax), steps=20,
                 extra=dict(eps=1e-3, dealias=True))
