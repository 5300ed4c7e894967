"""Synthetic fault meshes and seeded inputs.

Every workload is a structured mesh standing in for the paper's fault
models (section 4.1 uses a half-space nonplanar thrust fault meshed with
about 1e5 rectangles; its mesh files are not public).  The meshes here are
planar grids of equal squares; element order is row-major along strike
(k = iy * nx + ix), with iy counting down dip.

Conventions shared by both sides of the code:

* vertices are listed counter-clockwise seen from the +normal side,
  which for these grids points to the hanging-wall (upper) side;
* ``slip_dir`` is a unit vector in the fault plane: +strike for
  strike-slip, up-dip for thrust (hanging wall moving up).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MU = 32.0e9          # rigidity [Pa]
NU = 0.25            # Poisson ratio
CS = 3464.0          # S-wave speed [m/s]
V_PL = 1.0e-9        # plate rate [m/s]
V0 = 1.0e-6          # reference slip rate [m/s]
F0 = 0.6             # reference friction coefficient


@dataclass
class PlanarRectFault:
    nx: int                      # elements along strike
    ny: int                      # elements down dip
    h: float                     # element side [m]
    dip_deg: float               # dip angle [deg]
    slip: str                    # "strike" or "dip"
    verts: np.ndarray = field(repr=False)     # (N, 4, 3) float64
    slip_dir: np.ndarray = field(repr=False)  # (N, 3) float64
    ix: np.ndarray = field(repr=False)        # (N,) strike index
    iy: np.ndarray = field(repr=False)        # (N,) down-dip index

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def strike_vec(self) -> np.ndarray:
        return np.array([1.0, 0.0, 0.0])

    @property
    def downdip_vec(self) -> np.ndarray:
        c, s = _cos_sin_deg(self.dip_deg)
        return np.array([0.0, c, -s])


def _cos_sin_deg(deg: float):
    if deg == 90.0:
        return 0.0, 1.0
    r = np.deg2rad(deg)
    return float(np.cos(r)), float(np.sin(r))


def planar_rect_fault(nx: int, ny: int, h: float, dip_deg: float, slip: str) -> PlanarRectFault:
    """Grid of nx x ny squares of side h on a plane dipping ``dip_deg``.

    The top edge lies along the x axis through the origin; the plane goes
    down dip along (0, cos(dip), -sin(dip)).
    """
    if slip not in ("strike", "dip"):
        raise ValueError("slip must be 'strike' or 'dip'")
    c, s = _cos_sin_deg(dip_deg)
    iy, ix = np.divmod(np.arange(nx * ny, dtype=np.int64), nx)
    x0 = ix * h
    x1 = (ix + 1) * h
    d0 = iy * h
    d1 = (iy + 1) * h
    verts = np.empty((nx * ny, 4, 3), dtype=np.float64)
    for k, (xa, da) in enumerate(((x0, d0), (x1, d0), (x1, d1), (x0, d1))):
        verts[:, k, 0] = xa
        verts[:, k, 1] = da * c
        verts[:, k, 2] = -da * s
    if slip == "strike":
        sd = np.array([1.0, 0.0, 0.0])
    else:
        sd = np.array([0.0, -c, s])          # up-dip: thrust
    slip_dir = np.tile(sd, (nx * ny, 1))
    return PlanarRectFault(nx, ny, h, dip_deg, slip, verts, slip_dir, ix, iy)


# name -> (mesh args, H-matrix options, x seed)
WORKLOADS = {
    # planar vertical strike-slip fault, 64 x 32 squares of 100 m
    "planar64x32": dict(mesh=(64, 32, 100.0, 90.0, "strike"),
                        aca_eps=1e-6, leaf=32, eta=2.0, lattice=1, seed=0),
    # planar 30-degree dipping thrust, 480 x 256 squares of 50 m
    "dip30_480x256": dict(mesh=(480, 256, 50.0, 30.0, "dip"),
                          aca_eps=1e-5, leaf=64, eta=2.0, lattice=32, seed=2),
    # small lattice cases used by the parity tests (several lattice tiles,
    # ragged leaf sizes)
    "dip30_48x24": dict(mesh=(48, 24, 100.0, 30.0, "dip"),
                        aca_eps=1e-6, leaf=16, eta=2.0, lattice=4, seed=11),
    "dip30_150x70": dict(mesh=(150, 70, 100.0, 30.0, "dip"),
                         aca_eps=1e-6, leaf=32, eta=2.0, lattice=8, seed=12),
    "strike_37x23": dict(mesh=(37, 23, 100.0, 90.0, "strike"),
                         aca_eps=1e-5, leaf=20, eta=2.0, lattice=2, seed=13),
    # ensemble workload: N = 21000 (size of the paper-scale nonplanar mesh
    # used for many-member runs), planar stand-in, 64 members
    "dip30_150x140": dict(mesh=(150, 140, 100.0, 30.0, "dip"),
                          aca_eps=1e-6, leaf=32, eta=2.0, lattice=8, seed=3),
}


def config_fault(name: str) -> PlanarRectFault:
    return planar_rect_fault(*WORKLOADS[name]["mesh"])


def loguniform_rates(n: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Slip rates 10**(-12 + 3u), u ~ U[0, 1), from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    if nrhs is None:
        u = rng.random(n)
    else:
        u = rng.random((n, nrhs))
    return 10.0 ** (-12.0 + 3.0 * u)


def friction_params(f: PlanarRectFault) -> dict:
    """Rate-and-state parameters of the planar workloads.

    a = 0.010 everywhere; b = 0.015 inside the central 60 % of the fault
    (in along-strike and down-dip coordinates of the element centres) and
    0.005 outside; d_c = 0.01 m; sigma = 50 MPa.
    """
    s = (f.ix + 0.5) / f.nx - 0.5
    d = (f.iy + 0.5) / f.ny - 0.5
    vw = (np.abs(s) < 0.3) & (np.abs(d) < 0.3)
    n = f.n
    return dict(
        a=np.full(n, 0.010),
        b=np.where(vw, 0.015, 0.005),
        dc=np.full(n, 0.01),
        sigma=np.full(n, 50.0e6),
        vw=vw,
        V0=V0, f0=F0, V_pl=V_PL, eta_rad=MU / (2.0 * CS), mu=MU, nu=NU,
    )


def ensemble_params(f: PlanarRectFault, members: int, seed: int) -> dict:
    """Per-member friction of the many-member runs: per element and member,
    a - b ~ U[-0.006, 0.004] with b = 0.015 fixed (a = b + (a - b)), and
    d_c log-uniform in [0.005, 0.05] m, from numpy's default_rng(seed).
    Arrays are (n, members); sigma = 50 MPa and the constants as in
    friction_params."""
    rng = np.random.default_rng(seed)
    n = f.n
    amb = rng.uniform(-0.006, 0.004, (n, members))
    dc = 10.0 ** rng.uniform(np.log10(0.005), np.log10(0.05), (n, members))
    b = np.full((n, members), 0.015)
    return dict(a=b + amb, b=b, dc=dc, sigma=np.full(n, 50.0e6),
                V0=V0, f0=F0, V_pl=V_PL, eta_rad=MU / (2.0 * CS), mu=MU, nu=NU)
