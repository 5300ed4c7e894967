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
    # the benchmark fault at other sizes (same element size and options)
    "dip30_120x64": dict(mesh=(120, 64, 50.0, 30.0, "dip"),
                         aca_eps=1e-5, leaf=64, eta=2.0, lattice=32, seed=21),
    "dip30_240x128": dict(mesh=(240, 128, 50.0, 30.0, "dip"),
                          aca_eps=1e-5, leaf=64, eta=2.0, lattice=32, seed=22),
    "dip30_960x512": dict(mesh=(960, 512, 50.0, 30.0, "dip"),
                          aca_eps=1e-5, leaf=64, eta=2.0, lattice=32, seed=23),
}

# Stored entries and product time against N (the paper's memory and time
# studies, section 4), and against the lattice size at N = 122880, where
# lattice 1 is the normal H-matrix.
SIZE_SWEEP = ("dip30_120x64", "dip30_240x128", "dip30_480x256", "dip30_960x512")
LATTICE_SWEEP = (1, 8, 32)


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


def ensemble_params(f, members: int, seed: int) -> dict:
    """Per-member friction of the many-member runs: per element and member,
    a - b ~ U[-0.006, 0.004] with b = 0.015 fixed (a = b + (a - b)), and
    d_c log-uniform in [0.005, 0.05] m, from numpy's default_rng(seed).
    Arrays are (n, members); sigma = 50 MPa on a planar fault and the depth
    profile of triangle_friction_params on a TriangleFault (shared by all
    members); the constants as in friction_params."""
    rng = np.random.default_rng(seed)
    n = f.n
    amb = rng.uniform(-0.006, 0.004, (n, members))
    dc = 10.0 ** rng.uniform(np.log10(0.005), np.log10(0.05), (n, members))
    b = np.full((n, members), 0.015)
    sigma = triangle_friction_params(f)["sigma"] if isinstance(f, TriangleFault) else np.full(n, 50.0e6)
    return dict(a=b + amb, b=b, dc=dc, sigma=sigma,
                V0=V0, f0=F0, V_pl=V_PL, eta_rad=MU / (2.0 * CS), mu=MU, nu=NU)


@dataclass
class TriangleFault:
    nx: int                      # quads along strike
    ny: int                      # quads down dip
    verts: np.ndarray = field(repr=False)     # (N, 3, 3), N = 2 nx ny
    slip_dir: np.ndarray = field(repr=False)  # (N, 3) unit up-dip (thrust) directions
    xs: np.ndarray = field(repr=False)        # (N,) along-strike coordinate of the centroid
    ss: np.ndarray = field(repr=False)        # (N,) down-dip arc length of the centroid
    depth: np.ndarray = field(repr=False)     # (N,) depth of the centroid (>= 0)

    @property
    def n(self) -> int:
        return self.verts.shape[0]


def dip_profile(s, dip0_deg=30.0, amp_deg=10.0, wavelength=20.0e3, substeps=200000):
    """Fault trace in the (y, z) plane for a dip that varies down dip,
    delta(s) = dip0 + amp sin(2 pi s / wavelength) (s = down-dip arc length):
    y(s) = int_0^s cos(delta), z(s) = -int_0^s sin(delta), by the trapezoidal
    rule on a uniform grid of `substeps` intervals over [0, max(s)] and linear
    interpolation in between."""
    s = np.asarray(s, dtype=np.float64)
    smax = float(np.max(s))
    g = np.linspace(0.0, smax, substeps + 1)
    d = np.deg2rad(dip0_deg + amp_deg * np.sin(2.0 * np.pi * g / wavelength))
    h = g[1] - g[0]
    cy = np.concatenate([[0.0], np.cumsum(0.5 * h * (np.cos(d[1:]) + np.cos(d[:-1])))])
    cz = np.concatenate([[0.0], -np.cumsum(0.5 * h * (np.sin(d[1:]) + np.sin(d[:-1])))])
    return np.interp(s, g, cy), np.interp(s, g, cz)


def curved_thrust_fault(nx: int, ny: int, length: float = 40.0e3, width: float = 20.0e3,
                        dip0_deg: float = 30.0, amp_deg: float = 10.0, wavelength: float = 20.0e3) -> TriangleFault:
    """Nonplanar thrust fault: a surface translated along strike (x) whose
    dip varies down dip as in dip_profile, meshed by an nx x ny grid of quads
    (uniform in x and in arc length s), each split along its (i, j) -> (i+1, j+1)
    diagonal into triangles 2q and 2q + 1 (q = j nx + i).  Vertices are
    counter-clockwise seen from the hanging wall (+normal, upward); slip is
    up dip along each quad's chord (thrust)."""
    xs = np.linspace(0.0, length, nx + 1)
    sg = np.linspace(0.0, width, ny + 1)
    ys, zs = dip_profile(sg, dip0_deg, amp_deg, wavelength)
    P = lambda i, j: np.array([xs[i], ys[j], zs[j]])
    n = 2 * nx * ny
    verts = np.empty((n, 3, 3))
    slip = np.empty((n, 3))
    cx = np.empty(n)
    cs = np.empty(n)
    for j in range(ny):
        chord = P(0, j + 1) - P(0, j)
        up = -chord / np.linalg.norm(chord)
        for i in range(nx):
            q = j * nx + i
            a, b, c, d = P(i, j), P(i + 1, j), P(i + 1, j + 1), P(i, j + 1)
            verts[2 * q] = (a, b, c)
            verts[2 * q + 1] = (a, c, d)
            slip[2 * q] = slip[2 * q + 1] = up
            cx[2 * q] = (xs[i] + 2.0 * xs[i + 1]) / 3.0
            cs[2 * q] = (2.0 * sg[j] + sg[j + 1]) / 3.0
            cx[2 * q + 1] = (2.0 * xs[i] + xs[i + 1]) / 3.0
            cs[2 * q + 1] = (sg[j] + 2.0 * sg[j + 1]) / 3.0
    depth = -verts[:, :, 2].mean(axis=1)
    return TriangleFault(nx, ny, verts, slip, cx, cs, depth)


TRIANGLE_WORKLOADS = {
    # nonplanar thrust, 150 x 70 quads of ~267 x 286 m -> 21000 triangles
    "thrust_150x70": dict(mesh=(150, 70), aca_eps=1e-6, leaf=32, eta=2.0, lattice=8, seed=1),
    # small versions for the parity tests (same dip profile, coarser elements)
    "thrust_16x12": dict(mesh=(16, 12), aca_eps=1e-8, leaf=16, eta=2.0, lattice=2, seed=21),
    "thrust_40x24": dict(mesh=(40, 24), aca_eps=1e-7, leaf=24, eta=2.0, lattice=4, seed=22),
}


def config_triangle_fault(name: str) -> TriangleFault:
    return curved_thrust_fault(*TRIANGLE_WORKLOADS[name]["mesh"])


def triangle_friction_params(f: TriangleFault) -> dict:
    """Friction of the nonplanar fault: as friction_params (a = 0.010;
    b = 0.015 in the central 60 % along strike and down dip, by the
    centroids' (x, s), else 0.005; d_c = 0.01 m), with sigma rising linearly
    with the centroid depth from 20 MPa (shallowest) to 120 MPa (deepest)."""
    L = f.xs.max() + f.xs.min()
    W = f.ss.max() + f.ss.min()
    vw = (np.abs(f.xs / L - 0.5) < 0.3) & (np.abs(f.ss / W - 0.5) < 0.3)
    d0, d1 = f.depth.min(), f.depth.max()
    sigma = 20.0e6 + 100.0e6 * (f.depth - d0) / (d1 - d0)
    n = f.n
    return dict(a=np.full(n, 0.010), b=np.where(vw, 0.015, 0.005), dc=np.full(n, 0.01), sigma=sigma, vw=vw,
                V0=V0, f0=F0, V_pl=V_PL, eta_rad=MU / (2.0 * CS), mu=MU, nu=NU)
