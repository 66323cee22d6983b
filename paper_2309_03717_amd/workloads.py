"""Seeded synthetic workloads for the track x antenna radio-emission loop.

This module only draws inputs: particle tracks, antenna layouts, time windows
and media. It holds none of the emission arithmetic (no propagation, no field,
no deposition), so the HIP path and the FP64 oracle can both consume it.

The paper (§5) measures on tracks from a full CORSIKA 8 shower and on antenna
arrays of 160 to 10,000 antennas whose layouts it does not give; the seeded
workloads below stand in for them with the shapes, sizes and distributions of
the five workload configurations this library is measured on.

Tracks are drawn in blocks of ``BLOCK`` tracks, block ``b`` of workload ``k``
from ``SeedSequence([SEED_BASE + k, b])``, so the first ``n`` tracks of a
workload are the same whatever total size is requested, and a chunk of a large
workload can be regenerated on its own.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional

import numpy as np

C_LIGHT = 299792458.0          # m/s, exact
Z_AXIS = 10_000.0              # m, the axis point the reference plane front starts from
WINDOW_LEAD = 200e-9           # s, trace window opens this long before the reference arrival
N0_AIR = 2.92e-4               # sea-level refractivity n - 1
H_AIR = 8000.0                 # m, scale height of the exponential refractivity
EARTH_RADIUS = 6.371e6         # m, mean Earth radius for the spherical medium
SEED_BASE = 2309037170
BLOCK = 1 << 16                # tracks per seeded block
K_SI = 4.80320471518522e-18    # V*s, e / (4 pi eps0 c): SI prefactor of the fields

TRACK_FIELDS = ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1", "bx", "by", "bz", "qw")
GEOM_FIELDS = TRACK_FIELDS[:8]       # always float64
BETA_W_FIELDS = TRACK_FIELDS[8:]     # float64 (FP64 mode) or float32 (mixed mode)


# --------------------------------------------------------------------------- media
@dataclass(frozen=True)
class Medium:
    """Refractive-index model: ``uniform`` n = 1 + n0m1, ``exponential``
    n = 1 + n0m1 * exp(-z / h), ``tabulated`` n = 1 + n0m1 * f(z) with f
    piecewise linear through ``table`` (values at z0 + i * dz, constant beyond
    the first and last node), or ``spherical`` n = 1 + n0m1 * exp(-H / h) with
    H the height above a spherical Earth of radius ``earth_radius`` whose
    surface touches z = 0 at the origin."""
    kind: str = "uniform"
    n0m1: float = N0_AIR
    h: float = H_AIR
    table: Optional[tuple] = None
    z0: float = 0.0
    dz: float = 1.0
    earth_radius: float = 0.0

    def __post_init__(self):
        if self.kind not in ("uniform", "exponential", "tabulated", "spherical"):
            raise ValueError(f"unknown medium kind {self.kind!r}")
        if self.kind == "spherical" and not self.earth_radius >= 1000.0:
            raise ValueError("a spherical medium needs earth_radius >= 1000 m")
        if self.kind == "tabulated":
            if self.table is None or len(self.table) < 2 or not self.dz > 0:
                raise ValueError("a tabulated medium needs >= 2 nodes and dz > 0")
            object.__setattr__(self, "table", tuple(float(v) for v in self.table))

    @property
    def code(self) -> int:
        return {"uniform": 0, "exponential": 1, "tabulated": 2, "spherical": 3}[self.kind]


def _mean_index(medium: Medium, z_lo: float, z_hi: float) -> float:
    """Mean of n(z) over [z_lo, z_hi] by the trapezoid rule on 4097 points.

    Only used to place each antenna's trace window; it is deliberately not the
    propagator's closed form (and over the spherical Earth it ignores the
    curvature, which moves a vertical column's heights by well under 1 mm)."""
    if medium.kind == "uniform" or z_hi == z_lo:
        return 1.0 + medium.n0m1
    z = np.linspace(z_lo, z_hi, 4097)
    if medium.kind == "tabulated":
        nodes = medium.z0 + medium.dz * np.arange(len(medium.table))
        n = 1.0 + medium.n0m1 * np.interp(z, nodes, np.asarray(medium.table))
    else:
        n = 1.0 + medium.n0m1 * np.exp(-z / medium.h)
    return float(np.trapezoid(n, z) / (z_hi - z_lo))


# --------------------------------------------------------------------------- antennas
@dataclass
class AntennaArray:
    """Antenna positions (m), per-antenna window start t_start (s), bin width
    dt (s) and bin count n_bins. Trace of antenna a, bin k covers
    [t_start[a] + k dt, t_start[a] + (k + 1) dt)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    t_start: np.ndarray
    dt: float
    n_bins: int

    @property
    def m(self) -> int:
        return int(self.x.shape[0])


def grid_layout(nx: int, ny: int, spacing: float):
    """Rectangular grid centred on the shower axis at ground level."""
    i = np.arange(nx * ny)
    col, row = i % nx, i // nx
    x = (col - (nx - 1) / 2.0) * spacing
    y = (row - (ny - 1) / 2.0) * spacing
    return x.astype(np.float64), y.astype(np.float64), np.zeros(nx * ny)


def star_layout(arms: int = 8, per_arm: int = 20, step: float = 25.0):
    """Star pattern: ``arms`` azimuths j*360/arms, radii step*i for i=1..per_arm."""
    xs, ys = [], []
    for j in range(arms):
        phi = 2.0 * math.pi * j / arms
        for i in range(1, per_arm + 1):
            r = step * i
            xs.append(r * math.cos(phi))
            ys.append(r * math.sin(phi))
    return np.array(xs), np.array(ys), np.zeros(len(xs))


def rotated_grid_layout(m: int, spacing: float, angle: float):
    """m antennas filled row-major into a ceil(sqrt(m))-wide grid, rotated."""
    nx = int(math.ceil(math.sqrt(m)))
    ny = int(math.ceil(m / nx))
    x, y, z = grid_layout(nx, ny, spacing)
    x, y, z = x[:m], y[:m], z[:m]
    c, s = math.cos(angle), math.sin(angle)
    return c * x - s * y, s * x + c * y, z


def make_array(x, y, z, medium: Medium, dt: float, n_bins: int,
               lead: float = WINDOW_LEAD) -> AntennaArray:
    """Attach trace windows: each opens ``lead`` before the arrival of a plane
    front that leaves the axis point at height Z_AXIS at t = 0 and travels
    vertically down at the mean speed c / n over the column above the antenna."""
    z = np.asarray(z, dtype=np.float64)
    t_ref = np.array([_mean_index(medium, float(za), Z_AXIS) * (Z_AXIS - za) / C_LIGHT
                      for za in z])
    return AntennaArray(np.asarray(x, np.float64), np.asarray(y, np.float64), z,
                        t_ref - lead, float(dt), int(n_bins))


# --------------------------------------------------------------------------- tracks
@dataclass
class Tracks:
    """Structure-of-arrays straight tracks: start P0 at time t0, end P1 at t1,
    velocity beta (units of c) and charge x weight qw. Geometry is float64;
    beta and qw are float64 (FP64 mode) or float32 (mixed mode)."""
    x0: np.ndarray
    y0: np.ndarray
    z0: np.ndarray
    t0: np.ndarray
    x1: np.ndarray
    y1: np.ndarray
    z1: np.ndarray
    t1: np.ndarray
    bx: np.ndarray
    by: np.ndarray
    bz: np.ndarray
    qw: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x0.shape[0])

    def arrays(self) -> Dict[str, np.ndarray]:
        return {f: getattr(self, f) for f in TRACK_FIELDS}

    def to_mixed(self) -> "Tracks":
        """beta and qw rounded to float32 (the mixed-mode input format)."""
        kw = self.arrays()
        for f in BETA_W_FIELDS:
            kw[f] = np.ascontiguousarray(kw[f], dtype=np.float32)
        return Tracks(**kw)

    def widened(self) -> "Tracks":
        """Every field as float64 (float32 values widened exactly)."""
        return Tracks(**{f: np.ascontiguousarray(a, dtype=np.float64)
                         for f, a in self.arrays().items()})

    def slice(self, lo: int, hi: int) -> "Tracks":
        return Tracks(**{f: np.ascontiguousarray(a[lo:hi]) for f, a in self.arrays().items()})

    def take(self, idx) -> "Tracks":
        return Tracks(**{f: np.ascontiguousarray(a[idx]) for f, a in self.arrays().items()})

    @staticmethod
    def concat(parts: List["Tracks"]) -> "Tracks":
        return Tracks(**{f: np.concatenate([getattr(p, f) for p in parts]) for f in TRACK_FIELDS})


@dataclass(frozen=True)
class TrackRecipe:
    """Distribution of the synthetic tracks."""
    z_lo: float = 1_000.0          # start height range (m)
    z_hi: float = 10_000.0
    sigma: float = 50.0            # lateral Gaussian sigma around the vertical axis (m)
    cap_deg: float = 2.0           # direction within this angle of straight down
    len_lo: float = 0.1            # track length range (m)
    len_hi: float = 10.0
    beta_lo: float = 0.9
    beta_hi: float = 0.99999


def _draw_block(rng: np.random.Generator, n: int, r: TrackRecipe) -> Tracks:
    # fixed draw order: charge, z0, x0, y0, cos(theta), phi, length, beta
    q = np.where(rng.random(n) < 0.5, 1.0, -1.0)
    z0 = rng.uniform(r.z_lo, r.z_hi, n)
    x0 = rng.normal(0.0, r.sigma, n)
    y0 = rng.normal(0.0, r.sigma, n)
    cos_t = rng.uniform(math.cos(math.radians(r.cap_deg)), 1.0, n)   # uniform in solid angle
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    length = rng.uniform(r.len_lo, r.len_hi, n)
    beta = rng.uniform(r.beta_lo, r.beta_hi, n)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    ux, uy, uz = sin_t * np.cos(phi), sin_t * np.sin(phi), -cos_t
    x1, y1, z1 = x0 + length * ux, y0 + length * uy, z0 + length * uz
    # a front moving at c down the axis passes height z0 at (Z_AXIS - z0) / c
    t0 = (Z_AXIS - z0) / C_LIGHT
    t1 = t0 + length / (beta * C_LIGHT)
    return Tracks(x0, y0, z0, t0, x1, y1, z1, t1, beta * ux, beta * uy, beta * uz, q)


def draw_tracks(seed: int, n: int, recipe: TrackRecipe, start: int = 0) -> Tracks:
    """Tracks [start, start + n) of the workload seeded with ``seed``."""
    if n <= 0:
        z = np.zeros(0)
        return Tracks(*([z] * 12))
    parts = []
    b0, b1 = start // BLOCK, (start + n - 1) // BLOCK
    for b in range(b0, b1 + 1):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, b])))
        blk = _draw_block(rng, BLOCK, recipe)
        lo = max(start, b * BLOCK) - b * BLOCK
        hi = min(start + n, (b + 1) * BLOCK) - b * BLOCK
        parts.append(blk.slice(lo, hi))
    return parts[0] if len(parts) == 1 else Tracks.concat(parts)


@dataclass(frozen=True)
class ShowerRecipe:
    """A shower-like track stream (a stand-in for the particle tracks of one
    air shower, whose data the paper uses but does not publish): a thin
    particle front moving down a vertical axis at c, a longitudinal profile
    peaking at ``h_max`` (Gaussian in height, truncated), an exponential
    lateral density, a front that thickens away from the axis, short tracks
    close to the axis direction and a negative charge excess. Within each
    seeded block the tracks are ordered by emission time, so neighbouring
    tracks (the lanes of one wave) arrive at an antenna almost together."""
    h_max: float = 4_000.0       # m
    h_sigma: float = 1_500.0     # m
    z_lo: float = 300.0          # m, profile truncation
    z_hi: float = 12_000.0
    r_scale: float = 30.0        # m, lateral exponential scale
    front_ns: float = 1.0        # ns, front thickness on the axis, x (1 + r / 10 m)
    cap_deg: float = 5.0         # direction within this angle of straight down
    len_lo: float = 0.1          # m
    len_hi: float = 2.0
    beta_lo: float = 0.99
    beta_hi: float = 0.99999
    neg_frac: float = 0.6        # fraction of negative tracks


def _draw_shower_block(rng: np.random.Generator, n: int, r: ShowerRecipe) -> Tracks:
    # fixed draw order: charge, height, radius, azimuth, front delay,
    # cos(theta), phi, length, beta
    q = np.where(rng.random(n) < r.neg_frac, -1.0, 1.0)
    z0 = np.clip(rng.normal(r.h_max, r.h_sigma, n), r.z_lo, r.z_hi)
    rad = rng.exponential(r.r_scale, n)
    az = rng.uniform(0.0, 2.0 * math.pi, n)
    delay = np.abs(rng.normal(0.0, r.front_ns * 1e-9, n)) * (1.0 + rad / 10.0)
    cos_t = rng.uniform(math.cos(math.radians(r.cap_deg)), 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    length = rng.uniform(r.len_lo, r.len_hi, n)
    beta = rng.uniform(r.beta_lo, r.beta_hi, n)
    x0, y0 = rad * np.cos(az), rad * np.sin(az)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    ux, uy, uz = sin_t * np.cos(phi), sin_t * np.sin(phi), -cos_t
    x1, y1, z1 = x0 + length * ux, y0 + length * uy, z0 + length * uz
    t0 = (Z_AXIS - z0) / C_LIGHT + delay
    t1 = t0 + length / (beta * C_LIGHT)
    order = np.argsort(t0, kind="stable")
    return Tracks(x0, y0, z0, t0, x1, y1, z1, t1, beta * ux, beta * uy, beta * uz, q).take(order)


def shower_tracks(seed: int, n: int, recipe: ShowerRecipe = ShowerRecipe(),
                  start: int = 0) -> Tracks:
    """Tracks [start, start + n) of a shower-like stream (same block seeding
    as draw_tracks)."""
    if n <= 0:
        z = np.zeros(0)
        return Tracks(*([z] * 12))
    parts = []
    b0, b1 = start // BLOCK, (start + n - 1) // BLOCK
    for b in range(b0, b1 + 1):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, b])))
        blk = _draw_shower_block(rng, BLOCK, recipe)
        lo = max(start, b * BLOCK) - b * BLOCK
        hi = min(start + n, (b + 1) * BLOCK) - b * BLOCK
        parts.append(blk.slice(lo, hi))
    return parts[0] if len(parts) == 1 else Tracks.concat(parts)


SHOWER_SEED = SEED_BASE + 5


@dataclass(frozen=True)
class InclinedRecipe:
    """An inclined shower over a wide array, where the curvature of the Earth
    shows in the refractive index along the paths: the axis has zenith angle
    ``zenith_deg`` (azimuth 0: travelling towards +x) and meets the ground at
    the origin; emission points are uniform along the axis between
    ``axis_lo`` and ``axis_hi`` metres before the ground, with Gaussian
    offsets of ``sigma`` across it; directions lie within ``cap_deg`` of the
    axis (uniform in solid angle); a plane particle front moves down the axis
    at c from the axis point ``axis_hi`` before the ground at t = 0."""
    zenith_deg: float = 75.0
    axis_lo: float = 2_000.0     # m
    axis_hi: float = 40_000.0
    sigma: float = 200.0         # m
    cap_deg: float = 2.0
    len_lo: float = 0.1          # m
    len_hi: float = 10.0
    beta_lo: float = 0.9
    beta_hi: float = 0.99999

    def frame(self):
        """Unit vectors: the axis direction of motion u and two across it."""
        th = math.radians(self.zenith_deg)
        u = np.array([math.sin(th), 0.0, -math.cos(th)])
        e1 = np.array([math.cos(th), 0.0, math.sin(th)])
        e2 = np.array([0.0, 1.0, 0.0])
        return u, e1, e2

    def front_time(self, x, y, z):
        """When the plane front passes (x, y, z) (s)."""
        u, _, _ = self.frame()
        top = -self.axis_hi * u
        return ((x - top[0]) * u[0] + (y - top[1]) * u[1] + (z - top[2]) * u[2]) / C_LIGHT


def _draw_inclined_block(rng: np.random.Generator, n: int, r: InclinedRecipe) -> Tracks:
    # fixed draw order: charge, axis distance, two offsets, cos(theta), phi,
    # length, beta
    q = np.where(rng.random(n) < 0.5, 1.0, -1.0)
    sa = rng.uniform(r.axis_lo, r.axis_hi, n)
    a1 = rng.normal(0.0, r.sigma, n)
    a2 = rng.normal(0.0, r.sigma, n)
    cos_t = rng.uniform(math.cos(math.radians(r.cap_deg)), 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    length = rng.uniform(r.len_lo, r.len_hi, n)
    beta = rng.uniform(r.beta_lo, r.beta_hi, n)
    u, e1, e2 = r.frame()
    p0 = -sa[:, None] * u + a1[:, None] * e1 + a2[:, None] * e2
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    d = (cos_t[:, None] * u + (sin_t * np.cos(phi))[:, None] * e1
         + (sin_t * np.sin(phi))[:, None] * e2)
    p1 = p0 + length[:, None] * d
    t0 = r.front_time(p0[:, 0], p0[:, 1], p0[:, 2])
    t1 = t0 + length / (beta * C_LIGHT)
    return Tracks(p0[:, 0].copy(), p0[:, 1].copy(), p0[:, 2].copy(), t0, p1[:, 0].copy(),
                  p1[:, 1].copy(), p1[:, 2].copy(), t1, beta * d[:, 0], beta * d[:, 1],
                  beta * d[:, 2], q)


INCLINED_SEED = SEED_BASE + 6


def inclined_shower(n: int, recipe: InclinedRecipe = InclinedRecipe(), nx: int = 8,
                    spacing: float = 2_000.0, dt: float = 0.5e-9, n_bins: int = 8192,
                    seed: int = INCLINED_SEED):
    """n tracks of the inclined shower and an nx x nx ground grid whose
    windows open WINDOW_LEAD before the plane front passes each antenna
    (vacuum speed: refraction delays the pulse by tens of ns, inside the
    window). Returns (tracks, array)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0])))
    tr = _draw_inclined_block(rng, max(n, 0), recipe)
    x, y, z = grid_layout(nx, nx, spacing)
    t_start = recipe.front_time(x, y, z) - WINDOW_LEAD
    return tr, AntennaArray(x, y, z, t_start, float(dt), int(n_bins))


# --------------------------------------------------------------------------- workloads
@dataclass
class Workload:
    name: str
    seed: int
    n_tracks: int
    recipe: TrackRecipe
    array: AntennaArray
    medium: Medium
    formalisms: tuple
    precisions: tuple
    chunk: int = 0                  # tracks per streamed chunk (0: one call)
    notes: str = ""

    def tracks(self, n: Optional[int] = None, start: int = 0, mixed: bool = False) -> Tracks:
        n = self.n_tracks - start if n is None else n
        t = draw_tracks(self.seed, n, self.recipe, start)
        return t.to_mixed() if mixed else t


def layered_air(dz: float = 50.0, top: float = 20_000.0) -> Medium:
    """A tabulated atmosphere (a stand-in for a measured refractivity profile):
    exponential with an 8 km scale height up to 10 km and a 6.3 km one above,
    sampled every ``dz`` metres from 0 to ``top``."""
    z = np.arange(0.0, top + 0.5 * dz, dz)
    f = np.where(z < 10_000.0, np.exp(-z / 8_000.0),
                 math.exp(-10_000.0 / 8_000.0) * np.exp(-(z - 10_000.0) / 6_300.0))
    return Medium("tabulated", N0_AIR, H_AIR, tuple(f), 0.0, dz)


UNIFORM_AIR = Medium("uniform", N0_AIR, H_AIR)
EXPONENTIAL_AIR = Medium("exponential", N0_AIR, H_AIR)
SPHERICAL_AIR = Medium("spherical", N0_AIR, H_AIR, earth_radius=EARTH_RADIUS)
RECIPE_SMALL = TrackRecipe(1_000.0, 10_000.0, 50.0)
RECIPE_WIDE = TrackRecipe(500.0, 15_000.0, 100.0)


def config(k: int) -> Workload:
    """The five workload configurations (k = 0..4; 4 is returned by ``batched_showers``)."""
    if k == 0:
        x, y, z = grid_layout(4, 4, 100.0)
        arr = make_array(x, y, z, UNIFORM_AIR, 0.2e-9, 4096)
        return Workload("endpoint-fp64-1e4trk-16ant", SEED_BASE + 0, 10_000, RECIPE_SMALL, arr,
                        UNIFORM_AIR, ("endpoint",), ("fp64",))
    if k == 1:
        x, y, z = star_layout(8, 20, 25.0)
        arr = make_array(x, y, z, EXPONENTIAL_AIR, 0.1e-9, 4096)
        return Workload("star160-1e7trk-expn", SEED_BASE + 1, 10_000_000, RECIPE_WIDE, arr,
                        EXPONENTIAL_AIR, ("endpoint", "zhs"), ("fp64", "mixed"))
    if k == 2:
        x, y, z = grid_layout(64, 64, 50.0)
        arr = make_array(x, y, z, EXPONENTIAL_AIR, 0.2e-9, 4096)
        return Workload("grid4096-1e8trk-expn-mixed", SEED_BASE + 2, 100_000_000, RECIPE_WIDE, arr,
                        EXPONENTIAL_AIR, ("endpoint", "zhs"), ("mixed",), chunk=1 << 22)
    if k == 3:
        x, y, z = grid_layout(8, 8, 75.0)
        arr = make_array(x, y, z, EXPONENTIAL_AIR, 0.1e-9, 4096)
        return Workload("zhs-adjoint-1e6trk-64ant", SEED_BASE + 3, 1_000_000, RECIPE_WIDE, arr,
                        EXPONENTIAL_AIR, ("zhs",), ("mixed",))
    raise ValueError("configs are 0..3 here; use batched_showers() for the batched workload")


def perturbed_target(tracks: Tracks, medium: Medium, seed: int):
    """Target parameters for the differentiable-ZHS workload: every track moved
    by one N(0, 0.5 m) 3-vector (both ends, so beta and the times are kept),
    weights scaled by (1 + N(0, 0.05)), refractivity n0 - 1 scaled by 1.02."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1])))
    n = tracks.n
    d = rng.normal(0.0, 0.5, (3, n))
    w = 1.0 + rng.normal(0.0, 0.05, n)
    kw = tracks.arrays()
    kw = {f: np.array(a, copy=True) for f, a in kw.items()}
    for i, (a, b) in enumerate((("x0", "x1"), ("y0", "y1"), ("z0", "z1"))):
        kw[a] = kw[a] + d[i]
        kw[b] = kw[b] + d[i]
    kw["qw"] = (kw["qw"].astype(np.float64) * w).astype(kw["qw"].dtype)
    return Tracks(**kw), replace(medium, n0m1=medium.n0m1 * 1.02)


@dataclass
class Shower:
    index: int
    seed: int
    n_tracks: int
    array: AntennaArray
    medium: Medium
    formalism: str

    def tracks(self, mixed: bool = True) -> Tracks:
        t = draw_tracks(self.seed, self.n_tracks, RECIPE_WIDE)
        return t.to_mixed() if mixed else t


def batched_showers(n_showers: int = 256, seed: int = SEED_BASE + 4,
                    max_tracks: Optional[int] = None) -> List[Shower]:
    """Independent showers: track counts log-uniform in [1e4, 1e6], 16..512
    antennas on a rotated grid of random spacing, 2048..8192 bins (multiples of
    256) of 0.1..0.5 ns, Endpoint or ZHS and uniform or exponential medium
    with equal odds. ``max_tracks`` caps each shower (for small test runs)."""
    out = []
    for s in range(n_showers):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1_000_000 + s])))
        n = int(round(10.0 ** rng.uniform(4.0, 6.0)))
        m = int(rng.integers(16, 513))
        spacing = float(rng.uniform(25.0, 150.0))
        angle = float(rng.uniform(0.0, 2.0 * math.pi))
        n_bins = 256 * int(rng.integers(8, 33))
        dt = float(rng.uniform(0.1e-9, 0.5e-9))
        formalism = "endpoint" if rng.random() < 0.5 else "zhs"
        medium = UNIFORM_AIR if rng.random() < 0.5 else EXPONENTIAL_AIR
        if max_tracks is not None:
            n = min(n, max_tracks)
        x, y, z = rotated_grid_layout(m, spacing, angle)
        arr = make_array(x, y, z, medium, dt, n_bins)
        out.append(Shower(s, seed * 1000 + s, n, arr, medium, formalism))
    return out
