"""Seeded synthetic workloads (numpy only).

Every generator is deterministic in its seed.  The paper's own GEBCO grids are
not available, so a seeded fractal seafloor stands in for real bathymetry.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


@dataclass(frozen=True)
class GridSpec:
    """Pixel-centre grid: node (a, b) at (x0+(b+.5)dx, y0+(a+.5)dy)."""
    x0: float
    y0: float
    dx: float
    dy: float
    nx: int
    ny: int


@dataclass
class Soundings:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    grid: GridSpec
    radius: float
    power: float = 2.0
    min_pts: int = 1
    max_pts: int = 0          # 0 = no cap
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def checksum(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


# ------------------------------------------------------------------ seafloor --

def _hash01(ix: np.ndarray, iy: np.ndarray, salt: int) -> np.ndarray:
    """Counter-based uniform [0, 1) from integer lattice coordinates
    (splitmix64 finaliser over a mixed key)."""
    with np.errstate(over="ignore"):
        h = (ix.astype(np.int64).astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15))
        h ^= iy.astype(np.int64).astype(np.uint64) * np.uint64(0xC2B2AE3D27D4EB4F)
        h ^= np.uint64(salt & 0xFFFFFFFFFFFFFFFF)
        h ^= h >> np.uint64(30)
        h *= np.uint64(0xBF58476D1CE4E5B9)
        h ^= h >> np.uint64(27)
        h *= np.uint64(0x94D049BB133111EB)
        h ^= h >> np.uint64(31)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _corner_values(ix, iy, salt):
    """Lattice values U[-1, 1] at the four corners (ix, iy), (ix+1, iy),
    (ix, iy+1), (ix+1, iy+1).  The hash is evaluated once per lattice point of
    the inputs' bounding box and gathered (same values as hashing each corner
    directly); very large boxes hash the corners directly."""
    if ix.size == 0:
        e = np.zeros(ix.shape)
        return e, e, e, e
    ix0, iy0 = int(ix.min()), int(iy.min())
    nx, ny = int(ix.max()) - ix0 + 2, int(iy.max()) - iy0 + 2
    if nx * ny > 4 * ix.size + (1 << 16):
        return (2.0 * _hash01(ix, iy, salt) - 1.0, 2.0 * _hash01(ix + 1, iy, salt) - 1.0,
                2.0 * _hash01(ix, iy + 1, salt) - 1.0, 2.0 * _hash01(ix + 1, iy + 1, salt) - 1.0)
    gx = np.arange(nx, dtype=np.int64) + ix0
    gy = np.arange(ny, dtype=np.int64) + iy0
    table = (2.0 * _hash01(np.broadcast_to(gx[None, :], (ny, nx)),
                           np.broadcast_to(gy[:, None], (ny, nx)), salt) - 1.0).ravel()
    k = (iy - iy0) * nx + (ix - ix0)
    return table[k], table[k + 1], table[k + nx], table[k + nx + 1]


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def value_noise(x, y, seed: int = 2, octaves: int = 5, base_wavelength: float = 200.0):
    """Fractal value noise in [-1, 1]: octave o has wavelength base*2^-o and
    amplitude 0.5^o; lattice values U[-1, 1] from a seeded hash, blended with
    the quintic fade, normalised by the amplitude sum."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    acc = np.zeros(np.broadcast(x, y).shape)
    norm = 0.0
    for o in range(octaves):
        lam = base_wavelength * 2.0 ** (-o)
        amp = 0.5 ** o
        fx, fy = x / lam, y / lam
        ix, iy = np.floor(fx), np.floor(fy)
        tx, ty = _fade(fx - ix), _fade(fy - iy)
        ix = ix.astype(np.int64)
        iy = iy.astype(np.int64)
        salt = (seed * 0x100000001B3 + o * 0x9E3779B1) & 0xFFFFFFFFFFFFFFFF
        v00, v10, v01, v11 = _corner_values(ix, iy, salt)
        a = v00 + tx * (v10 - v00)
        b = v01 + tx * (v11 - v01)
        acc = acc + amp * (a + ty * (b - a))
        norm += amp
    return acc / norm


def seafloor_depth(x, y, seed: int = 2):
    """Positive depth D(x, y) = 5000 + 1000 V(x, y), so D lies in (4000, 6000)."""
    return 5000.0 + 1000.0 * value_noise(x, y, seed=seed)


# ------------------------------------------------------------------- cfg 1 --

def uniform_field(n=20000, seed=1, extent=1000.0, nodes=256):
    """Uniform soundings over a square with the analytic depth field
    z = -3000 + 40 sin(x/90) cos(y/130) + 15 sin((x+y)/55) + N(0, 0.5^2)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, extent, n)
    y = rng.uniform(0.0, extent, n)
    z = (-3000.0 + 40.0 * np.sin(x / 90.0) * np.cos(y / 130.0)
         + 15.0 * np.sin((x + y) / 55.0) + rng.normal(0.0, 0.5, n))
    d = extent / nodes
    return x, y, z, GridSpec(0.0, 0.0, d, d, nodes, nodes)


def workload_cfg1() -> Soundings:
    """20k uniform soundings in 1 km^2 -> 256^2 grid at 3.90625 m; IDW p=2,
    r=20 m, min 3, no cap; nearest neighbour with the same radius."""
    x, y, z, g = uniform_field()
    return Soundings(x, y, z, g, radius=20.0, power=2.0, min_pts=3, max_pts=0,
                     name="uniform-20k->256^2")


# ------------------------------------------------------------------- swath --

def swath(seed=2, extent=8192.0, n_lines=8, line_spacing=150.0, pings_per_line=625,
          beams=400, fan_deg=60.0, beam_width_deg=1.0, altitude=None,
          plane_offset=(0.0, 0.0), noise_frac=0.002, centre=None):
    """Multibeam soundings along a lawnmower track in grid-local metres.

    Lines run parallel to y at x_k = centre + (k - (n_lines-1)/2) * spacing;
    pings are evenly spaced along each line (odd lines reversed); beams are
    equiangular over +-fan_deg with a uniform jitter of +-beam_width/2.  The
    across-track offset is H tan(theta) with H the depth under the sensor (a
    surface sensor, altitude=None) or the given altitude (a deep vehicle).
    Depth z = -(D + e), e ~ N(0, (noise_frac D)^2), D from the fractal seafloor
    evaluated in the shared plane (grid-local + plane_offset)."""
    rng = np.random.default_rng(seed)
    if centre is None:
        centre = extent / 2.0
    ox, oy = plane_offset
    lines = centre + (np.arange(n_lines) - (n_lines - 1) / 2.0) * line_spacing
    ping_y = (np.arange(pings_per_line) + 0.5) * extent / pings_per_line
    step = 2.0 * fan_deg / beams
    theta0 = np.deg2rad(-fan_deg + (np.arange(beams) + 0.5) * step)
    xs, ys = [], []
    for k, xl in enumerate(lines):
        py = ping_y if k % 2 == 0 else ping_y[::-1]
        if altitude is None:
            h = seafloor_depth(xl + ox, py + oy, seed=seed)
        else:
            h = np.full(py.shape, float(altitude))
        jit = rng.uniform(-0.5, 0.5, (py.shape[0], beams)) * np.deg2rad(beam_width_deg)
        th = theta0[None, :] + jit
        xs.append(xl + h[:, None] * np.tan(th))
        ys.append(np.broadcast_to(py[:, None], th.shape))
    x = np.concatenate([a.reshape(-1) for a in xs])
    y = np.concatenate([a.reshape(-1) for a in ys]).astype(np.float64)
    dpt = seafloor_depth(x + ox, y + oy, seed=seed)
    z = -(dpt + rng.normal(0.0, 1.0, x.shape[0]) * noise_frac * dpt)
    return x, y, z


def workload_cfg2() -> Soundings:
    """2M soundings (8 lines x 625 pings x 400 beams, surface sensor, +-60 deg)
    -> 4096^2 grid at 2 m over [0, 8192)^2; IDW p=2, r=6 m, max 16, min 1."""
    x, y, z = swath(seed=2)
    g = GridSpec(0.0, 0.0, 2.0, 2.0, 4096, 4096)
    return Soundings(x, y, z, g, radius=6.0, power=2.0, min_pts=1, max_pts=16,
                     name="swath-2M->4096^2")


def workload_cfg4(easting=500000.0, northing=4000000.0) -> Soundings:
    """cfg2's soundings shifted to UTM-like absolute coordinates."""
    s = workload_cfg2()
    g = GridSpec(easting, northing, 2.0, 2.0, 4096, 4096)
    return Soundings(s.x + easting, s.y + northing, s.z, g, radius=6.0, power=2.0,
                     min_pts=1, max_pts=16, name="swath-2M-utm->4096^2")


def small_swath(seed=7, nodes=384, dx=2.0, n_lines=4, pings=160, beams=96,
                altitude=60.0, radius=6.0, max_pts=16, x0=0.0, y0=0.0,
                power=2.0, min_pts=1) -> Soundings:
    """A reduced swath for parity tests: a deep vehicle (fixed altitude) so
    that most soundings land on a small grid; same fractal seafloor."""
    extent = nodes * dx
    x, y, z = swath(seed=seed, extent=extent, n_lines=n_lines,
                    line_spacing=extent / (n_lines + 1), pings_per_line=pings,
                    beams=beams, altitude=altitude)
    g = GridSpec(x0, y0, dx, dx, nodes, nodes)
    return Soundings(x + x0, y + y0, z, g, radius=radius, power=power,
                     min_pts=min_pts, max_pts=max_pts, name=f"small-swath-{nodes}")


# ------------------------------------------------------------------- cfg 3 --

def workload_cfg3_tiles(n_tiles=256, seed=3, n_lo=1e3, n_hi=2e5,
                        sides=(64, 128, 256, 512, 1024), dx=2.0, plane_step=4096.0,
                        scale=1.0):
    """Independent uneven tiles: per tile, point count log-uniform in
    [n_lo, n_hi], side uniform over `sides`, points uniform over the tile,
    depth from the shared fractal seafloor at the tile's plane offset, IDW
    power uniform over {1, 2, 3}; r = 6 m, max 16, min 1.  `scale` shrinks the
    point counts (tests only)."""
    tiles = []
    for t in range(n_tiles):
        rng = np.random.default_rng([seed, t])
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))) * scale))
        side = int(sides[rng.integers(0, len(sides))])
        p = float(rng.integers(1, 4))
        ext = side * dx
        ox, oy = (t % 16) * plane_step, (t // 16) * plane_step
        x = rng.uniform(0.0, ext, n) + ox
        y = rng.uniform(0.0, ext, n) + oy
        dpt = seafloor_depth(x, y, seed=2)
        z = -(dpt + rng.normal(0.0, 1.0, n) * 0.002 * dpt)
        g = GridSpec(ox, oy, dx, dx, side, side)
        tiles.append(Soundings(x, y, z, g, radius=6.0, power=p, min_pts=1,
                               max_pts=16, name=f"tile{t}"))
    return tiles


# ------------------------------------------------------------------- cfg 5 --

@dataclass
class Request:
    vehicle: int
    t_arrival: float
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray


def _vehicle_requests(v, seed, duration, rate_hz, n_lo, n_hi, nodes, dx, beams, altitude,
                      line_spacing, ping_spacing):
    """Grid and request stream of vehicle v (its own random stream)."""
    ext = nodes * dx
    step = 120.0 / beams
    theta0 = np.deg2rad(-60.0 + (np.arange(beams) + 0.5) * step)
    rng = np.random.default_rng([seed, v])
    ox, oy = (v % 4) * 2 * ext, (v // 4) * 2 * ext
    grid = GridSpec(ox, oy, dx, dx, nodes, nodes)
    n_lines = max(1, int(ext // line_spacing))
    lines = (np.arange(n_lines) + 0.5) * line_spacing
    pings_per_line = int(ext // ping_spacing)
    t, ping, out = 0.0, 0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration:
            break
        n = int(rng.integers(n_lo, n_hi + 1))
        npings = -(-n // beams)
        ids = ping + np.arange(npings)
        ping += npings
        li = (ids // pings_per_line) % n_lines
        k = ids % pings_per_line
        py = (k + 0.5) * ping_spacing
        py = np.where(li % 2 == 0, py, ext - py)
        jit = rng.uniform(-0.5, 0.5, (npings, beams)) * np.deg2rad(1.0)
        th = theta0[None, :] + jit
        xs = (lines[li][:, None] + altitude * np.tan(th)).reshape(-1)[:n] + ox
        ys = np.broadcast_to(py[:, None], th.shape).reshape(-1)[:n] + oy
        dpt = seafloor_depth(xs, ys, seed=2)
        zs = -(dpt + rng.normal(0.0, 1.0, n) * 0.002 * dpt)
        out.append(Request(v, t, xs.astype(np.float64), ys.astype(np.float64), zs))
    return grid, out


def _vehicle_requests_star(a):
    return _vehicle_requests(*a)


def serving_schedule(n_vehicles=16, duration=60.0, rate_hz=20.0, n_lo=2000,
                     n_hi=50000, seed=5, nodes=2048, dx=2.0, beams=400,
                     altitude=150.0, line_spacing=512.0, ping_spacing=2.0,
                     max_requests=None, workers=1):
    """Per-vehicle Poisson request streams.  Each vehicle owns a nodes^2 grid
    at dx at its own offset in the shared plane and flies its own lawnmower
    (lines `line_spacing` apart, pings `ping_spacing` apart, wrapping around);
    a request of n soundings is ceil(n/beams) consecutive pings of a +-60 deg
    fan at `altitude`, truncated to n.  Returns (grids, requests sorted by
    arrival).  Vehicles draw from independent streams, so `workers` > 1
    generates them in forked processes with the same result (fork only from a
    process that has not initialised a GPU)."""
    args = [(v, seed, duration, rate_hz, n_lo, n_hi, nodes, dx, beams, altitude,
             line_spacing, ping_spacing) for v in range(n_vehicles)]
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, n_vehicles)) as pool:
            per = pool.map(_vehicle_requests_star, args, chunksize=1)
    else:
        per = [_vehicle_requests(*a) for a in args]
    grids = [g for g, _ in per]
    reqs = [r for _, rs in per for r in rs]
    reqs.sort(key=lambda r: (r.t_arrival, r.vehicle))
    if max_requests is not None:
        reqs = reqs[:max_requests]
    return grids, reqs


# ------------------------------------------------- grid-to-grid protocols --

def dem_on_grid(g: GridSpec, seed: int = 5) -> np.ndarray:
    """Elevation -D(x, y) of the fractal seafloor at the node centres of g,
    float64 [ny, nx]."""
    xs = g.x0 + (np.arange(g.nx) + 0.5) * g.dx
    ys = g.y0 + (np.arange(g.ny) + 0.5) * g.dy
    X, Y = np.meshgrid(xs, ys)
    return -seafloor_depth(X, Y, seed=seed)


def grid_a_case(points: int, h: float = 1.0, seed: int = 11, patch: int = 1024):
    """Row infill (Sec. V, grid A): a complete source grid and a destination
    grid whose rows lie midway between successive source rows, with about
    `points` destination nodes (nx ~ sqrt(points), ny = ceil(points / nx)).
    Sources larger than patch x patch repeat one DEM patch of that size
    (sampling the DEM node by node would take minutes at 1e8 nodes).
    Returns (src_spec, src float32 [ny+1, nx], dst_spec)."""
    nx = max(2, int(round(points ** 0.5)))
    ny = max(1, -(-points // nx))
    src = GridSpec(0.0, 0.0, h, h, nx, ny + 1)
    dst = GridSpec(0.0, 0.5 * h, h, h, nx, ny)
    pw, ph = min(nx, patch), min(ny + 1, patch)
    v = dem_on_grid(GridSpec(0.0, 0.0, h, h, pw, ph), seed).astype(np.float32)
    if (pw, ph) != (nx, ny + 1):
        v = np.tile(v, (-(-(ny + 1) // ph), -(-nx // pw)))[: ny + 1, :nx]
    return src, np.ascontiguousarray(v), dst


def grid_b_case(n_fine: int = 2048, frac: float = 0.05, h: float = 4.0, seed: int = 13,
                truth=None):
    """Random-removal infill (Sec. V, grid B) on the fractal seafloor.

    The truth is the DEM on a fine n_fine^2 grid at spacing h.  The recorded
    grid holds every other fine node (spacing 2h, its origin shifted by -h/2 so
    that coarse node (a, b) sits on fine node (2a, 2b)); round(frac * m) of its
    m nodes, drawn without replacement, are removed (NaN).  The interpolated
    points are every fine node whose value was not recorded.

    Returns a dict: truth_spec, truth (float64), coarse_spec, coarse (float32
    with NaN), removed (bool, coarse shape), interp (bool, fine shape) and
    x, y, z (float64) of the recorded nodes, for the scattered path.  A truth
    from an earlier call with the same n_fine, h and seed may be passed in to
    skip recomputing the DEM."""
    if n_fine % 2:
        raise ValueError("n_fine must be even")
    rng = np.random.default_rng(seed * 1000 + int(round(frac * 1e4)))
    tspec = GridSpec(0.0, 0.0, h, h, n_fine, n_fine)
    if truth is None:
        truth = dem_on_grid(tspec, seed)
    elif truth.shape != (n_fine, n_fine):
        raise ValueError("truth does not match n_fine")
    nc = n_fine // 2
    cspec = GridSpec(-0.5 * h, -0.5 * h, 2.0 * h, 2.0 * h, nc, nc)
    coarse = truth[::2, ::2].copy()
    m = nc * nc
    k = int(round(frac * m))
    removed = np.zeros(m, dtype=bool)
    removed[rng.choice(m, size=k, replace=False)] = True
    removed = removed.reshape(nc, nc)
    coarse[removed] = np.nan
    interp = np.ones((n_fine, n_fine), dtype=bool)
    interp[::2, ::2] = removed
    a, b = np.nonzero(~removed)
    x = cspec.x0 + (b + 0.5) * cspec.dx
    y = cspec.y0 + (a + 0.5) * cspec.dy
    return {"truth_spec": tspec, "truth": truth, "coarse_spec": cspec,
            "coarse": coarse.astype(np.float32), "removed": removed, "interp": interp,
            "x": x.astype(np.float64), "y": y.astype(np.float64),
            "z": coarse[~removed].astype(np.float64)}
