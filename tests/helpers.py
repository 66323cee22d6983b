"""Small builders shared by the tests: hand-made tracks and arrays."""
import numpy as np

from paper_2309_03717_amd import workloads as W
from paper_2309_03717_amd.workloads import AntennaArray, Medium, Tracks, C_LIGHT


def one_track(p0, p1, beta, t0=0.0, qw=1.0, t1=None):
    """A single straight track from p0 to p1 with velocity vector beta (units
    of c). t1 defaults to t0 + |p1 - p0| / (|beta| c)."""
    p0 = np.asarray(p0, float)
    p1 = np.asarray(p1, float)
    beta = np.asarray(beta, float)
    if t1 is None:
        t1 = t0 + np.linalg.norm(p1 - p0) / (np.linalg.norm(beta) * C_LIGHT)
    a = lambda v: np.array([v], dtype=np.float64)
    return Tracks(a(p0[0]), a(p0[1]), a(p0[2]), a(t0), a(p1[0]), a(p1[1]), a(p1[2]), a(t1),
                  a(beta[0]), a(beta[1]), a(beta[2]), a(qw))


def antennas(points, t_start, dt, n_bins):
    pts = np.asarray(points, float).reshape(-1, 3)
    ts = np.broadcast_to(np.asarray(t_start, float), (pts.shape[0],)).copy()
    return AntennaArray(pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy(), ts, float(dt),
                        int(n_bins))


def track_along(origin, direction, length, beta, t0=0.0, qw=1.0):
    d = np.asarray(direction, float)
    d = d / np.linalg.norm(d)
    p0 = np.asarray(origin, float)
    return one_track(p0, p0 + length * d, beta * d, t0=t0, qw=qw)


UNIFORM = lambda n: Medium("uniform", n - 1.0, 8000.0)


def planted(n, precision, seed=3, start=0):
    """n star-workload tracks (from track `start` on) with droppable ones
    planted: zero and small weights, non-finite fields, points (zero length
    and duration), tracks at rest, and the kept near-misses (zero length with
    a duration, a duration of zero with a length)."""
    a = W.config(1).tracks(n, start=start).arrays()
    for f in a:
        a[f] = a[f].copy()
    rng = np.random.default_rng(seed)
    pick = lambda: rng.random(n) < 0.06
    a["qw"][pick()] = 0.0
    a["qw"][pick()] *= 1e-4
    a["x0"][pick()] = np.nan
    a["t1"][pick()] = np.inf
    a["bz"][pick()] = -np.inf
    pts = pick()
    for f in ("x", "y", "z", "t"):
        a[f + "1"][pts] = a[f + "0"][pts]
    rest = pick()
    for f in ("bx", "by", "bz"):
        a[f][rest] = 0.0
    still = pick()                                   # kept: lasts but does not move in space
    for f in ("x", "y", "z"):
        a[f + "1"][still] = a[f + "0"][still]
    instant = pick()                                 # kept: moves in no time
    a["t1"][instant] = a["t0"][instant]
    tr = W.Tracks(**a)
    return tr.to_mixed() if precision == "mixed" else tr


def expected_mask(tr, qw_min):
    """The track filter's predicate, in numpy: every field finite, |qw| >
    qw_min, some velocity component nonzero, end differs from start."""
    f = {k: np.asarray(getattr(tr, k)).astype(np.float64) for k in W.TRACK_FIELDS}
    finite = np.all([np.isfinite(v) for v in f.values()], axis=0)
    with np.errstate(invalid="ignore"):
        moves = (f["bx"] != 0) | (f["by"] != 0) | (f["bz"] != 0)
        extends = ((f["x1"] != f["x0"]) | (f["y1"] != f["y0"]) | (f["z1"] != f["z0"])
                   | (f["t1"] != f["t0"]))
        heavy = np.abs(f["qw"]) > qw_min
    return finite & heavy & moves & extends
