"""Small builders shared by the tests: hand-made tracks and arrays."""
import numpy as np

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
