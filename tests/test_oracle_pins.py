"""Pins of the FP64 oracle to facts that do not come from the oracle itself:
closed forms of special geometries, numerical quadrature, the physics that
links the two formalisms (E = -dA/dt), conservation of the ZHS time integral,
exact cancellation of a split track, brute-force spreading, invariances of
the geometry and finite differences of the adjoint.

The paper (§1, §2) names the Endpoint and ZHS formalisms and the
straight-line propagator without printing their formulas, and prints no
worked example; so there is no golden value from the paper to compare with.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2309_03717_amd.workloads import (C_LIGHT, N0_AIR, Medium, Tracks, config, draw_tracks,
                                            RECIPE_WIDE, EXPONENTIAL_AIR, UNIFORM_AIR)
from helpers import antennas, one_track, track_along, UNIFORM

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

ULP = np.finfo(np.float64).eps


# ----------------------------------------------------------------- propagator
def test_distance_and_time_345(orc):
    """3-4-5 triangle: R = 5000 m exactly; in vacuum-like n = 1 the arrival
    time is T + R / c."""
    tr = one_track((0, 0, 4000.0), (0, 0, 3999.0), (0, 0, -0.9), t0=1e-6)
    ar = antennas([(3000.0, 0, 0)], 0.0, 1e-9, 100000)
    t, u, b = orc.propagate(tr, ar, UNIFORM(1.0))
    assert t[0, 0, 0] == pytest.approx(1e-6 + 5000.0 / C_LIGHT, rel=2 * ULP, abs=0)
    assert b[0, 0, 0] == int(math.floor((1e-6 + 5000.0 / C_LIGHT) / 1e-9))


@pytest.mark.parametrize("zp,za", [(10_000.0, 0.0), (500.0, 0.0), (15_000.0, 300.0),
                                   (1200.0, 1500.0), (700.0004, 700.0), (3.0, 2.9995)])
def test_effective_index_is_path_mean(orc, zp, za):
    """Exponential medium: n_eff = (t - T) c / R equals the mean of n(z) along
    the straight path, evaluated by adaptive quadrature (including the
    |dz| < 1 mm branch)."""
    md = EXPONENTIAL_AIR
    p = np.array([120.0, -40.0, zp])
    x = np.array([-35.0, 60.0, za])
    tr = one_track(p, p + [0, 0, -1.0], (0, 0, -0.99), t0=2e-6)
    ar = antennas([x], 0.0, 1e-9, 10)
    t, _, _ = orc.propagate(tr, ar, md)
    r = float(np.linalg.norm(x - p))
    neff = (t[0, 0, 0] - 2e-6) * C_LIGHT / r
    if abs(zp - za) > 0:
        mean = integrate.quad(lambda z: md.n0m1 * math.exp(-z / md.h), za, zp,
                              epsabs=0, epsrel=1e-13)[0] / (zp - za)
    else:
        mean = md.n0m1 * math.exp(-za / md.h)
    assert (neff - 1.0) == pytest.approx(mean, rel=1e-8)


def test_bin_edge_goes_up(orc):
    """A time exactly on a bin edge belongs to the bin above it; one ulp
    earlier it belongs to the bin below (power-of-two bin width makes u exact)."""
    dt = 2.0 ** -30
    tr = one_track((10.0, 0, 900.0), (10.0, 0, 899.0), (0, 0, -0.95))
    ar = antennas([(0, 0, 0)], 0.0, dt, 64)
    t, _, _ = orc.propagate(tr, ar, UNIFORM(1.000292))
    t_arr = t[0, 0, 0]
    ar_on = antennas([(0, 0, 0)], t_arr - 5 * dt, dt, 64)
    _, u, b = orc.propagate(tr, ar_on, UNIFORM(1.000292))
    assert u[0, 0, 0] == 5.0 and b[0, 0, 0] == 5
    ar_below = antennas([(0, 0, 0)], np.nextafter(t_arr - 5 * dt, 1.0), dt, 64)
    _, u2, b2 = orc.propagate(tr, ar_below, UNIFORM(1.000292))
    assert u2[0, 0, 0] < 5.0 and b2[0, 0, 0] == 4
    # outside the window on both sides
    ar_late = antennas([(0, 0, 0)], t_arr + dt, dt, 64)
    assert orc.propagate(tr, ar_late, UNIFORM(1.000292))[2][0, 0, 0] == -1
    ar_early = antennas([(0, 0, 0)], t_arr - 64 * dt, dt, 64)
    assert orc.propagate(tr, ar_early, UNIFORM(1.000292))[2][0, 0, 0] == -1


# ----------------------------------------------------------------- Endpoint
def _theta_geometry(theta, r, length=1.0, beta=0.9, n=1.000292, qw=1.0):
    """Track moving straight down from P0 = (0, 0, 2000); antenna at
    P0 + r (sin th, 0, -cos th): the line of sight makes angle th with beta."""
    p0 = np.array([0.0, 0.0, 2000.0])
    x = p0 + r * np.array([math.sin(theta), 0.0, -math.cos(theta)])
    tr = track_along(p0, (0, 0, -1), length, beta, qw=qw)
    return tr, x


@pytest.mark.parametrize("theta_deg,n", [(90.0, 1.000292), (30.0, 1.000292), (60.0, 1.5),
                                         (5.0, 1.000292), (20.0, 1.5)])
def test_endpoint_start_impulse_closed_form(orc, theta_deg, n):
    """Closed form for this geometry: with beta along -z and the line of sight
    at angle th, the start impulse is
        E = k qw beta sin th (cos th, 0, sin th) / ((1 - n beta cos th) R dt)
    (the perpendicular case th = 90 deg gives D = 1)."""
    th = math.radians(theta_deg)
    r, beta, dt, k, qw = 800.0, 0.9, 0.1e-9, 1.7, -1.0
    tr, x = _theta_geometry(th, r, beta=beta, n=n, qw=qw)
    t, u, b = orc.propagate(tr, antennas([x], 0.0, dt, 1), UNIFORM(n))
    k0 = int(math.floor(u[0, 0, 0]))
    ar = antennas([x], k0 * dt - 50 * dt, dt, 4096)    # start lands in bin 50
    tr_only_start = tr
    e = orc.traces("endpoint", tr_only_start, ar, UNIFORM(n), k=k)[0]
    _, u2, b2 = orc.propagate(tr, ar, UNIFORM(n))
    ks, ke = b2[0, 0, 0], b2[1, 0, 0]
    assert ks != ke, "geometry must separate the two impulses"
    d = 1.0 - n * beta * math.cos(th)
    expect = k * qw * beta * math.sin(th) * np.array([math.cos(th), 0.0, math.sin(th)]) / (d * r * dt)
    np.testing.assert_allclose(e[ks], expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())


def test_endpoint_transverse_and_linear(orc):
    """Every impulse is transverse to its line of sight (E . r = 0); flipping
    the charge negates the traces exactly; doubling qw doubles them exactly."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        p0 = rng.uniform([-300, -300, 500], [300, 300, 5000])
        direc = rng.normal(size=3)
        tr = track_along(p0, direc, rng.uniform(0.5, 5.0), rng.uniform(0.5, 0.999))
        x = rng.uniform([-500, -500, 0], [500, 500, 100])
        t, u, b = orc.propagate(tr, antennas([x], 0.0, 1e-10, 1), UNIFORM(1.000292))
        ar = antennas([x], (math.floor(u[0, 0, 0]) - 100) * 1e-10, 1e-10, 4096)
        e = orc.traces("endpoint", tr, ar, UNIFORM(1.000292))[0]
        _, _, bb = orc.propagate(tr, ar, UNIFORM(1.000292))
        ks, ke = bb[0, 0, 0], bb[1, 0, 0]
        if ks == ke:
            continue
        rhat = (x - p0) / np.linalg.norm(x - p0)
        assert abs(e[ks] @ rhat) <= 1e-12 * np.linalg.norm(e[ks])
        flip = Tracks(**{**tr.arrays(), "qw": -tr.qw})
        np.testing.assert_array_equal(orc.traces("endpoint", flip, ar, UNIFORM(1.000292))[0], -e)
        dbl = Tracks(**{**tr.arrays(), "qw": 2.0 * tr.qw})
        np.testing.assert_array_equal(orc.traces("endpoint", dbl, ar, UNIFORM(1.000292))[0], 2.0 * e)


def _split(tr: Tracks, f: float):
    a = tr.arrays()
    mid = {c: a[c + "0"] + f * (a[c + "1"] - a[c + "0"]) for c in ("x", "y", "z", "t")}
    first = Tracks(**{**a, "x1": mid["x"], "y1": mid["y"], "z1": mid["z"], "t1": mid["t"]})
    second = Tracks(**{**a, "x0": mid["x"], "y0": mid["y"], "z0": mid["z"], "t0": mid["t"]})
    return Tracks.concat([first, second])


@pytest.mark.parametrize("medium", [UNIFORM_AIR, EXPONENTIAL_AIR])
def test_endpoint_split_track_cancels(orc, medium):
    """Splitting a track at an interior point adds a stop and a start impulse
    at the same place and time: they cancel exactly, so the traces equal the
    unsplit track's up to summation rounding."""
    w = config(1)
    tr = w.tracks(200)
    split = Tracks.concat([_split(tr.take([i]), 0.37) for i in range(tr.n)])
    whole = orc.traces("endpoint", tr, w.array, medium)
    parts = orc.traces("endpoint", split, w.array, medium)
    scale = np.abs(whole).max()
    assert scale > 0
    np.testing.assert_allclose(parts, whole, rtol=0, atol=1e-12 * scale)


# ----------------------------------------------------------------- ZHS
@pytest.mark.parametrize("theta_deg,n", [(90.0, 1.000292), (40.0, 1.000292), (20.0, 1.5)])
def test_zhs_time_integral_closed_form(orc, theta_deg, n):
    """The ZHS box conserves its time integral: sum_k A_k dt = I with, for
    this geometry (angle th at the midpoint, beta along -z),
        I = -k qw L sin th (cos th, 0, sin th) / (c R_mid)."""
    th = math.radians(theta_deg)
    L, beta, r, dt, k, qw = 4.0, 0.95, 600.0, 0.1e-9, 1.0, 1.0
    p0 = np.array([0.0, 0.0, 3000.0])
    mid = p0 + [0, 0, -L / 2]
    x = mid + r * np.array([math.sin(th), 0.0, -math.cos(th)])
    tr = track_along(p0, (0, 0, -1), L, beta, qw=qw)
    _, u, _ = orc.propagate(tr, antennas([x], 0.0, dt, 1), UNIFORM(n))
    lo = math.floor(min(u[:, 0, 0]))
    ar = antennas([x], (lo - 300) * dt, dt, 8192)
    a = orc.traces("zhs", tr, ar, UNIFORM(n), k=k)[0]
    total = a.sum(axis=0) * dt
    expect = -k * qw * L * math.sin(th) * np.array([math.cos(th), 0.0, math.sin(th)]) / (C_LIGHT * r)
    np.testing.assert_allclose(total, expect, rtol=1e-12, atol=1e-13 * np.abs(expect).max())
    # and the potential is transverse to the midpoint line of sight
    rhat = (x - mid) / r
    assert np.abs(a @ rhat).max() <= 1e-12 * np.abs(a).max()


def test_zhs_spread_matches_brute_force_sampling(orc):
    """Each bin holds the fraction of the box [u_lo, u_hi] that overlaps it:
    compare with a 2e6-point uniform sampling of the box (O(1/m) agreement),
    including boxes clipped by either window edge."""
    rng = np.random.default_rng(11)
    md = UNIFORM(1.000292)
    m = 2_000_000
    checked = 0
    for trial in range(12):
        p0 = rng.uniform([-50, -50, 800], [50, 50, 3000])
        tr = track_along(p0, rng.normal(size=3) * [0.3, 0.3, 1] - [0, 0, 2], rng.uniform(2, 10),
                         rng.uniform(0.9, 0.999))
        x = rng.uniform([-400, -400, 0], [400, 400, 0])
        dt = 0.1e-9
        _, u, _ = orc.propagate(tr, antennas([x], 0.0, dt, 1), md)
        ulo, uhi = sorted(u[:, 0, 0])
        if uhi - ulo < 1.5:
            continue
        # shift so the box straddles bin 0, sits inside, or straddles the end
        for offset in (-0.4, 0.5, 1.3):
            nb = 64 + int(math.ceil(uhi - ulo))
            start_bin = math.floor(ulo) + int(offset * (uhi - ulo)) if offset != 0.5 else math.floor(ulo) - 10
            ar = antennas([x], start_bin * dt, dt, nb)
            _, uu, _ = orc.propagate(tr, ar, md)
            lo, hi = sorted(uu[:, 0, 0])
            a = orc.traces("zhs", tr, ar, md)[0]
            full = orc.traces("zhs", tr, antennas([x], (math.floor(lo) - 5 + start_bin) * dt, dt,
                                                   nb + 4096), md)[0]
            integral = full.sum(axis=0) * dt
            samples = lo + (hi - lo) * (np.arange(m) + 0.5) / m
            hist = np.bincount(np.floor(samples[(samples >= 0) & (samples < nb)]).astype(np.int64),
                               minlength=nb)[:nb] / m
            expect = hist[:, None] * integral[None, :] / dt
            np.testing.assert_allclose(a, expect, rtol=0, atol=3.0 / m * np.abs(integral).max() / dt
                                       * (1 + (hi - lo)))
            checked += 1
    assert checked >= 12


@pytest.mark.parametrize("n,theta_deg,beta", [(1.000292, 60.0, 0.95), (1.000292, 25.0, 0.999),
                                              (1.5, 70.0, 0.9), (1.5, 20.0, 0.99)])
def test_endpoint_and_zhs_agree(orc, n, theta_deg, beta):
    """The two formalisms describe the same radiation: E = -dA/dt, so on the
    interior bins of a wide box -dt * cumsum(E) equals A up to O(L/R) (the
    Endpoint impulses use the end-point geometry, ZHS the midpoint). The
    n = 1.5, 20 deg case lies inside the Cherenkov cone (1 - n beta cos th < 0),
    where only the signed Doppler factor gives the right sign. The box edges
    are the Endpoint impulse bins exactly."""
    th = math.radians(theta_deg)
    L, r, dt = 10.0, 2000.0, 0.1e-9
    p0 = np.array([0.0, 0.0, 4000.0])
    mid = p0 + [0, 0, -L / 2]
    x = mid + r * np.array([math.sin(th), 0.0, -math.cos(th)])
    tr = track_along(p0, (0, 0, -1), L, beta)
    md = UNIFORM(n)
    _, u, _ = orc.propagate(tr, antennas([x], 0.0, dt, 1), md)
    lo, hi = sorted(u[:, 0, 0])
    assert hi - lo > 20, "needs a wide box"
    ar = antennas([x], (math.floor(lo) - 100) * dt, dt, int(hi - lo) + 300)
    e = orc.traces("endpoint", tr, ar, md)[0]
    a = orc.traces("zhs", tr, ar, md)[0]
    _, _, b = orc.propagate(tr, ar, md)
    klo, khi = sorted(b[:, 0, 0])
    nz = np.flatnonzero(np.abs(a).max(axis=1) > 0)
    assert nz[0] == klo and nz[-1] == khi
    ez = np.flatnonzero(np.abs(e).max(axis=1) > 0)
    assert list(ez) == sorted({klo, khi})
    integ = -dt * np.cumsum(e, axis=0)
    inner = slice(klo + 1, khi)
    tol = 2.0 * L / r
    np.testing.assert_allclose(integ[inner], a[inner], rtol=tol, atol=tol * np.abs(a).max())
    inside_cone = 1.0 - n * beta * math.cos(th) < 0
    if inside_cone:   # the |D| reading would flip the sign of the integrated field
        assert np.sign(integ[inner][:, 0]).tolist() == np.sign(a[inner][:, 0]).tolist()


# ----------------------------------------------------------------- invariances
def test_thread_and_bunch_count_do_not_change_results(orc):
    """§5 (Figs. 6 and 7): pulses are identical for any number of threads; the
    oracle's antenna-bunch split gives bit-identical traces."""
    w = config(1)
    tr = w.tracks(3000)
    for f in ("endpoint", "zhs"):
        ref = orc.traces(f, tr, w.array, w.medium, n_threads=1)
        for th, bunch in ((3, 0), (8, 1), (5, 16), (2, 200)):
            np.testing.assert_array_equal(orc.traces(f, tr, w.array, w.medium, n_threads=th,
                                                     bunch=bunch), ref)


def test_track_order_permutation(orc):
    """Reordering tracks changes only the summation order."""
    w = config(0)
    tr = w.tracks(4000)
    perm = np.random.default_rng(3).permutation(tr.n)
    for f in ("endpoint", "zhs"):
        a = orc.traces(f, tr, w.array, w.medium)
        b = orc.traces(f, tr.take(perm), w.array, w.medium)
        scale = np.abs(a).max()
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-11 * scale)


def test_translation_invariance(orc):
    """Moving tracks and antennas together horizontally (any medium) or
    vertically (uniform medium) leaves the traces unchanged up to rounding."""
    w = config(0)
    tr = w.tracks(2000)
    ar = w.array
    for f in ("endpoint", "zhs"):
        for md, shift in ((EXPONENTIAL_AIR, (1024.0, -512.0, 0.0)), (UNIFORM_AIR, (0.0, 0.0, 256.0))):
            a = orc.traces(f, tr, ar, md)
            d = tr.arrays()
            tr2 = Tracks(**{**d, "x0": d["x0"] + shift[0], "x1": d["x1"] + shift[0],
                            "y0": d["y0"] + shift[1], "y1": d["y1"] + shift[1],
                            "z0": d["z0"] + shift[2], "z1": d["z1"] + shift[2]})
            ar2 = antennas(np.stack([ar.x + shift[0], ar.y + shift[1], ar.z + shift[2]], 1),
                           ar.t_start, ar.dt, ar.n_bins)
            b = orc.traces(f, tr2, ar2, md)
            err = np.linalg.norm(b - a) / np.linalg.norm(a)
            assert err < 1e-6, (f, md.kind, err)


def test_window_clipping_and_empty_inputs(orc):
    """Out-of-window tracks leave the traces untouched; zero tracks or zero
    antennas are valid and produce nothing."""
    w = config(0)
    tr = w.tracks(100)
    late = antennas(np.stack([w.array.x, w.array.y, w.array.z], 1), w.array.t_start + 1e-3,
                    w.array.dt, w.array.n_bins)
    for f in ("endpoint", "zhs"):
        assert not orc.traces(f, tr, late, w.medium).any()
        assert not orc.traces(f, tr.slice(0, 0), w.array, w.medium).any()
    empty = antennas(np.zeros((0, 3)), 0.0, 1e-10, 16)
    assert orc.traces("zhs", tr, empty, w.medium).shape == (0, 16, 3)


# ----------------------------------------------------------------- adjoint
def _loss(orc, tr, ar, md, g, k=1.0):
    return float(np.sum(g * orc.traces("zhs", tr, ar, md, k=k)))


def test_zhs_vjp_weight_is_exact_linear_share(orc):
    """A is linear in qw, so dL/dqw_i = L_i / qw_i with L_i the loss share of
    track i alone."""
    w = config(3)
    tr = w.tracks(40)
    g = np.random.default_rng(5).normal(size=(w.array.m, w.array.n_bins, 3))
    grads = orc.zhs_vjp(tr, w.array, w.medium, g, n_threads=3)
    for i in range(tr.n):
        li = _loss(orc, tr.take([i]), w.array, w.medium, g)
        assert grads["qw"][i] == pytest.approx(li / tr.qw[i], rel=1e-10, abs=1e-300)


def _adjoint_medium(name):
    from paper_2309_03717_amd.workloads import SPHERICAL_AIR, layered_air
    return {"exponential": config(3).medium, "layered": layered_air(),
            "spherical": SPHERICAL_AIR}[name]


def _with_n0(md, v):
    import dataclasses
    return dataclasses.replace(md, n0m1=v)


@pytest.mark.parametrize("medium", ["exponential", "layered", "spherical"])
def test_zhs_vjp_matches_central_differences(orc, medium):
    """Positions and n0 - 1 by central differences on the forward oracle
    (Richardson-extrapolated from steps h and 2h: h = 1e-5 m, 1e-6 relative),
    skipping tracks whose shift moves a box edge across a bin edge (the loss
    has a kink there). Narrow near-Cherenkov boxes make the loss strongly
    curved in the edge positions, hence the small steps. In the exponential,
    tabulated and spherical-Earth media (the last with horizontal components
    of the path-index gradient)."""
    w = config(3)
    md = _adjoint_medium(medium)
    rng = np.random.default_rng(9)
    tr = w.tracks(400)
    ar = w.array
    # keep tracks that reach at least one antenna window
    _, u, b = orc.propagate(tr, ar, md)
    reach = np.flatnonzero(((b >= 0).any(axis=0)).any(axis=1))[:12]
    tr = tr.take(reach)
    g = rng.normal(size=(ar.m, ar.n_bins, 3))
    grads = orc.zhs_vjp(tr, ar, md, g)

    def central(f, x0, h):
        return (f(x0 + h) - f(x0 - h)) / (2 * h)

    def richardson(f, x0, h):
        return (4.0 * central(f, x0, h) - central(f, x0, 2 * h)) / 3.0

    h = 1e-5
    checked = 0
    for i in range(tr.n):
        one = tr.take([i])
        _, u0, _ = orc.propagate(one, ar, md)
        scale = max(np.abs(grads["p0"][:, i]).max(), np.abs(grads["p1"][:, i]).max())
        for end in (0, 1):
            for c, comp in enumerate("xyz"):
                key = f"{comp}{end}"
                base = one.arrays()[key]

                def moved(v):
                    return Tracks(**{**one.arrays(), key: np.array([v])})

                crosses = False
                for s in (-2 * h, 2 * h):
                    _, us, _ = orc.propagate(moved(base[0] + s), ar, md)
                    crosses |= bool((np.floor(us) != np.floor(u0)).any())
                if crosses:
                    continue
                fd = richardson(lambda v: _loss(orc, moved(v), ar, md, g), base[0], h)
                an = grads["p0" if end == 0 else "p1"][c, i]
                assert abs(an - fd) <= 1e-5 * abs(fd) + 1e-6 * scale, (i, key, an, fd)
                checked += 1
    assert checked > 30
    # refractivity
    hn = 1e-6 * md.n0m1   # t is quantized to ~7e-21 s: smaller steps drown in rounding
    _, u0, _ = orc.propagate(tr, ar, md)
    keep = []
    for i in range(tr.n):
        ok = True
        for s in (-2 * hn, 2 * hn):
            _, us, _ = orc.propagate(tr.take([i]), ar, _with_n0(md, md.n0m1 + s))
            ok &= bool((np.floor(us[:, 0]) == np.floor(u0[:, i])).all())
        if ok:
            keep.append(i)
    sub = tr.take(keep)
    assert sub.n >= 6
    fd = richardson(lambda v: _loss(orc, sub, ar, _with_n0(md, v), g), md.n0m1, hn)
    an = orc.zhs_vjp(sub, ar, md, g)["n0m1"]
    assert an == pytest.approx(fd, rel=1e-5)


# --------------------------------------------------------- Endpoint adjoint
def _ep_loss(orc, tr, ar, md, g, k=1.0):
    return float(np.sum(g * orc.traces("endpoint", tr, ar, md, k=k)))


@pytest.mark.parametrize("cfg", [0, 3])
def test_endpoint_vjp_weight_is_exact_linear_share(orc, cfg):
    """E is linear in qw: dL/dqw_i = L_i / qw_i (uniform and exponential
    media)."""
    w = config(cfg)
    tr = w.tracks(40)
    g = np.random.default_rng(15).normal(size=(w.array.m, w.array.n_bins, 3))
    grads = orc.endpoint_vjp(tr, w.array, w.medium, g, n_threads=3)
    nonzero = 0
    for i in range(tr.n):
        li = _ep_loss(orc, tr.take([i]), w.array, w.medium, g)
        assert grads["qw"][i] == pytest.approx(li / tr.qw[i], rel=1e-10, abs=1e-300)
        nonzero += li != 0.0
    assert nonzero >= 10


@pytest.mark.parametrize("cfg,medium", [(0, None), (3, None), (3, "layered"), (3, "spherical")])
def test_endpoint_vjp_matches_central_differences(orc, cfg, medium):
    """Positions and n0 - 1 against Richardson-extrapolated central
    differences of the forward oracle (steps h and 2h; h = 1e-3 m and 1e-6
    relative), skipping shifts that move an impulse across a bin edge (the
    loss jumps there; the adjoint holds bins fixed); uniform, exponential,
    tabulated and spherical-Earth media (path index and source index)."""
    w = config(cfg)
    md, ar = (w.medium if medium is None else _adjoint_medium(medium)), w.array
    tr = w.tracks(400)
    _, u, b = orc.propagate(tr, ar, md)
    reach = np.flatnonzero(((b >= 0).any(axis=0)).any(axis=1))[:10]
    tr = tr.take(reach)
    g = np.random.default_rng(21).normal(size=(ar.m, ar.n_bins, 3))
    grads = orc.endpoint_vjp(tr, ar, md, g)

    def richardson(f, x0, h):
        c = lambda s: (f(x0 + s) - f(x0 - s)) / (2 * s)
        return (4.0 * c(h) - c(2 * h)) / 3.0

    h = 1e-3
    checked = 0
    for i in range(tr.n):
        one = tr.take([i])
        _, u0, _ = orc.propagate(one, ar, md)
        scale = max(np.abs(grads["p0"][:, i]).max(), np.abs(grads["p1"][:, i]).max())
        for end in (0, 1):
            for c, comp in enumerate("xyz"):
                key = f"{comp}{end}"
                base = float(one.arrays()[key][0])
                moved = lambda v: Tracks(**{**one.arrays(), key: np.array([v])})
                if any((np.floor(orc.propagate(moved(base + s), ar, md)[1]) != np.floor(u0)).any()
                       for s in (-2 * h, 2 * h)):
                    continue
                fd = richardson(lambda v: _ep_loss(orc, moved(v), ar, md, g), base, h)
                an = grads["p0" if end == 0 else "p1"][c, i]
                assert abs(an - fd) <= 1e-6 * abs(fd) + 1e-7 * scale, (i, key, an, fd)
                checked += 1
    assert checked > 30
    hn = 1e-6 * md.n0m1
    keep = [i for i in range(tr.n)
            if all((np.floor(orc.propagate(tr.take([i]), ar, _with_n0(md, md.n0m1 + s))[1])
                    == np.floor(orc.propagate(tr.take([i]), ar, md)[1])).all() for s in (-2 * hn, 2 * hn))]
    sub = tr.take(keep)
    assert sub.n >= 5
    fd = richardson(lambda v: _ep_loss(orc, sub, ar, _with_n0(md, v), g), md.n0m1, hn)
    an = orc.endpoint_vjp(sub, ar, md, g)["n0m1"]
    assert an == pytest.approx(fd, rel=1e-5)


def test_endpoint_vjp_inside_the_cherenkov_cone(orc):
    """Dense medium (n = 1.5) with antennas inside and outside the cone of a
    fast track (signed Doppler factor on both sides): central differences of
    every coordinate of both ends."""
    md = Medium("uniform", 0.5, 8000.0)
    ang = np.radians([5.0, 20.0, 40.0, 60.0])
    dist = np.array([300.0, 310.7, 322.9, 337.3])
    pts = np.stack([dist * np.sin(ang), np.zeros_like(ang), -dist * np.cos(ang)], 1)
    tr = track_along((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), 2.0, 0.99, qw=-1.3)
    t_ar = 300.0 * 1.5 / C_LIGHT
    ar = antennas(pts, t_ar - 50.0123e-9, 0.05e-9, 4096)
    g = np.random.default_rng(3).normal(size=(ar.m, ar.n_bins, 3))
    grads = orc.endpoint_vjp(tr, ar, md, g)
    h = 1e-4
    _, u0, _ = orc.propagate(tr, ar, md)
    checked = 0
    for end in (0, 1):
        for c, comp in enumerate("xyz"):
            key = f"{comp}{end}"
            base = float(tr.arrays()[key][0])
            moved = lambda v: Tracks(**{**tr.arrays(), key: np.array([v])})
            if any((np.floor(orc.propagate(moved(base + s), ar, md)[1]) != np.floor(u0)).any()
                   for s in (-2 * h, 2 * h)):
                continue
            fd = (_ep_loss(orc, moved(base + h), ar, md, g) - _ep_loss(orc, moved(base - h), ar, md, g)) / (2 * h)
            an = grads["p0" if end == 0 else "p1"][c, 0]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(grads["p0"]).max()), key
            checked += 1
    assert checked >= 5


# ----------------------------------------------------------------- tabulated medium
_TAB = Medium("tabulated", 3.1e-4, 8000.0, (1.0, 0.83, 0.61, 0.64, 0.40, 0.21, 0.17), -200.0, 500.0)


def _tab_f(md, z):
    nodes = md.z0 + md.dz * np.arange(len(md.table))
    return float(np.interp(z, nodes, np.asarray(md.table)))


@pytest.mark.parametrize("zp,za", [(2_300.0, 0.0), (5_000.0, -900.0), (9_000.0, 2_500.0),
                                   (130.0, 20.0), (-500.0, -350.0), (1_800.0004, 1_800.0),
                                   (1_050.0, 1_300.0)])
def test_tabulated_index_is_path_mean(orc, zp, za):
    """Tabulated medium (piecewise-linear profile, constant beyond its nodes):
    n_eff = (t - T) c / R equals the mean of n(z) along the path by adaptive
    quadrature, across node boundaries, below the first and above the last
    node, inside one cell and in the |dz| < 1 mm branch."""
    md = _TAB
    p = np.array([80.0, 35.0, zp])
    x = np.array([-15.0, 10.0, za])
    tr = one_track(p, p + [0, 0, -1.0], (0, 0, -0.99), t0=2e-6)
    ar = antennas([x], 0.0, 1e-9, 10)
    t, _, _ = orc.propagate(tr, ar, md)
    r = float(np.linalg.norm(x - p))
    neff = (t[0, 0, 0] - 2e-6) * C_LIGHT / r
    if abs(zp - za) >= 1e-3:
        nodes = list(md.z0 + md.dz * np.arange(len(md.table)))
        lo, hi = min(za, zp), max(za, zp)
        mean = integrate.quad(lambda z: md.n0m1 * _tab_f(md, z), lo, hi, points=nodes, limit=200,
                              epsabs=0, epsrel=1e-13)[0] / (hi - lo)
    else:
        mean = md.n0m1 * _tab_f(md, 0.5 * (zp + za))
    assert (neff - 1.0) == pytest.approx(mean, rel=1e-9)


def test_tabulated_constant_profile_equals_uniform(orc):
    """f = 1 everywhere: the tabulated propagator and fields equal the uniform
    medium's up to rounding of the path integral."""
    w = config(0)
    tr = w.tracks(300)
    flat = Medium("tabulated", w.medium.n0m1, 8000.0, (1.0, 1.0), 0.0, 1000.0)
    t_u, _, b_u = orc.propagate(tr, w.array, w.medium)
    t_t, _, b_t = orc.propagate(tr, w.array, flat)
    assert np.allclose(t_t, t_u, rtol=4e-16, atol=0)
    assert (b_t != b_u).mean() < 1e-3
    for f in ("endpoint", "zhs"):
        a = orc.traces(f, tr, w.array, w.medium)
        b = orc.traces(f, tr, w.array, flat)
        assert np.linalg.norm(b - a) <= 1e-6 * np.linalg.norm(a)


def test_tabulated_exponential_samples_approach_closed_form(orc):
    """A 10-m table of exp(-z/h): its path means agree with the exponential
    closed form within the interpolation error (relative h^-2 dz^2 / 8)."""
    z = np.arange(0.0, 20_000.0 + 5.0, 10.0)
    md_t = Medium("tabulated", N0_AIR, 8000.0, tuple(np.exp(-z / 8000.0)), 0.0, 10.0)
    w = config(1)
    tr = w.tracks(200)
    t_e, _, _ = orc.propagate(tr, w.array, w.medium)
    t_t, _, _ = orc.propagate(tr, w.array, md_t)
    T = np.stack([tr.t0, tr.t1])[:, :, None]
    # (n_eff - 1) R / c differs by at most 1e-6 relative
    assert np.all(np.abs((t_t - T) - (t_e - T)) <= 2e-6 * N0_AIR * (t_e - T) + 1e-18)



# ----------------------------------------------------------------- spherical Earth
from paper_2309_03717_amd.workloads import EARTH_RADIUS, SPHERICAL_AIR  # noqa: E402


def _sph_height(q, re):
    """Height above the sphere written the plain way, |q - C| - re, in long
    double (a different expression from the oracle's)."""
    x, y, z = (np.longdouble(v) for v in q)
    re = np.longdouble(re)
    return float(np.sqrt(x * x + y * y + (z + re) * (z + re)) - re)


def _neff_from_time(orc, md, p, x):
    tr = one_track(p, np.asarray(p) + [0, 0, -1.0], (0, 0, -0.99), t0=2e-6)
    ar = antennas([x], 0.0, 1e-9, 10)
    t, _, _ = orc.propagate(tr, ar, md)
    r = float(np.linalg.norm(np.asarray(x, float) - np.asarray(p, float)))
    return (t[0, 0, 0] - 2e-6) * C_LIGHT / r


def test_gauss_legendre_rule(orc):
    """The oracle's quadrature is the 8-point Gauss-Legendre rule on [0, 1]:
    it integrates s^j exactly for j = 0..15 (evaluated exactly on its double
    nodes and weights: relative error within 2 ulp) and not s^16; and it agrees
    with numpy's rule moved to [0, 1] (nodes (1 + x) / 2, weights w / 2) within
    numpy's own accuracy."""
    from fractions import Fraction
    s, w = orc.gl_rule()
    assert s.shape == (8,) and np.all(np.diff(s) > 0) and np.all(w > 0)
    sf = [Fraction(float(v)) for v in s]
    wf = [Fraction(float(v)) for v in w]
    for j in range(17):
        moment = sum(wk * sk ** j for sk, wk in zip(sf, wf))
        rel = abs(float(moment * (j + 1) - 1))
        if j < 16:
            assert rel <= 2 * ULP, (j, rel)
        else:
            assert rel > 1e-10
    x, wx = np.polynomial.legendre.leggauss(8)
    assert np.allclose(s, (1.0 + x) / 2.0, rtol=1e-14, atol=0)
    assert np.allclose(w, wx / 2.0, rtol=1e-14, atol=0)


@pytest.mark.parametrize("p,x", [
    ((0.0, 0.0, 12_000.0), (0.0, 0.0, 0.0)),            # radial: H = z along the path
    ((300.0, -150.0, 8_000.0), (1_200.0, 400.0, 0.0)),   # a near-vertical shower pair
    ((60_000.0, 0.0, 9_000.0), (0.0, 0.0, 0.0)),         # inclined, 60 km away
    ((-150_000.0, 20_000.0, 20_000.0), (0.0, 0.0, 5.0)),  # far and high
    ((-50_000.0, 0.0, 0.0), (50_000.0, 0.0, 0.0)),       # a chord along the ground
    ((0.0, 0.0, 50.0), (100.0, 0.0, 1_500.0)),           # antenna above the emission
])
def test_spherical_index_is_path_mean(orc, p, x):
    """Spherical Earth: n_eff = (t - T) c / R equals the mean of
    1 + n0m1 exp(-H/h) along the straight path by adaptive quadrature, with H
    = |q - C| - re evaluated independently."""
    md = SPHERICAL_AIR
    neff = _neff_from_time(orc, md, p, x)
    p_, d = np.asarray(p, float), np.asarray(x, float) - np.asarray(p, float)
    f = lambda s: md.n0m1 * math.exp(-_sph_height(p_ + s * d, md.earth_radius) / md.h)
    mean = integrate.quad(f, 0.0, 1.0, epsabs=0, epsrel=1e-13, limit=200)[0]
    assert (neff - 1.0) == pytest.approx(mean, rel=1e-9)


def test_spherical_chord_sees_the_ground_fall_away(orc):
    """A 100-km chord along z = 0 rises above the curved ground (H up to
    d^2 / (2 re) at its ends), so its mean index is below the flat 1 + n0m1:
    about 1 - d^2 / (6 re h) of it with d = 50 km."""
    md = SPHERICAL_AIR
    neff = _neff_from_time(orc, md, (-50_000.0, 0.0, 0.0), (50_000.0, 0.0, 0.0))
    approx = 1.0 - 50_000.0 ** 2 / (6 * EARTH_RADIUS * md.h)
    assert (neff - 1.0) / md.n0m1 == pytest.approx(approx, rel=2e-3)
    assert (neff - 1.0) / md.n0m1 < 0.995


def test_spherical_radial_and_flat_limits_equal_exponential(orc):
    """Along the vertical through the origin H = z, and for a huge radius the
    ground is flat: both reduce to the exponential closed form, to the
    quadrature's accuracy (bins may differ only at edges)."""
    w = config(1)
    tr = w.tracks(300)
    flat = Medium("spherical", N0_AIR, 8000.0, earth_radius=1e15)
    t_e, _, b_e = orc.propagate(tr, w.array, w.medium)
    t_f, _, b_f = orc.propagate(tr, w.array, flat)
    T = np.stack([tr.t0, tr.t1])[:, :, None]
    assert np.all(np.abs((t_f - T) - (t_e - T)) <= 1e-12 * N0_AIR * (t_e - T) + 4 * ULP * t_e)
    assert (b_f != b_e).mean() < 1e-3
    for zp in (500.0, 7_000.0, 15_000.0):
        n_s = _neff_from_time(orc, SPHERICAL_AIR, (0.0, 0.0, zp), (0.0, 0.0, 0.0))
        n_e = _neff_from_time(orc, EXPONENTIAL_AIR, (0.0, 0.0, zp), (0.0, 0.0, 0.0))
        assert (n_s - 1.0) == pytest.approx(n_e - 1.0, rel=1e-11)


def test_spherical_without_refractivity_is_vacuum_exactly(orc):
    """n0m1 = 0: every medium is vacuum; the spherical traces equal the
    uniform n = 1 traces bit for bit."""
    w = config(0)
    tr = w.tracks(200)
    vac_s = Medium("spherical", 0.0, 8000.0, earth_radius=EARTH_RADIUS)
    vac_u = Medium("uniform", 0.0, 8000.0)
    for f in ("endpoint", "zhs"):
        assert np.array_equal(orc.traces(f, tr, w.array, vac_s), orc.traces(f, tr, w.array, vac_u))


def test_spherical_rotation_about_the_vertical(orc):
    """The sphere is symmetric about the vertical through the origin: turning
    tracks and antennas by 90 degrees turns the fields with them."""
    w = config(1)
    tr = w.tracks(400)
    rot = Tracks(-tr.y0, tr.x0, tr.z0, tr.t0, -tr.y1, tr.x1, tr.z1, tr.t1, -tr.by, tr.bx, tr.bz,
                 tr.qw)
    a = w.array
    from paper_2309_03717_amd.workloads import AntennaArray
    ar = AntennaArray(-a.y, a.x.copy(), a.z.copy(), a.t_start, a.dt, a.n_bins)
    for f in ("endpoint", "zhs"):
        e0 = orc.traces(f, tr, a, SPHERICAL_AIR)
        e1 = orc.traces(f, rot, ar, SPHERICAL_AIR)
        turned = np.stack([-e0[..., 1], e0[..., 0], e0[..., 2]], axis=-1)
        assert np.abs(e0).max() > 0
        assert np.linalg.norm(e1 - turned) <= 1e-9 * np.linalg.norm(e0)


def test_spherical_endpoint_uses_the_height_above_the_sphere(orc):
    """Endpoint impulse of one far track end: D = 1 - n(P) beta.r with n(P)
    from the height above the sphere (not z), against a direct evaluation."""
    md = SPHERICAL_AIR
    p0 = np.array([-40_000.0, 3_000.0, 6_000.0])
    beta = np.array([0.70, -0.05, -0.70])
    tr = one_track(p0, p0 + 2.0 * beta / np.linalg.norm(beta), beta, t0=0.0)
    x = np.array([0.0, 0.0, 0.0])
    t, _, _ = orc.propagate(tr, antennas([x], 0.0, 1e-9, 10), md)
    dt = 0.2e-9
    ar = antennas([x], t[0, 0, 0] - 100.5 * dt, dt, 4096)   # the start lands mid-bin 100
    e = orc.traces("endpoint", tr, ar, md)
    d = x - p0
    r = np.linalg.norm(d)
    rhat = d / r
    n_src = 1.0 + md.n0m1 * math.exp(-_sph_height(p0, md.earth_radius) / md.h)
    doppler = 1.0 - n_src * float(beta @ rhat)
    v = rhat * float(beta @ rhat) - beta
    expect = v / (doppler * r * dt)
    assert np.allclose(e[0, 100], expect, rtol=1e-12, atol=0)
    # with n taken at z instead the value differs clearly
    n_flat = 1.0 + md.n0m1 * math.exp(-p0[2] / md.h)
    wrong = v / ((1.0 - n_flat * float(beta @ rhat)) * r * dt)
    assert not np.allclose(e[0, 100], wrong, rtol=1e-9, atol=0)


@pytest.mark.parametrize("formalism", ["endpoint", "zhs"])
def test_spherical_adjoints_on_far_tracks(orc, formalism):
    """Inclined shower over the spherical Earth (emission points 2-40 km out
    along a 75-degree axis): the horizontal components of the path-index and
    source-index gradients matter there. Central differences of the forward
    oracle in x, y and z of both ends (Richardson, h = 1e-4 m), skipping
    shifts that move an arrival across a bin edge."""
    from paper_2309_03717_amd.workloads import SPHERICAL_AIR, inclined_shower
    md = SPHERICAL_AIR
    tr, ar = inclined_shower(300)
    _, u, b = orc.propagate(tr, ar, md)
    reach = np.flatnonzero(((b >= 0).any(axis=0)).any(axis=1))
    far = reach[np.argsort(-np.abs(tr.x0[reach]))][:8]
    tr = tr.take(far)
    g = np.random.default_rng(31).normal(size=(ar.m, ar.n_bins, 3))
    vjp = orc.endpoint_vjp if formalism == "endpoint" else orc.zhs_vjp
    grads = vjp(tr, ar, md, g)
    loss = lambda t: float(np.sum(g * orc.traces(formalism, t, ar, md)))

    def richardson(f, x0, h):
        c = lambda s: (f(x0 + s) - f(x0 - s)) / (2 * s)
        return (4.0 * c(h) - c(2 * h)) / 3.0

    h = 1e-4
    checked = 0
    for i in range(tr.n):
        one = tr.take([i])
        _, u0, _ = orc.propagate(one, ar, md)
        scale = max(np.abs(grads["p0"][:, i]).max(), np.abs(grads["p1"][:, i]).max())
        for end in (0, 1):
            for c, comp in enumerate("xyz"):
                key = f"{comp}{end}"
                base = float(one.arrays()[key][0])
                moved = lambda v: Tracks(**{**one.arrays(), key: np.array([v])})
                if any((np.floor(orc.propagate(moved(base + s), ar, md)[1]) != np.floor(u0)).any()
                       for s in (-2 * h, 2 * h)):
                    continue
                fd = richardson(lambda v: loss(moved(v)), base, h)
                an = grads["p0" if end == 0 else "p1"][c, i]
                # the loss sums 64 antennas x 8192 bins: its rounding noise
                # over h is ~1e-6 of the track's largest gradient component
                assert abs(an - fd) <= 1e-5 * abs(fd) + 1e-6 * scale, (i, key, an, fd)
                checked += 1
    assert checked >= 20


def test_oracle_rounding_against_50_digit_evaluation(orc):
    """The oracle's FP64 arrival times are within 4 ulp of the same definition
    evaluated with 50 significant digits (mpmath, exact inputs), its bins are
    the 50-digit floor unless an arrival lies within 1e-9 bins of an edge, and
    each Endpoint impulse is within 1e-11 relative of its 50-digit value. A
    pin of the FP64 evaluation order and rounding (the formulas themselves are
    pinned by the closed forms and quadratures above)."""
    import mpmath as mp
    mp.mp.dps = 50
    w = config(1)
    md = w.medium                                     # exponential
    tr = w.tracks(8)
    pts = np.array([[25.0, 0.0, 0.0], [0.0, -300.0, 35.0], [212.0, 212.0, 120.0],
                    [-480.0, 60.0, 0.0005]])          # antennas at four heights
    t_start = np.array([w.array.t_start[0]] * 4)
    arr = antennas(pts, t_start, w.array.dt, w.array.n_bins)
    t_orc, u_orc, b_orc = orc.propagate(tr, arr, md)
    c = mp.mpf(C_LIGHT)
    n0m1, h = mp.mpf(md.n0m1), mp.mpf(md.h)
    dt = mp.mpf(arr.dt)
    nb = arr.n_bins
    F = lambda v: mp.mpf(float(v))

    def neff(zp, za):
        if abs(zp - za) >= mp.mpf("1e-3"):
            return 1 + n0m1 * h * (mp.exp(-za / h) - mp.exp(-zp / h)) / (zp - za)
        return 1 + n0m1 * mp.exp(-(zp + za) / (2 * h))

    ends = [("x0", "y0", "z0", "t0"), ("x1", "y1", "z1", "t1")]
    impulses = {}
    for e, (fx, fy, fz, ft) in enumerate(ends):
        for i in range(tr.n):
            p = [F(getattr(tr, f)[i]) for f in (fx, fy, fz)]
            T = F(getattr(tr, ft)[i])
            beta = [F(getattr(tr, f)[i]) for f in ("bx", "by", "bz")]
            for a in range(arr.m):
                x = [F(arr.x[a]), F(arr.y[a]), F(arr.z[a])]
                d = [x[k] - p[k] for k in range(3)]
                r = mp.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
                t = T + neff(p[2], x[2]) * r / c
                u = (t - F(arr.t_start[a])) / dt
                tf = float(t_orc[e, i, a])
                assert abs(mp.mpf(tf) - t) <= 4 * np.spacing(abs(tf)), (e, i, a)
                k = int(mp.floor(u))
                near_edge = abs(u - mp.nint(u)) < mp.mpf("1e-9")
                want = k if 0 <= u < nb else -1
                if not near_edge:
                    assert int(b_orc[e, i, a]) == want, (e, i, a, float(u))
                if want >= 0:
                    rhat = [v / r for v in d]
                    br = sum(beta[k2] * rhat[k2] for k2 in range(3))
                    nsrc = 1 + n0m1 * mp.exp(-p[2] / h)
                    D = 1 - nsrc * br
                    s = 1 if e == 0 else -1
                    qw = F(tr.qw[i])
                    E = [s * qw * (rhat[k2] * br - beta[k2]) / (D * r * dt) for k2 in range(3)]
                    impulses.setdefault((i, a), []).append((want, E))
    checked = 0
    for i in range(tr.n):
        got = orc.traces("endpoint", tr.take([i]), arr, md, k=1.0)
        for a in range(arr.m):
            want = {}
            for k, E in impulses.get((i, a), []):
                acc = want.setdefault(k, [mp.mpf(0)] * 3)
                for k2 in range(3):
                    acc[k2] += E[k2]
            nz = set(np.nonzero(np.any(got[a] != 0, axis=1))[0].tolist())
            assert nz <= set(want), (i, a)
            for k, E in want.items():
                scale = max(abs(v) for v in E)
                if scale == 0:
                    continue
                for k2 in range(3):
                    assert abs(mp.mpf(float(got[a, k, k2])) - E[k2]) <= mp.mpf("1e-11") * scale, \
                        (i, a, k, k2)
                checked += 1
    assert checked >= 16
