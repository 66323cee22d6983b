/*
 * radio_oracle.c -- plain, slow FP64 CPU oracle of the radio-emission loop.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline of the benchmark load this library. The product path never calls
 * it, and it shares no code, header, helper or constant table with the HIP
 * implementation.
 *
 * What it computes (§2, "Overview of the radio module", and Fig. 1): a
 * particle track is handed to a formalism, which loops over every antenna of
 * the array; for each (track, antenna) a propagator gives the emission path
 * (distance R, effective refractive index n_eff, arrival time) and the field
 * is computed and stored in that antenna's time trace. The two formalisms are
 * the Endpoint and the ZHS formalism (§1). The paper names them but prints
 * no formula; the expressions below are their far-field (Lienard-Wiechert)
 * forms:
 *
 *   Endpoint: at each track end, with sign s = +1 at the start and -1 at the
 *   stop, an impulse  E = s k qw [r x (r x beta)] / ((1 - n_src beta.r) R dt)
 *   lands in the bin of that end's arrival time.
 *
 *   ZHS: the vector potential of the whole segment is a box in time between
 *   the arrival times of its two ends, of time integral
 *   k qw beta_perp (T1 - T0) / R_mid, spread exactly over the bins it covers.
 *
 * k is the unit prefactor (e / (4 pi eps0 c) in SI, 1 in tests), dt the bin
 * width. Every function below is the plain definition, evaluated in double
 * precision, one (track, antenna) pair at a time.
 *
 * The timing chain (distance, n_eff, arrival time, bin) follows one fixed
 * operation order, because the bin index it yields must be reproduced exactly
 * by any other implementation of the same definition:
 *     d = X - P;  R = sqrt((dx*dx + dy*dy) + dz*dz)
 *     n_eff = 1 + n0m1                                   (uniform medium)
 *     n_eff = 1 + (n0m1*h) * ((eX - eP) / (zP - zX))     (exponential,
 *             e = exp(-(z / h)), |zP - zX| >= 1e-3 m)
 *     n_eff = 1 + n0m1 * exp(-(((zP + zX) * 0.5) / h))   (|zP - zX| < 1e-3 m)
 *     t = T + (n_eff * R) * (1 / c);   u = (t - t_start) * (1 / dt)
 *     in the window iff 0 <= u < n_bins; bin = floor(u)
 *
 * Parallel structure (§4): antennas are split into bunches handed to worker
 * threads. An antenna's trace depends on that antenna alone and its tracks
 * are always visited in order, so the result is bit-identical for any thread
 * count or bunch size (§5, Figs. 6 and 7).
 *
 * Media: uniform, exponential (the closed forms above) and tabulated: n(z) =
 * 1 + n0m1 f(z) with f piecewise linear through equally spaced nodes, whose
 * path mean is the exact integral of f over the path divided by its height
 * difference, evaluated in a fixed operation order (tab_F) that is part of
 * the timing chain. Spherical Earth: n = 1 + n0m1 exp(-H/h) with H the height
 * above a sphere of radius re touching z = 0 at the origin; its path mean has
 * no closed form and is the 8-point Gauss-Legendre quadrature along the
 * straight path, in the fixed order of spherical_index (also part of the
 * timing chain).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_VERSION 2
#define ORC_C_LIGHT 299792458.0 /* m/s, exact by definition of the metre */

typedef struct {
  int64_t n;
  const double *x0, *y0, *z0, *t0; /* start point (m) and time (s) */
  const double *x1, *y1, *z1, *t1; /* end point and time */
  const double *bx, *by, *bz;      /* velocity in units of c */
  const double *qw;                /* charge (units of e) times weight */
} orc_tracks;

typedef struct {
  int64_t m;
  const double *x, *y, *z; /* antenna positions (m) */
  const double *t_start;   /* time of the left edge of bin 0 (s) */
  double dt;               /* bin width (s) */
  int32_t n_bins;
} orc_antennas;

typedef struct {
  int32_t kind;  /* 0: uniform n = 1 + n0m1; 1: exponential n = 1 + n0m1 exp(-z/h);
                    2: tabulated n = 1 + n0m1 f(z) */
  double n0m1;   /* refractivity scale (at z = 0 for the exponential profile) */
  double h;      /* scale height (m), exponential only */
  /* tabulated only: f(z) is piecewise linear through f[i] at z0 + i dz
   * (i = 0 .. n_f - 1, n_f >= 2) and constant beyond the first and last node */
  const double *f;
  int32_t n_f;
  double z0, dz;
  double re;     /* 3, spherical Earth: n = 1 + n0m1 exp(-H/h), H the height above the
                    sphere of radius re (m) centred at (0, 0, -re) */
} orc_medium;

int orc_version(void) { return ORC_VERSION; }

/* ------------------------------------------------------------------ medium */

/* Tabulated profile: f(z), interpolated linearly between nodes. */
static double tab_f(const orc_medium *md, double z) {
  double t = (z - md->z0) * (1.0 / md->dz);
  int64_t last = md->n_f - 1;
  if (!(t > 0.0)) return md->f[0];
  if (t >= (double)last) return md->f[last];
  int64_t i = (int64_t)floor(t);
  double w = t - (double)i;
  return md->f[i] + w * (md->f[i + 1] - md->f[i]);
}

/* Tabulated profile: F(z), the integral of f from z0 to z, exact for the
 * piecewise-linear f: trapezoids of the whole cells below z, summed from the
 * first node up, plus the part of z's own cell; linear with slope f[0] below
 * z0 and f[last] above the last node. */
static double tab_F(const orc_medium *md, double z) {
  const double *f = md->f;
  const double dz = md->dz;
  int64_t last = md->n_f - 1;
  double t = (z - md->z0) * (1.0 / dz);
  if (!(t > 0.0)) return f[0] * (z - md->z0);
  int64_t i = t >= (double)last ? last : (int64_t)floor(t);
  double acc = 0.0;
  for (int64_t j = 1; j <= i; ++j) acc += (0.5 * dz) * (f[j - 1] + f[j]);
  if (i == last) return acc + f[last] * (z - (md->z0 + (double)last * dz));
  double w = t - (double)i;
  return acc + dz * (w * f[i] + (0.5 * w * w) * (f[i + 1] - f[i]));
}

/* Spherical Earth, centre C = (0, 0, -re). For a point q, rho2 = |q - C|^2 -
 * re^2 = (x^2 + y^2) + z (z + 2 re), and the height above the sphere is
 * |q - C| - re = rho2 / (|q - C| + re): the same number without subtracting
 * two radii. Returned: that height over the scale height h, with one
 * division. */
static double sphere_exponent(const orc_medium *md, double rho2) {
  return rho2 / ((sqrt(rho2 + md->re * md->re) + md->re) * md->h);
}

static double sphere_rho2(const orc_medium *md, double x, double y, double z) {
  return (x * x + y * y) + z * (z + (md->re + md->re));
}

/* The 8-point Gauss-Legendre rule moved from [-1, 1] to [0, 1]: nodes s_k =
 * (1 + x_k) / 2 in ascending order and weights w_k = 1 / ((1 - x_k^2)
 * P8'(x_k)^2) (half the classical ones, so that they sum to 1), x_k the roots
 * of the Legendre polynomial P8. Each root is found on its own by Newton's
 * method in long double, from the estimate -cos(pi (k + 3/4) / (8 + 1/2)),
 * with P8 and P7 from Bonnet's recurrence (j+1) P_{j+1} = (2j+1) x P_j -
 * j P_{j-1} and P8' = 8 (P7 - x P8) / (1 - x^2). */
#define ORC_GL 8
static double gl_node[ORC_GL], gl_weight[ORC_GL];
static pthread_once_t gl_once = PTHREAD_ONCE_INIT;

static void legendre8(long double x, long double *p8, long double *p7) {
  long double prev = 1.0L, cur = x;
  for (int j = 1; j < ORC_GL; ++j) {
    long double next = ((2 * j + 1) * x * cur - j * prev) / (j + 1);
    prev = cur;
    cur = next;
  }
  *p8 = cur;
  *p7 = prev;
}

static void gl_init(void) {
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int k = 0; k < ORC_GL; ++k) {
    long double x = -cosl(pi * (k + 0.75L) / (ORC_GL + 0.5L)), p8, p7, d;
    for (int it = 0; it < 100; ++it) {
      legendre8(x, &p8, &p7);
      d = ORC_GL * (p7 - x * p8) / (1.0L - x * x);
      long double step = p8 / d;
      x -= step;
      if (fabsl(step) < 1e-20L) break;
    }
    legendre8(x, &p8, &p7);
    d = ORC_GL * (p7 - x * p8) / (1.0L - x * x);
    gl_node[k] = (double)((1.0L + x) * 0.5L);
    gl_weight[k] = (double)(1.0L / ((1.0L - x * x) * d * d));
  }
}

/* The rule itself (for its pins): nodes and weights, ORC_GL of each. */
int orc_gl_rule(double *s, double *w) {
  pthread_once(&gl_once, gl_init);
  for (int k = 0; k < ORC_GL; ++k) {
    s[k] = gl_node[k];
    w[k] = gl_weight[k];
  }
  return ORC_GL;
}

/* Path mean of n from the emission point P to the antenna X over the
 * spherical Earth: 1 + n0m1 sum_k w_k exp(-H(q_k) / h) at the nodes q_k = P +
 * s_k (X - P), the terms added in ascending s_k. Along the line rho2 is a
 * quadratic in s: rho2(P + s d) = rho2(P) + s (2 (P - C).d + s d.d). */
static double spherical_index(const orc_medium *md, double px, double py, double pz, double ax,
                              double ay, double az) {
  pthread_once(&gl_once, gl_init);
  double dx = ax - px, dy = ay - py, dz = az - pz;
  double c0 = sphere_rho2(md, px, py, pz);
  double c1 = 2.0 * ((px * dx + py * dy) + (pz + md->re) * dz);
  double c2 = (dx * dx + dy * dy) + dz * dz;
  double sum = 0.0;
  for (int k = 0; k < ORC_GL; ++k) {
    double s = gl_node[k];
    sum = sum + gl_weight[k] * exp(-sphere_exponent(md, c0 + s * (c1 + s * c2)));
  }
  return 1.0 + md->n0m1 * sum;
}

/* Local refractive index n(z) at the emission point (§2: the propagator is
 * built from an environment; media of varying properties, §1). */
static double index_at(const orc_medium *md, double z) {
  if (md->kind == 0) return 1.0 + md->n0m1;
  if (md->kind == 2) return 1.0 + md->n0m1 * tab_f(md, z);
  return 1.0 + md->n0m1 * exp(-(z / md->h));
}

/* Effective index of the straight path from height zp to height za: the mean
 * of n(z) along the line, which for the exponential profile is
 * 1 + n0m1 * h * (exp(-za/h) - exp(-zp/h)) / (zp - za). */
static double effective_index(const orc_medium *md, double zp, double za) {
  if (md->kind == 0) return 1.0 + md->n0m1;
  double dz = zp - za;
  if (md->kind == 2) {   /* the mean of n along the path, from the integral F */
    if (fabs(dz) >= 1e-3) return 1.0 + md->n0m1 * ((tab_F(md, zp) - tab_F(md, za)) / dz);
    return 1.0 + md->n0m1 * tab_f(md, (zp + za) * 0.5);
  }
  if (fabs(dz) >= 1e-3) {
    double ep = exp(-(zp / md->h));
    double ea = exp(-(za / md->h));
    return 1.0 + (md->n0m1 * md->h) * ((ea - ep) / dz);
  }
  return 1.0 + md->n0m1 * exp(-(((zp + za) * 0.5) / md->h));
}

/* ------------------------------------------------------------- propagator */

typedef struct {
  double dx, dy, dz; /* antenna minus emission point */
  double r;          /* distance */
  double t;          /* arrival time */
  double u;          /* arrival time in bins from the window start */
} path;

/* Straight-line propagator (§2, Listing 2: the "simple" radio propagator):
 * emission at point (px,py,pz) and time tp, received at antenna a. */
static path propagate(const orc_antennas *ar, const orc_medium *md, int64_t a,
                      double px, double py, double pz, double tp) {
  const double inv_c = 1.0 / ORC_C_LIGHT;
  const double inv_dt = 1.0 / ar->dt;
  path p;
  p.dx = ar->x[a] - px;
  p.dy = ar->y[a] - py;
  p.dz = ar->z[a] - pz;
  p.r = sqrt((p.dx * p.dx + p.dy * p.dy) + p.dz * p.dz);
  double neff = md->kind == 3 ? spherical_index(md, px, py, pz, ar->x[a], ar->y[a], ar->z[a])
                              : effective_index(md, pz, ar->z[a]);
  p.t = tp + (neff * p.r) * inv_c;
  p.u = (p.t - ar->t_start[a]) * inv_dt;
  return p;
}

/* A tabulated medium needs at least two nodes and a positive spacing; the
 * exponential profiles a positive scale height; the sphere a radius of at
 * least 1 km. */
static int medium_ok(const orc_medium *md) {
  if (md->kind == 2) return md->f && md->n_f >= 2 && md->dz > 0.0;
  if (md->kind == 3) return md->h > 0.0 && md->re >= 1000.0 && isfinite(md->re);
  if (md->kind == 1) return md->h > 0.0;
  return md->kind == 0;
}

/* Bin of u, or -1 outside [0, n_bins) (NaN is outside). */
static int64_t bin_of(double u, int32_t n_bins) {
  if (u >= 0.0 && u < (double)n_bins) return (int64_t)floor(u);
  return -1;
}

/* ------------------------------------------------------------- formalisms */

/* A track with any non-finite field (position, time, velocity or weight)
 * contributes nothing. */
static int track_is_finite(const orc_tracks *tr, int64_t i) {
  return isfinite(tr->x0[i]) && isfinite(tr->y0[i]) && isfinite(tr->z0[i]) &&
         isfinite(tr->t0[i]) && isfinite(tr->x1[i]) && isfinite(tr->y1[i]) &&
         isfinite(tr->z1[i]) && isfinite(tr->t1[i]) && isfinite(tr->bx[i]) &&
         isfinite(tr->by[i]) && isfinite(tr->bz[i]) && isfinite(tr->qw[i]);
}

/* Endpoint formalism, one (track, antenna) pair: an impulse at each end. */
static void endpoint_pair(const orc_tracks *tr, int64_t i, const orc_antennas *ar,
                          const orc_medium *md, int64_t a, double k, double *trace) {
  if (!track_is_finite(tr, i)) return;
  for (int end = 0; end < 2; ++end) {
    double px = end ? tr->x1[i] : tr->x0[i];
    double py = end ? tr->y1[i] : tr->y0[i];
    double pz = end ? tr->z1[i] : tr->z0[i];
    double tp = end ? tr->t1[i] : tr->t0[i];
    double s = end ? -1.0 : 1.0;
    path p = propagate(ar, md, a, px, py, pz, tp);
    int64_t kb = bin_of(p.u, ar->n_bins);
    if (kb < 0 || p.r == 0.0) continue;
    double rx = p.dx / p.r, ry = p.dy / p.r, rz = p.dz / p.r;
    double bx = tr->bx[i], by = tr->by[i], bz = tr->bz[i];
    double bdotr = (bx * rx + by * ry) + bz * rz;
    double n_src = md->kind == 3
                       ? 1.0 + md->n0m1 * exp(-sphere_exponent(md, sphere_rho2(md, px, py, pz)))
                       : index_at(md, pz);
    double doppler = 1.0 - n_src * bdotr; /* signed */
    if (doppler == 0.0) continue;
    /* r x (r x beta) = r (beta.r) - beta */
    double vx = rx * bdotr - bx, vy = ry * bdotr - by, vz = rz * bdotr - bz;
    double amp = s * k * tr->qw[i] / (doppler * p.r * ar->dt);
    trace[3 * kb + 0] += amp * vx;
    trace[3 * kb + 1] += amp * vy;
    trace[3 * kb + 2] += amp * vz;
  }
}

/* Geometry of the ZHS segment as seen from antenna a: the time integral
 * I = k qw beta_perp (T1 - T0) / R_mid (returned per component), where the
 * distance and direction are taken at the segment midpoint; kq = k qw.
 * Returns 0 if the antenna sits on the midpoint. */
static int zhs_integral(const orc_tracks *tr, int64_t i, const orc_antennas *ar, int64_t a,
                        double kq, double integral[3]) {
  double mx = (tr->x0[i] + tr->x1[i]) * 0.5;
  double my = (tr->y0[i] + tr->y1[i]) * 0.5;
  double mz = (tr->z0[i] + tr->z1[i]) * 0.5;
  double dx = ar->x[a] - mx, dy = ar->y[a] - my, dz = ar->z[a] - mz;
  double rm = sqrt((dx * dx + dy * dy) + dz * dz);
  if (rm == 0.0) return 0;
  double rx = dx / rm, ry = dy / rm, rz = dz / rm;
  double bx = tr->bx[i], by = tr->by[i], bz = tr->bz[i];
  double bdotr = (bx * rx + by * ry) + bz * rz;
  double c = kq * (tr->t1[i] - tr->t0[i]) / rm;
  integral[0] = c * (bx - bdotr * rx);
  integral[1] = c * (by - bdotr * ry);
  integral[2] = c * (bz - bdotr * rz);
  return 1;
}

/* ZHS formalism, one pair: the box between the two arrival times, averaged
 * over each bin it overlaps (bin value = integral * overlap / width / dt). */
static void zhs_pair(const orc_tracks *tr, int64_t i, const orc_antennas *ar,
                     const orc_medium *md, int64_t a, double k, double *trace) {
  if (!track_is_finite(tr, i)) return;
  path ps = propagate(ar, md, a, tr->x0[i], tr->y0[i], tr->z0[i], tr->t0[i]);
  path pe = propagate(ar, md, a, tr->x1[i], tr->y1[i], tr->z1[i], tr->t1[i]);
  double ulo = ps.u < pe.u ? ps.u : pe.u;
  double uhi = ps.u < pe.u ? pe.u : ps.u;
  double nb = (double)ar->n_bins;
  if (!(uhi >= 0.0 && ulo < nb)) return; /* no overlap with the window (or NaN) */
  double integral[3];
  if (!zhs_integral(tr, i, ar, a, k * tr->qw[i], integral)) return;
  double klo = floor(ulo), khi = floor(uhi);
  if (klo == khi) { /* the whole box inside one bin */
    int64_t j = (int64_t)klo;
    if (j >= 0 && j < ar->n_bins)
      for (int c = 0; c < 3; ++c) trace[3 * j + c] += integral[c] / ar->dt;
    return;
  }
  double width = uhi - ulo;
  int64_t j0 = klo < 0.0 ? 0 : (int64_t)klo;
  int64_t j1 = khi >= nb ? ar->n_bins - 1 : (int64_t)khi;
  for (int64_t j = j0; j <= j1; ++j) {
    double left = ulo > (double)j ? ulo : (double)j;
    double right = uhi < (double)(j + 1) ? uhi : (double)(j + 1);
    double overlap = right - left;
    if (overlap <= 0.0) continue;
    for (int c = 0; c < 3; ++c) trace[3 * j + c] += integral[c] / ar->dt * (overlap / width);
  }
}

/* ------------------------------------------------------------ the loop */

typedef struct {
  int formalism;
  const orc_tracks *tr;
  const orc_antennas *ar;
  const orc_medium *md;
  double k;
  double *traces;
  int64_t bunch;
  int n_workers;
  int worker;
} loop_job;

/* Worker: antenna bunches worker, worker + n_workers, ... (§4: each task
 * computes the response of a bunch of antennas). For each antenna, all
 * tracks in order. */
static void *loop_worker(void *arg) {
  loop_job *job = (loop_job *)arg;
  int64_t m = job->ar->m;
  int64_t n_bunches = (m + job->bunch - 1) / job->bunch;
  size_t trace_len = (size_t)job->ar->n_bins * 3;
  for (int64_t b = job->worker; b < n_bunches; b += job->n_workers) {
    int64_t a_end = (b + 1) * job->bunch < m ? (b + 1) * job->bunch : m;
    for (int64_t a = b * job->bunch; a < a_end; ++a) {
      double *trace = job->traces + (size_t)a * trace_len;
      for (int64_t i = 0; i < job->tr->n; ++i) {
        if (job->formalism == 0)
          endpoint_pair(job->tr, i, job->ar, job->md, a, job->k, trace);
        else
          zhs_pair(job->tr, i, job->ar, job->md, a, job->k, trace);
      }
    }
  }
  return NULL;
}

/* Traces [m][n_bins][3] (components x, y, z), accumulated (+=) over every
 * (track, antenna) pair. formalism: 0 Endpoint (electric field, V/m with SI
 * k), 1 ZHS (vector potential, V s / m). n_threads >= 1 workers take antenna
 * bunches of `bunch` antennas (bunch <= 0: ceil(m / n_threads)).
 * Returns 0, or -1 on invalid arguments. */
int orc_traces(int formalism, const orc_tracks *tr, const orc_antennas *ar, const orc_medium *md,
               double k, double *traces, int n_threads, int64_t bunch) {
  if (!tr || !ar || !md || !traces || (formalism != 0 && formalism != 1)) return -1;
  if (ar->m < 0 || tr->n < 0 || ar->n_bins < 0 || !(ar->dt > 0.0) || !medium_ok(md)) return -1;
  if (ar->m == 0 || tr->n == 0 || ar->n_bins == 0) return 0;
  if (n_threads < 1) n_threads = 1;
  if (bunch <= 0) bunch = (ar->m + n_threads - 1) / n_threads;
  loop_job *jobs = (loop_job *)calloc((size_t)n_threads, sizeof(loop_job));
  pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  if (!jobs || !th) { free(jobs); free(th); return -1; }
  for (int w = 0; w < n_threads; ++w) {
    loop_job j = {formalism, tr, ar, md, k, traces, bunch, n_threads, w};
    jobs[w] = j;
  }
  int started = 0;
  for (int w = 1; w < n_threads; ++w)
    if (pthread_create(&th[w], NULL, loop_worker, &jobs[w]) == 0) ++started; else break;
  loop_worker(&jobs[0]);
  for (int w = 1; w <= started; ++w) pthread_join(th[w], NULL);
  /* workers that failed to start: run their share here */
  for (int w = started + 1; w < n_threads; ++w) loop_worker(&jobs[w]);
  free(jobs);
  free(th);
  return 0;
}

/* The propagator alone, for every (end, track, antenna): arrival time t,
 * window coordinate u and bin (-1 outside the window), each stored at index
 * (end * n + i) * m + a. Any output pointer may be NULL. */
int orc_propagate(const orc_tracks *tr, const orc_antennas *ar, const orc_medium *md,
                  double *t_out, double *u_out, int32_t *bin_out) {
  if (!tr || !ar || !md || !(ar->dt > 0.0) || !medium_ok(md)) return -1;
  for (int end = 0; end < 2; ++end)
    for (int64_t i = 0; i < tr->n; ++i)
      for (int64_t a = 0; a < ar->m; ++a) {
        path p = end ? propagate(ar, md, a, tr->x1[i], tr->y1[i], tr->z1[i], tr->t1[i])
                     : propagate(ar, md, a, tr->x0[i], tr->y0[i], tr->z0[i], tr->t0[i]);
        size_t o = ((size_t)end * (size_t)tr->n + (size_t)i) * (size_t)ar->m + (size_t)a;
        if (t_out) t_out[o] = p.t;
        if (u_out) u_out[o] = p.u;
        if (bin_out) bin_out[o] = (int32_t)bin_of(p.u, ar->n_bins);
      }
  return 0;
}

/* ---------------------------------------------------------- ZHS adjoint */

/* Integral of the piecewise-constant upstream gradient g (one component,
 * stride 3, zero outside [0, n_bins)) from 0 to u. */
static double cumulative(const double *g, int32_t n_bins, double u) {
  if (!(u > 0.0)) return 0.0;
  double acc = 0.0;
  int64_t full = u >= (double)n_bins ? n_bins : (int64_t)floor(u);
  for (int64_t j = 0; j < full; ++j) acc += g[3 * j];
  if (full < n_bins) acc += (u - (double)full) * g[3 * full];
  return acc;
}

static double value_at(const double *g, int32_t n_bins, double u) {
  if (!(u >= 0.0 && u < (double)n_bins)) return 0.0;
  return g[3 * (int64_t)floor(u)];
}

/* Tabulated profile: slope of f at z (the cell z falls in, as tab_f takes it;
 * zero beyond the first and last node, where f is constant). */
static double tab_slope(const orc_medium *md, double z) {
  double t = (z - md->z0) * (1.0 / md->dz);
  int64_t last = md->n_f - 1;
  if (!(t > 0.0) || t >= (double)last) return 0.0;
  int64_t i = (int64_t)floor(t);
  return (md->f[i + 1] - md->f[i]) / md->dz;
}

/* Gradient of the path index n_eff(P, X) with respect to the emission point
 * P (out_grad) and its derivative with respect to n0m1 (out_dn0):
 *   exponential: n = 1 + n0m1 h (e_X - e_P) / (z_P - z_X);
 *   tabulated:   n = 1 + n0m1 (F(z_P) - F(z_X)) / (z_P - z_X), dF/dz = f;
 *   both with n = 1 + n0m1 (local factor at the mid height) below 1 mm;
 *   spherical:   n = 1 + n0m1 S, S = sum_k w_k exp(-H(q_k) / h), q_k = P +
 *                s_k (X - P), and dH(q)/dq = (q - C) / |q - C|, dq_k/dP = 1 - s_k. */
static void index_gradient(const orc_medium *md, double px, double py, double pz, double ax,
                           double ay, double az, double out_grad[3], double *out_dn0) {
  out_grad[0] = out_grad[1] = out_grad[2] = 0.0;
  if (md->kind == 0) {
    *out_dn0 = 1.0;
    return;
  }
  if (md->kind == 3) {
    pthread_once(&gl_once, gl_init);
    double sum = 0.0, g[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < ORC_GL; ++k) {
      double s = gl_node[k];
      double qz = pz + s * (az - pz);
      double q[3] = {px + s * (ax - px), py + s * (ay - py), qz + md->re};   /* q - C */
      double rho2 = sphere_rho2(md, q[0], q[1], qz);
      double len = sqrt(rho2 + md->re * md->re);                            /* |q - C| */
      double e = exp(-((rho2 / (len + md->re)) / md->h));
      sum += gl_weight[k] * e;
      for (int j = 0; j < 3; ++j) g[j] += gl_weight[k] * e * (1.0 - s) * q[j] / len;
    }
    for (int j = 0; j < 3; ++j) out_grad[j] = -md->n0m1 * g[j] / md->h;
    *out_dn0 = sum;
    return;
  }
  double del = pz - az;
  if (fabs(del) >= 1e-3) {
    if (md->kind == 2) {
      double fbar = (tab_F(md, pz) - tab_F(md, az)) / del;
      out_grad[2] = md->n0m1 * (tab_f(md, pz) - fbar) / del;
      *out_dn0 = fbar;
    } else {
      double h = md->h, ep = exp(-pz / h), ea = exp(-az / h);
      double f = (ea - ep) / del;
      /* d f / d zp = (ep / h) / del - (ea - ep) / del^2 */
      out_grad[2] = md->n0m1 * h * ((ep / h) / del - (ea - ep) / (del * del));
      *out_dn0 = h * f;
    }
  } else {
    double mid = (pz + az) * 0.5;
    if (md->kind == 2) {
      out_grad[2] = md->n0m1 * tab_slope(md, mid) * 0.5;
      *out_dn0 = tab_f(md, mid);
    } else {
      double e = exp(-mid / md->h);
      out_grad[2] = -md->n0m1 * e / (2.0 * md->h);
      *out_dn0 = e;
    }
  }
}

/* The local (source) index n(P) of the Endpoint Doppler factor, with its
 * gradient in P and its derivative in n0m1. */
static double source_index(const orc_medium *md, double px, double py, double pz,
                           double out_grad[3], double *out_dn0) {
  out_grad[0] = out_grad[1] = out_grad[2] = 0.0;
  if (md->kind == 0) {
    *out_dn0 = 1.0;
    return 1.0 + md->n0m1;
  }
  if (md->kind == 3) {
    double q[3] = {px, py, pz + md->re};   /* P - C */
    double rho2 = sphere_rho2(md, px, py, pz);
    double len = sqrt(rho2 + md->re * md->re);
    double e = exp(-((rho2 / (len + md->re)) / md->h));
    for (int j = 0; j < 3; ++j) out_grad[j] = -md->n0m1 * (e / md->h) * q[j] / len;
    *out_dn0 = e;
    return 1.0 + md->n0m1 * exp(-sphere_exponent(md, sphere_rho2(md, px, py, pz)));
  }
  if (md->kind == 2) {
    out_grad[2] = md->n0m1 * tab_slope(md, pz);
    *out_dn0 = tab_f(md, pz);
    return 1.0 + md->n0m1 * tab_f(md, pz);
  }
  double e = exp(-(pz / md->h));
  out_grad[2] = -md->n0m1 * e / md->h;
  *out_dn0 = e;
  return 1.0 + md->n0m1 * e;
}

/* d t / d P and d t / d n0m1 of the arrival t = T + n_eff R / c at antenna a:
 * dR/dP = -(X - P) / R. */
static void time_derivatives(const orc_antennas *ar, const orc_medium *md, int64_t a,
                             double px, double py, double pz, double out_dp[3], double *out_dn) {
  double dx = ar->x[a] - px, dy = ar->y[a] - py, dz = ar->z[a] - pz;
  double r = sqrt((dx * dx + dy * dy) + dz * dz);
  double neff = md->kind == 3 ? spherical_index(md, px, py, pz, ar->x[a], ar->y[a], ar->z[a])
                              : effective_index(md, pz, ar->z[a]);
  double gn[3], dn0;
  index_gradient(md, px, py, pz, ar->x[a], ar->y[a], ar->z[a], gn, &dn0);
  out_dp[0] = (neff * (-dx / r) + r * gn[0]) / ORC_C_LIGHT;
  out_dp[1] = (neff * (-dy / r) + r * gn[1]) / ORC_C_LIGHT;
  out_dp[2] = (neff * (-dz / r) + r * gn[2]) / ORC_C_LIGHT;
  *out_dn = r * dn0 / ORC_C_LIGHT;
}

typedef struct {
  const orc_tracks *tr;
  const orc_antennas *ar;
  const orc_medium *md;
  double k;
  const double *grad;
  double *g_qw, *g_p0, *g_p1, *g_n_track;
  int64_t i_begin, i_end;
} vjp_job;

/* Vector-Jacobian product of the ZHS traces, per track: for L = sum G * A
 * with A the ZHS definition above, the exact derivatives with respect to the
 * track weight qw, its two end points P0, P1 and the refractivity n0m1, with
 * beta and the emission times held fixed. Per pair, with Phi the integral of
 * G and g = (Phi(u_hi) - Phi(u_lo)) / (u_hi - u_lo) (or G at the bin when
 * both ends share a bin), the pair's share of L is sum_c I_c g_c / dt. */
static void *vjp_worker(void *arg) {
  vjp_job *job = (vjp_job *)arg;
  const orc_tracks *tr = job->tr;
  const orc_antennas *ar = job->ar;
  const orc_medium *md = job->md;
  const double inv_dt = 1.0 / ar->dt;
  size_t trace_len = (size_t)ar->n_bins * 3;
  for (int64_t i = job->i_begin; i < job->i_end; ++i) {
    double gq = 0.0, gp0[3] = {0, 0, 0}, gp1[3] = {0, 0, 0}, gn = 0.0;
    double bx = tr->bx[i], by = tr->by[i], bz = tr->bz[i];
    for (int64_t a = 0; a < ar->m && track_is_finite(tr, i); ++a) {
      path ps = propagate(ar, md, a, tr->x0[i], tr->y0[i], tr->z0[i], tr->t0[i]);
      path pe = propagate(ar, md, a, tr->x1[i], tr->y1[i], tr->z1[i], tr->t1[i]);
      int start_is_lo = ps.u < pe.u;
      double ulo = start_is_lo ? ps.u : pe.u;
      double uhi = start_is_lo ? pe.u : ps.u;
      if (!(uhi >= 0.0 && ulo < (double)ar->n_bins)) continue;
      double integral[3];
      if (!zhs_integral(tr, i, ar, a, job->k * tr->qw[i], integral)) continue;
      const double *g = job->grad + (size_t)a * trace_len;
      int same_bin = floor(ulo) == floor(uhi);
      double gbar[3], dl_dulo = 0.0, dl_duhi = 0.0;
      for (int c = 0; c < 3; ++c) {
        if (same_bin) {
          gbar[c] = value_at(g + c, ar->n_bins, ulo);
        } else {
          double w = uhi - ulo;
          gbar[c] = (cumulative(g + c, ar->n_bins, uhi) - cumulative(g + c, ar->n_bins, ulo)) / w;
          dl_duhi += integral[c] * inv_dt * (value_at(g + c, ar->n_bins, uhi) - gbar[c]) / w;
          dl_dulo += integral[c] * inv_dt * (gbar[c] - value_at(g + c, ar->n_bins, ulo)) / w;
        }
      }
      /* weight: I is linear in qw, so dL/dqw is the share of L at qw = 1 */
      double unit[3];
      zhs_integral(tr, i, ar, a, job->k, unit);
      for (int c = 0; c < 3; ++c) gq += unit[c] * inv_dt * gbar[c];
      /* midpoint geometry: I = K (beta/R - (beta.d) d / R^3), d = X - M */
      double mx = (tr->x0[i] + tr->x1[i]) * 0.5, my = (tr->y0[i] + tr->y1[i]) * 0.5,
             mz = (tr->z0[i] + tr->z1[i]) * 0.5;
      double d[3] = {ar->x[a] - mx, ar->y[a] - my, ar->z[a] - mz};
      double r = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
      double kk = job->k * tr->qw[i] * (tr->t1[i] - tr->t0[i]);
      double gam[3] = {gbar[0] * inv_dt, gbar[1] * inv_dt, gbar[2] * inv_dt};
      double b[3] = {bx, by, bz};
      double gb = gam[0] * b[0] + gam[1] * b[1] + gam[2] * b[2];
      double gd = gam[0] * d[0] + gam[1] * d[1] + gam[2] * d[2];
      double bd = b[0] * d[0] + b[1] * d[1] + b[2] * d[2];
      double r3 = r * r * r, r5 = r3 * r * r;
      for (int j = 0; j < 3; ++j) {
        double dl_dd = kk * (-gb * d[j] / r3 - gd * b[j] / r3 - bd * gam[j] / r3 +
                             3.0 * bd * gd * d[j] / r5);
        /* d = X - (P0 + P1)/2: dL/dP0 = dL/dP1 = -dL/dd / 2 */
        gp0[j] += -0.5 * dl_dd;
        gp1[j] += -0.5 * dl_dd;
      }
      /* box edges: u = (t - t_start) / dt */
      double dts_dp[3], dte_dp[3], dts_dn, dte_dn;
      time_derivatives(ar, md, a, tr->x0[i], tr->y0[i], tr->z0[i], dts_dp, &dts_dn);
      time_derivatives(ar, md, a, tr->x1[i], tr->y1[i], tr->z1[i], dte_dp, &dte_dn);
      double dl_dus = start_is_lo ? dl_dulo : dl_duhi;
      double dl_due = start_is_lo ? dl_duhi : dl_dulo;
      for (int j = 0; j < 3; ++j) {
        gp0[j] += dl_dus * inv_dt * dts_dp[j];
        gp1[j] += dl_due * inv_dt * dte_dp[j];
      }
      gn += dl_dus * inv_dt * dts_dn + dl_due * inv_dt * dte_dn;
    }
    job->g_qw[i] = gq;
    for (int j = 0; j < 3; ++j) {
      job->g_p0[(size_t)j * tr->n + i] = gp0[j];
      job->g_p1[(size_t)j * tr->n + i] = gp1[j];
    }
    job->g_n_track[i] = gn;
  }
  return NULL;
}

/* ZHS vector-Jacobian product. grad: upstream gradient [m][n_bins][3] of a
 * scalar loss with respect to the traces. Outputs (overwritten): g_qw[n],
 * g_p0[3][n], g_p1[3][n] (component-major) and the scalar g_n0m1.
 * n_threads workers take contiguous track ranges; the n0m1 gradient is
 * summed over tracks in index order, so the result does not depend on the
 * thread count. */
int orc_zhs_vjp(const orc_tracks *tr, const orc_antennas *ar, const orc_medium *md, double k,
                const double *grad, double *g_qw, double *g_p0, double *g_p1, double *g_n0m1,
                int n_threads) {
  if (!tr || !ar || !md || !grad || !g_qw || !g_p0 || !g_p1 || !g_n0m1) return -1;
  if (!(ar->dt > 0.0) || tr->n < 0 || ar->m < 0) return -1;
  *g_n0m1 = 0.0;
  if (tr->n == 0) return 0;
  double *gn = (double *)calloc((size_t)tr->n, sizeof(double));
  if (!gn) return -1;
  if (n_threads < 1) n_threads = 1;
  vjp_job *jobs = (vjp_job *)calloc((size_t)n_threads, sizeof(vjp_job));
  pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  if (!jobs || !th) { free(gn); free(jobs); free(th); return -1; }
  int64_t per = (tr->n + n_threads - 1) / n_threads;
  for (int w = 0; w < n_threads; ++w) {
    int64_t lo = (int64_t)w * per, hi = lo + per;
    if (lo > tr->n) lo = tr->n;
    if (hi > tr->n) hi = tr->n;
    vjp_job j = {tr, ar, md, k, grad, g_qw, g_p0, g_p1, gn, lo, hi};
    jobs[w] = j;
  }
  int started = 0;
  for (int w = 1; w < n_threads; ++w)
    if (pthread_create(&th[w], NULL, vjp_worker, &jobs[w]) == 0) ++started; else break;
  vjp_worker(&jobs[0]);
  for (int w = 1; w <= started; ++w) pthread_join(th[w], NULL);
  for (int w = started + 1; w < n_threads; ++w) vjp_worker(&jobs[w]);
  double s = 0.0;
  for (int64_t i = 0; i < tr->n; ++i) s += gn[i];
  *g_n0m1 = s;
  free(gn);
  free(jobs);
  free(th);
  return 0;
}

/* ----------------------------------------------------- Endpoint adjoint */

typedef struct {
  const orc_tracks *tr;
  const orc_antennas *ar;
  const orc_medium *md;
  double k;
  const double *grad;
  double *g_qw, *g_p0, *g_p1, *g_n_track;
  int64_t i_begin, i_end;
} ep_vjp_job;

/* Vector-Jacobian product of the Endpoint traces, per track: for
 * L = sum G * E with E the Endpoint definition above, the derivatives with
 * respect to qw, the two end points and n0m1, with beta and the emission
 * times fixed. The bin an impulse lands in is piecewise constant in these
 * parameters, so only the impulse value is differentiated: with r = d / R,
 * b = beta.r, D = 1 - n_src b, V = r b - beta and A = s k qw / dt, an end's
 * share of L is f = A (g.V) / (D R), g = G at its bin, and
 *   df/dd_j = A [ (g.dV/dd_j) / (D R) + n_src (g.V) (db/dd_j) / (D^2 R)
 *                 - (g.V) r_j / (D R^2) ],
 *   dr_i/dd_j = (delta_ij - r_i r_j) / R,  db/dd_j = (beta_j - b r_j) / R,
 *   df/dn_src = A (g.V) b / (D^2 R),
 * with d = X - P (so df/dP = -df/dd) and n_src = 1 + n0m1 e(z_P), whose
 * height derivative adds to the z component. */
static void *ep_vjp_worker(void *arg) {
  ep_vjp_job *job = (ep_vjp_job *)arg;
  const orc_tracks *tr = job->tr;
  const orc_antennas *ar = job->ar;
  const orc_medium *md = job->md;
  size_t trace_len = (size_t)ar->n_bins * 3;
  for (int64_t i = job->i_begin; i < job->i_end; ++i) {
    double gq = 0.0, gp[2][3] = {{0, 0, 0}, {0, 0, 0}}, gn = 0.0;
    double beta[3] = {tr->bx[i], tr->by[i], tr->bz[i]};
    for (int64_t a = 0; a < ar->m && track_is_finite(tr, i); ++a) {
      const double *g_a = job->grad + (size_t)a * trace_len;
      for (int end = 0; end < 2; ++end) {
        double px = end ? tr->x1[i] : tr->x0[i];
        double py = end ? tr->y1[i] : tr->y0[i];
        double pz = end ? tr->z1[i] : tr->z0[i];
        double tp = end ? tr->t1[i] : tr->t0[i];
        double s = end ? -1.0 : 1.0;
        path p = propagate(ar, md, a, px, py, pz, tp);
        int64_t kb = bin_of(p.u, ar->n_bins);
        if (kb < 0 || p.r == 0.0) continue;
        double R = p.r;
        double r[3] = {p.dx / R, p.dy / R, p.dz / R};
        double b = (beta[0] * r[0] + beta[1] * r[1]) + beta[2] * r[2];
        double gsrc[3], dsrc_dn0;
        double n_src = source_index(md, px, py, pz, gsrc, &dsrc_dn0);
        double D = 1.0 - n_src * b;
        if (D == 0.0) continue;
        double V[3] = {r[0] * b - beta[0], r[1] * b - beta[1], r[2] * b - beta[2]};
        const double *g = g_a + 3 * kb;
        double gV = g[0] * V[0] + g[1] * V[1] + g[2] * V[2];
        double gr = g[0] * r[0] + g[1] * r[1] + g[2] * r[2];
        double A = s * job->k * tr->qw[i] / ar->dt;
        /* weight: f is linear in qw */
        gq += s * job->k / ar->dt * gV / (D * R);
        for (int j = 0; j < 3; ++j) {
          double db = (beta[j] - b * r[j]) / R;
          /* g.dV/dd_j = sum_i g_i [ (delta_ij - r_i r_j) b / R + r_i db_j ] */
          double gdV = (g[j] - gr * r[j]) * b / R + gr * db;
          double df = A * (gdV / (D * R) + n_src * gV * db / (D * D * R) - gV * r[j] / (D * R * R));
          gp[end][j] -= df;
        }
        double df_dn = A * gV * b / (D * D * R);   /* through n_src */
        gn += df_dn * dsrc_dn0;
        for (int j = 0; j < 3; ++j) gp[end][j] += df_dn * gsrc[j];
      }
    }
    job->g_qw[i] = gq;
    for (int j = 0; j < 3; ++j) {
      job->g_p0[(size_t)j * tr->n + i] = gp[0][j];
      job->g_p1[(size_t)j * tr->n + i] = gp[1][j];
    }
    job->g_n_track[i] = gn;
  }
  return NULL;
}

/* Endpoint vector-Jacobian product; arguments and outputs as orc_zhs_vjp. */
int orc_endpoint_vjp(const orc_tracks *tr, const orc_antennas *ar, const orc_medium *md,
                     double k, const double *grad, double *g_qw, double *g_p0, double *g_p1,
                     double *g_n0m1, int n_threads) {
  if (!tr || !ar || !md || !grad || !g_qw || !g_p0 || !g_p1 || !g_n0m1) return -1;
  if (!(ar->dt > 0.0) || tr->n < 0 || ar->m < 0) return -1;
  *g_n0m1 = 0.0;
  if (tr->n == 0) return 0;
  double *gn = (double *)calloc((size_t)tr->n, sizeof(double));
  if (!gn) return -1;
  if (n_threads < 1) n_threads = 1;
  ep_vjp_job *jobs = (ep_vjp_job *)calloc((size_t)n_threads, sizeof(ep_vjp_job));
  pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  if (!jobs || !th) { free(gn); free(jobs); free(th); return -1; }
  int64_t per = (tr->n + n_threads - 1) / n_threads;
  for (int w = 0; w < n_threads; ++w) {
    int64_t lo = (int64_t)w * per, hi = lo + per;
    if (lo > tr->n) lo = tr->n;
    if (hi > tr->n) hi = tr->n;
    ep_vjp_job j = {tr, ar, md, k, grad, g_qw, g_p0, g_p1, gn, lo, hi};
    jobs[w] = j;
  }
  int started = 0;
  for (int w = 1; w < n_threads; ++w)
    if (pthread_create(&th[w], NULL, ep_vjp_worker, &jobs[w]) == 0) ++started; else break;
  ep_vjp_worker(&jobs[0]);
  for (int w = 1; w <= started; ++w) pthread_join(th[w], NULL);
  for (int w = started + 1; w < n_threads; ++w) ep_vjp_worker(&jobs[w]);
  double sum = 0.0;
  for (int64_t i = 0; i < tr->n; ++i) sum += gn[i];
  *g_n0m1 = sum;
  free(gn);
  free(jobs);
  free(th);
  return 0;
}
