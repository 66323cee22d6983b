/* Drives every entry point of the CPU oracle (radio_oracle.c) on small
 * inputs, for the address and undefined-behaviour sanitizer build of
 * tests/test_oracle_sanitizers.py: all four media, both formalisms' traces
 * on one and on several threads, the propagator and both adjoints, with
 * tracks that are non-finite, of zero length, or sit exactly on an antenna.
 * Exits non-zero if any call rejects its arguments. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int64_t n;
  const double *x0, *y0, *z0, *t0, *x1, *y1, *z1, *t1, *bx, *by, *bz, *qw;
} orc_tracks;
typedef struct {
  int64_t m;
  const double *x, *y, *z, *t_start;
  double dt;
  int32_t n_bins;
} orc_antennas;
typedef struct {
  int32_t kind;
  double n0m1, h;
  const double *f;
  int32_t n_f;
  double z0, dz, re;
} orc_medium;

int orc_traces(int formalism, const orc_tracks *tr, const orc_antennas *ar, const orc_medium *md,
               double k, double *traces, int n_threads, int64_t bunch);
int orc_propagate(const orc_tracks *tr, const orc_antennas *ar, const orc_medium *md,
                  double *t_out, double *u_out, int32_t *bin_out);
int orc_zhs_vjp(const orc_tracks *tr, const orc_antennas *ar, const orc_medium *md, double k,
                const double *grad, double *g_qw, double *g_p0, double *g_p1, double *g_n0m1,
                int n_threads);
int orc_endpoint_vjp(const orc_tracks *tr, const orc_antennas *ar, const orc_medium *md,
                     double k, const double *grad, double *g_qw, double *g_p0, double *g_p1,
                     double *g_n0m1, int n_threads);

enum { N = 9, M = 4, B = 512 };

int main(void) {
  double x0[N], y0[N], z0[N], t0[N], x1[N], y1[N], z1[N], t1[N], bx[N], by[N], bz[N], qw[N];
  const double c = 299792458.0;
  for (int i = 0; i < N; ++i) {
    x0[i] = 10.0 * i - 40.0;
    y0[i] = 3.0 * i;
    z0[i] = 1000.0 + 50.0 * i;
    x1[i] = x0[i] + 0.1;
    y1[i] = y0[i];
    z1[i] = z0[i] - 2.0;
    bx[i] = 0.0;
    by[i] = 0.0;
    bz[i] = -0.95;
    qw[i] = i % 2 ? 1.0 : -1.0;
    t0[i] = (10000.0 - z0[i]) / c;
    t1[i] = t0[i] + 2.0 / (0.95 * c);
  }
  z0[1] = NAN;                 /* non-finite start */
  t1[2] = INFINITY;            /* non-finite time */
  x1[3] = x0[3]; y1[3] = y0[3]; z1[3] = z0[3]; t1[3] = t0[3];   /* a point */
  x0[4] = 0.0; y0[4] = 0.0; z0[4] = 0.0;                        /* on antenna 0 */
  const double ax[M] = {0.0, 100.0, -100.0, 30.0}, ay[M] = {0.0, 0.0, 50.0, -80.0};
  const double az[M] = {0.0, 0.0, 10.0, 0.0};
  double ts[M];
  for (int a = 0; a < M; ++a) ts[a] = (10000.0 - az[a]) / c * 1.0003 - 2e-7;
  orc_tracks tr = {N, x0, y0, z0, t0, x1, y1, z1, t1, bx, by, bz, qw};
  orc_antennas ar = {M, ax, ay, az, ts, 1e-9, B};
  double table[41];
  for (int i = 0; i < 41; ++i) table[i] = exp(-(500.0 * i) / 8000.0);
  orc_medium media[4] = {{0, 2.92e-4, 8000.0, NULL, 0, 0.0, 1.0, 0.0},
                         {1, 2.92e-4, 8000.0, NULL, 0, 0.0, 1.0, 0.0},
                         {2, 2.92e-4, 8000.0, table, 41, 0.0, 500.0, 0.0},
                         {3, 2.92e-4, 8000.0, NULL, 0, 0.0, 1.0, 6.371e6}};
  double *traces = calloc((size_t)M * B * 3, sizeof(double));
  double *grad = malloc((size_t)M * B * 3 * sizeof(double));
  double *t = malloc((size_t)2 * N * M * sizeof(double)), *u = malloc((size_t)2 * N * M * sizeof(double));
  int32_t *bin = malloc((size_t)2 * N * M * sizeof(int32_t));
  double gq[N], gp0[3 * N], gp1[3 * N], gn;
  for (int i = 0; i < M * B * 3; ++i) grad[i] = sin(0.37 * i);
  double sum = 0.0;
  int bad = 0;
  for (int k = 0; k < 4; ++k) {
    for (int f = 0; f < 2; ++f)
      for (int th = 1; th <= 3; th += 2) {
        for (int i = 0; i < M * B * 3; ++i) traces[i] = 0.0;
        bad |= orc_traces(f, &tr, &ar, &media[k], 1.0, traces, th, th == 1 ? 0 : 1) != 0;
        for (int i = 0; i < M * B * 3; ++i) sum += fabs(traces[i]);
      }
    bad |= orc_propagate(&tr, &ar, &media[k], t, u, bin) != 0;
    bad |= orc_zhs_vjp(&tr, &ar, &media[k], 1.0, grad, gq, gp0, gp1, &gn, 2) != 0;
    sum += fabs(gn);
    bad |= orc_endpoint_vjp(&tr, &ar, &media[k], 1.0, grad, gq, gp0, gp1, &gn, 2) != 0;
    sum += fabs(gn);
  }
  printf("oracle driver: %s, checksum %.6e\n", bad ? "a call failed" : "all calls ok", sum);
  free(traces);
  free(grad);
  free(t);
  free(u);
  free(bin);
  return bad;
}
