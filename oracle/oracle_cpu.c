/*
 * FP64 CPU oracle for gridding / degridding, plain C with OpenMP over channels.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests (as a faster twin of the numpy
 * oracle for large checks) and timed by the benchmark's CPU-baseline leg.  It
 * shares no code with the HIP library.
 *
 * It restates the same definitions as oracle.py:
 *   Section 5, Eq. (1): G = sum_i f(r) V_i delta(u - u_i, v - v_i), f zero beyond
 *   its support; computed as the C scatter the paper describes (each visibility
 *   adds its weighted values to the patch of pixels it covers).
 * The sampled kernel table tab[OS][W] is an input (built by oracle.py), rows are
 * phases r0..r0+OS-1 and columns taps t0..t0+W-1 with
 *   odd W:  r0 = -(OS/2), t0 = -(W-1)/2 ;  even W: r0 = 0, t0 = -W/2+1.
 *
 * Layouts: uvw [B][T][3] metres; vis, model [C][B][T] complex (re, im) float32 in,
 * double out; weights [C][B][T] float32; grids [C][N][N] complex double.
 * A sample is valid iff its weight is non-zero and all taps are on the grid.
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <string.h>

static const double C_LIGHT = 299792458.0;

typedef struct {
  int64_t cx, cy, rx, ry;
  int valid;
} sample_t;

static void snap(double u, double v, double s, int N, int W, int OS, float w, sample_t *o) {
  double x = u * s + N / 2.0;
  double y = v * s + N / 2.0;
  double xo = floor(x * OS + 0.5);
  double yo = floor(y * OS + 0.5);
  o->valid = 0;
  if (!(fabs(xo) < 1073741824.0) || !(fabs(yo) < 1073741824.0)) return;  /* also catches NaN */
  int64_t xs = (int64_t)xo, ys = (int64_t)yo;
  int64_t r0 = (W % 2) ? -(OS / 2) : 0;
  int64_t t0 = (W % 2) ? -(W - 1) / 2 : -(W / 2) + 1;
  /* floor division of (xs - r0) by OS */
  int64_t qx = xs - r0, qy = ys - r0;
  int64_t cx = (qx >= 0) ? qx / OS : -((-qx + OS - 1) / OS);
  int64_t cy = (qy >= 0) ? qy / OS : -((-qy + OS - 1) / OS);
  o->cx = cx; o->cy = cy; o->rx = xs - cx * OS; o->ry = ys - cy * OS;
  o->valid = (w != 0.0f) && cx + t0 >= 0 && cx + t0 + W - 1 <= N - 1 &&
             cy + t0 >= 0 && cy + t0 + W - 1 <= N - 1;
}

/* G_out[c] = grid of channel c (all C channels), overwritten. */
void orc_grid(int C, int B, int T, const double *uvw, const double *freq, const float *vis,
              const float *wts, int N, double du, int W, int OS, const double *tab, int conj,
              double *G_out) {
  int64_t r0 = (W % 2) ? -(OS / 2) : 0;
  int64_t t0 = (W % 2) ? -(W - 1) / 2 : -(W / 2) + 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < C; ++c) {
    double *G = G_out + (int64_t)c * N * N * 2;
    memset(G, 0, sizeof(double) * (size_t)N * N * 2);
    double s = freq[c] / (C_LIGHT * du);
    for (int copy = 0; copy <= conj; ++copy) {
      double sg = copy ? -1.0 : 1.0;
      for (int64_t i = 0; i < (int64_t)B * T; ++i) {
        int64_t idx = (int64_t)c * B * T + i;
        sample_t sm;
        snap(sg * uvw[i * 3], sg * uvw[i * 3 + 1], s, N, W, OS, wts[idx], &sm);
        if (!sm.valid) continue;
        double ar = (double)wts[idx] * vis[idx * 2];
        double ai = (double)wts[idx] * vis[idx * 2 + 1] * (copy ? -1.0 : 1.0);
        const double *ky = tab + (sm.ry - r0) * W;
        const double *kx = tab + (sm.rx - r0) * W;
        for (int jy = 0; jy < W; ++jy) {
          double *row = G + ((sm.cy + t0 + jy) * N + (sm.cx + t0)) * 2;
          for (int jx = 0; jx < W; ++jx) {
            double k = ky[jy] * kx[jx];
            row[jx * 2] += ar * k;
            row[jx * 2 + 1] += ai * k;
          }
        }
      }
    }
  }
}

/* M_out [C][B][T] complex double; 0 for invalid samples.  G_in [C][N][N] complex double. */
void orc_degrid(int C, int B, int T, const double *uvw, const double *freq, const float *wts,
                int N, double du, int W, int OS, const double *tab, const double *G_in,
                double *M_out) {
  int64_t r0 = (W % 2) ? -(OS / 2) : 0;
  int64_t t0 = (W % 2) ? -(W - 1) / 2 : -(W / 2) + 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < C; ++c) {
    const double *G = G_in + (int64_t)c * N * N * 2;
    double s = freq[c] / (C_LIGHT * du);
    for (int64_t i = 0; i < (int64_t)B * T; ++i) {
      int64_t idx = (int64_t)c * B * T + i;
      sample_t sm;
      snap(uvw[i * 3], uvw[i * 3 + 1], s, N, W, OS, wts[idx], &sm);
      double mr = 0.0, mi = 0.0;
      if (sm.valid) {
        const double *ky = tab + (sm.ry - r0) * W;
        const double *kx = tab + (sm.rx - r0) * W;
        for (int jy = 0; jy < W; ++jy) {
          const double *row = G + ((sm.cy + t0 + jy) * N + (sm.cx + t0)) * 2;
          for (int jx = 0; jx < W; ++jx) {
            double k = ky[jy] * kx[jx];
            mr += k * row[jx * 2];
            mi += k * row[jx * 2 + 1];
          }
        }
      }
      M_out[idx * 2] = mr;
      M_out[idx * 2 + 1] = mi;
    }
  }
}

/* Fused residual step (no conjugate copy): M = degrid(G_in); r = V - M;
 * G_out = grid(r, w); chi2_per_chan[c] = sum w |r|^2.  Any output may be NULL except G_out. */
void orc_grid_degrid(int C, int B, int T, const double *uvw, const double *freq,
                     const float *vis, const float *wts, int N, double du, int W, int OS,
                     const double *tab, const double *G_in, double *M_out, double *G_out,
                     double *chi2_per_chan) {
  int64_t r0 = (W % 2) ? -(OS / 2) : 0;
  int64_t t0 = (W % 2) ? -(W - 1) / 2 : -(W / 2) + 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < C; ++c) {
    const double *Gi = G_in + (int64_t)c * N * N * 2;
    double *Go = G_out + (int64_t)c * N * N * 2;
    memset(Go, 0, sizeof(double) * (size_t)N * N * 2);
    double s = freq[c] / (C_LIGHT * du);
    double chi2 = 0.0;
    for (int64_t i = 0; i < (int64_t)B * T; ++i) {
      int64_t idx = (int64_t)c * B * T + i;
      sample_t sm;
      snap(uvw[i * 3], uvw[i * 3 + 1], s, N, W, OS, wts[idx], &sm);
      double mr = 0.0, mi = 0.0;
      if (sm.valid) {
        const double *ky = tab + (sm.ry - r0) * W;
        const double *kx = tab + (sm.rx - r0) * W;
        for (int jy = 0; jy < W; ++jy) {
          const double *row = Gi + ((sm.cy + t0 + jy) * N + (sm.cx + t0)) * 2;
          for (int jx = 0; jx < W; ++jx) {
            double k = ky[jy] * kx[jx];
            mr += k * row[jx * 2];
            mi += k * row[jx * 2 + 1];
          }
        }
        double w = wts[idx];
        double rr = vis[idx * 2] - mr, ri = vis[idx * 2 + 1] - mi;
        chi2 += w * (rr * rr + ri * ri);
        double ar = w * rr, ai = w * ri;
        for (int jy = 0; jy < W; ++jy) {
          double *row = Go + ((sm.cy + t0 + jy) * N + (sm.cx + t0)) * 2;
          for (int jx = 0; jx < W; ++jx) {
            double k = ky[jy] * kx[jx];
            row[jx * 2] += ar * k;
            row[jx * 2 + 1] += ai * k;
          }
        }
      }
      if (M_out) {
        M_out[idx * 2] = mr;
        M_out[idx * 2 + 1] = mi;
      }
    }
    if (chi2_per_chan) chi2_per_chan[c] = chi2;
  }
}

int orc_num_threads(void) {
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
}

/* Thread count of the parallel loops above (the timed CPU baseline runs once on
 * every host core and once on a single core). */
void orc_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
