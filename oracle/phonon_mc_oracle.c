/*
 * phonon_mc_oracle.c -- plain FP64 CPU reference of the phonon Monte Carlo
 * of the wire domain (phonon paragraph and coupling paragraph of Hao, Zhao,
 * Xiao and Kronenfeld, arXiv:1707.09073).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite may load it (it is built
 * into the same liboracle.so as the electron reference, whose Philox it
 * calls); the GPU library shares no code with it.
 *
 * What it computes (the readings are listed in the design notes):
 *  - three identical acoustic branches (sine dispersion) on a grid of
 *    frequency bins: per bin the group velocity v_b, the heat capacity C_b
 *    (J/(m^3 K), all three branches, the bin's width included) and the
 *    relaxation rate 1/tau_b at the linearisation temperature;
 *  - energy-based deviational phonon packets in the steady state: the heat
 *    generated per subcell (the hot electrons' net phonon emission, handed
 *    from the non-propagating LO phonons to the acoustic branches in place)
 *    is split into N packets of equal power P/N, P the sum of |q_c| over the
 *    subcells; a subcell where absorption outweighs emission is a sink and
 *    its packets carry negative energy; each packet starts in a
 *    subcell drawn by |q_c|, with a bin drawn from C_b / tau_b (the
 *    distribution relaxation re-emits) and an isotropic direction, flies
 *    for exponential times of mean tau_b, and at each scattering takes a new
 *    bin from C_b / tau_b and a new isotropic direction; it ends at an
 *    isothermal face;
 *  - faces: specular (symmetry planes A and B), diffuse (adiabatic free
 *    surfaces, cosine-law re-emission), isothermal (absorbing);
 *  - the track-length estimator: the energy of subcell c is P/N times the
 *    signed total time packets spend in it, and its temperature rise that
 *    energy over C_v V_c (C_v = sum of C_b).
 *
 * Random numbers: Philox4x32-10 with counter (packet, event, sub, tag).
 * Event 0 is the emission: sub 0 the subcell and position, sub 1 the bin,
 * direction and first free time.  Scattering event j >= 1: sub 0 the new
 * bin, direction and free time.  The h-th diffuse wall hit (h >= 1) during
 * the flight that follows event j: sub 1 + h.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

#define PH_PI 3.14159265358979323846

enum { PH_SPECULAR = 0, PH_DIFFUSE = 1, PH_ISOTHERMAL = 2 };

typedef struct {
  double L_nm[3];
  int n_cells[3];
  int face[6]; /* x0, x1, y0, y1, z0, z1 */
  int n_bins;
  uint64_t seed;
  uint32_t instance;
  int max_events; /* scatterings plus wall reflections per packet; a packet past it is counted and dropped */
} or_ph_config;

typedef struct {
  uint64_t scatterings, wall_specular, wall_diffuse, absorbed[6], dropped;
  uint64_t segments; /* straight flight pieces: each ends at a cell boundary, a scattering or a face */
  double path_nm;
} or_ph_counts;

static double u01(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

static void ph_rng(const or_ph_config *c, uint32_t pk, uint32_t ev, uint32_t sub, uint32_t w[4]) {
  uint32_t ctr[4] = {pk, ev, sub, (c->instance << 4) | 5u};
  uint32_t key[2] = {(uint32_t)(c->seed & 0xffffffffu), (uint32_t)(c->seed >> 32)};
  or_philox(ctr, key, w);
}

/* first index i with u * total < cum[i] (cum nondecreasing, cum[n-1] = total) */
static int draw(const double *cum, int n, double u) {
  double x = u * cum[n - 1];
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (x < cum[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

static void iso_dir(double u1, double u2, double d[3]) {
  double mu = 2.0 * u1 - 1.0, s = sqrt(fmax(0.0, 1.0 - mu * mu)), ph = 2.0 * PH_PI * u2;
  d[0] = s * cos(ph);
  d[1] = s * sin(ph);
  d[2] = mu;
}

/* Run n_packets packets of the source `q_cell` (W per subcell, either sign)
 * with the bin tables v (nm/fs), cumulative re-emission weights (C_b / tau_b,
 * summed in bin order) and tau (fs).  Adds each subcell's signed packet time
 * (fs; a packet from a subcell with q < 0 counts negative) to t_cell and the
 * event counts to cnt; pk_events (may be NULL) receives each packet's number
 * of scatterings. */
void or_ph_run(const or_ph_config *c, const double *q_cell, const double *v_nmfs, const double *tau_fs,
               const double *cum_emit, long n_packets, int n_threads, double *t_cell, or_ph_counts *cnt,
               uint32_t *pk_events) {
  const int nx = c->n_cells[0], ny = c->n_cells[1], nz = c->n_cells[2], nc = nx * ny * nz, nb = c->n_bins;
  const double d[3] = {c->L_nm[0] / nx, c->L_nm[1] / ny, c->L_nm[2] / nz};
  const int nn[3] = {nx, ny, nz};
  double *cum_cell = malloc(sizeof(double) * nc);
  double acc = 0.0;
  for (int i = 0; i < nc; ++i) { acc += fabs(q_cell[i]); cum_cell[i] = acc; }
#ifdef _OPENMP
  int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
  int nt = 1;
  (void)n_threads;
#endif
  double *tt = calloc((size_t)nt * nc, sizeof(double));
  or_ph_counts *tc = calloc(nt, sizeof(or_ph_counts));
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(dynamic, 64)
#endif
  for (long pk = 0; pk < n_packets; ++pk) {
#ifdef _OPENMP
    int th = omp_get_thread_num();
#else
    int th = 0;
#endif
    double *T = tt + (size_t)th * nc;
    or_ph_counts *C = tc + th;
    uint32_t w[4];
    ph_rng(c, (uint32_t)pk, 0u, 0u, w);
    int cell = draw(cum_cell, nc, u01(w[0]));
    const double sg = q_cell[cell] < 0.0 ? -1.0 : 1.0; /* the packet's sign */
    int ic[3] = {cell / (ny * nz), (cell / nz) % ny, cell % nz};
    double r[3] = {(ic[0] + u01(w[1])) * d[0], (ic[1] + u01(w[2])) * d[1], (ic[2] + u01(w[3])) * d[2]};
    ph_rng(c, (uint32_t)pk, 0u, 1u, w);
    int b = draw(cum_emit, nb, u01(w[0]));
    double dir[3];
    iso_dir(u01(w[1]), u01(w[2]), dir);
    double left = -log(u01(w[3])) * tau_fs[b] * v_nmfs[b]; /* free path to the next scattering, nm */
    uint32_t ev = 0, hits = 0;
    long events = 0; /* scatterings and wall reflections, against the guard */
    for (;;) {
      /* distance to the next cell boundary along each axis */
      double tmin = left;
      int ax = -1;
      for (int a = 0; a < 3; ++a) {
        if (dir[a] > 0.0) {
          double s = ((ic[a] + 1) * d[a] - r[a]) / dir[a];
          if (s < tmin) { tmin = s; ax = a; }
        } else if (dir[a] < 0.0) {
          double s = (ic[a] * d[a] - r[a]) / dir[a];
          if (s < tmin) { tmin = s; ax = a; }
        }
      }
      if (tmin < 0.0) tmin = 0.0;
      C->segments++;
      const int cc = (ic[0] * ny + ic[1]) * nz + ic[2];
      T[cc] += sg * (tmin / v_nmfs[b]);
      C->path_nm += tmin;
      for (int a = 0; a < 3; ++a) r[a] += tmin * dir[a];
      left -= tmin;
      if (ax < 0) {
        /* scattering: a new bin and direction, a new free path */
        if (++events > c->max_events) { C->dropped++; break; }
        ++ev;
        C->scatterings++;
        hits = 0;
        ph_rng(c, (uint32_t)pk, ev, 0u, w);
        b = draw(cum_emit, nb, u01(w[0]));
        iso_dir(u01(w[1]), u01(w[2]), dir);
        left = -log(u01(w[3])) * tau_fs[b] * v_nmfs[b];
        continue;
      }
      /* the boundary of axis ax: the cell beyond, or a face */
      const int up = dir[ax] > 0.0;
      r[ax] = (ic[ax] + up) * d[ax];
      const int nxt = ic[ax] + (up ? 1 : -1);
      if (nxt >= 0 && nxt < nn[ax]) { ic[ax] = nxt; continue; }
      const int f = 2 * ax + up;
      if (c->face[f] == PH_ISOTHERMAL) { C->absorbed[f]++; break; }
      if (++events > c->max_events) { C->dropped++; break; }
      if (c->face[f] == PH_SPECULAR) {
        C->wall_specular++;
        dir[ax] = -dir[ax];
      } else {
        /* cosine-law re-emission into the domain */
        C->wall_diffuse++;
        ++hits;
        ph_rng(c, (uint32_t)pk, ev, 1u + hits, w);
        double ct = sqrt(u01(w[0])), st = sqrt(fmax(0.0, 1.0 - ct * ct)), ph = 2.0 * PH_PI * u01(w[1]);
        int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
        dir[ax] = up ? -ct : ct;
        dir[a1] = st * cos(ph);
        dir[a2] = st * sin(ph);
      }
    }
    if (pk_events) pk_events[pk] = ev;
  }
  for (int th = 0; th < nt; ++th) {
    for (int i = 0; i < nc; ++i) t_cell[i] += tt[(size_t)th * nc + i];
    or_ph_counts *s = tc + th;
    cnt->scatterings += s->scatterings; cnt->wall_specular += s->wall_specular;
    cnt->wall_diffuse += s->wall_diffuse; cnt->dropped += s->dropped; cnt->path_nm += s->path_nm;
    cnt->segments += s->segments;
    for (int f = 0; f < 6; ++f) cnt->absorbed[f] += s->absorbed[f];
  }
  free(tt);
  free(tc);
  free(cum_cell);
}
