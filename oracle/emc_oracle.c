/*
 * emc_oracle.c -- plain, slow, FP64 CPU reference of the ensemble electron
 * Monte Carlo step of Hao, Zhao, Xiao and Kronenfeld, "Hybrid electrothermal
 * simulation of a three-dimensional fin-shaped field-effect transistor based
 * on GaN nanowires" (arXiv:1707.09073).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library shares
 * no code with it: no headers, helpers, tables or constants.
 *
 * What it follows (the paper has no section headings; passages are named):
 *  - electron MC paragraph: three valleys Gamma1, U, Gamma3; Kane dispersion
 *    E(1+aE) = hbar^2 k^2 / 2m; energy-dependent mass m(1+2aE); ionized
 *    impurity, polar optical, acoustic deformation-potential and intervalley
 *    scattering; all dopants active; half-nanowire domain of 3x6x100
 *    subcells used to count electrons; Poisson refresh from the terminal
 *    voltages and the counted concentrations; heat counted per subcell.
 *  - phonon paragraph: the LO phonon at 91.2 meV is the hot-electron sink.
 *  - Table I: masses, valley offsets, nonparabolicity, dielectric constants,
 *    density, acoustic and intervalley deformation potentials.
 * The paper defers the rate formulas to its ref. [7]; the textbook
 * nonparabolic forms used here (Jacoboni & Reggiani 1983; Fawcett, Boardman
 * & Swain 1970; Brooks-Herring screening) and every other reading of a silent
 * point are listed in the design notes.
 *
 * Units inside the MC: E in eV, k in 1/nm, r in nm, t in fs, F in V/nm,
 * rates in 1/fs.  Rate formulas are evaluated in SI and converted.
 *
 * Pins: Philox against the published known-answer vectors; Kane and the DOS
 * against finite differences; every rate against its parabolic textbook limit
 * and against brute-force golden-rule quadrature; detailed balance; energy
 * conservation per event; the zero-field stationary mean energy; the Drude
 * transient; the Poisson solve against exact linear and manufactured
 * solutions.  Absolute device observables are "parity unpinned" (the paper
 * prints none).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 exact / recommended values, SI */
#define OR_QE 1.602176634e-19
#define OR_HBAR 1.054571817e-34
#define OR_M0 9.1093837015e-31
#define OR_KB 1.380649e-23
#define OR_EPS0 8.8541878128e-12
#define OR_PI 3.14159265358979323846

enum { OR_NV = 3, OR_NM = 10, OR_NF = 7 };
/* mechanism order used for the cumulative selection */
enum { OR_AC = 0, OR_II = 1, OR_POP_AB = 2, OR_POP_EM = 3, OR_IV0 = 4 };
/* per-cell factor slots */
enum { F_T = 0, F_FII = 1, F_NLO = 2, F_NLO1 = 3, F_NIV = 4, F_NIV1 = 5, F_B2 = 6 };

typedef struct {
  double m_eff[3], alpha[3], E_c[3];
  int Z[3];
  double eps_s, eps_inf, rho, D_ac_eV, D_iv_eVm, hw_lo_eV, hw_iv_eV, u_ac;
  int mode; /* 0 bulk, 1 device */
  int pad0;
  uint64_t seed;
  uint32_t instance;
  int n_particles, capacity;
  double dt_fs;
  int substeps;  /* sub-steps per flight interval (= per Poisson update) */
  int n_bins;
  double dE_eV;
  double T0_K, T_init_K, N_D_m3;
  double F_bulk[3];
  double L_nm[3];
  int n_cells[3];
  int pad1;
  double gate_x_nm[2];
  double Vgs, Vds, phi_offset;
} or_config;

typedef struct {
  uint64_t selections, self_events, overflow, real[OR_NV][OR_NM];
  uint64_t exits[2], injections[2];
  uint64_t reflect_guard;
} or_counts;

typedef struct {
  or_config c;
  int ncell, nx, ny, nz;
  double dx, dy, dz, Vc, w; /* cell size (nm), cell volume (nm^3), superparticle weight */
  /* rate shapes [v][b][m] (1/fs, per unit factor) and 4k^2 at bin midpoints [v][b] */
  double *shape, *k4;
  double *fac;   /* [cell][OR_NF] */
  double *Tcell; /* [cell] */
  double gamma[OR_NV];
  /* particles */
  double *k, *r; /* [cap][3] */
  int *valley, *alive;
  uint32_t *id;
  uint32_t next_id;
  uint32_t n_done; /* intervals completed */
  /* fields */
  double *phi, *field; /* [cell], [cell][3] */
  double *Lband;       /* banded Cholesky factor of the Poisson matrix */
  double *bc_rhs;      /* boundary contribution to the right-hand side (C) */
  int band;
  uint32_t *count;     /* electrons per cell after the last update */
  /* window tallies */
  uint64_t *heat;      /* [cell][4]: pop_em, pop_ab, iv_em, iv_ab */
  uint64_t *dens_sum;  /* [cell] */
  or_counts tot;
  uint32_t win_intervals;
  /* per-interval history, rows of 8 doubles (layout differs by mode; see
   * record_bulk and record_device) */
  double *hist;
  int hist_cap, hist_len;
  int err_capacity, err_nan;
  /* energy carried through the contacts (device mode): the total energy
   * (kinetic plus valley minimum, eV) of each electron that left in the
   * current interval, per slot, summed in slot order after the interval */
  double *eexit;
  signed char *xside; /* contact left through in this interval, -1 none */
  double e_exit[2], e_inj[2]; /* window sums, eV, source and drain */
  double *ework;              /* per slot: kinetic energy gained in free flight this interval, eV */
  double e_work;              /* window sum of ework, eV */
  double *eabs;               /* per slot: energy gained in phonon absorptions this interval, eV */
  double e_abs;               /* window sum of eabs, eV */
  double e_ens0;              /* ensemble total energy at the window start, eV */
} or_ctx;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): two multipliers, */
/* Weyl key schedule, ten rounds.                                       */
/* ------------------------------------------------------------------ */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* open-interval uniform in FP64: (w + 1/2) 2^-32 */
static double u01(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

static void rng(const or_ctx *X, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, uint32_t w[4]) {
  uint32_t ctr[4] = {c0, c1, c2, (X->c.instance << 4) | tag};
  uint32_t key[2] = {(uint32_t)(X->c.seed & 0xffffffffu), (uint32_t)(X->c.seed >> 32)};
  or_philox(ctr, key, w);
}

/* ------------------------------------------------------------------ */
/* Band model: Kane dispersion of the electron MC paragraph.           */
/* ------------------------------------------------------------------ */
static double ck(void) { return OR_HBAR * OR_HBAR / (2.0 * OR_M0 * OR_QE) * 1e18; } /* eV nm^2 */
static double cv(void) { return OR_HBAR / OR_M0 * 1e3; }                            /* nm^2/fs */
static double cf(void) { return OR_QE / OR_HBAR * 1e-15; }                          /* 1/(nm fs) per V/nm */

/* kinetic energy from gamma = E(1+aE): the positive root, written in the
 * form that stays finite for a = 0 */
double or_kane_energy(double gam, double a) { return 2.0 * gam / (1.0 + sqrt(1.0 + 4.0 * a * gam)); }

static double energy_of_k(const or_ctx *X, const double k[3], int v) {
  double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  return or_kane_energy(ck() * k2 / X->c.m_eff[v], X->c.alpha[v]);
}

/* group velocity hbar k / (m (1 + 2 a E)) in nm/fs */
static void velocity(const or_ctx *X, const double k[3], int v, double vel[3]) {
  double E = energy_of_k(X, k, v);
  double s = cv() / (X->c.m_eff[v] * (1.0 + 2.0 * X->c.alpha[v] * E));
  vel[0] = s * k[0]; vel[1] = s * k[1]; vel[2] = s * k[2];
}

/* ------------------------------------------------------------------ */
/* Scattering rates (SI, 1/s).  The paper lists the four mechanisms and  */
/* Table I; the formulas are the standard nonparabolic ones.             */
/* ------------------------------------------------------------------ */
/* density of states per spin per volume, 1/(J m^3), at kinetic energy E (eV) */
static double dos_si(const or_config *c, int v, double E) {
  if (E <= 0.0) return 0.0;
  double m = c->m_eff[v] * OR_M0;
  double gam = E * (1.0 + c->alpha[v] * E) * OR_QE; /* J */
  double f = 1.0 + 2.0 * c->alpha[v] * E;
  return pow(2.0 * m, 1.5) * sqrt(gam) * f / (4.0 * OR_PI * OR_PI * OR_HBAR * OR_HBAR * OR_HBAR);
}

double or_dos(const or_config *c, int v, double E) { return dos_si(c, v, E); }

static double bose(double hw_eV, double T) { return 1.0 / (exp(hw_eV * OR_QE / (OR_KB * T)) - 1.0); }

/* inverse screening length squared (Debye / Brooks-Herring), 1/m^2 */
static double beta2_si(const or_config *c, double T) {
  return OR_QE * OR_QE * c->N_D_m3 / (c->eps_s * OR_EPS0 * OR_KB * T);
}

/* acoustic deformation potential, elastic, equipartition */
static double w_ac(const or_config *c, int v, double E, double T) {
  double D = c->D_ac_eV * OR_QE;
  return 2.0 * OR_PI / OR_HBAR * D * D * OR_KB * T / (c->rho * c->u_ac * c->u_ac) * dos_si(c, v, E);
}

/* Brooks-Herring ionized impurity rate with the Kane k of energy E */
static double w_ii(const or_config *c, int v, double E, double T) {
  double eps = c->eps_s * OR_EPS0;
  double b2 = beta2_si(c, T);
  double gam = E * (1.0 + c->alpha[v] * E) * OR_QE;
  double kk = 2.0 * c->m_eff[v] * OR_M0 * gam / (OR_HBAR * OR_HBAR); /* k^2, 1/m^2 */
  double e4 = OR_QE * OR_QE * OR_QE * OR_QE;
  return 2.0 * OR_PI / OR_HBAR * c->N_D_m3 * e4 / (eps * eps) * dos_si(c, v, E) / (b2 * (b2 + 4.0 * kk));
}

/* Froehlich polar-optical rate with the nonparabolic overlap (Fawcett et al.)
 * without the phonon occupation factor; Ep is the final energy (eV) */
static double pop_core(const or_config *c, int v, double E, double Ep) {
  if (E <= 0.0 || Ep <= 0.0) return 0.0;
  double a = c->alpha[v];
  double g = E * (1.0 + a * E), gp = Ep * (1.0 + a * Ep); /* eV */
  double sg = sqrt(g), sgp = sqrt(gp);
  double A = 2.0 * (1.0 + a * E) * (1.0 + a * Ep) + a * (g + gp);
  A = A * A;
  double B = -2.0 * a * sg * sgp * (4.0 * (1.0 + a * E) * (1.0 + a * Ep) + a * (g + gp));
  double C = 4.0 * (1.0 + a * E) * (1.0 + a * Ep) * (1.0 + 2.0 * a * E) * (1.0 + 2.0 * a * Ep);
  double F0 = (A * log(fabs((sg + sgp) / (sg - sgp))) + B) / C;
  double w0 = c->hw_lo_eV * OR_QE / OR_HBAR;
  double m = c->m_eff[v] * OR_M0;
  double pref = OR_QE * OR_QE * w0 * sqrt(m) / (4.0 * sqrt(2.0) * OR_PI * OR_EPS0 * OR_HBAR) *
                (1.0 / c->eps_inf - 1.0 / c->eps_s);
  return pref * (1.0 + 2.0 * a * Ep) / sqrt(g * OR_QE) * F0;
}

/* intervalley deformation potential, v -> j, without occupation factor;
 * Ep is the final kinetic energy in valley j */
static double iv_core(const or_config *c, int v, int j, double Ep) {
  if (Ep <= 0.0) return 0.0;
  int Zp = (j == v) ? c->Z[v] - 1 : c->Z[j];
  if (Zp <= 0) return 0.0;
  double D = c->D_iv_eVm * OR_QE; /* J/m */
  double w = c->hw_iv_eV * OR_QE / OR_HBAR;
  return OR_PI * D * D * (double)Zp / (c->rho * w) * dos_si(c, j, Ep);
}

static double iv_final_energy(const or_config *c, int v, int j, int emit, double E) {
  return E + c->E_c[v] - c->E_c[j] + (emit ? -c->hw_iv_eV : c->hw_iv_eV);
}

/* analytic rate of mechanism m at energy E and lattice temperature T, 1/s */
double or_rate(const or_config *c, int v, int m, double E, double T) {
  if (E <= 0.0) return 0.0;
  if (m == OR_AC) return w_ac(c, v, E, T);
  if (m == OR_II) return w_ii(c, v, E, T);
  double N = bose(c->hw_lo_eV, T);
  if (m == OR_POP_AB) return N * pop_core(c, v, E, E + c->hw_lo_eV);
  if (m == OR_POP_EM) return (N + 1.0) * pop_core(c, v, E, E - c->hw_lo_eV);
  int j = (m - OR_IV0) / 2, emit = (m - OR_IV0) % 2;
  double Niv = bose(c->hw_iv_eV, T);
  return (emit ? Niv + 1.0 : Niv) * iv_core(c, v, j, iv_final_energy(c, v, j, emit, E));
}

/* ------------------------------------------------------------------ */
/* Rate tables on the 1 meV grid (value at each bin midpoint) and the   */
/* per-cell temperature factors.                                        */
/* ------------------------------------------------------------------ */
static void build_tables(or_ctx *X) {
  const or_config *c = &X->c;
  int nb = c->n_bins;
  for (int v = 0; v < OR_NV; ++v)
    for (int b = 0; b < nb; ++b) {
      double E = (b + 0.5) * c->dE_eV;
      double *S = X->shape + ((size_t)v * nb + b) * OR_NM;
      S[OR_AC] = w_ac(c, v, E, 1.0) * 1e-15;
      /* impurity: per unit (N_I / beta^2) with beta^2, 4k^2 in 1/nm^2 */
      {
        double eps = c->eps_s * OR_EPS0;
        double e4 = OR_QE * OR_QE * OR_QE * OR_QE;
        S[OR_II] = 2.0 * OR_PI / OR_HBAR * e4 / (eps * eps) * dos_si(c, v, E) * 1e-24;
      }
      S[OR_POP_AB] = pop_core(c, v, E, E + c->hw_lo_eV) * 1e-15;
      S[OR_POP_EM] = pop_core(c, v, E, E - c->hw_lo_eV) * 1e-15;
      for (int j = 0; j < OR_NV; ++j)
        for (int em = 0; em < 2; ++em)
          S[OR_IV0 + 2 * j + em] = iv_core(c, v, j, iv_final_energy(c, v, j, em, E)) * 1e-15;
      double gam = E * (1.0 + c->alpha[v] * E);
      X->k4[(size_t)v * nb + b] = 4.0 * gam * c->m_eff[v] / ck();
    }
}

static void cell_factors(or_ctx *X) {
  const or_config *c = &X->c;
  double NI_nm = c->N_D_m3 * 1e-27;
  for (int i = 0; i < X->ncell; ++i) {
    double T = X->Tcell[i];
    double *f = X->fac + (size_t)i * OR_NF;
    double b2 = beta2_si(c, T) * 1e-18;
    double N = bose(c->hw_lo_eV, T), Niv = bose(c->hw_iv_eV, T);
    f[F_T] = T;
    f[F_FII] = NI_nm / b2;
    f[F_NLO] = N;
    f[F_NLO1] = N + 1.0;
    f[F_NIV] = Niv;
    f[F_NIV1] = Niv + 1.0;
    f[F_B2] = b2;
  }
}

/* tabulated rate of mechanism m in cell factors f, 1/fs */
static double tab_term(const double *S, double k4, const double *f, int m) {
  switch (m) {
    case OR_AC: return f[F_T] * S[OR_AC];
    case OR_II: return (S[OR_II] * f[F_FII]) / (f[F_B2] + k4);
    case OR_POP_AB: return f[F_NLO] * S[OR_POP_AB];
    case OR_POP_EM: return f[F_NLO1] * S[OR_POP_EM];
    default: return (((m - OR_IV0) % 2) ? f[F_NIV1] : f[F_NIV]) * S[m];
  }
}

/* Gamma_v: the exact maximum of the tabulated total over bins and cells */
static void compute_gamma(or_ctx *X) {
  int nb = X->c.n_bins;
  for (int v = 0; v < OR_NV; ++v) {
    double g = 0.0;
    for (int i = 0; i < X->ncell; ++i) {
      const double *f = X->fac + (size_t)i * OR_NF;
      for (int b = 0; b < nb; ++b) {
        const double *S = X->shape + ((size_t)v * nb + b) * OR_NM;
        double k4 = X->k4[(size_t)v * nb + b];
        double cum = 0.0;
        for (int m = 0; m < OR_NM; ++m) cum += tab_term(S, k4, f, m);
        if (cum > g) g = cum;
      }
    }
    X->gamma[v] = g;
  }
}

/* ------------------------------------------------------------------ */
/* Geometry and the Poisson equation of the half nanowire.              */
/* ------------------------------------------------------------------ */
static int cell_index(const or_ctx *X, int ix, int iy, int iz) { return (ix * X->ny + iy) * X->nz + iz; }

static int cell_of(const or_ctx *X, const double r[3]) {
  if (X->c.mode == 0) return 0;
  int ix = (int)floor(r[0] / X->dx), iy = (int)floor(r[1] / X->dy), iz = (int)floor(r[2] / X->dz);
  if (ix < 0) ix = 0;
  if (ix >= X->nx) ix = X->nx - 1;
  if (iy < 0) iy = 0;
  if (iy >= X->ny) iy = X->ny - 1;
  if (iz < 0) iz = 0;
  if (iz >= X->nz) iz = X->nz - 1;
  return cell_index(X, ix, iy, iz);
}

static int gated(const or_ctx *X, int ix) {
  double xc = (ix + 0.5) * X->dx;
  return xc >= X->c.gate_x_nm[0] && xc <= X->c.gate_x_nm[1];
}

/* Assemble the finite-volume matrix (SPD, lower band) and its boundary
 * right-hand side, then factor it once with a banded Cholesky. */
static void poisson_setup(or_ctx *X) {
  int n = X->ncell, p = X->ny * X->nz;
  X->band = p;
  double eps = X->c.eps_s * OR_EPS0 * 1e-9; /* F/nm */
  double gx = eps * X->dy * X->dz / X->dx, gy = eps * X->dx * X->dz / X->dy, gz = eps * X->dx * X->dy / X->dz;
  double phig = X->c.Vgs + X->c.phi_offset;
  double *A = calloc((size_t)n * (p + 1), sizeof(double)); /* A[i][i-j] at i*(p+1)+(i-j) */
  memset(X->bc_rhs, 0, sizeof(double) * n);
#define AB(i, j) A[(size_t)(i) * (p + 1) + ((i) - (j))]
  for (int ix = 0; ix < X->nx; ++ix)
    for (int iy = 0; iy < X->ny; ++iy)
      for (int iz = 0; iz < X->nz; ++iz) {
        int i = cell_index(X, ix, iy, iz);
        /* x faces */
        if (ix > 0) { AB(i, i) += gx; AB(i, cell_index(X, ix - 1, iy, iz)) -= gx; }
        else { AB(i, i) += 2.0 * gx; X->bc_rhs[i] += 2.0 * gx * 0.0; }
        if (ix < X->nx - 1) AB(i, i) += gx; /* upper neighbour stored from its row */
        else { AB(i, i) += 2.0 * gx; X->bc_rhs[i] += 2.0 * gx * X->c.Vds; }
        /* y faces: y = 0 is the symmetry cut (Neumann); outer side gated */
        if (iy > 0) { AB(i, i) += gy; AB(i, cell_index(X, ix, iy - 1, iz)) -= gy; }
        if (iy < X->ny - 1) AB(i, i) += gy;
        else if (gated(X, ix)) { AB(i, i) += 2.0 * gy; X->bc_rhs[i] += 2.0 * gy * phig; }
        /* z faces: z = 0 rests on the film (Neumann); top gated */
        if (iz > 0) { AB(i, i) += gz; AB(i, cell_index(X, ix, iy, iz - 1)) -= gz; }
        if (iz < X->nz - 1) AB(i, i) += gz;
        else if (gated(X, ix)) { AB(i, i) += 2.0 * gz; X->bc_rhs[i] += 2.0 * gz * phig; }
      }
  /* banded Cholesky A = L L^T, L stored like A */
  double *L = X->Lband;
  memset(L, 0, sizeof(double) * (size_t)n * (p + 1));
#define LB(i, j) L[(size_t)(i) * (p + 1) + ((i) - (j))]
  for (int i = 0; i < n; ++i) {
    int j0 = i - p < 0 ? 0 : i - p;
    for (int j = j0; j <= i; ++j) {
      double s = AB(i, j);
      for (int k = j0; k < j; ++k)
        if (j - k <= p) s -= LB(i, k) * LB(j, k);
      if (i == j) LB(i, i) = sqrt(s);
      else LB(i, j) = s / LB(j, j);
    }
  }
#undef AB
  free(A);
}

/* solve L L^T phi = rhs */
static void chol_solve(const or_ctx *X, const double *rhs, double *phi) {
  int n = X->ncell, p = X->band;
  const double *L = X->Lband;
  double *y = malloc(sizeof(double) * n);
  for (int i = 0; i < n; ++i) {
    double s = rhs[i];
    int j0 = i - p < 0 ? 0 : i - p;
    for (int j = j0; j < i; ++j) s -= LB(i, j) * y[j];
    y[i] = s / LB(i, i);
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    int j1 = i + p > n - 1 ? n - 1 : i + p;
    for (int j = i + 1; j <= j1; ++j) s -= LB(j, i) * phi[j];
    phi[i] = s / LB(i, i);
  }
  free(y);
}
#undef LB

/* centred-difference field E = -grad(phi), V/nm.  A Dirichlet neighbour is
 * its face value half a cell away; a Neumann neighbour is the cell itself. */
static void field_from_phi(or_ctx *X) {
  double phig = X->c.Vgs + X->c.phi_offset;
  for (int ix = 0; ix < X->nx; ++ix)
    for (int iy = 0; iy < X->ny; ++iy)
      for (int iz = 0; iz < X->nz; ++iz) {
        int i = cell_index(X, ix, iy, iz);
        double pc = X->phi[i];
        double pe, de, pw, dw;
        if (ix < X->nx - 1) { pe = X->phi[cell_index(X, ix + 1, iy, iz)]; de = X->dx; }
        else { pe = X->c.Vds; de = 0.5 * X->dx; }
        if (ix > 0) { pw = X->phi[cell_index(X, ix - 1, iy, iz)]; dw = X->dx; }
        else { pw = 0.0; dw = 0.5 * X->dx; }
        double ex = -(pe - pw) / (de + dw);
        double pn, dn, ps, ds;
        if (iy < X->ny - 1) { pn = X->phi[cell_index(X, ix, iy + 1, iz)]; dn = X->dy; }
        else if (gated(X, ix)) { pn = phig; dn = 0.5 * X->dy; }
        else { pn = pc; dn = 0.0; }
        if (iy > 0) { ps = X->phi[cell_index(X, ix, iy - 1, iz)]; ds = X->dy; }
        else { ps = pc; ds = 0.0; }
        double ey = (dn + ds) > 0.0 ? -(pn - ps) / (dn + ds) : 0.0;
        double pt, dt, pb, db;
        if (iz < X->nz - 1) { pt = X->phi[cell_index(X, ix, iy, iz + 1)]; dt = X->dz; }
        else if (gated(X, ix)) { pt = phig; dt = 0.5 * X->dz; }
        else { pt = pc; dt = 0.0; }
        if (iz > 0) { pb = X->phi[cell_index(X, ix, iy, iz - 1)]; db = X->dz; }
        else { pb = pc; db = 0.0; }
        double ez = (dt + db) > 0.0 ? -(pt - pb) / (dt + db) : 0.0;
        X->field[3 * i + 0] = ex;
        X->field[3 * i + 1] = ey;
        X->field[3 * i + 2] = ez;
      }
}

/* right-hand side of the cell balance, in coulombs: e (N_D V_c - w n_c) */
static void poisson_solve_counts(or_ctx *X) {
  double ND_nm = X->c.N_D_m3 * 1e-27;
  double *rhs = malloc(sizeof(double) * X->ncell);
  for (int i = 0; i < X->ncell; ++i)
    rhs[i] = X->bc_rhs[i] + OR_QE * (ND_nm * X->Vc - X->w * (double)X->count[i]);
  chol_solve(X, rhs, X->phi);
  free(rhs);
  field_from_phi(X);
}

/* ------------------------------------------------------------------ */
/* Particles: initial Maxwellian, free flight, scattering.              */
/* ------------------------------------------------------------------ */
static void maxwell_k(const or_ctx *X, const uint32_t w[4], double T, double k[3]) {
  double sig = sqrt(X->c.m_eff[0] * OR_KB * T / OR_QE / (2.0 * ck())); /* 1/nm */
  double r1 = sqrt(-2.0 * log(u01(w[0]))), r2 = sqrt(-2.0 * log(u01(w[2])));
  double a1 = 2.0 * OR_PI * u01(w[1]), a2 = 2.0 * OR_PI * u01(w[3]);
  k[0] = sig * r1 * cos(a1);
  k[1] = sig * r1 * sin(a1);
  k[2] = sig * r2 * cos(a2);
}

static void init_particles(or_ctx *X) {
  for (int p = 0; p < X->c.capacity; ++p) {
    X->alive[p] = 0; X->valley[p] = 0; X->id[p] = 0;
    for (int d = 0; d < 3; ++d) X->k[3 * p + d] = X->r[3 * p + d] = 0.0;
  }
  for (int p = 0; p < X->c.n_particles; ++p) {
    uint32_t w[4];
    rng(X, (uint32_t)p, 0u, 0u, 1u, w);
    maxwell_k(X, w, X->c.T_init_K, X->k + 3 * p);
    if (X->c.mode == 1) {
      rng(X, (uint32_t)p, 0u, 1u, 1u, w);
      X->r[3 * p + 0] = u01(w[0]) * X->c.L_nm[0];
      X->r[3 * p + 1] = u01(w[1]) * X->c.L_nm[1];
      X->r[3 * p + 2] = u01(w[2]) * X->c.L_nm[2];
    }
    X->alive[p] = 1; X->valley[p] = 0; X->id[p] = (uint32_t)p;
  }
  X->next_id = (uint32_t)X->c.n_particles;
}

/* Free flight for time dt under the constant field F: k changes linearly
 * (exact), r by the trapezoid of the end-point velocities.  Returns -1 if
 * the particle stays inside, else the contact it left through (0 source,
 * 1 drain).  Lateral faces reflect specularly. */
static int drift(const or_ctx *X, double k[3], double r[3], int v, double dt, const double F[3], or_counts *tl) {
  double k1[3];
  double c = cf();
  for (int d = 0; d < 3; ++d) k1[d] = k[d] - c * F[d] * dt;
  if (X->c.mode == 1) {
    double v0[3], v1[3];
    velocity(X, k, v, v0);
    velocity(X, k1, v, v1);
    for (int d = 0; d < 3; ++d) r[d] += 0.5 * dt * (v0[d] + v1[d]);
  }
  for (int d = 0; d < 3; ++d) k[d] = k1[d];
  if (X->c.mode == 0) return -1;
  if (r[0] < 0.0) return 0;
  if (r[0] > X->c.L_nm[0]) return 1;
  for (int d = 1; d < 3; ++d) {
    double Ld = X->c.L_nm[d];
    int guard = 0;
    while ((r[d] < 0.0 || r[d] > Ld) && guard < 8) {
      r[d] = r[d] < 0.0 ? -r[d] : 2.0 * Ld - r[d];
      k[d] = -k[d];
      ++guard;
    }
    if (r[d] < 0.0 || r[d] > Ld) { r[d] = r[d] < 0.0 ? 0.0 : Ld; tl->reflect_guard++; }
  }
  return -1;
}

/* orthonormal basis around the unit vector n (Duff et al., JCGT 2017) */
void or_onb(const double n[3], double e1[3], double e2[3]) {
  double s = copysign(1.0, n[2]);
  double a = -1.0 / (s + n[2]);
  double b = n[0] * n[1] * a;
  e1[0] = 1.0 + s * n[0] * n[0] * a; e1[1] = s * b; e1[2] = -s * n[0];
  e2[0] = b; e2[1] = s + n[1] * n[1] * a; e2[2] = -n[1];
}

/* Select a mechanism with u1 * Gamma_v against the running sum of the
 * tabulated rates in the cell's factors; apply the final state.  Returns the
 * mechanism index, or -1 for self-scattering. */
static int scatter(const or_ctx *X, double k[3], int *pv, int cell, const uint32_t w[4], or_counts *tl,
                   uint64_t *heat) {
  const or_config *c = &X->c;
  int v = *pv, nb = c->n_bins;
  double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  double gam = ck() * k2 / c->m_eff[v];
  double E = or_kane_energy(gam, c->alpha[v]);
  double eb = E / c->dE_eV;
  int b;
  if (eb >= (double)nb) { b = nb - 1; tl->overflow++; }
  else b = (int)eb;
  const double *S = X->shape + ((size_t)v * nb + b) * OR_NM;
  double k4 = X->k4[(size_t)v * nb + b];
  const double *f = X->fac + (size_t)cell * OR_NF;
  double rs = u01(w[1]) * X->gamma[v];
  double cum = 0.0;
  int m = -1;
  for (int q = 0; q < OR_NM; ++q) {
    cum += tab_term(S, k4, f, q);
    if (rs < cum) { m = q; break; }
  }
  tl->selections++;
  if (m < 0) { tl->self_events++; return -1; }
  /* final valley and energy */
  int vp = v;
  double Ep;
  if (m == OR_AC || m == OR_II) Ep = E;
  else if (m == OR_POP_AB) Ep = E + c->hw_lo_eV;
  else if (m == OR_POP_EM) Ep = E - c->hw_lo_eV;
  else {
    vp = (m - OR_IV0) / 2;
    Ep = iv_final_energy(c, v, vp, (m - OR_IV0) % 2, E);
  }
  if (!(Ep > 0.0)) { tl->self_events++; return -1; } /* threshold bin: no final state */
  tl->real[v][m]++;
  if (heat) {
    if (m == OR_POP_EM) heat[4 * cell + 0]++;
    else if (m == OR_POP_AB) heat[4 * cell + 1]++;
    else if (m >= OR_IV0) heat[4 * cell + ((m - OR_IV0) % 2 ? 2 : 3)]++;
  }
  /* polar angle relative to the initial direction, sampled as X = 1 - cos:
   * sin = sqrt(X (2 - X)) keeps full relative accuracy for forward
   * scattering, where 1 - cos^2 would cancel */
  double u2 = u01(w[2]), u3 = u01(w[3]);
  double Xc;
  if (m == OR_II) {
    double a4 = 4.0 * k2 / f[F_B2];
    Xc = 2.0 * u2 / (1.0 + (1.0 - u2) * a4);
  } else if (m == OR_POP_AB || m == OR_POP_EM) {
    double gp = Ep * (1.0 + c->alpha[v] * Ep);
    double sg = sqrt(gam), sgp = sqrt(gp);
    double xi = 2.0 * sg * sgp / ((sg - sgp) * (sg - sgp));
    Xc = expm1(u2 * log1p(2.0 * xi)) / xi;
  } else {
    Xc = 2.0 * u2;
  }
  if (Xc < 0.0) Xc = 0.0;
  if (Xc > 2.0) Xc = 2.0;
  double ct = 1.0 - Xc;
  double st = sqrt(Xc * (2.0 - Xc));
  double ph = 2.0 * OR_PI * u3;
  double kn = sqrt(k2);
  double n[3] = {0.0, 0.0, 1.0};
  if (kn > 0.0) { n[0] = k[0] / kn; n[1] = k[1] / kn; n[2] = k[2] / kn; }
  double e1[3], e2[3];
  or_onb(n, e1, e2);
  double gp = Ep * (1.0 + c->alpha[vp] * Ep);
  double kp = sqrt(gp * c->m_eff[vp] / ck());
  double cp = cos(ph), sp = sin(ph);
  for (int d = 0; d < 3; ++d) k[d] = kp * (st * cp * e1[d] + st * sp * e2[d] + ct * n[d]);
  *pv = vp;
  return m;
}

double or_ensemble_energy(const or_ctx *X);

/* total energy of an electron: kinetic (Kane) plus its valley minimum, eV */
static double total_energy(const or_ctx *X, const double k[3], int v) { return energy_of_k(X, k, v) + X->c.E_c[v]; }

/* an electron of slot p left through contact `side` with valley v */
static void note_exit(or_ctx *X, int p, int side, int v) {
  X->eexit[p] = total_energy(X, X->k + 3 * p, v);
  X->xside[p] = (signed char)side;
}

/* One flight interval [0, K dt) of particle p (the field is constant over an
 * interval, so the remaining flight time is drawn afresh at its start; the
 * Poisson process of rate Gamma_v is memoryless). */
static void fly(or_ctx *X, int p, uint32_t n_int, or_counts *tl, uint64_t *heat) {
  const double TP = X->c.dt_fs * (double)X->c.substeps;
  double *k = X->k + 3 * p, *r = X->r + 3 * p;
  int v = X->valley[p];
  uint32_t idp = X->id[p];
  uint32_t w[4];
  uint32_t j = 0;
  double work = 0.0;     /* kinetic energy gained in the field over the flights, eV */
  double absorbed = 0.0; /* energy gained in phonon absorptions, eV */
  rng(X, idp, n_int, 0u, 0u, w);
  double t = 0.0;
  double tau = -log(u01(w[0])) / X->gamma[v];
  for (;;) {
    int cell = cell_of(X, r);
    const double *F = X->c.mode == 1 ? X->field + 3 * cell : X->c.F_bulk;
    double e0 = energy_of_k(X, k, v);
    if (t + tau >= TP) {
      int ex = drift(X, k, r, v, TP - t, F, tl);
      work += energy_of_k(X, k, v) - e0;
      if (ex >= 0) { X->alive[p] = 0; tl->exits[ex]++; note_exit(X, p, ex, v); }
      break;
    }
    int ex = drift(X, k, r, v, tau, F, tl);
    work += energy_of_k(X, k, v) - e0;
    if (ex >= 0) { X->alive[p] = 0; tl->exits[ex]++; note_exit(X, p, ex, v); break; }
    t += tau;
    ++j;
    rng(X, idp, n_int, j, 0u, w);
    cell = cell_of(X, r);
    double et = total_energy(X, k, v);
    int m = scatter(X, k, &v, cell, w, tl, heat);
    /* energy taken from absorbed phonons, from the electron's own energy
     * change (independent of the event counts) */
    if (m == OR_POP_AB || (m >= OR_IV0 && ((m - OR_IV0) & 1) == 0)) absorbed += total_energy(X, k, v) - et;
    tau = -log(u01(w[0])) / X->gamma[v];
  }
  X->valley[p] = v;
  X->ework[p] = work;
  X->eabs[p] = absorbed;
  if (!(isfinite(k[0]) && isfinite(k[1]) && isfinite(k[2]))) X->err_nan = 1;
}

static void add_counts(or_counts *a, const or_counts *b) {
  a->selections += b->selections; a->self_events += b->self_events; a->overflow += b->overflow;
  for (int v = 0; v < OR_NV; ++v)
    for (int m = 0; m < OR_NM; ++m) a->real[v][m] += b->real[v][m];
  a->exits[0] += b->exits[0]; a->exits[1] += b->exits[1];
  a->injections[0] += b->injections[0]; a->injections[1] += b->injections[1];
  a->reflect_guard += b->reflect_guard;
}

/* ------------------------------------------------------------------ */
/* Deposit, contact injection and the Poisson refresh.                  */
/* ------------------------------------------------------------------ */
static void deposit(or_ctx *X) {
  memset(X->count, 0, sizeof(uint32_t) * X->ncell);
  for (int p = 0; p < X->c.capacity; ++p)
    if (X->alive[p]) X->count[cell_of(X, X->r + 3 * p)]++;
}

/* Ohmic contacts: after each deposit the cells next to the source and drain
 * faces are refilled to charge neutrality with Maxwellian electrons at the
 * cell temperature, placed uniformly in the cell.  The q-th new electron
 * takes the q-th free slot (ascending) and identity next_id + q. */
static void inject(or_ctx *X, uint32_t u) {
  double ND_nm = X->c.N_D_m3 * 1e-27;
  long target = lround(ND_nm * X->Vc / X->w);
  int per = X->ny * X->nz;
  int slot = 0;
  uint32_t q = 0;
  for (int side = 0; side < 2; ++side)
    for (int l = 0; l < per; ++l) {
      int cell = side == 0 ? l : (X->nx - 1) * per + l;
      long need = target - (long)X->count[cell];
      int ix = side == 0 ? 0 : X->nx - 1;
      int iy = l / X->nz, iz = l % X->nz;
      for (long i = 0; i < need; ++i) {
        while (slot < X->c.capacity && X->alive[slot]) ++slot;
        if (slot >= X->c.capacity) { X->err_capacity = 1; return; }
        uint32_t w[4];
        rng(X, (uint32_t)cell, u, (uint32_t)i, 2u, w);
        maxwell_k(X, w, X->Tcell[cell], X->k + 3 * slot);
        rng(X, (uint32_t)cell, u, (uint32_t)i, 3u, w);
        X->r[3 * slot + 0] = (ix + u01(w[0])) * X->dx;
        X->r[3 * slot + 1] = (iy + u01(w[1])) * X->dy;
        X->r[3 * slot + 2] = (iz + u01(w[2])) * X->dz;
        X->valley[slot] = 0;
        X->alive[slot] = 1;
        X->id[slot] = X->next_id + q;
        X->e_inj[side] += total_energy(X, X->k + 3 * slot, 0);
        ++q;
        X->count[cell]++;
        X->tot.injections[side]++;
        ++slot;
      }
    }
  X->next_id += q;
}

void or_poisson_update(or_ctx *X) {
  if (X->c.mode != 1) return;
  deposit(X);
  inject(X, X->n_done);
  poisson_solve_counts(X);
}

/* ------------------------------------------------------------------ */
/* Public API                                                           */
/* ------------------------------------------------------------------ */
or_ctx *or_create(const or_config *cfg, const double *T_cells) {
  or_ctx *X = calloc(1, sizeof(or_ctx));
  X->c = *cfg;
  if (cfg->mode == 1) {
    X->nx = cfg->n_cells[0]; X->ny = cfg->n_cells[1]; X->nz = cfg->n_cells[2];
  } else {
    X->nx = X->ny = X->nz = 1;
  }
  X->ncell = X->nx * X->ny * X->nz;
  X->dx = cfg->L_nm[0] / X->nx; X->dy = cfg->L_nm[1] / X->ny; X->dz = cfg->L_nm[2] / X->nz;
  X->Vc = X->dx * X->dy * X->dz;
  X->w = cfg->mode == 1 ? cfg->N_D_m3 * 1e-27 * cfg->L_nm[0] * cfg->L_nm[1] * cfg->L_nm[2] / cfg->n_particles : 1.0;
  int nb = cfg->n_bins;
  X->shape = calloc((size_t)OR_NV * nb * OR_NM, sizeof(double));
  X->k4 = calloc((size_t)OR_NV * nb, sizeof(double));
  X->fac = calloc((size_t)X->ncell * OR_NF, sizeof(double));
  X->Tcell = calloc(X->ncell, sizeof(double));
  for (int i = 0; i < X->ncell; ++i) X->Tcell[i] = T_cells ? T_cells[i] : cfg->T0_K;
  int cap = cfg->capacity;
  X->k = calloc((size_t)cap * 3, sizeof(double));
  X->r = calloc((size_t)cap * 3, sizeof(double));
  X->valley = calloc(cap, sizeof(int));
  X->alive = calloc(cap, sizeof(int));
  X->id = calloc(cap, sizeof(uint32_t));
  X->phi = calloc(X->ncell, sizeof(double));
  X->field = calloc((size_t)X->ncell * 3, sizeof(double));
  X->bc_rhs = calloc(X->ncell, sizeof(double));
  X->Lband = calloc((size_t)X->ncell * (X->ny * X->nz + 1), sizeof(double));
  X->count = calloc(X->ncell, sizeof(uint32_t));
  X->heat = calloc((size_t)X->ncell * 4, sizeof(uint64_t));
  X->dens_sum = calloc(X->ncell, sizeof(uint64_t));
  X->hist_cap = 1 << 16;
  X->hist = calloc((size_t)X->hist_cap * 8, sizeof(double));
  X->eexit = calloc(cap, sizeof(double));
  X->ework = calloc(cap, sizeof(double));
  X->eabs = calloc(cap, sizeof(double));
  X->xside = malloc(cap);
  memset(X->xside, -1, cap);
  build_tables(X);
  cell_factors(X);
  compute_gamma(X);
  init_particles(X);
  /* the window starts before the first contact refill, which it counts */
  X->e_ens0 = or_ensemble_energy(X);
  if (cfg->mode == 1) {
    poisson_setup(X);
    or_poisson_update(X);
  }
  return X;
}

void or_destroy(or_ctx *X) {
  if (!X) return;
  free(X->shape); free(X->k4); free(X->fac); free(X->Tcell);
  free(X->k); free(X->r); free(X->valley); free(X->alive); free(X->id);
  free(X->phi); free(X->field); free(X->bc_rhs); free(X->Lband); free(X->count);
  free(X->heat); free(X->dens_sum); free(X->hist);
  free(X->eexit); free(X->xside); free(X->ework); free(X->eabs);
  free(X);
}

static void record_bulk(or_ctx *X) {
  if (X->hist_len >= X->hist_cap) return;
  double *row = X->hist + (size_t)X->hist_len * 8;
  memset(row, 0, sizeof(double) * 8);
  for (int p = 0; p < X->c.capacity; ++p) {
    if (!X->alive[p]) continue;
    double vel[3];
    int v = X->valley[p];
    velocity(X, X->k + 3 * p, v, vel);
    row[0] += 1.0;
    row[1] += vel[0]; row[2] += vel[1]; row[3] += vel[2];
    row[4] += energy_of_k(X, X->k + 3 * p, v);
    row[5 + v] += 1.0;
  }
  X->hist_len++;
}

/* Device-mode row after each refresh: the window's cumulative exits and
 * injections (source, drain), the electrons present, the mean potential (V)
 * and the root-mean-square field magnitude (V/nm) over the subcells, and the
 * number of intervals done.  The drain current and the field are the two
 * quantities whose constancy marks the steady state (electron MC
 * paragraph). */
static void record_device(or_ctx *X) {
  if (X->hist_len >= X->hist_cap) return;
  double *row = X->hist + (size_t)X->hist_len * 8;
  double n = 0.0, sphi = 0.0, sf2 = 0.0;
  for (int i = 0; i < X->ncell; ++i) {
    n += (double)X->count[i];
    sphi += X->phi[i];
    const double *F = X->field + 3 * i;
    sf2 += F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
  }
  row[0] = (double)X->tot.exits[0];
  row[1] = (double)X->tot.exits[1];
  row[2] = (double)X->tot.injections[0];
  row[3] = (double)X->tot.injections[1];
  row[4] = n;
  row[5] = sphi / X->ncell;
  row[6] = sqrt(sf2 / X->ncell);
  row[7] = (double)X->n_done;
  X->hist_len++;
}

/* total energy (kinetic plus valley minimum, eV) of the live electrons,
 * summed in slot order */
double or_ensemble_energy(const or_ctx *X) {
  double e = 0.0;
  for (int p = 0; p < X->c.capacity; ++p)
    if (X->alive[p]) e += total_energy(X, X->k + 3 * p, X->valley[p]);
  return e;
}

/* Advance n_intervals flight intervals (each K sub-steps), with a deposit,
 * contact injection and Poisson refresh after each in device mode. */
int or_run(or_ctx *X, int n_intervals, int n_threads) {
  int cap = X->c.capacity;
#ifdef _OPENMP
  int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
  int nt = 1;
  (void)n_threads;
#endif
  or_counts *tl = calloc(nt, sizeof(or_counts));
  uint64_t **heat = calloc(nt, sizeof(uint64_t *));
  for (int t = 0; t < nt; ++t) heat[t] = calloc((size_t)X->ncell * 4, sizeof(uint64_t));
  for (int it = 0; it < n_intervals; ++it) {
    uint32_t n_int = X->n_done;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static)
#endif
    for (int p = 0; p < cap; ++p) {
      if (!X->alive[p]) continue;
#ifdef _OPENMP
      int t = omp_get_thread_num();
#else
      int t = 0;
#endif
      fly(X, p, n_int, tl + t, heat[t]);
    }
    /* integer counts merged after every interval (any order gives the same
     * sums); exit energies in slot order, before the refill reuses slots */
    for (int t = 0; t < nt; ++t) {
      add_counts(&X->tot, tl + t);
      memset(tl + t, 0, sizeof(or_counts));
    }
    for (int p = 0; p < cap; ++p) {
      X->e_work += X->ework[p];
      X->e_abs += X->eabs[p];
      X->ework[p] = X->eabs[p] = 0.0;
      if (X->xside[p] >= 0) {
        X->e_exit[(int)X->xside[p]] += X->eexit[p];
        X->xside[p] = -1;
      }
    }
    X->n_done++;
    if (X->c.mode == 0) record_bulk(X);
    else {
      or_poisson_update(X);
      for (int i = 0; i < X->ncell; ++i) X->dens_sum[i] += X->count[i];
      record_device(X);
    }
    X->win_intervals++;
  }
  for (int t = 0; t < nt; ++t) {
    for (size_t i = 0; i < (size_t)X->ncell * 4; ++i) X->heat[i] += heat[t][i];
    free(heat[t]);
  }
  free(heat);
  free(tl);
  return X->err_capacity ? -3 : (X->err_nan ? -6 : 0);
}

void or_reset_window(or_ctx *X) {
  memset(&X->tot, 0, sizeof(or_counts));
  memset(X->heat, 0, sizeof(uint64_t) * X->ncell * 4);
  memset(X->dens_sum, 0, sizeof(uint64_t) * X->ncell);
  X->win_intervals = 0;
  X->hist_len = 0;
  X->e_exit[0] = X->e_exit[1] = X->e_inj[0] = X->e_inj[1] = X->e_work = X->e_abs = 0.0;
  X->e_ens0 = or_ensemble_energy(X);
}

void or_set_temperature(or_ctx *X, const double *T_cells) {
  for (int i = 0; i < X->ncell; ++i) X->Tcell[i] = T_cells[i];
  cell_factors(X);
  compute_gamma(X);
}

/* replace the rate shapes (test hook for synthetic mechanisms) */
void or_set_tables(or_ctx *X, const double *shape, const double *k4) {
  memcpy(X->shape, shape, sizeof(double) * OR_NV * X->c.n_bins * OR_NM);
  memcpy(X->k4, k4, sizeof(double) * OR_NV * X->c.n_bins);
  compute_gamma(X);
}

/* ---- accessors ---- */
int or_ncell(const or_ctx *X) { return X->ncell; }
double or_weight(const or_ctx *X) { return X->w; }
uint32_t or_intervals_done(const or_ctx *X) { return X->n_done; }
uint32_t or_window_intervals(const or_ctx *X) { return X->win_intervals; }
uint32_t or_next_id(const or_ctx *X) { return X->next_id; }
void or_gamma(const or_ctx *X, double *g) { memcpy(g, X->gamma, sizeof(double) * OR_NV); }
void or_tables(const or_ctx *X, double *shape, double *k4) {
  memcpy(shape, X->shape, sizeof(double) * OR_NV * X->c.n_bins * OR_NM);
  memcpy(k4, X->k4, sizeof(double) * OR_NV * X->c.n_bins);
}
void or_factors(const or_ctx *X, double *fac) { memcpy(fac, X->fac, sizeof(double) * X->ncell * OR_NF); }
void or_get_particles(const or_ctx *X, double *k, double *r, int32_t *valley, int32_t *alive, uint32_t *id) {
  int cap = X->c.capacity;
  memcpy(k, X->k, sizeof(double) * 3 * cap);
  memcpy(r, X->r, sizeof(double) * 3 * cap);
  for (int p = 0; p < cap; ++p) { valley[p] = X->valley[p]; alive[p] = X->alive[p]; }
  memcpy(id, X->id, sizeof(uint32_t) * cap);
}
void or_set_particles(or_ctx *X, const double *k, const double *r, const int32_t *valley, const int32_t *alive,
                      const uint32_t *id) {
  int cap = X->c.capacity;
  memcpy(X->k, k, sizeof(double) * 3 * cap);
  memcpy(X->r, r, sizeof(double) * 3 * cap);
  for (int p = 0; p < cap; ++p) { X->valley[p] = valley[p]; X->alive[p] = alive[p]; }
  memcpy(X->id, id, sizeof(uint32_t) * cap);
}
/* Resume hook: the number of intervals done (the interval index of the
 * flight streams and of the contact refill) and the next free identity, so
 * that a state taken from elsewhere continues on the same streams. */
void or_set_progress(or_ctx *X, int n_done, uint32_t next_id) {
  X->n_done = n_done;
  X->next_id = next_id;
}
void or_get_fields(const or_ctx *X, double *phi, double *field, uint32_t *count) {
  memcpy(phi, X->phi, sizeof(double) * X->ncell);
  memcpy(field, X->field, sizeof(double) * 3 * X->ncell);
  memcpy(count, X->count, sizeof(uint32_t) * X->ncell);
}
void or_get_counts(const or_ctx *X, uint64_t *out) {
  /* selections, self, overflow, real[3][10], exits[2], injections[2], reflect_guard */
  const or_counts *t = &X->tot;
  out[0] = t->selections; out[1] = t->self_events; out[2] = t->overflow;
  for (int v = 0; v < OR_NV; ++v)
    for (int m = 0; m < OR_NM; ++m) out[3 + v * OR_NM + m] = t->real[v][m];
  out[33] = t->exits[0]; out[34] = t->exits[1];
  out[35] = t->injections[0]; out[36] = t->injections[1];
  out[37] = t->reflect_guard;
}
void or_get_maps(const or_ctx *X, uint64_t *heat, uint64_t *dens_sum) {
  memcpy(heat, X->heat, sizeof(uint64_t) * 4 * X->ncell);
  memcpy(dens_sum, X->dens_sum, sizeof(uint64_t) * X->ncell);
}
int or_history(const or_ctx *X, double *rows, int max_rows) {
  int n = X->hist_len < max_rows ? X->hist_len : max_rows;
  memcpy(rows, X->hist, sizeof(double) * 8 * n);
  return n;
}

/* ------------------------------------------------------------------ */
/* Observables of the averaging window (electron MC paragraph: heat     */
/* counted per subcell, the steady state reached once current and field */
/* stop changing; the thermal-resistance passage: emitted phonon energy) */
/* ------------------------------------------------------------------ */
enum { OR_STEADY_BLOCKS = 10 };

/* Steady-state test of one per-interval series s[0..m): the last 2h values
 * (h = m/2) form two halves; each half's mean and its standard error come
 * from 10 batch means of h/10 consecutive values.  Steady (1) when the two
 * means differ by at most 3 combined standard errors, 0 otherwise, -1 when
 * a half holds fewer than 10 values.  out = {mean1, mean2, se1, se2}. */
int or_steady_test(const double *s, int m, double out[4]) {
  int h = m / 2, b = h / OR_STEADY_BLOCKS;
  out[0] = out[1] = out[2] = out[3] = 0.0;
  if (b < 1) return -1;
  for (int half = 0; half < 2; ++half) {
    int start = m - 2 * h + half * h;
    double bm[OR_STEADY_BLOCKS], mu = 0.0;
    for (int j = 0; j < OR_STEADY_BLOCKS; ++j) {
      double a = 0.0;
      for (int i = 0; i < b; ++i) a += s[start + j * b + i];
      bm[j] = a / b;
      mu += bm[j];
    }
    mu /= OR_STEADY_BLOCKS;
    double var = 0.0;
    for (int j = 0; j < OR_STEADY_BLOCKS; ++j) var += (bm[j] - mu) * (bm[j] - mu);
    out[half] = mu;
    out[2 + half] = sqrt(var / (OR_STEADY_BLOCKS * (OR_STEADY_BLOCKS - 1.0)));
  }
  return fabs(out[0] - out[1]) <= 3.0 * sqrt(out[2] * out[2] + out[3] * out[3]) ? 1 : 0;
}

typedef struct {
  int intervals;
  double t_window_s;
  /* device mode */
  double I_D, I_S;           /* A: e w (exits - injections) / t at the drain and source contacts */
  double P_heat_W, P_emit_W; /* net phonon emission and emission only (E_Emit / t), whole domain */
  double E_out_J[2], E_in_J[2]; /* total energy carried out of / into the domain, source and drain */
  double dE_ens_J;           /* change of the ensemble's total energy over the window */
  double W_field_J;          /* kinetic energy the electrons gained in free flight (work of the field) */
  double E_abs_J;            /* energy the electrons took from absorbed phonons */
  /* bulk mode */
  double v_drift_ms[3], mean_E_eV, valley_frac[3];
  /* steady state of the two series (device: drain current per interval, rms
   * field; bulk: mean v_z per interval, mean energy) */
  double half_mean[2][2], half_se[2][2];
  int steady; /* 1 both steady, 0 either not, -1 window too short */
} or_obs;

/* Per-subcell maps of the window: net phonon-emission power density and
 * emission-only power density (W/m^3), electron density (1/m^3). */
void or_power_maps(const or_ctx *X, double *q_net, double *q_emit, double *dens_m3) {
  double t = X->win_intervals * X->c.substeps * X->c.dt_fs * 1e-15;
  double vc = X->Vc * 1e-27, hlo = X->c.hw_lo_eV, hiv = X->c.hw_iv_eV;
  for (int i = 0; i < X->ncell; ++i) {
    const uint64_t *h = X->heat + 4 * i; /* LO emit, LO absorb, iv emit, iv absorb */
    double e_net = hlo * ((double)h[0] - (double)h[1]) + hiv * ((double)h[2] - (double)h[3]);
    double e_em = hlo * (double)h[0] + hiv * (double)h[2];
    if (q_net) q_net[i] = t > 0.0 ? X->w * OR_QE * e_net / (vc * t) : 0.0;
    if (q_emit) q_emit[i] = t > 0.0 ? X->w * OR_QE * e_em / (vc * t) : 0.0;
    if (dens_m3) dens_m3[i] = X->win_intervals ? X->w * (double)X->dens_sum[i] / X->win_intervals / vc : 0.0;
  }
}

void or_observables(const or_ctx *X, or_obs *o) {
  memset(o, 0, sizeof(*o));
  int m = X->hist_len;
  double TP = X->c.substeps * X->c.dt_fs * 1e-15;
  o->intervals = (int)X->win_intervals;
  o->t_window_s = X->win_intervals * TP;
  double *s1 = calloc(m > 0 ? m : 1, sizeof(double)), *s2 = calloc(m > 0 ? m : 1, sizeof(double));
  if (X->c.mode == 1) {
    double t = o->t_window_s, wq = X->w * OR_QE;
    const or_counts *c = &X->tot;
    if (t > 0.0) {
      o->I_D = wq * ((double)c->exits[1] - (double)c->injections[1]) / t;
      o->I_S = wq * ((double)c->exits[0] - (double)c->injections[0]) / t;
      double en = 0.0, ee = 0.0;
      for (int i = 0; i < X->ncell; ++i) {
        const uint64_t *h = X->heat + 4 * i;
        en += X->c.hw_lo_eV * ((double)h[0] - (double)h[1]) + X->c.hw_iv_eV * ((double)h[2] - (double)h[3]);
        ee += X->c.hw_lo_eV * (double)h[0] + X->c.hw_iv_eV * (double)h[2];
      }
      o->P_heat_W = wq * en / t;
      o->P_emit_W = wq * ee / t;
    }
    for (int sd = 0; sd < 2; ++sd) { o->E_out_J[sd] = wq * X->e_exit[sd]; o->E_in_J[sd] = wq * X->e_inj[sd]; }
    o->dE_ens_J = wq * (or_ensemble_energy(X) - X->e_ens0);
    o->W_field_J = wq * X->e_work;
    o->E_abs_J = wq * X->e_abs;
    /* per-interval drain current from the cumulative counts of the rows */
    for (int n = 0; n < m; ++n) {
      const double *r = X->hist + 8 * (size_t)n, *q = n > 0 ? X->hist + 8 * (size_t)(n - 1) : NULL;
      double dex = r[1] - (q ? q[1] : 0.0), dinj = r[3] - (q ? q[3] : 0.0);
      s1[n] = wq * (dex - dinj) / TP;
      s2[n] = r[6];
    }
  } else {
    for (int n = 0; n < m; ++n) {
      const double *r = X->hist + 8 * (size_t)n;
      double na = r[0] > 0.0 ? r[0] : 1.0;
      for (int d = 0; d < 3; ++d) o->v_drift_ms[d] += r[1 + d] / na * 1e6 / m; /* nm/fs -> m/s */
      o->mean_E_eV += r[4] / na / m;
      for (int v = 0; v < 3; ++v) o->valley_frac[v] += r[5 + v] / na / m;
      s1[n] = r[3] / na * 1e6;
      s2[n] = r[4] / na;
    }
  }
  double a[4], b[4];
  int f1 = or_steady_test(s1, m, a), f2 = or_steady_test(s2, m, b);
  for (int h = 0; h < 2; ++h) {
    o->half_mean[0][h] = a[h]; o->half_se[0][h] = a[2 + h];
    o->half_mean[1][h] = b[h]; o->half_se[1][h] = b[2 + h];
  }
  o->steady = (f1 < 0 || f2 < 0) ? -1 : (f1 && f2);
  free(s1);
  free(s2);
}

/* Solve the device Poisson problem for an arbitrary charge per cell (C);
 * the boundary terms of the configured terminals are added. */
void or_poisson_solve(or_ctx *X, const double *charge, double *phi, double *field) {
  double *rhs = malloc(sizeof(double) * X->ncell);
  for (int i = 0; i < X->ncell; ++i) rhs[i] = X->bc_rhs[i] + charge[i];
  chol_solve(X, rhs, X->phi);
  free(rhs);
  field_from_phi(X);
  memcpy(phi, X->phi, sizeof(double) * X->ncell);
  memcpy(field, X->field, sizeof(double) * 3 * X->ncell);
}

/* Single-event hooks used by the pins: draw n selections at fixed (v, E, cell)
 * with the interval-0 stream of identity `pid`, returning counts per
 * mechanism (index 10 = self). */
void or_sample_selection(const or_ctx *X, int v, double E, int cell, uint32_t pid, int n, uint64_t *counts) {
  double kk = sqrt(E * (1.0 + X->c.alpha[v] * E) * X->c.m_eff[v] / ck());
  for (int i = 0; i < n; ++i) {
    double k[3] = {0.0, 0.0, kk};
    int vv = v;
    or_counts tl;
    memset(&tl, 0, sizeof(tl));
    uint32_t w[4];
    rng(X, pid, 0u, (uint32_t)i, 0u, w);
    int m = scatter(X, k, &vv, cell, w, &tl, NULL);
    counts[m < 0 ? OR_NM : m]++;
  }
}

/* Apply one scattering event to (k, v) in `cell` with the given Philox words;
 * returns the mechanism (-1 self). */
int or_scatter_once(const or_ctx *X, double *k, int32_t *v, int cell, const uint32_t *w) {
  or_counts tl;
  memset(&tl, 0, sizeof(tl));
  int vv = *v;
  int m = scatter(X, k, &vv, cell, w, &tl, NULL);
  *v = vv;
  return m;
}
