/*
 * gfph.h -- C ABI of the phonon side of libgfmc.so (MI355X, gfx950): the
 * acoustic-phonon model of the phonon paragraph and Table II of Hao, Zhao,
 * Xiao and Kronenfeld, arXiv:1707.09073, the phonon scattering by free
 * electrons of Eq. (1), the diffuse-mismatch transmissivity of Eq. (2), the
 * interface resistance of Eq. (3), and the steady-state phonon packet Monte
 * Carlo of the wire domain that turns the electrons' emitted phonon power
 * into a temperature field (phonon and coupling paragraphs).
 *
 * Conventions: plain C; every call returns a ph_status (0 = PH_OK) and never
 * throws.  Device pointers are caller allocations (the library allocates no
 * device memory); work is enqueued on the caller's HIP stream (a hipStream_t
 * passed as void*) and is asynchronous unless a call says it synchronises.
 * Units SI unless stated: omega in rad/s, velocities m/s, temperatures K,
 * lengths of the packet domain nm.
 */
#ifndef GFPH_H
#define GFPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { PH_OK = 0, PH_E_ARG = -1, PH_E_HIP = -2 } ph_status;

/* One material of Table II: three identical acoustic branches with
 * omega = w_max sin(pi q / 2 q0) (q0 is the table's k0), and the relaxation
 * rate 1/tau = A omega^4 + B1 omega^2 T exp(-B2 / T) (impurity and Umklapp
 * scattering, phonon paragraph). */
typedef struct {
  double q0;    /* 1/m */
  double w_max; /* rad/s */
  double A;     /* s^3 */
  double B1;    /* s/K */
  double B2;    /* K */
} ph_material;

/* Free electrons of a doped wire for Eq. (1). */
typedef struct {
  double n_m3;   /* electron density, 1/m^3 (> 0) */
  double m_dos;  /* density-of-states effective mass, m0 */
  double D_a_eV; /* acoustic deformation potential, eV */
  double rho;    /* mass density, kg/m^3 */
  double v_g;    /* the averaged phonon group velocity of Eq. (1), m/s */
} ph_electrons;

/* Fermi level (eV from the band edge) of a parabolic band of mass m_dos (m0)
 * holding n_m3 electrons per m^3 at T_K (Fermi-Dirac statistics), written to
 * d_out (one device double).  Needed by Eq. (1).  PH_E_ARG for non-positive
 * inputs or a NULL pointer. */
int ph_fermi_level(double n_m3, double m_dos, double T_K, double *d_out, void *stream);

/* Frequency-bin tables of a material at temperature T_K: n_bins bins of
 * equal width over (0, w_max), values at the bin midpoints, written to
 * d_tables (device, FP64, [4][n_bins]): omega; group velocity; heat capacity
 * of the bin for the three branches, 3 hbar omega (d f_BE / dT) D(omega)
 * d omega with D = q^2 / (2 pi^2 v_g) (J/(m^3 K)); relaxation rate (1/s),
 * Table II's terms plus Eq. (1) when e is given (e may be NULL; then
 * d_fermi may be NULL too; otherwise d_fermi, one device double, receives the
 * Fermi level in eV).  n_bins 1..4096; PH_E_ARG otherwise. */
int ph_tables(const ph_material *m, const ph_electrons *e, double T_K, int n_bins, double *d_tables,
              double *d_fermi, void *stream);

/* Eq. (2) on the bins of material 1 (d_tables1 from ph_tables of m1): the
 * transmissivity tau_12(omega) = sum_p v_2 D_2 / (sum_p v_1 D_1 + sum_p v_2
 * D_2), zero where material 2 has no states, into d_tau12 (device,
 * [n_bins], may be NULL); and into d_sums (device, 2 doubles) Eq. (3),
 * 1/R_K = sum_p int v_1 c_1 tau_12 d omega / 4 (W/(m^2 K)), and the bulk
 * conductivity of material 1, sum_p int c_1 v_1^2 tau_1 d omega / 3
 * (W/(m K)), both as sums over the bins in a fixed order. */
int ph_interface(const ph_material *m1, const ph_material *m2, const double *d_tables1, int n_bins, double *d_tau12,
                 double *d_sums, void *stream);

/* Conductivity of a structure from the bins of one material (d_tables from
 * ph_tables): kappa = sum_b C_b v_b^2 / (3 (1/tau_b + v_b / d)), the bulk
 * mean free paths limited by the structure size d_m (Matthiessen's rule;
 * the coupling paragraph limits them by the film thickness and the wire
 * diameter for the Fourier analysis); d_m <= 0 gives the bulk value.  One
 * device double to d_kappa (W/(m K)), summed over the bins in order.
 * PH_E_ARG for a bad pointer or n_bins. */
int ph_conductivity(const double *d_tables, int n_bins, double d_m, double *d_kappa, void *stream);

/* Faces of the packet domain: specular (symmetry planes A and B of the
 * coupling paragraph), diffuse (adiabatic free surfaces, cosine-law
 * re-emission), isothermal (absorbing: the heat sink or the Fourier region
 * at the reference temperature). */
typedef enum { PH_SPECULAR = 0, PH_DIFFUSE = 1, PH_ISOTHERMAL = 2 } ph_face;

typedef struct {
  double L_nm[3];     /* box [0, L] per axis */
  int32_t n_cells[3]; /* subcells per axis (at most 4096 in all); index (ix*ny + iy)*nz + iz */
  int32_t face[6];    /* x = 0, x = L, y = 0, y = L, z = 0, z = L: a ph_face each */
  int32_t n_bins;     /* frequency bins of the tables (1..4096) */
  uint64_t seed;      /* Philox key */
  uint32_t instance;  /* enters every Philox counter (tag instance << 4 | 5) */
  int32_t max_events; /* scatterings plus wall reflections per packet before it is dropped and counted */
  int64_t n_packets;  /* 1 .. 2^32 */
} ph_mc_config;

/* Device workspace bytes of ph_mc_run for cfg (256-byte aligned), 0 if the
 * configuration is invalid. */
size_t ph_mc_workspace_bytes(const ph_mc_config *cfg);

/* Steady-state phonon packet Monte Carlo (phonon and coupling paragraphs):
 * the heat generated per subcell, d_q_cell (device, W per subcell, either
 * sign: the electrons' net phonon emission, negative where they absorb more
 * than they emit), is split into n_packets packets of equal power
 * P / n_packets, P the sum of |q|.  A packet starts at a uniform point of a
 * subcell drawn by |q|, with the sign of that subcell's q, in a bin drawn
 * from C_b / tau_b (what relaxation re-emits: the linearised relaxation-time
 * model, tables from ph_tables at the linearisation temperature) with an
 * isotropic direction; it flies for exponential times of mean tau_b at the
 * bin's group velocity, takes a new bin and direction at each scattering,
 * reflects at specular and diffuse faces and ends at an isothermal one.
 * Random numbers: Philox4x32-10 with counter (packet, event, sub, tag): event
 * 0 the emission (sub 0 the subcell and point, sub 1 the bin, direction and
 * first flight), event j the j-th scattering (sub 0), its h-th diffuse
 * reflection sub 1 + h.
 * Outputs: d_t_cell (device, ncell) the packets' signed total time per
 * subcell (fs); d_dT (device, ncell, may be NULL) the temperature rise over
 * the isothermal faces' reference, P t_c / (N C_v V_c) with C_v = sum_b C_b;
 * d_packet_scatterings (device, n_packets u32, may be NULL) each packet's
 * number of scatterings, for diagnostics; h_counts (host, 11 u64, may be
 * NULL; then nothing synchronises) scatterings, specular reflections, diffuse
 * reflections, packets absorbed at each of the six faces, packets dropped at
 * max_events, segments (straight pieces of flight: each ends at a subcell
 * boundary, a scattering or a face).  The per-subcell times are FP64 sums whose order varies between
 * runs at rounding level.  q must be finite.
 * PH_E_ARG for an invalid configuration or pointer, or a workspace that is
 * too small or not 256-byte aligned. */
int ph_mc_run(const ph_mc_config *cfg, const double *d_tables, const double *d_q_cell, double *d_t_cell,
              double *d_dT, uint32_t *d_packet_scatterings, uint64_t *h_counts, void *d_ws, size_t ws_bytes,
              void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GFPH_H */
