/*
 * gfhy.h -- C ABI of the electro-thermal coupling of libgfmc.so (MI355X,
 * gfx950): the self-consistent iteration of the coupling paragraph of Hao,
 * Zhao, Xiao and Kronenfeld, arXiv:1707.09073, in which the electron Monte
 * Carlo's heat map drives the phonon Monte Carlo, whose temperature map sets
 * the electron scattering rates, until the temperature no longer changes;
 * and the device thermal resistance of the thermal-resistance passage, the
 * largest acoustic-phonon temperature rise over the emitted phonon power.
 *
 * Conventions as in gfmc.h: every call returns an mc_status (0 = MC_OK) and
 * never throws; the library allocates no device memory (the caller passes a
 * workspace of hy_workspace_bytes); all work runs on the electron context's
 * stream.  The phonon domain of an instance is the instance's own box and
 * subcells (L_nm, n_cells of its mc_config), so its maps are the electron
 * maps cell for cell (index (ix*ny + iy)*nz + iz).
 */
#ifndef GFHY_H
#define GFHY_H

#include <stddef.h>
#include <stdint.h>

#include "gffo.h"
#include "gfmc.h"
#include "gfph.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  ph_material mat;          /* phonons of the wire (Table II) */
  ph_electrons elec;        /* Eq. (1) in the wire; elec.n_m3 = 0 leaves it out */
  int32_t n_bins;           /* frequency bins of the phonon tables, 1..4096 */
  int32_t face[6];          /* a ph_face for each face of the box: x = 0, x = L, y = 0, y = L, z = 0, z = L */
  int32_t max_events;       /* phonon event guard per packet */
  int64_t n_packets;        /* phonon packets per instance and iteration */
  uint64_t seed;            /* Philox key of the packets (tag instance << 4 | 5, one stream per instance) */
  double T_sink_K;          /* temperature of the isothermal faces */
  double T_lin_K;           /* linearisation temperature of the phonon tables; <= 0: each iteration the mean
                               subcell temperature of the instance at its start */
  int32_t warmup_intervals; /* electron intervals after a temperature change, not tallied (>= 0) */
  int32_t window_intervals; /* electron intervals tallied per iteration (>= 1) */
  int32_t max_iterations;   /* >= 1 */
  double relax;             /* T <- T + relax (T_sink + dT - T), 0 < relax <= 1 */
  double tol_K;             /* stop once every instance's largest change |T_sink + dT - T| is at most tol_K */
} hy_config;

/* The chip around the wire for the Fourier's-law stage of the iteration
 * (coupling paragraph: the Fourier analysis covers the whole chip, the
 * phonon Monte Carlo refines the temperature along the wire).  Every wire
 * of the array takes the instance's heat map; the chip's temperature below
 * each electron subcell column becomes that column's reference in place of
 * T_sink: T = T_chip(base) + dT_packets.  The packet domain's faces then
 * should pass the wire's heat to the film only (its foot isothermal, its
 * contact ends adiabatic). */
typedef struct {
  fo_config fo;                  /* grid, held faces (the sink), interface plane and R_K, solver settings; its
                                    T_sink_K is replaced by hy_config's, and its warm_start by the iteration's
                                    (each instance's solve starts from its previous one after the first) */
  const double *d_edges;         /* device: the chip's edges, as fo_solve takes them */
  const uint8_t *d_material;     /* device, per chip cell */
  const int32_t *d_src_index;    /* device, per chip cell: the electron subcell whose heat it takes, or -1 */
  const int32_t *d_base_index;   /* device, per electron subcell: the chip cell below its column (in the film) */
  double kappa_by_material[16];  /* W/(m K), by material id */
  int32_t n_materials;
  int32_t half_wires;            /* half-wires of the whole device: its power is half_wires x E_Emit */
} hy_chip;

/* One instance's record of one iteration. */
typedef struct {
  int32_t iteration, instance;
  int32_t source;           /* 0: heat map of an electron window; 1: the caller's warm-start map */
  int32_t steady;           /* the window's steady-state flag (mc_observables_out.steady); 0 for source 1 */
  double drain_current_A;   /* of the window (0 for source 1) */
  double heat_W;            /* net phonon-emission power over the domain: the phonon source */
  double emit_W;            /* emission-only power (E_Emit of the thermal-resistance passage) */
  double T_lin_K;           /* linearisation temperature of this iteration's phonon tables */
  double dT_max_K;          /* largest subcell temperature rise over T_sink (Delta T_ac) */
  double dT_mean_K;
  int32_t hot_cell;         /* subcell of dT_max */
  int32_t pad;
  double change_K;          /* largest |T_sink + dT - T| over the subcells, before relaxation */
  double R_th_KW;           /* dT_max / emit_W (0 when emit_W is 0) */
  uint64_t packets_absorbed, packets_dropped;
  /* with a chip (zero without): */
  double dT_junction_max_K; /* largest rise of the chip below the wire */
  double dT_fourier_max_K;  /* largest rise of the chip anywhere (the wire by Fourier's law) */
  double R_th_device_KW;    /* dT_max / (half_wires x emit_W): the device thermal resistance */
  double R_th_fourier_KW;   /* dT_fourier_max / (half_wires x emit_W) */
  int32_t fo_iterations;
  int32_t pad2;
} hy_record;

/* Device workspace bytes of hy_run on ctx with cfg (256-byte aligned), 0 if
 * the configuration is invalid for the context. */
size_t hy_workspace_bytes(const mc_ctx *ctx, const hy_config *cfg, const hy_chip *chip);

/* The coupled iteration over every instance of a device-mode context.  Per
 * iteration: every instance's electrons run warmup_intervals, a new window
 * opens (for every instance), they run window_intervals; each instance's net
 * heat map (W per subcell, mc_maps) is the source of a phonon packet run
 * (ph_tables at the linearisation temperature, ph_mc_run in the instance's
 * box with cfg's faces); T_new = T_sink + dT per subcell; the instance's
 * lattice temperature becomes T + relax (T_new - T) (mc_set_lattice_
 * temperature).  The iteration stops after max_iterations or once no
 * instance changed by more than tol_K.  The first iteration starts from the
 * temperatures the context holds.  h_heat0_Wm3 (host, [n_instances][ncell]
 * W/m^3, may be NULL): a warm start, e.g. a surrogate's heat map, used as the
 * first iteration's source in place of an electron window.
 * h_records (host, may be NULL) receives one record per instance and
 * iteration, in order, at most max_records; *n_records the number written,
 * *iterations the iterations done (either may be NULL).  Synchronises the
 * stream every iteration.  chip (may be NULL): the Fourier stage above, run
 * after each packet run on the same heat map.  Returns MC_OK; MC_E_ARG for a
 * bad argument or configuration (bulk mode, faces, sizes, a chip whose
 * indices or tables do not fit, a workspace that is too small or not
 * 256-byte aligned, a temperature that would not be positive); MC_E_RANGE
 * if a chip solve misses its tolerance; or the first error of an electron
 * call (its sticky device flags included), after writing the records done
 * so far. */
int hy_run(mc_ctx *ctx, const hy_config *cfg, const hy_chip *chip, const double *h_heat0_Wm3, void *d_ws,
           size_t ws_bytes, hy_record *h_records, int max_records, int *n_records, int *iterations);

#ifdef __cplusplus
}
#endif
#endif /* GFHY_H */
