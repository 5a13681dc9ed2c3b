/*
 * gfmc.h -- C ABI of the MI355X (gfx950) ensemble electron Monte Carlo
 * library libgfmc.so.
 *
 * The library advances an ensemble of electrons in wurtzite GaN by the method
 * of Hao, Zhao, Xiao and Kronenfeld, arXiv:1707.09073 (electron Monte Carlo
 * paragraph and Table I): Kane-nonparabolic free flight in the Gamma1, U and
 * Gamma3 valleys under the local field, scattering chosen by self-scattering
 * against tabulated ionized-impurity, polar-optical, acoustic and intervalley
 * rates, electrons counted in 3x6x100 subcells of the half nanowire, the
 * field refreshed from the Poisson equation with the terminal voltages, and
 * the electron-phonon energy exchange counted per subcell.
 *
 * Conventions for every entry point:
 *  - Plain C.  Every call returns an mc_status (0 = MC_OK, < 0 = error) and
 *    never throws or aborts; mc_status_string() names a code and
 *    mc_last_error() gives the detail of the last failure on a context.
 *  - The library never allocates device memory.  The caller passes one
 *    device workspace of at least mc_workspace_bytes() bytes (256-byte
 *    aligned) and keeps it alive until mc_destroy().  The library carves all
 *    device state out of it.
 *  - The caller owns the HIP stream (a hipStream_t passed as void*); all
 *    device work is enqueued on it asynchronously.  Calls that return host
 *    data (mc_tally, mc_maps, mc_history, mc_read_*) synchronise the stream.
 *  - Host pointers are caller-owned and only read or written during the call.
 *  - A context is not thread-safe; use one context per host thread.
 *
 * Units: energy eV, wave vector 1/nm, position nm, time fs, field V/nm,
 * potential V, doping and densities 1/m^3, temperature K.
 */
#ifndef GFMC_H
#define GFMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MC_OK = 0,
  MC_E_ARG = -1,      /* invalid argument or configuration */
  MC_E_HIP = -2,      /* a HIP runtime call failed */
  MC_E_CAPACITY = -3, /* particle slots exhausted, or identity space exhausted */
  MC_E_RANGE = -4,    /* an event-count guard was hit in a flight */
  MC_E_STATE = -5,    /* call not valid in the current state */
  MC_E_NAN = -6       /* a non-finite particle state was produced */
} mc_status;

typedef enum { MC_PREC_FP64 = 0, MC_PREC_FP32_STATE = 1 } mc_precision;
typedef enum { MC_BULK = 0, MC_DEVICE = 1 } mc_mode;

/* Material: Table I of the paper plus the readings of silent points.  Valley
 * order Gamma1, U, Gamma3. */
typedef struct {
  double m_eff[3];  /* band-edge effective mass, m0 */
  double alpha[3];  /* Kane nonparabolicity, 1/eV */
  double E_c[3];    /* valley minimum, eV */
  int32_t Z[3];     /* number of equivalent valleys */
  double eps_s, eps_inf; /* static and optical dielectric constants, eps0 */
  double rho;       /* mass density, kg/m^3 */
  double D_ac_eV;   /* acoustic deformation potential, eV */
  double D_iv_eVm;  /* intervalley deformation potential, eV/m */
  double hw_lo_eV;  /* LO phonon energy, eV */
  double hw_iv_eV;  /* intervalley phonon energy, eV */
  double u_ac;      /* sound velocity used by the acoustic rate, m/s */
} mc_material;

/* One instance (one bias point / one ensemble).  All instances of a context
 * must share material, mode, precision, time step, sub-steps, table grid and
 * geometry; seed, ensemble size, doping, temperatures and voltages may
 * differ. */
typedef struct {
  mc_mode mode;
  mc_precision prec;
  mc_material mat;
  uint64_t seed;         /* Philox key */
  uint32_t instance;     /* enters every Philox counter; unique per ensemble */
  int32_t n_particles;   /* initial electrons */
  int32_t capacity;      /* particle slots (>= n_particles) */
  double dt_fs;          /* sub-step */
  int32_t substeps;      /* sub-steps per flight interval = per Poisson refresh */
  int32_t n_bins;        /* rate-table bins */
  double dE_eV;          /* rate-table bin width */
  double T0_K;           /* uniform lattice temperature (see mc_set_lattice_temperature) */
  double T_init_K;       /* temperature of the initial Maxwellian */
  double N_D_m3;         /* donor density (all active: N_I = n = N_D) */
  double F_bulk[3];      /* bulk mode: uniform field, V/nm */
  double L_nm[3];        /* device mode: domain x (channel), y (cut width), z (height) */
  int32_t n_cells[3];    /* device mode: subcells along x, y, z */
  double gate_x_nm[2];   /* device mode: gated channel stretch */
  double Vgs, Vds, phi_offset; /* device mode: gate, drain, gate work-function offset (V) */
} mc_config;

/* Window tallies of one instance, accumulated since the last reset. */
typedef struct {
  uint32_t intervals;       /* flight intervals in the window */
  uint32_t intervals_total; /* intervals since mc_init */
  double t_window_fs;
  uint64_t n_alive;         /* electrons alive now */
  uint64_t selections;      /* scattering selections (real + self) */
  uint64_t self_events;
  uint64_t overflow;        /* selections above the table top (clamped to the last bin) */
  uint64_t real[3][10];     /* real events per initial valley and mechanism */
  uint64_t exits[2];        /* electrons absorbed by source (0) and drain (1) */
  uint64_t injections[2];   /* electrons injected at source and drain */
  uint64_t segments;        /* free-flight segments: alive x substeps + selections */
  uint64_t reflect_guard;   /* lateral reflections that needed clamping */
  double weight;            /* electrons per superparticle (device mode) */
  double drain_current_A;   /* e w (exits_D - injections_D) / t_window */
  int32_t flags;            /* sticky device error flags (mc_status of the first) */
} mc_tally_out;

/* Device pointers of one instance's structure-of-arrays particle state.
 * kx..z have `elem_bytes` bytes each (8 in FP64 mode, 4 in FP32 mode); meta
 * packs id << 3 | alive << 2 | valley. */
typedef struct {
  void *kx, *ky, *kz, *x, *y, *z;
  uint32_t *meta;
  int32_t capacity;
  int32_t elem_bytes;
} mc_particles_view;

typedef struct mc_ctx mc_ctx;

const char *mc_status_string(int status);
const char *mc_last_error(const mc_ctx *ctx);

/* Bytes of device workspace needed for `n_instances` configurations;
 * 0 if the configurations are invalid. */
size_t mc_workspace_bytes(const mc_config *cfgs, int n_instances);

/* Validate, build the rate tables (1 meV midpoints to the table top) and
 * per-subcell factors, the self-scattering bounds Gamma_v, the initial
 * Maxwellian ensemble, the Poisson factors and (device mode) the first
 * deposit/injection/Poisson refresh (electron MC paragraph).  MC_E_ARG for
 * capacity < n_particles, dt <= 0, table top < 3 eV, inconsistent instances,
 * a device grid with ny*nz > 32 or more than 4096 subcells, or a workspace
 * that is too small. */
int mc_init(mc_ctx **out, const mc_config *cfgs, int n_instances, void *d_workspace, size_t ws_bytes,
            void *hip_stream);
int mc_destroy(mc_ctx *ctx);

/* Per-subcell lattice temperature of one instance (ncell host doubles,
 * index (ix*ny + iy)*nz + iz; one value in bulk mode).  Rebuilds the
 * factors and Gamma_v: the lattice temperature sets the electron rates
 * (coupling paragraph). */
int mc_set_lattice_temperature(mc_ctx *ctx, int instance, const double *h_T_cells);

/* Replace the T-independent rate shapes (host [3][n_bins][10] doubles and
 * 4k^2 at bin midpoints [3][n_bins]) and rebuild Gamma_v. */
int mc_set_tables(mc_ctx *ctx, const double *h_shape, const double *h_k4);

/* Advance every instance by n_substeps sub-steps (a multiple of `substeps`)
 * (electron MC paragraph: free flight under the local field in the Kane
 * bands, scattering chosen by self-scattering among impurity, polar-optical,
 * acoustic and intervalley rates, the electron-phonon energy exchange counted
 * per subcell, the Poisson refresh).  Per interval: free flight and
 * scattering with heat counts for every live electron, then in device mode
 * the subcell deposit, the contact refill and the Poisson refresh.
 * Asynchronous on the context's stream; MC_E_ARG for a count that is not a
 * multiple of `substeps` or an unsupported launch shape, MC_E_HIP if a
 * launch or the graph capture fails.  Faults inside the kernels (event
 * guard, non-finite state, exhausted capacity) become sticky per-instance
 * flags that mc_tally returns. */
int mc_step(mc_ctx *ctx, int n_substeps);

/* Deposit electrons per subcell, refill the contact subcells to neutrality,
 * solve the Poisson equation and refresh the field, for all instances
 * (electron MC paragraph: the field follows from the terminal voltages and
 * the electron concentration counted in the subcells).  Device mode only
 * (MC_OK and nothing done in bulk mode); done after every interval by
 * mc_step.  Asynchronous; MC_E_HIP if a launch fails. */
int poisson_update(mc_ctx *ctx);

/* Copy the window tallies of one instance (electron MC paragraph: the
 * events behind the heat counted per subcell and the contact currents) into
 * the caller's h_out; reset_window != 0 starts a new window of every
 * instance afterwards (counts, maps and history rows).  Synchronises the
 * stream.  Returns MC_OK or the first sticky device error of the instance
 * (h_out filled either way), MC_E_ARG for a bad instance or pointer,
 * MC_E_HIP for a failed copy. */
int mc_tally(mc_ctx *ctx, int instance, mc_tally_out *h_out, int reset_window);

/* Window maps of one instance: h_heat4 [ncell][4] phonon counts (LO emit, LO
 * absorb, intervalley emit, intervalley absorb), h_dens_sum [ncell] electron
 * counts summed over the window's refreshes, and the derived FP64 maps:
 * h_heat_Wm3 the net phonon-emission power density w e (hw_LO (em - ab) +
 * hw_iv (em - ab)) / (V_c t_window), h_density_m3 the mean electron density
 * w <count> / V_c, h_emit_Wm3 the emission-only power density (the emitted
 * phonon energy of the thermal-resistance passage, per volume and time).
 * Heat is counted per subcell (electron MC paragraph).  Any pointer may be
 * NULL.  Synchronises the stream. */
int mc_maps(mc_ctx *ctx, int instance, uint64_t *h_heat4, uint64_t *h_dens_sum, double *h_heat_Wm3,
            double *h_density_m3, double *h_emit_Wm3);

/* Per-interval history rows (8 doubles each) since the last window reset,
 * at most 8192.
 * Bulk mode, at each interval end: live electrons, sum vx, sum vy, sum vz
 * (nm/fs), sum of kinetic energies (eV), electrons in Gamma1, U, Gamma3.
 * Device mode, after each refresh: the window's cumulative source exits,
 * drain exits, source injections and drain injections, the electrons present
 * after the refill, the mean potential (V) and the root-mean-square field
 * magnitude (V/nm) over the subcells, the intervals done since mc_init.
 * h_rows may be NULL (count only).  Synchronises the stream. */
int mc_history(mc_ctx *ctx, int instance, double *h_rows, int max_rows, int *n_rows);

/* Observables of one instance over the current window, computed on the host
 * from the window's counts and history rows (electron MC paragraph: heat
 * counted per subcell, steady state once current and field no longer
 * change; the thermal-resistance passage: the emitted phonon energy). */
typedef struct {
  uint32_t intervals;          /* intervals in the window */
  double t_window_fs;
  /* device mode */
  double drain_current_A;      /* e w (drain exits - drain injections) / t_window */
  double source_current_A;     /* e w (source exits - source injections) / t_window (negative when
                                  electrons enter at the source) */
  double heat_W;               /* net phonon-emission power over the domain */
  double emit_W;               /* emission-only power (emitted phonon energy / t_window) */
  /* bulk mode: window means of the per-interval ensemble averages */
  double drift_velocity_ms[3]; /* mean electron velocity, m/s */
  double mean_energy_eV;       /* mean kinetic energy */
  double valley_fraction[3];   /* Gamma1, U, Gamma3 */
  /* steady state.  Two per-interval series: device mode the drain current and
   * the rms field, bulk mode the mean v_z and the mean kinetic energy.  The
   * last 2h intervals of the window (h = intervals / 2) form two halves;
   * each half's mean and its standard error come from 10 batch means. */
  double half_mean[2][2];      /* [series][half] */
  double half_se[2][2];
  int32_t steady;              /* 1: both series' half means within 3 combined standard errors; 0: not;
                                  -1: a half holds fewer than 10 intervals */
} mc_observables_out;

/* Returns MC_OK, the first sticky device error of the instance (after
 * filling *out), or MC_E_ARG / MC_E_HIP.  Synchronises the stream. */
int mc_observables(mc_ctx *ctx, int instance, mc_observables_out *out);

/* Device pointers of one instance's particle state, the per-electron (k, r,
 * valley) ensemble of the electron MC paragraph, for in-place readers on the
 * context's stream.  The pointers stay owned by the workspace and valid
 * until mc_destroy; MC_E_ARG for a bad instance or pointer. */
int mc_particles(mc_ctx *ctx, int instance, mc_particles_view *out);

/* Copy one instance's particles to / from host arrays of `capacity` entries:
 * k[cap][3], r[cap][3] (FP64; r ignored and may be NULL in bulk mode),
 * valley, alive (int32), id (uint32).  Both are ordered after the work already
 * enqueued on the context's stream and complete before returning.  A write
 * checks every entry first (identity below 2^29, valley 0..2) and returns
 * MC_E_ARG without changing anything if one is bad.  After a write the live
 * electrons may sit in any slot: the particle kernel scans all of the
 * instance's slots until a refresh compacts them (results do not depend on
 * the slots; electrons are identified by id). */
int mc_read_particles(mc_ctx *ctx, int instance, double *h_k, double *h_r, int32_t *h_valley, int32_t *h_alive,
                      uint32_t *h_id);
int mc_write_particles(mc_ctx *ctx, int instance, const double *h_k, const double *h_r, const int32_t *h_valley,
                       const int32_t *h_alive, const uint32_t *h_id);

/* The configuration an instance was created with, and its current
 * per-subcell lattice temperature (ncell doubles).  MC_E_ARG for a bad
 * instance or pointer. */
int mc_get_config(const mc_ctx *ctx, int instance, mc_config *out);
int mc_get_lattice_temperature(const mc_ctx *ctx, int instance, double *h_T_cells);

/* Potential, field and electron counts of the last refresh (ncell entries). */
int mc_read_fields(mc_ctx *ctx, int instance, double *h_phi, double *h_field, uint32_t *h_count);

/* Rate shapes [3][n_bins][10], 4k^2 [3][n_bins], per-cell factors [ncell][7]
 * and Gamma_v [3] (1/fs) of one instance.  Any pointer may be NULL. */
int mc_read_tables(mc_ctx *ctx, int instance, double *h_shape, double *h_k4, double *h_factors, double *h_gamma);

/* Launch shape of the particle kernel: workgroup size (64..1024, multiple of
 * 64; above 512 only for FP32 state and variants 0, 2 and 3, else mc_step
 * returns MC_E_ARG) and tile
 * size (particles per tile, multiple of the workgroup size).
 * Variants 0 and 1 launch one workgroup per tile; variants 2 and 3 launch as
 * many workgroups as the GPU holds at once and use the tiles only for the
 * contact refill's free-slot counts.  Results do not depend on the shape.
 * MC_E_ARG if unsupported.  n_tiles reports the tiles, not the persistent
 * grid. */
int mc_set_launch(mc_ctx *ctx, int block, int tile);
int mc_get_launch(const mc_ctx *ctx, int *block, int *tile, int *n_tiles);

/* Subcells of the context's grid (nx * ny * nz in device mode, 1 in bulk
 * mode): the length of every per-subcell array of the API. */
int mc_get_ncell(const mc_ctx *ctx, int *ncell);

/* Number of instances of the context, and its HIP stream (the hipStream_t
 * given to mc_init, as void*): work a caller enqueues there is ordered with
 * the context's own. */
int mc_get_instances(const mc_ctx *ctx, int *n_instances);
int mc_get_stream(const mc_ctx *ctx, void **stream);

/* Residency of the particle kernel (current variant and precision) at
 * workgroup size `block`: workgroups per compute unit given its registers and
 * LDS histogram, and the device's compute units.  Lets a tuner pick tile
 * counts that fill whole rounds of resident workgroups.  MC_E_ARG for an
 * unsupported block, MC_E_HIP if the runtime query fails. */
int mc_occupancy(mc_ctx *ctx, int block, int *wg_per_cu, int *n_cu);

/* Particle-kernel variant: 0 = lane refill (each lane pulls the next electron
 * of its tile as soon as its own finishes the interval; default), 1 = one
 * electron per lane per pass, 2 = persistent (as many workgroups as the GPU
 * holds at once, each bound to one instance, in proportion to its slots at
 * first and then, with several instances, to its segments over the previous
 * interval, and owning every nw-th chunk of 128 slots of it, so each samples
 * the whole slot range and the launch is balanced however the live electrons
 * are spread over the slots), 3 = persistent with staged slots (as 2; each wavefront copies
 * the next 128 slots of its chunks into LDS while its lanes take electrons from
 * the current 128, which pays off while the state outgrows the Infinity
 * Cache).  Results are identical up to the compiler's floating-point
 * contraction choices in each variant (variants 0, 2 and 3 share the
 * per-electron code and give the same bits).  MC_E_ARG for another value,
 * MC_E_HIP if the occupancy query for variant 2 or 3 fails. */
int mc_set_variant(mc_ctx *ctx, int variant);

/* Replay each interval from a captured hipGraph (1) or launch eagerly (0). */
int mc_use_graph(mc_ctx *ctx, int enable);

/* Time the particle kernel and the refresh chain of every interval with HIP
 * events recorded on the context's stream (eager launches; graph replay is
 * switched off while profiling).  mc_profile_read synchronises and returns
 * total milliseconds and launch counts since the last reset. */
int mc_profile(mc_ctx *ctx, int enable);
int mc_profile_read(mc_ctx *ctx, double *flight_ms, int *n_flight, double *refresh_ms, int *n_refresh, int reset);

/* Checkpoint of the Monte Carlo state that evolves (electron MC paragraph:
 * the ensemble and its window tallies): particles, counters, tallies and
 * history, potential and field, refill plans, the interval counters and the
 * lattice temperatures.  With h_buf NULL, *bytes receives the size;
 * otherwise h_buf (caller-owned, *bytes long) receives the checkpoint and
 * *bytes its length (MC_E_ARG if too small).  Restoring into a context built
 * from the same configurations continues bit-identically: the checkpoint
 * carries the rate tables, factors and self-scattering bounds with the
 * temperatures; set-up products (the Poisson inverse) and per-interval
 * scratch stay the restoring context's own, and it keeps its launch shape.
 * A checkpoint starts
 * with a format word: mc_restore rejects (MC_E_ARG) one written by a
 * library whose layout differs, or one of another context's size.  Both
 * synchronise the stream. */
int mc_checkpoint(mc_ctx *ctx, void *h_buf, size_t *bytes);
int mc_restore(mc_ctx *ctx, const void *h_buf, size_t bytes);

/* ------------------------------------------------------------------------
 * MLP surrogate of the Monte Carlo: (Vgs, Vds, log10 doping, per-subcell
 * lattice temperature) -> per-subcell heat and electron-density maps.  It
 * stands in for the electron MC when the thermal side of the hybrid method
 * (coupling paragraph) needs heat maps for many temperature fields.  BF16
 * matrix-core GEMMs with FP32 accumulation, GELU (exact normal CDF) hidden
 * layers, FP32 master weights and Adam.  Device pointers below are caller
 * allocations of FP32 row-major [batch][n_in] inputs and [batch][n_out]
 * outputs.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_in;      /* raw input features */
  int32_t n_out;     /* outputs (any positive count; padded internally to a multiple of 8) */
  int32_t width;     /* hidden width (multiple of 8) */
  int32_t depth;     /* hidden layers */
  int32_t ensemble;  /* independently initialised members (spread = predicted error) */
  int32_t max_batch; /* largest batch of any call */
  uint64_t seed;     /* Philox key of the weight initialisation */
  float beta1, beta2, eps; /* Adam */
  float weight_decay;      /* decoupled (AdamW) decay of the weights, not the biases; 0 = plain Adam */
} sg_config;

typedef struct sg_ctx sg_ctx;

/* Device workspace bytes for cfg; 0 if invalid. */
size_t sg_workspace_bytes(const sg_config *cfg);
int sg_init(sg_ctx **out, const sg_config *cfg, void *d_workspace, size_t ws_bytes, void *hip_stream);
int sg_destroy(sg_ctx *ctx);
const char *sg_last_error(const sg_ctx *ctx);
/* K (inputs, the first padded to a multiple of 32) and N (outputs) of a weight layer. */
int sg_layer_dims(const sg_ctx *ctx, int layer, int *K, int *N);
/* Host FP32 per-feature mean and scale of inputs and outputs (z-scoring). */
int sg_set_normalization(sg_ctx *ctx, const float *h_x_mean, const float *h_x_std, const float *h_y_mean,
                         const float *h_y_std);
/* Normalised predictions of one member (asynchronous). */
int sg_forward(sg_ctx *ctx, int member, const float *d_x, int batch, float *d_pred);
/* Forward, mean-squared error on z-scored targets, gradients of every layer
 * (kept in the workspace); h_loss (may be NULL) gets the loss (synchronises). */
int sg_backward(sg_ctx *ctx, int member, const float *d_x, const float *d_y, int batch, float *h_loss);
/* One bias-corrected Adam step of one member from its last gradients
 * (Kingma & Ba: m and v moments, each divided by 1 - beta^t at step t). */
int sg_adam(sg_ctx *ctx, int member, float lr);
/* sg_backward then sg_adam for one member: the members of the ensemble are
 * trained independently (each on its own batches), which is what makes
 * their spread a measure of the error. */
int sg_train_step(sg_ctx *ctx, int member, const float *d_x, const float *d_y, int batch, float lr, float *h_loss);
/* De-normalised ensemble mean and spread of every output (d_std may be NULL;
 * sample standard deviation over the members), asynchronous.  The spread is
 * per output; sg_predict_or_mc reduces it to one predicted relative error. */
int sg_predict(sg_ctx *ctx, const float *d_x, int batch, float *d_mean, float *d_std);
/* sg_predict for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid it): the same
 * small-batch kernels, with their scratch (normalised inputs, activations,
 * split partial sums, the members' predictions) in a static 8 MiB device
 * array of the library instead of the context's workspace.  Each GPU holds
 * its own array until the process ends (its address is taken once per
 * device at sg_init); every call on a GPU shares it, so calls that overlap
 * on one GPU race.  Nothing in it needs clearing: each call writes what it
 * reads.  batch 1..8 (and at most the context's max_batch); MC_E_ARG for a
 * larger batch or a network whose scratch would not fit (the split count
 * shrinks to fit before that: 4 members of 1024 wide with 3602 outputs fit at
 * batch 8).  Results equal sg_predict's up to the order of the split sums.
 * Allocates nothing; asynchronous on the context's stream. */
int sg_predict_static(sg_ctx *ctx, const float *d_x, int batch, float *d_mean, float *d_std);

/* FP32 master parameters and last gradients of one layer: W [K][N], b [N]. */
int sg_get_params(sg_ctx *ctx, int member, int layer, float *h_W, float *h_b);
int sg_set_params(sg_ctx *ctx, int member, int layer, const float *h_W, const float *h_b);
int sg_get_grads(sg_ctx *ctx, int member, int layer, float *h_dW, float *h_db);

/* One query of sg_predict_or_mc (host memory). */
typedef struct {
  const float *h_x;        /* raw features [n_in]: Vgs, Vds, log10 doping (cm^-3), lattice T per subcell */
  const float *h_box_lo;   /* training box [n_in] of the features; both NULL: no box check */
  const float *h_box_hi;
  float calib;             /* calibration factor applied to the ensemble spread */
  float tol;               /* largest predicted relative error the surrogate may answer with */
  int32_t warm_substeps;   /* Monte Carlo fallback: sub-steps before the averaging window (>= 0) */
  int32_t window_substeps; /* sub-steps averaged (>= 1); both multiples of the context's interval */
} sg_query;

/* The surrogate's answer where it can vouch for it, the Monte Carlo's
 * elsewhere (coupling paragraph: heat maps for the thermal side).
 * The network's outputs are read as the encoding [heat shape (ncell),
 * density shape (ncell), log heat norm, log density norm], so n_out =
 * 2 ncell + 2; each map is its unit-norm shape times the exponential of its
 * log-norm (decoded from the ensemble mean).  The spread of an output is
 * the sample standard deviation over the members (divisor members - 1).
 * The predicted relative error is calib x the larger, over the two maps, of
 * hypot(|spread of the shape| / |mean shape|, spread of the log-norm)
 * (|.| the Euclidean norm over the ncell subcells).
 * When it exceeds tol, or the features leave the training box (each feature
 * within [lo, hi] widened by 1e-6 max(1, hi - lo)), the Monte Carlo runs on
 * instance `instance` of `mc`, which must be set up for the same point: the
 * same grid, Vgs, Vds, log10 doping and per-subcell temperature as the
 * features (relative 1e-5), else MC_E_ARG.  It runs warm_substeps sub-steps,
 * a window reset (of the whole context) and window_substeps sub-steps;
 * every instance of `mc` advances.  h_maps [2 ncell] receives heat (W/m^3,
 * the net map of mc_maps) then electron density (m^-3); h_pred_err (may be
 * NULL) the predicted error; used_mc (may be NULL) 1 if the Monte Carlo
 * answered.  Synchronises both contexts' streams.  Returns MC_OK; MC_E_ARG
 * for bad arguments, an output width that is not such an encoding, a
 * missing or mismatched `mc` when the Monte Carlo is needed; otherwise the
 * status of the Monte Carlo calls, including a sticky device error raised
 * during the window (the maps are then still filled). */
int sg_predict_or_mc(sg_ctx *ctx, mc_ctx *mc, int instance, const sg_query *query, double *h_maps,
                     float *h_pred_err, int *used_mc);

#ifdef __cplusplus
}
#endif
#endif /* GFMC_H */
