/*
 * gffo.h -- C ABI of the Fourier's-law heat spreading of libgfmc.so (MI355X,
 * gfx950): the chip-scale conduction outside the phonon Monte Carlo domain
 * of the coupling paragraph of Hao, Zhao, Xiao and Kronenfeld,
 * arXiv:1707.09073 (steady state, size-modified conductivities, the
 * GaN-substrate interface resistance of Eq. (3)).
 *
 * Conventions as in gfmc.h and gfph.h: plain C, every call returns an
 * mc_status (0 = MC_OK), the caller owns device memory (a workspace of
 * fo_workspace_bytes) and the HIP stream (void*), work is asynchronous
 * unless a call says it synchronises.  SI units.
 */
#ifndef GFFO_H
#define GFFO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A steady conduction problem on a tensor-product grid of n[0] x n[1] x n[2]
 * cells (index (i*ny + j)*nz + k), cell faces at the given edge coordinates.
 * Face conductance between neighbouring cells c, c' across a face of area
 * A: A / (d/(2 kappa_c) + d'/(2 kappa_c') [+ R_K on the interface plane]),
 * zero if either cell is void (kappa 0).  A face marked Dirichlet holds the
 * rise at 0 (the temperature at T_sink), with conductance A / (d/(2 kappa))
 * from the cell centre; other outer faces are adiabatic. */
typedef struct {
  int32_t n[3];
  int32_t dirichlet[6];   /* x = 0, x = L, y = 0, y = L, z = 0, z = L: 1 = held at T_sink, 0 = adiabatic */
  int32_t k_interface;    /* the z-face between cells k_interface - 1 and k_interface carries R_K; -1: none */
  double R_K_m2KW;        /* interface resistance, m^2 K / W (1 / the conductance of Eq. (3)) */
  double T_sink_K;
  int32_t max_iterations; /* conjugate-gradient iterations (>= 1) */
  double rtol;            /* stop when ||b - A x|| <= rtol ||b|| (2-norms, > 0) */
  int32_t warm_start;     /* 1: start from the rise d_T holds on entry (d_T - T_sink in live cells; an
                             earlier solution of a nearby problem), 0: from zero */
} fo_config;

/* Device workspace bytes for cfg (256-byte aligned), 0 if cfg is invalid
 * (a dimension < 1, more than 2^27 cells, bad flags or tolerances). */
size_t fo_workspace_bytes(const fo_config *cfg);

/* Solve for the temperature: d_edges (device, n[0]+1 + n[1]+1 + n[2]+1
 * increasing coordinates in m, the x edges, then y, then z), d_kappa
 * (device, ncell, W/(m K); 0 marks a void cell, which takes T_sink and no
 * heat), d_q (device, ncell, W generated in the cell), d_T (device, ncell,
 * in with warm_start, out, K).  Jacobi-preconditioned conjugate gradients
 * on the rise above T_sink, dot products reduced in a fixed order (results
 * do not depend on the launch); with warm_start the iteration starts from
 * the rise d_T holds, with the same stopping rule.  Synchronises the stream; *iterations and *rel_residual (may
 * be NULL) receive the iterations done and ||b - A x|| / ||b||.  MC_E_ARG for
 * an invalid configuration, pointer or workspace; MC_E_RANGE if the
 * tolerance is not reached within max_iterations (d_T then holds the last
 * iterate); MC_E_HIP for a failed launch. */
int fo_solve(const fo_config *cfg, const double *d_edges, const double *d_kappa, const double *d_q, double *d_T,
             int *iterations, double *rel_residual, void *d_ws, size_t ws_bytes, void *stream);

/* Per-cell inputs of a chip problem: d_kappa[c] = h_kappa_by_material[
 * d_material[c]] (host table of n_materials values, W/(m K); material ids
 * 0 .. n_materials - 1), and d_q[c] = scale * d_src[d_src_index[c]] where
 * d_src_index[c] >= 0 (the cell lies in a wire and takes that subcell's
 * heat: the electron Monte Carlo's map, W per subcell, times the ratio of
 * the cell's volume to the subcell's in `scale`), else 0.  Every wire takes
 * the same map (the coupling paragraph finds the heat generation of the
 * wires of the array nearly equal).  Device arrays of ncell entries (u8,
 * i32), d_src of n_src entries.  Asynchronous.  MC_E_ARG for a bad pointer,
 * count or material table (at most 16). */
int fo_chip_fields(const uint8_t *d_material, const double *h_kappa_by_material, int n_materials,
                   const int32_t *d_src_index, const double *d_src, int n_src, double scale, long long ncell,
                   double *d_kappa, double *d_q, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GFFO_H */
