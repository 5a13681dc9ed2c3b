// gfmc_kernels.h -- gfx950 particle kernels of the electron Monte Carlo step
// and the structures they share with the kernels around them
// (gfmc_refresh.h).
//
// One flight interval (K sub-steps, one Poisson refresh) is:
//   k_flight_refill  per lane-slot: free flight + self-scattering selection
//                    for K sub-steps, lanes refilled from an LDS queue of the
//                    tile's particles; mechanism counts, heat and the deposit
//                    of the survivors per subcell kept in LDS and added to
//                    the instance's sums at the end of the workgroup
//                    (k_flight: one particle per thread, same physics;
//                    k_flight_persist: resident workgroups, each working
//                    every nw-th chunk of its instance's slots).
// then, in gfmc_refresh.h:
//   k_inject_plan    moves the sums into the counts and heat, plans the
//                    refill of the contact subcells to neutrality (device
//                    mode) and forms the Poisson right-hand side (charge
//                    balance per cell with the terminal faces);
//   k_compact_scatter, k_inject_slots, k_inject_fill  compact the slots when
//                    holes have gathered, list the free slots, and create one
//                    electron per thread;
//   k_poisson_gemv/gemm  the potential from the dense inverse of the
//                    finite-volume Poisson matrix (built once at init by
//                    k_poisson_factor + k_poisson_inverse), then
//   k_field          the cell-centred field.
// Bulk mode replaces deposit, injection and Poisson by k_bulk_* (per-interval
// observables).
#pragma once
#include "gfmc_device.h"

namespace gfmc {

constexpr int kNCnt = 48;  // u64 counters per instance
enum {
  C_SEL = 0, C_SELF = 1, C_OVF = 2, C_REAL = 3, C_EXIT0 = 33, C_EXIT1 = 34, C_INJ0 = 35, C_INJ1 = 36,
  C_REFL = 37, C_PROC = 38
};
enum { CTL_INTERVAL = 0, CTL_WINDOW = 1 };
constexpr uint32_t kNoRow = 0xffffffffu;
// Per-interval history rows, 8 doubles each, per instance.  Bulk mode: live
// electrons, sum of vx, vy, vz (nm/fs), sum of kinetic energies (eV),
// electrons in Gamma1, U, Gamma3.  Device mode (after each refresh): the
// window's cumulative source exits, drain exits, source injections and drain
// injections, the electrons present after the refill, the mean potential (V)
// and the root-mean-square field magnitude (V/nm) over the subcells, and the
// intervals done since initialisation.
constexpr int kHistCap = 8192;

struct TileDesc {
  int inst;
  int count;
  long long start;  // first slot (global index)
};

struct InstParams {
  uint32_t key0, key1, tagw;
  int cap;
  long long base;
  int t0, t1;     // tile range of the instance
  int target;     // neutral electrons per contact subcell
  int w0, w1;     // persistent kernel: workgroups of the instance
  int nchunk;     // persistent kernel: slot chunks of the instance
  double N_D_nm;  // donors per nm^3
  double N_D_m3;  // donors per m^3
  double w;       // electrons per superparticle
  double Vgs, Vds, phig;
  double F[3];    // bulk field
  double T_init;
};

struct Plan {
  uint32_t Q, id0, u, pad;
  uint32_t alive;    // live electrons of the instance before the refill
  uint32_t compact;  // 1: compact the instance's slots in this refresh
  uint32_t hw;       // slots in use (relative): every live electron lies below it
  uint32_t row;      // history row of this refresh (device mode, after a flight), else kNoRow
  uint32_t need[64];
  uint32_t off[64];
};

template <typename T>
struct FlightArgs {
  const TileDesc* tiles;
  const InstParams* ip;
  const T* table;
  const T* fac;
  const T* field;
  const T* gamma;
  T *kx, *ky, *kz, *x, *y, *z;
  uint32_t* meta;
  unsigned long long* acc;  // device mode: the interval's histogram sums, [instance][5 ncell]
  uint32_t* tile_dead;
  unsigned long long* counters;
  int* flags;
  const uint32_t* ctl;
  const Plan* plan;     // lane-refill kernel (device mode): slots in use per instance
  const int* wg_inst;  // persistent kernel: instance of each workgroup
  int tile, chunk;     // persistent kernel: tile and chunk sizes (slots)
  int n_inst;
  uint32_t nt_slots;   // device mode: state is read non-temporally once more slots than this are in use
  Mat<T> M;
  Geo<T> G;
  int nb;
  T dE;
  T TP;
};

struct Cnt {
  uint32_t sel, self, ovf, ex0, ex1, refl, dead, proc;
};

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__device__ __forceinline__ void set_flag(int* flags, int inst, int code) { atomicCAS(flags + inst, 0, code); }

// Select a mechanism by u1 Gamma_v against the running sum of the tabulated
// rates of the cell; apply its final state.  Returns the mechanism, -1 = self.
template <typename T>
__device__ __forceinline__ int scatter(const FlightArgs<T>& a, const T* f, const T (&gam)[3], int& v, T& kx, T& ky,
                                       T& kz, const uint4 w, int cell, int ncell, Cnt& c, uint32_t* sh_heat,
                                       uint32_t* sh_real) {
  const Mat<T>& M = a.M;
  const T k2 = ksq(kx, ky, kz);
  const T g = Ar<T>::dv(M.ck * k2, pick3(M.m, v));
  const T E = kane_E(g, pick3(M.alpha, v));
  const T eb = Ar<T>::dv(E, a.dE);
  int b;
  if (!(eb < (T)a.nb)) { b = a.nb - 1; c.ovf++; }
  else b = (int)eb;
  const T* S = a.table + ((size_t)v * a.nb + b) * kTRow;
  T Sr[11];
#pragma unroll
  for (int q = 0; q < 11; ++q) Sr[q] = S[q];
  const T rs = Ar<T>::u01(w.y) * pick3(gam, v);
  T cum = (T)0;
  int m = -1;
#pragma unroll
  for (int q = 0; q < kNM; ++q) {
    cum += tab_term<T>(Sr, f, q);
    if (m < 0 && rs < cum) m = q;
  }
  c.sel++;
  if (m < 0) { c.self++; return -1; }
  int vp = v;
  T Ep;
  if (m <= 1) Ep = E;
  else if (m == 2) Ep = E + M.hw_lo;
  else if (m == 3) Ep = E - M.hw_lo;
  else {
    vp = (m - 4) >> 1;
    Ep = E + pick3(M.Ec, v) - pick3(M.Ec, vp) + (((m - 4) & 1) ? -M.hw_iv : M.hw_iv);
  }
  if (!(Ep > (T)0)) { c.self++; return -1; }
  atomicAdd(sh_real + v * kNM + m, 1u);
  {
    // heat slot: 0 LO emission, 1 LO absorption, 2 intervalley emission,
    // 3 intervalley absorption; none for the elastic mechanisms
    const int hs = m == 3 ? 0 : (m == 2 ? 1 : (m >= 4 ? (((m - 4) & 1) ? 2 : 3) : -1));
    if (hs >= 0) atomicAdd(sh_heat + hs * ncell + cell, 1u);
  }
  // polar angle relative to k, sampled as X = 1 - cos; sin = sqrt(X (2 - X))
  // keeps full relative accuracy for forward scattering
  const T u2 = Ar<T>::u01(w.z), u3 = Ar<T>::u01(w.w);
  T X;
  if (m == 2 || m == 3) {
    const T gp = Ep * ((T)1 + pick3(M.alpha, v) * Ep);
    const T sg = Ar<T>::sq(g), sgp = Ar<T>::sq(gp);
    const T xi = Ar<T>::dv((T)2 * sg * sgp, (sg - sgp) * (sg - sgp));
    X = Ar<T>::dv(Ar<T>::em1(u2 * Ar<T>::l1p((T)2 * xi)), xi);
  } else {
    // Brooks-Herring; with a4 = 0 the same expression is the isotropic
    // X = 2 u2 exactly (a division by 1)
    const T a4 = m == 1 ? Ar<T>::dv((T)4 * k2, f[6]) : (T)0;
    X = Ar<T>::dv((T)2 * u2, (T)1 + ((T)1 - u2) * a4);
  }
  X = fmin(fmax(X, (T)0), (T)2);
  const T ct = (T)1 - X;
  const T st = Ar<T>::sq(X * ((T)2 - X));
  T cp, sp;
  Ar<T>::cs2pi(u3, cp, sp);
  const T kn = Ar<T>::sq(k2);
  T nx = (T)0, ny = (T)0, nz = (T)1;
  if (kn > (T)0) { nx = Ar<T>::dv(kx, kn); ny = Ar<T>::dv(ky, kn); nz = Ar<T>::dv(kz, kn); }
  T e1[3], e2[3];
  onb<T>(nx, ny, nz, e1, e2);
  const T gpp = Ep * ((T)1 + pick3(M.alpha, vp) * Ep);
  const T kp = Ar<T>::sq(Ar<T>::dv(gpp * pick3(M.m, vp), M.ck));
  const T sc = st * cp, ss = st * sp;
  kx = kp * dot3(sc, e1[0], ss, e2[0], ct, nx);
  ky = kp * dot3(sc, e1[1], ss, e2[1], ct, ny);
  kz = kp * dot3(sc, e1[2], ss, e2[2], ct, nz);
  v = vp;
  return m;
}

// Free flight for dt in the field (fx, fy, fz): k exact, r by the trapezoid
// of the end-point velocities, specular lateral walls.  Returns -1 inside,
// else the contact left through (0 source, 1 drain).
template <typename T, bool DEV>
__device__ __forceinline__ int drift(const FlightArgs<T>& a, int v, T dt, T fx, T fy, T fz, T& kx, T& ky, T& kz,
                                     T& x, T& y, T& z, Cnt& c) {
  const Mat<T>& M = a.M;
  const T k1x = kx - M.cf * fx * dt, k1y = ky - M.cf * fy * dt, k1z = kz - M.cf * fz * dt;
  if (DEV) {
    const T s0 = vel_factor(M, v, energy(M, v, kx, ky, kz));
    const T s1 = vel_factor(M, v, energy(M, v, k1x, k1y, k1z));
    const T h = (T)0.5 * dt;  // explicit fused forms, as in drift_e
    x = fma(h, fma(s0, kx, s1 * k1x), x);
    y = fma(h, fma(s0, ky, s1 * k1y), y);
    z = fma(h, fma(s0, kz, s1 * k1z), z);
  }
  kx = k1x; ky = k1y; kz = k1z;
  if (!DEV) return -1;
  if (x < (T)0) return 0;
  if (x > a.G.L[0]) return 1;
  {
    const T L = a.G.L[1];
    int guard = 0;
    while ((y < (T)0 || y > L) && guard < 8) { y = y < (T)0 ? -y : (T)2 * L - y; ky = -ky; ++guard; }
    if (y < (T)0 || y > L) { y = y < (T)0 ? (T)0 : L; c.refl++; }
  }
  {
    const T L = a.G.L[2];
    int guard = 0;
    while ((z < (T)0 || z > L) && guard < 8) { z = z < (T)0 ? -z : (T)2 * L - z; kz = -kz; ++guard; }
    if (z < (T)0 || z > L) { z = z < (T)0 ? (T)0 : L; c.refl++; }
  }
  return -1;
}

// One flight interval [0, K dt) of one electron.  The field is constant over
// the interval, so the remaining flight time is drawn afresh at its start.
template <typename T, bool DEV>
__device__ __forceinline__ bool fly(const FlightArgs<T>& a, const InstParams& P, const T* fac, const T* field,
                                    const T (&gam)[3], uint32_t n_int, int ncell, int& v, uint32_t id, T& kx, T& ky,
                                    T& kz, T& x, T& y, T& z, Cnt& c, uint32_t* sh_heat, uint32_t* sh_real,
                                    bool& guard_hit) {
  uint4 w = philox(id, n_int, 0u, P.tagw, P.key0, P.key1);
  T t = (T)0;
  T tau = Ar<T>::dv(-Ar<T>::ln(Ar<T>::u01(w.x)), pick3(gam, v));
  uint32_t j = 0;
  for (;;) {
    int cell = DEV ? cell_of(a.G, x, y, z) : 0;
    const T* F = field + 4 * cell;
    const T fx = F[0], fy = F[1], fz = F[2];
    if (t + tau >= a.TP) {
      const int ex = drift<T, DEV>(a, v, a.TP - t, fx, fy, fz, kx, ky, kz, x, y, z, c);
      if (ex == 0) { c.ex0++; return false; }
      if (ex == 1) { c.ex1++; return false; }
      return true;
    }
    const int ex = drift<T, DEV>(a, v, tau, fx, fy, fz, kx, ky, kz, x, y, z, c);
    if (ex == 0) { c.ex0++; return false; }
    if (ex == 1) { c.ex1++; return false; }
    t += tau;
    ++j;
    if (j > (uint32_t)kMaxEvents) { guard_hit = true; return true; }
    w = philox(id, n_int, j, P.tagw, P.key0, P.key1);
    if (DEV) cell = cell_of(a.G, x, y, z);
    scatter<T>(a, fac + kFRow * cell, gam, v, kx, ky, kz, w, cell, ncell, c, sh_heat, sh_real);
    tau = Ar<T>::dv(-Ar<T>::ln(Ar<T>::u01(w.x)), pick3(gam, v));
  }
}

// LDS histogram of one tile: the electron deposit packed two subcells per
// word (16-bit halves; a tile holds at most kMaxTile slots, so a half never
// carries), then the four heat counters per subcell, the per-mechanism
// counters of the upper valleys (32 words), the event counters (8) and the
// refill queue head (1).  Packing the deposit keeps the histogram under
// 32 KB, so five 256-lane workgroups fit one CU.
constexpr int kMaxTile = 65535;
__host__ __device__ constexpr int dep_words(int ncell) { return (ncell + 1) / 2; }
__host__ __device__ constexpr int flight_lds_words(int ncell) { return dep_words(ncell) + 4 * ncell + 41; }
__device__ __forceinline__ void dep_add(uint32_t* dep, int cell) {
  atomicAdd(dep + (cell >> 1), 1u << (16 * (cell & 1)));
}
__device__ __forceinline__ uint32_t dep_get(const uint32_t* dep, int cell) {
  return (dep[cell >> 1] >> (16 * (cell & 1))) & 0xffffu;
}

template <typename T, bool DEV>
__global__ void __launch_bounds__(512) k_flight(FlightArgs<T> a) {
  extern __shared__ uint32_t sh[];
  const int ncell = DEV ? a.G.ncell : 1;
  uint32_t* sh_dep = sh;
  uint32_t* sh_heat = sh + dep_words(ncell);
  uint32_t* sh_real = sh_heat + 4 * ncell;
  uint32_t* sh_misc = sh_real + 32;
  const int nsh = flight_lds_words(ncell);
  for (int i = threadIdx.x; i < nsh; i += blockDim.x) sh[i] = 0u;
  __syncthreads();
  const TileDesc td = a.tiles[blockIdx.x];
  const InstParams P = a.ip[td.inst];
  const T* fac = a.fac + (size_t)td.inst * ncell * kFRow;
  const T* field = a.field + (size_t)td.inst * ncell * 4;
  const T* gp = a.gamma + td.inst * 4;
  const T gam[3] = {gp[0], gp[1], gp[2]};  // workgroup-uniform
  const uint32_t n_int = a.ctl[CTL_INTERVAL];
  Cnt c = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  bool guard_hit = false, nan_hit = false;
  for (int i = threadIdx.x; i < td.count; i += blockDim.x) {
    const long long p = td.start + i;
    const uint32_t meta = a.meta[p];
    if (!(meta & kAlive)) { c.dead++; continue; }
    c.proc++;
    T kx = a.kx[p], ky = a.ky[p], kz = a.kz[p];
    T x = (T)0, y = (T)0, z = (T)0;
    if (DEV) { x = a.x[p]; y = a.y[p]; z = a.z[p]; }
    int v = meta_valley(meta);
    const uint32_t id = meta_id(meta);
    const bool alive = fly<T, DEV>(a, P, fac, field, gam, n_int, ncell, v, id, kx, ky, kz, x, y, z, c, sh_heat,
                                   sh_real, guard_hit);
    if (!(isfinite(kx) && isfinite(ky) && isfinite(kz))) nan_hit = true;
    a.kx[p] = kx; a.ky[p] = ky; a.kz[p] = kz;
    if (DEV) { a.x[p] = x; a.y[p] = y; a.z[p] = z; }
    a.meta[p] = (id << 3) | (alive ? kAlive : 0u) | (uint32_t)v;
    if (!alive) c.dead++;
    else if (DEV) dep_add(sh_dep, cell_of(a.G, x, y, z));
  }
  if (guard_hit) set_flag(a.flags, td.inst, -4);
  if (nan_hit) set_flag(a.flags, td.inst, -6);
  {
    const uint32_t vals[8] = {c.sel, c.self, c.ovf, c.ex0, c.ex1, c.refl, c.dead, c.proc};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint32_t s = wave_sum(vals[q]);
      if ((threadIdx.x & 63) == 0 && s) atomicAdd(sh_misc + q, s);
    }
  }
  __syncthreads();
  if (DEV) {
    unsigned long long* h = a.acc + (size_t)td.inst * 5 * ncell;
    for (int i = threadIdx.x; i < 5 * ncell; i += blockDim.x) {
      const uint32_t v = i < ncell ? dep_get(sh_dep, i) : sh_heat[i - ncell];
      if (v) atomicAdd(h + i, (unsigned long long)v);
    }
  }
  unsigned long long* cnt = a.counters + (size_t)td.inst * kNCnt;
  for (int tid = threadIdx.x; tid < 39; tid += blockDim.x) {
    if (tid < 30) {
      if (sh_real[tid]) atomicAdd(cnt + C_REAL + tid, (unsigned long long)sh_real[tid]);
    } else if (tid < 38) {
      const int q = tid - 30;
      const int slot = q == 0 ? C_SEL : q == 1 ? C_SELF : q == 2 ? C_OVF : q == 3 ? C_EXIT0
                     : q == 4 ? C_EXIT1 : q == 5 ? C_REFL : q == 6 ? -1 : C_PROC;
      if (slot >= 0 && sh_misc[q]) atomicAdd(cnt + slot, (unsigned long long)sh_misc[q]);
    } else {
      a.tile_dead[blockIdx.x] = sh_misc[6];
    }
  }
}

// Scattering with the electron's kinetic energy E already known (kept by the
// lane between drift and scatter instead of being recomputed from k).  Table,
// factor and field rows are read as 16-byte vectors.  Real events of valley
// Gamma1 are counted in the lane's registers (rc), the rare upper-valley
// events by LDS atomics.  Returns the mechanism (-1 self) and updates E.
template <typename T>
__device__ __forceinline__ int scatter_e(const FlightArgs<T>& a, const T* Sr, const T* f, const T (&gam)[3], int& v,
                                         T& kx, T& ky, T& kz, T& E, const uint4 w, int cell, int ncell, Cnt& c,
                                         uint32_t* sh_heat, uint32_t* sh_real, uint32_t* rc) {
  const Mat<T>& M = a.M;
  const T rs = Ar<T>::u01(w.y) * pick3(gam, v);
  // the selected mechanism is the first whose running sum exceeds rs; the
  // terms are rates times occupations, none negative, so the running sums
  // do not decrease and that index is the count of sums at or below rs
  // (kNM: none exceeds it, self-scattering)
  T cum = (T)0;
  int m = 0;
#pragma unroll
  for (int q = 0; q < kNM; ++q) {
    cum += tab_term<T>(Sr, f, q);
    m += cum <= rs ? 1 : 0;
  }
  c.sel++;
  if (m == kNM) { c.self++; return -1; }
  // final energy by selects (every lane computes the intervalley form)
  const int vp = m >= 4 ? (m - 4) >> 1 : v;
  const T Eiv = E + pick3(M.Ec, v) - pick3(M.Ec, vp) + (((m - 4) & 1) ? -M.hw_iv : M.hw_iv);
  const T Ep = m <= 1 ? E : (m == 2 ? E + M.hw_lo : (m == 3 ? E - M.hw_lo : Eiv));
  if (!(Ep > (T)0)) { c.self++; return -1; }
  if (v == 0) {
#pragma unroll
    for (int q = 0; q < kNM; ++q) rc[q] += (m == q) ? 1u : 0u;
  } else {
    atomicAdd(sh_real + v * kNM + m, 1u);
  }
  {
    // heat slot: 0 LO emission, 1 LO absorption, 2 intervalley emission,
    // 3 intervalley absorption; none for the elastic mechanisms
    const int hs = m == 3 ? 0 : (m == 2 ? 1 : (m >= 4 ? (((m - 4) & 1) ? 2 : 3) : -1));
    if (hs >= 0) atomicAdd(sh_heat + hs * ncell + cell, 1u);
  }
  const T k2 = ksq(kx, ky, kz);
  const T g = E * ((T)1 + pick3(M.alpha, v) * E);
  const T u2 = Ar<T>::u01(w.z), u3 = Ar<T>::u01(w.w);
  T X;
  if (m == 2 || m == 3) {
    const T gp = Ep * ((T)1 + pick3(M.alpha, v) * Ep);
    const T sg = Ar<T>::sq(g), sgp = Ar<T>::sq(gp);
    const T xi = Ar<T>::dv((T)2 * sg * sgp, (sg - sgp) * (sg - sgp));
    X = Ar<T>::dv(Ar<T>::em1(u2 * Ar<T>::l1p((T)2 * xi)), xi);
  } else {
    // Brooks-Herring; with a4 = 0 the same expression is the isotropic
    // X = 2 u2 exactly (a division by 1)
    const T a4 = m == 1 ? Ar<T>::dv((T)4 * k2, f[6]) : (T)0;
    X = Ar<T>::dv((T)2 * u2, (T)1 + ((T)1 - u2) * a4);
  }
  X = fmin(fmax(X, (T)0), (T)2);
  const T ct = (T)1 - X;
  const T st = Ar<T>::sq(X * ((T)2 - X));
  T cp, sp;
  Ar<T>::cs2pi(u3, cp, sp);
  const T kn = Ar<T>::sq(k2);
  T nx = (T)0, ny = (T)0, nz = (T)1;
  if (kn > (T)0) { nx = Ar<T>::dv(kx, kn); ny = Ar<T>::dv(ky, kn); nz = Ar<T>::dv(kz, kn); }
  T e1[3], e2[3];
  onb<T>(nx, ny, nz, e1, e2);
  const T gpp = Ep * ((T)1 + pick3(M.alpha, vp) * Ep);
  const T kp = Ar<T>::sq(Ar<T>::dv(gpp * pick3(M.m, vp), M.ck));
  const T sc = st * cp, ss = st * sp;
  kx = kp * dot3(sc, e1[0], ss, e2[0], ct, nx);
  ky = kp * dot3(sc, e1[1], ss, e2[1], ct, ny);
  kz = kp * dot3(sc, e1[2], ss, e2[2], ct, nz);
  v = vp;
  E = Ep;
  return m;
}

// Specular reflection at the walls 0 and L of one axis: the first reflection
// by selects, further ones (a flight longer than the width) in a rare loop,
// a position still outside after 8 reflections clamped and counted.
template <typename T>
__device__ __forceinline__ void reflect(T L, T& y, T& ky, Cnt& c) {
  const bool lo = y < (T)0, hi = y > L;
  y = lo ? -y : (hi ? (T)2 * L - y : y);
  ky = (lo || hi) ? -ky : ky;
  if (y < (T)0 || y > L) {
    int guard = 1;
    while ((y < (T)0 || y > L) && guard < 8) { y = y < (T)0 ? -y : (T)2 * L - y; ky = -ky; ++guard; }
    if (y < (T)0 || y > L) { y = y < (T)0 ? (T)0 : L; c.refl++; }
  }
}

// Free flight with the energy E of the initial k known; on return E is the
// energy of the final k (needed by the next scattering).
template <typename T, bool DEV>
__device__ __forceinline__ int drift_e(const FlightArgs<T>& a, int v, T dt, T fx, T fy, T fz, T& kx, T& ky, T& kz,
                                       T& x, T& y, T& z, T& E, Cnt& c) {
  const Mat<T>& M = a.M;
  const T k1x = kx - M.cf * fx * dt, k1y = ky - M.cf * fy * dt, k1z = kz - M.cf * fz * dt;
  const T E1 = energy(M, v, k1x, k1y, k1z);
  if (DEV) {
    const T s0 = vel_factor(M, v, E);
    const T s1 = vel_factor(M, v, E1);
    // the trapezoid written with explicit fused multiply-adds: left to the
    // compiler, which of the two products it fuses can differ between the
    // kernels that inline this, and with it the last bit of the position
    const T h = (T)0.5 * dt;
    x = fma(h, fma(s0, kx, s1 * k1x), x);
    y = fma(h, fma(s0, ky, s1 * k1y), y);
    z = fma(h, fma(s0, kz, s1 * k1z), z);
  }
  kx = k1x; ky = k1y; kz = k1z;
  E = E1;
  if (!DEV) return -1;
  if (x < (T)0) return 0;
  if (x > a.G.L[0]) return 1;
  reflect<T>(a.G.L[1], y, ky, c);
  reflect<T>(a.G.L[2], z, kz, c);
  return -1;
}

// A load of particle state, which a launch reads once.  When the state in
// use outgrows the Infinity Cache (nt), the loads are non-temporal: the
// state streaming through from HBM then does not push out the lines of
// state the lanes are writing back (partly written until all their slots'
// electrons have ended the interval).  While the state fits the cache,
// plain loads keep it there, and are faster.
template <typename T>
__device__ __forceinline__ T sload(const T* p, bool nt) { return nt ? __builtin_nontemporal_load(p) : *p; }

// Whether the state in use (the slots below every instance's bound)
// outgrows the Infinity Cache: wavefront-uniform, from the refill plan.
template <typename T>
__device__ __forceinline__ bool state_outgrows_cache(const FlightArgs<T>& a) {
  unsigned long long n = 0;
  for (int i = 0; i < a.n_inst; ++i) n += a.plan[i].hw;
  return n > a.nt_slots;
}

// The electron a lane is working on in the lane-refill kernels.
template <typename T>
struct LaneE {
  T kx, ky, kz, x, y, z, t, E;
  int v;
  uint32_t id, j;
  uint32_t meta0;  // the slot's meta word when the lane took the electron
  long long p;  // slot
};

// Load slot p (the state together with the meta word: one memory round trip
// per slot; a free slot's stale state is discarded).  Returns whether the
// slot holds a live electron, which then becomes the lane's electron.
template <typename T, bool DEV>
__device__ __forceinline__ bool take_slot(const FlightArgs<T>& a, long long p, LaneE<T>& L, Cnt& c, bool nt) {
  const uint32_t meta = sload(a.meta + p, nt);
  const T lkx = sload(a.kx + p, nt), lky = sload(a.ky + p, nt), lkz = sload(a.kz + p, nt);
  T lx = (T)0, ly = (T)0, lz = (T)0;
  if (DEV) { lx = sload(a.x + p, nt); ly = sload(a.y + p, nt); lz = sload(a.z + p, nt); }
  if (!(meta & kAlive)) { c.dead++; return false; }
  c.proc++;
  L.p = p;
  L.meta0 = meta;
  L.kx = lkx; L.ky = lky; L.kz = lkz;
  L.x = lx; L.y = ly; L.z = lz;
  L.v = meta_valley(meta);
  L.id = meta_id(meta);
  L.j = 0;
  L.t = (T)0;
  L.E = energy(a.M, L.v, L.kx, L.ky, L.kz);
  return true;
}

// A slot's state loaded ahead of its use: the lane issues the loads when it
// claims the slot and takes the electron over (adopt) once its current one
// has ended, a segment later, so that the state's memory latency is covered
// by that segment's work instead of stalling the wavefront at the refill.
template <typename T>
struct Prefetch {
  uint32_t idx;  // slot within the tile
  uint32_t meta;
  T kx, ky, kz, x, y, z;
};

template <typename T, bool DEV>
__device__ __forceinline__ void prefetch_slot(const FlightArgs<T>& a, long long start, uint32_t idx, Prefetch<T>& F,
                                              bool nt) {
  const long long p = start + idx;
  F.idx = idx;
  F.meta = sload(a.meta + p, nt);
  F.kx = sload(a.kx + p, nt); F.ky = sload(a.ky + p, nt); F.kz = sload(a.kz + p, nt);
  F.x = (T)0; F.y = (T)0; F.z = (T)0;
  if (DEV) { F.x = sload(a.x + p, nt); F.y = sload(a.y + p, nt); F.z = sload(a.z + p, nt); }
}

// The prefetched slot becomes the lane's electron if it holds a live one
// (a free slot is counted and dropped), exactly as take_slot would load it.
template <typename T>
__device__ __forceinline__ bool adopt_slot(const FlightArgs<T>& a, long long start, const Prefetch<T>& F, LaneE<T>& L,
                                           Cnt& c) {
  if (!(F.meta & kAlive)) { c.dead++; return false; }
  c.proc++;
  L.p = start + F.idx;
  L.meta0 = F.meta;
  L.kx = F.kx; L.ky = F.ky; L.kz = F.kz;
  L.x = F.x; L.y = F.y; L.z = F.z;
  L.v = meta_valley(F.meta);
  L.id = meta_id(F.meta);
  L.j = 0;
  L.t = (T)0;
  L.E = energy(a.M, L.v, L.kx, L.ky, L.kz);
  return true;
}

// One segment of the lane's electron: the scattering event that ends the
// previous flight (none at the start of the interval, j = 0), then the flight
// to the next selection or to the end of the interval.  The rate-table row
// (pre-event valley and energy bin), the cell's factor row and its field are
// issued before the random numbers, whose arithmetic then covers their
// latency (the position does not change in an event, so the field row serves
// the flight after it).  Returns -2 while the interval goes on, -1 at its end
// (or at the event guard), 0 or 1 when the electron left through the source
// or drain contact.
template <typename T, bool DEV>
__device__ __forceinline__ int lane_segment(const FlightArgs<T>& a, const InstParams& P, const T* fac,
                                            const T* field, const T (&gam)[3], uint32_t n_int, int ncell,
                                            LaneE<T>& L, Cnt& c, uint32_t* sh_heat, uint32_t* sh_real, uint32_t* rc,
                                            bool& guard_hit) {
  const int cell = DEV ? cell_of(a.G, L.x, L.y, L.z) : 0;
  const T eb = Ar<T>::dv(L.E, a.dE);
  const bool ovf = !(eb < (T)a.nb);
  const int bin = (int)fmin(eb, (T)(a.nb - 1));  // NaN -> last bin
  T Sr[kTRow], f[kFRow], F[4];
  load_row<kTRow>(a.table + (uint32_t)((L.v * a.nb + bin) * kTRow), Sr);
  load_row<kFRow>(fac + kFRow * cell, f);
  load_row<4>(field + 4 * cell, F);
  __builtin_amdgcn_sched_barrier(0);  // keep the loads above the generator
  const uint4 w = philox(L.id, n_int, L.j, P.tagw, P.key0, P.key1);
  if (L.j > 0) {
    if (ovf) c.ovf++;
    scatter_e<T>(a, Sr, f, gam, L.v, L.kx, L.ky, L.kz, L.E, w, cell, ncell, c, sh_heat, sh_real, rc);
  }
  const T tau = Ar<T>::dv(-Ar<T>::ln(Ar<T>::u01(w.x)), pick3(gam, L.v));
  const bool last = L.t + tau >= a.TP;
  const int ex = drift_e<T, DEV>(a, L.v, last ? a.TP - L.t : tau, F[0], F[1], F[2], L.kx, L.ky, L.kz, L.x, L.y,
                                 L.z, L.E, c);
  if (ex >= 0) return ex;
  if (last) return -1;
  L.t += tau;
  ++L.j;
  if (L.j > (uint32_t)kMaxEvents) { guard_hit = true; return -1; }
  return -2;
}

// Write the lane's electron back at the end of its interval (ex as returned
// by lane_segment) and deposit it in its subcell if it is still inside.
template <typename T, bool DEV>
__device__ __forceinline__ void retire(const FlightArgs<T>& a, const LaneE<T>& L, int ex, Cnt& c, uint32_t* sh_dep,
                                       bool packed_dep, bool& nan_hit) {
  const bool alive = ex < 0;
  c.ex0 += (uint32_t)(ex == 0);  // as adds: a pair of guarded increments is merged into an indexed one in scratch
  c.ex1 += (uint32_t)(ex == 1);
  if (!(isfinite(L.kx) && isfinite(L.ky) && isfinite(L.kz))) nan_hit = true;
  const long long p = L.p;
  a.kx[p] = L.kx; a.ky[p] = L.ky; a.kz[p] = L.kz;
  if (DEV) { a.x[p] = L.x; a.y[p] = L.y; a.z[p] = L.z; }
  // the meta word changes only with the valley or at an exit: most
  // electrons leave it as it is, which spares one of the seven scattered
  // partial-line writes
  const uint32_t meta = (L.id << 3) | (alive ? kAlive : 0u) | (uint32_t)L.v;
  if (meta != L.meta0) a.meta[p] = meta;
  if (!alive) c.dead++;
  else if (DEV) {
    const int cell = cell_of(a.G, L.x, L.y, L.z);
    if (packed_dep) dep_add(sh_dep, cell);
    else atomicAdd(sh_dep + cell, 1u);
  }
}

// Workgroup end of the lane-refill kernels: per-lane counters summed into LDS,
// then the nonzero bins of the workgroup's histogram (deposit unpacked when
// packed) added to the instance's sums by 64-bit atomics, exact in any order,
// and the event counters added to the instance's totals.
template <bool DEV>
__device__ __forceinline__ void flush_workgroup(const Cnt& c, const uint32_t* rc, uint32_t* sh_dep, bool packed_dep,
                                                uint32_t* sh_heat, uint32_t* sh_real, uint32_t* sh_misc, int ncell,
                                                unsigned long long* hist, unsigned long long* cnt,
                                                uint32_t* tile_dead_out) {
  const int lane = threadIdx.x & 63;
  const uint32_t vals[8] = {c.sel, c.self, c.ovf, c.ex0, c.ex1, c.refl, c.dead, c.proc};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t s = wave_sum(vals[q]);
    if (lane == 0 && s) atomicAdd(sh_misc + q, s);
  }
#pragma unroll
  for (int q = 0; q < kNM; ++q) {
    const uint32_t s = wave_sum(rc[q]);
    if (lane == 0 && s) atomicAdd(sh_real + q, s);
  }
  __syncthreads();
  if (DEV && hist) {
    for (int i = threadIdx.x; i < 5 * ncell; i += blockDim.x) {
      const uint32_t v = i < ncell ? (packed_dep ? dep_get(sh_dep, i) : sh_dep[i]) : sh_heat[i - ncell];
      if (v) atomicAdd(hist + i, (unsigned long long)v);
    }
  }
  for (int tid = threadIdx.x; tid < 39; tid += blockDim.x) {
    if (tid < 30) {
      if (sh_real[tid]) atomicAdd(cnt + C_REAL + tid, (unsigned long long)sh_real[tid]);
    } else if (tid < 38) {
      const int q = tid - 30;
      const int slot = q == 0 ? C_SEL : q == 1 ? C_SELF : q == 2 ? C_OVF : q == 3 ? C_EXIT0
                     : q == 4 ? C_EXIT1 : q == 5 ? C_REFL : q == 6 ? -1 : C_PROC;
      if (slot >= 0 && sh_misc[q]) atomicAdd(cnt + slot, (unsigned long long)sh_misc[q]);
    } else if (tile_dead_out) {
      *tile_dead_out = sh_misc[6];
    }
  }
}

// Lane-refill variant: each lane works one segment per iteration (the start
// of an electron's interval, or one scattering event plus the next flight)
// and pulls the next electron of the tile from a workgroup queue as soon as
// its electron reaches the end of the interval, so lanes do not idle while
// the busiest lane of the wavefront finishes its events.  Each lane keeps
// the next slot it claimed from the queue prefetched (Prefetch), so that a
// refill rarely waits for the state's loads.  Per-electron arithmetic and
// random-number use are the same as in k_flight, and the order in which
// lanes take electrons changes no result (every electron has its own
// random-number stream; the histograms are sums of counts).
// Workgroups of up to 1024 lanes for FP32 state; FP64 state needs more than
// the 128 registers a 1024-lane workgroup leaves each lane, so 512 at most.
template <typename T>
__host__ __device__ constexpr int max_flight_block() { return sizeof(T) == 4 ? 1024 : 512; }

template <typename T, bool DEV>
__global__ void __launch_bounds__(max_flight_block<T>()) k_flight_refill(FlightArgs<T> a) {
  extern __shared__ uint32_t sh[];
  const int ncell = DEV ? a.G.ncell : 1;
  uint32_t* sh_dep = sh;
  uint32_t* sh_heat = sh + dep_words(ncell);
  uint32_t* sh_real = sh_heat + 4 * ncell;
  uint32_t* sh_misc = sh_real + 32;
  uint32_t* sh_q = sh_misc + 8;
  const int nsh = flight_lds_words(ncell);
  for (int i = threadIdx.x; i < nsh; i += blockDim.x) sh[i] = 0u;
  __syncthreads();
  const TileDesc td = a.tiles[blockIdx.x];
  const InstParams P = a.ip[td.inst];
  const T* fac = a.fac + (size_t)td.inst * ncell * kFRow;
  const T* field = a.field + (size_t)td.inst * ncell * 4;
  const T* gp = a.gamma + td.inst * 4;
  const T gam[3] = {gp[0], gp[1], gp[2]};  // workgroup-uniform
  const uint32_t n_int = a.ctl[CTL_INTERVAL];
  // slots of the tile below the instance's bound of slots in use; those
  // above it are free and only counted
  uint32_t lim = (uint32_t)td.count;
  if (DEV) {
    const uint32_t hw = a.plan[td.inst].hw, rel = (uint32_t)(td.start - P.base);
    lim = hw > rel ? min(lim, hw - rel) : 0u;
  }
  const bool nt = DEV && state_outgrows_cache(a);
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = (1ull << lane) - 1ull;
  Cnt c = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  if (threadIdx.x == 0) c.dead = (uint32_t)td.count - lim;
  bool guard_hit = false, nan_hit = false;
  bool has = false, exhausted = false, pf = false;
  LaneE<T> L = {};
  Prefetch<T> F = {};
  uint32_t rc[kNM];
#pragma unroll
  for (int q = 0; q < kNM; ++q) rc[q] = 0u;
  for (;;) {
    // refill: a lane without an electron adopts the slot it prefetched (a
    // free slot leaves it idle for this iteration); a lane without a
    // prefetched slot claims the next index of the tile's queue and issues
    // its loads, to be adopted in a later iteration.  The lane's electron is
    // written only here and in the segment, outside any inner loop, which
    // keeps the compiler from copying its state around the refill.
    if (!has && pf) {
      has = adopt_slot<T>(a, td.start, F, L, c);
      pf = false;
    }
    {
      const bool want = !pf && !exhausted;
      const unsigned long long m = __ballot(want);
      if (m) {
        const int first = __ffsll((long long)m) - 1;
        uint32_t base = 0;
        if (lane == first) base = atomicAdd(sh_q, (uint32_t)__popcll(m));
        base = __shfl(base, first);
        if (want) {
          const uint32_t idx = base + (uint32_t)__popcll(m & lt);
          if (idx < lim) {
            prefetch_slot<T, DEV>(a, td.start, idx, F, nt);
            pf = true;
          } else {
            exhausted = true;
          }
        }
      }
    }
    if (!__any(has || pf)) break;
    // Every lane runs the segment, so that the lane's electron is updated in
    // code without a branch around it.  A lane without an electron runs it on
    // its stale state (an electron it finished, or the zero state: its
    // subcell and energy bin are in range) with the event counter held at
    // zero, so that it selects no event and counts nothing, and its outcome
    // is dropped.
    if (!has) L.j = 0;
    const uint32_t refl0 = c.refl;
    const int r = lane_segment<T, DEV>(a, P, fac, field, gam, n_int, ncell, L, c, sh_heat, sh_real, rc, guard_hit);
    if (!has) c.refl = refl0;
    if (has && r > -2) {
      retire<T, DEV>(a, L, r, c, sh_dep, true, nan_hit);
      has = false;
    }
  }
  if (guard_hit) set_flag(a.flags, td.inst, -4);
  if (nan_hit) set_flag(a.flags, td.inst, -6);
  // a tile wholly above the bound holds no electron and adds nothing
  flush_workgroup<DEV>(c, rc, sh_dep, true, sh_heat, sh_real, sh_misc, ncell,
                       lim > 0 ? a.acc + (size_t)td.inst * 5 * ncell : nullptr,
                       a.counters + (size_t)td.inst * kNCnt, a.tile_dead + blockIdx.x);
}

// Persistent variant: as many workgroups as the GPU holds at once, each bound
// to one instance (a.wg_inst; w1 - w0 of them per instance, in proportion to
// its slots).  The instance's slots are cut into chunks of at most a.chunk
// consecutive slots that never straddle a tile; workgroup r of the instance
// owns chunks r, r + nw, r + 2 nw, ..., so every workgroup samples the whole
// slot range evenly and holds about the same number of live electrons however
// they are spread over the slots (the contact refill fills the lowest free
// slots, so live electrons gather at the front).  Its wavefronts take the
// workgroup's chunks one at a time from an LDS counter and refill their lanes
// from the current chunk.  No global queue: nothing to reset between
// launches.  One LDS histogram per workgroup, as in k_flight_refill (the host
// gives every instance enough workgroups that none owns more than kMaxTile
// slots, so the packed deposit cannot carry).  The part of a chunk at or above
// the bound of slots in use is counted free without being read.  Free slots are added to the tile's
// count by atomics, once per chunk and once per electron that leaves (the
// refill plan clears the counts after reading them).  Per-electron arithmetic
// and random-number use are those of k_flight_refill.
template <typename T, bool DEV>
__global__ void __launch_bounds__(max_flight_block<T>()) k_flight_persist(FlightArgs<T> a) {
  extern __shared__ uint32_t sh[];
  const int ncell = DEV ? a.G.ncell : 1;
  uint32_t* sh_dep = sh;
  uint32_t* sh_heat = sh + dep_words(ncell);
  uint32_t* sh_real = sh_heat + 4 * ncell;
  uint32_t* sh_misc = sh_real + 32;
  uint32_t* sh_claim = sh_misc + 8;
  const int nsh = flight_lds_words(ncell);
  for (int i = threadIdx.x; i < nsh; i += blockDim.x) sh[i] = 0u;
  __syncthreads();
  const int inst = a.wg_inst[blockIdx.x];
  const InstParams P = a.ip[inst];
  const T* fac = a.fac + (size_t)inst * ncell * kFRow;
  const T* field = a.field + (size_t)inst * ncell * 4;
  const T* gp = a.gamma + inst * 4;
  const T gam[3] = {gp[0], gp[1], gp[2]};  // workgroup-uniform
  const uint32_t n_int = a.ctl[CTL_INTERVAL];
  const int r = (int)blockIdx.x - P.w0, nw = P.w1 - P.w0;
  const bool nt = DEV && state_outgrows_cache(a);
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = (1ull << lane) - 1ull;
  const int cpt = (a.tile + a.chunk - 1) / a.chunk;  // chunks per tile
  // slots at or above the instance's bound of slots in use are free: they
  // are counted, not read
  const int hw = DEV ? (int)min(a.plan[inst].hw, (uint32_t)P.cap) : P.cap;
  Cnt c = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  bool guard_hit = false, nan_hit = false;
  bool has = false;
  // wavefront-uniform: no chunks left, current chunk [cpos, cend) of tile
  // ctile, free slots met in it so far
  bool exhausted = false;
  int cpos = 0, cend = 0, ctile = 0;
  uint32_t dacc = 0;
  int ltile = 0;  // tile of the lane's electron
  LaneE<T> L = {};
  uint32_t rc[kNM];
#pragma unroll
  for (int q = 0; q < kNM; ++q) rc[q] = 0u;
  for (;;) {
    bool want = !has && !exhausted;
    unsigned long long m = __ballot(want);
    while (m) {
      if (cpos >= cend) {
        if (DEV && lane == 0 && dacc) atomicAdd(a.tile_dead + ctile, dacc);
        dacc = 0;
        uint32_t i = 0;
        if (lane == 0) i = atomicAdd(sh_claim, 1u);
        i = __builtin_amdgcn_readfirstlane(i);
        const uint32_t k = (uint32_t)r + i * (uint32_t)nw;  // < nchunk + nw: no wrap
        if (k >= (uint32_t)P.nchunk) { exhausted = true; break; }
        const int t = (int)(k / (uint32_t)cpt), sub = (int)(k % (uint32_t)cpt);
        cpos = t * a.tile + sub * a.chunk;
        cend = min(cpos + a.chunk, min((t + 1) * a.tile, P.cap));
        ctile = P.t0 + t;
        if (cend > hw) {
          if (DEV && lane == 0) atomicAdd(a.tile_dead + ctile, (uint32_t)(cend - max(cpos, hw)));
          cend = max(cpos, hw);
        }
      }
      const int n = __popcll(m);
      const int take = min(n, cend - cpos);
      const int rank = __popcll(m & lt);
      bool live = false;
      if (want && rank < take) {
        live = take_slot<T, DEV>(a, P.base + cpos + rank, L, c, nt);
        has = live;
        ltile = ctile;
      }
      if (DEV) dacc += (uint32_t)__popcll(__ballot(want && rank < take && !live));
      cpos += take;
      want = !has;
      m = __ballot(want);
    }
    if (!__any(has)) break;
    if (has) {
      const int rr = lane_segment<T, DEV>(a, P, fac, field, gam, n_int, ncell, L, c, sh_heat, sh_real, rc, guard_hit);
      if (rr > -2) {
        retire<T, DEV>(a, L, rr, c, sh_dep, true, nan_hit);
        if (DEV && rr >= 0) atomicAdd(a.tile_dead + ltile, 1u);
        has = false;
      }
    }
  }
  if (guard_hit) set_flag(a.flags, inst, -4);
  if (nan_hit) set_flag(a.flags, inst, -6);
  flush_workgroup<DEV>(c, rc, sh_dep, true, sh_heat, sh_real, sh_misc, ncell, a.acc + (size_t)inst * 5 * ncell,
                       a.counters + (size_t)inst * kNCnt, nullptr);
}


// Slot state staged in LDS (variant 3, k_flight_persist_staged): each
// wavefront keeps two pieces of kPiece consecutive slots of its chunks, the
// one its lanes take electrons from and the next, whose loads go straight
// from global memory into LDS (global_load_lds, four bytes per lane, no
// registers; non-temporal) while the current one is used.  A refill then
// reads LDS, and the state's memory latency is covered by the work on the
// current piece.  This pays off while the state in use outgrows the
// Infinity Cache and every refill of variant 2 waits on HBM; while the
// state fits, variant 2 is faster, so the variants are timed and chosen.
// Piece layout: kx, ky, kz, x, y, z (kPiece values of T each), then the
// meta words.
// 128 slots: half the piece switches of 64, 1.8% faster with the state
// beyond the Infinity Cache; two pieces per wavefront take 112 KB of LDS
// for 1024 FP32 lanes.
constexpr int kPiece = 128;
template <typename T>
__host__ __device__ constexpr int piece_bytes() { return kPiece * (6 * (int)sizeof(T) + 4); }
typedef __attribute__((address_space(3))) void flight_lds_t;
typedef __attribute__((address_space(1))) void flight_glb_t;

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima): the staged
// loads have landed in LDS
__device__ __forceinline__ void wait_staged() {
  __builtin_amdgcn_s_waitcnt((0x7 << 4) | (0xF << 8));
  asm volatile("" ::: "memory");  // no LDS read of the staged piece moves above the wait
}

// Issue the non-temporal copy of cnt (1..kPiece) elements of E bytes from
// src into dst (LDS, wavefront-uniform): pass k moves bytes
// [256 k, 256 k + 256), lane l the four at 256 k + 4 l.  Lanes past the
// piece's end read its last four bytes instead (in bounds) and write LDS
// bytes that are never read.
template <int E>
__device__ __forceinline__ void stage_array(const void* src, char* dst, int cnt, int lane) {
  static_assert(kPiece * E % 256 == 0, "a piece's array is whole passes of 64 lanes x 4 bytes");
  const int last = cnt * E - 4;
#pragma unroll
  for (int k = 0; k < kPiece * E / 256; ++k) {
    const int b = min(256 * k + 4 * lane, last);
    __builtin_amdgcn_global_load_lds((flight_glb_t*)((const char*)src + b), (flight_lds_t*)(dst + 256 * k), 4, 0,
                                     2);
  }
}

template <typename T, bool DEV>
__device__ __forceinline__ void stage_piece(const FlightArgs<T>& a, long long first, int cnt, char* buf, int lane) {
  constexpr int A = kPiece * (int)sizeof(T);
  stage_array<sizeof(T)>(a.kx + first, buf, cnt, lane);
  stage_array<sizeof(T)>(a.ky + first, buf + A, cnt, lane);
  stage_array<sizeof(T)>(a.kz + first, buf + 2 * A, cnt, lane);
  if (DEV) {
    stage_array<sizeof(T)>(a.x + first, buf + 3 * A, cnt, lane);
    stage_array<sizeof(T)>(a.y + first, buf + 4 * A, cnt, lane);
    stage_array<sizeof(T)>(a.z + first, buf + 5 * A, cnt, lane);
  }
  stage_array<4>(a.meta + first, buf + 6 * A, cnt, lane);
}

// Slot i of a staged piece becomes the lane's electron if it holds a live
// one (a free slot is counted and dropped), as take_slot would load it.
template <typename T, bool DEV>
__device__ __forceinline__ bool take_staged(const FlightArgs<T>& a, const char* buf, int i, long long p, LaneE<T>& L,
                                            Cnt& c) {
  constexpr int A = kPiece * (int)sizeof(T);
  const uint32_t meta = ((const uint32_t*)(buf + 6 * A))[i];
  if (!(meta & kAlive)) { c.dead++; return false; }
  c.proc++;
  const T* v = (const T*)buf;
  L.p = p;
  L.meta0 = meta;
  L.kx = v[i]; L.ky = v[kPiece + i]; L.kz = v[2 * kPiece + i];
  L.x = (T)0; L.y = (T)0; L.z = (T)0;
  if (DEV) { L.x = v[3 * kPiece + i]; L.y = v[4 * kPiece + i]; L.z = v[5 * kPiece + i]; }
  L.v = meta_valley(meta);
  L.id = meta_id(meta);
  L.j = 0;
  L.t = (T)0;
  L.E = energy(a.M, L.v, L.kx, L.ky, L.kz);
  return true;
}

// Persistent variant with staged slots (variant 3): the workgroups, chunks
// and counting of k_flight_persist; its wavefronts cut each chunk into
// pieces of kPiece slots and stage them one ahead.  Per-electron arithmetic
// and random-number use are those of k_flight_refill.
template <typename T, bool DEV>
__global__ void __launch_bounds__(max_flight_block<T>()) k_flight_persist_staged(FlightArgs<T> a) {
  extern __shared__ uint32_t sh[];
  const int ncell = DEV ? a.G.ncell : 1;
  uint32_t* sh_dep = sh;
  uint32_t* sh_heat = sh + dep_words(ncell);
  uint32_t* sh_real = sh_heat + 4 * ncell;
  uint32_t* sh_misc = sh_real + 32;
  uint32_t* sh_claim = sh_misc + 8;
  const int nsh = flight_lds_words(ncell);
  for (int i = threadIdx.x; i < nsh; i += blockDim.x) sh[i] = 0u;
  __syncthreads();
  const int inst = a.wg_inst[blockIdx.x];
  const InstParams P = a.ip[inst];
  const T* fac = a.fac + (size_t)inst * ncell * kFRow;
  const T* field = a.field + (size_t)inst * ncell * 4;
  const T* gp = a.gamma + inst * 4;
  const T gam[3] = {gp[0], gp[1], gp[2]};  // workgroup-uniform
  const uint32_t n_int = a.ctl[CTL_INTERVAL];
  const int r = (int)blockIdx.x - P.w0, nw = P.w1 - P.w0;
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = (1ull << lane) - 1ull;
  const int cpt = (a.tile + a.chunk - 1) / a.chunk;  // chunks per tile
  // slots at or above the instance's bound of slots in use are free: they
  // are counted, not read
  const int hw = DEV ? (int)min(a.plan[inst].hw, (uint32_t)P.cap) : P.cap;
  Cnt c = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  bool guard_hit = false, nan_hit = false;
  bool has = false;
  // this wavefront's two staging buffers, after the histogram
  char* stage = (char*)(sh + nsh) + (size_t)(threadIdx.x >> 6) * 2 * piece_bytes<T>();
  // wavefront-uniform: no chunks left; the chunk being cut into pieces,
  // [cpos, cend) of tile ctile; the current piece [ppos, pend) in buffer b,
  // taken up to pcur, of tile ptile; the next piece [npos, nend) of tile
  // ntile in flight into buffer b ^ 1 (nvalid); free slots met in the
  // current piece's tile so far
  bool exhausted = false;
  int cpos = 0, cend = 0, ctile = 0;
  int b = 0, ppos = 0, pend = 0, pcur = 0, ptile = 0;
  bool nvalid = false;
  int npos = 0, nend = 0, ntile = 0;
  uint32_t dacc = 0;
  int ltile = 0;  // tile of the lane's electron
  LaneE<T> L = {};
  uint32_t rc[kNM];
#pragma unroll
  for (int q = 0; q < kNM; ++q) rc[q] = 0u;
  // the next piece of the wavefront's chunks (claiming chunks as they run
  // out), its loads issued into buffer b ^ 1
  auto stage_next = [&]() {
    nvalid = false;
    while (cpos >= cend) {
      uint32_t i = 0;
      if (lane == 0) i = atomicAdd(sh_claim, 1u);
      i = __builtin_amdgcn_readfirstlane(i);
      const uint32_t k = (uint32_t)r + i * (uint32_t)nw;  // < nchunk + nw: no wrap
      if (k >= (uint32_t)P.nchunk) return;
      const int t = (int)(k / (uint32_t)cpt), sub = (int)(k % (uint32_t)cpt);
      cpos = t * a.tile + sub * a.chunk;
      cend = min(cpos + a.chunk, min((t + 1) * a.tile, P.cap));
      ctile = P.t0 + t;
      if (cend > hw) {
        if (DEV && lane == 0) atomicAdd(a.tile_dead + ctile, (uint32_t)(cend - max(cpos, hw)));
        cend = max(cpos, hw);
      }
    }
    npos = cpos;
    nend = min(cpos + kPiece, cend);
    ntile = ctile;
    cpos = nend;
    stage_piece<T, DEV>(a, P.base + npos, nend - npos, stage + (b ^ 1) * piece_bytes<T>(), lane);
    nvalid = true;
  };
  stage_next();
  for (;;) {
    bool want = !has && !exhausted;
    unsigned long long m = __ballot(want);
    while (m) {
      if (pcur >= pend) {
        // the current piece is used up: move to the staged one and stage
        // the piece after it
        if (!nvalid) { exhausted = true; break; }
        wait_staged();
        if (DEV && ptile != ntile) {
          if (lane == 0 && dacc) atomicAdd(a.tile_dead + ptile, dacc);
          dacc = 0;
        }
        b ^= 1;
        ppos = npos; pend = nend; pcur = npos; ptile = ntile;
        stage_next();
      }
      const int n = __popcll(m);
      const int take = min(n, pend - pcur);
      const int rank = __popcll(m & lt);
      bool live = false;
      if (want && rank < take) {
        live = take_staged<T, DEV>(a, stage + b * piece_bytes<T>(), pcur + rank - ppos, P.base + pcur + rank, L, c);
        has = live;
        ltile = ptile;
      }
      if (DEV) dacc += (uint32_t)__popcll(__ballot(want && rank < take && !live));
      pcur += take;
      want = !has;
      m = __ballot(want);
    }
    if (!__any(has)) break;
    if (has) {
      const int rr = lane_segment<T, DEV>(a, P, fac, field, gam, n_int, ncell, L, c, sh_heat, sh_real, rc, guard_hit);
      if (rr > -2) {
        retire<T, DEV>(a, L, rr, c, sh_dep, true, nan_hit);
        if (DEV && rr >= 0) atomicAdd(a.tile_dead + ltile, 1u);
        has = false;
      }
    }
  }
  if (DEV && lane == 0 && dacc) atomicAdd(a.tile_dead + ptile, dacc);
  if (guard_hit) set_flag(a.flags, inst, -4);
  if (nan_hit) set_flag(a.flags, inst, -6);
  flush_workgroup<DEV>(c, rc, sh_dep, true, sh_heat, sh_real, sh_misc, ncell, a.acc + (size_t)inst * 5 * ncell,
                       a.counters + (size_t)inst * kNCnt, nullptr);
}

}  // namespace gfmc
