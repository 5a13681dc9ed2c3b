// phonon.hip -- the phonon side of the hybrid method on gfx950: bin tables
// of the sine-dispersion acoustic branches with their relaxation times
// (phonon paragraph, Table II) and the scattering by free electrons of
// Eq. (1); the diffuse-mismatch transmissivity of Eq. (2) and the interface
// resistance of Eq. (3); and the steady-state phonon packet Monte Carlo of
// the wire domain (phonon and coupling paragraphs).  C ABI in
// include/gfph.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "../../include/gfph.h"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kHbar = 1.054571817e-34;
constexpr double kKb = 1.380649e-23;
constexpr double kQe = 1.602176634e-19;
constexpr double kM0 = 9.1093837015e-31;

// ---------------------------------------------------------------------------
// Bin tables
// ---------------------------------------------------------------------------

// Group velocity (m/s) and density of states per branch and volume of the
// sine dispersion omega = w_max sin(pi q / 2 q0) at omega.
__device__ inline void sine_branch(const ph_material& m, double w, double& q, double& vg, double& dos) {
  const double s = fmin(w / m.w_max, 1.0);
  q = 2.0 * m.q0 / kPi * asin(s);
  vg = kPi / (2.0 * m.q0) * m.w_max * sqrt(fmax(0.0, (1.0 - s) * (1.0 + s)));
  dos = q * q / (2.0 * kPi * kPi * vg);
}

// d f_BE / dT = x / (T 4 sinh^2(x / 2)), x = hbar omega / k_B T
__device__ inline double bose_dT(double w, double T) {
  const double x = kHbar * w / (kKb * T);
  const double sh = sinh(0.5 * x);
  return x / (T * 4.0 * sh * sh);
}

// ln(1 + e^y) without overflow
__device__ inline double softplus(double y) { return y > 0.0 ? y + log1p(exp(-y)) : log1p(exp(y)); }

// Eq. (1): the braces rewritten as softplus(c - x) - softplus(-c - x), which
// equals hbar omega / k_B T - ln((1 + e^(x + c)) / (1 + e^(x - c))) with
// c = hbar omega / 2 k_B T and x the electron-energy offset of the equation.
__device__ inline double inv_tau_e(double w, double T, double EF_eV, const ph_electrons& e) {
  const double m = e.m_dos * kM0, Da = e.D_a_eV * kQe, kT = kKb * T;
  const double half = 0.5 * m * e.v_g * e.v_g;
  const double pref = Da * Da * m * m * m * e.v_g / (4.0 * kPi * kHbar * kHbar * kHbar * kHbar * e.rho) * kT / half;
  const double x = (half - EF_eV * kQe) / kT + kHbar * kHbar * w * w / (8.0 * m * e.v_g * e.v_g * kT);
  const double c = kHbar * w / (2.0 * kT);
  return pref * (softplus(c - x) - softplus(-c - x));
}

// Fermi level of a parabolic band: n = N_c F_1/2(eta) with
// F_1/2(eta) = (2/sqrt(pi)) int_0^inf sqrt(e) / (1 + e^(e - eta)) de, written
// with e = t^2 as (4/sqrt(pi)) int_0^inf t^2 / (1 + e^(t^2 - eta)) dt and
// summed by the composite Simpson rule over t in [0, sqrt(max(eta,0) + 50)]
// (8192 intervals, spread over the workgroup's threads).  Bisection on eta.
constexpr int kFdThreads = 256;
__global__ void __launch_bounds__(kFdThreads) k_fermi_level(double n_m3, double m_dos, double T, double* out) {
  __shared__ double red[kFdThreads / 64];
  __shared__ double s_eta;
  const double Nc = 2.0 * pow(m_dos * kM0 * kKb * T / (2.0 * kPi * kHbar * kHbar), 1.5);
  const double ef0 = kHbar * kHbar * pow(3.0 * kPi * kPi * n_m3, 2.0 / 3.0) / (2.0 * m_dos * kM0) / (kKb * T);
  double lo = fmin(-60.0, log(n_m3 / Nc) - 10.0), hi = fmax(200.0, 2.0 * ef0 + 10.0);
  constexpr int kIntervals = 8192;
  for (int it = 0; it < 200 && hi - lo > 1e-13 * fmax(1.0, fabs(hi)); ++it) {
    const double eta = 0.5 * (lo + hi);
    const double top = sqrt(fmax(eta, 0.0) + 50.0), h = top / kIntervals;
    double acc = 0.0;
    for (int i = threadIdx.x; i <= kIntervals; i += kFdThreads) {
      const double t = i * h;
      const double f = t * t / (1.0 + exp(fmin(t * t - eta, 700.0)));
      const double wgt = (i == 0 || i == kIntervals) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
      acc += wgt * f;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < kFdThreads / 64; ++w) s += red[w];
      const double F = 4.0 / sqrt(kPi) * s * h / 3.0;
      s_eta = Nc * F > n_m3 ? 1.0 : -1.0;
    }
    __syncthreads();
    if (s_eta > 0.0) hi = eta;
    else lo = eta;
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = 0.5 * (lo + hi) * kKb * T / kQe;
}

// One thread per bin: omega, group velocity (m/s), heat capacity of the bin
// for the three branches (J/(m^3 K)) and relaxation rate (1/s), stored
// [4][n_bins].
__global__ void k_ph_tables(ph_material m, int use_e, ph_electrons e, const double* __restrict__ EF, double T, int nb,
                            double* out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double dw = m.w_max / nb, w = (b + 0.5) * dw;
  double q, vg, dos;
  sine_branch(m, w, q, vg, dos);
  double it = m.A * w * w * w * w + m.B1 * w * w * T * exp(-m.B2 / T);
  if (use_e) it += inv_tau_e(w, T, *EF, e);
  out[b] = w;
  out[nb + b] = vg;
  out[2 * nb + b] = 3.0 * kHbar * w * bose_dT(w, T) * dos * dw;
  out[3 * nb + b] = it;
}

// Eq. (2) on the bins of material 1 and the sums of Eq. (3) and of the bulk
// conductivity, one workgroup: tau_12 per bin (optional), then
// sum v_1 C_1 tau_12 / 4 and sum C_1 v_1^2 tau_1 / 3 in a fixed order.
__global__ void __launch_bounds__(256) k_ph_interface(ph_material m1, ph_material m2, const double* __restrict__ tab1,
                                                      int nb, double* tau12_out, double* sums) {
  __shared__ double red[2][4];
  double a = 0.0, k = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const double w = tab1[b];
    double q1, v1, d1, q2, v2, d2;
    sine_branch(m1, w, q1, v1, d1);
    double t12 = 0.0;
    if (w < m2.w_max) {
      sine_branch(m2, w, q2, v2, d2);
      // three identical branches on each side
      const double s1 = 3.0 * v1 * d1, s2 = 3.0 * v2 * d2;
      t12 = s2 / (s1 + s2);
    }
    if (tau12_out) tau12_out[b] = t12;
    const double vb = tab1[nb + b], Cb = tab1[2 * nb + b], itb = tab1[3 * nb + b];
    a += vb * Cb * t12;
    k += Cb * vb * vb / itb;
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    k += __shfl_xor(k, o);
  }
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = a; red[1][threadIdx.x >> 6] = k; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sk = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { sa += red[0][w]; sk += red[1][w]; }
    sums[0] = sa / 4.0;
    sums[1] = sk / 3.0;
  }
}

// ---------------------------------------------------------------------------
// Phonon packet Monte Carlo
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ double uo(uint32_t w) {
#pragma clang fp contract(off)
  return ((double)w + 0.5) * (1.0 / 4294967296.0);
}

// first i with u * cum[n-1] < cum[i]
__device__ __forceinline__ int draw_cum(const double* cum, int n, double u) {
#pragma clang fp contract(off)
  const double x = u * cum[n - 1];
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (x < cum[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

__device__ __forceinline__ void iso(double u1, double u2, double d[3]) {
#pragma clang fp contract(off)
  const double mu = 2.0 * u1 - 1.0, s = sqrt(fmax(0.0, 1.0 - mu * mu)), ph = 2.0 * kPi * u2;
  d[0] = s * cos(ph);
  d[1] = s * sin(ph);
  d[2] = mu;
}

enum { CT_SCAT = 0, CT_SPEC = 1, CT_DIFF = 2, CT_ABS0 = 3, CT_DROP = 9, CT_SEG = 10, CT_N = 11 };

struct PhArgs {
  double L[3], d[3];
  int n[3], face[6], ncell, nb, max_events;
  uint32_t k0, k1, tag;
  long long n_packets;
  const double* q;         // [ncell] source power per subcell, W (either sign)
  const double* cum_cell;  // [ncell] cumulative |power| in subcell order
  const double* tab;       // [4][nb] bin tables
  const double* cum_emit;  // [nb] cumulative C_b / tau_b in bin order
  double* t_cell;          // [ncell] packet time per subcell, fs (atomic sums)
  uint32_t* pk_scat;       // [n_packets] scatterings of each packet (may be null)
  unsigned long long* counts;  // [CT_N]
  unsigned long long* next;    // packet counter of the launch
};

// Set-up of a run: cumulative |source| and re-emission weights, the packet
// counter and the tallies cleared.  The running sums keep the reference's
// order (one thread, element by element: the draws compare against them bit
// for bit); workgroup 0 first stages each sequence's terms in LDS, so that
// the serial loop waits on LDS rather than on global memory.
constexpr int kPhSetupBlock = 256;
__global__ void __launch_bounds__(kPhSetupBlock) k_ph_setup(const double* __restrict__ q, int ncell,
                                                            const double* __restrict__ tab, int nb, double* cum_cell,
                                                            double* cum_emit, double* t_cell,
                                                            unsigned long long* counts, unsigned long long* next,
                                                            double* sums) {
#pragma clang fp contract(off)
  __shared__ double buf[4096];  // ncell and nb are at most 4096
  if (blockIdx.x == 0) {
    // |q| per subcell, summed in subcell order
    for (int i = threadIdx.x; i < ncell; i += blockDim.x) buf[i] = fabs(q[i]);
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0;
#pragma unroll 8
      for (int i = 0; i < ncell; ++i) { a += buf[i]; cum_cell[i] = a; }
      sums[0] = a;  // total |power|, W: each packet carries sums[0] / N
    }
    __syncthreads();
    // re-emission weights C_b / tau_b, summed in bin order
    for (int b = threadIdx.x; b < nb; b += blockDim.x) buf[b] = tab[2 * nb + b] * tab[3 * nb + b];
    __syncthreads();
    if (threadIdx.x == 0) {
      double e = 0.0;
#pragma unroll 8
      for (int b = 0; b < nb; ++b) { e += buf[b]; cum_emit[b] = e; }
    }
    __syncthreads();
    // the heat capacity, summed in bin order
    for (int b = threadIdx.x; b < nb; b += blockDim.x) buf[b] = tab[2 * nb + b];
    __syncthreads();
    if (threadIdx.x == 0) {
      double cv = 0.0;
#pragma unroll 8
      for (int b = 0; b < nb; ++b) cv += buf[b];
      sums[1] = cv;  // volumetric heat capacity, J/(m^3 K)
      for (int i = 0; i < CT_N; ++i) counts[i] = 0ull;
      *next = 0ull;
    }
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += gridDim.x * blockDim.x) t_cell[i] = 0.0;
}

template <typename T>
__device__ __forceinline__ T get3(const T (&v)[3], int i) {
  return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]);
}
template <typename T>
__device__ __forceinline__ void set3(T (&v)[3], int i, T x) {
  v[0] = i == 0 ? x : v[0];
  v[1] = i == 1 ? x : v[1];
  v[2] = i == 2 ? x : v[2];
}

// One packet per lane.  A lane moves its packet straight to the next subcell
// boundary, scattering point or face (a few operations: the common step);
// what costs more, a scattering (a new bin, direction and free path), a
// diffuse reflection (a cosine-law direction) or a new packet (claimed from
// the launch's counter, 256 indices per wavefront at a time, then emitted),
// the lane only marks as pending.  The wavefront runs those paths together,
// once pending and free lanes make up half of its active lanes or no lane can
// move, so that the generator, the logarithm, sine and cosine and the binary
// searches run with most lanes busy instead of for the few that need them at
// each step.  Each packet still goes through the same operations in the same
// order with the same random numbers; only the interleaving of packets
// changes.  The bin tables and re-emission weights sit in LDS; each
// workgroup keeps its packet times per subcell in LDS and adds them to the
// global sums at the end (FP64 atomic adds: the order of the sums varies at
// rounding level).
constexpr int kPhBlock = 256;
constexpr int kPhChunk = 256;  // packet indices a wavefront claims at a time
enum { PH_MOVE = 0, PH_EMIT = 1, PH_SCATTER = 2, PH_WALL = 3 };
// Four wavefronts per SIMD (128 registers, 52 bytes per lane spilled): the
// lanes' waits on the LDS tables and tallies overlap more, 10.96 -> 10.27 ms
// per launch on the half-wire workload against three wavefronts without
// spills.
__global__ void __launch_bounds__(kPhBlock, 4) k_ph_packets(PhArgs a) {
  // separate multiplies and adds, as the FP64 reference rounds them: the
  // packet's path (and which boundary or face it meets first) then follows
  // the reference's arithmetic
#pragma clang fp contract(off)
  extern __shared__ double shd[];
  double* s_v = shd;                 // nm/fs
  double* s_tau = s_v + a.nb;        // fs
  double* s_cum = s_tau + a.nb;
  double* s_t = s_cum + a.nb;        // [ncell]
  for (int b = threadIdx.x; b < a.nb; b += blockDim.x) {
    s_v[b] = a.tab[a.nb + b] * 1e-6;
    s_tau[b] = 1e15 / a.tab[3 * a.nb + b];
    s_cum[b] = a.cum_emit[b];
  }
  for (int i = threadIdx.x; i < a.ncell; i += blockDim.x) s_t[i] = 0.0;
  // absorptions per face in LDS (rare; a face-indexed register array would
  // live in scratch memory); the frequent counts in plain registers
  __shared__ unsigned long long s_abs[6];
  if (threadIdx.x < 6) s_abs[threadIdx.x] = 0ull;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int ny = a.n[1], nz = a.n[2];
  const int faces = a.face[0] | a.face[1] << 2 | a.face[2] << 4 | a.face[3] << 6 | a.face[4] << 8 | a.face[5] << 10;
  unsigned long long n_seg = 0, n_scat = 0, n_spec = 0, n_diff = 0, n_drop = 0;
  bool has = false;                  // the lane holds a packet (moving or pending)
  int pend = PH_MOVE;                // what the packet waits for
  long long pk = 0;
  double r[3] = {0, 0, 0}, dir[3] = {0, 0, 1}, left = 0.0;
  double sg = 1.0;  // the packet's sign: negative from a subcell that is a net sink
  int ic[3] = {0, 0, 0}, b = 0, fax = 0;
  bool fup = false;                  // the face a pending diffuse reflection is at
  uint32_t ev = 0, hits = 0;
  long long events = 0;
  // wavefront-uniform chunk [cpos, cend) of packet indices claimed from the
  // launch's counter kPhChunk at a time; exhausted once the counter passes
  // the last packet
  long long cpos = 0, cend = 0;
  bool exhausted = false;
  for (;;) {
    const bool free_lane = !has && !exhausted;
    const int n_wait = __popcll(__ballot(free_lane || (has && pend != PH_MOVE)));
    const int n_mov = __popcll(__ballot(has && pend == PH_MOVE));
    if (n_wait + n_mov == 0) break;
    if (n_mov == 0 || 2 * n_wait >= n_wait + n_mov) {
      // ---- the expensive paths, for every lane that waits ----
      // free lanes take the next indices of the wavefront's chunk
      unsigned long long want = __ballot(!has && !exhausted);
      while (want) {
        if (cpos >= cend) {
          const int first = __ffsll((long long)want) - 1;
          unsigned long long base = 0;
          if (lane == first) base = atomicAdd(a.next, (unsigned long long)kPhChunk);
          base = __shfl(base, first);
          if ((long long)base >= a.n_packets) {
            exhausted = true;
            break;
          }
          cpos = (long long)base;
          cend = cpos + kPhChunk < a.n_packets ? cpos + kPhChunk : a.n_packets;
        }
        const long long take = min((long long)__popcll(want), cend - cpos);
        const long long rank = __popcll(want & ((1ull << lane) - 1ull));
        if (((want >> lane) & 1ull) && rank < take) {
          pk = cpos + rank;
          has = true;
          pend = PH_EMIT;
        }
        cpos += take;
        want = __ballot(!has && !exhausted);
      }
      // emission, first draw: the subcell (by |q|) and the point in it
      if (has && pend == PH_EMIT) {
        const uint4 w = philox((uint32_t)pk, 0u, 0u, a.tag, a.k0, a.k1);
        const int cell = draw_cum(a.cum_cell, a.ncell, uo(w.x));
        sg = a.q[cell] < 0.0 ? -1.0 : 1.0;
        ic[0] = cell / (ny * nz); ic[1] = (cell / nz) % ny; ic[2] = cell % nz;
        r[0] = (ic[0] + uo(w.y)) * a.d[0];
        r[1] = (ic[1] + uo(w.z)) * a.d[1];
        r[2] = (ic[2] + uo(w.w)) * a.d[2];
        ev = 0; hits = 0; events = 0;
      }
      if (has && pend != PH_MOVE) {
        // one generator call for every waiting packet: the emission's second
        // draw (packet, 0, 1), the j-th scattering (packet, j, 0), the h-th
        // diffuse reflection after it (packet, j, 1 + h)
        const uint32_t sub = pend == PH_WALL ? 1u + hits : (pend == PH_EMIT ? 1u : 0u);
        const uint4 w = philox((uint32_t)pk, ev, sub, a.tag, a.k0, a.k1);
        if (pend == PH_WALL) {
          const double ct = sqrt(uo(w.x)), st = sqrt(fmax(0.0, 1.0 - ct * ct)), ph = 2.0 * kPi * uo(w.y);
          // cosine-law direction about the inward normal of axis fax; the two
          // tangential components on axes fax + 1 and fax + 2 (cyclic)
          const double dn = fup ? -ct : ct, t1 = st * cos(ph), t2 = st * sin(ph);
          dir[0] = fax == 0 ? dn : (fax == 1 ? t2 : t1);
          dir[1] = fax == 1 ? dn : (fax == 2 ? t2 : t1);
          dir[2] = fax == 2 ? dn : (fax == 0 ? t2 : t1);
        } else {
          // a new bin (by C_b / tau_b), an isotropic direction, a free path
          b = draw_cum(s_cum, a.nb, uo(w.x));
          iso(uo(w.y), uo(w.z), dir);
          left = -log(uo(w.w)) * s_tau[b] * s_v[b];
        }
        pend = PH_MOVE;
      }
      continue;
    }
    if (!has || pend != PH_MOVE) continue;
    // ---- the common step: to the nearest subcell boundary, or to the
    // scattering point ----
    double tmin = left;
    int ax = -1;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if (dir[q] > 0.0) {
        const double s = ((ic[q] + 1) * a.d[q] - r[q]) / dir[q];
        if (s < tmin) { tmin = s; ax = q; }
      } else if (dir[q] < 0.0) {
        const double s = (ic[q] * a.d[q] - r[q]) / dir[q];
        if (s < tmin) { tmin = s; ax = q; }
      }
    }
    if (tmin < 0.0) tmin = 0.0;
    ++n_seg;
    const int cc = (ic[0] * ny + ic[1]) * nz + ic[2];
    unsafeAtomicAdd(s_t + cc, sg * (tmin / s_v[b]));
#pragma unroll
    for (int q = 0; q < 3; ++q) r[q] += tmin * dir[q];
    left -= tmin;
    if (ax < 0) {
      if (++events > a.max_events) {
        ++n_drop;
        if (a.pk_scat) a.pk_scat[pk] = ev;
        has = false;
        continue;
      }
      ++ev;
      ++n_scat;
      hits = 0;
      pend = PH_SCATTER;
      continue;
    }
    // the boundary of axis ax (per lane): selects instead of indexing, so
    // the three-component state stays in registers
    const double dax = get3(dir, ax);
    const bool up = dax > 0.0;
    const int icx = get3(ic, ax);
    set3(r, ax, (icx + (up ? 1 : 0)) * get3(a.d, ax));
    const int nxt = icx + (up ? 1 : -1);
    if (nxt >= 0 && nxt < get3(a.n, ax)) { set3(ic, ax, nxt); continue; }
    const int f = 2 * ax + (up ? 1 : 0);
    const int kind = (faces >> (2 * f)) & 3;
    if (kind == PH_ISOTHERMAL) {
      atomicAdd(s_abs + f, 1ull);
      if (a.pk_scat) a.pk_scat[pk] = ev;
      has = false;
      continue;
    }
    if (++events > a.max_events) {
      ++n_drop;
      if (a.pk_scat) a.pk_scat[pk] = ev;
      has = false;
      continue;
    }
    if (kind == PH_SPECULAR) {
      ++n_spec;
      set3(dir, ax, -dax);
    } else {
      ++n_diff;
      ++hits;
      fax = ax;
      fup = up;
      pend = PH_WALL;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a.ncell; i += blockDim.x)
    if (s_t[i] != 0.0) unsafeAtomicAdd(a.t_cell + i, s_t[i]);
  const unsigned long long mine[5] = {n_seg, n_scat, n_spec, n_diff, n_drop};
  const int slot[5] = {CT_SEG, CT_SCAT, CT_SPEC, CT_DIFF, CT_DROP};
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    unsigned long long s = mine[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0 && s) atomicAdd(a.counts + slot[i], s);
  }
  if (threadIdx.x < 6 && s_abs[threadIdx.x]) atomicAdd(a.counts + CT_ABS0 + threadIdx.x, s_abs[threadIdx.x]);
}

// temperature rise per subcell: P t_c / (N C_v V_c)
__global__ void k_ph_dT(const double* __restrict__ t_cell, const double* __restrict__ sums, int ncell,
                        double n_packets, double vc_m3, double* dT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncell) dT[i] = sums[0] * t_cell[i] * 1e-15 / (n_packets * sums[1] * vc_m3);
}

// size-limited conductivity: one workgroup, bins in order per thread, then a
// fixed tree
__global__ void __launch_bounds__(256) k_ph_conductivity(const double* __restrict__ tab, int nb, double d_m,
                                                         double* out) {
  __shared__ double s[256];
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const double v = tab[nb + b], C = tab[2 * nb + b], it = tab[3 * nb + b];
    const double rate = d_m > 0.0 ? it + v / d_m : it;
    a += C * v * v / (3.0 * rate);
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

struct PhLayout {
  size_t cum_cell, cum_emit, counts, next, sums, total;
};

PhLayout ph_layout(const ph_mc_config* c) {
  PhLayout L;
  size_t off = 0;
  auto take = [&](size_t b) { const size_t o = off; off += (b + 255) & ~(size_t)255; return o; };
  const size_t nc = (size_t)c->n_cells[0] * c->n_cells[1] * c->n_cells[2];
  L.cum_cell = take(8 * nc);
  L.cum_emit = take(8 * (size_t)c->n_bins);
  L.counts = take(8 * CT_N);
  L.next = take(8);
  L.sums = take(8 * 4);
  L.total = off;
  return L;
}

bool ph_valid(const ph_mc_config* c) {
  if (!c || c->n_bins < 1 || c->n_bins > 4096 || c->n_packets < 1 || c->n_packets > (1ll << 32) ||
      c->max_events < 1)
    return false;
  long long nc = 1;
  for (int d = 0; d < 3; ++d) {
    if (c->n_cells[d] < 1 || !(c->L_nm[d] > 0.0)) return false;
    nc *= c->n_cells[d];
  }
  if (nc > 4096) return false;
  for (int f = 0; f < 6; ++f)
    if (c->face[f] < PH_SPECULAR || c->face[f] > PH_ISOTHERMAL) return false;
  return c->instance < (1u << 27);
}

}  // namespace

extern "C" {

int ph_fermi_level(double n_m3, double m_dos, double T_K, double* d_out, void* stream) {
  if (!(n_m3 > 0.0) || !(m_dos > 0.0) || !(T_K > 0.0) || !d_out) return PH_E_ARG;
  k_fermi_level<<<1, kFdThreads, 0, (hipStream_t)stream>>>(n_m3, m_dos, T_K, d_out);
  return hipGetLastError() == hipSuccess ? PH_OK : PH_E_HIP;
}

int ph_tables(const ph_material* m, const ph_electrons* e, double T_K, int n_bins, double* d_tables,
              double* d_fermi, void* stream) {
  if (!m || !(m->w_max > 0.0) || !(m->q0 > 0.0) || !(T_K > 0.0) || n_bins < 1 || n_bins > 4096 || !d_tables)
    return PH_E_ARG;
  if (e && e->n_m3 > 0.0 && (!d_fermi || !(e->m_dos > 0.0) || !(e->rho > 0.0) || !(e->v_g > 0.0)))
    return PH_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const bool use_e = e && e->n_m3 > 0.0;
  ph_electrons ee;
  std::memset(&ee, 0, sizeof(ee));
  if (use_e) {
    ee = *e;
    const int rc = ph_fermi_level(e->n_m3, e->m_dos, T_K, d_fermi, stream);
    if (rc != PH_OK) return rc;
  }
  k_ph_tables<<<(n_bins + 255) / 256, 256, 0, st>>>(*m, use_e ? 1 : 0, ee, use_e ? d_fermi : nullptr, T_K, n_bins,
                                                    d_tables);
  return hipGetLastError() == hipSuccess ? PH_OK : PH_E_HIP;
}

int ph_interface(const ph_material* m1, const ph_material* m2, const double* d_tables1, int n_bins, double* d_tau12,
                 double* d_sums, void* stream) {
  if (!m1 || !m2 || !d_tables1 || n_bins < 1 || n_bins > 4096 || !d_sums) return PH_E_ARG;
  k_ph_interface<<<1, 256, 0, (hipStream_t)stream>>>(*m1, *m2, d_tables1, n_bins, d_tau12, d_sums);
  return hipGetLastError() == hipSuccess ? PH_OK : PH_E_HIP;
}

int ph_conductivity(const double* d_tables, int n_bins, double d_m, double* d_kappa, void* stream) {
  if (!d_tables || !d_kappa || n_bins < 1 || n_bins > 4096 || !std::isfinite(d_m)) return PH_E_ARG;
  k_ph_conductivity<<<1, 256, 0, (hipStream_t)stream>>>(d_tables, n_bins, d_m, d_kappa);
  return hipGetLastError() == hipSuccess ? PH_OK : PH_E_HIP;
}

size_t ph_mc_workspace_bytes(const ph_mc_config* c) { return ph_valid(c) ? ph_layout(c).total : 0; }

int ph_mc_run(const ph_mc_config* c, const double* d_tables, const double* d_q_cell, double* d_t_cell, double* d_dT,
              uint32_t* d_packet_scatterings, uint64_t* h_counts, void* d_ws, size_t ws_bytes, void* stream) {
  if (!ph_valid(c) || !d_tables || !d_q_cell || !d_t_cell) return PH_E_ARG;
  const PhLayout L = ph_layout(c);
  if (!d_ws || ws_bytes < L.total || ((uintptr_t)d_ws & 255u)) return PH_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)d_ws;
  const int nc = c->n_cells[0] * c->n_cells[1] * c->n_cells[2], nb = c->n_bins;
  PhArgs a;
  std::memset(&a, 0, sizeof(a));
  for (int d = 0; d < 3; ++d) {
    a.L[d] = c->L_nm[d];
    a.n[d] = c->n_cells[d];
    a.d[d] = c->L_nm[d] / c->n_cells[d];
  }
  for (int f = 0; f < 6; ++f) a.face[f] = c->face[f];
  a.ncell = nc;
  a.nb = nb;
  a.max_events = c->max_events;
  a.k0 = (uint32_t)(c->seed & 0xffffffffu);
  a.k1 = (uint32_t)(c->seed >> 32);
  a.tag = (c->instance << 4) | 5u;
  a.n_packets = c->n_packets;
  a.q = d_q_cell;
  a.cum_cell = (const double*)(ws + L.cum_cell);
  a.tab = d_tables;
  a.cum_emit = (const double*)(ws + L.cum_emit);
  a.t_cell = d_t_cell;
  a.pk_scat = d_packet_scatterings;
  a.counts = (unsigned long long*)(ws + L.counts);
  a.next = (unsigned long long*)(ws + L.next);
  double* sums = (double*)(ws + L.sums);
  k_ph_setup<<<(nc + kPhSetupBlock - 1) / kPhSetupBlock, kPhSetupBlock, 0, st>>>(
      d_q_cell, nc, d_tables, nb, (double*)(ws + L.cum_cell), (double*)(ws + L.cum_emit), d_t_cell, a.counts, a.next,
      sums);
  int dev = 0, ncu = 0, per = 0;
  const size_t lds = sizeof(double) * (3 * (size_t)nb + nc);
  if (lds > 160 * 1024) return PH_E_ARG;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_ph_packets, kPhBlock, lds) != hipSuccess)
    return PH_E_HIP;
  long long need = (c->n_packets + kPhBlock - 1) / kPhBlock;
  long long grid = (long long)ncu * (per > 0 ? per : 1);
  if (grid > need) grid = need;
  k_ph_packets<<<(unsigned)grid, kPhBlock, lds, st>>>(a);
  if (d_dT)
    k_ph_dT<<<(nc + 255) / 256, 256, 0, st>>>(d_t_cell, sums, nc, (double)c->n_packets,
                                             a.d[0] * a.d[1] * a.d[2] * 1e-27, d_dT);
  if (hipGetLastError() != hipSuccess) return PH_E_HIP;
  if (h_counts) {
    if (hipMemcpyAsync(h_counts, ws + L.counts, 8 * CT_N, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return PH_E_HIP;
  }
  return PH_OK;
}

}  // extern "C"
