// gfmc_refresh.h -- gfx950 kernels around the particle kernel: the summed
// subcell histograms, the contact refill, the Poisson refresh and field,
// the set-up kernels (rate tables, per-subcell factors, Gamma_v, the initial
// ensemble, the dense Poisson inverse) and the bulk-mode observables.
#pragma once
#include "gfmc_kernels.h"

namespace gfmc {

// Subcell grid of the Poisson problem (the discretisation is described with
// the Poisson kernels below).
struct PoisGeo {
  int nx, ny, nz, P;
  double dx, dy, dz, gx, gy, gz, gate0, gate1, Vc;
};

__device__ __forceinline__ bool gated(const PoisGeo& g, int ix) {
  const double xc = (ix + 0.5) * g.dx;
  return xc >= g.gate0 && xc <= g.gate1;
}

// Right-hand side of the balance of cell c (coulombs) holding n electrons:
// the terminal faces' Dirichlet terms plus the doping minus the electrons.
__device__ __forceinline__ double rhs_cell(const PoisGeo& g, const InstParams& I, int c, uint32_t n) {
  const int P = g.P;
  const int ix = c / P, l = c % P, iy = l / g.nz, iz = l % g.nz;
  double b = 0.0;
  if (ix == g.nx - 1) b += 2.0 * g.gx * I.Vds;
  if (gated(g, ix)) {
    if (iy == g.ny - 1) b += 2.0 * g.gy * I.phig;
    if (iz == g.nz - 1) b += 2.0 * g.gz * I.phig;
  }
  return b + kQ * (I.N_D_nm * g.Vc - I.w * (double)n);
}

// Every kernel that counts electrons or heat per subcell (the flight kernels,
// k_deposit outside a flight) keeps a histogram per workgroup in LDS and adds
// its nonzero bins to a u64 accumulator per instance by atomics: integer
// sums, the same in any order.  k_inject_plan then moves the accumulator into
// the electron count (bins [0, ncell)) and the window heat counts (bins
// [ncell, 5 ncell)) and clears it; k_field advances the interval counter.
// Deposit only (used outside a flight interval): live electrons per subcell
// into the instance's accumulator, free slots per tile.
template <typename T>
__global__ void k_deposit(const TileDesc* __restrict__ tiles, const T* __restrict__ x, const T* __restrict__ y,
                          const T* __restrict__ z, const uint32_t* __restrict__ meta, Geo<T> G,
                          unsigned long long* acc, uint32_t* tile_dead) {
  extern __shared__ uint32_t sh[];
  const int ncell = G.ncell;
  for (int i = threadIdx.x; i < 5 * ncell + 1; i += blockDim.x) sh[i] = 0u;
  __syncthreads();
  const TileDesc td = tiles[blockIdx.x];
  uint32_t dead = 0;
  for (int i = threadIdx.x; i < td.count; i += blockDim.x) {
    const long long p = td.start + i;
    if (meta[p] & kAlive) atomicAdd(sh + cell_of(G, x[p], y[p], z[p]), 1u);
    else ++dead;
  }
  dead = wave_sum(dead);
  if ((threadIdx.x & 63) == 0 && dead) atomicAdd(sh + 5 * ncell, dead);
  __syncthreads();
  unsigned long long* h = acc + (size_t)td.inst * 5 * ncell;
  for (int i = threadIdx.x; i < ncell; i += blockDim.x)
    if (sh[i]) atomicAdd(h + i, (unsigned long long)sh[i]);
  if (threadIdx.x == 0) tile_dead[blockIdx.x] = sh[5 * ncell];
}

// The refresh after the histograms are summed, per instance (grid y).  Workgroup 0
// plans the contact refill: the free-slot offsets of the instance's tiles
// (block-wide exclusive scan, each lane owning a contiguous run of tiles),
// the exact count of holes below the live count, then, in wavefront 0, the
// electrons needed per contact subcell and their offsets (the q-th new
// electron takes the q-th free slot), and the contact subcells' counts and
// Poisson right-hand side with their new electrons.  The other workgroups
// move the rest of the summed histogram into the counts, right-hand side,
// density and heat sums.
constexpr int kPlanThreads = 1024;
__global__ void __launch_bounds__(kPlanThreads) k_inject_plan(const InstParams* __restrict__ ip,
                                                              const TileDesc* __restrict__ tiles,
                                                              const uint32_t* __restrict__ meta, PoisGeo g,
                                                              int ncell, unsigned long long* acc, uint32_t* count,
                                                              unsigned long long* heat, int after_flight,
                                                              const uint32_t* __restrict__ tile_dead,
                                                              uint32_t* tile_off, Plan* plan, uint32_t* next_id,
                                                              unsigned long long* counters, int* flags,
                                                              const uint32_t* ctl, double* rhs_out,
                                                              unsigned long long* dens, double* hist) {
  __shared__ uint32_t s_wave[kPlanThreads / 64];
  __shared__ uint32_t s_holes[kPlanThreads / 64];
  __shared__ int s_edge;
  const int inst = blockIdx.y;
  const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6;
  const InstParams& I = ip[inst];
  const int nx = g.nx, P = g.P;
  if (blockIdx.x > 0) {
    // the other workgroups: one bin of the summed histogram per thread, the
    // accumulator cleared for the next interval.  A subcell's count and its
    // Poisson right-hand side (after a flight also its density sum); a heat
    // bin added to the window.  The contact subcells are left to workgroup 0.
    const int bin = (blockIdx.x - 1) * kPlanThreads + tid;
    if (bin >= 5 * ncell || (bin < ncell && (bin < P || bin >= ncell - P))) return;
    unsigned long long* a = acc + (size_t)inst * 5 * ncell + bin;
    const unsigned long long v = *a;
    *a = 0ull;
    if (bin < ncell) {
      const uint32_t n = (uint32_t)v;
      count[(size_t)inst * ncell + bin] = n;
      rhs_out[(size_t)inst * ncell + bin] = rhs_cell(g, I, bin, n);
      if (after_flight) dens[(size_t)inst * ncell + bin] += n;
    } else if (after_flight) {
      heat[(size_t)inst * 4 * ncell + (bin - ncell)] += v;
    }
    return;
  }
  // free slots per tile, exclusive prefix over the instance's tiles
  const int nt = I.t1 - I.t0;
  const int per = (nt + kPlanThreads - 1) / kPlanThreads;
  const int ta = I.t0 + tid * per, tb = min(I.t1, ta + per);
  uint32_t mine = 0;
  for (int t = ta; t < tb; ++t) mine += tile_dead[t];
  uint32_t inc = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o);
    if (l >= o) inc += y;
  }
  if (l == 63) s_wave[wv] = inc;
  __syncthreads();
  uint32_t before = 0, run = 0;
#pragma unroll
  for (int w = 0; w < kPlanThreads / 64; ++w) {
    const uint32_t t = s_wave[w];
    before += w < wv ? t : 0u;
    run += t;
  }
  uint32_t o = before + inc - mine;
  for (int t = ta; t < tb; ++t) {
    tile_off[t] = o;
    o += tile_dead[t];
  }
  // free slots below the live count: holes a compaction would close (the
  // free slots of the tiles wholly below it, plus those of the tile it falls
  // in, counted slot by slot, so the count does not depend on the tiling)
  const uint32_t alive = (uint32_t)I.cap - run;
  if (tid == 0) s_edge = -1;
  __syncthreads();
  uint32_t holes = 0;
  for (int t = ta; t < tb; ++t) {
    const long long s0 = tiles[t].start - I.base;
    if (s0 + tiles[t].count <= (long long)alive) holes += tile_dead[t];
    else if (s0 < (long long)alive) s_edge = t;  // one tile holds the position
  }
  __syncthreads();
  if (s_edge >= 0) {
    const long long s0 = tiles[s_edge].start;
    const int n = (int)((long long)alive - (s0 - I.base));
    for (int i = tid; i < n; i += kPlanThreads) holes += (meta[s0 + i] & kAlive) ? 0u : 1u;
  }
  holes = wave_sum(holes);
  if (l == 0) s_holes[wv] = holes;
  __syncthreads();
  if (wv == 0) {
    holes = 0;
#pragma unroll
    for (int w = 0; w < kPlanThreads / 64; ++w) holes += s_holes[w];
    // contact subcells: their summed counts straight from the accumulator
    unsigned long long* a = acc + (size_t)inst * 5 * ncell;
    int cell = -1;
    uint32_t need = 0, have = 0;
    if (l < 2 * P) {
      cell = l < P ? l : (nx - 1) * P + (l - P);
      have = (uint32_t)a[cell];
      a[cell] = 0ull;
      need = (int)have < I.target ? (uint32_t)(I.target - (int)have) : 0u;
    }
    // inclusive scan over the 64 lanes
    uint32_t ninc = need;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(ninc, d);
      if (l >= d) ninc += y;
    }
    uint32_t Q = __shfl(ninc, 63);
    const uint32_t off = ninc - need;
    if (run < Q) {
      if (l == 0) set_flag(flags, inst, -3);
      Q = run;
    }
    const uint32_t id0 = next_id[inst];
    if ((unsigned long long)id0 + Q >= (1ull << 29)) {
      if (l == 0) set_flag(flags, inst, -3);
      Q = 0;
    }
    uint32_t got = 0;
    if (cell >= 0) {
      // count, right-hand side and density sum of the contact subcell with
      // its new electrons
      got = off >= Q ? 0u : (off + need <= Q ? need : Q - off);
      const uint32_t n = have + got;
      const size_t o = (size_t)inst * ncell + cell;
      count[o] = n;
      rhs_out[o] = rhs_cell(g, I, cell, n);
      if (after_flight) dens[o] += n;
    }
    Plan* pl = plan + inst;
    pl->need[l] = need;
    pl->off[l] = off;
    const uint32_t src = wave_sum(l < P ? got : 0u), drn = wave_sum(l >= P ? got : 0u);
    if (l == 0) {
      pl->Q = Q;
      pl->id0 = id0;
      pl->u = ctl[CTL_INTERVAL] + (after_flight ? 1u : 0u);  // k_field advances the counter
      pl->alive = alive;
      const uint32_t compact = (unsigned long long)holes * 32u > alive ? 1u : 0u;
      pl->compact = compact;
      // new slots in use: after a compaction the live electrons fill [0, alive)
      // and the new ones follow them; otherwise the Q lowest free slots take
      // the new ones, so the bound grows only past alive + Q
      pl->hw = compact ? alive + Q : max(min(pl->hw, (uint32_t)I.cap), alive + Q);
      next_id[inst] = id0 + Q;
      unsigned long long* cn = counters + (size_t)inst * kNCnt;
      cn[C_INJ0] += src;
      cn[C_INJ1] += drn;
      // history row of an interval: the window's contact counts and the
      // electrons present; k_field adds the potential and field
      const uint32_t row = ctl[CTL_WINDOW];
      pl->row = (after_flight && row < (uint32_t)kHistCap) ? row : kNoRow;
      if (pl->row != kNoRow) {
        double* h = hist + ((size_t)inst * kHistCap + row) * 8;
        h[0] = (double)cn[C_EXIT0];
        h[1] = (double)cn[C_EXIT1];
        h[2] = (double)cn[C_INJ0];
        h[3] = (double)cn[C_INJ1];
        h[4] = (double)(alive + Q);
        h[7] = (double)(ctl[CTL_INTERVAL] + 1u);
      }
    }
  }
}

// Bound of slots in use of one instance, set by the host where it knows it
// (initial ensemble) or cannot (particles written from the host: capacity).
__global__ void k_set_hw(Plan* plan, int inst, uint32_t hw) {
  if (threadIdx.x == 0) plan[inst].hw = hw;
}

// Exclusive prefix sum of a[0..n) in place (n <= kShareMax, one workgroup of
// 256 threads, each a run of consecutive entries); returns the total.
__device__ inline int block_scan_excl(int* a, int n, int* tmp) {
  const int tid = threadIdx.x, per = (n + 255) / 256, b = min(n, tid * per), e = min(n, b + per);
  int s = 0;
  for (int i = b; i < e; ++i) s += a[i];
  tmp[tid] = s;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int v = tid >= o ? tmp[tid - o] : 0;
    __syncthreads();
    tmp[tid] += v;
    __syncthreads();
  }
  int run = tid ? tmp[tid - 1] : 0;
  const int total = tmp[255];
  for (int i = b; i < e; ++i) {
    const int v = a[i];
    a[i] = run;
    run += v;
  }
  __syncthreads();
  return total;
}

// Workgroups of the persistent particle kernels per instance, in proportion
// to each instance's segments (selections and electrons taken) over the
// previous interval rather than to its slots: per-electron work differs
// between bias points.  prev[0..n) holds the counts at the previous call and
// prev[n] is non-zero once they are valid (the host clears it whenever it
// sets the slot shares).  Each instance keeps at least one workgroup and
// enough that none owns more than max_chunks chunks, at most one per chunk;
// the shares add up to the launched grid (total, at most the chunks of all
// instances), the remainder of the rounding going to the instances with
// chunks to spare in instance order.  With no valid previous counts (the
// first interval, or counters put back by a restore) the shares stay.
// Which workgroup takes an electron does not change its result.
constexpr int kShareMax = 1024;
__global__ void __launch_bounds__(256) k_share_work(InstParams* ip, int n, const unsigned long long* counters,
                                                    unsigned long long* prev, int* wg_inst, int total, int max_chunks) {
  __shared__ unsigned long long s_work[kShareMax];
  __shared__ int s_share[kShareMax], s_room[kShareMax], s_tmp[256];
  __shared__ unsigned long long s_tot;
  __shared__ int s_ok, s_min;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_ok = prev[n] != 0ull;
    s_tot = 0ull;
    s_min = 0;
  }
  __syncthreads();
  unsigned long long tot = 0ull;
  int bad = 0, mins = 0;
  for (int i = tid; i < n; i += 256) {
    const unsigned long long cur = counters[(size_t)i * kNCnt + C_SEL] + counters[(size_t)i * kNCnt + C_PROC];
    const unsigned long long pv = prev[i];
    bad |= cur < pv;
    s_work[i] = cur >= pv ? cur - pv : 0ull;
    tot += s_work[i];
    prev[i] = cur;
    mins += max(1, (ip[i].nchunk + max_chunks - 1) / max_chunks);
  }
  if (bad) atomicAnd(&s_ok, 0);
  atomicAdd(&s_tot, tot);
  atomicAdd(&s_min, mins);
  __syncthreads();
  if (tid == 0) prev[n] = 1ull;
  if (!s_ok || s_tot == 0ull || s_min > total) return;
  const double E = (double)(total - s_min), T = (double)s_tot;
  for (int i = tid; i < n; i += 256) {
    const int nc = ip[i].nchunk;
    const int m = max(1, (nc + max_chunks - 1) / max_chunks);
    const int sh = min(nc, m + (int)(E * (double)s_work[i] / T));
    s_share[i] = sh;
    s_room[i] = nc - sh;
  }
  __syncthreads();
  // shares so far, and the remainder placed in instance order where chunks
  // are to spare
  int* sh_copy = reinterpret_cast<int*>(s_work);  // the work counts are no longer needed
  for (int i = tid; i < n; i += 256) sh_copy[i] = s_share[i];
  __syncthreads();
  const int assigned = block_scan_excl(sh_copy, n, s_tmp);
  const int R = total - assigned;
  block_scan_excl(s_room, n, s_tmp);  // s_room now holds the room before each instance
  for (int i = tid; i < n; i += 256) {
    const int room = ip[i].nchunk - s_share[i];
    s_share[i] += max(0, min(room, R - s_room[i]));
  }
  __syncthreads();
  for (int i = tid; i < n; i += 256) sh_copy[i] = s_share[i];
  __syncthreads();
  block_scan_excl(sh_copy, n, s_tmp);  // first workgroup of each instance
  for (int i = tid; i < n; i += 256) {
    const int w0 = sh_copy[i], w1 = w0 + s_share[i];
    ip[i].w0 = w0;
    ip[i].w1 = w1;
    for (int w = w0; w < w1; ++w) wg_inst[w] = i;
  }
}

// Stable compaction of an instance's slots (device mode), in a refresh where k_inject_plan
// found the free slots below the live count above 1/32 of the live
// electrons: every live electron keeps its order and moves to the slot of its
// rank among the live ones, and the free slots become the tail.  Electrons
// carry their identity, so the move changes no result; it keeps the particle
// kernel's tiles dense (holes cost it extra refill rounds).
// Pass 1, one 256-lane workgroup per tile, 256 consecutive slots per step:
// ranks from the tile's live prefix (its start minus the free slots before
// it, from k_inject_plan) and a block scan of the live flags; the state goes
// to the scratch arrays at that rank; the tile's free-slot count and offset
// are rewritten for the compacted layout.
template <typename T>
struct StateArrays {
  T *kx, *ky, *kz, *x, *y, *z;
  uint32_t* meta;
};

template <typename T>
__global__ void __launch_bounds__(256) k_compact_scatter(const TileDesc* __restrict__ tiles,
                                                         const InstParams* __restrict__ ip,
                                                         const Plan* __restrict__ plan, uint32_t* tile_off,
                                                         uint32_t* tile_dead, StateArrays<T> src,
                                                         StateArrays<T> dst) {
  __shared__ uint32_t s_wave[4];
  const TileDesc td = tiles[blockIdx.x];
  const Plan& pl = plan[td.inst];
  if (!pl.compact) return;
  const long long base = ip[td.inst].base;
  const uint32_t s0 = (uint32_t)(td.start - base), alive = pl.alive;
  uint32_t run = s0 - tile_off[blockIdx.x];  // live slots before this tile
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int b = 0; b < td.count; b += 256) {
    const int i = b + (int)threadIdx.x;
    const long long p = td.start + i;
    const uint32_t m = i < td.count ? src.meta[p] : 0u;
    const bool live = (m & kAlive) != 0;
    const unsigned long long bal = __ballot(live);
    if (lane == 0) s_wave[wave] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      before += w < wave ? s_wave[w] : 0u;
      total += s_wave[w];
    }
    const long long q = base + run + before + (uint32_t)__popcll(bal & lt);
    if (live && q < base + ip[td.inst].cap) {  // the bound always holds: tile counts match the flags
      dst.meta[q] = m;
      dst.kx[q] = src.kx[p]; dst.ky[q] = src.ky[p]; dst.kz[q] = src.kz[p];
      dst.x[q] = src.x[p]; dst.y[q] = src.y[p]; dst.z[q] = src.z[p];
    }
    run += total;
    __syncthreads();  // s_wave is rewritten by the next step
  }
  if (threadIdx.x == 0) {
    const uint32_t c = (uint32_t)td.count;
    const uint32_t live_after = alive > s0 ? min(c, alive - s0) : 0u;
    tile_dead[blockIdx.x] = c - live_after;
    tile_off[blockIdx.x] = s0 > alive ? s0 - alive : 0u;
  }
}

// Free-slot ranks of one tile (one 256-lane workgroup, 16 consecutive slots
// per lane and step), after the tile's part of a compaction if its instance
// compacts in this refresh: a block prefix scan of the lanes' free counts
// gives every free slot its instance-wide rank q, and the slot of rank q < Q
// is written to position q of the instance's slot list (relative slot index).
// Tiles whose first rank is already >= Q, or that hold no free slot, stop
// there.  Every tile's free count is cleared here once read.
template <typename T>
__global__ void __launch_bounds__(256) k_inject_slots(const TileDesc* __restrict__ tiles,
                                                      const InstParams* __restrict__ ip,
                                                      const Plan* __restrict__ plan,
                                                      const uint32_t* __restrict__ tile_off, uint32_t* tile_dead,
                                                      StateArrays<T> st, StateArrays<T> scr, uint32_t* slot_list) {
  __shared__ uint32_t s_wave[4];
  const TileDesc td = tiles[blockIdx.x];
  const Plan& pl = plan[td.inst];
  const uint32_t Q = pl.Q;
  if (pl.compact) {
    // second pass of a compaction: the tile's slots take back the compacted
    // state (below the live count) or are marked free
    const long long alive_end = ip[td.inst].base + (long long)pl.alive;
    for (int i = threadIdx.x; i < td.count; i += blockDim.x) {
      const long long p = td.start + i;
      if (p < alive_end) {
        st.meta[p] = scr.meta[p];
        st.kx[p] = scr.kx[p]; st.ky[p] = scr.ky[p]; st.kz[p] = scr.kz[p];
        st.x[p] = scr.x[p]; st.y[p] = scr.y[p]; st.z[p] = scr.z[p];
      } else {
        st.meta[p] = 0u;
      }
    }
    __syncthreads();  // the free-slot scan below reads these meta words
  }
  const uint32_t* meta = st.meta;
  uint32_t run = tile_off[blockIdx.x];
  const uint32_t ndead = tile_dead[blockIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) tile_dead[blockIdx.x] = 0u;  // the persistent kernel adds to it
  if (run >= Q || ndead == 0) return;
  const long long base = ip[td.inst].base;
  uint32_t* list = slot_list + base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool vec = (td.start & 3) == 0;  // 16-byte aligned meta rows
  for (int b = 0; b < td.count && run < Q; b += 256 * 16) {
    const int i0 = b + 16 * (int)threadIdx.x;
    const uint32_t* mp = meta + td.start + i0;
    uint32_t freem = 0;  // bit e: slot i0 + e is free
    if (vec && i0 + 16 <= td.count) {
      uint4 v[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) v[h] = reinterpret_cast<const uint4*>(mp)[h];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        freem |= ((v[h].x & kAlive) ? 0u : 1u) << (4 * h);
        freem |= ((v[h].y & kAlive) ? 0u : 1u) << (4 * h + 1);
        freem |= ((v[h].z & kAlive) ? 0u : 1u) << (4 * h + 2);
        freem |= ((v[h].w & kAlive) ? 0u : 1u) << (4 * h + 3);
      }
    } else {
      for (int e = 0; e < 16; ++e)
        if (i0 + e < td.count && !(mp[e] & kAlive)) freem |= 1u << e;
    }
    const uint32_t nd = (uint32_t)__popc(freem);
    uint32_t inc = nd;  // inclusive scan over the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const uint32_t t = s_wave[w];
      before += w < wave ? t : 0u;
      total += t;
    }
    uint32_t q = run + before + inc - nd;
    while (freem && q < Q) {
      const int e = __ffs(freem) - 1;
      freem &= freem - 1;
      list[q] = (uint32_t)(td.start + i0 + e - base);
      ++q;
    }
    run += total;
    __syncthreads();  // s_wave is rewritten by the next step
  }
}

// Contact refill (one thread per new electron q < Q of instance blockIdx.y):
// its contact subcell is the first whose cumulative need exceeds q, its
// wave vector a Maxwellian at that subcell's lattice temperature and its
// position uniform in the subcell, drawn from the counter (subcell,
// interval, index within the subcell); it takes slot list[q] and the
// identity next_id + q.
template <typename T>
__global__ void __launch_bounds__(256) k_inject_fill(const InstParams* __restrict__ ip,
                                                     const Plan* __restrict__ plan,
                                                     const uint32_t* __restrict__ slot_list,
                                                     const double* __restrict__ Tcell, Geo<T> G, double m_g1,
                                                     double ck, T* kx, T* ky, T* kz, T* x, T* y, T* z,
                                                     uint32_t* meta) {
  __shared__ uint32_t s_end[64];
  const int inst = blockIdx.y;
  const Plan& pl = plan[inst];
  const uint32_t Q = pl.Q;
  const uint32_t q0 = blockIdx.x * 256u;
  if (q0 >= Q) return;
  const int P = G.ny * G.nz, n2 = 2 * P;
  if (threadIdx.x < 64) s_end[threadIdx.x] = pl.off[threadIdx.x] + pl.need[threadIdx.x];
  __syncthreads();
  const uint32_t q = q0 + threadIdx.x;
  if (q >= Q) return;
  int lo = 0, hi = n2 - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (s_end[mid] > q) hi = mid; else lo = mid + 1;
  }
  const int l = lo;
  const InstParams I = ip[inst];
  const long long p = I.base + slot_list[I.base + q];
  const int side = l >= P ? 1 : 0;
  const int lc = side ? l - P : l;
  const int cell = side ? (G.nx - 1) * P + lc : lc;
  const uint32_t ii = q - pl.off[l];
  const uint4 w = philox((uint32_t)cell, pl.u, ii, I.tagw | 2u, I.key0, I.key1);
  const double Tc = Tcell[(size_t)inst * G.ncell + cell];
  const T sig = (T)sqrt(m_g1 * kKb * Tc / kQ / (2.0 * ck));
  const T r1 = Ar<T>::sq((T)-2 * Ar<T>::ln(Ar<T>::u01(w.x))), r2 = Ar<T>::sq((T)-2 * Ar<T>::ln(Ar<T>::u01(w.z)));
  T c1, s1, c2, s2;
  Ar<T>::cs2pi(Ar<T>::u01(w.y), c1, s1);
  Ar<T>::cs2pi(Ar<T>::u01(w.w), c2, s2);
  kx[p] = sig * r1 * c1;
  ky[p] = sig * r1 * s1;
  kz[p] = sig * r2 * c2;
  const uint4 w2 = philox((uint32_t)cell, pl.u, ii, I.tagw | 3u, I.key0, I.key1);
  const int ix = side ? G.nx - 1 : 0, iy = lc / G.nz, iz = lc % G.nz;
  x[p] = ((T)ix + Ar<T>::u01(w2.x)) * G.d[0];
  y[p] = ((T)iy + Ar<T>::u01(w2.y)) * G.d[1];
  z[p] = ((T)iz + Ar<T>::u01(w2.z)) * G.d[2];
  meta[p] = ((pl.id0 + q) << 3) | kAlive;
}

// Initial Maxwellian ensemble: slot p < N gets identity p.
template <typename T, bool DEV>
__global__ void k_init(const InstParams* __restrict__ ip, int inst, Geo<T> G, double m_g1, double ck, T* kx, T* ky,
                       T* kz, T* x, T* y, T* z, uint32_t* meta, int n) {
  const InstParams I = ip[inst];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= I.cap) return;
  const long long p = I.base + i;
  if (i >= n) {
    kx[p] = ky[p] = kz[p] = (T)0;
    if (DEV) x[p] = y[p] = z[p] = (T)0;
    meta[p] = 0u;
    return;
  }
  const uint4 w = philox((uint32_t)i, 0u, 0u, I.tagw | 1u, I.key0, I.key1);
  const T sig = (T)sqrt(m_g1 * kKb * I.T_init / kQ / (2.0 * ck));
  const T r1 = Ar<T>::sq((T)-2 * Ar<T>::ln(Ar<T>::u01(w.x))), r2 = Ar<T>::sq((T)-2 * Ar<T>::ln(Ar<T>::u01(w.z)));
  T c1, s1, c2, s2;
  Ar<T>::cs2pi(Ar<T>::u01(w.y), c1, s1);
  Ar<T>::cs2pi(Ar<T>::u01(w.w), c2, s2);
  kx[p] = sig * r1 * c1;
  ky[p] = sig * r1 * s1;
  kz[p] = sig * r2 * c2;
  if (DEV) {
    const uint4 w2 = philox((uint32_t)i, 0u, 1u, I.tagw | 1u, I.key0, I.key1);
    x[p] = Ar<T>::u01(w2.x) * G.L[0];
    y[p] = Ar<T>::u01(w2.y) * G.L[1];
    z[p] = Ar<T>::u01(w2.z) * G.L[2];
  }
  meta[p] = ((uint32_t)i << 3) | kAlive;
}

// Rate-shape tables on the bin midpoints, FP64, plus an FP32 copy.
__global__ void k_tables(RateMat R, int nb, double dE, double ck, double* t64, float* t32) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kNV * nb) return;
  const int v = idx / nb, b = idx % nb;
  const double E = (b + 0.5) * dE;
  double S[kTRow];
  const double D = R.D_ac * kQ;
  S[0] = 2.0 * kPi / kHbar * D * D * kKb / (R.rho * R.u_ac * R.u_ac) * dos_si(R, v, E) * 1e-15;
  const double eps = R.eps_s * kEps0;
  S[1] = 2.0 * kPi / kHbar * (kQ * kQ * kQ * kQ) / (eps * eps) * dos_si(R, v, E) * 1e-24;
  S[2] = pop_shape(R, v, E, E + R.hw_lo) * 1e-15;
  S[3] = pop_shape(R, v, E, E - R.hw_lo) * 1e-15;
  for (int j = 0; j < kNV; ++j)
    for (int em = 0; em < 2; ++em) {
      const double Ep = E + R.Ec[v] - R.Ec[j] + (em ? -R.hw_iv : R.hw_iv);
      S[4 + 2 * j + em] = iv_shape(R, v, j, Ep) * 1e-15;
    }
  S[10] = 4.0 * (E * (1.0 + R.alpha[v] * E)) * R.m[v] / ck;
  S[11] = 0.0;
  for (int q = 0; q < kTRow; ++q) {
    t64[(size_t)idx * kTRow + q] = S[q];
    t32[(size_t)idx * kTRow + q] = (float)S[q];
  }
}

// Temperature factors per subcell.
__global__ void k_factors(const double* __restrict__ Tcell, const InstParams* __restrict__ ip, int ncell,
                          double eps_s, double hw_lo, double hw_iv, double* f64, float* f32) {
  const int inst = blockIdx.y;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const double T = Tcell[(size_t)inst * ncell + c];
  const double ND = ip[inst].N_D_m3;
  const double b2 = kQ * kQ * ND / (eps_s * kEps0 * kKb * T) * 1e-18;
  const double N = 1.0 / (exp(hw_lo * kQ / (kKb * T)) - 1.0);
  const double Niv = 1.0 / (exp(hw_iv * kQ / (kKb * T)) - 1.0);
  double f[kFRow] = {T, ip[inst].N_D_nm / b2, N, N + 1.0, Niv, Niv + 1.0, b2, 0.0};
  const size_t o = ((size_t)inst * ncell + c) * kFRow;
  for (int q = 0; q < kFRow; ++q) { f64[o + q] = f[q]; f32[o + q] = (float)f[q]; }
}

// Gamma_v: the maximum of the tabulated total over bins and the instance's
// distinct-temperature subcells, in the precision that uses it.  Grid
// (instance, valley, chunk of kGammaReps distinct subcells); each block's
// maximum joins gamma (zeroed beforehand) by an atomic maximum on the bit
// pattern, which orders non-negative floats as their values.  A maximum does
// not depend on the order of its terms, so the result is the same for any
// split.
constexpr int kGammaReps = 32;

__device__ inline void atomic_max_nonneg(double* p, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}
__device__ inline void atomic_max_nonneg(float* p, float v) {
  atomicMax(reinterpret_cast<unsigned int*>(p), __float_as_uint(v));
}

template <typename T>
__global__ void k_gamma(const T* __restrict__ table, const T* __restrict__ fac, const int* __restrict__ reps,
                        const int* __restrict__ nrep, int ncell, int nb, T* gamma) {
  const int inst = blockIdx.x, v = blockIdx.y;
  const int r0 = blockIdx.z * kGammaReps;
  const int n = nrep[inst];
  if (r0 >= n) return;
  const int nr = min(kGammaReps, n - r0);
  __shared__ T smax[1024];
  T g = (T)0;
  for (int idx = threadIdx.x; idx < nr * nb; idx += blockDim.x) {
    const int r = r0 + idx / nb, b = idx % nb;
    const T* S = table + ((size_t)v * nb + b) * kTRow;
    const T* f = fac + ((size_t)inst * ncell + reps[(size_t)inst * ncell + r]) * kFRow;
    const T tot = tab_total<T>(S, f);
    g = tot > g ? tot : g;
  }
  smax[threadIdx.x] = g;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomic_max_nonneg(gamma + inst * 4 + v, smax[0]);
}

// ---------------------------------------------------------------------------
// Poisson: finite volumes on the subcell grid, eps_s eps0 uniform; Dirichlet
// faces half a cell from the centre (source x=0: 0 V; drain x=L: Vds; gated
// top and outer side: Vgs + offset), Neumann elsewhere.  The matrix is block
// tridiagonal in x with P = ny nz blocks; the x coupling is -gx I.
// Block LU: S_0 = D_0, S_i = D_i - gx^2 S_{i-1}^{-1}; M_i = S_i^{-1}.
// ---------------------------------------------------------------------------
// one workgroup; builds M_i for all slices (init only)
__global__ void k_poisson_factor(PoisGeo g, double* Minv) {
  __shared__ double A[32][65];  // [S | I] augmented, then [I | S^-1]
  __shared__ double Mprev[32][32];
  const int P = g.P;
  for (int ix = 0; ix < g.nx; ++ix) {
    const bool gt = gated(g, ix);
    for (int e = threadIdx.x; e < P * 2 * P; e += blockDim.x) {
      const int r = e / (2 * P), c = e % (2 * P);
      double val = 0.0;
      if (c < P) {
        const int iy = r / g.nz, iz = r % g.nz, jy = c / g.nz, jz = c % g.nz;
        if (r == c) {
          val += ix > 0 ? g.gx : 2.0 * g.gx;
          val += ix < g.nx - 1 ? g.gx : 2.0 * g.gx;
          val += iy > 0 ? g.gy : 0.0;
          val += iy < g.ny - 1 ? g.gy : (gt ? 2.0 * g.gy : 0.0);
          val += iz > 0 ? g.gz : 0.0;
          val += iz < g.nz - 1 ? g.gz : (gt ? 2.0 * g.gz : 0.0);
          if (ix > 0) val -= g.gx * g.gx * Mprev[r][c];
        } else {
          if (iz == jz && (iy - jy == 1 || jy - iy == 1)) val = -g.gy;
          if (iy == jy && (iz - jz == 1 || jz - iz == 1)) val = -g.gz;
          if (ix > 0) val -= g.gx * g.gx * Mprev[r][c];
        }
      } else {
        val = (c - P == r) ? 1.0 : 0.0;
      }
      A[r][c] = val;
    }
    __syncthreads();
    // Gauss-Jordan without pivoting (the matrix is symmetric positive definite)
    for (int k = 0; k < P; ++k) {
      const double piv = A[k][k];
      __syncthreads();
      for (int c = threadIdx.x; c < 2 * P; c += blockDim.x) A[k][c] /= piv;
      __syncthreads();
      for (int e = threadIdx.x; e < P * 2 * P; e += blockDim.x) {
        const int r = e / (2 * P), c = e % (2 * P);
        if (r != k) {
          const double f = A[r][k];
          if (c != k) A[r][c] -= f * A[k][c];
        }
      }
      __syncthreads();
      for (int r = threadIdx.x; r < P; r += blockDim.x)
        if (r != k) A[r][k] = 0.0;
      __syncthreads();
    }
    for (int e = threadIdx.x; e < P * P; e += blockDim.x) {
      const int r = e / P, c = e % P;
      const double m = A[r][P + c];
      Mprev[r][c] = m;
      Minv[((size_t)ix * P + r) * P + c] = m;
    }
    __syncthreads();
  }
}

// Block forward/backward sweep of one right-hand side held in LDS (`rhs`,
// ncell doubles), by one wavefront: lpr contiguous lanes per matrix row, each
// with up to kCpl columns of M_i, rows prefetched kPF steps ahead.  Leaves the
// solution in `h` (LDS, ncell doubles).
constexpr int kPF = 6;
constexpr int kCpl = 16;  // columns per lane: P <= 32 rows and at least 2 lanes per row
__device__ void block_sweep(const PoisGeo& g, const double* __restrict__ Minv, const double* rhs, double* h) {
  const int P = g.P, nx = g.nx;
  const int lane = threadIdx.x;
  const int lpr = min(8, 64 / P);
  const int r = lane / lpr, q = lane % lpr;
  const bool act = r < P;
  const int nsteps = 2 * nx - 1;
  auto slice = [nx](int s) { return s < nx ? s : 2 * nx - 2 - s; };
  double buf[kPF][kCpl];
#pragma unroll
  for (int k = 0; k < kPF; ++k) {
#pragma unroll
    for (int e = 0; e < kCpl; ++e) {
      const int col = q + lpr * e;
      buf[k][e] = (act && k < nsteps && col < P) ? Minv[((size_t)slice(k) * P + r) * P + col] : 0.0;
    }
  }
  for (int s0 = 0; s0 < nsteps; s0 += kPF) {
#pragma unroll
    for (int kk = 0; kk < kPF; ++kk) {
      const int s = s0 + kk;
      if (s < nsteps) {
        const int i = slice(s);
        double part = 0.0;
        if (act) {
#pragma unroll
          for (int e = 0; e < kCpl; ++e) {
            const int col = q + lpr * e;
            if (col < P) {
              const double vin = s < nx ? rhs[i * P + col] + (i > 0 ? g.gx * h[(i - 1) * P + col] : 0.0)
                                        : h[(i + 1) * P + col];
              part += buf[kk][e] * vin;
            }
          }
        }
        const int sn = s + kPF;
#pragma unroll
        for (int e = 0; e < kCpl; ++e) {
          const int col = q + lpr * e;
          buf[kk][e] = (act && sn < nsteps && col < P) ? Minv[((size_t)slice(sn) * P + r) * P + col] : 0.0;
        }
        double row = part;
        for (int o = 1; o < lpr; ++o) row += __shfl(part, (lane + o) & 63);
        __syncthreads();
        if (act && q == 0) {
          if (s < nx) h[i * P + r] = row;                 // h_i = M_i y_i
          else h[i * P + r] = h[i * P + r] + g.gx * row;  // x_i = h_i + gx M_i x_{i+1}
        }
        __syncthreads();
      }
    }
  }
}

// Dense inverse of the (symmetric) Poisson matrix, one column per
// wavefront: A^-1 e_j by the block sweep (init only).
__global__ void __launch_bounds__(64) k_poisson_inverse(PoisGeo g, const double* __restrict__ Minv, int ncell,
                                                        double* Ainv) {
  extern __shared__ double shd[];
  double* h = shd;
  double* rhs = shd + ncell;
  const int j = blockIdx.x;
  for (int c = threadIdx.x; c < ncell; c += 64) rhs[c] = c == j ? 1.0 : 0.0;
  __syncthreads();
  block_sweep(g, Minv, rhs, h);
  __syncthreads();
  for (int c = threadIdx.x; c < ncell; c += 64) Ainv[(size_t)j * ncell + c] = h[c];
}

// phi = A^-1 rhs: one wavefront per row, unit-stride reads of the
// (Infinity-Cache-resident) inverse.  Every output is summed in one fixed
// order -- lane l accumulates the products of columns j = l (mod 64) in
// ascending j with fused multiply-adds, then a butterfly over the lanes --
// which k_poisson_gemm repeats exactly, so a batched context gives the same
// potential as a context of one instance.
__device__ __forceinline__ double lane_butterfly(double s) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  return s;
}

__global__ void __launch_bounds__(256) k_poisson_gemv(const double* __restrict__ Ainv,
                                                      const double* __restrict__ rhs, int ncell, double* phi) {
  const int inst = blockIdx.y;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= ncell) return;
  const double* a = Ainv + (size_t)row * ncell;
  const double* b = rhs + (size_t)inst * ncell;
  double s = 0.0;
  // unrolled so the loads of several columns are in flight at once; the
  // sums stay in column order
#pragma unroll 8
  for (int j = lane; j < ncell; j += 64) s = fma(a[j], b[j], s);
  s = lane_butterfly(s);
  if (lane == 0) phi[(size_t)inst * ncell + row] = s;
}

// Many instances: Phi = A^-1 [rhs_0 ... rhs_n-1], register-blocked over R
// rows and G instances per wavefront, so each column element of the inverse
// is read once per G instances; same summation order as k_poisson_gemv.
template <int R, int G, int U>
__global__ void __launch_bounds__(256) k_poisson_gemm(const double* __restrict__ Ainv,
                                                      const double* __restrict__ rhs, int ncell, int n_inst,
                                                      double* phi) {
  const int lane = threadIdx.x & 63;
  const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * R;
  const int i0 = blockIdx.y * G;
  if (row0 >= ncell) return;
  double s[R][G];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int g = 0; g < G; ++g) s[r][g] = 0.0;
  const double* arow[R];
  const double* bcol[G];
#pragma unroll
  for (int r = 0; r < R; ++r) arow[r] = Ainv + (size_t)min(row0 + r, ncell - 1) * ncell;
#pragma unroll
  for (int g = 0; g < G; ++g) bcol[g] = rhs + (size_t)min(i0 + g, n_inst - 1) * ncell;
  // unrolled so several columns' loads are in flight; each sum stays in column order
#pragma unroll U
  for (int j = lane; j < ncell; j += 64) {
    double av[R], bv[G];
#pragma unroll
    for (int r = 0; r < R; ++r) av[r] = arow[r][j];
#pragma unroll
    for (int g = 0; g < G; ++g) bv[g] = bcol[g][j];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int g = 0; g < G; ++g) s[r][g] = fma(av[r], bv[g], s[r][g]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int g = 0; g < G; ++g) s[r][g] = lane_butterfly(s[r][g]);
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (row0 + r < ncell && i0 + g < n_inst) phi[(size_t)(i0 + g) * ncell + row0 + r] = s[r][g];
  }
}

// Centred-difference field E = -grad(phi): a Dirichlet neighbour is its face
// value half a cell away, a Neumann neighbour the cell itself.
// Cell-centred field E = -grad(phi) of subcell c (V/nm): centred
// differences; a Dirichlet neighbour (source, drain, gated face) is its face
// value half a cell away, a Neumann neighbour is the cell itself.
__device__ __forceinline__ void cell_field(const PoisGeo& g, const InstParams& I, const double* h, int c,
                                           double& ex, double& ey, double& ez) {
  const int P = g.P, nx = g.nx;
  const int ix = c / P, l = c % P, iy = l / g.nz, iz = l % g.nz;
  const double pc = h[c];
  const bool gt = gated(g, ix);
  double pe, de, pw, dw;
  if (ix < nx - 1) { pe = h[c + P]; de = g.dx; } else { pe = I.Vds; de = 0.5 * g.dx; }
  if (ix > 0) { pw = h[c - P]; dw = g.dx; } else { pw = 0.0; dw = 0.5 * g.dx; }
  ex = -(pe - pw) / (de + dw);
  double pn, dn, ps, ds;
  if (iy < g.ny - 1) { pn = h[c + g.nz]; dn = g.dy; }
  else if (gt) { pn = I.phig; dn = 0.5 * g.dy; }
  else { pn = pc; dn = 0.0; }
  if (iy > 0) { ps = h[c - g.nz]; ds = g.dy; } else { ps = pc; ds = 0.0; }
  ey = (dn + ds) > 0.0 ? -(pn - ps) / (dn + ds) : 0.0;
  double pt, dt, pb, db;
  if (iz < g.nz - 1) { pt = h[c + 1]; dt = g.dz; }
  else if (gt) { pt = I.phig; dt = 0.5 * g.dz; }
  else { pt = pc; dt = 0.0; }
  if (iz > 0) { pb = h[c - 1]; db = g.dz; } else { pb = pc; db = 0.0; }
  ez = (dt + db) > 0.0 ? -(pt - pb) / (dt + db) : 0.0;
}

// The field of every subcell (one per thread).  After a flight workgroup 0
// of each instance also completes the interval's history row with the mean
// potential and the root-mean-square field over all subcells (a fixed-order
// reduction), and one thread advances the interval counters.
__global__ void __launch_bounds__(256) k_field(PoisGeo g, const InstParams* __restrict__ ip,
                                               const double* __restrict__ phi_all, int ncell, double* field64,
                                               float* field32, uint32_t* ctl, int advance,
                                               const Plan* __restrict__ plan, double* hist) {
  __shared__ double s_red[2][4];
  const int inst = blockIdx.y;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const InstParams& I = ip[inst];
  const double* h = phi_all + (size_t)inst * ncell;
  if (advance && blockIdx.x == 0) {
    const uint32_t row = plan[inst].row;
    if (row != kNoRow) {
      double sp = 0.0, sf = 0.0;
      for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
        double ex, ey, ez;
        cell_field(g, I, h, q, ex, ey, ez);
        sp += h[q];
        sf += ex * ex + ey * ey + ez * ez;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        sp += __shfl_xor(sp, o);
        sf += __shfl_xor(sf, o);
      }
      if ((threadIdx.x & 63) == 0) { s_red[0][threadIdx.x >> 6] = sp; s_red[1][threadIdx.x >> 6] = sf; }
      __syncthreads();
      if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { a += s_red[0][w]; b += s_red[1][w]; }
        double* r = hist + ((size_t)inst * kHistCap + row) * 8;
        r[5] = a / ncell;
        r[6] = sqrt(b / ncell);
      }
    }
  }
  // the interval is complete: the refill plan has read the counter
  if (advance && c == 0 && inst == 0) {
    ctl[CTL_INTERVAL] += 1u;
    ctl[CTL_WINDOW] += 1u;
  }
  if (c >= ncell) return;
  double ex, ey, ez;
  cell_field(g, I, h, c, ex, ey, ez);
  const size_t o = ((size_t)inst * ncell + c) * 4;
  field64[o + 0] = ex; field64[o + 1] = ey; field64[o + 2] = ez; field64[o + 3] = 0.0;
  field32[o + 0] = (float)ex; field32[o + 1] = (float)ey; field32[o + 2] = (float)ez; field32[o + 3] = 0.0f;
}

// Bulk observables: per-tile partial sums in a fixed reduction order.
template <typename T>
__global__ void __launch_bounds__(256) k_bulk_partial(const TileDesc* __restrict__ tiles, const T* __restrict__ kx,
                                                      const T* __restrict__ ky, const T* __restrict__ kz,
                                                      const uint32_t* __restrict__ meta, Mat<T> M, double* bpart,
                                                      uint32_t* ctl, int advance) {
  __shared__ double s[8][256];
  const TileDesc td = tiles[blockIdx.x];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < td.count; i += 256) {
    const long long p = td.start + i;
    const uint32_t mt = meta[p];
    if (!(mt & kAlive)) continue;
    const int v = meta_valley(mt);
    const double x = (double)kx[p], y = (double)ky[p], z = (double)kz[p];
    const double k2 = x * x + y * y + z * z;
    const double m = (double)M.m[v], al = (double)M.alpha[v];
    const double gam = (double)M.ck * k2 / m;
    const double E = 2.0 * gam / (1.0 + sqrt(1.0 + 4.0 * al * gam));
    const double sv = (double)M.cv / (m * (1.0 + 2.0 * al * E));
    acc[0] += 1.0;
    acc[1] += sv * x; acc[2] += sv * y; acc[3] += sv * z;
    acc[4] += E;
    acc[5 + v] += 1.0;
  }
  for (int q = 0; q < 8; ++q) s[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o)
      for (int q = 0; q < 8; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 8) bpart[(size_t)blockIdx.x * 8 + threadIdx.x] = s[threadIdx.x][0];
  if (advance && blockIdx.x == 0 && threadIdx.x == 0) {
    ctl[CTL_INTERVAL] += 1u;
    ctl[CTL_WINDOW] += 1u;
  }
}

__global__ void k_bulk_reduce(const InstParams* __restrict__ ip, const double* __restrict__ bpart, double* hist,
                              int hist_cap, const uint32_t* ctl) {
  const int inst = blockIdx.x;
  const int q = threadIdx.x;
  if (q >= 8) return;
  const int row = (int)ctl[CTL_WINDOW] - 1;
  if (row < 0 || row >= hist_cap) return;
  double s = 0.0;
  for (int t = ip[inst].t0; t < ip[inst].t1; ++t) s += bpart[(size_t)t * 8 + q];
  hist[((size_t)inst * hist_cap + row) * 8 + q] = s;
}

__global__ void k_zero_window(unsigned long long* heat, unsigned long long* dens, unsigned long long* counters,
                              size_t nheat, size_t ndens, int n_inst, uint32_t* ctl) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nheat) heat[i] = 0ull;
  if (i < ndens) dens[i] = 0ull;
  if (i < (size_t)n_inst * kNCnt) counters[i] = 0ull;
  if (i == 0) ctl[CTL_WINDOW] = 0u;
}

}  // namespace gfmc
