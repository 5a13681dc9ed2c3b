// gfmc.hip -- host side of libgfmc.so: the C ABI declared in include/gfmc.h.
// Validates configurations, carves the caller's workspace, sequences the
// kernels of one flight interval on the caller's stream (optionally replayed
// from a captured hipGraph), and copies tallies back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/gfmc.h"
#include "gfmc_kernels.h"
#include "gfmc_refresh.h"

using namespace gfmc;

namespace {

struct Layout {
  size_t total = 0;
  std::vector<std::pair<size_t, size_t>> kept;  // regions a checkpoint carries: (offset, bytes)
  size_t take(size_t bytes) {
    const size_t off = total;
    total += (bytes + 255) & ~(size_t)255;
    return off;
  }
  // a region of evolving state (carried by checkpoints)
  size_t keep(size_t bytes) {
    const size_t off = take(bytes);
    if (bytes) kept.emplace_back(off, bytes);
    return off;
  }
};

struct Offsets {
  size_t table64, table32, fac64, fac32, field64, field32, phi, gamma64, gamma32, Tcell, count, heat, dens,
      counters, flags, ctl, next_id, ip, tiles, acc, tile_dead, tile_off, plan, slots, minv, ainv, rhs, hist, reps,
      nrep, bpart, wg_inst, share_prev;
  size_t kx, ky, kz, x, y, z, meta;
  size_t skx, sky, skz, sx, sy, sz, smeta;  // compaction scratch (device mode)
  std::vector<std::pair<size_t, size_t>> kept;  // evolving state: the regions a checkpoint carries
};

bool same_shared(const mc_config& a, const mc_config& b) {
  if (a.mode != b.mode || a.prec != b.prec || a.dt_fs != b.dt_fs || a.substeps != b.substeps ||
      a.n_bins != b.n_bins || a.dE_eV != b.dE_eV)
    return false;
  if (std::memcmp(&a.mat, &b.mat, sizeof(mc_material)) != 0) return false;
  if (a.mode == MC_DEVICE) {
    for (int d = 0; d < 3; ++d)
      if (a.L_nm[d] != b.L_nm[d] || a.n_cells[d] != b.n_cells[d]) return false;
    if (a.gate_x_nm[0] != b.gate_x_nm[0] || a.gate_x_nm[1] != b.gate_x_nm[1]) return false;
  }
  return true;
}

// Validate; returns an empty string when the configurations are usable.
std::string validate(const mc_config* c, int n) {
  if (!c || n <= 0) return "no configurations";
  for (int i = 0; i < n; ++i) {
    const mc_config& k = c[i];
    if (k.mode != MC_BULK && k.mode != MC_DEVICE) return "mode";
    if (k.prec != MC_PREC_FP64 && k.prec != MC_PREC_FP32_STATE) return "precision";
    if (k.n_particles <= 0 || k.capacity < k.n_particles) return "capacity < n_particles";
    if (!(k.dt_fs > 0.0) || k.substeps <= 0) return "dt and substeps must be positive";
    if (k.n_bins <= 0 || !(k.dE_eV > 0.0) || k.n_bins * k.dE_eV < 3.0 - 1e-9) return "table top below 3 eV";
    if (!(k.T0_K > 0.0) || !(k.T_init_K > 0.0) || !(k.N_D_m3 > 0.0)) return "temperature and doping must be positive";
    if (k.instance >= (1u << 27)) return "instance index too large";
    for (int v = 0; v < 3; ++v)
      if (!(k.mat.m_eff[v] > 0.0) || k.mat.alpha[v] < 0.0 || k.mat.Z[v] < 1) return "material";
    if (k.mode == MC_DEVICE) {
      const int P = k.n_cells[1] * k.n_cells[2];
      if (k.n_cells[0] < 2 || k.n_cells[1] < 1 || k.n_cells[2] < 1 || P > 32) return "grid (ny*nz <= 32, nx >= 2)";
      if ((long long)k.n_cells[0] * P > 4096) return "grid larger than 4096 subcells";
      if (2 * P > 64) return "grid";
      for (int d = 0; d < 3; ++d)
        if (!(k.L_nm[d] > 0.0)) return "domain size";
    }
    if (i > 0 && !same_shared(c[0], k)) return "instances differ in shared parameters";
  }
  return "";
}

int ncell_of(const mc_config& c) { return c.mode == MC_DEVICE ? c.n_cells[0] * c.n_cells[1] * c.n_cells[2] : 1; }

struct TilePlan {
  std::vector<TileDesc> tiles;
  std::vector<int> t0, t1;
};

TilePlan make_tiles(const mc_config* c, int n, int tile) {
  TilePlan tp;
  long long base = 0;
  for (int i = 0; i < n; ++i) {
    tp.t0.push_back((int)tp.tiles.size());
    for (int s = 0; s < c[i].capacity; s += tile) {
      TileDesc d;
      d.inst = i;
      d.count = std::min(tile, c[i].capacity - s);
      d.start = base + s;
      tp.tiles.push_back(d);
    }
    tp.t1.push_back((int)tp.tiles.size());
    base += c[i].capacity;
  }
  return tp;
}

int min_tile(const mc_config& c) { return c.mode == MC_DEVICE ? 1024 : 256; }

Offsets layout(const mc_config* c, int n, size_t* total) {
  Layout L;
  Offsets o;
  const int nb = c[0].n_bins, nc = ncell_of(c[0]);
  const bool dev = c[0].mode == MC_DEVICE;
  const bool f32 = c[0].prec == MC_PREC_FP32_STATE;
  size_t cap = 0;
  for (int i = 0; i < n; ++i) cap += (size_t)c[i].capacity;
  const size_t max_tiles = make_tiles(c, n, min_tile(c[0])).tiles.size();
  // keep(): state that evolves or that the caller may replace (tables); the
  // rest is rebuilt at set-up or rewritten within every interval
  o.table64 = L.keep(sizeof(double) * 3 * nb * kTRow);
  o.table32 = L.keep(sizeof(float) * 3 * nb * kTRow);
  o.fac64 = L.keep(sizeof(double) * n * nc * kFRow);
  o.fac32 = L.keep(sizeof(float) * n * nc * kFRow);
  o.field64 = L.keep(sizeof(double) * n * nc * 4);
  o.field32 = L.keep(sizeof(float) * n * nc * 4);
  o.phi = L.keep(sizeof(double) * n * nc);
  o.gamma64 = L.keep(sizeof(double) * n * 4);
  o.gamma32 = L.keep(sizeof(float) * n * 4);
  o.Tcell = L.keep(sizeof(double) * n * nc);
  o.count = L.keep(sizeof(uint32_t) * n * nc);
  o.heat = L.keep(sizeof(unsigned long long) * n * nc * 4);
  o.dens = L.keep(sizeof(unsigned long long) * n * nc);
  o.counters = L.keep(sizeof(unsigned long long) * n * kNCnt);
  o.flags = L.keep(sizeof(int) * n);
  o.ctl = L.keep(sizeof(uint32_t) * 16);
  o.next_id = L.keep(sizeof(uint32_t) * n);
  o.ip = L.take(sizeof(InstParams) * n);
  o.tiles = L.take(sizeof(TileDesc) * max_tiles);
  o.acc = L.keep(dev ? sizeof(unsigned long long) * n * 5 * nc : 0);
  o.tile_dead = L.take(sizeof(uint32_t) * max_tiles);
  o.tile_off = L.take(sizeof(uint32_t) * max_tiles);
  o.wg_inst = L.take(sizeof(int) * max_tiles);
  o.share_prev = L.take(sizeof(unsigned long long) * (n + 1));  // previous segment counts, valid flag
  o.plan = L.keep(sizeof(Plan) * n);
  o.slots = L.take(dev ? sizeof(uint32_t) * cap : 0);  // contact-refill slot list
  o.minv = L.take(dev ? sizeof(double) * c[0].n_cells[0] * (size_t)(c[0].n_cells[1] * c[0].n_cells[2]) *
                            (c[0].n_cells[1] * c[0].n_cells[2])
                      : 0);
  o.ainv = L.take(dev ? sizeof(double) * (size_t)nc * nc : 0);
  o.rhs = L.take(dev ? sizeof(double) * (size_t)n * nc : 0);
  o.hist = L.keep(sizeof(double) * n * kHistCap * 8);
  o.reps = L.keep(sizeof(int) * n * nc);
  o.nrep = L.keep(sizeof(int) * n);
  o.bpart = L.take(dev ? 0 : sizeof(double) * max_tiles * 8);
  const size_t es = f32 ? 4 : 8;
  o.kx = L.keep(es * cap);
  o.ky = L.keep(es * cap);
  o.kz = L.keep(es * cap);
  o.x = L.keep(dev ? es * cap : 0);
  o.y = L.keep(dev ? es * cap : 0);
  o.z = L.keep(dev ? es * cap : 0);
  o.meta = L.keep(sizeof(uint32_t) * cap);
  o.skx = L.take(dev ? es * cap : 0);
  o.sky = L.take(dev ? es * cap : 0);
  o.skz = L.take(dev ? es * cap : 0);
  o.sx = L.take(dev ? es * cap : 0);
  o.sy = L.take(dev ? es * cap : 0);
  o.sz = L.take(dev ? es * cap : 0);
  o.smeta = L.take(dev ? sizeof(uint32_t) * cap : 0);
  o.kept = L.kept;
  *total = L.total;
  return o;
}

}  // namespace

struct mc_ctx {
  std::vector<mc_config> cfg;
  int n_inst = 0;
  bool dev = false, f32 = false;
  hipStream_t st = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Offsets o;
  int nb = 0, ncell = 1, nx = 1, ny = 1, nz = 1, P = 1;
  int block = 256, tile = 0, n_tiles = 0;
  int max_tiles = 0;        // tiles at the smallest tile size: per-tile entries the workspace holds
  long long max_cap = 0;    // largest instance capacity
  // persistent kernels: workgroups, slots per chunk (128: one staged piece;
  // 256 was 1-2% slower and 64 4% slower, 512 and 1024 left the workgroups
  // unevenly loaded)
  int n_wg = 0, chunk = 128;
  unsigned inj_blocks = 0;  // refill grid: covers the most electrons one instance can need
  size_t total_cap = 0;
  std::vector<long long> base;
  std::vector<InstParams> ip;
  std::vector<std::vector<double>> Tcell;
  Mat<double> M64;
  Mat<float> M32;
  Geo<double> G64;
  Geo<float> G32;
  PoisGeo pg;
  double ck = 0.0;
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  int variant = 0;  // 0: lane refill, 1: one electron per lane, 2: persistent
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;   // triples: before flight, after flight, after refresh
  size_t ev_used = 0;
  std::string err;
  template <typename T> T* p(size_t off) { return reinterpret_cast<T*>(ws + off); }
};

namespace {

int fail(mc_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail((ctx), MC_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

void mats(mc_ctx* c) {
  const mc_material& m = c->cfg[0].mat;
  c->ck = kHbar * kHbar / (2.0 * kMe * kQ) * 1e18;
  const double cv = kHbar / kMe * 1e3, cf = kQ / kHbar * 1e-15;
  for (int v = 0; v < 3; ++v) {
    c->M64.m[v] = m.m_eff[v]; c->M64.alpha[v] = m.alpha[v]; c->M64.Ec[v] = m.E_c[v];
    c->M32.m[v] = (float)m.m_eff[v]; c->M32.alpha[v] = (float)m.alpha[v]; c->M32.Ec[v] = (float)m.E_c[v];
  }
  c->M64.hw_lo = m.hw_lo_eV; c->M64.hw_iv = m.hw_iv_eV; c->M64.ck = c->ck; c->M64.cv = cv; c->M64.cf = cf;
  c->M32.hw_lo = (float)m.hw_lo_eV; c->M32.hw_iv = (float)m.hw_iv_eV; c->M32.ck = (float)c->ck;
  c->M32.cv = (float)cv; c->M32.cf = (float)cf;
  const mc_config& k = c->cfg[0];
  c->G64.nx = c->nx; c->G64.ny = c->ny; c->G64.nz = c->nz; c->G64.ncell = c->ncell;
  c->G32.nx = c->nx; c->G32.ny = c->ny; c->G32.nz = c->nz; c->G32.ncell = c->ncell;
  for (int d = 0; d < 3; ++d) {
    const double L = c->dev ? k.L_nm[d] : 1.0;
    const int n = c->dev ? k.n_cells[d] : 1;
    c->G64.L[d] = L; c->G64.d[d] = L / n; c->G64.inv_d[d] = n / L;
    c->G32.L[d] = (float)L; c->G32.d[d] = (float)(L / n); c->G32.inv_d[d] = (float)(n / L);
  }
  if (c->dev) {
    PoisGeo& g = c->pg;
    g.nx = c->nx; g.ny = c->ny; g.nz = c->nz; g.P = c->P;
    g.dx = k.L_nm[0] / c->nx; g.dy = k.L_nm[1] / c->ny; g.dz = k.L_nm[2] / c->nz;
    const double eps = m.eps_s * kEps0 * 1e-9;
    g.gx = eps * g.dy * g.dz / g.dx; g.gy = eps * g.dx * g.dz / g.dy; g.gz = eps * g.dx * g.dy / g.dz;
    g.gate0 = k.gate_x_nm[0]; g.gate1 = k.gate_x_nm[1];
    g.Vc = g.dx * g.dy * g.dz;
  }
}

int flight_occupancy(mc_ctx* c, int variant, int block, int* wg_per_cu, int* n_cu);

// Tiles of the current tile size, and for the persistent kernel the chunks of
// each instance (chunks never straddle a tile) and its share of the
// workgroups the GPU holds at once (at least one each, in proportion to the
// chunks, at most one per chunk).
int upload_tiles(mc_ctx* c) {
  TilePlan tp = make_tiles(c->cfg.data(), c->n_inst, c->tile);
  c->n_tiles = (int)tp.tiles.size();
  const int cpt = (c->tile + c->chunk - 1) / c->chunk;
  long long tot = 0;
  for (int i = 0; i < c->n_inst; ++i) {
    InstParams& I = c->ip[i];
    I.t0 = tp.t0[i];
    I.t1 = tp.t1[i];
    const int nt = I.t1 - I.t0, last = I.cap - (nt - 1) * c->tile;
    I.nchunk = (nt - 1) * cpt + (last + c->chunk - 1) / c->chunk;
    tot += I.nchunk;
  }
  int wg = c->n_inst;
  if (c->variant >= 2) {
    int per = 0, ncu = 0, rc;
    if ((rc = flight_occupancy(c, c->variant, c->block, &per, &ncu)) != MC_OK) return rc;
    if (per < 1) return fail(c, MC_E_ARG, "persistent kernel does not fit this workgroup size");
    wg = std::max(c->n_inst, std::min(per * ncu, c->max_tiles));
  }
  // no workgroup may own more than kMaxTile slots (16-bit packed deposit)
  const int max_chunks = kMaxTile / c->chunk;
  std::vector<int> wg_inst;
  for (int i = 0; i < c->n_inst; ++i) {
    InstParams& I = c->ip[i];
    long long share = 1 + (long long)(wg - c->n_inst) * I.nchunk / std::max(1LL, tot);
    share = std::max<long long>(share, (I.nchunk + max_chunks - 1) / max_chunks);
    I.w0 = (int)wg_inst.size();
    I.w1 = I.w0 + (int)std::min<long long>(share, I.nchunk);
    wg_inst.resize(I.w1, i);
  }
  if ((int)wg_inst.size() > c->max_tiles) return fail(c, MC_E_ARG, "persistent grid exceeds the workgroup table");
  c->n_wg = (int)wg_inst.size();
  HIPCHK(c, hipMemcpyAsync(c->ws + c->o.tiles, tp.tiles.data(), sizeof(TileDesc) * tp.tiles.size(),
                           hipMemcpyHostToDevice, c->st));
  // the work-proportional shares start again from these slot shares
  HIPCHK(c, hipMemsetAsync(c->ws + c->o.share_prev, 0, sizeof(unsigned long long) * (c->n_inst + 1), c->st));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->o.wg_inst, wg_inst.data(), sizeof(int) * wg_inst.size(), hipMemcpyHostToDevice,
                           c->st));
  // free-slot counts start from zero under the new tiling
  HIPCHK(c, hipMemsetAsync(c->ws + c->o.tile_dead, 0, sizeof(uint32_t) * c->max_tiles, c->st));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->o.ip, c->ip.data(), sizeof(InstParams) * c->n_inst, hipMemcpyHostToDevice,
                           c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return MC_OK;
}

void drop_graph(mc_ctx* c) {
  if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
}

// factors and Gamma_v of every instance from the host temperature maps
int refresh_rates(mc_ctx* c) {
  std::vector<double> T((size_t)c->n_inst * c->ncell);
  std::vector<int> reps((size_t)c->n_inst * c->ncell, 0), nrep(c->n_inst, 0);
  for (int i = 0; i < c->n_inst; ++i) {
    std::map<double, int> seen;
    for (int q = 0; q < c->ncell; ++q) {
      const double t = c->Tcell[i][q];
      T[(size_t)i * c->ncell + q] = t;
      if (seen.emplace(t, q).second) reps[(size_t)i * c->ncell + nrep[i]++] = q;
    }
  }
  HIPCHK(c, hipMemcpyAsync(c->ws + c->o.Tcell, T.data(), sizeof(double) * T.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->o.reps, reps.data(), sizeof(int) * reps.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->o.nrep, nrep.data(), sizeof(int) * nrep.size(), hipMemcpyHostToDevice, c->st));
  const mc_material& m = c->cfg[0].mat;
  dim3 gf((c->ncell + 255) / 256, c->n_inst);
  k_factors<<<gf, 256, 0, c->st>>>(c->p<double>(c->o.Tcell), c->p<InstParams>(c->o.ip), c->ncell, m.eps_s,
                                   m.hw_lo_eV, m.hw_iv_eV, c->p<double>(c->o.fac64), c->p<float>(c->o.fac32));
  // Gamma_v as maxima over chunks of distinct subcells (zeroed first; this
  // runs outside any graph capture)
  HIPCHK(c, hipMemsetAsync(c->ws + c->o.gamma64, 0, sizeof(double) * 4 * c->n_inst, c->st));
  HIPCHK(c, hipMemsetAsync(c->ws + c->o.gamma32, 0, sizeof(float) * 4 * c->n_inst, c->st));
  dim3 gg(c->n_inst, 3, (c->ncell + kGammaReps - 1) / kGammaReps);
  k_gamma<double><<<gg, 256, 0, c->st>>>(c->p<double>(c->o.table64), c->p<double>(c->o.fac64), c->p<int>(c->o.reps),
                                         c->p<int>(c->o.nrep), c->ncell, c->nb, c->p<double>(c->o.gamma64));
  k_gamma<float><<<gg, 256, 0, c->st>>>(c->p<float>(c->o.table32), c->p<float>(c->o.fac32), c->p<int>(c->o.reps),
                                        c->p<int>(c->o.nrep), c->ncell, c->nb, c->p<float>(c->o.gamma32));
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->st));
  return MC_OK;
}

template <typename T>
FlightArgs<T> flight_args(mc_ctx* c, const Mat<T>& M, const Geo<T>& G, size_t tab, size_t fac, size_t field,
                          size_t gam) {
  FlightArgs<T> a;
  a.tiles = c->p<TileDesc>(c->o.tiles);
  a.ip = c->p<InstParams>(c->o.ip);
  a.table = c->p<T>(tab);
  a.fac = c->p<T>(fac);
  a.field = c->p<T>(field);
  a.gamma = c->p<T>(gam);
  a.kx = c->p<T>(c->o.kx); a.ky = c->p<T>(c->o.ky); a.kz = c->p<T>(c->o.kz);
  a.x = c->p<T>(c->o.x); a.y = c->p<T>(c->o.y); a.z = c->p<T>(c->o.z);
  a.meta = c->p<uint32_t>(c->o.meta);
  a.acc = c->p<unsigned long long>(c->o.acc);
  a.tile_dead = c->p<uint32_t>(c->o.tile_dead);
  a.counters = c->p<unsigned long long>(c->o.counters);
  a.flags = c->p<int>(c->o.flags);
  a.ctl = c->p<uint32_t>(c->o.ctl);
  a.wg_inst = c->p<int>(c->o.wg_inst);
  a.plan = c->p<Plan>(c->o.plan);
  a.tile = c->tile;
  a.chunk = c->chunk;
  a.n_inst = c->n_inst;
  // the Infinity Cache (256 MB) over the state bytes per slot
  a.nt_slots = (uint32_t)((256ull << 20) / (6 * sizeof(T) + sizeof(uint32_t)));
  a.M = M;
  a.G = G;
  a.nb = c->nb;
  a.dE = (T)c->cfg[0].dE_eV;
  a.TP = (T)(c->cfg[0].dt_fs * c->cfg[0].substeps);
  return a;
}

template <typename T>
StateArrays<T> state_arrays(mc_ctx* c, bool scratch) {
  const Offsets& o = c->o;
  StateArrays<T> a;
  a.kx = c->p<T>(scratch ? o.skx : o.kx); a.ky = c->p<T>(scratch ? o.sky : o.ky); a.kz = c->p<T>(scratch ? o.skz : o.kz);
  a.x = c->p<T>(scratch ? o.sx : o.x); a.y = c->p<T>(scratch ? o.sy : o.y); a.z = c->p<T>(scratch ? o.sz : o.z);
  a.meta = c->p<uint32_t>(scratch ? o.smeta : o.meta);
  return a;
}

// Stable compaction of the instances whose plan asks for it (the tiles of
// the other instances return at once): the gather into the scratch arrays,
// then, per tile, the copy back and the free-slot list.
template <typename T>
void enqueue_compaction_and_slots(mc_ctx* c) {
  const StateArrays<T> st = state_arrays<T>(c, false), scr = state_arrays<T>(c, true);
  k_compact_scatter<T><<<c->n_tiles, 256, 0, c->st>>>(c->p<TileDesc>(c->o.tiles), c->p<InstParams>(c->o.ip),
                                                       c->p<Plan>(c->o.plan), c->p<uint32_t>(c->o.tile_off),
                                                       c->p<uint32_t>(c->o.tile_dead), st, scr);
  k_inject_slots<T><<<c->n_tiles, 256, 0, c->st>>>(c->p<TileDesc>(c->o.tiles), c->p<InstParams>(c->o.ip),
                                                    c->p<Plan>(c->o.plan), c->p<uint32_t>(c->o.tile_off),
                                                    c->p<uint32_t>(c->o.tile_dead), st, scr,
                                                    c->p<uint32_t>(c->o.slots));
}

// deposit (or merged flight histogram), contact refill, Poisson, field
void enqueue_refresh(mc_ctx* c, bool after_flight) {
  const int nc = c->ncell;
  // merged counts and heat, refill plan and Poisson right-hand side:
  // workgroup 0 of each instance plans the refill, the others take the bins
  const int af = after_flight ? 1 : 0;
  dim3 gpl(1 + (5 * nc + kPlanThreads - 1) / kPlanThreads, c->n_inst);
  k_inject_plan<<<gpl, kPlanThreads, 0, c->st>>>(
      c->p<InstParams>(c->o.ip), c->p<TileDesc>(c->o.tiles), c->p<uint32_t>(c->o.meta), c->pg, nc,
      c->p<unsigned long long>(c->o.acc), c->p<uint32_t>(c->o.count), c->p<unsigned long long>(c->o.heat), af,
      c->p<uint32_t>(c->o.tile_dead), c->p<uint32_t>(c->o.tile_off), c->p<Plan>(c->o.plan),
      c->p<uint32_t>(c->o.next_id), c->p<unsigned long long>(c->o.counters), c->p<int>(c->o.flags),
      c->p<uint32_t>(c->o.ctl), c->p<double>(c->o.rhs), c->p<unsigned long long>(c->o.dens),
      c->p<double>(c->o.hist));
  if (c->f32) enqueue_compaction_and_slots<float>(c);
  else enqueue_compaction_and_slots<double>(c);
  const double mg1 = c->cfg[0].mat.m_eff[0];
  if (c->inj_blocks > 0) {
    dim3 gi(c->inj_blocks, c->n_inst);
    if (c->f32)
      k_inject_fill<float><<<gi, 256, 0, c->st>>>(c->p<InstParams>(c->o.ip), c->p<Plan>(c->o.plan),
                                                  c->p<uint32_t>(c->o.slots), c->p<double>(c->o.Tcell), c->G32, mg1,
                                                  c->ck, c->p<float>(c->o.kx), c->p<float>(c->o.ky),
                                                  c->p<float>(c->o.kz), c->p<float>(c->o.x), c->p<float>(c->o.y),
                                                  c->p<float>(c->o.z), c->p<uint32_t>(c->o.meta));
    else
      k_inject_fill<double><<<gi, 256, 0, c->st>>>(c->p<InstParams>(c->o.ip), c->p<Plan>(c->o.plan),
                                                   c->p<uint32_t>(c->o.slots), c->p<double>(c->o.Tcell), c->G64, mg1,
                                                   c->ck, c->p<double>(c->o.kx), c->p<double>(c->o.ky),
                                                   c->p<double>(c->o.kz), c->p<double>(c->o.x), c->p<double>(c->o.y),
                                                   c->p<double>(c->o.z), c->p<uint32_t>(c->o.meta));
  }
  dim3 gc((nc + 255) / 256, c->n_inst);
  if (c->n_inst == 1) {
    dim3 gv((nc + 3) / 4, 1);
    k_poisson_gemv<<<gv, 256, 0, c->st>>>(c->p<double>(c->o.ainv), c->p<double>(c->o.rhs), nc,
                                          c->p<double>(c->o.phi));
  } else {
    // 4 rows x 8 instances per wavefront: 2 rows x 16 instances halves the
    // passes over the inverse but doubles the loads of the right-hand sides,
    // and was slower (73 against 57 us for 64 instances)
    dim3 gg(((nc + 3) / 4 + 3) / 4, (c->n_inst + 7) / 8);
    k_poisson_gemm<4, 8, 4><<<gg, 256, 0, c->st>>>(c->p<double>(c->o.ainv), c->p<double>(c->o.rhs), nc, c->n_inst,
                                                   c->p<double>(c->o.phi));
  }
  k_field<<<gc, 256, 0, c->st>>>(c->pg, c->p<InstParams>(c->o.ip), c->p<double>(c->o.phi), nc,
                                 c->p<double>(c->o.field64), c->p<float>(c->o.field32), c->p<uint32_t>(c->o.ctl), af,
                                 c->p<Plan>(c->o.plan), c->p<double>(c->o.hist));
}

hipEvent_t prof_event(mc_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// LDS of a particle-kernel workgroup: the histogram (every variant), and
// for variant 3 each wavefront's two staged pieces of slots
size_t flight_lds_bytes(const mc_ctx* c, int variant, int block) {
  size_t b = sizeof(uint32_t) * flight_lds_words(c->ncell);
  if (variant == 3) b += (size_t)(block / 64) * 2 * (c->f32 ? piece_bytes<float>() : piece_bytes<double>());
  return b;
}

template <typename T>
void launch_flight(mc_ctx* c, const FlightArgs<T>& a) {
  const size_t lds = flight_lds_bytes(c, c->variant, c->block);
  if (c->variant == 3) {
    if (c->dev) k_flight_persist_staged<T, true><<<c->n_wg, c->block, lds, c->st>>>(a);
    else k_flight_persist_staged<T, false><<<c->n_wg, c->block, lds, c->st>>>(a);
  } else if (c->variant == 2) {
    if (c->dev) k_flight_persist<T, true><<<c->n_wg, c->block, lds, c->st>>>(a);
    else k_flight_persist<T, false><<<c->n_wg, c->block, lds, c->st>>>(a);
  } else if (c->variant == 0) {
    if (c->dev) k_flight_refill<T, true><<<c->n_tiles, c->block, lds, c->st>>>(a);
    else k_flight_refill<T, false><<<c->n_tiles, c->block, lds, c->st>>>(a);
  } else {
    if (c->dev) k_flight<T, true><<<c->n_tiles, c->block, lds, c->st>>>(a);
    else k_flight<T, false><<<c->n_tiles, c->block, lds, c->st>>>(a);
  }
}

template <typename T>
hipError_t occupancy_of(const mc_ctx* c, int variant, int block, int* n) {
  const size_t lds = flight_lds_bytes(c, variant, block);
  if (variant == 3)
    return c->dev ? hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_flight_persist_staged<T, true>, block, lds)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_flight_persist_staged<T, false>, block, lds);
  if (variant == 2)
    return c->dev ? hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_flight_persist<T, true>, block, lds)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_flight_persist<T, false>, block, lds);
  if (variant == 0)
    return c->dev ? hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_flight_refill<T, true>, block, lds)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_flight_refill<T, false>, block, lds);
  return c->dev ? hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_flight<T, true>, block, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_flight<T, false>, block, lds);
}

// Workgroups of the particle kernel (variant, precision of the context) that
// one compute unit holds at once, and the compute units of the current device.
int flight_occupancy(mc_ctx* c, int variant, int block, int* wg_per_cu, int* n_cu) {
  int n = 0;
  HIPCHK(c, c->f32 ? occupancy_of<float>(c, variant, block, &n) : occupancy_of<double>(c, variant, block, &n));
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  HIPCHK(c, hipDeviceGetAttribute(n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  *wg_per_cu = n;
  return MC_OK;
}

void enqueue_interval(mc_ctx* c) {
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
  if (c->profile) {
    e0 = prof_event(c); e1 = prof_event(c); e2 = prof_event(c);
    if (e0) (void)hipEventRecord(e0, c->st);
  }
  // several instances under a persistent kernel: workgroups follow the
  // previous interval's segments
  if (c->variant >= 2 && c->n_inst > 1 && c->n_inst <= kShareMax)
    k_share_work<<<1, 256, 0, c->st>>>(c->p<InstParams>(c->o.ip), c->n_inst, c->p<unsigned long long>(c->o.counters),
                                       c->p<unsigned long long>(c->o.share_prev), c->p<int>(c->o.wg_inst), c->n_wg,
                                       kMaxTile / c->chunk);
  if (c->f32)
    launch_flight<float>(c, flight_args<float>(c, c->M32, c->G32, c->o.table32, c->o.fac32, c->o.field32,
                                               c->o.gamma32));
  else
    launch_flight<double>(c, flight_args<double>(c, c->M64, c->G64, c->o.table64, c->o.fac64, c->o.field64,
                                                 c->o.gamma64));
  if (e1) (void)hipEventRecord(e1, c->st);
  if (c->dev) {
    enqueue_refresh(c, true);
  } else {
    if (c->f32)
      k_bulk_partial<float><<<c->n_tiles, 256, 0, c->st>>>(c->p<TileDesc>(c->o.tiles), c->p<float>(c->o.kx),
                                                           c->p<float>(c->o.ky), c->p<float>(c->o.kz),
                                                           c->p<uint32_t>(c->o.meta), c->M32, c->p<double>(c->o.bpart),
                                                           c->p<uint32_t>(c->o.ctl), 1);
    else
      k_bulk_partial<double><<<c->n_tiles, 256, 0, c->st>>>(c->p<TileDesc>(c->o.tiles), c->p<double>(c->o.kx),
                                                            c->p<double>(c->o.ky), c->p<double>(c->o.kz),
                                                            c->p<uint32_t>(c->o.meta), c->M64,
                                                            c->p<double>(c->o.bpart), c->p<uint32_t>(c->o.ctl), 1);
    k_bulk_reduce<<<c->n_inst, 64, 0, c->st>>>(c->p<InstParams>(c->o.ip), c->p<double>(c->o.bpart),
                                               c->p<double>(c->o.hist), kHistCap, c->p<uint32_t>(c->o.ctl));
  }
  if (e2) (void)hipEventRecord(e2, c->st);
}

}  // namespace

extern "C" {

const char* mc_status_string(int s) {
  switch (s) {
    case MC_OK: return "ok";
    case MC_E_ARG: return "invalid argument";
    case MC_E_HIP: return "HIP runtime error";
    case MC_E_CAPACITY: return "particle capacity or identity space exhausted";
    case MC_E_RANGE: return "event-count guard hit";
    case MC_E_STATE: return "invalid state";
    case MC_E_NAN: return "non-finite particle state";
    default: return "unknown status";
  }
}

const char* mc_last_error(const mc_ctx* c) { return c ? c->err.c_str() : "null context"; }

size_t mc_workspace_bytes(const mc_config* cfgs, int n) {
  if (!validate(cfgs, n).empty()) return 0;
  size_t total = 0;
  layout(cfgs, n, &total);
  return total;
}

int mc_init(mc_ctx** out, const mc_config* cfgs, int n, void* d_ws, size_t ws_bytes, void* stream) {
  if (!out) return MC_E_ARG;
  *out = nullptr;
  const std::string why = validate(cfgs, n);
  if (!why.empty()) return MC_E_ARG;
  size_t need = 0;
  Offsets o = layout(cfgs, n, &need);
  if (!d_ws || ws_bytes < need || ((uintptr_t)d_ws & 255u)) return MC_E_ARG;
  mc_ctx* c = new mc_ctx();
  c->cfg.assign(cfgs, cfgs + n);
  c->n_inst = n;
  c->dev = cfgs[0].mode == MC_DEVICE;
  c->f32 = cfgs[0].prec == MC_PREC_FP32_STATE;
  c->st = (hipStream_t)stream;
  c->ws = (char*)d_ws;
  c->ws_bytes = ws_bytes;
  c->o = o;
  c->nb = cfgs[0].n_bins;
  // variant 3's staged slot pieces take its LDS above the default 64 KB of
  // dynamic shared memory
  {
    const int lds_max = 160 * 1024;
    if (hipFuncSetAttribute((const void*)k_flight_persist_staged<float, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_max) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_flight_persist_staged<float, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_max) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_flight_persist_staged<double, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_max) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_flight_persist_staged<double, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_max) != hipSuccess) {
      delete c;
      return MC_E_HIP;
    }
  }
  if (c->dev) {
    c->nx = cfgs[0].n_cells[0]; c->ny = cfgs[0].n_cells[1]; c->nz = cfgs[0].n_cells[2];
  }
  c->P = c->ny * c->nz;
  c->ncell = c->nx * c->ny * c->nz;
  c->tile = c->dev ? 8192 : 1024;
  c->block = 256;
  c->max_tiles = (int)make_tiles(cfgs, n, min_tile(cfgs[0])).tiles.size();
  for (int i = 0; i < n; ++i) c->max_cap = std::max<long long>(c->max_cap, cfgs[i].capacity);
  mats(c);
  // per-instance parameters
  long long base = 0;
  c->ip.resize(n);
  c->Tcell.assign(n, std::vector<double>(c->ncell, 0.0));
  for (int i = 0; i < n; ++i) {
    const mc_config& k = cfgs[i];
    InstParams& I = c->ip[i];
    std::memset(&I, 0, sizeof(I));
    I.key0 = (uint32_t)(k.seed & 0xffffffffu);
    I.key1 = (uint32_t)(k.seed >> 32);
    I.tagw = k.instance << 4;
    I.cap = k.capacity;
    I.base = base;
    base += k.capacity;
    I.N_D_nm = k.N_D_m3 * 1e-27;
    I.N_D_m3 = k.N_D_m3;
    I.Vgs = k.Vgs; I.Vds = k.Vds; I.phig = k.Vgs + k.phi_offset;
    for (int d = 0; d < 3; ++d) I.F[d] = k.F_bulk[d];
    I.T_init = k.T_init_K;
    if (c->dev) {
      I.w = k.N_D_m3 * 1e-27 * k.L_nm[0] * k.L_nm[1] * k.L_nm[2] / k.n_particles;
      I.target = (int)std::lround(I.N_D_nm * c->pg.Vc / I.w);
    } else {
      I.w = 1.0;
    }
    for (int q = 0; q < c->ncell; ++q) c->Tcell[i][q] = k.T0_K;
  }
  c->total_cap = (size_t)base;
  if (c->dev) {
    // an instance places at most 2P*target electrons (all contact subcells
    // empty) and never more than its free slots
    long long qmax = 0;
    for (int i = 0; i < n; ++i)
      qmax = std::max(qmax, std::min<long long>(cfgs[i].capacity, 2LL * c->P * std::max(0, c->ip[i].target)));
    c->inj_blocks = (unsigned)((qmax + 255) / 256);
  }
  int rc;
  HIPCHK(c, hipMemsetAsync(c->ws, 0, need, c->st));
  if ((rc = upload_tiles(c)) != MC_OK) { *out = c; return rc; }
  // rate tables
  RateMat R;
  const mc_material& m = cfgs[0].mat;
  for (int v = 0; v < 3; ++v) { R.m[v] = m.m_eff[v]; R.alpha[v] = m.alpha[v]; R.Ec[v] = m.E_c[v]; R.Z[v] = m.Z[v]; }
  R.eps_s = m.eps_s; R.eps_inf = m.eps_inf; R.rho = m.rho; R.D_ac = m.D_ac_eV; R.D_iv = m.D_iv_eVm;
  R.hw_lo = m.hw_lo_eV; R.hw_iv = m.hw_iv_eV; R.u_ac = m.u_ac;
  k_tables<<<(3 * c->nb + 255) / 256, 256, 0, c->st>>>(R, c->nb, cfgs[0].dE_eV, c->ck, c->p<double>(o.table64),
                                                      c->p<float>(o.table32));
  HIPCHK(c, hipGetLastError());
  if ((rc = refresh_rates(c)) != MC_OK) { *out = c; return rc; }
  // bulk field: a single cell holding the uniform field
  if (!c->dev) {
    std::vector<double> f64((size_t)n * 4, 0.0);
    std::vector<float> f32((size_t)n * 4, 0.0f);
    for (int i = 0; i < n; ++i)
      for (int d = 0; d < 3; ++d) { f64[i * 4 + d] = cfgs[i].F_bulk[d]; f32[i * 4 + d] = (float)cfgs[i].F_bulk[d]; }
    HIPCHK(c, hipMemcpyAsync(c->ws + o.field64, f64.data(), sizeof(double) * f64.size(), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->ws + o.field32, f32.data(), sizeof(float) * f32.size(), hipMemcpyHostToDevice, c->st));
  }
  // ensembles
  std::vector<uint32_t> nid(n);
  for (int i = 0; i < n; ++i) {
    nid[i] = (uint32_t)cfgs[i].n_particles;
    const int grid = (cfgs[i].capacity + 255) / 256;
    if (c->f32) {
      if (c->dev)
        k_init<float, true><<<grid, 256, 0, c->st>>>(c->p<InstParams>(o.ip), i, c->G32, m.m_eff[0], c->ck,
                                                     c->p<float>(o.kx), c->p<float>(o.ky), c->p<float>(o.kz),
                                                     c->p<float>(o.x), c->p<float>(o.y), c->p<float>(o.z),
                                                     c->p<uint32_t>(o.meta), cfgs[i].n_particles);
      else
        k_init<float, false><<<grid, 256, 0, c->st>>>(c->p<InstParams>(o.ip), i, c->G32, m.m_eff[0], c->ck,
                                                      c->p<float>(o.kx), c->p<float>(o.ky), c->p<float>(o.kz),
                                                      nullptr, nullptr, nullptr, c->p<uint32_t>(o.meta),
                                                      cfgs[i].n_particles);
    } else {
      if (c->dev)
        k_init<double, true><<<grid, 256, 0, c->st>>>(c->p<InstParams>(o.ip), i, c->G64, m.m_eff[0], c->ck,
                                                      c->p<double>(o.kx), c->p<double>(o.ky), c->p<double>(o.kz),
                                                      c->p<double>(o.x), c->p<double>(o.y), c->p<double>(o.z),
                                                      c->p<uint32_t>(o.meta), cfgs[i].n_particles);
      else
        k_init<double, false><<<grid, 256, 0, c->st>>>(c->p<InstParams>(o.ip), i, c->G64, m.m_eff[0], c->ck,
                                                       c->p<double>(o.kx), c->p<double>(o.ky), c->p<double>(o.kz),
                                                       nullptr, nullptr, nullptr, c->p<uint32_t>(o.meta),
                                                       cfgs[i].n_particles);
    }
  }
  // the initial electrons fill the slots [0, N) of each instance
  for (int i = 0; i < n; ++i) k_set_hw<<<1, 64, 0, c->st>>>(c->p<Plan>(o.plan), i, (uint32_t)cfgs[i].n_particles);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->ws + o.next_id, nid.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, c->st));
  if (c->dev) {
    k_poisson_factor<<<1, 256, 0, c->st>>>(c->pg, c->p<double>(o.minv));
    k_poisson_inverse<<<c->ncell, 64, sizeof(double) * 2 * c->ncell, c->st>>>(c->pg, c->p<double>(o.minv), c->ncell,
                                                                             c->p<double>(o.ainv));
    HIPCHK(c, hipGetLastError());
    *out = c;
    if ((rc = poisson_update(c)) != MC_OK) return rc;
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  *out = c;
  return MC_OK;
}

int mc_destroy(mc_ctx* c) {
  if (!c) return MC_E_ARG;
  drop_graph(c);
  (void)hipStreamSynchronize(c->st);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
  return MC_OK;
}

int mc_set_lattice_temperature(mc_ctx* c, int inst, const double* h_T) {
  if (!c || inst < 0 || inst >= c->n_inst || !h_T) return fail(c, MC_E_ARG, "bad argument");
  for (int q = 0; q < c->ncell; ++q)
    if (!(h_T[q] > 0.0)) return fail(c, MC_E_ARG, "temperatures must be positive");
  c->Tcell[inst].assign(h_T, h_T + c->ncell);
  return refresh_rates(c);
}

int mc_set_tables(mc_ctx* c, const double* h_shape, const double* h_k4) {
  if (!c || !h_shape || !h_k4) return fail(c, MC_E_ARG, "bad argument");
  std::vector<double> t64((size_t)3 * c->nb * kTRow, 0.0);
  std::vector<float> t32(t64.size(), 0.0f);
  for (int v = 0; v < 3; ++v)
    for (int b = 0; b < c->nb; ++b) {
      const size_t r = (size_t)v * c->nb + b;
      for (int m = 0; m < kNM; ++m) t64[r * kTRow + m] = h_shape[r * kNM + m];
      t64[r * kTRow + 10] = h_k4[r];
    }
  for (size_t i = 0; i < t64.size(); ++i) t32[i] = (float)t64[i];
  HIPCHK(c, hipMemcpyAsync(c->ws + c->o.table64, t64.data(), sizeof(double) * t64.size(), hipMemcpyHostToDevice,
                           c->st));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->o.table32, t32.data(), sizeof(float) * t32.size(), hipMemcpyHostToDevice,
                           c->st));
  return refresh_rates(c);
}

int mc_step(mc_ctx* c, int n_substeps) {
  if (!c) return MC_E_ARG;
  const int K = c->cfg[0].substeps;
  if (n_substeps < 0 || n_substeps % K) return fail(c, MC_E_ARG, "n_substeps must be a multiple of substeps");
  const int n = n_substeps / K;
  if (c->block > 512 && (c->variant == 1 || !c->f32))
    return fail(c, MC_E_ARG, "workgroups of more than 512 lanes need FP32 state and a lane-refill variant");
  if (n == 0) return MC_OK;
  if (c->use_graph && !c->profile) {
    if (!c->gexec) {
      hipGraph_t g = nullptr;
      HIPCHK(c, hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
      enqueue_interval(c);
      const hipError_t le = hipGetLastError();
      HIPCHK(c, hipStreamEndCapture(c->st, &g));
      if (le != hipSuccess) { (void)hipGraphDestroy(g); return fail(c, MC_E_HIP, hipGetErrorString(le)); }
      const hipError_t ie = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) { c->gexec = nullptr; return fail(c, MC_E_HIP, hipGetErrorString(ie)); }
    }
    for (int i = 0; i < n; ++i) HIPCHK(c, hipGraphLaunch(c->gexec, c->st));
  } else {
    for (int i = 0; i < n; ++i) enqueue_interval(c);
    HIPCHK(c, hipGetLastError());
  }
  return MC_OK;
}

int poisson_update(mc_ctx* c) {
  if (!c) return MC_E_ARG;
  if (!c->dev) return MC_OK;
  const size_t lds = sizeof(uint32_t) * (5 * c->ncell + 1);
  if (c->f32)
    k_deposit<float><<<c->n_tiles, 256, lds, c->st>>>(c->p<TileDesc>(c->o.tiles), c->p<float>(c->o.x),
                                                     c->p<float>(c->o.y), c->p<float>(c->o.z),
                                                     c->p<uint32_t>(c->o.meta), c->G32,
                                                     c->p<unsigned long long>(c->o.acc), c->p<uint32_t>(c->o.tile_dead));
  else
    k_deposit<double><<<c->n_tiles, 256, lds, c->st>>>(c->p<TileDesc>(c->o.tiles), c->p<double>(c->o.x),
                                                      c->p<double>(c->o.y), c->p<double>(c->o.z),
                                                      c->p<uint32_t>(c->o.meta), c->G64,
                                                      c->p<unsigned long long>(c->o.acc), c->p<uint32_t>(c->o.tile_dead));
  enqueue_refresh(c, false);
  HIPCHK(c, hipGetLastError());
  return MC_OK;
}

int mc_tally(mc_ctx* c, int inst, mc_tally_out* out, int reset_window) {
  if (!c || inst < 0 || inst >= c->n_inst || !out) return fail(c, MC_E_ARG, "bad argument");
  std::vector<unsigned long long> cnt(kNCnt);
  uint32_t ctl[16];
  int flag = 0;
  HIPCHK(c, hipMemcpyAsync(cnt.data(), c->p<unsigned long long>(c->o.counters) + (size_t)inst * kNCnt,
                           sizeof(unsigned long long) * kNCnt, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(ctl, c->p<uint32_t>(c->o.ctl), sizeof(ctl), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(&flag, c->p<int>(c->o.flags) + inst, sizeof(int), hipMemcpyDeviceToHost, c->st));
  // alive count: number of live slots of this instance
  std::vector<uint32_t> meta(c->cfg[inst].capacity);
  HIPCHK(c, hipMemcpyAsync(meta.data(), c->p<uint32_t>(c->o.meta) + c->ip[inst].base, sizeof(uint32_t) * meta.size(),
                           hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  std::memset(out, 0, sizeof(*out));
  out->intervals = ctl[CTL_WINDOW];
  out->intervals_total = ctl[CTL_INTERVAL];
  const double TP = c->cfg[0].dt_fs * c->cfg[0].substeps;
  out->t_window_fs = TP * ctl[CTL_WINDOW];
  uint64_t alive = 0;
  for (uint32_t m : meta) alive += (m & kAlive) ? 1 : 0;
  out->n_alive = alive;
  out->selections = cnt[C_SEL];
  out->self_events = cnt[C_SELF];
  out->overflow = cnt[C_OVF];
  for (int v = 0; v < 3; ++v)
    for (int m = 0; m < kNM; ++m) out->real[v][m] = cnt[C_REAL + v * kNM + m];
  out->exits[0] = cnt[C_EXIT0]; out->exits[1] = cnt[C_EXIT1];
  out->injections[0] = cnt[C_INJ0]; out->injections[1] = cnt[C_INJ1];
  out->segments = cnt[C_PROC] * (uint64_t)c->cfg[0].substeps + cnt[C_SEL];
  out->reflect_guard = cnt[C_REFL];
  out->weight = c->ip[inst].w;
  const double tw = out->t_window_fs * 1e-15;
  out->drain_current_A =
      tw > 0 ? kQ * c->ip[inst].w * ((double)cnt[C_EXIT1] - (double)cnt[C_INJ1]) / tw : 0.0;
  out->flags = flag;
  if (reset_window) {
    const size_t nh = (size_t)c->n_inst * c->ncell * 4, nd = (size_t)c->n_inst * c->ncell;
    const size_t nmax = std::max(nh, (size_t)c->n_inst * kNCnt);
    k_zero_window<<<(unsigned)((nmax + 255) / 256), 256, 0, c->st>>>(
        c->p<unsigned long long>(c->o.heat), c->p<unsigned long long>(c->o.dens),
        c->p<unsigned long long>(c->o.counters), nh, nd, c->n_inst, c->p<uint32_t>(c->o.ctl));
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->st));
  }
  return flag;
}

int mc_maps(mc_ctx* c, int inst, uint64_t* h_heat4, uint64_t* h_dens, double* h_heat_Wm3, double* h_dens_m3,
            double* h_emit_Wm3) {
  if (!c || inst < 0 || inst >= c->n_inst) return fail(c, MC_E_ARG, "bad argument");
  const int nc = c->ncell;
  std::vector<unsigned long long> heat((size_t)4 * nc), dens(nc);
  uint32_t ctl[16];
  HIPCHK(c, hipMemcpyAsync(heat.data(), c->p<unsigned long long>(c->o.heat) + (size_t)inst * 4 * nc,
                           sizeof(unsigned long long) * 4 * nc, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(dens.data(), c->p<unsigned long long>(c->o.dens) + (size_t)inst * nc,
                           sizeof(unsigned long long) * nc, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(ctl, c->p<uint32_t>(c->o.ctl), sizeof(ctl), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  const double w = c->ip[inst].w;
  const double Vc_m3 = (c->dev ? c->pg.Vc : 1.0) * 1e-27;
  const double tw = c->cfg[0].dt_fs * c->cfg[0].substeps * ctl[CTL_WINDOW] * 1e-15;
  const mc_material& m = c->cfg[0].mat;
  for (int q = 0; q < nc; ++q) {
    const double em_lo = (double)heat[0 * nc + q], ab_lo = (double)heat[1 * nc + q];
    const double em_iv = (double)heat[2 * nc + q], ab_iv = (double)heat[3 * nc + q];
    if (h_heat4) {
      h_heat4[4 * q + 0] = heat[0 * nc + q]; h_heat4[4 * q + 1] = heat[1 * nc + q];
      h_heat4[4 * q + 2] = heat[2 * nc + q]; h_heat4[4 * q + 3] = heat[3 * nc + q];
    }
    if (h_dens) h_dens[q] = dens[q];
    if (h_heat_Wm3)
      h_heat_Wm3[q] = tw > 0 ? w * kQ * (m.hw_lo_eV * (em_lo - ab_lo) + m.hw_iv_eV * (em_iv - ab_iv)) / (Vc_m3 * tw)
                             : 0.0;
    if (h_dens_m3) h_dens_m3[q] = ctl[CTL_WINDOW] ? w * (double)dens[q] / ctl[CTL_WINDOW] / Vc_m3 : 0.0;
    if (h_emit_Wm3)
      h_emit_Wm3[q] = tw > 0 ? w * kQ * (m.hw_lo_eV * em_lo + m.hw_iv_eV * em_iv) / (Vc_m3 * tw) : 0.0;
  }
  return MC_OK;
}

int mc_history(mc_ctx* c, int inst, double* h_rows, int max_rows, int* n_rows) {
  if (!c || inst < 0 || inst >= c->n_inst || !n_rows || max_rows < 0) return fail(c, MC_E_ARG, "bad argument");
  *n_rows = 0;
  uint32_t ctl[16];
  HIPCHK(c, hipMemcpyAsync(ctl, c->p<uint32_t>(c->o.ctl), sizeof(ctl), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  const int n = std::min<int>((int)ctl[CTL_WINDOW], std::min(kHistCap, max_rows));
  if (n > 0 && h_rows) {
    HIPCHK(c, hipMemcpyAsync(h_rows, c->p<double>(c->o.hist) + (size_t)inst * kHistCap * 8, sizeof(double) * 8 * n,
                             hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
  }
  *n_rows = n;
  return MC_OK;
}

namespace {

// Two-halves test of one per-interval series: the last 2h values (h = m/2)
// split in halves, each half's mean and standard error from 10 batch means
// of h/10 consecutive values; steady when the means differ by no more than
// three combined standard errors.  -1 when a half has fewer than 10 values.
int halves_steady(const std::vector<double>& s, double mean[2], double se[2]) {
  constexpr int kBlocks = 10;
  const int m = (int)s.size(), h = m / 2, b = h / kBlocks;
  mean[0] = mean[1] = se[0] = se[1] = 0.0;
  if (b < 1) return -1;
  for (int half = 0; half < 2; ++half) {
    const int first = m - 2 * h + half * h;
    double bm[kBlocks];
    double mu = 0.0;
    for (int j = 0; j < kBlocks; ++j) {
      double acc = 0.0;
      for (int i = first + j * b; i < first + (j + 1) * b; ++i) acc += s[i];
      bm[j] = acc / b;
      mu += bm[j];
    }
    mu /= kBlocks;
    double ss = 0.0;
    for (int j = 0; j < kBlocks; ++j) ss += (bm[j] - mu) * (bm[j] - mu);
    mean[half] = mu;
    se[half] = std::sqrt(ss / (kBlocks * (kBlocks - 1.0)));
  }
  return std::fabs(mean[0] - mean[1]) <= 3.0 * std::hypot(se[0], se[1]) ? 1 : 0;
}

}  // namespace

int mc_observables(mc_ctx* c, int inst, mc_observables_out* out) {
  if (!c || inst < 0 || inst >= c->n_inst || !out) return fail(c, MC_E_ARG, "bad argument");
  std::memset(out, 0, sizeof(*out));
  int n = 0, rc;
  std::vector<double> rows((size_t)kHistCap * 8);
  if ((rc = mc_history(c, inst, rows.data(), kHistCap, &n)) != MC_OK) return rc;
  mc_tally_out t;
  std::memset(&t, 0, sizeof(t));
  rc = mc_tally(c, inst, &t, 0);
  if (rc != MC_OK && rc != t.flags) return rc;  // a runtime failure, not a sticky device flag
  const double TP = c->cfg[0].dt_fs * c->cfg[0].substeps * 1e-15;  // s
  out->intervals = t.intervals;
  out->t_window_fs = t.t_window_fs;
  std::vector<double> s1(n), s2(n);
  if (c->dev) {
    const double qw = kQ * c->ip[inst].w, tw = t.t_window_fs * 1e-15;
    if (tw > 0.0) {
      out->drain_current_A = qw * ((double)t.exits[1] - (double)t.injections[1]) / tw;
      out->source_current_A = qw * ((double)t.exits[0] - (double)t.injections[0]) / tw;
    }
    std::vector<uint64_t> heat4((size_t)4 * c->ncell);
    if ((rc = mc_maps(c, inst, heat4.data(), nullptr, nullptr, nullptr, nullptr)) != MC_OK) return rc;
    const mc_material& m = c->cfg[0].mat;
    double net = 0.0, emit = 0.0;  // eV
    for (int q = 0; q < c->ncell; ++q) {
      const uint64_t* h = heat4.data() + 4 * q;
      net += m.hw_lo_eV * ((double)h[0] - (double)h[1]) + m.hw_iv_eV * ((double)h[2] - (double)h[3]);
      emit += m.hw_lo_eV * (double)h[0] + m.hw_iv_eV * (double)h[2];
    }
    if (tw > 0.0) {
      out->heat_W = qw * net / tw;
      out->emit_W = qw * emit / tw;
    }
    // drain current of each interval from the window's cumulative counts
    for (int i = 0; i < n; ++i) {
      const double* r = rows.data() + 8 * (size_t)i;
      const double ex0 = i ? r[1 - 8] : 0.0, in0 = i ? r[3 - 8] : 0.0;
      s1[i] = qw * ((r[1] - ex0) - (r[3] - in0)) / TP;
      s2[i] = r[6];
    }
  } else {
    for (int i = 0; i < n; ++i) {
      const double* r = rows.data() + 8 * (size_t)i;
      const double na = r[0] > 0.0 ? r[0] : 1.0;
      for (int d = 0; d < 3; ++d) out->drift_velocity_ms[d] += r[1 + d] / na * 1e6 / n;  // nm/fs -> m/s
      out->mean_energy_eV += r[4] / na / n;
      for (int v = 0; v < 3; ++v) out->valley_fraction[v] += r[5 + v] / na / n;
      s1[i] = r[3] / na * 1e6;
      s2[i] = r[4] / na;
    }
  }
  const int f1 = halves_steady(s1, out->half_mean[0], out->half_se[0]);
  const int f2 = halves_steady(s2, out->half_mean[1], out->half_se[1]);
  out->steady = (f1 < 0 || f2 < 0) ? -1 : (f1 == 1 && f2 == 1 ? 1 : 0);
  return t.flags;
}

int mc_particles(mc_ctx* c, int inst, mc_particles_view* out) {
  if (!c || inst < 0 || inst >= c->n_inst || !out) return fail(c, MC_E_ARG, "bad argument");
  const size_t es = c->f32 ? 4 : 8;
  const long long b = c->ip[inst].base;
  out->kx = c->ws + c->o.kx + es * b; out->ky = c->ws + c->o.ky + es * b; out->kz = c->ws + c->o.kz + es * b;
  out->x = c->dev ? c->ws + c->o.x + es * b : nullptr;
  out->y = c->dev ? c->ws + c->o.y + es * b : nullptr;
  out->z = c->dev ? c->ws + c->o.z + es * b : nullptr;
  out->meta = c->p<uint32_t>(c->o.meta) + b;
  out->capacity = c->cfg[inst].capacity;
  out->elem_bytes = (int)es;
  return MC_OK;
}

int mc_read_particles(mc_ctx* c, int inst, double* h_k, double* h_r, int32_t* h_valley, int32_t* h_alive,
                      uint32_t* h_id) {
  if (!c || inst < 0 || inst >= c->n_inst) return fail(c, MC_E_ARG, "bad argument");
  const int cap = c->cfg[inst].capacity;
  const long long b = c->ip[inst].base;
  const size_t es = c->f32 ? 4 : 8;
  std::vector<char> buf[6];
  const size_t offs[6] = {c->o.kx, c->o.ky, c->o.kz, c->o.x, c->o.y, c->o.z};
  std::vector<uint32_t> meta(cap);
  for (int d = 0; d < 6; ++d) {
    if (d >= 3 && !c->dev) continue;
    buf[d].resize(es * cap);
    HIPCHK(c, hipMemcpyAsync(buf[d].data(), c->ws + offs[d] + es * b, es * cap, hipMemcpyDeviceToHost, c->st));
  }
  HIPCHK(c, hipMemcpyAsync(meta.data(), c->p<uint32_t>(c->o.meta) + b, sizeof(uint32_t) * cap, hipMemcpyDeviceToHost,
                           c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (int i = 0; i < cap; ++i) {
    for (int d = 0; d < 6; ++d) {
      double val = 0.0;
      if (d < 3 || c->dev) val = c->f32 ? (double)((float*)buf[d].data())[i] : ((double*)buf[d].data())[i];
      if (d < 3) { if (h_k) h_k[3 * i + d] = val; }
      else if (h_r) h_r[3 * i + d - 3] = val;
    }
    const uint32_t m = meta[i];
    if (h_valley) h_valley[i] = (int32_t)(m & 3u);
    if (h_alive) h_alive[i] = (m & kAlive) ? 1 : 0;
    if (h_id) h_id[i] = m >> 3;
  }
  return MC_OK;
}

int mc_write_particles(mc_ctx* c, int inst, const double* h_k, const double* h_r, const int32_t* h_valley,
                       const int32_t* h_alive, const uint32_t* h_id) {
  if (!c || inst < 0 || inst >= c->n_inst || !h_k || !h_valley || !h_alive || !h_id)
    return fail(c, MC_E_ARG, "bad argument");
  if (c->dev && !h_r) return fail(c, MC_E_ARG, "positions required in device mode");
  const int cap = c->cfg[inst].capacity;
  const long long b = c->ip[inst].base;
  const size_t es = c->f32 ? 4 : 8;
  // every input is checked before anything is copied: a rejected write
  // leaves the instance as it was
  std::vector<uint32_t> meta(cap);
  for (int i = 0; i < cap; ++i) {
    if (h_id[i] >= (1u << 29) || h_valley[i] < 0 || h_valley[i] > 2) return fail(c, MC_E_ARG, "bad particle");
    meta[i] = (h_id[i] << 3) | (h_alive[i] ? kAlive : 0u) | (uint32_t)h_valley[i];
  }
  const size_t offs[6] = {c->o.kx, c->o.ky, c->o.kz, c->o.x, c->o.y, c->o.z};
  std::vector<char> buf[6];
  for (int d = 0; d < 6; ++d) {
    if (d >= 3 && !c->dev) continue;
    buf[d].resize(es * cap);
    for (int i = 0; i < cap; ++i) {
      const double val = d < 3 ? h_k[3 * i + d] : h_r[3 * i + d - 3];
      if (c->f32) ((float*)buf[d].data())[i] = (float)val;
      else ((double*)buf[d].data())[i] = val;
    }
  }
  // the copies are ordered after every kernel already enqueued on the
  // context's stream (a write right after an asynchronous mc_step waits for
  // it) and complete before the call returns
  for (int d = 0; d < 6; ++d) {
    if (d >= 3 && !c->dev) continue;
    HIPCHK(c, hipMemcpyAsync(c->ws + offs[d] + es * b, buf[d].data(), es * cap, hipMemcpyHostToDevice, c->st));
  }
  HIPCHK(c, hipMemcpyAsync(c->p<uint32_t>(c->o.meta) + b, meta.data(), sizeof(uint32_t) * cap, hipMemcpyHostToDevice,
                           c->st));
  // live electrons may now lie anywhere in the instance's slots
  k_set_hw<<<1, 64, 0, c->st>>>(c->p<Plan>(c->o.plan), inst, (uint32_t)cap);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->st));
  return MC_OK;
}

int mc_get_config(const mc_ctx* c, int inst, mc_config* out) {
  if (!c || inst < 0 || inst >= c->n_inst || !out) return MC_E_ARG;
  *out = c->cfg[inst];
  return MC_OK;
}

int mc_get_lattice_temperature(const mc_ctx* c, int inst, double* h_T) {
  if (!c || inst < 0 || inst >= c->n_inst || !h_T) return MC_E_ARG;
  std::memcpy(h_T, c->Tcell[inst].data(), sizeof(double) * c->ncell);
  return MC_OK;
}

int mc_read_fields(mc_ctx* c, int inst, double* h_phi, double* h_field, uint32_t* h_count) {
  if (!c || inst < 0 || inst >= c->n_inst) return fail(c, MC_E_ARG, "bad argument");
  const int nc = c->ncell;
  std::vector<double> f((size_t)4 * nc);
  HIPCHK(c, hipMemcpyAsync(f.data(), c->p<double>(c->o.field64) + (size_t)inst * 4 * nc, sizeof(double) * 4 * nc,
                           hipMemcpyDeviceToHost, c->st));
  if (h_phi)
    HIPCHK(c, hipMemcpyAsync(h_phi, c->p<double>(c->o.phi) + (size_t)inst * nc, sizeof(double) * nc,
                             hipMemcpyDeviceToHost, c->st));
  if (h_count)
    HIPCHK(c, hipMemcpyAsync(h_count, c->p<uint32_t>(c->o.count) + (size_t)inst * nc, sizeof(uint32_t) * nc,
                             hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (h_field)
    for (int q = 0; q < nc; ++q)
      for (int d = 0; d < 3; ++d) h_field[3 * q + d] = f[4 * q + d];
  return MC_OK;
}

int mc_read_tables(mc_ctx* c, int inst, double* h_shape, double* h_k4, double* h_factors, double* h_gamma) {
  if (!c || inst < 0 || inst >= c->n_inst) return fail(c, MC_E_ARG, "bad argument");
  std::vector<double> t((size_t)3 * c->nb * kTRow), f((size_t)c->ncell * kFRow);
  double g[4];
  HIPCHK(c, hipMemcpyAsync(t.data(), c->p<double>(c->o.table64), sizeof(double) * t.size(), hipMemcpyDeviceToHost,
                           c->st));
  HIPCHK(c, hipMemcpyAsync(f.data(), c->p<double>(c->o.fac64) + (size_t)inst * c->ncell * kFRow,
                           sizeof(double) * f.size(), hipMemcpyDeviceToHost, c->st));
  if (c->f32) {
    float g32[4];
    HIPCHK(c, hipMemcpyAsync(g32, c->p<float>(c->o.gamma32) + inst * 4, sizeof(g32), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (int v = 0; v < 4; ++v) g[v] = g32[v];
  } else {
    HIPCHK(c, hipMemcpyAsync(g, c->p<double>(c->o.gamma64) + inst * 4, sizeof(g), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
  }
  for (int v = 0; v < 3; ++v)
    for (int b = 0; b < c->nb; ++b) {
      const size_t r = (size_t)v * c->nb + b;
      if (h_shape)
        for (int m = 0; m < kNM; ++m) h_shape[r * kNM + m] = t[r * kTRow + m];
      if (h_k4) h_k4[r] = t[r * kTRow + 10];
    }
  if (h_factors)
    for (int q = 0; q < c->ncell; ++q)
      for (int k = 0; k < 7; ++k) h_factors[q * 7 + k] = f[(size_t)q * kFRow + k];
  if (h_gamma)
    for (int v = 0; v < 3; ++v) h_gamma[v] = g[v];
  return MC_OK;
}

int mc_set_launch(mc_ctx* c, int block, int tile) {
  if (!c) return MC_E_ARG;
  if (block < 64 || block > 1024 || block % 64 || tile < min_tile(c->cfg[0]) || tile > kMaxTile || tile % block)
    return fail(c, MC_E_ARG, "unsupported launch shape");
  c->block = block;
  c->tile = tile;
  drop_graph(c);
  return upload_tiles(c);
}

int mc_set_variant(mc_ctx* c, int variant) {
  if (!c || variant < 0 || variant > 3) return fail(c, MC_E_ARG, "unknown kernel variant");
  c->variant = variant;
  drop_graph(c);
  return upload_tiles(c);
}

int mc_occupancy(mc_ctx* c, int block, int* wg_per_cu, int* n_cu) {
  if (!c || !wg_per_cu || !n_cu) return MC_E_ARG;
  if (block < 64 || block > 1024 || block % 64) return fail(c, MC_E_ARG, "unsupported block");
  return flight_occupancy(c, c->variant, block, wg_per_cu, n_cu);
}

int mc_get_launch(const mc_ctx* c, int* block, int* tile, int* n_tiles) {
  if (!c) return MC_E_ARG;
  if (block) *block = c->block;
  if (tile) *tile = c->tile;
  if (n_tiles) *n_tiles = c->n_tiles;
  return MC_OK;
}

int mc_get_ncell(const mc_ctx* c, int* ncell) {
  if (!c || !ncell) return MC_E_ARG;
  *ncell = c->ncell;
  return MC_OK;
}

int mc_get_instances(const mc_ctx* c, int* n) {
  if (!c || !n) return MC_E_ARG;
  *n = c->n_inst;
  return MC_OK;
}

int mc_get_stream(const mc_ctx* c, void** stream) {
  if (!c || !stream) return MC_E_ARG;
  *stream = (void*)c->st;
  return MC_OK;
}

int mc_use_graph(mc_ctx* c, int enable) {
  if (!c) return MC_E_ARG;
  c->use_graph = enable != 0;
  if (!c->use_graph) drop_graph(c);
  return MC_OK;
}

int mc_profile(mc_ctx* c, int enable) {
  if (!c) return MC_E_ARG;
  c->profile = enable != 0;
  return MC_OK;
}

int mc_profile_read(mc_ctx* c, double* flight_ms, int* n_flight, double* refresh_ms, int* n_refresh, int reset) {
  if (!c) return MC_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->st));
  double fm = 0.0, rm = 0.0;
  const int n = (int)(c->ev_used / 3);
  for (int i = 0; i < n; ++i) {
    float a = 0.f, b = 0.f;
    HIPCHK(c, hipEventElapsedTime(&a, c->ev_pool[3 * i], c->ev_pool[3 * i + 1]));
    HIPCHK(c, hipEventElapsedTime(&b, c->ev_pool[3 * i + 1], c->ev_pool[3 * i + 2]));
    fm += a;
    rm += b;
  }
  if (flight_ms) *flight_ms = fm;
  if (n_flight) *n_flight = n;
  if (refresh_ms) *refresh_ms = rm;
  if (n_refresh) *n_refresh = n;
  if (reset) c->ev_used = 0;
  return MC_OK;
}

// checkpoint = a format word, the byte count of the evolving state, the
// regions of the workspace that hold it (in layout order) and the host-side
// temperature maps.  Set-up products (the Poisson inverse), the tiling and
// the per-interval scratch (compaction copy, slot list, histogram merge,
// right-hand side) are not carried: the restoring context has its own and
// rewrites the rest.  The format word changes whenever the meaning of the
// carried state does.
constexpr uint64_t kCheckpointFormat = 0x67666d6300000004ull;  // "gfmc", 4: evolving regions only

namespace {
size_t kept_bytes(const Offsets& o) {
  size_t b = 0;
  for (const auto& r : o.kept) b += r.second;
  return b;
}
}  // namespace

int mc_checkpoint(mc_ctx* c, void* h_buf, size_t* bytes) {
  if (!c || !bytes) return MC_E_ARG;
  const size_t need = kept_bytes(c->o);
  const size_t tbytes = sizeof(double) * (size_t)c->n_inst * c->ncell;
  const size_t total = 2 * sizeof(uint64_t) + need + tbytes;
  if (!h_buf) { *bytes = total; return MC_OK; }
  if (*bytes < total) return fail(c, MC_E_ARG, "checkpoint buffer too small");
  std::memcpy(h_buf, &kCheckpointFormat, sizeof(uint64_t));
  char* b = (char*)h_buf + sizeof(uint64_t);
  const uint64_t n64 = need;
  std::memcpy(b, &n64, sizeof(n64));
  char* d = b + sizeof(n64);
  for (const auto& r : c->o.kept) {
    HIPCHK(c, hipMemcpyAsync(d, c->ws + r.first, r.second, hipMemcpyDeviceToHost, c->st));
    d += r.second;
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (int i = 0; i < c->n_inst; ++i)
    std::memcpy(d + sizeof(double) * (size_t)i * c->ncell, c->Tcell[i].data(), sizeof(double) * c->ncell);
  *bytes = total;
  return MC_OK;
}

int mc_restore(mc_ctx* c, const void* h_buf, size_t bytes) {
  if (!c || !h_buf) return MC_E_ARG;
  const size_t need = kept_bytes(c->o);
  const size_t tbytes = sizeof(double) * (size_t)c->n_inst * c->ncell;
  uint64_t fmt = 0, n64 = 0;
  if (bytes < 2 * sizeof(uint64_t)) return fail(c, MC_E_ARG, "checkpoint does not match");
  std::memcpy(&fmt, h_buf, sizeof(fmt));
  if (fmt != kCheckpointFormat) return fail(c, MC_E_ARG, "checkpoint from another library version");
  const char* b = (const char*)h_buf + sizeof(uint64_t);
  bytes -= sizeof(uint64_t);
  std::memcpy(&n64, b, sizeof(n64));
  if (n64 != need || bytes < sizeof(n64) + need + tbytes) return fail(c, MC_E_ARG, "checkpoint does not match");
  // keep the launch-shape-dependent tile table of this context
  const int blk = c->block, tl = c->tile;
  const char* d = b + sizeof(n64);
  for (const auto& r : c->o.kept) {
    HIPCHK(c, hipMemcpyAsync(c->ws + r.first, d, r.second, hipMemcpyHostToDevice, c->st));
    d += r.second;
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (int i = 0; i < c->n_inst; ++i)
    std::memcpy(c->Tcell[i].data(), d + sizeof(double) * (size_t)i * c->ncell, sizeof(double) * c->ncell);
  drop_graph(c);
  return mc_set_launch(c, blk, tl);
}

}  // extern "C"
