// hybrid.hip -- the electro-thermal iteration of the coupling paragraph on
// one GPU: electron Monte Carlo windows (mc_* of gfmc.h) and phonon packet
// runs (ph_* of gfph.h) alternate on the electron context's stream until the
// lattice temperature is steady; the device thermal resistance of the
// thermal-resistance passage comes out of every iteration.  C ABI in
// include/gfhy.h.
//
// The heavy work is the kernels behind mc_step and ph_mc_run.  Between them
// this file moves one map per instance each way (ncell doubles, at most 4096)
// and does the per-subcell coupling arithmetic of the iteration: the source
// q = h V_c, the new temperature T_sink + dT, its under-relaxed update.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/gfhy.h"

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

int from_ph(int rc) { return rc == PH_OK ? MC_OK : rc == PH_E_ARG ? MC_E_ARG : MC_E_HIP; }

// the chip's temperature below each electron subcell column (NaN for an
// index outside the chip, which the host refuses)
__global__ void k_hy_gather(const double* __restrict__ T_chip, long long nc_chip, const int32_t* __restrict__ base,
                            int n, double* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) {
    const long long b = base[c];
    out[c] = (b >= 0 && b < nc_chip) ? T_chip[b] : __longlong_as_double(0x7ff8000000000000ll);
  }
}

// largest value of a chip array (one workgroup, fixed order)
__global__ void __launch_bounds__(1024) k_hy_max(const double* __restrict__ v, long long n, double* out) {
  __shared__ double s[1024];
  double m = -1.0e300;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, v[i]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

// Per-instance slice of the workspace: tables [4][nb], Fermi level, source,
// packet times, temperature rise, and the packet run's own workspace.
struct Slice {
  size_t tab, fermi, q, t, dT, ph, ph_bytes, total;
};

Slice slice_of(int nb, int ncell, size_t ph_bytes) {
  Slice s;
  size_t off = 0;
  auto take = [&](size_t b) { const size_t o = off; off += up(b); return o; };
  s.tab = take(sizeof(double) * 4 * (size_t)nb);
  s.fermi = take(sizeof(double));
  s.q = take(sizeof(double) * ncell);
  s.t = take(sizeof(double) * ncell);
  s.dT = take(sizeof(double) * ncell);
  s.ph = take(ph_bytes);
  s.ph_bytes = ph_bytes;
  s.total = off;
  return s;
}

ph_mc_config phonon_domain(const mc_config& m, const hy_config& h, int inst) {
  ph_mc_config p;
  std::memset(&p, 0, sizeof(p));
  for (int d = 0; d < 3; ++d) {
    p.L_nm[d] = m.L_nm[d];
    p.n_cells[d] = m.n_cells[d];
  }
  for (int f = 0; f < 6; ++f) p.face[f] = h.face[f];
  p.n_bins = h.n_bins;
  p.seed = h.seed;
  p.instance = (uint32_t)inst;
  p.max_events = h.max_events;
  p.n_packets = h.n_packets;
  return p;
}

// The chip stage's region, shared by the instances (they run it in turn):
// conductivity, heat and temperature per chip cell, the gathered reference
// per subcell, the largest rise, the solver's workspace.
struct ChipSlice {
  size_t kap, q, T, base, mx, fo, fo_bytes, total;
  long long nc;
};

// Everything hy_run needs to know about the context, validated.
struct Plan {
  int n_inst = 0, ncell = 0;
  std::vector<mc_config> cfg;
  std::vector<ph_mc_config> ph;
  Slice sl;
  bool chip = false;
  fo_config fo;
  ChipSlice cs;
};

int plan_chip(const hy_config* h, const hy_chip* chip, int ncell, Plan* p) {
  if (!chip) return MC_OK;
  if (!chip->d_edges || !chip->d_material || !chip->d_src_index || !chip->d_base_index || chip->n_materials < 1 ||
      chip->n_materials > 16 || chip->half_wires < 1)
    return MC_E_ARG;
  for (int t = 0; t < chip->n_materials; ++t)
    if (!(chip->kappa_by_material[t] >= 0.0) || !std::isfinite(chip->kappa_by_material[t])) return MC_E_ARG;
  p->fo = chip->fo;
  p->fo.T_sink_K = h->T_sink_K;
  const size_t fb = fo_workspace_bytes(&p->fo);
  if (fb == 0) return MC_E_ARG;
  ChipSlice& c = p->cs;
  c.nc = (long long)p->fo.n[0] * p->fo.n[1] * p->fo.n[2];
  size_t off = 0;
  auto take = [&](size_t b) { const size_t o = off; off += up(b); return o; };
  c.kap = take(sizeof(double) * c.nc);
  c.q = take(sizeof(double) * c.nc);
  c.T = take(sizeof(double) * c.nc * (size_t)p->n_inst);  // per instance: each solve starts from its last
  c.base = take(sizeof(double) * ncell);
  c.mx = take(sizeof(double));
  c.fo = take(fb);
  c.fo_bytes = fb;
  c.total = off;
  p->chip = true;
  return MC_OK;
}

int plan_of(const mc_ctx* ctx, const hy_config* h, const hy_chip* chip, Plan* p) {
  if (!ctx || !h) return MC_E_ARG;
  if (mc_get_instances(ctx, &p->n_inst) != MC_OK || mc_get_ncell(ctx, &p->ncell) != MC_OK) return MC_E_ARG;
  if (h->window_intervals < 1 || h->warmup_intervals < 0 || h->max_iterations < 1 || !(h->relax > 0.0) ||
      h->relax > 1.0 || !(h->tol_K >= 0.0) || !(h->T_sink_K > 0.0) || !std::isfinite(h->T_lin_K))
    return MC_E_ARG;
  p->cfg.resize(p->n_inst);
  p->ph.resize(p->n_inst);
  size_t ph_bytes = 0;
  for (int i = 0; i < p->n_inst; ++i) {
    if (mc_get_config(ctx, i, &p->cfg[i]) != MC_OK || p->cfg[i].mode != MC_DEVICE) return MC_E_ARG;
    p->ph[i] = phonon_domain(p->cfg[i], *h, i);
    const size_t b = ph_mc_workspace_bytes(&p->ph[i]);
    if (b == 0) return MC_E_ARG;
    if (b > ph_bytes) ph_bytes = b;
  }
  p->sl = slice_of(h->n_bins, p->ncell, ph_bytes);
  return plan_chip(h, chip, p->ncell, p);
}

size_t total_bytes(const Plan& p) { return p.sl.total * (size_t)p.n_inst + (p.chip ? p.cs.total : 0); }

}  // namespace

extern "C" {

size_t hy_workspace_bytes(const mc_ctx* ctx, const hy_config* cfg, const hy_chip* chip) {
  Plan p;
  if (plan_of(ctx, cfg, chip, &p) != MC_OK) return 0;
  return total_bytes(p);
}

int hy_run(mc_ctx* ctx, const hy_config* h, const hy_chip* chip, const double* h_heat0, void* d_ws, size_t ws_bytes,
           hy_record* rec, int max_records, int* n_records, int* iterations) {
  if (n_records) *n_records = 0;
  if (iterations) *iterations = 0;
  Plan p;
  int rc = plan_of(ctx, h, chip, &p);
  if (rc != MC_OK) return rc;
  if (!d_ws || ((uintptr_t)d_ws & (kAlign - 1)) || ws_bytes < total_bytes(p) || max_records < 0)
    return MC_E_ARG;
  void* stream = nullptr;
  if (mc_get_stream(ctx, &stream) != MC_OK) return MC_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int nc = p.ncell, K = p.cfg[0].substeps;
  char* ws = (char*)d_ws;
  auto at = [&](int i, size_t off) { return ws + (size_t)i * p.sl.total + off; };

  std::vector<std::vector<double>> T(p.n_inst, std::vector<double>(nc));
  for (int i = 0; i < p.n_inst; ++i)
    if ((rc = mc_get_lattice_temperature(ctx, i, T[i].data())) != MC_OK) return rc;
  std::vector<double> heat(nc), q(nc), dT(nc), Tn(nc), base(nc, h->T_sink_K);
  char* cw = ws + p.sl.total * (size_t)p.n_inst;  // the chip region
  auto cat = [&](size_t off) { return (double*)(cw + off); };
  int written = 0;

  for (int it = 0; it < h->max_iterations; ++it) {
    const bool warm = it == 0 && h_heat0;
    if (!warm) {
      // the electrons at the current temperatures: settle, then one window
      if ((rc = mc_step(ctx, h->warmup_intervals * K)) != MC_OK) return rc;
      mc_tally_out tal;
      if ((rc = mc_tally(ctx, 0, &tal, 1)) != MC_OK) return rc;
      if ((rc = mc_step(ctx, h->window_intervals * K)) != MC_OK) return rc;
    }
    double worst = 0.0;
    for (int i = 0; i < p.n_inst; ++i) {
      hy_record r;
      std::memset(&r, 0, sizeof(r));
      r.iteration = it;
      r.instance = i;
      const mc_config& m = p.cfg[i];
      const double vc_m3 = (m.L_nm[0] / m.n_cells[0]) * (m.L_nm[1] / m.n_cells[1]) * (m.L_nm[2] / m.n_cells[2]) * 1e-27;
      if (warm) {
        r.source = 1;
        for (int c = 0; c < nc; ++c) heat[c] = h_heat0[(size_t)i * nc + c];
      } else {
        mc_observables_out ob;
        if ((rc = mc_observables(ctx, i, &ob)) != MC_OK) return rc;
        if ((rc = mc_maps(ctx, i, nullptr, nullptr, heat.data(), nullptr, nullptr)) != MC_OK) return rc;
        r.steady = ob.steady;
        r.drain_current_A = ob.drain_current_A;
        r.emit_W = ob.emit_W;
      }
      double hw = 0.0;
      for (int c = 0; c < nc; ++c) {
        if (!std::isfinite(heat[c])) return MC_E_ARG;
        q[c] = heat[c] * vc_m3;
        hw += q[c];
      }
      r.heat_W = hw;
      // phonon tables at the linearisation temperature, then the packets
      double tl = h->T_lin_K;
      if (!(tl > 0.0)) {
        double s = 0.0;
        for (int c = 0; c < nc; ++c) s += T[i][c];
        tl = s / nc;
      }
      r.T_lin_K = tl;
      double* d_tab = (double*)at(i, p.sl.tab);
      double* d_q = (double*)at(i, p.sl.q);
      double* d_dT = (double*)at(i, p.sl.dT);
      if (hipMemcpyAsync(d_q, q.data(), sizeof(double) * nc, hipMemcpyHostToDevice, st) != hipSuccess)
        return MC_E_HIP;
      const ph_electrons* el = h->elec.n_m3 > 0.0 ? &h->elec : nullptr;
      if ((rc = from_ph(ph_tables(&h->mat, el, tl, h->n_bins, d_tab, el ? (double*)at(i, p.sl.fermi) : nullptr,
                                  stream))) != MC_OK)
        return rc;
      uint64_t cnt[11];
      if ((rc = from_ph(ph_mc_run(&p.ph[i], d_tab, d_q, (double*)at(i, p.sl.t), d_dT, nullptr, cnt,
                                  at(i, p.sl.ph), p.sl.ph_bytes, stream))) != MC_OK)
        return rc;
      double fo_max = 0.0;
      if (p.chip) {
        // the Fourier stage: every wire takes this heat map; the chip's
        // temperature below each subcell column is its reference
        const ChipSlice& cs = p.cs;
        if ((rc = fo_chip_fields(chip->d_material, chip->kappa_by_material, chip->n_materials, chip->d_src_index,
                                 d_q, nc, 1.0, cs.nc, cat(cs.kap), cat(cs.q), stream)) != MC_OK)
          return rc;
        int fit = 0;
        double rel = 0.0;
        // each instance keeps its chip temperature; from the second
        // iteration its solve starts there (the heat map moves little)
        double* Ti = cat(cs.T) + (size_t)i * cs.nc;
        fo_config fo = p.fo;
        fo.warm_start = it > 0 ? 1 : 0;
        rc = fo_solve(&fo, chip->d_edges, cat(cs.kap), cat(cs.q), Ti, &fit, &rel, cw + cs.fo, cs.fo_bytes, stream);
        r.fo_iterations = fit;
        if (rc != MC_OK) return rc;
        k_hy_gather<<<(nc + 255) / 256, 256, 0, st>>>(Ti, cs.nc, chip->d_base_index, nc, cat(cs.base));
        k_hy_max<<<1, 1024, 0, st>>>(Ti, cs.nc, cat(cs.mx));
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(base.data(), cat(cs.base), sizeof(double) * nc, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&fo_max, cat(cs.mx), sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
          return MC_E_HIP;
      }
      if (hipMemcpyAsync(dT.data(), d_dT, sizeof(double) * nc, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return MC_E_HIP;
      for (int f = 0; f < 6; ++f) r.packets_absorbed += cnt[3 + f];
      r.packets_dropped = cnt[9];
      // the new temperature map and its under-relaxed update
      double mx = -1.0e300, sum = 0.0, change = 0.0, jmax = 0.0;
      int hot = 0;
      for (int c = 0; c < nc; ++c) {
        if (!std::isfinite(base[c])) return MC_E_ARG;
        const double rise = base[c] - h->T_sink_K + dT[c];
        if (rise > mx) { mx = rise; hot = c; }
        if (base[c] - h->T_sink_K > jmax) jmax = base[c] - h->T_sink_K;
        sum += rise;
        const double tn = base[c] + dT[c];
        const double d = std::fabs(tn - T[i][c]);
        if (d > change) change = d;
        Tn[c] = T[i][c] + h->relax * (tn - T[i][c]);
        if (!(Tn[c] > 0.0)) return MC_E_ARG;
      }
      r.dT_max_K = mx;
      r.dT_mean_K = sum / nc;
      r.hot_cell = hot;
      r.change_K = change;
      r.R_th_KW = r.emit_W > 0.0 ? mx / r.emit_W : 0.0;
      if (p.chip) {
        r.dT_junction_max_K = jmax;
        r.dT_fourier_max_K = fo_max - h->T_sink_K;
        const double P = chip->half_wires * r.emit_W;
        r.R_th_device_KW = P > 0.0 ? mx / P : 0.0;
        r.R_th_fourier_KW = P > 0.0 ? r.dT_fourier_max_K / P : 0.0;
      }
      if ((rc = mc_set_lattice_temperature(ctx, i, Tn.data())) != MC_OK) return rc;
      T[i] = Tn;
      if (change > worst) worst = change;
      if (rec && written < max_records) rec[written++] = r;
      if (n_records) *n_records = written;
    }
    if (iterations) *iterations = it + 1;
    if (worst <= h->tol_K) break;
  }
  return MC_OK;
}

}  // extern "C"
