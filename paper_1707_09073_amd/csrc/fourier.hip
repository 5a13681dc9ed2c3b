// fourier.hip -- Fourier's-law heat spreading on gfx950 (coupling paragraph:
// steady conduction outside the phonon Monte Carlo domain, with the
// GaN-substrate interface resistance of Eq. (3)).  C ABI in include/gffo.h.
//
// Cell-centred finite volumes on a tensor-product grid; the rise above the
// sink temperature solves a symmetric positive definite system, here by
// Jacobi-preconditioned conjugate gradients.  Face conductances are built
// once per solve (each face by both of its cells, from the same operands in
// the same order, so the operator is exactly symmetric); every iteration is
// a matrix-vector product, two dot products and three vector updates, all
// streaming HBM, in three kernels.  Dot products go through per-workgroup
// partial sums; the kernel that needs a dot product's value adds the
// partials itself, in every workgroup, in one fixed order (so every
// workgroup holds the same bits, and a solve gives the same bits for any
// launch), after it has issued its own cells' loads.  The conductance arrays
// and the search direction carry a zero halo of one x-plane at each end, so
// the matrix-vector product needs no cell coordinates: a neighbour across
// the grid's edge is either in the halo or, in y and z, a cell of the next
// column or plane whose face conductance is zero.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/gfmc.h"
#include "../../include/gffo.h"

namespace {

constexpr int kFoBlock = 256;
constexpr int kFoMaxBlocks = 1024;  // partial sums per dot product (each workgroup of a reading kernel adds them all)
constexpr int kFoUnroll = 4;        // cells per thread loaded before a dot product's partials are added
constexpr int kFoCheck = 25;        // iterations between convergence checks on the host

struct FoGrid {
  int nx, ny, nz;
  long long nc;
  const double* ex;  // nx + 1 edges
  const double* ey;  // ny + 1
  const double* ez;  // nz + 1
};

// Scalars of the iteration, on the device: r.z of the current iteration in
// slot S_RZ + (iteration & 1) (the direction kernel writes the next one into
// the other slot while its workgroups read this one), r.r, b.b.
enum { S_RZ = 0, S_RZ1, S_RR, S_BB, S_N };

__device__ inline double face_g(double k1, double k2, double d1, double d2, double area, double extra) {
  if (!(k1 > 0.0) || !(k2 > 0.0)) return 0.0;
  return area / (d1 / (2.0 * k1) + d2 / (2.0 * k2) + extra);
}

__device__ inline void cell_ijk(long long c, const FoGrid& g, int* i, int* j, int* k) {
  *k = (int)(c % g.nz);
  const long long t = c / g.nz;
  *j = (int)(t % g.ny);
  *i = (int)(t / g.ny);
}

// The cells [*c0, *c1) of this workgroup in the iteration kernels.  The grid
// has a multiple of 8 workgroups, cpw cells each (a multiple of kFoBlock);
// workgroups are dealt to the eight XCDs in turn (workgroup b to XCD b % 8),
// so workgroup b takes the (b / 8)-th span of XCD b % 8's eighth of the
// cells: each XCD sweeps one contiguous block of x-planes, and the x-
// neighbours a product reads lie in its own L2.
__device__ inline void wg_span(long long nc, long long cpw, long long* c0, long long* c1) {
  const long long per = gridDim.x / 8;
  const long long l = (blockIdx.x % 8) * per + blockIdx.x / 8;
  *c0 = l * cpw < nc ? l * cpw : nc;
  *c1 = *c0 + cpw < nc ? *c0 + cpw : nc;
}

// Workgroup total in a fixed order, returned to every thread: a butterfly
// across each wavefront (every lane adds the same two operands at each step,
// so every lane ends with the same bits), then the wavefront totals in
// wavefront order.
__device__ inline double wg_total(double v) {
  __shared__ double s[kFoBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = s[0];
#pragma unroll
  for (int w = 1; w < kFoBlock / 64; ++w) t += s[w];
  __syncthreads();  // s may be written again by the next call
  return t;
}

// Workgroup total into part[blockIdx.x].
__device__ inline void block_sum(double v, double* part) {
  const double t = wg_total(v);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Conductances to the +x, +y, +z neighbours, the diagonal (with the held
// faces), and the start of the iteration: x = 0, r = b = q (0 in voids),
// p = r / diag; partial sums of r.z and b.b.
__global__ void __launch_bounds__(kFoBlock) k_fo_setup(FoGrid g, const int* __restrict__ held, int k_if, double R_K,
                                                       const double* __restrict__ kap, const double* __restrict__ q,
                                                       double* gx, double* gy, double* gz, double* diag, double* x,
                                                       double* r, double* p, long long cpw, double* part_rz,
                                                       double* part_bb) {
  double rz = 0.0, bb = 0.0;
  const long long sx = (long long)g.ny * g.nz, sy = g.nz;
  long long c0, c1;
  wg_span(g.nc, cpw, &c0, &c1);
  for (long long c = c0 + threadIdx.x; c < c1; c += kFoBlock) {
    int i, j, k;
    cell_ijk(c, g, &i, &j, &k);
    const double dx = g.ex[i + 1] - g.ex[i], dy = g.ey[j + 1] - g.ey[j], dz = g.ez[k + 1] - g.ez[k];
    const double kc = kap[c];
    double gxp = 0.0, gyp = 0.0, gzp = 0.0, d = 0.0;
    if (i + 1 < g.nx) gxp = face_g(kc, kap[c + sx], dx, g.ex[i + 2] - g.ex[i + 1], dy * dz, 0.0);
    if (j + 1 < g.ny) gyp = face_g(kc, kap[c + sy], dy, g.ey[j + 2] - g.ey[j + 1], dx * dz, 0.0);
    if (k + 1 < g.nz)
      gzp = face_g(kc, kap[c + 1], dz, g.ez[k + 2] - g.ez[k + 1], dx * dy, k + 1 == k_if ? R_K : 0.0);
    // the same faces seen from the -x, -y, -z neighbours (same operands, same order)
    const double gxm = i > 0 ? face_g(kap[c - sx], kc, g.ex[i] - g.ex[i - 1], dx, dy * dz, 0.0) : 0.0;
    const double gym = j > 0 ? face_g(kap[c - sy], kc, g.ey[j] - g.ey[j - 1], dy, dx * dz, 0.0) : 0.0;
    const double gzm = k > 0 ? face_g(kap[c - 1], kc, g.ez[k] - g.ez[k - 1], dz, dx * dy, k == k_if ? R_K : 0.0) : 0.0;
    d = gxp + gxm + gyp + gym + gzp + gzm;
    if (kc > 0.0) {
      if (i == 0 && held[0]) d += dy * dz / (dx / (2.0 * kc));
      if (i == g.nx - 1 && held[1]) d += dy * dz / (dx / (2.0 * kc));
      if (j == 0 && held[2]) d += dx * dz / (dy / (2.0 * kc));
      if (j == g.ny - 1 && held[3]) d += dx * dz / (dy / (2.0 * kc));
      if (k == 0 && held[4]) d += dx * dy / (dz / (2.0 * kc));
      if (k == g.nz - 1 && held[5]) d += dx * dy / (dz / (2.0 * kc));
    }
    const bool live = kc > 0.0;
    if (!live) d = 1.0;
    const double b = live ? q[c] : 0.0;
    gx[c] = gxp;
    gy[c] = gyp;
    gz[c] = gzp;
    diag[c] = d;
    x[c] = 0.0;
    r[c] = b;
    const double z = b / d;
    p[c] = z;
    rz += b * z;
    bb += b * b;
  }
  // the halos: one x-plane of zeros before and after the conductances and p
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < sx; c += (long long)gridDim.x * blockDim.x) {
    gx[c - sx] = 0.0; gy[c - sx] = 0.0; gz[c - sx] = 0.0; p[c - sx] = 0.0;
    gx[g.nc + c] = 0.0; gy[g.nc + c] = 0.0; gz[g.nc + c] = 0.0; p[g.nc + c] = 0.0;
  }
  block_sum(rz, part_rz);
  block_sum(bb, part_bb);
}

// Ap = A p and partial sums of p.Ap.  gx, gy, gz and p have their halos (a
// zero conductance or a zero entry multiplies every neighbour outside the
// grid); the neighbour terms are subtracted in the order +x, -x, +y, -y, +z,
// -z.
__global__ void __launch_bounds__(kFoBlock) k_fo_spmv(long long nc, long long cpw, long long sx, long long sy,
                                                      const double* __restrict__ gx, const double* __restrict__ gy,
                                                      const double* __restrict__ gz, const double* __restrict__ diag,
                                                      const double* __restrict__ p, double* __restrict__ Ap,
                                                      double* part) {
  double acc = 0.0;
  long long c0, c1;
  wg_span(nc, cpw, &c0, &c1);
  for (long long c = c0 + threadIdx.x; c < c1; c += kFoBlock) {
    const double pc = p[c];
    double a = diag[c] * pc;
    a -= gx[c] * p[c + sx];
    a -= gx[c - sx] * p[c - sx];
    a -= gy[c] * p[c + sy];
    a -= gy[c - sy] * p[c - sy];
    a -= gz[c] * p[c + 1];
    a -= gz[c - 1] * p[c - 1];
    Ap[c] = a;
    acc += pc * a;
  }
  block_sum(acc, part);
}

// The n partial sums of a dot product, added by one workgroup of kFoBlock
// threads in a fixed order (strided per thread, then wg_total): every
// workgroup that calls this gets the same bits.
__device__ inline double sum_parts(const double* part, int n) {
  double v = 0.0;
  for (int t = threadIdx.x; t < n; t += kFoBlock) v += part[t];
  return wg_total(v);
}

// The iteration's scalars from the set-up's partial sums; r.r is b.b unless
// a warm start gave its own partials (part_rr non-null)
__global__ void __launch_bounds__(kFoBlock) k_fo_start(const double* part_rz, const double* part_bb,
                                                       const double* part_rr, int n, double* sc) {
  const double rz = sum_parts(part_rz, n), bb = sum_parts(part_bb, n);
  const double rr = part_rr ? sum_parts(part_rr, n) : bb;
  if (threadIdx.x == 0) {
    sc[S_RZ] = rz;
    sc[S_BB] = bb;
    sc[S_RR] = rr;
  }
}

// Warm start, first step: the initial rise x0 = T - T_sink (0 in void
// cells) into p, whose halos the set-up zeroed.
__global__ void __launch_bounds__(kFoBlock) k_fo_warm_x(long long nc, long long cpw, const double* __restrict__ kap,
                                                        const double* __restrict__ T, double T_sink, double* p) {
  long long c0, c1;
  wg_span(nc, cpw, &c0, &c1);
  for (long long c = c0 + threadIdx.x; c < c1; c += kFoBlock) p[c] = kap[c] > 0.0 ? T[c] - T_sink : 0.0;
}

// Warm start, second step (after Ap = A x0): x = x0, r = b - A x0 (r holds
// b), z = p = r / diag; partial sums of r.z and r.r.
__global__ void __launch_bounds__(kFoBlock) k_fo_warm_r(long long nc, long long cpw, const double* __restrict__ diag,
                                                        const double* __restrict__ Ap, double* p, double* x,
                                                        double* r, double* part_rz, double* part_rr) {
  double rz = 0.0, rr = 0.0;
  long long c0, c1;
  wg_span(nc, cpw, &c0, &c1);
  for (long long c = c0 + threadIdx.x; c < c1; c += kFoBlock) {
    x[c] = p[c];
    const double rc = r[c] - Ap[c];
    const double z = rc / diag[c];
    r[c] = rc;
    p[c] = z;
    rz += rc * z;
    rr += rc * rc;
  }
  block_sum(rz, part_rz);
  block_sum(rr, part_rr);
}

// alpha = r.z / p.Ap (p.Ap from the product's partials, added here);
// x += alpha p; r -= alpha Ap; partial sums of r.z (z = r / diag) and r.r.
// The first kFoUnroll cells of each thread are loaded before the partials
// are added, so their latency overlaps.
__global__ void __launch_bounds__(kFoBlock) k_fo_update(long long nc, long long cpw, int slot,
                                                        const double* __restrict__ part_pap, int n_part,
                                                        const double* __restrict__ sc, const double* __restrict__ diag,
                                                        const double* __restrict__ p, const double* __restrict__ Ap,
                                                        double* __restrict__ x, double* __restrict__ r,
                                                        double* part_rz, double* part_rr) {
  long long s0, s1;
  wg_span(nc, cpw, &s0, &s1);
  const long long stride = kFoBlock, c0 = s0 + threadIdx.x;
  double vp[kFoUnroll], vA[kFoUnroll], vx[kFoUnroll], vr[kFoUnroll], vd[kFoUnroll];
#pragma unroll
  for (int u = 0; u < kFoUnroll; ++u) {
    const long long c = c0 + u * stride;
    const bool in = c < s1;
    vp[u] = in ? p[c] : 0.0;
    vA[u] = in ? Ap[c] : 0.0;
    vx[u] = in ? x[c] : 0.0;
    vr[u] = in ? r[c] : 0.0;
    vd[u] = in ? diag[c] : 1.0;
  }
  const double pap = sum_parts(part_pap, n_part);
  const double alpha = pap > 0.0 ? sc[S_RZ + slot] / pap : 0.0;
  double rz = 0.0, rr = 0.0;
#pragma unroll
  for (int u = 0; u < kFoUnroll; ++u) {
    const long long c = c0 + u * stride;
    if (c < s1) {
      x[c] = vx[u] + alpha * vp[u];
      const double rc = vr[u] - alpha * vA[u];
      r[c] = rc;
      rz += rc * (rc / vd[u]);
      rr += rc * rc;
    }
  }
  for (long long c = c0 + kFoUnroll * stride; c < s1; c += stride) {
    x[c] += alpha * p[c];
    const double rc = r[c] - alpha * Ap[c];
    r[c] = rc;
    rz += rc * (rc / diag[c]);
    rr += rc * rc;
  }
  block_sum(rz, part_rz);
  block_sum(rr, part_rr);
}

// beta = r.z (new, from the update's partials, added here) / r.z (old, in
// slot); p = z + beta p.  Workgroup 0 also stores the new r.z in the other
// slot and r.r for the host's convergence check.
__global__ void __launch_bounds__(kFoBlock) k_fo_direction(long long nc, long long cpw, int slot,
                                                           const double* __restrict__ part_rz,
                                                           const double* __restrict__ part_rr, int n_part,
                                                           double* __restrict__ sc, const double* __restrict__ diag,
                                                           const double* __restrict__ r, double* __restrict__ p) {
  long long s0, s1;
  wg_span(nc, cpw, &s0, &s1);
  const long long stride = kFoBlock, c0 = s0 + threadIdx.x;
  double vr[kFoUnroll], vd[kFoUnroll], vp[kFoUnroll];
#pragma unroll
  for (int u = 0; u < kFoUnroll; ++u) {
    const long long c = c0 + u * stride;
    const bool in = c < s1;
    vr[u] = in ? r[c] : 0.0;
    vd[u] = in ? diag[c] : 1.0;
    vp[u] = in ? p[c] : 0.0;
  }
  const double rz = sum_parts(part_rz, n_part), rz_old = sc[S_RZ + slot];
  const double beta = rz_old > 0.0 ? rz / rz_old : 0.0;
  if (blockIdx.x == 0) {
    const double rr = sum_parts(part_rr, n_part);
    if (threadIdx.x == 0) {
      sc[S_RZ + (slot ^ 1)] = rz;
      sc[S_RR] = rr;
    }
  }
#pragma unroll
  for (int u = 0; u < kFoUnroll; ++u) {
    const long long c = c0 + u * stride;
    if (c < s1) p[c] = vr[u] / vd[u] + beta * vp[u];
  }
  for (long long c = c0 + kFoUnroll * stride; c < s1; c += stride) p[c] = r[c] / diag[c] + beta * p[c];
}

__global__ void __launch_bounds__(kFoBlock) k_fo_temperature(long long nc, const double* __restrict__ kap,
                                                             const double* __restrict__ x, double T_sink,
                                                             double* __restrict__ T) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < nc; c += (long long)gridDim.x * blockDim.x)
    T[c] = kap[c] > 0.0 ? T_sink + x[c] : T_sink;
}

struct KapTable {
  double v[16];
};

__global__ void __launch_bounds__(kFoBlock) k_fo_chip_fields(const uint8_t* __restrict__ mat, KapTable kt, int n_mat,
                                                             const int32_t* __restrict__ src_index,
                                                             const double* __restrict__ src, int n_src, double scale,
                                                             long long nc, double* kap, double* q) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < nc; c += (long long)gridDim.x * blockDim.x) {
    const int m = mat[c];
    double k = 0.0;
#pragma unroll
    for (int t = 0; t < 16; ++t) k = (t == m && t < n_mat) ? kt.v[t] : k;
    kap[c] = k;
    const int s = src_index[c];
    q[c] = (s >= 0 && s < n_src) ? scale * src[s] : 0.0;
  }
}

struct FoLayout {
  size_t gx, gy, gz, diag, x, r, p, Ap, part0, part1, part2, held, sc, total;
};

bool fo_valid(const fo_config* c) {
  if (!c || c->max_iterations < 1 || !(c->rtol > 0.0) || !std::isfinite(c->T_sink_K) || !(c->R_K_m2KW >= 0.0) ||
      (c->warm_start != 0 && c->warm_start != 1))
    return false;
  long long nc = 1;
  for (int d = 0; d < 3; ++d) {
    if (c->n[d] < 1) return false;
    nc *= c->n[d];
  }
  if (nc > (1ll << 27)) return false;
  int any = 0;
  for (int f = 0; f < 6; ++f) {
    if (c->dirichlet[f] != 0 && c->dirichlet[f] != 1) return false;
    any |= c->dirichlet[f];
  }
  if (!any) return false;  // no sink: the rise is not determined
  return c->k_interface == -1 || (c->k_interface >= 1 && c->k_interface < c->n[2]);
}

FoLayout fo_layout(const fo_config* c) {
  FoLayout L;
  const size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
  size_t off = 0;
  auto take = [&](size_t b) { const size_t o = off; off += (b + 255) & ~(size_t)255; return o; };
  const size_t halo = (size_t)c->n[1] * c->n[2];  // one x-plane before and after: offsets are of cell 0
  L.gx = take(8 * (nc + 2 * halo)) + 8 * halo;
  L.gy = take(8 * (nc + 2 * halo)) + 8 * halo;
  L.gz = take(8 * (nc + 2 * halo)) + 8 * halo;
  L.diag = take(8 * nc);
  L.x = take(8 * nc);
  L.r = take(8 * nc);
  L.p = take(8 * (nc + 2 * halo)) + 8 * halo;
  L.Ap = take(8 * nc);
  L.part0 = take(8 * kFoMaxBlocks);
  L.part1 = take(8 * kFoMaxBlocks);
  L.part2 = take(8 * kFoMaxBlocks);
  L.held = take(4 * 6);
  L.sc = take(8 * S_N);
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

size_t fo_workspace_bytes(const fo_config* c) { return fo_valid(c) ? fo_layout(c).total : 0; }

int fo_chip_fields(const uint8_t* d_material, const double* h_kappa_by_material, int n_materials,
                   const int32_t* d_src_index, const double* d_src, int n_src, double scale, long long ncell,
                   double* d_kappa, double* d_q, void* stream) {
  if (!d_material || !h_kappa_by_material || n_materials < 1 || n_materials > 16 || !d_src_index || !d_src ||
      n_src < 1 || ncell < 1 || !d_kappa || !d_q || !std::isfinite(scale))
    return MC_E_ARG;
  KapTable kt;
  for (int t = 0; t < 16; ++t) kt.v[t] = t < n_materials ? h_kappa_by_material[t] : 0.0;
  for (int t = 0; t < n_materials; ++t)
    if (!(kt.v[t] >= 0.0) || !std::isfinite(kt.v[t])) return MC_E_ARG;
  long long need = (ncell + kFoBlock - 1) / kFoBlock;
  const int nb = (int)(need < kFoMaxBlocks ? need : kFoMaxBlocks);
  k_fo_chip_fields<<<nb, kFoBlock, 0, (hipStream_t)stream>>>(d_material, kt, n_materials, d_src_index, d_src, n_src,
                                                             scale, ncell, d_kappa, d_q);
  return hipGetLastError() == hipSuccess ? MC_OK : MC_E_HIP;
}

int fo_solve(const fo_config* c, const double* d_edges, const double* d_kappa, const double* d_q, double* d_T,
             int* iterations, double* rel_residual, void* d_ws, size_t ws_bytes, void* stream) {
  if (iterations) *iterations = 0;
  if (rel_residual) *rel_residual = 0.0;
  if (!fo_valid(c) || !d_edges || !d_kappa || !d_q || !d_T) return MC_E_ARG;
  const FoLayout L = fo_layout(c);
  if (!d_ws || ws_bytes < L.total || ((uintptr_t)d_ws & 255u)) return MC_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)d_ws;
  auto P = [&](size_t off) { return (double*)(ws + off); };
  FoGrid g;
  g.nx = c->n[0];
  g.ny = c->n[1];
  g.nz = c->n[2];
  g.nc = (long long)g.nx * g.ny * g.nz;
  g.ex = d_edges;
  g.ey = d_edges + g.nx + 1;
  g.ez = d_edges + g.nx + 1 + g.ny + 1;
  // workgroups of the solve: about kFoUnroll cells per thread, at most
  // kFoMaxBlocks, a multiple of 8 (one span per XCD in turn); cpw cells each,
  // a multiple of kFoBlock, so that nb cpw >= nc
  const long long need = (g.nc + (long long)kFoBlock * kFoUnroll - 1) / ((long long)kFoBlock * kFoUnroll);
  const int nb = (int)(((need < kFoMaxBlocks ? need : kFoMaxBlocks) + 7) / 8 * 8);
  const long long cpw = ((g.nc + nb - 1) / nb + kFoBlock - 1) / kFoBlock * kFoBlock;
  const long long sx = (long long)g.ny * g.nz, sy = g.nz;
  if (hipMemcpyAsync(ws + L.held, c->dirichlet, sizeof(int) * 6, hipMemcpyHostToDevice, st) != hipSuccess)
    return MC_E_HIP;
  double* sc = P(L.sc);
  k_fo_setup<<<nb, kFoBlock, 0, st>>>(g, (const int*)(ws + L.held), c->k_interface, c->R_K_m2KW, d_kappa, d_q,
                                     P(L.gx), P(L.gy), P(L.gz), P(L.diag), P(L.x), P(L.r), P(L.p), cpw, P(L.part0),
                                     P(L.part1));
  if (c->warm_start) {
    // r = b - A x0 for the rise d_T holds; the product's p.Ap partials are
    // not used
    k_fo_warm_x<<<nb, kFoBlock, 0, st>>>(g.nc, cpw, d_kappa, d_T, c->T_sink_K, P(L.p));
    k_fo_spmv<<<nb, kFoBlock, 0, st>>>(g.nc, cpw, sx, sy, P(L.gx), P(L.gy), P(L.gz), P(L.diag), P(L.p), P(L.Ap),
                                       P(L.part2));
    k_fo_warm_r<<<nb, kFoBlock, 0, st>>>(g.nc, cpw, P(L.diag), P(L.Ap), P(L.p), P(L.x), P(L.r), P(L.part0),
                                         P(L.part2));
    k_fo_start<<<1, kFoBlock, 0, st>>>(P(L.part0), P(L.part1), P(L.part2), nb, sc);
  } else {
    k_fo_start<<<1, kFoBlock, 0, st>>>(P(L.part0), P(L.part1), nullptr, nb, sc);
  }
  if (hipGetLastError() != hipSuccess) return MC_E_HIP;
  double h[S_N];
  if (hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return MC_E_HIP;
  const double bb = h[S_BB];
  int it = 0, rc = MC_OK;
  double rel = 0.0;
  if (bb > 0.0) {
    const double stop = c->rtol * c->rtol * bb;
    // partial sums: p.Ap in part2 (written by the product, read by the
    // update), r.z and r.r in part0 and part1 (written by the update, read by
    // the direction kernel); the direction of the last iteration is formed
    // but not used
    for (;;) {
      const int slot = it & 1;
      k_fo_spmv<<<nb, kFoBlock, 0, st>>>(g.nc, cpw, sx, sy, P(L.gx), P(L.gy), P(L.gz), P(L.diag), P(L.p), P(L.Ap),
                                         P(L.part2));
      k_fo_update<<<nb, kFoBlock, 0, st>>>(g.nc, cpw, slot, P(L.part2), nb, sc, P(L.diag), P(L.p), P(L.Ap), P(L.x),
                                          P(L.r), P(L.part0), P(L.part1));
      k_fo_direction<<<nb, kFoBlock, 0, st>>>(g.nc, cpw, slot, P(L.part0), P(L.part1), nb, sc, P(L.diag), P(L.r),
                                             P(L.p));
      ++it;
      const bool check = it % kFoCheck == 0 || it == c->max_iterations;
      if (check) {
        if (hipGetLastError() != hipSuccess) return MC_E_HIP;
        if (hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          return MC_E_HIP;
        if (h[S_RR] <= stop) break;
        if (it >= c->max_iterations) {
          rc = MC_E_RANGE;
          break;
        }
      }
    }
    rel = std::sqrt(h[S_RR] / bb);
  }
  k_fo_temperature<<<nb, kFoBlock, 0, st>>>(g.nc, d_kappa, P(L.x), c->T_sink_K, d_T);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return MC_E_HIP;
  if (iterations) *iterations = it;
  if (rel_residual) *rel_residual = rel;
  return rc;
}

}  // extern "C"
