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
// streaming HBM (about 90 B per cell and iteration).  Dot products go
// through per-workgroup partial sums added in a fixed order, so a solve gives
// the same bits for any launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/gfmc.h"
#include "../../include/gffo.h"

namespace {

constexpr int kFoBlock = 256;
constexpr int kFoMaxBlocks = 4096;  // partial sums per dot product
constexpr int kFoCheck = 25;        // iterations between convergence checks on the host

struct FoGrid {
  int nx, ny, nz;
  long long nc;
  const double* ex;  // nx + 1 edges
  const double* ey;  // ny + 1
  const double* ez;  // nz + 1
};

// Scalars of the iteration, on the device.
enum { S_RZ = 0, S_PAP, S_ALPHA, S_BETA, S_RR, S_BB, S_N };

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

// Block sum in a fixed tree order into part[blockIdx.x].
__device__ inline void block_sum(double v, double* part) {
  __shared__ double s[kFoBlock];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = kFoBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// Conductances to the +x, +y, +z neighbours, the diagonal (with the held
// faces), and the start of the iteration: x = 0, r = b = q (0 in voids),
// p = r / diag; partial sums of r.z and b.b.
__global__ void __launch_bounds__(kFoBlock) k_fo_setup(FoGrid g, const int* __restrict__ held, int k_if, double R_K,
                                                       const double* __restrict__ kap, const double* __restrict__ q,
                                                       double* gx, double* gy, double* gz, double* diag, double* x,
                                                       double* r, double* p, double* part_rz, double* part_bb) {
  double rz = 0.0, bb = 0.0;
  const long long sx = (long long)g.ny * g.nz, sy = g.nz;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < g.nc;
       c += (long long)gridDim.x * blockDim.x) {
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
  block_sum(rz, part_rz);
  __syncthreads();
  block_sum(bb, part_bb);
}

// Ap = A p and partial sums of p.Ap
__global__ void __launch_bounds__(kFoBlock) k_fo_spmv(FoGrid g, const double* __restrict__ gx,
                                                      const double* __restrict__ gy, const double* __restrict__ gz,
                                                      const double* __restrict__ diag, const double* __restrict__ p,
                                                      double* __restrict__ Ap, double* part) {
  double acc = 0.0;
  const long long sx = (long long)g.ny * g.nz, sy = g.nz;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < g.nc;
       c += (long long)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_ijk(c, g, &i, &j, &k);
    const double pc = p[c];
    double a = diag[c] * pc;
    if (i + 1 < g.nx) a -= gx[c] * p[c + sx];
    if (i > 0) a -= gx[c - sx] * p[c - sx];
    if (j + 1 < g.ny) a -= gy[c] * p[c + sy];
    if (j > 0) a -= gy[c - sy] * p[c - sy];
    if (k + 1 < g.nz) a -= gz[c] * p[c + 1];
    if (k > 0) a -= gz[c - 1] * p[c - 1];
    Ap[c] = a;
    acc += pc * a;
  }
  block_sum(acc, part);
}

// One workgroup: the partial sums in a fixed order.
__device__ inline double sum_parts(const double* part, int n) {
  __shared__ double s[1024];
  double v = 0.0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) v += part[t];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  const double out = s[0];
  __syncthreads();
  return out;
}

__global__ void __launch_bounds__(1024) k_fo_start(const double* part_rz, const double* part_bb, int n, double* sc) {
  const double rz = sum_parts(part_rz, n), bb = sum_parts(part_bb, n);
  if (threadIdx.x == 0) {
    sc[S_RZ] = rz;
    sc[S_BB] = bb;
    sc[S_RR] = bb;
  }
}

__global__ void __launch_bounds__(1024) k_fo_alpha(const double* part, int n, double* sc) {
  const double pap = sum_parts(part, n);
  if (threadIdx.x == 0) {
    sc[S_PAP] = pap;
    sc[S_ALPHA] = pap > 0.0 ? sc[S_RZ] / pap : 0.0;
  }
}

// x += alpha p; r -= alpha Ap; partial sums of r.z (z = r / diag) and r.r
__global__ void __launch_bounds__(kFoBlock) k_fo_update(long long nc, const double* __restrict__ sc,
                                                        const double* __restrict__ diag, const double* __restrict__ p,
                                                        const double* __restrict__ Ap, double* __restrict__ x,
                                                        double* __restrict__ r, double* part_rz, double* part_rr) {
  const double alpha = sc[S_ALPHA];
  double rz = 0.0, rr = 0.0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < nc; c += (long long)gridDim.x * blockDim.x) {
    x[c] += alpha * p[c];
    const double rc = r[c] - alpha * Ap[c];
    r[c] = rc;
    rz += rc * (rc / diag[c]);
    rr += rc * rc;
  }
  block_sum(rz, part_rz);
  __syncthreads();
  block_sum(rr, part_rr);
}

__global__ void __launch_bounds__(1024) k_fo_beta(const double* part_rz, const double* part_rr, int n, double* sc) {
  const double rz = sum_parts(part_rz, n), rr = sum_parts(part_rr, n);
  if (threadIdx.x == 0) {
    sc[S_BETA] = sc[S_RZ] > 0.0 ? rz / sc[S_RZ] : 0.0;
    sc[S_RZ] = rz;
    sc[S_RR] = rr;
  }
}

// p = z + beta p
__global__ void __launch_bounds__(kFoBlock) k_fo_direction(long long nc, const double* __restrict__ sc,
                                                           const double* __restrict__ diag,
                                                           const double* __restrict__ r, double* __restrict__ p) {
  const double beta = sc[S_BETA];
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < nc; c += (long long)gridDim.x * blockDim.x)
    p[c] = r[c] / diag[c] + beta * p[c];
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
  size_t gx, gy, gz, diag, x, r, p, Ap, part0, part1, held, sc, total;
};

bool fo_valid(const fo_config* c) {
  if (!c || c->max_iterations < 1 || !(c->rtol > 0.0) || !std::isfinite(c->T_sink_K) || !(c->R_K_m2KW >= 0.0))
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
  L.gx = take(8 * nc);
  L.gy = take(8 * nc);
  L.gz = take(8 * nc);
  L.diag = take(8 * nc);
  L.x = take(8 * nc);
  L.r = take(8 * nc);
  L.p = take(8 * nc);
  L.Ap = take(8 * nc);
  L.part0 = take(8 * kFoMaxBlocks);
  L.part1 = take(8 * kFoMaxBlocks);
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
  long long need = (g.nc + kFoBlock - 1) / kFoBlock;
  const int nb = (int)(need < kFoMaxBlocks ? need : kFoMaxBlocks);
  if (hipMemcpyAsync(ws + L.held, c->dirichlet, sizeof(int) * 6, hipMemcpyHostToDevice, st) != hipSuccess)
    return MC_E_HIP;
  double* sc = P(L.sc);
  k_fo_setup<<<nb, kFoBlock, 0, st>>>(g, (const int*)(ws + L.held), c->k_interface, c->R_K_m2KW, d_kappa, d_q,
                                     P(L.gx), P(L.gy), P(L.gz), P(L.diag), P(L.x), P(L.r), P(L.p), P(L.part0),
                                     P(L.part1));
  k_fo_start<<<1, 1024, 0, st>>>(P(L.part0), P(L.part1), nb, sc);
  if (hipGetLastError() != hipSuccess) return MC_E_HIP;
  double h[S_N];
  if (hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return MC_E_HIP;
  const double bb = h[S_BB];
  int it = 0, rc = MC_OK;
  double rel = 0.0;
  if (bb > 0.0) {
    const double stop = c->rtol * c->rtol * bb;
    for (;;) {
      k_fo_spmv<<<nb, kFoBlock, 0, st>>>(g, P(L.gx), P(L.gy), P(L.gz), P(L.diag), P(L.p), P(L.Ap), P(L.part0));
      k_fo_alpha<<<1, 1024, 0, st>>>(P(L.part0), nb, sc);
      k_fo_update<<<nb, kFoBlock, 0, st>>>(g.nc, sc, P(L.diag), P(L.p), P(L.Ap), P(L.x), P(L.r), P(L.part0),
                                          P(L.part1));
      k_fo_beta<<<1, 1024, 0, st>>>(P(L.part0), P(L.part1), nb, sc);
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
      k_fo_direction<<<nb, kFoBlock, 0, st>>>(g.nc, sc, P(L.diag), P(L.r), P(L.p));
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
