// sg_kernels.h -- gfx950 kernels of the MLP surrogate that maps a bias point
// (Vgs, Vds, log10 doping, per-subcell lattice temperature) to the per-subcell
// heat and electron-density maps of the Monte Carlo.  BF16 operands on the
// matrix cores (v_mfma_f32_32x32x16_bf16) with FP32 accumulation; FP32 master
// weights and Adam moments.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Depth of the K slabs staged in LDS: 128 for the 64 x 64 workgroup tiles
// (each global round trip then feeds twice the matrix-core work of a 64-deep
// slab, at 128 registers per lane and 35 KB of LDS per workgroup), 64 for the
// 128 x 128 tiles (128-deep slabs would need 280 registers per lane: one
// wavefront per SIMD).  Rows of a slab are padded by 8 elements (16 bytes).
template <int TM> constexpr int slab_depth() { return TM == 32 ? 128 : 64; }

// LDS position of the 8-element k-chunk c (0..CPR-1) of tile row r: chunks
// are permuted within groups of 8 of the row by r / 8, so that the 2-byte
// stores of a transposed operand (lanes 8 rows apart) fall into different
// banks; a chunk stays contiguous for the 16-byte fragment reads.
template <int KP>
__device__ __forceinline__ int lds_at(int r, int c) { return r * KP + ((c ^ ((r >> 3) & 7)) << 3); }

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3, EPI_BIAS_GELU_ONLY = 4 };

struct GemmArgs {
  const bf16* A;
  long lda;
  const bf16* B;
  long ldb;
  int M, N, K;
  float* Cf;
  long ldcf;
  bf16* Cb;
  long ldcb;
  const float* bias;
  const float* Z;  // pre-activations for the GELU derivative
  long ldz;
  // split K (k_gemm, store epilogue): workgroup z of the grid's z range
  // takes k in [z kz, (z + 1) kz) and stores its partial product at
  // Cf + z zs; 0: no split
  int kz;
  long zs;
};

// GELU with the exact normal CDF: x Phi(x)
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
// d/dx [x Phi(x)] = Phi(x) + x phi(x)
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// Eight consecutive BF16 of row r, columns c .. c+7, of a [R x C] matrix with
// leading dimension ld (a multiple of 8): one 16-byte load when the chunk is
// inside, element loads with zero fill at ragged edges.
__device__ __forceinline__ uint4 load_chunk(const bf16* p, long ld, int r, int c, int R, int C) {
  if (r < R && c + 8 <= C) return *reinterpret_cast<const uint4*>(p + (long)r * ld + c);
  uint4 v;
  bf16* e = reinterpret_cast<bf16*>(&v);
#pragma unroll
  for (int q = 0; q < 8; ++q) e[q] = (r < R && c + q < C) ? p[(long)r * ld + c + q] : (bf16)0.0f;
  return v;
}

// The 32 x 32 block of C at (r0, c0) held by one wavefront's accumulator
// (lane l, item j: row 8 (j / 4) + 4 (l / 32) + j % 4, column l % 32), with
// the product's epilogue: store, + bias, + bias and GELU (pre-activation in
// FP32 and activation in BF16, or, for passes without a backward, the
// activation alone), or times the GELU derivative.
template <int EPI>
__device__ __forceinline__ void epilogue(const GemmArgs& g, const f32x16& acc, int r0, int c0, int lane) {
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int row = r0 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
    const int col = c0 + (lane & 31);
    if (row >= g.M || col >= g.N) continue;
    const float v = acc[j];
    if (EPI == EPI_STORE) {
      g.Cf[(long)row * g.ldcf + col] = v;
    } else if (EPI == EPI_BIAS) {
      g.Cf[(long)row * g.ldcf + col] = v + g.bias[col];
    } else if (EPI == EPI_BIAS_GELU) {
      const float z = v + g.bias[col];
      g.Cf[(long)row * g.ldcf + col] = z;
      g.Cb[(long)row * g.ldcb + col] = (bf16)gelu(z);
    } else if (EPI == EPI_BIAS_GELU_ONLY) {
      g.Cb[(long)row * g.ldcb + col] = (bf16)gelu(v + g.bias[col]);
    } else {
      g.Cb[(long)row * g.ldcb + col] = (bf16)(v * gelu_grad(g.Z[(long)row * g.ldz + col]));
    }
  }
}

// C[M x N] = opA(A)[M x K] opB(B)[K x N], BF16 in, FP32 accumulate, with an
// epilogue.  opA(i,k) = A[i*lda + k] (TA false) or A[k*lda + i] (TA true);
// opB(k,j) = B[k*ldb + j] (TB false) or B[j*ldb + k] (TB true).
// Workgroup tile 2 TM x 2 TM x 64, four waves of TM x TM (TM = 64: 2 x 2
// MFMA blocks each; TM = 32: one), TM = 32 for products whose 128 x 128
// tiles would leave compute units idle.  The next K slab is loaded into
// registers while the matrix cores work on the current one from LDS (LDS
// holds A as [i][k] and B as [j][k]).
template <bool TA, bool TB, int EPI, int TM>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
  constexpr int BK = slab_depth<TM>(), KP = BK + 8, CPR = BK / 8;
  if (g.kz > 0) {
    const int k0 = (int)blockIdx.z * g.kz;
    g.A += TA ? (long)k0 * g.lda : (long)k0;
    g.B += TB ? (long)k0 : (long)k0 * g.ldb;
    g.K = min(g.kz, g.K - k0);
    g.Cf += (long)blockIdx.z * g.zs;
  }
  constexpr int BM = 2 * TM, BN = 2 * TM, MB = TM / 32, NCH = BM * CPR / 256;
  __shared__ __attribute__((aligned(16))) bf16 As[BM * KP];
  __shared__ __attribute__((aligned(16))) bf16 Bs[BN * KP];  // n-major: Bs[n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * TM, wn = (wave & 1) * TM;
  f32x16 acc[MB][MB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[a][b][j] = 0.0f;
  // BM x CPR chunks of 8 elements per operand and slab, NCH per thread, along
  // each operand's contiguous dimension (a row of BK k is CPR chunks; a row of
  // BM elements is BM / 8)
  constexpr int RS = BM / 8;  // chunks per row of the transposed operands
  uint4 ra[NCH], rb[NCH];
  auto fetch_fast = [&](int k0) {  // every chunk of the slab in range
#pragma unroll
    for (int rep = 0; rep < NCH; ++rep) {
      const int ch = tid + 256 * rep;
      ra[rep] = !TA ? *reinterpret_cast<const uint4*>(g.A + (long)(m0 + ch / CPR) * g.lda + k0 + (ch % CPR) * 8)
                    : *reinterpret_cast<const uint4*>(g.A + (long)(k0 + ch / RS) * g.lda + m0 + (ch % RS) * 8);
      rb[rep] = TB ? *reinterpret_cast<const uint4*>(g.B + (long)(n0 + ch / CPR) * g.ldb + k0 + (ch % CPR) * 8)
                   : *reinterpret_cast<const uint4*>(g.B + (long)(k0 + ch / RS) * g.ldb + n0 + (ch % RS) * 8);
    }
  };
  auto fetch_checked = [&](int k0) {  // ragged edges: zero fill
#pragma unroll
    for (int rep = 0; rep < NCH; ++rep) {
      const int ch = tid + 256 * rep;
      ra[rep] = !TA ? load_chunk(g.A, g.lda, m0 + ch / CPR, k0 + (ch % CPR) * 8, g.M, g.K)
                    : load_chunk(g.A, g.lda, k0 + ch / RS, m0 + (ch % RS) * 8, g.K, g.M);
      rb[rep] = TB ? load_chunk(g.B, g.ldb, n0 + ch / CPR, k0 + (ch % CPR) * 8, g.N, g.K)
                   : load_chunk(g.B, g.ldb, k0 + ch / RS, n0 + (ch % RS) * 8, g.K, g.N);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int rep = 0; rep < NCH; ++rep) {
      const int ch = tid + 256 * rep;
      if (!TA) {
        *reinterpret_cast<uint4*>(As + lds_at<KP>(ch / CPR, ch % CPR)) = ra[rep];
      } else {
        const bf16* pv = reinterpret_cast<const bf16*>(&ra[rep]);
        const int kk = ch / RS, ic = (ch % RS) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) As[lds_at<KP>(ic + e, kk >> 3) + (kk & 7)] = pv[e];
      }
      if (TB) {
        *reinterpret_cast<uint4*>(Bs + lds_at<KP>(ch / CPR, ch % CPR)) = rb[rep];
      } else {
        const bf16* pv = reinterpret_cast<const bf16*>(&rb[rep]);
        const int kk = ch / RS, jc = (ch % RS) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) Bs[lds_at<KP>(jc + e, kk >> 3) + (kk & 7)] = pv[e];
      }
    }
  };
  auto mma = [&]() {
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      bf16x8 a[MB], b[MB];
#pragma unroll
      for (int mi = 0; mi < MB; ++mi)
        a[mi] = *reinterpret_cast<const bf16x8*>(As + lds_at<KP>(wm + mi * 32 + (lane & 31), (ks >> 3) + (lane >> 5)));
#pragma unroll
      for (int ni = 0; ni < MB; ++ni)
        b[ni] = *reinterpret_cast<const bf16x8*>(Bs + lds_at<KP>(wn + ni * 32 + (lane & 31), (ks >> 3) + (lane >> 5)));
#pragma unroll
      for (int mi = 0; mi < MB; ++mi)
#pragma unroll
        for (int ni = 0; ni < MB; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
  };
  // Interior workgroups (rows and columns in range) run the whole slabs with
  // plain 16-byte loads, the next slab's loads in flight during the current
  // slab's matrix-core work; the ragged last slab, and every slab of an edge
  // workgroup, take the checked loads.
  const int kfull = (m0 + BM <= g.M && n0 + BN <= g.N) ? (g.K / BK) * BK : 0;
  if (kfull > 0) {
    fetch_fast(0);
    for (int k0 = 0; k0 < kfull; k0 += BK) {
      stash();
      __syncthreads();
      if (k0 + BK < kfull) fetch_fast(k0 + BK);
      mma();
      __syncthreads();
    }
  }
  for (int k0 = kfull; k0 < g.K; k0 += BK) {
    fetch_checked(k0);
    stash();
    __syncthreads();
    mma();
    __syncthreads();
  }
#pragma unroll
  for (int mi = 0; mi < MB; ++mi)
#pragma unroll
    for (int ni = 0; ni < MB; ++ni) epilogue<EPI>(g, acc[mi][ni], m0 + wm + mi * 32, n0 + wn + ni * 32, lane);
}

// ---------------------------------------------------------------------------
// Products whose operands are both K-contiguous (A [M][K], B [N][K]: the
// forward products and dX): the K slabs go from global memory straight into
// LDS (global_load_lds_dwordx4: each lane's 16 bytes land at the wavefront's
// LDS base + 16 x lane), so no registers stage them; the next slabs' copies
// are in flight while the matrix cores work on the current one (S stages per
// workgroup).  These products are bound by how fast operand tiles reach the
// compute units from L2 (about 14 B per clock per CU measured), a rate that
// grows with the wavefronts issuing copies and not with the stages in flight,
// so the tiles are as large as the product allows while every compute unit
// still gets work (256 x 256, 128 x 128 or 128 x 64), with up to 16
// wavefronts per tile, and each XCD takes a
// contiguous eighth of the tiles (a few row tiles by all column tiles), so
// that its operands stay in its own L2.  Rows and K chunks outside the
// matrices read a 16-byte block of zeros.  K must be a multiple of 8.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

static __device__ __attribute__((aligned(16))) const uint4 g_zero16[1] = {{0u, 0u, 0u, 0u}};

// s_waitcnt with vmcnt <= n (expcnt and lgkmcnt not waited for)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

constexpr int kLdsBK = 64;
constexpr int kLdsChunks = kLdsBK / 8;                   // 16-byte chunks per slab row
// bytes of a workgroup's LDS: S stages, each an A slab of BM rows and a B
// slab of BN rows
template <int BM, int BN, int S = 2> constexpr int lds_bytes() { return S * (BM + BN) * kLdsChunks * 16; }

// LDS position (16-byte units) of chunk c of slab row r: chunks permuted by
// r & 7 within the row, so the fragment reads of 8 consecutive rows at one
// chunk fall on distinct bank groups
__device__ __forceinline__ int lds_pos(int r, int c) { return r * kLdsChunks + (c ^ (r & 7)); }

__host__ __device__ inline int lds_tiles(int M, int N, int BM, int BN) {
  return ((N + BN - 1) / BN) * ((M + BM - 1) / BM);
}

// Tile BM x BN with W wavefronts: 2 rows of W / 2 wavefronts, each
// BM / 2 x 2 BN / W, in 32 x 32 MFMA blocks.  S stages of LDS: while the
// matrix cores work on slab s, the copies of slabs s + 1 .. s + S - 1 are in
// flight.
template <int EPI, int BM, int BN, int W, int S = 2>
__global__ void __launch_bounds__(64 * W) k_gemm_lds(GemmArgs g) {
  constexpr int WM = BM / 2, WN = 2 * BN / W;      // a wavefront's share of the tile
  constexpr int MB = WM / 32, NB = WN / 32;        // its 32 x 32 MFMA blocks
  constexpr int SA = BM * kLdsChunks * 16, SB = BN * kLdsChunks * 16;
  constexpr int BA = BM / 8 / W, BB = BN / 8 / W;  // 1 KB blocks per wavefront and stage
  constexpr int LB = BA + BB;                      // copies per wavefront and stage
  static_assert(BA * W * 8 == BM && BB * W * 8 == BN, "slab rows must split evenly over the wavefronts");
  static_assert(S >= 2 && (S - 2) * LB <= 63, "vmcnt counts at most 63 copies in flight");
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // workgroup w runs on XCD w % 8; XCD x takes tiles [x per, (x + 1) per)
  const int gx = (g.N + BN - 1) / BN, T = lds_tiles(g.M, g.N, BM, BN), per = (T + 7) / 8;
  const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (t >= T) return;
  const int m0 = (t / gx) * BM, n0 = (t % gx) * BN;
  const int wm = (wave / (W / 2)) * WM, wn = (wave % (W / 2)) * WN;
  const int nk = (g.K + kLdsBK - 1) / kLdsBK;
  // one stage: 1 KB blocks of 8 slab rows spread over the wavefronts; lane l
  // of a block fills LDS unit l, i.e. row l / 8, the chunk that lds_pos puts
  // there
  auto copy = [&](const bf16* P, long ld, int rows, int row0, char* dst, int blk, int k0) {
    const int u = blk * 64 + lane;
    const int r = u / kLdsChunks, c = (u % kLdsChunks) ^ (r & 7);
    const int kk = k0 + c * 8;
    const bf16* p = (row0 + r < rows && kk < g.K) ? P + (long)(row0 + r) * ld + kk : (const bf16*)g_zero16;
    __builtin_amdgcn_global_load_lds((glb_void_t*)p, (lds_void_t*)(dst + blk * 1024), 16, 0, 0);
  };
  auto issue = [&](int s) {
    char* sa = lds + (s % S) * (SA + SB);
    char* sb = sa + SA;
    const int k0 = s * kLdsBK;
#pragma unroll
    for (int i = 0; i < BA; ++i) copy(g.A, g.lda, g.M, m0, sa, wave * BA + i, k0);
#pragma unroll
    for (int i = 0; i < BB; ++i) copy(g.B, g.ldb, g.N, n0, sb, wave * BB + i, k0);
  };
  f32x16 acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[a][b][j] = 0.0f;
  for (int s = 0; s < S - 1 && s < nk; ++s) issue(s);
  for (int s = 0; s < nk; ++s) {
    // this wavefront's copies of slab s have landed: the copies issued after
    // them (slabs s + 1 .. s + S - 2, LB each, in order) may still be in
    // flight, and near the end, where fewer were issued, nothing is.  The
    // barrier then covers every wavefront's copies, and every wavefront is
    // done reading the buffer that slab s + S - 1 goes into, slab s - 1's (a
    // plain barrier: a fence would also wait for stores that need not finish)
    if (s + S - 2 < nk)
      wait_vmcnt<(S - 2) * LB>();
    else
      wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if (s + S - 1 < nk) issue(s + S - 1);
    const bf16* sa = (const bf16*)(lds + (s % S) * (SA + SB));
    const bf16* sb = (const bf16*)(lds + (s % S) * (SA + SB) + SA);
#pragma unroll
    for (int ks = 0; ks < kLdsBK / 16; ++ks) {
      const int ch = ks * 2 + (lane >> 5);
      bf16x8 a[MB], b[NB];
#pragma unroll
      for (int mi = 0; mi < MB; ++mi) {
        const int r = wm + mi * 32 + (lane & 31);
        a[mi] = *reinterpret_cast<const bf16x8*>(sa + lds_pos(r, ch) * 8);
      }
#pragma unroll
      for (int ni = 0; ni < NB; ++ni) {
        const int r = wn + ni * 32 + (lane & 31);
        b[ni] = *reinterpret_cast<const bf16x8*>(sb + lds_pos(r, ch) * 8);
      }
#pragma unroll
      for (int mi = 0; mi < MB; ++mi)
#pragma unroll
        for (int ni = 0; ni < NB; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mi = 0; mi < MB; ++mi)
#pragma unroll
    for (int ni = 0; ni < NB; ++ni) epilogue<EPI>(g, acc[mi][ni], m0 + wm + mi * 32, n0 + wn + ni * 32, lane);
}

// Normalised BF16 input rows: (x - mean) / std, zero padding to ldx.
// Column k of the grid's x range, rows 4 blockIdx.y .. 4 blockIdx.y + 3: the
// four loads are issued before the stores (15.6 -> 11.5 us at 4096 x 1803
// against one element per thread with a 64-bit index division).
constexpr int kInRows = 4;
__global__ void k_input(const float* __restrict__ x, int M, int n_in, const float* __restrict__ mean,
                        const float* __restrict__ stdv, bf16* X0, int ldx) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ldx) return;
  const bool in = k < n_in;
  const float mu = in ? mean[k] : 0.0f, sd = in ? stdv[k] : 1.0f;
  const int i0 = blockIdx.y * kInRows;
  float v[kInRows];
#pragma unroll
  for (int r = 0; r < kInRows; ++r) v[r] = (in && i0 + r < M) ? x[(long)(i0 + r) * n_in + k] : 0.0f;
#pragma unroll
  for (int r = 0; r < kInRows; ++r)
    if (i0 + r < M) X0[(long)(i0 + r) * ldx + k] = (bf16)(in ? (v[r] - mu) / sd : 0.0f);
}

// MSE on z-scored targets; writes dL/dpred (BF16, row stride np, a multiple
// of 8, zero in the padding columns) and per-workgroup loss sums.  Thread t
// of the grid's x range takes columns 4t .. 4t+3 of rows blockIdx.y,
// blockIdx.y + gridDim.y, ...: 16-byte loads when n_out is a multiple of 4
// and both inputs are 16-byte aligned (every row then is), 8-byte stores.
// Workgroup (x, y)'s sum goes to loss_part[y gridDim.x + x].
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ pred, const float* __restrict__ y, int M,
                                              int n_out, int np, const float* __restrict__ ymean,
                                              const float* __restrict__ ystd, bf16* dpred, float* loss_part) {
  __shared__ float s[4];
  const int j0 = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
  float l = 0.0f;
  if (j0 < np) {
    float mu[4], sd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool out = j0 + q < n_out;
      mu[q] = out ? ymean[j0 + q] : 0.0f;
      sd[q] = out ? ystd[j0 + q] : 1.0f;
    }
    const float n = (float)((long)M * n_out);
    const bool vec = (n_out & 3) == 0 && j0 + 4 <= n_out && (((uintptr_t)pred | (uintptr_t)y) & 15) == 0;
#pragma unroll 4
    for (int i = blockIdx.y; i < M; i += gridDim.y) {
      const long o = (long)i * n_out + j0;
      float pv[4], yv[4];
      if (vec) {
        const float4 a = *reinterpret_cast<const float4*>(pred + o), b = *reinterpret_cast<const float4*>(y + o);
        pv[0] = a.x; pv[1] = a.y; pv[2] = a.z; pv[3] = a.w;
        yv[0] = b.x; yv[1] = b.y; yv[2] = b.z; yv[3] = b.w;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          pv[q] = j0 + q < n_out ? pred[o + q] : 0.0f;
          yv[q] = j0 + q < n_out ? y[o + q] : 0.0f;
        }
      }
      bf16 g[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        g[q] = (bf16)0.0f;
        if (j0 + q < n_out) {
          const float t = (yv[q] - mu[q]) / sd[q];
          const float d = pv[q] - t;
          l += d * d;
          g[q] = (bf16)(2.0f * d / n);
        }
      }
      *reinterpret_cast<uint2*>(dpred + (long)i * np + j0) = *reinterpret_cast<const uint2*>(g);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) loss_part[blockIdx.y * gridDim.x + blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// out[i] = part[i] + part[zs + i] + ... + part[(S - 1) zs + i], in that
// order (the split-K partial products of one GEMM, S <= 8): the S loads are
// in flight before their adds
__global__ void k_split_sum(const float* __restrict__ part, int S, long n, long zs, float* __restrict__ out) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float v[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) v[z] = z < S ? part[z * zs + i] : 0.0f;
    float t = v[0];
#pragma unroll
    for (int z = 1; z < 8; ++z)
      if (z < S) t += v[z];
    out[i] = t;
  }
}

// Column sums of a BF16 [M x N] gradient (bias gradient): one workgroup of
// kCsRows x 64 lanes per 64 columns and row block y (rows [y rp, (y + 1) rp)
// of the grid's y range); lane group r sums rows r, r + kCsRows, ... of the
// block (independent loads, unrolled), and the groups' sums are added in
// group order.  One row block writes out; several write part[y][N], which
// k_colsum_reduce adds in block order, so the result does not depend on
// timing.
constexpr int kCsRows = 16;
__global__ void __launch_bounds__(64 * kCsRows) k_colsum(const bf16* __restrict__ d, int M, int N, long ld, int rp,
                                                          float* out, float* part) {
  __shared__ float acc[kCsRows][64];
  const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + c;
  const int i0 = (int)blockIdx.y * rp, i1 = min(M, i0 + rp);
  float s = 0.0f;
  if (j < N) {
#pragma unroll 8
    for (int i = i0 + r; i < i1; i += kCsRows) s += (float)d[(long)i * ld + j];
  }
  acc[r][c] = s;
  __syncthreads();
  if (r == 0 && j < N) {
    float t = 0.0f;
#pragma unroll
    for (int g = 0; g < kCsRows; ++g) t += acc[g][c];
    if (gridDim.y == 1) out[j] = t;
    else part[(long)blockIdx.y * N + j] = t;
  }
}

// out[j] = part[0][j] + part[1][j] + ... in row-block order; eight loads in
// flight before their adds
__global__ void k_colsum_reduce(const float* __restrict__ part, int R, int N, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float t = 0.0f;
  for (int y0 = 0; y0 < R; y0 += 8) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = y0 + q < R ? part[(long)(y0 + q) * N + j] : 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (y0 + q < R) t += v[q];
  }
  out[j] = t;
}

// Adam (bias-corrected) on FP32 master weights with decoupled weight decay
// wd (Loshchilov & Hutter), then the BF16 copy.
__device__ __forceinline__ float adam_one(float& w, float& m, float& v, float g, float lr, float b1, float b2, float eps,
                                          float c1, float c2, float wd) {
  m = b1 * m + (1.0f - b1) * g;
  v = b2 * v + (1.0f - b2) * g * g;
  w = w - lr * ((m / c1) / (sqrtf(v / c2) + eps) + wd * w);
  return w;
}

// Four elements per thread: 16-byte loads and stores where the four are in
// range (the buffers are 256-byte aligned), one at a time at the tail.
__global__ void k_adam(float* w, float* m, float* v, const float* __restrict__ g, bf16* wb, long n, float lr,
                       float b1, float b2, float eps, float c1, float c2, float wd) {
  const long i0 = 4 * ((long)blockIdx.x * blockDim.x + threadIdx.x);
  if (i0 >= n) return;
  if (i0 + 4 <= n) {
    const float4 G = *reinterpret_cast<const float4*>(g + i0);
    float4 W = *reinterpret_cast<const float4*>(w + i0), M = *reinterpret_cast<const float4*>(m + i0),
           V = *reinterpret_cast<const float4*>(v + i0);
    adam_one(W.x, M.x, V.x, G.x, lr, b1, b2, eps, c1, c2, wd);
    adam_one(W.y, M.y, V.y, G.y, lr, b1, b2, eps, c1, c2, wd);
    adam_one(W.z, M.z, V.z, G.z, lr, b1, b2, eps, c1, c2, wd);
    adam_one(W.w, M.w, V.w, G.w, lr, b1, b2, eps, c1, c2, wd);
    *reinterpret_cast<float4*>(m + i0) = M;
    *reinterpret_cast<float4*>(v + i0) = V;
    *reinterpret_cast<float4*>(w + i0) = W;
    if (wb) {
      bf16 o[4] = {(bf16)W.x, (bf16)W.y, (bf16)W.z, (bf16)W.w};
      *reinterpret_cast<uint2*>(wb + i0) = *reinterpret_cast<const uint2*>(o);
    }
  } else {
    for (long i = i0; i < n; ++i) {
      float wi = w[i], mi = m[i], vi = v[i];
      adam_one(wi, mi, vi, g[i], lr, b1, b2, eps, c1, c2, wd);
      m[i] = mi;
      v[i] = vi;
      w[i] = wi;
      if (wb) wb[i] = (bf16)wi;
    }
  }
}

// N-major copy of a BF16 weight matrix: out[c][r] = in[r][c] for in R x C
// (row-major), through 32 x 32 LDS tiles (blockDim 32 x 8).  The forward
// products read their weights N-major, so that both operands of the GEMM are
// staged with 16-byte LDS stores along K.
__global__ void __launch_bounds__(256) k_transpose_bf16(const uint16_t* __restrict__ in, int R, int C,
                                                        uint16_t* __restrict__ out) {
  __shared__ uint16_t t[32][34];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int r = r0 + i, col = c0 + threadIdx.x;
    if (r < R && col < C) t[i][threadIdx.x] = in[(long)r * C + col];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int col = c0 + i, r = r0 + threadIdx.x;
    if (col < C && r < R) out[(long)col * R + r] = t[threadIdx.x][i];
  }
}

// Counter-based uniform initialisation U(-a, a) of FP32 master weights.
__global__ void k_init_weights(float* w, bf16* wb, long n, float a, uint32_t key0, uint32_t key1, uint32_t tag) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32), c2 = 0u, c3 = tag, k0 = key0, k1 = key1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  const float u = ((float)(c0 >> 8) + 0.5f) * (1.0f / 16777216.0f);
  const float wi = a * (2.0f * u - 1.0f);
  w[i] = wi;
  wb[i] = (bf16)wi;
}

// Ensemble mean and spread of de-normalised predictions.
__global__ void k_ensemble(const float* __restrict__ preds, int E, long per, int n_out, const float* __restrict__ ymean,
                           const float* __restrict__ ystd, float* mean_out, float* std_out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per) return;
  const int j = (int)(e % n_out);
  // two passes in normalised units: the spread is often far below the mean
  // (a one-pass sum of squares would cancel), and de-normalised values
  // (~1e24 for densities in m^-3) would overflow FP32 when squared
  float s = 0.0f;
  for (int q = 0; q < E; ++q) s += preds[q * per + e];
  const float mu = s / E;
  float s2 = 0.0f;
  for (int q = 0; q < E; ++q) {
    const float d = preds[q * per + e] - mu;
    s2 += d * d;
  }
  mean_out[e] = mu * ystd[j] + ymean[j];
  if (std_out) std_out[e] = E > 1 ? sqrtf(s2 / (E - 1)) * ystd[j] : 0.0f;
}

// ---------------------------------------------------------------------------
// Small-batch inference (M <= kSmallM rows): each layer is a stream over its
// BF16 weights, so it runs as a split-K GEMV across all ensemble members in
// one launch (grid: column blocks x K splits x members; one wavefront per
// workgroup, 8 consecutive columns per lane read as one 16-byte load), with
// FP32 partial sums per split and a second kernel that adds the splits in a
// fixed order and applies the bias (and GELU) epilogue.
constexpr int kSmallM = 8;
constexpr int kGvCols = 512;   // columns per wavefront
constexpr int kGvMaxSplit = 64;
constexpr int kMaxMembers = 16;

struct GemvArgs {
  const bf16* X;   // [member][M][ldx] (xse = 0: one input shared by all members)
  long ldx, xse;
  const bf16* W[kMaxMembers];  // [K][ldw] per member
  long ldw;
  int M, N, K, S;
  float* P;        // partials [member][S][M][N]
};

__device__ __forceinline__ void bf16x8_to_f32(const uint4 v, float* f) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    f[2 * i] = __uint_as_float(w[i] << 16);
    f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
}

template <int MT>
__global__ void __launch_bounds__(64) k_gemv(GemvArgs g) {
  const int e = blockIdx.z, s = blockIdx.y;
  const int n = blockIdx.x * kGvCols + 8 * (int)threadIdx.x;
  const int kc = (g.K + g.S - 1) / g.S, k0 = s * kc, k1 = min(g.K, k0 + kc);
  const bf16* __restrict__ W = g.W[e];
  const bf16* __restrict__ X = g.X + (long)e * g.xse;
  float acc[MT][8];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[m][j] = 0.0f;
  if (n >= g.N) return;  // N is a multiple of 8: a lane owns 8 columns or none
  int k = k0;
  for (; k + 4 <= k1; k += 4) {
    uint4 wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) wv[u] = *reinterpret_cast<const uint4*>(W + (long)(k + u) * g.ldw + n);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float wf[8];
      bf16x8_to_f32(wv[u], wf);
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const float xm = m < g.M ? (float)X[(long)m * g.ldx + k + u] : 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[m][j] = fmaf(xm, wf[j], acc[m][j]);
      }
    }
  }
  for (; k < k1; ++k) {
    float wf[8];
    bf16x8_to_f32(*reinterpret_cast<const uint4*>(W + (long)k * g.ldw + n), wf);
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const float xm = m < g.M ? (float)X[(long)m * g.ldx + k] : 0.0f;
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[m][j] = fmaf(xm, wf[j], acc[m][j]);
    }
  }
  float* P = g.P + ((long)e * g.S + s) * g.M * g.N;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    if (m >= g.M) break;
    float4* d = reinterpret_cast<float4*>(P + (long)m * g.N + n);
    d[0] = make_float4(acc[m][0], acc[m][1], acc[m][2], acc[m][3]);
    d[1] = make_float4(acc[m][4], acc[m][5], acc[m][6], acc[m][7]);
  }
}

struct GemvReduceArgs {
  const float* P;  // [member][S][M][N]
  int S, M, N, n_valid, E;
  const float* bias[kMaxMembers];
  float* outf;     // last layer: FP32 [member][M][ldo] (members ofs_e apart)
  bf16* outb;      // hidden layer: BF16 GELU activations [member][M][ldo]
  long ldo, ofs_e;
};

template <bool LAST>
__global__ void k_gemv_reduce(GemvReduceArgs r) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)r.M * r.n_valid;
  if (idx >= per * r.E) return;
  const int e = (int)(idx / per);
  const long rem = idx % per;
  const int m = (int)(rem / r.n_valid), n = (int)(rem % r.n_valid);
  const float* P = r.P + (long)e * r.S * r.M * r.N + (long)m * r.N + n;
  float acc = 0.0f;
  for (int s = 0; s < r.S; ++s) acc += P[(long)s * r.M * r.N];
  const float z = acc + r.bias[e][n];
  if (LAST) r.outf[e * r.ofs_e + (long)m * r.ldo + n] = z;
  else r.outb[e * r.ofs_e + (long)m * r.ldo + n] = (bf16)gelu(z);
}

}  // namespace sg
