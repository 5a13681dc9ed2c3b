// surrogate.hip -- host side of the MLP surrogate (sg_* in include/gfmc.h):
// workspace carving, weight initialisation, forward, loss and backward
// passes, Adam, ensemble prediction.  All arithmetic runs in sg_kernels.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gfmc.h"
#include "sg_kernels.h"

using namespace sg;

namespace {

struct Lay {
  size_t total = 0;
  size_t take(size_t b) {
    const size_t o = total;
    total += (b + 255) & ~(size_t)255;
    return o;
  }
};

struct LayerOff {
  size_t Wb, Wt, W, m, v, b, bm, bv, dW, db;  // Wb: BF16 [K][N]; Wt: its N-major copy [N][K]
};

struct SgLayout {
  int L = 0;              // weight layers = depth + 1
  int K0p = 0;            // padded input width
  int Np = 0;             // padded output width (zero weight columns beyond n_out)
  std::vector<int> K, N;  // per layer
  std::vector<std::vector<LayerOff>> lo;  // [member][layer]
  size_t xmean, xstd, ymean, ystd, X0, preds, dA0, dA1, loss, idx;
  size_t dWpart = 0;        // split-K partial products of dW
  size_t dbpart = 0;        // row-block column sums of the bias gradient
  size_t qx, qm, qs;        // one query of sg_predict_or_mc: features, mean, spread
  int msmall = 0;          // rows of the small-batch inference path
  size_t Asm, gvp;         // its activations [2][member][msmall][width] and split partials
  std::vector<size_t> Z, A;  // per hidden layer: pre-activation (FP32) and activation (BF16)
  size_t total = 0;
};

bool sg_valid(const sg_config* c) {
  // a width that is a multiple of 8 keeps every GEMM row 16-byte aligned
  // (the input and output widths are padded internally)
  return c && c->n_in > 0 && c->n_out > 0 && c->width > 0 && c->width % 8 == 0 && c->weight_decay >= 0.0f &&
         c->depth >= 1 && c->depth <= 16 && c->ensemble >= 1 && c->ensemble <= kMaxMembers && c->max_batch >= 1 &&
         c->max_batch <= 65536;
}


// Splits of K (the batch) for dW = X^T dZ [M x N] in 64 x 64 tiles: doubled,
// up to kDwSplitMax, while the workgroups stay within kDwSplitTarget and,
// for a batch K > 0, each split is a whole number of 128-deep slabs; 0 below
// 2 splits.  With K = 0, the most any batch can take (the workspace's
// partials).  Measured on the training step at batch 4096 (1803 -> 1024 x 4
// -> 3600): 1.029 ms without splits, 0.981 with at most 1024 workgroups,
// 0.939 with 2048, 0.910 with 4096, 0.905 with 8192 (twice the partials:
// 118 MB), 0.950 with 8192 and up to 16 splits.
constexpr int kDwSplitTarget = 4096, kDwSplitMax = 8;
// row blocks of the bias gradient's column sums, at most
constexpr int kCsMaxBlocks = 32;
// row slots of the loss kernel's grid (its partial sums: row slots x 1024-column blocks)
constexpr int kLossRows = 256;
int dw_splits(int M, int N, int K) {
  const long tiles = (long)((N + 63) / 64) * ((M + 63) / 64);
  int S = 1;
  while (S < kDwSplitMax && tiles * S * 2 <= kDwSplitTarget && (K == 0 || K % (2 * S * 128) == 0)) S *= 2;
  return S > 1 ? S : 0;
}

SgLayout sg_layout(const sg_config* c) {
  SgLayout s;
  Lay L;
  s.L = c->depth + 1;
  s.K0p = (c->n_in + 31) / 32 * 32;
  s.Np = (c->n_out + 7) / 8 * 8;
  for (int l = 0; l < s.L; ++l) {
    s.K.push_back(l == 0 ? s.K0p : c->width);
    s.N.push_back(l == s.L - 1 ? s.Np : c->width);
  }
  s.lo.resize(c->ensemble);
  for (int e = 0; e < c->ensemble; ++e)
    for (int l = 0; l < s.L; ++l) {
      const size_t n = (size_t)s.K[l] * s.N[l];
      LayerOff o;
      o.Wb = L.take(2 * n);
      o.Wt = L.take(2 * n);
      o.W = L.take(4 * n);
      o.m = L.take(4 * n);
      o.v = L.take(4 * n);
      o.b = L.take(4 * (size_t)s.N[l]);
      o.bm = L.take(4 * (size_t)s.N[l]);
      o.bv = L.take(4 * (size_t)s.N[l]);
      o.dW = L.take(4 * n);
      o.db = L.take(4 * (size_t)s.N[l]);
      s.lo[e].push_back(o);
    }
  const size_t MB = c->max_batch;
  s.xmean = L.take(4 * (size_t)c->n_in);
  s.xstd = L.take(4 * (size_t)c->n_in);
  s.ymean = L.take(4 * (size_t)c->n_out);
  s.ystd = L.take(4 * (size_t)c->n_out);
  s.X0 = L.take(2 * MB * s.K0p);
  for (int l = 0; l < s.L - 1; ++l) {
    s.Z.push_back(L.take(4 * MB * s.N[l]));
    s.A.push_back(L.take(2 * MB * s.N[l]));
  }
  s.preds = L.take(4 * MB * c->n_out * (size_t)c->ensemble);
  const size_t wmax = std::max(c->width, s.Np);
  s.dA0 = L.take(2 * MB * wmax);
  s.dA1 = L.take(2 * MB * wmax);
  s.loss = L.take(4 * (std::min<size_t>(MB, kLossRows) * ((s.Np + 1023) / 1024) + 1));
  size_t part = 0;
  for (int l = 0; l < s.L; ++l)
    part = std::max(part, (size_t)dw_splits(s.K[l], s.N[l], 0) * s.K[l] * s.N[l]);
  if (part > 0) s.dWpart = L.take(4 * part);
  s.dbpart = L.take(4 * (size_t)kCsMaxBlocks * wmax);
  s.msmall = (int)std::min<size_t>(kSmallM, MB);
  s.Asm = L.take(2 * 2 * (size_t)c->ensemble * s.msmall * c->width);
  s.gvp = L.take(4 * (size_t)c->ensemble * kGvMaxSplit * s.msmall * wmax);
  s.qx = L.take(4 * (size_t)c->n_in);
  s.qm = L.take(4 * (size_t)c->n_out);
  s.qs = L.take(4 * (size_t)c->n_out);
  s.idx = 0;
  s.total = L.total;
  return s;
}

unsigned blocks(long n, int t = 256) { return (unsigned)((n + t - 1) / t); }
dim3 loss_grid(int rows, int np) { return dim3((unsigned)((np + 1023) / 1024), (unsigned)std::min(rows, kLossRows)); }

}  // namespace

struct sg_ctx {
  sg_config c;
  SgLayout s;
  char* ws = nullptr;
  hipStream_t st = nullptr;
  std::vector<int> step;  // Adam step per member
  bool bad_gemm = false;  // a GEMM was refused (misaligned operands)
  int dev = 0;            // device current at sg_init
  std::string err;
  template <typename T> T* p(size_t o) { return reinterpret_cast<T*>(ws + o); }
};

namespace {

int sfail(sg_ctx* c, int code, const std::string& m) {
  if (c) c->err = m;
  return code;
}

#define SGCHK(ctx, expr)                                                                                  \
  do {                                                                                                   \
    hipError_t e_ = (expr);                                                                              \
    if (e_ != hipSuccess) return sfail((ctx), MC_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Dynamic LDS beyond the default 64 KB for the direct-to-LDS products of one
// epilogue
template <int EPI>
hipError_t allow_lds() {
  const auto attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e = hipFuncSetAttribute((const void*)k_gemm_lds<EPI, 256, 256, 16>, attr, lds_bytes<256, 256>());
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_gemm_lds<EPI, 128, 128, 8>, attr, lds_bytes<128, 128>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_gemm_lds<EPI, 128, 128, 8, 3>, attr, lds_bytes<128, 128, 3>());
  return e;
}

template <bool TA, bool TB, int EPI>
void gemm(sg_ctx* c, const GemmArgs& g, int splits = 1) {
  // the 16-byte tile loads need leading dimensions that are multiples of 8
  // elements and 16-byte aligned operands (all buffers come from the workspace)
  if ((g.lda & 7) || (g.ldb & 7) || ((uintptr_t)g.A & 15) || ((uintptr_t)g.B & 15)) {
    c->bad_gemm = true;
    return;
  }
  // forward products (both operands K-contiguous, K a multiple of 8):
  // direct-to-LDS slabs in the largest tiles that still give every compute
  // unit work.  The copies reach the compute units at a rate that grows with
  // the wavefronts issuing them, not with the slabs in flight (3 or 4 stages
  // of 128 x 128 tiles ran no faster than 2), so the large tiles take 8 or 16
  // wavefronts.  Measured at batch 4096 (µs per product, 4 wavefronts per
  // tile before): the 1024 -> 3600 output layer 53.3 -> 48.1 in 256 x 256
  // tiles; a hidden layer 21.2 (128 x 64) -> 20.1, the input layer 31.3 ->
  // 30.3 in 128 x 128 tiles, one per compute unit with three stages.  dX
  // (the GELU-derivative epilogue reads the pre-activations) stays in the
  // register-staged 64 x 64 tiles: 43 µs, against 47 in 128 x 64 direct-to-LDS
  // tiles and 43.7 in 128 x 128 tiles of 8 wavefronts.
  if (!TA && TB && EPI != EPI_GELU_GRAD && g.K % 8 == 0) {
    if (lds_tiles(g.M, g.N, 256, 256) >= 224) {
      const int T = lds_tiles(g.M, g.N, 256, 256);
      k_gemm_lds<EPI, 256, 256, 16><<<((T + 7) / 8) * 8, 1024, lds_bytes<256, 256>(), c->st>>>(g);
      return;
    }
    const int T128 = lds_tiles(g.M, g.N, 128, 128);
    if (T128 >= 512) {
      k_gemm_lds<EPI, 128, 128, 8><<<((T128 + 7) / 8) * 8, 512, lds_bytes<128, 128>(), c->st>>>(g);
      return;
    }
    if (T128 >= 256) {
      k_gemm_lds<EPI, 128, 128, 8, 3><<<((T128 + 7) / 8) * 8, 512, lds_bytes<128, 128, 3>(), c->st>>>(g);
      return;
    }
    if (lds_tiles(g.M, g.N, 128, 64) >= 512) {
      const int T = lds_tiles(g.M, g.N, 128, 64);
      k_gemm_lds<EPI, 128, 64, 4><<<((T + 7) / 8) * 8, 256, lds_bytes<128, 64>(), c->st>>>(g);
      return;
    }
  }
  // 128 x 128 tiles unless they would give fewer than two workgroups per
  // compute unit (256 on the MI355X); 64 x 64 tiles then
  const long big = (long)((g.N + 127) / 128) * ((g.M + 127) / 128);
  if (big >= 512 && splits == 1) {
    dim3 grid((g.N + 127) / 128, (g.M + 127) / 128);
    k_gemm<TA, TB, EPI, 64><<<grid, 256, 0, c->st>>>(g);
  } else {
    // split products (the grid's z range) take the 64 x 64 tiles
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, splits);
    k_gemm<TA, TB, EPI, 32><<<grid, 256, 0, c->st>>>(g);
  }
}

// The N-major copy of a layer's BF16 weights, after every change of them.
void enqueue_wt(sg_ctx* c, int e, int l) {
  const SgLayout& s = c->s;
  const LayerOff& o = s.lo[e][l];
  dim3 grid((s.N[l] + 31) / 32, (s.K[l] + 31) / 32);
  k_transpose_bf16<<<grid, dim3(32, 8), 0, c->st>>>(c->p<uint16_t>(o.Wb), s.K[l], s.N[l], c->p<uint16_t>(o.Wt));
}

GemmArgs ga(const bf16* A, long lda, const bf16* B, long ldb, int M, int N, int K) {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.M = M; g.N = N; g.K = K;
  return g;
}

// forward of one member on `batch` rows of raw FP32 inputs; normalised
// predictions to `out` (FP32 [batch][n_out]).  The hidden layers'
// pre-activations are kept (for the GELU derivative) only when a backward
// pass follows; the activations are the same either way.
void enqueue_forward(sg_ctx* c, int e, const float* d_x, int batch, float* out, bool keep_z) {
  const SgLayout& s = c->s;
  k_input<<<dim3(blocks(s.K0p), (batch + kInRows - 1) / kInRows), 256, 0, c->st>>>(
      d_x, batch, c->c.n_in, c->p<float>(s.xmean), c->p<float>(s.xstd), c->p<bf16>(s.X0), s.K0p);
  const bf16* X = c->p<bf16>(s.X0);
  long ldx = s.K0p;
  for (int l = 0; l < s.L; ++l) {
    const LayerOff& o = s.lo[e][l];
    GemmArgs g = ga(X, ldx, c->p<bf16>(o.Wt), s.K[l], batch, s.N[l], s.K[l]);  // weights N-major
    g.bias = c->p<float>(o.b);
    if (l < s.L - 1) {
      g.Cb = c->p<bf16>(s.A[l]); g.ldcb = s.N[l];
      if (keep_z) {
        g.Cf = c->p<float>(s.Z[l]); g.ldcf = s.N[l];
        gemm<false, true, EPI_BIAS_GELU>(c, g);
      } else {
        gemm<false, true, EPI_BIAS_GELU_ONLY>(c, g);
      }
      X = c->p<bf16>(s.A[l]);
      ldx = s.N[l];
    } else {
      g.N = c->c.n_out;  // only the real outputs are written
      g.Cf = out; g.ldcf = c->c.n_out;
      gemm<false, true, EPI_BIAS>(c, g);
    }
  }
}

// Scratch of the small-batch forward: normalised BF16 inputs [batch][K0p],
// two activation buffers [2][member][msmall][width], split partials
// [member][S][batch][N] with S at most max_split, and the members'
// normalised predictions [member][batch][n_out].
struct SmallScratch {
  bf16* X0;
  bf16* Asm;
  float* P;
  float* preds;
  int max_split;
};

// Small-batch forward of every member (batch <= msmall): split-K GEMV per
// layer over all members, then the ordered split sum with the epilogue.
// Normalised predictions to sc.preds [member][batch][n_out].
void enqueue_forward_small(sg_ctx* c, const float* d_x, int batch, const SmallScratch& sc) {
  const SgLayout& s = c->s;
  const int E = c->c.ensemble, width = c->c.width;
  k_input<<<dim3(blocks(s.K0p), (batch + kInRows - 1) / kInRows), 256, 0, c->st>>>(
      d_x, batch, c->c.n_in, c->p<float>(s.xmean), c->p<float>(s.xstd), sc.X0, s.K0p);
  const size_t abuf = (size_t)E * s.msmall * width;  // one activation buffer, all members
  int cur = -1;
  for (int l = 0; l < s.L; ++l) {
    const bool last = l == s.L - 1;
    GemvArgs g;
    std::memset(&g, 0, sizeof(g));
    if (l == 0) {
      g.X = sc.X0; g.ldx = s.K0p; g.xse = 0;
    } else {
      g.X = sc.Asm + (size_t)cur * abuf; g.ldx = width; g.xse = (long)s.msmall * width;
    }
    for (int e = 0; e < E; ++e) g.W[e] = c->p<bf16>(s.lo[e][l].Wb);
    g.ldw = s.N[l];
    g.M = batch; g.N = s.N[l]; g.K = s.K[l];
    const int ncb = (g.N + kGvCols - 1) / kGvCols;
    // about a thousand wavefronts per launch, at least 4 rows per split
    g.S = std::max(1, std::min({sc.max_split, 1024 / (ncb * E), g.K / 4}));
    g.P = sc.P;
    dim3 grid(ncb, g.S, E);
    if (batch <= 1) k_gemv<1><<<grid, 64, 0, c->st>>>(g);
    else if (batch <= 2) k_gemv<2><<<grid, 64, 0, c->st>>>(g);
    else if (batch <= 4) k_gemv<4><<<grid, 64, 0, c->st>>>(g);
    else k_gemv<8><<<grid, 64, 0, c->st>>>(g);
    GemvReduceArgs r;
    std::memset(&r, 0, sizeof(r));
    r.P = g.P; r.S = g.S; r.M = batch; r.N = g.N; r.E = E;
    for (int e = 0; e < E; ++e) r.bias[e] = c->p<float>(s.lo[e][l].b);
    if (last) {
      r.n_valid = c->c.n_out; r.outf = sc.preds; r.ldo = c->c.n_out; r.ofs_e = (long)batch * c->c.n_out;
      k_gemv_reduce<true><<<blocks((long)E * batch * r.n_valid), 256, 0, c->st>>>(r);
    } else {
      const int nxt = cur == 0 ? 1 : 0;
      r.n_valid = g.N; r.outb = sc.Asm + (size_t)nxt * abuf; r.ldo = width;
      r.ofs_e = (long)s.msmall * width;
      k_gemv_reduce<false><<<blocks((long)E * batch * r.n_valid), 256, 0, c->st>>>(r);
      cur = nxt;
    }
  }
}

SmallScratch workspace_scratch(sg_ctx* c) {
  const SgLayout& s = c->s;
  return SmallScratch{c->p<bf16>(s.X0), c->p<bf16>(s.Asm), c->p<float>(s.gvp), c->p<float>(s.preds), kGvMaxSplit};
}

// The allocation-free small-batch predictor's scratch: one array per GPU,
// held until the process ends, shared by every call on that GPU.  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// device that is current (the array's name is a host-side stand-in).
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char sg_static_scratch[kStaticScratchBytes];
std::mutex g_static_mu;
std::map<int, unsigned char*> g_static_ptr;  // device -> address of its sg_static_scratch

// Address of the static scratch on device `dev` (current), looked up once per
// device.
hipError_t static_scratch_of(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_static_mu);
  auto it = g_static_ptr.find(dev);
  if (it != g_static_ptr.end()) { *out = it->second; return hipSuccess; }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(sg_static_scratch));
  if (e != hipSuccess) return e;
  g_static_ptr[dev] = (unsigned char*)ptr;
  *out = (unsigned char*)ptr;
  return hipSuccess;
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

size_t sg_workspace_bytes(const sg_config* c) {
  if (!sg_valid(c)) return 0;
  return sg_layout(c).total;
}

int sg_init(sg_ctx** out, const sg_config* cfg, void* d_ws, size_t bytes, void* stream) {
  if (!out) return MC_E_ARG;
  *out = nullptr;
  if (!sg_valid(cfg)) return MC_E_ARG;
  SgLayout s = sg_layout(cfg);
  if (!d_ws || bytes < s.total || ((uintptr_t)d_ws & 255u)) return MC_E_ARG;
  sg_ctx* c = new sg_ctx();
  c->c = *cfg;
  c->s = s;
  c->ws = (char*)d_ws;
  c->st = (hipStream_t)stream;
  c->step.assign(cfg->ensemble, 0);
  *out = c;
  SGCHK(c, hipGetDevice(&c->dev));
  {
    unsigned char* scr = nullptr;  // the allocation-free predictor's scratch on this device
    SGCHK(c, static_scratch_of(c->dev, &scr));
  }
  // the direct-to-LDS products take up to 128 KB of dynamic LDS per workgroup
  SGCHK(c, allow_lds<EPI_BIAS>());
  SGCHK(c, allow_lds<EPI_BIAS_GELU>());
  SGCHK(c, allow_lds<EPI_BIAS_GELU_ONLY>());
  SGCHK(c, hipMemsetAsync(c->ws, 0, s.total, c->st));
  for (int e = 0; e < cfg->ensemble; ++e)
    for (int l = 0; l < s.L; ++l) {
      const long n = (long)s.K[l] * s.N[l];
      // variance-preserving uniform init on the true fan-in
      const int fan_in = l == 0 ? cfg->n_in : s.K[l];
      const float a = std::sqrt(3.0f / (float)fan_in);
      k_init_weights<<<blocks(n), 256, 0, c->st>>>(c->p<float>(s.lo[e][l].W), c->p<bf16>(s.lo[e][l].Wb), n, a,
                                                   (uint32_t)(cfg->seed & 0xffffffffu), (uint32_t)(cfg->seed >> 32),
                                                   (uint32_t)((5u << 24) | (e << 8) | l));
    }
  // padded input rows of layer 0 carry no weight
  std::vector<float> ones_x(cfg->n_in, 1.0f), ones_y(cfg->n_out, 1.0f);
  SGCHK(c, hipMemcpyAsync(c->ws + s.xstd, ones_x.data(), 4 * ones_x.size(), hipMemcpyHostToDevice, c->st));
  SGCHK(c, hipMemcpyAsync(c->ws + s.ystd, ones_y.data(), 4 * ones_y.size(), hipMemcpyHostToDevice, c->st));
  for (int e = 0; e < cfg->ensemble; ++e) {
    const int L1 = s.L - 1;
    if (s.Np > cfg->n_out) {
      const size_t n = (size_t)s.K[L1] * s.Np;
      std::vector<float> w(n);
      SGCHK(c, hipMemcpyAsync(w.data(), c->ws + s.lo[e][L1].W, 4 * n, hipMemcpyDeviceToHost, c->st));
      SGCHK(c, hipStreamSynchronize(c->st));
      std::vector<uint16_t> wb(n);
      for (size_t i = 0; i < n; ++i) {
        if ((int)(i % s.Np) >= cfg->n_out) w[i] = 0.0f;
        uint32_t u;
        std::memcpy(&u, &w[i], 4);
        wb[i] = (uint16_t)((u + ((u >> 16) & 1u) + 0x7FFFu) >> 16);
      }
      SGCHK(c, hipMemcpyAsync(c->ws + s.lo[e][L1].W, w.data(), 4 * n, hipMemcpyHostToDevice, c->st));
      SGCHK(c, hipMemcpyAsync(c->ws + s.lo[e][L1].Wb, wb.data(), 2 * n, hipMemcpyHostToDevice, c->st));
      SGCHK(c, hipStreamSynchronize(c->st));
    }
    const int pad = s.K0p - cfg->n_in;
    if (pad > 0) {
      std::vector<float> z((size_t)pad * s.N[0], 0.0f);
      std::vector<uint16_t> zb((size_t)pad * s.N[0], 0);
      SGCHK(c, hipMemcpyAsync(c->ws + s.lo[e][0].W + 4 * (size_t)cfg->n_in * s.N[0], z.data(), 4 * z.size(),
                              hipMemcpyHostToDevice, c->st));
      SGCHK(c, hipMemcpyAsync(c->ws + s.lo[e][0].Wb + 2 * (size_t)cfg->n_in * s.N[0], zb.data(), 2 * zb.size(),
                              hipMemcpyHostToDevice, c->st));
    }
  }
  for (int e = 0; e < cfg->ensemble; ++e)
    for (int l = 0; l < s.L; ++l) enqueue_wt(c, e, l);
  SGCHK(c, hipGetLastError());
  SGCHK(c, hipStreamSynchronize(c->st));
  return MC_OK;
}

int sg_destroy(sg_ctx* c) {
  if (!c) return MC_E_ARG;
  (void)hipStreamSynchronize(c->st);
  delete c;
  return MC_OK;
}

const char* sg_last_error(const sg_ctx* c) { return c ? c->err.c_str() : "null context"; }

int sg_layer_dims(const sg_ctx* c, int layer, int* K, int* N) {
  if (!c || layer < 0 || layer >= c->s.L) return MC_E_ARG;
  if (K) *K = c->s.K[layer];
  if (N) *N = layer == c->s.L - 1 ? c->c.n_out : c->s.N[layer];
  return MC_OK;
}

namespace {
// copy a [K][Nint] device matrix to a [K][Next] host matrix (Next <= Nint)
int get_strided(sg_ctx* c, size_t off, int K, int Nint, int Next, float* h) {
  std::vector<float> t((size_t)K * Nint);
  SGCHK(c, hipMemcpyAsync(t.data(), c->ws + off, 4 * t.size(), hipMemcpyDeviceToHost, c->st));
  SGCHK(c, hipStreamSynchronize(c->st));
  for (int k = 0; k < K; ++k) std::memcpy(h + (size_t)k * Next, t.data() + (size_t)k * Nint, 4 * (size_t)Next);
  return MC_OK;
}
}  // namespace

int sg_set_normalization(sg_ctx* c, const float* xm, const float* xs, const float* ym, const float* ys) {
  if (!c || !xm || !xs || !ym || !ys) return MC_E_ARG;
  for (int i = 0; i < c->c.n_in; ++i)
    if (!(xs[i] > 0.0f)) return sfail(c, MC_E_ARG, "input scale must be positive");
  for (int i = 0; i < c->c.n_out; ++i)
    if (!(ys[i] > 0.0f)) return sfail(c, MC_E_ARG, "output scale must be positive");
  const SgLayout& s = c->s;
  SGCHK(c, hipMemcpyAsync(c->ws + s.xmean, xm, 4 * (size_t)c->c.n_in, hipMemcpyHostToDevice, c->st));
  SGCHK(c, hipMemcpyAsync(c->ws + s.xstd, xs, 4 * (size_t)c->c.n_in, hipMemcpyHostToDevice, c->st));
  SGCHK(c, hipMemcpyAsync(c->ws + s.ymean, ym, 4 * (size_t)c->c.n_out, hipMemcpyHostToDevice, c->st));
  SGCHK(c, hipMemcpyAsync(c->ws + s.ystd, ys, 4 * (size_t)c->c.n_out, hipMemcpyHostToDevice, c->st));
  SGCHK(c, hipStreamSynchronize(c->st));
  return MC_OK;
}

int sg_forward(sg_ctx* c, int member, const float* d_x, int batch, float* d_pred) {
  if (!c || member < 0 || member >= c->c.ensemble || !d_x || !d_pred || batch < 1 || batch > c->c.max_batch)
    return sfail(c, MC_E_ARG, "bad argument");
  enqueue_forward(c, member, d_x, batch, d_pred, false);
  SGCHK(c, hipGetLastError());
  if (c->bad_gemm) return sfail(c, MC_E_ARG, "GEMM operands not 16-byte aligned");
  return MC_OK;
}

int sg_backward(sg_ctx* c, int member, const float* d_x, const float* d_y, int batch, float* h_loss) {
  if (!c || member < 0 || member >= c->c.ensemble || !d_x || !d_y || batch < 1 || batch > c->c.max_batch)
    return sfail(c, MC_E_ARG, "bad argument");
  const SgLayout& s = c->s;
  const int n_out = c->c.n_out;
  float* pred = c->p<float>(s.preds) + (size_t)member * c->c.max_batch * n_out;
  enqueue_forward(c, member, d_x, batch, pred, true);
  const long tot = (long)batch * n_out;
  bf16* dcur = c->p<bf16>(s.dA0);
  bf16* dnext = c->p<bf16>(s.dA1);
  k_loss<<<loss_grid(batch, s.Np), 256, 0, c->st>>>(pred, d_y, batch, n_out, s.Np, c->p<float>(s.ymean),
                                                     c->p<float>(s.ystd), dcur, c->p<float>(s.loss));
  for (int l = s.L - 1; l >= 0; --l) {
    const LayerOff& o = s.lo[member][l];
    const bf16* Xin = l == 0 ? c->p<bf16>(s.X0) : c->p<bf16>(s.A[l - 1]);
    const long ldx = l == 0 ? s.K0p : s.N[l - 1];
    // dW = X^T dZ   [K x N]
    GemmArgs gw = ga(Xin, ldx, dcur, s.N[l], s.K[l], s.N[l], batch);
    gw.Cf = c->p<float>(o.dW); gw.ldcf = s.N[l];
    const int S = dw_splits(s.K[l], s.N[l], batch);
    if (S > 1) {
      // S partial products over batch slices into the partials, then their
      // sum in slice order: S times the workgroups of one product over K
      const long n = (long)s.K[l] * s.N[l];
      gw.Cf = c->p<float>(s.dWpart);
      gw.kz = batch / S;
      gw.zs = n;
      gemm<true, false, EPI_STORE>(c, gw, S);
      k_split_sum<<<std::min<long>(blocks(n), 4096), 256, 0, c->st>>>(c->p<float>(s.dWpart), S, n, n,
                                                                      c->p<float>(o.dW));
    } else {
      gemm<true, false, EPI_STORE>(c, gw);
    }
    {
      // bias gradient: row blocks so that about 512 workgroups share the
      // batch (a 1024-wide layer has only 16 column blocks)
      const int nbx = (int)blocks(s.N[l], 64);
      const int R = std::max(1, std::min(kCsMaxBlocks, 512 / nbx));
      const int rp = (batch + R - 1) / R;
      const int Ry = (batch + rp - 1) / rp;
      k_colsum<<<dim3(nbx, Ry), 64 * kCsRows, 0, c->st>>>(dcur, batch, s.N[l], s.N[l], rp, c->p<float>(o.db),
                                                          c->p<float>(s.dbpart));
      if (Ry > 1) k_colsum_reduce<<<blocks(s.N[l], 64), 64, 0, c->st>>>(c->p<float>(s.dbpart), Ry, s.N[l], c->p<float>(o.db));
    }
    if (l > 0) {
      // dZ_{l-1} = (dZ_l W^T) * gelu'(Z_{l-1})
      GemmArgs gx = ga(dcur, s.N[l], c->p<bf16>(o.Wb), s.N[l], batch, s.K[l], s.N[l]);
      gx.Cb = dnext; gx.ldcb = s.K[l];
      gx.Z = c->p<float>(s.Z[l - 1]); gx.ldz = s.N[l - 1];
      gemm<false, true, EPI_GELU_GRAD>(c, gx);
      std::swap(dcur, dnext);
    }
  }
  SGCHK(c, hipGetLastError());
  if (c->bad_gemm) return sfail(c, MC_E_ARG, "GEMM operands not 16-byte aligned");
  if (h_loss) {
    const dim3 lg = loss_grid(batch, s.Np);
    const int nb = (int)(lg.x * lg.y);
    std::vector<float> part(nb);
    SGCHK(c, hipMemcpyAsync(part.data(), c->p<float>(s.loss), 4 * (size_t)nb, hipMemcpyDeviceToHost, c->st));
    SGCHK(c, hipStreamSynchronize(c->st));
    double acc = 0.0;
    for (float v : part) acc += v;
    *h_loss = (float)(acc / (double)tot);
  }
  return MC_OK;
}

int sg_adam(sg_ctx* c, int member, float lr) {
  if (!c || member < 0 || member >= c->c.ensemble || !(lr >= 0.0f)) return sfail(c, MC_E_ARG, "bad argument");
  const SgLayout& s = c->s;
  const int t = ++c->step[member];
  const float b1 = c->c.beta1, b2 = c->c.beta2;
  const float c1 = 1.0f - std::pow(b1, (float)t), c2 = 1.0f - std::pow(b2, (float)t);
  for (int l = 0; l < s.L; ++l) {
    const LayerOff& o = s.lo[member][l];
    // layer 0: only the rows of real inputs train (padding stays zero)
    const long n = (long)(l == 0 ? c->c.n_in : s.K[l]) * s.N[l];
    k_adam<<<blocks((n + 3) / 4), 256, 0, c->st>>>(c->p<float>(o.W), c->p<float>(o.m), c->p<float>(o.v), c->p<float>(o.dW),
                                         c->p<bf16>(o.Wb), n, lr, b1, b2, c->c.eps, c1, c2, c->c.weight_decay);
    k_adam<<<blocks((s.N[l] + 3) / 4), 256, 0, c->st>>>(c->p<float>(o.b), c->p<float>(o.bm), c->p<float>(o.bv),
                                              c->p<float>(o.db), nullptr, s.N[l], lr, b1, b2, c->c.eps, c1, c2, 0.0f);
    enqueue_wt(c, member, l);
  }
  SGCHK(c, hipGetLastError());
  return MC_OK;
}

int sg_train_step(sg_ctx* c, int member, const float* d_x, const float* d_y, int batch, float lr, float* h_loss) {
  int rc = sg_backward(c, member, d_x, d_y, batch, h_loss);
  if (rc != MC_OK) return rc;
  return sg_adam(c, member, lr);
}

int sg_predict(sg_ctx* c, const float* d_x, int batch, float* d_mean, float* d_std) {
  if (!c || !d_x || !d_mean || batch < 1 || batch > c->c.max_batch) return sfail(c, MC_E_ARG, "bad argument");
  const SgLayout& s = c->s;
  const long per = (long)batch * c->c.n_out;
  if (batch <= s.msmall) {
    enqueue_forward_small(c, d_x, batch, workspace_scratch(c));
  } else {
    for (int e = 0; e < c->c.ensemble; ++e)
      enqueue_forward(c, e, d_x, batch, c->p<float>(s.preds) + (size_t)e * per, false);
  }
  k_ensemble<<<blocks(per), 256, 0, c->st>>>(c->p<float>(s.preds), c->c.ensemble, per, c->c.n_out,
                                             c->p<float>(s.ymean), c->p<float>(s.ystd), d_mean, d_std);
  SGCHK(c, hipGetLastError());
  if (c->bad_gemm) return sfail(c, MC_E_ARG, "GEMM operands not 16-byte aligned");
  return MC_OK;
}

int sg_predict_static(sg_ctx* c, const float* d_x, int batch, float* d_mean, float* d_std) {
  if (!c || !d_x || !d_mean || batch < 1 || batch > c->s.msmall) return sfail(c, MC_E_ARG, "bad argument");
  const SgLayout& s = c->s;
  const int E = c->c.ensemble;
  unsigned char* base = nullptr;
  SGCHK(c, static_scratch_of(c->dev, &base));
  const size_t b_x0 = up256(2 * (size_t)batch * s.K0p);
  const size_t b_asm = up256(2 * 2 * (size_t)E * s.msmall * c->c.width);
  const size_t b_pred = up256(4 * (size_t)E * batch * c->c.n_out);
  const size_t nmax = (size_t)std::max(c->c.width, s.Np);
  const size_t per_split = 4 * (size_t)E * batch * nmax;  // partials of one K split, widest layer
  const size_t fixed = b_x0 + b_asm + b_pred;
  if (fixed + per_split > kStaticScratchBytes)
    return sfail(c, MC_E_ARG, "the network's small-batch scratch exceeds the static 8 MiB");
  SmallScratch sc;
  sc.X0 = (bf16*)base;
  sc.Asm = (bf16*)(base + b_x0);
  sc.preds = (float*)(base + b_x0 + b_asm);
  sc.P = (float*)(base + fixed);
  sc.max_split = (int)std::min<size_t>(kGvMaxSplit, (kStaticScratchBytes - fixed) / per_split);
  enqueue_forward_small(c, d_x, batch, sc);
  const long per = (long)batch * c->c.n_out;
  k_ensemble<<<blocks(per), 256, 0, c->st>>>(sc.preds, E, per, c->c.n_out, c->p<float>(s.ymean),
                                             c->p<float>(s.ystd), d_mean, d_std);
  SGCHK(c, hipGetLastError());
  return MC_OK;
}

int sg_predict_or_mc(sg_ctx* c, mc_ctx* mc, int instance, const sg_query* q, double* h_maps, float* h_pred_err,
                     int* used_mc) {
  if (!c || !q || !q->h_x || !h_maps || !(q->calib >= 0.0f)) return sfail(c, MC_E_ARG, "bad argument");
  const int n_in = c->c.n_in, n_out = c->c.n_out;
  if (n_out < 4 || (n_out - 2) % 2)
    return sfail(c, MC_E_ARG, "outputs are not [shape, shape, log-norm, log-norm] of two maps");
  const int nc = (n_out - 2) / 2;
  const SgLayout& s = c->s;
  SGCHK(c, hipMemcpyAsync(c->ws + s.qx, q->h_x, 4 * (size_t)n_in, hipMemcpyHostToDevice, c->st));
  int rc = sg_predict(c, c->p<float>(s.qx), 1, c->p<float>(s.qm), c->p<float>(s.qs));
  if (rc != MC_OK) return rc;
  std::vector<float> m(n_out), sd(n_out);
  SGCHK(c, hipMemcpyAsync(m.data(), c->ws + s.qm, 4 * (size_t)n_out, hipMemcpyDeviceToHost, c->st));
  SGCHK(c, hipMemcpyAsync(sd.data(), c->ws + s.qs, 4 * (size_t)n_out, hipMemcpyDeviceToHost, c->st));
  SGCHK(c, hipStreamSynchronize(c->st));
  // decoded maps and the spread of each: shape spread over shape norm, in
  // quadrature with the log-norm spread; the larger map's
  double spread = 0.0;
  for (int k = 0; k < 2; ++k) {
    double nm = 0.0, ns = 0.0;
    for (int i = 0; i < nc; ++i) {
      nm += (double)m[k * nc + i] * m[k * nc + i];
      ns += (double)sd[k * nc + i] * sd[k * nc + i];
    }
    spread = std::max(spread, std::hypot(std::sqrt(ns) / std::max(std::sqrt(nm), 1e-300), (double)sd[2 * nc + k]));
    const double scale = std::exp((double)m[2 * nc + k]);
    for (int i = 0; i < nc; ++i) h_maps[k * nc + i] = (double)m[k * nc + i] * scale;
  }
  const double perr = (double)q->calib * spread;
  bool inside = true;
  if (q->h_box_lo && q->h_box_hi)
    for (int j = 0; j < n_in; ++j) {
      const double lo = q->h_box_lo[j], hi = q->h_box_hi[j], pad = 1e-6 * std::max(1.0, std::fabs(hi - lo));
      if (!(q->h_x[j] >= lo - pad && q->h_x[j] <= hi + pad)) inside = false;
    }
  const bool fall = !(perr <= (double)q->tol) || !inside;  // a NaN error falls back too
  if (h_pred_err) *h_pred_err = (float)perr;
  if (used_mc) *used_mc = fall ? 1 : 0;
  if (!fall) return MC_OK;
  if (!mc) return sfail(c, MC_E_ARG, "the Monte Carlo is needed: no context given");
  // the instance must be set up for the queried point: same grid, voltages,
  // doping and lattice temperature (features are FP32: relative 1e-5)
  mc_config mcfg;
  int mnc = 0;
  if (mc_get_config(mc, instance, &mcfg) != MC_OK || mc_get_ncell(mc, &mnc) != MC_OK)
    return sfail(c, MC_E_ARG, "bad Monte Carlo instance");
  if (mnc != nc) return sfail(c, MC_E_ARG, "the Monte Carlo context's grid differs from the surrogate's maps");
  if (n_in != 3 + nc) return sfail(c, MC_E_ARG, "features are not (Vgs, Vds, log10 doping, T per subcell)");
  std::vector<double> T(nc);
  if (mc_get_lattice_temperature(mc, instance, T.data()) != MC_OK) return sfail(c, MC_E_ARG, "bad Monte Carlo instance");
  auto near = [](double a, double b) { return std::fabs(a - b) <= 1e-5 * std::max(1.0, std::fabs(b)); };
  bool same = near(mcfg.Vgs, q->h_x[0]) && near(mcfg.Vds, q->h_x[1]) && near(std::log10(mcfg.N_D_m3 * 1e-6), q->h_x[2]);
  for (int i = 0; i < nc && same; ++i) same = near(T[i], q->h_x[3 + i]);
  if (!same) return sfail(c, MC_E_ARG, "the Monte Carlo instance is set up for another bias point or temperature map");
  if (q->warm_substeps < 0 || q->window_substeps < 1) return sfail(c, MC_E_ARG, "bad Monte Carlo window");
  if ((rc = mc_step(mc, q->warm_substeps)) != MC_OK) return rc;
  mc_tally_out t;
  if ((rc = mc_tally(mc, instance, &t, 1)) != MC_OK) return rc;
  if ((rc = mc_step(mc, q->window_substeps)) != MC_OK) return rc;
  if ((rc = mc_maps(mc, instance, nullptr, nullptr, h_maps, h_maps + nc, nullptr)) != MC_OK) return rc;
  // a sticky device error raised during the window (the maps are filled)
  return mc_tally(mc, instance, &t, 0);
}

int sg_get_params(sg_ctx* c, int member, int layer, float* h_W, float* h_b) {
  if (!c || member < 0 || member >= c->c.ensemble || layer < 0 || layer >= c->s.L) return MC_E_ARG;
  const LayerOff& o = c->s.lo[member][layer];
  int N = 0;
  sg_layer_dims(c, layer, nullptr, &N);
  if (h_W) {
    const int rc = get_strided(c, o.W, c->s.K[layer], c->s.N[layer], N, h_W);
    if (rc != MC_OK) return rc;
  }
  if (h_b) SGCHK(c, hipMemcpyAsync(h_b, c->ws + o.b, 4 * (size_t)N, hipMemcpyDeviceToHost, c->st));
  SGCHK(c, hipStreamSynchronize(c->st));
  return MC_OK;
}

int sg_set_params(sg_ctx* c, int member, int layer, const float* h_W, const float* h_b) {
  if (!c || member < 0 || member >= c->c.ensemble || layer < 0 || layer >= c->s.L || !h_W || !h_b) return MC_E_ARG;
  const LayerOff& o = c->s.lo[member][layer];
  int N = 0;
  sg_layer_dims(c, layer, nullptr, &N);
  const int Ni = c->s.N[layer];
  const size_t n = (size_t)c->s.K[layer] * Ni;
  std::vector<float> w(n, 0.0f);
  for (int k = 0; k < c->s.K[layer]; ++k) std::memcpy(w.data() + (size_t)k * Ni, h_W + (size_t)k * N, 4 * (size_t)N);
  if (layer == 0)
    for (size_t i = (size_t)c->c.n_in * c->s.N[0]; i < n; ++i) w[i] = 0.0f;
  std::vector<float> bb(Ni, 0.0f);
  std::memcpy(bb.data(), h_b, 4 * (size_t)N);
  std::vector<uint16_t> wb(n);
  for (size_t i = 0; i < n; ++i) {
    // round to nearest even BF16
    uint32_t u;
    std::memcpy(&u, &w[i], 4);
    const uint32_t r = ((u >> 16) & 1u) + 0x7FFFu;
    wb[i] = (uint16_t)((u + r) >> 16);
  }
  SGCHK(c, hipMemcpyAsync(c->ws + o.W, w.data(), 4 * n, hipMemcpyHostToDevice, c->st));
  SGCHK(c, hipMemcpyAsync(c->ws + o.Wb, wb.data(), 2 * n, hipMemcpyHostToDevice, c->st));
  SGCHK(c, hipMemcpyAsync(c->ws + o.b, bb.data(), 4 * (size_t)Ni, hipMemcpyHostToDevice, c->st));
  enqueue_wt(c, member, layer);
  SGCHK(c, hipGetLastError());
  SGCHK(c, hipStreamSynchronize(c->st));
  return MC_OK;
}

int sg_get_grads(sg_ctx* c, int member, int layer, float* h_dW, float* h_db) {
  if (!c || member < 0 || member >= c->c.ensemble || layer < 0 || layer >= c->s.L) return MC_E_ARG;
  const LayerOff& o = c->s.lo[member][layer];
  int N = 0;
  sg_layer_dims(c, layer, nullptr, &N);
  if (h_dW) {
    const int rc = get_strided(c, o.dW, c->s.K[layer], c->s.N[layer], N, h_dW);
    if (rc != MC_OK) return rc;
  }
  if (h_db) SGCHK(c, hipMemcpyAsync(h_db, c->ws + o.db, 4 * (size_t)N, hipMemcpyDeviceToHost, c->st));
  SGCHK(c, hipStreamSynchronize(c->st));
  return MC_OK;
}

}  // extern "C"
