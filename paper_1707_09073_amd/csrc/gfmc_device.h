// gfmc_device.h -- device-side physics of the gfx950 electron Monte Carlo:
// counter-based Philox4x32-10, Kane dispersion, the nonparabolic scattering
// rates used to build the tables, and the per-particle free flight and
// scattering.  Method: Hao et al., arXiv:1707.09073, electron MC paragraph and
// Table I (three valleys, Kane model, the four mechanisms, subcell counting).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace gfmc {

// CODATA 2018, SI
constexpr double kQ = 1.602176634e-19;
constexpr double kHbar = 1.054571817e-34;
constexpr double kMe = 9.1093837015e-31;
constexpr double kKb = 1.380649e-23;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;

constexpr int kNV = 3;      // valleys Gamma1, U, Gamma3
constexpr int kNM = 10;     // mechanisms: ac, ii, pop_ab, pop_em, (iv_ab, iv_em) x 3 final valleys
constexpr int kTRow = 12;   // table row: 10 shapes, 4k^2, pad
constexpr int kFRow = 8;    // cell factors: T, N_I/b2, N_lo, N_lo+1, N_iv, N_iv+1, b2, pad
constexpr uint32_t kAlive = 4u;
constexpr int kMaxEvents = 1 << 15;  // events per flight interval before the guard trips

// meta word: id << 3 | alive << 2 | valley
__device__ __forceinline__ int meta_valley(uint32_t m) { int v = (int)(m & 3u); return v > 2 ? 2 : v; }
__device__ __forceinline__ uint32_t meta_id(uint32_t m) { return m >> 3; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).  Counter (c0..c3), key (k0, k1).
// ---------------------------------------------------------------------------
// The key (k0, k1) must be the same in every lane of the wavefront (every
// caller passes the instance seed).  The key schedule then stays in scalar
// registers and is recomputed with scalar adds at each call: the empty asm
// below keeps the compiler from hoisting the 20 round keys out of the
// callers' loops, which overflowed the scalar registers and spilled them.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1) {
  asm volatile("" : "+s"(k0), "+s"(k1));
  // one 32x32 -> 64-bit product per multiplier (v_mad_u64_u32 gives both halves)
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    // three-input XOR in one v_bitop3_b32 (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96),
                   n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// ---------------------------------------------------------------------------
// Arithmetic of the two precisions.  FP64 uses the correctly rounded library
// functions; FP32 uses the hardware transcendental unit (v_log/v_exp/v_sqrt/
// v_rcp/v_sin/v_cos; the trig units take revolutions).
// ---------------------------------------------------------------------------
template <typename T> struct Ar;
template <> struct Ar<double> {
  __device__ static double u01(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }
  __device__ static double ln(double x) { return log(x); }
  __device__ static double sq(double x) { return sqrt(x); }
  __device__ static double dv(double a, double b) { return a / b; }
  __device__ static void cs2pi(double u, double& c, double& s) {
    const double ph = 2.0 * kPi * u;
    c = cos(ph);
    s = sin(ph);
  }
  __device__ static double pw(double b, double e) { return pow(b, e); }
  __device__ static double em1(double x) { return expm1(x); }
  __device__ static double l1p(double x) { return log1p(x); }
  __device__ static double fl(double x) { return floor(x); }
  // position -> cell coordinate: a correctly rounded division in FP64
  __device__ static double cs(double x, double d, double) { return x / d; }
  // x clamped to [0, hi] (a NaN to 0)
  __device__ static double clamp0(double x, double hi) { return fmin(fmax(x, 0.0), hi); }
};
template <> struct Ar<float> {
  // 23 random bits so that (w + 1/2) 2^-23 is exact and lies in (0, 1)
  __device__ static float u01(uint32_t w) { return ((float)(w >> 9) + 0.5f) * (1.0f / 8388608.0f); }
  __device__ static float ln(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945f; }
  __device__ static float sq(float x) { return __builtin_amdgcn_sqrtf(x); }
  __device__ static float dv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
  __device__ static void cs2pi(float u, float& c, float& s) {
    c = __builtin_amdgcn_cosf(u);
    s = __builtin_amdgcn_sinf(u);
  }
  __device__ static float pw(float b, float e) { return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(b)); }
  // exp(x) - 1: a short series where exp(x) - 1 would cancel
  __device__ static float em1(float x) {
    const float s = x * (1.0f + 0.5f * x * (1.0f + x * (1.0f / 3.0f)));
    const float e = __builtin_amdgcn_exp2f(x * 1.44269504088896f) - 1.0f;
    return fabsf(x) < 1e-2f ? s : e;
  }
  // log(1 + x) for x >= 0 (the argument here is 2 xi >> 0)
  __device__ static float l1p(float x) { return __builtin_amdgcn_logf(1.0f + x) * 0.693147180559945f; }
  __device__ static float fl(float x) { return floorf(x); }
  __device__ static float cs(float x, float, float inv_d) { return x * inv_d; }
  // x clamped to [0, hi] in one v_med3_f32 (a NaN comes out as 0, 0 or hi:
  // in range either way)
  __device__ static float clamp0(float x, float hi) { return __builtin_amdgcn_fmed3f(x, 0.0f, hi); }
};

// Row loads of 16-byte vectors (rows are 16-byte aligned).
template <typename T, int N>
__device__ __forceinline__ void load_row(const T* p, T* out);
template <int N>
__device__ __forceinline__ void load_row(const float* p, float* out) {
#pragma unroll
  for (int i = 0; i < N / 4; ++i) {
    const float4 v = reinterpret_cast<const float4*>(p)[i];
    out[4 * i] = v.x; out[4 * i + 1] = v.y; out[4 * i + 2] = v.z; out[4 * i + 3] = v.w;
  }
}
template <int N>
__device__ __forceinline__ void load_row(const double* p, double* out) {
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const double2 v = reinterpret_cast<const double2*>(p)[i];
    out[2 * i] = v.x; out[2 * i + 1] = v.y;
  }
}

// Material constants in MC units, one precision.
template <typename T>
struct Mat {
  T m[3], alpha[3], Ec[3];
  T hw_lo, hw_iv;
  T ck;   // hbar^2 / (2 m0), eV nm^2
  T cv;   // hbar / m0, nm^2 / fs
  T cf;   // e / hbar, 1/(nm fs) per V/nm
};

// Geometry of the subcell grid (device mode).
template <typename T>
struct Geo {
  int nx, ny, nz, ncell;
  T L[3], d[3], inv_d[3];
};

// Per-valley constant for a lane's runtime valley index.  Written as bit
// masks so that it compiles to v_cndmask: an array of the kernel arguments
// indexed at run time is a memory load, and a ternary chain on the valley
// becomes divergent branches.
template <typename T>
__device__ __forceinline__ T pick3(const T (&a)[3], int v) {
  typedef typename std::conditional<sizeof(T) == 8, unsigned long long, unsigned int>::type U;
  const U x0 = __builtin_bit_cast(U, a[0]), x1 = __builtin_bit_cast(U, a[1]);
  U r = __builtin_bit_cast(U, a[2]);
  const U m0 = (U)0 - (U)(v == 0), m1 = (U)0 - (U)(v == 1);
  r = (x1 & m1) | (r & ~m1);
  r = (x0 & m0) | (r & ~m0);
  return __builtin_bit_cast(T, r);
}

// Kane: E from gamma = E (1 + a E), positive root, finite at a = 0.
template <typename T>
__device__ __forceinline__ T kane_E(T gam, T a) {
  return Ar<T>::dv((T)2 * gam, (T)1 + Ar<T>::sq((T)1 + (T)4 * a * gam));
}

// Sums of products written as explicit fused multiply-adds.  Left to the
// compiler, which product of such a sum it fuses can differ between two
// kernels that inline the same code, and with it the last bit; the kernels
// of the particle step must agree bit for bit.
template <typename T>
__device__ __forceinline__ T ksq(T kx, T ky, T kz) { return fma(kx, kx, fma(ky, ky, kz * kz)); }
template <typename T>
__device__ __forceinline__ T dot3(T a0, T b0, T a1, T b1, T a2, T b2) { return fma(a0, b0, fma(a1, b1, a2 * b2)); }

template <typename T>
__device__ __forceinline__ T energy(const Mat<T>& M, int v, T kx, T ky, T kz) {
  const T k2 = ksq(kx, ky, kz);
  return kane_E(Ar<T>::dv(M.ck * k2, pick3(M.m, v)), pick3(M.alpha, v));
}

// group-velocity factor: v = s k with s = hbar / (m (1 + 2 a E)), nm/fs per 1/nm
template <typename T>
__device__ __forceinline__ T vel_factor(const Mat<T>& M, int v, T E) {
  return Ar<T>::dv(M.cv, pick3(M.m, v) * ((T)1 + (T)2 * pick3(M.alpha, v) * E));
}

template <typename T>
__device__ __forceinline__ int cell_of(const Geo<T>& G, T x, T y, T z) {
  // clamp in floating point first so that non-finite input still lands in
  // range; a coordinate clamped to [0, n - 1] truncates to its floor
  const T fx = Ar<T>::clamp0(Ar<T>::cs(x, G.d[0], G.inv_d[0]), (T)(G.nx - 1));
  const T fy = Ar<T>::clamp0(Ar<T>::cs(y, G.d[1], G.inv_d[1]), (T)(G.ny - 1));
  const T fz = Ar<T>::clamp0(Ar<T>::cs(z, G.d[2], G.inv_d[2]), (T)(G.nz - 1));
  return ((int)fx * G.ny + (int)fy) * G.nz + (int)fz;
}

// ---------------------------------------------------------------------------
// Rate formulas (SI), FP64, used to fill the tables on the device.
// Standard nonparabolic forms for the four mechanisms of the paper.
// ---------------------------------------------------------------------------
struct RateMat {
  double m[3], alpha[3], Ec[3];
  int Z[3];
  double eps_s, eps_inf, rho, D_ac, D_iv, hw_lo, hw_iv, u_ac;
};

__device__ inline double dos_si(const RateMat& R, int v, double E) {
  if (E <= 0.0) return 0.0;
  const double m = R.m[v] * kMe;
  const double gam = E * (1.0 + R.alpha[v] * E) * kQ;
  return pow(2.0 * m, 1.5) * sqrt(gam) * (1.0 + 2.0 * R.alpha[v] * E) / (4.0 * kPi * kPi * kHbar * kHbar * kHbar);
}

// Froehlich polar-optical scattering with the Kane overlap (Fawcett,
// Boardman & Swain closed form), occupation factor excluded.
__device__ inline double pop_shape(const RateMat& R, int v, double E, double Ep) {
  if (E <= 0.0 || Ep <= 0.0) return 0.0;
  const double a = R.alpha[v];
  const double g = E * (1.0 + a * E), gp = Ep * (1.0 + a * Ep);
  const double sg = sqrt(g), sgp = sqrt(gp);
  const double p = (1.0 + a * E) * (1.0 + a * Ep);
  double A = 2.0 * p + a * (g + gp);
  A *= A;
  const double B = -2.0 * a * sg * sgp * (4.0 * p + a * (g + gp));
  const double C = 4.0 * p * (1.0 + 2.0 * a * E) * (1.0 + 2.0 * a * Ep);
  const double F0 = (A * log(fabs((sg + sgp) / (sg - sgp))) + B) / C;
  const double w0 = R.hw_lo * kQ / kHbar;
  const double pref = kQ * kQ * w0 * sqrt(R.m[v] * kMe) / (4.0 * sqrt(2.0) * kPi * kEps0 * kHbar) *
                      (1.0 / R.eps_inf - 1.0 / R.eps_s);
  return pref * (1.0 + 2.0 * a * Ep) / sqrt(g * kQ) * F0;
}

__device__ inline double iv_shape(const RateMat& R, int v, int j, double Ep) {
  if (Ep <= 0.0) return 0.0;
  const int Zp = (j == v) ? R.Z[v] - 1 : R.Z[j];
  if (Zp <= 0) return 0.0;
  const double D = R.D_iv * kQ;
  const double w = R.hw_iv * kQ / kHbar;
  return kPi * D * D * (double)Zp / (R.rho * w) * dos_si(R, j, Ep);
}

// ---------------------------------------------------------------------------
// Tabulated total and cumulative selection in a cell.  Same code serves the
// bound Gamma_v and the selection, so the bound holds in the kernel's own
// arithmetic.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T tab_term(const T* S, const T* f, int m) {
  switch (m) {
    case 0: return f[0] * S[0];
    case 1: return Ar<T>::dv(S[1] * f[1], f[6] + S[10]);
    case 2: return f[2] * S[2];
    case 3: return f[3] * S[3];
    default: return (((m - 4) & 1) ? f[5] : f[4]) * S[m];
  }
}

template <typename T>
__device__ __forceinline__ T tab_total(const T* S, const T* f) {
  T cum = (T)0;
#pragma unroll
  for (int m = 0; m < kNM; ++m) cum += tab_term<T>(S, f, m);
  return cum;
}

// Duff et al. (JCGT 2017) orthonormal basis around the unit vector n.
template <typename T>
__device__ __forceinline__ void onb(T nx, T ny, T nz, T e1[3], T e2[3]) {
  const T s = copysign((T)1, nz);
  const T a = Ar<T>::dv((T)-1, s + nz);
  const T b = nx * ny * a;
  e1[0] = (T)1 + s * nx * nx * a; e1[1] = s * b; e1[2] = -s * nx;
  e2[0] = b; e2[1] = s + ny * ny * a; e2[2] = -ny;
}

}  // namespace gfmc
