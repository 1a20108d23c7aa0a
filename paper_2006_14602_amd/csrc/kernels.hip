// HIP kernels (gfx950) of the DD-PMA hot path.
//
// One pseudo-time step of every (sub)domain is:
//   transmission      artificial-boundary nodes <- owner's time-n value (Sec. 3 eq.
//                     transmission_condition3)
//   stencil           F = log(|Omega_c| rho(xi + grad_h phi) det(I + D^2_h phi) / theta),
//                     centred differences (Sec. 3 eqs. pmae1d/pmae2d), mirror ghosts for the
//                     Neumann condition (Sec. 2 eq. nbd), F = 0 on artificial nodes
//   mode products     type-I DCT along each axis as dense matrix products on the matrix cores;
//                     the last forward product divides by 1 + gamma sum_k mu_k, the last inverse
//                     product adds dt * delta to phi on live nodes and the FP64 residual
//                     partial sums (Sec. 2 eq. dd_stop_criterion)
// plus, once per solve, the glue of the subdomain meshes and the FP64 Jacobian checks.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "pma_device.h"

namespace pma {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));

// Global-memory view of a pointer taken from a descriptor.  Accesses through a plain pointer
// loaded from memory compile to flat instructions, which also count as LDS operations: every
// wait for an LDS read would then drain the loads in flight as well.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ inline const gmem<T>* gp(const void* p) { return (const gmem<T>*)p; }
template <typename T>
__device__ inline gmem<T>* gpw(void* p) { return (gmem<T>*)p; }

// Raw buffer view of one array of `bytes` bytes (a 128-bit resource in scalar registers).  A load or
// store through it adds a wave-uniform byte offset (scalar register) to a per-lane one (vector
// register) in the memory unit, so forming the address costs no vector instruction, where a global
// access adds a 64-bit base to every lane's offset.  Callers keep every offset inside the array;
// the size in the resource is the array's, not a bound they rely on.
struct BufView {
  __amdgpu_buffer_rsrc_t r;
};
__device__ inline BufView buf_view(const void* p, unsigned bytes) {
  // word 3 of an untyped gfx9 buffer resource with stride 0: 32-bit data, offsets in bytes
  return {__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000)};
}
template <typename T>
__device__ inline T buf_ld(const BufView& b, unsigned voff, unsigned soff);
template <>
__device__ inline float buf_ld<float>(const BufView& b, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, (int)voff, (int)soff, 0));
}
template <>
__device__ inline double buf_ld<double>(const BufView& b, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)voff, (int)soff, 0));
}
__device__ inline void buf_st(const BufView& b, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), b.r, (int)voff, (int)soff, 0);
}
__device__ inline void buf_st(const BufView& b, unsigned voff, unsigned soff, double v) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), b.r, (int)voff, (int)soff, 0);
}

// The right-hand side F is evaluated by several kernels (the stencil alone, fused with the first
// product, inside the persistent step) whose results agree to the bit.  In the code that computes
// it, a multiply and an add are fused only where one expression holds both (explicit fma or
// contract(on)), never across statements, where the choice would depend on each kernel's code
// around them.
#pragma clang fp contract(on)

// ------------------------------------------------------------------------------------------
// monitor: rho(x) as 1 + its excess, each excess evaluated without cancellation
// ------------------------------------------------------------------------------------------

// sin(2 pi x): the FP32 form uses the hardware sine, whose argument is in revolutions
__device__ inline float sin2pi(float x) { return __builtin_amdgcn_sinf(x); }
__device__ inline double sin2pi(double x) { return sinpi(2.0 * x); }

// the monitor parameters of an instance in the working precision
__device__ inline const MonP<float>& mon_of(const InstDev& I, float) { return I.monf; }
__device__ inline const MonP<double>& mon_of(const InstDev& I, double) { return I.mond; }

// e^x as expk(x * kLog2e): FP32 takes the hardware 2^x with the factor log2(e) folded into the
// monitor constants; FP64 calls exp.  frcp: hardware reciprocal (FP32), division (FP64).
template <typename T> struct ExpK;
template <> struct ExpK<float> {
  static constexpr float kLog2e = 1.44269504088896341f;
  static __device__ inline float ex(float x) { return __builtin_amdgcn_exp2f(x); }
};
template <> struct ExpK<double> {
  static constexpr double kLog2e = 1.0;
  static __device__ inline double ex(double x) { return exp(x); }
};
__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// FP64 reciprocal: the hardware estimate refined by two Newton steps (each doubles the correct
// bits), within an ulp or so instead of the correctly rounded division's dozen instructions
__device__ inline double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// Natural log in FP64 for the right-hand side, from the classical reduction and series:
// y = m 2^k with m in [sqrt(1/2), sqrt(2)), log m = 2 atanh(s) with s = (m - 1) / (m + 1),
// |s| <= 0.1716, summed as 2 s (1 + z/3 + z^2/5 + .. + z^11/23), z = s^2 (truncation below
// 1e-19), then k ln 2 added in two parts (ln 2 split so that k ln2_hi is exact).  The rounding of
// these steps keeps the result within a few ulp of the correctly rounded log (an absolute error
// near 1e-16 in F, far inside the FP64 parity tolerance), in about 60 vector instructions where
// libm's double-double evaluation takes about 100.  Non-positive y gives -inf (0) or NaN, as log
// does.
__device__ inline double log_pos(double y) {
  int k;
  double m = frexp(y, &k);
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    k -= 1;
  }
  const double s = (m - 1.0) * frcp(m + 1.0);
  const double z = s * s;
  double p = 1.0 / 23;
  p = fma(p, z, 1.0 / 21);
  p = fma(p, z, 1.0 / 19);
  p = fma(p, z, 1.0 / 17);
  p = fma(p, z, 1.0 / 15);
  p = fma(p, z, 1.0 / 13);
  p = fma(p, z, 1.0 / 11);
  p = fma(p, z, 1.0 / 9);
  p = fma(p, z, 1.0 / 7);
  p = fma(p, z, 1.0 / 5);
  p = fma(p, z, 1.0 / 3);
  const double ts = 2.0 * s;
  const double lm = fma(ts * z, p, ts);
  const double dk = (double)k;
  const double r = fma(dk, 6.93147180369123816490e-01, fma(dk, 1.90821492927058770002e-10, lm));
  return y > 0.0 ? r : (y == 0.0 ? -__builtin_inf() : __builtin_nan(""));
}

// 4 a e / (1 + e)^2 = a sech^2(z) for e = e^{-2|z|} (no overflow for large |z|)
template <typename T>
__device__ inline T sech2_of(T a4, T e) {
  const T q = T(1) + e;
  return a4 * e * frcp(q * q);
}
// 1 + a sech^2(z), the 1 added in the same fused multiply-add
template <typename T>
__device__ inline T one_plus_sech2(T a4, T e) {
  const T q = T(1) + e;
  return a4 * e * frcp(q * q) + T(1);
}

// F = log(vol / theta) + log(rho (1 + e)), the second term as one log of the product (FP64:
// log_pos; FP32: the hardware log2); the product stays far from the denormal range while the
// mesh is untangled, and its rounding (one unit in the last place of a number near 1) is an
// absolute error of the same size in F
__device__ inline double rhs_of(double lvt, double rho, double e) { return lvt + log_pos(rho * (1.0 + e)); }
__device__ inline float rhs_of(float lvt, float rho, float e) {
  return __builtin_amdgcn_logf(rho * (1.f + e)) * 0.693147180559945309f + lvt;
}

__device__ inline bool is_artificial(int art, int k, int i, int n) {
  return (i == 0 && ((art >> (2 * k)) & 1)) || (i == n - 1 && ((art >> (2 * k + 1)) & 1));
}

template <typename T>
__device__ inline bool finite_(T x) { return isfinite(x); }

// ------------------------------------------------------------------------------------------
// K1/K2: stencil + monitor + log (the right-hand side F), Neumann ghosts by mirroring.
// ------------------------------------------------------------------------------------------

// mirror an index across a face (Neumann ghost), then keep it inside the array (rows beyond the
// array's end only feed outputs that are not stored)
__device__ inline int mirror_clamp(int i, int n) {
  if (i < 0) i = -i;
  if (i > n - 1) i = 2 * (n - 1) - i;
  return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

// Tile handled by this workgroup.  Workgroups are dispatched round-robin over the eight XCDs
// (workgroup b runs on XCD b % 8), each XCD with its own L2.  The tiles are handed out so that
// XCD x takes one contiguous run of the launch table: the tiles of one subdomain, which share
// halo rows and DCT matrices, then meet in the same L2.  A bijection of [0, gridDim.x).
__device__ inline int xcd_tile() {
  const int b = blockIdx.x, n = gridDim.x;
  const int q = n >> 3, r = n & 7, x = b & 7, j = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + j;
}

// mirror index for the Neumann ghost of phi: -1 -> 1, n -> n - 2
__device__ inline int mlo(int i) { return i > 0 ? i - 1 : 1; }
__device__ inline int mhi(int i, int n) { return i < n - 1 ? i + 1 : n - 2; }

// Monitor parameters of one kind, held in registers for a whole block so that evaluating rho at
// a node reads no memory, with the constants of the exponentials pre-scaled (nk = -2 k log2 e for
// the sech^2 kinds).  rho<DIM>(x) is 1 plus an excess evaluated without cancellation, the 1 added
// in the excess's last fused multiply-add.
template <typename T, int MK> struct MonReg;

template <typename T> struct MonReg<T, MON_CONST> {
  T rh;
  __device__ explicit MonReg(const MonP<T>& m) : rh(m.amp) {}
  template <int DIM> __device__ T rho(T, T, T) const { return rh; }
};

template <typename T> struct MonReg<T, MON_RADIAL> {
  T a4, nk, c0, c1, c2, r02;
  __device__ explicit MonReg(const MonP<T>& m)
      : a4(T(4) * m.amp), nk(T(-2) * m.k * ExpK<T>::kLog2e), c0(m.c[0]), c1(m.c[1]), c2(m.c[2]), r02(m.r02) {}
  template <int DIM> __device__ T rho(T x0, T x1, T x2) const {
    const T d0 = x0 - c0, d1 = x1 - c1;
    T r2 = d0 * d0 + d1 * d1;
    if (DIM == 3) r2 += (x2 - c2) * (x2 - c2);
    return one_plus_sech2(a4, ExpK<T>::ex(nk * fabs(r2 - r02)));
  }
};

template <typename T> struct MonReg<T, MON_SINE> {
  T a4, nk, c1, r0;
  __device__ explicit MonReg(const MonP<T>& m)
      : a4(T(4) * m.amp), nk(T(-2) * m.k * ExpK<T>::kLog2e), c1(m.c[1]), r0(m.r0) {}
  template <int DIM> __device__ T rho(T x0, T x1, T) const {
    return one_plus_sech2(a4, ExpK<T>::ex(nk * fabs(x1 - c1 - r0 * sin2pi(x0))));
  }
};

template <typename T> struct MonReg<T, MON_GAUSS> {
  int nb;
  T amp[4], nh[4], c0[4], c1[4], c2[4];
  __device__ explicit MonReg(const MonP<T>& m) : nb(m.nb) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      amp[b] = m.bamp[b];
      nh[b] = m.bnh[b] * ExpK<T>::kLog2e;
      c0[b] = m.bc[b][0];
      c1[b] = m.bc[b][1];
      c2[b] = m.bc[b][2];
    }
  }
  template <int DIM> __device__ T rho(T x0, T x1, T x2) const {
    T acc = T(1);
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (b < nb) {
        const T d0 = x0 - c0[b], d1 = x1 - c1[b];
        T r2 = d0 * d0 + d1 * d1;
        if (DIM == 3) r2 += (x2 - c2[b]) * (x2 - c2[b]);
        acc += amp[b] * ExpK<T>::ex(r2 * nh[b]);
      }
    return acc;
  }
};

template <typename T> struct MonReg<T, MON_SEPARABLE> {
  T a4[3], nk[3], c[3];
  __device__ explicit MonReg(const MonP<T>& m) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      a4[q] = T(4) * m.aa[q];
      nk[q] = T(-2) * m.ka[q] * ExpK<T>::kLog2e;
      c[q] = m.c[q];
    }
  }
  __device__ T factor(int q, T x) const { return one_plus_sech2(a4[q], ExpK<T>::ex(nk[q] * fabs(x - c[q]))); }
  template <int DIM> __device__ T rho(T x0, T x1, T x2) const {
    T p = factor(0, x0) * factor(1, x1);
    if (DIM == 3) p *= factor(2, x2);
    return p;
  }
};

// Arc-length monitors rho = sqrt(1 + g2), g2 = |grad u|^2 (Sec. 4, eq. monitfn), as 1 plus the
// excess g2 / (1 + sqrt(1 + g2)), free of cancellation where g2 is small.
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double fsqrt(double x) { return sqrt(x); }
template <typename T>
__device__ inline T arclen_rho(T g2) { return g2 * frcp(T(1) + fsqrt(T(1) + g2)) + T(1); }

// sine and cosine of an angle given as a * r2: FP32 takes the hardware sine and cosine, whose
// argument is in revolutions (a pre-divided by 2 pi); FP64 calls sincos on radians.
template <typename T> struct Turn;
template <> struct Turn<float> {
  static constexpr float kScale = 0.159154943091895336f;  // 1 / (2 pi)
  static __device__ inline void sc(float a, float& s, float& c) {
    s = __builtin_amdgcn_sinf(a);
    c = __builtin_amdgcn_cosf(a);
  }
};
template <> struct Turn<double> {
  static constexpr double kScale = 1.0;
  static __device__ inline void sc(double a, double& s, double& c) { sincos(a, &s, &c); }
};

// u = 1 / (1 + exp((x_0 + x_1 - r0) / (2 eps))): grad u = -(1, 1) sech^2(a) / (8 eps),
// a = (x_0 + x_1 - r0) / (4 eps), so g2 = 2 sech^4(a) / (8 eps)^2
template <typename T> struct MonReg<T, MON_ARC_FRONT> {
  T a4, nk, s0;
  __device__ explicit MonReg(const MonP<T>& m)
      : a4(T(4) * T(1.41421356237309505) / (T(8) * m.k)), nk(T(-0.5) / m.k * ExpK<T>::kLog2e), s0(m.r0) {}
  template <int DIM> __device__ T rho(T x0, T x1, T) const {
    const T g = sech2_of(a4, ExpK<T>::ex(nk * fabs(x0 + x1 - s0)));
    return arclen_rho(g * g);
  }
};

// u = 1 + amp / (1 + q), q = k r^2 cos^2(t - w r^2) about c.  With d = x - c,
// P = d_0 cos(w r^2) + d_1 sin(w r^2) (= r cos(t - w r^2)) and Q = d_1 cos(w r^2) - d_0 sin(w r^2),
// q = k P^2 and grad q = 2 k P ((cos, sin)(w r^2) + 2 w Q d): no angle and no division by r.
template <typename T> struct MonReg<T, MON_ARC_SPIRAL> {
  T amp, kq, w2, wt, c0, c1;
  __device__ explicit MonReg(const MonP<T>& m)
      : amp(m.amp), kq(m.k), w2(T(2) * m.tw), wt(m.tw * Turn<T>::kScale), c0(m.c[0]), c1(m.c[1]) {}
  template <int DIM> __device__ T rho(T x0, T x1, T) const {
    const T d0 = x0 - c0, d1 = x1 - c1;
    const T r2 = d0 * d0 + d1 * d1;
    T S, C;
    Turn<T>::sc(wt * r2, S, C);
    const T P = d0 * C + d1 * S, Q = d1 * C - d0 * S;
    const T q1 = T(1) + kq * P * P;
    const T f = T(2) * amp * kq * P * frcp(q1 * q1);
    const T g0 = f * (C + w2 * Q * d0), g1 = f * (S + w2 * Q * d1);
    return arclen_rho(g0 * g0 + g1 * g1);
  }
};

// u = sum_b tanh(k (|x - c_b|^2 - r0^2)): grad u = sum_b 2 k sech^2(k (|x - c_b|^2 - r0^2)) (x - c_b)
template <typename T> struct MonReg<T, MON_ARC_SPHERES> {
  int nb;
  T a4, nk, r02;
  T c0[kMaxBumps], c1[kMaxBumps], c2[kMaxBumps];
  __device__ explicit MonReg(const MonP<T>& m)
      : nb(m.nb), a4(T(8) * m.k), nk(T(-2) * m.k * ExpK<T>::kLog2e), r02(m.r02) {
#pragma unroll
    for (int b = 0; b < kMaxBumps; ++b) {
      c0[b] = m.bc[b][0];
      c1[b] = m.bc[b][1];
      c2[b] = m.bc[b][2];
    }
  }
  template <int DIM> __device__ T rho(T x0, T x1, T x2) const {
    T g0 = T(0), g1 = T(0), g2 = T(0);
#pragma unroll
    for (int b = 0; b < kMaxBumps; ++b)
      if (b < nb) {
        const T d0 = x0 - c0[b], d1 = x1 - c1[b], d2 = DIM == 3 ? x2 - c2[b] : T(0);
        const T r2 = d0 * d0 + d1 * d1 + d2 * d2;
        const T s = sech2_of(a4, ExpK<T>::ex(nk * fabs(r2 - r02)));
        g0 += s * d0;
        g1 += s * d1;
        g2 += s * d2;
      }
    return arclen_rho(g0 * g0 + g1 * g1 + g2 * g2);
  }
};

// Status of the nodes of a block: whether some 1 + e seen was <= 0 (det(I + D^2 phi) <= 0 is a
// tangled mesh).  A non-finite F needs no test here: every DCT product
// carries it (NaN and inf times any coefficient, zero included, stay non-finite) into the update
// of its line, and the update kernels flag a non-finite update.
template <typename T>
struct NodeCheck {
  // the least 1 + e this lane has seen, kept by a compare and a select per node (a flag kept per
  // lane across the store's branch costs two vector instructions more); a NaN never compares
  // less, so a state already non-finite (flagged by the update) does not count as tangled
  T lo = T(1);
  __device__ inline void add(T one_plus_e) { lo = one_plus_e < lo ? one_plus_e : lo; }
  // only where `on` (a node that is not artificial)
  __device__ inline void add_if(bool on, T one_plus_e) { lo = on && one_plus_e < lo ? one_plus_e : lo; }
  __device__ inline int bits() const { return lo <= T(0) ? ST_TANGLED : 0; }
};

// Per-workgroup constants of a subdomain, copied into registers once.
template <typename T>
struct StencilCtx {
  T lvt, a0, a1, a2, h0, h1, h2;
  int n0, n1, n2, off0, off1, off2, art, inst;
};


constexpr int kStR = 16;                               // output rows per chunk (2D: i0, 3D: i1)
constexpr int kStWmax = 72;                            // widest block along the last axis
constexpr int kStS = kStWmax + 2;                      // LDS row stride
constexpr int kStHR = kStR + 2;                        // staged rows per chunk
constexpr int kStPts = (kStR * kStWmax + 255) / 256;   // output nodes per thread per chunk
constexpr int kStLd = (kStHR + 3) / 4;                 // staged rows per wave

// Halo staging of one 18 x (W + 2) block, a fixed number of loads per thread so that the wait
// before a commit only has to cover that block's loads: wave w loads rows w, w + 4, .., w + 16
// at column lane (a row past the 18th is loaded clamped and not staged), and thread t < 180
// loads element (t / 10, 64 + t % 10) of the columns beyond the wave width (clamped when the
// block is narrower).  Values land in registers first, so later chunks' loads are in flight
// while the current chunk is computed.  Column offsets (bytes) are fixed for the block.
constexpr int kStPre = kStLd + 1;  // loads per thread per chunk

struct HaloCols {
  unsigned bA;  // byte offset of column `lane` (mirrored index along the last axis)
  unsigned bE;  // byte offset of this thread's element beyond the wave width
  int rE;       // its row within the block (clamped to the last staged row)
  int sE;       // its LDS offset within the block, or -1 (no such element)
};

template <typename T>
__device__ inline HaloCols halo_cols(int col0, int W, int n) {
  const int lane = threadIdx.x & 63, t = threadIdx.x;
  HaloCols h;
  h.bA = (unsigned)mirror_clamp(col0 + lane - 1, n) * sizeof(T);
  const int re = t / 10, ce = 64 + t % 10;
  const bool ok = re < kStHR && ce < W + 2;
  h.rE = min(re, kStHR - 1);
  h.bE = (unsigned)mirror_clamp(col0 + ce - 1, n) * sizeof(T);
  h.sE = ok ? re * kStS + ce : -1;
  return h;
}

// rowo[k]: byte offset of staged row wave + 4 k (wave-uniform); this thread's extra element sits
// at byte offset vE (per lane) + sE (wave-uniform)
template <typename T>
__device__ inline void halo_issue(T (&pre)[kStPre], const HaloCols& hc, const BufView& src,
                                  const unsigned (&rowo)[kStLd], unsigned vE, unsigned sE) {
#pragma unroll
  for (int k = 0; k < kStLd; ++k) pre[k] = buf_ld<T>(src, hc.bA, rowo[k]);
  pre[kStLd] = buf_ld<T>(src, vE, sE);
}

template <typename T>
__device__ inline void halo_commit(T* slot, const HaloCols& hc, const T (&pre)[kStPre]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kStLd; ++k) {
    const int r = wave + 4 * k;
    if (r < kStHR) slot[r * kStS + lane] = pre[k];
  }
  if (hc.sE >= 0) slot[hc.sE] = pre[kStLd];
}

// Wait until every vector-memory load of this wave has returned (s_waitcnt vmcnt(0); expcnt and
// lgkmcnt left free).  Issued once after the per-block parameter loads: the in-order vmcnt
// counter could otherwise make the first use of a parameter inside the chunk loop wait for the
// next chunk's prefetch as well.
__device__ inline void vmem_drain() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The output nodes of a thread within a 16-row x W-column chunk: slot m is linear index
// tid + 256 m, fixed for every chunk of the block.  Every slot is evaluated (an absent one reads
// a valid LDS cell) and masked afterwards, so the node loop has no divergent branch but the
// store's.
template <typename T>
struct Slots {
  int lds[kStPts];       // LDS element offset of the node's centre
  unsigned out[kStPts];  // byte offset in the chunk's output block
  int row[kStPts];       // row within the chunk (kStR: no node)
  T xc[kStPts];          // coordinate along the last axis: a + (global index) h
  int valid;             // bit m: slot m holds a node
  int live;              // bit m: ... whose column (3D: row and column) is not artificial
  int wave;              // bit m: some lane of this wave holds a node in slot m (uniform)
};

// bit m of the result: some lane of the wave has bit m set in `bits`
__device__ inline int wave_any_bits(int bits) {
  int r = 0;
#pragma unroll
  for (int m = 0; m < kStPts; ++m) r |= (__ballot((bits >> m) & 1) != 0) ? 1 << m : 0;
  return __builtin_amdgcn_readfirstlane(r);
}

// The output nodes of a thread in the 2D march (as Slots), in the form the node loop reads with
// the fewest vector instructions: the LDS byte offset of the node's upper-left neighbour, so the
// nine stencil reads are immediate offsets from one register; the global row index kept as T
// (whole numbers, exact) and stepped by kStR per chunk instead of converted per node; the valid
// and live flags as lane masks in scalar registers, which the selects and the store's branch use
// as they are.
template <typename T>
struct Slots2 {
  unsigned lds[kStPts];  // LDS byte offset of element (row - 1, column - 1) of the staged block
  unsigned out[kStPts];  // byte offset in the chunk's output block
  int row[kStPts];       // row within the chunk (kStR: no node)
  T xc[kStPts];          // coordinate along the last axis: a + (global index) h
  T gr[kStPts];          // global row index of the node in the current chunk
  uint64_t valid[kStPts];  // lanes whose slot m holds a node (wave-uniform lane mask)
  uint64_t live[kStPts];   // ... whose column is not artificial
};

// 2D: rows [row0, row0 + nrows) x columns [col0, col0 + W) of a subdomain, 16 rows per chunk.
// The artificial nodes were filled by the transmission gather before the launch.
template <typename T, int MK>
__device__ inline void stencil_march2(const StencilCtx<T>& K, const MonP<T>& mp, const T* phi_, T* F_, T* sm,
                                      int row0, int nrows, int col0, int W, int& bad) {
  const MonReg<T, MK> M(mp);
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int n0 = K.n0, n1 = K.n1;
  const unsigned rowb = (unsigned)n1 * sizeof(T);  // bytes per row
  // one view per array: a 2D subdomain (axes of at most 1025 nodes) holds at most 8.4 MB
  const BufView phi = buf_view(phi_, (unsigned)n0 * rowb), F = buf_view(F_, (unsigned)n0 * rowb);
  const HaloCols hc = halo_cols<T>(col0, W, n1);
  const T h0 = K.h0, h1 = K.h1;
  Slots2<T> sl;
#pragma unroll
  for (int m = 0; m < kStPts; ++m) {
    const int idx = (int)threadIdx.x + 256 * m;
    const int rr = idx / W, cc = idx - rr * W;
    const bool ok = idx < kStR * W;
    sl.lds[m] = (unsigned)(ok ? rr * kStS + cc : 0) * sizeof(T);
    sl.out[m] = (unsigned)(rr * n1 + cc) * sizeof(T);
    sl.row[m] = ok ? rr : kStR;
    sl.xc[m] = fma(T(K.off1 + col0 + cc), h1, K.a1);
    sl.gr[m] = T(K.off0 + row0 + (ok ? rr : 0));
    sl.valid[m] = __ballot(ok);
    sl.live[m] = __ballot(ok && !is_artificial(K.art, 1, col0 + cc, n1));
  }
  const T r2h0 = T(1) / (T(2) * h0), r2h1 = T(1) / (T(2) * h1);
  const T rh00 = T(1) / (h0 * h0), rh11 = T(1) / (h1 * h1), r4h01 = T(1) / (T(4) * h0 * h1);
  NodeCheck<T> chk;
  const int rend = row0 + nrows;
  // two chunks' loads in flight: the registers of chunk k are reloaded with chunk k + 2 as soon
  // as chunk k is in LDS (the loop is unrolled by two so each register set has fixed names)
  T preA[kStPre], preB[kStPre];
  // the row of this thread's extra element, rb + rE - 1, needs no mirror away from the array's
  // first and last rows: its offset is then a per-block one plus a wave-uniform one
  const unsigned vEi = hc.bE + (unsigned)hc.rE * rowb;
  auto issue = [&](T (&pre)[kStPre], int rb) {
    unsigned rowo[kStLd];
#pragma unroll
    for (int k = 0; k < kStLd; ++k) rowo[k] = (unsigned)mirror_clamp(rb + wv + 4 * k - 1, n0) * rowb;
    unsigned vE, sE;
    if (rb >= 1 && rb + kStHR - 2 <= n0 - 1) {
      vE = vEi;
      sE = (unsigned)(rb - 1) * rowb;
    } else {
      asm volatile("");  // keeps the per-lane mirror in this (rare, uniform) branch
      vE = hc.bE + (unsigned)mirror_clamp(rb + hc.rE - 1, n0) * rowb;
      sE = 0;
    }
    halo_issue(pre, hc, phi, rowo, vE, sE);
  };
  // EDGE: the first or last chunk of the block, whose rows may lie beyond the block or on an
  // artificial face; its flags are derived per node, the interior chunks use the block's masks
  auto chunk = [&](T (&pre)[kStPre], int rb, auto edge_tag) {
    constexpr bool EDGE = decltype(edge_tag)::value;
    if (rb != row0) __syncthreads();  // every thread is done reading the previous chunk
    halo_commit(sm, hc, pre);
    __syncthreads();
    // issued unconditionally (past the block it loads clamped rows just read): the number of
    // memory operations between a load and its use must not depend on the path, or the wait
    // before the commit would have to drain the other register set's loads as well
    issue(pre, rb + 2 * kStR);
    const unsigned Fc = (unsigned)(rb * n1 + col0) * sizeof(T);  // the chunk's output block
    const int rlim = min(kStR, rend - rb);
    const int rlo = (rb == 0 && (K.art & 1)) ? 0 : -1;
    const int rhi = (rb + kStR > n0 - 1 && (K.art & 2)) ? n0 - 1 - rb : -1;
#pragma unroll
    for (int m = 0; m < kStPts; ++m) {
      if (sl.valid[m] != 0) {  // some node of this wave in slot m (uniform branch)
        bool lv = __builtin_amdgcn_inverse_ballot_w64(sl.live[m]);
        bool st = __builtin_amdgcn_inverse_ballot_w64(sl.valid[m]);
        if constexpr (EDGE) {
          const int rr = sl.row[m];
          st = st && rr < rlim;
          lv = lv && rr < rlim && rr != rlo && rr != rhi;
        }
        const T* t = (const T*)((const char*)sm + sl.lds[m]);  // upper-left neighbour
        const T c0 = t[kStS + 1];
        const T xm = t[1], xp = t[2 * kStS + 1], ym = t[kStS], yp = t[kStS + 2];
        const T hxx = (xp - T(2) * c0 + xm) * rh00;
        const T hyy = (yp - T(2) * c0 + ym) * rh11;
        const T hxy = (t[2 * kStS + 2] - t[2 * kStS] - t[2] + t[0]) * r4h01;
        const T e = hxx + hyy + (hxx * hyy - hxy * hxy);  // det(I + D^2 phi) - 1
        // x + grad phi: the node's coordinate a + (global index) h, then the central difference
        const T x0 = fma(xp - xm, r2h0, fma(sl.gr[m], h0, K.a0));
        const T x1 = fma(yp - ym, r2h1, sl.xc[m]);
        const T fv = rhs_of(K.lvt, M.template rho<2>(x0, x1, T(0)), e);
        const T f = lv ? fv : T(0);
        chk.add_if(lv, T(1) + e);
        if (st) buf_st(F, sl.out[m], Fc, f);
      }
      sl.gr[m] += T(kStR);
    }
  };
  auto any_chunk = [&](T (&pre)[kStPre], int rb) {
    const bool edge = rb + kStR > rend || (rb == 0 && (K.art & 1)) || (rb + kStR > n0 - 1 && (K.art & 2));
    if (edge) chunk(pre, rb, std::true_type{});
    else chunk(pre, rb, std::false_type{});
  };
  vmem_drain();
  issue(preA, row0);
  issue(preB, row0 + kStR);
  int rb = row0;
  for (; rb + kStR < rend; rb += 2 * kStR) {  // both chunks of a pair on every path
    any_chunk(preA, rb);
    any_chunk(preB, rb + kStR);
  }
  if (rb < rend) any_chunk(preA, rb);
  bad |= chk.bits();
}

// 3D: planes [p0, p0 + np) of a 16-row (i1) x W-column (i2) block; a ring of three staged planes
// in LDS, the next plane loading while the current one is computed.  The artificial nodes were
// filled by the transmission gather before the launch.
template <typename T, int MK>
__device__ inline void stencil_march3(const StencilCtx<T>& K, const MonP<T>& mp, const T* phi_, T* F_, T* sm,
                                      int p0, int np, int row0, int col0, int W, int& bad) {
  const MonReg<T, MK> M(mp);
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int n0 = K.n0, n1 = K.n1, n2 = K.n2;
  const unsigned rowb = (unsigned)n2 * sizeof(T), plb = (unsigned)n1 * rowb;  // bytes per row, plane
  // one buffer view per plane (a subdomain may exceed the 4 GiB reach of a view's offsets)
  auto plane = [&](const void* a, int p) { return buf_view((const char*)a + (size_t)p * plb, plb); };
  const HaloCols hc = halo_cols<T>(col0, W, n2);
  // the staged rows of the block are the same on every plane
  unsigned rowo[kStLd];
#pragma unroll
  for (int k = 0; k < kStLd; ++k) rowo[k] = (unsigned)mirror_clamp(row0 + wv + 4 * k - 1, n1) * rowb;
  const unsigned vE = hc.bE + (unsigned)mirror_clamp(row0 + hc.rE - 1, n1) * rowb;
  constexpr int PL = kStHR * kStS;
  const T h0 = K.h0, h1 = K.h1, h2 = K.h2;
  Slots<T> sl;
  T x1s[kStPts];
  sl.valid = 0;
  sl.live = 0;
#pragma unroll
  for (int m = 0; m < kStPts; ++m) {
    const int idx = (int)threadIdx.x + 256 * m;
    const int rr = idx / W, cc = idx - rr * W;
    const int j = row0 + rr, k = col0 + cc;
    const bool ok = idx < kStR * W && j < n1;
    sl.lds[m] = ok ? (rr + 1) * kStS + cc + 1 : kStS + 1;
    sl.out[m] = (unsigned)(rr * n2 + cc) * sizeof(T);
    sl.row[m] = ok ? rr : kStR;
    sl.xc[m] = fma(T(K.off2 + k), h2, K.a2);
    x1s[m] = fma(T(K.off1 + j), h1, K.a1);
    sl.valid |= ok ? 1 << m : 0;
    sl.live |= (ok && !is_artificial(K.art, 1, j, n1) && !is_artificial(K.art, 2, k, n2)) ? 1 << m : 0;
  }
  sl.wave = wave_any_bits(sl.valid);
  const T r2h0 = T(1) / (T(2) * h0), r2h1 = T(1) / (T(2) * h1), r2h2 = T(1) / (T(2) * h2);
  const T rh00 = T(1) / (h0 * h0), rh11 = T(1) / (h1 * h1), rh22 = T(1) / (h2 * h2);
  const T r4h01 = T(1) / (T(4) * h0 * h1), r4h02 = T(1) / (T(4) * h0 * h2), r4h12 = T(1) / (T(4) * h1 * h2);
  NodeCheck<T> chk;
  // plane p0 - 1 -> LDS slot 0, p0 -> slot 1, p0 + q + 1 -> slot (q + 2) % 3; two planes' loads in
  // flight (register sets A / B alternate, the loop is unrolled by two)
  T preA[kStPre], preB[kStPre];
  auto issue = [&](T (&pre)[kStPre], int p) { halo_issue(pre, hc, plane(phi_, mirror_clamp(p, n0)), rowo, vE, 0u); };
  auto step = [&](T (&pre)[kStPre], int q) {
    const int p = p0 + q;
    __syncthreads();  // the slot about to be refilled is no longer read
    halo_commit(sm + ((q + 2) % 3) * PL, hc, pre);
    __syncthreads();
    issue(pre, p + 3);  // unconditional, as in the 2D march
    const int sp = (q % 3) * PL, scur = ((q + 1) % 3) * PL, sn = ((q + 2) % 3) * PL;
    const int live = is_artificial(K.art, 0, p, n0) ? 0 : sl.live;
    const T x0b = fma(T(K.off0 + p), h0, K.a0);
    const BufView Fp = plane(F_, p);
    const unsigned Fc = (unsigned)(row0 * n2 + col0) * sizeof(T);  // the plane's output block
#pragma unroll
    for (int m = 0; m < kStPts; ++m) {
      if (!((sl.wave >> m) & 1)) continue;  // no node of this wave in slot m (uniform branch)
      const T* c = sm + scur + sl.lds[m];
      const T* a = sm + sp + sl.lds[m];
      const T* b = sm + sn + sl.lds[m];
      const T c0 = c[0];
      const T xm = a[0], xp = b[0];
      const T ym = c[-kStS], yp = c[kStS];
      const T zm = c[-1], zp = c[1];
      const T d00 = (xp - T(2) * c0 + xm) * rh00;
      const T d11 = (yp - T(2) * c0 + ym) * rh11;
      const T d22 = (zp - T(2) * c0 + zm) * rh22;
      const T d01 = (b[kStS] - b[-kStS] - a[kStS] + a[-kStS]) * r4h01;
      const T d02 = (b[1] - b[-1] - a[1] + a[-1]) * r4h02;
      const T d12 = (c[kStS + 1] - c[kStS - 1] - c[-kStS + 1] + c[-kStS - 1]) * r4h12;
      // det(I + H) - 1 = tr H + (sum of principal 2x2 minors) + det H
      const T tr = d00 + d11 + d22;
      const T m2 = (d00 * d11 - d01 * d01) + (d00 * d22 - d02 * d02) + (d11 * d22 - d12 * d12);
      const T d3 = d00 * (d11 * d22 - d12 * d12) - d01 * (d01 * d22 - d12 * d02) + d02 * (d01 * d12 - d11 * d02);
      const T e = tr + m2 + d3;
      // x + grad phi (central differences)
      const T y0 = fma(xp - xm, r2h0, x0b), y1 = fma(yp - ym, r2h1, x1s[m]), y2 = fma(zp - zm, r2h2, sl.xc[m]);
      const T fv = rhs_of(K.lvt, M.template rho<3>(y0, y1, y2), e);
      const bool lv = (live >> m) & 1;
      const T f = lv ? fv : T(0);
      chk.add_if(lv, T(1) + e);
      if ((sl.valid >> m) & 1) buf_st(Fp, sl.out[m], Fc, f);
    }
  };
  vmem_drain();
  issue(preA, p0 - 1);
  halo_commit(sm, hc, preA);
  issue(preA, p0);
  halo_commit(sm + PL, hc, preA);
  issue(preA, p0 + 1);
  issue(preB, p0 + 2);
  int q = 0;
  for (; q + 1 < np; q += 2) {  // both planes of a pair on every path
    step(preA, q);
    step(preB, q + 1);
  }
  if (q < np) step(preA, q);
  bad |= chk.bits();
}

#pragma clang fp contract(fast)  // the compiler's default for HIP again

template <typename T>
__device__ inline const MonP<T>* load_ctx(const StepArgs& sa, int sub, StencilCtx<T>& K, const T*& phi, T*& F) {
  const SubDev& S = sa.subs[sub];
  const InstDev& I = sa.insts[S.inst];
  K.lvt = T(I.log_vol_theta);
  K.a0 = T(S.a[0]);
  K.a1 = T(S.a[1]);
  K.a2 = T(S.a[2]);
  K.h0 = T(S.h[0]);
  K.h1 = T(S.h[1]);
  K.h2 = T(S.h[2]);
  K.n0 = S.n[0];
  K.n1 = S.n[1];
  K.n2 = S.n[2];
  K.off0 = S.off[0];
  K.off1 = S.off[1];
  K.off2 = S.off[2];
  K.art = S.art;
  K.inst = S.inst;
  phi = (const T*)S.phi;
  F = (T*)S.F;
  return &mon_of(I, T(0));
}

// Stencil into F (2D subdomains).  tile = (sub, row0, col0 | W << 16, nrows): the block of rows
// [row0, row0 + nrows) and columns [col0, col0 + W), W <= 72, marched 16 rows at a time.  Mirror
// ghosts are applied while staging; the node loop is specialised per monitor kind.  A step
// launches the transmission gather first, so every halo value is the local array's.
template <typename T>
__global__ __launch_bounds__(256) void stencil2_kernel(const int4* __restrict__ tiles, int ntiles, StepArgs sa) {
  __shared__ T sm[kStHR * kStS];
  const int tix = xcd_tile();
  if (tix >= ntiles) return;
  const int4 tl = tiles[tix];
  StencilCtx<T> K;
  const T* phi;
  T* F;
  const MonP<T>* mp = load_ctx(sa, tl.x, K, phi, F);
  const int row0 = tl.y, col0 = tl.z & 0xffff, W = tl.z >> 16, nrows = tl.w;
  int bad = 0;
  switch (mp->kind) {
    case MON_CONST: stencil_march2<T, MON_CONST>(K, *mp, phi, F, sm, row0, nrows, col0, W, bad); break;
    case MON_RADIAL: stencil_march2<T, MON_RADIAL>(K, *mp, phi, F, sm, row0, nrows, col0, W, bad); break;
    case MON_SINE: stencil_march2<T, MON_SINE>(K, *mp, phi, F, sm, row0, nrows, col0, W, bad); break;
    case MON_GAUSS: stencil_march2<T, MON_GAUSS>(K, *mp, phi, F, sm, row0, nrows, col0, W, bad); break;
    case MON_ARC_FRONT: stencil_march2<T, MON_ARC_FRONT>(K, *mp, phi, F, sm, row0, nrows, col0, W, bad); break;
    case MON_ARC_SPIRAL: stencil_march2<T, MON_ARC_SPIRAL>(K, *mp, phi, F, sm, row0, nrows, col0, W, bad); break;
    case MON_ARC_SPHERES: stencil_march2<T, MON_ARC_SPHERES>(K, *mp, phi, F, sm, row0, nrows, col0, W, bad); break;
    default: stencil_march2<T, MON_SEPARABLE>(K, *mp, phi, F, sm, row0, nrows, col0, W, bad); break;
  }
  if (bad) atomicOr(&sa.status[K.inst], bad);
}

// Stencil into F (3D subdomains).  tile = (sub, p0 | np << 16, row0, col0 | W << 16): planes
// [p0, p0 + np) of the block of 16 rows (i1) from row0 and W <= 72 columns (i2) from col0.
template <typename T>
__global__ __launch_bounds__(256) void stencil3_kernel(const int4* __restrict__ tiles, int ntiles, StepArgs sa) {
  __shared__ T sm[3 * kStHR * kStS];
  const int tix = xcd_tile();
  if (tix >= ntiles) return;
  const int4 tl = tiles[tix];
  StencilCtx<T> K;
  const T* phi;
  T* F;
  const MonP<T>* mp = load_ctx(sa, tl.x, K, phi, F);
  const int p0 = tl.y & 0xffff, np = tl.y >> 16, row0 = tl.z, col0 = tl.w & 0xffff, W = tl.w >> 16;
  int bad = 0;
  switch (mp->kind) {
    case MON_CONST: stencil_march3<T, MON_CONST>(K, *mp, phi, F, sm, p0, np, row0, col0, W, bad); break;
    case MON_RADIAL: stencil_march3<T, MON_RADIAL>(K, *mp, phi, F, sm, p0, np, row0, col0, W, bad); break;
    case MON_SINE: stencil_march3<T, MON_SINE>(K, *mp, phi, F, sm, p0, np, row0, col0, W, bad); break;
    case MON_GAUSS: stencil_march3<T, MON_GAUSS>(K, *mp, phi, F, sm, p0, np, row0, col0, W, bad); break;
    case MON_ARC_FRONT: stencil_march3<T, MON_ARC_FRONT>(K, *mp, phi, F, sm, p0, np, row0, col0, W, bad); break;
    case MON_ARC_SPIRAL: stencil_march3<T, MON_ARC_SPIRAL>(K, *mp, phi, F, sm, p0, np, row0, col0, W, bad); break;
    case MON_ARC_SPHERES: stencil_march3<T, MON_ARC_SPHERES>(K, *mp, phi, F, sm, p0, np, row0, col0, W, bad); break;
    default: stencil_march3<T, MON_SEPARABLE>(K, *mp, phi, F, sm, p0, np, row0, col0, W, bad); break;
  }
  if (bad) atomicOr(&sa.status[K.inst], bad);
}

// ------------------------------------------------------------------------------------------
// block reductions (256 threads, fixed order)
// ------------------------------------------------------------------------------------------

__device__ inline double block_sum256(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// block_sum256 for a workgroup of NW waves (red holds NW doubles); NW = 4 adds in the same order
template <int NW>
__device__ inline double block_sum_w(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = (red[0] + red[1]) + (red[2] + red[3]);
  if (NW == 8) r += (red[4] + red[5]) + (red[6] + red[7]);
  __syncthreads();
  return r;
}

__device__ inline double block_min256(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------------------------------
// K3/K4/K5: the preconditioner's mode products on the matrix cores.
//
// A mode product contracts one axis of a subdomain array with an n x n DCT matrix.  Both DCT
// matrices are symmetric, so every operand is read as "row r of a row-major matrix": rows of the
// A operand are its rows, columns of the B operand are rows of B^T = B.  A 16 x 16 output block
// takes KB-deep fragments; lane l supplies row l % 16 at k offsets set by g = l / 16:
//   fp16 (16x16x32):   k = 8 g .. 8 g + 7      f32 / f64 (16x16x4):   k = g
// Data operands are staged whole-K in LDS (zero padded to ld); basis fragments stream from L2.
//
// Three kernels cover every product of a step:
//   fwd_last   stencil of 16 rows -> LDS, then  T[rows, :] = F[rows, :] * A_last
//   strip      a 16-column strip of the [n_axis][rest] view: Y = Bas * X (axis 0 or the middle
//              axis in 3D); PAIR: Y = B_0 * (S o (A_0 * X)) with the spectral scale in between
//   inv_last   16 rows: delta = T[rows, :] * B_last, then phi += dt (delta - shift) on live
//              nodes and the FP64 residual partial sum
// ------------------------------------------------------------------------------------------

template <int KIND> struct Op;

// Fragment-major order of a DCT matrix for the 16x16x4 products (FP32 and FP64): entry (r, k) of a
// matrix with ldb (a multiple of 4) padded columns sits at ((r / 16) (ldb / 4) + k / 4) 64 +
// (k % 4) 16 + r % 16.  The fragment of row block r / 16 and k steps k0 .. k0 + 3 (k0 a multiple
// of 4) is then one contiguous run in lane order (lane l = 16 g + l16 takes row l16, k = k0 + g):
// a wave's load touches 2 (FP32) or 4 (FP64) cache lines instead of 16.
__device__ inline long frag_index(int ldb, int r, int k0, int g) {
  return ((long)(r >> 4) * (ldb >> 2) + (k0 >> 2)) * 64 + g * 16 + (r & 15);
}

template <> struct Op<PREC_SPLIT16> {
  typedef float T;
  typedef float4_t acc_t;
  enum { KB = 32, LDS_BYTES = 4, SCALED = 1 };
  struct frag { half8_t hi, lo; };
  // The data operand is staged in LDS in fp32; once its block scale is known, presplit turns it
  // in place into fp16 hi + lo of x * 2^t (block floating point: small entries keep their absolute
  // accuracy relative to the tile's largest one instead of falling to fp16 subnormals).  Each
  // group of 8 fp32 entries (32 bytes) becomes 8 hi then 8 lo halves, so a fragment is two 16-byte
  // reads and every entry is converted once, not once per product that reads it.
  static __device__ inline void put(char* lds, int ld, int r, int k, float x) { ((float*)lds)[r * ld + k] = x; }
  // rows [0, rows) of stride ld entries, k in [0, kend) (kend a multiple of 8); row r takes the
  // scale sc[r / rows_per_scale].  All threads of the workgroup take part; a barrier must follow.
  static __device__ inline void presplit(char* lds, int ld, int rows, int kend, const float* sc,
                                         int rows_per_scale) {
    const int groups = kend >> 3;
    for (int idx = threadIdx.x; idx < rows * groups; idx += blockDim.x) {
      const int r = idx / groups, k = (idx - r * groups) * 8;
      const float s = sc[r / rows_per_scale];
      float4_t* p = (float4_t*)((float*)lds + r * ld + k);
      const float4_t u = p[0], v = p[1];
      half8_t hi, lo;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float x = u[i] * s, y = v[i] * s;
        const _Float16 hx = (_Float16)x, hy = (_Float16)y;
        hi[i] = hx;
        hi[4 + i] = hy;
        lo[i] = (_Float16)(x - (float)hx);
        lo[4 + i] = (_Float16)(y - (float)hy);
      }
      half8_t* q = (half8_t*)p;
      q[0] = hi;
      q[1] = lo;
    }
  }
  static __device__ inline frag lds_frag(const char* lds, int ld, int r, int k0, int g, float) {
    const half8_t* p = (const half8_t*)((const float*)lds + r * ld + k0 + 8 * g);
    frag f;
    f.hi = p[0];
    f.lo = p[1];
    return f;
  }
  // a fragment of an operand still in fp32, split on the fly: the products with a basis copy in
  // LDS read each data fragment once per wave, where a separate pass would only add latency
  static __device__ inline frag lds_frag_cvt(const char* lds, int ld, int r, int k0, int g, float sc) {
    const float4_t* p = (const float4_t*)((const float*)lds + r * ld + k0 + 8 * g);
    const float4_t u = p[0], v = p[1];
    frag f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float x = u[i] * sc, y = v[i] * sc;
      const _Float16 hx = (_Float16)x, hy = (_Float16)y;
      f.hi[i] = hx;
      f.hi[4 + i] = hy;
      f.lo[i] = (_Float16)(x - (float)hx);
      f.lo[4 + i] = (_Float16)(y - (float)hy);
    }
    return f;
  }
  static __device__ inline frag glob_frag(const void* hi, const void* lo, int ld, int r, int k0, int g) {
    frag f;
    f.hi = *(const gmem<half8_t>*)(gp<_Float16>(hi) + (long)r * ld + k0 + 8 * g);
    f.lo = *(const gmem<half8_t>*)(gp<_Float16>(lo) + (long)r * ld + k0 + 8 * g);
    return f;
  }
  // basis fragment from a copy of the basis in LDS (same layout as in global memory)
  static __device__ inline frag lbasis_frag(const char* hi, const char* lo, int ld, int r, int k0, int g) {
    frag f;
    f.hi = *(const half8_t*)((const _Float16*)hi + r * ld + k0 + 8 * g);
    f.lo = *(const half8_t*)((const _Float16*)lo + r * ld + k0 + 8 * g);
    return f;
  }
  static __device__ inline frag zero_frag() {
    frag f;
    f.hi = half8_t{0, 0, 0, 0, 0, 0, 0, 0};
    f.lo = half8_t{0, 0, 0, 0, 0, 0, 0, 0};
    return f;
  }
  enum { BASIS_BYTES = 4 };  // LDS bytes per basis entry (hi + lo)
  // row strides pad 16 bytes beyond the padded axis length: the 16 rows of a fragment then start
  // in distinct LDS bank groups (operand: fp32 entries; basis: fp16 entries per array)
  enum { OPAD = 4, BPAD = 8 };
  static __device__ inline void mma(acc_t& c, const frag& a, const frag& b) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.lo, b.hi, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi, b.lo, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi, b.hi, c, 0, 0, 0);
  }
  static __device__ inline int crow(int g, int q) { return 4 * g + q; }
};

template <> struct Op<PREC_F32> {
  typedef float T;
  typedef float4_t acc_t;
  enum { KB = 4, LDS_BYTES = 4, SCALED = 0 };
  typedef float frag;
  static __device__ inline void put(char* lds, int ld, int r, int k, float x) { ((float*)lds)[r * ld + k] = x; }
  static __device__ inline void presplit(char*, int, int, int, const float*, int) {}
  static __device__ inline frag lds_frag(const char* lds, int ld, int r, int k0, int g, float) {
    return ((const float*)lds)[r * ld + k0 + g];
  }
  static __device__ inline frag lds_frag_cvt(const char* lds, int ld, int r, int k0, int g, float sc) {
    return lds_frag(lds, ld, r, k0, g, sc);
  }
  // basis matrices are stored fragment-major (see frag_index): one fragment is 256 contiguous
  // bytes, one per lane in lane order
  static __device__ inline frag glob_frag(const void* p, const void*, int ldb, int r, int k0, int g) {
    return gp<float>(p)[frag_index(ldb, r, k0, g)];
  }
  static __device__ inline frag lbasis_frag(const char* p, const char*, int ldb, int r, int k0, int g) {
    return ((const float*)p)[frag_index(ldb, r, k0, g)];
  }
  static __device__ inline frag zero_frag() { return 0.f; }
  enum { BASIS_BYTES = 4, OPAD = 4 };
  static __device__ inline void mma(acc_t& c, frag a, frag b) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int crow(int g, int q) { return 4 * g + q; }
};

template <> struct Op<PREC_F64> {
  typedef double T;
  typedef double4_t acc_t;
  enum { KB = 4, LDS_BYTES = 8, SCALED = 0 };
  typedef double frag;
  static __device__ inline void put(char* lds, int ld, int r, int k, double x) { ((double*)lds)[r * ld + k] = x; }
  static __device__ inline void presplit(char*, int, int, int, const float*, int) {}
  static __device__ inline frag lds_frag(const char* lds, int ld, int r, int k0, int g, float) {
    return ((const double*)lds)[r * ld + k0 + g];
  }
  static __device__ inline frag lds_frag_cvt(const char* lds, int ld, int r, int k0, int g, float sc) {
    return lds_frag(lds, ld, r, k0, g, sc);
  }
  // basis matrices fragment-major (see frag_index): one fragment is 512 contiguous bytes
  static __device__ inline frag glob_frag(const void* p, const void*, int ldb, int r, int k0, int g) {
    return gp<double>(p)[frag_index(ldb, r, k0, g)];
  }
  static __device__ inline frag lbasis_frag(const char* p, const char*, int ldb, int r, int k0, int g) {
    return ((const double*)p)[frag_index(ldb, r, k0, g)];
  }
  static __device__ inline frag zero_frag() { return 0.0; }
  enum { BASIS_BYTES = 8, OPAD = 2 };
  static __device__ inline void mma(acc_t& c, frag a, frag b) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // the f64 product interleaves rows: register q of lane group g holds row g + 4 q
  static __device__ inline int crow(int g, int q) { return g + 4 * q; }
};

// Basis fragments requested per batch: 8 for the 16x16x4 products (FP32, FP64: one k step per
// product, 32 k per batch, which divides every padded axis length), 4 for the split form
template <int KIND>
struct Depth {
  static constexpr int U = Op<KIND>::KB == 4 ? 8 : 4;
};

// N k steps from k0 (all within the contraction): the N basis fragments are requested first,
// then the N products are issued in ascending k.  BASIS_A: the basis fragment is the A operand
// (rows of the output), else the B operand (columns).
template <int KIND, bool BASIS_A, int N>
__device__ inline void mma_steps(typename Op<KIND>::acc_t& acc, const char* lds, int ldo, float sc, const void* bh,
                                 const void* bl, int ldb, int brow, int l16, int g, int k0) {
  typedef Op<KIND> O;
  typename O::frag b[N];
#pragma unroll
  for (int u = 0; u < N; ++u) b[u] = O::glob_frag(bh, bl, ldb, brow, k0 + u * O::KB, g);
#pragma unroll
  for (int u = 0; u < N; ++u) {
    const typename O::frag d = O::lds_frag(lds, ldo, l16, k0 + u * O::KB, g, sc);
    if constexpr (BASIS_A) O::mma(acc, b[u], d);
    else O::mma(acc, d, b[u]);
  }
}

// the last rem (< Depth) k steps from k0: one unrolled body per count, chosen once (rem is uniform)
template <int KIND, bool BASIS_A, int R>
__device__ inline void mma_tail(typename Op<KIND>::acc_t& acc, const char* lds, int ldo, float sc, const void* bh,
                                const void* bl, int ldb, int brow, int l16, int g, int k0, int rem) {
  if constexpr (R > 0) {
    if (rem == R) mma_steps<KIND, BASIS_A, R>(acc, lds, ldo, sc, bh, bl, ldb, brow, l16, g, k0);
    else mma_tail<KIND, BASIS_A, R - 1>(acc, lds, ldo, sc, bh, bl, ldb, brow, l16, g, k0, rem);
  }
}

// acc += the k steps [kb, ke) of (LDS operand rows) x (basis rows as columns), or the mirror
// image (BASIS_A), in ascending k.  kb and ke are multiples of the k step; ke is the axis length
// rounded up to the k step, so no product multiplies padding.  Basis fragments come from L2 in
// batches (Depth) requested before any is used, so their latencies overlap; the accumulator chain
// has no per-step branch (a conditional product would make the compiler copy the accumulator out
// and back, waiting for each product to finish).
template <int KIND, bool BASIS_A>
__device__ inline void mma_range(typename Op<KIND>::acc_t& acc, const char* lds, int kb, int ke, int ldo, float sc,
                                 const void* bh, const void* bl, int ldb, int brow, int l16, int g) {
  typedef Op<KIND> O;
  constexpr int U = Depth<KIND>::U;
  int k0 = kb;
  for (; k0 + U * O::KB <= ke; k0 += U * O::KB)
    mma_steps<KIND, BASIS_A, U>(acc, lds, ldo, sc, bh, bl, ldb, brow, l16, g, k0);
  mma_tail<KIND, BASIS_A, U - 1>(acc, lds, ldo, sc, bh, bl, ldb, brow, l16, g, k0, (ke - k0) / O::KB);
}

template <int KIND>
__device__ inline void mma_lds_by_basis_k(typename Op<KIND>::acc_t& acc, const char* lds, int kb, int ke, int ldo,
                                          float sc, const void* bh, const void* bl, int ldb, int brow, int l16, int g) {
  mma_range<KIND, false>(acc, lds, kb, ke, ldo, sc, bh, bl, ldb, brow, l16, g);
}

// the two halves [0, ks) and [ks, ke) into lo and hi, each in ascending k as mma_lds_by_basis_k
// takes it, with the basis fragments of both halves in flight together while both have full
// batches left
template <int KIND>
__device__ inline void mma_lds_by_basis_2h(typename Op<KIND>::acc_t& lo, typename Op<KIND>::acc_t& hi,
                                           const char* lds, int ks, int ke, int ldo, float sc, const void* bh,
                                           const void* bl, int ldb, int brow, int l16, int g) {
  typedef Op<KIND> O;
  constexpr int U = Depth<KIND>::U / 2;
  const int m = min(ks, ke - ks);
  int k0 = 0;
  for (; k0 + U * O::KB <= m; k0 += U * O::KB) {
    typename O::frag a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] = O::glob_frag(bh, bl, ldb, brow, k0 + u * O::KB, g);
      b[u] = O::glob_frag(bh, bl, ldb, brow, ks + k0 + u * O::KB, g);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      O::mma(lo, O::lds_frag(lds, ldo, l16, k0 + u * O::KB, g, sc), a[u]);
      O::mma(hi, O::lds_frag(lds, ldo, l16, ks + k0 + u * O::KB, g, sc), b[u]);
    }
  }
  mma_range<KIND, false>(lo, lds, k0, ks, ldo, sc, bh, bl, ldb, brow, l16, g);
  mma_range<KIND, false>(hi, lds, ks + k0, ke, ldo, sc, bh, bl, ldb, brow, l16, g);
}

template <int KIND>
__device__ inline void mma_lds_by_basis(typename Op<KIND>::acc_t& acc, const char* lds, int ke, int ldo, float sc,
                                        const void* bh, const void* bl, int ldb, int brow, int l16, int g) {
  mma_range<KIND, false>(acc, lds, 0, ke, ldo, sc, bh, bl, ldb, brow, l16, g);
}

template <int KIND>
__device__ inline void mma_basis_by_lds(typename Op<KIND>::acc_t& acc, const void* ah, const void* al, int ldb,
                                        const char* lds, int ke, int ldo, float sc, int arow, int l16, int g) {
  mma_range<KIND, true>(acc, lds, 0, ke, ldo, sc, ah, al, ldb, arow, l16, g);
}

// contraction length of an axis of n nodes: n rounded up to the k step of the products
template <int KIND>
__device__ inline int kext(int n) {
  return (n + Op<KIND>::KB - 1) / Op<KIND>::KB * Op<KIND>::KB;
}

// acc[t] += basis rows (row block wave + NW t, basis from L2) x the LDS data operand over k < ke,
// k outermost: the N row blocks of the wave advance together, each accumulator in ascending k
// (the order of mma_basis_by_lds, so the results are the same bits), the data fragment of a k step
// read once for all of them, and the basis fragments of GU k steps of all N blocks requested
// before the first product.  N: the wave's count of existing row blocks (uniform), chosen once.
template <int KIND, int NW, int RB, int N, int GU>
__device__ inline void mma_gbasis_rows_n(typename Op<KIND>::acc_t (&acc)[RB], const void* bh, const void* bl,
                                         int ldb, const char* lds, int ke, int ldo, float sc, int wave, int l16,
                                         int g) {
  typedef Op<KIND> O;
  int row[N];
#pragma unroll
  for (int t = 0; t < N; ++t) row[t] = (wave + NW * t) * 16 + l16;
  int k0 = 0;
  for (; k0 + GU * O::KB <= ke; k0 += GU * O::KB) {
    typename O::frag a[GU][N];
#pragma unroll
    for (int u = 0; u < GU; ++u)
#pragma unroll
      for (int t = 0; t < N; ++t) a[u][t] = O::glob_frag(bh, bl, ldb, row[t], k0 + u * O::KB, g);
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const typename O::frag b = O::lds_frag(lds, ldo, l16, k0 + u * O::KB, g, sc);
#pragma unroll
      for (int t = 0; t < N; ++t) O::mma(acc[t], a[u][t], b);
    }
  }
  for (; k0 < ke; k0 += O::KB) {
    typename O::frag a[N];
#pragma unroll
    for (int t = 0; t < N; ++t) a[t] = O::glob_frag(bh, bl, ldb, row[t], k0, g);
    const typename O::frag b = O::lds_frag(lds, ldo, l16, k0, g, sc);
#pragma unroll
    for (int t = 0; t < N; ++t) O::mma(acc[t], a[t], b);
  }
}

template <int KIND, int NW, int RB, int GU, int N = RB>
__device__ inline void mma_gbasis_rows(typename Op<KIND>::acc_t (&acc)[RB], const void* bh, const void* bl, int ldb,
                                       const char* lds, int ke, int ldo, float sc, int wave, int nrb, int l16,
                                       int g) {
  if constexpr (N > 0) {
    if (wave + NW * (N - 1) < nrb)
      mma_gbasis_rows_n<KIND, NW, RB, N, GU>(acc, bh, bl, ldb, lds, ke, ldo, sc, wave, l16, g);
    else
      mma_gbasis_rows<KIND, NW, RB, GU, N - 1>(acc, bh, bl, ldb, lds, ke, ldo, sc, wave, nrb, l16, g);
  }
}

// Products with a basis copy in LDS take at most 12 row (column) blocks: three per wave.
constexpr int kLdsRb = 3;

// acc[t] += basis rows (row block wave + NW t, a basis copy in LDS) x the LDS data operand, k
// outermost: the data fragment of a k step is read (and split) once for all row blocks, the basis
// fragments of all row blocks are requested before the first product, and the independent
// accumulators keep the matrix cores busy.  Only the row blocks below nrb are computed: the wave's
// count of them is uniform, so the choice is made once, outside the k loop, and each accumulator
// chain stays free of branches.  Accumulators of missing row blocks are left untouched.
template <int KIND, int NW, int RB, int N>
__device__ inline void mma_lbasis_rows_n(typename Op<KIND>::acc_t (&acc)[RB], const char* bh, const char* bl,
                                         int ldb, const char* lds, int ld, int ldo, float sc, int wave, int l16,
                                         int g) {
  typedef Op<KIND> O;
  int row[N];
#pragma unroll
  for (int t = 0; t < N; ++t) row[t] = (wave + NW * t) * 16 + l16;
  for (int k0 = 0; k0 < ld; k0 += O::KB) {
    typename O::frag a[N];
#pragma unroll
    for (int t = 0; t < N; ++t) a[t] = O::lbasis_frag(bh, bl, ldb, row[t], k0, g);
    const typename O::frag b = O::lds_frag_cvt(lds, ldo, l16, k0, g, sc);
#pragma unroll
    for (int t = 0; t < N; ++t) O::mma(acc[t], a[t], b);
  }
}

template <int KIND, int NW, int RB, int N = RB>
__device__ inline void mma_lbasis_rows(typename Op<KIND>::acc_t (&acc)[RB], const char* bh, const char* bl,
                                       int ldb, const char* lds, int ld, int ldo, float sc, int wave, int nrb,
                                       int l16, int g) {
  if constexpr (N > 0) {
    if (wave + NW * (N - 1) < nrb)  // row blocks 0 .. N - 1 of this wave exist
      mma_lbasis_rows_n<KIND, NW, RB, N>(acc, bh, bl, ldb, lds, ld, ldo, sc, wave, l16, g);
    else
      mma_lbasis_rows<KIND, NW, RB, N - 1>(acc, bh, bl, ldb, lds, ld, ldo, sc, wave, nrb, l16, g);
  }
}

// acc[t] += LDS data rows x basis rows (column block wave + NW t) of a basis copy in LDS, k
// outermost; NW waves take RB column blocks each, and only the column blocks below nrb are
// computed (chosen once per wave, as above)
template <int KIND, int NW, int RB, int N>
__device__ inline void mma_rows_lbasis_n(typename Op<KIND>::acc_t (&acc)[RB], const char* lds, int ld, int ldo,
                                         float sc, const char* bh, const char* bl, int ldb, int wave, int l16,
                                         int g) {
  typedef Op<KIND> O;
  int row[N];
#pragma unroll
  for (int t = 0; t < N; ++t) row[t] = (wave + NW * t) * 16 + l16;
  for (int k0 = 0; k0 < ld; k0 += O::KB) {
    typename O::frag b[N];
#pragma unroll
    for (int t = 0; t < N; ++t) b[t] = O::lbasis_frag(bh, bl, ldb, row[t], k0, g);
    const typename O::frag a = O::lds_frag_cvt(lds, ldo, l16, k0, g, sc);
#pragma unroll
    for (int t = 0; t < N; ++t) O::mma(acc[t], a, b[t]);
  }
}

template <int KIND, int NW, int RB, int N = RB>
__device__ inline void mma_rows_lbasis_w(typename Op<KIND>::acc_t (&acc)[RB], const char* lds, int ld, int ldo,
                                         float sc, const char* bh, const char* bl, int ldb, int wave, int nrb, int l16,
                                         int g) {
  if constexpr (N > 0) {
    if (wave + NW * (N - 1) < nrb)
      mma_rows_lbasis_n<KIND, NW, RB, N>(acc, lds, ld, ldo, sc, bh, bl, ldb, wave, l16, g);
    else
      mma_rows_lbasis_w<KIND, NW, RB, N - 1>(acc, lds, ld, ldo, sc, bh, bl, ldb, wave, nrb, l16, g);
  }
}

// Copy `bytes` (a multiple of 16) from global memory into LDS with direct-to-LDS loads, which
// need no registers and are all in flight together: wave w of nwaves copies the 1 KiB chunks w,
// w + nwaves, ..,
// lane l bytes [16 l, 16 l + 16) of a chunk.  Complete after vmem_drain() and a barrier.
__device__ inline void lds_dma(char* dst, const void* src, int bytes, int nwaves = 4) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  for (int ch = wave; ch * 1024 < bytes; ch += nwaves)
    if (ch * 1024 + lane * 16 < bytes)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)((const char*)src + ch * 1024 + lane * 16),
                                       (__attribute__((address_space(3))) void*)(dst + ch * 1024), 16, 0, 0);
}

constexpr int kMaxLd = 576;            // widest padded axis of the regular strip kernel (36 row
                                       // blocks); longer axes take strip_long_kernel
constexpr int kLongMaxLd = 1056;       // widest padded axis at all (1025 nodes)
constexpr int kColU = kMaxLd / 64;      // column loads per row and lane

// Stage rows [row0, row0 + 16) x columns [0, ld) of a row-major R x C array into LDS as the data
// operand (row stride ldo; zero beyond R and C); returns this thread's largest magnitude.  With NW
// waves, wave w takes rows w + NW j, lane l columns l + 64 u; the loads of two rows are issued
// before any is used, so a tile costs 8 / NW memory round trips rather than one per element.
template <int KIND, int NW = 4>
__device__ inline float stage_rows16(char* lds, int ld, int ldo, const gmem<typename Op<KIND>::T>* src, int row0,
                                     int R, int C) {
  typedef Op<KIND> O;
  typedef typename O::T T;
  static_assert(NW == 4 || NW == 8, "16 rows over 4 or 8 waves");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float amax = 0.f;
  // rows longer than kMaxLd (long axes) in chunks of kMaxLd columns; one chunk otherwise
  for (int cb = 0; cb < ld; cb += kMaxLd) {
#pragma unroll
    for (int jp = 0; jp < 8 / NW; ++jp) {
      T v[2][kColU];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = wave + NW * (2 * jp + j);
        const bool rok = row0 + r < R;
        const gmem<T>* rp = src + (long)(rok ? row0 + r : 0) * C;
#pragma unroll
        for (int u = 0; u < kColU; ++u) {
          const int k = cb + lane + 64 * u;
          v[j][u] = (rok && k < C) ? rp[k] : T(0);
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = wave + NW * (2 * jp + j);
#pragma unroll
        for (int u = 0; u < kColU; ++u) {
          const int k = cb + lane + 64 * u;
          if (k < ld) {
            O::put(lds, ldo, r, k, v[j][u]);
            if (O::SCALED) amax = fmaxf(amax, fabsf((float)v[j][u]));
          }
        }
      }
    }
  }
  return amax;
}

// Stage the 16-column strip [col0, col0 + 16) of a row-major K x ncol array transposed into LDS
// (operand row c = strip column, k = index along the axis, row stride ldo; zero beyond K and
// ncol); returns this thread's largest magnitude.  With NTH threads, thread t takes column t % 16
// and rows t / 16 + (NTH / 16) j; 192 rows are in flight per batch.
template <int KIND, int NTH = 256>
__device__ inline float stage_strip16(char* lds, int ld, int ldo, const gmem<typename Op<KIND>::T>* src, int K,
                                      int ncol, int col0) {
  typedef Op<KIND> O;
  typedef typename O::T T;
  constexpr int RS = NTH / 16;       // rows per pass
  constexpr int B = 192 / RS;        // loads in flight per thread per batch (192 rows per batch)
  const int c = threadIdx.x & 15, k0 = threadIdx.x >> 4;
  const bool cok = col0 + c < ncol;
  float amax = 0.f;
  for (int kb = 0; kb < ld; kb += RS * B) {
    T v[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int k = kb + k0 + RS * j;
      v[j] = (cok && k < K) ? src[(long)k * ncol + col0 + c] : T(0);
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int k = kb + k0 + RS * j;
      if (k < ld) {
        O::put(lds, ldo, c, k, v[j]);
        if (O::SCALED) amax = fmaxf(amax, fabsf((float)v[j]));
      }
    }
  }
  return amax;
}

// power-of-two scale bringing the tile's largest magnitude to [2^13, 2^14) (1 for an all-zero
// tile); every thread passes its own running maximum
__device__ inline float tile_scale(float amax, float* red) {
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
  __syncthreads();
  const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  __syncthreads();
  if (!(m > 0.f) || !isfinite(m)) return 1.f;
  int e;
  frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
  return ldexpf(1.f, 14 - e);
}

// tile_scale for a workgroup of NW waves (red holds NW floats)
template <int NW>
__device__ inline float tile_scale_w(float amax, float* red) {
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
  __syncthreads();
  float m = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) m = fmaxf(m, red[w]);
  __syncthreads();
  if (!(m > 0.f) || !isfinite(m)) return 1.f;
  int e;
  frexpf(m, &e);
  return ldexpf(1.f, 14 - e);
}

// forward transform along the last axis for 16 rows x up to 64 columns: T = F * A_last
template <int KIND>
__global__ __launch_bounds__(256) void fwd_last_kernel(const int4* __restrict__ tiles, int ntiles, StepArgs sa) {
  typedef Op<KIND> O;
  typedef typename O::T T;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int tix = xcd_tile();
  if (tix >= ntiles) return;
  const int4 tl = tiles[tix];
  const SubDev& S = sa.subs[tl.x];
  const int la = S.dim - 1;
  const int R = S.dim == 2 ? S.n[0] : S.n[0] * S.n[1];
  const int C = S.n[la];
  const AxisDev& A = S.ax[la];
  const int ld = A.ld;
  const int row0 = tl.y, col0 = tl.z;
  __shared__ float red[4];
  const gmem<T>* __restrict__ src = gp<T>(S.F);
  const int ldo = ld + O::OPAD;
  const float amax = stage_rows16<KIND>(lds, ld, ldo, src, row0, R, C);
  const float sc = O::SCALED ? tile_scale(amax, red) : 1.f;
  __syncthreads();
  if (O::SCALED) {
    O::presplit(lds, ldo, 16, ld, &sc, 16);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
  const int cb = (col0 >> 4) + wave;
  if (cb * 16 >= C) return;
  typename O::acc_t acc = {0, 0, 0, 0};
  mma_lds_by_basis<KIND>(acc, lds, kext<KIND>(C), ldo, sc, A.fwd, A.fwdl, A.ldb, cb * 16 + l16, l16, g);
  gmem<T>* __restrict__ out = gpw<T>(S.T);
  const T us = T(A.fwd_unscale) / T(sc);
  const int c = cb * 16 + l16;
  for (int q = 0; q < 4; ++q) {
    const int r = row0 + O::crow(g, q);
    if (r < R && c < C) out[(long)r * C + c] = acc[q] * us;
  }
}

// shift removed from phi each step: mean of the DC coefficient over the instance's first I.pin
// subdomains (all of them in the parallel form; the first one, which opens every sweep, in the
// alternating forms, so that every subdomain of a sweep removes the same constant).
// The coefficients are summed across a wave: lane l adds those of subdomains l, l + 64, .. in that
// order, then a butterfly adds the lanes, which leaves the same bits in every lane, wave and
// workgroup.  dc_first_load requests the first of them early (before the tile is staged), so that
// round trip overlaps the staging instead of following it.
template <typename T>
__device__ inline T dc_first_load(const StepArgs& sa, int pin, int first_sub) {
  return pin ? gp<T>(sa.dc)[first_sub + min((int)threadIdx.x & 63, pin - 1)] : T(0);
}

template <typename T>
__device__ inline T instance_shift(const StepArgs& sa, int pin, int first_sub, T d0) {
  if (!pin) return T(0);
  const int lane = threadIdx.x & 63;
  const gmem<T>* dc = gp<T>(sa.dc);
  T s = lane < pin ? d0 : T(0);
  for (int q = lane + 64; q < pin; q += 64) s += dc[first_sub + q];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  return s / T(pin);
}

// shape and artificial faces of a subdomain, copied into registers (stores to the state arrays
// could otherwise alias the descriptor and force reloads)
struct BoxReg {
  int dim, n0, n1, n2, art;
};
__device__ inline BoxReg box_of(const SubDev& S) { return BoxReg{S.dim, S.n[0], S.n[1], S.n[2], S.art}; }

// trapezoid weight (without prod h) and live flag of a node
__device__ inline void node_weight(const BoxReg& B, int i0, int i1, int i2, double& w, bool& live) {
  w = ((i0 == 0 || i0 == B.n0 - 1) ? 0.5 : 1.0) * ((i1 == 0 || i1 == B.n1 - 1) ? 0.5 : 1.0);
  live = !is_artificial(B.art, 0, i0, B.n0) && !is_artificial(B.art, 1, i1, B.n1);
  if (B.dim == 3) {
    if (i2 == 0 || i2 == B.n2 - 1) w *= 0.5;
    if (is_artificial(B.art, 2, i2, B.n2)) live = false;
  }
}

// inverse transform along the last axis for 16 rows x up to 64 columns, fused with the update
// phi += dt (delta - shift) and the residual partial sum.  Input: F.
// Push transmission: the subdomain's entries S.pfirst[t] .. S.pfirst[t + 1] of S.push, t = tile.w
// the tile's index among the subdomain's inverse-last tiles (destination node's device address as
// low and high words, row | later << 8, column within the tile), are those whose source node lies
// in the tile;
// after the update each such node's new value is written into the artificial node of the other
// subdomain, which is the owner's value the transmission condition gives it for the next step.
// In an alternating sweep a destination that is updated later in the same step has not removed
// this step's shift yet: later = 1 entries add dt * shift back, so every subdomain sees its
// neighbours' values relative to the same constant.
// The contraction is summed as two halves, lo (the first ceil(steps / 2) k steps) + hi, in every
// form, so the result does not depend on the form a launch takes.  NW = 4: wave w computes both
// halves of column block w.  NW = 8 (launches of few tiles, where a wave's chain of dependent
// basis loads is the launch's duration): waves w and w + 4 take the two halves for column block w,
// and wave w adds its partner's half through LDS before the update.
// (four waves: at least seven workgroups per compute unit, which the register budget allows, for
// the launches of many tiles that take this form)
// one tile (entry tix of the launch table) of the inverse last-axis product and update
template <int KIND, int NW>
__device__ inline void inv_last_tile(int tix, const int4* __restrict__ tiles, int part_base, const StepArgs& sa) {
  typedef Op<KIND> O;
  typedef typename O::T T;
  typedef typename O::acc_t acc_t;
  static_assert(NW == 4 || NW == 8, "four column blocks, one or two waves each");
  constexpr int KS = NW / 4;  // waves per column block
  extern __shared__ __attribute__((aligned(16))) char lds[];
  __shared__ double red[NW];
  __shared__ float redf[NW];
  __shared__ T stash[16][64];
  __shared__ acc_t xch[KS > 1 ? 4 : 1][64];
  const int4 tl = tiles[tix];
  const SubDev& S = sa.subs[tl.x];
  const InstDev& I = sa.insts[S.inst];
  const int la = S.dim - 1;
  const int R = S.dim == 2 ? S.n[0] : S.n[0] * S.n[1];
  const int C = S.n[la];
  const AxisDev& A = S.ax[la];
  const int ld = A.ld;
  const int row0 = tl.y, col0 = tl.z;
  const gmem<T>* __restrict__ src = gp<T>(S.F);
  const int ldo = ld + O::OPAD;
  // every descriptor field is read into registers before the first barrier: later reads could not
  // use the scalar cache and would wait for all earlier vector memory operations
  const T dt = T(I.dt);
  const int pin = I.pin, first_sub = I.first_sub;
  const BoxReg box = box_of(S);
  const double hs = S.h[0] * S.h[1] * (S.dim == 3 ? S.h[2] : 1.0);
  const int inst = S.inst;
  const void* invh = A.inv;
  const void* invl = A.invl;
  const int ldb = A.ldb;
  gmem<T>* __restrict__ phi = gpw<T>(S.phi);
  const int4* __restrict__ push = S.push;
  const int* __restrict__ pfirst = S.pfirst;
  const int pf0 = pfirst ? pfirst[tl.w] : 0, pf1 = pfirst ? pfirst[tl.w + 1] : 0;
  const T d0 = dc_first_load<T>(sa, pin, first_sub);
  const float amax = stage_rows16<KIND, NW>(lds, ld, ldo, src, row0, R, C);
  const float sc = O::SCALED ? tile_scale_w<NW>(amax, redf) : 1.f;
  __syncthreads();
  if (O::SCALED) {
    O::presplit(lds, ldo, 16, ld, &sc, 16);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
  const int cw = wave & 3, kh = wave >> 2;  // column block within the tile; half of the contraction
  const int cb = (col0 >> 4) + cw;
  const bool active = cb * 16 < C;
  const T isc = T(1) / T(sc);
  // first half: the first ceil(steps / 2) k steps
  const int ke = kext<KIND>(C);  // the contraction stops at the axis length (k-step granularity)
  const int ksplit = min(ke, ((ke + 2 * O::KB - 1) / (2 * O::KB)) * O::KB);
  const int c = cb * 16 + l16;
  acc_t acc = {0, 0, 0, 0};
  T old[4];
  if (active) {
    // the update's phi values are requested before the product so their latency overlaps it
    if (kh == 0) {
      for (int q = 0; q < 4; ++q) {
        const int r = row0 + O::crow(g, q);
        old[q] = (r < R && c < C) ? phi[(long)r * C + c] : T(0);
      }
    }
    if (KS > 1) {
      mma_lds_by_basis_k<KIND>(acc, lds, kh ? ksplit : 0, kh ? ke : ksplit, ldo, sc, invh, invl, ldb, c, l16, g);
    } else {
      acc_t hi = {0, 0, 0, 0};
      mma_lds_by_basis_2h<KIND>(acc, hi, lds, ksplit, ke, ldo, sc, invh, invl, ldb, c, l16, g);
      for (int q = 0; q < 4; ++q) acc[q] += hi[q];
    }
  }
  const T shift = instance_shift<T>(sa, pin, first_sub, d0);
  if (KS > 1) {
    if (kh == 1 && active) xch[cw][lane] = acc;
    __syncthreads();
  }
  double part = 0.0;
  if (kh == 0 && active) {
    if (KS > 1) {
      const acc_t o = xch[cw][lane];
      for (int q = 0; q < 4; ++q) acc[q] += o[q];
    }
    bool bad = false;
    for (int q = 0; q < 4; ++q) {
      const int r = row0 + O::crow(g, q);
      if (r < R && c < C) {
        int i0, i1, i2;
        if (box.dim == 2) {
          i0 = r; i1 = c; i2 = 0;
        } else {
          i0 = r / box.n1; i1 = r - i0 * box.n1; i2 = c;
        }
        double w;
        bool live;
        node_weight(box, i0, i1, i2, w, live);
        if (live) {
          const T val = acc[q] * isc;
          const T u = dt * val;
          const T nv = old[q] + dt * (val - shift);
          phi[(long)r * C + c] = nv;
          if (pf1 > pf0) stash[O::crow(g, q)][cw * 16 + l16] = nv;
          part += w * (double)u * (double)u;
          bad |= !finite_(u);
        }
      }
    }
    if (bad) atomicOr(&sa.status[inst], ST_NONFINITE);
  }
  if (pf1 > pf0) {
    __syncthreads();
    for (int e = pf0 + (int)threadIdx.x; e < pf1; e += 64 * NW) {
      const int4 P = push[e];
      T v = stash[P.z & 0xFF][P.w];
      if (P.z >> 8) v += dt * shift;
      const unsigned long long a = ((unsigned long long)(unsigned)P.y << 32) | (unsigned)P.x;
      *gpw<T>((void*)(uintptr_t)a) = v;
    }
  }
  const double tot = block_sum_w<NW>(part, red);
  if (threadIdx.x == 0) {
    sa.partials[part_base + tix] = tot * hs;
    if (pin && tl.x == first_sub && row0 == 0 && col0 == 0) sa.shift_acc[inst] += (double)dt * (double)shift;
  }
}

template <int KIND, int NW>
__global__ __launch_bounds__(64 * NW, NW == 4 ? 7 : 1) void inv_last_kernel(const int4* __restrict__ tiles, int ntiles,
                                                                           int part_base, StepArgs sa) {
  const int tix = xcd_tile();
  if (tix >= ntiles) return;
  inv_last_tile<KIND, NW>(tix, tiles, part_base, sa);
}

// Spectral factors of axes 1 and 2 for column c of the [n0][rest] view of a pair product: the
// axis-1 factor, the axis-2 factor (3D) and their weights gamma_1 h_1^-2, gamma_2 h_2^-2.  Loaded
// without a branch (c clamped into range; a 2D view reads axis 1 twice and weights the second by 0)
// so the loads stay in flight with the rest of the prologue; value() combines them in one fixed
// rounding order, shared by every kernel that applies the spectral scale.
template <typename T>
struct RestSig {
  T r1, r2, g1, g2;
  __device__ inline T value() const { return fma(g1, r1, g2 * r2); }
};

template <typename T>
__device__ inline RestSig<T> rest_sig(const SubDev& S, int c, int ncol) {
  const bool three = S.dim == 3;
  const gmem<T>* s1 = gp<T>(S.ax[1].sig);
  const gmem<T>* s2 = three ? gp<T>(S.ax[2].sig) : s1;
  const int cc = min(c, ncol - 1);
  const int n2 = three ? S.n[2] : 1;
  const int k1 = three ? cc / n2 : cc, k2 = three ? cc - k1 * n2 : 0;
  RestSig<T> r;
  r.r1 = s1[k1];
  r.r2 = s2[k2];
  r.g1 = T(S.gh2[1]);
  r.g2 = three ? T(S.gh2[2]) : T(0);
  return r;
}

// NW waves per workgroup: latency-bound launches (one workgroup per compute unit or fewer) take 8,
// so each wave's chain of row blocks, which is the launch's duration, is halved; launches of many
// strips take 4, which keeps more workgroups resident per compute unit.

// 16-column strip of the [n_axis][rest] view (axis 0), or of one [n1][n2] slab (axis 1, 3D;
// tile.y = slab index i0).  src / dst: 0 = F, 1 = T.
//   PAIR = false: dst = Bas * src, Bas the forward (inv = 0) or inverse (inv = 1) basis
//   PAIR = true (axis 0): dst = B_0 * (S o (A_0 * src)), S the spectral scale
//                         1 / (1 + sum_k gamma mu_k); the DC coefficient is recorded
// When the strip and the basis fit in the launch's LDS (lcap bytes), the basis is copied into LDS
// once (direct-to-LDS loads, in flight together with the strip) and every product reads LDS only.
// The pair reuses the forward matrix for the inverse, on both paths: with D = diag(w) (w = 1/2 at
// both ends, else 1) the DCT-I matrices satisfy B = (N / 2) D^-1 A D^-1, and the powers of two D^-1
// and N / 2 fold exactly into the spectral scale and the store.  The LDS path needs only A in LDS;
// the global path doing the same keeps the two bitwise equal, so a request's result does not
// depend on which path its launch takes.
// one 16-column strip (entry tix of the launch table)
template <int KIND, bool PAIR, int NW, int RBW = (36 + NW - 1) / NW>
__device__ inline void strip_tile(int tix, const int4* __restrict__ tiles, int axis, int inv, int src_sel, int lcap,
                                  const StepArgs& sa) {
  typedef Op<KIND> O;
  typedef typename O::T T;
  constexpr int MAXRB = RBW;                       // row blocks per wave: n <= 16 NW RBW (576 by default)
  constexpr int RBL = (4 * kLdsRb + NW - 1) / NW;  // the same with the basis in LDS (n <= 192)
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int4 tl = tiles[tix];
  const SubDev& S = sa.subs[tl.x];
  const int K = S.n[axis];
  const AxisDev& A = S.ax[axis];
  const int ld = A.ld;
  int ncol;
  long base;
  if (axis == 0) {
    ncol = S.dim == 2 ? S.n[1] : S.n[1] * S.n[2];
    base = 0;
  } else {
    ncol = S.n[2];
    base = (long)tl.y * S.n[1] * S.n[2];
  }
  const int col0 = tl.z;
  const gmem<T>* __restrict__ src = gp<T>(src_sel ? S.T : S.F) + base;
  gmem<T>* __restrict__ dst = gpw<T>(src_sel ? S.F : S.T) + base;
  __shared__ float red[NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
  const int uwave = __builtin_amdgcn_readfirstlane(wave);  // the same, known uniform
  const int nrb = (K + 15) >> 4;
  const int c = col0 + l16;
  const void* b1h = (PAIR || !inv) ? A.fwd : A.inv;
  const void* b1l = (PAIR || !inv) ? A.fwdl : A.invl;
  // basis copy in LDS after the strip: nrb * 16 rows of stride ldb (split form: hi, then lo)
  const int ldo = ld + O::OPAD, ldb = A.ldb;
  const int dbytes = 16 * ldo * O::LDS_BYTES;
  const int bbytes = nrb * 16 * ldb * (O::BASIS_BYTES / (O::SCALED ? 2 : 1));
  const bool lbasis = nrb <= 4 * kLdsRb && dbytes + (O::SCALED ? 2 : 1) * bbytes <= lcap;
  static_assert(RBL <= MAXRB, "LDS-basis row blocks fit the accumulators");
  char* lbh = lds + dbytes;
  char* lbl = lbh + bbytes;
  // PAIR: the factors of axes 1 and 2 of this lane's column, requested before the products; the
  // axis-0 factors are read when the scale is applied (held through the products they would take
  // 4 MAXRB registers per lane, in FP64 the difference between one and two workgroups per compute
  // unit for the eight-wave form)
  RestSig<T> rs{T(0), T(0), T(0), T(0)};
  const gmem<T>* s0 = gp<T>(S.ax[0].sig);
  if constexpr (PAIR) rs = rest_sig<T>(S, c, ncol);
  // every descriptor field is read before the basis copy is issued: loads after it would be
  // vector loads (the copy may write memory, as far as the compiler knows), and each of their
  // waits would also wait for the copy
  const T fwd_unscale = T(A.fwd_unscale);
  const T g0 = T(S.gh2[0]);
  if (lbasis) {
    lds_dma(lbh, b1h, bbytes, NW);
    if (O::SCALED) lds_dma(lbl, b1l, bbytes, NW);
  }
  // strip transposed into LDS: operand row c = strip column, k = index along the axis
  const float amax = stage_strip16<KIND, 64 * NW>(lds, ld, ldo, src, K, ncol, col0);
  const float sc = O::SCALED ? tile_scale_w<NW>(amax, red) : 1.f;
  if (lbasis) vmem_drain();
  __syncthreads();
  if (O::SCALED && !lbasis) {  // the LDS-basis products split each fragment on the fly
    O::presplit(lds, ldo, 16, ld, &sc, 16);
    __syncthreads();
  }
  typename O::acc_t acc[MAXRB];
  const T us1 = ((PAIR || !inv) ? fwd_unscale : T(1)) / T(sc);
#pragma unroll
  for (int t = 0; t < MAXRB; ++t) acc[t] = typename O::acc_t{0, 0, 0, 0};
  if (lbasis) {
    typename O::acc_t a3[RBL];
#pragma unroll
    for (int t = 0; t < RBL; ++t) a3[t] = typename O::acc_t{0, 0, 0, 0};
    mma_lbasis_rows<KIND, NW, RBL>(a3, lbh, lbl, ldb, lds, ld, ldo, sc, uwave, nrb, l16, g);
#pragma unroll
    for (int t = 0; t < RBL; ++t) acc[t] = a3[t];
  } else if constexpr (KIND == PREC_F64 && MAXRB <= 3) {  // FP64, three row blocks per wave: k outermost
    mma_gbasis_rows<KIND, NW, MAXRB, 2>(acc, b1h, b1l, ldb, lds, kext<KIND>(K), ldo, sc, uwave, nrb, l16, g);
  } else {
#pragma unroll
    for (int t = 0; t < MAXRB; ++t) {
      const int rb = wave + NW * t;
      if (rb < nrb) mma_basis_by_lds<KIND>(acc[t], b1h, b1l, ldb, lds, kext<KIND>(K), ldo, sc, rb * 16 + l16, l16, g);
    }
  }
  if constexpr (!PAIR) {
#pragma unroll
    for (int t = 0; t < MAXRB; ++t) {
      const int rb = wave + NW * t;
      if (rb >= nrb) continue;
      for (int q = 0; q < 4; ++q) {
        const int i = rb * 16 + O::crow(g, q);
        if (i < K && c < ncol) dst[(long)i * ncol + c] = acc[t][q] * us1;
      }
    }
  } else {
    // spectral scale; coefficient index (k0, k1[, k2]) = (i, c) with c split over axes 1, 2,
    // and D^-1 (x 2 at i = 0 and i = K - 1) ahead of the forward matrix reused.  The axis-0
    // factors are loaded unconditionally (clamped indices; out-of-range values discarded), all in
    // flight together: a load under a branch would wait for every earlier load.
    const T rest = rs.value();
    T sig0[MAXRB * 4];
#pragma unroll
    for (int t = 0; t < MAXRB; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) sig0[t * 4 + q] = s0[min((wave + NW * t) * 16 + O::crow(g, q), K - 1)];
#pragma unroll
    for (int t = 0; t < MAXRB; ++t) {
      const int rb = wave + NW * t;
      for (int q = 0; q < 4; ++q) {
        const int i = rb * 16 + O::crow(g, q);
        T y = T(0);
        if (rb < nrb && i < K && c < ncol) {
          const T val = acc[t][q] * us1;
          if (i == 0 && c == 0) gpw<T>(sa.dc)[tl.x] = val;
          y = val / (T(1) + g0 * sig0[t * 4 + q] + rest);
          if (i == 0 || i == K - 1) y *= T(2);
        }
        acc[t][q] = y;
      }
    }
    __syncthreads();  // every wave is done reading the strip
    float ymax = 0.f;
#pragma unroll
    for (int t = 0; t < MAXRB; ++t) {
      const int rb = wave + NW * t;
      if (rb >= nrb) continue;
      for (int q = 0; q < 4; ++q) {
        O::put(lds, ldo, l16, rb * 16 + O::crow(g, q), acc[t][q]);
        if (O::SCALED) ymax = fmaxf(ymax, fabsf((float)acc[t][q]));
      }
    }
    const float sy = O::SCALED ? tile_scale_w<NW>(ymax, red) : 1.f;
    // zero the padding rows nrb*16 .. ld of the operand
    for (int idx = threadIdx.x; idx < 16 * (ld - nrb * 16); idx += 64 * NW) {
      const int k = nrb * 16 + idx / 16, cc = idx & 15;
      O::put(lds, ldo, cc, k, T(0));
    }
    __syncthreads();
    if (O::SCALED && !lbasis) {
      O::presplit(lds, ldo, 16, ld, &sy, 16);
      __syncthreads();
    }
    // store scale: (N / 2) D^-1, the split form's 2^-s and 1 / sy
    const T half_n = T(K - 1) / T(2);
    const T os = fwd_unscale * half_n / T(sy);
#pragma unroll
    for (int t = 0; t < MAXRB; ++t) acc[t] = typename O::acc_t{0, 0, 0, 0};
    if (lbasis) {
      typename O::acc_t a3[RBL];
#pragma unroll
      for (int t = 0; t < RBL; ++t) a3[t] = typename O::acc_t{0, 0, 0, 0};
      mma_lbasis_rows<KIND, NW, RBL>(a3, lbh, lbl, ldb, lds, ld, ldo, sy, uwave, nrb, l16, g);
#pragma unroll
      for (int t = 0; t < RBL; ++t) acc[t] = a3[t];
    } else if constexpr (KIND == PREC_F64 && MAXRB <= 3) {
      mma_gbasis_rows<KIND, NW, MAXRB, 2>(acc, b1h, b1l, ldb, lds, kext<KIND>(K), ldo, sy, uwave, nrb, l16, g);
    } else {
#pragma unroll
      for (int t = 0; t < MAXRB; ++t) {
        const int rb = wave + NW * t;
        if (rb < nrb)
          mma_basis_by_lds<KIND>(acc[t], b1h, b1l, ldb, lds, kext<KIND>(K), ldo, sy, rb * 16 + l16, l16, g);
      }
    }
#pragma unroll
    for (int t = 0; t < MAXRB; ++t) {
      const int rb = wave + NW * t;
      if (rb >= nrb) continue;
      for (int q = 0; q < 4; ++q) {
        const int i = rb * 16 + O::crow(g, q);
        if (i < K && c < ncol) dst[(long)i * ncol + c] = acc[t][q] * ((i == 0 || i == K - 1) ? T(2) * os : os);
      }
    }
  }
}

// RBW: row blocks per wave; launches whose axes are at most 16 NW RBW long take a form with fewer
// accumulators (eight waves, RBW = 3: axes up to 384, fewer registers per wave, more workgroups
// per compute unit)
template <int KIND, bool PAIR, int NW, int RBW = (36 + NW - 1) / NW>
__global__ __launch_bounds__(64 * NW) void strip_kernel(const int4* __restrict__ tiles, int ntiles, int axis, int inv,
                                                        int src_sel, int lcap, StepArgs sa) {
  const int tix = xcd_tile();
  if (tix >= ntiles) return;
  strip_tile<KIND, PAIR, NW, RBW>(tix, tiles, axis, inv, src_sel, lcap, sa);
}

// ------------------------------------------------------------------------------------------
// Long axes (padded length above kMaxLd, up to kLongMaxLd): the same 16-column strip products as
// strip_kernel (global-basis path, four waves), with the output rows taken in groups of 36 row
// blocks so the accumulators stay in registers.  PAIR: the spectral coefficients of every group
// are scaled and written to the destination array, then, once all of them are there, read back
// (agent-scope loads, which do not hit stale first-level cache lines) into LDS as the operand of
// the inverse product, whose groups overwrite them.  Each workgroup reads and writes only its own
// 16 columns of the destination.  Same formulas and accumulation order per output as
// strip_kernel's global-basis path.
// ------------------------------------------------------------------------------------------

template <typename T>
__device__ inline T load_agent(const gmem<T>* p) {
  return __hip_atomic_load((T*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int KIND, bool PAIR>
__global__ __launch_bounds__(256) void strip_long_kernel(const int4* __restrict__ tiles, int ntiles, int axis,
                                                         int inv, int src_sel, StepArgs sa) {
  typedef Op<KIND> O;
  typedef typename O::T T;
  constexpr int NW = 4, GRB = 9;            // row blocks per wave per group; a group is 36 blocks
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int tix = xcd_tile();
  if (tix >= ntiles) return;
  const int4 tl = tiles[tix];
  const SubDev& S = sa.subs[tl.x];
  const int K = S.n[axis];
  const AxisDev& A = S.ax[axis];
  const int ld = A.ld, ldb = A.ldb, ldo = ld + O::OPAD;
  int ncol;
  long base;
  if (axis == 0) {
    ncol = S.dim == 2 ? S.n[1] : S.n[1] * S.n[2];
    base = 0;
  } else {
    ncol = S.n[2];
    base = (long)tl.y * S.n[1] * S.n[2];
  }
  const int col0 = tl.z;
  const gmem<T>* __restrict__ src = gp<T>(src_sel ? S.T : S.F) + base;
  gmem<T>* __restrict__ dst = gpw<T>(src_sel ? S.F : S.T) + base;
  __shared__ float red[NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
  const int nrb = (K + 15) >> 4;
  const int c = col0 + l16;
  const int ke = kext<KIND>(K);
  const void* b1h = (PAIR || !inv) ? A.fwd : A.inv;
  const void* b1l = (PAIR || !inv) ? A.fwdl : A.invl;
  const T fwd_unscale = T(A.fwd_unscale);
  const T g0 = T(S.gh2[0]);
  const gmem<T>* s0 = gp<T>(S.ax[0].sig);
  RestSig<T> rs{T(0), T(0), T(0), T(0)};
  if constexpr (PAIR) rs = rest_sig<T>(S, c, ncol);
  const float amax = stage_strip16<KIND, 64 * NW>(lds, ld, ldo, src, K, ncol, col0);
  const float sc = O::SCALED ? tile_scale_w<NW>(amax, red) : 1.f;
  __syncthreads();
  if (O::SCALED) {
    O::presplit(lds, ldo, 16, ld, &sc, 16);
    __syncthreads();
  }
  const T us1 = ((PAIR || !inv) ? fwd_unscale : T(1)) / T(sc);
  for (int rg = 0; rg < nrb; rg += NW * GRB) {
    typename O::acc_t acc[GRB];
#pragma unroll
    for (int t = 0; t < GRB; ++t) {
      acc[t] = typename O::acc_t{0, 0, 0, 0};
      const int rb = rg + wave + NW * t;
      if (rb < nrb) mma_basis_by_lds<KIND>(acc[t], b1h, b1l, ldb, lds, ke, ldo, sc, rb * 16 + l16, l16, g);
    }
#pragma unroll
    for (int t = 0; t < GRB; ++t) {
      const int rb = rg + wave + NW * t;
      if (rb >= nrb) continue;
      for (int q = 0; q < 4; ++q) {
        const int i = rb * 16 + O::crow(g, q);
        if (i >= K || c >= ncol) continue;
        const T val = acc[t][q] * us1;
        if constexpr (!PAIR) {
          dst[(long)i * ncol + c] = val;
        } else {
          // spectral scale with D^-1 ahead of the forward matrix reused for the inverse
          if (i == 0 && c == 0) gpw<T>(sa.dc)[tl.x] = val;
          T y = val / (T(1) + g0 * T(s0[i]) + rs.value());
          if (i == 0 || i == K - 1) y *= T(2);
          dst[(long)i * ncol + c] = y;
        }
      }
    }
  }
  if constexpr (PAIR) {
    __threadfence();   // the coefficients are in L2 before any wave reads them back
    __syncthreads();   // and every wave is done reading the strip
    float ymax = 0.f;
    {
      const int cc = threadIdx.x & 15, k0 = threadIdx.x >> 4;
      const bool cok = col0 + cc < ncol;
      for (int k = k0; k < ld; k += 16) {
        const T y = (cok && k < K) ? load_agent(dst + (long)k * ncol + col0 + cc) : T(0);
        O::put(lds, ldo, cc, k, y);
        if (O::SCALED) ymax = fmaxf(ymax, fabsf((float)y));
      }
    }
    const float sy = O::SCALED ? tile_scale_w<NW>(ymax, red) : 1.f;
    __syncthreads();
    if (O::SCALED) {
      O::presplit(lds, ldo, 16, ld, &sy, 16);
      __syncthreads();
    }
    // store scale: (N / 2) D^-1, the split form's 2^-s and 1 / sy
    const T os = fwd_unscale * (T(K - 1) / T(2)) / T(sy);
    for (int rg = 0; rg < nrb; rg += NW * GRB) {
      typename O::acc_t acc[GRB];
#pragma unroll
      for (int t = 0; t < GRB; ++t) {
        acc[t] = typename O::acc_t{0, 0, 0, 0};
        const int rb = rg + wave + NW * t;
        if (rb < nrb) mma_basis_by_lds<KIND>(acc[t], A.fwd, A.fwdl, ldb, lds, ke, ldo, sy, rb * 16 + l16, l16, g);
      }
#pragma unroll
      for (int t = 0; t < GRB; ++t) {
        const int rb = rg + wave + NW * t;
        if (rb >= nrb) continue;
        for (int q = 0; q < 4; ++q) {
          const int i = rb * 16 + O::crow(g, q);
          if (i < K && c < ncol) dst[(long)i * ncol + c] = acc[t][q] * ((i == 0 || i == K - 1) ? T(2) * os : os);
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Wide strips for large batches: four 16-column blocks [col0, col0 + 64) per workgroup.  With
// thousands of strips the DCT matrices, read whole by every workgroup, dominate the traffic; here
// each basis fragment is fetched once and multiplied into all four blocks.  Every column block
// keeps its own block scale and its own accumulation order, so each output equals the 16-column
// kernel's (global-basis path) bit for bit.  Padded axis length at most kWideMaxLd.
// ------------------------------------------------------------------------------------------

constexpr int kWideMaxLd = 320;
constexpr int kWideNc = 4;                          // 16-column blocks per workgroup
constexpr int kWideRb = (kWideMaxLd / 16 + 3) / 4;  // row blocks per wave

// per-column-block power-of-two scales (as tile_scale, one per 16 columns): lane l of every wave
// holds column block l / 16's running maximum
__device__ inline void tile_scale4(float amax, float* red, float* out) {
  for (int o = 8; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if ((lane & 15) == 0) red[wave * 4 + (lane >> 4)] = amax;
  __syncthreads();
#pragma unroll
  for (int cb = 0; cb < kWideNc; ++cb) {
    const float m = fmaxf(fmaxf(red[cb], red[4 + cb]), fmaxf(red[8 + cb], red[12 + cb]));
    float sc = 1.f;
    if (m > 0.f && isfinite(m)) {
      int e;
      frexpf(m, &e);
      sc = ldexpf(1.f, 14 - e);
    }
    out[cb] = sc;
  }
  __syncthreads();
}

// N k steps from k0 of one row block against NC column blocks: N basis fragments requested
// first, each multiplied into every block
template <int KIND, int NC, int N>
__device__ inline void wide_steps(typename Op<KIND>::acc_t (&acc)[NC], const char* lds, int ldo, const float* scl,
                                  const void* bh, const void* bl, int ldb, int arow, int l16, int g, int k0) {
  typedef Op<KIND> O;
  typename O::frag a[N];
#pragma unroll
  for (int u = 0; u < N; ++u) a[u] = O::glob_frag(bh, bl, ldb, arow, k0 + u * O::KB, g);
#pragma unroll
  for (int u = 0; u < N; ++u)
#pragma unroll
    for (int cb = 0; cb < NC; ++cb)
      O::mma(acc[cb], a[u], O::lds_frag(lds, ldo, cb * 16 + l16, k0 + u * O::KB, g, scl[cb]));
}

template <int KIND, int NC, int R>
__device__ inline void wide_tail(typename Op<KIND>::acc_t (&acc)[NC], const char* lds, int ldo, const float* scl,
                                 const void* bh, const void* bl, int ldb, int arow, int l16, int g, int k0, int rem) {
  if constexpr (R > 0) {
    if (rem == R) wide_steps<KIND, NC, R>(acc, lds, ldo, scl, bh, bl, ldb, arow, l16, g, k0);
    else wide_tail<KIND, NC, R - 1>(acc, lds, ldo, scl, bh, bl, ldb, arow, l16, g, k0, rem);
  }
}

template <int KIND, bool PAIR>
__global__ __launch_bounds__(256) void strip4_kernel(const int4* __restrict__ tiles, int ntiles, int axis, int inv,
                                                     int src_sel, StepArgs sa) {
  typedef Op<KIND> O;
  typedef typename O::T T;
  constexpr int NC = kWideNc, MAXRB = kWideRb;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  __shared__ float red[16];
  const int tix = xcd_tile();
  if (tix >= ntiles) return;
  const int4 tl = tiles[tix];
  const SubDev& S = sa.subs[tl.x];
  const int K = S.n[axis];
  const AxisDev& A = S.ax[axis];
  const int ld = A.ld, ldb = A.ldb, ldo = ld + O::OPAD;
  int ncol;
  long base;
  if (axis == 0) {
    ncol = S.dim == 2 ? S.n[1] : S.n[1] * S.n[2];
    base = 0;
  } else {
    ncol = S.n[2];
    base = (long)tl.y * S.n[1] * S.n[2];
  }
  const int col0 = tl.z;
  const gmem<T>* __restrict__ src = gp<T>(src_sel ? S.T : S.F) + base;
  gmem<T>* __restrict__ dst = gpw<T>(src_sel ? S.F : S.T) + base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
  const int nrb = (K + 15) >> 4;
  const void* b1h = (PAIR || !inv) ? A.fwd : A.inv;
  const void* b1l = (PAIR || !inv) ? A.fwdl : A.invl;
  // PAIR: spectral factors, requested before the products
  T sig0[PAIR ? MAXRB * 4 : 1];
  RestSig<T> rs[NC];
#pragma unroll
  for (int cb = 0; cb < NC; ++cb) rs[cb] = RestSig<T>{T(0), T(0), T(0), T(0)};
  if constexpr (PAIR) {
    const gmem<T>* s0 = gp<T>(S.ax[0].sig);
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) rs[cb] = rest_sig<T>(S, col0 + cb * 16 + l16, ncol);
    // unconditional loads (clamped indices): see the 16-column kernel
    T raw[MAXRB * 4];
#pragma unroll
    for (int t = 0; t < MAXRB; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) raw[t * 4 + q] = s0[min((wave + 4 * t) * 16 + O::crow(g, q), K - 1)];
#pragma unroll
    for (int t = 0; t < MAXRB; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        sig0[t * 4 + q] = (wave + 4 * t) * 16 + O::crow(g, q) < K ? raw[t * 4 + q] : T(0);
  }
  // stage the 64 columns transposed (operand row = column within the tile); thread t takes column
  // t % 64 and rows t / 64 + 4 j, twelve loads in flight per batch
  float amax = 0.f;
  {
    constexpr int B = 12;
    const int c = threadIdx.x & 63, k0 = threadIdx.x >> 6;
    const bool cok = col0 + c < ncol;
    for (int kb = 0; kb < ld; kb += 4 * B) {
      T v[B];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int k = kb + k0 + 4 * j;
        v[j] = (cok && k < K) ? src[(long)k * ncol + col0 + c] : T(0);
      }
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int k = kb + k0 + 4 * j;
        if (k < ld) {
          O::put(lds, ldo, c, k, v[j]);
          if (O::SCALED) amax = fmaxf(amax, fabsf((float)v[j]));
        }
      }
    }
  }
  float sc[NC];
  if (O::SCALED) tile_scale4(amax, red, sc);
  else {
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) sc[cb] = 1.f;
  }
  __syncthreads();
  if (O::SCALED) {
    O::presplit(lds, ldo, 64, ld, sc, 16);
    __syncthreads();
  }
  typename O::acc_t acc[MAXRB][NC];
#pragma unroll
  for (int t = 0; t < MAXRB; ++t)
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) acc[t][cb] = typename O::acc_t{0, 0, 0, 0};
  // acc[t][cb] += basis rows of row block wave + 4 t x column block cb over k < kext(K); each
  // basis fragment is loaded once (four k steps ahead) and used for the four blocks
  const int ke = kext<KIND>(K);
  auto products = [&](const void* bh, const void* bl, const float* scl) {
#pragma unroll
    for (int t = 0; t < MAXRB; ++t) {
      const int rb = wave + 4 * t;
      if (rb >= nrb) continue;
      const int arow = rb * 16 + l16;
      constexpr int U = 4;
      int k0 = 0;
      for (; k0 + U * O::KB <= ke; k0 += U * O::KB)
        wide_steps<KIND, NC, U>(acc[t], lds, ldo, scl, bh, bl, ldb, arow, l16, g, k0);
      wide_tail<KIND, NC, U - 1>(acc[t], lds, ldo, scl, bh, bl, ldb, arow, l16, g, k0, (ke - k0) / O::KB);
    }
  };

  products(b1h, b1l, sc);
  if constexpr (!PAIR) {
    const T fu = (!inv) ? T(A.fwd_unscale) : T(1);
#pragma unroll
    for (int t = 0; t < MAXRB; ++t) {
      const int rb = wave + 4 * t;
      if (rb >= nrb) continue;
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) {
        const int c = col0 + cb * 16 + l16;
        const T us = fu / T(sc[cb]);
        for (int q = 0; q < 4; ++q) {
          const int i = rb * 16 + O::crow(g, q);
          if (i < K && c < ncol) dst[(long)i * ncol + c] = acc[t][cb][q] * us;
        }
      }
    }
  } else {
    const T g0 = T(S.gh2[0]);
    T rest[NC];
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) rest[cb] = rs[cb].value();
    float ym[NC];  // largest |y| this lane holds in each column block
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) ym[cb] = 0.f;
#pragma unroll
    for (int t = 0; t < MAXRB; ++t) {
      const int rb = wave + 4 * t;
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) {
        const int c = col0 + cb * 16 + l16;
        const T us1 = T(A.fwd_unscale) / T(sc[cb]);
        for (int q = 0; q < 4; ++q) {
          const int i = rb * 16 + O::crow(g, q);
          T y = T(0);
          if (rb < nrb && i < K && c < ncol) {
            const T val = acc[t][cb][q] * us1;
            if (i == 0 && c == 0) gpw<T>(sa.dc)[tl.x] = val;
            y = val / (T(1) + g0 * sig0[t * 4 + q] + rest[cb]);
            if (i == 0 || i == K - 1) y *= T(2);
          }
          acc[t][cb][q] = y;
          if (O::SCALED) ym[cb] = fmaxf(ym[cb], fabsf((float)y));
        }
      }
    }
    __syncthreads();  // every wave is done reading the staged columns
#pragma unroll
    for (int t = 0; t < MAXRB; ++t) {
      const int rb = wave + 4 * t;
      if (rb >= nrb) continue;
#pragma unroll
      for (int cb = 0; cb < NC; ++cb)
        for (int q = 0; q < 4; ++q) O::put(lds, ldo, cb * 16 + l16, rb * 16 + O::crow(g, q), acc[t][cb][q]);
    }
    // zero the padding rows nrb*16 .. ld of the operand
    for (int idx = threadIdx.x; idx < 64 * (ld - nrb * 16); idx += 256) {
      const int k = nrb * 16 + idx / 64, cc = idx & 63;
      O::put(lds, ldo, cc, k, T(0));
    }
    float sy[NC];
    if (O::SCALED) {
      // block maxima: lane l's values all belong to column block (its own) cb for each cb slot;
      // reduce each slot over the 16 lanes of a column group, then over waves and lane groups
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) {
        float m = ym[cb];
        for (int o = 8; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));  // over l16
        m = fmaxf(m, __shfl_xor(m, 16, 64));                                   // over g
        m = fmaxf(m, __shfl_xor(m, 32, 64));
        ym[cb] = m;
      }
      if (lane == 0) {
#pragma unroll
        for (int cb = 0; cb < NC; ++cb) red[wave * 4 + cb] = ym[cb];
      }
      __syncthreads();
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) {
        const float m = fmaxf(fmaxf(red[cb], red[4 + cb]), fmaxf(red[8 + cb], red[12 + cb]));
        float v = 1.f;
        if (m > 0.f && isfinite(m)) {
          int e;
          frexpf(m, &e);
          v = ldexpf(1.f, 14 - e);
        }
        sy[cb] = v;
      }
    } else {
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) sy[cb] = 1.f;
    }
    __syncthreads();
    if (O::SCALED) {
      O::presplit(lds, ldo, 64, ld, sy, 16);
      __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < MAXRB; ++t)
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) acc[t][cb] = typename O::acc_t{0, 0, 0, 0};
    products(A.fwd, A.fwdl, sy);  // the inverse from the forward matrix, as the 16-column kernel
    const T fwd_unscale = T(A.fwd_unscale), half_n = T(K - 1) / T(2);
#pragma unroll
    for (int t = 0; t < MAXRB; ++t) {
      const int rb = wave + 4 * t;
      if (rb >= nrb) continue;
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) {
        const int c = col0 + cb * 16 + l16;
        const T os = fwd_unscale * half_n / T(sy[cb]);
        for (int q = 0; q < 4; ++q) {
          const int i = rb * 16 + O::crow(g, q);
          if (i < K && c < ncol) dst[(long)i * ncol + c] = acc[t][cb][q] * ((i == 0 || i == K - 1) ? T(2) * os : os);
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Stencil fused with the forward product along the last axis (2D): a workgroup takes 16 full
// rows [row0, row0 + 16) of a subdomain, computes F there straight into the LDS operand of the
// mode product, and writes T[rows, :] = F[rows, :] * A_1.  F never goes through HBM, and a step
// saves a launch.  The axis-1 basis is copied into LDS alongside the halo when it fits (lcap).
// ------------------------------------------------------------------------------------------

constexpr int kFuseMaxLd = 320;           // widest last axis (padded) the fused kernel takes
constexpr int kFuseU = kFuseMaxLd / 64;   // column groups per lane
// Eight waves per workgroup: at the sizes where this kernel is latency-bound (one workgroup per
// compute unit) two waves per SIMD hide each other's LDS and transcendental latencies in the
// stencil, and the product's column blocks spread over twice as many waves.
constexpr int kFuseWaves = 8;
constexpr int kFuseRb = (4 * kLdsRb + kFuseWaves - 1) / kFuseWaves;  // LDS-basis column blocks per wave

// LDS layout of the fused kernel: operand [16][ld + OPAD] | halo [18][ld + 4] (rounded to 1 KiB)
// | basis copy (rows of stride ldb)
template <int KIND>
__host__ __device__ inline int fused_halo_bytes(int ld) {
  return ((18 * (ld + 4) * (int)sizeof(typename Op<KIND>::T) + 1023) / 1024) * 1024;
}

// (multiplies and adds fused as in the stencil kernels: see the note above the monitor code)
#pragma clang fp contract(on)
template <int KIND, int MK>
__device__ inline void fused_nodes2(const StencilCtx<typename Op<KIND>::T>& K,
                                    const MonReg<typename Op<KIND>::T, MK>& M, const typename Op<KIND>::T* halo,
                                    int HS, char* op, int ld, int ldo, int row0,
                                    NodeCheck<typename Op<KIND>::T>& chk, float& amax) {
  typedef Op<KIND> O;
  typedef typename O::T T;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n0 = K.n0, n1 = K.n1;
  const T h0 = K.h0, h1 = K.h1;
  const T r2h0 = T(1) / (T(2) * h0), r2h1 = T(1) / (T(2) * h1);
  const T rh00 = T(1) / (h0 * h0), rh11 = T(1) / (h1 * h1), r4h01 = T(1) / (T(4) * h0 * h1);
#pragma unroll
  for (int k = 0; k < 16 / kFuseWaves; ++k) {
    const int rr = wave + kFuseWaves * k, i = row0 + rr;
    const bool rlive = i < n0 && !is_artificial(K.art, 0, i, n0);
    const T x0b = fma(T(K.off0 + i), h0, K.a0);
#pragma unroll
    for (int u = 0; u < kFuseU; ++u) {
      const int j = lane + 64 * u;
      if (j >= ld) continue;
      T f = T(0);
      if (rlive && j < n1 && !is_artificial(K.art, 1, j, n1)) {
        const T* c = halo + (rr + 1) * HS + j + 1;
        const T c0 = c[0];
        const T xm = c[-HS], xp = c[HS], ym = c[-1], yp = c[1];
        const T hxx = (xp - T(2) * c0 + xm) * rh00;
        const T hyy = (yp - T(2) * c0 + ym) * rh11;
        const T hxy = (c[HS + 1] - c[HS - 1] - c[-HS + 1] + c[-HS - 1]) * r4h01;
        const T e = hxx + hyy + (hxx * hyy - hxy * hxy);  // det(I + D^2 phi) - 1
        // x + grad phi: the node's coordinate a + (global index) h, then the central difference
        const T x0 = fma(xp - xm, r2h0, x0b);
        const T x1 = fma(yp - ym, r2h1, fma(T(K.off1 + j), h1, K.a1));
        f = rhs_of(K.lvt, M.template rho<2>(x0, x1, T(0)), e);
        chk.add(T(1) + e);
      }
      O::put(op, ldo, rr, j, f);
      if (O::SCALED) amax = fmaxf(amax, fabsf((float)f));
    }
  }
}

#pragma clang fp contract(fast)  // the compiler's default for HIP again

// One tile of the fused kernel for monitor kind MK.  Every descriptor and monitor field is read
// into registers first: a read after the basis copy or a barrier could not use the scalar cache
// (either may write memory, as far as the compiler knows) and would wait for all earlier vector
// memory operations, the copy included.
template <int KIND, int MK>
__device__ inline void stencil_fwd2_tile(const int4 tl, const StencilCtx<typename Op<KIND>::T>& K,
                                         const MonP<typename Op<KIND>::T>* mp, const typename Op<KIND>::T* phi_,
                                         int lcap, const StepArgs& sa) {
  typedef Op<KIND> O;
  typedef typename O::T T;
  constexpr int NW = kFuseWaves;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  __shared__ float red[NW];
  const MonReg<T, MK> M(*mp);
  const SubDev& S = sa.subs[tl.x];
  const AxisDev& A = S.ax[1];
  const int ld = A.ld, ldo = ld + O::OPAD, ldb = A.ldb, n0 = K.n0, n1 = K.n1, row0 = tl.y;
  const void* fwdh = A.fwd;
  const void* fwdl = A.fwdl;
  const T fwd_unscale = T(A.fwd_unscale);
  gmem<T>* out = gpw<T>(S.T);
  const int HS = ld + 4;
  char* op = lds;
  T* halo = (T*)(lds + 16 * ldo * O::LDS_BYTES);
  const int nrb = (n1 + 15) >> 4;
  const int bbytes = nrb * 16 * ldb * (O::BASIS_BYTES / (O::SCALED ? 2 : 1));
  char* lbh = (char*)halo + fused_halo_bytes<KIND>(ld);
  char* lbl = lbh + bbytes;
  const bool lbasis =
      nrb <= 4 * kLdsRb && 16 * ldo * O::LDS_BYTES + fused_halo_bytes<KIND>(ld) + (O::SCALED ? 2 : 1) * bbytes <= lcap;
  if (lbasis) {
    lds_dma(lbh, fwdh, bbytes, NW);
    if (O::SCALED) lds_dma(lbl, fwdl, bbytes, NW);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
  // halo rows row0 - 1 .. row0 + 16, columns -1 .. n1 (mirror ghosts): wave w rows w + NW k, lane
  // columns lane + 64 u, all loads in flight before the first LDS write
  {
    constexpr int HR = (18 + NW - 1) / NW;  // halo rows per wave
    const gmem<T>* phi = (const gmem<T>*)phi_;
    T v[HR][kFuseU];
#pragma unroll
    for (int k = 0; k < HR; ++k) {
      const int r = wave + NW * k;
      const gmem<T>* row = phi + (long)mirror_clamp(row0 + r - 1, n0) * n1;
#pragma unroll
      for (int u = 0; u < kFuseU; ++u) {
        const int c = lane + 64 * u;
        v[k][u] = (r < 18 && c < n1 + 2) ? row[mirror_clamp(c - 1, n1)] : T(0);
      }
    }
#pragma unroll
    for (int k = 0; k < HR; ++k) {
      const int r = wave + NW * k;
#pragma unroll
      for (int u = 0; u < kFuseU; ++u) {
        const int c = lane + 64 * u;
        if (r < 18 && c < n1 + 2) halo[r * HS + c] = v[k][u];
      }
    }
  }
  __syncthreads();
  NodeCheck<T> chk;
  float amax = 0.f;
  fused_nodes2<KIND, MK>(K, M, halo, HS, op, ld, ldo, row0, chk, amax);
  const float sc = O::SCALED ? tile_scale_w<NW>(amax, red) : 1.f;
  if (lbasis) vmem_drain();
  __syncthreads();
  if (O::SCALED && !lbasis) {  // the LDS-basis products split each fragment on the fly
    O::presplit(lds, ldo, 16, ld, &sc, 16);
    __syncthreads();
  }
  const T us = fwd_unscale / T(sc);
  constexpr int NT = (kFuseMaxLd / 16 + NW - 1) / NW;
  typename O::acc_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = typename O::acc_t{0, 0, 0, 0};
  if (lbasis) {
    typename O::acc_t a3[kFuseRb];
#pragma unroll
    for (int t = 0; t < kFuseRb; ++t) a3[t] = typename O::acc_t{0, 0, 0, 0};
    mma_rows_lbasis_w<KIND, NW, kFuseRb>(a3, op, ld, ldo, sc, lbh, lbl, ldb, __builtin_amdgcn_readfirstlane(wave),
                                         nrb, l16, g);
#pragma unroll
    for (int t = 0; t < kFuseRb; ++t) acc[t] = a3[t];
  } else {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int cb = wave + NW * t;
      if (cb < nrb) mma_lds_by_basis<KIND>(acc[t], op, kext<KIND>(n1), ldo, sc, fwdh, fwdl, ldb, cb * 16 + l16, l16, g);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int cb = wave + NW * t;
    if (cb >= nrb) break;
    const int c = cb * 16 + l16;
    for (int q = 0; q < 4; ++q) {
      const int r = row0 + O::crow(g, q);
      if (r < n0 && c < n1) out[(long)r * n1 + c] = acc[t][q] * us;
    }
  }
  const int bad = chk.bits();
  if (bad) atomicOr(&sa.status[K.inst], bad);
}

// tile = (sub, row0, 0, 0)
template <int KIND>
__device__ __attribute__((always_inline)) inline void stencil_fwd2_dispatch(const int4 tl, int lcap,
                                                                           const StepArgs& sa);

template <int KIND>
__global__ __launch_bounds__(64 * kFuseWaves) void stencil_fwd2_kernel(const int4* __restrict__ tiles, int ntiles,
                                                                       int lcap, StepArgs sa) {
  const int tix = xcd_tile();
  if (tix >= ntiles) return;
  stencil_fwd2_dispatch<KIND>(tiles[tix], lcap, sa);
}

// one fused tile: the monitor kind chosen once, the node loop specialised for it.  Always inlined:
// as a called function it would read the step descriptors through flat loads of a stack copy and
// size every caller's registers for its widest monitor specialisation (FP64: 99 -> 248 VGPRs)
template <int KIND>
__device__ __attribute__((always_inline)) inline void stencil_fwd2_dispatch(const int4 tl, int lcap,
                                                                           const StepArgs& sa) {
  typedef typename Op<KIND>::T T;
  StencilCtx<T> K;
  const T* phi_;
  T* F_;
  const MonP<T>* mp = load_ctx(sa, tl.x, K, phi_, F_);
  switch (mp->kind) {
    case MON_CONST: stencil_fwd2_tile<KIND, MON_CONST>(tl, K, mp, phi_, lcap, sa); break;
    case MON_RADIAL: stencil_fwd2_tile<KIND, MON_RADIAL>(tl, K, mp, phi_, lcap, sa); break;
    case MON_SINE: stencil_fwd2_tile<KIND, MON_SINE>(tl, K, mp, phi_, lcap, sa); break;
    case MON_GAUSS: stencil_fwd2_tile<KIND, MON_GAUSS>(tl, K, mp, phi_, lcap, sa); break;
    case MON_ARC_FRONT: stencil_fwd2_tile<KIND, MON_ARC_FRONT>(tl, K, mp, phi_, lcap, sa); break;
    case MON_ARC_SPIRAL: stencil_fwd2_tile<KIND, MON_ARC_SPIRAL>(tl, K, mp, phi_, lcap, sa); break;
    case MON_ARC_SPHERES: stencil_fwd2_tile<KIND, MON_ARC_SPHERES>(tl, K, mp, phi_, lcap, sa); break;
    default: stencil_fwd2_tile<KIND, MON_SEPARABLE>(tl, K, mp, phi_, lcap, sa); break;
  }
}

// ------------------------------------------------------------------------------------------
// One persistent launch per step (2D, preconditioned, parallel coupling).  The three phases of a
// step -- fused stencil + forward last-axis product, axis-0 pair, inverse last-axis product with
// the update and the push transmission -- run in one kernel, separated by grid-wide barriers;
// each workgroup loops over the tiles of a phase (XCD-aware: the workgroups of XCD x take one
// contiguous run of every table).  The tile bodies are the per-launch kernels' own, so results
// are bitwise those of the phase launches.  The host launches at most as many workgroups as the
// device holds at once (occupancy query), and every barrier wait is bounded: on timeout it sets
// ST_SYNC in every instance's status and goes on, so the kernel always ends.
// ------------------------------------------------------------------------------------------

// tiles [first, first + count) of a table of n for this workgroup, stride: the XCD's workgroups
__device__ inline void persist_range(int n, int& first, int& count, int& stride) {
  const int G = gridDim.x, b = blockIdx.x;
  const int q = n >> 3, r = n & 7, x = b & 7, j = b >> 3;
  const int start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  const int cnt = q + (x < r ? 1 : 0);
  first = start + j;
  count = cnt - j;
  stride = G >> 3;
}

// barrier words, each on its own 128-byte line: [0] arrivals of the groups, [32] generation,
// [64 + 32 j] arrivals within group j (workgroups b with b % 8 == j)
constexpr int kBarGen = 32, kBarGroup = 64, kBarWords = 64 + 8 * 32;

__device__ inline void grid_barrier(const PersistArgs& pa, const StepArgs& sa) {
  // each wave's stores of the phase have reached L2 (gfx9: stores count in vmcnt), then one
  // thread per workgroup publishes them at agent scope (release: L2 write-back), arrives in its
  // group (the last of a group arrives for it at the top), waits with plain agent-scope polls,
  // and takes the others' writes (acquire: L1/L2 invalidation)
  vmem_drain();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned* top = pa.bar;
    unsigned* gen = pa.bar + kBarGen;
    const int grp = blockIdx.x & 7;
    unsigned* mine = pa.bar + kBarGroup + 32 * grp;
    const unsigned in_grp = (gridDim.x >> 3);  // the grid is a multiple of 8
    const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool last = false;
    if (__hip_atomic_fetch_add(mine, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == in_grp - 1) {
      __hip_atomic_store(mine, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = __hip_atomic_fetch_add(top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 7u;
    }
    if (last) {
      __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned it = 0;
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++it > pa.spin) {
          for (int q = 0; q < pa.ninst; ++q) atomicOr(&sa.status[q], ST_SYNC);
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

template <int KIND>
__global__ __launch_bounds__(64 * kFuseWaves) void step2_persist_kernel(PersistArgs pa, StepArgs sa) {
  static_assert(kFuseWaves == 8, "the persistent step runs the eight-wave tile bodies");
  int first, count, stride;
  persist_range(pa.n_fused, first, count, stride);
  for (int t = first, k = 0; k < count; t += stride, k += stride) {
    stencil_fwd2_dispatch<KIND>(pa.t_fused[t], pa.lcap, sa);
    __syncthreads();
  }
  grid_barrier(pa, sa);
  persist_range(pa.n_pair, first, count, stride);
  for (int t = first, k = 0; k < count; t += stride, k += stride) {
    strip_tile<KIND, true, 8>(t, pa.t_pair, 0, 0, pa.pair_src, pa.lcap, sa);
    __syncthreads();
  }
  grid_barrier(pa, sa);
  persist_range(pa.n_inv, first, count, stride);
  for (int t = first, k = 0; k < count; t += stride, k += stride) {
    inv_last_tile<KIND, 8>(t, pa.t_inv, pa.part_base, sa);
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------
// forward Euler update (gamma = 0): phi += dt F on live nodes, residual partials
// ------------------------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void euler_kernel(const int4* __restrict__ tiles, int ntiles,
                                                    int part_base, StepArgs sa) {
  __shared__ double red[4];
  const int tix = xcd_tile();
  if (tix >= ntiles) return;
  const int4 tl = tiles[tix];
  const SubDev& S = sa.subs[tl.x];
  const InstDev& I = sa.insts[S.inst];
  const int d = S.dim;
  const int n0 = S.n[0], n1 = S.n[1], n2 = S.n[2];
  const int R = (d == 2) ? n0 : n0 * n1;
  const int C = (d == 2) ? n1 : n2;
  const int row = tl.y + (threadIdx.x >> 6);
  const int col = tl.z + (threadIdx.x & 63);
  double acc = 0.0;
  if (row < R && col < C) {
    const int i0 = (d == 2) ? row : row / n1;
    const int i1 = (d == 2) ? col : row - (row / n1) * n1;
    const int i2 = (d == 2) ? 0 : col;
    double w;
    bool live;
    node_weight(box_of(S), i0, i1, i2, w, live);
    if (live) {
      const long v = (long)row * C + col;
      gmem<T>* phi = gpw<T>(S.phi);
      const T u = T(I.dt) * gp<T>(S.F)[v];
      phi[v] += u;
      acc = w * (double)u * (double)u;
      if (!finite_(u)) atomicOr(&sa.status[S.inst], ST_NONFINITE);
    }
  }
  double hs = S.h[0] * S.h[1] * (d == 3 ? S.h[2] : 1.0);
  double tot = block_sum256(acc, red);
  if (threadIdx.x == 0) sa.partials[part_base + tix] = tot * hs;
}

// ------------------------------------------------------------------------------------------
// K6: transmission (gather of owners' time-n values into artificial nodes)
// entry = (dst subdomain, dst element, src subdomain, src element)
// ------------------------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void transmit_kernel(const SubDev* __restrict__ subs,
                                                       const int4* __restrict__ ent, int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const int4 e = ent[i];
  gpw<T>(subs[e.x].phi)[e.y] = gp<T>(subs[e.z].phi)[e.w];
}

// ------------------------------------------------------------------------------------------
// K8: residual per instance = max over subdomains of sqrt(sum of partials) (fixed order)
// ------------------------------------------------------------------------------------------

__global__ __launch_bounds__(256) void resid_kernel(const SubDev* __restrict__ subs,
                                                    const InstDev* __restrict__ insts, int ninst,
                                                    const double* __restrict__ partials, double* out) {
  // one workgroup per instance, wave w taking subdomains w, w + 4, ..: each subdomain's partial
  // sums are added in a fixed order (lanes strided by 64 with eight loads in flight per lane, then a
  // butterfly within the wave, lane 0's result kept), the same for any number of instances; the
  // instance's residual is the largest subdomain's
  __shared__ double red[4];
  const int q = blockIdx.x;
  if (q >= ninst) return;
  const InstDev& I = insts[q];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double best = 0.0;
  for (int s = I.first_sub + w; s < I.first_sub + I.nsub; s += 4) {
    const double* __restrict__ pp = partials + subs[s].part0;
    const int np = subs[s].nparts;
    double acc = 0.0;
    int p = lane;
    for (; p + 7 * 64 < np; p += 8 * 64) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = pp[p + 64 * u];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; p < np; p += 64) acc += pp[p];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    best = fmax(best, acc);
  }
  if (lane == 0) red[w] = best;
  __syncthreads();
  if (threadIdx.x == 0) out[q] = sqrt(fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}

// ------------------------------------------------------------------------------------------
// state conversion: phi <-> Psi (FP64), in the subdomain's own layout or gathered from a
// global array
// ------------------------------------------------------------------------------------------

template <typename T>
__global__ void phi_from_psi_kernel(SubDev S, const double* __restrict__ psi, int global_layout,
                                    int g1, int g2) {
  const long tot = (long)S.n[0] * S.n[1] * S.n[2];
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < tot;
       v += (long)gridDim.x * blockDim.x) {
    const int i2 = (int)(v % S.n[2]);
    const int i1 = (int)((v / S.n[2]) % S.n[1]);
    const int i0 = (int)(v / ((long)S.n[2] * S.n[1]));
    double q = 0.0;
    const int idx[3] = {i0, i1, i2};
    for (int k = 0; k < S.dim; ++k) {
      const double x = S.a[k] + (double)(S.off[k] + idx[k]) * S.h[k];
      q += x * x;
    }
    long src = v;
    if (global_layout) src = ((long)(S.off[0] + i0) * g1 + (S.off[1] + i1)) * g2 + (S.dim == 3 ? S.off[2] + i2 : 0);
    ((T*)S.phi)[v] = (T)(psi[src] - 0.5 * q);
  }
}

// artificial-boundary nodes are left untouched: they hold the caller's Dirichlet data
template <typename T>
__global__ void psi_from_phi_kernel(SubDev S, double* __restrict__ psi, const double* shift_acc) {
  const long tot = (long)S.n[0] * S.n[1] * S.n[2];
  const double sh = shift_acc[S.inst];
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < tot;
       v += (long)gridDim.x * blockDim.x) {
    const int i2 = (int)(v % S.n[2]);
    const int i1 = (int)((v / S.n[2]) % S.n[1]);
    const int i0 = (int)(v / ((long)S.n[2] * S.n[1]));
    double q = 0.0;
    const int idx[3] = {i0, i1, i2};
    bool art = false;
    for (int k = 0; k < S.dim; ++k) art |= is_artificial(S.art, k, idx[k], S.n[k]);
    if (art) continue;
    for (int k = 0; k < S.dim; ++k) {
      const double x = S.a[k] + (double)(S.off[k] + idx[k]) * S.h[k];
      q += x * x;
    }
    psi[v] = (double)((const T*)S.phi)[v] + 0.5 * q + sh;
  }
}

// ------------------------------------------------------------------------------------------
// K7 + K9: glue (each global node from its owner) and FP64 Jacobian checks
// ------------------------------------------------------------------------------------------

struct GlueArgs {
  const SubDev* subs;
  int first_sub;
  int dim;
  int parts[3];
  int n[3];
  const int* own[3];     // owner part per global node index, per axis
  double a[3], h[3];
  double* mesh;          // dim * prod(n)
  double* psi;           // prod(n) or null
  const double* shift_acc;
  int inst;
  double* minpart;       // one per block
};

template <typename T>
__global__ __launch_bounds__(256) void glue_kernel(GlueArgs g) {
  __shared__ double red[4];
  const long tot = (long)g.n[0] * g.n[1] * (g.dim == 3 ? g.n[2] : 1);
  const long v = blockIdx.x * 256L + threadIdx.x;
  double mdet = 1e300;
  if (v < tot) {
    int gi[3];
    if (g.dim == 2) {
      gi[0] = (int)(v / g.n[1]);
      gi[1] = (int)(v - (long)gi[0] * g.n[1]);
      gi[2] = 0;
    } else {
      gi[2] = (int)(v % g.n[2]);
      gi[1] = (int)((v / g.n[2]) % g.n[1]);
      gi[0] = (int)(v / ((long)g.n[2] * g.n[1]));
    }
    int o[3] = {0, 0, 0};
    for (int k = 0; k < g.dim; ++k) o[k] = g.own[k][gi[k]];
    const int sidx = g.first_sub + (o[0] * g.parts[1] + o[1]) * (g.dim == 3 ? g.parts[2] : 1) +
                     (g.dim == 3 ? o[2] : 0);
    const SubDev& S = g.subs[sidx];
    const T* phi = (const T*)S.phi;
    int l[3], lm[3], lp[3];
    long st[3];
    st[g.dim - 1] = 1;
    for (int k = g.dim - 2; k >= 0; --k) st[k] = st[k + 1] * S.n[k + 1];
    long c = 0;
    for (int k = 0; k < g.dim; ++k) {
      l[k] = gi[k] - S.off[k];
      lm[k] = mlo(l[k]);
      lp[k] = mhi(l[k], S.n[k]);
      c += l[k] * st[k];
    }
    const double pc = (double)phi[c];
    double gr[3], H[3][3];
    double q = 0.0;
    for (int k = 0; k < g.dim; ++k) {
      const double fm = (double)phi[c + (lm[k] - l[k]) * st[k]];
      const double fp = (double)phi[c + (lp[k] - l[k]) * st[k]];
      gr[k] = (fp - fm) / (2.0 * g.h[k]);
      H[k][k] = 1.0 + (fp - 2.0 * pc + fm) / (g.h[k] * g.h[k]);
      const double x = g.a[k] + gi[k] * g.h[k];
      g.mesh[k * tot + v] = x + gr[k];
      q += x * x;
    }
    for (int k = 0; k < g.dim; ++k)
      for (int j = k + 1; j < g.dim; ++j) {
        const long dk = (long)(lp[k] - l[k]) * st[k], dkm = (long)(lm[k] - l[k]) * st[k];
        const long dj = (long)(lp[j] - l[j]) * st[j], djm = (long)(lm[j] - l[j]) * st[j];
        const double x = ((double)phi[c + dk + dj] - (double)phi[c + dk + djm] -
                          (double)phi[c + dkm + dj] + (double)phi[c + dkm + djm]) /
                         (4.0 * g.h[k] * g.h[j]);
        H[k][j] = x;
        H[j][k] = x;
      }
    if (g.psi) g.psi[v] = pc + 0.5 * q + g.shift_acc[g.inst];
    if (g.dim == 2) {
      mdet = H[0][0] * H[1][1] - H[0][1] * H[1][0];
    } else {
      mdet = H[0][0] * (H[1][1] * H[2][2] - H[1][2] * H[2][1]) -
             H[0][1] * (H[1][0] * H[2][2] - H[1][2] * H[2][0]) +
             H[0][2] * (H[1][0] * H[2][1] - H[1][1] * H[2][0]);
    }
  }
  const double mn = block_min256(mdet, red);
  if (threadIdx.x == 0) g.minpart[blockIdx.x] = mn;
}

// signed cell measure: quad area (shoelace) in 2D, minimum corner Jacobian in 3D
__global__ __launch_bounds__(256) void cell_kernel(const double* __restrict__ mesh, int dim,
                                                   int n0, int n1, int n2, double* minpart) {
  __shared__ double red[4];
  const long c0 = n0 - 1, c1 = n1 - 1, c2 = (dim == 3) ? n2 - 1 : 1;
  const long tot = c0 * c1 * c2;
  // chunk b of 256 cells from the XCD-aware order: each XCD reads one contiguous run of the mesh
  const int tix = xcd_tile();
  const long v = tix * 256L + threadIdx.x;
  double best = 1e300;
  if (v < tot) {
    if (dim == 2) {
      const long i = v / c1, j = v - (v / c1) * c1;
      const long np = (long)n0 * n1;
      const double* X = mesh;
      const double* Y = mesh + np;
      const long p00 = i * n1 + j, p10 = (i + 1) * n1 + j, p11 = (i + 1) * n1 + j + 1, p01 = i * n1 + j + 1;
      best = 0.5 * ((X[p00] * Y[p10] - X[p10] * Y[p00]) + (X[p10] * Y[p11] - X[p11] * Y[p10]) +
                    (X[p11] * Y[p01] - X[p01] * Y[p11]) + (X[p01] * Y[p00] - X[p00] * Y[p01]));
    } else {
      const long k = v % c2, j = (v / c2) % c1, i = v / (c2 * c1);
      const long np = (long)n0 * n1 * n2;
      auto P = [&](long a, long b, long c, int comp) {
        return mesh[comp * np + (a * n1 + b) * n2 + c];
      };
      for (int q = 0; q < 8; ++q) {
        const int a = q >> 2, bb = (q >> 1) & 1, cc = q & 1;
        double e[3][3];
        for (int comp = 0; comp < 3; ++comp) {
          const double base = P(i + a, j + bb, k + cc, comp);
          e[0][comp] = P(i + 1 - a, j + bb, k + cc, comp) - base;
          e[1][comp] = P(i + a, j + 1 - bb, k + cc, comp) - base;
          e[2][comp] = P(i + a, j + bb, k + 1 - cc, comp) - base;
        }
        const double cx = e[1][1] * e[2][2] - e[1][2] * e[2][1];
        const double cy = e[1][2] * e[2][0] - e[1][0] * e[2][2];
        const double cz = e[1][0] * e[2][1] - e[1][1] * e[2][0];
        const double sgn = (double)((1 - 2 * a) * (1 - 2 * bb) * (1 - 2 * cc));
        best = fmin(best, sgn * (e[0][0] * cx + e[0][1] * cy + e[0][2] * cz));
      }
    }
  }
  const double mn = block_min256(best, red);
  if (threadIdx.x == 0) minpart[tix] = mn;
}

__global__ __launch_bounds__(256) void min_reduce_kernel(const double* __restrict__ x, long n,
                                                         double* out) {
  __shared__ double red[4];
  double m = 1e300;
  for (long i = threadIdx.x; i < n; i += 256) m = fmin(m, x[i]);
  const double r = block_min256(m, red);
  if (threadIdx.x == 0) *out = r;
}

// ------------------------------------------------------------------------------------------
// host launch wrappers
// ------------------------------------------------------------------------------------------

static inline unsigned nblk(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_transmit(int prec, const SubDev* subs, const int4* ent, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (prec == PREC_F64)
    hipLaunchKernelGGL(transmit_kernel<double>, dim3(nblk(count, 256)), dim3(256), 0, s, subs, ent, count);
  else
    hipLaunchKernelGGL(transmit_kernel<float>, dim3(nblk(count, 256)), dim3(256), 0, s, subs, ent, count);
  return hipGetLastError();
}

hipError_t launch_stencil(int prec, int dim, const int4* tiles, int ntiles, const StepArgs& sa, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (dim == 2) {
    if (prec == PREC_F64)
      hipLaunchKernelGGL(stencil2_kernel<double>, dim3(ntiles), dim3(256), 0, s, tiles, ntiles, sa);
    else
      hipLaunchKernelGGL(stencil2_kernel<float>, dim3(ntiles), dim3(256), 0, s, tiles, ntiles, sa);
  } else {
    if (prec == PREC_F64)
      hipLaunchKernelGGL(stencil3_kernel<double>, dim3(ntiles), dim3(256), 0, s, tiles, ntiles, sa);
    else
      hipLaunchKernelGGL(stencil3_kernel<float>, dim3(ntiles), dim3(256), 0, s, tiles, ntiles, sa);
  }
  return hipGetLastError();
}

hipError_t launch_euler(int prec, const int4* tiles, int ntiles, int part_base, const StepArgs& sa,
                        hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (prec == PREC_F64)
    hipLaunchKernelGGL(euler_kernel<double>, dim3(ntiles), dim3(256), 0, s, tiles, ntiles, part_base, sa);
  else
    hipLaunchKernelGGL(euler_kernel<float>, dim3(ntiles), dim3(256), 0, s, tiles, ntiles, part_base, sa);
  return hipGetLastError();
}

// LDS bytes of a 16-row data operand for a padded axis length ld (row stride ld + 16 bytes)
static inline size_t op_lds(int prec, int ld) {
  return (size_t)16 * (ld + (prec == PREC_F64 ? 2 : 4)) * (prec == PREC_F64 ? 8 : 4);
}

hipError_t launch_fwd_last(int prec, const int4* tiles, int ntiles, int maxld, const StepArgs& sa, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const size_t sh = op_lds(prec, maxld);
  if (prec == PREC_F64)
    hipLaunchKernelGGL(fwd_last_kernel<PREC_F64>, dim3(ntiles), dim3(256), sh, s, tiles, ntiles, sa);
  else if (prec == PREC_F32)
    hipLaunchKernelGGL(fwd_last_kernel<PREC_F32>, dim3(ntiles), dim3(256), sh, s, tiles, ntiles, sa);
  else
    hipLaunchKernelGGL(fwd_last_kernel<PREC_SPLIT16>, dim3(ntiles), dim3(256), sh, s, tiles, ntiles, sa);
  return hipGetLastError();
}

hipError_t launch_inv_last(int prec, const int4* tiles, int ntiles, int maxld, int part_base, int eight_max,
                           const StepArgs& sa, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const size_t sh = op_lds(prec, maxld);
  const bool eight = ntiles <= eight_max;  // latency-bound: at most two workgroups per compute unit
#define PMA_INV(K)                                                                                                    \
  do {                                                                                                                \
    if (eight)                                                                                                        \
      hipLaunchKernelGGL((inv_last_kernel<K, 8>), dim3(ntiles), dim3(512), sh, s, tiles, ntiles, part_base, sa);     \
    else                                                                                                              \
      hipLaunchKernelGGL((inv_last_kernel<K, 4>), dim3(ntiles), dim3(256), sh, s, tiles, ntiles, part_base, sa);     \
  } while (0)
  if (prec == PREC_F64)
    PMA_INV(PREC_F64);
  else if (prec == PREC_F32)
    PMA_INV(PREC_F32);
  else
    PMA_INV(PREC_SPLIT16);
#undef PMA_INV
  return hipGetLastError();
}

// fused stencil + forward last-axis product (2D); lneed: the launch's largest LDS footprint
hipError_t launch_stencil_fwd2(int prec, const int4* tiles, int ntiles, int lneed, const StepArgs& sa, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const size_t sh = (size_t)lneed;
  if (prec == PREC_F64)
    hipLaunchKernelGGL(stencil_fwd2_kernel<PREC_F64>, dim3(ntiles), dim3(64 * kFuseWaves), sh, s, tiles, ntiles, lneed, sa);
  else if (prec == PREC_F32)
    hipLaunchKernelGGL(stencil_fwd2_kernel<PREC_F32>, dim3(ntiles), dim3(64 * kFuseWaves), sh, s, tiles, ntiles, lneed, sa);
  else
    hipLaunchKernelGGL(stencil_fwd2_kernel<PREC_SPLIT16>, dim3(ntiles), dim3(64 * kFuseWaves), sh, s, tiles, ntiles, lneed, sa);
  return hipGetLastError();
}

// LDS bytes of the fused kernel for a last axis of padded length ld and basis row stride ldb with
// n nodes (basis copied or not)
int fused_lds_bytes(int prec, int ld, int ldb, int n, bool basis) {
  const int ob = prec == PREC_F64 ? 8 : 4;
  const int hb = prec == PREC_F64 ? fused_halo_bytes<PREC_F64>(ld) : fused_halo_bytes<PREC_F32>(ld);
  const int bb = prec == PREC_F64 ? 8 : 4;  // basis bytes per entry (split form: hi + lo)
  return (int)op_lds(prec, ld) + hb + (basis ? ((n + 15) / 16) * 16 * ldb * bb : 0);
}

// lneed: the largest LDS footprint (strip + basis copy) among the launch's subdomains whose copy
// fits in a workgroup's LDS (0: none); such tiles take the LDS-basis path
hipError_t launch_strip(int prec, bool pair, const int4* tiles, int ntiles, int maxld, int lneed, int axis, int inv,
                        int src_sel, int eight_max, const StepArgs& sa, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (maxld > kLongMaxLd) return hipErrorInvalidValue;
  if (maxld > kMaxLd) {  // long axes
    const size_t shl = op_lds(prec, maxld);
#define PMA_LONG(K, P) \
  hipLaunchKernelGGL((strip_long_kernel<K, P>), dim3(ntiles), dim3(256), shl, s, tiles, ntiles, axis, inv, src_sel, sa)
    if (prec == PREC_F64) {
      if (pair) PMA_LONG(PREC_F64, true); else PMA_LONG(PREC_F64, false);
    } else if (prec == PREC_F32) {
      if (pair) PMA_LONG(PREC_F32, true); else PMA_LONG(PREC_F32, false);
    } else {
      if (pair) PMA_LONG(PREC_SPLIT16, true); else PMA_LONG(PREC_SPLIT16, false);
    }
#undef PMA_LONG
    return hipGetLastError();
  }
  const size_t sh = std::max<size_t>(op_lds(prec, maxld), (size_t)lneed);
  const int lcap = (int)sh;
  const bool eight = ntiles <= eight_max;  // latency-bound: at most two workgroups per compute unit
#define PMA_STRIP(K, P)                                                                                         \
  do {                                                                                                          \
    if (eight && maxld <= 16 * 8 * 3)                                                                           \
      hipLaunchKernelGGL((strip_kernel<K, P, 8, 3>), dim3(ntiles), dim3(512), sh, s, tiles, ntiles, axis, inv,  \
                         src_sel, lcap, sa);                                                                    \
    else if (eight)                                                                                             \
      hipLaunchKernelGGL((strip_kernel<K, P, 8>), dim3(ntiles), dim3(512), sh, s, tiles, ntiles, axis, inv,     \
                         src_sel, lcap, sa);                                                                    \
    else                                                                                                        \
      hipLaunchKernelGGL((strip_kernel<K, P, 4>), dim3(ntiles), dim3(256), sh, s, tiles, ntiles, axis, inv,     \
                         src_sel, lcap, sa);                                                                    \
  } while (0)
  if (prec == PREC_F64) {
    if (pair) PMA_STRIP(PREC_F64, true); else PMA_STRIP(PREC_F64, false);
  } else if (prec == PREC_F32) {
    if (pair) PMA_STRIP(PREC_F32, true); else PMA_STRIP(PREC_F32, false);
  } else {
    if (pair) PMA_STRIP(PREC_SPLIT16, true); else PMA_STRIP(PREC_SPLIT16, false);
  }
#undef PMA_STRIP
  return hipGetLastError();
}

hipError_t launch_strip4(int prec, bool pair, const int4* tiles, int ntiles, int maxld, int axis, int inv,
                         int src_sel, const StepArgs& sa, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (prec == PREC_F64 || maxld > kWideMaxLd) return hipErrorInvalidValue;
  const size_t sh = (size_t)64 * (maxld + Op<PREC_F32>::OPAD) * 4;
#define PMA_STRIP4(K, P) \
  hipLaunchKernelGGL((strip4_kernel<K, P>), dim3(ntiles), dim3(256), sh, s, tiles, ntiles, axis, inv, src_sel, sa)
  if (prec == PREC_F32) {
    if (pair) PMA_STRIP4(PREC_F32, true); else PMA_STRIP4(PREC_F32, false);
  } else {
    if (pair) PMA_STRIP4(PREC_SPLIT16, true); else PMA_STRIP4(PREC_SPLIT16, false);
  }
#undef PMA_STRIP4
  return hipGetLastError();
}

// kernels using more than 64 KiB of dynamic LDS must say so once per process
hipError_t enable_large_lds() {
  static hipError_t rc = [] {
    // 160 KiB per workgroup on gfx950; the strip kernels' LDS-basis path asks for at most lim
    const int lim = 160 * 1024 - 4096;
    hipError_t e = hipSuccess;
    const void* ks[] = {(const void*)fwd_last_kernel<PREC_F64>, (const void*)fwd_last_kernel<PREC_F32>,
                        (const void*)fwd_last_kernel<PREC_SPLIT16>, (const void*)inv_last_kernel<PREC_F64, 4>,
                        (const void*)inv_last_kernel<PREC_F32, 4>, (const void*)inv_last_kernel<PREC_SPLIT16, 4>,
                        (const void*)inv_last_kernel<PREC_F64, 8>, (const void*)inv_last_kernel<PREC_F32, 8>,
                        (const void*)inv_last_kernel<PREC_SPLIT16, 8>,
                        (const void*)strip_kernel<PREC_F64, true, 4>, (const void*)strip_kernel<PREC_F64, false, 4>,
                        (const void*)strip_kernel<PREC_F32, true, 4>, (const void*)strip_kernel<PREC_F32, false, 4>,
                        (const void*)strip_kernel<PREC_SPLIT16, true, 4>, (const void*)strip_kernel<PREC_SPLIT16, false, 4>,
                        (const void*)strip_kernel<PREC_F64, true, 8>, (const void*)strip_kernel<PREC_F64, false, 8>,
                        (const void*)strip_kernel<PREC_F32, true, 8>, (const void*)strip_kernel<PREC_F32, false, 8>,
                        (const void*)strip_kernel<PREC_SPLIT16, true, 8>, (const void*)strip_kernel<PREC_SPLIT16, false, 8>,
                        (const void*)strip_kernel<PREC_F64, true, 8, 3>, (const void*)strip_kernel<PREC_F64, false, 8, 3>,
                        (const void*)strip_kernel<PREC_F32, true, 8, 3>, (const void*)strip_kernel<PREC_F32, false, 8, 3>,
                        (const void*)strip_kernel<PREC_SPLIT16, true, 8, 3>,
                        (const void*)strip_kernel<PREC_SPLIT16, false, 8, 3>,
                        (const void*)stencil_fwd2_kernel<PREC_F64>, (const void*)stencil_fwd2_kernel<PREC_F32>,
                        (const void*)stencil_fwd2_kernel<PREC_SPLIT16>, (const void*)strip4_kernel<PREC_F32, true>,
                        (const void*)strip4_kernel<PREC_F32, false>, (const void*)strip4_kernel<PREC_SPLIT16, true>,
                        (const void*)strip4_kernel<PREC_SPLIT16, false>, (const void*)strip_long_kernel<PREC_F64, true>,
                        (const void*)strip_long_kernel<PREC_F64, false>, (const void*)strip_long_kernel<PREC_F32, true>,
                        (const void*)strip_long_kernel<PREC_F32, false>, (const void*)strip_long_kernel<PREC_SPLIT16, true>,
                        (const void*)strip_long_kernel<PREC_SPLIT16, false>, (const void*)step2_persist_kernel<PREC_F64>,
                        (const void*)step2_persist_kernel<PREC_F32>, (const void*)step2_persist_kernel<PREC_SPLIT16>};
    for (const void* k : ks) {
      // whatever the kernel's static LDS leaves of the 160 KiB (at most lim)
      hipFuncAttributes fa{};
      hipError_t r = hipFuncGetAttributes(&fa, k);
      if (r == hipSuccess)
        r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                std::min(lim, 160 * 1024 - (int)fa.sharedSizeBytes));
      if (r != hipSuccess) e = r;
    }
    (void)hipGetLastError();  // the status is returned, not left pending for the next launch
    return e;
  }();
  return rc;
}

hipError_t launch_resid(const SubDev* subs, const InstDev* insts, int ninst, const double* partials,
                        double* out, hipStream_t s) {
  if (ninst <= 0) return hipSuccess;
  hipLaunchKernelGGL(resid_kernel, dim3(ninst), dim3(256), 0, s, subs, insts, ninst, partials, out);
  return hipGetLastError();
}

hipError_t launch_phi_from_psi(int prec, const SubDev& S, const double* psi, int global_layout, int g1,
                               int g2, hipStream_t s) {
  const long tot = (long)S.n[0] * S.n[1] * S.n[2];
  const unsigned g = (unsigned)std::min<long>(nblk(tot, 256), 4096);
  if (prec == PREC_F64)
    hipLaunchKernelGGL(phi_from_psi_kernel<double>, dim3(g), dim3(256), 0, s, S, psi, global_layout, g1, g2);
  else
    hipLaunchKernelGGL(phi_from_psi_kernel<float>, dim3(g), dim3(256), 0, s, S, psi, global_layout, g1, g2);
  return hipGetLastError();
}

hipError_t launch_psi_from_phi(int prec, const SubDev& S, double* psi, const double* shift_acc,
                               hipStream_t s) {
  const long tot = (long)S.n[0] * S.n[1] * S.n[2];
  const unsigned g = (unsigned)std::min<long>(nblk(tot, 256), 4096);
  if (prec == PREC_F64)
    hipLaunchKernelGGL(psi_from_phi_kernel<double>, dim3(g), dim3(256), 0, s, S, psi, shift_acc);
  else
    hipLaunchKernelGGL(psi_from_phi_kernel<float>, dim3(g), dim3(256), 0, s, S, psi, shift_acc);
  return hipGetLastError();
}

long glue_blocks(long nodes) { return nblk(nodes, 256); }

hipError_t launch_glue(int prec, const GlueArgs& g, hipStream_t s) {
  const long tot = (long)g.n[0] * g.n[1] * (g.dim == 3 ? g.n[2] : 1);
  if (prec == PREC_F64)
    hipLaunchKernelGGL(glue_kernel<double>, dim3(nblk(tot, 256)), dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(glue_kernel<float>, dim3(nblk(tot, 256)), dim3(256), 0, s, g);
  return hipGetLastError();
}

long cell_blocks(int dim, const int* n) {
  long t = (long)(n[0] - 1) * (n[1] - 1) * (dim == 3 ? (n[2] - 1) : 1);
  return nblk(t, 256);
}

hipError_t launch_cells(const double* mesh, int dim, const int* n, double* minpart, hipStream_t s) {
  const long nb = cell_blocks(dim, n);
  hipLaunchKernelGGL(cell_kernel, dim3(nb), dim3(256), 0, s, mesh, dim, n[0], n[1], n[2], minpart);
  return hipGetLastError();
}

// Mesh quality (Sec. 4.5): E = |Omega_c| (rho(x) / theta) J at every node of the glued mesh, J the
// Jacobian det(dx / dxi) from second-order differences of the mesh (one-sided three-point at the
// box faces).  Each block leaves sum w E^2 (w: trapezoid weight times prod h) and max E.
template <int MK>
__global__ __launch_bounds__(256) void quality_kernel(const double* __restrict__ mesh, int dim, int n0, int n1,
                                                      int n2, double h0, double h1, double h2, MonP<double> mp,
                                                      double vol_theta, double* __restrict__ part) {
  __shared__ double red[4];
  const int n[3] = {n0, n1, dim == 3 ? n2 : 1};
  const double h[3] = {h0, h1, h2};
  const long tot = (long)n[0] * n[1] * n[2];
  // chunk b of 256 nodes from the XCD-aware order: each XCD reads one contiguous run of the mesh
  // (its planes then stay in one L2); partial b still belongs to chunk b
  const int tix = xcd_tile();
  const long v = tix * 256L + threadIdx.x;
  double sum = 0.0, mx = -1e300;
  if (v < tot) {
    const int i[3] = {(int)(v / ((long)n[1] * n[2])), (int)((v / n[2]) % n[1]), (int)(v % n[2])};
    const long st[3] = {(long)n[1] * n[2], n[2], 1};
    double Jm[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, x[3] = {0, 0, 0};
    double w = 1.0;
    for (int c = 0; c < dim; ++c) x[c] = mesh[c * tot + v];
    for (int k = 0; k < dim; ++k) {
      const int a = i[k], nk = n[k];
      w *= (a == 0 || a == nk - 1 ? 0.5 : 1.0) * h[k];
      for (int c = 0; c < dim; ++c) {
        const double* X = mesh + c * tot + v;
        double d;
        if (a == 0) d = (-3.0 * X[0] + 4.0 * X[st[k]] - X[2 * st[k]]) / (2.0 * h[k]);
        else if (a == nk - 1) d = (3.0 * X[0] - 4.0 * X[-st[k]] + X[-2 * st[k]]) / (2.0 * h[k]);
        else d = (X[st[k]] - X[-st[k]]) / (2.0 * h[k]);
        Jm[c][k] = d;
      }
    }
    const double J = Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) -
                     Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0]) +
                     Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
    const MonReg<double, MK> M(mp);
    const double rho = dim == 3 ? M.template rho<3>(x[0], x[1], x[2]) : M.template rho<2>(x[0], x[1], 0.0);
    const double E = vol_theta * rho * J;
    sum = w * E * E;
    mx = E;
  }
  const double s = block_sum256(sum, red);
  __syncthreads();
  const double m = -block_min256(-mx, red);
  if (threadIdx.x == 0) {
    part[2 * tix] = s;
    part[2 * tix + 1] = m;
  }
}

// E_2 = sqrt(sum w E^2 / |Omega_c|) and E_max from the per-block pairs
__global__ __launch_bounds__(256) void quality_reduce_kernel(const double* __restrict__ part, long nb, double vol,
                                                             double* out) {
  __shared__ double red[4];
  double s = 0.0, m = -1e300;
  for (long b = threadIdx.x; b < nb; b += 256) {
    s += part[2 * b];
    m = fmax(m, part[2 * b + 1]);
  }
  const double ts = block_sum256(s, red);
  __syncthreads();
  const double tm = -block_min256(-m, red);
  if (threadIdx.x == 0) {
    out[0] = sqrt(ts / vol);
    out[1] = tm;
  }
}

hipError_t launch_quality(const double* mesh, int dim, const int* n, const double* h, const MonP<double>& mp,
                          double vol, double theta, double* part, double* out, hipStream_t s) {
  const long tot = (long)n[0] * n[1] * (dim == 3 ? n[2] : 1);
  const long nb = nblk(tot, 256);
  const double vt = vol / theta;
  const double h2 = dim == 3 ? h[2] : 1.0;
#define PMA_QUALITY(MK)                                                                                          \
  hipLaunchKernelGGL(quality_kernel<MK>, dim3(nb), dim3(256), 0, s, mesh, dim, n[0], n[1], n[2], h[0], h[1], h2, \
                     mp, vt, part)
  switch (mp.kind) {
    case MON_CONST: PMA_QUALITY(MON_CONST); break;
    case MON_RADIAL: PMA_QUALITY(MON_RADIAL); break;
    case MON_SINE: PMA_QUALITY(MON_SINE); break;
    case MON_GAUSS: PMA_QUALITY(MON_GAUSS); break;
    case MON_SEPARABLE: PMA_QUALITY(MON_SEPARABLE); break;
    case MON_ARC_FRONT: PMA_QUALITY(MON_ARC_FRONT); break;
    case MON_ARC_SPIRAL: PMA_QUALITY(MON_ARC_SPIRAL); break;
    default: PMA_QUALITY(MON_ARC_SPHERES); break;
  }
#undef PMA_QUALITY
  hipLaunchKernelGGL(quality_reduce_kernel, dim3(1), dim3(256), 0, s, part, nb, vol, out);
  return hipGetLastError();
}

hipError_t launch_min_reduce(const double* x, long n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(min_reduce_kernel, dim3(1), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

// the persistent step: static LDS of the kernel, and how many workgroups of 512 threads with
// `dyn` bytes of dynamic LDS the device holds at once (0 if none fits)
int persist_capacity(int prec, size_t dyn, int* static_lds) {
  const void* k = prec == PREC_F64 ? (const void*)step2_persist_kernel<PREC_F64>
                  : prec == PREC_F32 ? (const void*)step2_persist_kernel<PREC_F32>
                                     : (const void*)step2_persist_kernel<PREC_SPLIT16>;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, k) != hipSuccess) return 0;
  if (static_lds) *static_lds = (int)fa.sharedSizeBytes;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64 * kFuseWaves, dyn) != hipSuccess) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

hipError_t launch_step2_persist(int prec, int grid, size_t dyn, const PersistArgs& pa, const StepArgs& sa,
                                hipStream_t s) {
  if (grid <= 0 || (grid & 7)) return hipErrorInvalidValue;
  if (prec == PREC_F64)
    hipLaunchKernelGGL(step2_persist_kernel<PREC_F64>, dim3(grid), dim3(64 * kFuseWaves), dyn, s, pa, sa);
  else if (prec == PREC_F32)
    hipLaunchKernelGGL(step2_persist_kernel<PREC_F32>, dim3(grid), dim3(64 * kFuseWaves), dyn, s, pa, sa);
  else
    hipLaunchKernelGGL(step2_persist_kernel<PREC_SPLIT16>, dim3(grid), dim3(64 * kFuseWaves), dyn, s, pa, sa);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Fixed device scratch for the entry point that allocates nothing: one array per GPU, loaded
// with the code object and held until the process ends.  In host code `scratch` names a host
// stand-in, not device memory: kernels and copies take the address that hipGetSymbolAddress
// returns for the current device, looked up once per device and kept here.
// ------------------------------------------------------------------------------------------

static __device__ __align__(256) char scratch[kScratchBytes];

static constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices];

hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* scratch_ptr(int device) {
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

}  // namespace pma
