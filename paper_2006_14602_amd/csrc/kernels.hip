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

// ------------------------------------------------------------------------------------------
// monitor: log rho(x), computed as log1p of the excess over 1 where rho = 1 + (...)
// ------------------------------------------------------------------------------------------

__device__ inline float dexp(float x) { return expf(x); }
__device__ inline double dexp(double x) { return exp(x); }
__device__ inline float dlog1p(float x) { return log1pf(x); }
__device__ inline double dlog1p(double x) { return log1p(x); }
__device__ inline float dlog(float x) { return logf(x); }
__device__ inline double dlog(double x) { return log(x); }
__device__ inline float dsinpi(float x) { return sinpif(x); }
__device__ inline double dsinpi(double x) { return sinpi(x); }

// sech^2(z) = 4 e^{-2|z|} / (1 + e^{-2|z|})^2 (no overflow for large |z|)
template <typename T>
__device__ inline T sech2(T z) {
  T e = dexp(T(-2) * fabs(z));
  T q = T(1) + e;
  return T(4) * e / (q * q);
}

template <typename T>
__device__ inline T log_rho(const MonitorDev& m, int dim, T x0, T x1, T x2) {
  switch (m.kind) {
    case MON_CONST:
      return dlog(T(m.amp));
    case MON_RADIAL: {
      T d0 = x0 - T(m.c[0]), d1 = x1 - T(m.c[1]);
      T r2 = d0 * d0 + d1 * d1;
      if (dim == 3) {
        T d2 = x2 - T(m.c[2]);
        r2 += d2 * d2;
      }
      return dlog1p(T(m.amp) * sech2(T(m.k) * (r2 - T(m.r0) * T(m.r0))));
    }
    case MON_SINE: {
      T s = x1 - T(m.c[1]) - T(m.r0) * dsinpi(T(2) * x0);
      return dlog1p(T(m.amp) * sech2(T(m.k) * s));
    }
    case MON_GAUSS: {
      T acc = T(0);
      for (int b = 0; b < m.nb; ++b) {
        T d0 = x0 - T(m.bc[b][0]), d1 = x1 - T(m.bc[b][1]);
        T r2 = d0 * d0 + d1 * d1;
        if (dim == 3) {
          T d2 = x2 - T(m.bc[b][2]);
          r2 += d2 * d2;
        }
        T w = T(m.bw[b]);
        acc += T(m.bamp[b]) * dexp(-r2 / (T(2) * w * w));
      }
      return dlog1p(acc);
    }
    case MON_SEPARABLE: {
      T r = dlog1p(T(m.amp_axes[0]) * sech2(T(m.k_axes[0]) * (x0 - T(m.c[0])))) +
            dlog1p(T(m.amp_axes[1]) * sech2(T(m.k_axes[1]) * (x1 - T(m.c[1]))));
      if (dim == 3) r += dlog1p(T(m.amp_axes[2]) * sech2(T(m.k_axes[2]) * (x2 - T(m.c[2]))));
      return r;
    }
  }
  return T(0);
}

__device__ inline bool is_artificial(int art, int k, int i, int n) {
  return (i == 0 && ((art >> (2 * k)) & 1)) || (i == n - 1 && ((art >> (2 * k + 1)) & 1));
}

// mirror index for the Neumann ghost of phi: -1 -> 1, n -> n - 2
__device__ inline int mlo(int i) { return i > 0 ? i - 1 : 1; }
__device__ inline int mhi(int i, int n) { return i < n - 1 ? i + 1 : n - 2; }

template <typename T>
__device__ inline bool finite_(T x) { return isfinite(x); }

// ------------------------------------------------------------------------------------------
// K1/K2: stencil + monitor + log.  Tile = 4 rows x 64 columns of the [rows][last axis] view.
// ------------------------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void stencil_kernel(const int4* __restrict__ tiles, int ntiles,
                                                      StepArgs sa) {
  if ((int)blockIdx.x >= ntiles) return;
  const int4 tl = tiles[blockIdx.x];
  const SubDev& S = sa.subs[tl.x];
  const InstDev& I = sa.insts[S.inst];
  const int d = S.dim;
  const int n0 = S.n[0], n1 = S.n[1], n2 = S.n[2];
  const int R = (d == 2) ? n0 : n0 * n1;
  const int C = (d == 2) ? n1 : n2;
  const int row = tl.y + (threadIdx.x >> 6);
  const int col = tl.z + (threadIdx.x & 63);
  if (row >= R || col >= C) return;
  const T* __restrict__ phi = (const T*)S.phi;
  T* __restrict__ F = (T*)S.F;
  const T h0 = T(S.h[0]), h1 = T(S.h[1]), h2 = T(S.h[2]);
  if (d == 2) {
    const int i = row, j = col;
    const long v = (long)i * n1 + j;
    if (is_artificial(S.art, 0, i, n0) || is_artificial(S.art, 1, j, n1)) {
      F[v] = T(0);
      return;
    }
    const int im = mlo(i), ip = mhi(i, n0), jm = mlo(j), jp = mhi(j, n1);
    const T c = phi[v];
    const T xm = phi[(long)im * n1 + j], xp = phi[(long)ip * n1 + j];
    const T ym = phi[(long)i * n1 + jm], yp = phi[(long)i * n1 + jp];
    const T mm = phi[(long)im * n1 + jm], mp = phi[(long)im * n1 + jp];
    const T pm = phi[(long)ip * n1 + jm], pp = phi[(long)ip * n1 + jp];
    const T gx = (xp - xm) / (T(2) * h0);
    const T gy = (yp - ym) / (T(2) * h1);
    const T hxx = (xp - T(2) * c + xm) / (h0 * h0);
    const T hyy = (yp - T(2) * c + ym) / (h1 * h1);
    const T hxy = (pp - pm - mp + mm) / (T(4) * h0 * h1);
    const T e = hxx + hyy + (hxx * hyy - hxy * hxy);  // det(I + D^2 phi) - 1
    const T x0 = T(S.a[0]) + T(S.off[0] + i) * h0 + gx;
    const T x1 = T(S.a[1]) + T(S.off[1] + j) * h1 + gy;
    const T f = T(I.log_vol_theta) + log_rho<T>(I.mon, 2, x0, x1, T(0)) + dlog1p(e);
    F[v] = f;
    if (!(T(1) + e > T(0))) atomicOr(&sa.status[S.inst], ST_TANGLED);
    else if (!finite_(f)) atomicOr(&sa.status[S.inst], ST_NONFINITE);
  } else {
    const int i = row / n1, j = row - (row / n1) * n1, k = col;
    const long s1 = n2, s0 = (long)n1 * n2;
    const long v = i * s0 + j * s1 + k;
    if (is_artificial(S.art, 0, i, n0) || is_artificial(S.art, 1, j, n1) ||
        is_artificial(S.art, 2, k, n2)) {
      F[v] = T(0);
      return;
    }
    const long im = mlo(i) * s0, ip = mhi(i, n0) * s0;
    const long jm = mlo(j) * s1, jp = mhi(j, n1) * s1;
    const long km = mlo(k), kp = mhi(k, n2);
    const long I0 = i * s0, J0 = j * s1, K0 = k;
    const T c = phi[v];
    const T xm = phi[im + J0 + K0], xp = phi[ip + J0 + K0];
    const T ym = phi[I0 + jm + K0], yp = phi[I0 + jp + K0];
    const T zm = phi[I0 + J0 + km], zp = phi[I0 + J0 + kp];
    const T xy = (phi[ip + jp + K0] - phi[ip + jm + K0] - phi[im + jp + K0] + phi[im + jm + K0]);
    const T xz = (phi[ip + J0 + kp] - phi[ip + J0 + km] - phi[im + J0 + kp] + phi[im + J0 + km]);
    const T yz = (phi[I0 + jp + kp] - phi[I0 + jp + km] - phi[I0 + jm + kp] + phi[I0 + jm + km]);
    const T gx = (xp - xm) / (T(2) * h0);
    const T gy = (yp - ym) / (T(2) * h1);
    const T gz = (zp - zm) / (T(2) * h2);
    const T a = (xp - T(2) * c + xm) / (h0 * h0);
    const T b = (yp - T(2) * c + ym) / (h1 * h1);
    const T q = (zp - T(2) * c + zm) / (h2 * h2);
    const T p = xy / (T(4) * h0 * h1);
    const T r = xz / (T(4) * h0 * h2);
    const T s = yz / (T(4) * h1 * h2);
    // det(I + H) - 1 = tr H + (sum of principal 2x2 minors) + det H
    const T tr = a + b + q;
    const T m2 = (a * b - p * p) + (a * q - r * r) + (b * q - s * s);
    const T dt3 = a * (b * q - s * s) - p * (p * q - s * r) + r * (p * s - b * r);
    const T e = tr + m2 + dt3;
    const T x0 = T(S.a[0]) + T(S.off[0] + i) * h0 + gx;
    const T x1 = T(S.a[1]) + T(S.off[1] + j) * h1 + gy;
    const T x2 = T(S.a[2]) + T(S.off[2] + k) * h2 + gz;
    const T f = T(I.log_vol_theta) + log_rho<T>(I.mon, 3, x0, x1, x2) + dlog1p(e);
    F[v] = f;
    if (!(T(1) + e > T(0))) atomicOr(&sa.status[S.inst], ST_TANGLED);
    else if (!finite_(f)) atomicOr(&sa.status[S.inst], ST_NONFINITE);
  }
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

__device__ inline double block_min256(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
  __syncthreads();
  return r;
}

// shift removed from phi each step: mean over the instance's subdomains of the DC coefficient
template <typename T>
__device__ inline T instance_shift(const StepArgs& sa, const InstDev& I) {
  if (!I.pin) return T(0);
  const T* dc = (const T*)sa.dc;
  T s = T(0);
  for (int q = 0; q < I.nsub; ++q) s += dc[I.first_sub + q];
  return s / T(I.nsub);
}

// trapezoid weight (without prod h) and live flag of a node
__device__ inline void node_weight(const SubDev& S, int i0, int i1, int i2, double& w, bool& live) {
  w = 1.0;
  live = true;
  const int idx[3] = {i0, i1, i2};
  for (int k = 0; k < S.dim; ++k) {
    if (idx[k] == 0 || idx[k] == S.n[k] - 1) w *= 0.5;
    if (is_artificial(S.art, k, idx[k], S.n[k])) live = false;
  }
}

// ------------------------------------------------------------------------------------------
// forward Euler update (gamma = 0): phi += dt F on live nodes, residual partials
// ------------------------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void euler_kernel(const int4* __restrict__ tiles, int ntiles,
                                                    int part_base, StepArgs sa) {
  __shared__ double red[4];
  if ((int)blockIdx.x >= ntiles) return;
  const int4 tl = tiles[blockIdx.x];
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
    node_weight(S, i0, i1, i2, w, live);
    if (live) {
      const long v = (long)row * C + col;
      T* phi = (T*)S.phi;
      const T u = T(I.dt) * ((const T*)S.F)[v];
      phi[v] += u;
      acc = w * (double)u * (double)u;
      if (!finite_(u)) atomicOr(&sa.status[S.inst], ST_NONFINITE);
    }
  }
  double hs = S.h[0] * S.h[1] * (d == 3 ? S.h[2] : 1.0);
  double tot = block_sum256(acc, red);
  if (threadIdx.x == 0) sa.partials[part_base + blockIdx.x] = tot * hs;
}

// ------------------------------------------------------------------------------------------
// K3/K4/K5: batched mode products on the matrix cores, 64 x 64 output tile, 4 waves of 32 x 32
// ------------------------------------------------------------------------------------------

template <int KIND> struct GemmTraits;
template <> struct GemmTraits<PREC_F64> { typedef double T; enum { BK = 16 }; };
template <> struct GemmTraits<PREC_F32> { typedef float T; enum { BK = 16 }; };
template <> struct GemmTraits<PREC_SPLIT16> { typedef float T; enum { BK = 32 }; };

template <typename T>
__device__ inline void mfma4(T a, T b, typename std::conditional<sizeof(T) == 8, double4_t, float4_t>::type& c);

template <>
__device__ inline void mfma4<double>(double a, double b, double4_t& c) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <>
__device__ inline void mfma4<float>(float a, float b, float4_t& c) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int KIND>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmJob* __restrict__ jobs,
                                                   const int4* __restrict__ tiles, int ntiles,
                                                   int part_base, StepArgs sa) {
  typedef typename GemmTraits<KIND>::T T;
  typedef typename std::conditional<sizeof(T) == 8, double4_t, float4_t>::type acc_t;
  constexpr int BK = GemmTraits<KIND>::BK;
  __shared__ double red[4];
  if ((int)blockIdx.x >= ntiles) return;
  const int4 tl = tiles[blockIdx.x];
  const GemmJob& J = jobs[tl.x];
  const int M = J.M, N = J.N, K = J.K;
  const int m0 = tl.y, n0 = tl.z, b = tl.w;
  const T* __restrict__ P = (const T*)J.P + (long)b * J.sP;
  const T* __restrict__ Q = (const T*)J.Q + (long)b * J.sQ;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, lg = lane >> 4;

  acc_t acc[2][2];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) acc[r][c] = acc_t{0, 0, 0, 0};

  if constexpr (KIND != PREC_SPLIT16) {
    __shared__ T Ps[64][BK + 1];
    __shared__ T Qs[BK][64 + 16];
    const int prow = tid >> 2, pk = (tid & 3) * 4;
    const int qk = tid >> 4, qn = (tid & 15) * 4;
    for (int k0 = 0; k0 < K; k0 += BK) {
      {
        const int m = m0 + prow;
        for (int j = 0; j < 4; ++j) {
          const int k = k0 + pk + j;
          Ps[prow][pk + j] = (m < M && k < K) ? P[(long)m * J.ldp + k] : T(0);
        }
        const int k = k0 + qk;
        for (int j = 0; j < 4; ++j) {
          const int n = n0 + qn + j;
          Qs[qk][qn + j] = (k < K && n < N) ? Q[(long)k * J.ldq + n] : T(0);
        }
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        T a[2], bv[2];
        for (int r = 0; r < 2; ++r) a[r] = Ps[wm * 32 + r * 16 + l16][kk * 4 + lg];
        for (int c = 0; c < 2; ++c) bv[c] = Qs[kk * 4 + lg][wn * 32 + c * 16 + l16];
        for (int r = 0; r < 2; ++r)
          for (int c = 0; c < 2; ++c) mfma4<T>(a[r], bv[c], acc[r][c]);
      }
      __syncthreads();
    }
  } else {
    // fp16 hi + lo split of both operands; three products per k block, FP32 accumulation
    __shared__ _Float16 Ph[64][BK + 8], Pl[64][BK + 8];
    __shared__ _Float16 Qh[64][BK + 8], Ql[64][BK + 8];  // transposed: [n][k]
    const int prow = tid >> 2, pk = (tid & 3) * 8;
    const int qk = tid >> 3, qn = (tid & 7) * 8;
    for (int k0 = 0; k0 < K; k0 += BK) {
      {
        const int m = m0 + prow;
        for (int j = 0; j < 8; ++j) {
          const int k = k0 + pk + j;
          const float x = (m < M && k < K) ? P[(long)m * J.ldp + k] : 0.f;
          const _Float16 hi = (_Float16)x;
          Ph[prow][pk + j] = hi;
          Pl[prow][pk + j] = (_Float16)(x - (float)hi);
        }
        const int k = k0 + qk;
        for (int j = 0; j < 8; ++j) {
          const int n = n0 + qn + j;
          const float x = (k < K && n < N) ? Q[(long)k * J.ldq + n] : 0.f;
          const _Float16 hi = (_Float16)x;
          Qh[qn + j][qk] = hi;
          Ql[qn + j][qk] = (_Float16)(x - (float)hi);
        }
      }
      __syncthreads();
      half8_t ah[2], al[2], bh[2], bl[2];
      for (int r = 0; r < 2; ++r) {
        ah[r] = *(const half8_t*)&Ph[wm * 32 + r * 16 + l16][lg * 8];
        al[r] = *(const half8_t*)&Pl[wm * 32 + r * 16 + l16][lg * 8];
      }
      for (int c = 0; c < 2; ++c) {
        bh[c] = *(const half8_t*)&Qh[wn * 32 + c * 16 + l16][lg * 8];
        bl[c] = *(const half8_t*)&Ql[wn * 32 + c * 16 + l16][lg * 8];
      }
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[r], bh[c], acc[r][c], 0, 0, 0);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[r], bl[c], acc[r][c], 0, 0, 0);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[r], bh[c], acc[r][c], 0, 0, 0);
        }
      __syncthreads();
    }
  }

  // ---------------- epilogue ----------------
  // row of accumulator register q within a 16 x 16 block: the f64 product interleaves rows
  // (row = lane/16 + 4 q), the f32-accumulating products keep them together (4 lane/16 + q)
  auto crow = [](int g, int q) { return KIND == PREC_F64 ? g + 4 * q : 4 * g + q; };
  const T us = T(J.unscale);
  T* __restrict__ Cp = (T*)J.C + (long)b * J.sC;
  const int epi = J.epi;
  if (epi == EPI_NONE) {
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c)
        for (int q = 0; q < 4; ++q) {
          const int m = m0 + wm * 32 + r * 16 + crow(lg, q);
          const int n = n0 + wn * 32 + c * 16 + l16;
          if (m < M && n < N) Cp[(long)m * J.ldc + n] = acc[r][c][q] * us;
        }
    return;
  }
  const SubDev& S = sa.subs[J.sub];
  if (epi == EPI_SCALE) {
    // left product along axis 0 completes the forward transform: m = k0, n = (k1[, k2])
    const T* s0 = (const T*)S.sig[0];
    const T* s1 = (const T*)S.sig[1];
    const T* s2 = (const T*)S.sig[2];
    const T g0 = T(S.gh2[0]), g1 = T(S.gh2[1]), g2 = T(S.gh2[2]);
    const int n2 = S.n[2];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c)
        for (int q = 0; q < 4; ++q) {
          const int m = m0 + wm * 32 + r * 16 + crow(lg, q);
          const int n = n0 + wn * 32 + c * 16 + l16;
          if (m < M && n < N) {
            const T val = acc[r][c][q] * us;
            T den;
            if (S.dim == 2) {
              den = T(1) + g0 * s0[m] + g1 * s1[n];
            } else {
              const int k1 = n / n2, k2 = n - (n / n2) * n2;
              den = T(1) + g0 * s0[m] + g1 * s1[k1] + g2 * s2[k2];
            }
            Cp[(long)m * J.ldc + n] = val / den;
            if (m == 0 && n == 0) ((T*)sa.dc)[J.sub] = val;
          }
        }
    return;
  }
  // EPI_UPDATE: right product along the last axis completes the inverse transform:
  // m = flat index over the leading axes, n = last-axis index; C is phi.
  const InstDev& I = sa.insts[S.inst];
  const T shift = instance_shift<T>(sa, I);
  const T dt = T(I.dt);
  double part = 0.0;
  bool bad = false;
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c)
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm * 32 + r * 16 + crow(lg, q);
        const int n = n0 + wn * 32 + c * 16 + l16;
        if (m < M && n < N) {
          const T val = acc[r][c][q] * us;
          int i0, i1, i2;
          if (S.dim == 2) {
            i0 = m; i1 = n; i2 = 0;
          } else {
            i0 = m / S.n[1]; i1 = m - i0 * S.n[1]; i2 = n;
          }
          double w;
          bool live;
          node_weight(S, i0, i1, i2, w, live);
          if (live) {
            const T u = dt * val;
            Cp[(long)m * J.ldc + n] += dt * (val - shift);
            part += w * (double)u * (double)u;
            bad |= !finite_(u);
          }
        }
      }
  if (bad) atomicOr(&sa.status[S.inst], ST_NONFINITE);
  const double hs = S.h[0] * S.h[1] * (S.dim == 3 ? S.h[2] : 1.0);
  const double tot = block_sum256(part, red);
  if (tid == 0) {
    sa.partials[part_base + blockIdx.x] = tot * hs;
    if (I.pin && J.sub == I.first_sub && m0 == 0 && n0 == 0 && b == 0)
      sa.shift_acc[S.inst] += (double)dt * (double)shift;
  }
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
  ((T*)subs[e.x].phi)[e.y] = ((const T*)subs[e.z].phi)[e.w];
}

// ------------------------------------------------------------------------------------------
// K8: residual per instance = max over subdomains of sqrt(sum of partials) (fixed order)
// ------------------------------------------------------------------------------------------

__global__ void resid_kernel(const SubDev* __restrict__ subs, const InstDev* __restrict__ insts,
                             int ninst, const double* __restrict__ partials, double* out) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < ninst; q += gridDim.x * blockDim.x) {
    const InstDev& I = insts[q];
    double best = 0.0;
    for (int s = I.first_sub; s < I.first_sub + I.nsub; ++s) {
      double acc = 0.0;
      for (int p = 0; p < subs[s].nparts; ++p) acc += partials[subs[s].part0 + p];
      best = fmax(best, acc);
    }
    out[q] = sqrt(best);
  }
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
  const long v = blockIdx.x * 256L + threadIdx.x;
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
  if (threadIdx.x == 0) minpart[blockIdx.x] = mn;
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

hipError_t launch_stencil(int prec, const int4* tiles, int ntiles, const StepArgs& sa, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (prec == PREC_F64)
    hipLaunchKernelGGL(stencil_kernel<double>, dim3(ntiles), dim3(256), 0, s, tiles, ntiles, sa);
  else
    hipLaunchKernelGGL(stencil_kernel<float>, dim3(ntiles), dim3(256), 0, s, tiles, ntiles, sa);
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

hipError_t launch_gemm(int prec, const GemmJob* jobs, const int4* tiles, int ntiles, int part_base,
                       const StepArgs& sa, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (prec == PREC_F64)
    hipLaunchKernelGGL(gemm_kernel<PREC_F64>, dim3(ntiles), dim3(256), 0, s, jobs, tiles, ntiles, part_base, sa);
  else if (prec == PREC_F32)
    hipLaunchKernelGGL(gemm_kernel<PREC_F32>, dim3(ntiles), dim3(256), 0, s, jobs, tiles, ntiles, part_base, sa);
  else
    hipLaunchKernelGGL(gemm_kernel<PREC_SPLIT16>, dim3(ntiles), dim3(256), 0, s, jobs, tiles, ntiles, part_base, sa);
  return hipGetLastError();
}

hipError_t launch_resid(const SubDev* subs, const InstDev* insts, int ninst, const double* partials,
                        double* out, hipStream_t s) {
  if (ninst <= 0) return hipSuccess;
  hipLaunchKernelGGL(resid_kernel, dim3(nblk(ninst, 256)), dim3(256), 0, s, subs, insts, ninst, partials, out);
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

hipError_t launch_min_reduce(const double* x, long n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(min_reduce_kernel, dim3(1), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

}  // namespace pma
