// Host runtime of the DD-PMA library: device arena, DCT bases, theta, partition, per-request
// plans, the batched / plain step executors, the serving loop and the C ABI of include/pma.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pma.h"
#include "pma_device.h"

namespace pma {

// kernels.hip
hipError_t launch_transmit(int prec, const SubDev* subs, const int4* ent, int count, hipStream_t s);
hipError_t scratch_init(int device);
void* scratch_ptr(int device);
int persist_capacity(int prec, size_t dyn, int* static_lds);
hipError_t launch_step2_persist(int prec, int grid, size_t dyn, const PersistArgs& pa, const StepArgs& sa,
                                hipStream_t s);
hipError_t launch_stencil(int prec, int dim, const int4* tiles, int ntiles, const StepArgs& sa, hipStream_t s);
hipError_t launch_stencil_fwd2(int prec, const int4* tiles, int ntiles, int lneed, const StepArgs& sa, hipStream_t s);
int fused_lds_bytes(int prec, int ld, int ldb, int n, bool basis);
hipError_t launch_euler(int prec, const int4* tiles, int ntiles, int part_base, const StepArgs& sa,
                        hipStream_t s);
hipError_t launch_fwd_last(int prec, const int4* tiles, int ntiles, int maxld, const StepArgs& sa, hipStream_t s);
hipError_t launch_inv_last(int prec, const int4* tiles, int ntiles, int maxld, int part_base, int eight_max,
                           const StepArgs& sa, hipStream_t s);
hipError_t launch_strip4(int prec, bool pair, const int4* tiles, int ntiles, int maxld, int axis, int inv,
                         int src_sel, const StepArgs& sa, hipStream_t s);
hipError_t launch_strip(int prec, bool pair, const int4* tiles, int ntiles, int maxld, int lneed, int axis, int inv,
                        int src_sel, int eight_max, const StepArgs& sa, hipStream_t s);
hipError_t enable_large_lds();
hipError_t launch_resid(const SubDev* subs, const InstDev* insts, int ninst, const double* partials,
                        double* out, hipStream_t s);
hipError_t launch_phi_from_psi(int prec, const SubDev& S, const double* psi, int global_layout, int g1,
                               int g2, hipStream_t s);
hipError_t launch_psi_from_phi(int prec, const SubDev& S, double* psi, const double* shift_acc,
                               hipStream_t s);
struct GlueArgs {
  const SubDev* subs;
  int first_sub;
  int dim;
  int parts[3];
  int n[3];
  const int* own[3];
  double a[3], h[3];
  double* mesh;
  double* psi;
  const double* shift_acc;
  int inst;
  double* minpart;
};
long glue_blocks(long nodes);
hipError_t launch_glue(int prec, const GlueArgs& g, hipStream_t s);
long cell_blocks(int dim, const int* n);
hipError_t launch_cells(const double* mesh, int dim, const int* n, double* minpart, hipStream_t s);
hipError_t launch_min_reduce(const double* x, long n, double* out, hipStream_t s);
hipError_t launch_quality(const double* mesh, int dim, const int* n, const double* h, const MonP<double>& mp,
                          double vol, double theta, double* part, double* out, hipStream_t s);

// ------------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------------

static thread_local std::string g_err = "no error";

struct Err {
  int code;
};

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) throw Err{fail(PMA_E_HIP, "%s failed: %s (%s:%d)", #expr,        \
                                         hipGetErrorString(e_), __FILE__, __LINE__)};      \
  } while (0)

static void thr(int code, const char* msg) { throw Err{fail(code, "%s", msg)}; }

// ------------------------------------------------------------------------------------------
// device arena: one allocation of the whole budget, first-fit sub-allocation
// ------------------------------------------------------------------------------------------

class Arena {
 public:
  static constexpr size_t kAlign = 256;
  bool ready() const { return base_ != nullptr; }
  void init(char* base, size_t size) {
    base_ = base;
    size_ = size;
    free_.clear();
    free_[0] = size;
    used_ = 0;
  }
  char* base() const { return base_; }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  // returns nullptr when no hole is large enough
  void* alloc(size_t bytes) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    if (bytes == 0) bytes = kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        size_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > bytes) free_[off + bytes] = sz - bytes;
        live_[off] = bytes;
        used_ += bytes;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(void* p) {
    if (!p) return;
    size_t off = (char*)p - base_;
    auto it = live_.find(off);
    if (it == live_.end()) return;
    size_t sz = it->second;
    live_.erase(it);
    used_ -= sz;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + sz == nx->first) {
      sz += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == off) {
        pv->second += sz;
        return;
      }
    }
    free_[off] = sz;
  }
  static size_t round(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_, live_;
};

// ------------------------------------------------------------------------------------------
// DCT-I bases.  For an axis with nodes j = 0..N (n = N + 1):
//   forward A_kj = (2/N) w_k w_j cos(pi k j / N),  inverse B_jk = cos(pi k j / N),
//   w_0 = w_N = 1/2, else 1;  B A = I  and  B e_k is an eigenvector of the ghost-reflection
//   Neumann second difference with eigenvalue -(4/h^2) sin^2(pi k / (2N)).
// Both matrices are symmetric, so a mode product along any axis is an "NN" product.
// ------------------------------------------------------------------------------------------

// DCT-I matrices of one axis length n in one precision, kept in the arena while requests use
// them (refs) and afterwards as a cache, evicted least recently used when the arena is full
struct Basis {
  int n = 0, prec = 0, rows = 0, ld = 0;  // rows = round_up(n, 16), ld = round_up(n, 32)
  int ldb = 0;                             // row stride: ld plus 16 bytes
  int refs = 0;
  uint64_t last_use = 0;
  char* mem = nullptr;
  size_t bytes = 0;
  const void *fwd = nullptr, *fwdl = nullptr, *inv = nullptr, *invl = nullptr, *sig = nullptr;
  float fwd_unscale = 1.0f;
};

static double cos_pi_frac(long p, long q) {
  // cos(pi p / q) with p reduced mod 2q exactly
  long r = p % (2 * q);
  return std::cos(M_PI * (double)r / (double)q);
}

static void basis_host(int n, std::vector<double>& A, std::vector<double>& B, std::vector<double>& sig) {
  const int N = n - 1;
  A.assign((size_t)n * n, 0.0);
  B.assign((size_t)n * n, 0.0);
  sig.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    const double wk = (k == 0 || k == N) ? 0.5 : 1.0;
    for (int j = 0; j < n; ++j) {
      const double wj = (j == 0 || j == N) ? 0.5 : 1.0;
      const double c = cos_pi_frac((long)k * j, N);
      A[(size_t)k * n + j] = (2.0 / N) * wk * wj * c;
      B[(size_t)j * n + k] = c;
    }
    const double s = std::sin(M_PI * k / (2.0 * N));
    sig[k] = 4.0 * s * s;
  }
}

// ------------------------------------------------------------------------------------------
// theta = int_box rho (FP64)
// ------------------------------------------------------------------------------------------

static double sech2_h(double z) {
  double e = std::exp(-2.0 * std::fabs(z));
  return 4.0 * e / ((1.0 + e) * (1.0 + e));
}

// gradient of the solution u behind an arc-length monitor (Cartesian form: with
// P = d_0 cos(w r^2) + d_1 sin(w r^2) = r cos(t - w r^2) and Q = d_1 cos(w r^2) - d_0 sin(w r^2),
// the spiral's q = k P^2 has grad q = 2 k P ((cos, sin)(w r^2) + 2 w Q d))
static void grad_u_host(const pma_monitor& m, int dim, const double* x, double* g) {
  g[0] = g[1] = g[2] = 0.0;
  if (m.kind == PMA_MON_ARCLEN_FRONT) {
    // u(1 - u) = sech^2(s / 2) / 4, s = (x_0 + x_1 - r0) / (2 eps)
    const double du = -0.25 * sech2_h((x[0] + x[1] - m.r0) / (4.0 * m.k)) / (2.0 * m.k);
    g[0] = g[1] = du;
  } else if (m.kind == PMA_MON_ARCLEN_SPIRAL) {
    const double d0 = x[0] - m.c[0], d1 = x[1] - m.c[1], r2 = d0 * d0 + d1 * d1;
    const double C = std::cos(m.twist * r2), S = std::sin(m.twist * r2);
    const double P = d0 * C + d1 * S, Q = d1 * C - d0 * S, q = m.k * P * P;
    const double f = -m.amp * 2.0 * m.k * P / ((1.0 + q) * (1.0 + q));
    g[0] = f * (C + 2.0 * m.twist * Q * d0);
    g[1] = f * (S + 2.0 * m.twist * Q * d1);
  } else if (m.kind == PMA_MON_ARCLEN_SPHERES) {
    for (int b = 0; b < m.nbumps; ++b) {
      double d[3] = {0, 0, 0}, r2 = 0.0;
      for (int k = 0; k < dim; ++k) {
        d[k] = x[k] - m.bc[b][k];
        r2 += d[k] * d[k];
      }
      const double s = 2.0 * m.k * sech2_h(m.k * (r2 - m.r0 * m.r0));
      for (int k = 0; k < dim; ++k) g[k] += s * d[k];
    }
  }
}

static double rho_host(const pma_monitor& m, int dim, const double* x) {
  switch (m.kind) {
    case PMA_MON_CONST:
      return m.amp;
    case PMA_MON_SECH2_RADIAL: {
      double r2 = 0;
      for (int k = 0; k < dim; ++k) r2 += (x[k] - m.c[k]) * (x[k] - m.c[k]);
      return 1.0 + m.amp * sech2_h(m.k * (r2 - m.r0 * m.r0));
    }
    case PMA_MON_SECH2_SINE:
      return 1.0 + m.amp * sech2_h(m.k * (x[1] - m.c[1] - m.r0 * std::sin(2.0 * M_PI * x[0])));
    case PMA_MON_GAUSS_SUM: {
      double s = 1.0;
      for (int b = 0; b < m.nbumps; ++b) {
        double r2 = 0;
        for (int k = 0; k < dim; ++k) r2 += (x[k] - m.bc[b][k]) * (x[k] - m.bc[b][k]);
        s += m.bamp[b] * std::exp(-r2 / (2.0 * m.bw[b] * m.bw[b]));
      }
      return s;
    }
    case PMA_MON_SEPARABLE_SECH2: {
      double p = 1.0;
      for (int k = 0; k < dim; ++k) p *= 1.0 + m.amp_axes[k] * sech2_h(m.k_axes[k] * (x[k] - m.c[k]));
      return p;
    }
    case PMA_MON_ARCLEN_FRONT:
    case PMA_MON_ARCLEN_SPIRAL:
    case PMA_MON_ARCLEN_SPHERES: {
      double g[3];
      grad_u_host(m, dim, x, g);
      double g2 = 0.0;
      for (int k = 0; k < dim; ++k) g2 += g[k] * g[k];
      return std::sqrt(1.0 + g2);
    }
  }
  return NAN;
}

static void gl8(double a, double b, int panels, std::vector<double>& x, std::vector<double>& w) {
  static const double t[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                              -0.1834346424956498, 0.1834346424956498,  0.5255324099163290,
                              0.7966664774136267,  0.9602898564975363};
  static const double wt[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                               0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                               0.2223810344533745, 0.1012285362903763};
  x.clear();
  w.clear();
  const double hp = (b - a) / panels;
  for (int p = 0; p < panels; ++p) {
    const double mid = a + (p + 0.5) * hp, half = 0.5 * hp;
    for (int q = 0; q < 8; ++q) {
      x.push_back(mid + half * t[q]);
      w.push_back(half * wt[q]);
    }
  }
}

// int over [lo, hi] of rho - 1 by tensor Gauss-Legendre (`panels` panels of 8 nodes per axis),
// the first axis split over host threads
static double excess_integral(const pma_monitor& m, int d, const double* lo, const double* hi, int panels) {
  std::vector<double> xs[3], ws[3];
  for (int k = 0; k < d; ++k) gl8(lo[k], hi[k], panels, xs[k], ws[k]);
  const size_t n0 = xs[0].size();
  const int nth = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  std::vector<double> part(nth, 0.0);
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t]() {
      double acc = 0.0;
      double x[3] = {0, 0, 0};
      for (size_t i = t; i < n0; i += nth) {
        x[0] = xs[0][i];
        double a1 = 0.0;
        for (size_t j = 0; j < xs[1].size(); ++j) {
          x[1] = xs[1][j];
          if (d == 2) {
            a1 += ws[1][j] * (rho_host(m, 2, x) - 1.0);
          } else {
            double a2 = 0.0;
            for (size_t k = 0; k < xs[2].size(); ++k) {
              x[2] = xs[2][k];
              a2 += ws[2][k] * (rho_host(m, 3, x) - 1.0);
            }
            a1 += ws[1][j] * a2;
          }
        }
        acc += ws[0][i] * a1;
      }
      part[t] = acc;
    });
  for (auto& t : th) t.join();
  double s = 0.0;
  for (double p : part) s += p;
  return s;
}

static double theta_host(const pma_grid& g, const pma_monitor& m) {
  const int d = g.dim;
  double vol = 1.0;
  for (int k = 0; k < d; ++k) vol *= g.hi[k] - g.lo[k];
  switch (m.kind) {
    case PMA_MON_CONST:
      return m.amp * vol;
    case PMA_MON_GAUSS_SUM: {
      double tot = vol;
      for (int b = 0; b < m.nbumps; ++b) {
        double p = m.bamp[b];
        const double s = std::sqrt(2.0) * m.bw[b];
        for (int k = 0; k < d; ++k)
          p *= m.bw[b] * std::sqrt(M_PI / 2.0) *
               (std::erf((g.hi[k] - m.bc[b][k]) / s) - std::erf((g.lo[k] - m.bc[b][k]) / s));
        tot += p;
      }
      return tot;
    }
    case PMA_MON_SEPARABLE_SECH2: {
      double p = 1.0;
      for (int k = 0; k < d; ++k)
        p *= (g.hi[k] - g.lo[k]) + (m.amp_axes[k] / m.k_axes[k]) *
                                       (std::tanh(m.k_axes[k] * (g.hi[k] - m.c[k])) -
                                        std::tanh(m.k_axes[k] * (g.lo[k] - m.c[k])));
      return p;
    }
    case PMA_MON_SECH2_SINE: {
      // the x_1 integral is elementary: int sech^2(k(y - c - s)) dy = tanh(k(y - c - s)) / k
      std::vector<double> x, w;
      const double L0 = g.hi[0] - g.lo[0];
      const int panels = (int)std::ceil(4.0 * m.k * (1.0 + 2.0 * M_PI * std::fabs(m.r0)) * L0 / M_PI) + 16;
      gl8(g.lo[0], g.hi[0], panels, x, w);
      double acc = 0.0;
      for (size_t q = 0; q < x.size(); ++q) {
        const double s = m.c[1] + m.r0 * std::sin(2.0 * M_PI * x[q]);
        acc += w[q] * (std::tanh(m.k * (g.hi[1] - s)) - std::tanh(m.k * (g.lo[1] - s))) / m.k;
      }
      double rest = 1.0;
      for (int k = 2; k < d; ++k) rest *= g.hi[k] - g.lo[k];
      return vol + m.amp * acc * rest;
    }
    case PMA_MON_SECH2_RADIAL: {
      // tensor Gauss-Legendre; panels short against 1/(k r0), the width of the shell
      double L = 0;
      for (int k = 0; k < d; ++k) L = std::max(L, g.hi[k] - g.lo[k]);
      const int panels = (int)std::ceil(3.0 * m.k * std::max(m.r0, 0.1) * L) + 8;
      return vol + excess_integral(m, d, g.lo, g.hi, panels);
    }
    case PMA_MON_ARCLEN_FRONT: {
      // rho depends on s = x_0 + x_1 only: int rho = int rho(s) len(s) ds with len(s) the length
      // of the segment x_0 + x_1 = s inside the box; Gauss-Legendre between the kinks of len(s)
      double br[5] = {g.lo[0] + g.lo[1], g.lo[0] + g.hi[1], g.hi[0] + g.lo[1], g.hi[0] + g.hi[1],
                      std::min(std::max(m.r0, g.lo[0] + g.lo[1]), g.hi[0] + g.hi[1])};
      std::sort(br, br + 5);
      double tot = 0.0;
      std::vector<double> xs, ws;
      for (int q = 0; q < 4; ++q) {
        if (!(br[q + 1] > br[q])) continue;
        const int panels = (int)std::ceil(2.0 * (br[q + 1] - br[q]) / (M_PI * m.k)) + 16;
        gl8(br[q], br[q + 1], panels, xs, ws);
        for (size_t i = 0; i < xs.size(); ++i) {
          const double sv = xs[i];
          const double len = std::max(0.0, std::min(g.hi[0], sv - g.lo[1]) - std::max(g.lo[0], sv - g.hi[1]));
          const double x[3] = {sv - 0.5 * m.r0, 0.5 * m.r0, 0.0};
          tot += ws[i] * rho_host(m, 2, x) * len;
        }
      }
      return tot;
    }
    case PMA_MON_ARCLEN_SPIRAL: {
      // ridges of u narrow to ~ 1 / (sqrt(k) 2 twist r^2) far from the centre
      double rmax = 0.0;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          rmax = std::max(rmax, std::hypot((a ? g.hi[0] : g.lo[0]) - m.c[0], (b ? g.hi[1] : g.lo[1]) - m.c[1]));
      const double scale = 1.0 / (std::sqrt(std::max(m.k, 1.0)) * 2.0 * std::max(m.twist, 1.0) * rmax * rmax);
      const double L = std::max(g.hi[0] - g.lo[0], g.hi[1] - g.lo[1]);
      const int panels = std::min(2048, (int)std::ceil(2.0 * L / scale) + 16);
      return vol + excess_integral(m, d, g.lo, g.hi, panels);
    }
    case PMA_MON_ARCLEN_SPHERES: {
      // rho - 1 < 1e-30 farther than R from every centre, R^2 = r0^2 + 40 / k
      const double R = std::sqrt(m.r0 * m.r0 + 40.0 / std::max(m.k, 1e-300));
      if (m.nbumps == 1) {
        bool inside = true;
        for (int k = 0; k < d; ++k) inside &= g.lo[k] <= m.bc[0][k] - R && m.bc[0][k] + R <= g.hi[k];
        if (inside) {  // radial integral: vol + |S^{d-1}| int_0^R (rho(r) - 1) r^{d-1} dr
          std::vector<double> xs, ws;
          const int panels = (int)std::ceil(8.0 * m.k * std::max(m.r0, 0.05) * R) + 64;
          double tot = 0.0;
          const double br[3] = {0.0, std::min(m.r0, R), R};
          for (int q = 0; q < 2; ++q) {
            if (!(br[q + 1] > br[q])) continue;
            gl8(br[q], br[q + 1], panels, xs, ws);
            for (size_t i = 0; i < xs.size(); ++i) {
              double x[3] = {m.bc[0][0] + xs[i], m.bc[0][1], m.bc[0][2]};
              tot += ws[i] * (rho_host(m, d, x) - 1.0) * (d == 2 ? xs[i] : xs[i] * xs[i]);
            }
          }
          return vol + (d == 2 ? 2.0 * M_PI : 4.0 * M_PI) * tot;
        }
      }
      double lo[3], hi[3];
      for (int k = 0; k < d; ++k) {
        lo[k] = hi[k] = m.bc[0][k];
        for (int b = 0; b < m.nbumps; ++b) {
          lo[k] = std::min(lo[k], m.bc[b][k] - R);
          hi[k] = std::max(hi[k], m.bc[b][k] + R);
        }
        lo[k] = std::max(lo[k], g.lo[k]);
        hi[k] = std::min(hi[k], g.hi[k]);
        if (!(hi[k] > lo[k])) return vol;
      }
      double L = 0;
      for (int k = 0; k < d; ++k) L = std::max(L, hi[k] - lo[k]);
      const double scale = M_PI / (4.0 * m.k * std::max(m.r0, 0.05));
      const int panels = std::min(d == 2 ? 2048 : 72, (int)std::ceil(2.0 * L / scale) + 8);
      return vol + excess_integral(m, d, lo, hi, panels);
    }
  }
  return NAN;
}

// ------------------------------------------------------------------------------------------
// partition (Sec. 3): cores c_m = floor(m N / M), subdomain m spans
// [max(0, c_m - floor(ov/2)), min(N, c_{m+1} + ceil(ov/2))], owner = part whose core holds the
// node (the last node belongs to the last part)
// ------------------------------------------------------------------------------------------

// largest subdomain extent per axis: a 16-row tile of the widest axis (1056 padded entries) fits a
// workgroup's LDS in FP64; axes beyond 576 padded entries take the long-axis strip kernel
static constexpr int kMaxAxisNodes = 1025;

struct AxisSplit {
  std::vector<int> cores;            // M + 1
  std::vector<std::pair<int, int>> ranges;
  std::vector<int> owner;            // per node
};

static AxisSplit split_axis(int nnodes, int M, int ov) {
  AxisSplit a;
  const int N = nnodes - 1;
  for (int m = 0; m <= M; ++m) a.cores.push_back((int)(((long)m * N) / M));
  for (int m = 0; m < M; ++m)
    a.ranges.push_back({std::max(0, a.cores[m] - ov / 2), std::min(N, a.cores[m + 1] + (ov + 1) / 2)});
  a.owner.resize(nnodes);
  for (int v = 0, m = 0; v < nnodes; ++v) {
    while (m < M - 1 && v >= a.cores[m + 1]) ++m;
    a.owner[v] = m;
  }
  return a;
}

static void validate_grid(const pma_grid& g) {
  if (g.dim != 2 && g.dim != 3) thr(PMA_E_INVAL, "dim must be 2 or 3");
  for (int k = 0; k < g.dim; ++k) {
    if (g.n[k] < 5) thr(PMA_E_INVAL, "need at least 5 nodes per axis");
    if (!(g.hi[k] > g.lo[k])) thr(PMA_E_INVAL, "box must have hi > lo");
  }
}

static void validate_monitor(const pma_monitor& m, int dim) {
  if (m.kind < PMA_MON_CONST || m.kind > PMA_MON_ARCLEN_SPHERES) thr(PMA_E_INVAL, "unknown monitor kind");
  if (m.kind == PMA_MON_GAUSS_SUM && (m.nbumps < 1 || m.nbumps > 4)) thr(PMA_E_INVAL, "nbumps must be 1..4");
  if (m.kind == PMA_MON_ARCLEN_SPHERES && (m.nbumps < 1 || m.nbumps > PMA_MAX_BUMPS))
    thr(PMA_E_INVAL, "nbumps must be 1..9");
  if (m.kind == PMA_MON_SECH2_SINE && dim < 2) thr(PMA_E_INVAL, "sine monitor needs dim >= 2");
  if ((m.kind == PMA_MON_ARCLEN_FRONT || m.kind == PMA_MON_ARCLEN_SPIRAL) && dim != 2)
    thr(PMA_E_INVAL, "the front and spiral monitors are two-dimensional");
  if (m.kind == PMA_MON_ARCLEN_FRONT && !(m.k > 0)) thr(PMA_E_INVAL, "front monitor needs k = eps > 0");
  if ((m.kind == PMA_MON_ARCLEN_SPIRAL || m.kind == PMA_MON_ARCLEN_SPHERES) && !(m.k >= 0))
    thr(PMA_E_INVAL, "monitor needs k >= 0");
  if (m.kind == PMA_MON_CONST && !(m.amp > 0)) thr(PMA_E_INVAL, "constant monitor must be positive");
}

static void validate_time(const pma_time& t) {
  if (!(t.dt > 0) || !(t.gamma >= 0) || t.max_steps < 0 || !(t.tol >= 0)) thr(PMA_E_INVAL, "bad time parameters");
  if (t.precision < PMA_FP64 || t.precision > PMA_FP32_SPLIT16) thr(PMA_E_INVAL, "bad precision");
  if (t.exec != PMA_EXEC_BATCHED && t.exec != PMA_EXEC_PLAIN) thr(PMA_E_INVAL, "bad exec form");
}

struct SubHost {
  int lo[3] = {0, 0, 0}, n[3] = {1, 1, 1};
  int art = 0;
};

static void partition_host(const pma_grid& g, const pma_dd* dd, std::vector<SubHost>& subs,
                           int parts[3], std::vector<int> own[3]) {
  validate_grid(g);
  int P[3] = {1, 1, 1}, OV[3] = {0, 0, 0};
  if (dd) {
    if (dd->mode != PMA_DD_PARALLEL && dd->mode != PMA_DD_ALTERNATING && dd->mode != PMA_DD_COLOURED)
      thr(PMA_E_INVAL, "unknown decomposition coupling mode");
    for (int k = 0; k < g.dim; ++k) {
      P[k] = dd->parts[k];
      OV[k] = dd->overlap_cells[k];
      if (P[k] < 1) thr(PMA_E_INVAL, "parts must be >= 1");
      if (P[k] > 1 && OV[k] < 2) thr(PMA_E_INVAL, "overlap must be >= 2 cells on a split axis");
    }
  }
  AxisSplit ax[3];
  for (int k = 0; k < 3; ++k) {
    if (k < g.dim) ax[k] = split_axis(g.n[k], P[k], OV[k]);
    else {
      ax[k].cores = {0, 0};
      ax[k].ranges = {{0, 0}};
      ax[k].owner = {0};
    }
    parts[k] = k < g.dim ? P[k] : 1;
    own[k] = ax[k].owner;
  }
  subs.clear();
  for (int p0 = 0; p0 < parts[0]; ++p0)
    for (int p1 = 0; p1 < parts[1]; ++p1)
      for (int p2 = 0; p2 < parts[2]; ++p2) {
        SubHost s;
        const int pp[3] = {p0, p1, p2};
        for (int k = 0; k < g.dim; ++k) {
          auto r = ax[k].ranges[pp[k]];
          s.lo[k] = r.first;
          s.n[k] = r.second - r.first + 1;
          if (r.second - r.first < 4) thr(PMA_E_INVAL, "a subdomain has fewer than 4 cells on an axis");
          if (r.second - r.first + 1 > kMaxAxisNodes)
            thr(PMA_E_INVAL, "a subdomain axis has more than 1025 nodes: use more parts");
          if (r.first > 0) s.art |= 1 << (2 * k);
          if (r.second < g.n[k] - 1) s.art |= 1 << (2 * k + 1);
        }
        subs.push_back(s);
      }
  // every artificial node must lie strictly inside its owner's range (not on the owner's own
  // artificial faces), so transmission reads only computed values
  for (int k = 0; k < g.dim; ++k)
    for (int m = 0; m < parts[k]; ++m) {
      const auto r = ax[k].ranges[m];
      const int ends[2] = {r.first, r.second};
      for (int e = 0; e < 2; ++e) {
        const int v = ends[e];
        if (v == 0 || v == g.n[k] - 1) continue;
        const int o = ax[k].owner[v];
        const auto ro = ax[k].ranges[o];
        if (!(v > ro.first || ro.first == 0) || !(v < ro.second || ro.second == g.n[k] - 1) || o == m)
          thr(PMA_E_INVAL, "overlap too small for this split: a boundary node is not inside its owner");
      }
    }
}

// ------------------------------------------------------------------------------------------
// per-request plan and device state
// ------------------------------------------------------------------------------------------

struct Ctx;

struct Instance {
  // request
  pma_grid grid{};
  pma_dd dd{};
  pma_monitor mon{};
  pma_time tm{};
  int prec = 0;
  double theta = 0;
  bool whole = true;  // single domain
  // plan
  int dim = 2;
  int parts[3] = {1, 1, 1};
  std::vector<SubHost> subs;
  std::vector<int> own[3];
  std::vector<int4> trans;  // (dst local sub, dst elem, src local sub, src elem)
  std::vector<int> push_cnt;  // push entries per source subdomain (preconditioned DD requests)
  std::vector<int> trans_first;  // per dst sub, into trans (size nsub + 1)
  std::vector<int> level;        // sweep level per subdomain (all 0 in the parallel form)
  int nlevels = 1;
  bool alternating = false;
  // device memory
  char* block = nullptr;
  size_t bytes = 0;
  std::vector<void*> phi, F, T;
  int4* trans_dev = nullptr;     // the transmission list on the device (in the block)
  std::vector<int4*> push_dev;   // per subdomain, in the block (see SubDev::push)
  std::vector<int*> pfirst_dev;
  std::vector<int4> push_host;   // their sources, kept while the copies may be in flight
  std::vector<int> pfirst_host;
  int* own_dev[3] = {nullptr, nullptr, nullptr};
  double* mesh_dev = nullptr;
  double* psi_dev = nullptr;
  double* minpart = nullptr;
  long minpart_n = 0;
  double* stats_dev = nullptr;  // [min det, min cell, quality E_2, quality E_max]
  // progress
  int steps_done = 0;
  int status = PMA_OK;
  double resid = 0;
  // solve-subdomain mode (no glue)
  bool single_sub_mode = false;
  // serving
  uint64_t ticket = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  double arrival_s = 0;
  std::vector<double> mesh_host;
  std::vector<Basis*> bases_used;
  bool initialized = false;
  double shift_acc = 0;          // constant removed from phi so far (FP64)
  double min_det = 0, min_cell = 0;
  double stats_host[4] = {0, 0, 0, 0};
  const double* psi0_dev = nullptr;  // warm start (global layout, device)
  std::vector<double> psi0_host;     // served requests: the caller's Psi^0, copied at submit
  bool want_psi = false;             // served requests: keep the final Psi for the poll
  std::vector<double> psi_host;      // served requests: the final Psi
  std::string err;                   // served requests: why the request failed
  double* user_psi = nullptr;        // single-subdomain mode: caller's device buffer
  bool ext_mem = false;              // block and bases in caller-provided memory (the fixed
                                     // scratch), not in the arena; bases owned, not cached
  size_t elem() const { return prec == PMA_FP64 ? 8 : 4; }
  long gnodes() const { return (long)grid.n[0] * grid.n[1] * (dim == 3 ? grid.n[2] : 1); }
};

static long sub_nodes(const SubHost& s) { return (long)s.n[0] * s.n[1] * s.n[2]; }

static constexpr int kRows = 16, kCols = 64, kStrip = 16;  // mode-product tiles

// inverse-last tiles of a subdomain: kRows x kCols blocks of its [rows][last axis] view (rows =
// n0 in 2D, n0 n1 in 3D); nct = column blocks per row block
static int inv_tiles(const int n[3], int dim, int& nct) {
  const int R = dim == 2 ? n[0] : n[0] * n[1], C = n[dim - 1];
  nct = (C + kCols - 1) / kCols;
  return ((R + kRows - 1) / kRows) * nct;
}

static bool uses_push(const Instance& I) { return I.tm.gamma > 0 && !I.push_cnt.empty(); }

static void build_coupling(Instance& I);

static void build_plan(Instance& I) {
  I.dim = I.grid.dim;
  validate_monitor(I.mon, I.dim);
  validate_time(I.tm);
  I.prec = I.tm.precision;
  const pma_dd* ddp = nullptr;
  I.whole = true;
  for (int k = 0; k < I.dim; ++k)
    if (I.dd.parts[k] > 1) I.whole = false;
  if (!I.whole) ddp = &I.dd;
  partition_host(I.grid, ddp, I.subs, I.parts, I.own);
  I.theta = I.mon.theta > 0 ? I.mon.theta : theta_host(I.grid, I.mon);
  if (!(I.theta > 0) || !std::isfinite(I.theta)) thr(PMA_E_INVAL, "theta must be positive and finite");
  build_coupling(I);
}

// transmission lists and sweep levels of a partitioned instance
static void build_coupling(Instance& I) {
  // transmission lists: walk the artificial faces only; a node on several artificial faces is
  // listed once, under the first face (axis order, low side first) that holds it
  const int ns = (int)I.subs.size();
  I.trans.clear();
  I.trans_first.assign(ns + 1, 0);
  for (int s = 0; s < ns; ++s) {
    I.trans_first[s] = (int)I.trans.size();
    const SubHost& S = I.subs[s];
    if (S.art == 0) continue;
    for (int k = 0; k < I.dim; ++k)
      for (int e = 0; e < 2; ++e) {
        if (!(S.art >> (2 * k + e) & 1)) continue;
        const int fixed = e == 0 ? 0 : S.n[k] - 1;
        int lo[3] = {0, 0, 0}, hi[3] = {S.n[0], S.n[1], S.n[2]};
        lo[k] = fixed;
        hi[k] = fixed + 1;
        for (int i0 = lo[0]; i0 < hi[0]; ++i0)
          for (int i1 = lo[1]; i1 < hi[1]; ++i1)
            for (int i2 = lo[2]; i2 < hi[2]; ++i2) {
              const int li[3] = {i0, i1, i2};
              bool earlier = false;
              for (int k2 = 0; k2 < I.dim && !earlier; ++k2)
                for (int e2 = 0; e2 < 2; ++e2) {
                  if (k2 * 2 + e2 >= k * 2 + e) break;
                  if (!(S.art >> (2 * k2 + e2) & 1)) continue;
                  if (li[k2] == (e2 == 0 ? 0 : S.n[k2] - 1)) earlier = true;
                }
              if (earlier) continue;
              int o[3] = {0, 0, 0}, gi[3] = {0, 0, 0};
              for (int kk = 0; kk < I.dim; ++kk) {
                gi[kk] = S.lo[kk] + li[kk];
                o[kk] = I.own[kk][gi[kk]];
              }
              const int src = (o[0] * I.parts[1] + o[1]) * I.parts[2] + o[2];
              const SubHost& O = I.subs[src];
              long se = 0, de = 0;
              for (int kk = 0; kk < 3; ++kk) {
                const int ol = (kk < I.dim) ? gi[kk] - O.lo[kk] : 0;
                se = se * O.n[kk] + ol;
                de = de * S.n[kk] + li[kk];
              }
              I.trans.push_back(int4{s, (int)de, src, (int)se});
            }
      }
  }
  I.trans_first[ns] = (int)I.trans.size();
  I.push_cnt.assign(ns, 0);
  for (const int4& t : I.trans) I.push_cnt[t.z]++;
  bool any = false;
  for (int c : I.push_cnt) any |= c > 0;
  if (!any) I.push_cnt.clear();
  // Sweep levels of the alternating forms (Algorithm 1).  The subdomains are visited one at a
  // time in the sweep order; a subdomain's level is one more than the highest level among the
  // subdomains it exchanges values with that come before it in the sweep.  Two subdomains of
  // one level never exchange values, so advancing a whole level at once gives exactly the
  // one-at-a-time sweep, while a subdomain still reads the latest values of every neighbour.
  I.level.assign(ns, 0);
  I.nlevels = 1;
  I.alternating = !I.whole && I.dd.mode != PMA_DD_PARALLEL;
  if (I.alternating) {
    std::vector<int> sweep(ns), pos(ns);
    for (int q = 0; q < ns; ++q) sweep[q] = q;  // block order, axis 0 slowest
    if (I.dd.mode == PMA_DD_COLOURED) {
      auto parity = [&](int q) {
        const int p2 = q % I.parts[2], p1 = (q / I.parts[2]) % I.parts[1], p0 = q / (I.parts[1] * I.parts[2]);
        return (p0 % 2) * 4 + (p1 % 2) * 2 + (p2 % 2);
      };
      std::stable_sort(sweep.begin(), sweep.end(), [&](int a, int b) { return parity(a) < parity(b); });
    }
    for (int i = 0; i < ns; ++i) pos[sweep[i]] = i;
    std::vector<std::vector<int>> nb(ns);
    for (const int4& t : I.trans) {
      nb[t.x].push_back(t.z);
      nb[t.z].push_back(t.x);
    }
    for (int i = 0; i < ns; ++i) {
      const int q = sweep[i];
      int lv = 0;
      for (int o : nb[q])
        if (pos[o] < i) lv = std::max(lv, I.level[o] + 1);
      I.level[q] = lv;
      I.nlevels = std::max(I.nlevels, lv + 1);
    }
  }
}

// per-block partial results of the final checks, one buffer reused in turn: the glue's minima
// (one per block), the cell minima (one per block), the quality sums and maxima (two per block)
static long partials_count(const Instance& I) {
  return std::max(2 * glue_blocks(I.gnodes()), cell_blocks(I.dim, I.grid.n));
}

// bytes of the instance block (state arrays + glue buffers)
static size_t instance_bytes(const Instance& I) {
  size_t b = 0;
  for (const auto& s : I.subs) b += 3 * Arena::round(sub_nodes(s) * I.elem());
  if (!I.single_sub_mode) {
    for (int k = 0; k < I.dim; ++k) b += Arena::round(I.grid.n[k] * sizeof(int));
    b += Arena::round(I.dim * I.gnodes() * sizeof(double));   // mesh
    b += Arena::round(I.gnodes() * sizeof(double));           // psi (in/out)
    b += Arena::round(partials_count(I) * sizeof(double));
  }
  b += Arena::round(4 * sizeof(double));
  if (!I.trans.empty()) b += Arena::round(I.trans.size() * sizeof(int4));
  if (uses_push(I))
    for (size_t s = 0; s < I.subs.size(); ++s)
      if (I.push_cnt[s]) {
        int nct;
        b += Arena::round((size_t)I.push_cnt[s] * sizeof(int4)) +
             Arena::round((size_t)(inv_tiles(I.subs[s].n, I.dim, nct) + 1) * sizeof(int));
      }
  return b;
}

// ------------------------------------------------------------------------------------------
// context
// ------------------------------------------------------------------------------------------

struct Batch;
struct Server;

}  // namespace pma

struct pma_ctx {
  int device = 0;
  size_t budget = 0;
  void* (*alloc_cb)(size_t, void*, void*) = nullptr;
  void (*free_cb)(void*, void*, void*) = nullptr;
  void* alloc_user = nullptr;
  void* arena_mem = nullptr;
  bool arena_from_cb = false;
  pma::Arena arena;
  hipStream_t stream = nullptr;
  std::recursive_mutex mu;  // guards arena, bases, stream work of synchronous calls
  std::map<std::pair<int, int>, pma::Basis*> bases;  // (n, precision)
  uint64_t basis_clock = 0;
  pma::Server* server = nullptr;
  std::mutex server_mu;  // creation of the server thread
};

namespace pma {

static void ensure_arena(pma_ctx* c) {
  if (c->arena.ready()) return;
  HIPCHK(hipSetDevice(c->device));
  void* p = nullptr;
  if (c->alloc_cb) {
    p = c->alloc_cb(c->budget, (void*)c->stream, c->alloc_user);
    if (!p) thr(PMA_E_NOMEM, "allocator callback could not provide the arena");
    c->arena_from_cb = true;
  } else {
    if (hipMalloc(&p, c->budget) != hipSuccess) thr(PMA_E_NOMEM, "hipMalloc of the arena failed");
    c->arena_from_cb = false;
  }
  c->arena_mem = p;
  c->arena.init((char*)p, c->budget);
}

// drop the least recently used basis no request is using; false if there is none
static bool evict_basis(pma_ctx* c) {
  auto victim = c->bases.end();
  for (auto it = c->bases.begin(); it != c->bases.end(); ++it)
    if (it->second->refs == 0 && (victim == c->bases.end() || it->second->last_use < victim->second->last_use))
      victim = it;
  if (victim == c->bases.end()) return false;
  c->arena.release(victim->second->mem);
  delete victim->second;
  c->bases.erase(victim);
  return true;
}

static void* arena_alloc(pma_ctx* c, size_t b) {
  ensure_arena(c);
  while (true) {
    void* p = c->arena.alloc(b);
    if (p) return p;
    if (!evict_basis(c)) thr(PMA_E_NOMEM, "device arena exhausted");
  }
}


static int round_up(int x, int m) { return (x + m - 1) / m * m; }

// row stride of the DCT matrices.  Split form: the padded length plus 16 bytes, so that the 16
// rows of a matrix-core fragment start in distinct LDS bank groups when the matrix is copied into
// LDS.  FP32 and FP64: the padded length; these matrices are stored fragment-major (frag_pos), so
// a fragment is contiguous in memory and in LDS.
static int basis_stride(int n, int prec) {
  return round_up(n, 32) + (prec == PMA_FP32_SPLIT16 ? 8 : 0);
}

// position of entry (r, k) of an FP32 / FP64 matrix with ldb padded columns, fragment-major: the
// 16 x 4 fragment of row block r / 16 and k group k / 4 is 64 consecutive entries, k % 4 major
static size_t frag_pos(int ldb, int r, int k) {
  return ((size_t)(r / 16) * (ldb / 4) + k / 4) * 64 + (k % 4) * 16 + r % 16;
}

static size_t basis_bytes(int n, int prec) {
  const size_t rl = (size_t)round_up(n, 16) * basis_stride(n, prec);
  if (prec == PMA_FP64) return 2 * Arena::round(rl * 8) + Arena::round((size_t)n * 8);
  if (prec == PMA_FP32) return 2 * Arena::round(rl * 4) + Arena::round((size_t)n * 4);
  return 4 * Arena::round(rl * 2) + Arena::round((size_t)n * 4);
}

// the DCT matrices of axis length n in precision prec, written to device memory mem
// (basis_bytes(n, prec) bytes); the Basis describes where each matrix sits
static std::unique_ptr<Basis> fill_basis(int n, int prec, char* mem) {
  if (n > kMaxAxisNodes) thr(PMA_E_INVAL, "a subdomain axis has more than 1025 nodes: split it further");
  std::vector<double> A, B, sig;
  basis_host(n, A, B, sig);
  std::unique_ptr<Basis> b(new Basis);
  b->n = n;
  b->prec = prec;
  b->rows = round_up(n, 16);
  b->ld = round_up(n, 32);
  b->ldb = basis_stride(n, prec);
  const size_t rl = (size_t)b->rows * b->ldb;
  b->bytes = basis_bytes(n, prec);
  b->mem = mem;
  char* p = b->mem;
  auto put = [&](const void* src, size_t sz) {
    HIPCHK(hipMemcpy(p, src, sz, hipMemcpyHostToDevice));
    const void* q = p;
    p += Arena::round(sz);
    return q;
  };
  {
    if (prec == PMA_FP64) {
      std::vector<double> A64(rl, 0.0), B64(rl, 0.0);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          A64[frag_pos(b->ldb, i, j)] = A[(size_t)i * n + j];
          B64[frag_pos(b->ldb, i, j)] = B[(size_t)i * n + j];
        }
      b->fwd = put(A64.data(), rl * 8);
      b->inv = put(B64.data(), rl * 8);
      b->sig = put(sig.data(), (size_t)n * 8);
    } else {
      std::vector<float> sig32(n);
      for (int i = 0; i < n; ++i) sig32[i] = (float)sig[i];
      if (prec == PMA_FP32) {
        std::vector<float> A32(rl, 0.f), B32(rl, 0.f);
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) {
            A32[frag_pos(b->ldb, i, j)] = (float)A[(size_t)i * n + j];
            B32[frag_pos(b->ldb, i, j)] = (float)B[(size_t)i * n + j];
          }
        b->fwd = put(A32.data(), rl * 4);
        b->inv = put(B32.data(), rl * 4);
      } else {
        // forward matrix pre-scaled by 2^s (largest entry in [1, 2)), both split into fp16 hi + lo
        double amax = 0;
        for (size_t i = 0; i < (size_t)n * n; ++i) amax = std::max(amax, std::fabs(A[i]));
        const int se = -(int)std::floor(std::log2(amax));
        const double sc = std::ldexp(1.0, se);
        b->fwd_unscale = (float)std::ldexp(1.0, -se);
        std::vector<_Float16> Ahi(rl, (_Float16)0.f), Alo(rl, (_Float16)0.f), Bhi(rl, (_Float16)0.f),
            Blo(rl, (_Float16)0.f);
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) {
            const size_t src = (size_t)i * n + j, dst = (size_t)i * b->ldb + j;
            const double as = A[src] * sc;
            Ahi[dst] = (_Float16)as;
            Alo[dst] = (_Float16)(as - (double)Ahi[dst]);
            Bhi[dst] = (_Float16)B[src];
            Blo[dst] = (_Float16)(B[src] - (double)Bhi[dst]);
          }
        b->fwd = put(Ahi.data(), rl * 2);
        b->fwdl = put(Alo.data(), rl * 2);
        b->inv = put(Bhi.data(), rl * 2);
        b->invl = put(Blo.data(), rl * 2);
      }
      b->sig = put(sig32.data(), (size_t)n * 4);
    }
  }
  return b;
}

static Basis* get_basis(pma_ctx* c, int n, int prec) {
  auto key = std::make_pair(n, prec);
  auto it = c->bases.find(key);
  if (it != c->bases.end()) {
    it->second->last_use = ++c->basis_clock;
    return it->second;
  }
  if (n > kMaxAxisNodes) thr(PMA_E_INVAL, "a subdomain axis has more than 1025 nodes: split it further");
  char* mem = (char*)arena_alloc(c, basis_bytes(n, prec));
  std::unique_ptr<Basis> b;
  try {
    b = fill_basis(n, prec, mem);
  } catch (...) {
    c->arena.release(mem);
    throw;
  }
  b->last_use = ++c->basis_clock;
  Basis* raw = b.release();
  c->bases[key] = raw;
  return raw;
}

static std::vector<int> distinct_axis_sizes(const Instance& I) {
  std::vector<int> ns;
  for (const auto& s : I.subs)
    for (int k = 0; k < I.dim; ++k)
      if (std::find(ns.begin(), ns.end(), s.n[k]) == ns.end()) ns.push_back(s.n[k]);
  return ns;
}

// arena bytes the instance's bases still need (0 for cached ones); none for forward Euler
static size_t new_basis_bytes(pma_ctx* c, const Instance& I) {
  if (I.tm.gamma == 0.0) return 0;
  size_t b = 0;
  for (int n : distinct_axis_sizes(I))
    if (!c->bases.count(std::make_pair(n, I.prec))) b += basis_bytes(n, I.prec);
  return b;
}

// bytes of cached bases that no request uses and the request I does not need: arena_alloc
// evicts them when it runs out of room, so they count as free when admitting I
static size_t evictable_basis_bytes(pma_ctx* c, const Instance& I) {
  std::vector<int> mine;
  if (I.tm.gamma != 0.0) mine = distinct_axis_sizes(I);
  size_t b = 0;
  for (auto& kv : c->bases) {
    const Basis* B = kv.second;
    if (B->refs != 0) continue;
    if (B->prec == I.prec && std::find(mine.begin(), mine.end(), B->n) != mine.end()) continue;
    b += Arena::round(B->bytes);
  }
  return b;
}

static size_t all_basis_bytes(const Instance& I) {
  if (I.tm.gamma == 0.0) return 0;
  size_t b = 0;
  for (int n : distinct_axis_sizes(I)) b += basis_bytes(n, I.tm.precision);
  return b;
}

// Push transmission of a preconditioned DD request, once per allocation: for every transmission
// entry, the inverse-last kernel of the tile holding the source node writes the node's new value
// into the destination (an artificial node of another subdomain of the request).  Entries carry
// the destination's device address, so the tables depend on the request alone and batches of
// any membership use them as they are.
template <typename Take>
static void build_push_tables(pma_ctx* c, Instance& I, Take& take) {
  const int ns = (int)I.subs.size();
  std::vector<int> ebase(ns + 1, 0), tbase(ns + 1, 0), nct(ns, 1);
  for (int s = 0; s < ns; ++s) {
    ebase[s + 1] = ebase[s] + I.push_cnt[s];
    tbase[s + 1] = tbase[s] + (I.push_cnt[s] ? inv_tiles(I.subs[s].n, I.dim, nct[s]) + 1 : 0);
  }
  auto tile_of = [&](const int4& t, int& r, int& col) {
    const SubHost& S = I.subs[t.z];
    const int C = S.n[I.dim - 1];
    r = t.w / C;
    col = t.w - r * C;
    return (r / kRows) * nct[t.z] + col / kCols;
  };
  // counts per local tile, then each entry in its tile's slot (list order kept within a tile)
  I.pfirst_host.assign(tbase[ns], 0);
  for (const int4& t : I.trans) {
    int r, col;
    I.pfirst_host[tbase[t.z] + tile_of(t, r, col) + 1]++;
  }
  for (int s = 0; s < ns; ++s)
    for (int k = tbase[s] + 1; k < tbase[s + 1]; ++k) I.pfirst_host[k] += I.pfirst_host[k - 1];
  std::vector<int> fill(I.pfirst_host);
  I.push_host.assign(ebase[ns], int4{0, 0, 0, 0});
  for (const int4& t : I.trans) {
    int r, col;
    const int lt = tile_of(t, r, col);
    const int later = I.level[t.x] > I.level[t.z] ? 1 : 0;  // destination updated later this step
    const unsigned long long addr = (unsigned long long)(uintptr_t)I.phi[t.x] + I.elem() * (size_t)t.y;
    I.push_host[ebase[t.z] + fill[tbase[t.z] + lt]++] =
        int4{(int)(unsigned)(addr & 0xffffffffull), (int)(unsigned)(addr >> 32), (r % kRows) | (later << 8),
             col % kCols};
  }
  I.push_dev.assign(ns, nullptr);
  I.pfirst_dev.assign(ns, nullptr);
  for (int s = 0; s < ns; ++s) {
    if (!I.push_cnt[s]) continue;
    I.push_dev[s] = (int4*)take((size_t)I.push_cnt[s] * sizeof(int4));
    I.pfirst_dev[s] = (int*)take((size_t)(tbase[s + 1] - tbase[s]) * sizeof(int));
    HIPCHK(hipMemcpyAsync(I.push_dev[s], I.push_host.data() + ebase[s], (size_t)I.push_cnt[s] * sizeof(int4),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(I.pfirst_dev[s], I.pfirst_host.data() + tbase[s],
                          (size_t)(tbase[s + 1] - tbase[s]) * sizeof(int), hipMemcpyHostToDevice, c->stream));
  }
}

// device bytes of an instance with its own copy of every basis (the allocation-free path)
static size_t instance_bytes_with_bases(const Instance& I) {
  size_t b = Arena::round(instance_bytes(I));
  if (I.tm.gamma > 0)
    for (int n : distinct_axis_sizes(I)) b += Arena::round(basis_bytes(n, I.prec));
  return b;
}

// ext: caller-provided device memory of ext_cap bytes (the fixed scratch) holding the block and
// private copies of the bases instead of the arena and the basis cache; returns the bytes used
static size_t alloc_instance(pma_ctx* c, Instance& I, char* ext = nullptr, size_t ext_cap = 0) {
  I.bytes = instance_bytes(I);
  I.ext_mem = ext != nullptr;
  if (ext) {
    if (instance_bytes_with_bases(I) > ext_cap) thr(PMA_E_INVAL, "internal: scratch too small for the instance");
    I.block = ext;
  } else {
    I.block = (char*)arena_alloc(c, I.bytes);
  }
  char* p = I.block;
  auto take = [&](size_t sz) {
    char* q = p;
    p += Arena::round(sz);
    return q;
  };
  I.phi.clear();
  I.F.clear();
  I.T.clear();
  for (const auto& s : I.subs) {
    const size_t b = sub_nodes(s) * I.elem();
    I.phi.push_back(take(b));
    I.F.push_back(take(b));
    I.T.push_back(take(b));
  }
  if (!I.single_sub_mode) {
    for (int k = 0; k < I.dim; ++k) I.own_dev[k] = (int*)take(I.grid.n[k] * sizeof(int));
    I.mesh_dev = (double*)take(I.dim * I.gnodes() * sizeof(double));
    I.psi_dev = (double*)take(I.gnodes() * sizeof(double));
    I.minpart_n = partials_count(I);
    I.minpart = (double*)take(I.minpart_n * sizeof(double));
    for (int k = 0; k < I.dim; ++k)
      HIPCHK(hipMemcpyAsync(I.own_dev[k], I.own[k].data(), I.grid.n[k] * sizeof(int),
                            hipMemcpyHostToDevice, c->stream));
  }
  I.stats_dev = (double*)take(4 * sizeof(double));
  I.trans_dev = nullptr;
  if (!I.trans.empty()) {
    I.trans_dev = (int4*)take(I.trans.size() * sizeof(int4));
    HIPCHK(hipMemcpyAsync(I.trans_dev, I.trans.data(), I.trans.size() * sizeof(int4), hipMemcpyHostToDevice,
                          c->stream));
  }
  if (uses_push(I)) build_push_tables(c, I, take);
  I.bases_used.clear();
  if (ext) {
    char* q = I.block + Arena::round(I.bytes);
    if (I.tm.gamma > 0) {
      try {
        for (int n : distinct_axis_sizes(I)) {
          I.bases_used.push_back(fill_basis(n, I.prec, q).release());
          q += Arena::round(basis_bytes(n, I.prec));
        }
      } catch (...) {
        for (auto* b : I.bases_used) delete b;
        I.bases_used.clear();
        I.block = nullptr;
        throw;
      }
    }
    return (size_t)(q - I.block);
  }
  if (I.tm.gamma > 0) {
    try {
      for (int n : distinct_axis_sizes(I)) {
        Basis* b = get_basis(c, n, I.prec);
        b->refs++;
        I.bases_used.push_back(b);
      }
    } catch (...) {
      for (auto* b : I.bases_used) b->refs--;
      I.bases_used.clear();
      c->arena.release(I.block);
      I.block = nullptr;
      throw;
    }
  }
  return Arena::round(I.bytes);
}

// warm start: the caller's global Psi^0 (host) into the instance's Psi buffer, from which the
// initial state of every subdomain is taken (on the context's stream)
static void upload_psi0(pma_ctx* c, Instance& I, const double* psi0) {
  if (!psi0) return;
  if (I.single_sub_mode) thr(PMA_E_INVAL, "internal: warm start of a single-subdomain solve");
  HIPCHK(hipMemcpyAsync(I.psi_dev, psi0, I.gnodes() * 8, hipMemcpyHostToDevice, c->stream));
  I.psi0_dev = I.psi_dev;
}

// the basis of axis length n among those the instance holds (cached or its own copy)
static const Basis* basis_of(const Instance& I, int n) {
  for (const Basis* b : I.bases_used)
    if (b->n == n) return b;
  thr(PMA_E_HIP, "internal: no basis of the instance for an axis length");
  return nullptr;
}

static void free_instance(pma_ctx* c, Instance& I) {
  if (I.ext_mem) {
    for (auto* b : I.bases_used) delete b;   // private copies in the caller's memory
    I.bases_used.clear();
    I.block = nullptr;
    return;
  }
  for (auto* b : I.bases_used) b->refs--;
  I.bases_used.clear();
  if (I.block) c->arena.release(I.block);
  I.block = nullptr;
}

// ------------------------------------------------------------------------------------------
// batch: every subdomain of a set of instances (one precision) advanced by shared launches
// ------------------------------------------------------------------------------------------

static constexpr int kStRows = 4, kStCols = 64;     // forward-Euler tiles
static constexpr int kStChunk = 16, kStWmax = 72;  // stencil: rows per chunk, widest block
static constexpr int kPhases = 8;
static constexpr int kLdsBasisCap = 160 * 1024 - 4096;  // dynamic LDS a workgroup may take
// Copying the basis into LDS removes the basis loads from a strip workgroup's critical path but
// leaves room for one workgroup per CU: worth it while a launch has at most about two
// workgroups per CU (latency-bound), not for large batches that rely on occupancy.
static constexpr int kLdsBasisMaxTiles = 512;
static constexpr int kWideMaxLd = 320;  // widest padded axis of the 64-column strip kernel
static constexpr size_t kBarBytes = (64 + 8 * 32) * 4;  // the persistent step's barrier words

struct SubRange {
  int first, count;
};

// Tile table of one launch: entries plus, per subdomain, its contiguous range (plain form).
struct Table {
  std::vector<int4> h;
  std::vector<SubRange> rng;
  int4* d = nullptr;
  int maxld = 32;
  int lneed = 0;     // strip / fused launches: largest LDS footprint with the basis copied in (if it fits)
  int lneed_nb = 0;  // fused launches: largest LDS footprint without the basis copy
  // rng is indexed by batch subdomain; subdomains are laid out in the batch's launch order
  void begin_sub(int gs) { rng[gs] = SubRange{(int)h.size(), 0}; }
  void end_sub(int gs) { rng[gs].count = (int)h.size() - rng[gs].first; }
  int size() const { return (int)h.size(); }
};

template <typename T>
static void fill_monitor(const pma_monitor& m, MonP<T>& p) {
  p.kind = m.kind;
  p.nb = m.nbumps;
  p.amp = (T)m.amp;
  p.k = (T)m.k;
  p.r0 = (T)m.r0;
  p.r02 = (T)(m.r0 * m.r0);
  for (int q = 0; q < 3; ++q) {
    p.c[q] = (T)m.c[q];
    p.aa[q] = (T)m.amp_axes[q];
    p.ka[q] = (T)m.k_axes[q];
  }
  p.tw = (T)m.twist;
  for (int b = 0; b < kMaxBumps; ++b) {
    p.bamp[b] = (T)m.bamp[b];
    p.bnh[b] = (m.kind == PMA_MON_GAUSS_SUM && b < m.nbumps) ? (T)(-1.0 / (2.0 * m.bw[b] * m.bw[b])) : (T)0;
    for (int q = 0; q < 3; ++q) p.bc[b][q] = (T)m.bc[b][q];
  }
}

// Phases of a step, in launch order:
//   0 transmission                1 stencil (F)                       2 forward-Euler update
//   3 forward product along the last axis
//   4 forward product along the middle axis (3D)
//   5 forward product + spectral scale + inverse product along axis 0
//   6 inverse product along the middle axis (3D)
//   7 inverse product along the last axis + update + residual partials
struct Batch {
  pma_ctx* ctx = nullptr;
  int prec = 0;
  std::vector<Instance*> insts;
  std::vector<SubDev> h_subs;
  std::vector<InstDev> h_insts;
  // a step's transmission: pushed by the inverse-last kernel of the owner (gamma > 0), or pulled
  // by the gather before the stencil (forward-Euler instances)
  std::vector<int4> h_pull;
  std::vector<SubRange> pull_rng;
  // launch order: subdomains sorted by sweep level (stable); level L holds positions
  // lvl_first[L] .. lvl_first[L + 1] - 1 of `order`, and every launch table and the pull list
  // are laid out in this order, so one level is one contiguous range of each
  std::vector<int> glevel, order, lvl_first;
  int nlev = 1;
  int4* d_pull = nullptr;
  Table tab[kPhases];  // tab[0] unused (transmission has its own list)
  int part_base_eu = 0, part_base_inv = 0, npartials = 0;
  char* dmem = nullptr;
  SubDev* d_subs = nullptr;
  InstDev* d_insts = nullptr;
  void* d_dc = nullptr;
  double *d_partials = nullptr, *d_shift = nullptr, *d_resid = nullptr;
  int* d_status = nullptr;
  double* h_resid = nullptr;
  int* h_status = nullptr;
  size_t pinned_cap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // kGraphSteps steps captured back to back in one graph: runs of steps replay it, so the host
  // submits one graph per kGraphSteps steps; the remainder replays the one-step graph
  static constexpr int kGraphSteps = 8;
  hipGraph_t graph_n = nullptr;
  hipGraphExec_t gexec_n = nullptr;
  // the remainder of a run (1 .. kGraphSteps - 1 steps) as one graph per length, captured on
  // first use, so a run of any length submits ceil(steps / kGraphSteps) graphs
  hipGraph_t graph_r[kGraphSteps] = {};
  hipGraphExec_t gexec_r[kGraphSteps] = {};
  bool use_graph = true;  // replay captured steps; false: launch the phases directly
  StepArgs sa{};

  size_t dcap = 0;  // capacity of dmem: launch tables live outside the request arena
  // allocation-free path: launch tables in caller-provided device memory (the fixed scratch),
  // residual and status read back into ordinary host memory
  char* ext_tab = nullptr;
  size_t ext_tab_cap = 0;
  std::vector<double> hv_resid;
  std::vector<int> hv_status;

  ~Batch() {
    clear_device();
    if (dmem) hipFree(dmem);
    if (!ext_tab) {
      if (h_resid) hipHostFree(h_resid);
      if (h_status) hipHostFree(h_status);
    }
  }

  // forget the launch set (the table buffer is kept for the next build)
  void clear_device() {
    drop_graphs();
    built = false;
  }

  void drop_graphs() {
    if (gexec) hipGraphExecDestroy(gexec);
    if (graph) hipGraphDestroy(graph);
    if (gexec_n) hipGraphExecDestroy(gexec_n);
    if (graph_n) hipGraphDestroy(graph_n);
    gexec = nullptr;
    graph = nullptr;
    gexec_n = nullptr;
    graph_n = nullptr;
    for (int r = 0; r < kGraphSteps; ++r) {
      if (gexec_r[r]) hipGraphExecDestroy(gexec_r[r]);
      if (graph_r[r]) hipGraphDestroy(graph_r[r]);
      gexec_r[r] = nullptr;
      graph_r[r] = nullptr;
    }
  }
  bool built = false;

  static AxisDev axis_dev(const Basis* b) {
    AxisDev a{};
    a.ld = b->ld;
    a.ldb = b->ldb;
    a.fwd = b->fwd;
    a.fwdl = b->fwdl;
    a.inv = b->inv;
    a.invl = b->invl;
    a.sig = b->sig;
    a.fwd_unscale = b->fwd_unscale;
    return a;
  }

  // Stencil blocks of subdomain gs: W <= 72 columns of the last axis (balanced over the axis),
  // marching `march` chunks (2D: 16-row chunks of axis 0; 3D: planes of axis 0 over 16 rows of
  // axis 1) per workgroup.
  void stencil_tiles(int gs, int march, std::vector<int4>& out) const {
    const SubDev& sd = h_subs[gs];
    if (fused_[gs]) {  // 16 full rows per workgroup, stencil + forward last-axis product
      for (int r = 0; r < sd.n[0]; r += kStChunk) out.push_back(int4{gs, r, 0, 0});
      return;
    }
    const int n0 = sd.n[0], n1 = sd.n[1], nl = sd.n[sd.dim - 1];
    const int nct = (nl + kStWmax - 1) / kStWmax;
    const int W = (nl + nct - 1) / nct;
    if (sd.dim == 2) {
      const int rows = kStChunk * march;
      for (int r = 0; r < n0; r += rows)
        for (int c = 0; c < n1; c += W)
          out.push_back(int4{gs, r, c | (std::min(W, n1 - c) << 16), std::min(rows, n0 - r)});
    } else {
      for (int p = 0; p < n0; p += march)
        for (int r = 0; r < n1; r += kStChunk)
          for (int c = 0; c < nl; c += W)
            out.push_back(int4{gs, p | (std::min(march, n0 - p) << 16), r, c | (std::min(W, nl - c) << 16)});
    }
  }
  // 2D subdomains of preconditioned instances take the stencil fused with the forward product
  // along the last axis when that axis is at most 320 wide (padded)
  bool fuse = true;
  std::vector<char> fused_;
  int stencil_kind(int gs) const { return fused_[gs] ? 4 : h_subs[gs].dim; }
  // chunks per workgroup when not tuned: enough workgroups to fill the chip several times over
  int st_march = 1;
  int stencil_march_default() const {
    size_t t1 = 0;
    std::vector<int4> tmp;
    for (size_t gs = 0; gs < h_subs.size(); ++gs) {
      tmp.clear();
      stencil_tiles((int)gs, 1, tmp);
      t1 += tmp.size();
    }
    return (int)std::max<size_t>(1, std::min<size_t>(64, t1 / 8192));
  }
  // the stencil tile table rebuilt for another march length (same device buffer: march 1 is the
  // largest table); the captured step graphs are dropped
  void set_stencil_march(int march) {
    st_march = march;
    Table& t = tab[1];
    t.h.clear();
    t.rng.assign(h_subs.size(), SubRange{0, 0});
    for (int gs : order) {
      t.begin_sub(gs);
      stencil_tiles(gs, march, t.h);
      t.end_sub(gs);
    }
    if (t.h.size() > st_cap) thr(PMA_E_HIP, "stencil table exceeds its buffer");
    HIPCHK(hipMemcpyAsync(t.d, t.h.data(), t.h.size() * 16, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    drop_graphs();
  }
  size_t st_cap = 0;

  // launch-shape thresholds (tuned by pma_plan_tune; results do not depend on them): launches of
  // at most eight_max tiles take eight-wave workgroups, of at most lbasis_max tiles copy the DCT
  // matrices into LDS where they fit
  int eight_max = 512, lbasis_max = kLdsBasisMaxTiles;
  int lds_basis(const Table& t, int count) const { return count <= lbasis_max ? t.lneed : 0; }

  // 64-column strips (phases 4-6) when every launch of a 16-column table would exceed
  // kLdsBasisMaxTiles strips: every strip then reads its axis' DCT matrices from L2, and four
  // blocks per workgroup read them a quarter as often.  A launch of fewer strips (a sweep level of
  // an alternating request) is latency-bound and keeps the narrow strips.  Bitwise the same
  // results; FP32 and split forms, axes up to kWideMaxLd.  (In FP64 the 64-column operand leaves
  // room for one workgroup per compute unit, whose staging then no longer overlaps other
  // workgroups' products: measured 1.45x slower on the 256-instance batch, not used.)
  bool wide_ok = true;
  bool wide_[kPhases] = {};
  void choose_wide() {
    long cols[kPhases] = {0}, cols64[kPhases] = {0};
    std::vector<long> lcnt((size_t)nlev * kPhases, 0);  // strips per sweep level and phase
    int mld[kPhases] = {0};
    for (auto& w : wide_) w = false;
    if (!wide_ok || prec == PMA_FP64) return;
    for (size_t gs = 0; gs < h_subs.size(); ++gs) {
      const SubDev& sd = h_subs[gs];
      if (insts[sd.inst]->tm.gamma == 0.0) continue;
      long* cnt = &lcnt[(size_t)glevel[gs] * kPhases];
      const int rest = sd.dim == 2 ? sd.n[1] : sd.n[1] * sd.n[2];
      cnt[5] += (rest + kStrip - 1) / kStrip;
      cols[5] += rest;
      cols64[5] += (rest + 63) / 64 * 64;
      mld[5] = std::max(mld[5], sd.ax[0].ld);
      if (sd.dim == 3) {
        const long c = (long)sd.n[0] * ((sd.n[2] + kStrip - 1) / kStrip);
        cnt[4] += c;
        cnt[6] += c;
        for (int ph : {4, 6}) {
          cols[ph] += (long)sd.n[0] * sd.n[2];
          cols64[ph] += (long)sd.n[0] * ((sd.n[2] + 63) / 64 * 64);
        }
        mld[4] = std::max(mld[4], sd.ax[1].ld);
        mld[6] = std::max(mld[6], sd.ax[1].ld);
      }
    }
    // and only where 64-column tiles are mostly full (a 68-wide slab would waste half its second tile)
    for (int ph = 4; ph <= 6; ++ph) {
      long least = -1;
      for (int L = 0; L < nlev; ++L) {
        const long c = lcnt[(size_t)L * kPhases + ph];
        if (c > 0) least = least < 0 ? c : std::min(least, c);
      }
      wide_[ph] = least > kLdsBasisMaxTiles && mld[ph] <= kWideMaxLd && 5 * cols[ph] >= 4 * cols64[ph];
    }
  }

  // strip launches copy an axis' basis into LDS when strip + basis fit in a workgroup's LDS:
  // 16 x ld operand entries and round_up(n, 16) x ld basis entries (split form: hi + lo)
  void note_lds(Table& t, int n, int ld) const {
    const int ob = prec == PMA_FP64 ? 8 : 4;
    const int bb = prec == PMA_FP64 ? 8 : 4;  // basis bytes per entry (split form: hi + lo)
    const int need = 16 * (ld + 16 / ob) * ob + ((n + 15) / 16) * 16 * basis_stride(n, prec) * bb;
    if (need <= kLdsBasisCap) t.lneed = std::max(t.lneed, need);
  }

  // The gather lists of forward-Euler requests (the preconditioned ones push their transmission
  // from the inverse-last kernel, with per-request tables made at allocation).
  void build_pull_lists() {
    pull_rng.assign(h_subs.size(), SubRange{0, 0});
    for (int gs : order) {
      SubRange pr{(int)h_pull.size(), 0};
      const Instance& I = *insts[h_subs[gs].inst];
      if (I.tm.gamma == 0.0) {
        const int first = h_insts[h_subs[gs].inst].first_sub, s = gs - first;
        for (int e = I.trans_first[s]; e < I.trans_first[s + 1]; ++e) {
          const int4 t = I.trans[e];
          h_pull.push_back(int4{first + t.x, t.y, first + t.z, t.w});
        }
      }
      pr.count = (int)h_pull.size() - pr.first;
      pull_rng[gs] = pr;
    }
  }

  void build() {
    HIPCHK(enable_large_lds());
    clear_device();
    h_subs.clear();
    h_insts.clear();
    h_pull.clear();
    pull_rng.clear();
    for (auto& t : tab) t = Table();
    for (size_t q = 0; q < insts.size(); ++q) {
      Instance& I = *insts[q];
      InstDev id{};
      fill_monitor(I.mon, id.mond);
      fill_monitor(I.mon, id.monf);
      double vol = 1.0;
      for (int k = 0; k < I.dim; ++k) vol *= I.grid.hi[k] - I.grid.lo[k];
      id.log_vol_theta = std::log(vol / I.theta);
      id.dt = I.tm.dt;
      id.first_sub = (int)h_subs.size();
      id.nsub = (int)I.subs.size();
      // removing a constant from phi is invisible to every derivative only if every artificial
      // node is refilled from the same instance (transmission); held Dirichlet data of a lone
      // subdomain would be left behind by the shift.  The parallel form removes the mean DC
      // coefficient of all subdomains; an alternating sweep must remove one constant known
      // before its later levels run: the DC coefficient of subdomain 0, the first of the sweep
      id.pin = (I.tm.gamma > 0 && !I.single_sub_mode) ? (I.alternating ? 1 : (int)I.subs.size()) : 0;
      h_insts.push_back(id);
      for (size_t s = 0; s < I.subs.size(); ++s) {
        const SubHost& S = I.subs[s];
        SubDev sd{};
        sd.dim = I.dim;
        for (int k = 0; k < 3; ++k) {
          sd.n[k] = S.n[k];
          sd.off[k] = S.lo[k];
          if (k < I.dim) {
            sd.a[k] = I.grid.lo[k];
            sd.h[k] = (I.grid.hi[k] - I.grid.lo[k]) / (I.grid.n[k] - 1);
            sd.gh2[k] = I.tm.gamma / (sd.h[k] * sd.h[k]);
            if (I.tm.gamma > 0) sd.ax[k] = axis_dev(basis_of(I, S.n[k]));
          } else {
            sd.a[k] = 0;
            sd.h[k] = 1;
            sd.gh2[k] = 0;
          }
        }
        sd.art = S.art;
        sd.inst = (int)q;
        sd.phi = I.phi[s];
        sd.F = I.F[s];
        sd.T = I.T[s];
        const bool push = uses_push(I) && I.push_dev[s];
        sd.push = push ? I.push_dev[s] : nullptr;
        sd.pfirst = push ? I.pfirst_dev[s] : nullptr;
        h_subs.push_back(sd);
      }
    }
    // sweep levels and the launch order
    glevel.assign(h_subs.size(), 0);
    nlev = 1;
    for (size_t q = 0; q < insts.size(); ++q) {
      if (insts[q]->level.size() != insts[q]->subs.size()) thr(PMA_E_HIP, "internal: plan without sweep levels");
      for (size_t s = 0; s < insts[q]->subs.size(); ++s) {
        glevel[h_insts[q].first_sub + s] = insts[q]->level[s];
        nlev = std::max(nlev, insts[q]->nlevels);
      }
    }
    order.resize(h_subs.size());
    for (size_t gs = 0; gs < order.size(); ++gs) order[gs] = (int)gs;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return glevel[a] < glevel[b]; });
    lvl_first.assign(nlev + 1, (int)order.size());
    for (int p = (int)order.size() - 1; p >= 0; --p) lvl_first[glevel[order[p]]] = p;
    for (int L = nlev - 1; L >= 0; --L) lvl_first[L] = std::min(lvl_first[L], lvl_first[L + 1]);
    fused_.assign(h_subs.size(), 0);
    for (size_t gs = 0; gs < h_subs.size(); ++gs) {
      const SubDev& sd = h_subs[gs];
      fused_[gs] = fuse && sd.dim == 2 && insts[sd.inst]->tm.gamma > 0 && sd.ax[1].ld <= 320;
    }
    st_march = stencil_march_default();
    {
      std::vector<int4> tmp;
      for (size_t gs = 0; gs < h_subs.size(); ++gs) stencil_tiles((int)gs, 1, tmp);
      st_cap = tmp.size();
    }
    // transmission lists, subdomain by subdomain (an instance's entries stay contiguous)
    // tiles, subdomain by subdomain in launch order
    choose_wide();
    const int sw4 = wide_[4] ? 4 * kStrip : kStrip, sw5 = wide_[5] ? 4 * kStrip : kStrip;
    for (int ph = 1; ph < kPhases; ++ph) tab[ph].rng.assign(h_subs.size(), SubRange{0, 0});
    {
      for (int gs : order) {
        const SubDev& sd = h_subs[gs];
        const Instance& I = *insts[sd.inst];
        const int n0 = sd.n[0], n1 = sd.n[1], n2 = sd.n[2];
        const int R = I.dim == 2 ? n0 : n0 * n1, C = I.dim == 2 ? n1 : n2;
        for (int ph = 1; ph < kPhases; ++ph) tab[ph].begin_sub(gs);
        stencil_tiles(gs, st_march, tab[1].h);
        if (I.tm.gamma == 0.0) {
          for (int r = 0; r < R; r += kStRows)
            for (int c = 0; c < C; c += kStCols) tab[2].h.push_back(int4{gs, r, c, 0});
        } else {
          const int la = I.dim - 1;
          if (!fused_[gs]) {
            for (int r = 0; r < R; r += kRows)
              for (int c = 0; c < C; c += kCols) tab[3].h.push_back(int4{gs, r, c, 0});
            tab[3].maxld = std::max(tab[3].maxld, sd.ax[la].ld);
          } else {
            const int nb = fused_lds_bytes(prec, sd.ax[1].ld, sd.ax[1].ldb, n1, false);
            const int wb = fused_lds_bytes(prec, sd.ax[1].ld, sd.ax[1].ldb, n1, true);
            tab[1].lneed = std::max(tab[1].lneed, wb <= kLdsBasisCap ? wb : nb);
            tab[1].lneed_nb = std::max(tab[1].lneed_nb, nb);
          }
          if (I.dim == 3) {
            for (int i0 = 0; i0 < n0; ++i0)
              for (int c = 0; c < n2; c += sw4) {  // phases 4 and 6 share the width
                tab[4].h.push_back(int4{gs, i0, c, 0});
                tab[6].h.push_back(int4{gs, i0, c, 0});
              }
            tab[4].maxld = std::max(tab[4].maxld, sd.ax[1].ld);
            tab[6].maxld = std::max(tab[6].maxld, sd.ax[1].ld);
            note_lds(tab[4], n1, sd.ax[1].ld);
            note_lds(tab[6], n1, sd.ax[1].ld);
          }
          const int rest = I.dim == 2 ? n1 : n1 * n2;
          for (int c = 0; c < rest; c += sw5) tab[5].h.push_back(int4{gs, 0, c, 0});
          tab[5].maxld = std::max(tab[5].maxld, sd.ax[0].ld);
          note_lds(tab[5], n0, sd.ax[0].ld);
          // (w: the tile's index among the subdomain's inverse-last tiles, for its push entries)
          const int nct = (C + kCols - 1) / kCols;
          for (int r = 0; r < R; r += kRows)
            for (int c = 0; c < C; c += kCols) tab[7].h.push_back(int4{gs, r, c, (r / kRows) * nct + c / kCols});
          tab[7].maxld = std::max(tab[7].maxld, sd.ax[la].ld);
        }
        for (int ph = 1; ph < kPhases; ++ph) tab[ph].end_sub(gs);
      }
    }
    // residual partial sums: inverse-last tiles, then Euler tiles
    part_base_inv = 0;
    part_base_eu = tab[7].size();
    npartials = tab[7].size() + tab[2].size();
    for (size_t gs = 0; gs < h_subs.size(); ++gs) {
      SubDev& sd = h_subs[gs];
      const Instance& I = *insts[sd.inst];
      if (I.tm.gamma == 0.0) {
        sd.part0 = part_base_eu + tab[2].rng[gs].first;
        sd.nparts = tab[2].rng[gs].count;
      } else {
        sd.part0 = part_base_inv + tab[7].rng[gs].first;
        sd.nparts = tab[7].rng[gs].count;
      }
    }
    build_pull_lists();
    // device block
    const size_t nsub = h_subs.size(), ninst = h_insts.size();
    const size_t el = prec == PMA_FP64 ? 8 : 4;
    size_t bytes = Arena::round(nsub * sizeof(SubDev)) + Arena::round(ninst * sizeof(InstDev)) +
                   Arena::round(h_pull.size() * 16 + 16) + Arena::round(nsub * el) +
                   Arena::round((size_t)(npartials + 1) * 8) + 2 * Arena::round(ninst * 8) + Arena::round(ninst * 4) +
                   Arena::round(kBarBytes);
    for (int ph = 1; ph < kPhases; ++ph) bytes += Arena::round((ph == 1 ? st_cap : tab[ph].h.size()) * 16 + 16);
    if (ext_tab) {
      if (bytes > ext_tab_cap) thr(PMA_E_INVAL, "launch tables exceed the fixed scratch");
    } else if (bytes > dcap) {
      if (dmem) {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipFree(dmem));
        dmem = nullptr;
      }
      dcap = std::max(bytes, 2 * dcap);
      if (hipMalloc((void**)&dmem, dcap) != hipSuccess) {
        dmem = nullptr;
        dcap = 0;
        thr(PMA_E_NOMEM, "launch tables: device allocation failed");
      }
    }
    char* p = ext_tab ? ext_tab : dmem;
    auto take = [&](size_t sz) {
      char* q = p;
      p += Arena::round(sz);
      return q;
    };
    hipStream_t st = ctx->stream;
    auto up = [&](void* dst, const void* src, size_t sz) {
      if (sz) HIPCHK(hipMemcpyAsync(dst, src, sz, hipMemcpyHostToDevice, st));
    };
    d_subs = (SubDev*)take(nsub * sizeof(SubDev));
    d_insts = (InstDev*)take(ninst * sizeof(InstDev));
    d_pull = (int4*)take(h_pull.size() * 16 + 16);
    for (int ph = 1; ph < kPhases; ++ph) tab[ph].d = (int4*)take((ph == 1 ? st_cap : tab[ph].h.size()) * 16 + 16);
    d_dc = take(nsub * el);
    d_partials = (double*)take((size_t)(npartials + 1) * 8);
    d_shift = (double*)take(ninst * 8);
    d_resid = (double*)take(ninst * 8);
    d_status = (int*)take(ninst * 4);
    d_bar = (unsigned*)take(kBarBytes);
    up(d_subs, h_subs.data(), nsub * sizeof(SubDev));
    up(d_insts, h_insts.data(), ninst * sizeof(InstDev));
    up(d_pull, h_pull.data(), h_pull.size() * 16);
    for (int ph = 1; ph < kPhases; ++ph) up(tab[ph].d, tab[ph].h.data(), tab[ph].h.size() * 16);
    HIPCHK(hipMemsetAsync(d_dc, 0, nsub * el, st));
    HIPCHK(hipMemsetAsync(d_partials, 0, (size_t)(npartials + 1) * 8, st));
    HIPCHK(hipMemsetAsync(d_status, 0, ninst * 4, st));
    HIPCHK(hipMemsetAsync(d_bar, 0, kBarBytes, st));
    HIPCHK(hipMemsetAsync(d_resid, 0, ninst * 8, st));
    // accumulated shifts continue across rebuilds
    std::vector<double> sh(ninst, 0.0);
    for (size_t q = 0; q < ninst; ++q) sh[q] = insts[q]->shift_acc;
    up(d_shift, sh.data(), ninst * 8);
    if (ext_tab) {
      hv_resid.assign(ninst + 1, 0.0);
      hv_status.assign(ninst + 1, 0);
      h_resid = hv_resid.data();
      h_status = hv_status.data();
    } else if (ninst + 1 > pinned_cap) {
      if (h_resid) hipHostFree(h_resid);
      if (h_status) hipHostFree(h_status);
      h_resid = nullptr;
      h_status = nullptr;
      pinned_cap = std::max<size_t>(64, 2 * (ninst + 1));
      HIPCHK(hipHostMalloc((void**)&h_resid, pinned_cap * 8, 0));
      HIPCHK(hipHostMalloc((void**)&h_status, pinned_cap * 4, 0));
    }
    sa.subs = d_subs;
    sa.insts = d_insts;
    sa.dc = d_dc;
    sa.partials = d_partials;
    sa.shift_acc = d_shift;
    sa.status = d_status;
    persist = want_persist && persist_eligible();
    HIPCHK(hipStreamSynchronize(st));
    built = true;
  }

  // launch one phase over the table range [first, first + count)
  void launch_range(int ph, int first, int count, hipStream_t st) {
    if (count <= 0) return;
    const Table& t = tab[ph];
    switch (ph) {
      case 1:
        if (stencil_kind_ == 4)
          HIPCHK(launch_stencil_fwd2(prec, t.d + first, count, count <= lbasis_max ? t.lneed : t.lneed_nb, sa, st));
        else
          HIPCHK(launch_stencil(prec, stencil_kind_, t.d + first, count, sa, st));
        break;
      case 2: HIPCHK(launch_euler(prec, t.d + first, count, part_base_eu + first, sa, st)); break;
      case 3: HIPCHK(launch_fwd_last(prec, t.d + first, count, t.maxld, sa, st)); break;
      case 4:
        if (wide_[4]) HIPCHK(launch_strip4(prec, false, t.d + first, count, t.maxld, 1, 0, 1, sa, st));
        else HIPCHK(launch_strip(prec, false, t.d + first, count, t.maxld, lds_basis(t, count), 1, 0, 1, eight_max, sa, st));
        break;
      case 5:  // 2D: T -> F;  3D: F -> T (pair_src_ set by launch_phase)
        if (wide_[5]) HIPCHK(launch_strip4(prec, true, t.d + first, count, t.maxld, 0, 0, pair_src_, sa, st));
        else HIPCHK(launch_strip(prec, true, t.d + first, count, t.maxld, lds_basis(t, count), 0, 0, pair_src_, eight_max, sa, st));
        break;
      case 6:
        if (wide_[6]) HIPCHK(launch_strip4(prec, false, t.d + first, count, t.maxld, 1, 1, 1, sa, st));
        else HIPCHK(launch_strip(prec, false, t.d + first, count, t.maxld, lds_basis(t, count), 1, 1, 1, eight_max, sa, st));
        break;
      case 7:
        HIPCHK(launch_inv_last(prec, t.d + first, count, t.maxld, part_base_inv + first, eight_max, sa, st));
        break;
    }
  }
  int pair_src_ = 1;
  int stencil_kind_ = 2;

  // One persistent launch per step (form 2): the fused stencil, the axis-0 pair and the inverse
  // last-axis kernel's tile bodies in one kernel with grid-wide barriers between them.  Taken
  // when asked for (want_persist) and the batch allows it: one sweep level, every subdomain 2D,
  // preconditioned and fused, the pair on 16-column strips of regular axes.  Results are
  // bitwise those of the phase launches.
  bool want_persist = false;
  bool persist = false;
  int persist_grid = 0;
  size_t persist_dyn = 0;
  unsigned* d_bar = nullptr;
  std::string persist_why;  // why the batch cannot take the persistent step
  bool persist_eligible() {
    persist_why.clear();
    if (nlev != 1) persist_why = "alternating sweeps";
    for (size_t gs = 0; gs < h_subs.size() && persist_why.empty(); ++gs)
      if (!fused_[gs]) persist_why = "a subdomain is not a fused 2D preconditioned one (3D, forward Euler, or a last axis above 320)";
    if (persist_why.empty() && !h_pull.empty()) persist_why = "transmission by gather";
    if (persist_why.empty() && (wide_[5] || tab[5].maxld > 576)) persist_why = "wide or long axis-0 strips";
    if (persist_why.empty()) {
      // dynamic LDS: the largest tile footprint (with LDS basis copies where they fit), capped by
      // what the kernel's static LDS leaves
      int stat = 0;
      persist_capacity(prec, 0, &stat);
      const size_t cap = (size_t)(160 * 1024 - stat - 4096);
      const size_t el = prec == PMA_FP64 ? 8 : 4, op = 16 * ((size_t)tab[7].maxld + (prec == PMA_FP64 ? 2 : 4)) * el;
      const size_t least = std::max({(size_t)tab[1].lneed_nb, op, 16 * ((size_t)tab[5].maxld + (prec == PMA_FP64 ? 2 : 4)) * el});
      const size_t want = std::max({least, (size_t)tab[1].lneed, (size_t)tab[5].lneed});
      if (least > cap) {
        persist_why = "tiles too large for one kernel's LDS";
      } else {
        persist_dyn = std::min(want, cap);
        // as many workgroups as the largest phase has tiles (a multiple of 8), at most what the
        // device holds at once: fewer arrivals per barrier for small batches
        int most = 0;
        for (int ph : {1, 5, 7}) {
          const Table& t = tab[ph];
          const int p0 = lvl_first[0], p1 = lvl_first[1];
          most = std::max(most, t.rng[order[p1 - 1]].first + t.rng[order[p1 - 1]].count - t.rng[order[p0]].first);
        }
        persist_grid = std::min(persist_capacity(prec, persist_dyn, nullptr) / 8 * 8, (most + 7) / 8 * 8);
        if (persist_grid <= 0) persist_why = "no co-resident grid";
      }
    }
    return persist_why.empty();
  }

  void launch_persist(hipStream_t st) {
    PersistArgs pa{};
    auto total = [&](int ph) {
      const Table& t = tab[ph];
      const int p0 = lvl_first[0], p1 = lvl_first[1];
      return t.rng[order[p1 - 1]].first + t.rng[order[p1 - 1]].count - t.rng[order[p0]].first;
    };
    pa.t_fused = tab[1].d;
    pa.t_pair = tab[5].d;
    pa.t_inv = tab[7].d;
    pa.n_fused = total(1);
    pa.n_pair = total(5);
    pa.n_inv = total(7);
    pa.bar = d_bar;
    pa.pair_src = 1;  // 2D: the pair reads T, writes F
    pa.part_base = part_base_inv;
    pa.lcap = (int)persist_dyn;
    pa.ninst = (int)h_insts.size();
    pa.spin = 1u << 18;  // well under a second per wait: far beyond any phase, still bounded
    HIPCHK(launch_step2_persist(prec, persist_grid, persist_dyn, pa, sa, st));
  }

  // one phase of a step over sweep level L (-1: every level in turn): the level's subdomains in
  // one launch, or one subdomain per launch (plain)
  void launch_phase(int ph, bool plain, hipStream_t st, int L = -1) {
    if (ph == 0) {  // every request's whole transmission list as a gather (timed on its own)
      for (size_t q = 0; q < insts.size(); ++q) {
        const Instance& I = *insts[q];
        const int first = h_insts[q].first_sub;
        if (I.trans.empty()) continue;
        if (!plain) {
          HIPCHK(launch_transmit(prec, d_subs + first, I.trans_dev, (int)I.trans.size(), st));
        } else {
          for (size_t s = 0; s < I.subs.size(); ++s) {
            const int f = I.trans_first[s], n = I.trans_first[s + 1] - f;
            if (n) HIPCHK(launch_transmit(prec, d_subs + first, I.trans_dev + f, n, st));
          }
        }
      }
      return;
    }
    if (L < 0) {
      for (int l = 0; l < nlev; ++l) launch_phase(ph, plain, st, l);
      return;
    }
    const int p0 = lvl_first[L], p1 = lvl_first[L + 1];
    if (p1 <= p0) return;
    const Table& t = tab[ph];
    if (ph == 1 || ph == 5) {
      // 2D, fused 2D and 3D subdomains take different stencil kernels, and the axis-0 pair reads
      // T in 2D and F in 3D: launch the groups separately
      auto key = [&](int p) { return ph == 1 ? stencil_kind(order[p]) : h_subs[order[p]].dim; };
      for (int kv = 2; kv <= 4; ++kv) {
        pair_src_ = kv == 2 ? 1 : 0;
        stencil_kind_ = kv;
        int p = p0;
        while (p < p1) {
          if (key(p) != kv) {
            ++p;
            continue;
          }
          if (plain) {
            launch_range(ph, t.rng[order[p]].first, t.rng[order[p]].count, st);
            ++p;
            continue;
          }
          int e = p;  // contiguous run of subdomains of this kind
          while (e < p1 && key(e) == kv) ++e;
          const int f = t.rng[order[p]].first, l = t.rng[order[e - 1]].first + t.rng[order[e - 1]].count;
          launch_range(ph, f, l - f, st);
          p = e;
        }
      }
      return;
    }
    if (!plain) {
      const int f = t.rng[order[p0]].first, l = t.rng[order[p1 - 1]].first + t.rng[order[p1 - 1]].count;
      launch_range(ph, f, l - f, st);
    } else {
      for (int p = p0; p < p1; ++p) launch_range(ph, t.rng[order[p]].first, t.rng[order[p]].count, st);
    }
  }

  // a step, sweep level by sweep level (one level in the parallel form): the gather of
  // forward-Euler subdomains (the others received their owners' values from the inverse-last
  // kernels that updated those owners), then the stencil and the update
  void launch_step(bool plain, hipStream_t st) {
    if (persist && !plain) {
      launch_persist(st);
      return;
    }
    for (int L = 0; L < nlev; ++L) {
      const int p0 = lvl_first[L], p1 = lvl_first[L + 1];
      if (p1 <= p0) continue;
      if (!plain) {
        const int f = pull_rng[order[p0]].first;
        const int l = pull_rng[order[p1 - 1]].first + pull_rng[order[p1 - 1]].count;
        if (l > f) HIPCHK(launch_transmit(prec, d_subs, d_pull + f, l - f, st));
      } else {
        for (int p = p0; p < p1; ++p) {
          const SubRange& r = pull_rng[order[p]];
          if (r.count) HIPCHK(launch_transmit(prec, d_subs, d_pull + r.first, r.count, st));
        }
      }
      for (int ph = 1; ph < kPhases; ++ph) launch_phase(ph, plain, st, L);
    }
  }

  // algorithmic work per step of each phase: 2 M N K flops per product; compulsory bytes with
  // each operand and result touched once (the DCT matrices are n x n and stay in cache)
  void phase_work(double* flops, double* bytes) const {
    const double el = prec == PMA_FP64 ? 8.0 : 4.0;
    for (int ph = 0; ph < kPhases; ++ph) flops[ph] = bytes[ph] = 0.0;
    for (const Instance* I : insts) bytes[0] += (double)I->trans.size() * 2 * el;
    for (size_t q = 0; q < h_subs.size(); ++q) {
      const SubDev& s = h_subs[q];
      const double n0 = s.n[0], n1 = s.n[1], n2 = s.n[2];
      const double nodes = n0 * n1 * n2;
      bytes[1] += 2 * el * nodes;
      if (tab[2].rng[q].count) {
        bytes[2] += 3 * el * nodes;
        continue;
      }
      const double nl = s.dim == 2 ? n1 : n2;
      if (fused_[q]) {
        flops[1] += 2.0 * nodes * nl;  // the stencil writes T = F A_1 instead of F
      } else {
        flops[3] += 2.0 * nodes * nl;
        bytes[3] += 2 * el * nodes;
      }
      if (s.dim == 3) {
        flops[4] += 2.0 * nodes * n1;
        flops[6] += 2.0 * nodes * n1;
        bytes[4] += 2 * el * nodes;
        bytes[6] += 2 * el * nodes;
      }
      flops[5] += 4.0 * nodes * n0;
      bytes[5] += 2 * el * nodes;
      flops[7] += 2.0 * nodes * nl;
      bytes[7] += 3 * el * nodes;
    }
  }

  // nsteps steps of the batched launches, captured in order into one graph
  void capture(int nsteps, hipGraph_t& g_out, hipGraphExec_t& e_out) {
    hipStream_t st = ctx->stream;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      for (int k = 0; k < nsteps; ++k) launch_step(false, st);
    } catch (...) {
      hipGraph_t g = nullptr;
      hipStreamEndCapture(st, &g);
      if (g) hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(st, &g_out));
    HIPCHK(hipGraphInstantiate(&e_out, g_out, nullptr, nullptr, 0));
  }

  void step(bool plain) {
    hipStream_t st = ctx->stream;
    if (plain || !use_graph) {
      launch_step(plain, st);
    } else {
      if (!gexec) capture(1, graph, gexec);
      HIPCHK(hipGraphLaunch(gexec, st));
    }
  }

  // nsteps steps: the same launches in the same order as nsteps calls of step()
  void steps(bool plain, int nsteps) {
    if (!plain && use_graph) {
      for (; nsteps >= kGraphSteps; nsteps -= kGraphSteps) {
        if (!gexec_n) capture(kGraphSteps, graph_n, gexec_n);
        HIPCHK(hipGraphLaunch(gexec_n, ctx->stream));
      }
      if (nsteps > 1) {
        if (!gexec_r[nsteps]) capture(nsteps, graph_r[nsteps], gexec_r[nsteps]);
        HIPCHK(hipGraphLaunch(gexec_r[nsteps], ctx->stream));
        nsteps = 0;
      }
    }
    for (; nsteps > 0; --nsteps) step(plain);
  }

  // residual + status to pinned host memory (asynchronous)
  void read_progress() {
    hipStream_t st = ctx->stream;
    HIPCHK(launch_resid(d_subs, d_insts, (int)h_insts.size(), d_partials, d_resid, st));
    HIPCHK(hipMemcpyAsync(h_resid, d_resid, h_insts.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_status, d_status, h_insts.size() * 4, hipMemcpyDeviceToHost, st));
  }
};

static int status_code(int bits) {
  if (bits & ST_TANGLED) return PMA_E_TANGLED;
  if (bits & ST_NONFINITE) return PMA_E_NONFINITE;
  if (bits & ST_SYNC) return PMA_E_HIP;  // a grid barrier of the persistent step timed out
  return PMA_OK;
}

// initial state of every subdomain of instance q: phi = Psi0 - |xi|^2/2 from a global FP64 array
// on the device (warm start), from the caller's subdomain buffer (single-subdomain mode), or 0
// (Psi^0 = |xi|^2/2, Sec. 2 eq. incond)
static void init_state(pma_ctx* c, Instance& I, const Batch& B, int q) {
  const int first = B.h_insts[q].first_sub;
  for (size_t s = 0; s < I.subs.size(); ++s) {
    const SubDev& sd = B.h_subs[first + s];
    if (I.single_sub_mode) {
      HIPCHK(launch_phi_from_psi(I.prec, sd, I.user_psi, 0, 0, 0, c->stream));
    } else if (I.psi0_dev) {
      HIPCHK(launch_phi_from_psi(I.prec, sd, I.psi0_dev, 1, I.grid.n[1], I.dim == 3 ? I.grid.n[2] : 1, c->stream));
    } else {
      HIPCHK(hipMemsetAsync(I.phi[s], 0, sub_nodes(I.subs[s]) * I.elem(), c->stream));
    }
  }
  I.initialized = true;
}

// glue + Jacobian checks of instance q (asynchronous).  Mesh, optional Psi and the two minima
// land in the instance's device buffers; a single-subdomain solve writes Psi back instead.
static void finalize_instance(pma_ctx* c, Instance& I, Batch& B, int q, bool want_psi) {
  hipStream_t st = c->stream;
  const int first = B.h_insts[q].first_sub;
  if (I.single_sub_mode) {
    HIPCHK(launch_psi_from_phi(I.prec, B.h_subs[first], I.user_psi, B.d_shift, st));
    return;
  }
  // refresh the artificial nodes so owned nodes next to them see current neighbours
  if (!I.trans.empty()) HIPCHK(launch_transmit(I.prec, B.d_subs + first, I.trans_dev, (int)I.trans.size(), st));
  GlueArgs g{};
  g.subs = B.d_subs;
  g.first_sub = first;
  g.dim = I.dim;
  for (int k = 0; k < 3; ++k) {
    g.parts[k] = I.parts[k];
    g.n[k] = k < I.dim ? I.grid.n[k] : 1;
    g.own[k] = k < I.dim ? I.own_dev[k] : nullptr;
    g.a[k] = k < I.dim ? I.grid.lo[k] : 0;
    g.h[k] = k < I.dim ? (I.grid.hi[k] - I.grid.lo[k]) / (I.grid.n[k] - 1) : 1;
  }
  g.mesh = I.mesh_dev;
  g.psi = want_psi ? I.psi_dev : nullptr;
  g.shift_acc = B.d_shift;
  g.inst = q;
  g.minpart = I.minpart;
  HIPCHK(launch_glue(I.prec, g, st));
  HIPCHK(launch_min_reduce(I.minpart, glue_blocks(I.gnodes()), I.stats_dev, st));
  HIPCHK(launch_cells(I.mesh_dev, I.dim, I.grid.n, I.minpart, st));
  HIPCHK(launch_min_reduce(I.minpart, cell_blocks(I.dim, I.grid.n), I.stats_dev + 1, st));
  MonP<double> mp;
  fill_monitor(I.mon, mp);
  double vol = 1.0, h[3] = {1, 1, 1};
  for (int k = 0; k < I.dim; ++k) {
    vol *= I.grid.hi[k] - I.grid.lo[k];
    h[k] = (I.grid.hi[k] - I.grid.lo[k]) / (I.grid.n[k] - 1);
  }
  if (2 * glue_blocks(I.gnodes()) > I.minpart_n || cell_blocks(I.dim, I.grid.n) > I.minpart_n)
    thr(PMA_E_HIP, "internal: partial-result buffer too small");
  HIPCHK(launch_quality(I.mesh_dev, I.dim, I.grid.n, h, mp, vol, I.theta, I.minpart, I.stats_dev + 2, st));
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static void save_shifts(Batch& B) {
  if (!B.built || B.insts.empty()) return;
  std::vector<double> sh(B.insts.size());
  HIPCHK(hipMemcpy(sh.data(), B.d_shift, sh.size() * 8, hipMemcpyDeviceToHost));
  for (size_t q = 0; q < sh.size(); ++q) B.insts[q]->shift_acc = sh[q];
}

// Run instances (one precision) to their step counts, finishing each as soon as it stops.
// Instances that stop earlier than others leave the shared launches (the batch is rebuilt from
// the survivors; their device state is untouched).
// ext_tab: launch tables in caller-provided device memory of ext_tab_cap bytes and steps launched
// directly (no captured graphs): nothing is allocated on the way
static void run_to_end(pma_ctx* c, const std::vector<Instance*>& all, int prec, bool plain, bool want_psi,
                       char* ext_tab = nullptr, size_t ext_tab_cap = 0) {
  hipStream_t st = c->stream;
  std::vector<Instance*> live = all;
  while (!live.empty()) {
    Batch B;
    B.ctx = c;
    B.prec = prec;
    B.insts = live;
    B.fuse = !plain;  // the plain method keeps one launch per kernel
    if (ext_tab) {
      B.ext_tab = ext_tab;
      B.ext_tab_cap = ext_tab_cap;
      B.use_graph = false;
    }
    B.build();
    for (size_t q = 0; q < live.size(); ++q)
      if (!live[q]->initialized) init_state(c, *live[q], B, (int)q);
    std::vector<char> fin(live.size(), 0);
    bool any = false;
    while (!any) {
      int chunk = 1 << 30;
      int R = 1 << 30;
      for (auto* I : live) {
        chunk = std::min(chunk, I->tm.max_steps - I->steps_done);
        if (I->tm.tol > 0) R = std::min(R, std::max(1, I->tm.resid_every) - I->steps_done % std::max(1, I->tm.resid_every));
      }
      chunk = std::max(0, std::min(chunk, R));
      B.steps(plain, chunk);
      for (auto* I : live) I->steps_done += chunk;
      B.read_progress();
      HIPCHK(hipStreamSynchronize(st));
      for (size_t q = 0; q < live.size(); ++q) {
        Instance& I = *live[q];
        I.resid = B.h_resid[q];
        const int code = status_code(B.h_status[q]);
        if (code != PMA_OK && I.status == PMA_OK) I.status = code;
        const bool conv = I.tm.tol > 0 && chunk > 0 && I.resid <= I.tm.tol;
        if (I.status != PMA_OK || I.steps_done >= I.tm.max_steps || conv) {
          fin[q] = 1;
          any = true;
        }
      }
    }
    save_shifts(B);
    std::vector<Instance*> rest;
    for (size_t q = 0; q < live.size(); ++q) {
      if (!fin[q]) {
        rest.push_back(live[q]);
        continue;
      }
      if (live[q]->status == PMA_OK) finalize_instance(c, *live[q], B, (int)q, want_psi);
    }
    HIPCHK(hipStreamSynchronize(st));
    live.swap(rest);
  }
}

// ------------------------------------------------------------------------------------------
// serving: continuous batching
// ------------------------------------------------------------------------------------------

// Locks: the context's mutex (ctx->mu: the arena, the basis cache, the stream) and the server's
// (mu: queue, states, results).  A thread that holds both takes ctx->mu first, everywhere; the
// caller-side calls (submit, poll, server info) take mu alone.  Admission used to take them in the
// opposite order (mu, then ctx->mu inside the loop), harmless while only the server thread holds
// both, but a deadlock against any second thread that finishes requests in the tick's order.
struct Server {
  pma_ctx* ctx = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<Instance*> queue;                 // submitted, not admitted
  std::vector<Instance*> running;              // admitted (server thread only)
  std::unordered_map<uint64_t, Instance*> all; // every live ticket
  std::unordered_map<uint64_t, int> state;
  int finished = 0;
  size_t arena_used = 0;                       // arena bytes in use, published under mu
  std::unique_ptr<Batch> batch[3];             // per precision
  bool dirty = true;

  void start() { th = std::thread([this] { loop(); }); }

  void shutdown() {
    {
      std::lock_guard<std::mutex> g(mu);
      stop = true;
    }
    cv.notify_all();
    if (th.joinable()) th.join();
    std::lock_guard<std::recursive_mutex> cg(ctx->mu);
    hipStreamSynchronize(ctx->stream);
    for (auto& b : batch) b.reset();
    for (auto& kv : all) {
      free_instance(ctx, *kv.second);
      delete kv.second;
    }
    all.clear();
  }

  size_t request_bytes(const Instance& I) { return Arena::round(instance_bytes(I)) + new_basis_bytes(ctx, I); }

  // admit queued requests in arrival order while they fit (no overtaking); caller holds ctx->mu
  // and mu, in that order.  blocked: true while the head of the queue waits for memory: nothing
  // can be admitted before a running request finishes, so a tick may run until the first of them
  // does
  bool blocked = false;

  void admit_locked() {
    blocked = false;
    while (!queue.empty()) {
      Instance* I = queue.front();
      const size_t need = request_bytes(*I);
      try {
        ensure_arena(ctx);
        // cached bases nobody uses are evicted by the allocation itself, so they do not block
        if (ctx->arena.used() - evictable_basis_bytes(ctx, *I) + need > ctx->arena.size()) {
          blocked = true;
          arena_used = ctx->arena.used();
          break;
        }
        alloc_instance(ctx, *I);
        if (!I->psi0_host.empty()) {
          upload_psi0(ctx, *I, I->psi0_host.data());
          HIPCHK(hipStreamSynchronize(ctx->stream));  // the host copy may go now
          std::vector<double>().swap(I->psi0_host);
        }
      } catch (Err& e) {
        // fragmented or full: wait for running requests to free memory; with none running no
        // memory will come free (the allocation has already evicted every unused basis), so
        // the request fails
        if (e.code == PMA_E_NOMEM && !running.empty()) {
          blocked = true;
          arena_used = ctx->arena.used();
          break;
        }
        I->err = g_err;
        I->status = e.code;
        I->t_done = now_s();
        state[I->ticket] = PMA_FAILED;
        queue.pop_front();
        finished++;
        continue;
      }
      arena_used = ctx->arena.used();
      queue.pop_front();
      I->t_admit = now_s();
      running.push_back(I);
      state[I->ticket] = PMA_RUNNING;
      dirty = true;
    }
  }

  void loop() {
    while (true) {
      {
        std::unique_lock<std::mutex> g(mu);
        cv.wait(g, [&] { return stop || !queue.empty() || !running.empty(); });
        if (stop) return;
      }
      bool idle, wait_for_memory;
      {
        std::lock_guard<std::recursive_mutex> cg(ctx->mu);
        std::lock_guard<std::mutex> g(mu);
        admit_locked();
        idle = running.empty();
        wait_for_memory = blocked;
      }
      if (idle) {
        std::this_thread::sleep_for(std::chrono::microseconds(200));
        continue;
      }
      try {
        tick(wait_for_memory ? kLongTick : kShortTick);
      } catch (Err& e) {
        std::lock_guard<std::recursive_mutex> cg(ctx->mu);
        std::lock_guard<std::mutex> g(mu);
        hipStreamSynchronize(ctx->stream);
        for (auto* I : running) {
          I->err = g_err;
          I->status = e.code;
          I->t_done = now_s();
          state[I->ticket] = PMA_FAILED;
          free_instance(ctx, *I);
          finished++;
        }
        arena_used = ctx->arena.used();
        running.clear();
        for (auto& b : batch) b.reset();
        dirty = true;
      }
    }
  }

  // steps per tick: short while arrivals could be admitted, long (ending when the first running
  // request finishes) while the queue waits for memory
  static constexpr int kShortTick = 32, kLongTick = 64;

  // membership changed: rebuild the launch tables in place; the steps are captured as graphs and
  // replayed for the rest of the membership
  void rebuild() {
    hipStream_t st = ctx->stream;
    for (int p = 0; p < 3; ++p) {
      if (batch[p]) save_shifts(*batch[p]);
      std::vector<Instance*> v;
      for (auto* I : running)
        if (I->prec == p) v.push_back(I);
      if (v.empty()) {
        if (batch[p]) {
          batch[p]->clear_device();
          batch[p]->insts.clear();
        }
        continue;
      }
      if (!batch[p]) batch[p].reset(new Batch);
      batch[p]->ctx = ctx;
      batch[p]->prec = p;
      batch[p]->use_graph = true;
      batch[p]->insts = v;
      batch[p]->build();
      for (size_t q = 0; q < v.size(); ++q)
        if (!v[q]->initialized) init_state(ctx, *v[q], *batch[p], (int)q);
    }
    HIPCHK(hipStreamSynchronize(st));
    dirty = false;
  }

  // advance every running request a few steps in shared launches; finish the ones that end
  void tick(int max_chunk) {
    std::lock_guard<std::recursive_mutex> cg(ctx->mu);
    hipStream_t st = ctx->stream;
    if (dirty) rebuild();
    int chunk = 1 << 30;
    for (auto* I : running) {
      chunk = std::min(chunk, I->tm.max_steps - I->steps_done);
      if (I->tm.tol > 0) {  // a TOL request is checked on its residual cadence
        const int R = std::max(1, I->tm.resid_every);
        chunk = std::min(chunk, R - I->steps_done % R);
      }
    }
    chunk = std::max(0, std::min(chunk, max_chunk));
    for (int p = 0; p < 3; ++p)  // the batches share no data: each takes its run of steps in turn
      if (batch[p] && !batch[p]->insts.empty()) batch[p]->steps(false, chunk);
    for (auto* I : running) I->steps_done += chunk;
    for (int p = 0; p < 3; ++p)
      if (batch[p] && !batch[p]->insts.empty()) batch[p]->read_progress();
    HIPCHK(hipStreamSynchronize(st));
    std::vector<Instance*> done;
    for (int p = 0; p < 3; ++p) {
      if (!batch[p] || batch[p]->insts.empty()) continue;
      for (size_t q = 0; q < batch[p]->insts.size(); ++q) {
        Instance* I = batch[p]->insts[q];
        const int code = status_code(batch[p]->h_status[q]);
        if (code != PMA_OK && I->status == PMA_OK) I->status = code;
        I->resid = batch[p]->h_resid[q];
        const bool conv = I->tm.tol > 0 && chunk > 0 && I->resid <= I->tm.tol;
        if (I->status != PMA_OK || I->steps_done >= I->tm.max_steps || conv) done.push_back(I);
      }
    }
    if (!done.empty()) {
      for (int p = 0; p < 3; ++p)
        if (batch[p] && !batch[p]->insts.empty()) save_shifts(*batch[p]);
      for (auto* I : done) {
        if (I->status != PMA_OK) continue;
        Batch& B = *batch[I->prec];
        const int q = (int)(std::find(B.insts.begin(), B.insts.end(), I) - B.insts.begin());
        finalize_instance(ctx, *I, B, q, I->want_psi);
        I->mesh_host.resize((size_t)I->dim * I->gnodes());
        HIPCHK(hipMemcpyAsync(I->mesh_host.data(), I->mesh_dev, I->mesh_host.size() * 8, hipMemcpyDeviceToHost, st));
        if (I->want_psi) {
          I->psi_host.resize(I->gnodes());
          HIPCHK(hipMemcpyAsync(I->psi_host.data(), I->psi_dev, I->psi_host.size() * 8, hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipMemcpyAsync(I->stats_host, I->stats_dev, 32, hipMemcpyDeviceToHost, st));
      }
      HIPCHK(hipStreamSynchronize(st));
      for (auto* I : done) {
        if (I->status != PMA_OK) continue;
        I->min_det = I->stats_host[0];
        I->min_cell = I->stats_host[1];
        if (!(I->min_det > 0) || !(I->min_cell > 0)) I->status = PMA_E_TANGLED;
      }
      // the finished requests' memory is released below, after the device is done with it
      for (auto& b : batch)
        if (b) {
          b->clear_device();
          b->insts.clear();
        }
      dirty = true;
    }
    std::lock_guard<std::mutex> g(mu);
    for (auto* I : done) {
      I->t_done = now_s();
      state[I->ticket] = I->status == PMA_OK ? PMA_DONE : PMA_FAILED;
      running.erase(std::find(running.begin(), running.end(), I));
      free_instance(ctx, *I);
      finished++;
    }
    arena_used = ctx->arena.used();
    if (!queue.empty()) admit_locked();
  }
};

}  // namespace pma

// ------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------

using namespace pma;

#define API_BEGIN try {
#define API_END                                              \
  }                                                          \
  catch (Err & e) {                                          \
    return e.code;                                           \
  }                                                          \
  catch (std::bad_alloc&) {                                  \
    return fail(PMA_E_NOMEM, "host allocation failed");      \
  }                                                          \
  catch (...) {                                              \
    return fail(PMA_E_INVAL, "unexpected internal error");   \
  }

extern "C" {

const char* pma_last_error(void) { return g_err.c_str(); }

int pma_create(int hip_device, size_t hbm_budget_bytes, pma_ctx** out) {
  API_BEGIN
  if (!out) return fail(PMA_E_INVAL, "out is NULL");
  *out = nullptr;
  int nd = 0;
  if (hipGetDeviceCount(&nd) != hipSuccess || hip_device < 0 || hip_device >= nd)
    return fail(PMA_E_HIP, "no such HIP device %d", hip_device);
  HIPCHK(hipSetDevice(hip_device));
  // the fixed scratch of the allocation-free entry point: its address on this device, looked up
  // once per device with the device current
  if (scratch_init(hip_device) != hipSuccess) return fail(PMA_E_HIP, "device scratch lookup failed");
  pma_ctx* c = new pma_ctx;
  c->device = hip_device;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : ((size_t)8 << 30);
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(PMA_E_HIP, "stream creation failed");
  }
  *out = c;
  return PMA_OK;
  API_END
}

int pma_destroy(pma_ctx* c) {
  API_BEGIN
  if (!c) return PMA_OK;
  if (c->server) {
    c->server->shutdown();
    delete c->server;
    c->server = nullptr;
  }
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  for (auto& kv : c->bases) delete kv.second;  // memory goes with the arena
  c->bases.clear();
  if (c->arena_mem) {
    if (c->arena_from_cb && c->free_cb) c->free_cb(c->arena_mem, (void*)c->stream, c->alloc_user);
    else if (!c->arena_from_cb) hipFree(c->arena_mem);
  }
  if (c->stream) hipStreamDestroy(c->stream);
  delete c;
  return PMA_OK;
  API_END
}

int pma_set_allocator(pma_ctx* c, void* (*alloc)(size_t, void*, void*), void (*free_)(void*, void*, void*),
                      void* user) {
  API_BEGIN
  if (!c || !alloc || !free_) return fail(PMA_E_INVAL, "NULL argument");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->arena.ready()) return fail(PMA_E_INVAL, "allocator must be installed before the first solve");
  c->alloc_cb = alloc;
  c->free_cb = free_;
  c->alloc_user = user;
  return PMA_OK;
  API_END
}

int pma_partition(const pma_grid* grid, const pma_dd* dd, int cap, int* nsub, int* ranges, int* faces) {
  API_BEGIN
  if (!grid || !nsub) return fail(PMA_E_INVAL, "NULL argument");
  std::vector<SubHost> subs;
  int parts[3];
  std::vector<int> own[3];
  partition_host(*grid, dd, subs, parts, own);
  *nsub = (int)subs.size();
  if ((ranges || faces) && (int)subs.size() > cap) return fail(PMA_E_INVAL, "cap too small");
  for (size_t s = 0; s < subs.size(); ++s)
    for (int k = 0; k < 3; ++k) {
      if (ranges) {
        ranges[s * 6 + 2 * k] = subs[s].lo[k];
        ranges[s * 6 + 2 * k + 1] = subs[s].lo[k] + subs[s].n[k] - 1;
      }
      if (faces) {
        faces[s * 6 + 2 * k] = (subs[s].art >> (2 * k)) & 1;
        faces[s * 6 + 2 * k + 1] = (subs[s].art >> (2 * k + 1)) & 1;
      }
    }
  return PMA_OK;
  API_END
}

int pma_sweep_levels(const pma_grid* grid, const pma_dd* dd, int cap, int* nsub, int* levels) {
  API_BEGIN
  if (!grid || !dd || !nsub) return fail(PMA_E_INVAL, "NULL argument");
  Instance I;
  I.grid = *grid;
  I.dd = *dd;
  I.dim = grid->dim;
  I.whole = true;
  for (int k = 0; k < grid->dim && k < 3; ++k)
    if (dd->parts[k] > 1) I.whole = false;
  partition_host(I.grid, dd, I.subs, I.parts, I.own);
  build_coupling(I);
  *nsub = (int)I.subs.size();
  if (levels) {
    if ((int)I.subs.size() > cap) return fail(PMA_E_INVAL, "cap too small");
    for (size_t q = 0; q < I.subs.size(); ++q) levels[q] = I.level[q];
  }
  return PMA_OK;
  API_END
}

int pma_theta(const pma_grid* grid, const pma_monitor* mon, double* out) {
  API_BEGIN
  if (!grid || !mon || !out) return fail(PMA_E_INVAL, "NULL argument");
  validate_grid(*grid);
  validate_monitor(*mon, grid->dim);
  *out = theta_host(*grid, *mon);
  return PMA_OK;
  API_END
}

static void fill_stats(pma_stats* st, const Instance& I, double ms) {
  if (!st) return;
  st->steps_done = I.steps_done;
  st->status = I.status;
  st->final_resid = I.resid;
  st->min_det = I.min_det;
  st->min_cell = I.min_cell;
  st->quality_e2 = I.stats_host[2];
  st->quality_emax = I.stats_host[3];
  st->theta = I.theta;
  st->ms_total = ms;
  st->ms_queue = 0;
}

static void default_dd(Instance& I, const pma_dd* dd) {
  if (dd) I.dd = *dd;
  else {
    for (int k = 0; k < 3; ++k) {
      I.dd.parts[k] = 1;
      I.dd.overlap_cells[k] = 0;
    }
    I.dd.mode = PMA_DD_PARALLEL;
  }
  for (int k = I.grid.dim; k < 3; ++k) I.dd.parts[k] = 1;
}

// copy results of finished instances to the host and apply the final positivity check
static void collect(pma_ctx* c, const std::vector<Instance*>& v, double* const* mesh_outs,
                    double* const* psi_outs) {
  for (size_t q = 0; q < v.size(); ++q) {
    Instance& I = *v[q];
    if (I.status != PMA_OK) continue;
    if (mesh_outs && mesh_outs[q])
      HIPCHK(hipMemcpyAsync(mesh_outs[q], I.mesh_dev, (size_t)I.dim * I.gnodes() * 8, hipMemcpyDeviceToHost, c->stream));
    if (psi_outs && psi_outs[q])
      HIPCHK(hipMemcpyAsync(psi_outs[q], I.psi_dev, I.gnodes() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(I.stats_host, I.stats_dev, 32, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  for (auto* I : v) {
    if (I->status != PMA_OK) continue;
    I->min_det = I->stats_host[0];
    I->min_cell = I->stats_host[1];
    if (!(I->min_det > 0) || !(I->min_cell > 0)) I->status = PMA_E_TANGLED;
  }
}

static int status_fail(int code) {
  return fail(code, code == PMA_E_TANGLED ? "mesh folded (det D^2 Psi <= 0 during a step, or a final cell of "
                                           "non-positive measure)" : "non-finite update");
}

int pma_dd_mesh(pma_ctx* c, const pma_grid* grid, const pma_dd* dd, const pma_monitor* mon, const pma_time* tm,
                const double* psi0, double* mesh_out, double* psi_out, pma_stats* st) {
  API_BEGIN
  if (!c || !grid || !mon || !tm || !mesh_out) return fail(PMA_E_INVAL, "NULL argument");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIPCHK(hipSetDevice(c->device));
  const double t0 = now_s();
  Instance I;
  I.grid = *grid;
  default_dd(I, dd);
  I.mon = *mon;
  I.tm = *tm;
  build_plan(I);
  alloc_instance(c, I);
  int rc = PMA_OK;
  try {
    if (psi0) {
      HIPCHK(hipMemcpyAsync(I.psi_dev, psi0, I.gnodes() * 8, hipMemcpyHostToDevice, c->stream));
      I.psi0_dev = I.psi_dev;
    }
    std::vector<Instance*> v{&I};
    run_to_end(c, v, I.prec, tm->exec == PMA_EXEC_PLAIN, psi_out != nullptr);
    double* mo[1] = {mesh_out};
    double* po[1] = {psi_out};
    collect(c, v, mo, po);
  } catch (Err& e) {
    rc = e.code;
    hipStreamSynchronize(c->stream);
  }
  free_instance(c, I);
  fill_stats(st, I, (now_s() - t0) * 1e3);
  if (rc != PMA_OK) return rc;
  if (I.status != PMA_OK) return status_fail(I.status);
  return PMA_OK;
  API_END
}

int pma_dd_mesh_batch(pma_ctx* c, int count, const pma_request* reqs, double* const* mesh_outs, pma_stats* stats) {
  API_BEGIN
  if (!c || count < 0 || (count && (!reqs || !mesh_outs))) return fail(PMA_E_INVAL, "bad arguments");
  if (count == 0) return PMA_OK;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIPCHK(hipSetDevice(c->device));
  const double t0 = now_s();
  std::vector<std::unique_ptr<Instance>> insts;
  const int prec = reqs[0].time.precision;
  for (int i = 0; i < count; ++i) {
    std::unique_ptr<Instance> I(new Instance);
    I->grid = reqs[i].grid;
    default_dd(*I, &reqs[i].dd);
    I->mon = reqs[i].mon;
    I->tm = reqs[i].time;
    if (I->tm.precision != prec) return fail(PMA_E_INVAL, "all requests of a batch must share the precision");
    build_plan(*I);
    insts.push_back(std::move(I));
  }
  int rc = PMA_OK;
  std::vector<Instance*> raw;
  try {
    for (size_t i = 0; i < insts.size(); ++i) {
      Instance& I = *insts[i];
      alloc_instance(c, I);
      raw.push_back(&I);
      upload_psi0(c, I, reqs[i].psi0);
    }
    run_to_end(c, raw, prec, reqs[0].time.exec == PMA_EXEC_PLAIN, false);
    collect(c, raw, mesh_outs, nullptr);
  } catch (Err& e) {
    rc = e.code;
    hipStreamSynchronize(c->stream);
  }
  const double ms = (now_s() - t0) * 1e3;
  for (int q = 0; q < (int)raw.size(); ++q) {
    if (stats) fill_stats(&stats[q], *raw[q], ms);
    if (raw[q]->status != PMA_OK && rc == PMA_OK) rc = raw[q]->status;
  }
  for (auto* I : raw) free_instance(c, *I);
  if (rc != PMA_OK) return fail(rc, "at least one request of the batch failed (%d)", rc);
  return PMA_OK;
  API_END
}

}  // extern "C"

namespace pma {

// the context's stream replaced by another for the duration of a call (under the context lock)
struct StreamSwap {
  pma_ctx* c;
  hipStream_t saved;
  StreamSwap(pma_ctx* c_, hipStream_t s) : c(c_), saved(c_->stream) { c->stream = s; }
  ~StreamSwap() { c->stream = saved; }
};

static int solve_subdomain(pma_ctx* c, const pma_grid* global, const int lo[3], const int hi[3],
                           const int face_kind[6], const pma_monitor* mon, const pma_time* tm, void* psi_dev,
                           void* hip_stream, pma_stats* st, bool noalloc);

}  // namespace pma

extern "C" {

int pma_solve_subdomain(pma_ctx* c, const pma_grid* global, const int lo[3], const int hi[3], const int face_kind[6],
                        const pma_monitor* mon, const pma_time* tm, void* psi_dev, void* hip_stream, pma_stats* st) {
  return solve_subdomain(c, global, lo, hi, face_kind, mon, tm, psi_dev, hip_stream, st, false);
}

int pma_solve_subdomain_noalloc(pma_ctx* c, const pma_grid* global, const int lo[3], const int hi[3],
                                const int face_kind[6], const pma_monitor* mon, const pma_time* tm, void* psi_dev,
                                void* hip_stream, pma_stats* st) {
  return solve_subdomain(c, global, lo, hi, face_kind, mon, tm, psi_dev, hip_stream, st, true);
}

}  // extern "C"

namespace pma {

static int solve_subdomain(pma_ctx* c, const pma_grid* global, const int lo[3], const int hi[3],
                           const int face_kind[6], const pma_monitor* mon, const pma_time* tm, void* psi_dev,
                           void* hip_stream, pma_stats* st, bool noalloc) {
  API_BEGIN
  if (!c || !global || !lo || !hi || !face_kind || !mon || !tm || !psi_dev) return fail(PMA_E_INVAL, "NULL argument");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIPCHK(hipSetDevice(c->device));
  const double t0 = now_s();
  validate_grid(*global);
  Instance I;
  I.grid = *global;
  I.mon = *mon;
  I.tm = *tm;
  I.single_sub_mode = true;
  I.dim = global->dim;
  validate_monitor(I.mon, I.dim);
  validate_time(I.tm);
  I.prec = tm->precision;
  SubHost S;
  for (int k = 0; k < I.dim; ++k) {
    if (lo[k] < 0 || hi[k] > global->n[k] - 1 || hi[k] - lo[k] < 4 || hi[k] - lo[k] + 1 > kMaxAxisNodes)
      return fail(PMA_E_INVAL, "bad subdomain range");
    S.lo[k] = lo[k];
    S.n[k] = hi[k] - lo[k] + 1;
    for (int e = 0; e < 2; ++e) {
      const int fk = face_kind[2 * k + e];
      const bool on_box = e == 0 ? lo[k] == 0 : hi[k] == global->n[k] - 1;
      if (fk == PMA_FACE_ARTIFICIAL) S.art |= 1 << (2 * k + e);
      else if (fk != PMA_FACE_NEUMANN || !on_box)
        return fail(PMA_E_INVAL, "Neumann faces must lie on the box boundary");
    }
  }
  I.subs = {S};
  I.trans_first = {0, 0};
  I.level = {0};
  I.nlevels = 1;
  I.theta = mon->theta > 0 ? mon->theta : theta_host(I.grid, I.mon);
  I.user_psi = (double*)psi_dev;
  hipStream_t user = (hipStream_t)hip_stream;
  if (noalloc) {
    // everything in the fixed scratch of this device, kernels on the caller's stream, steps
    // launched directly: no device, pinned-host or graph allocation, no event
    char* scr = (char*)scratch_ptr(c->device);
    if (!scr) return fail(PMA_E_HIP, "device scratch of device %d not set up", c->device);
    // state and DCT matrices first, launch tables and reduction buffers (well under
    // kScratchTables for one subdomain) after them
    constexpr size_t kScratchTables = (size_t)1 << 20;
    const size_t need = instance_bytes_with_bases(I);
    if (need > kScratchBytes - kScratchTables)
      return fail(PMA_E_INVAL, "subdomain needs %zu bytes of state and DCT matrices; the allocation-free entry point "
                  "holds at most %zu (use pma_solve_subdomain)", need, kScratchBytes - kScratchTables);
    int rc = PMA_OK;
    {
      StreamSwap sw(c, user);
      try {
        const size_t used = alloc_instance(c, I, scr, kScratchBytes - kScratchTables);
        std::vector<Instance*> v{&I};
        run_to_end(c, v, I.prec, tm->exec == PMA_EXEC_PLAIN, false, scr + used, kScratchBytes - used);
        HIPCHK(hipStreamSynchronize(user));
      } catch (Err& e) {
        rc = e.code;
        hipStreamSynchronize(user);
      }
    }
    free_instance(c, I);
    fill_stats(st, I, (now_s() - t0) * 1e3);
    if (rc != PMA_OK) return rc;
    if (I.status != PMA_OK) return status_fail(I.status);
    return PMA_OK;
  }
  alloc_instance(c, I);
  int rc = PMA_OK;
  hipEvent_t ev = nullptr;
  try {
    // the work runs after what the caller queued on its stream, and the caller's stream waits
    // for the result
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, user));
    HIPCHK(hipStreamWaitEvent(c->stream, ev, 0));
    std::vector<Instance*> v{&I};
    run_to_end(c, v, I.prec, tm->exec == PMA_EXEC_PLAIN, false);
    HIPCHK(hipEventRecord(ev, c->stream));
    HIPCHK(hipStreamWaitEvent(user, ev, 0));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipStreamSynchronize(user));
  } catch (Err& e) {
    rc = e.code;
    hipStreamSynchronize(c->stream);
  }
  if (ev) hipEventDestroy(ev);
  free_instance(c, I);
  fill_stats(st, I, (now_s() - t0) * 1e3);
  if (rc != PMA_OK) return rc;
  if (I.status != PMA_OK) return status_fail(I.status);
  return PMA_OK;
  API_END
}

}  // namespace pma

// ---- resident plans -------------------------------------------------------------------------


struct pma_plan {
  pma_ctx* ctx = nullptr;
  std::vector<std::unique_ptr<pma::Instance>> insts;
  std::unique_ptr<pma::Batch> batch;
  bool plain = false;
};

extern "C" {

int pma_plan_create(pma_ctx* c, int count, const pma_request* reqs, pma_plan** out) {
  API_BEGIN
  if (!c || count <= 0 || !reqs || !out) return fail(PMA_E_INVAL, "bad arguments");
  *out = nullptr;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIPCHK(hipSetDevice(c->device));
  std::unique_ptr<pma_plan> P(new pma_plan);
  P->ctx = c;
  const int prec = reqs[0].time.precision;
  P->plain = reqs[0].time.exec == PMA_EXEC_PLAIN;
  for (int i = 0; i < count; ++i) {
    std::unique_ptr<Instance> I(new Instance);
    I->grid = reqs[i].grid;
    default_dd(*I, &reqs[i].dd);
    I->mon = reqs[i].mon;
    I->tm = reqs[i].time;
    if (I->tm.precision != prec) return fail(PMA_E_INVAL, "all requests of a plan must share the precision");
    build_plan(*I);
    P->insts.push_back(std::move(I));
  }
  std::vector<Instance*> raw;
  try {
    for (size_t i = 0; i < P->insts.size(); ++i) {
      alloc_instance(c, *P->insts[i]);
      raw.push_back(P->insts[i].get());
      upload_psi0(c, *P->insts[i], reqs[i].psi0);
    }
    P->batch.reset(new Batch);
    P->batch->fuse = !P->plain;  // the plain method keeps one launch per kernel
    P->batch->ctx = c;
    P->batch->prec = prec;
    P->batch->insts = raw;
    P->batch->build();
    for (size_t q = 0; q < raw.size(); ++q) init_state(c, *raw[q], *P->batch, (int)q);
    HIPCHK(hipStreamSynchronize(c->stream));
  } catch (Err& e) {
    hipStreamSynchronize(c->stream);
    P->batch.reset();
    for (auto* I : raw) free_instance(c, *I);
    return e.code;
  }
  *out = P.release();
  return PMA_OK;
  API_END
}

int pma_plan_step(pma_plan* P, int nsteps) {
  API_BEGIN
  if (!P || nsteps < 0) return fail(PMA_E_INVAL, "bad arguments");
  std::lock_guard<std::recursive_mutex> g(P->ctx->mu);
  P->batch->steps(P->plain, nsteps);
  for (auto& I : P->insts) I->steps_done += nsteps;
  return PMA_OK;
  API_END
}

int pma_plan_sync(pma_plan* P) {
  API_BEGIN
  if (!P) return fail(PMA_E_INVAL, "bad arguments");
  std::lock_guard<std::recursive_mutex> g(P->ctx->mu);
  P->batch->read_progress();
  HIPCHK(hipStreamSynchronize(P->ctx->stream));
  int rc = PMA_OK;
  for (size_t q = 0; q < P->insts.size(); ++q) {
    Instance& I = *P->insts[q];
    I.resid = P->batch->h_resid[q];
    const int code = status_code(P->batch->h_status[q]);
    if (code != PMA_OK && I.status == PMA_OK) I.status = code;
    if (I.status != PMA_OK && rc == PMA_OK) rc = I.status;
  }
  if (rc != PMA_OK) return status_fail(rc);
  return PMA_OK;
  API_END
}

int pma_plan_phase_times(pma_plan* P, int nsteps, double* ms, double* flops, double* bytes, int cap, int* nph) {
  API_BEGIN
  if (!P || nsteps <= 0 || !ms || cap < kPhases || !nph) return fail(PMA_E_INVAL, "bad arguments");
  std::lock_guard<std::recursive_mutex> g(P->ctx->mu);
  *nph = kPhases;
  Batch& B = *P->batch;
  pma_ctx* c = P->ctx;
  hipStream_t st = c->stream;
  // snapshot the state every phase may change (phi, accumulated shifts), restored afterwards
  size_t snap = 0;
  for (auto& I : P->insts)
    for (auto& sub : I->subs) snap += Arena::round(sub_nodes(sub) * I->elem());
  snap += Arena::round(P->insts.size() * 8);
  char* save = (char*)arena_alloc(c, snap);
  auto copy_state = [&](bool out) {
    char* q = save;
    for (auto& I : P->insts)
      for (size_t s = 0; s < I->subs.size(); ++s) {
        const size_t b = sub_nodes(I->subs[s]) * I->elem();
        HIPCHK(hipMemcpyAsync(out ? (void*)q : I->phi[s], out ? I->phi[s] : (void*)q, b, hipMemcpyDeviceToDevice, st));
        q += Arena::round(b);
      }
    HIPCHK(hipMemcpyAsync(out ? (void*)q : (void*)B.d_shift, out ? (void*)B.d_shift : (void*)q, P->insts.size() * 8,
                          hipMemcpyDeviceToDevice, st));
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  try {
    copy_state(true);
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // each phase alone, nsteps launches back to back between two events on the kernels' stream
    for (int ph = 0; ph < kPhases; ++ph) {
      B.launch_phase(ph, P->plain, st);  // warm
      HIPCHK(hipEventRecord(e0, st));
      for (int k = 0; k < nsteps; ++k) B.launch_phase(ph, P->plain, st);
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, e0, e1));
      ms[ph] = t / nsteps;
    }
    if (cap > kPhases) {  // the FP64 residual reduction (every R steps, and at the end)
      const int ni = (int)B.h_insts.size();
      HIPCHK(launch_resid(B.d_subs, B.d_insts, ni, B.d_partials, B.d_resid, st));
      HIPCHK(hipEventRecord(e0, st));
      for (int k = 0; k < nsteps; ++k) HIPCHK(launch_resid(B.d_subs, B.d_insts, ni, B.d_partials, B.d_resid, st));
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, e0, e1));
      ms[kPhases] = t / nsteps;
    }
    copy_state(false);
    HIPCHK(hipStreamSynchronize(st));
  } catch (Err&) {
    hipStreamSynchronize(st);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    c->arena.release(save);
    throw;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->arena.release(save);
  std::vector<double> fl(kPhases, 0.0), by(kPhases, 0.0);
  B.phase_work(fl.data(), by.data());
  for (int ph = 0; ph < kPhases; ++ph) {
    if (flops) flops[ph] = fl[ph];
    if (bytes) bytes[ph] = by[ph];
  }
  if (cap > kPhases) {
    *nph = kPhases + 1;
    if (flops) flops[kPhases] = (double)B.npartials;
    if (bytes) bytes[kPhases] = (double)B.npartials * 8.0;
  }
  return PMA_OK;
  API_END
}

int pma_plan_set_fusion(pma_plan* P, int on) {
  API_BEGIN
  if (!P) return fail(PMA_E_INVAL, "bad arguments");
  std::lock_guard<std::recursive_mutex> g(P->ctx->mu);
  for (auto& I : P->insts)
    if (I->steps_done > 0) return fail(PMA_E_INVAL, "fusion can only be changed before the first step");
  P->batch->fuse = on != 0;
  P->batch->build();
  return PMA_OK;
  API_END
}

int pma_plan_set_persistent(pma_plan* P, int on) {
  API_BEGIN
  if (!P) return fail(PMA_E_INVAL, "bad arguments");
  std::lock_guard<std::recursive_mutex> g(P->ctx->mu);
  if (P->plain) return fail(PMA_E_INVAL, "the plain form launches one subdomain per kernel");
  Batch& B = *P->batch;
  if (on && !B.persist_eligible()) return fail(PMA_E_INVAL, "no persistent step for this plan: %s", B.persist_why.c_str());
  B.want_persist = on != 0;
  B.persist = B.want_persist;
  B.drop_graphs();
  return PMA_OK;
  API_END
}

int pma_plan_set_wide_strips(pma_plan* P, int on) {
  API_BEGIN
  if (!P) return fail(PMA_E_INVAL, "bad arguments");
  std::lock_guard<std::recursive_mutex> g(P->ctx->mu);
  for (auto& I : P->insts)
    if (I->steps_done > 0) return fail(PMA_E_INVAL, "strip width can only be changed before the first step");
  P->batch->wide_ok = on != 0;
  P->batch->build();
  return PMA_OK;
  API_END
}

int pma_plan_set_march(pma_plan* P, int march) {
  API_BEGIN
  if (!P || march < 1 || march > 4096) return fail(PMA_E_INVAL, "march must be in 1..4096");
  std::lock_guard<std::recursive_mutex> g(P->ctx->mu);
  P->batch->set_stencil_march(march);
  return PMA_OK;
  API_END
}

int pma_plan_autotune(pma_plan* P, int reps, int* march, double* ms, int cap, int* ncand) {
  API_BEGIN
  if (!P || reps <= 0 || !march) return fail(PMA_E_INVAL, "bad arguments");
  std::lock_guard<std::recursive_mutex> g(P->ctx->mu);
  Batch& B = *P->batch;
  hipStream_t st = P->ctx->stream;
  // the longest useful march: every subdomain's axis 0 in one workgroup
  int most = 1;
  for (const SubDev& sd : B.h_subs) most = std::max(most, sd.dim == 2 ? (sd.n[0] + kStChunk - 1) / kStChunk : sd.n[0]);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = B.st_march, k = 0;
  double best_ms = 1e300;
  try {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int m = 1;; m *= 2) {
      const int cand = std::min(m, most);
      B.set_stencil_march(cand);
      B.launch_phase(1, P->plain, st);  // warm
      HIPCHK(hipEventRecord(e0, st));
      for (int r = 0; r < reps; ++r) B.launch_phase(1, P->plain, st);
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, e0, e1));
      const double per = (double)t / reps;
      if (ms && k < cap) ms[k] = per;
      ++k;
      if (per < best_ms) {
        best_ms = per;
        best = cand;
      }
      if (cand == most || m >= 64) break;
    }
    B.set_stencil_march(best);
  } catch (Err&) {
    hipStreamSynchronize(st);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    throw;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *march = best;
  if (ncand) *ncand = k;
  return PMA_OK;
  API_END
}

}  // extern "C"

namespace pma {

// the tuning cache's key: the device, the precision and coarse buckets of the plan's shape
static std::string tune_key(const pma_plan* P) {
  const Batch& B = *P->batch;
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, P->ctx->device) != hipSuccess) thr(PMA_E_HIP, "device query failed");
  long nodes = 0, subs = (long)B.h_subs.size();
  int maxld = 0, dims = 0, euler = 0;
  for (const SubDev& sd : B.h_subs) {
    nodes += (long)sd.n[0] * sd.n[1] * sd.n[2];
    for (int k = 0; k < sd.dim; ++k) maxld = std::max(maxld, (sd.n[k] + 31) / 32 * 32);
    dims |= 1 << sd.dim;
    euler |= P->insts[sd.inst]->tm.gamma == 0.0;
  }
  auto pow2 = [](long v) { long p = 1; while (p < v) p <<= 1; return p; };
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s|prec%d|%s|subs%ld|nodes%ld|ld%d|dims%d|euler%d|levels%d", prop.gcnArchName, B.prec,
                P->plain ? "plain" : "batched", pow2(subs), pow2(nodes), maxld, dims, euler, B.nlev);
  return buf;
}

struct TuneChoice {
  int march = 1, persistent = 0, eight_max = 512, lbasis_max = kLdsBasisMaxTiles;
  double ms = 0;
};

static bool tune_cache_find(const char* path, const std::string& key, TuneChoice& c) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    char k[300];
    TuneChoice t;
    if (std::sscanf(line, "%299[^\t]\t%d\t%d\t%d\t%d\t%lf", k, &t.march, &t.persistent, &t.eight_max,
                    &t.lbasis_max, &t.ms) == 6 && key == k) {
      c = t;  // the last entry for the key wins
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

static void tune_cache_add(const char* path, const std::string& key, const TuneChoice& c) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) thr(PMA_E_INVAL, "tuning cache: cannot open the file for appending");
  std::fprintf(f, "%s\t%d\t%d\t%d\t%d\t%.6f\n", key.c_str(), c.march, c.persistent, c.eight_max, c.lbasis_max, c.ms);
  std::fclose(f);
}

static void apply_choice(pma_plan* P, const TuneChoice& c) {
  Batch& B = *P->batch;
  B.set_stencil_march(c.march);
  B.eight_max = c.eight_max;
  B.lbasis_max = c.lbasis_max;
  B.want_persist = c.persistent != 0 && !P->plain && B.persist_eligible();
  B.persist = B.want_persist;
  B.drop_graphs();
}

}  // namespace pma

extern "C" {

int pma_plan_tune(pma_plan* P, int reps, const char* cache_path, pma_tuning* out) {
  API_BEGIN
  if (!P || reps <= 0 || !out) return fail(PMA_E_INVAL, "bad arguments");
  std::lock_guard<std::recursive_mutex> g(P->ctx->mu);
  *out = pma_tuning{};
  const std::string key = tune_key(P);
  TuneChoice best;
  if (tune_cache_find(cache_path, key, best)) {
    apply_choice(P, best);
    out->march = best.march;
    out->persistent = P->batch->persist ? 1 : 0;
    out->eight_max = best.eight_max;
    out->lbasis_max = best.lbasis_max;
    out->step_ms = best.ms;
    out->from_cache = 1;
    return PMA_OK;
  }
  // the stencil's launch shape on its own (it writes only F), then whole steps of every launch
  // configuration on a copy of the state, restored afterwards
  int march = 1;
  const int rc = pma_plan_autotune(P, reps, &march, nullptr, 0, nullptr);
  if (rc != PMA_OK) return rc;
  Batch& B = *P->batch;
  pma_ctx* c = P->ctx;
  hipStream_t st = c->stream;
  size_t snap = 0;
  for (auto& I : P->insts)
    for (auto& sub : I->subs) snap += Arena::round(sub_nodes(sub) * I->elem());
  snap += 2 * Arena::round(P->insts.size() * 8);
  char* save = (char*)arena_alloc(c, snap);
  auto copy_state = [&](bool out_) {
    char* q = save;
    for (auto& I : P->insts)
      for (size_t s2 = 0; s2 < I->subs.size(); ++s2) {
        const size_t b = sub_nodes(I->subs[s2]) * I->elem();
        HIPCHK(hipMemcpyAsync(out_ ? (void*)q : I->phi[s2], out_ ? I->phi[s2] : (void*)q, b, hipMemcpyDeviceToDevice, st));
        q += Arena::round(b);
      }
    HIPCHK(hipMemcpyAsync(out_ ? (void*)q : (void*)B.d_shift, out_ ? (void*)B.d_shift : (void*)q, P->insts.size() * 8,
                          hipMemcpyDeviceToDevice, st));
    q += Arena::round(P->insts.size() * 8);
    HIPCHK(hipMemcpyAsync(out_ ? (void*)q : (void*)B.d_status, out_ ? (void*)B.d_status : (void*)q, P->insts.size() * 4,
                          hipMemcpyDeviceToDevice, st));
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int ncand = 0;
  best.ms = 1e300;
  try {
    copy_state(true);
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const bool can_persist = !P->plain && B.persist_eligible();
    for (int pers = 0; pers <= (can_persist ? 1 : 0); ++pers)
      for (int em : {0, 512, 1 << 30})
        for (int lm : {0, (int)kLdsBasisMaxTiles, 1 << 30}) {
          TuneChoice t;
          t.march = march;
          t.persistent = pers;
          t.eight_max = em;
          t.lbasis_max = lm;
          apply_choice(P, t);
          B.launch_step(P->plain, st);  // warm
          HIPCHK(hipEventRecord(e0, st));
          for (int r = 0; r < reps; ++r) B.launch_step(P->plain, st);
          HIPCHK(hipEventRecord(e1, st));
          HIPCHK(hipEventSynchronize(e1));
          float ms = 0;
          HIPCHK(hipEventElapsedTime(&ms, e0, e1));
          t.ms = (double)ms / reps;
          ++ncand;
          if (t.ms < best.ms) best = t;
          copy_state(false);
          copy_state(true);
        }
    copy_state(false);
    HIPCHK(hipStreamSynchronize(st));
  } catch (Err&) {
    hipStreamSynchronize(st);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    c->arena.release(save);
    throw;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->arena.release(save);
  apply_choice(P, best);
  tune_cache_add(cache_path, key, best);
  out->march = best.march;
  out->persistent = B.persist ? 1 : 0;
  out->eight_max = best.eight_max;
  out->lbasis_max = best.lbasis_max;
  out->step_ms = best.ms;
  out->from_cache = 0;
  out->candidates = ncand;
  return PMA_OK;
  API_END
}

int pma_plan_mesh(pma_plan* P, int i, double* mesh_out, pma_stats* st) {
  API_BEGIN
  if (!P || i < 0 || i >= (int)P->insts.size() || !mesh_out) return fail(PMA_E_INVAL, "bad arguments");
  std::lock_guard<std::recursive_mutex> g(P->ctx->mu);
  Instance& I = *P->insts[i];
  P->batch->read_progress();
  HIPCHK(hipStreamSynchronize(P->ctx->stream));
  I.resid = P->batch->h_resid[i];
  const int code = status_code(P->batch->h_status[i]);
  if (code != PMA_OK && I.status == PMA_OK) I.status = code;
  if (I.status == PMA_OK) {
    finalize_instance(P->ctx, I, *P->batch, i, false);
    std::vector<Instance*> v{&I};
    double* mo[1] = {mesh_out};
    collect(P->ctx, v, mo, nullptr);
  }
  fill_stats(st, I, 0.0);
  if (I.status != PMA_OK) return status_fail(I.status);
  return PMA_OK;
  API_END
}

int pma_plan_destroy(pma_plan* P) {
  API_BEGIN
  if (!P) return PMA_OK;
  {
    std::lock_guard<std::recursive_mutex> g(P->ctx->mu);
    hipStreamSynchronize(P->ctx->stream);
    P->batch.reset();
    for (auto& I : P->insts) free_instance(P->ctx, *I);
  }
  delete P;
  return PMA_OK;
  API_END
}

// a request's instance with its plan built (validates the request)
static std::unique_ptr<Instance> planned_request(const pma_request* req) {
  std::unique_ptr<Instance> I(new Instance);
  I->grid = req->grid;
  I->dd = req->dd;
  for (int k = I->grid.dim; k < 3; ++k) I->dd.parts[k] = 1;
  I->mon = req->mon;
  I->tm = req->time;
  I->arrival_s = req->arrival_s;
  build_plan(*I);
  return I;
}

int pma_request_bytes(const pma_request* req, size_t* bytes) {
  API_BEGIN
  if (!req || !bytes) return fail(PMA_E_INVAL, "NULL argument");
  std::unique_ptr<Instance> I = planned_request(req);
  *bytes = Arena::round(instance_bytes(*I)) + all_basis_bytes(*I);
  return PMA_OK;
  API_END
}

int pma_submit(pma_ctx* c, const pma_request* req, uint64_t* ticket) {
  API_BEGIN
  if (!c || !req || !ticket) return fail(PMA_E_INVAL, "NULL argument");
  std::unique_ptr<Instance> I = planned_request(req);
  // budget check without the context lock (the server thread holds it while it steps): the
  // bound counts every DCT basis the request uses, cached or not
  const size_t need = Arena::round(instance_bytes(*I)) + all_basis_bytes(*I);
  if (need > c->budget) return fail(PMA_E_BUDGET, "request needs %zu bytes, budget is %zu", need, c->budget);
  if (req->psi0) I->psi0_host.assign(req->psi0, req->psi0 + I->gnodes());
  I->want_psi = req->want_psi != 0;
  {
    std::lock_guard<std::mutex> g(c->server_mu);
    if (!c->server) {
      c->server = new Server;
      c->server->ctx = c;
      c->server->start();
    }
  }
  Server* s = c->server;
  {
    std::lock_guard<std::mutex> g(s->mu);
    I->ticket = s->next_ticket++;
    I->t_submit = now_s();
    *ticket = I->ticket;
    s->state[I->ticket] = PMA_PENDING;
    s->all[I->ticket] = I.get();
    s->queue.push_back(I.release());
  }
  s->cv.notify_all();
  return PMA_OK;
  API_END
}

int pma_poll(pma_ctx* c, uint64_t ticket, int* state, double* mesh_out, pma_stats* st) {
  return pma_poll_psi(c, ticket, state, mesh_out, nullptr, st);
}

int pma_poll_psi(pma_ctx* c, uint64_t ticket, int* state, double* mesh_out, double* psi_out, pma_stats* st) {
  API_BEGIN
  if (!c || !state) return fail(PMA_E_INVAL, "NULL argument");
  Server* s = c->server;
  if (!s) return fail(PMA_E_NOTFOUND, "unknown ticket");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->state.find(ticket);
  if (it == s->state.end()) return fail(PMA_E_NOTFOUND, "unknown ticket");
  if (psi_out && !s->all[ticket]->want_psi) return fail(PMA_E_INVAL, "the request was submitted without want_psi");
  *state = it->second;
  if (*state == PMA_DONE || *state == PMA_FAILED) {
    Instance* I = s->all[ticket];
    if (*state == PMA_DONE && mesh_out) std::memcpy(mesh_out, I->mesh_host.data(), I->mesh_host.size() * 8);
    if (*state == PMA_DONE && psi_out) std::memcpy(psi_out, I->psi_host.data(), I->psi_host.size() * 8);
    if (*state == PMA_FAILED)  // the cause, readable through pma_last_error on the caller's thread
      fail(I->status, "%s", I->err.empty() ? (I->status == PMA_E_TANGLED ? "mesh folded" : I->status == PMA_E_NONFINITE
                                                                                          ? "non-finite update"
                                                                                          : "request failed")
                                           : I->err.c_str());
    if (st) {
      fill_stats(st, *I, (I->t_done - I->t_submit) * 1e3);
      st->ms_queue = (I->t_admit > 0 ? I->t_admit - I->t_submit : 0) * 1e3;
    }
    s->all.erase(ticket);
    s->state.erase(it);
    delete I;
  }
  return PMA_OK;
  API_END
}

int pma_server_info(pma_ctx* c, int* queued, int* running, int* finished, size_t* bytes) {
  API_BEGIN
  if (!c) return fail(PMA_E_INVAL, "NULL argument");
  Server* s = c->server;
  if (!s) {
    if (queued) *queued = 0;
    if (running) *running = 0;
    if (finished) *finished = 0;
    if (bytes) *bytes = 0;
    return PMA_OK;
  }
  std::lock_guard<std::mutex> g(s->mu);
  if (queued) *queued = (int)s->queue.size();
  if (running) *running = (int)s->running.size();
  if (finished) *finished = s->finished;
  if (bytes) *bytes = s->arena_used;
  return PMA_OK;
  API_END
}

}  // extern "C"
