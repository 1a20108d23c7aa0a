// Device-visible descriptors shared by the host runtime and the HIP kernels.
//
// Layout of a (sub)domain in HBM: node (i0, i1[, i2]) of an n0 x n1 [x n2] box is element
// (i0 * n1 + i1) [* n2 + i2] (last axis fastest).  Each subdomain owns three arrays of that
// shape in the working precision:
//   phi  the state phi = Psi - |xi|^2 / 2 (so grad Psi = xi + grad phi, D^2 Psi = I + D^2 phi,
//        and the Neumann condition of Sec. 2 eq. nbd becomes a plain mirror for phi)
//   F    the right-hand side, then the spectral coefficients
//   T    scratch for the mode products of the preconditioner
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace pma {

enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_SPLIT16 = 2 };

enum MonKind {
  MON_CONST = 0, MON_RADIAL = 1, MON_SINE = 2, MON_GAUSS = 3, MON_SEPARABLE = 4,
  MON_ARC_FRONT = 5, MON_ARC_SPIRAL = 6, MON_ARC_SPHERES = 7
};
constexpr int kMaxBumps = 9;

// status bits raised by kernels (per instance)
enum { ST_TANGLED = 1, ST_NONFINITE = 2, ST_SYNC = 4 };  // ST_SYNC: a grid barrier wait timed out

// Monitor parameters, precomputed on the host in the working precision:
//   rho = amp                                              (MON_CONST)
//   rho = 1 + amp sech^2(k (|x - c|^2 - r02))              (MON_RADIAL, r02 = r0^2)
//   rho = 1 + amp sech^2(k (x_1 - c_1 - r0 sin(2 pi x_0)))  (MON_SINE)
//   rho = 1 + sum_b bamp_b exp(bnh_b |x - bc_b|^2)          (MON_GAUSS, bnh = -1 / (2 w^2))
//   rho = prod_k (1 + aa_k sech^2(ka_k (x_k - c_k)))        (MON_SEPARABLE)
// and the arc-length monitors rho = sqrt(1 + |grad u|^2) (Sec. 4, eq. monitfn) of
//   u = 1 / (1 + exp((x_0 + x_1 - r0) / (2 k)))             (MON_ARC_FRONT, k = eps)
//   u = 1 + amp / (1 + k r^2 cos^2(t - tw r^2)), polar about c  (MON_ARC_SPIRAL)
//   u = sum_b tanh(k (|x - bc_b|^2 - r02))                  (MON_ARC_SPHERES)
template <typename T>
struct MonP {
  int kind, nb;
  T amp, k, r0, r02, tw;
  T c[3], aa[3], ka[3];
  T bamp[kMaxBumps], bnh[kMaxBumps], bc[kMaxBumps][3];
};

// DCT-I basis of one axis of a subdomain, in the precision of the solve.  Matrices have
// round_up(n, 16) rows of ld = round_up(n, 32) entries, zero padded, row-major with row stride
// ldb; both are symmetric, so row j also serves as column j.
struct AxisDev {
  const void* fwd;     // forward transform (split form: fp16 hi part of 2^s * A)
  const void* fwdl;    // split form: fp16 lo part of 2^s * A (else null)
  const void* inv;     // inverse transform (split form: fp16 hi part)
  const void* invl;    // split form: fp16 lo part
  const void* sig;     // 4 sin^2(pi k / (2 N)), k = 0..n-1, working precision
  int ld;              // padded axis length (multiple of 32): the products' K extent
  int ldb;             // row stride of the matrices: ld plus 16 bytes (LDS bank spread)
  float fwd_unscale;   // 2^-s (split form), else 1
};

struct SubDev {
  int dim;
  int n[3];            // nodes per axis (n[2] = 1 in 2D)
  int off[3];          // global index of local node 0 per axis
  int art;             // bit 2k: low face of axis k artificial; bit 2k+1: high face
  int inst;            // instance slot
  int part0, nparts;   // residual partial sums owned by this subdomain
  int pad_;
  void* phi;
  void* F;
  void* T;
  // push transmission (preconditioned steps; null without artificial nodes owned elsewhere):
  // entries (destination node's device address as low and high words, row | later << 8, column)
  // of the nodes this subdomain owns for its neighbours, grouped by the inverse-last tile that
  // holds the node; pfirst[t] .. pfirst[t + 1] are those of local tile t (row block t / nct,
  // column block t % nct of the [rows][last axis] view, 16 x 64 nodes)
  const int4* push;
  const int* pfirst;
  double a[3];         // global box lower corner
  double h[3];         // grid spacing
  double gh2[3];       // gamma / h_k^2
  AxisDev ax[3];
};

struct InstDev {
  MonP<double> mond;
  MonP<float> monf;
  double log_vol_theta;  // log(|Omega_c| / theta)
  double dt;
  int first_sub, nsub;
  int pin;               // > 0: subtract each step the mean DC coefficient of subdomains
                         // first_sub .. first_sub + pin - 1 (gamma > 0)
  int pad_;
};

struct StepArgs {
  const SubDev* subs;
  const InstDev* insts;
  void* dc;              // per-subdomain DC coefficient of the current step (working precision)
  double* partials;      // residual partial sums (FP64)
  double* shift_acc;     // per-instance accumulated constant removed from phi (FP64)
  int* status;           // per-instance status bits
};

// one persistent launch per step (2D, preconditioned, parallel coupling): the three phases' tile
// tables, and the grid barrier's words (arrivals, generation)
struct PersistArgs {
  const int4* t_fused;
  const int4* t_pair;
  const int4* t_inv;
  unsigned* bar;
  int n_fused, n_pair, n_inv;
  int pair_src, part_base, lcap;
  int ninst;
  unsigned spin;  // bound on each barrier wait (polls of about 64 cycles)
};

// bytes of the fixed device scratch used by the entry point that allocates nothing
constexpr size_t kScratchBytes = (size_t)32 << 20;

}  // namespace pma
