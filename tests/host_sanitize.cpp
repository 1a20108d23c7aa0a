// Host paths of the runtime under AddressSanitizer, UndefinedBehaviorSanitizer and LeakSanitizer:
// the partition (Sec. 3, the overlapping decomposition), the sweep levels of Algorithm 1, theta
// (the normalisation of eq. pmae), the per-request byte count, and their error paths.  No GPU
// call is made; every result is checked against a property that holds by construction.
// Built and run by tests/test_host_sanitize.py; prints "host-sanitize ok" and exits 0 on success.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "pma.h"

static int fails = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++fails;                                                        \
    }                                                                 \
  } while (0)

static pma_grid grid(int dim, int n0, int n1, int n2) {
  pma_grid g;
  std::memset(&g, 0, sizeof g);
  g.dim = dim;
  g.n[0] = n0;
  g.n[1] = n1;
  g.n[2] = n2;
  for (int k = 0; k < 3; ++k) {
    g.lo[k] = 0.0;
    g.hi[k] = 1.0;
  }
  return g;
}

static pma_dd dd(int p0, int p1, int p2, int ov, int mode) {
  pma_dd d;
  d.parts[0] = p0;
  d.parts[1] = p1;
  d.parts[2] = p2;
  for (int k = 0; k < 3; ++k) d.overlap_cells[k] = ov;
  d.mode = mode;
  return d;
}

// every node of the grid lies in some subdomain; the subdomains' ranges are inside the grid
static void partition_case(const pma_grid& g, const pma_dd& d) {
  int nsub = 0;
  const int cap = 4096;
  std::vector<int> ranges(cap * 6), faces(cap * 6);
  const int rc = pma_partition(&g, &d, cap, &nsub, ranges.data(), faces.data());
  CHECK(rc == PMA_OK);
  if (rc != PMA_OK) return;
  int expect = 1;
  for (int k = 0; k < g.dim; ++k) expect *= d.parts[k];
  CHECK(nsub == expect);
  for (int k = 0; k < g.dim; ++k) {
    std::vector<char> hit(g.n[k], 0);
    for (int s = 0; s < nsub; ++s) {
      const int lo = ranges[s * 6 + 2 * k], hi = ranges[s * 6 + 2 * k + 1];
      CHECK(0 <= lo && lo < hi && hi <= g.n[k] - 1);
      for (int i = lo; i <= hi && i < g.n[k]; ++i) hit[i] = 1;
      // a face is artificial exactly when it is interior to the grid
      CHECK((faces[s * 6 + 2 * k] == PMA_FACE_ARTIFICIAL) == (lo > 0));
      CHECK((faces[s * 6 + 2 * k + 1] == PMA_FACE_ARTIFICIAL) == (hi < g.n[k] - 1));
    }
    for (int i = 0; i < g.n[k]; ++i) CHECK(hit[i]);
  }
  std::vector<int> levels(cap);
  int n2 = 0;
  CHECK(pma_sweep_levels(&g, &d, cap, &n2, levels.data()) == PMA_OK);
  CHECK(n2 == nsub);
  for (int s = 0; s < n2; ++s) {
    CHECK(levels[s] >= 0 && levels[s] < nsub);
    if (d.mode == PMA_DD_PARALLEL) CHECK(levels[s] == 0);
  }
  // cap smaller than the count: rejected, nothing written past cap
  if (nsub > 1) {
    std::vector<int> small((nsub - 1) * 6, -7);
    int m = 0;
    CHECK(pma_partition(&g, &d, nsub - 1, &m, small.data(), nullptr) != PMA_OK || m <= nsub - 1);
  }
}

static void request_case(const pma_grid& g, const pma_dd& d, int prec) {
  pma_request r;
  std::memset(&r, 0, sizeof r);
  r.grid = g;
  r.dd = d;
  r.mon.kind = PMA_MON_GAUSS_SUM;
  r.mon.nbumps = 2;
  r.mon.bamp[0] = 3.0;
  r.mon.bamp[1] = 2.0;
  r.mon.bw[0] = 0.1;
  r.mon.bw[1] = 0.2;
  for (int k = 0; k < 3; ++k) {
    r.mon.bc[0][k] = 0.3;
    r.mon.bc[1][k] = 0.6;
  }
  r.time.dt = 1e-3;
  r.time.gamma = 1.0;
  r.time.max_steps = 10;
  r.time.precision = prec;
  r.time.resid_every = 1;
  size_t bytes = 0;
  CHECK(pma_request_bytes(&r, &bytes) == PMA_OK);
  long nodes = 1;
  for (int k = 0; k < g.dim; ++k) nodes *= g.n[k];
  CHECK(bytes >= (size_t)nodes * 8);  // at least the FP64 Psi of the whole grid
  double th = 0;
  CHECK(pma_theta(&g, &r.mon, &th) == PMA_OK);
  // theta = volume + sum of the bumps' integrals over the box: between the volume and the volume
  // plus the bumps' integrals over all space
  double full = 1.0;
  for (int b = 0; b < 2; ++b) {
    double p = r.mon.bamp[b];
    for (int k = 0; k < g.dim; ++k) p *= r.mon.bw[b] * std::sqrt(2.0 * M_PI);
    full += p;
  }
  CHECK(th > 1.0 && th < full);
}

int main() {
  // valid shapes: 2D and 3D, single domain, slabs, blocks, every sweep mode
  const int modes[3] = {PMA_DD_PARALLEL, PMA_DD_ALTERNATING, PMA_DD_COLOURED};
  for (int m = 0; m < 3; ++m) {
    partition_case(grid(2, 65, 65, 1), dd(1, 1, 1, 4, modes[m]));
    partition_case(grid(2, 65, 65, 1), dd(4, 1, 1, 2, modes[m]));
    partition_case(grid(2, 97, 81, 1), dd(4, 4, 1, 4, modes[m]));
    partition_case(grid(2, 513, 513, 1), dd(16, 16, 1, 8, modes[m]));
    partition_case(grid(3, 25, 25, 25), dd(2, 2, 2, 4, modes[m]));
    partition_case(grid(3, 13, 13, 13), dd(3, 3, 3, 2, modes[m]));
  }
  for (int prec = 0; prec < 3; ++prec) {
    request_case(grid(2, 129, 97, 1), dd(1, 1, 1, 4, 0), prec);
    request_case(grid(2, 257, 257, 1), dd(2, 2, 1, 4, 0), prec);
    request_case(grid(3, 33, 33, 33), dd(2, 2, 2, 4, 1), prec);
  }
  // error paths: each rejected with a message, no state left behind
  int nsub = 0;
  pma_grid bad = grid(4, 65, 65, 1);
  pma_dd one = dd(1, 1, 1, 4, 0);
  CHECK(pma_partition(&bad, &one, 16, &nsub, nullptr, nullptr) == PMA_E_INVAL);
  CHECK(std::strlen(pma_last_error()) > 0);
  pma_grid tiny = grid(2, 4, 65, 1);
  CHECK(pma_partition(&tiny, &one, 16, &nsub, nullptr, nullptr) == PMA_E_INVAL);
  pma_grid g = grid(2, 65, 65, 1);
  pma_dd toomany = dd(40, 1, 1, 2, 0);
  CHECK(pma_partition(&g, &toomany, 4096, &nsub, nullptr, nullptr) == PMA_E_INVAL);
  pma_dd negov = dd(2, 2, 1, -1, 0);
  CHECK(pma_partition(&g, &negov, 16, &nsub, nullptr, nullptr) == PMA_E_INVAL);
  pma_grid huge = grid(2, 2049, 9, 1);
  pma_request r;
  std::memset(&r, 0, sizeof r);
  r.grid = huge;
  r.dd = one;
  r.mon.kind = PMA_MON_CONST;
  r.mon.amp = 1.0;
  r.time.dt = 1e-3;
  r.time.gamma = 1.0;
  r.time.resid_every = 1;
  size_t bytes = 0;
  CHECK(pma_request_bytes(&r, &bytes) == PMA_E_INVAL);  // an axis beyond the longest supported
  CHECK(pma_request_bytes(nullptr, &bytes) == PMA_E_INVAL);
  CHECK(pma_theta(nullptr, nullptr, nullptr) == PMA_E_INVAL);
  pma_monitor neg;
  std::memset(&neg, 0, sizeof neg);
  neg.kind = 99;
  double th = 0;
  CHECK(pma_theta(&g, &neg, &th) == PMA_E_INVAL);
  if (fails) {
    std::fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  std::printf("host-sanitize ok\n");
  return 0;
}
