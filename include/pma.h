/*
 * pma.h -- C ABI of the MI355X DD-PMA adaptive mesh library.
 *
 * The library computes adaptive meshes x = grad Psi by pseudo-time stepping the parabolic
 * Monge-Ampere equation  dPsi/dtau = log(|Omega_c| rho(grad Psi) det D^2 Psi)  (Sulman, Nguyen,
 * Haynes, Huang, arXiv 2006.14602, Sec. 2 eq. pmae) with Psi(xi,0) = |xi|^2/2 (eq. incond) and
 * the sliding boundary condition grad Psi . n = xi . n (eq. nbd), on a uniform grid of a box,
 * either on the whole box or on overlapping subdomains coupled by the non-iterative parallel
 * transmission condition (Sec. 3, eq. transmission_condition3), then glues the subdomain
 * meshes (Sec. 4.5).
 *
 * Discretisation and step (the paper integrates each step with an ODE solver; this library
 * takes one preconditioned explicit step per pseudo-time step):
 *   F     = log(|Omega_c| rho(grad_h Psi) det D^2_h Psi / theta),  theta = int_Omega rho
 *           (centred differences, Sec. 3 eqs. pmae1d/pmae2d; rho normalised as in Sec. 2)
 *   delta = (I - gamma L_h)^{-1} F  with L_h the Neumann Laplacian of each (sub)domain,
 *           inverted by type-I DCTs applied as dense matrix products; gamma = 0 is forward Euler
 *   Psi  += dt * delta   (not on artificial-boundary nodes, which hold transmitted values)
 * Residual: ||Psi^{n+1} - Psi^n||_2 with the trapezoid rule (Sec. 2 eq. dd_stop_criterion),
 * maximum over subdomains.
 *
 * Conventions for every entry point:
 *   - Return value: PMA_OK (0) or a negative PMA_E_* code.  Nothing throws or aborts across
 *     the ABI; pma_last_error() gives a readable message for the calling thread.
 *   - Grid arrays are row-major with the LAST axis fastest: node (i0, i1[, i2]) of a grid with
 *     n[] nodes per axis is element (i0 * n[1] + i1) [* n[2] + i2].  Node i of axis k sits at
 *     lo[k] + i * (hi[k] - lo[k]) / (n[k] - 1).
 *   - Meshes are returned as dim planes of prod(n) doubles: all x_0, then all x_1 [, x_2].
 *   - Host buffers are owned by the caller and must hold the stated number of elements.
 *   - A context serialises its own calls; different contexts may be used from different
 *     threads.
 */
#ifndef PMA_H
#define PMA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  PMA_OK = 0,
  PMA_E_INVAL = -1,     /* invalid argument or shape */
  PMA_E_NOMEM = -2,     /* device arena exhausted or allocation failed */
  PMA_E_HIP = -3,       /* a HIP runtime call failed */
  PMA_E_TANGLED = -4,   /* the mesh folded: det D^2_h Psi <= 0 at a node during a step, or a
                           cell of the final mesh with non-positive measure */
  PMA_E_NONFINITE = -5, /* a non-finite right-hand side or update */
  PMA_E_BUDGET = -6,    /* request larger than the whole HBM budget */
  PMA_E_NOTFOUND = -7,  /* unknown or retired ticket */
  PMA_E_BUSY = -8       /* server queue full */
};

/* arithmetic form of a solve */
enum {
  PMA_FP64 = 0,         /* FP64 state, FP64 stencils, FP64 matrix-core DCT products */
  PMA_FP32 = 1,         /* FP32 state (Psi - |xi|^2/2), FP32 stencils and DCT products */
  PMA_FP32_SPLIT16 = 2  /* FP32 state and stencils; DCT products as fp16 hi+lo pairs with
                           FP32 accumulation (three matrix-core products per tile) */
};

/* execution form */
enum {
  PMA_EXEC_BATCHED = 0, /* every subdomain advanced by the same launches, replayed as a graph */
  PMA_EXEC_PLAIN = 1    /* one subdomain per launch, no graph (the comparison baseline) */
};

/* decomposition coupling */
enum {
  PMA_DD_PARALLEL = 0,    /* Sec. 3 eq. transmission_condition3: neighbours' time-n values */
  PMA_DD_ALTERNATING = 1, /* Algorithm 1 (eqs. transmission_condition1/2): the subdomains are
                             updated in turn within a step, in block order (axis 0 slowest),
                             each taking the owners' latest values at its artificial nodes */
  PMA_DD_COLOURED = 2     /* Algorithm 1 with the 2^d parity classes of the block index as the
                             sweep: classes in lexicographic order of the parity tuple */
};

enum { PMA_FACE_NEUMANN = 0, PMA_FACE_ARTIFICIAL = 1 };

/* monitor (mesh density) functions rho(x); theta = int rho is computed when theta == 0 */
enum {
  PMA_MON_CONST = 0,          /* rho = amp */
  PMA_MON_SECH2_RADIAL = 1,   /* rho = 1 + amp sech^2(k (|x - c|^2 - r0^2)) */
  PMA_MON_SECH2_SINE = 2,     /* rho = 1 + amp sech^2(k (x_1 - c[1] - r0 sin(2 pi x_0))) */
  PMA_MON_GAUSS_SUM = 3,      /* rho = 1 + sum_b bamp[b] exp(-|x - bc[b]|^2 / (2 bw[b]^2)) */
  PMA_MON_SEPARABLE_SECH2 = 4, /* rho = prod_k (1 + amp_axes[k] sech^2(k_axes[k] (x_k - c[k]))) */
  /* arc-length monitors rho = sqrt(1 + |grad u|^2) of given solutions u (Sec. 4, eq. monitfn):  */
  PMA_MON_ARCLEN_FRONT = 5,   /* 2D: u = 1 / (1 + exp((x_0 + x_1 - r0) / (2 k)))  (eq. test_fn1;
                                 the paper takes k = 0.01, r0 = 1) */
  PMA_MON_ARCLEN_SPIRAL = 6,  /* 2D: u = 1 + amp / (1 + k r^2 cos^2(t - twist r^2)), r and t the
                                 polar coordinates about c (eq. test_fn2: amp 9, k 100, twist 20,
                                 c = (0.7, 0.5)) */
  PMA_MON_ARCLEN_SPHERES = 7  /* u = sum_{b < nbumps} tanh(k (|x - bc[b]|^2 - r0^2))
                                 (eqs. test_fn3d1, test_fn3d2); nbumps 1..9 */
};

#define PMA_MAX_BUMPS 9

/* request states */
enum { PMA_PENDING = 0, PMA_RUNNING = 1, PMA_DONE = 2, PMA_FAILED = 3 };

typedef struct pma_ctx pma_ctx;

typedef struct {
  int dim;          /* 2 or 3 */
  int n[3];         /* nodes per axis (>= 5); n[2] ignored in 2D */
  double lo[3];     /* box lower corner */
  double hi[3];     /* box upper corner (hi > lo) */
} pma_grid;

typedef struct {
  int kind;         /* PMA_MON_* */
  int nbumps;       /* PMA_MON_GAUSS_SUM: 1..4; PMA_MON_ARCLEN_SPHERES: 1..9 */
  double amp, k, r0;
  double c[3];
  double amp_axes[3], k_axes[3];
  double bamp[PMA_MAX_BUMPS], bw[PMA_MAX_BUMPS], bc[PMA_MAX_BUMPS][3];
  double twist;     /* PMA_MON_ARCLEN_SPIRAL */
  double theta;     /* int_Omega rho; 0 -> computed by the library (FP64 quadrature) */
} pma_monitor;

typedef struct {
  double dt;        /* pseudo-time step > 0 */
  double gamma;     /* preconditioner weight >= 0 (0: forward Euler) */
  double tol;       /* stop when the residual <= tol (0: run max_steps) */
  int max_steps;    /* >= 0 */
  int precision;    /* PMA_FP64 / PMA_FP32 / PMA_FP32_SPLIT16 */
  int resid_every;  /* residual cadence R >= 1 (steps) */
  int exec;         /* PMA_EXEC_BATCHED / PMA_EXEC_PLAIN */
} pma_time;

typedef struct {
  int parts[3];         /* subdomains per axis (>= 1) */
  int overlap_cells[3]; /* overlap in cells per axis (>= 2 where parts > 1) */
  int mode;             /* PMA_DD_PARALLEL / PMA_DD_ALTERNATING / PMA_DD_COLOURED; two subdomains
                           are never updated together if one reads the other, so the alternating
                           forms equal the one-subdomain-at-a-time sweep exactly */
} pma_dd;

typedef struct {
  int steps_done;
  int status;           /* PMA_OK or the failure code */
  double final_resid;   /* last computed residual (FP64) */
  double min_det;       /* min over owned nodes of det D^2_h Psi (FP64) */
  double min_cell;      /* min signed cell area (2D) / corner Jacobian (3D) of the mesh (FP64) */
  double theta;         /* normalisation used */
  double ms_total;      /* wall time of the solve; for served requests: submit -> done */
  double ms_queue;      /* served requests: submit -> admission */
  double quality_e2;    /* mesh quality (Sec. 4.5): E = |Omega_c| (rho(x) / theta) J at every node,
                           J = det(dx/dxi) by second-order differences of the glued mesh;
                           E_2 = (int E^2 / |Omega_c|)^(1/2) by the trapezoid rule (1 on an
                           equidistributing mesh); FP64 */
  double quality_emax;  /* max over nodes of E */
} pma_stats;

typedef struct {
  pma_grid grid;
  pma_dd dd;            /* parts all 1 -> single domain */
  pma_monitor mon;
  pma_time time;
  double arrival_s;     /* caller's timestamp, echoed back; not used for scheduling */
  const double* psi0;   /* optional host array of prod(n) doubles: the initial Psi (warm start,
                           Sec. 2: resuming a solve, or the previous mesh of a time-dependent
                           problem); NULL: Psi^0 = |xi|^2/2.  pma_submit copies it; the batch
                           and plan calls read it during the call */
  int want_psi;         /* served requests: keep the glued final Psi for pma_poll_psi */
} pma_request;

/* ---- context -------------------------------------------------------------------------- */

/* Create a context on HIP device `hip_device` with a device-memory budget of
 * `hbm_budget_bytes` (0 -> 8 GiB).  The budget is one arena, allocated on first use through
 * the allocator installed by pma_set_allocator (hipMalloc if none); every solve's arrays and
 * the DCT bases are carved from it.  *out receives the context. */
int pma_create(int hip_device, size_t hbm_budget_bytes, pma_ctx** out);

/* Stop the server (finishing nothing further), release all device memory, free the context. */
int pma_destroy(pma_ctx* ctx);

/* Install the device allocator used for the arena (e.g. a framework's caching allocator).
 * Must be called before the first solve.  alloc returns NULL on failure. */
int pma_set_allocator(pma_ctx* ctx, void* (*alloc)(size_t bytes, void* stream, void* user),
                      void (*free_)(void* ptr, void* stream, void* user), void* user);

/* ---- one subdomain (Sec. 3 eqs. pmae1d/pmae2d on Omega_i) ------------------------------- */

/* Advance one subdomain of `global` for time->max_steps steps (or to time->tol) in place.
 * lo[k]..hi[k] are the subdomain's global node ranges (inclusive); face_kind[2k] / [2k+1] is the
 * kind of its low / high face on axis k (PMA_FACE_NEUMANN on the box boundary, or
 * PMA_FACE_ARTIFICIAL, whose nodes keep the Dirichlet values found in psi_dev: the transmission
 * condition eq. pmae1cd held fixed).
 * psi_dev: caller-owned DEVICE buffer of prod(hi-lo+1) doubles holding Psi (row-major, last axis
 * fastest); it is read at the start and overwritten with the result.  hip_stream: caller's
 * hipStream_t (NULL: the default stream); the call returns after the stream has finished the
 * work.  st may be NULL. */
int pma_solve_subdomain(pma_ctx* ctx, const pma_grid* global, const int lo[3], const int hi[3],
                        const int face_kind[6], const pma_monitor* mon, const pma_time* time,
                        void* psi_dev, void* hip_stream, pma_stats* st);

/* The same solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): it calls no hipMalloc,
 * hipFree, pinned-host or graph allocation and creates no event.  The subdomain's state, its DCT
 * matrices, launch tables and reduction buffers live in one fixed device scratch of 32 MiB per
 * GPU, part of the library's code object (held until the process ends); its address is looked up
 * per device by pma_create.  The kernels run on hip_stream itself, launched directly (no
 * captured graphs), and the call returns after that stream has finished.  Arguments, layout,
 * ownership and results are those of pma_solve_subdomain, bitwise.
 * Limit: the subdomain's three state arrays (prod(hi - lo + 1) elements each, 8 bytes in FP64,
 * 4 otherwise) plus one DCT basis per distinct axis length must fit 31 MiB: PMA_E_INVAL with the
 * byte counts otherwise.  The scratch keeps the last call's contents; every call initialises
 * what it reads.  Calls on one GPU share the scratch: calls that overlap in time on the same GPU
 * (from different contexts or threads) race and must be serialised by the caller. */
int pma_solve_subdomain_noalloc(pma_ctx* ctx, const pma_grid* global, const int lo[3], const int hi[3],
                                const int face_kind[6], const pma_monitor* mon, const pma_time* time,
                                void* psi_dev, void* hip_stream, pma_stats* st);

/* ---- whole mesh (Sec. 3 parallel DD-PMA, Sec. 4.5 glue) ---------------------------------- */

/* Compute the adaptive mesh of `grid`, single domain if dd is NULL or all parts are 1, else the
 * overlapping block decomposition of dd (cores floor(m N / M), each subdomain extended by
 * floor(ov/2) cells below and ceil(ov/2) above, clipped to the box; each node owned by the part
 * whose core holds it, the last node by the last part).
 * psi0: optional host array of prod(n) doubles, the initial Psi (warm start, Sec. 2); NULL means
 * Psi^0 = |xi|^2/2.  mesh_out: host array of dim * prod(n) doubles.  psi_out: optional host
 * array of prod(n) doubles receiving the glued Psi.  st may be NULL.
 * Errors: PMA_E_INVAL for dim not 2/3, fewer than 5 nodes on an axis, a subdomain with fewer
 * than 4 cells on an axis, or overlap < 2 cells where an axis is split; PMA_E_TANGLED /
 * PMA_E_NONFINITE if the iteration breaks down (mesh_out is then unspecified). */
int pma_dd_mesh(pma_ctx* ctx, const pma_grid* grid, const pma_dd* dd, const pma_monitor* mon,
                const pma_time* time, const double* psi0, double* mesh_out, double* psi_out,
                pma_stats* st);

/* Many independent meshes advanced together (all subdomains of all requests in the same
 * launches; each request stops at its own step count).  mesh_outs[i] receives request i's mesh
 * (dim * prod(n) doubles); stats may be NULL.  Every request must use the same precision.
 * Returns the first failure code, after finishing the others. */
int pma_dd_mesh_batch(pma_ctx* ctx, int count, const pma_request* reqs, double* const* mesh_outs,
                      pma_stats* stats);

/* ---- resident solves (state kept in device memory between calls) ---------------------------- */

/* A plan holds `count` requests (one precision) on the device, initialised to Psi^0, and lets
 * the caller advance them step by step in the shared launches of pma_dd_mesh_batch (or one
 * subdomain per launch when time.exec is PMA_EXEC_PLAIN).  Requests' max_steps and tol are not
 * used: the caller decides how many steps to take.  *out receives the plan. */
typedef struct pma_plan pma_plan;
int pma_plan_create(pma_ctx* ctx, int count, const pma_request* reqs, pma_plan** out);

/* Enqueue nsteps pseudo-time steps of every request on the context's stream and return without
 * waiting. */
int pma_plan_step(pma_plan* plan, int nsteps);

/* Wait until every enqueued step has finished; PMA_E_TANGLED / PMA_E_NONFINITE if a request has
 * broken down. */
int pma_plan_sync(pma_plan* plan);

/* Phases of one step, in launch order:
 *   0 transmission of artificial-boundary values     1 stencil: right-hand side F (fused 2D:
 *                                                       and its forward last-axis product)
 *   2 forward-Euler update (gamma = 0)                3 forward DCT along the last axis
 *   4 forward DCT along the middle axis (3D)          5 forward DCT + spectral scale + inverse DCT
 *                                                       along axis 0
 *   6 inverse DCT along the middle axis (3D)          7 inverse DCT along the last axis + update
 * Times each phase on its own: nsteps launches back to back between two HIP events on the
 * stream the kernels run on; ms[ph] receives the mean device milliseconds per launch (cap >= 8
 * entries).  flops[] and bytes[] (may be NULL) receive each phase's algorithmic floating-point
 * operations and compulsory HBM bytes per launch.  With cap >= 9, entry 8 is the FP64 residual
 * reduction that runs every R steps (flops: partial sums added; bytes: partial sums read).  The
 * plan's state is saved before and restored after (the call needs device memory for one copy of
 * it).  *nphases receives 8, or 9 with cap >= 9. */
int pma_plan_phase_times(pma_plan* plan, int nsteps, double* ms, double* flops, double* bytes, int cap,
                         int* nphases);

/* Autotuner of the stencil's launch shape (phase 1).  A stencil workgroup marches over `march`
 * consecutive chunks of a block: 16-row chunks of axis 0 in 2D, planes of axis 0 in 3D (over
 * 16 rows of axis 1); longer marches amortise the block's set-up and keep the next chunk's loads
 * in flight, shorter ones give more workgroups.  Candidates march = 1, 2, 4, .. 64 (capped at
 * the longest useful value) are each timed over `reps` back-to-back launches on the plan's own
 * state between two HIP events; the fastest is kept for every later step (the captured step
 * graphs are rebuilt).  The stencil reads phi and writes only F, which every step recomputes,
 * so the results of the plan do not change (bitwise).  *march receives the choice; ms[k]
 * (may be NULL, cap entries) the mean milliseconds per launch of candidate k; *ncand (may be
 * NULL) the number of candidates timed.  Errors: PMA_E_INVAL for a NULL plan or march, or
 * reps <= 0. */
int pma_plan_autotune(pma_plan* plan, int reps, int* march, double* ms, int cap, int* ncand);

/* Result of pma_plan_tune. */
typedef struct {
  int march;        /* stencil chunks per workgroup (pma_plan_autotune) */
  int persistent;   /* 1: one persistent launch per step (pma_plan_set_persistent) */
  int eight_max;    /* launches of at most this many tiles take eight-wave workgroups (else four) */
  int lbasis_max;   /* launches of at most this many tiles copy the DCT matrices into LDS where
                       they fit (else read them from L2) */
  double step_ms;   /* mean device milliseconds per step of the choice (as timed when cached) */
  int from_cache;   /* 1: taken from the cache file without timing */
  int candidates;   /* step configurations timed */
} pma_tuning;

/* Autotuner of the plan's launch configuration: the stencil's march length (pma_plan_autotune),
 * then whole steps timed for every combination of the step form (phase launches, or one
 * persistent launch where the plan allows it), the eight-wave threshold (0, 512, all) and the
 * LDS-basis threshold (0, 512, all), reps steps each between two HIP events, on a copy of the
 * plan's state that is restored afterwards; the fastest is kept.  Results of the plan do not
 * depend on the choice (bitwise).  cache_path (may be NULL): a text file of earlier choices keyed
 * by the device architecture, the precision and coarse buckets of the plan's shape (subdomain
 * count and node count rounded up to powers of two, widest padded axis, dimensions, forward
 * Euler, sweep levels); a matching entry is applied without timing, a new choice is appended.
 * Errors: PMA_E_INVAL for a NULL plan or out, reps <= 0, or a cache file that cannot be written;
 * PMA_E_NOMEM if the state copy does not fit the arena. */
int pma_plan_tune(pma_plan* plan, int reps, const char* cache_path, pma_tuning* out);

/* Fix the stencil's march length (see pma_plan_autotune) for every later step of the plan;
 * values beyond a subdomain's extent cover that subdomain's whole axis 0 in one workgroup.
 * Results do not depend on it (bitwise).  Errors: PMA_E_INVAL for a NULL plan or march outside
 * 1..4096. */
int pma_plan_set_march(pma_plan* plan, int march);

/* Turn the fused stencil on (default) or off for the plan's 2D subdomains of preconditioned
 * requests whose last axis is at most 320 wide (padded): the stencil of 16 full rows is computed
 * into LDS and multiplied by the forward last-axis DCT matrix in the same kernel (phase 1 then
 * also does phase 3's product for them).  Off: separate stencil and product launches, F through
 * HBM.  Results are the same up to the order of rounding (both paths evaluate the same formulas);
 * the switch exists to time the stencil on its own.  Only before the plan's first step.
 * Errors: PMA_E_INVAL for a NULL plan or a plan that has already stepped. */
int pma_plan_set_fusion(pma_plan* plan, int on);

/* Allow (on != 0, the default) or forbid the 64-column strip kernel of the axis products, which a
 * plan uses when its 16-column strip tables would exceed 512 strips (FP32 and split forms, axes up
 * to 320 padded nodes): each DCT matrix fragment is then read once for four column blocks.
 * Results are bitwise the same either way (each column block keeps its own block scale and
 * accumulation order); the switch exists to time and test both.  Only before the first step:
 * PMA_E_INVAL afterwards. */
int pma_plan_set_wide_strips(pma_plan* plan, int on);

/* Advance each step of the plan in one persistent launch (on != 0) instead of one launch per
 * phase (form (2) of the method's batched execution): the fused stencil + forward last-axis
 * product, the axis-0 pair and the inverse last-axis product with the update and the pushed
 * transmission (Sec. 3: one exchange per step) run in one kernel whose workgroups loop over the
 * tiles of each phase, with grid-wide barriers between phases.  The grid is sized to the
 * workgroups the device holds at once; each barrier wait is bounded, and a timeout fails the
 * requests with PMA_E_HIP instead of hanging.  Results are bitwise those of the phase launches.
 * Available for plans whose subdomains are all 2D, preconditioned (gamma > 0) and fused (last
 * axis at most 320 padded), coupled in parallel, with regular axis-0 strips: PMA_E_INVAL
 * otherwise, with the reason in pma_last_error().  May be switched at any time. */
int pma_plan_set_persistent(pma_plan* plan, int on);

/* Glue request i's mesh (dim * prod(n) doubles) into host memory; st may be NULL. */
int pma_plan_mesh(pma_plan* plan, int i, double* mesh_out, pma_stats* st);

/* Release the plan's device memory. */
int pma_plan_destroy(pma_plan* plan);

/* ---- serving (continuous batching) ------------------------------------------------------- */

/* Queue a request (copied) and return its ticket without blocking.  A background thread admits
 * queued requests in arrival order while their bytes fit the HBM budget, advances every admitted
 * request one step per tick in shared launches, and finishes each at its own step count.
 * PMA_E_BUDGET if the request can never fit the budget. */
int pma_submit(pma_ctx* ctx, const pma_request* req, uint64_t* ticket);

/* State of a ticket.  When DONE, copies the mesh into mesh_out (dim * prod(n) doubles, may be
 * NULL) and the stats into st, and retires the ticket: later calls return PMA_E_NOTFOUND.
 * FAILED also retires it (st->status holds the cause; pma_last_error() describes it). */
int pma_poll(pma_ctx* ctx, uint64_t ticket, int* state, double* mesh_out, pma_stats* st);

/* pma_poll that also copies the glued final Psi (prod(n) doubles) into psi_out when DONE: the
 * warm start of the next solve (Sec. 2), e.g. resubmitted with it as psi0.  The request must
 * have been submitted with want_psi set: PMA_E_INVAL otherwise (the ticket is not retired). */
int pma_poll_psi(pma_ctx* ctx, uint64_t ticket, int* state, double* mesh_out, double* psi_out, pma_stats* st);

/* Server counters: requests queued, running, finished (done or failed, retired or not); device
 * bytes of the context's arena in use (request state and cached DCT bases) as of the server's
 * last admission or release. */
int pma_server_info(pma_ctx* ctx, int* queued, int* running, int* finished, size_t* bytes_in_use);

/* Device bytes a request occupies in a context's arena while it runs: its state arrays, mesh,
 * Psi and reduction partials, plus every DCT basis it uses (bases are shared between requests of
 * the same axis lengths and precision, and kept as an evictable cache afterwards).  pma_submit
 * refuses requests above the budget by this count (PMA_E_BUDGET).  Host only.  Errors:
 * PMA_E_INVAL for a NULL argument or an invalid request (as pma_dd_mesh). */
int pma_request_bytes(const pma_request* req, size_t* bytes);

/* ---- host-only helpers (no GPU needed) ------------------------------------------------------ */

/* Partition as pma_dd_mesh does.  *nsub receives the number of subdomains; if ranges is not
 * NULL it receives nsub*6 ints (lo0, hi0, lo1, hi1, lo2, hi2 per subdomain, subdomains in
 * row-major part order) and faces (if not NULL) nsub*6 PMA_FACE_* values. cap bounds nsub. */
int pma_partition(const pma_grid* grid, const pma_dd* dd, int cap, int* nsub, int* ranges,
                  int* faces);

/* Sweep level of every subdomain (row-major part order) under dd->mode, as the solver uses it:
 * 0 for all in the parallel form; in the alternating forms (Algorithm 1) a subdomain's level is
 * one more than the highest level among the subdomains it exchanges artificial-node values with
 * that precede it in the sweep, and the solver advances the levels in order, each in one launch
 * set.  *nsub receives the number of subdomains; levels (if not NULL) receives nsub ints; cap
 * bounds nsub.  Errors: PMA_E_INVAL for an invalid grid or decomposition. */
int pma_sweep_levels(const pma_grid* grid, const pma_dd* dd, int cap, int* nsub, int* levels);

/* theta = int_box rho in FP64 (closed forms where they exist, else Gauss-Legendre quadrature). */
int pma_theta(const pma_grid* grid, const pma_monitor* mon, double* theta_out);

/* Message describing the last failure on the calling thread (never NULL). */
const char* pma_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PMA_H */
