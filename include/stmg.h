/*
 * stmg.h -- C ABI of the MI355X space-time multigrid library for the
 * eddy-current equation  sigma du/dt + curl(nu curl u) = f  on a tetrahedral
 * mesh with lowest-order Nedelec elements and upwind DG in time.
 *
 * Method (Neumueller & Schwalsberger, "A parallel space-time multigrid method
 * for the eddy-current equation", 2019):
 *   - all-at-once space-time system L x = f, block lower bidiagonal, slab block
 *     A = K_t (x) M + M_t (x) K, coupling -N_t (x) M (section 2.1, eq. (1));
 *   - damped block-Jacobi smoother S with exact slab solves (eq. (2));
 *   - nodal auxiliary-space correction A = G Sigma_t K_n^{-1} G^T (eq. (8));
 *   - hybrid smoother SAS (section 4; the other orders it compares are
 *     options), V-cycle over time meshes with spatial coarsening where the
 *     local anisotropy rule (eq. (3)) holds;
 *   - convergence rates by power iteration (section 5.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Edges: the distinct vertex pairs of the finest mesh's tetrahedra, stored as
 *   (tail, head) with tail < head, numbered in lexicographic order of
 *   (tail, head). The edge DOF is the line integral of the field from tail to
 *   head. The same rule numbers the edges of every coarse mesh.
 * Boundary: a face that belongs to exactly one tetrahedron is a boundary face;
 *   its edges and vertices are boundary DOFs. Section 3 allows two homogeneous
 *   conditions (stmg_problem.bc): Dirichlet, u x n = 0, eliminates them;
 *   Neumann, mu^{-1} curl u x n = 0, is natural and keeps every edge as a
 *   DOF. Under Neumann the nodal space of the correction (eq. (8)) leaves out
 *   the mesh's vertex 0 as a gauge: G maps constants to zero, so the other
 *   vertices' gradients span the same space and K_n stays SPD (the mesh must
 *   be connected). "Interior" below means "not eliminated": every edge under
 *   Neumann.
 * Vectors at the ABI (device pointers, FP64, caller-owned, contiguous):
 *   full layout     [Nt][pt+1][n_edges]   all edges of the finest mesh;
 *                   boundary entries of inputs are ignored, of outputs are 0.
 *   level layout    [N][pt+1][n_interior] interior edges of that level's mesh
 *                   in ascending edge order (used by the per-level entry
 *                   points meant for testing).
 *   Component k of slab n is the coefficient of the Legendre polynomial
 *   psi_0 = 1, psi_1 = 2s - 1 on that slab (s in [0,1]).
 * Right-hand side: the discrete load b[n][k][e] = int_{I_n} int f . phi_e psi_k.
 *   The optional initial value u0 [n_edges] adds psi_k(0) M u0 to slab 0 (the
 *   M u^0 term of eq. (1)).
 * Streams: every device operation is enqueued on the stream given to
 *   stmg_setup (NULL = default stream); entry points that return a host value
 *   synchronise that stream. A handle is not re-entrant.
 * Errors: every int-returning function returns STMG_OK or one of the codes
 *   below; stmg_strerror names it, stmg_last_error_message gives detail.
 */
#ifndef STMG_H
#define STMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  STMG_OK = 0,
  STMG_EINVAL = 1,    /* bad sizes or arguments (Nt not 2^k, pt not 0/1, sigma <= 0 ...) */
  STMG_ENOMEM = 2,    /* host or device allocation failed */
  STMG_ENOTCONV = 3,  /* max_cycles reached before rtol; x holds the last iterate */
  STMG_ENUMERIC = 4,  /* NaN/Inf in data or residual, zero pivot in a factorisation */
  STMG_EHIP = 5,      /* HIP runtime error (no device, launch failure ...) */
  STMG_EAGAIN = 6,    /* serving: result not ready yet */
  STMG_ENOSYS = 7     /* entry point not available for this handle (e.g. built with host_only) */
};

enum { STMG_FP64 = 0, STMG_FP32_REFINED = 1 };
enum { STMG_BC_DIRICHLET = 0, STMG_BC_NEUMANN = 1 };
/* Nodal solve of the auxiliary correction (eq. (8)). STMG_NODAL_EXACT:
 * K_n^{-1} applied exactly with its Cholesky factor, as the analysis of
 * section 4.1 assumes. k in 1..STMG_NODAL_CHEBYSHEV_MAX: no nodal factor;
 * K_n^{-1} replaced by k steps of the Jacobi-preconditioned Chebyshev
 * iteration from zero on [lmax / 30, lmax], lmax the Gershgorin bound of
 * D^{-1} K_n (the inexact spatial solves of section 5). The V-cycle stays a
 * fixed linear iteration with the same fixed point; its rate changes. */
enum { STMG_NODAL_EXACT = 0, STMG_NODAL_CHEBYSHEV_MAX = 16 };
/* Slab solves of the smoother (eq. (2)). STMG_SLAB_EXACT: A^{-1} applied
 * exactly with the slab factor of the level's mesh. k in
 * 1..STMG_SLAB_TWOGRID_MAX: on levels with N > 1 whose mesh has a coarser
 * one, A z = w (A = mu M + tau K after the diagonalisation of the slab's time
 * block: mu = 2 + i sqrt(2) for p_t = 1, 1 for p_t = 0) is solved inexactly
 * (section 5) by k steps of Richardson iteration from zero, z <- z + B (w -
 * A z), B one two-grid cycle: two sweeps of [a damped edge Jacobi step,
 * omega 1/2, with diag(A); a Jacobi step on the gradients G y with
 * diag(mu K_n), the Galerkin operator G^T A G = mu K_n], the exact solve of
 * the Galerkin coarse operator P^T A P = mu M_c + tau K_c with the coarser
 * mesh's factor, and the two sweeps with their steps reversed. The V-cycle
 * stays a fixed linear iteration with the same fixed point. */
enum { STMG_SLAB_EXACT = 0, STMG_SLAB_TWOGRID_MAX = 16 };
/* Smoother sequences (section 4) of the steps S (damped block Jacobi,
 * eq. (2)) and A (nodal auxiliary correction, eq. (8)). A name reads like a
 * product of matrices, right to left: before the coarse-grid correction SA
 * applies A, then S; after it the same steps run in reversed order (S, then
 * A). SAS is the method's choice; S_ONLY (= SS) drops A; the others are the
 * orders the paper compares with SAS in section 4.1. */
enum {
  STMG_SMOOTH_SAS = 0,
  STMG_SMOOTH_S_ONLY = 1,
  STMG_SMOOTH_SA = 2,
  STMG_SMOOTH_AS = 3,
  STMG_SMOOTH_SSA = 4,
  STMG_SMOOTH_ASS = 5,
  STMG_SMOOTH_SSAS = 6,
  STMG_SMOOTH_SSASS = 7
};

/* One mesh of a nested hierarchy. Coarse meshes (index >= 1) describe their
 * relation to the next finer mesh:
 *   vertex_parent[v_fine][2] = (a, b): the finer vertex is the midpoint of this
 *     mesh's vertices a and b (a == b: it coincides with vertex a);
 *   tet_parent[t_fine]: this mesh's tetrahedron containing the finer one.
 * Only nested refinements are meaningful (Freudenthal/Kuhn or red). */
typedef struct {
  int32_t n_vertices;
  const double *coords;          /* host [n_vertices][3] */
  int32_t n_tets;
  const int32_t *tets;           /* host [n_tets][4], 0-based vertex ids */
  const int32_t *vertex_parent;  /* NULL on mesh 0; host [n_vertices(finer)][2] */
  const int32_t *tet_parent;     /* NULL on mesh 0; host [n_tets(finer)] */
} stmg_mesh;

/* The problem of section 3: sigma du/dt + curl nu curl u = f on Omega x (0,T),
 * sigma and nu (= mu^{-1}) piecewise constant per tetrahedron of mesh 0,
 * tau = T/Nt, DG degree pt in time (0 = implicit Euler of eq. (1)). */
typedef struct {
  int32_t n_meshes;              /* >= 1; meshes[0] is the finest */
  const stmg_mesh *meshes;       /* host array of n_meshes */
  const double *sigma;           /* host [meshes[0].n_tets], > 0 */
  const double *nu;              /* host [meshes[0].n_tets], >= 0 */
  double T;                      /* > 0 */
  int32_t Nt;                    /* power of two */
  int32_t pt;                    /* 0 or 1 */
  int32_t bc;                    /* STMG_BC_DIRICHLET (0) or STMG_BC_NEUMANN (section 3) */
} stmg_problem;

typedef struct {
  double omega;                  /* smoother damping, 0.5 (eq. (2)) */
  double lambda_crit;            /* spatial coarsening threshold, 0.1 (section 5.1) */
  int32_t allow_space_coarsening;/* 1: apply eq. (3); 0: coarsen in time only */
  int32_t smoother;              /* STMG_SMOOTH_* sequence, default STMG_SMOOTH_SAS */
  int32_t precision;             /* STMG_FP64 | STMG_FP32_REFINED */
  double rtol;                   /* relative residual target of stmg_solve, default 1e-8 */
  int32_t max_cycles;            /* cap of stmg_solve, default 100 */
  int32_t host_only;             /* 1: build host data only (no device), for tests */
  int32_t stream_chunk;          /* residual shape: max values per lane of a row segment, 0 = default (16),
                                    1..16; 32 = LDS-tiled residual (rows in tiles of 64, union staged in LDS) */
  int32_t row_schedule;          /* residual row visiting order: 0 = Hilbert order of edge midpoints with wide rows
                                    in groups of 4 per wavefront (default), 1 = storage order, one row per
                                    wavefront, 2 = Hilbert order, one row per wavefront, 3 = Morton order, groups
                                    of 4; the curve is fixed at setup (stmg_set_stream_tuning switches only
                                    between values with the same curve, or to 1) */
  int32_t leaf_size;             /* nested-dissection leaf size in vertices, default 8 */
  int32_t gemm_rows;             /* supernode GEMM row tile: 0 = chosen per launch, 64 or 32 forced */
  int32_t factor_transpose;      /* also keep P^T for the backward solves: -1 auto, 0 never, 1 always */
  int32_t gemm_splitk;           /* solve K split: 0 auto, -1 never, k >= 2 forced k-way (testing) */
  int32_t device_factor;         /* numeric factorisation: -1 (default) on the GPU when the finest slab
                                    factor has >= 1e6 entries, else on the host; 1 GPU; 0 host */
  int32_t nodal;                 /* STMG_NODAL_EXACT, or k Chebyshev steps (1..16) for K_n^{-1} */
  int32_t graph;                 /* 1 (default): stmg_cycles and stmg_solve capture one iteration as a HIP
                                    graph at first use and replay it (bitwise the same iterates); 0: launch
                                    every kernel each cycle. Launches are eager while profiling. */
  int32_t slab;                  /* STMG_SLAB_EXACT (default), or k (1..16): the slab solves of every level
                                    with N > 1 whose mesh has a coarser one (problem.meshes[mesh + 1]) are
                                    replaced by k steps of Richardson iteration from zero, each preconditioned
                                    by one two-grid cycle on the two meshes (section 5 solves the spatial
                                    problems inexactly); such a level keeps the slab factor of the coarser
                                    mesh only. In the precision form the iteration runs in the FP32
                                    smoother (FP32 diagonals, matrix values and coarse factors). */
} stmg_options;

typedef struct {
  int32_t cycles;                /* V-cycles performed */
  double rel_res;                /* final ||b - L x||_2 / ||b||_2 over interior DOFs */
  double setup_s;                /* wall time of stmg_setup */
  double solve_s;                /* wall time of the last stmg_solve */
  const double *res_history;     /* [cycles] relative residuals, owned by the handle */
} stmg_report;

typedef struct {
  int32_t n_edges;               /* all edges of mesh 0 (full layout width) */
  int32_t n_levels;              /* space-time levels, finest first */
  int32_t pt;
  int64_t device_bytes;          /* device memory held by the handle */
  int64_t factor_bytes;          /* of which triangular factors */
} stmg_info_t;

typedef struct {
  int32_t mesh;                  /* index into problem.meshes */
  int32_t N;                     /* slabs */
  double tau;
  int32_t n_e;                   /* interior edges of that mesh */
  int32_t n_v;                   /* interior vertices */
  int64_t nnz_pattern;           /* nonzeros of the shared M/K pattern */
  int64_t factor_nnz_slab;       /* entries of the slab-block factor L as stored (lower incl. diag,
                                    dense supernode blocks) */
  int64_t factor_nnz_nodal;      /* the same for the nodal factor */
  int32_t n_supernodes_slab;
  double lambda;                 /* eq. (3) anisotropy of this level (its tau, its mesh) */
  int64_t factor_nnz_slab_struct;  /* structural nonzeros of the slab factor L (column counts of the
                                      elimination tree; the zeros of dense supernode blocks excluded) */
  int64_t factor_nnz_nodal_struct; /* the same for the nodal factor */
  int32_t slab_factor_mesh;      /* mesh of the slab factor the level keeps: `mesh` (exact slab solves) or
                                    mesh + 1 (inexact ones, option slab); the slab factor fields above
                                    describe that factor */
  int32_t slab_steps;            /* 0: exact slab solves; k: k two-grid Richardson steps */
} stmg_level_info_t;

typedef struct stmg_handle stmg_handle;

const char *stmg_strerror(int code);
/* Thread-local message of the last failing call in this thread. */
const char *stmg_last_error_message(void);
void stmg_default_options(stmg_options *opt);

/* Build everything a solve needs: topology, FP64 assembly of M, K (Whitney
 * elements, section 3), the space-time hierarchy (time halving, eq. (3) for
 * space), Galerkin coarse operators, nested-dissection orderings, symbolic and
 * numeric factorisations of every level's slab block and nodal matrix K_n, and
 * uploads to HBM. Host arrays are borrowed for the call only. `stream` is a
 * hipStream_t (NULL = default stream). Refuses with STMG_ENOMEM, before any
 * device allocation, when its device-memory estimate exceeds the free memory.
 * GPU factorisations of the slab levels after the largest run on up to 8
 * worker threads, each with its own stream and rocBLAS handle (fewer when
 * their temporaries would not fit; at most the environment's
 * STMG_SETUP_THREADS); the call returns when all are done. STMG_VERBOSE=1 in
 * the environment prints the setup's phases and timings on stderr. On failure
 * *out is NULL and nothing leaks. */
int stmg_setup(const stmg_problem *prob, const stmg_options *opt, void *stream,
               stmg_handle **out);
void stmg_destroy(stmg_handle *h);

int stmg_info(const stmg_handle *h, stmg_info_t *info);
int stmg_level_info(const stmg_handle *h, int32_t level, stmg_level_info_t *info);
/* Edge list of mesh 0: *edge_vertices points to [n_edges][2] (tail, head),
 * owned by the handle. */
int stmg_edges(const stmg_handle *h, int32_t *n_edges, const int32_t **edge_vertices);

/* Solve L x = b (+ initial value) by V-cycles until ||b - Lx|| <= rtol ||b||
 * (section 2.1; tolerance as in section 6). rhs_dev, x_dev: full layout.
 * u0_dev, x0_dev may be NULL (zero). x_dev may alias x0_dev. Returns
 * STMG_ENOTCONV (x holds the last iterate) if max_cycles is reached,
 * STMG_ENUMERIC on a non-finite residual. rep may be NULL. */
int stmg_solve(stmg_handle *h, const double *rhs_dev, const double *u0_dev,
               const double *x0_dev, double *x_dev, stmg_report *rep);

/* Split form of stmg_solve for benchmarking and resuming:
 *   stmg_load:   take rhs (+u0) and initial guess (NULL = 0) into the
 *                handle's internal layout; returns ||b||_2 in *bnorm.
 *   stmg_cycles: n_cycles iterations, each one V-cycle followed by the
 *                residual norm; res_host (may be NULL) receives the n_cycles
 *                relative residuals (this synchronises the stream).
 *   stmg_store:  write the current iterate in full layout. */
int stmg_load(stmg_handle *h, const double *rhs_dev, const double *u0_dev,
              const double *x0_dev, double *bnorm);
int stmg_cycles(stmg_handle *h, int32_t n_cycles, double *res_host);
int stmg_store(stmg_handle *h, double *x_dev);

/* One iteration on caller data, for benchmarks: x <- one V-cycle (section
 * 2.1; in the precision form one refinement step: FP32 V-cycle on the FP64
 * residual, FP64 update) applied to the iterate x for the right-hand side
 * rhs, both device pointers in full layout; x is read and overwritten (its
 * boundary entries become 0). Enqueued on the handle's stream without
 * synchronising; replaces the handle's loaded right-hand side and iterate. */
int stmg_vcycle(stmg_handle *h, const double *rhs_dev, double *x_dev);

/* stmg_cycles for several handles at once (1 to 8, each loaded with
 * stmg_load): n_cycles iterations of every handle, with the slab and nodal
 * solves of each step merged over the handles into one launch per tree
 * height (the slabs of one level of all handles solved together, each with
 * its own factor). The handles must share N_t, p_t, the precision form and
 * the smoother (STMG_EINVAL otherwise, or if a handle appears twice). Runs
 * on the first handle's stream after synchronising the others' streams, and
 * returns when done. Every handle's iterates, norms and histories are
 * bitwise those of stmg_cycles on that handle alone. res_host (may be NULL)
 * receives [n][n_cycles] relative residuals. */
int stmg_cycles_batched(stmg_handle *const *hs, int32_t n, int32_t n_cycles, double *res_host);

/* Convergence rate by power iteration (section 5.1, determining the
 * convergence rates and lambda_crit): V-cycles with a zero right-hand side,
 * starting from the error x0_dev (device, full layout [Nt][pt+1][n_edges];
 * only interior edges are read; typically uniform in [0, 1]), with the l2
 * norm of the iterate taken after every cycle. Runs max_cycles cycles
 * (1..8192), or stops at the first cycle whose norm is below underflow
 * times the starting norm. *rate = the largest reduction factor
 * ||x_k|| / ||x_{k-1}||; rates_host (may be NULL; room for max_cycles
 * values) receives every factor and *n_done (may be NULL) their number.
 * FP64 form only: STMG_EINVAL for a handle in the precision form, a zero
 * x0 or an argument out of range; STMG_ENUMERIC on a non-finite norm. The
 * handle's loaded right-hand side and iterate are replaced (b = 0, x = the
 * last iterate). */
int stmg_power_rate(stmg_handle *h, const double *x0_dev, int32_t max_cycles, double underflow,
                    double *rate, double *rates_host, int32_t *n_done);

/* r = b - L x on the finest level, full layout (r's boundary entries are 0).
 * u0_dev may be NULL. */
int stmg_residual(stmg_handle *h, const double *x_dev, const double *rhs_dev,
                  const double *u0_dev, double *r_dev);

/* stmg_residual for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, same r = b - L x from the same kernels; the
 * internal-layout temporaries (x, b and r, n_interior_edges * Nt * (pt+1)
 * doubles each), which stmg_residual allocates on its first call, come
 * from a fixed device array of 64 MiB that the library holds on every GPU
 * it runs on until the process ends. No device memory is allocated or
 * freed and the stream is not synchronised: r is ready when the handle's
 * stream reaches it. STMG_EINVAL if 3 * n_interior_edges * Nt * (pt+1)
 * exceeds 8 Mi doubles, or if the current device is not the one the handle
 * was set up on. Every call on one GPU uses that GPU's one array and leaves
 * its contents behind (the next call overwrites all it reads): calls that
 * overlap on one GPU, from different streams or handles, race. */
int stmg_residual_noalloc(stmg_handle *h, const double *x_dev, const double *rhs_dev,
                          const double *u0_dev, double *r_dev);

/* Per-level operations in level layout, for parity tests:
 *   STMG_OP_RESIDUAL  out = b - L_l x                    (in = x, in2 = b)
 *   STMG_OP_SMOOTH_S  out = x + omega A_l^{-1}(b - L_l x) (eq. (2))
 *   STMG_OP_NODAL_A   out = x + G Sigma_t K_n^{-1} G^T (b - L_l x) (eq. (8))
 *   STMG_OP_SAS       out = the handle's pre-smoother (S(A(S(x))) for SAS,
 *                     section 4)
 *   STMG_OP_SLAB_SOLVE out = (I (x) A_l^{-1}) in          (in2 unused)
 *   STMG_OP_RESTRICT  out (level l+1) = (P_t^T (x) P_s^T) in (level l)
 *   STMG_OP_PROLONG   out (level l-1) = (P_t (x) P_s) in (level l)
 *   STMG_OP_VCYCLE    out = V-cycle from level l on x = in, rhs = in2
 * `in`, `in2`, `out` are distinct device buffers. */
enum {
  STMG_OP_RESIDUAL = 0, STMG_OP_SMOOTH_S = 1, STMG_OP_NODAL_A = 2, STMG_OP_SAS = 3,
  STMG_OP_SLAB_SOLVE = 4, STMG_OP_RESTRICT = 5, STMG_OP_PROLONG = 6, STMG_OP_VCYCLE = 7
};
int stmg_level_apply(stmg_handle *h, int32_t level, int32_t op, const double *in_dev,
                     const double *in2_dev, double *out_dev);

/* Host copies of level-l spatial operators over that level's interior DOFs in
 * ascending order, as CSR (row_ptr [n+1], col [nnz], val [nnz]); pass NULL
 * arrays to query sizes (*n, *nnz). which: 0 = M, 1 = K, 2 = G (edges x
 * vertices), 3 = K_n, 4 = P_e from level l's mesh to the next finer mesh's
 * (rows = finer interior edges). Works on host_only handles. */
int stmg_export_matrix(const stmg_handle *h, int32_t level, int32_t which, int32_t *n_rows,
                       int32_t *n_cols, int64_t *nnz, int64_t *row_ptr, int32_t *col,
                       double *val);

/* Launch timing for roofline accounting. stmg_profile(h, 1) clears the
 * counters and brackets every subsequent supernode-GEMM and residual launch
 * with HIP events recorded on the handle's stream; stmg_profile(h, 0) stops.
 * stmg_profile_count synchronises the stream and aggregates per kernel
 * (instantiation names as "k_sn_gemm<cd,64,64,bwdT>", "k_residual<double,8,2>");
 * stmg_profile_get returns kernel i's name, launch count, summed duration
 * and summed algorithmic work: flops (one multiply-add per factor entry and
 * right-hand side for the solves; two per nonzero and column for M and K in
 * the residual) and bytes (each operand read once, each result written
 * once). Timing adds no synchronisation inside a cycle. */
int stmg_profile(stmg_handle *h, int32_t enable);
int stmg_profile_count(stmg_handle *h, int32_t *n_kernels);
int stmg_profile_get(stmg_handle *h, int32_t i, char *name, int32_t name_len, int64_t *launches,
                     double *total_ms, double *flops, double *bytes);

/* Changes the residual's launch shape after setup (same meaning and values
 * as the stream_chunk and row_schedule options); results do not depend on
 * it except for the summation order of the residual norm. STMG_EINVAL on an
 * unknown value. For tuning on a live handle without a second setup. */
int stmg_set_stream_tuning(stmg_handle *h, int32_t stream_chunk, int32_t row_schedule);

/* ------------------------------------------------------------- serving
 * A continuous-batching request server. Requests (problem + rhs on the host)
 * get their host setup on worker threads, are admitted to the GPU when their
 * estimated device bytes fit the HBM budget and a slot is free, get their
 * device setup (factorisation, uploads) on a worker thread and their own
 * stream, and are iterated
 * concurrently (one non-blocking HIP stream per active request, one
 * iteration in flight each, convergence polled without blocking); results
 * return to host memory and the request's device memory is released on its
 * stream. Requests of the same cycle shape whose iterations are due together
 * run them batched (their slabs' solves of each level merged into one launch
 * per tree height; see stmg_server_options.batch). Each request computes its
 * values with the same instructions in the same order as it would alone,
 * with deterministic reductions, so its result does not depend on the mix.
 * Thread-safe; the calling thread never blocks on the GPU except in
 * stmg_server_wait. */
typedef struct stmg_server stmg_server;
typedef struct {
  int64_t hbm_budget;            /* device bytes the server may hold; <= 0: 90% of free memory */
  int32_t max_active;            /* requests on the GPU at once (default 16) */
  int32_t setup_threads;         /* host setup workers (default 4) */
  int32_t batch;                 /* 1 (default): due iterations of requests with the same N_t, p_t,
                                    precision form, smoother and nodal solve, and finest interior edge
                                    counts within a factor of 2, run batched (stmg_cycles_batched's
                                    merged solves, up to 8 requests, on a shared stream); 0: never */
} stmg_server_options;
typedef struct {
  int64_t submitted, completed, failed, active, pending;
  double p50_s, p99_s, mean_s;   /* latency from submit to result ready (completed requests) */
  double throughput_req_s;       /* completed / (last completion - first submission) */
  double throughput_dofs;        /* sum over completed of n_e N_t (p_t+1) x cycles, same span */
  int64_t hbm_reserved, hbm_peak, hbm_budget;
  int64_t batched_iterations;    /* batched iterations run (each over 2 to 8 requests) */
  int64_t batched_members;       /* request iterations inside them */
} stmg_server_stats_t;

void stmg_server_default_options(stmg_server_options *opt);
int stmg_server_create(const stmg_server_options *opt, stmg_server **out);
/* Copies the problem (all arrays), options and rhs [Nt][pt+1][n_edges] (and u0
 * [n_edges], may be NULL) from host memory; returns a ticket at once. */
int stmg_submit(stmg_server *s, const stmg_problem *prob, const stmg_options *opt, const double *rhs_host,
                const double *u0_host, uint64_t *ticket);
/* STMG_EAGAIN while the request is queued or running. Otherwise copies the
 * solution (full layout, may be NULL to drop it), fills rep (res_history is
 * NULL), forgets the ticket and returns the request's status: STMG_OK,
 * STMG_ENOTCONV (x is the last iterate), STMG_ENOMEM (larger than the
 * budget), STMG_EINVAL, STMG_ENUMERIC or STMG_EHIP. */
int stmg_poll(stmg_server *s, uint64_t ticket, double *x_host, stmg_report *rep);
/* Blocks until the request has finished or timeout_s passed (STMG_EAGAIN). */
int stmg_server_wait(stmg_server *s, uint64_t ticket, double timeout_s);
int stmg_server_stats(stmg_server *s, stmg_server_stats_t *stats);
/* Stops the threads, waits for in-flight device work and frees everything. */
void stmg_server_destroy(stmg_server *s);

/* Failure injection for tests of the error paths. Arms the k-th allocation
 * the library makes from now on (k >= 1; device buffers and temporaries,
 * and the host arrays of topology, assembly, ordering and factorisation) to
 * fail as if memory were exhausted: the call that reaches it returns
 * STMG_ENOMEM after releasing everything it had allocated. k <= 0 disarms.
 * Returns the number of allocations counted since the previous call and
 * restarts the count. Process-wide; concurrent setups share the count. */
int64_t stmg_debug_fail_alloc(int64_t k);

/* Host copy of a level's factor: which = 0 slab block (complex for pt = 1:
 * values interleaved re, im), 1 nodal matrix K_n. host_only handles return
 * the host factorisation; device handles copy their FP64 panels back from
 * HBM (STMG_ENOSYS for levels that keep only FP32 panels).
 * Layout as used by the solves: DOF new = perm^{-1}(old) in nested-dissection
 * order; supernode s owns columns [col0[s], col0[s+1]), below-diagonal rows
 * rows[rptr[s] .. rptr[s+1]) (new numbering) and the column-major panel
 * P_s = [inv(L_ss); -L_{R,s} inv(L_ss)] at panel + panel_off[s] (scalars).
 * Pass NULL arrays to query sizes. */
int stmg_export_factor(const stmg_handle *h, int32_t level, int32_t which, int32_t *n, int32_t *ns,
                       int64_t *n_rows_total, int64_t *n_panel, int32_t *is_complex, int32_t *perm,
                       int32_t *col0, int64_t *rptr, int32_t *rows, int64_t *panel_off, double *panel);

#ifdef __cplusplus
}
#endif
#endif /* STMG_H */
