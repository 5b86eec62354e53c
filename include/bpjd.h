/*
 * bpjd.h -- C ABI of the MI355X (gfx950) two-level block preconditioned
 * Jacobi-Davidson eigensolver.
 *
 * Problem (Section 2.2, eq. DiscreteVariational, and Algorithm 3.1 of Liang,
 * Wang, Xu, "A Two-Level Block Preconditioned Jacobi-Davidson Method for
 * Multiple and Clustered Eigenvalues of Elliptic Operators"): given the
 * finite-element stiffness matrix K (the form a(.,.)) and mass matrix M (the
 * form b(.,.)), both symmetric, M positive definite, find the k smallest
 * eigenpairs  K x_i = lambda_i M x_i  with  X^T M X = I  (b(u_i,u_j) =
 * delta_ij).  The two-level preconditioner of Section 3 (eq.
 * Preconditioner) needs a coarse space V^H (given by a prolongation P whose
 * range is V^H) and overlapping subdomains (local dof sets of V^(l),
 * Section 2.3); they are passed explicitly (bpjd_dd) or built from a
 * structured coarse grid (bpjd_dd_geom).
 *
 * Conventions
 *   - every function returns an int status: BPJD_OK (0), BPJD_PENDING (>0)
 *     or a negative BPJD_ERR_* code; nothing throws across the ABI;
 *     bpjd_last_error(ctx) gives a human-readable detail of the last failed
 *     call on a context, bpjd_last_error(NULL) that of the calling thread.
 *   - CSR matrices are 0-based, square, with sorted column indices and no
 *     duplicates; K and M store the full symmetric pattern.  K and M may have
 *     different patterns: the library works on their union.
 *   - block vectors (X_init, eigvecs) are row-major n x ncols arrays (the
 *     ncols values of one dof are contiguous).
 *   - "mem" fields say where a pointer lives: BPJD_MEM_HOST or
 *     BPJD_MEM_DEVICE (device memory of the context's GPU).
 *   - input arrays are borrowed for the duration of a call and copied; the
 *     caller may free them on return.  Output buffers are caller-allocated.
 *     Handles are freed only by their *_destroy call.
 *   - all device work of a context is ordered on its HIP stream; a call
 *     that returns results in host memory synchronises that stream.
 *   - device memory: every device byte the library holds comes from the
 *     context's allocator (bpjd_allocator; the default is hipMalloc/hipFree),
 *     obtained when a problem is created (or, for served requests, from the
 *     server's block, obtained when the server is created); solving allocates
 *     nothing.
 *   - one thread per problem; a context may be shared by several problems.
 */
#ifndef BPJD_H
#define BPJD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define BPJD_OK                0
#define BPJD_PENDING           1   /* serving: result not ready yet */
#define BPJD_ERR_ARG          -1   /* bad argument (NULL, size, option) */
#define BPJD_ERR_CSR          -2   /* malformed CSR (bounds, order, not square, asymmetric pattern) */
#define BPJD_ERR_DD           -3   /* bad decomposition: uncovered dof, empty subdomain, s >= dim V^H, band too wide */
#define BPJD_ERR_NOT_SPD      -4   /* M, M_H or a Gram matrix not positive definite; singular local pivot */
#define BPJD_ERR_NOCONV       -5   /* max_iter reached; outputs hold the last iterate */
#define BPJD_ERR_OOM          -6   /* device allocation failed */
#define BPJD_ERR_HIP          -7   /* HIP runtime error */
#define BPJD_ERR_OVER_BUDGET  -8   /* serving: request can never fit the HBM budget */
#define BPJD_ERR_STATE        -9   /* call not valid in the object's current state */

#define BPJD_MEM_HOST    0
#define BPJD_MEM_DEVICE  1

/* stop rule (Algorithm 3.1, Step 4, and the residual rule of the configs) */
#define BPJD_STOP_RESIDUAL  0   /* max_{i<k} ||K x_i - lambda_i M x_i||_2 / (lambda_i ||M x_i||_2) <= tol */
#define BPJD_STOP_PAPER     1   /* sum_{i<s} |lambda_i^{k+1} - lambda_i^k| < tol */

/* subspace W^{k+1} (remark after Algorithm 3.1) */
#define BPJD_SUBSPACE_UU   0    /* W^{k+1} = U^{k-1} + U^k + span{t_i}  (fixed dimension 3s) */
#define BPJD_SUBSPACE_U    1    /* W^{k+1} = U^k + span{t_i}            (fixed dimension 2s) */
#define BPJD_SUBSPACE_GROW 2    /* W^{k+1} = W^k + span{t_i} (Algorithm 3.1, Step 3 as written:
                                   dimension s (k+1) after k steps) */

/* precision of the local subdomain factorisations and solves */
#define BPJD_PREC_FP64   0      /* everything in FP64 */
#define BPJD_PREC_MIXED  1      /* local factor/solve in FP32; residual, projection, coarse solve, RR in FP64 */

/* largest block size s = k + guard (the Rayleigh-Ritz problem has dimension <= 3 s) */
#define BPJD_MAX_BLOCK   20

typedef struct bpjd_ctx bpjd_ctx;
typedef struct bpjd_problem bpjd_problem;
typedef struct bpjd_server bpjd_server;

typedef struct {
    int32_t n_rows, n_cols;
    int64_t nnz;
    const int32_t* rowptr;      /* n_rows + 1 */
    const int32_t* col;         /* nnz */
    const double*  val;         /* nnz */
    int32_t mem;                /* BPJD_MEM_HOST or BPJD_MEM_DEVICE (all three arrays) */
} bpjd_csr;

/* Explicit decomposition (Section 2.3).  P: n x n_H prolongation, range(P) =
 * V^H; subdomain l holds the dofs sub_idx[sub_ptr[l] .. sub_ptr[l+1]) (any
 * order; they are the dofs interior to the enlarged subdomain Omega'_l).
 * Every dof must lie in at least one subdomain.  sub_ptr/sub_idx: host. */
typedef struct {
    bpjd_csr P;
    int32_t n_sub;
    const int32_t* sub_ptr;     /* n_sub + 1 */
    const int32_t* sub_idx;
} bpjd_dd;

/* Structured decomposition for P1 on a domain made of cells of a coarse grid
 * of lines cx[0..n_cx) x cy[0..n_cy) (each coarse cell cut by its "/"
 * diagonal, like the fine cells), whose fine mesh refines that grid: a
 * rectangle, or a union of coarse cells such as the L-shaped domain of
 * Section 6.  The library builds P (nodal interpolation of the coarse P1 hat
 * functions at the dof coordinates; a coarse vertex has a hat function when a
 * dof sits on it) and the subdomains Omega_l of Section 2.3: each closed coarse
 * cell, or each closed coarse triangle (cell_shape), grown by
 * (overlap_layers - 1) graph layers of the union pattern of K and M, i.e.
 * overlap delta = overlap_layers * h; cells or triangles holding no dof are
 * skipped.  All arrays: host. */
#define BPJD_CELL_SQUARE    0   /* Omega_l = a coarse cell (two coarse triangles) */
#define BPJD_CELL_TRIANGLE  1   /* Omega_l = a coarse triangle (the coarse elements, as in Section 6) */
typedef struct {
    const double* coords;       /* n x 2, row-major (x, y) of each dof */
    int32_t n_cx, n_cy;
    const double* cx;
    const double* cy;
    int32_t overlap_layers;     /* >= 1 */
    int32_t cell_shape;         /* BPJD_CELL_SQUARE or BPJD_CELL_TRIANGLE */
} bpjd_dd_geom;

typedef struct {
    int32_t k;                  /* eigenpairs wanted (>= 1) */
    int32_t guard;              /* extra block columns: block size s = k + guard <= BPJD_MAX_BLOCK
                                   (Assumption 1 remark) */
    int32_t max_iter;           /* outer iterations before BPJD_ERR_NOCONV */
    double  tol;                /* tolerance of the stop rule */
    int32_t stop_rule;          /* BPJD_STOP_* */
    int32_t subspace;           /* BPJD_SUBSPACE_* */
    int32_t precision;          /* BPJD_PREC_* */
    int32_t n_init;             /* 0, or columns of X_init added to the coarse start (Step 1) */
    const double* X_init;       /* host, n x n_init row-major, or NULL */
    int32_t profile;            /* 0: off; 1: time every phase with HIP events (bpjd_stats.phase_ms);
                                   2: time only the local-solve phase (two events per iteration) */
    int32_t graphs;             /* 1 (default): each outer iteration is captured once per problem as a
                                   HIP graph and replayed; 0: kernels are launched one by one.
                                   Graphs are not used while phases are timed, nor for served
                                   requests.  A capture needs the context's stream to be a
                                   created (non-null) stream with no device-wide synchronisation
                                   (another thread's hipFree, hipDeviceSynchronize) meanwhile. */
    int32_t autotune;           /* 1 (default): when a problem is first set up, the launch shapes that
                                   leave the arithmetic unchanged (threads per system of the windowed
                                   local solver: 64, 128 or 256; one or two SpMM columns per lane) are
                                   timed on its own data and the fastest is kept, per process and keyed
                                   by the problem's shape (and appended to the file named by the
                                   environment variable BPJD_TUNE_CACHE, read at the first tuning, when
                                   it is set).  Results are the same bit for bit either way.
                                   0: fixed choices (256 threads, two columns per lane). */
    int32_t local_threads;      /* threads per system of the windowed local solver: 0 (default) =
                                   the autotuner's choice (256 without autotune), or exactly 64,
                                   128 or 256, which also selects the windowed solver where the
                                   wide blocked one would run.  The local solver is chosen by the
                                   largest half-bandwidth w and lower entries per local row E:
                                   blocked MFMA with a 64-row window (w <= 48, E <= 8) or a 96-row
                                   window (w <= 80, E <= 8); in mixed precision the wide blocked
                                   solver with a 192-row window (49 <= w <= 176, E <= 20); the
                                   windowed LDS solver otherwise (w <= 191).  The windowed
                                   solver's arithmetic is the same for all thread counts. */
    int32_t spmm_form;          /* lane layout of the fused K/M SpMM: 0 (default) = the autotuner's
                                   choice (BPJD_SPMM_PAIRS without autotune); or exactly one of
                                   BPJD_SPMM_*.  Every form adds a row's entries in the same order,
                                   so the results are the same bit for bit. */
} bpjd_opts;

/* SpMM lane layouts (bpjd_opts.spmm_form) */
#define BPJD_SPMM_PAIRS   1     /* two adjacent columns per lane (even block sizes; else as COLUMN) */
#define BPJD_SPMM_COLUMN  2     /* one column per lane, a power-of-two group of lanes per row */
#define BPJD_SPMM_FLAT    3     /* one lane per (row, column), lanes numbered row by row */

/* phases timed when bpjd_opts.profile = 1 (profile = 2: BPJD_PHASE_LOCAL only) */
#define BPJD_PHASE_LOCAL     0  /* batched local factor + solve kernel */
#define BPJD_PHASE_SPMM      1  /* fused K/M SpMM */
#define BPJD_PHASE_COARSE    2  /* restriction + coarse eigenbasis apply */
#define BPJD_PHASE_GATHER    3  /* subdomain gather + overlap scatter/prolongation */
#define BPJD_PHASE_ORTHO     4  /* projection + M-orthonormalisation */
#define BPJD_PHASE_RR        5  /* Rayleigh-Ritz (Gram, small eigenproblem, basis update) */
#define BPJD_PHASE_RESIDUAL  6  /* residual block and norms */
#define BPJD_PHASE_SETUP     7  /* Galerkin + coarse eigenproblem + start block */
#define BPJD_NUM_PHASES      8

typedef struct {
    int32_t iterations;         /* outer iterations performed */
    int32_t converged;          /* 1 if the stop rule was met */
    double  stop_value;         /* sum_{i<s} |lambda_i^{k+1} - lambda_i^k| of the last iteration */
    double  max_residual;       /* max_{i<k} rho_i of the returned pairs */
    double  setup_ms;           /* device numeric setup (Galerkin, coarse eigenproblem, start block) */
    double  iterate_ms;         /* outer iterations */
    int32_t n_sub;              /* subdomains */
    int32_t n_coarse;           /* dim V^H */
    int32_t max_local;          /* largest subdomain */
    int32_t max_band;           /* largest local half-bandwidth */
    double  residuals[64];      /* rho_i of the returned pairs, i < min(k, 64) */
    double  phase_ms[8];        /* device time per phase (profile = 1), summed over the solve */
    int32_t phase_count[8];     /* launches timed per phase */
    double  queue_ms;           /* served requests: submission to admission (0 for bpjd_solve) */
    double  latency_ms;         /* served requests: submission to result in host memory */
    int32_t graph_iterations;   /* outer iterations replayed from a captured HIP graph */
    int32_t spmm_form;          /* SpMM lane layout the solve used (BPJD_SPMM_*) */
} bpjd_stats;

/* Default options: k as given, guard 0, max_iter 500, tol 1e-8, residual
 * stop rule, UU subspace, mixed precision, no initial block. */
void bpjd_opts_default(bpjd_opts* o, int32_t k);

/* Trace.  When the environment variable BPJD_TRACE is set as a problem is created
 * ("1" or "stderr": standard error; any other value: a file the lines are appended
 * to), the library writes one JSON object per line:
 *   {"event": "create", "stage": ..., "ms": ...}        host planning stages;
 *   {"event": "iteration", "problem", "it", "fresh", "rho_max", "stop_value",
 *    "lambda": [s values], "rho": [k values]}          every residual read-back;
 *   {"event": "rayleigh_ritz", "problem", "it", "m", "dropped_in", "dropped_out",
 *    "theta": [m values]}                               every UU/U Rayleigh-Ritz step;
 *   {"event": "solve", "problem", "iterations", "converged", "stop_value",
 *    "setup_ms", "iterate_ms"}                          the end of each solve.
 * A traced problem launches its iterations directly (no graph replay) and
 * synchronises its stream once per Rayleigh-Ritz step. */

/* ---- context ----------------------------------------------------------- */
/* Device memory provider of a context (for instance a framework's caching
 * allocator).  alloc(bytes, user) returns device memory of the context's GPU,
 * at least 256-byte aligned, or NULL when it cannot; free(ptr, user) gives it
 * back.  The library calls them from the thread that creates or destroys a
 * problem or a server; it synchronises the context's stream before it frees,
 * so no kernel still uses a block handed back. */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void  (*free)(void* ptr, void* user);
    void* user;
} bpjd_allocator;

/* device: HIP device ordinal.  allocator: NULL for hipMalloc/hipFree, else
 * copied (its callbacks and user pointer must stay valid until
 * bpjd_ctx_destroy).  hip_stream: a hipStream_t to order all work on, or NULL
 * for a stream the context creates (default priority).
 * Errors: BPJD_ERR_ARG (bad ordinal, an allocator with one callback), _HIP. */
int  bpjd_ctx_create(int device, const bpjd_allocator* allocator, void* hip_stream, bpjd_ctx** out);
void bpjd_ctx_destroy(bpjd_ctx* ctx);

/* ---- problems ---------------------------------------------------------- */
/* Validates K, M and the decomposition, builds the structural data (union
 * pattern, subdomain maps, local band layout, coarse pattern) on the host
 * and uploads it together with the matrix values.  Device memory for the
 * whole solve is allocated here; bpjd_solve allocates nothing.
 * Local solver limits (half-bandwidth w in the subdomain's ascending dof order):
 * w <= 191 and at most 64 lower entries per local row; the windowed solver used
 * above w = 80 (or above 8 lower entries) keeps (w+1)^2 + 2(w+1) entries of the
 * solve precision in one workgroup's LDS (160 KB on MI355X: FP64 up to w = 141,
 * FP32 up to 191).  Beyond these the call returns BPJD_ERR_DD before any launch.
 * Errors: BPJD_ERR_ARG, _CSR, _DD, _OOM, _HIP. */
int bpjd_problem_create(bpjd_ctx* ctx, const bpjd_csr* K, const bpjd_csr* M,
                        const bpjd_dd* dd, const bpjd_opts* opts, bpjd_problem** out);
int bpjd_problem_create_geom(bpjd_ctx* ctx, const bpjd_csr* K, const bpjd_csr* M,
                             const bpjd_dd_geom* geom, const bpjd_opts* opts, bpjd_problem** out);
void bpjd_problem_destroy(bpjd_problem* p);

/* Replace the values of K and M (same patterns as at creation), host or
 * device arrays of the original nnz of each matrix. */
int bpjd_problem_set_values(bpjd_problem* p, const double* Kval, const double* Mval, int32_t mem);

/* Size queries: n (dofs), n_H, number of subdomains, block size s. */
int bpjd_problem_dims(const bpjd_problem* p, int32_t* n, int32_t* n_coarse, int32_t* n_sub, int32_t* s);

/* Device bytes the problem holds (what a server's HBM budget counts for it). */
int bpjd_problem_footprint(const bpjd_problem* p, uint64_t* bytes);

/* Subdomain sizes n_l and local half-bandwidths w_l (arrays of n_sub, host). */
int bpjd_problem_local_sizes(const bpjd_problem* p, int32_t* n_l, int32_t* bw);

/* Run Algorithm 3.1: device numeric setup (Galerkin coarse operators, coarse
 * generalized eigenproblem, start block, Step 1) and outer iterations (Steps
 * 2-4) until the stop rule holds.  eigvals: k doubles ascending; eigvecs:
 * n x k row-major, M-orthonormal; either may be NULL.  mem says where both
 * live.  st may be NULL.  Returns BPJD_OK, or BPJD_ERR_NOCONV with the last
 * iterate in the outputs, or another error. */
int bpjd_solve(bpjd_problem* p, double* eigvals, double* eigvecs, int32_t mem, bpjd_stats* st);

/* ---- stage entry points (one piece of an outer iteration each) ---------- */
/* Two-level preconditioner (eq. Preconditioner) applied to the residual
 * block of (X, lambda): with F = M X diag(lambda) - K X,
 *   Z_i = P (B_0,i)^{-1} Q^H_{s+1} Q^H r_i + sum_l R_l^T (K_l - sigma_{l,i} M_l)^{-1} R_l F_i,
 * where sigma_{l,i} = lambda_i whenever K_l - lambda_i M_l is positive definite
 * (the local solvability the analysis of Section 3 rests on: the lowest local
 * eigenvalue is of order H^{-2m}, far above lambda_i), and sigma_{l,i} = 0 on a
 * subdomain where it is not (the LDL^T factorisation met a negative pivot:
 * a strong coefficient contrast put a local Dirichlet eigenvalue below
 * lambda_i); there the local solve is K_l^{-1}, a positive definite Schwarz
 * solve.  Needs the coarse eigenbasis: call bpjd_setup first (bpjd_solve does).
 * X, Z: n x s row-major; lambda: s values.  All three in `mem`. */
int bpjd_setup(bpjd_problem* p);
int bpjd_apply_preconditioner(bpjd_problem* p, const double* X, const double* lambda,
                              double* Z, int32_t mem);
/* Fused SpMM  KX = K X, MX = M X  for an n x ncols block (ncols <= 64). */
int bpjd_spmm(bpjd_problem* p, const double* X, int32_t ncols, double* KX, double* MX, int32_t mem);
/* Coarse eigenvalues (ascending, n_H values) from the last setup. */
int bpjd_coarse_eigenvalues(bpjd_problem* p, double* lamH, int32_t mem);

/* ---- allocation-free call -------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops that forbid allocation): the coarse generalized eigenproblem of
 * the numeric setup (the spectral split of V^H behind the coarse term, computed
 * by bpjd_setup and read by bpjd_coarse_eigenvalues) on caller-given dense
 * matrices, with no allocation of any kind and no host synchronisation.
 *   K_H Y = M_H Y diag(lamH),  Y^T M_H Y = I,  lamH ascending.
 * KH, MH: n_H x n_H row-major symmetric (M_H positive definite), lower bandwidth
 * bw (entries farther than bw from the diagonal are zero; n_H - 1 if unknown),
 * read only.  lamH: n_H values; Y: n_H x n_H row-major, eigenvector j in column
 * j; info: one int32 set to 0, or to 2 when M_H is not positive definite.  All
 * device pointers of the context's GPU.  The work is enqueued on the context's
 * stream and the call returns at once (results and info are valid when that
 * stream reaches this point).  Working arrays: a fixed device array of the
 * library, about 8 MB per GPU, held until the process ends, shared by every
 * call on that GPU: calls that overlap in time on one GPU race.  Errors (before
 * anything is enqueued): BPJD_ERR_ARG (NULL, n_H outside 1..320, bw outside
 * 0..n_H-1), BPJD_ERR_STATE, BPJD_ERR_HIP. */
int bpjd_coarse_eigen_noalloc(bpjd_ctx* ctx, int32_t n_H, int32_t bw, const double* KH, const double* MH,
                              double* lamH, double* Y, int32_t* info);

/* ---- serving: continuous batching of independent solves ------------------
 * A server solves many problems of the form above (a stream of requests,
 * each its own K, M, decomposition and options) on the context's GPU.
 * Requests are admitted in submission order as soon as a solve slot is free
 * and the request's device footprint fits the HBM budget; every admitted
 * request runs Algorithm 3.1 on a slot of its own (its own stream), and the
 * outer iterations of all admitted requests advance together, so their
 * kernels overlap on the device.  A request's result does not depend on what
 * else runs.  Served matrices and decompositions are host arrays; they are
 * copied at submission.  Submit and poll may be called from any thread. */
typedef struct {
    uint64_t submitted;         /* requests accepted by bpjd_server_submit */
    uint64_t completed;         /* requests with a final status (success or error) */
    uint64_t failed;            /* completed with an error other than BPJD_ERR_NOCONV */
    uint32_t queued;            /* waiting for admission */
    uint32_t running;           /* admitted, on the device */
    uint32_t peak_running;      /* most requests on the device at once */
    uint32_t max_slots;
    uint64_t budget_bytes;      /* HBM budget of admitted requests */
    uint64_t bytes_in_use;      /* device bytes of the admitted requests */
    uint64_t peak_bytes;        /* largest bytes_in_use seen */
} bpjd_server_info;

/* hbm_budget_bytes: device bytes all admitted requests may hold together (0:
 * 90 % of the device memory free at creation).  max_slots: requests on the
 * device at once, 1..64.  Errors: BPJD_ERR_ARG, _HIP. */
int  bpjd_server_create(bpjd_ctx* ctx, size_t hbm_budget_bytes, int32_t max_slots, bpjd_server** out);
/* Queue one request; exactly one of dd / geom is given (as for
 * bpjd_problem_create / _create_geom).  The problem is validated when it is
 * planned for admission: errors found then (BPJD_ERR_CSR, _DD, _ARG, and
 * BPJD_ERR_OVER_BUDGET when it can never fit the budget) are returned by
 * bpjd_server_poll.  Errors here: BPJD_ERR_ARG, _DD, _STATE (shutting down). */
int  bpjd_server_submit(bpjd_server* s, const bpjd_csr* K, const bpjd_csr* M, const bpjd_dd* dd,
                        const bpjd_dd_geom* geom, const bpjd_opts* opts, uint64_t* req_id);
/* BPJD_PENDING while the request is queued or running.  Otherwise its final
 * status (as bpjd_solve's), with eigvals (k) and eigvecs (n x k row-major)
 * copied to the host buffers given (either may be NULL) and the request
 * released: a later poll of the same id is BPJD_ERR_ARG. */
int  bpjd_server_poll(bpjd_server* s, uint64_t req_id, double* eigvals, double* eigvecs, bpjd_stats* st);
int  bpjd_server_get_info(bpjd_server* s, bpjd_server_info* out);
/* Stops admission, waits for the solves on the device, frees everything;
 * requests not yet polled are dropped. */
void bpjd_server_destroy(bpjd_server* s);

/* ---- errors ------------------------------------------------------------ */
const char* bpjd_strerror(int code);
/* ctx != NULL: the message of the last failed call made on that context (on
 * its problems or its server) from any thread; NULL: the last failure of the
 * calling thread.  The text is copied into storage of the calling thread and
 * stays valid until that thread's next call of bpjd_last_error. */
const char* bpjd_last_error(const bpjd_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* BPJD_H */
