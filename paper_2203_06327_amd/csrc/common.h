// Internal declarations shared by the library's translation units.
// Every kernel is launched through a host launcher defined next to it, so the
// .hip files link without relocatable device code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bpjd.h"

namespace bpjd {

// ---- error plumbing ---------------------------------------------------------
// fail()/set_error() record the message for the calling thread and, while an ABI call
// on a context is in progress on this thread (CtxScope), for that context as well.
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
// JSON-lines trace (environment variable BPJD_TRACE: "1"/"stderr", or a file to append to)
bool trace_on();
void trace_line(const std::string& json);
struct CtxScope {
    explicit CtxScope(bpjd_ctx* c);
    ~CtxScope();
    bpjd_ctx* prev;
};

// ---- device memory -----------------------------------------------------------
// Sub-allocator over one device block (a server's HBM budget): first fit over an
// address-ordered free list with coalescing, 4096-byte granularity.  Thread-safe.
struct DevArena {
    std::mutex mu;
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;    // offset -> length
    static size_t round(size_t b) { return (std::max<size_t>(b, 8) + 4095) & ~size_t(4095); }
    void* alloc(size_t bytes);
    void release(void* p, size_t bytes);
    // places blocks of all these sizes at once (first fit, in order), or none of them
    bool alloc_all(const std::vector<size_t>& sizes, std::vector<void*>& out);
};
// one device block of a problem and how it was obtained
struct DevBlock {
    void* ptr;
    size_t bytes;
    int route;                          // 0 hipMalloc, 1 the context's allocator, 2 the arena
};

#define BPJD_HIP(call)                                                                 \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::bpjd::fail(BPJD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define BPJD_TRY(expr)              \
    do {                            \
        int r_ = (expr);            \
        if (r_ < 0) return r_;      \
    } while (0)

// Device status word bits raised by kernels (read back by the host).
enum : int {
    STATUS_LOCAL_PIVOT = 1,       // zero/non-finite pivot in a local LDL^T factorisation
    STATUS_COARSE_NOT_SPD = 2,    // M_H not positive definite
    STATUS_GRAM_DROP = 4,         // a new direction was linearly dependent and dropped
    STATUS_NONFINITE = 8,         // NaN/Inf met in a reduction
};

inline int grid_for(long long work, int block) {
    long long g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 2147483647LL) g = 2147483647LL;
    return (int)g;
}

// Column-blocked n x (blocks * bw) matrices: element (r, c) lies at
// (c / bw) * bs + r * ld + c % bw, i.e. consecutive row-major n x bw blocks (ld = bw,
// bs = n * bw).  A plain row-major matrix is bw >= its column count, bs unused.
struct BlockGeom {
    int ld;
    int bw;
    long long bs;
    __host__ __device__ long long col_offset(int c) const { return (long long)(c / bw) * bs + c % bw; }
};

// ---- launchers: block linear algebra (blas.hip) -------------------------------
// KX = K X, MX = M X on the union pattern (km holds (K, M) value pairs).
void launch_spmm_km(hipStream_t st, int n, const int* rowptr, const int* col, const double2* km,
                    const double* X, int ldx, int ncols, double* KX, int ldk, double* MX, int ldm, int variant = 0);
// Y = A * B with A CSR (rows x ?) and B dense (row-major, ldb), ncols columns; Y(ldy).
// accumulate: Y += instead of Y =.
void launch_csr_dense(hipStream_t st, int rows, const int* ptr, const int* col, const double* val,
                      const double* B, int ldb, int ncols, double* Y, int ldy, bool accumulate);
// F = MX diag(lam) - KX; colsq[0..s) = ||F_i||^2, colsq[s..2s) = ||MX_i||^2 (two-pass, deterministic).
void launch_residual(hipStream_t st, int n, int s, const double* KX, int ldk, const double* MX, int ldm,
                     const double* lam, double* F, int ldf, double* partial, int npart, double* colsq, double* aux,
                     const int* status);
// C (a x b, row-major) = A^T B with A: n x a, B: n x b, both laid out as g; deterministic
// two-pass.
void launch_gram(hipStream_t st, int n, int a, int b, const double* A, const double* B, BlockGeom g,
                 double* partial, int npart, double* C);
// Y(:, 0..b) = beta*Y + alpha * A(:, 0..a) * C, C a x b row-major (ldc = b), A and Y laid
// out as g.  Batched over up to three (A, Y) pairs sharing C: Y_k = beta Y_k + alpha A_k C
// (a, b <= 64).
void launch_gemm_rows(hipStream_t st, int n, int a, int b, double alpha, const double* const* A, double* const* Y,
                      int count, BlockGeom g, const double* C, double beta);
// Batched in place Y_k = Y_k C (b <= 64), Y laid out as g.
void launch_rightmul_rows(hipStream_t st, int n, int b, double* const* Y, int count, BlockGeom g, const double* C);
// Copy/convert helpers.
void launch_copy_cols(hipStream_t st, int n, int ncols, const double* src, int lds, double* dst, int ldd);
void launch_fill(hipStream_t st, long long count, double* dst, double value);
int  num_partials(int n);

// ---- launchers: preconditioner (precond.hip) --------------------------------
void launch_galerkin(hipStream_t st, int n, int nH, const int* rowptr, const int* col, const double2* km,
                     const int* Pptr, const int* Pcol, const double* Pval,
                     const int* PTptr, const int* PTcol, const double* PTval,
                     const int* kpptr, const int* kpcol, double2* kpval,
                     const int* khptr, const int* khcol, int nnzKH, double* KH, double* MH);
// Zhat = Y (C / (lamH_j - lam_i), rows j < s zeroed) with C = Y^T G; G = P^T F.
void launch_coarse_apply(hipStream_t st, int n, int nH, int s,
                         const int* PTptr, const int* PTcol, const double* PTval,
                         const double* F, int ldf, const double* Y, const double* YT, const double* lamH,
                         const double* lam, double* G, double* Cw, double* Zhat, int maxPT, double* part,
                         long long part_cap);
void launch_gather_f64(hipStream_t st, int sumN, int s, const int* subidx, const double* F, int ldf, double* Floc);
void launch_gather_f32(hipStream_t st, int sumN, int s, const int* subidx, const double* F, int ldf, float* Floc);
// Batched local LDL^T factor + solve, one wavefront per (subdomain, shift).  Shift
// lambda_i, or 0 for a system whose factorisation meets a negative pivot (the local
// matrix is indefinite).  mode 0 solves every system (the windowed solver redoes an
// indefinite one in place); mode 1 redoes the blocked solver's indefinite systems
// with shift 0 (no-op for the windowed solver).  negflag: nsub * s ints of scratch.
// Floc/zloc: [s][sumN].  Local rows come as E fixed slots (band offset sd, (K, M)
// pair sv).  blocked = 4 or 6: the MFMA solver with a window of 16 * blocked rows
// (band <= 48 or <= 80, E <= 8; Lwork: bws x 16 panels per (l, i)); blocked = 0: the
// windowed solver (Lwork: n_l (bw_l + 1) per (l, i)).
void launch_local_solve_f64(hipStream_t st, int mode, int nsub, int s, int maxC, long long sumN,
                            const int* subptr, const int* bw, int blocked, int E, int bws, const int* sd,
                            const double2* sv,
                            const double* lam, const double* Floc, double* zloc, double* Lwork,
                            const long long* Loff, const int* sysord, int* status, int* negflag,
                            int threads = 256);
void launch_local_solve_f32(hipStream_t st, int mode, int nsub, int s, int maxC, long long sumN,
                            const int* subptr, const int* bw, int blocked, int E, int bws, const int* sd,
                            const double2* sv,
                            const double* lam, const float* Floc, float* zloc, float* Lwork,
                            const long long* Loff, const int* sysord, int* status, int* negflag,
                            int threads = 256);
// Numeric local extraction: fixed-slot lower entries (offset, (K, M)) of every local row.
void launch_extract_local(hipStream_t st, long long sumN, int E, const int* lptr, const int* ldd, const int* lpos,
                          const double2* km, int* sd, double2* sv);
// Z(d, i) = sum_b P(d,b) Zhat(b,i) + sum_{(l,r) covering d} zloc_i(l,r)  (deterministic order).
void launch_scatter_f64(hipStream_t st, int n, int s, int sumN, const int* Pptr, const int* Pcol, const double* Pval,
                        const double* Zhat, const int* rptr, const int* ridx, const double* zloc, double* Z, int ldz);
void launch_scatter_f32(hipStream_t st, int n, int s, int sumN, const int* Pptr, const int* Pcol, const double* Pval,
                        const double* Zhat, const int* rptr, const int* ridx, const float* zloc, double* Z, int ldz);

// ---- launchers: small dense kernels (dense.hip) -----------------------------
// Lower Cholesky of an n x n SPD matrix (row-major, in place, lower part); status bit on failure.
void launch_cholesky(hipStream_t st, int n, int bw, double* A, int* status, int status_bit);
// Solve L X = B for X (L lower n x n, B n x nrhs row-major with ldb), in place in B.
void launch_trsm_band(hipStream_t st, int n, int bw, int nrhs, const double* L, double* X, int ldx, bool backward);
// Symmetric eigensolver (cyclic Jacobi, one workgroup): A n x n (destroyed), eigenvalues
// ascending in w, eigenvectors as columns of V (n x n row-major). work: 2 n^2 doubles.
// Symmetric eigensolver for n <= 1024 (Householder tridiagonalisation, bisection,
// inverse iteration with re-orthogonalised clusters, back-transformation): A (n x n)
// destroyed, eigenvalues ascending in w, eigenvectors as columns of V.
// work: n*n doubles, small: 3n doubles, scratch: 5 n*n doubles.
void launch_sym_eig(hipStream_t st, int n, double* A, double* w, double* V, double* work, double* small,
                    double* scratch, int* status);
// Transpose-copy helpers for the coarse eigenproblem.
void launch_transpose(hipStream_t st, int n, const double* A, double* AT);
// CholQR coefficients: G (b x b) -> C = D^{-1/2} L^{-T} (G scaled by D = diag(G) = L L^T);
// directions with a pivot below the drop tolerance get a zero column and dropped[j] = 1.
void launch_cholqr_coef(hipStream_t st, int b, const double* G, double* C, int* dropped, int* status);
// Growing subspace: write the Gram block C ((m + s) x s: W^T K T for the m + s columns of
// W, T included) into the symmetric H (ld ldh) as rows/columns m .. m + s - 1; a dropped
// (zero) new column j gets the diagonal entry 4 trace(H) + 1, above every Ritz value.
void launch_grow_place(hipStream_t st, int m, int s, const double* C, const int* dropped, double* H, int ldh);
// Rayleigh-Ritz coefficient step: given H (m x m) and the dropped flags of all m columns
// of W, returns theta (m), Cfull (m x 2s) = [Q_s | orthonormal basis of span{E_x, Q_s}
// minus Q_s] and the dropped flags of the new basis' first 2s (or s) columns.
void launch_rr_coef(hipStream_t st, int m, int s, int with_p, const double* H, const int* drop_in, int* drop_out,
                    double* theta, double* lam, double* Cfull);

// ---- allocation-free coarse eigenproblem (noalloc.hip) --------------------------
// Looks up this device's scratch address; called once per device with it current.
int noalloc_init(int device);

// ---- problem creation in two steps and the stepwise solve (api.hip) ----------
struct HostPlan;
// Validate and plan a problem on the host (no device memory); fills footprint.
int plan_problem(bpjd_ctx* ctx, const bpjd_csr* K, const bpjd_csr* M, const bpjd_dd* dd, const bpjd_dd_geom* geom,
                 const bpjd_opts* opts, bpjd_problem** out);
// Allocate and upload a planned problem (on p->ctx's device).
int materialize_problem(bpjd_problem* p);
// Sizes of the device blocks materialize_problem will allocate for a planned problem.
std::vector<size_t> planned_blocks(bpjd_problem* p);
// One solve as a sequence of stages, each ending in a read-back event.
struct SolveRun;
int  run_create(bpjd_problem* p, SolveRun** out);
void run_destroy(SolveRun* r);
int  run_begin(SolveRun* r);       // enqueue the numeric setup
int  run_poll(SolveRun* r);        // 1: pending read-back arrived, 0: not yet, < 0: error
int  run_wait(SolveRun* r);        // spin until run_poll != 0
int  run_advance(SolveRun* r);     // 1: finished, 0: next stage enqueued, < 0: error
int  run_finish(SolveRun* r, double* eigvals, double* eigvecs, int mem, bpjd_stats* st);

}  // namespace bpjd

// ---- the opaque objects ---------------------------------------------------------
struct bpjd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bpjd_allocator alloc{};            // alloc.alloc == NULL: hipMalloc / hipFree
    bpjd::DevArena* arena = nullptr;   // a server's slot: device memory comes from the server's block
    double* hbuf = nullptr;            // a server's slot: its pinned read-back buffer (owned by the server)
    std::mutex err_mu;
    std::string last_error;            // message of the last failed ABI call on this context
};

// Host arrays that are filled right after they are sized: resize leaves their elements
// uninitialised (no zero pass over tens of megabytes before the copy that overwrites it).
template <typename T>
struct DefaultInitAlloc : std::allocator<T> {
    template <typename U>
    struct rebind {
        using other = DefaultInitAlloc<U>;
    };
    DefaultInitAlloc() = default;
    template <typename U>
    DefaultInitAlloc(const DefaultInitAlloc<U>&) noexcept {}
    template <typename U>
    void construct(U* q) noexcept {
        ::new (static_cast<void*>(q)) U;
    }
    template <typename U, typename... Args>
    void construct(U* q, Args&&... args) {
        ::new (static_cast<void*>(q)) U(std::forward<Args>(args)...);
    }
};
template <typename T>
using fillvec = std::vector<T, DefaultInitAlloc<T>>;

struct bpjd_problem {
    bpjd_ctx* ctx = nullptr;
    bpjd_opts opts{};
    int n = 0, nH = 0, nsub = 0, s = 0, k = 0;
    long long nnz = 0;                 // union pattern
    long long sumN = 0;                // sum of subdomain sizes
    int maxN = 0, maxBW = 0, maxC = 0;
    long long nnzK = 0, nnzM = 0;
    fillvec<long long> Kmap, Mmap;     // original nnz position -> union position
    std::vector<double> X_init;        // n x s (host copy), optional
    int n_init = 0;

    // device structural data
    int *rowptr = nullptr, *col = nullptr;
    double2* km = nullptr;
    int *Pptr = nullptr, *Pcol = nullptr; double* Pval = nullptr;
    int *PTptr = nullptr, *PTcol = nullptr; double* PTval = nullptr;
    int *kpptr = nullptr, *kpcol = nullptr; double2* kpval = nullptr;
    int *khptr = nullptr, *khcol = nullptr;
    int *subptr = nullptr, *subidx = nullptr, *bw = nullptr;
    int *lptr = nullptr, *ldd = nullptr, *lpos = nullptr;
    int *rptr = nullptr, *ridx = nullptr;
    long long* Loff = nullptr;
    int* sysord = nullptr;             // launch order of the local systems (larger subdomains first)
    int slotE = 0;                     // fixed slots per local row (lower entries incl. the diagonal)
    bool blocked = false;              // local solver: blocked MFMA (true) or windowed
    int mfma_nt = 0;                   // blocked solver's window tile-rows (4 or 6), 0 = windowed
    int bws = 64;                      // stored rows per factor column (blocked solver)
    int* sd = nullptr;
    double2* sv = nullptr;

    // device numeric workspace
    double *KH = nullptr, *MH = nullptr, *Y = nullptr, *lamH = nullptr, *jwork = nullptr;
    double* esmall = nullptr;
    double* YT = nullptr;              // coarse eigenvectors, transposed
    double* escratch = nullptr;
    double *W[2] = {nullptr, nullptr}, *KW[2] = {nullptr, nullptr}, *MW[2] = {nullptr, nullptr};
    double *F = nullptr, *Z = nullptr, *Zhat = nullptr, *G = nullptr, *Cw = nullptr;
    void *Floc = nullptr, *zloc = nullptr, *Lwork = nullptr;
    double *partial = nullptr, *colsq = nullptr, *lam = nullptr;
    double *gsmall = nullptr, *csmall = nullptr, *Hm = nullptr, *theta = nullptr, *Cfull = nullptr, *rrwork = nullptr;
    int *dropped[2] = {nullptr, nullptr}, *status = nullptr;   // per-buffer flags of W's columns
    int* negflag = nullptr;            // per (subdomain, shift): indefinite local matrix
    // W^{k+1} = W^k + span{t} (BPJD_SUBSPACE_GROW): the basis and M times it as n x s blocks
    // (block stride as W), the projected K (grow_cap x grow_cap) and the eigensolver's arrays
    int grow_cap = 0;                  // largest dimension of W (a multiple of s), 0 unless GROW
    double *Wg = nullptr, *MWg = nullptr, *Hg = nullptr, *Hw = nullptr, *Vg = nullptr, *thetag = nullptr;
    double *Cg = nullptr, *Qg = nullptr, *gwork = nullptr, *gsmall2 = nullptr, *gscratch = nullptr;
    int* dropg = nullptr;              // dropped (zero) columns of W
    double* hbuf = nullptr;            // pinned host mirror for per-iteration scalars
    int npart = 0;
    int nnzKH = 0;
    int maxPT = 0;                     // largest coarse basis support (entries of a row of P^T)
    int bwH = 0;                       // lower bandwidth of K_H, M_H (and of L)
    bool trace = false;
    std::vector<int> h_nl, h_bw;     // host copies of subdomain sizes / half-bandwidths
    bool setup_done = false;
    std::vector<bpjd::DevBlock> allocations;
    std::vector<void*> reserved;       // served problem: its blocks, placed in the server's block at admission
    std::vector<size_t> reserved_bytes;
    size_t reserved_next = 0;          // next reserved block to hand out
    bool own_hbuf = false;
    bpjd::HostPlan* plan = nullptr;    // host arrays between planning and materialisation
    hipGraphExec_t graph_exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [buffer][P in W]
    bool graph_failed = false;         // capture unavailable: launch directly
    bool tuned = false;                // launch shapes chosen (autotuner or fixed)
    int ldlt_threads = 256;            // threads per system of the windowed local solver
    int spmm_variant = 0;              // SpMM form: 0 two columns per lane where allowed, 1 one column
                                       // per lane (power-of-two group per row), 2 one lane per (row, column)
    size_t footprint = 0;              // device bytes of the problem (allocation granularity included)
};
