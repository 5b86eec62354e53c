// C ABI, structural setup on the host, and the outer iteration of Algorithm 3.1.
//
// Host work is limited to structure: validating the CSR input, the union
// pattern of K and M, subdomain dof sets, the local band layout, the coarse
// prolongation P for structured grids and the symbolic patterns of the
// Galerkin products.  Every numeric step of a solve (Galerkin coarse
// operators, the coarse eigenproblem, SpMM, residuals, the preconditioner,
// orthonormalisation, Rayleigh-Ritz) runs in the HIP kernels of this library.
#include <algorithm>
#include <fstream>
#include <map>
#include <mutex>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <numeric>
#include <climits>
#include <thread>

#include "common.h"

namespace bpjd {

static thread_local std::string g_last_error;
static thread_local bpjd_ctx* g_scope_ctx = nullptr;   // context of the ABI call in progress
static thread_local std::string g_error_copy;          // bpjd_last_error(ctx) storage

// largest dimension of a growing subspace W (its projected eigenproblem is dense)
static constexpr int kGrowMaxDim = 1024;

// largest half-bandwidth and lower entries per row handled by the blocked (MFMA) local solver
static constexpr int kBlockedMaxBand = 48;       // 64-row window (4 tile-rows)
static constexpr int kBlockedWideMaxBand = 80;   // 96-row window (6 tile-rows)
static constexpr int kBlockedMaxSlots = 8;
// the wide blocked solver (FP32, 192-row window): half-bandwidths 49..176, up to 20 lower
// entries per row (elements with several dofs per vertex, three dimensions)
static constexpr int kWideMinBand = 49;
static constexpr int kWideMaxBand = 176;
static constexpr int kWideMaxSlots = 20;

// Host planning runs its per-row, per-dof and per-subdomain loops on up to 16 threads.
// Every loop writes disjoint outputs, or per-item results merged in item order, so the
// plan does not depend on the number of threads.
static int planning_threads() {
    static const int nt = [] {
        const unsigned h = std::thread::hardware_concurrency();
        return (int)std::min(16u, std::max(1u, h));
    }();
    return nt;
}

// f(lo, hi, t) over [0, n) in contiguous chunks, chunk t on its own thread; small ranges
// stay on the calling thread.
template <class F>
static void parallel_chunks(long long n, F&& f, long long min_chunk = 8192) {
    const int nt = (int)std::min<long long>(planning_threads(), std::max<long long>(1, n / min_chunk));
    if (nt <= 1) {
        f(0LL, n, 0);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    for (int t = 1; t < nt; ++t) th.emplace_back([&f, n, nt, t] { f(n * t / nt, n * (t + 1) / nt, t); });
    f(0LL, n / nt, 0);
    for (auto& x : th) x.join();
}

// The lowest failing item over the chunks of a parallel check (INT_MAX: none).
struct FirstBad {
    std::vector<std::pair<int, int>> at = std::vector<std::pair<int, int>>(planning_threads(), {INT_MAX, 0});
    void set(int t, int item, int kind) {
        if (item < at[t].first) at[t] = {item, kind};
    }
    std::pair<int, int> get() const { return *std::min_element(at.begin(), at.end()); }
};

void set_error(const std::string& msg) {
    g_last_error = msg;
    if (bpjd_ctx* c = g_scope_ctx) {
        std::lock_guard<std::mutex> g(c->err_mu);
        c->last_error = msg;
    }
}

int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

CtxScope::CtxScope(bpjd_ctx* c) : prev(g_scope_ctx) { g_scope_ctx = c; }
CtxScope::~CtxScope() { g_scope_ctx = prev; }

// ---- device memory ----------------------------------------------------------------
// ---- trace: JSON lines ------------------------------------------------------------
// Enabled by the environment variable BPJD_TRACE, read when a problem is created (a
// problem keeps the setting it was created with): "1" or "stderr" writes to stderr, any
// other value names a file the lines are appended to.
static std::mutex g_trace_mu;
static FILE* g_trace_f = nullptr;
static std::string g_trace_target;    // value of BPJD_TRACE the stream was opened for

bool trace_on() {
    std::lock_guard<std::mutex> g(g_trace_mu);
    const char* v = std::getenv("BPJD_TRACE");
    const std::string target = v ? v : "";
    if (target != g_trace_target) {
        if (g_trace_f && g_trace_f != stderr) std::fclose(g_trace_f);
        g_trace_f = nullptr;
        g_trace_target = target;
        if (target == "1" || target == "stderr") g_trace_f = stderr;
        else if (!target.empty()) g_trace_f = std::fopen(target.c_str(), "a");
    }
    return g_trace_f != nullptr;
}

// Writes one line to the stream of the last trace_on() that found tracing on (a problem
// created while tracing keeps writing there, to stderr if the stream was closed since).
void trace_line(const std::string& json) {
    std::lock_guard<std::mutex> g(g_trace_mu);
    FILE* f = g_trace_f ? g_trace_f : stderr;
    std::fputs(json.c_str(), f);
    std::fputc('\n', f);
    std::fflush(f);
}

// Wall time of the host planning stages of one problem creation
struct StageClock {
    bool on = trace_on();
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    void mark(const char* stage) {
        if (!on) return;
        const auto now = std::chrono::steady_clock::now();
        char buf[160];
        std::snprintf(buf, sizeof buf, "{\"event\": \"create\", \"stage\": \"%s\", \"ms\": %.3f}", stage,
                      std::chrono::duration<double, std::milli>(now - t).count());
        trace_line(buf);
        t = now;
    }
};

static std::string json_doubles(const double* v, int count, const char* fmt = "%.15g") {
    std::string o = "[";
    char buf[40];
    for (int q = 0; q < count; ++q) {
        std::snprintf(buf, sizeof buf, fmt, v[q]);
        if (q) o += ", ";
        o += std::isfinite(v[q]) ? buf : "null";
    }
    return o + "]";
}

void* DevArena::alloc(size_t bytes) {
    const size_t b = round(bytes);
    std::lock_guard<std::mutex> g(mu);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < b) continue;
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > b) free_[off + b] = len - b;
        return base + off;
    }
    return nullptr;
}

void DevArena::release(void* ptr, size_t bytes) {
    const size_t b = round(bytes);
    size_t off = (size_t)((char*)ptr - base), len = b;
    std::lock_guard<std::mutex> g(mu);
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {                      // merge with the free block before
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            off = prev->first;
            len += prev->second;
            free_.erase(prev);
        }
    }
    if (next != free_.end() && off + len == next->first) {   // and the one after
        len += next->second;
        free_.erase(next);
    }
    free_[off] = len;
}

bool DevArena::alloc_all(const std::vector<size_t>& sizes, std::vector<void*>& out) {
    std::lock_guard<std::mutex> g(mu);
    std::map<size_t, size_t> f = free_;
    std::vector<void*> got;
    got.reserve(sizes.size());
    for (size_t bytes : sizes) {
        const size_t b = round(bytes);
        bool placed = false;
        for (auto it = f.begin(); it != f.end(); ++it) {
            if (it->second < b) continue;
            const size_t off = it->first, len = it->second;
            f.erase(it);
            if (len > b) f[off + b] = len - b;
            got.push_back(base + off);
            placed = true;
            break;
        }
        if (!placed) return false;
    }
    free_.swap(f);
    out.swap(got);
    return true;
}

// A device block for problem p: from the server's block (a served problem), the
// context's allocator, or hipMalloc.
static void* dev_alloc(bpjd_problem* p, size_t bytes, int* route) {
    bpjd_ctx* c = p->ctx;
    if (c->arena) {          // blocks reserved at admission, handed out in allocation order
        *route = 2;
        return p->reserved_next < p->reserved.size() ? p->reserved[p->reserved_next++] : nullptr;
    }
    if (c->alloc.alloc) {
        *route = 1;
        return c->alloc.alloc(bytes, c->alloc.user);
    }
    *route = 0;
    void* d = nullptr;
    return hipMalloc(&d, bytes) == hipSuccess ? d : nullptr;
}

static void dev_free(bpjd_problem* p, const DevBlock& b) {
    bpjd_ctx* c = p->ctx;
    if (b.route == 2) c->arena->release(b.ptr, b.bytes);
    else if (b.route == 1) c->alloc.free(b.ptr, c->alloc.user);
    else (void)hipFree(b.ptr);
}

struct HostCSR {
    int n = 0;
    fillvec<int> ptr, col;      // every element written by the copy in read_csr
    fillvec<double> val;
};

static int read_csr(const bpjd_csr* A, const char* name, HostCSR& out, hipStream_t st) {
    if (!A || !A->rowptr || !A->col || !A->val) return fail(BPJD_ERR_ARG, std::string(name) + ": NULL array");
    if (A->n_rows <= 0 || A->n_rows != A->n_cols) return fail(BPJD_ERR_CSR, std::string(name) + ": not square");
    const int n = A->n_rows;
    out.n = n;
    out.ptr.resize(n + 1);
    if (A->mem == BPJD_MEM_DEVICE) {
        BPJD_HIP(hipMemcpyAsync(out.ptr.data(), A->rowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, st));
        BPJD_HIP(hipStreamSynchronize(st));
    } else {
        std::memcpy(out.ptr.data(), A->rowptr, sizeof(int) * (n + 1));
    }
    if (out.ptr[0] != 0 || (long long)out.ptr[n] != A->nnz)
        return fail(BPJD_ERR_CSR, std::string(name) + ": rowptr[0] != 0 or rowptr[n] != nnz");
    for (int i = 0; i < n; ++i)
        if (out.ptr[i + 1] < out.ptr[i]) return fail(BPJD_ERR_CSR, std::string(name) + ": rowptr not monotone");
    out.col.resize(A->nnz);
    out.val.resize(A->nnz);
    if (A->mem == BPJD_MEM_DEVICE) {
        // touch the fresh pages on every planning thread first, so that the copy does not
        // take their first-use faults one by one
        parallel_chunks(A->nnz, [&](long long lo, long long hi, int) {
            for (long long q = lo; q < hi; q += 512) {
                out.col[q] = 0;
                out.val[q] = 0.0;
            }
        });
        BPJD_HIP(hipMemcpyAsync(out.col.data(), A->col, sizeof(int) * A->nnz, hipMemcpyDeviceToHost, st));
        BPJD_HIP(hipMemcpyAsync(out.val.data(), A->val, sizeof(double) * A->nnz, hipMemcpyDeviceToHost, st));
        BPJD_HIP(hipStreamSynchronize(st));
    } else {
        const int* cs = A->col;
        const double* vs = A->val;
        parallel_chunks(A->nnz, [&](long long lo, long long hi, int) {
            std::memcpy(out.col.data() + lo, cs + lo, sizeof(int) * (hi - lo));
            std::memcpy(out.val.data() + lo, vs + lo, sizeof(double) * (hi - lo));
        });
    }
    FirstBad bad;
    parallel_chunks(n, [&](long long lo, long long hi, int t) {
        for (int i = (int)lo; i < (int)hi; ++i) {
            for (int p = out.ptr[i]; p < out.ptr[i + 1]; ++p) {
                const int c = out.col[p];
                const int kind = (c < 0 || c >= n) ? 1 : (p > out.ptr[i] && c <= out.col[p - 1]) ? 2
                                                        : !std::isfinite(out.val[p]) ? 3 : 0;
                if (kind) {
                    bad.set(t, i, kind);
                    return;
                }
            }
        }
    });
    const int kind = bad.get().second;
    if (kind == 1) return fail(BPJD_ERR_CSR, std::string(name) + ": column index out of range");
    if (kind == 2) return fail(BPJD_ERR_CSR, std::string(name) + ": columns not strictly increasing in a row");
    if (kind == 3) return fail(BPJD_ERR_CSR, std::string(name) + ": non-finite value");
    return BPJD_OK;
}

// Union pattern of K and M with the position maps of both inputs.
struct Pattern {
    int n = 0;
    std::vector<int> ptr;
    fillvec<int> col;                 // every element written by build_union
    fillvec<long long> Kmap, Mmap;
};

// Row i of the union pattern: merge of the sorted columns of K and M; with emit, the
// columns go to out and the positions of K's and M's entries to Kmap / Mmap.
template <bool emit>
static int union_row(const HostCSR& K, const HostCSR& M, int i, int* out, long long pos, long long* Kmap,
                     long long* Mmap) {
    int a = K.ptr[i], b = M.ptr[i], cnt = 0;
    const int ae = K.ptr[i + 1], be = M.ptr[i + 1];
    while (a < ae || b < be) {
        const int c = (b >= be || (a < ae && K.col[a] < M.col[b])) ? K.col[a] : M.col[b];
        if (emit) {
            if (a < ae && K.col[a] == c) Kmap[a] = pos + cnt;
            if (b < be && M.col[b] == c) Mmap[b] = pos + cnt;
            out[cnt] = c;
        }
        if (a < ae && K.col[a] == c) ++a;
        if (b < be && M.col[b] == c) ++b;
        ++cnt;
    }
    return cnt;
}

static int build_union(const HostCSR& K, const HostCSR& M, Pattern& U) {
    const int n = K.n;
    U.n = n;
    U.ptr.assign(n + 1, 0);
    parallel_chunks(n, [&](long long lo, long long hi, int) {
        for (int i = (int)lo; i < (int)hi; ++i) U.ptr[i + 1] = union_row<false>(K, M, i, nullptr, 0, nullptr, nullptr);
    });
    for (int i = 0; i < n; ++i) U.ptr[i + 1] += U.ptr[i];
    U.col.resize(U.ptr[n]);
    U.Kmap.resize(K.col.size());
    U.Mmap.resize(M.col.size());
    parallel_chunks(n, [&](long long lo, long long hi, int) {
        for (int i = (int)lo; i < (int)hi; ++i)
            union_row<true>(K, M, i, U.col.data() + U.ptr[i], U.ptr[i], U.Kmap.data(), U.Mmap.data());
    });
    // structural symmetry of the union pattern
    FirstBad bad;
    parallel_chunks(n, [&](long long lo, long long hi, int t) {
        for (int i = (int)lo; i < (int)hi; ++i) {
            for (int p = U.ptr[i]; p < U.ptr[i + 1]; ++p) {
                const int j = U.col[p];
                if (!std::binary_search(U.col.begin() + U.ptr[j], U.col.begin() + U.ptr[j + 1], i)) {
                    bad.set(t, i, 1);
                    return;
                }
            }
        }
    });
    if (bad.get().second) return fail(BPJD_ERR_CSR, "pattern of K + M is not symmetric");
    return BPJD_OK;
}

// ---- structured P1 decomposition ----------------------------------------------
// Coarse P1 on the grid cx x cy, each coarse cell cut by its "/" diagonal;
// nodal interpolation at the dof coordinates (same rule as the fine mesh).  A
// coarse vertex carries a coarse basis function when a fine dof sits on it (on a
// rectangle every interior coarse vertex; on a domain with fixed inner edges, such
// as the L-shape, only the free ones), numbered row by row, x fastest.
static void build_p1_prolongation(int n, const double* xy, const std::vector<double>& cx,
                                  const std::vector<double>& cy, HostCSR& P, int& nH) {
    const int ncx = (int)cx.size() - 1, ncy = (int)cy.size() - 1;
    double hmin = 1e300;
    for (int i = 0; i < ncx; ++i) hmin = std::min(hmin, cx[i + 1] - cx[i]);
    for (int i = 0; i < ncy; ++i) hmin = std::min(hmin, cy[i + 1] - cy[i]);
    const double tol = 1e-9 * hmin;
    // free coarse vertices: a fine dof lies on the vertex
    std::vector<int> vnum((size_t)(ncx + 1) * (ncy + 1), -1);
    std::vector<char> hit((size_t)(ncx + 1) * (ncy + 1), 0);
    std::vector<int> onv(n, -1);      // interior coarse vertex a dof sits on, or -1
    parallel_chunks(n, [&](long long lo, long long hi, int) {
        for (int d = (int)lo; d < (int)hi; ++d) {
            const double x = xy[2 * d], y = xy[2 * d + 1];
            const int a = (int)(std::lower_bound(cx.begin(), cx.end(), x - tol) - cx.begin());
            const int b = (int)(std::lower_bound(cy.begin(), cy.end(), y - tol) - cy.begin());
            if (a >= 1 && a <= ncx - 1 && b >= 1 && b <= ncy - 1 && std::fabs(cx[a] - x) <= tol &&
                std::fabs(cy[b] - y) <= tol)
                onv[d] = b * (ncx + 1) + a;
        }
    });
    for (int d = 0; d < n; ++d)
        if (onv[d] >= 0) hit[onv[d]] = 1;
    nH = 0;
    for (int b = 1; b < ncy; ++b)
        for (int a = 1; a < ncx; ++a)
            if (hit[(size_t)b * (ncx + 1) + a]) vnum[(size_t)b * (ncx + 1) + a] = nH++;
    // at most three entries per dof (the vertices of its coarse triangle), sorted by
    // coarse index, then compacted
    std::vector<int> ecol((size_t)3 * n);
    std::vector<double> eval((size_t)3 * n);
    P.n = n;
    P.ptr.assign(n + 1, 0);
    parallel_chunks(n, [&](long long lo, long long hi, int) {
        for (int d = (int)lo; d < (int)hi; ++d) {
            const double x = xy[2 * d], y = xy[2 * d + 1];
            int a = (int)(std::upper_bound(cx.begin(), cx.end(), x) - cx.begin()) - 1;
            int b = (int)(std::upper_bound(cy.begin(), cy.end(), y) - cy.begin()) - 1;
            a = std::min(std::max(a, 0), ncx - 1);
            b = std::min(std::max(b, 0), ncy - 1);
            const double xi = (x - cx[a]) / (cx[a + 1] - cx[a]);
            const double eta = (y - cy[b]) / (cy[b + 1] - cy[b]);
            int va[3], vb[3];
            double w[3];
            if (xi >= eta) {
                va[0] = a; vb[0] = b; w[0] = 1.0 - xi;
                va[1] = a + 1; vb[1] = b; w[1] = xi - eta;
                va[2] = a + 1; vb[2] = b + 1; w[2] = eta;
            } else {
                va[0] = a; vb[0] = b; w[0] = 1.0 - eta;
                va[1] = a + 1; vb[1] = b + 1; w[1] = xi;
                va[2] = a; vb[2] = b + 1; w[2] = eta - xi;
            }
            std::pair<int, double> ent[3];
            int ne = 0;
            for (int k = 0; k < 3; ++k) {
                const int c = vnum[(size_t)vb[k] * (ncx + 1) + va[k]];
                if (c >= 0 && w[k] != 0.0) ent[ne++] = {c, w[k]};
            }
            std::sort(ent, ent + ne);
            for (int k = 0; k < ne; ++k) {
                ecol[(size_t)3 * d + k] = ent[k].first;
                eval[(size_t)3 * d + k] = ent[k].second;
            }
            P.ptr[d + 1] = ne;
        }
    });
    for (int d = 0; d < n; ++d) P.ptr[d + 1] += P.ptr[d];
    P.col.resize(P.ptr[n]);
    P.val.resize(P.ptr[n]);
    parallel_chunks(n, [&](long long lo, long long hi, int) {
        for (int d = (int)lo; d < (int)hi; ++d)
            for (int k = 0; k < P.ptr[d + 1] - P.ptr[d]; ++k) {
                P.col[P.ptr[d] + k] = ecol[(size_t)3 * d + k];
                P.val[P.ptr[d] + k] = eval[(size_t)3 * d + k];
            }
    });
}

// Subdomains: each closed coarse cell (cell_shape BPJD_CELL_SQUARE), or each of the
// two closed coarse triangles a cell is cut into by its "/" diagonal
// (BPJD_CELL_TRIANGLE, the lower-right one first), plus (layers - 1) graph layers of
// the union pattern.  Cells or triangles that hold no dof are skipped.
static int build_geom_subdomains(const Pattern& U, const double* xy, const std::vector<double>& cx,
                                 const std::vector<double>& cy, int layers, int shape, std::vector<int>& sptr,
                                 std::vector<int>& sidx) {
    if (layers < 1) return fail(BPJD_ERR_ARG, "overlap_layers must be >= 1");
    if (shape != BPJD_CELL_SQUARE && shape != BPJD_CELL_TRIANGLE) return fail(BPJD_ERR_ARG, "unknown cell_shape");
    const int n = U.n;
    const int ncx = (int)cx.size() - 1, ncy = (int)cy.size() - 1;
    const int parts = shape == BPJD_CELL_TRIANGLE ? 2 : 1;
    double hmin = 1e300;
    for (int i = 0; i < ncx; ++i) hmin = std::min(hmin, cx[i + 1] - cx[i]);
    for (int i = 0; i < ncy; ++i) hmin = std::min(hmin, cy[i + 1] - cy[i]);
    const double tol = 1e-9 * hmin;
    // closed-cell membership: each dof lies in at most two closed cells per axis
    std::vector<std::vector<int>> cell((size_t)ncx * ncy * parts);
    for (int d = 0; d < n; ++d) {
        const double x = xy[2 * d], y = xy[2 * d + 1];
        int a0 = (int)(std::upper_bound(cx.begin(), cx.end(), x) - cx.begin()) - 1;
        int b0 = (int)(std::upper_bound(cy.begin(), cy.end(), y) - cy.begin()) - 1;
        for (int B = std::max(0, b0 - 1); B <= std::min(ncy - 1, b0 + 1); ++B) {
            if (!(y >= cy[B] - tol && y <= cy[B + 1] + tol)) continue;
            for (int A = std::max(0, a0 - 1); A <= std::min(ncx - 1, a0 + 1); ++A) {
                if (!(x >= cx[A] - tol && x <= cx[A + 1] + tol)) continue;
                const size_t c = (size_t)B * ncx + A;
                if (parts == 1) {
                    cell[c].push_back(d);
                } else {
                    // side of the cell's diagonal: xi - eta >= 0 below it, <= 0 above it
                    const double dg = (x - cx[A]) / (cx[A + 1] - cx[A]) - (y - cy[B]) / (cy[B + 1] - cy[B]);
                    if (dg >= -1e-9) cell[2 * c].push_back(d);
                    if (dg <= 1e-9) cell[2 * c + 1].push_back(d);
                }
            }
        }
    }
    // each cell grows by (layers - 1) graph layers; cells in parallel, a mark array per thread
    const long long ncell = (long long)cell.size();
    std::vector<std::vector<int>> grown(ncell);
    std::vector<std::vector<int>> marks(planning_threads());
    parallel_chunks(ncell, [&](long long lo, long long hi, int t) {
        std::vector<int>& mark = marks[t];
        mark.assign(n, -1);
        std::vector<int> frontier, next;
        for (long long c = lo; c < hi; ++c) {
            std::vector<int> members = cell[c];
            for (int d : members) mark[d] = (int)c;
            frontier = members;
            for (int layer = 1; layer < layers; ++layer) {
                next.clear();
                for (int d : frontier) {
                    for (int q = U.ptr[d]; q < U.ptr[d + 1]; ++q) {
                        const int e = U.col[q];
                        if (mark[e] != (int)c) {
                            mark[e] = (int)c;
                            members.push_back(e);
                            next.push_back(e);
                        }
                    }
                }
                frontier.swap(next);
            }
            std::sort(members.begin(), members.end());
            grown[c].swap(members);
        }
    }, 1);
    sptr.assign(1, 0);
    sidx.clear();
    for (long long c = 0; c < ncell; ++c) {
        if (grown[c].empty()) continue;
        sidx.insert(sidx.end(), grown[c].begin(), grown[c].end());
        sptr.push_back((int)sidx.size());
    }
    return BPJD_OK;
}

static int upload(bpjd_problem* p, void** dst, const void* src, size_t bytes) {
    if (bytes == 0) bytes = 8;
    int route = 0;
    void* d = dev_alloc(p, bytes, &route);
    if (!d) {
        (void)hipGetLastError();
        return fail(BPJD_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    p->allocations.push_back(DevBlock{d, bytes, route});
    // on the problem's own stream (never the legacy stream, which would wait for, or be
    // refused by, another stream's capture); materialize_problem synchronises it
    if (src) BPJD_HIP(hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, p->ctx->stream));
    *dst = d;
    return BPJD_OK;
}

template <typename T>
static int upload_vec(bpjd_problem* p, T** dst, const std::vector<T>& v) {
    return upload(p, (void**)dst, v.empty() ? nullptr : v.data(), v.size() * sizeof(T));
}

template <typename T>
static int alloc_dev(bpjd_problem* p, T** dst, size_t count) {
    return upload(p, (void**)dst, nullptr, count * sizeof(T));
}

// Host-side result of planning a problem: every array the device copy needs.
struct HostPlan {
    std::vector<int> rowptr;
    fillvec<int> col;
    fillvec<double2> km;        // every element written when the plan is made
    fillvec<int> Pptr, Pcol;
    fillvec<double> Pval;
    std::vector<int> PTptr, PTcol;
    std::vector<double> PTval;
    std::vector<int> kpptr, kpcol, khptr, khcol;
    std::vector<int> sptr, sidx, bw, lptr, ldd, lpos, rptr, ridx;
    std::vector<long long> Loff;
    std::vector<int> sysord;    // launch order of the (subdomain, shift) systems
    bool blocked = false;
    int maxE = 0, bws = 64;
    long long Ltot = 0;
    size_t elt = 8;
};

// Distance in doubles between consecutive n x s blocks of W, K W and M W: n s rounded
// up to even, so that every block starts on a 16-byte boundary.
static inline long long block_stride(int n, int s) { return ((long long)n * s + 1) & ~1LL; }

// The one list of device arrays of a problem.  `op(dst, src, bytes)` either allocates
// (and uploads src when non-NULL) or only counts bytes, so the footprint used for
// admission and the real allocation cannot drift apart.
template <class Op>
static int device_layout(bpjd_problem* p, const HostPlan& h, Op&& op) {
    int rc = BPJD_OK;
    auto put = [&](auto** dst, const auto& v) {
        using E = typename std::decay_t<decltype(v)>::value_type;
        int r = op((void**)dst, v.empty() ? nullptr : (const void*)v.data(), v.size() * sizeof(E));
        if (r < 0 && rc == BPJD_OK) rc = r;
    };
    auto zero = [&](auto** dst, size_t count) {
        using E = std::remove_pointer_t<std::remove_pointer_t<decltype(dst)>>;
        int r = op((void**)dst, nullptr, count * sizeof(E));
        if (r < 0 && rc == BPJD_OK) rc = r;
    };
    const int n = p->n, nH = p->nH, s = p->s;
    put(&p->rowptr, h.rowptr);
    put(&p->col, h.col);
    put(&p->km, h.km);
    put(&p->Pptr, h.Pptr);
    put(&p->Pcol, h.Pcol);
    put(&p->Pval, h.Pval);
    put(&p->PTptr, h.PTptr);
    put(&p->PTcol, h.PTcol);
    put(&p->PTval, h.PTval);
    put(&p->kpptr, h.kpptr);
    put(&p->kpcol, h.kpcol);
    zero(&p->kpval, h.kpcol.size());
    put(&p->khptr, h.khptr);
    put(&p->khcol, h.khcol);
    put(&p->subptr, h.sptr);
    put(&p->subidx, h.sidx);
    put(&p->bw, h.bw);
    put(&p->lptr, h.lptr);
    put(&p->ldd, h.ldd);
    put(&p->lpos, h.lpos);
    put(&p->rptr, h.rptr);
    put(&p->ridx, h.ridx);
    put(&p->Loff, h.Loff);
    put(&p->sysord, h.sysord);
    zero(&p->sd, (size_t)p->sumN * h.maxE);
    zero(&p->sv, (size_t)p->sumN * h.maxE);
    const size_t nH2 = (size_t)nH * nH;
    zero(&p->KH, nH2);
    zero(&p->MH, nH2);
    zero(&p->Y, nH2);
    zero(&p->jwork, nH2);
    zero(&p->lamH, nH);
    zero(&p->esmall, 6 * (size_t)nH + 1);
    zero(&p->YT, nH2);
    zero(&p->escratch, 8 * nH2);
    const size_t blk = 3 * (size_t)block_stride(n, s);
    for (int b = 0; b < 2; ++b) {
        zero(&p->W[b], blk);
        zero(&p->KW[b], blk);
        zero(&p->MW[b], blk);
    }
    zero(&p->F, (size_t)n * s);
    zero(&p->Z, (size_t)n * s);
    zero(&p->Zhat, (size_t)nH * s);
    zero(&p->G, (size_t)nH * s);
    zero(&p->Cw, (size_t)nH * s);
    {
        int r = op(&p->Floc, nullptr, h.elt * s * p->sumN);
        if (r < 0 && rc == BPJD_OK) rc = r;
        r = op(&p->zloc, nullptr, h.elt * s * p->sumN);
        if (r < 0 && rc == BPJD_OK) rc = r;
        r = op(&p->Lwork, nullptr, h.elt * h.Ltot);
        if (r < 0 && rc == BPJD_OK) rc = r;
    }
    zero(&p->partial, (size_t)p->npart * 4096);
    zero(&p->colsq, 256);     // [0, 2s) column norms, [128, 128+s) shifts, [192] status
    zero(&p->lam, 64);
    zero(&p->gsmall, 64 * 64);
    zero(&p->csmall, 64 * 64);
    zero(&p->Hm, 64 * 64);
    zero(&p->theta, 64);
    zero(&p->Cfull, 64 * 128);
    zero(&p->dropped[0], 64);
    zero(&p->dropped[1], 64);
    zero(&p->status, 4);
    zero(&p->negflag, (size_t)p->nsub * s);
    {
        const size_t gc = (size_t)p->grow_cap;
        const size_t gb = gc ? (size_t)(gc / s) * block_stride(n, s) : 0;
        zero(&p->Wg, gb);
        zero(&p->MWg, gb);
        zero(&p->Hg, gc * gc);
        zero(&p->Hw, gc * gc);
        zero(&p->Vg, gc * gc);
        zero(&p->thetag, gc);
        zero(&p->Cg, gc * s);
        zero(&p->Qg, gc * s);
        zero(&p->gwork, gc * gc);
        zero(&p->gsmall2, 6 * gc + 1);
        zero(&p->gscratch, 6 * gc * gc);
        zero(&p->dropg, gc);
    }
    return rc;
}

// Everything after the decomposition is known: local band layout, reverse
// map, Galerkin patterns.  Builds the problem's host plan and its device
// footprint; materialize_problem allocates and uploads.
// K, M, U and P are consumed (their arrays move into the plan).
static int finish_create(bpjd_ctx* ctx, HostCSR& K, HostCSR& M, Pattern& U, HostCSR& P,
                         int nH, std::vector<int>& sptr, std::vector<int>& sidx, const bpjd_opts* opts,
                         bpjd_problem** out, StageClock& clk) {
    const int n = U.n;
    const int nsub = (int)sptr.size() - 1;
    if (nsub < 1) return fail(BPJD_ERR_DD, "no subdomains");
    const int s = opts->k + opts->guard;
    if (opts->k < 1 || opts->guard < 0 || s > BPJD_MAX_BLOCK)
        return fail(BPJD_ERR_ARG, "need 1 <= k and k + guard <= " + std::to_string(BPJD_MAX_BLOCK));
    if (s >= nH) return fail(BPJD_ERR_DD, "block size s must be smaller than dim V^H");
    if (nH > 1024) return fail(BPJD_ERR_DD, "coarse space larger than 1024 is not supported");
    if (opts->n_init != 0 && opts->n_init != s) return fail(BPJD_ERR_ARG, "n_init must be 0 or k + guard");
    if (opts->n_init && !opts->X_init) return fail(BPJD_ERR_ARG, "X_init is NULL");
    if (opts->stop_rule != BPJD_STOP_RESIDUAL && opts->stop_rule != BPJD_STOP_PAPER)
        return fail(BPJD_ERR_ARG, "unknown stop rule");
    if (opts->subspace != BPJD_SUBSPACE_UU && opts->subspace != BPJD_SUBSPACE_U &&
        opts->subspace != BPJD_SUBSPACE_GROW)
        return fail(BPJD_ERR_ARG, "unknown subspace choice");
    if (opts->precision != BPJD_PREC_FP64 && opts->precision != BPJD_PREC_MIXED)
        return fail(BPJD_ERR_ARG, "unknown precision");
    if (opts->profile < 0 || opts->profile > 2) return fail(BPJD_ERR_ARG, "profile must be 0, 1 or 2");
    if (opts->local_threads != 0 && opts->local_threads != 64 && opts->local_threads != 128 &&
        opts->local_threads != 256)
        return fail(BPJD_ERR_ARG, "local_threads must be 0, 64, 128 or 256");
    if (opts->spmm_form < 0 || opts->spmm_form > BPJD_SPMM_FLAT)
        return fail(BPJD_ERR_ARG, "spmm_form must be 0 or one of BPJD_SPMM_*");
    if (!(opts->tol > 0.0) || opts->max_iter < 0) return fail(BPJD_ERR_ARG, "bad tol or max_iter");

    // coverage and local orderings (ascending global index); subdomains in parallel
    {
        FirstBad bad;
        parallel_chunks(nsub, [&](long long lo, long long hi, int t) {
            for (int l = (int)lo; l < (int)hi; ++l) {
                if (sptr[l + 1] <= sptr[l]) {
                    bad.set(t, l, 1);
                    return;
                }
                std::sort(sidx.begin() + sptr[l], sidx.begin() + sptr[l + 1]);
                for (int q = sptr[l]; q < sptr[l + 1]; ++q) {
                    const int kind = (sidx[q] < 0 || sidx[q] >= n) ? 2 : (q > sptr[l] && sidx[q] == sidx[q - 1]) ? 3 : 0;
                    if (kind) {
                        bad.set(t, l, kind);
                        return;
                    }
                }
            }
        }, 16);
        const int kind = bad.get().second;
        if (kind == 1) return fail(BPJD_ERR_DD, "empty subdomain");
        if (kind == 2) return fail(BPJD_ERR_DD, "subdomain index out of range");
        if (kind == 3) return fail(BPJD_ERR_DD, "duplicate dof in a subdomain");
    }
    std::vector<int> cover(n, 0);
    for (int q = 0; q < sptr[nsub]; ++q) cover[sidx[q]] = 1;
    for (int d = 0; d < n; ++d)
        if (!cover[d]) return fail(BPJD_ERR_DD, "dof " + std::to_string(d) + " lies in no subdomain");
    clk.mark("cover");

    // lower band entries of every local row (band offset and position in the union
    // pattern): counted, then written, subdomains in parallel with a local-index map per
    // thread
    const long long sumN = sptr[nsub];
    std::vector<int> lptr(sumN + 1, 0), ldd, lpos, bw(nsub, 0);
    std::vector<std::vector<int>> gls(planning_threads());
    auto band_pass = [&](const bool write) {
        parallel_chunks(nsub, [&](long long lo, long long hi, int t) {
            std::vector<int>& gl = gls[t];
            if ((int)gl.size() != n) gl.assign(n, -1);
            for (int l = (int)lo; l < (int)hi; ++l) {
                const int off = sptr[l], nl = sptr[l + 1] - off;
                for (int r = 0; r < nl; ++r) gl[sidx[off + r]] = r;
                for (int r = 0; r < nl; ++r) {
                    const int g = sidx[off + r];
                    int cnt = 0;
                    for (int p = U.ptr[g]; p < U.ptr[g + 1]; ++p) {
                        const int c = gl[U.col[p]];
                        if (c >= 0 && c <= r) {
                            if (write) {
                                ldd[lptr[off + r] + cnt] = r - c;
                                lpos[lptr[off + r] + cnt] = p;
                            } else {
                                bw[l] = std::max(bw[l], r - c);
                            }
                            ++cnt;
                        }
                    }
                    if (!write) lptr[off + r + 1] = cnt;
                }
                for (int r = 0; r < nl; ++r) gl[sidx[off + r]] = -1;
            }
        }, 16);
    };
    band_pass(false);
    for (long long q = 0; q < sumN; ++q) lptr[q + 1] += lptr[q];
    ldd.resize(lptr[sumN]);
    lpos.resize(lptr[sumN]);
    band_pass(true);
    int maxN = 0, maxBW = 0;
    for (int l = 0; l < nsub; ++l) {
        maxN = std::max(maxN, sptr[l + 1] - sptr[l]);
        maxBW = std::max(maxBW, bw[l]);
    }
    clk.mark("local_band");
    hipDeviceProp_t prop;
    BPJD_HIP(hipGetDeviceProperties(&prop, ctx->device));
    const size_t elt = opts->precision == BPJD_PREC_MIXED ? sizeof(float) : sizeof(double);
    const int maxC = maxBW + 1;
    const size_t shmem = (size_t)(maxC * maxC + 2 * maxC) * elt;
    if (shmem > prop.sharedMemPerBlock)
        return fail(BPJD_ERR_DD, "local half-bandwidth " + std::to_string(maxBW) + " too wide for the local solver");

    // reverse map dof -> positions in subdomain order
    std::vector<int> rptr(n + 1, 0), ridx(sumN);
    for (long long q = 0; q < sumN; ++q) rptr[sidx[q] + 1]++;
    for (int d = 0; d < n; ++d) rptr[d + 1] += rptr[d];
    {
        std::vector<int> fillp(rptr.begin(), rptr.end() - 1);
        for (long long q = 0; q < sumN; ++q) ridx[fillp[sidx[q]]++] = (int)q;
    }
    // factor storage per (subdomain, shift): the blocked solver keeps, per 16-column
    // panel, the band part of each column (bws rows from the diagonal down), the windowed
    // solver one band column per row
    int maxE = 0;
    for (long long q = 0; q < sumN; ++q) maxE = std::max(maxE, lptr[q + 1] - lptr[q]);
    const bool narrow = maxBW <= kBlockedWideMaxBand && maxE <= kBlockedMaxSlots;
    // the wide solver where the windowed one would run (mixed precision only: the
    // window's tiles are FP32), unless the caller fixed the windowed solver's threads
    const bool wide = !narrow && opts->precision == BPJD_PREC_MIXED && opts->local_threads == 0 &&
                      maxBW >= kWideMinBand && maxBW <= kWideMaxBand && maxE <= kWideMaxSlots;
    const bool blocked = narrow || wide;
    const int nt = wide ? 12 : !blocked ? 0 : (maxBW <= kBlockedMaxBand ? 4 : 6);   // window tile-rows
    // the windowed solver gives each lane at most three entries of a window row and loads
    // the slots of a block of rows one slot per lane
    if (!blocked && (maxBW > 191 || maxE > 64))
        return fail(BPJD_ERR_DD, "local half-bandwidth above 191 or more than 64 lower entries in a local row");
    // stored rows per factor column: the band part (rounded up to 4; the factor traffic
    // bounds the backward sweep), except FP32 with the 96- and 192-row windows, which keep
    // full columns
    const int win = 16 * std::max(nt, 4);
    const int bws = (opts->precision == BPJD_PREC_MIXED && (nt == 6 || nt == 12))
                        ? win
                        : ((std::min(win, maxBW + 1) + 3) / 4) * 4;
    std::vector<long long> Loff(nsub, 0);
    long long Ltot = 0;
    for (int l = 0; l < nsub; ++l) {
        Loff[l] = Ltot;
        const long long nl = sptr[l + 1] - sptr[l];
        Ltot += blocked ? (long long)s * ((nl + 15) / 16) * 16 * bws : (long long)s * nl * (bw[l] + 1);
    }
    // the local solvers take system sysord[b] in workgroup b: larger subdomains first, so
    // the last systems to start, which run while the device empties, are the smallest
    std::vector<int> sysord((size_t)nsub * s);
    {
        std::vector<int> byl(nsub);
        std::iota(byl.begin(), byl.end(), 0);
        std::stable_sort(byl.begin(), byl.end(),
                         [&](int x, int y) { return sptr[x + 1] - sptr[x] > sptr[y + 1] - sptr[y]; });
        for (int q = 0; q < nsub; ++q)
            for (int i = 0; i < s; ++i) sysord[(size_t)q * s + i] = byl[q] * s + i;
    }

    clk.mark("reverse_map");
    // P^T and Galerkin patterns
    std::vector<int> PTptr(nH + 1, 0), PTcol(P.col.size());
    std::vector<double> PTval(P.col.size());
    for (int c : P.col) {
        if (c < 0 || c >= nH) return fail(BPJD_ERR_DD, "P column index out of range");
        PTptr[c + 1]++;
    }
    for (int a = 0; a < nH; ++a) PTptr[a + 1] += PTptr[a];
    {
        std::vector<int> fillp(PTptr.begin(), PTptr.end() - 1);
        for (int d = 0; d < n; ++d)
            for (int q = P.ptr[d]; q < P.ptr[d + 1]; ++q) {
                const int e = fillp[P.col[q]]++;
                PTcol[e] = d;
                PTval[e] = P.val[q];
            }
    }
    for (int a = 0; a < nH; ++a)
        if (PTptr[a + 1] == PTptr[a]) return fail(BPJD_ERR_DD, "coarse basis function with empty support");
    // patterns of K P (n x n_H) and of K_H = P^T K P: the distinct columns of each row
    // are collected with a last-seen marker per coarse dof (a marker array per thread),
    // counted in one pass and written sorted in a second
    // (a row of K P has a few dozen; gathering and sorting all the repeats was the bulk of
    // the host planning for elements with many dofs per vertex)
    std::vector<std::vector<int>> marks(planning_threads());
    auto sparse_product_pattern = [&](const int rows, auto&& row_cols, std::vector<int>& ptr, std::vector<int>& cols) {
        ptr.assign(rows + 1, 0);
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1) {
                for (int i = 0; i < rows; ++i) ptr[i + 1] += ptr[i];
                cols.resize(ptr[rows]);
            }
            parallel_chunks(rows, [&](long long lo, long long hi, int t) {
                std::vector<int>& mark = marks[t];
                mark.assign(nH, -1);
                std::vector<int> tmp;
                for (int i = (int)lo; i < (int)hi; ++i) {
                    tmp.clear();
                    row_cols(i, [&](const int c) {
                        if (mark[c] != i) {
                            mark[c] = i;
                            tmp.push_back(c);
                        }
                    });
                    if (pass == 0) {
                        ptr[i + 1] = (int)tmp.size();
                    } else {
                        std::sort(tmp.begin(), tmp.end());
                        std::copy(tmp.begin(), tmp.end(), cols.begin() + ptr[i]);
                    }
                }
            }, 256);
        }
    };
    std::vector<int> kpptr, kpcol, khptr, khcol;
    sparse_product_pattern(n, [&](const int i, auto&& add) {
        for (int q = U.ptr[i]; q < U.ptr[i + 1]; ++q) {
            const int j = U.col[q];
            for (int r = P.ptr[j]; r < P.ptr[j + 1]; ++r) add(P.col[r]);
        }
    }, kpptr, kpcol);
    sparse_product_pattern(nH, [&](const int a, auto&& add) {
        for (int q = PTptr[a]; q < PTptr[a + 1]; ++q) {
            const int i = PTcol[q];
            for (int t = kpptr[i]; t < kpptr[i + 1]; ++t) add(kpcol[t]);
        }
    }, khptr, khcol);

    clk.mark("galerkin_pattern");
    bpjd_problem* p = new bpjd_problem();
    p->ctx = ctx;
    p->opts = *opts;
    p->opts.X_init = nullptr;
    p->n = n;
    p->nH = nH;
    p->nsub = nsub;
    p->s = s;
    p->k = opts->k;
    p->nnz = (long long)U.col.size();
    p->sumN = sumN;
    p->maxN = maxN;
    p->maxBW = maxBW;
    p->maxC = maxC;
    p->nnzK = (long long)K.col.size();
    p->nnzM = (long long)M.col.size();
    p->n_init = opts->n_init;
    p->nnzKH = (int)khcol.size();
    for (int a2 = 0; a2 < nH; ++a2) p->maxPT = std::max(p->maxPT, PTptr[a2 + 1] - PTptr[a2]);
    p->bwH = 0;                                    // lower bandwidth of the coarse matrices
    for (int a = 0; a < nH; ++a)
        for (int q = khptr[a]; q < khptr[a + 1]; ++q) p->bwH = std::max(p->bwH, a - khcol[q]);
    p->trace = trace_on();
    if (opts->local_threads) p->ldlt_threads = opts->local_threads;
    if (opts->spmm_form) p->spmm_variant = opts->spmm_form - 1;
    p->h_bw = bw;
    p->h_nl.resize(nsub);
    for (int l = 0; l < nsub; ++l) p->h_nl[l] = sptr[l + 1] - sptr[l];
    if (opts->n_init) p->X_init.assign(opts->X_init, opts->X_init + (size_t)n * s);

    auto* h = new HostPlan();
    p->plan = h;
    h->km.resize(p->nnz);
    parallel_chunks(n, [&](long long lo, long long hi, int) {   // rows of the union pattern
        for (long long q = U.ptr[lo]; q < U.ptr[hi]; ++q) h->km[q] = make_double2(0.0, 0.0);
        for (long long q = K.ptr[lo]; q < K.ptr[hi]; ++q) h->km[U.Kmap[q]].x = K.val[q];
        for (long long q = M.ptr[lo]; q < M.ptr[hi]; ++q) h->km[U.Mmap[q]].y = M.val[q];
    });
    p->Kmap = std::move(U.Kmap);
    p->Mmap = std::move(U.Mmap);
    h->rowptr = std::move(U.ptr);
    h->col = std::move(U.col);
    h->Pptr = std::move(P.ptr);
    h->Pcol = std::move(P.col);
    h->Pval = std::move(P.val);
    h->PTptr = std::move(PTptr);
    h->PTcol = std::move(PTcol);
    h->PTval = std::move(PTval);
    h->kpptr = std::move(kpptr);
    h->kpcol = std::move(kpcol);
    h->khptr = std::move(khptr);
    h->khcol = std::move(khcol);
    h->sptr = std::move(sptr);
    h->sidx = std::move(sidx);
    h->bw = std::move(bw);
    h->lptr = std::move(lptr);
    h->ldd = std::move(ldd);
    h->lpos = std::move(lpos);
    h->rptr = std::move(rptr);
    h->ridx = std::move(ridx);
    h->Loff = std::move(Loff);
    h->sysord = std::move(sysord);
    h->blocked = blocked;
    h->maxE = maxE;
    h->bws = bws;
    h->Ltot = Ltot;
    h->elt = elt;
    p->slotE = maxE;
    p->blocked = blocked;
    p->mfma_nt = nt;
    if (blocked) p->bws = bws;
    p->npart = num_partials(n);
    if (opts->subspace == BPJD_SUBSPACE_GROW)   // dim W <= 1024 (the dense eigensolver's reach)
        p->grow_cap = s * std::max(2, std::min(kGrowMaxDim / s, opts->max_iter + 1));
    size_t bytes = 0;
    device_layout(p, *h, [&](void**, const void*, size_t b) {
        bytes += (std::max<size_t>(b, 8) + 4095) & ~size_t(4095);   // allocation granularity
        return BPJD_OK;
    });
    p->footprint = bytes;
    clk.mark("host_plan");
    *out = p;
    return BPJD_OK;
}

// Allocate the device memory of a planned problem and upload its structural data
// (synchronous copies); releases the host plan.  On failure the problem keeps what
// was allocated, for bpjd_problem_destroy.
int materialize_problem(bpjd_problem* p) {
    if (!p->plan) return fail(BPJD_ERR_STATE, "problem already materialised");
    StageClock clk;
    BPJD_HIP(hipSetDevice(p->ctx->device));
    int rc = device_layout(p, *p->plan, [&](void** dst, const void* src, size_t b) {
        return upload(p, dst, src, b);
    });
    // the plan's host arrays are the sources of the copies just enqueued
    if (hipStreamSynchronize(p->ctx->stream) != hipSuccess && rc == BPJD_OK)
        rc = fail(BPJD_ERR_HIP, "upload of the problem's structure failed");
    if (rc == BPJD_OK) {
        if (p->ctx->hbuf) {
            p->hbuf = p->ctx->hbuf;           // a server slot's read-back buffer
        } else if (hipHostMalloc((void**)&p->hbuf, 4096 * sizeof(double)) != hipSuccess) {
            p->hbuf = nullptr;
            rc = fail(BPJD_ERR_OOM, "pinned host allocation failed");
        } else {
            p->own_hbuf = true;
        }
    }
    delete p->plan;
    p->plan = nullptr;
    clk.mark("allocate_upload");
    return rc;
}

// Sizes of the device blocks a planned problem will allocate, in allocation order.
std::vector<size_t> planned_blocks(bpjd_problem* p) {
    std::vector<size_t> out;
    if (!p->plan) return out;
    device_layout(p, *p->plan, [&](void**, const void*, size_t b) {
        out.push_back(b ? b : 8);
        return BPJD_OK;
    });
    return out;
}

static int read_pair(const bpjd_csr* K, const bpjd_csr* M, HostCSR& hK, HostCSR& hM, Pattern& U, hipStream_t st,
                     StageClock* clk) {
    BPJD_TRY(read_csr(K, "K", hK, st));
    BPJD_TRY(read_csr(M, "M", hM, st));
    if (hK.n != hM.n) return fail(BPJD_ERR_CSR, "K and M differ in size");
    clk->mark("read_csr");
    BPJD_TRY(build_union(hK, hM, U));
    clk->mark("union_pattern");
    return BPJD_OK;
}

// ---- numeric pieces ------------------------------------------------------------
// The blocks W = [X | P | T], K W and M W are stored as consecutive row-major n x s
// blocks (column c of W lies in block c / s), so a kernel that touches one block reads
// and writes whole rows of it.
static inline double* blkp(const bpjd_problem* p, double* base, int c) {
    return base + (size_t)(c / p->s) * block_stride(p->n, p->s);
}
static inline BlockGeom wgeom(const bpjd_problem* p) { return BlockGeom{p->s, p->s, block_stride(p->n, p->s)}; }

// HIP-event timing of solve phases (bpjd_opts.profile).  Events come from a
// pool; elapsed times are collected at the host synchronisation point of
// every outer iteration.
struct PhaseTimer {
    hipStream_t st = nullptr;
    unsigned mask = ~0u;           // phases that are timed
    std::vector<hipEvent_t> ev;
    std::vector<int> phase;
    size_t used = 0;
    double ms[BPJD_NUM_PHASES] = {0};
    int count[BPJD_NUM_PHASES] = {0};
    int open = -1;
    ~PhaseTimer() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    void begin(int ph) {
        if (!(mask & (1u << ph))) return;
        if (used + 2 > ev.size()) {
            for (int i = 0; i < 32; ++i) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                ev.push_back(e);
            }
            phase.resize(ev.size() / 2);
        }
        (void)hipEventRecord(ev[used], st);
        phase[used / 2] = ph;
        open = ph;
    }
    void end() {
        if (open < 0) return;
        (void)hipEventRecord(ev[used + 1], st);
        used += 2;
        open = -1;
    }
    void collect() {   // call after the stream has been synchronised
        for (size_t i = 0; i < used; i += 2) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) == hipSuccess) {
                ms[phase[i / 2]] += t;
                count[phase[i / 2]] += 1;
            }
        }
        used = 0;
    }
};

#define PH_BEGIN(T, ph) do { if (T) (T)->begin(ph); } while (0)
#define PH_END(T) do { if (T) (T)->end(); } while (0)

static int check_status(bpjd_problem* p) {
    int st = 0;
    BPJD_HIP(hipMemcpyAsync(&st, p->status, sizeof(int), hipMemcpyDeviceToHost, p->ctx->stream));
    BPJD_HIP(hipStreamSynchronize(p->ctx->stream));
    if (st & STATUS_COARSE_NOT_SPD) return fail(BPJD_ERR_NOT_SPD, "coarse mass matrix M_H is not positive definite");
    if (st & STATUS_LOCAL_PIVOT) return fail(BPJD_ERR_NOT_SPD, "singular pivot in a local factorisation");
    return BPJD_OK;
}

// Galerkin coarse operators and the full coarse generalized eigenproblem
// K_H y = lambda^H M_H y, Y^T M_H Y = I (Cholesky M_H = L L^T, symmetric
// eigensolver on L^{-1} K_H L^{-T}, Y = L^{-T} V).
static void coarse_setup(bpjd_problem* p) {
    hipStream_t st = p->ctx->stream;
    const int nH = p->nH;
    launch_extract_local(st, p->sumN, p->slotE, p->lptr, p->ldd, p->lpos, p->km, p->sd, p->sv);
    launch_galerkin(st, p->n, nH, p->rowptr, p->col, p->km, p->Pptr, p->Pcol, p->Pval, p->PTptr, p->PTcol, p->PTval,
                    p->kpptr, p->kpcol, p->kpval, p->khptr, p->khcol, p->nnzKH, p->KH, p->MH);
    // K_H y = lambda M_H y  ->  C z = lambda z with C = L^{-1} K_H L^{-T}, y = L^{-T} z;
    // L keeps the band of M_H, so the reductions are banded triangular solves
    const size_t nH2 = (size_t)nH * nH;
    double* E0 = p->escratch;                  // L^{-1} K_H, then the eigenvectors z
    double* E1 = p->escratch + nH2;            // Householder reflectors
    double* E2 = p->escratch + 2 * nH2;        // inverse-iteration scratch (6 nH^2)
    const int bw = p->bwH;
    launch_cholesky(st, nH, bw, p->MH, p->status, STATUS_COARSE_NOT_SPD);          // MH <- L
    launch_copy_cols(st, nH, nH, p->KH, nH, E0, nH);
    launch_trsm_band(st, nH, bw, nH, p->MH, E0, nH, false);                       // L^{-1} K_H
    launch_transpose(st, nH, E0, p->jwork);                                       // K_H L^{-T}
    launch_trsm_band(st, nH, bw, nH, p->MH, p->jwork, nH, false);                 // L^{-1} K_H L^{-T}
    launch_sym_eig(st, nH, p->jwork, p->lamH, E0, E1, p->esmall, E2, p->status);   // z
    launch_copy_cols(st, nH, nH, E0, nH, p->Y, nH);
    launch_trsm_band(st, nH, bw, nH, p->MH, p->Y, nH, true);                      // Y = L^{-T} Z
    launch_transpose(st, nH, p->Y, p->YT);
}

// Apply the two-level preconditioner to F (n x s, ld s) with shifts p->lam; Z (ld ldz).
static void apply_precond(bpjd_problem* p, const double* F, double* Z, int ldz, PhaseTimer* T) {
    hipStream_t st = p->ctx->stream;
    const int s = p->s;
    PH_BEGIN(T, BPJD_PHASE_COARSE);
    launch_coarse_apply(st, p->n, p->nH, s, p->PTptr, p->PTcol, p->PTval, F, s, p->Y, p->YT, p->lamH, p->lam, p->G,
                        p->Cw, p->Zhat, p->maxPT, p->partial, (long long)p->npart * 4096);
    PH_END(T);
    const bool mixed = p->opts.precision == BPJD_PREC_MIXED;
    PH_BEGIN(T, BPJD_PHASE_GATHER);
    if (mixed) launch_gather_f32(st, (int)p->sumN, s, p->subidx, F, s, (float*)p->Floc);
    else launch_gather_f64(st, (int)p->sumN, s, p->subidx, F, s, (double*)p->Floc);
    PH_END(T);
    // mode 0 (timed as the local phase), then mode 1: the systems found indefinite again
    // with shift 0 (a launch whose waves return at once when there are none)
    for (int mode = 0; mode < 2; ++mode) {
        if (mode == 0) PH_BEGIN(T, BPJD_PHASE_LOCAL);
        if (mixed)
            launch_local_solve_f32(st, mode, p->nsub, s, p->maxC, p->sumN, p->subptr, p->bw, p->mfma_nt,
                                   p->slotE, p->bws, p->sd, p->sv, p->lam, (const float*)p->Floc, (float*)p->zloc,
                                   (float*)p->Lwork, p->Loff, p->sysord, p->status, p->negflag, p->ldlt_threads);
        else
            launch_local_solve_f64(st, mode, p->nsub, s, p->maxC, p->sumN, p->subptr, p->bw, p->mfma_nt,
                                   p->slotE, p->bws, p->sd, p->sv, p->lam, (const double*)p->Floc,
                                   (double*)p->zloc, (double*)p->Lwork, p->Loff, p->sysord, p->status, p->negflag,
                                   p->ldlt_threads);
        if (mode == 0) PH_END(T);
    }
    PH_BEGIN(T, BPJD_PHASE_GATHER);
    if (mixed)
        launch_scatter_f32(st, p->n, s, (int)p->sumN, p->Pptr, p->Pcol, p->Pval, p->Zhat, p->rptr, p->ridx,
                           (const float*)p->zloc, Z, ldz);
    else
        launch_scatter_f64(st, p->n, s, (int)p->sumN, p->Pptr, p->Pcol, p->Pval, p->Zhat, p->rptr, p->ridx,
                           (const double*)p->zloc, Z, ldz);
    PH_END(T);
}

// M-orthonormalise the T block (columns ct..ct+s of buffer b) against the first
// ct columns (classical Gram-Schmidt, two passes) and within itself
// (Cholesky-QR, two passes).  K T and M T are updated by the same linear maps.
// T (columns ct.. of buffer b) <- M-orthonormal basis of (I - [X P][X P]^T M) T:
// two classical Gram-Schmidt passes against [X P] (Gram matrices (M [X P])^T T, so
// only T itself is updated), then K T and M T by one SpMM, then two Cholesky-QR
// passes applied to T, K T and M T alike.
static void orthonormalize_T(bpjd_problem* p, int b, int ct, PhaseTimer* T) {
    hipStream_t st = p->ctx->stream;
    const int n = p->n, s = p->s;
    const BlockGeom g = wgeom(p);
    double *W = p->W[b], *KW = p->KW[b], *MW = p->MW[b];
    double* T0 = blkp(p, W, ct);
    const double* src1[1] = {W};
    double* dst1[1] = {T0};
    double* dst3[3] = {T0, blkp(p, KW, ct), blkp(p, MW, ct)};
    PH_BEGIN(T, BPJD_PHASE_ORTHO);
    for (int pass = 0; pass < 2 && ct > 0; ++pass) {
        launch_gram(st, n, ct, s, MW, T0, g, p->partial, p->npart, p->csmall);
        launch_gemm_rows(st, n, ct, s, -1.0, src1, dst1, 1, g, p->csmall, 1.0);
    }
    PH_END(T);
    PH_BEGIN(T, BPJD_PHASE_SPMM);
    launch_spmm_km(st, n, p->rowptr, p->col, p->km, T0, s, s, dst3[1], s, dst3[2], s, p->spmm_variant);
    PH_END(T);
    PH_BEGIN(T, BPJD_PHASE_ORTHO);
    for (int pass = 0; pass < 2; ++pass) {
        launch_gram(st, n, s, s, T0, dst3[2], g, p->partial, p->npart, p->gsmall);
        launch_cholqr_coef(st, s, p->gsmall, p->csmall, p->dropped[b] + ct, p->status);
        launch_rightmul_rows(st, n, s, dst3, 3, g, p->csmall);
    }
    PH_END(T);
}

// Rayleigh-Ritz on W = buffer a (m columns), new X (and P when with_p) into buffer b.
static void rayleigh_ritz(bpjd_problem* p, int a, int b, int m, int with_p, PhaseTimer* T) {
    hipStream_t st = p->ctx->stream;
    const int n = p->n, s = p->s;
    const BlockGeom g = wgeom(p);
    PH_BEGIN(T, BPJD_PHASE_RR);
    launch_gram(st, n, m, m, p->W[a], p->KW[a], g, p->partial, p->npart, p->Hm);
    launch_rr_coef(st, m, s, with_p, p->Hm, p->dropped[a], p->dropped[b], p->theta, p->lam, p->Cfull);
    const int cw = with_p ? 2 * s : s;
    const double* src3[3] = {p->W[a], p->KW[a], p->MW[a]};
    double* dst3[3] = {p->W[b], p->KW[b], p->MW[b]};
    launch_gemm_rows(st, n, m, cw, 1.0, src3, dst3, 3, g, p->Cfull, 0.0);
    PH_END(T);
}

}  // namespace bpjd

// ======================================================================================
// numeric driver
// ======================================================================================
namespace bpjd {

static int run_setup(bpjd_problem* p) {
    hipStream_t st = p->ctx->stream;
    BPJD_HIP(hipSetDevice(p->ctx->device));
    BPJD_HIP(hipMemsetAsync(p->status, 0, sizeof(int), st));
    coarse_setup(p);
    BPJD_TRY(check_status(p));
    p->setup_done = true;
    return BPJD_OK;
}

// Start block (Step 1 with H~ = H): X = P Y_s, Lambda = lambda^H_{1..s}; with a
// caller block X_init, W^0 = span{P Y_s, X_init} and a Rayleigh-Ritz step.
static int start_block(bpjd_problem* p) {
    hipStream_t st = p->ctx->stream;
    const int n = p->n, s = p->s, ld = s;
    BPJD_HIP(hipMemsetAsync(p->dropped[0], 0, 64 * sizeof(int), st));
    BPJD_HIP(hipMemsetAsync(p->dropped[1], 0, 64 * sizeof(int), st));
    launch_csr_dense(st, n, p->Pptr, p->Pcol, p->Pval, p->Y, p->nH, s, p->W[0], ld, false);
    launch_copy_cols(st, 1, s, p->lamH, s, p->lam, s);
    launch_spmm_km(st, n, p->rowptr, p->col, p->km, p->W[0], ld, s, p->KW[0], ld, p->MW[0], ld, p->spmm_variant);
    if (p->n_init) {
        BPJD_HIP(hipMemcpyAsync(blkp(p, p->W[0], s), p->X_init.data(), sizeof(double) * n * s,
                                hipMemcpyHostToDevice, st));
        orthonormalize_T(p, 0, s, nullptr);
        rayleigh_ritz(p, 0, 1, 2 * s, 0, nullptr);
        // result in buffer 1: move it back to buffer 0 (the iteration starts from buffer 0)
        launch_copy_cols(st, n, s, p->W[1], ld, p->W[0], ld);
        launch_copy_cols(st, n, s, p->KW[1], ld, p->KW[0], ld);
        launch_copy_cols(st, n, s, p->MW[1], ld, p->MW[0], ld);
        BPJD_HIP(hipMemsetAsync(p->dropped[0], 0, 64 * sizeof(int), st));
    }
    return BPJD_OK;
}

// One solve as a state machine, so that several solves can share the device: every
// stage ends with an asynchronous read-back of a few scalars and an event; the next
// stage is enqueued once that event has completed (run_poll / run_advance).  A plain
// bpjd_solve drives one machine to the end; the server interleaves many.
struct SolveRun {
    bpjd_problem* p = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, erb = nullptr;
    PhaseTimer timer;
    PhaseTimer* T = nullptr;
    enum Stage { IDLE, SETUP, ITER, DONE, FAILED } stage = IDLE;
    int cur = 0;        // buffer holding X (and P)
    int np = 0;         // columns of P in use (0 or s)
    int it = 0;         // outer iteration whose residual is being read back
    int iters = 0;
    int graph_iters = 0;    // iterations launched as a graph replay
    int grow_m = 0;         // GROW: columns of W in use
    bool converged = false;
    bool fresh = false; // the residual being read back comes from K X, M X formed from X itself
    double stop_value = NAN;
    std::vector<double> lam_prev, lam_now, rho;
    ~SolveRun() {
        for (hipEvent_t x : {e0, e1, e2, erb})
            if (x) (void)hipEventDestroy(x);
    }
};

int run_create(bpjd_problem* p, SolveRun** out) {
    auto* r = new SolveRun();
    r->p = p;
    const int s = p->s;
    r->lam_prev.assign(s, 0.0);
    r->lam_now.assign(s, 0.0);
    r->rho.assign(s, 0.0);
    r->timer.st = p->ctx->stream;
    if (p->opts.profile == 2) r->timer.mask = 1u << BPJD_PHASE_LOCAL;
    r->T = p->opts.profile ? &r->timer : nullptr;
    if (hipEventCreate(&r->e0) != hipSuccess || hipEventCreate(&r->e1) != hipSuccess ||
        hipEventCreate(&r->e2) != hipSuccess ||
        hipEventCreateWithFlags(&r->erb, hipEventDisableTiming) != hipSuccess) {
        delete r;
        return fail(BPJD_ERR_HIP, "hipEventCreate failed");
    }
    *out = r;
    return BPJD_OK;
}

void run_destroy(SolveRun* r) { delete r; }

// residual block F = M X Lambda - K X and its column norms, then one read-back of the
// column norms, shifts and status word into the pinned mirror, then the event
static int enqueue_residual_work(SolveRun* r, int a) {
    bpjd_problem* p = r->p;
    hipStream_t st = p->ctx->stream;
    const int n = p->n, s = p->s;
    PH_BEGIN(r->T, BPJD_PHASE_RESIDUAL);
    launch_residual(st, n, s, p->KW[a], s, p->MW[a], s, p->lam, p->F, s, p->partial, p->npart, p->colsq,
                    p->colsq + 128, p->status);
    PH_END(r->T);
    BPJD_HIP(hipMemcpyAsync(p->hbuf, p->colsq, sizeof(double) * 193, hipMemcpyDeviceToHost, st));
    return BPJD_OK;
}

static int enqueue_residual(SolveRun* r) {
    BPJD_TRY(enqueue_residual_work(r, r->cur));
    BPJD_HIP(hipEventRecord(r->erb, r->p->ctx->stream));
    return BPJD_OK;
}

// One outer iteration after the stop test (Steps 2 and 3, then the next residual and
// its read-back) on buffers a -> 1 - a with np columns of P in W.
static void enqueue_iteration(SolveRun* r, int a, int np) {
    bpjd_problem* p = r->p;
    const int s = p->s;
    const bool uu = p->opts.subspace == BPJD_SUBSPACE_UU;
    const int ct = s + np;
    apply_precond(p, p->F, blkp(p, p->W[a], ct), s, r->T);
    orthonormalize_T(p, a, ct, r->T);
    rayleigh_ritz(p, a, 1 - a, ct + s, uu ? 1 : 0, r->T);
}

// Chunks of whole n x s blocks of a growing basis, at most 64 columns each (the limit of
// the Gram and tall-times-small kernels): calls f(first column, columns).
template <class F>
static void for_chunks(int m, int s, F&& f) {
    const int per = std::max(1, 64 / s) * s;
    for (int c0 = 0; c0 < m; c0 += per) f(c0, std::min(per, m - c0));
}

// Start of W^0 = span{X} for the growing subspace: W and M W take X and M X (buffer 0,
// block 0), the projected matrix H = X^T K X.
static void grow_start(SolveRun* r) {
    bpjd_problem* p = r->p;
    hipStream_t st = p->ctx->stream;
    const int n = p->n, s = p->s;
    const BlockGeom g = wgeom(p);
    (void)hipMemsetAsync(p->dropg, 0, sizeof(int) * p->grow_cap, st);   // GROW is never graph-captured
    launch_copy_cols(st, n, s, p->W[0], s, p->Wg, s);
    launch_copy_cols(st, n, s, p->MW[0], s, p->MWg, s);
    launch_gram(st, n, s, s, p->W[0], p->KW[0], g, p->partial, p->npart, p->Cg);
    launch_grow_place(st, 0, s, p->Cg, p->dropg, p->Hg, p->grow_cap);
    r->grow_m = s;
}

// One outer iteration with W^{k+1} = W^k + span{t_i} (Algorithm 3.1, Step 3 as written):
// t_i into block 1 of buffer 0, two classical Gram-Schmidt passes against all of W (with
// the stored M W), K T and M T by one SpMM, two Cholesky-QR passes; T and M T become
// W's next block; the new column block of H = W^T K W from one Gram product with K T;
// the lowest s eigenpairs of H (dense symmetric eigensolver); X = W Q_s and K X, M X by
// one SpMM, then the next residual.  Shapes change every step, so it is not captured.
static int enqueue_iteration_grow(SolveRun* r) {
    bpjd_problem* p = r->p;
    hipStream_t st = p->ctx->stream;
    const int n = p->n, s = p->s;
    const BlockGeom g = wgeom(p);
    const long long bsp = block_stride(n, s);
    const int m = r->grow_m;
    if (m + s > p->grow_cap)
        return fail(BPJD_ERR_NOCONV, "growing subspace reached its dimension limit (" + std::to_string(p->grow_cap) +
                                         ")");
    double* T = blkp(p, p->W[0], s);
    double* KT = blkp(p, p->KW[0], s);
    double* MT = blkp(p, p->MW[0], s);
    apply_precond(p, p->F, T, s, r->T);
    PH_BEGIN(r->T, BPJD_PHASE_ORTHO);
    for (int pass = 0; pass < 2; ++pass) {
        for_chunks(m, s, [&](int c0, int cc) {
            launch_gram(st, n, cc, s, p->MWg + (c0 / s) * bsp, T, g, p->partial, p->npart, p->Cg + (size_t)c0 * s);
        });
        for_chunks(m, s, [&](int c0, int cc) {
            const double* src[1] = {p->Wg + (c0 / s) * bsp};
            double* dst[1] = {T};
            launch_gemm_rows(st, n, cc, s, -1.0, src, dst, 1, g, p->Cg + (size_t)c0 * s, 1.0);
        });
    }
    PH_END(r->T);
    PH_BEGIN(r->T, BPJD_PHASE_SPMM);
    launch_spmm_km(st, n, p->rowptr, p->col, p->km, T, s, s, KT, s, MT, s, p->spmm_variant);
    PH_END(r->T);
    PH_BEGIN(r->T, BPJD_PHASE_ORTHO);
    double* dst3[3] = {T, KT, MT};
    for (int pass = 0; pass < 2; ++pass) {
        launch_gram(st, n, s, s, T, MT, g, p->partial, p->npart, p->gsmall);
        launch_cholqr_coef(st, s, p->gsmall, p->csmall, p->dropg + m, p->status);
        launch_rightmul_rows(st, n, s, dst3, 3, g, p->csmall);
    }
    launch_copy_cols(st, n, s, T, s, p->Wg + (m / s) * bsp, s);
    launch_copy_cols(st, n, s, MT, s, p->MWg + (m / s) * bsp, s);
    PH_END(r->T);
    PH_BEGIN(r->T, BPJD_PHASE_RR);
    const int mn = m + s;
    for_chunks(mn, s, [&](int c0, int cc) {
        launch_gram(st, n, cc, s, p->Wg + (c0 / s) * bsp, KT, g, p->partial, p->npart, p->Cg + (size_t)c0 * s);
    });
    launch_grow_place(st, m, s, p->Cg, p->dropg, p->Hg, p->grow_cap);
    launch_copy_cols(st, mn, mn, p->Hg, p->grow_cap, p->Hw, mn);
    launch_sym_eig(st, mn, p->Hw, p->thetag, p->Vg, p->gwork, p->gsmall2, p->gscratch, p->status);
    launch_copy_cols(st, mn, s, p->Vg, mn, p->Qg, s);
    launch_copy_cols(st, 1, s, p->thetag, s, p->lam, s);
    for_chunks(mn, s, [&](int c0, int cc) {
        const double* src[1] = {p->Wg + (c0 / s) * bsp};
        double* dst[1] = {p->W[0]};
        launch_gemm_rows(st, n, cc, s, 1.0, src, dst, 1, g, p->Qg + (size_t)c0 * s, c0 == 0 ? 0.0 : 1.0);
    });
    PH_END(r->T);
    PH_BEGIN(r->T, BPJD_PHASE_SPMM);
    launch_spmm_km(st, n, p->rowptr, p->col, p->km, p->W[0], s, s, p->KW[0], s, p->MW[0], s, p->spmm_variant);
    PH_END(r->T);
    r->grow_m = mn;
    return BPJD_OK;
}

// The same iteration as a HIP graph: captured from the problem's stream the first time
// a (buffer, P columns) combination occurs, then replayed; its kernel arguments are the
// problem's fixed buffers and sizes.  Returns false when capture is not available (the
// caller then launches the kernels directly and stops trying for this problem).
static bool launch_iteration_graph(SolveRun* r, int a, int np) {
    bpjd_problem* p = r->p;
    hipStream_t st = p->ctx->stream;
    hipGraphExec_t& ge = p->graph_exec[a][np > 0 ? 1 : 0];
    if (!ge) {
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
        enqueue_iteration(r, a, np);
        const int rc = enqueue_residual_work(r, 1 - a);
        if (hipStreamEndCapture(st, &g) != hipSuccess || rc < 0 || !g) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return false;   // nothing was enqueued: the caller launches the iteration directly
        }
        const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            ge = nullptr;
            (void)hipGetLastError();
            return false;
        }
    }
    return hipGraphLaunch(ge, st) == hipSuccess;
}

int run_begin(SolveRun* r) {
    bpjd_problem* p = r->p;
    hipStream_t st = p->ctx->stream;
    BPJD_HIP(hipSetDevice(p->ctx->device));
    BPJD_HIP(hipEventRecord(r->e0, st));
    PH_BEGIN(r->T, BPJD_PHASE_SETUP);
    BPJD_HIP(hipMemsetAsync(p->status, 0, sizeof(int), st));
    coarse_setup(p);
    BPJD_HIP(hipMemcpyAsync(p->hbuf + 256, p->status, sizeof(int), hipMemcpyDeviceToHost, st));
    BPJD_HIP(hipEventRecord(r->erb, st));
    r->stage = SolveRun::SETUP;
    return BPJD_OK;
}

// 1: the pending read-back has arrived; 0: not yet; < 0: HIP error
int run_poll(SolveRun* r) {
    const hipError_t q = hipEventQuery(r->erb);
    if (q == hipSuccess) return 1;
    if (q == hipErrorNotReady) return 0;
    return fail(BPJD_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
}

int run_wait(SolveRun* r) {
    // spin (no yield): the next launches follow the read-back as closely as possible
    int q;
    while ((q = run_poll(r)) == 0) {
    }
    return q < 0 ? q : BPJD_OK;
}

// ---- autotuner ----------------------------------------------------------------------
// Launch shapes that leave the data layout and the arithmetic unchanged (results are the
// same bit for bit) are timed on the problem's own data when it is first set up: the
// threads per system of the windowed local solver (64, 128 or 256) and the SpMM form (two
// columns per lane or one).  The fastest is kept per process, keyed by the problem's shape,
// and appended to the file named by BPJD_TUNE_CACHE when that is set (read at the first
// tuning of the process).
namespace {
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("BPJD_TUNE_CACHE");
    if (!path) return;
    std::ifstream in(path);
    std::string key, rest;
    while (std::getline(in, rest)) {
        const size_t sp = rest.rfind(' ');
        if (sp == std::string::npos) continue;
        key = rest.substr(0, sp);
        try {
            g_tune[key] = std::stoi(rest.substr(sp + 1));
        } catch (...) {
        }
    }
}
}  // namespace

// milliseconds per call of `launch` on st: one warm-up call, then `reps` timed calls
template <class Launch>
static int time_launch(hipStream_t st, Launch&& launch, int reps, float* ms) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return fail(BPJD_ERR_HIP, "autotune: hipEventCreate failed");
    }
    launch();
    hipError_t e = hipEventRecord(a, st);
    for (int q = 0; q < reps; ++q) launch();
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail(BPJD_ERR_HIP, std::string("autotune timing: ") + hipGetErrorString(e));
    *ms = t / reps;
    return BPJD_OK;
}

// the cached choice for `key`, else the fastest of `cands` timed with run(candidate)
template <class Run>
static int tune_choice(const std::string& key, const std::vector<int>& cands, hipStream_t st, Run&& run, int* out) {
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end() && std::find(cands.begin(), cands.end(), it->second) != cands.end()) {
            *out = it->second;
            return BPJD_OK;
        }
    }
    int best = cands[0];
    float tbest = 0.f;
    for (size_t q = 0; q < cands.size(); ++q) {
        float t = 0.f;
        BPJD_TRY(time_launch(st, [&] { run(cands[q]); }, 2, &t));
        if (q == 0 || t < tbest) {
            tbest = t;
            best = cands[q];
        }
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto ins = g_tune.emplace(key, best);     // another thread may have tuned the same shape first
    *out = ins.first->second;
    if (ins.second) {
        if (const char* path = std::getenv("BPJD_TUNE_CACHE")) {
            std::ofstream o(path, std::ios::app);
            o << key << ' ' << best << '\n';
        }
    }
    return BPJD_OK;
}

// Runs after the first numeric setup of a problem, outside any stream capture.  The SpMM
// candidates write buffer 1's products (not yet in use); the local-solve candidates solve
// zero right-hand sides with the current shifts (the factorisations are the real ones).
static int autotune(bpjd_problem* p) {
    hipStream_t st = p->ctx->stream;
    const int s = p->s;
    const bool mixed = p->opts.precision == BPJD_PREC_MIXED;
    char key[192];
    if (p->opts.spmm_form == 0) {
        std::snprintf(key, sizeof key, "spmm n%d nnz%lld c%d", p->n, p->nnz, s);
        const std::vector<int> cands = s % 2 == 0 ? std::vector<int>{0, 1, 2} : std::vector<int>{1, 2};
        BPJD_TRY(tune_choice(key, cands, st, [&](int v) {
            launch_spmm_km(st, p->n, p->rowptr, p->col, p->km, p->W[0], s, s, p->KW[1], s, p->MW[1], s, v);
        }, &p->spmm_variant));
    }
    if (!p->blocked && p->opts.local_threads == 0) {
        BPJD_HIP(hipMemsetAsync(p->Floc, 0, (size_t)p->sumN * s * (mixed ? sizeof(float) : sizeof(double)), st));
        std::snprintf(key, sizeof key, "ldlt %s s%d sub%d n%d w%d e%d", mixed ? "f32" : "f64", s, p->nsub, p->maxN,
                      p->maxBW, p->slotE);
        BPJD_TRY(tune_choice(key, {64, 128, 256}, st, [&](int th) {
            if (mixed)
                launch_local_solve_f32(st, 0, p->nsub, s, p->maxC, p->sumN, p->subptr, p->bw, 0, p->slotE, p->bws,
                                       p->sd, p->sv, p->lam, (const float*)p->Floc, (float*)p->zloc,
                                       (float*)p->Lwork, p->Loff, p->sysord, p->status, p->negflag, th);
            else
                launch_local_solve_f64(st, 0, p->nsub, s, p->maxC, p->sumN, p->subptr, p->bw, 0, p->slotE, p->bws,
                                       p->sd, p->sv, p->lam, (const double*)p->Floc, (double*)p->zloc,
                                       (double*)p->Lwork, p->Loff, p->sysord, p->status, p->negflag, th);
        }, &p->ldlt_threads));
    }
    return BPJD_OK;
}

static int advance_setup(SolveRun* r) {
    bpjd_problem* p = r->p;
    const int st_word = *reinterpret_cast<const int*>(p->hbuf + 256);
    if (st_word & STATUS_COARSE_NOT_SPD) return fail(BPJD_ERR_NOT_SPD, "coarse mass matrix M_H is not positive definite");
    if (st_word & STATUS_LOCAL_PIVOT) return fail(BPJD_ERR_NOT_SPD, "singular pivot in a local factorisation");
    p->setup_done = true;
    BPJD_TRY(start_block(p));
    if (p->opts.subspace == BPJD_SUBSPACE_GROW) grow_start(r);
    if (!p->tuned) {
        if (p->opts.autotune) BPJD_TRY(autotune(p));
        p->tuned = true;
    }
    PH_END(r->T);
    BPJD_HIP(hipEventRecord(r->e1, p->ctx->stream));
    BPJD_TRY(enqueue_residual(r));
    r->stage = SolveRun::ITER;
    return 0;
}

static int advance_iter(SolveRun* r) {
    bpjd_problem* p = r->p;
    hipStream_t st = p->ctx->stream;
    const int s = p->s, k = p->k;
    const bool uu = p->opts.subspace == BPJD_SUBSPACE_UU;
    const double* h = p->hbuf;
    const int hstatus = *reinterpret_cast<const int*>(h + 192);
    if (r->T) r->T->collect();
    if (hstatus & STATUS_LOCAL_PIVOT) return fail(BPJD_ERR_NOT_SPD, "singular pivot in a local factorisation");
    for (int i = 0; i < s; ++i) {
        r->lam_now[i] = h[128 + i];
        r->rho[i] = std::sqrt(h[i]) / (std::fabs(r->lam_now[i]) * std::sqrt(h[s + i]));
    }
    double rmax = 0.0;
    bool finite = true;
    for (int i = 0; i < k; ++i) {
        rmax = std::max(rmax, r->rho[i]);
        finite = finite && std::isfinite(r->rho[i]);
    }
    if (!finite) return fail(BPJD_ERR_NOT_SPD, "non-finite residual (breakdown)");
    if (r->it > 0) {
        r->stop_value = 0.0;
        for (int i = 0; i < s; ++i) r->stop_value += std::fabs(r->lam_now[i] - r->lam_prev[i]);
    }
    if (p->trace) {
        char head[200];
        std::snprintf(head, sizeof head,
                      "{\"event\": \"iteration\", \"problem\": \"%p\", \"it\": %d, \"fresh\": %s, "
                      "\"rho_max\": %.6e, \"stop_value\": %.6e, ",
                      (const void*)p, r->it, r->fresh ? "true" : "false", rmax, r->it > 0 ? r->stop_value : 0.0);
        trace_line(std::string(head) + "\"lambda\": " + json_doubles(r->lam_now.data(), s) +
                   ", \"rho\": " + json_doubles(r->rho.data(), k, "%.6e") + "}");
    }
    bool stop = false;
    if (p->opts.stop_rule == BPJD_STOP_RESIDUAL && rmax <= p->opts.tol) {
        if (!r->fresh) {
            // K X and M X are carried through the Rayleigh-Ritz updates (X <- W Q with
            // K X <- (K W) Q), and rounding lets them drift from the products of X itself
            // by about u |K| |X| per update: far above the residual for a fourth-order
            // operator on a fine mesh.  The stop is decided on products formed afresh.
            PH_BEGIN(r->T, BPJD_PHASE_SPMM);
            launch_spmm_km(st, p->n, p->rowptr, p->col, p->km, p->W[r->cur], s, s, p->KW[r->cur], s,
                           p->MW[r->cur], s, p->spmm_variant);
            PH_END(r->T);
            r->fresh = true;
            BPJD_TRY(enqueue_residual(r));
            return 0;
        }
        stop = r->converged = true;
    }
    if (p->opts.stop_rule == BPJD_STOP_PAPER && r->it > 0 && r->stop_value < p->opts.tol) stop = r->converged = true;
    if (r->it == p->opts.max_iter) stop = true;
    if (stop) {
        BPJD_HIP(hipEventRecord(r->e2, st));
        r->stage = SolveRun::DONE;
        return 1;
    }
    r->lam_prev = r->lam_now;

    // Step 2: t_i = (I - X X^T M) (B_i)^{-1} r_i, written straight into the T slot of W.
    // The projection (I - X X^T M) of Step 2 is the first Gram-Schmidt pass of
    // the M-orthonormalisation against [X | P] below (same subspace W^{k+1}).
    const int a = r->cur;
    const int ct = s + r->np;
    if (p->opts.subspace == BPJD_SUBSPACE_GROW) {
        BPJD_TRY(enqueue_iteration_grow(r));
        r->fresh = true;        // K X and M X come from an SpMM of X itself
        r->iters = ++r->it;
        BPJD_TRY(enqueue_residual(r));
        return 0;
    }
    // Step 3: Rayleigh-Ritz on W = [X | P | T]; then the next residual and its read-back.
    // Replayed as a HIP graph unless phases are timed, the iteration is traced, or the
    // caller turned graphs off.
    const bool graph = p->opts.graphs && !r->T && !p->trace && !p->graph_failed;
    r->fresh = false;
    if (graph && launch_iteration_graph(r, a, r->np)) {
        r->graph_iters++;
        r->cur = 1 - a;
        r->np = uu ? s : 0;
        r->iters = ++r->it;
        BPJD_HIP(hipEventRecord(r->erb, st));
        return 0;
    }
    if (graph) {
        p->graph_failed = true;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
            return fail(BPJD_ERR_HIP, "stream left in capture mode by a failed graph capture");
        (void)hipGetLastError();
    }
    enqueue_iteration(r, a, r->np);
    if (p->trace) {
        int fl[128];
        BPJD_HIP(hipMemcpyAsync(fl, p->dropped[a], sizeof(int) * (ct + s), hipMemcpyDeviceToHost, st));
        BPJD_HIP(hipMemcpyAsync(fl + 64, p->dropped[1 - a], sizeof(int) * 2 * s, hipMemcpyDeviceToHost, st));
        double th[64];
        BPJD_HIP(hipMemcpyAsync(th, p->theta, sizeof(double) * (ct + s), hipMemcpyDeviceToHost, st));
        BPJD_HIP(hipStreamSynchronize(st));
        std::string din, dout;
        for (int q = 0; q < ct + s; ++q) din += fl[q] ? '1' : '0';
        for (int q = 0; q < 2 * s; ++q) dout += fl[64 + q] ? '1' : '0';
        char head[160];
        std::snprintf(head, sizeof head, "{\"event\": \"rayleigh_ritz\", \"problem\": \"%p\", \"it\": %d, \"m\": %d, ",
                      (const void*)p, r->it, ct + s);
        trace_line(std::string(head) + "\"dropped_in\": \"" + din + "\", \"dropped_out\": \"" + dout +
                   "\", \"theta\": " + json_doubles(th, ct + s, "%.10g") + "}");
    }
    r->cur = 1 - a;
    r->np = uu ? s : 0;
    r->iters = ++r->it;
    BPJD_TRY(enqueue_residual(r));
    return 0;
}

// Consume the arrived read-back and enqueue the next stage: 1 = the stop rule (or the
// iteration cap) was reached, 0 = more work was enqueued, < 0 = error.
int run_advance(SolveRun* r) {
    int rc;
    switch (r->stage) {
        case SolveRun::SETUP: rc = advance_setup(r); break;
        case SolveRun::ITER: rc = advance_iter(r); break;
        case SolveRun::DONE: return 1;
        default: return fail(BPJD_ERR_STATE, "solve not started");
    }
    if (rc < 0) r->stage = SolveRun::FAILED;
    return rc;
}

// Copy the result out (eigvals: k values; eigvecs: n x k row-major; both in `mem`) and
// fill the statistics.  Synchronises the problem's stream.
int run_finish(SolveRun* r, double* eigvals, double* eigvecs, int mem, bpjd_stats* stats) {
    bpjd_problem* p = r->p;
    if (r->stage != SolveRun::DONE) return fail(BPJD_ERR_STATE, "solve has not finished");
    hipStream_t st = p->ctx->stream;
    const int n = p->n, s = p->s, k = p->k;
    BPJD_HIP(hipEventSynchronize(r->e2));
    if (r->T) r->T->collect();
    float ms_setup = 0.f, ms_iter = 0.f;
    BPJD_HIP(hipEventElapsedTime(&ms_setup, r->e0, r->e1));
    BPJD_HIP(hipEventElapsedTime(&ms_iter, r->e1, r->e2));
    const int a = r->cur;
    if (eigvals) {
        if (mem == BPJD_MEM_DEVICE) {
            BPJD_HIP(hipMemcpyAsync(eigvals, p->lam, sizeof(double) * k, hipMemcpyDeviceToDevice, st));
        } else {
            std::memcpy(eigvals, r->lam_now.data(), sizeof(double) * k);
        }
    }
    if (eigvecs) {
        if (mem == BPJD_MEM_DEVICE) {
            launch_copy_cols(st, n, k, p->W[a], s, eigvecs, k);
        } else {
            launch_copy_cols(st, n, k, p->W[a], s, p->Z, k);
            BPJD_HIP(hipMemcpyAsync(eigvecs, p->Z, sizeof(double) * n * k, hipMemcpyDeviceToHost, st));
        }
    }
    BPJD_HIP(hipStreamSynchronize(st));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iterations = r->iters;
        stats->graph_iterations = r->graph_iters;
        if (p->trace) {
            char buf[256];
            std::snprintf(buf, sizeof buf,
                          "{\"event\": \"solve\", \"problem\": \"%p\", \"iterations\": %d, \"converged\": %s, "
                          "\"stop_value\": %.6e, \"setup_ms\": %.3f, \"iterate_ms\": %.3f}",
                          (const void*)p, r->iters, r->converged ? "true" : "false", r->stop_value, ms_setup, ms_iter);
            trace_line(buf);
        }
        stats->spmm_form = (p->spmm_variant == 0 && p->s % 2) ? BPJD_SPMM_COLUMN : p->spmm_variant + 1;
        stats->converged = r->converged ? 1 : 0;
        stats->stop_value = r->stop_value;
        double rmax = 0.0;
        for (int i = 0; i < k; ++i) rmax = std::max(rmax, r->rho[i]);
        stats->max_residual = rmax;
        for (int i = 0; i < k && i < 64; ++i) stats->residuals[i] = r->rho[i];
        stats->setup_ms = ms_setup;
        stats->iterate_ms = ms_iter;
        stats->n_sub = p->nsub;
        stats->n_coarse = p->nH;
        stats->max_local = p->maxN;
        stats->max_band = p->maxBW;
        for (int q = 0; q < BPJD_NUM_PHASES; ++q) {
            stats->phase_ms[q] = r->timer.ms[q];
            stats->phase_count[q] = r->timer.count[q];
        }
    }
    if (!r->converged) return fail(BPJD_ERR_NOCONV, "maximum number of iterations reached");
    return BPJD_OK;
}

static int run_solve(bpjd_problem* p, double* eigvals, double* eigvecs, int mem, bpjd_stats* stats) {
    SolveRun* raw = nullptr;
    BPJD_TRY(run_create(p, &raw));
    std::unique_ptr<SolveRun> r(raw);
    BPJD_TRY(run_begin(r.get()));
    for (;;) {
        BPJD_TRY(run_wait(r.get()));
        const int q = run_advance(r.get());
        if (q < 0) return q;
        if (q == 1) break;
    }
    return run_finish(r.get(), eigvals, eigvecs, mem, stats);
}

}  // namespace bpjd

// ======================================================================================
// C ABI
// ======================================================================================
using namespace bpjd;

extern "C" {

void bpjd_opts_default(bpjd_opts* o, int32_t k) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->k = k;
    o->guard = 0;
    o->max_iter = 500;
    o->tol = 1e-8;
    o->stop_rule = BPJD_STOP_RESIDUAL;
    o->subspace = BPJD_SUBSPACE_UU;
    o->precision = BPJD_PREC_MIXED;
    o->n_init = 0;
    o->X_init = nullptr;
    o->graphs = 1;
    o->autotune = 1;
}

int bpjd_ctx_create(int device, const bpjd_allocator* allocator, void* hip_stream, bpjd_ctx** out) {
    if (!out) return fail(BPJD_ERR_ARG, "out is NULL");
    if (allocator && (!allocator->alloc) != (!allocator->free))
        return fail(BPJD_ERR_ARG, "allocator needs both alloc and free (or neither)");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(BPJD_ERR_HIP, "no HIP device");
    if (device < 0 || device >= count) return fail(BPJD_ERR_ARG, "device ordinal out of range");
    BPJD_HIP(hipSetDevice(device));
    BPJD_TRY(noalloc_init(device));
    bpjd_ctx* c = new bpjd_ctx();
    c->device = device;
    if (allocator) c->alloc = *allocator;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) {
            delete c;
            return fail(BPJD_ERR_HIP, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    *out = c;
    return BPJD_OK;
}

void bpjd_ctx_destroy(bpjd_ctx* ctx) {
    if (!ctx) return;
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

}  // extern "C"

namespace bpjd {

static int plan_dd(bpjd_ctx* ctx, const bpjd_csr* K, const bpjd_csr* M, const bpjd_dd* dd,
                   const bpjd_opts* opts, bpjd_problem** out) {
    StageClock clk;
    HostCSR hK, hM, P;
    Pattern U;
    BPJD_TRY(read_pair(K, M, hK, hM, U, ctx->stream, &clk));
    if (dd->P.n_rows != U.n || dd->P.n_cols < 1) return fail(BPJD_ERR_DD, "P must be n x n_H");
    {
        // P is rectangular: read it without the square check
        bpjd_csr Pc = dd->P;
        const int nH = Pc.n_cols;
        Pc.n_cols = Pc.n_rows;
        HostCSR tmp;
        // reuse the reader for bounds/order checks against n_rows, then re-check columns against n_H
        int rc = read_csr(&Pc, "P", tmp, ctx->stream);
        if (rc < 0 && rc != BPJD_ERR_CSR) return rc;
        if (rc == BPJD_ERR_CSR) return fail(BPJD_ERR_DD, "P: " + std::string(g_last_error));
        for (int c : tmp.col)
            if (c >= nH) return fail(BPJD_ERR_DD, "P column index out of range");
        P = std::move(tmp);
        if (dd->n_sub < 1 || !dd->sub_ptr || !dd->sub_idx) return fail(BPJD_ERR_DD, "no subdomains");
        std::vector<int> sptr(dd->sub_ptr, dd->sub_ptr + dd->n_sub + 1);
        if (sptr[0] != 0) return fail(BPJD_ERR_DD, "sub_ptr[0] must be 0");
        for (int l = 0; l < dd->n_sub; ++l)
            if (sptr[l + 1] < sptr[l]) return fail(BPJD_ERR_DD, "sub_ptr not monotone");
        std::vector<int> sidx(dd->sub_idx, dd->sub_idx + sptr[dd->n_sub]);
        clk.mark("prolongation");
        return finish_create(ctx, hK, hM, U, P, nH, sptr, sidx, opts, out, clk);
    }
}

static int plan_geom(bpjd_ctx* ctx, const bpjd_csr* K, const bpjd_csr* M, const bpjd_dd_geom* g,
                     const bpjd_opts* opts, bpjd_problem** out) {
    if (!g->coords || !g->cx || !g->cy || g->n_cx < 2 || g->n_cy < 2) return fail(BPJD_ERR_ARG, "bad coarse grid");
    StageClock clk;
    HostCSR hK, hM, P;
    Pattern U;
    BPJD_TRY(read_pair(K, M, hK, hM, U, ctx->stream, &clk));
    std::vector<double> cx(g->cx, g->cx + g->n_cx), cy(g->cy, g->cy + g->n_cy);
    for (size_t i = 0; i + 1 < cx.size(); ++i)
        if (!(cx[i + 1] > cx[i])) return fail(BPJD_ERR_ARG, "cx not increasing");
    for (size_t i = 0; i + 1 < cy.size(); ++i)
        if (!(cy[i + 1] > cy[i])) return fail(BPJD_ERR_ARG, "cy not increasing");
    int nH = 0;
    build_p1_prolongation(U.n, g->coords, cx, cy, P, nH);
    clk.mark("prolongation");
    if (nH < 1) return fail(BPJD_ERR_DD, "coarse grid has no interior vertex");
    std::vector<int> sptr, sidx;
    BPJD_TRY(build_geom_subdomains(U, g->coords, cx, cy, g->overlap_layers, g->cell_shape, sptr, sidx));
    clk.mark("subdomains");
    return finish_create(ctx, hK, hM, U, P, nH, sptr, sidx, opts, out, clk);
}

// Host planning of a problem (validation, structure, footprint) without device memory;
// exactly one of dd / geom is used.
int plan_problem(bpjd_ctx* ctx, const bpjd_csr* K, const bpjd_csr* M, const bpjd_dd* dd, const bpjd_dd_geom* geom,
                 const bpjd_opts* opts, bpjd_problem** out) {
    if (!ctx || !K || !M || (!dd && !geom) || !opts || !out) return fail(BPJD_ERR_ARG, "NULL argument");
    return dd ? plan_dd(ctx, K, M, dd, opts, out) : plan_geom(ctx, K, M, geom, opts, out);
}

static int create_now(bpjd_ctx* ctx, const bpjd_csr* K, const bpjd_csr* M, const bpjd_dd* dd,
                      const bpjd_dd_geom* geom, const bpjd_opts* opts, bpjd_problem** out) {
    bpjd_problem* p = nullptr;
    BPJD_TRY(plan_problem(ctx, K, M, dd, geom, opts, &p));
    const int rc = materialize_problem(p);
    if (rc < 0) {
        bpjd_problem_destroy(p);
        return rc;
    }
    *out = p;
    return BPJD_OK;
}

}  // namespace bpjd

extern "C" {

int bpjd_problem_create(bpjd_ctx* ctx, const bpjd_csr* K, const bpjd_csr* M, const bpjd_dd* dd,
                        const bpjd_opts* opts, bpjd_problem** out) {
    CtxScope cs_(ctx);
    if (!ctx || !K || !M || !dd || !opts || !out) return fail(BPJD_ERR_ARG, "NULL argument");
    return create_now(ctx, K, M, dd, nullptr, opts, out);
}

int bpjd_problem_create_geom(bpjd_ctx* ctx, const bpjd_csr* K, const bpjd_csr* M, const bpjd_dd_geom* g,
                             const bpjd_opts* opts, bpjd_problem** out) {
    CtxScope cs_(ctx);
    if (!ctx || !K || !M || !g || !opts || !out) return fail(BPJD_ERR_ARG, "NULL argument");
    return create_now(ctx, K, M, nullptr, g, opts, out);
}

void bpjd_problem_destroy(bpjd_problem* p) {
    if (!p) return;
    delete p->plan;
    for (auto& row : p->graph_exec)
        for (hipGraphExec_t ge : row)
            if (ge) (void)hipGraphExecDestroy(ge);
    // no kernel of this problem may still use a block handed back (an allocator or the
    // server's block may give it out again at once)
    if (!p->allocations.empty()) (void)hipStreamSynchronize(p->ctx->stream);
    for (const DevBlock& b : p->allocations) dev_free(p, b);
    if (p->ctx && p->ctx->arena)            // reserved blocks never handed out
        for (size_t q = p->reserved_next; q < p->reserved.size(); ++q)
            p->ctx->arena->release(p->reserved[q], p->reserved_bytes[q]);
    if (p->hbuf && p->own_hbuf) (void)hipHostFree(p->hbuf);
    delete p;
}

int bpjd_problem_set_values(bpjd_problem* p, const double* Kval, const double* Mval, int32_t mem) {
    CtxScope cs_(p ? p->ctx : nullptr);
    if (!p || !Kval || !Mval) return fail(BPJD_ERR_ARG, "NULL argument");
    std::vector<double> kv(p->nnzK), mv(p->nnzM);
    if (mem == BPJD_MEM_DEVICE) {
        BPJD_HIP(hipMemcpyAsync(kv.data(), Kval, sizeof(double) * p->nnzK, hipMemcpyDeviceToHost, p->ctx->stream));
        BPJD_HIP(hipMemcpyAsync(mv.data(), Mval, sizeof(double) * p->nnzM, hipMemcpyDeviceToHost, p->ctx->stream));
        BPJD_HIP(hipStreamSynchronize(p->ctx->stream));
    } else {
        std::memcpy(kv.data(), Kval, sizeof(double) * p->nnzK);
        std::memcpy(mv.data(), Mval, sizeof(double) * p->nnzM);
    }
    std::vector<double2> km(p->nnz, make_double2(0.0, 0.0));
    for (long long q = 0; q < p->nnzK; ++q) km[p->Kmap[q]].x = kv[q];
    for (long long q = 0; q < p->nnzM; ++q) km[p->Mmap[q]].y = mv[q];
    BPJD_HIP(hipMemcpyAsync(p->km, km.data(), sizeof(double2) * p->nnz, hipMemcpyHostToDevice, p->ctx->stream));
    BPJD_HIP(hipStreamSynchronize(p->ctx->stream));
    p->setup_done = false;
    return BPJD_OK;
}

int bpjd_problem_dims(const bpjd_problem* p, int32_t* n, int32_t* n_coarse, int32_t* n_sub, int32_t* s) {
    CtxScope cs_(p ? p->ctx : nullptr);
    if (!p) return fail(BPJD_ERR_ARG, "NULL problem");
    if (n) *n = p->n;
    if (n_coarse) *n_coarse = p->nH;
    if (n_sub) *n_sub = p->nsub;
    if (s) *s = p->s;
    return BPJD_OK;
}

int bpjd_problem_footprint(const bpjd_problem* p, uint64_t* bytes) {
    CtxScope cs_(p ? p->ctx : nullptr);
    if (!p || !bytes) return fail(BPJD_ERR_ARG, "NULL argument");
    *bytes = p->footprint;
    return BPJD_OK;
}

int bpjd_problem_local_sizes(const bpjd_problem* p, int32_t* n_l, int32_t* bw) {
    CtxScope cs_(p ? p->ctx : nullptr);
    if (!p || !n_l || !bw) return fail(BPJD_ERR_ARG, "NULL argument");
    for (int l = 0; l < p->nsub; ++l) {
        n_l[l] = p->h_nl[l];
        bw[l] = p->h_bw[l];
    }
    return BPJD_OK;
}

int bpjd_solve(bpjd_problem* p, double* eigvals, double* eigvecs, int32_t mem, bpjd_stats* st) {
    CtxScope cs_(p ? p->ctx : nullptr);
    if (!p) return fail(BPJD_ERR_ARG, "NULL problem");
    if (mem != BPJD_MEM_HOST && mem != BPJD_MEM_DEVICE) return fail(BPJD_ERR_ARG, "bad mem");
    return run_solve(p, eigvals, eigvecs, mem, st);
}

int bpjd_setup(bpjd_problem* p) {
    CtxScope cs_(p ? p->ctx : nullptr);
    if (!p) return fail(BPJD_ERR_ARG, "NULL problem");
    return run_setup(p);
}

int bpjd_apply_preconditioner(bpjd_problem* p, const double* X, const double* lambda, double* Z, int32_t mem) {
    CtxScope cs_(p ? p->ctx : nullptr);
    if (!p || !X || !lambda || !Z) return fail(BPJD_ERR_ARG, "NULL argument");
    if (!p->setup_done) return fail(BPJD_ERR_STATE, "call bpjd_setup first");
    hipStream_t st = p->ctx->stream;
    const int n = p->n, s = p->s, ld = s;
    const hipMemcpyKind kin = mem == BPJD_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    BPJD_HIP(hipMemcpyAsync(p->Z, X, sizeof(double) * n * s, kin, st));
    BPJD_HIP(hipMemcpyAsync(p->lam, lambda, sizeof(double) * s, kin, st));
    launch_copy_cols(st, n, s, p->Z, s, p->W[1], ld);
    launch_spmm_km(st, n, p->rowptr, p->col, p->km, p->W[1], ld, s, p->KW[1], ld, p->MW[1], ld, p->spmm_variant);
    BPJD_HIP(hipMemsetAsync(p->status, 0, sizeof(int), st));
    launch_residual(st, n, s, p->KW[1], ld, p->MW[1], ld, p->lam, p->F, s, p->partial, p->npart, p->colsq, nullptr,
                    p->status);
    apply_precond(p, p->F, p->Z, p->s, nullptr);
    const hipMemcpyKind kout = mem == BPJD_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    BPJD_HIP(hipMemcpyAsync(Z, p->Z, sizeof(double) * n * s, kout, st));
    BPJD_HIP(hipStreamSynchronize(st));
    return check_status(p);
}

int bpjd_spmm(bpjd_problem* p, const double* X, int32_t ncols, double* KX, double* MX, int32_t mem) {
    CtxScope cs_(p ? p->ctx : nullptr);
    if (!p || !X || !KX || !MX) return fail(BPJD_ERR_ARG, "NULL argument");
    if (ncols < 1 || ncols > 3 * p->s) return fail(BPJD_ERR_ARG, "ncols must be in [1, 3s]");
    hipStream_t st = p->ctx->stream;
    const size_t bytes = sizeof(double) * (size_t)p->n * ncols;
    const double* dX = X;
    if (mem == BPJD_MEM_HOST) {
        BPJD_HIP(hipMemcpyAsync(p->W[1], X, bytes, hipMemcpyHostToDevice, st));
        dX = p->W[1];
    }
    double* dK = mem == BPJD_MEM_HOST ? p->KW[1] : KX;
    double* dM = mem == BPJD_MEM_HOST ? p->MW[1] : MX;
    launch_spmm_km(st, p->n, p->rowptr, p->col, p->km, dX, ncols, ncols, dK, ncols, dM, ncols, p->spmm_variant);
    if (mem == BPJD_MEM_HOST) {
        BPJD_HIP(hipMemcpyAsync(KX, dK, bytes, hipMemcpyDeviceToHost, st));
        BPJD_HIP(hipMemcpyAsync(MX, dM, bytes, hipMemcpyDeviceToHost, st));
    }
    BPJD_HIP(hipStreamSynchronize(st));
    return BPJD_OK;
}

int bpjd_coarse_eigenvalues(bpjd_problem* p, double* lamH, int32_t mem) {
    CtxScope cs_(p ? p->ctx : nullptr);
    if (!p || !lamH) return fail(BPJD_ERR_ARG, "NULL argument");
    if (!p->setup_done) return fail(BPJD_ERR_STATE, "call bpjd_setup first");
    const hipMemcpyKind k = mem == BPJD_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    BPJD_HIP(hipMemcpyAsync(lamH, p->lamH, sizeof(double) * p->nH, k, p->ctx->stream));
    BPJD_HIP(hipStreamSynchronize(p->ctx->stream));
    return BPJD_OK;
}

const char* bpjd_strerror(int code) {
    switch (code) {
        case BPJD_OK: return "ok";
        case BPJD_PENDING: return "pending";
        case BPJD_ERR_ARG: return "invalid argument";
        case BPJD_ERR_CSR: return "malformed CSR matrix";
        case BPJD_ERR_DD: return "invalid domain decomposition";
        case BPJD_ERR_NOT_SPD: return "matrix not positive definite / breakdown";
        case BPJD_ERR_NOCONV: return "not converged";
        case BPJD_ERR_OOM: return "out of device memory";
        case BPJD_ERR_HIP: return "HIP runtime error";
        case BPJD_ERR_OVER_BUDGET: return "request exceeds the memory budget";
        case BPJD_ERR_STATE: return "invalid state";
        default: return "unknown error";
    }
}

const char* bpjd_last_error(const bpjd_ctx* ctx) {
    if (!ctx) return g_last_error.c_str();
    bpjd_ctx* c = const_cast<bpjd_ctx*>(ctx);
    std::lock_guard<std::mutex> g(c->err_mu);
    g_error_copy = c->last_error;
    return g_error_copy.c_str();
}

}  // extern "C"
