// Block linear algebra on n x c row-major FP64 blocks: fused SpMM with K and M,
// residual block, Gram products, tall-times-small products.  All reductions are
// two-pass with a fixed summation order, so results do not depend on timing.
#include <algorithm>
#include <cstdint>

#include "common.h"

namespace bpjd {

static inline int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// ---------------------------------------------------------------------------
// Fused SpMM on the union pattern: one thread per (row, column); the threads of
// a row read the same (col, K, M) triple and contiguous pieces of X rows.
__global__ void spmm_km_kernel(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                               const double2* __restrict__ km, const double* __restrict__ X, int ldx,
                               int ncols, int cshift, double* __restrict__ KX, int ldk,
                               double* __restrict__ MX, int ldm) {
    // a row is handled by a group of G = 2^cshift lanes (one per column of X).  Its
    // entries are taken 8 at a time (G at a time when G < 8): lane g of the group loads
    // entry g, the group shares them by lane shuffles, and then every lane loads the 8
    // X entries of its column, so each entry's index and value pair is fetched once per
    // row and not once per column.  Sums keep the entry order.
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = t >> cshift;
    const int G = 1 << cshift;
    const int c = t & (G - 1);
    const int gbase = (threadIdx.x & 63) & ~(G - 1);   // first lane of the row's group (G <= 64)
    const int CH = G < 8 ? G : 8;
    const int cc = min(c, ncols - 1);                  // lanes past the last column load in bounds
    int p0 = 0, p1 = 0;
    if (r < n) {
        p0 = rowptr[r];
        p1 = rowptr[r + 1];
    }
    double ak = 0.0, am = 0.0;
    for (int pb = p0; pb < p1; pb += CH) {             // same trip count for the whole group
        const int pg = min(pb + min(c, CH - 1), p1 - 1);
        const int cg = col[pg];
        const double2 vg = km[pg];
        int cj[8];
        double vk[8], vm[8], xj[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int src = gbase + (j < CH ? j : 0);
            cj[j] = __shfl(cg, src, 64);
            vk[j] = __shfl(vg.x, src, 64);
            vm[j] = __shfl(vg.y, src, 64);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) xj[j] = X[(long long)cj[j] * ldx + cc];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j < CH && pb + j < p1) {
                ak = fma(vk[j], xj[j], ak);
                am = fma(vm[j], xj[j], am);
            }
        }
    }
    if (r < n && c < ncols) {
        KX[(long long)r * ldk + c] = ak;
        MX[(long long)r * ldm + c] = am;
    }
}

// The same product for an even number of columns: a lane owns two adjacent columns
// (16-byte loads and stores), a row a group of G = 2^cshift lanes.  The row's entries
// are taken 8 at a time (2G when 2G < 8); lane g of the group loads entries g and g + G,
// the group shares them by lane shuffles.
__global__ void spmm_km_pair_kernel(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                                    const double2* __restrict__ km, const double* __restrict__ X, int ldx,
                                    int ncols, int cshift, double* __restrict__ KX, int ldk,
                                    double* __restrict__ MX, int ldm) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = t >> cshift;
    const int G = 1 << cshift;
    const int c = t & (G - 1);                         // columns 2c, 2c + 1
    const int gbase = (threadIdx.x & 63) & ~(G - 1);
    const int CH = 2 * G < 8 ? 2 * G : 8;
    const int cc = min(2 * c, ncols - 2);              // lanes past the last pair load in bounds
    int p0 = 0, p1 = 0;
    if (r < n) {
        p0 = rowptr[r];
        p1 = rowptr[r + 1];
    }
    double ak0 = 0.0, ak1 = 0.0, am0 = 0.0, am1 = 0.0;
    for (int pb = p0; pb < p1; pb += CH) {             // same trip count for the whole group
        const int pa = min(pb + min(c, CH - 1), p1 - 1);
        const int pc = min(pb + min(c + G, CH - 1), p1 - 1);
        const int ca = col[pa], cb = col[pc];
        const double2 va = km[pa], vb = km[pc];
        int cj[8];
        double vk[8], vm[8];
        double2 xj[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int jj = j < CH ? j : 0;
            if (jj < G) {                              // uniform: G is the same for every lane
                cj[j] = __shfl(ca, gbase + jj, 64);
                vk[j] = __shfl(va.x, gbase + jj, 64);
                vm[j] = __shfl(va.y, gbase + jj, 64);
            } else {
                cj[j] = __shfl(cb, gbase + jj - G, 64);
                vk[j] = __shfl(vb.x, gbase + jj - G, 64);
                vm[j] = __shfl(vb.y, gbase + jj - G, 64);
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) xj[j] = *reinterpret_cast<const double2*>(X + (long long)cj[j] * ldx + cc);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j < CH && pb + j < p1) {
                ak0 = fma(vk[j], xj[j].x, ak0);
                ak1 = fma(vk[j], xj[j].y, ak1);
                am0 = fma(vm[j], xj[j].x, am0);
                am1 = fma(vm[j], xj[j].y, am1);
            }
        }
    }
    if (r < n && 2 * c < ncols) {
        *reinterpret_cast<double2*>(KX + (long long)r * ldk + 2 * c) = make_double2(ak0, ak1);
        *reinterpret_cast<double2*>(MX + (long long)r * ldm + 2 * c) = make_double2(am0, am1);
    }
}

// The same product with one lane per (row, column), lanes numbered row by row
// (t = r * ncols + c), so no lane idles for a column count that is not a power of two and
// the stores of a wave are one contiguous run when ldk = ldm = ncols.  A wavefront stages
// the index and value pairs of its rows in LDS, 64 entries at a time with one coalesced
// load per array, and every lane reads its row's entries from there (the lanes of a row
// read the same address).  Sums keep the entry order.
__global__ __launch_bounds__(256) void spmm_km_flat_kernel(int n, const int* __restrict__ rowptr,
                                                           const int* __restrict__ col,
                                                           const double2* __restrict__ km,
                                                           const double* __restrict__ X, int ldx, int ncols,
                                                           double* __restrict__ KX, int ldk,
                                                           double* __restrict__ MX, int ldm) {
    __shared__ int scol[4][64];
    __shared__ double2 skm[4][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // 32-bit lane numbers (n * ncols < 2^32 is checked at launch): a 64-bit division
    // would be most of this kernel's instructions
    const unsigned t0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
    const unsigned t = t0 + lane;
    const unsigned nc = (unsigned)ncols;
    const int rfirst = (int)(t0 / nc);
    if (rfirst >= n) return;                           // the whole wavefront (t0 is shared)
    const unsigned tl = (t0 + 63) / nc;
    const int rlast = (int)(tl < (unsigned)(n - 1) ? tl : (unsigned)(n - 1));
    const int r = (int)(t / nc);
    const int c = (int)(t - (unsigned)r * nc);
    const bool active = r < n;
    const int rr = active ? r : rlast;
    const int p0 = rowptr[rr], p1 = active ? rowptr[rr + 1] : p0;
    const int e0 = rowptr[rfirst], e1 = rowptr[rlast + 1];
    double ak = 0.0, am = 0.0;
    for (int cb = e0; cb < e1; cb += 64) {
        const int e = min(cb + lane, e1 - 1);          // in bounds; entries past e1 are never read
        scol[wv][lane] = col[e];
        skm[wv][lane] = km[e];
        __builtin_amdgcn_wave_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const int q0 = max(p0, cb), q1 = min(p1, cb + 64);   // this lane's entries in the chunk
        for (int qb = q0; qb < q1; qb += 8) {
            int cj[8];
            double2 v[8];
            double xj[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int o = min(qb + j, q1 - 1) - cb;
                cj[j] = scol[wv][o];
                v[j] = skm[wv][o];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) xj[j] = X[(long long)cj[j] * ldx + c];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (qb + j < q1) {
                    ak = fma(v[j].x, xj[j], ak);
                    am = fma(v[j].y, xj[j], am);
                }
            }
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_wave_barrier();
    }
    if (active) {
        KX[(long long)r * ldk + c] = ak;
        MX[(long long)r * ldm + c] = am;
    }
}

void launch_spmm_km(hipStream_t st, int n, const int* rowptr, const int* col, const double2* km,
                    const double* X, int ldx, int ncols, double* KX, int ldk, double* MX, int ldm, int variant) {
    // column pairs need even column counts and leading dimensions and 16-byte aligned
    // blocks (every block of the library is a hipMalloc base plus multiples of 16 bytes);
    // variant 1 keeps one column per lane in a power-of-two group per row, variant 2 one
    // lane per (row, column).  All forms add a row's entries in the same order.
    if (variant == 2 && (long long)n * ncols < (1LL << 32) - 256) {
        const long long work = (long long)n * ncols;
        hipLaunchKernelGGL(spmm_km_flat_kernel, dim3(grid_for(work, 256)), dim3(256), 0, st, n, rowptr, col, km, X,
                           ldx, ncols, KX, ldk, MX, ldm);
        return;
    }
    const bool pair = variant == 0 && (ncols % 2 == 0) && (ldx % 2 == 0) && (ldk % 2 == 0) && (ldm % 2 == 0) &&
                      ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(KX) |
                        reinterpret_cast<uintptr_t>(MX)) % 16 == 0);
    const int lanes = pair ? ncols / 2 : ncols;
    const int cp = pow2_at_least(lanes);
    int sh = 0;
    while ((1 << sh) < cp) ++sh;
    const long long work = (long long)n << sh;
    if (pair)
        hipLaunchKernelGGL(spmm_km_pair_kernel, dim3(grid_for(work, 256)), dim3(256), 0, st, n, rowptr, col, km, X,
                           ldx, ncols, sh, KX, ldk, MX, ldm);
    else
        hipLaunchKernelGGL(spmm_km_kernel, dim3(grid_for(work, 256)), dim3(256), 0, st, n, rowptr, col, km, X, ldx,
                           ncols, sh, KX, ldk, MX, ldm);
}

// ---------------------------------------------------------------------------
__global__ void csr_dense_kernel(int rows, const int* __restrict__ ptr, const int* __restrict__ col,
                                 const double* __restrict__ val, const double* __restrict__ B, int ldb,
                                 int ncols, int cshift, double* __restrict__ Y, int ldy, int accumulate) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = t >> cshift;
    const int c = t & ((1 << cshift) - 1);
    if (r >= rows || c >= ncols) return;
    double acc = 0.0;
    for (int p = ptr[r]; p < ptr[r + 1]; ++p) acc = fma(val[p], B[(long long)col[p] * ldb + c], acc);
    double* y = Y + (long long)r * ldy + c;
    *y = accumulate ? (*y + acc) : acc;
}

void launch_csr_dense(hipStream_t st, int rows, const int* ptr, const int* col, const double* val,
                      const double* B, int ldb, int ncols, double* Y, int ldy, bool accumulate) {
    const int cp = pow2_at_least(ncols);
    int sh = 0;
    while ((1 << sh) < cp) ++sh;
    const long long work = (long long)rows << sh;
    hipLaunchKernelGGL(csr_dense_kernel, dim3(grid_for(work, 256)), dim3(256), 0, st, rows, ptr, col, val, B, ldb,
                       ncols, sh, Y, ldy, accumulate ? 1 : 0);
}

// ---------------------------------------------------------------------------
int num_partials(int n) {
    int p = (n + 255) / 256;
    if (p < 1) p = 1;
    if (p > 2048) p = 2048;
    return p;
}

// out[o] = sum_p partial[o][p] for a [len][npart] array of partials: one
// workgroup per output, strided per-thread sums and a fixed tree (deterministic).
__global__ void reduce_partials_kernel(int npart, int len, const double* __restrict__ partial,
                                       double* __restrict__ out) {
    __shared__ double red[256];
    const int o = blockIdx.x;
    const int t = threadIdx.x;
    const double* src = partial + (long long)o * npart;
    double acc = 0.0;
    for (int p = t; p < npart; p += 256) acc += src[p];
    red[t] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (t < k) red[t] += red[t + k];
        __syncthreads();
    }
    if (t == 0) out[o] = red[0];
}

static void launch_reduce(hipStream_t st, int npart, int len, const double* partial, double* out) {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(len), dim3(256), 0, st, npart, len, partial, out);
}

// Residual block and column sums of squares.  Thread t works on column t % s
// for rows (t / s) + k * (threads / s) of the block's row range, then a tree
// reduction over the row slots gives one partial per column and block.
__global__ void residual_kernel(int n, int s, const double* __restrict__ KX, int ldk,
                                const double* __restrict__ MX, int ldm, const double* __restrict__ lam,
                                double* __restrict__ F, int ldf, int chunk, double* __restrict__ partial,
                                double* __restrict__ aux, const int* __restrict__ status) {
    __shared__ double red[2][256];
    const int t = threadIdx.x;
    // the shifts and the status word travel to the host with the column norms
    if (aux != nullptr && blockIdx.x == 0) {
        if (t < s) aux[t] = lam[t];
        if (t == 0) *reinterpret_cast<int*>(aux + 64) = *status;
    }
    const int slots = blockDim.x / s;
    const int c = t % s;
    const int rs = t / s;
    const int r0 = blockIdx.x * chunk;
    const int r1 = min(n, r0 + chunk);
    double sf = 0.0, sm = 0.0;
    if (rs < slots) {
        const double lc = lam[c];
        for (int r = r0 + rs; r < r1; r += slots) {
            const double m = MX[(long long)r * ldm + c];
            const double f = m * lc - KX[(long long)r * ldk + c];
            F[(long long)r * ldf + c] = f;
            sf = fma(f, f, sf);
            sm = fma(m, m, sm);
        }
    }
    red[0][t] = (rs < slots) ? sf : 0.0;
    red[1][t] = (rs < slots) ? sm : 0.0;
    __syncthreads();
    if (t < s) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < slots; ++k) {
            a += red[0][k * s + t];
            b += red[1][k * s + t];
        }
        partial[(long long)t * gridDim.x + blockIdx.x] = a;
        partial[(long long)(s + t) * gridDim.x + blockIdx.x] = b;
    }
}

void launch_residual(hipStream_t st, int n, int s, const double* KX, int ldk, const double* MX, int ldm,
                     const double* lam, double* F, int ldf, double* partial, int npart, double* colsq, double* aux,
                     const int* status) {
    const int chunk = (n + npart - 1) / npart;
    hipLaunchKernelGGL(residual_kernel, dim3(npart), dim3(256), 0, st, n, s, KX, ldk, MX, ldm, lam, F, ldf, chunk,
                       partial, aux, status);
    launch_reduce(st, npart, 2 * s, partial, colsq);
}

// ---------------------------------------------------------------------------
// Gram product C = A^T B (a, b <= 64) with FP64 16x16x4 MFMAs: the rows are the
// contraction index.  A workgroup of four wavefronts per chunk of rows: wavefront w
// takes the k-steps of 4 rows numbered w, w + 4, ... and keeps U of them in flight; for
// a k-step, lane l supplies A[r + l/16][16 tp + l%16] and B[r + l/16][16 tq + l%16]
// straight from the row-major blocks.  The four accumulators are added in LDS in a
// fixed order, one partial per workgroup ([a*b][npart]), and the partials are reduced
// in a second pass in a fixed order.
typedef double dx4_t __attribute__((ext_vector_type(4)));

template <int TA, int TB>
__global__ __launch_bounds__(256) void gram_mfma_kernel(int n, int a, int b, const double* __restrict__ A,
                                                        const double* __restrict__ B, BlockGeom g, int chunk,
                                                        double* __restrict__ partial) {
    __shared__ double red[3][TA * TB * 4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    long long oa[TA], ob[TB];                   // column offsets of this lane's elements
#pragma unroll
    for (int p = 0; p < TA; ++p) oa[p] = g.col_offset(16 * p + lr);
#pragma unroll
    for (int q = 0; q < TB; ++q) ob[q] = g.col_offset(16 * q + lr);
    const int r0 = blockIdx.x * chunk;
    const int r1 = min(n, r0 + chunk);
    dx4_t acc[TA][TB];
#pragma unroll
    for (int p = 0; p < TA; ++p)
#pragma unroll
        for (int q = 0; q < TB; ++q) acc[p][q] = dx4_t{0.0, 0.0, 0.0, 0.0};
    constexpr int U = 4;                        // k-steps whose loads are in flight together
    for (int r = r0 + 4 * w; r < r1; r += 16 * U) {
        double av[U][TA], bv[U][TB];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int rr = r + 16 * u + lk;
            const bool rok = rr < r1;
#pragma unroll
            for (int p = 0; p < TA; ++p) {
                const int c = 16 * p + lr;
                av[u][p] = (rok && c < a) ? A[oa[p] + (long long)rr * g.ld] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < TB; ++q) {
                const int c = 16 * q + lr;
                bv[u][q] = (rok && c < b) ? B[ob[q] + (long long)rr * g.ld] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int p = 0; p < TA; ++p)
#pragma unroll
                for (int q = 0; q < TB; ++q)
                    acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][p], bv[u][q], acc[p][q], 0, 0, 0);
    }
    if (w > 0) {
#pragma unroll
        for (int p = 0; p < TA; ++p)
#pragma unroll
            for (int q = 0; q < TB; ++q)
#pragma unroll
                for (int i = 0; i < 4; ++i) red[w - 1][(p * TB + q) * 4 + i][lane] = acc[p][q][i];
    }
    __syncthreads();
    if (w != 0) return;
    // FP64 accumulator element i of lane l: row l/16 + 4 i, column l%16 of the 16x16 tile
#pragma unroll
    for (int p = 0; p < TA; ++p)
#pragma unroll
        for (int q = 0; q < TB; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = (p * TB + q) * 4 + i;
                const double v = ((acc[p][q][i] + red[0][e][lane]) + red[1][e][lane]) + red[2][e][lane];
                const int row = 16 * p + lk + 4 * i, col = 16 * q + lr;
                if (row < a && col < b) partial[(long long)(row * b + col) * gridDim.x + blockIdx.x] = v;
            }
}

// The same Gram product for the blocked layout with whole runs (ld = bw, a and b multiples
// of bw, 16-byte aligned block bases, bs even): the workgroup's chunk is taken in
// sub-tiles of gr rows whose runs of A and B are copied into LDS by direct
// global-to-LDS loads (16 bytes per lane), double-buffered: the copy of sub-tile i + 1 is
// in flight while sub-tile i is multiplied.  Wavefront w takes k-steps w, w + 4, ... of
// each sub-tile.  The sub-tile height gr (64, 48 or 32 rows) is the largest whose two
// buffers fit in 64 KB: each wait covers one round trip, so the bytes in flight per
// workgroup set the bandwidth (32-row sub-tiles of 26 to 39 columns fell short of it).
constexpr int GM_ROWS_MAX = 64;

// direct global-to-LDS copies: lane l's 16 (4) bytes at g land at l + 16 (4) * lane bytes,
// l the same for the whole wavefront; completion is counted by vmcnt
__device__ inline void lds_dma16(const double* g, double* l) {
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(g),
                                     (__attribute__((address_space(3))) void*)(l), 16, 0, 0);
}
__device__ inline void lds_dma4(const unsigned* g, unsigned* l) {
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(g),
                                     (__attribute__((address_space(3))) void*)(l), 4, 0, 0);
}

__device__ inline void lds_copy_runs(const double* src, long long bs, long long goff, int cnt, double* dst,
                                     int runl, int nrun, int w, int lane, int t) {
    const int npair = cnt >> 1;
    const int nch = (npair + 63) >> 6;
    for (int j = w; j < nrun * nch; j += 4) {
        const int jb = j / nch, ch = j - jb * nch;
        const int e2 = 64 * ch + lane;
        if (e2 < npair) lds_dma16(src + jb * bs + goff + 2 * e2, dst + jb * runl + 128 * ch);
    }
    if (cnt & 1)
        for (int jb = t; jb < nrun; jb += 256) dst[jb * runl + cnt - 1] = src[jb * bs + goff + cnt - 1];
}

template <int TA, int TB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TA * TB >= 16 ? 2 : 3))) void gram_flat_kernel(
    int n, int a, int b, const double* __restrict__ A,
                                                        const double* __restrict__ B, int bw, long long bs,
                                                        int chunk, int gr, double* __restrict__ partial) {
    extern __shared__ __align__(16) double gm_smem[];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63, lr = lane & 15, lk = lane >> 4;
    const int runl = gr * bw;
    const int nra = a / bw, nrb = b / bw;
    const int bufsz = gr * (a + b);       // one sub-tile: A's runs, then B's
    const int r0 = blockIdx.x * chunk;
    const int r1 = min(n, r0 + chunk);
    const int nst = (r1 - r0 + gr - 1) / gr;
    // LDS offsets of this lane's columns within a sub-tile (-1: past a or b)
    int oa[TA], ob[TB];
#pragma unroll
    for (int p = 0; p < TA; ++p) {
        const int c = 16 * p + lr, jb = c / bw;
        oa[p] = (c < a) ? jb * runl + (c - jb * bw) : -1;
    }
#pragma unroll
    for (int q = 0; q < TB; ++q) {
        const int c = 16 * q + lr, jb = c / bw;
        ob[q] = (c < b) ? gr * a + jb * runl + (c - jb * bw) : -1;
    }
    auto fetch = [&](int i) {
        const int rs = r0 + gr * i;
        const int cnt = min(gr, r1 - rs) * bw;
        double* buf = gm_smem + (i & 1) * bufsz;
        lds_copy_runs(A, bs, (long long)rs * bw, cnt, buf, runl, nra, w, lane, t);
        lds_copy_runs(B, bs, (long long)rs * bw, cnt, buf + gr * a, runl, nrb, w, lane, t);
    };
    dx4_t acc[TA][TB];
#pragma unroll
    for (int p = 0; p < TA; ++p)
#pragma unroll
        for (int q = 0; q < TB; ++q) acc[p][q] = dx4_t{0.0, 0.0, 0.0, 0.0};
    if (nst > 0) fetch(0);
    for (int i = 0; i < nst; ++i) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();                       // sub-tile i is in; sub-tile i - 1's buffer is free
        if (i + 1 < nst) fetch(i + 1);
        const double* buf = gm_smem + (i & 1) * bufsz;
        const int rows = min(gr, r1 - (r0 + gr * i));
        for (int h = 0; h < (gr >> 4); ++h) {
            const int row = 4 * (w + 4 * h) + lk;
            const bool rok = row < rows;
            double av[TA], bv[TB];
#pragma unroll
            for (int p = 0; p < TA; ++p) av[p] = (rok && oa[p] >= 0) ? buf[oa[p] + row * bw] : 0.0;
#pragma unroll
            for (int q = 0; q < TB; ++q) bv[q] = (rok && ob[q] >= 0) ? buf[ob[q] + row * bw] : 0.0;
#pragma unroll
            for (int p = 0; p < TA; ++p)
#pragma unroll
                for (int q = 0; q < TB; ++q)
                    acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
        }
    }
    // wavefronts 1..3 hand their accumulators over in two rounds (LDS of the sub-tile
    // buffers); wavefront 0 adds them in the order 1, 2, 3
    constexpr int NE = TA * TB * 4;
    double* red = gm_smem;                     // [2][NE][64]
    __syncthreads();                           // every sub-tile read is done
    if (w == 1 || w == 2) {
#pragma unroll
        for (int p = 0; p < TA; ++p)
#pragma unroll
            for (int q = 0; q < TB; ++q)
#pragma unroll
                for (int i = 0; i < 4; ++i) red[((w - 1) * NE + (p * TB + q) * 4 + i) * 64 + lane] = acc[p][q][i];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int p = 0; p < TA; ++p)
#pragma unroll
            for (int q = 0; q < TB; ++q)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = (p * TB + q) * 4 + i;
                    acc[p][q][i] = (acc[p][q][i] + red[e * 64 + lane]) + red[(NE + e) * 64 + lane];
                }
    }
    __syncthreads();
    if (w == 3) {
#pragma unroll
        for (int p = 0; p < TA; ++p)
#pragma unroll
            for (int q = 0; q < TB; ++q)
#pragma unroll
                for (int i = 0; i < 4; ++i) red[((p * TB + q) * 4 + i) * 64 + lane] = acc[p][q][i];
    }
    __syncthreads();
    if (w != 0) return;
    // FP64 accumulator element i of lane l: row l/16 + 4 i, column l%16 of the 16x16 tile
#pragma unroll
    for (int p = 0; p < TA; ++p)
#pragma unroll
        for (int q = 0; q < TB; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = (p * TB + q) * 4 + i;
                const double v = acc[p][q][i] + red[e * 64 + lane];
                const int row = 16 * p + lk + 4 * i, col = 16 * q + lr;
                if (row < a && col < b) partial[(long long)(row * b + col) * gridDim.x + blockIdx.x] = v;
            }
}

// Workgroups of `kernel` resident at once on the current device (0 if unknown).
template <typename K>
static int resident_blocks(K kernel, size_t smem) {
    int dev = 0, cu = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, smem) != hipSuccess) return 0;
    return nb * cu;
}

// The flat Gram's rows are split into as many chunks as workgroups fit on the device at
// once (at most npart; whole sub-tiles per chunk): every chunk then runs in the first
// and only round, with no tail round of a few long workgroups.  Returns the grid.
template <int TA, int TB>
static int gram_flat_launch(hipStream_t st, size_t smem, int gr, int n, int a, int b, const double* A,
                            const double* B, int bw, long long bs, int npart, double* partial) {
    auto kernel = gram_flat_kernel<TA, TB>;
    int groups = resident_blocks(kernel, smem);
    groups = (groups <= 0) ? npart : std::min(groups, npart);
    const int chunk = (((n + groups - 1) / groups) + gr - 1) / gr * gr;
    const int grid = std::max(1, (n + chunk - 1) / chunk);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(256), smem, st, n, a, b, A, B, bw, bs, chunk, gr, partial);
    return grid;
}

template <int TA>
static int gram_flat_dispatch_b(hipStream_t st, int TB, size_t smem, int gr, int n, int a, int b, const double* A,
                                const double* B, int bw, long long bs, int npart, double* partial) {
    switch (TB) {
        case 1: return gram_flat_launch<TA, 1>(st, smem, gr, n, a, b, A, B, bw, bs, npart, partial);
        case 2: return gram_flat_launch<TA, 2>(st, smem, gr, n, a, b, A, B, bw, bs, npart, partial);
        case 3: return gram_flat_launch<TA, 3>(st, smem, gr, n, a, b, A, B, bw, bs, npart, partial);
        default: return gram_flat_launch<TA, 4>(st, smem, gr, n, a, b, A, B, bw, bs, npart, partial);
    }
}

template <int TA>
static void gram_dispatch_b(hipStream_t st, int TB, int grid, int n, int a, int b, const double* A,
                            const double* B, BlockGeom g, int chunk, double* partial) {
    switch (TB) {
        case 1: hipLaunchKernelGGL((gram_mfma_kernel<TA, 1>), dim3(grid), dim3(256), 0, st, n, a, b, A, B, g, chunk, partial); break;
        case 2: hipLaunchKernelGGL((gram_mfma_kernel<TA, 2>), dim3(grid), dim3(256), 0, st, n, a, b, A, B, g, chunk, partial); break;
        case 3: hipLaunchKernelGGL((gram_mfma_kernel<TA, 3>), dim3(grid), dim3(256), 0, st, n, a, b, A, B, g, chunk, partial); break;
        default: hipLaunchKernelGGL((gram_mfma_kernel<TA, 4>), dim3(grid), dim3(256), 0, st, n, a, b, A, B, g, chunk, partial); break;
    }
}

void launch_gram(hipStream_t st, int n, int a, int b, const double* A, const double* B, BlockGeom g,
                 double* partial, int npart, double* C) {
    // at least 64 rows per workgroup (one k-step per wavefront and in-flight slot), at
    // most npart workgroups
    int chunk = 64;
    while ((n + chunk - 1) / chunk > npart) chunk *= 2;
    const int grid = (n + chunk - 1) / chunk;
    const int TA = (a + 15) / 16, TB = (b + 15) / 16;
    // the flat form: whole runs of the blocked layout, 16-byte aligned; LDS for two
    // sub-tiles, or for the accumulator hand-over when that is larger
    int gr = GM_ROWS_MAX;                      // sub-tile rows: two sub-tiles within 64 KB
    while (gr > 32 && 2 * (size_t)gr * (a + b) * sizeof(double) > 65536) gr -= 16;
    const size_t smem = sizeof(double) * std::max<size_t>(2 * (size_t)gr * (a + b), 2 * (size_t)TA * TB * 256);
    if (g.ld == g.bw && g.bw >= 1 && a % g.bw == 0 && b % g.bw == 0 && g.bs % 2 == 0 && smem <= 65536 &&
        ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0) {
        int fgrid;
        switch (TA) {
            case 1: fgrid = gram_flat_dispatch_b<1>(st, TB, smem, gr, n, a, b, A, B, g.bw, g.bs, npart, partial); break;
            case 2: fgrid = gram_flat_dispatch_b<2>(st, TB, smem, gr, n, a, b, A, B, g.bw, g.bs, npart, partial); break;
            case 3: fgrid = gram_flat_dispatch_b<3>(st, TB, smem, gr, n, a, b, A, B, g.bw, g.bs, npart, partial); break;
            default: fgrid = gram_flat_dispatch_b<4>(st, TB, smem, gr, n, a, b, A, B, g.bw, g.bs, npart, partial); break;
        }
        launch_reduce(st, fgrid, a * b, partial, C);
        return;
    }
    switch (TA) {
        case 1: gram_dispatch_b<1>(st, TB, grid, n, a, b, A, B, g, chunk, partial); break;
        case 2: gram_dispatch_b<2>(st, TB, grid, n, a, b, A, B, g, chunk, partial); break;
        case 3: gram_dispatch_b<3>(st, TB, grid, n, a, b, A, B, g, chunk, partial); break;
        default: gram_dispatch_b<4>(st, TB, grid, n, a, b, A, B, g, chunk, partial); break;
    }
    launch_reduce(st, grid, a * b, partial, C);
}

// ---------------------------------------------------------------------------
// Tall-times-small products Y = beta Y + alpha A C (a, b <= 64): a block
// stages 64 rows of A and the coefficients in LDS with coalesced loads, forms
// the 64 x b result in LDS and writes it back row-contiguously.  Up to three
// (A, Y) pairs share one launch (blockIdx.y); with A == Y (in-place Y = Y C)
// every row is read before any is written.
struct Triple {
    const double* A[3];
    double* Y[3];
};

constexpr int GR_ROWS = 64;
constexpr int GR_MAXC = 64;

// Dynamic LDS: the block's A rows (GR_ROWS x (a + 1), padded against bank conflicts)
// and C (a x b, zero-padded to whole k-steps and column tiles).  With the blocked
// layout (row-major n x bw blocks, a and b multiples of bw: every use here), the
// block's rows of each n x bw block form one contiguous run of GR_ROWS * bw values:
// it is read and written as a flat array with 16-byte accesses (consecutive threads
// on consecutive addresses) and placed in, or taken from, LDS by (row, column).
// Otherwise each column is read by strided loads.  The product is formed with FP64
// 16x16x4 MFMAs: wavefront w takes rows 16 w .. 16 w + 15 of the block and every
// 16-column tile of the result; for a k-step, lane l supplies A[16 w + l % 16][k0 + l / 16]
// and C[k0 + l / 16][16 q + l % 16] from LDS.  Each output is one fixed-order sum over k
// (the k-steps in order, four products per step as the MFMA adds them), so the result
// does not depend on the launch.  With A == Y (in place) every row of the block is read
// before any is written.
__global__ __launch_bounds__(256) void gemm_rows_kernel(int n, int a, int b, double alpha, Triple T, BlockGeom g,
                                                        const double* __restrict__ C, double beta, int flat) {
    extern __shared__ double gr_smem[];
    const int ak = (a + 3) & ~3;               // k padded to whole k-steps
    const int bq = (b + 15) & ~15;             // columns padded to whole tiles
    const int ap = ak + 1;
    double* sA = gr_smem;                      // [GR_ROWS][ak + 1]; later the result [GR_ROWS][bq + 1]
    double* sC = gr_smem + GR_ROWS * (ap > bq + 1 ? ap : bq + 1);   // [ak][bq]
    const int t = threadIdx.x;
    const int r0 = blockIdx.x * GR_ROWS;
    const int rows = min(GR_ROWS, n - r0);
    const double* A = T.A[blockIdx.y];
    double* Y = T.Y[blockIdx.y];
    // Index arithmetic: a thread's (row, column) positions advance by fixed strides, so
    // each takes one division up front (a division per element was most of the
    // instructions of this memory-bound kernel).
    {
        int k = t / bq, q = t - k * bq;                    // element t of C (ak x bq)
        const int dk = 256 / bq, dq = 256 - dk * bq;
        for (int e = t; e < ak * bq; e += 256) {
            sC[e] = (k < a && q < b) ? C[k * b + q] : 0.0;
            k += dk;
            q += dq;
            if (q >= bq) {
                q -= bq;
                ++k;
            }
        }
    }
    if (ak > a)                                            // k padding: at most three columns
        for (int e = t; e < GR_ROWS * 4; e += 256)
            if ((e & 3) < ak - a) sA[(e >> 2) * ap + a + (e & 3)] = 0.0;
    if (rows < GR_ROWS)
        for (int e = t; e < (GR_ROWS - rows) * a; e += 256) sA[(rows + e / a) * ap + e % a] = 0.0;
    const int bw = g.bw;
    // pair e2 = t + 256 i of a run starts at element 2 e2: row and column, and the stride
    const int row_t = (2 * t) / bw, col_t = 2 * t - row_t * bw;
    const int drow = 512 / bw, dcol = 512 - drow * bw;
    if (flat) {
        const int cnt = rows * bw;             // values of one block's run (odd only in the last block)
        const int nrun = a / bw;
        for (int jb = 0; jb < nrun; ++jb) {
            const double* run = A + jb * g.bs + (long long)r0 * bw;
            const double2* src = reinterpret_cast<const double2*>(run);
            int row = row_t, col = col_t;
            for (int e2 = t; 2 * e2 + 1 < cnt; e2 += 256) {
                const double2 v = src[e2];
                sA[row * ap + jb * bw + col] = v.x;
                if (col + 1 < bw) sA[row * ap + jb * bw + col + 1] = v.y;
                else sA[(row + 1) * ap + jb * bw] = v.y;
                row += drow;
                col += dcol;
                if (col >= bw) {
                    col -= bw;
                    ++row;
                }
            }
            if ((cnt & 1) && t == 0) sA[(rows - 1) * ap + jb * bw + bw - 1] = run[cnt - 1];
        }
    } else {
        const int rpp = 256 / a;               // rows per pass of the load
        const int p = t % a, rr0 = t / a;
        const long long op = g.col_offset(p);
        if (rr0 < rpp) {
            for (int rr = rr0; rr < rows; rr += rpp) sA[rr * ap + p] = A[op + (long long)(r0 + rr) * g.ld];
        }
    }
    __syncthreads();
    const int w = t >> 6, lane = t & 63, lr = lane & 15, lk = lane >> 4;
    const double* arow = sA + (16 * w + lr) * ap + lk;
    dx4_t acc[GR_MAXC / 16];
#pragma unroll
    for (int qt = 0; qt < GR_MAXC / 16; ++qt) {
        acc[qt] = dx4_t{0.0, 0.0, 0.0, 0.0};
        if (16 * qt < bq) {
            const double* ccol = sC + lk * bq + 16 * qt + lr;
            for (int k0 = 0; k0 < ak; k0 += 4)
                acc[qt] = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[k0], ccol[k0 * bq], acc[qt], 0, 0, 0);
        }
    }
    __syncthreads();                           // every MFMA operand has been read
    // the result through LDS: element i of lane l is row l / 16 + 4 i, column l % 16 of
    // a tile
    const int yp = bq + 1;
#pragma unroll
    for (int qt = 0; qt < GR_MAXC / 16; ++qt)
        if (16 * qt < bq)
#pragma unroll
            for (int i = 0; i < 4; ++i) sA[(16 * w + lk + 4 * i) * yp + 16 * qt + lr] = acc[qt][i];
    __syncthreads();
    if (flat) {
        const int cnt = rows * bw;
        const int nrun = b / bw;
        for (int jb = 0; jb < nrun; ++jb) {
            double* run = Y + jb * g.bs + (long long)r0 * bw;
            double2* dst = reinterpret_cast<double2*>(run);
            if ((cnt & 1) && t == 0) {
                const double v = sA[(rows - 1) * yp + jb * bw + bw - 1];
                run[cnt - 1] = (beta == 0.0) ? alpha * v : fma(beta, run[cnt - 1], alpha * v);
            }
            int row = row_t, col = col_t;
            for (int e2 = t; 2 * e2 + 1 < cnt; e2 += 256) {
                const double v0 = sA[row * yp + jb * bw + col];
                const double v1 = (col + 1 < bw) ? sA[row * yp + jb * bw + col + 1] : sA[(row + 1) * yp + jb * bw];
                double2 o;
                if (beta == 0.0) {
                    o = make_double2(alpha * v0, alpha * v1);
                } else {
                    const double2 old = dst[e2];
                    o = make_double2(fma(beta, old.x, alpha * v0), fma(beta, old.y, alpha * v1));
                }
                dst[e2] = o;
                row += drow;
                col += dcol;
                if (col >= bw) {
                    col -= bw;
                    ++row;
                }
            }
        }
    } else {
        for (int e = t; e < rows * b; e += 256) {
            const int row = e / b, q = e - row * b;
            double* y = Y + g.col_offset(q) + (long long)(r0 + row) * g.ld;
            const double v = sA[row * yp + q];
            *y = (beta == 0.0) ? alpha * v : fma(beta, *y, alpha * v);
        }
    }
}

// The same product for the blocked layout with whole runs (ld = bw >= 4, a and b
// multiples of bw, 16-byte aligned block bases, bs even): a block's rows of each n x bw
// block of A (and of Y when beta != 0) form one contiguous run of GR_ROWS * bw values,
// copied into LDS as it lies in memory by direct global-to-LDS loads of 16 bytes per lane
// (C too, or 4 bytes per lane when C is only 8-byte aligned), every load of the tile
// issued before the first is waited for.  The MFMAs read the
// runs in place (lane l's column k lies in run k / bw at column k % bw, advanced by four
// per k-step), in the same k-order as gemm_rows_kernel, so both give identical results.
// The result is laid out as Y's runs in LDS (over A's) and written with 16-byte stores.

__global__ __launch_bounds__(256) void gemm_flat_kernel(int n, int a, int b, double alpha, Triple T, int bw,
                                                        long long bs, const double* __restrict__ C, double beta) {
    extern __shared__ __align__(16) double gf_smem[];
    const int runl = GR_ROWS * bw;             // LDS stride of the runs
    const int nra = a / bw, nrb = b / bw;
    double* sA = gf_smem;                      // A's runs, then Y's
    double* sO = sA + GR_ROWS * max(a, b);     // old Y's runs (beta != 0)
    double* sC = sO + (beta != 0.0 ? GR_ROWS * b : 0);   // C, a x b row-major
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int r0 = blockIdx.x * GR_ROWS;
    const int rows = min(GR_ROWS, n - r0);
    const int cnt = rows * bw;                 // values per run (odd only in the last block)
    const int npair = cnt >> 1;
    const int nch = (npair + 63) >> 6;         // 64-pair chunks per run
    const double* A = T.A[blockIdx.y];
    double* Y = T.Y[blockIdx.y];
    const long long goff = (long long)r0 * bw;
    // wave w copies chunks w, w + 4, ... of the runs; the odd last value by a plain load
    auto copy_runs = [&](const double* src, double* dst, int nrun) {
        for (int j = w; j < nrun * nch; j += 4) {
            const int jb = j / nch, ch = j - jb * nch;
            const int e2 = 64 * ch + lane;
            if (e2 < npair) lds_dma16(src + jb * bs + goff + 2 * e2, dst + jb * runl + 128 * ch);
        }
        if (cnt & 1)
            for (int jb = t; jb < nrun; jb += 256) dst[jb * runl + cnt - 1] = src[jb * bs + goff + cnt - 1];
    };
    copy_runs(A, sA, nra);
    if (beta != 0.0) copy_runs(Y, sO, nrb);
    if ((reinterpret_cast<uintptr_t>(C) & 15) == 0) {
        // C in 16-byte pieces (the odd last value by a plain load)
        const int np = (a * b) >> 1;
        for (int j = w; 64 * j < np; j += 4)
            if (64 * j + lane < np) lds_dma16(C + 2 * (64 * j + lane), sC + 128 * j);
        if (((a * b) & 1) && t == 0) sC[a * b - 1] = C[a * b - 1];
    } else {
        // C as 32-bit words, 4 bytes per lane (any 8-byte aligned C)
        const int nw = 2 * a * b;
        const unsigned* cw = reinterpret_cast<const unsigned*>(C);
        unsigned* scw = reinterpret_cast<unsigned*>(sC);
        for (int j = w; 64 * j < nw; j += 4)
            if (64 * j + lane < nw) lds_dma4(cw + 64 * j + lane, scw + 64 * j);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    const int ak = (a + 3) & ~3;
    const double* arow = sA + (16 * w + lr) * bw;
    int kb = 0, kc = lk;                       // run and column of this lane's k (bw >= 4)
    dx4_t acc[GR_MAXC / 16];
#pragma unroll
    for (int qt = 0; qt < GR_MAXC / 16; ++qt) acc[qt] = dx4_t{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < ak; k0 += 4) {
        const int k = k0 + lk;
        const double av = (k < a) ? arow[kb * runl + kc] : 0.0;
#pragma unroll
        for (int qt = 0; qt < GR_MAXC / 16; ++qt) {
            const int q = 16 * qt + lr;
            if (16 * qt < b) {
                const double cv = (k < a && q < b) ? sC[k * b + q] : 0.0;
                acc[qt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, cv, acc[qt], 0, 0, 0);
            }
        }
        kc += 4;
        if (kc >= bw) {
            kc -= bw;
            ++kb;
        }
    }
    __syncthreads();                           // every MFMA operand has been read
    // element i of lane l is row l / 16 + 4 i, column l % 16 of a tile
#pragma unroll
    for (int qt = 0; qt < GR_MAXC / 16; ++qt) {
        const int q = 16 * qt + lr;
        if (16 * qt < b && q < b) {
            const int jq = q / bw;
            double* dst = sA + jq * runl + (q - jq * bw) + (16 * w + lk) * bw;
#pragma unroll
            for (int i = 0; i < 4; ++i) dst[4 * i * bw] = acc[qt][i];
        }
    }
    __syncthreads();
    for (int jb = 0; jb < nrb; ++jb) {
        const double* l = sA + jb * runl;
        const double* lo = sO + jb * runl;
        double* g = Y + jb * bs + goff;
        for (int e2 = t; e2 < npair; e2 += 256) {
            const double2 v = *reinterpret_cast<const double2*>(l + 2 * e2);
            double2 o;
            if (beta == 0.0) {
                o = make_double2(alpha * v.x, alpha * v.y);
            } else {
                const double2 old = *reinterpret_cast<const double2*>(lo + 2 * e2);
                o = make_double2(fma(beta, old.x, alpha * v.x), fma(beta, old.y, alpha * v.y));
            }
            *reinterpret_cast<double2*>(g + 2 * e2) = o;
        }
        if ((cnt & 1) && t == 0) {
            const double v = l[cnt - 1];
            g[cnt - 1] = (beta == 0.0) ? alpha * v : fma(beta, lo[cnt - 1], alpha * v);
        }
    }
}

static size_t gemm_flat_smem(int a, int b, double beta) {
    return sizeof(double) * ((size_t)GR_ROWS * (a > b ? a : b) + (beta != 0.0 ? (size_t)GR_ROWS * b : 0) +
                             (size_t)a * b);
}

static size_t gemm_rows_smem(int a, int b) {
    const size_t ak = (a + 3) & ~3, bq = (b + 15) & ~15;
    const size_t rowsz = ak + 1 > bq + 1 ? ak + 1 : bq + 1;
    return sizeof(double) * ((size_t)GR_ROWS * rowsz + ak * bq);
}

// blocked layout with whole blocks and 16-byte aligned block bases: flat row runs
static int gemm_rows_flat(int a, int b, BlockGeom g, const double* const* A, const double* const* Y, int count) {
    if (g.ld != g.bw || a % g.bw || b % g.bw || (g.bs % 2) || ((long long)GR_ROWS * g.bw) % 2) return 0;
    for (int k = 0; k < count; ++k)
        if ((reinterpret_cast<uintptr_t>(A[k]) | reinterpret_cast<uintptr_t>(Y[k])) % 16) return 0;
    return 1;
}

void launch_gemm_rows(hipStream_t st, int n, int a, int b, double alpha, const double* const* A, double* const* Y,
                      int count, BlockGeom g, const double* C, double beta) {
    Triple T{};
    for (int k = 0; k < count; ++k) {
        T.A[k] = A[k];
        T.Y[k] = Y[k];
    }
    const int flat = gemm_rows_flat(a, b, g, A, Y, count);
    if (flat && g.bw >= 4 && gemm_flat_smem(a, b, beta) <= 65536) {
        hipLaunchKernelGGL(gemm_flat_kernel, dim3(grid_for(n, GR_ROWS), count), dim3(256), gemm_flat_smem(a, b, beta),
                           st, n, a, b, alpha, T, g.bw, g.bs, C, beta);
        return;
    }
    hipLaunchKernelGGL(gemm_rows_kernel, dim3(grid_for(n, GR_ROWS), count), dim3(256), gemm_rows_smem(a, b), st, n, a,
                       b, alpha, T, g, C, beta, flat);
}

void launch_rightmul_rows(hipStream_t st, int n, int b, double* const* Y, int count, BlockGeom g, const double* C) {
    Triple T{};
    for (int k = 0; k < count; ++k) {
        T.A[k] = Y[k];
        T.Y[k] = Y[k];
    }
    const int flat = gemm_rows_flat(b, b, g, Y, Y, count);
    if (flat && g.bw >= 4 && gemm_flat_smem(b, b, 0.0) <= 65536) {
        hipLaunchKernelGGL(gemm_flat_kernel, dim3(grid_for(n, GR_ROWS), count), dim3(256), gemm_flat_smem(b, b, 0.0),
                           st, n, b, b, 1.0, T, g.bw, g.bs, C, 0.0);
        return;
    }
    hipLaunchKernelGGL(gemm_rows_kernel, dim3(grid_for(n, GR_ROWS), count), dim3(256), gemm_rows_smem(b, b), st, n, b,
                       b, 1.0, T, g, C, 0.0, flat);
}

// ---------------------------------------------------------------------------
__global__ void copy_cols_kernel(int n, int ncols, const double* __restrict__ src, int lds, double* __restrict__ dst,
                                 int ldd) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)n * ncols) return;
    const long long r = t / ncols;
    const int c = (int)(t % ncols);
    dst[r * ldd + c] = src[r * lds + c];
}

void launch_copy_cols(hipStream_t st, int n, int ncols, const double* src, int lds, double* dst, int ldd) {
    hipLaunchKernelGGL(copy_cols_kernel, dim3(grid_for((long long)n * ncols, 256)), dim3(256), 0, st, n, ncols, src,
                       lds, dst, ldd);
}

__global__ void fill_kernel(long long count, double* __restrict__ dst, double value) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = value;
}

void launch_fill(hipStream_t st, long long count, double* dst, double value) {
    if (count <= 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, count, dst, value);
}

}  // namespace bpjd
