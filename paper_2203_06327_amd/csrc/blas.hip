// Block linear algebra on n x c row-major FP64 blocks: fused SpMM with K and M,
// residual block, Gram products, tall-times-small products.  All reductions are
// two-pass with a fixed summation order, so results do not depend on timing.
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
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = t >> cshift;
    const int c = t & ((1 << cshift) - 1);
    if (r >= n || c >= ncols) return;
    double ak = 0.0, am = 0.0;
    for (int p = rowptr[r]; p < rowptr[r + 1]; ++p) {
        const double2 v = km[p];
        const double x = X[(long long)col[p] * ldx + c];
        ak = fma(v.x, x, ak);
        am = fma(v.y, x, am);
    }
    KX[(long long)r * ldk + c] = ak;
    MX[(long long)r * ldm + c] = am;
}

void launch_spmm_km(hipStream_t st, int n, const int* rowptr, const int* col, const double2* km,
                    const double* X, int ldx, int ncols, double* KX, int ldk, double* MX, int ldm) {
    const int cp = pow2_at_least(ncols);
    int sh = 0;
    while ((1 << sh) < cp) ++sh;
    const long long work = (long long)n << sh;
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
                                double* __restrict__ F, int ldf, int chunk, double* __restrict__ partial) {
    __shared__ double red[2][256];
    const int t = threadIdx.x;
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
                     const double* lam, double* F, int ldf, double* partial, int npart, double* colsq) {
    const int chunk = (n + npart - 1) / npart;
    hipLaunchKernelGGL(residual_kernel, dim3(npart), dim3(256), 0, st, n, s, KX, ldk, MX, ldm, lam, F, ldf, chunk,
                       partial);
    launch_reduce(st, npart, 2 * s, partial, colsq);
}

// ---------------------------------------------------------------------------
// Gram product C = A^T B, a, b <= 64.  Each block stages 16 rows of A and B in
// LDS and accumulates up to 16 outputs per thread.
__global__ void gram_partial_kernel(int n, int a, int b, const double* __restrict__ A, int lda,
                                    const double* __restrict__ B, int ldb, int chunk,
                                    double* __restrict__ partial) {
    __shared__ double sA[16][64];
    __shared__ double sB[16][64];
    const int t = threadIdx.x;
    const int r0 = blockIdx.x * chunk;
    const int r1 = min(n, r0 + chunk);
    const int nout = a * b;
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int rb = r0; rb < r1; rb += 16) {
        for (int idx = t; idx < 16 * 64; idx += blockDim.x) {
            const int rr = idx >> 6, p = idx & 63;
            const int r = rb + rr;
            sA[rr][p] = (r < r1 && p < a) ? A[(long long)r * lda + p] : 0.0;
            sB[rr][p] = (r < r1 && p < b) ? B[(long long)r * ldb + p] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int o = t + u * 256;
            if (o < nout) {
                const int p = o / b, q = o % b;
                double v = acc[u];
#pragma unroll
                for (int rr = 0; rr < 16; ++rr) v = fma(sA[rr][p], sB[rr][q], v);
                acc[u] = v;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int o = t + u * 256;
        if (o < nout) partial[(long long)o * gridDim.x + blockIdx.x] = acc[u];
    }
}

void launch_gram(hipStream_t st, int n, int a, int b, const double* A, int lda, const double* B, int ldb,
                 double* partial, int npart, double* C) {
    const int chunk = (n + npart - 1) / npart;
    hipLaunchKernelGGL(gram_partial_kernel, dim3(npart), dim3(256), 0, st, n, a, b, A, lda, B, ldb, chunk, partial);
    launch_reduce(st, npart, a * b, partial, C);
}

// ---------------------------------------------------------------------------
__global__ void gemm_small_kernel(int n, int a, int b, int cshift, double alpha, const double* __restrict__ A,
                                  int lda, const double* __restrict__ C, double beta, double* __restrict__ Y,
                                  int ldy) {
    __shared__ double sC[64 * 64];
    for (int idx = threadIdx.x; idx < a * b; idx += blockDim.x) sC[idx] = C[idx];
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = t >> cshift;
    const int q = t & ((1 << cshift) - 1);
    if (r >= n || q >= b) return;
    const double* arow = A + (long long)r * lda;
    double acc = 0.0;
    for (int p = 0; p < a; ++p) acc = fma(arow[p], sC[p * b + q], acc);
    double* y = Y + (long long)r * ldy + q;
    *y = (beta == 0.0) ? alpha * acc : fma(beta, *y, alpha * acc);
}

void launch_gemm_small(hipStream_t st, int n, int a, int b, double alpha, const double* A, int lda,
                       const double* C, double beta, double* Y, int ldy) {
    const int cp = pow2_at_least(b);
    int sh = 0;
    while ((1 << sh) < cp) ++sh;
    const long long work = (long long)n << sh;
    hipLaunchKernelGGL(gemm_small_kernel, dim3(grid_for(work, 256)), dim3(256), 0, st, n, a, b, sh, alpha, A, lda, C,
                       beta, Y, ldy);
}

// In-place Y = Y * C (C b x b): a block stages 256/bpad rows of Y in LDS.
__global__ void rightmul_kernel(int n, int b, int cshift, double* __restrict__ Y, int ldy,
                                const double* __restrict__ C) {
    __shared__ double sC[64 * 64];
    __shared__ double sY[256];
    for (int idx = threadIdx.x; idx < b * b; idx += blockDim.x) sC[idx] = C[idx];
    const int rows = blockDim.x >> cshift;
    const int rr = threadIdx.x >> cshift;
    const int q = threadIdx.x & ((1 << cshift) - 1);
    const int r = blockIdx.x * rows + rr;
    double* yrow = Y + (long long)r * ldy;
    sY[threadIdx.x] = (r < n && q < b) ? yrow[q] : 0.0;
    __syncthreads();
    if (r >= n || q >= b) return;
    double acc = 0.0;
    const double* srow = sY + (rr << cshift);
    for (int p = 0; p < b; ++p) acc = fma(srow[p], sC[p * b + q], acc);
    yrow[q] = acc;
}

void launch_rightmul_inplace(hipStream_t st, int n, int b, double* Y, int ldy, const double* C) {
    const int cp = pow2_at_least(b);
    int sh = 0;
    while ((1 << sh) < cp) ++sh;
    const int rows = 256 >> sh;
    hipLaunchKernelGGL(rightmul_kernel, dim3(grid_for(n, rows)), dim3(256), 0, st, n, b, sh, Y, ldy, C);
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
