// Small dense FP64 kernels: banded Cholesky and triangular solves, the symmetric
// eigensolver (Householder tridiagonalisation, multisection on Sturm counts, inverse
// iteration) used for the coarse generalized eigenproblem (Section 3, coarse spectral
// split) and, in one workgroup, for the Rayleigh-Ritz problem (Algorithm 3.1, Step 3),
// Cholesky-QR coefficients and the coefficient-space step that keeps
// W^{k+1} = U^{k-1} + U^k + span{t}.
#include "common.h"

namespace bpjd {

constexpr int RR_MAX = 3 * BPJD_MAX_BLOCK;   // largest Rayleigh-Ritz dimension (3 s)
// up to this order the reduction to tridiagonal form runs in one workgroup; above it,
// two launches per column spread the trailing update over all compute units
constexpr int TRIDIAG_ONE_WG_MAX = 320;

// ---------------------------------------------------------------------------
// Block-wide sum with wave reductions (two barriers); every thread gets the result.
__device__ inline double block_sum_fast(double v, double* red) {
    const int t = threadIdx.x, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();                       // red may still be read by a previous call
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < nw; ++w) r += red[w];   // same order in every thread
    return r;
}

// Reciprocal from the hardware estimate refined by two Newton steps (within a few ulps
// of the rounded quotient).
__device__ inline double rcp_refined(double q) {
    double r = __builtin_amdgcn_rcp(q);
    r = fma(r, fma(-q, r, 1.0), r);
    r = fma(r, fma(-q, r, 1.0), r);
    return r;
}

// Right-looking Cholesky M = L L^T in place (one workgroup) of a matrix with lower
// bandwidth bw (entries with i - j > bw are zero; bw = n - 1 for a dense matrix): L
// keeps that band, so step k only updates rows and columns k+1 .. k+bw.  The current
// column is staged in LDS, the trailing window is updated with a fixed (row, column)
// map per thread, and the threads owning the next column write it to LDS as well, so
// that no step waits on a global load.  The strict upper triangle receives L^T, so that
// rows of L^T are contiguous for the backward solve.
__global__ __launch_bounds__(1024) void cholesky_kernel(int n, int bw, double* __restrict__ A,
                                                        int* __restrict__ status, int status_bit) {
    __shared__ double col[1024];     // column k of the trailing matrix (rows k..n-1)
    __shared__ double lk[1024];      // column k of L
    const int t = threadIdx.x, bd = blockDim.x;
    int bad = 0;
    for (int i = t; i < n; i += bd) col[i] = A[i * n];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        // rows k+1+bw.. of column k+1 enter the window only now: read them from A
        if (k > 0 && t == 0 && k + bw < n) col[k + bw] = A[(k + bw) * n + k];
        __syncthreads();
        double d = col[k];
        if (!(d > 0.0) || !isfinite(d)) {
            bad = 1;
            d = 1.0;
        }
        const double piv = sqrt(d), inv = 1.0 / piv;
        const int m = min(n - k - 1, bw);       // rows below the diagonal inside the band
        for (int i = k + 1 + t; i <= k + m; i += bd) {
            const double l = col[i] * inv;
            lk[i] = l;
            A[i * n + k] = l;
        }
        if (t == 0) A[k * n + k] = piv;
        __syncthreads();
        if (m > 0) {
            const int rs = bd / m, jj = t % m, r0 = t / m;
            if (r0 < rs) {
                const int j = k + 1 + jj;
                const double lj = lk[j];
                int ii = r0;
                if (ii < jj) ii += ((jj - ii + rs - 1) / rs) * rs;   // first owned row on or below the diagonal
                // batches of 8 rows: all loads are issued before the first store
                for (; ii < m; ii += 8 * rs) {
                    double a[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int iu = ii + u * rs;
                        a[u] = (iu < m) ? A[(k + 1 + iu) * n + j] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int iu = ii + u * rs;
                        if (iu < m) {
                            const int i = k + 1 + iu;
                            const double v = a[u] - lk[i] * lj;
                            A[i * n + j] = v;
                            if (jj == 0) col[i] = v;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1 + t; j < n; j += bd) A[i * n + j] = A[j * n + i];
    if (bad && t == 0) atomicOr(status, status_bit);
}

// The same factorisation for bands narrower than NB with the band held in registers:
// one workgroup of ceil(n / 64) wavefronts, thread j owning column j (entries j..j+NB-1,
// zero beyond the band).  The elimination runs in the square-root-free form: step k
// publishes the unscaled column k and 1 / d_k in LDS (two buffers, alternating with k);
// after one barrier the owner of column j = k + dd (dd = 1..bw) subtracts
// a_k[dd + e] a_k[dd] / d_k from its entry e.  Nothing in the loop touches global
// memory and the only division is the refined reciprocal of the pivot.  At the end
// thread j scales its column by 1 / sqrt(d_j) (L = L~ D^{1/2}) and writes it below the
// diagonal and, as row j of L^T, above it.
template <int NB>
__global__ __launch_bounds__(1024) void cholesky_reg_kernel(int n, int bw, double* __restrict__ A,
                                                            int* __restrict__ status, int status_bit) {
    __shared__ double lk[2][2 * NB];       // published column; entry 0 holds 1 / d_k, entries >= NB stay zero
    const int j = threadIdx.x;
    double a[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) a[e] = (j < n && e <= bw && j + e < n) ? A[(long long)(j + e) * n + j] : 0.0;
    for (int i = threadIdx.x; i < 4 * NB; i += blockDim.x) (&lk[0][0])[i] = 0.0;
    __syncthreads();
    int bad = 0;
    for (int k = 0; k < n; ++k) {
        double* buf = lk[k & 1];
        if (j == k) {
            if (!(a[0] > 0.0) || !isfinite(a[0])) {
                bad = 1;
                a[0] = 1.0;
            }
            buf[0] = rcp_refined(a[0]);
#pragma unroll
            for (int e = 1; e < NB; ++e) buf[e] = a[e];
        }
        __syncthreads();
        const int dd = j - k;
        if (dd >= 1 && dd <= bw) {
            double lv[NB];
#pragma unroll
            for (int e = 0; e < NB; ++e) lv[e] = buf[dd + e];
            const double c = lv[0] * buf[0];
#pragma unroll
            for (int e = 0; e < NB; ++e) a[e] = fma(-lv[e], c, a[e]);
        }
    }
    if (j < n) {
        const double piv = sqrt(a[0]), inv = 1.0 / piv;
#pragma unroll
        for (int e = 0; e < NB; ++e)
            if (e <= bw && j + e < n) {
                const double l = (e == 0) ? piv : a[e] * inv;
                A[(long long)(j + e) * n + j] = l;
                A[(long long)j * n + j + e] = l;
            }
    }
    if (bad) atomicOr(status, status_bit);
}

void launch_cholesky(hipStream_t st, int n, int bw, double* A, int* status, int status_bit) {
    const int threads = ((n + 63) / 64) * 64;
    if (n <= 1024 && bw < 20)
        hipLaunchKernelGGL(cholesky_reg_kernel<20>, dim3(1), dim3(threads), 0, st, n, bw, A, status, status_bit);
    else if (n <= 1024 && bw < 36)
        hipLaunchKernelGGL(cholesky_reg_kernel<36>, dim3(1), dim3(threads), 0, st, n, bw, A, status, status_bit);
    else
        hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(1024), 0, st, n, bw, A, status, status_bit);
}

// Triangular solves with a banded lower triangular L (n x n, lower bandwidth bw) and
// n_rhs right-hand sides, in place on X (row stride ldx): forward X <- L^{-1} X, or
// backward X <- L^{-T} X.  One wavefront per 64 right-hand sides, one lane per column.
// Narrow bands (bw < 64): per row, lane e reads band entry e of L (row r left of the
// diagonal, or column r below it) and lane bw' the diagonal, a row ahead, together with
// the next right-hand side; the entries are shared through LDS and the last results of
// each lane stay in an LDS ring, so the recurrence never waits on global memory.
// Wider bands read L and earlier results from global memory.
template <bool NARROW>
__global__ __launch_bounds__(64) void trsm_band_kernel(int n, int bw, int nrhs, const double* __restrict__ L,
                                                       double* __restrict__ X, int ldx, int backward) {
    __shared__ double lw[65];
    __shared__ double ring[NARROW ? 64 : 1][64];
    const int lane = threadIdx.x;
    const int c = blockIdx.x * 64 + lane;
    const bool live = c < nrhs;
    auto row_of = [&](int step) -> int { return backward ? n - 1 - step : step; };
    auto rowcount = [&](int r) -> int { return backward ? min(bw, n - 1 - r) : min(bw, r); };
    // global index of band entry e (0-based, away from the diagonal) of row r
    auto lidx = [&](int r, int e) -> long long {
        return backward ? (long long)(r + 1 + e) * n + r : (long long)r * n + (r - 1 - e);
    };
    if (NARROW) {
        // the raw loads are kept and the selection is made a row later, so the loads stay
        // in flight for a whole row
        auto load_row = [&](int r, double& lval, bool& lok, double& bval) {
            const int cnt = rowcount(r);
            // one unconditional vector load per lane (index clamped onto the diagonal)
            const long long idx = (lane < cnt) ? lidx(r, lane) : (long long)r * n + r;
            lval = L[idx];
            lok = lane <= cnt;
            bval = X[(long long)r * ldx + (live ? c : 0)];
        };
        double pre_l = 0.0, pre_b = 0.0;
        bool pre_ok = false;
        if (n > 0) load_row(row_of(0), pre_l, pre_ok, pre_b);
        for (int step = 0; step < n; ++step) {
            const int r = row_of(step);
            const int cnt = rowcount(r);
            const double cur_l = pre_ok ? pre_l : 0.0, cur_b = pre_b;
            if (step + 1 < n) load_row(row_of(step + 1), pre_l, pre_ok, pre_b);
            lw[lane] = cur_l;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_wave_barrier();
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            double acc0 = cur_b, acc1 = 0.0;
            int e = 0;
            for (; e + 1 < cnt; e += 2) {
                const int ja = backward ? r + 1 + e : r - 1 - e;
                const int jb = backward ? ja + 1 : ja - 1;
                acc0 = fma(-lw[e], ring[ja & 63][lane], acc0);
                acc1 = fma(-lw[e + 1], ring[jb & 63][lane], acc1);
            }
            if (e < cnt) {
                const int ja = backward ? r + 1 + e : r - 1 - e;
                acc0 = fma(-lw[e], ring[ja & 63][lane], acc0);
            }
            const double x = (acc0 + acc1) / lw[cnt];
            if (live) X[(long long)r * ldx + c] = x;
            ring[r & 63][lane] = x;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_wave_barrier();
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
    } else {
        if (!live) return;
        for (int step = 0; step < n; ++step) {
            const int r = row_of(step);
            const int cnt = rowcount(r);
            double acc0 = X[(long long)r * ldx + c], acc1 = 0.0;
            int e = 0;
            for (; e + 1 < cnt; e += 2) {
                const int ja = backward ? r + 1 + e : r - 1 - e;
                const int jb = backward ? ja + 1 : ja - 1;
                acc0 = fma(-L[lidx(r, e)], X[(long long)ja * ldx + c], acc0);
                acc1 = fma(-L[lidx(r, e + 1)], X[(long long)jb * ldx + c], acc1);
            }
            if (e < cnt) {
                const int ja = backward ? r + 1 + e : r - 1 - e;
                acc0 = fma(-L[lidx(r, e)], X[(long long)ja * ldx + c], acc0);
            }
            X[(long long)r * ldx + c] = (acc0 + acc1) / L[(long long)r * n + r];
        }
    }
}

// Narrow bands (bw < NB) with the recent results in registers: the row loop is unrolled
// by NB, so result t sits in register t mod NB and every band term has a fixed
// register.  Steps t (row t forward, row n-1-t backward) go in blocks of NB; the band
// entries of a block (row r of L left of the diagonal forward, row r of L^T right of
// it backward, both contiguous) and its right-hand sides are loaded one block ahead
// into registers and moved to LDS at the block's start, where every lane reads the
// band entries as broadcasts.  Entry e = 0 holds the reciprocal of the diagonal.
// Terms beyond the band or the matrix are zero, so every step sums the same NB - 1
// terms: even and odd distances in two partial sums (farthest first), then the
// nearest result, so only one multiply-add per step waits on the previous step.
template <int NB>
__global__ __launch_bounds__(64) void trsm_reg_kernel(int n, int bw, int nrhs, const double* __restrict__ L,
                                                      double* __restrict__ X, int ldx, int backward) {
    constexpr int SPL = (NB * NB + 63) / 64;        // band values staged per lane
    __shared__ double lb[NB * NB];                  // lb[u * NB + e]: block step u, band entry e
    __shared__ double bx[NB][64];                   // right-hand sides of the block
    const int lane = threadIdx.x;
    const int c = blockIdx.x * 64 + lane;
    const bool live = c < nrhs;
    const int cc = live ? c : 0;
    const int sg = backward ? 1 : -1;
    double stg[SPL], bnx[NB], xr[NB];
    auto load_block = [&](int t0) {
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            const int f = lane + 64 * q, u = f / NB, e = f - u * NB, t = t0 + u;
            const int r = backward ? n - 1 - t : t, col = r + sg * e;
            stg[q] = (f < NB * NB && t < n && e <= bw && col >= 0 && col < n) ? L[(long long)r * n + col] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int t = t0 + u;
            bnx[u] = (t < n) ? X[(long long)(backward ? n - 1 - t : t) * ldx + cc] : 0.0;
        }
    };
    // results of block t0 are stored at the start of the next block, before its loads
    // are issued, so the wait for those loads never waits on fresh stores
    auto store_block = [&](int t0) {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int t = t0 + u;
            if (live && t < n) X[(long long)(backward ? n - 1 - t : t) * ldx + c] = xr[u];
        }
    };
#pragma unroll
    for (int u = 0; u < NB; ++u) xr[u] = 0.0;
    load_block(0);
    for (int t0 = 0; t0 < n; t0 += NB) {
        __syncthreads();                            // the previous block's LDS reads are done
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            const int f = lane + 64 * q;
            const double v = stg[q], rv = rcp_refined(v);
            if (f < NB * NB) lb[f] = (f % NB != 0) ? v : (v != 0.0 ? rv : 0.0);
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) bx[u][lane] = bnx[u];
        __syncthreads();
        if (t0 > 0) store_block(t0 - NB);
        if (t0 + NB < n) load_block(t0 + NB);
        // software pipeline: the band entries of step u + 1 are read from LDS while step u
        // computes
        double lv[2][NB];
#pragma unroll
        for (int e = 0; e < NB; ++e) lv[0][e] = lb[e];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            if (u + 1 < NB) {
#pragma unroll
                for (int e = 0; e < NB; ++e) lv[(u + 1) & 1][e] = lb[(u + 1) * NB + e];
            }
            const double* l = lv[u & 1];
            double se = bx[u][lane], so = 0.0;
#pragma unroll
            for (int e = NB - 1; e >= 2; --e) {
                if (e & 1) so = fma(l[e], xr[(u - e + NB) % NB], so);
                else se = fma(-l[e], xr[(u - e + NB) % NB], se);
            }
            xr[u] = fma(-l[1], xr[(u - 1 + NB) % NB], se - so) * l[0];
        }
    }
    store_block(((n - 1) / NB) * NB);
}

void launch_trsm_band(hipStream_t st, int n, int bw, int nrhs, const double* L, double* X, int ldx, bool backward) {
    if (bw < 20)
        hipLaunchKernelGGL(trsm_reg_kernel<20>, dim3(grid_for(nrhs, 64)), dim3(64), 0, st, n, bw, nrhs, L, X, ldx,
                           backward ? 1 : 0);
    else if (bw < 36)
        hipLaunchKernelGGL(trsm_reg_kernel<36>, dim3(grid_for(nrhs, 64)), dim3(64), 0, st, n, bw, nrhs, L, X, ldx,
                           backward ? 1 : 0);
    else if (bw < 64)
        hipLaunchKernelGGL(trsm_band_kernel<true>, dim3(grid_for(nrhs, 64)), dim3(64), 0, st, n, bw, nrhs, L, X, ldx,
                           backward ? 1 : 0);
    else
        hipLaunchKernelGGL(trsm_band_kernel<false>, dim3(grid_for(nrhs, 64)), dim3(64), 0, st, n, bw, nrhs, L, X, ldx,
                           backward ? 1 : 0);
}

__global__ void transpose_kernel(int n, const double* __restrict__ A, double* __restrict__ AT) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * n) return;
    const int i = (int)(e / n), j = (int)(e % n);
    AT[(long long)j * n + i] = A[e];
}

void launch_transpose(hipStream_t st, int n, const double* A, double* AT) {
    hipLaunchKernelGGL(transpose_kernel, dim3(grid_for((long long)n * n, 256)), dim3(256), 0, st, n, A, AT);
}

// ---------------------------------------------------------------------------
// Householder reduction of the symmetric A (n x n, one workgroup of 512 threads) to
// tridiagonal form T = Q^T A Q.  Step k: reflector H_k = I - tau_k v v^T (v_0 = 1)
// annihilating A[k+2.., k]; A22 <- H_k A22 H_k as A22 - v w^T - w v^T with
// p = tau A22 v, w = p - (tau/2)(p^T v) v.  One pass over the matrix per step: the
// updated column k+1 is formed first (in LDS) and gives the next reflector v', and the
// pass that applies the rank-2 update to rows and columns k+2.. also accumulates
// A22' v' (column sums, A being symmetric) for the next step.  Column and row k+1 are
// not written back; they are only needed as the next column, which stays in LDS.
// Outputs: diag, off (T), the reflectors Vh (row k = v of step k, from column k+1)
// and tau.
__device__ inline double tridiag_reflector(int n, int k, const double* col, double* vk, double* Vh, double* tau,
                                           double* diag, double* off, double* wred) {
    // col[i] = current A[k + i][k], i = 0 .. n-k-1; writes vk[i] (rows k+1+i) and returns tau_k
    const int t = threadIdx.x, bd = blockDim.x, m = n - k - 1;
    double acc = 0.0;
    for (int i = 2 + t; i <= m; i += bd) acc = fma(col[i], col[i], acc);
    const double xn2 = block_sum_fast(acc, wred);
    const double alpha = col[1];
    double tk, scale, beta;
    if (xn2 == 0.0) {
        tk = 0.0;
        scale = 0.0;
        beta = alpha;
    } else {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tk = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
    }
    if (t == 0) {
        tau[k] = tk;
        off[k] = beta;
        diag[k] = col[0];
    }
    for (int i = t; i < m; i += bd) {
        const double vi = (i == 0) ? 1.0 : col[1 + i] * scale;
        vk[i] = vi;
        Vh[(long long)k * n + k + 1 + i] = vi;
    }
    __syncthreads();
    return tk;
}

__global__ __launch_bounds__(512) void tridiag_kernel(int n, double* __restrict__ A, double* __restrict__ Vh,
                                                       double* __restrict__ tau, double* __restrict__ diag,
                                                       double* __restrict__ off) {
    __shared__ double vbuf[2][1024];  // current and next reflector
    __shared__ double w[1024];
    __shared__ double col[1024];      // the column being reduced, col[i] = A[k + i][k]
    __shared__ double pp[1024];       // A22 v (unscaled) for the current step
    __shared__ double red[1024];
    __shared__ double wred[16];
    const int t = threadIdx.x, bd = blockDim.x;
    if (n <= 2) {
        if (t == 0) {
            diag[0] = A[0];
            if (n == 2) {
                off[0] = A[n];
                diag[1] = A[n + 1];
            }
            off[n - 1] = 0.0;
        }
        return;
    }
    // Sweep over the square block of rows and columns r0..n-1 (mr = n - r0): thread
    // (jj, rg) owns column jj and rows rg, rg + rs, ...; with upd, entries first take
    // a -= v[i+1] w[j+1] + w[i+1] v[j+1] (v, w indexed from row r0 - 1) and are written
    // back; then pp[j] = sum_i a[i][j] x[i] with a fixed summation order.
    auto sweep = [&](int r0, bool upd, const double* vv, const double* x) {
        const int mr = n - r0;
        const int rs = bd / mr, jj = t % mr, rg = t / mr;
        if (rg < rs) {
            const int j = r0 + jj;
            const double vj = upd ? vv[jj + 1] : 0.0, wj = upd ? w[jj + 1] : 0.0;
            double acc = 0.0;
            // the thread's rows are rg + rs q, q < nq; full batches of 8 rows go through two
            // alternating buffers, each loaded one batch ahead of its update and store.  The
            // loads are unconditional (the batch index is clamped), so the wait before a
            // batch's use covers that batch only; the last nq % 8 rows follow one by one.
            const int nq = (mr - rg + rs - 1) / rs, nb = nq / 8;
            double a0[8], a1[8];
            auto load8 = [&](int b, double* dst) {
                const int q0 = 8 * min(b, nb - 1);
#pragma unroll
                for (int u = 0; u < 8; ++u) dst[u] = A[(long long)(r0 + rg + (q0 + u) * rs) * n + j];
            };
            auto row = [&](int iu, double val) {
                if (upd) {
                    val -= vv[iu + 1] * wj + w[iu + 1] * vj;
                    A[(long long)(r0 + iu) * n + j] = val;
                }
                acc = fma(val, x[iu], acc);
            };
            auto work8 = [&](int b, const double* src) {
#pragma unroll
                for (int u = 0; u < 8; ++u) row(rg + (8 * b + u) * rs, src[u]);
            };
            if (nb > 0) load8(0, a0);
            for (int b = 0; b < nb; b += 2) {
                load8(b + 1, a1);
                work8(b, a0);
                load8(b + 2, a0);
                if (b + 1 < nb) work8(b + 1, a1);
            }
            for (int q = 8 * nb; q < nq; ++q) {
                const int iu = rg + q * rs;
                row(iu, A[(long long)(r0 + iu) * n + j]);
            }
            red[rg * mr + jj] = acc;
        }
        __syncthreads();
        for (int j = t; j < mr; j += bd) {
            double s = 0.0;
            for (int g = 0; g < rs; ++g) s += red[g * mr + j];
            pp[j] = s;
        }
        __syncthreads();
    };
    for (int i = t; i < n; i += bd) col[i] = A[(long long)i * n];
    __syncthreads();
    int cur = 0;
    double tk = tridiag_reflector(n, 0, col, vbuf[0], Vh, tau, diag, off, wred);
    sweep(1, false, nullptr, vbuf[0]);                 // pp = A22 v_0
    for (int k = 0;; ++k) {
        const int m = n - k - 1;                       // A22: rows and columns k+1 .. n-1
        const double* v = vbuf[cur];
        // w = tau p - (tau / 2)(tau p^T v) v, with p = A22 v in pp
        double acc = 0.0;
        for (int i = t; i < m; i += bd) acc = fma(pp[i], v[i], acc);
        const double pv = block_sum_fast(acc, wred);
        for (int i = t; i < m; i += bd) w[i] = (tk == 0.0) ? 0.0 : tk * pp[i] - 0.5 * tk * tk * pv * v[i];
        __syncthreads();
        if (k + 3 >= n) {                              // A22 is the last 2 x 2 block
            if (t == 0) {
                const int r = k + 1;
                diag[r] = A[(long long)r * n + r] - 2.0 * v[0] * w[0];
                off[r] = A[(long long)(r + 1) * n + r] - (v[1] * w[0] + w[1] * v[0]);
                diag[r + 1] = A[(long long)(r + 1) * n + r + 1] - 2.0 * v[1] * w[1];
                off[r + 1] = 0.0;
            }
            break;
        }
        // column k+1 after the update, then its reflector
        for (int i = t; i < m; i += bd) col[i] = A[(long long)(k + 1 + i) * n + k + 1] - (v[i] * w[0] + w[i] * v[0]);
        __syncthreads();
        const double tn = tridiag_reflector(n, k + 1, col, vbuf[cur ^ 1], Vh, tau, diag, off, wred);
        // rank-2 update of rows/columns k+2.. and pp = A22' v'
        sweep(k + 2, true, v, vbuf[cur ^ 1]);
        cur ^= 1;
        tk = tn;
    }
}

// the value of lane l of a wavefront, in every lane
__device__ inline double lane_bcast(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wavefront with DPP row operations (no LDS traffic); the
// total is returned in every lane.  Lanes of rows excluded by a row mask add zero.
template <int CTRL, int ROWMASK>
__device__ inline double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double wave_sum_dpp(double v) {
    v += dpp_f64<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xF>(v);   // row_half_mirror: sums of 8
    v += dpp_f64<0x140, 0xF>(v);   // row_mirror: sums of the 16-lane row
    v += dpp_f64<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3: lane 63 holds the total
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Householder reduction of the symmetric A (n x n) to tridiagonal form T = Q^T A Q,
// one reflector H_k = I - tau_k v v^T (v_0 = 1) per column, with the trailing update
// A22 <- A22 - v w^T - w v^T (p = tau A22 v, w = p - (tau/2)(p^T v) v) applied lazily:
//   the head of step k: finishes w_{k-1} from p, forms row k of the current matrix with
//     the pending update of step k-1 applied on the fly, and builds v_k;
//   the sweep (one wavefront per trailing row j, all compute units): applies the
//     pending update of step k-1 to row j of A22 and forms (A22 v_k)_j.
// A is symmetric, so rows stand for columns and every access is row-contiguous.
// Outputs: diag, off (T), the reflectors Vh (row k = v_k, from column k+1), tau.
// pbuf (n) carries A22 v_k from one launch to the next; wbuf receives w_k.
// Head of step k (any block size): finishes w_{k-1} from p, forms row k of the current
// matrix with the pending update of step k-1 applied on the fly, and builds v_k.
__device__ void tridiag_head(int n, int k, const double* __restrict__ A, double* __restrict__ Vh,
                             double* __restrict__ tau, const double* __restrict__ pbuf, double* __restrict__ wbuf,
                             double* __restrict__ diag, double* __restrict__ off, double* r, double* wred) {
    const int t = threadIdx.x, bd = blockDim.x;
    if (k >= 1) {
        // w_{k-1} = tau p - (tau/2)(tau p^T v) v over rows k..n-1
        const int kp = k - 1;
        const double tp = tau[kp];
        const double* vp = Vh + (long long)kp * n;
        // this thread's rows (at most four: n <= 1024, at least 256 threads): p, v and row
        // k of A are loaded together up front, not once per phase
        constexpr int MAXI = 4;
        double pv[MAXI], vv[MAXI], av[MAXI], wv[MAXI];
#pragma unroll
        for (int j = 0; j < MAXI; ++j) {
            const int i = min(k + t + j * bd, n - 1);
            pv[j] = pbuf[i];
            vv[j] = vp[i];
            av[j] = A[(long long)k * n + i];
        }
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < MAXI; ++j)
            if (k + t + j * bd < n) acc = fma(tp * pv[j], vv[j], acc);
        const double half_tpv = 0.5 * tp * block_sum_fast(acc, wred);
#pragma unroll
        for (int j = 0; j < MAXI; ++j) {
            const int i = k + t + j * bd;
            wv[j] = tp * pv[j] - half_tpv * vv[j];
            if (i < n) wbuf[i] = wv[j];
        }
        __syncthreads();
        const double vk = vp[k], wk = wbuf[k];
#pragma unroll
        for (int j = 0; j < MAXI; ++j) {
            const int i = k + t + j * bd;
            if (i < n) r[i] = av[j] - (vk * wv[j] + wk * vv[j]);
        }
    } else {
        for (int i = t; i < n; i += bd) r[i] = A[i];
    }
    __syncthreads();
    if (k + 2 >= n) {                      // last 2 x 2 block (k = n - 2) or n = 1
        if (t == 0) {
            diag[k] = r[k];
            if (k + 1 < n) {
                off[k] = r[k + 1];
                double d1 = A[(long long)(n - 1) * n + n - 1];
                if (k >= 1) {
                    const double* vp = Vh + (long long)(k - 1) * n;
                    d1 -= 2.0 * vp[n - 1] * wbuf[n - 1];
                }
                diag[n - 1] = d1;
            }
            off[n - 1] = 0.0;
        }
        return;
    }
    double acc = 0.0;
    for (int i = k + 2 + t; i < n; i += bd) acc = fma(r[i], r[i], acc);
    const double xn2 = block_sum_fast(acc, wred);
    const double alpha = r[k + 1];
    double tk, scale, beta;
    if (xn2 == 0.0) {
        tk = 0.0;
        scale = 0.0;
        beta = alpha;
    } else {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tk = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
    }
    if (t == 0) {
        tau[k] = tk;
        off[k] = beta;
        diag[k] = r[k];
    }
    double* vk = Vh + (long long)k * n;
    for (int i = k + 1 + t; i < n; i += bd) vk[i] = (i == k + 1) ? 1.0 : r[i] * scale;
}

__global__ __launch_bounds__(1024) void tridiag_head_kernel(int n, int k, const double* __restrict__ A,
                                                            double* __restrict__ Vh, double* __restrict__ tau,
                                                            const double* __restrict__ pbuf,
                                                            double* __restrict__ wbuf, double* __restrict__ diag,
                                                            double* __restrict__ off) {
    __shared__ double r[1024];            // row k of the current matrix, r[i] for i >= k
    __shared__ double wred[16];
    tridiag_head(n, k, A, Vh, tau, pbuf, wbuf, diag, off, r, wred);
}

// Step k (1 <= k <= n - 3; step 0 takes v_0 from tridiag_head_kernel): one wavefront
// per trailing row j > k, each working alone (no LDS, no barriers).  The wavefront first
// forms the head of step k over the rows i = k + 1 + lane + 64 u, u < U (64 U >= n): w_{k-1}
// from p_{k-1} (pin), row k of the current matrix with the pending update of step k-1
// applied, and the reflector v_k, with its sums over the wavefront by DPP (every
// wavefront adds in the same order, so all hold the same v_k); wave 0 of workgroup 0
// (row k + 1) stores v_k, tau_k, diag[k] and off[k].  Then it applies the pending
// update of step k-1 to row j of A22 and forms (A22 v_k)_j into pout.  p alternates
// between two buffers, so a wavefront that starts late still reads the previous step's;
// each column costs one launch.  All of row j's and the head's loads are issued first.
__global__ __launch_bounds__(256) void tridiag_step_kernel(int n, int k, double* __restrict__ A,
                                                           double* __restrict__ Vh, double* __restrict__ tau,
                                                           const double* __restrict__ pin, double* __restrict__ pout,
                                                           double* __restrict__ diag, double* __restrict__ off) {
    const int lane = threadIdx.x & 63;
    const int j = k + 1 + blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;                    // row k + 1 (the writer's) is always in range
    const bool writer = blockIdx.x == 0 && threadIdx.x < 64;
    double* row = A + (long long)j * n;
    constexpr int U = 16;
    const int i0 = k + 1 + lane;
    double rv[U];
    if (k == 0) {
        double kv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = min(i0 + 64 * u, n - 1);
            rv[u] = row[i];
            kv[u] = Vh[i];
        }
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + 64 * u < n) acc = fma(rv[u], kv[u], acc);
        acc = wave_sum_dpp(acc);
        if (lane == 0) pout[j] = acc;
        return;
    }
    const double* vp = Vh + (long long)(k - 1) * n;
    const double* ak_row = A + (long long)k * n;
    double pv[U], vv[U], av[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = min(i0 + 64 * u, n - 1);
        rv[u] = row[i];
        pv[u] = pin[i];
        vv[u] = vp[i];
        av[u] = ak_row[i];
    }
    const double tp = tau[k - 1];
    const double pk = pin[k], vk = vp[k], ak = ak_row[k];
    const double pj = pin[j], vj = vp[j];
    // w_{k-1} = tau p - (tau/2)(tau p^T v) v over rows k..n-1
    double acc = (lane == 0) ? tp * pk * vk : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (i0 + 64 * u < n) acc = fma(tp * pv[u], vv[u], acc);
    const double half_tpv = 0.5 * tp * wave_sum_dpp(acc);
    const double wk = tp * pk - half_tpv * vk;
    const double wj = tp * pj - half_tpv * vj;
    double wv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) wv[u] = tp * pv[u] - half_tpv * vv[u];
    // row k of the current matrix (entries k + 1 ..) and the reflector of row k
    double r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = av[u] - (vk * wv[u] + wk * vv[u]);
    double xs = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = i0 + 64 * u;
        if (i > k + 1 && i < n) xs = fma(r[u], r[u], xs);
    }
    const double xn2 = wave_sum_dpp(xs);
    const double alpha = lane_bcast(r[0], 0);          // entry k + 1
    double tk, scale, beta;
    if (xn2 == 0.0) {
        tk = 0.0;
        scale = 0.0;
        beta = alpha;
    } else {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tk = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
    }
    double vkn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) vkn[u] = (i0 + 64 * u == k + 1) ? 1.0 : r[u] * scale;
    if (writer) {
        if (lane == 0) {
            tau[k] = tk;
            off[k] = beta;
            diag[k] = ak - (vk * wk + wk * vk);
        }
        double* vrow = Vh + (long long)k * n;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + 64 * u < n) vrow[i0 + 64 * u] = vkn[u];
    }
    // row j: the pending update of step k-1, then (A22 v_k)_j
    double pacc = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = i0 + 64 * u;
        if (i < n) {
            const double a = rv[u] - (vj * wv[u] + wj * vv[u]);
            row[i] = a;
            pacc = fma(a, vkn[u], pacc);
        }
    }
    pacc = wave_sum_dpp(pacc);
    if (lane == 0) pout[j] = pacc;
}

// Eigenvalues of the symmetric tridiagonal matrix (diag d, off-diagonal e,
// e[i] coupling i and i+1) by bisection on Sturm counts: thread j finds the
// j-th smallest eigenvalue.  count(x) = number of negative pivots of the
// LDL^T factorisation of T - x I.
// The quotient e^2 / q uses the hardware reciprocal refined by two Newton steps
// (within a few ulps of the rounded quotient): the count is that of a T whose
// off-diagonal entries are perturbed by a few ulps, well inside the backward error
// the recurrence has anyway; |q| >= pivmin keeps the reciprocal finite.
// The operands of four steps are loaded before they enter the recurrence, so the
// chain only waits on arithmetic.
__device__ inline int sturm_count(int n, const double* d, const double* e2, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
    int i = 1;
    for (; i + 3 < n; i += 4) {
        double dv[4], ev[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            dv[u] = d[i + u] - x;
            ev[u] = e2[i + u - 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            q = dv[u] - ev[u] * rcp_refined(q);
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += (q < 0.0);
        }
    }
    for (; i < n; ++i) {
        q = (d[i] - x) - e2[i - 1] * rcp_refined(q);
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0);
    }
    return cnt;
}

// sum_i a[i * sa] b[i * sb], i < len, over LDS or registers-backed arrays: four
// independent accumulators and operands loaded four at a time, so the loads of one
// group are in flight together (fixed summation order)
__device__ inline double dot_strided(const double* a, int sa, const double* b, int sb, int len) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int i = 0;
    for (; i + 3 < len; i += 4) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            x[u] = a[(i + u) * sa];
            y[u] = b[(i + u) * sb];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = fma(x[u], y[u], acc[u]);
    }
    for (; i < len; ++i) acc[0] = fma(a[i * sa], b[i * sb], acc[0]);
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Bisection with 32-way multisection: 32 threads per eigenvalue (several workgroups)
// evaluate Sturm counts at 32 interior points of the current interval, which then
// shrinks by a factor 33 per round.  Eigenvalue j (ascending) is the point where
// count(x) passes j.  Every workgroup stages d and e^2 in LDS and forms the same
// Gershgorin interval.
constexpr int BISECT_G = 32;
__global__ __launch_bounds__(256) void tridiag_bisect_kernel(int n, const double* __restrict__ dg,
                                                             const double* __restrict__ eg, double* __restrict__ w) {
    __shared__ double d[1024];
    __shared__ double e2[1024];
    __shared__ double red[2][256];
    const int t = threadIdx.x, bd = blockDim.x;
    double lo = 1e300, hi = -1e300;
    for (int i = t; i < n; i += bd) {
        d[i] = dg[i];
        const double ei = (i + 1 < n) ? eg[i] : 0.0;
        e2[i] = ei * ei;
        const double el = (i > 0) ? fabs(eg[i - 1]) : 0.0;
        const double er = fabs(ei);
        lo = fmin(lo, dg[i] - el - er);
        hi = fmax(hi, dg[i] + el + er);
    }
    red[0][t] = lo;
    red[1][t] = hi;
    __syncthreads();
    for (int o = bd / 2; o > 0; o >>= 1) {
        if (t < o) {
            red[0][t] = fmin(red[0][t], red[0][t + o]);
            red[1][t] = fmax(red[1][t], red[1][t + o]);
        }
        __syncthreads();
    }
    const double glo = red[0][0], ghi = red[1][0];
    const double tnorm = fmax(fabs(glo), fabs(ghi));
    const double pivmin = 1e-300 + 1e-30 * tnorm * tnorm;
    constexpr int G = BISECT_G;
    const int tt = blockIdx.x * bd + t;
    const int j = tt / G, r = tt % G;
    const int gl = (t & 63) - r;                   // first lane of this thread's group
    bool done = j >= n;
    double a = glo - 1e-14 * tnorm - 1e-300, b = ghi + 1e-14 * tnorm + 1e-300;
    for (int it = 0; it < 200 && __any(!done); ++it) {
        if (!done && (!(0.5 * (a + b) > a && 0.5 * (a + b) < b) || (b - a) <= 2.3e-16 * fmax(fabs(a), fabs(b))))
            done = true;
        const double x = a + (b - a) / (double)(G + 1) * (double)(r + 1);
        const bool above = !done && sturm_count(n, d, e2, x, pivmin) > j;
        // the first of the G points whose count exceeds j closes the interval
        const unsigned long long grp = (__ballot(above) >> gl) & ((1ull << G) - 1ull);
        if (!done) {
            const double h = (b - a) / (double)(G + 1);
            if (grp) {
                const int q = __ffsll((long long)grp) - 1;
                const double na = (q > 0) ? a + h * (double)q : a;
                b = a + h * (double)(q + 1);
                a = na;
            } else {
                a = a + h * (double)G;
            }
        }
    }
    if (j < n && r == 0) w[j] = 0.5 * (a + b);
}

// Inverse iteration for every eigenvalue (one thread each): three solves of
// (T - lambda_j I) x = b with a partial-pivoting LU of the tridiagonal matrix
// (U has two superdiagonals), starting from a fixed vector.  Scratch and result
// vectors are interleaved ([i][j]) so accesses coalesce across threads.  The sweeps
// run in batches of INVIT_B steps whose operands are loaded one batch ahead into two
// alternating buffers, so the recurrences wait on arithmetic, not on memory.  Each solve's right-hand side is the
// previous solution scaled to unit norm.
// Output: X[i][j] = component i of eigenvector j (unit 2-norm).
constexpr int INVIT_B = 16;
__global__ __launch_bounds__(64) void tridiag_invit_kernel(int n, const double* __restrict__ dg,
                                                           const double* __restrict__ eg,
                                                           const double* __restrict__ w, double* __restrict__ X,
                                                           double* __restrict__ u0, double* __restrict__ u1,
                                                           double* __restrict__ u2, double* __restrict__ mu,
                                                           double* __restrict__ pv, double* __restrict__ y) {
    __shared__ double d[1024];
    __shared__ double e[1024];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        d[i] = dg[i];
        e[i] = (i + 1 < n) ? eg[i] : 0.0;
    }
    __syncthreads();
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    constexpr int B = INVIT_B;
    // u0: 1 / U diagonal; u1, u2: U super-diagonals; mu: multipliers; pv: 1.0 where rows
    // were swapped; y: forward-sweep result (all [n][n], interleaved over eigenvalues)
#define IDX(i) ((long long)(i) * n + j)
    const double lam = w[j];
    double tn = 0.0;
    for (int i = 0; i < n; ++i) tn = fmax(tn, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + fabs(e[i]));
    const double tiny = 2.3e-16 * fmax(tn, 1e-300);
    // factorisation P (T - lam I) = L U; pv[i] = 1 where rows i and i+1 were swapped
    double a0 = d[0] - lam, a1 = (n > 1) ? e[0] : 0.0, a2 = 0.0;   // current row (cols i, i+1, i+2)
    for (int i = 0; i + 1 < n; ++i) {
        const double sub = e[i];                                      // next row: (sub, d[i+1]-lam, e[i+1])
        const double nd = d[i + 1] - lam;
        const double ne = e[i + 1];
        double p0, p1, p2, m;
        const bool swap = fabs(sub) > fabs(a0);
        if (swap) {
            m = a0 / sub;
            p0 = sub;
            p1 = nd;
            p2 = ne;
            const double na0 = a1 - m * nd, na1 = a2 - m * ne;
            a0 = na0;
            a1 = na1;
        } else {
            p0 = (a0 == 0.0) ? tiny : a0;
            m = sub / p0;
            p1 = a1;
            p2 = a2;
            a0 = nd - m * a1;
            a1 = ne - m * a2;
        }
        a2 = 0.0;
        u0[IDX(i)] = 1.0 / ((fabs(p0) < tiny) ? copysign(tiny, p0 == 0.0 ? 1.0 : p0) : p0);
        pv[IDX(i)] = swap ? 1.0 : 0.0;
        u1[IDX(i)] = p1;
        u2[IDX(i)] = p2;
        mu[IDX(i)] = m;
    }
    u0[IDX(n - 1)] = 1.0 / ((fabs(a0) < tiny) ? copysign(tiny, a0 == 0.0 ? 1.0 : a0) : a0);
    u1[IDX(n - 1)] = 0.0;                      // no super-diagonals in the last row
    u2[IDX(n - 1)] = 0.0;
    // first right-hand side: a fixed vector with varying entries
    for (int i = 0; i < n; ++i) X[IDX(i)] = 1.0 + 0.5 * sin(0.7 * i + 0.3 * j);
    double scale = 1.0;                        // 1 / norm of the previous solution
    for (int sweep = 0; sweep < 3; ++sweep) {
        // apply the row operations to the right-hand side: b -> y (steps i = 0 .. n-2)
        double cX[B] = {}, cM[B] = {}, cP[B] = {}, nX[B] = {}, nM[B] = {}, nP[B] = {};
        // loads are unconditional with clamped indices (n >= 2), so every wait covers
        // exactly the batch about to be used
        auto fload = [&](int i0, double* bx, double* bm, double* bp) {
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int i = min(i0 + u, n - 2);
                bx[u] = X[IDX(i + 1)];
                bm[u] = mu[IDX(i)];
                bp[u] = pv[IDX(i)];
            }
        };
        double cur = X[IDX(0)] * scale;
        auto fwork = [&](int i0, const double* bx, const double* bm, const double* bp) {
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int i = i0 + u;
                if (i + 1 < n) {
                    double nxt = bx[u] * scale;
                    if (bp[u] != 0.0) {
                        const double tmp = cur;
                        cur = nxt;
                        nxt = tmp;
                    }
                    y[IDX(i)] = cur;
                    cur = nxt - bm[u] * cur;
                }
            }
        };
        // two alternating batch buffers, each loaded one batch ahead of its use
        if (n >= 2) fload(0, cX, cM, cP);
        for (int i0 = 0; i0 + 1 < n; i0 += 2 * B) {
            fload(i0 + B, nX, nM, nP);
            fwork(i0, cX, cM, cP);
            fload(i0 + 2 * B, cX, cM, cP);
            if (i0 + B + 1 < n) fwork(i0 + B, nX, nM, nP);
        }
        y[IDX(n - 1)] = cur;
        // back substitution with U: y -> X (steps i = n-1 .. 0)
        double cY[B] = {}, c1[B] = {}, c2[B] = {}, c0[B] = {}, nY[B] = {}, n1[B] = {}, n2[B] = {}, n0[B] = {};
        auto bload = [&](int i0, double* by, double* b1, double* b2, double* b0) {
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int i = max(i0 - u, 0);
                by[u] = y[IDX(i)];
                b1[u] = u1[IDX(i)];
                b2[u] = u2[IDX(i)];
                b0[u] = u0[IDX(i)];
            }
        };
        double x1 = 0.0, x2 = 0.0;
        double nrm = 0.0;
        auto bwork = [&](int i0, const double* by, const double* b1, const double* b2, const double* b0) {
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int i = i0 - u;
                if (i >= 0) {
                    const double xi = (by[u] - b1[u] * x1 - b2[u] * x2) * b0[u];
                    X[IDX(i)] = xi;
                    x2 = x1;
                    x1 = xi;
                    nrm = fma(xi, xi, nrm);
                }
            }
        };
        bload(n - 1, cY, c1, c2, c0);
        for (int i0 = n - 1; i0 >= 0; i0 -= 2 * B) {
            bload(i0 - B, nY, n1, n2, n0);
            bwork(i0, cY, c1, c2, c0);
            bload(i0 - 2 * B, cY, c1, c2, c0);
            if (i0 - B >= 0) bwork(i0 - B, nY, n1, n2, n0);
        }
        scale = 1.0 / sqrt(nrm);
    }
    // unit norm: read in batches, then write back
    for (int i0 = 0; i0 < n; i0 += B) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (i0 + u < n) v[u] = X[IDX(i0 + u)];
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (i0 + u < n) X[IDX(i0 + u)] = v[u] * scale;
    }
#undef IDX
}

// orders the LDS accesses of one wavefront before and after (its LDS operations execute
// in issue order; this keeps the compiler from reordering them)
__device__ inline void wave_sync_fence() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Eigenvectors of clustered eigenvalues (consecutive gaps below 1e-3 |T|) from
// inverse iteration span the cluster's invariant subspace but are not individually
// accurate.  One wavefront (one workgroup) per run of clustered eigenvalues (runs are
// found from the unrefined values w_in, split into chunks of at most 32): two
// Gram-Schmidt passes, then a Rayleigh-Ritz step on the chunk (Jacobi on X_c^T T X_c)
// that rotates the basis into eigenvectors and refines the eigenvalues (written to w).
// The chunk's columns are held contiguously (one strided read and one strided write of
// X per chunk; every pass in between reads contiguous vectors): in LDS for chunks of up
// to CLUSTER_LDS_COLS columns, so the chains of dependent dot products wait on LDS
// rather than on memory; wider chunks use rows start .. start + cs - 1 of the n x n
// scratch Xn.  Both forms do the same operations in the same order.
constexpr int CLUSTER_LDS_COLS = 16;

__device__ __forceinline__ void cluster_chunk(int n, int start, int cs, double* xc0, const double* __restrict__ dg,
                                              const double* __restrict__ eg, double* __restrict__ w,
                                              double* __restrict__ X, double* Tc, double* Qc, int lane) {
    // the chunk's columns, contiguous: xc(q) = column start + q of X
    auto xc = [&](const int q) { return xc0 + (long long)q * n; };
    for (int i = lane; i < n; i += 64)
        for (int q = 0; q < cs; ++q) xc(q)[i] = X[(long long)i * n + start + q];
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    // two Gram-Schmidt passes over the chunk's columns
    for (int c = 0; c < cs; ++c) {
        double* vc = xc(c);
        for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < c; ++q) {
                const double* vq = xc(q);
                double acc = 0.0;
                for (int i = lane; i < n; i += 64) acc = fma(vq[i], vc[i], acc);
                const double cq = wave_sum_d(acc);
                for (int i = lane; i < n; i += 64) vc[i] -= cq * vq[i];
            }
        double acc = 0.0;
        for (int i = lane; i < n; i += 64) acc = fma(vc[i], vc[i], acc);
        const double inv = 1.0 / sqrt(wave_sum_d(acc));
        for (int i = lane; i < n; i += 64) vc[i] *= inv;
    }
    // the product with T reads neighbours that other lanes wrote: their stores complete first
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    // Tc = X_c^T T X_c
    for (int pp = 0; pp < cs; ++pp)
        for (int qq = pp; qq < cs; ++qq) {
            const double* vp = xc(pp);
            const double* vq = xc(qq);
            double acc = 0.0;
            for (int i = lane; i < n; i += 64) {
                double tx = dg[i] * vq[i];
                if (i > 0) tx = fma(eg[i - 1], vq[i - 1], tx);
                if (i + 1 < n) tx = fma(eg[i], vq[i + 1], tx);
                acc = fma(vp[i], tx, acc);
            }
            const double v = wave_sum_d(acc);
            if (lane == 0) {
                Tc[pp * 33 + qq] = v;
                Tc[qq * 33 + pp] = v;
            }
        }
    __builtin_amdgcn_wave_barrier();
    // cyclic Jacobi on the cs x cs matrix: every lane computes the same rotation and
    // lane k updates entry k of the two rows and columns (each rotation applies the
    // column updates, then the row updates, as a serial sweep would)
    for (int e2 = lane; e2 < cs * 33; e2 += 64) Qc[e2] = (e2 % 33 == e2 / 33) ? 1.0 : 0.0;
    wave_sync_fence();
    for (int sweep = 0; sweep < 50; ++sweep) {
        bool rot = false;
        for (int pp = 0; pp < cs; ++pp)
            for (int qq = pp + 1; qq < cs; ++qq) {
                const double apq = Tc[pp * 33 + qq];
                const double app = Tc[pp * 33 + pp], aqq = Tc[qq * 33 + qq];
                if (!(fabs(apq) > 2.3e-16 * sqrt(fabs(app * aqq))) || apq == 0.0) continue;
                rot = true;
                const double tau = (aqq - app) / (2.0 * apq);
                const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + tt * tt), sn = tt * c;
                const int k = lane;
                if (k < cs) {
                    const double akp = Tc[k * 33 + pp], akq = Tc[k * 33 + qq];
                    Tc[k * 33 + pp] = c * akp - sn * akq;
                    Tc[k * 33 + qq] = sn * akp + c * akq;
                }
                wave_sync_fence();
                if (k < cs) {
                    const double apk = Tc[pp * 33 + k], aqk = Tc[qq * 33 + k];
                    const double vkp = Qc[k * 33 + pp], vkq = Qc[k * 33 + qq];
                    Qc[k * 33 + pp] = c * vkp - sn * vkq;
                    Qc[k * 33 + qq] = sn * vkp + c * vkq;
                    Tc[pp * 33 + k] = c * apk - sn * aqk;
                    Tc[qq * 33 + k] = sn * apk + c * aqk;
                }
                wave_sync_fence();
                if (lane == 0) {
                    Tc[pp * 33 + qq] = 0.0;
                    Tc[qq * 33 + pp] = 0.0;
                }
                wave_sync_fence();
            }
        if (!rot) break;
    }
    if (lane == 0) {
        for (int pp = 0; pp < cs; ++pp) {          // selection sort of the pairs
            int best = pp;
            for (int qq = pp + 1; qq < cs; ++qq)
                if (Tc[qq * 33 + qq] < Tc[best * 33 + best]) best = qq;
            if (best != pp) {
                const double tmp = Tc[pp * 33 + pp];
                Tc[pp * 33 + pp] = Tc[best * 33 + best];
                Tc[best * 33 + best] = tmp;
                for (int k = 0; k < cs; ++k) {
                    const double v = Qc[k * 33 + pp];
                    Qc[k * 33 + pp] = Qc[k * 33 + best];
                    Qc[k * 33 + best] = v;
                }
            }
            w[start + pp] = Tc[pp * 33 + pp];
        }
    }
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    // X_c <- X_c Q_c, from the contiguous copy into the columns of X
    for (int i = lane; i < n; i += 64)
        for (int q = 0; q < cs; ++q) {
            double v = 0.0;
            for (int pp = 0; pp < cs; ++pp) v = fma(xc(pp)[i], Qc[pp * 33 + q], v);
            X[(long long)i * n + start + q] = v;
        }
    // the next chunk of the run overwrites the LDS copy
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__global__ __launch_bounds__(64) void tridiag_cluster_kernel(int n, const double* __restrict__ dg,
                                                             const double* __restrict__ eg,
                                                             const double* __restrict__ w_in, double* __restrict__ w,
                                                             double* __restrict__ X, double* __restrict__ Xn) {
    __shared__ double xs[CLUSTER_LDS_COLS * 1024];    // n <= 1024
    __shared__ double Tc[32 * 33];
    __shared__ double Qc[32 * 33];
    const int lane = threadIdx.x;
    const int j = blockIdx.x;
    if (j >= n) return;
    const double tn = fmax(fabs(w_in[0]), fabs(w_in[n - 1]));
    const double gap_tol = 1e-3 * tn;
    if (j > 0 && w_in[j] - w_in[j - 1] <= gap_tol) return;     // not the start of a run
    int e = j + 1;
    while (e < n && w_in[e] - w_in[e - 1] <= gap_tol) ++e;
    if (e - j == 1) return;
    for (int start = j; start < e; start += 32) {
        const int cs = min(32, e - start);
        if (cs < 2) break;
        if (cs <= CLUSTER_LDS_COLS)
            cluster_chunk(n, start, cs, xs, dg, eg, w, X, Tc, Qc, lane);
        else
            cluster_chunk(n, start, cs, Xn + (long long)start * n, dg, eg, w, X, Tc, Qc, lane);
    }
}

// Z <- H_0 H_1 ... H_{n-3} Z (eigenvectors of the reduced matrix back to the original
// basis).  One wavefront per column: the column stays in registers, lane l holding rows
// l, l + 64, ... (RPL rows per lane, n <= 64 RPL); each reflector costs a coalesced read
// of v, a DPP wave reduction and an update.  Reflectors are read D steps ahead into a
// register ring (fixed slots: the loop is unrolled by D), tau from an LDS copy.
template <int RPL, int D>
__global__ __launch_bounds__(256) void tridiag_back_kernel(int n, const double* __restrict__ Vh,
                                                           const double* __restrict__ tau, double* __restrict__ Z) {
    __shared__ double ts[1024];
    for (int i = threadIdx.x; i < n; i += blockDim.x) ts[i] = tau[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;
    double z[RPL], vb[D][RPL], tb[D];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        z[r] = (i < n) ? Z[i * n + j] : 0.0;
    }
    // raw row k of Vh (indices clamped into the matrix); entries i <= k are masked
    // to zero when the reflector is applied
    auto load_v = [&](int k, double* dst, double& t) {
        const int kc = max(k, 0);
#pragma unroll
        for (int r = 0; r < RPL; ++r) dst[r] = Vh[kc * n + min(lane + 64 * r, n - 1)];
        t = ts[kc];
    };
    // reflector k = n - 3 - step is applied at step 0, 1, ..., n - 3
#pragma unroll
    for (int u = 0; u < D; ++u) load_v(n - 3 - u, vb[u], tb[u]);
    for (int s0 = 0; s0 + 2 < n; s0 += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            // steps past the last reflector (k < 0) have v = 0 and leave z unchanged, so
            // the unrolled body has no branches and every load is counted exactly
            const int k = n - 3 - (s0 + u);
            double v[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                v[r] = (k >= 0 && i > k && i < n) ? vb[u][r] : 0.0;
            }
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) acc = fma(v[r], z[r], acc);
            const double dk = tb[u] * wave_sum_dpp(acc);
#pragma unroll
            for (int r = 0; r < RPL; ++r) z[r] = fma(-dk, v[r], z[r]);
            load_v(k - D, vb[u], tb[u]);
            __builtin_amdgcn_sched_barrier(0);     // keep the prefetch D steps ahead of its use
        }
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i < n) Z[i * n + j] = z[r];
    }
}

void launch_sym_eig(hipStream_t st, int n, double* A, double* w, double* V, double* work, double* small,
                    double* scratch, int* status) {
    // work: n*n (reflectors); small: 6n + 1 (tau, diag, off, unrefined eigenvalues, the two
    // buffers of A22 v, one spare entry);
    // scratch: 6 n*n (inverse iteration, then the cluster rotation)
    double* tau = small;
    double* diag = small + n;
    double* off = small + 2 * n;
    double* w0 = small + 3 * n;
    double* pbuf = small + 4 * n;
    double* wbuf = small + 5 * n;
    if (n <= TRIDIAG_ONE_WG_MAX) {
        // small matrices: one workgroup does every step (no per-column launches)
        hipLaunchKernelGGL(tridiag_kernel, dim3(1), dim3(512), 0, st, n, A, work, tau, diag, off);
    } else {
        // p of step k goes to pb[k & 1]; the last 2 x 2 block is the head of step n - 2,
        // with 256 threads like the heads formed inside the steps
        double* pb[2] = {pbuf, wbuf};
        hipLaunchKernelGGL(tridiag_head_kernel, dim3(1), dim3(1024), 0, st, n, 0, A, work, tau, pbuf, wbuf, diag, off);
        for (int k = 0; k + 2 < n; ++k)
            hipLaunchKernelGGL(tridiag_step_kernel, dim3(grid_for(n - k - 1, 4)), dim3(256), 0, st, n, k, A, work,
                               tau, pb[(k + 1) & 1], pb[k & 1], diag, off);
        hipLaunchKernelGGL(tridiag_head_kernel, dim3(1), dim3(256), 0, st, n, n - 2, A, work, tau, pb[(n - 3) & 1],
                           pb[(n - 2) & 1], diag, off);
    }
    hipLaunchKernelGGL(tridiag_bisect_kernel, dim3(grid_for((long long)n * BISECT_G, 256)), dim3(256), 0, st, n, diag,
                       off, w0);
    const long long n2 = (long long)n * n;
    hipLaunchKernelGGL(tridiag_invit_kernel, dim3(grid_for(n, 64)), dim3(64), 0, st, n, diag, off, w0, V, scratch,
                       scratch + n2, scratch + 2 * n2, scratch + 3 * n2, scratch + 4 * n2, scratch + 5 * n2);
    (void)hipMemcpyAsync(w, w0, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(tridiag_cluster_kernel, dim3(n), dim3(64), 0, st, n, diag, off, w0, w, V, scratch);
    if (n <= 256)
        hipLaunchKernelGGL((tridiag_back_kernel<4, 8>), dim3(grid_for(n, 4)), dim3(256), 0, st, n, work, tau, V);
    else if (n <= 512)
        hipLaunchKernelGGL((tridiag_back_kernel<8, 6>), dim3(grid_for(n, 4)), dim3(256), 0, st, n, work, tau, V);
    else
        hipLaunchKernelGGL((tridiag_back_kernel<16, 4>), dim3(grid_for(n, 4)), dim3(256), 0, st, n, work, tau, V);
}

// ---------------------------------------------------------------------------
// Cholesky-QR coefficients for a b x b Gram matrix G = T^T M T (b <= 64):
// S = D^{-1/2} G D^{-1/2}, S = L L^T, C = D^{-1/2} L^{-T}; T C is M-orthonormal.
// A direction whose pivot falls below the drop tolerance is linearly dependent
// on the previous ones: its column of C is zero and dropped[j] = 1.
__global__ void cholqr_coef_kernel(int b, const double* __restrict__ G, double* __restrict__ C,
                                   int* __restrict__ dropped, int* __restrict__ status) {
    __shared__ double S[64 * 64];
    __shared__ double Li[64 * 64];
    __shared__ double dsc[64];
    __shared__ int drop[64];
    const int t = threadIdx.x, bd = blockDim.x;
    for (int j = t; j < b; j += bd) {
        const double d = G[j * b + j];
        const bool ok = (d > 0.0) && isfinite(d);
        dsc[j] = ok ? 1.0 / sqrt(d) : 0.0;
        drop[j] = ok ? 0 : 1;
    }
    __syncthreads();
    for (int e = t; e < b * b; e += bd) {
        const int i = e / b, j = e % b;
        S[e] = 0.5 * (G[i * b + j] + G[j * b + i]) * dsc[i] * dsc[j];
    }
    __syncthreads();
    for (int k = 0; k < b; ++k) {
        if (t == 0) {
            const double p = S[k * b + k];
            if (drop[k] || !(p > 1e-13)) {
                drop[k] = 1;
                S[k * b + k] = 1.0;
            } else {
                S[k * b + k] = sqrt(p);
            }
        }
        __syncthreads();
        const double piv = S[k * b + k];
        const bool dk = drop[k] != 0;
        for (int i = k + 1 + t; i < b; i += bd) S[i * b + k] = dk ? 0.0 : S[i * b + k] / piv;
        __syncthreads();
        for (int e = t; e < b * b; e += bd) {
            const int i = e / b, j = e % b;
            if (i > k && j > k && j <= i) S[i * b + j] -= S[i * b + k] * S[j * b + k];
        }
        __syncthreads();
    }
    // Li = L^{-1}, one column per thread (forward substitution on unit vectors)
    for (int c = t; c < b; c += bd) {
        for (int r = 0; r < b; ++r) {
            double acc = (r == c) ? 1.0 : 0.0;
            for (int q = c; q < r; ++q) acc -= S[r * b + q] * Li[q * b + c];
            Li[r * b + c] = (r < c) ? 0.0 : acc / S[r * b + r];
        }
    }
    __syncthreads();
    // C = D^{-1/2} Li^T, dropped columns zeroed
    for (int e = t; e < b * b; e += bd) {
        const int i = e / b, j = e % b;
        C[e] = drop[j] ? 0.0 : dsc[i] * Li[j * b + i];
    }
    for (int j = t; j < b; j += bd) {
        dropped[j] = drop[j];
        if (drop[j]) atomicOr(status, STATUS_GRAM_DROP);
    }
}

void launch_cholqr_coef(hipStream_t st, int b, const double* G, double* C, int* dropped, int* status) {
    hipLaunchKernelGGL(cholqr_coef_kernel, dim3(1), dim3(256), 0, st, b, G, C, dropped, status);
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz coefficients on the m x m projected matrix H = W^T K W (m <= RR_MAX,
// s <= RR_S_MAX), one workgroup of 256 threads.  W = [X | P | T] (or [X | T]) is
// M-orthonormal except for dropped (zero) columns (drop_in), which are left out; the
// update only needs the s lowest Ritz pairs Q_s, Theta_s:
//   1. Householder reduction of the kept block to tridiagonal T (reflectors kept);
//   2. the s lowest eigenvalues of T by multisection on Sturm counts;
//   3. their eigenvectors by two inverse-iteration solves with a pivoted LU of T - theta I
//      (distinct start vectors per eigenvalue, so degenerate pairs span their subspace);
//   4. two classical Gram-Schmidt passes over them, then the reflectors back;
//   5. C_p: the part of span{E_x, Q_s} orthogonal to Q_s (E_x = old X coordinates), so
//      that span{W Q_s, W C_p} = U^k + U^{k+1}: b_j = (I - Q_s Q_s^T) e_j with two CGS
//      passes against Q_s and the previous columns; a direction whose norm is then
//      below 1e-12 (the old Ritz vector already lies in the new span) is dropped (zero
//      column, drop_out[s + j] = 1); drop_out[0..s) = 0.
// Wavefront 0 works on row i of the kept block (and of every vector in steps 4 to 6)
// in lane i, with the data in LDS, so the reduction, the Gram-Schmidt passes, the
// back-transformation and C_p need no workgroup barriers; the multisection uses all
// four wavefronts.  The loops stay compact: the kernel runs once per iteration, so
// fully unrolled code would be fetched from L2 instruction by instruction.
// Outputs theta[0..s) ascending (theta[s..m) = +inf) and Cfull = [Q_s | C_p] (m x cw).
constexpr int RR_S_MAX = BPJD_MAX_BLOCK;

__device__ inline void wave_lds_sync() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// S[c] = sum over the wavefront's 64 lanes of v[c] for c < cnt (<= RR_S_MAX), every lane
// receiving every sum.  Sixteen columns at a time through an LDS transpose (buf: 64 x 17
// doubles): lane l adds column l % 16 over rows l / 16, l / 16 + 4, ... (four chains),
// then two lane exchanges combine the four lane groups, in a fixed order.
__device__ inline void wave_sums16(const double (&v)[RR_S_MAX], double (&S)[RR_S_MAX], int cnt, double* buf,
                                   int lane) {
#pragma unroll
    for (int base = 0; base < RR_S_MAX; base += 16) {
        if (base < cnt) {
#pragma unroll
            for (int c = 0; c < 16; ++c) buf[lane * 17 + c] = (base + c < RR_S_MAX) ? v[base + c] : 0.0;
            wave_lds_sync();
            const int c = lane & 15, r0 = lane >> 4;
            double part[4] = {0.0, 0.0, 0.0, 0.0};     // four chains, added pairwise
#pragma unroll
            for (int r = 0; r < 16; ++r) part[r & 3] += buf[(r0 + 4 * r) * 17 + c];
            double acc = (part[0] + part[1]) + (part[2] + part[3]);
            wave_lds_sync();
            acc += __shfl_xor(acc, 16, 64);
            acc += __shfl_xor(acc, 32, 64);
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (base + k < RR_S_MAX) S[base + k] = lane_bcast(acc, k);
        }
    }
}

template <int NM>
__global__ __launch_bounds__(256) void rr_coef_kernel(int m, int s, int with_p, const double* __restrict__ H,
                                                      const int* __restrict__ drop_in, int* __restrict__ drop_out,
                                                      double* __restrict__ theta, double* __restrict__ lam,
                                                      double* __restrict__ Cfull) {
    constexpr int SD = RR_S_MAX + 1;
    __shared__ double Al[NM][NM + 1];               // the kept block, reduced in place
    __shared__ double vL[64], wL[64];
    __shared__ double dd[NM], ee[NM], e2[NM], tauv[NM], wv[RR_S_MAX];
    __shared__ double Zs[NM * SD];                  // eigenvectors of T, then of the kept block (n x ns)
    __shared__ double Qs[NM * SD];                  // Q_s in all coordinates (m x s)
    __shared__ double Vk[NM][64];                   // reflector k (row = lane), then C_p columns
    __shared__ double bL[64], cL[2 * RR_S_MAX + 1];
    __shared__ double iu0[RR_S_MAX * NM], iu1[RR_S_MAX * NM], iu2[RR_S_MAX * NM], iy[RR_S_MAX * NM];
    __shared__ int keep_idx[NM];
    __shared__ int mk;
    __shared__ double tbuf[64 * 17];               // wave_sums16's transposition
    const int t = threadIdx.x, lane = t & 63;
    const bool w0 = t < 64;
    if (t == 0) {
        int c = 0;
        for (int i = 0; i < m; ++i)
            if (!drop_in[i]) keep_idx[c++] = i;
        mk = c;
        for (int i = c; i < NM; ++i) keep_idx[i] = 0;
    }
    __syncthreads();
    const int n = mk;
    const int ns = min(s, n);
    // 1. reduction to tridiagonal form (wavefront 0, lane i = row i of the kept block in
    //    LDS); a compact loop, so the code stays in the instruction cache
    if (w0) {
        if (lane < n) {
            const int gi = keep_idx[lane];
            for (int j = 0; j < n; ++j) {
                const int gj = keep_idx[j];
                Al[lane][j] = 0.5 * (H[gi * m + gj] + H[gj * m + gi]);
            }
        }
        wave_lds_sync();
        for (int k = 0; k + 2 < n; ++k) {
            const double xk = (lane < n) ? Al[lane][k] : 0.0;
            const double xn2 = wave_sum_dpp(lane >= k + 2 ? xk * xk : 0.0);
            const double alpha = lane_bcast(xk, k + 1);
            const double dk = lane_bcast(xk, k);
            double tk = 0.0, scale = 0.0, beta = alpha;
            if (xn2 != 0.0) {
                beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
                tk = (beta - alpha) * rcp_refined(beta);
                scale = rcp_refined(alpha - beta);
            }
            const double vi = (lane == k + 1) ? 1.0 : ((lane >= k + 2 && lane < n) ? xk * scale : 0.0);
            Vk[k][lane] = vi;
            if (lane == 0) {
                tauv[k] = tk;
                dd[k] = dk;
                ee[k] = beta;
            }
            if (tk != 0.0) {
                // p = tau A22 v (rows k+1..), w = p - (tau/2)(p^T v) v, A22 -= v w^T + w v^T
                vL[lane] = vi;
                wave_lds_sync();
                double p = 0.0;
                if (lane > k && lane < n) p = tk * dot_strided(&Al[lane][k + 1], 1, &vL[k + 1], 1, n - k - 1);
                const double pv = wave_sum_dpp(p * vi);
                const double wi = p - 0.5 * tk * pv * vi;
                wL[lane] = wi;
                wave_lds_sync();
                if (lane > k && lane < n)
                    for (int j = k + 1; j < n; ++j) Al[lane][j] -= vi * wL[j] + wi * vL[j];
                wave_lds_sync();
            }
        }
        if (lane == 0) {
            if (n >= 2) {
                dd[n - 2] = Al[n - 2][n - 2];
                ee[n - 2] = Al[n - 1][n - 2];
                dd[n - 1] = Al[n - 1][n - 1];
            } else if (n == 1) {
                dd[0] = Al[0][0];
            }
            if (n >= 1) ee[n - 1] = 0.0;
        }
    }
    __syncthreads();
    for (int i = t; i < n; i += blockDim.x) e2[i] = ee[i] * ee[i];
    double glo = 1e300, ghi = -1e300;
    for (int i = 0; i < n; ++i) {
        const double el = (i > 0) ? fabs(ee[i - 1]) : 0.0, er = fabs(ee[i]);
        glo = fmin(glo, dd[i] - el - er);
        ghi = fmax(ghi, dd[i] + el + er);
    }
    __syncthreads();
    const double tnorm = fmax(fabs(glo), fabs(ghi));
    const double pivmin = 1e-300 + 1e-30 * tnorm * tnorm;
    // 2. the ns lowest eigenvalues: G threads per eigenvalue (G divides 64)
    {
        const int G = (ns <= 8) ? 32 : ((ns <= 16) ? 16 : 8);
        const int j = t / G, r = t % G;
        const int gl = (t & 63) - r;
        bool done = j >= ns;
        double a = glo - 1e-14 * tnorm - 1e-300, b = ghi + 1e-14 * tnorm + 1e-300;
        for (int it = 0; it < 200 && __any(!done); ++it) {
            if (!done && (!(0.5 * (a + b) > a && 0.5 * (a + b) < b) ||
                          (b - a) <= 2.3e-16 * fmax(fabs(a), fabs(b))))
                done = true;
            const double x = a + (b - a) / (double)(G + 1) * (double)(r + 1);
            const bool above = !done && sturm_count(n, dd, e2, x, pivmin) > j;
            // the first of the group's points whose count exceeds j closes the interval
            const unsigned long long grp = (__ballot(above) >> gl) & ((1ull << G) - 1ull);
            if (!done) {
                const double h = (b - a) / (double)(G + 1);
                if (grp) {
                    const int q = __ffsll((long long)grp) - 1;
                    const double na = (q > 0) ? a + h * (double)q : a;
                    b = a + h * (double)(q + 1);
                    a = na;
                } else {
                    a = a + h * (double)G;
                }
            }
        }
        if (j < ns && r == 0) wv[j] = 0.5 * (a + b);
    }
    __syncthreads();
    // 3. inverse iteration, thread j: solve (T - theta_j I) x = b twice with a partial-
    //    pivoting LU (U has two super-diagonals), refactoring on the fly each solve; the
    //    start vector is a fixed integer hash of (i, j)
    if (t < ns) {
        const int j = t;
        const double lmb = wv[j];
        const double tiny = 2.3e-16 * fmax(tnorm, 1e-300);
        double* u0 = iu0 + j * NM;                 // reciprocal pivots
        double* u1 = iu1 + j * NM;
        double* u2 = iu2 + j * NM;
        double* y = iy + j * NM;
        for (int i = 0; i < n; ++i)
            y[i] = 0.5 + (double)((((unsigned int)i + 1u) * 2654435761u + ((unsigned int)j + 1u) * 40503u) >> 22) / 1024.0;
        auto guard = [&](double p) { return (fabs(p) < tiny) ? copysign(tiny, p == 0.0 ? 1.0 : p) : p; };
        for (int sweep = 0; sweep < 2; ++sweep) {
            double a0 = dd[0] - lmb, a1 = (n > 1) ? ee[0] : 0.0, a2 = 0.0;
            double yc = y[0];
            for (int i = 0; i + 1 < n; ++i) {
                const double sub = ee[i], nd = dd[i + 1] - lmb, ne = (i + 2 < n) ? ee[i + 1] : 0.0;
                double yn = y[i + 1];
                double p0, p1, p2;
                if (fabs(sub) > fabs(a0)) {
                    const double mlt = a0 * rcp_refined(sub);
                    p0 = sub;
                    p1 = nd;
                    p2 = ne;
                    const double tmp = yc;
                    yc = yn;
                    yn = tmp - mlt * yn;
                    const double na0 = a1 - mlt * nd, na1 = a2 - mlt * ne;
                    a0 = na0;
                    a1 = na1;
                } else {
                    const double piv = guard(a0);
                    const double mlt = sub * rcp_refined(piv);
                    p0 = piv;
                    p1 = a1;
                    p2 = a2;
                    yn = yn - mlt * yc;
                    a0 = nd - mlt * a1;
                    a1 = ne - mlt * a2;
                }
                a2 = 0.0;
                u0[i] = rcp_refined(guard(p0));
                u1[i] = p1;
                u2[i] = p2;
                y[i] = yc;
                yc = yn;
            }
            u0[n - 1] = rcp_refined(guard(a0));
            u1[n - 1] = 0.0;                       // no super-diagonals in the last row
            u2[n - 1] = 0.0;
            y[n - 1] = yc;
            double x1 = 0.0, x2 = 0.0, nrm = 0.0;
            for (int i = n - 1; i >= 0; --i) {
                const double xi = (y[i] - u1[i] * x1 - u2[i] * x2) * u0[i];
                y[i] = xi;
                x2 = x1;
                x1 = xi;
                nrm = fma(xi, xi, nrm);
            }
            const double inv = 1.0 / sqrt(nrm);
            for (int i = 0; i < n; ++i) y[i] *= inv;
        }
        for (int i = 0; i < n; ++i) Zs[i * SD + j] = y[i];
    }
    __syncthreads();
    if (!w0) return;
    // Steps 4 to 6 run in wavefront 0 with row i of every vector in registers of lane i
    // (compile-time column loops, guarded by the uniform counts); the inner products of
    // a step are lane-parallel products summed together by wave_sums16.
    // 4. two CGS passes over the ns vectors (columns of Z), then Z <- H_0 ... H_{n-3} Z
    double z[RR_S_MAX], pr[RR_S_MAX], S[RR_S_MAX];
#pragma unroll
    for (int c = 0; c < RR_S_MAX; ++c) {
        z[c] = (lane < n && c < ns) ? Zs[lane * SD + c] : 0.0;
        S[c] = 0.0;
    }
    for (int j = 0; j < ns; ++j) {
        double zj = 0.0;
#pragma unroll
        for (int c = 0; c < RR_S_MAX; ++c)
            if (c == j) zj = z[c];
        for (int pass = 0; pass < 2 && j > 0; ++pass) {
#pragma unroll
            for (int c = 0; c < RR_S_MAX; ++c) pr[c] = (c < j) ? z[c] * zj : 0.0;
            wave_sums16(pr, S, j, tbuf, lane);
            double upd = 0.0;
#pragma unroll
            for (int c = 0; c < RR_S_MAX; ++c)
                if (c < j) upd = fma(S[c], z[c], upd);
            zj -= upd;
        }
        zj *= 1.0 / sqrt(wave_sum_dpp(zj * zj));
#pragma unroll
        for (int c = 0; c < RR_S_MAX; ++c)
            if (c == j) z[c] = zj;
    }
    for (int k = n - 3; k >= 0; --k) {
        const double tk = tauv[k];
        if (tk == 0.0) continue;
        // Z -= v_k (tau_k v_k^T Z); v_k is zero outside rows k + 1 .. n - 1
        const double vi = (lane < n) ? Vk[k][lane] : 0.0;
#pragma unroll
        for (int c = 0; c < RR_S_MAX; ++c) pr[c] = (c < ns) ? vi * z[c] : 0.0;
        wave_sums16(pr, S, ns, tbuf, lane);
#pragma unroll
        for (int c = 0; c < RR_S_MAX; ++c)
            if (c < ns) z[c] -= (tk * S[c]) * vi;
    }
    // 5. Q_s in all coordinates (row r in lane r); missing pairs (fewer kept columns
    //    than s) are unit vectors of dropped coordinates with an infinite value
    for (int e = lane; e < m * SD; e += 64) Qs[e] = 0.0;
    wave_lds_sync();
    if (lane < n)
#pragma unroll
        for (int c = 0; c < RR_S_MAX; ++c)
            if (c < ns) Qs[keep_idx[lane] * SD + c] = z[c];
    if (lane == 0) {
        int c = ns;
        for (int i = 0; i < m && c < s; ++i)
            if (drop_in[i]) {
                Qs[i * SD + c] = 1.0;
                wv[c] = INFINITY;
                ++c;
            }
    }
    wave_lds_sync();
    const int cw = with_p ? 2 * s : s;
    for (int i = lane; i < m; i += 64) theta[i] = (i < s) ? wv[i] : INFINITY;
    if (lane < s) lam[lane] = wv[lane];             // the new shifts
    if (lane < m)
        for (int c = 0; c < s; ++c) Cfull[lane * cw + c] = Qs[lane * SD + c];
    if (lane < cw) drop_out[lane] = 0;
    if (!with_p) return;
    // 6. C_p: b_j = e_j - Q_s Q_s[j, :]^T, two CGS passes against Q_s and the C_p columns
    //    so far; row lane of Q_s in q, of C_p in cp
    double q[RR_S_MAX], cp[RR_S_MAX], S2[RR_S_MAX];
#pragma unroll
    for (int c = 0; c < RR_S_MAX; ++c) {
        q[c] = (lane < m && c < s) ? Qs[lane * SD + c] : 0.0;
        cp[c] = 0.0;
        S2[c] = 0.0;
    }
    for (int j = 0; j < s; ++j) {
        double dq = 0.0;
#pragma unroll
        for (int c = 0; c < RR_S_MAX; ++c)
            if (c < s) dq = fma(q[c], Qs[j * SD + c], dq);
        double bj = (lane < m) ? (((lane == j) ? 1.0 : 0.0) - dq) : 0.0;
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
            for (int c = 0; c < RR_S_MAX; ++c) pr[c] = (c < s) ? bj * q[c] : 0.0;
            wave_sums16(pr, S, s, tbuf, lane);
            if (j > 0) {
#pragma unroll
                for (int c = 0; c < RR_S_MAX; ++c) pr[c] = (c < j) ? bj * cp[c] : 0.0;
                wave_sums16(pr, S2, j, tbuf, lane);
            }
            double upd = 0.0;
#pragma unroll
            for (int c = 0; c < RR_S_MAX; ++c)
                if (c < s) upd = fma(S[c], q[c], upd);
#pragma unroll
            for (int c = 0; c < RR_S_MAX; ++c)
                if (c < j) upd = fma(S2[c], cp[c], upd);
            bj -= upd;
        }
        const double nrm = sqrt(wave_sum_dpp(bj * bj));
        const bool keep = nrm > 1e-12;
        const double cpj = (lane < m && keep) ? bj * (1.0 / nrm) : 0.0;
#pragma unroll
        for (int c = 0; c < RR_S_MAX; ++c)
            if (c == j) cp[c] = cpj;
        if (lane == 0) drop_out[s + j] = keep ? 0 : 1;
        if (lane < m) Cfull[lane * cw + s + j] = cpj;
    }
}

// Rows and columns m .. m + s - 1 of the projected matrix of a growing basis (one
// workgroup): off-diagonal entries from the new Gram block, the new diagonal block
// symmetrised, and dropped columns decoupled with a diagonal entry above every
// eigenvalue (H is positive semidefinite, so 4 trace + 1 exceeds its spectrum).
__global__ __launch_bounds__(256) void grow_place_kernel(int m, int s, const double* __restrict__ C,
                                                         const int* __restrict__ dropped, double* __restrict__ H,
                                                         int ldh) {
    const int t = threadIdx.x;
    const int mn = m + s;
    for (int e = t; e < mn * s; e += blockDim.x) {
        const int r = e / s, c = e - r * s;
        const int j = m + c;
        double v;
        if (r < m) {
            v = C[e];
        } else {
            const int c2 = r - m;
            v = 0.5 * (C[e] + C[(m + c) * s + c2]);
        }
        if (dropped[j] || dropped[r]) v = 0.0;
        H[(long long)r * ldh + j] = v;
        H[(long long)j * ldh + r] = v;
    }
    __syncthreads();
    if (t == 0) {
        double tr = 0.0;
        for (int j = 0; j < mn; ++j)
            if (!dropped[j]) tr += fabs(H[(long long)j * ldh + j]);
        for (int j = 0; j < mn; ++j)
            if (dropped[j]) H[(long long)j * ldh + j] = 4.0 * tr + 1.0;
    }
}

void launch_grow_place(hipStream_t st, int m, int s, const double* C, const int* dropped, double* H, int ldh) {
    hipLaunchKernelGGL(grow_place_kernel, dim3(1), dim3(256), 0, st, m, s, C, dropped, H, ldh);
}

void launch_rr_coef(hipStream_t st, int m, int s, int with_p, const double* H, const int* drop_in, int* drop_out,
                    double* theta, double* lam, double* Cfull) {
    if (m <= 24)
        hipLaunchKernelGGL(rr_coef_kernel<24>, dim3(1), dim3(256), 0, st, m, s, with_p, H, drop_in, drop_out, theta,
                           lam, Cfull);
    else if (m <= 48)
        hipLaunchKernelGGL(rr_coef_kernel<48>, dim3(1), dim3(256), 0, st, m, s, with_p, H, drop_in, drop_out, theta,
                           lam, Cfull);
    else
        hipLaunchKernelGGL(rr_coef_kernel<64>, dim3(1), dim3(256), 0, st, m, s, with_p, H, drop_in, drop_out, theta,
                           lam, Cfull);
}

}  // namespace bpjd
