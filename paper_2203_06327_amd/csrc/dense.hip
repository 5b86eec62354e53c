// Small dense FP64 kernels that run in a single workgroup: Cholesky,
// triangular solves, the cyclic Jacobi symmetric eigensolver used for the
// coarse generalized eigenproblem (Section 3, coarse spectral split) and the
// Rayleigh-Ritz problem (Algorithm 3.1, Step 3), Cholesky-QR coefficients and
// the coefficient-space step that keeps W^{k+1} = U^{k-1} + U^k + span{t}.
#include "common.h"

namespace bpjd {

static constexpr int JACOBI_MAX_SWEEPS = 60;

// ---------------------------------------------------------------------------
// Right-looking Cholesky, lower, row-major, in place; upper part zeroed.
__global__ void cholesky_kernel(int n, double* __restrict__ A, int* __restrict__ status, int status_bit) {
    __shared__ double piv;
    __shared__ int bad;
    const int t = threadIdx.x, bd = blockDim.x;
    if (t == 0) bad = 0;
    for (int k = 0; k < n; ++k) {
        if (t == 0) {
            double d = A[(long long)k * n + k];
            if (!(d > 0.0) || !isfinite(d)) {
                bad = 1;
                d = 1.0;
            }
            piv = sqrt(d);
            A[(long long)k * n + k] = piv;
        }
        __syncthreads();
        const double inv = 1.0 / piv;
        for (int i = k + 1 + t; i < n; i += bd) A[(long long)i * n + k] *= inv;
        __syncthreads();
        const int m = n - k - 1;
        for (long long e = t; e < (long long)m * m; e += bd) {
            const int i = k + 1 + (int)(e / m), j = k + 1 + (int)(e % m);
            if (j <= i) A[(long long)i * n + j] -= A[(long long)i * n + k] * A[(long long)j * n + k];
        }
        __syncthreads();
    }
    for (long long e = t; e < (long long)n * n; e += bd) {
        const int i = (int)(e / n), j = (int)(e % n);
        if (j > i) A[e] = 0.0;
    }
    if (t == 0 && bad) atomicOr(status, status_bit);
}

void launch_cholesky(hipStream_t st, int n, double* A, int* status, int status_bit) {
    hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(1024), 0, st, n, A, status, status_bit);
}

// Triangular solve with many right-hand sides, right-looking: a workgroup owns
// 32 columns of B; for each row r it finishes x_r and updates the rows still to
// come (coalesced along the rows of B).
__global__ void trsm_lower_kernel(int n, int nrhs, const double* __restrict__ L, double* __restrict__ B, int ldb,
                                  int transposeL) {
    const int c0 = blockIdx.x * 32;
    const int t = threadIdx.x, bd = blockDim.x;
    const int nc = min(32, nrhs - c0);
    for (int step = 0; step < n; ++step) {
        const int r = transposeL ? (n - 1 - step) : step;
        const double inv = 1.0 / L[(long long)r * n + r];
        if (t < nc) B[(long long)r * ldb + c0 + t] *= inv;
        __syncthreads();
        // remaining rows q: forward q > r uses L[q][r]; backward (L^T) q < r uses L[r][q]
        const int qn = transposeL ? r : (n - 1 - r);
        for (int e = t; e < qn * 32; e += bd) {
            const int qi = e >> 5, c = e & 31;
            if (c >= nc) continue;
            const int q = transposeL ? qi : (r + 1 + qi);
            const double l = transposeL ? L[(long long)r * n + q] : L[(long long)q * n + r];
            B[(long long)q * ldb + c0 + c] -= l * B[(long long)r * ldb + c0 + c];
        }
        __syncthreads();
    }
}

void launch_trsm_lower(hipStream_t st, int n, int nrhs, const double* L, double* B, int ldb, bool transposeL) {
    hipLaunchKernelGGL(trsm_lower_kernel, dim3(grid_for(nrhs, 32)), dim3(256), 0, st, n, nrhs, L, B, ldb,
                       transposeL ? 1 : 0);
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
// Cyclic Jacobi with the round-robin (circle) ordering: every round applies
// N/2 disjoint rotations; a sweep is N-1 rounds.  A (n x n, symmetric) and V
// (n x n) may live in LDS or global memory.  On return A is diagonal to
// working precision and A_in = V diag(A) V^T.
__device__ void jacobi_core(int n, double* A, double* V, double* cs, int* pr, double* red) {
    __shared__ int rotated;
    const int t = threadIdx.x, bd = blockDim.x;
    const int N = n + (n & 1);
    const int half = N / 2;
    (void)red;
    for (long long e = t; e < (long long)n * n; e += bd) V[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
    __syncthreads();
    // Threshold Jacobi: a rotation is skipped when |a_pq| <= eps sqrt(|a_pp a_qq|); a
    // sweep without rotations ends the iteration (relative accuracy of every eigenvalue).
    for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
        if (t == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < N - 1; ++r) {
            for (int k = t; k < half; k += bd) {
                int p, q;
                if (k == 0) {
                    p = r;
                    q = N - 1;
                } else {
                    p = (r + k) % (N - 1);
                    q = (r - k + N - 1) % (N - 1);
                }
                if (p > q) {
                    const int tmp = p;
                    p = q;
                    q = tmp;
                }
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = A[(long long)p * n + q];
                    const double app = A[(long long)p * n + p], aqq = A[(long long)q * n + q];
                    if (fabs(apq) > 2.3e-16 * sqrt(fabs(app * aqq)) && apq != 0.0) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                        rotated = 1;
                    }
                }
                cs[2 * k] = c;
                cs[2 * k + 1] = s;
                pr[2 * k] = p;
                pr[2 * k + 1] = q;
            }
            __syncthreads();
            // rows p, q of A
            for (long long e = t; e < (long long)half * n; e += bd) {
                const int k = (int)(e / n), j = (int)(e % n);
                const double s = cs[2 * k + 1];
                const int q = pr[2 * k + 1];
                if (s == 0.0 || q >= n) continue;
                const double c = cs[2 * k];
                const int p = pr[2 * k];
                const double apj = A[(long long)p * n + j], aqj = A[(long long)q * n + j];
                A[(long long)p * n + j] = c * apj - s * aqj;
                A[(long long)q * n + j] = s * apj + c * aqj;
            }
            __syncthreads();
            // columns p, q of A and of V
            for (long long e = t; e < (long long)half * n; e += bd) {
                const int k = (int)(e / n), i = (int)(e % n);
                const double s = cs[2 * k + 1];
                const int q = pr[2 * k + 1];
                if (s == 0.0 || q >= n) continue;
                const double c = cs[2 * k];
                const int p = pr[2 * k];
                const double aip = A[(long long)i * n + p], aiq = A[(long long)i * n + q];
                A[(long long)i * n + p] = c * aip - s * aiq;
                A[(long long)i * n + q] = s * aip + c * aiq;
                const double vip = V[(long long)i * n + p], viq = V[(long long)i * n + q];
                V[(long long)i * n + p] = c * vip - s * viq;
                V[(long long)i * n + q] = s * vip + c * viq;
            }
            __syncthreads();
            // the rotation annihilates a_pq exactly; drop the rounding residue
            for (int k = t; k < half; k += bd) {
                const int q = pr[2 * k + 1];
                if (cs[2 * k + 1] != 0.0 && q < n) {
                    const int p = pr[2 * k];
                    A[(long long)p * n + q] = 0.0;
                    A[(long long)q * n + p] = 0.0;
                }
            }
            __syncthreads();
        }
        const int any = rotated;
        __syncthreads();
        if (!any) break;
    }
}

// Ascending order of the diagonal of A; writes w and the permuted columns of V.
__device__ void jacobi_sort(int n, const double* A, const double* V, double* w, double* Vout) {
    const int t = threadIdx.x, bd = blockDim.x;
    for (int i = t; i < n; i += bd) {
        const double di = A[(long long)i * n + i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double dj = A[(long long)j * n + j];
            rank += (dj < di) || (dj == di && j < i);
        }
        w[rank] = di;
        for (int r = 0; r < n; ++r) Vout[(long long)r * n + rank] = V[(long long)r * n + i];
    }
}

__global__ void jacobi_global_kernel(int n, double* __restrict__ A, double* __restrict__ w,
                                     double* __restrict__ Vout, double* __restrict__ work) {
    __shared__ double cs[2 * 1024];
    __shared__ int pr[2 * 1024];
    __shared__ double red[2 * 1024];
    jacobi_core(n, A, work, cs, pr, red);
    __syncthreads();
    jacobi_sort(n, A, work, w, Vout);
}

void launch_jacobi_eig(hipStream_t st, int n, double* A, double* w, double* V, double* work) {
    hipLaunchKernelGGL(jacobi_global_kernel, dim3(1), dim3(1024), 0, st, n, A, w, V, work);
}

// ---------------------------------------------------------------------------
// Dense symmetric eigensolver for the coarse problem (n <= 1024), in three
// single-workgroup kernels: Householder reduction to tridiagonal form, the
// implicit QL iteration with Wilkinson shifts on the tridiagonal matrix, and
// back-transformation by the stored reflectors.
//
// tridiag: A (n x n, full symmetric storage, row-major) is reduced in place;
// reflector k (acting on rows k+1..n-1) is v_k with v_k[0] = 1, stored in
// Vh[k][k+1..n) together with tau[k]; diag/off receive the tridiagonal matrix.
__global__ void tridiag_kernel(int n, double* __restrict__ A, double* __restrict__ Vh, double* __restrict__ tau,
                               double* __restrict__ diag, double* __restrict__ off) {
    __shared__ double v[1024];
    __shared__ double w[1024];
    __shared__ double red[1024];
    __shared__ double sc[4];
    const int t = threadIdx.x, bd = blockDim.x;
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        const double* colk = A + (long long)(k + 1) * n + k;     // x_i = A[k+1+i][k]
        double acc = 0.0;
        for (int i = 1 + t; i < m; i += bd) {
            const double x = colk[(long long)i * n];
            acc += x * x;
        }
        red[t] = acc;
        __syncthreads();
        for (int o = bd / 2; o > 0; o >>= 1) {
            if (t < o) red[t] += red[t + o];
            __syncthreads();
        }
        if (t == 0) {
            const double alpha = colk[0];
            const double xn2 = red[0];
            if (xn2 == 0.0) {
                sc[0] = 0.0;                 // tau
                sc[1] = 0.0;                 // scale
                off[k] = alpha;
            } else {
                const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
                sc[0] = (beta - alpha) / beta;
                sc[1] = 1.0 / (alpha - beta);
                off[k] = beta;
            }
            tau[k] = sc[0];
        }
        __syncthreads();
        const double tk = sc[0], scale = sc[1];
        for (int i = t; i < m; i += bd) {
            const double vi = (i == 0) ? 1.0 : colk[(long long)i * n] * scale;
            v[i] = vi;
            Vh[(long long)k * n + k + 1 + i] = vi;
        }
        __syncthreads();
        if (tk != 0.0) {
            // p = tau A22 v; A22 is symmetric, so thread j reads column j (coalesced across threads)
            for (int j = t; j < m; j += bd) {
                const double* colj = A + (long long)(k + 1) * n + (k + 1) + j;
                double pj = 0.0;
                for (int i = 0; i < m; ++i) pj = fma(colj[(long long)i * n], v[i], pj);
                w[j] = tk * pj;
            }
            __syncthreads();
            double pv = 0.0;
            for (int i = t; i < m; i += bd) pv += w[i] * v[i];
            red[t] = pv;
            __syncthreads();
            for (int o = bd / 2; o > 0; o >>= 1) {
                if (t < o) red[t] += red[t + o];
                __syncthreads();
            }
            const double half_tpv = 0.5 * tk * red[0];
            __syncthreads();
            for (int i = t; i < m; i += bd) w[i] -= half_tpv * v[i];
            __syncthreads();
            // A22 -= v w^T + w v^T, row by row with threads along the row
            for (int i = 0; i < m; ++i) {
                double* row = A + (long long)(k + 1 + i) * n + (k + 1);
                const double vi = v[i], wi = w[i];
                for (int j = t; j < m; j += bd) row[j] -= vi * w[j] + wi * v[j];
            }
        }
        __syncthreads();
    }
    for (int i = t; i < n; i += bd) diag[i] = A[(long long)i * n + i];
    if (t == 0) {
        if (n >= 2) off[n - 2] = A[(long long)(n - 1) * n + (n - 2)];
        off[n - 1] = 0.0;
    }
}

// Implicit QL with Wilkinson shifts on the symmetric tridiagonal matrix
// (diag d, off-diagonal e with e[i] coupling i and i+1).  Thread 0 runs the
// scalar recurrence of one sweep and records its Givens rotations in LDS; all
// threads then apply them to their rows of Z (Z starts as the identity).  On
// return d holds the eigenvalues (unordered) and the columns of Z the
// eigenvectors of the tridiagonal matrix.
__global__ void tridiag_ql_kernel(int n, double* __restrict__ dg, double* __restrict__ eg, double* __restrict__ Z,
                                  int* __restrict__ status) {
    __shared__ double d[1024];
    __shared__ double e[1024];
    __shared__ double rc[1024];
    __shared__ double rs[1024];
    __shared__ int s_first, s_last, s_stop;
    const int t = threadIdx.x, bd = blockDim.x;
    for (int i = t; i < n; i += bd) {
        d[i] = dg[i];
        e[i] = eg[i];
    }
    for (long long q = t; q < (long long)n * n; q += bd) Z[q] = ((q / n) == (q % n)) ? 1.0 : 0.0;
    __syncthreads();
    int l = 0, iter = 0;    // thread 0's state
    while (true) {
        if (t == 0) {
            s_stop = 1;
            while (l < n) {
                int m = l;
                while (m < n - 1 && fabs(e[m]) > 2.3e-16 * (fabs(d[m]) + fabs(d[m + 1]))) ++m;
                if (m == l) {
                    ++l;
                    iter = 0;
                    continue;
                }
                if (++iter > 100) {
                    atomicOr(status, STATUS_COARSE_NOT_SPD);
                    l = n;
                    break;
                }
                // shift from the leading 2 x 2 block of the unreduced part
                const double theta = (d[l + 1] - d[l]) / (2.0 * e[l]);
                const double rad = sqrt(theta * theta + 1.0);
                double g = d[m] - d[l] + e[l] / (theta + copysign(rad, theta));
                double sn = 1.0, cs = 1.0, shift_acc = 0.0;
                int i = m - 1;
                bool split = false;
                for (; i >= l; --i) {
                    const double f = sn * e[i];
                    const double b = cs * e[i];
                    const double r = sqrt(f * f + g * g);
                    e[i + 1] = r;
                    if (r == 0.0) {               // the block splits: undo the pending shift and restart
                        d[i + 1] -= shift_acc;
                        e[m] = 0.0;
                        split = true;
                        break;
                    }
                    sn = f / r;
                    cs = g / r;
                    const double gg = d[i + 1] - shift_acc;
                    const double rr = (d[i] - gg) * sn + 2.0 * cs * b;
                    shift_acc = sn * rr;
                    d[i + 1] = gg + shift_acc;
                    g = cs * rr - b;
                    rc[i] = cs;
                    rs[i] = sn;
                }
                if (!split) {
                    d[l] -= shift_acc;
                    e[l] = g;
                    e[m] = 0.0;
                }
                s_first = m - 1;                  // rotations i = m-1 down to s_last were recorded
                s_last = split ? i + 1 : l;
                s_stop = 0;
                break;
            }
        }
        __syncthreads();
        if (s_stop) break;
        const int i0 = s_first, i1 = s_last;
        for (int row = t; row < n; row += bd) {
            double* zr = Z + (long long)row * n;
            double carry = zr[i0 + 1];
            for (int i = i0; i >= i1; --i) {
                const double zi = zr[i];
                zr[i + 1] = rs[i] * zi + rc[i] * carry;
                carry = rc[i] * zi - rs[i] * carry;
            }
            zr[i1] = carry;
        }
        __syncthreads();
    }
    for (int i = t; i < n; i += bd) dg[i] = d[i];
}

// Z <- H_0 H_1 ... H_{n-3} Z (eigenvectors of the reduced matrix back to the
// original basis).  Per reflector: the row vector v^T Z (threads along a row of Z,
// rows in sequence: coalesced), then the rank-one update.
__global__ void tridiag_back_kernel(int n, const double* __restrict__ Vh, const double* __restrict__ tau,
                                    double* __restrict__ Z) {
    __shared__ double dot[1024];
    const int t = threadIdx.x, bd = blockDim.x;
    for (int k = n - 3; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;
        const double* vk = Vh + (long long)k * n;
        for (int j = t; j < n; j += bd) {
            double acc = 0.0;
            for (int i = k + 1; i < n; ++i) acc = fma(vk[i], Z[(long long)i * n + j], acc);
            dot[j] = tk * acc;
        }
        __syncthreads();
        for (int i = k + 1; i < n; ++i) {
            const double vi = vk[i];
            double* zr = Z + (long long)i * n;
            for (int j = t; j < n; j += bd) zr[j] -= vi * dot[j];
        }
        __syncthreads();
    }
}

// Ascending order of d with the matching columns of Z.
__global__ void sort_pairs_kernel(int n, const double* __restrict__ d, const double* __restrict__ Z,
                                  double* __restrict__ w, double* __restrict__ Zout) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double di = d[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
        const double dj = d[j];
        rank += (dj < di) || (dj == di && j < i);
    }
    w[rank] = di;
    for (int r = 0; r < n; ++r) Zout[(long long)r * n + rank] = Z[(long long)r * n + i];
}

void launch_sym_eig(hipStream_t st, int n, double* A, double* w, double* V, double* work, double* small,
                    int* status) {
    // work: n*n (reflectors, then eigenvectors before sorting); small: 3n (tau, diag, off)
    double* tau = small;
    double* diag = small + n;
    double* off = small + 2 * n;
    hipLaunchKernelGGL(tridiag_kernel, dim3(1), dim3(1024), 0, st, n, A, work, tau, diag, off);
    hipLaunchKernelGGL(tridiag_ql_kernel, dim3(1), dim3(1024), 0, st, n, diag, off, A, status);
    hipLaunchKernelGGL(tridiag_back_kernel, dim3(1), dim3(1024), 0, st, n, work, tau, A);
    hipLaunchKernelGGL(sort_pairs_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, n, diag, A, w, V);
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
// Rayleigh-Ritz in coefficient space.  W = [X | P | T] (or [X | T]) is
// M-orthonormal except for dropped (zero) columns, H = W^T K W (m x m, m <= 64).
// Dropped columns (drop_in) are left out of the eigensolve and get an
// infinite Ritz value, so they never enter the s lowest Ritz pairs.  Outputs theta (ascending) and Cfull =
// [Q_s | C_p], where C_p spans the part of span{E_x, Q_s} orthogonal to Q_s
// (E_x = the old X coordinates), so that span{W Q_s, W C_p} = U^k + U^{k+1}.
// A C_p direction whose norm before normalisation is below 1e-12 (the old
// Ritz vector already lies in the new span) is dropped: zero column and
// drop_out[s + j] = 1; drop_out[0..s) = 0.
__global__ void rr_coef_kernel(int m, int s, int with_p, const double* __restrict__ H,
                               const int* __restrict__ drop_in, int* __restrict__ drop_out,
                               double* __restrict__ theta, double* __restrict__ Cfull) {
    __shared__ double A[64 * 64];
    __shared__ double V[64 * 64];
    __shared__ double Q[64 * 64];
    __shared__ double cs[128];
    __shared__ int pr[128];
    __shared__ double red[512];
    __shared__ double wv[64];
    __shared__ double nrm;
    __shared__ int keep_idx[64];
    __shared__ int mk;
    const int t = threadIdx.x, bd = blockDim.x;
    // Dropped (zero) columns are removed before the eigensolve and come back as
    // unit vectors with an infinite Ritz value after the kept pairs.
    if (t == 0) {
        int c = 0;
        for (int i = 0; i < m; ++i)
            if (!drop_in[i]) keep_idx[c++] = i;
        mk = c;
    }
    __syncthreads();
    const int nk = mk;
    for (int e = t; e < nk * nk; e += bd) {
        const int i = keep_idx[e / nk], j = keep_idx[e % nk];
        A[e] = 0.5 * (H[i * m + j] + H[j * m + i]);
    }
    __syncthreads();
    jacobi_core(nk, A, V, cs, pr, red);
    __syncthreads();
    jacobi_sort(nk, A, V, wv, Q);          // Q: nk x nk, stride nk
    __syncthreads();
    for (int e = t; e < m * m; e += bd) V[e] = 0.0;
    __syncthreads();
    for (int e = t; e < nk * nk; e += bd) {
        const int r = e / nk, c = e % nk;
        V[keep_idx[r] * m + c] = Q[e];
    }
    if (t == 0) {
        int c = nk;
        for (int i = 0; i < m; ++i)
            if (drop_in[i]) {
                V[i * m + c] = 1.0;
                wv[c] = INFINITY;
                ++c;
            }
    }
    __syncthreads();
    for (int e = t; e < m * m; e += bd) Q[e] = V[e];
    __syncthreads();
    for (int i = t; i < m; i += bd) theta[i] = wv[i];
    const int cw = with_p ? 2 * s : s;
    for (int e = t; e < m * s; e += bd) {
        const int r = e / s, j = e % s;
        Cfull[r * cw + j] = Q[r * m + j];
    }
    for (int j = t; j < cw; j += bd) drop_out[j] = 0;
    if (!with_p) return;
    // C_p columns: b_j = sum_{k >= s} Q[:,k] Q[j,k] = (I - Q_s Q_s^T) e_j, orthogonalised
    // (two classical Gram-Schmidt passes) against Q_s and the previous C_p columns.
    double* Cp = V;   // reuse: m x s, row-major
    __syncthreads();
    for (int j = 0; j < s; ++j) {
        for (int r = t; r < m; r += bd) {
            double acc = 0.0;
            for (int k = s; k < m; ++k) acc += Q[r * m + k] * Q[j * m + k];
            A[r] = acc;
        }
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            for (int q = t; q < s + j; q += bd) {
                double acc = 0.0;
                for (int r = 0; r < m; ++r) acc += A[r] * (q < s ? Q[r * m + q] : Cp[r * s + (q - s)]);
                red[q] = acc;
            }
            __syncthreads();
            for (int r = t; r < m; r += bd) {
                double v = A[r];
                for (int q = 0; q < s + j; ++q) v -= red[q] * (q < s ? Q[r * m + q] : Cp[r * s + (q - s)]);
                A[64 + r] = v;
            }
            __syncthreads();
            for (int r = t; r < m; r += bd) A[r] = A[64 + r];
            __syncthreads();
        }
        if (t == 0) {
            double acc = 0.0;
            for (int r = 0; r < m; ++r) acc += A[r] * A[r];
            nrm = sqrt(acc);
        }
        __syncthreads();
        const bool keep = nrm > 1e-12;
        const double inv = keep ? 1.0 / nrm : 0.0;
        for (int r = t; r < m; r += bd) Cp[r * s + j] = A[r] * inv;
        if (t == 0) drop_out[s + j] = keep ? 0 : 1;
        __syncthreads();
    }
    for (int e = t; e < m * s; e += bd) {
        const int r = e / s, j = e % s;
        Cfull[r * cw + s + j] = Cp[r * s + j];
    }
}

void launch_rr_coef(hipStream_t st, int m, int s, int with_p, const double* H, const int* drop_in, int* drop_out,
                    double* theta, double* Cfull) {
    hipLaunchKernelGGL(rr_coef_kernel, dim3(1), dim3(256), 0, st, m, s, with_p, H, drop_in, drop_out, theta, Cfull);
}

}  // namespace bpjd
