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
// Cyclic Jacobi on the symmetric n x n matrix A (row stride lda, shared memory) with
// the round-robin ordering: each round rotates n/2 disjoint (p, q) pairs at once.
// Threshold variant: a rotation is skipped when |a_pq| <= eps sqrt(|a_pp a_qq|); a
// sweep without rotations ends the iteration (relative accuracy of every eigenvalue).
// V (stride ldv) receives the eigenvectors as columns.  Thread t owns pairs
// k0, k0 + kstep, ... and columns j0, j0 + jstep, ... (one integer division per
// thread), so the inner loops carry no index arithmetic beyond additions.
__device__ void jacobi_core(int n, double* A, int lda, double* V, int ldv, double* cs, int* pr) {
    __shared__ int rotated;
    const int t = threadIdx.x, bd = blockDim.x;
    const int N = n + (n & 1);
    const int half = N / 2;
    int k0, kstep, j0, jstep;
    if (n <= bd) {
        k0 = t / n;
        kstep = bd / n;
        j0 = t - k0 * n;
        jstep = n;
    } else {
        k0 = 0;
        kstep = 1;
        j0 = t;
        jstep = bd;
    }
    if (k0 >= kstep) k0 = half;                 // idle thread
    for (int i = 0; i < n; ++i)
        for (int j = t; j < n; j += bd) V[i * ldv + j] = (i == j) ? 1.0 : 0.0;
    __syncthreads();
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
                    p = r + k;
                    if (p >= N - 1) p -= N - 1;
                    q = r - k;
                    if (q < 0) q += N - 1;
                }
                if (p > q) {
                    const int tmp = p;
                    p = q;
                    q = tmp;
                }
                double c = 1.0, sn = 0.0;
                if (q < n) {
                    const double apq = A[p * lda + q];
                    const double app = A[p * lda + p], aqq = A[q * lda + q];
                    if (fabs(apq) > 2.3e-16 * sqrt(fabs(app * aqq)) && apq != 0.0) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        sn = tt * c;
                        rotated = 1;
                    }
                }
                cs[2 * k] = c;
                cs[2 * k + 1] = sn;
                pr[2 * k] = p;
                pr[2 * k + 1] = q;
            }
            __syncthreads();
            // rows p, q of A
            for (int k = k0; k < half; k += kstep) {
                const double sn = cs[2 * k + 1];
                const int q = pr[2 * k + 1];
                if (sn == 0.0 || q >= n) continue;
                const double c = cs[2 * k];
                const int p = pr[2 * k];
                for (int j = j0; j < n; j += jstep) {
                    const double apj = A[p * lda + j], aqj = A[q * lda + j];
                    A[p * lda + j] = c * apj - sn * aqj;
                    A[q * lda + j] = sn * apj + c * aqj;
                }
            }
            __syncthreads();
            // columns p, q of A and of V; the rotation annihilates a_pq exactly, so the
            // rounding residue at (p, q) and (q, p) is replaced by zero
            for (int k = k0; k < half; k += kstep) {
                const double sn = cs[2 * k + 1];
                const int q = pr[2 * k + 1];
                if (sn == 0.0 || q >= n) continue;
                const double c = cs[2 * k];
                const int p = pr[2 * k];
                for (int i = j0; i < n; i += jstep) {
                    const double aip = A[i * lda + p], aiq = A[i * lda + q];
                    A[i * lda + p] = (i == q) ? 0.0 : c * aip - sn * aiq;
                    A[i * lda + q] = (i == p) ? 0.0 : sn * aip + c * aiq;
                    const double vip = V[i * ldv + p], viq = V[i * ldv + q];
                    V[i * ldv + p] = c * vip - sn * viq;
                    V[i * ldv + q] = sn * vip + c * viq;
                }
            }
            __syncthreads();
        }
        const int any = rotated;
        __syncthreads();
        if (!any) break;
    }
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
            // p = tau A22 v; A22 is symmetric, so column j is read by 4 threads (row
            // quarters), coalesced across neighbouring j, then summed in a fixed order
            {
                const int qtr = t >> 8, jt = t & 255;
                for (int j0 = 0; j0 < m; j0 += 256) {
                    const int j = j0 + jt;
                    double pj = 0.0;
                    if (j < m) {
                        const double* colj = A + (long long)(k + 1) * n + (k + 1) + j;
                        for (int i = qtr; i < m; i += 4) pj = fma(colj[(long long)i * n], v[i], pj);
                    }
                    red[t] = pj;
                    __syncthreads();
                    if (qtr == 0 && j < m) w[j] = tk * (((red[jt] + red[256 + jt]) + red[512 + jt]) + red[768 + jt]);
                    __syncthreads();
                }
            }
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

// Eigenvalues of the symmetric tridiagonal matrix (diag d, off-diagonal e,
// e[i] coupling i and i+1) by bisection on Sturm counts: thread j finds the
// j-th smallest eigenvalue.  count(x) = number of negative pivots of the
// LDL^T factorisation of T - x I.
__device__ inline int sturm_count(int n, const double* d, const double* e2, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
    for (int i = 1; i < n; ++i) {
        q = d[i] - x - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0);
    }
    return cnt;
}

__global__ void tridiag_bisect_kernel(int n, const double* __restrict__ dg, const double* __restrict__ eg,
                                      double* __restrict__ w) {
    __shared__ double d[1024];
    __shared__ double e2[1024];
    __shared__ double red[2][1024];
    const int t = threadIdx.x, bd = blockDim.x;
    double lo = 1e300, hi = -1e300, emax = 0.0;
    for (int i = t; i < n; i += bd) {
        d[i] = dg[i];
        const double ei = (i + 1 < n) ? eg[i] : 0.0;
        e2[i] = ei * ei;
        const double el = (i > 0) ? fabs(eg[i - 1]) : 0.0;
        const double er = fabs(ei);
        lo = fmin(lo, dg[i] - el - er);
        hi = fmax(hi, dg[i] + el + er);
        emax = fmax(emax, er);
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
    for (int j = t; j < n; j += bd) {
        double a = glo - 1e-14 * tnorm - 1e-300, b = ghi + 1e-14 * tnorm + 1e-300;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (a + b);
            if (!(mid > a && mid < b) || (b - a) <= 2.3e-16 * fmax(fabs(a), fabs(b))) break;
            if (sturm_count(n, d, e2, mid, pivmin) > j) b = mid;
            else a = mid;
        }
        w[j] = 0.5 * (a + b);
    }
}

// Inverse iteration for every eigenvalue (one thread each): three solves of
// (T - lambda_j I) x = b with a partial-pivoting LU of the tridiagonal matrix
// (U has two superdiagonals), starting from a fixed vector.  Scratch and
// result vectors are interleaved ([i][j]) so accesses coalesce across threads.
// Output: X[i][j] = component i of eigenvector j (unit 2-norm).
__global__ void tridiag_invit_kernel(int n, const double* __restrict__ dg, const double* __restrict__ eg,
                                     const double* __restrict__ w, double* __restrict__ X,
                                     double* __restrict__ scratch) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double* u0 = scratch;                        // U diagonal            [n][n]
    double* u1 = scratch + (long long)n * n;     // U first superdiagonal
    double* u2 = scratch + 2LL * n * n;          // U second superdiagonal
    double* mu = scratch + 3LL * n * n;          // multipliers, sign bit of pivot flag folded into pv
    double* pv = scratch + 4LL * n * n;          // 1.0 where rows were swapped
#define IDX(i) ((long long)(i) * n + j)
    const double lam = w[j];
    double tn = 0.0;
    for (int i = 0; i < n; ++i) tn = fmax(tn, fabs(dg[i]) + (i > 0 ? fabs(eg[i - 1]) : 0.0) + (i + 1 < n ? fabs(eg[i]) : 0.0));
    const double tiny = 2.3e-16 * fmax(tn, 1e-300);
    // factorisation P (T - lam I) = L U
    double a0 = dg[0] - lam, a1 = (n > 1) ? eg[0] : 0.0, a2 = 0.0;   // current row (cols i, i+1, i+2)
    for (int i = 0; i + 1 < n; ++i) {
        const double sub = eg[i];                                     // next row: (sub, d[i+1]-lam, e[i+1])
        const double nd = dg[i + 1] - lam;
        const double ne = (i + 2 < n) ? eg[i + 1] : 0.0;
        if (fabs(sub) > fabs(a0)) {
            const double m = a0 / sub;
            u0[IDX(i)] = sub;
            u1[IDX(i)] = nd;
            u2[IDX(i)] = ne;
            mu[IDX(i)] = m;
            pv[IDX(i)] = 1.0;
            const double na0 = a1 - m * nd, na1 = a2 - m * ne;
            a0 = na0;
            a1 = na1;
            a2 = 0.0;
        } else {
            const double piv = (a0 == 0.0) ? tiny : a0;
            const double m = sub / piv;
            u0[IDX(i)] = piv;
            u1[IDX(i)] = a1;
            u2[IDX(i)] = a2;
            mu[IDX(i)] = m;
            pv[IDX(i)] = 0.0;
            a0 = nd - m * a1;
            a1 = ne - m * a2;
            a2 = 0.0;
        }
    }
    u0[IDX(n - 1)] = (fabs(a0) < tiny) ? copysign(tiny, a0 == 0.0 ? 1.0 : a0) : a0;
    for (int i = 0; i + 1 < n; ++i)
        if (fabs(u0[IDX(i)]) < tiny) u0[IDX(i)] = copysign(tiny, u0[IDX(i)] == 0.0 ? 1.0 : u0[IDX(i)]);
    // right-hand side: a fixed vector with varying entries
    for (int i = 0; i < n; ++i) X[IDX(i)] = 1.0 + 0.5 * sin(0.7 * i + 0.3 * j);
    for (int sweep = 0; sweep < 3; ++sweep) {
        // apply the row operations: forward
        for (int i = 0; i + 1 < n; ++i) {
            double xi = X[IDX(i)], xn = X[IDX(i + 1)];
            if (pv[IDX(i)] != 0.0) {
                const double tmp = xi;
                xi = xn;
                xn = tmp;
            }
            X[IDX(i)] = xi;
            X[IDX(i + 1)] = xn - mu[IDX(i)] * xi;
        }
        // back substitution with U
        double x1 = 0.0, x2 = 0.0;
        double nrm = 0.0;
        for (int i = n - 1; i >= 0; --i) {
            const double xi = (X[IDX(i)] - u1[IDX(i)] * x1 - u2[IDX(i)] * x2) / u0[IDX(i)];
            X[IDX(i)] = xi;
            x2 = x1;
            x1 = xi;
            nrm += xi * xi;
        }
        const double inv = 1.0 / sqrt(nrm);
        for (int i = 0; i < n; ++i) X[IDX(i)] *= inv;
    }
#undef IDX
}

// Eigenvectors of clustered eigenvalues (consecutive gaps below 1e-3 |T|) from
// inverse iteration span the cluster's invariant subspace but are not
// individually accurate.  Per cluster: two Gram-Schmidt passes, then a
// Rayleigh-Ritz step on the cluster (Jacobi on X_c^T T X_c by one thread) that
// rotates the basis into eigenvectors and refines the eigenvalues.  One
// workgroup, threads along the vectors; ytmp: n * 32 doubles.
__global__ void tridiag_cluster_kernel(int n, const double* __restrict__ dg, const double* __restrict__ eg,
                                       double* __restrict__ w, double* __restrict__ X, double* __restrict__ ytmp) {
    __shared__ double red[1024];
    __shared__ double Tc[32 * 32];
    __shared__ double Qc[32 * 32];
    const int t = threadIdx.x, bd = blockDim.x;
    const double tn = fmax(fabs(w[0]), fabs(w[n - 1]));
    const double gap_tol = 1e-3 * tn;
    auto block_sum = [&](double v) -> double {
        red[t] = v;
        __syncthreads();
        for (int o = bd / 2; o > 0; o >>= 1) {
            if (t < o) red[t] += red[t + o];
            __syncthreads();
        }
        const double r = red[0];
        __syncthreads();
        return r;
    };
    int start = 0;
    for (int jj = 1; jj <= n; ++jj) {
        if (jj < n && w[jj] - w[jj - 1] <= gap_tol && jj - start < 32) continue;
        const int cs = jj - start;
        if (cs > 1) {
            for (int j = start; j < jj; ++j) {
                for (int pass = 0; pass < 2; ++pass) {
                    for (int q = start; q < j; ++q) {
                        double acc = 0.0;
                        for (int i = t; i < n; i += bd) acc += X[(long long)i * n + q] * X[(long long)i * n + j];
                        const double cq = block_sum(acc);
                        for (int i = t; i < n; i += bd) X[(long long)i * n + j] -= cq * X[(long long)i * n + q];
                        __syncthreads();
                    }
                }
                double acc = 0.0;
                for (int i = t; i < n; i += bd) acc += X[(long long)i * n + j] * X[(long long)i * n + j];
                const double inv = 1.0 / sqrt(block_sum(acc));
                for (int i = t; i < n; i += bd) X[(long long)i * n + j] *= inv;
                __syncthreads();
            }
            // y_q = T x_q, Tc = X_c^T T X_c
            for (int q = 0; q < cs; ++q) {
                const int jq = start + q;
                for (int i = t; i < n; i += bd) {
                    double v = dg[i] * X[(long long)i * n + jq];
                    if (i > 0) v += eg[i - 1] * X[(long long)(i - 1) * n + jq];
                    if (i + 1 < n) v += eg[i] * X[(long long)(i + 1) * n + jq];
                    ytmp[(long long)i * 32 + q] = v;
                }
            }
            __syncthreads();
            for (int pq = 0; pq < cs * cs; ++pq) {
                const int pp = pq / cs, qq = pq % cs;
                if (qq < pp) continue;
                double acc = 0.0;
                for (int i = t; i < n; i += bd) acc += X[(long long)i * n + start + pp] * ytmp[(long long)i * 32 + qq];
                const double v = block_sum(acc);
                if (t == 0) {
                    Tc[pp * cs + qq] = v;
                    Tc[qq * cs + pp] = v;
                }
            }
            __syncthreads();
            if (t == 0) {
                // cyclic Jacobi on the cs x cs matrix, then ascending sort of the pairs
                for (int e = 0; e < cs * cs; ++e) Qc[e] = (e / cs == e % cs) ? 1.0 : 0.0;
                for (int sweep = 0; sweep < 50; ++sweep) {
                    bool rot = false;
                    for (int pp = 0; pp < cs; ++pp)
                        for (int qq = pp + 1; qq < cs; ++qq) {
                            const double apq = Tc[pp * cs + qq];
                            const double app = Tc[pp * cs + pp], aqq = Tc[qq * cs + qq];
                            if (!(fabs(apq) > 2.3e-16 * sqrt(fabs(app * aqq))) || apq == 0.0) continue;
                            rot = true;
                            const double tau = (aqq - app) / (2.0 * apq);
                            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                            const double c = 1.0 / sqrt(1.0 + tt * tt), sn = tt * c;
                            for (int k = 0; k < cs; ++k) {
                                const double akp = Tc[k * cs + pp], akq = Tc[k * cs + qq];
                                Tc[k * cs + pp] = c * akp - sn * akq;
                                Tc[k * cs + qq] = sn * akp + c * akq;
                            }
                            for (int k = 0; k < cs; ++k) {
                                const double apk = Tc[pp * cs + k], aqk = Tc[qq * cs + k];
                                Tc[pp * cs + k] = c * apk - sn * aqk;
                                Tc[qq * cs + k] = sn * apk + c * aqk;
                            }
                            Tc[pp * cs + qq] = 0.0;
                            Tc[qq * cs + pp] = 0.0;
                            for (int k = 0; k < cs; ++k) {
                                const double vkp = Qc[k * cs + pp], vkq = Qc[k * cs + qq];
                                Qc[k * cs + pp] = c * vkp - sn * vkq;
                                Qc[k * cs + qq] = sn * vkp + c * vkq;
                            }
                        }
                    if (!rot) break;
                }
                for (int pp = 0; pp < cs; ++pp) {          // selection sort of the pairs
                    int best = pp;
                    for (int qq = pp + 1; qq < cs; ++qq)
                        if (Tc[qq * cs + qq] < Tc[best * cs + best]) best = qq;
                    if (best != pp) {
                        const double tmp = Tc[pp * cs + pp];
                        Tc[pp * cs + pp] = Tc[best * cs + best];
                        Tc[best * cs + best] = tmp;
                        for (int k = 0; k < cs; ++k) {
                            const double v = Qc[k * cs + pp];
                            Qc[k * cs + pp] = Qc[k * cs + best];
                            Qc[k * cs + best] = v;
                        }
                    }
                    w[start + pp] = Tc[pp * cs + pp];
                }
            }
            __syncthreads();
            // rotate the cluster basis: X_c <- X_c Q_c (row-wise, old values staged in ytmp)
            for (int i = t; i < n; i += bd) {
                for (int q = 0; q < cs; ++q) ytmp[(long long)i * 32 + q] = X[(long long)i * n + start + q];
                for (int q = 0; q < cs; ++q) {
                    double v = 0.0;
                    for (int pp = 0; pp < cs; ++pp) v += ytmp[(long long)i * 32 + pp] * Qc[pp * cs + q];
                    X[(long long)i * n + start + q] = v;
                }
            }
            __syncthreads();
        }
        start = jj;
    }
}

// Z <- H_0 H_1 ... H_{n-3} Z (eigenvectors of the reduced matrix back to the
// original basis).  Columns are independent: each workgroup owns 8 columns and
// applies every reflector to them (threads split the rows for the dot products).
__global__ void tridiag_back_kernel(int n, const double* __restrict__ Vh, const double* __restrict__ tau,
                                    double* __restrict__ Z) {
    __shared__ double red[8][33];
    __shared__ double dot[8];
    const int t = threadIdx.x;
    const int c = t & 7, rg = t >> 3;          // 8 columns x 32 row groups
    const int j = blockIdx.x * 8 + c;
    const bool live = j < n;
    for (int k = n - 3; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;
        const double* vk = Vh + (long long)k * n;
        double acc = 0.0;
        if (live)
            for (int i = k + 1 + rg; i < n; i += 32) acc = fma(vk[i], Z[(long long)i * n + j], acc);
        red[c][rg] = acc;
        __syncthreads();
        if (rg == 0) {
            double sum = 0.0;
            for (int q = 0; q < 32; ++q) sum += red[c][q];
            dot[c] = tk * sum;
        }
        __syncthreads();
        const double dc = dot[c];
        if (live)
            for (int i = k + 1 + rg; i < n; i += 32) Z[(long long)i * n + j] -= dc * vk[i];
        __syncthreads();
    }
}

void launch_sym_eig(hipStream_t st, int n, double* A, double* w, double* V, double* work, double* small,
                    double* scratch, int* status) {
    // work: n*n (reflectors); small: 3n (tau, diag, off); scratch: 5 n*n (inverse iteration)
    (void)status;
    double* tau = small;
    double* diag = small + n;
    double* off = small + 2 * n;
    hipLaunchKernelGGL(tridiag_kernel, dim3(1), dim3(1024), 0, st, n, A, work, tau, diag, off);
    hipLaunchKernelGGL(tridiag_bisect_kernel, dim3(1), dim3(1024), 0, st, n, diag, off, w);
    hipLaunchKernelGGL(tridiag_invit_kernel, dim3(grid_for(n, 64)), dim3(64), 0, st, n, diag, off, w, V, scratch);
    hipLaunchKernelGGL(tridiag_cluster_kernel, dim3(1), dim3(256), 0, st, n, diag, off, w, V, scratch);
    hipLaunchKernelGGL(tridiag_back_kernel, dim3(grid_for(n, 8)), dim3(256), 0, st, n, work, tau, V);
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
// Rayleigh-Ritz coefficients on the m x m projected matrix H (m <= RR_MAX).
// Dropped columns (drop_in) are left out of the eigensolve and get an infinite Ritz
// value, so they never enter the s lowest Ritz pairs.  Outputs theta (ascending) and
// Cfull = [Q_s | C_p], where C_p spans the part of span{E_x, Q_s} orthogonal to Q_s
// (E_x = the old X coordinates), so that span{W Q_s, W C_p} = U^k + U^{k+1}.
// Because Q is orthogonal, (I - Q_s Q_s^T) e_j = Q_{>s} g_j with g_j = (row j of
// Q_{>s})^T, so C_p = Q_{>s} orth(g_0 .. g_{s-1}); a direction whose norm after two
// Gram-Schmidt passes is below 1e-12 (the old Ritz vector already lies in the new
// span) is dropped: zero column and drop_out[s + j] = 1; drop_out[0..s) = 0.
constexpr int RR_MAX = 48;
__global__ __launch_bounds__(256) void rr_coef_kernel(int m, int s, int with_p, const double* __restrict__ H,
                                                      const int* __restrict__ drop_in, int* __restrict__ drop_out,
                                                      double* __restrict__ theta, double* __restrict__ Cfull) {
    constexpr int LD = RR_MAX + 1;
    __shared__ double A[RR_MAX * LD];
    __shared__ double V[RR_MAX * LD];
    __shared__ double Q[RR_MAX * LD];
    __shared__ double cs[RR_MAX];
    __shared__ int pr[RR_MAX];
    __shared__ double wv[RR_MAX];
    __shared__ double red[RR_MAX];
    __shared__ int keep_idx[RR_MAX];
    __shared__ int mk;
    const int t = threadIdx.x, bd = blockDim.x;
    if (t == 0) {
        int c = 0;
        for (int i = 0; i < m; ++i)
            if (!drop_in[i]) keep_idx[c++] = i;
        mk = c;
    }
    __syncthreads();
    const int nk = mk;
    for (int i = 0; i < nk; ++i)
        for (int j = t; j < nk; j += bd) {
            const int gi = keep_idx[i], gj = keep_idx[j];
            A[i * LD + j] = 0.5 * (H[gi * m + gj] + H[gj * m + gi]);
        }
    __syncthreads();
    if (nk > 0) jacobi_core(nk, A, LD, V, LD, cs, pr);
    __syncthreads();
    // ascending order of the kept Ritz values; Q (m x m) = eigenvectors placed back at the
    // kept coordinates, followed by unit vectors (infinite value) for the dropped ones
    for (int e = t; e < m * LD; e += bd) Q[e] = 0.0;
    __syncthreads();
    for (int i = t; i < nk; i += bd) {
        const double di = A[i * LD + i];
        int rank = 0;
        for (int j = 0; j < nk; ++j) {
            const double dj = A[j * LD + j];
            rank += (dj < di) || (dj == di && j < i);
        }
        wv[rank] = di;
        for (int r = 0; r < nk; ++r) Q[keep_idx[r] * LD + rank] = V[r * LD + i];
    }
    if (t == 0) {
        int c = nk;
        for (int i = 0; i < m; ++i)
            if (drop_in[i]) {
                Q[i * LD + c] = 1.0;
                wv[c] = INFINITY;
                ++c;
            }
    }
    __syncthreads();
    for (int i = t; i < m; i += bd) theta[i] = wv[i];
    const int cw = with_p ? 2 * s : s;
    for (int r = 0; r < m; ++r)
        for (int j = t; j < s; j += bd) Cfull[r * cw + j] = Q[r * LD + j];
    for (int j = t; j < cw; j += bd) drop_out[j] = 0;
    if (!with_p) return;
    // G (stored in A, (m - s) x s, stride LD): column j = g_j, then orthonormalised in
    // place column by column with two classical Gram-Schmidt passes
    const int mg = m - s;
    for (int e = t; e < mg * s; e += bd) {
        const int k = e / s, j = e - k * s;
        A[k * LD + j] = Q[j * LD + s + k];
    }
    __syncthreads();
    for (int j = 0; j < s; ++j) {
        for (int pass = 0; pass < 2; ++pass) {
            for (int q = t; q < j; q += bd) {
                double acc = 0.0;
                for (int k = 0; k < mg; ++k) acc = fma(A[k * LD + q], A[k * LD + j], acc);
                red[q] = acc;
            }
            __syncthreads();
            for (int k = t; k < mg; k += bd) {
                double v = A[k * LD + j];
                for (int q = 0; q < j; ++q) v -= red[q] * A[k * LD + q];
                A[k * LD + j] = v;
            }
            __syncthreads();
        }
        if (t < 64) {
            double acc = 0.0;
            for (int k = t; k < mg; k += 64) acc = fma(A[k * LD + j], A[k * LD + j], acc);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (t == 0) red[RR_MAX - 1] = sqrt(acc);
        }
        __syncthreads();
        const double nrm = red[RR_MAX - 1];
        const bool keep = nrm > 1e-12;
        const double inv = keep ? 1.0 / nrm : 0.0;
        for (int k = t; k < mg; k += bd) A[k * LD + j] *= inv;
        if (t == 0) drop_out[s + j] = keep ? 0 : 1;
        __syncthreads();
    }
    // C_p = Q_{>s} G
    for (int e = t; e < m * s; e += bd) {
        const int r = e / s, j = e - r * s;
        double acc = 0.0;
        for (int k = 0; k < mg; ++k) acc = fma(Q[r * LD + s + k], A[k * LD + j], acc);
        Cfull[r * cw + s + j] = acc;
    }
}

void launch_rr_coef(hipStream_t st, int m, int s, int with_p, const double* H, const int* drop_in, int* drop_out,
                    double* theta, double* Cfull) {
    hipLaunchKernelGGL(rr_coef_kernel, dim3(1), dim3(256), 0, st, m, s, with_p, H, drop_in, drop_out, theta, Cfull);
}

}  // namespace bpjd
