// Two-level additive Schwarz preconditioner of Section 3 (eq. Preconditioner):
//   Z_i = P (B_0,i)^{-1} Q^H_{s+1} Q^H r_i  +  sum_l R_l^T (K_l - lambda_i M_l)^{-1} R_l F_i
// with F_i = lambda_i M x_i - K x_i the residual in the dual (load-vector) form.
//
// Coarse term: G = P^T F; on the coarse eigenbasis (Y, lambda^H), components
// j < s are removed (Q^H_{s+1}) and the others divided by lambda^H_j - lambda_i.
// Local term: per (subdomain l, shift i) an LDL^T factorisation of the banded
// local matrix K_l - lambda_i M_l and one solve.  Subdomain values are
// gathered into a contiguous per-shift array, solved, and summed back in a
// fixed order per dof (gather form of the overlapping scatter).
#include "common.h"

namespace bpjd {

// ---------------------------------------------------------------------------
// Galerkin coarse operators K_H = P^T K P, M_H = P^T M P on a host-computed
// pattern: first KP (fine rows, coarse columns), then one thread per nonzero
// of the coarse pattern.  Every sum runs in a fixed order.
__global__ void galerkin_kp_kernel(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                                   const double2* __restrict__ km, const int* __restrict__ Pptr,
                                   const int* __restrict__ Pcol, const double* __restrict__ Pval,
                                   const int* __restrict__ kpptr, const int* __restrict__ kpcol,
                                   double2* __restrict__ kpval) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int e0 = kpptr[i], e1 = kpptr[i + 1];
    for (int e = e0; e < e1; ++e) kpval[e] = make_double2(0.0, 0.0);
    for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const int j = col[p];
        const double2 v = km[p];
        for (int q = Pptr[j]; q < Pptr[j + 1]; ++q) {
            const int b = Pcol[q];
            const double w = Pval[q];
            for (int e = e0; e < e1; ++e) {
                if (kpcol[e] == b) {
                    kpval[e].x = fma(v.x, w, kpval[e].x);
                    kpval[e].y = fma(v.y, w, kpval[e].y);
                    break;
                }
            }
        }
    }
}

__global__ void galerkin_kh_kernel(int nH, int nnzKH, const int* __restrict__ PTptr, const int* __restrict__ PTcol,
                                   const double* __restrict__ PTval, const int* __restrict__ kpptr,
                                   const int* __restrict__ kpcol, const double2* __restrict__ kpval,
                                   const int* __restrict__ khptr, const int* __restrict__ khcol,
                                   double* __restrict__ KH, double* __restrict__ MH) {
    __shared__ double rk[256], rm[256];
    const int e2 = blockIdx.x;
    const int t = threadIdx.x;
    // coarse row a of this pattern entry (binary search in khptr)
    int lo = 0, hi = nH;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (khptr[mid] <= e2) lo = mid; else hi = mid;
    }
    const int a = lo;
    const int b = khcol[e2];
    double ak = 0.0, am = 0.0;
    for (int q = PTptr[a] + t; q < PTptr[a + 1]; q += 256) {
        const int i = PTcol[q];
        const double w = PTval[q];
        for (int e = kpptr[i]; e < kpptr[i + 1]; ++e) {
            if (kpcol[e] == b) {
                ak = fma(w, kpval[e].x, ak);
                am = fma(w, kpval[e].y, am);
                break;
            }
        }
    }
    rk[t] = ak;
    rm[t] = am;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            rk[t] += rk[t + o];
            rm[t] += rm[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        KH[(long long)a * nH + b] = rk[0];
        MH[(long long)a * nH + b] = rm[0];
    }
}

void launch_galerkin(hipStream_t st, int n, int nH, const int* rowptr, const int* col, const double2* km,
                     const int* Pptr, const int* Pcol, const double* Pval,
                     const int* PTptr, const int* PTcol, const double* PTval,
                     const int* kpptr, const int* kpcol, double2* kpval,
                     const int* khptr, const int* khcol, int nnzKH, double* KH, double* MH) {
    launch_fill(st, (long long)nH * nH, KH, 0.0);
    launch_fill(st, (long long)nH * nH, MH, 0.0);
    hipLaunchKernelGGL(galerkin_kp_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, n, rowptr, col, km, Pptr, Pcol,
                       Pval, kpptr, kpcol, kpval);
    hipLaunchKernelGGL(galerkin_kh_kernel, dim3(nnzKH), dim3(256), 0, st, nH, nnzKH, PTptr,
                       PTcol, PTval, kpptr, kpcol, kpval, khptr, khcol, KH, MH);
}

// ---------------------------------------------------------------------------
// Coarse term.

// Cw[j][i] = (y_j^T G_i) / (lambda^H_j - lambda_i) for j >= s; one workgroup per
// coarse eigenvector j reads row j of Y^T (contiguous) and reduces per column i.
__global__ void coarse_coef_kernel(int nH, int s, const double* __restrict__ YT, const double* __restrict__ G,
                                   const double* __restrict__ lamH, const double* __restrict__ lam,
                                   double* __restrict__ Cw) {
    __shared__ double red[16][64];
    const int j = blockIdx.x;
    const int t = threadIdx.x;                 // 64 threads: 4 column groups x 16 row slots
    const int ig = t & 3, rs = t >> 2;
    if (j < s) {                               // Q^H_{s+1} removes the first s coarse eigenvectors
        for (int i = t; i < s; i += 64) Cw[j * s + i] = 0.0;
        return;
    }
    const double* yrow = YT + (long long)j * nH;
    for (int i0 = 0; i0 < s; i0 += 4) {
        const int i = i0 + ig;
        double acc = 0.0;
        if (i < s) {
            constexpr int U = 4;               // loads of U row steps together, same sum order
            for (int b0 = rs; b0 < nH; b0 += 16 * U) {
                double yv[U], gv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int b = min(b0 + 16 * u, nH - 1);
                    yv[u] = yrow[b];
                    gv[u] = G[b * s + i];
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (b0 + 16 * u < nH) acc = fma(yv[u], gv[u], acc);
            }
        }
        red[rs][ig] = acc;
        __syncthreads();
        if (rs == 0 && i < s) {
            double sum = 0.0;
            for (int k = 0; k < 16; ++k) sum += red[k][ig];
            Cw[j * s + i] = sum / (lamH[j] - lam[i]);
        }
        __syncthreads();
    }
}

// Zhat[b][i] = sum_{j >= s} Y[b][j] Cw[j][i]: one wavefront per coarse row b reads the
// row contiguously, keeps s (<= BPJD_MAX_BLOCK) partial sums per lane and reduces them
// across lanes.
__global__ __launch_bounds__(64) void coarse_back_kernel(int nH, int s, const double* __restrict__ Y,
                                                         const double* __restrict__ Cw, double* __restrict__ Zhat) {
    const int b = blockIdx.x, lane = threadIdx.x;
    const double* yrow = Y + (long long)b * nH;
    double acc[BPJD_MAX_BLOCK];
#pragma unroll
    for (int i = 0; i < BPJD_MAX_BLOCK; ++i) acc[i] = 0.0;
    for (int j0 = s + lane; j0 < nH; j0 += 128) {
        // two row steps whose loads are issued together; the sum keeps the order of j
        const int j1 = min(j0 + 64, nH - 1);
        const double y0 = yrow[j0], y1 = yrow[j1];
        const double* c0 = Cw + j0 * s;
        const double* c1 = Cw + j1 * s;
        double cv0[BPJD_MAX_BLOCK], cv1[BPJD_MAX_BLOCK];
#pragma unroll
        for (int i = 0; i < BPJD_MAX_BLOCK; ++i) {
            cv0[i] = (i < s) ? c0[i] : 0.0;
            cv1[i] = (i < s) ? c1[i] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < BPJD_MAX_BLOCK; ++i)
            if (i < s) acc[i] = fma(y0, cv0[i], acc[i]);
        if (j0 + 64 < nH)
#pragma unroll
            for (int i = 0; i < BPJD_MAX_BLOCK; ++i)
                if (i < s) acc[i] = fma(y1, cv1[i], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < BPJD_MAX_BLOCK; ++i) {
        if (i < s) {
            double v = acc[i];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) Zhat[b * s + i] = v;
        }
    }
}


// G = P^T F, chunked: workgroup (k, a) takes the k-th chunk of `chunk` support entries
// of coarse dof a.  Thread t works on column t % s of the entries t / s, t / s + slots,
// ... (slots = 256 / s), so the lanes of one entry read its row of F contiguously;
// the per-entry-slot sums are then added in slot order for each column.  With one
// chunk the sum is G itself, else it goes to part[a][k][i] and restrict_sum_kernel
// adds the chunks in order (deterministic either way).
__global__ __launch_bounds__(256) void restrict_cols_kernel(int s, int nchunk, int chunk,
                                                            const int* __restrict__ PTptr,
                                                            const int* __restrict__ PTcol,
                                                            const double* __restrict__ PTval,
                                                            const double* __restrict__ F, int ldf,
                                                            double* __restrict__ out) {
    __shared__ double red[256];
    const int k = blockIdx.x, a = blockIdx.y;
    const int t = threadIdx.x;
    const int slots = 256 / s;
    const int c = t % s, e = t / s;
    const int q0 = PTptr[a] + k * chunk;
    const int q1 = min(q0 + chunk, PTptr[a + 1]);
    double acc = 0.0;
    if (e < slots) {
        // U entries at a time: their indices, then their F values, are loaded together
        // (a chain of dependent loads per entry otherwise); the sum keeps the entry order
        constexpr int U = 8;
        for (int qb = q0 + e; qb < q1; qb += U * slots) {
            int col[U];
            double w[U], f[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = min(qb + u * slots, q1 - 1);
                col[u] = PTcol[q];
                w[u] = PTval[q];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) f[u] = F[(long long)col[u] * ldf + c];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (qb + u * slots < q1) acc = fma(w[u], f[u], acc);
        }
    }
    red[t] = acc;
    __syncthreads();
    if (t < s) {
        double v = 0.0;
        for (int j = 0; j < slots; ++j) v += red[j * s + t];
        out[((long long)a * nchunk + k) * s + t] = v;
    }
}

__global__ void restrict_sum_kernel(int nH, int s, int nchunk, const double* __restrict__ part,
                                    double* __restrict__ G) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nH * s) return;
    const int a = t / s, i = t - a * s;
    double acc = 0.0;
    for (int k = 0; k < nchunk; ++k) acc += part[((long long)a * nchunk + k) * s + i];
    G[t] = acc;
}

void launch_coarse_apply(hipStream_t st, int n, int nH, int s, const int* PTptr, const int* PTcol,
                         const double* PTval, const double* F, int ldf, const double* Y, const double* YT,
                         const double* lamH, const double* lam, double* G, double* Cw, double* Zhat,
                         int maxPT, double* part, long long part_cap) {
    (void)n;
    // chunks of at most 512 support entries, one workgroup per (chunk, coarse dof), so
    // that even a few coarse dofs with wide supports fill the device; a single chunk
    // writes G directly, several go through the ordered second pass
    long long chunk = 512;
    while (chunk < maxPT && (long long)nH * s * ((maxPT + chunk - 1) / chunk) > part_cap) chunk *= 2;
    const long long nchunk = std::max<long long>(1, (maxPT + chunk - 1) / chunk);
    if (nchunk == 1) {
        hipLaunchKernelGGL(restrict_cols_kernel, dim3(1, nH), dim3(256), 0, st, s, 1, (int)chunk, PTptr, PTcol,
                           PTval, F, ldf, G);
    } else {
        hipLaunchKernelGGL(restrict_cols_kernel, dim3((int)nchunk, nH), dim3(256), 0, st, s, (int)nchunk, (int)chunk,
                           PTptr, PTcol, PTval, F, ldf, part);
        hipLaunchKernelGGL(restrict_sum_kernel, dim3((nH * s + 255) / 256), dim3(256), 0, st, nH, s, (int)nchunk,
                           part, G);
    }
    hipLaunchKernelGGL(coarse_coef_kernel, dim3(nH), dim3(64), 0, st, nH, s, YT, G, lamH, lam, Cw);
    hipLaunchKernelGGL(coarse_back_kernel, dim3(nH), dim3(64), 0, st, nH, s, Y, Cw, Zhat);
}

// ---------------------------------------------------------------------------
// Gather R_l F into per-shift contiguous arrays Floc[i][pos] (pos runs over
// all subdomains' dofs in subdomain order), converting to the solve precision.
// Staged through LDS: a workgroup takes GT consecutive positions, reads their rows
// of F with consecutive threads on consecutive columns of a row, and writes each
// shift's GT values with consecutive threads on consecutive positions.
constexpr int GT = 256;

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(int sumN, int s, const int* __restrict__ subidx,
                                                     const double* __restrict__ F, int ldf, T* __restrict__ Floc) {
    extern __shared__ __align__(16) unsigned char gather_smem[];
    T (*tile)[GT + 1] = reinterpret_cast<T (*)[GT + 1]>(gather_smem);   // [s][GT + 1]
    __shared__ int rowi[GT];
    const int pos0 = blockIdx.x * GT;
    const int cnt = min(GT, sumN - pos0);
    const int t = threadIdx.x;
    if (t < cnt) rowi[t] = subidx[pos0 + t];
    __syncthreads();
    {
        // element e = t + 256 k is (row p, shift i) = (e / s, e % s): one division, then strides
        int p = t / s, i = t - p * s;
        const int dp = 256 / s, di = 256 - dp * s;
        for (int e = t; e < cnt * s; e += 256) {
            tile[i][p] = (T)F[(long long)rowi[p] * ldf + i];
            p += dp;
            i += di;
            if (i >= s) {
                i -= s;
                ++p;
            }
        }
    }
    __syncthreads();
    for (int e = t; e < GT * s; e += 256) {
        const int i = e / GT, p = e - i * GT;
        if (p < cnt) Floc[(long long)i * sumN + pos0 + p] = tile[i][p];
    }
}

void launch_gather_f64(hipStream_t st, int sumN, int s, const int* subidx, const double* F, int ldf, double* Floc) {
    hipLaunchKernelGGL(gather_kernel<double>, dim3(grid_for(sumN, GT)), dim3(256), sizeof(double) * s * (GT + 1), st,
                       sumN, s, subidx, F, ldf, Floc);
}
void launch_gather_f32(hipStream_t st, int sumN, int s, const int* subidx, const double* F, int ldf, float* Floc) {
    hipLaunchKernelGGL(gather_kernel<float>, dim3(grid_for(sumN, GT)), dim3(256), sizeof(float) * s * (GT + 1), st,
                       sumN, s, subidx, F, ldf, Floc);
}

// ---------------------------------------------------------------------------
// Local solves.  One 64-lane workgroup per (subdomain l, shift i).  The local
// matrix A = K_l - lambda_i M_l has half-bandwidth w in the subdomain's dof
// order; its active window (rows j..j+w, band offsets 0..w) lives in LDS as a
// circular buffer of C = w+1 rows.  Right-looking LDL^T: at step j the pivot
// d_j = A_jj, the column l_{j+a,j} = A_{j+a,j}/d_j is stored, and the window is
// updated A_{j+a,j+a-b} -= l_{j+a,j} A_{j+b,j}.  The forward substitution with
// the unit lower factor runs in the same sweep; the backward sweep reads the
// stored columns back.  Rows enter the window from the sparse lower pattern of
// the union matrix (lptr/ldd/lpos: local row -> band offset, union nnz index).
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The windowed solver, like the blocked one below, runs one wavefront per workgroup
// and exchanges LDS data within the step loops through wave_sync (defined with the
// blocked solver): a wave barrier without the memory fence of __syncthreads.
__device__ inline void wave_sync();

// Workgroup barrier for data exchanged through LDS only: waits for this wave's LDS
// accesses, not for its outstanding global loads and stores.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

constexpr int kLdltMaxThreads = 256;   // up to four waves per system in the forward phase

// Local LDL^T factor + solve for bands too wide for the blocked solver (or rows with more
// than 8 lower entries): one workgroup of one to four waves (the launch picks it) per
// (subdomain, shift), the band window of C = w + 1 rows in LDS as a circular buffer.
// Step j scales column j and updates the window: every thread takes fixed chunks of the
// rows below the pivot, so the step's work is spread over all waves.  Wave 0 then puts row j + C into the
// freed slot and copies column j + 1 out for the next step.  The entering rows come from
// the fixed-slot arrays (band offset, (K, M) pair) and are loaded a block of RB rows at a
// time, one block ahead, one slot per lane.  The backward sweep (wave 0) reads the stored
// factor columns D steps ahead in a register ring.
template <typename T>
__global__ __launch_bounds__(kLdltMaxThreads) void local_ldlt_kernel(
    int s, int E, const int* __restrict__ subptr, const int* __restrict__ bwv, const int* __restrict__ sd,
    const double2* __restrict__ sv, const double* __restrict__ lam, const T* __restrict__ Floc, long long ldF,
    T* __restrict__ zloc, T* __restrict__ Lwork, const long long* __restrict__ Loff, int* __restrict__ status) {
    extern __shared__ unsigned char smem_raw[];
    T* win = reinterpret_cast<T*>(smem_raw);
    const int sys = blockIdx.x;
    const int l = sys / s;
    const int i = sys - l * s;
    const int off = subptr[l];
    const int nl = subptr[l + 1] - off;
    const int w = bwv[l];
    const int C = w + 1;
    T* ywin = win + C * C;
    T* zwin = ywin + C;
    // column j of the window, contiguous (cwin[b] = A(j + b, j)), during the forward phase
    // only: it shares the storage of the backward sweep's z (the LDS footprint decides
    // how many systems share a compute unit)
    T* cwin = zwin;
    double shift = lam[i];      // 0 when K_l - lambda_i M_l is not positive definite
    T* Lc = Lwork + Loff[l] + (long long)i * nl * C;
    const T* f = Floc + (long long)i * ldF + off;
    T* z = zloc + (long long)i * ldF + off;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;    // 64, 128 or 256
    const int lane = tid & 63;
    const bool wave0 = tid < 64;    // entering rows, column copies and the backward sweep
    // entering rows in blocks of RB rows, lane = (row d of the block, slot e); EP = slots
    // per row rounded up to a power of two (E <= 64)
    int EP = 1;
    while (EP < E) EP <<= 1;
    const int RB = 64 / EP;
    const int ld = lane / EP, le = lane - ld * EP;
    int bsd = -1, nsd = -1;            // slot of this lane in the current / next block
    double2 bsv = make_double2(0.0, 0.0), nsv = bsv;
    T bf = T(0), nf = T(0);            // right-hand side of row d of the block
    auto load_block = [&](const int r0, int& dsd, double2& dsv, T& df) {
        const int r = r0 + ld;
        const bool ok = r < nl && le < E;
        const long long k = ok ? (long long)(off + r) * E + le : 0LL;
        dsd = sd[k];
        dsv = sv[k];
        if (!ok) dsd = -1;
        df = f[min(r, nl - 1)];
    };
    // this thread's share of each step's window update: the rows j + a, a = 1..w, go in
    // pairs (q + 1, w - q), q < ceil(w/2) <= 96, of w + 1 entries together, and each pair
    // is cut into S chunks of Lch consecutive entries.  Item (q, h) = chunk h of pair q;
    // there are npair * S <= max(nthr, npair) < 2 nthr items, so a thread has at most two:
    // tid and tid + nthr.
    const int npair = (w + 1) / 2;
    const int S = max(1, nthr / npair);
    const int Lch = (w + S) / S;
    const int nitem = npair * S;
    const int pq0 = tid / S, ph0 = tid - pq0 * S;
    const int it1 = tid + nthr;
    const int pq1 = it1 / S, ph1 = it1 - pq1 * S;
    auto copy_column = [&](const int jn) {   // column jn of the window into cwin (wave 0)
        const int sn = jn % C;
        for (int b = lane; b < C; b += 64) {
            const int rb = sn + b - (sn + b >= C ? C : 0);
            cwin[b] = win[rb * C + b];
        }
    };

    int bad = 0;
    // forward phase; a negative pivot (indefinite local matrix) runs it again with shift 0
    for (int attempt = 0;; ++attempt) {
        for (int e = tid; e < C * C + 2 * C; e += nthr) win[e] = T(0);
        __syncthreads();
        int bstart = C;
        if (wave0) {
            // rows 0 .. C-1 start the window
            for (int r0 = 0; r0 < min(C, nl); r0 += RB) {
                int dsd;
                double2 dsv;
                T df;
                load_block(r0, dsd, dsv, df);
                const int r = r0 + ld;
                if (r < min(C, nl)) {
                    if (dsd >= 0) win[r * C + dsd] = (T)(dsv.x - shift * dsv.y);
                    if (le == 0) ywin[r] = df;
                }
            }
            // blocks of the rows entering from step 0 on (row C + j at step j)
            load_block(bstart, bsd, bsv, bf);
            load_block(bstart + RB, nsd, nsv, nf);
            wave_sync();
            copy_column(0);
        }
        __syncthreads();

        bad = 0;
        int neg = 0;
        for (int j = 0; j < nl; ++j) {
            const int sj = j % C;
            T dj = cwin[0];
            if (!(dj == dj) || dj == T(0) || !isfinite((double)dj)) {
                bad = 1;
                dj = T(1);
            }
            neg |= dj < T(0);
            const T inv = T(1) / dj;
            const T yj = ywin[sj];
            // entries b = b0..b1 of row j + a: -= l_{j+a} * column j (entry b), 8 at a time
            // (the column is never written in this step, so all 16 loads of a group are
            // issued before its first update)
            auto update_range = [&](const int a, const int b0, const int b1) {
                const int ra = sj + a - (sj + a >= C ? C : 0);     // slot of row j + a
                T* rowa = win + ra * C;
                const T lsc = cwin[a] * inv;
                int b = b0;
                for (; b + 7 <= b1; b += 8) {
                    T cv[8], rv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        cv[u] = cwin[b + u];
                        rv[u] = rowa[a - b - u];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) rowa[a - b - u] = rv[u] - lsc * cv[u];
                }
                for (; b <= b1; ++b) rowa[a - b] -= lsc * cwin[b];
            };
            auto finish_row = [&](const int a) {   // multiplier stored, forward substitution
                const int ra = sj + a - (sj + a >= C ? C : 0);
                const T lsc = cwin[a] * inv;
                ywin[ra] -= lsc * yj;
                Lc[(long long)j * C + a] = lsc;
            };
            auto update_item = [&](const int q, const int h) {
                const int a1 = q + 1, a2 = w - q;
                const int n1 = (j + a1 < nl) ? a1 : 0;                     // entries of row j + a1
                const int n2 = (a2 != a1 && j + a2 < nl) ? a2 : 0;         // and of row j + a2
                const int lo = h * Lch, hi = min(lo + Lch, n1 + n2);       // this chunk: [lo, hi)
                if (lo < min(hi, n1)) update_range(a1, lo + 1, min(hi, n1));
                if (hi > max(lo, n1)) update_range(a2, max(lo, n1) - n1 + 1, hi - n1);
                if (h == 0) {
                    if (n1) finish_row(a1);
                    if (n2) finish_row(a2);
                }
            };
            if (tid < nitem) update_item(pq0, ph0);
            if (it1 < nitem) update_item(pq1, ph1);
            if (tid == 0) {
                Lc[(long long)j * C] = dj;
                z[j] = yj * inv;
            }
            lds_barrier();
            if (wave0) {
                // the pivot row's slot takes row j + C; then column j + 1 is copied out
                T* row = win + sj * C;
                for (int e = lane; e < C; e += 64) row[e] = T(0);
                wave_sync();
                const int rn = j + C;
                if (rn < nl) {
                    if (rn == bstart + RB) {       // next block becomes current; fetch the one after
                        bstart += RB;
                        bsd = nsd;
                        bsv = nsv;
                        bf = nf;
                        load_block(bstart + RB, nsd, nsv, nf);
                    }
                    if (ld == rn - bstart) {
                        if (bsd >= 0) row[bsd] = (T)(bsv.x - shift * bsv.y);
                        if (le == 0) ywin[sj] = bf;
                    }
                }
                wave_sync();
                if (j + 1 < nl) copy_column(j + 1);
            }
            lds_barrier();
        }
        if (attempt > 0 || !neg) break;    // every thread reads the same pivots
        shift = 0.0;
    }
    for (int e = tid; e < C; e += nthr) zwin[e] = T(0);     // it held column values
    __syncthreads();    // the stored factor and forward values are complete before they are read back
    if (!wave0) return;
    // backward sweep with the unit upper factor L^T; the columns of steps j - 1 .. j - D
    // are in flight while step j is summed (lane owns entries a = lane + 1, lane + 65,
    // lane + 129)
    constexpr int D = 4;
    T la[D], lb[D], lc3[D], zq[D];
    auto fetch_col = [&](const int j, T& va, T& vb, T& vc, T& vz) {
        const int jc = max(j, 0);
        const int a1 = lane + 1, a2 = lane + 65, a3 = lane + 129;
        va = (a1 <= w && jc + a1 < nl) ? Lc[(long long)jc * C + a1] : T(0);
        vb = (a2 <= w && jc + a2 < nl) ? Lc[(long long)jc * C + a2] : T(0);
        vc = (a3 <= w && jc + a3 < nl) ? Lc[(long long)jc * C + a3] : T(0);
        vz = z[jc];
    };
#pragma unroll
    for (int u = 0; u < D; ++u) fetch_col(nl - 1 - u, la[u], lb[u], lc3[u], zq[u]);
    for (int jj = nl - 1; jj >= 0; jj -= D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int j = jj - u;
            if (j >= 0) {
                const int sj = j % C;
                const int a1 = lane + 1, a2 = lane + 65;
                const int r1 = sj + a1 - (sj + a1 >= C ? C : 0);
                T part = la[u] * zwin[(a1 <= w) ? r1 : 0];
                if (a2 <= w) {
                    const int r2 = sj + a2 - (sj + a2 >= C ? C : 0);
                    part += lb[u] * zwin[r2];
                }
                const int a3 = lane + 129;
                if (a3 <= w) {
                    const int r3 = sj + a3 - (sj + a3 >= C ? C : 0);
                    part += lc3[u] * zwin[r3];
                }
                const T zj0 = zq[u];
                fetch_col(j - D, la[u], lb[u], lc3[u], zq[u]);
                part = wave_sum(part);
                if (lane == 0) {
                    const T zj = zj0 - part;
                    zwin[sj] = zj;
                    z[j] = zj;
                }
                wave_sync();
            }
        }
    }
    if (bad && lane == 0) atomicOr(status, STATUS_LOCAL_PIVOT);
}

// ---------------------------------------------------------------------------
// Local solves, blocked: the same LDL^T of the banded K_l - lambda_i M_l, one
// wavefront per (subdomain, shift), for half-bandwidths w <= 48.  The active
// window is 64 rows = 4 tile-rows of 16; its lower tiles live in MFMA
// accumulators.  Per panel of 16 columns: the panel is moved to one row per
// lane and factored column by column (pivots by lane broadcast), the forward
// substitution advances, the panel is stored for the backward sweep, and the
// trailing window takes the update -L21 D L21^T with 16x16x4 MFMAs.  The
// window then slides by 16 rows and a new tile-row enters from the sparse
// lower pattern.  Rows past the end of the subdomain are identity padding.
// The blocked solver's workgroup is a single wavefront: its LDS accesses execute
// in issue order, so exchanging data through LDS only needs the compiler not to
// reorder them (a wave barrier), not a workgroup barrier with its memory fence
// (which would wait for the outstanding global loads and stores).
__device__ inline void wave_sync() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);   // no compiler reordering of memory accesses
    __builtin_amdgcn_wave_barrier();
}

// sum over the four lanes of a quad (lanes 4j .. 4j+3) with DPP quad permutations
__device__ inline float quad_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));   // [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));   // [2,3,0,1]
    return v;
}
__device__ inline double dpp_double(double v, const int ctrl_sel) {
    const long long b = __double_as_longlong(v);
    int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
    if (ctrl_sel == 0) {
        lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
        hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
    } else {
        lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
        hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double quad_sum(double v) {
    v += dpp_double(v, 0);
    v += dpp_double(v, 1);
    return v;
}

typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef double doublex4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaTile;
template <>
struct MfmaTile<float> {
    typedef floatx4_t acc;
    __device__ static inline acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // accumulator element i of a lane sits at row 4*(lane/16) + i, column lane%16
    __device__ static inline int row(int lane, int i) { return 4 * (lane >> 4) + i; }
    // LDS position of tile row r such that the rows of one lane are adjacent
    __device__ static inline int pos(int r) { return r; }
    __device__ static inline float bcast(float v, int src) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
    }
    // reciprocal of a pivot: hardware estimate (about 1 ulp in FP32)
    __device__ static inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
};
template <>
struct MfmaTile<double> {
    typedef doublex4_t acc;
    __device__ static inline acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // FP64: element i of a lane sits at row lane/16 + 4*i, column lane%16
    __device__ static inline int row(int lane, int i) { return (lane >> 4) + 4 * i; }
    // LDS position of tile row r such that the rows of one lane (r = g + 4 i) are adjacent
    __device__ static inline int pos(int r) { return 4 * (r & 3) + (r >> 2); }
    __device__ static inline double bcast(double v, int src) {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
    // reciprocal of a pivot: hardware estimate refined by two Newton steps
    __device__ static inline double recip(double x) {
        double r = __builtin_amdgcn_rcp(x);
        r = fma(r, fma(-x, r, 1.0), r);
        r = fma(r, fma(-x, r, 1.0), r);
        return r;
    }
};

// Window of NT tile-rows (R = 16 NT rows): NT = 4 for half-bandwidths up to 48, NT = 6
// for up to 80.  Rows 0..63 of the window are one per lane ("set 1"); with NT = 6,
// rows 64..95 are held by lanes 0..31 as a second set of registers ("set 2").
// Register budget: the FP32 64-row instance is held to 168 registers (three waves per
// SIMD instead of two; it has no spills), the others keep the compiler's choice.
template <typename T, int NT>
struct BandWaves {
    static constexpr int value = (sizeof(T) == 4 && NT == 4) ? 3 : 1;
};

template <typename T, int MODE, int NT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(BandWaves<T, NT>::value, 8))) void local_band_mfma_kernel(
    int s, int E, int BWS, const int* __restrict__ subptr, const int* __restrict__ sd, const double2* __restrict__ sv,
    const double* __restrict__ lam, const T* __restrict__ Floc, long long ldF, T* __restrict__ zloc,
    T* __restrict__ Lwork, const long long* __restrict__ Loff, const int* __restrict__ sysord,
    int* __restrict__ status, int* __restrict__ negflag) {
    constexpr int mode = MODE;
    using MT = MfmaTile<T>;
    using acc_t = typename MT::acc;
    constexpr int R = 16 * NT;
    constexpr bool TWO = R > 64;            // a second set of window rows (64 .. R-1)
    static_assert(R <= 128 && (NT == 4 || NT == 6), "window of 64 or 96 rows");
    constexpr int EPL = 2;                  // slot entries a lane carries (E <= 4 * EPL)
    // LDS: panT (column-major panel, accumulator -> row-per-lane), pan (row-major factored
    // panel, -> MFMA operands; reused column-major by the backward sweep), nrowT (the
    // tile-row entering the window, column-major with rows permuted so that the four
    // accumulator rows of a lane are adjacent), vec (shift of the right-hand side)
    // (strides keep 16-byte alignment and spread lanes over banks: with PS = 84 and
    // QS = 20 FP32 words, the 16-byte accesses of 16 consecutive rows (lr * PS, lr * QS)
    // fall on distinct banks; the FP64 sizes keep a workgroup under 20 KB so that eight
    // fit in one compute unit's LDS)
    constexpr int PS = TWO ? (sizeof(T) == 4 ? 124 : 114) : (sizeof(T) == 4 ? 84 : 82);
    constexpr int QS = sizeof(T) == 4 ? 20 : 18;
    static_assert(16 * PS >= R * QS, "pan aliases panT");
    __shared__ __align__(16) T panT[16][PS];
    __shared__ __align__(16) T nrowT[R][QS];
    T (*pan)[QS] = reinterpret_cast<T (*)[QS]>(&panT[0][0]);   // free once a[] is read
    __shared__ T vec[R];
    __shared__ T colsum[16];
    auto VEC = [&](const int r) -> T& { return vec[r]; };
    auto CSUM = [&](const int c) -> T& { return colsum[c]; };
    const int sys = sysord[blockIdx.x];        // larger subdomains first (host-planned order)
    // mode 0: shift lambda_i, and negflag[sys] records a negative pivot (K_l - lambda_i M_l
    // indefinite); mode 1: only the recorded systems, again with shift 0
    if (mode && !negflag[sys]) return;
    const int l = sys / s;
    const int i = sys - l * s;
    const int off = subptr[l];
    const int nl = subptr[l + 1] - off;
    const int npan = (nl + 15) >> 4;
    const double lamd = mode ? 0.0 : lam[i];
    const int lane = threadIdx.x, lr = lane & 15, lg = lane >> 4;
    const int q = lane >> 2, slot0 = lane & 3;
    T* Lp = Lwork + Loff[l] + (long long)i * npan * (16 * BWS);
    const T* f = Floc + (long long)i * ldF + off;
    T* z = zloc + (long long)i * ldF + off;

    acc_t A[NT][NT];
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = 0; J < NT; ++J) A[I][J] = acc_t{T(0), T(0), T(0), T(0)};
    for (int e = lane; e < R * QS; e += 64) (&nrowT[0][0])[e] = T(0);

    // fixed-slot lower entries of local row r: band offset sd (-1 = empty), (K, M) values sv.
    // The loads are issued unconditionally (from a clamped index) and consumed only when
    // the rows are placed, so that they stay in flight across a whole panel step.
    int pdr[EPL];
    double2 pvr[EPL];
    bool pok[EPL];
    auto fetch = [&](const int rb) {       // entries of row rb + q for this lane's slots
        const int r = rb + q;
#pragma unroll
        for (int u = 0; u < EPL; ++u) {
            const int e = slot0 + 4 * u;
            pok[u] = (r < nl && e < E);
            const long long k = pok[u] ? (long long)(off + r) * E + e : 0LL;
            pdr[u] = sd[k];
            pvr[u] = sv[k];
        }
    };
    // tile-row I of the window <- the fetched rows rb..rb+15, window column base cb.
    // Entries are scattered into the zeroed nrowT, gathered in accumulator layout, and
    // the scattered positions are zeroed again.
    const int qpos = MT::pos(q);
    auto place = [&](const int I, const int rb, const int cb) {
        const int r = rb + q;
        int col[EPL];
#pragma unroll
        for (int u = 0; u < EPL; ++u) {
            col[u] = -1;
            if (r < nl) {
                if (pok[u] && pdr[u] >= 0) col[u] = r - pdr[u] - cb;
            } else if (u == 0 && slot0 == 0) {
                col[u] = r - cb;
            }
        }
#pragma unroll
        for (int u = 0; u < EPL; ++u)
            if (col[u] >= 0) nrowT[col[u]][qpos] = (r < nl) ? (T)(pvr[u].x - lamd * pvr[u].y) : T(1);
        wave_sync();
#pragma unroll
        for (int J = 0; J < NT; ++J) {
            if (J <= I) {
                const T* src = &nrowT[16 * J + lr][4 * lg];
#pragma unroll
                for (int ii = 0; ii < 4; ++ii) A[I][J][ii] = src[ii];
            }
        }
        wave_sync();
#pragma unroll
        for (int u = 0; u < EPL; ++u)
            if (col[u] >= 0) nrowT[col[u]][qpos] = T(0);
        wave_sync();
    };

#pragma unroll
    for (int I = 0; I < NT; ++I) {
        fetch(16 * I);
        place(I, 16 * I, 0);
    }
    T y = (lane < nl) ? f[lane] : T(0);
    T y2 = T(0);
    if constexpr (TWO) {   // an unconditional, clamped load and a select
        const T fv = f[min(64 + (lane & 31), nl - 1)];
        y2 = (lane < R - 64 && 64 + lane < nl) ? fv : T(0);
    }
    int bad = 0, neg = 0;

    for (int P = 0; P < npan; ++P) {
        const int base = 16 * P;
        // prefetch the tile-row entering after this panel and its right-hand side
        fetch(base + 16 * NT);
        const int rnew = base + 16 + lane;
        const T fraw = f[min(rnew, nl - 1)];
        const int rnew2 = base + 80 + lane;            // set 2: window row 64 + lane after the slide
        const T fraw2 = TWO ? f[min(rnew2, nl - 1)] : T(0);
        // panel (tile column 0) -> one row per lane, through the column-major panT
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) panT[lr][16 * I + MT::row(lane, ii)] = A[I][0][ii];
        wave_sync();
        T a[16], a2[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) a[c] = panT[c][lane];
        if constexpr (TWO) {
#pragma unroll
            for (int c = 0; c < 16; ++c) a2[c] = panT[c][min(64 + lane, R - 1)];
        }
        // column c: the broadcasts of row c are all issued before the updates that use
        // them (a scheduling barrier keeps them apart), so each lands in an SGPR of its own
        // and no update waits out the SGPR-write hazard of the broadcast just before it
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const T u = a[c];
            const T dc = MT::bcast(u, c);
            const T rc = MT::recip(dc);
            T bc[16];
#pragma unroll
            for (int c2 = c + 1; c2 < 16; ++c2) bc[c2] = MT::bcast(u, c2);
            const T yc = MT::bcast(y, c);
            __builtin_amdgcn_sched_barrier(0);
            const T lt = u * rc;
#pragma unroll
            for (int c2 = c + 1; c2 < 16; ++c2) a[c2] -= lt * bc[c2];
            if (lane > c) y -= lt * yc;
            a[c] = (lane == c) ? dc : lt;
            if constexpr (TWO) {       // rows 64.. lie below the panel: plain elimination
                const T lt2 = a2[c] * rc;
#pragma unroll
                for (int c2 = c + 1; c2 < 16; ++c2) a2[c2] -= lt2 * MT::bcast(u, c2);
                y2 -= lt2 * yc;
                a2[c] = lt2;
            }
        }
        // store the factored panel and D^{-1} L^{-1} f of its 16 rows: column c keeps its
        // band part, window rows c .. c + BWS - 1 (lanes write consecutive values)
        T* Lpan = Lp + (long long)P * (16 * BWS) + lane;
        // three forms, chosen at compile time for FP32 so that its loop holds one of them:
        // FP32, 64-row window: the band part of each column (rows c .. c + BWS - 1), stored
        // by every lane (a lane outside the band repeats, by a lane shuffle, the value of
        // the nearest band row, at that row's address); FP32, 96-row window: full columns
        // (BWS == R); FP64: full columns or the masked band part
        if constexpr (sizeof(T) == 4 && !TWO) {
            T* Lb = Lp + (long long)P * (16 * BWS);
            // the 16 shuffles are all issued before the first store (one LDS wait, not 16)
            T sv[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) sv[c] = __shfl(a[c], min(max(lane, c), c + BWS - 1), 64);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int lc = min(max(lane, c), c + BWS - 1);
                Lb[c * BWS + (lc - c)] = sv[c];
            }
        } else if (sizeof(T) == 4 || BWS >= R) {
#pragma unroll
            for (int c = 0; c < 16; ++c) Lpan[c * R] = a[c];
            if constexpr (TWO) {
                if constexpr (sizeof(T) == 4) {
                    // rows 64.. by every lane: lanes 32.. repeat the values of lanes 0..31
#pragma unroll
                    for (int c = 0; c < 16; ++c) Lpan[c * R + 64 + (lane & 31) - lane] = __shfl(a2[c], lane & 31, 64);
                } else if (lane < R - 64) {
#pragma unroll
                    for (int c = 0; c < 16; ++c) Lpan[c * R + 64] = a2[c];
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (lane >= c && lane - c < BWS) Lpan[c * BWS - c] = a[c];
            if constexpr (TWO) {
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    if (lane < R - 64 && 64 + lane - c < BWS) Lpan[c * BWS - c + 64] = a2[c];
            }
        }
        wave_sync();
#pragma unroll
        for (int c = 0; c < 16; ++c) pan[lane][c] = a[c];
        if constexpr (TWO) {
            if (lane < R - 64) {
#pragma unroll
                for (int c = 0; c < 16; ++c) pan[64 + lane][c] = a2[c];
            }
        }
        wave_sync();
        if constexpr (sizeof(T) == 4) {
            // the pivots of the panel, one per lane: a zero, tiny or non-finite pivot marks
            // the factorisation as failed (checked once per panel, off the elimination chain)
            const T dl = pan[lane & 15][lane & 15];
            if (lane < 16 && base + lane < nl) {
                bad |= !(fabs(dl) > T(1e-30) && fabs(dl) < T(1e30));
                neg |= dl < T(0);
            }
            // D^{-1} L^{-1} f of the panel rows, stored by every lane (each group of 16 lanes
            // writes the same 16 values; rows past the end repeat the last row's value), so
            // no store sits under a branch and the compiler's memory counters stay exact
            // across the loop (the prefetched loads then stay in flight)
            const int zr = min(lane & 15, nl - 1 - base);
            const T zv = __shfl(y * MT::recip(dl), zr, 64);
            z[base + zr] = zv;
        } else {
            // FP64: the masked form (the shuffles of the form above cost this instance more
            // registers than they save)
            if (lane < 16 && base + lane < nl) {
                const T dl = pan[lane][lane];
                bad |= !(fabs(dl) > T(1e-30) && fabs(dl) < T(1e30));
                neg |= dl < T(0);
                z[base + lane] = y * MT::recip(dl);
            }
        }
        // trailing update of tiles (I, J), 1 <= J <= I: -= L_I D L_J^T; k-step k of a lane
        // group lg covers panel column 4 lg + k, so each lane reads 4 adjacent columns
        T dcol[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) dcol[k] = pan[4 * lg + k][4 * lg + k];
        T aop[NT][4], bop[NT][4];
#pragma unroll
        for (int I = 1; I < NT; ++I) {
            const T* src = &pan[16 * I + lr][4 * lg];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T lv = src[k];
                bop[I][k] = lv;
                aop[I][k] = -lv * dcol[k];
            }
        }
        __builtin_amdgcn_sched_barrier(0);      // every operand read is issued before the first MFMA
#pragma unroll
        for (int I = 1; I < NT; ++I)
#pragma unroll
            for (int J = 1; J <= I; ++J)
#pragma unroll
                for (int k = 0; k < 4; ++k) A[I][J] = MT::mma(aop[I][k], bop[J][k], A[I][J]);
        wave_sync();
        // slide the window by 16 rows
#pragma unroll
        for (int I = 1; I < NT; ++I)
#pragma unroll
            for (int J = 1; J <= I; ++J) A[I - 1][J - 1] = A[I][J];
        if (P + 1 < npan) place(NT - 1, base + 16 * NT, base + 16);
        // shift the right-hand side by 16 window rows; fresh rows enter at the bottom
        VEC(lane) = y;
        if constexpr (TWO) {
            if (lane < R - 64) VEC(64 + lane) = y2;
        }
        wave_sync();
        y = (lane < R - 16) ? VEC(min(lane + 16, R - 1)) : ((rnew < nl) ? fraw : T(0));
        if constexpr (TWO) y2 = (lane < R - 80) ? VEC(min(80 + lane, R - 1)) : ((lane < R - 64 && rnew2 < nl) ? fraw2 : T(0));
        wave_sync();
    }

    // backward sweep with L^T, panel by panel from the end; zw holds z of the window rows.
    // Two register buffers alternate: a panel is read two steps before it is used, so
    // the loads overlap two panel steps; indices are clamped so every load is in bounds.
    T zw = T(0), zw2 = T(0);                // z of window rows lane (and 64 + lane)
    T (*bt)[PS] = panT;                     // column-major panel copy
    T bufA[16], bufB[16], bufA2[16], bufB2[16];
    T zA, zB;
    auto load_panel = [&](const int P, T (&dst)[16], T (&dst2)[16], T& zdst) {
        const int Pc = max(P, 0);
        const T* Lpan = Lp + (long long)Pc * (16 * BWS) + lane;
        if constexpr (sizeof(T) == 4 && !TWO) {
            // band part: every lane loads the nearest band row of its column (in bounds)
            // and keeps it only where its own row lies in the band
            const T* Lb = Lp + (long long)Pc * (16 * BWS);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int lc = min(max(lane, c), c + BWS - 1);
                const T v = Lb[c * BWS + (lc - c)];
                dst[c] = (lc == lane) ? v : T(0);
            }
        } else if (sizeof(T) == 4 || BWS >= R) {
#pragma unroll
            for (int c = 0; c < 16; ++c) dst[c] = Lpan[c * R];
            if constexpr (TWO) {
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    const T v = Lpan[c * R + 64 + (lane & 31) - lane];   // in bounds for every lane
                    dst2[c] = (lane < R - 64) ? v : T(0);
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < 16; ++c) dst[c] = (lane >= c && lane - c < BWS) ? Lpan[c * BWS - c] : T(0);
            if constexpr (TWO) {
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    dst2[c] = (lane < R - 64 && 64 + lane - c < BWS) ? Lpan[c * BWS - c + 64] : T(0);
            }
        }
        zdst = z[min(16 * Pc + lr, nl - 1)];
    };
    auto back_step = [&](const int P, T (&a)[16], T (&a2)[16], T& zb) {
        const int base = 16 * P;
        const T zc0 = (lane < 16 && base + lane < nl) ? zb : T(0);
        VEC(lane) = zw;
        if constexpr (TWO) {
            if (lane < R - 64) VEC(64 + lane) = zw2;
        }
        wave_sync();
        zw = (lane >= 16) ? VEC(max(lane - 16, 0)) : T(0);
        if constexpr (TWO) zw2 = (lane < R - 64) ? VEC(min(48 + lane, R - 1)) : T(0);
        wave_sync();
        // column-major copy of the panel in LDS (reusing the panel buffer): rows below
        // the panel hold L(r, c) z_r, the 16 panel rows hold L(r, c) itself
#pragma unroll
        for (int c = 0; c < 16; ++c) bt[c][lane] = (lane >= 16) ? a[c] * zw : a[c];
        if constexpr (TWO) {
            if (lane < R - 64) {
#pragma unroll
                for (int c = 0; c < 16; ++c) bt[c][64 + lane] = a2[c] * zw2;
            }
        }
        wave_sync();
        // this buffer is free again: start reading the panel two steps further down
        load_panel(P - 2, a, a2, zb);
        // contributions of the R - 16 rows below the panel: lane (c, quarter) sums
        // (R - 16) / 4 rows of column c, then the four quarters are added with quad
        // permutations
        {
            constexpr int RQ = (R - 16) / 4;
            const int c = lane >> 2, qq = lane & 3;
            const T* src = &bt[c][16 + RQ * qq];
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < RQ; ++j) acc += src[j];
            acc = quad_sum(acc);
            if (qq == 0) CSUM(c) = acc;
        }
        // multipliers L(r, lane) of the rows r above which this lane's row lies, zero
        // elsewhere (selected here, off the dependent chain of the solve below)
        T lt[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const T v = bt[lr][r];
            lt[r] = (lane < r) ? v : T(0);
        }
        wave_sync();
        // unit upper triangular solve with the panel's 16 x 16 block, one row per step
        // (a lane at or below row r subtracts 0 * z_r, which leaves its value unchanged)
        T val = zc0 - CSUM(lr);
#pragma unroll
        for (int r = 15; r > 0; --r) {
            const T zr = MT::bcast(val, r);
            val -= lt[r] * zr;
        }
        if (lane < 16) zw = val;
        if constexpr (sizeof(T) == 4) {
            const int zr = min(lane & 15, nl - 1 - base);
            const T zv = __shfl(val, zr, 64);
            z[base + zr] = zv;            // every lane (duplicates write equal values)
        } else {
            if (lane < 16 && base + lane < nl) z[base + lane] = val;
        }
        wave_sync();
    };
    load_panel(npan - 1, bufA, bufA2, zA);
    load_panel(npan - 2, bufB, bufB2, zB);
    for (int P = npan - 1; P >= 0; P -= 2) {
        back_step(P, bufA, bufA2, zA);
        if (P >= 1) back_step(P - 1, bufB, bufB2, zB);
    }
    if (__any(bad) && lane == 0) atomicOr(status, STATUS_LOCAL_PIVOT);   // pivots were checked per lane
    const bool indefinite = __any(neg);
    if (mode == 0 && lane == 0) negflag[sys] = indefinite ? 1 : 0;
}

// Local extraction (numeric setup): the lower entries of every local row of
// every subdomain in fixed slots, band offset and (K, M) value pair.
__global__ void extract_local_kernel(long long sumN, int E, const int* __restrict__ lptr, const int* __restrict__ ldd,
                                     const int* __restrict__ lpos, const double2* __restrict__ km,
                                     int* __restrict__ sd, double2* __restrict__ sv) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= sumN) return;
    const int e0 = lptr[r], e1 = lptr[r + 1];
    for (int e = 0; e < E; ++e) {
        const bool has = e0 + e < e1;
        sd[r * E + e] = has ? ldd[e0 + e] : -1;
        sv[r * E + e] = has ? km[lpos[e0 + e]] : make_double2(0.0, 0.0);
    }
}

void launch_extract_local(hipStream_t st, long long sumN, int E, const int* lptr, const int* ldd, const int* lpos,
                          const double2* km, int* sd, double2* sv) {
    hipLaunchKernelGGL(extract_local_kernel, dim3(grid_for(sumN, 256)), dim3(256), 0, st, sumN, E, lptr, ldd, lpos,
                       km, sd, sv);
}

// Local solves, blocked, wide bands (FP32): the blocked LDL^T above with a window of
// 192 rows (12 tile-rows, half-bandwidths up to 176) and up to 20 lower entries per row
// (fourth-order and three-dimensional elements).  One workgroup of four wavefronts per
// (subdomain, shift).  The 78 lower tiles of the window live in LDS (16 x 16 FP32 in accumulator order:
// element (r, c) at 4 (16 (r / 4) + c) + r % 4, so that lane l's four accumulator values,
// rows 4 (l / 16) + 0..3 of column l % 16, are the 16 bytes at 16 l), one ring per tile
// diagonal d = I - J: the tiles of diagonal d
// belong to absolute tile-rows TR = P + d .. P + 11 and take slot TR mod (12 - d) of the
// ring, so when the window slides the retiring panel tile of each ring frees exactly the
// slot its entering tile needs (TR = P + 12 = P + d mod 12 - d) and nothing moves.  Per
// panel: the panel tiles are read to one row per lane (three row sets, rows 64 w + lane
// on wave w < 3) and factored with lane broadcasts (wave 0 records each step of the pivot
// block for the two other sets); wave 3 scatters the next tile-row into the freed slots;
// the factored panel goes to HBM (full 192-row columns) and, row-major, to LDS as MFMA
// operands; each of the 66 trailing tiles is read, takes -L_I D L_J^T with four 16x16x4
// MFMAs and is written back.  The right-hand side shifts through LDS; the backward sweep sums the
// contributions of the 176 rows below each panel through a column-major LDS copy.
constexpr int WIDE_NT = 12;                 // tile-rows of the window
constexpr int WIDE_R = 16 * WIDE_NT;        // window rows (192)
constexpr int WIDE_EPL = 5;                 // fixed slots a lane carries (E <= 20)
constexpr int WIDE_TILES = WIDE_NT * (WIDE_NT + 1) / 2;   // 78 ring slots

// first ring slot of diagonal d and its ring size
__host__ __device__ constexpr int wide_ring_base(int d) { return WIDE_NT * d - d * (d - 1) / 2; }
__host__ __device__ constexpr int wide_ring_size(int d) { return WIDE_NT - d; }

template <int MODE>
__global__ __launch_bounds__(256) void local_band_wide_kernel(
    int s, int E, const int* __restrict__ subptr, const int* __restrict__ bwv, const int* __restrict__ sd,
    const double2* __restrict__ sv,
    const double* __restrict__ lam, const float* __restrict__ Floc, long long ldF, float* __restrict__ zloc,
    float* __restrict__ Lwork, const long long* __restrict__ Loff, const int* __restrict__ sysord,
    int* __restrict__ status, int* __restrict__ negflag) {
    // Four wavefronts per system, one per SIMD.  Wave w < 3 holds window rows 64 w ..
    // 64 w + 63 (row set w); wave 3 brings in the entering tile-rows.  Wave 0 eliminates
    // the pivot block (and its rows 16..63) while wave 3 places the next tile-row; waves 1
    // and 2 then apply the recorded steps to rows 64..191.  The trailing tile-rows are
    // split over the four waves (16-17 tiles each at a full band); the backward sweep
    // runs on wave 0.  Barriers are LDS-only except one full barrier after the forward
    // sweep (the factor columns waves 1 and 2 stored are read back by wave 0).
    using T = float;
    using MT = MfmaTile<T>;
    using acc_t = typename MT::acc;
    constexpr int NT = WIDE_NT, R = WIDE_R, EPL = WIDE_EPL;
    constexpr int QS = 20;                     // row stride of the factored panel (16-byte rows, spread banks)
    constexpr int PS = 196;                    // backward sweep: column stride of its panel copy
    static_assert(WIDE_TILES * 256 >= 16 * PS, "the backward sweep's copy aliases the tile rings");
    __shared__ __align__(16) T tiles[WIDE_TILES * 256];
    __shared__ __align__(16) T pan[R][QS];
    __shared__ T vec[R];
    __shared__ T colsum[16];
    __shared__ T ucol[16][17];                 // column c of the panel at elimination step c
    __shared__ T urc[16], uyc[16];             // pivot reciprocal and y_c of step c
    const int sys = sysord[blockIdx.x];        // larger subdomains first (host-planned order)
    if (MODE && !negflag[sys]) return;         // uniform over the workgroup
    const int l = sys / s;
    const int i = sys - l * s;
    const int off = subptr[l];
    const int nl = subptr[l + 1] - off;
    const int npan = (nl + 15) >> 4;
    // tile-rows of the panel that can hold a nonzero (rows r - c <= w below the panel's
    // columns): the trailing update of the others adds zero and is skipped
    const int imax = min(NT - 1, (bwv[l] + 15) >> 4);
    const double lamd = MODE ? 0.0 : lam[i];
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int q = lane >> 2, slot0 = lane & 3;
    T* Lp = Lwork + Loff[l] + (long long)i * npan * (16 * R);
    const float* f = Floc + (long long)i * ldF + off;
    float* z = zloc + (long long)i * ldF + off;
    // tile (I, J) of the window of panel P: ring d = I - J, absolute tile-row P + I
    auto tile = [&](const int P, const int I, const int J) -> T* {
        const int d = I - J;
        return tiles + (wide_ring_base(d) + (P + I) % wide_ring_size(d)) * 256;
    };

    int pdr[EPL];
    double2 pvr[EPL];
    bool pok[EPL];
    auto fetch = [&](const int rb) {           // slots of row rb + q for this lane
        const int r = rb + q;
#pragma unroll
        for (int u = 0; u < EPL; ++u) {
            const int e = slot0 + 4 * u;
            pok[u] = (r < nl && e < E);
            const long long k = pok[u] ? (long long)(off + r) * E + e : 0LL;
            pdr[u] = sd[k];
            pvr[u] = sv[k];
        }
    };
    // the fetched rows rb..rb+15 as tile-row I of panel P's window (its tiles zeroed
    // before): entry (row, column) of the window goes to tile (I, column / 16)
    auto place = [&](const int P, const int I, const int rb) {
        const int r = rb + q;
        const int cb = 16 * P;                 // first column of the window
#pragma unroll
        for (int u = 0; u < EPL; ++u) {
            int cw = -1;
            T v = T(1);
            if (r < nl) {
                if (pok[u] && pdr[u] >= 0) {
                    cw = r - pdr[u] - cb;
                    v = (T)(pvr[u].x - lamd * pvr[u].y);
                }
            } else if (u == 0 && slot0 == 0) {
                cw = r - cb;                   // identity row past the end
            }
            if (cw >= 0) {
                const int J = cw >> 4, d = I - J;
                T* t = tiles + (wide_ring_base(d) + (P + I) % wide_ring_size(d)) * 256;
                t[4 * (16 * (q >> 2) + (cw & 15)) + (q & 3)] = v;
            }
        }
    };
    auto zero_row_tiles = [&](const int P, const int I) {   // the tiles (I, 0..I)
#pragma unroll
        for (int J = 0; J <= I; ++J)
            reinterpret_cast<floatx4_t*>(tile(P, I, J))[lane] = floatx4_t{T(0), T(0), T(0), T(0)};
    };
    // panel row lr of tile (I, 0): its 16 columns
    auto read_row = [&](const int P, const int I, T (&dst)[16]) {
        const T* t = tiles + (wide_ring_base(I) + (P + I) % wide_ring_size(I)) * 256 + 64 * (lr >> 2) + (lr & 3);
#pragma unroll
        for (int c = 0; c < 16; ++c) dst[c] = t[4 * c];
    };
    // rows below the pivot block: the elimination steps with the values recorded by wave 0
    // (constant trip counts, so that every loop unrolls and the rows stay in registers)
    auto eliminate_below = [&](T (&ar)[16], T& yr) {
#pragma clang loop unroll(full)
        for (int c = 0; c < 16; ++c) {
            const T rc = urc[c], yc = uyc[c];
            T urow[16];
#pragma clang loop unroll(full)
            for (int c2 = 0; c2 < 16; ++c2) urow[c2] = ucol[c][c2];
            const T lt = ar[c] * rc;
#pragma clang loop unroll(full)
            for (int c2 = 0; c2 < 16; ++c2)
                if (c2 > c) ar[c2] -= lt * urow[c2];
            yr -= lt * yc;
            ar[c] = lt;
        }
    };

    // the first window: wave w clears and fills tile-rows 3 w .. 3 w + 2 (a tile-row's
    // entries all lie in its own tiles)
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const int I = 3 * wv + u;
        zero_row_tiles(0, I);
        fetch(16 * I);
        wave_sync();
        place(0, I, 16 * I);
    }
    // right-hand sides: wave w < 3 holds rows 64 w .. 64 w + 63
    T ya = T(0);
    if (wv < 3) {
        const int r0 = 64 * wv + lane;
        const T fa = f[min(r0, nl - 1)];                    // unconditional, clamped, then selected
        ya = (r0 < nl) ? fa : T(0);
    }
    lds_barrier();
    int bad = 0, neg = 0;

    for (int P = 0; P < npan; ++P) {
        const int base = 16 * P;
        const int rnew = base + 16 + 128 + lane;           // set 2 row after the slide (lanes 48..63)
        T fraw = T(0);
        if (wv == 3) fetch(base + R);                      // the tile-row entering after this panel
        if (wv == 2) fraw = f[min(rnew, nl - 1)];
        // panel rows: row 64 w + lane is row lr of tile (4 w + lg, 0)
        T a0[16];
        if (wv < 3) read_row(P, 4 * wv + lg, a0);
        lds_barrier();                                     // the panel tiles are free
        if (wv == 0) {
            // rows 0..63: elimination with lane broadcasts; step c's column (rows c..15),
            // the pivot reciprocal and y_c are recorded for the rows below
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const T u = a0[c];
                const T dc = MT::bcast(u, c);
                const T rc = MT::recip(dc);
                const T yc = MT::bcast(ya, c);
                if (lane < 16) ucol[c][lane] = u;
                if (lane == 0) {
                    urc[c] = rc;
                    uyc[c] = yc;
                }
                T urow[16];
#pragma unroll
                for (int c2 = c + 1; c2 < 16; ++c2) urow[c2] = MT::bcast(u, c2);
                const T lt = u * rc;
#pragma unroll
                for (int c2 = c + 1; c2 < 16; ++c2) a0[c2] -= lt * urow[c2];
                if (lane > c) ya -= lt * yc;
                a0[c] = (lane == c) ? dc : lt;
            }
        } else if (wv == 3 && P + 1 < npan) {
            // the next tile-row takes the panel tiles' slots
            zero_row_tiles(P + 1, NT - 1);
            wave_sync();
            place(P + 1, NT - 1, base + R);
        }
        lds_barrier();
        // rows 64..127 (wave 1) and 128..191 (wave 2) lie below the panel
        if (wv == 1 || wv == 2) eliminate_below(a0, ya);
        // the factored panel's full columns (window rows 0..191) for the backward sweep,
        // and its rows, row-major, as MFMA operands
        if (wv < 3) {
            T* Lb = Lp + (long long)P * (16 * R) + lane + 64 * wv;
#pragma unroll
            for (int c = 0; c < 16; ++c) Lb[c * R] = a0[c];
            T (*prow)[QS] = pan + 64 * wv + lane;
#pragma unroll
            for (int c = 0; c < 16; ++c) prow[0][c] = a0[c];
        }
        lds_barrier();
        if (wv == 0) {
            // pivots of the panel (checked once per panel) and D^{-1} L^{-1} f of its rows,
            // stored by every lane (rows past the end repeat the last row's value)
            const T dl = pan[lane & 15][lane & 15];
            if (lane < 16 && base + lane < nl) {
                bad |= !(fabs(dl) > T(1e-30) && fabs(dl) < T(1e30));
                neg |= dl < T(0);
            }
            const int zr = min(lane & 15, nl - 1 - base);
            const T zv = __shfl(ya * MT::recip(dl), zr, 64);
            z[base + zr] = zv;
        }
        // trailing update of tiles (I, J), 1 <= J <= I: -= L_I D L_J^T; tile-rows
        // {1, 5, 11} on wave 0, {6, 10} on wave 1, {7, 9} on wave 2 and {2, 3, 4, 8} on
        // wave 3 (16-17 tiles each).
        // Per tile-row: its tiles are read together, their MFMAs interleaved, then written
        // back to their ring slots (the next panel's tiles (I - 1, J - 1)).
        T dcol[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) dcol[k] = pan[4 * lg + k][4 * lg + k];
        T bop[NT][4];
#pragma unroll
        for (int J = 1; J < NT; ++J) {
            const T* src = &pan[16 * J + lr][4 * lg];
#pragma unroll
            for (int k = 0; k < 4; ++k) bop[J][k] = src[k];
        }
#pragma clang loop unroll(full)
        for (int I = 1; I < NT; ++I) {
            constexpr long long kOwner = 0x0123'2103'3300LL;   // nibble I: the wave of tile-row I
            const int owner = (int)((kOwner >> (4 * I)) & 15);
            if (I <= imax && wv == owner) {                // uniform per wave
                T aop[4];
#pragma clang loop unroll(full)
                for (int k = 0; k < 4; ++k) aop[k] = -bop[I][k] * dcol[k];
                acc_t acc[NT];
#pragma clang loop unroll(full)
                for (int J = 1; J <= I; ++J) acc[J] = reinterpret_cast<const floatx4_t*>(tile(P, I, J))[lane];
#pragma clang loop unroll(full)
                for (int k = 0; k < 4; ++k)
#pragma clang loop unroll(full)
                    for (int J = 1; J <= I; ++J) acc[J] = MT::mma(aop[k], bop[J][k], acc[J]);
#pragma clang loop unroll(full)
                for (int J = 1; J <= I; ++J) reinterpret_cast<floatx4_t*>(tile(P, I, J))[lane] = acc[J];
            }
        }
        // shift the right-hand side by 16 window rows; fresh rows enter at the bottom
        if (wv < 3) vec[64 * wv + lane] = ya;
        lds_barrier();
        if (wv < 2) ya = vec[64 * wv + 16 + lane];
        else if (wv == 2) ya = (lane < 48) ? vec[144 + lane] : ((rnew < nl) ? fraw : T(0));
        lds_barrier();                                     // tiles and vec complete for the next panel
    }
    __syncthreads();                                       // waves 1 and 2's factor columns are in memory
    if (wv != 0) return;

    // backward sweep with L^T (wave 0), panel by panel from the end; zw holds z of the
    // window rows (three row sets)
    constexpr int NS = 3;
    T zw[NS] = {T(0), T(0), T(0)};
    T (*bt)[PS] = reinterpret_cast<T (*)[PS]>(tiles);
    T bufA[NS][16], bufB[NS][16];
    T zA, zB;
    auto load_panel = [&](const int P, T (&dst)[NS][16], T& zdst) {
        const int Pc = max(P, 0);
        const T* Lpan = Lp + (long long)Pc * (16 * R) + lane;
#pragma unroll
        for (int c = 0; c < 16; ++c)
#pragma unroll
            for (int k = 0; k < NS; ++k) dst[k][c] = Lpan[c * R + 64 * k];
        zdst = z[min(16 * Pc + lr, nl - 1)];
    };
    auto back_step = [&](const int P, T (&a)[NS][16], T& zb) {
        const int base = 16 * P;
        const T zc0 = (lane < 16 && base + lane < nl) ? zb : T(0);
#pragma unroll
        for (int k = 0; k < NS; ++k) vec[64 * k + lane] = zw[k];
        wave_sync();
        zw[0] = (lane >= 16) ? vec[max(lane - 16, 0)] : T(0);
        zw[1] = vec[48 + lane];
        zw[2] = vec[112 + lane];
        wave_sync();
        // column-major copy of the panel: rows below the panel hold L(r, c) z_r, the 16
        // panel rows hold L(r, c) itself
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            bt[c][lane] = (lane >= 16) ? a[0][c] * zw[0] : a[0][c];
            bt[c][64 + lane] = a[1][c] * zw[1];
            bt[c][128 + lane] = a[2][c] * zw[2];
        }
        wave_sync();
        load_panel(P - 2, a, zb);                          // this buffer is free again
        {
            // contributions of the 176 rows below the panel: lane (c, quarter) sums 44 rows
            constexpr int RQ = (R - 16) / 4;
            const int c = lane >> 2, qq = lane & 3;
            const T* src = &bt[c][16 + RQ * qq];
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < RQ; ++j) acc += src[j];
            acc = quad_sum(acc);
            if (qq == 0) colsum[c] = acc;
        }
        T lt[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) lt[r] = bt[lr][r];
        wave_sync();
        T val = zc0 - colsum[lr];
#pragma unroll
        for (int r = 15; r > 0; --r) {
            const T zr = MT::bcast(val, r);
            if (lane < r) val -= lt[r] * zr;
        }
        if (lane < 16) zw[0] = val;
        const int zr = min(lane & 15, nl - 1 - base);
        const T zv = __shfl(val, zr, 64);
        z[base + zr] = zv;
        wave_sync();
    };
    load_panel(npan - 1, bufA, zA);
    load_panel(npan - 2, bufB, zB);
    for (int P = npan - 1; P >= 0; P -= 2) {
        back_step(P, bufA, zA);
        if (P >= 1) back_step(P - 1, bufB, zB);
    }
    if (__any(bad) && lane == 0) atomicOr(status, STATUS_LOCAL_PIVOT);
    const bool indefinite = __any(neg);
    if (MODE == 0 && lane == 0) negflag[sys] = indefinite ? 1 : 0;
}

template <typename T>
static void launch_local_mfma(hipStream_t st, int mode, int nt, int nsub, int s, int E, int bws, long long sumN,
                              const int* subptr, const int* bw, const int* sd, const double2* sv, const double* lam, const T* Floc,
                              T* zloc, T* Lwork, const long long* Loff, const int* sysord, int* status, int* negflag) {
    // mode 0: every system with shift lambda_i; mode 1: the systems found indefinite,
    // again with shift 0 (its waves return at once when no system was flagged).
    // nt: window tile-rows (4 or 6; 12: the wide FP32 kernel, whose stored columns are full)
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(nsub * s), dim3(64), 0, st, s, E, bws, subptr, sd, sv, lam, Floc, sumN, zloc,
                           Lwork, Loff, sysord, status, negflag);
    };
    if (nt == 4) {
        if (mode == 0) go(local_band_mfma_kernel<T, 0, 4>);
        else go(local_band_mfma_kernel<T, 1, 4>);
    } else if (nt == WIDE_NT) {
        if constexpr (sizeof(T) == 4) {
            auto wide = [&](auto kernel) {
                hipLaunchKernelGGL(kernel, dim3(nsub * s), dim3(256), 0, st, s, E, subptr, bw, sd, sv, lam, Floc,
                                   sumN, zloc, Lwork, Loff, sysord, status, negflag);
            };
            if (mode == 0) wide(local_band_wide_kernel<0>);
            else wide(local_band_wide_kernel<1>);
        }
    } else {
        if (mode == 0) go(local_band_mfma_kernel<T, 0, 6>);
        else go(local_band_mfma_kernel<T, 1, 6>);
    }
}

template <typename T>
static void launch_local(hipStream_t st, int nsub, int s, int maxC, long long sumN, const int* subptr, const int* bw,
                         int E, const int* sd, const double2* sv, const double* lam, const T* Floc, T* zloc,
                         T* Lwork, const long long* Loff, int* status, int threads) {
    const size_t shmem = (size_t)(maxC * maxC + 2 * maxC) * sizeof(T);
    hipLaunchKernelGGL(local_ldlt_kernel<T>, dim3(nsub * s), dim3(threads), shmem, st, s, E, subptr, bw, sd, sv, lam, Floc,
                       sumN, zloc, Lwork, Loff, status);
}

void launch_local_solve_f64(hipStream_t st, int mode, int nsub, int s, int maxC, long long sumN,
                            const int* subptr, const int* bw, int blocked, int E, int bws, const int* sd,
                            const double2* sv, const double* lam, const double* Floc, double* zloc, double* Lwork,
                            const long long* Loff, const int* sysord, int* status, int* negflag, int threads) {
    if (blocked) {
        launch_local_mfma<double>(st, mode, blocked, nsub, s, E, bws, sumN, subptr, bw, sd, sv, lam, Floc, zloc, Lwork, Loff,
                               sysord, status, negflag);
        return;
    }
    if (mode == 0)   // the windowed solver takes its second pass inside the kernel
        launch_local<double>(st, nsub, s, maxC, sumN, subptr, bw, E, sd, sv, lam, Floc, zloc, Lwork, Loff, status,
                             threads);
}

void launch_local_solve_f32(hipStream_t st, int mode, int nsub, int s, int maxC, long long sumN,
                            const int* subptr, const int* bw, int blocked, int E, int bws, const int* sd,
                            const double2* sv, const double* lam, const float* Floc, float* zloc, float* Lwork,
                            const long long* Loff, const int* sysord, int* status, int* negflag, int threads) {
    if (blocked) {
        launch_local_mfma<float>(st, mode, blocked, nsub, s, E, bws, sumN, subptr, bw, sd, sv, lam, Floc, zloc, Lwork, Loff,
                               sysord, status, negflag);
        return;
    }
    if (mode == 0)   // the windowed solver takes its second pass inside the kernel
        launch_local<float>(st, nsub, s, maxC, sumN, subptr, bw, E, sd, sv, lam, Floc, zloc, Lwork, Loff, status,
                            threads);
}

// ---------------------------------------------------------------------------
// Z(d, i) = sum_b P(d,b) Zhat(b,i) + sum over the (subdomain, local row) copies
// of dof d of zloc_i, in the order of the reverse map (deterministic).
template <typename T>
__global__ __launch_bounds__(256) void scatter_kernel(int n, int s, long long sumN, const int* __restrict__ Pptr,
                                                      const int* __restrict__ Pcol, const double* __restrict__ Pval,
                                                      const double* __restrict__ Zhat, const int* __restrict__ rptr,
                                                      const int* __restrict__ ridx, const T* __restrict__ zloc,
                                                      double* __restrict__ Z, int ldz) {
    // one dof per thread, every shift in registers: for a shift, consecutive threads read
    // consecutive local positions of zloc_i (the dofs of a subdomain keep their order);
    // the sums go through LDS so that Z is written with consecutive threads on
    // consecutive columns of a row
    extern __shared__ double scatter_tile[];   // [s][257]: shift i of dof d0 + r at i * 257 + r
    const int t = threadIdx.x;
    const int d0 = blockIdx.x * 256;
    const int d = d0 + t;
    const int cnt = min(256, n - d0);
    if (d < n) {
        double acc[BPJD_MAX_BLOCK];
#pragma unroll
        for (int i = 0; i < BPJD_MAX_BLOCK; ++i) acc[i] = 0.0;
        const int p0 = Pptr[d], p1 = Pptr[d + 1], e0 = rptr[d], e1 = rptr[d + 1];
        // the indices (and weights) of four entries, and of four copies, are loaded
        // together before their values; the sums keep the entry and copy order
        constexpr int U = 4;
        for (int qb = p0; qb < p1; qb += U) {
            int pc[U];
            double pv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = min(qb + u, p1 - 1);
                pc[u] = Pcol[q];
                pv[u] = Pval[q];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (qb + u < p1)
#pragma unroll
                    for (int i = 0; i < BPJD_MAX_BLOCK; ++i)
                        if (i < s) acc[i] = fma(pv[u], Zhat[pc[u] * s + i], acc[i]);
        }
        for (int eb = e0; eb < e1; eb += U) {
            int ri[U];
#pragma unroll
            for (int u = 0; u < U; ++u) ri[u] = ridx[min(eb + u, e1 - 1)];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (eb + u < e1)
#pragma unroll
                    for (int i = 0; i < BPJD_MAX_BLOCK; ++i)
                        if (i < s) acc[i] += (double)zloc[(long long)i * sumN + ri[u]];
        }
#pragma unroll
        for (int i = 0; i < BPJD_MAX_BLOCK; ++i)
            if (i < s) scatter_tile[i * 257 + t] = acc[i];
    }
    __syncthreads();
    int r = t / s, i = t - r * s;                      // element e = t + 256 k: (e / s, e % s)
    const int dr = 256 / s, di = 256 - dr * s;
    for (int e = t; e < cnt * s; e += 256) {
        Z[(long long)(d0 + r) * ldz + i] = scatter_tile[i * 257 + r];
        r += dr;
        i += di;
        if (i >= s) {
            i -= s;
            ++r;
        }
    }
}

void launch_scatter_f64(hipStream_t st, int n, int s, int sumN, const int* Pptr, const int* Pcol, const double* Pval,
                        const double* Zhat, const int* rptr, const int* ridx, const double* zloc, double* Z, int ldz) {
    hipLaunchKernelGGL(scatter_kernel<double>, dim3(grid_for(n, 256)), dim3(256), sizeof(double) * s * 257, st, n, s,
                       (long long)sumN, Pptr, Pcol, Pval, Zhat, rptr, ridx, zloc, Z, ldz);
}

void launch_scatter_f32(hipStream_t st, int n, int s, int sumN, const int* Pptr, const int* Pcol, const double* Pval,
                        const double* Zhat, const int* rptr, const int* ridx, const float* zloc, double* Z, int ldz) {
    hipLaunchKernelGGL(scatter_kernel<float>, dim3(grid_for(n, 256)), dim3(256), sizeof(double) * s * 257, st, n, s,
                       (long long)sumN, Pptr, Pcol, Pval, Zhat, rptr, ridx, zloc, Z, ldz);
}

}  // namespace bpjd
