// The coarse generalized eigenproblem without device allocation, for callers that
// cannot allocate (code under HIP graph capture, serving loops that forbid it).
//
// Same kernels and the same steps as the coarse part of the numeric setup (Section 3,
// the spectral split V^H = U^H_s (+) U^H_{s+1} that the coarse term of eq.
// Preconditioner uses): M_H = L L^T (banded Cholesky), C = L^{-1} K_H L^{-T}, the
// symmetric eigensolver on C, Y = L^{-T} Z.  The working arrays live in `scratch`, a
// file-scope device array of fixed size (one copy per GPU, held for the life of the
// process); its device address is looked up once per device when a context is created
// on it.  Calls on one GPU share that array: calls that overlap in time on one GPU
// (two streams, two threads) race on it.
#include "common.h"

namespace bpjd {

constexpr int kNoAllocMaxCoarse = 320;   // largest n_H: the one-workgroup tridiagonalisation
// L (n^2), K_H copy then Z (n^2), C (n^2), reflectors (n^2), inverse-iteration scratch
// (6 n^2), eigensolver vectors (6 n + 1)
constexpr long long kNoAllocScratchDoubles =
    10LL * kNoAllocMaxCoarse * kNoAllocMaxCoarse + 6LL * kNoAllocMaxCoarse + 64;

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's `scratch` (the host-side symbol is only a stand-in).
// Called with `device` current; once per device.
int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(BPJD_ERR_ARG, "device ordinal above the supported range");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return BPJD_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(BPJD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<double*>(ptr);
    return BPJD_OK;
}

__global__ void clear_info_kernel(int* info) { *info = 0; }

}  // namespace bpjd

using namespace bpjd;

extern "C" int bpjd_coarse_eigen_noalloc(bpjd_ctx* ctx, int32_t n_H, int32_t bw, const double* KH, const double* MH,
                                         double* lamH, double* Y, int32_t* info) {
    CtxScope cs_(ctx);
    if (!ctx || !KH || !MH || !lamH || !Y || !info) return fail(BPJD_ERR_ARG, "NULL argument");
    if (n_H < 1 || n_H > kNoAllocMaxCoarse)
        return fail(BPJD_ERR_ARG, "n_H = " + std::to_string(n_H) + " outside 1.." + std::to_string(kNoAllocMaxCoarse) +
                                      " (the fixed scratch of the allocation-free call)");
    if (bw < 0 || bw > n_H - 1) return fail(BPJD_ERR_ARG, "bandwidth outside 0..n_H-1");
    double* base = nullptr;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch_ptr[ctx->device];
    }
    if (!base) return fail(BPJD_ERR_STATE, "scratch address of the device not set up");
    BPJD_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const long long n2 = (long long)n_H * n_H;
    double* L = base;                 // M_H, factored in place
    double* E0 = base + n2;           // L^{-1} K_H, then the eigenvectors Z of C
    double* Cm = base + 2 * n2;       // C = L^{-1} K_H L^{-T} (destroyed by the eigensolver)
    double* E1 = base + 3 * n2;       // Householder reflectors
    double* E2 = base + 4 * n2;       // inverse-iteration scratch (6 n^2)
    double* small = base + 10 * n2;   // 6 n + 1
    hipLaunchKernelGGL(clear_info_kernel, dim3(1), dim3(1), 0, st, reinterpret_cast<int*>(info));
    launch_copy_cols(st, n_H, n_H, MH, n_H, L, n_H);
    launch_cholesky(st, n_H, bw, L, reinterpret_cast<int*>(info), STATUS_COARSE_NOT_SPD);
    launch_copy_cols(st, n_H, n_H, KH, n_H, E0, n_H);
    launch_trsm_band(st, n_H, bw, n_H, L, E0, n_H, false);        // L^{-1} K_H
    launch_transpose(st, n_H, E0, Cm);                            // K_H L^{-T}
    launch_trsm_band(st, n_H, bw, n_H, L, Cm, n_H, false);        // L^{-1} K_H L^{-T}
    launch_sym_eig(st, n_H, Cm, lamH, E0, E1, small, E2, reinterpret_cast<int*>(info));
    launch_copy_cols(st, n_H, n_H, E0, n_H, Y, n_H);
    launch_trsm_band(st, n_H, bw, n_H, L, Y, n_H, true);          // Y = L^{-T} Z
    BPJD_HIP(hipGetLastError());
    return BPJD_OK;
}
