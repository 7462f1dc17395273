// Diagnostic entry points (include/lrr_diag.h): the solver's building blocks
// exposed one by one for isolated checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "../../include/lrr_diag.h"

struct lrr_ctx;   // defined in solver.hip

namespace lrr {
lrr_status ctx_fail(lrr_ctx* ctx, lrr_status st, const std::string& msg);
int ctx_device(const lrr_ctx* ctx);
}  // namespace lrr

namespace {

__global__ void k_pad_copy(const double* __restrict__ src, int lds, long sstride, double* __restrict__ dst,
                           int L, const int* __restrict__ ls) {
    const int b = blockIdx.y;
    const int l = ls[b];
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)L * L) return;
    const int i = (int)(idx % L), j = (int)(idx / L);
    dst[(long)b * L * L + idx] = (i < l && j < l) ? src[b * sstride + i + (long)j * lds] : 0.0;
}

__global__ void k_unpad(const double* __restrict__ Wp, int L, double* __restrict__ W, int ldw, long stride,
                        const double* __restrict__ lamp, double* __restrict__ lam, int ldlam,
                        const int* __restrict__ ls) {
    const int b = blockIdx.y;
    const int l = ls[b];
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)l * l) return;
    const int i = (int)(idx % l), j = (int)(idx / l);
    W[b * stride + i + (long)j * ldw] = Wp[(long)b * L * L + i + (long)j * L];
    if (i == 0) lam[(long)b * ldlam + j] = lamp[(long)b * L + j];
}

template <class F>
lrr_status run(lrr_ctx* ctx, F&& f) {
    try {
        if (hipSetDevice(lrr::ctx_device(ctx)) != hipSuccess)
            return lrr::ctx_fail(ctx, LRR_EDEVICE, "hipSetDevice failed");
        return f();
    } catch (const lrr::HipError& e) {
        return lrr::ctx_fail(ctx, LRR_EDEVICE, e.msg);
    }
}

}  // namespace

extern "C" {

lrr_status lrr_diag_dgemm(lrr_ctx* ctx, int ta, int tb, int M, int N, int K, double alpha, const double* A,
                          int lda, const double* B, int ldb, double beta, double* C, int ldc, void* stream) {
    return lrr_diag_gemm(ctx, LRR_FP64, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream);
}

lrr_status lrr_diag_gemm(lrr_ctx* ctx, int precision, int ta, int tb, int M, int N, int K, double alpha,
                         const double* A, int lda, const double* B, int ldb, double beta, double* C, int ldc,
                         void* stream) {
    if (!ctx) return lrr::ctx_fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (precision != LRR_FP64 && precision != LRR_FP32 && precision != LRR_MIXED_BF16)
        return lrr::ctx_fail(ctx, LRR_EINVAL, "unknown precision");
    if (M <= 0 || N <= 0 || K <= 0 || !A || !B || !C) return lrr::ctx_fail(ctx, LRR_EINVAL, "bad GEMM arguments");
    if (lda < (ta ? K : M) || ldb < (tb ? N : K) || ldc < M) return lrr::ctx_fail(ctx, LRR_EINVAL, "leading dimension too small");
    if (precision == LRR_FP64 && (lda >= lrr::kGemmMaxLd || ldb >= lrr::kGemmMaxLd))
        return lrr::ctx_fail(ctx, LRR_EINVAL, "lda and ldb must be below 4194304");
    return run(ctx, [&]() -> lrr_status {
        hipStream_t s = static_cast<hipStream_t>(stream);
        lrr::GemmDesc h{A, B, C, M, N, K, lda, ldb, ldc, alpha, beta, nullptr, nullptr};
        lrr::GemmDesc* d = nullptr;
        LRR_HIP(hipMalloc((void**)&d, sizeof(h)));
        LRR_HIP(hipMemcpy(d, &h, sizeof(h), hipMemcpyHostToDevice));
        const int mode = precision == LRR_FP32 ? lrr::kGemmFP32
                         : precision == LRR_MIXED_BF16 ? lrr::kGemmBF16X3 : lrr::kGemmFP64;
        // A^T A (the same pointer and stride on both sides): the symmetric
        // kernel computes the tiles on and above the diagonal and mirrors them
        if (mode == lrr::kGemmFP64 && ta && !tb && A == B && lda == ldb && M == N)
            lrr::launch_dgemm_sym(d, 1, N, s, true);
        else
            lrr::launch_xgemm(d, 1, M, N, ta != 0, tb != 0, mode, s);
        LRR_HIP(hipStreamSynchronize(s));
        LRR_HIP(hipFree(d));
        return LRR_OK;
    });
}

lrr_status lrr_diag_spd_inverse(lrr_ctx* ctx, int m, int n, const double* A, int lda, double* Kinv, int ldk,
                                void* stream) {
    if (!ctx) return lrr::ctx_fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (m <= 0 || n <= 0 || !A || !Kinv || lda < m || ldk < m)
        return lrr::ctx_fail(ctx, LRR_EINVAL, "bad arguments");
    if (lda >= lrr::kGemmMaxLd || ldk >= lrr::kGemmMaxLd) return lrr::ctx_fail(ctx, LRR_EINVAL, "leading dimensions must be below 4194304");
    return run(ctx, [&]() -> lrr_status {
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t mm = (size_t)m * m;
        double *K, *Lb, *Li, *Tb, *Di;
        int* info;
        lrr::GemmDesc* d;
        const int nd = lrr::spd_inverse_desc_count(m) + 1;
        LRR_HIP(hipMalloc((void**)&K, sizeof(double) * mm));
        LRR_HIP(hipMalloc((void**)&Lb, sizeof(double) * mm));
        LRR_HIP(hipMalloc((void**)&Li, sizeof(double) * mm));
        LRR_HIP(hipMalloc((void**)&Tb, sizeof(double) * mm));
        LRR_HIP(hipMalloc((void**)&Di, sizeof(double) * (size_t)m * 32));
        LRR_HIP(hipMalloc((void**)&info, sizeof(int)));
        LRR_HIP(hipMalloc((void**)&d, sizeof(lrr::GemmDesc) * nd));
        lrr::GemmDesc h{A, A, K, m, m, n, lda, lda, m, 1.0, 0.0, nullptr, nullptr};
        LRR_HIP(hipMemcpy(d + nd - 1, &h, sizeof(h), hipMemcpyHostToDevice));
        lrr::launch_dgemm(d + nd - 1, 1, m, m, false, true, s);
        lrr::launch_add_identity(K, m, m, 1.0, s);
        lrr::spd_inverse(K, m, Lb, Li, Di, Tb, d, info, s);
        lrr::launch_copy_cols(K, m, Kinv, ldk, m, m, s);
        int hinfo = 0;
        LRR_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
        LRR_HIP(hipStreamSynchronize(s));
        (void)hipFree(K); (void)hipFree(Lb); (void)hipFree(Li); (void)hipFree(Tb);
        (void)hipFree(Di); (void)hipFree(info); (void)hipFree(d);
        if (hinfo != 0) return lrr::ctx_fail(ctx, LRR_ENUMERIC, "matrix not positive definite");
        return LRR_OK;
    });
}

lrr_status lrr_diag_syevj(lrr_ctx* ctx, int count, const int* l, const double* B, int ldb, long strideB,
                          double* lam, int ldlam, double* W, int eig_block, int* sweeps, void* stream) {
    if (!ctx) return lrr::ctx_fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (count <= 0 || !l || !B || !lam || !W) return lrr::ctx_fail(ctx, LRR_EINVAL, "bad arguments");
    int maxl = 0;
    for (int i = 0; i < count; ++i) {
        if (l[i] <= 0 || l[i] > ldb || l[i] > ldlam) return lrr::ctx_fail(ctx, LRR_EINVAL, "bad order");
        maxl = std::max(maxl, l[i]);
    }
    if (strideB < (long)ldb * maxl) return lrr::ctx_fail(ctx, LRR_EINVAL, "stride too small");
    const int bs = (eig_block == 32) ? 32 : 16;
    const int L = ((maxl + 2 * bs - 1) / (2 * bs)) * (2 * bs);
    return run(ctx, [&]() -> lrr_status {
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t LL = (size_t)L * L;
        double *Bp, *Wp, *Rp, *lamp, *scale;
        int *st, *run_on, *ls, *any, *prot, *lo;
        lrr::EigDesc* dd;
        LRR_HIP(hipMalloc((void**)&Bp, sizeof(double) * LL * count));
        LRR_HIP(hipMalloc((void**)&Wp, sizeof(double) * LL * count));
        LRR_HIP(hipMalloc((void**)&Rp, sizeof(double) * (size_t)L * 2 * bs * count));
        LRR_HIP(hipMalloc((void**)&lamp, sizeof(double) * (size_t)L * count));
        LRR_HIP(hipMalloc((void**)&scale, sizeof(double) * count));
        LRR_HIP(hipMalloc((void**)&st, sizeof(int) * 2 * count));
        LRR_HIP(hipMalloc((void**)&run_on, sizeof(int) * count));
        LRR_HIP(hipMalloc((void**)&ls, sizeof(int) * count));
        LRR_HIP(hipMalloc((void**)&any, sizeof(int)));
        const int npair = L / (2 * bs);
        LRR_HIP(hipMalloc((void**)&prot, sizeof(int) * npair * count));
        // no threshold here: every pair of indices is resolved
        LRR_HIP(hipMalloc((void**)&lo, sizeof(int) * (size_t)L * count));
        LRR_HIP(hipMemsetAsync(lo, 0, sizeof(int) * (size_t)L * count, s));
        LRR_HIP(hipMalloc((void**)&dd, sizeof(lrr::EigDesc) * count));
        std::vector<lrr::EigDesc> hd(count);
        std::vector<int> ones(count, 1);
        for (int i = 0; i < count; ++i)
            hd[i] = lrr::EigDesc{Bp + LL * i, Wp + LL * i, Rp + (size_t)L * 2 * bs * i, lamp + (size_t)L * i,
                                 L, l[i], run_on + i, st + 2 * i, scale + i, prot + npair * i,
                                 lo + (size_t)L * i, nullptr};
        LRR_HIP(hipMemcpy(dd, hd.data(), sizeof(lrr::EigDesc) * count, hipMemcpyHostToDevice));
        LRR_HIP(hipMemcpy(run_on, ones.data(), sizeof(int) * count, hipMemcpyHostToDevice));
        LRR_HIP(hipMemcpy(ls, l, sizeof(int) * count, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_pad_copy, dim3((unsigned)((LL + 255) / 256), count), dim3(256), 0, s, B, ldb,
                           strideB, Bp, L, ls);
        for (int i = 0; i < count; ++i) lrr::launch_set_identity(Wp + LL * i, L, s);
        lrr::launch_jacobi_init(dd, count, s);
        const int nb = L / bs;
        int sw = 0, h_any = 1;
        for (sw = 0; sw <= 60; ++sw) {
            LRR_HIP(hipMemsetAsync(any, 0, sizeof(int), s));
            lrr::launch_jacobi_check(dd, count, L, any, s);
            LRR_HIP(hipMemcpyAsync(&h_any, any, sizeof(int), hipMemcpyDeviceToHost, s));
            LRR_HIP(hipStreamSynchronize(s));
            if (h_any == 0 || sw == 60) break;
            for (int r = 0; r < nb - 1; ++r) lrr::launch_jacobi_round(dd, count, L, bs, r, s);
        }
        lrr::launch_jacobi_eigvals(dd, count, s);
        hipLaunchKernelGGL(k_unpad, dim3((unsigned)((LL + 255) / 256), count), dim3(256), 0, s, Wp, L, W, ldb,
                           strideB, lamp, lam, ldlam, ls);
        LRR_HIP(hipStreamSynchronize(s));
        if (sweeps) *sweeps = sw;
        (void)hipFree(Bp); (void)hipFree(Wp); (void)hipFree(Rp); (void)hipFree(lamp); (void)hipFree(scale);
        (void)hipFree(st); (void)hipFree(run_on); (void)hipFree(ls); (void)hipFree(any); (void)hipFree(dd);
        (void)hipFree(prot);
        (void)hipFree(lo);
        return LRR_OK;
    });
}

}  // extern "C"
