// Entry point that allocates no device memory: (I + A A^T)^{-1}, the
// factorisation of the Z-step, with every work buffer in one statically
// allocated device array instead of hipMalloc'ed memory.
//
// `scratch` is a file-scope device array; each GPU the library runs on holds
// its own copy (at its own address) from module load until the process ends.
// Host code never passes the array's name to a kernel or a copy (in host code
// it is a host-side stand-in, not a device address): the device address is
// taken once per device with hipGetSymbolAddress, with that device current, and
// kept in scratch_ptr[device].  Every call on one GPU shares that GPU's array,
// so calls that overlap on one GPU (two streams, two host threads) race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "common.hpp"
#include "kernels.hpp"
#include "../../include/lrr_diag.h"

struct lrr_ctx;   // defined in solver.hip

namespace lrr {
lrr_status ctx_fail(lrr_ctx* ctx, lrr_status st, const std::string& msg);
int ctx_device(const lrr_ctx* ctx);
}  // namespace lrr

namespace {

constexpr int kNoAllocMaxM = 1024;    // largest order m the scratch array serves
constexpr int kMaxDevices = 64;

constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// layout of the scratch array for order m: K, the Cholesky factor, the inverse
// factor and a temporary (m x m each), the inverted diagonal blocks (m x 32),
// the pivot flag and the GEMM descriptors of the blocked factorisation
struct Carve {
    size_t K, Lb, Li, Tb, Di, info, desc, end;
};
constexpr int desc_count(int m) { return 4 * ((m + 31) / 32) + 1 + 1; }
constexpr Carve carve(int m) {
    const size_t mm = sizeof(double) * (size_t)m * m;
    Carve c{};
    c.K = 0;
    c.Lb = align256(c.K + mm);
    c.Li = align256(c.Lb + mm);
    c.Tb = align256(c.Li + mm);
    c.Di = align256(c.Tb + mm);
    c.info = align256(c.Di + sizeof(double) * (size_t)m * 32);
    c.desc = align256(c.info + sizeof(int));
    c.end = align256(c.desc + sizeof(lrr::GemmDesc) * (size_t)desc_count(m));
    return c;
}
constexpr size_t kScratchBytes = carve(kNoAllocMaxM).end;   // 32.3 MiB

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex scratch_mu;
unsigned char* scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev`, looked up once.
lrr_status scratch_base(lrr_ctx* ctx, int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return lrr::ctx_fail(ctx, LRR_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return lrr::ctx_fail(ctx, LRR_EDEVICE,
                                 std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        scratch_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = scratch_ptr[dev];
    return LRR_OK;
}

}  // namespace

extern "C" lrr_status lrr_diag_spd_inverse_noalloc(lrr_ctx* ctx, int m, int n, const double* A, int lda,
                                                   double* Kinv, int ldk, void* stream) {
    if (!ctx) return lrr::ctx_fail(nullptr, LRR_EINVAL, "ctx must not be NULL");
    if (m <= 0 || n <= 0 || !A || !Kinv || lda < m || ldk < m)
        return lrr::ctx_fail(ctx, LRR_EINVAL, "bad arguments");
    if (lda >= lrr::kGemmMaxLd || ldk >= lrr::kGemmMaxLd) return lrr::ctx_fail(ctx, LRR_EINVAL, "leading dimensions must be below 4194304");
    if (m > kNoAllocMaxM)
        return lrr::ctx_fail(ctx, LRR_EINVAL,
                             "m = " + std::to_string(m) + " exceeds the no-allocation limit of " +
                                 std::to_string(kNoAllocMaxM));
    try {
        const int dev = lrr::ctx_device(ctx);
        if (hipSetDevice(dev) != hipSuccess) return lrr::ctx_fail(ctx, LRR_EDEVICE, "hipSetDevice failed");
        unsigned char* base = nullptr;
        const lrr_status st = scratch_base(ctx, dev, &base);
        if (st != LRR_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const Carve c = carve(m);
        double* K = reinterpret_cast<double*>(base + c.K);
        double* Lb = reinterpret_cast<double*>(base + c.Lb);
        double* Li = reinterpret_cast<double*>(base + c.Li);
        double* Tb = reinterpret_cast<double*>(base + c.Tb);
        double* Di = reinterpret_cast<double*>(base + c.Di);
        int* info = reinterpret_cast<int*>(base + c.info);
        lrr::GemmDesc* d = reinterpret_cast<lrr::GemmDesc*>(base + c.desc);
        const int nd = desc_count(m);
        // K = A A^T (the GEMM writes every entry, beta = 0: the previous call's
        // contents are never read), + I, then the blocked factorisation, which
        // clears the factor buffers and the pivot flag itself
        const lrr::GemmDesc h{A, A, K, m, m, n, lda, lda, m, 1.0, 0.0, nullptr, nullptr};
        LRR_HIP(hipMemcpyAsync(d + nd - 1, &h, sizeof(h), hipMemcpyHostToDevice, s));
        lrr::launch_dgemm(d + nd - 1, 1, m, m, false, true, s);
        lrr::launch_add_identity(K, m, m, 1.0, s);
        lrr::spd_inverse(K, m, Lb, Li, Di, Tb, d, info, s);   // synchronises the stream before returning
        lrr::launch_copy_cols(K, m, Kinv, ldk, m, m, s);
        int hinfo = 0;
        LRR_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
        LRR_HIP(hipStreamSynchronize(s));
        if (hinfo != 0) return lrr::ctx_fail(ctx, LRR_ENUMERIC, "matrix not positive definite");
        return LRR_OK;
    } catch (const lrr::HipError& e) {
        return lrr::ctx_fail(ctx, LRR_EDEVICE, e.msg);
    }
}
