// Entry points that allocate nothing, for callers that cannot call hipMalloc (code
// under HIP graph capture, tight serving loops, harnesses that forbid allocation).
//
// Their scratch memory is one file-scope device array, `scratch`, of a fixed size.
// Each GPU the library runs on holds its own copy at its own address, resolved once
// per device with hipGetSymbolAddress while that device is current (from
// labpsd_ctx_create); host code only ever passes that resolved address to kernels.
// Every call on one GPU shares the array: calls that overlap on one GPU (on
// different streams, or from different threads) race.
#include <mutex>

#include "common.h"

namespace labpsd {

namespace {

// 1 MiB of FP64 partial sums
constexpr size_t kScratchDoubles = size_t(1) << 17;
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

}  // namespace

void noalloc_setup(int device) {
    LABPSD_REQUIRE(device >= 0 && device < kMaxDevices, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return;
    double* ptr = nullptr;
    LABPSD_HIP(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
    LABPSD_REQUIRE(ptr != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
    g_ptr[device] = ptr;
}

static double* scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    double* p = (device >= 0 && device < kMaxDevices) ? g_ptr[device] : nullptr;
    if (!p) throw Error{LABPSD_ESTATE, "scratch array of this device was not set up (labpsd_ctx_create)"};
    return p;
}

size_t noalloc_scratch_doubles() { return kScratchDoubles; }

}  // namespace labpsd

using namespace labpsd;

extern "C" labpsd_status labpsd_residual_noalloc(labpsd_ctx* ctx, int64_t n, int m, const double* PsiH,
                                                 const double* PsiS, int64_t ld, const double* E,
                                                 double sigma0, double* R, int64_t ldr, double* res,
                                                 double* rnorm) {
    return abi_guard([&]() -> labpsd_status {
        LABPSD_REQUIRE(ctx && PsiH && PsiS && E && R && res && rnorm, "NULL argument");
        LABPSD_REQUIRE(n >= 1 && m >= 0 && ld >= n && ldr >= n, "bad sizes");
        const int nblk = residual_blocks(n);
        const size_t need = 2 * (size_t)nblk * (size_t)m;
        LABPSD_REQUIRE(need <= kScratchDoubles,
                       "residual of " + std::to_string(m) + " columns of " + std::to_string(n) +
                           " rows needs " + std::to_string(need) + " scratch doubles; the static array holds " +
                           std::to_string(kScratchDoubles) + " (2 * ceil(n / 4096) * m must not exceed it)");
        double* part = scratch_of(ctx->device);
        launch_residual(n, m, PsiH, PsiS, ld, E, sigma0, R, ldr, part, nblk, ctx->stream);
        launch_residual_finish(m, part, nblk, res, rnorm, ctx->stream);
        return LABPSD_OK;
    });
}
