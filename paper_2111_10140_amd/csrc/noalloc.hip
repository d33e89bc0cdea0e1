// Allocation-free variant of the product (Sec. 4.3, K alpha ~ Phi D Phi^* alpha,
// summed over the windows of Sec. 5): the same batched stages as
// anova_matvec, with their work space (grids, spread regions, tile sums,
// interpolated values) and launch tables in a static device array instead
// of memory the library allocates, for callers that cannot allocate device
// memory.
//
// The array is a file-scope __device__ symbol.  Its name in host code is
// not a device address: the address is taken once per device with
// hipGetSymbolAddress (each device holds its own copy) and only that
// address is handed to kernels and copies.  Nothing in the array has to
// start at zero: every stage writes all of what a later stage reads
// (regions, tile sums, the whole grid, one value per point).
#include <cmath>
#include <mutex>

#include "anova_internal.h"

namespace anova {
namespace {

// Maximum work space of one call: 64 MiB per device, held until the
// process ends.  A float32 product at N = 1e6 with three 3-D windows and
// one column needs about 14 MB.
constexpr size_t kScratchBytes = (size_t)64 << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;

// Device address of this device's scratch array, looked up on the first
// call on the device (with the device current).
char *scratch_base(int dev) {
    static std::mutex mu;
    static char *addr[kMaxDevices] = {};
    ANOVA_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        ANOVA_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        ANOVA_REQUIRE(ptr != nullptr, "static work space has no device address");
        addr[dev] = static_cast<char *>(ptr);
    }
    return addr[dev];
}

}  // namespace
}  // namespace anova

using namespace anova;

extern "C" anova_status anova_matvec_noalloc(anova_plan_t p, const double *alpha, double *out,
                                             int32_t nrhs, int64_t ld, double beta,
                                             void *stream) {
    return guarded([&] {
        ANOVA_REQUIRE(p != nullptr, "NULL plan");
        ANOVA_REQUIRE(alpha != nullptr && out != nullptr, "NULL vector");
        ANOVA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        ANOVA_REQUIRE(ld >= p->N, "ld must be >= N");
        ANOVA_REQUIRE(std::isfinite(beta), "beta must be finite");
        int dev = 0;
        ANOVA_HIP_CHECK(hipGetDevice(&dev));
        ANOVA_REQUIRE(dev == p->device, "the current device is not the plan's device");
        char *base = scratch_base(dev);
        hipStream_t s = static_cast<hipStream_t>(stream);
        // an earlier call on this stream may still be reading the tables
        // and work space that this call overwrites
        ANOVA_HIP_CHECK(hipStreamSynchronize(s));
        BatchProblem bp;
        bp.plan = p;
        bp.alpha = alpha;
        bp.out = out;
        bp.nrhs = nrhs;
        bp.ld = ld;
        bp.beta = beta;
        const ExternalSpace ext{base, kScratchBytes};
        Batch b;
        b.build({bp}, &ext);
        b.run(s, nullptr);
    });
}

extern "C" int64_t anova_matvec_noalloc_max_bytes(void) { return (int64_t)kScratchBytes; }
