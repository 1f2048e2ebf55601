// dtw_noalloc.hip -- fixed device scratch of rawalign_dtw_batch_noalloc.
//
// The batch path needs scratch beyond its inputs and outputs: the planning
// histogram, counts and queue heads, the per-route pair lists, and one
// stripe-edge slot per resident wave of the multi-stripe kernel.  The
// allocating entry points take it from per-(device, stream) hipMalloc
// buffers.  For callers that cannot allocate, it lives here instead, in one
// file-scope device array of fixed size that every GPU holds from the moment
// the library's code is loaded on it until the process ends.
//
// The array's name is a host-side stand-in in host code, not a device
// address: the address of each device's copy is looked up once per device
// with hipGetSymbolAddress and only that address is ever handed to kernels.
#include <mutex>

#include "internal.h"

namespace {

using namespace ra;

constexpr size_t kAlign = 256;
constexpr size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Layout: planning words | pair lists | edge slots, each 256-byte aligned.
constexpr size_t kWordsBytes = round_up(sizeof(int32_t) * ((size_t)kNumRoutes * kBuckets + 2 * kNumRoutes));
constexpr size_t kListBytes = round_up(sizeof(int32_t) * (size_t)kNumRoutes * kNoallocMaxPairs);
constexpr size_t kEdgeBytes = sizeof(float) * (size_t)kNoallocEdgeSlots * kEdgeCap;
constexpr size_t kScratchBytes = kWordsBytes + kListBytes + kEdgeBytes;
static_assert(kScratchBytes == kNoallocScratchBytes, "scratch size");

static __device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

namespace ra {

hipError_t noalloc_scratch(int dev, PlanScratch &out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    void *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        p = g_ptr[dev];
        if (!p) {
            // The caller has made `dev` current; each device holds its own
            // copy of the array at its own address.
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            if (!p) return hipErrorInvalidSymbol;
            g_ptr[dev] = p;
        }
    }
    char *base = static_cast<char *>(p);
    out.hist = reinterpret_cast<int32_t *>(base);
    out.counts = out.hist + kNumRoutes * kBuckets;
    out.queue = out.counts + kNumRoutes;
    out.list = reinterpret_cast<int32_t *>(base + kWordsBytes);
    out.capacity = kNoallocMaxPairs;
    out.edge = reinterpret_cast<float *>(base + kWordsBytes + kListBytes);
    out.rowbuf = nullptr;
    return hipSuccess;
}

}  // namespace ra
