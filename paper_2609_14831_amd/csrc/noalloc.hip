// Allocation-free forward action: cut_graph_apply with the partial rows of its
// chunked / tiled forward pass kept in a fixed, file-scope device array instead
// of the handle's reserved work area.  For callers that cannot allocate device
// memory (stream capture, tight serving loops).
#include <mutex>

#include "internal.h"

namespace cut {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

// One copy per device, held until the process ends.  Its name is only a
// host-side stand-in: kernels receive the per-device address looked up below.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

static std::mutex scratch_mu;
static double* scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `dev` (which must be the current device):
// looked up once per device and kept.
static double* scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) CUT_FAIL(CUT_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            CUT_FAIL(CUT_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        scratch_dev[dev] = (double*)p;
    }
    return scratch_dev[dev];
}

}  // namespace cut

using namespace cut;

extern "C" cut_status cut_graph_apply_noalloc(cut_graph_t h, int32_t which, int32_t precision, int64_t nsets,
                                              int64_t nops, const void* eta, int64_t lde, const void* x,
                                              int64_t ldx, double* y, int64_t ldy, uint32_t flags, void* stream) {
    ABI_BEGIN
    Graph& g = checked(h);
    size_t pb = 0;
    const PassArgs p = apply_args(g, which, precision, nsets, nops, eta, lde, x, ldx, y, ldy, flags, &pb);
    if (pb > kScratchBytes)
        CUT_FAIL(CUT_E_INVAL,
                 "cut_graph_apply_noalloc: this shape and tiling need %zu bytes of partial rows, the fixed "
                 "scratch holds %zu (fewer columns, longer chunks or CUT_TILE_NO_CHUNKS)",
                 pb, kScratchBytes);
    DeviceGuard dg(g.device);
    double* part = pb ? scratch_on(g.device) : nullptr;
    launch_forward(g, EPI_Y, p, part, (hipStream_t)stream);
    HIP_CHECK(hipGetLastError());
    ABI_END
}
