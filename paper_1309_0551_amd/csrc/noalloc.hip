// noalloc.hip -- the library's fixed device scratch array and lgt_force_noalloc,
// the fermion force with its two scratch vectors in that array instead of
// context workspace, for callers that cannot allocate device memory.
//
// The array is a file-scope device variable: every GPU the library runs on
// holds its own copy until the process ends. In host code its name is only a
// host-side stand-in, so its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// ever passed to kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "ctx.hpp"

namespace lgt {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};
} // namespace

lgt_status scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(LGT_ERR_UNSUPPORTED, "device %d: at most %d devices are supported", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return LGT_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(LGT_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device,
                    hipGetErrorString(e));
    g_scratch[device] = ptr;
    return LGT_OK;
}

void *scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[device];
}

} // namespace lgt

using namespace lgt;

extern "C" lgt_status lgt_force_noalloc(lgt_ctx *c, const lgt_links *U, const double *X, double scale, double *G)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    lgt_status s;
    if ((s = check_links(U, true, &f)) != LGT_OK) return s;
    // X and Y = D_oe X in native layout, one FP64 parity vector each, Y at the
    // next 256-byte boundary after X
    const size_t v64 = (size_t)c->g.Vh * 48;
    const size_t off = (v64 + 255) / 256 * 256;
    if (off + v64 > kScratchBytes)
        return fail(LGT_ERR_UNSUPPORTED, "lgt_force_noalloc needs %zu bytes of scratch for V/2 = %d sites; the "
                    "array holds %zu (V/2 <= %zu)", off + v64, c->g.Vh, kScratchBytes, (kScratchBytes - 255) / 96);
    if ((s = check_ptr(X, "X")) != LGT_OK) return s;
    if ((s = check_ptr(G, "G")) != LGT_OK) return s;
    if (!std::isfinite(scale)) return fail(LGT_ERR_ARG, "scale must be finite");
    unsigned char *base = (unsigned char *)scratch_ptr(c->device);
    if (!base) return fail(LGT_ERR_DEVICE, "no scratch address for device %d", c->device);
    DeviceScope ds(c->device);
    return force_run(c, U, f, X, scale, G, (double *)base, (double *)(base + off));
}
