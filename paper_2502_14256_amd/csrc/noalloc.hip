// Allocation-free solve: ldk_solve with its intermediate rows in a fixed
// device array of the library instead of a caller workspace, for callers
// that cannot allocate (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).
//
// The array lives in device memory of every GPU the library runs on and
// stays there until the process ends.  Host code never uses its name as an
// address (on the host the name is only a stand-in): its device address is
// looked up once per device with hipGetSymbolAddress and kept in
// g_scratch_ptr[device].
#include <mutex>

#include "common.hpp"

namespace ldk {

namespace {

static __device__ __align__(256) unsigned char scratch[LDK_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[MAX_DEVICES];

}  // namespace

// Looks up this device's copy of the scratch array (once per device; the
// device must be current).  Called by ldk_init's per-device set-up and, if
// that has not run on this device, by the entry point's first call.
int noalloc_setup()
{
    int dev = 0;
    LDK_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return LDK_ENOTSUP;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[dev]) return LDK_OK;
    void *p = nullptr;
    LDK_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return LDK_EDEVICE;
    g_scratch_ptr[dev] = p;
    return LDK_OK;
}

}  // namespace ldk

extern "C" int ldk_solve_noalloc(int kind, int R, int nrhs, int m, int dtype, const double *lam,
                                 double sigma2, const void *y, void *c, ldk_stream stream)
{
    using namespace ldk;
    if (kind != LDK_LATTICE && kind != LDK_DNET_B2) return LDK_EINVAL;
    if (dtype != LDK_F64 && dtype != LDK_F32) return LDK_EINVAL;
    if (m < 0 || m > LDK_MAX_M || R < 0 || nrhs < 0) return LDK_EINVAL;
    const size_t need = ldk_workspace_bytes(LDK_OP_SOLVE, kind, (int64_t)R * nrhs, m, dtype);
    if (need > (size_t)LDK_NOALLOC_SCRATCH_BYTES) return LDK_ETOOBIG;
    int st = ensure_init();  // twiddle tables and, on this device, the scratch address
    if (st) return st;
    st = noalloc_setup();
    if (st) return st;
    int dev = 0;
    LDK_HIP_CHECK(hipGetDevice(&dev));
    void *ws = need ? g_scratch_ptr[dev] : nullptr;
    return ldk_solve(kind, R, nrhs, m, dtype, lam, sigma2, y, c, ws, stream);
}
