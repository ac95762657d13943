// Library state: per-device twiddle tables, error reporting, version.
#include <cmath>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace ldk {

__device__ cplx<double> g_tw_hi_f64[TW_SIZE];
__device__ cplx<double> g_tw_lo_f64[TW_SIZE];
__device__ cplx<float> g_tw_hi_f32[TW_SIZE];
__device__ cplx<float> g_tw_lo_f32[TW_SIZE];

static thread_local int t_last_hip_error = 0;

void set_hip_error(hipError_t e) { t_last_hip_error = (int)e; }

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_init_mutex;
bool g_ready[MAX_DEVICES];

// exp(-2 pi i q / N) in extended precision, rounded once to the target type.
void fill_table(int log_n, std::vector<cplx<double>> &d, std::vector<cplx<float>> &f)
{
    const long double two_pi = 6.283185307179586476925286766559005768L;
    const long double N = std::ldexp(1.0L, log_n);
    d.resize(TW_SIZE);
    f.resize(TW_SIZE);
    for (int q = 0; q < TW_SIZE; ++q) {
        const long double ang = -two_pi * (long double)q / N;
        const long double c = cosl(ang), s = sinl(ang);
        d[q] = {(double)c, (double)s};
        f[q] = {(float)c, (float)s};
    }
}
}  // namespace

int ensure_init()
{
    int dev = 0;
    LDK_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return LDK_ENOTSUP;
    std::lock_guard<std::mutex> lock(g_init_mutex);
    if (g_ready[dev]) return LDK_OK;
    std::vector<cplx<double>> hd, ld;
    std::vector<cplx<float>> hf, lf;
    fill_table(TW_BITS, hd, hf);
    fill_table(TW_MAX_LOG, ld, lf);
    LDK_HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(g_tw_hi_f64), hd.data(), sizeof(cplx<double>) * TW_SIZE));
    LDK_HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(g_tw_lo_f64), ld.data(), sizeof(cplx<double>) * TW_SIZE));
    LDK_HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(g_tw_hi_f32), hf.data(), sizeof(cplx<float>) * TW_SIZE));
    LDK_HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(g_tw_lo_f32), lf.data(), sizeof(cplx<float>) * TW_SIZE));
    LDK_HIP_CHECK(hipDeviceSynchronize());
    // per-device set-up of the allocation-free entry point's scratch address
    const int st = noalloc_setup();
    if (st) return st;
    g_ready[dev] = true;
    return LDK_OK;
}

}  // namespace ldk

extern "C" {

int ldk_init(void) { return ldk::ensure_init(); }

int ldk_last_hip_error(void) { return ldk::t_last_hip_error; }

const char *ldk_version(void) { return "0.1.0"; }

const char *ldk_strerror(int status)
{
    switch (status) {
    case LDK_OK: return "ok";
    case LDK_EINVAL: return "invalid argument";
    case LDK_ENOTSUP: return "unsupported combination of arguments";
    case LDK_EDEVICE: return "HIP runtime error (see ldk_last_hip_error)";
    case LDK_ENOTSPD: return "matrix not positive definite (lambda + sigma^2 <= 0)";
    case LDK_ETOOBIG: return "input exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
    }
}

}  // extern "C"
