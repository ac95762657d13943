// Checked entry points (solve and log-det that report a matrix that is not
// positive definite) and the interval quantiles used by the RQMC and
// Bayesian-cubature intervals, all in library code.
//
// K + sigma^2 I = V (Lambda + sigma^2 I) conj(V) with V unitary (Sec. 5.4),
// so it is positive definite exactly when every lambda_k + sigma^2 > 0.  The
// checked calls count the eigenvalues that fail this on the device, wait for
// the count, and return LDK_ENOTSPD without enqueueing the solve or log-det
// when it is not zero.
#include <cmath>
#include <mutex>

#include "common.hpp"

namespace ldk {

namespace {

// One counter per device (each device holds its own copy); the checked
// calls are serialised by g_check_mutex, since they share it.
__device__ unsigned int g_notspd_count;

constexpr int MAX_DEVICES = 64;
std::mutex g_check_mutex;
unsigned int *g_count_ptr[MAX_DEVICES];

__global__ void k_zero_count(unsigned int *count) { *count = 0u; }

// Counts k with !(lambda_k + sigma2 > 0) (NaN counts as failing).
__global__ __launch_bounds__(256) void k_count_notspd(const double *__restrict__ lam, int64_t total,
                                                      double sigma2, unsigned int *count)
{
    unsigned int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * 256)
        bad += !(lam[i] + sigma2 > 0.0);
    // wave sum, then one atomic per wave that saw a failure
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) bad += __shfl_xor(bad, o, 64);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(count, bad);
}

// Number of eigenvalues of R rows of 2^m with lambda + sigma2 <= 0, after
// the work already on `s`.  Synchronises s.  Caller holds g_check_mutex.
int count_notspd(const double *lam, int64_t total, double sigma2, hipStream_t s,
                 unsigned int *bad)
{
    int dev = 0;
    LDK_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return LDK_ENOTSUP;
    if (!g_count_ptr[dev]) {
        void *p = nullptr;
        LDK_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(g_notspd_count)));
        g_count_ptr[dev] = static_cast<unsigned int *>(p);
    }
    unsigned int *count = g_count_ptr[dev];
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, count);
    LDK_LAUNCH_CHECK();
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_count_notspd, dim3((unsigned)blocks), dim3(256), 0, s, lam, total, sigma2,
                       count);
    LDK_LAUNCH_CHECK();
    unsigned int h = 0;
    LDK_HIP_CHECK(hipMemcpyAsync(&h, count, sizeof(h), hipMemcpyDeviceToHost, s));
    LDK_HIP_CHECK(hipStreamSynchronize(s));
    *bad = h;
    return LDK_OK;
}

// ---------------------------------------------------------------------------
// Quantiles (host code)
// ---------------------------------------------------------------------------

// Standard normal CDF through erfc (no cancellation in either tail).
double norm_cdf(double x) { return 0.5 * std::erfc(-x * 0.70710678118654752440); }

// Standard normal quantile.  Start: Abramowitz and Stegun 26.2.23 (a rational
// approximation in t = sqrt(-2 log q), q the smaller tail, absolute error
// below 4.5e-4); then Halley steps on Phi(x) - p, whose derivative phi(x) and
// second derivative -x phi(x) are closed forms.  Three steps take the start
// to full double precision (Halley converges cubically).
double norm_quantile(double p)
{
    if (p == 0.5) return 0.0;
    const double q = p < 0.5 ? p : 1.0 - p;
    const double t = std::sqrt(-2.0 * std::log(q));
    double x = t - (2.515517 + t * (0.802853 + t * 0.010328)) /
                       (1.0 + t * (1.432788 + t * (0.189269 + t * 0.001308)));
    if (p < 0.5) x = -x;
    for (int it = 0; it < 4; ++it) {
        // Phi(x) - p, from the smaller tail so that nothing cancels
        const double res = p < 0.5 ? norm_cdf(x) - p : (1.0 - p) - norm_cdf(-x);
        const double phi = 0.39894228040143267794 * std::exp(-0.5 * x * x);
        if (!(phi > 0.0)) break;
        const double u = res / phi;
        // Halley: f = Phi - p, f' = phi, f'' = -x phi
        const double step = u / (1.0 + 0.5 * x * u);
        x -= step;
        if (std::fabs(step) <= 1e-17 * std::fabs(x)) break;
    }
    return x;
}

// Regularised incomplete beta I_x(a, b) by its continued fraction (DLMF
// 8.17.22), evaluated with the modified Lentz method, on the side where it
// converges fast (x < (a + 1) / (a + b + 2)); the symmetry
// I_x(a, b) = 1 - I_{1-x}(b, a) gives the other side.
double betacf(double a, double b, double x)
{
    const double tiny = 1e-300;
    double c = 1.0, d = 1.0 - (a + b) * x / (a + 1.0);
    if (std::fabs(d) < tiny) d = tiny;
    d = 1.0 / d;
    double h = d;
    for (int mm = 1; mm <= 10000; ++mm) {
        const double m2 = 2.0 * mm;
        // even step d_{2m} = m (b - m) x / ((a + 2m - 1)(a + 2m))
        double an = mm * (b - mm) * x / ((a + m2 - 1.0) * (a + m2));
        d = 1.0 + an * d;
        if (std::fabs(d) < tiny) d = tiny;
        c = 1.0 + an / c;
        if (std::fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        h *= d * c;
        // odd step d_{2m+1} = -(a + m)(a + b + m) x / ((a + 2m)(a + 2m + 1))
        an = -(a + mm) * (a + b + mm) * x / ((a + m2) * (a + m2 + 1.0));
        d = 1.0 + an * d;
        if (std::fabs(d) < tiny) d = tiny;
        c = 1.0 + an / c;
        if (std::fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        const double del = d * c;
        h *= del;
        if (std::fabs(del - 1.0) < 1e-16) break;
    }
    return h;
}

// ln Gamma(a + 1/2) - ln Gamma(a).  For a >= 8 from Stirling's series of
// each term (coefficients B_2k / (2k (2k - 1)): 1/12, -1/360, 1/1260,
// -1/1680, 1/1188), arranged so that nothing large cancels:
//   a log1p(1 / (2a)) + (1/2) log a - 1/2 + sum_k c_k ((a + 1/2)^(1-2k) - a^(1-2k));
// below 8 the library lgamma (values of a few units, little cancellation).
double lgamma_half_ratio(double a)
{
    if (a < 8.0) return std::lgamma(a + 0.5) - std::lgamma(a);
    const double c[5] = {1.0 / 12.0, -1.0 / 360.0, 1.0 / 1260.0, -1.0 / 1680.0, 1.0 / 1188.0};
    double corr = 0.0;
    const double ia = 1.0 / a, ib = 1.0 / (a + 0.5);
    double pa = ia, pb = ib;  // a^(1-2k), (a+1/2)^(1-2k)
    for (int k = 0; k < 5; ++k) {
        corr += c[k] * (pb - pa);
        pa *= ia * ia;
        pb *= ib * ib;
    }
    return a * std::log1p(0.5 * ia) + 0.5 * std::log(a) - 0.5 + corr;
}

// Upper tail P(T > t) of Student's t with nu degrees of freedom, t > 0:
// (1/2) I_x(nu/2, 1/2) with x = nu / (nu + t^2) and 1 - x = t^2 / (nu + t^2),
// both formed from t (not as 1 - x), and the prefactor
// x^a (1 - x)^(1/2) / B(a, 1/2) from log1p(t^2 / nu) and the ratio above
// (B(a, 1/2) = Gamma(a) Gamma(1/2) / Gamma(a + 1/2)).  The continued fraction
// runs on the side where it converges fast; on the other side the result is
// 1 - I_{1-x}(1/2, a), where it is at least about 0.04 (t^2 below about 3),
// so the subtraction costs at most a digit and a half.
double t_upper(double t, double nu)
{
    const double a = 0.5 * nu, b = 0.5;
    const double t2 = t * t;
    const double x = nu / (nu + t2), y = t2 / (nu + t2);
    const double lpre = -a * std::log1p(t2 / nu) + std::log(t) - 0.5 * std::log(nu + t2) +
                        lgamma_half_ratio(a) - 0.5 * std::log(3.14159265358979323846);
    const double pre = std::exp(lpre);  // x^a (1-x)^b / B(a, b)
    if (x < (a + 1.0) / (a + b + 2.0)) return 0.5 * pre * betacf(a, b, x) / a;
    return 0.5 * (1.0 - pre * betacf(b, a, y) / b);
}

// Student-t quantile.  nu = 1 and 2 have closed forms (the Cauchy tangent;
// (2p - 1) / sqrt(2 p (1 - p))).  Otherwise start from the Cornish-Fisher
// expansion about the normal quantile (Abramowitz and Stegun 26.7.5, terms
// to nu^-4) and take Newton steps on the upper tail, whose derivative is
// the density f(t) = (1 + t^2 / nu)^{-(nu+1)/2} / (sqrt(nu) B(nu/2, 1/2)).
double t_quantile(double p, double nu)
{
    if (p == 0.5) return 0.0;
    // Cauchy: tan(pi (p - 1/2)) = -1 / tan(pi p), taken on the smaller tail
    // (p - 1/2 would cancel for small p)
    if (nu == 1.0)
        return p < 0.5 ? -1.0 / std::tan(3.14159265358979323846 * p)
                       : 1.0 / std::tan(3.14159265358979323846 * (1.0 - p));
    if (nu == 2.0) return (2.0 * p - 1.0) / std::sqrt(2.0 * p * (1.0 - p));
    const bool upper = p > 0.5;
    const double q = upper ? 1.0 - p : p;  // target tail probability
    const double x = -norm_quantile(q);    // > 0
    const double x2 = x * x;
    const double g1 = (x2 + 1.0) * x / 4.0;
    const double g2 = ((5.0 * x2 + 16.0) * x2 + 3.0) * x / 96.0;
    const double g3 = (((3.0 * x2 + 19.0) * x2 + 17.0) * x2 - 15.0) * x / 384.0;
    const double g4 = ((((79.0 * x2 + 776.0) * x2 + 1482.0) * x2 - 1920.0) * x2 - 945.0) * x / 92160.0;
    double t = x + (g1 + (g2 + (g3 + g4 / nu) / nu) / nu) / nu;
    const double lnorm = std::lgamma(0.5 * (nu + 1.0)) - std::lgamma(0.5 * nu) -
                         0.5 * std::log(nu * 3.14159265358979323846);
    for (int it = 0; it < 50; ++it) {
        const double f = std::exp(lnorm - 0.5 * (nu + 1.0) * std::log1p(t * t / nu));
        if (!(f > 0.0)) break;
        const double step = (t_upper(t, nu) - q) / f;  // d(upper)/dt = -f
        double tn = t + step;
        if (tn <= 0.0) tn = 0.5 * t;
        const double dd = std::fabs(tn - t);
        t = tn;
        if (dd <= 4e-16 * t) break;
    }
    return upper ? t : -t;
}

}  // namespace

}  // namespace ldk

using namespace ldk;

extern "C" {

int ldk_solve_checked(int kind, int R, int nrhs, int m, int dtype, const double *lam, double sigma2,
                      const void *y, void *c, void *ws, ldk_stream stream)
{
    // argument checks first (an invalid call has no side effects): the
    // plain entry point validates the same arguments, so run its checks on
    // a zero-row call shape-wise equivalent before touching the device
    if (kind != LDK_LATTICE && kind != LDK_DNET_B2) return LDK_EINVAL;
    if (dtype != LDK_F64 && dtype != LDK_F32) return LDK_EINVAL;
    if (m < 0 || m > LDK_MAX_M || R < 0 || nrhs < 0 || !lam || !y || !c) return LDK_EINVAL;
    if (!(sigma2 >= 0.0)) return LDK_EINVAL;
    if ((int64_t)R * nrhs == 0) return LDK_OK;
    if (ldk_workspace_bytes(LDK_OP_SOLVE, kind, (int64_t)R * nrhs, m, dtype) && !ws)
        return LDK_EINVAL;
    std::lock_guard<std::mutex> lock(g_check_mutex);
    unsigned int bad = 0;
    const int st = count_notspd(lam, (int64_t)R << m, sigma2, as_stream(stream), &bad);
    if (st) return st;
    if (bad) return LDK_ENOTSPD;
    return ldk_solve(kind, R, nrhs, m, dtype, lam, sigma2, y, c, ws, stream);
}

int ldk_logdet_checked(int R, int m, const double *lam, double sigma2, double *out, void *ws,
                       ldk_stream stream)
{
    if (m < 0 || m > LDK_MAX_M || R < 0 || R > 65535 || !lam || !out || !(sigma2 >= 0.0))
        return LDK_EINVAL;
    if (R == 0) return LDK_OK;
    if (!ws) return LDK_EINVAL;
    std::lock_guard<std::mutex> lock(g_check_mutex);
    unsigned int bad = 0;
    const int st = count_notspd(lam, (int64_t)R << m, sigma2, as_stream(stream), &bad);
    if (st) return st;
    if (bad) return LDK_ENOTSPD;
    return ldk_logdet(R, m, lam, sigma2, out, ws, stream);
}

double ldk_normal_quantile(double p)
{
    if (!(p > 0.0 && p < 1.0)) return __builtin_nan("");
    return norm_quantile(p);
}

int ldk_student_t_quantile(double p, int dof, double *out)
{
    if (!out || !(p > 0.0 && p < 1.0) || dof < 1) return LDK_EINVAL;
    *out = t_quantile(p, (double)dof);
    return std::isfinite(*out) ? LDK_OK : LDK_EINVAL;
}

}  // extern "C"
