// Poisson noise of a transient frame (Algorithm 1 step 2.4, after the blur
// of step 2.3), gfx950:
//     T = Poisson(tau * sigma_n) / sigma_n,  sigma_n = Var(tau) / 10^(nr / 10),
// Var the population variance of the whole frame.
//
// k_noise_moments / k_noise_scale   frame mean and variance: per-thread
//     Welford updates, merged pairwise (Chan et al.) in fixed trees within
//     each block and then across the blocks, all fp64, so the result is
//     reproducible.
// k_poisson   one element per thread (grid-stride).  Uniform t of element i
//     is word t mod 4 of Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC
//     2011) at counter (i, t / 4, 0, 0), key (seed, 0x4e4c4f53), scaled from
//     its top 53 bits.  lambda < 10: inversion by sequential search;
//     otherwise Hormann's transformed rejection with squeeze (PTRS).  exp,
//     log and log k! use fixed recipes of IEEE basic operations (compiled
//     without contraction), so the integer decisions are those of any
//     implementation performing the same operations in the same order.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace nlos {

namespace {

constexpr int kNoiseBlock = 256;

struct Moments {
    double n, mean, m2;
};

__device__ __forceinline__ Moments merge(Moments a, Moments b)
{
    if (b.n == 0.0) return a;
    if (a.n == 0.0) return b;
    Moments r;
    r.n = a.n + b.n;
    const double d = b.mean - a.mean;
    r.mean = a.mean + d * (b.n / r.n);
    r.m2 = (a.m2 + b.m2) + d * d * (a.n * (b.n / r.n));
    return r;
}

__device__ Moments block_merge(Moments m)
{
    __shared__ double sn[kNoiseBlock], smean[kNoiseBlock], sm2[kNoiseBlock];
    sn[threadIdx.x] = m.n;
    smean[threadIdx.x] = m.mean;
    sm2[threadIdx.x] = m.m2;
    __syncthreads();
    for (int w = kNoiseBlock / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const Moments a{sn[threadIdx.x], smean[threadIdx.x], sm2[threadIdx.x]};
            const Moments b{sn[threadIdx.x + w], smean[threadIdx.x + w], sm2[threadIdx.x + w]};
            const Moments r = merge(a, b);
            sn[threadIdx.x] = r.n;
            smean[threadIdx.x] = r.mean;
            sm2[threadIdx.x] = r.m2;
        }
        __syncthreads();
    }
    return Moments{sn[0], smean[0], sm2[0]};
}

}  // namespace

__global__ void __launch_bounds__(kNoiseBlock) k_noise_moments(const float* tau, int64_t n, double* part)
{
    Moments m{0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kNoiseBlock;
    for (int64_t i = (int64_t)blockIdx.x * kNoiseBlock + threadIdx.x; i < n; i += stride) {
        const double x = (double)tau[i];
        m.n = m.n + 1.0;
        const double d = x - m.mean;
        m.mean = m.mean + d / m.n;
        m.m2 = m.m2 + d * (x - m.mean);
    }
    m = block_merge(m);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = m.n;
        part[3 * blockIdx.x + 1] = m.mean;
        part[3 * blockIdx.x + 2] = m.m2;
    }
}

// One workgroup: thread t merges blocks t, t + 256, ... in order, then the
// per-thread moments are merged pairwise in a fixed tree -> mean, population
// variance, sigma_n.
__global__ void __launch_bounds__(kNoiseBlock) k_noise_scale(const double* part, int nb, double nr_db, double* out)
{
    Moments m{0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kNoiseBlock)
        m = merge(m, Moments{part[3 * b], part[3 * b + 1], part[3 * b + 2]});
    m = block_merge(m);
    if (threadIdx.x == 0) {
        const double var = m.n > 0.0 ? m.m2 / m.n : 0.0;
        out[0] = m.mean;
        out[1] = var;
        out[2] = var / pow(10.0, nr_db / 10.0);
    }
}

// ---------------------------------------------------------------------------
namespace {

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        const uint64_t a0 = 0xD2E7470EE14C6C93ull * c[0], h0 = __umul64hi(0xD2E7470EE14C6C93ull, c[0]);
        const uint64_t a1 = 0xCA5A826395121157ull * c[2], h1 = __umul64hi(0xCA5A826395121157ull, c[2]);
        const uint64_t n0 = h1 ^ c[1] ^ k0, n2 = h0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = a1;
        c[2] = n2;
        c[3] = a0;
    }
}

__device__ __forceinline__ double uniform_t(uint64_t seed, int64_t i, int t)
{
    uint64_t c[4] = {(uint64_t)i, (uint64_t)(t / 4), 0ull, 0ull};
    philox4x64_10(c, seed, 0x4e4c4f53ull);
    return (double)(c[t % 4] >> 11) * (1.0 / 9007199254740992.0);
}

constexpr double kLn2Hi = 6.93147180369123816490e-01;
constexpr double kLn2Lo = 1.90821492927058770002e-10;
constexpr double kLog2e = 1.44269504088896338700e+00;
constexpr double kPi = 3.14159265358979323846;

// e^x = 2^n e^r, |r| <= ln2 / 2, Taylor terms to r^13; 0 below -708.
__device__ double rexp(double x)
{
    if (x < -708.0) return 0.0;
    const double n = floor(x * kLog2e + 0.5);
    const double r = (x - n * kLn2Hi) - n * kLn2Lo;
    double s = 1.0, t = 1.0;
    for (int k = 1; k <= 13; ++k) {
        t = t * r / (double)k;
        s = s + t;
    }
    return ldexp(s, (int)n);
}

// log x = e ln2 + 2 atanh((m - 1) / (m + 1)), m in [1/sqrt2, sqrt2), series to s^29.
__device__ double rlog(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        e = e - 1;
    }
    const double s = (m - 1.0) / (m + 1.0), s2 = s * s;
    double t = s, acc = 0.0;
    for (int k = 1; k <= 29; k += 2) {
        acc = acc + t / (double)k;
        t = t * s2;
    }
    return 2.0 * acc + ((double)e * kLn2Hi + (double)e * kLn2Lo);
}

// log k!: the product below 20, Stirling's series above.
__device__ double rlogfact(double k)
{
    if (k < 20.0) {
        double f = 1.0;
        for (double i = 2.0; i <= k; i = i + 1.0) f = f * i;
        return rlog(f);
    }
    const double ik = 1.0 / k, ik2 = ik * ik;
    const double series = ik * (1.0 / 12.0 - ik2 * (1.0 / 360.0 - ik2 * (1.0 / 1260.0 - ik2 * (1.0 / 1680.0))));
    return (k * rlog(k) - k) + 0.5 * rlog(2.0 * kPi * k) + series;
}

__device__ int64_t poisson_count(double lam, uint64_t seed, int64_t i)
{
    if (!(lam > 0.0)) return 0;
    if (lam < 10.0) {
        const double u = uniform_t(seed, i, 0);
        double p = rexp(-lam), F = p;
        int64_t k = 0;
        while (u > F && k < 1000) {
            k = k + 1;
            p = p * lam / (double)k;
            F = F + p;
        }
        return k;
    }
    const double slam = sqrt(lam), loglam = rlog(lam);
    const double b = 0.931 + 2.53 * slam;
    const double a = -0.059 + 0.02483 * b;
    const double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    const double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (int it = 0; it < 100000; ++it) {
        const double U = uniform_t(seed, i, 2 * it) - 0.5;
        const double V = uniform_t(seed, i, 2 * it + 1);
        const double us = 0.5 - fabs(U);
        const double kd = floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && V <= vr) return (int64_t)kd;
        if (kd < 0.0 || (us < 0.013 && V > us)) continue;
        const double lhs = (rlog(V) + rlog(invalpha)) - rlog(a / (us * us) + b);
        const double rhs = (-lam + kd * loglam) - rlogfact(kd);
        if (lhs <= rhs) return (int64_t)kd;
    }
    return -1;
}

}  // namespace

__global__ void __launch_bounds__(kNoiseBlock)
    k_poisson(const float* tau, int64_t n, const double* sigma_n, uint64_t seed, float* out)
{
    const double sn = *sigma_n;
    const bool ok = sn > 0.0 && isfinite(sn);
    const int64_t stride = (int64_t)gridDim.x * kNoiseBlock;
    for (int64_t i = (int64_t)blockIdx.x * kNoiseBlock + threadIdx.x; i < n; i += stride) {
        if (!ok) {
            out[i] = 0.f;
            continue;
        }
        const double t = (double)tau[i];
        const double lam = t > 0.0 ? t * sn : 0.0;
        out[i] = (float)((double)poisson_count(lam, seed, i) / sn);
    }
}

hipError_t launch_noise_scale(const float* tau, int64_t n, double nr_db, double* out, double* part, int nb,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_noise_moments, dim3((unsigned)nb), dim3(kNoiseBlock), 0, st, tau, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_noise_scale, dim3(1), dim3(kNoiseBlock), 0, st, part, nb, nr_db, out);
    return hipGetLastError();
}

hipError_t launch_poisson(const float* tau, int64_t n, const double* sigma_n, uint64_t seed, float* out,
                          hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + kNoiseBlock - 1) / kNoiseBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_poisson, dim3((unsigned)blocks), dim3(kNoiseBlock), 0, st, tau, n, sigma_n, seed, out);
    return hipGetLastError();
}

}  // namespace nlos
