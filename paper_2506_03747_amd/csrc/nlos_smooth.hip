// Smooth time response and its adjoint (confocal), gfx950.
//
// The hard forward bins each pair's arrival; its gradient with respect to
// depth is zero almost everywhere.  The smooth forward gives each pair the
// continuous Gaussian response of the detector jitter (Section 2, temporal
// jitter; sigma = FWHM / (2 sqrt(2 ln 2)) / dt in bins):
//     tau_s[s][k] = sum_p w_sp N(k + 1/2 - u_sp),  |k - floor(u_sp)| <= Rs,
// Rs = ceil(6 sigma), N the normalised Gaussian.  The weight w and arrival u
// are those of the hard forward (Eq. (1) with the cosine and stand-off
// extensions).  Arrivals are computed in fp64: an fp32 distance puts u off by
// ~1e-4 bins at u ~ 1000, which would move the Gaussian samples by ~1e-5.
//
// k_smooth_mom   forward for support radii 12, 16, 20: eight (radius 12) or
//                six moments of the sub-bin offset per pair into LDS rows,
//                then a convolution of each moment row with the matching
//                Gaussian-derivative kernel, four bins per thread from
//                registers.
// k_smooth       forward otherwise: a workgroup owns a tile of scan points
//                (LDS rows of 64-bit fixed-point bins), a lane one patch;
//                2 Rs + 1 LDS adds per pair, Gaussian samples by a
//                three-exponential recurrence.
// k_adj_moments, k_adjoint_mom   adjoint for support radii 12, 16, 20: the
//                upstream gradient's correlations with the Gaussian's
//                derivatives once per scan point, then per pair two series in
//                the sub-bin offset.
// k_adjoint      gather otherwise: a lane owns one patch and loops over a range of scan
//                points whose upstream-gradient rows are staged in LDS; per
//                pair G0 = sum g N(x), G1 = sum g (x / sigma^2) N(x) give
//                dL/dw = G0 and dL/du = w G1; per-record partial gradients
//                (fp64) per scan range, summed in a fixed order afterwards
//                (k_adjoint_reduce, one thread per output word).
// k_grad_scatter / k_grad_gather   record gradients -> depth and albedo maps
//                through the central-difference normals and true areas.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nlos_device.h"
#include "nlos_internal.h"

namespace nlos {

namespace {

typedef unsigned long long u64s;

__device__ __forceinline__ int smooth_active(const SmoothArgs& a)
{
    int n = a.n_cap;
    if (a.n_active) {
        n = *a.n_active;
        n = n < 0 ? 0 : (n > a.n_cap ? a.n_cap : n);
    }
    return n;
}

// A wave-uniform value, kept in scalar registers.
__device__ __forceinline__ float uniform_f(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ double uniform_d(double v)
{
    const long long b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Weight, arrival and their patch derivatives of one confocal pair.
struct PairS {
    float w;        // weight
    float w_a;      // w / a
    float dw_dz;    // dw / dpz
    float dwn;      // dw / dn = dwn * (dx, dy, pz)
    float du_dz;    // du / dpz (bins per metre)
    double u;       // arrival (bins), fp64
};

__device__ __forceinline__ PairS pair_smooth(float4 A, float4 B, float wx, float wy, double o, float gg,
                                             double inv, bool cosines, bool derivs)
{
    PairS r;
    const float dx = A.x - wx, dy = A.y - wy, pz = A.z;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, pz * pz));
    const float ri2 = __builtin_amdgcn_rcpf(r2);   // weights only: 1 ulp is ample
    const float ri4 = ri2 * ri2;
    // fp64 arrival from the same fp32 coordinates: (2 r + o) * inv, with
    // 2 r = 2 rf + (r^2 - rf^2) / rf, rf an fp32 square root: one Newton step,
    // the residual exact in fp64 (relative error ~1e-14, far below what the
    // Gaussian samples can see; r^2 > 0 since pz > 0)
    const double ex = (double)A.x - (double)wx, ey = (double)A.y - (double)wy, ez = (double)pz;
    const double r2d = (ex * ex + ey * ey) + ez * ez;
    const float rf = __builtin_amdgcn_sqrtf((float)r2d);
    const double rfd = (double)rf;
    const double rr = fma((double)__builtin_amdgcn_rcpf(rf), fma(-rfd, rfd, r2d), rfd + rfd);
    r.u = (rr + o) * inv;
    if (cosines) {
        // w = a gg pz^2 c^2 / r^8, c = -n.(p - w) clamped at 0
        const float c = fmaxf(-(B.x * dx + B.y * dy + B.z * pz), 0.f);
        const float k = gg * pz * pz * ri4 * ri4;
        r.w_a = k * c * c;
        r.w = A.w * r.w_a;
        if (derivs) {
            r.dw_dz = A.w * k * (2.f * c * c * __builtin_amdgcn_rcpf(pz) - 2.f * c * B.z) - r.w * 8.f * pz * ri2;
            r.dwn = -2.f * A.w * k * c;
        }
    } else {
        r.w_a = gg * ri4;
        r.w = A.w * r.w_a;
        if (derivs) {
            r.dw_dz = -r.w * 4.f * pz * ri2;
            r.dwn = 0.f;
        }
    }
    if (derivs) r.du_dz = (float)inv * 2.f * pz * __builtin_amdgcn_rsqf(r2);   // (gradients: 1 ulp is ample)
    return r;
}

}  // namespace

// ---------------------------------------------------------------------------
// Smooth forward.  RS > 0: the support radius is RS (= a.Rs), known at
// compile time, so a pair whose whole support lies inside the window takes a
// straight-line tap sequence with no bounds tests and the tap offsets folded
// into the LDS instructions; RS = 0, or a support that crosses the window's
// ends, takes the general loop.
template <int TX, int TY, bool COS, int RS>
__global__ void __launch_bounds__(kBlock) k_smooth(const SmoothArgs a)
{
    constexpr int NH = TX * TY;
    extern __shared__ __align__(16) unsigned char smem[];
    u64s* hist = reinterpret_cast<u64s*>(smem);
    double* so = reinterpret_cast<double*>(smem + (size_t)NH * a.stride * 8);
    float* sg = reinterpret_cast<float*>(so + NH);
    float* red = sg + NH;
    const int n_act = smooth_active(a);
    const int split = (int)(blockIdx.x % a.n_split);
    const int tile = (int)(blockIdx.x / a.n_split);
    const int tx0 = (tile / a.tiles_y) * TX, ty0 = (tile % a.tiles_y) * TY;
    const int chunk = (n_act + a.n_split - 1) / a.n_split;
    const int pb = min(n_act, split * chunk), pe = min(n_act, pb + chunk);

    for (int i = threadIdx.x; i < NH * a.stride; i += blockDim.x) hist[i] = 0ull;
    if (threadIdx.x < NH) {
        const int j = threadIdx.x;
        const int ix = min(tx0 + j / TY, a.rx.n - 1), iy = min(ty0 + j % TY, a.ry.n - 1);
        double off, g;
        device_leg(canon(a.rx, ix), canon(a.ry, iy), a.cx, a.cy, a.s, &off, &g);
        so[j] = off + off;
        sg[j] = (float)(g * g);
    }
    float wx[TX], wy[TY];
#pragma unroll
    for (int c = 0; c < TX; ++c) wx[c] = canon(a.rx, min(tx0 + c, a.rx.n - 1));
#pragma unroll
    for (int r = 0; r < TY; ++r) wy[r] = canon(a.ry, min(ty0 + r, a.ry.n - 1));
    // weight bound over the record summaries: a_max / r_min^4 (every cosine
    // factor and stand-off weight is at most 1) -> fixed-point scale
    float wb = 0.f;
    {
        const float x0 = fminf(wx[0], wx[TX - 1]), x1 = fmaxf(wx[0], wx[TX - 1]);
        const float y0 = fminf(wy[0], wy[TY - 1]), y1 = fmaxf(wy[0], wy[TY - 1]);
        for (int i = threadIdx.x; i < a.n_stats; i += blockDim.x) {
            const StatF c = load_stat(a.stats, i);
            if (c.count <= 0) continue;
            const float ddx = fmaxf(fmaxf(x0 - c.x1, c.x0 - x1), 0.f);
            const float ddy = fmaxf(fmaxf(y0 - c.y1, c.y0 - y1), 0.f);
            const float r2 = fmaf(ddx, ddx, fmaf(ddy, ddy, c.z0 * c.z0));
            wb = fmaxf(wb, c.amax / (r2 * r2));
        }
    }
    wb = wave_max_f(wb);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = wb;
    __syncthreads();
    float W = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) W = fmaxf(W, red[w]);
    const float s = W > 0.f ? 2147483648.0f / (W * a.norm) : 1.0f;   // increments <= 2^31
    const float sn = s * a.norm;
    const int T = a.T, Rs = a.Rs;
    const float inv_s2 = a.inv_s2, c1 = a.c1;

    for (int base = pb; base < pe; base += blockDim.x) {
        const int p = base + (int)threadIdx.x;
        if (p >= pe) continue;
        const float4 A = a.patches[2 * (size_t)p];
        const float4 B = a.patches[2 * (size_t)p + 1];
#pragma unroll
        for (int c = 0; c < TX; ++c) {
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                const int j = c * TY + r;
                if (tx0 + c >= a.rx.n || ty0 + r >= a.ry.n) continue;
                const PairS q = pair_smooth(A, B, wx[c], wy[r], so[j], sg[j], a.inv, COS, false);
                const double k0d = floor(q.u);
                if (q.w <= 0.f || k0d + Rs < 0.0 || k0d - Rs > (double)(T - 1)) continue;
                const int k0 = (int)k0d;
                const float f = (float)(q.u - k0d);
                const float x0 = 0.5f - f;
                const float amp = q.w * sn;
                u64s* row = hist + (size_t)j * a.stride;
                // centre and upward: e_{m+1} = e_m q_m, q_{m+1} = q_m c1
                float e = __expf(-0.5f * x0 * x0 * inv_s2);
                const float e0 = e;
                float qm = __expf(-(1.0f - f) * inv_s2);
                if (RS > 0 && k0 >= RS && k0 + RS < T) {
                    u64s* ctr = row + k0;
#pragma unroll
                    for (int m = 0; m <= RS; ++m) {
                        __hip_atomic_fetch_add(ctr + m, (u64s)(uint32_t)fmaf(amp, e, 0.5f), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                        e *= qm;
                        qm *= c1;
                    }
                    e = e0;
                    float dm = __expf(-f * inv_s2);
#pragma unroll
                    for (int m = 1; m <= RS; ++m) {
                        e *= dm;
                        dm *= c1;
                        __hip_atomic_fetch_add(ctr - m, (u64s)(uint32_t)fmaf(amp, e, 0.5f), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    continue;
                }
                for (int m = 0; m <= Rs; ++m) {
                    const int k = k0 + m;
                    if (k >= T) break;
                    if (k >= 0) {
                        const uint32_t inc = (uint32_t)fmaf(amp, e, 0.5f);
                        if (inc) __hip_atomic_fetch_add(row + k, (u64s)inc, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    e *= qm;
                    qm *= c1;
                }
                // downward: e_{m-1} = e_m d_m, d_{m-1} = d_m c1
                e = e0;
                float dm = __expf(-f * inv_s2);
                for (int m = -1; m >= -Rs; --m) {
                    e *= dm;
                    dm *= c1;
                    const int k = k0 + m;
                    if (k < 0) break;
                    if (k < T) {
                        const uint32_t inc = (uint32_t)fmaf(amp, e, 0.5f);
                        if (inc) __hip_atomic_fetch_add(row + k, (u64s)inc, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            }
        }
    }
    __syncthreads();
    const float inv_s = 1.0f / s;
    for (int i = threadIdx.x; i < NH * T; i += blockDim.x) {
        const int j = i / T, t = i - j * T;
        const int ix = tx0 + j / TY, iy = ty0 + j % TY;
        if (ix >= a.rx.n || iy >= a.ry.n) continue;
        const u64s x = hist[(size_t)j * a.stride + t];
        const float v = fmaf((float)(uint32_t)(x >> 32), 4294967296.0f, (float)(uint32_t)x) * inv_s;
        float* o = a.out + ((size_t)ix * a.ry.n + iy) * (size_t)T + t;
        if (a.atomic_out)
            unsafeAtomicAdd(o, v);
        else
            *o = v;
    }
}

// ---------------------------------------------------------------------------
// Smooth forward by moments.  With t = f - 1/2 the pair's sub-bin offset
// about the centre of its bin k0 = floor(u), its contribution w N(d + 1/2 - f)
// to bin k0 + d is the Taylor series sum_m (-t)^m / m! w N^(m)(d).  A pair
// therefore adds w (-t)^m to moment row m at bin k0 (one LDS add per moment
// instead of 2 Rs + 1), and the flush convolves each moment row with
// K_m(d) = N^(m)(d) / m! over |d| <= Rs, the same support as the direct sum.
// N^(m)(d) = N(d) (-1/sigma)^m He_m(d / sigma) (He: probabilists' Hermite
// polynomials).  With |t| <= 1/2, the series cut after m = 7 (radius 12,
// sigma > 11/6 bins) is within 7e-8 of the direct sum (relative L2 over the
// support, every t), and cut after m = 5 (radii 16 and 20, sigma > 2.5 bins)
// within 1.2e-6.  Moments are signed 64-bit fixed point (two's complement
// sums), increments |w (-t)^m| s <= 2^30.

// Taps K_m(d) = N^(m)(d) / m! = N(d) (-1/sigma)^m He_m(d / sigma) / m!,
// m < n_moments, |d| <= RS, into kt[m pitch + d + RS] (fp64, then fp32).
template <int RS>
__device__ __forceinline__ void moment_taps(const SmoothArgs& a, float* kt, int n_moments, int pitch)
{
    constexpr int ND = 2 * RS + 1;
    for (int i = threadIdx.x; i < n_moments * ND; i += blockDim.x) {
        const int m = i / ND, d = i % ND - RS;
        const double sig = (double)a.sigma, x = d / sig;
        double h0 = 1.0, h1 = x;   // He_0, He_1
        for (int n = 1; n < m; ++n) {
            const double h2 = x * h1 - n * h0;
            h0 = h1;
            h1 = h2;
        }
        const double he = m == 0 ? 1.0 : h1;
        double f = 1.0;
        for (int n = 2; n <= m; ++n) f *= n;
        kt[m * pitch + d + RS] = (float)((double)a.norm * exp(-0.5 * x * x) * he * pow(-1.0 / sig, m) / f);
    }
}

template <bool COS, int RS, bool PITCH>
__global__ void __launch_bounds__(kBlock) k_smooth_mom(const SmoothArgs a)
{
    constexpr int NP = smooth_mom_shape(RS).points, NM = smooth_mom_shape(RS).moments, NR = NP * NM, ND = 2 * RS + 1;
    constexpr int NDP = (ND + 3) & ~3;             // tap row pitch: rows start 16-byte aligned
    extern __shared__ __align__(16) unsigned char smem[];
    u64s* hist = reinterpret_cast<u64s*>(smem);   // row (point c, moment m) = c NM + m; bin k0 at k0 + RS
    // (PITCH: the rows at the compile-time pitch, which the host passes as the stride)
    const int stride = PITCH ? smooth_mom_pitch(RS) : a.stride;
    double* so = reinterpret_cast<double*>(smem + (size_t)NR * stride * 8);
    float* sg = reinterpret_cast<float*>(so + NP);
    float* red = sg + NP;
    constexpr int KT_OFF = (NP * 12 + 64 * 4 + 15) & ~15;   // past so, sg and red
    static_assert(KT_OFF + NM * NDP * 4 <= 2048, "the taps must fit the 2 KiB past the moment rows");
    float* kt = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(so) + KT_OFF);   // [NM][NDP], 16-byte aligned
    const int n_act = smooth_active(a);
    const int split = (int)(blockIdx.x % a.n_split);
    const int tile = (int)(blockIdx.x / a.n_split);
    const int tx0 = (tile / a.tiles_y) * NP, ty0 = tile % a.tiles_y;
    const int chunk = (n_act + a.n_split - 1) / a.n_split;
    const int pb = min(n_act, split * chunk), pe = min(n_act, pb + chunk);
    const int T = a.T;

    for (int i = threadIdx.x; i < NR * stride; i += kBlock) hist[i] = 0ull;
    if (threadIdx.x < NP) {
        const int c = threadIdx.x;
        double off, g;
        device_leg(canon(a.rx, min(tx0 + c, a.rx.n - 1)), canon(a.ry, ty0), a.cx, a.cy, a.s, &off, &g);
        so[c] = off + off;
        sg[c] = (float)(g * g);
    }
    moment_taps<RS>(a, kt, NM, NDP);
    float wx[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) wx[c] = canon(a.rx, min(tx0 + c, a.rx.n - 1));
    const float wy = canon(a.ry, ty0);
    // weight bound over the record summaries: a_max / r_min^4 -> scale
    float wb = 0.f;
    {
        const float x0 = fminf(wx[0], wx[NP - 1]), x1 = fmaxf(wx[0], wx[NP - 1]);
        for (int i = threadIdx.x; i < a.n_stats; i += kBlock) {
            const StatF c = load_stat(a.stats, i);
            if (c.count <= 0) continue;
            const float ddx = fmaxf(fmaxf(x0 - c.x1, c.x0 - x1), 0.f);
            const float ddy = fmaxf(fmaxf(wy - c.y1, c.y0 - wy), 0.f);
            const float r2 = fmaf(ddx, ddx, fmaf(ddy, ddy, c.z0 * c.z0));
            wb = fmaxf(wb, c.amax / (r2 * r2));
        }
    }
    wb = wave_max_f(wb);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = wb;
    __syncthreads();
    float W = 0.f;
    for (int w = 0; w < kBlock / 64; ++w) W = fmaxf(W, red[w]);
    const float s = W > 0.f ? 1073741824.0f / W : 1.0f;   // |increments| <= 2^30
    double soc[NP];
    float sgc[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        soc[c] = so[c];
        sgc[c] = sg[c];
    }

    for (int base = pb; base < pe; base += kBlock) {
        const int p = base + (int)threadIdx.x;
        if (p >= pe) continue;
        const float4 A = a.patches[2 * (size_t)p];
        const float4 B = a.patches[2 * (size_t)p + 1];
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            if (tx0 + c >= a.rx.n) continue;
            const PairS q = pair_smooth(A, B, wx[c], wy, soc[c], sgc[c], a.inv, COS, false);
            const double k0d = floor(q.u);
            const int k0 = (int)k0d;   // u >= 0; a saturated conversion fails the test below
            // the support [k0 - RS, k0 + RS] meets the bins [0, T)
            if (q.w <= 0.f || (uint32_t)k0 + (uint32_t)RS > (uint32_t)(T - 1 + 2 * RS)) continue;
            const float mt = 0.5f - (float)(q.u - k0d);   // -t
            float v = q.w * s;
            u64s* r0 = hist + (size_t)(c * NM) * stride + (k0 + RS);
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                // even moments are non-negative (w > 0, (-t)^m >= 0): no sign extension
                const int iv = __float2int_rn(v);
                const u64s inc = (m & 1) ? (u64s)(long long)iv : (u64s)(uint32_t)iv;
                __hip_atomic_fetch_add(r0 + (size_t)m * stride, inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                v *= mt;
            }
        }
    }
    __syncthreads();
    // moment rows -> float, in place (row r keeps its byte offset; values
    // pass through registers so that no thread overwrites what another reads)
    const int L = T + 2 * RS;
    constexpr int kMaxPer = 24;
    float vals[kMaxPer];
    const int n_vals = NR * L;
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) {
        const int i = (int)threadIdx.x + k * kBlock;
        vals[k] = 0.f;
        if (i < n_vals) {
            const int r = i / L, b = i - r * L;
            const u64s x = hist[(size_t)r * stride + b];
            vals[k] = fmaf((float)(int32_t)(uint32_t)(x >> 32), 4294967296.0f, (float)(uint32_t)x);
        }
    }
    __syncthreads();
    float* F = reinterpret_cast<float*>(smem);     // row r at float offset 2 r stride
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) {
        const int i = (int)threadIdx.x + k * kBlock;
        if (i < n_vals) {
            const int r = i / L, b = i - r * L;
            F[(size_t)r * 2 * stride + b] = vals[k];
        }
    }
    __syncthreads();
    // Each thread takes V consecutive bins of one scan point and holds, per
    // moment, their window of V + 2 RS samples and the moment's taps in
    // registers (16-byte LDS reads; row starts and k0 are multiples of four
    // floats).  A bin's sum runs over m, then d.  Window samples past the
    // row's T + 2 RS values reach only bins >= T, which are not written.
    const float inv_sc = 1.0f / s;
    constexpr int V = 4, NW = (V + 2 * RS + 3) / 4;
    const int nseg = (T + V - 1) / V;
    const bool vec_out = !a.atomic_out && (T & 3) == 0 && ((uintptr_t)a.out & 15) == 0;
    for (int o = threadIdx.x; o < NP * nseg; o += kBlock) {
        const int c = o / nseg, k0 = (o - c * nseg) * V;
        if (tx0 + c >= a.rx.n) continue;
        float acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = 0.f;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            // bin k0 + v, offset d = dd - RS, reads F at k0 + v + 2 RS - dd
            const float4* f4 = reinterpret_cast<const float4*>(F + (size_t)(c * NM + m) * 2 * stride + k0);
            const float4* t4 = reinterpret_cast<const float4*>(kt + m * NDP);
            float w[4 * NW], t[NDP];
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const float4 x = f4[q];
                w[4 * q] = x.x;
                w[4 * q + 1] = x.y;
                w[4 * q + 2] = x.z;
                w[4 * q + 3] = x.w;
            }
#pragma unroll
            for (int q = 0; q < NDP / 4; ++q) {
                const float4 x = t4[q];
                t[4 * q] = x.x;
                t[4 * q + 1] = x.y;
                t[4 * q + 2] = x.z;
                t[4 * q + 3] = x.w;
            }
#pragma unroll
            for (int dd = 0; dd < ND; ++dd) {
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] = fmaf(w[v + 2 * RS - dd], t[dd], acc[v]);
            }
        }
        float* dst = a.out + ((size_t)(tx0 + c) * a.ry.n + ty0) * (size_t)T + k0;
        if (vec_out && k0 + V <= T) {
            *reinterpret_cast<float4*>(dst) = make_float4(acc[0] * inv_sc, acc[1] * inv_sc, acc[2] * inv_sc, acc[3] * inv_sc);
            continue;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (k0 + v >= T) break;
            if (a.atomic_out)
                unsafeAtomicAdd(dst + v, acc[v] * inv_sc);
            else
                dst[v] = acc[v] * inv_sc;
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint gather.  RS as in k_smooth: a support inside the window takes a
// straight-line tap sequence (G1 = x0 G0 + sum g N(x) m there).
template <bool COS, int RS>
__global__ void __launch_bounds__(kBlock) k_adjoint(const SmoothArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int T = a.T, Rs = a.Rs, NR = a.rows;
    float* rowbuf = reinterpret_cast<float*>(smem);                        // [NR][T]
    double* so = reinterpret_cast<double*>(smem + (((size_t)NR * T * 4 + 15) & ~(size_t)15));
    float* swx = reinterpret_cast<float*>(so + NR);
    float* swy = swx + NR;
    float* sg = swy + NR;
    const int n_act = smooth_active(a);
    const int p = (int)blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
    const int split = (int)blockIdx.y;
    const int S = a.rx.n * a.ry.n;
    const int per = (S + a.n_split - 1) / a.n_split;
    const int s0 = min(S, split * per), s1 = min(S, s0 + per);
    const bool live = p < n_act;
    float4 A = make_float4(0.f, 0.f, 1.f, 0.f), B = make_float4(0.f, 0.f, -1.f, 0.f);
    if (live) {
        A = a.patches[2 * (size_t)p];
        B = a.patches[2 * (size_t)p + 1];
    }
    double gz = 0.0, ga = 0.0, gnx = 0.0, gny = 0.0, gnz = 0.0;
    const float inv_s2 = a.inv_s2, c1 = a.c1;

    for (int j0 = s0; j0 < s1; j0 += NR) {
        const int nr = min(NR, s1 - j0);
        __syncthreads();
        // stage rows [j0, j0 + nr) of the upstream gradient (float4 when aligned)
        if ((T & 3) == 0) {
            const float4* src = reinterpret_cast<const float4*>(a.grad_out + (size_t)j0 * T);
            float4* dst = reinterpret_cast<float4*>(rowbuf);
            for (int i = threadIdx.x; i < nr * (T >> 2); i += blockDim.x) dst[i] = src[i];
        } else {
            const float* src = a.grad_out + (size_t)j0 * T;
            for (int i = threadIdx.x; i < nr * T; i += blockDim.x) rowbuf[i] = src[i];
        }
        if (threadIdx.x < nr) {
            const int h = j0 + threadIdx.x;
            const float wx = canon(a.rx, h / a.ry.n), wy = canon(a.ry, h % a.ry.n);
            double off, g;
            device_leg(wx, wy, a.cx, a.cy, a.s, &off, &g);
            so[threadIdx.x] = off + off;
            swx[threadIdx.x] = wx;
            swy[threadIdx.x] = wy;
            sg[threadIdx.x] = (float)(g * g);
        }
        __syncthreads();
        if (!live) continue;
        for (int jj = 0; jj < nr; ++jj) {
            const PairS q = pair_smooth(A, B, swx[jj], swy[jj], so[jj], sg[jj], a.inv, COS, true);
            const double k0d = floor(q.u);
            if (k0d + Rs < 0.0 || k0d - Rs > (double)(T - 1)) continue;
            const int k0 = (int)k0d;
            const float f = (float)(q.u - k0d);
            const float* g = rowbuf + (size_t)jj * T;
            // G0 = sum g N(x), G1 = sum g x N(x), x = m + 1/2 - f (N without
            // its normalisation; applied below)
            float G0 = 0.f, G1 = 0.f;
            const float x0 = 0.5f - f;
            float e = __expf(-0.5f * x0 * x0 * inv_s2);
            const float e0 = e;
            float qm = __expf(-(1.0f - f) * inv_s2);
            if (RS > 0 && k0 >= RS && k0 + RS < T) {
                const float* gc = g + k0;
                float G1m = 0.f;
#pragma unroll
                for (int m = 0; m <= RS; ++m) {
                    const float gv = gc[m] * e;
                    G0 += gv;
                    G1m = fmaf(gv, (float)m, G1m);
                    e *= qm;
                    qm *= c1;
                }
                e = e0;
                float dm = __expf(-f * inv_s2);
#pragma unroll
                for (int m = 1; m <= RS; ++m) {
                    e *= dm;
                    dm *= c1;
                    const float gv = gc[-m] * e;
                    G0 += gv;
                    G1m = fmaf(gv, -(float)m, G1m);
                }
                G1 = fmaf(x0, G0, G1m);
            } else {
                for (int m = 0; m <= Rs; ++m) {
                    const int k = k0 + m;
                    if (k >= T) break;
                    if (k >= 0) {
                        const float gv = g[k] * e;
                        G0 += gv;
                        G1 = fmaf(gv, x0 + (float)m, G1);
                    }
                    e *= qm;
                    qm *= c1;
                }
                e = e0;
                float dm = __expf(-f * inv_s2);
                for (int m = -1; m >= -Rs; --m) {
                    e *= dm;
                    dm *= c1;
                    const int k = k0 + m;
                    if (k < 0) break;
                    if (k < T) {
                        const float gv = g[k] * e;
                        G0 += gv;
                        G1 = fmaf(gv, x0 + (float)m, G1);
                    }
                }
            }
            G0 *= a.norm;
            G1 *= a.norm * inv_s2;
            // dL/dw = G0, dL/du = w G1
            const float dz = fmaf(G0, q.dw_dz, q.w * G1 * q.du_dz);
            gz += (double)dz;
            ga += (double)(G0 * q.w_a);
            if (COS) {
                const float gn = G0 * q.dwn;
                gnx += (double)(gn * (A.x - swx[jj]));
                gny += (double)(gn * (A.y - swy[jj]));
                gnz += (double)(gn * A.z);
            }
        }
    }
    if (live) {
        double* o = a.partial + ((size_t)split * a.n_cap + p) * kAdjStride;
        o[0] = gz;
        o[1] = ga;
        o[2] = gnx;
        o[3] = gny;
        o[4] = gnz;
    }
}

// ---------------------------------------------------------------------------
// Adjoint by moments.  For a pair with bin k0 and t = f - 1/2 (as in
// k_smooth_mom), G0 = sum_k g[k] N(x) and G1 = sum_k g[k] (x / sigma^2) N(x)
// = -sum_k g[k] N'(x) over the support are the series
//     G0 = sum_m (-t)^m C_m[k0],   G1 = -sum_m (-t)^m (m + 1) C_{m+1}[k0]
// (m = 0 .. n - 2, n = adj_moments(Rs)) of the correlations
// C_m[k0] = sum_{|d|<=Rs} g[k0 + d] K_m(d), K_m = N^(m) / m!.  k_adj_moments
// computes C_0 .. C_{n-1} once per scan point (bins k0 = -Rs .. T + Rs - 1,
// stored at k0 + Rs); k_adjoint_mom then needs n LDS reads and two Horner
// sums per pair instead of 2 Rs + 1 taps.
template <int RS>
__global__ void __launch_bounds__(256) k_adj_taps(const SmoothArgs a)
{
    moment_taps<RS>(a, a.mtaps, adj_moments(RS), 2 * RS + 1);
}

// Correlation rows.  A thread produces V = 4 consecutive bins j0 .. j0 + 3
// (bins k0 = j - RS of a row of L = T + 2 RS) of every row of one scan point,
// from a register window of that point's upstream gradient g[j0 - 2 RS ..
// j0 + 3] (zero outside 0 .. T - 1).  Threads map flat onto (scan
// point, group of 4 bins), so every lane of every wavefront has work and no
// row is staged anywhere first.  The kernels have the parity of their order,
// K_m(-d) = (-1)^m K_m(d) exactly (He_m has the parity of m, and every
// operation of moment_taps is symmetric in the sign of d), so
//     C_m[k0] = K_m(0) g[k0] + sum_{d=1..RS} K_m(d) (g[k0 + d] + (-1)^m g[k0 - d]):
// a bin's mirrored sums serve every even row and its mirrored differences
// every odd row, 2 RS adds and about RS + 1 fmas per row where the full
// support takes 2 RS + 1 fmas.  The kernels are scalar reads (the same for
// every lane, written by an earlier launch), fma operands in scalar
// registers, one row at a time.  ALIGNED (T a multiple of 4, so L is too,
// and both arrays 16-byte aligned): the window arrives as 16-byte reads, each
// wholly inside the row or wholly in the zero padding, and each row's four
// bins go out as one 16-byte store.
template <int RS, bool ALIGNED>
__global__ void __launch_bounds__(256) k_adj_moments(const SmoothArgs a)
{
    constexpr int V = 4, NM = adj_moments(RS), ND = 2 * RS + 1, W = V + 2 * RS;
    static_assert(W % 4 == 0, "the window is whole 16-byte pieces");
    const int T = a.T, L = a.mlen, Q = (L + V - 1) / V;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)(a.rx.n * a.ry.n) * Q) return;
    const int s = (int)(t / Q), j0 = (int)(t % Q) * V;
    const float* g = a.grad_out + (size_t)s * T;
    const int kw = j0 - 2 * RS;   // gradient index of window word 0
    float w[W];
    if constexpr (ALIGNED) {
#pragma unroll
        for (int q = 0; q < W / 4; ++q) {
            const int k = kw + 4 * q;
            const float4 v = (k >= 0 && k < T) ? *reinterpret_cast<const float4*>(g + k) : make_float4(0.f, 0.f, 0.f, 0.f);
            w[4 * q] = v.x;
            w[4 * q + 1] = v.y;
            w[4 * q + 2] = v.z;
            w[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < W; ++q) w[q] = (kw + q >= 0 && kw + q < T) ? g[kw + q] : 0.f;
    }
    const __attribute__((address_space(4))) float* kc = (const __attribute__((address_space(4))) float*)a.mtaps;
    float* out = a.moments + (size_t)s * NM * L + j0;
    // bin j0 + v: g[k0 + d] = w[v + RS + d] (k0 = j0 + v - RS)
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        // mirrored sums (even rows) or differences (odd rows) of every bin
        float x[V][RS];
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int d = 1; d <= RS; ++d)
                x[v][d - 1] = par == 0 ? w[v + RS + d] + w[v + RS - d] : w[v + RS + d] - w[v + RS - d];
        // one row at a time: its kernel in scalar registers
#pragma unroll 1
        for (int m = par; m < NM; m += 2) {
            const int c = m * ND + RS;   // K_m(0)
            float acc[V];
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = par == 0 ? w[v + RS] * kc[c] : 0.f;
#pragma unroll
            for (int d = 1; d <= RS; ++d) {
                const float k = kc[c + d];
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] = fmaf(x[v][d - 1], k, acc[v]);
            }
            if constexpr (ALIGNED) {
                // j0 and L are multiples of 4, so j0 + 3 < L
                *reinterpret_cast<float4*>(out + (size_t)m * L) = make_float4(acc[0], acc[1], acc[2], acc[3]);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (j0 + v < L) out[(size_t)m * L + v] = acc[v];
            }
        }
    }
}

template <bool COS, int RS, bool DB>
__global__ void __launch_bounds__(kBlock) k_adjoint_mom(const SmoothArgs a)
{
    constexpr int NM = adj_moments(RS), MT = NM - 2, PPT = kAdjPatches, NB = DB ? 2 : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int T = a.T, L = a.mlen, NR = a.rows;
    // NB buffers of NR scan points' rows [NR][NM][L], then per buffer the
    // points' offsets (fp64), positions and gains
    const size_t buf_bytes = ((size_t)NR * NM * L * 4 + 15) & ~(size_t)15;
    double* so = reinterpret_cast<double*>(smem + NB * buf_bytes);
    float* swx = reinterpret_cast<float*>(so + NB * NR);
    float* swy = swx + NB * NR;
    float* sg = swy + NB * NR;
    const int n_act = smooth_active(a);
    const int split = (int)blockIdx.y;
    const int S = a.rx.n * a.ry.n;
    const int per = (S + a.n_split - 1) / a.n_split;
    const int s0 = min(S, split * per), s1 = min(S, s0 + per);
    float4 A[PPT], B[PPT];
    bool live[PPT];
    double gz[PPT], ga[PPT], gnx[PPT], gny[PPT], gnz[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int p = ((int)blockIdx.x * PPT + i) * kBlock + (int)threadIdx.x;
        live[i] = p < n_act;
        A[i] = make_float4(0.f, 0.f, 1.f, 0.f);
        B[i] = make_float4(0.f, 0.f, -1.f, 0.f);
        if (live[i]) {
            A[i] = a.patches[2 * (size_t)p];
            B[i] = a.patches[2 * (size_t)p + 1];
        }
        gz[i] = ga[i] = gnx[i] = gny[i] = gnz[i] = 0.0;
    }
    // the constants of scan points [j, j + nr) into buffer b
    auto stage_consts = [&](int b, int j, int nr) {
        if ((int)threadIdx.x < nr) {
            const int h = j + (int)threadIdx.x;
            const float wx = canon(a.rx, h / a.ry.n), wy = canon(a.ry, h % a.ry.n);
            double off, g;
            device_leg(wx, wy, a.cx, a.cy, a.s, &off, &g);
            so[b * NR + threadIdx.x] = off + off;
            swx[b * NR + threadIdx.x] = wx;
            swy[b * NR + threadIdx.x] = wy;
            sg[b * NR + threadIdx.x] = (float)(g * g);
        }
    };
    // DB: the rows of scan points [j, j + nr) into buffer b by global->LDS
    // loads, 16 bytes per lane at the wavefront's LDS base + 16 lane; they
    // land while the other buffer is in use.  Wavefront w moves the pieces of
    // 64 float4 numbered w, w + 16, ... (L is a multiple of 4: whole pieces
    // of the contiguous rows, the last one masked past the end)
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = (int)threadIdx.x & 63;
    auto stage_rows_db = [&](int b, int j, int nr) {
        const float4* s4 = reinterpret_cast<const float4*>(a.moments + (size_t)j * NM * L);
        float* dst = reinterpret_cast<float*>(smem + b * buf_bytes);
        const int n4 = nr * NM * (L >> 2);
        for (int pc = wave; pc * 64 < n4; pc += kBlock / 64) {
            const int i = pc * 64 + lane;
            if (i < n4)
                __builtin_amdgcn_global_load_lds((const void*)(s4 + i),
                                                 (__attribute__((address_space(3))) void*)(dst + (size_t)pc * 256), 16,
                                                 0, 0);
        }
    };
    const int nst = s1 > s0 ? (s1 - s0 + NR - 1) / NR : 0;
    if (DB && nst > 0) {
        stage_rows_db(0, s0, min(NR, s1 - s0));
        stage_consts(0, s0, min(NR, s1 - s0));
    }
    for (int st = 0; st < nst; ++st) {
        const int j0 = s0 + st * NR;
        const int nr = min(NR, s1 - j0);
        const int b = DB ? (st & 1) : 0;
        if (DB) {
            // this wavefront's loads into buffer b have landed; past the
            // barrier every wavefront's have, and buffer b ^ 1 (the stage
            // before) is no longer read: the next stage goes there
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (st + 1 < nst) {
                stage_rows_db(b ^ 1, j0 + NR, min(NR, s1 - j0 - NR));
                stage_consts(b ^ 1, j0 + NR, min(NR, s1 - j0 - NR));
            }
        } else {
            __syncthreads();
            // stage the correlation rows of scan points [j0, j0 + nr): contiguous
            float* rowbuf = reinterpret_cast<float*>(smem);
            const float* src = a.moments + (size_t)j0 * NM * L;
            if ((L & 3) == 0) {
                // four loads in flight per thread before their LDS stores (a load
                // past the end rereads the last element; its store is skipped)
                const float4* s4 = reinterpret_cast<const float4*>(src);
                float4* d4 = reinterpret_cast<float4*>(rowbuf);
                const int n4 = nr * NM * (L >> 2);
                for (int i0 = threadIdx.x; i0 < n4; i0 += 4 * kBlock) {
                    const int last = n4 - 1;
                    const float4 v0 = s4[min(i0, last)];
                    const float4 v1 = s4[min(i0 + kBlock, last)];
                    const float4 v2 = s4[min(i0 + 2 * kBlock, last)];
                    const float4 v3 = s4[min(i0 + 3 * kBlock, last)];
                    __builtin_amdgcn_sched_barrier(0);
                    d4[i0] = v0;
                    if (i0 + kBlock < n4) d4[i0 + kBlock] = v1;
                    if (i0 + 2 * kBlock < n4) d4[i0 + 2 * kBlock] = v2;
                    if (i0 + 3 * kBlock < n4) d4[i0 + 3 * kBlock] = v3;
                }
            } else {
                for (int i = threadIdx.x; i < nr * NM * L; i += kBlock) rowbuf[i] = src[i];
            }
            stage_consts(0, j0, nr);
            __syncthreads();
        }
        const float* rowbuf = reinterpret_cast<const float*>(smem + b * buf_bytes);
        for (int jj = 0; jj < nr; ++jj) {
            // the scan point's constants, read once for the patches below
            const float wxj = uniform_f(swx[b * NR + jj]), wyj = uniform_f(swy[b * NR + jj]),
                        gj = uniform_f(sg[b * NR + jj]);
            const double oj = uniform_d(so[b * NR + jj]);
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                if (!live[i]) continue;
                const PairS q = pair_smooth(A[i], B[i], wxj, wyj, oj, gj, a.inv, COS, true);
                const double k0d = floor(q.u);
                const int k0 = (int)k0d;   // u >= 0; a saturated conversion fails the test below
                if ((uint32_t)k0 + (uint32_t)RS > (uint32_t)(T - 1 + 2 * RS)) continue;
                const float mt = 0.5f - (float)(q.u - k0d);   // -t
                const float* c = rowbuf + (size_t)jj * NM * L + (k0 + RS);
                float G0 = c[MT * L], G1 = (float)(MT + 1) * c[(MT + 1) * L];
#pragma unroll
                for (int m = MT - 1; m >= 0; --m) {
                    G0 = fmaf(G0, mt, c[m * L]);
                    G1 = fmaf(G1, mt, (float)(m + 1) * c[(m + 1) * L]);
                }
                G1 = -G1;
                // dL/dw = G0, dL/du = w G1
                const float dz = fmaf(G0, q.dw_dz, q.w * G1 * q.du_dz);
                gz[i] += (double)dz;
                ga[i] += (double)(G0 * q.w_a);
                if (COS) {
                    const float gn = G0 * q.dwn;
                    gnx[i] += (double)(gn * (A[i].x - wxj));
                    gny[i] += (double)(gn * (A[i].y - wyj));
                    gnz[i] += (double)(gn * A[i].z);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int p = ((int)blockIdx.x * PPT + i) * kBlock + (int)threadIdx.x;
        if (!live[i]) continue;
        double* o = a.partial + ((size_t)split * a.n_cap + p) * kAdjStride;
        o[0] = gz[i];
        o[1] = ga[i];
        o[2] = gnx[i];
        o[3] = gny[i];
        o[4] = gnz[i];
    }
}

// Sum the per-split partials in split order -> grad_rec [n_cap][8] floats
// {0, 0, dL/dpz, dL/da, dL/dn_x, dL/dn_y, dL/dn_z, 0}; zeros past n_active.
__global__ void __launch_bounds__(256) k_adjoint_reduce(const SmoothArgs a, float* grad_rec)
{
    // one thread per output word of a record: words 2 .. 6 sum their field's
    // partials over the splits in split order (32 splits' values read before
    // any is added, so that their latencies overlap), words 0, 1 and 7 are 0
    const int n_act = smooth_active(a);
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t p = t >> 3;
    const int k = (int)(t & 7) - 2;
    if (p >= a.n_cap) return;
    double g = 0.0;
    if (p < n_act && k >= 0 && k < kAdjStride) {
        constexpr int kB = 32;
        const size_t step = (size_t)a.n_cap * kAdjStride;
        const double* q = a.partial + (size_t)p * kAdjStride + k;
        int sp = 0;
        for (; sp + kB <= a.n_split; sp += kB) {
            double v[kB];
#pragma unroll
            for (int i = 0; i < kB; ++i) v[i] = q[(size_t)(sp + i) * step];
#pragma unroll
            for (int i = 0; i < kB; ++i) g += v[i];
        }
        for (; sp < a.n_split; ++sp) g += q[(size_t)sp * step];
    }
    grad_rec[t] = (float)g;
}

// ---------------------------------------------------------------------------
// Record gradients -> maps.
__device__ __forceinline__ float deriv_f(const float* d, int n, int i, int64_t stride, float h)
{
    if (n < 2) return 0.f;
    if (i == 0) return (d[stride] - d[0]) / h;
    if (i == n - 1) return (d[0] - d[-stride]) / h;
    return (d[stride] - d[-stride]) / (2.f * h);
}

__global__ void k_grad_zero(const GradMapArgs g, int64_t npx)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += stride) {
        g.scratch[i] = 0.f;
        g.scratch[npx + i] = 0.f;
        g.scratch[2 * npx + i] = 0.f;
        if (g.grad_albedo) g.grad_albedo[i] = 0.f;
    }
}

// Per record: dL/dpz as is; dL/dD_x, dL/dD_y through n = (D_x, D_y, -1)/len
// and a = rho dx dy len (cosines); dL/drho = dL/da * area.  Written to the
// record's own pixel, so no two records collide.
__global__ void __launch_bounds__(256) k_grad_scatter(const GradMapArgs g, int64_t npx)
{
    int n = g.n_cap;
    if (g.n_active) {
        n = *g.n_active;
        n = n < 0 ? 0 : (n > g.n_cap ? g.n_cap : n);
    }
    const int p = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (p >= n) return;
    const int idx = __float_as_int(g.patches[2 * (size_t)p + 1].w);
    const int ix = idx / g.ay.n, iy = idx % g.ay.n;
    const float* D = g.depth + idx;
    const float gx = deriv_f(D, g.ax.n, ix, g.ay.n, g.hx);
    const float gy = deriv_f(D, g.ay.n, iy, 1, g.hy);
    const float len = sqrtf(1.f + gx * gx + gy * gy);
    const float rho = g.albedo ? g.albedo[idx] : 0.5f;
    const float* q = g.grad_rec + (size_t)p * 8;
    const float dpz = q[2], da = q[3], dnx = q[4], dny = q[5], dnz = q[6];
    const float area = g.hx * g.hy * (g.cosines ? len : 1.f);
    if (g.grad_albedo) g.grad_albedo[idx] = da * area;
    g.scratch[idx] = dpz;
    if (g.cosines) {
        const float il = 1.f / len;
        const float il3 = il * il * il;
        const float dot = dnx * gx + dny * gy - dnz;
        const float darea = da * rho * g.hx * g.hy * il;
        g.scratch[npx + idx] = dnx * il - dot * gx * il3 + darea * gx;
        g.scratch[2 * npx + idx] = dny * il - dot * gy * il3 + darea * gy;
    }
}

// Coefficient of D[i] in the derivative at sample i' (|i - i'| <= 1) of an
// axis of n samples with spacing h (central inside, one-sided at borders).
__device__ __forceinline__ float stencil(int n, int ip, int i, float h)
{
    if (n < 2) return 0.f;
    if (ip == 0) return (i == 1 ? 1.f : (i == 0 ? -1.f : 0.f)) / h;
    if (ip == n - 1) return (i == n - 1 ? 1.f : (i == n - 2 ? -1.f : 0.f)) / h;
    return (i == ip + 1 ? 1.f : (i == ip - 1 ? -1.f : 0.f)) / (2.f * h);
}

__global__ void __launch_bounds__(256) k_grad_gather(const GradMapArgs g, int64_t npx)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= npx) return;
    const int nx = g.ax.n, ny = g.ay.n;
    const int ix = (int)(idx / ny), iy = (int)(idx % ny);
    float v = g.scratch[idx];
    const float* sx = g.scratch + npx;
    const float* sy = g.scratch + 2 * npx;
    for (int d = -1; d <= 1; ++d) {
        const int jx = ix + d;
        if (jx >= 0 && jx < nx) v = fmaf(sx[(int64_t)jx * ny + iy], stencil(nx, jx, ix, g.hx), v);
        const int jy = iy + d;
        if (jy >= 0 && jy < ny) v = fmaf(sy[(int64_t)ix * ny + jy], stencil(ny, jy, iy, g.hy), v);
    }
    g.grad_depth[idx] = v;
}

// ---------------------------------------------------------------------------
// Launchers.
template <int TX, int TY, int RS>
static hipError_t launch_smooth_rs(const SmoothArgs& a, int64_t n_blocks, size_t lds, hipStream_t st)
{
    const void* k = a.cosines ? (const void*)k_smooth<TX, TY, true, RS> : (const void*)k_smooth<TX, TY, false, RS>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (a.cosines)
        hipLaunchKernelGGL((k_smooth<TX, TY, true, RS>), dim3((unsigned)n_blocks), dim3(kBlock), lds, st, a);
    else
        hipLaunchKernelGGL((k_smooth<TX, TY, false, RS>), dim3((unsigned)n_blocks), dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

// Support radii with a straight-line tap sequence: ceil(6 sigma) for the
// jitter widths of the paper's configurations (FWHM / bin = 70/16, 50/8,
// 30/4 ps give 12, 16, 20); any other radius runs the general loop.
template <int TX, int TY>
static hipError_t launch_smooth_shape(const SmoothArgs& a, int64_t n_blocks, size_t lds, hipStream_t st)
{
    if (a.Rs == 12) return launch_smooth_rs<TX, TY, 12>(a, n_blocks, lds, st);
    if (a.Rs == 16) return launch_smooth_rs<TX, TY, 16>(a, n_blocks, lds, st);
    if (a.Rs == 20) return launch_smooth_rs<TX, TY, 20>(a, n_blocks, lds, st);
    return launch_smooth_rs<TX, TY, 0>(a, n_blocks, lds, st);
}

hipError_t launch_smooth(const SmoothArgs& a, int tx, int ty, int64_t n_blocks, size_t lds, hipStream_t st)
{
    if (n_blocks <= 0) return hipSuccess;
    if (n_blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (tx == 4 && ty == 4) return launch_smooth_shape<4, 4>(a, n_blocks, lds, st);
    if (tx == 4 && ty == 2) return launch_smooth_shape<4, 2>(a, n_blocks, lds, st);
    if (tx == 2 && ty == 2) return launch_smooth_shape<2, 2>(a, n_blocks, lds, st);
    if (tx == 2 && ty == 1) return launch_smooth_shape<2, 1>(a, n_blocks, lds, st);
    if (tx == 1 && ty == 1) return launch_smooth_shape<1, 1>(a, n_blocks, lds, st);
    return hipErrorInvalidValue;
}

bool smooth_moments_radius(int rs) { return rs == 12 || rs == 16 || rs == 20; }

template <int RS, bool PITCH>
static hipError_t launch_smooth_mom_pitch(const SmoothArgs& a, int64_t n_blocks, size_t lds, hipStream_t st)
{
    const void* k = a.cosines ? (const void*)k_smooth_mom<true, RS, PITCH> : (const void*)k_smooth_mom<false, RS, PITCH>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (a.cosines)
        hipLaunchKernelGGL((k_smooth_mom<true, RS, PITCH>), dim3((unsigned)n_blocks), dim3(kBlock), lds, st, a);
    else
        hipLaunchKernelGGL((k_smooth_mom<false, RS, PITCH>), dim3((unsigned)n_blocks), dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

template <int RS>
static hipError_t launch_smooth_mom_rs(const SmoothArgs& a, int64_t n_blocks, size_t lds, hipStream_t st)
{
    return a.stride == smooth_mom_pitch(RS) ? launch_smooth_mom_pitch<RS, true>(a, n_blocks, lds, st)
                                            : launch_smooth_mom_pitch<RS, false>(a, n_blocks, lds, st);
}

hipError_t launch_smooth_moments(const SmoothArgs& a, int64_t n_blocks, size_t lds, hipStream_t st)
{
    if (n_blocks <= 0) return hipSuccess;
    if (n_blocks > 0x7fffffff) return hipErrorInvalidValue;
    // the flush keeps at most 24 values per thread in registers
    const SmoothMomShape sh = smooth_mom_shape(a.Rs);
    if ((int64_t)sh.points * sh.moments * (a.T + 2 * a.Rs) > 24 * (int64_t)kBlock) return hipErrorInvalidValue;
    if (a.stride < a.T + 2 * a.Rs) return hipErrorInvalidValue;
    // moment rows, then 2 KiB for the scan points' offsets, the reduction and the taps
    if (lds < (size_t)sh.points * sh.moments * a.stride * 8 + 2048) return hipErrorInvalidValue;
    if (a.Rs == 12) return launch_smooth_mom_rs<12>(a, n_blocks, lds, st);
    if (a.Rs == 16) return launch_smooth_mom_rs<16>(a, n_blocks, lds, st);
    if (a.Rs == 20) return launch_smooth_mom_rs<20>(a, n_blocks, lds, st);
    return hipErrorInvalidValue;
}

template <int RS>
static hipError_t launch_adjoint_rs(const SmoothArgs& a, const dim3& grid, size_t lds, hipStream_t st)
{
    const void* k = a.cosines ? (const void*)k_adjoint<true, RS> : (const void*)k_adjoint<false, RS>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (a.cosines)
        hipLaunchKernelGGL((k_adjoint<true, RS>), grid, dim3(kBlock), lds, st, a);
    else
        hipLaunchKernelGGL((k_adjoint<false, RS>), grid, dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_adjoint(const SmoothArgs& a, int64_t patch_blocks, size_t lds, hipStream_t st)
{
    if (patch_blocks > 0) {
        if (patch_blocks > 0x7fffffff || a.n_split > 65535) return hipErrorInvalidValue;
        const dim3 grid((unsigned)patch_blocks, (unsigned)a.n_split);
        if (a.Rs == 12) return launch_adjoint_rs<12>(a, grid, lds, st);
        if (a.Rs == 16) return launch_adjoint_rs<16>(a, grid, lds, st);
        if (a.Rs == 20) return launch_adjoint_rs<20>(a, grid, lds, st);
        return launch_adjoint_rs<0>(a, grid, lds, st);
    }
    return hipSuccess;
}

template <int RS, bool DB>
static hipError_t launch_adjoint_gather(const SmoothArgs& a, const dim3& grid, size_t lds, hipStream_t st)
{
    const void* k = a.cosines ? (const void*)k_adjoint_mom<true, RS, DB> : (const void*)k_adjoint_mom<false, RS, DB>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (a.cosines)
        hipLaunchKernelGGL((k_adjoint_mom<true, RS, DB>), grid, dim3(kBlock), lds, st, a);
    else
        hipLaunchKernelGGL((k_adjoint_mom<false, RS, DB>), grid, dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

template <int RS>
static hipError_t launch_adjoint_mom_rs(const SmoothArgs& a, int64_t patch_blocks, size_t lds, int dbuf, hipStream_t st)
{
    const int S = a.rx.n * a.ry.n;
    hipLaunchKernelGGL(k_adj_taps<RS>, dim3(1), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // one thread per (scan point, 4 bins of a correlation row)
    const int64_t n_thr = (int64_t)S * ((a.mlen + 3) / 4);
    const unsigned blocks = (unsigned)((n_thr + 255) / 256);
    const bool aligned = (a.T & 3) == 0 && ((uintptr_t)a.grad_out & 15) == 0 && ((uintptr_t)a.moments & 15) == 0;
    if (aligned)
        hipLaunchKernelGGL((k_adj_moments<RS, true>), dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_adj_moments<RS, false>), dim3(blocks), dim3(256), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // two row buffers when the plan gave the LDS for them and the rows are
    // whole, aligned 16-byte pieces; else one (the same rows per stage)
    const bool db = dbuf && (a.mlen & 3) == 0 && ((uintptr_t)a.moments & 15) == 0 &&
                    lds >= adj_mom_lds(2, a.rows, adj_moments(RS), a.mlen);
    const dim3 grid((unsigned)patch_blocks, (unsigned)a.n_split);
    if (db) return launch_adjoint_gather<RS, true>(a, grid, lds, st);
    return launch_adjoint_gather<RS, false>(a, grid, lds, st);
}

hipError_t launch_adjoint_moments(const SmoothArgs& a, int64_t patch_blocks, size_t lds, int dbuf, hipStream_t st)
{
    if (patch_blocks <= 0) return hipSuccess;
    if (patch_blocks > 0x7fffffff || a.n_split > 65535 || a.rows < 1 || a.mlen != a.T + 2 * a.Rs) return hipErrorInvalidValue;
    if (!smooth_moments_radius(a.Rs) || lds < adj_mom_lds(1, a.rows, adj_moments(a.Rs), a.mlen)) return hipErrorInvalidValue;
    if (a.Rs == 12) return launch_adjoint_mom_rs<12>(a, patch_blocks, lds, dbuf, st);
    if (a.Rs == 16) return launch_adjoint_mom_rs<16>(a, patch_blocks, lds, dbuf, st);
    if (a.Rs == 20) return launch_adjoint_mom_rs<20>(a, patch_blocks, lds, dbuf, st);
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint_reduce(const SmoothArgs& a, float* grad_rec, hipStream_t st)
{
    if (a.n_cap <= 0) return hipSuccess;
    const int64_t blocks = ((int64_t)a.n_cap * 8 + 255) / 256;   // one thread per output word
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adjoint_reduce, dim3((unsigned)blocks), dim3(256), 0, st, a, grad_rec);
    return hipGetLastError();
}

hipError_t launch_grad_maps(const GradMapArgs& g, hipStream_t st)
{
    const int64_t npx = (int64_t)g.ax.n * g.ay.n;
    int64_t zb = (npx + 255) / 256;
    if (zb > 8192) zb = 8192;
    hipLaunchKernelGGL(k_grad_zero, dim3((unsigned)zb), dim3(256), 0, st, g, npx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g.n_cap > 0) {
        hipLaunchKernelGGL(k_grad_scatter, dim3((unsigned)((g.n_cap + 255) / 256)), dim3(256), 0, st, g, npx);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_grad_gather, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, st, g, npx);
    return hipGetLastError();
}

}  // namespace nlos
