// Pair kernels of the transient NLOS forward operator (gfx950).
//
// For every wall scan point and hidden patch (Section 2, Eq. (1), extended
// with Lambertian cosines and device legs), the kernels bin the pair's weight
// into the scan point's time histogram and then blur each histogram with the
// Gaussian jitter of Section 2 (Algorithm 1, step 2.3) while writing it out.
//
// Work decomposition (one workgroup = 16 waves = 1024 lanes):
//   * a workgroup owns a tile of histograms -- TX x TY detector points (times
//     TL laser points, non-confocal) -- over one window of output bins; the
//     histograms live in LDS for the whole pass;
//   * each lane owns one patch at a time (coalesced 32-byte record loads; the
//     record order keeps a wavefront's 64 patches within a small patch of the
//     surface) and loops over the tile's histograms with the wall point
//     wave-uniform, so per-column / per-row terms of the distance are hoisted;
//   * a wavefront skips a tile outright when a lower bound of every one of its
//     arrivals lies past the window;
//   * a pair is evaluated in fp32 (one v_rsq_f32 per leg); pairs whose fp32
//     arrival lies within the guard band of a bin edge go to an LDS queue and
//     are re-binned in fp64 before the flush (queue overflow re-bins in
//     place), so every bin equals the fp64 one;
//   * histograms accumulate in 64-bit fixed point with LDS integer atomics
//     (ds_add_u64): a pair adds round(w * s) as a 32-bit increment, with
//     s = 2^31 / W and W >= every weight the tile can see (a / r_min^4 over
//     the workgroup's patches, from a pre-pass).  On gfx950 an LDS float atomic
//     add costs about 3 cycles per active lane, the 64-bit integer add a few
//     cycles per wavefront;
//   * the flush converts back to float, applies the jitter taps with a sliding
//     register window and writes the histograms with coalesced stores (or
//     float atomics into a zeroed output when patches are split over
//     workgroups).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nlos_device.h"
#include "nlos_internal.h"

namespace nlos {

typedef unsigned long long u64;

size_t lds_bytes_for(int slots, int stride, int q_cap)
{
    size_t b = (size_t)slots * (size_t)stride * 8;   // u64 histograms
    b += (size_t)q_cap * 8;                            // queue: index + increment
    b += (size_t)slots * 8;                            // fp64 path offset per slot
    b += (size_t)slots * 4 * 8;                        // fp32 tables
    b += 128;                                          // counter, reduction scratch
    return (b + 255) & ~(size_t)255;
}

// LDS layout (8-byte aligned: histograms, queue and fp64 table come first).
struct Lds {
    u64* hist;
    uint32_t* qidx;
    uint32_t* qinc;
    double* so;     // [slots] fp64 path offset o (both device legs)
    float* wlx;     // [slots] laser point (confocal: = detector point)
    float* wly;
    float* wdx;     // [slots] detector point
    float* wdy;
    float* oil;     // [slots] fp32(o_l * inv + delta)   (confocal: fp32(o * inv + delta))
    float* oid;     // [slots] fp32(o_d * inv)           (confocal: unused)
    float* gg;      // [slots] g_l * g_d
    float* pad;
    uint32_t* qcount;
    float* red;     // [16] per-wave maxima
};

__device__ __forceinline__ Lds lds_layout(unsigned char* base, int slots, int stride, int q_cap)
{
    Lds L;
    L.hist = (u64*)base;
    L.qidx = (uint32_t*)(L.hist + (size_t)slots * stride);
    L.qinc = L.qidx + q_cap;
    L.so = (double*)(L.qinc + q_cap);
    L.wlx = (float*)(L.so + slots);
    L.wly = L.wlx + slots;
    L.wdx = L.wly + slots;
    L.wdy = L.wdx + slots;
    L.oil = L.wdy + slots;
    L.oid = L.oil + slots;
    L.gg = L.oid + slots;
    L.pad = L.gg + slots;
    L.qcount = (uint32_t*)(L.pad + slots);
    L.red = (float*)(L.qcount + 4);
    return L;
}

__device__ __forceinline__ void lds_add(u64* p, uint32_t inc)
{
    __hip_atomic_fetch_add(p, (u64)inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ float uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Squared distance from patch (px, py, pz) to the nearest and the farthest
// point of the wall rectangle [x0, x1] x [y0, y1].
__device__ __forceinline__ float rect_r2_min(float px, float py, float pz2, float x0, float x1, float y0,
                                             float y1)
{
    const float dx = fmaxf(fmaxf(x0 - px, px - x1), 0.f);
    const float dy = fmaxf(fmaxf(y0 - py, py - y1), 0.f);
    return fmaf(dx, dx, fmaf(dy, dy, pz2));
}

__device__ __forceinline__ float rect_r2_max(float px, float py, float pz2, float x0, float x1, float y0,
                                             float y1)
{
    const float dx = fmaxf(fabsf(px - x0), fabsf(px - x1));
    const float dy = fmaxf(fabsf(py - y0), fabsf(py - y1));
    return fmaf(dx, dx, fmaf(dy, dy, pz2));
}

// Block-wide maximum of a non-negative float (wave butterfly, then LDS).
__device__ __forceinline__ float block_max(float v, float* red)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float m = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, red[w]);
    return m;
}

// Flush 4 consecutive outputs t..t+3 (< t1) of one histogram row:
// out[t] = gg * sum_j taps[j + R] * H[t - j], with H holding bins [hb, he)
// (fixed point, scaled back by inv_s) and zero elsewhere (zero padding).  The
// 4 + 2R histogram values are read once into a sliding register window.
__device__ __forceinline__ void flush_group(const FwdArgs& a, const u64* H, double inv_s, int hb, int he,
                                            int t, int t1, float gg, float* out, bool vec)
{
    const int R = a.R;
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
    for (int e = -R; e <= 3 + R; ++e) {
        const int x = t + e;
        const float v = (x >= hb && x < he) ? (float)((double)H[x - hb] * inv_s) : 0.f;
        // output t+m uses tap index m - e + R
        const int i0 = -e + R;
        if (i0 >= 0 && i0 <= 2 * R) acc0 = fmaf(a.taps[i0], v, acc0);
        if (i0 + 1 >= 0 && i0 + 1 <= 2 * R) acc1 = fmaf(a.taps[i0 + 1], v, acc1);
        if (i0 + 2 >= 0 && i0 + 2 <= 2 * R) acc2 = fmaf(a.taps[i0 + 2], v, acc2);
        if (i0 + 3 >= 0 && i0 + 3 <= 2 * R) acc3 = fmaf(a.taps[i0 + 3], v, acc3);
    }
    acc0 *= gg;
    acc1 *= gg;
    acc2 *= gg;
    acc3 *= gg;
    if (a.atomic_out) {
        unsafeAtomicAdd(out + t, acc0);
        if (t + 1 < t1) unsafeAtomicAdd(out + t + 1, acc1);
        if (t + 2 < t1) unsafeAtomicAdd(out + t + 2, acc2);
        if (t + 3 < t1) unsafeAtomicAdd(out + t + 3, acc3);
    } else if (vec && t + 3 < t1) {
        *reinterpret_cast<float4*>(out + t) = make_float4(acc0, acc1, acc2, acc3);
    } else {
        out[t] = acc0;
        if (t + 1 < t1) out[t + 1] = acc1;
        if (t + 2 < t1) out[t + 2] = acc2;
        if (t + 3 < t1) out[t + 3] = acc3;
    }
}

// Block -> (laser tile, detector tile, time window, patch split).
struct BlockPos {
    int tile_l, tile_x, tile_y;
    int t0w, t1w, hb, he;
    int pb, pe;   // patch range
};

__device__ __forceinline__ BlockPos block_pos(const FwdArgs& a, int n_act)
{
    BlockPos b;
    int id = (int)blockIdx.x;
    const int split = id % a.n_split;
    id /= a.n_split;
    const int twi = id % a.n_tw;
    id /= a.n_tw;
    const int tile_d = id % (a.tiles_x * a.tiles_y);
    b.tile_l = id / (a.tiles_x * a.tiles_y);
    b.tile_x = tile_d / a.tiles_y;
    b.tile_y = tile_d % a.tiles_y;
    b.t0w = twi * a.tw;
    b.t1w = min(a.T, b.t0w + a.tw);
    b.hb = max(0, b.t0w - a.R);
    b.he = min(a.T, b.t1w + a.R);
    const int chunk = (n_act + a.n_split - 1) / a.n_split;
    b.pb = min(n_act, split * chunk);
    b.pe = min(n_act, b.pb + chunk);
    return b;
}

__device__ __forceinline__ int active_count(const FwdArgs& a)
{
    int n = a.n_cap;
    if (a.n_active) {
        n = *a.n_active;
        n = n < 0 ? 0 : (n > a.n_cap ? a.n_cap : n);
    }
    return n;
}

// Queue overflow: re-bin the pair in fp64 right away (out of line: it is
// rare, and keeping it out of the unrolled pair loop keeps its fp64 work off
// the common path).
__device__ __attribute__((noinline)) void guard_overflow(u64* hist_row, const float4* patches, int p,
                                                         float wlx, float wly, float wdx, float wdy,
                                                         double o, double inv, int hb, int Tl, uint32_t inc)
{
    const float4 A = patches[2 * (size_t)p];
    const int kl = exact_bin(A.x, A.y, A.z, wlx, wly, wdx, wdy, o, inv) - hb;
    if ((unsigned)kl < (unsigned)Tl) lds_add(hist_row + kl, inc);
}

// Push a guard pair to the LDS queue (re-binned in fp64 before the flush).
__device__ __forceinline__ void guard_push(const Lds& L, const FwdArgs& a, int p, int j, uint32_t inc, int hb,
                                           int Tl)
{
    const uint32_t slot = __hip_atomic_fetch_add(L.qcount, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
    if (slot < (uint32_t)a.q_cap) {
        L.qidx[slot] = ((uint32_t)p << 8) | (uint32_t)j;
        L.qinc[slot] = inc;
    } else {
        guard_overflow(L.hist + (size_t)j * a.stride, a.patches, p, L.wlx[j], L.wly[j], L.wdx[j], L.wdy[j],
                       L.so[j], a.inv, hb, Tl, inc);
    }
}

// Drain the guard queue: exact fp64 bin for every queued pair.
__device__ __forceinline__ void guard_drain(const Lds& L, const FwdArgs& a, int hb, int Tl)
{
    const uint32_t nq = min(*L.qcount, (uint32_t)a.q_cap);
    for (uint32_t i = threadIdx.x; i < nq; i += blockDim.x) {
        const uint32_t e = L.qidx[i];
        const int p = (int)(e >> 8), j = (int)(e & 255u);
        const float4 A = a.patches[2 * (size_t)p];
        const int kl = exact_bin(A.x, A.y, A.z, L.wlx[j], L.wly[j], L.wdx[j], L.wdy[j], L.so[j], a.inv) - hb;
        if ((unsigned)kl < (unsigned)Tl) lds_add(L.hist + (size_t)j * a.stride + kl, L.qinc[i]);
    }
}

// Load patch p of [pb, pe) or, past the range, a stand-in patch whose arrival
// lies at least 64 bins past the window (never binned, never queued, culled).
__device__ __forceinline__ void load_patch(const FwdArgs& a, int p, int pe, float4* A, float4* B)
{
    *A = make_float4(a.dummy_x, 0.f, 1.f, 0.f);
    *B = make_float4(0.f, 0.f, -1.f, 0.f);
    if (p < pe) {
        *A = a.patches[2 * (size_t)p];
        *B = a.patches[2 * (size_t)p + 1];
    }
}

// Scale of the fixed-point histograms: s = 2^31 / W, W = max over the
// workgroup's patches of a / (r_l,min^2 r_d,min^2), an upper bound of every
// pair weight of the tile (cosine factors <= 1, r >= r_min).
__device__ __forceinline__ float weight_scale(const FwdArgs& a, const Lds& L, int pb, int pe, float lx0,
                                              float lx1, float ly0, float ly1, float dx0, float dx1,
                                              float dy0, float dy1)
{
    float wmax = 0.f;
    for (int p = pb + (int)threadIdx.x; p < pe; p += blockDim.x) {
        const float4 A = a.patches[2 * (size_t)p];
        const float pz2 = A.z * A.z;
        const float r2l = rect_r2_min(A.x, A.y, pz2, lx0, lx1, ly0, ly1);
        const float r2d = rect_r2_min(A.x, A.y, pz2, dx0, dx1, dy0, dy1);
        wmax = fmaxf(wmax, A.w / (r2l * r2d));
    }
    const float W = block_max(wmax, L.red);
    return W > 0.f ? 2147483648.0f / W : 1.0f;
}

// ---------------------------------------------------------------------------
// Confocal: tile of TX x TY scan points; slot j = c * TY + r.
template <int TX, int TY, bool COS, bool WIN>
__global__ void __launch_bounds__(kBlock) k_confocal(const FwdArgs a)
{
    constexpr int NS = TX * TY;
    extern __shared__ __align__(16) unsigned char smem[];
    const Lds L = lds_layout(smem, NS, a.stride, a.q_cap);
    const int n_act = active_count(a);
    const BlockPos bp = block_pos(a, n_act);
    const int hb = WIN ? bp.hb : 0, Tl = WIN ? bp.he - bp.hb : a.T;

    for (int i = threadIdx.x; i < NS * a.stride; i += blockDim.x) L.hist[i] = 0ull;
    if (threadIdx.x == 0) *L.qcount = 0u;
    if (threadIdx.x < NS) {
        const int j = threadIdx.x;
        const int ix = min(bp.tile_x * TX + j / TY, a.rx.n - 1);
        const int iy = min(bp.tile_y * TY + j % TY, a.ry.n - 1);
        const float wx = canon(a.rx, ix), wy = canon(a.ry, iy);
        double off, g;
        device_leg(wx, wy, a.cx, a.cy, a.s, &off, &g);
        const double o = off + off;
        L.so[j] = o;
        L.wlx[j] = wx;
        L.wly[j] = wy;
        L.wdx[j] = wx;
        L.wdy[j] = wy;
        L.oil[j] = (float)(o * a.inv + (double)a.delta);
        L.gg[j] = (float)(g * g);
    }
    __syncthreads();

    float wx[TX], wy[TY], oi[NS];
#pragma unroll
    for (int c = 0; c < TX; ++c) wx[c] = uniform(L.wdx[c * TY]);
#pragma unroll
    for (int r = 0; r < TY; ++r) wy[r] = uniform(L.wdy[r]);
    float oi_min = 3.0e38f, oi_max = 0.f;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        oi[j] = L.oil[j];   // kept in VGPRs: the arrival fma then reads one SGPR (inv2)
        oi_min = fminf(oi_min, oi[j]);
        oi_max = fmaxf(oi_max, oi[j]);
    }
    float x0 = wx[0], x1 = wx[0], y0 = wy[0], y1 = wy[0];
#pragma unroll
    for (int c = 1; c < TX; ++c) {
        x0 = fminf(x0, wx[c]);
        x1 = fmaxf(x1, wx[c]);
    }
#pragma unroll
    for (int r = 1; r < TY; ++r) {
        y0 = fminf(y0, wy[r]);
        y1 = fmaxf(y1, wy[r]);
    }
    const float inv2 = a.inv2_f, two_delta = a.two_delta;
    const float s = weight_scale(a, L, bp.pb, bp.pe, x0, x1, y0, y1, x0, x1, y0, y1);
    // a wavefront skips the tile when every arrival is at least 2 bins past
    // the window (the bound is exact up to fp32 rounding, far below 2 bins)
    const float cut_hi = (float)(hb + Tl + 2);
    const float cut_lo = (float)(hb - 2);

    for (int base = bp.pb; base < bp.pe; base += blockDim.x) {
        const int p = base + (int)threadIdx.x;
        float4 A, B;
        load_patch(a, p, bp.pe, &A, &B);
        const PatchC pc = patch_consts(A, B, COS);
        {
            const float r2lo = rect_r2_min(pc.px, pc.py, pc.pz2, x0, x1, y0, y1);
            bool out = fmaf(__builtin_amdgcn_sqrtf(r2lo), inv2, oi_min) >= cut_hi;
            if (WIN) {
                const float r2hi = rect_r2_max(pc.px, pc.py, pc.pz2, x0, x1, y0, y1);
                out = out || fmaf(__builtin_amdgcn_sqrtf(r2hi), inv2, oi_max) < cut_lo;
            }
            if (__all(out)) continue;
        }
        const float aps = (COS ? pc.ap : A.w) * s;
        float cx2[TX], axv[TX], cy2[TY], byv[TY];
#pragma unroll
        for (int c = 0; c < TX; ++c) col_terms(pc, wx[c], &cx2[c], &axv[c]);
#pragma unroll
        for (int r = 0; r < TY; ++r) row_terms(pc, wy[r], &cy2[r], &byv[r]);
#pragma unroll
        for (int c = 0; c < TX; ++c) {
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                const int j = c * TY + r;
                const Leg lg = leg_eval(cx2[c], cy2[r], axv[c], byv[r], COS);
                const float w = fmaf(lg.rr, inv2, oi[j]);
                const Decision d = decide(w, two_delta);
                const uint32_t inc = (uint32_t)fmaf(COS ? lg.q * lg.q : lg.ri4, aps, 0.5f);
                const int kl = d.k - hb;
                if (d.sure) {
                    if ((unsigned)kl < (unsigned)Tl) lds_add(L.hist + j * a.stride + kl, inc);
                } else if ((unsigned)kl <= (unsigned)Tl) {
                    guard_push(L, a, p, j, inc, hb, Tl);
                }
            }
        }
    }
    __syncthreads();
    guard_drain(L, a, hb, Tl);
    __syncthreads();

    const double inv_s = 1.0 / (double)s;
    const int ng = (bp.t1w - bp.t0w + 3) / 4;
    const bool vec = ((a.T & 3) == 0) && ((bp.t0w & 3) == 0);
    for (int idx = threadIdx.x; idx < NS * ng; idx += blockDim.x) {
        const int j = idx / ng, g = idx - j * ng;
        const int ix = bp.tile_x * TX + j / TY, iy = bp.tile_y * TY + j % TY;
        if (ix >= a.rx.n || iy >= a.ry.n) continue;
        float* out = a.out + ((size_t)ix * a.ry.n + iy) * (size_t)a.T;
        flush_group(a, L.hist + (size_t)j * a.stride, inv_s, bp.hb, bp.he, bp.t0w + 4 * g, bp.t1w, L.gg[j],
                    out, vec);
    }
}

// ---------------------------------------------------------------------------
// Non-confocal: tile of TL laser points x (TX x TY) detector points;
// slot j = (l * TX + c) * TY + r.
template <int TL, int TX, int TY, bool COS, bool WIN>
__global__ void __launch_bounds__(kBlock) k_nonconfocal(const FwdArgs a)
{
    constexpr int ND = TX * TY;
    constexpr int NS = TL * ND;
    extern __shared__ __align__(16) unsigned char smem[];
    const Lds L = lds_layout(smem, NS, a.stride, a.q_cap);
    const int n_act = active_count(a);
    const BlockPos bp = block_pos(a, n_act);
    const int hb = WIN ? bp.hb : 0, Tl = WIN ? bp.he - bp.hb : a.T;
    const int n_laser = a.lx.n * a.ly.n;

    for (int i = threadIdx.x; i < NS * a.stride; i += blockDim.x) L.hist[i] = 0ull;
    if (threadIdx.x == 0) *L.qcount = 0u;
    if (threadIdx.x < NS) {
        const int j = threadIdx.x;
        const int l = min(bp.tile_l * TL + j / ND, n_laser - 1);
        const int dj = j % ND;
        const int ix = min(bp.tile_x * TX + dj / TY, a.rx.n - 1);
        const int iy = min(bp.tile_y * TY + dj % TY, a.ry.n - 1);
        const float lx = canon(a.lx, l / a.ly.n), ly = canon(a.ly, l % a.ly.n);
        const float wx = canon(a.rx, ix), wy = canon(a.ry, iy);
        double off_l, g_l, off_d, g_d;
        device_leg(lx, ly, a.cx, a.cy, a.s, &off_l, &g_l);
        device_leg(wx, wy, a.cx, a.cy, a.s, &off_d, &g_d);
        L.so[j] = off_l + off_d;
        L.wlx[j] = lx;
        L.wly[j] = ly;
        L.wdx[j] = wx;
        L.wdy[j] = wy;
        L.oil[j] = (float)(off_l * a.inv + (double)a.delta);
        L.oid[j] = (float)(off_d * a.inv);
        L.gg[j] = (float)(g_l * g_d);
    }
    __syncthreads();

    float lxs[TL], lys[TL], oil[TL], wx[TX], wy[TY], oid[ND];
    float lx0 = 3.0e38f, lx1 = -3.0e38f, ly0 = 3.0e38f, ly1 = -3.0e38f;
    float oil_min = 3.0e38f, oil_max = 0.f, oid_min = 3.0e38f, oid_max = 0.f;
#pragma unroll
    for (int l = 0; l < TL; ++l) {
        lxs[l] = uniform(L.wlx[l * ND]);
        lys[l] = uniform(L.wly[l * ND]);
        oil[l] = uniform(L.oil[l * ND]);
        lx0 = fminf(lx0, lxs[l]);
        lx1 = fmaxf(lx1, lxs[l]);
        ly0 = fminf(ly0, lys[l]);
        ly1 = fmaxf(ly1, lys[l]);
        oil_min = fminf(oil_min, oil[l]);
        oil_max = fmaxf(oil_max, oil[l]);
    }
#pragma unroll
    for (int c = 0; c < TX; ++c) wx[c] = uniform(L.wdx[c * TY]);
#pragma unroll
    for (int r = 0; r < TY; ++r) wy[r] = uniform(L.wdy[r]);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        oid[d] = uniform(L.oid[d]);
        oid_min = fminf(oid_min, oid[d]);
        oid_max = fmaxf(oid_max, oid[d]);
    }
    float x0 = wx[0], x1 = wx[0], y0 = wy[0], y1 = wy[0];
#pragma unroll
    for (int c = 1; c < TX; ++c) {
        x0 = fminf(x0, wx[c]);
        x1 = fmaxf(x1, wx[c]);
    }
#pragma unroll
    for (int r = 1; r < TY; ++r) {
        y0 = fminf(y0, wy[r]);
        y1 = fmaxf(y1, wy[r]);
    }
    const float inv = a.inv_f, two_delta = a.two_delta;
    const float s = weight_scale(a, L, bp.pb, bp.pe, lx0, lx1, ly0, ly1, x0, x1, y0, y1);
    const float cut_hi = (float)(hb + Tl + 2);
    const float cut_lo = (float)(hb - 2);
    const float o_min = oil_min + oid_min, o_max = oil_max + oid_max;

    for (int base = bp.pb; base < bp.pe; base += blockDim.x) {
        const int p = base + (int)threadIdx.x;
        float4 A, B;
        load_patch(a, p, bp.pe, &A, &B);
        const PatchC pc = patch_consts(A, B, COS);
        {
            const float rl = __builtin_amdgcn_sqrtf(rect_r2_min(pc.px, pc.py, pc.pz2, lx0, lx1, ly0, ly1));
            const float rd = __builtin_amdgcn_sqrtf(rect_r2_min(pc.px, pc.py, pc.pz2, x0, x1, y0, y1));
            bool out = fmaf(rl + rd, inv, o_min) >= cut_hi;
            if (WIN) {
                const float Rl = __builtin_amdgcn_sqrtf(rect_r2_max(pc.px, pc.py, pc.pz2, lx0, lx1, ly0, ly1));
                const float Rd = __builtin_amdgcn_sqrtf(rect_r2_max(pc.px, pc.py, pc.pz2, x0, x1, y0, y1));
                out = out || fmaf(Rl + Rd, inv, o_max) < cut_lo;
            }
            if (__all(out)) continue;
        }
        // laser legs
        float ul[TL], fl[TL];
#pragma unroll
        for (int l = 0; l < TL; ++l) {
            float cx2, axv, cy2, byv;
            col_terms(pc, lxs[l], &cx2, &axv);
            row_terms(pc, lys[l], &cy2, &byv);
            const Leg lg = leg_eval(cx2, cy2, axv, byv, COS);
            ul[l] = fmaf(lg.rr, inv, oil[l]);
            fl[l] = (COS ? lg.q * pc.ap : lg.ri2 * A.w) * s;
        }
        // detector legs
        float cx2[TX], axv[TX], cy2[TY], byv[TY];
#pragma unroll
        for (int c = 0; c < TX; ++c) col_terms(pc, wx[c], &cx2[c], &axv[c]);
#pragma unroll
        for (int r = 0; r < TY; ++r) row_terms(pc, wy[r], &cy2[r], &byv[r]);
#pragma unroll
        for (int c = 0; c < TX; ++c) {
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                const int dj = c * TY + r;
                const Leg lg = leg_eval(cx2[c], cy2[r], axv[c], byv[r], COS);
                const float ud = fmaf(lg.rr, inv, oid[dj]);
                const float fd = COS ? lg.q : lg.ri2;
#pragma unroll
                for (int l = 0; l < TL; ++l) {
                    const int j = l * ND + dj;
                    const float w = ul[l] + ud;
                    const Decision d = decide(w, two_delta);
                    const uint32_t inc = (uint32_t)fmaf(fl[l], fd, 0.5f);
                    const int kl = d.k - hb;
                    if (d.sure) {
                        if ((unsigned)kl < (unsigned)Tl) lds_add(L.hist + j * a.stride + kl, inc);
                    } else if ((unsigned)kl <= (unsigned)Tl) {
                        guard_push(L, a, p, j, inc, hb, Tl);
                    }
                }
            }
        }
    }
    __syncthreads();
    guard_drain(L, a, hb, Tl);
    __syncthreads();

    const double inv_s = 1.0 / (double)s;
    const size_t S = (size_t)a.rx.n * a.ry.n;
    const int ng = (bp.t1w - bp.t0w + 3) / 4;
    const bool vec = ((a.T & 3) == 0) && ((bp.t0w & 3) == 0);
    for (int idx = threadIdx.x; idx < NS * ng; idx += blockDim.x) {
        const int j = idx / ng, g = idx - j * ng;
        const int l = bp.tile_l * TL + j / ND;
        const int dj = j % ND;
        const int ix = bp.tile_x * TX + dj / TY, iy = bp.tile_y * TY + dj % TY;
        if (l >= n_laser || ix >= a.rx.n || iy >= a.ry.n) continue;
        float* out = a.out + ((size_t)l * S + (size_t)ix * a.ry.n + iy) * (size_t)a.T;
        flush_group(a, L.hist + (size_t)j * a.stride, inv_s, bp.hb, bp.he, bp.t0w + 4 * g, bp.t1w, L.gg[j],
                    out, vec);
    }
}

// ---------------------------------------------------------------------------
// Bin export (test hook): same device functions and decision rule.
__global__ void __launch_bounds__(256) k_debug_bins(const DebugArgs d)
{
    const FwdArgs& a = d.f;
    const int n_act = active_count(a);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int S = a.rx.n * a.ry.n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < d.n_pairs; idx += stride) {
        const int64_t h = idx / a.n_cap;
        const int p = (int)(idx - h * a.n_cap);
        if (p >= n_act) {
            d.bins[idx] = INT32_MIN;
            if (d.u_fast) d.u_fast[idx] = 0.0;
            if (d.u_exact) d.u_exact[idx] = 0.0;
            continue;
        }
        const int l = (int)(h / S), dd = (int)(h % S);
        const int ix = dd / a.ry.n, iy = dd % a.ry.n;
        const float wx = canon(a.rx, ix), wy = canon(a.ry, iy);
        float lx = wx, ly = wy;
        if (!d.confocal) {
            lx = canon(a.lx, l / a.ly.n);
            ly = canon(a.ly, l % a.ly.n);
        }
        const float4 A = a.patches[2 * (size_t)p];
        const float4 B = a.patches[2 * (size_t)p + 1];
        const PatchC pc = patch_consts(A, B, a.cosines != 0);
        double off_l, g_l, off_d, g_d;
        device_leg(lx, ly, a.cx, a.cy, a.s, &off_l, &g_l);
        device_leg(wx, wy, a.cx, a.cy, a.s, &off_d, &g_d);
        const double o = off_l + off_d;
        float w;
        if (d.confocal) {
            const float oi = (float)(o * a.inv + (double)a.delta);
            float cx2, axv, cy2, byv;
            col_terms(pc, wx, &cx2, &axv);
            row_terms(pc, wy, &cy2, &byv);
            const Leg lg = leg_eval(cx2, cy2, axv, byv, a.cosines != 0);
            w = fmaf(lg.rr, a.inv2_f, oi);
        } else {
            const float oil = (float)(off_l * a.inv + (double)a.delta);
            const float oid = (float)(off_d * a.inv);
            float cx2, axv, cy2, byv;
            col_terms(pc, lx, &cx2, &axv);
            row_terms(pc, ly, &cy2, &byv);
            const Leg ll = leg_eval(cx2, cy2, axv, byv, a.cosines != 0);
            col_terms(pc, wx, &cx2, &axv);
            row_terms(pc, wy, &cy2, &byv);
            const Leg ld = leg_eval(cx2, cy2, axv, byv, a.cosines != 0);
            w = fmaf(ll.rr, a.inv_f, oil) + fmaf(ld.rr, a.inv_f, oid);
        }
        const Decision dc = decide(w, a.two_delta);
        double ue;
        const int ke = exact_bin(A.x, A.y, A.z, lx, ly, wx, wy, o, a.inv, &ue);
        // the forward kernels trust the fp32 bin only when it is sure and in
        // the window; everything else is decided in fp64
        d.bins[idx] = (dc.sure && dc.k >= 0 && dc.k < a.T) ? dc.k : ke;
        if (d.u_fast) d.u_fast[idx] = (double)w - (double)a.delta;
        if (d.u_exact) d.u_exact[idx] = ue;
    }
}

__global__ void k_fill(float* out, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = 0.f;
}

// ---------------------------------------------------------------------------
// Launchers.
template <typename K>
static hipError_t launch_k(K kern, const FwdArgs& a, const Plan& plan, hipStream_t st)
{
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)plan.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)plan.n_blocks), dim3(kBlock), plan.lds_bytes, st, a);
    return hipGetLastError();
}

#define NLOS_CONF_CASE(X, Y)                                                              \
    if (plan.tx == X && plan.ty == Y) {                                                   \
        if (plan.n_tw > 1)                                                                \
            return a.cosines ? launch_k(k_confocal<X, Y, true, true>, a, plan, st)        \
                             : launch_k(k_confocal<X, Y, false, true>, a, plan, st);      \
        return a.cosines ? launch_k(k_confocal<X, Y, true, false>, a, plan, st)           \
                         : launch_k(k_confocal<X, Y, false, false>, a, plan, st);         \
    }
#define NLOS_NC_CASE(TLV, X, Y)                                                           \
    if (plan.tl == TLV && plan.tx == X && plan.ty == Y) {                                 \
        if (plan.n_tw > 1)                                                                \
            return a.cosines ? launch_k(k_nonconfocal<TLV, X, Y, true, true>, a, plan, st) \
                             : launch_k(k_nonconfocal<TLV, X, Y, false, true>, a, plan, st); \
        return a.cosines ? launch_k(k_nonconfocal<TLV, X, Y, true, false>, a, plan, st)   \
                         : launch_k(k_nonconfocal<TLV, X, Y, false, false>, a, plan, st); \
    }

bool tile_supported(bool confocal, int tx, int ty, int tl)
{
    if (confocal) {
        return (tx == 4 && ty == 4) || (tx == 8 && ty == 4) || (tx == 2 && ty == 4) ||
               (tx == 2 && ty == 2) || (tx == 1 && ty == 2) || (tx == 1 && ty == 1);
    }
    return (tl == 4 && tx == 2 && ty == 2) || (tl == 2 && tx == 2 && ty == 2) ||
           (tl == 2 && tx == 1 && ty == 2) || (tl == 1 && tx == 1 && ty == 2) ||
           (tl == 1 && tx == 1 && ty == 1);
}

hipError_t launch_forward(const FwdArgs& a, const Plan& plan, bool confocal, hipStream_t st)
{
    if (plan.n_blocks <= 0) return hipSuccess;
    if (confocal) {
        NLOS_CONF_CASE(4, 4)
        NLOS_CONF_CASE(8, 4)
        NLOS_CONF_CASE(2, 4)
        NLOS_CONF_CASE(2, 2)
        NLOS_CONF_CASE(1, 2)
        NLOS_CONF_CASE(1, 1)
    } else {
        NLOS_NC_CASE(4, 2, 2)
        NLOS_NC_CASE(2, 2, 2)
        NLOS_NC_CASE(2, 1, 2)
        NLOS_NC_CASE(1, 1, 2)
        NLOS_NC_CASE(1, 1, 1)
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fill(float* out, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, out, n);
    return hipGetLastError();
}

hipError_t launch_debug(const DebugArgs& d, hipStream_t st)
{
    if (d.n_pairs <= 0) return hipSuccess;
    int64_t blocks = (d.n_pairs + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_debug_bins, dim3((unsigned)blocks), dim3(256), 0, st, d);
    return hipGetLastError();
}

}  // namespace nlos
