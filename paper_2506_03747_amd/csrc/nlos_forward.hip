// Pair kernels of the transient NLOS forward operator (gfx950).
//
// For every wall scan point and hidden patch (Section 2, Eq. (1), extended
// with Lambertian cosines and device legs), the kernels bin the pair's weight
// into the scan point's time histogram and then blur each histogram with the
// Gaussian jitter of Section 2 (Algorithm 1, step 2.3) while writing it out.
//
// Work decomposition (one workgroup = 16 waves = 1024 lanes):
//   * histograms are grouped in units -- TX x TY detector points (times TL
//     laser points, non-confocal); a workgroup owns one unit, or two when
//     units are few: then every workgroup estimates the work of all units from
//     summaries of the records, sorts the estimates in LDS and takes the k-th
//     lightest with the k-th heaviest unit, which evens out the load when a
//     workgroup per CU is all there is;
//   * the histograms live in LDS for the whole pass, over one window of
//     output bins;
//   * each lane owns one patch at a time (coalesced 32-byte record loads; the
//     record order keeps a wavefront's 64 patches within a small square of the
//     surface) and loops over the unit's histograms with the wall point
//     wave-uniform, so per-column / per-row terms of the distance are hoisted;
//   * a wavefront skips a unit outright when a lower bound of every one of its
//     arrivals lies past the window;
//   * a pair is evaluated in fp32 (one v_rsq_f32 per leg); pairs whose fp32
//     arrival lies within the guard band of a bin edge go to an LDS queue and
//     are re-binned in fp64 before the flush (queue overflow re-bins in
//     place), so every bin equals the fp64 one;
//   * histograms accumulate in 64-bit fixed point with LDS integer atomics
//     (ds_add_u64): a pair adds round(w * s) as a 32-bit increment, with
//     s = 2^31 / W and W >= every weight the workgroup's units can see
//     (a_max / r_min^4 over the record summaries).  On gfx950 an LDS float
//     atomic add costs about 3 cycles per active lane, the 64-bit integer add
//     a few cycles per wavefront;
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

constexpr int kQueueWaves = kBlock / 64;   // the guard queue has one segment per wavefront

size_t lds_bytes_for(int slots, int stride, int q_cap)
{
    size_t b = (size_t)slots * (size_t)stride * 8;   // u64 histograms
    b += (size_t)q_cap * 8;                            // queue: (record, slot) + increment
    b += (size_t)slots * 8;                            // fp64 path offset per slot
    b += (size_t)slots * 8;                            // output row per slot
    b += (size_t)slots * 4 * 8;                        // fp32 tables
    b += 64 * 4 + 16;                                  // reduction scratch, chunk counter
    return (b + 255) & ~(size_t)255;
}

// LDS layout (8-byte aligned: histograms, queue and fp64 table come first).
struct Lds {
    u64* hist;
    uint2* q;       // guard queue: kQueueWaves segments of (record << 8 | slot, increment)
    double* so;     // [slots] fp64 path offset o (both device legs)
    long long* row; // [slots] output histogram index, -1: not written
    float* wlx;     // [slots] laser point (confocal: = detector point)
    float* wly;
    float* wdx;     // [slots] detector point
    float* wdy;
    float* oil;     // [slots] fp32(o_l * inv + delta)   (confocal: fp32(o * inv + delta))
    float* oid;     // [slots] fp32(o_d * inv)           (confocal: unused)
    float* gg;      // [slots] g_l * g_d
    float* pad;
    float* red;     // [64] per-wave reduction scratch
    uint32_t* next; // next 64-record chunk of the pair loop
};

__device__ __forceinline__ Lds lds_layout(unsigned char* base, int slots, int stride, int q_cap)
{
    Lds L;
    L.hist = (u64*)base;
    L.q = (uint2*)(L.hist + (size_t)slots * stride);
    L.so = (double*)(L.q + q_cap);
    L.row = (long long*)(L.so + slots);
    L.wlx = (float*)(L.row + slots);
    L.wly = L.wlx + slots;
    L.wdx = L.wly + slots;
    L.wdy = L.wdx + slots;
    L.oil = L.wdy + slots;
    L.oid = L.oil + slots;
    L.gg = L.oid + slots;
    L.pad = L.gg + slots;
    L.red = L.pad + slots;
    L.next = (uint32_t*)(L.red + 64);
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

// Squared lateral distance between two axis-aligned rectangles.
__device__ __forceinline__ float rect_rect_d2(float ax0, float ax1, float ay0, float ay1, float bx0, float bx1,
                                              float by0, float by1)
{
    const float dx = fmaxf(fmaxf(ax0 - bx1, bx0 - ax1), 0.f);
    const float dy = fmaxf(fmaxf(ay0 - by1, by0 - ay1), 0.f);
    return fmaf(dx, dx, dy * dy);
}

// Block-wide maxima of N non-negative floats, in place (DPP within each
// wavefront, then LDS; `red` holds N floats per wavefront).
template <int N>
__device__ __forceinline__ void block_max(float* v, float* red)
{
#pragma unroll
    for (int k = 0; k < N; ++k) {
        v[k] = wave_max_f(v[k]);
        if ((threadIdx.x & 63) == 0) red[(threadIdx.x >> 6) * N + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        float m = 0.f;
        for (int w = 0; w < kBlock / 64; ++w) m = fmaxf(m, red[w * N + k]);
        v[k] = m;
    }
}

// Device buffers named by the arguments are global memory; saying so keeps
// the accesses global (not flat) when the pointer itself was loaded from a
// table, so they do not share the LDS wait counter.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 load4(const float4* p, size_t i)
{
    const v4f v = gmem(reinterpret_cast<const v4f*>(p))[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

// The first three words of record half i (the pair loop does not read the
// fourth; a 12-byte load leaves no dead register that an in-flight load
// would still be writing).
typedef float v3f __attribute__((ext_vector_type(3)));
__device__ __forceinline__ float4 load3(const float4* p, size_t i)
{
    const v3f v = *gmem(reinterpret_cast<const v3f*>(p + i));
    return make_float4(v.x, v.y, v.z, 0.f);
}

// Both halves of record r, 0 <= r < NLOS_MAX_PATCHES = 2^24, so that its
// byte offset fits 32 bits: the loads take the base as a scalar and a 32-bit
// offset per lane.
__device__ __forceinline__ void load_record(const float4* p, int r, float4& A, float4& B)
{
    const uint32_t off = (uint32_t)r * 32u;
    const __attribute__((address_space(1))) char* b = (const __attribute__((address_space(1))) char*)p;
    const v4f va = *(const __attribute__((address_space(1))) v4f*)(b + off);
    const v3f vb = *(const __attribute__((address_space(1))) v3f*)(b + off + 16u);
    A = make_float4(va.x, va.y, va.z, va.w);
    B = make_float4(vb.x, vb.y, vb.z, 0.f);
}

// Stands in for a missing device count, so that the count is always one
// load with no branch before it (the kernels' first argument reads then go
// out together instead of one after another).
__device__ const int32_t kNoCount = 0x7fffffff;

__device__ __forceinline__ int active_count(const FwdArgs& a)
{
    // a scalar read: the count was written before this kernel started and
    // does not change while it runs (kernel start invalidates the scalar cache)
    const int32_t* c = a.n_active ? a.n_active : &kNoCount;
    const int n = *(const __attribute__((address_space(4))) int32_t*)(c);
    return n < 0 ? 0 : (n > a.n_cap ? a.n_cap : n);
}

__device__ __forceinline__ void lds_sub(u64* p, uint32_t dec)
{
    __hip_atomic_fetch_add(p, 0ull - (u64)dec, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Guard correction: the pair was added at its fp32 bin kf (0 <= kf <= Tl);
// move it to the fp64 bin when they differ (the row sums are exact modulo
// 2^64, and every final bin is a sum of non-negative increments).
__device__ __forceinline__ void guard_fix(u64* hist_row, int kf, int ke, int Tl, uint32_t inc)
{
    if (ke == kf) return;
    lds_sub(hist_row + kf, inc);
    if ((unsigned)ke < (unsigned)Tl) lds_add(hist_row + ke, inc);
}

// Queue overflow: correct the pair right away (out of line: it is rare, and
// keeping it out of the unrolled pair loop keeps its fp64 work off the
// common path).
__device__ __attribute__((noinline)) void guard_overflow(u64* hist_row, const float4* patches, int p, int kf,
                                                         float wlx, float wly, float wdx, float wdy,
                                                         double o, double inv, int hb, int Tl, uint32_t inc)
{
    const float4 A = load4(patches, 2 * (size_t)p);
    guard_fix(hist_row, kf, exact_bin(A.x, A.y, A.z, wlx, wly, wdx, wdy, o, inv) - hb, Tl, inc);
}

// Guard pairs: every pair whose fp32 bin lies in 0 .. Tl is added there; the
// pairs whose fp32 arrival lies within the guard band of a bin edge (lane
// mask `m`, uniform, every lane of the wavefront present) are also queued and
// moved to their fp64 bin after the pair loop.  Each wavefront appends to its
// own queue segment (qw entries) and keeps the fill `qn`, uniform, in a
// register, so a push waits for nothing.  A full segment corrects in place.
__device__ __forceinline__ void guard_push(const Lds& L, const FwdArgs& a, uint64_t m, int p, int j, int kf,
                                           uint32_t inc, int hb, int Tl, int wave, int qw, int& qn)
{
    if (m == 0ull) return;
    const bool want = (m >> (threadIdx.x & 63)) & 1ull;
    const int n = __popcll(m);
    if (qn + n <= qw) {
        if (want) {
            const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            L.q[wave * qw + qn + r] = make_uint2(((uint32_t)p << 8) | (uint32_t)j, inc);
        }
        qn += n;
    } else if (want) {
        guard_overflow(L.hist + (size_t)j * a.stride, a.prep ? a.prep : a.patches, p, kf, L.wlx[j], L.wly[j],
                       L.wdx[j], L.wdy[j], L.so[j], a.inv, hb, Tl, inc);
    }
}

// fp32 arrival (in bins, + delta) of record (A, B) at slot j, by the same
// operations as the pair loop: coordinates in bins (times sig), then one fma
// per leg.
template <bool CONF>
__device__ __forceinline__ float fast_arrival(const FwdArgs& a, const Lds& L, float4 A, int j)
{
    const float sig = CONF ? a.inv2_f : a.inv_f;
    // (the arrival uses the coordinates only: no normal terms)
    const PatchC pc = patch_consts_scaled(A, make_float4(0.f, 0.f, 0.f, 0.f), false, sig);
    float cx2, axv, cy2, byv;
    col_terms(pc, L.wdx[j] * sig, &cx2, &axv);
    row_terms(pc, L.wdy[j] * sig, &cy2, &byv);
    const Leg ld = leg_eval_at(cx2, cy2, axv, byv, CONF ? L.oil[j] : L.oid[j], false);
    if (CONF) return ld.rr;
    col_terms(pc, L.wlx[j] * sig, &cx2, &axv);
    row_terms(pc, L.wly[j] * sig, &cy2, &byv);
    const Leg ll = leg_eval_at(cx2, cy2, axv, byv, L.oil[j], false);
    return ll.rr + ld.rr;
}

// After the wavefront's pair loop: its own segment (qn entries), one entry
// per lane; other wavefronts may still be adding (all adds commute).  The
// coordinates come from the stream the pair loop read (records, or their
// pair-loop constants, which keep them as recorded).
template <bool CONF>
__device__ __forceinline__ void guard_drain(const Lds& L, const FwdArgs& a, int hb, int Tl, int wave, int qw, int qn)
{
    const float4* src = a.prep ? a.prep : a.patches;
    for (int e = (int)threadIdx.x & 63; e < qn; e += 64) {
        const uint2 q = L.q[wave * qw + e];
        const int p = (int)(q.x >> 8), j = (int)(q.x & 255u);
        const float4 A = load4(src, 2 * (size_t)p);
        const int kf = decide(fast_arrival<CONF>(a, L, A, j), a.two_delta).k - hb;
        const int ke = exact_bin(A.x, A.y, A.z, L.wlx[j], L.wly[j], L.wdx[j], L.wdy[j], L.so[j], a.inv) - hb;
        guard_fix(L.hist + (size_t)j * a.stride, kf, ke, Tl, q.y);
    }
}

// Load patch p of [pb, pe) or, past the range, a stand-in patch whose arrival
// lies at least 64 bins past the window (never binned, never queued, culled).

// ---------------------------------------------------------------------------
// Record summaries: one workgroup per kStatBlock consecutive records.
__device__ __forceinline__ void chunk_stats_body(const FwdArgs& a, ChunkStat* st, int blk)
{
    __shared__ float red[6][kStatBlock / 64];
    const int n_act = active_count(a);
    const int p = blk * kStatBlock + (int)threadIdx.x;
    float v[6] = {3.0e38f, 3.0e38f, 3.0e38f, 3.0e38f, 3.0e38f, 0.f};   // x0, -x1, y0, -y1, z0, amax
    if (p < n_act) {
        const float4 A = load4(a.patches, 2 * (size_t)p);
        v[0] = A.x;
        v[1] = -A.x;
        v[2] = A.y;
        v[3] = -A.y;
        v[4] = A.z;
        v[5] = A.w;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float x = k == 5 ? wave_extreme_f<true>(v[k]) : wave_extreme_f<false>(v[k]);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float r[6] = {3.0e38f, 3.0e38f, 3.0e38f, 3.0e38f, 3.0e38f, 0.f};
        for (int w = 0; w < kStatBlock / 64; ++w)
            for (int k = 0; k < 6; ++k) r[k] = (k == 5) ? fmaxf(r[k], red[k][w]) : fminf(r[k], red[k][w]);
        ChunkStat c;
        c.x0 = ord_f(r[0]);
        c.x1 = ord_f(-r[1]);
        c.y0 = ord_f(r[2]);
        c.y1 = ord_f(-r[3]);
        c.z0 = ord_f(r[4]);
        c.amax = ord_f(r[5]);
        c.count = max(0, min(kStatBlock, n_act - blk * kStatBlock));
        c.pad = 0;
        st[blk] = c;
    }
}

__global__ void __launch_bounds__(kStatBlock) k_chunk_stats(const FwdArgs a, ChunkStat* st)
{
    chunk_stats_body(a, st, (int)blockIdx.x);
}

// Wall rectangles of the aligned block of histograms that holds unit u --
// 4 x 4 scan points (confocal), or 2 lasers x 2 x 2 detectors -- in
// approximate fp32 grid coordinates (only used for bounds): detector points
// [dx0,dx1]x[dy0,dy1], laser points [lx0,lx1]x[ly0,ly1] (= the detector
// rectangle, confocal).  Every supported unit shape tiles these blocks, so a
// histogram's bound, and with it its fixed-point scale, is the same whatever
// unit the plan chose (alone, batched or in a serving tick).
struct UnitRect {
    float dx0, dx1, dy0, dy1, lx0, lx1, ly0, ly1;
};

__device__ __forceinline__ float approx_coord(const Axis& ax, int i)
{
    return (float)ax.a0 + ((float)i + 0.5f) * (float)ax.step;
}

constexpr int kScaleBlockConf = 4;      // scan points per side of a confocal scale block
constexpr int kScaleBlockNonconf = 2;   // detectors per side and lasers of a non-confocal one

template <bool CONF, int TL, int TX, int TY>
__device__ __forceinline__ UnitRect unit_rect(const FwdArgs& a, int u)
{
    static_assert(CONF ? (kScaleBlockConf % TX == 0 && kScaleBlockConf % TY == 0)
                       : (kScaleBlockNonconf % TX == 0 && kScaleBlockNonconf % TY == 0 &&
                          kScaleBlockNonconf % TL == 0),
                  "units tile the scale blocks");
    constexpr int B = CONF ? kScaleBlockConf : kScaleBlockNonconf;
    UnitRect R;
    const int uy = u % a.tiles_y;
    const int ux = (u / a.tiles_y) % a.tiles_x;
    const int ul = u / (a.tiles_y * a.tiles_x);
    const int ix0 = (ux * TX) / B * B, ix1 = min(ix0 + B, a.rx.n) - 1;
    const int iy0 = (uy * TY) / B * B, iy1 = min(iy0 + B, a.ry.n) - 1;
    R.dx0 = approx_coord(a.rx, ix0);
    R.dx1 = approx_coord(a.rx, ix1);
    R.dy0 = approx_coord(a.ry, iy0);
    R.dy1 = approx_coord(a.ry, iy1);
    if (CONF) {
        R.lx0 = R.dx0;
        R.lx1 = R.dx1;
        R.ly0 = R.dy0;
        R.ly1 = R.dy1;
    } else {
        const int n_laser = a.lx.n * a.ly.n;
        const int l0 = (ul * TL) / B * B;
        R.lx0 = R.ly0 = 3.0e38f;
        R.lx1 = R.ly1 = -3.0e38f;
        for (int l = l0; l < min(l0 + B, n_laser); ++l) {
            const float x = approx_coord(a.lx, l / a.ly.n), y = approx_coord(a.ly, l % a.ly.n);
            R.lx0 = fminf(R.lx0, x);
            R.lx1 = fmaxf(R.lx1, x);
            R.ly0 = fminf(R.ly0, y);
            R.ly1 = fmaxf(R.ly1, y);
        }
    }
    return R;
}

// Upper bound of every pair weight of unit u (of its scale block):
// a_max / (r_l,min^2 r_d,min^2) over the record summaries (cosine factors
// are at most 1).
template <bool CONF, int TL, int TX, int TY>
__device__ __forceinline__ float unit_weight_bound(const FwdArgs& a, int u, const StatF& c)
{
    const UnitRect R = unit_rect<CONF, TL, TX, TY>(a, u);
    if (c.count <= 0) return 0.f;
    const float z2 = c.z0 * c.z0;
    const float rd2 = rect_rect_d2(R.dx0, R.dx1, R.dy0, R.dy1, c.x0, c.x1, c.y0, c.y1) + z2;
    const float rl2 = CONF ? rd2 : rect_rect_d2(R.lx0, R.lx1, R.ly0, R.ly1, c.x0, c.x1, c.y0, c.y1) + z2;
    return c.amax / (rl2 * rd2);
}

// Units of this workgroup: u[0] and, when paired, u[1] (-1 if none).
// Paired units are the unit (x, y) of a laser tile and the unit shifted by
// half the unit grid in both directions (torus shift): a unit near the middle
// of the wall -- where most pairs land in the window -- goes with one near the
// border.  Groups enumerate the half of the grid the shift maps onto the
// other half; grids with both sides odd pair g with n-1-g in unit order.
template <bool PAIR>
__device__ __forceinline__ void pick_units(const FwdArgs& a, int grp, int* u)
{
    if (!PAIR) {
        u[0] = grp;
        return;
    }
    const int tx = a.tiles_x, ty = a.tiles_y, plane = tx * ty;
    if (a.plan) {
        const int half = plane / 2;
        const int ul = grp / half, h = grp % half;
        int ux, uy, vx, vy;
        if ((ty & 1) == 0) {
            ux = h / (ty / 2);
            uy = h % (ty / 2);
            vx = (ux + tx / 2) % tx;
            vy = uy + ty / 2;
        } else {
            ux = h % (tx / 2);
            uy = h / (tx / 2);
            vx = ux + tx / 2;
            vy = (uy + ty / 2) % ty;
        }
        u[0] = ul * plane + ux * ty + uy;
        u[1] = ul * plane + vx * ty + vy;
        return;
    }
    const int partner = a.n_units - 1 - grp;
    u[0] = grp;
    u[1] = partner != grp ? partner : -1;
}

// floor(d / 8) for any sign, at compile time where d is a constant
__host__ __device__ constexpr int floor_div8(int d) { return d >= 0 ? d / 8 : -((7 - d) / 8); }

// A 64-bit fixed-point sum (low, high words) as fp32: exact enough, since the
// sum is < 2^56 and only fp32 precision is kept.  The empty asm keeps each
// word a 32-bit operand (otherwise the conversion is widened to a 64-bit one).
__device__ __forceinline__ float u64_to_float(uint2 x)
{
    uint32_t hi = x.y, lo = x.x;
    asm("" : "+v"(hi), "+v"(lo));
    return fmaf((float)hi, 4294967296.0f, (float)lo);
}

// Flush of the workgroup's rows, in three steps:
//  1. a row's fixed-point bins become floats in the skewed layout, in place,
//     by one wavefront from start to end: the float row starts where the
//     histogram row starts and never reaches past it, and a batch of eight
//     64-bin chunks is read before any float of it is written, while the
//     floats of chunks up to c end before the words of chunk c + 1 begin (a
//     wavefront's LDS operations run in order);
//  2. zeros around the bins;
//  3. the jitter for taps zero-padded to radius RM, in segments of 64 V
//     outputs: lane l of segment s takes the V consecutive outputs from
//     o0 = 64 V s + V l, reading its window of V + 2 RM words at compile-time
//     offsets from one address (nine words apart from its neighbours:
//     distinct banks); each output is sum_k g[k] H[t + RM - k], accumulated
//     by fma in increasing k, and a complete, 16-byte aligned lane writes its
//     V outputs as two 16-byte stores.
// With at least as many rows as wavefronts, wavefront w takes rows w,
// w + waves, ... through all three steps and waits on no other.  With fewer
// rows, the segments of step 3 are dealt to every wavefront after a barrier
// (a segment reads floats another wavefront wrote), so that the wavefronts
// without a row share the jitter; each output is computed the same way.

// Steps 1 and 2 for row j (bin i at logical word lead - off + i).
__device__ __forceinline__ void flush_convert(const FwdArgs& a, const Lds& L, int j, int Tl, int lead, int off,
                                              int np, int lane)
{
    const int nch = (Tl + 63) >> 6;
    const int d = lane - off;                   // logical word of bin 64 c + lane: lead + 64 c + d
    const int dp = d + floor_div8(d);
    float* Fr = reinterpret_cast<float*>(L.hist + (size_t)j * a.stride);
    const uint2* Hr = reinterpret_cast<const uint2*>(L.hist) + (size_t)j * a.stride;
    for (int c0 = 0; c0 < nch; c0 += 8) {
        uint2 x[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) x[b] = Hr[min((c0 + b) * 64 + lane, Tl - 1)];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int xb = lead + 64 * (c0 + b);
            if (c0 + b < nch && (c0 + b) * 64 + lane < Tl) Fr[xb + (xb >> 3) + dp] = u64_to_float(x[b]);
        }
    }
    for (int e = lane; e < np; e += 64) {
        const int x = e < lead - off ? e : e + Tl;
        Fr[x + (x >> 3)] = 0.f;
    }
}

// Step 3 for segment s of row j (output row `row` of the operator).
template <int RM>
__device__ __forceinline__ void flush_segment(const FwdArgs& a, const Lds& L, int j, long long row,
                                              const float (&g)[2 * RM + 1], int s, int lead, int nt, int o_last,
                                              int t0w, int lane)
{
    constexpr int V = kFlushV;
    constexpr int K = 2 * RM + 1;
    constexpr int W = V + 2 * RM;
    constexpr int B0 = -RM + floor_div8(-RM);   // physical offset of window word 0 from output o0
    const float* Fr = reinterpret_cast<const float*>(L.hist + (size_t)j * a.stride);
    const float gg = L.gg[j];
    const int o0 = s * 64 * V + lane * V;
    const int x0 = lead + min(o0, o_last);     // logical word of output o0, 8 | x0 (lanes past the end: the last window)
    const float* h = Fr + (x0 + (x0 >> 3)) + B0;
    float w[W];
#pragma unroll
    for (int q = 0; q < W; ++q) w[q] = h[(q - RM) + floor_div8(q - RM) - B0];
    float acc[V];
#pragma unroll
    for (int m = 0; m < V; ++m) {
        float sum = 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) sum = fmaf(g[k], w[m + 2 * RM - k], sum);
        acc[m] = sum * gg;
    }
    if (o0 >= nt) return;
    const size_t first = (size_t)row * (size_t)a.T + (size_t)(t0w + o0);
    __attribute__((address_space(1))) float* orow = gmem(a.out) + first;
    if (a.atomic_out) {
#pragma unroll
        for (int m = 0; m < V; ++m)
            if (o0 + m < nt) unsafeAtomicAdd((float*)(orow + m), acc[m]);
    } else if (o0 + V <= nt && (first & 3) == 0) {
        typedef float v4f __attribute__((ext_vector_type(4)));
        typedef __attribute__((address_space(1))) v4f gv4f;
        reinterpret_cast<gv4f*>(orow)[0] = v4f{acc[0], acc[1], acc[2], acc[3]};
        reinterpret_cast<gv4f*>(orow)[1] = v4f{acc[4], acc[5], acc[6], acc[7]};
    } else {
#pragma unroll
        for (int m = 0; m < V; ++m)
            if (o0 + m < nt) orow[m] = acc[m];
    }
}

template <int RM, int NS>
__device__ __forceinline__ void flush_rows(const FwdArgs& a, const Lds& L, int Tl, int hb, int t0w, int t1w)
{
    constexpr int V = kFlushV;
    constexpr int K = 2 * RM + 1;
    constexpr int n_waves = kBlock / 64;
    const int R = a.R;
    const int RMr = RM > 16 ? jitter_rm(R) : RM;   // the radius the host sized the rows for
    const int lead = flush_lead(RMr), Lr = flush_row_logical(Tl, RMr);
    const int off = t0w - hb;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float g[K];
    if (RM <= 16) {
        const int sh = RM - R;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float t = a.taps[min(max(k - sh, 0), 2 * R)];
            g[k] = (k >= sh && k - sh <= 2 * R) ? t : 0.f;
        }
    }
    const int nt = t1w - t0w;
    const int nseg = (nt + 64 * V - 1) / (64 * V);
    const int o_last = (nt - 1) & ~(V - 1);     // window of the lanes past the end (inside the row)
    const int np = Lr - Tl;
    if (RM <= 16 && NS < n_waves) {
        if (wave < NS && L.row[wave] >= 0) flush_convert(a, L, wave, Tl, lead, off, np, lane);
        __syncthreads();
        for (int it = wave; it < NS * nseg; it += n_waves) {
            const int j = it / nseg;
            const long long row = L.row[j];
            if (row >= 0) flush_segment<RM>(a, L, j, row, g, it - j * nseg, lead, nt, o_last, t0w, lane);
        }
        return;
    }
    for (int j = wave; j < NS; j += n_waves) {
        const long long row = L.row[j];
        if (row < 0) continue;
        flush_convert(a, L, j, Tl, lead, off, np, lane);
        if (RM > 16) {
            // wide kernels: one output per lane, generic tap loop
            const float* Fr = reinterpret_cast<const float*>(L.hist + (size_t)j * a.stride);
            const float gg = L.gg[j];
            for (int tt = lane; tt < nt; tt += 64) {
                float acc = 0.f;
                for (int i = 0; i <= 2 * R; ++i) {
                    const int x = lead + tt + R - i;    // H[t + R - i]
                    acc = fmaf(a.taps[i], Fr[x + (x >> 3)], acc);
                }
                acc *= gg;
                __attribute__((address_space(1))) float* out = gmem(a.out) + (size_t)row * (size_t)a.T + t0w + tt;
                if (a.atomic_out)
                    unsafeAtomicAdd((float*)out, acc);
                else
                    *out = acc;
            }
            continue;
        }
        for (int s = 0; s < nseg; ++s) flush_segment<RM>(a, L, j, row, g, s, lead, nt, o_last, t0w, lane);
    }
}

// Flush: histograms (fixed point in LDS) -> float rows -> Gaussian jitter ->
// output, after every pair of the workgroup has been added (the caller's
// barrier); one compiled radius per rounded jitter radius.
template <int NS>
__device__ __forceinline__ void flush(const FwdArgs& a, const Lds& L, int hb, int Tl, int t0w, int t1w)
{
    const int RM = jitter_rm(a.R);
    if (RM == 2) {
        flush_rows<2, NS>(a, L, Tl, hb, t0w, t1w);
    } else if (RM == 4) {
        flush_rows<4, NS>(a, L, Tl, hb, t0w, t1w);
    } else if (RM == 6) {
        flush_rows<6, NS>(a, L, Tl, hb, t0w, t1w);
    } else if (RM == 8) {
        flush_rows<8, NS>(a, L, Tl, hb, t0w, t1w);
    } else if (RM == 12) {
        flush_rows<12, NS>(a, L, Tl, hb, t0w, t1w);
    } else if (RM == 16) {
        flush_rows<16, NS>(a, L, Tl, hb, t0w, t1w);
    } else {
        flush_rows<17, NS>(a, L, Tl, hb, t0w, t1w);   // any radius past 16: the generic tap loop
    }
}

// ---------------------------------------------------------------------------
// The pair kernel.  Slot j of the workgroup: unit k = j / NH, then within the
// unit (laser l, column c, row r) with j % NH = (l * TX + c) * TY + r.
template <bool CONF, int TL, int TX, int TY, bool COS, bool WIN, bool PAIR>
__device__ __forceinline__ void forward_body(const FwdArgs& a, int block_id)
{
    constexpr int ND = TX * TY;
    constexpr int NH = TL * ND;
    constexpr int NU = PAIR ? 2 : 1;
    constexpr int NS = NU * NH;
    extern __shared__ __align__(16) unsigned char smem[];
    const Lds L = lds_layout(smem, NS, a.stride, a.q_cap);
    // The reads of the set-up first, so that their latencies overlap each
    // other, the LDS clear and the tables below.  The scalar arguments the
    // set-up uses are read together (one wait, where each use would otherwise
    // wait for its own read).  Then the count and, with one patch range (it
    // starts at record 0), the records of the wavefront's first chunk: a
    // wavefront's first two chunks are 2 w and 2 w + 1, the later ones come
    // from a counter in LDS.  The first chunk is read before the count is
    // known, so lanes past the capacity read the last slot and lanes past the
    // count are replaced by the stand-in record in the loop.  Last, the
    // summaries.
    asm volatile("" ::"s"(a.n_active), "s"(a.stats), "s"(a.patches), "s"(a.prep), "s"(a.n_cap), "s"(a.n_stats),
                 "s"(a.n_split), "s"(a.n_tw), "s"(a.tw), "s"(a.T), "s"(a.R), "s"(a.stride), "s"(a.q_cap),
                 "s"(a.tiles_x), "s"(a.tiles_y), "s"(a.plan), "s"(a.n_units));
    asm volatile("" ::"s"(a.rx.a0), "s"(a.rx.step), "s"(a.rx.n), "s"(a.ry.a0), "s"(a.ry.step), "s"(a.ry.n),
                 "s"(a.cx), "s"(a.cy), "s"(a.s), "s"(a.inv), "s"(a.delta));
    if (!CONF) asm volatile("" ::"s"(a.lx.a0), "s"(a.lx.step), "s"(a.lx.n), "s"(a.ly.a0), "s"(a.ly.step), "s"(a.ly.n));
    const int n_act = active_count(a);
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const bool prep = a.prep != nullptr;
    const float4* src = prep ? a.prep : a.patches;
    const bool early = a.n_split == 1 && a.n_cap > 0;
    float4 An = make_float4(0.f, 0.f, 0.f, 0.f), Bn = An;
    if (early) {
        const int pl = min(2 * wave * 64 + lane, a.n_cap - 1);
        load_record(src, pl, An, Bn);
    }
    // this thread's summary, read now and decoded where the bound needs it
    // (three words of the second half: the fourth is padding, and a dead
    // destination word of a read in flight invites a wait on its reuse)
    typedef int v4i __attribute__((ext_vector_type(4)));
    typedef int v3i __attribute__((ext_vector_type(3)));
    v4i st0a = {0, 0, 0, 0};
    v3i st0b = {0, 0, 0};
    if ((int)threadIdx.x < a.n_stats) {
        const __attribute__((address_space(1))) v4i* g = (const __attribute__((address_space(1))) v4i*)a.stats;
        st0a = g[2 * (size_t)threadIdx.x];
        st0b = *(const __attribute__((address_space(1))) v3i*)(g + 2 * (size_t)threadIdx.x + 1);
    }

    int id = block_id;
    const int split = id % a.n_split;
    id /= a.n_split;
    const int twi = id % a.n_tw;
    const int grp = id / a.n_tw;
    const int t0w = twi * a.tw, t1w = min(a.T, t0w + a.tw);
    const int hbw = max(0, t0w - a.R), hew = min(a.T, t1w + a.R);
    const int hb = WIN ? hbw : 0, Tl = WIN ? hew - hbw : a.T;
    const int chunk = (n_act + a.n_split - 1) / a.n_split;
    const int pb = min(n_act, split * chunk), pe = min(n_act, pb + chunk);
    const int n_laser = a.lx.n * a.ly.n;

    int unit[NU];
    pick_units<PAIR>(a, grp, unit);
    bool uvalid[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) uvalid[k] = unit[k] >= 0;
    int unit_on[NU];   // the same, made scalar for the pair loop's per-chunk test
#pragma unroll
    for (int k = 0; k < NU; ++k) unit_on[k] = __builtin_amdgcn_readfirstlane(unit[k] >= 0 ? 1 : 0);

    for (int i = threadIdx.x; i < NS * a.stride / 2; i += kBlock) reinterpret_cast<uint4*>(L.hist)[i] = uint4{0, 0, 0, 0};
    if (threadIdx.x == 0) *L.next = 2u * (kBlock / 64);
    if (threadIdx.x < NS) {
        const int j = threadIdx.x;
        const int k = j / NH, jl = j % NH;
        // (NU <= 2: selects, so that the small arrays stay in registers)
        const bool kv = k == 0 ? uvalid[0] : uvalid[NU - 1];
        const int u = kv ? (k == 0 ? unit[0] : unit[NU - 1]) : unit[0];
        const int uy = u % a.tiles_y, ux = (u / a.tiles_y) % a.tiles_x, ul = u / (a.tiles_y * a.tiles_x);
        const int dj = jl % ND;
        const int ix_u = ux * TX + dj / TY, iy_u = uy * TY + dj % TY, l_u = ul * TL + jl / ND;
        L.row[j] = (kv && ix_u < a.rx.n && iy_u < a.ry.n && l_u < (CONF ? 1 : n_laser))
                       ? ((long long)l_u * a.rx.n + ix_u) * a.ry.n + iy_u
                       : -1ll;
        const int ix = min(ix_u, a.rx.n - 1);
        const int iy = min(iy_u, a.ry.n - 1);
        const float wx = canon(a.rx, ix), wy = canon(a.ry, iy);
        double off_d, g_d;
        device_leg(wx, wy, a.cx, a.cy, a.s, &off_d, &g_d);
        L.wdx[j] = wx;
        L.wdy[j] = wy;
        if (CONF) {
            const double o = off_d + off_d;
            L.so[j] = o;
            L.wlx[j] = wx;
            L.wly[j] = wy;
            L.oil[j] = (float)(o * a.inv + (double)a.delta);
            L.gg[j] = (float)(g_d * g_d);
        } else {
            const int l = min(ul * TL + jl / ND, n_laser - 1);
            const float lx = canon(a.lx, l / a.ly.n), ly = canon(a.ly, l % a.ly.n);
            double off_l, g_l;
            device_leg(lx, ly, a.cx, a.cy, a.s, &off_l, &g_l);
            L.so[j] = off_l + off_d;
            L.wlx[j] = lx;
            L.wly[j] = ly;
            L.oil[j] = (float)(off_l * a.inv + (double)a.delta);
            L.oid[j] = (float)(off_d * a.inv);
            L.gg[j] = (float)(g_l * g_d);
        }
    }
    // weight bound of each unit over the record summaries -> its fixed-point
    // scale s_k = 2^31 / W_k, so that a unit of weak pairs keeps its
    // precision beside a strong one; the row gains take 1 / s_k, so rows come
    // out in the operator's units
    float wbk[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) wbk[k] = 0.f;
    for (int i = threadIdx.x; i < a.n_stats; i += kBlock) {
        const StatF c = i == (int)threadIdx.x ? decode_stat(st0a, v4i{st0b.x, st0b.y, st0b.z, 0}) : load_stat(a.stats, i);
#pragma unroll
        for (int k = 0; k < NU; ++k)
            if (uvalid[k]) wbk[k] = fmaxf(wbk[k], unit_weight_bound<CONF, TL, TX, TY>(a, unit[k], c));
    }
    block_max<NU>(wbk, L.red);   // includes a barrier: the tables above are visible
    float sk[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) sk[k] = wbk[k] > 0.f ? 2147483648.0f / wbk[k] : 1.0f;
    if (threadIdx.x < NS) L.gg[threadIdx.x] *= 1.0f / ((int)threadIdx.x < NH ? sk[0] : sk[NU - 1]);
    // the pair loop works in bins: coordinates times sig, so its weights
    // carry sig^-4, which the scale it applies takes back
    const float sig = CONF ? a.inv2_f : a.inv_f;
    const float s4 = (sig * sig) * (sig * sig);
#pragma unroll
    for (int k = 0; k < NU; ++k) sk[k] = fminf(sk[k] * s4, 3.0e38f);

    // per-unit wall points and bounds, wave-uniform
    float lxs[NU][TL], lys[NU][TL], oil[NU][TL], wx[NU][TX], wy[NU][TY], oi[NS];
    float lx0[NU], lx1[NU], ly0[NU], ly1[NU], x0[NU], x1[NU], y0[NU], y1[NU], omin[NU], omax[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        const int b = k * NH;
        lx0[k] = ly0[k] = x0[k] = y0[k] = omin[k] = 3.0e38f;
        lx1[k] = ly1[k] = x1[k] = y1[k] = -3.0e38f;
        omax[k] = 0.f;
#pragma unroll
        for (int l = 0; l < TL; ++l) {
            lxs[k][l] = uniform(L.wlx[b + l * ND] * sig);
            lys[k][l] = uniform(L.wly[b + l * ND] * sig);
            oil[k][l] = uniform(L.oil[b + l * ND]);
            lx0[k] = fminf(lx0[k], lxs[k][l]);
            lx1[k] = fmaxf(lx1[k], lxs[k][l]);
            ly0[k] = fminf(ly0[k], lys[k][l]);
            ly1[k] = fmaxf(ly1[k], lys[k][l]);
        }
#pragma unroll
        for (int c = 0; c < TX; ++c) {
            wx[k][c] = uniform(L.wdx[b + c * TY] * sig);
            x0[k] = fminf(x0[k], wx[k][c]);
            x1[k] = fmaxf(x1[k], wx[k][c]);
        }
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            wy[k][r] = uniform(L.wdy[b + r] * sig);
            y0[k] = fminf(y0[k], wy[k][r]);
            y1[k] = fmaxf(y1[k], wy[k][r]);
        }
#pragma unroll
        for (int jj = 0; jj < NH; ++jj) {
            // confocal: arrival offset per scan point; non-confocal: detector
            // offset (slots of laser 0 cover every detector point)
            oi[b + jj] = CONF ? L.oil[b + jj] : L.oid[b + jj];
            const float ov = CONF ? oi[b + jj] : oi[b + jj] + L.oil[b + jj];
            omin[k] = fminf(omin[k], ov);
            omax[k] = fmaxf(omax[k], ov);
        }
    }
    const float two_delta = a.two_delta;
    // a wavefront skips a unit when every arrival is at least 2 bins past the
    // window (the bound is exact up to fp32 rounding, far below 2 bins)
    const float cut_hi = (float)(hb + Tl + 2);
    const float cut_lo = (float)(hb - 2);
    float cut_r2[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        // squared distance (in bins) past which every confocal arrival is
        // beyond cut_hi, or (non-confocal) the square of the smallest sum of
        // the two wall-to-patch legs that puts it there (enlarged by 1e-5
        // relative: the fp32 squares and root round)
        const float rc = fmaxf(cut_hi - omin[k], 0.f);
        cut_r2[k] = rc * rc * 1.00001f;
    }

    const int qw = a.q_cap / kQueueWaves;
    int qn = 0;
    // Wavefronts take 64-record chunks from a counter in LDS, so they finish
    // together however unevenly culling thins the chunks.  A wavefront holds
    // two: the records of the next one are loaded while the current one is
    // evaluated, and the one after is claimed meanwhile.
    int n_eval = 0;   // pairs evaluated by this wavefront (counted only on request)
    int chunk_id = __builtin_amdgcn_readfirstlane(2 * wave);
    int next_id = chunk_id + 1;
    // records as written by the geometry, or (prep) their pair-loop
    // constants, which the one-call path writes beside them
    if (!early && pb + chunk_id * 64 < pe) {
        const int pl = min(pb + chunk_id * 64 + lane, pe - 1);
        load_record(src, pl, An, Bn);
    }
    for (;;) {
        const int base = pb + chunk_id * 64;
        if (base >= pe) break;
        // lanes past the range take a stand-in record at x = dummy_x with
        // zero weight: every arrival of that position lies past the window
        const int p = base + lane;
        // (only the last chunk has lanes past the range: a wave-uniform test
        // keeps the selects off every other chunk)
        if (base + 64 > pe && p >= pe) {
            if (prep) {
                An = make_float4(a.dummy_x, 0.f, 1.f, 0.f);
                Bn = make_float4(0.f, 0.f, 0.f, 0.f);
            } else {
                An = make_float4(a.dummy_x, 0.f, 1.f, 0.f);
                Bn = make_float4(0.f, 0.f, -1.f, 0.f);
            }
        }
        PatchC pc;
        float aw;
        if (prep) {
            // the coordinates in bins, as patch_consts_scaled computes them
            pc.px = An.x * sig;
            pc.py = An.y * sig;
            const float pzs = An.z * sig;
            pc.pz2 = pzs * pzs;
            pc.ap = An.w;
            pc.mnxs = Bn.x;
            pc.mnys = Bn.y;
            pc.c0s = Bn.z;
            aw = An.w;
        } else {
            pc = patch_consts_scaled(An, Bn, COS, sig);
            aw = An.w;
        }
        // records of the next chunk, into the registers the current ones
        // have just left (past the range: the last record, never used)
        {
            const int pl = min(pb + next_id * 64 + lane, pe - 1);
            load_record(src, pl, An, Bn);
        }
        int claim = 0;
        if (lane == 0) claim = (int)atomicAdd(L.next, 1u);
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            if (unit_on[k] == 0) continue;
            {
                bool out;
                if (CONF) {
                    out = rect_r2_min(pc.px, pc.py, pc.pz2, x0[k], x1[k], y0[k], y1[k]) >= cut_r2[k];
                } else {
                    // (r_l + r_d)^2 = r_l^2 + r_d^2 + 2 sqrt(r_l^2 r_d^2): one root
                    const float dd = rect_r2_min(pc.px, pc.py, pc.pz2, x0[k], x1[k], y0[k], y1[k]);
                    const float dl = rect_r2_min(pc.px, pc.py, pc.pz2, lx0[k], lx1[k], ly0[k], ly1[k]);
                    out = fmaf(2.f, __builtin_amdgcn_sqrtf(dd * dl), dd + dl) >= cut_r2[k];
                }
                if (WIN) {
                    const float Rd = __builtin_amdgcn_sqrtf(rect_r2_max(pc.px, pc.py, pc.pz2, x0[k], x1[k], y0[k], y1[k]));
                    const float Rl = CONF ? Rd
                                          : __builtin_amdgcn_sqrtf(
                                                rect_r2_max(pc.px, pc.py, pc.pz2, lx0[k], lx1[k], ly0[k], ly1[k]));
                    out = out || (Rl + Rd) + omax[k] < cut_lo;
                }
                if (__all(out)) continue;
            }
            n_eval += min(64, pe - base) * NH;
            const int b = k * NH;
            float cx2[TX], axv[TX], cy2[TY], byv[TY];
            if (CONF) {
                const float aps = (COS ? pc.ap : aw) * sk[k];
#pragma unroll
                for (int c = 0; c < TX; ++c) col_terms(pc, wx[k][c], &cx2[c], &axv[c]);
#pragma unroll
                for (int r = 0; r < TY; ++r) row_terms(pc, wy[k][r], &cy2[r], &byv[r]);
#pragma unroll
                for (int c = 0; c < TX; ++c) {
#pragma unroll
                    for (int r = 0; r < TY; ++r) {
                        const int j = b + c * TY + r;
                        const Leg lg = leg_eval_at(cx2[c], cy2[r], axv[c], byv[r], oi[j], COS);
                        const float w = lg.rr;
                        const Decision d = decide(w, two_delta);
                        const uint32_t inc = (uint32_t)fmaf(COS ? lg.q * lg.q : lg.ri4, aps, 0.5f);
                        const int kl = d.k - hb;
                        // bins 0 .. Tl exist (Tl: a spare past the window, never
                        // flushed); lane masks are taken before the divergent add
                        const uint64_t m_unsure = __builtin_amdgcn_ballot_w64((unsigned)kl <= (unsigned)Tl) &
                                                  ~__builtin_amdgcn_ballot_w64(d.sure);
                        if ((unsigned)kl <= (unsigned)Tl) lds_add(L.hist + j * a.stride + kl, inc);
                        guard_push(L, a, m_unsure, p, j, kl, inc, hb, Tl, wave, qw, qn);
                    }
                }
            } else {
                // laser legs
                float ul[TL], fl[TL];
#pragma unroll
                for (int l = 0; l < TL; ++l) {
                    float lcx2, lax, lcy2, lby;
                    col_terms(pc, lxs[k][l], &lcx2, &lax);
                    row_terms(pc, lys[k][l], &lcy2, &lby);
                    const Leg lg = leg_eval_at(lcx2, lcy2, lax, lby, oil[k][l], COS);
                    ul[l] = lg.rr;
                    fl[l] = (COS ? lg.q * pc.ap : lg.ri2 * aw) * sk[k];
                }
#pragma unroll
                for (int c = 0; c < TX; ++c) col_terms(pc, wx[k][c], &cx2[c], &axv[c]);
#pragma unroll
                for (int r = 0; r < TY; ++r) row_terms(pc, wy[k][r], &cy2[r], &byv[r]);
#pragma unroll
                for (int c = 0; c < TX; ++c) {
#pragma unroll
                    for (int r = 0; r < TY; ++r) {
                        const int dj = c * TY + r;
                        const Leg lg = leg_eval_at(cx2[c], cy2[r], axv[c], byv[r], oi[b + dj], COS);
                        const float ud = lg.rr;
                        const float fd = COS ? lg.q : lg.ri2;
#pragma unroll
                        for (int l = 0; l < TL; ++l) {
                            const int j = b + l * ND + dj;
                            const float w = ul[l] + ud;
                            const Decision d = decide(w, two_delta);
                            const uint32_t inc = (uint32_t)fmaf(fl[l], fd, 0.5f);
                            const int kl = d.k - hb;
                            const uint64_t m_unsure = __builtin_amdgcn_ballot_w64((unsigned)kl <= (unsigned)Tl) &
                                                      ~__builtin_amdgcn_ballot_w64(d.sure);
                            if ((unsigned)kl <= (unsigned)Tl) lds_add(L.hist + j * a.stride + kl, inc);
                            guard_push(L, a, m_unsure, p, j, kl, inc, hb, Tl, wave, qw, qn);
                        }
                    }
                }
            }
        }
        chunk_id = next_id;
        next_id = __builtin_amdgcn_readfirstlane(claim);
    }
    guard_drain<CONF>(L, a, hb, Tl, wave, qw, qn);
    if (a.eval_pairs && lane == 0) atomicAdd(a.eval_pairs, (unsigned long long)n_eval);
    __syncthreads();
    flush<NS>(a, L, hb, Tl, t0w, t1w);
}

template <bool CONF, int TL, int TX, int TY, bool COS, bool WIN, bool PAIR>
__global__ void __launch_bounds__(kBlock) k_forward(const FwdArgs a)
{
    forward_body<CONF, TL, TX, TY, COS, WIN, PAIR>(a, (int)blockIdx.x);
}

// Request of workgroup `block` in a batch: the last i with first[i] <= block
// (first[] ascending, first[0] = 0); uniform across the workgroup.
__device__ __forceinline__ int batch_slot(const int64_t* first, int n, int64_t block)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= block) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Batched pair kernel: one launch over the workgroups of every request of one
// kernel variant, requests ordered by decreasing work per workgroup.
// The table is a separate restrict-qualified argument: nothing the kernel
// stores can alias it, so its fields are read once with scalar loads.
template <bool CONF, int TL, int TX, int TY, bool COS, bool WIN, bool PAIR>
__global__ void __launch_bounds__(kBlock)
    k_forward_batch(const FwdArgs* __restrict__ tab, const int32_t* __restrict__ req,
                    const int64_t* __restrict__ first, int n)
{
    const int i = batch_slot(first, n, (int64_t)blockIdx.x);
    const FwdArgs& a = tab[req[i]];
    forward_body<CONF, TL, TX, TY, COS, WIN, PAIR>(a, (int)((int64_t)blockIdx.x - first[i]));
}

// ---------------------------------------------------------------------------
// Serving tick, pairs: one workgroup per (request, workgroup) item of the
// tick's list; the workgroup runs its request's variant of the pair kernel.
// (A persistent loop over claimed items keeps state live across items and
// spills.)
int tick_variant(int tx, int ty, bool cosines)
{
    int s = -1;
    if (tx == 4 && ty == 4) s = 0;
    else if (tx == 4 && ty == 2) s = 1;
    else if (tx == 2 && ty == 2) s = 2;
    else if (tx == 2 && ty == 1) s = 3;
    else if (tx == 1 && ty == 1) s = 4;
    return s < 0 ? -1 : s + (cosines ? 0 : kTickShapes);
}

// The list's arrays are restrict-qualified arguments (fixed addresses in the
// tick's workspace): nothing the kernel stores can alias them, so the
// request's arguments are read once with scalar loads.
__global__ void __launch_bounds__(kBlock)
    k_tick_pairs(const TickList* __restrict__ L, const FwdArgs* __restrict__ fwd,
                 const int32_t* __restrict__ variant, const int64_t* __restrict__ ffirst)
{
    const int n = L->n;
    const int64_t t = (int64_t)blockIdx.x;
    if (n <= 0 || t >= ffirst[n]) return;
    const int i = batch_slot(ffirst, n, t);
    const FwdArgs& a = fwd[i];
    const int blk = (int)(t - ffirst[i]);
    switch (variant[i]) {
    case 0: forward_body<true, 1, 4, 4, true, false, true>(a, blk); break;
    case 1: forward_body<true, 1, 4, 2, true, false, true>(a, blk); break;
    case 2: forward_body<true, 1, 2, 2, true, false, true>(a, blk); break;
    case 3: forward_body<true, 1, 2, 1, true, false, true>(a, blk); break;
    case 4: forward_body<true, 1, 1, 1, true, false, true>(a, blk); break;
    case 5: forward_body<true, 1, 4, 4, false, false, true>(a, blk); break;
    case 6: forward_body<true, 1, 4, 2, false, false, true>(a, blk); break;
    case 7: forward_body<true, 1, 2, 2, false, false, true>(a, blk); break;
    case 8: forward_body<true, 1, 2, 1, false, false, true>(a, blk); break;
    case 9: forward_body<true, 1, 1, 1, false, false, true>(a, blk); break;
    default: break;
    }
}

const void* tick_pairs_kernel() { return (const void*)k_tick_pairs; }

hipError_t prepare_tick_pairs(size_t lds_bytes)
{
    return hipFuncSetAttribute((const void*)k_tick_pairs, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t launch_tick_pairs(const TickArrays& t, int64_t grid, size_t lds_bytes, hipStream_t st)
{
    hipError_t e = prepare_tick_pairs(lds_bytes);
    if (e != hipSuccess) return e;
    if (grid < 1 || grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tick_pairs, dim3((unsigned)grid), dim3(kBlock), lds_bytes, st, t.list, t.fwd, t.variant,
                       t.ffirst);
    return hipGetLastError();
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
        const float sig = d.confocal ? a.inv2_f : a.inv_f;
        const PatchC pc = patch_consts_scaled(A, B, a.cosines != 0, sig);
        double off_l, g_l, off_d, g_d;
        device_leg(lx, ly, a.cx, a.cy, a.s, &off_l, &g_l);
        device_leg(wx, wy, a.cx, a.cy, a.s, &off_d, &g_d);
        const double o = off_l + off_d;
        float w;
        if (d.confocal) {
            const float oi = (float)(o * a.inv + (double)a.delta);
            float cx2, axv, cy2, byv;
            col_terms(pc, wx * sig, &cx2, &axv);
            row_terms(pc, wy * sig, &cy2, &byv);
            w = leg_eval_at(cx2, cy2, axv, byv, oi, a.cosines != 0).rr;
        } else {
            const float oil = (float)(off_l * a.inv + (double)a.delta);
            const float oid = (float)(off_d * a.inv);
            float cx2, axv, cy2, byv;
            col_terms(pc, lx * sig, &cx2, &axv);
            row_terms(pc, ly * sig, &cy2, &byv);
            const Leg ll = leg_eval_at(cx2, cy2, axv, byv, oil, a.cosines != 0);
            col_terms(pc, wx * sig, &cx2, &axv);
            row_terms(pc, wy * sig, &cy2, &byv);
            const Leg ld = leg_eval_at(cx2, cy2, axv, byv, oid, a.cosines != 0);
            w = ll.rr + ld.rr;
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

__global__ void __launch_bounds__(kStatBlock) k_chunk_stats_batch(const BatchList b)
{
    const int i = batch_slot(b.first, b.n, (int64_t)blockIdx.x);
    const FwdArgs& a = b.tab[b.req[i]];
    chunk_stats_body(a, a.stats, (int)((int64_t)blockIdx.x - b.first[i]));
}

// Zero the outputs of the listed requests (those accumulated with atomics):
// blockIdx.y selects the entry, kFillBlocksPerRequest blocks stride over it.
__global__ void __launch_bounds__(256) k_fill_batch(const BatchList b)
{
    const FwdArgs& a = b.tab[b.req[blockIdx.y]];
    const size_t n = (size_t)a.out_len;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a.out[i] = 0.f;
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

template <bool CONF, int TL, int TX, int TY>
static hipError_t launch_shape(const FwdArgs& a, const Plan& plan, hipStream_t st)
{
    if (plan.pair) {
        return a.cosines ? launch_k(k_forward<CONF, TL, TX, TY, true, false, true>, a, plan, st)
                         : launch_k(k_forward<CONF, TL, TX, TY, false, false, true>, a, plan, st);
    }
    return a.cosines ? launch_k(k_forward<CONF, TL, TX, TY, true, true, false>, a, plan, st)
                     : launch_k(k_forward<CONF, TL, TX, TY, false, true, false>, a, plan, st);
}

bool tile_supported(bool confocal, int tx, int ty, int tl)
{
    if (confocal) {
        return tl == 1 && ((tx == 4 && ty == 4) || (tx == 4 && ty == 2) || (tx == 2 && ty == 2) ||
                           (tx == 2 && ty == 1) || (tx == 1 && ty == 1));
    }
    return (tl == 2 && tx == 2 && ty == 2) || (tl == 2 && tx == 1 && ty == 2) ||
           (tl == 1 && tx == 1 && ty == 2) || (tl == 1 && tx == 1 && ty == 1);
}

hipError_t launch_forward(const FwdArgs& a, const Plan& plan, bool confocal, hipStream_t st)
{
    if (plan.n_blocks <= 0) return hipSuccess;
    if (confocal) {
        if (plan.tx == 4 && plan.ty == 4) return launch_shape<true, 1, 4, 4>(a, plan, st);
        if (plan.tx == 4 && plan.ty == 2) return launch_shape<true, 1, 4, 2>(a, plan, st);
        if (plan.tx == 2 && plan.ty == 2) return launch_shape<true, 1, 2, 2>(a, plan, st);
        if (plan.tx == 2 && plan.ty == 1) return launch_shape<true, 1, 2, 1>(a, plan, st);
        if (plan.tx == 1 && plan.ty == 1) return launch_shape<true, 1, 1, 1>(a, plan, st);
    } else {
        if (plan.tl == 2 && plan.tx == 2 && plan.ty == 2) return launch_shape<false, 2, 2, 2>(a, plan, st);
        if (plan.tl == 2 && plan.tx == 1 && plan.ty == 2) return launch_shape<false, 2, 1, 2>(a, plan, st);
        if (plan.tl == 1 && plan.tx == 1 && plan.ty == 2) return launch_shape<false, 1, 1, 2>(a, plan, st);
        if (plan.tl == 1 && plan.tx == 1 && plan.ty == 1) return launch_shape<false, 1, 1, 1>(a, plan, st);
    }
    return hipErrorInvalidValue;
}

template <typename K>
static hipError_t launch_kb(K kern, const BatchList& b, int64_t n_blocks, size_t lds_bytes, hipStream_t st)
{
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)n_blocks), dim3(kBlock), lds_bytes, st, b.tab, b.req, b.first, b.n);
    return hipGetLastError();
}

template <bool CONF, int TL, int TX, int TY>
static hipError_t launch_shape_batch(const BatchList& b, int64_t n_blocks, size_t lds, bool cos, bool pair,
                                     hipStream_t st)
{
    if (pair) {
        return cos ? launch_kb(k_forward_batch<CONF, TL, TX, TY, true, false, true>, b, n_blocks, lds, st)
                   : launch_kb(k_forward_batch<CONF, TL, TX, TY, false, false, true>, b, n_blocks, lds, st);
    }
    return cos ? launch_kb(k_forward_batch<CONF, TL, TX, TY, true, true, false>, b, n_blocks, lds, st)
               : launch_kb(k_forward_batch<CONF, TL, TX, TY, false, true, false>, b, n_blocks, lds, st);
}

hipError_t launch_forward_batch(const BatchList& b, int64_t n_blocks, size_t lds, int tl, int tx, int ty,
                                bool confocal, bool cos, bool pair, hipStream_t st)
{
    if (n_blocks <= 0) return hipSuccess;
    if (n_blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (confocal) {
        if (tx == 4 && ty == 4) return launch_shape_batch<true, 1, 4, 4>(b, n_blocks, lds, cos, pair, st);
        if (tx == 4 && ty == 2) return launch_shape_batch<true, 1, 4, 2>(b, n_blocks, lds, cos, pair, st);
        if (tx == 2 && ty == 2) return launch_shape_batch<true, 1, 2, 2>(b, n_blocks, lds, cos, pair, st);
        if (tx == 2 && ty == 1) return launch_shape_batch<true, 1, 2, 1>(b, n_blocks, lds, cos, pair, st);
        if (tx == 1 && ty == 1) return launch_shape_batch<true, 1, 1, 1>(b, n_blocks, lds, cos, pair, st);
    } else {
        if (tl == 2 && tx == 2 && ty == 2) return launch_shape_batch<false, 2, 2, 2>(b, n_blocks, lds, cos, pair, st);
        if (tl == 2 && tx == 1 && ty == 2) return launch_shape_batch<false, 2, 1, 2>(b, n_blocks, lds, cos, pair, st);
        if (tl == 1 && tx == 1 && ty == 2) return launch_shape_batch<false, 1, 1, 2>(b, n_blocks, lds, cos, pair, st);
        if (tl == 1 && tx == 1 && ty == 1) return launch_shape_batch<false, 1, 1, 1>(b, n_blocks, lds, cos, pair, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_stats_batch(const BatchList& b, int64_t n_blocks, hipStream_t st)
{
    if (n_blocks <= 0) return hipSuccess;
    if (n_blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chunk_stats_batch, dim3((unsigned)n_blocks), dim3(kStatBlock), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_fill_batch(const BatchList& b, hipStream_t st)
{
    if (b.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_batch, dim3(kFillBlocksPerRequest, (unsigned)b.n), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_stats(const FwdArgs& a, ChunkStat* stats, hipStream_t st)
{
    if (a.n_stats <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_stats, dim3((unsigned)a.n_stats), dim3(kStatBlock), 0, st, a, stats);
    return hipGetLastError();
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
