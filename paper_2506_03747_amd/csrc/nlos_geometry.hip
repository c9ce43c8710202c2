// Depth map (+ albedo, + mask) -> patch records (Section 2 depth-to-volume
// mapping; Algorithm 1 step 2.1), gfx950.
//
// Three launches, no host synchronisation:
//   1. count:   present pixels per block of the record enumeration order;
//   2. scan:    one workgroup turns the block counts into offsets and writes
//               the number of present patches;
//   3. scatter: each present pixel computes its record (canonical position,
//               normal from central differences, albedo * area) and writes it
//               at offset + rank within the block (wave ballots).
// Enumeration order: 16x16-pixel blocks (x major over blocks), each split
// into 4 phases (ix mod 2, iy mod 2) of 8x8 pixels at stride 2.  A wavefront
// of 64 consecutive records then covers one small square of the surface (so a
// whole wavefront can be culled against a scan tile) while neighbouring lanes
// sit 2 pixels apart (so their arrivals fall in fewer common bins).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nlos_device.h"
#include "nlos_internal.h"

namespace nlos {

__device__ __forceinline__ bool enum_pixel(const GeomArgs& a, int64_t e, int* ix, int* iy)
{
    if (e >= a.n_enum) return false;
    const int64_t chunk = e >> 6;
    const int w = (int)(e & 63);
    const int phase = (int)(chunk & 3);
    const int64_t blk = chunk >> 2;
    const int bxi = (int)(blk / a.by), byi = (int)(blk % a.by);
    *ix = bxi * kBlockPx + (w >> 3) * 2 + (phase >> 1);
    *iy = byi * kBlockPx + (w & 7) * 2 + (phase & 1);
    return *ix < a.ax.n && *iy < a.ay.n;
}

// The samples of map index idx, read together before any is used (where an
// albedo or mask map is absent, its read goes to the depth map and is not
// used), and whether they make a present pixel.
struct Samples {
    float z, rho;
    bool m;
};

__device__ __forceinline__ Samples read_samples(const GeomArgs& a, int64_t idx)
{
    const float* al = a.albedo ? a.albedo : a.depth;
    const uint8_t* mk = a.mask ? a.mask : reinterpret_cast<const uint8_t*>(a.depth);
    const float z = a.depth[idx], r = al[idx];
    const uint8_t m = mk[idx];
    return Samples{z, a.albedo ? r : 0.5f, a.mask ? m != 0 : true};
}

__device__ __forceinline__ bool is_present(const Samples& s)
{
    return s.m && s.rho > 0.f && isfinite(s.z) && s.z > 0.f;
}

__device__ __forceinline__ void count_body(const GeomArgs& a, int blk)
{
    __shared__ int wave_cnt[kGeomBlock / 64];
    const int64_t e = (int64_t)blk * kGeomBlock + threadIdx.x;
    int ix = 0, iy = 0;
    const bool in_map = enum_pixel(a, e, &ix, &iy);
    // (lanes without a pixel read index 0 of the map and use nothing)
    const Samples smp = read_samples(a, in_map ? (int64_t)ix * a.ay.n + iy : 0);
    // (every sample taken, so that no read waits for the mask's or albedo's
    // value before it is issued)
    asm volatile("" ::"v"(smp.z), "v"(smp.rho), "v"((int)smp.m));
    const bool p = in_map && is_present(smp);
    const unsigned long long bal = __ballot(p);
    if ((threadIdx.x & 63) == 0) wave_cnt[threadIdx.x >> 6] = (int)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        int cnt = 0;
#pragma unroll
        for (int w = 0; w < kGeomBlock / 64; ++w) cnt += wave_cnt[w];
        a.counts[blk] = cnt;
    }
    // empty record summaries for the scatter to merge into: block b clears
    // kGeomBlock / kStatBlock of them (the blocks cover n_enum >= n_stats * kStatBlock
    // pixels, so every summary is cleared before the scatter launch)
    constexpr int kPer = kGeomBlock / kStatBlock;
    if (a.stats && threadIdx.x < kPer * 8) {
        const int i = blk * kPer + (int)threadIdx.x / 8, f = (int)threadIdx.x % 8;
        if (i < a.n_stats) {
            // x0, x1, y0, y1, z0, amax, count, pad: min fields start high, max fields low
            const int v = (f >= 6) ? 0 : ((f == 0 || f == 2 || f == 4) ? INT32_MAX : INT32_MIN);
            reinterpret_cast<int32_t*>(a.stats + i)[f] = v;
        }
    }
}

__global__ void __launch_bounds__(kGeomBlock) k_geom_count(const GeomArgs a) { count_body(a, (int)blockIdx.x); }

__device__ __forceinline__ void scan_body(const GeomArgs& a)
{
    __shared__ int part[1024];
    const int n = a.n_blocks;
    const int per = (n + 1023) / 1024;
    const int b0 = min(n, (int)threadIdx.x * per), b1 = min(n, b0 + per);
    int s = 0;
    for (int i = b0; i < b1; ++i) s += a.counts[i];
    part[threadIdx.x] = s;
    __syncthreads();
    // inclusive Hillis-Steele scan over the 1024 partial sums
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = part[threadIdx.x] - s;
    for (int i = b0; i < b1; ++i) {
        a.offsets[i] = run;
        run += a.counts[i];
    }
    if (threadIdx.x == 1023) *a.n_active = part[1023];
}

__global__ void __launch_bounds__(1024) k_geom_scan(const GeomArgs a) { scan_body(a); }

// Records of one enumeration block at base + (rank among the present pixels
// before it).  base is the exclusive prefix of the block counts: read from
// `offsets`, or (offsets null) summed here from the counts.  With `stats`,
// the block also merges its records into the summaries of kStatBlock
// consecutive records (cleared by the count pass).
__device__ __forceinline__ void scatter_body(const GeomArgs& a, int blk)
{
    __shared__ int wave_cnt[kGeomBlock / 64];
    __shared__ int red[kGeomBlock / 64];
    const int64_t e = (int64_t)blk * kGeomBlock + threadIdx.x;
    int ix = 0, iy = 0;
    const bool in_map = enum_pixel(a, e, &ix, &iy);
    const int64_t idx = (int64_t)ix * a.ay.n + iy;
    // every global read of the block is issued before any of them is used
    // (the counts of the blocks before this one, the pixel, its neighbours),
    // so that their latencies overlap
    // (lanes without a pixel read index 0 of the map and use nothing; the
    // counts past the first kGeomBlock blocks are read last)
    int sum = 0;
    if (a.offsets)
        sum = threadIdx.x == 0 ? a.offsets[blk] : 0;
    else
        sum = (int)threadIdx.x < blk ? a.counts[threadIdx.x] : 0;
    const int64_t ci = in_map ? idx : 0;
    const Samples smp = read_samples(a, ci);
    // neighbours for the normal (the sample itself where the one-sided
    // difference does not use one)
    const float* D = a.depth + ci;
    const int64_t dxp = in_map && ix + 1 < a.ax.n ? (int64_t)a.ay.n : 0;
    const int64_t dxm = in_map && ix > 0 ? -(int64_t)a.ay.n : 0;
    const int dyp = in_map && iy + 1 < a.ay.n ? 1 : 0;
    const int dym = in_map && iy > 0 ? -1 : 0;
    const float zxp = D[dxp], zxm = D[dxm], zyp = D[dyp], zym = D[dym];
    if (!a.offsets)
        for (int i = (int)threadIdx.x + kGeomBlock; i < blk; i += kGeomBlock) sum += a.counts[i];
    const float z = smp.z, rho = smp.rho;
    const bool p = in_map && is_present(smp);
    const unsigned long long bal = __ballot(p);
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const int rank = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_cnt[wave] = __popcll(bal);
    sum = wave_reduce_i<2>(sum);
    if (lane == 0) red[wave] = sum;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < kGeomBlock / 64; ++w) base += red[w];
    int off = base + rank;
    for (int w = 0; w < wave; ++w) off += wave_cnt[w];
    if (!a.offsets && blk == a.n_blocks - 1 && threadIdx.x == 0) {
        int tot = base;
        for (int w = 0; w < kGeomBlock / 64; ++w) tot += wave_cnt[w];
        *a.n_active = tot;
    }

    float4 A = make_float4(0.f, 0.f, 0.f, 0.f);
    if (p) {
        // central differences inside, one-sided at the borders, 0 for a
        // single sample (the same operations as before the reads moved up)
        const float gx = a.ax.n < 2 ? 0.f
                         : ix == 0 ? (zxp - z) / a.hx
                         : ix == a.ax.n - 1 ? (z - zxm) / a.hx
                         : (zxp - zxm) / (2.f * a.hx);
        const float gy = a.ay.n < 2 ? 0.f
                         : iy == 0 ? (zyp - z) / a.hy
                         : iy == a.ay.n - 1 ? (z - zym) / a.hy
                         : (zyp - zym) / (2.f * a.hy);
        const float len = sqrtf(1.f + gx * gx + gy * gy);
        const float area = a.hx * a.hy * (a.cosines ? len : 1.f);
        A = make_float4(canon(a.ax, ix), canon(a.ay, iy), z, rho * area);
        const float4 B = make_float4(gx / len, gy / len, -1.f / len, __int_as_float((int)idx));
        a.patches[2 * (int64_t)off] = A;
        a.patches[2 * (int64_t)off + 1] = B;
        if (a.prep) {
            // the constants the pair loop derives from this record, by the
            // same function, so that it need not derive them per chunk; the
            // coordinates stay unscaled (the loop scales them per chunk, and
            // the fp64 re-binning of guard-band pairs needs them as recorded)
            const PatchC pc = patch_consts_scaled(A, B, a.cosines != 0, a.prep_sig);
            a.prep[2 * (int64_t)off] = make_float4(A.x, A.y, A.z, pc.ap);
            a.prep[2 * (int64_t)off + 1] = make_float4(pc.mnxs, pc.mnys, pc.c0s, 0.f);
        }
    }
    if (!a.stats) return;   // uniform across the block

    // Record summaries, one per kStatBlock consecutive records.  The block's
    // records are consecutive, [base, base + n), with n <= kStatBlock, so
    // they meet at most two summaries, cb and cb + 1 (sides 0 and 1).  Each
    // wavefront reduces its lanes of each side it has, the block combines
    // its wavefronts' values in LDS, and 14 lanes merge the two sides' seven
    // fields into the summaries with integer atomics on the order-preserving
    // images (min and max commute, so the result does not depend on the
    // order of the merges).
    static_assert(kGeomBlock <= kStatBlock, "a block's records meet at most two summaries");
    __shared__ int part[kGeomBlock / 64][2][7];
    const int cb = base / kStatBlock;
    const int side = off / kStatBlock - cb;   // 0 or 1 where p
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        const bool in = p && side == sd;
        const unsigned long long m = __ballot(in);
        int v[7] = {INT32_MAX, INT32_MIN, INT32_MAX, INT32_MIN, INT32_MAX, INT32_MIN, (int)__popcll(m)};
        if (m != 0ull) {   // uniform
            v[0] = wave_reduce_i<0>(in ? ord_f(A.x) : INT32_MAX);
            v[1] = wave_reduce_i<1>(in ? ord_f(A.x) : INT32_MIN);
            v[2] = wave_reduce_i<0>(in ? ord_f(A.y) : INT32_MAX);
            v[3] = wave_reduce_i<1>(in ? ord_f(A.y) : INT32_MIN);
            v[4] = wave_reduce_i<0>(in ? ord_f(A.z) : INT32_MAX);
            v[5] = wave_reduce_i<1>(in ? ord_f(A.w) : INT32_MIN);
        }
        if (lane < 7) {
            int x = v[0];
#pragma unroll
            for (int f = 1; f < 7; ++f) x = lane == f ? v[f] : x;
            part[wave][sd][lane] = x;
        }
    }
    __syncthreads();
    if (threadIdx.x < 14) {
        const int sd = (int)threadIdx.x / 7, f = (int)threadIdx.x % 7;
        int x = part[0][sd][f], cnt = part[0][sd][6];
#pragma unroll
        for (int w = 1; w < kGeomBlock / 64; ++w) {
            const int y = part[w][sd][f];
            x = f == 6 ? x + y : ((f & 1) ? max(x, y) : min(x, y));
            cnt += part[w][sd][6];
        }
        const int c = cb + sd;
        if (cnt > 0 && c < a.n_stats) {
            // fields x0, x1, y0, y1, z0, amax, count: minima at even f < 6
            int32_t* t = reinterpret_cast<int32_t*>(a.stats + c) + f;
            if (f == 6)
                atomicAdd(t, x);
            else if (f & 1)
                atomicMax(t, x);
            else
                atomicMin(t, x);
        }
    }
}

__global__ void __launch_bounds__(kGeomBlock) k_geom_scatter(const GeomArgs a) { scatter_body(a, (int)blockIdx.x); }

// Batched geometry: the enumeration blocks of all depth maps in one launch
// per phase (count, scan with one workgroup per map, scatter).
__device__ __forceinline__ int geom_slot(const GeomList& g, int64_t block)
{
    int lo = 0, hi = g.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.first[mid] <= block) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(kGeomBlock) k_geom_count_batch(const GeomList g)
{
    const int i = geom_slot(g, (int64_t)blockIdx.x);
    count_body(g.tab[i], (int)((int64_t)blockIdx.x - g.first[i]));
}

__global__ void __launch_bounds__(1024) k_geom_scan_batch(const GeomList g)
{
    if (g.tab[blockIdx.x].offsets) scan_body(g.tab[blockIdx.x]);
}

__global__ void __launch_bounds__(kGeomBlock) k_geom_scatter_batch(const GeomList g)
{
    const int i = geom_slot(g, (int64_t)blockIdx.x);
    scatter_body(g.tab[i], (int)((int64_t)blockIdx.x - g.first[i]));
}

// ---------------------------------------------------------------------------
// Serving tick, geometry: persistent workgroups take the items of a pass in
// a fixed stride (item t goes to workgroup t mod grid; the items are
// 256-pixel blocks of equal cost, and a shared ticket counter would make
// every claim a contended atomic).  Count pass items: every enumeration
// block of every map, then the zero-fill of the outputs that take float
// atomics; scatter pass items: every block again (a map's scatter reads the
// counts of its blocks before it, all written by the count pass).  No item
// waits for another.
__device__ __forceinline__ int tick_slot(const int64_t* first, int n, int64_t t)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(kGeomBlock) k_tick_count(const TickList* __restrict__ L)
{
    const int n = L->n;
    if (n <= 0) return;
    const int64_t g_total = L->gfirst[n], z_total = L->zfirst[n];
    for (int64_t t = blockIdx.x; t < g_total + z_total; t += gridDim.x) {
        if (t < g_total) {
            const int i = tick_slot(L->gfirst, n, t);
            count_body(L->geom[i], (int)(t - L->gfirst[i]));
        } else {
            const int64_t tz = t - g_total;
            const int i = tick_slot(L->zfirst, n, tz);
            const FwdArgs& a = L->fwd[i];
            const int64_t b0 = (tz - L->zfirst[i]) * kTickFillFloats;
            const int64_t b1 = min(b0 + kTickFillFloats, (int64_t)a.out_len);
            for (int64_t k = b0 + threadIdx.x; k < b1; k += kGeomBlock) a.out[k] = 0.f;
        }
        __syncthreads();   // the item's shared memory is free before the next one
    }
}

__global__ void __launch_bounds__(kGeomBlock) k_tick_scatter(const TickList* __restrict__ L)
{
    const int n = L->n;
    if (n <= 0) return;
    const int64_t g_total = L->gfirst[n];
    for (int64_t t = blockIdx.x; t < g_total; t += gridDim.x) {
        const int i = tick_slot(L->gfirst, n, t);
        scatter_body(L->geom[i], (int)(t - L->gfirst[i]));
        __syncthreads();   // the item's shared memory is free before the next one
    }
}

const void* tick_count_kernel() { return (const void*)k_tick_count; }
const void* tick_scatter_kernel() { return (const void*)k_tick_scatter; }

hipError_t launch_tick_geometry(const TickList* list, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_tick_count, dim3(grid), dim3(kGeomBlock), 0, st, list);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tick_scatter, dim3(grid), dim3(kGeomBlock), 0, st, list);
    return hipGetLastError();
}

// Two launches (count, scatter) when the scatter can sum the counts itself
// (a.offsets null), three (count, scan, scatter) otherwise.
hipError_t launch_geometry(const GeomArgs& a, hipStream_t st)
{
    if (a.n_blocks <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_geom_count, dim3(a.n_blocks), dim3(kGeomBlock), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.offsets) {
        hipLaunchKernelGGL(k_geom_scan, dim3(1), dim3(1024), 0, st, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_geom_scatter, dim3(a.n_blocks), dim3(kGeomBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_geometry_batch(const GeomList& g, int64_t n_blocks, bool need_scan, hipStream_t st)
{
    if (g.n <= 0 || n_blocks <= 0) return hipSuccess;
    if (n_blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_geom_count_batch, dim3((unsigned)n_blocks), dim3(kGeomBlock), 0, st, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (need_scan) {
        hipLaunchKernelGGL(k_geom_scan_batch, dim3((unsigned)g.n), dim3(1024), 0, st, g);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_geom_scatter_batch, dim3((unsigned)n_blocks), dim3(kGeomBlock), 0, st, g);
    return hipGetLastError();
}

}  // namespace nlos
