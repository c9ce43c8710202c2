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

__device__ __forceinline__ bool is_present(const GeomArgs& a, int64_t idx)
{
    const float z = a.depth[idx];
    const float rho = a.albedo ? a.albedo[idx] : 0.5f;
    const bool m = a.mask ? (a.mask[idx] != 0) : true;
    return m && rho > 0.f && isfinite(z) && z > 0.f;
}

__device__ __forceinline__ void count_body(const GeomArgs& a, int blk)
{
    const int64_t e = (int64_t)blk * kGeomBlock + threadIdx.x;
    int ix = 0, iy = 0;
    bool p = enum_pixel(a, e, &ix, &iy);
    if (p) p = is_present(a, (int64_t)ix * a.ay.n + iy);
    const int cnt = __syncthreads_count(p);
    if (threadIdx.x == 0) a.counts[blk] = cnt;
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

// Derivative of the depth map along one axis (central inside, one-sided at
// the borders, 0 for a single sample); `d` points at sample i, stride between
// samples in elements.
__device__ __forceinline__ float deriv(const float* d, int n, int i, int64_t stride, float h)
{
    if (n < 2) return 0.f;
    if (i == 0) return (d[stride] - d[0]) / h;
    if (i == n - 1) return (d[0] - d[-stride]) / h;
    return (d[stride] - d[-stride]) / (2.f * h);
}

__device__ __forceinline__ void scatter_body(const GeomArgs& a, int blk)
{
    __shared__ int wave_cnt[kGeomBlock / 64];
    const int64_t e = (int64_t)blk * kGeomBlock + threadIdx.x;
    int ix = 0, iy = 0;
    bool p = enum_pixel(a, e, &ix, &iy);
    const int64_t idx = (int64_t)ix * a.ay.n + iy;
    if (p) p = is_present(a, idx);
    const unsigned long long bal = __ballot(p);
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const int rank = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_cnt[wave] = __popcll(bal);
    __syncthreads();
    if (!p) return;
    int off = a.offsets[blk];
    for (int w = 0; w < wave; ++w) off += wave_cnt[w];
    off += rank;

    const float* D = a.depth + idx;
    const float z = D[0];
    const float rho = a.albedo ? a.albedo[idx] : 0.5f;
    const float gx = deriv(D, a.ax.n, ix, a.ay.n, a.hx);
    const float gy = deriv(D, a.ay.n, iy, 1, a.hy);
    const float len = sqrtf(1.f + gx * gx + gy * gy);
    const float area = a.hx * a.hy * (a.cosines ? len : 1.f);
    a.patches[2 * (int64_t)off] = make_float4(canon(a.ax, ix), canon(a.ay, iy), z, rho * area);
    a.patches[2 * (int64_t)off + 1] = make_float4(gx / len, gy / len, -1.f / len, __int_as_float((int)idx));
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

__global__ void __launch_bounds__(1024) k_geom_scan_batch(const GeomList g) { scan_body(g.tab[blockIdx.x]); }

__global__ void __launch_bounds__(kGeomBlock) k_geom_scatter_batch(const GeomList g)
{
    const int i = geom_slot(g, (int64_t)blockIdx.x);
    scatter_body(g.tab[i], (int)((int64_t)blockIdx.x - g.first[i]));
}

hipError_t launch_geometry(const GeomArgs& a, hipStream_t st)
{
    if (a.n_blocks <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_geom_count, dim3(a.n_blocks), dim3(kGeomBlock), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_geom_scan, dim3(1), dim3(1024), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_geom_scatter, dim3(a.n_blocks), dim3(kGeomBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_geometry_batch(const GeomList& g, int64_t n_blocks, hipStream_t st)
{
    if (g.n <= 0 || n_blocks <= 0) return hipSuccess;
    if (n_blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_geom_count_batch, dim3((unsigned)n_blocks), dim3(kGeomBlock), 0, st, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_geom_scan_batch, dim3((unsigned)g.n), dim3(1024), 0, st, g);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_geom_scatter_batch, dim3((unsigned)n_blocks), dim3(kGeomBlock), 0, st, g);
    return hipGetLastError();
}

}  // namespace nlos
