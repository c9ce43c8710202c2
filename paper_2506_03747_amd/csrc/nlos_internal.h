// Internal interface between the C ABI layer (nlos_abi.cpp) and the HIP
// kernels (nlos_geometry.hip, nlos_forward.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace nlos {

constexpr int kMaxRadius = 127;
constexpr int kMaxTaps = 2 * kMaxRadius + 1;

// Radius the jitter taps are zero-padded to in the pair kernels' flush (one
// compiled variant per value); the host sizes the histogram rows from it.
__host__ __device__ inline int jitter_rm(int R)
{
    return R <= 2 ? 2 : (R <= 4 ? 4 : (R <= 6 ? 6 : (R <= 8 ? 8 : (R <= 12 ? 12 : (R <= 16 ? 16 : R)))));
}

// The flush turns each histogram row into a float row in the same LDS: logical
// word x (zeros, the bins, zeros) is stored at physical word x + floor(x / 8),
// one spare word per eight, so that lanes reading eight consecutive words
// apiece (a stride of nine) hit distinct banks.  Output t0w + o of the row
// sits at logical word flush_lead + o.  The host sizes histogram rows so that
// a float row fits in the bytes of its histogram row.
constexpr int kFlushV = 8;   // consecutive outputs per lane
__host__ __device__ inline int flush_lead(int RM) { return ((RM + 7) & ~7) + 8; }
__host__ __device__ inline int flush_row_logical(int tl, int RM) { return (flush_lead(RM) + tl + RM + 8 + 7) & ~7; }
__host__ __device__ inline int flush_row_words(int tl, int RM) { return flush_row_logical(tl, RM) / 8 * 9; }

constexpr int kBlock = 1024;           // threads per workgroup of the pair kernels
constexpr int kBlockPx = 16;           // record order: 16x16-pixel blocks, 4 stride-2 phases

// Canonical cell-centred coordinate: fp32(a0 + (i + 0.5) * step), computed in
// fp64 (a0 = c - half, step = 2 half / n, both computed on the host in fp64).
struct Axis {
    double a0, step;
    int32_t n;
};

struct ChunkStat;

struct GeomArgs {
    const float* depth;
    const float* albedo;   // nullable -> 0.5
    const uint8_t* mask;   // nullable -> all present
    float4* patches;       // [n][2] float4 records
    int32_t* n_active;
    int32_t* counts;       // workspace: per enumeration block
    int32_t* offsets;      // workspace: exclusive prefix of counts; null: each
                           // scatter block sums the counts before it
    ChunkStat* stats;      // nullable: [n_stats] summaries, one per kStatBlock consecutive records (the
                           // partition k_chunk_stats uses), cleared by the count pass, merged by the scatter
    int32_t n_stats;
    Axis ax, ay;
    float hx, hy;          // spacings
    int32_t bx, by;        // ceil(n / 16) per axis
    int64_t n_enum;        // 256 * bx * by
    int32_t n_blocks;      // ceil(n_enum / kGeomBlock)
    int32_t cosines;
    float4* prep;          // nullable: [n][2] the pair loop's per-record constants ({x, y, z} as recorded, then the
                           // weight and normal terms in the pair loop's units)
    float prep_sig;        // the pair loop's bins per metre (its scale of coordinates)
};
constexpr int kGeomBlock = 256;

// Summary of kStatBlock consecutive patch records: lateral bounding box,
// smallest depth, largest a, record count.  Used to bound the pair weights
// (and so the fixed-point scales); both the one-call path and nlos_forward
// build them over the same partition, so both get the same scales.  The six
// float fields are stored as order-preserving int32 images (ord_f).
struct ChunkStat {
    int32_t x0, x1, y0, y1, z0, amax;
    int32_t count, pad;
};
static_assert(sizeof(ChunkStat) == 32, "summaries are read as two int4");
constexpr int kStatBlock = 256;

struct StatF {
    float x0, x1, y0, y1, z0, amax;
    int32_t count;
};

// Minimum, maximum or sum (OP 0, 1, 2) of v over the 64 lanes of a
// wavefront, every lane active: partial results within rows of 16 lanes by
// row shifts, then across rows by the row broadcasts; lane 63 ends with the
// result.  Lanes a DPP step does not write keep the identity.
template <int OP>
__device__ __forceinline__ int wave_reduce_i(int v)
{
    constexpr int id = OP == 0 ? INT32_MAX : (OP == 1 ? INT32_MIN : 0);
#define NLOS_DPP_STEP(ctrl, rows)                                                          \
    {                                                                                      \
        const int t = __builtin_amdgcn_update_dpp(id, v, ctrl, rows, 0xf, false);         \
        v = OP == 0 ? min(v, t) : (OP == 1 ? max(v, t) : v + t);                           \
    }
    NLOS_DPP_STEP(0x111, 0xf)   // row_shr:1
    NLOS_DPP_STEP(0x112, 0xf)   // row_shr:2
    NLOS_DPP_STEP(0x114, 0xf)   // row_shr:4
    NLOS_DPP_STEP(0x118, 0xf)   // row_shr:8
    NLOS_DPP_STEP(0x142, 0xa)   // row_bcast:15 into rows 1 and 3
    NLOS_DPP_STEP(0x143, 0xc)   // row_bcast:31 into rows 2 and 3
#undef NLOS_DPP_STEP
    return __builtin_amdgcn_readlane(v, 63);
}

// Maximum (MAX true) or minimum of v over the 64 lanes of a wavefront (every
// lane active), the same DPP steps on the bits of v with -inf or +inf as the
// identity.
template <bool MAX>
__device__ __forceinline__ float wave_extreme_f(float v)
{
    constexpr int id = MAX ? (int)0xff800000 : 0x7f800000;   // -inf, +inf
#define NLOS_DPP_STEP(ctrl, rows)                                                                  \
    {                                                                                              \
        const float t = __int_as_float(__builtin_amdgcn_update_dpp(id, __float_as_int(v), ctrl, rows, 0xf, false)); \
        v = MAX ? fmaxf(v, t) : fminf(v, t);                                                       \
    }
    NLOS_DPP_STEP(0x111, 0xf)   // row_shr:1
    NLOS_DPP_STEP(0x112, 0xf)   // row_shr:2
    NLOS_DPP_STEP(0x114, 0xf)   // row_shr:4
    NLOS_DPP_STEP(0x118, 0xf)   // row_shr:8
    NLOS_DPP_STEP(0x142, 0xa)   // row_bcast:15 into rows 1 and 3
    NLOS_DPP_STEP(0x143, 0xc)   // row_bcast:31 into rows 2 and 3
#undef NLOS_DPP_STEP
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ float wave_max_f(float v) { return wave_extreme_f<true>(v); }

__device__ __forceinline__ int32_t ord_f(float f)
{
    const int32_t b = __float_as_int(f);
    return b >= 0 ? b : b ^ 0x7FFFFFFF;
}

__device__ __forceinline__ float unord_f(int32_t k) { return __int_as_float(k >= 0 ? k : k ^ 0x7FFFFFFF); }

__device__ __forceinline__ StatF decode_stat(int __attribute__((ext_vector_type(4))) c0,
                                             int __attribute__((ext_vector_type(4))) c1)
{
    StatF r;
    r.x0 = unord_f(c0.x);
    r.x1 = unord_f(c0.y);
    r.y0 = unord_f(c0.z);
    r.y1 = unord_f(c0.w);
    r.z0 = unord_f(c1.x);
    r.amax = unord_f(c1.y);
    r.count = c1.z;
    return r;
}

__device__ __forceinline__ StatF load_stat(const ChunkStat* st, int i)
{
    typedef int v4i __attribute__((ext_vector_type(4)));
    const __attribute__((address_space(1))) v4i* g = (const __attribute__((address_space(1))) v4i*)st;
    return decode_stat(g[2 * (size_t)i], g[2 * (size_t)i + 1]);
}

// Arguments of the pair kernels (confocal and non-confocal).
struct FwdArgs {
    const float4* patches;
    const float4* prep;        // nullable: the records' pair-loop constants, same order: {x, y, z, ap} (coordinates
                               // as recorded), {mnxs, mnys, c0s, 0} (PatchC, scaled)
    const int32_t* n_active;   // nullable
    int32_t n_cap;
    float* out;
    int64_t out_len;           // floats in out
    Axis rx, ry;               // relay (detector) grid
    Axis lx, ly;               // laser grid (non-confocal)
    double cx, cy, s;          // device position (cx, cy, s)
    double inv;                // 1 / (c dt), bins per metre
    float inv_f;               // fp32(inv)
    float inv2_f;              // fp32(2 inv)
    float delta;               // guard half-width, bins
    float two_delta;
    float dummy_x;             // x of a stand-in patch arriving >= T + 64 bins
    int32_t T;
    int32_t tiles_x, tiles_y;  // units over the detector grid
    int32_t tiles_l;           // units over the laser points (non-confocal)
    int32_t n_units;           // tiles_l * tiles_x * tiles_y
    int32_t pair;              // 1: a workgroup owns two units
    int32_t plan;              // 1: units paired by a torus shift of half the unit grid
    ChunkStat* stats;          // [n_stats] summaries of the records
    int32_t n_stats;
    int32_t n_split;           // patch ranges per unit pair
    int32_t tw, n_tw;          // output time window per workgroup, and count
    int32_t stride;            // floats per LDS histogram row
    int32_t q_cap;             // guard-queue entries
    int32_t atomic_out;        // 1: accumulate into a zeroed output
    int32_t cosines;
    int32_t R;
    unsigned long long* eval_pairs;   // nullable: += (wavefront lanes in range) x (unit histograms) per
                                      // evaluated (wavefront, unit) block, i.e. the pairs the loop evaluated
    float taps[kMaxTaps];
};

// Work list of a batched launch: workgroup b runs request req[i] with local
// workgroup index b - first[i], where i is the last entry with first[i] <= b.
struct BatchList {
    const FwdArgs* tab;        // device table of per-request arguments
    const int32_t* req;        // [n] request of each entry
    const int64_t* first;      // [n] first workgroup of each entry (ascending)
    int32_t n;
};

struct GeomList {
    const GeomArgs* tab;       // device table, one entry per depth map
    const int64_t* first;      // [n] first enumeration block of each map
    int32_t n;
};

// A serving tick: the records of a list of depth maps and their histograms,
// by three launches over a device work list of (request, block) items: the
// count and scatter passes with fixed persistent grids, the pairs with one
// workgroup per item.  The list lives in device memory, so the launches do
// not depend on the requests (but for the pair grid) and one graph serves
// every tick.
// Pair-kernel variants a tick runs: confocal, two units per workgroup, the
// five unit shapes, cosines on and off (tick_variant).
constexpr int kTickShapes = 5;
constexpr int kTickVariants = 2 * kTickShapes;
constexpr int kTickFillFloats = 1 << 16;   // floats per zero-fill item
struct TickList {
    const GeomArgs* geom;     // [n] in request order
    const FwdArgs* fwd;       // [n] in pair order: decreasing work per workgroup
    const int32_t* variant;   // [n] pair order
    const int64_t* gfirst;    // [n + 1] first enumeration block of each map (exclusive prefix, request order)
    const int64_t* zfirst;    // [n + 1] first zero-fill item (outputs that take float atomics; pair order)
    const int64_t* ffirst;    // [n + 1] first pair-kernel workgroup (pair order)
    int32_t n;
    int32_t pad;
};
int tick_variant(int tx, int ty, bool cosines);   // -1: not a tick variant
hipError_t launch_tick_geometry(const TickList* list, int grid, hipStream_t st);
// device addresses of a tick's list and of the arrays the pair kernel reads
struct TickArrays {
    const TickList* list;
    const FwdArgs* fwd;
    const int32_t* variant;
    const int64_t* ffirst;
};
hipError_t launch_tick_pairs(const TickArrays& t, int64_t grid, size_t lds_bytes, hipStream_t st);
hipError_t prepare_tick_pairs(size_t lds_bytes);
// the tick's kernels, for graph nodes: count and scatter (persistent, grid
// 2 x CUs, kGeomBlock threads; argument: the list), pairs (one workgroup per
// item, kBlock threads; arguments: the four TickArrays pointers)
const void* tick_count_kernel();
const void* tick_scatter_kernel();
const void* tick_pairs_kernel();

// Smooth time response (continuous Gaussian) and its adjoint, confocal.
struct SmoothArgs {
    const float4* patches;
    const int32_t* n_active;   // nullable
    int32_t n_cap;
    float* out;                // forward: [S][T]
    const float* grad_out;     // adjoint: upstream gradient [S][T]
    double* partial;           // adjoint: [n_split][n_cap][5] per-split record gradients
    Axis rx, ry;
    double cx, cy, s;          // device position
    double inv;                // bins per metre
    float sigma;               // bins
    float norm;                // 1 / (sigma sqrt(2 pi))
    float inv_s2;              // 1 / sigma^2
    float c1;                  // exp(-1 / sigma^2)
    int32_t T;
    int32_t Rs;                // support radius, bins
    int32_t tiles_x, tiles_y;  // forward: scan tiles
    int32_t n_split;           // forward: patch ranges per tile; adjoint: scan ranges
    int32_t stride;            // forward: u64 bins per LDS row
    int32_t rows;              // adjoint: rows staged in LDS at a time
    int32_t atomic_out;
    int32_t cosines;
    ChunkStat* stats;
    int32_t n_stats;
    float* moments;            // adjoint by moments: [S][adj_moments(Rs)][mlen] correlations
    float* mtaps;              // adjoint by moments: kernels K_m(d), [adj_moments(Rs)][2 Rs + 1]
    int32_t mlen;              // T + 2 Rs
};

// Record gradients -> map gradients (depth-stencil adjoint).
struct GradMapArgs {
    const float* depth;
    const float* albedo;       // nullable -> 0.5
    const float4* patches;
    const int32_t* n_active;   // nullable
    int32_t n_cap;
    const float* grad_rec;     // [n_cap][8]: d/d(pz, a, n_x, n_y, n_z) at 2..6
    float* grad_depth;
    float* grad_albedo;        // nullable
    float* scratch;            // [3][nx * ny]: d/dpz, d/dD_x, d/dD_y per pixel
    Axis ax, ay;
    float hx, hy;
    int32_t cosines;
};

// FFT (light-cone) route: N x N scan, M = T time bins (a power of two).
struct LctArgs {
    const float* depth;
    const float* albedo;       // nullable -> 0.5
    const uint8_t* mask;       // nullable
    int32_t N, M;
    double dz;                 // c dt / 2
    double cone;               // (4 slope)^2, slope = w / (M c dt)
    int32_t R;                 // jitter half-width
    double taps[kMaxTaps];
};

// Debug/test hook arguments.
struct DebugArgs {
    FwdArgs f;
    int32_t* bins;
    double* u_fast;
    double* u_exact;
    int64_t n_pairs;
    int32_t confocal;
};

// Launch plan of the pair kernel.
struct Plan {
    int tx, ty, tl;        // unit: detector points along x, y; laser points
    int pair;              // two units per workgroup
    int plan;              // torus-shift pairing of units
    int64_t groups;        // workgroups per (time window, patch split)
    int n_split;
    int tw, n_tw;
    int stride;
    int q_cap;
    size_t lds_bytes;
    int64_t n_blocks;
};

size_t lds_bytes_for(int slots, int stride, int q_cap);
bool tile_supported(bool confocal, int tx, int ty, int tl);

hipError_t launch_geometry(const GeomArgs& a, hipStream_t st);
constexpr int kScanFreeBlocks = 4096;   // up to this many blocks, the scatter sums the counts itself
hipError_t launch_forward(const FwdArgs& a, const Plan& plan, bool confocal, hipStream_t st);
hipError_t launch_stats(const FwdArgs& a, ChunkStat* stats, hipStream_t st);
hipError_t launch_fill(float* out, size_t n, hipStream_t st);
hipError_t launch_debug(const DebugArgs& a, hipStream_t st);

hipError_t launch_smooth(const SmoothArgs& a, int tx, int ty, int64_t n_blocks, size_t lds, hipStream_t st);
// Smooth forward by moments of the sub-bin offset (support radii 12, 16, 20):
// scan points per workgroup and moment rows per point (the series is cut
// after m = moments - 1: 7 at radius 12, 5 at 16 and 20, where sigma > 2.5
// bins makes the terms fall faster).
struct SmoothMomShape {
    int points, moments;
};
constexpr SmoothMomShape smooth_mom_shape(int rs) { return rs == 12 ? SmoothMomShape{2, 8} : SmoothMomShape{3, 6}; }
// The rows' pitch (u64 bins) used whenever the rows take more than half the
// LDS (one workgroup per CU either way): the largest even pitch whose rows
// and 2 KiB of constants fit in 160 KiB, known at compile time so that the
// rows' offsets go into the LDS instructions' immediate field.
constexpr int smooth_mom_pitch(int rs)
{
    return ((163840 - 2048) / (smooth_mom_shape(rs).points * smooth_mom_shape(rs).moments * 8)) & ~1;
}
bool smooth_moments_radius(int rs);
hipError_t launch_smooth_moments(const SmoothArgs& a, int64_t n_blocks, size_t lds, hipStream_t st);
// Adjoint by moments (the same radii): adj_moments correlation rows per scan
// point, kAdjPatches patches per thread in the gather.
// Correlation rows per scan point: C_0 .. C_{n-1} give G0 to the power
// n - 2 of the sub-bin offset and G1 to the same power; 9 at radius 12, 7 at
// 16 and 20 (sigma > 2.5 bins).
constexpr int adj_moments(int rs) { return rs == 12 ? 9 : 7; }
constexpr int kAdjPatches = 4;
// LDS of the moment gather: `buffers` copies (2: the next scan points' rows
// land while the current ones are used) of `rows` scan points' correlation
// rows, rounded to 16 bytes, and 24 bytes of constants per point.
inline size_t adj_mom_lds(int buffers, int rows, int nm, int L)
{
    return (size_t)buffers * ((((size_t)rows * nm * L * 4 + 15) & ~(size_t)15) + (size_t)rows * 24);
}
hipError_t launch_adjoint_moments(const SmoothArgs& a, int64_t patch_blocks, size_t lds, int dbuf, hipStream_t st);
hipError_t launch_adjoint(const SmoothArgs& a, int64_t patch_blocks, size_t lds, hipStream_t st);
hipError_t launch_adjoint_reduce(const SmoothArgs& a, float* grad_rec, hipStream_t st);
hipError_t launch_grad_maps(const GradMapArgs& g, hipStream_t st);
constexpr int kAdjStride = 5;   // doubles per record in the adjoint partials

hipError_t launch_noise_scale(const float* tau, int64_t n, double nr_db, double* out, double* part, int nb,
                              hipStream_t st);
hipError_t launch_poisson(const float* tau, int64_t n, const double* sigma_n, uint64_t seed, float* out,
                          hipStream_t st);
constexpr int kNoiseMomentBlocks = 1024;

int lct_fft_work_bytes(int N, int M, size_t* bytes);
hipError_t launch_lct(const LctArgs& a, double2* vol, double2* psf, void* fft_work, float* out, hipStream_t st,
                      int* fft_status);

// Batched launches (one launch each over all requests of the list).
hipError_t launch_geometry_batch(const GeomList& g, int64_t n_blocks, bool need_scan, hipStream_t st);
hipError_t launch_stats_batch(const BatchList& b, int64_t n_blocks, hipStream_t st);
constexpr int kFillBlocksPerRequest = 64;
hipError_t launch_fill_batch(const BatchList& b, hipStream_t st);
hipError_t launch_forward_batch(const BatchList& b, int64_t n_blocks, size_t lds_bytes, int tl, int tx, int ty,
                                bool confocal, bool cosines, bool pair, hipStream_t st);

}  // namespace nlos
