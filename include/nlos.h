/*
 * nlos.h -- C ABI of the MI355X (gfx950) transient NLOS forward operator.
 *
 * The operator simulates the time-resolved measurement of a non-line-of-sight
 * setup (arXiv 2506.03747): a hidden surface given as a depth map and an
 * albedo map, a planar relay wall at z = 0 scanned on a grid, a pulsed laser
 * and a time-resolved detector.  For every wall scan point and every hidden
 * patch it computes the three-bounce path (device -> wall -> patch -> wall ->
 * device), the Lambertian radiometric weight with inverse-square falloff, bins
 * the weight into the scan point's histogram and blurs each histogram with the
 * detector's Gaussian time jitter.
 *
 *   Section 2, Eq. (1): tau(x',y',t) = iiint rho / r^4 delta(2 r - t c) dx dy dz
 *   Section 2, depth-to-volume mapping (Algorithm 1, step 2.1): the hidden
 *     object is a depth map plus an albedo map (0.5 when absent).
 *   Section 2, temporal jitter (Algorithm 1, step 2.3): per-trace Gaussian,
 *     sigma = FWHM / (2 sqrt(2 ln 2)), kernel length 2 ceil(2 sigma) + 1.
 *
 * Conventions (they fix points the paper leaves open):
 *   - c = 299 792 458 m/s.  Grids are cell-centred: cell i of n over
 *     [c - half, c + half] sits at fp32((c - half) + (i + 0.5) * (2 half / n)),
 *     computed in fp64 and rounded once.
 *   - Maps and outputs are indexed [x][y] (x major); histograms are [x'][y'][t]
 *     with t contiguous; non-confocal output is [laser][x'][y'][t], laser
 *     points also x major.
 *   - The device (laser and detector) sits on the wall normal through the
 *     relay-grid centre at distance s = standoff_m.  Time 0 is the gate 2 s / c.
 *     Each device leg adds (L - s) to the path and weighs (s / L)^3, with
 *     L the device-to-wall-point distance; s = 0 means calibrated data with no
 *     device legs (Eq. (1) as printed).
 *   - Path u (in bins) = ((r_l + r_d) + o) * (1 / (c dt)), o the sum of the
 *     two device-leg offsets; bin k = floor(u), kept when 0 <= k < T.  The bin
 *     index is that of the fp64 evaluation of this expression (in this order,
 *     IEEE round-to-nearest, no fused multiply-add) from the fp32 coordinates,
 *     exactly: the kernels evaluate pairs in fp32 and re-evaluate in fp64
 *     every pair whose fp32 arrival lies too close to a bin edge to decide.
 *   - Weight with NLOS_F_COSINES: a * cos_wall,l * cos_patch,l * cos_patch,d *
 *     cos_wall,d / (r_l^2 r_d^2) * g_l * g_d, patch cosines clamped at 0,
 *     a = albedo * true patch area; without the flag a / (r_l^2 r_d^2) * g_l *
 *     g_d with a = albedo * projected area.  No global constant (pi, c, dt).
 *   - Jitter taps are normalised to sum 1; zero padding outside [0, T).
 *
 * Ownership and execution: the caller owns every buffer (device memory
 * unless stated otherwise).  The library never allocates, frees or
 * synchronises inside these calls: work is enqueued on the caller's stream
 * (`stream` is a hipStream_t; NULL = the null stream) and the call returns
 * immediately.  Host-side argument checks happen before anything is
 * enqueued; a rejected call enqueues nothing.  Calls on distinct streams are
 * independent; the library's only global state is its error slot (per
 * thread).
 *
 * Errors: every int-returning call gives NLOS_OK (0) or a negative code:
 *   NLOS_EINVAL  bad sizes or parameters, a null required pointer, a
 *                misaligned buffer, a limit below exceeded;
 *   NLOS_ENOSPC  the workspace passed is smaller than required;
 *   NLOS_EHIP    a HIP runtime call failed (nlos_last_hip_error() has its code);
 *   NLOS_ENODEV  no usable GPU.
 * No C++ exception crosses this boundary.
 */
#ifndef NLOS_H
#define NLOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NLOS_ABI_VERSION 2

#define NLOS_OK 0
#define NLOS_EINVAL (-1)
#define NLOS_ENOSPC (-2)
#define NLOS_EHIP (-3)
#define NLOS_ENODEV (-4)

/* flags */
#define NLOS_F_COSINES 1u /* Lambertian cosines and true patch area (default) */

/* limits */
#define NLOS_MAX_BINS (1 << 22)        /* T */
#define NLOS_MAX_RADIUS 127            /* jitter half-width R = ceil(2 sigma) */
#define NLOS_MAX_PATCHES (1 << 24)     /* records per call */
#define NLOS_MAX_GRID 65536            /* nx, ny of any grid */
#define NLOS_RECORD_FLOATS 8           /* floats per patch record (32 bytes) */

/* A cell-centred grid of nx x ny points on the wall plane z = 0 (or the lateral
 * grid of a depth map) covering [cx-half_x, cx+half_x] x [cy-half_y, cy+half_y],
 * metres. */
typedef struct nlos_grid {
    int32_t nx, ny;
    double half_x, half_y;
    double cx, cy;
} nlos_grid;

/* System parameters (Algorithm 1 inputs; Section 1 lists relay surface,
 * stand-off distance, time resolution and acquisition window). */
typedef struct nlos_params {
    nlos_grid relay;   /* confocal scan grid, or the detector grid when laser.nx > 0 */
    nlos_grid laser;   /* laser grid; nx = ny = 0 -> confocal */
    double standoff_m; /* s >= 0 (0: calibrated, no device legs) */
    double bin_ps;     /* dt > 0, picoseconds */
    int32_t n_bins;    /* T, 1..NLOS_MAX_BINS; window [2s/c, 2s/c + T dt) */
    uint32_t flags;    /* NLOS_F_COSINES */
    double fwhm_ps;    /* jitter FWHM >= 0, picoseconds; 0 -> no jitter */
} nlos_params;

/* Version of this ABI (NLOS_ABI_VERSION). */
int nlos_abi_version(void);

/* Static description of an error code; never NULL. */
const char* nlos_strerror(int code);

/* hipError_t of the last HIP failure on this thread (0 if none). */
int nlos_last_hip_error(void);

/* Bytes of workspace nlos_patches_from_depth needs for grid g (written to
 * *bytes, a host pointer). */
int nlos_patches_workspace_bytes(const nlos_grid* g, size_t* bytes);

/*
 * Depth map (+ albedo, + mask) -> patch records (Section 2 depth-to-volume
 * mapping; Algorithm 1 step 2.1).
 *   g       host pointer: lateral grid of the maps (g->nx * g->ny pixels).
 *   depth   device float [nx][ny], metres along +z from the wall.
 *   albedo  device float [nx][ny] in [0, 1], or NULL for 0.5 everywhere
 *           (8-bit maps are divided by 255 by the caller).
 *   mask    device uint8 [nx][ny], nonzero = present, or NULL for all.
 *   flags   NLOS_F_COSINES selects the true patch area
 *           dx dy sqrt(1 + D_x^2 + D_y^2), else the projected area dx dy;
 *           pass the same flags to nlos_forward.
 *   patches device float [nx*ny][8], 16-byte aligned: the first *n_active
 *           records are the present patches
 *              { x, y, z, a = albedo * area, n_x, n_y, n_z, bits(int32 ix*ny+iy) }
 *           with n = (D_x, D_y, -1) / sqrt(1 + D_x^2 + D_y^2) from central
 *           differences of the depth map (one-sided at the border); the rest
 *           of the buffer is left unspecified.  A pixel is present when its
 *           mask is nonzero, its albedo > 0 and its depth finite and > 0.
 *           Records come in a fixed, deterministic order: 16x16-pixel
 *           blocks (x major), each as 4 stride-2 phases of 8x8 pixels, so any
 *           64 consecutive records cover a small square of the surface.
 *   n_active device int32[1]: number of present patches.
 *   ws, ws_bytes device workspace of at least nlos_patches_workspace_bytes.
 * Limits: nx*ny <= NLOS_MAX_PATCHES.
 */
int nlos_patches_from_depth(const nlos_grid* g, const float* depth, const float* albedo,
                            const uint8_t* mask, uint32_t flags, float* patches,
                            int32_t* n_active, void* ws, size_t ws_bytes, void* stream);

/* Bytes of workspace nlos_forward needs (written to *bytes, host pointer):
 * 32 bytes per block of 256 records (summaries used to cull, balance the work
 * and bound the pair weights), rounded up to 256. */
int nlos_forward_workspace_bytes(const nlos_params* p, int32_t n_patches, size_t* bytes);

/*
 * Forward operator (Section 2 Eq. (1) with the conventions above, then the
 * Gaussian jitter of Section 2 / Algorithm 1 step 2.3).
 *   p          host pointer to the parameters.
 *   patches    device float [n_patches][8] records as written by
 *              nlos_patches_from_depth (16-byte aligned).
 *   n_patches  capacity of `patches` (0..NLOS_MAX_PATCHES).
 *   n_active   device int32[1] with the number of leading records to use
 *              (clamped to [0, n_patches]), or NULL to use n_patches.
 *   out        device float, fully overwritten, 16-byte aligned:
 *              confocal [relay.nx][relay.ny][T];
 *              non-confocal [laser.nx*laser.ny][relay.nx][relay.ny][T].
 *   ws, ws_bytes device workspace, 16-byte aligned, at least
 *              nlos_forward_workspace_bytes (may be NULL when that size is 0);
 *              overwritten by the call, so calls that share a workspace must be
 *              ordered on one stream.
 * Precision: each pair's weight is found in fp32 and accumulated in 64-bit
 * fixed point: it adds round(w * s_u), s_u = 2^31 / W_u, where the block u of
 * histograms -- the aligned 4 x 4 scan points that hold the histogram
 * (confocal), or 2 lasers x 2 x 2 detectors (non-confocal), whatever unit
 * the plan chose -- has the bound
 *   W_u = max over the summaries of 256 consecutive records of
 *         a_max / ((d_l^2 + z_min^2) (d_d^2 + z_min^2)),
 * d_l, d_d the lateral distances from the summary's bounding box to the
 * block's laser and detector rectangles.  A pair's rounding is therefore at
 * most g_l g_d W_u / 2^32; the fp32 weight is within a few ulp of its fp64
 * value except where a patch cosine cancels (grazing patches), where the
 * error is that of the fp32 record normals.  As the scales depend on the
 * records and the block only, every call that computes a histogram
 * (nlos_forward, nlos_simulate, the batched calls, a serving tick) gives the
 * same bits, except where patches are split over workgroups (float atomics).
 */
int nlos_forward(const nlos_params* p, const float* patches, int32_t n_patches,
                 const int32_t* n_active, float* out, void* ws, size_t ws_bytes, void* stream);

/*
 * nlos_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same launches and results (bit for bit) with the record summaries in a
 * scratch array the library holds on each GPU it runs on (512 KiB, kept
 * until the process ends; its address is looked up on the first call on a
 * device, with that device current, so `stream` must belong to the current
 * device).  The call itself allocates nothing.
 *   n_patches  at most NLOS_NOALLOC_MAX_PATCHES, else NLOS_ENOSPC.
 * Calls on one GPU share the scratch: calls that overlap in time on one GPU
 * (on different streams, or from several threads without ordering) race and
 * give wrong results; order them on one stream.  Other arguments and errors
 * as nlos_forward.
 */
#define NLOS_NOALLOC_MAX_PATCHES (1 << 22)

int nlos_forward_noalloc(const nlos_params* p, const float* patches, int32_t n_patches,
                         const int32_t* n_active, float* out, void* stream);

/*
 * The whole path in one call: nlos_patches_from_depth for the depth map on
 * grid g (flags = p->flags) followed by nlos_forward over its records, with
 * the record summaries built while the records are written (no separate
 * pass).  patches [g.nx*g.ny][8] and n_active are written as by
 * nlos_patches_from_depth, bit for bit; the summaries cover the same records
 * as nlos_forward's (256 consecutive records each), so the fixed-point scales
 * are the same and out equals nlos_forward's bit for bit, except where
 * patches are split over workgroups (nlos_get_plan n_split > 1: partial
 * histograms are then added with float atomics, in no fixed order).
 * ws: at least nlos_simulate_workspace_bytes, 256-byte aligned.
 * probe: NULL, or instrumentation of the call (host pointer, read during the
 * call only).
 */
typedef struct nlos_probe {
    void* forward_mark;                 /* hipEvent_t recorded on the stream right before
                                           the pair kernel (to time it), or NULL */
    unsigned long long* evaluated_pairs; /* device uint64, 8-byte aligned, or NULL: the pair
                                           kernel adds the number of (histogram, patch) pairs
                                           it evaluated; the rest were culled as arriving
                                           past the window (the caller zeroes it) */
} nlos_probe;

int nlos_simulate_workspace_bytes(const nlos_params* p, const nlos_grid* g, size_t* bytes);

int nlos_simulate(const nlos_params* p, const nlos_grid* g, const float* depth, const float* albedo,
                  const uint8_t* mask, float* patches, int32_t* n_active, float* out, void* ws, size_t ws_bytes,
                  const nlos_probe* probe, void* stream);

/*
 * Batched calls: many independent scenes (uneven sizes, time windows, bin
 * widths, jitter) in one launch per kernel phase, as a serving loop issues
 * them (Algorithm 1 runs the forward model once per frame of a sequence).
 * Each request computes exactly what the single call computes for it.
 *
 * The library writes a small table (per-request kernel arguments and the
 * work lists) into host memory and copies it to the start of the device
 * workspace on `stream` before the kernels:
 *   table, table_bytes  host buffer of at least *table_bytes of the _sizes
 *           call, owned by the caller; pinned memory (hipHostMalloc) keeps
 *           the copy asynchronous.  It must stay untouched until the stream
 *           has passed the call.  NULL: the library uses a per-thread pageable
 *           buffer, and the copy may then block the host until the stream
 *           reaches it.
 *   ws, ws_bytes  device workspace, 16-byte aligned, at least *ws_bytes of
 *           the _sizes call; calls sharing it must be ordered on one stream.
 * Requests of one call must not share an output buffer.  n may be 0 (no-op).
 * A rejected request rejects the whole call before anything is enqueued.
 */
typedef struct nlos_depth_request {
    nlos_grid grid;          /* lateral grid of the maps */
    const float* depth;      /* device [nx][ny] */
    const float* albedo;     /* device [nx][ny] or NULL (0.5) */
    const uint8_t* mask;     /* device [nx][ny] or NULL (all present) */
    uint32_t flags;          /* NLOS_F_COSINES */
    float* patches;          /* device [nx*ny][8] records, 16-byte aligned */
    int32_t* n_active;       /* device int32[1] */
} nlos_depth_request;

typedef struct nlos_request {
    nlos_params params;
    const float* patches;    /* device [n_patches][8] records */
    int32_t n_patches;       /* capacity of patches */
    const int32_t* n_active; /* device int32[1] or NULL (use n_patches) */
    float* out;              /* device output, layout as for nlos_forward */
} nlos_request;

/* Table and workspace sizes of nlos_patches_batched (host pointers). */
int nlos_patches_batched_sizes(const nlos_depth_request* reqs, int32_t n, size_t* table_bytes,
                               size_t* ws_bytes);

/* nlos_patches_from_depth for every request: three launches in all. */
int nlos_patches_batched(const nlos_depth_request* reqs, int32_t n, void* table, size_t table_bytes,
                         void* ws, size_t ws_bytes, void* stream);

/* Table and workspace sizes of nlos_forward_batched (host pointers). */
int nlos_forward_batched_sizes(const nlos_request* reqs, int32_t n, size_t* table_bytes, size_t* ws_bytes);

/*
 * nlos_forward for every request: one launch of record summaries, one of
 * output zeroing when a request needs it, and one pair-kernel launch per
 * kernel variant present (tile shape, confocal or not, cosines, time
 * windows).  Each request gets a share of the GPU's workgroups in proportion
 * to its pairs; within a launch the workgroups with the most work start first.
 */
int nlos_forward_batched(const nlos_request* reqs, int32_t n, void* table, size_t table_bytes, void* ws,
                         size_t ws_bytes, void* stream);

/*
 * Serving ticks: the whole path (depth maps -> records -> histograms) for a
 * list of requests, as a serving loop runs it once per tick (Algorithm 1
 * runs the forward model once per frame; many scenes share one tick here).
 * A tick is a fixed sequence of four operations on one stream: a copy of a
 * host table to the start of the workspace, then three kernels over the
 * (request, block) items the copied table lists: depth-map counts and output
 * zeroing, then record scatter with summaries and pair-loop constants (both
 * persistent, a fixed grid of 2 x CUs striding over the items), then pairs,
 * binning, guard, jitter and write-out (one workgroup per item).  Only the
 * pair grid depends on the requests, so a tick is one HIP graph launch (see
 * nlos_tick_graph_*) after rewriting the table with nlos_tick_plan.  Each request's records, n_active and output are
 * those of nlos_simulate for it alone, bit for bit (outputs that take float
 * atomics to 1e-6).
 * Supported requests: confocal, maps of at most 1024 x 1024 enumeration
 * pixels (4096 blocks of 256), plans that pair units over the whole window
 * (nlos_get_plan pair = 1, n_windows = 1); anything else is NLOS_EINVAL
 * from nlos_tick_plan (serve it through nlos_simulate).
 */
typedef struct nlos_sim_request {
    nlos_params params;
    nlos_grid grid;          /* lateral grid of the maps */
    const float* depth;      /* device [nx][ny] */
    const float* albedo;     /* device [nx][ny] or NULL (0.5) */
    const uint8_t* mask;     /* device [nx][ny] or NULL (all present) */
    float* patches;          /* device [nx*ny][8] records, 16-byte aligned */
    int32_t* n_active;       /* device int32[1] */
    float* out;              /* device output [relay.nx][relay.ny][T], 16-byte aligned */
} nlos_sim_request;

typedef struct nlos_tick_caps {
    int32_t max_requests;    /* 1..4096 per tick */
    int64_t max_pixels;      /* sum of nx * ny over a tick's requests */
} nlos_tick_caps;

/* Host table and device workspace bytes of a tick with these capacities
 * (host pointers). */
int nlos_tick_sizes(const nlos_tick_caps* caps, size_t* table_bytes, size_t* ws_bytes);

/* Write the tick table for n requests (0..max_requests) into the host
 * buffer `table` (at least *table_bytes; pinned memory keeps the copy
 * asynchronous); the table holds device addresses inside `ws` (256-byte
 * aligned, at least *ws_bytes), where the tick keeps its summaries and
 * constants.  Host only: nothing is enqueued.  The table must stay untouched
 * until the stream has passed the tick's copy. */
int nlos_tick_plan(const nlos_tick_caps* caps, const nlos_sim_request* reqs, int32_t n, void* table,
                   size_t table_bytes, void* ws, size_t ws_bytes);

/* Enqueue a tick on `stream`: the copy of `table` into `ws`, then the three
 * kernels (count and scatter persistent with a grid of 2 x CUs; pairs with
 * one workgroup per item of the planned table).  Ticks that overlap in time
 * need their own table and workspace. */
int nlos_tick_launch(const nlos_tick_caps* caps, const void* table, void* ws, size_t ws_bytes, void* stream);

/*
 * The same tick as one HIP graph, instantiated once for a table and a
 * workspace: create builds it (copy node, three kernel nodes; this is the
 * only step that creates runtime objects), then each tick is nlos_tick_plan
 * into `table` followed by nlos_tick_graph_launch, which sets the pair
 * node's grid to the tick's item count (hipGraphExecKernelNodeSetParams)
 * and launches the graph: one launch per tick, nothing allocated.  A graph
 * and its table/workspace serve one tick at a time (wait for the previous
 * launch to pass before planning the next); ticks in flight together need a
 * graph each.  destroy frees the graph (NULL is a no-op).
 */
typedef struct nlos_tick_graph nlos_tick_graph;

int nlos_tick_graph_create(const nlos_tick_caps* caps, const void* table, void* ws, size_t ws_bytes,
                           nlos_tick_graph** graph);

int nlos_tick_graph_launch(nlos_tick_graph* graph, void* stream);

int nlos_tick_graph_destroy(nlos_tick_graph* graph);

/*
 * Smooth time response and its adjoint (confocal only).  The hard forward
 * bins each arrival, so its output does not vary smoothly with the patch
 * depths.  The smooth forward gives every pair the continuous, normalised
 * Gaussian response of the detector jitter (Section 2, temporal jitter;
 * sigma = FWHM / (2 sqrt(2 ln 2)) / dt bins) instead of hard binning plus
 * blur:
 *     tau_s[s][k] = sum_p w_sp N(k + 1/2 - u_sp)  for |k - floor(u_sp)| <= Rs,
 * Rs = ceil(6 sigma), 0 <= k < T, with w and u exactly as in nlos_forward.
 * Arrivals outside the window still reach in-window bins within Rs.
 * Requires fwhm_ps > 0 and sigma * 6 <= 1024 bins; one T-bin histogram of
 * 64-bit bins must fit in LDS (T <= ~20000).  For Rs of 12, 16 or 20 bins
 * (when the rows fit in LDS) the Gaussian samples are taken as a series in
 * the sub-bin offset t = u - floor(u) - 1/2: each pair adds w (-t)^m,
 * m <= 7 (Rs = 12) or m <= 5 (Rs = 16, 20), and the rows are convolved with
 * N^(m) / m!; the series is within 7e-8 resp. 1.2e-6 (relative L2 over the
 * support) of the samples.
 */
int nlos_forward_smooth_workspace_bytes(const nlos_params* p, int32_t n_patches, size_t* bytes);

/* Smooth forward; arguments as nlos_forward (confocal output [nx][ny][T]). */
int nlos_forward_smooth(const nlos_params* p, const float* patches, int32_t n_patches,
                        const int32_t* n_active, float* out, void* ws, size_t ws_bytes, void* stream);

/* Workspace of nlos_adjoint: per-record partial gradients (fp64) of each
 * range of scan points; for support radii ceil(6 sigma) of 12, 16 or 20 bins
 * it starts with the correlations of the upstream gradient rows with the
 * Gaussian's derivatives (fp32 [nx*ny][n][T + 2 radius], n = 9 at radius 12,
 * 7 at 16 and 20).  256-byte aligned. */
int nlos_adjoint_workspace_bytes(const nlos_params* p, int32_t n_patches, size_t* bytes);

/*
 * Adjoint of the smooth forward with respect to the patch records: given the
 * upstream gradient G = dL/dtau_s (device float [nx][ny][T], 16-byte
 * aligned), writes for every record p (device float [n_patches][8], 16-byte
 * aligned)
 *     { 0, 0, dL/dz, dL/da, dL/dn_x, dL/dn_y, dL/dn_z, 0 }
 * (records past *n_active get zeros).  Per pair dL/dw = sum_k G N(x_k) and
 * dL/du = w sum_k G (x_k / sigma^2) N(x_k), x_k = k + 1/2 - u, chained
 * through w(z, n, a) and u(z).  The step of the support with floor(u) is
 * not differentiated (below the tail at 6 sigma).  For support radii of 12,
 * 16 or 20 bins both sums are evaluated as series in the sub-bin offset
 * (t = u - floor(u) - 1/2, terms up to t^7 at radius 12, t^5 at 16 and 20)
 * of precomputed correlations of G with the Gaussian's derivatives.  Deterministic: partial sums per scan
 * range are added in a fixed order.
 */
int nlos_adjoint(const nlos_params* p, const float* patches, int32_t n_patches, const int32_t* n_active,
                 const float* grad_out, float* grad_patches, void* ws, size_t ws_bytes, void* stream);

/* Workspace of nlos_patches_adjoint: 12 bytes per pixel. */
int nlos_patches_adjoint_workspace_bytes(const nlos_grid* g, size_t* bytes);

/*
 * Adjoint of nlos_patches_from_depth: record gradients (from nlos_adjoint,
 * records as written by nlos_patches_from_depth for the same maps and flags)
 * -> gradients of the depth map (device float [nx][ny], every pixel: a
 * masked pixel's depth still enters its neighbours' normals) and of the
 * albedo map (device float [nx][ny] or NULL; zero where no record).  The
 * chain runs through z = D, n = (D_x, D_y, -1) / len and a = albedo * area,
 * area = dx dy len with NLOS_F_COSINES (dx dy without), and the central /
 * one-sided differences that give D_x and D_y.  The mask is not needed:
 * each record carries its pixel index.
 */
int nlos_patches_adjoint(const nlos_grid* g, const float* depth, const float* albedo, uint32_t flags,
                         const float* patches, const int32_t* n_active, const float* grad_patches,
                         float* grad_depth, float* grad_albedo, void* ws, size_t ws_bytes, void* stream);

/*
 * Poisson noise of a frame (Algorithm 1 step 2.4, applied after the blur of
 * step 2.3):  T = Poisson(tau * sigma_n) / sigma_n with
 * sigma_n = Var(tau) / 10^(nr / 10), Var the population variance of the whole
 * frame (every histogram and bin).
 */
/* Workspace of nlos_noise_scale: fp64 moments of up to 1024 blocks. */
int nlos_noise_scale_workspace_bytes(int64_t n, size_t* bytes);

/* stats (device double[3], 8-byte aligned) <- { mean, Var, sigma_n } of the n
 * floats of tau (device); fp64 throughout, merged in a fixed order
 * (reproducible). */
int nlos_noise_scale(const float* tau, int64_t n, double nr_db, double* stats, void* ws, size_t ws_bytes,
                     void* stream);

/*
 * out[i] = Poisson(max(tau[i], 0) * s) / s for the n elements, s = *sigma_n
 * (device double, e.g. stats + 2); out is all zeros when s <= 0 or not finite.
 * out may be tau (in place).  Uniform t of element i is word t mod 4 of
 * Philox4x64-10 (Salmon et al., SC 2011) at counter (i, t / 4, 0, 0) and key
 * (seed, 0x4e4c4f53), mapped to [0, 1) by its top 53 bits.  Counts come from
 * inversion by sequential search for lambda < 10 and from Hormann's
 * transformed rejection with squeeze (PTRS, 1993) above; exp, log and log k!
 * follow fixed recipes of IEEE basic operations, so the counts are a
 * deterministic function of (tau[i], s, seed, i).
 */
int nlos_poisson_noise(const float* tau, int64_t n, const double* sigma_n, uint64_t seed, float* out,
                       void* stream);

/*
 * The paper's FFT ("light-cone") forward route (Section 2, Eq. (3)-(5);
 * Algorithm 1 steps 1.1-2.3) as a cross-check of the direct operator: a
 * confocal N x N scan (relay.nx == relay.ny, half_x == half_y = w) whose
 * depth map is the same N x N grid, no stand-off, flags 0 (Eq. (1) without
 * cosines), T = M a power of two.  Steps: depth layer j = floor(D / dz),
 * dz = c dt / 2; fold to u = J^2 (J = j + 1) with weight 1 / J and pairwise
 * means down to M samples; 3-D convolution (fp64 FFTs on the zero-padded
 * (2N, 2N, 2M) grid) with the cone that puts lateral offset n cells (x = n / N)
 * at layer round((4 slope)^2 (x^2 + y^2) M), slope = w / (M c dt), layers past
 * the window dropped; back to time bins by the mean over each bin's v-span
 * [j^2, (j+1)^2) divided by (J dz)^3; Gaussian jitter.  Output float
 * [N][N][M].  The first call for a size creates and keeps an FFT plan (the
 * FFT library allocates its tables then); later calls allocate nothing.  A
 * failure inside the FFT library gives NLOS_EHIP with nlos_last_hip_error()
 * = -1.  The workspace (two complex fp64 volumes + FFT work) is about
 * 32 * (2N)^2 * 2M bytes, 256-byte aligned.
 */
int nlos_lct_workspace_bytes(const nlos_params* p, size_t* bytes);

int nlos_lct_forward(const nlos_params* p, const float* depth, const float* albedo, const uint8_t* mask,
                     float* out, void* ws, size_t ws_bytes, void* stream);

/*
 * Launch planning.  The forward groups histograms in units (confocal: TX x TY
 * scan points; non-confocal: TL laser points x TX x TY detectors; supported:
 * confocal 4x4, 4x2, 2x2, 2x1, 1x1; non-confocal TL,TX,TY = 2,2,2 / 2,1,2 /
 * 1,1,2 / 1,1,1).  A tuning table, measured by the autotuner, names the unit
 * per class of problems; the first matching entry whose unit fits in LDS is
 * used, otherwise the built-in rule (largest unit that fits and still gives
 * one workgroup per CU).  The table is the library's only shared state: it is
 * copied, read under a lock, and replaced as a whole.
 */
typedef struct nlos_tuning_entry {
    int32_t confocal;        /* 1: confocal, 0: non-confocal */
    int32_t t_min, t_max;    /* n_bins range, inclusive */
    int64_t h_min, h_max;    /* histogram count range (S or L*S), inclusive */
    int32_t tl, tx, ty;      /* unit */
} nlos_tuning_entry;

typedef struct nlos_plan_info {
    int32_t tl, tx, ty;      /* unit */
    int32_t pair;            /* 1: two units per workgroup over the whole window */
    int32_t n_split;         /* patch ranges per unit pair */
    int32_t n_windows;       /* time windows (1 unless a histogram exceeds LDS) */
    int64_t workgroups;
    int64_t lds_bytes;
} nlos_plan_info;

/* Replace the tuning table (n = 0 clears it).  Entries naming an unsupported
 * unit or an empty range are rejected (the table is then left unchanged). */
int nlos_set_tuning(const nlos_tuning_entry* entries, int32_t n);

/* The plan nlos_forward would use for these parameters (host only). */
int nlos_get_plan(const nlos_params* p, int32_t n_patches, nlos_plan_info* info);

/*
 * Test hook: the bin index of every (histogram, record) pair, decided by the
 * same device functions and the same fp32-then-fp64 rule as nlos_forward.
 *   bins    device int32 [H][n_patches], H = histograms of the output
 *           (S confocal, L*S non-confocal); records at or beyond *n_active get
 *           INT32_MIN.  Bins outside [0, T) are still reported (the exact
 *           floor of the fp64 arrival), so every pair can be checked.
 *   u_fast  device double [H][n_patches] or NULL: the fp32 arrival (in bins)
 *           the kernels use to decide (exactly representable in fp64).
 *   u_exact device double [H][n_patches] or NULL: the fp64 arrival.
 * Limits: H * n_patches <= 2^31.
 */
int nlos_debug_bins(const nlos_params* p, const float* patches, int32_t n_patches,
                    const int32_t* n_active, int32_t* bins, double* u_fast, double* u_exact,
                    void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NLOS_H */
