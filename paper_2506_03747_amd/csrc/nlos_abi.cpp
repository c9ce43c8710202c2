// C ABI layer of the transient NLOS forward operator: argument checks,
// jitter taps, the launch plan (tile shape, time windows, patch split) and
// error reporting.  Every arithmetic step of the operator runs in the HIP
// kernels; this file only prepares their arguments.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "nlos.h"
#include "nlos_internal.h"

namespace {

thread_local int g_last_hip = 0;

constexpr double kC = 299792458.0;   // m/s
constexpr size_t kLdsMax = 163840;   // LDS per workgroup on gfx950
constexpr int kQueueDefault = 2048;
constexpr int kTargetBlocks = 256;   // one workgroup per CU

int hip_fail(hipError_t e)
{
    g_last_hip = (int)e;
    return NLOS_EHIP;
}

int device_check()
{
    static std::once_flag once;
    static int status = NLOS_OK;
    std::call_once(once, [] {
        int n = 0;
        const hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || n <= 0) {
            status = NLOS_ENODEV;
            g_last_hip = (int)e;
        }
    });
    return status;
}

bool finite(double v) { return std::isfinite(v); }

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

bool grid_ok(const nlos_grid* g)
{
    return g && g->nx >= 1 && g->ny >= 1 && g->nx <= NLOS_MAX_GRID && g->ny <= NLOS_MAX_GRID &&
           finite(g->half_x) && finite(g->half_y) && g->half_x > 0 && g->half_y > 0 &&
           finite(g->cx) && finite(g->cy);
}

nlos::Axis axis(double half, double c, int32_t n)
{
    nlos::Axis a;
    a.a0 = c - half;
    a.step = (2.0 * half) / (double)n;
    a.n = n;
    return a;
}

// Jitter taps (Section 2): sigma in bins = FWHM / (2 sqrt(2 ln 2)) / dt,
// R = ceil(2 sigma), normalised Gaussian; FWHM = 0 -> identity.
int jitter_taps(double fwhm_ps, double bin_ps, float* taps, int32_t* R_out)
{
    if (fwhm_ps == 0.0) {
        taps[0] = 1.0f;
        *R_out = 0;
        return NLOS_OK;
    }
    const double sigma = fwhm_ps / (2.0 * std::sqrt(2.0 * std::log(2.0))) / bin_ps;
    const double rr = std::ceil(2.0 * sigma);
    if (!(rr <= (double)NLOS_MAX_RADIUS)) return NLOS_EINVAL;
    const int R = (int)rr;
    double g[nlos::kMaxTaps];
    double sum = 0.0;
    for (int j = -R; j <= R; ++j) {
        g[j + R] = std::exp(-(double)j * (double)j / (2.0 * sigma * sigma));
        sum += g[j + R];
    }
    for (int i = 0; i < 2 * R + 1; ++i) taps[i] = (float)(g[i] / sum);
    *R_out = R;
    return NLOS_OK;
}

bool is_confocal(const nlos_params* p) { return p->laser.nx == 0 && p->laser.ny == 0; }

int params_ok(const nlos_params* p)
{
    if (!p || !grid_ok(&p->relay)) return NLOS_EINVAL;
    if (!is_confocal(p) && !grid_ok(&p->laser)) return NLOS_EINVAL;
    if (!finite(p->standoff_m) || p->standoff_m < 0) return NLOS_EINVAL;
    if (!finite(p->bin_ps) || !(p->bin_ps > 0)) return NLOS_EINVAL;
    if (p->n_bins < 1 || p->n_bins > NLOS_MAX_BINS) return NLOS_EINVAL;
    if (!finite(p->fwhm_ps) || p->fwhm_ps < 0) return NLOS_EINVAL;
    if ((p->flags & ~NLOS_F_COSINES) != 0) return NLOS_EINVAL;
    return NLOS_OK;
}

int64_t n_hist(const nlos_params* p)
{
    const int64_t S = (int64_t)p->relay.nx * p->relay.ny;
    const int64_t L = is_confocal(p) ? 1 : (int64_t)p->laser.nx * p->laser.ny;
    return S * L;
}

// Fill the kernel arguments common to the pair kernels and the bin export.
int fill_args(const nlos_params* p, const float* patches, int32_t n_patches, const int32_t* n_active,
              float* out, nlos::FwdArgs* a)
{
    std::memset(a, 0, sizeof(*a));
    a->patches = reinterpret_cast<const float4*>(patches);
    a->n_active = n_active;
    a->n_cap = n_patches;
    a->out = out;
    a->rx = axis(p->relay.half_x, p->relay.cx, p->relay.nx);
    a->ry = axis(p->relay.half_y, p->relay.cy, p->relay.ny);
    if (is_confocal(p)) {
        a->lx = a->rx;
        a->ly = a->ry;
    } else {
        a->lx = axis(p->laser.half_x, p->laser.cx, p->laser.nx);
        a->ly = axis(p->laser.half_y, p->laser.cy, p->laser.ny);
    }
    a->cx = p->relay.cx;
    a->cy = p->relay.cy;
    a->s = p->standoff_m;
    a->inv = 1.0 / (kC * (p->bin_ps * 1e-12));
    a->inv_f = (float)a->inv;
    a->inv2_f = (float)(2.0 * a->inv);
    a->T = p->n_bins;
    // Guard half-width: the fp32 arrival is within a few ulp (relative) of
    // the fp64 one for pairs near the window; 16 ulp of T + 2 bins keeps a
    // factor >= 2 over the bound derived for the fast path.
    a->delta = (float)(16.0 * ((double)p->n_bins + 2.0) * std::ldexp(1.0, -24));
    a->two_delta = 2.0f * a->delta;
    // stand-in patch for idle lanes: beyond every wall point by (T + 64) / (2 inv)
    // metres, so both legs add up to at least T + 64 bins
    double reach = p->relay.cx + p->relay.half_x;
    if (!is_confocal(p)) reach = std::max(reach, p->laser.cx + p->laser.half_x);
    a->dummy_x = (float)(reach + ((double)p->n_bins + 64.0) / (2.0 * a->inv) + 1.0);
    a->cosines = (p->flags & NLOS_F_COSINES) ? 1 : 0;
    return jitter_taps(p->fwhm_ps, p->bin_ps, a->taps, &a->R);
}

struct Cand {
    int tl, tx, ty;
};

int64_t stats_count(int32_t n_patches) { return ((int64_t)n_patches + nlos::kStatBlock - 1) / nlos::kStatBlock; }

// Launch plan.  Histograms are grouped in units (candidate shapes below,
// largest first); a workgroup owns two units when the histograms of both fit
// in the 160 KB of LDS over the whole window (taking the largest shape that
// still gives at least one workgroup per CU), else one unit of one histogram
// over a window of bins (time windows).  Patches are split over workgroups
// when there are fewer workgroups than CUs.  Units are ordered by estimated
// work inside the kernel when their count keeps that cheap.
// Tuning table (nlos_set_tuning): the unit shape to use per (geometry,
// window length, histogram count) class, found by measurement.  Read under a
// lock by every plan; replaced as a whole.
std::mutex g_tune_mu;
std::vector<nlos_tuning_entry> g_tune;

bool tuned_unit(bool conf, int32_t T, int64_t H, Cand* c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& e : g_tune) {
        if ((e.confocal != 0) != conf || T < e.t_min || T > e.t_max || H < e.h_min || H > e.h_max) continue;
        c->tl = e.tl;
        c->tx = e.tx;
        c->ty = e.ty;
        return true;
    }
    return false;
}

int make_plan(const nlos_params* p, int32_t n_patches, int R, int64_t target, nlos::Plan* plan)
{
    const bool conf = is_confocal(p);
    static const Cand conf_c[] = {{1, 4, 4}, {1, 4, 2}, {1, 2, 2}, {1, 2, 1}, {1, 1, 1}};
    static const Cand nc_c[] = {{2, 2, 2}, {2, 1, 2}, {1, 1, 2}, {1, 1, 1}};
    const Cand* cands = conf ? conf_c : nc_c;
    const int nc = conf ? 5 : 4;
    // a tuned shape comes first among the candidates (it is used when its
    // histograms fit in LDS; the usual rule decides otherwise)
    Cand tuned_list[6];
    Cand tuned;
    if (tuned_unit(conf, p->n_bins, n_hist(p), &tuned)) {
        int k = 0;
        tuned_list[k++] = tuned;
        for (int i = 0; i < nc; ++i)
            if (cands[i].tl != tuned.tl || cands[i].tx != tuned.tx || cands[i].ty != tuned.ty) tuned_list[k++] = cands[i];
        cands = tuned_list;
    }
    const bool forced = cands == tuned_list;
    const int T = p->n_bins;
    const int64_t L = conf ? 1 : (int64_t)p->laser.nx * p->laser.ny;
    int q_cap = kQueueDefault;

    // u64 bins per histogram row (at least tl + 1: bin tl is a spare that
    // takes the pairs just past the window), even, and reused by the flush as
    // a float row of flush_row_words(tl, RM) words (RM = the jitter radius
    // rounded up to a compiled variant), so 2 * stride >= that
    const int RM = nlos::jitter_rm(R);
    auto stride_of = [RM](int tl) {
        return std::max((tl + 2) & ~1, ((nlos::flush_row_words(tl, RM) + 1) / 2 + 1) & ~1);
    };
    auto units_of = [&](const Cand& c) {
        return ((L + c.tl - 1) / c.tl) * (int64_t)((p->relay.nx + c.tx - 1) / c.tx) *
               (int64_t)((p->relay.ny + c.ty - 1) / c.ty);
    };
    int chosen = -1, largest = -1;
    for (int i = 0; i < nc; ++i) {
        const int slots = 2 * cands[i].tl * cands[i].tx * cands[i].ty;
        if (nlos::lds_bytes_for(slots, stride_of(T), q_cap) > kLdsMax) continue;
        if (largest < 0) largest = i;
        if ((forced && i == 0) || (units_of(cands[i]) + 1) / 2 >= target) {
            chosen = i;
            break;
        }
    }
    if (chosen < 0) chosen = largest;
    int tw = T, n_tw = 1, pair = 1;
    if (chosen < 0) {
        // even two single histograms do not fit: one histogram per workgroup
        // over a window of the time axis
        chosen = nc - 1;
        pair = 0;
        q_cap = 1024;
        const size_t fixed = nlos::lds_bytes_for(1, 0, q_cap);
        const int tl_max = (int)((kLdsMax - fixed - 256) / 8) & ~1;
        tw = tl_max - 2 * R;
        if (tw < 64) return NLOS_EINVAL;
        tw &= ~3;
        n_tw = (T + tw - 1) / tw;
    }
    const Cand c = cands[chosen];
    const int tl_len = (n_tw == 1) ? T : std::min(T, tw + 2 * R);
    const int slots = (pair ? 2 : 1) * c.tl * c.tx * c.ty;
    plan->tl = c.tl;
    plan->tx = c.tx;
    plan->ty = c.ty;
    plan->pair = pair;
    plan->tw = tw;
    plan->n_tw = n_tw;
    plan->stride = stride_of(tl_len);
    plan->q_cap = q_cap;
    plan->lds_bytes = nlos::lds_bytes_for(slots, plan->stride, q_cap);
    if (plan->lds_bytes > kLdsMax || plan->stride <= tl_len) return NLOS_EINVAL;
    const int64_t units = units_of(c);
    const int64_t groups = pair ? (units + 1) / 2 : units;
    // torus-shift pairing needs an even side in the unit plane (x or y)
    const int64_t utx = (p->relay.nx + c.tx - 1) / c.tx, uty = (p->relay.ny + c.ty - 1) / c.ty;
    plan->plan = (pair && ((utx % 2) == 0 || (uty % 2) == 0)) ? 1 : 0;
    plan->groups = groups;
    const int64_t tiles = groups * n_tw;
    int64_t split = 1;
    if (tiles < target) {
        split = (target + tiles - 1) / tiles;
        const int64_t by_patches = std::max<int64_t>(1, n_patches / nlos::kBlock);
        split = std::min(split, by_patches);
    }
    plan->n_split = (int)split;
    plan->n_blocks = tiles * split;
    if (plan->n_blocks > 0x7fffffff || units > 0x7fffffff) return NLOS_EINVAL;
    return NLOS_OK;
}

// Workspace of nlos_forward: record summaries, then the planned unit pairs.
size_t stats_bytes(int32_t n_patches)
{
    return ((size_t)stats_count(n_patches) * sizeof(nlos::ChunkStat) + 255) & ~(size_t)255;
}

int forward_workspace(const nlos_params* p, int32_t n_patches, size_t* bytes, nlos::Plan* plan_out,
                      int64_t target = kTargetBlocks)
{
    float taps[nlos::kMaxTaps];
    int32_t R = 0;
    int rc = jitter_taps(p->fwhm_ps, p->bin_ps, taps, &R);
    if (rc != NLOS_OK) return rc;
    nlos::Plan plan;
    rc = make_plan(p, n_patches, R, target, &plan);
    if (rc != NLOS_OK) return rc;
    *bytes = stats_bytes(n_patches);
    if (plan_out) *plan_out = plan;
    return NLOS_OK;
}

// Checks of one forward request, its plan (for `target` workgroups) and its
// kernel arguments (all but the summaries pointer); *ws_need = workspace.
int setup_forward(const nlos_params* p, const float* patches, int32_t n_patches, const int32_t* n_active,
                  float* out, int64_t target, nlos::FwdArgs* a, nlos::Plan* plan, size_t* ws_need)
{
    int rc = params_ok(p);
    if (rc != NLOS_OK) return rc;
    if (n_patches < 0 || n_patches > NLOS_MAX_PATCHES || !out) return NLOS_EINVAL;
    if (n_patches > 0 && !patches) return NLOS_EINVAL;
    if ((patches && !aligned(patches, 16)) || !aligned(out, 16) || (n_active && !aligned(n_active, 4)))
        return NLOS_EINVAL;
    rc = forward_workspace(p, n_patches, ws_need, plan, target);
    if (rc != NLOS_OK) return rc;
    rc = fill_args(p, patches, n_patches, n_active, out, a);
    if (rc != NLOS_OK) return rc;
    const bool conf = is_confocal(p);
    a->out_len = n_hist(p) * (int64_t)p->n_bins;
    a->tiles_l = conf ? 1 : (p->laser.nx * p->laser.ny + plan->tl - 1) / plan->tl;
    a->tiles_x = (p->relay.nx + plan->tx - 1) / plan->tx;
    a->tiles_y = (p->relay.ny + plan->ty - 1) / plan->ty;
    a->n_units = a->tiles_l * a->tiles_x * a->tiles_y;
    a->pair = plan->pair;
    a->plan = plan->plan;
    a->stats = nullptr;
    a->n_stats = (int32_t)stats_count(n_patches);
    a->n_split = plan->n_split;
    a->tw = plan->tw;
    a->n_tw = plan->n_tw;
    a->stride = plan->stride;
    a->q_cap = plan->q_cap;
    a->atomic_out = plan->n_split > 1 ? 1 : 0;
    return NLOS_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Host table of a batched forward call, copied as one block to the start of
// the device workspace: per-request kernel arguments, then the work lists
// (records summaries, output zeroing, one list per kernel variant).
struct FwdBatch {
    struct Group {
        int tl, tx, ty;
        bool conf, cos, pair;
        std::vector<int32_t> req;
        std::vector<int64_t> first;
        int64_t n_blocks = 0;
        size_t lds = 0;
        size_t req_off = 0, first_off = 0;
    };
    std::vector<nlos::FwdArgs> args;
    std::vector<nlos::Plan> plans;
    std::vector<Group> groups;
    std::vector<int32_t> stat_req, fill_req;
    std::vector<int64_t> stat_first;
    int64_t stat_blocks = 0;
    size_t tab_off = 0, stat_req_off = 0, stat_first_off = 0, fill_req_off = 0;
    size_t table_bytes = 0, ws_bytes = 0;
    std::vector<size_t> stats_off;
};

// Plan every request (each gets a share of the GPU's workgroups in proportion
// to its pairs), group them by kernel variant and order each group by
// decreasing work per workgroup, so the longest workgroups start first.
int plan_batch(const nlos_request* reqs, int32_t n, FwdBatch* b)
{
    if (n < 0 || (n > 0 && !reqs)) return NLOS_EINVAL;
    b->args.resize(n);
    b->plans.resize(n);
    b->stats_off.resize(n);
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
        if (params_ok(&reqs[i].params) != NLOS_OK) return NLOS_EINVAL;
        total += (double)n_hist(&reqs[i].params) * (double)std::max(reqs[i].n_patches, 1);
    }
    std::vector<double> work(n);
    for (int i = 0; i < n; ++i) {
        const nlos_request& r = reqs[i];
        const double pairs = (double)n_hist(&r.params) * (double)std::max(r.n_patches, 1);
        const int64_t target = std::max<int64_t>(1, (int64_t)std::ceil(kTargetBlocks * pairs / total));
        size_t need = 0;
        const int rc = setup_forward(&r.params, r.patches, r.n_patches, r.n_active, r.out, target, &b->args[i],
                                     &b->plans[i], &need);
        if (rc != NLOS_OK) return rc;
        work[i] = pairs / (double)std::max<int64_t>(1, b->plans[i].n_blocks);
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    for (int i : order) {
        const nlos::Plan& pl = b->plans[i];
        const bool conf = is_confocal(&reqs[i].params);
        const bool cos = b->args[i].cosines != 0;
        FwdBatch::Group* g = nullptr;
        for (auto& h : b->groups)
            if (h.tl == pl.tl && h.tx == pl.tx && h.ty == pl.ty && h.conf == conf && h.cos == cos &&
                h.pair == (pl.pair != 0))
                g = &h;
        if (!g) {
            b->groups.emplace_back();
            g = &b->groups.back();
            g->tl = pl.tl;
            g->tx = pl.tx;
            g->ty = pl.ty;
            g->conf = conf;
            g->cos = cos;
            g->pair = pl.pair != 0;
        }
        if (pl.n_blocks > 0) {
            g->req.push_back(i);
            g->first.push_back(g->n_blocks);
            g->n_blocks += pl.n_blocks;
            g->lds = std::max(g->lds, pl.lds_bytes);
        }
        if (b->args[i].n_stats > 0) {
            b->stat_req.push_back(i);
            b->stat_first.push_back(b->stat_blocks);
            b->stat_blocks += b->args[i].n_stats;
        }
        if (b->args[i].atomic_out) b->fill_req.push_back(i);
    }
    // table layout
    size_t off = 0;
    b->tab_off = off;
    off = align_up(off + sizeof(nlos::FwdArgs) * (size_t)n, 16);
    b->stat_req_off = off;
    off = align_up(off + 4 * b->stat_req.size(), 16);
    b->stat_first_off = off;
    off = align_up(off + 8 * b->stat_first.size(), 16);
    b->fill_req_off = off;
    off = align_up(off + 4 * b->fill_req.size(), 16);
    for (auto& g : b->groups) {
        g.req_off = off;
        off = align_up(off + 4 * g.req.size(), 16);
        g.first_off = off;
        off = align_up(off + 8 * g.first.size(), 16);
    }
    b->table_bytes = align_up(off, 256);
    off = b->table_bytes;
    for (int i = 0; i < n; ++i) {
        b->stats_off[i] = off;
        off = align_up(off + sizeof(nlos::ChunkStat) * (size_t)b->args[i].n_stats, 256);
    }
    b->ws_bytes = off;
    return NLOS_OK;
}

template <typename T>
void put(unsigned char* base, size_t off, const std::vector<T>& v)
{
    if (!v.empty()) std::memcpy(base + off, v.data(), sizeof(T) * v.size());
}

thread_local std::vector<unsigned char> g_table;

// Copy `bytes` of host table to the device workspace on `st`; the table is
// the caller's buffer when given, else this thread's pageable buffer.
hipError_t upload_table(void* ws, const unsigned char* table, size_t bytes, hipStream_t st)
{
    return hipMemcpyAsync(ws, table, bytes, hipMemcpyHostToDevice, st);
}

// Geometry batch: per-map arguments and the enumeration-block prefix.
struct GeomBatch {
    std::vector<nlos::GeomArgs> args;
    std::vector<int64_t> first;
    int64_t n_blocks = 0;
    size_t tab_off = 0, first_off = 0, table_bytes = 0, ws_bytes = 0;
    std::vector<size_t> counts_off;
};

int geom_args(const nlos_grid* g, const float* depth, const float* albedo, const uint8_t* mask, uint32_t flags,
              float* patches, int32_t* n_active, nlos::GeomArgs* a)
{
    if (!grid_ok(g) || !depth || !patches || !n_active) return NLOS_EINVAL;
    if ((int64_t)g->nx * g->ny > NLOS_MAX_PATCHES) return NLOS_EINVAL;
    if ((flags & ~NLOS_F_COSINES) != 0) return NLOS_EINVAL;
    if (!aligned(patches, 16) || !aligned(depth, 4) || (albedo && !aligned(albedo, 4)) || !aligned(n_active, 4))
        return NLOS_EINVAL;
    std::memset(a, 0, sizeof(*a));
    a->depth = depth;
    a->albedo = albedo;
    a->mask = mask;
    a->patches = reinterpret_cast<float4*>(patches);
    a->n_active = n_active;
    a->ax = axis(g->half_x, g->cx, g->nx);
    a->ay = axis(g->half_y, g->cy, g->ny);
    a->hx = (float)a->ax.step;
    a->hy = (float)a->ay.step;
    a->bx = (g->nx + nlos::kBlockPx - 1) / nlos::kBlockPx;
    a->by = (g->ny + nlos::kBlockPx - 1) / nlos::kBlockPx;
    a->n_enum = (int64_t)nlos::kBlockPx * nlos::kBlockPx * a->bx * a->by;
    a->n_blocks = (int32_t)((a->n_enum + nlos::kGeomBlock - 1) / nlos::kGeomBlock);
    a->cosines = (flags & NLOS_F_COSINES) ? 1 : 0;
    return NLOS_OK;
}

int plan_geom_batch(const nlos_depth_request* reqs, int32_t n, GeomBatch* b)
{
    if (n < 0 || (n > 0 && !reqs)) return NLOS_EINVAL;
    b->args.resize(n);
    b->first.resize(n);
    b->counts_off.resize(n);
    for (int i = 0; i < n; ++i) {
        const nlos_depth_request& r = reqs[i];
        const int rc = geom_args(&r.grid, r.depth, r.albedo, r.mask, r.flags, r.patches, r.n_active, &b->args[i]);
        if (rc != NLOS_OK) return rc;
        b->first[i] = b->n_blocks;
        b->n_blocks += b->args[i].n_blocks;
    }
    size_t off = 0;
    b->tab_off = 0;
    off = align_up(sizeof(nlos::GeomArgs) * (size_t)n, 16);
    b->first_off = off;
    off = align_up(off + 8 * (size_t)n, 256);
    b->table_bytes = off;
    for (int i = 0; i < n; ++i) {
        b->counts_off[i] = off;
        off = align_up(off + 8 * (size_t)b->args[i].n_blocks, 256);
    }
    b->ws_bytes = off;
    return NLOS_OK;
}

// ---------------------------------------------------------------------------
// Smooth forward and adjoint (confocal).
constexpr int kSmoothMaxRadius = 1024;

int smooth_setup(const nlos_params* p, const float* patches, int32_t n_patches, const int32_t* n_active,
                 nlos::SmoothArgs* a)
{
    int rc = params_ok(p);
    if (rc != NLOS_OK) return rc;
    if (!is_confocal(p) || !(p->fwhm_ps > 0.0)) return NLOS_EINVAL;
    if (n_patches < 0 || n_patches > NLOS_MAX_PATCHES) return NLOS_EINVAL;
    if (n_patches > 0 && !patches) return NLOS_EINVAL;
    if ((patches && !aligned(patches, 16)) || (n_active && !aligned(n_active, 4))) return NLOS_EINVAL;
    std::memset(a, 0, sizeof(*a));
    const double sigma = p->fwhm_ps / (2.0 * std::sqrt(2.0 * std::log(2.0))) / p->bin_ps;
    const double rs = std::ceil(6.0 * sigma);
    if (!(rs <= (double)kSmoothMaxRadius) || !(sigma > 1e-3)) return NLOS_EINVAL;
    a->patches = reinterpret_cast<const float4*>(patches);
    a->n_active = n_active;
    a->n_cap = n_patches;
    a->rx = axis(p->relay.half_x, p->relay.cx, p->relay.nx);
    a->ry = axis(p->relay.half_y, p->relay.cy, p->relay.ny);
    a->cx = p->relay.cx;
    a->cy = p->relay.cy;
    a->s = p->standoff_m;
    a->inv = 1.0 / (kC * (p->bin_ps * 1e-12));
    a->sigma = (float)sigma;
    a->norm = (float)(1.0 / (sigma * std::sqrt(2.0 * 3.14159265358979323846)));
    a->inv_s2 = (float)(1.0 / (sigma * sigma));
    a->c1 = (float)std::exp(-1.0 / (sigma * sigma));
    a->T = p->n_bins;
    a->Rs = (int32_t)rs;
    a->cosines = (p->flags & NLOS_F_COSINES) ? 1 : 0;
    return NLOS_OK;
}

struct SmoothPlan {
    int tx, ty;
    int64_t tiles, n_blocks;
    size_t lds;
    int moments;   // 1: k_smooth_mom (moment rows), 0: k_smooth (taps)
    int stride;    // u64 bins per LDS row
};

size_t smooth_lds(int nh, int stride) { return (size_t)nh * stride * 8 + (size_t)nh * 12 + 64 * 4 + 64; }

int smooth_plan(const nlos_params* p, int32_t n_patches, int rs, SmoothPlan* sp, int* split)
{
    static const int shapes[5][2] = {{4, 4}, {4, 2}, {2, 2}, {2, 1}, {1, 1}};
    const int T = p->n_bins;
    // moments of the sub-bin offset when the support radius has a compiled
    // variant and the moment rows (with a halo of rs bins on both sides) fit
    sp->moments = 0;
    sp->stride = T;
    if (nlos::smooth_moments_radius(rs)) {
        int stride = (T + 2 * rs + 1) & ~1;
        const nlos::SmoothMomShape sh = nlos::smooth_mom_shape(rs);
        const int64_t rows = (int64_t)sh.points * sh.moments;
        // rows that take more than half the LDS leave one workgroup per CU:
        // then the compile-time pitch, which costs no occupancy
        if ((size_t)rows * stride * 8 + 2048 > kLdsMax / 2 && stride <= nlos::smooth_mom_pitch(rs))
            stride = nlos::smooth_mom_pitch(rs);
        const size_t lds = (size_t)rows * stride * 8 + 2048;
        if (lds <= kLdsMax && rows * (T + 2 * rs) <= 24 * (int64_t)nlos::kBlock) {
            sp->moments = 1;
            sp->stride = stride;
            sp->tx = sh.points;
            sp->ty = 1;
            sp->tiles = (int64_t)((p->relay.nx + sp->tx - 1) / sp->tx) * p->relay.ny;
            int64_t sv = 1;
            if (sp->tiles < kTargetBlocks) {
                sv = (kTargetBlocks + sp->tiles - 1) / sp->tiles;
                sv = std::min<int64_t>(sv, std::max<int64_t>(1, n_patches / nlos::kBlock));
            }
            *split = (int)sv;
            sp->n_blocks = sp->tiles * sv;
            sp->lds = lds;
            return NLOS_OK;
        }
    }
    int chosen = -1, largest = -1;
    for (int i = 0; i < 5; ++i) {
        if (smooth_lds(shapes[i][0] * shapes[i][1], T) > kLdsMax) continue;
        if (largest < 0) largest = i;
        const int64_t tiles = (int64_t)((p->relay.nx + shapes[i][0] - 1) / shapes[i][0]) *
                              ((p->relay.ny + shapes[i][1] - 1) / shapes[i][1]);
        if (tiles >= kTargetBlocks) {
            chosen = i;
            break;
        }
    }
    if (chosen < 0) chosen = largest;
    if (chosen < 0) return NLOS_EINVAL;   // one histogram of T bins does not fit in LDS
    sp->tx = shapes[chosen][0];
    sp->ty = shapes[chosen][1];
    sp->tiles = (int64_t)((p->relay.nx + sp->tx - 1) / sp->tx) * ((p->relay.ny + sp->ty - 1) / sp->ty);
    int64_t sv = 1;
    if (sp->tiles < kTargetBlocks) {
        sv = (kTargetBlocks + sp->tiles - 1) / sp->tiles;
        sv = std::min<int64_t>(sv, std::max<int64_t>(1, n_patches / nlos::kBlock));
    }
    *split = (int)sv;
    sp->n_blocks = sp->tiles * sv;
    sp->lds = smooth_lds(sp->tx * sp->ty, T);
    return NLOS_OK;
}

// Scan ranges of the adjoint: enough workgroups to fill the GPU twice.
int adjoint_split(const nlos_params* p, int32_t n_patches)
{
    const int64_t S = (int64_t)p->relay.nx * p->relay.ny;
    const int64_t pbk = std::max<int64_t>(1, ((int64_t)n_patches + nlos::kBlock - 1) / nlos::kBlock);
    int64_t sv = (2 * kTargetBlocks + pbk - 1) / pbk;
    sv = std::max<int64_t>(1, std::min<int64_t>(sv, std::min<int64_t>(S, 65535)));
    return (int)sv;
}

int adjoint_rows(int T)
{
    const int64_t fixed = 32 * 24 + 256;
    const int64_t rows = (int64_t)(kLdsMax - fixed) / (4 * (int64_t)T);
    return (int)std::min<int64_t>(32, rows);
}

size_t adjoint_lds(int rows, int T) { return (((size_t)rows * T * 4 + 15) & ~(size_t)15) + (size_t)rows * 24; }

// Plan of the adjoint: by moments (correlation rows computed once per scan
// point, in the workspace ahead of the partials) when the support radius has
// a compiled variant and its rows fit in LDS, else the tap gather.
struct AdjPlan {
    int moments, rows, split, mlen;
    int dbuf;          // moment gather: two row buffers, one filled while the other is read
    int64_t pbk;       // patch blocks of the gather
    size_t c_bytes;    // kernel taps (256 bytes per 64 floats), then correlation rows [S][adj_moments][mlen] fp32
    size_t taps_bytes; // the taps' share of c_bytes
    size_t lds;
};

int adjoint_plan(const nlos_params* p, int32_t n_patches, int rs, AdjPlan* ap)
{
    const int T = p->n_bins;
    const int64_t S = (int64_t)p->relay.nx * p->relay.ny;
    ap->moments = 0;
    ap->dbuf = 0;
    ap->mlen = 0;
    ap->c_bytes = 0;
    ap->taps_bytes = 0;
    if (nlos::smooth_moments_radius(rs)) {
        const int L = T + 2 * rs;
        const int nm = nlos::adj_moments(rs);
        const int64_t per_row = (int64_t)nm * L * 4;
        const int64_t rows = std::min<int64_t>(5, ((int64_t)kLdsMax - 1024) / per_row);
        // correlation pass: gradient row (rounded to 16 bytes), then the taps
        const size_t lds_pre = (size_t)((T + 4 * rs + 8 + 3) & ~3) * 4 + (size_t)nm * (2 * rs + 1) * 4;
        if (rows >= 1 && lds_pre <= kLdsMax) {
            ap->moments = 1;
            ap->rows = (int)rows;
            // double-buffered staging when two buffers of at least one scan
            // point fit and the rows are whole 16-byte pieces
            ap->dbuf = 0;
            if ((L & 3) == 0) {
                int r2 = 5;
                while (r2 >= 1 && nlos::adj_mom_lds(2, r2, nm, L) > kLdsMax) --r2;
                if (r2 >= 1) {
                    ap->dbuf = 1;
                    ap->rows = r2;
                }
            }
            ap->mlen = L;
            const int64_t per_block = (int64_t)nlos::kAdjPatches * nlos::kBlock;
            ap->pbk = ((int64_t)n_patches + per_block - 1) / per_block;
            const int64_t pb = std::max<int64_t>(1, ap->pbk);
            int64_t sv = (2 * kTargetBlocks + pb - 1) / pb;
            ap->split = (int)std::max<int64_t>(1, std::min<int64_t>(sv, std::min<int64_t>(S, 65535)));
            ap->taps_bytes = ((size_t)nm * (2 * rs + 1) * 4 + 255) & ~(size_t)255;
            ap->c_bytes = ap->taps_bytes + (((size_t)S * nm * L * 4 + 255) & ~(size_t)255);
            ap->lds = nlos::adj_mom_lds(ap->dbuf ? 2 : 1, ap->rows, nm, L);
            return NLOS_OK;
        }
    }
    ap->rows = adjoint_rows(T);
    if (ap->rows < 1) return NLOS_EINVAL;
    ap->split = adjoint_split(p, n_patches);
    ap->pbk = ((int64_t)n_patches + nlos::kBlock - 1) / nlos::kBlock;
    ap->lds = adjoint_lds(ap->rows, T);
    return NLOS_OK;
}

// ---------------------------------------------------------------------------
// FFT (light-cone) route.
int lct_setup(const nlos_params* p, nlos::LctArgs* a, int64_t* n3)
{
    if (params_ok(p) != NLOS_OK || !is_confocal(p)) return NLOS_EINVAL;
    const int N = p->relay.nx, M = p->n_bins;
    if (p->relay.ny != N || p->relay.half_x != p->relay.half_y || p->standoff_m != 0.0 || p->flags != 0)
        return NLOS_EINVAL;
    if ((M & (M - 1)) != 0 || M > (1 << 16) || N > 4096) return NLOS_EINVAL;
    const int64_t n = (int64_t)(2 * N) * (2 * N) * (2 * M);
    if (n > ((int64_t)1 << 34)) return NLOS_EINVAL;
    std::memset(a, 0, sizeof(*a));
    const double dt = p->bin_ps * 1e-12;
    const double slope = p->relay.half_x / ((double)M * kC * dt);
    a->N = N;
    a->M = M;
    a->dz = kC * dt / 2.0;
    a->cone = (4.0 * slope) * (4.0 * slope);
    // jitter taps in fp64 (Section 2): sigma = FWHM / (2 sqrt(2 ln 2)) / dt bins, R = ceil(2 sigma)
    if (p->fwhm_ps == 0.0) {
        a->R = 0;
        a->taps[0] = 1.0;
    } else {
        const double sigma = p->fwhm_ps / (2.0 * std::sqrt(2.0 * std::log(2.0))) / p->bin_ps;
        const double rr = std::ceil(2.0 * sigma);
        if (!(rr <= (double)nlos::kMaxRadius)) return NLOS_EINVAL;
        a->R = (int)rr;
        double sum = 0.0;
        for (int j = -a->R; j <= a->R; ++j) {
            a->taps[j + a->R] = std::exp(-(double)(j * j) / (2.0 * sigma * sigma));
            sum += a->taps[j + a->R];
        }
        for (int i = 0; i <= 2 * a->R; ++i) a->taps[i] /= sum;
    }
    *n3 = n;
    return NLOS_OK;
}

// ---------------------------------------------------------------------------
// Serving ticks.  The table (host, then its copy at the start of the device
// workspace): TickList, then per request GeomArgs, FwdArgs, variant and the
// three block prefixes; the requests' counts, summaries
// and pair-loop constants follow in the workspace.  Its size depends only on
// the capacities, so every tick copies the same bytes.
struct TickLayout {
    size_t list, geom, fwd, variant, gfirst, zfirst, ffirst, table_bytes;
};

TickLayout tick_layout(int32_t max_requests)
{
    TickLayout t;
    size_t off = 0;
    const size_t m = (size_t)max_requests;
    t.list = off;
    off = align_up(off + sizeof(nlos::TickList), 16);
    t.geom = off;
    off = align_up(off + sizeof(nlos::GeomArgs) * m, 16);
    t.fwd = off;
    off = align_up(off + sizeof(nlos::FwdArgs) * m, 16);
    t.variant = off;
    off = align_up(off + 4 * m, 16);
    t.gfirst = off;
    off = align_up(off + 8 * (m + 1), 16);
    t.zfirst = off;
    off = align_up(off + 8 * (m + 1), 16);
    t.ffirst = off;
    off = align_up(off + 8 * (m + 1), 16);
    t.table_bytes = align_up(off, 256);
    return t;
}

bool caps_ok(const nlos_tick_caps* c)
{
    return c && c->max_requests >= 1 && c->max_requests <= 4096 && c->max_pixels >= 0 &&
           c->max_pixels <= ((int64_t)1 << 31);
}

// Workspace bytes past the table for a map of npx pixels with n_blocks
// enumeration blocks: block counts, summaries, pair-loop constants.
size_t tick_request_bytes(int64_t npx, int64_t n_blocks)
{
    return align_up((size_t)n_blocks * 4, 256) + stats_bytes((int32_t)npx) + align_up((size_t)npx * 32, 256);
}

// The same for the capacities: n_blocks <= ceil(n_enum / kGeomBlock) with n_enum
// <= npx + 16 (nx + ny) + 256 <= 17 npx + 256 summed over the requests.
size_t tick_ws_bytes(const nlos_tick_caps* c)
{
    const TickLayout t = tick_layout(c->max_requests);
    const size_t px = (size_t)c->max_pixels, m = (size_t)c->max_requests;
    const size_t blocks = (17 * px + 256 * m) / nlos::kGeomBlock + m;
    return t.table_bytes + align_up(blocks * 4, 256) + 256 * m +                     // counts
           align_up((px / nlos::kStatBlock + m) * sizeof(nlos::ChunkStat), 256) + 256 * m +   // summaries
           align_up(px * 32, 256) + 256 * m;                                          // constants
}

// Dynamic LDS of the tick's pair kernel: what any plan may use.
constexpr size_t kTickLds = kLdsMax - 256;

// Device addresses of the list and the pair kernel's arrays in a tick's workspace.
nlos::TickArrays tick_arrays(void* ws, const TickLayout& t)
{
    unsigned char* d = static_cast<unsigned char*>(ws);
    nlos::TickArrays a;
    a.list = reinterpret_cast<const nlos::TickList*>(d + t.list);
    a.fwd = reinterpret_cast<const nlos::FwdArgs*>(d + t.fwd);
    a.variant = reinterpret_cast<const int32_t*>(d + t.variant);
    a.ffirst = reinterpret_cast<const int64_t*>(d + t.ffirst);
    return a;
}

// Pair-kernel items of a planned tick, read from its host table.
int64_t tick_pair_items(const void* table, const TickLayout& t)
{
    const unsigned char* host = static_cast<const unsigned char*>(table);
    const nlos::TickList* L = reinterpret_cast<const nlos::TickList*>(host + t.list);
    return reinterpret_cast<const int64_t*>(host + t.ffirst)[L->n];
}

int g_cu_count[64] = {};

int cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return kTargetBlocks;
    if (g_cu_count[dev] <= 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = kTargetBlocks;
        g_cu_count[dev] = n;
    }
    return g_cu_count[dev];
}

// Scratch of nlos_forward_noalloc: the record summaries, for up to
// NLOS_NOALLOC_MAX_PATCHES records, in a file-scope device array (each GPU
// the library runs on holds its own copy until the process ends).  Host code
// never uses the array's name as an address: its device address on each GPU
// comes from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoAllocScratchBytes =
    (size_t)((NLOS_NOALLOC_MAX_PATCHES + nlos::kStatBlock - 1) / nlos::kStatBlock) * sizeof(nlos::ChunkStat);
static_assert(kNoAllocScratchBytes == 512 * 1024, "the stated scratch size");
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device (null on
// failure, with the HIP error recorded).
void* scratch_on_current_device()
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        g_last_hip = (int)(e != hipSuccess ? e : hipErrorInvalidDevice);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            g_last_hip = (int)(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

// A tick as a HIP graph: the table copy and the three kernels, instantiated
// once; per tick only the pair kernel's grid (the tick's item count) is set
// before the launch.
struct nlos_tick_graph {
    nlos_tick_caps caps;
    const void* table = nullptr;
    void* ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t pairs = nullptr;
    hipKernelNodeParams pp;
    nlos::TickArrays arr;                    // device addresses in the workspace
    void* args[1] = {nullptr};               // geometry kernels' arguments: &arr.list
    void* pair_args[4] = {nullptr, nullptr, nullptr, nullptr};   // the pair kernel's: &arr.*
    int64_t launched_items = -1;             // grid the executable graph holds
};

extern "C" {

int nlos_abi_version(void) { return NLOS_ABI_VERSION; }

const char* nlos_strerror(int code)
{
    switch (code) {
    case NLOS_OK: return "ok";
    case NLOS_EINVAL: return "invalid argument";
    case NLOS_ENOSPC: return "workspace too small";
    case NLOS_EHIP: return "HIP runtime error";
    case NLOS_ENODEV: return "no usable GPU";
    default: return "unknown error";
    }
}

int nlos_last_hip_error(void) { return g_last_hip; }

int nlos_patches_workspace_bytes(const nlos_grid* g, size_t* bytes)
{
    if (!grid_ok(g) || !bytes) return NLOS_EINVAL;
    const int64_t bx = (g->nx + nlos::kBlockPx - 1) / nlos::kBlockPx;
    const int64_t by = (g->ny + nlos::kBlockPx - 1) / nlos::kBlockPx;
    const int64_t n_enum = (int64_t)nlos::kBlockPx * nlos::kBlockPx * bx * by;
    const int64_t blocks = (n_enum + nlos::kGeomBlock - 1) / nlos::kGeomBlock;
    *bytes = (size_t)(2 * blocks * sizeof(int32_t) + 256);
    return NLOS_OK;
}

int nlos_patches_from_depth(const nlos_grid* g, const float* depth, const float* albedo,
                            const uint8_t* mask, uint32_t flags, float* patches, int32_t* n_active,
                            void* ws, size_t ws_bytes, void* stream)
{
    nlos::GeomArgs a;
    const int rc = geom_args(g, depth, albedo, mask, flags, patches, n_active, &a);
    if (rc != NLOS_OK) return rc;
    if (!ws || !aligned(ws, 4)) return NLOS_EINVAL;
    size_t need = 0;
    nlos_patches_workspace_bytes(g, &need);
    if (ws_bytes < need) return NLOS_ENOSPC;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    a.counts = reinterpret_cast<int32_t*>(ws);
    a.offsets = a.n_blocks <= nlos::kScanFreeBlocks ? nullptr : a.counts + a.n_blocks;
    const hipError_t e = nlos::launch_geometry(a, (hipStream_t)stream);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_patches_batched_sizes(const nlos_depth_request* reqs, int32_t n, size_t* table_bytes, size_t* ws_bytes)
{
    if (!table_bytes || !ws_bytes) return NLOS_EINVAL;
    GeomBatch b;
    const int rc = plan_geom_batch(reqs, n, &b);
    if (rc != NLOS_OK) return rc;
    *table_bytes = b.table_bytes;
    *ws_bytes = b.ws_bytes;
    return NLOS_OK;
}

int nlos_patches_batched(const nlos_depth_request* reqs, int32_t n, void* table, size_t table_bytes, void* ws,
                         size_t ws_bytes, void* stream)
{
    GeomBatch b;
    const int rc = plan_geom_batch(reqs, n, &b);
    if (rc != NLOS_OK) return rc;
    if (n == 0) return NLOS_OK;
    if (!ws || !aligned(ws, 16)) return NLOS_EINVAL;
    if (ws_bytes < b.ws_bytes || (table && table_bytes < b.table_bytes)) return NLOS_ENOSPC;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    unsigned char* wsb = static_cast<unsigned char*>(ws);
    bool need_scan = false;
    for (int i = 0; i < n; ++i) {
        b.args[i].counts = reinterpret_cast<int32_t*>(wsb + b.counts_off[i]);
        const bool scan = b.args[i].n_blocks > nlos::kScanFreeBlocks;
        b.args[i].offsets = scan ? b.args[i].counts + b.args[i].n_blocks : nullptr;
        need_scan = need_scan || scan;
    }
    unsigned char* host = static_cast<unsigned char*>(table);
    if (!host) {
        g_table.resize(b.table_bytes);
        host = g_table.data();
    }
    std::memcpy(host + b.tab_off, b.args.data(), sizeof(nlos::GeomArgs) * (size_t)n);
    put(host, b.first_off, b.first);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = upload_table(ws, host, b.table_bytes, st);
    if (e != hipSuccess) return hip_fail(e);
    nlos::GeomList gl;
    gl.tab = reinterpret_cast<const nlos::GeomArgs*>(wsb + b.tab_off);
    gl.first = reinterpret_cast<const int64_t*>(wsb + b.first_off);
    gl.n = n;
    e = nlos::launch_geometry_batch(gl, b.n_blocks, need_scan, st);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_forward_workspace_bytes(const nlos_params* p, int32_t n_patches, size_t* bytes)
{
    if (params_ok(p) != NLOS_OK || !bytes || n_patches < 0 || n_patches > NLOS_MAX_PATCHES)
        return NLOS_EINVAL;
    return forward_workspace(p, n_patches, bytes, nullptr);
}

int nlos_forward(const nlos_params* p, const float* patches, int32_t n_patches, const int32_t* n_active,
                 float* out, void* ws, size_t ws_bytes, void* stream)
{
    nlos::FwdArgs a;
    nlos::Plan plan;
    size_t need = 0;
    int rc = setup_forward(p, patches, n_patches, n_active, out, kTargetBlocks, &a, &plan, &need);
    if (rc != NLOS_OK) return rc;
    if (ws_bytes < need) return NLOS_ENOSPC;
    if (need > 0 && !ws) return NLOS_EINVAL;
    if (ws && !aligned(ws, 16)) return NLOS_EINVAL;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    a.stats = reinterpret_cast<nlos::ChunkStat*>(ws);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = nlos::launch_stats(a, a.stats, st);
    if (e != hipSuccess) return hip_fail(e);
    if (a.atomic_out) {
        e = nlos::launch_fill(out, (size_t)a.out_len, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    e = nlos::launch_forward(a, plan, is_confocal(p), st);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_tick_sizes(const nlos_tick_caps* caps, size_t* table_bytes, size_t* ws_bytes)
{
    if (!caps_ok(caps) || !table_bytes || !ws_bytes) return NLOS_EINVAL;
    *table_bytes = tick_layout(caps->max_requests).table_bytes;
    *ws_bytes = tick_ws_bytes(caps);
    return NLOS_OK;
}

int nlos_tick_plan(const nlos_tick_caps* caps, const nlos_sim_request* reqs, int32_t n, void* table,
                   size_t table_bytes, void* ws, size_t ws_bytes)
{
    if (!caps_ok(caps) || n < 0 || n > caps->max_requests || (n > 0 && !reqs) || !table || !ws ||
        !aligned(ws, 256))
        return NLOS_EINVAL;
    const TickLayout t = tick_layout(caps->max_requests);
    if (table_bytes < t.table_bytes || ws_bytes < tick_ws_bytes(caps)) return NLOS_ENOSPC;
    unsigned char* host = static_cast<unsigned char*>(table);
    unsigned char* dev = static_cast<unsigned char*>(ws);
    std::memset(host, 0, t.table_bytes);
    nlos::GeomArgs* geom = reinterpret_cast<nlos::GeomArgs*>(host + t.geom);
    nlos::FwdArgs* fwd = reinterpret_cast<nlos::FwdArgs*>(host + t.fwd);
    int32_t* variant = reinterpret_cast<int32_t*>(host + t.variant);
    int64_t* gfirst = reinterpret_cast<int64_t*>(host + t.gfirst);
    int64_t* zfirst = reinterpret_cast<int64_t*>(host + t.zfirst);
    int64_t* ffirst = reinterpret_cast<int64_t*>(host + t.ffirst);
    int64_t pixels = 0;
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
        const nlos_sim_request& r = reqs[i];
        if (params_ok(&r.params) != NLOS_OK || !grid_ok(&r.grid)) return NLOS_EINVAL;
        pixels += (int64_t)r.grid.nx * r.grid.ny;
        total += (double)n_hist(&r.params) * (double)((int64_t)r.grid.nx * r.grid.ny);
    }
    if (pixels > caps->max_pixels) return NLOS_ENOSPC;
    // per request: geometry (request order) and its forward plan; each
    // request gets a share of the GPU's workgroups in proportion to its pairs
    std::vector<nlos::FwdArgs> fa(n);
    std::vector<nlos::Plan> pl(n);
    std::vector<int32_t> var(n);
    std::vector<double> work(n);
    size_t off = t.table_bytes;
    for (int i = 0; i < n; ++i) {
        const nlos_sim_request& r = reqs[i];
        nlos::GeomArgs& ga = geom[i];
        int rc = geom_args(&r.grid, r.depth, r.albedo, r.mask, r.params.flags, r.patches, r.n_active, &ga);
        if (rc != NLOS_OK) return rc;
        // one pass per map: the scatter sums the counts before its block itself
        if (ga.n_blocks > nlos::kScanFreeBlocks) return NLOS_EINVAL;
        const int32_t npx = r.grid.nx * r.grid.ny;
        const double pairs = (double)n_hist(&r.params) * (double)npx;
        const int64_t target = std::max<int64_t>(1, (int64_t)std::ceil(kTargetBlocks * pairs / std::max(total, 1.0)));
        size_t need = 0;
        rc = setup_forward(&r.params, r.patches, npx, r.n_active, r.out, target, &fa[i], &pl[i], &need);
        if (rc != NLOS_OK) return rc;
        const nlos::Plan& plan = pl[i];
        const int v = nlos::tick_variant(plan.tx, plan.ty, fa[i].cosines != 0);
        if (!is_confocal(&r.params) || !plan.pair || plan.n_tw != 1 || v < 0 || plan.lds_bytes > kTickLds)
            return NLOS_EINVAL;
        var[i] = v;
        work[i] = pairs / (double)std::max<int64_t>(1, plan.n_blocks);
        // workspace regions of this request (device addresses)
        ga.counts = reinterpret_cast<int32_t*>(dev + off);
        ga.offsets = nullptr;
        off += align_up((size_t)ga.n_blocks * 4, 256);
        fa[i].stats = reinterpret_cast<nlos::ChunkStat*>(dev + off);
        ga.stats = fa[i].stats;
        ga.n_stats = fa[i].n_stats;
        off += stats_bytes(npx);
        ga.prep = reinterpret_cast<float4*>(dev + off);
        ga.prep_sig = fa[i].inv2_f;
        fa[i].prep = ga.prep;
        off += align_up((size_t)npx * 32, 256);
        if (off > ws_bytes) return NLOS_ENOSPC;
        gfirst[i + 1] = gfirst[i] + ga.n_blocks;
    }
    // pair items in decreasing work per workgroup, so the longest
    // workgroups start first and the tick ends with short ones
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    for (int k = 0; k < n; ++k) {
        const int i = order[k];
        fwd[k] = fa[i];
        variant[k] = var[i];
        zfirst[k + 1] = zfirst[k] + (fa[i].atomic_out ? (fa[i].out_len + nlos::kTickFillFloats - 1) /
                                                            nlos::kTickFillFloats : 0);
        ffirst[k + 1] = ffirst[k] + pl[i].n_blocks;
    }
    nlos::TickList* L = reinterpret_cast<nlos::TickList*>(host + t.list);
    L->geom = reinterpret_cast<const nlos::GeomArgs*>(dev + t.geom);
    L->fwd = reinterpret_cast<const nlos::FwdArgs*>(dev + t.fwd);
    L->variant = reinterpret_cast<const int32_t*>(dev + t.variant);
    L->gfirst = reinterpret_cast<const int64_t*>(dev + t.gfirst);
    L->zfirst = reinterpret_cast<const int64_t*>(dev + t.zfirst);
    L->ffirst = reinterpret_cast<const int64_t*>(dev + t.ffirst);
    L->n = n;
    return NLOS_OK;
}

int nlos_tick_launch(const nlos_tick_caps* caps, const void* table, void* ws, size_t ws_bytes, void* stream)
{
    if (!caps_ok(caps) || !table || !ws || !aligned(ws, 256)) return NLOS_EINVAL;
    const TickLayout t = tick_layout(caps->max_requests);
    if (ws_bytes < tick_ws_bytes(caps)) return NLOS_ENOSPC;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(ws, table, t.table_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e);
    const nlos::TickArrays arr = tick_arrays(ws, t);
    e = nlos::launch_tick_geometry(arr.list, 2 * cu_count(), st);
    if (e != hipSuccess) return hip_fail(e);
    e = nlos::launch_tick_pairs(arr, std::max<int64_t>(1, tick_pair_items(table, t)), kTickLds, st);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_tick_graph_destroy(nlos_tick_graph* g)
{
    if (!g) return NLOS_OK;
    hipError_t e = hipSuccess;
    if (g->exec) e = hipGraphExecDestroy(g->exec);
    if (g->graph) {
        const hipError_t e2 = hipGraphDestroy(g->graph);
        if (e == hipSuccess) e = e2;
    }
    delete g;
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_tick_graph_create(const nlos_tick_caps* caps, const void* table, void* ws, size_t ws_bytes,
                           nlos_tick_graph** out)
{
    if (!out) return NLOS_EINVAL;
    *out = nullptr;
    if (!caps_ok(caps) || !table || !ws || !aligned(ws, 256)) return NLOS_EINVAL;
    if (ws_bytes < tick_ws_bytes(caps)) return NLOS_ENOSPC;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    const TickLayout t = tick_layout(caps->max_requests);
    nlos_tick_graph* g = new (std::nothrow) nlos_tick_graph();
    if (!g) return NLOS_EHIP;
    g->caps = *caps;
    g->table = table;
    g->ws = ws;
    g->arr = tick_arrays(ws, t);
    g->args[0] = &g->arr.list;
    g->pair_args[0] = &g->arr.list;
    g->pair_args[1] = &g->arr.fwd;
    g->pair_args[2] = &g->arr.variant;
    g->pair_args[3] = &g->arr.ffirst;
    hipError_t e = nlos::prepare_tick_pairs(kTickLds);
    if (e == hipSuccess) e = hipGraphCreate(&g->graph, 0);
    hipGraphNode_t copy = nullptr, count = nullptr, scatter = nullptr;
    if (e == hipSuccess)
        e = hipGraphAddMemcpyNode1D(&copy, g->graph, nullptr, 0, ws, table, t.table_bytes, hipMemcpyHostToDevice);
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.gridDim = dim3((unsigned)(2 * cu_count()));
    kp.blockDim = dim3(nlos::kGeomBlock);
    kp.sharedMemBytes = 0;
    kp.kernelParams = g->args;
    kp.extra = nullptr;
    if (e == hipSuccess) {
        kp.func = const_cast<void*>(nlos::tick_count_kernel());
        e = hipGraphAddKernelNode(&count, g->graph, &copy, 1, &kp);
    }
    if (e == hipSuccess) {
        kp.func = const_cast<void*>(nlos::tick_scatter_kernel());
        e = hipGraphAddKernelNode(&scatter, g->graph, &count, 1, &kp);
    }
    std::memset(&g->pp, 0, sizeof(g->pp));
    g->pp.func = const_cast<void*>(nlos::tick_pairs_kernel());
    g->pp.gridDim = dim3(1);
    g->pp.blockDim = dim3(nlos::kBlock);
    g->pp.sharedMemBytes = (unsigned)kTickLds;
    g->pp.kernelParams = g->pair_args;
    g->pp.extra = nullptr;
    if (e == hipSuccess) e = hipGraphAddKernelNode(&g->pairs, g->graph, &scatter, 1, &g->pp);
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        nlos_tick_graph_destroy(g);
        return hip_fail(e);
    }
    g->launched_items = 1;
    *out = g;
    return NLOS_OK;
}

int nlos_tick_graph_launch(nlos_tick_graph* g, void* stream)
{
    if (!g || !g->exec) return NLOS_EINVAL;
    const TickLayout t = tick_layout(g->caps.max_requests);
    const int64_t items = std::max<int64_t>(1, tick_pair_items(g->table, t));
    if (items > 0x7fffffff) return NLOS_EINVAL;
    hipError_t e = hipSuccess;
    if (items != g->launched_items) {
        g->pp.gridDim = dim3((unsigned)items);
        e = hipGraphExecKernelNodeSetParams(g->exec, g->pairs, &g->pp);
        if (e != hipSuccess) return hip_fail(e);
        g->launched_items = items;
    }
    e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_forward_noalloc(const nlos_params* p, const float* patches, int32_t n_patches, const int32_t* n_active,
                         float* out, void* stream)
{
    nlos::FwdArgs a;
    nlos::Plan plan;
    size_t need = 0;
    int rc = setup_forward(p, patches, n_patches, n_active, out, kTargetBlocks, &a, &plan, &need);
    if (rc != NLOS_OK) return rc;
    if (n_patches > NLOS_NOALLOC_MAX_PATCHES || need > kNoAllocScratchBytes) return NLOS_ENOSPC;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    void* ws = scratch_on_current_device();
    if (!ws) return NLOS_EHIP;
    // the same launches as nlos_forward, with the summaries in the scratch
    // array (every summary the pair kernel reads is written first)
    a.stats = reinterpret_cast<nlos::ChunkStat*>(ws);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = nlos::launch_stats(a, a.stats, st);
    if (e != hipSuccess) return hip_fail(e);
    if (a.atomic_out) {
        e = nlos::launch_fill(out, (size_t)a.out_len, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    e = nlos::launch_forward(a, plan, is_confocal(p), st);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_simulate_workspace_bytes(const nlos_params* p, const nlos_grid* g, size_t* bytes)
{
    if (!bytes || !grid_ok(g) || (int64_t)g->nx * g->ny > NLOS_MAX_PATCHES) return NLOS_EINVAL;
    size_t geo = 0, fwd = 0;
    int rc = nlos_patches_workspace_bytes(g, &geo);
    if (rc != NLOS_OK) return rc;
    rc = nlos_forward_workspace_bytes(p, g->nx * g->ny, &fwd);
    if (rc != NLOS_OK) return rc;
    // the geometry's block counts, the record summaries (those of
    // nlos_forward), then the records' pair-loop constants, 32 bytes per record
    *bytes = align_up(geo, 256) + align_up(fwd, 256) + (size_t)g->nx * g->ny * 32;
    return NLOS_OK;
}

int nlos_simulate(const nlos_params* p, const nlos_grid* g, const float* depth, const float* albedo,
                  const uint8_t* mask, float* patches, int32_t* n_active, float* out, void* ws, size_t ws_bytes,
                  const nlos_probe* probe, void* stream)
{
    if (probe && probe->evaluated_pairs && !aligned(probe->evaluated_pairs, 8)) return NLOS_EINVAL;
    nlos::GeomArgs ga;
    int rc = geom_args(g, depth, albedo, mask, p ? p->flags : 0u, patches, n_active, &ga);
    if (rc != NLOS_OK) return rc;
    const int32_t n_patches = g->nx * g->ny;
    nlos::FwdArgs a;
    nlos::Plan plan;
    size_t need_fwd = 0;
    rc = setup_forward(p, patches, n_patches, n_active, out, kTargetBlocks, &a, &plan, &need_fwd);
    if (rc != NLOS_OK) return rc;
    size_t need = 0;
    rc = nlos_simulate_workspace_bytes(p, g, &need);
    if (rc != NLOS_OK) return rc;
    if (ws_bytes < need) return NLOS_ENOSPC;
    if (!ws || !aligned(ws, 256)) return NLOS_EINVAL;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    size_t geo = 0;
    nlos_patches_workspace_bytes(g, &geo);
    unsigned char* w = static_cast<unsigned char*>(ws);
    ga.counts = reinterpret_cast<int32_t*>(w);
    ga.offsets = ga.n_blocks <= nlos::kScanFreeBlocks ? nullptr : ga.counts + ga.n_blocks;
    // record summaries over the partition nlos_forward uses (kStatBlock
    // consecutive records; a.n_stats from setup_forward), cleared by the count
    // pass and merged by the scatter: the same summaries, so the same
    // fixed-point scales and the same output bits as the two calls
    a.stats = reinterpret_cast<nlos::ChunkStat*>(w + align_up(geo, 256));
    ga.stats = a.stats;
    ga.n_stats = a.n_stats;
    // the scatter also writes each record's pair-loop constants (scaled as
    // the pair loop scales: by 2 / (c dt) confocal, 1 / (c dt) otherwise)
    ga.prep = reinterpret_cast<float4*>(w + align_up(geo, 256) + align_up(need_fwd, 256));
    ga.prep_sig = is_confocal(p) ? a.inv2_f : a.inv_f;
    a.prep = ga.prep;
    a.eval_pairs = probe ? probe->evaluated_pairs : nullptr;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = nlos::launch_geometry(ga, st);
    if (e != hipSuccess) return hip_fail(e);
    if (probe && probe->forward_mark) {
        e = hipEventRecord((hipEvent_t)probe->forward_mark, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (a.atomic_out) {
        e = nlos::launch_fill(out, (size_t)a.out_len, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    e = nlos::launch_forward(a, plan, is_confocal(p), st);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_forward_batched_sizes(const nlos_request* reqs, int32_t n, size_t* table_bytes, size_t* ws_bytes)
{
    if (!table_bytes || !ws_bytes) return NLOS_EINVAL;
    FwdBatch b;
    const int rc = plan_batch(reqs, n, &b);
    if (rc != NLOS_OK) return rc;
    *table_bytes = b.table_bytes;
    *ws_bytes = b.ws_bytes;
    return NLOS_OK;
}

int nlos_forward_batched(const nlos_request* reqs, int32_t n, void* table, size_t table_bytes, void* ws,
                         size_t ws_bytes, void* stream)
{
    FwdBatch b;
    const int rc = plan_batch(reqs, n, &b);
    if (rc != NLOS_OK) return rc;
    if (n == 0) return NLOS_OK;
    if (!ws || !aligned(ws, 16)) return NLOS_EINVAL;
    if (ws_bytes < b.ws_bytes || (table && table_bytes < b.table_bytes)) return NLOS_ENOSPC;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    unsigned char* wsb = static_cast<unsigned char*>(ws);
    for (int i = 0; i < n; ++i) b.args[i].stats = reinterpret_cast<nlos::ChunkStat*>(wsb + b.stats_off[i]);
    unsigned char* host = static_cast<unsigned char*>(table);
    if (!host) {
        g_table.resize(b.table_bytes);
        host = g_table.data();
    }
    std::memcpy(host + b.tab_off, b.args.data(), sizeof(nlos::FwdArgs) * (size_t)n);
    put(host, b.stat_req_off, b.stat_req);
    put(host, b.stat_first_off, b.stat_first);
    put(host, b.fill_req_off, b.fill_req);
    for (const auto& g : b.groups) {
        put(host, g.req_off, g.req);
        put(host, g.first_off, g.first);
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = upload_table(ws, host, b.table_bytes, st);
    if (e != hipSuccess) return hip_fail(e);
    const nlos::FwdArgs* tab = reinterpret_cast<const nlos::FwdArgs*>(wsb + b.tab_off);
    nlos::BatchList bl;
    bl.tab = tab;
    bl.req = reinterpret_cast<const int32_t*>(wsb + b.stat_req_off);
    bl.first = reinterpret_cast<const int64_t*>(wsb + b.stat_first_off);
    bl.n = (int32_t)b.stat_req.size();
    e = nlos::launch_stats_batch(bl, b.stat_blocks, st);
    if (e != hipSuccess) return hip_fail(e);
    if (!b.fill_req.empty()) {
        bl.req = reinterpret_cast<const int32_t*>(wsb + b.fill_req_off);
        bl.first = nullptr;
        bl.n = (int32_t)b.fill_req.size();
        e = nlos::launch_fill_batch(bl, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    for (const auto& g : b.groups) {
        if (g.req.empty()) continue;
        bl.req = reinterpret_cast<const int32_t*>(wsb + g.req_off);
        bl.first = reinterpret_cast<const int64_t*>(wsb + g.first_off);
        bl.n = (int32_t)g.req.size();
        e = nlos::launch_forward_batch(bl, g.n_blocks, g.lds, g.tl, g.tx, g.ty, g.conf, g.cos, g.pair, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    return NLOS_OK;
}

int nlos_forward_smooth_workspace_bytes(const nlos_params* p, int32_t n_patches, size_t* bytes)
{
    nlos::SmoothArgs a;
    if (!bytes) return NLOS_EINVAL;
    int rc = smooth_setup(p, nullptr, 0, nullptr, &a);
    if (rc != NLOS_OK) return rc;
    if (n_patches < 0 || n_patches > NLOS_MAX_PATCHES) return NLOS_EINVAL;
    SmoothPlan sp;
    int split = 1;
    rc = smooth_plan(p, n_patches, a.Rs, &sp, &split);
    if (rc != NLOS_OK) return rc;
    *bytes = stats_bytes(n_patches);
    return NLOS_OK;
}

int nlos_forward_smooth(const nlos_params* p, const float* patches, int32_t n_patches, const int32_t* n_active,
                        float* out, void* ws, size_t ws_bytes, void* stream)
{
    nlos::SmoothArgs a;
    int rc = smooth_setup(p, patches, n_patches, n_active, &a);
    if (rc != NLOS_OK) return rc;
    if (!out || !aligned(out, 16)) return NLOS_EINVAL;
    SmoothPlan sp;
    int split = 1;
    rc = smooth_plan(p, n_patches, a.Rs, &sp, &split);
    if (rc != NLOS_OK) return rc;
    const size_t need = stats_bytes(n_patches);
    if (ws_bytes < need) return NLOS_ENOSPC;
    if (need > 0 && (!ws || !aligned(ws, 16))) return NLOS_EINVAL;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    a.out = out;
    a.tiles_x = (p->relay.nx + sp.tx - 1) / sp.tx;
    a.tiles_y = (p->relay.ny + sp.ty - 1) / sp.ty;
    a.n_split = split;
    a.stride = sp.stride;
    a.atomic_out = split > 1 ? 1 : 0;
    a.stats = reinterpret_cast<nlos::ChunkStat*>(ws);
    a.n_stats = (int32_t)stats_count(n_patches);
    hipStream_t st = (hipStream_t)stream;
    // record summaries through the hard forward's kernel (same records)
    nlos::FwdArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    fa.patches = a.patches;
    fa.n_active = a.n_active;
    fa.n_cap = a.n_cap;
    fa.n_stats = a.n_stats;
    hipError_t e = nlos::launch_stats(fa, a.stats, st);
    if (e != hipSuccess) return hip_fail(e);
    if (a.atomic_out) {
        e = nlos::launch_fill(out, (size_t)n_hist(p) * (size_t)p->n_bins, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    e = sp.moments ? nlos::launch_smooth_moments(a, sp.n_blocks, sp.lds, st)
                   : nlos::launch_smooth(a, sp.tx, sp.ty, sp.n_blocks, sp.lds, st);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_adjoint_workspace_bytes(const nlos_params* p, int32_t n_patches, size_t* bytes)
{
    nlos::SmoothArgs a;
    if (!bytes) return NLOS_EINVAL;
    int rc = smooth_setup(p, nullptr, 0, nullptr, &a);
    if (rc != NLOS_OK) return rc;
    if (n_patches < 0 || n_patches > NLOS_MAX_PATCHES) return NLOS_EINVAL;
    AdjPlan ap;
    rc = adjoint_plan(p, n_patches, a.Rs, &ap);
    if (rc != NLOS_OK) return rc;
    *bytes = ap.c_bytes + (size_t)ap.split * (size_t)n_patches * nlos::kAdjStride * sizeof(double);
    return NLOS_OK;
}

int nlos_adjoint(const nlos_params* p, const float* patches, int32_t n_patches, const int32_t* n_active,
                 const float* grad_out, float* grad_patches, void* ws, size_t ws_bytes, void* stream)
{
    nlos::SmoothArgs a;
    int rc = smooth_setup(p, patches, n_patches, n_active, &a);
    if (rc != NLOS_OK) return rc;
    if (!grad_out || !aligned(grad_out, 16) || !grad_patches || !aligned(grad_patches, 16)) return NLOS_EINVAL;
    AdjPlan ap;
    rc = adjoint_plan(p, n_patches, a.Rs, &ap);
    if (rc != NLOS_OK) return rc;
    size_t need = 0;
    rc = nlos_adjoint_workspace_bytes(p, n_patches, &need);
    if (rc != NLOS_OK) return rc;
    if (ws_bytes < need) return NLOS_ENOSPC;
    if (need > 0 && (!ws || !aligned(ws, 256))) return NLOS_EINVAL;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    a.grad_out = grad_out;
    a.mtaps = ap.moments ? static_cast<float*>(ws) : nullptr;
    a.moments = ap.moments ? reinterpret_cast<float*>(static_cast<char*>(ws) + ap.taps_bytes) : nullptr;
    a.mlen = ap.mlen;
    a.partial = reinterpret_cast<double*>(static_cast<char*>(ws) + ap.c_bytes);
    a.n_split = ap.split;
    a.rows = ap.rows;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = ap.moments ? nlos::launch_adjoint_moments(a, ap.pbk, ap.lds, ap.dbuf, st)
                              : nlos::launch_adjoint(a, ap.pbk, ap.lds, st);
    if (e != hipSuccess) return hip_fail(e);
    e = nlos::launch_adjoint_reduce(a, grad_patches, st);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_patches_adjoint_workspace_bytes(const nlos_grid* g, size_t* bytes)
{
    if (!grid_ok(g) || !bytes) return NLOS_EINVAL;
    if ((int64_t)g->nx * g->ny > NLOS_MAX_PATCHES) return NLOS_EINVAL;
    *bytes = (size_t)3 * (size_t)g->nx * (size_t)g->ny * sizeof(float);
    return NLOS_OK;
}

int nlos_patches_adjoint(const nlos_grid* g, const float* depth, const float* albedo, uint32_t flags,
                         const float* patches, const int32_t* n_active, const float* grad_patches,
                         float* grad_depth, float* grad_albedo, void* ws, size_t ws_bytes, void* stream)
{
    size_t need = 0;
    int rc = nlos_patches_adjoint_workspace_bytes(g, &need);
    if (rc != NLOS_OK) return rc;
    if (!depth || !patches || !grad_patches || !grad_depth || (flags & ~NLOS_F_COSINES) != 0) return NLOS_EINVAL;
    if (!aligned(patches, 16) || !aligned(grad_patches, 16) || !aligned(depth, 4) || !aligned(grad_depth, 4) ||
        (albedo && !aligned(albedo, 4)) || (grad_albedo && !aligned(grad_albedo, 4)) ||
        (n_active && !aligned(n_active, 4)))
        return NLOS_EINVAL;
    if (ws_bytes < need) return NLOS_ENOSPC;
    if (!ws || !aligned(ws, 4)) return NLOS_EINVAL;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    nlos::GradMapArgs a;
    std::memset(&a, 0, sizeof(a));
    a.depth = depth;
    a.albedo = albedo;
    a.patches = reinterpret_cast<const float4*>(patches);
    a.n_active = n_active;
    a.n_cap = (int32_t)((int64_t)g->nx * g->ny);
    a.grad_rec = grad_patches;
    a.grad_depth = grad_depth;
    a.grad_albedo = grad_albedo;
    a.scratch = static_cast<float*>(ws);
    a.ax = axis(g->half_x, g->cx, g->nx);
    a.ay = axis(g->half_y, g->cy, g->ny);
    a.hx = (float)a.ax.step;
    a.hy = (float)a.ay.step;
    a.cosines = (flags & NLOS_F_COSINES) ? 1 : 0;
    const hipError_t e = nlos::launch_grad_maps(a, (hipStream_t)stream);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_noise_scale_workspace_bytes(int64_t n, size_t* bytes)
{
    if (n < 0 || !bytes) return NLOS_EINVAL;
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(nlos::kNoiseMomentBlocks, (n + 255) / 256));
    *bytes = (size_t)(3 * nb) * sizeof(double);
    return NLOS_OK;
}

int nlos_noise_scale(const float* tau, int64_t n, double nr_db, double* stats, void* ws, size_t ws_bytes,
                     void* stream)
{
    size_t need = 0;
    if (nlos_noise_scale_workspace_bytes(n, &need) != NLOS_OK || !std::isfinite(nr_db)) return NLOS_EINVAL;
    if ((n > 0 && (!tau || !aligned(tau, 4))) || !stats || !aligned(stats, 8)) return NLOS_EINVAL;
    if (ws_bytes < need) return NLOS_ENOSPC;
    if (!ws || !aligned(ws, 8)) return NLOS_EINVAL;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    const int nb = (int)(need / (3 * sizeof(double)));
    const hipError_t e =
        nlos::launch_noise_scale(tau, n, nr_db, stats, static_cast<double*>(ws), nb, (hipStream_t)stream);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_poisson_noise(const float* tau, int64_t n, const double* sigma_n, uint64_t seed, float* out,
                       void* stream)
{
    if (n < 0 || !sigma_n || !aligned(sigma_n, 8)) return NLOS_EINVAL;
    if (n > 0 && (!tau || !out || !aligned(tau, 4) || !aligned(out, 4))) return NLOS_EINVAL;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    const hipError_t e = nlos::launch_poisson(tau, n, sigma_n, seed, out, (hipStream_t)stream);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

int nlos_lct_workspace_bytes(const nlos_params* p, size_t* bytes)
{
    nlos::LctArgs a;
    int64_t n3 = 0;
    if (!bytes) return NLOS_EINVAL;
    int rc = lct_setup(p, &a, &n3);
    if (rc != NLOS_OK) return rc;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    size_t work = 0;
    if (nlos::lct_fft_work_bytes(a.N, a.M, &work) != 0) {
        g_last_hip = -1;
        return NLOS_EHIP;
    }
    *bytes = 2 * (size_t)n3 * 16 + align_up(work, 256);
    return NLOS_OK;
}

int nlos_lct_forward(const nlos_params* p, const float* depth, const float* albedo, const uint8_t* mask, float* out,
                     void* ws, size_t ws_bytes, void* stream)
{
    nlos::LctArgs a;
    int64_t n3 = 0;
    int rc = lct_setup(p, &a, &n3);
    if (rc != NLOS_OK) return rc;
    if (!depth || !out || !aligned(depth, 4) || !aligned(out, 4) || (albedo && !aligned(albedo, 4))) return NLOS_EINVAL;
    size_t need = 0;
    rc = nlos_lct_workspace_bytes(p, &need);
    if (rc != NLOS_OK) return rc;
    if (ws_bytes < need) return NLOS_ENOSPC;
    if (!ws || !aligned(ws, 256)) return NLOS_EINVAL;
    a.depth = depth;
    a.albedo = albedo;
    a.mask = mask;
    unsigned char* w = static_cast<unsigned char*>(ws);
    double2* vol = reinterpret_cast<double2*>(w);
    double2* psf = reinterpret_cast<double2*>(w + (size_t)n3 * 16);
    void* work = w + 2 * (size_t)n3 * 16;
    int fft = 0;
    const hipError_t e = nlos::launch_lct(a, vol, psf, work, out, (hipStream_t)stream, &fft);
    if (e != hipSuccess) return hip_fail(e);
    if (fft != 0) {
        g_last_hip = -1;
        return NLOS_EHIP;
    }
    return NLOS_OK;
}

int nlos_set_tuning(const nlos_tuning_entry* entries, int32_t n)
{
    if (n < 0 || (n > 0 && !entries) || n > 4096) return NLOS_EINVAL;
    for (int32_t i = 0; i < n; ++i) {
        const nlos_tuning_entry& e = entries[i];
        if (e.t_min > e.t_max || e.h_min > e.h_max || !nlos::tile_supported(e.confocal != 0, e.tx, e.ty, e.tl))
            return NLOS_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.assign(entries, entries + n);
    return NLOS_OK;
}

int nlos_get_plan(const nlos_params* p, int32_t n_patches, nlos_plan_info* info)
{
    if (params_ok(p) != NLOS_OK || !info || n_patches < 0 || n_patches > NLOS_MAX_PATCHES) return NLOS_EINVAL;
    float taps[nlos::kMaxTaps];
    int32_t R = 0;
    int rc = jitter_taps(p->fwhm_ps, p->bin_ps, taps, &R);
    if (rc != NLOS_OK) return rc;
    nlos::Plan plan;
    rc = make_plan(p, n_patches, R, kTargetBlocks, &plan);
    if (rc != NLOS_OK) return rc;
    info->tl = plan.tl;
    info->tx = plan.tx;
    info->ty = plan.ty;
    info->pair = plan.pair;
    info->n_split = plan.n_split;
    info->n_windows = plan.n_tw;
    info->workgroups = plan.n_blocks;
    info->lds_bytes = (int64_t)plan.lds_bytes;
    return NLOS_OK;
}

int nlos_debug_bins(const nlos_params* p, const float* patches, int32_t n_patches, const int32_t* n_active,
                    int32_t* bins, double* u_fast, double* u_exact, void* stream)
{
    int rc = params_ok(p);
    if (rc != NLOS_OK) return rc;
    if (n_patches < 0 || n_patches > NLOS_MAX_PATCHES || !bins) return NLOS_EINVAL;
    if (n_patches > 0 && !patches) return NLOS_EINVAL;
    if ((patches && !aligned(patches, 16)) || !aligned(bins, 4) || (u_fast && !aligned(u_fast, 8)) ||
        (u_exact && !aligned(u_exact, 8)))
        return NLOS_EINVAL;
    const int64_t pairs = n_hist(p) * (int64_t)n_patches;
    if (pairs > ((int64_t)1 << 31)) return NLOS_EINVAL;
    nlos::DebugArgs d;
    std::memset(&d, 0, sizeof(d));
    rc = fill_args(p, patches, n_patches, n_active, nullptr, &d.f);
    if (rc != NLOS_OK) return rc;
    const int dev = device_check();
    if (dev != NLOS_OK) return dev;
    d.bins = bins;
    d.u_fast = u_fast;
    d.u_exact = u_exact;
    d.n_pairs = pairs;
    d.confocal = is_confocal(p) ? 1 : 0;
    const hipError_t e = nlos::launch_debug(d, (hipStream_t)stream);
    return e == hipSuccess ? NLOS_OK : hip_fail(e);
}

}  // extern "C"
