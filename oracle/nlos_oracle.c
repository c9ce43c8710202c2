/*
 * nlos_oracle.c -- plain FP64 brute-force oracle of the transient NLOS forward
 * operator (arXiv 2506.03747).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  The product (the
 * HIP library) never links, calls or includes anything from here, and this
 * file includes nothing from the product.
 *
 * What it computes (every function below names the passage it follows):
 *   Section 2, Eq. (1): the confocal transient
 *       tau(x',y',t) = iiint rho(x,y,z) / r^4 * delta(2 r - t c) dx dy dz,
 *   with the hidden object given as a depth map and an albedo map
 *   (Section 2, depth-to-volume mapping; Algorithm 1, step 2.1), so the volume
 *   integral becomes a sum over depth-map patches; each patch lands in the
 *   time bin of its round-trip path length.  The weight is extended with the
 *   Lambertian cosines at wall and patch and with the device-to-wall
 *   ("stand-off") legs; with the cosine flag cleared and zero stand-off it is
 *   Eq. (1)'s 1/r^4 exactly.
 *   Section 2, temporal jitter (and Algorithm 1, step 2.3): each trace is
 *   convolved along t only with a Gaussian, sigma = FWHM / (2 sqrt(2 ln 2)),
 *   kernel length 2*ceil(2 sigma)+1.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * document with its reason):
 *   - c = 299 792 458 m/s; t = 0 at the gate 2 s / c (s = stand-off);
 *   - grids are cell-centred, coordinates rounded once to fp32 ("canonical
 *     inputs") and promoted to fp64 for all later arithmetic;
 *   - the device (laser + SPAD) sits on the wall normal through the relay-grid
 *     centre at distance s; each stand-off leg adds (L - s) to the path and
 *     weighs (s / L)^3; s = 0 means calibrated data with no stand-off legs;
 *   - half-open bins, k = floor(u), u = ((r_l + r_d) + o) * (1 / (c dt)),
 *     evaluated in exactly that order with IEEE round-to-nearest, no FMA;
 *   - Gaussian taps normalised to sum 1, zero padding outside [0, T);
 *   - normals from central differences of the depth map (one-sided at the
 *     border), true patch area with cosines, projected area without.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_C_LIGHT 299792458.0 /* m/s, exact SI value */
#define ORACLE_PI 3.14159265358979323846

typedef struct {
    int32_t nx, ny;
    double half_x, half_y; /* half side lengths (m) */
    double cx, cy;         /* centre on the wall plane z = 0 (m) */
} oracle_grid;

typedef struct {
    oracle_grid relay;  /* scan grid (confocal) or detector grid */
    oracle_grid laser;  /* nx = ny = 0 -> confocal */
    double standoff_m;  /* s >= 0 */
    double bin_ps;      /* dt > 0 */
    int32_t n_bins;     /* T */
    double fwhm_ps;     /* >= 0; 0 -> no jitter */
    int32_t cosines;    /* 1 -> Lambertian cosines and true patch area */
} oracle_params;

int oracle_abi_version(void) { return 1; }

#ifdef _OPENMP
#include <omp.h>
#endif
/* Threads the brute-force loop runs on. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Cell-centred coordinate of cell i of n over [c-half, c+half], computed in
 * fp64 in this order and rounded once to fp32 (canonical input). */
static double grid_coord(double half, double c, int32_t n, int32_t i)
{
    double a = c - half;
    double step = (2.0 * half) / (double)n;
    double v = a + ((double)i + 0.5) * step;
    return (double)(float)v;
}

void oracle_grid_coords(const oracle_grid* g, double* xs, double* ys)
{
    for (int32_t i = 0; i < g->nx; ++i) xs[i] = grid_coord(g->half_x, g->cx, g->nx, i);
    for (int32_t j = 0; j < g->ny; ++j) ys[j] = grid_coord(g->half_y, g->cy, g->ny, j);
}

/* 1 / (c dt) in bins per metre, computed once in this order. */
double oracle_inv_bin(double bin_ps) { return 1.0 / (ORACLE_C_LIGHT * (bin_ps * 1e-12)); }

/* Derivative of the depth map along one axis at index i (n samples, spacing
 * h): central difference inside, one-sided at the two borders, 0 if n == 1. */
static double deriv(const double* d, int32_t n, int64_t stride, int32_t i, double h)
{
    if (n < 2) return 0.0;
    if (i == 0) return (d[stride] - d[0]) / h;
    if (i == n - 1) return (d[(int64_t)(n - 1) * stride] - d[(int64_t)(n - 2) * stride]) / h;
    return (d[(int64_t)(i + 1) * stride] - d[(int64_t)(i - 1) * stride]) / (2.0 * h);
}

/*
 * Depth (+ albedo) map -> patch records (Section 2 depth-to-volume mapping;
 * Algorithm 1 step 2.1), maps in fp64.  Maps are [nx][ny] (x major).  A null
 * albedo means 0.5 everywhere, as in the paper.  A patch is present when its
 * mask entry is nonzero (or the mask is null), its albedo is > 0 and its
 * depth is finite and > 0.  Output per pixel, 8 doubles:
 *   px, py, pz, a, n_x, n_y, n_z, present
 * with a = albedo * area; area = dx dy sqrt(1 + D_x^2 + D_y^2) with cosines,
 * dx dy without; n = (D_x, D_y, -1) / sqrt(1 + D_x^2 + D_y^2) (towards the wall).
 */
int32_t oracle_patches_f64(const oracle_grid* g, const double* depth, const double* albedo,
                           const uint8_t* mask, int32_t cosines, double* rec)
{
    const int32_t nx = g->nx, ny = g->ny;
    const double hx = (2.0 * g->half_x) / (double)nx;
    const double hy = (2.0 * g->half_y) / (double)ny;
    int32_t present_count = 0;
    for (int32_t ix = 0; ix < nx; ++ix) {
        for (int32_t iy = 0; iy < ny; ++iy) {
            const int64_t idx = (int64_t)ix * ny + iy;
            const double z = depth[idx];
            const double rho = albedo ? albedo[idx] : 0.5;
            const int present = (!mask || mask[idx] != 0) && rho > 0.0 && isfinite(z) && z > 0.0;
            const double gx = deriv(depth + iy, nx, ny, ix, hx);
            const double gy = deriv(depth + (int64_t)ix * ny, ny, 1, iy, hy);
            const double len = sqrt(1.0 + gx * gx + gy * gy);
            double* o = rec + idx * 8;
            o[0] = grid_coord(g->half_x, g->cx, nx, ix);
            o[1] = grid_coord(g->half_y, g->cy, ny, iy);
            o[2] = z;
            o[3] = present ? rho * hx * hy * (cosines ? len : 1.0) : 0.0;
            o[4] = gx / len;
            o[5] = gy / len;
            o[6] = -1.0 / len;
            o[7] = present ? 1.0 : 0.0;
            present_count += present;
        }
    }
    return present_count;
}

/* The same from fp32 maps (the product's input precision): every fp32 value
 * is exactly representable in fp64, so this is oracle_patches_f64 of them. */
int32_t oracle_patches(const oracle_grid* g, const float* depth, const float* albedo,
                       const uint8_t* mask, int32_t cosines, double* rec)
{
    const int64_t n = (int64_t)g->nx * g->ny;
    double* d = (double*)malloc(sizeof(double) * (size_t)n);
    double* a = albedo ? (double*)malloc(sizeof(double) * (size_t)n) : NULL;
    if (!d || (albedo && !a)) { free(d); free(a); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        d[i] = (double)depth[i];
        if (a) a[i] = (double)albedo[i];
    }
    const int32_t r = oracle_patches_f64(g, d, a, mask, cosines, rec);
    free(d);
    free(a);
    return r;
}

/*
 * Gaussian jitter taps (Section 2, temporal jitter; Algorithm 1 input list):
 * sigma in bins = FWHM / (2 sqrt(2 ln 2)) / dt, R = ceil(2 sigma), kernel
 * length 2R+1, g_j = exp(-j^2 / (2 sigma^2)) normalised to sum 1.
 * FWHM = 0 gives the identity (R = 0).  Returns R, or -1 if 2R+1 > cap.
 */
int32_t oracle_taps(double fwhm_ps, double bin_ps, double* taps, int32_t cap)
{
    if (!(fwhm_ps > 0.0)) {
        if (cap < 1) return -1;
        taps[0] = 1.0;
        return 0;
    }
    const double sigma = fwhm_ps / (2.0 * sqrt(2.0 * log(2.0))) / bin_ps;
    const int32_t R = (int32_t)ceil(2.0 * sigma);
    if (2 * R + 1 > cap) return -1;
    double sum = 0.0;
    for (int32_t j = -R; j <= R; ++j) {
        taps[j + R] = exp(-((double)j * (double)j) / (2.0 * sigma * sigma));
        sum += taps[j + R];
    }
    for (int32_t j = 0; j < 2 * R + 1; ++j) taps[j] /= sum;
    return R;
}

/* Stand-off leg of wall point (wx, wy): path offset (L - s) and weight
 * (s / L)^3, device at (cx, cy, s).  s = 0: no leg (offset 0, weight 1). */
static void standoff_leg(double wx, double wy, double cx, double cy, double s,
                         double* offset, double* weight)
{
    if (s > 0.0) {
        const double ex = wx - cx, ey = wy - cy;
        const double L = sqrt((ex * ex + ey * ey) + s * s);
        *offset = L - s;
        *weight = (s / L) * (s / L) * (s / L);
    } else {
        *offset = 0.0;
        *weight = 1.0;
    }
}

/*
 * Forward operator, brute force over every (laser point, detector point,
 * patch) triple; confocal is the same formula with the laser point equal to
 * the detector point (Section 2, Eq. (1) and the confocal layout).
 *
 *   H[h][k] = sum_p w_hp [floor(u_hp) = k],  0 <= k < T
 *   tau[h][k] = sum_{|j|<=R, 0<=k-j<T} g_j H[h][k-j]
 *
 * Output histogram h indexes (laser l, detector d) as h = l * S + d with
 * d = dx * ny + dy ([x'][y'][t] layout); confocal has l = 0 only.
 * `subset` (nullable) lists the h to compute, in output order.
 * `hist`, `tau`: [n_out][T] (nullable).  `bins`: [n_out][P] (nullable): the
 * exact bin index floor(u) of every pair (INT32_MIN for absent patches).
 * Returns 0, or -1 on bad arguments.
 */
int32_t oracle_forward(const oracle_params* prm, const double* rec, int32_t P,
                       const int32_t* subset, int32_t n_subset,
                       double* hist, double* tau, int32_t* bins)
{
    const oracle_grid* rg = &prm->relay;
    const int confocal = prm->laser.nx <= 0 || prm->laser.ny <= 0;
    const oracle_grid* lg = confocal ? rg : &prm->laser;
    const int64_t S = (int64_t)rg->nx * rg->ny;
    const int64_t L = confocal ? 1 : (int64_t)lg->nx * lg->ny;
    const int64_t n_out = subset ? n_subset : L * S;
    const int32_t T = prm->n_bins;
    if (T < 1 || !(prm->bin_ps > 0.0) || prm->standoff_m < 0.0 || P < 0) return -1;

    double taps[1024];
    const int32_t R = oracle_taps(prm->fwhm_ps, prm->bin_ps, taps, 1024);
    if (R < 0) return -1;
    const double inv = oracle_inv_bin(prm->bin_ps);
    const double s = prm->standoff_m;

    double* rx = (double*)malloc(sizeof(double) * (size_t)(rg->nx + rg->ny));
    double* lx = (double*)malloc(sizeof(double) * (size_t)(lg->nx + lg->ny));
    if (!rx || !lx) { free(rx); free(lx); return -1; }
    oracle_grid_coords(rg, rx, rx + rg->nx);
    oracle_grid_coords(lg, lx, lx + lg->nx);

    int32_t err = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t oi = 0; oi < n_out; ++oi) {
        const int64_t h = subset ? subset[oi] : oi;
        if (h < 0 || h >= L * S) { err = -1; continue; }
        const int64_t l = h / S, d = h % S;
        /* detector point d = (dx, dy); laser point l (or d itself, confocal) */
        const double wdx = rx[d / rg->ny], wdy = rx[rg->nx + d % rg->ny];
        double wlx, wly;
        if (confocal) { wlx = wdx; wly = wdy; }
        else { wlx = lx[l / lg->ny]; wly = lx[lg->nx + l % lg->ny]; }
        double o_l, g_l, o_d, g_d;
        standoff_leg(wlx, wly, rg->cx, rg->cy, s, &o_l, &g_l);
        standoff_leg(wdx, wdy, rg->cx, rg->cy, s, &o_d, &g_d);
        const double o = o_l + o_d;

        double* H = (double*)calloc((size_t)T, sizeof(double));
        if (!H) { err = -1; continue; }
        for (int32_t p = 0; p < P; ++p) {
            const double* q = rec + (int64_t)p * 8;
            if (q[7] == 0.0) {
                if (bins) bins[oi * P + p] = INT32_MIN;
                continue;
            }
            const double px = q[0], py = q[1], pz = q[2];
            /* laser leg: wall point -> patch */
            const double alx = px - wlx, aly = py - wly, alz = pz;
            const double r_l = sqrt((alx * alx + aly * aly) + alz * alz);
            /* detector leg: patch -> wall point */
            const double adx = px - wdx, ady = py - wdy, adz = pz;
            const double r_d = sqrt((adx * adx + ady * ady) + adz * adz);
            /* arrival time in bins after the gate */
            const double u = ((r_l + r_d) + o) * inv;
            const double kf = floor(u);
            const int32_t k = kf < -2147483648.0 ? INT32_MIN : (kf > 2147483647.0 ? INT32_MAX : (int32_t)kf);
            if (bins) bins[oi * P + p] = k;
            if (k < 0 || k >= T) continue;
            double w;
            if (prm->cosines) {
                /* wall normal +z; patch normal n; cosines clamp at 0 */
                const double cw_l = alz / r_l;
                const double cw_d = adz / r_d;
                double cp_l = -(q[4] * alx + q[5] * aly + q[6] * alz) / r_l;
                double cp_d = -(q[4] * adx + q[5] * ady + q[6] * adz) / r_d;
                if (cp_l < 0.0) cp_l = 0.0;
                if (cp_d < 0.0) cp_d = 0.0;
                w = q[3] * cw_l * cp_l * cp_d * cw_d / (r_l * r_l * r_d * r_d);
            } else {
                w = q[3] / (r_l * r_l * r_d * r_d);
            }
            H[k] += w * g_l * g_d;
        }
        if (hist) memcpy(hist + oi * T, H, sizeof(double) * (size_t)T);
        if (tau) {
            double* out = tau + oi * T;
            for (int32_t k = 0; k < T; ++k) {
                double acc = 0.0;
                for (int32_t j = -R; j <= R; ++j) {
                    const int32_t src = k - j;
                    if (src >= 0 && src < T) acc += taps[j + R] * H[src];
                }
                out[k] = acc;
            }
        }
        free(H);
    }
    free(rx);
    free(lx);
    return err;
}

/* ------------------------------------------------------------------------
 * Smooth time response and its gradient (the differentiable forward; a
 * reading, since the paper bins hard).  Each pair adds w * N(k + 1/2 - u) to
 * bin k, where N is the normalised continuous Gaussian in bin units with the
 * jitter's sigma (sigma = FWHM / (2 sqrt(2 ln 2)) / dt, Section 2 temporal
 * jitter), over the bins within Rs = ceil(6 sigma) of floor(u) that lie in
 * [0, T).  Loss L = 1/2 sum_{h,k} (tau_s[h][k] - y[h][k])^2.
 * ------------------------------------------------------------------------ */

static double smooth_sigma(double fwhm_ps, double bin_ps)
{
    return fwhm_ps / (2.0 * sqrt(2.0 * log(2.0))) / bin_ps;
}

/* Support radius Rs = ceil(6 sigma) in bins, or -1 if FWHM <= 0. */
int32_t oracle_smooth_radius(double fwhm_ps, double bin_ps)
{
    if (!(fwhm_ps > 0.0) || !(bin_ps > 0.0)) return -1;
    const double r = ceil(6.0 * smooth_sigma(fwhm_ps, bin_ps));
    return r > 1.0e6 ? -1 : (int32_t)r;
}

static double gauss(double x, double sigma)
{
    return exp(-(x * x) / (2.0 * sigma * sigma)) / (sigma * sqrt(2.0 * ORACLE_PI));
}

/* One (laser point, detector point, patch) pair: arrival u (bins), weight w,
 * and the derivatives of w and u with respect to the patch depth pz and of w
 * with respect to the patch normal (dw_dn[3]) and the patch factor a (w_a).
 * gg = g_l g_d (stand-off leg weights), o = leg offsets (m).
 * With cosines w = a gg pz^2 c_l c_d / (r_l^4 r_d^4), c = max(0, -n . (p - w)),
 * which is a gg cw_l cp_l cp_d cw_d / (r_l^2 r_d^2) with cw = pz / r and
 * cp = c / r; without, w = a gg / (r_l^2 r_d^2). */
static void pair_eval(const double* q, double wlx, double wly, double wdx, double wdy, double o,
                      double gg, double inv, int cosines, double* u, double* w, double* w_a,
                      double* dw_dpz, double* dw_dn, double* du_dpz)
{
    const double px = q[0], py = q[1], pz = q[2];
    const double alx = px - wlx, aly = py - wly, alz = pz;
    const double adx = px - wdx, ady = py - wdy, adz = pz;
    const double r_l = sqrt((alx * alx + aly * aly) + alz * alz);
    const double r_d = sqrt((adx * adx + ady * ady) + adz * adz);
    *u = ((r_l + r_d) + o) * inv;
    *du_dpz = inv * (pz / r_l + pz / r_d);
    const double rl2 = r_l * r_l, rd2 = r_d * r_d;
    if (cosines) {
        double c_l = -(q[4] * alx + q[5] * aly + q[6] * alz);
        double c_d = -(q[4] * adx + q[5] * ady + q[6] * adz);
        if (c_l <= 0.0 || c_d <= 0.0) {
            *w = *w_a = *dw_dpz = 0.0;
            dw_dn[0] = dw_dn[1] = dw_dn[2] = 0.0;
            return;
        }
        const double den = (rl2 * rl2) * (rd2 * rd2);
        const double F = pz * pz * c_l * c_d / den;
        /* dc/dpz = -n_z; d(r^4)/dpz = 4 r^2 pz */
        const double dF_dpz = (2.0 * pz * c_l * c_d - pz * pz * q[6] * c_d - pz * pz * c_l * q[6]) / den
                              - F * (4.0 * pz / rl2 + 4.0 * pz / rd2);
        /* dc_l/dn = -(p - w_l), dc_d/dn = -(p - w_d) */
        const double k = pz * pz / den;
        dw_dn[0] = q[3] * gg * k * (-alx * c_d - adx * c_l);
        dw_dn[1] = q[3] * gg * k * (-aly * c_d - ady * c_l);
        dw_dn[2] = q[3] * gg * k * (-alz * c_d - adz * c_l);
        *w_a = gg * F;
        *w = q[3] * gg * F;
        *dw_dpz = q[3] * gg * dF_dpz;
    } else {
        const double F = 1.0 / (rl2 * rd2);
        *w_a = gg * F;
        *w = q[3] * gg * F;
        *dw_dpz = -(*w) * (2.0 * pz / rl2 + 2.0 * pz / rd2);
        dw_dn[0] = dw_dn[1] = dw_dn[2] = 0.0;
    }
}

/* Bin range [k_lo, k_hi] of a pair's smooth response clipped to [0, T). */
static int smooth_range(double u, int32_t Rs, int32_t T, int32_t* k_lo, int32_t* k_hi)
{
    const double k0 = floor(u);
    const double lo = k0 - (double)Rs, hi = k0 + (double)Rs;
    if (hi < 0.0 || lo > (double)(T - 1)) return 0;
    *k_lo = lo < 0.0 ? 0 : (int32_t)lo;
    *k_hi = hi > (double)(T - 1) ? T - 1 : (int32_t)hi;
    return 1;
}

/* Wall points and leg terms of histogram h (as in oracle_forward). */
static void hist_setup(const oracle_params* prm, const double* rx, const double* lx, int64_t h, double* wlx,
                       double* wly, double* wdx, double* wdy, double* o, double* gg)
{
    const oracle_grid* rg = &prm->relay;
    const int confocal = prm->laser.nx <= 0 || prm->laser.ny <= 0;
    const oracle_grid* lg = confocal ? rg : &prm->laser;
    const int64_t S = (int64_t)rg->nx * rg->ny;
    const int64_t l = h / S, d = h % S;
    *wdx = rx[d / rg->ny];
    *wdy = rx[rg->nx + d % rg->ny];
    if (confocal) { *wlx = *wdx; *wly = *wdy; }
    else { *wlx = lx[l / lg->ny]; *wly = lx[lg->nx + l % lg->ny]; }
    double o_l, g_l, o_d, g_d;
    standoff_leg(*wlx, *wly, rg->cx, rg->cy, prm->standoff_m, &o_l, &g_l);
    standoff_leg(*wdx, *wdy, rg->cx, rg->cy, prm->standoff_m, &o_d, &g_d);
    *o = o_l + o_d;
    *gg = g_l * g_d;
}

/*
 * Smooth forward: tau_s[h][k] = sum_p w_hp N(k + 1/2 - u_hp) over the support
 * above.  Layout and `subset` as in oracle_forward.  Returns 0 or -1.
 */
int32_t oracle_forward_smooth(const oracle_params* prm, const double* rec, int32_t P,
                              const int32_t* subset, int32_t n_subset, double* tau)
{
    const oracle_grid* rg = &prm->relay;
    const int confocal = prm->laser.nx <= 0 || prm->laser.ny <= 0;
    const oracle_grid* lg = confocal ? rg : &prm->laser;
    const int64_t S = (int64_t)rg->nx * rg->ny;
    const int64_t L = confocal ? 1 : (int64_t)lg->nx * lg->ny;
    const int64_t n_out = subset ? n_subset : L * S;
    const int32_t T = prm->n_bins;
    const int32_t Rs = oracle_smooth_radius(prm->fwhm_ps, prm->bin_ps);
    if (T < 1 || !(prm->bin_ps > 0.0) || prm->standoff_m < 0.0 || P < 0 || Rs < 0 || !tau) return -1;
    const double sigma = smooth_sigma(prm->fwhm_ps, prm->bin_ps);
    const double inv = oracle_inv_bin(prm->bin_ps);
    double* rx = (double*)malloc(sizeof(double) * (size_t)(rg->nx + rg->ny));
    double* lx = (double*)malloc(sizeof(double) * (size_t)(lg->nx + lg->ny));
    if (!rx || !lx) { free(rx); free(lx); return -1; }
    oracle_grid_coords(rg, rx, rx + rg->nx);
    oracle_grid_coords(lg, lx, lx + lg->nx);
    int32_t err = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t oi = 0; oi < n_out; ++oi) {
        const int64_t h = subset ? subset[oi] : oi;
        if (h < 0 || h >= L * S) { err = -1; continue; }
        double wlx, wly, wdx, wdy, o, gg;
        hist_setup(prm, rx, lx, h, &wlx, &wly, &wdx, &wdy, &o, &gg);
        double* out = tau + oi * T;
        for (int32_t k = 0; k < T; ++k) out[k] = 0.0;
        for (int32_t p = 0; p < P; ++p) {
            const double* q = rec + (int64_t)p * 8;
            if (q[7] == 0.0) continue;
            double u, w, w_a, dw_dpz, dw_dn[3], du_dpz;
            pair_eval(q, wlx, wly, wdx, wdy, o, gg, inv, prm->cosines, &u, &w, &w_a, &dw_dpz, dw_dn, &du_dpz);
            int32_t k_lo, k_hi;
            if (w == 0.0 || !smooth_range(u, Rs, T, &k_lo, &k_hi)) continue;
            for (int32_t k = k_lo; k <= k_hi; ++k) out[k] += w * gauss(((double)k + 0.5) - u, sigma);
        }
    }
    free(rx);
    free(lx);
    return err;
}

/*
 * Error model of an fp32 evaluation of the direct operator (Section 2,
 * Eq. (1), with the cosines and stand-off legs of oracle_forward): the
 * per-histogram tolerance of the parity tests, not part of the operator.
 * The histogram bins are exact (the fast path re-bins in fp64), so the
 * error of an fp32 evaluation is the error of each in-window pair's weight.
 * That weight is w = K c_l c_d (K = a gg cw_l cw_d / (r_l^2 r_d^2),
 * c = max(0, n . (w - p)) / r the patch cosine of each leg); its factors
 * come within a few ulp except the patch cosines, whose numerator
 * n . (w - p) cancels for grazing patches: fp32 record normals, fp32
 * coordinates (each rounded before the difference is taken) and fp32
 * arithmetic give it an error of up to e1 times the magnitudes it is built
 * from, so each cosine is uncertain by
 *     dc = e1 (|n_x| (|p_x| + |w_x|) + |n_y| (|p_y| + |w_y|) + |n_z p_z|) / r.
 * Per bin k of histogram h this accumulates, over the in-window pairs,
 *     err[h][k] = sum_p e0 w_p + K_p (dc_l c_d + c_l dc_d + dc_l dc_d)
 * (the last terms bound |K ((c_l + dc_l)(c_d + dc_d) - c_l c_d)|, clamped
 * pairs included: c = 0 may still become dc), and
 *     count[h][k] = number of in-window pairs,
 * from which a test bounds rounding that is absolute per pair; gain[h] is
 * the histogram's stand-off weight g_l g_d.  Without cosines only the e0
 * term remains.  Layout and `subset` as in oracle_forward; err and count
 * are [n_out][T], gain [n_out] (each may be NULL).  Returns 0 or -1.
 */
int32_t oracle_forward_error_model(const oracle_params* prm, const double* rec, int32_t P,
                                   const int32_t* subset, int32_t n_subset, double e0, double e1,
                                   double* err, double* count, double* gain)
{
    const oracle_grid* rg = &prm->relay;
    const int confocal = prm->laser.nx <= 0 || prm->laser.ny <= 0;
    const oracle_grid* lg = confocal ? rg : &prm->laser;
    const int64_t S = (int64_t)rg->nx * rg->ny;
    const int64_t L = confocal ? 1 : (int64_t)lg->nx * lg->ny;
    const int64_t n_out = subset ? n_subset : L * S;
    const int32_t T = prm->n_bins;
    if (T < 1 || !(prm->bin_ps > 0.0) || prm->standoff_m < 0.0 || P < 0 || !(e0 >= 0.0) || !(e1 >= 0.0))
        return -1;
    const double inv = oracle_inv_bin(prm->bin_ps);
    double* rx = (double*)malloc(sizeof(double) * (size_t)(rg->nx + rg->ny));
    double* lx = (double*)malloc(sizeof(double) * (size_t)(lg->nx + lg->ny));
    if (!rx || !lx) { free(rx); free(lx); return -1; }
    oracle_grid_coords(rg, rx, rx + rg->nx);
    oracle_grid_coords(lg, lx, lx + lg->nx);
    int32_t rc = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t oi = 0; oi < n_out; ++oi) {
        const int64_t h = subset ? subset[oi] : oi;
        if (h < 0 || h >= L * S) { rc = -1; continue; }
        double wlx, wly, wdx, wdy, o, gg;
        hist_setup(prm, rx, lx, h, &wlx, &wly, &wdx, &wdy, &o, &gg);
        if (gain) gain[oi] = gg;
        double* E = err ? err + oi * T : NULL;
        double* N = count ? count + oi * T : NULL;
        for (int32_t k = 0; k < T; ++k) {
            if (E) E[k] = 0.0;
            if (N) N[k] = 0.0;
        }
        for (int32_t p = 0; p < P; ++p) {
            const double* q = rec + (int64_t)p * 8;
            if (q[7] == 0.0) continue;
            const double px = q[0], py = q[1], pz = q[2];
            const double alx = px - wlx, aly = py - wly, alz = pz;
            const double adx = px - wdx, ady = py - wdy, adz = pz;
            const double r_l = sqrt((alx * alx + aly * aly) + alz * alz);
            const double r_d = sqrt((adx * adx + ady * ady) + adz * adz);
            const double u = ((r_l + r_d) + o) * inv;
            const double kf = floor(u);
            if (!(kf >= 0.0 && kf < (double)T)) continue;
            const int32_t k = (int32_t)kf;
            double e;
            if (prm->cosines) {
                const double K = q[3] * gg * (alz / r_l) * (adz / r_d) / (r_l * r_l * r_d * r_d);
                double c_l = -(q[4] * alx + q[5] * aly + q[6] * alz) / r_l;
                double c_d = -(q[4] * adx + q[5] * ady + q[6] * adz) / r_d;
                if (c_l < 0.0) c_l = 0.0;
                if (c_d < 0.0) c_d = 0.0;
                const double dc_l =
                    e1 * (fabs(q[4]) * (fabs(px) + fabs(wlx)) + fabs(q[5]) * (fabs(py) + fabs(wly)) + fabs(q[6] * pz)) / r_l;
                const double dc_d =
                    e1 * (fabs(q[4]) * (fabs(px) + fabs(wdx)) + fabs(q[5]) * (fabs(py) + fabs(wdy)) + fabs(q[6] * pz)) / r_d;
                e = e0 * (K * c_l * c_d) + K * (dc_l * c_d + c_l * dc_d + dc_l * dc_d);
            } else {
                e = e0 * (q[3] * gg / (r_l * r_l * r_d * r_d));
            }
            if (E) E[k] += e;
            if (N) N[k] += 1.0;
        }
    }
    free(rx);
    free(lx);
    return rc;
}

/* dL/d(pz, a, n_x, n_y, n_z) of one present record q, summed over every
 * histogram, for upstream gradient G = dL/dtau_s [H][T]: per pair
 * dL/dw = G0 = sum_k G N(x_k) and dL/du = w G1, G1 = sum_k G (x_k / sigma^2)
 * N(x_k), x_k = k + 1/2 - u.  Written to o8[2..6]. */
static void record_grad(const oracle_params* prm, const double* rx, const double* lx, int64_t H,
                        const double* q, const double* G, int32_t Rs, double sigma, double inv, double* o8)
{
    const int32_t T = prm->n_bins;
    double gpz = 0.0, ga = 0.0, gn[3] = {0.0, 0.0, 0.0};
    for (int64_t h = 0; h < H; ++h) {
        double wlx, wly, wdx, wdy, o, gg;
        hist_setup(prm, rx, lx, h, &wlx, &wly, &wdx, &wdy, &o, &gg);
        double u, w, w_a, dw_dpz, dw_dn[3], du_dpz;
        pair_eval(q, wlx, wly, wdx, wdy, o, gg, inv, prm->cosines, &u, &w, &w_a, &dw_dpz, dw_dn, &du_dpz);
        int32_t k_lo, k_hi;
        if (!smooth_range(u, Rs, T, &k_lo, &k_hi)) continue;
        const double* r = G + h * T;
        double G0 = 0.0, G1 = 0.0;
        for (int32_t k = k_lo; k <= k_hi; ++k) {
            const double x = ((double)k + 0.5) - u;
            const double nv = gauss(x, sigma);
            G0 += r[k] * nv;
            G1 += r[k] * (x / (sigma * sigma)) * nv;
        }
        /* dL/dw = G0, dL/du = w G1 */
        gpz += G0 * dw_dpz + w * G1 * du_dpz;
        ga += G0 * w_a;
        gn[0] += G0 * dw_dn[0];
        gn[1] += G0 * dw_dn[1];
        gn[2] += G0 * dw_dn[2];
    }
    o8[2] = gpz;
    o8[3] = ga;
    o8[4] = gn[0];
    o8[5] = gn[1];
    o8[6] = gn[2];
}

/*
 * Record gradients for an arbitrary upstream gradient G [L*S][T] (the adjoint
 * of the smooth forward with respect to the records), for the records listed
 * in `subset` (nullable: all P).  grad_rec [n][8]: entries 2..6 as above,
 * zeros elsewhere and for absent records.  Returns 0 or -1.
 */
int32_t oracle_adjoint_records(const oracle_params* prm, const double* rec, int32_t P, const double* G,
                               const int32_t* subset, int32_t n_subset, double* grad_rec)
{
    const oracle_grid* rg = &prm->relay;
    const int confocal = prm->laser.nx <= 0 || prm->laser.ny <= 0;
    const oracle_grid* lg = confocal ? rg : &prm->laser;
    const int64_t H = (int64_t)rg->nx * rg->ny * (confocal ? 1 : (int64_t)lg->nx * lg->ny);
    const int32_t Rs = oracle_smooth_radius(prm->fwhm_ps, prm->bin_ps);
    if (Rs < 0 || prm->n_bins < 1 || !G || !grad_rec || P < 0) return -1;
    const int64_t n = subset ? n_subset : P;
    double* rx = (double*)malloc(sizeof(double) * (size_t)(rg->nx + rg->ny));
    double* lx = (double*)malloc(sizeof(double) * (size_t)(lg->nx + lg->ny));
    if (!rx || !lx) { free(rx); free(lx); return -1; }
    oracle_grid_coords(rg, rx, rx + rg->nx);
    oracle_grid_coords(lg, lx, lx + lg->nx);
    const double sigma = smooth_sigma(prm->fwhm_ps, prm->bin_ps);
    const double inv = oracle_inv_bin(prm->bin_ps);
    int32_t err = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t p = subset ? subset[i] : i;
        double* o8 = grad_rec + i * 8;
        for (int k = 0; k < 8; ++k) o8[k] = 0.0;
        if (p < 0 || p >= P) { err = -1; continue; }
        if (rec[p * 8 + 7] == 0.0) continue;
        record_grad(prm, rx, lx, H, rec + p * 8, G, Rs, sigma, inv, o8);
    }
    free(rx);
    free(lx);
    return err;
}

/*
 * Gradient of L with respect to the depth and albedo maps (fp64 maps, as
 * oracle_patches_f64), by the chain rule through each pair's weight and
 * arrival, the patch records, and the central-difference normals and areas.
 *   y            target [L*S][T].
 *   loss         L (host double).
 *   grad_depth   [nx][ny] (nullable);  grad_albedo [nx][ny] (nullable): with a
 *                null albedo map, the gradient with respect to that constant
 *                0.5 map.
 *   grad_rec     [nx*ny][8] (nullable): dL/d(pz, a, n_x, n_y, n_z) of each
 *                present pixel's record at entries 2..6, zeros elsewhere.
 * The support of each pair's response moves with floor(u); that step is not
 * differentiated (its contribution is below the Gaussian tail at 6 sigma).
 */
int32_t oracle_smooth_grad(const oracle_params* prm, const oracle_grid* g, const double* depth,
                           const double* albedo, const uint8_t* mask, const double* y, double* loss,
                           double* grad_depth, double* grad_albedo, double* grad_rec)
{
    const oracle_grid* rg = &prm->relay;
    const int confocal = prm->laser.nx <= 0 || prm->laser.ny <= 0;
    const oracle_grid* lg = confocal ? rg : &prm->laser;
    const int64_t H = (int64_t)rg->nx * rg->ny * (confocal ? 1 : (int64_t)lg->nx * lg->ny);
    const int32_t T = prm->n_bins;
    const int32_t Rs = oracle_smooth_radius(prm->fwhm_ps, prm->bin_ps);
    if (Rs < 0 || T < 1 || !y || !loss) return -1;
    const int32_t nx = g->nx, ny = g->ny;
    const int64_t npx = (int64_t)nx * ny;
    const double hx = (2.0 * g->half_x) / (double)nx;
    const double hy = (2.0 * g->half_y) / (double)ny;
    const double sigma = smooth_sigma(prm->fwhm_ps, prm->bin_ps);
    const double inv = oracle_inv_bin(prm->bin_ps);

    double* rec = (double*)malloc(sizeof(double) * 8 * (size_t)npx);
    double* tau = (double*)malloc(sizeof(double) * (size_t)(H * T));
    double* gr = (double*)calloc((size_t)npx * 8, sizeof(double));
    double* rx = (double*)malloc(sizeof(double) * (size_t)(rg->nx + rg->ny));
    double* lx = (double*)malloc(sizeof(double) * (size_t)(lg->nx + lg->ny));
    if (!rec || !tau || !gr || !rx || !lx) { free(rec); free(tau); free(gr); free(rx); free(lx); return -1; }
    oracle_patches_f64(g, depth, albedo, mask, prm->cosines, rec);
    int32_t rc = oracle_forward_smooth(prm, rec, (int32_t)npx, NULL, 0, tau);
    if (rc != 0) { free(rec); free(tau); free(gr); free(rx); free(lx); return rc; }
    /* residual and loss */
    double L2 = 0.0;
    for (int64_t i = 0; i < H * T; ++i) {
        tau[i] -= y[i];
        L2 += tau[i] * tau[i];
    }
    *loss = 0.5 * L2;
    oracle_grid_coords(rg, rx, rx + rg->nx);
    oracle_grid_coords(lg, lx, lx + lg->nx);

    /* record gradients: for each present patch, sum over every histogram */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < npx; ++p) {
        if (rec[p * 8 + 7] == 0.0) continue;
        record_grad(prm, rx, lx, H, rec + p * 8, tau, Rs, sigma, inv, gr + p * 8);
    }

    /* records -> maps: pz = D; a = rho * area(gx, gy); n = (gx, gy, -1) / len */
    if (grad_depth) for (int64_t i = 0; i < npx; ++i) grad_depth[i] = 0.0;
    if (grad_albedo) for (int64_t i = 0; i < npx; ++i) grad_albedo[i] = 0.0;
    for (int32_t ix = 0; ix < nx; ++ix) {
        for (int32_t iy = 0; iy < ny; ++iy) {
            const int64_t idx = (int64_t)ix * ny + iy;
            if (rec[idx * 8 + 7] == 0.0) continue;
            const double* o8 = gr + idx * 8;
            const double rho = albedo ? albedo[idx] : 0.5;
            const double gx = deriv(depth + iy, nx, ny, ix, hx);
            const double gy = deriv(depth + (int64_t)ix * ny, ny, 1, iy, hy);
            const double len = sqrt(1.0 + gx * gx + gy * gy);
            if (grad_albedo) grad_albedo[idx] = o8[3] * hx * hy * (prm->cosines ? len : 1.0);
            if (!grad_depth) continue;
            grad_depth[idx] += o8[2];
            if (!prm->cosines) continue;
            /* dn/dgx = e_x / len - (gx, gy, -1) gx / len^3 (and likewise gy);
             * d(area)/dgx = dx dy gx / len */
            const double l3 = len * len * len;
            const double dot = o8[4] * gx + o8[5] * gy - o8[6];
            const double dL_dgx = o8[4] / len - dot * gx / l3 + o8[3] * rho * hx * hy * gx / len;
            const double dL_dgy = o8[5] / len - dot * gy / l3 + o8[3] * rho * hx * hy * gy / len;
            /* derivative stencils of deriv() */
            if (nx >= 2) {
                if (ix == 0) { grad_depth[idx + ny] += dL_dgx / hx; grad_depth[idx] -= dL_dgx / hx; }
                else if (ix == nx - 1) { grad_depth[idx] += dL_dgx / hx; grad_depth[idx - ny] -= dL_dgx / hx; }
                else { grad_depth[idx + ny] += dL_dgx / (2.0 * hx); grad_depth[idx - ny] -= dL_dgx / (2.0 * hx); }
            }
            if (ny >= 2) {
                if (iy == 0) { grad_depth[idx + 1] += dL_dgy / hy; grad_depth[idx] -= dL_dgy / hy; }
                else if (iy == ny - 1) { grad_depth[idx] += dL_dgy / hy; grad_depth[idx - 1] -= dL_dgy / hy; }
                else { grad_depth[idx + 1] += dL_dgy / (2.0 * hy); grad_depth[idx - 1] -= dL_dgy / (2.0 * hy); }
            }
        }
    }
    if (grad_rec) memcpy(grad_rec, gr, sizeof(double) * 8 * (size_t)npx);
    free(rec); free(tau); free(gr); free(rx); free(lx);
    return 0;
}

/* ------------------------------------------------------------------------
 * Poisson noise (Algorithm 1 step 2.4, after the blur of step 2.3):
 *   T = Poisson(tau * sigma_n) / sigma_n,  sigma_n = Var(tau) / 10^(nr / 10),
 * Var the population variance over the whole frame.  Random numbers come
 * from the counter-based Philox4x64-10 generator (Salmon, Moraes, Dror and
 * Shaw, SC 2011), so any element can be drawn independently: uniform t of
 * element i is word t mod 4 of Philox(counter (i, t / 4, 0, 0), key
 * (seed, 0x4e4c4f53)), mapped to [0, 1) by its top 53 bits.  Counts come from
 * inversion by sequential search for lambda < 10 and from Hormann's
 * transformed rejection with squeeze (PTRS, 1993) above.  exp, log and
 * log k! are evaluated by the fixed recipes below from IEEE basic operations
 * only, so that an implementation doing the same operations in the same
 * order reaches the same integer decisions.
 * ------------------------------------------------------------------------ */

static void philox_mulhilo(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    const unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* Philox4x64 with 10 rounds: each round multiplies words 0 and 2 by the two
 * round constants and mixes high halves, the other words and the key; the
 * key is advanced by the two Weyl constants between rounds. */
void oracle_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        uint64_t hi0, lo0, hi1, lo1;
        philox_mulhilo(0xD2E7470EE14C6C93ull, c0, &hi0, &lo0);
        philox_mulhilo(0xCA5A826395121157ull, c2, &hi1, &lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static double noise_uniform(uint64_t seed, int64_t i, int t)
{
    const uint64_t ctr[4] = {(uint64_t)i, (uint64_t)(t / 4), 0, 0};
    const uint64_t key[2] = {seed, 0x4e4c4f53ull};
    uint64_t o[4];
    oracle_philox4x64(ctr, key, o);
    return (double)(o[t % 4] >> 11) * (1.0 / 9007199254740992.0);
}

#define NX_LN2_HI 6.93147180369123816490e-01
#define NX_LN2_LO 1.90821492927058770002e-10
#define NX_LOG2E 1.44269504088896338700e+00

/* e^x: x = n ln2 + r, |r| <= ln2 / 2, e^r by its Taylor polynomial to r^13
 * (Horner-free running term), scaled by 2^n; 0 below -708. */
double oracle_nx_exp(double x)
{
    if (x < -708.0) return 0.0;
    const double n = floor(x * NX_LOG2E + 0.5);
    const double r = (x - n * NX_LN2_HI) - n * NX_LN2_LO;
    double s = 1.0, t = 1.0;
    for (int k = 1; k <= 13; ++k) {
        t = t * r / (double)k;
        s = s + t;
    }
    return ldexp(s, (int)n);
}

/* log x, x > 0: x = m 2^e with m in [1/sqrt2, sqrt2), log m = 2 atanh(s),
 * s = (m - 1) / (m + 1), by its series to s^29. */
double oracle_nx_log(double x)
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
    return 2.0 * acc + ((double)e * NX_LN2_HI + (double)e * NX_LN2_LO);
}

/* log k! for integer k >= 0: the product for k < 20, else Stirling's series
 * k log k - k + log(2 pi k) / 2 + 1/(12k) - 1/(360k^3) + 1/(1260k^5) - 1/(1680k^7). */
double oracle_nx_logfact(double k)
{
    if (k < 20.0) {
        double f = 1.0;
        for (double i = 2.0; i <= k; i = i + 1.0) f = f * i;
        return oracle_nx_log(f);
    }
    const double ik = 1.0 / k, ik2 = ik * ik;
    const double series = ik * (1.0 / 12.0 - ik2 * (1.0 / 360.0 - ik2 * (1.0 / 1260.0 - ik2 * (1.0 / 1680.0))));
    return (k * oracle_nx_log(k) - k) + 0.5 * oracle_nx_log(2.0 * ORACLE_PI * k) + series;
}

/* One Poisson count of mean lam >= 0 from element i's uniforms. */
int64_t oracle_poisson_count(double lam, uint64_t seed, int64_t i)
{
    if (!(lam > 0.0)) return 0;
    if (lam < 10.0) {
        /* inversion: smallest k with u <= F(k) */
        const double u = noise_uniform(seed, i, 0);
        double p = oracle_nx_exp(-lam), F = p;
        int64_t k = 0;
        while (u > F && k < 1000) {
            k = k + 1;
            p = p * lam / (double)k;
            F = F + p;
        }
        return k;
    }
    /* transformed rejection with squeeze */
    const double slam = sqrt(lam), loglam = oracle_nx_log(lam);
    const double b = 0.931 + 2.53 * slam;
    const double a = -0.059 + 0.02483 * b;
    const double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    const double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (int it = 0; it < 100000; ++it) {
        const double U = noise_uniform(seed, i, 2 * it) - 0.5;
        const double V = noise_uniform(seed, i, 2 * it + 1);
        const double us = 0.5 - fabs(U);
        const double kd = floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && V <= vr) return (int64_t)kd;
        if (kd < 0.0 || (us < 0.013 && V > us)) continue;
        const double lhs = (oracle_nx_log(V) + oracle_nx_log(invalpha)) - oracle_nx_log(a / (us * us) + b);
        const double rhs = (-lam + kd * loglam) - oracle_nx_logfact(kd);
        if (lhs <= rhs) return (int64_t)kd;
    }
    return -1;
}

/* Counts for an array of means (distribution checks). */
void oracle_poisson_counts(const double* lam, int64_t n, uint64_t seed, int64_t* k)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) k[i] = oracle_poisson_count(lam[i], seed, i);
}

/* mean, population variance and sigma_n = Var / 10^(nr / 10) of a frame. */
void oracle_noise_scale(const float* tau, int64_t n, double nr_db, double* out)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (double)tau[i];
    const double mean = n > 0 ? s / (double)n : 0.0;
    double v = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double d = (double)tau[i] - mean;
        v += d * d;
    }
    const double var = n > 0 ? v / (double)n : 0.0;
    out[0] = mean;
    out[1] = var;
    out[2] = var / pow(10.0, nr_db / 10.0);
}

/* T = Poisson(tau * sigma_n) / sigma_n elementwise (0 where sigma_n <= 0 or
 * not finite; negative tau counts as 0), written as fp32. */
void oracle_poisson_noise(const float* tau, int64_t n, double sigma_n, uint64_t seed, float* out)
{
    const int ok = sigma_n > 0.0 && isfinite(sigma_n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (!ok) { out[i] = 0.0f; continue; }
        const double t = (double)tau[i];
        const double lam = t > 0.0 ? t * sigma_n : 0.0;
        out[i] = (float)((double)oracle_poisson_count(lam, seed, i) / sigma_n);
    }
}
