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
static double deriv(const float* d, int32_t n, int64_t stride, int32_t i, double h)
{
    if (n < 2) return 0.0;
    if (i == 0) return ((double)d[stride] - (double)d[0]) / h;
    if (i == n - 1) return ((double)d[(int64_t)(n - 1) * stride] - (double)d[(int64_t)(n - 2) * stride]) / h;
    return ((double)d[(int64_t)(i + 1) * stride] - (double)d[(int64_t)(i - 1) * stride]) / (2.0 * h);
}

/*
 * Depth (+ albedo) map -> patch records (Section 2 depth-to-volume mapping;
 * Algorithm 1 step 2.1).  Maps are [nx][ny] (x major).  A null albedo means
 * 0.5 everywhere, as in the paper.  A patch is present when its mask entry is
 * nonzero (or the mask is null), its albedo is > 0 and its depth is finite and
 * > 0.  Output per pixel, 8 doubles:
 *   px, py, pz, a, n_x, n_y, n_z, present
 * with a = albedo * area; area = dx dy sqrt(1 + D_x^2 + D_y^2) with cosines,
 * dx dy without; n = (D_x, D_y, -1) / sqrt(1 + D_x^2 + D_y^2) (towards the wall).
 */
int32_t oracle_patches(const oracle_grid* g, const float* depth, const float* albedo,
                       const uint8_t* mask, int32_t cosines, double* rec)
{
    const int32_t nx = g->nx, ny = g->ny;
    const double hx = (2.0 * g->half_x) / (double)nx;
    const double hy = (2.0 * g->half_y) / (double)ny;
    int32_t present_count = 0;
    for (int32_t ix = 0; ix < nx; ++ix) {
        for (int32_t iy = 0; iy < ny; ++iy) {
            const int64_t idx = (int64_t)ix * ny + iy;
            const double z = (double)depth[idx];
            const double rho = albedo ? (double)albedo[idx] : 0.5;
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
