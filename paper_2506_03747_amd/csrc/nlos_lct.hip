// The paper's FFT ("light-cone") forward route, gfx950: Section 2 rewrites
// Eq. (1) with u = z^2, v = (t c / 2)^2 as a 3-D convolution of the
// resampled volume with a cone (Eq. (3)-(5)), evaluated with 3-D FFTs
// (Algorithm 1 steps 1.1-2.3).  A cross-check of the direct operator, for a
// confocal N x N scan co-registered with the depth map, no stand-off, no
// cosine terms (Eq. (1) as printed), M = T a power of two.
//
//   k_lct_clear / k_lct_volume   R_z V on the (2N, 2N, 2M) zero-padded grid:
//       pixel (x, y) at depth layer j = floor(D / dz) (dz = c dt / 2) adds
//       albedo / (J M), J = j + 1, at coarse v-sample (J^2 - 1) / M (the
//       1 / sqrt(i) fold to i = J^2 of M^2 samples, then pairwise means).
//   k_lct_psf    cone: lateral offset n = -N .. N-1 cells at x = n / N,
//       layers z = k / M; 1 at the layer(s) nearest (4 slope)^2 (x^2 + y^2)
//       when below M, slope = w / (M c dt).
//   FFT, product, inverse FFT (hipFFT, fp64: the v^(-3/2) resampling below
//       amplifies the first bins ~1e8-fold over the last, and fp32 transform
//       noise would swamp them).
//   k_lct_out    time bin j: mean of the convolution over its fine v-span
//       [j^2, (j+1)^2), divided by (J dz)^3 (Eq. (3)).
//   k_lct_jitter Gaussian jitter (Section 2 / step 2.3), fp32 output.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <utility>

#include "nlos_internal.h"

namespace nlos {

__global__ void k_lct_clear(double2* a, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = make_double2(0.0, 0.0);
}

__global__ void k_lct_volume(const LctArgs a, double2* vol)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int N = a.N, M = a.M;
    if (p >= (int64_t)N * N) return;
    const double D = (double)a.depth[p];
    const double A = a.albedo ? (double)a.albedo[p] : 0.5;
    const bool present = (!a.mask || a.mask[p] != 0) && A > 0.0 && isfinite(D) && D > 0.0;
    if (!present) return;
    const double jd = floor(D / a.dz);
    if (!(jd >= 0.0 && jd < (double)M)) return;
    const int64_t J = (int64_t)jd + 1;
    const int64_t c = (J * J - 1) / M;
    const int x = (int)(p / N), y = (int)(p % N);
    vol[((int64_t)x * 2 * N + y) * 2 * M + c] = make_double2((1.0 / (double)J) / (double)M * A, 0.0);
}

// One thread per element of the (2N, 2N, 2M) grid (coalesced stores); each
// finds its column's nearest layer(s) to (4 slope)^2 (x^2 + y^2): the
// candidates next to zs M (the true nearest layers are among them), every
// one at the minimal distance marked (ties), layers >= M dropped.  Past the
// grid the minimum falls on the last layer, which is dropped.
__global__ void k_lct_psf(const LctArgs a, double2* psf, int64_t n3)
{
    const int N = a.N, M = a.M;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n3; p += stride) {
        const int k = (int)(p % (2 * M));
        const int64_t col = p / (2 * M);
        const int ix = (int)(col / (2 * N)), iy = (int)(col % (2 * N));
        double v = 0.0;
        if (k < M) {
            const int nx = ix < N ? ix : ix - 2 * N, ny = iy < N ? iy : iy - 2 * N;
            const double x = (double)nx / (double)N, y = (double)ny / (double)N;
            const double zs = a.cone * (x * x + y * y);
            const double kf = floor(zs * (double)M);
            double best = fabs(zs - (double)(2 * M - 1) / (double)M);
            for (int d = -1; d <= 2; ++d) {
                const double kk = kf + d;
                if (kk < 0.0 || kk > (double)(2 * M - 1)) continue;
                best = fmin(best, fabs(zs - kk / (double)M));
            }
            if (fabs(zs - (double)k / (double)M) == best) v = 1.0;
        }
        psf[p] = make_double2(v, 0.0);
    }
}

__global__ void k_lct_mul(double2* vol, const double2* psf, int64_t n, double scale)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double2 u = vol[i], v = psf[i];
        vol[i] = make_double2((u.x * v.x - u.y * v.y) * scale, (u.x * v.y + u.y * v.x) * scale);
    }
}

__global__ void k_lct_out(const LctArgs a, const double2* conv, double* pre)
{
    const int N = a.N, M = a.M;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)N * N * M) return;
    const int j = (int)(p % M);
    const int64_t xy = p / M;
    const int x = (int)(xy / N), y = (int)(xy % N);
    const double2* col = conv + ((int64_t)x * 2 * N + y) * 2 * M;
    const int64_t lo = (int64_t)j * j, hi = (int64_t)(j + 1) * (j + 1);
    double s = 0.0;
    for (int64_t c = lo / M; c <= (hi - 1) / M && c < M; ++c) {
        const int64_t ov = min(hi, (c + 1) * M) - max(lo, c * M);
        if (ov > 0) s += (double)ov / (double)(2 * j + 1) * col[c].x;
    }
    const double v = ((double)(j + 1) * a.dz) * ((double)(j + 1) * a.dz);
    pre[p] = s / pow(v, 1.5);
}

__global__ void k_lct_jitter(const LctArgs a, const double* pre, float* out)
{
    const int M = a.M;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)a.N * a.N * M) return;
    const int t = (int)(p % M);
    const double* row = pre + (p - t);
    double acc = 0.0;
    for (int i = -a.R; i <= a.R; ++i) {
        const int src = t - i;
        if (src >= 0 && src < M) acc += a.taps[i + a.R] * row[src];
    }
    out[p] = (float)acc;
}

// ---------------------------------------------------------------------------
// FFT plans: one per (N, M), created on first use and kept (the FFT library
// allocates its tables then); execution is serialised per plan because the
// stream and work area are plan state.
namespace {

struct PlanEntry {
    hipfftHandle plan = nullptr;
    size_t work = 0;
    bool ok = false;
};

std::mutex g_plan_mu;
std::map<std::pair<int, int>, PlanEntry> g_plans;

PlanEntry* get_plan(int N, int M)
{
    auto& e = g_plans[std::make_pair(N, M)];
    if (e.ok) return &e;
    if (hipfftCreate(&e.plan) != HIPFFT_SUCCESS) return nullptr;
    if (hipfftSetAutoAllocation(e.plan, 0) != HIPFFT_SUCCESS ||
        hipfftMakePlan3d(e.plan, 2 * N, 2 * N, 2 * M, HIPFFT_Z2Z, &e.work) != HIPFFT_SUCCESS) {
        hipfftDestroy(e.plan);
        e.plan = nullptr;
        return nullptr;
    }
    e.ok = true;
    return &e;
}

}  // namespace

int lct_fft_work_bytes(int N, int M, size_t* bytes)
{
    std::lock_guard<std::mutex> lk(g_plan_mu);
    PlanEntry* e = get_plan(N, M);
    if (!e) return -1;
    *bytes = e->work;
    return 0;
}

static hipError_t grid_launch_check() { return hipGetLastError(); }

hipError_t launch_lct(const LctArgs& a, double2* vol, double2* psf, void* fft_work, float* out, hipStream_t st,
                      int* fft_status)
{
    *fft_status = 0;
    const int N = a.N, M = a.M;
    const int64_t n3 = (int64_t)(2 * N) * (2 * N) * (2 * M);
    const unsigned cb = (unsigned)std::min<int64_t>(8192, (n3 + 255) / 256);
    hipLaunchKernelGGL(k_lct_clear, dim3(cb), dim3(256), 0, st, vol, n3);
    hipError_t e = grid_launch_check();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lct_volume, dim3((unsigned)(((int64_t)N * N + 255) / 256)), dim3(256), 0, st, a, vol);
    if ((e = grid_launch_check()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lct_psf, dim3(cb), dim3(256), 0, st, a, psf, n3);
    if ((e = grid_launch_check()) != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        PlanEntry* pe = get_plan(N, M);
        if (!pe || hipfftSetStream(pe->plan, st) != HIPFFT_SUCCESS ||
            hipfftSetWorkArea(pe->plan, fft_work) != HIPFFT_SUCCESS ||
            hipfftExecZ2Z(pe->plan, reinterpret_cast<hipfftDoubleComplex*>(vol),
                          reinterpret_cast<hipfftDoubleComplex*>(vol), HIPFFT_FORWARD) != HIPFFT_SUCCESS ||
            hipfftExecZ2Z(pe->plan, reinterpret_cast<hipfftDoubleComplex*>(psf),
                          reinterpret_cast<hipfftDoubleComplex*>(psf), HIPFFT_FORWARD) != HIPFFT_SUCCESS) {
            *fft_status = -1;
            return hipSuccess;
        }
        hipLaunchKernelGGL(k_lct_mul, dim3(cb), dim3(256), 0, st, vol, psf, n3, 1.0 / (double)n3);
        if ((e = grid_launch_check()) != hipSuccess) return e;
        if (hipfftExecZ2Z(pe->plan, reinterpret_cast<hipfftDoubleComplex*>(vol),
                          reinterpret_cast<hipfftDoubleComplex*>(vol), HIPFFT_BACKWARD) != HIPFFT_SUCCESS) {
            *fft_status = -1;
            return hipSuccess;
        }
    }
    const int64_t no = (int64_t)N * N * M;
    double* pre = reinterpret_cast<double*>(psf);   // the transformed cone is no longer needed
    hipLaunchKernelGGL(k_lct_out, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, st, a, vol, pre);
    if ((e = grid_launch_check()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_lct_jitter, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, st, a, pre, out);
    return grid_launch_check();
}

}  // namespace nlos
