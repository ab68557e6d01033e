// Fused update kernels of the iterative reconstructions of Sec. 4.2 of
// Hauptmann, Kunyansky & Poimala (arXiv 2510.24687), run between the
// library's A / A* launches:
//   projected-gradient NNLS (eq. eqn:NNLS, eq:NNLS-projstep, eqn:projectionHalfCircle)
//   Chambolle-Pock / PDHG for TV-regularised least squares (eqs. eqn:PDHG-dual,
//   eqn:PDHG-primal, eqn:PDHG-relaxation) with K = [A; grad_h], the data term
//   1/2 ||A f - g||^2_Y, the regulariser lam * sum h^2 |grad_h f| and f >= 0.
// grad_h uses forward differences divided by h with a zero last difference
// (Neumann); div_h is minus its adjoint, so <grad_h f, p> = -<f, div_h p>.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>

#include "pat_internal.h"

#include <mutex>

namespace pat {
int plan_image_size(pat_plan p, int* n, int* nt, int* m, double* h, int* is_f64);
int plan_device(pat_plan p);
}

namespace {

constexpr int NT = 256;

template <typename T>
__global__ __launch_bounds__(NT) void k_axpby(long count, T a, const T* x, T b, const T* y, T* r)
{
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < count; i += (long)gridDim.x * NT)
        r[i] = a * x[i] + (y ? b * y[i] : T(0));
}

template <typename T>
__global__ __launch_bounds__(NT) void k_nnls(long count, T* f, const T* grad, T tau, const T* support)
{
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < count; i += (long)gridDim.x * NT) {
        T v = f[i] - tau * grad[i];
        v = v > T(0) ? v : T(0);
        f[i] = support ? v * support[i] : v;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_dual_data(long count, T* q, const T* Af, const T* g, T sigma)
{
    const T inv = T(1) / (T(1) + sigma);
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < count; i += (long)gridDim.x * NT)
        q[i] = (q[i] + sigma * (Af[i] - g[i])) * inv;
}

// p = (px, py) stored as two n x n planes per image: p[b][0] = x-differences, p[b][1] = y-differences
template <typename T>
__global__ __launch_bounds__(NT) void k_dual_tv(int B, int n, T* p, const T* fbar, T sigma, T lam, T inv_h)
{
    const long per = (long)n * n;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < B * per; i += (long)gridDim.x * NT) {
        const long b = i / per, k = i - b * per;
        const int r = (int)(k / n), c = (int)(k - (long)r * n);
        const T* fb = fbar + b * per;
        const T gx = c < n - 1 ? (fb[k + 1] - fb[k]) * inv_h : T(0);
        const T gy = r < n - 1 ? (fb[k + n] - fb[k]) * inv_h : T(0);
        T* px = p + b * 2 * per;
        T* py = px + per;
        T ax = px[k] + sigma * gx, ay = py[k] + sigma * gy;
        const T mag = sqrt(ax * ax + ay * ay);
        const T s = mag > lam ? lam / mag : T(1);
        px[k] = ax * s;
        py[k] = ay * s;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_primal(int B, int n, T* f, T* fbar, const T* Aq, const T* p, T tau, T theta,
                                               T inv_h, const T* support)
{
    const long per = (long)n * n;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < B * per; i += (long)gridDim.x * NT) {
        const long b = i / per, k = i - b * per;
        const int r = (int)(k / n), c = (int)(k - (long)r * n);
        const T* px = p + b * 2 * per;
        const T* py = px + per;
        // div_h p = (px[c] - px[c-1])/h + (py[r] - py[r-1])/h, with the last difference excluded
        T dx = (c < n - 1 ? px[k] : T(0)) - (c > 0 ? px[k - 1] : T(0));
        T dy = (r < n - 1 ? py[k] : T(0)) - (r > 0 ? py[k - n] : T(0));
        const T div = (dx + dy) * inv_h;
        const T f_old = f[i];
        T v = f_old - tau * (Aq[i] - div);
        v = v > T(0) ? v : T(0);
        if (support) v *= support[i];
        f[i] = v;
        fbar[i] = v + theta * (v - f_old);
    }
}

// Deterministic inner product, first stage: per-block partial sums of x*y
// (FP64 accumulation), blocks = gridDim.x.
template <typename T>
__global__ __launch_bounds__(NT) void k_dot_partial(long count, const T* x, const T* y, double* part)
{
    __shared__ double red[NT];
    double acc = 0.0;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < count; i += (long)gridDim.x * NT)
        acc += (double)x[i] * (double)y[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = NT / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// second stage: out[0] = sum of nparts partials (one block)
__global__ __launch_bounds__(NT) void k_dot_final(const double* part, int nparts, double* out)
{
    __shared__ double red[NT];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += NT) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = NT / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// Batched inner products: out[b] = sum_i x_b[i] y_b[i] in FP64, blocks (DOT_PARTS, B),
// a fixed summation order (grid-stride per thread, tree per block, tree over blocks).
constexpr int DOT_PARTS = 64;

template <typename T>
__global__ __launch_bounds__(NT) void k_dotb_partial(long count, long stride, const T* x, const T* y, double* part)
{
    __shared__ double red[NT];
    const int b = blockIdx.y;
    const T* xb = x + (size_t)b * stride;
    const T* yb = y + (size_t)b * stride;
    double acc = 0.0;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < count; i += (long)gridDim.x * NT)
        acc += (double)xb[i] * (double)yb[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = NT / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)b * DOT_PARTS + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NT) void k_dotb_final(const double* part, int nparts, double* out)
{
    __shared__ double red[NT];
    const int b = blockIdx.x;
    red[threadIdx.x] = threadIdx.x < nparts ? part[(size_t)b * DOT_PARTS + threadIdx.x] : 0.0;
    __syncthreads();
    for (int k = NT / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = red[0];
}

// x *= 1 / sqrt(*ss) (ss on the device)
template <typename T>
__global__ __launch_bounds__(NT) void k_scale_rsqrt(long count, T* x, const double* ss)
{
    const T s = (T)(1.0 / sqrt(*ss > 0.0 ? *ss : 1.0));
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < count; i += (long)gridDim.x * NT) x[i] *= s;
}

// deterministic start vector: a counter-based hash of the index mapped to [-1, 1)
template <typename T>
__global__ __launch_bounds__(NT) void k_hash_fill(long count, T* x, unsigned seed)
{
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < count; i += (long)gridDim.x * NT) {
        unsigned v = (unsigned)i * 0x9E3779B9u ^ seed;
        v ^= v >> 16; v *= 0x85EBCA6Bu; v ^= v >> 13; v *= 0xC2B2AE35u; v ^= v >> 16;
        x[i] = (T)((double)v * (2.0 / 4294967296.0) - 1.0);
    }
}

// Partial sums of pat_dot_batched_noalloc: DOT_PARTS doubles per image for at
// most DOT_NOALLOC_MAX_B images (2 MiB), one copy per GPU that the library
// runs on, held until the process ends.  Host code never passes the symbol
// itself to a kernel (in host code it names a host-side stand-in): it uses the
// device address that hipGetSymbolAddress returns for the current device.
constexpr int DOT_NOALLOC_MAX_B = 4096;

}  // namespace

static __device__ __align__(256) double scratch[DOT_PARTS * DOT_NOALLOC_MAX_B];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on device dev (which must be current), looked up
// once per device and kept.
int scratch_address(int dev, double** out)
{
    if (dev < 0 || dev >= MAX_DEVICES) {
        pat::set_error("pat_dot_batched_noalloc: device index out of range");
        return PAT_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            pat::set_error(std::string("pat_dot_batched_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return PAT_EHIP;
        }
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return PAT_OK;
}

int grid_for(long count)
{
    long g = (count + NT - 1) / NT;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

int launch_status(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        pat::set_error(std::string(what) + ": " + hipGetErrorString(e));
        return PAT_EHIP;
    }
    return PAT_OK;
}

}  // namespace

extern "C" {

int pat_axpby(pat_plan p, long count, double a, const void* x, double b, const void* y, void* r, void* stream)
{
    int n, nt, m, f64;
    double h;
    if (!p || !x || !r || count < 0) { pat::set_error("pat_axpby: bad arguments"); return PAT_EINVAL; }
    if (pat::plan_image_size(p, &n, &nt, &m, &h, &f64)) return PAT_EINVAL;
    if (count == 0) return PAT_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (f64)
        k_axpby<double><<<grid_for(count), NT, 0, st>>>(count, a, (const double*)x, b, (const double*)y, (double*)r);
    else
        k_axpby<float><<<grid_for(count), NT, 0, st>>>(count, (float)a, (const float*)x, (float)b, (const float*)y, (float*)r);
    return launch_status("pat_axpby");
}

int pat_dot_batched(pat_plan p, int B, long count, long stride, const void* x, const void* y, double* out,
                    double* scratch, void* stream)
{
    int n, nt, m, f64;
    double h;
    if (!p || !x || !y || !out || !scratch || B < 1 || count < 1 || stride < count) {
        pat::set_error("pat_dot_batched: bad arguments");
        return PAT_EINVAL;
    }
    if (pat::plan_image_size(p, &n, &nt, &m, &h, &f64)) return PAT_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int parts = std::min(DOT_PARTS, grid_for(count));
    const dim3 grid(parts, B);
    if (f64)
        k_dotb_partial<double><<<grid, NT, 0, st>>>(count, stride, (const double*)x, (const double*)y, scratch);
    else
        k_dotb_partial<float><<<grid, NT, 0, st>>>(count, stride, (const float*)x, (const float*)y, scratch);
    k_dotb_final<<<B, NT, 0, st>>>(scratch, parts, out);
    return launch_status("pat_dot_batched");
}

int pat_dot_batched_noalloc(pat_plan p, int B, long count, long stride, const void* x, const void* y, double* out,
                            void* stream)
{
    int n, nt, m, f64;
    double h;
    if (!p || !x || !y || !out || B < 1 || count < 1 || stride < count) {
        pat::set_error("pat_dot_batched_noalloc: bad arguments");
        return PAT_EINVAL;
    }
    if (B > DOT_NOALLOC_MAX_B) {
        pat::set_error("pat_dot_batched_noalloc: batch " + std::to_string(B) + " exceeds the static scratch limit of " +
                       std::to_string(DOT_NOALLOC_MAX_B) + " images (use pat_dot_batched with a scratch buffer)");
        return PAT_EINVAL;
    }
    if (pat::plan_image_size(p, &n, &nt, &m, &h, &f64)) return PAT_EINVAL;
    const int dev = pat::plan_device(p);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) {
        pat::set_error("pat_dot_batched_noalloc: no HIP device");
        return PAT_EHIP;
    }
    if (cur != dev) {
        pat::set_error("pat_dot_batched_noalloc: the plan's device is not the current device");
        return PAT_EINVAL;
    }
    double* part = nullptr;
    int rc = scratch_address(dev, &part);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // every partial that k_dotb_final reads is written by k_dotb_partial first,
    // so the scratch needs no clearing between calls
    const int parts = std::min(DOT_PARTS, grid_for(count));
    const dim3 grid(parts, B);
    if (f64)
        k_dotb_partial<double><<<grid, NT, 0, st>>>(count, stride, (const double*)x, (const double*)y, part);
    else
        k_dotb_partial<float><<<grid, NT, 0, st>>>(count, stride, (const float*)x, (const float*)y, part);
    k_dotb_final<<<B, NT, 0, st>>>(part, parts, out);
    return launch_status("pat_dot_batched_noalloc");
}

int pat_nnls_update(pat_plan p, int B, void* f, const void* grad, double tau, const void* support, void* stream)
{
    int n, nt, m, f64;
    double h;
    if (!p || !f || !grad || B < 1) { pat::set_error("pat_nnls_update: bad arguments"); return PAT_EINVAL; }
    if (pat::plan_image_size(p, &n, &nt, &m, &h, &f64)) return PAT_EINVAL;
    const long count = (long)B * n * n;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (f64)
        k_nnls<double><<<grid_for(count), NT, 0, st>>>(count, (double*)f, (const double*)grad, tau, (const double*)support);
    else
        k_nnls<float><<<grid_for(count), NT, 0, st>>>(count, (float*)f, (const float*)grad, (float)tau, (const float*)support);
    return launch_status("pat_nnls_update");
}

int pat_cp_dual_data(pat_plan p, int B, void* q, const void* Afbar, const void* g, double sigma, void* stream)
{
    int n, nt, m, f64;
    double h;
    if (!p || !q || !Afbar || !g || B < 1) { pat::set_error("pat_cp_dual_data: bad arguments"); return PAT_EINVAL; }
    if (pat::plan_image_size(p, &n, &nt, &m, &h, &f64)) return PAT_EINVAL;
    const long count = (long)B * nt * m;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (f64)
        k_dual_data<double><<<grid_for(count), NT, 0, st>>>(count, (double*)q, (const double*)Afbar, (const double*)g, sigma);
    else
        k_dual_data<float><<<grid_for(count), NT, 0, st>>>(count, (float*)q, (const float*)Afbar, (const float*)g, (float)sigma);
    return launch_status("pat_cp_dual_data");
}

int pat_cp_dual_tv(pat_plan p, int B, void* pgrad, const void* fbar, double sigma, double lam, void* stream)
{
    int n, nt, m, f64;
    double h;
    if (!p || !pgrad || !fbar || B < 1 || !(lam >= 0)) { pat::set_error("pat_cp_dual_tv: bad arguments"); return PAT_EINVAL; }
    if (pat::plan_image_size(p, &n, &nt, &m, &h, &f64)) return PAT_EINVAL;
    const long count = (long)B * n * n;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (f64)
        k_dual_tv<double><<<grid_for(count), NT, 0, st>>>(B, n, (double*)pgrad, (const double*)fbar, sigma, lam, 1.0 / h);
    else
        k_dual_tv<float><<<grid_for(count), NT, 0, st>>>(B, n, (float*)pgrad, (const float*)fbar, (float)sigma, (float)lam,
                                                          (float)(1.0 / h));
    return launch_status("pat_cp_dual_tv");
}

int pat_cp_primal(pat_plan p, int B, void* f, void* fbar, const void* Astar_q, const void* pgrad, double tau,
                  double theta, const void* support, void* stream)
{
    int n, nt, m, f64;
    double h;
    if (!p || !f || !fbar || !Astar_q || !pgrad || B < 1) { pat::set_error("pat_cp_primal: bad arguments"); return PAT_EINVAL; }
    if (pat::plan_image_size(p, &n, &nt, &m, &h, &f64)) return PAT_EINVAL;
    const long count = (long)B * n * n;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (f64)
        k_primal<double><<<grid_for(count), NT, 0, st>>>(B, n, (double*)f, (double*)fbar, (const double*)Astar_q,
                                                          (const double*)pgrad, tau, theta, 1.0 / h, (const double*)support);
    else
        k_primal<float><<<grid_for(count), NT, 0, st>>>(B, n, (float*)f, (float*)fbar, (const float*)Astar_q,
                                                         (const float*)pgrad, (float)tau, (float)theta, (float)(1.0 / h),
                                                         (const float*)support);
    return launch_status("pat_cp_primal");
}

}  // extern "C"

namespace {

template <typename T>
int opnorm_run(pat_plan p, int n, int nt, int m, int iters, double* norm, void* ws, hipStream_t st)
{
    const long fc = (long)n * n, gc = (long)nt * m;
    T *f = nullptr, *u = nullptr, *g = nullptr;
    double *part = nullptr, *scal = nullptr;
    constexpr int NPART = 256;
    int rc = PAT_OK;
    auto cleanup = [&]() {
        if (f) (void)hipFree(f);
        if (u) (void)hipFree(u);
        if (g) (void)hipFree(g);
        if (part) (void)hipFree(part);
        if (scal) (void)hipFree(scal);
    };
    if (hipMalloc(&f, sizeof(T) * fc) != hipSuccess || hipMalloc(&u, sizeof(T) * fc) != hipSuccess ||
        hipMalloc(&g, sizeof(T) * gc) != hipSuccess || hipMalloc(&part, sizeof(double) * NPART) != hipSuccess ||
        hipMalloc(&scal, sizeof(double) * 2) != hipSuccess) {
        cleanup();
        pat::set_error("pat_opnorm_estimate: allocation failed");
        return PAT_ENOMEM;
    }
    const int gb = std::min(NPART, grid_for(fc));
    k_hash_fill<T><<<grid_for(fc), NT, 0, st>>>(fc, f, 12345u);
    for (int it = 0; it < iters && !rc; ++it) {
        // f /= ||f||;  u = A* A f;  lambda = <f, u> / <f, f> (the X weights cancel)
        k_dot_partial<T><<<gb, NT, 0, st>>>(fc, f, f, part);
        k_dot_final<<<1, NT, 0, st>>>(part, gb, scal);
        k_scale_rsqrt<T><<<grid_for(fc), NT, 0, st>>>(fc, f, scal);
        if ((rc = launch_status("pat_opnorm_estimate"))) break;
        if ((rc = pat_forward(p, f, g, ws, st))) break;
        if ((rc = pat_adjoint(p, g, u, ws, st))) break;
        k_dot_partial<T><<<gb, NT, 0, st>>>(fc, f, u, part);
        k_dot_final<<<1, NT, 0, st>>>(part, gb, scal + 1);
        if ((rc = launch_status("pat_opnorm_estimate"))) break;
        std::swap(f, u);
    }
    double lam = 0.0;
    if (!rc) {
        if (hipMemcpyAsync(&lam, scal + 1, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            pat::set_error("pat_opnorm_estimate: read-back failed");
            rc = PAT_EHIP;
        }
    }
    cleanup();
    if (!rc) *norm = std::sqrt(std::max(lam, 0.0));
    return rc;
}

}  // namespace

extern "C" {

int pat_opnorm_estimate(pat_plan p, int iters, double* norm, void* ws, void* stream)
{
    int n, nt, m, f64;
    double h;
    if (!p || !norm || !ws || iters < 1) { pat::set_error("pat_opnorm_estimate: bad arguments"); return PAT_EINVAL; }
    if (pat::plan_image_size(p, &n, &nt, &m, &h, &f64)) return PAT_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return f64 ? opnorm_run<double>(p, n, nt, m, iters, norm, ws, st) : opnorm_run<float>(p, n, nt, m, iters, norm, ws, st);
}

}  // extern "C"
