// Kernels of the learned primal-dual reconstructor (eqs. eq:LPD_dual,
// eq:LPD_primal and the training loss eq:emp_loss of Hauptmann, Kunyansky &
// Poimala, arXiv 2510.24687, Sec. 4.2.1): 3x3 convolutions (stride 1, zero
// padding 1) as implicit GEMMs on the BF16 matrix cores with FP32
// accumulation, bias / PReLU / residual fused into the epilogue; the weight
// gradient as a second MFMA contraction over pixels with a deterministic
// two-stage sum; PReLU backward; weight packing; Adam with cosine decay.
//
// Matrix cores: v_mfma_f32_16x16x32_bf16 for the 32-channel NHWC inputs
// (one tap's 32 channels per instruction), v_mfma_f32_16x16x16_bf16
// (__builtin_amdgcn_mfma_f32_16x16x16bf16_1k) for the planar inputs and the
// weight gradient.  Operand layout for a wave (64 lanes, l = lane; KS = 32 or
// 16 reduction entries per instruction, V = KS / 4 per lane):
//   A (16 x KS, rows i, reduction k): lane l holds A[l % 16][V (l / 16) + e]
//   B (KS x 16, reduction k, cols j): lane l holds B[V (l / 16) + e][l % 16]
//   D (16 x 16):                      lane l holds D[4 (l / 16) + r][l % 16], r = 0..3
// Convolution GEMM: rows = 16 pixels of one image row, cols = output channels,
// reduction k = tap * CINP + channel, tap = 3 ky + kx (correlation, the usual
// deep-learning convention).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "pat_internal.h"

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int NT = 256;     // 4 waves
constexpr int GROUPS = 4;   // 16-pixel groups per wave: a block covers 256 pixels of one row
constexpr int HID = 32;     // hidden channels (NHWC channel pitch)

__device__ __forceinline__ short to_bf16(float x)
{
    // round to nearest, ties to even (inputs are finite)
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

struct ConvArgs {
    int B, H, W, cin, cout;
    const float* in[4];      // planar input planes (FP32, cin of them)
    const short* in16;       // NHWC input (bf16, 32 channels)
    float* out[4];           // planar outputs (FP32; null = channel not written)
    short* out16;            // NHWC output (bf16)
    const float* res[4];     // planar residuals (null = none)
    float scale[4];          // planar input scales (planar in) / planar output scales (planar out)
    const short* weight;     // packed bf16 [CT*16][9*CINP]
    const float* bias;       // [cout] or null
    const float* alpha;      // PReLU slopes [cout] (forward) or of the PReLU being differentiated
    float* pre;              // forward, NHWC out: FP32 copy of the pre-activation, or null
    const float* bwd_pre;    // backward, NHWC out: pre-activation of the PReLU being differentiated
    float* part;             // backward: per-block partial sums [block][64]
};

// 4 consecutive reduction entries k..k+3 (one tap, channels c..c+3) of pixel (y, x)
template <int CINP, bool PLANAR>
__device__ __forceinline__ bf16x4 gather4(const ConvArgs& a, int b, int y, int x, int k)
{
    const int tap = k / CINP, c = k - tap * CINP;
    const int sy = y + tap / 3 - 1, sx = x + tap % 3 - 1;
    const bool in = tap < 9 && x < a.W && sy >= 0 && sy < a.H && sx >= 0 && sx < a.W;
    const size_t p = ((size_t)b * a.H + sy) * a.W + sx;
    if (PLANAR) {
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (in) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (c + e < a.cin) v[e] = a.in[c + e][p] * a.scale[c + e];
        }
        bf16x4 r;
#pragma unroll
        for (int e = 0; e < 4; ++e) r[e] = to_bf16(v[e]);
        return r;
    } else {
        bf16x4 r = {0, 0, 0, 0};
        if (in) r = *reinterpret_cast<const bf16x4*>(a.in16 + p * HID + c);
        return r;
    }
}

// Block: 256 consecutive pixels of one image row; wave w covers pixels
// 64 w .. 64 w + 63 as GROUPS groups of 16.  Weights are staged in LDS once.
// NHWC outputs have two epilogues: forward (bias, PReLU, bf16 activation and
// optional FP32 pre-activation) and backward (the input gradient of a layer
// followed by the PReLU backward of the layer below: gx = ga * (pre > 0 ? 1 :
// alpha), stored bf16, with per-block partial sums of gx and ga * pre * [pre
// <= 0] for the bias and slope gradients).
template <int CINP, bool PLANAR_IN, int CT, bool PLANAR_OUT, bool BWD>
__global__ __launch_bounds__(NT) void conv3x3_fwd(ConvArgs a)
{
    constexpr int K = 9 * CINP;
    constexpr int KP = (K + 15) / 16 * 16;
    __shared__ __align__(16) short wl[CT * 16 * KP];
    __shared__ float red[BWD ? 4 * 4 * 2 * CT * 16 : 1];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = blockIdx.z, y = blockIdx.y;
    const int xw = blockIdx.x * (64 * GROUPS) + wave * (16 * GROUPS);
    for (int i = threadIdx.x; i < CT * 16 * KP; i += NT) {
        const int co = i / KP, k = i - co * KP;
        wl[i] = (k < K) ? a.weight[(size_t)co * K + k] : (short)0;
    }
    __syncthreads();
    const bool active = xw < a.W;
    f32x4 acc[GROUPS][CT];
#pragma unroll
    for (int g = 0; g < GROUPS; ++g)
#pragma unroll
        for (int t = 0; t < CT; ++t) acc[g][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kq = 4 * (lane >> 4);
    if constexpr (!PLANAR_IN && CINP % 32 == 0) {
        // 32 reduction entries (one tap's 32 channels) per instruction: 16-byte
        // operand loads from the NHWC input and from the staged weights
        if (active) {
            for (int k0 = 0; k0 < KP; k0 += 32) {
                const int tap = k0 / CINP, c = k0 - tap * CINP + 8 * (lane >> 4);
                const int dy = tap / 3 - 1, dx = tap % 3 - 1;
                s16x8 bv[CT];
#pragma unroll
                for (int t = 0; t < CT; ++t)
                    bv[t] = *reinterpret_cast<const s16x8*>(wl + (t * 16 + (lane & 15)) * KP + k0 + 8 * (lane >> 4));
#pragma unroll
                for (int g = 0; g < GROUPS; ++g) {
                    const int x = xw + 16 * g + (lane & 15), sy = y + dy, sx = x + dx;
                    s16x8 av = {0, 0, 0, 0, 0, 0, 0, 0};
                    if (x < a.W && sy >= 0 && sy < a.H && sx >= 0 && sx < a.W)
                        av = *reinterpret_cast<const s16x8*>(a.in16 + (((size_t)b * a.H + sy) * a.W + sx) * HID + c);
#pragma unroll
                    for (int t = 0; t < CT; ++t)
                        acc[g][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                                             __builtin_bit_cast(bf16x8, bv[t]),
                                                                             acc[g][t], 0, 0, 0);
                }
            }
        }
    } else if (active) {
        for (int k0 = 0; k0 < KP; k0 += 16) {
            bf16x4 bv[CT];
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const short* wp = wl + (t * 16 + (lane & 15)) * KP + k0 + kq;
                bv[t][0] = wp[0]; bv[t][1] = wp[1]; bv[t][2] = wp[2]; bv[t][3] = wp[3];
            }
#pragma unroll
            for (int g = 0; g < GROUPS; ++g) {
                const bf16x4 av = gather4<CINP, PLANAR_IN>(a, b, y, xw + 16 * g + (lane & 15), k0 + kq);
#pragma unroll
                for (int t = 0; t < CT; ++t)
                    acc[g][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv[t], acc[g][t], 0, 0, 0);
            }
        }
    }
    float sb[CT], sa[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) sb[t] = sa[t] = 0.f;
    if (active) {
#pragma unroll
        for (int g = 0; g < GROUPS; ++g) {
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const int co = t * 16 + (lane & 15);
                if (co >= a.cout) continue;
                const float bias = a.bias ? a.bias[co] : 0.f;
                const float alpha = a.alpha ? a.alpha[co] : 1.f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int x = xw + 16 * g + 4 * (lane >> 4) + r;
                    if (x >= a.W) continue;
                    float v = acc[g][t][r] + bias;
                    const size_t pix = ((size_t)b * a.H + y) * a.W + x;
                    if (PLANAR_OUT) {
                        float* o = a.out[co];
                        if (!o) continue;
                        v *= a.scale[co];
                        if (a.res[co]) v += a.res[co][pix];
                        o[pix] = v;
                    } else if (BWD) {
                        const float xp = a.bwd_pre[pix * HID + co];
                        const float gx = xp > 0.f ? v : alpha * v;
                        sb[t] += gx;
                        if (!(xp > 0.f)) sa[t] += v * xp;
                        a.out16[pix * HID + co] = to_bf16(gx);
                    } else {
                        if (a.pre) a.pre[pix * HID + co] = v;
                        if (a.alpha) v = v > 0.f ? v : alpha * v;
                        a.out16[pix * HID + co] = to_bf16(v);
                    }
                }
            }
        }
    }
    if (BWD) {
        // block partials: channel co = t*16 + (lane & 15), summed over the 4 lane
        // groups and the 4 waves in a fixed order
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            red[((wave * 4 + (lane >> 4)) * 2 + 0) * CT * 16 + t * 16 + (lane & 15)] = sb[t];
            red[((wave * 4 + (lane >> 4)) * 2 + 1) * CT * 16 + t * 16 + (lane & 15)] = sa[t];
        }
        __syncthreads();
        if (threadIdx.x < 2 * HID) {
            const int kind = threadIdx.x / HID, co = threadIdx.x % HID;
            float s = 0.f;
            if (co < CT * 16)
                for (int q = 0; q < 16; ++q) s += red[(q * 2 + kind) * CT * 16 + co];
            const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            a.part[blk * 64 + threadIdx.x] = s;
        }
    }
}

// Weight-gradient partials of one chunk (ROWS image rows of one image):
//   part[chunk][co][k] = sum_p grad[p][co] * patch[p][k]
// as an MFMA contraction with rows = output channels (A = grad), columns = k
// (B = patch), reduction over the chunk's pixels.  With CT = 2 waves 0,1 take
// output tile 0 and waves 2,3 tile 1, splitting the k tiles even / odd; with
// CT = 1 the k tiles go round-robin over the 4 waves.  Accumulators stay in
// registers for the whole chunk.
struct WgradArgs {
    ConvArgs x;              // x.in / x.in16: layer input as in the forward; x.cout: output channels
    const float* grad;       // planar gradient of the layer output (cout == 1), or null
    const short* grad16;     // NHWC bf16 gradient of the layer output
    int rows;                // image rows per chunk
    float* part;             // [chunks][CT*16][KP]
};

template <int CINP, bool PLANAR_IN, int CT, bool PLANAR_G>
__global__ __launch_bounds__(NT) void conv3x3_wgrad(WgradArgs w)
{
    constexpr int K = 9 * CINP;
    constexpr int KP = (K + 15) / 16 * 16;
    constexpr int KT = KP / 16;
    constexpr int STRIDE = CT == 2 ? 2 : 4;
    constexpr int MAXT = (KT + STRIDE - 1) / STRIDE;
    const ConvArgs& a = w.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = blockIdx.y;
    const int chunk = b * gridDim.x + blockIdx.x;
    const int y0 = blockIdx.x * w.rows;
    const int y1 = min(a.H, y0 + w.rows);
    const int npix = (y1 - y0) * a.W;
    const int tco = CT == 2 ? (wave >> 1) : 0;
    const int tk0 = CT == 2 ? (wave & 1) : wave;
    const int co = tco * 16 + (lane & 15);
    f32x4 acc[MAXT];
#pragma unroll
    for (int j = 0; j < MAXT; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int p0 = 0; p0 < npix; p0 += 16) {
        int yy[4], xx[4];
        bf16x4 av;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int pl = p0 + 4 * (lane >> 4) + e;
            yy[e] = pl < npix ? y0 + pl / a.W : -10;
            xx[e] = pl < npix ? pl % a.W : 0;
            short gv = 0;
            if (yy[e] >= 0 && co < a.cout) {
                const size_t pix = ((size_t)b * a.H + yy[e]) * a.W + xx[e];
                gv = PLANAR_G ? to_bf16(w.grad[pix]) : w.grad16[pix * HID + co];
            }
            av[e] = gv;
        }
#pragma unroll
        for (int j = 0; j < MAXT; ++j) {
            const int tk = tk0 + STRIDE * j;
            if (tk >= KT) continue;
            const int kk = tk * 16 + (lane & 15);
            const int tap = kk / CINP, c = kk - tap * CINP;
            bf16x4 bv;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                short pv = 0;
                const int sy = yy[e] + tap / 3 - 1, sx = xx[e] + tap % 3 - 1;
                if (kk < K && yy[e] >= 0 && sy >= 0 && sy < a.H && sx >= 0 && sx < a.W) {
                    const size_t sp = ((size_t)b * a.H + sy) * a.W + sx;
                    if (PLANAR_IN) pv = c < a.cin ? to_bf16(a.in[c][sp] * a.scale[c]) : (short)0;
                    else pv = a.in16[sp * HID + c];
                }
                bv[e] = pv;
            }
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[j], 0, 0, 0);
        }
    }
    float* dst = w.part + (size_t)chunk * (CT * 16) * KP;
#pragma unroll
    for (int j = 0; j < MAXT; ++j) {
        const int tk = tk0 + STRIDE * j;
        if (tk >= KT) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            dst[(size_t)(tco * 16 + 4 * (lane >> 4) + r) * KP + tk * 16 + (lane & 15)] = acc[j][r];
    }
}

// Deterministic column sums of a row-major partials array part[nrows][ncols]
// (FP64 accumulation in a fixed order).  A block covers 16 consecutive
// columns with 16 row groups: thread (c, g) sums rows g, g + 16, ... of
// column c, then the 16 group sums are added in LDS in a fixed order.
// Output mapping: with cinp == 0, out[j] (+)= sum_i part[i][j]; with cinp > 0
// the columns are weight-gradient entries (co, k = tap * cinp + ci) of a
// [rows][kp] tile and the sum goes to the FP32 layout gw[co][ci][tap]
// (entries with ci >= cin, k >= 9 cinp or co >= cout are padding).
__global__ __launch_bounds__(NT) void reduce_partials(const float* part, int nrows, int ncols, int kp, int cinp,
                                                      int cout, int cin, float* out, int accumulate)
{
    __shared__ double red[16][17];
    const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int j = blockIdx.x * 16 + c;
    double s = 0.0;
    if (j < ncols) {
#pragma unroll 4
        for (int i = g; i < nrows; i += 16) s += part[(size_t)i * ncols + j];
    }
    red[g][c] = s;
    __syncthreads();
    if (g == 0 && j < ncols) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += red[k][c];
        int o = j;
        if (cinp > 0) {
            const int co = j / kp, k = j - co * kp, tap = k / cinp, ci = k - tap * cinp;
            if (co >= cout || tap >= 9 || ci >= cin) return;
            o = (co * cin + ci) * 9 + tap;
        }
        out[o] = accumulate ? out[o] + (float)t : (float)t;
    }
}

// per-block partial sums of a planar array
__global__ __launch_bounds__(NT) void plane_sum(long count, const float* g, float* part)
{
    __shared__ float s[NT];
    float acc = 0.f;
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < count; i += (long)gridDim.x * NT) acc += g[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = NT / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// Pack FP32 weights w[cout][cin][3][3] into the bf16 layout the conv kernel
// stages: dst[co_e][tap * CINP + ci_e] for the effective convolution.  With
// transpose = 0 the effective convolution is w itself; with transpose = 1 it
// is the input-gradient convolution: cin_e = cout, cout_e = cin and
// w_e[co_e][ci_e][ky][kx] = w[ci_e][co_e][2 - ky][2 - kx].
__global__ __launch_bounds__(NT) void pack_weights(const float* w, int cout, int cin, int transpose, int cinp,
                                                   int rows, short* dst)
{
    const int K = 9 * cinp;
    const int i = blockIdx.x * NT + threadIdx.x;
    if (i >= rows * K) return;
    const int coe = i / K, k = i - coe * K;
    const int tap = k / cinp, cie = k - tap * cinp;
    const int coe_n = transpose ? cin : cout, cie_n = transpose ? cout : cin;
    float v = 0.f;
    if (coe < coe_n && cie < cie_n) {
        if (transpose) v = w[((size_t)cie * cin + coe) * 9 + (8 - tap)];
        else v = w[((size_t)coe * cin + cie) * 9 + tap];
    }
    dst[i] = to_bf16(v);
}

// Squared L2 norm of the gradient, two deterministic stages: per-block FP64
// partial sums, then one block adds them in a fixed order into *out.
__global__ __launch_bounds__(NT) void sumsq_partial(long count, const float* g, double* part)
{
    __shared__ double red[NT];
    double acc = 0.0;
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < count; i += (long)gridDim.x * NT) acc += (double)g[i] * g[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = NT / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NT) void sumsq_final(const double* part, int nparts, double* out)
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

// Adam (bias-corrected moments) with a cosine-decayed step size; the step
// counter lives on the device so that a captured training step can be
// replayed unchanged.  t = *step + 1 on entry.  With gsq != null the
// gradient is first scaled by min(1, clip / ||g||), ||g||^2 = *gsq.
__global__ __launch_bounds__(NT) void adam_step(long count, float* p, const float* g, float* m, float* v,
                                                const int* step, float lr0, float lr_min, int total, float b1,
                                                float b2, float eps, const double* gsq, float clip)
{
    const int t = *step + 1;
    const float gs = (gsq && *gsq > (double)clip * clip) ? (float)(clip / sqrt(*gsq)) : 1.f;
    const float frac = fminf(1.f, (float)(t - 1) / (float)(total > 1 ? total - 1 : 1));
    const float lr = lr_min + 0.5f * (lr0 - lr_min) * (1.f + cosf(3.14159265358979f * frac));
    const float c1 = 1.f / (1.f - powf(b1, (float)t));
    const float c2 = 1.f / (1.f - powf(b2, (float)t));
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < count; i += (long)gridDim.x * NT) {
        const float gi = g[i] * gs;
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

__global__ void step_increment(int* step)
{
    if (threadIdx.x == 0) *step += 1;
}

int status(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        pat::set_error(std::string(what) + ": " + hipGetErrorString(e));
        return PAT_EHIP;
    }
    return PAT_OK;
}

int cinp_of(int in_planar) { return in_planar ? 4 : HID; }
int ct_of(int cout) { return cout > 16 ? 2 : 1; }

ConvArgs make_args(const pat_conv_desc* d)
{
    ConvArgs a;
    a.B = d->B; a.H = d->H; a.W = d->W; a.cin = d->cin; a.cout = d->cout;
    for (int i = 0; i < 4; ++i) {
        a.in[i] = static_cast<const float*>(d->in[i]);
        a.out[i] = static_cast<float*>(d->out[i]);
        a.res[i] = static_cast<const float*>(d->residual[i]);
        a.scale[i] = d->scale[i];
    }
    a.in16 = d->in_planar ? nullptr : static_cast<const short*>(d->in[0]);
    a.out16 = d->out_planar ? nullptr : static_cast<short*>(d->out[0]);
    a.weight = static_cast<const short*>(d->weight);
    a.bias = static_cast<const float*>(d->bias);
    a.alpha = static_cast<const float*>(d->alpha);
    a.pre = static_cast<float*>(d->pre);
    a.bwd_pre = static_cast<const float*>(d->bwd_pre);
    a.part = static_cast<float*>(d->partials);
    return a;
}

int check_desc(const pat_conv_desc* d, const char* who)
{
    auto fail = [&](int code, const char* why) {
        pat::set_error(std::string(who) + ": " + why);
        return code;
    };
    if (!d) return fail(PAT_EINVAL, "null descriptor");
    if (d->B < 1 || d->H < 1 || d->W < 1 || d->H > 65535 || d->B > 65535) return fail(PAT_EINVAL, "bad B, H or W");
    if (d->in_planar ? (d->cin < 1 || d->cin > 4) : d->cin != HID)
        return fail(PAT_EUNSUPPORTED, "cin must be 1..4 (planar) or 32 (NHWC)");
    if (d->out_planar ? (d->cout < 1 || d->cout > 4) : d->cout != HID)
        return fail(PAT_EUNSUPPORTED, "cout must be 1..4 (planar) or 32 (NHWC)");
    for (int i = 0; i < (d->in_planar ? d->cin : 1); ++i)
        if (!d->in[i]) return fail(PAT_EINVAL, "missing input plane");
    if (!d->weight) return fail(PAT_EINVAL, "missing weights");
    if (d->out_planar && (d->pre || d->alpha || d->bwd_pre)) return fail(PAT_EUNSUPPORTED, "PReLU needs an NHWC output");
    if (d->bwd_pre && (!d->alpha || !d->partials || !d->grad_bias_alpha || d->pre || d->bias))
        return fail(PAT_EINVAL, "the PReLU-backward epilogue needs alpha, partials, grad_bias_alpha and no bias / pre");
    return PAT_OK;
}

dim3 conv_grid(const pat_conv_desc* d) { return dim3((d->W + 64 * GROUPS - 1) / (64 * GROUPS), d->H, d->B); }

}  // namespace

extern "C" {

long pat_conv_packed_size(int cout_e, int cin_e, int in_planar)
{
    if (cout_e < 1 || cout_e > HID || cin_e < 1 || (in_planar ? cin_e > 4 : cin_e != HID)) return -1;
    return (long)ct_of(cout_e) * 16 * 9 * cinp_of(in_planar);
}

int pat_conv_pack_weights(const void* w, int cout, int cin, int transpose, int in_planar, void* dst, void* stream)
{
    const int coe = transpose ? cin : cout, cie = transpose ? cout : cin;
    if (!w || !dst || pat_conv_packed_size(coe, cie, in_planar) < 0) {
        pat::set_error("pat_conv_pack_weights: bad arguments");
        return PAT_EINVAL;
    }
    const int rows = ct_of(coe) * 16, cinp = cinp_of(in_planar);
    const int total = rows * 9 * cinp;
    pack_weights<<<(total + NT - 1) / NT, NT, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        static_cast<const float*>(w), cout, cin, transpose, cinp, rows, static_cast<short*>(dst));
    return status("pack_weights");
}

long pat_conv_bwd_partials(const pat_conv_desc* d)
{
    if (!d || d->B < 1 || d->H < 1 || d->W < 1) return -1;
    const dim3 g = conv_grid(d);
    return (long)g.x * g.y * g.z * 64;
}

int pat_conv3x3(const pat_conv_desc* d, void* stream)
{
    int rc = check_desc(d, "pat_conv3x3");
    if (rc) return rc;
    if (!d->out_planar && !d->out[0]) { pat::set_error("pat_conv3x3: missing output"); return PAT_EINVAL; }
    ConvArgs a = make_args(d);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid = conv_grid(d);
    const bool bwd = d->bwd_pre != nullptr;
    if (d->in_planar && !d->out_planar) {
        if (bwd) conv3x3_fwd<4, true, 2, false, true><<<grid, NT, 0, st>>>(a);
        else conv3x3_fwd<4, true, 2, false, false><<<grid, NT, 0, st>>>(a);
    } else if (!d->in_planar && !d->out_planar) {
        if (bwd) conv3x3_fwd<HID, false, 2, false, true><<<grid, NT, 0, st>>>(a);
        else conv3x3_fwd<HID, false, 2, false, false><<<grid, NT, 0, st>>>(a);
    } else if (!d->in_planar && d->out_planar) {
        conv3x3_fwd<HID, false, 1, true, false><<<grid, NT, 0, st>>>(a);
    } else {
        conv3x3_fwd<4, true, 1, true, false><<<grid, NT, 0, st>>>(a);
    }
    if ((rc = status("pat_conv3x3"))) return rc;
    if (bwd) {
        reduce_partials<<<4, NT, 0, st>>>(static_cast<const float*>(d->partials), (int)(grid.x * grid.y * grid.z), 64, 0,
                                          0, 0, 0, static_cast<float*>(d->grad_bias_alpha), d->accumulate);
        rc = status("reduce_partials");
    }
    return rc;
}

long pat_conv_wgrad_partials(const pat_conv_desc* d, int rows_per_chunk)
{
    if (!d || rows_per_chunk < 1 || d->H < 1 || d->B < 1 || d->cout < 1 || d->cout > HID) return -1;
    const long chunks = (d->H + rows_per_chunk - 1) / rows_per_chunk;
    const int kp = (9 * cinp_of(d->in_planar) + 15) / 16 * 16;
    return chunks * d->B * ct_of(d->cout) * 16 * kp;
}

int pat_conv3x3_wgrad(const pat_conv_desc* d, const void* grad_out, int rows_per_chunk, void* partials,
                      void* grad_w, int accumulate, void* stream)
{
    int rc = check_desc(d, "pat_conv3x3_wgrad");
    if (rc) return rc;
    if (!grad_out || !partials || !grad_w || rows_per_chunk < 1) {
        pat::set_error("pat_conv3x3_wgrad: bad arguments");
        return PAT_EINVAL;
    }
    if (d->out_planar && d->cout != 1) {
        pat::set_error("pat_conv3x3_wgrad: a planar output gradient needs cout == 1");
        return PAT_EUNSUPPORTED;
    }
    WgradArgs w;
    w.x = make_args(d);
    w.grad = d->out_planar ? static_cast<const float*>(grad_out) : nullptr;
    w.grad16 = d->out_planar ? nullptr : static_cast<const short*>(grad_out);
    w.rows = rows_per_chunk;
    w.part = static_cast<float*>(partials);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int chunks = (d->H + rows_per_chunk - 1) / rows_per_chunk;
    dim3 grid(chunks, d->B);
    const int cinp = cinp_of(d->in_planar), ct = ct_of(d->cout);
    const int kp = (9 * cinp + 15) / 16 * 16;
    if (d->in_planar && ct == 2) conv3x3_wgrad<4, true, 2, false><<<grid, NT, 0, st>>>(w);
    else if (d->in_planar) conv3x3_wgrad<4, true, 1, true><<<grid, NT, 0, st>>>(w);
    else if (ct == 2) conv3x3_wgrad<HID, false, 2, false><<<grid, NT, 0, st>>>(w);
    else conv3x3_wgrad<HID, false, 1, true><<<grid, NT, 0, st>>>(w);
    if ((rc = status("conv3x3_wgrad"))) return rc;
    const int ncols = ct * 16 * kp;
    reduce_partials<<<(ncols + 15) / 16, NT, 0, st>>>(static_cast<const float*>(partials), chunks * d->B, ncols, kp, cinp,
                                                      d->cout, d->cin, static_cast<float*>(grad_w), accumulate);
    return status("reduce_partials");
}

int pat_plane_sum(long count, const void* g, void* partials, int nblocks, void* out, int accumulate, void* stream)
{
    if (!g || !partials || !out || nblocks < 1 || count < 1) {
        pat::set_error("pat_plane_sum: bad arguments");
        return PAT_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    plane_sum<<<nblocks, NT, 0, st>>>(count, static_cast<const float*>(g), static_cast<float*>(partials));
    int rc = status("plane_sum");
    if (rc) return rc;
    reduce_partials<<<1, NT, 0, st>>>(static_cast<const float*>(partials), nblocks, 1, 0, 0, 0, 0,
                                      static_cast<float*>(out), accumulate);
    return status("reduce_partials");
}

int pat_adam(long count, void* param, const void* grad, void* m, void* v, void* step, double lr, double lr_min,
             int total_steps, double beta1, double beta2, double eps, double clip, void* scratch, void* stream)
{
    if (!param || !grad || !m || !v || !step || count < 1 || total_steps < 1 || !(lr >= 0) || !(lr_min >= 0) ||
        !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0) || !(clip >= 0) ||
        (clip > 0 && !scratch)) {
        pat::set_error("pat_adam: bad arguments");
        return PAT_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    long blocks = (count + NT - 1) / NT;
    if (blocks > 4096) blocks = 4096;
    double* gsq = nullptr;
    if (clip > 0) {
        constexpr int NPART = 64;
        double* part = static_cast<double*>(scratch);
        gsq = part + NPART;
        sumsq_partial<<<(int)std::min<long>(blocks, NPART), NT, 0, st>>>(count, static_cast<const float*>(grad), part);
        sumsq_final<<<1, NT, 0, st>>>(part, (int)std::min<long>(blocks, NPART), gsq);
        int rc = status("sumsq");
        if (rc) return rc;
    }
    adam_step<<<(int)blocks, NT, 0, st>>>(count, static_cast<float*>(param), static_cast<const float*>(grad),
                                          static_cast<float*>(m), static_cast<float*>(v), static_cast<const int*>(step),
                                          (float)lr, (float)lr_min, total_steps, (float)beta1, (float)beta2, (float)eps,
                                          gsq, (float)clip);
    int rc = status("adam_step");
    if (rc) return rc;
    step_increment<<<1, 64, 0, st>>>(static_cast<int*>(step));
    return status("step_increment");
}

}  // extern "C"
