// Kernels of the U-Net variant of the learned primal-dual networks (Sec. 4.2.1
// of Hauptmann, Kunyansky & Poimala, arXiv 2510.24687: four scales, three
// window-2 down- and up-sampling steps, two 3x3 convolutions with batch
// normalisation and ReLU per scale, 32 filters at the first scale doubled at
// every down-sampling).
//
// One generic implicit-GEMM convolution on the BF16 matrix cores covers every
// product of the network: the 3x3 convolutions, their input gradients (the
// same GEMM with transposed, tap-flipped weights), the 2x2 stride-2
// transposed convolution of the up-sampling (one GEMM per output parity) and
// its input gradient (four taps read at stride 2).  A GEMM row is a pixel of
// an "iteration grid"; tap t reads the source pixel (s y + dy_t, s x + dx_t);
// the row's result goes to the destination pixel (o y + oy, o x + ox).  The
// reduction index is k = tap * cin + channel, channels of a two-source input
// are the concatenation [src0 | src1] (the skip connection, without a copy).
//
// Matrix cores: v_mfma_f32_16x16x32_bf16 (gfx950) where every source has a
// multiple of 32 channels, v_mfma_f32_16x16x16_bf16 otherwise (the 16-channel
// padded network input); FP32 accumulation.  Wave operand layout (lane l,
// KS = 32 or 16 reduction entries per instruction, V = KS / 4 per lane):
//   A (16 x KS, rows i, reduction k): lane l holds A[l % 16][V (l / 16) + e]
//   B (KS x 16, reduction k, cols j): lane l holds B[V (l / 16) + e][l % 16]
//   D (16 x 16):                      lane l holds D[4 (l / 16) + r][l % 16]
// Weights are packed so that one wave's B operand is 64 V contiguous bf16.
//
// Activations are NHWC bf16 (the MFMA operands), convolution outputs and
// activation gradients NHWC FP32.  Batch-normalisation statistics, weight
// gradients and the head's sums are deterministic: fixed partitions, FP64
// partial sums, a fixed summation order, no atomics.
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

constexpr int NT = 256;

__device__ __forceinline__ short f2bf(float x)
{
    // round to nearest, ties to even (inputs are finite)
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ float bf2f(short v) { return __uint_as_float(((uint32_t)(uint16_t)v) << 16); }

// Sum over chunks q < chunks of part[q * stride + col] for the 16 columns
// col0 .. col0 + 15 of a block: thread (c = tid % 16, g = tid / 16) adds chunks
// g, g + 16, ... in FP64; the 16 group sums of column c are then added in
// order by thread (c, 0).  Returns the column sum on threads with g == 0
// (col0 + c < ncols), 0 elsewhere.  Every thread of the block must call it.
__device__ double chunk_sum16(const double* part, int chunks, long stride, long col0, long ncols, double* red)
{
    const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
    const long col = col0 + c;
    double s = 0.0;
    if (col < ncols)
        for (int q = g; q < chunks; q += 16) s += part[(size_t)q * stride + col];
    __syncthreads();
    red[threadIdx.x] = s;
    __syncthreads();
    double t = 0.0;
    if (g == 0)
        for (int k = 0; k < 16; ++k) t += red[k * 16 + c];
    return t;
}

__device__ double chunk_sum16f(const float* part, int chunks, long stride, long col0, long ncols, double* red)
{
    const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
    const long col = col0 + c;
    double s = 0.0;
    if (col < ncols)
        for (int q = g; q < chunks; q += 16) s += part[(size_t)q * stride + col];
    __syncthreads();
    red[threadIdx.x] = s;
    __syncthreads();
    double t = 0.0;
    if (g == 0)
        for (int k = 0; k < 16; ++k) t += red[k * 16 + c];
    return t;
}

struct GConv {
    int B, H, W;             // iteration grid
    const short* src0;       // NHWC bf16, c0 channels
    const short* src1;       // NHWC bf16, c1 channels (concatenated after src0), or null with c1 = 0
    int c0, c1;
    int Hs, Ws, istr, ntaps;
    int dy[9], dx[9];
    const short* wp;         // packed weights
    int cout;
    void* dst0;              // channels [0, d0)
    void* dst1;              // channels [d0, d0 + d1)
    int d0, d1, bf0, bf1, acc0, acc1;
    int Ho, Wo, ostr, oy, ox;
};

__device__ __forceinline__ void store_out(void* base, size_t idx, float v, int bf, int acc)
{
    if (bf) {
        static_cast<short*>(base)[idx] = f2bf(v);
    } else {
        float* p = static_cast<float*>(base) + idx;
        *p = acc ? *p + v : v;
    }
}

// One wave computes 64 rows (4 groups of 16) x 16 CTW output channels.  Waves
// are independent (no LDS, no barrier): a wave whose row tile lies past the
// grid returns at once.
template <int CTW>
__global__ __launch_bounds__(NT) void gconv_kernel(GConv a)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nct = a.cout / (16 * CTW);
    const long gw = (long)blockIdx.x * 4 + wave;
    const long R = (long)a.B * a.H * a.W;
    const long rt = gw / nct;
    const int ct = (int)(gw - rt * nct);
    if (rt * 64 >= R) return;
    const int cs16 = (a.c0 + a.c1) >> 4, KT = a.ntaps * cs16;
    int by[4], bx[4], bb[4];
    bool rv[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const long row = rt * 64 + g * 16 + (lane & 15);
        rv[g] = row < R;
        const long r = rv[g] ? row : 0;
        bx[g] = (int)(r % a.W);
        const long t = r / a.W;
        by[g] = (int)(t % a.H);
        bb[g] = (int)(t / a.H);
    }
    f32x4 acc[4][CTW];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int j = 0; j < CTW; ++j) acc[g][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kq = 4 * (lane >> 4);
    const short* wbase = a.wp + (size_t)ct * CTW * KT * 256 + lane * 4;
    for (int t = 0; t < a.ntaps; ++t) {
        long sp[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int sy = a.istr * by[g] + a.dy[t], sx = a.istr * bx[g] + a.dx[t];
            sp[g] = (rv[g] && sy >= 0 && sy < a.Hs && sx >= 0 && sx < a.Ws) ? ((long)bb[g] * a.Hs + sy) * a.Ws + sx : -1;
        }
        for (int cs = 0; cs < cs16; ++cs) {
            const short* base;
            int pitch;
            if (cs * 16 < a.c0) {
                base = a.src0 + cs * 16 + kq;
                pitch = a.c0;
            } else {
                base = a.src1 + (cs * 16 - a.c0) + kq;
                pitch = a.c1;
            }
            const int kt = t * cs16 + cs;
            bf16x4 bv[CTW];
#pragma unroll
            for (int j = 0; j < CTW; ++j) bv[j] = *reinterpret_cast<const bf16x4*>(wbase + ((size_t)j * KT + kt) * 256);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                bf16x4 av = {0, 0, 0, 0};
                if (sp[g] >= 0) av = *reinterpret_cast<const bf16x4*>(base + (size_t)sp[g] * pitch);
#pragma unroll
                for (int j = 0; j < CTW; ++j)
                    acc[g][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv[j], acc[g][j], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long row = rt * 64 + g * 16 + 4 * (lane >> 4) + r;
            if (row >= R) continue;
            const int x = (int)(row % a.W);
            const long tt = row / a.W;
            const int y = (int)(tt % a.H), b = (int)(tt / a.H);
            const size_t op = ((size_t)b * a.Ho + a.ostr * y + a.oy) * a.Wo + a.ostr * x + a.ox;
#pragma unroll
            for (int j = 0; j < CTW; ++j) {
                const int co = (ct * CTW + j) * 16 + (lane & 15);
                const float v = acc[g][j][r];
                if (co < a.d0) store_out(a.dst0, op * a.d0 + co, v, a.bf0, a.acc0);
                else store_out(a.dst1, op * a.d1 + (co - a.d0), v, a.bf1, a.acc1);
            }
        }
    }
}

// The same GEMM with 32 reduction entries per instruction (c0, c1 multiples
// of 32): 16-byte operand loads, and the loads of step kt + 1 are issued
// before the matrix instructions of step kt so that they overlap.
template <int CTW>
__global__ __launch_bounds__(NT) void gconv32_kernel(GConv a)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nct = a.cout / (16 * CTW);
    const long gw = (long)blockIdx.x * 4 + wave;
    const long R = (long)a.B * a.H * a.W;
    const long rt = gw / nct;
    const int ct = (int)(gw - rt * nct);
    if (rt * 64 >= R) return;
    const int cs32 = (a.c0 + a.c1) >> 5, KT = a.ntaps * cs32;
    int by[4], bx[4], bb[4];
    bool rv[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const long row = rt * 64 + g * 16 + (lane & 15);
        rv[g] = row < R;
        const long r = rv[g] ? row : 0;
        bx[g] = (int)(r % a.W);
        const long t = r / a.W;
        by[g] = (int)(t % a.H);
        bb[g] = (int)(t / a.H);
    }
    f32x4 acc[4][CTW];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int j = 0; j < CTW; ++j) acc[g][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kq = 8 * (lane >> 4);
    const short* wbase = a.wp + (size_t)ct * CTW * KT * 512 + lane * 8;
    s16x8 an[4], bn[CTW];
    auto load = [&](int kt) {
        const int t = kt / cs32, cs = kt - t * cs32;
        const short* base;
        int pitch;
        if (cs * 32 < a.c0) {
            base = a.src0 + cs * 32 + kq;
            pitch = a.c0;
        } else {
            base = a.src1 + (cs * 32 - a.c0) + kq;
            pitch = a.c1;
        }
        const int dy = a.dy[t], dx = a.dx[t];
#pragma unroll
        for (int j = 0; j < CTW; ++j) bn[j] = *reinterpret_cast<const s16x8*>(wbase + ((size_t)j * KT + kt) * 512);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int sy = a.istr * by[g] + dy, sx = a.istr * bx[g] + dx;
            s16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (rv[g] && sy >= 0 && sy < a.Hs && sx >= 0 && sx < a.Ws)
                v = *reinterpret_cast<const s16x8*>(base + (((size_t)bb[g] * a.Hs + sy) * a.Ws + sx) * pitch);
            an[g] = v;
        }
    };
    load(0);
    for (int kt = 0; kt < KT; ++kt) {
        s16x8 ac[4], bc[CTW];
#pragma unroll
        for (int g = 0; g < 4; ++g) ac[g] = an[g];
#pragma unroll
        for (int j = 0; j < CTW; ++j) bc[j] = bn[j];
        if (kt + 1 < KT) load(kt + 1);
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int j = 0; j < CTW; ++j)
                acc[g][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ac[g]),
                                                                     __builtin_bit_cast(bf16x8, bc[j]), acc[g][j], 0, 0,
                                                                     0);
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long row = rt * 64 + g * 16 + 4 * (lane >> 4) + r;
            if (row >= R) continue;
            const int x = (int)(row % a.W);
            const long tt = row / a.W;
            const int y = (int)(tt % a.H), b = (int)(tt / a.H);
            const size_t op = ((size_t)b * a.Ho + a.ostr * y + a.oy) * a.Wo + a.ostr * x + a.ox;
#pragma unroll
            for (int j = 0; j < CTW; ++j) {
                const int co = (ct * CTW + j) * 16 + (lane & 15);
                const float v = acc[g][j][r];
                if (co < a.d0) store_out(a.dst0, op * a.d0 + co, v, a.bf0, a.acc0);
                else store_out(a.dst1, op * a.d1 + (co - a.d0), v, a.bf1, a.acc1);
            }
        }
    }
}

// The 3x3 stride-1 convolution (zero padding 1, destination = iteration grid)
// with LDS tiles, for sources with multiples of 32 channels and W divisible by
// 16.  A block owns 256 output pixels of one image, a TH x TW tile (TW = 64,
// 32 or 16 dividing W, TH = 256 / TW), and 16 NCT output channels.  For each
// 32-channel chunk it stages the input tile with its one-pixel halo,
// (TH + 2) x (TW + 2) pixels x 32 channels, and the chunk's packed weights
// of all 9 taps, then every wave runs the 9 taps from LDS: wave w computes
// tile pixels 64 w .. 64 w + 63 (4 groups of 16, row-major in the tile).  The
// four 16-byte pieces of a staged pixel p are rotated by p / 4, so that the
// 16 consecutive pixels a quarter-wave reads land in distinct banks.
constexpr int LDS_A_SHORTS = 6 * 66 * 32;   // largest staged tile: TW = 64, TH = 4

template <int NCT>
__global__ __launch_bounds__(NT) void gconv3_lds(GConv a, int TW)
{
    __shared__ __align__(16) short As[LDS_A_SHORTS];
    __shared__ __align__(16) short Bs[9 * NCT * 512];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int TH = 256 / TW, PW = TW + 2, NP = (TH + 2) * PW;
    const int tilesX = a.W / TW, tilesY = (a.H + TH - 1) / TH;
    int tile = blockIdx.x;
    const int tx0 = (tile % tilesX) * TW;
    tile /= tilesX;
    const int ty0 = (tile % tilesY) * TH;
    const int b = tile / tilesY;
    const int ct0 = blockIdx.y * NCT;
    const int cs32 = (a.c0 + a.c1) >> 5, KT = 9 * cs32;
    int oy[4], ox[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int p = wave * 64 + g * 16 + (lane & 15);
        oy[g] = p / TW;
        ox[g] = p - oy[g] * TW;
    }
    f32x4 acc[4][NCT];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int j = 0; j < NCT; ++j) acc[g][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int q = lane >> 4;
    for (int cs = 0; cs < cs32; ++cs) {
        const short* base;
        int pitch;
        if (cs * 32 < a.c0) {
            base = a.src0 + cs * 32;
            pitch = a.c0;
        } else {
            base = a.src1 + (cs * 32 - a.c0);
            pitch = a.c1;
        }
        __syncthreads();   // the previous chunk's reads are done
        for (int i = threadIdx.x; i < NP * 4; i += NT) {
            const int pp = i >> 2, pc = i & 3;
            const int yy = ty0 - 1 + pp / PW, xx = tx0 - 1 + pp % PW;
            s16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
                v = *reinterpret_cast<const s16x8*>(base + (((size_t)b * a.H + yy) * a.W + xx) * pitch + pc * 8);
            *reinterpret_cast<s16x8*>(As + pp * 32 + ((pc + (pp >> 2)) & 3) * 8) = v;
        }
        for (int i = threadIdx.x; i < 9 * NCT * 64; i += NT) {
            const int ln = i & 63, rest = i >> 6;
            const int j = rest % NCT, t = rest / NCT;
            *reinterpret_cast<s16x8*>(Bs + (t * NCT + j) * 512 + ln * 8) =
                *reinterpret_cast<const s16x8*>(a.wp + (((size_t)(ct0 + j) * KT + t * cs32 + cs) * 64 + ln) * 8);
        }
        __syncthreads();
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3, dx = t - 3 * (t / 3);   // staged tile starts one pixel up and left
            s16x8 bv[NCT];
#pragma unroll
            for (int j = 0; j < NCT; ++j) bv[j] = *reinterpret_cast<const s16x8*>(Bs + (t * NCT + j) * 512 + lane * 8);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int pp = (oy[g] + dy) * PW + ox[g] + dx;
                const s16x8 av = *reinterpret_cast<const s16x8*>(As + pp * 32 + ((q + (pp >> 2)) & 3) * 8);
#pragma unroll
                for (int j = 0; j < NCT; ++j)
                    acc[g][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                                         __builtin_bit_cast(bf16x8, bv[j]), acc[g][j],
                                                                         0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = wave * 64 + g * 16 + 4 * (lane >> 4) + r;
            const int ty = p / TW, y = ty0 + ty, x = tx0 + (p - ty * TW);
            if (y >= a.H) continue;
            const size_t op = ((size_t)b * a.H + y) * a.W + x;
#pragma unroll
            for (int j = 0; j < NCT; ++j) {
                const int co = (ct0 + j) * 16 + (lane & 15);
                const float v = acc[g][j][r];
                if (co < a.d0) store_out(a.dst0, op * a.d0 + co, v, a.bf0, a.acc0);
                else store_out(a.dst1, op * a.d1 + (co - a.d0), v, a.bf1, a.acc1);
            }
        }
    }
}

// Packed weights (V = 8 when cip is a multiple of 32, else 4; KS = 4 V):
// entry ((ctile * KT + kt) * 64 + lane) * V + e holds the effective weight
// W_e[co][k] with co = 16 ctile + lane % 16 and k = KS kt + V (lane / 16) + e,
// k = tap * cip + ci; W_e[co][ci][tap] = w[off + co s_co + ci s_ci + tap' s_t]
// (tap' = ntaps - 1 - tap when flipped), zero for co >= co_e or ci >= ci_e.
__global__ __launch_bounds__(NT) void gconv_pack(const float* w, int co_e, int ci_e, int cip, int ntaps, long off,
                                                 long s_co, long s_ci, long s_t, int flip, long total, short* dst)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= total) return;
    const int lv = cip % 32 == 0 ? 3 : 2, V = 1 << lv;        // bf16 per lane: 8 or 4
    const int e = (int)(i & (V - 1)), lane = (int)((i >> lv) & 63);
    const long rest = i >> (lv + 6);
    const int KT = ntaps * cip / (4 * V);
    const int kt = (int)(rest % KT), ctile = (int)(rest / KT);
    const int co = ctile * 16 + (lane & 15);
    const int k = kt * 4 * V + V * (lane >> 4) + e;
    const int tap = k / cip, ci = k - tap * cip;
    float v = 0.f;
    if (co < co_e && ci < ci_e) v = w[off + co * s_co + ci * s_ci + (long)(flip ? ntaps - 1 - tap : tap) * s_t];
    dst[i] = f2bf(v);
}

// Weight-gradient partials of one chunk of rows:
//   part[chunk][co][k] = sum_rows g[out(row)][co] * src[in(row, tap(k))][ci(k)]
// as an MFMA contraction (rows of A = output channels, columns of B = k,
// reduction over the chunk's rows, 32 per 16x16x32 instruction).  A block
// computes a 64 x 64 tile; WG_ROWS rows at a time are staged in LDS with
// 16-byte loads (8 channels per thread and row); wave w owns output channels
// 16 w .. 16 w + 15 of the tile.
struct GWgrad {
    GConv a;
    const short* g;          // NHWC bf16 gradient of the output, pitch cout, on the destination grid
    long rpc;                // rows per chunk (multiple of WG_ROWS)
    float* part;
};

constexpr int WG_ROWS = 128;

__global__ __launch_bounds__(NT) void gwgrad_kernel(GWgrad w)
{
    __shared__ __align__(16) short Gs[WG_ROWS][64];
    __shared__ __align__(16) short Ps[WG_ROWS][64];
    const GConv& a = w.a;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cin = a.c0 + a.c1, K = a.ntaps * cin;
    const int k0 = blockIdx.x * 64, co0 = blockIdx.y * 64;
    const long chunk = blockIdx.z;
    const long R = (long)a.B * a.H * a.W;
    const long r0 = chunk * w.rpc, r1 = min(R, r0 + w.rpc);
    // this thread stages rows sr, sr + 32, ... of each step, columns s8 .. s8 + 7
    const int sr = threadIdx.x >> 3, s8 = (threadIdx.x & 7) * 8;
    const int ks = k0 + s8, co_s = co0 + s8;
    const bool kin = ks < K, cin_ok = co_s < a.cout;
    int tdy = 0, tdx = 0, pitch = 1;
    const short* sbase = a.src0;
    if (kin) {
        const int tap = ks / cin, ci = ks - tap * cin;
        tdy = a.dy[tap];
        tdx = a.dx[tap];
        if (ci < a.c0) {
            sbase = a.src0 + ci;
            pitch = a.c0;
        } else {
            sbase = a.src1 + (ci - a.c0);
            pitch = a.c1;
        }
    }
    f32x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the global loads of step rb + WG_ROWS are issued before the matrix
    // instructions of step rb, so that they overlap
    int4 gv[WG_ROWS / 32], pv[WG_ROWS / 32];
    auto load = [&](long rb) {
#pragma unroll
        for (int h = 0; h < WG_ROWS / 32; ++h) {
            const long row = rb + sr + 32 * h;
            gv[h] = int4{0, 0, 0, 0};
            pv[h] = int4{0, 0, 0, 0};
            if (row < r1) {
                const int x = (int)(row % a.W);
                const long tt = row / a.W;
                const int y = (int)(tt % a.H), b = (int)(tt / a.H);
                if (cin_ok) {
                    const size_t op = ((size_t)b * a.Ho + a.ostr * y + a.oy) * a.Wo + a.ostr * x + a.ox;
                    gv[h] = *reinterpret_cast<const int4*>(w.g + op * a.cout + co_s);
                }
                if (kin) {
                    const int sy = a.istr * y + tdy, sx = a.istr * x + tdx;
                    if (sy >= 0 && sy < a.Hs && sx >= 0 && sx < a.Ws)
                        pv[h] = *reinterpret_cast<const int4*>(sbase + (((size_t)b * a.Hs + sy) * a.Ws + sx) * pitch);
                }
            }
        }
    };
    if (r0 < r1) load(r0);
    for (long rb = r0; rb < r1; rb += WG_ROWS) {
        __syncthreads();
#pragma unroll
        for (int h = 0; h < WG_ROWS / 32; ++h) {
            *reinterpret_cast<int4*>(&Gs[sr + 32 * h][s8]) = gv[h];
            *reinterpret_cast<int4*>(&Ps[sr + 32 * h][s8]) = pv[h];
        }
        __syncthreads();
        if (rb + WG_ROWS < r1) load(rb + WG_ROWS);
#pragma unroll
        for (int h = 0; h < WG_ROWS / 32; ++h) {
            s16x8 av;
#pragma unroll
            for (int e = 0; e < 8; ++e) av[e] = Gs[32 * h + 8 * (lane >> 4) + e][wave * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                s16x8 bv;
#pragma unroll
                for (int e = 0; e < 8; ++e) bv[e] = Ps[32 * h + 8 * (lane >> 4) + e][j * 16 + (lane & 15)];
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                                 __builtin_bit_cast(bf16x8, bv), acc[j], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = co0 + wave * 16 + 4 * (lane >> 4) + r, k = k0 + j * 16 + (lane & 15);
            if (co < a.cout && k < K) w.part[((size_t)chunk * a.cout + co) * K + k] = acc[j][r];
        }
    }
}

// dw[off + co s_co + ci s_ci + tap s_t] (+)= sum over chunks of part[chunk][co][k]
// (FP64, fixed order: chunk_sum16); entries with ci >= ci_real are padding.
// A block reduces 16 consecutive (co, k) entries.
__global__ __launch_bounds__(NT) void gwgrad_reduce(const float* part, int chunks, int cout, int K, int cin,
                                                    int ci_real, float* dw, long off, long s_co, long s_ci, long s_t,
                                                    int accumulate)
{
    __shared__ double red[NT];
    const long total = (long)cout * K;
    const long idx0 = (long)blockIdx.x * 16;
    const double s = chunk_sum16f(part, chunks, total, idx0, total, red);
    const long idx = idx0 + (threadIdx.x & 15);
    if ((threadIdx.x >> 4) != 0 || idx >= total) return;
    const int co = (int)(idx / K), k = (int)(idx - (long)co * K);
    const int tap = k / cin, ci = k - tap * cin;
    if (ci >= ci_real) return;
    float* o = dw + off + co * s_co + ci * s_ci + tap * s_t;
    *o = accumulate ? *o + (float)s : (float)s;
}

// ---- batch normalisation (+ ReLU) ------------------------------------------
// Rows r = 0..R-1 of an NHWC FP32 array with C channels (C divides 256).
// Chunk q covers rows [q rpc, (q + 1) rpc); thread (g, c) sums rows
// r0 + g, r0 + g + G, ... (G = 256 / C); the G group sums are added in order.

__global__ __launch_bounds__(NT) void bn_partial(long R, int C, const float* z, long rpc, double* part)
{
    __shared__ double red[2][NT];
    const int G = NT / C, g = threadIdx.x / C, c = threadIdx.x - g * C;
    const long r0 = (long)blockIdx.x * rpc, r1 = min(R, r0 + rpc);
    // four independent accumulator pairs (rows r0 + g + G (4 i + u)), added
    // in order at the end: loads of four rows are in flight at once
    double s4[4] = {0.0, 0.0, 0.0, 0.0}, ss4[4] = {0.0, 0.0, 0.0, 0.0};
    for (long r = r0 + g; r < r1; r += 4 * G) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long rr = r + u * G;
            const double v = rr < r1 ? (double)z[(size_t)rr * C + c] : 0.0;
            s4[u] += v;
            ss4[u] += v * v;
        }
    }
    red[0][threadIdx.x] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    red[1][threadIdx.x] = (ss4[0] + ss4[1]) + (ss4[2] + ss4[3]);
    __syncthreads();
    if (threadIdx.x < C) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < G; ++q) {
            a += red[0][q * C + threadIdx.x];
            b += red[1][q * C + threadIdx.x];
        }
        part[(size_t)blockIdx.x * 2 * C + threadIdx.x] = a;
        part[(size_t)blockIdx.x * 2 * C + C + threadIdx.x] = b;
    }
}

// block b finishes channels 16 b .. 16 b + 15
__global__ __launch_bounds__(NT) void bn_final(int chunks, int C, long R, const double* part, float* mean,
                                               float* invstd, float* rmean, float* rvar, double momentum, double eps,
                                               int training)
{
    __shared__ double red[NT];
    const int c = blockIdx.x * 16 + (threadIdx.x & 15);
    if (training) {
        const double s = chunk_sum16(part, chunks, 2L * C, blockIdx.x * 16, C, red);
        const double ss = chunk_sum16(part + C, chunks, 2L * C, blockIdx.x * 16, C, red);
        if ((threadIdx.x >> 4) != 0 || c >= C) return;
        const double mu = s / (double)R;
        const double var = fmax(ss / (double)R - mu * mu, 0.0);
        mean[c] = (float)mu;
        invstd[c] = (float)(1.0 / sqrt(var + eps));
        if (rmean) {
            rmean[c] = (float)((1.0 - momentum) * rmean[c] + momentum * mu);
            rvar[c] = (float)((1.0 - momentum) * rvar[c] + momentum * var * (double)R / (double)(R > 1 ? R - 1 : 1));
        }
    } else {
        if ((threadIdx.x >> 4) != 0 || c >= C) return;
        mean[c] = rmean[c];
        invstd[c] = (float)(1.0 / sqrt((double)rvar[c] + eps));
    }
}

__global__ __launch_bounds__(NT) void bn_apply(long total, int C, const float* z, const float* mean,
                                               const float* invstd, const float* gamma, const float* beta, short* out)
{
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < total; i += (long)gridDim.x * NT) {
        const int c = (int)(i % C);
        const float y = gamma[c] * ((z[i] - mean[c]) * invstd[c]) + beta[c];
        out[i] = f2bf(y > 0.f ? y : 0.f);
    }
}

__global__ __launch_bounds__(NT) void bn_bwd_partial(long R, int C, const float* z, const float* ga,
                                                     const float* mean, const float* invstd, const float* gamma,
                                                     const float* beta, long rpc, double* part)
{
    __shared__ double red[2][NT];
    const int G = NT / C, g = threadIdx.x / C, c = threadIdx.x - g * C;
    const long r0 = (long)blockIdx.x * rpc, r1 = min(R, r0 + rpc);
    const float mu = mean[c], is = invstd[c], gm = gamma[c], bt = beta[c];
    double a4[4] = {0.0, 0.0, 0.0, 0.0}, b4[4] = {0.0, 0.0, 0.0, 0.0};
    for (long r = r0 + g; r < r1; r += 4 * G) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long rr = r + u * G;
            if (rr < r1) {
                const size_t i = (size_t)rr * C + c;
                const float xh = (z[i] - mu) * is;
                const float y = gm * xh + bt;
                const float gy = y > 0.f ? ga[i] : 0.f;
                a4[u] += gy;
                b4[u] += (double)gy * xh;
            }
        }
    }
    red[0][threadIdx.x] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    red[1][threadIdx.x] = (b4[0] + b4[1]) + (b4[2] + b4[3]);
    __syncthreads();
    if (threadIdx.x < C) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < G; ++q) {
            a += red[0][q * C + threadIdx.x];
            b += red[1][q * C + threadIdx.x];
        }
        part[(size_t)blockIdx.x * 2 * C + threadIdx.x] = a;
        part[(size_t)blockIdx.x * 2 * C + C + threadIdx.x] = b;
    }
}

// sums[c] = sum gy, sums[C + c] = sum gy xhat (kept for the apply pass);
// dbeta (+)= sum gy, dgamma (+)= sum gy xhat
// block b finishes channels 16 b .. 16 b + 15
__global__ __launch_bounds__(NT) void bn_bwd_final(int chunks, int C, double* part, float* dgamma, float* dbeta,
                                                   int accumulate)
{
    __shared__ double red[NT];
    const int c = blockIdx.x * 16 + (threadIdx.x & 15);
    const double s1 = chunk_sum16(part, chunks, 2L * C, blockIdx.x * 16, C, red);
    const double s2 = chunk_sum16(part + C, chunks, 2L * C, blockIdx.x * 16, C, red);
    if ((threadIdx.x >> 4) != 0 || c >= C) return;
    double* sums = part + (size_t)chunks * 2 * C;
    sums[c] = s1;
    sums[C + c] = s2;
    dbeta[c] = accumulate ? dbeta[c] + (float)s1 : (float)s1;
    dgamma[c] = accumulate ? dgamma[c] + (float)s2 : (float)s2;
}

__global__ __launch_bounds__(NT) void bn_bwd_apply(long total, int C, long R, const float* z, const float* ga,
                                                   const float* mean, const float* invstd, const float* gamma,
                                                   const float* beta, const double* sums, short* gz)
{
    const float inv_r = (float)(1.0 / (double)R);
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < total; i += (long)gridDim.x * NT) {
        const int c = (int)(i % C);
        const float xh = (z[i] - mean[c]) * invstd[c];
        const float y = gamma[c] * xh + beta[c];
        const float gy = y > 0.f ? ga[i] : 0.f;
        const float m1 = (float)sums[c] * inv_r, m2 = (float)sums[C + c] * inv_r;
        gz[i] = f2bf(gamma[c] * invstd[c] * (gy - m1 - xh * m2));
    }
}

// ---- 2x2 max pooling ---------------------------------------------------------
// Window order (0,0), (0,1), (1,0), (1,1); the first maximum wins.

__device__ __forceinline__ int argmax4(const short* in, size_t base, size_t dxs, size_t dys, size_t* at)
{
    size_t pos[4] = {base, base + dxs, base + dys, base + dys + dxs};
    int best = 0;
    float bv = bf2f(in[pos[0]]);
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        const float v = bf2f(in[pos[k]]);
        if (v > bv) {
            bv = v;
            best = k;
        }
    }
    *at = pos[best];
    return best;
}

__global__ __launch_bounds__(NT) void maxpool_fwd(long total, int H, int W, int C, const short* in, short* out)
{
    const int Ho = H / 2, Wo = W / 2;
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < total; i += (long)gridDim.x * NT) {
        const int c = (int)(i % C);
        const long p = i / C;
        const int xo = (int)(p % Wo);
        const long t = p / Wo;
        const int yo = (int)(t % Ho), b = (int)(t / Ho);
        const size_t base = (((size_t)b * H + 2 * yo) * W + 2 * xo) * C + c;
        size_t at;
        argmax4(in, base, (size_t)C, (size_t)W * C, &at);
        out[i] = in[at];
    }
}

__global__ __launch_bounds__(NT) void maxpool_bwd(long total, int H, int W, int C, const short* in, const float* gout,
                                                  float* gin)
{
    const int Ho = H / 2, Wo = W / 2;
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < total; i += (long)gridDim.x * NT) {
        const int c = (int)(i % C);
        const long p = i / C;
        const int xo = (int)(p % Wo);
        const long t = p / Wo;
        const int yo = (int)(t % Ho), b = (int)(t / Ho);
        const size_t base = (((size_t)b * H + 2 * yo) * W + 2 * xo) * C + c;
        size_t at;
        argmax4(in, base, (size_t)C, (size_t)W * C, &at);
        gin[at] += gout[i];
    }
}

// ---- planar inputs <-> NHWC, and the 1x1 output head -------------------------

struct Planes {
    const float* in[4];
    float scale[4];
    float* g[4];
    const float* res[4];
};

__global__ __launch_bounds__(NT) void nhwc_pack(long total, int cin, int cp, Planes pl, short* out)
{
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < total; i += (long)gridDim.x * NT) {
        const int c = (int)(i % cp);
        const long p = i / cp;
        float v = 0.f;
        if (c < cin) v = pl.in[c][p] * pl.scale[c];
        out[i] = f2bf(v);
    }
}

__global__ __launch_bounds__(NT) void nhwc_unpack_grad(long R, int cin, int cp, const float* g, Planes pl)
{
    for (long p = (long)blockIdx.x * NT + threadIdx.x; p < R; p += (long)gridDim.x * NT) {
        for (int c = 0; c < cin; ++c) {
            if (!pl.g[c]) continue;
            const float r = pl.res[c] ? pl.res[c][p] : 0.f;
            pl.g[c][p] = r + pl.scale[c] * g[(size_t)p * cp + c];
        }
    }
}

// out[p] = res[p] + b + sum_c w[c] act[p][c]
__global__ __launch_bounds__(NT) void head_fwd(long R, int C, const short* act, const float* w, const float* b,
                                               const float* res, float* out)
{
    for (long p = (long)blockIdx.x * NT + threadIdx.x; p < R; p += (long)gridDim.x * NT) {
        float s = b ? b[0] : 0.f;
        const short* ap = act + (size_t)p * C;
        for (int c = 0; c < C; ++c) s += w[c] * bf2f(ap[c]);
        out[p] = (res ? res[p] : 0.f) + s;
    }
}

// gact[p][c] = w[c] g[p]
__global__ __launch_bounds__(NT) void head_bwd_input(long total, int C, const float* w, const float* g, float* gact)
{
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < total; i += (long)gridDim.x * NT) {
        const int c = (int)(i % C);
        gact[i] = w[c] * g[i / C];
    }
}

// part[chunk][c] = sum_p g[p] act[p][c] (c < C), part[chunk][C] = sum_p g[p]
__global__ __launch_bounds__(NT) void head_bwd_partial(long R, int C, const short* act, const float* g, long rpc,
                                                       double* part)
{
    __shared__ double red[2][NT];
    const int G = NT / C, q = threadIdx.x / C, c = threadIdx.x - q * C;
    const long r0 = (long)blockIdx.x * rpc, r1 = min(R, r0 + rpc);
    double s4[4] = {0.0, 0.0, 0.0, 0.0}, g4[4] = {0.0, 0.0, 0.0, 0.0};
    for (long p = r0 + q; p < r1; p += 4 * G) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long pp = p + u * G;
            if (pp < r1) {
                const double gp = g[pp];
                s4[u] += gp * bf2f(act[(size_t)pp * C + c]);
                g4[u] += gp;
            }
        }
    }
    red[0][threadIdx.x] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    red[1][threadIdx.x] = (g4[0] + g4[1]) + (g4[2] + g4[3]);
    __syncthreads();
    if (threadIdx.x < C) {
        double a = 0.0;
        for (int k = 0; k < G; ++k) a += red[0][k * C + threadIdx.x];
        part[(size_t)blockIdx.x * (C + 1) + threadIdx.x] = a;
    }
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int k = 0; k < G; ++k) a += red[1][k * C];   // column c = 0 of every group carries sum g
        part[(size_t)blockIdx.x * (C + 1) + C] = a;
    }
}

// out[c] (+)= sum over chunks of part[chunk][c], c < ncols (FP64, fixed order:
// chunk_sum16); a block reduces 16 columns
__global__ __launch_bounds__(NT) void col_reduce(const double* part, int chunks, int ncols, float* out, int accumulate)
{
    __shared__ double red[NT];
    const double s = chunk_sum16(part, chunks, ncols, blockIdx.x * 16L, ncols, red);
    const int c = blockIdx.x * 16 + (threadIdx.x & 15);
    if ((threadIdx.x >> 4) != 0 || c >= ncols) return;
    out[c] = accumulate ? out[c] + (float)s : (float)s;
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

int fail(const char* who, const char* why, int code = PAT_EINVAL)
{
    pat::set_error(std::string(who) + ": " + why);
    return code;
}

int grid_of(long total) { return (int)std::min<long>(std::max<long>((total + NT - 1) / NT, 1), 8192); }

// chunk count for the row-partitioned reductions over R rows of C channels:
// about 16 K elements per chunk (at least 8 rows), at most 4096 chunks, so
// that narrow and wide layers alike put enough blocks in flight
int bn_chunks(long R, int C)
{
    const long rows = std::max<long>(8, 16384 / std::max(C, 1));
    return (int)std::max<long>(1, std::min<long>(4096, R / rows));
}

int check_gconv(const pat_gconv_desc* d, const char* who)
{
    if (!d) return fail(who, "null descriptor");
    if (d->B < 1 || d->H < 1 || d->W < 1 || d->Hs < 1 || d->Ws < 1 || d->Ho < 1 || d->Wo < 1)
        return fail(who, "bad grid sizes");
    if (d->ntaps < 1 || d->ntaps > 9) return fail(who, "ntaps must be 1..9");
    if (!d->src[0] || d->csrc[0] < 16 || d->csrc[0] % 16 || d->csrc[1] < 0 || d->csrc[1] % 16 ||
        (d->csrc[1] > 0 && !d->src[1]))
        return fail(who, "source channel counts must be multiples of 16 (src[1] optional)", PAT_EUNSUPPORTED);
    if (d->cout < 16 || d->cout % 16) return fail(who, "cout must be a positive multiple of 16", PAT_EUNSUPPORTED);
    if (d->in_stride < 1 || d->out_stride < 1 || d->oy < 0 || d->ox < 0) return fail(who, "bad strides or offsets");
    if ((long)d->out_stride * (d->H - 1) + d->oy >= d->Ho || (long)d->out_stride * (d->W - 1) + d->ox >= d->Wo)
        return fail(who, "destination mapping leaves the destination grid");
    if (!d->weight) return fail(who, "missing weights");
    return PAT_OK;
}

GConv make_gconv(const pat_gconv_desc* d)
{
    GConv a;
    a.B = d->B; a.H = d->H; a.W = d->W;
    a.src0 = static_cast<const short*>(d->src[0]);
    a.src1 = static_cast<const short*>(d->src[1]);
    a.c0 = d->csrc[0]; a.c1 = d->csrc[1];
    a.Hs = d->Hs; a.Ws = d->Ws; a.istr = d->in_stride; a.ntaps = d->ntaps;
    for (int t = 0; t < 9; ++t) {
        a.dy[t] = t < d->ntaps ? d->dy[t] : 0;
        a.dx[t] = t < d->ntaps ? d->dx[t] : 0;
    }
    a.wp = static_cast<const short*>(d->weight);
    a.cout = d->cout;
    a.dst0 = d->dst[0]; a.dst1 = d->dst[1];
    a.d0 = d->cdst[0]; a.d1 = d->cdst[1];
    a.bf0 = d->dst_bf16[0]; a.bf1 = d->dst_bf16[1];
    a.acc0 = d->accumulate[0]; a.acc1 = d->accumulate[1];
    a.Ho = d->Ho; a.Wo = d->Wo; a.ostr = d->out_stride; a.oy = d->oy; a.ox = d->ox;
    return a;
}

Planes make_planes(int cin, const void* const* in, const float* scales, void* const* g, const void* const* res)
{
    Planes pl;
    for (int c = 0; c < 4; ++c) {
        pl.in[c] = (in && c < cin) ? static_cast<const float*>(in[c]) : nullptr;
        pl.scale[c] = (scales && c < cin) ? scales[c] : 1.f;
        pl.g[c] = (g && c < cin) ? static_cast<float*>(g[c]) : nullptr;
        pl.res[c] = (res && c < cin) ? static_cast<const float*>(res[c]) : nullptr;
    }
    return pl;
}

}  // namespace

extern "C" {

long pat_gconv_packed_size(int cout, int cip, int ntaps)
{
    if (cout < 16 || cout % 16 || cip < 16 || cip % 16 || ntaps < 1 || ntaps > 9) return -1;
    return (long)cout * ntaps * cip;
}

int pat_gconv_pack(const void* w, int co_e, int ci_e, int cout, int cip, int ntaps, long off, long s_co, long s_ci,
                   long s_t, int flip, void* dst, void* stream)
{
    const long total = pat_gconv_packed_size(cout, cip, ntaps);
    if (!w || !dst || total < 0 || co_e < 1 || co_e > cout || ci_e < 1 || ci_e > cip || off < 0)
        return fail("pat_gconv_pack", "bad arguments");
    gconv_pack<<<(int)((total + NT - 1) / NT), NT, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        static_cast<const float*>(w), co_e, ci_e, cip, ntaps, off, s_co, s_ci, s_t, flip, total,
        static_cast<short*>(dst));
    return status("gconv_pack");
}

int pat_gconv(const pat_gconv_desc* d, void* stream)
{
    int rc = check_gconv(d, "pat_gconv");
    if (rc) return rc;
    if (d->cdst[0] < 0 || d->cdst[1] < 0 || d->cdst[0] + d->cdst[1] != d->cout || (d->cdst[0] > 0 && !d->dst[0]) ||
        (d->cdst[1] > 0 && !d->dst[1]))
        return fail("pat_gconv", "destination channel split must cover cout");
    if ((d->dst_bf16[0] && d->accumulate[0]) || (d->dst_bf16[1] && d->accumulate[1]))
        return fail("pat_gconv", "bf16 destinations cannot accumulate", PAT_EUNSUPPORTED);
    const bool x32 = d->csrc[0] % 32 == 0 && d->csrc[1] % 32 == 0;
    if (!x32 && (d->csrc[0] + d->csrc[1]) % 32 == 0)
        return fail("pat_gconv", "when the channel total is a multiple of 32 every source must be one",
                    PAT_EUNSUPPORTED);
    GConv a = make_gconv(d);
    const int ctw = d->cout % 64 == 0 ? 4 : (d->cout % 32 == 0 ? 2 : 1);
    const long rows = (long)d->B * d->H * d->W;
    const long waves = (rows + 63) / 64 * (d->cout / (16 * ctw));
    const long blocks = (waves + 3) / 4;
    if (blocks > 0x7fffffffL) return fail("pat_gconv", "grid too large", PAT_EUNSUPPORTED);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    bool plain3 = x32 && d->ntaps == 9 && d->in_stride == 1 && d->out_stride == 1 && d->oy == 0 && d->ox == 0 &&
                  d->Hs == d->H && d->Ws == d->W && d->Ho == d->H && d->Wo == d->W && d->W % 16 == 0 &&
                  d->cout % 32 == 0;
    for (int t = 0; plain3 && t < 9; ++t) plain3 = d->dy[t] == t / 3 - 1 && d->dx[t] == t % 3 - 1;
    if (plain3) {
        const int TW = d->W % 64 == 0 ? 64 : (d->W % 32 == 0 ? 32 : 16), TH = 256 / TW;
        const long tiles = (long)d->B * ((d->H + TH - 1) / TH) * (d->W / TW);
        if (tiles > 0x7fffffffL) return fail("pat_gconv", "grid too large", PAT_EUNSUPPORTED);
        if (d->cout % 64 == 0) gconv3_lds<4><<<dim3((unsigned)tiles, d->cout / 64), NT, 0, st>>>(a, TW);
        else gconv3_lds<2><<<dim3((unsigned)tiles, d->cout / 32), NT, 0, st>>>(a, TW);
        return status("gconv3_lds");
    }
    if (x32) {
        if (ctw == 4) gconv32_kernel<4><<<(unsigned)blocks, NT, 0, st>>>(a);
        else if (ctw == 2) gconv32_kernel<2><<<(unsigned)blocks, NT, 0, st>>>(a);
        else gconv32_kernel<1><<<(unsigned)blocks, NT, 0, st>>>(a);
    } else {
        if (ctw == 4) gconv_kernel<4><<<(unsigned)blocks, NT, 0, st>>>(a);
        else if (ctw == 2) gconv_kernel<2><<<(unsigned)blocks, NT, 0, st>>>(a);
        else gconv_kernel<1><<<(unsigned)blocks, NT, 0, st>>>(a);
    }
    return status("gconv_kernel");
}

long pat_gconv_wgrad_partials(const pat_gconv_desc* d, int chunks)
{
    if (!d || chunks < 1 || d->ntaps < 1 || d->cout < 1) return -1;
    return (long)chunks * d->cout * d->ntaps * (d->csrc[0] + d->csrc[1]);
}

int pat_gconv_wgrad(const pat_gconv_desc* d, const void* grad, int chunks, void* partials, void* dw, int ci_real,
                    long off, long s_co, long s_ci, long s_t, int accumulate, void* stream)
{
    int rc = check_gconv(d, "pat_gconv_wgrad");
    if (rc) return rc;
    const int cin = d->csrc[0] + d->csrc[1];
    if (!grad || !partials || !dw || chunks < 1 || chunks > 65535 || ci_real < 1 || ci_real > cin || off < 0)
        return fail("pat_gconv_wgrad", "bad arguments");
    GWgrad w;
    w.a = make_gconv(d);
    w.g = static_cast<const short*>(grad);
    const long rows = (long)d->B * d->H * d->W;
    w.rpc = ((rows + chunks - 1) / chunks + WG_ROWS - 1) / WG_ROWS * WG_ROWS;
    w.part = static_cast<float*>(partials);
    const int K = d->ntaps * cin;
    const int used = (int)((rows + w.rpc - 1) / w.rpc);   // chunks that hold rows
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    dim3 grid((K + 63) / 64, (d->cout + 63) / 64, used);
    gwgrad_kernel<<<grid, NT, 0, st>>>(w);
    if ((rc = status("gwgrad_kernel"))) return rc;
    const long total = (long)d->cout * K;
    gwgrad_reduce<<<(int)((total + 15) / 16), NT, 0, st>>>(w.part, used, d->cout, K, cin, ci_real,
                                                               static_cast<float*>(dw), off, s_co, s_ci, s_t,
                                                               accumulate);
    return status("gwgrad_reduce");
}

long pat_bn_partials(long rows, int channels)
{
    if (rows < 1 || channels < 1 || channels > 256 || 256 % channels) return -1;
    return ((long)bn_chunks(rows, channels) + 1) * 2 * channels;
}

int pat_bn_forward(long rows, int channels, const void* z, const void* gamma, const void* beta, void* mean,
                   void* invstd, void* running_mean, void* running_var, double momentum, double eps, int training,
                   void* out, void* partials, void* stream)
{
    if (pat_bn_partials(rows, channels) < 0) return fail("pat_bn_forward", "channels must divide 256", PAT_EUNSUPPORTED);
    if (!z || !gamma || !beta || !mean || !invstd || !out || !(eps > 0) || !(momentum >= 0 && momentum <= 1) ||
        (training && !partials) || (!training && (!running_mean || !running_var)) ||
        ((running_mean == nullptr) != (running_var == nullptr)))
        return fail("pat_bn_forward", "bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int chunks = bn_chunks(rows, channels);
    const long rpc = (rows + chunks - 1) / chunks;
    if (training) {
        bn_partial<<<chunks, NT, 0, st>>>(rows, channels, static_cast<const float*>(z), rpc,
                                          static_cast<double*>(partials));
        int rc = status("bn_partial");
        if (rc) return rc;
    }
    bn_final<<<(channels + 15) / 16, NT, 0, st>>>(chunks, channels, rows, static_cast<const double*>(partials), static_cast<float*>(mean),
                               static_cast<float*>(invstd), static_cast<float*>(running_mean),
                               static_cast<float*>(running_var), momentum, eps, training);
    int rc = status("bn_final");
    if (rc) return rc;
    const long total = rows * channels;
    bn_apply<<<grid_of(total), NT, 0, st>>>(total, channels, static_cast<const float*>(z),
                                            static_cast<const float*>(mean), static_cast<const float*>(invstd),
                                            static_cast<const float*>(gamma), static_cast<const float*>(beta),
                                            static_cast<short*>(out));
    return status("bn_apply");
}

int pat_bn_backward(long rows, int channels, const void* z, const void* grad_act, const void* gamma, const void* beta,
                    const void* mean, const void* invstd, void* grad_z, void* dgamma, void* dbeta, int accumulate,
                    void* partials, void* stream)
{
    if (pat_bn_partials(rows, channels) < 0) return fail("pat_bn_backward", "channels must divide 256", PAT_EUNSUPPORTED);
    if (!z || !grad_act || !gamma || !beta || !mean || !invstd || !grad_z || !dgamma || !dbeta || !partials)
        return fail("pat_bn_backward", "bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int chunks = bn_chunks(rows, channels);
    const long rpc = (rows + chunks - 1) / chunks;
    const float* zf = static_cast<const float*>(z);
    const float* gf = static_cast<const float*>(grad_act);
    const float* mf = static_cast<const float*>(mean);
    const float* sf = static_cast<const float*>(invstd);
    const float* gm = static_cast<const float*>(gamma);
    const float* bt = static_cast<const float*>(beta);
    double* part = static_cast<double*>(partials);
    bn_bwd_partial<<<chunks, NT, 0, st>>>(rows, channels, zf, gf, mf, sf, gm, bt, rpc, part);
    int rc = status("bn_bwd_partial");
    if (rc) return rc;
    bn_bwd_final<<<(channels + 15) / 16, NT, 0, st>>>(chunks, channels, part, static_cast<float*>(dgamma), static_cast<float*>(dbeta),
                                   accumulate);
    if ((rc = status("bn_bwd_final"))) return rc;
    const long total = rows * channels;
    bn_bwd_apply<<<grid_of(total), NT, 0, st>>>(total, channels, rows, zf, gf, mf, sf, gm, bt,
                                                part + (size_t)chunks * 2 * channels, static_cast<short*>(grad_z));
    return status("bn_bwd_apply");
}

int pat_maxpool2(int B, int H, int W, int C, const void* in, void* out, void* stream)
{
    if (!in || !out || B < 1 || H < 2 || W < 2 || H % 2 || W % 2 || C < 1) return fail("pat_maxpool2", "bad arguments");
    const long total = (long)B * (H / 2) * (W / 2) * C;
    maxpool_fwd<<<grid_of(total), NT, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        total, H, W, C, static_cast<const short*>(in), static_cast<short*>(out));
    return status("maxpool_fwd");
}

int pat_maxpool2_backward(int B, int H, int W, int C, const void* in, const void* grad_out, void* grad_in, void* stream)
{
    if (!in || !grad_out || !grad_in || B < 1 || H < 2 || W < 2 || H % 2 || W % 2 || C < 1)
        return fail("pat_maxpool2_backward", "bad arguments");
    const long total = (long)B * (H / 2) * (W / 2) * C;
    maxpool_bwd<<<grid_of(total), NT, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        total, H, W, C, static_cast<const short*>(in), static_cast<const float*>(grad_out),
        static_cast<float*>(grad_in));
    return status("maxpool_bwd");
}

int pat_nhwc_pack(long pixels, int cin, int cpad, const void* const* planes, const float* scales, void* out,
                  void* stream)
{
    if (!planes || !out || pixels < 1 || cin < 1 || cin > 4 || cpad < cin) return fail("pat_nhwc_pack", "bad arguments");
    for (int c = 0; c < cin; ++c)
        if (!planes[c]) return fail("pat_nhwc_pack", "missing input plane");
    Planes pl = make_planes(cin, planes, scales, nullptr, nullptr);
    const long total = pixels * cpad;
    nhwc_pack<<<grid_of(total), NT, 0, reinterpret_cast<hipStream_t>(stream)>>>(total, cin, cpad, pl,
                                                                               static_cast<short*>(out));
    return status("nhwc_pack");
}

int pat_nhwc_unpack_grad(long pixels, int cin, int cpad, const void* grad, const float* scales, void* const* grad_planes,
                         const void* const* residual, void* stream)
{
    if (!grad || !grad_planes || pixels < 1 || cin < 1 || cin > 4 || cpad < cin)
        return fail("pat_nhwc_unpack_grad", "bad arguments");
    Planes pl = make_planes(cin, nullptr, scales, grad_planes, residual);
    nhwc_unpack_grad<<<grid_of(pixels), NT, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        pixels, cin, cpad, static_cast<const float*>(grad), pl);
    return status("nhwc_unpack_grad");
}

int pat_head_forward(long pixels, int C, const void* act, const void* w, const void* b, const void* residual,
                     void* out, void* stream)
{
    if (!act || !w || !out || pixels < 1 || C < 1) return fail("pat_head_forward", "bad arguments");
    head_fwd<<<grid_of(pixels), NT, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        pixels, C, static_cast<const short*>(act), static_cast<const float*>(w), static_cast<const float*>(b),
        static_cast<const float*>(residual), static_cast<float*>(out));
    return status("head_fwd");
}

long pat_head_partials(long pixels, int C)
{
    if (pixels < 1 || C < 1 || C > 256 || 256 % C) return -1;
    return (long)bn_chunks(pixels, C) * (C + 1);
}

int pat_head_backward(long pixels, int C, const void* act, const void* w, const void* grad_out, void* grad_act,
                      void* grad_wb, int accumulate, void* partials, void* stream)
{
    if (pat_head_partials(pixels, C) < 0) return fail("pat_head_backward", "C must divide 256", PAT_EUNSUPPORTED);
    if (!act || !w || !grad_out || !grad_act || !grad_wb || !partials) return fail("pat_head_backward", "bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const long total = pixels * C;
    head_bwd_input<<<grid_of(total), NT, 0, st>>>(total, C, static_cast<const float*>(w),
                                                  static_cast<const float*>(grad_out), static_cast<float*>(grad_act));
    int rc = status("head_bwd_input");
    if (rc) return rc;
    const int chunks = bn_chunks(pixels, C);
    const long rpc = (pixels + chunks - 1) / chunks;
    head_bwd_partial<<<chunks, NT, 0, st>>>(pixels, C, static_cast<const short*>(act),
                                            static_cast<const float*>(grad_out), rpc, static_cast<double*>(partials));
    if ((rc = status("head_bwd_partial"))) return rc;
    col_reduce<<<(C + 1 + 15) / 16, NT, 0, st>>>(static_cast<const double*>(partials), chunks, C + 1,
                                                     static_cast<float*>(grad_wb), accumulate);
    return status("col_reduce");
}

}  // extern "C"
