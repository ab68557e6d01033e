// HIP kernels (gfx950) and C-ABI entry points for the fast circular-geometry
// photoacoustic operators of Hauptmann, Kunyansky & Poimala (arXiv 2510.24687).
//
// Forward chain (Algorithm 1, Sec. 3.1), one launch per stage, batched over
// images in gridDim.y:
//   rows_fwd   pre-correct, zero-extend and FFT two image rows at a time (real
//              rows packed into one complex FFT) -> half spectrum per row
//   cols_fwd   FFT along y for a block of spectrum columns -> extended half grid
//              (extra columns beyond both ends hold the conjugate-symmetric values)
//   ring_fwd   per ring: gather the half ring from the grid with the w x w
//              kernel (step 3), fill the other half by conjugate symmetry, ring
//              FFT (step 4, eq. E:eq3), Bessel/taper/quadrature weights -> V(l,k)
//   dct        per harmonic: cosine sum over rings (step 5, eq. E:inverse_cos_tr)
//              as a 2M-point FFT -> G_k(t_j)
//   lowk_fwd   exact low-frequency quadrature for harmonics 0..klow
//   synth_fwd  per pair of time rows: fold harmonics onto the m_full detector
//              grid and inverse FFT (steps 6-7, eq. E:FourSerForg), keep the arc
// The adjoint runs the exact transposes in reverse order; the transpose of the
// gather is a deterministic per-tile spread (no global atomics).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <memory>
#include <new>
#include <queue>
#include <string>
#include <vector>

#include "pat_internal.h"

namespace pat {
const char* last_error();
}

namespace {

constexpr int NT = 256;  // threads per block for every kernel
constexpr int FFT_REGS = 16;                 // complex values per thread and pass in lds_fft
constexpr int FFT_BLOCK_POINTS = FFT_REGS * NT;  // nb * N limit of one lds_fft call

template <typename T>
struct cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.x, -a.y}; }
// multiply by i^k
template <typename T>
__device__ __forceinline__ cx<T> mul_ipow(cx<T> a, int k)
{
    switch (k & 3) {
        case 0: return a;
        case 1: return {-a.y, a.x};
        case 2: return {-a.x, -a.y};
        default: return {a.y, -a.x};
    }
}

__device__ __forceinline__ void sincos_t(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_t(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ float sqrt_t(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
__device__ __forceinline__ float ceil_t(float x) { return ceilf(x); }
__device__ __forceinline__ double ceil_t(double x) { return ceil(x); }

// ---------------------------------------------------------------------------
// FFT of `nb` independent sequences of length N = 2^logN held in LDS at
// buf + b*stride: Stockham autosort (natural order in and out, no bit
// reversal) with radix-16/8/4/2 butterflies computed in registers, so an
// N = 4096 transform takes three LDS round trips.  A pass with radix R and
// sub-transform length Ns reads x[t + r N/R], multiplies by W_{Ns R}^{r k}
// (k = t mod Ns), does a length-R DFT and writes to (t/Ns) Ns R + k + r Ns.
// tw holds e^{-2 pi i k/Nmax}; `inv` selects e^{+...} (no 1/N).  Requires
// blockDim.x == NT and nb*N <= FFT_BLOCK_POINTS (each thread keeps at most
// FFT_REGS complex values of one pass in registers).  Ends synchronised.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void dft4(cx<T>& a, cx<T>& b, cx<T>& c, cx<T>& e, bool inv)
{
    cx<T> s0 = a + c, d0 = a - c, s1 = b + e, d1 = b - e;
    cx<T> jd1 = inv ? cx<T>{-d1.y, d1.x} : cx<T>{d1.y, -d1.x};  // -i d1 (forward) / +i d1 (inverse)
    a = s0 + s1;
    c = s0 - s1;
    b = d0 + jd1;
    e = d0 - jd1;
}

template <typename T, int R>
__device__ __forceinline__ void dft_reg(cx<T>* v, bool inv);

template <>
__device__ __forceinline__ void dft_reg<float, 2>(cx<float>* v, bool) { cx<float> t = v[0]; v[0] = t + v[1]; v[1] = t - v[1]; }
template <>
__device__ __forceinline__ void dft_reg<double, 2>(cx<double>* v, bool) { cx<double> t = v[0]; v[0] = t + v[1]; v[1] = t - v[1]; }

template <typename T>
__device__ __forceinline__ void dft4_arr(cx<T>* v, bool inv) { dft4(v[0], v[1], v[2], v[3], inv); }
template <>
__device__ __forceinline__ void dft_reg<float, 4>(cx<float>* v, bool inv) { dft4_arr(v, inv); }
template <>
__device__ __forceinline__ void dft_reg<double, 4>(cx<double>* v, bool inv) { dft4_arr(v, inv); }

// e^{-2 pi i m/16}, m = 0..15
__constant__ const double W16C[16] = {1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977, 0.0,
                                      -0.38268343236508977, -0.70710678118654752, -0.92387953251128674, -1.0,
                                      -0.92387953251128674, -0.70710678118654752, -0.38268343236508977, 0.0,
                                      0.38268343236508977, 0.70710678118654752, 0.92387953251128674};

template <typename T>
__device__ __forceinline__ cx<T> w16(int m, bool inv)
{
    // cos(2 pi m/16), -sin(2 pi m/16) (forward)
    const T c = (T)W16C[m & 15];
    const T s = (T)W16C[(m + 12) & 15];  // cos(2 pi (m-4)/16) = sin(2 pi m/16)
    return inv ? cx<T>{c, s} : cx<T>{c, -s};
}

// size N1*N2 DFT from N2 DFTs of size N1 (stride N2), twiddles W_N^{n2 k1}, N1 DFTs of size N2
template <typename T, int R>
__device__ __forceinline__ void dft_split(cx<T>* v, bool inv)
{
    constexpr int N1 = 4, N2 = R / 4;
    cx<T> a[N2][N1];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) a[n2][n1] = v[N2 * n1 + n2];
        dft4(a[n2][0], a[n2][1], a[n2][2], a[n2][3], inv);
#pragma unroll
        for (int k1 = 1; k1 < N1; ++k1)
            if (n2 > 0) a[n2][k1] = cmul(a[n2][k1], w16<T>((16 / R) * n2 * k1, inv));
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
        if (N2 == 2) {
            cx<T> t = a[0][k1];
            v[k1] = t + a[1][k1];
            v[k1 + 4] = t - a[1][k1];
        } else {
            cx<T> b0 = a[0][k1], b1 = a[1][k1], b2 = a[2][k1], b3 = a[3][k1];
            dft4(b0, b1, b2, b3, inv);
            v[k1] = b0;
            v[k1 + 4] = b1;
            v[k1 + 8] = b2;
            v[k1 + 12] = b3;
        }
    }
}
template <>
__device__ __forceinline__ void dft_reg<float, 8>(cx<float>* v, bool inv) { dft_split<float, 8>(v, inv); }
template <>
__device__ __forceinline__ void dft_reg<double, 8>(cx<double>* v, bool inv) { dft_split<double, 8>(v, inv); }
template <>
__device__ __forceinline__ void dft_reg<float, 16>(cx<float>* v, bool inv) { dft_split<float, 16>(v, inv); }
template <>
__device__ __forceinline__ void dft_reg<double, 16>(cx<double>* v, bool inv) { dft_split<double, 16>(v, inv); }

// The transform buffer is passed as an LDS (address space 3) pointer and the
// twiddle table as a global (address space 1) pointer: the pass is not
// inlined, and with generic pointers every access would become a FLAT
// instruction with 64-bit address arithmetic.
#define PAT_LDS __attribute__((address_space(3)))
#define PAT_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ cx<T> ld_lds(const PAT_LDS cx<T>* p) { return {p->x, p->y}; }
template <typename T>
__device__ __forceinline__ void st_lds(PAT_LDS cx<T>* p, cx<T> v) { p->x = v.x; p->y = v.y; }
template <typename T>
__device__ __forceinline__ cx<T> ld_glb(const PAT_GLOBAL cx<T>* p) { return {p->x, p->y}; }

// LDS index of element i of an FFT buffer: with PAD one slot of padding
// after every 8 entries, so that the strided stores of the first radix-8
// passes (stride 8 and 64 entries) fall in distinct banks.  Sequence starts
// and strides are multiples of 8, so phys(a + i) = phys(a) + phys(i).
template <bool PAD>
__host__ __device__ constexpr int lds_phys(int i) { return PAD ? i + (i >> 3) : i; }

// A power-of-two pass of a transform of length N = f 2^logN, f = 1 or 3 (f3):
// the sequences' stride between butterfly inputs is N/R.
template <typename T, int R, bool PAD = false>
__device__ __noinline__ void stockham_pass(PAT_LDS cx<T>* buf, int logN, int logNs, int nb, int stride,
                                              const PAT_GLOBAL cx<T>* __restrict__ tw, int logNmax, bool inv, bool twtab,
                                              int f3)
{
    constexpr int LR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
    constexpr int BPT = FFT_REGS / R;
    const int lnbf = logN - LR;
    const int nbf = f3 ? 3 << lnbf : 1 << lnbf;
    const int total = nb * nbf;
    const int sh = logNmax - logNs - LR;
    // without the full table: the entries W^1, W^2, W^4, W^8 of the thread's
    // butterflies, loaded before the LDS reads (their latency overlaps those
    // and the barrier)
    cx<T> wp[BPT][LR];
    if (logNs > 0 && !twtab) {
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int it = threadIdx.x + u * NT;
            if (it < total) {
                const int b = f3 ? (it >> lnbf) / 3 : it >> lnbf, t = it - b * nbf;
                const int k = t & ((1 << logNs) - 1);
#pragma unroll
                for (int e = 0; e < LR; ++e) wp[u][e] = ld_glb(tw + ((k << e) << sh));
            }
        }
    }
    cx<T> v[BPT][R];
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int it = threadIdx.x + u * NT;
        if (it < total) {
            const int b = f3 ? (it >> lnbf) / 3 : it >> lnbf, t = it - b * nbf;
            const PAT_LDS cx<T>* s = buf + lds_phys<PAD>(b * stride);
#pragma unroll
            for (int r = 0; r < R; ++r) v[u][r] = ld_lds(s + lds_phys<PAD>(t + r * nbf));
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int it = threadIdx.x + u * NT;
        if (it < total) {
            const int b = f3 ? (it >> lnbf) / 3 : it >> lnbf, t = it - b * nbf;
            const int k = t & ((1 << logNs) - 1);
            if (logNs > 0) {
                if (twtab) {
                    // W^r read from the table for every r
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        cx<T> w = ld_glb(tw + ((r * k) << sh));
                        if (inv) w.y = -w.y;
                        v[u][r] = cmul(v[u][r], w);
                    }
                } else {
                    // W^r for r = 1..R-1 from the table entries W^1, W^2, W^4, W^8 (at
                    // most three products each): fewer table reads, more arithmetic
#pragma unroll
                    for (int e = 0; e < LR; ++e)
                        if (inv) wp[u][e].y = -wp[u][e].y;
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        cx<T> w = {T(1), T(0)};
                        bool first = true;
#pragma unroll
                        for (int e = 0; e < LR; ++e) {
                            if (r & (1 << e)) {
                                w = first ? wp[u][e] : cmul(w, wp[u][e]);
                                first = false;
                            }
                        }
                        v[u][r] = cmul(v[u][r], w);
                    }
                }
            }
            dft_reg<T, R>(v[u], inv);
            PAT_LDS cx<T>* s = buf + lds_phys<PAD>(b * stride);
            const int base = ((t >> logNs) << (logNs + LR)) + k;
#pragma unroll
            for (int r = 0; r < R; ++r) st_lds(s + lds_phys<PAD>(base + (r << logNs)), v[u][r]);
        }
    }
    __syncthreads();
}

template <typename T, bool PAD = false>
__device__ void lds_fft(cx<T>* buf, int logN, int nb, int stride, const cx<T>* __restrict__ tw, int logNmax,
                        bool inverse, int maxlr, bool twtab, int f3 = 0)
{
    if (logN == 0) return;
    const int P = (logN + maxlr - 1) / maxlr;  // passes; radices as equal as possible, at most 2^maxlr
    PAT_LDS cx<T>* lbuf = (PAT_LDS cx<T>*)buf;
    const PAT_GLOBAL cx<T>* gtw = (const PAT_GLOBAL cx<T>*)tw;
    int logNs = 0;
    for (int p = 0; p < P; ++p) {
        const int lr = logN / P + (p < logN % P ? 1 : 0);
        switch (lr) {
            case 1: stockham_pass<T, 2, PAD>(lbuf, logN, logNs, nb, stride, gtw, logNmax, inverse, twtab, f3); break;
            case 2: stockham_pass<T, 4, PAD>(lbuf, logN, logNs, nb, stride, gtw, logNmax, inverse, twtab, f3); break;
            case 3: stockham_pass<T, 8, PAD>(lbuf, logN, logNs, nb, stride, gtw, logNmax, inverse, twtab, f3); break;
            default: stockham_pass<T, 16, PAD>(lbuf, logN, logNs, nb, stride, gtw, logNmax, inverse, twtab, f3); break;
        }
        logNs += lr;
    }
}

// The last pass of a length N = 3 * 2^logN2 transform (after the power-of-two
// passes): radix 3 with sub-transform length Ns = 2^logN2, twiddles W_N^{r t}
// read from twd (the 2N-th roots e^{-2 pi i j/(2N)}: W_N^{r t} = twd[2 r t]).
template <typename T, bool PAD = false>
__device__ __noinline__ void stockham_pass3(PAT_LDS cx<T>* buf, int logN2, int nb, int stride,
                                               const PAT_GLOBAL cx<T>* __restrict__ twd, bool inv, int tsh)
{
    constexpr int BPT = FFT_REGS / 3;
    const int nbf = 1 << logN2;
    const int total = nb << logN2;
    const T h3 = T(0.86602540378443864676);  // sqrt(3)/2
    // twiddles first (their latency overlaps the LDS reads and the barrier)
    cx<T> w1s[BPT], w2s[BPT];
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int it = threadIdx.x + u * NT;
        if (it < total) {
            const int t = it & (nbf - 1);
            w1s[u] = ld_glb(twd + ((2 * t) << tsh));
            w2s[u] = ld_glb(twd + ((4 * t) << tsh));
        }
    }
    cx<T> v[BPT][3];
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int it = threadIdx.x + u * NT;
        if (it < total) {
            const int b = it >> logN2, t = it & (nbf - 1);
            const PAT_LDS cx<T>* s = buf + lds_phys<PAD>(b * stride);
#pragma unroll
            for (int r = 0; r < 3; ++r) v[u][r] = ld_lds(s + lds_phys<PAD>(t + r * nbf));
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int it = threadIdx.x + u * NT;
        if (it < total) {
            const int b = it >> logN2, t = it & (nbf - 1);
            cx<T> w1 = w1s[u], w2 = w2s[u];
            if (inv) { w1.y = -w1.y; w2.y = -w2.y; }
            const cx<T> a0 = v[u][0], a1 = cmul(v[u][1], w1), a2 = cmul(v[u][2], w2);
            const cx<T> sm = a1 + a2, df = a1 - a2;
            const cx<T> m = {a0.x - T(0.5) * sm.x, a0.y - T(0.5) * sm.y};
            // forward: y1 = m - i h3 df, y2 = m + i h3 df (inverse: signs swapped)
            const cx<T> jd = inv ? cx<T>{-h3 * df.y, h3 * df.x} : cx<T>{h3 * df.y, -h3 * df.x};
            PAT_LDS cx<T>* s = buf + lds_phys<PAD>(b * stride);
            st_lds(s + lds_phys<PAD>(t), a0 + sm);
            st_lds(s + lds_phys<PAD>(t + nbf), m + jd);
            st_lds(s + lds_phys<PAD>(t + 2 * nbf), m - jd);
        }
    }
    __syncthreads();
}

// Transform of nb sequences of length N = 3 * 2^logN2: the power-of-two passes
// on the 2^logN2 factor, then the radix-3 pass.  The radix-3 pass keeps
// FFT_REGS / 3 butterflies per thread, so nb * N <= (FFT_REGS / 3) * 3 * NT.
// twd holds the 2N'-th roots of unity of a length N' = N 2^tsh.
template <typename T, bool PAD = false>
__device__ void lds_fft3(cx<T>* buf, int logN2, int nb, int stride, const cx<T>* __restrict__ tw, int logNmax,
                         const cx<T>* __restrict__ twd, bool inverse, int maxlr, bool twtab, int tsh = 0)
{
    lds_fft<T, PAD>(buf, logN2, nb, stride, tw, logNmax, inverse, maxlr, twtab, 1);
    stockham_pass3<T, PAD>((PAT_LDS cx<T>*)buf, logN2, nb, stride, (const PAT_GLOBAL cx<T>*)twd, inverse, tsh);
}

// MI355X dispatches consecutive workgroups of a grid round-robin over its 8
// XCDs, each with its own L2.  Kernels whose neighbouring work items share
// cache lines (adjacent columns, adjacent rings, neighbouring tiles) renumber
// their workgroups so that each XCD receives one contiguous range of the
// logical (x, y) grid: logical = xcd * (count on earlier XCDs) + arrival index.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ void xcd_remap(int lin, int nx, int total, int& bx, int& by)
{
    const int xcd = lin % NUM_XCD, local = lin / NUM_XCD;
    const int per = total / NUM_XCD, rem = total % NUM_XCD;
    const int logical = (xcd < rem) ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
    bx = logical % nx;
    by = logical / nx;
}
// Block lin of a table-driven launch over nz image groups: entry
// (lin / (NUM_XCD nz)) NUM_XCD + lin mod NUM_XCD of the table (so that the
// entry's XCD is the block's), image group (lin / NUM_XCD) mod nz.
__host__ __device__ inline void table_block(int lin, int nz, int& entry, int& z)
{
    entry = (lin / (NUM_XCD * nz)) * NUM_XCD + lin % NUM_XCD;
    z = (lin / NUM_XCD) % nz;
}

__device__ __forceinline__ void xcd_block(int& bx, int& by)
{
    xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x, gridDim.x * gridDim.y, bx, by);
}

// Block coordinates of a kernel body: (x, y, z) of the stage's logical grid
// and its x extent.  The single-plan kernels take them from the hardware
// grid; the grouped kernels (several plans in one launch) derive them from
// the block's rank inside its plan's range.
struct Blk {
    int x, y, z, nx;
};
__device__ __forceinline__ Blk blk_xcd()
{
    int bx, by;
    xcd_block(bx, by);
    return {bx, by, (int)blockIdx.z, (int)gridDim.x};
}
__device__ __forceinline__ Blk blk_plain() { return {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, (int)gridDim.x}; }

// The update step of an iterative reconstruction (Sec. 4.2) fused into the
// last launch of an operator chain: synth_fwd's trace stores for A, rows_adj's
// image stores for A*.  Element indices run over a contiguous batch (traces
// nt * m apart, images n * n apart); the arithmetic is that of the separate
// update kernels (pat_axpby, pat_cp_dual_data, pat_nnls_update, pat_cp_primal).
enum { EPI_NONE = 0, EPI_RESIDUAL, EPI_CP_DUAL, EPI_NNLS, EPI_CP_PRIMAL };
template <typename T>
struct Epi {
    int kind;
    const T* g;           // RESIDUAL, CP_DUAL: the data
    T sigma, inv1ps;      // CP_DUAL: q <- (q + sigma (A fbar - g)) / (1 + sigma), inv1ps = 1 / (1 + sigma)
    T* f;                 // NNLS, CP_PRIMAL: the iterate, updated in place
    T* fbar;              // CP_PRIMAL: the relaxed iterate
    const T* p;           // CP_PRIMAL: the TV dual, two n x n planes per image
    const T* support;     // NNLS, CP_PRIMAL: optional mask multiplied into f
    T tau, theta, inv_h;
};

// Plan data as seen by the kernels.
template <typename T>
struct Dev {
    int n, m, nt, mf, logmf;
    int Ng, logNg, w, hw, Rw, Ew;
    int Ep;                     // row pitch of E in cells: Ew rounded up to 16 (128-byte rows of tiles)
    int M, log2M, L, K, Kp, klow, lcorr, npts;
    int logNmax;
    int colsCW, dctCW;
    int colsLCW, dctLCW;        // log2 of the two (powers of two)
    int dct_stash;              // 1: the cosine transform stashes its input columns in LDS
    int dct_one;                // 1: the cosine transform uses one M-point FFT per column (dct_cos_body)
    int dct_wave;               // FP32 cosine transform with one wave per column group: variant
                                // (M3 << 8) | log2 of M's power-of-two factor; 0: not used
    int dwCB;                   // columns per block of dct_wave
    int wfRows;                 // log2 Ng when the FP32 row and column FFT passes run one wave per
                                // sequence (rows_fwd_w, cols_fwd_w, ...), else 0
    int wfSynth;                // log2 m_full for the wave form of the angular synthesis, else 0
    int fft_lr;                 // largest FFT pass radix is 2^fft_lr (3 or 4)
    int tw_table;               // 1: FFT passes read every twiddle from the table
    T beta, shift, half;        // half = Ng / (2 Lambda): grid cells per unit lambda
    T beta_l2e;                 // beta * log2(e)
    T lamh;                     // h: u = lambda h cos(phi)
    T dlam, pre_scale, adj_scale;
    double mask_r2, a, h;       // mask test in double (same decision as the oracle)
    const T* Dq;                // n
    const T* lam;               // L
    const int* ringN;           // L
    const int* ringLog;         // L
    const int* ringOff;         // L
    const int* ringK;           // L
    const int* ringM3;          // L: 1 when ring l has 3 * 2^ringLog[l] points
    const cx<T>* twr;           // 2 Nr3: e^{-2 pi i j/(2 Nr3)} (ring radix-3 twiddles)
    int logNr3;                 // log2(Nr3 / 3)
    const T* Tb;                // L x Kp
    const T* Mk;                // (klow+1) x nt x lcorr (forward: each t_j's row contiguous)
    const T* MkT;               // (klow+1) x lcorr x nt, the same values (adjoint: t_j fastest)
    const cx<T>* phase;         // Kp
    const cx<T>* tw;            // Nmax
    const cx<T>* twd;           // 2M: e^{-2 pi i j/(2M)} (cosine-transform twiddles)
    int m3;                     // 1: M = 3 * 2^log2M
    int mf3;                    // 1: mf = 3 * 2^logmf
    const cx<T>* twm;           // 2 mf: e^{-2 pi i j/(2 mf)} (angular-transform twiddles)
    const cx<T>* pos;           // npts: grid position (x, y) of each half-ring sample
    const cx<T>* ph;            // npts: its point phase e^{-i shift h (x + y) / half}, evaluated in
                                // FP64 (the adjoint's table; the gathers evaluate point_phase)
    T phase_k;                  // -shift * h / half: point phase per grid cell of x + y
    // bin order of the FP32 spread (spread_bins): samples sorted by the cell of
    // their first tap, (gy0 mod Ng) * Ew + gx0 + hw, ring order within a bin
    const int* binRing;         // npts: ring-order index of the sample in each bin-order slot
    const int* ringBin;         // npts: bin-order slot of each ring-order sample
    const int* binStart;        // Ng * Ew + 1: first slot of each bin
    const int* spOrder;         // spCount: spread_bins dispatch table (spread_order)
    int spCount;
    const int* gbOrder;         // gbCount: gather_bins dispatch table (gather_order)
    int gbCount;
    const cx<T>* binPos;        // npts: positions in bin order
    int binned;                 // 1: the adjoint spreads with spread_bins
    // approximate inverse (Sec. 3.3): its tables, and the per-call switches of
    // the adjoint kernels that it reuses
    const T* Tbi;               // L x Kp: Tb with J_k' for J_k
    const T* MkiT;              // (klow+1) x lcorr x nt: MkT with J_k' and sin
    double R2;                  // R^2: the detector disk Omega
    int sine;                   // 1: the transform over t is the sine transform
    int ubp;                    // 1: rows_adj writes v everywhere plus the partial sums of v over
                                //    Omega \ Omega_0 (part, one double per block and image)
    double* part;
    Epi<T> epi;                 // fused update step (kind EPI_NONE outside the fused entry points)
};

// Trace element out[o] (o: its offset from the output's base, contiguous batch) of A applied to the iterate.
template <typename T>
__device__ __forceinline__ void put_trace(const Dev<T>& d, T* out, size_t o, T v)
{
    const Epi<T>& e = d.epi;
    if (e.kind == EPI_RESIDUAL) {
        out[o] = v - e.g[o];
    } else if (e.kind == EPI_CP_DUAL) {
        out[o] = (out[o] + e.sigma * (v - e.g[o])) * e.inv1ps;  // out is the dual variable q
    } else {
        out[o] = v;
    }
}

// Image element (image b, row r, column c) of A* applied to the traces; out:
// the image output of a plain adjoint call.
template <typename T>
__device__ __forceinline__ void put_image(const Dev<T>& d, T* out, int b, int r, int c, T a)
{
    const Epi<T>& e = d.epi;
    const int n = d.n;
    const long per = (long)n * n;
    const long k = (long)r * n + c, i = (long)b * per + k;
    if (e.kind == EPI_NNLS) {
        T v = e.f[i] - e.tau * a;
        v = v > T(0) ? v : T(0);
        e.f[i] = e.support ? v * e.support[i] : v;
    } else if (e.kind == EPI_CP_PRIMAL) {
        const T* px = e.p + (long)b * 2 * per;
        const T* py = px + per;
        T dx = (c < n - 1 ? px[k] : T(0)) - (c > 0 ? px[k - 1] : T(0));
        T dy = (r < n - 1 ? py[k] : T(0)) - (r > 0 ? py[k - n] : T(0));
        const T div = (dx + dy) * e.inv_h;
        const T f_old = e.f[i];
        T v = f_old - e.tau * (a - div);
        v = v > T(0) ? v : T(0);
        if (e.support) v *= e.support[i];
        e.f[i] = v;
        e.fbar[i] = v + e.theta * (v - f_old);
    } else {
        out[k] = a;
    }
}

template <typename T>
__device__ __forceinline__ bool in_mask(const Dev<T>& d, int p, int q)
{
    if (d.mask_r2 <= 0.0) return true;
    double x = -d.a + (q + 0.5) * d.h, y = -d.a + (p + 0.5) * d.h;
    return x * x + y * y <= d.mask_r2;
}

// Pixel centre in Omega \ Omega_0: inside the detector disk and outside the
// mask disk (no mask: Omega_0 is the whole image and the set is empty).
template <typename T>
__device__ __forceinline__ bool in_annulus(const Dev<T>& d, int p, int q)
{
    if (d.mask_r2 <= 0.0) return false;
    double x = -d.a + (q + 0.5) * d.h, y = -d.a + (p + 0.5) * d.h;
    double r2 = x * x + y * y;
    return r2 <= d.R2 && !(r2 <= d.mask_r2);
}

// exponential-of-semicircle kernel at offset `dd` cells:
// exp(beta (sqrt(1 - z^2) - 1)), z = 2 dd / w, zero for |z| >= 1.  The FP32
// form uses the hardware square root and base-2 exponential (about 1e-7
// relative error, far below the FP32 operator's error); the gather and the
// spread evaluate the same function, so A* stays the transpose of A.
__device__ __forceinline__ double es_w(double dd, double two_over_w, double beta, double)
{
    double z = dd * two_over_w;
    double s = 1.0 - z * z;
    return s > 0.0 ? exp(beta * (sqrt(s) - 1.0)) : 0.0;
}
__device__ __forceinline__ float es_w(float dd, float two_over_w, float, float beta_log2e)
{
    const float z = dd * two_over_w;
    const float s = 1.f - z * z;
    return s > 0.f ? __builtin_amdgcn_exp2f(beta_log2e * (__builtin_amdgcn_sqrtf(s) - 1.f)) : 0.f;
}

// Grid position, first taps and weights of half-ring sample si of ring l
// (WMAX is the stencil width w: 6 for FP32 plans, 13 for FP64 plans).
template <typename T, int WMAX>
struct Taps {
    int gx0, gy0;
    T wx[WMAX], wy[WMAX];
    cx<T> ph;  // e^{-i shift (u + v)}
};

// Grid position (cells) of half-ring sample si of a ring with N samples at
// radius lam: x = lam * Ng/(2 Lambda) * cos(2 pi s/N), s = si - N/4.  The
// gather and the spread both call this, so they select identical taps.
template <typename T>
__device__ __forceinline__ void point_xy(const Dev<T>& d, int p, T& x, T& y)
{
    const cx<T> q = d.pos[p];
    x = q.x;
    y = q.y;
}

// e^{-i shift (u + v)} of a sample at grid position (x, y): u + v = h lam (cos + sin) = h (x + y)/half
template <typename T>
__device__ __forceinline__ cx<T> point_phase(const Dev<T>& d, T x, T y)
{
    T ps, pc;
    sincos_t(d.phase_k * (x + y), &ps, &pc);
    return {pc, ps};
}

template <typename T, int WMAX>
__device__ __forceinline__ void point_taps(const Dev<T>& d, int p, Taps<T, WMAX>& tp)
{
    T x, y;
    point_xy(d, p, x, y);
    T hwf = T(0.5) * T(WMAX);
    tp.gx0 = (int)ceil_t(x - hwf);
    tp.gy0 = (int)ceil_t(y - hwf);
    T tw_ = T(2) / T(WMAX);
#pragma unroll
    for (int j = 0; j < WMAX; ++j) {
        tp.wx[j] = es_w(x - T(tp.gx0 + j), tw_, d.beta, d.beta_l2e);
        tp.wy[j] = es_w(y - T(tp.gy0 + j), tw_, d.beta, d.beta_l2e);
    }
    tp.ph = point_phase(d, x, y);
}

// ---------------------------------------------------------------------------
// forward kernels
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void rows_fwd_body(const Dev<T>& d, Blk bk, const T* __restrict__ f, long fstride, cx<T>* R,
                                               size_t ws_img)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    int bx_, b;
    bx_ = bk.x;
    b = bk.y;
    const int p1 = 2 * bx_, p2 = p1 + 1;
    const T* fb = f + (size_t)b * fstride;
    cx<T>* Rb = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(R) + (size_t)b * ws_img);
    const int Ng = d.Ng, n = d.n;
    for (int i = threadIdx.x; i < Ng; i += blockDim.x) buf[i] = {T(0), T(0)};
    __syncthreads();
    const T s1 = p1 < n ? d.Dq[p1] * d.pre_scale : T(0);
    const T s2 = p2 < n ? d.Dq[p2] * d.pre_scale : T(0);
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        int qi = (q - n / 2 + Ng) & (Ng - 1);
        T a = (p1 < n && in_mask(d, p1, q)) ? fb[(size_t)p1 * n + q] * d.Dq[q] * s1 : T(0);
        T c = (p2 < n && in_mask(d, p2, q)) ? fb[(size_t)p2 * n + q] * d.Dq[q] * s2 : T(0);
        buf[qi] = {a, c};
    }
    __syncthreads();
    lds_fft(buf, d.logNg, 1, 0, d.tw, d.logNmax, false, d.fft_lr, d.tw_table);
    for (int g = threadIdx.x; g <= Ng / 2; g += blockDim.x) {
        cx<T> zg = buf[g], zm = buf[(Ng - g) & (Ng - 1)];
        cx<T> x1 = {T(0.5) * (zg.x + zm.x), T(0.5) * (zg.y - zm.y)};
        cx<T> x2 = {T(0.5) * (zg.y + zm.y), T(0.5) * (zm.x - zg.x)};
        if (p1 < n) Rb[(size_t)p1 * d.Rw + g] = x1;
        if (p2 < n) Rb[(size_t)p2 * d.Rw + g] = x2;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void rows_fwd(Dev<T> d, const T* __restrict__ f, long fstride, cx<T>* R,
                                               size_t ws_img)
{
    rows_fwd_body<T>(d, blk_xcd(), f, fstride, R, ws_img);
}

template <typename T>
__device__ __forceinline__ void cols_fwd_body(const Dev<T>& d, Blk bk, const cx<T>* R, cx<T>* E, size_t ws_img)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    int bx_, b;
    bx_ = bk.x;
    b = bk.y;
    const int CW = d.colsCW, lcw = d.colsLCW, x0 = bx_ * CW;
    const int Ng = d.Ng, n = d.n;
    const cx<T>* Rb = reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(R) + (size_t)b * ws_img);
    cx<T>* Eb = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(E) + (size_t)b * ws_img);
    for (int i = threadIdx.x; i < CW * Ng; i += blockDim.x) buf[i] = {T(0), T(0)};
    __syncthreads();
    for (int i = threadIdx.x; i < CW * n; i += blockDim.x) {
        int p = i >> lcw, c = i & (CW - 1);
        int gx = x0 + c;
        if (gx < d.Rw) buf[c * Ng + ((p - n / 2 + Ng) & (Ng - 1))] = Rb[(size_t)p * d.Rw + gx];
    }
    __syncthreads();
    lds_fft(buf, d.logNg, CW, Ng, d.tw, d.logNmax, false, d.fft_lr, d.tw_table);
    for (int i = threadIdx.x; i < CW * Ng; i += blockDim.x) {
        int gy = i >> lcw, c = i & (CW - 1);
        int gx = x0 + c;
        if (gx >= d.Rw) continue;
        cx<T> v = buf[c * Ng + gy];
        Eb[(size_t)gy * d.Ep + gx + d.hw] = v;
        int gym = (Ng - gy) & (Ng - 1);
        if (gx >= 1 && gx <= d.hw) Eb[(size_t)gym * d.Ep + d.hw - gx] = conjg(v);
        if (gx >= Ng / 2 - d.hw && gx <= Ng / 2 - 1) Eb[(size_t)gym * d.Ep + d.hw + Ng - gx] = conjg(v);
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void cols_fwd(Dev<T> d, const cx<T>* R, cx<T>* E, size_t ws_img)
{
    cols_fwd_body<T>(d, blk_xcd(), R, E, ws_img);
}

// The ring transforms of nb images (ring l: N = 2^logN or 3 * 2^logN points),
// as many sequences per lds_fft call as its register budget allows.
// FP32 ring buffers are padded (lds_phys<true>): LDS of ring_lds bytes.
template <typename T>
constexpr bool RING_PAD = sizeof(T) == 4;

template <typename T>
__device__ __forceinline__ void ring_fft(const Dev<T>& d, int l, cx<T>* buf, int N, int logN, int nb, bool inverse)
{
    constexpr bool PAD = RING_PAD<T>;
    if (d.ringM3[l]) {
        const int per_call = max(1, min(nb, ((FFT_REGS / 3) * 3 * NT) / N));
        for (int i = 0; i < nb; i += per_call)
            lds_fft3<T, PAD>(buf + lds_phys<PAD>(i * N), logN, min(per_call, nb - i), N, d.tw, d.logNmax, d.twr,
                             inverse, d.fft_lr, d.tw_table, d.logNr3 - logN);
    } else {
        const int per_call = max(1, min(nb, FFT_BLOCK_POINTS >> logN));
        for (int i = 0; i < nb; i += per_call)
            lds_fft<T, PAD>(buf + lds_phys<PAD>(i * N), logN, min(per_call, nb - i), N, d.tw, d.logNmax, inverse,
                            d.fft_lr, d.tw_table);
    }
}

// loads per thread that the ring kernels' data loops issue together
constexpr int RING_CH = 4;

// One block per (ring, group of up to G images): the taps, weights and phase
// of each half-ring sample are computed once and applied to every image of
// the group (the transcendental work does not depend on the image).
template <typename T, int WMAX>
__device__ __forceinline__ void ring_fwd_body(const Dev<T>& d, Blk bk, const cx<T>* E, const cx<T>* Pin, cx<T>* V,
                                               cx<T>* Ulow, size_t ws_img, int B, int G)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    int l, grp;
    l = bk.x;
    grp = bk.y;
    const int b0 = grp * G, nb = min(G, B - b0);
    const int N = d.ringN[l], logN = d.ringLog[l], Kl = d.ringK[l];
    const int mask = d.Ng - 1;
    if (Pin) {
        // samples gathered by gather_bins, phase applied, grouped as this
        // kernel reads them: image group grp holds npts x nb values, sample-major
        const cx<T>* src = Pin + (size_t)b0 * d.npts + (size_t)d.ringOff[l] * nb;
        // value t = si nb + i, in chunks of RING_CH loads per thread issued
        // together (si, i by shifts when nb is a power of two)
        const int nv = (N / 2) * nb;
        const int lnb = (nb & (nb - 1)) == 0 ? __ffs(nb) - 1 : -1;
        for (int t0 = 0; t0 < nv; t0 += RING_CH * NT) {
            cx<T> v[RING_CH];
#pragma unroll
            for (int u = 0; u < RING_CH; ++u) {
                const int t = t0 + u * NT + threadIdx.x;
                if (t < nv) v[u] = src[t];
            }
#pragma unroll
            for (int u = 0; u < RING_CH; ++u) {
                const int t = t0 + u * NT + threadIdx.x;
                if (t < nv) {
                    const int si = lnb >= 0 ? t >> lnb : t / nb, i = t - si * nb, s = si - N / 4, bo = i * N;
                    buf[lds_phys<RING_PAD<T>>(bo + (s < 0 ? s + N : s))] = v[u];
                    buf[lds_phys<RING_PAD<T>>(bo + (s + N / 2))] = conjg(v[u]);
                }
            }
        }
    } else
#pragma unroll 2
    for (int si = threadIdx.x; si < N / 2; si += blockDim.x) {
        Taps<T, WMAX> tp;
        point_taps<T, WMAX>(d, d.ringOff[l] + si, tp);
        const int s = si - N / 4;
        for (int i = 0; i < nb; ++i) {
            const cx<T>* Eb = reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(E) + (size_t)(b0 + i) * ws_img);
            cx<T> acc = {T(0), T(0)};
#pragma unroll
            for (int jy = 0; jy < WMAX; ++jy) {
                const cx<T>* row = Eb + (size_t)((tp.gy0 + jy) & mask) * d.Ep + tp.gx0 + d.hw;
                cx<T> racc = {T(0), T(0)};
#pragma unroll
                for (int jx = 0; jx < WMAX; ++jx) racc = racc + row[jx] * tp.wx[jx];
                acc = acc + racc * tp.wy[jy];
            }
            const cx<T> v = cmul(acc, tp.ph);
            const int bo = i * N;
            buf[lds_phys<RING_PAD<T>>(bo + (s < 0 ? s + N : s))] = v;          // s in [-N/4, N/4)
            buf[lds_phys<RING_PAD<T>>(bo + (s + N / 2))] = conjg(v);
        }
    }
    __syncthreads();
    ring_fft(d, l, buf, N, logN, nb, false);
    const T invN = T(1) / T(N);
    // chunks of RING_CH harmonics per thread: their table values are loaded
    // together, before any store of the chunk
    for (int k0 = 0; k0 < d.Kp; k0 += RING_CH * NT) {
        T tb[RING_CH];
#pragma unroll
        for (int u = 0; u < RING_CH; ++u) {
            const int k = k0 + u * NT + threadIdx.x;
            tb[u] = (k <= Kl && k < d.Kp) ? d.Tb[(size_t)l * d.Kp + k] : T(0);
        }
        for (int i = 0; i < nb; ++i) {
            const int bo = i * N;
            cx<T>* Vb = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(V) + (size_t)(b0 + i) * ws_img);
            cx<T>* Ub = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(Ulow) + (size_t)(b0 + i) * ws_img);
#pragma unroll
            for (int u = 0; u < RING_CH; ++u) {
                const int k = k0 + u * NT + threadIdx.x;
                if (k >= d.Kp) continue;
                cx<T> out = {T(0), T(0)};
                if (k <= Kl) out = mul_ipow(buf[lds_phys<RING_PAD<T>>(bo + (k))] * tb[u], k);
                Vb[(size_t)l * d.Kp + k] = out;
                if (l < d.lcorr && k <= d.klow) Ub[(size_t)l * (d.klow + 1) + k] = (k <= Kl ? buf[lds_phys<RING_PAD<T>>(bo + (k))] : cx<T>{T(0), T(0)}) * invN;
            }
        }
    }
}

template <typename T, int WMAX>
__global__ __launch_bounds__(NT) void ring_fwd(Dev<T> d, const cx<T>* E, const cx<T>* Pin, cx<T>* V, cx<T>* Ulow,
                                               size_t ws_img, int B, int G)
{
    ring_fwd_body<T, WMAX>(d, blk_xcd(), E, Pin, V, Ulow, ws_img, B, G);
}

// ---------------------------------------------------------------------------
// FP32 gather over samples sorted by bin (the order of spread_bins): a block
// owns the 16 x 16 bins of a tile and BC images, stages the 21 x 21 cells
// their stencils reach (rows mod Ng; each cell's BC values as one padded row)
// in LDS with coalesced 16-byte loads, and each thread then interpolates
// whole samples from LDS: the taps, weights and phase of point_taps and the
// summation order of ring_fwd (row sums over x, then over y), so the values
// equal those of ring_fwd's own gather.  Output in the image groups of
// ring_fwd (G images per block): image b of group c = b / G (nc images) goes
// to Pout[c G npts + p nc + b - c G], p the sample's ring-order index, so
// that ring_fwd reads contiguous runs.
// ---------------------------------------------------------------------------
constexpr int GB_TILE = 16;
constexpr int GB_BC = 8;  // images per block (35 KB of LDS: 4 blocks per CU)
__host__ __device__ constexpr int gather_bins_row(int bc) { return bc + 2; }   // cx per staged cell
__host__ __device__ constexpr size_t gather_bins_lds(int bc)
{
    return 256 + 8 * (size_t)(GB_TILE + 5) * (GB_TILE + 5) * (size_t)gather_bins_row(bc);
}

template <int BC>
__device__ __forceinline__ void gather_bins_body(const Dev<float>& d, Blk bk, const cx<float>* E, cx<float>* Pout, int B,
                                                 int G, size_t ws_img)
{
    constexpr int W = 6, TS = GB_TILE, NC = TS + W - 1, CR = gather_bins_row(BC), TPS = BC / 2;
    static_assert(TS <= 32 && CR % 2 == 0, "tile and LDS layout");
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    int* s_vo = reinterpret_cast<int*>(smem_raw);           // TS + 1 run offsets
    int* s_gs = s_vo + 32;                                   // TS first slots
    float4* s_cell = reinterpret_cast<float4*>(smem_raw + 256);  // NC x NC cells of CR / 2 float4
    const int tid = threadIdx.x;
    const int ex0 = bk.x * TS, ty0 = bk.y * TS;
    const int Ng = d.Ng, mask = Ng - 1, Ew = d.Ew;
    const int b0 = bk.z * BC, nb = min(BC, B - b0);
    const int e_end = min(ex0 + TS, Ew);
    if (tid < TS) {
        const int row = (ty0 + tid) & mask;
        const int a = d.binStart[(size_t)row * Ew + ex0], b = d.binStart[(size_t)row * Ew + e_end];
        s_gs[tid] = a;
        s_vo[tid + 1] = b - a;
    }
    // stage the cells: (row, column, image pair) tasks, coalesced along the
    // row; every load is issued before the first is stored
    constexpr int ITG = (NC * NC * TPS + NT - 1) / NT;
    float4 xs[ITG];
#pragma unroll
    for (int it = 0; it < ITG; ++it) {
        const int t = tid + it * NT;
        const int m = t % TPS, c = t / TPS;
        const int lx = c % NC, ly = c / NC;
        const int ex = ex0 + lx, gy = (ty0 + ly) & mask;
        xs[it] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (t < NC * NC * TPS && ex < Ew) {
            const int k = 2 * m;
            if (k < nb) {
                const cx<float> v = reinterpret_cast<const cx<float>*>(reinterpret_cast<const char*>(E) +
                                                                     (size_t)(b0 + k) * ws_img)[(size_t)gy * d.Ep + ex];
                xs[it].x = v.x; xs[it].y = v.y;
            }
            if (k + 1 < nb) {
                const cx<float> v = reinterpret_cast<const cx<float>*>(reinterpret_cast<const char*>(E) +
                                                                     (size_t)(b0 + k + 1) * ws_img)[(size_t)gy * d.Ep + ex];
                xs[it].z = v.x; xs[it].w = v.y;
            }
        }
    }
#pragma unroll
    for (int it = 0; it < ITG; ++it) {
        const int t = tid + it * NT;
        if (t < NC * NC * TPS) s_cell[(t / TPS) * (CR / 2) + t % TPS] = xs[it];
    }
    __syncthreads();
    if (tid == 0) {
        s_vo[0] = 0;
        for (int q = 0; q < TS; ++q) s_vo[q + 1] += s_vo[q];
    }
    __syncthreads();
    const int S = s_vo[TS];
    const float hwf = 0.5f * float(W), tw_ = 2.f / float(W);
    // slot of sample v (v increases along a thread's loop, so the bin row q only advances)
    int q = 0;
    auto slot = [&](int v) {
        while (q + 1 < TS && s_vo[q + 1] <= v) ++q;
        return s_gs[q] + v - s_vo[q];
    };
    // software pipeline: the next sample's position and ring index are loaded
    // while this one is interpolated
    cx<float> pq_next = {0.f, 0.f};
    int pr_next = 0;
    if (tid < S) {
        const int g = slot(tid);
        pq_next = d.binPos[g];
        pr_next = d.binRing[g];
    }
    for (int v = tid; v < S; v += NT) {
        const cx<float> pq = pq_next;
        const size_t pr = (size_t)pr_next;
        if (v + NT < S) {
            const int g = slot(v + NT);
            pq_next = d.binPos[g];
            pr_next = d.binRing[g];
        }
        const int gx0 = (int)ceil_t(pq.x - hwf);
        const int gy0 = (int)ceil_t(pq.y - hwf);
        float wx[W];
#pragma unroll
        for (int j = 0; j < W; ++j) wx[j] = es_w(pq.x - float(gx0 + j), tw_, d.beta, d.beta_l2e);
        const cx<float> ph = point_phase(d, pq.x, pq.y);
        const int lx0 = gx0 + d.hw - ex0, ly0 = (gy0 - ty0) & mask;  // both in [0, TS)
        const float4* base = s_cell + (ly0 * NC + lx0) * (CR / 2);
        // one stencil row at a time (its y-weight evaluated once there), all
        // BC images of the row's taps in registers
        float4 acc[TPS];
#pragma unroll
        for (int m = 0; m < TPS; ++m) acc[m] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 1
        for (int jy = 0; jy < W; ++jy) {
            const float wyj = es_w(pq.y - float(gy0 + jy), tw_, d.beta, d.beta_l2e);
            const float4* rowp = base + jy * NC * (CR / 2);
#pragma unroll
            for (int m = 0; m < TPS; ++m) {
                float4 racc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int jx = 0; jx < W; ++jx) {
                    const float4 c = rowp[jx * (CR / 2) + m];
                    racc.x += c.x * wx[jx];
                    racc.y += c.y * wx[jx];
                    racc.z += c.z * wx[jx];
                    racc.w += c.w * wx[jx];
                }
                acc[m].x += racc.x * wyj;
                acc[m].y += racc.y * wyj;
                acc[m].z += racc.z * wyj;
                acc[m].w += racc.w * wyj;
            }
        }
#pragma unroll
        for (int m = 0; m < TPS; ++m) {
            const cx<float> v0 = cmul(cx<float>{acc[m].x, acc[m].y}, ph);
            const cx<float> v1 = cmul(cx<float>{acc[m].z, acc[m].w}, ph);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int k = 2 * m + u, bi = b0 + k;
                if (k < nb) {
                    const int c = bi / G, nc = min(G, B - c * G);
                    Pout[(size_t)c * G * d.npts + pr * nc + (bi - c * G)] = u ? v1 : v0;
                }
            }
        }
    }
}

// Block lin does the tile of table entry and image group table_block(lin)
// (gbOrder: tx | ty << 12, per XCD a contiguous run of tiles taken longest
// first by a cost estimate, see gather_order and xcd_table; -1: nothing).
template <int BC>
__global__ __launch_bounds__(NT, 4) void gather_bins(Dev<float> d, const cx<float>* E, cx<float>* Pout, int B, int G,
                                                     size_t ws_img, int nz)
{
    int entry, z;
    table_block(blockIdx.x, nz, entry, z);
    const int t = d.gbOrder[entry];
    if (t < 0) return;  // padding of a shorter XCD list
    gather_bins_body<BC>(d, Blk{t & 0xfff, t >> 12, z, 0}, E, Pout, B, G, ws_img);
}

// Sum over aligned groups of W consecutive lanes (W a power of two <= 64),
// butterfly order: every lane of a group returns the group's sum.
template <typename T>
__device__ __forceinline__ cx<T> group_sum(cx<T> v, int W)
{
    for (int o = 1; o < W; o <<= 1) {
        v.x += __shfl_xor(v.x, o, W);
        v.y += __shfl_xor(v.y, o, W);
    }
    return v;
}

// Inclusive prefix sum over aligned groups of W consecutive lanes.
template <typename T>
__device__ __forceinline__ cx<T> group_scan(cx<T> v, int W)
{
    const int lane = threadIdx.x & (W - 1);
    for (int o = 1; o < W; o <<= 1) {
        const T ux = __shfl_up(v.x, o, W), uy = __shfl_up(v.y, o, W);
        if (lane >= o) { v.x += ux; v.y += uy; }
    }
    return v;
}

// The cosine sum with ONE M-point FFT per column (the DCT-I of each column's
// real and imaginary parts at once).  With f_j = in(j), j = 0..M (zero outside
// the valid rows) and s_j = sin(pi j/M), the sequence
//   g_j = (f_j + f_{M-j})/2 - s_j (f_j - f_{M-j}),  j = 0..M-1  (f_{M-0} = f_M)
// has the transform G_q = sum_j g_j e^{2 pi i j q/M}, and the interior sums
// F_y = (f_0 + (-1)^y f_M)/2 + sum_{0<x<M} f_x cos(pi x y/M) satisfy
//   F_{2q} = (G_q + G_{M-q})/2,   F_{2q+1} = F_{2q-1} - (i/2)(G_q - G_{M-q}),
// F_1 = (f_0 - f_M)/2 + sum_{0<x<M} f_x cos(pi x/M) (a direct sum); the odd
// outputs are a prefix sum over q, done per column in a fixed order (serial
// chunks, then a scan of the chunk totals).  out(y) = F_y + (f_0 + (-1)^y f_M)/2.
template <typename T>
__device__ __forceinline__ void dct_cos_body(const Dev<T>& d, Blk bk, const cx<T>* in, cx<T>* out, size_t ws_img,
                                             int adjoint)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    __shared__ cx<T> red[16];     // one entry per lane group (a column's lanes inside one wave;
    __shared__ cx<T> red2[16];    // at most 16 groups: CW <= 16, or 4 waves)
    const int bx_ = bk.x, b = bk.y;
    const int CW = d.dctCW, lcw = d.dctLCW, k0 = bx_ * CW;
    const int M = d.M, logM = d.log2M;
    const cx<T>* ib = reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(in) + (size_t)b * ws_img);
    cx<T>* ob = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(out) + (size_t)b * ws_img);
    const int x_lo = adjoint ? 1 : 0, x_hi = adjoint ? d.nt + 1 : d.L;
    const int nx = x_hi - x_lo;
    const int nout = adjoint ? d.L : d.nt;
    const int ymax = adjoint ? d.L - 1 : d.nt;                 // outputs y = y0 .. ymax
    const int Q = ymax >= 1 ? ((ymax - 1) >> 1) : 0;          // odd outputs need S_0 .. S_Q
    const int SQ = (M >> 1) + 1;                               // scan row pitch (Q < SQ)
    cx<T>* scan = buf + CW * M;                                // CW x SQ
    cx<T>* stash = scan + CW * SQ;                             // CW x nx (with d.dct_stash)
    if (d.dct_stash) {
        for (int i = threadIdx.x; i < CW * nx; i += blockDim.x) {
            const int row = i >> lcw, c = i & (CW - 1);
            const int k = k0 + c;
            stash[c * nx + row] = k < d.Kp ? ib[(size_t)row * d.Kp + k] : cx<T>{T(0), T(0)};
        }
        __syncthreads();
    }
    auto fval = [&](int c, int j) -> cx<T> {
        if (j < x_lo || j >= x_hi || k0 + c >= d.Kp) return cx<T>{T(0), T(0)};
        return d.dct_stash ? stash[c * nx + (j - x_lo)] : ib[(size_t)(j - x_lo) * d.Kp + k0 + c];
    };
    // thread group of each column: TC = NT / CW consecutive threads
    const int TC = NT / CW, c_me = threadIdx.x / TC, lt = threadIdx.x - c_me * TC;
    // F_1's interior sum, reduced in a fixed order: lanes of the column's group
    // within each wave (butterfly), then the column's waves in index order
    const int GW = TC < 64 ? TC : 64;          // lanes of one column inside a wave
    const int NW = TC / GW;                    // waves of one column
    {
        cx<T> acc = {T(0), T(0)};
        for (int j = 1 + lt; j < M; j += TC) acc = acc + fval(c_me, j) * d.twd[j].x;   // cos(pi j/M)
        acc = group_sum(acc, GW);
        if ((lt & (GW - 1)) == 0) red[threadIdx.x / GW] = acc;
    }
    // g into buf
    for (int i = threadIdx.x; i < CW * M; i += blockDim.x) {
        const int j = i >> lcw, c = i & (CW - 1);
        const cx<T> fj = fval(c, j), fm = fval(c, M - j);
        const T sj = -d.twd[j].y;                                                     // sin(pi j/M)
        buf[c * M + j] = {T(0.5) * (fj.x + fm.x) - sj * (fj.x - fm.x), T(0.5) * (fj.y + fm.y) - sj * (fj.y - fm.y)};
    }
    __syncthreads();
    // F_1 of each column (every thread of the column's group)
    const cx<T> f0 = fval(c_me, 0), fM = fval(c_me, M);
    cx<T> F1 = {T(0.5) * (f0.x - fM.x), T(0.5) * (f0.y - fM.y)};
    for (int w = 0; w < NW; ++w) F1 = F1 + red[c_me * NW + w];
    if (d.m3) lds_fft3(buf, logM, CW, M, d.tw, d.logNmax, d.twd, true, d.fft_lr, d.tw_table);
    else lds_fft(buf, logM, CW, M, d.tw, d.logNmax, true, d.fft_lr, d.tw_table);
    // S_q = sum_{p=1..q} D_p, D_p = -(i/2)(G_p - G_{M-p}): serial chunks of CH values per thread
    const int CH = (Q + TC - 1) / TC;
    {
        const cx<T>* Gc = buf + c_me * M;
        cx<T> run = {T(0), T(0)};
        const int q0 = 1 + lt * CH;
        for (int q = q0; q < q0 + CH && q <= Q; ++q) {
            const cx<T> dg = Gc[q] - Gc[M - q];
            run = run + cx<T>{T(0.5) * dg.y, T(-0.5) * dg.x};
            scan[c_me * SQ + q] = run;
        }
        // scan of the chunk totals over the column's lanes: within each wave by
        // shuffles, then the totals of the column's earlier waves
        const cx<T> incl = group_scan(run, GW);
        if ((lt & (GW - 1)) == GW - 1) red2[threadIdx.x / GW] = incl;
        cx<T> offs = {__shfl_up(incl.x, 1, GW), __shfl_up(incl.y, 1, GW)};   // exclusive prefix in the wave
        if ((lt & (GW - 1)) == 0) offs = {T(0), T(0)};
        __syncthreads();
        for (int w = 0; w < (lt / GW); ++w) offs = offs + red2[c_me * NW + w];
        for (int q = q0; q < q0 + CH && q <= Q; ++q) scan[c_me * SQ + q] = scan[c_me * SQ + q] + offs;
        if (lt == 0) scan[c_me * SQ] = F1;                            // slot 0 holds F_1
        __syncthreads();
    }
    // outputs: y = orow (+1 in the forward)
    for (int i = threadIdx.x; i < CW * nout; i += blockDim.x) {
        const int orow = i >> lcw, c = i & (CW - 1);
        const int k = k0 + c;
        if (k >= d.Kp) continue;
        const int y = adjoint ? orow : orow + 1;
        cx<T> F;
        if (y & 1) {
            const int q = y >> 1;
            F = scan[c * SQ];
            if (q > 0) F = F + scan[c * SQ + q];
        } else {
            const int q = y >> 1;
            const cx<T> a = buf[c * M + q], bq = buf[c * M + (q == 0 ? 0 : M - q)];
            F = (a + bq) * T(0.5);
        }
        const cx<T> e0 = fval(c, 0), eM = fval(c, M);
        const T sgn = (y & 1) ? T(-1) : T(1);
        ob[(size_t)orow * d.Kp + k] = {F.x + T(0.5) * (e0.x + sgn * eM.x), F.y + T(0.5) * (e0.y + sgn * eM.y)};
    }
}

// Cosine sum on CW columns of a row-major [rows][Kp] array:
//   forward: in = V [L][Kp] (x = l),       out = G [nt][Kp] (y = j = 1..nt)
//   adjoint: in = G [nt][Kp] (x = j),      out = V [L][Kp] (y = l = 0..L-1)
//   out(y) = sum_x in(x) cos(pi x y / M) = (X(y) + X(-y))/2, X(y) = sum_x in(x) e^{i pi x y/M},
//   or with d.sine sum_x in(x) sin(pi x y / M) = (X(y) - X(-y))/(2i).
// Outputs are split by parity, y = 2y' + r: X(2y'+r) is the M-point inverse DFT of
// in(x) e^{i pi x r/M} (folded mod M) at y', and X(-y) = that DFT at (-y'-r) mod M.
// Two M-point FFTs replace one 2M-point FFT of a zero-padded column.
template <typename T>
__device__ __forceinline__ void dct_cols_body(const Dev<T>& d, Blk bk, const cx<T>* in, cx<T>* out, size_t ws_img, int adjoint)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int bx_ = bk.x, b = bk.y;
    const int CW = d.dctCW, lcw = d.dctLCW, k0 = bx_ * CW;
    const int M = d.M, logM = d.log2M;
    const cx<T>* ib = reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(in) + (size_t)b * ws_img);
    cx<T>* ob = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(out) + (size_t)b * ws_img);
    // valid input indices x in [x_lo, x_hi), stored at row x - x_lo
    const int x_lo = adjoint ? 1 : 0, x_hi = adjoint ? d.nt + 1 : d.L;
    const int nx = x_hi - x_lo;
    const int nout = adjoint ? d.L : d.nt;
    // With enough LDS the block's input columns are read from HBM once into a
    // stash (column-major, CW x nx) and both parities are formed from it.
    cx<T>* stash = buf + CW * M;
    if (d.dct_stash) {
        for (int i = threadIdx.x; i < CW * nx; i += blockDim.x) {
            const int row = i >> lcw, c = i & (CW - 1);
            const int k = k0 + c;
            stash[c * nx + row] = k < d.Kp ? ib[(size_t)row * d.Kp + k] : cx<T>{T(0), T(0)};
        }
        __syncthreads();
    }
    for (int r = 0; r < 2; ++r) {
        for (int i = threadIdx.x; i < CW * M; i += blockDim.x) {
            const int xs = i >> lcw, c = i & (CW - 1);  // slot xs = x mod M
            const int k = k0 + c;
            cx<T> acc = {T(0), T(0)};
            if (k < d.Kp) {
                for (int x = xs; x < x_hi; x += M) {
                    if (x < x_lo) continue;
                    cx<T> v = d.dct_stash ? stash[c * nx + (x - x_lo)] : ib[(size_t)(x - x_lo) * d.Kp + k];
                    if (r) v = cmul(v, conjg(d.twd[x]));  // e^{i pi x/M}, x < 2M
                    acc = acc + v;
                }
            }
            buf[c * M + xs] = acc;
        }
        __syncthreads();
        if (d.m3) lds_fft3(buf, logM, CW, M, d.tw, d.logNmax, d.twd, true, d.fft_lr, d.tw_table);
        else lds_fft(buf, logM, CW, M, d.tw, d.logNmax, true, d.fft_lr, d.tw_table);
        // output rows of parity r only: y = orow (+ 1 in the forward), y = 2 y' + r
        const int o0 = adjoint ? r : 1 - r;
        const int nr = o0 < nout ? (nout - o0 + 1) / 2 : 0;
        for (int i = threadIdx.x; i < CW * nr; i += blockDim.x) {
            const int j = i >> lcw, c = i & (CW - 1);
            const int orow = o0 + 2 * j;
            const int k = k0 + c;
            if (k >= d.Kp) continue;
            const int y = adjoint ? orow : orow + 1;
            const int yp = (y - r) >> 1;
            const int ypp = (M - yp - r) == M ? 0 : M - yp - r;
            // cos: (X(y) + X(-y))/2;  sin: (X(y) - X(-y))/(2i)
            const cx<T> xp = buf[c * M + yp], xm = buf[c * M + ypp];
            ob[(size_t)orow * d.Kp + k] = d.sine ? cx<T>{T(0.5) * (xp.y - xm.y), T(0.5) * (xm.x - xp.x)}
                                                 : (xp + xm) * T(0.5);
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void dct_cols(Dev<T> d, const cx<T>* in, cx<T>* out, size_t ws_img, int adjoint)
{
    if (d.sine || !d.dct_one) dct_cols_body<T>(d, blk_xcd(), in, out, ws_img, adjoint);
    else dct_cos_body<T>(d, blk_xcd(), in, out, ws_img, adjoint);
}

// ---------------------------------------------------------------------------
// Cosine transform, FP32, one wave per column group, lengths fixed at compile
// time.  The same sums as dct_cos_body (the DCT-I of each column's real and
// imaginary parts by ONE M-point FFT, the odd outputs as a prefix sum), laid
// out for a 64-lane wave:
//   * a block of DW_WAVES waves owns DW_WAVES * NC adjacent columns (NC columns
//     per wave when M is short, so that every wave transforms WPTS = NC * M
//     points); it loads their input rows into LDS with row-segment loads and
//     writes the output rows back the same way, so HBM sees contiguous
//     segments of all the block's columns at once;
//   * each wave then works on its own columns with wave-level ordering only:
//     the pre-processing g_j, the Stockham passes (radix 8, a radix-4 or -2
//     remainder, then radix 3 for M = 3 * 2^a) with the butterfly counts and
//     strides known at compile time, and the post-processing, whose prefix
//     sum is a per-lane serial chunk plus a fixed-order wave scan of the
//     chunk totals;
//   * column buffers are padded by one entry in eight, which keeps the
//     early passes' scattered writes (stride 8 entries) on distinct banks.
// ---------------------------------------------------------------------------
constexpr int DW_LPC = 128;             // lanes (two waves) per column group
constexpr int DW_GROUPS = NT / DW_LPC;  // column groups per block

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ constexpr int dw_phys(int i) { return i + (i >> 3); }

template <int M3, int LOGP>
struct DwShape {
    static constexpr int M = (M3 ? 3 : 1) << LOGP;
    static constexpr int WPTS = M3 ? (M >= 1536 ? M : 1536) : (M >= 1024 ? M : 1024);
    static constexpr int NC = WPTS / M;                       // columns per column group
    static constexpr int CB = NC * DW_GROUPS;                 // columns per block
    // column pitch in LDS: slots 0..M (padded), rounded to 8 mod 32 entries so
    // that the block's columns start 16 banks apart in the row-segment phases
    static constexpr int CP = (dw_phys(M) + 1 + 23) / 32 * 32 + 8;
    static constexpr size_t LDS = sizeof(cx<float>) * (size_t)CB * CP;
};

template <bool INV>
__device__ __forceinline__ void dft3_f(cx<float>& a0, cx<float>& a1, cx<float>& a2)
{
    const float h3 = 0.86602540378443864676f;
    const cx<float> sm = a1 + a2, df = a1 - a2;
    const cx<float> m = {a0.x - 0.5f * sm.x, a0.y - 0.5f * sm.y};
    const cx<float> jd = INV ? cx<float>{-h3 * df.y, h3 * df.x} : cx<float>{h3 * df.y, -h3 * df.x};
    a0 = a0 + sm;
    a1 = m + jd;
    a2 = m - jd;
}

// Twiddles W^r, r = 1 .. R-1, of a radix-R butterfly from the table entries
// W^(2^e) that tab(e) returns (at most three products each, no further loads).
template <int R, typename Tab>
__device__ __forceinline__ void tw_powers(Tab tab, cx<float> (&w)[R])
{
    constexpr int LR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
    cx<float> wp[LR];
#pragma unroll
    for (int e = 0; e < LR; ++e) wp[e] = tab(e);
#pragma unroll
    for (int r = 1; r < R; ++r) {
        bool first = true;
#pragma unroll
        for (int e = 0; e < LR; ++e)
            if (r & (1 << e)) {
                w[r] = first ? wp[e] : cmul(w[r], wp[e]);
                first = false;
            }
    }
}

// One Stockham pass over the wave's NC sequences of length M (radix R,
// sub-transform length NS), inverse direction (e^{+2 pi i ...}), in place:
// every lane reads all its inputs before any lane writes.  twd holds
// e^{-2 pi i j / (2M)}.
template <int M, int NC, int CP, int R, int NS>
__device__ __forceinline__ void dw_pass(PAT_LDS cx<float>* buf, const PAT_GLOBAL cx<float>* __restrict__ twd, int lane)
{
    constexpr int L = DW_LPC;
    constexpr int NBS = M / R;               // butterflies per sequence
    constexpr int NBT = NC * NBS;            // butterflies of the column group
    constexpr int PER = (NBT + L - 1) / L;   // butterflies per lane (the last round may be partial)
    // twiddles W_{R NS}^{r k} = twd[r k STEP], conjugated (inverse direction).
    // k = t mod NS: for NS <= L it is lane mod NS for every butterfly of the
    // lane (loaded once); for the radix-3 pass (NS = 2^LOGP >= L) it is
    // lane + L u' and W_M^k = W_M^lane W_M^{L u'} (the second factor uniform).
    // They do not depend on the data: loaded first, so that their latency
    // overlaps the LDS reads and the barrier.
    constexpr int STEP = 2 * M / (R * NS);
    constexpr int LR = R == 2 ? 1 : R == 4 ? 2 : 3;
    cx<float> traw[LR];
    if constexpr (NS > 1 && NS <= L && R != 3) {
        const int k = lane & (NS - 1);
#pragma unroll
        for (int e = 0; e < LR; ++e) traw[e] = ld_glb(twd + ((k * STEP) << e));
    }
    cx<float> wlane = {1.f, 0.f}, wu3[PER];
    if constexpr (R == 3) {
        static_assert(NS >= L, "radix-3 pass after sub-transforms of at least L points");
        wlane = ld_glb(twd + 2 * lane);
        wlane.y = -wlane.y;
#pragma unroll
        for (int u = 0; u < PER; ++u) wu3[u] = ld_glb(twd + 2 * L * ((u % (NS / L))));   // uniform: W_M^{L u'}
    }
    cx<float> v[PER][R];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int t = lane + L * u;
        if (NBT % L != 0 && t >= NBT) continue;
        const int b = t / NBS, tt = t - b * NBS;
        const PAT_LDS cx<float>* s = buf + b * CP;
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = ld_lds(s + dw_phys(tt + r * NBS));
    }
    __syncthreads();
    cx<float> wl[R];
    if constexpr (NS > 1 && NS <= L && R != 3)
        tw_powers<R>([&](int e) { cx<float> w = traw[e]; w.y = -w.y; return w; }, wl);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int t = lane + L * u;
        if (NBT % L != 0 && t >= NBT) continue;
        const int b = t / NBS, tt = t - b * NBS;
        const int k = tt % NS;
        if constexpr (R == 3) {
            cx<float> wu = wu3[u];
            wu.y = -wu.y;
            const cx<float> w1 = cmul(wlane, wu), w2 = cmul(w1, w1);
            v[u][1] = cmul(v[u][1], w1);
            v[u][2] = cmul(v[u][2], w2);
        } else if constexpr (NS > L) {
            cx<float> w[R];
            tw_powers<R>([&](int e) { cx<float> x = ld_glb(twd + ((k * STEP) << e)); x.y = -x.y; return x; }, w);
#pragma unroll
            for (int r = 1; r < R; ++r) v[u][r] = cmul(v[u][r], w[r]);
        } else if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[u][r] = cmul(v[u][r], wl[r]);
        }
        if constexpr (R == 3) dft3_f<true>(v[u][0], v[u][1], v[u][2]);
        else dft_reg<float, R>(v[u], true);
        PAT_LDS cx<float>* s = buf + b * CP;
        const int base = (tt / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) st_lds(s + dw_phys(base + r * NS), v[u][r]);
    }
    __syncthreads();
}

// radix of pass p of the power-of-two factor 2^LOGP: radix 8 while at least
// three bits remain, then 4 or 2
__host__ __device__ constexpr int dw_radix(int LOGP, int p)
{
    return (LOGP - 3 * p >= 3) ? 8 : (LOGP - 3 * p == 2 ? 4 : 2);
}
__host__ __device__ constexpr int dw_npass(int LOGP) { return LOGP / 3 + (LOGP % 3 ? 1 : 0); }
__host__ __device__ constexpr int dw_ns(int LOGP, int p) { return p == 0 ? 1 : dw_ns(LOGP, p - 1) * dw_radix(LOGP, p - 1); }

template <int M, int NC, int CP, int LOGP, int P>
__device__ __forceinline__ void dw_pow2_passes(PAT_LDS cx<float>* buf, const PAT_GLOBAL cx<float>* twd, int lane)
{
    if constexpr (P < dw_npass(LOGP)) {
        dw_pass<M, NC, CP, dw_radix(LOGP, P), dw_ns(LOGP, P)>(buf, twd, lane);
        dw_pow2_passes<M, NC, CP, LOGP, P + 1>(buf, twd, lane);
    }
}

// Fixed-order sum over the 64 lanes (butterfly); every lane gets the total.
__device__ __forceinline__ cx<float> wave_sum(cx<float> v)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        v.x += __shfl_xor(v.x, o, 64);
        v.y += __shfl_xor(v.y, o, 64);
    }
    return v;
}

// Exclusive prefix over the 64 lanes in lane order (Hillis-Steele; fixed order).
__device__ __forceinline__ cx<float> wave_excl_scan(cx<float> v, int lane)
{
    cx<float> s = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const float ux = __shfl_up(s.x, o, 64), uy = __shfl_up(s.y, o, 64);
        if (lane >= o) { s.x += ux; s.y += uy; }
    }
    return s - v;
}

// Column block: forward (adjoint = 0) in = V [L][Kp] -> out = G [nt][Kp],
// out row j holds y = j + 1; adjoint in = G (x = j + 1) -> out = V, row y.
template <int M3, int LOGP, bool SINE>
__device__ __forceinline__ void dct_wave_body(const Dev<float>& d, Blk bk, const cx<float>* in, cx<float>* out,
                                              size_t ws_img, int adjoint)
{
    using S = DwShape<M3, LOGP>;
    constexpr int M = S::M, NC = S::NC, CB = S::CB, CP = S::CP;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    PAT_LDS cx<float>* lbuf = (PAT_LDS cx<float>*)reinterpret_cast<cx<float>*>(smem_raw);
    const PAT_GLOBAL cx<float>* twd = (const PAT_GLOBAL cx<float>*)d.twd;
    const int k0 = bk.x * CB, b = bk.y;
    const cx<float>* ib = reinterpret_cast<const cx<float>*>(reinterpret_cast<const char*>(in) + (size_t)b * ws_img);
    cx<float>* ob = reinterpret_cast<cx<float>*>(reinterpret_cast<char*>(out) + (size_t)b * ws_img);
    const int x_lo = adjoint ? 1 : 0, x_hi = adjoint ? d.nt + 1 : d.L;   // f_x = in row x - x_lo
    const int nx = x_hi - x_lo;
    const int nout = adjoint ? d.L : d.nt;
    const int y0 = adjoint ? 0 : 1, ymax = adjoint ? d.L - 1 : d.nt;
    const int Kp = d.Kp;
    // SINE: out(y) = sum_x f_x sin(pi x y / M) (the approximate inverse), else the cosine sum
    constexpr bool sine = SINE;
    constexpr int L = DW_LPC;
    const int grp = threadIdx.x / L, lane = threadIdx.x - grp * L, wv = lane >> 6;
    // the twiddles of step (2), e^{-i pi j/M} for j = lane + L v: the lane's
    // factor times a uniform one, loaded before the column data
    constexpr int PJ = M / L;
    static_assert(M % L == 0 && NC <= 4, "M must be a multiple of the column group");
    const cx<float> wlane = ld_glb(twd + lane);
    cx<float> wuni[PJ];
#pragma unroll
    for (int v = 0; v < PJ; ++v) wuni[v] = ld_glb(twd + L * v);
    // (1) block: input rows of the CB columns -> column buffers, slots x = 0..M,
    // in chunks of 8 loads per thread, all issued before the chunk's stores
    for (int i0 = 0; i0 < CB * nx; i0 += 8 * NT) {
        cx<float> v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * NT + threadIdx.x;
            const int row = i / CB, c = i - row * CB;
            if (i < CB * nx) v[u] = ld_glb((const PAT_GLOBAL cx<float>*)(ib + (size_t)row * Kp + k0 + c));
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * NT + threadIdx.x;
            const int row = i / CB, c = i - row * CB;
            // the sine sum has no x = 0 or x = M terms (their sines vanish)
            const int x = row + x_lo;
            if (i < CB * nx) st_lds(lbuf + c * CP + dw_phys(x), (sine && (x == 0 || x == M)) ? cx<float>{0.f, 0.f} : v[u]);
        }
    }
    const int nzero = x_lo + (M + 1 - x_hi);   // slots [0, x_lo) and [x_hi, M]
    for (int i = threadIdx.x; i < CB * nzero; i += NT) {
        const int z = i / CB, c = i - z * CB;
        const int x = z < x_lo ? z : x_hi + (z - x_lo);
        st_lds(lbuf + c * CP + dw_phys(x), cx<float>{0.f, 0.f});
    }
    __syncthreads();
    // block-wide partial results of the two waves of each column group
    __shared__ cx<float> red[DW_GROUPS][4][2];
    PAT_LDS cx<float>* wb = lbuf + grp * NC * CP;
    // (2) per column: F_1's interior sum and g_j = (f_j + f_{M-j})/2 - sin(pi j/M) (f_j - f_{M-j});
    // sine: g_j = sin(pi j/M) (f_j + f_{M-j}) + (f_j - f_{M-j})/2 (F_1 unused)
    cx<float> F1[NC], e0[NC], eM[NC];
    {
        cx<float> gv[NC][PJ];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const PAT_LDS cx<float>* col = wb + c * CP;
            e0[c] = ld_lds(col);
            eM[c] = ld_lds(col + dw_phys(M));
            cx<float> acc = {0.f, 0.f};
#pragma unroll
            for (int v = 0; v < PJ; ++v) {
                const int j = lane + L * v;
                const cx<float> fj = ld_lds(col + dw_phys(j));
                const cx<float> fm = ld_lds(col + dw_phys(M - j));
                const cx<float> w = cmul(wlane, wuni[v]);   // (cos(pi j/M), -sin(pi j/M))
                acc = acc + fj * w.x;
                const float sj = -w.y;
                gv[c][v] = sine ? cx<float>{sj * (fj.x + fm.x) + 0.5f * (fj.x - fm.x), sj * (fj.y + fm.y) + 0.5f * (fj.y - fm.y)}
                                : cx<float>{0.5f * (fj.x + fm.x) - sj * (fj.x - fm.x), 0.5f * (fj.y + fm.y) - sj * (fj.y - fm.y)};
            }
            acc = wave_sum(acc);
            if ((lane & 63) == 0) red[grp][c][wv] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            // the group's two wave sums in a fixed order; sum over x = 0..M-1 of
            // f_x cos(pi x/M) minus f_0, plus (f_0 - f_M)/2
            const cx<float> acc = red[grp][c][0] + red[grp][c][1];
            F1[c] = {acc.x - 0.5f * (e0[c].x + eM[c].x), acc.y - 0.5f * (e0[c].y + eM[c].y)};
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int v = 0; v < PJ; ++v) st_lds(wb + c * CP + dw_phys(lane + L * v), gv[c][v]);
        __syncthreads();
    }
    // (3) G_q = sum_j g_j e^{2 pi i j q/M}
    dw_pow2_passes<M, NC, CP, LOGP, 0>(wb, twd, lane);
    if constexpr (M3) dw_pass<M, NC, CP, 3, (1 << LOGP)>(wb, twd, lane);
    // (4) outputs: lane l owns q = CH l + 1 .. CH (l + 1): F_{2q} = (G_q + G_{M-q})/2,
    // F_{2q+1} = F_1 + S_q, S_q = sum_{p=1..q} -(i/2)(G_p - G_{M-p});
    // out(y) = F_y + (f_0 + (-1)^y f_M)/2, written to slot y - y0.
    // Sine (the real-data identities Re G_q = S_{2q+1} - S_{2q-1}, Im G_q = S_{2q},
    // extended linearly to complex data): S_{2q} = -(i/2)(G_q - G_{M-q}),
    // S_{2q+1} = S_1 + sum_{p=1..q} (G_p + G_{M-p})/2, S_1 = G_0/2, S_0 = 0.
    cx<float> G0[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) G0[c] = ld_lds(wb + c * CP);
    const int Q = (ymax + 1) >> 1;             // q needed: even y = 2q <= ymax, odd y = 2q + 1 <= ymax
    constexpr int CHMAX = (M / 2 + L - 1) / L; // Q <= M/2
    const int CH = (Q + L - 1) / L;
    cx<float> outv[NC][CHMAX][2];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const PAT_LDS cx<float>* col = wb + c * CP;
        cx<float> run = {0.f, 0.f};
        cx<float> pre[CHMAX];
#pragma unroll
        for (int i = 0; i < CHMAX; ++i) {
            const int q = lane * CH + 1 + i;
            cx<float> ev = {0.f, 0.f};
            if (i < CH && q <= M / 2) {
                const cx<float> gq = ld_lds(col + dw_phys(q)), gm = ld_lds(col + dw_phys(M - q));
                const cx<float> anti = {0.5f * (gq.y - gm.y), -0.5f * (gq.x - gm.x)}, sym = (gq + gm) * 0.5f;
                run = run + (sine ? sym : anti);
                ev = sine ? anti : sym;
            }
            pre[i] = run;
            outv[c][i][0] = ev;
        }
        // exclusive prefix of the chunk totals over the group's lanes: within each
        // wave, then the first wave's total for the second (fixed order)
        cx<float> off = wave_excl_scan(run, lane & 63);
        const cx<float> incl = off + run;
        if ((lane & 63) == 63) red[grp][c][wv] = incl;
        __syncthreads();
        if (wv == 1) off = off + red[grp][c][0];
        __syncthreads();
        const float hx0 = 0.5f * e0[c].x, hy0 = 0.5f * e0[c].y, hxM = 0.5f * eM[c].x, hyM = 0.5f * eM[c].y;
        const cx<float> S1 = G0[c] * 0.5f;
#pragma unroll
        for (int i = 0; i < CHMAX; ++i) {
            const cx<float> S = off + pre[i];
            // y = 2q (even) and y = 2q + 1 (odd)
            if (sine) {
                outv[c][i][1] = S1 + S;
            } else {
                outv[c][i][0] = {outv[c][i][0].x + hx0 + hxM, outv[c][i][0].y + hy0 + hyM};
                outv[c][i][1] = {F1[c].x + S.x + hx0 - hxM, F1[c].y + S.y + hy0 - hyM};
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        PAT_LDS cx<float>* col = wb + c * CP;
#pragma unroll
        for (int i = 0; i < CHMAX; ++i) {
            const int q = lane * CH + 1 + i;
            if (i < CH) {
                const int ye = 2 * q, yo = 2 * q + 1;
                if (ye <= ymax) st_lds(col + dw_phys(ye - y0), outv[c][i][0]);
                if (yo <= ymax) st_lds(col + dw_phys(yo - y0), outv[c][i][1]);
            }
        }
        if (lane == 0) {
            // y = 1: F_1 + (f_0 - f_M)/2; y = 0 (adjoint only): G_0 + (f_0 + f_M)/2
            // (sine: S_1 = G_0/2 and S_0 = 0)
            if (sine) {
                st_lds(col + dw_phys(1 - y0), G0[c] * 0.5f);
                if (y0 == 0) st_lds(col, cx<float>{0.f, 0.f});
            } else {
                st_lds(col + dw_phys(1 - y0), cx<float>{F1[c].x + 0.5f * (e0[c].x - eM[c].x), F1[c].y + 0.5f * (e0[c].y - eM[c].y)});
                if (y0 == 0) st_lds(col, cx<float>{G0[c].x + 0.5f * (e0[c].x + eM[c].x), G0[c].y + 0.5f * (e0[c].y + eM[c].y)});
            }
        }
    }
    __syncthreads();
    // (5) block: output rows of the CB columns
    for (int i = threadIdx.x; i < CB * nout; i += NT) {
        const int row = i / CB, c = i - row * CB;
        const cx<float> v = ld_lds(lbuf + c * CP + dw_phys(row));
        ob[(size_t)row * Kp + k0 + c] = v;
    }
}

// SINE: the sine sum of the approximate inverse (its own kernel, so that the
// cosine kernel keeps its register budget)
template <int M3, int LOGP, bool SINE>
__global__ __launch_bounds__(NT) void dct_wave(Dev<float> d, const cx<float>* in, cx<float>* out, size_t ws_img,
                                               int adjoint)
{
    dct_wave_body<M3, LOGP, SINE>(d, blk_xcd(), in, out, ws_img, adjoint);
}

// variant code of dct_wave: (M3 << 8) | LOGP, 0 = none
#define PAT_DW_VARIANTS(X) X(1, 7) X(1, 8) X(1, 9) X(0, 8) X(0, 9) X(0, 10)

// the grouped launches (A and A* only, never the inverse's sine sum) take the cosine form
__device__ __forceinline__ void dct_wave_dispatch(const Dev<float>& d, Blk bk, const cx<float>* in, cx<float>* out,
                                                  size_t ws_img, int adjoint)
{
    switch (d.dct_wave) {
#define PAT_DW_CASE(a, b) \
    case ((a) << 8) | (b): dct_wave_body<a, b, false>(d, bk, in, out, ws_img, adjoint); break;
        PAT_DW_VARIANTS(PAT_DW_CASE)
#undef PAT_DW_CASE
        default: break;
    }
}

// ---------------------------------------------------------------------------
// Power-of-two transforms of one 64-lane wave (FP32): the 2D FFT's row and
// column passes and the angular synthesis, with lengths known at compile time.
// Each wave owns one sequence of N = 2^LOGN points in a padded LDS buffer
// (dw_phys: one pad entry every eight) and runs Stockham passes whose
// butterfly counts, strides and radices (8 and 16, or 4 for N = 256) are
// constants; only wave-level ordering is needed between passes.  Twiddles come
// from the plan's table e^{-2 pi i j / Nmax}.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int wf_radix(int LOGN, int p)
{
    return LOGN == 8 ? 4 : LOGN == 9 ? 8 : LOGN == 10 ? (p < 2 ? 8 : 16) : LOGN == 11 ? (p < 1 ? 8 : 16) : 16;
}
__host__ __device__ constexpr int wf_npass(int LOGN) { return LOGN == 8 ? 4 : 3; }
__host__ __device__ constexpr int wf_ns(int LOGN, int p) { return p == 0 ? 1 : wf_ns(LOGN, p - 1) * wf_radix(LOGN, p - 1); }
__host__ __device__ constexpr int wf_log2(int v) { return v <= 1 ? 0 : 1 + wf_log2(v / 2); }

template <int N, int R, int NS, bool INV>
__device__ __forceinline__ void wf_pass(PAT_LDS cx<float>* buf, const PAT_GLOBAL cx<float>* __restrict__ tw, int logNmax,
                                        int lane)
{
    constexpr int NB = N / R;
    constexpr int PER = NB / 64;
    static_assert(NB % 64 == 0, "butterflies must fill the wave");
    cx<float> v[PER][R];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int t = lane + 64 * u;
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = ld_lds(buf + dw_phys(t + r * NB));
    }
    wave_sync();
    // twiddles W_{R NS}^{r k} = tw[(r k) << sh] from W^1, W^2, W^4 (, W^8);
    // for NS <= 64, k = lane mod NS for every butterfly of the lane
    const int sh = logNmax - wf_log2(R * NS);
    auto tab = [&](int k, int e) {
        cx<float> w = ld_glb(tw + ((k << e) << sh));
        if (INV) w.y = -w.y;
        return w;
    };
    cx<float> wl[R];
    if constexpr (NS > 1 && NS <= 64) tw_powers<R>([&](int e) { return tab(lane & (NS - 1), e); }, wl);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int t = lane + 64 * u;
        const int k = t % NS;
        if constexpr (NS > 64) {
            cx<float> w[R];
            tw_powers<R>([&](int e) { return tab(k, e); }, w);
#pragma unroll
            for (int r = 1; r < R; ++r) v[u][r] = cmul(v[u][r], w[r]);
        } else if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[u][r] = cmul(v[u][r], wl[r]);
        }
        dft_reg<float, R>(v[u], INV);
        const int base = (t / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) st_lds(buf + dw_phys(base + r * NS), v[u][r]);
    }
    wave_sync();
}

template <int LOGN, bool INV, int P = 0>
__device__ __forceinline__ void wf_fft(PAT_LDS cx<float>* buf, const PAT_GLOBAL cx<float>* tw, int logNmax, int lane)
{
    if constexpr (P < wf_npass(LOGN)) {
        wf_pass<(1 << LOGN), wf_radix(LOGN, P), wf_ns(LOGN, P), INV>(buf, tw, logNmax, lane);
        wf_fft<LOGN, INV, P + 1>(buf, tw, logNmax, lane);
    }
}

constexpr int WF_WAVES = 4;                 // waves (sequences) per block
__host__ __device__ constexpr int wf_pitch(int LOGN) { return (dw_phys(1 << LOGN) + 1 + 23) / 32 * 32 + 8; }

// rows_fwd with one wave per pair of image rows (p1 = 2 pair, p2 = p1 + 1): the
// pre-corrected rows, zero-extended to Ng and packed as one complex sequence,
// one FFT, then the half spectra of both rows.
template <int LOGN>
__device__ __forceinline__ void rows_fwd_w_body(const Dev<float>& d, Blk bk, const float* __restrict__ f, long fstride,
                                                cx<float>* R, size_t ws_img)
{
    constexpr int Ng = 1 << LOGN;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    PAT_LDS cx<float>* buf = (PAT_LDS cx<float>*)reinterpret_cast<cx<float>*>(smem_raw) + wave * wf_pitch(LOGN);
    const int pair = bk.x * WF_WAVES + wave, b = bk.y;
    const int n = d.n, p1 = 2 * pair, p2 = p1 + 1;
    if (p1 >= n) return;   // whole wave: no block-wide synchronisation follows
    const float* fb = f + (size_t)b * fstride;
    cx<float>* Rb = reinterpret_cast<cx<float>*>(reinterpret_cast<char*>(R) + (size_t)b * ws_img);
    const float s1 = d.Dq[p1] * d.pre_scale;
    const float s2 = p2 < n ? d.Dq[p2] * d.pre_scale : 0.f;
    const int h = n / 2;
    // chunks of 8 positions per lane, loaded before the chunk's stores
    for (int i0 = 0; i0 < Ng; i0 += 8 * 64) {
        float dq[8], x1[8], x2[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            // position i holds column q = i + n/2 (i < n - n/2) or q = i - Ng + n/2 (i >= Ng - n/2)
            const int i = i0 + u * 64 + lane;
            const int q = i < n - h ? i + h : (i >= Ng - h ? i - Ng + h : -1);
            dq[u] = x1[u] = x2[u] = 0.f;
            if (i < Ng && q >= 0) {
                dq[u] = d.Dq[q];
                if (in_mask(d, p1, q)) x1[u] = fb[(size_t)p1 * n + q];
                if (p2 < n && in_mask(d, p2, q)) x2[u] = fb[(size_t)p2 * n + q];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * 64 + lane;
            if (i < Ng) st_lds(buf + dw_phys(i), cx<float>{x1[u] * dq[u] * s1, x2[u] * dq[u] * s2});
        }
    }
    wave_sync();
    wf_fft<LOGN, false>(buf, (const PAT_GLOBAL cx<float>*)d.tw, d.logNmax, lane);
    for (int g = lane; g <= Ng / 2; g += 64) {
        const cx<float> zg = ld_lds(buf + dw_phys(g)), zm = ld_lds(buf + dw_phys((Ng - g) & (Ng - 1)));
        const cx<float> x1 = {0.5f * (zg.x + zm.x), 0.5f * (zg.y - zm.y)};
        const cx<float> x2 = {0.5f * (zg.y + zm.y), 0.5f * (zm.x - zg.x)};
        Rb[(size_t)p1 * d.Rw + g] = x1;
        if (p2 < n) Rb[(size_t)p2 * d.Rw + g] = x2;
    }
}

// rows_adj with one wave per pair of image rows (transpose of rows_fwd_w_body).
template <int LOGN>
__device__ __forceinline__ void rows_adj_w_body(const Dev<float>& d, Blk bk, const cx<float>* R, float* f, long fstride,
                                                size_t ws_img)
{
    constexpr int Ng = 1 << LOGN, hN = Ng / 2;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    PAT_LDS cx<float>* buf = (PAT_LDS cx<float>*)reinterpret_cast<cx<float>*>(smem_raw) + wave * wf_pitch(LOGN);
    const int pair = bk.x * WF_WAVES + wave, b = bk.y;
    const int n = d.n, p1 = 2 * pair, p2 = p1 + 1;
    if (p1 >= n) return;
    const bool has2 = p2 < n;
    const cx<float>* Rb = reinterpret_cast<const cx<float>*>(reinterpret_cast<const char*>(R) + (size_t)b * ws_img);
    float* fb = f + (size_t)b * fstride;
    // chunks of 8 positions per lane: R entries g (g <= Ng/2) or Ng - g, loaded
    // before the chunk's stores
    for (int g0 = 0; g0 < Ng; g0 += 8 * 64) {
        cx<float> ra[8], rb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int g = g0 + u * 64 + lane, gg = g <= hN ? g : Ng - g;
            ra[u] = rb[u] = cx<float>{0.f, 0.f};
            if (g < Ng) {
                ra[u] = Rb[(size_t)p1 * d.Rw + gg];
                if (has2) rb[u] = Rb[(size_t)p2 * d.Rw + gg];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int g = g0 + u * 64 + lane;
            if (g >= Ng) continue;
            cx<float> xa, xb;
            if (g == 0 || g == hN) {
                xa = {ra[u].x, 0.f};
                xb = {rb[u].x, 0.f};
            } else if (g < hN) {
                xa = ra[u] * 0.5f;
                xb = rb[u] * 0.5f;
            } else {
                xa = conjg(ra[u]) * 0.5f;
                xb = conjg(rb[u]) * 0.5f;
            }
            st_lds(buf + dw_phys(g), cx<float>{xa.x - xb.y, xa.y + xb.x});
        }
    }
    wave_sync();
    wf_fft<LOGN, true>(buf, (const PAT_GLOBAL cx<float>*)d.tw, d.logNmax, lane);
    const float s1 = d.Dq[p1] * d.pre_scale * d.adj_scale;
    const float s2 = has2 ? d.Dq[p2] * d.pre_scale * d.adj_scale : 0.f;
    for (int q0 = 0; q0 < n; q0 += 8 * 64) {
        // the chunk's Dq, loaded before its stores
        float dq[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * 64 + lane;
            dq[u] = q < n ? d.Dq[q] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * 64 + lane;
            if (q >= n) continue;
            const cx<float> v = ld_lds(buf + dw_phys((q - n / 2 + Ng) & (Ng - 1)));
            put_image(d, fb, b, p1, q, in_mask(d, p1, q) ? v.x * dq[u] * s1 : 0.f);
            if (has2) put_image(d, fb, b, p2, q, in_mask(d, p2, q) ? v.y * dq[u] * s2 : 0.f);
        }
    }
}

// cols_fwd with one wave per spectrum column: the block's WF_WAVES adjacent
// columns are loaded and stored as row segments, each wave transforms its own.
template <int LOGN>
__device__ __forceinline__ void cols_fwd_w_body(const Dev<float>& d, Blk bk, const cx<float>* R, cx<float>* E,
                                                size_t ws_img)
{
    constexpr int Ng = 1 << LOGN, CB = WF_WAVES, CP = wf_pitch(LOGN);
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    PAT_LDS cx<float>* lbuf = (PAT_LDS cx<float>*)reinterpret_cast<cx<float>*>(smem_raw);
    const int x0 = bk.x * CB, b = bk.y, n = d.n;
    const cx<float>* Rb = reinterpret_cast<const cx<float>*>(reinterpret_cast<const char*>(R) + (size_t)b * ws_img);
    cx<float>* Eb = reinterpret_cast<cx<float>*>(reinterpret_cast<char*>(E) + (size_t)b * ws_img);
    // rows p of R land at (p - n/2) mod Ng; positions [n - n/2, Ng - n/2) stay zero
    const int h = n / 2, nz = Ng - n;
    // chunks of 8 loads per thread, issued before the chunk's stores
    for (int i0 = 0; i0 < CB * n; i0 += 8 * NT) {
        cx<float> v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * NT + threadIdx.x, p = i / CB, gx = x0 + (i - p * CB);
            v[u] = (i < CB * n && gx < d.Rw) ? Rb[(size_t)p * d.Rw + gx] : cx<float>{0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * NT + threadIdx.x, p = i / CB, c = i - p * CB;
            if (i < CB * n) st_lds(lbuf + c * CP + dw_phys((p - h + Ng) & (Ng - 1)), v[u]);
        }
    }
    for (int i = threadIdx.x; i < CB * nz; i += NT) {
        const int z = i / CB, c = i - z * CB;
        st_lds(lbuf + c * CP + dw_phys(n - h + z), cx<float>{0.f, 0.f});
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    wf_fft<LOGN, false>(lbuf + wave * CP, (const PAT_GLOBAL cx<float>*)d.tw, d.logNmax, lane);
    __syncthreads();
    for (int i = threadIdx.x; i < CB * Ng; i += NT) {
        const int gy = i / CB, c = i - gy * CB;
        const int gx = x0 + c;
        if (gx >= d.Rw) continue;
        const cx<float> v = ld_lds(lbuf + c * CP + dw_phys(gy));
        Eb[(size_t)gy * d.Ep + gx + d.hw] = v;
        const int gym = (Ng - gy) & (Ng - 1);
        if (gx >= 1 && gx <= d.hw) Eb[(size_t)gym * d.Ep + d.hw - gx] = conjg(v);
        if (gx >= Ng / 2 - d.hw && gx <= Ng / 2 - 1) Eb[(size_t)gym * d.Ep + d.hw + Ng - gx] = conjg(v);
    }
}

// cols_adj with one wave per spectrum column (transpose of cols_fwd_w_body).
template <int LOGN>
__device__ __forceinline__ void cols_adj_w_body(const Dev<float>& d, Blk bk, const cx<float>* E, cx<float>* R,
                                                size_t ws_img)
{
    constexpr int Ng = 1 << LOGN, CB = WF_WAVES, CP = wf_pitch(LOGN);
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    PAT_LDS cx<float>* lbuf = (PAT_LDS cx<float>*)reinterpret_cast<cx<float>*>(smem_raw);
    const int x0 = bk.x * CB, b = bk.y, n = d.n;
    const cx<float>* Eb = reinterpret_cast<const cx<float>*>(reinterpret_cast<const char*>(E) + (size_t)b * ws_img);
    cx<float>* Rb = reinterpret_cast<cx<float>*>(reinterpret_cast<char*>(R) + (size_t)b * ws_img);
    // chunks of 8 cells per thread, loaded before the chunk's stores (the
    // margin folds, rare, load their second operand in place)
    for (int i0 = 0; i0 < CB * Ng; i0 += 8 * NT) {
        cx<float> v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * NT + threadIdx.x, gy = i / CB, gx = x0 + (i - gy * CB);
            v[u] = (i < CB * Ng && gx < d.Rw) ? Eb[(size_t)gy * d.Ep + gx + d.hw] : cx<float>{0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * NT + threadIdx.x, gy = i / CB, c = i - gy * CB, gx = x0 + c;
            if (i >= CB * Ng) continue;
            if (gx < d.Rw) {
                const int gym = (Ng - gy) & (Ng - 1);
                if (gx >= 1 && gx <= d.hw) v[u] = v[u] + conjg(Eb[(size_t)gym * d.Ep + d.hw - gx]);
                if (gx >= Ng / 2 - d.hw && gx <= Ng / 2 - 1) v[u] = v[u] + conjg(Eb[(size_t)gym * d.Ep + d.hw + Ng - gx]);
            }
            st_lds(lbuf + c * CP + dw_phys(gy), v[u]);
        }
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    wf_fft<LOGN, true>(lbuf + wave * CP, (const PAT_GLOBAL cx<float>*)d.tw, d.logNmax, lane);
    __syncthreads();
    for (int i = threadIdx.x; i < CB * n; i += NT) {
        const int p = i / CB, c = i - p * CB;
        const int gx = x0 + c;
        if (gx < d.Rw) Rb[(size_t)p * d.Rw + gx] = ld_lds(lbuf + c * CP + dw_phys((p - n / 2 + Ng) & (Ng - 1)));
    }
}

// synth_fwd with one wave per pair of time rows (j1 = 2 pair, j2 = j1 + 1):
// Q_r = Herm(Z1)_r + i Herm(Z2)_r from the folded harmonics (each lane owns the
// pair r, mf - r and reads both straight from G), one inverse FFT of mf points,
// real and imaginary parts to the two trace rows.
template <int LOGM>
__device__ __forceinline__ void synth_fwd_w_body(const Dev<float>& d, Blk bk, const cx<float>* G, float* g, long gstride,
                                                 size_t ws_img)
{
    constexpr int mf = 1 << LOGM;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    PAT_LDS cx<float>* buf = (PAT_LDS cx<float>*)reinterpret_cast<cx<float>*>(smem_raw) + wave * wf_pitch(LOGM);
    const int pair = bk.x * WF_WAVES + wave, b = bk.y;
    const int j1 = 2 * pair, j2 = j1 + 1;
    if (j1 >= d.nt) return;
    const bool has2 = j2 < d.nt;
    const cx<float>* Gb = reinterpret_cast<const cx<float>*>(reinterpret_cast<const char*>(G) + (size_t)b * ws_img);
    const cx<float>* G1 = Gb + (size_t)j1 * d.Kp;
    const cx<float>* G2 = Gb + (size_t)j2 * d.Kp;
    // fold of harmonic row `row` onto residue r: the terms k = r, r + mf, ... <= K
    // in that order; the first term's operands are passed in (loaded ahead)
    auto fold = [&](const cx<float>* row, int r, cx<float> ph0, cx<float> v0) -> cx<float> {
        cx<float> z = {0.f, 0.f};
        if (r <= d.K) z = z + cmul(ph0 * (r == 0 ? 1.f : 2.f), v0);
        for (int k = r + mf; k <= d.K; k += mf) z = z + cmul(d.phase[k] * 2.f, row[k]);
        return z;
    };
    // chunks of SY_CH residues per lane: the first terms' phases and values of
    // both rows are loaded together before any is used
    constexpr int SY_CH = 4;
    for (int r0 = 0; r0 <= mf / 2; r0 += SY_CH * 64) {
        cx<float> p0[SY_CH], pm0[SY_CH], a0[SY_CH], am0[SY_CH], c0[SY_CH], cm0[SY_CH];
#pragma unroll
        for (int u = 0; u < SY_CH; ++u) {
            const int r = r0 + u * 64 + lane, rm = r == 0 ? 0 : mf - r;
            const cx<float> z = {0.f, 0.f};
            p0[u] = pm0[u] = a0[u] = am0[u] = c0[u] = cm0[u] = z;
            if (r > mf / 2) continue;
            if (r <= d.K) {
                p0[u] = d.phase[r];
                a0[u] = G1[r];
                if (has2) c0[u] = G2[r];
            }
            if (rm <= d.K) {
                pm0[u] = d.phase[rm];
                am0[u] = G1[rm];
                if (has2) cm0[u] = G2[rm];
            }
        }
#pragma unroll
        for (int u = 0; u < SY_CH; ++u) {
            const int r = r0 + u * 64 + lane, rm = r == 0 ? 0 : mf - r;
            if (r > mf / 2) continue;
            const cx<float> a = fold(G1, r, p0[u], a0[u]), am = fold(G1, rm, pm0[u], am0[u]);
            const cx<float> c = has2 ? fold(G2, r, p0[u], c0[u]) : cx<float>{0.f, 0.f};
            const cx<float> cm = has2 ? fold(G2, rm, pm0[u], cm0[u]) : cx<float>{0.f, 0.f};
            const cx<float> h1 = {0.5f * (a.x + am.x), 0.5f * (a.y - am.y)};
            const cx<float> h2 = {0.5f * (c.x + cm.x), 0.5f * (c.y - cm.y)};
            st_lds(buf + dw_phys(r), cx<float>{h1.x - h2.y, h1.y + h2.x});
            if (rm != r) st_lds(buf + dw_phys(rm), cx<float>{h1.x + h2.y, h2.x - h1.y});
        }
    }
    wave_sync();
    wf_fft<LOGM, true>(buf, (const PAT_GLOBAL cx<float>*)d.tw, d.logNmax, lane);
    for (int i = lane; i < d.m; i += 64) {
        const cx<float> v = ld_lds(buf + dw_phys(i));
        put_trace(d, g, (size_t)b * gstride + (size_t)j1 * d.m + i, v.x);
        if (has2) put_trace(d, g, (size_t)b * gstride + (size_t)j2 * d.m + i, v.y);
    }
}

// synth_adj with one wave per pair of time rows (transpose of synth_fwd_w_body).
template <int LOGM>
__device__ __forceinline__ void synth_adj_w_body(const Dev<float>& d, Blk bk, const float* g, long gstride, cx<float>* G,
                                                 size_t ws_img)
{
    constexpr int mf = 1 << LOGM;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    PAT_LDS cx<float>* buf = (PAT_LDS cx<float>*)reinterpret_cast<cx<float>*>(smem_raw) + wave * wf_pitch(LOGM);
    const int pair = bk.x * WF_WAVES + wave, b = bk.y;
    const int j1 = 2 * pair, j2 = j1 + 1;
    if (j1 >= d.nt) return;
    const bool has2 = j2 < d.nt;
    const float* gb = g + (size_t)b * gstride;
    cx<float>* Gb = reinterpret_cast<cx<float>*>(reinterpret_cast<char*>(G) + (size_t)b * ws_img);
    // chunks of 8 entries per lane, all loads issued before the chunk's stores
    for (int i0 = 0; i0 < mf; i0 += 8 * 64) {
        float a[8], c[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * 64 + lane;
            a[u] = (i < mf && i < d.m) ? gb[(size_t)j1 * d.m + i] : 0.f;
            c[u] = (i < mf && i < d.m && has2) ? gb[(size_t)j2 * d.m + i] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * 64 + lane;
            if (i < mf) st_lds(buf + dw_phys(i), cx<float>{a[u], c[u]});
        }
    }
    wave_sync();
    wf_fft<LOGM, false>(buf, (const PAT_GLOBAL cx<float>*)d.tw, d.logNmax, lane);
    for (int k0 = 0; k0 < d.Kp; k0 += 4 * 64) {
        // the chunk's phases, loaded before its stores
        cx<float> phk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * 64 + lane;
            phk[u] = k <= d.K ? d.phase[k] : cx<float>{0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * 64 + lane;
            if (k >= d.Kp) continue;
            cx<float> y1 = {0.f, 0.f}, y2 = {0.f, 0.f};
            if (k <= d.K) {
                const int r = k & (mf - 1), rm = r == 0 ? 0 : mf - r;
                const cx<float> zr = ld_lds(buf + dw_phys(r)), zm = ld_lds(buf + dw_phys(rm));
                y1 = {0.5f * (zr.x + zm.x), 0.5f * (zr.y - zm.y)};
                y2 = {0.5f * (zr.y + zm.y), 0.5f * (zm.x - zr.x)};
                const cx<float> ph = conjg(phk[u]) * (k == 0 ? 1.f : 2.f);
                y1 = cmul(ph, y1);
                y2 = cmul(ph, y2);
            }
            Gb[(size_t)j1 * d.Kp + k] = y1;
            if (has2) Gb[(size_t)j2 * d.Kp + k] = y2;
        }
    }
}

#define PAT_WF_SIZES(X) X(8) X(9) X(10) X(11)

template <int LOGN>
__global__ __launch_bounds__(NT) void rows_fwd_w(Dev<float> d, const float* __restrict__ f, long fstride, cx<float>* R,
                                                 size_t ws_img)
{
    rows_fwd_w_body<LOGN>(d, blk_xcd(), f, fstride, R, ws_img);
}
template <int LOGN>
__global__ __launch_bounds__(NT) void rows_adj_w(Dev<float> d, const cx<float>* R, float* f, long fstride, size_t ws_img)
{
    rows_adj_w_body<LOGN>(d, blk_xcd(), R, f, fstride, ws_img);
}
template <int LOGN>
__global__ __launch_bounds__(NT) void cols_fwd_w(Dev<float> d, const cx<float>* R, cx<float>* E, size_t ws_img)
{
    cols_fwd_w_body<LOGN>(d, blk_xcd(), R, E, ws_img);
}
template <int LOGN>
__global__ __launch_bounds__(NT) void cols_adj_w(Dev<float> d, const cx<float>* E, cx<float>* R, size_t ws_img)
{
    cols_adj_w_body<LOGN>(d, blk_xcd(), E, R, ws_img);
}
template <int LOGM>
__global__ __launch_bounds__(NT) void synth_fwd_w(Dev<float> d, const cx<float>* G, float* g, long gstride, size_t ws_img)
{
    synth_fwd_w_body<LOGM>(d, blk_xcd(), G, g, gstride, ws_img);
}
template <int LOGM>
__global__ __launch_bounds__(NT) void synth_adj_w(Dev<float> d, const float* g, long gstride, cx<float>* G, size_t ws_img)
{
    synth_adj_w_body<LOGM>(d, blk_xcd(), g, gstride, G, ws_img);
}

__device__ __forceinline__ void rows_fwd_w_dispatch(const Dev<float>& d, Blk bk, const float* f, long fs, cx<float>* R,
                                                    size_t wi)
{
    switch (d.wfRows) {
#define PAT_WF_CASE(L) \
    case L: rows_fwd_w_body<L>(d, bk, f, fs, R, wi); break;
        PAT_WF_SIZES(PAT_WF_CASE)
#undef PAT_WF_CASE
        default: break;
    }
}
__device__ __forceinline__ void rows_adj_w_dispatch(const Dev<float>& d, Blk bk, const cx<float>* R, float* f, long fs,
                                                    size_t wi)
{
    switch (d.wfRows) {
#define PAT_WF_CASE(L) \
    case L: rows_adj_w_body<L>(d, bk, R, f, fs, wi); break;
        PAT_WF_SIZES(PAT_WF_CASE)
#undef PAT_WF_CASE
        default: break;
    }
}
__device__ __forceinline__ void cols_fwd_w_dispatch(const Dev<float>& d, Blk bk, const cx<float>* R, cx<float>* E, size_t wi)
{
    switch (d.wfRows) {
#define PAT_WF_CASE(L) \
    case L: cols_fwd_w_body<L>(d, bk, R, E, wi); break;
        PAT_WF_SIZES(PAT_WF_CASE)
#undef PAT_WF_CASE
        default: break;
    }
}
__device__ __forceinline__ void cols_adj_w_dispatch(const Dev<float>& d, Blk bk, const cx<float>* E, cx<float>* R, size_t wi)
{
    switch (d.wfRows) {
#define PAT_WF_CASE(L) \
    case L: cols_adj_w_body<L>(d, bk, E, R, wi); break;
        PAT_WF_SIZES(PAT_WF_CASE)
#undef PAT_WF_CASE
        default: break;
    }
}
__device__ __forceinline__ void synth_fwd_w_dispatch(const Dev<float>& d, Blk bk, const cx<float>* G, float* g, long gs,
                                                     size_t wi)
{
    switch (d.wfSynth) {
#define PAT_WF_CASE(L) \
    case L: synth_fwd_w_body<L>(d, bk, G, g, gs, wi); break;
        PAT_WF_SIZES(PAT_WF_CASE)
#undef PAT_WF_CASE
        default: break;
    }
}
__device__ __forceinline__ void synth_adj_w_dispatch(const Dev<float>& d, Blk bk, const float* g, long gs, cx<float>* G,
                                                     size_t wi)
{
    switch (d.wfSynth) {
#define PAT_WF_CASE(L) \
    case L: synth_adj_w_body<L>(d, bk, g, gs, G, wi); break;
        PAT_WF_SIZES(PAT_WF_CASE)
#undef PAT_WF_CASE
        default: break;
    }
}

// G_k(t_j) += i^k sum_l Mk[k][j][l] Ulow[l][k], k = 0..klow.  Each group of
// LK_LANES consecutive lanes owns one (j, k) output: lane p sums the terms
// l = p, p + LK_LANES, ..., then the group adds its partial sums in a fixed
// (butterfly) order, so every output is a short chain of loads.
constexpr int LK_LANES = 8;

template <typename T>
__device__ __forceinline__ void lowk_fwd_body(const Dev<T>& d, Blk bk, const cx<T>* Ulow, cx<T>* G, size_t ws_img)
{
    const int b = bk.y;
    const cx<T>* Ub = reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(Ulow) + (size_t)b * ws_img);
    cx<T>* Gb = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(G) + (size_t)b * ws_img);
    const int items = d.nt * (d.klow + 1);
    const int p = threadIdx.x & (LK_LANES - 1);
    for (int it = (bk.x * NT + (int)threadIdx.x) / LK_LANES; it < items; it += bk.nx * NT / LK_LANES) {
        const int j = it / (d.klow + 1), k = it - j * (d.klow + 1);
        const T* row = d.Mk + ((size_t)k * d.nt + j) * d.lcorr;
        cx<T> acc = {T(0), T(0)};
        for (int l = p; l < d.lcorr; l += LK_LANES) acc = acc + Ub[(size_t)l * (d.klow + 1) + k] * row[l];
        acc = group_sum(acc, LK_LANES);
        if (p == 0) {
            cx<T>* dst = Gb + (size_t)j * d.Kp + k;
            *dst = *dst + mul_ipow(acc, k);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void lowk_fwd(Dev<T> d, const cx<T>* Ulow, cx<T>* G, size_t ws_img)
{
    lowk_fwd_body<T>(d, blk_plain(), Ulow, G, ws_img);
}

template <typename T>
__device__ __forceinline__ void synth_fwd_body(const Dev<T>& d, Blk bk, const cx<T>* G, T* g, long gstride, size_t ws_img)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* Z1 = reinterpret_cast<cx<T>*>(smem_raw);
    cx<T>* Z2 = Z1 + d.mf;
    int bx_, b;
    bx_ = bk.x;
    b = bk.y;
    const int j1 = 2 * bx_, j2 = j1 + 1;
    const int mf = d.mf;
    const cx<T>* Gb = reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(G) + (size_t)b * ws_img);
    const bool has2 = j2 < d.nt;
    for (int r = threadIdx.x; r < mf; r += blockDim.x) {
        cx<T> z1 = {T(0), T(0)}, z2 = {T(0), T(0)};
        for (int k = r; k <= d.K; k += mf) {
            cx<T> ph = d.phase[k] * (k == 0 ? T(1) : T(2));
            z1 = z1 + cmul(ph, Gb[(size_t)j1 * d.Kp + k]);
            if (has2) z2 = z2 + cmul(ph, Gb[(size_t)j2 * d.Kp + k]);
        }
        Z1[r] = z1;
        Z2[r] = z2;
    }
    __syncthreads();
    // Q_r = Herm(Z1)_r + i Herm(Z2)_r,  Herm(Z)_r = (Z_r + conj(Z_{-r}))/2.
    // Each thread owns the pair (r, mf - r) and rewrites both entries of Z1 in place.
    for (int r = threadIdx.x; r <= mf / 2; r += blockDim.x) {
        int rm = r == 0 ? 0 : mf - r;
        cx<T> a = Z1[r], am = Z1[rm], c = Z2[r], cm = Z2[rm];
        cx<T> h1 = {T(0.5) * (a.x + am.x), T(0.5) * (a.y - am.y)};
        cx<T> h2 = {T(0.5) * (c.x + cm.x), T(0.5) * (c.y - cm.y)};
        Z1[r] = {h1.x - h2.y, h1.y + h2.x};
        if (rm != r) Z1[rm] = {h1.x + h2.y, h2.x - h1.y};
    }
    __syncthreads();
    if (d.mf3) lds_fft3(Z1, d.logmf, 1, 0, d.tw, d.logNmax, d.twm, true, d.fft_lr, d.tw_table);
    else lds_fft(Z1, d.logmf, 1, 0, d.tw, d.logNmax, true, d.fft_lr, d.tw_table);
    for (int i = threadIdx.x; i < d.m; i += blockDim.x) {
        put_trace(d, g, (size_t)b * gstride + (size_t)j1 * d.m + i, Z1[i].x);
        if (has2) put_trace(d, g, (size_t)b * gstride + (size_t)j2 * d.m + i, Z1[i].y);
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void synth_fwd(Dev<T> d, const cx<T>* G, T* g, long gstride, size_t ws_img)
{
    synth_fwd_body<T>(d, blk_xcd(), G, g, gstride, ws_img);
}

// ---------------------------------------------------------------------------
// adjoint kernels (exact transposes, reverse order)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void synth_adj_body(const Dev<T>& d, Blk bk, const T* g, long gstride, cx<T>* G, size_t ws_img)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* Z = reinterpret_cast<cx<T>*>(smem_raw);
    int bx_, b;
    bx_ = bk.x;
    b = bk.y;
    const int j1 = 2 * bx_, j2 = j1 + 1;
    const int mf = d.mf;
    const bool has2 = j2 < d.nt;
    const T* gb = g + (size_t)b * gstride;
    cx<T>* Gb = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(G) + (size_t)b * ws_img);
    for (int i = threadIdx.x; i < mf; i += blockDim.x) {
        T a = i < d.m ? gb[(size_t)j1 * d.m + i] : T(0);
        T c = (i < d.m && has2) ? gb[(size_t)j2 * d.m + i] : T(0);
        Z[i] = {a, c};
    }
    __syncthreads();
    if (d.mf3) lds_fft3(Z, d.logmf, 1, 0, d.tw, d.logNmax, d.twm, false, d.fft_lr, d.tw_table);
    else lds_fft(Z, d.logmf, 1, 0, d.tw, d.logNmax, false, d.fft_lr, d.tw_table);
    for (int k = threadIdx.x; k < d.Kp; k += blockDim.x) {
        cx<T> y1 = {T(0), T(0)}, y2 = {T(0), T(0)};
        if (k <= d.K) {
            const int r = k % mf, rm = r == 0 ? 0 : mf - r;
            cx<T> zr = Z[r], zm = Z[rm];
            y1 = {T(0.5) * (zr.x + zm.x), T(0.5) * (zr.y - zm.y)};
            y2 = {T(0.5) * (zr.y + zm.y), T(0.5) * (zm.x - zr.x)};
            cx<T> ph = conjg(d.phase[k]) * (k == 0 ? T(1) : T(2));
            y1 = cmul(ph, y1);
            y2 = cmul(ph, y2);
        }
        Gb[(size_t)j1 * d.Kp + k] = y1;
        if (has2) Gb[(size_t)j2 * d.Kp + k] = y2;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void synth_adj(Dev<T> d, const T* g, long gstride, cx<T>* G, size_t ws_img)
{
    synth_adj_body<T>(d, blk_xcd(), g, gstride, G, ws_img);
}

// Ulow_hat[l][k] = conj(i^k) sum_j Mk[k][j][l] G_hat[j][k]; one block per ring l
// (the transposed copy MkT, so that lanes read consecutive t_j).  Wave w of the
// block handles k = w, w + 4, ...: its lanes sum strided runs of j, then the wave
// adds them in a fixed (butterfly) order -- no block-wide synchronisation.
template <typename T>
__device__ __forceinline__ void lowk_adj_body(const Dev<T>& d, Blk bk, const cx<T>* G, cx<T>* Ulow, size_t ws_img)
{
    const int b = bk.y, l = bk.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const cx<T>* Gb = reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(G) + (size_t)b * ws_img);
    cx<T>* Ub = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(Ulow) + (size_t)b * ws_img);
    for (int k = wave; k <= d.klow; k += NT / 64) {
        const T* row = d.MkT + ((size_t)k * d.lcorr + l) * d.nt;
        cx<T> acc = {T(0), T(0)};
        for (int j = lane; j < d.nt; j += 64) acc = acc + Gb[(size_t)j * d.Kp + k] * row[j];
        acc = group_sum(acc, 64);
        if (lane == 0) Ub[(size_t)l * (d.klow + 1) + k] = mul_ipow(acc, (4 - (k & 3)) & 3);
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void lowk_adj(Dev<T> d, const cx<T>* G, cx<T>* Ulow, size_t ws_img)
{
    lowk_adj_body<T>(d, blk_plain(), G, Ulow, ws_img);
}

// Samples are written image-minor, Pol[k * B + b], already multiplied by the
// conjugate point phase, for the batched spreads below (whole rows of B values
// per sample: the spreads' staging reads them whole); k is the ring-order
// index ringOff[l] + si, or for the binned spread the sample's bin-order slot,
// so that spread_bins stages the runs of a bin row as contiguous memory.
template <typename T, int WMAX>
__device__ __forceinline__ void ring_adj_body(const Dev<T>& d, Blk bk, const cx<T>* V, const cx<T>* Ulow, cx<T>* Pol, int B,
                                              int G, size_t ws_img)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    // no XCD renumbering here: contiguous ranges of rings would unbalance the XCDs
    const int grp = bk.x, l = bk.y;
    const int b0 = grp * G, nb = min(G, B - b0);
    const int N = d.ringN[l], logN = d.ringLog[l], Kl = d.ringK[l];
    const T invN = T(1) / T(N);
    // per image, chunks of RING_CH harmonics per thread whose loads are issued together
    for (int i = 0; i < nb; ++i) {
        const cx<T>* Vb = reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(V) + (size_t)(b0 + i) * ws_img);
        const cx<T>* Ub = reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(Ulow) + (size_t)(b0 + i) * ws_img);
        for (int k0 = 0; k0 < N; k0 += RING_CH * NT) {
            cx<T> vv[RING_CH], uu[RING_CH];
            T tb[RING_CH];
#pragma unroll
            for (int u = 0; u < RING_CH; ++u) {
                const int k = k0 + u * NT + threadIdx.x;
                vv[u] = {T(0), T(0)};
                uu[u] = {T(0), T(0)};
                tb[u] = T(0);
                if (k < N && k <= Kl) {
                    vv[u] = Vb[(size_t)l * d.Kp + k];
                    tb[u] = d.Tb[(size_t)l * d.Kp + k];
                    if (l < d.lcorr && k <= d.klow) uu[u] = Ub[(size_t)l * (d.klow + 1) + k];
                }
            }
#pragma unroll
            for (int u = 0; u < RING_CH; ++u) {
                const int k = k0 + u * NT + threadIdx.x;
                if (k >= N) continue;
                cx<T> v = {T(0), T(0)};
                if (k <= Kl) {
                    v = mul_ipow(vv[u] * tb[u], (4 - (k & 3)) & 3);
                    if (l < d.lcorr && k <= d.klow) v = v + uu[u] * invN;
                }
                buf[lds_phys<RING_PAD<T>>(i * N + k)] = v;
            }
        }
    }
    __syncthreads();
    ring_fft(d, l, buf, N, logN, nb, true);
    const int off = d.ringOff[l];
    for (int si0 = 0; si0 < N / 2; si0 += RING_CH * NT) {
        // the chunk's point phases and destination slots, loaded together before its stores
        cx<T> phq[RING_CH];
        size_t kq[RING_CH];
#pragma unroll
        for (int u = 0; u < RING_CH; ++u) {
            const int si = si0 + u * NT + threadIdx.x;
            phq[u] = {T(0), T(0)};
            kq[u] = 0;
            if (si < N / 2) {
                phq[u] = d.ph[off + si];
                kq[u] = d.binned ? (size_t)d.ringBin[off + si] : (size_t)(off + si);
            }
        }
#pragma unroll
        for (int u = 0; u < RING_CH; ++u) {
            const int si = si0 + u * NT + threadIdx.x;
            if (si >= N / 2) continue;
            const int s = si - N / 4;
            const cx<T> ph = conjg(phq[u]);
            cx<T>* dst = Pol + kq[u] * B + b0;
            // transpose of the conjugate-symmetric fill, then of the point phase
            auto sample = [&](int i) {
                const int bo = i * N;
                const cx<T> a = buf[lds_phys<RING_PAD<T>>(bo + (s < 0 ? s + N : s))];
                const cx<T> c = buf[lds_phys<RING_PAD<T>>(bo + s + N / 2)];
                return cmul(a + conjg(c), ph);
            };
            int i = 0;
            if constexpr (sizeof(T) == 4) {
                // FP32 pairs of images as one 16-byte store (the bin-order slots
                // scatter the samples: one store instruction per pair, not two)
                if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0)
                    for (; i + 1 < nb; i += 2) {
                        const cx<T> v0 = sample(i), v1 = sample(i + 1);
                        *reinterpret_cast<float4*>(dst + i) = make_float4(v0.x, v0.y, v1.x, v1.y);
                    }
            }
            for (; i < nb; ++i) dst[i] = sample(i);
        }
    }
}

// The image groups of one ring write disjoint parts of the same Pol rows; with
// a ring count that is a multiple of the XCD count, all groups of ring l run
// back to back on XCD l mod 8, so those partial rows meet in one L2 before
// they are written back (rings stay spread round-robin over the XCDs).
template <typename T, int WMAX>
__global__ __launch_bounds__(NT) void ring_adj(Dev<T> d, const cx<T>* V, const cx<T>* Ulow, cx<T>* Pol, int B, int G,
                                               size_t ws_img)
{
    Blk bk = blk_plain();
    if (gridDim.y % NUM_XCD == 0) {
        const int lin = blockIdx.x + gridDim.x * blockIdx.y;
        const int xcd = lin % NUM_XCD, slot = lin / NUM_XCD, ng = gridDim.x;
        bk.x = slot % ng;
        bk.y = (slot / ng) * NUM_XCD + xcd;
    }
    ring_adj_body<T, WMAX>(d, bk, V, Ulow, Pol, B, G, ws_img);
}

// Transpose of the gather.  Each wave owns an 8 x 8 tile of cells of the
// extended half grid (one cell per lane) and BC images.  A sample at grid
// position (x, y) feeds cell (gx, gy) exactly when gx - ceil(x - w/2) lies in
// [0, w) and (gy - ceil(y - w/2)) mod Ng lies in [0, w) -- the gather's own tap
// rule -- so every sample that can feed the tile lies in the tile's box
// widened by w/2 (plus half a cell).  The lanes first compute, one ring per
// lane, the interval of sample angles where the ring crosses that box (asin of
// the box's y-band intersected with acos of its x-band); then the whole wave
// walks those samples in lockstep: position and the BC image values of the
// current sample are the same for every lane (scalar loads, one cache line),
// each lane tests the tap rule for its own cell and accumulates weight *
// value.  No atomics; a fixed summation order per cell.
template <typename T, int W, int BC, bool STAGED>
__device__ __forceinline__ void spread_tiles_body(const Dev<T>& d, Blk bk, const cx<T>* Pol, int B, cx<T>* E, size_t ws_img)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // staging slots (dynamic LDS, spread_tiles_lds bytes): 64 positions and
    // 64 * BC values per wave
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    cx<T>* st_pos = lds + wave * 64;
    cx<T>* st_val = lds + 4 * 64 + wave * 64 * BC;
    int bxt, byt;
    bxt = bk.x;
    byt = bk.y;
    const int tx0 = bxt * 16 + (wave & 1) * 8;   // first column of the wave's tile
    const int ty0 = byt * 16 + (wave >> 1) * 8;  // first row
    const int e = tx0 + (lane & 7), gy = ty0 + (lane >> 3);
    const int b0 = bk.z * BC;
    const int nb = min(BC, B - b0);
    const int Ng = d.Ng, mask = Ng - 1;
    const bool valid = e < d.Ew && gy < Ng;
    const int gx = e - d.hw;
    const T hwf = T(0.5) * T(W), tw_ = T(2) / T(W);
    const T rstep = d.half * d.dlam;  // ring spacing in cells
    const T TWO_PI = T(6.283185307179586);
    cx<T> acc[BC];
#pragma unroll
    for (int k = 0; k < BC; ++k) acc[k] = {T(0), T(0)};
    if (ty0 < Ng && tx0 < d.Ew) {
        const int gys0 = ty0 < Ng / 2 ? ty0 : ty0 - Ng;  // signed first row (tiles never straddle Ng/2)
        const int gxf = tx0 - d.hw;
        for (int wrap = 0; wrap < 2; ++wrap) {
            int ys = gys0;
            if (wrap) {
                if (gys0 > -Ng / 2 + W + 2 && gys0 + 8 < Ng / 2 - W - 2) break;
                ys = gys0 > 0 ? gys0 - Ng : gys0 + Ng;
            }
            const T xa = max(T(gxf) - hwf - T(0.5), T(0)), xb = T(gxf + 7) + hwf + T(0.5);
            const T ya = T(ys) - hwf - T(0.5), yb = T(ys + 7) + hwf + T(0.5);
            if (xb <= T(0)) continue;
            const T dy = ya > T(0) ? ya : (yb < T(0) ? -yb : T(0));
            const T rmin = sqrt_t(xa * xa + dy * dy);
            const T rmax = sqrt_t(xb * xb + max(ya * ya, yb * yb));
            const int l0 = max(0, (int)(rmin / rstep) - 1);
            const int l1 = min(d.L - 1, (int)(rmax / rstep) + 1);
            for (int rb = l0; rb <= l1; rb += 64) {
                // this lane's ring: sample-index intervals [u_lo, u_hi] and [v_lo, v_hi]
                const int l = rb + lane;
                int u_lo = 1, u_hi = 0, v_lo = 1, v_hi = 0;
                if (l <= l1) {
                    const int N = d.ringN[l], q4 = N >> 2, off = d.ringOff[l] + q4;
                    const T rho = d.lam[l] * d.half;
                    if (rho <= T(0)) {
                        u_lo = off - q4;
                        u_hi = off + q4 - 1;
                    } else if (rho >= rmin - T(1) && rho <= rmax + T(1)) {
                        const T f = T(N) / TWO_PI;
                        const T pya = asin(max(T(-1), min(T(1), ya / rho)));
                        const T pyb = asin(max(T(-1), min(T(1), yb / rho)));
                        const T pxl = acos(max(T(-1), min(T(1), xb / rho)));
                        const T pxh = acos(max(T(-1), min(T(1), xa / rho)));
                        const T a0 = max(pya, pxl), a1 = min(pyb, pxh);      // upper branch of the x-band
                        const T c0 = max(pya, -pxh), c1 = min(pyb, -pxl);    // lower branch
                        int s0 = 1, s1 = 0, t0 = 1, t1 = 0;
                        if (a0 <= a1) {
                            s0 = max(-q4, (int)ceil_t(a0 * f - T(0.05)));
                            s1 = min(q4 - 1, (int)floor(a1 * f + T(0.05)));
                        }
                        if (c0 <= c1) {
                            t0 = max(-q4, (int)ceil_t(c0 * f - T(0.05)));
                            t1 = min(q4 - 1, (int)floor(c1 * f + T(0.05)));
                        }
                        if (s0 <= s1 && t0 <= t1 && t1 >= s0 - 1 && t0 <= s1 + 1) {  // touching: merge
                            s0 = min(s0, t0);
                            s1 = max(s1, t1);
                            t0 = 1;
                            t1 = 0;
                        }
                        u_lo = off + s0; u_hi = off + s1;
                        v_lo = off + t0; v_hi = off + t1;
                    }
                }
                const int nr = min(64, l1 - rb + 1);
                for (int r = 0; r < nr; ++r) {
                    for (int part = 0; part < 2; ++part) {
                        const int plo = __builtin_amdgcn_readlane(part ? v_lo : u_lo, r);
                        const int phi = __builtin_amdgcn_readlane(part ? v_hi : u_hi, r);
                        if (plo > phi) continue;
                        if constexpr (STAGED) {
                            // up to 64 samples at a time: lane j stages sample base + j (its
                            // position and BC image values, coalesced vector loads) in the
                            // wave's LDS slots, then the wave walks them in lockstep reading
                            // LDS (uniform addresses: broadcast).  Only this wave touches its
                            // slots, so ordering within the wave is all that is needed.
                            for (int base = plo; base <= phi; base += 64) {
                                const int cnt = min(64, phi - base + 1);
                                __builtin_amdgcn_wave_barrier();
                                if (lane < cnt) {
                                    const cx<T>* src = Pol + (size_t)(base + lane) * B + b0;
                                    st_pos[lane] = d.pos[base + lane];
#pragma unroll
                                    for (int k = 0; k < BC; ++k) st_val[lane * BC + k] = src[k];
                                }
                                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                                __builtin_amdgcn_wave_barrier();
                                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 4
                                for (int j = 0; j < cnt; ++j) {
                                    const cx<T> q = st_pos[j];
                                    const int gx0 = (int)ceil_t(q.x - hwf);
                                    const int gy0 = (int)ceil_t(q.y - hwf);
                                    const int jx = gx - gx0;
                                    const int jy = (gy - gy0) & mask;
                                    if (valid && (unsigned)jx < (unsigned)W && jy < W) {
                                        const T wgt = es_w(q.x - T(gx0 + jx), tw_, d.beta, d.beta_l2e) *
                                                      es_w(q.y - T(gy0 + jy), tw_, d.beta, d.beta_l2e);
#pragma unroll
                                        for (int k = 0; k < BC; ++k) acc[k] = acc[k] + st_val[j * BC + k] * wgt;
                                    }
                                }
                            }
                            continue;
                        }
                        // samples are walked with their position and image values loaded one
                        // sample ahead (scalar loads complete in any order, so each wait covers
                        // everything outstanding: the loads for sample p + 1 are issued right
                        // after the wait for sample p and overlap its arithmetic).  Entries past
                        // the batch are padding or the next point's values and only reach
                        // accumulators that are never stored.
                        cx<T> qn = d.pos[plo];
                        cx<T> vn[BC];
                        {
                            const cx<T>* src = Pol + (size_t)plo * B + b0;
#pragma unroll
                            for (int k = 0; k < BC; ++k) vn[k] = src[k];
                        }
                        for (int p = plo; p <= phi; ++p) {
                            const cx<T> q = qn;
                            cx<T> val[BC];
#pragma unroll
                            for (int k = 0; k < BC; ++k) val[k] = vn[k];
                            if (p < phi) {
                                qn = d.pos[p + 1];
                                const cx<T>* src = Pol + (size_t)(p + 1) * B + b0;
#pragma unroll
                                for (int k = 0; k < BC; ++k) vn[k] = src[k];
                            }
                            const int gx0 = (int)ceil_t(q.x - hwf);
                            const int gy0 = (int)ceil_t(q.y - hwf);
                            const int jx = gx - gx0;
                            const int jy = (gy - gy0) & mask;
                            if (valid && (unsigned)jx < (unsigned)W && jy < W) {
                                const T wgt = es_w(q.x - T(gx0 + jx), tw_, d.beta, d.beta_l2e) *
                                              es_w(q.y - T(gy0 + jy), tw_, d.beta, d.beta_l2e);
#pragma unroll
                                for (int k = 0; k < BC; ++k) acc[k] = acc[k] + val[k] * wgt;
                            }
                        }
                    }
                }
            }
        }
    }
    if (valid) {
#pragma unroll
        for (int k = 0; k < BC; ++k)
            if (k < nb) {
                cx<T>* Eb = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(E) + (size_t)(b0 + k) * ws_img);
                Eb[(size_t)gy * d.Ep + e] = acc[k];
            }
    }
}

// Tiles walk very different sample counts: the rows of tiles next to y = 0
// (block rows 0 and gridDim.y - 1, the two sides of the periodic grid) hold the
// densest, smallest rings.  Blocks are therefore dispatched in the row order
// 0, last, 1, last - 1, ... (hardware order, no XCD remapping), so that the
// longest walks start first instead of last.
template <typename T, int W, int BC, bool STAGED>
__global__ __launch_bounds__(NT) void spread_tiles(Dev<T> d, const cx<T>* Pol, int B, cx<T>* E, size_t ws_img)
{
    Blk bk = blk_plain();
    const int k = bk.y;
    bk.y = (k & 1) ? (int)gridDim.y - 1 - (k >> 1) : (k >> 1);
    spread_tiles_body<T, W, BC, STAGED>(d, bk, Pol, B, E, ws_img);
}

// Dynamic LDS bytes of spread_tiles with image group bc (element size cs).
__host__ __device__ constexpr size_t spread_tiles_lds(bool staged, int bc, size_t cs)
{
    return staged ? cs * 4 * 64 * (size_t)(bc + 1) : 0;
}

// ---------------------------------------------------------------------------
// FP32 transpose of the gather over samples sorted by bin: the bin of a sample
// is the cell of its first tap, gy0 = ceil(y - w/2) mod Ng and
// gx0 = ceil(x - w/2) (ring order within a bin).  Cell (gx, gy) receives
// exactly the samples of the bins gx0 in [gx - w + 1, gx], gy0 in
// [gy - w + 1, gy]: in each of those w bin rows, one contiguous run of slots.
// A block owns a 16 x 16 tile of cells (one per thread) and BC images.  It
// stages the runs of the tile's 21 bin rows in LDS, at most SB samples per
// pass, one row of floats per sample: its BC values (contiguous in Pol, which
// ring_adj writes in bin order for these plans) and its 2w kernel weights,
// evaluated once per staged sample: the x weight of tap k at place
// (gx0 + k) mod w, so that a cell finds its own by its column, and the y
// weights by tap.  Every lane then walks its own w runs: a lane visits only
// the ~31 samples that feed its cell, where the lockstep walk of spread_tiles
// visits the union of the tile's windows (~5x more), and spends a product of
// two staged weights and the BC multiply-adds per sample.  Summation order
// per cell: bin row, then slot, whatever the pass split; no atomics.
// The few tiles whose cells receive far more samples than the rest (the
// densest small rings, next to the origin) are done as four blocks of 8 x 8
// cells with four lanes per cell: lane k takes the slots k, k + 4, ... of
// each run, and the four partial sums are added in a fixed order, (p0 + p1)
// + (p2 + p3), so those cells differ from the one-lane order by rounding only
// and every call gives the same bits.
// ---------------------------------------------------------------------------
constexpr int SB_TILE = 16;
// samples per pass: the largest count whose rows fit four blocks in a CU's LDS
__host__ __device__ constexpr int spread_bins_cap(int bc) { return bc >= 16 ? 224 : 352; }
// floats per staged sample: 2 BC values, then w x weights and w y weights
__host__ __device__ constexpr int spread_bins_row(int bc) { return 2 * bc + 12; }
__host__ __device__ constexpr size_t spread_bins_lds(int bc)
{
    return 256 + 4 * (size_t)spread_bins_cap(bc) * (size_t)spread_bins_row(bc);
}

// TS = SB_TILE: the 16 x 16 tile (bk.x, bk.y), one lane per cell; TS = 8:
// quadrant sub (x half sub & 1, y half sub >> 1) of that tile, four lanes per cell.
template <int BC, int TS>
__device__ __forceinline__ void spread_bins_body(const Dev<float>& d, Blk bk, int sub, const cx<float>* Pol, int B,
                                                 cx<float>* E, size_t ws_img)
{
    constexpr int W = 6, NR = TS + W - 1, LPC = NT / (TS * TS);  // lanes per cell
    constexpr int SB = spread_bins_cap(BC), RW = spread_bins_row(BC), TPS = BC / 2;
    constexpr int IT = (SB * TPS + NT - 1) / NT;  // staging tasks per thread and pass
    static_assert(NR <= 32 && (LPC == 1 || LPC == 4) && LPC * TS * TS == NT && RW == 2 * BC + 2 * W && RW % 4 == 0 &&
                      NT % TPS == 0,
                  "tile and LDS layout");
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    int* s_vo = reinterpret_cast<int*>(smem_raw);            // NR + 1 run offsets (virtual index)
    int* s_gs = s_vo + 32;                                   // NR first slots
    float* s_row = reinterpret_cast<float*>(smem_raw + 256); // SB rows of RW floats
    const int tid = threadIdx.x, cell = tid / LPC, part = tid % LPC;
    const int cx_ = cell % TS, cy = cell / TS;
    const int ex0 = bk.x * SB_TILE + (sub & 1) * TS, ty0 = bk.y * SB_TILE + (sub >> 1) * TS;
    const int e = ex0 + cx_, gy = ty0 + cy;
    const int Ng = d.Ng, mask = Ng - 1, Ew = d.Ew;
    const int b0 = bk.z * BC, nb = min(BC, B - b0);
    const bool valid = e < Ew;  // Ng is a multiple of the tile
    const int gx = e - d.hw;
    const int e_lo = max(ex0 - (W - 1), 0), e_hi = min(ex0 + TS - 1, Ew - 1);
    // the runs of the tile's bin rows: first slots, and offsets by a scan in the first wave
    if (tid < 64) {
        int a = 0, len = 0;
        if (tid < NR && e_hi >= e_lo) {
            const int row = (ty0 - (W - 1) + tid) & mask;
            a = d.binStart[(size_t)row * Ew + e_lo];
            len = d.binStart[(size_t)row * Ew + e_hi + 1] - a;
        }
        int inc = len;
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (tid >= o) inc += t;
        }
        if (tid < NR) {
            s_gs[tid] = a;
            s_vo[tid + 1] = inc;
        }
        if (tid == 0) s_vo[0] = 0;
    }
    __syncthreads();
    const int S = s_vo[NR];
    // this lane's runs (virtual indices) in its bin rows q = cy .. cy + W - 1
    int lo[W], hi[W];
#pragma unroll
    for (int r = 0; r < W; ++r) {
        lo[r] = 0;
        hi[r] = 0;
        if (valid) {
            const int q = cy + r, row = (ty0 - (W - 1) + q) & mask;
            const int a = d.binStart[(size_t)row * Ew + max(e - (W - 1), 0)];
            const int b = d.binStart[(size_t)row * Ew + e + 1];
            lo[r] = s_vo[q] + a - s_gs[q];
            hi[r] = s_vo[q] + b - s_gs[q];
        }
    }
    const float hwf = 0.5f * float(W), tw_ = 2.f / float(W);
    const int rx = (gx + W) % W;          // place of this cell's x weight (gx >= -w/2)
    const int mth = tid % TPS;            // image pair of this thread's staging tasks
    float4 acc[TPS];
#pragma unroll
    for (int m = 0; m < TPS; ++m) acc[m] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int pv = 0; pv < S; pv += SB) {
        const int cnt = min(SB, S - pv);
        __syncthreads();  // the previous pass's walk is done with the rows
        // staging: task (v, mth) loads image pair mth of staged sample v and
        // evaluates weights mth, mth + TPS, ... of its 2w; the loads of all
        // tasks are issued before any is used
        float4 xv[IT];
        cx<float> pp[IT];
        int q = 0;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int v = tid / TPS + it * (NT / TPS);
            xv[it] = make_float4(0.f, 0.f, 0.f, 0.f);
            pp[it] = {0.f, 0.f};
            if (v < cnt) {
                const int vv = pv + v;
                while (s_vo[q + 1] <= vv) ++q;
                const size_t g = (size_t)(s_gs[q] + vv - s_vo[q]);
                const cx<float>* src = Pol + g * B + b0 + 2 * mth;
                if (2 * mth < nb) { xv[it].x = src[0].x; xv[it].y = src[0].y; }
                if (2 * mth + 1 < nb) { xv[it].z = src[1].x; xv[it].w = src[1].y; }
                pp[it] = d.binPos[g];
            }
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int v = tid / TPS + it * (NT / TPS);
            if (v < cnt) {
                float* row = s_row + v * RW;
                reinterpret_cast<float4*>(row)[mth] = xv[it];
                const int gx0 = (int)ceil_t(pp[it].x - hwf), gy0 = (int)ceil_t(pp[it].y - hwf);
#pragma unroll
                for (int k = mth; k < 2 * W; k += TPS) {
                    if (k < W) row[2 * BC + (gx0 + k + W) % W] = es_w(pp[it].x - float(gx0 + k), tw_, d.beta, d.beta_l2e);
                    else row[2 * BC + k] = es_w(pp[it].y - float(gy0 + k - W), tw_, d.beta, d.beta_l2e);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < W; ++r) {
            // the binning puts every staged sample of this run inside the
            // cell's stencil: x tap gx - gx0 and y tap w - 1 - r
            const int a = max(lo[r], pv) - pv, b = min(hi[r], pv + cnt) - pv;
            for (int j = a + part; j < b; j += LPC) {
                const float* row = s_row + j * RW;
                float4 val[TPS];
#pragma unroll
                for (int m = 0; m < TPS; ++m) val[m] = reinterpret_cast<const float4*>(row)[m];
                const float wgt = row[2 * BC + rx] * row[2 * BC + W + (W - 1 - r)];
#pragma unroll
                for (int m = 0; m < TPS; ++m) {
                    acc[m].x += val[m].x * wgt;
                    acc[m].y += val[m].y * wgt;
                    acc[m].z += val[m].z * wgt;
                    acc[m].w += val[m].w * wgt;
                }
            }
        }
    }
    if constexpr (LPC > 1) {
        // the cell's LPC = 4 adjacent lanes: (p0 + p1) + (p2 + p3) on every lane
#pragma unroll
        for (int o = 1; o < LPC; o <<= 1)
#pragma unroll
            for (int m = 0; m < TPS; ++m) {
                acc[m].x += __shfl_xor(acc[m].x, o, 64);
                acc[m].y += __shfl_xor(acc[m].y, o, 64);
                acc[m].z += __shfl_xor(acc[m].z, o, 64);
                acc[m].w += __shfl_xor(acc[m].w, o, 64);
            }
    }
    if (valid) {
#pragma unroll
        for (int m = 0; m < TPS; ++m) {
            if (m % LPC != part) continue;  // one lane of the cell stores each image pair
            const cx<float> lo2[2] = {{acc[m].x, acc[m].y}, {acc[m].z, acc[m].w}};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = 2 * m + h;
                if (k < nb) {
                    cx<float>* Eb = reinterpret_cast<cx<float>*>(reinterpret_cast<char*>(E) + (size_t)(b0 + k) * ws_img);
                    Eb[(size_t)gy * d.Ep + e] = lo2[h];
                }
            }
        }
    }
}

// Dispatch order: block lin does the tile of table entry and image group
// table_block(lin) of the plan's table spOrder (tx | ty << 12 | quadrant << 24
// | split << 26; -1: nothing).  Per XCD the table holds a contiguous run of
// tiles (their halos shared through its L2) taken longest first by a cost
// estimate, so that the last blocks to start are short ones; a tile that
// would end after the balanced share of a block slot appears as its four
// split quadrants (spread_order, xcd_table).
template <int BC>
__global__ __launch_bounds__(NT) void spread_bins(Dev<float> d, const cx<float>* Pol, int B, cx<float>* E, size_t ws_img,
                                                  int nz)
{
    int entry, z;
    table_block(blockIdx.x, nz, entry, z);
    const int t = d.spOrder[entry];
    if (t < 0) return;  // padding of a shorter XCD list
    const Blk bk = {t & 0xfff, (t >> 12) & 0xfff, z, 0};
    if (t >> 26) spread_bins_body<BC, SB_TILE / 2>(d, bk, (t >> 24) & 3, Pol, B, E, ws_img);
    else spread_bins_body<BC, SB_TILE>(d, bk, 0, Pol, B, E, ws_img);
}

template <typename T>
__device__ __forceinline__ void cols_adj_body(const Dev<T>& d, Blk bk, const cx<T>* E, cx<T>* R, size_t ws_img)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    int bx_, b;
    bx_ = bk.x;
    b = bk.y;
    const int CW = d.colsCW, lcw = d.colsLCW, x0 = bx_ * CW;
    const int Ng = d.Ng, n = d.n;
    const cx<T>* Eb = reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(E) + (size_t)b * ws_img);
    cx<T>* Rb = reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(R) + (size_t)b * ws_img);
    for (int i = threadIdx.x; i < CW * Ng; i += blockDim.x) {
        int gy = i >> lcw, c = i & (CW - 1);
        int gx = x0 + c;
        cx<T> v = {T(0), T(0)};
        if (gx < d.Rw) {
            v = Eb[(size_t)gy * d.Ep + gx + d.hw];
            int gym = (Ng - gy) & (Ng - 1);
            if (gx >= 1 && gx <= d.hw) v = v + conjg(Eb[(size_t)gym * d.Ep + d.hw - gx]);
            if (gx >= Ng / 2 - d.hw && gx <= Ng / 2 - 1) v = v + conjg(Eb[(size_t)gym * d.Ep + d.hw + Ng - gx]);
        }
        buf[c * Ng + gy] = v;
    }
    __syncthreads();
    lds_fft(buf, d.logNg, CW, Ng, d.tw, d.logNmax, true, d.fft_lr, d.tw_table);
    for (int i = threadIdx.x; i < CW * n; i += blockDim.x) {
        int p = i >> lcw, c = i & (CW - 1);
        int gx = x0 + c;
        if (gx < d.Rw) Rb[(size_t)p * d.Rw + gx] = buf[c * Ng + ((p - n / 2 + Ng) & (Ng - 1))];
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void cols_adj(Dev<T> d, const cx<T>* E, cx<T>* R, size_t ws_img)
{
    cols_adj_body<T>(d, blk_xcd(), E, R, ws_img);
}

// Sum of one double per thread over the block in a fixed order (lane
// butterflies within each wave, then the waves in index order); every thread
// returns the total.  Must be reached by all threads of the block.
__device__ __forceinline__ double block_sum_fixed(double v)
{
    __shared__ double wsum[NT / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wave = threadIdx.x >> 6;
    __syncthreads();  // wsum may still be read by a previous call
    if ((threadIdx.x & 63) == 0) wsum[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += wsum[w];
    return t;
}

template <typename T>
__device__ __forceinline__ void rows_adj_body(const Dev<T>& d, Blk bk, const cx<T>* R, T* f, long fstride, size_t ws_img)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    int bx_, b;
    bx_ = bk.x;
    b = bk.y;
    const int p1 = 2 * bx_, p2 = p1 + 1;
    const int Ng = d.Ng, n = d.n, hN = Ng / 2;
    const cx<T>* Rb = reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(R) + (size_t)b * ws_img);
    T* fb = f + (size_t)b * fstride;
    const bool has2 = p2 < n;
    for (int g = threadIdx.x; g < Ng; g += blockDim.x) {
        cx<T> xa, xb;
        if (g == 0 || g == hN) {
            xa = {Rb[(size_t)p1 * d.Rw + g].x, T(0)};
            xb = {has2 ? Rb[(size_t)p2 * d.Rw + g].x : T(0), T(0)};
        } else if (g < hN) {
            xa = Rb[(size_t)p1 * d.Rw + g] * T(0.5);
            xb = has2 ? Rb[(size_t)p2 * d.Rw + g] * T(0.5) : cx<T>{T(0), T(0)};
        } else {
            xa = conjg(Rb[(size_t)p1 * d.Rw + (Ng - g)]) * T(0.5);
            xb = has2 ? conjg(Rb[(size_t)p2 * d.Rw + (Ng - g)]) * T(0.5) : cx<T>{T(0), T(0)};
        }
        buf[g] = {xa.x - xb.y, xa.y + xb.x};
    }
    __syncthreads();
    lds_fft(buf, d.logNg, 1, 0, d.tw, d.logNmax, true, d.fft_lr, d.tw_table);
    const T s1 = d.Dq[p1] * d.pre_scale * d.adj_scale;
    const T s2 = has2 ? d.Dq[p2] * d.pre_scale * d.adj_scale : T(0);
    if (!d.ubp) {
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            cx<T> v = buf[(q - n / 2 + Ng) & (Ng - 1)];
            put_image(d, fb, b, p1, q, in_mask(d, p1, q) ? v.x * d.Dq[q] * s1 : T(0));
            if (has2) put_image(d, fb, b, p2, q, in_mask(d, p2, q) ? v.y * d.Dq[q] * s2 : T(0));
        }
        return;
    }
    // back-projection of the approximate inverse: v everywhere, and this
    // block's sum of v over Omega \ Omega_0 (fixed order: lanes, waves)
    double acc = 0.0;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        cx<T> v = buf[(q - n / 2 + Ng) & (Ng - 1)];
        const T v1 = v.x * d.Dq[q] * s1, v2 = v.y * d.Dq[q] * s2;
        fb[(size_t)p1 * n + q] = v1;
        if (in_annulus(d, p1, q)) acc += (double)v1;
        if (has2) {
            fb[(size_t)p2 * n + q] = v2;
            if (in_annulus(d, p2, q)) acc += (double)v2;
        }
    }
    const double tot = block_sum_fixed(acc);
    if (threadIdx.x == 0) {
        double* pb = reinterpret_cast<double*>(reinterpret_cast<char*>(d.part) + (size_t)b * ws_img);
        pb[bx_] = tot;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void rows_adj(Dev<T> d, const cx<T>* R, T* f, long fstride, size_t ws_img)
{
    rows_adj_body<T>(d, blk_xcd(), R, f, fstride, ws_img);
}

// Last steps of the approximate inverse (Alg. 3): the constant C of eq.
// E:silly_integral, C = -(sum of v over the pixel centres of Omega \ Omega_0)
// / (their count), from rows_adj's per-block partial sums, then
// f = v + C on Omega_0 and 0 elsewhere.  Every block reduces the same
// partials in the same order, so all blocks use the same C.
template <typename T>
__global__ __launch_bounds__(NT) void ubp_apply(Dev<T> d, T* f, long fstride, int nparts, double inv_count,
                                                size_t ws_img)
{
    const int b = blockIdx.y;
    const double* pb = reinterpret_cast<const double*>(reinterpret_cast<const char*>(d.part) + (size_t)b * ws_img);
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += NT) acc += pb[i];
    const T C = (T)(-block_sum_fixed(acc) * inv_count);
    T* fb = f + (size_t)b * fstride;
    const int n = d.n;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n * n; i += gridDim.x * NT) {
        const int p = i / n, q = i - p * n;
        fb[i] = in_mask(d, p, q) ? fb[i] + C : T(0);
    }
}

// ---------------------------------------------------------------------------
// Measurement operator B of eq. E:real_meas on detector traces (time-major
// nt x m): B g = D(e^{-gamma t} g), D the Fourier filter eta in t applied to
// each trace zero-extended to N = 2^ceil(log2(2 nt)) samples and cut back to
// nt; B* g = e^{-gamma t} D_conj(eta) g.  One block owns CW adjacent
// detectors (coalesced row segments) and packs them in pairs as the real and
// imaginary parts of CW/2 complex sequences: since eta(-xi) = conj(eta(xi)),
// filtering the packed sequence by eta on the whole DFT circle filters both
// real traces at once.
// ---------------------------------------------------------------------------
template <typename T>
struct FiltDev {
    int nt, m, N, logN, CW, lcw, fft_lr;
    const cx<T>* H;    // N: eta on the DFT circle (conjugate-symmetric), 1/N folded in
    const cx<T>* tw;   // N: e^{-2 pi i k / N}
    const T* att;      // nt: e^{-gamma t_j}
};

template <typename T>
__global__ __launch_bounds__(NT) void trace_filter(FiltDev<T> d, const T* in, long istride, T* out, long ostride,
                                                   int adjoint)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const Blk bk = blk_xcd();
    const int i0 = bk.x * d.CW, b = bk.y;
    const int N = d.N, CW = d.CW, np = CW >> 1;
    const T* ib = in + (size_t)b * istride;
    T* ob = out + (size_t)b * ostride;
    T* bre = reinterpret_cast<T*>(buf);
    for (int idx = threadIdx.x; idx < CW * N; idx += NT) {
        const int j = idx >> d.lcw, c = idx & (CW - 1);
        T v = T(0);
        if (j < d.nt && i0 + c < d.m) {
            v = ib[(size_t)j * d.m + i0 + c];
            if (!adjoint) v *= d.att[j];
        }
        bre[2 * ((c >> 1) * N + j) + (c & 1)] = v;   // pair c/2: even -> real, odd -> imaginary
    }
    __syncthreads();
    const int per = max(1, min(np, FFT_BLOCK_POINTS >> d.logN));   // sequences per lds_fft call
    for (int q = 0; q < np; q += per) lds_fft(buf + q * N, d.logN, min(per, np - q), N, d.tw, d.logN, false, d.fft_lr, true);
    for (int k = threadIdx.x; k < N; k += NT) {
        cx<T> h = d.H[k];
        if (adjoint) h.y = -h.y;
        for (int q = 0; q < np; ++q) buf[q * N + k] = cmul(buf[q * N + k], h);
    }
    __syncthreads();
    for (int q = 0; q < np; q += per) lds_fft(buf + q * N, d.logN, min(per, np - q), N, d.tw, d.logN, true, d.fft_lr, true);
    for (int idx = threadIdx.x; idx < CW * d.nt; idx += NT) {
        const int j = idx >> d.lcw, c = idx & (CW - 1);
        if (i0 + c >= d.m) continue;
        T v = bre[2 * ((c >> 1) * N + j) + (c & 1)];
        if (adjoint) v *= d.att[j];
        ob[(size_t)j * d.m + i0 + c] = v;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// plan object and C ABI
// ---------------------------------------------------------------------------
struct pat_plan_s {
    pat::HostPlan H;
    int max_batch = 1;
    int device = 0;
    size_t ws_img = 0;                    // workspace bytes per image (pat_workspace_size / batch)
    size_t ws_stride = 0;                 // bytes between per-image slices; the batch's sample array follows them
    size_t offR, offE, offV, offG, offU, offC, offP;  // byte offsets inside one image's workspace
    double inv_count = 0.0;               // 1 / (pixel centres in Omega \ Omega_0), 0 if none
    std::vector<void*> allocs;
    size_t table_bytes = 0;
    Dev<float> df{};
    Dev<double> dd{};
    // launch-shape choices (defaults from LDS limits; replaced by the autotuner's)
    int cols_cw = 1, dct_cw = 1, ring_g = 1, spread_bc = 16, fft_lr = 4, tw_table = 0, spread_staged = 1;
    int dct_wave_on = 1;                  // 1: use dct_wave where the plan's lengths allow it
    int wave_fft_on = 1;                  // 1: wave forms of the row / column / synthesis FFT kernels
    int bin_ok = 0;                       // 1: the bin tables of spread_bins exist (FP32 plans)
    int tuned = 0;                        // 1: measured now, 2: read from the tuning cache
    double tuned_ms = 0.0;
    // optional per-stage timing with HIP events recorded on the launch stream
    bool timing = false;
    unsigned timing_mask = ~0u;            // stages whose launches get events
    std::vector<hipEvent_t> ev_pool;       // pairs (start, end)
    std::vector<int> ev_stage;             // stage of each recorded pair
    size_t ev_used = 0;
};

struct pat_filter_s {
    int nt = 0, m = 0, N = 0, cw = 2, device = 0;
    pat_dtype dt = PAT_F32;
    std::vector<void*> allocs;
    FiltDev<float> df{};
    FiltDev<double> dd{};
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Row pitch of E in cells: the extended width Ew rounded up to 16, so that a
// tile's row of 16 cells is whole cache lines.
int e_pitch(const pat::Params& P) { return (P.Ew + 15) / 16 * 16; }

constexpr size_t SPREAD_PAD = 16;  // >= the spread's image group BC

void layout(pat_plan_s* p)
{
    const pat::Params& P = p->H.P;
    size_t cs = (P.dt == PAT_F64) ? 16 : 8;
    size_t o = 0;
    p->offR = o; o = align256(o + cs * (size_t)P.n * P.Rw);
    p->offE = o; o = align256(o + cs * (size_t)P.Ng * e_pitch(P));
    p->offV = o; o = align256(o + cs * (size_t)P.L * P.Kp);
    p->offG = o; o = align256(o + cs * (size_t)P.nt * P.Kp);
    p->offU = o; o = align256(o + cs * (size_t)P.lcorr * (P.klow + 1));
    p->offC = o; o = align256(o + sizeof(double) * (size_t)((P.n + 1) / 2));  // inverse: rows_adj partial sums
    p->ws_stride = o;
    // the adjoint's half-ring samples, image-minor: B * npts values after the B slices
    // (plus SPREAD_PAD values: the spread reads whole groups of images per sample)
    p->offP = 0;
    p->ws_img = o + align256(cs * ((size_t)P.npts + SPREAD_PAD));
}

int lds_cols(const pat::Params& P)
{
    size_t cs = (P.dt == PAT_F64) ? 16 : 8;
    int cw = 16;
    while (cw > 1 && ((size_t)cw * P.Ng * cs > 65536 || (size_t)cw * P.Ng > FFT_BLOCK_POINTS)) cw >>= 1;
    return cw;
}

// largest number of images per ring_fwd block that fits 64 KiB of LDS (at most 4)
// LDS bytes of a ring kernel block with G images (FP32 buffers padded)
size_t ring_lds(const pat::Params& P, int G)
{
    if (P.dt == PAT_F64) return (size_t)16 * G * P.max_ring;
    return (size_t)8 * lds_phys<true>(G * P.max_ring);
}

int ring_group_max(const pat::Params& P)
{
    int g = 4;
    while (g > 1 && ring_lds(P, g) > 65536) g >>= 1;
    return g;
}

// the cosine transform's LDS: CW columns of M points, plus the stash of the
// CW input columns (max(L, nt) rows) when that still fits 64 KiB
// cosine-transform block LDS per column: the FFT buffer (M), with the one-FFT
// form also the prefix sums (M/2 + 1), and, if it fits, the stashed input.
// The one-FFT kernel also holds two NT-entry reduction arrays (static LDS),
// which count against the same 64 KiB.
size_t dct_budget(const pat::Params& P)
{
    const size_t cs = (P.dt == PAT_F64) ? 16 : 8;
    return 65536 - 2 * (size_t)NT * cs;
}

int dct_one_ok(const pat::Params& P, int cw)
{
    const size_t cs = (P.dt == PAT_F64) ? 16 : 8;
    return (size_t)cw * ((size_t)P.M + P.M / 2 + 1) * cs <= dct_budget(P) ? 1 : 0;
}

int ilog2i(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// dct_wave variant for the plan's cosine-transform length (FP32; M = 384, 768,
// 1536 or 256 .. 1024; the forward input rows must fit the M + 1 slots), 0 if none
int dw_variant(const pat::Params& P)
{
    if (P.dt != PAT_F32 || P.L > P.M + 1 || P.nt > P.M) return 0;
    const int m3 = P.m3 ? 1 : 0;
    const int logp = ilog2i(m3 ? P.M / 3 : P.M);
    const int code = (m3 << 8) | logp;
    switch (code) {
#define PAT_DW_OK(a, b) case ((a) << 8) | (b):
        PAT_DW_VARIANTS(PAT_DW_OK)
#undef PAT_DW_OK
            break;
        default: return 0;
    }
    return code;
}

// log2 of the row / column FFT length and of the angular transform length for
// the wave-form kernels (FP32, powers of two 256 .. 2048), 0 where they do not apply
int wf_rows_variant(const pat::Params& P)
{
    const int l = ilog2i(P.Ng);
    return (P.dt == PAT_F32 && (1 << l) == P.Ng && l >= 8 && l <= 11) ? l : 0;
}
int wf_synth_variant(const pat::Params& P)
{
    const int l = ilog2i(P.mf);
    return (P.dt == PAT_F32 && !P.mf3 && (1 << l) == P.mf && l >= 8 && l <= 11) ? l : 0;
}
size_t wf_lds(int logn) { return sizeof(cx<float>) * WF_WAVES * (size_t)wf_pitch(logn); }

// columns per block and dynamic LDS bytes of a dct_wave variant
int dw_columns(int code)
{
    switch (code) {
#define PAT_DW_CB(a, b) \
    case ((a) << 8) | (b): return DwShape<a, b>::CB;
        PAT_DW_VARIANTS(PAT_DW_CB)
#undef PAT_DW_CB
        default: return 1;
    }
}
size_t dw_lds(int code)
{
    switch (code) {
#define PAT_DW_LDS(a, b) \
    case ((a) << 8) | (b): return DwShape<a, b>::LDS;
        PAT_DW_VARIANTS(PAT_DW_LDS)
#undef PAT_DW_LDS
        default: return 0;
    }
}

// launches of the wave-form row / column / synthesis kernels (FP32 plans)
#define PAT_WF_SWITCH(var, KERNEL, grid, lds, ...)                         \
    switch (var) {                                                         \
        case 8: KERNEL<8><<<grid, NT, lds, st>>>(__VA_ARGS__); break;      \
        case 9: KERNEL<9><<<grid, NT, lds, st>>>(__VA_ARGS__); break;      \
        case 10: KERNEL<10><<<grid, NT, lds, st>>>(__VA_ARGS__); break;    \
        case 11: KERNEL<11><<<grid, NT, lds, st>>>(__VA_ARGS__); break;    \
        default: return PAT_EINVAL;                                        \
    }

dim3 wf_grid_rows(const Dev<float>& d, int B) { return dim3(((d.n + 1) / 2 + WF_WAVES - 1) / WF_WAVES, B); }
dim3 wf_grid_cols(const Dev<float>& d, int B) { return dim3((d.Rw + WF_WAVES - 1) / WF_WAVES, B); }
dim3 wf_grid_synth(const Dev<float>& d, int B) { return dim3(((d.nt + 1) / 2 + WF_WAVES - 1) / WF_WAVES, B); }

int launch_rows_fwd_w(const Dev<float>& d, int B, const float* f, long fs, cx<float>* R, size_t wi, hipStream_t st)
{
    PAT_WF_SWITCH(d.wfRows, rows_fwd_w, wf_grid_rows(d, B), wf_lds(d.wfRows), d, f, fs, R, wi)
    return PAT_OK;
}
int launch_rows_adj_w(const Dev<float>& d, int B, const cx<float>* R, float* f, long fs, size_t wi, hipStream_t st)
{
    PAT_WF_SWITCH(d.wfRows, rows_adj_w, wf_grid_rows(d, B), wf_lds(d.wfRows), d, R, f, fs, wi)
    return PAT_OK;
}
int launch_cols_fwd_w(const Dev<float>& d, int B, const cx<float>* R, cx<float>* E, size_t wi, hipStream_t st)
{
    PAT_WF_SWITCH(d.wfRows, cols_fwd_w, wf_grid_cols(d, B), wf_lds(d.wfRows), d, R, E, wi)
    return PAT_OK;
}
int launch_cols_adj_w(const Dev<float>& d, int B, const cx<float>* E, cx<float>* R, size_t wi, hipStream_t st)
{
    PAT_WF_SWITCH(d.wfRows, cols_adj_w, wf_grid_cols(d, B), wf_lds(d.wfRows), d, E, R, wi)
    return PAT_OK;
}
int launch_synth_fwd_w(const Dev<float>& d, int B, const cx<float>* G, float* g, long gs, size_t wi, hipStream_t st)
{
    PAT_WF_SWITCH(d.wfSynth, synth_fwd_w, wf_grid_synth(d, B), wf_lds(d.wfSynth), d, G, g, gs, wi)
    return PAT_OK;
}
int launch_synth_adj_w(const Dev<float>& d, int B, const float* g, long gs, cx<float>* G, size_t wi, hipStream_t st)
{
    PAT_WF_SWITCH(d.wfSynth, synth_adj_w, wf_grid_synth(d, B), wf_lds(d.wfSynth), d, g, gs, G, wi)
    return PAT_OK;
}

int launch_dct_wave(const Dev<float>& d, int B, const cx<float>* in, cx<float>* out, size_t wi, int adjoint,
                    hipStream_t st)
{
    switch (d.dct_wave) {
#define PAT_DW_LAUNCH(a, b) \
    case ((a) << 8) | (b): \
        if (d.sine)                                                                                                   \
            dct_wave<a, b, true><<<dim3(d.Kp / DwShape<a, b>::CB, B), NT, DwShape<a, b>::LDS, st>>>(d, in, out, wi, adjoint); \
        else                                                                                                          \
            dct_wave<a, b, false><<<dim3(d.Kp / DwShape<a, b>::CB, B), NT, DwShape<a, b>::LDS, st>>>(d, in, out, wi, adjoint); \
        break;
        PAT_DW_VARIANTS(PAT_DW_LAUNCH)
#undef PAT_DW_LAUNCH
        default: return PAT_EINVAL;
    }
    return PAT_OK;
}

size_t dct_base(const pat::Params& P, int cw)
{
    return (size_t)P.M + (dct_one_ok(P, cw) ? (size_t)(P.M / 2 + 1) : 0);
}

int dct_stash_ok(const pat::Params& P, int cw)
{
    const size_t cs = (P.dt == PAT_F64) ? 16 : 8;
    return (size_t)cw * (dct_base(P, cw) + std::max(P.L, P.nt)) * cs <= dct_budget(P) ? 1 : 0;
}

size_t dct_lds(const pat::Params& P, int cw)
{
    const size_t cs = (P.dt == PAT_F64) ? 16 : 8;
    return cs * cw * (dct_base(P, cw) + (dct_stash_ok(P, cw) ? std::max(P.L, P.nt) : 0));
}

// points one lds_fft call holds: FFT_REGS per thread and pass, i.e. 16 NT for
// power-of-two lengths, 15 NT when the radix-3 pass is needed
int fft_points(const pat::Params& P) { return P.m3 ? (FFT_REGS / 3) * 3 * NT : FFT_BLOCK_POINTS; }

int lds_dct(const pat::Params& P)
{
    size_t cs = (P.dt == PAT_F64) ? 16 : 8;
    int cw = 16;
    while (cw > 1 && ((size_t)cw * P.M * cs > 65536 || cw * P.M > fft_points(P))) cw >>= 1;
    return cw;
}

// Dispatch table of a tiled kernel from its tiles' estimated costs (in
// row-major tile order).  The hardware deals consecutive workgroups to the
// NUM_XCD XCDs in turn, so the table holds one list per XCD, interleaved:
// entry j * NUM_XCD + x is the j-th tile of XCD x.  Each XCD receives one
// contiguous run of the row-major order (runs of equal total cost), so that
// neighbouring tiles, which stage the same halo, read it through one L2.
// Within its list an XCD takes its tiles by decreasing cost, dispatched in a
// simulation of its `slots` concurrent blocks to the slot that frees first;
// with `split` set, a tile that would end after split_at times the balanced
// share of a slot is listed as its four quadrants instead (cost / 4 x 1.2
// each).  Lists are padded to equal length with -1 (an empty block).
// Entries: tx | ty << 12 | quadrant << 24 | split << 26.
std::vector<int> xcd_table(const std::vector<std::pair<double, int>>& tiles, int slots, bool split, double split_at)
{
    double total = 0;
    for (const auto& t : tiles) total += t.first;
    std::vector<std::vector<int>> lists(NUM_XCD);
    size_t next = 0;
    double done = 0;
    for (int x = 0; x < NUM_XCD; ++x) {
        // this XCD's run: tiles until the cumulative cost reaches (x + 1) / NUM_XCD of the total
        std::vector<std::pair<double, int>> mine;
        const double upto = total * (x + 1) / NUM_XCD;
        while (next < tiles.size() && (x == NUM_XCD - 1 || done + 0.5 * tiles[next].first <= upto)) {
            done += tiles[next].first;
            mine.push_back(tiles[next++]);
        }
        std::sort(mine.begin(), mine.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
            return a.first != b.first ? a.first > b.first : a.second < b.second;
        });
        double part = 0;
        for (const auto& t : mine) part += t.first;
        const double limit = split_at * part / std::max(slots, 1);
        std::priority_queue<double, std::vector<double>, std::greater<double>> slot_free;
        for (int k = 0; k < std::max(slots, 1); ++k) slot_free.push(0.0);
        auto dispatch = [&](double c) {
            const double t = slot_free.top();
            slot_free.pop();
            slot_free.push(t + c);
        };
        for (const auto& t : mine) {
            if (split && slot_free.top() + t.first > limit) {
                for (int qd = 0; qd < 4; ++qd) {
                    lists[x].push_back(t.second | qd << 24 | 1 << 26);
                    dispatch(t.first / 4 * 1.2);
                }
            } else {
                lists[x].push_back(t.second);
                dispatch(t.first);
            }
        }
    }
    size_t len = 0;
    for (const auto& l : lists) len = std::max(len, l.size());
    std::vector<int> table(len * NUM_XCD, -1);
    for (int x = 0; x < NUM_XCD; ++x)
        for (size_t k = 0; k < lists[x].size(); ++k) table[k * NUM_XCD + x] = lists[x][k];
    return table;
}

// spread_bins over the 16 x 16 cell tiles of the Ng x Ew grid (bin table
// `start`): a tile's cost is estimated as 53 + S + 2.9 wmax, S the samples
// its bin rows stage and wmax the longest walk of its four waves (per wave,
// the sum over the w bin rows of the longest run among its 64 cells), the
// proportions of a least-squares fit of measured block durations; heavy
// tiles and the tiles of the last round are split (xcd_table).  Empty if a
// tile index does not fit its field.
constexpr double SPREAD_SPLIT = 1.1;
std::vector<int> spread_order(const pat::Params& P, const std::vector<int>& start, int slots)
{
    const int W = P.w, Ng = P.Ng, Ew = P.Ew, mask = Ng - 1, TS = 16;
    const int nx = (Ew + TS - 1) / TS, ny = Ng / TS;
    if (nx >= 4096 || ny >= 4096 || ny * TS != Ng) return {};
    auto run = [&](int row, int lo, int hi) {  // samples in bins lo..hi of a bin row
        lo = std::max(lo, 0);
        hi = std::min(hi, Ew - 1);
        return hi < lo ? 0 : start[(size_t)row * Ew + hi + 1] - start[(size_t)row * Ew + lo];
    };
    std::vector<std::pair<double, int>> tiles;
    for (int ty = 0; ty < ny; ++ty)
        for (int tx = 0; tx < nx; ++tx) {
            double S = 0, wmax = 0;
            for (int q = 0; q < TS + W - 1; ++q)
                S += run((ty * TS - (W - 1) + q) & mask, tx * TS - (W - 1), tx * TS + TS - 1);
            for (int wv = 0; wv < NT / 64; ++wv) {
                double steps = 0;
                for (int r = 0; r < W; ++r) {
                    int longest = 0;
                    for (int cy = wv * (64 / TS); cy < (wv + 1) * (64 / TS); ++cy) {
                        const int row = (ty * TS + cy - (W - 1) + r) & mask;
                        for (int cx = 0; cx < TS && tx * TS + cx < Ew; ++cx)
                            longest = std::max(longest, run(row, tx * TS + cx - (W - 1), tx * TS + cx));
                    }
                    steps += longest;
                }
                wmax = std::max(wmax, steps);
            }
            tiles.push_back({53.0 + S + 2.9 * wmax, tx | ty << 12});
        }
    return xcd_table(tiles, slots / NUM_XCD, true, SPREAD_SPLIT);
}

// gather_bins over its 16 x 16 bin tiles: a tile's cost is estimated as
// 675 + S + 573 ceil(S / NT), S the samples of its bins (one thread per
// sample, in rounds of NT), the proportions of a least-squares fit of
// measured block durations.  Entries tx | ty << 12 (xcd_table, no splits).
std::vector<int> gather_order(const pat::Params& P, const std::vector<int>& start, int slots)
{
    const int Ng = P.Ng, Ew = P.Ew, TS = 16;
    const int nx = (Ew + TS - 1) / TS, ny = Ng / TS;
    if (nx >= 4096 || ny >= 4096 || ny * TS != Ng) return {};
    std::vector<std::pair<double, int>> tiles;
    for (int ty = 0; ty < ny; ++ty)
        for (int tx = 0; tx < nx; ++tx) {
            const int e1 = std::min(tx * TS + TS, Ew);
            double S = 0;
            for (int row = ty * TS; row < ty * TS + TS; ++row)
                S += start[(size_t)row * Ew + e1] - start[(size_t)row * Ew + tx * TS];
            tiles.push_back({675.0 + S + 573.0 * std::ceil(S / NT), tx | ty << 12});
        }
    return xcd_table(tiles, slots / NUM_XCD, false, 0.0);
}

template <typename T>
int upload(pat_plan_s* p, Dev<T>& d)
{
    const pat::HostPlan& H = p->H;
    const pat::Params& P = H.P;
    auto put = [&](const void* src, size_t bytes, const void** dst) -> int {
        void* ptr = nullptr;
        if (bytes == 0) bytes = 16;
        if (hipMalloc(&ptr, bytes) != hipSuccess) return PAT_ENOMEM;
        p->allocs.push_back(ptr);
        p->table_bytes += bytes;
        if (src && hipMemcpy(ptr, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return PAT_EHIP;
        *dst = ptr;
        return PAT_OK;
    };
    auto conv = [](const std::vector<double>& v) {
        std::vector<T> o(v.size());
        for (size_t i = 0; i < v.size(); ++i) o[i] = (T)v[i];
        return o;
    };
    std::vector<T> Dq = conv(H.Dq), lam = conv(H.lam), Tb = conv(H.Tb), Mk = conv(H.Mk), ph = conv(H.phase),
                   tw = conv(H.tw);
    int rc;
    if ((rc = put(Dq.data(), Dq.size() * sizeof(T), (const void**)&d.Dq))) return rc;
    if ((rc = put(lam.data(), lam.size() * sizeof(T), (const void**)&d.lam))) return rc;
    if ((rc = put(H.ringN.data(), H.ringN.size() * sizeof(int), (const void**)&d.ringN))) return rc;
    if ((rc = put(H.ringLog.data(), H.ringLog.size() * sizeof(int), (const void**)&d.ringLog))) return rc;
    if ((rc = put(H.ringOff.data(), H.ringOff.size() * sizeof(int), (const void**)&d.ringOff))) return rc;
    if ((rc = put(H.ringK.data(), H.ringK.size() * sizeof(int), (const void**)&d.ringK))) return rc;
    if ((rc = put(H.ringM3.data(), H.ringM3.size() * sizeof(int), (const void**)&d.ringM3))) return rc;
    {
        std::vector<T> twr = conv(H.twr);
        if ((rc = put(twr.data(), twr.size() * sizeof(T), (const void**)&d.twr))) return rc;
        d.logNr3 = ilog2i(std::max(P.Nr3, 3) / 3);
    }
    if ((rc = put(Tb.data(), Tb.size() * sizeof(T), (const void**)&d.Tb))) return rc;
    if ((rc = put(Mk.data(), Mk.size() * sizeof(T), (const void**)&d.Mk))) return rc;
    // the low-k matrices of the adjoint direction with t_j fastest
    auto transpose_lowk = [&](const std::vector<double>& src) {
        std::vector<T> o(src.size());
        for (int k = 0; k <= P.klow; ++k)
            for (int j = 0; j < P.nt; ++j)
                for (int l = 0; l < P.lcorr; ++l)
                    o[((size_t)k * P.lcorr + l) * P.nt + j] = (T)src[((size_t)k * P.nt + j) * P.lcorr + l];
        return o;
    };
    {
        std::vector<T> MkT = transpose_lowk(H.Mk);
        if ((rc = put(MkT.data(), MkT.size() * sizeof(T), (const void**)&d.MkT))) return rc;
    }
    if ((rc = put(ph.data(), ph.size() * sizeof(T), (const void**)&d.phase))) return rc;
    if ((rc = put(tw.data(), tw.size() * sizeof(T), (const void**)&d.tw))) return rc;
    std::vector<T> twd = conv(H.twd);
    if ((rc = put(twd.data(), twd.size() * sizeof(T), (const void**)&d.twd))) return rc;
    std::vector<T> twm = conv(H.twm);
    if ((rc = put(twm.data(), twm.size() * sizeof(T), (const void**)&d.twm))) return rc;
    std::vector<T> pos = conv(H.pos);
    if ((rc = put(pos.data(), pos.size() * sizeof(T), (const void**)&d.pos))) return rc;
    // point phase of every sample, e^{-i shift (u + v)} with u + v = h (x + y) / half,
    // evaluated in FP64 from the FP64 positions
    std::vector<T> pph(2 * (size_t)P.npts);
    {
        const double k = -P.shift * P.h / (0.5 * P.Ng / P.Lam);
        for (int q = 0; q < P.npts; ++q) {
            const double a = k * (H.pos[2 * (size_t)q] + H.pos[2 * (size_t)q + 1]);
            pph[2 * (size_t)q] = (T)std::cos(a);
            pph[2 * (size_t)q + 1] = (T)std::sin(a);
        }
    }
    if ((rc = put(pph.data(), pph.size() * sizeof(T), (const void**)&d.ph))) return rc;
    d.binRing = nullptr; d.ringBin = nullptr; d.binStart = nullptr; d.binPos = nullptr; d.binned = 0;
    d.spOrder = nullptr; d.spCount = 0; d.gbOrder = nullptr; d.gbCount = 0;
    if constexpr (sizeof(T) == 4) {
        // counting sort of the samples by the cell of their first tap, computed
        // with the same FP32 operations as the kernels' tap rule
        const size_t nb = (size_t)P.Ng * P.Ew;
        std::vector<int> key(P.npts), start(nb + 1, 0), ring(P.npts), rbin(P.npts);
        bool ok = true;
        const float hwf = 0.5f * (float)P.w;
        for (int q = 0; q < P.npts && ok; ++q) {
            const int gx0 = (int)std::ceil(pos[2 * (size_t)q] - hwf);
            const int gy0 = (int)std::ceil(pos[2 * (size_t)q + 1] - hwf);
            const int e0 = gx0 + P.hw, row = gy0 & (P.Ng - 1);
            if (e0 < 0 || e0 >= P.Ew) ok = false;
            key[q] = row * P.Ew + e0;
        }
        if (ok) {
            for (int q = 0; q < P.npts; ++q) ++start[(size_t)key[q] + 1];
            for (size_t k = 0; k < nb; ++k) start[k + 1] += start[k];
            std::vector<int> fill(start.begin(), start.end() - 1);
            std::vector<T> bpos(2 * (size_t)P.npts);
            for (int q = 0; q < P.npts; ++q) {
                const int slot = fill[key[q]]++;
                ring[slot] = q;
                rbin[q] = slot;
                bpos[2 * (size_t)slot] = pos[2 * (size_t)q];
                bpos[2 * (size_t)slot + 1] = pos[2 * (size_t)q + 1];
            }
            if ((rc = put(ring.data(), ring.size() * sizeof(int), (const void**)&d.binRing))) return rc;
            if ((rc = put(rbin.data(), rbin.size() * sizeof(int), (const void**)&d.ringBin))) return rc;
            if ((rc = put(start.data(), start.size() * sizeof(int), (const void**)&d.binStart))) return rc;
            if ((rc = put(bpos.data(), bpos.size() * sizeof(T), (const void**)&d.binPos))) return rc;
            // four blocks of spread_bins (and of gather_bins) fit a CU's LDS at once
            int ncu = 0;
            if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || ncu < 1)
                ncu = 256;
            const std::vector<int> order = spread_order(P, start, 4 * ncu), gorder = gather_order(P, start, 4 * ncu);
            if (!order.empty() && !gorder.empty()) {
                if ((rc = put(order.data(), order.size() * sizeof(int), (const void**)&d.spOrder))) return rc;
                if ((rc = put(gorder.data(), gorder.size() * sizeof(int), (const void**)&d.gbOrder))) return rc;
                d.spCount = (int)order.size();
                d.gbCount = (int)gorder.size();
                p->bin_ok = 1;
            }
        }
    }
    if (!p->bin_ok && p->spread_staged == 2) p->spread_staged = 1;
    d.binned = p->spread_staged == 2 ? 1 : 0;
    std::vector<T> Tbi = conv(H.Tbi), MkiT = transpose_lowk(H.Mki);
    if ((rc = put(Tbi.data(), Tbi.size() * sizeof(T), (const void**)&d.Tbi))) return rc;
    if ((rc = put(MkiT.data(), MkiT.size() * sizeof(T), (const void**)&d.MkiT))) return rc;
    d.n = P.n; d.m = P.m; d.nt = P.nt; d.mf = P.mf; d.mf3 = P.mf3; d.logmf = ilog2i(P.mf3 ? P.mf / 3 : P.mf);
    d.Ng = P.Ng; d.logNg = ilog2i(P.Ng); d.w = P.w; d.hw = P.hw; d.Rw = P.Rw; d.Ew = P.Ew; d.Ep = e_pitch(P);
    d.M = P.M; d.m3 = P.m3; d.log2M = ilog2i(P.m3 ? P.M / 3 : P.M); d.L = P.L; d.K = P.K; d.Kp = P.Kp; d.klow = P.klow; d.lcorr = P.lcorr;
    d.npts = P.npts; d.logNmax = ilog2i(P.Nmax);
    d.colsCW = p->cols_cw;
    d.dctCW = p->dct_cw;
    d.colsLCW = ilog2i(p->cols_cw);
    d.dctLCW = ilog2i(p->dct_cw);
    d.dct_stash = dct_stash_ok(P, p->dct_cw);
    d.dct_one = dct_one_ok(P, p->dct_cw);
    d.dct_wave = p->dct_wave_on ? dw_variant(P) : 0;
    d.dwCB = dw_columns(d.dct_wave);
    d.wfRows = p->wave_fft_on ? wf_rows_variant(P) : 0;
    d.wfSynth = p->wave_fft_on ? wf_synth_variant(P) : 0;
    d.fft_lr = p->fft_lr;
    d.tw_table = p->tw_table;
    d.phase_k = (T)(-P.shift * P.h / (0.5 * P.Ng / P.Lam));
    d.beta = (T)P.beta; d.beta_l2e = (T)(P.beta * 1.4426950408889634); d.shift = (T)P.shift; d.half = (T)(0.5 * P.Ng / P.Lam); d.lamh = (T)P.h;
    d.dlam = (T)P.dlam; d.pre_scale = (T)P.pre_scale; d.adj_scale = (T)P.adj_scale;
    d.mask_r2 = P.g.mask_radius > 0 ? P.g.mask_radius * P.g.mask_radius : 0.0;
    d.a = P.g.a; d.h = P.h;
    d.R2 = P.g.R * P.g.R;
    d.sine = 0; d.ubp = 0; d.part = nullptr;
    d.epi = Epi<T>{};
    // pixel centres in Omega \ Omega_0, with the kernels' own test
    long cnt = 0;
    if (d.mask_r2 > 0.0)
        for (int pp = 0; pp < P.n; ++pp)
            for (int q = 0; q < P.n; ++q) {
                double x = -d.a + (q + 0.5) * d.h, y = -d.a + (pp + 0.5) * d.h;
                double r2 = x * x + y * y;
                if (r2 <= d.R2 && !(r2 <= d.mask_r2)) ++cnt;
            }
    p->inv_count = cnt > 0 ? 1.0 / (double)cnt : 0.0;
    return PAT_OK;
}

int fail(int code, const std::string& msg)
{
    pat::set_error(msg);
    return code;
}

int check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PAT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return PAT_OK;
}

// Records a start/end event pair around one launch when timing is enabled.
struct StageTimer {
    pat_plan_s* p;
    hipStream_t st;
    int stage;
    bool on;
    StageTimer(pat_plan_s* p_, hipStream_t st_, int stage_)
        : p(p_), st(st_), stage(stage_), on(p_->timing && ((p_->timing_mask >> stage_) & 1u))
    {
        if (!on) return;
        if (p->ev_used * 2 + 2 > p->ev_pool.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { p->timing = false; return; }
            p->ev_pool.push_back(a);
            p->ev_pool.push_back(b);
        }
        (void)hipEventRecord(p->ev_pool[2 * p->ev_used], st);
    }
    ~StageTimer()
    {
        if (!on || !p->timing) return;
        (void)hipEventRecord(p->ev_pool[2 * p->ev_used + 1], st);
        if (p->ev_stage.size() <= p->ev_used) p->ev_stage.resize(p->ev_used + 1);
        p->ev_stage[p->ev_used] = stage;
        ++p->ev_used;
    }
};

template <typename T, int WMAX>
int run_forward(pat_plan_s* p, const Dev<T>& d, int B, const T* f, long fs, T* g, long gs, char* ws, hipStream_t st)
{
    const size_t wi = p->ws_stride;
    const size_t cs = sizeof(cx<T>);
    cx<T>* R = reinterpret_cast<cx<T>*>(ws + p->offR);
    cx<T>* E = reinterpret_cast<cx<T>*>(ws + p->offE);
    cx<T>* V = reinterpret_cast<cx<T>*>(ws + p->offV);
    cx<T>* G = reinterpret_cast<cx<T>*>(ws + p->offG);
    cx<T>* U = reinterpret_cast<cx<T>*>(ws + p->offU);
    int rc;
    {
        StageTimer tm(p, st, 0);
        if constexpr (sizeof(T) == 4) {
            if (d.wfRows) {
                if ((rc = launch_rows_fwd_w(d, B, f, fs, R, wi, st))) return fail(rc, "rows_fwd: no wave variant");
            } else {
                rows_fwd<T><<<dim3((d.n + 1) / 2, B), NT, cs * d.Ng, st>>>(d, f, fs, R, wi);
            }
        } else {
            rows_fwd<T><<<dim3((d.n + 1) / 2, B), NT, cs * d.Ng, st>>>(d, f, fs, R, wi);
        }
    }
    if ((rc = check_launch("rows_fwd"))) return rc;
    {
        StageTimer tm(p, st, 1);
        if constexpr (sizeof(T) == 4) {
            if (d.wfRows) {
                if ((rc = launch_cols_fwd_w(d, B, R, E, wi, st))) return fail(rc, "cols_fwd: no wave variant");
            } else {
                cols_fwd<T><<<dim3((d.Rw + d.colsCW - 1) / d.colsCW, B), NT, cs * d.Ng * d.colsCW, st>>>(d, R, E, wi);
            }
        } else {
            cols_fwd<T><<<dim3((d.Rw + d.colsCW - 1) / d.colsCW, B), NT, cs * d.Ng * d.colsCW, st>>>(d, R, E, wi);
        }
    }
    if ((rc = check_launch("cols_fwd"))) return rc;
    {
        const cx<T>* Pin = nullptr;
        const int G = std::max(1, std::min(p->ring_g, B));
        if constexpr (sizeof(T) == 4) {
            if (d.binned) {
                // the batch's sample array (the adjoint's Pol) holds the gathered samples
                StageTimer tg(p, st, PAT_STAGE_GATHER_FWD);
                cx<T>* Pg = reinterpret_cast<cx<T>*>(ws + (size_t)B * p->ws_stride);
                const int nz = (B + GB_BC - 1) / GB_BC;
                gather_bins<GB_BC><<<d.gbCount * nz, NT, gather_bins_lds(GB_BC), st>>>(d, E, Pg, B, G, wi, nz);
                Pin = Pg;
            }
            if ((rc = check_launch("gather_bins"))) return rc;
        }
        StageTimer tm(p, st, 2);
        ring_fwd<T, WMAX><<<dim3(d.L, (B + G - 1) / G), NT, ring_lds(p->H.P, G), st>>>(d, E, Pin, V, U, wi, B, G);
    }
    if ((rc = check_launch("ring_fwd"))) return rc;
    {
        StageTimer tm(p, st, 3);
        if constexpr (sizeof(T) == 4) {
            if (d.dct_wave) {
                if ((rc = launch_dct_wave(d, B, V, G, wi, 0, st))) return fail(rc, "dct_fwd: no dct_wave variant");
            } else {
                dct_cols<T><<<dim3((d.Kp + d.dctCW - 1) / d.dctCW, B), NT, dct_lds(p->H.P, d.dctCW), st>>>(d, V, G, wi, 0);
            }
        } else {
            dct_cols<T><<<dim3((d.Kp + d.dctCW - 1) / d.dctCW, B), NT, dct_lds(p->H.P, d.dctCW), st>>>(d, V, G, wi, 0);
        }
    }
    if ((rc = check_launch("dct_fwd"))) return rc;
    {
        StageTimer tm(p, st, 4);
        lowk_fwd<T><<<dim3((d.nt * (d.klow + 1) * LK_LANES + NT - 1) / NT, B), NT, 0, st>>>(d, U, G, wi);
    }
    if ((rc = check_launch("lowk_fwd"))) return rc;
    {
        StageTimer tm(p, st, 5);
        if constexpr (sizeof(T) == 4) {
            if (d.wfSynth) {
                if ((rc = launch_synth_fwd_w(d, B, G, g, gs, wi, st))) return fail(rc, "synth_fwd: no wave variant");
            } else {
                synth_fwd<T><<<dim3((d.nt + 1) / 2, B), NT, cs * 2 * d.mf, st>>>(d, G, g, gs, wi);
            }
        } else {
            synth_fwd<T><<<dim3((d.nt + 1) / 2, B), NT, cs * 2 * d.mf, st>>>(d, G, g, gs, wi);
        }
    }
    return check_launch("synth_fwd");
}

template <typename T, int WMAX>
int run_adjoint(pat_plan_s* p, const Dev<T>& d, int B, const T* g, long gs, T* f, long fs, char* ws, hipStream_t st)
{
    const size_t wi = p->ws_stride;
    const size_t cs = sizeof(cx<T>);
    cx<T>* R = reinterpret_cast<cx<T>*>(ws + p->offR);
    cx<T>* E = reinterpret_cast<cx<T>*>(ws + p->offE);
    cx<T>* V = reinterpret_cast<cx<T>*>(ws + p->offV);
    cx<T>* G = reinterpret_cast<cx<T>*>(ws + p->offG);
    cx<T>* U = reinterpret_cast<cx<T>*>(ws + p->offU);
    cx<T>* Pol = reinterpret_cast<cx<T>*>(ws + (size_t)B * p->ws_stride);
    const pat::Params& P = p->H.P;
    int rc;
    {
        StageTimer tm(p, st, 6);
        if constexpr (sizeof(T) == 4) {
            if (d.wfSynth) {
                if ((rc = launch_synth_adj_w(d, B, g, gs, G, wi, st))) return fail(rc, "synth_adj: no wave variant");
            } else {
                synth_adj<T><<<dim3((d.nt + 1) / 2, B), NT, cs * d.mf, st>>>(d, g, gs, G, wi);
            }
        } else {
            synth_adj<T><<<dim3((d.nt + 1) / 2, B), NT, cs * d.mf, st>>>(d, g, gs, G, wi);
        }
    }
    if ((rc = check_launch("synth_adj"))) return rc;
    {
        StageTimer tm(p, st, 7);
        lowk_adj<T><<<dim3(d.lcorr, B), NT, 0, st>>>(d, G, U, wi);
    }
    if ((rc = check_launch("lowk_adj"))) return rc;
    {
        StageTimer tm(p, st, 8);
        if constexpr (sizeof(T) == 4) {
            if (d.dct_wave) {
                if ((rc = launch_dct_wave(d, B, G, V, wi, 1, st))) return fail(rc, "dct_adj: no dct_wave variant");
            } else {
                dct_cols<T><<<dim3((d.Kp + d.dctCW - 1) / d.dctCW, B), NT, dct_lds(p->H.P, d.dctCW), st>>>(d, G, V, wi, 1);
            }
        } else {
            dct_cols<T><<<dim3((d.Kp + d.dctCW - 1) / d.dctCW, B), NT, dct_lds(p->H.P, d.dctCW), st>>>(d, G, V, wi, 1);
        }
    }
    if ((rc = check_launch("dct_adj"))) return rc;
    {
        StageTimer tm(p, st, 9);
        const int Gr = std::max(1, std::min(p->ring_g, B));
        ring_adj<T, WMAX><<<dim3((B + Gr - 1) / Gr, d.L), NT, ring_lds(P, Gr), st>>>(d, V, U, Pol, B, Gr, wi);
    }
    if ((rc = check_launch("ring_adj"))) return rc;
    {
        StageTimer tm(p, st, 10);
        constexpr int BCL = sizeof(T) == 4 ? 16 : 8;  // image group of the spread: BCL or BCL / 2
        const dim3 grid((d.Ew + 15) / 16, (d.Ng + 15) / 16, 1);
        const dim3 g1(grid.x, grid.y, (B + BCL - 1) / BCL), g2(grid.x, grid.y, (B + BCL / 2 - 1) / (BCL / 2));
        const size_t l1 = spread_tiles_lds(true, BCL, cs), l2 = spread_tiles_lds(true, BCL / 2, cs);
        bool done = false;
        if constexpr (sizeof(T) == 4) {
            if (d.binned) {
                const int nz1 = (int)g1.z, nz2 = (int)g2.z;
                if (p->spread_bc >= BCL)
                    spread_bins<BCL><<<d.spCount * nz1, NT, spread_bins_lds(BCL), st>>>(d, Pol, B, E, wi, nz1);
                else
                    spread_bins<BCL / 2><<<d.spCount * nz2, NT, spread_bins_lds(BCL / 2), st>>>(d, Pol, B, E, wi, nz2);
                done = true;
            }
        }
        if (!done) {
            if (p->spread_bc >= BCL) {
                if (p->spread_staged) spread_tiles<T, WMAX, BCL, true><<<g1, NT, l1, st>>>(d, Pol, B, E, wi);
                else spread_tiles<T, WMAX, BCL, false><<<g1, NT, 0, st>>>(d, Pol, B, E, wi);
            } else {
                if (p->spread_staged) spread_tiles<T, WMAX, BCL / 2, true><<<g2, NT, l2, st>>>(d, Pol, B, E, wi);
                else spread_tiles<T, WMAX, BCL / 2, false><<<g2, NT, 0, st>>>(d, Pol, B, E, wi);
            }
        }
    }
    if ((rc = check_launch("spread_adj"))) return rc;
    {
        StageTimer tm(p, st, 11);
        if constexpr (sizeof(T) == 4) {
            if (d.wfRows) {
                if ((rc = launch_cols_adj_w(d, B, E, R, wi, st))) return fail(rc, "cols_adj: no wave variant");
            } else {
                cols_adj<T><<<dim3((d.Rw + d.colsCW - 1) / d.colsCW, B), NT, cs * d.Ng * d.colsCW, st>>>(d, E, R, wi);
            }
        } else {
            cols_adj<T><<<dim3((d.Rw + d.colsCW - 1) / d.colsCW, B), NT, cs * d.Ng * d.colsCW, st>>>(d, E, R, wi);
        }
    }
    if ((rc = check_launch("cols_adj"))) return rc;
    {
        StageTimer tm(p, st, 12);
        if constexpr (sizeof(T) == 4) {
            if (d.wfRows && !d.ubp) {
                if ((rc = launch_rows_adj_w(d, B, R, f, fs, wi, st))) return fail(rc, "rows_adj: no wave variant");
            } else {
                rows_adj<T><<<dim3((d.n + 1) / 2, B), NT, cs * d.Ng, st>>>(d, R, f, fs, wi);
            }
        } else {
            rows_adj<T><<<dim3((d.n + 1) / 2, B), NT, cs * d.Ng, st>>>(d, R, f, fs, wi);
        }
    }
    return check_launch("rows_adj");
}

// Approximate inverse (Alg. 3): the adjoint chain with the inverse's tables
// (J_k' for J_k, the sine transform over t, scale -2c s) computes the
// back-projection v of every pixel and the partial sums over
// Omega \ Omega_0; ubp_apply adds the constant and restricts to Omega_0.
template <typename T, int WMAX>
int run_inverse(pat_plan_s* p, const Dev<T>& d, int B, const T* g, long gs, T* f, long fs, char* ws, hipStream_t st)
{
    Dev<T> di = d;
    di.Tb = d.Tbi;
    di.MkT = d.MkiT;
    di.sine = 1;
    di.ubp = 1;
    di.adj_scale = (T)p->H.P.inv_scale;
    di.part = reinterpret_cast<double*>(ws + p->offC);
    int rc = run_adjoint<T, WMAX>(p, di, B, g, gs, f, fs, ws, st);
    if (rc) return rc;
    const int n = d.n;
    const int blocks = std::max(1, std::min((n * n + 4 * NT - 1) / (4 * NT), 256));
    ubp_apply<T><<<dim3(blocks, B), NT, 0, st>>>(di, f, fs, (n + 1) / 2, p->inv_count, p->ws_stride);
    return check_launch("ubp_apply");
}

// ---------------------------------------------------------------------------
// Grouped launches: plans of different sizes (same precision) run each stage
// as one launch whose blocks cover the grids of all plans back to back.  A
// block finds its plan from the per-stage block offsets (padded to multiples
// of the XCD count), rebuilds its stage coordinates and runs the same kernel
// body as the single-plan launch, so results are identical to per-plan calls.
// ---------------------------------------------------------------------------
constexpr int GROUP_MAX = 5;  // plans per group: their Dev copies fill the 4 KB of kernel arguments

template <typename T>
struct GroupPlan {
    Dev<T> d;
    const T* fin;
    T* fout;
    const T* gin;
    T* gout;
    long fs, gs;
    char *R, *E, *V, *Gh, *U, *Pol;
    size_t wi;
    int B, G, staged;
    int off[PAT_NUM_STAGES];
};

// the binned gather (FP32 plans with binned samples), launched before RING_FWD
constexpr int STAGE_GATHER = PAT_STAGE_GATHER_FWD;

template <typename T>
struct GroupArgs {
    GroupPlan<T> p[GROUP_MAX];
    int nplans;
};

template <typename T>
__host__ __device__ inline void stage_grid(const Dev<T>& d, int S, int B, int G, int BC, int& nx, int& ny, int& nz)
{
    nz = 1;
    switch (S) {
        case PAT_STAGE_ROWS_FWD:
        case PAT_STAGE_ROWS_ADJ:
            nx = d.wfRows ? ((d.n + 1) / 2 + WF_WAVES - 1) / WF_WAVES : (d.n + 1) / 2;
            ny = B;
            break;
        case PAT_STAGE_COLS_FWD:
        case PAT_STAGE_COLS_ADJ:
            nx = d.wfRows ? (d.Rw + WF_WAVES - 1) / WF_WAVES : (d.Rw + d.colsCW - 1) / d.colsCW;
            ny = B;
            break;
        case PAT_STAGE_RING_FWD: nx = d.L; ny = (B + G - 1) / G; break;
        case PAT_STAGE_DCT_FWD:
        case PAT_STAGE_DCT_ADJ: nx = d.dct_wave ? d.Kp / d.dwCB : (d.Kp + d.dctCW - 1) / d.dctCW; ny = B; break;
        case PAT_STAGE_LOWK_FWD: nx = (d.nt * (d.klow + 1) * LK_LANES + NT - 1) / NT; ny = B; break;
        case PAT_STAGE_SYNTH_FWD:
        case PAT_STAGE_SYNTH_ADJ:
            nx = d.wfSynth ? ((d.nt + 1) / 2 + WF_WAVES - 1) / WF_WAVES : (d.nt + 1) / 2;
            ny = B;
            break;
        case PAT_STAGE_LOWK_ADJ: nx = d.lcorr; ny = B; break;
        case PAT_STAGE_RING_ADJ: nx = (B + G - 1) / G; ny = d.L; break;
        case STAGE_GATHER:
            if (d.binned) { nx = d.gbCount; ny = 1; nz = (B + GB_BC - 1) / GB_BC; }
            else { nx = 0; ny = 1; }
            break;
        default:  // spread: the binned form walks the plan's dispatch table
            nz = (B + BC - 1) / BC;
            if (d.binned) { nx = d.spCount; ny = 1; }
            else { nx = (d.Ew + 15) / 16; ny = (d.Ng + 15) / 16; }
            break;
    }
}

template <typename T, int WMAX, int S>
__global__ __launch_bounds__(NT) void grouped_stage(GroupArgs<T> ga)
{
    constexpr int BC = sizeof(T) == 4 ? 16 : 8;
    const int lin = blockIdx.x;
    int pi = 0;
    while (pi + 1 < ga.nplans && lin >= ga.p[pi + 1].off[S]) ++pi;
    const GroupPlan<T>& q = ga.p[pi];
    int nx, ny, nz;
    stage_grid(q.d, S, q.B, q.G, BC, nx, ny, nz);
    const int local = lin - q.off[S], plane = nx * ny;
    if (local >= plane * nz) return;  // padding block
    Blk bk;
    bk.nx = nx;
    bk.z = local / plane;
    const int r = local - bk.z * plane;
    if (S == PAT_STAGE_LOWK_FWD || S == PAT_STAGE_LOWK_ADJ || S == PAT_STAGE_RING_ADJ) {
        bk.x = r % nx;
        bk.y = r / nx;
    } else {
        xcd_remap(r, nx, plane, bk.x, bk.y);
    }
    cx<T>* R = reinterpret_cast<cx<T>*>(q.R);
    cx<T>* E = reinterpret_cast<cx<T>*>(q.E);
    cx<T>* V = reinterpret_cast<cx<T>*>(q.V);
    cx<T>* Gh = reinterpret_cast<cx<T>*>(q.Gh);
    cx<T>* U = reinterpret_cast<cx<T>*>(q.U);
    cx<T>* Pol = reinterpret_cast<cx<T>*>(q.Pol);
    if constexpr (sizeof(T) == 4) {
        if constexpr (S == PAT_STAGE_ROWS_FWD)
            if (q.d.wfRows) { rows_fwd_w_dispatch(q.d, bk, q.fin, q.fs, R, q.wi); return; }
        if constexpr (S == PAT_STAGE_COLS_FWD)
            if (q.d.wfRows) { cols_fwd_w_dispatch(q.d, bk, R, E, q.wi); return; }
        if constexpr (S == PAT_STAGE_SYNTH_FWD)
            if (q.d.wfSynth) { synth_fwd_w_dispatch(q.d, bk, Gh, q.gout, q.gs, q.wi); return; }
        if constexpr (S == PAT_STAGE_SYNTH_ADJ)
            if (q.d.wfSynth) { synth_adj_w_dispatch(q.d, bk, q.gin, q.gs, Gh, q.wi); return; }
        if constexpr (S == PAT_STAGE_COLS_ADJ)
            if (q.d.wfRows) { cols_adj_w_dispatch(q.d, bk, E, R, q.wi); return; }
        if constexpr (S == PAT_STAGE_ROWS_ADJ)
            if (q.d.wfRows && !q.d.ubp) { rows_adj_w_dispatch(q.d, bk, R, q.fout, q.fs, q.wi); return; }
    }
    if constexpr (S == PAT_STAGE_ROWS_FWD) rows_fwd_body<T>(q.d, bk, q.fin, q.fs, R, q.wi);
    if constexpr (S == PAT_STAGE_COLS_FWD) cols_fwd_body<T>(q.d, bk, R, E, q.wi);
    if constexpr (S == STAGE_GATHER) {
        // entry local / nz of the plan's dispatch table, as the single-plan launch
        if constexpr (sizeof(T) == 4) {
            int entry, z;
            table_block(local, nz, entry, z);
            const int t = q.d.gbOrder[entry];
            if (t < 0) return;
            gather_bins_body<GB_BC>(q.d, Blk{t & 0xfff, t >> 12, z, 0}, E, Pol, q.B, q.G, q.wi);
        }
    }
    if constexpr (S == PAT_STAGE_RING_FWD) ring_fwd_body<T, WMAX>(q.d, bk, E, q.d.binned ? Pol : nullptr, V, U, q.wi, q.B, q.G);
    if constexpr (S == PAT_STAGE_DCT_FWD) {
        if constexpr (sizeof(T) == 4) {
            if (q.d.dct_wave) { dct_wave_dispatch(q.d, bk, V, Gh, q.wi, 0); return; }
        }
        if (q.d.dct_one) dct_cos_body<T>(q.d, bk, V, Gh, q.wi, 0);
        else dct_cols_body<T>(q.d, bk, V, Gh, q.wi, 0);
    }
    if constexpr (S == PAT_STAGE_LOWK_FWD) lowk_fwd_body<T>(q.d, bk, U, Gh, q.wi);
    if constexpr (S == PAT_STAGE_SYNTH_FWD) synth_fwd_body<T>(q.d, bk, Gh, q.gout, q.gs, q.wi);
    if constexpr (S == PAT_STAGE_SYNTH_ADJ) synth_adj_body<T>(q.d, bk, q.gin, q.gs, Gh, q.wi);
    if constexpr (S == PAT_STAGE_LOWK_ADJ) lowk_adj_body<T>(q.d, bk, Gh, U, q.wi);
    if constexpr (S == PAT_STAGE_DCT_ADJ) {
        if constexpr (sizeof(T) == 4) {
            if (q.d.dct_wave) { dct_wave_dispatch(q.d, bk, Gh, V, q.wi, 1); return; }
        }
        if (q.d.dct_one) dct_cos_body<T>(q.d, bk, Gh, V, q.wi, 1);
        else dct_cols_body<T>(q.d, bk, Gh, V, q.wi, 1);
    }
    if constexpr (S == PAT_STAGE_RING_ADJ) ring_adj_body<T, WMAX>(q.d, bk, V, U, Pol, q.B, q.G, q.wi);
    if constexpr (S == PAT_STAGE_SPREAD_ADJ) {
        if constexpr (sizeof(T) == 4) {
            if (q.d.binned) {
                // entry local / nz of the plan's dispatch table for image group
                // local mod nz, as the single-plan launch
                int entry, z;
                table_block(local, nz, entry, z);
                const int t = q.d.spOrder[entry];
                if (t < 0) return;
                const Blk tb = {t & 0xfff, (t >> 12) & 0xfff, z, 0};
                if (t >> 26) spread_bins_body<BC, SB_TILE / 2>(q.d, tb, (t >> 24) & 3, Pol, q.B, E, q.wi);
                else spread_bins_body<BC, SB_TILE>(q.d, tb, 0, Pol, q.B, E, q.wi);
                return;
            }
        }
        if (q.staged) spread_tiles_body<T, WMAX, BC, true>(q.d, bk, Pol, q.B, E, q.wi);
        else spread_tiles_body<T, WMAX, BC, false>(q.d, bk, Pol, q.B, E, q.wi);
    }
    if constexpr (S == PAT_STAGE_COLS_ADJ) cols_adj_body<T>(q.d, bk, E, R, q.wi);
    if constexpr (S == PAT_STAGE_ROWS_ADJ) rows_adj_body<T>(q.d, bk, R, q.fout, q.fs, q.wi);
}

inline const Dev<float>& dev_of(const pat_plan_s* p, float*) { return p->df; }
inline const Dev<double>& dev_of(const pat_plan_s* p, double*) { return p->dd; }

// dynamic LDS bytes of stage S for plan p with ring group G
size_t stage_lds(const pat_plan_s* p, int S, int G)
{
    const pat::Params& P = p->H.P;
    const size_t cs = (P.dt == PAT_F64) ? 16 : 8;
    switch (S) {
        case PAT_STAGE_ROWS_FWD:
        case PAT_STAGE_ROWS_ADJ:
        case PAT_STAGE_COLS_FWD:
        case PAT_STAGE_COLS_ADJ:
            if (p->df.wfRows) return wf_lds(p->df.wfRows);
            return cs * P.Ng * ((S == PAT_STAGE_COLS_FWD || S == PAT_STAGE_COLS_ADJ) ? p->cols_cw : 1);
        case PAT_STAGE_RING_FWD: return ring_lds(P, G);
        case PAT_STAGE_DCT_FWD:
        case PAT_STAGE_DCT_ADJ: return p->df.dct_wave ? dw_lds(p->df.dct_wave) : dct_lds(P, p->dct_cw);
        case PAT_STAGE_SYNTH_FWD: return p->df.wfSynth ? wf_lds(p->df.wfSynth) : cs * 2 * P.mf;
        case PAT_STAGE_SYNTH_ADJ: return p->df.wfSynth ? wf_lds(p->df.wfSynth) : cs * P.mf;
        case PAT_STAGE_RING_ADJ: return ring_lds(P, G);
        case PAT_STAGE_SPREAD_ADJ: {
            const int bc = (P.dt == PAT_F64) ? 8 : 16;  // the grouped launch's image group
            if (P.dt == PAT_F32 && p->spread_staged == 2) return spread_bins_lds(bc);
            return spread_tiles_lds(p->spread_staged != 0, bc, cs);
        }
        case STAGE_GATHER: return (P.dt == PAT_F32 && p->spread_staged == 2) ? gather_bins_lds(GB_BC) : 0;
        default: return 0;
    }
}

template <int S, typename T, int WMAX>
int launch_grouped(const GroupArgs<T>& ga, int blocks, size_t lds, hipStream_t st)
{
    grouped_stage<T, WMAX, S><<<blocks, NT, lds, st>>>(ga);
    return check_launch("grouped stage");
}

template <typename T, int WMAX>
int group_run(const std::vector<pat_plan_s*>& plans, bool adjoint, const int* batch, const void* const* in,
              void* const* out, void* const* ws, hipStream_t st)
{
    static_assert(sizeof(GroupArgs<T>) <= 4000, "grouped kernel arguments exceed the kernarg limit");
    constexpr int BC = sizeof(T) == 4 ? 16 : 8;
    GroupArgs<T> ga;
    std::memset(&ga, 0, sizeof(ga));
    ga.nplans = (int)plans.size();
    int total[PAT_NUM_STAGES] = {0};
    size_t lds[PAT_NUM_STAGES] = {0};
    for (int i = 0; i < ga.nplans; ++i) {
        pat_plan_s* p = plans[i];
        const pat::Params& P = p->H.P;
        GroupPlan<T>& q = ga.p[i];
        const int B = batch[i];
        if (B < 1 || B > p->max_batch) return fail(PAT_ESMALL, "pat_group: batch outside [1, max_batch] of a plan");
        if (!in[i] || !out[i] || !ws[i]) return fail(PAT_EINVAL, "pat_group: null pointer");
        q.d = dev_of(p, (T*)nullptr);
        q.B = B;
        q.G = std::max(1, std::min(p->ring_g, B));
        q.staged = p->spread_staged;
        q.fs = (long)P.n * P.n;
        q.gs = (long)P.nt * P.m;
        if (adjoint) {
            q.gin = static_cast<const T*>(in[i]);
            q.fout = static_cast<T*>(out[i]);
        } else {
            q.fin = static_cast<const T*>(in[i]);
            q.gout = static_cast<T*>(out[i]);
        }
        char* w = static_cast<char*>(ws[i]);
        q.R = w + p->offR; q.E = w + p->offE; q.V = w + p->offV; q.Gh = w + p->offG; q.U = w + p->offU;
        q.Pol = w + (size_t)B * p->ws_stride;
        q.wi = p->ws_stride;
        for (int S = 0; S < PAT_NUM_STAGES; ++S) {
            int nx, ny, nz;
            stage_grid(q.d, S, B, q.G, BC, nx, ny, nz);
            q.off[S] = total[S];
            total[S] += (nx * ny * nz + NUM_XCD - 1) / NUM_XCD * NUM_XCD;
            lds[S] = std::max(lds[S], stage_lds(p, S, q.G));
        }
    }
    int rc;
    if (!adjoint) {
        if ((rc = launch_grouped<PAT_STAGE_ROWS_FWD, T, WMAX>(ga, total[0], lds[0], st))) return rc;
        if ((rc = launch_grouped<PAT_STAGE_COLS_FWD, T, WMAX>(ga, total[1], lds[1], st))) return rc;
        if (total[STAGE_GATHER] > 0 &&
            (rc = launch_grouped<STAGE_GATHER, T, WMAX>(ga, total[STAGE_GATHER], lds[STAGE_GATHER], st)))
            return rc;
        if ((rc = launch_grouped<PAT_STAGE_RING_FWD, T, WMAX>(ga, total[2], lds[2], st))) return rc;
        if ((rc = launch_grouped<PAT_STAGE_DCT_FWD, T, WMAX>(ga, total[3], lds[3], st))) return rc;
        if ((rc = launch_grouped<PAT_STAGE_LOWK_FWD, T, WMAX>(ga, total[4], lds[4], st))) return rc;
        return launch_grouped<PAT_STAGE_SYNTH_FWD, T, WMAX>(ga, total[5], lds[5], st);
    }
    if ((rc = launch_grouped<PAT_STAGE_SYNTH_ADJ, T, WMAX>(ga, total[6], lds[6], st))) return rc;
    if ((rc = launch_grouped<PAT_STAGE_LOWK_ADJ, T, WMAX>(ga, total[7], lds[7], st))) return rc;
    if ((rc = launch_grouped<PAT_STAGE_DCT_ADJ, T, WMAX>(ga, total[8], lds[8], st))) return rc;
    if ((rc = launch_grouped<PAT_STAGE_RING_ADJ, T, WMAX>(ga, total[9], lds[9], st))) return rc;
    if ((rc = launch_grouped<PAT_STAGE_SPREAD_ADJ, T, WMAX>(ga, total[10], lds[10], st))) return rc;
    if ((rc = launch_grouped<PAT_STAGE_COLS_ADJ, T, WMAX>(ga, total[11], lds[11], st))) return rc;
    return launch_grouped<PAT_STAGE_ROWS_ADJ, T, WMAX>(ga, total[12], lds[12], st);
}

// ---------------------------------------------------------------------------
// Launch-shape autotuner.  Choices: the largest FFT pass radix (16 or 8), the
// column count of the column-FFT and cosine-transform blocks, the number of
// images per ring_fwd block and per spread group.  Defaults follow the LDS
// limits; with a tuning cache path the plan looks its geometry / batch /
// device up in the cache and otherwise times every candidate of one choice
// at a time (forward + adjoint at the plan's max_batch, zero data: the
// kernels' work does not depend on the values) and appends the winner.
// ---------------------------------------------------------------------------
void default_tune(pat_plan_s* p)
{
    const pat::Params& P = p->H.P;
    p->cols_cw = lds_cols(P);
    p->dct_cw = lds_dct(P);
    p->ring_g = ring_group_max(P);
    p->spread_bc = (P.dt == PAT_F64) ? 8 : 16;
    p->fft_lr = 4;
    p->tw_table = 0;
    p->spread_staged = (P.dt == PAT_F64) ? 1 : 2;  // FP32: the binned spread (if its tables build)
    p->dct_wave_on = 1;
    p->wave_fft_on = 1;
}

void apply_tune(pat_plan_s* p)
{
    p->df.colsCW = p->dd.colsCW = p->cols_cw;
    p->df.dctCW = p->dd.dctCW = p->dct_cw;
    p->df.colsLCW = p->dd.colsLCW = ilog2i(p->cols_cw);
    p->df.dctLCW = p->dd.dctLCW = ilog2i(p->dct_cw);
    p->df.fft_lr = p->dd.fft_lr = p->fft_lr;
    p->df.tw_table = p->dd.tw_table = p->tw_table;
    p->df.dct_stash = p->dd.dct_stash = dct_stash_ok(p->H.P, p->dct_cw);
    p->df.dct_one = p->dd.dct_one = dct_one_ok(p->H.P, p->dct_cw);
    p->df.dct_wave = p->dd.dct_wave = p->dct_wave_on ? dw_variant(p->H.P) : 0;
    p->df.dwCB = p->dd.dwCB = dw_columns(p->df.dct_wave);
    p->df.wfRows = p->dd.wfRows = p->wave_fft_on ? wf_rows_variant(p->H.P) : 0;
    p->df.wfSynth = p->dd.wfSynth = p->wave_fft_on ? wf_synth_variant(p->H.P) : 0;
    p->df.binned = (p->spread_staged == 2 && p->bin_ok) ? 1 : 0;
    p->dd.binned = 0;
}

bool pow2_in(int v, int hi) { return v >= 1 && v <= hi && (v & (v - 1)) == 0; }

bool tune_valid(const pat_plan_s* p)
{
    const pat::Params& P = p->H.P;
    const int bcl = (P.dt == PAT_F64) ? 8 : 16;
    return pow2_in(p->cols_cw, lds_cols(P)) && pow2_in(p->dct_cw, lds_dct(P)) && pow2_in(p->ring_g, ring_group_max(P)) &&
           (p->spread_bc == bcl || p->spread_bc == bcl / 2) && (p->fft_lr == 3 || p->fft_lr == 4) &&
           (p->tw_table == 0 || p->tw_table == 1) &&
           (p->spread_staged == 0 || p->spread_staged == 1 || (p->spread_staged == 2 && p->bin_ok)) &&
           (p->dct_wave_on == 0 || p->dct_wave_on == 1) && (p->wave_fft_on == 0 || p->wave_fft_on == 1);
}

std::string tune_key(const pat_plan_s* p)
{
    const pat::Params& P = p->H.P;
    const pat_geometry& g = P.g;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == ' ' || ch == '|') ch = '_';
    char buf[640];
    std::snprintf(buf, sizeof(buf),
                  "pat-tune-1 arch=%s dtype=%d n=%d m=%d nt=%d a=%.17g R=%.17g c=%.17g theta0=%.17g arc=%.17g T=%.17g "
                  "rho=%.17g mask=%.17g batch=%d",
                  arch.c_str(), (int)P.dt, g.n, g.m, g.nt, g.a, g.R, g.c, g.theta0, g.arc, g.T, g.taper_rho,
                  g.mask_radius, p->max_batch);
    return buf;
}

bool tune_lookup(pat_plan_s* p, const char* path, const std::string& key)
{
    FILE* fp = std::fopen(path, "r");
    if (!fp) return false;
    bool found = false;
    std::vector<char> line(4096);
    while (std::fgets(line.data(), (int)line.size(), fp)) {
        std::string l(line.data());
        const size_t bar = l.find(" | ");
        if (bar == std::string::npos || l.compare(0, bar, key) != 0 || bar != key.size()) continue;
        pat_plan_s t = *p;
        double ms = 0;
        t.tw_table = 0;
        t.spread_staged = 0;
        t.dct_wave_on = 0;
        t.wave_fft_on = 0;
        const int got = std::sscanf(l.c_str() + bar + 3,
                                    "cols_cw=%d dct_cw=%d ring_group=%d spread_images=%d fft_radix_log2=%d ms=%lf "
                                    "twiddle_table=%d spread_staged=%d dct_wave=%d wave_fft=%d",
                                    &t.cols_cw, &t.dct_cw, &t.ring_g, &t.spread_bc, &t.fft_lr, &ms, &t.tw_table,
                                    &t.spread_staged, &t.dct_wave_on, &t.wave_fft_on);
        if (got >= 6 && tune_valid(&t)) {
            p->cols_cw = t.cols_cw; p->dct_cw = t.dct_cw; p->ring_g = t.ring_g; p->spread_bc = t.spread_bc;
            p->fft_lr = t.fft_lr; p->tw_table = t.tw_table; p->spread_staged = t.spread_staged; p->tuned_ms = ms;
            p->dct_wave_on = t.dct_wave_on;
            p->wave_fft_on = t.wave_fft_on;
            found = true;  // keep scanning: the last matching line wins
        }
    }
    std::fclose(fp);
    return found;
}

void tune_store(const pat_plan_s* p, const char* path, const std::string& key)
{
    FILE* fp = std::fopen(path, "a");
    if (!fp) return;
    std::fprintf(fp,
                 "%s | cols_cw=%d dct_cw=%d ring_group=%d spread_images=%d fft_radix_log2=%d ms=%.6f twiddle_table=%d "
                 "spread_staged=%d dct_wave=%d wave_fft=%d\n",
                 key.c_str(), p->cols_cw, p->dct_cw, p->ring_g, p->spread_bc, p->fft_lr, p->tuned_ms, p->tw_table,
                 p->spread_staged, p->dct_wave_on, p->wave_fft_on);
    std::fclose(fp);
}

template <typename T, int WMAX>
int run_forward(pat_plan_s* p, const Dev<T>& d, int B, const T* f, long fs, T* g, long gs, char* ws, hipStream_t st);
template <typename T, int WMAX>
int run_adjoint(pat_plan_s* p, const Dev<T>& d, int B, const T* g, long gs, T* f, long fs, char* ws, hipStream_t st);

template <typename T, int WMAX>
int tune_search(pat_plan_s* p, const Dev<T>& d)
{
    const pat::Params& P = p->H.P;
    const int B = p->max_batch;
    const long fsz = (long)P.n * P.n, gsz = (long)P.nt * P.m;
    void *ws = nullptr, *f = nullptr, *g = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = PAT_OK;
    auto cleanup = [&]() {
        if (ws) (void)hipFree(ws);
        if (f) (void)hipFree(f);
        if (g) (void)hipFree(g);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
    };
    if (hipMalloc(&ws, p->ws_img * (size_t)B) != hipSuccess || hipMalloc(&f, sizeof(T) * fsz * B) != hipSuccess ||
        hipMalloc(&g, sizeof(T) * gsz * B) != hipSuccess) {
        cleanup();
        return fail(PAT_ENOMEM, "autotuner: workspace allocation failed");
    }
    if (hipMemset(f, 0, sizeof(T) * fsz * B) != hipSuccess || hipMemset(g, 0, sizeof(T) * gsz * B) != hipSuccess ||
        hipStreamCreate(&st) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(PAT_EHIP, "autotuner: set-up failed");
    }
    // one untimed pair, then TUNE_REPS timed pairs
    constexpr int TUNE_REPS = 8;
    auto measure = [&](double& ms) -> int {
        apply_tune(p);
        for (int rep = 0; rep <= TUNE_REPS; ++rep) {
            if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) return PAT_EHIP;
            int r = run_forward<T, WMAX>(p, d, B, (const T*)f, fsz, (T*)g, gsz, (char*)ws, st);
            if (!r) r = run_adjoint<T, WMAX>(p, d, B, (const T*)g, gsz, (T*)f, fsz, (char*)ws, st);
            if (r) return r;
        }
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return PAT_EHIP;
        float t = 0;
        if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) return PAT_EHIP;
        ms = t / TUNE_REPS;
        return PAT_OK;
    };
    const int bcl = (P.dt == PAT_F64) ? 8 : 16;
    struct Choice {
        int* field;
        std::vector<int> cands;
    };
    std::vector<int> cw, dw, rg;
    for (int v = lds_cols(P); v >= 1; v >>= 1) cw.push_back(v);
    for (int v = lds_dct(P); v >= 1; v >>= 1) dw.push_back(v);
    for (int v = ring_group_max(P); v >= 1; v >>= 1) rg.push_back(v);
    std::vector<Choice> choices = {{&p->fft_lr, {4, 3}},
                                   {&p->tw_table, {0, 1}},
                                   {&p->cols_cw, cw},
                                   {&p->dct_cw, dw},
                                   {&p->ring_g, rg},
                                   {&p->spread_bc, {bcl, bcl / 2}},
                                   {&p->spread_staged, p->bin_ok ? std::vector<int>{2, 1, 0} : std::vector<int>{1, 0}},
                                   {&p->dct_wave_on, {1, 0}},
                                   {&p->wave_fft_on, {1, 0}}};
    // the first run of a plan loads the kernels' code: one measurement is
    // discarded before the baseline; a candidate replaces the current choice
    // only when it is more than 1 % faster (the run-to-run spread of a
    // measurement), one choice at a time in the order above
    double best = 0;
    if ((rc = measure(best)) || (rc = measure(best))) { cleanup(); return fail(rc, "autotuner: timing run failed"); }
    for (Choice& c : choices) {
        int keep = *c.field;
        for (int v : c.cands) {
            if (v == keep) continue;
            *c.field = v;
            double ms = 0;
            if ((rc = measure(ms))) { cleanup(); return fail(rc, "autotuner: timing run failed"); }
            if (ms < 0.99 * best) {
                best = ms;
                keep = v;
            }
        }
        *c.field = keep;
    }
    apply_tune(p);
    p->tuned_ms = best;
    cleanup();
    return PAT_OK;
}

int autotune(pat_plan_s* p, const char* path)
{
    const std::string key = tune_key(p);
    if (tune_lookup(p, path, key)) {
        apply_tune(p);
        p->tuned = 2;
        return PAT_OK;
    }
    int rc = (p->H.P.dt == PAT_F64) ? tune_search<double, 13>(p, p->dd) : tune_search<float, 6>(p, p->df);
    if (rc) return rc;
    p->tuned = 1;
    tune_store(p, path, key);
    return PAT_OK;
}

int lds_ok(const pat::Params& P, std::string& err)
{
    size_t cs = (P.dt == PAT_F64) ? 16 : 8;
    size_t need = std::max({cs * P.Ng, ring_lds(P, 1), cs * (size_t)P.M, cs * 2 * (size_t)P.mf});
    int longest = std::max({P.Ng, P.max_ring, P.mf3 ? 0 : P.mf});
    const int mf3_points = (FFT_REGS / 3) * 3 * NT;   // with a radix-3 pass
    if (need > 65536 || longest > FFT_BLOCK_POINTS || P.M > fft_points(P) || (P.mf3 && P.mf > mf3_points)) {
        err = "problem too large for the single-block LDS transforms (64 KiB, 4096 points)";
        return PAT_EUNSUPPORTED;
    }
    return PAT_OK;
}

void fill_info(const pat::Params& P, pat_plan_info* info, size_t ws_img, size_t table_bytes, const pat_plan_s* p)
{
    std::memset(info, 0, sizeof(*info));
    if (p) {
        info->tune_fft_radix_log2 = p->fft_lr;
        info->tune_cols_per_block = p->cols_cw;
        info->tune_dct_cols_per_block = p->dct_cw;
        info->tune_ring_images = p->ring_g;
        info->tune_spread_images = p->spread_bc;
        info->tune_twiddle_table = p->tw_table;
        info->tune_spread_staged = p->spread_staged;
        info->tune_dct_wave = p->df.dct_wave ? 1 : 0;
        info->tune_wave_fft = (p->df.wfRows || p->df.wfSynth) ? 1 : 0;
        info->tuned = p->tuned;
        info->tuned_ms = p->tuned_ms;
    }
    info->n = P.n; info->m = P.m; info->nt = P.nt; info->m_full = P.mf;
    info->grid = P.Ng; info->stencil = P.w; info->rings = P.L; info->dct_half = P.M;
    info->kmax = P.K; info->kpad = P.Kp; info->klow = P.klow; info->lcorr = P.lcorr;
    info->ring_points = P.npts; info->max_ring = P.max_ring; info->spread_tiles = ((P.Ew + 15) / 16) * ((P.Ng + 15) / 16);
    info->dlam = P.dlam; info->period = P.period; info->lambda_max = P.Lam;
    info->ws_per_image = ws_img; info->table_bytes = table_bytes;
}

}  // namespace

namespace pat {
int plan_device(pat_plan p) { return p ? p->device : -1; }

int plan_image_size(pat_plan p, int* n, int* nt, int* m, double* h, int* is_f64)
{
    if (!p) return PAT_EINVAL;
    *n = p->H.P.n;
    *nt = p->H.P.nt;
    *m = p->H.P.m;
    *h = p->H.P.h;
    *is_f64 = p->H.P.dt == PAT_F64;
    return PAT_OK;
}
}  // namespace pat

namespace {

// operators with a fused update step (contiguous batches)
int fused_args(pat_plan p, int B, const void* a, const void* b, const void* c, const void* ws, const char* who)
{
    if (!p || !a || !b || !c || !ws) return fail(PAT_EINVAL, std::string(who) + ": null pointer");
    if (B < 1 || B > p->max_batch) return fail(PAT_ESMALL, std::string(who) + ": B outside [1, max_batch]");
    return PAT_OK;
}

template <typename T, int WMAX>
int fused_call(pat_plan_s* p, bool adjoint, int B, const void* in, void* out, Epi<T> e, void* ws, void* stream)
{
    const pat::Params& P = p->H.P;
    Dev<T> d = dev_of(p, (T*)nullptr);
    d.epi = e;
    const long fs = (long)P.n * P.n, gs = (long)P.nt * P.m;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (adjoint) return run_adjoint<T, WMAX>(p, d, B, (const T*)in, gs, (T*)out, fs, (char*)ws, st);
    return run_forward<T, WMAX>(p, d, B, (const T*)in, fs, (T*)out, gs, (char*)ws, st);
}

template <typename T>
Epi<T> epi_of(int kind, const void* g, double sigma, void* f, void* fbar, const void* pgrad, const void* support,
                     double tau, double theta, double h)
{
    Epi<T> e{};
    e.kind = kind;
    e.g = static_cast<const T*>(g);
    e.sigma = (T)sigma;
    e.inv1ps = T(1) / (T(1) + e.sigma);
    e.f = static_cast<T*>(f);
    e.fbar = static_cast<T*>(fbar);
    e.p = static_cast<const T*>(pgrad);
    e.support = static_cast<const T*>(support);
    e.tau = (T)tau;
    e.theta = (T)theta;
    e.inv_h = (T)(1.0 / h);
    return e;
}

}  // namespace

extern "C" {

const char* pat_status_string(int code)
{
    switch (code) {
        case PAT_OK: return "ok";
        case PAT_EINVAL: return "invalid argument";
        case PAT_EUNSUPPORTED: return "unsupported configuration";
        case PAT_ENOMEM: return "out of memory";
        case PAT_EHIP: return "HIP runtime error";
        case PAT_ESMALL: return "workspace or batch too small";
        default: return "unknown status";
    }
}

const char* pat_last_error(void) { return pat::last_error(); }

int pat_debug_bessel(double x, int K, double* out)
{
    if (!out || K < 0) return fail(PAT_EINVAL, "pat_debug_bessel: bad arguments");
    pat::bessel_j_all(x, K, out);
    return PAT_OK;
}

int pat_plan_query(const pat_geometry* g, pat_dtype dt, pat_plan_info* info)
{
    if (!g || !info) return fail(PAT_EINVAL, "pat_plan_query: null argument");
    pat_plan_s tmp;
    std::string err;
    int rc = pat::build_host_plan(*g, dt, tmp.H, err);
    if (rc) return fail(rc, err);
    if ((rc = lds_ok(tmp.H.P, err))) return fail(rc, err);
    layout(&tmp);
    default_tune(&tmp);
    fill_info(tmp.H.P, info, tmp.ws_img, 0, &tmp);
    return PAT_OK;
}

int pat_plan_create(pat_plan* out, const pat_geometry* g, pat_dtype dt, int max_batch, const char* tuning_cache_path)
{
    if (!out) return fail(PAT_EINVAL, "pat_plan_create: out is NULL");
    *out = nullptr;
    if (!g) return fail(PAT_EINVAL, "pat_plan_create: geometry is NULL");
    if (max_batch < 1) return fail(PAT_EINVAL, "pat_plan_create: max_batch must be >= 1");
    std::unique_ptr<pat_plan_s> p(new pat_plan_s());
    std::string err;
    int rc = pat::build_host_plan(*g, dt, p->H, err);
    if (rc) return fail(rc, err);
    if ((rc = lds_ok(p->H.P, err))) return fail(rc, err);
    if (p->H.P.w != (dt == PAT_F64 ? 13 : 6)) return fail(PAT_EUNSUPPORTED, "stencil width does not match the compiled kernels");
    p->max_batch = max_batch;
    layout(p.get());
    default_tune(p.get());
    if (hipGetDevice(&p->device) != hipSuccess) return fail(PAT_EHIP, "pat_plan_create: no HIP device");
    rc = (dt == PAT_F64) ? upload<double>(p.get(), p->dd) : upload<float>(p.get(), p->df);
    if (rc) {
        for (void* a : p->allocs) (void)hipFree(a);
        return fail(rc, "pat_plan_create: table upload failed");
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        for (void* a : p->allocs) (void)hipFree(a);
        return fail(PAT_EHIP, "pat_plan_create: device synchronisation failed");
    }
    if (tuning_cache_path && tuning_cache_path[0]) {
        if ((rc = autotune(p.get(), tuning_cache_path))) {
            for (void* a : p->allocs) (void)hipFree(a);
            return rc;
        }
    }
    *out = p.release();
    return PAT_OK;
}

struct pat_group_s {
    std::vector<pat_plan_s*> plans;
    bool f64 = false;
};

int pat_group_create(pat_group* out, int count, const pat_plan* plans)
{
    if (!out) return fail(PAT_EINVAL, "pat_group_create: out is NULL");
    *out = nullptr;
    if (!plans || count < 1) return fail(PAT_EINVAL, "pat_group_create: need at least one plan");
    if (count > GROUP_MAX) return fail(PAT_EUNSUPPORTED, "pat_group_create: more plans than a group holds");
    std::unique_ptr<pat_group_s> g(new pat_group_s());
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) return fail(PAT_EINVAL, "pat_group_create: NULL plan");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(PAT_EINVAL, "pat_group_create: a plan appears twice");
        const bool f64 = plans[i]->H.P.dt == PAT_F64;
        if (i > 0 && f64 != g->f64) return fail(PAT_EINVAL, "pat_group_create: plans of different precision");
        if (i > 0 && plans[i]->device != g->plans[0]->device) return fail(PAT_EINVAL, "pat_group_create: plans on different devices");
        g->f64 = f64;
        g->plans.push_back(plans[i]);
    }
    *out = g.release();
    return PAT_OK;
}

int pat_group_destroy(pat_group g)
{
    if (!g) return fail(PAT_EINVAL, "pat_group_destroy: NULL group");
    delete g;
    return PAT_OK;
}

int pat_group_forward(pat_group g, const int* batch, const void* const* f, void* const* gout, void* const* ws,
                      void* stream)
{
    if (!g || !batch || !f || !gout || !ws) return fail(PAT_EINVAL, "pat_group_forward: null argument");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return g->f64 ? group_run<double, 13>(g->plans, false, batch, f, gout, ws, st)
                  : group_run<float, 6>(g->plans, false, batch, f, gout, ws, st);
}

int pat_group_adjoint(pat_group g, const int* batch, const void* const* gin, void* const* f, void* const* ws,
                      void* stream)
{
    if (!g || !batch || !gin || !f || !ws) return fail(PAT_EINVAL, "pat_group_adjoint: null argument");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return g->f64 ? group_run<double, 13>(g->plans, true, batch, gin, f, ws, st)
                  : group_run<float, 6>(g->plans, true, batch, gin, f, ws, st);
}

int pat_plan_destroy(pat_plan p)
{
    if (!p) return fail(PAT_EINVAL, "pat_plan_destroy: NULL plan");
    for (void* a : p->allocs) (void)hipFree(a);
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    delete p;
    return PAT_OK;
}

int pat_plan_get_info(pat_plan p, pat_plan_info* info)
{
    if (!p || !info) return fail(PAT_EINVAL, "pat_plan_get_info: null argument");
    fill_info(p->H.P, info, p->ws_img, p->table_bytes, p);
    return PAT_OK;
}

int pat_workspace_size(pat_plan p, int batch, size_t* bytes)
{
    if (!p || !bytes) return fail(PAT_EINVAL, "pat_workspace_size: null argument");
    if (batch < 1 || batch > p->max_batch) return fail(PAT_ESMALL, "pat_workspace_size: batch outside [1, max_batch]");
    *bytes = p->ws_img * (size_t)batch;
    return PAT_OK;
}

int pat_adjoint_scale(pat_plan p, double* s)
{
    if (!p || !s) return fail(PAT_EINVAL, "pat_adjoint_scale: null argument");
    *s = p->H.P.adj_scale;
    return PAT_OK;
}

int pat_forward_batched(pat_plan p, int B, const void* f, long f_stride, void* g, long g_stride, void* ws,
                        void* stream)
{
    if (!p || !f || !g || !ws) return fail(PAT_EINVAL, "pat_forward_batched: null pointer");
    const pat::Params& P = p->H.P;
    if (B < 1 || B > p->max_batch) return fail(PAT_ESMALL, "pat_forward_batched: B outside [1, max_batch]");
    if (f_stride < (long)P.n * P.n || g_stride < (long)P.nt * P.m)
        return fail(PAT_EINVAL, "pat_forward_batched: stride smaller than one image");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (P.dt == PAT_F64)
        return run_forward<double, 13>(p, p->dd, B, (const double*)f, f_stride, (double*)g, g_stride, (char*)ws, st);
    return run_forward<float, 6>(p, p->df, B, (const float*)f, f_stride, (float*)g, g_stride, (char*)ws, st);
}

int pat_adjoint_batched(pat_plan p, int B, const void* g, long g_stride, void* f, long f_stride, void* ws,
                        void* stream)
{
    if (!p || !f || !g || !ws) return fail(PAT_EINVAL, "pat_adjoint_batched: null pointer");
    const pat::Params& P = p->H.P;
    if (B < 1 || B > p->max_batch) return fail(PAT_ESMALL, "pat_adjoint_batched: B outside [1, max_batch]");
    if (f_stride < (long)P.n * P.n || g_stride < (long)P.nt * P.m)
        return fail(PAT_EINVAL, "pat_adjoint_batched: stride smaller than one image");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (P.dt == PAT_F64)
        return run_adjoint<double, 13>(p, p->dd, B, (const double*)g, g_stride, (double*)f, f_stride, (char*)ws, st);
    return run_adjoint<float, 6>(p, p->df, B, (const float*)g, g_stride, (float*)f, f_stride, (char*)ws, st);
}

int pat_forward_residual(pat_plan p, int B, const void* f, const void* g, void* r, void* ws, void* stream)
{
    int rc;
    if ((rc = fused_args(p, B, f, g, r, ws, "pat_forward_residual"))) return rc;
    if (p->H.P.dt == PAT_F64)
        return fused_call<double, 13>(p, false, B, f, r, epi_of<double>(EPI_RESIDUAL, g, 0, 0, 0, 0, 0, 0, 0, 1), ws, stream);
    return fused_call<float, 6>(p, false, B, f, r, epi_of<float>(EPI_RESIDUAL, g, 0, 0, 0, 0, 0, 0, 0, 1), ws, stream);
}

int pat_forward_cp_dual(pat_plan p, int B, const void* fbar, const void* g, void* q, double sigma, void* ws, void* stream)
{
    int rc;
    if ((rc = fused_args(p, B, fbar, g, q, ws, "pat_forward_cp_dual"))) return rc;
    if (!(sigma > 0)) return fail(PAT_EINVAL, "pat_forward_cp_dual: sigma must be positive");
    if (p->H.P.dt == PAT_F64)
        return fused_call<double, 13>(p, false, B, fbar, q, epi_of<double>(EPI_CP_DUAL, g, sigma, 0, 0, 0, 0, 0, 0, 1),
                                      ws, stream);
    return fused_call<float, 6>(p, false, B, fbar, q, epi_of<float>(EPI_CP_DUAL, g, sigma, 0, 0, 0, 0, 0, 0, 1), ws,
                                stream);
}

int pat_adjoint_nnls(pat_plan p, int B, const void* r, void* f, double tau, const void* support, void* ws, void* stream)
{
    int rc;
    if ((rc = fused_args(p, B, r, f, f, ws, "pat_adjoint_nnls"))) return rc;
    if (p->H.P.dt == PAT_F64)
        return fused_call<double, 13>(p, true, B, r, f, epi_of<double>(EPI_NNLS, 0, 0, f, 0, 0, support, tau, 0, 1), ws,
                                      stream);
    return fused_call<float, 6>(p, true, B, r, f, epi_of<float>(EPI_NNLS, 0, 0, f, 0, 0, support, tau, 0, 1), ws, stream);
}

int pat_adjoint_cp_primal(pat_plan p, int B, const void* q, const void* pgrad, void* f, void* fbar, double tau,
                          double theta, const void* support, void* ws, void* stream)
{
    int rc;
    if ((rc = fused_args(p, B, q, pgrad, f, ws, "pat_adjoint_cp_primal"))) return rc;
    if (!fbar) return fail(PAT_EINVAL, "pat_adjoint_cp_primal: null pointer");
    const double h = p->H.P.h;
    if (p->H.P.dt == PAT_F64)
        return fused_call<double, 13>(p, true, B, q, f,
                                      epi_of<double>(EPI_CP_PRIMAL, 0, 0, f, fbar, pgrad, support, tau, theta, h), ws, stream);
    return fused_call<float, 6>(p, true, B, q, f, epi_of<float>(EPI_CP_PRIMAL, 0, 0, f, fbar, pgrad, support, tau, theta, h),
                                ws, stream);
}

int pat_inverse_batched(pat_plan p, int B, const void* g, long g_stride, void* f, long f_stride, void* ws,
                        void* stream)
{
    if (!p || !f || !g || !ws) return fail(PAT_EINVAL, "pat_inverse_batched: null pointer");
    const pat::Params& P = p->H.P;
    if (B < 1 || B > p->max_batch) return fail(PAT_ESMALL, "pat_inverse_batched: B outside [1, max_batch]");
    if (f_stride < (long)P.n * P.n || g_stride < (long)P.nt * P.m)
        return fail(PAT_EINVAL, "pat_inverse_batched: stride smaller than one image");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (P.dt == PAT_F64)
        return run_inverse<double, 13>(p, p->dd, B, (const double*)g, g_stride, (double*)f, f_stride, (char*)ws, st);
    return run_inverse<float, 6>(p, p->df, B, (const float*)g, g_stride, (float*)f, f_stride, (char*)ws, st);
}

int pat_inverse(pat_plan p, const void* g, void* f, void* ws, void* stream)
{
    if (!p) return fail(PAT_EINVAL, "pat_inverse: NULL plan");
    return pat_inverse_batched(p, 1, g, (long)p->H.P.nt * p->H.P.m, f, (long)p->H.P.n * p->H.P.n, ws, stream);
}

int pat_timing_start(pat_plan p)
{
    return pat_timing_start_stages(p, ~0u);
}

int pat_timing_start_stages(pat_plan p, unsigned stage_mask)
{
    if (!p) return fail(PAT_EINVAL, "pat_timing_start: NULL plan");
    p->timing = true;
    p->timing_mask = stage_mask;
    p->ev_used = 0;
    return PAT_OK;
}

int pat_timing_stop(pat_plan p, double* ms, int* launches, int nstages)
{
    if (!p || !ms || !launches || nstages < PAT_NUM_STAGES) return fail(PAT_EINVAL, "pat_timing_stop: bad arguments");
    for (int i = 0; i < nstages; ++i) { ms[i] = 0.0; launches[i] = 0; }
    for (size_t i = 0; i < p->ev_used; ++i) {
        if (hipEventSynchronize(p->ev_pool[2 * i + 1]) != hipSuccess) return fail(PAT_EHIP, "pat_timing_stop: event sync failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, p->ev_pool[2 * i], p->ev_pool[2 * i + 1]) != hipSuccess)
            return fail(PAT_EHIP, "pat_timing_stop: elapsed time failed");
        ms[p->ev_stage[i]] += t;
        launches[p->ev_stage[i]] += 1;
    }
    p->timing = false;
    p->ev_used = 0;
    return PAT_OK;
}

int pat_filter_length(int nt, int* N)
{
    if (!N || nt < 1) return fail(PAT_EINVAL, "pat_filter_length: bad arguments");
    long L = 1;
    while (L < 2L * nt) L *= 2;
    *N = (int)std::min<long>(L, 1L << 30);
    return PAT_OK;
}

int pat_filter_create(pat_filter* out, int nt, double T, int m, double gamma, const double* eta, int neta,
                      pat_dtype dt)
{
    if (!out || !eta) return fail(PAT_EINVAL, "pat_filter_create: null argument");
    *out = nullptr;
    if (nt < 1 || m < 1 || !(T > 0.0) || !std::isfinite(T) || !std::isfinite(gamma))
        return fail(PAT_EINVAL, "pat_filter_create: need nt >= 1, m >= 1, finite T > 0 and finite gamma");
    if (dt != PAT_F32 && dt != PAT_F64) return fail(PAT_EINVAL, "pat_filter_create: bad dtype");
    int N = 0;
    pat_filter_length(nt, &N);
    if (N > FFT_BLOCK_POINTS)
        return fail(PAT_EUNSUPPORTED, "pat_filter_create: nt > " + std::to_string(FFT_BLOCK_POINTS / 2) +
                                          " (single-block transform)");
    if (neta != N / 2 + 1)
        return fail(PAT_EINVAL, "pat_filter_create: eta must hold N/2 + 1 = " + std::to_string(N / 2 + 1) +
                                    " complex values (N = pat_filter_length(nt))");
    for (int k = 0; k < 2 * neta; ++k)
        if (!std::isfinite(eta[k])) return fail(PAT_EINVAL, "pat_filter_create: eta is not finite");
    // the response on the whole DFT circle (real filter: eta(-xi) = conj(eta(xi)),
    // real at 0 and N/2), with the inverse transform's 1/N folded in
    std::vector<double> H(2 * (size_t)N), tw(2 * (size_t)N), att(nt);
    for (int k = 0; k < N; ++k) {
        const int kk = k <= N / 2 ? k : N - k;
        double re = eta[2 * kk], im = (kk == 0 || kk == N / 2) ? 0.0 : eta[2 * kk + 1];
        if (k > N / 2) im = -im;
        H[2 * k] = re / N;
        H[2 * k + 1] = im / N;
        const double a = -2.0 * M_PI * k / N;
        tw[2 * k] = std::cos(a);
        tw[2 * k + 1] = std::sin(a);
    }
    for (int j = 0; j < nt; ++j) att[j] = std::exp(-gamma * (j + 1) * T / nt);
    auto* f = new (std::nothrow) pat_filter_s();
    if (!f) return fail(PAT_ENOMEM, "pat_filter_create: out of host memory");
    f->nt = nt; f->m = m; f->N = N; f->dt = dt;
    // detectors per block: pairs of traces, as many sequences as 32 KiB of LDS
    // holds (at most 8; more LDS per block costs occupancy: measured slower)
    const size_t cs = dt == PAT_F64 ? 16 : 8;
    int cw = 2 * (int)std::max<size_t>(1, std::min<size_t>(8, 32768 / (cs * (size_t)N)));
    f->cw = cw;
    if (hipGetDevice(&f->device) != hipSuccess) { delete f; return fail(PAT_EHIP, "pat_filter_create: no device"); }
    auto put = [&](const std::vector<double>& v, bool f64, const void** dst) -> int {
        const size_t es = f64 ? 8 : 4;
        void* ptr = nullptr;
        if (hipMalloc(&ptr, std::max<size_t>(16, v.size() * es)) != hipSuccess) return PAT_ENOMEM;
        f->allocs.push_back(ptr);
        hipError_t e;
        if (f64) {
            e = hipMemcpy(ptr, v.data(), v.size() * 8, hipMemcpyHostToDevice);
        } else {
            std::vector<float> c(v.begin(), v.end());
            e = hipMemcpy(ptr, c.data(), c.size() * 4, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) return PAT_EHIP;
        *dst = ptr;
        return PAT_OK;
    };
    const bool f64 = dt == PAT_F64;
    const void *dH = nullptr, *dtw = nullptr, *datt = nullptr;
    int rc;
    if ((rc = put(H, f64, &dH)) || (rc = put(tw, f64, &dtw)) || (rc = put(att, f64, &datt))) {
        pat_filter_destroy(f);
        return fail(rc, "pat_filter_create: device allocation or copy failed");
    }
    int lcw = 0;
    while ((1 << lcw) < cw) ++lcw;
    int logN = 0;
    while ((1 << logN) < N) ++logN;
    if (f64) f->dd = FiltDev<double>{nt, m, N, logN, cw, lcw, 4, (const cx<double>*)dH, (const cx<double>*)dtw,
                                     (const double*)datt};
    else f->df = FiltDev<float>{nt, m, N, logN, cw, lcw, 4, (const cx<float>*)dH, (const cx<float>*)dtw,
                                (const float*)datt};
    *out = f;
    return PAT_OK;
}

int pat_filter_destroy(pat_filter f)
{
    if (!f) return PAT_OK;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev != f->device) (void)hipSetDevice(f->device);
    for (void* ptr : f->allocs) (void)hipFree(ptr);
    if (dev != f->device) (void)hipSetDevice(dev);
    delete f;
    return PAT_OK;
}

int pat_filter_apply(pat_filter f, int adjoint, int B, const void* in, long in_stride, void* out, long out_stride,
                     void* stream)
{
    if (!f || !in || !out) return fail(PAT_EINVAL, "pat_filter_apply: null pointer");
    const long img = (long)f->nt * f->m;
    if (B < 1 || in_stride < img || out_stride < img)
        return fail(PAT_EINVAL, "pat_filter_apply: need B >= 1 and strides >= nt*m");
    const size_t es = f->dt == PAT_F64 ? 8 : 4;
    const char* a0 = (const char*)in;
    const char* a1 = a0 + ((size_t)(B - 1) * in_stride + img) * es;
    const char* b0 = (const char*)out;
    const char* b1 = b0 + ((size_t)(B - 1) * out_stride + img) * es;
    const bool overlap = a0 < b1 && b0 < a1;
    if (overlap && !(a0 == b0 && in_stride == out_stride))
        return fail(PAT_EINVAL, "pat_filter_apply: input and output overlap (in place needs the same pointer and stride)");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid((f->m + f->cw - 1) / f->cw, B);
    const size_t lds = (size_t)(f->cw / 2) * f->N * (f->dt == PAT_F64 ? 16 : 8);
    if (f->dt == PAT_F64)
        trace_filter<double><<<grid, NT, lds, st>>>(f->dd, (const double*)in, in_stride, (double*)out, out_stride,
                                                   adjoint ? 1 : 0);
    else
        trace_filter<float><<<grid, NT, lds, st>>>(f->df, (const float*)in, in_stride, (float*)out, out_stride,
                                                  adjoint ? 1 : 0);
    return check_launch("trace_filter");
}

int pat_forward(pat_plan p, const void* f, void* g, void* ws, void* stream)
{
    if (!p) return fail(PAT_EINVAL, "pat_forward: NULL plan");
    return pat_forward_batched(p, 1, f, (long)p->H.P.n * p->H.P.n, g, (long)p->H.P.nt * p->H.P.m, ws, stream);
}

int pat_adjoint(pat_plan p, const void* g, void* f, void* ws, void* stream)
{
    if (!p) return fail(PAT_EINVAL, "pat_adjoint: NULL plan");
    return pat_adjoint_batched(p, 1, g, (long)p->H.P.nt * p->H.P.m, f, (long)p->H.P.n * p->H.P.n, ws, stream);
}

}  // extern "C"
