/*
 * pat.h -- C ABI of the MI355X (gfx950) library for the fast circular-geometry
 * photoacoustic operators of Hauptmann, Kunyansky & Poimala,
 * "Fast algorithms enabling optimization and deep learning for photoacoustic
 * tomography in a circular detection geometry" (arXiv 2510.24687).
 *
 * Operators
 *   A  : initial pressure f on an n x n grid  ->  traces g(t_j, z_i) on the
 *        detector circle (the wave operator of Sec. 2.1, eq. E:green_conv),
 *        evaluated in O(n^2 log n) by the harmonic route of Sec. 3.1
 *        (Algorithm 1: 2D FFT, Cartesian->polar interpolation, angular FFT
 *        per ring, Bessel-weighted cosine transform per harmonic, angular
 *        synthesis per time sample, restriction to the arc).
 *   A* : the adjoint of A under the L2 inner products of eq.
 *        eqn:innerProducts (Sec. 2.1, eq. E:adjoint), computed as the exact
 *        weighted transpose of the discrete A: A* = s A^T with
 *        s = (T/nt)(R*arc/m)/h^2 (Algorithm 2 of Sec. 3.2 in transposed
 *        form; see pat_adjoint_scale).
 *
 * Discrete model.  A sampled image is the band-limited function whose 2D
 * Fourier transform is W(|xi|) F(xi), F(xi) = (h^2/2pi) sum_pq f_pq
 * exp(-i xi.x_pq) (the transform convention of Sec. 2.1.1), W a smooth radial
 * taper equal to 1 on [0, taper_rho*Lambda] and 0 from Lambda = pi/h on.
 * The returned traces are the exact wave solution (eq. E:kwave) for that
 * function, up to the algorithm's approximation error (bounded per plan; FP32
 * plans stay below 1e-5 relative L2 before rounding).
 *
 * Layout and conventions
 *   pixel centres  x_pq = (-a + (q+1/2)h, -a + (p+1/2)h), h = 2a/n;
 *   f              row-major f[p*n + q] (p = y index, q = x index);
 *   detectors      theta_i = theta0 + i*arc/m, z_i = R (cos, sin)(theta_i),
 *                  i = 0..m-1; 2*pi*m/arc must be an integer m_full (the
 *                  detectors are a subset of m_full equispaced angles);
 *   times          t_j = (j+1) T/nt, j = 0..nt-1 (samples on (0, T]);
 *   g              row-major g[j*m + i] (time-major, detector fastest);
 *   batches        image b of a batch starts at f + b*f_stride (elements),
 *                  its traces at g + b*g_stride.
 *   precision      PAT_F32 plans read/write float, PAT_F64 plans double.
 *
 * Ownership.  The caller owns every buffer passed in (inputs, outputs and the
 * workspace; all device memory).  A plan owns its device tables and frees
 * them in pat_plan_destroy.  Plans are immutable after creation.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  All
 * compute calls are asynchronous on it: they enqueue kernels and return.
 * Two calls that run concurrently must use distinct workspaces.
 *
 * Errors.  Every function returns PAT_OK (0) or a negative status; nothing
 * throws across the ABI.  pat_last_error() returns a thread-local detail
 * string for the most recent failure on the calling thread.
 */
#ifndef PAT_H
#define PAT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PAT_OK = 0,
    PAT_EINVAL = -1,       /* invalid argument (null pointer, bad size, bad geometry) */
    PAT_EUNSUPPORTED = -2, /* valid but unsupported configuration (e.g. m_full not a power of two) */
    PAT_ENOMEM = -3,       /* device or host allocation failed */
    PAT_EHIP = -4,         /* a HIP runtime call or kernel launch failed */
    PAT_ESMALL = -5        /* workspace or batch capacity too small */
};

typedef enum { PAT_F32 = 0, PAT_F64 = 1 } pat_dtype;

/* Acquisition geometry (problem statement of Sec. 2: speed of sound c,
 * detector circle of radius R, m detectors on an arc Gamma of the circle,
 * nt samples on (0, T]); image grid n x n on [-a, a]^2. */
typedef struct {
    int n;              /* image is n x n, n >= 8                               */
    double a;           /* image half-width (image covers [-a, a]^2)            */
    double R;           /* detector-circle radius                               */
    double c;           /* speed of sound                                       */
    int m;              /* number of detectors                                  */
    double theta0;      /* angle of detector 0 (radians)                        */
    double arc;         /* angular extent covered: detector spacing is arc/m    */
    int nt;             /* number of time samples                               */
    double T;           /* final time                                           */
    double taper_rho;   /* W = 1 on [0, taper_rho*Lambda]; 0 < taper_rho < 1    */
    double mask_radius; /* 0: none; else f restricted to |x| <= mask_radius in
                           A and A* (the projection Pi_Omega0 of Algorithm 2)   */
} pat_geometry;

typedef struct pat_plan_s* pat_plan;

/* Parameters the plan chose (for diagnostics and tests). */
typedef struct {
    int n, m, nt, m_full;
    int grid;           /* oversampled Cartesian FFT size (per side)             */
    int stencil;        /* interpolation stencil width w (cells per direction)   */
    int rings;          /* number of polar rings L (lambda_l = l*dlam < Lambda)  */
    int dct_half;       /* M: the cosine transform uses a 2M-point FFT           */
    int kmax;           /* largest angular harmonic K                            */
    int kpad;           /* harmonic row pitch (K+1 rounded up)                   */
    int klow;           /* harmonics 0..klow get the low-frequency correction    */
    int lcorr;          /* rings entering the low-frequency correction           */
    int ring_points;    /* half-ring sample count summed over rings              */
    int max_ring;       /* largest ring FFT size                                 */
    int spread_tiles;   /* tiles of the adjoint's deterministic spread           */
    double dlam;        /* ring spacing in lambda                                */
    double period;      /* time period 2*pi/(c*dlam) of the cosine transform     */
    double lambda_max;  /* Lambda = pi/h                                         */
    size_t ws_per_image;/* workspace bytes per image                             */
    size_t table_bytes; /* device bytes held by the plan                         */
    /* launch shapes in use (defaults from the LDS limits, or the autotuner's)   */
    int tune_fft_radix_log2;      /* largest FFT pass radix 2^x (3 or 4)            */
    int tune_cols_per_block;      /* spectrum columns per column-FFT block          */
    int tune_dct_cols_per_block;  /* harmonics per cosine-transform block           */
    int tune_ring_images;         /* images per ring-gather block                   */
    int tune_spread_images;       /* images per spread group                        */
    int tune_twiddle_table;       /* 1: FFT passes read every twiddle from a table,
                                     0: derive them from four table entries         */
    int tune_spread_staged;       /* spread form: 2 (FP32 only) samples sorted by
                                     the cell of their first tap, each lane walking
                                     its own runs, with the binned gather in the
                                     forward; 1 tiles staging samples through LDS;
                                     0 tiles reading them with scalar loads         */
    int tune_dct_wave;            /* 1: the FP32 cosine transform runs one wave per
                                     column group with compile-time lengths         */
    int tune_wave_fft;            /* 1: the FP32 row / column / angular FFT kernels
                                     run one wave per sequence                      */
    int tuned;                    /* 0 defaults, 1 measured at creation, 2 cached   */
    double tuned_ms;              /* forward + adjoint ms at max_batch when tuned   */
} pat_plan_info;

/* Create a plan: validates the geometry, computes its tables on the host in
 * FP64 (Bessel functions by Miller's backward recurrence, gridding kernel and
 * its transform, low-frequency quadrature, sample positions) and uploads them.
 * max_batch bounds the batch of later calls (>= 1).
 * tuning_cache_path: NULL or "" keeps the default launch shapes.  Otherwise
 * the plan looks up its key (device architecture, dtype, geometry, max_batch)
 * in that text file (one line per entry, "key | choices"; the last matching
 * line wins); if absent it times the candidate launch shapes (FFT pass radix,
 * twiddle source, columns per transform block, images per ring-gather block
 * and per spread group, spread sample staging, the wave-per-column cosine
 * transform) one choice at a time with forward + adjoint at max_batch (after
 * one discarded run, 8 timed pairs per candidate), keeps a candidate only if
 * it is more than 1 % faster than the current choice, and appends a line.  A missing or unreadable file is treated as
 * empty; a line that fails validation is ignored.  The search allocates and
 * frees a temporary workspace.
 * Synchronises the current device.  Returns PAT_OK and *out, or an error
 * (then *out is NULL). */
int pat_plan_create(pat_plan* out, const pat_geometry* g, pat_dtype dt, int max_batch,
                    const char* tuning_cache_path);

/* Same parameters and host tables as pat_plan_create, but no device work:
 * fills *info only.  Usable without a GPU. */
int pat_plan_query(const pat_geometry* g, pat_dtype dt, pat_plan_info* info);

int pat_plan_destroy(pat_plan p);
int pat_plan_get_info(pat_plan p, pat_plan_info* info);

/* Device workspace bytes needed for a batch of `batch` images (<= max_batch). */
int pat_workspace_size(pat_plan p, int batch, size_t* bytes);

/* g = A f for one image.  f: n*n device elements, g: nt*m device elements. */
int pat_forward(pat_plan p, const void* f, void* g, void* ws, void* stream);

/* f = A* g (weighted adjoint) for one image. */
int pat_adjoint(pat_plan p, const void* g, void* f, void* ws, void* stream);

/* Batched forms: B images (1 <= B <= max_batch), strides in elements
 * (f_stride >= n*n, g_stride >= nt*m). */
int pat_forward_batched(pat_plan p, int B, const void* f, long f_stride, void* g, long g_stride,
                        void* ws, void* stream);
int pat_adjoint_batched(pat_plan p, int B, const void* g, long g_stride, void* f, long f_stride,
                        void* ws, void* stream);

/* f = A^-1 g: the approximate inverse of Sec. 3.3 (Algorithm 3), for one
 * image and batched (same arguments and strides as pat_adjoint*).
 *   v(x) = 2 c^2 sum_{j,i} w_t w_th g[j][i] d/dn(z_i) G_W(t_j, x - z_i)
 * is the universal back-projection (eq. E:inverse truncated to the measured
 * times, eq. E:approx_UBP) with G_W the fundamental solution of the
 * band-limited model above (spectrum W(|xi|) sin(c|xi|t)/(2 pi c|xi|)),
 * w_t = T/nt, w_th = R*arc/m, and the normal n(z) pointing into the disk
 * (the sign with which the formula returns f; that of eq. E:Four_coef_v).
 * Arc data count as the full circle extended by zero (Alg. 3, step 1).  It is
 * evaluated like A*: angular FFT per time sample, sine transform per
 * harmonic times (-i)^k J_k'(lambda R) (eq. E:Four_coef_v), ring synthesis,
 * spread to the grid, inverse 2D FFT.  Then, with a mask (mask_radius > 0,
 * Omega_0 = the disk |x| <= mask_radius): C = -(mean of v over the pixel
 * centres with mask_radius < |x| <= R), eq. E:silly_integral, and
 * f = v + C on Omega_0, 0 outside.  Without a mask, f = v (Omega_0 is the
 * whole image, so no pixel lies in Omega \ Omega_0 and C = 0).
 * A^-1 is a left inverse for data of the full circle recorded long enough
 * (T well beyond the diameter), not the inverse of the discrete A.
 * Asynchronous on `stream`; capturable in a HIP graph; uses the same
 * workspace size as the adjoint. */
int pat_inverse(pat_plan p, const void* g, void* f, void* ws, void* stream);
int pat_inverse_batched(pat_plan p, int B, const void* g, long g_stride, void* f, long f_stride,
                        void* ws, void* stream);

/* ---- Measurement operator B (eq. E:real_meas, Sec. 2) --------------------
 * Real data are the ideal traces damped by e^{-gamma t} and passed through
 * the transducer's frequency response eta (a 1D Fourier filter in t, the
 * same for every detector):  B g = D(e^{-gamma t} g),  D h = F^-1(eta F h).
 * Discretisation: each trace (t_j = (j+1) T/nt) is zero-extended to
 * N = pat_filter_length(nt) samples (the smallest power of two >= 2 nt), so
 * that the filter's wrap-around does not fold the end of a record into its
 * start; F is the N-point DFT, the result is cut back to the nt samples.
 * eta is given at the N/2 + 1 frequencies xi_k = 2 pi k / (N T/nt),
 * k = 0..N/2, as (re, im) pairs; the negative frequencies are the
 * conjugates (a real filter) and the imaginary parts at k = 0 and N/2 are
 * ignored.  The adjoint under the trace inner product is
 * B* g = e^{-gamma t} F^-1(conj(eta) F g) (same extension and cut).
 * The operator acts on time-major traces (nt x m, detector fastest) and
 * commutes with everything A does per time sample, so B A f is
 * pat_forward then pat_filter_apply, and A* B* g the reverse.
 * Limits: nt <= 2048 (one-block transform).  The filter keeps its own
 * device tables (eta on the DFT circle, twiddles, e^{-gamma t_j}) on the
 * device current at creation. */
typedef struct pat_filter_s* pat_filter;
int pat_filter_length(int nt, int* N);
int pat_filter_create(pat_filter* out, int nt, double T, int m, double gamma, const double* eta, int neta,
                      pat_dtype dt);
int pat_filter_destroy(pat_filter f);
/* B (adjoint = 0) or B* (adjoint = 1) on B traces: in / out device arrays of
 * the filter's dtype, image b at in + b*in_stride (elements, >= nt*m).
 * In place when out == in with the same stride; any other overlap is
 * rejected (PAT_EINVAL).  Asynchronous on `stream`; capturable. */
int pat_filter_apply(pat_filter f, int adjoint, int B, const void* in, long in_stride, void* out, long out_stride,
                     void* stream);

/* ---- Groups of plans (batching of uneven image sizes) --------------------
 * A group runs the forward (or adjoint) chains of up to 5 plans of the same
 * precision together: each stage is ONE kernel launch whose blocks cover
 * every plan's grid (13 launches per A + A* pair for the whole group, 14
 * with binned FP32 plans, instead of that many per plan), with results
 * identical to per-plan calls.  The group
 * keeps pointers to the plans (they must outlive it; each plan at most once)
 * and uses their launch shapes, except that the spread takes its widest image
 * group.  Per plan i: batch[i] images (1..max_batch),
 * contiguous inputs / outputs (image stride n*n, trace stride nt*m), and its
 * own workspace ws[i] of pat_workspace_size(plan_i, batch[i]) bytes.
 * Asynchronous on `stream`; capturable in a HIP graph. */
typedef struct pat_group_s* pat_group;
int pat_group_create(pat_group* out, int count, const pat_plan* plans);
int pat_group_destroy(pat_group g);
int pat_group_forward(pat_group g, const int* batch, const void* const* f, void* const* gout, void* const* ws,
                      void* stream);
int pat_group_adjoint(pat_group g, const int* batch, const void* const* gin, void* const* f, void* const* ws,
                      void* stream);

/* s such that A* = s A^T: s = (T/nt) (R*arc/m) / h^2, the rectangle-rule
 * weights of the inner products eqn:innerProducts. */
int pat_adjoint_scale(pat_plan p, double* s);

const char* pat_status_string(int code);
const char* pat_last_error(void);

/* Stage timing.  Stages of the forward and adjoint chains, in launch order;
 * PAT_STAGE_GATHER_FWD (the FP32 binned gather, launched between COLS_FWD and
 * RING_FWD when tune_spread_staged == 2) is numbered last. */
enum {
    PAT_STAGE_ROWS_FWD = 0, PAT_STAGE_COLS_FWD, PAT_STAGE_RING_FWD, PAT_STAGE_DCT_FWD, PAT_STAGE_LOWK_FWD,
    PAT_STAGE_SYNTH_FWD, PAT_STAGE_SYNTH_ADJ, PAT_STAGE_LOWK_ADJ, PAT_STAGE_DCT_ADJ, PAT_STAGE_RING_ADJ,
    PAT_STAGE_SPREAD_ADJ, PAT_STAGE_COLS_ADJ, PAT_STAGE_ROWS_ADJ, PAT_STAGE_GATHER_FWD, PAT_NUM_STAGES
};

/* Start recording a HIP event pair on the launch stream around every kernel
 * of later pat_forward* / pat_adjoint* calls on this plan (no host syncs are
 * added).  pat_timing_stop waits for the recorded events, writes the summed
 * milliseconds and launch counts per stage into ms[] / launches[] (arrays of
 * at least PAT_NUM_STAGES entries) and turns recording off.  Not for plans
 * used from several threads at once. */
int pat_timing_start(pat_plan p);
int pat_timing_stop(pat_plan p, double* ms, int* launches, int nstages);
/* As pat_timing_start, with events only around the launches of the stages
 * whose bit (1u << stage) is set in stage_mask (the others run unrecorded). */
int pat_timing_start_stages(pat_plan p, unsigned stage_mask);

/* ---- Fused update steps of the iterative reconstructions (Sec. 4.2) ------
 * All operate on device arrays of the plan's precision, asynchronously on
 * `stream`; images are laid out as in pat_forward_batched (contiguous,
 * stride n*n for images, nt*m for traces).  `support` (may be NULL) is a
 * B x n x n array multiplied into the result (the projection Pi_Omega0). */

/* r = a x + b y over `count` elements (y may be NULL: r = a x). */
int pat_axpby(pat_plan p, long count, double a, const void* x, double b, const void* y, void* r, void* stream);

/* out[b] = sum_{i < count} x[b*stride + i] * y[b*stride + i] for b < B, in FP64
 * with a fixed summation order (deterministic); x, y of the plan's
 * precision.  out: B device doubles; scratch: 64*B device doubles.  Used for
 * the iterations' stopping rule (norm of an update, Sec. 4.3) and objectives. */
int pat_dot_batched(pat_plan p, int B, long count, long stride, const void* x, const void* y, double* out,
                    double* scratch, void* stream);

/* pat_dot_batched without a scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the 64 partial sums per image live in a
 * static device array of the library (2 MiB, one per GPU, held until the
 * process ends), so B <= 4096 (else PAT_EINVAL with a message).  Same
 * arguments, layout and result as pat_dot_batched (bit-identical); the plan's
 * device must be the current device.  Calls on one GPU share that array:
 * calls that overlap in time on one GPU (different streams, threads) race and
 * must be serialised by the caller.  Allocates nothing. */
int pat_dot_batched_noalloc(pat_plan p, int B, long count, long stride, const void* x, const void* y, double* out,
                            void* stream);

/* Projected gradient step of NNLS (eq:NNLS-projstep, eqn:projectionHalfCircle):
 * f = support * max(0, f - tau * grad) for B images. */
int pat_nnls_update(pat_plan p, int B, void* f, const void* grad, double tau, const void* support, void* stream);

/* Chambolle-Pock dual step for the data term 1/2 ||A f - g||^2 (eqn:PDHG-dual):
 * q = (q + sigma (Afbar - g)) / (1 + sigma), B trace arrays. */
int pat_cp_dual_data(pat_plan p, int B, void* q, const void* Afbar, const void* g, double sigma, void* stream);

/* Dual step for lam * TV: p = proj_{|p| <= lam}(p + sigma grad_h fbar); p holds
 * two n x n planes (x- then y-differences) per image; grad_h = forward
 * differences / h with a zero last difference. */
int pat_cp_dual_tv(pat_plan p, int B, void* pgrad, const void* fbar, double sigma, double lam, void* stream);

/* Primal step and extrapolation (eqn:PDHG-primal, eqn:PDHG-relaxation in the
 * usual Chambolle-Pock form): f_new = support * max(0, f - tau (Astar_q - div_h p)),
 * fbar = f_new + theta (f_new - f), f = f_new. */
int pat_cp_primal(pat_plan p, int B, void* f, void* fbar, const void* Astar_q, const void* pgrad, double tau,
                  double theta, const void* support, void* stream);

/* The operators with an update step fused into their last launch (the
 * synthesis of A, the row transforms of A*): one launch chain per iteration
 * half instead of the chain plus a separate pass over the traces or images.
 * Contiguous batches (B <= max_batch, images n*n apart, traces nt*m apart),
 * `workspace` as for pat_forward_batched; the arithmetic of the update equals
 * that of the separate kernels above. */

/* r = A f - g (the NNLS residual); r may be g. */
int pat_forward_residual(pat_plan p, int B, const void* f, const void* g, void* r, void* workspace, void* stream);

/* q = (q + sigma (A fbar - g)) / (1 + sigma) (eqn:PDHG-dual, data part); sigma > 0. */
int pat_forward_cp_dual(pat_plan p, int B, const void* fbar, const void* g, void* q, double sigma, void* workspace,
                        void* stream);

/* f = support * max(0, f - tau A* r) (eq:NNLS-projstep with the gradient A* r). */
int pat_adjoint_nnls(pat_plan p, int B, const void* r, void* f, double tau, const void* support, void* workspace,
                     void* stream);

/* f_new = support * max(0, f - tau (A* q - div_h p)), fbar = f_new + theta (f_new - f),
 * f = f_new (eqn:PDHG-primal, eqn:PDHG-relaxation as pat_cp_primal, with A* q
 * computed in the same chain); pgrad as in pat_cp_dual_tv. */
int pat_adjoint_cp_primal(pat_plan p, int B, const void* q, const void* pgrad, void* f, void* fbar, double tau,
                          double theta, const void* support, void* workspace, void* stream);

/* ---- Learned primal-dual reconstructor (Sec. 4.2.1, eqs. eq:LPD_dual,
 * eq:LPD_primal, loss eq:emp_loss) -----------------------------------------
 * The dual and primal networks are stacks of 3x3 convolutions (stride 1,
 * zero padding 1, cross-correlation) between tensors of two layouts:
 *   planar: up to 4 separate FP32 B x H x W planes (batch stride H*W), e.g.
 *           the LPD inputs q, A f, y or f, A* q, and the 1-channel outputs;
 *   NHWC:   B x H x W x 32 hidden feature maps or their gradients, channel
 *           fastest, stored as bfloat16 (the precision the matrix cores take).
 * Operands are rounded to bfloat16 (nearest-even) and multiplied on the
 * matrix cores with FP32 accumulation.  Weights are FP32 masters
 * w[cout][cin][3][3] packed by pat_conv_pack_weights.  All calls are
 * asynchronous on `stream`; pointers are device pointers owned by the caller.
 * Errors: PAT_EINVAL for null or inconsistent arguments, PAT_EUNSUPPORTED for
 * channel counts other than 1..4 (planar) / 32 (NHWC), PAT_EHIP on a launch
 * failure. */
typedef struct {
    int B, H, W;
    int cin, cout;        /* planar: 1..4; NHWC: 32                                */
    int in_planar;        /* input layout                                          */
    int out_planar;       /* output layout                                         */
    const void* in[4];    /* planar: FP32 in[0..cin-1]; NHWC: bf16 in[0]            */
    void* out[4];         /* planar: FP32 out[c] (NULL = not written); NHWC: bf16 out[0] */
    const void* residual[4]; /* planar outputs: added after scaling (NULL = none)   */
    float scale[4];       /* planar input: plane c is multiplied by scale[c];
                             planar output: out[c] = residual[c] + scale[c] * (conv + bias) */
    const void* weight;   /* packed bf16 weights (pat_conv_pack_weights)            */
    const void* bias;     /* FP32 [cout] or NULL                                    */
    const void* alpha;    /* FP32 [cout] PReLU slopes or NULL (NHWC outputs only)   */
    void* pre;            /* forward, NHWC outputs: FP32 NHWC copy of the
                             pre-activation, or NULL                                */
    const void* bwd_pre;  /* non-NULL selects the backward epilogue (NHWC output):
                             the convolution is an input gradient ga, and the
                             output is gx = ga * (bwd_pre > 0 ? 1 : alpha), the
                             gradient before the PReLU whose FP32 pre-activation
                             is bwd_pre; grad_bias_alpha[0..31] (+)= sum gx and
                             grad_bias_alpha[32..63] (+)= sum ga * bwd_pre *
                             [bwd_pre <= 0] (the bias and slope gradients)      */
    void* partials;       /* backward epilogue: pat_conv_bwd_partials floats      */
    void* grad_bias_alpha;/* backward epilogue: 64 FP32 outputs                   */
    int accumulate;       /* backward epilogue: 0 overwrite, 1 add               */
} pat_conv_desc;

/* Elements (bf16) of a packed weight array for an effective convolution with
 * cout_e outputs and cin_e inputs of the given layout; -1 if unsupported. */
long pat_conv_packed_size(int cout_e, int cin_e, int in_planar);

/* Pack w[cout][cin][3][3] (FP32, device) to bf16.  transpose = 0: the
 * forward convolution.  transpose = 1: the input-gradient convolution
 * (cin_e = cout, cout_e = cin, kernel flipped), so that the gradient with
 * respect to the layer input is pat_conv3x3 of the output gradient.
 * in_planar is the layout of the effective convolution's input. */
int pat_conv_pack_weights(const void* w, int cout, int cin, int transpose, int in_planar, void* dst, void* stream);

/* Forward epilogue: out = act(conv3x3(in) + bias) (NHWC out; act = PReLU if
 * alpha, pre gets the value before it) or out[c] = residual[c] + scale[c]
 * (conv3x3(in) + bias)[c] (planar out).  Backward epilogue: see bwd_pre. */
int pat_conv3x3(const pat_conv_desc* d, void* stream);

/* Floats of FP32 scratch the backward epilogue of pat_conv3x3 needs. */
long pat_conv_bwd_partials(const pat_conv_desc* d);

/* Floats of FP32 scratch pat_conv3x3_wgrad needs for this layer and chunking. */
long pat_conv_wgrad_partials(const pat_conv_desc* d, int rows_per_chunk);

/* Weight gradient of the layer d (d->in as in the forward, d->cout outputs):
 * grad_w[co][ci][ky][kx] (+)= sum_{b,y,x} grad_out[b,y,x,co] * in[b, y+ky-1,
 * x+kx-1, ci] (scaled planar inputs as in the forward), with operands rounded
 * to bf16 and the sum taken per chunk of rows_per_chunk image rows on the
 * matrix cores, then over chunks in FP64 in a fixed order (deterministic).
 * grad_out has d's output layout (planar FP32 needs cout == 1; NHWC bf16).
 * accumulate = 0 overwrites grad_w, 1 adds to it. */
int pat_conv3x3_wgrad(const pat_conv_desc* d, const void* grad_out, int rows_per_chunk, void* partials,
                      void* grad_w, int accumulate, void* stream);

/* out[0] (+)= sum of count FP32 values (the bias gradient of a 1-channel
 * planar layer); partials: nblocks floats of scratch. */
int pat_plane_sum(long count, const void* g, void* partials, int nblocks, void* out, int accumulate, void* stream);

/* One Adam step (bias-corrected first and second moments) over count FP32
 * parameters with step size lr_t = lr_min + (lr - lr_min) (1 + cos(pi s)) / 2,
 * s = min(1, (t-1) / (total_steps-1)), t = *step + 1 read from the device;
 * *step is then incremented on the device, so a captured step replays as is.
 * clip > 0 first scales the gradient by min(1, clip / ||grad||_2) (global
 * norm, computed on the device into `scratch`, >= 65 doubles); clip = 0
 * disables it (scratch may be NULL). */
int pat_adam(long count, void* param, const void* grad, void* m, void* v, void* step, double lr, double lr_min,
             int total_steps, double beta1, double beta2, double eps, double clip, void* scratch, void* stream);

/* ---- U-Net networks of the learned primal-dual reconstructor (Sec. 4.2.1:
 * four scales, three window-2 down- and up-sampling steps, two 3x3
 * convolutions each followed by batch normalisation and ReLU per scale, 32
 * filters at the first scale doubled at every down-sampling) ---------------
 * Layouts: activations are NHWC bfloat16 (B x H x W x C, channel fastest),
 * convolution outputs and activation gradients NHWC FP32.  Every product runs
 * on the matrix cores with bf16 operands and FP32 accumulation; every sum
 * (statistics, weight gradients) is deterministic.  Pointers are device
 * pointers owned by the caller; calls are asynchronous on `stream` and
 * capturable.  Errors: PAT_EINVAL for null or inconsistent arguments,
 * PAT_EUNSUPPORTED for channel counts the kernels do not take, PAT_EHIP on
 * a launch failure. */

/* A generic convolution as an implicit GEMM.  GEMM rows are the pixels
 * (b, y, x) of the iteration grid B x H x W.  Tap t (of ntaps) reads the
 * source pixel (in_stride y + dy[t], in_stride x + dx[t]) of the Hs x Ws
 * source grid (zero outside it); the reduction index is k = t cin + c over
 * the concatenated channels [src[0] (csrc[0]) | src[1] (csrc[1])], cin =
 * csrc[0] + csrc[1].  The row's cout results go to destination pixel
 * (out_stride y + oy, out_stride x + ox) of the Ho x Wo grid: channels
 * [0, cdst[0]) to dst[0] (pitch cdst[0]), the rest to dst[1] (pitch cdst[1]),
 * each either bf16 (dst_bf16) or FP32 (overwritten or, with accumulate,
 * added to).  Examples: a 3x3 convolution (zero padding 1) has taps
 * (t/3 - 1, t%3 - 1); its input gradient is the same with transposed,
 * flipped weights; the 2x2 stride-2 transposed convolution is one 1-tap GEMM
 * per output parity (out_stride 2, offset (i, j)); its input gradient has the
 * 4 taps (i, j) read at in_stride 2.  csrc[] and cout must be multiples of 16;
 * when csrc[0] + csrc[1] is a multiple of 32 each csrc[] must be one too
 * (the weights are then packed for the 32-deep matrix instruction). */
typedef struct {
    int B, H, W;                 /* iteration grid                           */
    const void* src[2];          /* NHWC bf16 sources (src[1] may be NULL)   */
    int csrc[2];                 /* their channel counts (csrc[1] may be 0)  */
    int Hs, Ws, in_stride;       /* source grid and stride                   */
    int ntaps;                   /* 1..9                                     */
    int dy[9], dx[9];            /* tap offsets                              */
    const void* weight;          /* pat_gconv_pack output for (cout, cin, ntaps) */
    int cout;                    /* GEMM columns                             */
    void* dst[2];                /* destinations                              */
    int cdst[2];                 /* channel split: cdst[0] + cdst[1] = cout   */
    int dst_bf16[2];             /* 1: store bf16, 0: FP32                    */
    int accumulate[2];           /* FP32 destinations: add instead of store   */
    int Ho, Wo;                  /* destination grid                          */
    int out_stride, oy, ox;      /* destination mapping                       */
} pat_gconv_desc;

/* bf16 elements of a packed weight array: cout * ntaps * cip (cout, cip
 * multiples of 16, ntaps 1..9), or -1. */
long pat_gconv_packed_size(int cout, int cip, int ntaps);

/* Pack FP32 weights to the layout pat_gconv reads: the effective weight of
 * output column co < co_e, input channel ci < ci_e and tap t is
 * w[off + co s_co + ci s_ci + t' s_t] with t' = flip ? ntaps - 1 - t : t;
 * columns co_e..cout-1 and channels ci_e..cip-1 are zero (padding). */
int pat_gconv_pack(const void* w, int co_e, int ci_e, int cout, int cip, int ntaps, long off, long s_co, long s_ci,
                   long s_t, int flip, void* dst, void* stream);

/* The convolution d (see pat_gconv_desc). */
int pat_gconv(const pat_gconv_desc* d, void* stream);

/* FP32 scratch floats pat_gconv_wgrad needs with `chunks` row chunks. */
long pat_gconv_wgrad_partials(const pat_gconv_desc* d, int chunks);

/* Weight gradient of the convolution d: for every column co and reduction
 * index k = t cin + ci, sum over the rows of grad[dest(row)][co] *
 * src[source(row, t)][ci] (grad: NHWC bf16 with pitch cout on d's
 * destination grid; d's dst fields are ignored), accumulated on the matrix
 * cores per chunk of rows, then over the chunks in FP64 in a fixed order;
 * written (accumulate = 0) or added to dw[off + co s_co + ci s_ci + t s_t]
 * for ci < ci_real. */
int pat_gconv_wgrad(const pat_gconv_desc* d, const void* grad, int chunks, void* partials, void* dw, int ci_real,
                    long off, long s_co, long s_ci, long s_t, int accumulate, void* stream);

/* Scratch (doubles) of the batch-normalisation calls for rows x channels
 * (channels must divide 256), or -1. */
long pat_bn_partials(long rows, int channels);

/* Batch normalisation and ReLU of z (rows x channels, NHWC FP32): training =
 * 1 takes the batch mean and biased variance over the rows (FP64 sums) into
 * mean / invstd = 1 / sqrt(var + eps) and, if running_mean is not NULL,
 * updates running_mean += momentum (mean - running_mean), running_var +=
 * momentum (var rows / (rows - 1) - running_var); training = 0 uses the
 * running statistics.  out = bf16(max(0, gamma (z - mean) invstd + beta)). */
int pat_bn_forward(long rows, int channels, const void* z, const void* gamma, const void* beta, void* mean,
                   void* invstd, void* running_mean, void* running_var, double momentum, double eps, int training,
                   void* out, void* partials, void* stream);

/* Backward of pat_bn_forward (training mode) given grad_act = d loss / d out
 * (FP32 NHWC): gy = grad_act [gamma xhat + beta > 0], xhat = (z - mean)
 * invstd; dbeta (+)= sum gy, dgamma (+)= sum gy xhat; grad_z = bf16(gamma
 * invstd (gy - mean(gy) - xhat mean(gy xhat))). */
int pat_bn_backward(long rows, int channels, const void* z, const void* grad_act, const void* gamma, const void* beta,
                    const void* mean, const void* invstd, void* grad_z, void* dgamma, void* dbeta, int accumulate,
                    void* partials, void* stream);

/* 2x2 max pooling of NHWC bf16 (H, W even); the first maximum in the order
 * (0,0), (0,1), (1,0), (1,1) is taken.  The backward adds grad_out (FP32,
 * H/2 x W/2) to grad_in (FP32, H x W) at each window's maximum. */
int pat_maxpool2(int B, int H, int W, int C, const void* in, void* out, void* stream);
int pat_maxpool2_backward(int B, int H, int W, int C, const void* in, const void* grad_out, void* grad_in, void* stream);

/* Network inputs: out[p][c] = bf16(scales[c] planes[c][p]) for c < cin (1..4),
 * zero for cin <= c < cpad.  The backward writes grad_planes[c][p] =
 * residual[c][p] + scales[c] grad[p][c] (grad: FP32 NHWC with pitch cpad;
 * NULL entries of grad_planes are skipped, NULL residual entries add 0);
 * scales is a host array. */
int pat_nhwc_pack(long pixels, int cin, int cpad, const void* const* planes, const float* scales, void* out,
                  void* stream);
int pat_nhwc_unpack_grad(long pixels, int cin, int cpad, const void* grad, const float* scales, void* const* grad_planes,
                         const void* const* residual, void* stream);

/* 1x1 output layer: out[p] = residual[p] + b[0] + sum_c w[c] act[p][c]
 * (act NHWC bf16 with C channels; b, residual may be NULL). */
int pat_head_forward(long pixels, int C, const void* act, const void* w, const void* b, const void* residual,
                     void* out, void* stream);

/* Scratch (doubles) of pat_head_backward, or -1 (C must divide 256). */
long pat_head_partials(long pixels, int C);

/* Backward of the head: grad_act[p][c] = w[c] grad_out[p] (FP32 NHWC);
 * grad_wb[c] (+)= sum_p grad_out[p] act[p][c] for c < C and grad_wb[C] (+)=
 * sum_p grad_out[p] (the bias), FP64 sums in a fixed order. */
int pat_head_backward(long pixels, int C, const void* act, const void* w, const void* grad_out, void* grad_act,
                      void* grad_wb, int accumulate, void* partials, void* stream);

/* ||A|| (operator norm from the X to the Y inner products of
 * eqn:innerProducts) by power iteration on A*A: `iters` steps from a fixed
 * pseudo-random start, the Rayleigh quotient <f, A*A f>_X / <f, f>_X of the
 * last step.  For step sizes of the iterative solvers (Sec. 4.2).  ws: a
 * workspace for batch 1.  Allocates (and frees) two images, one trace and a
 * few scalars of device memory and synchronises `stream` once at the end. */
int pat_opnorm_estimate(pat_plan p, int iters, double* norm, void* ws, void* stream);

/* Host-side checks of plan internals (no GPU needed).  Fills out[0..K] with
 * J_k(x) for k = 0..K computed by the plan's Miller recurrence. */
int pat_debug_bessel(double x, int K, double* out);

#ifdef __cplusplus
}
#endif

#endif /* PAT_H */
