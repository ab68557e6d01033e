/*
 * pat_oracle.c -- plain CPU FP64 oracle for the circular-geometry
 * photoacoustic forward operator A, its weighted adjoint A* and the
 * back-projection of the approximate inverse A^-1.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, call or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * What it computes (Hauptmann, Kunyansky, Poimala, arXiv 2510.24687):
 *
 *   The paper writes the pressure as the inverse 2D Fourier transform of
 *   f^(xi) cos(c|xi| t) (Sec. 2.1.1, eq. E:kwave) and measures it on the
 *   detector circle (problem statement, Sec. 2).  A sampled image f_pq is
 *   read as the band-limited function whose transform is
 *       W(|xi|) F(xi),   F(xi) = (h^2/2pi) sum_pq f_pq exp(-i xi.x_pq),
 *   (F is the unitary transform of Sec. 2.1.1 applied to the samples, W a
 *   smooth radial taper that vanishes at the Nyquist radius Lambda = pi/h).
 *   Integrating E:kwave over the angle of xi with the Jacobi-Anger identity
 *   (eq. E:Anger, k = 0) gives, at detector z_i and time t_j,
 *
 *       [A f]_{ji} = sum_pq f_pq Q(t_j, |z_i - x_pq|),
 *       Q(t, d)    = (h^2/2pi) int_0^Lambda W(l) l J0(l d) cos(c l t) dl.
 *
 *   The l-integral is evaluated by a composite Gauss-Legendre rule whose
 *   nodes and weights the caller supplies (fixed for a given geometry).
 *   The weighted adjoint follows from the L2 inner products of
 *   eq. eqn:innerProducts discretised by the rectangle rule:
 *       <f1,f2>_X = h^2 sum f1 f2,   <g1,g2>_Y = w_t w_th sum g1 g2,
 *   w_t = T/nt, w_th = R*arc/m, so A* = (w_t w_th / h^2) A^T exactly
 *   (eq. E:adjoint is the continuous counterpart).
 *
 * Conventions:
 *   pixel centres  x_pq = (-a + (q+1/2) h, -a + (p+1/2) h), h = 2a/n,
 *                  f stored row-major f[p*n + q] (p indexes y, q indexes x);
 *   detectors      theta_i = theta0 + i*arc/m, z_i = R (cos, sin)(theta_i);
 *   times          t_j = (j+1) T/nt, j = 0..nt-1;
 *   traces         g stored row-major g[j*m + i] (time-major).
 *   mask           if mask_radius > 0 only pixels with |x_pq| <= mask_radius
 *                  enter A, and A* is zero outside that disk.
 *   taper          W = 1 on [0, rho*Lambda]; on (rho*Lambda, Lambda)
 *                  W = e^{-1/u} / (e^{-1/u} + e^{-1/(1-u)}),
 *                  u = (Lambda - l) / ((1-rho) Lambda); W = 0 beyond Lambda.
 *
 * Sums over pixels use Neumaier compensated summation.  J0 and J1 are the
 * C library's j0() and j1().  Loops are parallel over detectors / pixels with OpenMP,
 * which changes no arithmetic.
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n;
    double a, R, c;
    int m;
    double theta0, arc;
    int nt;
    double T, rho, mask_radius;
} ora_geom;

/* smooth radial taper W, see header */
double ora_taper(double lam, double Lam, double rho)
{
    if (lam <= rho * Lam) return 1.0;
    if (lam >= Lam) return 0.0;
    double u = (Lam - lam) / ((1.0 - rho) * Lam);
    double e1 = exp(-1.0 / u), e2 = exp(-1.0 / (1.0 - u));
    return e1 / (e1 + e2);
}

static double pix_x(const ora_geom* G, int q) { double h = 2.0 * G->a / G->n; return -G->a + (q + 0.5) * h; }

static int pix_in(const ora_geom* G, int p, int q)
{
    if (G->mask_radius <= 0.0) return 1;
    double x = pix_x(G, q), y = pix_x(G, p);
    return x * x + y * y <= G->mask_radius * G->mask_radius;
}

static void neumaier_add(double* s, double* comp, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *comp += (*s - t) + v;
    else *comp += (v - t) + *s;
    *s = t;
}

/* coefficient of node l in Q: (h^2/2pi) w_l W(lam_l) lam_l */
static double* node_coef(const ora_geom* G, int nl, const double* lam, const double* wl)
{
    double h = 2.0 * G->a / G->n, Lam = M_PI / h;
    double* cf = malloc(sizeof(double) * nl);
    for (int l = 0; l < nl; ++l)
        cf[l] = (h * h / (2.0 * M_PI)) * wl[l] * ora_taper(lam[l], Lam, G->rho) * lam[l];
    return cf;
}

/* cos(c lam_l t_j), table [j][l] */
static double* cos_table(const ora_geom* G, int nl, const double* lam)
{
    double* ct = malloc(sizeof(double) * (size_t)G->nt * nl);
    for (int j = 0; j < G->nt; ++j) {
        double t = (j + 1) * G->T / G->nt;
        for (int l = 0; l < nl; ++l) ct[(size_t)j * nl + l] = cos(G->c * lam[l] * t);
    }
    return ct;
}

/*
 * Forward operator on selected detectors.
 *   f    : n*n image
 *   dets : ndet detector indices (NULL -> all m, ndet ignored)
 *   g    : output nt x ndet, row-major [j][ii]
 */
int ora_forward(const ora_geom* G, const double* f, int nl, const double* lam, const double* wl,
                int ndet, const int* dets, double* g)
{
    if (!G || !f || !lam || !wl || !g || G->n <= 0 || G->m <= 0 || G->nt <= 0 || nl <= 0) return -1;
    if (!dets) ndet = G->m;
    int n = G->n, nt = G->nt;
    double* cf = node_coef(G, nl, lam, wl);
    double* ct = cos_table(G, nl, lam);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int ii = 0; ii < ndet; ++ii) {
        int i = dets ? dets[ii] : ii;
        double th = G->theta0 + i * G->arc / G->m;
        double zx = G->R * cos(th), zy = G->R * sin(th);
        double* S = calloc((size_t)nl, sizeof(double));
        double* C = calloc((size_t)nl, sizeof(double));
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                double v = f[(size_t)p * n + q];
                if (v == 0.0 || !pix_in(G, p, q)) continue;
                double d = hypot(zx - pix_x(G, q), zy - pix_x(G, p));
                for (int l = 0; l < nl; ++l) neumaier_add(&S[l], &C[l], v * j0(lam[l] * d));
            }
        for (int l = 0; l < nl; ++l) S[l] = (S[l] + C[l]) * cf[l];
        for (int j = 0; j < nt; ++j) {
            double s = 0.0, cmp = 0.0;
            const double* row = ct + (size_t)j * nl;
            for (int l = 0; l < nl; ++l) neumaier_add(&s, &cmp, row[l] * S[l]);
            g[(size_t)j * ndet + ii] = s + cmp;
        }
        free(S); free(C);
    }
    free(cf); free(ct);
    return 0;
}

/*
 * Weighted adjoint A* = (w_t w_th / h^2) A^T on selected pixels.
 *   g    : full nt x m traces
 *   pix  : npix flat pixel indices p*n+q (NULL -> all n*n, npix ignored)
 *   f    : output, npix values
 */
int ora_adjoint(const ora_geom* G, const double* g, int nl, const double* lam, const double* wl,
                int npix, const int* pix, double* f)
{
    if (!G || !f || !lam || !wl || !g || G->n <= 0 || G->m <= 0 || G->nt <= 0 || nl <= 0) return -1;
    int n = G->n, m = G->m, nt = G->nt;
    if (!pix) npix = n * n;
    double h = 2.0 * G->a / n;
    double scale = (G->T / nt) * (G->R * G->arc / m) / (h * h);
    double* cf = node_coef(G, nl, lam, wl);
    double* ct = cos_table(G, nl, lam);
    /* Cg[i][l] = cf_l * sum_j g[j][i] cos(c lam_l t_j) */
    double* Cg = malloc(sizeof(double) * (size_t)m * nl);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < m; ++i) {
        for (int l = 0; l < nl; ++l) {
            double s = 0.0, cmp = 0.0;
            for (int j = 0; j < nt; ++j) neumaier_add(&s, &cmp, g[(size_t)j * m + i] * ct[(size_t)j * nl + l]);
            Cg[(size_t)i * nl + l] = (s + cmp) * cf[l];
        }
    }
    double* zx = malloc(sizeof(double) * m);
    double* zy = malloc(sizeof(double) * m);
    for (int i = 0; i < m; ++i) {
        double th = G->theta0 + i * G->arc / m;
        zx[i] = G->R * cos(th); zy[i] = G->R * sin(th);
    }
    #pragma omp parallel for schedule(dynamic, 4)
    for (int kk = 0; kk < npix; ++kk) {
        int idx = pix ? pix[kk] : kk;
        int p = idx / n, q = idx % n;
        if (!pix_in(G, p, q)) { f[kk] = 0.0; continue; }
        double x = pix_x(G, q), y = pix_x(G, p);
        double s = 0.0, cmp = 0.0;
        for (int i = 0; i < m; ++i) {
            double d = hypot(zx[i] - x, zy[i] - y);
            const double* row = Cg + (size_t)i * nl;
            for (int l = 0; l < nl; ++l) neumaier_add(&s, &cmp, row[l] * j0(lam[l] * d));
        }
        f[kk] = scale * (s + cmp);
    }
    free(cf); free(ct); free(Cg); free(zx); free(zy);
    return 0;
}

/*
 * Back-projection v of the universal inversion formula (eq. E:inverse,
 * truncated to the measured times as in eq. E:approx_UBP) for the
 * band-limited model: the fundamental solution G of eq. E:green_conv is
 * replaced by G_W, the inverse transform of W(|xi|) sin(c|xi|t)/(2 pi c|xi|)
 * (eq. E:Fourier_Green with the unitary transform of Sec. 2.1.1), so that
 *
 *   d/dn(z) G_W(t, x - z) = (n(z).(x - z)) / (2 pi c)
 *                           int_0^Lambda W(l) l [J1(l d)/d] sin(c l t) dl,   d = |x - z|,
 *
 * for a unit normal n(z), and the time and arc integrals are the rectangle
 * rules of eqn:innerProducts (w_t = T/nt, w_th = R arc/m).  With this G the
 * formula returns f (not -f) when n(z) is the normal pointing INTO the disk,
 * n_i = -z_i/R; that is also the sign of the paper's Fourier coefficients
 * of v (eq. E:Four_coef_v), whose derivation (Appendix) differentiates
 * e^{-i xi.z} with the opposite sign.  For a speed of sound c the formula
 * (written for c = 1) becomes v = 2 c^2 int int g d/dn G_W, hence
 *
 *   v(x_pq) = (2 c w_t w_th / 2pi) sum_i (z_i/R).(z_i - x_pq)
 *             sum_l w_l W(l) l [J1(l d_ipq)/d_ipq] sum_j g[j][i] sin(c l t_j).
 *
 * J1(l d)/d -> l/2 as d -> 0.  No mask and no constant here: the caller adds
 * the constant of eq. E:silly_integral and restricts to the support.
 *   g    : full nt x m traces
 *   pix  : npix flat pixel indices p*n+q (NULL -> all n*n, npix ignored)
 *   v    : output, npix values
 */
int ora_ubp(const ora_geom* G, const double* g, int nl, const double* lam, const double* wl,
            int npix, const int* pix, double* v)
{
    if (!G || !v || !lam || !wl || !g || G->n <= 0 || G->m <= 0 || G->nt <= 0 || nl <= 0) return -1;
    int n = G->n, m = G->m, nt = G->nt;
    if (!pix) npix = n * n;
    double h = 2.0 * G->a / n, Lam = M_PI / h;
    double scale = 2.0 * G->c * (G->T / nt) * (G->R * G->arc / m) / (2.0 * M_PI);
    /* st[j][l] = sin(c l t_j);  Sg[i][l] = w_l W_l l * sum_j g[j][i] st[j][l] */
    double* st = malloc(sizeof(double) * (size_t)nt * nl);
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < nt; ++j) {
        double t = (j + 1) * G->T / nt;
        for (int l = 0; l < nl; ++l) st[(size_t)j * nl + l] = sin(G->c * lam[l] * t);
    }
    double* Sg = malloc(sizeof(double) * (size_t)m * nl);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < m; ++i) {
        for (int l = 0; l < nl; ++l) {
            double s = 0.0, cmp = 0.0;
            for (int j = 0; j < nt; ++j) neumaier_add(&s, &cmp, g[(size_t)j * m + i] * st[(size_t)j * nl + l]);
            Sg[(size_t)i * nl + l] = (s + cmp) * wl[l] * ora_taper(lam[l], Lam, G->rho) * lam[l];
        }
    }
    free(st);
    double* zx = malloc(sizeof(double) * m);
    double* zy = malloc(sizeof(double) * m);
    double* nx = malloc(sizeof(double) * m);
    double* ny = malloc(sizeof(double) * m);
    for (int i = 0; i < m; ++i) {
        double th = G->theta0 + i * G->arc / m;
        nx[i] = cos(th); ny[i] = sin(th);
        zx[i] = G->R * nx[i]; zy[i] = G->R * ny[i];
    }
    #pragma omp parallel for schedule(dynamic, 4)
    for (int kk = 0; kk < npix; ++kk) {
        int idx = pix ? pix[kk] : kk;
        int p = idx / n, q = idx % n;
        double x = pix_x(G, q), y = pix_x(G, p);
        double s = 0.0, cmp = 0.0;
        for (int i = 0; i < m; ++i) {
            double dx = x - zx[i], dy = y - zy[i];
            double d = hypot(dx, dy);
            double nd = -(nx[i] * dx + ny[i] * dy);   /* inward normal . (x - z_i) */
            const double* row = Sg + (size_t)i * nl;
            double si = 0.0, ci = 0.0;
            for (int l = 0; l < nl; ++l) {
                double k1 = d > 0.0 ? j1(lam[l] * d) / d : 0.5 * lam[l];
                neumaier_add(&si, &ci, row[l] * k1);
            }
            neumaier_add(&s, &cmp, nd * (si + ci));
        }
        v[kk] = scale * (s + cmp);
    }
    free(Sg); free(zx); free(zy); free(nx); free(ny);
    return 0;
}

/*
 * Semi-closed form for a sum of Gaussians f(x) = sum_b amp_b exp(-|x-c_b|^2 / (2 s_b^2))
 * (continuous f, no grid).  Its transform is amp s^2 exp(-s^2|xi|^2/2) exp(-i xi.c),
 * so E:kwave with the Jacobi-Anger reduction gives the one-dimensional integral
 *     g(t,z) = sum_b amp_b s_b^2 int_0^inf Wt(l) exp(-s_b^2 l^2/2) l J0(l |z-c_b|) cos(c l t) dl,
 * with Wt = W (taper of a grid with Nyquist radius Lam_taper) if use_taper,
 * else Wt = 1.  The nodes must cover the support of the integrand.
 *   blobs : nb x 4 rows (cx, cy, sigma, amp)
 *   g     : output nt x ndet
 */
int ora_gauss(const ora_geom* G, int nb, const double* blobs, int use_taper, double Lam_taper,
              int nl, const double* lam, const double* wl, int ndet, const int* dets, double* g)
{
    if (!G || !blobs || !lam || !wl || !g || nb <= 0 || nl <= 0) return -1;
    if (!dets) ndet = G->m;
    int nt = G->nt;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int ii = 0; ii < ndet; ++ii) {
        int i = dets ? dets[ii] : ii;
        double th = G->theta0 + i * G->arc / G->m;
        double zx = G->R * cos(th), zy = G->R * sin(th);
        double* S = calloc((size_t)nl, sizeof(double));
        for (int l = 0; l < nl; ++l) {
            double s = 0.0, cmp = 0.0;
            for (int b = 0; b < nb; ++b) {
                const double* B = blobs + 4 * b;
                double d = hypot(zx - B[0], zy - B[1]);
                double sg = B[2];
                neumaier_add(&s, &cmp, B[3] * sg * sg * exp(-0.5 * sg * sg * lam[l] * lam[l]) * j0(lam[l] * d));
            }
            double wt = use_taper ? ora_taper(lam[l], Lam_taper, G->rho) : 1.0;
            S[l] = (s + cmp) * wl[l] * wt * lam[l];
        }
        for (int j = 0; j < nt; ++j) {
            double t = (j + 1) * G->T / nt;
            double s = 0.0, cmp = 0.0;
            for (int l = 0; l < nl; ++l) neumaier_add(&s, &cmp, S[l] * cos(G->c * lam[l] * t));
            g[(size_t)j * ndet + ii] = s + cmp;
        }
        free(S);
    }
    return 0;
}
