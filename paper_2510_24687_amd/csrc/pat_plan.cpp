// Host-side plan builder: chooses the discretisation of the fast operator for
// a geometry and computes every table in FP64.
//
// The fast forward operator follows Algorithm 1 of Hauptmann, Kunyansky &
// Poimala (arXiv 2510.24687, Sec. 3.1):
//   (1-2) zero-extend f and take a 2D FFT -- here on a grid oversampled by
//         sigma >= 2 after dividing f by the Fourier transform of the gridding
//         kernel, so that
//   (3)   Cartesian->polar interpolation is a w x w convolution with an
//         exponential-of-semicircle kernel (a non-uniform FFT of type 2)
//         instead of the paper's bilinear rule on a refined grid;
//   (4)   per ring, an FFT over the angle gives F_k(lambda) (eq. E:eq3);
//   (5)   per harmonic, g_k(t) = i^k int lambda F_k J_k(lambda R) cos(c lambda t)
//         (eq. E:eq2 / E:inverse_cos_tr) by the trapezoid rule on the ring
//         grid, i.e. a discrete cosine transform; the lowest harmonics get an
//         exact quadrature near lambda = 0 (the paper's special treatment of
//         k = -1, 0, 1) through a small precomputed matrix;
//   (6-7) per time sample, the angular synthesis of eq. E:FourSerForg on the
//         full circle of m_full detectors, restricted to the arc.
// The tables below are those steps' weights.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>

#include "pat_internal.h"

namespace pat {

static thread_local std::string g_last_error;
void set_error(const std::string& s) { g_last_error = s; }
const char* last_error() { return g_last_error.c_str(); }

static int next_pow2(long v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

static int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

void bessel_j_all(double x, int K, double* out)
{
    for (int k = 0; k <= K; ++k) out[k] = 0.0;
    x = std::fabs(x);
    if (x == 0.0) {
        out[0] = 1.0;
        return;
    }
    int N = std::max(K, (int)std::ceil(x)) + 60 + (int)std::ceil(15.0 * std::cbrt(x));
    if (N % 2) ++N;
    double jp1 = 0.0, j = 1.0, sum = 0.0;
    for (int k = N; k >= 1; --k) {
        if (k <= K) out[k] = j;
        if (k % 2 == 0) sum += j;
        double jm1 = (2.0 * k / x) * j - jp1;
        jp1 = j;
        j = jm1;
        if (std::fabs(j) > 1e250) {
            j *= 1e-250;
            jp1 *= 1e-250;
            sum *= 1e-250;
            for (int i = k; i <= K; ++i) out[i] *= 1e-250;
        }
    }
    out[0] = j;
    double norm = j + 2.0 * sum;
    for (int k = 0; k <= K; ++k) out[k] /= norm;
}

// Smooth radial taper of the band-limited model.
static double taper(double lam, double Lam, double rho)
{
    if (lam <= rho * Lam) return 1.0;
    if (lam >= Lam) return 0.0;
    double u = (Lam - lam) / ((1.0 - rho) * Lam);
    double e1 = std::exp(-1.0 / u), e2 = std::exp(-1.0 / (1.0 - u));
    return e1 / (e1 + e2);
}

// Low-frequency cut chi(lambda) = erfc((lambda - lam_c)/lam_s)/2, zero beyond lam_c + 6 lam_s.
static double chi(double lam, double lam_c, double lam_s)
{
    if (lam >= lam_c + 6.0 * lam_s) return 0.0;
    return 0.5 * std::erfc((lam - lam_c) / lam_s);
}

// phi_hat(omega) = int_{-w/2}^{w/2} phi(d) cos(omega d) dd, via d = (w/2) sin(theta).
static double es_transform(double omega, int w, double beta, const std::vector<double>& gx,
                           const std::vector<double>& gw)
{
    double s = 0.0;
    for (size_t i = 0; i < gx.size(); ++i) {
        double th = 0.5 * M_PI * gx[i];
        double ct = std::cos(th);
        s += gw[i] * std::exp(beta * (ct - 1.0)) * std::cos(omega * 0.5 * w * std::sin(th)) * ct;
    }
    return s * 0.5 * M_PI * 0.5 * w;
}

// Band-limited interpolation kernel: sinc with a Gaussian window.
static double sinc_kernel(double x, int Ls, double r)
{
    if (std::fabs(x) > Ls) return 0.0;
    double s = (x == 0.0) ? 1.0 : std::sin(M_PI * x) / (M_PI * x);
    return s * std::exp(-0.5 * x * x / (r * r));
}

int build_host_plan(const pat_geometry& g, pat_dtype dt, HostPlan& H, std::string& err)
{
    Params& P = H.P;
    std::memset(&P, 0, sizeof(P));
    P.g = g;
    P.dt = dt;
    if (dt != PAT_F32 && dt != PAT_F64) { err = "dtype must be PAT_F32 or PAT_F64"; return PAT_EINVAL; }
    if (g.n < 8 || g.n > 8192) { err = "n must be in [8, 8192]"; return PAT_EINVAL; }
    if (g.m < 1 || g.nt < 1) { err = "m and nt must be positive"; return PAT_EINVAL; }
    if (!(g.a > 0) || !(g.R > 0) || !(g.c > 0) || !(g.T > 0)) { err = "a, R, c, T must be positive"; return PAT_EINVAL; }
    if (!(g.arc > 0) || g.arc > 2 * M_PI * (1 + 1e-12)) { err = "arc must be in (0, 2 pi]"; return PAT_EINVAL; }
    if (!(g.taper_rho > 0 && g.taper_rho < 1)) { err = "taper_rho must be in (0, 1)"; return PAT_EINVAL; }
    if (g.mask_radius < 0) { err = "mask_radius must be >= 0"; return PAT_EINVAL; }
    double mfd = 2 * M_PI * g.m / g.arc;
    long mf = std::lround(mfd);
    if (std::fabs(mfd - mf) > 1e-6 * mfd || mf < g.m) {
        err = "2*pi*m/arc must be an integer >= m (detectors on a uniform full-circle grid)";
        return PAT_EINVAL;
    }
    const bool mf_pow2 = (mf & (mf - 1)) == 0;
    const bool mf_3pow2 = mf % 3 == 0 && ((mf / 3) & (mf / 3 - 1)) == 0;
    if (!(mf_pow2 || mf_3pow2) || mf < 4 || mf > 65536) {
        err = "full-circle detector count 2*pi*m/arc must be 2^a or 3*2^a in [4, 65536]";
        return PAT_EUNSUPPORTED;
    }
    const bool f64 = (dt == PAT_F64);
    P.n = g.n; P.m = g.m; P.nt = g.nt; P.mf = (int)mf; P.mf3 = mf_pow2 ? 0 : 1;
    P.h = 2.0 * g.a / g.n;
    P.Lam = M_PI / P.h;
    P.rmax = std::sqrt(2.0) * (g.a - 0.5 * P.h);
    if (g.mask_radius > 0) P.rmax = std::min(P.rmax, g.mask_radius);
    P.shift = 0.5 - (0.5 * g.n - g.n / 2);
    P.eps = f64 ? 1e-13 : 1e-7;
    P.Ng = next_pow2(2L * g.n);
    P.w = f64 ? 13 : 6;
    P.hw = (P.w + 1) / 2;
    P.beta = 2.30 * P.w;
    P.Rw = P.Ng / 2 + 1;
    P.Ew = P.Ng / 2 + 1 + 2 * P.hw;
    P.pre_scale = P.h * P.h / (2.0 * M_PI);
    P.adj_scale = (g.T / g.nt) * (g.R * g.arc / g.m) / (P.h * P.h);
    // The back-projection of the approximate inverse has the adjoint's form
    // with J_k' for J_k, sin for cos and the factor 2c; its sign is that of
    // the normal pointing into the disk (the left-inverse sign).
    P.inv_scale = -2.0 * g.c * P.adj_scale;

    // time period of the discrete cosine sum: the part of g_k(t) that is not the
    // slow 2D tail lives in |c t| <= R + rmax plus the spread caused by the taper
    const double ct = g.c * g.T / g.nt;
    const double lg = std::log(1.0 / P.eps);
    double spread = 0.25 * lg * lg / ((1.0 - g.taper_rho) * P.Lam) + 0.25;
    double Pmin = g.c * g.T + P.rmax + g.R + spread;
    long Mneed = (long)std::ceil(Pmin / (2.0 * ct));
    // the cosine transform's half length: the smallest 2^a or 3 * 2^a that covers
    // the period and the time samples (the ring count L scales with M)
    {
        const long need = std::max<long>(Mneed, g.nt);
        const long m2 = next_pow2(need);
        long m3 = 3;
        while (m3 < need) m3 *= 2;
        P.M = (int)std::min(m2, m3);
        P.m3 = (P.M % 3 == 0) ? 1 : 0;
    }
    P.period = 2.0 * P.M * ct;
    P.dlam = 2.0 * M_PI / P.period;
    P.L = (int)std::ceil(P.Lam / P.dlam - 1e-9);
    if (P.L > 2 * P.M) { err = "internal: ring count exceeds cosine-transform length"; return PAT_EUNSUPPORTED; }
    if (P.M > (1 << 16)) { err = "nt*c*(R+rmax+cT)/T too large"; return PAT_EUNSUPPORTED; }

    // low-frequency split (margin left in the period beyond the compact part)
    double margin = P.period - g.c * g.T - P.rmax - g.R;
    P.lam_s = 2.0 * std::sqrt(lg) / std::max(margin, 1e-3);
    P.lam_c = 6.0 * P.lam_s;
    P.klow = f64 ? 4 : 2;
    P.Ls = f64 ? 32 : 16;
    double lam_end = P.lam_c + 6.0 * P.lam_s;
    P.lcorr = std::min(P.L, (int)std::floor(lam_end / P.dlam) + P.Ls + 2);

    // rings
    const double cA = f64 ? 9.0 : 6.0, mphi = f64 ? 64.0 : 32.0;
    H.lam.resize(P.L);
    H.ringN.resize(P.L);
    H.ringLog.resize(P.L);
    H.ringM3.resize(P.L);
    H.ringOff.resize(P.L);
    H.ringK.resize(P.L);
    int off = 0, K = 0, maxN = 0;
    for (int l = 0; l < P.L; ++l) {
        double lam = l * P.dlam;
        double x = lam * g.R;
        double kedge = x + cA * std::cbrt(x) + 4.0;
        double need = std::max({16.0, lam * (g.R + P.rmax) + mphi, 2.0 * kedge + 2.0});
        // ring length: the smallest 2^a or 3 * 2^a (a >= 2) covering `need`
        const long need_i = (long)std::ceil(need);
        long N3 = 12;
        while (N3 < need_i) N3 *= 2;
        int N = (int)std::min<long>(next_pow2(need_i), N3);
        int Kl = std::min(N / 2 - 1, (int)std::ceil(kedge));
        H.lam[l] = lam;
        H.ringN[l] = N;
        H.ringM3[l] = (N % 3 == 0) ? 1 : 0;
        H.ringLog[l] = ilog2(H.ringM3[l] ? N / 3 : N);
        if (H.ringM3[l]) P.Nr3 = std::max(P.Nr3, N);
        H.ringOff[l] = off;
        H.ringK[l] = Kl;
        off += N / 2;
        K = std::max(K, Kl);
        maxN = std::max(maxN, N);
    }
    P.npts = off;
    P.max_ring = maxN;
    P.K = K;
    P.Kp = ((K + 1 + 15) / 16) * 16;
    P.Nmax = (int)next_pow2(std::max({P.Ng, 2 * P.M, maxN, P.mf}));

    // pre-correction: 1/phi_hat(2 pi q'/Ng)
    {
        std::vector<double> gx, gw;
        gauss_legendre(256, gx, gw);
        H.Dq.resize(g.n);
        for (int q = 0; q < g.n; ++q) {
            int qp = q - g.n / 2;
            H.Dq[q] = 1.0 / es_transform(2.0 * M_PI * qp / P.Ng, P.w, P.beta, gx, gw);
        }
    }

    // Bessel/taper/trapezoid weights per ring and harmonic (1/N_l folded in)
    // (Tbi: the same with the derivative J_k' = (J_{k-1} - J_{k+1})/2, J_0' = -J_1)
    H.Tb.assign((size_t)P.L * P.Kp, 0.0);
    H.Tbi.assign((size_t)P.L * P.Kp, 0.0);
    {
        std::vector<double> J(K + 2);
        for (int l = 0; l < P.L; ++l) {
            double lam = H.lam[l];
            bessel_j_all(lam * g.R, K + 1, J.data());
            double trap = (l == 0) ? 0.5 * P.dlam : P.dlam;
            double base = taper(lam, P.Lam, g.taper_rho) * lam * trap / H.ringN[l];
            double cut = 1.0 - chi(lam, P.lam_c, P.lam_s);
            for (int k = 0; k <= H.ringK[l]; ++k) {
                double wk = base * (k <= P.klow ? cut : 1.0);
                double dJ = k == 0 ? -J[1] : 0.5 * (J[k - 1] - J[k + 1]);
                H.Tb[(size_t)l * P.Kp + k] = wk * J[k];
                H.Tbi[(size_t)l * P.Kp + k] = wk * dJ;
            }
        }
    }

    // low-frequency correction: exact quadrature over [0, lam_c + 6 lam_s] of
    // chi W lambda J_k(lambda R) cos(c lambda t_j) F_k(lambda), with F_k
    // interpolated from the ring samples (it is band-limited of type rmax;
    // samples at negative lambda are (-1)^k times the mirrored ones); Mki is
    // the same with J_k' and sin, for the approximate inverse.
    {
        int nq = 12;
        std::vector<double> gx, gw;
        gauss_legendre(nq, gx, gw);
        double pw = 0.5 * P.dlam;
        int npan = (int)std::ceil(lam_end / pw);
        double bfrac = P.rmax * P.dlam / M_PI;
        if (bfrac >= 0.95) { err = "internal: ring spacing too coarse for interpolation"; return PAT_EUNSUPPORTED; }
        double r = std::sqrt(P.Ls / ((1.0 - bfrac) * M_PI));
        H.Mk.assign((size_t)(P.klow + 1) * g.nt * P.lcorr, 0.0);
        H.Mki.assign((size_t)(P.klow + 1) * g.nt * P.lcorr, 0.0);
        std::vector<double> Jn(P.klow + 2), dJn(P.klow + 1);
        std::vector<double> cosv(g.nt), sinv(g.nt);
        for (int pi = 0; pi < npan; ++pi) {
            double lo = pi * pw, hi = std::min(lam_end, lo + pw);
            for (int qi = 0; qi < nq; ++qi) {
                double mu = 0.5 * (hi - lo) * gx[qi] + 0.5 * (hi + lo);
                double nu = 0.5 * (hi - lo) * gw[qi];
                double base = nu * chi(mu, P.lam_c, P.lam_s) * taper(mu, P.Lam, g.taper_rho) * mu;
                if (base == 0.0) continue;
                bessel_j_all(mu * g.R, P.klow + 1, Jn.data());
                for (int k = 0; k <= P.klow; ++k) dJn[k] = k == 0 ? -Jn[1] : 0.5 * (Jn[k - 1] - Jn[k + 1]);
                for (int j = 0; j < g.nt; ++j) {
                    cosv[j] = std::cos(g.c * mu * (j + 1) * g.T / g.nt);
                    sinv[j] = std::sin(g.c * mu * (j + 1) * g.T / g.nt);
                }
                double xs = mu / P.dlam;
                int l0 = std::max(0, (int)std::floor(xs - P.Ls) - 1);
                int l1 = std::min(P.lcorr - 1, (int)std::ceil(xs + P.Ls) + 1);
                for (int l = l0; l <= l1; ++l) {
                    double sp = sinc_kernel(xs - l, P.Ls, r);
                    double sm = (l >= 1) ? sinc_kernel(xs + l, P.Ls, r) : 0.0;
                    for (int k = 0; k <= P.klow; ++k) {
                        double s = sp + ((k & 1) ? -sm : sm);
                        double c = base * Jn[k] * s, ci = base * dJn[k] * s;
                        double* row = &H.Mk[((size_t)k * g.nt) * P.lcorr + l];
                        double* rowi = &H.Mki[((size_t)k * g.nt) * P.lcorr + l];
                        for (int j = 0; j < g.nt; ++j) {
                            row[(size_t)j * P.lcorr] += c * cosv[j];
                            rowi[(size_t)j * P.lcorr] += ci * sinv[j];
                        }
                    }
                }
                // mirrored samples of rings l <= Ls near lambda = 0 are covered by sm above
            }
        }
    }

    // detector phase e^{i k theta0}
    H.phase.resize(2 * P.Kp);
    for (int k = 0; k < P.Kp; ++k) {
        double a = std::fmod(k * g.theta0, 2 * M_PI);
        H.phase[2 * k] = std::cos(a);
        H.phase[2 * k + 1] = std::sin(a);
    }
    // twiddles e^{-2 pi i k/Nmax}
    H.tw.resize(2 * P.Nmax);
    for (int k = 0; k < P.Nmax; ++k) {
        double a = -2.0 * M_PI * k / P.Nmax;
        H.tw[2 * k] = std::cos(a);
        H.tw[2 * k + 1] = std::sin(a);
    }

    // angular-transform twiddles e^{-2 pi i j/(2 m_full)} (its radix-3 pass)
    H.twm.resize(2 * 2 * (size_t)P.mf);
    for (int j = 0; j < 2 * P.mf; ++j) {
        double a = -M_PI * j / P.mf;
        H.twm[2 * j] = std::cos(a);
        H.twm[2 * j + 1] = std::sin(a);
    }

    // ring-transform twiddles e^{-2 pi i j/(2 Nr3)} (radix-3 pass of 3 * 2^a rings)
    {
        const int Nr = std::max(P.Nr3, 3);
        H.twr.resize(2 * 2 * (size_t)Nr);
        for (int j = 0; j < 2 * Nr; ++j) {
            double a = -M_PI * j / Nr;
            H.twr[2 * j] = std::cos(a);
            H.twr[2 * j + 1] = std::sin(a);
        }
    }

    // cosine-transform twiddles e^{-2 pi i j/(2M)}
    H.twd.resize(2 * 2 * (size_t)P.M);
    for (int j = 0; j < 2 * P.M; ++j) {
        double a = -M_PI * j / P.M;
        H.twd[2 * j] = std::cos(a);
        H.twd[2 * j + 1] = std::sin(a);
    }

    // grid positions (cells) of every half-ring sample, shared by the gather
    // and its transpose so both select identical taps
    H.pos.resize(2 * (size_t)P.npts);
    {
        const double half = 0.5 * P.Ng / P.Lam;
        for (int l = 0; l < P.L; ++l) {
            int N = H.ringN[l];
            for (int si = 0; si < N / 2; ++si) {
                int s = si - N / 4;
                double ph = 2.0 * M_PI * s / N;
                H.pos[2 * ((size_t)H.ringOff[l] + si)] = H.lam[l] * half * std::cos(ph);
                H.pos[2 * ((size_t)H.ringOff[l] + si) + 1] = H.lam[l] * half * std::sin(ph);
            }
        }
    }
    if (H.ringN.back() > 4096) { err = "internal: ring FFT larger than 4096"; return PAT_EUNSUPPORTED; }
    return PAT_OK;
}

}  // namespace pat
