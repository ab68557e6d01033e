// Internal declarations shared by the host plan builder (pat_plan.cpp) and
// the HIP kernels/entry points (pat_kernels.hip).
#pragma once

#include <cstddef>
#include <string>
#include <vector>

#include "../../include/pat.h"

namespace pat {

// Everything the plan decides, derived from the geometry and the precision.
struct Params {
    pat_geometry g;
    pat_dtype dt;
    int n, m, nt, mf;       // image side, detectors, time samples, full-circle detector count
    int mf3;                // 1 when mf = 3 * 2^a (else a power of two)
    double h, Lam, rmax;    // pixel size, Nyquist radius pi/h, largest |x| entering A
    double shift;           // x_q = h (q' + shift), q' = q - n/2 (integer division)
    int Ng;                 // oversampled Cartesian grid (per side), power of two
    int w, hw;              // stencil width, half-width ceil(w/2)
    double beta;            // exponential-of-semicircle kernel parameter
    int Rw;                 // row-pass width Ng/2 + 1
    int Ew;                 // extended half-grid width Ng/2 + 1 + 2 hw
    double eps;             // target size of each neglected term
    int M;                  // cosine transform via a 2M-point FFT; M = 2^a or 3 * 2^a
    int m3;                 // 1 when M = 3 * 2^a
    double period, dlam;    // time period of the discrete cosine sum, ring spacing
    int L;                  // rings lambda_l = l dlam < Lam
    int K, Kp;              // largest harmonic, row pitch of the harmonic arrays
    int klow;               // harmonics 0..klow get the low-frequency correction
    int Ls;                 // half-width of the band-limited interpolation kernel (samples)
    double lam_c, lam_s;    // low-frequency split: erfc step centre and width
    int lcorr;              // rings feeding the low-frequency correction
    int Nmax;               // twiddle table length (largest FFT)
    int max_ring;           // largest ring FFT
    int Nr3 = 0;            // largest ring of 3 * 2^a points (0: none)
    int npts;               // half-ring samples over all rings
    double pre_scale;       // h^2 / (2 pi)
    double adj_scale;       // (T/nt)(R arc/m)/h^2
    double inv_scale;       // -2 c adj_scale: the approximate inverse's back-projection
};

struct HostPlan {
    Params P;
    std::vector<double> Dq;                 // n: 1/phi_hat(2 pi q'/Ng)
    std::vector<double> lam;                // L
    std::vector<int> ringN, ringLog, ringOff, ringK;  // L (ringLog: log2 of N, or of N/3 when ringM3)
    std::vector<int> ringM3;                          // L: 1 when the ring has 3 * 2^a points
    std::vector<double> twr;                          // 2*(2 Nr3): e^{-2 pi i j/(2 Nr3)}, ring radix-3 twiddles
    std::vector<double> Tb;                 // L x Kp, real Bessel/taper/quadrature weights (1/N_l folded)
    std::vector<double> Mk;                 // (klow+1) x nt x lcorr
    std::vector<double> Tbi;                // L x Kp: as Tb with J_k' in place of J_k (approximate inverse)
    std::vector<double> Mki;                // (klow+1) x nt x lcorr: as Mk with J_k' and sin in place of J_k and cos
    std::vector<double> phase;              // 2*Kp: e^{i k theta0} (re, im)
    std::vector<double> tw;                 // 2*Nmax: e^{-2 pi i k / Nmax} (re, im)
    std::vector<double> twd;                // 2*(2M): e^{-2 pi i j / (2M)} (re, im), cosine-transform twiddles
    std::vector<double> twm;                // 2*(2mf): e^{-2 pi i j / (2mf)}, angular-transform twiddles
    std::vector<double> pos;                // 2*npts: grid position (x, y) of each half-ring sample
};

// Fills P and all host tables.  Returns PAT_OK or an error with `err` set.
int build_host_plan(const pat_geometry& g, pat_dtype dt, HostPlan& out, std::string& err);

// J_k(x), k = 0..K, by Miller's backward recurrence normalised with
// J_0 + 2 sum_k J_2k = 1.
void bessel_j_all(double x, int K, double* out);

void set_error(const std::string& s);

}  // namespace pat
