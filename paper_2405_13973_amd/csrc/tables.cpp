// Host-side generation of the translation matrices of the GPU FMM.
//
// In the box-scaled normalised basis (fmm_math.hpp) the operators between
// boxes of side h (targets) and sources follow from the addition theorems
//   Rh-form:  R_n^m(a + b) = sum_{j,k} R_j^k(a) R_{n-j}^{m-k}(b)
//   I-form:   I_j^k(r + t) = sum_{n,m} (-1)^n conj(R_n^m(r)) I_{j+n}^{k+m}(t)
// of the unnormalised R_n^m = Rh_n^m / nu_n^m, I_n^m = nu_n^m Ih_n^m,
// nu_n^m = sqrt((n+|m|)!(n-|m|)!).  Rescaled:
//   M2M  Mh'_n^m = sum conj(Rh_j^k(d)) Mh_{n-j}^{m-k} 2^{-(n-j)} nu_n^m / (nu_j^k nu_{n-j}^{m-k})
//   L2L  Lh'_j^k = sum Lh_n^m conj(Rh_{n-j}^{m-k}(d)) 2^{-(j+1)} nu_n^m / (nu_{n-j}^{m-k} nu_j^k)
//   M2L  Lh_n^m  = (-1)^n sum Mh_j^k Ih_{j+n}^{k+m}(-s) nu_{j+n}^{k+m} / (nu_j^k nu_n^m)
// with d the child centre minus the parent centre in parent box units and
// s the source centre minus the target centre in box units.  Each complex
// map is assembled into a real matrix on the (Re, Im, m >= 0) storage using
// c_n^{-m} = (-1)^m conj(c_n^m).
#include <cmath>
#include <complex>
#include <vector>

#include "fmm_math.hpp"

namespace pt {
namespace {

using cd = std::complex<double>;

struct Harm {
    int nmax;
    std::vector<double> re, im;
    Harm(int nmax_, double x, double y, double z) : nmax(nmax_), re((nmax_ + 1) * (nmax_ + 2) / 2), im(re.size())
    {
        rhat_all<double>(nmax, x, y, z, re.data(), im.data());
    }
    // Rh_n^m for any |m| <= n
    cd R(int n, int m) const
    {
        const int am = m < 0 ? -m : m;
        cd v(re[n * (n + 1) / 2 + am], im[n * (n + 1) / 2 + am]);
        if (m < 0) v = ((am & 1) ? -1.0 : 1.0) * std::conj(v);
        return v;
    }
};

double nu(int n, int m)
{
    const int am = m < 0 ? -m : m;
    double f = 1.0;
    for (int k = 2; k <= n + am; ++k) f *= k;
    for (int k = 2; k <= n - am; ++k) f *= k;
    return std::sqrt(f);
}

// Add C * c_in to c_out in real storage, where c_in = input coefficient (j, k)
// (any sign of k) and c_out = output (n, m), m >= 0; T is K x K row-major.
void assemble(double *T, int K, int n, int m, int j, int k, cd C)
{
    const int ak = k < 0 ? -k : k;
    const double s = (k < 0 && (ak & 1)) ? -1.0 : 1.0;
    const int cre = sidx_re(j, ak);
    const int cim = ak > 0 ? sidx_im(j, ak) : -1;
    const int rre = sidx_re(n, m);
    const int rim = m > 0 ? sidx_im(n, m) : -1;
    const double Cr = C.real(), Ci = C.imag();
    // c_in = a + i b (k >= 0) or s (a - i b) (k < 0)
    if (k >= 0) {
        T[rre * K + cre] += Cr;
        if (cim >= 0) T[rre * K + cim] += -Ci;
        if (rim >= 0) {
            T[rim * K + cre] += Ci;
            if (cim >= 0) T[rim * K + cim] += Cr;
        }
    } else {
        T[rre * K + cre] += s * Cr;
        T[rre * K + cim] += s * Ci;
        if (rim >= 0) {
            T[rim * K + cre] += s * Ci;
            T[rim * K + cim] += -s * Cr;
        }
    }
}

}  // namespace

int build_operator_tables(int p, double *m2m, double *l2l, double *m2l)
{
    if (p < 0 || p > kMaxP) return -1;
    const int K = kcoef(p);
    std::vector<double> nut((2 * p + 1) * (2 * p + 1) * 2 + 2);
    auto NU = [&](int n, int m) { return nut[n * (2 * p + 1) + (m < 0 ? -m : m)]; };
    for (int n = 0; n <= 2 * p; ++n)
        for (int m = 0; m <= n; ++m) nut[n * (2 * p + 1) + m] = nu(n, m);

    for (int o = 0; o < 8; ++o) {
        const double dx = (((o >> 2) & 1) - 0.5) * 0.5;
        const double dy = (((o >> 1) & 1) - 0.5) * 0.5;
        const double dz = ((o & 1) - 0.5) * 0.5;
        const Harm h(p, dx, dy, dz);
        if (m2m) {
            double *T = m2m + (size_t)o * K * K;
            for (int i = 0; i < K * K; ++i) T[i] = 0.0;
            for (int n = 0; n <= p; ++n)
                for (int m = 0; m <= n; ++m)
                    for (int jp = 0; jp <= n; ++jp)        // input degree
                        for (int kp = -jp; kp <= jp; ++kp) {  // input order
                            const int j = n - jp, k = m - kp;
                            if (k < -j || k > j) continue;
                            const cd C = std::conj(h.R(j, k)) * std::ldexp(1.0, -jp) * NU(n, m) / (NU(j, k) * NU(jp, kp));
                            assemble(T, K, n, m, jp, kp, C);
                        }
        }
        if (l2l) {
            double *T = l2l + (size_t)o * K * K;
            for (int i = 0; i < K * K; ++i) T[i] = 0.0;
            for (int j = 0; j <= p; ++j)
                for (int k = 0; k <= j; ++k)
                    for (int n = j; n <= p; ++n)
                        for (int m = -n; m <= n; ++m) {
                            if (m - k < -(n - j) || m - k > n - j) continue;
                            const cd C = std::conj(h.R(n - j, m - k)) * std::ldexp(1.0, -(j + 1)) * NU(n, m) /
                                         (NU(n - j, m - k) * NU(j, k));
                            assemble(T, K, j, k, n, m, C);
                        }
        }
    }
    if (m2l) {
        for (int dx = -3; dx <= 3; ++dx)
            for (int dy = -3; dy <= 3; ++dy)
                for (int dz = -3; dz <= 3; ++dz) {
                    double *T = m2l + (size_t)((dx + 3) * 49 + (dy + 3) * 7 + (dz + 3)) * K * K;
                    for (int i = 0; i < K * K; ++i) T[i] = 0.0;
                    if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
                    const double tx = -dx, ty = -dy, tz = -dz;  // target minus source
                    const double r2 = tx * tx + ty * ty + tz * tz;
                    const Harm h(2 * p, tx, ty, tz);
                    for (int n = 0; n <= p; ++n)
                        for (int m = 0; m <= n; ++m)
                            for (int j = 0; j <= p; ++j)
                                for (int k = -j; k <= j; ++k) {
                                    const int N = j + n, Mo = k + m;
                                    const cd Ih = h.R(N, Mo) / std::pow(r2, N + 0.5);
                                    const cd C = ((n & 1) ? -1.0 : 1.0) * Ih * NU(N, Mo) / (NU(j, k) * NU(n, m));
                                    assemble(T, K, n, m, j, k, C);
                                }
                }
    }
    return 0;
}

void build_recurrence_table(int p, double *rec)
{
    const int Q = kq(p);
    for (int i = 0; i < kRecFields * Q; ++i) rec[i] = 0.0;
    for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m) {
            const int q = n * (n + 1) / 2 + m;
            if (n == m) rec[q] = m == 0 ? 1.0 : -std::sqrt((2.0 * m - 1.0) / (2.0 * m));
            else if (n == m + 1) rec[q] = std::sqrt(2.0 * m + 1.0);
            else {
                rec[q] = (2.0 * n - 1.0) / std::sqrt((double)(n + m) * (n - m));
                rec[Q + q] = std::sqrt((double)(n + m - 1) * (n - m - 1) / ((double)(n + m) * (n - m)));
            }
            if (n < p) {
                rec[2 * Q + q] = std::sqrt((double)(n + 1 + m) * (n + 1 - m)) * (m > 0 ? 2.0 : 1.0);
                rec[3 * Q + q] = std::sqrt((double)(n + m + 2) * (n + m + 1));
                rec[4 * Q + q] = std::sqrt((double)(n - m + 2) * (n - m + 1));
            }
        }
}

}  // namespace pt
