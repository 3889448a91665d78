// Solid harmonics and expansion storage of the GPU fast multipole method.
//
// Expansions follow the paper's Sec. 2.3 (multipole expansion eq. FMM_coul,
// local expansion eq. FMM_local, truncation at degree p) in a basis chosen
// for the GPU: normalised regular solid harmonics
//     Rh_n^m(u) = sqrt((n-m)!/(n+m)!) (-1)^m r^n P_n^m(cos theta) e^{i m phi},  m >= 0
// (P without the Condon-Shortley sign), Rh_n^{-m} = (-1)^m conj(Rh_n^m), and
// irregular ones Ih_n^m(u) = Rh_n^m(u) / r^{2n+1}.  With these,
//     1/|x - a| = sum_{n,m} conj(Rh_n^m(a)) Ih_n^m(x)            (|a| < |x|).
// A box of side h and centre c stores
//     multipole  Mh_n^m = sum_i conj(Rh_n^m((x_i - c)/h))        (unit charges)
//                phi(x) = (1/h) sum Mh_n^m Ih_n^m((x - c)/h)
//     local      phi(x) = (1/h) sum Lh_n^m conj(Rh_n^m((x - c)/h))
// i.e. coefficients scaled by the box size, so that every translation
// operator between boxes of one level is independent of the level and all
// entries are O(1) (what makes FP32 usable).
//
// Real storage: for degree n, [Re c_n^0, Re c_n^1, Im c_n^1, ..., Re c_n^n, Im c_n^n]
// at offset n^2; K = (p+1)^2 reals per expansion, padded to a multiple of 16.
#pragma once

#include <cmath>

#include "pt_common.hpp"

namespace pt {

__host__ __device__ inline int kcoef(int p) { return (p + 1) * (p + 1); }
__host__ __device__ inline int kpad(int p) { return (kcoef(p) + 15) & ~15; }
__host__ __device__ inline int sidx_re(int n, int m) { return m == 0 ? n * n : n * n + 2 * m - 1; }
__host__ __device__ inline int sidx_im(int n, int m) { return n * n + 2 * m; }  // m > 0

// Rh_n^m(u) for 0 <= m <= n <= p, packed at n(n+1)/2 + m.  Recurrences:
//   Rh_m^m     = -sqrt((2m-1)/(2m)) (x + i y) Rh_{m-1}^{m-1}
//   Rh_{m+1}^m = sqrt(2m+1) z Rh_m^m
//   Rh_n^m     = ((2n-1) z Rh_{n-1}^m - sqrt((n+m-1)(n-m-1)) r^2 Rh_{n-2}^m) / sqrt((n+m)(n-m))
template <typename T>
__host__ __device__ inline void rhat_all(int p, T x, T y, T z, T *re, T *im)
{
    const T r2 = x * x + y * y + z * z;
    T dre = 1, dim = 0;  // Rh_m^m
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            const T f = -sqrt(T(2 * m - 1) / T(2 * m));
            const T nre = f * (x * dre - y * dim);
            const T nim = f * (x * dim + y * dre);
            dre = nre;
            dim = nim;
        }
        int i0 = m * (m + 1) / 2 + m;
        re[i0] = dre;
        im[i0] = dim;
        if (m + 1 > p) continue;
        const T f1 = sqrt(T(2 * m + 1)) * z;
        int i1 = (m + 1) * (m + 2) / 2 + m;
        re[i1] = f1 * dre;
        im[i1] = f1 * dim;
        for (int n = m + 2; n <= p; ++n) {
            const T a = T(2 * n - 1) * z;
            const T b = sqrt(T((n + m - 1) * (n - m - 1))) * r2;
            const T inv = T(1) / sqrt(T((n + m) * (n - m)));
            const int in = n * (n + 1) / 2 + m, i1_ = (n - 1) * n / 2 + m, i2 = (n - 2) * (n - 1) / 2 + m;
            re[in] = (a * re[i1_] - b * re[i2]) * inv;
            im[in] = (a * im[i1_] - b * im[i2]) * inv;
        }
    }
}

// Recurrence factors, per packed index q = n(n+1)/2 + m (0 <= m <= n <= p),
// stored as rec[f * Kq + q], Kq = (p+1)(p+2)/2:
//   f = 0 (ra): n == m:   -sqrt((2m-1)/(2m))  (1 for m = 0)   Rh_m^m = ra (x + i y) Rh_{m-1}^{m-1}
//               n == m+1: sqrt(2m+1)                          Rh_n^m = ra z Rh_{n-1}^m
//               n >= m+2: (2n-1)/sqrt((n+m)(n-m))             Rh_n^m = ra z Rh_{n-1}^m - rb r^2 Rh_{n-2}^m
//   f = 1 (rb): sqrt((n+m-1)(n-m-1)/((n+m)(n-m))) for n >= m+2, else 0
//   f = 2..4: L2P weights of Rh_n^m (n < p), see l2p_field:
//         sqrt((n+1+m)(n+1-m)) (doubled for m > 0), sqrt((n+m+2)(n+m+1)), sqrt((n-m+2)(n-m+1))
__host__ __device__ constexpr int kq(int p) { return (p + 1) * (p + 2) / 2; }
constexpr int kRecFields = 5;

// Field of a local expansion (L2P).  The expansion is re-centred exactly at
// the evaluation point u (box units); its degree-1 coefficients are
//   L'_1^k = sum_{n>=1,m} Lh_n^m conj(Rh_{n-1}^{m-k}(u)) nu_n^m / nu_{n-1}^{m-k},  k = 0, 1,
// and with R_1^0 = z, R_1^{+-1} = -+(x +- i y)/2 the field is
//   E h^2 = (Re L'_1^1, Im L'_1^1, -L'_1^0).
// Every Rh_{n'}^mu (mu >= 0) enters L'_1^1 twice: with Lh_{n'+1}^{mu+1} and,
// through the mirrored order -mu, with -conj(Lh_{n'+1}^{mu-1}).
// L is the real storage; the result is E * h^2 (caller divides by h^2).
template <typename T>
__host__ __device__ inline void l2p_field(int p, const T *L, const T *rec, T x, T y, T z, T &ex, T &ey, T &ez)
{
    const int Q = kq(p);
    const T r2 = x * x + y * y + z * z;
    T g0 = 0, g1r = 0, g1i = 0;
    T dre = 1, dim = 0;  // Rh_mu^mu
    for (int mu = 0; mu <= p - 1; ++mu) {
        if (mu > 0) {
            const T f = rec[mu * (mu + 1) / 2 + mu];
            const T nre = f * (x * dre - y * dim);
            const T nim = f * (x * dim + y * dre);
            dre = nre;
            dim = nim;
        }
        T r1re = 0, r1im = 0, r0re = 0, r0im = 0;  // Rh_{n-2}, Rh_{n-1} along the column
        for (int np = mu; np <= p - 1; ++np) {
            const int q = np * (np + 1) / 2 + mu;
            T cre, cim;  // Rh_np^mu
            if (np == mu) {
                cre = dre;
                cim = dim;
            } else {
                const T a = rec[q] * z, b = rec[Q + q] * r2;
                cre = a * r0re - b * r1re;
                cim = a * r0im - b * r1im;
            }
            r1re = r0re;
            r1im = r0im;
            r0re = cre;
            r0im = cim;
            const int n = np + 1;
            {  // k = 0: Lh_n^mu conj(Rh), doubled for mu > 0 (mirror term)
                const T lre = L[sidx_re(n, mu)];
                const T lim = mu > 0 ? L[sidx_im(n, mu)] : T(0);
                g0 += rec[2 * Q + q] * (lre * cre + lim * cim);
            }
            {  // k = 1, (a): Lh_n^{mu+1} conj(Rh_np^mu)
                const T lre = L[sidx_re(n, mu + 1)];
                const T lim = L[sidx_im(n, mu + 1)];
                const T w = rec[3 * Q + q];
                g1r += w * (lre * cre + lim * cim);
                g1i += w * (lim * cre - lre * cim);
            }
            if (mu >= 1) {  // k = 1, (b): -conj(Lh_n^{mu-1}) Rh_np^mu
                const T lre = L[sidx_re(n, mu - 1)];
                const T lim = mu - 1 > 0 ? L[sidx_im(n, mu - 1)] : T(0);
                const T w = rec[4 * Q + q];
                g1r -= w * (lre * cre + lim * cim);
                g1i -= w * (lre * cim - lim * cre);
            }
        }
    }
    ex = g1r;
    ey = g1i;
    ez = -g0;
}

// Field and value of a local expansion: l2p_field's field, plus the value
//   phi h = sum_{n<=p} [Lh_n^0 Rh_n^0 + 2 sum_{m>0} Re(Lh_n^m conj(Rh_n^m))]
// (orders m and -m of a real potential are complex conjugates); the columns
// run to degree p for the value, the field terms stop at degree p - 1.
template <typename T>
__host__ __device__ inline void l2p_field_pot(int p, const T *L, const T *rec, T x, T y, T z, T &ex, T &ey, T &ez,
                                              T &pot)
{
    const int Q = kq(p);
    const T r2 = x * x + y * y + z * z;
    T g0 = 0, g1r = 0, g1i = 0, v = 0;
    T dre = 1, dim = 0;  // Rh_mu^mu
    for (int mu = 0; mu <= p; ++mu) {
        if (mu > 0) {
            const T f = rec[mu * (mu + 1) / 2 + mu];
            const T nre = f * (x * dre - y * dim);
            const T nim = f * (x * dim + y * dre);
            dre = nre;
            dim = nim;
        }
        T r1re = 0, r1im = 0, r0re = 0, r0im = 0;
        for (int np = mu; np <= p; ++np) {
            const int q = np * (np + 1) / 2 + mu;
            T cre, cim;  // Rh_np^mu
            if (np == mu) {
                cre = dre;
                cim = dim;
            } else {
                const T a = rec[q] * z, b = rec[Q + q] * r2;
                cre = a * r0re - b * r1re;
                cim = a * r0im - b * r1im;
            }
            r1re = r0re;
            r1im = r0im;
            r0re = cre;
            r0im = cim;
            if (mu == 0) v += L[sidx_re(np, 0)] * cre;
            else v += T(2) * (L[sidx_re(np, mu)] * cre + L[sidx_im(np, mu)] * cim);
            if (np == p) continue;
            const int n = np + 1;
            {
                const T lre = L[sidx_re(n, mu)];
                const T lim = mu > 0 ? L[sidx_im(n, mu)] : T(0);
                g0 += rec[2 * Q + q] * (lre * cre + lim * cim);
            }
            {
                const T lre = L[sidx_re(n, mu + 1)];
                const T lim = L[sidx_im(n, mu + 1)];
                const T w = rec[3 * Q + q];
                g1r += w * (lre * cre + lim * cim);
                g1i += w * (lim * cre - lre * cim);
            }
            if (mu >= 1) {
                const T lre = L[sidx_re(n, mu - 1)];
                const T lim = mu - 1 > 0 ? L[sidx_im(n, mu - 1)] : T(0);
                const T w = rec[4 * Q + q];
                g1r -= w * (lre * cre + lim * cim);
                g1i -= w * (lre * cim - lim * cre);
            }
        }
    }
    ex = g1r;
    ey = g1i;
    ez = -g0;
    pot = v;
}

// conj(Rh_n^m(u)) of one point in real storage order into out[s * stride]
// (s the storage index), from the recurrence table; only the orders m in
// [m_lo, m_hi) are written (each by the same operations as in a full pass).
template <typename T>
__host__ __device__ inline void p2m_terms(int p, const T *rec, T x, T y, T z, T *out, int stride, int m_lo = 0,
                                          int m_hi = 1 << 30)
{
    const int Q = kq(p);
    const T r2 = x * x + y * y + z * z;
    T dre = 1, dim = 0;
    for (int m = 0; m <= p && m < m_hi; ++m) {
        if (m > 0) {
            const T f = rec[m * (m + 1) / 2 + m];
            const T nre = f * (x * dre - y * dim);
            const T nim = f * (x * dim + y * dre);
            dre = nre;
            dim = nim;
        }
        if (m < m_lo) continue;
        T r1re = 0, r1im = 0, r0re = 0, r0im = 0;
        for (int n = m; n <= p; ++n) {
            const int q = n * (n + 1) / 2 + m;
            T cre, cim;
            if (n == m) {
                cre = dre;
                cim = dim;
            } else {
                const T a = rec[q] * z, b = rec[Q + q] * r2;
                cre = a * r0re - b * r1re;
                cim = a * r0im - b * r1im;
            }
            r1re = r0re;
            r1im = r0im;
            r0re = cre;
            r0im = cim;
            out[sidx_re(n, m) * stride] = cre;
            if (m > 0) out[sidx_im(n, m) * stride] = -cim;
        }
    }
}

// Reflections of space act on the coefficients as diagonal +-1 matrices S:
// z -> -z multiplies c_n^m by (-1)^(n+m); y -> -y conjugates (Im -> -Im);
// x -> -x gives (-1)^m conj.  Hence the M2L operator of source offset
// d = (dx, dy, dz) is T_d = S T_|d| S with S the reflections of the negative
// components, and only the 56 operators of offsets with non-negative
// components are stored.  refl_bits(i) packs, for storage index i, whether
// the x (bit 0), y (bit 1), z (bit 2) reflection flips its sign; a mask of
// reflections flips it iff popcount(mask & refl_bits) is odd.
__host__ __device__ inline int refl_bits(int i)
{
    const int n = (int)sqrt((double)i + 0.5);
    const int r = i - n * n;
    const int m = (r + 1) >> 1;
    const int im = (r > 0 && !(r & 1)) ? 1 : 0;
    return ((m & 1) ^ im) | (im << 1) | (((n + m) & 1) << 2);
}
// index of the stored M2L operator for |offset| (each component 0..3)
__host__ __device__ inline int m2l_base(int ax, int ay, int az) { return ax * 16 + ay * 4 + az; }

// Host-only: recurrence table (kRecFields x kq(p) doubles), see above.
void build_recurrence_table(int p, double *rec);

// Host-only: the dense real operator matrices (row = output coefficient,
// column = input coefficient, K x K each, row-major) for degree p:
//   m2m[8]  child octant o -> parent  (child centre at parent centre + ((2o-1)/4) h_parent)
//   l2l[8]  parent -> child octant o
//   m2l[343] source box at integer offset d = (dx,dy,dz) in [-3,3]^3 from the
//            target box (same level), index (dx+3)*49 + (dy+3)*7 + (dz+3);
//            entries of touching offsets are left zero.
// Returns 0 on success.
int build_operator_tables(int p, double *m2m, double *l2l, double *m2l);

}  // namespace pt
