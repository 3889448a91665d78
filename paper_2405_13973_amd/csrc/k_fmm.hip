// Upward pass, downward pass and evaluation of the GPU FMM (Zaris et al.,
// Sec. 2.3): multipole expansions of the leaves (P2M), merged into parents
// (M2M), multipole-to-local conversion over the V lists (M2L), parent local
// expansions shifted to children (L2L), then per ion the far field of its
// leaf's local expansion (L2P) plus the near field by direct summation (P2P).
//
// T is the expansion / near-field type: double for the FP64 form, float for
// the mixed form.  Box centres, ion-to-centre offsets and the integrator stay
// FP64 in both; in the mixed form the offsets are rounded to FP32 only after
// the FP64 subtraction, and near-field sums are compensated (Kahan).
#include "fmm_math.hpp"
#include "pt_common.hpp"
#include "pt_kernels.hpp"

namespace pt {

__device__ inline int octant_of(int ix, int iy, int iz) { return ((ix & 1) << 2) | ((iy & 1) << 1) | (iz & 1); }

// Rh_n^m(u) by its column recurrence (m >= 0).
template <typename T>
__device__ inline void rhat_nm(int n, int m, T x, T y, T z, T &re, T &im)
{
    T dre = 1, dim = 0;
    for (int k = 1; k <= m; ++k) {
        const T f = -sqrt(T(2 * k - 1) / T(2 * k));
        const T a = f * (x * dre - y * dim);
        const T b = f * (x * dim + y * dre);
        dre = a;
        dim = b;
    }
    if (n == m) {
        re = dre;
        im = dim;
        return;
    }
    const T r2 = x * x + y * y + z * z;
    const T f1 = sqrt(T(2 * m + 1)) * z;
    T pre = dre, pim = dim, cre = f1 * dre, cim = f1 * dim;
    for (int k = m + 2; k <= n; ++k) {
        const T a = T(2 * k - 1) * z;
        const T b = sqrt(T((k + m - 1) * (k - m - 1))) * r2;
        const T inv = T(1) / sqrt(T((k + m) * (k - m)));
        const T nre = (a * cre - b * pre) * inv;
        const T nim = (a * cim - b * pim) * inv;
        pre = cre;
        pim = cim;
        cre = nre;
        cim = nim;
    }
    re = cre;
    im = cim;
}

// P2M: one block per box, threads over coefficients, ions in ascending order.
template <typename T>
__global__ __launch_bounds__(128) void k_p2m(BoxTable bt, const double *__restrict__ sp, int ntot, int p, int Kp,
                                             T *__restrict__ M)
{
    const int b = blockIdx.x;
    if (!bt.leaf[b]) return;
    const double4 g = bt.geo[b];
    const double ih = 1.0 / g.w;
    const int K = kcoef(p);
    const int i0 = bt.begin[b], i1 = bt.end[b];
    for (int s = threadIdx.x; s < Kp; s += blockDim.x) {
        T acc = 0;
        if (s < K) {
            const int n = (int)sqrt((double)s);
            const int r = s - n * n;
            const int m = (r + 1) >> 1;
            const bool is_im = r > 0 && !(r & 1);
            for (int i = i0; i < i1; ++i) {
                const T ux = (T)((sp[i] - g.x) * ih);
                const T uy = (T)((sp[ntot + i] - g.y) * ih);
                const T uz = (T)((sp[2 * ntot + i] - g.z) * ih);
                T re, im;
                rhat_nm<T>(n, m, ux, uy, uz, re, im);
                acc += is_im ? -im : re;
            }
        }
        M[(size_t)b * Kp + s] = acc;
    }
}

// M2M for the boxes [b0, b1) of one level: parent += T_m2m[octant(child)] child.
// Tt is column-major (Tt[o][j][i] = T[o][i][j]) so that threads read rows coalesced.
template <typename T>
__global__ __launch_bounds__(128) void k_m2m(BoxTable bt, int b0, int K, int Kp, const T *__restrict__ Tt,
                                             T *__restrict__ M)
{
    const int b = b0 + blockIdx.x;
    if (bt.leaf[b]) return;
    const int c0 = bt.child[b], c1 = c0 + bt.nchild[b];
    for (int i = threadIdx.x; i < Kp; i += blockDim.x) {
        T acc = 0;
        if (i < K)
            for (int ch = c0; ch < c1; ++ch) {
                const T *Tm = Tt + (size_t)octant_of(bt.ix[ch], bt.iy[ch], bt.iz[ch]) * K * K;
                const T *Mc = M + (size_t)ch * Kp;
                for (int j = 0; j < K; ++j) acc += Tm[(size_t)j * K + i] * Mc[j];
            }
        M[(size_t)b * Kp + i] = acc;
    }
}

// M2L into the boxes [b0, b1): L = sum over the window of T_m2l[offset] M_src.
// Boxes above level 2 get zero.
template <typename T>
__global__ __launch_bounds__(128) void k_m2l(BoxTable bt, int b0, int K, int Kp, const int32_t *__restrict__ vtab,
                                             const T *__restrict__ Tt, const T *__restrict__ M, T *__restrict__ L)
{
    const int b = b0 + blockIdx.x;
    const int cx = bt.ix[b] & 1, cy = bt.iy[b] & 1, cz = bt.iz[b] & 1;
    const int32_t *row = vtab + (size_t)b * kWin;
    const bool active = bt.level[b] >= 2;
    for (int i = threadIdx.x; i < Kp; i += blockDim.x) {
        T acc = 0;
        if (i < K && active)
            for (int w = 0; w < kWin; ++w) {
                const int src = row[w];
                if (src < 0) continue;
                const int dx = w / 36 - 2 - cx, dy = (w / 6) % 6 - 2 - cy, dz = w % 6 - 2 - cz;
                const T *Tm = Tt + (size_t)((dx + 3) * 49 + (dy + 3) * 7 + (dz + 3)) * K * K;
                const T *Ms = M + (size_t)src * Kp;
                for (int j = 0; j < K; ++j) acc += Tm[(size_t)j * K + i] * Ms[j];
            }
        L[(size_t)b * Kp + i] = acc;
    }
}

// L2L for the boxes [b0, b1) of one level (>= 3): child += T_l2l[octant] parent.
template <typename T>
__global__ __launch_bounds__(128) void k_l2l(BoxTable bt, int b0, int K, int Kp, const T *__restrict__ Tt,
                                             T *__restrict__ L)
{
    const int b = b0 + blockIdx.x;
    const int P = bt.parent[b];
    const T *Tm = Tt + (size_t)octant_of(bt.ix[b], bt.iy[b], bt.iz[b]) * K * K;
    const T *Lp = L + (size_t)P * Kp;
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
        T acc = 0;
        for (int j = 0; j < K; ++j) acc += Tm[(size_t)j * K + i] * Lp[j];
        L[(size_t)b * Kp + i] += acc;
    }
}

// Far field (L2P) + near field (P2P) of every ion of a leaf.  Writes the
// field per unit charge in batch order.
template <typename T>
__global__ __launch_bounds__(64) void k_eval(BoxTable bt, const double *__restrict__ sp, int ntot, int p, int Kp,
                                             const T *__restrict__ L, const int2 *__restrict__ near,
                                             const int32_t *__restrict__ near_cnt, int stride,
                                             const uint32_t *__restrict__ vals, int use_far, double *__restrict__ E)
{
    const int b = blockIdx.x;
    if (!bt.leaf[b]) return;
    const double4 g = bt.geo[b];
    const double ih = 1.0 / g.w;
    const T *Lb = L + (size_t)b * Kp;
    const int2 *row = near + (size_t)b * stride;
    const int nn = near_cnt[b];
    for (int k = bt.begin[b] + threadIdx.x; k < bt.end[b]; k += blockDim.x) {
        const double xd = sp[k], yd = sp[ntot + k], zd = sp[2 * ntot + k];
        double fx = 0.0, fy = 0.0, fz = 0.0;
        if (use_far) {
            T ex, ey, ez;
            l2p_field<T>(p, Lb, (T)((xd - g.x) * ih), (T)((yd - g.y) * ih), (T)((zd - g.z) * ih), ex, ey, ez);
            fx = (double)ex * ih * ih;
            fy = (double)ey * ih * ih;
            fz = (double)ez * ih * ih;
        }
        // near field, offsets from the target leaf centre
        const T xi = (T)(xd - g.x), yi = (T)(yd - g.y), zi = (T)(zd - g.z);
        T sx = 0, sy = 0, sz = 0, cx = 0, cy = 0, cz = 0;  // Kahan sums of per-range partials
        for (int r = 0; r < nn; ++r) {
            const int2 rg = row[r];
            T px = 0, py = 0, pz = 0;
            for (int j = rg.x; j < rg.y; ++j) {
                const T dx = xi - (T)(sp[j] - g.x);
                const T dy = yi - (T)(sp[ntot + j] - g.y);
                const T dz = zi - (T)(sp[2 * ntot + j] - g.z);
                const T r2 = dx * dx + dy * dy + dz * dz;
                const T ri = (r2 > T(0) && j != k) ? rsqrt(r2) : T(0);
                const T w = ri * ri * ri;
                px += dx * w;
                py += dy * w;
                pz += dz * w;
            }
            {
                T y_ = px - cx, t_ = sx + y_;
                cx = (t_ - sx) - y_;
                sx = t_;
                y_ = py - cy;
                t_ = sy + y_;
                cy = (t_ - sy) - y_;
                sy = t_;
                y_ = pz - cz;
                t_ = sz + y_;
                cz = (t_ - sz) - y_;
                sz = t_;
            }
        }
        const int gi = (int)vals[k];
        E[gi] = fx + (double)sx;
        E[ntot + gi] = fy + (double)sy;
        E[2 * ntot + gi] = fz + (double)sz;
    }
}

// ---------------------------------------------------------------- launchers

template <typename T>
void launch_upward(const BoxTable &bt, const double *sp, int ntot, int p, const TreeSummary &hs, const T *m2m_t,
                   T *M, hipStream_t st)
{
    const int K = kcoef(p), Kp = kpad(p);
    if (hs.nbox > 0) k_p2m<T><<<hs.nbox, 128, 0, st>>>(bt, sp, ntot, p, Kp, M);
    for (int l = kMaxLevel - 1; l >= 2; --l) {
        const int b0 = hs.level_start[l], b1 = hs.level_start[l + 1];
        if (b1 > b0) k_m2m<T><<<b1 - b0, 128, 0, st>>>(bt, b0, K, Kp, m2m_t, M);
    }
}

template <typename T>
void launch_m2l(const BoxTable &bt, int p, const TreeSummary &hs, const int32_t *vtab, const T *m2l_t, const T *M,
                T *L, hipStream_t st)
{
    const int K = kcoef(p), Kp = kpad(p);
    if (hs.nbox > 0) k_m2l<T><<<hs.nbox, 128, 0, st>>>(bt, 0, K, Kp, vtab, m2l_t, M, L);
}

template <typename T>
void launch_downward(const BoxTable &bt, int p, const TreeSummary &hs, const T *l2l_t, T *L, hipStream_t st)
{
    const int K = kcoef(p), Kp = kpad(p);
    for (int l = 3; l <= kMaxLevel; ++l) {
        const int b0 = hs.level_start[l], b1 = hs.level_start[l + 1];
        if (b1 > b0) k_l2l<T><<<b1 - b0, 128, 0, st>>>(bt, b0, K, Kp, l2l_t, L);
    }
}

template <typename T>
void launch_eval(const BoxTable &bt, const double *sp, int ntot, int p, int nbox, const T *L, const int2 *near,
                 const int32_t *near_cnt, int stride, const uint32_t *vals, int use_far, double *E, hipStream_t st)
{
    if (nbox > 0)
        k_eval<T><<<nbox, 64, 0, st>>>(bt, sp, ntot, p, kpad(p), L, near, near_cnt, stride, vals, use_far, E);
}

template void launch_upward<double>(const BoxTable &, const double *, int, int, const TreeSummary &, const double *,
                                    double *, hipStream_t);
template void launch_upward<float>(const BoxTable &, const double *, int, int, const TreeSummary &, const float *,
                                   float *, hipStream_t);
template void launch_m2l<double>(const BoxTable &, int, const TreeSummary &, const int32_t *, const double *,
                                 const double *, double *, hipStream_t);
template void launch_m2l<float>(const BoxTable &, int, const TreeSummary &, const int32_t *, const float *,
                                const float *, float *, hipStream_t);
template void launch_downward<double>(const BoxTable &, int, const TreeSummary &, const double *, double *,
                                      hipStream_t);
template void launch_downward<float>(const BoxTable &, int, const TreeSummary &, const float *, float *, hipStream_t);
template void launch_eval<double>(const BoxTable &, const double *, int, int, int, const double *, const int2 *,
                                  const int32_t *, int, const uint32_t *, int, double *, hipStream_t);
template void launch_eval<float>(const BoxTable &, const double *, int, int, int, const float *, const int2 *,
                                 const int32_t *, int, const uint32_t *, int, double *, hipStream_t);

}  // namespace pt
