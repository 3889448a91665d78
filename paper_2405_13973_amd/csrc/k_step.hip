// Integrator, photon kicks, bounding boxes, Morton keys and the direct
// Coulomb sum.  All kernels are batched: a launch covers every ion of every
// crystal in the batch; ion_crystal[g] maps a batch index to its crystal.
//
// Step (Zaris et al., Sec. 2.2, eq. time_ev2):
//   U0(dt/2) -> kick at t + dt/2 (eq. velocity_kick: trap + wall + Coulomb,
//   plus Poisson photon recoils of eq. laser_kick) -> U0(dt/2),
// U0 the exact gyration about B z-hat (eq. U0, rotation sense of the
// Lorentz force on q B > 0: clockwise) with free flight along z.
#include <algorithm>

#include "pt_common.hpp"
#include "pt_kernels.hpp"

namespace pt {

// Exact U0(dt/2): v rotates by -omega_c dt/2 about z; x moves along the arc.
// Every multiply-add is an explicit fma, so that each kernel that makes the
// half drift (the bounding-box kernel, the kick that also makes the next
// step's drift) computes the same bits.
__device__ inline void u0_half(const CrystalDev &c, double &x, double &y, double &z, double &vx, double &vy,
                               double vz)
{
    const double nx = fma(vy, c.b_half, fma(vx, c.a_half, x));
    const double ny = fma(vy, c.a_half, fma(-vx, c.b_half, y));
    const double nvx = fma(vy, c.s_half, vx * c.c_half);
    const double nvy = fma(vy, c.c_half, -vx * c.s_half);
    x = nx;
    y = ny;
    z = fma(vz, 0.5 * c.dt, z);
    vx = nvx;
    vy = nvy;
}

__global__ void k_ion_crystal(const CrystalDev *__restrict__ cs, int nc, int ntot, int32_t *__restrict__ ion_crystal)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ntot) return;
    int lo = 0, hi = nc - 1;  // last crystal with ion_off <= g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cs[mid].ion_off <= g) lo = mid;
        else hi = mid - 1;
    }
    ion_crystal[g] = lo;
}

__global__ void k_zero_words(uint64_t *__restrict__ p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_fill_u64(uint64_t *__restrict__ p, uint64_t v0, uint64_t v1, int n_pairs)
{
    // pattern: six words per crystal, three v0 then three v1
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pairs * 6) p[i] = (i % 6) < 3 ? v0 : v1;
}

// Per-crystal min/max of the positions of the block's active threads into the
// bounding-box copy of this workgroup (ordered-integer atomics): a wave
// reduction when the wave is uniform in crystal, then a block reduction
// through LDS when all its waves agree; else per-wave atomics.  Called by every
// thread of the workgroup.
__device__ void bbox_add(bool active, int c, double x, double y, double z, unsigned long long *__restrict__ bbox_all,
                         int bstride)
{
    unsigned long long *bbox = bbox_all + (size_t)(blockIdx.x % kBBoxCopies) * bstride;
    unsigned long long v[6] = {~0ull, ~0ull, ~0ull, 0ull, 0ull, 0ull};
    if (active) {
        v[0] = dbl_to_ordered(x);
        v[1] = dbl_to_ordered(y);
        v[2] = dbl_to_ordered(z);
        v[3] = v[0];
        v[4] = v[1];
        v[5] = v[2];
    }
    __shared__ unsigned long long wv[4][6];
    __shared__ int wc[4];
    const unsigned long long act = __ballot(active);
    const int first = act ? __ffsll((long long)act) - 1 : 0;
    const int cref = __shfl(c, first);
    const bool uniform = act != 0 && __ballot(active && c != cref) == 0;
    if (uniform) {
        for (int off = 32; off > 0; off >>= 1)
            for (int k = 0; k < 6; ++k) {
                const unsigned long long o = __shfl_xor(v[k], off);
                v[k] = k < 3 ? (o < v[k] ? o : v[k]) : (o > v[k] ? o : v[k]);
            }
    } else if (active) {
        for (int k = 0; k < 6; ++k) {
            if (k < 3) atomicMin(&bbox[6 * c + k], v[k]);
            else atomicMax(&bbox[6 * c + k], v[k]);
        }
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        wc[w] = uniform ? cref : (act ? -1 : -2);  // -2: no ion in this wave
        for (int k = 0; k < 6; ++k) wv[w][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        int cb = -3;
        bool same = true;
        for (int k = 0; k < nw; ++k) {
            if (wc[k] == -2) continue;
            if (wc[k] == -1 || (cb != -3 && wc[k] != cb)) same = false;
            cb = wc[k];
        }
        if (same && cb >= 0) {
            unsigned long long r[6] = {~0ull, ~0ull, ~0ull, 0ull, 0ull, 0ull};
            for (int k = 0; k < nw; ++k)
                if (wc[k] >= 0)
                    for (int j = 0; j < 6; ++j) r[j] = j < 3 ? (wv[k][j] < r[j] ? wv[k][j] : r[j])
                                                             : (wv[k][j] > r[j] ? wv[k][j] : r[j]);
            for (int j = 0; j < 6; ++j) {
                if (j < 3) atomicMin(&bbox[6 * cb + j], r[j]);
                else atomicMax(&bbox[6 * cb + j], r[j]);
            }
        } else {
            for (int k = 0; k < nw; ++k)
                if (wc[k] >= 0)
                    for (int j = 0; j < 6; ++j) {
                        if (j < 3) atomicMin(&bbox[6 * wc[k] + j], wv[k][j]);
                        else atomicMax(&bbox[6 * wc[k] + j], wv[k][j]);
                    }
        }
    }
}

// Optional half drift of the state into the working copy (positions only
// are copied without the drift), then per-crystal min/max of x, y, z
// (ordered-integer atomics; min/max is exact, so the result does not depend
// on the order).  The regions of zr are zeroed on the way (grid-stride).
__global__ void k_drift_bbox(const CrystalDev *__restrict__ cs, const int32_t *__restrict__ ion_crystal, int ntot,
                             int do_drift, unsigned long long *__restrict__ bbox_all, int bstride,
                             const int32_t *__restrict__ halt, ZeroRegions zr)
{
    if (halt && *halt) return;  // a halted run: the same word for every workgroup
    for (int r = 0; r < kZeroRegions; ++r)  // counters of the steps that follow start at zero
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < zr.n[r]; i += gridDim.x * blockDim.x)
            zr.p[r][i] = 0ull;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = g < ntot;
    int c = 0;
    double x = 0.0, y = 0.0, z = 0.0;
    if (active) {
        c = ion_crystal[g];
        const CrystalDev &cd = cs[c];
        const int i = g - cd.ion_off;
        const int n = cd.n;
        const double *s = cd.state;
        double *m = cd.mid;
        x = s[i];
        y = s[n + i];
        z = s[2 * n + i];
        if (do_drift) {
            double vx = s[3 * n + i], vy = s[4 * n + i];
            const double vz = s[5 * n + i];
            u0_half(cd, x, y, z, vx, vy, vz);
            m[3 * n + i] = vx;
            m[4 * n + i] = vy;
            m[5 * n + i] = vz;
        }
        m[i] = x;
        m[n + i] = y;
        m[2 * n + i] = z;
    }
    bbox_add(active, c, x, y, z, bbox_all, bstride);
}

// Root cube of every crystal (one thread each).
__global__ void k_roots(const unsigned long long *__restrict__ bbox, int nc, int bstride, RootCube *__restrict__ roots)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nc) roots[c] = root_of(bbox, bstride, c);
}

// Sort keys and values of every ion (ion_sort_key).
__global__ void k_keys(const CrystalDev *__restrict__ cs, const int32_t *__restrict__ ion_crystal,
                       const RootCube *__restrict__ roots, int ntot, uint64_t *__restrict__ keys,
                       uint32_t *__restrict__ vals, const int32_t *__restrict__ halt)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ntot || (halt && *halt)) return;
    keys[g] = ion_sort_key(cs, ion_crystal, roots, g);
    vals[g] = (uint32_t)g;
}

// Kick at the midpoint time and the second half drift.  E holds the Coulomb
// field per unit charge (sum_j (x_i - x_j)/r^3) in batch order, SoA, or,
// with kp.part set, its far field, to which the ion's near-field item
// partials are added here in item order (as the far-field kernel would add
// them, the same FP64 values).  BEAMS:
// some crystal of the batch uses the beam-mode laser (the variant that holds
// the per-beam rate and count code).  NEXT: the next step of the same batch
// follows, and its first half drift is done here as well, from the state
// just computed (as k_drift_bbox would read it back): the working copy, the
// bounding boxes, and the regions of zr zeroed.
template <bool BEAMS, bool NEXT>
__global__ void k_kick_drift(const CrystalDev *__restrict__ cs, const int32_t *__restrict__ ion_crystal, int ntot,
                             int kstep, const double *__restrict__ E, TreeSummary *__restrict__ sum, int call_k,
                             ZeroRegions zr, unsigned long long *__restrict__ bbox_all, int bstride, KickPartials kp)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (sum && sum->halt) {
        // the step's tree or lists did not fit their buffers: the state stays
        // at the last completed step, which the host reads from fail_step
        // (the whole grid returns: the word is the same for every workgroup)
        if (g == 0 && sum->fail_step < 0) sum->fail_step = call_k;
        return;
    }
    const bool active = g < ntot;
    int c = 0;
    double bx = 0.0, by = 0.0, bz = 0.0;  // the next step's drifted position (NEXT)
    if (active) {
    c = ion_crystal[g];
    const CrystalDev &cd = cs[c];
    const int i = g - cd.ion_off;
    const int n = cd.n;
    double *m = cd.mid;
    double *s = cd.state;
    double x = m[i], y = m[n + i], z = m[2 * n + i];
    double vx = m[3 * n + i], vy = m[4 * n + i], vz = m[5 * n + i];
    // artificial damping, first half: the velocity relative to the rigid
    // clockwise rotation omega_r (y, -x, 0) (at rest in the rotating frame)
    // shrinks by exp(-damping dt / 2)
    auto damp_half = [&]() {
        const double rx = cd.omega_r * y, ry = -cd.omega_r * x;
        vx = rx + cd.damp_f * (vx - rx);
        vy = ry + cd.damp_f * (vy - ry);
        vz = cd.damp_f * vz;
    };
    if (cd.damp_on) damp_half();
    const uint64_t step = cd.step0 + (uint64_t)kstep;
    const double t = cd.t0 + (double)step * cd.dt;
    const double tm = t + 0.5 * cd.dt;
    // trap: -q grad(k_z (2z^2 - x^2 - y^2)/4)
    double fx = 0.5 * cd.qkz * x, fy = 0.5 * cd.qkz * y, fz = -cd.qkz * z;
    if (cd.delta != 0.0) {  // rotating wall at the midpoint time
        const double C = cos(2.0 * cd.omega_r * tm), S = sin(2.0 * cd.omega_r * tm);
        const double w = 0.5 * cd.qkz * cd.delta;
        fx -= w * (x * C - y * S);
        fy += w * (y * C + x * S);
    }
    double ex = E[g], ey = E[ntot + g], ez = E[2 * ntot + g];
    if (kp.part) {
        const int2 po = kp.poff[g];
        if (kp.f32) {
            const float *pp = static_cast<const float *>(kp.part) + (size_t)po.x * 3;
            for (int j = 0; j < po.y; ++j, pp += 64 * 3) {
                ex += (double)pp[0];
                ey += (double)pp[1];
                ez += (double)pp[2];
            }
        } else {
            const double *pp = static_cast<const double *>(kp.part) + (size_t)po.x * 3;
            for (int j = 0; j < po.y; ++j, pp += 64 * 3) {
                ex += pp[0];
                ey += pp[1];
                ez += pp[2];
            }
        }
    }
    fx += cd.coul * ex;
    fy += cd.coul * ey;
    fz += cd.coul * ez;
    const double vmx = vx, vmy = vy, vmz = vz;  // midpoint velocity, before the kick (beam rates)
    const double kdt = cd.dt * cd.inv_m;
    vx += fx * kdt;
    vy += fy * kdt;
    vz += fz * kdt;
    int32_t nph = 0;
    if (BEAMS && cd.laser_on == 2) {
        // beams, eq. (scattering_rate): per beam a Poisson count with mean
        // rate * dt (slot l << 16), then per photon an absorption recoil
        // along khat and an isotropic emission recoil (slots (l << 16) | j)
        const uint32_t k0 = (uint32_t)cd.seed, k1 = (uint32_t)(cd.seed >> 32);
        const double g2 = 0.25 * cd.gamma0 * cd.gamma0;
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int l = 0; l < cd.n_beams; ++l) {
            const BeamDev &b = cd.beam[l];
            double S = b.s0;
            if (!b.uniform) {
                const double dy = y - b.offset_y;
                S = b.s0 * exp(-(dy * dy / (b.waist_y * b.waist_y) + z * z / (b.waist_z * b.waist_z)));
            }
            const double kv = cd.kwave * (b.khat[0] * vmx + b.khat[1] * vmy + b.khat[2] * vmz);
            const double dd = b.detuning - kv;
            const double lam = S * cd.gamma0 * g2 / (g2 * (1.0 + 2.0 * S) + dd * dd) * cd.dt;
            uint32_t w[4] = {(uint32_t)i, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)l << 16};
            philox4x32_10(w, k0, k1);
            const double u = u53(w[0], w[1]);
            // inversion of the Poisson CDF p_0 = e^-lam, p_k = p_{k-1} lam / k
            double pk = exp(-lam), F = pk;
            int cnt = 16;
            for (int k = 0; k <= 16; ++k) {
                if (k > 0) {
                    pk = pk * lam / (double)k;
                    F = F + pk;
                }
                if (u < F) {
                    cnt = k;
                    break;
                }
            }
            double ex = 0.0, ey = 0.0, ez = 0.0;
            for (int j = 1; j <= cnt; ++j) {
                uint32_t d[4] = {(uint32_t)i, (uint32_t)step, (uint32_t)(step >> 32), ((uint32_t)l << 16) | (uint32_t)j};
                philox4x32_10(d, k0, k1);
                const double ct = 2.0 * u53(d[0], d[1]) - 1.0;
                const double ph = 2.0 * kPi * u53(d[2], d[3]);
                const double st = sqrt(1.0 - ct * ct);
                double sp, cp;
                sincos(ph, &sp, &cp);
                ex += st * cp;
                ey += st * sp;
                ez += ct;
            }
            ax += cd.recoil * ((double)cnt * b.khat[0] + ex);
            ay += cd.recoil * ((double)cnt * b.khat[1] + ey);
            az += cd.recoil * ((double)cnt * b.khat[2] + ez);
            nph += cnt;
        }
        vx += ax;
        vy += ay;
        vz += az;
    } else if (cd.laser_on) {
        uint32_t w[4] = {(uint32_t)i, (uint32_t)step, (uint32_t)(step >> 32), 0u};
        const uint32_t k0 = (uint32_t)cd.seed, k1 = (uint32_t)(cd.seed >> 32);
        philox4x32_10(w, k0, k1);
        const double u = u53(w[0], w[1]);
        nph = 16;
        for (int k = 0; k <= 16; ++k)
            if (u < cd.poisson_F[k]) {
                nph = k;
                break;
            }
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int j = 1; j <= nph; ++j) {
            uint32_t d[4] = {(uint32_t)i, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)j};
            philox4x32_10(d, k0, k1);
            const double ct = 2.0 * u53(d[0], d[1]) - 1.0;
            const double ph = 2.0 * kPi * u53(d[2], d[3]);
            const double st = sqrt(1.0 - ct * ct);
            double sp, cp;
            sincos(ph, &sp, &cp);
            ax += st * cp;
            ay += st * sp;
            az += ct;
        }
        vx += cd.recoil * ax;
        vy += cd.recoil * ay;
        vz += cd.recoil * az;
    }
    cd.photons[i] = nph;
    if (cd.damp_on) damp_half();  // second half, after the kick
    u0_half(cd, x, y, z, vx, vy, vz);
    s[i] = x;
    s[n + i] = y;
    s[2 * n + i] = z;
    s[3 * n + i] = vx;
    s[4 * n + i] = vy;
    s[5 * n + i] = vz;
    // a non-finite value is flagged for the host, which reports it at its
    // next synchronising call (plain stores: every writer writes 1)
    if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(vx) && isfinite(vy) && isfinite(vz))) {
        *cd.nonfinite = 1;
        *cd.ctx_nonfinite = 1;
    }
    if constexpr (NEXT) {
        u0_half(cd, x, y, z, vx, vy, vz);
        m[i] = x;
        m[n + i] = y;
        m[2 * n + i] = z;
        m[3 * n + i] = vx;
        m[4 * n + i] = vy;
        m[5 * n + i] = vz;
        bx = x;
        by = y;
        bz = z;
    }
    }
    if constexpr (NEXT) {
        for (int r = 0; r < kZeroRegions; ++r)  // counters of the next evaluation start at zero
            for (int j = g; j < zr.n[r]; j += gridDim.x * blockDim.x) zr.p[r][j] = 0ull;
        bbox_add(active, c, bx, by, bz, bbox_all, bstride);
    }
}

// Direct Coulomb field E_i = sum_{j != i} (x_i - x_j)/|x_i - x_j|^3 (FP64);
// with POT also the potential sum_{j != i} 1/|x_i - x_j| (both per unit
// charge; the pair term of eq. hamiltonian).  Work split: direct_chunks.
//
// First level: block (c, first, chunk) takes targets first + lane + 64 t of
// crystal c and chunk `chunk` of its sources.  Each wave walks its own piece
// of the chunk in ascending order, kDirUnroll sources at a time; the source index
// is the same for the whole wave, so the sources arrive by scalar loads and
// enter the arithmetic as scalar operands, with no LDS staging or barrier in
// the loop.  The block's waves then add their sums in wave order through LDS
// and store the chunk's partials.
//
// Pair arithmetic.  r2 carries an offset of 2^-680, below the rounding of
// any r2 above 2^-626 (separations above 1e-94 m), so that r2 > 0 also for
// coincident ions.  r^-3 comes from the hardware reciprocal square root y0,
// whose relative error is about 5e-8, by the second-order correction
//   r^-3 = y0^3 (1 - e)^(-3/2) = y0^3 (1 + 3/2 e + 15/8 e^2 + O(e^3)),  e = 1 - r2 y0^2,
// which is within an ulp or two of the correctly rounded value (the e^3 term is
// below 1e-22).  A pair at zero separation contributes nothing: its
// dx = dy = dz = 0 multiply a finite weight (about 2^1020), and for the
// potential it is masked.  That includes j = i, so the loop has no index
// test and no branch.
constexpr double kDirR2Offset = 0x1p-680;
constexpr int kDirUnroll = 4;  // sources per scalar load of each coordinate

template <bool POT>
__global__ __launch_bounds__(64 * kDirWaves) __attribute__((amdgpu_waves_per_eu(8))) void k_direct(const CrystalDev *__restrict__ cs,
                                                           const DirBlock *__restrict__ tab,
                                                           double *__restrict__ part)
{
    constexpr int NC = POT ? 4 : 3;
    __shared__ double red[kDirWaves - 1][NC][kDirTile];
    const DirBlock blk = tab[blockIdx.x];
    const CrystalDev &cd = cs[blk.c];
    const int n = cd.n, chunks = direct_chunks(n), len = direct_piece(n);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int j0 = min(n, (blk.chunk * kDirWaves + wave) * len), j1 = min(n, j0 + len);
    // the positions, as global memory: with the wave-uniform index below the
    // compiler then reads them with scalar loads
    using gdouble = const __attribute__((address_space(1))) double;
    gdouble *__restrict__ x = (gdouble *)cd.mid;
    gdouble *__restrict__ y = x + n;
    gdouble *__restrict__ z = y + n;
    double xi[kDirT], yi[kDirT], zi[kDirT], acc[kDirT][NC];
#pragma unroll
    for (int t = 0; t < kDirT; ++t) {
        const int i = blk.first + 64 * t + lane;
        const int ii = i < n ? i : 0;
        xi[t] = x[ii];
        yi[t] = y[ii];
        zi[t] = z[ii];
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[t][k] = 0.0;
    }
    // the correction's constants, held in registers (a VGPR and an SGPR) so
    // that the compiler neither rematerialises them per pair nor needs two
    // scalar operands in one instruction
    double c15 = 1.5, c1875 = 1.875, c05 = 0.5, c0375 = 0.375;
    __asm__("" : "+v"(c15));
    __asm__("" : "+s"(c1875));
    if constexpr (POT) {
        __asm__("" : "+v"(c05));
        __asm__("" : "+s"(c0375));
    }
    auto add_source = [&](double xj, double yj, double zj) {
#pragma unroll
        for (int t = 0; t < kDirT; ++t) {
            const double dx = xi[t] - xj, dy = yi[t] - yj, dz = zi[t] - zj;
            const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, kDirR2Offset)));
            const double y0 = __builtin_amdgcn_rsq(r2);
            const double y2 = y0 * y0;
            const double y3 = y2 * y0;
            const double e = fma(-r2, y2, 1.0);
            const double w = fma(y3, e * fma(e, c1875, c15), y3);
            acc[t][0] = fma(dx, w, acc[t][0]);
            acc[t][1] = fma(dy, w, acc[t][1]);
            acc[t][2] = fma(dz, w, acc[t][2]);
            if constexpr (POT) {
                // r^-1 = y0 (1 + e/2 + 3/8 e^2 + O(e^3))
                const double ri = fma(y0 * e, fma(e, c0375, c05), y0);
                acc[t][NC - 1] += r2 > kDirR2Offset ? ri : 0.0;
            }
        }
    };
    int j = j0;
    for (; j + kDirUnroll <= j1; j += kDirUnroll) {
#pragma unroll
        for (int u = 0; u < kDirUnroll; ++u) add_source(x[j + u], y[j + u], z[j + u]);
    }
    for (; j < j1; ++j) add_source(x[j], y[j], z[j]);
    if (wave > 0) {
#pragma unroll
        for (int t = 0; t < kDirT; ++t)
#pragma unroll
            for (int k = 0; k < NC; ++k) red[wave - 1][k][64 * t + lane] = acc[t][k];
    }
    __syncthreads();
    if (wave == 0) {
        double *__restrict__ out = part + cd.dpart + (size_t)blk.chunk * n;
#pragma unroll
        for (int t = 0; t < kDirT; ++t) {
            const int i = blk.first + 64 * t + lane;
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                double a = acc[t][k];
                for (int w = 0; w < kDirWaves - 1; ++w) a += red[w][k][64 * t + lane];
                if (i < n) out[(size_t)k * chunks * n + i] = a;
            }
        }
    }
}

// Second level: ion g adds its crystal's chunk partials in chunk order.
template <bool POT>
__global__ void k_direct_finish(const CrystalDev *__restrict__ cs, const int32_t *__restrict__ ion_crystal, int ntot,
                                const double *__restrict__ part, double *__restrict__ E, double *__restrict__ PHI)
{
    constexpr int NC = POT ? 4 : 3;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ntot) return;
    const CrystalDev &cd = cs[ion_crystal[g]];
    const int n = cd.n, chunks = direct_chunks(n);
    const double *__restrict__ p = part + cd.dpart + (g - cd.ion_off);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        double a = p[(size_t)k * chunks * n];
        for (int s = 1; s < chunks; ++s) a += p[((size_t)k * chunks + s) * n];
        if (k < 3) E[(size_t)k * ntot + g] = a;
        else PHI[g] = a;
    }
}

// ---------------------------------------------------------------- launchers

void launch_ion_crystal(const CrystalDev *cs, int nc, int ntot, int32_t *ion_crystal, hipStream_t st)
{
    if (ntot > 0) k_ion_crystal<<<ceil_div(ntot, 256), 256, 0, st>>>(cs, nc, ntot, ion_crystal);
}

void launch_bbox_reset(unsigned long long *bbox, int nc, hipStream_t st)
{
    const int pairs = (int)(bbox_words(nc) / 6);
    k_fill_u64<<<ceil_div(6 * pairs, 256), 256, 0, st>>>((uint64_t *)bbox, ~0ull, 0ull, pairs);
}

// Up to kZeroRegions regions of 64-bit words zeroed by one launch.
__global__ void k_zero_regions(ZeroRegions z)
{
    const int r = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < z.n[r]; i += gridDim.x * blockDim.x) z.p[r][i] = 0ull;
}

void launch_zero_regions(const ZeroRegions &z, hipStream_t st)
{
    int most = 0;
    for (int r = 0; r < kZeroRegions; ++r) most = std::max(most, z.n[r]);
    if (most > 0) k_zero_regions<<<dim3(std::min(ceil_div(most, 256), 64), kZeroRegions), 256, 0, st>>>(z);
}

void launch_zero_u64(uint64_t *p, int n, hipStream_t st)
{
    if (n > 0) k_zero_words<<<ceil_div(n, 256), 256, 0, st>>>(p, n);
}

void launch_drift_bbox(const CrystalDev *cs, const int32_t *ion_crystal, int ntot, int nc, int do_drift,
                       unsigned long long *bbox, const int32_t *halt, const ZeroRegions &zr, hipStream_t st)
{
    if (ntot > 0)
        k_drift_bbox<<<ceil_div(ntot, 256), 256, 0, st>>>(cs, ion_crystal, ntot, do_drift, bbox, bbox_stride(nc), halt,
                                                          zr);
}

void launch_roots(const unsigned long long *bbox, int nc, RootCube *roots, hipStream_t st)
{
    k_roots<<<ceil_div(nc, 64), 64, 0, st>>>(bbox, nc, bbox_stride(nc), roots);
}

void launch_keys(const CrystalDev *cs, const int32_t *ion_crystal, const RootCube *roots, int ntot, uint64_t *keys,
                 uint32_t *vals, const int32_t *halt, hipStream_t st)
{
    if (ntot > 0) k_keys<<<ceil_div(ntot, 256), 256, 0, st>>>(cs, ion_crystal, roots, ntot, keys, vals, halt);
}

void launch_kick_drift(const CrystalDev *cs, const int32_t *ion_crystal, int ntot, int kstep, const double *E,
                       bool beams, TreeSummary *sum, int call_k, const NextDrift *next, const KickPartials *kp,
                       hipStream_t st)
{
    if (ntot <= 0) return;
    const int grid = ceil_div(ntot, 256);
    const KickPartials k = kp ? *kp : KickPartials{nullptr, nullptr, 0};
    if (next) {
        const int bs = bbox_stride(next->nc);
        if (beams)
            k_kick_drift<true, true><<<grid, 256, 0, st>>>(cs, ion_crystal, ntot, kstep, E, sum, call_k, next->zr,
                                                           next->bbox, bs, k);
        else
            k_kick_drift<false, true><<<grid, 256, 0, st>>>(cs, ion_crystal, ntot, kstep, E, sum, call_k, next->zr,
                                                            next->bbox, bs, k);
    } else {
        if (beams)
            k_kick_drift<true, false><<<grid, 256, 0, st>>>(cs, ion_crystal, ntot, kstep, E, sum, call_k,
                                                            ZeroRegions{}, nullptr, 0, k);
        else
            k_kick_drift<false, false><<<grid, 256, 0, st>>>(cs, ion_crystal, ntot, kstep, E, sum, call_k,
                                                             ZeroRegions{}, nullptr, 0, k);
    }
}

// The run reset (one thread).
__global__ void k_run_reset(TreeSummary *__restrict__ sum)
{
    sum->halt = 0;
    sum->fail_step = -1;
    sum->refine_overflow = 0;
}


void launch_run_reset(TreeSummary *sum, hipStream_t st) { k_run_reset<<<1, 1, 0, st>>>(sum); }

void launch_direct(const CrystalDev *cs, const DirBlock *tab, int nblk, const int32_t *ion_crystal, int ntot,
                   double *part, double *E, double *phi, hipStream_t st)
{
    if (nblk <= 0 || ntot <= 0) return;
    if (phi) {
        k_direct<true><<<nblk, 64 * kDirWaves, 0, st>>>(cs, tab, part);
        k_direct_finish<true><<<ceil_div(ntot, 256), 256, 0, st>>>(cs, ion_crystal, ntot, part, E, phi);
    } else {
        k_direct<false><<<nblk, 64 * kDirWaves, 0, st>>>(cs, tab, part);
        k_direct_finish<false><<<ceil_div(ntot, 256), 256, 0, st>>>(cs, ion_crystal, ntot, part, E, nullptr);
    }
}

// The ion sums below (potential and rotating-frame energies) go over the
// sum block table: block k takes ions blk_first[k] + t kSumTB + thread
// (t < kSumT) of crystal blk_crystal[k].
constexpr int kSumTB = 256;
constexpr int kSumT = 2;

int sum_ions_per_block() { return kSumTB * kSumT; }

// Potential sums, first level: each block of the sum block table
// (kSumT x kSumTB ions of one crystal) adds its ions' potentials in a fixed
// tree into part[block]; blocks depend only on the crystal's own size, so the
// sums do not depend on the batch.
__global__ __launch_bounds__(kSumTB) void k_phi_partial(const CrystalDev *__restrict__ cs,
                                                        const int32_t *__restrict__ blk_crystal,
                                                        const int32_t *__restrict__ blk_first,
                                                        const double *__restrict__ phi, double *__restrict__ part)
{
    __shared__ double acc[kSumTB];
    const CrystalDev &cd = cs[blk_crystal[blockIdx.x]];
    double a = 0.0;
    for (int t = 0; t < kSumT; ++t) {
        const int i = blk_first[blockIdx.x] + t * kSumTB + threadIdx.x;
        if (i < cd.n) a += phi[cd.ion_off + i];
    }
    acc[threadIdx.x] = a;
    __syncthreads();
    for (int h = kSumTB / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) acc[threadIdx.x] += acc[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// Second level: one wave per crystal c adds the NC-component partial sums of
// its blocks (the contiguous run of blk_crystal == c, found by binary
// search): lane l takes blocks l, l + 64, ... in order, then the lanes'
// sums are added in a fixed tree, so the result depends only on the
// crystal's own blocks.
__device__ inline int first_block(const int32_t *blk_crystal, int nblk, int c)
{
    int lo = 0, hi = nblk;
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (blk_crystal[m] < c) lo = m + 1;
        else hi = m;
    }
    return lo;
}

template <int NC>
__global__ __launch_bounds__(64) void k_blocks_finish(const int32_t *__restrict__ blk_crystal, int nblk,
                                                      const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double acc[NC][64];
    const int c = blockIdx.x, lane = threadIdx.x;
    const int b0 = first_block(blk_crystal, nblk, c), b1 = first_block(blk_crystal, nblk, c + 1);
    double s[NC];
    for (int k = 0; k < NC; ++k) s[k] = 0.0;
    for (int b = b0 + lane; b < b1; b += 64)
        for (int k = 0; k < NC; ++k) s[k] += part[NC * b + k];
    for (int k = 0; k < NC; ++k) acc[k][lane] = s[k];
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
        if (lane < h)
            for (int k = 0; k < NC; ++k) acc[k][lane] += acc[k][lane + h];
        __syncthreads();
    }
    if (lane < NC) out[NC * c + lane] = acc[lane][0];
}

void launch_phi_sum(const CrystalDev *cs, const int32_t *blk_crystal, const int32_t *blk_first, int nblk, int nc,
                    const double *phi, double *part, double *out, hipStream_t st)
{
    if (nc <= 0) return;
    if (nblk > 0) k_phi_partial<<<nblk, kSumTB, 0, st>>>(cs, blk_crystal, blk_first, phi, part);
    k_blocks_finish<1><<<nc, 64, 0, st>>>(blk_crystal, nblk, part, out);
}

// Rotating frame (eq. rotation) at the state's time t = t0 + step dt: the
// position turned about z by omega_r t, the velocity the time derivative of
// the turned position, v_r = R v + omega_r (-y_r, x_r, 0).  (c, s) = cos and
// sin of omega_r t, computed once per crystal by the caller.
__device__ inline void frame_turn(const CrystalDev &cd, double *ts)
{
    const double t = cd.t0 + (double)cd.step0 * cd.dt;
    sincos(cd.omega_r * t, &ts[1], &ts[0]);
}

__device__ inline void to_rotating(const CrystalDev &cd, int i, const double ts[2], double xr[3], double vr[3])
{
    const int n = cd.n;
    const double *s = cd.state;
    const double c = ts[0], sn = ts[1];
    const double x = s[i], y = s[n + i], vx = s[3 * n + i], vy = s[4 * n + i];
    xr[0] = c * x - sn * y;
    xr[1] = sn * x + c * y;
    xr[2] = s[2 * n + i];
    vr[0] = c * vx - sn * vy - cd.omega_r * xr[1];
    vr[1] = sn * vx + c * vy + cd.omega_r * xr[0];
    vr[2] = s[5 * n + i];
}

// Rotating-frame sums, first level: each block of the sum block table
// (kSumT x kSumTB ions of one crystal) adds the axial and planar kinetic
// energies of the rotating-frame velocities and the external terms of eq.
// (pe_rot),
//   m wz^2 z_r^2 / 2 - m (wr^2 - wc wr + wz^2 / 2)(x_r^2 + y_r^2) / 2 + q k_z delta (x_r^2 - y_r^2) / 4
// (m wz^2 = q k_z), in a fixed tree, into part[block][3].  Blocks depend only
// on the crystal's own size, so the sums do not depend on the batch.
__global__ __launch_bounds__(kSumTB) void k_rot_partial(const CrystalDev *__restrict__ cs,
                                                        const int32_t *__restrict__ blk_crystal,
                                                        const int32_t *__restrict__ blk_first,
                                                        double *__restrict__ part)
{
    __shared__ double acc[3][kSumTB];
    __shared__ double ts[2];
    const CrystalDev &cd = cs[blk_crystal[blockIdx.x]];
    if (threadIdx.x == 0) frame_turn(cd, ts);
    __syncthreads();
    const double wr = cd.omega_r, wz2 = cd.qkz / cd.mass;
    const double radial = 0.5 * cd.mass * (wr * wr - cd.wc * wr + 0.5 * wz2);
    double ka = 0.0, kp = 0.0, pe = 0.0;
    for (int t = 0; t < kSumT; ++t) {
        const int i = blk_first[blockIdx.x] + t * kSumTB + threadIdx.x;
        if (i >= cd.n) continue;
        double xr[3], vr[3];
        to_rotating(cd, i, ts, xr, vr);
        ka += 0.5 * cd.mass * vr[2] * vr[2];
        kp += 0.5 * cd.mass * (vr[0] * vr[0] + vr[1] * vr[1]);
        pe += 0.5 * cd.qkz * xr[2] * xr[2] - radial * (xr[0] * xr[0] + xr[1] * xr[1]) +
              0.25 * cd.qkz * cd.delta * (xr[0] * xr[0] - xr[1] * xr[1]);
    }
    acc[0][threadIdx.x] = ka;
    acc[1][threadIdx.x] = kp;
    acc[2][threadIdx.x] = pe;
    __syncthreads();
    for (int h = kSumTB / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 3; ++k) acc[k][threadIdx.x] += acc[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = acc[threadIdx.x][0];
}

// Rotating-frame positions and velocities of every ion, SoA (6 x ntot, batch order).
__global__ void k_rot_state(const CrystalDev *__restrict__ cs, const int32_t *__restrict__ ion_crystal, int ntot,
                            double *__restrict__ out)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ntot) return;
    const CrystalDev &cd = cs[ion_crystal[g]];
    double ts[2], xr[3], vr[3];
    frame_turn(cd, ts);
    to_rotating(cd, g - cd.ion_off, ts, xr, vr);
    for (int k = 0; k < 3; ++k) {
        out[(size_t)k * ntot + g] = xr[k];
        out[(size_t)(3 + k) * ntot + g] = vr[k];
    }
}

void launch_rot_sums(const CrystalDev *cs, const int32_t *blk_crystal, const int32_t *blk_first, int nblk, int nc,
                     double *part, double *out, hipStream_t st)
{
    if (nc <= 0) return;
    if (nblk > 0) k_rot_partial<<<nblk, kSumTB, 0, st>>>(cs, blk_crystal, blk_first, part);
    k_blocks_finish<3><<<nc, 64, 0, st>>>(blk_crystal, nblk, part, out);
}

void launch_rot_state(const CrystalDev *cs, const int32_t *ion_crystal, int ntot, double *out, hipStream_t st)
{
    if (ntot > 0) k_rot_state<<<ceil_div(ntot, 256), 256, 0, st>>>(cs, ion_crystal, ntot, out);
}

}  // namespace pt
