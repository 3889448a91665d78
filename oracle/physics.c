/*
 * Oracle: trap and wall forces, direct Coulomb sum, the cyclotronic
 * integrator, Philox4x32-10 and the Poisson photon-recoil kicks.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain FP64 loops; OpenMP only
 * splits independent per-ion loops, never a reduction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* ---------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the
 * published multipliers, the key bumped by the published Weyl constants
 * between rounds.  The paper under test only asks for Poisson-distributed
 * photon counts and random unit vectors (Sec. 2.2); the counter-based
 * generator makes the draws a pure function of (seed, ion, step, slot).
 * ------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        if (round < 9) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A double in [0,1) from 53 bits of two words: 27 high bits of w0, 26 of w1. */
static double or_u53(uint32_t w0, uint32_t w1)
{
    double hi = (double)(w0 >> 5);
    double lo = (double)(w1 >> 6);
    return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0);
}

static void or_draw(uint64_t seed, uint32_t ion, uint64_t step, uint32_t slot, uint32_t w[4])
{
    uint32_t ctr[4] = {ion, (uint32_t)step, (uint32_t)(step >> 32), slot};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, w);
}

/* Cumulative Poisson table F_0..F_16 for mean lam, accumulated term by term:
 * p_0 = exp(-lam), p_k = p_{k-1} lam / k, F_k = F_{k-1} + p_k. */
void or_poisson_cdf(double lam, double F[17])
{
    double pk = exp(-lam);
    double acc = pk;
    F[0] = acc;
    for (int k = 1; k <= 16; ++k) {
        pk = pk * lam / (double)k;
        acc = acc + pk;
        F[k] = acc;
    }
}

/* Photon count by inversion: the smallest k with u < F_k, capped at 16. */
static int or_poisson_count(double u, const double F[17])
{
    for (int k = 0; k <= 16; ++k)
        if (u < F[k]) return k;
    return 16;
}

/* Photon counts for every ion at one step (slot 0 of each ion's stream). */
void or_photon_counts(int n, uint64_t seed, uint64_t step, double mean, int32_t *counts)
{
    double F[17];
    or_poisson_cdf(mean, F);
    for (int i = 0; i < n; ++i) {
        uint32_t w[4];
        or_draw(seed, (uint32_t)i, step, 0u, w);
        counts[i] = or_poisson_count(or_u53(w[0], w[1]), F);
    }
}

/* Sum of n isotropic unit vectors of ion `ion` at `step`, slots 1..n
 * (cos(theta) uniform in [-1,1], azimuth uniform in [0, 2 pi)). */
static void or_recoil_dirs(uint64_t seed, uint32_t ion, uint64_t step, int n, double acc[3])
{
    acc[0] = acc[1] = acc[2] = 0.0;
    for (int j = 1; j <= n; ++j) {
        uint32_t w[4];
        or_draw(seed, ion, step, (uint32_t)j, w);
        double ct = 2.0 * or_u53(w[0], w[1]) - 1.0;
        double ph = 2.0 * OR_PI * or_u53(w[2], w[3]);
        double st = sqrt(1.0 - ct * ct);
        acc[0] += st * cos(ph);
        acc[1] += st * sin(ph);
        acc[2] += ct;
    }
}

/* ---------------------------------------------------------------------
 * External forces (Sec. 2.1).  phi_trap = k_z (2z^2 - x^2 - y^2)/4 with
 * k_z = m omega_z^2 / q; the force on charge q is -q grad(phi).
 * phi_wall = k_z delta (x^2 + y^2) cos(2(varphi + omega_r t)) / 4, and
 * r^2 cos(2 varphi + 2 omega_r t) = (x^2 - y^2) C - 2 x y S with
 * C = cos(2 omega_r t), S = sin(2 omega_r t).
 * ------------------------------------------------------------------- */
void or_external_force(double q, double m, const or_trap *tr, double t, const double x[3], double F[3])
{
    double kz = m * tr->omega_z * tr->omega_z / q;
    double C = cos(2.0 * tr->omega_r * t);
    double S = sin(2.0 * tr->omega_r * t);
    /* -q d/dx of the trap term, then of the wall term */
    F[0] = 0.5 * q * kz * x[0] - 0.5 * q * kz * tr->delta * (x[0] * C - x[1] * S);
    F[1] = 0.5 * q * kz * x[1] + 0.5 * q * kz * tr->delta * (x[1] * C + x[0] * S);
    F[2] = -q * kz * x[2];
}

/* Coulomb force by the direct pairwise sum: the gradient of the pair term of
 * eq. (hamiltonian); the 1/(8 pi eps0) there counts each pair twice, so the
 * force on i is k_e q^2 sum_{j != i} (x_i - x_j)/|x_i - x_j|^3.  A pair at
 * zero separation contributes nothing.  pos, F: n x 3 row-major. */
void or_coulomb_direct(int n, const double *pos, double q, double *F)
{
    double ke = 1.0 / (4.0 * OR_PI * OR_EPS0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = pos[3 * i] - pos[3 * j];
            double dy = pos[3 * i + 1] - pos[3 * j + 1];
            double dz = pos[3 * i + 2] - pos[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            double w = 1.0 / (r2 * r);
            fx += dx * w;
            fy += dy * w;
            fz += dz * w;
        }
        F[3 * i] = ke * q * q * fx;
        F[3 * i + 1] = ke * q * q * fy;
        F[3 * i + 2] = ke * q * q * fz;
    }
}

/* Direct Coulomb sum for a subset of target ions (used for sampled checks
 * at sizes where the full sum is too slow). */
void or_coulomb_direct_sampled(int n, const double *pos, double q, int ns, const int32_t *idx, double *F)
{
    double ke = 1.0 / (4.0 * OR_PI * OR_EPS0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a < ns; ++a) {
        int i = idx[a];
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = pos[3 * i] - pos[3 * j];
            double dy = pos[3 * i + 1] - pos[3 * j + 1];
            double dz = pos[3 * i + 2] - pos[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            double w = 1.0 / (r2 * r);
            fx += dx * w;
            fy += dy * w;
            fz += dz * w;
        }
        F[3 * a] = ke * q * q * fx;
        F[3 * a + 1] = ke * q * q * fy;
        F[3 * a + 2] = ke * q * q * fz;
    }
}

/* Coulomb potential at each ion, phi_i = k_e q sum_{j != i} 1/r_ij (volts):
 * the pair term of eq. (hamiltonian) per unit charge, the phi^dir of
 * eq. (rms_pot).  Pairs at zero separation are left out. */
void or_coulomb_potential_direct(int n, const double *pos, double q, double *phi)
{
    double ke = 1.0 / (4.0 * OR_PI * OR_EPS0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = pos[3 * i] - pos[3 * j];
            double dy = pos[3 * i + 1] - pos[3 * j + 1];
            double dz = pos[3 * i + 2] - pos[3 * j + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r > 0.0) s += 1.0 / r;
        }
        phi[i] = ke * q * s;
    }
}

/* The same for the ions listed in idx only (phi: ns values). */
void or_coulomb_potential_direct_sampled(int n, const double *pos, double q, int ns, const int32_t *idx, double *phi)
{
    double ke = 1.0 / (4.0 * OR_PI * OR_EPS0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a < ns; ++a) {
        int i = idx[a];
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = pos[3 * i] - pos[3 * j];
            double dy = pos[3 * i + 1] - pos[3 * j + 1];
            double dz = pos[3 * i + 2] - pos[3 * j + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r > 0.0) s += 1.0 / r;
        }
        phi[a] = ke * q * s;
    }
}

/* Coulomb potential energy (1/2) sum_i q phi_coul(x_i) = k_e q^2 sum_{i<j} 1/r_ij. */
double or_coulomb_energy(int n, const double *pos, double q)
{
    double ke = 1.0 / (4.0 * OR_PI * OR_EPS0);
    double e = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double dx = pos[3 * i] - pos[3 * j];
            double dy = pos[3 * i + 1] - pos[3 * j + 1];
            double dz = pos[3 * i + 2] - pos[3 * j + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r > 0.0) e += 1.0 / r;
        }
    return ke * q * q * e;
}

/* Lab-frame energy of eq. (hamiltonian) with delta = 0: kinetic energy
 * (p - qA)^2/2m = m v^2/2, trap energy q phi_trap, Coulomb pair energy. */
double or_energy(int n, const double *pos, const double *vel, double q, double m, const or_trap *tr)
{
    double kz = m * tr->omega_z * tr->omega_z / q;
    double ek = 0.0, et = 0.0;
    for (int i = 0; i < n; ++i) {
        const double *x = pos + 3 * i, *v = vel + 3 * i;
        ek += 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        et += q * 0.25 * kz * (2.0 * x[2] * x[2] - x[0] * x[0] - x[1] * x[1]);
    }
    return ek + et + or_coulomb_energy(n, pos, q);
}

/* ---------------------------------------------------------------------
 * Rotating frame, eq. (rotation): positions turned about z by the angle
 * omega_r t, (x_r, y_r) = (x cos - y sin, x sin + y cos); velocities are the
 * time derivatives of the rotated positions, v_r = R v + omega_r (-y_r, x_r, 0).
 * A crystal turning clockwise (seen from +z) at omega_r -- the sense of the
 * rotating wall cos(2(varphi + omega_r t)) -- is at rest in this frame.
 * ------------------------------------------------------------------- */
void or_rotating_frame(int n, const double *pos, const double *vel, double omega_r, double t, double *pos_r,
                       double *vel_r)
{
    double c = cos(omega_r * t), s = sin(omega_r * t);
    for (int i = 0; i < n; ++i) {
        const double *x = pos + 3 * i, *v = vel + 3 * i;
        double xr = c * x[0] - s * x[1], yr = s * x[0] + c * x[1];
        pos_r[3 * i] = xr;
        pos_r[3 * i + 1] = yr;
        pos_r[3 * i + 2] = x[2];
        vel_r[3 * i] = c * v[0] - s * v[1] - omega_r * yr;
        vel_r[3 * i + 1] = s * v[0] + c * v[1] + omega_r * xr;
        vel_r[3 * i + 2] = v[2];
    }
}

/* Rotating-frame energy at time t, eq. (pe_rot) (its first line, which follows
 * from eqs. pot_trap and pot_wall; see below) plus the kinetic energy of the
 * rotating-frame velocities:
 *   out[0] = sum m vz_r^2 / 2                                  axial kinetic
 *   out[1] = sum m (vx_r^2 + vy_r^2) / 2                        planar kinetic
 *   out[2] = sum [ m wz^2 z_r^2 / 2 - m (wr^2 - wc wr + wz^2/2)(x_r^2 + y_r^2) / 2
 *                  + q k_z delta (x_r^2 - y_r^2) / 4 ]           external terms
 *   out[3] = k_e q^2 sum_{i<j} 1/r_ij                           Coulomb
 *   out[4] = the total.
 * With k_z = m wz^2 / q and wc = q B / m.  The printed C_x, C_y form of the
 * same equation carries the wall term as -m wz^2 delta (x_r^2 - y_r^2)/2, a
 * factor -2 away; the rotating wall of eq. (pot_wall) seen in this frame is
 * q k_z delta (x_r^2 - y_r^2) / 4, the term used here. */
void or_rotating_energy(int n, const double *pos, const double *vel, double q, double m, const or_trap *tr, double t,
                        double out[5])
{
    double wz = tr->omega_z, wr = tr->omega_r, wc = q * tr->B / m;
    double kz = m * wz * wz / q;
    double *xr = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *vr = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    or_rotating_frame(n, pos, vel, wr, t, xr, vr);
    double ka = 0.0, kp = 0.0, pe = 0.0;
    for (int i = 0; i < n; ++i) {
        const double *x = xr + 3 * i, *v = vr + 3 * i;
        double rho2 = x[0] * x[0] + x[1] * x[1];
        ka += 0.5 * m * v[2] * v[2];
        kp += 0.5 * m * (v[0] * v[0] + v[1] * v[1]);
        pe += 0.5 * m * wz * wz * x[2] * x[2] - 0.5 * m * (wr * wr - wc * wr + 0.5 * wz * wz) * rho2 +
              0.25 * q * kz * tr->delta * (x[0] * x[0] - x[1] * x[1]);
    }
    out[0] = ka;
    out[1] = kp;
    out[2] = pe;
    out[3] = or_coulomb_energy(n, xr, q);
    out[4] = ka + kp + pe + out[3];
    free(xr);
    free(vr);
}

/* ---------------------------------------------------------------------
 * U0(tau), eq. (U0): exact motion of a charge in the uniform field B z-hat
 * with no electric field.  m dv/dt = q v x B gives dvx/dt = wc vy,
 * dvy/dt = -wc vx (wc = qB/m), i.e. clockwise gyration for q B > 0; the
 * printed matrix has the opposite rotation sense and a zero (6,6) entry,
 * read here as the Lorentz solution with v_z conserved.  z drifts freely.
 * ------------------------------------------------------------------- */
void or_u0(int n, double *pos, double *vel, double wc, double tau)
{
    for (int i = 0; i < n; ++i) {
        double *x = pos + 3 * i, *v = vel + 3 * i;
        double vx = v[0], vy = v[1];
        if (wc == 0.0) {
            x[0] += vx * tau;
            x[1] += vy * tau;
        } else {
            double c = cos(wc * tau), s = sin(wc * tau);
            x[0] += (vx * s + vy * (1.0 - c)) / wc;
            x[1] += (vx * (c - 1.0) + vy * s) / wc;
            v[0] = vx * c + vy * s;
            v[1] = -vx * s + vy * c;
        }
        x[2] += v[2] * tau;
    }
}

/* ---------------------------------------------------------------------
 * Beam mode, eq. (scattering_rate): the photon absorption rate of an ion at
 * x with velocity v from beam l,
 *   gamma = S gamma0 (gamma0/2)^2 / ((gamma0/2)^2 (1 + 2 S) + (Delta - k.v)^2),
 * with k = (2 pi / lambda) khat and the saturation S of the beam's profile.
 * ------------------------------------------------------------------- */
static void or_unit(const double a[3], double u[3])
{
    double r = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    u[0] = a[0] / r;
    u[1] = a[1] / r;
    u[2] = a[2] / r;
}

double or_scattering_rate(const or_laser *la, int l, const double x[3], const double v[3])
{
    const or_beam *b = &la->beam[l];
    double kh[3];
    or_unit(b->khat, kh);
    double S = b->s0;
    if (!b->uniform) {
        double dy = x[1] - b->offset_y, z = x[2];
        S = b->s0 * exp(-(dy * dy / (b->waist_y * b->waist_y) + z * z / (b->waist_z * b->waist_z)));
    }
    double k = 2.0 * OR_PI / la->wavelength;
    double kv = k * (kh[0] * v[0] + kh[1] * v[1] + kh[2] * v[2]);
    double dd = b->detuning - kv;
    double g2 = 0.25 * la->gamma0 * la->gamma0;
    return S * la->gamma0 * g2 / (g2 * (1.0 + 2.0 * S) + dd * dd);
}

/* Velocity change of eq. (laser_kick) for ion `ion` at `step` in beam mode:
 * per beam a Poisson count n_l with mean gamma_l dt (slot l << 16), then
 * n_l absorptions along khat_l and n_l isotropic emissions (slots
 * (l << 16) | j), each of momentum h / lambda.  Returns the total count. */
static int or_beam_kick(const or_laser *la, uint64_t seed, uint32_t ion, uint64_t step, double m, double dt,
                        const double x[3], const double v[3], double dv[3])
{
    double rec = OR_H_PLANCK / (la->wavelength * m);
    int total = 0;
    dv[0] = dv[1] = dv[2] = 0.0;
    for (int l = 0; l < la->n_beams; ++l) {
        double F[17], kh[3];
        or_poisson_cdf(or_scattering_rate(la, l, x, v) * dt, F);
        uint32_t w[4];
        or_draw(seed, ion, step, (uint32_t)l << 16, w);
        int cnt = or_poisson_count(or_u53(w[0], w[1]), F);
        double e[3] = {0.0, 0.0, 0.0};
        for (int j = 1; j <= cnt; ++j) {
            or_draw(seed, ion, step, ((uint32_t)l << 16) | (uint32_t)j, w);
            double ct = 2.0 * or_u53(w[0], w[1]) - 1.0;
            double ph = 2.0 * OR_PI * or_u53(w[2], w[3]);
            double st = sqrt(1.0 - ct * ct);
            e[0] += st * cos(ph);
            e[1] += st * sin(ph);
            e[2] += ct;
        }
        or_unit(la->beam[l].khat, kh);
        for (int d = 0; d < 3; ++d) dv[d] += rec * ((double)cnt * kh[d] + e[d]);
        total += cnt;
    }
    return total;
}

/* Artificial damping (the outlook of the paper's conclusion: momenta slowly
 * decreased while the crystal evolves): the velocity relative to the frame of
 * eq. (rotation) -- v minus the clockwise rigid rotation omega_r (y, -x, 0),
 * the motion at rest in that frame -- is multiplied by exp(-damping dt / 2),
 * once before and once after the kick, so that the split step stays
 * symmetric and the damped fixed point sits within O(dt^2) of the rotating
 * frame's equilibrium. */
static void or_damp_half(const or_trap *tr, double dt, const double x[3], double v[3])
{
    double f = exp(-0.5 * tr->damping * dt);
    double rig[3] = {tr->omega_r * x[1], -tr->omega_r * x[0], 0.0};
    for (int d = 0; d < 3; ++d) v[d] = rig[d] + f * (v[d] - rig[d]);
}

/* Coulomb force by the FMM (fmm.c). */
int or_fmm_coulomb(int n, const double *pos, double q, int p, int leaf_size, double *F);

/* One full step per eqs. (time_ev2) and (velocity_kick): U0(dt/2), kick with
 * trap + wall + Coulomb forces at the midpoint time t + dt/2 plus photon
 * recoils, U0(dt/2).  The step index `step` keys the photon streams and the
 * time is t = t0 + step dt.  photons (nullable) receives the counts. */
int or_step(int n, double *pos, double *vel, double q, double m, const or_trap *tr, const or_laser *la,
            const or_force *fo, double t0, double dt, uint64_t seed, uint64_t step, int32_t *photons)
{
    double wc = q * tr->B / m;
    double t = t0 + (double)step * dt;
    double tm = t + 0.5 * dt;
    double *Fc = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!Fc) return -2;
    or_u0(n, pos, vel, wc, 0.5 * dt);
    if (fo->method == 0) {
        or_coulomb_direct(n, pos, q, Fc);
    } else {
        int rc = or_fmm_coulomb(n, pos, q, fo->p, fo->leaf_size, Fc);
        if (rc) { free(Fc); return rc; }
    }
    double F[17];
    int beams = la && la->mode == 2 && la->n_beams > 0;
    int laser_on = la && !beams && la->mode != 2 && la->mean_per_step > 0.0;
    if (laser_on) or_poisson_cdf(la->mean_per_step, F);
    double recoil = laser_on ? OR_H_PLANCK / (la->wavelength * m) : 0.0;
    for (int i = 0; i < n; ++i) {
        if (tr->damping > 0.0) or_damp_half(tr, dt, pos + 3 * i, vel + 3 * i);
        double fe[3], vmid[3] = {vel[3 * i], vel[3 * i + 1], vel[3 * i + 2]};
        or_external_force(q, m, tr, tm, pos + 3 * i, fe);
        for (int d = 0; d < 3; ++d) vel[3 * i + d] += (fe[d] + Fc[3 * i + d]) * dt / m;
        int cnt = 0;
        if (beams) {
            /* rates at the midpoint state: positions after the first half
             * drift, velocities before the kick */
            double dv[3];
            cnt = or_beam_kick(la, seed, (uint32_t)i, step, m, dt, pos + 3 * i, vmid, dv);
            for (int d = 0; d < 3; ++d) vel[3 * i + d] += dv[d];
        } else if (laser_on) {
            uint32_t w[4];
            or_draw(seed, (uint32_t)i, step, 0u, w);
            cnt = or_poisson_count(or_u53(w[0], w[1]), F);
            double acc[3];
            or_recoil_dirs(seed, (uint32_t)i, step, cnt, acc);
            for (int d = 0; d < 3; ++d) vel[3 * i + d] += recoil * acc[d];
        }
        if (photons) photons[i] = cnt;
        if (tr->damping > 0.0) or_damp_half(tr, dt, pos + 3 * i, vel + 3 * i);
    }
    or_u0(n, pos, vel, wc, 0.5 * dt);
    free(Fc);
    return 0;
}

/* nsteps consecutive steps starting at step index step0. */
int or_run(int n, double *pos, double *vel, double q, double m, const or_trap *tr, const or_laser *la,
           const or_force *fo, double t0, double dt, uint64_t seed, uint64_t step0, int nsteps, int32_t *photons)
{
    for (int s = 0; s < nsteps; ++s) {
        int rc = or_step(n, pos, vel, q, m, tr, la, fo, t0, dt, seed, step0 + (uint64_t)s, photons);
        if (rc) return rc;
    }
    return 0;
}
