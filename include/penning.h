/*
 * penning.h -- C ABI of the MI355X (gfx950) Penning-trap ion-crystal library.
 *
 * The library advances N ions of one species (charge q, mass m) in a Penning
 * trap: a uniform field B z-hat, the harmonic trap potential
 * phi_trap = k_z (2z^2 - x^2 - y^2)/4 with k_z = m omega_z^2 / q, and the
 * rotating-wall potential phi_wall = k_z delta (x^2+y^2) cos(2(varphi + omega_r t))/4
 * (Zaris et al., arXiv 2405.13973, Sec. 2.1, eqs. pot_trap, pot_wall,
 * hamiltonian), with Coulomb interactions between all ions.  Time stepping is
 * the split operator U(t, dt) = U0(dt/2) Ukick(t + dt/2; dt) U0(dt/2) of
 * Sec. 2.2 (eqs. time_ev2, U0, velocity_kick), U0 being the exact gyration in
 * B.  Coulomb forces come from a direct O(N^2) sum or from a 3D Laplace fast
 * multipole method (Sec. 2.3); photon recoils are Poisson-distributed kicks
 * (eq. laser_kick), at a fixed mean or from laser beams (eq. scattering_rate).
 *
 * Conventions
 *   - SI units.  Positions in m, velocities in m/s, forces in N, time in s.
 *   - Host arrays are n x 3, row-major (x0 y0 z0 x1 y1 z1 ...), in ion-id
 *     (creation) order; every output is in ion-id order.
 *   - The caller owns every buffer it passes; create copies the state into
 *     device memory owned by the library until pt_destroy_crystal.
 *   - Every call returns a pt_status; on failure pt_last_error() gives a
 *     message (thread-local, valid until the next failing call on the thread).
 *     No call throws across the ABI.  Calls on one context are not
 *     thread-safe: serialise them.
 *   - Work is queued on the context's HIP stream.  pt_step and
 *     pt_step_batch return once their work is queued (with the FMM, only the
 *     first step of a new batch waits, twice, to measure its tree);
 *     pt_read_state, pt_compute_forces and pt_synchronize wait for
 *     completion.
 */
#ifndef PENNING_H
#define PENNING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PT_OK = 0,
    PT_EINVAL = -1,    /* invalid argument (NULL, size, non-finite value, unconfined trap, ...) */
    PT_ENOMEM = -2,    /* the context's HBM budget or the device ran out of memory */
    PT_EDEVICE = -3,   /* a HIP runtime call failed */
    PT_ENUMERIC = -4,  /* non-finite state detected after a step */
    PT_EBUSY = -5      /* object still in use (e.g. destroying a context that owns crystals) */
} pt_status;

typedef struct pt_ctx pt_ctx;
typedef struct pt_crystal pt_crystal;

/* Trap parameters (Sec. 2.1).  omega_z and omega_r in rad/s.  dt_s is the
 * step length and t0_s the time of step 0: step k runs from t0 + k dt to
 * t0 + (k+1) dt.  Requires dt > 0 and radial confinement of a single ion,
 * omega_c^2 > 2 omega_z^2 with omega_c = qB/m (else PT_EINVAL).
 * damping_per_s >= 0 (0 = off): artificial damping, the paper's proposal for
 * finding crystal equilibria -- each step multiplies the velocity relative to
 * the frame turning at omega_r (eq. rotation), v - omega_r (y, -x, 0), by
 * exp(-damping dt / 2) just before and again just after the kick, so the
 * crystal relaxes to a minimum of the rotating-frame potential energy
 * (eq. pe_rot); the split keeps the damped fixed point within O(dt^2) of it.
 * Modes without kinetic energy relax slowly (E x B modes when omega_r is far
 * from omega_c / 2, where B - 2 m omega_r / q vanishes). */
typedef struct {
    double B_T;
    double omega_z;
    double delta;
    double omega_r;
    double dt_s;
    double t0_s;
    double damping_per_s;
} pt_trap_params;

/* One laser beam of eq. (scattering_rate).  khat: propagation direction
 * (any non-zero length; normalised by the library).  detuning: Delta_l in
 * rad/s.  s0 >= 0: peak saturation parameter.  uniform = 1: the saturation
 * is s0 everywhere (a beam much wider than the crystal); uniform = 0: the 2D
 * Gaussian profile of the paper's cooling appendix in lab coordinates,
 * S = s0 exp(-(y - offset_y)^2 / waist_y^2 - z^2 / waist_z^2) (waists > 0, m),
 * which describes beams propagating along +-x such as the planar beam. */
typedef struct {
    double khat[3];
    double detuning;
    double s0;
    double waist_y, waist_z;
    double offset_y;
    int uniform;
} pt_beam;

#define PT_MAX_BEAMS 4

/* Photon model (Sec. 2.2, eqs. scattering_rate and laser_kick).  Draws come
 * from Philox4x32-10 keyed by the crystal seed, counter (ion id, step,
 * slot); a count is the inversion of the Poisson CDF (capped at 16) at the
 * uniform of its slot.
 *   mode 0: off.
 *   mode 1: every ion scatters a Poisson number of photons per step with
 *     mean mean_per_step (0 <= mean <= 2), each an emission recoil
 *     h/(wavelength m) in a uniformly random direction; slot 0 decides the
 *     count, slot j >= 1 the j-th direction.
 *   mode 2: n_beams (1..PT_MAX_BEAMS) beams with natural linewidth gamma0
 *     (rad/s).  Per ion, beam l and step, the count has mean gamma_l dt with
 *     the rate of eq. (scattering_rate) at the midpoint position and the
 *     velocity before the kick, k_l = (2 pi / wavelength) khat_l; each photon
 *     adds h/(wavelength m) along khat_l (absorption) and the same in a
 *     uniformly random direction (emission).  Slot (l << 16) decides beam l's
 *     count, slot (l << 16) | j its j-th emission.  Requires gamma0 dt <= 4, so
 *     that no mean exceeds 2 (the largest rate is gamma0 / 2).
 * PT_EINVAL for other modes or non-finite / out-of-range values. */
typedef struct {
    int mode;
    double mean_per_step;
    double wavelength_m;
    double gamma0;
    int n_beams;
    pt_beam beam[PT_MAX_BEAMS];
} pt_laser_params;

/* Coulomb solver.  method 0: direct pairwise sum (FP64).  method 1: FMM with
 * maximum expansion degree p (1 <= p <= 20) and leaf size leaf_size (a box
 * is divided while it holds more than leaf_size ions, down to level 16).
 * precision 0: FP64 throughout.  precision 1: mixed -- FP32 expansions,
 * FP32 matrix-core M2L, FP32 near field with compensated sums (separations
 * from 31-bit fixed-point offsets in each leaf's near frame, exact to a
 * quantum of about 1e-9 of the leaf side); positions, box-centre offsets and
 * the integrator stay FP64. */
typedef struct {
    int method;
    int p;
    int leaf_size;
    int precision;
} pt_force_params;

/* Context: one HIP device and stream.  hbm_budget_bytes caps the device
 * memory the context allocates (0 = no cap).  hip_stream is a hipStream_t
 * (for example torch.cuda.current_stream().cuda_stream) or NULL for a
 * stream the context creates.  The stream must outlive the context. */
pt_status pt_ctx_create(int hip_device, uint64_t hbm_budget_bytes, void *hip_stream, pt_ctx **out);
/* PT_EBUSY while crystals created on it still exist. */
pt_status pt_ctx_destroy(pt_ctx *ctx);
/* Device bytes currently allocated by the context. */
pt_status pt_ctx_memory(pt_ctx *ctx, uint64_t *bytes_in_use, uint64_t *budget);

/* Crystal of n >= 1 ions with positions pos_xyz and velocities vel_xyz
 * (host, n x 3).  Default parameters: B = 4.5 T, omega_z = 2 pi 1.5 MHz,
 * delta = omega_r = 0, dt = 1 ns, t0 = 0, laser off, direct method.  Step
 * counter starts at 0.  PT_ENOMEM if the context budget would be exceeded. */
pt_status pt_create_crystal(pt_ctx *ctx, int64_t n, const double *pos_xyz, const double *vel_xyz, double charge_C,
                            double mass_kg, uint64_t seed, pt_crystal **out);
/* Same, from device buffers (n x 3, FP64, e.g. torch tensors' data_ptr()),
 * read on the context stream. */
pt_status pt_create_crystal_device(pt_ctx *ctx, int64_t n, const double *pos_xyz_dev, const double *vel_xyz_dev,
                                   double charge_C, double mass_kg, uint64_t seed, pt_crystal **out);
pt_status pt_destroy_crystal(pt_crystal *c);

pt_status pt_set_trap_params(pt_crystal *c, const pt_trap_params *p);
pt_status pt_set_laser_params(pt_crystal *c, const pt_laser_params *p);
pt_status pt_set_force_params(pt_crystal *c, const pt_force_params *p);
/* Overwrite the state (host, n x 3) and the step counter. */
pt_status pt_set_state(pt_crystal *c, const double *pos_xyz, const double *vel_xyz, int64_t step);

/* Coulomb force k_e q^2 sum_{j != i} (x_i - x_j)/|x_i - x_j|^3 on every ion
 * at the current positions, with the crystal's force parameters (host
 * output, n x 3, ion-id order).  Trap and wall forces are not included. */
pt_status pt_compute_forces(pt_crystal *c, double *F_out);
/* Same for several crystals evaluated together in one batch (each crystal's
 * result identical to its own pt_compute_forces); F_out[k] is crystal k's
 * host output.  All crystals must share the context and force parameters. */
pt_status pt_compute_forces_batch(pt_crystal *const *cs, int n_crystals, double *const *F_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the Coulomb
 * force of pt_compute_forces by the direct sum, written to a DEVICE buffer
 * F_dev (n x 3 doubles, ion-id order, owned by the caller), queued on the
 * context's stream and not waited for (pt_synchronize waits).  The result is
 * bit-identical to pt_compute_forces with the direct method.  Its work
 * buffers live in one fixed per-GPU device array of 24 MiB, set up when the
 * context is created; the call itself allocates nothing.  Limits: the
 * crystal's force method must be the direct sum and n <= PT_NOALLOC_MAX_IONS
 * (else PT_EINVAL).  Every such call on one GPU shares that array, and the
 * array keeps the last call's contents: calls that overlap on one GPU (e.g.
 * from two contexts on different streams) race and must be serialised by the
 * caller.  Errors: PT_EINVAL, PT_EDEVICE. */
#define PT_NOALLOC_MAX_IONS 131072
pt_status pt_compute_forces_noalloc(pt_crystal *c, double *F_dev);

/* Coulomb potential phi_i = k_e q sum_{j != i} 1/|x_i - x_j| (volts) at every
 * ion at the current positions -- the pair term of eq. (hamiltonian) per unit
 * charge, the quantity the paper's potential error (eq. rms_pot) compares --
 * by the crystal's force method: the direct sum, or the FMM with the local
 * expansion's value (eq. FMM_local) plus the near field.  Host output, n
 * doubles, ion-id order; pairs at zero separation are left out.  Trap and
 * wall potentials are not included.  Batch form as pt_compute_forces_batch.
 * Errors: PT_EINVAL (NULL arguments, batch rules), PT_ENOMEM, PT_EDEVICE. */
pt_status pt_compute_potential(pt_crystal *c, double *phi_out);
pt_status pt_compute_potential_batch(pt_crystal *const *cs, int n_crystals, double *const *phi_out);
/* Coulomb energy U = (1/2) q sum_i phi_i (joules) at the current positions
 * (the pair part of eq. hamiltonian), with phi as pt_compute_potential; the
 * sum over ions runs on the device in a fixed order (FP64), so only one
 * double per crystal crosses to the host.  U_out: n_crystals doubles. */
pt_status pt_coulomb_energy(pt_crystal *c, double *U_out);
pt_status pt_coulomb_energy_batch(pt_crystal *const *cs, int n_crystals, double *U_out);

/* Rotating-frame diagnostics (eqs. rotation, pe_rot, temp_ax, temp_pl) of the
 * current state at its time t = t0 + step dt.  The frame turns about z by
 * omega_r t (a crystal turning clockwise at omega_r, the sense of the rotating
 * wall, is at rest in it); velocities are the time derivatives of the turned
 * positions.  Energies in J, temperatures in K:
 *   ke_axial = sum m vz_r^2 / 2, ke_planar = sum m (vx_r^2 + vy_r^2) / 2,
 *   pe_external = sum [m wz^2 z_r^2 / 2 - m (wr^2 - wc wr + wz^2/2)(x_r^2 + y_r^2) / 2
 *                      + q k_z delta (x_r^2 - y_r^2) / 4]   (wc = qB/m, k_z = m wz^2 / q),
 *   pe_coulomb = (1/2) q sum phi_i by the crystal's force method (pt_coulomb_energy),
 *   energy = the sum of the four: the rotating-frame energy that eq. (rms_en)
 *     compares, conserved by the dynamics also with the rotating wall on,
 *   temp_axial = m sum vz_r^2 / (N k_b), temp_planar = m sum (vx_r^2 + vy_r^2) / (2 N k_b):
 *     the instantaneous terms of eqs. (temp_ax) and (temp_pl), whose time averages
 *     those equations take; eq. (temp_pe) is (2/3)(pe_external + pe_coulomb - PE_0)/(N k_b)
 *     for a reference configuration's energy PE_0 computed the same way.
 * The sums over ions run on the device in a fixed order (FP64).  The wall
 * term follows eq. (pot_wall) seen in the rotating frame (the printed C_x,
 * C_y form of eq. pe_rot carries a different factor). */
typedef struct {
    double t;
    double ke_axial;
    double ke_planar;
    double pe_external;
    double pe_coulomb;
    double energy;
    double temp_axial;
    double temp_planar;
} pt_diagnostics;
pt_status pt_rotating_diagnostics(pt_crystal *c, pt_diagnostics *out);
pt_status pt_rotating_diagnostics_batch(pt_crystal *const *cs, int n_crystals, pt_diagnostics *out);
/* Positions and velocities of the current state in the rotating frame (host,
 * n x 3 each, ion-id order; either may be NULL). */
pt_status pt_read_rotating_state(pt_crystal *c, double *pos_r, double *vel_r);

/* Advance n_steps >= 0 steps (eq. time_ev2 with eq. velocity_kick). */
pt_status pt_step(pt_crystal *c, int64_t n_steps);
/* Advance crystal k by n_steps[k] steps; crystals still stepping are
 * batched together so that each phase of a step is one launch for all of
 * them.  Results are identical to stepping each crystal alone.
 * With the FMM, the first step of a batch measures its tree and lists (two
 * host waits) and sizes the work buffers for them with room to grow; the
 * following steps are queued with no host wait, the kernels reading every
 * count on the device.  If a step's tree or lists outgrow that room, the
 * device stops the run before that step's kick (state and photon counts stay
 * at the last completed step), and the context's next call (any call, e.g.
 * pt_synchronize or pt_read_state) reads this back and runs the remaining
 * steps again from there, measuring first: results do not depend on it.
 * Errors: PT_EINVAL (NULL, negative counts, batch rules), PT_ENOMEM and
 * PT_EDEVICE (the crystals then stand at their last completed step, which
 * pt_read_state reports). */
pt_status pt_step_batch(pt_crystal *const *cs, int n_crystals, const int64_t *n_steps);
pt_status pt_synchronize(pt_ctx *ctx);

/* Copy out the state (host, n x 3; pos/vel/step/t/photons may be NULL).
 * photons receives each ion's photon count of the last step taken. */
pt_status pt_read_state(pt_crystal *c, double *pos, double *vel, int64_t *step, double *t, int32_t *photons);

/* Octree and interaction lists of the last FMM evaluation of crystal c.
 * sizes[0..3] = boxes, levels, V entries, near entries.  With the array
 * arguments NULL only sizes is filled.  Boxes are in (level, Morton prefix)
 * order; keys (n, 48-bit Morton) and perm (n, ion ids in (key, id) order)
 * follow ion id / sorted order; coords n_box x 3 integer box coordinates at
 * the box's level; v_off/v_src and near_off/near_src are CSR lists with
 * sources in ascending box order; root = lower corner xyz and side. */
pt_status pt_debug_export_tree(pt_crystal *c, int64_t sizes[4], uint64_t *keys, int32_t *perm, int32_t *level,
                               int32_t *parent, int32_t *ion_begin, int32_t *ion_end, int32_t *coords,
                               uint8_t *is_leaf, int32_t *v_off, int32_t *v_src, int32_t *near_off,
                               int32_t *near_src, double *root);

/* Per-phase GPU time of force evaluations, measured with HIP events:
 * ms[0] sort+tree+lists (P2M runs on a second stream of the context
 * beside the lists), [1] M2M with the M2L bucketing and the near-field work
 * items, [2] the M2L matrix-core kernel,
 * [3] M2L reduction + L2L, [4] the P2P kernel (it runs on a second stream
 * of the context, concurrently with [1]-[3]), [5] waiting for the P2P
 * kernel plus L2P and the near-field partial sums, [6] total (the direct
 * method has all its time in [0]) -- each the mean over the evaluations
 * since timing was last switched on (count receives their number; may be
 * NULL).
 * pt_ctx_set_timing(ctx, n) with n >= 1 starts a new measurement that
 * records the events of every n-th evaluation (each recorded event is a
 * packet in the stream, so a sparse n perturbs the timed steps less); 0 stops
 * it; PT_EINVAL for n < 0.  The event sets of up to 64 evaluations stay in
 * flight, so recording adds no host wait. */
pt_status pt_ctx_set_timing(pt_ctx *ctx, int enable);
pt_status pt_ctx_phase_times(pt_ctx *ctx, double ms[7], int64_t *count);

/* Share of the chip the near field takes while the far field runs beside
 * it (a schedule parameter of the FMM evaluation, which changes no result):
 * per_cu near-field workgroups per compute unit, 1..8, or 0 for the default
 * (3 when the near field forks before the upward pass, the mixed form; 4
 * when it forks after it, the FP64 form).  The environment variable
 * PT_NEAR_PER_CU sets it at context creation.  PT_EINVAL for another value;
 * waits for pending steps. */
pt_status pt_ctx_set_near_share(pt_ctx *ctx, int per_cu);

/* Which branch keeps the context's stream when the FMM evaluation forks the
 * near field off before the upward pass (the mixed form with leaves of 128
 * ions or more; a schedule parameter, which changes no result): 1 = the near
 * field stays and the far field (upward pass, M2L, L2L, far-field L2P) goes
 * to the second stream, 0 = the near field goes there, -1 (the default) =
 * chosen from the last measured batch's balance (the near field stays when
 * it has more than 2000 ordered pairs per V pair or the batch has fewer than
 * 1e6 V pairs).  The environment variable PT_NEAR_MAIN sets it at context
 * creation.  PT_EINVAL for another value; waits for pending steps. */
pt_status pt_ctx_set_fork(pt_ctx *ctx, int mode);

/* Work counts of the last FMM evaluation: [0] boxes, [1] leaves, [2] M2L
 * pairs, [3] P2P pairs (ordered, i != j counted), [4] levels, [5] ions. */
pt_status pt_ctx_work_counts(pt_ctx *ctx, int64_t counts[6]);

/* Step statistics since the context was created (each pointer nullable):
 * FMM evaluations of steps queued on capacities, FMM evaluations that
 * measured their batch's counts (with host waits), and runs of queued steps
 * that a capacity overflow sent back (see pt_step_batch).  Waits for pending
 * steps. */
pt_status pt_ctx_step_stats(pt_ctx *ctx, int64_t *queued, int64_t *measured, int64_t *reruns);

const char *pt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
