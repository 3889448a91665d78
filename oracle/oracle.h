/*
 * Penning-trap ion-crystal oracle: plain, slow, FP64 CPU reference.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU library.
 *
 * Every function follows a passage of Zaris et al., "Numerical simulations
 * of 3D ion crystal dynamics in a Penning trap using the fast multipole
 * method" (arXiv 2405.13973), cited by section / equation label:
 *   forces ........ Sec. 2.1, eqs. (pot_trap), (pot_wall), (hamiltonian)
 *   potential ..... eq. (hamiltonian) pair term per unit charge, eq. (rms_pot)
 *   integrator .... Sec. 2.2, eqs. (time_ev1), (time_ev2), (U0), (velocity_kick)
 *   photons ....... Sec. 2.2, eq. (laser_kick) and the Poisson-count passage
 *   FMM ........... Sec. 2.3, eqs. (FMM_coul), (multipole_error), (FMM_local),
 *                   and the "Algorithm" subsection (octree, upward and
 *                   downward passes, near field by direct summation).
 * Units are SI throughout.
 */
#ifndef PENNING_ORACLE_H
#define PENNING_ORACLE_H
#include <stdint.h>

/* Physical constants (CODATA 2022, SI). */
#define OR_E_CHARGE 1.602176634e-19
#define OR_H_PLANCK 6.62607015e-34
#define OR_K_BOLTZ 1.380649e-23
#define OR_EPS0 8.8541878188e-12
#define OR_AMU 1.66053906892e-27
#define OR_PI 3.14159265358979323846

/* Trap description: B along +z, axial frequency omega_z (rad/s), rotating
 * wall strength delta and rotation omega_r (rad/s).  damping (1/s, 0 = off):
 * the artificial damping of the paper's outlook -- the velocity relative to
 * the frame turning at omega_r (eq. rotation) is multiplied by
 * exp(-damping dt / 2) just before the kick and again just after it, so one
 * step damps it by exp(-damping dt) in two symmetric halves. */
typedef struct {
    double B;
    double omega_z;
    double delta;
    double omega_r;
    double damping;
} or_trap;

/* One laser beam of eq. (scattering_rate): propagation direction khat
 * (normalised before use), detuning Delta (rad/s), peak saturation s0 and
 * either a uniform profile (S = s0) or the 2D Gaussian of the cooling
 * appendix, S = s0 exp(-(y - offset_y)^2 / waist_y^2 - z^2 / waist_z^2),
 * in lab coordinates (m). */
typedef struct {
    double khat[3];
    double detuning;
    double s0;
    double waist_y, waist_z;
    double offset_y;
    int uniform;
} or_beam;

#define OR_MAX_BEAMS 4

/* Photon model.  mode 1 (or mode 0 with mean_per_step > 0): the fixed-mean
 * isotropic model -- per ion and per step a Poisson number of photons with
 * mean `mean_per_step`, each an emission recoil of h/(lambda m) in a
 * uniformly random direction.  mode 2: the beams of eq. (scattering_rate)
 * with natural linewidth gamma0 (rad/s), absorption and emission recoils of
 * eq. (laser_kick).  Otherwise off. */
typedef struct {
    double mean_per_step;
    double wavelength;
    int mode;
    double gamma0;
    int n_beams;
    or_beam beam[OR_MAX_BEAMS];
} or_laser;

/* Coulomb method: 0 = direct pairwise sum, 1 = fast multipole method. */
typedef struct {
    int method;
    int p;          /* maximum expansion degree */
    int leaf_size;  /* a box is split iff it holds more than leaf_size ions */
} or_force;

/* Octree produced by the oracle (see fmm.c). Boxes in canonical order:
 * ascending level, then ascending Morton prefix. */
typedef struct {
    int n;                 /* ions */
    int nbox;
    int nlevels;           /* deepest level + 1 */
    double lo[3], W;       /* root cube: lower corner and side */
    uint64_t *key;         /* 48-bit Morton key of each ion, in ion-id order */
    int32_t *perm;         /* perm[k] = id of the k-th ion in (key, id) order */
    /* per box */
    int32_t *level, *parent, *child_first, *nchild, *ion_begin, *ion_end;
    int32_t *ix, *iy, *iz; /* integer coordinates at its level */
    uint8_t *is_leaf;
    /* interaction lists in CSR form */
    int32_t *v_off, *v_src;        /* V list per box (M2L sources) */
    int32_t *near_off, *near_src;  /* near list per box (P2P source boxes, leaves only) */
} or_tree;

#endif
