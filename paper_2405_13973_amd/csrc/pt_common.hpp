// Internal declarations shared by the HIP sources of libpenning.
//
// Data layout in HBM (one context, one batch of crystals per launch):
//   - each crystal owns its state: one FP64 block x[n] y[n] z[n] vx[n] vy[n] vz[n]
//     (structure of arrays, ion-id order) and photons[n];
//   - a batch numbers all its ions consecutively, crystal by crystal; the
//     per-ion workspace (keys, sorted positions, field) is indexed by that
//     batch index or by the sorted slot;
//   - boxes of all crystals of a batch live in one table ordered by
//     (level, crystal, Morton prefix), so one launch per level covers the
//     whole batch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/penning.h"

namespace pt {

constexpr int kMaxLevel = 16;   // keys hold 16 bits per axis
constexpr int kMaxP = 20;
constexpr int kMaxKp = ((kMaxP + 1) * (kMaxP + 1) + 15) & ~15;
constexpr int kWin = 216;       // 6x6x6 window of M2L source offsets per target box
constexpr int kNeigh = 27;      // 3x3x3 colleague slots
constexpr int kP2PChunk = 2048; // near-field sources per work item (items are cut at range boundaries)
constexpr int kNearMax = kNeigh + 26 * kMaxLevel;  // near ranges of a leaf, at most
constexpr double kPi = 3.14159265358979323846;

// Physical constants (CODATA 2022, SI).
constexpr double kECharge = 1.602176634e-19;
constexpr double kPlanck = 6.62607015e-34;
constexpr double kEps0 = 8.8541878188e-12;
constexpr double kBoltzmann = 1.380649e-23;

// Everything a batched kernel needs to know about one crystal.  Built on
// the host each time a batch is formed and copied to the device.
// One laser beam (eq. scattering_rate): unit direction, detuning (rad/s),
// peak saturation and profile (uniform, or Gaussian in y and z).
constexpr int kMaxBeams = 4;
struct BeamDev {
    double khat[3];
    double detuning;
    double s0;
    double waist_y, waist_z, offset_y;
    int32_t uniform;
    int32_t pad;
};

struct CrystalDev {
    double *state;        // 6 n doubles, see above
    // Working copy of the state for the current evaluation, same layout:
    // the first half drift writes here, every kernel up to the kick reads
    // here, and only the kick writes the crystal's own state, so a step that
    // fails before its kick leaves the state as it was.
    double *mid;
    int32_t *photons;     // n
    int32_t *nonfinite;   // set to 1 by the kick when it produces a non-finite value
    int32_t *ctx_nonfinite;  // the same, one word for the whole context
    int32_t n;
    int32_t ion_off;      // first batch index of this crystal
    // integrator (host-computed in FP64)
    double dt, t0;
    double c_half, s_half;  // cos / sin of omega_c dt/2
    double a_half, b_half;  // sin(omega_c dt/2)/omega_c, (1 - cos)/omega_c  (dt/2, 0 when B = 0)
    double qkz;             // q k_z = m omega_z^2
    double delta, omega_r;
    double inv_m;
    double damp_f;          // exp(-damping dt / 2), applied before and after the kick
    double mass;            // m (rotating-frame diagnostics)
    double wc;              // omega_c = q B / m
    double coul;            // k_e q^2
    double recoil;          // h / (lambda m), 0 when the laser is off
    double poisson_F[17];   // cumulative Poisson table of the photon mean
    int32_t laser_on;       // 1: fixed-mean photons, 2: beams
    int32_t n_beams;
    int32_t damp_on;        // artificial damping of the rotating-frame velocity
    int32_t pad2;
    double gamma0;          // natural linewidth (rad/s), beams only
    double kwave;           // 2 pi / wavelength (1/m)
    BeamDev beam[kMaxBeams];
    uint64_t seed;
    uint64_t step0;         // step index of the first step of the current call
    int64_t dpart;          // first double of this crystal's direct-sum partials (see direct_chunks)
};

// Root cube of a crystal: lower corner o, side W, quantisation scale 2^16/W.
struct RootCube {
    double o[3];
    double W;
    double S;
    double pad[3];
};

// Device size summary of the current tree (read back by the measuring
// evaluation), with the run state of a queued sequence of steps: halt is set
// (and stays set) when a step's tree or lists exceed the capacities its
// buffers were sized for, after which every kernel of the sequence does
// nothing and each kick leaves the state as it was; fail_step is the
// sequence's first step that was not completed (-1: none).
struct TreeSummary {
    int32_t level_start[kMaxLevel + 2];  // boxes of level l: [level_start[l], level_start[l+1])
    int32_t nbox;
    int32_t sort_error;  // non-zero: the sort's look-back gave up waiting (see k_radix_pass)
    int32_t halt;
    int32_t fail_step;
    int32_t refine_overflow;  // non-zero: a queued step's sort by the top digits left a run too long to finish
};

// Capacities of a queued force evaluation's buffers and grids: boxes, tree
// levels, near-field work items, M2L pairs, and boxes per level.
struct Caps {
    int32_t nbox, nlev, items, pairs;
    int32_t lvl[kMaxLevel + 1];
};

// ---------------------------------------------------------------- helpers

__host__ __device__ inline uint64_t spread3_16(uint64_t x)
{
    x &= 0xFFFFull;
    x = (x | (x << 16)) & 0x0000FF0000FFull;
    x = (x | (x << 8)) & 0x00F00F00F00Full;
    x = (x | (x << 4)) & 0x0C30C30C30C3ull;
    x = (x | (x << 2)) & 0x249249249249ull;
    return x;
}

__host__ __device__ inline uint32_t compact3_16(uint64_t x)
{
    x &= 0x249249249249ull;
    x = (x | (x >> 2)) & 0x0C30C30C30C3ull;
    x = (x | (x >> 4)) & 0x00F00F00F00Full;
    x = (x | (x >> 8)) & 0x0000FF0000FFull;
    x = (x | (x >> 16)) & 0xFFFFull;
    return (uint32_t)x;
}

// Morton code of integer coordinates: x in the top bit of each triple.
__host__ __device__ inline uint64_t morton3(uint32_t ix, uint32_t iy, uint32_t iz)
{
    return (spread3_16(ix) << 2) | (spread3_16(iy) << 1) | spread3_16(iz);
}

// Monotone map of a double onto uint64 so that integer min/max order doubles.
__host__ __device__ inline uint64_t dbl_to_ordered(double v)
{
    uint64_t u;
    __builtin_memcpy(&u, &v, sizeof(u));
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__host__ __device__ inline double ordered_to_dbl(uint64_t u)
{
    uint64_t b = (u & 0x8000000000000000ull) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
    double d;
    __builtin_memcpy(&d, &b, sizeof(d));
    return d;
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32 -> 64 bit
// products with multipliers 0xD2511F53 and 0xCD9E8D57; the key advances by
// the Weyl increments 0x9E3779B9, 0xBB67AE85 between rounds.
__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)0xD2511F53u * c[0];
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t x0 = (uint32_t)(pb >> 32) ^ c[1] ^ k0;
        const uint32_t x2 = (uint32_t)(pa >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)pb;
        c[3] = (uint32_t)pa;
        c[0] = x0;
        c[2] = x2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform double in [0,1) from the high 27 bits of a and the high 26 of b.
__host__ __device__ inline double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Work split of the direct sum over a crystal of n ions.  A block takes
// kDirTile targets (kDirT per lane of one wave) and one of direct_chunks(n)
// contiguous chunks of the sources; each of its kDirWaves waves takes its own
// piece of direct_piece(n) sources of that chunk (the last pieces shorter or
// empty).  The block writes the chunk's partial sums, NC x chunks x n
// doubles per crystal from CrystalDev::dpart (component k, chunk s, ion i at
// (k chunks + s) n + i), and each ion then adds its chunks in order.  Both
// numbers depend on n alone, so a crystal's sums are formed in the same
// order whatever batch it is in.  Chunks are chosen to give about
// kDirBlocksWanted blocks for one crystal, with pieces of at least
// kDirMinPiece sources.
constexpr int kDirT = 2;
constexpr int kDirTile = 64 * kDirT;
constexpr int kDirWaves = 8;
constexpr int kDirBlocksWanted = 4096;
constexpr int kDirMaxChunks = 16;
constexpr int kDirMinPiece = 64;

__host__ __device__ constexpr int direct_chunks(int n)
{
    const int tiles = (n + kDirTile - 1) / kDirTile;
    int s = tiles > 0 ? (kDirBlocksWanted + tiles - 1) / tiles : 1;
    const int by_piece = n / (kDirWaves * kDirMinPiece);
    if (s > by_piece) s = by_piece;
    if (s > kDirMaxChunks) s = kDirMaxChunks;
    return s < 1 ? 1 : s;
}

__host__ __device__ constexpr int direct_piece(int n)
{
    const int pieces = direct_chunks(n) * kDirWaves;
    return ((n + pieces - 1) / pieces + 7) / 8 * 8;
}

// One block of the direct sum: crystal c, its targets first..first+kDirTile-1,
// source chunk `chunk`.
struct DirBlock {
    int32_t c, first, chunk, pad;
};

}  // namespace pt

// Error plumbing for host code.
void pt_set_error(const char *fmt, ...);
#define PT_HIP(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            pt_set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            return PT_EDEVICE;                                                                    \
        }                                                                                         \
    } while (0)
