// Upward pass, downward pass and evaluation of the GPU FMM (Zaris et al.,
// Sec. 2.3): multipole expansions of the leaves (P2M), merged into parents
// (M2M), multipole-to-local conversion over the V lists (M2L), parent local
// expansions shifted to children (L2L), then per ion the far field of its
// leaf's local expansion (L2P) plus the near field by direct summation (P2P).
//
// T is the expansion / near-field type: double for the FP64 form, float for
// the mixed form.  Box centres, ion-to-centre offsets and the integrator stay
// FP64 in both; in the mixed form the offsets are rounded to FP32 only after
// the FP64 subtraction, and FP32 near-field sums are compensated (Kahan).
#include <algorithm>

#include "fmm_math.hpp"
#include "pt_common.hpp"
#include "pt_kernels.hpp"

namespace pt {

__device__ inline int octant_of(int ix, int iy, int iz) { return ((ix & 1) << 2) | ((iy & 1) << 1) | (iz & 1); }

// P2M: one 256-thread block per leaf.  Ions are taken `chunk` (64, or 32 when
// the tile would exceed 64 KiB) at a time into an LDS tile
// [coefficient][ion] of conj(Rh_n^m): lane j of every wave takes ion j, and
// the four waves split the orders m (kP2MWaves ranges of about equal term
// counts; each wave runs the m recurrence from m = 0 to reach its first
// order), so each term is computed by the same operations as in one pass
// over all m.  Then each thread sums one coefficient (two when Kp > 256)
// over the tile's ions, in four interleaved partial sums (ions j = 0, 1, 2,
// 3 mod 4) added in a fixed order, which keeps the LDS reads independent of
// one another.
constexpr int kP2MWaves = 4;
constexpr int kP2MThreads = 64 * kP2MWaves;
constexpr int kP2MMaxPer = 2;  // coefficients per thread: Kp <= 512

template <typename T>
static int p2m_chunk(int Kp, int leaf_size)
{
    return leaf_size > 32 && (size_t)Kp * 65 * sizeof(T) <= 65536 ? 64 : 32;
}

// First order m of wave w's range: the orders are cut where the running
// count of terms (p - m + 1 per order) reaches w / kP2MWaves of the total.
__device__ inline int p2m_first_order(int p, int w)
{
    const int total = (p + 1) * (p + 2) / 2;
    int m = 0, run = 0;
    while (m <= p && run * kP2MWaves < w * total) run += p - m++ + 1;
    return m;
}

template <typename T>
__global__ __launch_bounds__(kP2MThreads) void k_p2m(BoxTable bt, const TreeSummary *__restrict__ sum,
                                                     const double *__restrict__ sp, int ntot, int p, int Kp,
                                                     int chunk, const T *__restrict__ rec, T *__restrict__ M)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *C = reinterpret_cast<T *>(smem_raw);  // [Kp][chunk + 1]
    __shared__ T rec_s[2 * kq(kMaxP)];      // the recurrence fields the expansion needs
    const int b = blockIdx.x;
    if (sum->halt || b >= sum->nbox || !bt.leaf[b]) return;
    const double4 g = bt.geo[b];
    const double ih = 1.0 / g.w;
    const int K = kcoef(p);
    for (int i = threadIdx.x; i < 2 * kq(p); i += kP2MThreads) rec_s[i] = rec[i];
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m_lo = p2m_first_order(p, w), m_hi = w + 1 < kP2MWaves ? p2m_first_order(p, w + 1) : p + 1;
    const int i0 = bt.begin[b], i1 = bt.end[b];
    const int ld = chunk + 1;  // odd: the rows of a column fall in distinct banks
    T acc[kP2MMaxPer];
#pragma unroll
    for (int r = 0; r < kP2MMaxPer; ++r) acc[r] = T(0);
    for (int c0 = i0; c0 < i1; c0 += chunk) {
        const int cnt = min(chunk, i1 - c0);
        if (lane < cnt && m_lo < m_hi) {
            const int i = c0 + lane;
            p2m_terms<T>(p, rec_s, (T)((sp[i] - g.x) * ih), (T)((sp[ntot + i] - g.y) * ih),
                         (T)((sp[2 * ntot + i] - g.z) * ih), C + lane, ld, m_lo, m_hi);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kP2MMaxPer; ++r) {
            const int s = threadIdx.x + kP2MThreads * r;
            if (s < K) {
                const T *row = C + s * ld;
                T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
                int j = 0;
                for (; j + 4 <= cnt; j += 4) {
                    s0 += row[j];
                    s1 += row[j + 1];
                    s2 += row[j + 2];
                    s3 += row[j + 3];
                }
                if (j < cnt) s0 += row[j];
                if (j + 1 < cnt) s1 += row[j + 1];
                if (j + 2 < cnt) s2 += row[j + 2];
                acc[r] += (s0 + s1) + (s2 + s3);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kP2MMaxPer; ++r) {
        const int s = threadIdx.x + kP2MThreads * r;
        if (s < Kp) M[(size_t)b * Kp + s] = s < K ? acc[r] : T(0);
    }
}

// ---------------------------------------------------------------- M2M / L2L
//
// The translations between levels are dense contractions on the matrix cores:
// with scaled coefficients the 8 child-to-parent (M2M) and the 8
// parent-to-child (L2L) operators do not depend on level or crystal, so one
// level's boxes of every crystal form the columns of one GEMM per octant
// slot,
//     out[:, boxes] (+)= sum_slots A_slot (Kp x Kp) * X[src(slot, boxes)] (Kp x n).
// A workgroup of 4 waves takes 64 boxes (16 per wave) and one slot group; per
// slot it stages k-chunks of the operator (column-major, zero padded) and of
// the 64 source expansions in LDS, and every wave runs v_mfma 16x16x4 over
// all row blocks of its 16 columns.  Slot groups (one octant each) write
// separate partial sums that a second kernel adds in group order, so every
// box's sum has a fixed order whatever tile it landed in (batch-invariant,
// deterministic).  (M2L, the conversion over the V lists, is organised by
// operator instead: k_m2l.hip.)

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 op(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }  // output row of element r
};
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int kM2LWaves = 4;           // 16 target columns per wave
constexpr int kM2LCols = 16 * kM2LWaves;
constexpr int kM2LRB = 12;             // row blocks (of 16) per workgroup: Kp <= 192 in one pass

// One translation GEMM serves M2M and L2L:
//   out[t] (op) sum over slots s of  A[op(s)] * X[src(t, s)]
// targets t: either bucket lists (cnt non-null; with lvl non-null each
// bucket's list starts at the level's first box index) or the box range
// [b0, b0 + n);
// src(t, s) = srctab[t * src_stride + col(s)] (-1: no source); an operator
// index above 255 carries reflection signs (mask = index >> 8).
// Output modes: 0 partial sums per slot group, 1 overwrite (skipping targets
// flagged in `skip`), 2 accumulate.
struct XlateArgs {
    const int32_t *cnt;   // bucket sizes (bucketed targets) or nullptr
    const int32_t *list;  // bucket lists, list_stride apart
    int list_stride;
    int nbucket;          // 8 (by parity) or 1
    // target range when cnt == nullptr: [b0, b0 + nrange), or with lvl non-null
    // the boxes of tree level `level`, [lvl[level], lvl[level + 1]) read on
    // the device (lvl = the summary's level_start)
    int b0, nrange;
    const int32_t *lvl;
    int level;
    const TreeSummary *sum;  // the run state: nothing is done once it halts
    int tile_stride, ngroup, nrowgrp, Kp;
    const int2 *slots;    // per bucket nslot entries {source column, operator index}
    int nslot;
    const int32_t *srctab;
    int src_stride;
    const uint8_t *skip;  // mode 1 only
    int mode;
    int nbox;
};

constexpr int kXSlots = 32;  // slots per workgroup, at most

// Software-pipelined: the (slot, k-chunk) steps of a tile run as one
// sequence; the loads of step i+1 are issued into registers before the
// matrix-core work of step i, so their latency overlaps it.  NRB (row blocks
// of 16 per workgroup) and KC (the k-chunk of a step: 16, or 48 for small
// grids, where the chain of steps rather than the matrix cores bounds the
// time) are compile-time constants so the matrix-core loop has no branches;
// neither changes the order in which a target's terms are accumulated.
// Every load is unconditional: k-chunks divide Kp,
// rows past Kp (PARTIAL row groups only) read an in-bounds address and are
// replaced by zero, and a missing source reads X[zrow], an expansion row
// kept at zero.
// ROLE only names the kernel symbol (1 M2M, 2 L2L) so that profiles tell
// the uses apart.
template <typename T, int NRB, bool PARTIAL, int ROLE, int KC>
__global__ __launch_bounds__(64 * kM2LWaves) void k_xlate(XlateArgs a, const T *__restrict__ At,
                                                         const T *__restrict__ X, T *__restrict__ out)
{
    // the upward and downward passes run beside the near field: a raised wave
    // priority keeps their short per-level launches from waiting behind its waves
    __builtin_amdgcn_s_setprio(1);
    using MF = Mfma<T>;
    constexpr int ROWS = NRB * 16;
    constexpr int NT = 64 * kM2LWaves;
    constexpr int kXA = KC * ROWS / NT;  // operator values staged per thread (exact)
    constexpr int kXB = KC * kM2LCols / NT;
    __shared__ T As[KC][ROWS];             // operator chunk, [k][row]
    __shared__ T Bsh[kM2LCols][KC + 1];    // source chunk, [target][k] (padded: no bank conflicts)
    __shared__ int32_t tgt_s[kM2LCols];
    __shared__ int32_t src_s[kXSlots][kM2LCols];
    __shared__ int32_t act_s[kXSlots + 1];  // active slots (local index); act_s[kXSlots] = count
    __shared__ int32_t op_s[kXSlots];       // operator index (+ 256 x reflection mask) of each local slot
    __shared__ uint8_t cbits_s[kMaxKp];     // reflection sign bits of each coefficient
    const int Kp = a.Kp;
    const int zrow = a.nbox;  // all-zero expansion row
    for (int i = threadIdx.x; i < Kp; i += 64 * kM2LWaves) cbits_s[i] = (uint8_t)refl_bits(i);
    const int lin = blockIdx.x;
    const int o = lin % a.nbucket;
    int rest = lin / a.nbucket;
    const int rg = rest % a.nrowgrp;
    rest /= a.nrowgrp;
    const int g = rest % a.ngroup;
    const int tile0 = rest / a.ngroup;
    if (a.sum->halt) return;
    const int b0 = a.lvl ? a.lvl[a.level] : a.b0;
    const int n = a.cnt ? a.cnt[o] : (a.lvl ? a.lvl[a.level + 1] - b0 : a.nrange);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int row0 = rg * ROWS;
    const int s0 = (a.nslot * g) / a.ngroup, s1 = (a.nslot * (g + 1)) / a.ngroup;
    const int ns = s1 - s0;  // <= kXSlots (the launcher guarantees it)
    const int nchunk = Kp / KC;
    // per-thread staging map (fixed for the kernel)
    int a_off[kXA];
    bool a_ok[kXA];
#pragma unroll
    for (int j = 0; j < kXA; ++j) {
        const int e = tid + NT * j;
        const int kk = e / ROWS, r = e - kk * ROWS;
        a_ok[j] = !PARTIAL || row0 + r < Kp;
        a_off[j] = a_ok[j] ? kk * Kp + r : 0;
    }
    int b_t[kXB], b_k[kXB];  // source values staged per thread: target, k
#pragma unroll
    for (int j = 0; j < kXB; ++j) {
        b_t[j] = (tid + NT * j) / KC;
        b_k[j] = (tid + NT * j) % KC;
    }
    T ra[kXA], rb_[kXB];
    auto load_step = [&](int step) {
        const int q = step / nchunk;
        const int sl = act_s[q];
        const int k0 = (step - q * nchunk) * KC;
        const T *Ad = At + (size_t)(op_s[sl] & 255) * Kp * Kp + (size_t)k0 * Kp + row0;
#pragma unroll
        for (int j = 0; j < kXA; ++j) {
            const T v = Ad[a_off[j]];
            ra[j] = PARTIAL ? (a_ok[j] ? v : T(0)) : v;
        }
#pragma unroll
        for (int j = 0; j < kXB; ++j) rb_[j] = X[(size_t)src_s[sl][b_t[j]] * Kp + k0 + b_k[j]];
    };
    for (int tile = tile0; tile * kM2LCols < n; tile += a.tile_stride) {
        __syncthreads();  // previous tile finished with the shared arrays
        if (tid < kM2LCols) {
            const int t = tile * kM2LCols + tid;
            tgt_s[tid] = t < n ? (a.cnt ? a.list[(size_t)o * a.list_stride + (a.lvl ? b0 : 0) + t] : b0 + t) : -1;
        }
        if (tid < ns) op_s[tid] = a.slots[o * a.nslot + s0 + tid].y;
        __syncthreads();
        for (int e = tid; e < ns * kM2LCols; e += NT) {
            const int sl = e / kM2LCols, t = e - sl * kM2LCols;
            const int tg = tgt_s[t];
            const int sidx = tg >= 0 ? a.srctab[(size_t)tg * a.src_stride + a.slots[o * a.nslot + s0 + sl].x] : -1;
            src_s[sl][t] = sidx >= 0 ? sidx : zrow;
        }
        __syncthreads();
        if (wave == 0) {  // compact the slots that have at least one source, in slot order
            int cnt = 0;
            for (int sl = 0; sl < ns; ++sl) {
                const bool has = __ballot(src_s[sl][lane] != zrow) != 0ull;
                if (has) {
                    if (lane == 0) act_s[cnt] = sl;
                    ++cnt;
                }
            }
            if (lane == 0) act_s[kXSlots] = cnt;
        }
        __syncthreads();
        const int nsteps = act_s[kXSlots] * nchunk;
        typename MF::v4 acc[NRB];
#pragma unroll
        for (int r = 0; r < NRB; ++r) acc[r] = typename MF::v4{0, 0, 0, 0};
        // Reflected operators A = S T_base S: the column signs S go onto the
        // staged sources; the row signs are carried by the accumulator, which
        // holds S(cur) times the partial result and is re-signed only when
        // the reflection mask changes from one slot to the next.
        auto resign = [&](int flipmask) {
#pragma unroll
            for (int r = 0; r < NRB; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = row0 + r * 16 + MF::row(lane, q);
                    if ((!PARTIAL || row < Kp) && (__popc(flipmask & cbits_s[row]) & 1)) acc[r][q] = -acc[r][q];
                }
        };
        int cur = 0;
        if (nsteps > 0) load_step(0);
        for (int step = 0; step < nsteps; ++step) {
            const int q = step / nchunk;
            const int k0 = (step - q * nchunk) * KC;
            const int mask = op_s[act_s[q]] >> 8;
            __syncthreads();  // the previous step is done reading As / Bsh
#pragma unroll
            for (int j = 0; j < kXA; ++j) (&As[0][0])[tid + NT * j] = ra[j];
#pragma unroll
            for (int j = 0; j < kXB; ++j) {
                const bool bneg = __popc(mask & cbits_s[k0 + b_k[j]]) & 1;
                Bsh[b_t[j]][b_k[j]] = bneg ? -rb_[j] : rb_[j];
            }
            if (mask != cur) {
                resign(mask ^ cur);
                cur = mask;
            }
            __syncthreads();
            if (step + 1 < nsteps) load_step(step + 1);
#pragma unroll
            for (int k4 = 0; k4 < KC; k4 += 4) {
                const int kk = k4 + (lane >> 4);
                const T bv = Bsh[wave * 16 + (lane & 15)][kk];
                T av[NRB];
#pragma unroll
                for (int r = 0; r < NRB; ++r) av[r] = As[kk][r * 16 + (lane & 15)];
#pragma unroll
                for (int r = 0; r < NRB; ++r) acc[r] = MF::op(av[r], bv, acc[r]);
            }
            // Schedule: the LDS reads of k-step i + 1 issue as one group ahead
            // of the matrix-core instructions of step i, so that their latency
            // hides behind matrix work instead of stalling every instruction
            // pair (the default schedule reuses one register pair and waits).
            __builtin_amdgcn_sched_group_barrier(0x100, NRB + 1, 0);
#pragma unroll
            for (int k4 = 4; k4 < KC; k4 += 4) {
                __builtin_amdgcn_sched_group_barrier(0x100, NRB + 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NRB, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, NRB, 0);
        }
        if (cur) resign(cur);
        const int tg = tgt_s[wave * 16 + (lane & 15)];
        if (tg >= 0 && !(a.mode == 1 && a.skip[tg])) {
            T *dst = out + (a.mode == 0 ? ((size_t)g * a.nbox + tg) * Kp : (size_t)tg * Kp) + row0;
#pragma unroll
            for (int r = 0; r < NRB; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = r * 16 + MF::row(lane, q);
                    if (!PARTIAL || row0 + row < Kp) {
                        T &d = dst[row];
                        d = a.mode == 2 ? d + acc[r][q] : acc[r][q];
                    }
                }
        }
    }
}

// Row groups of a translation GEMM: the Kp output rows (Kp / 16 blocks of 16)
// are split over nrowgrp workgroups, each holding ceil(blocks / nrowgrp)
// blocks (at most kM2LRB).  Small problems take more row groups, so that the
// grid still fills the chip (about kXMinGrid workgroups); the split does not
// change any summation order.
constexpr long kXMinGrid = 128;
constexpr long kXWideGrid = 768;
// Beside a near field of four or five workgroups per compute unit (72 VGPRs
// per wave), a SIMD keeps 224 or 152 VGPRs free: the translations then use
// 16-value k-chunks and at most this many row blocks per workgroup (the
// compiled variants need at most 144 VGPRs), so their waves find room
// instead of waiting for near-field workgroups to finish.
constexpr int kXNarrowRB = 7;
static void xlate_rows(XlateArgs &a, long base_grid, bool narrow)
{
    const int blocks = a.Kp / 16;
    int nrg = ceil_div(blocks, narrow ? kXNarrowRB : kM2LRB);
    while (nrg < blocks && base_grid * nrg < kXMinGrid) {
        // next row-group count that shrinks the per-workgroup block count
        const int nrb = ceil_div(blocks, nrg);
        while (nrg < blocks && ceil_div(blocks, nrg) == nrb) ++nrg;
    }
    a.nrowgrp = nrg;
}

template <typename T, int ROLE>
static void launch_xlate(const XlateArgs &a, int grid, const T *At, const T *X, T *out, bool narrow, hipStream_t st)
{
    const int blocks = a.Kp / 16;
    const int nrb = ceil_div(blocks, a.nrowgrp);
    const bool partial = nrb * a.nrowgrp != blocks;
    // k-chunks of 48 when the grid is too small to hide a step's load
    // latency behind other workgroups' matrix-core work
    const bool wide = !narrow && a.Kp % 48 == 0 && (long)grid < kXWideGrid;
    switch ((nrb * 2 + (partial ? 1 : 0)) * 2 + (wide ? 1 : 0)) {
#define PT_XL(NB)                                                                                       \
    case 4 * NB: k_xlate<T, NB, false, ROLE, 16><<<grid, 64 * kM2LWaves, 0, st>>>(a, At, X, out); break; \
    case 4 * NB + 2: k_xlate<T, NB, true, ROLE, 16><<<grid, 64 * kM2LWaves, 0, st>>>(a, At, X, out); break;
#define PT_XLW(NB)                                                                                      \
    case 4 * NB + 1: k_xlate<T, NB, false, ROLE, 48><<<grid, 64 * kM2LWaves, 0, st>>>(a, At, X, out); break; \
    case 4 * NB + 3: k_xlate<T, NB, true, ROLE, 48><<<grid, 64 * kM2LWaves, 0, st>>>(a, At, X, out); break;
        PT_XL(1) PT_XL(2) PT_XL(3) PT_XL(4) PT_XL(5) PT_XL(6) PT_XL(7) PT_XL(8) PT_XL(9) PT_XL(10) PT_XL(11)
        PT_XL(12)
        PT_XLW(1) PT_XLW(2) PT_XLW(3) PT_XLW(4) PT_XLW(5) PT_XLW(6) PT_XLW(7) PT_XLW(8) PT_XLW(9) PT_XLW(10)
        PT_XLW(11) PT_XLW(12)
#undef PT_XL
#undef PT_XLW
    default: break;
    }
}

// The boxes of tree level `level` ([lvl[level], lvl[level + 1]), read on the
// device): out = (mode 2: out +) sum of the slot-group partials, in group
// order; mode 1 leaves the boxes flagged in skip untouched.  Grid-stride.
template <typename T>
__global__ void k_xlate_reduce(const TreeSummary *__restrict__ sum, int level, int Kp, int nbox, int ngroup, int mode,
                               const uint8_t *__restrict__ skip, const T *__restrict__ part, T *__restrict__ out)
{
    __builtin_amdgcn_s_setprio(1);  // beside the near field, as k_xlate
    if (sum->halt) return;
    const int b0 = sum->level_start[level], n = sum->level_start[level + 1] - b0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)n * Kp;
         e += (size_t)gridDim.x * blockDim.x) {
        const int b = b0 + (int)(e / Kp);
        const size_t off = (size_t)b * Kp + e % Kp;
        if (mode == 1 && skip[b]) continue;
        T acc = 0;
        for (int g = 0; g < ngroup; ++g) acc += part[(size_t)g * nbox * Kp + off];
        out[off] = mode == 2 ? out[off] + acc : acc;
    }
}

// Near field (P2P) of one work item per 256-thread workgroup (grid-stride
// over the items): up to 64 targets of a leaf against the sources of a run of
// its near ranges.  The ranges are concatenated and staged through LDS
// kP2PStage sources at a time, so the pair loop reads only LDS and a barrier
// pair serves hundreds of sources rather than one leaf.  FP64 form: staged
// FP64 positions, FP64 separations.  Mixed form: staged as 31-bit fixed-point
// coordinates in the target leaf's near frame (a cube about the leaf's centre
// that holds all its near sources; offsets made in FP64, one quantum = the
// frame side / 2^31), so that a separation is an exact integer difference
// converted once to FP32: its error is at most a quantum (about 1e-9 of the
// leaf's side) whatever the pair's distance, where offsets rounded to FP32
// would carry ~1e-7 of the box size into every separation (the rare very
// close pairs of random crystals then dominate the RMS force error).  The loop works in quanta (r^2 offset by the softening
// in quanta^2) and the partials are scaled back to metres when written.
// r^-3 is the FP32 hardware reciprocal square root (1 ulp) cubed in the mixed
// form, and the hardware FP64 estimate refined as in the direct sum in the
// FP64 form.  An item with nt targets gives each
// target floor(256 / nt) threads (phases), which take source blocks round
// robin; within a block sources are summed plainly and each block is added
// to the phase's total, with Kahan compensation in FP32 (plainly in FP64).
// The phases of a target are then added in phase order.  Four waves share
// one staged tile, so that a compute unit holds enough waves to hide the
// latency of the pair arithmetic.
// Partial fields go to part[item][target][3]; with POT the potential sum
// sum 1/r over the pairs with r > 0 comes along, in part[item][target][4].
constexpr int kP2PStage = 512;
constexpr int kP2PThreads = 256;  // four waves share one staged source tile

// Added to every FP32 near-field r^2 (m^2, in quanta^2 in the loop): 1/r^3
// stays finite; at 0.1 micrometre the relative change is 1e-10, far below
// FP32 rounding.
constexpr double kSoft2 = 1e-24;

// A coordinate offset d >= 0 within a frame of side 2^31 / s as a 31-bit
// fixed-point integer (s quanta per metre; truncated, clamped to the frame).
__device__ inline uint32_t p2p_quant(double d, double s)
{
    return (uint32_t)fmin(fmax(d * s, 0.0), 2147483647.0);
}
// Added to every FP64 near-field r^2 (m^2): below the rounding of any r^2
// above 2^-626, and the weight at r = 0 (about 2^1020) stays finite.
constexpr double kSoft2F64 = 0x1p-680;

template <typename T, bool POT>
__global__ __launch_bounds__(kP2PThreads) void k_p2p(BoxTable bt, const TreeSummary *__restrict__ sum,
                                                     const double *__restrict__ sp, int ntot,
                                                     const int2 *__restrict__ near, int stride,
                                                     const int4 *__restrict__ work, const uint32_t *__restrict__ n_items_p,
                                                     T *__restrict__ part, int *__restrict__ queue,
                                                     const double *__restrict__ near_ext)
{
    if (sum->halt) return;
    const int n_items = (int)*n_items_p;
    constexpr int NT = kP2PThreads;
    constexpr int NC = POT ? 4 : 3;  // partial components per target
    constexpr int kU = kP2PStage / NT;
    // staged sources as (x, y) pairs and z: 24 B per source, so that six of
    // these workgroups and one translation-GEMM workgroup share a compute
    // unit's LDS when the two kernels run side by side
    __shared__ double2 sxy[kP2PStage];
    __shared__ double szz[kP2PStage];
    // the mixed form's staged fixed-point coordinates reuse the (x, y) pairs' space
    uint4 *const sq = reinterpret_cast<uint4 *>(sxy);
    __shared__ int pre_s[kNearMax + 1];  // prefix of the item's range lengths
    __shared__ int beg_s[kNearMax];      // first ion of each range minus its prefix
    __shared__ int total_s;
    // the phases' hand-off arrays reuse the staging buffer once an item's
    // sources are done (NC x NT values of T fit in it)
    static_assert(sizeof(T) * 4 * NT <= sizeof(double2) * kP2PStage, "hand-off arrays must fit the stage");
    T *const hx = reinterpret_cast<T *>(sxy), *const hy = hx + NT, *const hz = hy + NT, *const hp = hz + NT;
    const int tid = threadIdx.x, lane = tid & 63;
    __shared__ int it_s;
    for (int round = 0;; ++round) {
        // the next item: with a queue (a grid capped below the item count),
        // taken from it as workgroups free up, which balances items of very
        // different sizes; without, the k-th of the grid stride.  Every item
        // writes its own partials, so the order changes no result.
        __syncthreads();  // the previous item is done with the shared arrays
        if (tid == 0) it_s = queue ? atomicAdd(queue, 1) : (int)blockIdx.x + round * (int)gridDim.x;
        __syncthreads();
        const int it = it_s;
        if (it >= n_items) break;
        const int4 w = work[it];
        const int b = w.x;
        const int2 *row = near + (size_t)b * stride;
        const int nt = max(1, min(64, bt.end[b] - w.y));
        const int nph = NT / nt;                            // phases per target (>= 4)
        const int blk = nph <= 4 ? 32 : 16;                 // sources per block
        const int ti = tid % nt, ph = tid / nt;             // ph >= nph: idle thread
        const int k = w.y + ti;
        const double xi = sp[k], yi = sp[ntot + k], zi = sp[2 * ntot + k];
        // Mixed form: separations are differences of 31-bit fixed-point
        // coordinates in the leaf's near frame (the cube of half side
        // near_ext[b] about the leaf's centre, which holds every near source;
        // one quantum is 2 near_ext / 2^31, and the difference of two such
        // integers is exact), converted to FP32 and kept in quanta until the
        // partials are scaled back to metres.
        double4 fc{};
        double qs = 0.0;
        uint32_t qx = 0, qy = 0, qz = 0;
        float soft_q = 0.0f, back2 = 0.0f, back1 = 0.0f;
        if constexpr (sizeof(T) == 4) {
            fc = bt.geo[b];
            fc.w = near_ext[b];  // half side of the frame
            qs = 1073741824.0 / fc.w;
            qx = p2p_quant(xi - fc.x + fc.w, qs);
            qy = p2p_quant(yi - fc.y + fc.w, qs);
            qz = p2p_quant(zi - fc.z + fc.w, qs);
            const double qm = fc.w / 1073741824.0;  // metres per quantum
            soft_q = (float)(kSoft2 / (qm * qm));
            back2 = (float)(1.0 / (qm * qm));
            back1 = (float)(1.0 / qm);
        }
        const int nr = min(w.w - w.z, kNearMax);
        if (tid < 64) {  // prefix of the range lengths, by the first wave
            int total = 0;
            for (int r0 = 0; r0 < nr; r0 += 64) {
                const int r = r0 + lane;
                int2 rg = make_int2(0, 0);
                if (r < nr) rg = row[w.z + r];
                int x = rg.y - rg.x;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const int y = __shfl_up(x, off);
                    if (lane >= off) x += y;
                }
                if (r < nr) {
                    pre_s[r + 1] = total + x;
                    beg_s[r] = rg.x - (total + x - (rg.y - rg.x));
                }
                total += __shfl(x, 63);
            }
            if (lane == 0) {
                pre_s[0] = 0;
                total_s = total;
            }
        }
        __syncthreads();
        const int total = total_s;
        T ax = 0, ay = 0, az = 0, cx = 0, cy = 0, cz = 0, av = 0, cv = 0;
        for (int s0 = 0; s0 < total; s0 += kP2PStage) {
            const int n = min(kP2PStage, total - s0);
            // source index of each staged position: binary search for the
            // first, then a forward walk (positions grow by NT)
            int js[kU];
            {
                int a = 0, e = nr;  // last r with pre_s[r] <= pos
                const int pos0 = s0 + tid;
                while (e - a > 1) {
                    const int m = (a + e) >> 1;
                    if (pre_s[m] <= pos0) a = m;
                    else e = m;
                }
                int r = a;
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int pos = s0 + tid + NT * u;
                    js[u] = -1;
                    if (tid + NT * u < n) {
                        while (r + 1 < nr && pre_s[r + 1] <= pos) ++r;
                        js[u] = beg_s[r] + pos;
                    }
                }
            }
            double sx[kU], sy[kU], sz[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int j = js[u] >= 0 ? js[u] : 0;
                sx[u] = sp[j];
                sy[u] = sp[ntot + j];
                sz[u] = sp[2 * ntot + j];
            }
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (js[u] >= 0) {
                    if constexpr (sizeof(T) == 4) {
                        sq[tid + NT * u] =
                            make_uint4(p2p_quant(sx[u] - fc.x + fc.w, qs), p2p_quant(sy[u] - fc.y + fc.w, qs),
                                       p2p_quant(sz[u] - fc.z + fc.w, qs), 0u);
                    } else {
                        sxy[tid + NT * u] = make_double2(sx[u], sy[u]);
                        szz[tid + NT * u] = sz[u];
                    }
                }
            __syncthreads();
            for (int q0 = ph < nph ? ph * blk : n; q0 < n; q0 += nph * blk) {
                const int q1 = min(n, q0 + blk);
                T px = 0, py = 0, pz = 0, pv = 0;
#pragma unroll 4
                for (int q = q0; q < q1; ++q) {
                    T dx, dy, dz;
                    if constexpr (sizeof(T) == 4) {
                        const uint4 v = sq[q];
                        dx = (float)(int32_t)(qx - v.x);
                        dy = (float)(int32_t)(qy - v.y);
                        dz = (float)(int32_t)(qz - v.z);
                    } else {
                        const double2 v = sxy[q];
                        dx = xi - v.x;
                        dy = yi - v.y;
                        dz = zi - szz[q];
                    }
                    // r = 0 (the target itself or a coincident ion) must give a
                    // finite 1/r^3, whose contribution is then exactly zero since
                    // dx = dy = dz = 0: r^2 carries a tiny offset (folded into
                    // the first FMA).  The potential has no such factor: there,
                    // pairs with r = 0 are left out.
                    T rinv = T(0), ww;
                    bool apart = true;
                    if constexpr (sizeof(T) == 4) {
                        const T r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, soft_q)));
                        rinv = __builtin_amdgcn_rsqf(r2);  // 1 ulp
                        ww = rinv * rinv * rinv;
                        if constexpr (POT) apart = r2 > soft_q;
                    } else {
                        // r^-3 = y0^3 (1 + 3/2 e + 15/8 e^2), r^-1 = y0 (1 + e/2 + 3/8 e^2),
                        // e = 1 - r2 y0^2, from the hardware estimate y0 (relative
                        // error about 5e-8), as in the direct sum
                        const T r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, kSoft2F64)));
                        const T y0 = __builtin_amdgcn_rsq(r2);
                        const T y2 = y0 * y0, y3 = y2 * y0;
                        const T e = fma(-r2, y2, 1.0);
                        ww = fma(y3, e * fma(e, 1.875, 1.5), y3);
                        if constexpr (POT) {
                            rinv = fma(y0 * e, fma(e, 0.375, 0.5), y0);
                            apart = r2 > kSoft2F64;
                        }
                    }
                    px += dx * ww;
                    py += dy * ww;
                    pz += dz * ww;
                    if constexpr (POT) pv += apart ? rinv : T(0);
                }
                if constexpr (sizeof(T) == 4) {
                    T y_ = px - cx, t_ = ax + y_;
                    cx = (t_ - ax) - y_;
                    ax = t_;
                    y_ = py - cy;
                    t_ = ay + y_;
                    cy = (t_ - ay) - y_;
                    ay = t_;
                    y_ = pz - cz;
                    t_ = az + y_;
                    cz = (t_ - az) - y_;
                    az = t_;
                    if constexpr (POT) {
                        y_ = pv - cv;
                        t_ = av + y_;
                        cv = (t_ - av) - y_;
                        av = t_;
                    }
                } else {
                    ax += px;
                    ay += py;
                    az += pz;
                    if constexpr (POT) av += pv;
                }
            }
            __syncthreads();  // all reads of the stage done before the next one
        }
        // phases 1.. hand their sums to phase 0, added in phase order
        hx[tid] = ax;
        hy[tid] = ay;
        hz[tid] = az;
        if constexpr (POT) hp[tid] = av;
        __syncthreads();
        if (ph == 0) {
            for (int h = 1; h < nph; ++h) {
                ax += hx[h * nt + ti];
                ay += hy[h * nt + ti];
                az += hz[h * nt + ti];
                if constexpr (POT) av += hp[h * nt + ti];
            }
            T *dst = part + ((size_t)it * 64 + ti) * NC;
            if constexpr (sizeof(T) == 4) {  // quanta back to metres
                ax *= back2;
                ay *= back2;
                az *= back2;
                if constexpr (POT) av *= back1;
            }
            dst[0] = ax;
            dst[1] = ay;
            dst[2] = az;
            if constexpr (POT) dst[3] = av;
        }
    }
}

// Far field (L2P) of every ion of a leaf plus its near-field item partials,
// added in item order.  Writes the field per unit charge in batch order; with
// POT also the potential per unit charge (sum 1/r) into PHI.  MODE 0 does
// both; MODE 1 only the far field (stored in E / PHI), so that it can run
// before the near field has finished; MODE 2 then adds the partials to the
// stored values.  The FP64 values and the order of the additions are the
// same in both ways.
template <typename T, bool POT, int MODE>
__global__ __launch_bounds__(256) void k_far(BoxTable bt, const double *__restrict__ sp, int ntot, int p, int Kp,
                                            const T *__restrict__ L, const T *__restrict__ rec,
                                            const uint32_t *__restrict__ item_off,
                                            const int32_t *__restrict__ src_items, const T *__restrict__ part,
                                            const uint32_t *__restrict__ vals, double *__restrict__ E,
                                            double *__restrict__ PHI, const TreeSummary *__restrict__ sum,
                                            int2 *__restrict__ poff)
{
    constexpr int NC = POT ? 4 : 3;
    __shared__ T rec_s[kRecFields * kq(kMaxP)];
    __shared__ T Lb[kMaxKp];
    const int b = blockIdx.x;
    if (sum->halt || b >= sum->nbox || !bt.leaf[b]) return;
    const double4 g = bt.geo[b];
    const double ih = 1.0 / g.w;
    if constexpr (MODE != 2) {
        for (int i = threadIdx.x; i < kRecFields * kq(p); i += blockDim.x) rec_s[i] = rec[i];
        for (int i = threadIdx.x; i < Kp; i += blockDim.x) Lb[i] = L[(size_t)b * Kp + i];
        __syncthreads();
    }
    const int si = src_items[b];
    const uint32_t base = item_off[b];
    for (int k = bt.begin[b] + threadIdx.x; k < bt.end[b]; k += blockDim.x) {
        const int tl = k - bt.begin[b];
        const int gi = (int)vals[k];
        double fx, fy, fz, fv = 0.0;
        if constexpr (MODE == 2) {
            fx = E[gi];
            fy = E[ntot + gi];
            fz = E[2 * ntot + gi];
            if constexpr (POT) fv = PHI[gi];
        } else {
            const double xd = sp[k], yd = sp[ntot + k], zd = sp[2 * ntot + k];
            T ex, ey, ez, ev = 0;
            const T ux = (T)((xd - g.x) * ih), uy = (T)((yd - g.y) * ih), uz = (T)((zd - g.z) * ih);
            if constexpr (POT) l2p_field_pot<T>(p, Lb, rec_s, ux, uy, uz, ex, ey, ez, ev);
            else l2p_field<T>(p, Lb, rec_s, ux, uy, uz, ex, ey, ez);
            fx = (double)ex * ih * ih;
            fy = (double)ey * ih * ih;
            fz = (double)ez * ih * ih;
            fv = (double)ev * ih;
        }
        if constexpr (MODE == 1)
            if (poff) poff[gi] = make_int2((int)((base + (tl >> 6) * si) * 64 + (tl & 63)), si);
        if constexpr (MODE != 1) {
            const T *pp = part + ((size_t)(base + (tl >> 6) * si) * 64 + (tl & 63)) * NC;
            for (int j = 0; j < si; ++j, pp += 64 * NC) {
                fx += (double)pp[0];
                fy += (double)pp[1];
                fz += (double)pp[2];
                if constexpr (POT) fv += (double)pp[3];
            }
        }
        E[gi] = fx;
        E[ntot + gi] = fy;
        E[2 * ntot + gi] = fz;
        if constexpr (POT) PHI[gi] = fv;
    }
}

// ---------------------------------------------------------------- launchers

static XlateArgs xlate_base(int Kp, int nbox)
{
    XlateArgs a{};
    a.nbucket = 1;
    a.ngroup = 1;
    a.nrowgrp = 1;
    a.Kp = Kp;
    a.nbox = nbox;
    return a;
}

// A level of M2M (mode 1) or L2L (mode 2): 8 octant slots, split into
// groups whose partial sums a second kernel adds in group order.  The
// level's boxes are read on the device; grids cover cap boxes (more boxes
// are still covered, by striding).
template <typename T>
static void launch_level_xlate(const BoxTable &bt, const TreeSummary *sum, int Kp, int nbox, int level, int cap,
                               int mode, const T *ops, const int2 *oct_slots, const int32_t *srctab, T *X, T *part,
                               bool narrow, hipStream_t st)
{
    const int tiles = std::max(1, ceil_div(cap, kM2LCols));
    XlateArgs a = xlate_base(Kp, nbox);
    a.lvl = sum->level_start;
    a.level = level;
    a.sum = sum;
    a.ngroup = 8;  // one octant slot per group: summation order independent of the batch
    a.tile_stride = tiles;
    a.slots = oct_slots;
    a.nslot = 8;
    a.srctab = srctab;
    a.src_stride = 8;
    a.mode = 0;
    xlate_rows(a, (long)tiles * a.ngroup, narrow);
    if (mode == 1) launch_xlate<T, 1>(a, tiles * a.ngroup * a.nrowgrp, ops, X, part, narrow, st);
    else launch_xlate<T, 2>(a, tiles * a.ngroup * a.nrowgrp, ops, X, part, narrow, st);
    const size_t tot = (size_t)std::max(1, cap) * Kp;
    k_xlate_reduce<T><<<(unsigned)std::min<size_t>((tot + 255) / 256, 8192), 256, 0, st>>>(
        sum, level, Kp, nbox, a.ngroup, mode, bt.leaf, part, X);
}

template <typename T>
void launch_p2m(const BoxTable &bt, const TreeSummary *sum, const double *sp, int ntot, int p, int nbox, const T *rec,
                T *M, int leaf_size, hipStream_t st)
{
    const int Kp = kpad(p);
    const int chunk = p2m_chunk<T>(Kp, leaf_size);
    const size_t smem = (size_t)Kp * (chunk + 1) * sizeof(T);
    if (nbox > 0) k_p2m<T><<<nbox, kP2MThreads, smem, st>>>(bt, sum, sp, ntot, p, Kp, chunk, rec, M);
}

template <typename T>
void launch_m2m(const BoxTable &bt, const TreeSummary *sum, int p, const Caps &cap, const T *m2m_pad,
                const int2 *oct_slots, const int32_t *child_oct, T *M, T *part, bool narrow, hipStream_t st)
{
    // level by level: parents of level l gather their children by octant
    const int Kp = kpad(p);
    for (int l = std::min(cap.nlev, kMaxLevel + 1) - 2; l >= 2; --l) {
        if (cap.lvl[l] <= 0 || cap.lvl[l + 1] <= 0) continue;  // no boxes, or no children below
        launch_level_xlate<T>(bt, sum, Kp, cap.nbox, l, cap.lvl[l], 1, m2m_pad, oct_slots, child_oct, M, part, narrow,
                              st);
    }
}

int m2l_groups(int)
{
    // M2M and L2L: one group per octant slot (8), a constant, so that the
    // summation order does not depend on the batch
    return 8;
}

template <typename T>
void launch_downward(const BoxTable &bt, const TreeSummary *sum, int p, const Caps &cap, const T *l2l_pad,
                     const int2 *oct_slots, const int32_t *parent_oct, const uint32_t *l2l_cnt,
                     const int32_t *l2l_list, T *L, bool narrow, hipStream_t st)
{
    const int Kp = kpad(p);
    // L2L level by level (3 and deeper): the level's boxes in 8 octant
    // buckets, so that every column of a tile shares its operator; each box
    // has exactly one source (its parent), so the product is added to L
    // directly.  A box's column is computed by the same instructions as with
    // 8 octant slot groups (where the 7 other groups read the zero row and add
    // exact zeros), so the result is the same.
    for (int l = 3; l < std::min(cap.nlev, kMaxLevel + 1); ++l) {
        if (cap.lvl[l] <= 0) continue;
        const int tiles = std::max(1, ceil_div(cap.lvl[l], kM2LCols));
        XlateArgs a = xlate_base(Kp, cap.nbox);
        a.cnt = (const int32_t *)l2l_cnt + 8 * l;
        a.list = l2l_list;
        a.list_stride = cap.nbox;
        a.nbucket = 8;
        a.lvl = sum->level_start;
        a.level = l;
        a.sum = sum;
        a.ngroup = 1;
        a.tile_stride = tiles;
        a.slots = oct_slots;  // bucket o: slot {octant o, operator o}
        a.nslot = 1;
        a.srctab = parent_oct;
        a.src_stride = 8;
        a.mode = 2;
        xlate_rows(a, (long)tiles * a.nbucket, narrow);
        launch_xlate<T, 2>(a, tiles * a.nbucket * a.nrowgrp, l2l_pad, L, L, narrow, st);
    }
}

template <typename T>
void launch_near(const BoxTable &bt, const TreeSummary *sum, const double *sp, int ntot, const int2 *near, int stride,
                 const int4 *work, const uint32_t *n_items, int cap_items, T *part, bool pot, int max_grid, int *queue,
                 const double *near_ext, hipStream_t st)
{
    if (cap_items <= 0) return;
    const int grid = std::min(cap_items, max_grid);
    if (pot)
        k_p2p<T, true>
            <<<grid, kP2PThreads, 0, st>>>(bt, sum, sp, ntot, near, stride, work, n_items, part, queue, near_ext);
    else
        k_p2p<T, false>
            <<<grid, kP2PThreads, 0, st>>>(bt, sum, sp, ntot, near, stride, work, n_items, part, queue, near_ext);
}

size_t near_lds_bytes()
{
    return sizeof(double2) * kP2PStage + sizeof(double) * kP2PStage + sizeof(int) * (2 * kNearMax + 3);
}

template <typename T>
void launch_far(const BoxTable &bt, const TreeSummary *sum, const double *sp, int ntot, int p, int nbox, const T *L,
                const T *rec, const uint32_t *item_off, const int32_t *src_items, const T *part, const uint32_t *vals,
                double *E, double *phi, int leaf_size, int mode, hipStream_t st, int2 *poff)
{
    // one thread per ion of a leaf where the leaf size allows
    const int tb = std::min(256, std::max(64, (leaf_size + 63) / 64 * 64));
    if (nbox <= 0) return;
#define PT_FAR(M)                                                                                                   \
    if (phi)                                                                                                        \
        k_far<T, true, M><<<nbox, tb, 0, st>>>(bt, sp, ntot, p, kpad(p), L, rec, item_off, src_items, part, vals, E, \
                                               phi, sum, nullptr);                                                  \
    else                                                                                                            \
        k_far<T, false, M><<<nbox, tb, 0, st>>>(bt, sp, ntot, p, kpad(p), L, rec, item_off, src_items, part, vals,  \
                                                E, nullptr, sum, poff);
    if (mode == 1) {
        PT_FAR(1)
    } else if (mode == 2) {
        PT_FAR(2)
    } else {
        PT_FAR(0)
    }
#undef PT_FAR
}

#define PT_INST(T)                                                                                                  \
    template void launch_p2m<T>(const BoxTable &, const TreeSummary *, const double *, int, int, int, const T *,     \
                                T *, int, hipStream_t);                                                            \
    template void launch_m2m<T>(const BoxTable &, const TreeSummary *, int, const Caps &, const T *, const int2 *,   \
                                const int32_t *, T *, T *, bool, hipStream_t);                                     \
    template void launch_downward<T>(const BoxTable &, const TreeSummary *, int, const Caps &, const T *,            \
                                     const int2 *, const int32_t *, const uint32_t *, const int32_t *, T *, bool,    \
                                     hipStream_t);                                                                 \
    template void launch_near<T>(const BoxTable &, const TreeSummary *, const double *, int, const int2 *, int,      \
                                 const int4 *, const uint32_t *, int, T *, bool, int, int *, const double *,       \
                                 hipStream_t);                                                                     \
    template void launch_far<T>(const BoxTable &, const TreeSummary *, const double *, int, int, int, const T *,     \
                                const T *, const uint32_t *, const int32_t *, const T *, const uint32_t *, double *, \
                                double *, int, int, hipStream_t, int2 *);
PT_INST(float)
PT_INST(double)
#undef PT_INST

}  // namespace pt
