// Launch wrappers of the HIP kernels (one translation unit per group).
#pragma once

#include "pt_common.hpp"

namespace pt {

// Box table of a batch, structure of arrays, boxes ordered by
// (level, crystal, Morton prefix).
struct BoxTable {
    int32_t *level, *crystal, *begin, *end, *parent, *child, *nchild, *ix, *iy, *iz;
    uint64_t *key;    // crystal << 3l | Morton prefix
    uint8_t *leaf;
    double4 *geo;     // centre xyz, side h
};

// M2L by base operator: operator slots (56 used), non-touching window slots
// per parity, and the slices of the operator totals (the counting
// workgroups' atomics spread over them)
constexpr int kM2LOps = 64;
constexpr int kM2LSlots = 189;
constexpr int kM2LOpSlices = 16;

// parity (ix & 1, iy & 1, iz & 1) of box b as a 3-bit number
__device__ inline int box_parity(const BoxTable &bt, int b)
{
    return ((bt.ix[b] & 1) << 2) | ((bt.iy[b] & 1) << 1) | (bt.iz[b] & 1);
}

// Workgroup scans (blockDim.x a multiple of 64).
// Exclusive scan of one value per thread; block_total gets the sum.  lds_w:
// blockDim.x / 64 + 1 words.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *lds_w, uint32_t &block_total)
{
    // inclusive wave scan, then wave totals through LDS
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds_w[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int k = 0; k < nw; ++k) {
            const uint32_t t = lds_w[k];
            lds_w[k] = run;
            run += t;
        }
        lds_w[nw] = run;
    }
    __syncthreads();
    block_total = lds_w[nw];
    return lds_w[w] + x - v;
}

// a[i] <- base + a[0] + ... + a[i-1] for i < n, in place, by one workgroup
// (rounds of kScanRound consecutive values per thread); returns the sum of
// the n values.  lds_w as above.
constexpr int kScanRound = 8;
__device__ inline uint32_t block_scan_inplace(uint32_t *__restrict__ a, int n, uint32_t base, uint32_t *lds_w)
{
    uint32_t carry = 0;
    for (int r0 = 0; r0 < n; r0 += (int)blockDim.x * kScanRound) {
        const int i0 = r0 + (int)threadIdx.x * kScanRound;
        uint32_t v[kScanRound], s = 0;
#pragma unroll
        for (int k = 0; k < kScanRound; ++k) {
            v[k] = i0 + k < n ? a[i0 + k] : 0u;
            s += v[k];
        }
        uint32_t tot;
        uint32_t run = base + carry + block_excl_scan(s, lds_w, tot);
#pragma unroll
        for (int k = 0; k < kScanRound; ++k) {
            if (i0 + k < n) a[i0 + k] = run;
            run += v[k];
        }
        carry += tot;
        __syncthreads();  // lds_w is reused by the next round
    }
    return carry;
}

// k_step.hip
void launch_ion_crystal(const CrystalDev *cs, int nc, int ntot, int32_t *ion_crystal, hipStream_t st);
// Bounding boxes: kBBoxCopies copies of [crystal][6] ordered-integer words,
// bbox_stride(nc) words apart (a multiple of 6 and of 128 bytes), so that the
// atomics of different workgroups spread over separate cache lines; the
// root cubes reduce the copies.  The buffer holds bbox_words(nc) words.
// launch_bbox_reset empties them; after an FMM evaluation's drift has filled
// them, its tree-level kernel empties them again (once every reader is done).
constexpr int kBBoxCopies = 16;
constexpr int bbox_stride(int nc) { return (6 * nc + 47) / 48 * 48; }
constexpr size_t bbox_words(int nc) { return (size_t)kBBoxCopies * bbox_stride(nc); }
void launch_bbox_reset(unsigned long long *bbox, int nc, hipStream_t st);

// Root cube of crystal c from its bounding-box copies, in the exact
// operation order of the tree contract: W = max extent (1e-9 m if zero),
// o = (lo + hi)/2 - W/2, S = 2^16 / W.
__device__ inline RootCube root_of(const unsigned long long *__restrict__ bbox, int bstride, int c)
{
#pragma clang fp contract(off)
    unsigned long long w[6];
    for (int k = 0; k < 6; ++k) w[k] = bbox[6 * c + k];
    for (int cp = 1; cp < kBBoxCopies; ++cp)
        for (int k = 0; k < 6; ++k) {
            const unsigned long long o = bbox[(size_t)cp * bstride + 6 * c + k];
            w[k] = k < 3 ? (o < w[k] ? o : w[k]) : (o > w[k] ? o : w[k]);
        }
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = ordered_to_dbl(w[d]);
        hi[d] = ordered_to_dbl(w[3 + d]);
    }
    double W = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double e = hi[d] - lo[d];
        if (e > W) W = e;
    }
    if (W == 0.0) W = 1e-9;
    RootCube r;
    for (int d = 0; d < 3; ++d) {
        const double ctr = 0.5 * (lo[d] + hi[d]);
        r.o[d] = ctr - 0.5 * W;
    }
    r.W = W;
    r.S = 65536.0 / W;
    r.pad[0] = r.pad[1] = r.pad[2] = 0.0;
    return r;
}
void launch_zero_u64(uint64_t *p, int n, hipStream_t st);
// Several small regions of 64-bit words (n[r] = 0: unused slot) zeroed in one launch.
constexpr int kZeroRegions = 4;
struct ZeroRegions {
    uint64_t *p[kZeroRegions];
    int n[kZeroRegions];
};
void launch_zero_regions(const ZeroRegions &z, hipStream_t st);
// halt (nullable, here and below): a run-state word; once set, nothing is
// done.  zr: 64-bit words zeroed on the way (for the kernels that follow).
void launch_drift_bbox(const CrystalDev *cs, const int32_t *ion_crystal, int ntot, int nc, int do_drift,
                       unsigned long long *bbox, const int32_t *halt, const ZeroRegions &zr, hipStream_t st);
// Root cubes of the nc crystals from the bounding boxes (which are left as
// they are).
void launch_roots(const unsigned long long *bbox, int nc, RootCube *roots, hipStream_t st);
// 64-bit sort key of batch ion g: its crystal index above a 48-bit Morton
// key of its position quantised to the crystal's root cube (floor((x - o) S),
// clamped to [0, 2^16 - 1]; subtract then multiply, never fused).
__device__ inline uint64_t ion_sort_key(const CrystalDev *__restrict__ cs, const int32_t *__restrict__ ion_crystal,
                                        const RootCube *__restrict__ roots, int g)
{
#pragma clang fp contract(off)
    const int c = ion_crystal[g];
    const CrystalDev &cd = cs[c];
    const int i = g - cd.ion_off;
    const int n = cd.n;
    const RootCube r = roots[c];
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
        double f = floor((cd.mid[d * n + i] - r.o[d]) * r.S);
        if (!(f >= 0.0)) f = 0.0;
        if (f > 65535.0) f = 65535.0;
        q[d] = (uint32_t)f;
    }
    return ((uint64_t)c << 48) | morton3(q[0], q[1], q[2]);
}
void launch_keys(const CrystalDev *cs, const int32_t *ion_crystal, const RootCube *roots, int ntot, uint64_t *keys,
                 uint32_t *vals, const int32_t *halt, hipStream_t st);
// beams: some crystal of the batch uses the beam-mode laser
// With sum non-null (the FMM), a halted run leaves the state as it was and
// records its first such step in sum->fail_step.
// call_k: the step's index within its pt_step_batch call (what fail_step records).
// next (nullable): the next step of the same batch follows; its first half
// drift is done by the same launch (as launch_drift_bbox with do_drift = 1:
// the working copy, the bounding boxes bbox of nc crystals, zr zeroed), and
// its evaluation then skips launch_drift_bbox.
struct NextDrift {
    unsigned long long *bbox;
    int nc;
    ZeroRegions zr;
};
// Near-field item partials the kick adds to E itself (in place of launch_far
// mode 2, with the same values and order of additions): part (FP32 when f32,
// else FP64; 3 components), and per ion (batch order) poff = {first partial
// row, number of source items}, the rows 64 apart.
struct KickPartials {
    const void *part;
    const int2 *poff;
    int f32;
};
// kp (nullable): E holds the far field only, and the kick adds the partials.
void launch_kick_drift(const CrystalDev *cs, const int32_t *ion_crystal, int ntot, int kstep, const double *E,
                       bool beams, TreeSummary *sum, int call_k, const NextDrift *next, const KickPartials *kp,
                       hipStream_t st);
// Direct field into E (3 x ntot); with phi non-null also the potential per
// unit charge sum_{j != i} 1/r_ij into phi (ntot).  tab: the nblk blocks of
// the batch (direct_chunks); part: the crystals' partials, 4 x chunks x n
// doubles per crystal from its dpart (3 x when phi is null).
void launch_direct(const CrystalDev *cs, const DirBlock *tab, int nblk, const int32_t *ion_crystal, int ntot,
                   double *part, double *E, double *phi, hipStream_t st);
// Ions per block of the sum block table (blk_crystal / blk_first) that the
// two per-crystal sums below go over.
int sum_ions_per_block();
// Per crystal c of the batch: out[c] = sum of phi over its ions (fixed order),
// over the sum block table; part: nblk doubles of workspace.
void launch_phi_sum(const CrystalDev *cs, const int32_t *blk_crystal, const int32_t *blk_first, int nblk, int nc,
                    const double *phi, double *part, double *out, hipStream_t st);
// Per crystal c: out[3c..3c+2] = rotating-frame axial KE, planar KE and the
// external terms of eq. (pe_rot), at the state's time (fixed order), over
// the sum block table; part: 3 x nblk doubles of workspace.
void launch_rot_sums(const CrystalDev *cs, const int32_t *blk_crystal, const int32_t *blk_first, int nblk, int nc,
                     double *part, double *out, hipStream_t st);
// Rotating-frame positions and velocities, SoA 6 x ntot in batch order.
void launch_rot_state(const CrystalDev *cs, const int32_t *ion_crystal, int ntot, double *out, hipStream_t st);

// k_tree.hip
int scan_partials(int n);  // workspace entries launch_scan needs for n elements
void launch_scan(uint32_t *a, int n, uint32_t *partial, uint32_t *total, hipStream_t st);
int sort_blocks(int n);
// Single-pass-per-digit radix sort of (k0, v0) by the 8-bit digits
// first..passes-1 (bits 8 first to 8 passes; passes <= 8), stable: with
// first = 0 and keys below 2^(8 passes) a full sort.  state holds
// radix_state_words(n) uint32 whose first radix_state_zero_words() must be
// zero on entry; the error word is state + radix_state_err().  Returns 1
// when the result is in (k1, v1), 0 when in (k0, v0), -1 when passes is out
// of range.
size_t radix_state_words(int n);
constexpr int radix_state_zero_words() { return 8 * 256 + 8 + 2; }
constexpr int radix_state_err() { return 8 * 256 + 8; }
// halt (nullable): a run-state word; when it is set the passes do nothing.
// keys (nullable): the sort keys are computed on the way (ion_sort_key of
// batch ion i into k0[i], v0[i] = i), in place of launch_roots and
// launch_keys: every workgroup makes the root cubes of the crystals of its
// tile out of the bounding boxes (bbox, nc) and writes them to roots (the
// same values, whichever workgroup writes).
struct KeySource {
    const CrystalDev *cs;
    const int32_t *ion_crystal;
    const unsigned long long *bbox;
    int nc;
    RootCube *roots;
};
int launch_radix_sort(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int n, int passes, int first,
                      uint32_t *state, const int32_t *halt, const KeySource *keys, hipStream_t st);
// After a stable sort by key >> shift: orders every run of equal key >> shift
// by (key, value), which completes the full sort, and gathers the sorted
// positions as launch_gather does.  A run longer than kRefineMax sets
// sum->refine_overflow and halts the run instead.
constexpr int kRefineMax = 32;
// Morton levels (3 bits each) by which the sort of a queued step orders
// before the runs are refined: whole 8-bit digits.
constexpr int kSortTopLevels = 8;
static_assert((3 * kSortTopLevels) % 8 == 0, "the top levels must fill whole digits");
void launch_sort_refine(uint64_t *keys, uint32_t *vals, int n, int shift, TreeSummary *sum, const CrystalDev *cs,
                        const int32_t *ion_crystal, double *sp, hipStream_t st);
void launch_radix_pass(const uint64_t *kin, const uint32_t *vin, uint64_t *kout, uint32_t *vout, int n, int shift,
                       uint32_t *hist, uint32_t *partial, hipStream_t st);
void launch_gather(const CrystalDev *cs, const int32_t *ion_crystal, const uint32_t *vals, int ntot, double *sp,
                   const int32_t *halt, hipStream_t st);
int tree_blocks(int ntot);
// box_end: ntot x (kMaxLevel + 1) ints, the end of every box at its first ion
// (filled by launch_tree_count, read by launch_tree_build).
// check (nullable): capacities the tree must fit, else the run halts (a
// queued step: the summary then halts the run).
// bbox (nc crystals): emptied on the way (the sort has read it).
void launch_tree_count(const CrystalDev *cs, const uint64_t *keys, int ntot, int leaf_size, uint32_t *rep_mask,
                       int32_t *box_end, uint32_t *blockcnt, uint32_t *partial, uint32_t *total,
                       const uint32_t *sort_err, TreeSummary *sum, const Caps *check, unsigned long long *bbox,
                       int nc, hipStream_t st);
// launch_tree_build writes the box table except its links (parent, child,
// nchild), which launch_lists adds.
void launch_tree_build(const CrystalDev *cs, const RootCube *roots, const uint64_t *keys, int ntot, int leaf_size,
                       const uint32_t *rep_mask, const int32_t *box_end, const uint32_t *scanned, const BoxTable &bt,
                       const TreeSummary *sum, int nbox, hipStream_t st);
// The tree links, the colleagues, the octant tables, the V and near lists.
// Also counts the near-field work items {leaf, first target, range begin,
// range end}: item_off (nbox, scanned in place to offsets), src_items (nbox),
// n_items (device total).  launch_p2p_items then writes them into work.
// Work counts: near_pairs (nbox) = near-field pairs per leaf.  near_ext
// (nbox, leaves only): the largest per-axis distance from a leaf's centre to
// a point of its near boxes.
// L2L buckets: the boxes of levels >= 3 by tree level and octant,
// l2l_list[o * nbox + level_start[l] + i] for i < l2l_cnt[8 l + o] (order
// within a bucket unspecified: every box's result is computed alone);
// l2l_cnt must be zero beforehand.
constexpr int kL2LCounts = 8 * (kMaxLevel + 1);
static_assert(kL2LCounts % 2 == 0, "L2L counts are cleared as 64-bit words");
// zr: 64-bit words to zero on the way (the first kernel clears them).
// item_off gets the item counts per leaf; launch_list_scans scans them.
// The V pairs are counted on the way: per box (pcnt, nbox) and per
// (operator, box) (cnt_ob, kM2LOps rows of the tree's box count), with the
// operator totals added into op_total (m2l_op_total_words() words, slices of
// kM2LOps, zero beforehand: one of the zr regions).  slots: per parity the
// kM2LSlots non-touching window slots {slot, base operator + 256 x
// reflection mask}.
void launch_lists(const BoxTable &bt, const TreeSummary *sum, int nbox, int32_t *coll, int32_t *vtab, int stride,
                  int2 *near, int32_t *near_cnt, int64_t *near_pairs, int32_t *child_oct, int32_t *parent_oct,
                  uint32_t *l2l_cnt, int32_t *l2l_list, const ZeroRegions &zr, uint32_t *item_off,
                  int32_t *src_items, int32_t *cuts, const int2 *slots, uint32_t *pcnt, uint32_t *cnt_ob,
                  uint32_t *op_total, double *near_ext, hipStream_t st);
// cuts (stride per box): first near range of each source item of a leaf.
// check (nullable, a queued evaluation): near-field items (total[1]) and M2L
// pairs (total[2]) must fit their capacities, else the run halts here and no
// item is written.
void launch_p2p_items(const BoxTable &bt, TreeSummary *sum, int nbox, const int32_t *near_cnt, int stride,
                      const uint32_t *item_off, const int32_t *src_items, const int32_t *cuts, int4 *work,
                      const uint32_t *total, const Caps *check, hipStream_t st);

// k_fmm.hip
// rec: recurrence table (fmm_math.hpp), kRecFields x kq(p) entries.
// m2m_pad / l2l_pad: 8 operators, Kp x Kp column-major, zero padded;
// oct_slots: the 8 slots {octant, octant}; child_oct / parent_oct: 8 x nbox.
// Every launcher below takes the device summary `sum`; its kernels do nothing
// once sum->halt is set.  Grids cover nbox = the box capacity (boxes past the
// tree's own count do nothing); level ranges and item counts are read on the
// device.
template <typename T>
void launch_p2m(const BoxTable &bt, const TreeSummary *sum, const double *sp, int ntot, int p, int nbox, const T *rec,
                T *M, int leaf_size, hipStream_t st);
// narrow: beside a near field of four or more workgroups per compute unit
// (mixed form), translation variants that need fewer registers (M2M and L2L).
template <typename T>
void launch_m2m(const BoxTable &bt, const TreeSummary *sum, int p, const Caps &cap, const T *m2m_pad,
                const int2 *oct_slots, const int32_t *child_oct, T *M, T *part, bool narrow, hipStream_t st);
int m2l_groups(int n2);  // slot groups of M2M / L2L partial sums (partial-sum buffer: groups x nbox x Kp)
// L2L, level by level: each box of an octant bucket adds its parent's local
// expansion shifted by its octant's operator (l2l_cnt / l2l_list as above).
template <typename T>
void launch_downward(const BoxTable &bt, const TreeSummary *sum, int p, const Caps &cap, const T *l2l_pad,
                     const int2 *oct_slots, const int32_t *parent_oct, const uint32_t *l2l_cnt,
                     const int32_t *l2l_list, T *L, bool narrow, hipStream_t st);
// Near field over the work items into part (item x 64 x 3; with pot the
// potential sum as a fourth component, item x 64 x 4); *n_items items (on the
// device, at most cap_items), at most max_grid workgroups, which take the
// items from *queue (zero before the launch) or, with queue NULL, stride over
// them.
template <typename T>
// near_ext: per leaf the half side of the frame of the mixed form's
// fixed-point coordinates (launch_lists).
void launch_near(const BoxTable &bt, const TreeSummary *sum, const double *sp, int ntot, const int2 *near, int stride,
                 const int4 *work, const uint32_t *n_items, int cap_items, T *part, bool pot, int max_grid, int *queue,
                 const double *near_ext, hipStream_t st);
// Near-field workgroups per compute unit while the far field runs beside the
// near field: with four, two M2L GEMM workgroups still fit in every compute
// unit's LDS, whichever kernel reaches the unit first.  When the near field
// forks before the upward pass (mixed form), three: the translation
// workgroups of the upward pass then also find registers beside it.
constexpr int kNearPerCUConcurrent = 4;
constexpr int kNearPerCUEarly = 3;
// LDS of one near-field workgroup (its staged sources and range tables).
size_t near_lds_bytes();
// Far field (L2P) + the item partials per ion into E (batch order); with phi
// non-null also the potential per unit charge (part then holds 4 components).
// mode 0: both; 1: the far field only (into E / phi); 2: adds the partials to
// what mode 1 stored (the same values as mode 0).  poff (nullable, mode 1):
// each ion's partial rows for a kick that adds them (KickPartials).
template <typename T>
void launch_far(const BoxTable &bt, const TreeSummary *sum, const double *sp, int ntot, int p, int nbox, const T *L,
                const T *rec, const uint32_t *item_off, const int32_t *src_items, const T *part, const uint32_t *vals,
                double *E, double *phi, int leaf_size, int mode, hipStream_t st, int2 *poff = nullptr);
// Starts a run: halt = 0, fail_step = -1.
void launch_run_reset(TreeSummary *sum, hipStream_t st);

// k_m2l.hip: M2L organised by base operator.
// slots: per parity the 189 non-touching window slots {slot, base operator +
// 256 x reflection mask (bit 0: dx < 0, bit 1: dy < 0, bit 2: dz < 0)}.
// launch_list_scans: one launch scans the list counts in place: pcnt -> first row of R per box
// (*npairs <- the number of V pairs), cnt_ob -> first bucket place per
// (operator, box), item_off (nbox item counts of the near field) -> first
// item per leaf (*n_items <- their number), and writes the operator table
// op_beg / chunk_off (m2l_ops() + 1 ints each: each operator's first bucket
// place and the prefix of its work-unit counts); *near_total <- the sum of
// the near-field pairs per leaf (near_pairs, nbox).
int m2l_ops();
int m2l_op_total_words();
void launch_list_scans(const TreeSummary *sum, int nbox, uint32_t *pcnt, uint32_t *cnt_ob, const uint32_t *op_total,
                       uint32_t *npairs, uint32_t *item_off, uint32_t *n_items, int32_t *op_beg, int32_t *chunk_off,
                       const int64_t *near_pairs, unsigned long long *near_total, hipStream_t st);
// bucket: npairs int4 {source box, row of R, reflection mask, 0}.
void launch_m2l_emit(const BoxTable &bt, const TreeSummary *sum, int nbox, const int32_t *vtab, const int2 *slots,
                     const uint32_t *pair_off, const uint32_t *ob_off, int4 *bucket, hipStream_t st);
// LDS of one GEMM workgroup: at most this much for the operator rows, and at
// most this many row blocks of 16 (compiled variants).  max_rb caps the row
// blocks further: kM2LSmallRowBlocks for batches whose near field outweighs
// M2L (three workgroups then fit a compute unit beside the near field),
// kM2LMaxRowBlocks otherwise (fewer operator reloads per product).
constexpr size_t kM2LLdsBudget = 48 << 10;
constexpr int kM2LMaxRowBlocks = 6;
constexpr int kM2LSmallRowBlocks = 3;
template <typename T>
size_t m2l_gemm_lds(int Kp, int max_rb);
// A: the 64 base operators, row-major Kp x Kp each (row = output coefficient),
// zero padded; M: nbox + 1 expansion rows (row nbox zero); R: npairs x Kp.
template <typename T>
void launch_m2l_gemm(const TreeSummary *sum, int Kp, int max_rb, int nbox, int grid, const int32_t *chunk_off,
                     const int32_t *op_beg, const int4 *bucket, const T *A, const T *M, T *R, hipStream_t st);
// L = per box the sum of its rows of R in order (pair_off: the scanned pcnt).
template <typename T>
void launch_m2l_sum(const TreeSummary *sum, int nbox, int Kp, const uint32_t *pair_off, const uint32_t *npairs,
                    const T *R, T *L, hipStream_t st);
// Persistent M2L workgroups per compute unit: as many as the LDS holds (at
// most kM2LMaxPerCU) next to lds_beside bytes taken by a kernel running
// beside it; the grid is sized to what can be resident, since the static
// split of the work would leave late-starting workgroups as a tail.
constexpr size_t kLdsPerCU = 160 << 10;
constexpr int kM2LMaxPerCU = 4;
template <typename T>
int m2l_per_cu(int Kp, int max_rb, size_t lds_beside);

// noalloc.hip: the fixed scratch of pt_compute_forces_noalloc (direct sum of
// one crystal of at most kNoAllocMaxIons ions).
constexpr int kNoAllocMaxIons = PT_NOALLOC_MAX_IONS;
constexpr size_t kNoAllocScratchBytes = (size_t)24 << 20;
// Byte offsets of its regions for n ions.
struct NoAllocLayout {
    size_t desc, bbox, ion_crystal, tab, mid, part, E, total;
    int nblk;
};
NoAllocLayout noalloc_layout(int n);
// The device address of this device's scratch (looked up once per device,
// with the device current).
pt_status noalloc_scratch(int device, void **out);
void launch_noalloc_setup(const CrystalDev &d, CrystalDev *desc, int32_t *ion_crystal, int n, DirBlock *tab, int nblk,
                          hipStream_t st);
void launch_scale_field(const double *E, int n, double s, double *F, hipStream_t st);

}  // namespace pt
