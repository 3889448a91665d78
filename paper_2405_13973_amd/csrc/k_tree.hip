// Morton sort, adaptive octree and interaction lists (Zaris et al., Sec. 2.3,
// "Algorithm": smallest enclosing cube, recursive octants, a box divided only
// when it holds more than leaf_size ions).
//
// Contract shared with the reference tree: ions sorted by (crystal, 48-bit
// key, batch index); boxes ordered by (level, crystal, Morton prefix); a box
// is split iff it holds more than leaf_size ions and its level is below 16;
// only non-empty children exist.
//
// Lists, for box B at level l with integer coordinates b:
//   colleagues  the (up to) 27 same-level boxes with |b' - b| <= 1 (B included)
//   V(B)        children of the parent's colleagues that do not touch B; they
//               are stored densely in a 6x6x6 window (index from the offset and
//               B's octant) so that targets of one octant share operators
//   near(T)     for a leaf T: the ion ranges of T's colleagues (leaf or not) and
//               of the leaf colleagues of T's ancestors -- every ion pair not
//               served by a multipole-to-local conversion
#include <type_traits>

#include "pt_common.hpp"
#include "pt_kernels.hpp"

namespace pt {

// --------------------------------------------------------------- scan

// Exclusive prefix sum of n uint32 in place: block sums of 8192-element
// chunks, then each chunk scanned with its offset, which each block adds up
// itself from the sums of the chunks before it (a few dozen at the sizes
// here); one chunk needs only the second launch.  *total (optional) gets the
// sum.  (block_excl_scan: pt_kernels.hpp.)
constexpr int kScanTB = 1024;
constexpr int kScanPer = 8;
constexpr int kScanChunk = kScanPer * kScanTB;

__global__ void k_set_u32(uint32_t *__restrict__ p, uint32_t v) { *p = v; }

__global__ __launch_bounds__(kScanTB) void k_scan_reduce(const uint32_t *__restrict__ a, int n,
                                                         uint32_t *__restrict__ partial)
{
    __shared__ uint32_t w[kScanTB / 64 + 1];
    const int base = blockIdx.x * kScanChunk + kScanPer * threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) s += base + k < n ? a[base + k] : 0u;
    uint32_t tot;
    block_excl_scan(s, w, tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__device__ void scan_down_chunk(uint32_t *__restrict__ a, int n, const uint32_t *__restrict__ partial,
                                uint32_t *__restrict__ total);

__global__ __launch_bounds__(kScanTB) void k_scan_down(uint32_t *__restrict__ a, int n,
                                                       const uint32_t *__restrict__ partial,
                                                       uint32_t *__restrict__ total)
{
    scan_down_chunk(a, n, partial, total);
}

__device__ void scan_down_chunk(uint32_t *__restrict__ a, int n, const uint32_t *__restrict__ partial,
                                uint32_t *__restrict__ total)
{
    __shared__ uint32_t w[kScanTB / 64 + 1];
    // offset of this chunk: the sum of the chunk sums before it
    uint32_t pre = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += kScanTB) pre += partial[i];
    uint32_t off;
    block_excl_scan(pre, w, off);
    __syncthreads();  // w is reused below
    const int base = blockIdx.x * kScanChunk + kScanPer * threadIdx.x;
    uint32_t v[kScanPer], s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < n ? a[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = off + block_excl_scan(s, w, tot);
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) a[base + k] = run;
        run += v[k];
    }
}

// --------------------------------------------------------------- radix sort

constexpr int kSortTB = 256;
constexpr int kSortItems = 4;
constexpr int kSortTile = kSortTB * kSortItems;
constexpr int kSortWideN = 400000;  // keys from which a pass takes 2 kSortItems keys per thread

__global__ __launch_bounds__(kSortTB) void k_radix_hist(const uint64_t *__restrict__ keys, int n, int shift,
                                                        uint32_t *__restrict__ hist, int nblk)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int r = 0; r < kSortItems; ++r) {
        const int i = blockIdx.x * kSortTile + r * kSortTB + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: items are ranked in tile order (round, wave, lane); equal
// digits within a wave are found with eight ballots.
__global__ __launch_bounds__(kSortTB) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                           const uint32_t *__restrict__ vin,
                                                           uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                           int n, int shift, const uint32_t *__restrict__ hist,
                                                           int nblk)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kSortTB / 64][256];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    base[tid] = hist[tid * nblk + blockIdx.x];
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortItems; ++r) {
        for (int k = 0; k < kSortTB / 64; ++k) wcnt[k][tid] = 0;
        __syncthreads();
        const int i = blockIdx.x * kSortTile + r * kSortTB + tid;
        const bool valid = i < n;
        const uint64_t key = valid ? kin[i] : 0ull;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const unsigned long long bb = __ballot(on);
            peers &= on ? bb : ~bb;
        }
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + rank;
            for (int k = 0; k < w; ++k) pos += wcnt[k][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int k = 0; k < kSortTB / 64; ++k) add += wcnt[k][tid];
        base[tid] += add;
        __syncthreads();
    }
}

// ------------------------------------------- single-pass-per-digit radix sort
//
// One kernel counts all digits of all passes over the keys (global digit
// histograms) and clears the look-back flags; then every pass is one kernel
// with decoupled look-back: a workgroup takes the next tile number from a
// counter (tiles are therefore numbered in the order their workgroups
// started, so every tile a workgroup waits for is already running), counts
// its tile's digits, publishes them, and adds up the counts published by the
// tiles before it (stopping at the first tile that has published its
// inclusive prefix), then publishes its own inclusive prefix and scatters.
// Ranking inside a tile is the stable order (round, wave, lane) of the
// multi-kernel sort above, so both sorts give the same result.  A bounded
// spin sets *err instead of waiting forever.
//
// Workspace (RadixState, radix_state_words): ghist[kMaxPasses][256] uint32,
// ctr[kMaxPasses] uint32, err uint32, then flags[kMaxPasses][ntile][256]
// uint64 (status in the top two bits, count below); ghist, ctr and err must
// be zero before k_radix_prepare.
constexpr int kMaxPasses = 8;
constexpr uint64_t kFlagAgg = 1ull << 62, kFlagIncl = 2ull << 62, kFlagCount = (1ull << 62) - 1;
constexpr int kSpinMax = 1 << 20;

// KEYS: the keys (and values) are computed here from the root cubes and
// written out, rather than read.
template <bool KEYS, int ITEMS>
__global__ __launch_bounds__(kSortTB) void k_radix_prepare(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                           KeySource src, int n, int passes, int first,
                                                           uint32_t *__restrict__ ghist,
                                                           uint64_t *__restrict__ flags, int ntile,
                                                           const int32_t *__restrict__ halt)
{
    if (halt && *halt) return;  // a halted run (every workgroup sees the same word)
    __shared__ uint32_t cnt[kMaxPasses][256];
    const int tid = threadIdx.x;
    for (int p = first; p < passes; ++p) {
        cnt[p][tid] = 0;
        flags[((size_t)p * ntile + blockIdx.x) * 256 + tid] = 0ull;
    }
    if constexpr (KEYS) {
        // the root cubes of the crystals of this tile (batch ions are in
        // crystal order), before any key of the tile needs them
        const int i0 = blockIdx.x * kSortTB * ITEMS, i1 = min(n, i0 + kSortTB * ITEMS) - 1;
        const int c0 = src.ion_crystal[i0], c1 = src.ion_crystal[i1];
        for (int c = c0 + tid; c <= c1; c += kSortTB) src.roots[c] = root_of(src.bbox, bbox_stride(src.nc), c);
    }
    __syncthreads();
    for (int r = 0; r < ITEMS; ++r) {
        const int i = (blockIdx.x * ITEMS + r) * kSortTB + tid;
        if (i < n) {
            uint64_t key;
            if constexpr (KEYS) {
                key = ion_sort_key(src.cs, src.ion_crystal, src.roots, i);
                keys[i] = key;
                vals[i] = (uint32_t)i;
            } else {
                key = keys[i];
            }
            for (int p = first; p < passes; ++p) atomicAdd(&cnt[p][(key >> (8 * p)) & 255u], 1u);
        }
    }
    __syncthreads();
    for (int p = first; p < passes; ++p)
        if (cnt[p][tid]) atomicAdd(&ghist[p * 256 + tid], cnt[p][tid]);
}

// Sorted position of slot k: that of batch ion g = vals[k].
__device__ inline void gather_slot(const CrystalDev *__restrict__ cs, const int32_t *__restrict__ ion_crystal,
                                   int ntot, double *__restrict__ sp, int k, uint32_t g)
{
    const CrystalDev &cd = cs[ion_crystal[g]];
    const int i = (int)g - cd.ion_off;
    sp[k] = cd.mid[i];
    sp[ntot + k] = cd.mid[cd.n + i];
    sp[2 * ntot + k] = cd.mid[2 * cd.n + i];
}

// Completes a stable sort by key >> shift: each run of equal key >> shift is
// ordered by (key, value) by the thread at its first slot (insertion sort;
// runs hold one or two slots at the sizes of interest).  The order a full
// sort gives -- by key, equal keys by value, values ascending on entry -- is
// what this produces, since the stable sort kept each run in value order.
// The same thread then gathers the sorted positions of its run's slots.
__global__ void k_sort_refine(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, int n, int shift,
                              TreeSummary *__restrict__ sum, const CrystalDev *__restrict__ cs,
                              const int32_t *__restrict__ ion_crystal, double *__restrict__ sp)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || sum->halt) return;
    const uint64_t run = keys[k] >> shift;
    if (k > 0 && (keys[k - 1] >> shift) == run) return;  // not the first slot of its run
    int e = k + 1;
    while (e < n && e - k <= kRefineMax && (keys[e] >> shift) == run) ++e;
    if (e - k > kRefineMax) {
        // plain stores: every writer writes 1
        sum->refine_overflow = 1;
        sum->halt = 1;
        return;
    }
    for (int i = k + 1; i < e; ++i) {
        const uint64_t kk = keys[i];
        const uint32_t vv = vals[i];
        int j = i - 1;
        while (j >= k && (keys[j] > kk || (keys[j] == kk && vals[j] > vv))) {
            keys[j + 1] = keys[j];
            vals[j + 1] = vals[j];
            --j;
        }
        keys[j + 1] = kk;
        vals[j + 1] = vv;
    }
    for (int i = k; i < e; ++i) gather_slot(cs, ion_crystal, n, sp, i, vals[i]);
}

template <int ITEMS>
__global__ __launch_bounds__(kSortTB) void k_radix_pass(const uint64_t *__restrict__ kin,
                                                        const uint32_t *__restrict__ vin,
                                                        uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                        int n, int pass, const uint32_t *__restrict__ ghist,
                                                        uint64_t *__restrict__ flags, int ntile,
                                                        uint32_t *__restrict__ ctr, uint32_t *__restrict__ err,
                                                        const int32_t *__restrict__ halt)
{
    if (halt && *halt) return;  // set before the sort starts: every workgroup returns, none waits
    constexpr int NW = kSortTB / 64;
    __shared__ uint32_t wcnt[ITEMS][NW][256];  // digit counts per (round, wave), then their prefixes
    __shared__ uint32_t base_s[256];
    __shared__ uint32_t lds_w[NW + 1];
    __shared__ int tile_s;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int shift = 8 * pass;
    if (tid == 0) tile_s = (int)atomicAdd(&ctr[pass], 1u);
    for (int r = 0; r < ITEMS; ++r)
        for (int q = 0; q < NW; ++q) wcnt[r][q][tid] = 0;
    __syncthreads();
    const int tile = tile_s;
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint64_t key[ITEMS];
    uint32_t val[ITEMS], dig[ITEMS];
    int rnk[ITEMS];
    bool ok[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int i = (tile * ITEMS + r) * kSortTB + tid;
        ok[r] = i < n;
        key[r] = ok[r] ? kin[i] : 0ull;
        val[r] = ok[r] ? vin[i] : 0u;
        dig[r] = (uint32_t)(key[r] >> shift) & 255u;
        unsigned long long peers = __ballot(ok[r]);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (dig[r] >> bit) & 1u;
            const unsigned long long bb = __ballot(on);
            peers &= on ? bb : ~bb;
        }
        rnk[r] = __popcll(peers & lt);
        if (ok[r] && rnk[r] == 0) wcnt[r][w][dig[r]] = (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // thread d: exclusive prefix of digit d over (round, wave), tile total
    uint32_t run = 0;
    for (int r = 0; r < ITEMS; ++r)
        for (int q = 0; q < NW; ++q) {
            const uint32_t c = wcnt[r][q][tid];
            wcnt[r][q][tid] = run;
            run += c;
        }
    const uint32_t mine = run;
    uint64_t *fl = flags + (size_t)pass * ntile * 256;
    // the count travels inside the flag word, so relaxed device-scope atomics
    // suffice (no other data is published)
    __hip_atomic_store(&fl[(size_t)tile * 256 + tid], (tile == 0 ? kFlagIncl : kFlagAgg) | mine, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    // look back over the earlier tiles
    uint64_t excl = 0;
    for (int t = tile - 1; t >= 0; --t) {
        uint64_t f = 0;
        int spins = 0;
        do {
            f = __hip_atomic_load(&fl[(size_t)t * 256 + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } while ((f >> 62) == 0 && ++spins < kSpinMax);
        if ((f >> 62) == 0) {
            atomicOr(err, 1u);
            break;
        }
        excl += f & kFlagCount;
        if ((f >> 62) == 2) break;
    }
    if (tile > 0)
        __hip_atomic_store(&fl[(size_t)tile * 256 + tid], kFlagIncl | (excl + mine), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    // first slot of digit d for this tile: keys of smaller digits + earlier tiles
    uint32_t tot;
    const uint32_t gex = block_excl_scan(ghist[pass * 256 + tid], lds_w, tot);
    base_s[tid] = gex + (uint32_t)excl;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
        if (ok[r]) {
            const uint32_t pos = base_s[dig[r]] + wcnt[r][w][dig[r]] + rnk[r];
            kout[pos] = key[r];
            vout[pos] = val[r];
        }
}

// Sorted positions: slot k takes the position of batch ion vals[k].
__global__ void k_gather(const CrystalDev *__restrict__ cs, const int32_t *__restrict__ ion_crystal,
                         const uint32_t *__restrict__ vals, int ntot, double *__restrict__ sp,
                         const int32_t *__restrict__ halt)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ntot || (halt && *halt)) return;
    gather_slot(cs, ion_crystal, ntot, sp, k, vals[k]);
}

// --------------------------------------------------------------- octree

// First level (1..kMaxLevel) at which two 48-bit Morton keys of one crystal
// differ, or kMaxLevel + 1 if they are equal.
__host__ __device__ inline int first_diff_level(uint64_t a, uint64_t b)
{
    const uint64_t x = (a ^ b) & 0xFFFFFFFFFFFFull;
    return x == 0 ? kMaxLevel + 1 : kMaxLevel - (63 - __builtin_clzll(x)) / 3;
}

// The levels at which sorted slot k is the first ion of a box (bit l), and the
// end of each such box (end[l]), for the crystal occupying [lo_c, hi_c).
//   - k starts a run of equal level-l prefixes for every l >= L, L the first
//     level where keys[k - 1] and keys[k] differ (0 at the crystal's start);
//   - that run is a box iff its parent run holds more than leaf ions (boxes
//     split iff they exceed leaf), which for l = L is decided within leaf
//     slots on either side of k, and for l > L (where the parent run starts
//     at k) by whether slot k + leaf shares k's level-(l - 1) prefix;
//   - a box's end is the first slot past k with a larger prefix.
__host__ __device__ inline uint32_t slot_box_levels(const uint64_t *__restrict__ keys, int k, int lo_c, int hi_c,
                                                    int leaf, int32_t *__restrict__ end)
{
    const uint64_t key = keys[k];
    int L = 0;
    if (k > lo_c) {
        L = first_diff_level(keys[k - 1], key);
        if (L > kMaxLevel) return 0u;
        // the level-(L - 1) run around k: [a, c) within [k - leaf, k + leaf]
        const int sh = 3 * (kMaxLevel - L + 1);
        const uint64_t pre = key >> sh;
        int a = k - leaf > lo_c ? k - leaf : lo_c, a1 = k - 1;  // first with prefix pre (k - 1 has it)
        int c = k + 1, c1 = hi_c < k + leaf + 1 ? hi_c : k + leaf + 1;  // first with a larger prefix, or c1
        while (a < a1 || c < c1) {
            if (a < a1) {
                const int m = (a + a1) >> 1;
                if ((keys[m] >> sh) < pre) a = m + 1;
                else a1 = m;
            }
            if (c < c1) {
                const int m = (c + c1) >> 1;
                if ((keys[m] >> sh) <= pre) c = m + 1;
                else c1 = m;
            }
        }
        if (c - a <= leaf) return 0u;  // the parent is a leaf (or k is inside one)
    }
    // deeper levels: boxes down to D, the first level where keys[k + leaf] differs
    const int D = k + leaf < hi_c ? first_diff_level(key, keys[k + leaf]) : 0;
    const int lmax = D > L ? (D < kMaxLevel ? D : kMaxLevel) : L;
    uint32_t mask = 0u;
    int bound = hi_c;
    for (int l = L; l <= lmax; ++l) {
        mask |= 1u << l;
        if (l == 0) {
            end[0] = hi_c;
            continue;
        }
        // the run holds slot k + leaf for l < D, not for l >= D
        const int sh = 3 * (kMaxLevel - l);
        const uint64_t pre = key >> sh;
        int c = l < D ? k + leaf + 1 : k + 1;
        int c1 = l < D ? bound : (bound < k + leaf ? bound : k + leaf);
        // wide ranges (the large boxes' representatives, the kernel's longest
        // chains): 8-way steps, 7 probes loaded at once; then bisection
        while (c1 - c > 64) {
            const int st = (c1 - c + 7) / 8;
            uint64_t pk[7];
#pragma unroll
            for (int i = 0; i < 7; ++i) pk[i] = keys[c + (i + 1) * st - 1];  // all < c1
            int nf = 0;
#pragma unroll
            for (int i = 0; i < 7; ++i) nf += (pk[i] >> sh) <= pre;
            const int c0 = c;
            c = c0 + nf * st;
            if (nf < 7) c1 = c0 + (nf + 1) * st - 1;
        }
        while (c < c1) {
            const int m = (c + c1) >> 1;
            if ((keys[m] >> sh) <= pre) c = m + 1;
            else c1 = m;
        }
        end[l] = c;
        bound = c;
    }
    return mask;
}

// The tree summary from the scanned per-level counts (one thread): level
// starts, box count, sort error; a queued step also checks the tree against
// its capacities.
__device__ void tree_summary(const uint32_t *__restrict__ scanned, int nblk, uint32_t nbox_total,
                             const uint32_t *__restrict__ sort_err, TreeSummary *__restrict__ sum, const Caps &cap,
                             int check)
{
    if (sum->halt) return;
    const int32_t err = sort_err ? (int32_t)*sort_err : 0;
    sum->sort_error = err;
    int nlev = 0;
    for (int l = 0; l <= kMaxLevel; ++l) {
        sum->level_start[l] = (int32_t)scanned[l * nblk];
        if (l > 0 && sum->level_start[l] > sum->level_start[l - 1]) nlev = l;
    }
    const int32_t nbox = (int32_t)nbox_total;
    sum->level_start[kMaxLevel + 1] = nbox;
    sum->nbox = nbox;
    if (nbox > sum->level_start[kMaxLevel]) nlev = kMaxLevel + 1;
    // a queued step: boxes and levels must fit the capacities (a level
    // holding more boxes than its grid covers is still covered, by striding;
    // only the buffers sized by these counts can overflow), and the sort
    // must have finished
    if (check && (nbox > cap.nbox || nlev > cap.nlev || err != 0)) sum->halt = 1;
}

// For every sorted slot: the levels at which it is the first ion of an
// existing box (bit l of rep_mask).
__global__ __launch_bounds__(256) void k_tree_levels(const CrystalDev *__restrict__ cs,
                                                     const uint64_t *__restrict__ keys, int ntot, int leaf_size,
                                                     uint32_t *__restrict__ rep_mask, int32_t *__restrict__ box_end,
                                                     uint32_t *__restrict__ blockcnt, int nblk,
                                                     const int32_t *__restrict__ halt,
                                                     unsigned long long *__restrict__ bbox, int bbox_n)
{
    if (halt && *halt) return;
    // the bounding boxes are read: emptied for the next drift (grid-stride)
    for (int i = blockIdx.x * 256 + threadIdx.x; i < bbox_n; i += gridDim.x * 256) bbox[i] = (i % 6) < 3 ? ~0ull : 0ull;
    // rep_mask[k]: the levels at which slot k is the first ion of a box;
    // box_end[k][l]: the end of that level-l box (written for those levels only);
    // blockcnt[l][block]: how many such slots of this block start a level-l box
    __shared__ uint32_t wc[4][kMaxLevel + 1];
    const int k = blockIdx.x * 256 + threadIdx.x;
    uint32_t mask = 0u;
    if (k < ntot) {
        const int c = (int)(keys[k] >> 48);
        const int lo = cs[c].ion_off;
        mask = slot_box_levels(keys, k, lo, lo + cs[c].n, leaf_size, box_end + (size_t)k * (kMaxLevel + 1));
        rep_mask[k] = mask;
    }
    const int w = threadIdx.x >> 6;
    for (int l = 0; l <= kMaxLevel; ++l) {
        const int cnt = __popcll(__ballot((mask >> l) & 1u));
        if ((threadIdx.x & 63) == 0) wc[w][l] = (uint32_t)cnt;
    }
    __syncthreads();
    if (threadIdx.x <= kMaxLevel)
        blockcnt[threadIdx.x * nblk + blockIdx.x] = wc[0][threadIdx.x] + wc[1][threadIdx.x] + wc[2][threadIdx.x] +
                                                    wc[3][threadIdx.x];
}

__global__ void k_tree_summary(const uint32_t *__restrict__ scanned, int nblk, const uint32_t *__restrict__ total,
                               const uint32_t *__restrict__ sort_err, TreeSummary *__restrict__ sum, Caps cap,
                               int check)
{
    if (threadIdx.x == 0) tree_summary(scanned, nblk, *total, sort_err, sum, cap, check);
}

// The per-level counts in one scan chunk: scanned in place by one
// workgroup, whose first thread then writes the summary (the scanned counts
// and the total are this workgroup's own writes).
__global__ __launch_bounds__(kScanTB) void k_scan_tree_summary(uint32_t *__restrict__ a, int nblk,
                                                               uint32_t *__restrict__ total,
                                                               const uint32_t *__restrict__ sort_err,
                                                               TreeSummary *__restrict__ sum, Caps cap, int check)
{
    scan_down_chunk(a, (kMaxLevel + 1) * nblk, nullptr, total);
    __syncthreads();
    if (threadIdx.x == 0) tree_summary(a, nblk, *total, sort_err, sum, cap, check);
}

// Writes one box record per (slot, level) representative.
__global__ __launch_bounds__(256) void k_tree_emit(const CrystalDev *__restrict__ cs,
                                                   const RootCube *__restrict__ roots,
                                                   const uint64_t *__restrict__ keys, int ntot, int leaf_size,
                                                   const uint32_t *__restrict__ rep_mask,
                                                   const int32_t *__restrict__ box_end,
                                                   const uint32_t *__restrict__ scanned, int nblk, BoxTable bt,
                                                   const TreeSummary *__restrict__ sum)
{
    __shared__ uint32_t wc[4][kMaxLevel + 1];
    if (sum->halt) return;
    const int k = blockIdx.x * 256 + threadIdx.x;
    const uint32_t mask = k < ntot ? rep_mask[k] : 0u;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long lt = (1ull << lane) - 1ull;
    int rank[kMaxLevel + 1];
    for (int l = 0; l <= kMaxLevel; ++l) {
        const unsigned long long b = __ballot((mask >> l) & 1u);
        rank[l] = __popcll(b & lt);
        if (lane == 0) wc[w][l] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    if (mask == 0) return;
    const uint64_t key = keys[k];
    const int c = (int)(key >> 48);
    const RootCube rc = roots[c];
    const int lo = k;  // the box starts at its representative
    for (int l = 0; l <= kMaxLevel; ++l) {
        if (!((mask >> l) & 1u)) continue;
        const int hi = box_end[(size_t)k * (kMaxLevel + 1) + l];
        uint32_t idx = scanned[l * nblk + blockIdx.x] + (uint32_t)rank[l];
        for (int q = 0; q < w; ++q) idx += wc[q][l];
        const int sh = 3 * (kMaxLevel - l);
        const uint64_t mort = (key & 0xFFFFFFFFFFFFull) >> sh;
        const uint32_t ix = compact3_16(mort >> 2), iy = compact3_16(mort >> 1), iz = compact3_16(mort);
        const double h = ldexp(rc.W, -l);
        bt.level[idx] = l;
        bt.crystal[idx] = c;
        bt.key[idx] = key >> sh;
        bt.begin[idx] = lo;
        bt.end[idx] = hi;
        bt.ix[idx] = (int32_t)ix;
        bt.iy[idx] = (int32_t)iy;
        bt.iz[idx] = (int32_t)iz;
        bt.leaf[idx] = (hi - lo <= leaf_size || l == kMaxLevel) ? 1 : 0;
        bt.geo[idx] = make_double4(rc.o[0] + ((double)ix + 0.5) * h, rc.o[1] + ((double)iy + 0.5) * h,
                                   rc.o[2] + ((double)iz + 0.5) * h, h);
    }
}

// Parent / children of box b by binary search over the neighbouring levels
// (boxes of one level are ordered by their first ion), written to the box
// table and returned.
__device__ inline void box_links(BoxTable bt, const TreeSummary *__restrict__ sum, int b, int &parent_out,
                                 int &child_out, int &nch_out)
{
    const int l = bt.level[b];
    const int beg = bt.begin[b];
    int parent = -1;
    if (l > 0) {
        int lo = sum->level_start[l - 1], hi = sum->level_start[l] - 1;  // last with begin <= beg
        while (lo < hi) {
            const int m = (lo + hi + 1) >> 1;
            if (bt.begin[m] <= beg) lo = m;
            else hi = m - 1;
        }
        parent = lo;
    }
    bt.parent[b] = parent;
    int child = -1, nch = 0;
    if (!bt.leaf[b] && l < kMaxLevel) {
        int lo = sum->level_start[l + 1], hi = sum->level_start[l + 2];
        int a = lo, e = hi;
        while (a < e) {  // first with begin >= beg
            const int m = (a + e) >> 1;
            if (bt.begin[m] < beg) a = m + 1;
            else e = m;
        }
        child = a;
        const int end = bt.end[b];
        int c2 = a, e2 = hi;
        while (c2 < e2) {  // first with begin >= end
            const int m = (c2 + e2) >> 1;
            if (bt.begin[m] < end) c2 = m + 1;
            else e2 = m;
        }
        nch = c2 - a;
    }
    bt.child[b] = child;
    bt.nchild[b] = nch;
    parent_out = parent;
    child_out = child;
    nch_out = nch;
}

// The links of box b (box_links) and the source maps of the M2M / L2L
// translation GEMMs, 8 slots per box indexed by octant: child_oct[b][o] =
// child of b in octant o, parent_oct[b][o] = parent of b in b's own octant
// slot (-1 elsewhere); and the L2L buckets (boxes of levels >= 3 by level and
// octant, l2l_cnt zeroed beforehand).  Thread b of nthreads (b: the box); the
// regions of zr are zeroed on the way (grid-stride over the nthreads).
__device__ void links_oct_tables(BoxTable bt, const TreeSummary *__restrict__ sum, int32_t *__restrict__ child_oct,
                                 int32_t *__restrict__ parent_oct, uint32_t *__restrict__ l2l_cnt,
                                 int32_t *__restrict__ l2l_list, int list_stride, const ZeroRegions &zr, int b,
                                 int nthreads)
{
    for (int r = 0; r < kZeroRegions; ++r)  // words the later kernels need zeroed
        for (int i = b; i < zr.n[r]; i += nthreads) zr.p[r][i] = 0ull;
    if (sum->halt || b >= sum->nbox) return;
    int parent, child, nch;
    box_links(bt, sum, b, parent, child, nch);
    int32_t ch[8], pa[8];
    for (int o = 0; o < 8; ++o) ch[o] = pa[o] = -1;
    for (int c = child, e = child + nch; c < e; ++c)
        ch[((bt.ix[c] & 1) << 2) | ((bt.iy[c] & 1) << 1) | (bt.iz[c] & 1)] = c;
    const int oct = ((bt.ix[b] & 1) << 2) | ((bt.iy[b] & 1) << 1) | (bt.iz[b] & 1);
    pa[oct] = parent;
    for (int o = 0; o < 8; ++o) {
        child_oct[(size_t)b * 8 + o] = ch[o];
        parent_oct[(size_t)b * 8 + o] = pa[o];
    }
    const int l = bt.level[b];
    if (l >= 3) {
        const uint32_t i = atomicAdd(&l2l_cnt[8 * l + oct], 1u);
        l2l_list[(size_t)oct * list_stride + sum->level_start[l] + i] = b;
    }
}

// Same-level neighbours (offsets in [-1,1]^3, slot (dx+1)*9 + (dy+1)*3 + (dz+1)),
// one thread per (box, slot): a binary search of the level's sorted keys.
__device__ void colleagues(BoxTable bt, const TreeSummary *__restrict__ sum, int32_t *__restrict__ coll, int i)
{
    const int nbox = sum->nbox;
    if (sum->halt || i >= nbox * kNeigh) return;
    const int b = i / kNeigh, s = i - b * kNeigh;
    const int l = bt.level[b];
    const int lim = 1 << l;
    const int nx = bt.ix[b] + s / 9 - 1, ny = bt.iy[b] + (s / 3) % 3 - 1, nz = bt.iz[b] + s % 3 - 1;
    int found = -1;
    if (s == 13) {
        found = b;
    } else if (nx >= 0 && ny >= 0 && nz >= 0 && nx < lim && ny < lim && nz < lim) {
        const uint64_t want = ((uint64_t)bt.crystal[b] << (3 * l)) | morton3(nx, ny, nz);
        const int l1 = sum->level_start[l + 1];
        int a = sum->level_start[l], e = l1;
        while (a < e) {
            const int m = (a + e) >> 1;
            if (bt.key[m] < want) a = m + 1;
            else e = m;
        }
        if (a < l1 && bt.key[a] == want) found = a;
    }
    coll[i] = found;
}

// Colleagues (the first ncb workgroups, one thread per (box, slot)) and the
// links with the octant tables (the rest, one thread per box) in one launch:
// both read only the box table the tree emitter wrote (the links of a box are
// computed by its own thread before its octant tables use them).
__global__ __launch_bounds__(256) void k_oct_colleagues(BoxTable bt, const TreeSummary *__restrict__ sum,
                                                        int32_t *__restrict__ coll, int ncb,
                                                        int32_t *__restrict__ child_oct,
                                                        int32_t *__restrict__ parent_oct,
                                                        uint32_t *__restrict__ l2l_cnt,
                                                        int32_t *__restrict__ l2l_list, int list_stride, ZeroRegions zr)
{
    if ((int)blockIdx.x < ncb) {
        colleagues(bt, sum, coll, blockIdx.x * 256 + threadIdx.x);
        return;
    }
    links_oct_tables(bt, sum, child_oct, parent_oct, l2l_cnt, l2l_list, list_stride, zr,
                     ((int)blockIdx.x - ncb) * 256 + threadIdx.x, ((int)gridDim.x - ncb) * 256);
}

// Near lists of the leaves: ion ranges, stride entries per box.  The near
// field of a leaf is then cut into work items of at most kP2PChunk sources
// (cut at range boundaries) times chunks of 64 targets, so that no single
// workgroup carries a coarse boundary leaf with thousands of near sources.
__device__ inline int p2p_src_items(const int2 *row, int cnt, int32_t *cut)
{
    int items = 0, acc = 0;
    for (int r = 0; r < cnt; ++r) {
        const int len = row[r].y - row[r].x;
        if (acc > 0 && acc + len > kP2PChunk) {
            ++items;
            acc = 0;
        }
        if (acc == 0) cut[items] = r;  // first range of source item `items`
        acc += len;
    }
    return items + (acc > 0 ? 1 : 0);
}

// The lists of one box, one workgroup of 256 threads per box.
//
// V list into the dense window table (-1 = no source), one thread per window
// cell.  Window cell (wx, wy, wz) of a box with parity (cx, cy, cz) is the
// same-level box at offset (wx-2-cx, wy-2-cy, wz-2-cz); its parent is the
// colleague of the box's parent in slot (wx>>1, wy>>1, wz>>1) and it sits in
// that parent's octant (wx&1, wy&1, wz&1).  Cells touching the box are not in
// the list.  Its V pairs are then counted in total (pcnt) and per base
// operator (cnt_ob, a row per operator), the operator totals added into one
// of the kM2LOpSlices slices of op_total.
//
// Near list of a leaf (the first wave): ion ranges, stride entries per box,
// appended in a fixed order -- the leaf's own colleagues (slot order, itself
// included), then the leaf colleagues of each ancestor from the parent up
// (slot order, the ancestor itself excluded) -- compacted with ballots,
// staged in LDS and written out coalesced; then its near-field work items
// are counted, and near_ext gets the largest per-axis distance from the
// leaf's centre to a point of its near boxes (the frame of the mixed near
// field's fixed-point coordinates).
__global__ __launch_bounds__(256) void k_box_lists(BoxTable bt, const TreeSummary *__restrict__ sum,
                                                   const int32_t *__restrict__ coll,
                                                   const int32_t *__restrict__ child_oct, int32_t *__restrict__ vtab,
                                                   const int2 *__restrict__ slots, uint32_t *__restrict__ pcnt,
                                                   uint32_t *__restrict__ cnt_ob, uint32_t *__restrict__ op_total,
                                                   int stride, int2 *__restrict__ near, int32_t *__restrict__ near_cnt,
                                                   uint32_t *__restrict__ items, int32_t *__restrict__ src_items,
                                                   int32_t *__restrict__ cuts, int64_t *__restrict__ pairs,
                                                   double *__restrict__ near_ext)
{
    __shared__ int32_t win_s[kWin];
    __shared__ uint32_t per_op[kM2LOps];
    __shared__ uint32_t vtot_s;
    __shared__ int2 row_s[kNearMax];
    __shared__ int anc_s[kMaxLevel + 1];
    __shared__ int nanc_s;
    const int b = blockIdx.x, tid = threadIdx.x;
    if (sum->halt) return;
    // the grid may cover more boxes than the tree has (a capacity): those
    // count no V pairs and no items, so that the scans of the counts stay exact
    if (b >= sum->nbox) {
        if (tid == 0) {
            pcnt[b] = 0;
            near_cnt[b] = 0;
            items[b] = 0;
            src_items[b] = 0;
            pairs[b] = 0;
        }
        return;
    }
    const bool v_box = bt.level[b] >= 2, leaf = bt.leaf[b];
    if (tid < kWin) {
        const int w = tid;
        int src = -1;
        if (v_box) {
            const int wx = w / 36, wy = (w / 6) % 6, wz = w % 6;
            const int dx = wx - 2 - (bt.ix[b] & 1), dy = wy - 2 - (bt.iy[b] & 1), dz = wz - 2 - (bt.iz[b] & 1);
            if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) {
                const int Q = coll[(size_t)bt.parent[b] * kNeigh + (wx >> 1) * 9 + (wy >> 1) * 3 + (wz >> 1)];
                if (Q >= 0) src = child_oct[(size_t)Q * 8 + (((wx & 1) << 2) | ((wy & 1) << 1) | (wz & 1))];
            }
        }
        vtab[(size_t)b * kWin + w] = src;
        win_s[w] = src;
    }
    if (tid < kM2LOps) per_op[tid] = 0;
    if (tid == 0) {
        vtot_s = 0;
        int n = 0;
        if (leaf)
            for (int A = bt.parent[b]; A >= 0 && n <= kMaxLevel; A = bt.parent[A]) anc_s[n++] = A;
        nanc_s = n;
    }
    __syncthreads();
    if (v_box && tid < kM2LSlots) {
        const int2 sl = slots[box_parity(bt, b) * kM2LSlots + tid];
        if (win_s[sl.x] >= 0) {
            atomicAdd(&per_op[sl.y & 255], 1u);
            atomicAdd(&vtot_s, 1u);
        }
    }
    // the near list, in the first wave (its ballots are the wave's)
    const int lane = tid & 63;
    int cnt = 0;
    long long srcs = 0;
    double ext = 0.0;  // largest per-axis distance from b's centre to a point of a near box
    if (leaf && tid < 64) {
        const int nanc = nanc_s;
        const uint64_t below = (1ull << lane) - 1ull;
        const double4 gb = bt.geo[b];
        auto append = [&](int Q) {
            const bool v = Q >= 0;
            const uint64_t m = __ballot(v);
            const int at = cnt + __popcll(m & below);
            if (v && at < kNearMax) {
                const int2 rg = make_int2(bt.begin[Q], bt.end[Q]);
                row_s[at] = rg;
                srcs += rg.y - rg.x;
                const double4 gq = bt.geo[Q];
                ext = fmax(ext, fmax(fmax(fabs(gq.x - gb.x), fabs(gq.y - gb.y)), fabs(gq.z - gb.z)) + 0.5 * gq.w);
            }
            cnt += __popcll(m);
        };
        append(lane < kNeigh ? coll[(size_t)b * kNeigh + lane] : -1);
        for (int a0 = 0; a0 < nanc; a0 += 2) {
            const int a = a0 + (lane >> 5), s = lane & 31;
            int Q = -1;
            if (a < nanc && s < kNeigh && s != 13) {
                Q = coll[(size_t)anc_s[a] * kNeigh + s];
                if (Q >= 0 && !bt.leaf[Q]) Q = -1;
            }
            append(Q);
        }
        cnt = min(cnt, min(stride, kNearMax));  // stride = 27 + 26 x (levels - 1) bounds cnt
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            srcs += __shfl_xor(srcs, off);
            ext = fmax(ext, __shfl_xor(ext, off));
        }
    }
    __syncthreads();
    if (tid < kM2LOps) {
        cnt_ob[(size_t)tid * sum->nbox + b] = per_op[tid];
        if (per_op[tid]) atomicAdd(&op_total[(b % kM2LOpSlices) * kM2LOps + tid], per_op[tid]);  // integer sums
    }
    if (tid == 0) pcnt[b] = vtot_s;
    if (tid < 64) {
        if (!leaf) {
            if (tid == 0) {
                near_cnt[b] = 0;
                items[b] = 0;
                src_items[b] = 0;
                pairs[b] = 0;
            }
            return;
        }
        int2 *row = near + (size_t)b * stride;
        for (int r = lane; r < cnt; r += 64) row[r] = row_s[r];
        if (lane == 0) {
            near_cnt[b] = cnt;
            const long long nt = bt.end[b] - bt.begin[b];
            const int si = p2p_src_items(row_s, cnt, cuts + (size_t)b * stride);
            src_items[b] = si;
            items[b] = (uint32_t)(si * ((nt + 63) / 64));
            pairs[b] = nt * srcs - nt;  // near-field pairs of the leaf (self excluded)
            near_ext[b] = ext;
        }
    }
}

// Work items {leaf, first target, first range, end range} at the scanned
// offsets, one wave per leaf: item tc * si + j pairs target chunk tc with
// source item j (ranges cut[j] .. cut[j + 1]).
__global__ __launch_bounds__(64) void k_p2p_items(BoxTable bt, TreeSummary *__restrict__ sum,
                                                  const int32_t *__restrict__ near_cnt, int stride,
                                                  const uint32_t *__restrict__ item_off,
                                                  const int32_t *__restrict__ src_items,
                                                  const int32_t *__restrict__ cuts, int4 *__restrict__ work,
                                                  const uint32_t *__restrict__ total, Caps cap, int check)
{
    const int b = blockIdx.x;
    if (sum->halt) return;
    // a queued step: items and M2L pairs must fit their capacities; every
    // workgroup reads the same counts, so none writes past the buffers (plain
    // stores: every writer writes 1)
    if (check && (total[1] > (uint32_t)cap.items || total[2] > (uint32_t)cap.pairs)) {
        if (threadIdx.x == 0) sum->halt = 1;
        return;
    }
    if (b >= sum->nbox || !bt.leaf[b]) return;
    const int32_t *cut = cuts + (size_t)b * stride;
    const int cnt = near_cnt[b], si = src_items[b];
    const int nt = bt.end[b] - bt.begin[b];
    const uint32_t w0 = item_off[b];
    for (int j = threadIdx.x; j < si; j += 64) {
        const int r0 = cut[j], r1 = j + 1 < si ? cut[j + 1] : cnt;
        for (int tc = 0; tc * 64 < nt; ++tc) work[w0 + tc * si + j] = make_int4(b, bt.begin[b] + 64 * tc, r0, r1);
    }
}

// ---------------------------------------------------------------- launchers

int scan_partials(int n) { return ceil_div(n, kScanChunk); }

void launch_scan(uint32_t *a, int n, uint32_t *partial, uint32_t *total, hipStream_t st)
{
    if (n <= 0) {
        if (total) k_set_u32<<<1, 1, 0, st>>>(total, 0u);
        return;
    }
    const int nb = scan_partials(n);
    if (nb > 1) k_scan_reduce<<<nb, kScanTB, 0, st>>>(a, n, partial);  // one chunk reads no partials
    k_scan_down<<<nb, kScanTB, 0, st>>>(a, n, partial, total);
}

int sort_blocks(int n) { return ceil_div(n, kSortTile); }

void launch_radix_pass(const uint64_t *kin, const uint32_t *vin, uint64_t *kout, uint32_t *vout, int n, int shift,
                       uint32_t *hist, uint32_t *partial, hipStream_t st)
{
    const int nblk = sort_blocks(n);
    k_radix_hist<<<nblk, kSortTB, 0, st>>>(kin, n, shift, hist, nblk);
    launch_scan(hist, 256 * nblk, partial, nullptr, st);
    k_radix_scatter<<<nblk, kSortTB, 0, st>>>(kin, vin, kout, vout, n, shift, hist, nblk);
}

void launch_gather(const CrystalDev *cs, const int32_t *ion_crystal, const uint32_t *vals, int ntot, double *sp,
                   const int32_t *halt, hipStream_t st)
{
    k_gather<<<ceil_div(ntot, 256), 256, 0, st>>>(cs, ion_crystal, vals, ntot, sp, halt);
}

size_t radix_state_words(int n) { return (size_t)kMaxPasses * 256 + kMaxPasses + 1 + 1 +
                                        2 * (size_t)kMaxPasses * sort_blocks(n) * 256; }

int launch_radix_sort(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int n, int passes, int first,
                      uint32_t *state, const int32_t *halt, const KeySource *keys, hipStream_t st)
{
    if (passes > kMaxPasses || first < 0 || first > passes || n <= 0) return -1;
    auto run = [&](auto items_tag) {
        constexpr int ITEMS = decltype(items_tag)::value;
        const int ntile = ceil_div(n, kSortTB * ITEMS);  // at most sort_blocks(n): the workspace fits
        uint32_t *ghist = state, *ctr = state + kMaxPasses * 256, *err = ctr + kMaxPasses;
        uint64_t *flags = (uint64_t *)(state + kMaxPasses * 256 + kMaxPasses + 2);  // 8-byte aligned
        if (keys)
            k_radix_prepare<true, ITEMS>
                <<<ntile, kSortTB, 0, st>>>(k0, v0, *keys, n, passes, first, ghist, flags, ntile, halt);
        else
            k_radix_prepare<false, ITEMS>
                <<<ntile, kSortTB, 0, st>>>(k0, v0, KeySource{}, n, passes, first, ghist, flags, ntile, halt);
        for (int p = first; p < passes; ++p) {
            const bool odd = (p - first) % 2;
            k_radix_pass<ITEMS><<<ntile, kSortTB, 0, st>>>(odd ? k1 : k0, odd ? v1 : v0, odd ? k0 : k1,
                                                           odd ? v0 : v1, n, p, ghist, flags, ntile, ctr, err, halt);
        }
    };
    // large batches take tiles of 8 keys per thread: fewer tiles in each
    // pass's look-back; below that, 4 keep more workgroups on the chip
    if (n >= kSortWideN)
        run(std::integral_constant<int, 2 * kSortItems>{});
    else
        run(std::integral_constant<int, kSortItems>{});
    return (passes - first) % 2;  // 1: the result is in (k1, v1)
}

void launch_sort_refine(uint64_t *keys, uint32_t *vals, int n, int shift, TreeSummary *sum, const CrystalDev *cs,
                        const int32_t *ion_crystal, double *sp, hipStream_t st)
{
    if (n > 0) k_sort_refine<<<ceil_div(n, 256), 256, 0, st>>>(keys, vals, n, shift, sum, cs, ion_crystal, sp);
}

int tree_blocks(int ntot) { return ceil_div(ntot, 256); }

void launch_tree_count(const CrystalDev *cs, const uint64_t *keys, int ntot, int leaf_size, uint32_t *rep_mask,
                       int32_t *box_end, uint32_t *blockcnt, uint32_t *partial, uint32_t *total,
                       const uint32_t *sort_err, TreeSummary *sum, const Caps *check, unsigned long long *bbox,
                       int nc, hipStream_t st)
{
    const int nblk = tree_blocks(ntot);
    const int n = (kMaxLevel + 1) * nblk;
    const Caps cap = check ? *check : Caps{};
    k_tree_levels<<<nblk, 256, 0, st>>>(cs, keys, ntot, leaf_size, rep_mask, box_end, blockcnt, nblk, &sum->halt,
                                        bbox, (int)bbox_words(nc));
    if (scan_partials(n) == 1) {  // one chunk: the summary comes with the scan
        k_scan_tree_summary<<<1, kScanTB, 0, st>>>(blockcnt, nblk, total, sort_err, sum, cap, check ? 1 : 0);
        return;
    }
    launch_scan(blockcnt, n, partial, total, st);
    k_tree_summary<<<1, 64, 0, st>>>(blockcnt, nblk, total, sort_err, sum, cap, check ? 1 : 0);
}

void launch_tree_build(const CrystalDev *cs, const RootCube *roots, const uint64_t *keys, int ntot, int leaf_size,
                       const uint32_t *rep_mask, const int32_t *box_end, const uint32_t *scanned, const BoxTable &bt,
                       const TreeSummary *sum, int nbox, hipStream_t st)
{
    const int nblk = tree_blocks(ntot);
    k_tree_emit<<<nblk, 256, 0, st>>>(cs, roots, keys, ntot, leaf_size, rep_mask, box_end, scanned, nblk, bt, sum);
}

void launch_lists(const BoxTable &bt, const TreeSummary *sum, int nbox, int32_t *coll, int32_t *vtab, int stride,
                  int2 *near, int32_t *near_cnt, int64_t *near_pairs, int32_t *child_oct, int32_t *parent_oct,
                  uint32_t *l2l_cnt, int32_t *l2l_list, const ZeroRegions &zr, uint32_t *item_off,
                  int32_t *src_items, int32_t *cuts, const int2 *slots, uint32_t *pcnt, uint32_t *cnt_ob,
                  uint32_t *op_total, double *near_ext, hipStream_t st)
{
    const int ncb = ceil_div(nbox * kNeigh, 256);
    k_oct_colleagues<<<ncb + ceil_div(nbox, 256), 256, 0, st>>>(bt, sum, coll, ncb, child_oct, parent_oct, l2l_cnt,
                                                                l2l_list, nbox, zr);
    k_box_lists<<<nbox, 256, 0, st>>>(bt, sum, coll, child_oct, vtab, slots, pcnt, cnt_ob, op_total, stride, near,
                                      near_cnt, item_off, src_items, cuts, near_pairs, near_ext);
}

void launch_p2p_items(const BoxTable &bt, TreeSummary *sum, int nbox, const int32_t *near_cnt, int stride,
                      const uint32_t *item_off, const int32_t *src_items, const int32_t *cuts, int4 *work,
                      const uint32_t *total, const Caps *check, hipStream_t st)
{
    k_p2p_items<<<nbox, 64, 0, st>>>(bt, sum, near_cnt, stride, item_off, src_items, cuts, work, total,
                                     check ? *check : Caps{}, check ? 1 : 0);
}

}  // namespace pt
