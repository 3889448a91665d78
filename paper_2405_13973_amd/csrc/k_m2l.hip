// M2L, the multipole-to-local conversion over the V lists (Zaris et al.,
// Sec. 2.3, eq. FMM_local; downward pass), as a dense contraction on the
// matrix cores, organised by operator.
//
// With coefficients scaled by the box side, the conversion from a source box
// S to a target box T of the same level depends only on their offset d (one
// of the 316 offsets in [-3,3]^3 outside [-1,1]^3):  L_T += T_d M_S.  T_d is
// S T_|d| S for the 56 stored base operators of offsets with non-negative
// components, S the diagonal sign matrix of the reflections of d's negative
// components.  So every V pair (T, S) is a matrix-vector product with one of
// 56 base matrices plus sign flips, and the pairs that share a base matrix
// form one GEMM:
//   1. pairs are counted per target and per base operator (with the V
//      lists, in the box-list kernel of the tree code), and scans give
//      each pair a row in a result buffer R (targets in box order, a target's
//      pairs in the order of its parity's slot table) and a place in its
//      operator's bucket (operators in order, then boxes, then slots);
//   2. a persistent workgroup takes a contiguous run of work units -- 64
//      pairs of one operator bucket times one group of output rows -- keeps
//      that row group of the base operator in LDS while it stays on the same
//      operator, and computes the 64 products on the matrix cores
//      (16 columns per wave), the column signs applied to the loaded source
//      coefficients and the row signs to the results, each product written to
//      its own row of R;
//   3. L_T is the sum of its rows of R in order.
// Every product is computed by the same instructions whichever workgroup,
// batch or column it lands in, and each target's sum runs in its fixed slot
// order, so results are deterministic and do not depend on the batch.  No
// work is spent on absent sources: a unit multiplies only existing pairs
// (the last unit of a bucket is padded with the zero expansion row).
#include <algorithm>

#include "fmm_math.hpp"
#include "pt_common.hpp"
#include "pt_kernels.hpp"

namespace pt {

namespace {

constexpr int kOps = kM2LOps;
constexpr int kSlots = kM2LSlots;
constexpr int kCols = 64;  // pairs per work unit (16 per wave)
constexpr int kGemmThreads = 256;
constexpr int kOpSlices = kM2LOpSlices;

template <typename T>
struct MfmaOp;
template <>
struct MfmaOp<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 op(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }  // output row of element r
};
template <>
struct MfmaOp<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// 16 bytes of T: the unit of every operand load (VEC values).
template <typename T>
struct Vec16 {
    static constexpr int N = 16 / sizeof(T);
    T v[N];
};

}  // namespace

// Pass 1, one launch of kOps + 4 workgroups (kScanThreads each) after the
// counts of the box lists: workgroup o < kOps scans its operator's row of cnt_ob from the
// operator's first bucket place (the totals of the operators before it), so
// the places are those of one scan of cnt_ob in (operator, box) order;
// workgroup kOps scans pcnt, kOps + 1 the near-field item counts, kOps + 2
// writes the operator table from the totals and kOps + 3 adds up the
// near-field pairs.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void k_list_scans(const TreeSummary *__restrict__ sum, int nbox_cap,
                                                             uint32_t *__restrict__ pcnt, uint32_t *__restrict__ cnt_ob,
                                                             const uint32_t *__restrict__ op_total,
                                                             uint32_t *__restrict__ npairs,
                                                             uint32_t *__restrict__ item_off,
                                                             uint32_t *__restrict__ n_items,
                                                             int32_t *__restrict__ op_beg,
                                                             int32_t *__restrict__ chunk_off,
                                                             const int64_t *__restrict__ near_pairs,
                                                             unsigned long long *__restrict__ near_total)
{
    __shared__ uint32_t lds_w[kScanThreads / 64 + 1];
    __shared__ uint32_t tot_s[kOps];
    if (sum->halt) return;
    const int g = blockIdx.x, tid = threadIdx.x;
    const int nbox = sum->nbox;
    if (tid < kOps) {  // the operator totals: sums over the slices
        uint32_t t = 0;
        for (int sl = 0; sl < kOpSlices; ++sl) t += op_total[sl * kOps + tid];
        tot_s[tid] = t;
    }
    __syncthreads();
    if (g < kOps) {
        uint32_t base = 0;
        for (int o = 0; o < g; ++o) base += tot_s[o];
        block_scan_inplace(cnt_ob + (size_t)g * nbox, nbox, base, lds_w);
    } else if (g == kOps) {
        const uint32_t tot = block_scan_inplace(pcnt, nbox_cap, 0u, lds_w);
        if (tid == 0) *npairs = tot;
    } else if (g == kOps + 1) {
        const uint32_t tot = block_scan_inplace(item_off, nbox_cap, 0u, lds_w);
        if (tid == 0) *n_items = tot;
    } else if (g == kOps + 3) {
        // the near-field pairs of all leaves (integer sum: any order)
        __shared__ unsigned long long ws[kScanThreads / 64];
        unsigned long long acc = 0;
        for (int b = tid; b < nbox_cap; b += kScanThreads) acc += (unsigned long long)near_pairs[b];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if ((tid & 63) == 0) ws[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0) {
            unsigned long long t = 0;
            for (int w = 0; w < kScanThreads / 64; ++w) t += ws[w];
            *near_total = t;
        }
    } else if (tid < 64) {
        // per operator its bucket's first entry (op_beg[o], op_beg[kOps] = all
        // pairs) and the prefix of its work-unit counts (chunk_off)
        const int o = tid;
        const uint32_t t = tot_s[o];
        uint32_t c = (t + kCols - 1) / kCols;  // inclusive wave scan of the unit counts
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t z = __shfl_up(c, off);
            if (o >= off) c += z;
        }
        uint32_t first = 0;  // exclusive prefix of the totals
        for (int k = 0; k < o; ++k) first += tot_s[k];
        op_beg[o] = (int32_t)first;
        chunk_off[o + 1] = (int32_t)c;
        if (o == 0) chunk_off[0] = 0;
        if (o == kOps - 1) op_beg[kOps] = (int32_t)(first + t);
    }
}

// Pass 2, one workgroup per box, after the scans of pcnt (-> the box's
// first row of R) and cnt_ob (-> the box's first place in each operator
// bucket): each pair's bucket entry {source box, row of R, reflection mask}.
// Ranks follow the slot order, so the layout is deterministic: a slot's rank
// among the box's pairs and among those of its operator come from ballots
// within each wave plus the counts of the waves before it.
__global__ __launch_bounds__(256) void k_m2l_emit(BoxTable bt, const TreeSummary *__restrict__ sum,
                                                  const int32_t *__restrict__ vtab, const int2 *__restrict__ slots,
                                                  const uint32_t *__restrict__ pair_off,
                                                  const uint32_t *__restrict__ ob_off, int4 *__restrict__ bucket)
{
    __builtin_amdgcn_s_setprio(1);  // may run beside the near field, as the GEMM
    constexpr int NW = 256 / 64;
    __shared__ uint32_t wave_cnt[NW];
    __shared__ uint32_t wave_op_cnt[NW][kOps];
    const int b = blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int nbox = sum->nbox;
    if (sum->halt || b >= nbox || bt.level[b] < 2) return;
    wave_op_cnt[w][lane] = 0;
    int src = -1, opw = 0;
    if (tid < kSlots) {
        const int2 s = slots[box_parity(bt, b) * kSlots + tid];
        src = vtab[(size_t)b * kWin + s.x];
        opw = s.y;
    }
    const bool valid = src >= 0;
    const int op = opw & 255;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const unsigned long long vb = __ballot(valid);
    unsigned long long peers = vb;  // valid lanes of this wave with the same operator
#pragma unroll
    for (int bit = 0; bit < 6; ++bit) {
        const bool on = (op >> bit) & 1;
        const unsigned long long m = __ballot(on);
        peers &= on ? m : ~m;
    }
    __syncthreads();  // wave_op_cnt cleared
    if (lane == 0) wave_cnt[w] = (uint32_t)__popcll(vb);
    if (valid && __popcll(peers & lt) == 0) wave_op_cnt[w][op] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (!valid) return;
    uint32_t rank = (uint32_t)__popcll(vb & lt), rank_op = (uint32_t)__popcll(peers & lt);
    for (int k = 0; k < w; ++k) {
        rank += wave_cnt[k];
        rank_op += wave_op_cnt[k][op];
    }
    const uint32_t pos = ob_off[(size_t)op * nbox + b] + rank_op;
    bucket[pos] = make_int4(src, (int)(pair_off[b] + rank), opw >> 8, 0);
}

// Pass 4: the products.  Work unit u (of nrg * U, U = chunk_off[64]) is row
// group rg = u / U of chunk u % U; each workgroup takes a contiguous run of
// units, so it mostly stays on one operator and one row group.
//
// Operand layout: a step covers 4 VEC values of k.  Lane l (column j = l % 16,
// quarter q = l / 16) loads the 16 bytes of source coefficients k = 4 VEC s +
// VEC q + e (e < VEC) and reads the same k of row (l % 16) of each row block
// from LDS with one 16-byte read; the e-th matrix-core instruction of the
// step takes element e of both, i.e. the contraction runs over a fixed
// permutation of k, the same for every product.
template <typename T, int NRB, int STEPS>
__global__ __launch_bounds__(kGemmThreads) void k_m2l_gemm(const TreeSummary *__restrict__ sum, int Kp, int nrg, int zrow,
                                                           const int32_t *__restrict__ chunk_off_g,
                                                           const int32_t *__restrict__ op_beg_g,
                                                           const int4 *__restrict__ bucket, const T *__restrict__ A,
                                                           const T *__restrict__ M, T *__restrict__ R)
{
    using MF = MfmaOp<T>;
    using V = Vec16<T>;
    constexpr int VEC = V::N;
    constexpr int ROWS = NRB * 16;
    // runs beside the near field: a raised wave priority lets these waves
    // (long dependency chains on the matrix cores) issue first when ready
    __builtin_amdgcn_s_setprio(1);
    if (sum->halt) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int strideE = Kp + VEC;  // row stride of the LDS operator rows (16-byte reads without bank conflicts)
    T *As = reinterpret_cast<T *>(smem_raw);                               // [ROWS][strideE]
    // sign of coefficient k under reflection mask m: sgn[m * Kp + k] (0 or 1)
    uint8_t *sgn = reinterpret_cast<uint8_t *>(As + (size_t)ROWS * strideE);  // [8][Kp]
    __shared__ int32_t chunk_off[kOps + 1], op_beg[kOps + 1];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int i = tid; i <= kOps; i += kGemmThreads) {
        chunk_off[i] = chunk_off_g[i];
        op_beg[i] = op_beg_g[i];
    }
    for (int i = tid; i < 8 * Kp; i += kGemmThreads) sgn[i] = (uint8_t)(__popc((i / Kp) & refl_bits(i % Kp)) & 1);
    __syncthreads();
    const int U = chunk_off[kOps];
    const long units = (long)U * nrg;
    const int u0 = (int)(units * blockIdx.x / gridDim.x), u1 = (int)(units * (blockIdx.x + 1) / gridDim.x);
    // STEPS > 0: the step count, fixed at compile time (a multiple of three)
    constexpr bool TRIPLE = STEPS > 0;
    const int steps = TRIPLE ? STEPS : Kp / (4 * VEC);
    const int j = lane & 15, q = lane >> 4;
    // a unit's operator, row group and pair range, and this lane's pair
    struct Unit {
        int op, rg, beg, end;
        int4 pe;  // {source box, row of R (-1: none), reflection mask, 0}
    };
    auto unit_of = [&](int u) {
        Unit t;
        t.rg = u / U;
        const int ch = u - t.rg * U;
        t.op = 0;  // the bucket holding chunk ch: last o with chunk_off[o] <= ch
        for (int step = 32; step > 0; step >>= 1)
            if (t.op + step <= kOps && chunk_off[t.op + step] <= ch) t.op += step;
        t.beg = op_beg[t.op] + (ch - chunk_off[t.op]) * kCols;
        t.end = min(t.beg + kCols, op_beg[t.op + 1]);
        const int col = t.beg + wave * 16 + j;
        t.pe = col < t.end ? bucket[col] : make_int4(zrow, -1, 0, 0);
        return t;
    };
    // 16 bytes of source coefficients of box `box` for step s
    auto load_b = [&](int box, int s) {
        return *reinterpret_cast<const V *>(M + (size_t)box * Kp + q * VEC + (size_t)s * 4 * VEC);
    };
    // their column signs, applied when step s uses them
    auto signed_b = [&](V v, int m, int s) {
        const uint8_t *g = sgn + m * Kp + s * 4 * VEC + q * VEC;
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (g[e]) v.v[e] = -v.v[e];
        return v;
    };
    // operator rows of a step from LDS
    const T *arow = As + (size_t)j * strideE + q * VEC;
    auto load_a = [&](int s, V *a) {
#pragma unroll
        for (int r = 0; r < NRB; ++r) a[r] = *reinterpret_cast<const V *>(arow + (size_t)r * 16 * strideE + s * 4 * VEC);
    };
    if (u0 >= u1) return;
    int cur_op = -1, cur_rg = -1;
    Unit cu = unit_of(u0);
    // Source coefficients sit in three register slots, step s in slot s % 3,
    // loaded two steps ahead of their use, so each load's wait comes right
    // before its use and no register copy waits for it.  With a step count
    // fixed at compile time (a multiple of three) the steps are straight-
    // line code and every step issues its load: the last two steps of a unit
    // load the next unit's first two (slots 0 and 1), or repeat this unit's
    // when it is the last, so the compiler can count each load's wait.
    // Otherwise the unit's first two steps are loaded at its start and the
    // tail is guarded.
    V bq0, bq1, bq2;
    if (TRIPLE) {
        bq0 = load_b(cu.pe.x, 0);
        bq1 = load_b(cu.pe.x, 1);
    }
    for (int u = u0; u < u1; ++u) {
        const bool has_next = u + 1 < u1;
        Unit nx = cu;
        if (has_next) nx = unit_of(u + 1);
        if (cu.op != cur_op || cu.rg != cur_rg) {
            __syncthreads();  // every wave is done with the previous rows
            const T *src = A + (size_t)cu.op * Kp * Kp;
            const int row0 = cu.rg * ROWS;
            const int vecs = ROWS * (Kp / VEC);
            for (int e = tid; e < vecs; e += kGemmThreads) {
                const int r = e / (Kp / VEC), c = (e - r * (Kp / VEC)) * VEC;
                V v;
                if (row0 + r < Kp) v = *reinterpret_cast<const V *>(src + (size_t)(row0 + r) * Kp + c);
                else
                    for (int k = 0; k < VEC; ++k) v.v[k] = T(0);
                *reinterpret_cast<V *>(As + (size_t)r * strideE + c) = v;
            }
            __syncthreads();
            cur_op = cu.op;
            cur_rg = cu.rg;
        }
        if (!TRIPLE) {
            bq0 = load_b(cu.pe.x, 0);
            if (steps > 1) bq1 = load_b(cu.pe.x, 1);
        }
        typename MF::v4 acc[NRB];
#pragma unroll
        for (int r = 0; r < NRB; ++r) acc[r] = typename MF::v4{0, 0, 0, 0};
        V a0[NRB], a1[NRB];
        load_a(0, a0);
        // one step: load step s + 2 into slot `to` (past the end: the next
        // unit's step s + 2 - steps), then multiply with slot `use`
        auto step = [&](int s, const V &use, V &to) {
            const int ns = s + 2;
            if (TRIPLE) {
                const bool in = ns < steps;
                to = load_b(in ? cu.pe.x : nx.pe.x, in ? ns : ns - steps);
            } else if (ns < steps) {
                to = load_b(cu.pe.x, ns);
            }
            // keep the load here: the scheduler would otherwise sink it to
            // its use two steps on and wait for it there
            __builtin_amdgcn_sched_barrier(0);
            load_a(min(s + 1, steps - 1), a1);
            const V bs = signed_b(use, cu.pe.z, s);
            // consecutive instructions update different accumulators, so
            // none waits for the previous one's result
#pragma unroll
            for (int e = 0; e < VEC; ++e)
#pragma unroll
                for (int r = 0; r < NRB; ++r) acc[r] = MF::op(a0[r].v[e], bs.v[e], acc[r]);
#pragma unroll
            for (int r = 0; r < NRB; ++r) a0[r] = a1[r];
        };
        auto three = [&](int s) {
            step(s, bq0, bq2);
            if (TRIPLE || s + 1 < steps) step(s + 1, bq1, bq0);
            if (TRIPLE || s + 2 < steps) step(s + 2, bq2, bq1);
        };
        if constexpr (TRIPLE) {
#pragma unroll
            for (int s = 0; s < STEPS; s += 3) three(s);
        } else {
            for (int s = 0; s < steps; s += 3) three(s);
        }
        if (cu.pe.y >= 0) {
            const int row0 = cu.rg * ROWS;
            T *dst = R + (size_t)cu.pe.y * Kp + row0;
#pragma unroll
            for (int r = 0; r < NRB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = r * 16 + MF::row(lane, e);
                    if (row0 + row < Kp) {
                        const T v = acc[r][e];
                        dst[row] = sgn[cu.pe.z * Kp + row0 + row] ? -v : v;
                    }
                }
        }
        cu = nx;
    }
}

// Pass 5: L_T = sum of T's rows of R in order (zero for boxes above level 2
// or without V pairs); a box's rows run from pair_off[b] to the next box's
// first row (npairs after the last box).  One thread per 16 bytes of
// coefficients; the row loads are issued in groups of 8 ahead of their
// additions, which stay in row order.
template <typename T>
__global__ void k_m2l_sum(const TreeSummary *__restrict__ sum, int Kp, const uint32_t *__restrict__ pair_off,
                          const uint32_t *__restrict__ npairs, const T *__restrict__ R, T *__restrict__ L)
{
    __builtin_amdgcn_s_setprio(1);  // runs beside the near field, as the GEMM
    using V = Vec16<T>;
    constexpr int VEC = V::N;
    if (sum->halt) return;
    const int nbox = sum->nbox;
    const int per_box = Kp / VEC;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)nbox * per_box;
         e += (size_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / per_box), c = (int)(e - (size_t)b * per_box) * VEC;
        const int n = (int)((b + 1 < nbox ? pair_off[b + 1] : *npairs) - pair_off[b]);
        const T *r = R + (size_t)pair_off[b] * Kp + c;
        V acc;
        for (int i = 0; i < VEC; ++i) acc.v[i] = T(0);
        int k = 0;
        for (; k + 8 <= n; k += 8) {
            V v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = *reinterpret_cast<const V *>(r + (size_t)(k + u) * Kp);
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int i = 0; i < VEC; ++i) acc.v[i] += v[u].v[i];
        }
        for (; k < n; ++k) {
            const V v = *reinterpret_cast<const V *>(r + (size_t)k * Kp);
#pragma unroll
            for (int i = 0; i < VEC; ++i) acc.v[i] += v.v[i];
        }
        *reinterpret_cast<V *>(L + (size_t)b * Kp + c) = acc;
    }
}

// ---------------------------------------------------------------- launchers

void launch_list_scans(const TreeSummary *sum, int nbox, uint32_t *pcnt, uint32_t *cnt_ob, const uint32_t *op_total,
                       uint32_t *npairs, uint32_t *item_off, uint32_t *n_items, int32_t *op_beg, int32_t *chunk_off,
                       const int64_t *near_pairs, unsigned long long *near_total, hipStream_t st)
{
    if (nbox <= 0) return;
    k_list_scans<<<kOps + 4, kScanThreads, 0, st>>>(sum, nbox, pcnt, cnt_ob, op_total, npairs, item_off, n_items,
                                                    op_beg, chunk_off, near_pairs, near_total);
}

int m2l_ops() { return kOps; }
int m2l_op_total_words() { return kOps * kOpSlices; }

void launch_m2l_emit(const BoxTable &bt, const TreeSummary *sum, int nbox, const int32_t *vtab, const int2 *slots,
                     const uint32_t *pair_off, const uint32_t *ob_off, int4 *bucket, hipStream_t st)
{
    if (nbox <= 0) return;
    k_m2l_emit<<<nbox, 256, 0, st>>>(bt, sum, vtab, slots, pair_off, ob_off, bucket);
}

// Row blocks of 16 per workgroup: as many as fit the LDS share of one
// workgroup (two per compute unit beside the near field), at most max_rb,
// balanced over the row groups.
template <typename T>
static int m2l_row_blocks(int Kp, int max_rb, int &nrg)
{
    const int blocks = Kp / 16;
    const size_t per_block = (size_t)16 * (Kp + 16 / sizeof(T)) * sizeof(T);
    const int fit = std::max(1, (int)(kM2LLdsBudget / per_block));
    nrg = ceil_div(blocks, std::max(1, std::min({fit, kM2LMaxRowBlocks, max_rb})));
    return ceil_div(blocks, nrg);
}

template <typename T>
size_t m2l_gemm_lds(int Kp, int max_rb)
{
    int nrg;
    const int nrb = m2l_row_blocks<T>(Kp, max_rb, nrg);
    return (size_t)nrb * 16 * (Kp + 16 / sizeof(T)) * sizeof(T) + (size_t)8 * Kp;
}

template <typename T>
int m2l_per_cu(int Kp, int max_rb, size_t lds_beside)
{
    const size_t lds = m2l_gemm_lds<T>(Kp, max_rb) + 2 * (kOps + 1) * sizeof(int32_t);
    const size_t room = kLdsPerCU > lds_beside ? kLdsPerCU - lds_beside : 0;
    return std::max(1, std::min(kM2LMaxPerCU, (int)(room / lds)));
}

template <typename T>
void launch_m2l_gemm(const TreeSummary *sum, int Kp, int max_rb, int nbox, int grid, const int32_t *chunk_off,
                     const int32_t *op_beg, const int4 *bucket, const T *A, const T *M, T *R, hipStream_t st)
{
    int nrg;
    const int nrb = m2l_row_blocks<T>(Kp, max_rb, nrg);
    const size_t lds = m2l_gemm_lds<T>(Kp, max_rb);
    const int steps = Kp / (4 * (16 / (int)sizeof(T)));
    // order 11 (144 coefficients) runs with its step count fixed at compile time
    constexpr int kFixed = 144 / (4 * (16 / (int)sizeof(T)));
    switch (nrb) {
#define PT_G(NB)                                                                                          \
    case NB:                                                                                              \
        if (steps == kFixed)                                                                              \
            k_m2l_gemm<T, NB, kFixed>                                                                     \
                <<<grid, kGemmThreads, lds, st>>>(sum, Kp, nrg, nbox, chunk_off, op_beg, bucket, A, M, R); \
        else                                                                                              \
            k_m2l_gemm<T, NB, 0>                                                                          \
                <<<grid, kGemmThreads, lds, st>>>(sum, Kp, nrg, nbox, chunk_off, op_beg, bucket, A, M, R); \
        break;
        PT_G(1) PT_G(2) PT_G(3) PT_G(4) PT_G(5) PT_G(6)
#undef PT_G
    default: break;
    }
}

template <typename T>
void launch_m2l_sum(const TreeSummary *sum, int nbox, int Kp, const uint32_t *pair_off, const uint32_t *npairs,
                    const T *R, T *L, hipStream_t st)
{
    const size_t tot = (size_t)nbox * (Kp / (16 / sizeof(T)));
    if (tot)
        k_m2l_sum<T><<<(unsigned)std::min<size_t>((tot + 63) / 64, 65535), 64, 0, st>>>(sum, Kp, pair_off, npairs, R,
                                                                                      L);
}

template int m2l_per_cu<float>(int, int, size_t);
template int m2l_per_cu<double>(int, int, size_t);
template size_t m2l_gemm_lds<float>(int, int);
template size_t m2l_gemm_lds<double>(int, int);
template void launch_m2l_gemm<float>(const TreeSummary *, int, int, int, int, const int32_t *, const int32_t *,
                                     const int4 *, const float *, const float *, float *, hipStream_t);
template void launch_m2l_gemm<double>(const TreeSummary *, int, int, int, int, const int32_t *, const int32_t *,
                                      const int4 *, const double *, const double *, double *, hipStream_t);
template void launch_m2l_sum<float>(const TreeSummary *, int, int, const uint32_t *, const uint32_t *,
                                    const float *, float *, hipStream_t);
template void launch_m2l_sum<double>(const TreeSummary *, int, int, const uint32_t *, const uint32_t *,
                                     const double *, double *, hipStream_t);

}  // namespace pt
