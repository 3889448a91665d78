// Host runtime of libpenning: contexts, crystals, device memory under an HBM
// budget, the batched step loop and the force-evaluation pipeline.
//
// Per force evaluation of a batch (all crystals of one pt_step_batch /
// pt_compute_forces_batch call that are still active):
//   bbox (fused with the first half drift when stepping) -> root cubes and
//   keys with the digit counts -> LSD radix sort (8-bit digits over
//   crystal + 48 key bits) ->
//   gather sorted positions -> per-level box counts -> [one host read-back of
//   the box count per level] -> box table + links -> colleagues, V windows,
//   near lists -> P2M, M2M per level -> M2L -> L2L per level -> L2P + P2P.
// The direct method replaces everything after the bbox by one kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "fmm_math.hpp"
#include "pt_common.hpp"
#include "pt_kernels.hpp"

using namespace pt;

// Capacities of queued steps: the measured counts times this slack (raised
// after an overflow, see settle()).
constexpr double kCapsSlack = 1.5;
// When the two branches split before the upward pass, the near field keeps
// the main stream (and starts without waiting for the fork) if it outweighs
// M2L -- more than kNearFirstRatio near-field pairs per V pair, where the near
// field alone outlasts the M2L GEMM alone (~2e12 near pairs/s against ~1.1e9
// V pairs/s at p = 11) -- or if M2L is small, fewer than kNearFirstPairs V
// pairs (measured: 1e5-ion spheres at 270k V pairs gain 20%, 3e5 with 345k are
// even); otherwise the far field keeps it (1e6-ion spheres, ~3M V pairs: the
// far branch is the longer one, and starting it second costs 30%).
constexpr double kNearFirstRatio = 2000.0;
constexpr double kNearFirstPairs = 1.0e6;
// First digit the sort of a queued step orders by (the top kSortTopLevels
// levels; lowered after a run too long to refine, see settle()).
constexpr int kPsortFirst = (48 - 3 * kSortTopLevels) / 8;

// ---------------------------------------------------------------- errors

static thread_local char g_err[512] = "";

void pt_set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

#define PT_REQUIRE(cond, ...)          \
    do {                               \
        if (!(cond)) {                 \
            pt_set_error(__VA_ARGS__); \
            return PT_EINVAL;          \
        }                              \
    } while (0)

#define PT_TRY(expr)                  \
    do {                              \
        pt_status s_ = (expr);        \
        if (s_ != PT_OK) return s_;   \
    } while (0)

// ---------------------------------------------------------------- objects

namespace {

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct Tables {
    int p = -1;
    double *m2m_d = nullptr, *l2l_d = nullptr, *m2l_d = nullptr;
    float *m2m_f = nullptr, *l2l_f = nullptr, *m2l_f = nullptr;
    int2 *slots = nullptr;      // [8][189] {window slot, operator index}
    int2 *oct_slots = nullptr;  // [8] {octant, octant}
    double *rec_d = nullptr;
    float *rec_f = nullptr;
};

}  // namespace

struct pt_crystal {
    pt_ctx *ctx = nullptr;
    int64_t n = 0;
    double q = 0, m = 0;
    uint64_t seed = 0;
    pt_trap_params trap{};
    pt_laser_params laser{};
    pt_force_params force{};
    int64_t step = 0;
    double *d_state = nullptr;   // 6 n
    int32_t *d_photons = nullptr;
    int32_t *d_nonfinite = nullptr;  // set by the kick when the state turns non-finite
};

// Timed phases of a force evaluation (events 0..6 bracket them): sort+tree+
// lists, P2M+M2M, M2L, M2L reduce+L2L, P2P, L2P + near-field partials, total.
constexpr int kPhases = 7;
// Event sets of timed evaluations kept in flight: the host collects a set
// only when the ring is full or the times are asked for, so timing adds no
// host wait to a run of up to this many evaluations.
constexpr int kTimingRing = 64;
// Queued steps between two looks at the run state: every kCheckEvery steps
// the run's fail_step is copied to the host behind the work, and a look at a
// copy stops the queueing once a step halted; the host waits for a copy only
// when it is more than kCheckAhead copies ahead, so a halted run wastes at
// most about (kCheckAhead + 1) kCheckEvery steps while the device always has
// work queued.
constexpr int kCheckEvery = 8;
constexpr int kCheckSlots = 8;
constexpr int kCheckAhead = 2;
// Leaf size from which the near field runs concurrently with M2L / L2L.
constexpr int kConcurrentLeaf = 128;

struct pt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // the near field runs on its own stream, beside the far-field chain;
    // fork / join events order it after the lists and before the L2P kernel
    hipStream_t near_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_tree = nullptr, ev_p2m = nullptr, ev_read = nullptr;
    int num_cu = 1;  // compute units of the device
    hipEvent_t ev_near[kTimingRing][2] = {};  // timing of the P2P kernel (its own stream)
    bool near_timed[kTimingRing] = {};
    int near_concurrent = -1;  // -1: by leaf size; 0 / 1: forced (PT_NEAR_CONCURRENT)
    int near_per_cu = 0;  // near-field workgroups per CU beside the far field (PT_NEAR_PER_CU; 0: by schedule)
    int near_early = -1;  // -1: by precision; 0 / 1: forced (PT_NEAR_EARLY): near field forks before the upward pass
    int near_main = -1;   // forking before the upward pass: 1 = the far field forks, the near field stays,
                          // 0 = the near field forks, -1 = by the measured balance (PT_NEAR_MAIN)
    bool near_first = false;  // the last measured batch's near field outweighs its M2L
    ZeroRegions last_zr{};    // words the last evaluation's drift zeroed (for a kick that makes the next drift)
    // first Morton digit the sort of a queued step orders by (the runs of
    // equal higher digits are then refined): starts at the top kSortTopLevels
    // levels, one digit lower after every run that is too long to refine, 0 =
    // the full sort (PT_PARTIAL_SORT=0 starts there)
    int psort_first = kPsortFirst;
    bool psort_off = false;  // PT_PARTIAL_SORT=0: every queued step sorts all digits
    uint64_t budget = 0, used = 0;
    int live = 0;
    int32_t *d_nonfinite = nullptr;  // set by any kick of this context that produces a non-finite value
    bool no_queue = false;           // every evaluation measures (PT_QUEUED_STEPS=0)
    bool tight_caps = false;         // capacities one box short of the measured tree (PT_CAPS_TIGHT=1: tests)
    bool eval_halted = false;        // the last measuring evaluation found its run halted
    int64_t reruns = 0;              // queued runs re-run after a capacity overflow
    int64_t n_queued = 0, n_measured = 0;  // FMM evaluations of steps, by kind
    char *noalloc = nullptr;         // this device's fixed scratch (pt_compute_forces_noalloc)
    std::map<void *, size_t> allocs;
    // workspace (grow-only)
    std::map<std::string, DevBuf> ws;
    Tables tables;
    // pinned host staging
    CrystalDev *h_desc = nullptr;
    int h_desc_cap = 0;
    TreeSummary *h_sum = nullptr;
    int32_t *h_fail = nullptr;                 // pinned: kCheckSlots copies of fail_step
    hipEvent_t ev_check[kCheckSlots] = {};
    unsigned long long *h_counters = nullptr;
    // last force evaluation (for the debug export and statistics)
    std::vector<pt_crystal *> last_batch;
    std::vector<int32_t> last_off;
    uint64_t *last_keys = nullptr;
    uint32_t *last_vals = nullptr;
    int last_ntot = 0, last_was_fmm = 0, last_stride = 0, last_p = 0, last_prec = 0;
    Caps last_cap{};   // capacities (measuring: exact counts) of the last FMM evaluation
    Caps measured{};   // counts of the last measuring evaluation
    // capacities for queued steps, valid for one batch (its crystals, size
    // and force parameters)
    bool caps_ok = false;
    Caps caps{};
    double caps_slack = kCapsSlack;  // raised by half after each overflow of a batch, up to 4
    std::vector<pt_crystal *> caps_batch;
    int caps_ntot = 0;
    pt_force_params caps_force{};
    // the last pt_step_batch call, until its outcome has been read back: a
    // step that halted (see TreeSummary) is re-run from there on
    struct Pending {
        bool active = false;
        std::vector<pt_crystal *> cs;
        std::vector<int64_t> n_steps, step_start;
    } pending;
    // timing: a ring of event sets, ring_cur the set of the evaluation being
    // queued, ring_pending sets recorded and not yet collected (the oldest at
    // ring_cur - ring_pending)
    int timing = 0;         // the evaluation being queued records its events
    int timing_every = 0;   // set by pt_ctx_set_timing: record every timing_every-th evaluation (0: none)
    int64_t timing_evals = 0;
    bool ring_made = false;
    int ring_cur = 0, ring_pending = 0;
    hipEvent_t ev[kTimingRing][kPhases] = {};
    double phase_sum[kPhases] = {};
    int64_t phase_count = 0;
};

// ---------------------------------------------------------------- memory

static pt_status ctx_alloc(pt_ctx *ctx, void **out, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (ctx->budget && ctx->used + bytes > ctx->budget) {
        pt_set_error("HBM budget exceeded: %llu + %llu > %llu bytes", (unsigned long long)ctx->used,
                     (unsigned long long)bytes, (unsigned long long)ctx->budget);
        return PT_ENOMEM;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        pt_set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? PT_ENOMEM : PT_EDEVICE;
    }
    ctx->used += bytes;
    ctx->allocs[p] = bytes;
    *out = p;
    return PT_OK;
}

static void ctx_free(pt_ctx *ctx, void *p)
{
    if (!p) return;
    auto it = ctx->allocs.find(p);
    if (it != ctx->allocs.end()) {
        ctx->used -= it->second;
        ctx->allocs.erase(it);
    }
    (void)hipFree(p);
}

// Workspace buffer `name` of at least `bytes` (contents not preserved on growth).
template <typename T>
static pt_status ws_get(pt_ctx *ctx, const char *name, size_t bytes, T **out)
{
    DevBuf &b = ctx->ws[name];
    if (b.bytes < bytes) {
        if (b.ptr) {
            PT_HIP(hipStreamSynchronize(ctx->stream));
            ctx_free(ctx, b.ptr);
            b.ptr = nullptr;
            b.bytes = 0;
        }
        size_t want = bytes + bytes / 4 + 256;
        PT_TRY(ctx_alloc(ctx, &b.ptr, want));
        b.bytes = want;
    }
    *out = (T *)b.ptr;
    return PT_OK;
}

// ---------------------------------------------------------------- tables

static pt_status ensure_tables(pt_ctx *ctx, int p)
{
    Tables &t = ctx->tables;
    if (t.p == p) return PT_OK;
    PT_HIP(hipStreamSynchronize(ctx->stream));
    for (void *q : {(void *)t.m2m_d, (void *)t.l2l_d, (void *)t.m2l_d, (void *)t.m2m_f, (void *)t.l2l_f,
                    (void *)t.m2l_f, (void *)t.slots, (void *)t.oct_slots, (void *)t.rec_d, (void *)t.rec_f})
        ctx_free(ctx, q);
    t = Tables{};
    const int K = kcoef(p);
    const size_t KK = (size_t)K * K;
    const int Kp = kpad(p);
    std::vector<double> m2m(8 * KK), l2l(8 * KK), m2l(343 * KK);
    if (build_operator_tables(p, m2m.data(), l2l.data(), m2l.data()) != 0) {
        pt_set_error("operator tables: unsupported p = %d", p);
        return PT_EINVAL;
    }
    // for the matrix cores: column-major (A[j][i] = T[i][j]), zero-padded to Kp x Kp
    auto pad_cm = [&](std::vector<double> &v, int count) {
        std::vector<double> pad((size_t)count * Kp * Kp, 0.0);
        for (int c = 0; c < count; ++c)
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j) pad[(size_t)c * Kp * Kp + (size_t)j * Kp + i] = v[c * KK + (size_t)i * K + j];
        v.swap(pad);
    };
    // M2L: only offsets with non-negative components are kept (64 slots,
    // index m2l_base); the others follow by reflection signs in the kernel
    std::vector<double> base((size_t)64 * KK, 0.0);
    for (int ax = 0; ax <= 3; ++ax)
        for (int ay = 0; ay <= 3; ++ay)
            for (int az = 0; az <= 3; ++az)
                std::copy(m2l.begin() + (size_t)((ax + 3) * 49 + (ay + 3) * 7 + (az + 3)) * KK,
                          m2l.begin() + (size_t)((ax + 3) * 49 + (ay + 3) * 7 + (az + 3) + 1) * KK,
                          base.begin() + (size_t)m2l_base(ax, ay, az) * KK);
    m2l.swap(base);
    pad_cm(m2m, 8);
    pad_cm(l2l, 8);
    // M2L operators row-major (row = output coefficient), zero-padded to Kp x Kp
    {
        std::vector<double> pad((size_t)64 * Kp * Kp, 0.0);
        for (int c = 0; c < 64; ++c)
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j) pad[(size_t)c * Kp * Kp + (size_t)i * Kp + j] = m2l[c * KK + (size_t)i * K + j];
        m2l.swap(pad);
    }
    auto upload = [&](const std::vector<double> &v, double **dd, float **df) -> pt_status {
        PT_TRY(ctx_alloc(ctx, (void **)dd, v.size() * sizeof(double)));
        PT_HIP(hipMemcpy(*dd, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
        std::vector<float> f(v.begin(), v.end());
        PT_TRY(ctx_alloc(ctx, (void **)df, f.size() * sizeof(float)));
        PT_HIP(hipMemcpy(*df, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
        return PT_OK;
    };
    PT_TRY(upload(m2m, &t.m2m_d, &t.m2m_f));
    PT_TRY(upload(l2l, &t.l2l_d, &t.l2l_f));
    PT_TRY(upload(m2l, &t.m2l_d, &t.m2l_f));
    std::vector<double> rec((size_t)kRecFields * kq(p));
    build_recurrence_table(p, rec.data());
    PT_TRY(upload(rec, &t.rec_d, &t.rec_f));
    // the 189 non-touching slots of each parity's 6x6x6 window as {window
    // index, base operator + 256 x reflection mask}, ordered by mask (the
    // kernel re-signs its accumulators when the mask changes)
    std::vector<int2> sl;
    for (int o = 0; o < 8; ++o) {
        const int cx = (o >> 2) & 1, cy = (o >> 1) & 1, cz = o & 1;
        std::vector<int2> par;
        for (int w = 0; w < kWin; ++w) {
            const int dx = w / 36 - 2 - cx, dy = (w / 6) % 6 - 2 - cy, dz = w % 6 - 2 - cz;
            if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
            const int mask = (dx < 0 ? 1 : 0) | (dy < 0 ? 2 : 0) | (dz < 0 ? 4 : 0);
            par.push_back(make_int2(w, m2l_base(std::abs(dx), std::abs(dy), std::abs(dz)) + 256 * mask));
        }
        std::stable_sort(par.begin(), par.end(), [](int2 a, int2 b) { return a.y < b.y; });
        sl.insert(sl.end(), par.begin(), par.end());
    }
    if (sl.size() != 8 * 189) {
        pt_set_error("window slot table has %zu entries", sl.size());
        return PT_EDEVICE;
    }
    PT_TRY(ctx_alloc(ctx, (void **)&t.slots, sl.size() * sizeof(int2)));
    PT_HIP(hipMemcpy(t.slots, sl.data(), sl.size() * sizeof(int2), hipMemcpyHostToDevice));
    int2 os[8];
    for (int o = 0; o < 8; ++o) os[o] = make_int2(o, o);
    PT_TRY(ctx_alloc(ctx, (void **)&t.oct_slots, sizeof(os)));
    PT_HIP(hipMemcpy(t.oct_slots, os, sizeof(os), hipMemcpyHostToDevice));
    t.p = p;
    return PT_OK;
}

// ---------------------------------------------------------------- batch

struct Batch {
    std::vector<pt_crystal *> cs;
    std::vector<int32_t> off;
    int ntot = 0;
    CrystalDev *d_desc = nullptr;
    int32_t *ion_crystal = nullptr;
    int32_t *blk_crystal = nullptr, *blk_first = nullptr;  // sum block table (per-crystal ion sums)
    int nblk_sum = 0;
    DirBlock *dir_tab = nullptr;  // direct-sum block table (direct method only)
    int nblk_dir = 0;
    int64_t dir_part = 0;  // doubles of the direct sum's chunk partials
    bool beams = false;    // some crystal uses the beam-mode laser
};

static void fill_desc(const pt_crystal *c, int off, double *mid, CrystalDev &d)
{
    std::memset(&d, 0, sizeof(d));
    d.state = c->d_state;
    d.mid = mid + 6 * (size_t)off;
    d.photons = c->d_photons;
    d.nonfinite = c->d_nonfinite;
    d.ctx_nonfinite = c->ctx->d_nonfinite;
    d.n = (int32_t)c->n;
    d.ion_off = off;
    d.dt = c->trap.dt_s;
    d.t0 = c->trap.t0_s;
    const double wc = c->q * c->trap.B_T / c->m;
    const double th = wc * 0.5 * c->trap.dt_s;
    d.c_half = std::cos(th);
    d.s_half = std::sin(th);
    if (wc != 0.0) {
        d.a_half = d.s_half / wc;
        d.b_half = (1.0 - d.c_half) / wc;
    } else {
        d.a_half = 0.5 * c->trap.dt_s;
        d.b_half = 0.0;
    }
    d.qkz = c->m * c->trap.omega_z * c->trap.omega_z;
    d.delta = c->trap.delta;
    d.omega_r = c->trap.omega_r;
    d.inv_m = 1.0 / c->m;
    d.damp_f = c->trap.damping_per_s > 0.0 ? std::exp(-0.5 * c->trap.damping_per_s * c->trap.dt_s) : 1.0;
    d.damp_on = c->trap.damping_per_s > 0.0 ? 1 : 0;
    d.mass = c->m;
    d.wc = wc;
    d.coul = c->q * c->q / (4.0 * kPi * kEps0);
    const bool on = c->laser.mode == 1 && c->laser.mean_per_step > 0.0;
    d.laser_on = on ? 1 : 0;
    d.recoil = on ? kPlanck / (c->laser.wavelength_m * c->m) : 0.0;
    // cumulative Poisson table p_0 = e^-lam, p_k = p_{k-1} lam / k
    double pk = std::exp(-(on ? c->laser.mean_per_step : 0.0)), acc = pk;
    d.poisson_F[0] = acc;
    for (int k = 1; k <= 16; ++k) {
        pk = pk * (on ? c->laser.mean_per_step : 0.0) / (double)k;
        acc = acc + pk;
        d.poisson_F[k] = acc;
    }
    const bool beams = c->laser.mode == 2;
    if (beams) {
        d.laser_on = 2;
        d.recoil = kPlanck / (c->laser.wavelength_m * c->m);
        d.kwave = 2.0 * kPi / c->laser.wavelength_m;
        d.gamma0 = c->laser.gamma0;
        d.n_beams = c->laser.n_beams;
        for (int l = 0; l < c->laser.n_beams; ++l) {
            const pt_beam &b = c->laser.beam[l];
            BeamDev &e = d.beam[l];
            const double r = std::sqrt(b.khat[0] * b.khat[0] + b.khat[1] * b.khat[1] + b.khat[2] * b.khat[2]);
            for (int k = 0; k < 3; ++k) e.khat[k] = b.khat[k] / r;
            e.detuning = b.detuning;
            e.s0 = b.s0;
            e.waist_y = b.waist_y;
            e.waist_z = b.waist_z;
            e.offset_y = b.offset_y;
            e.uniform = b.uniform ? 1 : 0;
        }
    }
    d.seed = c->seed;
    d.step0 = (uint64_t)c->step;
}

static pt_status form_batch(pt_ctx *ctx, const std::vector<pt_crystal *> &cs, Batch &b)
{
    b.cs = cs;
    b.off.assign(cs.size() + 1, 0);
    long long tot = 0;
    for (size_t i = 0; i < cs.size(); ++i) {
        b.off[i] = (int32_t)tot;
        tot += cs[i]->n;
    }
    PT_REQUIRE(tot < (1ll << 31) - (1 << 20), "batch of %lld ions is too large", tot);
    b.off[cs.size()] = (int32_t)tot;
    b.ntot = (int)tot;
    const int nc = (int)cs.size();
    PT_TRY(ws_get(ctx, "desc", sizeof(CrystalDev) * nc, &b.d_desc));
    PT_TRY(ws_get(ctx, "ion_crystal", sizeof(int32_t) * std::max(1, b.ntot), &b.ion_crystal));
    double *mid;
    PT_TRY(ws_get(ctx, "mid", sizeof(double) * 6 * (size_t)std::max(1, b.ntot), &mid));
    if (ctx->h_desc_cap < nc) {
        PT_HIP(hipStreamSynchronize(ctx->stream));
        if (ctx->h_desc) (void)hipHostFree(ctx->h_desc);
        ctx->h_desc = nullptr;
        PT_HIP(hipHostMalloc((void **)&ctx->h_desc, sizeof(CrystalDev) * nc * 2));
        ctx->h_desc_cap = nc * 2;
    } else {
        PT_HIP(hipStreamSynchronize(ctx->stream));  // staging buffer may still be read by a copy
    }
    for (int i = 0; i < nc; ++i) fill_desc(cs[i], b.off[i], mid, ctx->h_desc[i]);
    // direct method: chunk partials of each crystal (4 x chunks x n doubles)
    // and the block table over (crystal, source chunk, target tile)
    const bool direct = nc > 0 && cs[0]->force.method == 0;
    std::vector<DirBlock> dtab;
    b.dir_part = 0;
    if (direct)
        for (int i = 0; i < nc; ++i) {
            const int n = (int)cs[i]->n, chunks = direct_chunks(n), tiles = ceil_div(n, kDirTile);
            ctx->h_desc[i].dpart = b.dir_part;
            b.dir_part += 4 * (int64_t)chunks * n;
            for (int s = 0; s < chunks; ++s)
                for (int t = 0; t < tiles; ++t) dtab.push_back(DirBlock{i, t * kDirTile, s, 0});
        }
    b.beams = false;
    for (int i = 0; i < nc; ++i) b.beams = b.beams || cs[i]->laser.mode == 2;
    PT_HIP(hipMemcpyAsync(b.d_desc, ctx->h_desc, sizeof(CrystalDev) * nc, hipMemcpyHostToDevice, ctx->stream));
    launch_ion_crystal(b.d_desc, nc, b.ntot, b.ion_crystal, ctx->stream);
    // bounding boxes start empty; the root-cube kernel empties them again after each use
    unsigned long long *bbox;
    PT_TRY(ws_get(ctx, "bbox", sizeof(unsigned long long) * bbox_words(nc), &bbox));
    launch_bbox_reset(bbox, nc, ctx->stream);
    // sum block table: each block serves ions of one crystal
    const int tpb = sum_ions_per_block();
    std::vector<int32_t> bc, bf;
    for (int i = 0; i < nc; ++i)
        for (int64_t f = 0; f < cs[i]->n; f += tpb) {
            bc.push_back(i);
            bf.push_back((int32_t)f);
        }
    b.nblk_sum = (int)bc.size();
    PT_TRY(ws_get(ctx, "blk_crystal", sizeof(int32_t) * std::max<size_t>(1, bc.size()), &b.blk_crystal));
    PT_TRY(ws_get(ctx, "blk_first", sizeof(int32_t) * std::max<size_t>(1, bf.size()), &b.blk_first));
    b.nblk_dir = (int)dtab.size();
    if (direct) PT_TRY(ws_get(ctx, "dir_tab", sizeof(DirBlock) * std::max<size_t>(1, dtab.size()), &b.dir_tab));
    if (!bc.empty()) {
        PT_HIP(hipMemcpyAsync(b.blk_crystal, bc.data(), bc.size() * 4, hipMemcpyHostToDevice, ctx->stream));
        PT_HIP(hipMemcpyAsync(b.blk_first, bf.data(), bf.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    }
    if (!dtab.empty())
        PT_HIP(hipMemcpyAsync(b.dir_tab, dtab.data(), dtab.size() * sizeof(DirBlock), hipMemcpyHostToDevice,
                              ctx->stream));
    if (!bc.empty() || !dtab.empty()) PT_HIP(hipStreamSynchronize(ctx->stream));  // pageable sources
    return PT_OK;
}

static pt_status finish_timing(pt_ctx *ctx);
static pt_status settle(pt_ctx *ctx);

static void mark(pt_ctx *ctx, int i, hipStream_t on = nullptr)
{
    if (ctx->timing) (void)hipEventRecord(ctx->ev[ctx->ring_cur][i], on ? on : ctx->stream);
}

// Collects the oldest recorded event set into the running sums.
static pt_status collect_oldest(pt_ctx *ctx)
{
    const int s = (ctx->ring_cur - ctx->ring_pending + kTimingRing) % kTimingRing;
    PT_HIP(hipEventSynchronize(ctx->ev[s][kPhases - 1]));
    float ms;
    for (int i = 0; i < kPhases - 1; ++i) {
        // phase 4: the P2P kernel on its own stream (it overlaps phases 1-3)
        if (i == 4 && ctx->near_timed[s]) PT_HIP(hipEventElapsedTime(&ms, ctx->ev_near[s][0], ctx->ev_near[s][1]));
        else PT_HIP(hipEventElapsedTime(&ms, ctx->ev[s][i], ctx->ev[s][i + 1]));
        ctx->phase_sum[i] += ms;
    }
    PT_HIP(hipEventElapsedTime(&ms, ctx->ev[s][0], ctx->ev[s][kPhases - 1]));
    ctx->phase_sum[kPhases - 1] += ms;
    ctx->phase_count++;
    ctx->ring_pending--;
    return PT_OK;
}

// Starts the event set of a new timed evaluation (collecting the oldest set
// first when the ring is full).
static pt_status timing_begin(pt_ctx *ctx)
{
    ctx->timing = ctx->timing_every > 0 && ctx->timing_evals++ % ctx->timing_every == 0 ? 1 : 0;
    if (!ctx->timing) return PT_OK;
    if (ctx->ring_pending == kTimingRing) PT_TRY(collect_oldest(ctx));
    ctx->near_timed[ctx->ring_cur] = false;
    return PT_OK;
}

// Marks the current set recorded and moves to the next one.
static void timing_end(pt_ctx *ctx)
{
    if (!ctx->timing) return;
    ctx->ring_pending++;
    ctx->ring_cur = (ctx->ring_cur + 1) % kTimingRing;
}

static BoxTable box_table(pt_ctx *ctx)
{
    BoxTable t{};
    auto g = [&](const char *n) { return ctx->ws[n].ptr; };
    t.level = (int32_t *)g("b_level");
    t.crystal = (int32_t *)g("b_crystal");
    t.begin = (int32_t *)g("b_begin");
    t.end = (int32_t *)g("b_end");
    t.parent = (int32_t *)g("b_parent");
    t.child = (int32_t *)g("b_child");
    t.nchild = (int32_t *)g("b_nchild");
    t.ix = (int32_t *)g("b_ix");
    t.iy = (int32_t *)g("b_iy");
    t.iz = (int32_t *)g("b_iz");
    t.key = (uint64_t *)g("b_key");
    t.leaf = (uint8_t *)g("b_leaf");
    t.geo = (double4 *)g("b_geo");
    return t;
}

// Capacities for queued evaluations of a batch whose measured counts are m:
// room for a tree that grows from step to step (slack times as many boxes,
// items and pairs, a quarter more boxes per level, as many levels).
static Caps grow_caps(const Caps &m, double slack)
{
    Caps c = m;
    c.nbox = (int)(m.nbox * slack) + 16;
    c.items = (int)(m.items * slack) + 64;
    c.pairs = (int)(m.pairs * slack) + 256;
    for (int l = 0; l <= kMaxLevel; ++l) c.lvl[l] = l < m.nlev ? m.lvl[l] + m.lvl[l] / 4 + 8 : 0;
    return c;
}


// Coulomb field per unit charge of every ion of the batch into E (3 x ntot,
// batch order); with phi non-null also the potential per unit charge
// (sum_{j != i} 1/r_ij, ntot).  Starts with the bounding boxes of the
// positions, after the first half drift when drift is 1 (halt_aware: the
// drift is skipped once the run has halted); drift 2: the previous step's
// kick has made the drift and the boxes already.
//
// With the FMM, two ways: measuring (queued == nullptr), where the host
// reads back the tree's size and then the numbers of near-field items and
// M2L pairs and sizes everything exactly (two host waits), the counts going
// to ctx->measured; or queued, where buffers and grids are sized from the
// capacities *queued, kernels read the counts on the device, nothing is read
// back, and a count above its capacity halts the run on the device (the
// step's kick then leaves the state as it was, see TreeSummary).
static pt_status eval_field(pt_ctx *ctx, Batch &b, const pt_force_params &fp, double *E, double *phi,
                            const Caps *queued, int drift, bool halt_aware, KickPartials *leave = nullptr)
{
    hipStream_t st = ctx->stream;
    if (leave) *leave = KickPartials{nullptr, nullptr, 0};
    const int ntot = b.ntot, nc = (int)b.cs.size();
    unsigned long long *bbox;
    PT_TRY(ws_get(ctx, "bbox", sizeof(unsigned long long) * bbox_words(nc), &bbox));
    ctx->last_batch = b.cs;
    ctx->last_off = b.off;
    ctx->last_ntot = ntot;
    ctx->last_was_fmm = fp.method == 1;
    if (fp.method == 0) {
        PT_REQUIRE(b.nblk_dir > 0 || ntot == 0, "batch formed without the direct-sum block table");
        double *part;
        PT_TRY(ws_get(ctx, "dir_part", sizeof(double) * (size_t)std::max<int64_t>(1, b.dir_part), &part));
        ctx->last_zr = ZeroRegions{};
        if (drift != 2) launch_drift_bbox(b.d_desc, b.ion_crystal, ntot, nc, drift, bbox, nullptr, ZeroRegions{}, st);
        PT_TRY(timing_begin(ctx));
        mark(ctx, 0);
        launch_direct(b.d_desc, b.dir_tab, b.nblk_dir, b.ion_crystal, ntot, part, E, phi, st);
        for (int i = 1; i <= kPhases - 1; ++i) mark(ctx, i);
        timing_end(ctx);
        return PT_OK;
    }
    const int p = fp.p, s = fp.leaf_size;
    RootCube *roots;
    uint64_t *k0, *k1;
    uint32_t *v0, *v1, *hist, *rep, *bcnt, *total;
    double *sp;
    TreeSummary *dsum;
    PT_TRY(ws_get(ctx, "roots", sizeof(RootCube) * nc, &roots));
    PT_TRY(ws_get(ctx, "keys0", sizeof(uint64_t) * ntot, &k0));
    PT_TRY(ws_get(ctx, "keys1", sizeof(uint64_t) * ntot, &k1));
    PT_TRY(ws_get(ctx, "vals0", sizeof(uint32_t) * ntot, &v0));
    PT_TRY(ws_get(ctx, "vals1", sizeof(uint32_t) * ntot, &v1));
    PT_TRY(ws_get(ctx, "hist", sizeof(uint32_t) * 256 * sort_blocks(ntot), &hist));
    PT_TRY(ws_get(ctx, "rep", sizeof(uint32_t) * ntot, &rep));
    int32_t *box_end;
    PT_TRY(ws_get(ctx, "box_end", sizeof(int32_t) * (kMaxLevel + 1) * (size_t)ntot, &box_end));
    PT_TRY(ws_get(ctx, "bcnt", sizeof(uint32_t) * (kMaxLevel + 1) * tree_blocks(ntot), &bcnt));
    PT_TRY(ws_get(ctx, "total", sizeof(uint32_t) * 4, &total));
    uint32_t *scan_part;
    const int scan_n = std::max(256 * sort_blocks(ntot), (kMaxLevel + 1) * tree_blocks(ntot));
    PT_TRY(ws_get(ctx, "scan_part", sizeof(uint32_t) * (scan_partials(scan_n) + 1), &scan_part));
    PT_TRY(ws_get(ctx, "sp", sizeof(double) * 3 * ntot, &sp));
    PT_TRY(ws_get(ctx, "sum", sizeof(TreeSummary), &dsum));
    int cbits = 0;
    while ((1 << cbits) < nc) ++cbits;
    const int passes = (48 + cbits + 7) / 8;
    uint32_t *rstate;
    PT_TRY(ws_get(ctx, "radix_state", sizeof(uint32_t) * radix_state_words(ntot), &rstate));
    const uint32_t *sort_err = nullptr;
    uint32_t *l2l_cnt;
    PT_TRY(ws_get(ctx, "l2l_cnt", sizeof(uint32_t) * kL2LCounts, &l2l_cnt));
    {
        // the drift also zeroes the sort's counters and the L2L bucket counts
        ZeroRegions zr{};
        zr.p[0] = (uint64_t *)rstate;
        zr.n[0] = passes <= 8 ? radix_state_zero_words() / 2 : 0;
        zr.p[1] = (uint64_t *)l2l_cnt;
        zr.n[1] = kL2LCounts / 2;
        ctx->last_zr = zr;  // a kick that also makes the next step's drift zeroes the same words
        if (drift != 2)
            launch_drift_bbox(b.d_desc, b.ion_crystal, ntot, nc, drift, bbox, halt_aware ? &dsum->halt : nullptr, zr,
                              st);
    }
    PT_TRY(timing_begin(ctx));
    mark(ctx, 0);
    // root cubes and keys: made by the sort's first kernel (else by two launches)
    const KeySource key_src{b.d_desc, b.ion_crystal, bbox, nc, roots};
    if (passes > 8) {
        launch_roots(bbox, nc, roots, st);
        launch_keys(b.d_desc, b.ion_crystal, roots, ntot, k0, v0, &dsum->halt, st);
    }
    // A queued step sorts by the top digits only (the Morton levels down to
    // kSortTopLevels and the crystal) and orders each run of equal top digits
    // by (key, value): the same order as the full sort while every run is
    // short, which holds unless very many ions share a cell of that level; a
    // longer run halts the step, which is run again, and the context's later
    // queued steps sort by one digit more.
    const int first = queued && passes <= 8 ? ctx->psort_first : 0;
    const bool partial = first > 0;
    if (passes <= 8) {
        if (launch_radix_sort(k0, v0, k1, v1, ntot, passes, first, rstate, &dsum->halt, &key_src, st) == 1) {
            std::swap(k0, k1);
            std::swap(v0, v1);
        }
        if (partial) launch_sort_refine(k0, v0, ntot, 8 * first, dsum, b.d_desc, b.ion_crystal, sp, st);
        sort_err = rstate + radix_state_err();
    } else {
        for (int ps = 0; ps < passes; ++ps) {
            launch_radix_pass(k0, v0, k1, v1, ntot, 8 * ps, hist, scan_part, st);
            std::swap(k0, k1);
            std::swap(v0, v1);
        }
    }
    if (!partial) launch_gather(b.d_desc, b.ion_crystal, v0, ntot, sp, &dsum->halt, st);  // else done by the refine
    launch_tree_count(b.d_desc, k0, ntot, s, rep, box_end, bcnt, scan_part, total, sort_err, dsum, queued, bbox, nc,
                      st);
    Caps cap{};
    if (queued) {
        cap = *queued;  // the tree summary has checked the tree against it
    } else {
        PT_HIP(hipMemcpyAsync(ctx->h_sum, dsum, sizeof(TreeSummary), hipMemcpyDeviceToHost, st));
        PT_HIP(hipStreamSynchronize(st));
        const TreeSummary hs = *ctx->h_sum;
        ctx->eval_halted = hs.halt != 0;
        if (hs.halt) {
            // an earlier step of this run halted: nothing more is done (every
            // kernel would skip, and the counts read back are stale)
            for (int i = 1; i <= kPhases - 1; ++i) mark(ctx, i);
            timing_end(ctx);
            return PT_OK;
        }
        if (hs.sort_error) {
            pt_set_error("radix sort: a workgroup gave up waiting for its predecessors' digit counts");
            return PT_EDEVICE;
        }
        cap.nbox = hs.nbox;
        for (int l = 0; l <= kMaxLevel; ++l) {
            cap.lvl[l] = hs.level_start[l + 1] - hs.level_start[l];
            if (cap.lvl[l] > 0) cap.nlev = l + 1;
        }
    }
    const int nbox = cap.nbox;
    const int stride = kNeigh + 26 * std::max(0, cap.nlev - 1);
    const int Kp = kpad(p);
    const size_t esz = fp.precision == 1 ? sizeof(float) : sizeof(double);
    void *scratch;
    const char *i32names[] = {"b_level", "b_crystal", "b_begin", "b_end", "b_parent", "b_child", "b_nchild",
                              "b_ix",    "b_iy",      "b_iz",    "near_cnt"};
    for (const char *nm : i32names) PT_TRY(ws_get(ctx, nm, sizeof(int32_t) * nbox, (int32_t **)&scratch));
    PT_TRY(ws_get(ctx, "b_key", sizeof(uint64_t) * nbox, (uint64_t **)&scratch));
    PT_TRY(ws_get(ctx, "b_leaf", sizeof(uint8_t) * nbox, (uint8_t **)&scratch));
    PT_TRY(ws_get(ctx, "b_geo", sizeof(double4) * nbox, (double4 **)&scratch));
    int32_t *coll, *vtab, *near_cnt;
    int2 *near;
    void *M, *L;
    PT_TRY(ws_get(ctx, "coll", sizeof(int32_t) * kNeigh * (size_t)nbox, &coll));
    PT_TRY(ws_get(ctx, "vtab", sizeof(int32_t) * kWin * (size_t)nbox, &vtab));
    PT_TRY(ws_get(ctx, "near", sizeof(int2) * (size_t)stride * nbox, &near));
    // one extra row each (index nbox), kept at zero: the translation GEMMs
    // read it for missing sources
    PT_TRY(ws_get(ctx, "M", esz * Kp * (size_t)(nbox + 1), (char **)&M));
    PT_TRY(ws_get(ctx, "L", esz * Kp * (size_t)(nbox + 1), (char **)&L));
    near_cnt = (int32_t *)ctx->ws["near_cnt"].ptr;
    PT_TRY(ensure_tables(ctx, p));
    const BoxTable bt = box_table(ctx);
    launch_tree_build(b.d_desc, roots, k0, ntot, s, rep, box_end, bcnt, bt, dsum, nbox, st);
    // P2M needs only the boxes and the sorted positions: it runs on the
    // second stream while the lists are built and the work-item count is read
    // back; M2M waits for it
    PT_HIP(hipEventRecord(ctx->ev_tree, st));
    PT_HIP(hipStreamWaitEvent(ctx->near_stream, ctx->ev_tree, 0));
    if (fp.precision == 1)
        launch_p2m<float>(bt, dsum, sp, ntot, p, nbox, ctx->tables.rec_f, (float *)M, s, ctx->near_stream);
    else
        launch_p2m<double>(bt, dsum, sp, ntot, p, nbox, ctx->tables.rec_d, (double *)M, s, ctx->near_stream);
    PT_HIP(hipEventRecord(ctx->ev_p2m, ctx->near_stream));
    int32_t *child_oct, *parent_oct, *src_items;
    uint32_t *item_off;
    PT_TRY(ws_get(ctx, "child_oct", sizeof(int32_t) * 8 * (size_t)nbox, &child_oct));
    PT_TRY(ws_get(ctx, "parent_oct", sizeof(int32_t) * 8 * (size_t)nbox, &parent_oct));
    int32_t *l2l_list;
    PT_TRY(ws_get(ctx, "l2l_list", sizeof(int32_t) * 8 * (size_t)nbox, &l2l_list));
    PT_TRY(ws_get(ctx, "item_off", sizeof(uint32_t) * (size_t)nbox, &item_off));
    PT_TRY(ws_get(ctx, "src_items", sizeof(int32_t) * (size_t)nbox, &src_items));
    int64_t *near_pairs;
    PT_TRY(ws_get(ctx, "near_pairs", sizeof(int64_t) * (size_t)nbox, &near_pairs));
    double *near_ext;
    PT_TRY(ws_get(ctx, "near_ext", sizeof(double) * (size_t)nbox, &near_ext));
    int32_t *cuts;
    PT_TRY(ws_get(ctx, "p2p_cuts", sizeof(int32_t) * (size_t)stride * nbox, &cuts));
    uint32_t *m2l_pcnt, *m2l_cnt_ob, *m2l_op_total;
    PT_TRY(ws_get(ctx, "m2l_pcnt", sizeof(uint32_t) * (size_t)nbox, &m2l_pcnt));
    PT_TRY(ws_get(ctx, "m2l_cnt_ob", sizeof(uint32_t) * (size_t)m2l_ops() * nbox, &m2l_cnt_ob));
    PT_TRY(ws_get(ctx, "m2l_op_total", sizeof(uint32_t) * (size_t)m2l_op_total_words(), &m2l_op_total));
    int32_t *m2l_ops_tab;
    PT_TRY(ws_get(ctx, "m2l_ops_tab", sizeof(int32_t) * 2 * (m2l_ops() + 1), &m2l_ops_tab));
    int32_t *m2l_op_beg = m2l_ops_tab, *m2l_chunk_off = m2l_ops_tab + m2l_ops() + 1;
    int32_t *p2p_queue;
    PT_TRY(ws_get(ctx, "p2p_queue", sizeof(uint64_t), &p2p_queue));
    {
        // zeroed by the list builders: the zero rows of M and L (read for
        // absent sources), the near-field item queue and the M2L operator
        // totals
        ZeroRegions zr{};
        zr.p[0] = (uint64_t *)((char *)M + esz * Kp * (size_t)nbox);
        zr.p[1] = (uint64_t *)((char *)L + esz * Kp * (size_t)nbox);
        zr.p[2] = (uint64_t *)p2p_queue;
        zr.p[3] = (uint64_t *)m2l_op_total;
        zr.n[0] = zr.n[1] = (int)(esz * Kp / 8);
        zr.n[2] = 1;
        zr.n[3] = m2l_op_total_words() / 2;
        launch_lists(bt, dsum, nbox, coll, vtab, stride, near, near_cnt, near_pairs, child_oct, parent_oct, l2l_cnt,
                     l2l_list, zr, item_off, src_items, cuts, ctx->tables.slots, m2l_pcnt, m2l_cnt_ob, m2l_op_total,
                     near_ext, st);
    }
    // M2L pairs: counted with the lists and scanned here, so that their
    // number comes back with the near-field item count
    unsigned long long *near_total;
    PT_TRY(ws_get(ctx, "near_total", sizeof(unsigned long long), &near_total));
    launch_list_scans(dsum, nbox, m2l_pcnt, m2l_cnt_ob, m2l_op_total, total + 2, item_off, total + 1, m2l_op_beg,
                      m2l_chunk_off, near_pairs, near_total, st);
    // near-field work items and M2L pairs: their numbers size the item,
    // partial and pair buffers.  Measuring, they are read back (the host waits
    // for an event right after the copy, not for the stream); queued, the
    // item writer checks them against the capacities and halts the run on
    // overflow.
    if (!queued) {
        PT_HIP(hipMemcpyAsync(ctx->h_counters, total + 1, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        PT_HIP(hipMemcpyAsync(ctx->h_counters + 1, near_total, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        PT_HIP(hipEventRecord(ctx->ev_read, st));
    }
    void *xl_part;
    const int ngroup = m2l_groups(0);
    PT_TRY(ws_get(ctx, "xl_part", esz * Kp * (size_t)nbox * ngroup, (char **)&xl_part));
    mark(ctx, 1);
    const Tables &tb = ctx->tables;
    if (!queued) {
        PT_HIP(hipEventSynchronize(ctx->ev_read));
        cap.items = (int)((uint32_t *)ctx->h_counters)[0];
        cap.pairs = (int)((uint32_t *)ctx->h_counters)[1];
        // which branch of an early split stays on the main stream, for this
        // evaluation and the batch's queued steps
        ctx->near_first = (double)ctx->h_counters[1] > kNearFirstRatio * (double)cap.pairs ||
                          (double)cap.pairs < kNearFirstPairs;
    }
    const int n_items = cap.items, n_pairs = cap.pairs;
    int4 *work, *m2l_bucket;
    void *m2l_R;
    PT_TRY(ws_get(ctx, "m2l_bucket", sizeof(int4) * (size_t)std::max(1, n_pairs), &m2l_bucket));
    PT_TRY(ws_get(ctx, "m2l_R", esz * Kp * (size_t)std::max(1, n_pairs), (char **)&m2l_R));
    void *ppart;
    PT_TRY(ws_get(ctx, "p2p_work", sizeof(int4) * (size_t)std::max(1, n_items), &work));
    const int ncomp = phi ? 4 : 3;  // near-field partial components per target
    PT_TRY(ws_get(ctx, "p2p_part", esz * 64 * ncomp * (size_t)std::max(1, n_items), (char **)&ppart));
    launch_p2p_items(bt, dsum, nbox, near_cnt, stride, item_off, src_items, cuts, work, total, queued, st);
    auto run = [&](auto tag) -> pt_status {
        using T = decltype(tag);
        const bool f = sizeof(T) == sizeof(float);
        const T *m2m = f ? (const T *)tb.m2m_f : (const T *)tb.m2m_d;
        const T *m2l = f ? (const T *)tb.m2l_f : (const T *)tb.m2l_d;  // row-major base operators
        const T *l2l = f ? (const T *)tb.l2l_f : (const T *)tb.l2l_d;
        const T *rec = f ? (const T *)tb.rec_f : (const T *)tb.rec_d;
        // near field on its own stream, concurrently with M2L and L2L (vector
        // ALUs beside matrix cores) when leaves are large enough for the near
        // field to rival the far field, joining before L2P; the far-field
        // kernels beside it raise their wave priority.  It needs only the
        // sorted positions and its work items: in the mixed form it forks as
        // soon as those exist (after P2M on its stream), beside the upward
        // pass too; the FP64 near field's registers leave no room for the
        // upward pass's workgroups, so there it forks after the upward pass
        // (measured, both).  With small leaves M2L dominates and sharing the
        // chip only slows it: the near field then runs after L2L on the main
        // stream.
        const bool concurrent = ctx->near_concurrent > 0 || (ctx->near_concurrent < 0 && s >= kConcurrentLeaf);
        const bool early = concurrent && (ctx->near_early >= 0 ? ctx->near_early > 0 : f);
        // beside the near field, a kick that follows can add the near-field
        // partials itself (the last far-field launch then falls away)
        int2 *poff = nullptr;
        if (leave && concurrent && !phi) PT_TRY(ws_get(ctx, "poff", sizeof(int2) * (size_t)ntot, &poff));
        auto finish = [&]() {
            if (poff)
                *leave = KickPartials{ppart, poff, f ? 1 : 0};
            else
                launch_far<T>(bt, dsum, sp, ntot, p, nbox, (const T *)L, rec, item_off, src_items, (const T *)ppart,
                              v0, E, phi, s, concurrent ? 2 : 0, st);
        };
        const int near_cap = ctx->near_per_cu > 0 ? ctx->near_per_cu : early ? kNearPerCUEarly : kNearPerCUConcurrent;
        hipStream_t ns = concurrent ? ctx->near_stream : st;
        // translations that leave room for their waves beside a large near field
        const bool narrow = f && concurrent && near_cap >= 4;
        // M2L workgroups of fewer row blocks beside a near field that
        // outweighs M2L (the batch has fewer than kNearFirstPairs V pairs):
        // three fit a compute unit beside it and keep pace at any share;
        // with many V pairs M2L is the longer branch and the larger row
        // groups reload each operator fewer times (measured both ways)
        const int m2l_rb = concurrent && (double)n_pairs < kNearFirstPairs ? kM2LSmallRowBlocks : kM2LMaxRowBlocks;
        auto near_field = [&](hipStream_t on) -> pt_status {
            if (ctx->timing) PT_HIP(hipEventRecord(ctx->ev_near[ctx->ring_cur][0], on));
            const int max_grid = concurrent ? near_cap * ctx->num_cu : 16384;
            // beside the far field the grid is capped and the workgroups take
            // items from a queue; alone, one workgroup per item (no queue: its
            // atomics would serialise over the many small items of small leaves)
            launch_near<T>(bt, dsum, sp, ntot, near, stride, work, total + 1, n_items, (T *)ppart, phi != nullptr,
                           max_grid, concurrent ? p2p_queue : nullptr, near_ext, on);
            if (ctx->timing) PT_HIP(hipEventRecord(ctx->ev_near[ctx->ring_cur][1], on));
            ctx->near_timed[ctx->ring_cur] = ctx->timing;
            return PT_OK;
        };
        if (early && (ctx->near_main > 0 || (ctx->near_main < 0 && ctx->near_first))) {
            // forking before the upward pass: the far field goes to the second
            // stream (after P2M there) and the near field stays on the main
            // stream, right after its work items, so the branch that decides
            // the step starts without waiting for a fork (measured: a few per
            // cent; forking after the upward pass, the FP64 form, keeps the
            // near field on the second stream, which is faster there)
            PT_HIP(hipEventRecord(ctx->ev_fork, st));
            PT_HIP(hipStreamWaitEvent(ns, ctx->ev_fork, 0));
            // the near field is submitted first, so that a host slower than
            // the device (a profiler, say) does not hold it back behind the
            // far branch's launches
            PT_TRY(near_field(st));
            launch_m2m<T>(bt, dsum, p, cap, m2m, tb.oct_slots, child_oct, (T *)M, (T *)xl_part, narrow, ns);
            launch_m2l_emit(bt, dsum, nbox, vtab, ctx->tables.slots, m2l_pcnt, m2l_cnt_ob, m2l_bucket, ns);
            mark(ctx, 2, ns);
            const int m2l_grid = ctx->num_cu * m2l_per_cu<T>(Kp, m2l_rb, near_cap * near_lds_bytes());
            launch_m2l_gemm<T>(dsum, Kp, m2l_rb, nbox, m2l_grid, m2l_chunk_off, m2l_op_beg, m2l_bucket, m2l, (const T *)M,
                               (T *)m2l_R, ns);
            mark(ctx, 3, ns);
            launch_m2l_sum<T>(dsum, nbox, Kp, m2l_pcnt, total + 2, (const T *)m2l_R, (T *)L, ns);
            launch_downward<T>(bt, dsum, p, cap, l2l, tb.oct_slots, parent_oct, l2l_cnt, l2l_list, (T *)L, narrow, ns);
            mark(ctx, 4, ns);
            launch_far<T>(bt, dsum, sp, ntot, p, nbox, (const T *)L, rec, item_off, src_items, (const T *)ppart, v0, E,
                          phi, s, 1, ns, poff);
            mark(ctx, 5, ns);
            PT_HIP(hipEventRecord(ctx->ev_join, ns));
            PT_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0));
            finish();
            return PT_OK;
        }
        auto fork = [&]() -> pt_status {
            PT_HIP(hipEventRecord(ctx->ev_fork, st));
            PT_HIP(hipStreamWaitEvent(ns, ctx->ev_fork, 0));
            PT_TRY(near_field(ns));
            PT_HIP(hipEventRecord(ctx->ev_join, ns));
            return PT_OK;
        };
        if (early) PT_TRY(fork());
        // upward pass (after P2M on the second stream), then the M2L buckets
        PT_HIP(hipStreamWaitEvent(st, ctx->ev_p2m, 0));
        launch_m2m<T>(bt, dsum, p, cap, m2m, tb.oct_slots, child_oct, (T *)M, (T *)xl_part, narrow, st);
        launch_m2l_emit(bt, dsum, nbox, vtab, ctx->tables.slots, m2l_pcnt, m2l_cnt_ob, m2l_bucket, st);
        if (concurrent && !early) PT_TRY(fork());
        mark(ctx, 2);
        const int m2l_grid =
            ctx->num_cu * m2l_per_cu<T>(Kp, m2l_rb, concurrent ? near_cap * near_lds_bytes() : 0);
        launch_m2l_gemm<T>(dsum, Kp, m2l_rb, nbox, m2l_grid, m2l_chunk_off, m2l_op_beg, m2l_bucket, m2l, (const T *)M,
                           (T *)m2l_R, st);
        mark(ctx, 3);
        launch_m2l_sum<T>(dsum, nbox, Kp, m2l_pcnt, total + 2, (const T *)m2l_R, (T *)L, st);
        launch_downward<T>(bt, dsum, p, cap, l2l, tb.oct_slots, parent_oct, l2l_cnt, l2l_list, (T *)L, narrow, st);
        mark(ctx, 4);
        if (!concurrent) {
            PT_TRY(near_field(st));
        } else {
            // beside the near field, the far field of every ion is evaluated
            // before the join and the near-field partials added after it
            launch_far<T>(bt, dsum, sp, ntot, p, nbox, (const T *)L, rec, item_off, src_items, (const T *)ppart, v0,
                          E, phi, s, 1, st, poff);
        }
        mark(ctx, 5);
        if (concurrent) PT_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0));
        finish();
        return PT_OK;
    };
    PT_TRY(fp.precision == 1 ? run(float(0)) : run(double(0)));
    mark(ctx, 6);
    timing_end(ctx);
    if (!queued) ctx->measured = cap;
    ctx->last_cap = cap;
    ctx->last_stride = stride;
    ctx->last_p = p;
    ctx->last_prec = fp.precision;
    ctx->last_keys = k0;  // the ping-pong buffer holding the sorted result
    ctx->last_vals = v0;
    return PT_OK;
}

// The device summary of the last FMM evaluation (waits for the stream).
static pt_status read_summary(pt_ctx *ctx, TreeSummary &out)
{
    PT_HIP(hipStreamSynchronize(ctx->stream));
    PT_HIP(hipMemcpy(&out, ctx->ws["sum"].ptr, sizeof(TreeSummary), hipMemcpyDeviceToHost));
    return PT_OK;
}

// Adds the phase times of every recorded evaluation to the running sums.
static pt_status finish_timing(pt_ctx *ctx)
{
    while (ctx->ring_pending > 0) PT_TRY(collect_oldest(ctx));
    return PT_OK;
}

// ---------------------------------------------------------------- validation

static bool finite_all(const double *a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

static pt_status check_trap(const pt_crystal *c, const pt_trap_params *p)
{
    PT_REQUIRE(p, "trap params NULL");
    const double v[7] = {p->B_T, p->omega_z, p->delta, p->omega_r, p->dt_s, p->t0_s, p->damping_per_s};
    PT_REQUIRE(finite_all(v, 7), "trap params must be finite");
    PT_REQUIRE(p->damping_per_s >= 0.0, "damping must be >= 0");
    PT_REQUIRE(p->dt_s > 0.0, "dt must be > 0");
    PT_REQUIRE(p->omega_z >= 0.0, "omega_z must be >= 0");
    const double wc = c->q * p->B_T / c->m;
    PT_REQUIRE(p->omega_z == 0.0 || wc * wc > 2.0 * p->omega_z * p->omega_z,
               "trap does not confine: omega_c^2 = %g <= 2 omega_z^2 = %g", wc * wc,
               2.0 * p->omega_z * p->omega_z);
    return PT_OK;
}

static pt_status check_force(const pt_force_params *p)
{
    PT_REQUIRE(p, "force params NULL");
    PT_REQUIRE(p->method == 0 || p->method == 1, "method must be 0 (direct) or 1 (fmm)");
    PT_REQUIRE(p->precision == 0 || p->precision == 1, "precision must be 0 or 1");
    if (p->method == 1) {
        PT_REQUIRE(p->p >= 1 && p->p <= kMaxP, "p must be in [1, %d]", kMaxP);
        PT_REQUIRE(p->leaf_size >= 1 && p->leaf_size <= 4096, "leaf_size must be in [1, 4096]");
    }
    return PT_OK;
}

// ---------------------------------------------------------------- C ABI

extern "C" {

const char *pt_last_error(void) { return g_err; }

// Releases everything a context holds (also a partly created one).
static void release_ctx(pt_ctx *ctx)
{
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->near_stream) (void)hipStreamSynchronize(ctx->near_stream);
    for (auto &kv : ctx->allocs) (void)hipFree(kv.first);
    ctx->allocs.clear();
    if (ctx->h_desc) (void)hipHostFree(ctx->h_desc);
    if (ctx->h_sum) (void)hipHostFree(ctx->h_sum);
    if (ctx->h_fail) (void)hipHostFree(ctx->h_fail);
    for (hipEvent_t e : ctx->ev_check)
        if (e) (void)hipEventDestroy(e);
    if (ctx->h_counters) (void)hipHostFree(ctx->h_counters);
    for (auto &set : ctx->ev)
        for (auto &e : set)
            if (e) (void)hipEventDestroy(e);
    for (auto &pair : ctx->ev_near)
        for (auto &e : pair)
            if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : {ctx->ev_fork, ctx->ev_join, ctx->ev_tree, ctx->ev_p2m, ctx->ev_read})
        if (e) (void)hipEventDestroy(e);
    if (ctx->near_stream) (void)hipStreamDestroy(ctx->near_stream);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

static pt_status init_ctx(pt_ctx *ctx, void *hip_stream)
{
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        PT_HIP(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    PT_HIP(hipHostMalloc((void **)&ctx->h_sum, sizeof(TreeSummary)));
    PT_HIP(hipHostMalloc((void **)&ctx->h_fail, sizeof(int32_t) * kCheckSlots));
    for (auto &e : ctx->ev_check) PT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    PT_HIP(hipHostMalloc((void **)&ctx->h_counters, sizeof(unsigned long long) * 2));
    PT_HIP(hipStreamCreateWithFlags(&ctx->near_stream, hipStreamNonBlocking));
    if (const char *e = getenv("PT_NEAR_CONCURRENT")) ctx->near_concurrent = atoi(e) ? 1 : 0;
    if (const char *e = getenv("PT_NEAR_PER_CU")) ctx->near_per_cu = std::max(1, std::min(8, atoi(e)));
    if (const char *e = getenv("PT_NEAR_EARLY")) ctx->near_early = atoi(e) ? 1 : 0;
    if (const char *e = getenv("PT_NEAR_MAIN")) ctx->near_main = atoi(e) ? 1 : 0;
    if (const char *e = getenv("PT_PARTIAL_SORT"))
        if (!atoi(e)) {
            ctx->psort_first = 0;
            ctx->psort_off = true;
        }
    if (const char *e = getenv("PT_QUEUED_STEPS")) ctx->no_queue = atoi(e) == 0;
    if (const char *e = getenv("PT_CAPS_TIGHT")) ctx->tight_caps = atoi(e) != 0;
    PT_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    PT_HIP(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    PT_HIP(hipEventCreateWithFlags(&ctx->ev_tree, hipEventDisableTiming));
    PT_HIP(hipEventCreateWithFlags(&ctx->ev_p2m, hipEventDisableTiming));
    PT_HIP(hipEventCreateWithFlags(&ctx->ev_read, hipEventDisableTiming));
    PT_HIP(hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    ctx->num_cu = std::max(1, ctx->num_cu);
    PT_TRY(ctx_alloc(ctx, (void **)&ctx->d_nonfinite, sizeof(int32_t)));
    PT_TRY(noalloc_scratch(ctx->device, (void **)&ctx->noalloc));
    PT_HIP(hipMemsetAsync(ctx->d_nonfinite, 0, sizeof(int32_t), ctx->stream));
    PT_HIP(hipStreamSynchronize(ctx->stream));
    return PT_OK;
}

pt_status pt_ctx_create(int hip_device, uint64_t hbm_budget_bytes, void *hip_stream, pt_ctx **out)
{
    PT_REQUIRE(out, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        pt_set_error("no HIP device available");
        return PT_EDEVICE;
    }
    PT_REQUIRE(hip_device >= 0 && hip_device < ndev, "device %d out of range [0, %d)", hip_device, ndev);
    PT_HIP(hipSetDevice(hip_device));
    pt_ctx *ctx = new pt_ctx();
    ctx->device = hip_device;
    ctx->budget = hbm_budget_bytes;
    const pt_status st = init_ctx(ctx, hip_stream);
    if (st != PT_OK) {
        release_ctx(ctx);
        return st;
    }
    *out = ctx;
    return PT_OK;
}

pt_status pt_ctx_destroy(pt_ctx *ctx)
{
    PT_REQUIRE(ctx, "ctx is NULL");
    (void)settle(ctx);
    if (ctx->live > 0) {
        pt_set_error("context still owns %d crystals", ctx->live);
        return PT_EBUSY;
    }
    release_ctx(ctx);
    return PT_OK;
}

pt_status pt_ctx_memory(pt_ctx *ctx, uint64_t *bytes_in_use, uint64_t *budget)
{
    PT_REQUIRE(ctx, "ctx is NULL");
    if (bytes_in_use) *bytes_in_use = ctx->used;
    if (budget) *budget = ctx->budget;
    return PT_OK;
}

static pt_status create_common(pt_ctx *ctx, int64_t n, double charge, double mass, uint64_t seed, pt_crystal **out)
{
    PT_REQUIRE(ctx && out, "NULL argument");
    *out = nullptr;
    PT_REQUIRE(n >= 1 && n < (1ll << 30), "n must be in [1, 2^30)");
    PT_REQUIRE(std::isfinite(charge) && charge != 0.0, "charge must be finite and non-zero");
    PT_REQUIRE(std::isfinite(mass) && mass > 0.0, "mass must be finite and > 0");
    std::unique_ptr<pt_crystal> c(new pt_crystal());
    c->ctx = ctx;
    c->n = n;
    c->q = charge;
    c->m = mass;
    c->seed = seed;
    c->trap = {4.5, 2.0 * kPi * 1.5e6, 0.0, 0.0, 1e-9, 0.0, 0.0};
    if ((c->q * 4.5 / c->m) * (c->q * 4.5 / c->m) <= 2.0 * c->trap.omega_z * c->trap.omega_z) c->trap.omega_z = 0.0;
    c->laser = {0, 0.0, 313e-9};
    c->force = {0, 8, 32, 0};
    PT_HIP(hipSetDevice(ctx->device));
    PT_TRY(ctx_alloc(ctx, (void **)&c->d_state, sizeof(double) * 6 * (size_t)n));
    pt_status s = ctx_alloc(ctx, (void **)&c->d_photons, sizeof(int32_t) * (size_t)n);
    if (s == PT_OK) s = ctx_alloc(ctx, (void **)&c->d_nonfinite, sizeof(int32_t));
    if (s != PT_OK) {
        ctx_free(ctx, c->d_state);
        ctx_free(ctx, c->d_photons);
        return s;
    }
    PT_HIP(hipMemsetAsync(c->d_photons, 0, sizeof(int32_t) * n, ctx->stream));
    PT_HIP(hipMemsetAsync(c->d_nonfinite, 0, sizeof(int32_t), ctx->stream));
    *out = c.release();
    ctx->live++;
    return PT_OK;
}

// Interleaved n x 3 host array -> SoA device block (6 n doubles: pos then vel).
static pt_status upload_state(pt_crystal *c, const double *pos, const double *vel)
{
    const int64_t n = c->n;
    std::vector<double> soa(6 * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            soa[d * n + i] = pos[3 * i + d];
            soa[(3 + d) * n + i] = vel[3 * i + d];
        }
    PT_HIP(hipMemcpy(c->d_state, soa.data(), sizeof(double) * 6 * n, hipMemcpyHostToDevice));
    return PT_OK;
}

pt_status pt_create_crystal(pt_ctx *ctx, int64_t n, const double *pos_xyz, const double *vel_xyz, double charge_C,
                            double mass_kg, uint64_t seed, pt_crystal **out)
{
    PT_REQUIRE(pos_xyz && vel_xyz, "pos/vel NULL");
    PT_REQUIRE(n >= 1 && n < (1ll << 30), "n must be in [1, 2^30)");
    PT_REQUIRE(finite_all(pos_xyz, 3 * n) && finite_all(vel_xyz, 3 * n), "non-finite position or velocity");
    PT_TRY(create_common(ctx, n, charge_C, mass_kg, seed, out));
    pt_status s = upload_state(*out, pos_xyz, vel_xyz);
    if (s != PT_OK) {
        pt_destroy_crystal(*out);
        *out = nullptr;
    }
    return s;
}

pt_status pt_create_crystal_device(pt_ctx *ctx, int64_t n, const double *pos_dev, const double *vel_dev,
                                   double charge_C, double mass_kg, uint64_t seed, pt_crystal **out)
{
    PT_REQUIRE(pos_dev && vel_dev, "pos/vel NULL");
    PT_TRY(create_common(ctx, n, charge_C, mass_kg, seed, out));
    std::vector<double> p(3 * (size_t)n), v(3 * (size_t)n);
    pt_status s = PT_OK;
    if (hipMemcpyAsync(p.data(), pos_dev, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(v.data(), vel_dev, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        pt_set_error("reading device buffers failed");
        s = PT_EDEVICE;
    } else if (!finite_all(p.data(), 3 * n) || !finite_all(v.data(), 3 * n)) {
        pt_set_error("non-finite position or velocity");
        s = PT_EINVAL;
    } else {
        s = upload_state(*out, p.data(), v.data());
    }
    if (s != PT_OK) {
        pt_destroy_crystal(*out);
        *out = nullptr;
    }
    return s;
}

pt_status pt_destroy_crystal(pt_crystal *c)
{
    PT_REQUIRE(c, "crystal is NULL");
    pt_ctx *ctx = c->ctx;
    (void)settle(ctx);
    (void)hipStreamSynchronize(ctx->stream);
    if (std::find(ctx->caps_batch.begin(), ctx->caps_batch.end(), c) != ctx->caps_batch.end()) ctx->caps_ok = false;
    ctx_free(ctx, c->d_state);
    ctx_free(ctx, c->d_photons);
    ctx_free(ctx, c->d_nonfinite);
    auto &lb = ctx->last_batch;
    if (std::find(lb.begin(), lb.end(), c) != lb.end()) lb.clear();
    ctx->live--;
    delete c;
    return PT_OK;
}

// Beam mode: gamma0 dt <= 4 keeps every per-step photon mean <= 2 (the
// largest rate of eq. scattering_rate is gamma0 / 2, reached at S -> inf).
static bool beams_fit_step(const pt_laser_params &l, double dt) { return l.mode != 2 || l.gamma0 * dt <= 4.0; }

pt_status pt_set_trap_params(pt_crystal *c, const pt_trap_params *p)
{
    PT_REQUIRE(c, "crystal is NULL");
    PT_TRY(settle(c->ctx));
    PT_TRY(check_trap(c, p));
    PT_REQUIRE(beams_fit_step(c->laser, p->dt_s), "gamma0 dt = %g exceeds 4 with the crystal's laser beams",
               c->laser.gamma0 * p->dt_s);
    c->trap = *p;
    return PT_OK;
}

pt_status pt_set_laser_params(pt_crystal *c, const pt_laser_params *p)
{
    PT_REQUIRE(c && p, "NULL argument");
    PT_TRY(settle(c->ctx));
    PT_REQUIRE(p->mode >= 0 && p->mode <= 2, "laser mode must be 0, 1 or 2");
    if (p->mode == 1) {
        PT_REQUIRE(std::isfinite(p->mean_per_step) && p->mean_per_step >= 0.0 && p->mean_per_step <= 2.0,
                   "photon mean must be in [0, 2]");
        PT_REQUIRE(std::isfinite(p->wavelength_m) && p->wavelength_m > 0.0, "wavelength must be > 0");
    }
    if (p->mode == 2) {
        PT_REQUIRE(std::isfinite(p->wavelength_m) && p->wavelength_m > 0.0, "wavelength must be > 0");
        PT_REQUIRE(std::isfinite(p->gamma0) && p->gamma0 > 0.0, "gamma0 must be > 0");
        PT_REQUIRE(p->n_beams >= 1 && p->n_beams <= PT_MAX_BEAMS, "n_beams must be in [1, %d]", PT_MAX_BEAMS);
        for (int l = 0; l < p->n_beams; ++l) {
            const pt_beam &b = p->beam[l];
            const double v[7] = {b.khat[0], b.khat[1], b.khat[2], b.detuning, b.s0, b.waist_y, b.offset_y};
            PT_REQUIRE(finite_all(v, 7) && std::isfinite(b.waist_z), "beam %d: non-finite parameter", l);
            PT_REQUIRE(b.khat[0] != 0.0 || b.khat[1] != 0.0 || b.khat[2] != 0.0, "beam %d: khat is zero", l);
            PT_REQUIRE(b.s0 >= 0.0, "beam %d: s0 must be >= 0", l);
            PT_REQUIRE(b.uniform || (b.waist_y > 0.0 && b.waist_z > 0.0), "beam %d: waists must be > 0", l);
        }
        PT_REQUIRE(beams_fit_step(*p, c->trap.dt_s), "gamma0 dt = %g exceeds 4 (photon means above 2 per step)",
                   p->gamma0 * c->trap.dt_s);
    }
    c->laser = *p;
    return PT_OK;
}

pt_status pt_set_force_params(pt_crystal *c, const pt_force_params *p)
{
    PT_REQUIRE(c, "crystal is NULL");
    PT_TRY(settle(c->ctx));
    PT_TRY(check_force(p));
    c->force = *p;
    return PT_OK;
}

pt_status pt_set_state(pt_crystal *c, const double *pos, const double *vel, int64_t step)
{
    PT_REQUIRE(c && pos && vel, "NULL argument");
    PT_REQUIRE(step >= 0, "step must be >= 0");
    PT_REQUIRE(finite_all(pos, 3 * c->n) && finite_all(vel, 3 * c->n), "non-finite position or velocity");
    PT_TRY(settle(c->ctx));
    PT_HIP(hipStreamSynchronize(c->ctx->stream));
    PT_TRY(upload_state(c, pos, vel));
    PT_HIP(hipMemset(c->d_nonfinite, 0, sizeof(int32_t)));
    c->step = step;
    return PT_OK;
}

static bool same_force(const pt_force_params &a, const pt_force_params &b)
{
    if (a.method != b.method) return false;
    if (a.method == 0) return true;
    return a.p == b.p && a.leaf_size == b.leaf_size && a.precision == b.precision;
}

static pt_status check_batch(pt_crystal *const *cs, int nc)
{
    PT_REQUIRE(cs && nc >= 1, "empty batch");
    for (int i = 0; i < nc; ++i) {
        PT_REQUIRE(cs[i], "crystal %d is NULL", i);
        PT_REQUIRE(cs[i]->ctx == cs[0]->ctx, "crystals of one batch must share the context");
        PT_REQUIRE(same_force(cs[i]->force, cs[0]->force), "crystals of one batch must share force parameters");
        for (int j = 0; j < i; ++j) PT_REQUIRE(cs[j] != cs[i], "crystal %d appears twice", i);
    }
    return PT_OK;
}

// One Coulomb evaluation of a batch at its current positions: forces (F_out),
// potentials (phi_out), Coulomb energies (U_out) and / or rotating-frame
// diagnostics (diag), each optional.
static pt_status evaluate_batch(pt_crystal *const *cs, int n_crystals, double *const *F_out, double *const *phi_out,
                                double *U_out, pt_diagnostics *diag = nullptr)
{
    std::vector<double> U_diag;
    if (diag && !U_out) {
        U_diag.resize((size_t)n_crystals);
        U_out = U_diag.data();
    }
    pt_ctx *ctx = cs[0]->ctx;
    PT_TRY(settle(ctx));
    PT_HIP(hipSetDevice(ctx->device));
    if (cs[0]->force.method == 1) {  // a fresh run state for the measuring evaluation
        TreeSummary *dsum;
        PT_TRY(ws_get(ctx, "sum", sizeof(TreeSummary), &dsum));
        launch_run_reset(dsum, ctx->stream);
    }
    Batch b;
    PT_TRY(form_batch(ctx, std::vector<pt_crystal *>(cs, cs + n_crystals), b));
    double *E, *phi = nullptr, *usum = nullptr;
    PT_TRY(ws_get(ctx, "E", sizeof(double) * 3 * (size_t)b.ntot, &E));
    if (phi_out || U_out) PT_TRY(ws_get(ctx, "phi", sizeof(double) * (size_t)std::max(1, b.ntot), &phi));
    if (U_out) PT_TRY(ws_get(ctx, "phi_sum", sizeof(double) * (size_t)n_crystals, &usum));
    PT_TRY(eval_field(ctx, b, cs[0]->force, E, phi, nullptr, 0, false));
    std::vector<double> h, hp, hu;
    if (F_out) {
        h.resize(3 * (size_t)b.ntot);
        PT_HIP(hipMemcpyAsync(h.data(), E, sizeof(double) * 3 * b.ntot, hipMemcpyDeviceToHost, ctx->stream));
    }
    if (phi_out) {
        hp.resize((size_t)b.ntot);
        PT_HIP(hipMemcpyAsync(hp.data(), phi, sizeof(double) * b.ntot, hipMemcpyDeviceToHost, ctx->stream));
    }
    if (U_out) {
        double *ppart;
        PT_TRY(ws_get(ctx, "phi_part", sizeof(double) * (size_t)std::max(1, b.nblk_sum), &ppart));
        launch_phi_sum(b.d_desc, b.blk_crystal, b.blk_first, b.nblk_sum, n_crystals, phi, ppart, usum, ctx->stream);
        hu.resize((size_t)n_crystals);
        PT_HIP(hipMemcpyAsync(hu.data(), usum, sizeof(double) * n_crystals, hipMemcpyDeviceToHost, ctx->stream));
    }
    std::vector<double> hr;
    if (diag) {
        double *rsum, *rpart;
        PT_TRY(ws_get(ctx, "rot_sum", sizeof(double) * 3 * (size_t)n_crystals, &rsum));
        PT_TRY(ws_get(ctx, "rot_part", sizeof(double) * 3 * (size_t)std::max(1, b.nblk_sum), &rpart));
        launch_rot_sums(b.d_desc, b.blk_crystal, b.blk_first, b.nblk_sum, n_crystals, rpart, rsum, ctx->stream);
        hr.resize(3 * (size_t)n_crystals);
        PT_HIP(hipMemcpyAsync(hr.data(), rsum, sizeof(double) * 3 * n_crystals, hipMemcpyDeviceToHost, ctx->stream));
    }
    PT_HIP(hipStreamSynchronize(ctx->stream));
    PT_TRY(finish_timing(ctx));
    for (int c = 0; c < n_crystals; ++c) {
        const double ke = 1.0 / (4.0 * kPi * kEps0), q = cs[c]->q;
        const int off = b.off[c];
        if (F_out)
            for (int64_t i = 0; i < cs[c]->n; ++i)
                for (int d = 0; d < 3; ++d) F_out[c][3 * i + d] = ke * q * q * h[(size_t)d * b.ntot + off + i];
        if (phi_out)
            for (int64_t i = 0; i < cs[c]->n; ++i) phi_out[c][i] = ke * q * hp[(size_t)off + i];
        if (U_out) U_out[c] = 0.5 * ke * q * q * hu[c];
        if (diag) {
            pt_diagnostics &d = diag[c];
            const double nkb = (double)cs[c]->n * kBoltzmann;
            d.t = cs[c]->trap.t0_s + (double)cs[c]->step * cs[c]->trap.dt_s;
            d.ke_axial = hr[3 * c];
            d.ke_planar = hr[3 * c + 1];
            d.pe_external = hr[3 * c + 2];
            d.pe_coulomb = U_out[c];
            d.energy = d.ke_axial + d.ke_planar + d.pe_external + d.pe_coulomb;
            d.temp_axial = 2.0 * d.ke_axial / nkb;
            d.temp_planar = d.ke_planar / nkb;
        }
    }
    return PT_OK;
}

pt_status pt_compute_forces_batch(pt_crystal *const *cs, int n_crystals, double *const *F_out)
{
    PT_TRY(check_batch(cs, n_crystals));
    PT_REQUIRE(F_out, "F_out NULL");
    for (int i = 0; i < n_crystals; ++i) PT_REQUIRE(F_out[i], "F_out[%d] NULL", i);
    return evaluate_batch(cs, n_crystals, F_out, nullptr, nullptr);
}

pt_status pt_compute_potential_batch(pt_crystal *const *cs, int n_crystals, double *const *phi_out)
{
    PT_TRY(check_batch(cs, n_crystals));
    PT_REQUIRE(phi_out, "phi_out NULL");
    for (int i = 0; i < n_crystals; ++i) PT_REQUIRE(phi_out[i], "phi_out[%d] NULL", i);
    return evaluate_batch(cs, n_crystals, nullptr, phi_out, nullptr);
}

pt_status pt_compute_potential(pt_crystal *c, double *phi_out)
{
    return pt_compute_potential_batch(&c, 1, &phi_out);
}

pt_status pt_coulomb_energy_batch(pt_crystal *const *cs, int n_crystals, double *U_out)
{
    PT_TRY(check_batch(cs, n_crystals));
    PT_REQUIRE(U_out, "U_out NULL");
    return evaluate_batch(cs, n_crystals, nullptr, nullptr, U_out);
}

pt_status pt_coulomb_energy(pt_crystal *c, double *U_out) { return pt_coulomb_energy_batch(&c, 1, U_out); }

pt_status pt_rotating_diagnostics_batch(pt_crystal *const *cs, int n_crystals, pt_diagnostics *out)
{
    PT_TRY(check_batch(cs, n_crystals));
    PT_REQUIRE(out, "out NULL");
    return evaluate_batch(cs, n_crystals, nullptr, nullptr, nullptr, out);
}

pt_status pt_rotating_diagnostics(pt_crystal *c, pt_diagnostics *out)
{
    return pt_rotating_diagnostics_batch(&c, 1, out);
}

pt_status pt_read_rotating_state(pt_crystal *c, double *pos_r, double *vel_r)
{
    PT_REQUIRE(c, "crystal is NULL");
    pt_ctx *ctx = c->ctx;
    PT_TRY(settle(ctx));
    PT_HIP(hipSetDevice(ctx->device));
    Batch b;
    PT_TRY(form_batch(ctx, std::vector<pt_crystal *>{c}, b));
    double *rs;
    PT_TRY(ws_get(ctx, "rot_state", sizeof(double) * 6 * (size_t)b.ntot, &rs));
    launch_rot_state(b.d_desc, b.ion_crystal, b.ntot, rs, ctx->stream);
    std::vector<double> h(6 * (size_t)b.ntot);
    PT_HIP(hipMemcpyAsync(h.data(), rs, sizeof(double) * 6 * b.ntot, hipMemcpyDeviceToHost, ctx->stream));
    PT_HIP(hipStreamSynchronize(ctx->stream));
    for (int64_t i = 0; i < c->n; ++i)
        for (int d = 0; d < 3; ++d) {
            if (pos_r) pos_r[3 * i + d] = h[(size_t)d * b.ntot + i];
            if (vel_r) vel_r[3 * i + d] = h[(size_t)(3 + d) * b.ntot + i];
        }
    return PT_OK;
}

pt_status pt_compute_forces(pt_crystal *c, double *F_out)
{
    return pt_compute_forces_batch(&c, 1, &F_out);
}

// The direct-sum path of pt_compute_forces on the device's fixed scratch:
// every work buffer is a region of that array, the descriptor and block table
// are written by a kernel, and the forces go to the caller's device buffer.
pt_status pt_compute_forces_noalloc(pt_crystal *c, double *F_dev)
{
    PT_REQUIRE(c && F_dev, "NULL argument");
    PT_REQUIRE(c->force.method == 0, "pt_compute_forces_noalloc supports the direct method only");
    PT_REQUIRE(c->n <= kNoAllocMaxIons, "n = %lld exceeds the no-allocation limit of %d ions", (long long)c->n,
               kNoAllocMaxIons);
    pt_ctx *ctx = c->ctx;
    PT_TRY(settle(ctx));  // steps still pending are completed first
    const int n = (int)c->n;
    const NoAllocLayout l = noalloc_layout(n);
    PT_REQUIRE(l.total <= kNoAllocScratchBytes, "scratch layout of %zu bytes exceeds %zu", l.total,
               kNoAllocScratchBytes);
    PT_HIP(hipSetDevice(ctx->device));
    char *base = ctx->noalloc;
    CrystalDev d;
    fill_desc(c, 0, (double *)(base + l.mid), d);
    CrystalDev *desc = (CrystalDev *)(base + l.desc);
    int32_t *ion_crystal = (int32_t *)(base + l.ion_crystal);
    DirBlock *tab = (DirBlock *)(base + l.tab);
    unsigned long long *bbox = (unsigned long long *)(base + l.bbox);
    double *part = (double *)(base + l.part), *E = (double *)(base + l.E);
    hipStream_t st = ctx->stream;
    d.dpart = 0;
    launch_noalloc_setup(d, desc, ion_crystal, n, tab, l.nblk, st);
    launch_bbox_reset(bbox, 1, st);
    launch_drift_bbox(desc, ion_crystal, n, 1, 0, bbox, nullptr, ZeroRegions{}, st);
    launch_direct(desc, tab, l.nblk, ion_crystal, n, part, E, nullptr, st);
    const double ke = 1.0 / (4.0 * kPi * kEps0), q = c->q;
    launch_scale_field(E, n, ke * q * q, F_dev, st);
    PT_HIP(hipGetLastError());
    return PT_OK;
}

// Queues n_steps[i] steps of crystal i (all of one context and force
// parameters).  With the FMM, the first evaluation of a batch that has no
// valid capacities measures its counts (two host waits); the following steps
// are queued on capacities grown from them, with no host wait.  The outcome
// is read back by settle() at the context's next call.
// Whether `sub` is `all` with some crystals left out (order kept).
static bool ordered_subset(const std::vector<pt_crystal *> &sub, const std::vector<pt_crystal *> &all)
{
    size_t j = 0;
    for (pt_crystal *c : sub) {
        while (j < all.size() && all[j] != c) ++j;
        if (j == all.size()) return false;
        ++j;
    }
    return true;
}

static pt_status step_run(pt_ctx *ctx, pt_crystal *const *cs, int n_crystals, const int64_t *n_steps)
{
    int64_t kmax = 0;
    for (int i = 0; i < n_crystals; ++i) kmax = std::max(kmax, n_steps[i]);
    PT_HIP(hipSetDevice(ctx->device));
    const pt_force_params fp = cs[0]->force;
    const bool fmm = fp.method == 1;
    TreeSummary *dsum = nullptr;
    if (fmm) {
        PT_TRY(ws_get(ctx, "sum", sizeof(TreeSummary), &dsum));
        launch_run_reset(dsum, ctx->stream);
    }
    ctx->pending.active = true;
    ctx->pending.cs.assign(cs, cs + n_crystals);
    ctx->pending.n_steps.assign(n_steps, n_steps + n_crystals);
    ctx->pending.step_start.resize(n_crystals);
    for (int i = 0; i < n_crystals; ++i) ctx->pending.step_start[i] = cs[i]->step;
    Batch b;
    int formed_for = -1;
    int64_t group_start = 0;  // step at which the current batch was formed
    int drift = 1;            // 2: the previous kick made this step's first half drift
    int checks = 0, looked = 0;  // run-state copies issued, and looked at
    // Each crystal's step counter advances as its steps are queued, so that
    // after a failure it counts exactly the completed steps; a step that
    // fails before its kick leaves the state as it was (the half drift and
    // everything up to the kick work on a copy).
    for (int64_t k = 0; k < kmax; ++k) {
        if (fmm && k > 0 && k % kCheckEvery == 0) {
            // look at the copies that have landed, waiting only for those more
            // than kCheckAhead checks back (the host stays at most that many
            // segments ahead of the device, which keeps as many queued), then
            // issue one
            bool halted = false;
            while (looked < checks && !halted) {
                const int sl = looked % kCheckSlots;
                if (checks - looked > kCheckAhead) {
                    PT_HIP(hipEventSynchronize(ctx->ev_check[sl]));
                } else {
                    const hipError_t q = hipEventQuery(ctx->ev_check[sl]);
                    if (q == hipErrorNotReady) break;
                    PT_HIP(q);
                }
                halted = ctx->h_fail[sl] >= 0;
                ++looked;
            }
            if (halted) break;  // the next call re-runs from the halted step (settle)
            if (checks - looked < kCheckSlots) {
                const int sl = checks % kCheckSlots;
                PT_HIP(hipMemcpyAsync(ctx->h_fail + sl, &dsum->fail_step, sizeof(int32_t), hipMemcpyDeviceToHost,
                                      ctx->stream));
                PT_HIP(hipEventRecord(ctx->ev_check[sl], ctx->stream));
                ++checks;
            }
        }
        // crystals still stepping; the batch is re-formed only when one finishes
        int nactive = 0;
        for (int i = 0; i < n_crystals; ++i) nactive += n_steps[i] > k;
        if (nactive != formed_for) {
            std::vector<pt_crystal *> act;
            for (int i = 0; i < n_crystals; ++i)
                if (n_steps[i] > k) act.push_back(cs[i]);
            // descriptors hold the step index of the first step of this group
            PT_TRY(form_batch(ctx, act, b));
            formed_for = nactive;
            group_start = k;
            drift = 1;
        }
        double *E;
        PT_TRY(ws_get(ctx, "E", sizeof(double) * 3 * (size_t)b.ntot, &E));
        // queued on the capacities measured for this batch or for one it is
        // part of (crystals that finished their steps drop out: every count a
        // capacity bounds is a sum or maximum over the crystals)
        const bool queued = fmm && ctx->caps_ok && b.ntot <= ctx->caps_ntot && same_force(ctx->caps_force, fp) &&
                            ordered_subset(b.cs, ctx->caps_batch);
        ctx->eval_halted = false;
        KickPartials kp{};
        PT_TRY(eval_field(ctx, b, fp, E, nullptr, queued ? &ctx->caps : nullptr, drift, fmm, &kp));
        if (fmm) (queued ? ctx->n_queued : ctx->n_measured)++;
        if (fmm && !queued && !ctx->eval_halted) {
            // the slack grown by overflows belongs to the batch that overflowed:
            // a batch of other crystals (or other force parameters) starts anew
            if (!ordered_subset(b.cs, ctx->caps_batch) || !same_force(ctx->caps_force, fp)) {
                ctx->caps_slack = kCapsSlack;
                if (!ctx->psort_off) ctx->psort_first = kPsortFirst;  // and the sort's depth
            }
            ctx->caps = grow_caps(ctx->measured, ctx->caps_slack);
            if (ctx->tight_caps) ctx->caps.nbox = std::max(1, ctx->measured.nbox - 1);
            ctx->caps_batch = b.cs;
            ctx->caps_ntot = b.ntot;
            ctx->caps_force = fp;
            ctx->caps_ok = !ctx->no_queue;
        }
        // step index = descriptor step0 (set when the batch formed) + kstep;
        // when the next step keeps this batch, the kick also makes its first
        // half drift and bounding boxes (one launch fewer per step)
        int next_active = 0;
        for (int i = 0; i < n_crystals; ++i) next_active += n_steps[i] > k + 1;
        const bool fuse = k + 1 < kmax && next_active == nactive;
        NextDrift nd{};
        if (fuse) {
            nd.bbox = (unsigned long long *)ctx->ws["bbox"].ptr;
            nd.nc = (int)b.cs.size();
            nd.zr = ctx->last_zr;
        }
        launch_kick_drift(b.d_desc, b.ion_crystal, b.ntot, (int)(k - group_start), E, b.beams, dsum, (int)k,
                          fuse ? &nd : nullptr, kp.part ? &kp : nullptr, ctx->stream);
        drift = fuse ? 2 : 1;
        for (pt_crystal *c : b.cs) c->step++;
    }
    PT_HIP(hipGetLastError());
    return PT_OK;
}

// Reads back the outcome of the last queued steps: if a step halted on the
// device (its tree or lists outgrew the capacities), every crystal stands at
// the last completed step; the step counters are set to it and the rest is
// run again from there, starting with a measuring evaluation (so each pass
// completes at least one step).
static pt_status settle(pt_ctx *ctx)
{
    while (ctx->pending.active) {
        ctx->pending.active = false;
        auto it = ctx->ws.find("sum");
        if (it == ctx->ws.end() || ctx->pending.cs.empty() || ctx->pending.cs[0]->force.method != 1) return PT_OK;
        TreeSummary ts;
        PT_HIP(hipStreamSynchronize(ctx->stream));
        PT_HIP(hipMemcpy(&ts, it->second.ptr, sizeof(TreeSummary), hipMemcpyDeviceToHost));
        if (ts.fail_step < 0) return PT_OK;
        auto &pd = ctx->pending;
        const int n = (int)pd.cs.size();
        std::vector<int64_t> rest(n);
        for (int i = 0; i < n; ++i) {
            const int64_t done = std::min<int64_t>(pd.n_steps[i], ts.fail_step);
            pd.cs[i]->step = pd.step_start[i] + done;
            rest[i] = pd.n_steps[i] - done;
        }
        ctx->caps_ok = false;
        if (ts.refine_overflow) {
            ctx->psort_first = std::max(0, ctx->psort_first - 1);  // sort by one more digit from now on
        } else {
            ctx->caps_slack = std::min(4.0, ctx->caps_slack * 1.5);
        }
        ctx->reruns++;
        if (ts.sort_error) {
            pt_set_error("radix sort: a workgroup gave up waiting for its predecessors' digit counts");
            return PT_EDEVICE;
        }
        std::vector<pt_crystal *> cs = pd.cs;
        PT_TRY(step_run(ctx, cs.data(), n, rest.data()));
    }
    return PT_OK;
}

pt_status pt_step_batch(pt_crystal *const *cs, int n_crystals, const int64_t *n_steps)
{
    PT_TRY(check_batch(cs, n_crystals));
    PT_REQUIRE(n_steps, "n_steps NULL");
    for (int i = 0; i < n_crystals; ++i) PT_REQUIRE(n_steps[i] >= 0, "n_steps must be >= 0");
    PT_TRY(settle(cs[0]->ctx));
    return step_run(cs[0]->ctx, cs, n_crystals, n_steps);
}

pt_status pt_step(pt_crystal *c, int64_t n_steps) { return pt_step_batch(&c, 1, &n_steps); }

pt_status pt_synchronize(pt_ctx *ctx)
{
    PT_REQUIRE(ctx, "ctx is NULL");
    PT_TRY(settle(ctx));
    PT_HIP(hipStreamSynchronize(ctx->stream));
    PT_HIP(hipGetLastError());
    int32_t flag = 0;
    PT_HIP(hipMemcpy(&flag, ctx->d_nonfinite, sizeof(flag), hipMemcpyDeviceToHost));
    if (flag) {
        PT_HIP(hipMemset(ctx->d_nonfinite, 0, sizeof(int32_t)));
        pt_set_error("a step produced a non-finite position or velocity (pt_read_state names the crystal)");
        return PT_ENUMERIC;
    }
    return PT_OK;
}

pt_status pt_read_state(pt_crystal *c, double *pos, double *vel, int64_t *step, double *t, int32_t *photons)
{
    PT_REQUIRE(c, "crystal is NULL");
    pt_ctx *ctx = c->ctx;
    PT_TRY(settle(ctx));
    const int64_t n = c->n;
    std::vector<double> soa(6 * (size_t)n);
    PT_HIP(hipMemcpyAsync(soa.data(), c->d_state, sizeof(double) * 6 * n, hipMemcpyDeviceToHost, ctx->stream));
    if (photons)
        PT_HIP(hipMemcpyAsync(photons, c->d_photons, sizeof(int32_t) * n, hipMemcpyDeviceToHost, ctx->stream));
    int32_t flag = 0;
    PT_HIP(hipMemcpyAsync(&flag, c->d_nonfinite, sizeof(flag), hipMemcpyDeviceToHost, ctx->stream));
    PT_HIP(hipStreamSynchronize(ctx->stream));
    bool finite = flag == 0;
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            const double x = soa[d * n + i], v = soa[(3 + d) * n + i];
            if (pos) pos[3 * i + d] = x;
            if (vel) vel[3 * i + d] = v;
            finite = finite && std::isfinite(x) && std::isfinite(v);
        }
    if (step) *step = c->step;
    if (t) *t = c->trap.t0_s + (double)c->step * c->trap.dt_s;
    if (!finite) {
        pt_set_error("state holds non-finite values");
        return PT_ENUMERIC;
    }
    return PT_OK;
}

pt_status pt_ctx_set_near_share(pt_ctx *ctx, int per_cu)
{
    PT_REQUIRE(ctx, "ctx is NULL");
    PT_REQUIRE(per_cu >= 0 && per_cu <= 8, "near-field workgroups per compute unit must be 0 (default) .. 8");
    PT_TRY(settle(ctx));
    ctx->near_per_cu = per_cu;
    return PT_OK;
}

pt_status pt_ctx_set_fork(pt_ctx *ctx, int mode)
{
    PT_REQUIRE(ctx, "ctx is NULL");
    PT_REQUIRE(mode >= -1 && mode <= 1, "fork direction must be -1 (by the measured balance), 0 or 1");
    PT_TRY(settle(ctx));
    ctx->near_main = mode;
    return PT_OK;
}

pt_status pt_ctx_set_timing(pt_ctx *ctx, int enable)
{
    PT_REQUIRE(ctx, "ctx is NULL");
    PT_REQUIRE(enable >= 0, "timing: 0 (off) or n >= 1 (every n-th evaluation)");
    PT_TRY(settle(ctx));
    PT_TRY(finish_timing(ctx));
    if (enable && !ctx->ring_made) {
        for (auto &set : ctx->ev)
            for (auto &e : set) PT_HIP(hipEventCreate(&e));
        for (auto &pair : ctx->ev_near)
            for (auto &e : pair) PT_HIP(hipEventCreate(&e));
        ctx->ring_made = true;
    }
    ctx->timing = 0;
    ctx->timing_every = enable > 0 ? enable : 0;
    ctx->timing_evals = 0;
    for (double &v : ctx->phase_sum) v = 0.0;
    ctx->phase_count = 0;
    return PT_OK;
}

pt_status pt_ctx_phase_times(pt_ctx *ctx, double ms[7], int64_t *count)
{
    PT_REQUIRE(ctx && ms, "NULL argument");
    PT_TRY(settle(ctx));
    PT_TRY(finish_timing(ctx));
    for (int i = 0; i < kPhases; ++i) ms[i] = ctx->phase_count ? ctx->phase_sum[i] / (double)ctx->phase_count : 0.0;
    if (count) *count = ctx->phase_count;
    return PT_OK;
}

pt_status pt_ctx_step_stats(pt_ctx *ctx, int64_t *queued, int64_t *measured, int64_t *reruns)
{
    PT_REQUIRE(ctx, "ctx is NULL");
    PT_TRY(settle(ctx));
    if (queued) *queued = ctx->n_queued;
    if (measured) *measured = ctx->n_measured;
    if (reruns) *reruns = ctx->reruns;
    return PT_OK;
}

pt_status pt_ctx_work_counts(pt_ctx *ctx, int64_t counts[6])
{
    PT_REQUIRE(ctx && counts, "NULL argument");
    PT_TRY(settle(ctx));
    for (int i = 0; i < 6; ++i) counts[i] = 0;
    counts[5] = ctx->last_ntot;
    if (!ctx->last_was_fmm) return PT_OK;
    TreeSummary ls;
    PT_TRY(read_summary(ctx, ls));
    const int nbox = ls.nbox;
    std::vector<int64_t> np(nbox);
    uint32_t tot[4];
    PT_HIP(hipMemcpy(tot, ctx->ws["total"].ptr, sizeof(tot), hipMemcpyDeviceToHost));
    PT_HIP(hipMemcpy(np.data(), ctx->ws["near_pairs"].ptr, np.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    const int64_t nv = tot[2];  // V pairs: the scan total of the last evaluation's per-box counts
    int64_t nn = 0;
    for (int64_t x : np) nn += x;
    std::vector<uint8_t> leaf(nbox);
    PT_HIP(hipMemcpy(leaf.data(), ctx->ws["b_leaf"].ptr, nbox, hipMemcpyDeviceToHost));
    int64_t nl = 0;
    for (uint8_t x : leaf) nl += x;
    int nlev = 0;
    for (int l = 0; l <= kMaxLevel; ++l)
        if (ls.level_start[l + 1] > ls.level_start[l]) nlev = l + 1;
    counts[0] = nbox;
    counts[1] = nl;
    counts[2] = nv;
    counts[3] = nn;
    counts[4] = nlev;
    return PT_OK;
}

pt_status pt_debug_export_tree(pt_crystal *c, int64_t sizes[4], uint64_t *keys, int32_t *perm, int32_t *level,
                               int32_t *parent, int32_t *ion_begin, int32_t *ion_end, int32_t *coords,
                               uint8_t *is_leaf, int32_t *v_off, int32_t *v_src, int32_t *near_off,
                               int32_t *near_src, double *root)
{
    PT_REQUIRE(c && sizes, "NULL argument");
    pt_ctx *ctx = c->ctx;
    PT_TRY(settle(ctx));
    auto &lb = ctx->last_batch;
    auto it = std::find(lb.begin(), lb.end(), c);
    PT_REQUIRE(ctx->last_was_fmm && it != lb.end(), "no FMM evaluation of this crystal to export");
    const int ci = (int)(it - lb.begin());
    const int off = ctx->last_off[ci];
    const int n = (int)c->n;
    TreeSummary ls;
    PT_TRY(read_summary(ctx, ls));
    const int nbox = ls.nbox, ntot = ctx->last_ntot, stride = ctx->last_stride;
    auto dl = [&](const char *nm, void *dst, size_t bytes) -> pt_status {
        PT_HIP(hipMemcpy(dst, ctx->ws[nm].ptr, bytes, hipMemcpyDeviceToHost));
        return PT_OK;
    };
    std::vector<int32_t> bl(nbox), bcr(nbox), bb(nbox), be(nbox), bp(nbox), bx(nbox), by(nbox), bz(nbox), vt,
        nc(nbox);
    std::vector<uint8_t> blf(nbox);
    PT_TRY(dl("b_level", bl.data(), 4 * nbox));
    PT_TRY(dl("b_crystal", bcr.data(), 4 * nbox));
    PT_TRY(dl("b_begin", bb.data(), 4 * nbox));
    PT_TRY(dl("b_end", be.data(), 4 * nbox));
    PT_TRY(dl("b_parent", bp.data(), 4 * nbox));
    PT_TRY(dl("b_ix", bx.data(), 4 * nbox));
    PT_TRY(dl("b_iy", by.data(), 4 * nbox));
    PT_TRY(dl("b_iz", bz.data(), 4 * nbox));
    PT_TRY(dl("b_leaf", blf.data(), nbox));
    PT_TRY(dl("near_cnt", nc.data(), 4 * nbox));
    vt.resize((size_t)kWin * nbox);
    PT_TRY(dl("vtab", vt.data(), 4 * vt.size()));
    std::vector<int2> nr((size_t)stride * nbox);
    PT_TRY(dl("near", nr.data(), sizeof(int2) * nr.size()));
    std::vector<uint64_t> sk(ntot);
    std::vector<uint32_t> sv(ntot);
    PT_HIP(hipMemcpy(sk.data(), ctx->last_keys, 8 * ntot, hipMemcpyDeviceToHost));
    PT_HIP(hipMemcpy(sv.data(), ctx->last_vals, 4 * ntot, hipMemcpyDeviceToHost));
    std::vector<RootCube> rts(lb.size());
    PT_HIP(hipMemcpy(rts.data(), ctx->ws["roots"].ptr, sizeof(RootCube) * lb.size(), hipMemcpyDeviceToHost));
    // boxes of this crystal, in global (level, crystal, prefix) order
    std::vector<int32_t> g2l(nbox, -1), l2g;
    for (int b = 0; b < nbox; ++b)
        if (bcr[b] == ci) {
            g2l[b] = (int32_t)l2g.size();
            l2g.push_back(b);
        }
    const int nb = (int)l2g.size();
    // leaves of this crystal by first ion (for expanding near ranges)
    std::vector<std::pair<int, int>> leaves;
    for (int lb_ = 0; lb_ < nb; ++lb_)
        if (blf[l2g[lb_]]) leaves.push_back({bb[l2g[lb_]], lb_});
    std::sort(leaves.begin(), leaves.end());
    std::vector<std::vector<int32_t>> V(nb), NE(nb);
    int64_t nv = 0, nn = 0;
    int nlev = 0;
    for (int lb_ = 0; lb_ < nb; ++lb_) {
        const int g = l2g[lb_];
        nlev = std::max(nlev, bl[g] + 1);
        for (int w = 0; w < kWin; ++w) {
            const int s = vt[(size_t)g * kWin + w];
            if (s >= 0) V[lb_].push_back(g2l[s]);
        }
        std::sort(V[lb_].begin(), V[lb_].end());
        nv += V[lb_].size();
        if (blf[g]) {
            for (int r = 0; r < nc[g]; ++r) {
                const int2 rg = nr[(size_t)g * stride + r];
                auto lo = std::lower_bound(leaves.begin(), leaves.end(), std::make_pair(rg.x, -1));
                for (; lo != leaves.end() && lo->first < rg.y; ++lo) NE[lb_].push_back(lo->second);
            }
            std::sort(NE[lb_].begin(), NE[lb_].end());
            nn += NE[lb_].size();
        }
    }
    sizes[0] = nb;
    sizes[1] = nlev;
    sizes[2] = nv;
    sizes[3] = nn;
    if (keys || perm)
        for (int k = 0; k < n; ++k) {
            const int id = (int)sv[off + k] - off;
            if (keys) keys[id] = sk[off + k] & 0xFFFFFFFFFFFFull;
            if (perm) perm[k] = id;
        }
    for (int lb_ = 0; lb_ < nb; ++lb_) {
        const int g = l2g[lb_];
        if (level) level[lb_] = bl[g];
        if (parent) parent[lb_] = bp[g] >= 0 ? g2l[bp[g]] : -1;
        if (ion_begin) ion_begin[lb_] = bb[g] - off;
        if (ion_end) ion_end[lb_] = be[g] - off;
        if (coords) {
            coords[3 * lb_] = bx[g];
            coords[3 * lb_ + 1] = by[g];
            coords[3 * lb_ + 2] = bz[g];
        }
        if (is_leaf) is_leaf[lb_] = blf[g];
    }
    if (v_off) {
        int64_t a = 0;
        for (int lb_ = 0; lb_ < nb; ++lb_) {
            v_off[lb_] = (int32_t)a;
            if (v_src)
                for (int32_t s : V[lb_]) v_src[a++] = s;
            else
                a += V[lb_].size();
        }
        v_off[nb] = (int32_t)a;
    }
    if (near_off) {
        int64_t a = 0;
        for (int lb_ = 0; lb_ < nb; ++lb_) {
            near_off[lb_] = (int32_t)a;
            if (near_src)
                for (int32_t s : NE[lb_]) near_src[a++] = s;
            else
                a += NE[lb_].size();
        }
        near_off[nb] = (int32_t)a;
    }
    if (root) {
        root[0] = rts[ci].o[0];
        root[1] = rts[ci].o[1];
        root[2] = rts[ci].o[2];
        root[3] = rts[ci].W;
    }
    return PT_OK;
}

}  // extern "C"
