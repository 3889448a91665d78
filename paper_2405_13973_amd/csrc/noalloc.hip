// Fixed device scratch of the force entry point that allocates nothing
// (pt_compute_forces_noalloc), and the two small kernels only it uses.
//
// The scratch is one file-scope device array per GPU, held until the process
// ends.  Host code never uses the array's name as an address: at context
// creation the device's copy is looked up once with hipGetSymbolAddress (with
// that device current) and the address is kept per device; kernels receive
// that address as an argument.  Every call on one GPU shares its array, so
// calls that overlap on one GPU race (they must be serialised, which the
// single stream of a context does for calls through one context).
#include <algorithm>
#include <mutex>

#include "pt_common.hpp"
#include "pt_kernels.hpp"

namespace pt {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};
}  // namespace

pt_status noalloc_scratch(int device, void **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (device < 0 || device >= kMaxDevices) {
        pt_set_error("device %d: the no-allocation scratch supports devices 0..%d", device, kMaxDevices - 1);
        return PT_EINVAL;
    }
    if (!g_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            pt_set_error("hipGetSymbolAddress(scratch) on device %d failed: %s", device, hipGetErrorString(e));
            return PT_EDEVICE;
        }
        g_addr[device] = p;
    }
    *out = g_addr[device];
    return PT_OK;
}

// Bytes of the regions for n ions, 256-aligned each.
constexpr size_t up256(size_t b) { return (b + 255) / 256 * 256; }

constexpr size_t noalloc_bytes(int n)
{
    const size_t nblk = (size_t)direct_chunks(n) * ((n + kDirTile - 1) / kDirTile);
    return up256(sizeof(CrystalDev)) + up256(sizeof(unsigned long long) * bbox_words(1)) + up256(4 * (size_t)n) +
           up256(sizeof(DirBlock) * nblk) + up256(sizeof(double) * 3 * (size_t)n) +
           up256(sizeof(double) * 3 * (size_t)direct_chunks(n) * n) + up256(sizeof(double) * 3 * (size_t)n);
}

// The largest layout up to kNoAllocMaxIons ions: the partials grow with
// chunks x n, which peaks where a tile count is full, so those sizes (and the
// limit itself) are the ones to check.
constexpr bool noalloc_fits()
{
    for (int tiles = 1; (long long)(tiles - 1) * kDirTile < kNoAllocMaxIons; ++tiles) {
        const int n = tiles * kDirTile < kNoAllocMaxIons ? tiles * kDirTile : kNoAllocMaxIons;
        if (noalloc_bytes(n) > kNoAllocScratchBytes) return false;
    }
    return true;
}
static_assert(noalloc_fits(), "the no-allocation scratch must hold the layout of every size up to its limit");

NoAllocLayout noalloc_layout(int n)
{
    const int nblk = direct_chunks(n) * ceil_div(n, kDirTile);
    NoAllocLayout l{};
    size_t o = 0;
    l.desc = o;
    o += up256(sizeof(CrystalDev));
    l.bbox = o;
    o += up256(sizeof(unsigned long long) * bbox_words(1));
    l.ion_crystal = o;
    o += up256(sizeof(int32_t) * (size_t)n);
    l.tab = o;
    o += up256(sizeof(DirBlock) * (size_t)nblk);
    l.mid = o;  // positions only: x[n] y[n] z[n]
    o += up256(sizeof(double) * 3 * (size_t)n);
    l.part = o;  // the direct sum's chunk partials, 3 x chunks x n
    o += up256(sizeof(double) * 3 * (size_t)direct_chunks(n) * n);
    l.E = o;
    o += up256(sizeof(double) * 3 * (size_t)n);
    l.total = o;
    l.nblk = nblk;
    return l;
}

// One crystal's descriptor, its ion -> crystal map (all zero) and the
// direct-sum block table (block k: target tile k mod tiles, source chunk
// k / tiles), written by kernels rather than copied from the host.
__global__ void k_noalloc_setup(CrystalDev d, CrystalDev *__restrict__ desc, int32_t *__restrict__ ion_crystal, int n,
                                DirBlock *__restrict__ tab, int nblk)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) *desc = d;
    if (g < n) ion_crystal[g] = 0;
    if (g < nblk) {
        const int tiles = (n + kDirTile - 1) / kDirTile;
        tab[g] = DirBlock{0, (g % tiles) * kDirTile, g / tiles, 0};
    }
}

// F (n x 3, ion order) = s * E (SoA 3 x n): one rounding per component, the
// same product the host forms for pt_compute_forces.
__global__ void k_scale_field(const double *__restrict__ E, int n, double s, double *__restrict__ F)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 3 * n) return;
    const int i = e / 3, d = e - 3 * i;
    F[e] = s * E[(size_t)d * n + i];
}

void launch_noalloc_setup(const CrystalDev &d, CrystalDev *desc, int32_t *ion_crystal, int n, DirBlock *tab, int nblk,
                          hipStream_t st)
{
    const int m = std::max(1, std::max(n, nblk));
    k_noalloc_setup<<<ceil_div(m, 256), 256, 0, st>>>(d, desc, ion_crystal, n, tab, nblk);
}

void launch_scale_field(const double *E, int n, double s, double *F, hipStream_t st)
{
    if (n > 0) k_scale_field<<<ceil_div(3 * (long long)n, 256), 256, 0, st>>>(E, n, s, F);
}

}  // namespace pt
