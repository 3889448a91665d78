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

NoAllocLayout noalloc_layout(int n)
{
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const int nblk = ceil_div(n, direct_targets_per_block());
    NoAllocLayout l{};
    size_t o = 0;
    l.desc = o;
    o += up(sizeof(CrystalDev));
    l.bbox = o;
    o += up(sizeof(unsigned long long) * bbox_words(1));
    l.ion_crystal = o;
    o += up(sizeof(int32_t) * (size_t)n);
    l.blk_crystal = o;
    o += up(sizeof(int32_t) * (size_t)nblk);
    l.blk_first = o;
    o += up(sizeof(int32_t) * (size_t)nblk);
    l.mid = o;  // positions only: x[n] y[n] z[n]
    o += up(sizeof(double) * 3 * (size_t)n);
    l.E = o;
    o += up(sizeof(double) * 3 * (size_t)n);
    l.total = o;
    l.nblk = nblk;
    return l;
}

// One crystal's descriptor, its ion -> crystal map (all zero) and the
// direct-sum block table (block k: targets from k * tpb), written by kernels
// rather than copied from the host.
__global__ void k_noalloc_setup(CrystalDev d, CrystalDev *__restrict__ desc, int32_t *__restrict__ ion_crystal, int n,
                                int32_t *__restrict__ blk_crystal, int32_t *__restrict__ blk_first, int nblk, int tpb)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) *desc = d;
    if (g < n) ion_crystal[g] = 0;
    if (g < nblk) {
        blk_crystal[g] = 0;
        blk_first[g] = g * tpb;
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

void launch_noalloc_setup(const CrystalDev &d, CrystalDev *desc, int32_t *ion_crystal, int n, int32_t *blk_crystal,
                          int32_t *blk_first, int nblk, hipStream_t st)
{
    const int m = std::max(1, std::max(n, nblk));
    k_noalloc_setup<<<ceil_div(m, 256), 256, 0, st>>>(d, desc, ion_crystal, n, blk_crystal, blk_first, nblk,
                                                      direct_targets_per_block());
}

void launch_scale_field(const double *E, int n, double s, double *F, hipStream_t st)
{
    if (n > 0) k_scale_field<<<ceil_div(3 * (long long)n, 256), 256, 0, st>>>(E, n, s, F);
}

}  // namespace pt
