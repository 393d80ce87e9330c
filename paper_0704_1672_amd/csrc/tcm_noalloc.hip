// A variant of tcm_moments that allocates nothing, for callers that cannot call the device
// allocator (code under graph capture, tight serving loops, harnesses that forbid it): the
// caller passes device inputs and outputs, and every scratch byte of the moment pass (the plan
// record, item lists, statistics, tile partials) lives in one file-scope device array of a
// fixed size, held by each device the library runs on until the process ends.  Calls on one
// device share that array, so calls that overlap on a device race (issue them on one stream,
// or wait between them).
#include <mutex>

#include "tcm_runtime.h"

namespace tcm {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;     // 32 MiB per device
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];

// The device address of `scratch` on `device` (the current device), looked up once per device:
// in host code the array's name is a host-side stand-in, so launches and copies use this address.
int noalloc_init(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return TCM_EINVAL;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return TCM_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return TCM_EDEVICE;
    }
    g_scratch_ptr[device] = p;
    return TCM_OK;
}

static void* scratch_of(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_ptr[device];
}

// Writes the one-molecule plan into the scratch: the molecule record, its statistics items
// (molecule 0, chunk k) and tile items (molecule 0, tile * m-blocks + block), and clears the
// error flag (a kernel, not a memset or copy).
__global__ __launch_bounds__(WG) void tcm_noalloc_setup(MolWork mw, MolWork* dst, int32_t* stats_items, int n_stats,
                                                        int32_t* tile_items, int n_tiles, int32_t* err)
{
    const int i = (int)(blockIdx.x * WG + threadIdx.x), stride = (int)(gridDim.x * WG);
    if (i == 0) {
        *dst = mw;
        *err = 0;
    }
    for (int k = i; k < n_stats; k += stride) {
        stats_items[2 * k] = 0;
        stats_items[2 * k + 1] = k;
    }
    for (int k = i; k < n_tiles; k += stride) {
        tile_items[2 * k] = 0;
        tile_items[2 * k + 1] = k;
    }
}

}  // namespace tcm

using namespace tcm;

extern "C" int tcm_moments_noalloc(tcm_ctx* t, const double* d_x, const double* d_y, const double* d_z,
                                   const double* d_q, int64_t n, const double* centre, int L, int prec, double* d_Q,
                                   double* d_meta)
{
    if (!t || !d_Q || !d_meta || n < 0 || L < 0 || L > LMAX || (prec != TCM_F64 && prec != TCM_F32C)) return TCM_EINVAL;
    if (n > 0 && (!d_x || !d_y || !d_z || !d_q)) return TCM_EINVAL;
    if (centre && !(std::isfinite(centre[0]) && std::isfinite(centre[1]) && std::isfinite(centre[2]))) return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    char* base = (char*)scratch_of(c.device);
    if (!base) return TCM_EDEVICE;
    // the plan tcm_moments builds for one molecule: the same tiling, items and kernels
    MolWork w{};
    w.x = d_x; w.y = d_y; w.z = d_z; w.q = d_q;
    w.n = n;
    w.L = L;
    w.prec = prec;
    w.kper = c.kper_for(prec, L, n);
    w.nblk = num_blocks_for(prec, L);
    const int64_t tile_atoms = (int64_t)WG * w.kper;
    const int64_t nt = n > 0 ? (n + tile_atoms - 1) / tile_atoms : 1;
    const int64_t ns = stats_items_for(n);
    const int64_t nitems = nt * w.nblk;
    w.ntiles = (int32_t)nt;
    w.nstats = (int32_t)ns;
    w.has_centre = centre ? 1 : 0;
    if (centre) { w.centre[0] = centre[0]; w.centre[1] = centre[1]; w.centre[2] = centre[2]; }
    w.Q = d_Q;
    w.meta = d_meta;
    w.part_off = w.stats_off = w.r2_off = 0;
    // scratch layout (256-byte aligned pieces); too large a molecule is refused
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t o_mw = 0;
    const size_t o_si = up(o_mw + sizeof(MolWork));
    const size_t o_ti = up(o_si + sizeof(int32_t) * 2 * (size_t)ns);
    const size_t o_err = up(o_ti + sizeof(int32_t) * 2 * (size_t)nitems);
    const size_t o_part = up(o_err + sizeof(int32_t));
    const size_t part_bytes = prec == TCM_F32C ? sizeof(float) * 2 * (size_t)nt * nh(L) : sizeof(double) * (size_t)nt * nh(L);
    const size_t o_stats = up(o_part + part_bytes);
    const size_t o_r2 = up(o_stats + sizeof(double) * 10 * (size_t)ns);
    const size_t total = o_r2 + sizeof(double) * (size_t)nt;
    if (nt > (1 << 24) || total > NOALLOC_SCRATCH_BYTES) return TCM_ENOMEM;
    DevPlan P{};
    P.mols = (const MolWork*)(base + o_mw);
    P.pairs = nullptr;
    P.stats_items = (const int32_t*)(base + o_si);
    P.tile_items = (const int32_t*)(base + o_ti);
    P.nmol = 1;
    P.npairs = 0;
    P.n_stats = (int32_t)ns;
    P.n_tiles = (int32_t)nitems;
    P.err = (int32_t*)(base + o_err);
    P.part_f = (float*)(base + o_part);
    P.part_d = (double*)(base + o_part);
    P.stats_part = (double*)(base + o_stats);
    P.r2_part = (double*)(base + o_r2);
    P.invk = (const double*)c.t_invk.p;
    P.invf = (const double*)c.t_invf.p;
    P.rot = (const double*)c.t_rot.p;
    P.fact = (const double*)c.t_fact.p;
    hipStream_t s = c.stream;
    const int64_t nset = std::max<int64_t>(ns, nitems);
    const unsigned grid = (unsigned)std::min<int64_t>(1024, (nset + WG - 1) / WG);
    hipLaunchKernelGGL(tcm_noalloc_setup, dim3(grid > 0 ? grid : 1), dim3(WG), 0, s, w, (MolWork*)(base + o_mw),
                       (int32_t*)(base + o_si), (int)ns, (int32_t*)(base + o_ti), (int)nitems, P.err);
    if (hipGetLastError() != hipSuccess ||
        launch_stats(P, 0, (int)ns, s) != hipSuccess ||
        launch_stats_finalize(P, 0, 1, s) != hipSuccess ||
        launch_tiles(prec, L, P, (int)ns, (int)(ns + nitems), s) != hipSuccess ||
        launch_moments_finalize(P, s) != hipSuccess)
        return TCM_EDEVICE;
    return TCM_OK;
}
