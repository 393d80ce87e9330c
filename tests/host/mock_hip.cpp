// Definitions of the HIP stand-in (tests/host/hip/hip_runtime.h) and of kernel launchers
// that imitate the kernels' effect on the data the host reads back: moment tables are filled
// with the molecule's atom count, a pair's energy is Q_A[0] + 1e-3 Q_B[0] (so every result
// names the two fragments it was computed from), the eq. 2 test uses the radius the
// statistics step reports.  Test infrastructure only.
#include "hip/hip_runtime.h"
#include <atomic>
#include <random>
#include <mutex>
#include "tcm_runtime.h"
static std::mutex g_mu;
static std::mt19937 g_rng(getenv("MOCK_SEED") ? atoi(getenv("MOCK_SEED")) : 1);
static const int g_delay = getenv("MOCK_DELAY") ? atoi(getenv("MOCK_DELAY")) : 3;
// Fault injection for the failure-handling tests: with mock_set_faults(a, k), every a-th
// device allocation and every k-th tile launch fails (0 = never).
static std::atomic<int> g_fail_alloc{0}, g_fail_launch{0};
static std::atomic<long> g_alloc_calls{0}, g_launch_calls{0}, g_faults{0};
static bool fail_now(std::atomic<int>& every, std::atomic<long>& calls)
{
    const int e = every.load();
    if (e <= 0 || ++calls % e != 0) return false;
    ++g_faults;
    return true;
}
extern "C" {
void mock_set_faults(int alloc_every, int launch_every)
{
    g_alloc_calls = 0; g_launch_calls = 0; g_faults = 0;
    g_fail_alloc = alloc_every; g_fail_launch = launch_every;
}
long mock_faults_fired() { return g_faults.load(); }
hipError_t hipMalloc(void** p, size_t n)
{
    if (fail_now(g_fail_alloc, g_alloc_calls)) { *p = nullptr; return 2; }
    *p = malloc(n); if (*p) memset(*p, 0xAB, n); return *p ? 0 : 2;
}
hipError_t hipFree(void* p) { free(p); return 0; }
hipError_t hipMallocAsync(void** p, size_t n, hipStream_t) { return hipMalloc(p, n); }
hipError_t hipFreeAsync(void* p, hipStream_t) { free(p); return 0; }
hipError_t hipDeviceGetDefaultMemPool(hipMemPool_t* pool, int) { *pool = nullptr; return 0; }
hipError_t hipMemPoolSetAttribute(hipMemPool_t, hipMemPoolAttr, void*) { return 0; }
hipError_t hipMemPoolTrimTo(hipMemPool_t, size_t) { return 0; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = malloc(n); return *p ? 0 : 2; }
hipError_t hipHostFree(void* p) { free(p); return 0; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { memcpy(d, s, n); return 0; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { memcpy(d, s, n); return 0; }
hipError_t hipStreamSynchronize(hipStream_t) { return 0; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = (hipStream_t)malloc(8); return 0; }
hipError_t hipStreamDestroy(hipStream_t s) { free(s); return 0; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return 0; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t)calloc(1, 8); return 0; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = (hipEvent_t)calloc(1, 8); return 0; }
hipError_t hipEventDestroy(hipEvent_t e) { free(e); return 0; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { *(int*)e = g_delay; return 0; }
// an event completes after a few queries: launches stay "in flight" for a while
hipError_t hipEventQuery(hipEvent_t e) { std::lock_guard<std::mutex> g(g_mu); int* c = (int*)e; if (*c > 0 && (g_rng() % 2)) --*c; return *c > 0 ? hipErrorNotReady : 0; }
hipError_t hipEventSynchronize(hipEvent_t e) { *(int*)e = 0; return 0; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 1.f; return 0; }
hipError_t hipGetLastError() { return 0; }
hipError_t hipSetDevice(int) { return 0; }
hipError_t hipGetDeviceCount(int* n) { *n = 1; return 0; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) { p->multiProcessorCount = 4; return 0; }
hipError_t hipStreamBeginCapture(hipStream_t, int) { return 0; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = (hipGraph_t)malloc(8); return 0; }
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, void*, void*, size_t) { *e = (hipGraphExec_t)malloc(8); return 0; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return 0; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { free(e); return 0; }
hipError_t hipGraphDestroy(hipGraph_t g) { free(g); return 0; }
}
namespace tcm {
// kernels: pairs write U = 1 + index and status OK; everything else is a no-op on data
int noalloc_init(int) { return 0; }
int num_blocks_for(int prec, int L) { return prec == TCM_F32C ? num_blocks(L, BUDGET_F32) : num_blocks(L, BUDGET_F64); }
hipError_t launch_clear(int32_t* p, int64_t n, hipStream_t) { memset(p, 0, n * 4); return 0; }
hipError_t launch_stats(const DevPlan&, int, int, hipStream_t) { return 0; }
hipError_t launch_stats_finalize(const DevPlan& P, int b, int e, hipStream_t) {
    for (int m = b; m < e; ++m) { P.mols[m].meta[3] = 1.0; }
    return 0; }
hipError_t launch_moments_finalize(const DevPlan& P, hipStream_t) {
    for (int m = 0; m < P.nmol; ++m) { const MolWork& w = P.mols[m];
        for (int h = 0; h < nh(w.L); ++h) w.Q[h] = w.n; w.meta[3] = 0.5; }
    return 0; }
hipError_t launch_tiles(int, int, const DevPlan&, int, int, hipStream_t) { return fail_now(g_fail_launch, g_launch_calls) ? 1 : 0; }
hipError_t launch_scan(const double*, const double*, int, int, double, double, double, int, const double*,
                       const double*, const double*, double*, const double*, int64_t nR, double* U, int32_t* status,
                       hipStream_t) {
    for (int64_t k = 0; k < nR; ++k) { U[k] = 0.0; status[k] = 0; }
    return 0; }
hipError_t launch_alu_probe(int, void*, int, int, hipStream_t) { return 0; }
hipError_t launch_abs_sum(const double*, int64_t, double* out, hipStream_t) { out[0] = 1.0; return 0; }
hipError_t launch_gather8(const double* const* src, int64_t K, double* dst, hipStream_t) {
    for (int64_t i = 0; i < 8 * K; ++i) dst[i] = src[i >> 3][i & 7];
    return 0; }
hipError_t launch_pairs_ft(const DevPlan& P, int b, int e, double* FT, double*, double*, hipStream_t) {
    for (int p = b; p < e; ++p) { const PairWork& w = P.pairs[p];
        double R = sqrt(w.R[0]*w.R[0]+w.R[1]*w.R[1]+w.R[2]*w.R[2]);
        const bool ok = (w.flags & TCM_UNCHECKED) || R > w.metaA[3] + w.metaB[3];
        P.status[w.out] = ok ? 0 : TCM_EDOMAIN;
        for (int k = 0; k < 10; ++k) FT[10 * w.out + k] = ok ? w.QA[0] + 1e-3 * w.QB[0] : NAN; }
    return 0; }
hipError_t launch_atom_forces(const double*, int, int, const double*, const double*, const double*, const double*,
                              int64_t, const double*, double*, hipStream_t) { return 0; }
hipError_t launch_pairs_choose(const DevPlan& P, int b, int e, double, int32_t* Lout, double* bout, hipStream_t) {
    for (int p = b; p < e; ++p) { const PairWork& w = P.pairs[p]; Lout[w.out] = w.L; bout[w.out] = 0.0; }
    return 0; }
hipError_t launch_pairs_regroup(const DevPlan& P, int n, const int32_t* Lc, int32_t*, PairWork* pairs2, double* frame2,
                                int32_t* go, hipStream_t) {
    int q = 0;
    for (int L = LMAX; L >= 0; --L)
        for (int p = 0; p < n; ++p)
            if (Lc[P.pairs[p].out] == L) {
                pairs2[q] = P.pairs[p];
                pairs2[q].L = L;
                for (int c = 0; c < 2 * FRAME_N; ++c) frame2[(size_t)c * n + q] = P.frame[(size_t)c * n + p];
                ++q;
            }
    for (int g = 0; g * PAIR_LANES < n; ++g) go[g] = pairs2[g * PAIR_LANES].L;
    return 0; }
hipError_t launch_pairs(const DevPlan& P, int b, int e, hipStream_t) {
    for (int p = b; p < e; ++p) { const PairWork& w = P.pairs[p]; double s = w.QA[0] + 1e-3 * w.QB[0];
        double R = sqrt(w.R[0]*w.R[0]+w.R[1]*w.R[1]+w.R[2]*w.R[2]);
        if (!(w.flags & TCM_UNCHECKED) && !(R > w.metaA[3] + w.metaB[3])) { P.status[w.out] = TCM_EDOMAIN; P.U[w.out] = 0; }
        else { P.status[w.out] = 0; P.U[w.out] = s; } }
    return 0; }
}
