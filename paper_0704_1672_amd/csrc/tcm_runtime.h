// Host runtime of libtcm: context, device buffers, resident molecules, batch planning.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tcm.h"
#include "tcm_internal.h"

namespace tcm {

int num_blocks_for(int prec, int L);
// Statistics items of a molecule of n atoms (one per chunk of STATS_CHUNK atoms, at most 8192).
int64_t stats_items_for(int64_t n);
// Looks up, once per device (that device current), the device address of the static scratch
// array of the allocation-free entry point.
int noalloc_init(int device);
hipError_t launch_clear(int32_t* p, int64_t n, hipStream_t s);
hipError_t launch_stats(const DevPlan& P, int begin, int end, hipStream_t s);
hipError_t launch_pairs(const DevPlan& P, int begin, int end, hipStream_t s);
// Adaptive truncation: each pair's smallest order meeting tol and its bound, into Lout[out] and
// bout[out] (the plan's pair records are left as they are).
hipError_t launch_pairs_choose(const DevPlan& P, int begin, int end, double tol, int32_t* Lout, double* bout,
                               hipStream_t s);
// Lists the pairs again by decreasing chosen order Lc[out] into pairs2 / frame2 (the copies take
// that order) and writes the group orders of that listing; cnt: 2 (LMAX + 1) ints of scratch.
hipError_t launch_pairs_regroup(const DevPlan& P, int npairs, const int32_t* Lc, int32_t* cnt, PairWork* pairs2,
                                double* frame2, int32_t* gorder2, hipStream_t s);
hipError_t launch_stats_finalize(const DevPlan& P, int mol_begin, int mol_end, hipStream_t s);
hipError_t launch_moments_finalize(const DevPlan& P, hipStream_t s);
hipError_t launch_tiles(int prec, int L, const DevPlan& P, int begin, int end, hipStream_t s);
hipError_t launch_scan(const double* QA, const double* QB, int L, int triangular, double rho, double aA, double aB,
                       int unchecked, const double* invf, const double* rot, const double* quat, double* T,
                       const double* R, int64_t nR, double* U, int32_t* status, hipStream_t s);
// Forces and torques: FT[out][10] per pair (U, F_B, tau_A, tau_B); wscr and atab (both or
// neither) receive the per-atom coefficient tables of the pairs (one pair per call when set).
hipError_t launch_pairs_ft(const DevPlan& P, int begin, int end, double* FT, double* wscr, double* atab,
                           hipStream_t s);
hipError_t launch_alu_probe(int prec, void* out, int blocks, int iters, hipStream_t s);
hipError_t launch_abs_sum(const double* q, int64_t n, double* out, hipStream_t s);
hipError_t launch_gather8(const double* const* src, int64_t K, double* dst, hipStream_t s);
// Per-atom forces of side 0 (A) or 1 (B) from the tables launch_pairs_ft wrote to atab.
hipError_t launch_atom_forces(const double* atab, int side, int L, const double* x, const double* y, const double* z,
                              const double* q, int64_t n, const double* centre, double* F, hipStream_t s);

struct Ctx;

// A device allocation charged against the context's HBM budget.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

struct Mol {
    int64_t id = 0;
    int64_t n = 0;
    const double* x = nullptr;     // device SoA
    const double* y = nullptr;
    const double* z = nullptr;
    const double* q = nullptr;
    DevBuf atoms;                  // owned storage when uploaded
    int prec = TCM_F32C;
    int has_centre = 0;
    double centre[3] = {0, 0, 0};
    DevBuf moments;                // (Lcap+1)^2 FP64 resident moments
    DevBuf meta;                   // 5 FP64: centre, radius, scale
    int plan_refs = 0;             // live plans whose launches read or write these buffers
    int Lcached = -1;              // order of valid resident moments (-1: none)
    double radius_host = -1.0;     // meta[3] read back to the host, -1 until then; reset
                                   // whenever the moments are recomputed
    bool absq_dev = false;         // sum |q_i| (truncation bound) is in meta[5] on the device
    uint64_t last_use = 0;
    int plan_want = INT32_MIN;     // scratch of one request planning pass (under the context
    int plan_job = -1;             // lock): required order (-1 = reuse) and moment job index
};

// Everything one launch needs, described on the host.
struct MolJob {
    const double *x, *y, *z, *q;
    int64_t n;
    int L, prec, has_centre;
    double centre[3];
    double* Q;
    double* meta;
};

struct PairJob {
    const double* QA;
    const double* QB;
    const double* metaA;
    const double* metaB;
    int depA, depB;
    int L, flags;
    double R[3];
    double quat[4];
    int has_rot;
};


// Device-side state of a planned batch: the uploaded plan blob, scratch and outputs, and
// the streams and events its launches fork onto.
constexpr int NLANES = 2;          // streams the tile launches of a run are spread over

struct Workspace {
    DevBuf blob, sync, part_f, part_d, stats, r2, outU, outS, prot, pum;
    void* hstage = nullptr;        // pinned host staging for the blob
    size_t hstage_cap = 0;
    hipEvent_t staged = nullptr;   // recorded after the last copy out of hstage
    hipStream_t aux[NLANES] = {};  // the lanes of tile launches (forked from the run's stream)
    hipEvent_t fork = nullptr;
    hipEvent_t join[NLANES] = {};
    std::vector<hipEvent_t> gev;   // per group: its statistics and centre/scale are done
};

struct BuiltPlan {
    DevPlan P{};
    int n_items = 0;
    int n_stats = 0;
    int n_tiles = 0;
    struct Group {                 // molecules of one (precision, L): one tile launch
        int prec, L, begin, end;   // tile item range (tile numbering, before n_stats offset)
        int mol_begin, mol_end;    // molecule range
        int stats_begin, stats_end;
        double work;               // moment flops of the group (its tile launch's size)
    };
    Workspace* ws = nullptr;
    std::vector<Group> groups;
    int npairs = 0;
    int64_t sync_ints = 0;
    int64_t atoms = 0;
    double moment_flops = 0.0;
};

struct Ctx {
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    std::atomic<size_t> budget{0}; // 0 = unbounded
    std::atomic<size_t> used{0};
    DevBuf t_invk, t_invf, t_rot, t_fact;
    std::mutex mu;                 // guards molecules, tuning and the shared workspace
    std::unordered_map<int64_t, std::unique_ptr<Mol>> mols;
    int64_t next_id = 1;
    uint64_t use_clock = 0;
    Workspace ws;                  // shared by the synchronous entry points
    DevBuf tmp_atoms, tmp_q;       // one-shot uploads
    DevBuf scan_g, scan_r, scan_u, scan_s;   // translation scan: pair-tensor table, host-side I/O
    DevBuf force_ft, force_w, force_t, force_a, force_b;   // forces: outputs, coefficient tables, host-side I/O
    DevBuf adapt;                  // adaptive batches: chosen orders and bounds per pair
    DevBuf gather;                 // K record pointers, then K gathered 8-double records
    void* hpin = nullptr;          // pinned staging for one-shot uploads
    size_t hpin_cap = 0;
    std::map<int64_t, int> tune;   // key(prec, L, bucket) -> kper
    int f32_run_max = 64;          // longest plain FP32 run of a thread (caps kper of TCM_F32C)
    // serving
    struct Server* server = nullptr;

    int alloc(DevBuf& b, size_t bytes);      // grow-only, budget checked
    void release(DevBuf& b);
    // Stream-ordered variants (the device's default pool keeps freed memory cached), for
    // buffers allocated and freed while other launches run: no device-wide synchronisation.
    int alloc_async(DevBuf& b, size_t bytes, hipStream_t s);
    void release_async(DevBuf& b, hipStream_t s);
    int ensure_pinned(size_t bytes);
    int kper_for(int prec, int L, int64_t n);
};

// planning / running (tcm_runtime.cpp)
int build_plan(Ctx* c, Workspace& ws, const std::vector<MolJob>& mols,
               const std::vector<PairJob>& pairs, BuiltPlan& bp, hipStream_t s);
// energy = false leaves out the energy pair launch (callers that launch their own pair kernel)
int run_plan(Ctx* c, const BuiltPlan& bp, hipStream_t s, bool serial, hipEvent_t* ev, bool energy = true);
size_t workspace_growth(Ctx* c, const Workspace& ws, const std::vector<MolJob>& mols,
                        const std::vector<PairJob>& pairs);
int check_err(Ctx* c, const BuiltPlan& bp, hipStream_t s);
void free_workspace(Ctx* c, Workspace& ws);
int64_t tune_key(int prec, int L, int64_t n);

// Adaptive truncation over the pairs of a built plan, on device buffers carved from one
// allocation: the chosen order and its bound per output, the pair records and frames listed
// again by chosen order, the group orders of that listing and the regrouping's counters; P2
// is the contraction launch over the regrouped listing (U and status those of the plan).
struct AdaptBufs {
    double* bound = nullptr;
    int32_t* L = nullptr;
    int32_t* cnt = nullptr;
    DevPlan P2{};
    int npj = 0;
};
int adapt_setup(Ctx& c, DevBuf& buf, const BuiltPlan& bp, AdaptBufs& ab);
// order choice, regrouping and the contraction, ordered on s
int adapt_launch(const BuiltPlan& bp, const AdaptBufs& ab, double tol, hipStream_t s);

// serving (tcm_server.cpp)
void server_destroy(Ctx* c);

}  // namespace tcm

struct tcm_ctx {
    tcm::Ctx c;
};

struct tcm_plan {
    tcm::Ctx* ctx = nullptr;       // the context that created it (destroy plans first)
    tcm::Workspace ws;
    tcm::BuiltPlan bp;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int npairs = 0;
    // adaptive plans: the tolerance, the order choice's outputs and the regrouped listing
    bool adaptive = false;
    double tol = 0.0;
    tcm::DevBuf adapt;
    tcm::AdaptBufs ab;
    std::vector<tcm::Mol*> refs;   // molecules the plan names (pinned: not released while it lives)
    std::vector<std::pair<tcm::Mol*, int>> computed;   // moments each run writes, and their order
};
