// Serving loop of libtcm: continuous batching of pair-energy requests.
//
// One host thread per context runs the loop
//   1. retire finished launches (HIP event query): publish U / status / latency per ticket,
//      mark the moments they computed as resident, release fragment references;
//   2. while a launch slot is free and requests are pending: admit requests in arrival order
//      into a batch -- a fragment that is resident is a cache hit; a new fragment is copied
//      into server-owned device memory after HBM admission (when the context's budget would
//      be exceeded, the atoms of idle fragments are evicted least recently used first, while
//      their moment tables -- 8.7 KB each -- stay resident, so a later request of the same
//      fragment at an order it already holds is still served; a whole fragment is dropped only
//      when the moment arena cannot grow); a request is admitted whole -- both of its
//      fragments -- or waits, and a waiting request fetches nothing; a request whose fragment
//      is being computed by an in-flight launch waits for it;
//   3. launch the batch on the slot's own stream (statistics, per-order tile kernels, pair
//      kernel -- the same kernels as tcm_batch_energy) followed by asynchronous copies of the
//      results into the slot's pinned buffers and an event.
// With several slots the launches of consecutive batches run concurrently on the device.
// Each fragment's moments are computed with a tiling that depends only on (precision, L,
// n), so a result does not depend on which other requests shared its launch.
#include <chrono>
#include <cmath>
#include <cstring>
#include <list>

#include "tcm_runtime.h"

namespace tcm {

using clock_t_ = std::chrono::steady_clock;

struct SMol {
    int64_t key = 0;
    int64_t n = 0;
    int prec = TCM_F32C;
    DevBuf atoms;                  // FP64 SoA, owned (copy mode)
    const double* src[4] = {nullptr, nullptr, nullptr, nullptr};   // borrowed atoms
    double* moments = nullptr;     // slot of the moment arena: (LMAX+1)^2 table + 8 meta
    int slot = -1;
    int Lcached = -1;              // valid resident order
    bool atoms_gone = false;       // atoms evicted (moments kept): only orders <= Lcached are served
    int busy = 0;                  // being computed by an in-flight launch
    int refs = 0;                  // referenced by in-flight launches
    int pin = 0;                   // referenced by the batch being formed (not evictable)
    std::list<int64_t>::iterator lru;
};

struct SReq {
    uint64_t ticket;
    tcm_request r;
    clock_t_::time_point t_submit;
    bool waited = false;           // counted once in the deferred statistic
};

struct SResult {
    double U;
    int32_t status;
    double latency;
};

struct Slot {
    bool busy = false;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    Workspace ws;
    BuiltPlan bp;
    void* hpin = nullptr;          // U[cap] doubles, status[cap] ints, err int
    int cap = 0;
    int npairs = 0;                // pair jobs launched
    std::vector<SReq> reqs;        // requests of the batch (in order)
    std::vector<int> job_of;       // pair job index of each request, -1 = failed before launch
    std::vector<int32_t> pre_status;
    std::vector<std::pair<SMol*, int>> computed;
    std::vector<SMol*> refd;
};

// Fixed-size slots for resident moment tables ((LMAX+1)^2 + 8 doubles each), carved from
// device chunks allocated once, so admission never calls the device allocator for moments.
constexpr int ARENA_SLOT = (LMAX + 1) * (LMAX + 1) + 8;
constexpr int ARENA_CHUNK = 64;

struct Server {
    Ctx* c = nullptr;
    std::vector<DevBuf> arena;
    std::vector<int> free_slots;
    tcm_server_cfg cfg{};
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::deque<SReq> pending;
    std::unordered_map<uint64_t, SResult> done;
    std::unordered_map<uint64_t, int> live;    // submitted, not yet polled
    std::unordered_map<int64_t, std::unique_ptr<SMol>> cache;
    std::list<int64_t> lru;        // front = most recently used
    std::vector<Slot> slots;
    uint64_t next_ticket = 1;
    int64_t completed = 0, launches = 0, hits = 0, misses = 0, deferred = 0, evictions = 0;
    int64_t dropped = 0;           // fragments dropped whole (moment slot reclaimed)
    int64_t gone = 0;              // requests needing an order above the resident one of a
                                   // fragment whose atoms were evicted (TCM_ENOTFOUND)
    int inflight = 0;
};

static double seconds_since(clock_t_::time_point t)
{
    return std::chrono::duration<double>(clock_t_::now() - t).count();
}

// Copied atoms are freed in stream order on `s`: no launch still reads them (refs == 0 or the
// fragment was never launched), and the pool orders any reuse behind this point of `s`.
// Borrowed atoms are only forgotten.
static void drop_atoms(Server* S, SMol* m, hipStream_t s)
{
    S->c->release_async(m->atoms, s);
    for (auto& p : m->src) p = nullptr;
    m->atoms_gone = true;
}

static void free_mol(Server* S, SMol* m, hipStream_t s)
{
    S->c->release_async(m->atoms, s);
    if (m->slot >= 0) S->free_slots.push_back(m->slot);
    m->slot = -1;
    m->moments = nullptr;
}

static bool evictable(const SMol* m) { return m->refs == 0 && m->pin == 0 && !m->busy; }

static bool take_slot(Server* S, SMol* m, hipStream_t s)
{
    if (S->free_slots.empty()) {
        DevBuf b;
        if (S->c->alloc(b, sizeof(double) * ARENA_SLOT * ARENA_CHUNK) == TCM_OK) {
            const int base = (int)S->arena.size() * ARENA_CHUNK;
            S->arena.push_back(b);
            for (int i = ARENA_CHUNK - 1; i >= 0; --i) S->free_slots.push_back(base + i);
        } else {
            // the arena cannot grow: drop the least recently used idle fragment whole
            for (auto it = S->lru.end(); it != S->lru.begin();) {
                --it;
                auto f = S->cache.find(*it);
                SMol* v = f->second.get();
                if (v != m && evictable(v) && v->slot >= 0) {
                    free_mol(S, v, s);
                    S->lru.erase(it);
                    S->cache.erase(f);
                    ++S->dropped;
                    break;
                }
            }
            if (S->free_slots.empty()) return false;
        }
    }
    m->slot = S->free_slots.back();
    S->free_slots.pop_back();
    m->moments = (double*)S->arena[m->slot / ARENA_CHUNK].p + (size_t)(m->slot % ARENA_CHUNK) * ARENA_SLOT;
    return true;
}

// Device bytes a new fragment takes from the budget: its copied atoms (moment tables live in
// the arena, charged when a chunk is added).
static size_t mol_bytes(int64_t n, bool borrow)
{
    if (borrow) return 0;
    const size_t b = sizeof(double) * 4 * (size_t)(n > 0 ? n : 1);
    return b < 256 ? 256 : b;      // the allocator's minimum
}

// Evict the atoms of idle fragments (least recently used first; their moment tables stay)
// until `need` more bytes fit the budget.  Evicts nothing when even evicting every idle
// fragment's atoms would not make enough room.
static bool make_room(Server* S, size_t need, hipStream_t s)
{
    Ctx* c = S->c;
    const size_t budget = c->budget;
    if (!budget) return true;
    if (c->used.load() + need <= budget) return true;
    size_t idle = 0;
    for (auto& kv : S->cache)
        if (evictable(kv.second.get())) idle += kv.second->atoms.cap;
    const size_t used = c->used.load();
    if (used + need > budget + idle) return false;
    for (auto it = S->lru.end(); c->used.load() + need > budget && it != S->lru.begin();) {
        --it;
        SMol* m = S->cache.find(*it)->second.get();
        if (evictable(m) && m->atoms.cap > 0) {
            drop_atoms(S, m, s);
            ++S->evictions;
        }
    }
    return c->used.load() + need <= budget;
}

// Remove a fragment created by the current admission pass that will not be used.
static void destroy_mol(Server* S, SMol* m, hipStream_t s)
{
    const int64_t key = m->key;
    free_mol(S, m, s);
    S->lru.erase(m->lru);
    S->cache.erase(key);
}

static void touch(Server* S, SMol* m)
{
    S->lru.erase(m->lru);
    S->lru.push_front(m->key);
    m->lru = S->lru.begin();
}

static int copy_atoms(SMol* m, const double* const src[4], bool host, hipStream_t s)
{
    if (m->n == 0) return TCM_OK;
    double* d = (double*)m->atoms.p;
    for (int k = 0; k < 4; ++k)
        if (hipMemcpyAsync(d + k * m->n, src[k], sizeof(double) * m->n,
                           host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s) != hipSuccess)
            return TCM_EDEVICE;
    return TCM_OK;
}

// Finish a launch (called with S->mu held).  failed: the launch never ran (host-side
// error); its requests already carry their status and nothing it would have computed is
// marked resident.
static void retire(Server* S, Slot& sl, bool failed)
{
    const double* U = (const double*)sl.hpin;
    const int32_t* st = (const int32_t*)(U + sl.cap);
    const int32_t err = failed ? 1 : st[sl.cap];
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        SResult r;
        const int j = sl.job_of[i];
        if (j < 0) {
            r.status = sl.pre_status[i];
            r.U = std::nan("");
        } else {
            r.status = err ? TCM_EDEVICE : st[j];
            r.U = (r.status == TCM_OK) ? U[j] : std::nan("");
        }
        r.latency = seconds_since(sl.reqs[i].t_submit);
        S->done[sl.reqs[i].ticket] = r;
    }
    for (auto& pr : sl.computed) {
        pr.first->busy = 0;
        if (!err) pr.first->Lcached = pr.second;
    }
    for (SMol* m : sl.refd) --m->refs;
    S->completed += (int64_t)sl.reqs.size();
    sl.reqs.clear();
    sl.busy = false;
    --S->inflight;
}

// Admit pending requests into slot `sl` and launch them (called with S->mu held).
static void admit_and_launch(Server* S, Slot& sl)
{
    Ctx* c = S->c;
    std::map<SMol*, int> need;             // fragment -> order to compute in this launch
    std::vector<SMol*> refd;
    std::vector<SReq> batch;
    std::vector<int32_t> pre;
    std::deque<SReq> keep;
    // Resolve one side of a request without side effects: a resident fragment, a new one to
    // fetch (fresh), a resident one whose evicted atoms the request brings again (refetch),
    // or a status (TCM_EAGAIN: wait for an in-flight launch; TCM_ENOTFOUND).
    struct Side {
        SMol* m = nullptr;
        bool fresh = false;
        bool refetch = false;
        bool gone = false;         // TCM_ENOTFOUND because the atoms were evicted
        int status = TCM_OK;
    };
    auto look = [&](int64_t key, const double* const atoms[4], int64_t n, int L) -> Side {
        Side sd;
        const bool has = atoms[0] && atoms[1] && atoms[2] && atoms[3];
        auto f = S->cache.find(key);
        if (f != S->cache.end()) {
            SMol* m = f->second.get();
            if (m->busy) { sd.status = TCM_EAGAIN; return sd; }          // being computed
            auto nd = need.find(m);
            const bool recompute = m->Lcached < L && (nd == need.end() || nd->second < L);
            // an in-flight launch still reads this table: do not rewrite it
            if (recompute && m->refs > 0) { sd.status = TCM_EAGAIN; return sd; }
            if (recompute && m->atoms_gone) {
                // a higher order than the resident one needs the atoms back
                if (!(has || n == 0) || n != m->n) { sd.status = TCM_ENOTFOUND; sd.gone = true; return sd; }
                sd.refetch = true;
            }
            sd.m = m;
            return sd;
        }
        if (!(has || n == 0)) { sd.status = TCM_ENOTFOUND; return sd; }
        sd.fresh = true;
        return sd;
    };
    // Bring the evicted atoms of a resident fragment back (bytes already admitted).
    auto refetch = [&](SMol* m, const double* const atoms[4], int flags) -> int {
        if (flags & TCM_BORROW_ATOMS) {
            for (int k = 0; k < 4; ++k) m->src[k] = atoms[k];
        } else {
            if (c->alloc_async(m->atoms, sizeof(double) * 4 * (size_t)(m->n > 0 ? m->n : 1), sl.stream) != TCM_OK)
                return TCM_EAGAIN;
            if (copy_atoms(m, atoms, (flags & TCM_HOST_ATOMS) != 0, sl.stream) != TCM_OK) {
                S->c->release_async(m->atoms, sl.stream);
                return TCM_EDEVICE;
            }
            const double* d = (const double*)m->atoms.p;
            for (int k = 0; k < 4; ++k) m->src[k] = d + k * m->n;
        }
        m->atoms_gone = false;
        return TCM_OK;
    };
    // Create a fragment whose device bytes have been admitted; its atoms are copied on the
    // launch stream of this batch, ahead of the kernels that read them.
    auto create = [&](int64_t key, const double* const atoms[4], int64_t n, int prec, int flags,
                      int* status) -> SMol* {
        auto m = std::make_unique<SMol>();
        m->key = key;
        m->n = n;
        m->prec = prec;
        if (!take_slot(S, m.get(), sl.stream)) { *status = TCM_EAGAIN; return nullptr; }
        if (flags & TCM_BORROW_ATOMS) {
            for (int k = 0; k < 4; ++k) m->src[k] = atoms[k];
        } else {
            if (c->alloc_async(m->atoms, sizeof(double) * 4 * (size_t)(n > 0 ? n : 1), sl.stream) != TCM_OK) {
                free_mol(S, m.get(), sl.stream);
                *status = TCM_EAGAIN;
                return nullptr;
            }
            if (copy_atoms(m.get(), atoms, (flags & TCM_HOST_ATOMS) != 0, sl.stream) != TCM_OK) {
                free_mol(S, m.get(), sl.stream);
                *status = TCM_EDEVICE;
                return nullptr;
            }
            const double* d = (const double*)m->atoms.p;
            for (int k = 0; k < 4; ++k) m->src[k] = d + k * n;
        }
        S->lru.push_front(key);
        m->lru = S->lru.begin();
        SMol* raw = m.get();
        S->cache[key] = std::move(m);
        return raw;
    };
    // Workspace growth of the launch if the batch so far took one more request whose sides
    // are (a or a fresh fragment of n_a atoms) and (b or n_b), at order L.
    int npairs_batch = 0;
    auto growth_with = [&](const Side& sa, const Side& sb, const tcm_request& r) -> size_t {
        std::vector<MolJob> mj;
        std::map<SMol*, int> lv(need.begin(), need.end());
        for (const Side* sd : {&sa, &sb}) {
            if (sd->m && sd->m->Lcached < r.L) {
                auto it = lv.find(sd->m);
                if (it == lv.end()) lv[sd->m] = r.L; else if (it->second < r.L) it->second = r.L;
            }
        }
        for (auto& kv : lv) {
            MolJob j{};
            j.n = kv.first->n;
            j.L = std::max(kv.second, kv.first->Lcached);
            j.prec = kv.first->prec;
            mj.push_back(j);
        }
        const bool same = r.key_b == r.key_a;
        for (int side = 0; side < (same ? 1 : 2); ++side) {
            if (!(side == 0 ? sa.fresh : sb.fresh)) continue;
            MolJob j{};
            j.n = side == 0 ? r.n_a : r.n_b;
            j.L = r.L;
            j.prec = r.precision;
            mj.push_back(j);
        }
        return workspace_growth(c, sl.ws, mj, std::vector<PairJob>(npairs_batch + 1));
    };
    // Admit one request: both fragments resident or fetched, with room in the budget for
    // them and for the launch's workspace, or nothing changes.
    auto admit = [&](const tcm_request& r, SMol** pa, SMol** pb) -> int {
        const bool same = r.key_b == r.key_a;
        Side sa = look(r.key_a, r.atoms_a, r.n_a, r.L);
        Side sb = same ? sa : look(r.key_b, r.atoms_b, r.n_b, r.L);
        if (sa.status == TCM_ENOTFOUND || sb.status == TCM_ENOTFOUND) {
            if (sa.gone || sb.gone) ++S->gone;
            return TCM_ENOTFOUND;
        }
        if (sa.status != TCM_OK || sb.status != TCM_OK) return TCM_EAGAIN;
        const bool borrow = (r.flags & TCM_BORROW_ATOMS) != 0;
        const int nfresh = (sa.fresh ? 1 : 0) + (sb.fresh && !same ? 1 : 0);
        size_t bytes = (sa.fresh || sa.refetch ? mol_bytes(r.n_a, borrow) : 0) +
                       (!same && (sb.fresh || sb.refetch) ? mol_bytes(r.n_b, borrow) : 0);
        if ((int)S->free_slots.size() < nfresh) bytes += sizeof(double) * ARENA_SLOT * ARENA_CHUNK;
        if (c->budget) bytes += growth_with(sa, sb, r);
        if (bytes) {
            // resident sides of this request must survive the eviction
            if (sa.m) ++sa.m->pin;
            if (sb.m) ++sb.m->pin;
            const bool ok = make_room(S, bytes, sl.stream);
            if (sa.m) --sa.m->pin;
            if (sb.m) --sb.m->pin;
            if (!ok) return TCM_EAGAIN;
        }
        int st = TCM_OK;
        // atoms brought back for a higher order (their bytes were admitted above)
        if (sa.refetch && (st = refetch(sa.m, r.atoms_a, r.flags)) != TCM_OK) return st;
        if (!same && sb.refetch && (st = refetch(sb.m, r.atoms_b, r.flags)) != TCM_OK) return st;
        SMol* a = sa.m;
        if (sa.fresh && !(a = create(r.key_a, r.atoms_a, r.n_a, r.precision, r.flags, &st))) return st;
        SMol* b = same ? a : sb.m;
        if (sb.fresh && !same) {
            ++a->pin;
            b = create(r.key_b, r.atoms_b, r.n_b, r.precision, r.flags, &st);
            --a->pin;
            if (!b) {
                if (sa.fresh) destroy_mol(S, a, sl.stream);      // no copy may outlive a deferred request
                return st;
            }
        }
        *pa = a;
        *pb = b;
        return TCM_OK;
    };
    const int maxp = S->cfg.max_batch_pairs > 0 ? S->cfg.max_batch_pairs : 64;
    while (!S->pending.empty() && (int)batch.size() < maxp) {
        SReq q = S->pending.front();
        S->pending.pop_front();
        const tcm_request& r = q.r;
        SMol* a = nullptr;
        SMol* b = nullptr;
        const int st = admit(r, &a, &b);
        if (st != TCM_OK) {
            if (st == TCM_EAGAIN) {
                if (!q.waited) ++S->deferred;
                q.waited = true;
                keep.push_back(q);
                continue;
            }
            batch.push_back(q);
            pre.push_back(st);
            continue;
        }
        for (SMol* m : {a, b}) {
            auto nd = need.find(m);
            if (m->Lcached >= r.L || (nd != need.end() && nd->second >= r.L)) ++S->hits; else ++S->misses;
            if (m->Lcached < r.L) {
                auto it = need.find(m);
                if (it == need.end()) need[m] = r.L;
                else if (r.L > it->second) it->second = r.L;
            }
            touch(S, m);
            ++m->pin;                      // later admissions in this pass must not evict it
            refd.push_back(m);
        }
        batch.push_back(q);
        pre.push_back(TCM_OK);
        ++npairs_batch;
    }
    if (batch.empty() && S->inflight == 0 && !keep.empty()) {
        // nothing in flight can free memory or finish a fragment: the oldest deferred
        // request can never be admitted
        batch.push_back(keep.front());
        pre.push_back(TCM_ENOMEM);
        keep.pop_front();
    }
    for (auto it = keep.rbegin(); it != keep.rend(); ++it) S->pending.push_front(*it);
    if (batch.empty()) return;
    // jobs
    std::vector<MolJob> mj;
    std::map<SMol*, int> jobidx;
    sl.computed.clear();
    for (auto& kv : need) {
        SMol* m = kv.first;
        const int L = std::max(kv.second, m->Lcached);
        MolJob j{};
        j.x = m->src[0]; j.y = m->src[1]; j.z = m->src[2]; j.q = m->src[3];
        j.n = m->n;
        j.L = L;
        j.prec = m->prec;
        j.Q = m->moments;
        j.meta = m->moments + (ARENA_SLOT - 8);
        jobidx[m] = (int)mj.size();
        mj.push_back(j);
        m->busy = 1;
        m->Lcached = -1;
        sl.computed.push_back({m, L});
    }
    std::vector<PairJob> pj;
    sl.job_of.assign(batch.size(), -1);
    // the batch's pins become in-flight references (released when the launch retires)
    for (SMol* m : refd) {
        --m->pin;
        ++m->refs;
    }
    sl.refd = refd;
    for (size_t i = 0; i < batch.size(); ++i) {
        if (pre[i] != TCM_OK) continue;
        const tcm_request& r = batch[i].r;
        SMol* a = S->cache.find(r.key_a)->second.get();
        SMol* b = S->cache.find(r.key_b)->second.get();
        PairJob j{};
        j.QA = a->moments;
        j.QB = b->moments;
        j.metaA = a->moments + (ARENA_SLOT - 8);
        j.metaB = b->moments + (ARENA_SLOT - 8);
        auto fa = jobidx.find(a), fb = jobidx.find(b);
        j.depA = fa == jobidx.end() ? -1 : fa->second;
        j.depB = fb == jobidx.end() ? -1 : fb->second;
        j.L = r.L;
        j.flags = r.flags & (TCM_UNCHECKED | TCM_TRIANGULAR);
        for (int d = 0; d < 3; ++d) j.R[d] = r.R[d];
        for (int d = 0; d < 4; ++d) j.quat[d] = r.quat_b[d];
        j.has_rot = !(r.quat_b[0] > 0 && r.quat_b[1] == 0 && r.quat_b[2] == 0 && r.quat_b[3] == 0);
        sl.job_of[i] = (int)pj.size();
        pj.push_back(j);
    }
    sl.reqs = batch;
    sl.pre_status = pre;
    sl.npairs = (int)pj.size();
    // pinned result buffer
    const int cap = (int)batch.size();
    if (cap > sl.cap) {
        if (sl.hpin) (void)hipHostFree(sl.hpin);
        sl.hpin = nullptr;
        sl.cap = 0;
        if (hipHostMalloc(&sl.hpin, (sizeof(double) + sizeof(int32_t)) * cap + 64, hipHostMallocDefault) == hipSuccess)
            sl.cap = cap;
    }
    int rc = sl.cap >= cap ? TCM_OK : TCM_ENOMEM;
    // the launch's workspace comes out of the same budget: evict idle fragments first
    if (rc == TCM_OK) (void)make_room(S, workspace_growth(c, sl.ws, mj, pj), sl.stream);
    if (rc == TCM_OK) rc = build_plan(c, sl.ws, mj, pj, sl.bp, sl.stream);
    if (rc == TCM_OK) rc = run_plan(c, sl.bp, sl.stream, false, nullptr);
    double* hU = (double*)sl.hpin;
    int32_t* hS = (int32_t*)(hU + sl.cap);
    if (rc == TCM_OK && sl.npairs > 0) {
        if (hipMemcpyAsync(hU, sl.bp.P.U, sizeof(double) * sl.npairs, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
            hipMemcpyAsync(hS, sl.bp.P.status, sizeof(int32_t) * sl.npairs, hipMemcpyDeviceToHost, sl.stream) != hipSuccess)
            rc = TCM_EDEVICE;
    }
    if (rc == TCM_OK && hipMemcpyAsync(hS + sl.cap, sl.bp.P.err, sizeof(int32_t), hipMemcpyDeviceToHost, sl.stream) != hipSuccess)
        rc = TCM_EDEVICE;
    if (rc == TCM_OK && hipEventRecord(sl.ev, sl.stream) != hipSuccess) rc = TCM_EDEVICE;
    sl.busy = true;
    ++S->inflight;
    ++S->launches;
    if (rc != TCM_OK) {
        // the launch failed on the host side: fail its requests, keep the server running
        (void)hipStreamSynchronize(sl.stream);
        for (size_t i = 0; i < batch.size(); ++i)
            if (sl.job_of[i] >= 0) { sl.job_of[i] = -1; sl.pre_status[i] = rc; }
        retire(S, sl, true);
    }
}

static void server_loop(Server* S)
{
    (void)hipSetDevice(S->c->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progress = false;
        for (Slot& sl : S->slots) {
            if (sl.busy && hipEventQuery(sl.ev) == hipSuccess) {
                retire(S, sl, false);
                progress = true;
            }
        }
        if (S->stop && S->pending.empty() && S->inflight == 0) break;
        for (Slot& sl : S->slots) {
            if (!sl.busy && !S->pending.empty()) {
                const size_t before = S->pending.size();
                admit_and_launch(S, sl);
                if (sl.busy || S->pending.size() != before) progress = true;
            }
        }
        if (!progress) {
            if (S->inflight > 0) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(10));
                lk.lock();
            } else {
                // a system-clock deadline (pthread_cond_timedwait), which thread sanitizers
                // intercept, unlike the steady-clock wait; the 5 ms is only a re-check period
                S->cv.wait_until(lk, std::chrono::system_clock::now() + std::chrono::milliseconds(5));
            }
        }
    }
}

void server_destroy(Ctx* c)
{
    Server* S = c->server;
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    for (Slot& sl : S->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        free_workspace(c, sl.ws);
        if (sl.hpin) (void)hipHostFree(sl.hpin);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto& kv : S->cache) free_mol(S, kv.second.get(), nullptr);
    (void)hipStreamSynchronize(nullptr);
    {   // hand the pool's cached fragment memory back to the device
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, c->device) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
        (void)hipGetLastError();
    }
    for (DevBuf& b : S->arena) c->release(b);
    delete S;
    c->server = nullptr;
}

}  // namespace tcm

using namespace tcm;

extern "C" int tcm_server_start(tcm_ctx* t, const tcm_server_cfg* cfg)
{
    if (!t || !cfg || cfg->max_inflight_batches < 1 || cfg->max_inflight_batches > 16 || cfg->max_batch_pairs < 1 ||
        cfg->queue_capacity < 1)
        return TCM_EINVAL;
    Ctx& c = t->c;
    if (c.server) return TCM_EINVAL;
    (void)hipSetDevice(c.device);
    Server* S = new (std::nothrow) Server();
    if (!S) return TCM_ENOMEM;
    S->c = &c;
    S->cfg = *cfg;
    S->slots.resize(cfg->max_inflight_batches);
    for (Slot& sl : S->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
            c.server = S;
            server_destroy(&c);
            return TCM_EDEVICE;
        }
    }
    c.server = S;
    S->th = std::thread(server_loop, S);
    return TCM_OK;
}

extern "C" int tcm_submit(tcm_ctx* t, const tcm_request* r, uint64_t* ticket)
{
    if (!t || !r || !ticket || !t->c.server) return TCM_EINVAL;
    if (r->L < 0 || r->L > LMAX || (r->precision != TCM_F64 && r->precision != TCM_F32C)) return TCM_EINVAL;
    if (!std::isfinite(r->R[0]) || !std::isfinite(r->R[1]) || !std::isfinite(r->R[2])) return TCM_EINVAL;
    const double qq = r->quat_b[0] * r->quat_b[0] + r->quat_b[1] * r->quat_b[1] + r->quat_b[2] * r->quat_b[2] +
                      r->quat_b[3] * r->quat_b[3];
    if (!std::isfinite(qq) || !(qq > 0) || r->n_a < 0 || r->n_b < 0) return TCM_EINVAL;
    Server* S = t->c.server;
    {
        std::lock_guard<std::mutex> g(S->mu);
        if (S->stop) return TCM_EINVAL;
        if ((int)S->pending.size() >= S->cfg.queue_capacity) return TCM_EAGAIN;
        SReq q;
        q.ticket = S->next_ticket++;
        q.r = *r;
        q.t_submit = clock_t_::now();
        S->pending.push_back(q);
        S->live[q.ticket] = 1;
        *ticket = q.ticket;
    }
    S->cv.notify_one();
    return TCM_OK;
}

extern "C" int tcm_poll(tcm_ctx* t, uint64_t ticket, double* U, int32_t* st, double* lat)
{
    if (!t || !t->c.server) return TCM_EINVAL;
    Server* S = t->c.server;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->done.find(ticket);
    if (it == S->done.end()) return S->live.count(ticket) ? TCM_EAGAIN : TCM_ENOTFOUND;
    if (U) *U = it->second.U;
    if (st) *st = it->second.status;
    if (lat) *lat = it->second.latency;
    S->done.erase(it);
    S->live.erase(ticket);
    return TCM_OK;
}

extern "C" int tcm_server_stop(tcm_ctx* t)
{
    if (!t || !t->c.server) return TCM_EINVAL;
    server_destroy(&t->c);
    return TCM_OK;
}

extern "C" int tcm_server_stats(tcm_ctx* t, int64_t* completed, int64_t* launches, int64_t* hits, int64_t* misses,
                                int64_t* deferred, int64_t* evictions, int64_t* dropped, int64_t* gone)
{
    if (!t || !t->c.server) return TCM_EINVAL;
    Server* S = t->c.server;
    std::lock_guard<std::mutex> g(S->mu);
    if (completed) *completed = S->completed;
    if (launches) *launches = S->launches;
    if (hits) *hits = S->hits;
    if (misses) *misses = S->misses;
    if (deferred) *deferred = S->deferred;
    if (evictions) *evictions = S->evictions;
    if (dropped) *dropped = S->dropped;
    if (gone) *gone = S->gone;
    return TCM_OK;
}
