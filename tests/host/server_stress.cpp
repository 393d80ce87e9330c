// Random request streams against the serving loop (compiled for the CPU with the HIP
// stand-in) under tight HBM budgets: every ticket completes, every successful result names
// the two fragments of its request, device memory never exceeds the budget.
#include "tcm.h"
#include <vector>
#include <random>
#include <cstdio>
#include <thread>
#include <chrono>
#include <cmath>
#include <map>
// Plans return their device memory to the context's budget when destroyed.
static int plan_lifecycle() {
    tcm_ctx* ctx; if (tcm_create(&ctx, 0, 0, 0)) return 1;
    std::vector<double> xyz(3 * 5000, 1.0), q(5000, 0.5);
    for (int i = 0; i < 5000; ++i) xyz[3 * i] = i * 1e-3;
    tcm_mol_id a, b;
    if (tcm_mol_upload(ctx, xyz.data(), q.data(), 5000, nullptr, TCM_F32C, &a) ||
        tcm_mol_upload(ctx, xyz.data(), q.data(), 5000, nullptr, TCM_F64, &b)) return 2;
    // the molecules' own moment tables grow to the largest order a plan asks for (they stay
    // with the molecules): warm up with every order first, then every plan must give back
    // exactly what it took
    size_t base = 0;
    for (int rep = 0; rep < 60; ++rep) {
        if (rep == 10) tcm_mem_info(ctx, &base, nullptr);
        tcm_pair_req r[2] = {};
        r[0].a = a; r[0].b = b; r[0].R[0] = 100.0; r[0].quat_b[0] = 1; r[0].L = 8 + rep % 9;
        r[1] = r[0]; r[1].L = 3;
        tcm_plan* p;
        if (tcm_plan_create(ctx, r, 2, rep & 1, &p)) { printf("plan_create failed\n"); return 3; }
        if (tcm_plan_run(ctx, p)) return 4;
        tcm_plan_destroy(p);
        size_t u; tcm_mem_info(ctx, &u, nullptr);
        if (rep >= 10 && u != base) { printf("plan %d: used %zu != %zu after destroy\n", rep, u, base); return 5; }
    }
    {   // a live plan pins its molecules; its moments count as resident only once it has run
        tcm_mol_id c2;
        if (tcm_mol_upload(ctx, xyz.data(), q.data(), 4000, nullptr, TCM_F32C, &c2)) return 6;
        tcm_pair_req r = {};
        r.a = a; r.b = c2; r.R[0] = 100.0; r.quat_b[0] = 1; r.L = 6;
        tcm_plan* p;
        if (tcm_plan_create(ctx, &r, 1, 0, &p)) return 7;
        if (tcm_mol_release(ctx, c2) != TCM_EAGAIN) { printf("release of a planned molecule allowed\n"); return 8; }
        std::vector<double> Q(49);
        // not run yet: a reuse recomputes instead of reading the plan's unwritten table
        if (tcm_mol_moments(ctx, c2, 6, TCM_REUSE, Q.data(), nullptr, nullptr) || Q[0] != 4000.0) {
            printf("reuse before the plan ran read %g\n", Q[0]);
            return 9;
        }
        if (tcm_plan_run(ctx, p)) return 10;
        tcm_plan_destroy(p);
        if (tcm_mol_release(ctx, c2) != TCM_OK) return 11;
    }
    tcm_destroy(ctx);
    printf("plan lifecycle ok\n");
    return 0;
}

extern "C" void mock_set_faults(int alloc_every, int launch_every);
extern "C" long mock_faults_fired();

// Injected failures: every 13th device allocation and every 29th tile launch fail while 400
// requests are served (new fragments copied or borrowed, resident ones reused).  Every ticket
// must complete; a request either succeeds with the right value or fails alone with
// TCM_ENOMEM / TCM_EDEVICE; with the faults off again a fresh batch must succeed entirely;
// and after the server stops the context's device memory is back where it started.
static int fault_injection() {
    tcm_ctx* ctx; if (tcm_create(&ctx, 0, 0, 0)) return 1;
    size_t base; tcm_mem_info(ctx, &base, nullptr);
    std::mt19937 rng(99);
    const int nfr = 16;
    std::vector<std::vector<double>> fr(nfr);
    std::vector<int64_t> nat(nfr);
    for (int f = 0; f < nfr; ++f) { nat[f] = 1 + rng() % 5000; fr[f].assign(4 * nat[f], 1.0); }
    tcm_server_cfg cfg{3, 8, 1024, 0};
    if (tcm_server_start(ctx, &cfg)) return 2;
    auto serve = [&](int nreq, int64_t key0, int& ok, int& failed, int& bad) -> int {
        std::vector<uint64_t> tk; std::vector<int> fa, fb;
        for (int i = 0; i < nreq; ++i) {
            tcm_request r{}; int a = rng() % nfr, b = rng() % nfr;
            const bool fresh = (rng() % 3) != 0;
            r.key_a = fresh ? key0 + 2 * i : a; r.key_b = fresh ? key0 + 2 * i + 1 : b;
            if (!fresh) { a = (int)r.key_a; b = (int)r.key_b; }
            for (int k = 0; k < 4; ++k) { r.atoms_a[k] = fr[a].data() + k * nat[a]; r.atoms_b[k] = fr[b].data() + k * nat[b]; }
            r.n_a = nat[a]; r.n_b = nat[b];
            r.R[0] = 100.0; r.quat_b[0] = 1; r.L = rng() % 17; r.precision = rng() % 2;
            r.flags = (rng() % 2) ? TCM_BORROW_ATOMS : 0;
            uint64_t t; int rc;
            while ((rc = tcm_submit(ctx, &r, &t)) == TCM_EAGAIN) std::this_thread::sleep_for(std::chrono::microseconds(50));
            if (rc) { printf("faults: submit rc %d\n", rc); return 3; }
            tk.push_back(t); fa.push_back(a); fb.push_back(b);
        }
        int done = 0;
        std::vector<char> got(nreq, 0);
        auto t0 = std::chrono::steady_clock::now();
        while (done < nreq) {
            for (int i = 0; i < nreq; ++i) {
                if (got[i]) continue;
                double U, lat; int32_t st;
                const int rc = tcm_poll(ctx, tk[i], &U, &st, &lat);
                if (rc == TCM_EAGAIN) continue;
                if (rc != TCM_OK) { printf("faults: poll rc %d\n", rc); return 4; }
                got[i] = 1; ++done;
                if (st == TCM_OK) {
                    const double want = nat[fa[i]] + 1e-3 * nat[fb[i]];
                    if (std::fabs(U - want) > 1e-9 * want) ++bad; else ++ok;
                } else if (st == TCM_ENOMEM || st == TCM_EDEVICE) {
                    ++failed;
                } else {
                    ++bad;
                }
            }
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(20)) { printf("faults: stuck at %d/%d\n", done, nreq); return 5; }
        }
        return 0;
    };
    int ok = 0, failed = 0, bad = 0;
    mock_set_faults(13, 29);
    if (int rc = serve(400, 1000, ok, failed, bad)) return rc;
    const long fired = mock_faults_fired();
    mock_set_faults(0, 0);
    int ok2 = 0, failed2 = 0, bad2 = 0;
    if (int rc = serve(100, 100000, ok2, failed2, bad2)) return rc;
    tcm_server_stop(ctx);
    size_t used; tcm_mem_info(ctx, &used, nullptr);
    tcm_destroy(ctx);
    printf("faults: fired %ld | ok %d failed %d bad %d | after: ok %d failed %d bad %d | used %zu base %zu %s\n",
           fired, ok, failed, bad, ok2, failed2, bad2, used, base,
           (fired > 0 && failed > 0 && ok > 0 && bad == 0 && ok2 == 100 && used == base) ? "ok" : "FAIL");
    if (!(fired > 0 && failed > 0 && ok > 0 && bad == 0 && ok2 == 100 && used == base)) return 6;
    return 0;
}

int main(int argc, char** argv) {
    if (int rc = plan_lifecycle()) return 10 + rc;
    if (int rc = fault_injection()) return 20 + rc;
    int seeds = argc > 1 ? atoi(argv[1]) : 20;
    for (int seed = 0; seed < seeds; ++seed) {
        std::mt19937 rng(seed);
        tcm_ctx* ctx; if (tcm_create(&ctx, 0, 0, 0)) return 1;
        size_t used; tcm_mem_info(ctx, &used, nullptr);
        int nfr = 12 + seed % 10;
        std::vector<std::vector<double>> fr(nfr);
        std::vector<int64_t> nat(nfr);
        for (int f = 0; f < nfr; ++f) { nat[f] = 1 + rng() % 20000; fr[f].assign(4 * nat[f], 1.0); }
        tcm_server_cfg cfg{1 + (int)(rng() % 4), 1 + (int)(rng() % 8), 64, 0};
        if (tcm_server_start(ctx, &cfg)) return 2;
        tcm_set_budget(ctx, used + 600000 + rng() % 2000000);
        std::vector<uint64_t> tk; std::vector<int> fa, fb, Ls;
        std::map<int64_t, int> seen;
        int nreq = 300;
        for (int i = 0; i < nreq; ++i) {
            tcm_request r{}; int a = rng() % nfr, b = rng() % nfr;
            r.key_a = a; r.key_b = b;
            bool with_atoms = (rng() % 4) != 0;
            for (int k = 0; k < 4; ++k) { r.atoms_a[k] = with_atoms ? fr[a].data() + k * nat[a] : nullptr; r.atoms_b[k] = with_atoms ? fr[b].data() + k * nat[b] : nullptr; }
            r.n_a = nat[a]; r.n_b = nat[b];
            r.R[0] = (rng() % 10 == 0) ? 0.1 : 100.0; r.quat_b[0] = 1; r.L = rng() % 33; r.precision = rng() % 2;
            r.flags = (rng() % 3 == 0) ? TCM_BORROW_ATOMS : 0;
            uint64_t t; int rc;
            while ((rc = tcm_submit(ctx, &r, &t)) == TCM_EAGAIN) std::this_thread::sleep_for(std::chrono::microseconds(50));
            if (rc) { printf("submit rc %d\n", rc); return 3; }
            tk.push_back(t); fa.push_back(a); fb.push_back(b); Ls.push_back(r.L);
        }
        int done = 0, bad = 0, nomem = 0, nf = 0, dom = 0;
        auto t0 = std::chrono::steady_clock::now();
        std::vector<char> got(nreq, 0);
        while (done < nreq) {
            for (int i = 0; i < nreq; ++i) {
                if (got[i]) continue;
                double U, lat; int32_t st;
                int rc = tcm_poll(ctx, tk[i], &U, &st, &lat);
                if (rc == TCM_OK) {
                    got[i] = 1; ++done;
                    if (st == TCM_OK) { double want = nat[fa[i]] + 1e-3 * nat[fb[i]]; if (std::fabs(U - want) > 1e-9 * want) { ++bad; if (bad < 5) printf("bad i=%d a=%d(n=%ld) b=%d(n=%ld) U=%.6f want=%.6f L=%d\n", i, fa[i], (long)nat[fa[i]], fb[i], (long)nat[fb[i]], U, want, Ls[i]); } }
                    else if (st == TCM_ENOMEM) ++nomem; else if (st == TCM_ENOTFOUND) ++nf; else if (st == TCM_EDOMAIN) ++dom; else ++bad;
                } else if (rc != TCM_EAGAIN) { printf("poll rc %d\n", rc); return 4; }
            }
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(20)) { printf("seed %d: stuck at %d/%d\n", seed, done, nreq); return 5; }
        }
        int64_t c, l, h, m, d, e, dr, g; tcm_server_stats(ctx, &c, &l, &h, &m, &d, &e, &dr, &g);
        size_t u2, b2; tcm_mem_info(ctx, &u2, &b2);
        printf("seed %d: done %d bad %d nomem %d notfound %d edomain %d | launches %lld hits %lld misses %lld deferred %lld evictions %lld | used %zu <= budget %zu %s\n",
               seed, done, bad, nomem, nf, dom, (long long)l, (long long)h, (long long)m, (long long)d, (long long)e, u2, b2, u2 <= b2 ? "ok" : "OVER");
        tcm_server_stop(ctx);
        tcm_destroy(ctx);
        if (bad) return 6;
        if (e > m) { printf("seed %d: %lld evictions > %lld misses (fragments fetched and dropped)\n", seed, (long long)e, (long long)m); return 7; }
    }
    return 0;
}
