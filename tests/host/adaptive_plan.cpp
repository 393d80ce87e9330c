// Adaptive plans on the HIP stand-in: a plan's energies, statuses, orders and bounds equal the
// one-shot adaptive call's on every run, its device memory goes back to the context's budget
// when it is destroyed, and creations that fail under injected allocation failures give back
// what they took.
#include "tcm.h"
#include <vector>
#include <cstdio>
extern "C" void mock_set_faults(int alloc_every, int launch_every);
int main()
{
    tcm_ctx* ctx;
    if (tcm_create(&ctx, 0, 0, 0)) return 1;
    std::vector<double> xyz(3 * 3000, 1.0), q(3000, 0.5);
    for (int i = 0; i < 3000; ++i) xyz[3 * i] = i * 1e-3;
    tcm_mol_id a, b;
    if (tcm_mol_upload(ctx, xyz.data(), q.data(), 3000, nullptr, TCM_F64, &a) ||
        tcm_mol_upload(ctx, xyz.data(), q.data(), 2000, nullptr, TCM_F32C, &b))
        return 2;
    const int n = 300;
    std::vector<tcm_pair_req> r(n);
    for (int i = 0; i < n; ++i) {
        r[i] = tcm_pair_req{};
        r[i].a = a; r[i].b = b; r[i].R[0] = 50.0 + i; r[i].quat_b[0] = 1.0; r[i].L = 4 + i % 13;
    }
    std::vector<double> U1(n), B1(n), U(n), B(n);
    std::vector<int32_t> L1(n), S1(n), Lc(n), S(n);
    if (tcm_batch_energy_adaptive(ctx, r.data(), n, 1e-3, U1.data(), L1.data(), B1.data(), S1.data())) return 3;
    size_t base = 0;
    for (int rep = 0; rep < 6; ++rep) {
        tcm_plan* p;
        if (tcm_plan_create_adaptive(ctx, r.data(), n, 1e-3, rep & 1, &p)) return 4;
        for (int k = 0; k < 2; ++k) {
            if (tcm_plan_run(ctx, p) || tcm_plan_results(ctx, p, U.data(), S.data()) ||
                tcm_plan_orders(ctx, p, Lc.data(), B.data()))
                return 5;
            for (int i = 0; i < n; ++i)
                if (U[i] != U1[i] || S[i] != S1[i] || Lc[i] != L1[i] || B[i] != B1[i]) {
                    printf("pair %d differs\n", i);
                    return 6;
                }
        }
        tcm_plan_destroy(p);
        size_t u;
        tcm_mem_info(ctx, &u, nullptr);
        if (rep == 1) base = u;
        if (rep > 1 && u != base) {
            printf("used %zu != %zu after destroy\n", u, base);
            return 7;
        }
    }
    {   // fixed-order plans have no orders; a tolerance must be positive
        tcm_plan* p;
        if (tcm_plan_create(ctx, r.data(), n, 0, &p)) return 8;
        if (tcm_plan_orders(ctx, p, Lc.data(), B.data()) != TCM_EINVAL) return 9;
        tcm_plan_destroy(p);
        if (tcm_plan_create_adaptive(ctx, r.data(), n, 0.0, 0, &p) != TCM_EINVAL) return 10;
    }
    size_t u0;
    tcm_mem_info(ctx, &u0, nullptr);
    int failed = 0;
    for (int every = 1; every <= 12; ++every) {
        mock_set_faults(every, 0);
        tcm_plan* p = nullptr;
        const int rc = tcm_plan_create_adaptive(ctx, r.data(), n, 1e-3, every & 1, &p);
        mock_set_faults(0, 0);
        if (rc == TCM_OK) tcm_plan_destroy(p);
        else ++failed;
        size_t u;
        tcm_mem_info(ctx, &u, nullptr);
        if (u != u0) {
            printf("faults every %d allocations: used %zu != %zu\n", every, u, u0);
            return 11;
        }
    }
    if (failed == 0) return 12;
    printf("adaptive plans ok (%d creations failed under injected faults)\n", failed);
    tcm_mol_release(ctx, a);
    tcm_mol_release(ctx, b);
    tcm_destroy(ctx);
    return 0;
}
