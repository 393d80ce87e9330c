// Host runtime of libtcm: context and FP64 coefficient tables, resident molecules, the
// batch planner, graph-captured plans, tuning.  Every arithmetic step of the method runs
// in the HIP kernels of tcm_kernels.hip; the host only validates, plans and copies.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <string>

#include "tcm_runtime.h"

namespace tcm {

// ------------------------------------------------------------------ buffers
int Ctx::alloc(DevBuf& b, size_t bytes)
{
    if (bytes <= b.cap && b.p) return TCM_OK;
    size_t want = bytes < 256 ? 256 : bytes;
    if (b.p) {
        if (hipFree(b.p) != hipSuccess) return TCM_EDEVICE;
        used -= b.cap;
        b.p = nullptr;
        b.cap = 0;
    }
    if (budget && used.load() + want > budget) return TCM_ENOMEM;
    void* p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return TCM_ENOMEM;
    }
    b.p = p;
    b.cap = want;
    used += want;
    return TCM_OK;
}

int Ctx::alloc_async(DevBuf& b, size_t bytes, hipStream_t s)
{
    if (bytes <= b.cap && b.p) return TCM_OK;
    release_async(b, s);
    const size_t want = bytes < 256 ? 256 : bytes;
    if (budget && used.load() + want > budget) return TCM_ENOMEM;
    void* p = nullptr;
    if (hipMallocAsync(&p, want, s) != hipSuccess) {
        (void)hipGetLastError();
        return TCM_ENOMEM;
    }
    b.p = p;
    b.cap = want;
    used += want;
    return TCM_OK;
}

void Ctx::release_async(DevBuf& b, hipStream_t s)
{
    if (b.p) {
        (void)hipFreeAsync(b.p, s);
        used -= b.cap;
        b.p = nullptr;
        b.cap = 0;
    }
}

void Ctx::release(DevBuf& b)
{
    if (b.p) {
        (void)hipFree(b.p);
        used -= b.cap;
    }
    b.p = nullptr;
    b.cap = 0;
}

int Ctx::ensure_pinned(size_t bytes)
{
    if (bytes <= hpin_cap && hpin) return TCM_OK;
    if (hpin) (void)hipHostFree(hpin);
    hpin = nullptr;
    hpin_cap = 0;
    size_t want = bytes < 4096 ? 4096 : bytes;
    if (hipHostMalloc(&hpin, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return TCM_ENOMEM;
    }
    hpin_cap = want;
    return TCM_OK;
}

static int bucket_of(int64_t n)
{
    int b = 0;
    while (b < 40 && (int64_t(1) << (b + 1)) <= n) ++b;
    return b;
}

int64_t tune_key(int prec, int L, int64_t n) { return (int64_t)prec * 100000 + L * 100 + bucket_of(n); }

// Atoms per thread per tile.  A function of (precision, L, n) only, so a molecule's tiling --
// and therefore every rounding of its moments -- is the same whatever else shares a launch.
// In the FP32 path a thread sums its kper atoms in plain FP32 (everything above is merged with
// TwoSum), so kper is part of that path's error bound, (8(l+1) + 2 kper + 64) 2^-24 times the
// absolute sum of a moment: it never exceeds the context's cap f32_run_max.
int Ctx::kper_for(int prec, int L, int64_t n)
{
    int k;
    auto it = tune.find(tune_key(prec, L, n));
    if (it != tune.end()) {
        k = it->second;
    } else {
        // default: aim at ~16 tiles per molecule, 4 <= kper <= 64, powers of two
        int64_t want = n / (WG * 16);
        k = 4;
        while (k < 64 && k < want) k <<= 1;
    }
    if (prec == TCM_F32C && k > f32_run_max) k = f32_run_max;
    return k;
}

// ------------------------------------------------------------------ FP64 tables
// Racah-normalised solid harmonics C_lm(x, y, z), packed, m >= 0, by the standard
// recurrences (used only to build the rotation tables below).
static void racah_packed(int L, double x, double y, double z, double* out)
{
    const double r2 = x * x + y * y + z * z;
    std::vector<double> cr((L + 1) * (L + 1)), ci((L + 1) * (L + 1));
    auto at = [&](int l, int m) { return l * (l + 1) / 2 + m; };
    cr.assign((L + 1) * (L + 2) / 2, 0.0);
    ci.assign((L + 1) * (L + 2) / 2, 0.0);
    cr[0] = 1.0;
    for (int m = 1; m <= L; ++m) {
        const double f = -std::sqrt((2.0 * m - 1.0) / (2.0 * m));
        const double pr = cr[at(m - 1, m - 1)], pi = ci[at(m - 1, m - 1)];
        cr[at(m, m)] = f * (x * pr - y * pi);
        ci[at(m, m)] = f * (x * pi + y * pr);
    }
    for (int m = 0; m < L; ++m) {
        const double f = std::sqrt(2.0 * m + 1.0) * z;
        cr[at(m + 1, m)] = f * cr[at(m, m)];
        ci[at(m + 1, m)] = f * ci[at(m, m)];
    }
    for (int m = 0; m <= L; ++m)
        for (int l = m + 2; l <= L; ++l) {
            const double d = std::sqrt((double)l * l - (double)m * m);
            const double a = (2.0 * l - 1.0) / d;
            const double b = std::sqrt(((double)l - 1.0) * (l - 1.0) - (double)m * m) / d;
            cr[at(l, m)] = a * z * cr[at(l - 1, m)] - b * r2 * cr[at(l - 2, m)];
            ci[at(l, m)] = a * z * ci[at(l - 1, m)] - b * r2 * ci[at(l - 2, m)];
        }
    for (int l = 0; l <= L; ++l) {
        out[l * l] = cr[at(l, 0)];
        for (int m = 1; m <= l; ++m) {
            out[l * l + 2 * m - 1] = cr[at(l, m)];
            out[l * l + 2 * m] = ci[at(l, m)];
        }
    }
}

static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            const double dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        const double dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

// Rotation tables.  D^l maps the packed order-l moments of a set of charges to those of the
// charges rotated by +90 degrees about x ((x, y, z) -> (x, -z, y)); built by exact quadrature
// of C_l(X p) C_l(p) over the sphere (Gauss-Legendre in cos theta with l+1 nodes, 2l+1
// equispaced phi: exact for the degree-2l integrands).  The inverse follows from the
// orthogonality norms g = 4pi/(2l+1) * (1 for m = 0, 1/2 for the Re/Im parts of m > 0):
// invariance of the sphere measure gives D G D^T = G, so (D^{-1})_ij = D_ji g_i / g_j.
// Both matrices are sparse: a 90 degree rotation about x maps each real basis function of one
// cos / sin type and m parity onto functions of one type and one m parity, so row i's nonzero
// columns are the packed indices max(0, jb_i + 4k), k = 0 .. cnt_i - 1 (a quarter of the
// entries); every other entry is zero up to the quadrature's rounding, which is checked here.
// Compressed layout (all doubles): hdr[l] = offset of order l's block, l = 0 .. Lmax; block l =
// codes[2n] (rows of D, then of D^{-1}: (jb + 1) + 65536 cnt), then the nonzero values of D
// and of D^{-1}, K = l/2 + 1 slots per row, stored slot by slot (row i's slot k at k n + i) so
// that the lanes computing consecutive rows read consecutive addresses.
static int compress_rotation(const std::vector<double>& dense, int n, double* codes, double* vals)
{
    const int l = (n - 1) / 2, K = l / 2 + 1;
    double mx = 0.0;
    for (double v : dense) mx = std::max(mx, std::fabs(v));
    for (int i = 0; i < n; ++i) {
        // the row's class from its largest entry: column 0 is (cos, m = 0), odd j is
        // (cos, m = (j+1)/2), even j > 0 is (sin, m = j/2); the class holds every m of that
        // parity and type (some members can vanish by accident, so they are kept)
        int jm = 0;
        for (int j = 1; j < n; ++j)
            if (std::fabs(dense[i * n + j]) > std::fabs(dense[i * n + jm])) jm = j;
        const bool sn = jm > 0 && !(jm & 1);
        const int m = jm == 0 ? 0 : sn ? jm / 2 : (jm + 1) / 2;
        const int m0 = sn ? ((m & 1) ? 1 : 2) : (m & 1);
        const int jb = sn ? 2 * m0 : 2 * m0 - 1;
        const int cnt = m0 <= l ? (l - m0) / 2 + 1 : 0;
        if (cnt < 1 || cnt > K) return -1;
        std::vector<char> in(n, 0);
        for (int k = 0; k < cnt; ++k) {
            const int j = std::max(0, jb + 4 * k);
            in[j] = 1;
            vals[(size_t)k * n + i] = dense[i * n + j];
        }
        for (int j = 0; j < n; ++j)          // nothing outside the class but rounding
            if (!in[j] && std::fabs(dense[i * n + j]) > 1e-12 * mx) return -1;
        codes[i] = (double)(jb + 1) + 65536.0 * (double)cnt;
    }
    return 0;
}

static std::vector<double> build_rotation_tables(int Lmax)
{
    std::vector<double> out((size_t)Lmax + 1, 0.0);
    std::vector<double> cp((Lmax + 1) * (Lmax + 1)), cx((Lmax + 1) * (Lmax + 1));
    for (int l = 0; l <= Lmax; ++l) {
        const int n = 2 * l + 1, K = l / 2 + 1;
        if (Lmax != LMAX || out.size() != (size_t)rot_block_offset(l)) return {};   // the kernels' layout
        out[l] = (double)out.size();
        const size_t base = out.size();
        out.resize(base + 2 * (size_t)n + 2 * (size_t)K * n, 0.0);
        std::vector<double> gx, gw;
        gauss_legendre(l + 1, gx, gw);
        std::vector<double> D(n * n, 0.0);
        for (int a = 0; a <= l; ++a) {
            const double ct = gx[a], st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
            for (int b = 0; b < n; ++b) {
                const double ph = 2.0 * M_PI * b / n;
                const double px = st * std::cos(ph), py = st * std::sin(ph), pz = ct;
                const double wt = gw[a] * 2.0 * M_PI / n;
                racah_packed(l, px, py, pz, cp.data());
                racah_packed(l, px, -pz, py, cx.data());
                const double* u = cp.data() + l * l;
                const double* v = cx.data() + l * l;
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) D[i * n + j] += wt * v[i] * u[j];
            }
        }
        const double g0 = 4.0 * M_PI / n;
        auto g = [&](int i) { return i == 0 ? g0 : 0.5 * g0; };
        std::vector<double> Dd(n * n), Di(n * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Dd[i * n + j] = D[i * n + j] / g(j);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Di[i * n + j] = Dd[j * n + i] * g(i) / g(j);
        double* blk = out.data() + base;
        if (compress_rotation(Dd, n, blk, blk + 2 * n) != 0 ||
            compress_rotation(Di, n, blk + n, blk + 2 * n + (size_t)K * n) != 0)
            return {};
        // the pair kernels take a row's first column from its class (rot_class_jb)
        for (int inv = 0; inv < 2; ++inv)
            for (int i = 0; i < n; ++i) {
                const bool sn = i > 0 && !(i & 1);
                const int m = i == 0 ? 0 : sn ? i / 2 : (i + 1) / 2;
                if (std::fmod(blk[inv * n + i], 65536.0) != (double)(rot_class_jb(sn, m, l) + 1)) return {};
            }
    }
    return out;
}

// 1/k_lm of the normalised recurrence (k_mm = (-1)^m sqrt((2m)!)/(2m-1)!!,
// k_{m+1,m} = k_mm / sqrt(2m+1), k_lm = k_{l-1,m} xi_lm / A_lm, A_lm = (2l-1)/sqrt(l^2-m^2))
// and 1/sqrt((l+m)!(l-m)!), per packed index.
static void build_norm_tables(int Lmax, std::vector<double>& invk, std::vector<double>& invf)
{
    const int NH = (Lmax + 1) * (Lmax + 1);
    invk.assign(NH, 0.0);
    invf.assign(NH, 0.0);
    std::vector<long double> fact(2 * Lmax + 2);
    fact[0] = 1.0L;
    for (size_t i = 1; i < fact.size(); ++i) fact[i] = fact[i - 1] * (long double)i;
    for (int m = 0; m <= Lmax; ++m) {
        long double dfac = 1.0L;
        for (int j = 1; j < 2 * m; j += 2) dfac *= j;
        long double k = ((m & 1) ? -1.0L : 1.0L) * std::sqrt(fact[2 * m]) / dfac;
        long double xi = 1.0L;
        for (int l = m; l <= Lmax; ++l) {
            if (l == m + 1) {
                k = k / std::sqrt((long double)(2 * m + 1));
            } else if (l >= m + 2) {
                xi = ((2.0L * l - 1.0L) * (2.0L * l - 3.0L) / (((long double)l - 1 - m) * ((long double)l - 1 + m))) / xi;
                const long double A = (2.0L * l - 1.0L) / std::sqrt((long double)l * l - (long double)m * m);
                k = k * xi / A;
            }
            const double ik = (double)(1.0L / k);
            const double f = (double)(1.0L / std::sqrt(fact[l + m] * fact[l - m]));
            if (m == 0) {
                invk[l * l] = ik;
                invf[l * l] = f;
            } else {
                invk[l * l + 2 * m - 1] = invk[l * l + 2 * m] = ik;
                invf[l * l + 2 * m - 1] = invf[l * l + 2 * m] = f;
            }
        }
    }
}

// ------------------------------------------------------------------ planning
static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Device bytes build_plan would add to ws for these jobs (growth of each buffer beyond its
// current capacity), so that a caller can make room under its HBM budget first.
// Statistics items of a molecule: one per chunk of STATS_CHUNK atoms, at most STATS_ITEMS_MAX;
// a larger molecule gives each item a run of consecutive chunks (the kernel derives the run
// length from the chunk and item counts), so its centre/scale merge reads few records.
constexpr int64_t STATS_ITEMS_MAX = 8192;
int64_t stats_items_for(int64_t n)
{
    const int64_t nch = n > 0 ? (n + STATS_CHUNK - 1) / STATS_CHUNK : 1;
    const int64_t per = (nch + STATS_ITEMS_MAX - 1) / STATS_ITEMS_MAX;
    return (nch + per - 1) / per;
}

size_t workspace_growth(Ctx* c, const Workspace& ws, const std::vector<MolJob>& mols, const std::vector<PairJob>& pairs)
{
    int64_t off_f = 0, off_d = 0, off_s = 0, off_r2 = 0, nitems = 0;
    for (const MolJob& j : mols) {
        const int kper = c->kper_for(j.prec, j.L, j.n);
        const int64_t ta = (int64_t)WG * kper;
        const int64_t nt = j.n > 0 ? (j.n + ta - 1) / ta : 1;
        nitems += nt * num_blocks_for(j.prec, j.L) + 8 * num_blocks_for(j.prec, j.L);   // with the padding
        const int64_t ns = stats_items_for(j.n);
        if (j.prec == TCM_F32C) off_f += 2 * nt * nh(j.L); else off_d += nt * nh(j.L);
        off_s += ns;
        off_r2 += nt;
    }
    const size_t nmol = mols.size(), np = pairs.size();
    int plmax = 0;
    for (const PairJob& j : pairs) plmax = std::max(plmax, j.L);
    const size_t blob = sizeof(MolWork) * nmol + (sizeof(PairWork) + sizeof(double) * 2 * FRAME_N) * np +
                        sizeof(int32_t) * (np / PAIR_LANES + 1) + 2 * sizeof(int32_t) * (size_t)off_s +
                        2 * sizeof(int32_t) * (size_t)nitems + 1536;
    const size_t np1 = np > 0 ? np : 1;
    const size_t need[10] = {blob, sizeof(int32_t),
                             sizeof(float) * (size_t)(off_f > 0 ? off_f : 1), sizeof(double) * (size_t)(off_d > 0 ? off_d : 1),
                             sizeof(double) * 10 * (size_t)(off_s > 0 ? off_s : 1), sizeof(double) * (size_t)(off_r2 > 0 ? off_r2 : 1),
                             sizeof(double) * np1, sizeof(int32_t) * np1,
                             sizeof(double) * 2 * (size_t)nh(plmax) * np1, sizeof(double) * (size_t)(plmax + 1) * np1};
    const DevBuf* have[10] = {&ws.blob, &ws.sync, &ws.part_f, &ws.part_d, &ws.stats, &ws.r2, &ws.outU, &ws.outS,
                              &ws.prot, &ws.pum};
    size_t grow = 0;
    for (int i = 0; i < 10; ++i) {
        const size_t want = need[i] < 256 ? 256 : need[i];
        if (want > have[i]->cap) grow += want;
    }
    return grow;
}

// body(k0, k1) over [0, n) in contiguous chunks, on up to 8 host threads when n is large
// (the chunks must touch disjoint memory).
template <typename F>
static void host_parallel(int n, F&& body)
{
    const unsigned hc = std::thread::hardware_concurrency();
    const int nt = n >= 8192 ? (int)std::min(8u, hc > 0 ? hc : 1u) : 1;
    if (nt <= 1) {
        body(0, n);
        return;
    }
    const int per = (n + nt - 1) / nt;
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) {
        const int k0 = t * per, k1 = std::min(n, k0 + per);
        if (k0 < k1) th.emplace_back([&body, k0, k1] { body(k0, k1); });
    }
    body(0, std::min(n, per));
    for (std::thread& x : th) x.join();
}

int build_plan(Ctx* c, Workspace& ws, const std::vector<MolJob>& mols_in, const std::vector<PairJob>& pairs_in,
               BuiltPlan& bp, hipStream_t s)
{
    // molecules sorted by (precision, L): each group's tiles are one launch of the tile
    // kernel compiled for that order
    const int nmol = (int)mols_in.size(), npairs = (int)pairs_in.size();
    std::vector<int> order(nmol), newidx(nmol);
    for (int i = 0; i < nmol; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int u, int v) {
        if (mols_in[u].prec != mols_in[v].prec) return mols_in[u].prec < mols_in[v].prec;
        return mols_in[u].L < mols_in[v].L;
    });
    std::vector<MolJob> mols(nmol);
    for (int i = 0; i < nmol; ++i) {
        mols[i] = mols_in[order[i]];
        newidx[order[i]] = i;
    }
    std::vector<MolWork> mw(nmol);
    std::vector<int32_t> sp(nmol + 1, 0), tp(nmol + 1, 0);
    int64_t off_f = 0, off_d = 0, off_s = 0, off_r2 = 0;
    double flops = 0.0;
    int64_t atoms = 0;
    for (int i = 0; i < nmol; ++i) {
        const MolJob& j = mols[i];
        MolWork& w = mw[i];
        w.x = j.x; w.y = j.y; w.z = j.z; w.q = j.q;
        w.n = j.n;
        w.L = j.L;
        w.prec = j.prec;
        w.kper = c->kper_for(j.prec, j.L, j.n);
        w.nblk = num_blocks_for(j.prec, j.L);
        const int64_t tile_atoms = (int64_t)WG * w.kper;
        const int64_t nt = j.n > 0 ? (j.n + tile_atoms - 1) / tile_atoms : 1;
        const int64_t ns = stats_items_for(j.n);
        if (nt > (1 << 24) || ns > (1 << 24)) return TCM_EINVAL;
        w.ntiles = (int)nt;
        w.nstats = (int)ns;
        w.has_centre = j.has_centre;
        w.centre[0] = j.centre[0]; w.centre[1] = j.centre[1]; w.centre[2] = j.centre[2];
        w.Q = j.Q;
        w.meta = j.meta;
        w.stats_off = off_s;
        w.r2_off = off_r2;
        if (j.prec == TCM_F32C) {
            w.part_off = off_f;
            off_f += 2 * nt * nh(j.L);
        } else {
            w.part_off = off_d;
            off_d += nt * nh(j.L);
        }
        off_s += ns;
        off_r2 += nt;
        sp[i + 1] = sp[i] + (int32_t)ns;
        const int64_t ti = (int64_t)tp[i] + nt * w.nblk;
        if (ti > (1 << 30)) return TCM_EINVAL;
        tp[i + 1] = (int32_t)ti;
        flops += 6.0 * (j.L + 1) * (j.L + 2) * (double)j.n;
        atoms += j.n;
    }
    // pair launch order: largest contractions first (cost ~ (L+1)^4 plus the rotation), so the
    // launch's tail holds the cheap ones; a stable counting sort by L (every pair writes
    // U[out], so the order changes no result).  The records are written in this order
    // straight into the staging buffer below.
    int pair_lmax = 0;
    for (const PairJob& j : pairs_in) pair_lmax = std::max(pair_lmax, j.L);
    std::vector<int32_t> porder(npairs);
    {
        std::vector<int32_t> start(pair_lmax + 2, 0);
        for (const PairJob& j : pairs_in) ++start[pair_lmax - j.L + 1];
        for (int k = 1; k <= pair_lmax + 1; ++k) start[k] += start[k - 1];
        for (int p = 0; p < npairs; ++p) porder[start[pair_lmax - pairs_in[p].L]++] = p;
    }
    // tile items of each (precision, L) group: the tiles in decreasing estimated cost (per-thread
    // instructions: atoms x (recurrence + set-up) + the compensated reduction, summed over the
    // tile's m-blocks), and the m-blocks of one tile on one XCD back to back: workgroup b of a
    // launch runs on XCD b mod 8, so tile j of the group takes the positions
    // 8 (nblk floor(j / 8) + blk) + j mod 8 -- its atoms are read from HBM once and the other
    // m-blocks find them in that XCD's L2.  Positions past the group's tiles (the last round of
    // eight) hold no item (molecule -1).
    std::vector<int64_t> gbeg, gend;                    // item range of each group
    std::vector<int32_t> items;
    {
        std::vector<std::pair<int64_t, int64_t>> key;     // (-cost, tile: molecule << 32 | t)
        int i0 = 0;
        int64_t pos0 = 0;
        while (i0 < nmol) {
            int i1 = i0;
            while (i1 < nmol && mols[i1].prec == mols[i0].prec && mols[i1].L == mols[i0].L) ++i1;
            key.clear();
            const int nblk = mw[i0].nblk;
            for (int i = i0; i < i1; ++i) {
                const MolWork& w = mw[i];
                const Partition part = make_partition(w.L, w.prec == TCM_F32C ? BUDGET_F32 : BUDGET_F64);
                for (int t = 0; t < w.ntiles; ++t) {
                    const int64_t span = std::min<int64_t>(w.n - (int64_t)t * WG * w.kper, (int64_t)WG * w.kper);
                    const int64_t per_thread = (std::max<int64_t>(span, 0) + WG - 1) / WG;
                    int64_t cost = 0;
                    for (int b = 0; b < w.nblk; ++b) {
                        int acc = 0;
                        for (int m = part.start[b]; m < part.start[b + 1]; ++m) acc += chain_cost(w.L, m);
                        cost += per_thread * (5 * acc / 2 + 40) + 9 * acc + 300;
                    }
                    key.push_back({-cost, ((int64_t)i << 32) | t});
                }
            }
            std::stable_sort(key.begin(), key.end(),
                             [](const std::pair<int64_t, int64_t>& u, const std::pair<int64_t, int64_t>& v) {
                                 return u.first < v.first;
                             });
            const int64_t T = (int64_t)key.size();
            const int64_t ng = 8 * (int64_t)nblk * ((T + 7) / 8);
            if (pos0 + ng > (1 << 30)) return TCM_EINVAL;
            items.resize(2 * (size_t)(pos0 + ng));
            for (int64_t q = pos0; q < pos0 + ng; ++q) {
                items[2 * q] = -1;
                items[2 * q + 1] = 0;
            }
            for (int64_t jt = 0; jt < T; ++jt) {
                const int i = (int)(key[jt].second >> 32), t = (int)(key[jt].second & 0xffffffff);
                for (int b = 0; b < nblk; ++b) {
                    const int64_t q = pos0 + 8 * ((int64_t)nblk * (jt / 8) + b) + jt % 8;
                    items[2 * q] = i;
                    items[2 * q + 1] = t * nblk + b;
                }
            }
            gbeg.push_back(pos0);
            gend.push_back(pos0 + ng);
            pos0 += ng;
            i0 = i1;
        }
    }
    const int64_t nitems = (int64_t)items.size() / 2;
    // blob layout
    const size_t o_mw = 0;
    const size_t o_pw = align_up(o_mw + sizeof(MolWork) * nmol, 256);
    const size_t o_sp = align_up(o_pw + sizeof(PairWork) * npairs, 256);
    const size_t o_ti = align_up(o_sp + sizeof(int32_t) * 2 * (size_t)(sp[nmol] > 0 ? sp[nmol] : 1), 256);
    const size_t o_fr = align_up(o_ti + sizeof(int32_t) * 2 * (size_t)(nitems > 0 ? nitems : 1), 256);
    const size_t o_go = align_up(o_fr + sizeof(double) * 2 * FRAME_N * (size_t)npairs, 256);
    const int64_t pgroups = (npairs + PAIR_LANES - 1) / PAIR_LANES;
    const size_t blob = align_up(o_go + sizeof(int32_t) * (size_t)(pgroups > 0 ? pgroups : 1), 256);
    int rc;
    if ((rc = c->alloc(ws.blob, blob)) != TCM_OK) return rc;
    // the staging buffer may still feed the previous plan's copy: wait for that copy only (not
    // for the rest of the stream, where a server slot has just queued its atom copies)
    if (!ws.staged) {
        if (hipEventCreateWithFlags(&ws.staged, hipEventDisableTiming) != hipSuccess) {
            ws.staged = nullptr;
            return TCM_EDEVICE;
        }
    } else if (hipEventSynchronize(ws.staged) != hipSuccess) {
        return TCM_EDEVICE;
    }
    if (blob > ws.hstage_cap) {
        if (ws.hstage) (void)hipHostFree(ws.hstage);
        ws.hstage = nullptr;
        ws.hstage_cap = 0;
        if (hipHostMalloc(&ws.hstage, blob, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return TCM_ENOMEM;
        }
        ws.hstage_cap = blob;
    }
    char* h = (char*)ws.hstage;
    if (nmol) std::memcpy(h + o_mw, mw.data(), sizeof(MolWork) * nmol);
    bool uniform = true;                                  // every group reaches pair_lmax
    const double* qa_all = npairs > 0 ? pairs_in[0].QA : nullptr;
    const double* qb_all = npairs > 0 ? pairs_in[0].QB : nullptr;
    for (const PairJob& j : pairs_in) {
        if (j.QA != qa_all) qa_all = nullptr;
        if (j.QB != qb_all) qb_all = nullptr;
    }
    {
        // the pair records in launch order and the rotation frames of both sides,
        // [side][FRAME_N][pair] (each pair's own: the chunks of pairs are independent)
        PairWork* pw = (PairWork*)(h + o_pw);
        double* fr = (double*)(h + o_fr);
        host_parallel(npairs, [&](int k0, int k1) {
            for (int k = k0; k < k1; ++k) {
                const int p = porder[k];
                const PairJob& j = pairs_in[p];
                PairWork& w = pw[k];
                w.QA = j.QA; w.QB = j.QB; w.metaA = j.metaA; w.metaB = j.metaB;
                w.depA = j.depA >= 0 ? newidx[j.depA] : -1;
                w.depB = j.depB >= 0 ? newidx[j.depB] : -1;
                w.L = j.L; w.flags = j.flags;
                for (int d = 0; d < 3; ++d) w.R[d] = j.R[d];
                for (int d = 0; d < 4; ++d) w.quat[d] = j.quat[d];
                w.has_rot = j.has_rot;
                w.out = p;
                double f[2][FRAME_N];
                side_frame(w.R, w.quat, false, f[0]);
                side_frame(w.R, w.quat, w.has_rot != 0, f[1]);
                for (int side = 0; side < 2; ++side)
                    for (int cc = 0; cc < FRAME_N; ++cc) fr[((size_t)side * FRAME_N + cc) * npairs + k] = f[side][cc];
            }
        });
        int32_t* go = (int32_t*)(h + o_go);
        for (int64_t g = 0; g < pgroups; ++g) go[g] = -1;
        for (int k = 0; k < npairs; ++k) go[k / PAIR_LANES] = std::max(go[k / PAIR_LANES], pw[k].L);
        for (int64_t g = 0; g < pgroups; ++g) uniform = uniform && go[g] == pair_lmax;
    }
    {
        int32_t* si = (int32_t*)(h + o_sp);                // (molecule, chunk) of each STATS item
        for (int i = 0; i < nmol; ++i)
            for (int32_t k = sp[i]; k < sp[i + 1]; ++k) {
                si[2 * k] = i;
                si[2 * k + 1] = k - sp[i];
            }
    }
    if (nitems) std::memcpy(h + o_ti, items.data(), sizeof(int32_t) * 2 * (size_t)nitems);
    bp.groups.clear();
    for (int i = 0; i < nmol; ++i) {
        if (bp.groups.empty() || bp.groups.back().prec != mols[i].prec || bp.groups.back().L != mols[i].L) {
            const int64_t g = (int64_t)bp.groups.size();
            bp.groups.push_back({mols[i].prec, mols[i].L, (int32_t)gbeg[g], (int32_t)gend[g], i, i, sp[i], sp[i], 0.0});
        }
        BuiltPlan::Group& G = bp.groups.back();
        G.work += 6.0 * (mols[i].L + 1) * (mols[i].L + 2) * (double)mols[i].n;
        G.mol_end = i + 1;
        G.stats_end = sp[i + 1];
    }
    bp.ws = &ws;
    const int64_t sync_ints = 1;                            // the error flag
    if ((rc = c->alloc(ws.sync, sizeof(int32_t) * sync_ints)) != TCM_OK) return rc;
    if ((rc = c->alloc(ws.part_f, sizeof(float) * (off_f > 0 ? off_f : 1))) != TCM_OK) return rc;
    if ((rc = c->alloc(ws.part_d, sizeof(double) * (off_d > 0 ? off_d : 1))) != TCM_OK) return rc;
    if ((rc = c->alloc(ws.stats, sizeof(double) * 10 * (off_s > 0 ? off_s : 1))) != TCM_OK) return rc;
    if ((rc = c->alloc(ws.r2, sizeof(double) * (off_r2 > 0 ? off_r2 : 1))) != TCM_OK) return rc;
    if ((rc = c->alloc(ws.outU, sizeof(double) * (npairs > 0 ? npairs : 1))) != TCM_OK) return rc;
    if ((rc = c->alloc(ws.outS, sizeof(int32_t) * (npairs > 0 ? npairs : 1))) != TCM_OK) return rc;
    const size_t np1 = npairs > 0 ? (size_t)npairs : 1;
    if ((rc = c->alloc(ws.prot, sizeof(double) * 2 * (size_t)nh(pair_lmax) * np1)) != TCM_OK) return rc;
    if ((rc = c->alloc(ws.pum, sizeof(double) * (size_t)(pair_lmax + 2) * np1)) != TCM_OK) return rc;
    if (hipMemcpyAsync(ws.blob.p, ws.hstage, blob, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(ws.staged, s) != hipSuccess)
        return TCM_EDEVICE;
    char* d = (char*)ws.blob.p;
    DevPlan& P = bp.P;
    P.mols = (const MolWork*)(d + o_mw);
    P.pairs = (const PairWork*)(d + o_pw);
    P.stats_items = (const int32_t*)(d + o_sp);
    P.tile_items = (const int32_t*)(d + o_ti);
    P.nmol = nmol;
    P.npairs = npairs;
    P.pair_lmax = pair_lmax;
    P.n_stats = sp[nmol];
    P.n_tiles = (int32_t)nitems;
    P.err = (int32_t*)ws.sync.p;
    P.frame = (const double*)(d + o_fr);
    P.gorder = (int32_t*)(d + o_go);
    P.gorder_uniform = uniform ? 1 : 0;
    P.qa_all = qa_all;
    P.qb_all = qb_all;
    P.part_f = (float*)ws.part_f.p;
    P.part_d = (double*)ws.part_d.p;
    P.stats_part = (double*)ws.stats.p;
    P.r2_part = (double*)ws.r2.p;
    P.U = (double*)ws.outU.p;
    P.status = (int32_t*)ws.outS.p;
    P.invk = (const double*)c->t_invk.p;
    P.invf = (const double*)c->t_invf.p;
    P.rot = (const double*)c->t_rot.p;
    P.rotr = P.rot + rot_tables_len();
    P.fact = (const double*)c->t_fact.p;
    P.prot = (double*)ws.prot.p;
    P.pum = (double*)ws.pum.p;
    bp.n_stats = P.n_stats;
    bp.n_tiles = tp[nmol];                                  // work items (no padding positions)
    bp.npairs = npairs;
    bp.n_items = P.n_stats + P.n_tiles + npairs;
    bp.sync_ints = sync_ints;
    bp.atoms = atoms;
    bp.moment_flops = flops;
    return TCM_OK;
}

static int ensure_aux(Workspace& ws, size_t ngroups)
{
    for (int k = 0; k < NLANES; ++k) {
        if (!ws.aux[k] && hipStreamCreateWithFlags(&ws.aux[k], hipStreamNonBlocking) != hipSuccess) {
            ws.aux[k] = nullptr;
            return TCM_EDEVICE;
        }
        if (!ws.join[k] && hipEventCreateWithFlags(&ws.join[k], hipEventDisableTiming) != hipSuccess) {
            ws.join[k] = nullptr;
            return TCM_EDEVICE;
        }
    }
    if (!ws.fork && hipEventCreateWithFlags(&ws.fork, hipEventDisableTiming) != hipSuccess) {
        ws.fork = nullptr;
        return TCM_EDEVICE;
    }
    while (ws.gev.size() < ngroups) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return TCM_EDEVICE;
        ws.gev.push_back(e);
    }
    return TCM_OK;
}

static void destroy_streams(Workspace& ws)
{
    for (int k = 0; k < NLANES; ++k) {
        if (ws.aux[k]) (void)hipStreamDestroy(ws.aux[k]);
        ws.aux[k] = nullptr;
        if (ws.join[k]) (void)hipEventDestroy(ws.join[k]);
        ws.join[k] = nullptr;
    }
    if (ws.fork) (void)hipEventDestroy(ws.fork);
    ws.fork = nullptr;
    for (hipEvent_t e : ws.gev) (void)hipEventDestroy(e);
    ws.gev.clear();
}

// Issue the launches of one run (every kernel has one workgroup per item); the moment
// finalisation and the pair launch end it on s.
//   serial (serial = true): one statistics launch over every molecule of the batch, one
//     centre/scale launch, the tile launch of each (precision, L) group in turn on s (the
//     order a captured graph replays); with ev (5 events) the elapsed time of each step is
//     measured on the launch stream.
//   lanes (serial = false): the groups' tile launches are spread over NLANES streams forked
//     from s, balanced by work (largest first, each to the lightest lane), each lane issuing
//     its smallest launch first, so that the two lanes' workgroups interleave as slots free up
//     and a small group's items fill the tail of a large one.  The statistics (HBM bound) and
//     centre/scale of each group run on s, group by group in the order the lanes start them,
//     and a tile launch waits only for its own group's: the statistics of later groups run
//     beside the ALU-bound tiles of earlier ones.  (The process's streams share four hardware
//     queues: s and two lanes, not one stream per group.)
int run_plan(Ctx* c, const BuiltPlan& bp, hipStream_t s, bool serial, hipEvent_t* ev, bool energy)
{
    (void)c;
    const int S = bp.n_stats;
    const int ng = (int)bp.groups.size();
    if (launch_clear(bp.P.err, bp.sync_ints, s) != hipSuccess) return TCM_EDEVICE;
    auto group_tiles = [&](int g, hipStream_t st) {
        const BuiltPlan::Group& G = bp.groups[g];
        return launch_tiles(G.prec, G.L, bp.P, S + G.begin, S + G.end, st) == hipSuccess;
    };
    if (!serial && ng > 1 && bp.ws && ensure_aux(*bp.ws, (size_t)ng) == TCM_OK) {
        Workspace& ws = *bp.ws;
        std::vector<int> order(ng);
        for (int g = 0; g < ng; ++g) order[g] = g;
        std::stable_sort(order.begin(), order.end(),
                         [&](int u, int v) { return bp.groups[u].work > bp.groups[v].work; });
        const int nl = ng < NLANES ? ng : NLANES;
        double load[NLANES] = {};
        std::vector<int> lanes[NLANES];
        for (int g : order) {
            int lane = 0;
            for (int k = 1; k < nl; ++k)
                if (load[k] < load[lane]) lane = k;
            load[lane] += bp.groups[g].work;
            lanes[lane].push_back(g);
        }
        // each lane's launches smallest first; the statistics in the order the lanes start them
        std::vector<int> stats_order;
        for (size_t r = 0;; ++r) {
            bool any = false;
            for (int k = 0; k < nl; ++k)
                if (r < lanes[k].size()) {
                    stats_order.push_back(lanes[k][lanes[k].size() - 1 - r]);
                    any = true;
                }
            if (!any) break;
        }
        if (hipEventRecord(ws.fork, s) != hipSuccess) return TCM_EDEVICE;
        for (int k = 0; k < nl; ++k)
            if (hipStreamWaitEvent(ws.aux[k], ws.fork, 0) != hipSuccess) return TCM_EDEVICE;
        for (int g : stats_order) {
            const BuiltPlan::Group& G = bp.groups[g];
            if (launch_stats(bp.P, G.stats_begin, G.stats_end, s) != hipSuccess ||
                launch_stats_finalize(bp.P, G.mol_begin, G.mol_end, s) != hipSuccess ||
                hipEventRecord(ws.gev[g], s) != hipSuccess)
                return TCM_EDEVICE;
        }
        for (int k = 0; k < nl; ++k)
            for (auto it = lanes[k].rbegin(); it != lanes[k].rend(); ++it) {
                if (hipStreamWaitEvent(ws.aux[k], ws.gev[*it], 0) != hipSuccess) return TCM_EDEVICE;
                if (!group_tiles(*it, ws.aux[k])) return TCM_EDEVICE;
            }
        for (int k = 0; k < nl; ++k) {
            if (hipEventRecord(ws.join[k], ws.aux[k]) != hipSuccess) return TCM_EDEVICE;
            if (hipStreamWaitEvent(s, ws.join[k], 0) != hipSuccess) return TCM_EDEVICE;
        }
    } else {
        if (ev && hipEventRecord(ev[0], s) != hipSuccess) return TCM_EDEVICE;
        if (launch_stats(bp.P, 0, S, s) != hipSuccess) return TCM_EDEVICE;
        if (launch_stats_finalize(bp.P, 0, bp.P.nmol, s) != hipSuccess) return TCM_EDEVICE;
        if (ev && hipEventRecord(ev[1], s) != hipSuccess) return TCM_EDEVICE;
        for (int g = 0; g < ng; ++g)
            if (!group_tiles(g, s)) return TCM_EDEVICE;
    }
    if (ev && hipEventRecord(ev[2], s) != hipSuccess) return TCM_EDEVICE;
    if (launch_moments_finalize(bp.P, s) != hipSuccess) return TCM_EDEVICE;
    if (ev && hipEventRecord(ev[3], s) != hipSuccess) return TCM_EDEVICE;
    if (energy && launch_pairs(bp.P, 0, bp.npairs, s) != hipSuccess) return TCM_EDEVICE;
    if (ev && hipEventRecord(ev[4], s) != hipSuccess) return TCM_EDEVICE;
    return TCM_OK;
}

int check_err(Ctx* c, const BuiltPlan& bp, hipStream_t s)
{
    (void)c;
    int32_t err = 0;
    if (hipMemcpyAsync(&err, bp.P.err, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess) return TCM_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return TCM_EDEVICE;
    return err ? TCM_EDEVICE : TCM_OK;
}

// Device arrays of a finished plan read back through the context's pinned buffer, then the
// plan's error flag checked: into pinned memory the copies stay asynchronous and are waited on
// once (into pageable memory each copy is staged and waited on by itself).  dst[k] receives
// bytes[k] from src[k].  The context is locked; the pinned buffer is grown only after the
// stream has drained (an upload queued earlier may still read it).
static int read_back(Ctx& c, const BuiltPlan& bp, hipStream_t s, int n, const void* const* src, void* const* dst,
                     const size_t* bytes)
{
    size_t total = 64;
    for (int k = 0; k < n; ++k) total += (bytes[k] + 15) & ~size_t(15);
    if (total > c.hpin_cap && hipStreamSynchronize(s) != hipSuccess) return TCM_EDEVICE;
    int rc;
    if ((rc = c.ensure_pinned(total)) != TCM_OK) return rc;
    char* h = (char*)c.hpin;
    int32_t* herr = (int32_t*)h;
    size_t off = 64;
    for (int k = 0; k < n; ++k) {
        if (bytes[k] && hipMemcpyAsync(h + off, src[k], bytes[k], hipMemcpyDeviceToHost, s) != hipSuccess)
            return TCM_EDEVICE;
        off += (bytes[k] + 15) & ~size_t(15);
    }
    if (hipMemcpyAsync(herr, bp.P.err, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return TCM_EDEVICE;
    if (*herr) return TCM_EDEVICE;
    off = 64;
    for (int k = 0; k < n; ++k) {
        if (bytes[k]) std::memcpy(dst[k], h + off, bytes[k]);
        off += (bytes[k] + 15) & ~size_t(15);
    }
    return TCM_OK;
}

void free_workspace(Ctx* c, Workspace& ws)
{
    destroy_streams(ws);
    c->release(ws.blob); c->release(ws.sync); c->release(ws.part_f); c->release(ws.part_d);
    c->release(ws.stats); c->release(ws.r2); c->release(ws.outU); c->release(ws.outS);
    c->release(ws.prot); c->release(ws.pum);
    if (ws.staged) (void)hipEventSynchronize(ws.staged);
    if (ws.hstage) (void)hipHostFree(ws.hstage);
    ws.hstage = nullptr;
    ws.hstage_cap = 0;
    if (ws.staged) (void)hipEventDestroy(ws.staged);
    ws.staged = nullptr;
}

}  // namespace tcm

// ====================================================================== C ABI
using namespace tcm;

static bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

extern "C" const char* tcm_strerror(int st)
{
    switch (st) {
    case TCM_OK: return "ok";
    case TCM_EINVAL: return "invalid argument";
    case TCM_EDOMAIN: return "separation condition |R0| > a_A + a_B (eq. 2) violated";
    case TCM_ENOMEM: return "out of device memory or HBM budget";
    case TCM_EDEVICE: return "HIP device error";
    case TCM_EAGAIN: return "queue full, retry";
    case TCM_ENOTFOUND: return "unknown molecule id or ticket";
    default: return "unknown status";
    }
}

extern "C" int tcm_create(tcm_ctx** out, int device, size_t budget, int flags)
{
    (void)flags;
    if (!out) return TCM_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return TCM_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return TCM_EDEVICE;
    // the static scratch of tcm_moments_noalloc on this device (its address, looked up once)
    if (noalloc_init(device) != TCM_OK) return TCM_EDEVICE;
    tcm_ctx* t = new (std::nothrow) tcm_ctx();
    if (!t) return TCM_ENOMEM;
    Ctx& c = t->c;
    c.device = device;
    c.budget = budget;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c.num_cu = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&c.own_stream, hipStreamNonBlocking) != hipSuccess) {
        delete t;
        return TCM_EDEVICE;
    }
    c.stream = c.own_stream;
    {   // stream-ordered allocations return to a pool that keeps up to the budget's worth of
        // freed memory, so that freeing and re-allocating fragments costs no device sync
        hipMemPool_t pool;
        uint64_t keep = budget ? (uint64_t)budget : UINT64_MAX;
        if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess)
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        (void)hipGetLastError();
    }
    std::vector<double> invk, invf;
    build_norm_tables(LMAX, invk, invf);
    std::vector<double> rot = build_rotation_tables(LMAX);
    if (rot.size() != (size_t)rot_tables_len()) {   // the rotation matrices lost their sparsity pattern
        tcm_destroy(t);
        return TCM_EDEVICE;
    }
    // the row-by-row copy read by the pair launches
    rot.resize(2 * (size_t)rot_tables_len(), 0.0);
    for (int l = 0; l <= LMAX; ++l) {
        const int n = 2 * l + 1, K = l / 2 + 1;
        const double* src = rot.data() + rot_block_offset(l);
        double* dst = rot.data() + rot_tables_len() + rot_block_offset(l);
        for (int inv = 0; inv < 2; ++inv)
            for (int i = 0; i < n; ++i) {
                double* row = dst + (size_t)(inv * n + i) * (K + 1);
                row[0] = src[inv * n + i];
                for (int k = 0; k < K; ++k) row[1 + k] = src[2 * n + (size_t)inv * K * n + (size_t)k * n + i];
            }
    }
    std::vector<double> fact(FACT_N);        // k! (long double products, rounded once)
    {
        long double f = 1.0L;
        for (int k = 0; k < (int)fact.size(); ++k) {
            if (k > 0) f *= (long double)k;
            fact[k] = (double)f;
        }
    }
    int rc;
    if ((rc = c.alloc(c.t_invk, invk.size() * sizeof(double))) != TCM_OK ||
        (rc = c.alloc(c.t_invf, invf.size() * sizeof(double))) != TCM_OK ||
        (rc = c.alloc(c.t_rot, rot.size() * sizeof(double))) != TCM_OK ||
        (rc = c.alloc(c.t_fact, fact.size() * sizeof(double))) != TCM_OK) {
        tcm_destroy(t);
        return rc;
    }
    if (hipMemcpy(c.t_invk.p, invk.data(), invk.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.t_invf.p, invf.data(), invf.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.t_fact.p, fact.data(), fact.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.t_rot.p, rot.data(), rot.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        tcm_destroy(t);
        return TCM_EDEVICE;
    }
    const char* tf = std::getenv("TCM_AUTOTUNE_CACHE");
    if (tf) (void)tcm_tune_load(t, tf);
    *out = t;
    return TCM_OK;
}

extern "C" void tcm_destroy(tcm_ctx* t)
{
    if (!t) return;
    Ctx& c = t->c;
    (void)hipSetDevice(c.device);
    server_destroy(&c);
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    for (auto& kv : c.mols) {
        c.release(kv.second->atoms);
        c.release(kv.second->moments);
        c.release(kv.second->meta);
    }
    c.mols.clear();
    free_workspace(&c, c.ws);
    c.release(c.tmp_atoms);
    c.release(c.tmp_q);
    c.release(c.scan_g); c.release(c.scan_r); c.release(c.scan_u); c.release(c.scan_s);
    c.release(c.force_ft); c.release(c.force_w); c.release(c.force_t); c.release(c.force_a); c.release(c.force_b);
    c.release(c.adapt);
    c.release(c.gather);
    c.release(c.t_invk);
    c.release(c.t_invf);
    c.release(c.t_rot);
    c.release(c.t_fact);
    if (c.hpin) (void)hipHostFree(c.hpin);
    if (c.own_stream) (void)hipStreamDestroy(c.own_stream);
    delete t;
}

extern "C" int tcm_set_stream(tcm_ctx* t, void* s)
{
    if (!t) return TCM_EINVAL;
    std::lock_guard<std::mutex> g(t->c.mu);
    t->c.stream = s ? (hipStream_t)s : t->c.own_stream;
    return TCM_OK;
}

extern "C" void* tcm_get_stream(tcm_ctx* t) { return t ? (void*)t->c.stream : nullptr; }

extern "C" int tcm_mem_info(tcm_ctx* t, size_t* used, size_t* budget)
{
    if (!t) return TCM_EINVAL;
    if (used) *used = t->c.used.load();
    if (budget) *budget = t->c.budget;
    return TCM_OK;
}

extern "C" int tcm_set_budget(tcm_ctx* t, size_t budget)
{
    if (!t) return TCM_EINVAL;
    t->c.budget = budget;
    return TCM_OK;
}

// Upload host AoS atoms into tmp_atoms as SoA; returns device pointers.
static int upload_atoms(Ctx& c, DevBuf& dst, const double* coords, const double* charges, int64_t n,
                        const double* d[4], hipStream_t s)
{
    const size_t bytes = sizeof(double) * 4 * (size_t)(n > 0 ? n : 1);
    int rc;
    if ((rc = c.alloc(dst, bytes)) != TCM_OK) return rc;
    if ((rc = c.ensure_pinned(bytes)) != TCM_OK) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return TCM_EDEVICE;
    double* h = (double*)c.hpin;
    for (int64_t i = 0; i < n; ++i) {
        h[i] = coords[3 * i];
        h[n + i] = coords[3 * i + 1];
        h[2 * n + i] = coords[3 * i + 2];
        h[3 * n + i] = charges[i];
    }
    if (n > 0 && hipMemcpyAsync(dst.p, h, sizeof(double) * 4 * n, hipMemcpyHostToDevice, s) != hipSuccess)
        return TCM_EDEVICE;
    double* b = (double*)dst.p;
    d[0] = b; d[1] = b + n; d[2] = b + 2 * n; d[3] = b + 3 * n;
    return TCM_OK;
}

static int validate_atoms(const double* coords, const double* charges, int64_t n)
{
    if (n < 0 || (n > 0 && (!coords || !charges))) return TCM_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!finite3(coords + 3 * i) || !std::isfinite(charges[i])) return TCM_EINVAL;
    return TCM_OK;
}

extern "C" int tcm_moments(tcm_ctx* t, const double* coords, const double* charges, int64_t n, const double* centre,
                           int L, int prec, double* Q_out, double* radius_out, double* centre_out)
{
    if (!t || !Q_out || L < 0 || L > LMAX || (prec != TCM_F64 && prec != TCM_F32C)) return TCM_EINVAL;
    if (centre && !finite3(centre)) return TCM_EINVAL;
    int rc = validate_atoms(coords, charges, n);
    if (rc != TCM_OK) return rc;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    hipStream_t s = c.stream;
    const double* d[4];
    if ((rc = upload_atoms(c, c.tmp_atoms, coords, charges, n, d, s)) != TCM_OK) return rc;
    const size_t qbytes = sizeof(double) * (nh(L) + 8);
    if ((rc = c.alloc(c.tmp_q, qbytes)) != TCM_OK) return rc;
    MolJob j{};
    j.x = d[0]; j.y = d[1]; j.z = d[2]; j.q = d[3];
    j.n = n;
    j.L = L;
    j.prec = prec;
    j.has_centre = centre ? 1 : 0;
    if (centre) { j.centre[0] = centre[0]; j.centre[1] = centre[1]; j.centre[2] = centre[2]; }
    j.Q = (double*)c.tmp_q.p;
    j.meta = j.Q + nh(L);
    BuiltPlan bp;
    if ((rc = build_plan(&c, c.ws, {j}, {}, bp, s)) != TCM_OK) return rc;
    if ((rc = run_plan(&c, bp, s, false, nullptr)) != TCM_OK) return rc;
    std::vector<double> host(nh(L) + 5);
    if (hipMemcpyAsync(host.data(), j.Q, sizeof(double) * (nh(L) + 5), hipMemcpyDeviceToHost, s) != hipSuccess)
        return TCM_EDEVICE;
    if ((rc = check_err(&c, bp, s)) != TCM_OK) return rc;
    std::memcpy(Q_out, host.data(), sizeof(double) * nh(L));
    if (radius_out) *radius_out = host[nh(L) + 3];
    if (centre_out) { centre_out[0] = host[nh(L)]; centre_out[1] = host[nh(L) + 1]; centre_out[2] = host[nh(L) + 2]; }
    return TCM_OK;
}

extern "C" int tcm_pair_energy(tcm_ctx* t, const double* QA, double aA, const double* QB, double aB, const double* R,
                               const double* quat, int L, int flags, double* U_out)
{
    if (!t || !QA || !QB || !R || !U_out || L < 0 || L > LMAX) return TCM_EINVAL;
    if (!finite3(R)) return TCM_EINVAL;
    if (!(flags & TCM_UNCHECKED) && !(std::isfinite(aA) && std::isfinite(aB) && aA >= 0 && aB >= 0)) return TCM_EINVAL;
    if (quat) {
        const double qq = quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3];
        if (!std::isfinite(qq) || !(qq > 0)) return TCM_EINVAL;
    }
    const int NHl = nh(L);
    for (int i = 0; i < NHl; ++i)
        if (!std::isfinite(QA[i]) || !std::isfinite(QB[i])) return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    hipStream_t s = c.stream;
    int rc;
    const size_t cnt = 2 * (size_t)NHl + 16;
    if ((rc = c.alloc(c.tmp_q, sizeof(double) * cnt)) != TCM_OK) return rc;
    if ((rc = c.ensure_pinned(sizeof(double) * cnt)) != TCM_OK) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return TCM_EDEVICE;
    double* h = (double*)c.hpin;
    std::memcpy(h, QA, sizeof(double) * NHl);
    std::memcpy(h + NHl, QB, sizeof(double) * NHl);
    double* meta = h + 2 * NHl;
    for (int i = 0; i < 16; ++i) meta[i] = 0.0;
    meta[3] = (flags & TCM_UNCHECKED) ? 0.0 : aA;
    meta[8 + 3] = (flags & TCM_UNCHECKED) ? 0.0 : aB;
    if (hipMemcpyAsync(c.tmp_q.p, h, sizeof(double) * cnt, hipMemcpyHostToDevice, s) != hipSuccess) return TCM_EDEVICE;
    double* dq = (double*)c.tmp_q.p;
    PairJob pj{};
    pj.QA = dq;
    pj.QB = dq + NHl;
    pj.metaA = dq + 2 * NHl;
    pj.metaB = dq + 2 * NHl + 8;
    pj.depA = pj.depB = -1;
    pj.L = L;
    pj.flags = flags;
    for (int k = 0; k < 3; ++k) pj.R[k] = R[k];
    pj.quat[0] = 1.0;
    pj.has_rot = 0;
    if (quat) {
        for (int k = 0; k < 4; ++k) pj.quat[k] = quat[k];
        pj.has_rot = 1;
    }
    BuiltPlan bp;
    if ((rc = build_plan(&c, c.ws, {}, {pj}, bp, s)) != TCM_OK) return rc;
    if ((rc = run_plan(&c, bp, s, false, nullptr)) != TCM_OK) return rc;
    double U = 0.0;
    int32_t st = 0;
    {
        const void* src[2] = {bp.P.U, bp.P.status};
        void* dst[2] = {&U, &st};
        const size_t bytes[2] = {sizeof(double), sizeof(int32_t)};
        if ((rc = read_back(c, bp, s, 2, src, dst, bytes)) != TCM_OK) return rc;
    }
    if (st != TCM_OK) return st;
    *U_out = U;
    return TCM_OK;
}

// ---------------------------------------------------------------- resident molecules
// The molecule's record and its moment table at the largest order (8.7 KB) are allocated
// here, once, so that no computation on it allocates device memory.
static int add_mol(Ctx& c, std::unique_ptr<Mol> m, tcm_mol_id* id_out)
{
    int rc = c.alloc(m->meta, sizeof(double) * 8);
    if (rc == TCM_OK) rc = c.alloc(m->moments, sizeof(double) * nh(LMAX));
    if (rc != TCM_OK) {
        c.release(m->meta);
        c.release(m->atoms);
        return rc;
    }
    m->id = c.next_id++;
    *id_out = m->id;
    c.mols[m->id] = std::move(m);
    return TCM_OK;
}

extern "C" int tcm_mol_upload(tcm_ctx* t, const double* coords, const double* charges, int64_t n, const double* centre,
                              int prec, tcm_mol_id* id_out)
{
    if (!t || !id_out || (prec != TCM_F64 && prec != TCM_F32C)) return TCM_EINVAL;
    if (centre && !finite3(centre)) return TCM_EINVAL;
    int rc = validate_atoms(coords, charges, n);
    if (rc != TCM_OK) return rc;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    auto m = std::make_unique<Mol>();
    const double* d[4];
    if ((rc = upload_atoms(c, m->atoms, coords, charges, n, d, c.stream)) != TCM_OK) return rc;
    if (hipStreamSynchronize(c.stream) != hipSuccess) return TCM_EDEVICE;
    m->x = d[0]; m->y = d[1]; m->z = d[2]; m->q = d[3];
    m->n = n;
    m->prec = prec;
    m->has_centre = centre ? 1 : 0;
    if (centre) { m->centre[0] = centre[0]; m->centre[1] = centre[1]; m->centre[2] = centre[2]; }
    return add_mol(c, std::move(m), id_out);
}

extern "C" int tcm_mol_register_device(tcm_ctx* t, const double* dx, const double* dy, const double* dz,
                                       const double* dq, int64_t n, const double* centre, int prec, tcm_mol_id* id_out)
{
    if (!t || !id_out || n < 0 || (n > 0 && (!dx || !dy || !dz || !dq)) || (prec != TCM_F64 && prec != TCM_F32C))
        return TCM_EINVAL;
    if (centre && !finite3(centre)) return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    auto m = std::make_unique<Mol>();
    m->x = dx; m->y = dy; m->z = dz; m->q = dq;
    m->n = n;
    m->prec = prec;
    m->has_centre = centre ? 1 : 0;
    if (centre) { m->centre[0] = centre[0]; m->centre[1] = centre[1]; m->centre[2] = centre[2]; }
    return add_mol(c, std::move(m), id_out);
}

extern "C" int tcm_mol_release(tcm_ctx* t, tcm_mol_id id)
{
    if (!t) return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.mols.find(id);
    if (it == c.mols.end()) return TCM_ENOTFOUND;
    if (it->second->plan_refs > 0) return TCM_EAGAIN;      // a live plan still reads or writes it
    (void)hipStreamSynchronize(c.stream);
    c.release(it->second->atoms);
    c.release(it->second->moments);
    c.release(it->second->meta);
    c.mols.erase(it);
    return TCM_OK;
}

namespace tcm {
// Molecule jobs and pair jobs of a batch of resident-molecule requests.  A molecule named
// by several requests is computed once, at the largest order any of them needs (its
// resident table keeps the larger order if it already had one); requests flagged
// TCM_REUSE read resident moments of sufficient order without recomputing them.
struct ReqPlan {
    std::vector<MolJob> mj;
    std::vector<PairJob> pj;
    std::vector<int> pj_req;                 // request index of each pair job
    std::vector<std::pair<Mol*, int>> computed;
    std::vector<int32_t> pre_status;         // per request: TCM_OK or a host-side error
    std::vector<Mol*> side;                  // per request: its two molecules (null on error)
};

int plan_requests(Ctx& c, const tcm_pair_req* reqs, int64_t np, bool allow_reuse, ReqPlan& rp)
{
    // one pass over the requests: each molecule's required order kept in its planning scratch
    // (touched lists the molecules in first-use order; ordered by id below)
    std::vector<Mol*> touched;
    std::vector<Mol*>& side = rp.side;
    side.assign((size_t)2 * np, nullptr);
    rp.pre_status.assign(np, TCM_OK);
    for (int64_t i = 0; i < np; ++i) {
        const tcm_pair_req& r = reqs[i];
        const double qq = r.quat_b[0] * r.quat_b[0] + r.quat_b[1] * r.quat_b[1] +
                          r.quat_b[2] * r.quat_b[2] + r.quat_b[3] * r.quat_b[3];
        if (r.L < 0 || r.L > LMAX || !finite3(r.R) || !std::isfinite(qq) || !(qq > 0)) {
            rp.pre_status[i] = TCM_EINVAL;
            continue;
        }
        auto ia = c.mols.find(r.a), ib = c.mols.find(r.b);
        if (ia == c.mols.end() || ib == c.mols.end()) {
            rp.pre_status[i] = TCM_ENOTFOUND;
            continue;
        }
        side[2 * i] = ia->second.get();
        side[2 * i + 1] = ib->second.get();
        for (Mol* m : {side[2 * i], side[2 * i + 1]}) {
            const bool reuse = allow_reuse && (r.flags & TCM_REUSE) && m->Lcached >= r.L;
            const int want = reuse ? -1 : r.L;
            if (m->plan_want == INT32_MIN) {
                touched.push_back(m);
                m->plan_want = want;
            } else if (want > m->plan_want) {
                m->plan_want = want;
            }
        }
    }
    std::sort(touched.begin(), touched.end(), [](const Mol* u, const Mol* v) { return u->id < v->id; });
    int rc = TCM_OK;
    for (Mol* m : touched) {
        if (m->plan_want < 0) continue;
        int L = m->plan_want;
        if (m->Lcached > L) L = m->Lcached;
        if (m->moments.cap < sizeof(double) * nh(L) && (rc = c.alloc(m->moments, sizeof(double) * nh(L))) != TCM_OK)
            break;
        MolJob j{};
        j.x = m->x; j.y = m->y; j.z = m->z; j.q = m->q;
        j.n = m->n;
        j.L = L;
        j.prec = m->prec;
        j.has_centre = m->has_centre;
        for (int d = 0; d < 3; ++d) j.centre[d] = m->centre[d];
        j.Q = (double*)m->moments.p;
        j.meta = (double*)m->meta.p;
        m->plan_job = (int)rp.mj.size();
        rp.mj.push_back(j);
        rp.computed.push_back({m, L});
        m->Lcached = -1;                      // invalid until this run completes
        m->radius_host = -1.0;
    }
    if (rc == TCM_OK) {
        rp.pj.reserve(np);
        rp.pj_req.reserve(np);
        for (int64_t i = 0; i < np; ++i) {
            if (rp.pre_status[i] != TCM_OK) continue;
            const tcm_pair_req& r = reqs[i];
            Mol* a = side[2 * i];
            Mol* b = side[2 * i + 1];
            PairJob j{};
            j.QA = (const double*)a->moments.p;
            j.QB = (const double*)b->moments.p;
            j.metaA = (const double*)a->meta.p;
            j.metaB = (const double*)b->meta.p;
            j.depA = a->plan_job;
            j.depB = b->plan_job;
            j.L = r.L;
            j.flags = r.flags;
            for (int d = 0; d < 3; ++d) j.R[d] = r.R[d];
            for (int d = 0; d < 4; ++d) j.quat[d] = r.quat_b[d];
            j.has_rot = !(r.quat_b[0] > 0 && r.quat_b[1] == 0 && r.quat_b[2] == 0 && r.quat_b[3] == 0);
            rp.pj.push_back(j);
            rp.pj_req.push_back((int)i);
            a->last_use = b->last_use = ++c.use_clock;
        }
    }
    for (Mol* m : touched) {
        m->plan_want = INT32_MIN;
        m->plan_job = -1;
    }
    return rc;
}

void mark_computed(ReqPlan& rp)
{
    for (auto& pr : rp.computed) {
        pr.first->Lcached = pr.second;
        pr.first->radius_host = -1.0;
    }
}
}  // namespace tcm

extern "C" int tcm_mol_moments(tcm_ctx* t, tcm_mol_id id, int L, int flags, double* Q_out, double* radius_out,
                               double* centre_out)
{
    if (!t || !Q_out || L < 0 || L > LMAX) return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    auto it = c.mols.find(id);
    if (it == c.mols.end()) return TCM_ENOTFOUND;
    Mol* m = it->second.get();
    hipStream_t s = c.stream;
    int rc;
    if (!((flags & TCM_REUSE) && m->Lcached >= L)) {
        int Lc = m->Lcached > L ? m->Lcached : L;
        if (m->moments.cap < sizeof(double) * nh(Lc) && (rc = c.alloc(m->moments, sizeof(double) * nh(Lc))) != TCM_OK)
            return rc;
        MolJob j{};
        j.x = m->x; j.y = m->y; j.z = m->z; j.q = m->q;
        j.n = m->n;
        j.L = Lc;
        j.prec = m->prec;
        j.has_centre = m->has_centre;
        for (int d = 0; d < 3; ++d) j.centre[d] = m->centre[d];
        j.Q = (double*)m->moments.p;
        j.meta = (double*)m->meta.p;
        m->Lcached = -1;
        m->radius_host = -1.0;
        BuiltPlan bp;
        if ((rc = build_plan(&c, c.ws, {j}, {}, bp, s)) != TCM_OK) return rc;
        if ((rc = run_plan(&c, bp, s, false, nullptr)) != TCM_OK) return rc;
        if ((rc = check_err(&c, bp, s)) != TCM_OK) return rc;
        m->Lcached = Lc;
    }
    std::vector<double> meta(5);
    if (hipMemcpyAsync(Q_out, m->moments.p, sizeof(double) * nh(L), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(meta.data(), m->meta.p, sizeof(double) * 5, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return TCM_EDEVICE;
    if (radius_out) *radius_out = meta[3];
    if (centre_out) { centre_out[0] = meta[0]; centre_out[1] = meta[1]; centre_out[2] = meta[2]; }
    m->last_use = ++c.use_clock;
    return TCM_OK;
}

static int first_error(const int32_t* st, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (st[i] != TCM_OK) return st[i];
    return TCM_OK;
}

// The batch path with the context locked and current.
// Run planned requests (moment jobs and pair jobs) and scatter the results to request order.
static int run_requests(Ctx& c, ReqPlan& rp, int64_t np, double* U_out, int32_t* status_out)
{
    hipStream_t s = c.stream;
    int rc;
    BuiltPlan bp;
    if ((rc = build_plan(&c, c.ws, rp.mj, rp.pj, bp, s)) != TCM_OK) return rc;
    if ((rc = run_plan(&c, bp, s, false, nullptr)) != TCM_OK) return rc;
    const int npj = (int)rp.pj.size();
    std::vector<double> U(npj > 0 ? npj : 1);
    std::vector<int32_t> st(npj > 0 ? npj : 1);
    {
        const void* src[2] = {bp.P.U, bp.P.status};
        void* dst[2] = {U.data(), st.data()};
        const size_t bytes[2] = {sizeof(double) * (size_t)npj, sizeof(int32_t) * (size_t)npj};
        if ((rc = read_back(c, bp, s, 2, src, dst, bytes)) != TCM_OK) return rc;
    }
    mark_computed(rp);
    for (int64_t i = 0; i < np; ++i) {
        status_out[i] = rp.pre_status[i];
        U_out[i] = std::nan("");
    }
    for (int k = 0; k < npj; ++k) {
        status_out[rp.pj_req[k]] = st[k];
        U_out[rp.pj_req[k]] = st[k] == TCM_OK ? U[k] : std::nan("");
    }
    return first_error(status_out, np);
}

static int batch_energy_locked(Ctx& c, const tcm_pair_req* reqs, int64_t np, double* U_out, int32_t* status_out)
{
    ReqPlan rp;
    int rc = plan_requests(c, reqs, np, true, rp);
    if (rc != TCM_OK) return rc;
    return run_requests(c, rp, np, U_out, status_out);
}

extern "C" int tcm_batch_energy(tcm_ctx* t, const tcm_pair_req* reqs, int64_t np, double* U_out, int32_t* status_out)
{
    if (!t || np < 0 || (np > 0 && (!reqs || !U_out || !status_out))) return TCM_EINVAL;
    if (np > (1 << 26)) return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    return batch_energy_locked(c, reqs, np, U_out, status_out);
}

// Every pair of K resident fragments at their own positions: the moments of each fragment
// once (order L), the centres read back, then one batch of K(K-1)/2 contractions with
// R = c_j - c_i.
extern "C" int tcm_all_pairs(tcm_ctx* t, const tcm_mol_id* ids, int64_t K, int L, int flags, double* U_out,
                             int32_t* status_out)
{
    if (!t || K < 0 || (K > 0 && !ids) || L < 0 || L > LMAX) return TCM_EINVAL;
    const int64_t np = K * (K - 1) / 2;
    if (K > 11585 || (np > 0 && (!U_out || !status_out))) return TCM_EINVAL;   // np <= 2^26
    if (np == 0) return TCM_OK;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    hipStream_t s = c.stream;
    for (int64_t i = 0; i < K; ++i)
        if (c.mols.find(ids[i]) == c.mols.end()) return TCM_ENOTFOUND;
    // moments (and centres) of every fragment: one request per fragment, paired with itself
    std::vector<tcm_pair_req> one((size_t)K);
    for (int64_t i = 0; i < K; ++i) {
        one[i] = tcm_pair_req{};
        one[i].a = one[i].b = ids[i];
        one[i].R[0] = 1.0;
        one[i].quat_b[0] = 1.0;
        one[i].L = L;
        one[i].flags = flags & TCM_REUSE;
    }
    ReqPlan rp;
    int rc = plan_requests(c, one.data(), K, (flags & TCM_REUSE) != 0, rp);
    if (rc != TCM_OK) return rc;
    if ((rc = first_error(rp.pre_status.data(), K)) != TCM_OK) return rc;
    if (!rp.mj.empty()) {
        BuiltPlan bp;
        if ((rc = build_plan(&c, c.ws, rp.mj, {}, bp, s)) != TCM_OK) return rc;
        if ((rc = run_plan(&c, bp, s, false, nullptr)) != TCM_OK) return rc;
        if ((rc = check_err(&c, bp, s)) != TCM_OK) return rc;
        mark_computed(rp);
    }
    // the K centre records gathered on the device and read back in one copy
    std::vector<double> meta((size_t)K * 8);
    std::vector<const double*> src((size_t)K);
    for (int64_t i = 0; i < K; ++i) src[i] = (const double*)c.mols[ids[i]]->meta.p;
    const size_t pbytes = align_up(sizeof(double*) * (size_t)K, 256);
    if ((rc = c.alloc(c.gather, pbytes + sizeof(double) * 8 * (size_t)K)) != TCM_OK) return rc;
    const double* const* dsrc = (const double* const*)c.gather.p;
    double* dmeta = (double*)((char*)c.gather.p + pbytes);
    if (hipMemcpyAsync((void*)dsrc, src.data(), sizeof(double*) * (size_t)K, hipMemcpyHostToDevice, s) != hipSuccess ||
        launch_gather8(dsrc, K, dmeta, s) != hipSuccess ||
        hipMemcpyAsync(meta.data(), dmeta, sizeof(double) * 8 * (size_t)K, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return TCM_EDEVICE;
    std::vector<tcm_pair_req> reqs((size_t)np);
    int64_t k = 0;
    for (int64_t i = 0; i < K; ++i)
        for (int64_t j = i + 1; j < K; ++j, ++k) {
            tcm_pair_req& r = reqs[(size_t)k];
            r = tcm_pair_req{};
            r.a = ids[i];
            r.b = ids[j];
            for (int d = 0; d < 3; ++d) r.R[d] = meta[(size_t)j * 8 + d] - meta[(size_t)i * 8 + d];
            r.quat_b[0] = 1.0;
            r.L = L;
            r.flags = (flags & (TCM_UNCHECKED | TCM_TRIANGULAR)) | TCM_REUSE;
        }
    return batch_energy_locked(c, reqs.data(), np, U_out, status_out);
}

// ---------------------------------------------------------------- plans (graph replay)
static int abs_sums(Ctx& c, const ReqPlan& rp, hipStream_t s);

// One run of a plan on s: the moment pass, then the contraction (adaptive plans: the order
// choice, the regrouping and the contraction at the chosen orders).  ev (may be null): the
// phase events of run_plan, the last one recorded after the contraction.
static int plan_issue(Ctx& c, tcm_plan* pl, hipStream_t s, bool serial, hipEvent_t* ev)
{
    int rc = run_plan(&c, pl->bp, s, serial, ev, !pl->adaptive);
    if (rc == TCM_OK && pl->adaptive) {
        rc = adapt_launch(pl->bp, pl->ab, pl->tol, s);
        if (rc == TCM_OK && ev && hipEventRecord(ev[4], s) != hipSuccess) rc = TCM_EDEVICE;
    }
    return rc;
}

static int plan_create(tcm_ctx* t, const tcm_pair_req* reqs, int64_t np, int use_graph, bool adaptive, double tol,
                       tcm_plan** out)
{
    if (!t || !out || np < 0 || (np > 0 && !reqs)) return TCM_EINVAL;
    if (adaptive && !(tol > 0.0)) return TCM_EINVAL;
    *out = nullptr;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    hipStream_t s = c.stream;
    ReqPlan rp;
    int rc = plan_requests(c, reqs, np, false, rp);
    if (rc != TCM_OK) return rc;
    if (first_error(rp.pre_status.data(), np) != TCM_OK) return first_error(rp.pre_status.data(), np);
    tcm_plan* pl = new (std::nothrow) tcm_plan();
    if (!pl) return TCM_ENOMEM;
    pl->ctx = &c;
    pl->adaptive = adaptive;
    pl->tol = tol;
    if ((rc = build_plan(&c, pl->ws, rp.mj, rp.pj, pl->bp, s)) != TCM_OK ||
        (adaptive && ((rc = adapt_setup(c, pl->adapt, pl->bp, pl->ab)) != TCM_OK ||
                      (rc = abs_sums(c, rp, s)) != TCM_OK))) {
        c.release(pl->adapt);
        free_workspace(&c, pl->ws);
        delete pl;
        return rc;
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
        c.release(pl->adapt);
        free_workspace(&c, pl->ws);
        delete pl;
        return TCM_EDEVICE;
    }
    // the moments become valid when a run is issued (tcm_plan_run marks them then); until the
    // plan is destroyed its molecules are pinned, so the buffers its launches address stay
    pl->computed = rp.computed;
    for (size_t k = 0; k < rp.side.size(); ++k) {
        Mol* m = rp.side[k];
        if (m && std::find(pl->refs.begin(), pl->refs.end(), m) == pl->refs.end()) pl->refs.push_back(m);
    }
    for (Mol* m : pl->refs) ++m->plan_refs;
    pl->npairs = (int)np;
    if (use_graph) {
        hipStream_t cs = nullptr;
        bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            // the serial order: the graph runtime replays a captured fork/join one node at a
            // time anyway, and serially the statistics are a single launch over the batch
            int r2 = plan_issue(c, pl, cs, true, nullptr);
            hipGraph_t gr = nullptr;
            ok = hipStreamEndCapture(cs, &gr) == hipSuccess && r2 == TCM_OK;
            if (ok) {
                pl->graph = gr;
                ok = hipGraphInstantiate(&pl->exec, gr, nullptr, nullptr, 0) == hipSuccess;
            } else if (gr) {
                (void)hipGraphDestroy(gr);
            }
        }
        if (cs) (void)hipStreamDestroy(cs);
        if (!ok) {
            (void)hipGetLastError();
            for (Mol* m : pl->refs) --m->plan_refs;      // the context lock is held here
            pl->refs.clear();
            pl->ctx = nullptr;
            if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
            if (pl->graph) (void)hipGraphDestroy(pl->graph);
            c.release(pl->adapt);
            free_workspace(&c, pl->ws);
            delete pl;
            return TCM_EDEVICE;
        }
    }
    *out = pl;
    return TCM_OK;
}

extern "C" int tcm_plan_create(tcm_ctx* t, const tcm_pair_req* reqs, int64_t np, int use_graph, tcm_plan** out)
{
    return plan_create(t, reqs, np, use_graph, false, 0.0, out);
}

extern "C" int tcm_plan_create_adaptive(tcm_ctx* t, const tcm_pair_req* reqs, int64_t np, double tol, int use_graph,
                                        tcm_plan** out)
{
    return plan_create(t, reqs, np, use_graph, true, tol, out);
}

// A run issued on the context's stream: the moments it writes count as resident from here on
// (later work on that stream is ordered behind it), at exactly the plan's order.
static void plan_issued(Ctx& c, tcm_plan* pl)
{
    std::lock_guard<std::mutex> g(c.mu);
    for (auto& pr : pl->computed) {
        pr.first->Lcached = pr.second;
        pr.first->radius_host = -1.0;
    }
}

extern "C" int tcm_plan_run(tcm_ctx* t, tcm_plan* pl)
{
    if (!t || !pl || pl->ctx != &t->c) return TCM_EINVAL;
    Ctx& c = t->c;
    (void)hipSetDevice(c.device);
    int rc;
    if (pl->exec) rc = hipGraphLaunch(pl->exec, c.stream) == hipSuccess ? TCM_OK : TCM_EDEVICE;
    else rc = plan_issue(c, pl, c.stream, false, nullptr);
    if (rc == TCM_OK) plan_issued(c, pl);
    return rc;
}

extern "C" int tcm_plan_run_phased(tcm_ctx* t, tcm_plan* pl)
{
    if (!t || !pl || pl->ctx != &t->c) return TCM_EINVAL;
    (void)hipSetDevice(t->c.device);
    const int rc = plan_issue(t->c, pl, t->c.stream, true, nullptr);
    if (rc == TCM_OK) plan_issued(t->c, pl);
    return rc;
}

extern "C" int tcm_plan_run_timed(tcm_ctx* t, tcm_plan* pl, double* ms_out)
{
    if (!t || !pl || !ms_out || pl->ctx != &t->c) return TCM_EINVAL;
    Ctx& c = t->c;
    (void)hipSetDevice(c.device);
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int rc = TCM_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) rc = TCM_EDEVICE;
    if (rc == TCM_OK) rc = plan_issue(c, pl, c.stream, true, ev);
    if (rc == TCM_OK) plan_issued(c, pl);
    if (rc == TCM_OK && hipEventSynchronize(ev[4]) != hipSuccess) rc = TCM_EDEVICE;
    for (int k = 0; rc == TCM_OK && k < 4; ++k) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
        ms_out[k] = ms;
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

extern "C" int tcm_plan_results(tcm_ctx* t, tcm_plan* pl, double* U_out, int32_t* status_out)
{
    if (!t || !pl) return TCM_EINVAL;
    Ctx& c = t->c;
    hipStream_t s = c.stream;
    const int n = pl->bp.npairs;
    if (U_out && n && hipMemcpyAsync(U_out, pl->bp.P.U, sizeof(double) * n, hipMemcpyDeviceToHost, s) != hipSuccess)
        return TCM_EDEVICE;
    if (status_out && n &&
        hipMemcpyAsync(status_out, pl->bp.P.status, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s) != hipSuccess)
        return TCM_EDEVICE;
    return check_err(&c, pl->bp, s);
}

extern "C" int tcm_plan_orders(tcm_ctx* t, tcm_plan* pl, int32_t* L_out, double* bound_out)
{
    if (!t || !pl || pl->ctx != &t->c || !pl->adaptive) return TCM_EINVAL;
    Ctx& c = t->c;
    hipStream_t s = c.stream;
    const int n = pl->bp.npairs;
    if (L_out && n && hipMemcpyAsync(L_out, pl->ab.L, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s) != hipSuccess)
        return TCM_EDEVICE;
    if (bound_out && n &&
        hipMemcpyAsync(bound_out, pl->ab.bound, sizeof(double) * n, hipMemcpyDeviceToHost, s) != hipSuccess)
        return TCM_EDEVICE;
    return check_err(&c, pl->bp, s);
}

extern "C" int tcm_plan_device_outputs(tcm_plan* pl, double** dU, int32_t** dS)
{
    if (!pl) return TCM_EINVAL;
    if (dU) *dU = pl->bp.P.U;
    if (dS) *dS = pl->bp.P.status;
    return TCM_OK;
}

extern "C" int tcm_plan_info(tcm_plan* pl, int64_t* atoms, double* flops, int64_t* tiles, int64_t* pairs)
{
    if (!pl) return TCM_EINVAL;
    if (atoms) *atoms = pl->bp.atoms;
    if (flops) *flops = pl->bp.moment_flops;
    if (tiles) *tiles = pl->bp.n_tiles;
    if (pairs) *pairs = pl->bp.npairs;
    return TCM_OK;
}

extern "C" void tcm_plan_destroy(tcm_plan* pl)
{
    if (!pl) return;
    if (pl->ctx) {                           // its launches may still run: let them finish
        std::lock_guard<std::mutex> g(pl->ctx->mu);
        (void)hipStreamSynchronize(pl->ctx->stream);
        for (Mol* m : pl->refs) --m->plan_refs;
    }
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    // the plan's buffers were charged to the context that created it (plans are destroyed
    // before their context): return them to its budget
    if (pl->ctx) pl->ctx->release(pl->adapt);
    free_workspace(pl->ctx, pl->ws);
    delete pl;
}

// ---------------------------------------------------------------- tuning
extern "C" int tcm_tune_get(tcm_ctx* t, int prec, int L, int64_t n, int* k)
{
    if (!t || !k || L < 0 || L > LMAX || n < 0) return TCM_EINVAL;
    std::lock_guard<std::mutex> g(t->c.mu);
    *k = t->c.kper_for(prec, L, n);
    return TCM_OK;
}

extern "C" int tcm_tune_set(tcm_ctx* t, int prec, int L, int64_t n, int k)
{
    if (!t || L < 0 || L > LMAX || n < 0 || k < 1 || k > 1024) return TCM_EINVAL;
    std::lock_guard<std::mutex> g(t->c.mu);
    if (t->c.server) return TCM_EAGAIN;      // tilings are fixed while a server runs
    t->c.tune[tune_key(prec, L, n)] = k;
    return TCM_OK;
}

extern "C" int tcm_set_fp32_run(tcm_ctx* t, int kmax)
{
    if (!t || kmax < 1 || kmax > 1024) return TCM_EINVAL;
    std::lock_guard<std::mutex> g(t->c.mu);
    if (t->c.server) return TCM_EAGAIN;
    t->c.f32_run_max = kmax;
    return TCM_OK;
}

extern "C" int tcm_tune_save(tcm_ctx* t, const char* path)
{
    if (!t || !path) return TCM_EINVAL;
    std::lock_guard<std::mutex> g(t->c.mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return TCM_EINVAL;
    std::fprintf(f, "# tcm tuning table: key kper (key = prec*100000 + L*100 + log2 bucket)\n");
    for (auto& kv : t->c.tune) std::fprintf(f, "%lld %d\n", (long long)kv.first, kv.second);
    std::fclose(f);
    return TCM_OK;
}

extern "C" int tcm_tune_load(tcm_ctx* t, const char* path)
{
    if (!t || !path) return TCM_EINVAL;
    FILE* f = std::fopen(path, "r");
    if (!f) return TCM_ENOTFOUND;
    std::lock_guard<std::mutex> g(t->c.mu);
    if (t->c.server) {
        std::fclose(f);
        return TCM_EAGAIN;                   // tilings are fixed while a server runs
    }
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        long long key;
        int k;
        if (std::sscanf(line, "%lld %d", &key, &k) == 2 && k >= 1 && k <= 1024) t->c.tune[key] = k;
    }
    std::fclose(f);
    return TCM_OK;
}

// Times each candidate kper for (precision, L, n's size bucket) with HIP events around the
// tile launches of a synthetic batch: copies of one molecule of n atoms (points in a ball,
// charges in [-1, 1]), enough copies to fill the device, so the measurement reflects batched
// throughput rather than launch latency.
// ---------------------------------------------------------------- translation scan
extern "C" int tcm_scan_translations(tcm_ctx* t, tcm_mol_id a, tcm_mol_id b, int L, const double* quat_b, int flags,
                                     const double* R, int64_t nR, double* U_out, int32_t* status_out)
{
    if (!t || L < 0 || L > LMAX || nR < 0 || (nR > 0 && (!R || !U_out || !status_out))) return TCM_EINVAL;
    if (nR > (int64_t(1) << 31)) return TCM_EINVAL;
    if (quat_b) {
        const double qq = quat_b[0] * quat_b[0] + quat_b[1] * quat_b[1] + quat_b[2] * quat_b[2] + quat_b[3] * quat_b[3];
        if (!std::isfinite(qq) || !(qq > 0)) return TCM_EINVAL;
    }
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    hipStream_t s = c.stream;
    const bool dev = (flags & TCM_DEVICE_IO) != 0;
    // moments of A and B at order L (a one-pair request, R and pose unused here)
    tcm_pair_req req{};
    req.a = a;
    req.b = b;
    req.R[0] = 1.0;
    req.quat_b[0] = 1.0;
    req.L = L;
    req.flags = flags & TCM_REUSE;
    ReqPlan rp;
    int rc = plan_requests(c, &req, 1, (flags & TCM_REUSE) != 0, rp);
    if (rc != TCM_OK) return rc;
    if (rp.pre_status[0] != TCM_OK) return rp.pre_status[0];
    if (!rp.mj.empty()) {
        BuiltPlan bp;
        if ((rc = build_plan(&c, c.ws, rp.mj, {}, bp, s)) != TCM_OK) return rc;
        if ((rc = run_plan(&c, bp, s, true, nullptr)) != TCM_OK) return rc;
        if ((rc = check_err(&c, bp, s)) != TCM_OK) return rc;
        mark_computed(rp);
    }
    Mol* ma = c.mols[a].get();
    Mol* mb = c.mols[b].get();
    if (ma->radius_host < 0.0 || mb->radius_host < 0.0) {   // radii of eq. 2, read once per computation
        double meta[2][8];
        if (hipMemcpyAsync(meta[0], ma->meta.p, sizeof(double) * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(meta[1], mb->meta.p, sizeof(double) * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return TCM_EDEVICE;
        ma->radius_host = meta[0][3];
        mb->radius_host = meta[1][3];
    }
    const double aA = ma->radius_host, aB = mb->radius_host;
    const double rho = aA + aB > 0.0 ? aA + aB : 1.0;
    const bool tri = (flags & TCM_TRIANGULAR) != 0;
    const int64_t Lt = tri ? L : 2 * (int64_t)L;                 // largest total order L' = l1 + l2
    const int64_t NG = (Lt + 1) * (Lt + 2) / 2;
    if ((rc = c.alloc(c.scan_g, sizeof(double) * 4 * NG)) != TCM_OK) return rc;   // table rows of 4 doubles
    const double* dR = R;
    double* dU = U_out;
    int32_t* dS = status_out;
    if (!dev && nR > 0) {
        if ((rc = c.alloc(c.scan_r, sizeof(double) * 3 * nR)) != TCM_OK ||
            (rc = c.alloc(c.scan_u, sizeof(double) * nR)) != TCM_OK ||
            (rc = c.alloc(c.scan_s, sizeof(int32_t) * nR)) != TCM_OK)
            return rc;
        if (hipMemcpyAsync(c.scan_r.p, R, sizeof(double) * 3 * nR, hipMemcpyHostToDevice, s) != hipSuccess)
            return TCM_EDEVICE;
        dR = (const double*)c.scan_r.p;
        dU = (double*)c.scan_u.p;
        dS = (int32_t*)c.scan_s.p;
    }
    if (launch_scan((const double*)ma->moments.p, (const double*)mb->moments.p, L, tri ? 1 : 0, rho, aA, aB,
                    (flags & TCM_UNCHECKED) ? 1 : 0, (const double*)c.t_invf.p, (const double*)c.t_rot.p, quat_b,
                    (double*)c.scan_g.p, dR, nR, dU, dS, s) != hipSuccess)
        return TCM_EDEVICE;
    if (dev || nR == 0) return TCM_OK;
    if (hipMemcpyAsync(U_out, dU, sizeof(double) * nR, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(status_out, dS, sizeof(int32_t) * nR, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return TCM_EDEVICE;
    return TCM_OK;
}

// ---------------------------------------------------------------- ALU calibration
extern "C" int tcm_alu_calibrate(tcm_ctx* t, int precision, double* tflops_out)
{
    if (!t || !tflops_out || (precision != TCM_F64 && precision != TCM_F32C)) return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    hipStream_t s = c.stream;
    const int blocks = 32 * c.num_cu, iters = 4096, reps = 5;
    DevBuf buf;
    int rc = c.alloc(buf, sizeof(double) * (size_t)blocks * WG);
    if (rc != TCM_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.0f;
    rc = TCM_EDEVICE;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
        launch_alu_probe(precision, buf.p, blocks, iters, s) == hipSuccess && hipEventRecord(e0, s) == hipSuccess) {
        bool ok = true;
        for (int r = 0; r < reps && ok; ++r) ok = launch_alu_probe(precision, buf.p, blocks, iters, s) == hipSuccess;
        if (ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f) {
            const double flops = (double)reps * blocks * WG * 16.0 * iters * 2.0;
            *tflops_out = flops / (ms * 1e-3) / 1e12;
            rc = TCM_OK;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c.release(buf);
    return rc;
}

// ---------------------------------------------------------------- adaptive truncation
// Bound on |U_coulomb - U_L| for the square truncation: with alpha = a_A/R, beta = a_B/R and
// S = sum |q|, the (l1, l2) term of the double Taylor series of 1/|R + r_B - r_A| is at most
// C(l1+l2, l1) a_A^l1 a_B^l2 / R^{l1+l2+1}, and summing the terms outside the square gives
// S_A S_B / (R (1 - alpha - beta)) [(alpha/(1-beta))^{L+1} + (beta/(1-alpha))^{L+1}]
// (infinite when alpha + beta >= 1).

namespace tcm {

int adapt_setup(Ctx& c, DevBuf& buf, const BuiltPlan& bp, AdaptBufs& ab)
{
    const int npj = bp.npairs;
    const size_t np1 = npj > 0 ? (size_t)npj : 1, ngr = (np1 + PAIR_LANES - 1) / PAIR_LANES;
    const size_t o_L = align_up(sizeof(double) * np1, 256);
    const size_t o_pw = align_up(o_L + sizeof(int32_t) * np1, 256);
    const size_t o_fr = align_up(o_pw + sizeof(PairWork) * np1, 256);
    const size_t o_go = align_up(o_fr + sizeof(double) * 2 * FRAME_N * np1, 256);
    const size_t o_cn = align_up(o_go + sizeof(int32_t) * ngr, 256);
    int rc;
    if ((rc = c.alloc(buf, o_cn + sizeof(int32_t) * 2 * (LMAX + 1))) != TCM_OK) return rc;
    char* ad = (char*)buf.p;
    ab.bound = (double*)ad;
    ab.L = (int32_t*)(ad + o_L);
    ab.cnt = (int32_t*)(ad + o_cn);
    ab.P2 = bp.P;                                        // the contraction over the regrouped listing
    ab.P2.pairs = (const PairWork*)(ad + o_pw);
    ab.P2.frame = (const double*)(ad + o_fr);
    ab.P2.gorder = (int32_t*)(ad + o_go);
    ab.P2.gorder_uniform = 0;                            // the orders are chosen on the device
    ab.npj = npj;
    return TCM_OK;
}

int adapt_launch(const BuiltPlan& bp, const AdaptBufs& ab, double tol, hipStream_t s)
{
    if (launch_pairs_choose(bp.P, 0, ab.npj, tol, ab.L, ab.bound, s) != hipSuccess ||
        launch_pairs_regroup(bp.P, ab.npj, ab.L, ab.cnt, const_cast<PairWork*>(ab.P2.pairs),
                             const_cast<double*>(ab.P2.frame), ab.P2.gorder, s) != hipSuccess ||
        launch_pairs(ab.P2, 0, ab.npj, s) != hipSuccess)
        return TCM_EDEVICE;
    return TCM_OK;
}

}  // namespace tcm

// sum |q| (meta[5], the bound's charge scale) of the planned molecules that lack it, once per
// molecule, ordered on s
static int abs_sums(Ctx& c, const ReqPlan& rp, hipStream_t s)
{
    (void)c;
    std::vector<Mol*> need;
    for (size_t k = 0; k < rp.side.size(); ++k) {
        Mol* m = rp.side[k];
        if (m && !m->absq_dev) {
            m->absq_dev = true;
            need.push_back(m);
        }
    }
    for (Mol* m : need)
        if (launch_abs_sum(m->q, m->n, (double*)m->meta.p + 5, s) != hipSuccess) {
            for (Mol* x : need) x->absq_dev = false;
            return TCM_EDEVICE;
        }
    return TCM_OK;
}

extern "C" int tcm_batch_energy_adaptive(tcm_ctx* t, const tcm_pair_req* reqs, int64_t np, double tol, double* U_out,
                                         int32_t* L_out, double* bound_out, int32_t* status_out)
{
    if (!t || np < 0 || (np > 0 && (!reqs || !U_out || !status_out)) || !(tol > 0.0)) return TCM_EINVAL;
    if (np > (1 << 26)) return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    hipStream_t s = c.stream;
    // one plan at each request's maximum order; every step on the device, one read-back:
    // moments (computed or reused), sum |q| of molecules that lack it (meta[5], once per
    // molecule), each pair's order chosen, the pairs listed again by chosen order, the
    // contractions at those orders
    ReqPlan rp;
    int rc = plan_requests(c, reqs, np, true, rp);
    if (rc != TCM_OK) return rc;
    BuiltPlan bp;
    if ((rc = build_plan(&c, c.ws, rp.mj, rp.pj, bp, s)) != TCM_OK) return rc;
    const int npj = (int)rp.pj.size();
    AdaptBufs ab;
    if ((rc = adapt_setup(c, c.adapt, bp, ab)) != TCM_OK) return rc;
    if ((rc = run_plan(&c, bp, s, false, nullptr, false)) != TCM_OK) return rc;
    if ((rc = abs_sums(c, rp, s)) != TCM_OK) return rc;
    if ((rc = adapt_launch(bp, ab, tol, s)) != TCM_OK) return rc;
    double* dB = ab.bound;
    int32_t* dL = ab.L;
    std::vector<double> U(npj > 0 ? npj : 1), B(npj > 0 ? npj : 1);
    std::vector<int32_t> st(npj > 0 ? npj : 1), Lc(npj > 0 ? npj : 1);
    {
        const void* src[4] = {bp.P.U, bp.P.status, dB, dL};
        void* dst[4] = {U.data(), st.data(), B.data(), Lc.data()};
        const size_t nd = sizeof(double) * (size_t)npj, ni = sizeof(int32_t) * (size_t)npj;
        const size_t bytes[4] = {nd, ni, nd, ni};
        if ((rc = read_back(c, bp, s, 4, src, dst, bytes)) != TCM_OK) return rc;
    }
    mark_computed(rp);
    for (int64_t i = 0; i < np; ++i) {
        status_out[i] = rp.pre_status[i];
        U_out[i] = std::nan("");
        if (L_out) L_out[i] = -1;
        if (bound_out) bound_out[i] = std::nan("");
    }
    for (int k = 0; k < npj; ++k) {
        const int64_t i = rp.pj_req[k];
        status_out[i] = st[k];
        if (st[k] != TCM_OK) continue;
        U_out[i] = U[k];
        if (L_out) L_out[i] = Lc[k];
        if (bound_out) bound_out[i] = B[k];
    }
    return first_error(status_out, np);
}

// ---------------------------------------------------------------- forces and torques
constexpr int FT_N = 10;

extern "C" int tcm_pair_forces(tcm_ctx* t, tcm_mol_id a, tcm_mol_id b, const double* R, const double* quat_b, int L,
                               int flags, double* out, double* forces_A, double* forces_B)
{
    if (!t || !R || !out || L < 0 || L > LMAX || (flags & TCM_TRIANGULAR)) return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    hipStream_t s = c.stream;
    for (int k = 0; k < FT_N; ++k) out[k] = std::nan("");
    tcm_pair_req req{};
    req.a = a;
    req.b = b;
    for (int d = 0; d < 3; ++d) req.R[d] = R[d];
    if (quat_b)
        for (int d = 0; d < 4; ++d) req.quat_b[d] = quat_b[d];
    else
        req.quat_b[0] = 1.0;
    req.L = L;
    req.flags = flags & (TCM_REUSE | TCM_UNCHECKED);
    ReqPlan rp;
    int rc = plan_requests(c, &req, 1, (flags & TCM_REUSE) != 0, rp);
    if (rc != TCM_OK) return rc;
    if (rp.pre_status[0] != TCM_OK) return rp.pre_status[0];
    BuiltPlan bp;
    if ((rc = build_plan(&c, c.ws, rp.mj, rp.pj, bp, s)) != TCM_OK) return rc;
    if ((rc = run_plan(&c, bp, s, false, nullptr, false)) != TCM_OK) return rc;   // the force kernel writes U
    const bool atoms = forces_A || forces_B;
    const int nr = (L + 1) * (L + 2) / 2, na = L * (L + 1) / 2;
    if ((rc = c.alloc(c.force_ft, sizeof(double) * FT_N)) != TCM_OK) return rc;
    if (atoms && ((rc = c.alloc(c.force_w, sizeof(double) * 4 * nr)) != TCM_OK ||
                  (rc = c.alloc(c.force_t, sizeof(double) * (36 + 16 * (size_t)na))) != TCM_OK))
        return rc;
    if (launch_pairs_ft(bp.P, 0, 1, (double*)c.force_ft.p, atoms ? (double*)c.force_w.p : nullptr,
                        atoms ? (double*)c.force_t.p : nullptr, s) != hipSuccess)
        return TCM_EDEVICE;
    Mol* ma = c.mols[a].get();
    Mol* mb = c.mols[b].get();
    const bool dev = (flags & TCM_DEVICE_IO) != 0;
    double* FA = forces_A;
    double* FB = forces_B;
    if (atoms && !dev) {
        if (forces_A && (rc = c.alloc(c.force_a, sizeof(double) * 3 * std::max<int64_t>(ma->n, 1))) != TCM_OK) return rc;
        if (forces_B && (rc = c.alloc(c.force_b, sizeof(double) * 3 * std::max<int64_t>(mb->n, 1))) != TCM_OK) return rc;
        FA = forces_A ? (double*)c.force_a.p : nullptr;
        FB = forces_B ? (double*)c.force_b.p : nullptr;
    }
    // (at L = 0 the tables are empty and the kernel writes zero forces)
    const double* atab = (const double*)c.force_t.p;
    if (FA && launch_atom_forces(atab, 0, L, ma->x, ma->y, ma->z, ma->q, ma->n, (const double*)ma->meta.p, FA, s) !=
                  hipSuccess)
        return TCM_EDEVICE;
    if (FB && launch_atom_forces(atab, 1, L, mb->x, mb->y, mb->z, mb->q, mb->n, (const double*)mb->meta.p, FB, s) !=
                  hipSuccess)
        return TCM_EDEVICE;
    double ft[FT_N];
    int32_t st = TCM_OK;
    if (hipMemcpyAsync(ft, c.force_ft.p, sizeof(ft), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&st, bp.P.status, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return TCM_EDEVICE;
    if (atoms && !dev) {
        if (forces_A && ma->n > 0 &&
            hipMemcpyAsync(forces_A, FA, sizeof(double) * 3 * ma->n, hipMemcpyDeviceToHost, s) != hipSuccess)
            return TCM_EDEVICE;
        if (forces_B && mb->n > 0 &&
            hipMemcpyAsync(forces_B, FB, sizeof(double) * 3 * mb->n, hipMemcpyDeviceToHost, s) != hipSuccess)
            return TCM_EDEVICE;
    }
    if ((rc = check_err(&c, bp, s)) != TCM_OK) return rc;    // synchronises the stream
    mark_computed(rp);
    if (st != TCM_OK) {
        if (!dev) {
            if (forces_A) std::fill(forces_A, forces_A + 3 * ma->n, std::nan(""));
            if (forces_B) std::fill(forces_B, forces_B + 3 * mb->n, std::nan(""));
        }
        return st;
    }
    for (int k = 0; k < FT_N; ++k) out[k] = ft[k];
    return TCM_OK;
}

extern "C" int tcm_batch_forces(tcm_ctx* t, const tcm_pair_req* reqs, int64_t np, double* out, int32_t* status_out)
{
    if (!t || np < 0 || (np > 0 && (!reqs || !out || !status_out))) return TCM_EINVAL;
    if (np > (1 << 26)) return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipSetDevice(c.device);
    hipStream_t s = c.stream;
    // the force kernel differentiates the square truncation only: triangular items are
    // invalid (given an order outside the accepted range, so that planning rejects them)
    std::vector<tcm_pair_req> rq(reqs, reqs + np);
    for (tcm_pair_req& r : rq)
        if (r.flags & TCM_TRIANGULAR) r.L = -1;
    ReqPlan rp;
    int rc = plan_requests(c, rq.data(), np, true, rp);
    if (rc != TCM_OK) return rc;
    BuiltPlan bp;
    if ((rc = build_plan(&c, c.ws, rp.mj, rp.pj, bp, s)) != TCM_OK) return rc;
    if ((rc = run_plan(&c, bp, s, false, nullptr, false)) != TCM_OK) return rc;   // the force kernel writes U
    const int npj = (int)rp.pj.size();
    std::vector<double> ft((size_t)FT_N * (npj > 0 ? npj : 1));
    std::vector<int32_t> st(npj > 0 ? npj : 1);
    if (npj > 0) {
        if ((rc = c.alloc(c.force_ft, sizeof(double) * FT_N * npj)) != TCM_OK) return rc;
        if (launch_pairs_ft(bp.P, 0, npj, (double*)c.force_ft.p, nullptr, nullptr, s) != hipSuccess)
            return TCM_EDEVICE;
    }
    {
        const void* src[2] = {c.force_ft.p, bp.P.status};
        void* dst[2] = {ft.data(), st.data()};
        const size_t bytes[2] = {npj > 0 ? sizeof(double) * FT_N * (size_t)npj : 0, sizeof(int32_t) * (size_t)npj};
        if ((rc = read_back(c, bp, s, 2, src, dst, bytes)) != TCM_OK) return rc;
    }
    mark_computed(rp);
    for (int64_t i = 0; i < np; ++i) {
        status_out[i] = rp.pre_status[i];
        for (int k = 0; k < FT_N; ++k) out[FT_N * i + k] = std::nan("");
    }
    for (int k = 0; k < npj; ++k) {
        const int64_t i = rp.pj_req[k];
        status_out[i] = st[k];
        if (st[k] == TCM_OK)
            for (int j = 0; j < FT_N; ++j) out[FT_N * i + j] = ft[(size_t)FT_N * k + j];
    }
    return first_error(status_out, np);
}

// Batch-aware tuning: the tile launch of each (precision, L) group of the batch is timed for
// every candidate kper (applied to all the group's size buckets), and the fastest is kept
// for every size bucket of the group's molecules.
extern "C" int tcm_autotune_batch(tcm_ctx* t, const tcm_pair_req* reqs, int64_t npairs, double* best_ms)
{
    if (!t || npairs < 0 || (npairs > 0 && !reqs)) return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    if (c.server) return TCM_EAGAIN;         // tilings are fixed while a server runs
    (void)hipSetDevice(c.device);
    hipStream_t s = c.stream;
    ReqPlan rp;
    int rc = plan_requests(c, reqs, npairs, false, rp);   // molecules are recomputed afterwards
    if (rc != TCM_OK) return rc;
    if (best_ms) *best_ms = 0.0;
    if (rp.mj.empty()) return TCM_OK;
    std::map<std::pair<int, int>, std::vector<int64_t>> sizes;   // (prec, L) -> molecule sizes
    for (const MolJob& j : rp.mj) sizes[{j.prec, j.L}].push_back(j.n);
    std::map<int64_t, int> saved;                                 // tune entries to restore on failure
    for (auto& kv : sizes)
        for (int64_t n : kv.second) {
            const int64_t key = tune_key(kv.first.first, kv.first.second, n);
            auto it = c.tune.find(key);
            saved[key] = it == c.tune.end() ? 0 : it->second;
        }
    std::map<std::pair<int, int>, std::pair<double, int>> best;    // (prec, L) -> (ms, kper)
    std::vector<hipEvent_t> ev(2 * sizes.size(), nullptr);
    for (auto& e : ev)
        if (rc == TCM_OK && hipEventCreate(&e) != hipSuccess) rc = TCM_EDEVICE;
    bool any64 = false;                                           // FP64 groups try every candidate
    for (auto& kv : sizes) any64 |= kv.first.first == TCM_F64;
    for (int k = 16; rc == TCM_OK && k <= 256; k <<= 1) {
        if (!any64 && k > std::max(16, c.f32_run_max)) break;     // FP32 groups are capped
        for (auto& kv : sizes)
            for (int64_t n : kv.second) c.tune[tune_key(kv.first.first, kv.first.second, n)] = k;
        BuiltPlan bp;
        if ((rc = build_plan(&c, c.ws, rp.mj, {}, bp, s)) != TCM_OK) break;
        const int ng = (int)bp.groups.size();
        if (launch_clear(bp.P.err, bp.sync_ints, s) != hipSuccess ||
            launch_stats(bp.P, 0, bp.n_stats, s) != hipSuccess ||
            launch_stats_finalize(bp.P, 0, bp.P.nmol, s) != hipSuccess) {
            rc = TCM_EDEVICE;
            break;
        }
        std::vector<double> ms(ng, 1e300);
        for (int rep = 0; rc == TCM_OK && rep < 3; ++rep) {
            for (int gi = 0; gi < ng && rc == TCM_OK; ++gi) {
                const BuiltPlan::Group& G = bp.groups[gi];
                if (hipEventRecord(ev[2 * gi], s) != hipSuccess ||
                    launch_tiles(G.prec, G.L, bp.P, bp.n_stats + G.begin, bp.n_stats + G.end, s) != hipSuccess ||
                    hipEventRecord(ev[2 * gi + 1], s) != hipSuccess)
                    rc = TCM_EDEVICE;
            }
            if (rc == TCM_OK && hipStreamSynchronize(s) != hipSuccess) rc = TCM_EDEVICE;
            for (int gi = 0; gi < ng && rc == TCM_OK; ++gi) {
                float e = 0.f;
                (void)hipEventElapsedTime(&e, ev[2 * gi], ev[2 * gi + 1]);
                if (rep > 0 || gi > 0) ms[gi] = std::min(ms[gi], (double)e);   // the very first launch warms up
            }
        }
        for (int gi = 0; gi < ng && rc == TCM_OK; ++gi) {
            const std::pair<int, int> key{bp.groups[gi].prec, bp.groups[gi].L};
            const int keff = key.first == TCM_F32C ? std::min(k, c.f32_run_max) : k;   // as kper_for applies it
            auto it = best.find(key);
            if (it == best.end() || ms[gi] < it->second.first) best[key] = {ms[gi], keff};
        }
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc != TCM_OK) {
        for (auto& kv : saved) {
            if (kv.second) c.tune[kv.first] = kv.second; else c.tune.erase(kv.first);
        }
        return rc;
    }
    double total = 0.0;
    for (auto& kv : sizes) {
        const auto& b = best[kv.first];
        total += b.first;
        for (int64_t n : kv.second) c.tune[tune_key(kv.first.first, kv.first.second, n)] = b.second;
    }
    if (best_ms) *best_ms = total;
    return TCM_OK;
}

extern "C" int tcm_autotune(tcm_ctx* t, int prec, int L, int64_t n, int* best_k, double* best_ms)
{
    if (!t || L < 0 || L > LMAX || n <= 0 || n > (int64_t(1) << 30) || (prec != TCM_F64 && prec != TCM_F32C))
        return TCM_EINVAL;
    Ctx& c = t->c;
    std::lock_guard<std::mutex> g(c.mu);
    if (c.server) return TCM_EAGAIN;         // tilings are fixed while a server runs
    (void)hipSetDevice(c.device);
    hipStream_t s = c.stream;
    std::vector<double> coords(3 * n), charges(n);
    uint64_t st = 0x9e3779b97f4a7c15ULL ^ (uint64_t)n;
    auto rnd = [&]() {
        st ^= st << 13; st ^= st >> 7; st ^= st << 17;
        return (double)(st >> 11) * 0x1.0p-53;
    };
    for (int64_t i = 0; i < n; ++i) {
        double v[3];
        do {
            for (double& e : v) e = 2 * rnd() - 1;
        } while (v[0] * v[0] + v[1] * v[1] + v[2] * v[2] > 1.0);
        for (int d = 0; d < 3; ++d) coords[3 * i + d] = 10.0 * v[d];
        charges[i] = 2 * rnd() - 1;
    }
    // enough copies that every candidate's launch holds many waves of items (at least 64M
    // atoms, or 4096 copies of a small molecule): the timing is then the steady-state
    // throughput a large batch sees, not the fill of a half-empty device
    int64_t reps = (int64_t(64) << 20) / n;
    if (reps < 1) reps = 1;
    if (reps > 4096) reps = 4096;
    DevBuf atoms, qbuf;
    const double* d[4];
    int rc = upload_atoms(c, atoms, coords.data(), charges.data(), n, d, s);
    if (rc == TCM_OK) rc = c.alloc(qbuf, sizeof(double) * (nh(L) + 8) * reps);
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    for (auto& e : ev)
        if (rc == TCM_OK && hipEventCreate(&e) != hipSuccess) rc = TCM_EDEVICE;
    const int64_t key = tune_key(prec, L, n);
    const bool had = c.tune.count(key) > 0;
    const int old = had ? c.tune[key] : 0;
    double bestt = 1e300;
    int bestk = 0;
    const int kmax = prec == TCM_F32C ? std::max(8, std::min(256, c.f32_run_max)) : 256;
    for (int k = 8; rc == TCM_OK && k <= kmax; k <<= 1) {
        c.tune[key] = k;
        std::vector<MolJob> jobs(reps);
        for (int64_t r = 0; r < reps; ++r) {
            MolJob& j = jobs[r];
            j = MolJob{};
            j.x = d[0]; j.y = d[1]; j.z = d[2]; j.q = d[3];
            j.n = n;
            j.L = L;
            j.prec = prec;
            j.Q = (double*)qbuf.p + r * (nh(L) + 8);
            j.meta = j.Q + nh(L);
        }
        BuiltPlan bp;
        if ((rc = build_plan(&c, c.ws, jobs, {}, bp, s)) != TCM_OK) break;
        double tot = 0.0;
        for (int rep = 0; rep < 4 && rc == TCM_OK; ++rep) {
            rc = run_plan(&c, bp, s, true, ev);
            if (rc == TCM_OK) rc = check_err(&c, bp, s);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[1], ev[2]);
            if (rep > 0) tot += ms;             // first repetition is warm-up
        }
        if (rc == TCM_OK && tot / 3 < bestt) {
            bestt = tot / 3;
            bestk = k;
        }
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    c.release(atoms);
    c.release(qbuf);
    if (rc != TCM_OK || bestk == 0) {
        if (had) c.tune[key] = old; else c.tune.erase(key);
        return rc != TCM_OK ? rc : TCM_EDEVICE;
    }
    c.tune[key] = bestk;
    if (best_k) *best_k = bestk;
    if (best_ms) *best_ms = bestt / (double)reps;
    return TCM_OK;
}
