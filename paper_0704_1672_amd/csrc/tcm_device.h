// HIP device code of libtcm for gfx950 (MI355X).  Steps of the two-centre multipole (TCM) hot
// path and where they run:
//   a0 STATS  centroid and scale of each molecule                  (HBM bound)
//   a1 TILE   eq. (8) moments of a tile of atoms, one m-block       (FP32/FP64 vector ALU)
//   a2        fixed-order merge of the tile partials, unscaling     (last TILE item)
//   a3-a5 PAIR  Wigner rotation of B, irregular harmonics of R0, eq. (9) contraction
//
// Moment recurrence.  The paper evaluates Q_lm = sum_i q_i r_i^l sqrt(4pi/(2l+1)) Y_lm
// (eq. (8)).  Here every atom's harmonics come from a three-term recurrence on the
// direction cosines c = cos(theta), u = sin(theta) e^{i phi} in a normalisation T_lm = k_lm
// R_lm / r^l (R_lm the Racah-normalised solid harmonic) chosen so that
//     T_mm = u^m,   T_{m+1,m} = c T_mm,   T_lm = xi_lm c T_{l-1,m} - T_{l-2,m},
// with rational xi_lm (xi_{m+1,m} = 1, xi_lm xi_{l-1,m} = (2l-1)(2l-3)/((l-1)^2-m^2)).
// The recurrence step then costs one multiply (xi*c) plus one FMA per component and the
// accumulation acc += (q r^l) T one FMA per component; k_lm is divided out once per
// molecule in FP64.  Coordinates are centred and divided by a scale s >= max|r_i| in
// FP64 before the FP32 cast, so |T| <= 7.2 for l <= 32 and no FP32 overflow can occur.
//
// Compensated accumulation (FP32 path): each thread sums its kper atoms in plain FP32,
// then every merge above that -- across the 256 threads of the tile and across tiles --
// is a double-float (hi, lo) TwoSum merge in a fixed order, so a molecule's moments do
// not depend on what else shares the launch.
// Device code of the moment pass (a1) and its fixed-order finalisation (a2), shared by the
// per-(precision, L) tile translation units.
#pragma once
#include "tcm.h"
#include "tcm_internal.h"

namespace tcm {


// ------------------------------------------------------------------ small helpers
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e)
{
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// (ah, al) += (bh, bl), double-float
__device__ __forceinline__ void df_add(float& ah, float& al, float bh, float bl)
{
    float s, e;
    two_sum(ah, bh, s, e);
    e += al + bl;
    ah = s + e;
    al = e - (ah - s);
}

__device__ __forceinline__ int atomic_load_acq(int* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_store_rel(int* p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int atomic_add_acqrel(int* p, int v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ recurrence constants
__host__ __device__ constexpr double xi_lm(int l, int m)
{
    double xi = 1.0;                         // xi_{m+1,m}
    for (int j = m + 2; j <= l; ++j)
        xi = ((2.0 * j - 1.0) * (2.0 * j - 3.0) / (((double)j - 1.0 - m) * ((double)j - 1.0 + m))) / xi;
    return xi;
}

// accumulator offset of (l, m) within the m-block [M0, ...] of order L (real part;
// the imaginary part of m > 0 follows at +1)
__host__ __device__ constexpr int acc_index(int L, int M0, int m, int l)
{
    int o = 0;
    for (int mm = M0; mm < m; ++mm) o += chain_cost(L, mm);
    return o + (l - m) * (m > 0 ? 2 : 1);
}

__host__ __device__ constexpr int acc_count(int L, int M0, int M1)
{
    int o = 0;
    for (int mm = M0; mm <= M1; ++mm) o += chain_cost(L, mm);
    return o;
}

// Runtime inverse: accumulator a of block [M0..] -> packed index h.
__device__ inline int acc_to_packed(int L, int M0, int a)
{
    int m = M0;
    while (a >= chain_cost(L, m)) { a -= chain_cost(L, m); ++m; }
    int per = (m > 0 ? 2 : 1);
    int l = m + a / per;
    int part = a % per;
    return m == 0 ? l * l : l * l + 2 * m - 1 + part;
}

// One step of the l-chain for fixed m, l = LC .. L (template recursion so that xi_lm is a
// compile-time literal and every accumulator index is static).
template <typename F, int L, int M0, int M, int LC>
struct Chain {
    __device__ __forceinline__ static void run(F* acc, const F* w, F c, F& t1r, F& t1i, F& t2r, F& t2i)
    {
        if constexpr (LC <= L) {
            constexpr F xi = (F)xi_lm(LC, M);
            const F xc = xi * c;
            const F nr = fma(xc, t1r, -t2r);
            constexpr int o = acc_index(L, M0, M, LC);
            acc[o] = fma(w[LC], nr, acc[o]);
            t2r = t1r;
            t1r = nr;
            if constexpr (M > 0) {
                const F ni = fma(xc, t1i, -t2i);
                acc[o + 1] = fma(w[LC], ni, acc[o + 1]);
                t2i = t1i;
                t1i = ni;
            }
            Chain<F, L, M0, M, LC + 1>::run(acc, w, c, t1r, t1i, t2r, t2i);
        }
    }
};

// All chains m = M .. M1 of the block.  (sr, si) = T_{M,M} on entry.
template <typename F, int L, int M0, int M1, int M>
struct Block {
    __device__ __forceinline__ static void run(F* acc, const F* w, F c, F ur, F ui, F sr, F si)
    {
        if constexpr (M <= M1) {
            constexpr int o = acc_index(L, M0, M, M);
            acc[o] = fma(w[M], sr, acc[o]);
            if constexpr (M > 0) acc[o + 1] = fma(w[M], si, acc[o + 1]);
            if constexpr (M < L) {
                F t2r = sr, t2i = si;
                F t1r = c * sr, t1i = (M > 0) ? c * si : (F)0;   // T_{M+1,M}
                constexpr int o1 = acc_index(L, M0, M, M + 1);
                acc[o1] = fma(w[M + 1], t1r, acc[o1]);
                if constexpr (M > 0) acc[o1 + 1] = fma(w[M + 1], t1i, acc[o1 + 1]);
                Chain<F, L, M0, M, M + 2>::run(acc, w, c, t1r, t1i, t2r, t2i);
            }
            if constexpr (M < M1) {
                const F nr = sr * ur - si * ui;     // T_{M+1,M+1} = u T_{M,M}
                const F ni = sr * ui + si * ur;
                Block<F, L, M0, M1, M + 1>::run(acc, w, c, ur, ui, nr, ni);
            }
        }
    }
};

// Harmonics of one atom for m-block [M0, M1]: c = cos theta, u = (ur, ui), r = |rho|,
// q = charge.
template <typename F, int L, int M0, int M1>
__device__ __forceinline__ void atom_block(F* acc, F c, F ur, F ui, F r, F q)
{
    F w[L + 1];
    w[0] = q;
#pragma unroll
    for (int l = 1; l <= L; ++l) w[l] = w[l - 1] * r;
    // u^M0 by successive products, the same sequence the chains use from one m to the next:
    // every T_mm is then the same rounded value whatever the m-block partition, so a
    // molecule's moments up to order l do not depend on the order L it is computed at
    F sr = (F)1, si = (F)0;
#pragma unroll
    for (int m = 1; m <= M0; ++m) {
        const F nr = sr * ur - si * ui;
        si = sr * ui + si * ur;
        sr = nr;
    }
    Block<F, L, M0, M1, M0>::run(acc, w, c, ur, ui, sr, si);
}

// ------------------------------------------------------------------ shared memory
// One static buffer, reused by every item kind (a workgroup runs one item at a time).
constexpr int TILE_SMEM_BYTES = 37 * 1024;   // tile kernels: transposed reductions
constexpr int RED_COLS_F32 = 32;             // columns per transpose-reduction chunk
constexpr int RED_COLS_F64 = 16;

struct TileCtx {
    const MolWork* mw;
    int tile;
    int blk;
    double cx, cy, cz, inv_s;
};

// Transposed reduction of NA per-thread FP32 accumulators over the 256 threads of the
// workgroup: each column is summed by 8 threads with a TwoSum cascade over 32 rows, the
// 8 double-float partials are merged in order, and (hi, lo) is written to out.
template <int NA>
__device__ __forceinline__ void reduce_write_f32(const float* acc, char* smem, int L, int M0,
                                                  float* out_hi, float* out_lo)
{
    float* red = reinterpret_cast<float*>(smem);                     // [WG][33]
    float* grp = red + WG * (RED_COLS_F32 + 1);                       // [8][32][2]
    const int tid = threadIdx.x;
    constexpr int NCH = (NA + RED_COLS_F32 - 1) / RED_COLS_F32;
    static_assert(WG == 256, "reduction layout assumes 256 threads");
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
#pragma unroll
        for (int j = 0; j < RED_COLS_F32; ++j) {
            const int a = ch * RED_COLS_F32 + j;
            red[tid * (RED_COLS_F32 + 1) + j] = (a < NA) ? acc[a < NA ? a : 0] : 0.0f;
        }
        __syncthreads();
        {
            const int col = tid & 31, g = tid >> 5;
            float hi = 0.0f, lo = 0.0f;
            for (int r = 0; r < 32; ++r) {
                float s, e;
                two_sum(hi, red[(g * 32 + r) * (RED_COLS_F32 + 1) + col], s, e);
                hi = s;
                lo += e;
            }
            grp[(g * 32 + col) * 2] = hi;
            grp[(g * 32 + col) * 2 + 1] = lo;
        }
        __syncthreads();
        if (tid < 32) {
            const int a = ch * RED_COLS_F32 + tid;
            if (a < NA) {
                float hi = grp[tid * 2], lo = grp[tid * 2 + 1];
                for (int g = 1; g < 8; ++g) df_add(hi, lo, grp[(g * 32 + tid) * 2], grp[(g * 32 + tid) * 2 + 1]);
                const int h = acc_to_packed(L, M0, a);
                out_hi[h] = hi;
                out_lo[h] = lo;
            }
        }
        __syncthreads();
    }
}

template <int NA>
__device__ __forceinline__ void reduce_write_f64(const double* acc, char* smem, int L, int M0, double* out)
{
    double* red = reinterpret_cast<double*>(smem);                   // [WG][17]
    double* grp = red + WG * (RED_COLS_F64 + 1);                      // [16][16]
    const int tid = threadIdx.x;
    constexpr int NCH = (NA + RED_COLS_F64 - 1) / RED_COLS_F64;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
#pragma unroll
        for (int j = 0; j < RED_COLS_F64; ++j) {
            const int a = ch * RED_COLS_F64 + j;
            red[tid * (RED_COLS_F64 + 1) + j] = (a < NA) ? acc[a < NA ? a : 0] : 0.0;
        }
        __syncthreads();
        {
            const int col = tid & 15, g = tid >> 4;                   // 16 groups of 16 rows
            double s = 0.0;
            for (int r = 0; r < 16; ++r) s += red[(g * 16 + r) * (RED_COLS_F64 + 1) + col];
            grp[g * 16 + col] = s;
        }
        __syncthreads();
        if (tid < 16) {
            const int a = ch * RED_COLS_F64 + tid;
            if (a < NA) {
                double s = grp[tid];
                for (int g = 1; g < 16; ++g) s += grp[g * 16 + tid];
                out[acc_to_packed(L, M0, a)] = s;
            }
        }
        __syncthreads();
    }
}

// Atom loads.  Each tile reads its atoms through buffer descriptors based at the tile's first
// atom with the tile's byte length as the range, so offsets are 32-bit and a read past the
// tile's end returns 0 instead of touching memory (the indices are also clamped).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int RSRC_WORD3 = 0x00020000;       // raw 32-bit access, gfx9 family

// The arguments are wavefront-uniform (one molecule per workgroup item); reading them
// through readfirstlane keeps the descriptor in scalar registers.
__device__ __forceinline__ rsrc_t tile_rsrc(const double* base, int64_t first, uint32_t bytes)
{
    const uint64_t a = (uint64_t)(base + first);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const uint32_t nb = __builtin_amdgcn_readfirstlane(bytes);
    return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), (short)0, (int)nb, RSRC_WORD3);
}

__device__ __forceinline__ double bload(rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

struct AtomIn {
    double x, y, z, q;
};

struct TileSrc {
    rsrc_t x, y, z, q;
};

__device__ __forceinline__ AtomIn load_atom(const TileSrc& t, uint32_t off)
{
    AtomIn v;
    v.x = bload(t.x, off);
    v.y = bload(t.y, off);
    v.z = bload(t.z, off);
    v.q = bload(t.q, off);
    return v;
}

template <typename F, int L, int M0, int M1>
__device__ __forceinline__ void tile_item(const TileCtx& tc, const DevPlan& P, char* smem)
{
    constexpr int NA = acc_count(L, M0, M1);
    const MolWork& mw = *tc.mw;
    F acc[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] = (F)0;
    const int tid = threadIdx.x;
    // the tile: atoms [first, first + span) of the molecule, thread tid takes first + tid,
    // first + tid + WG, ...
    const int64_t first = (int64_t)tc.tile * WG * mw.kper;
    const int span = (int)min(mw.n - first, (int64_t)WG * mw.kper);
    const uint32_t bytes = (uint32_t)span * 8u;
    TileSrc src;
    src.x = tile_rsrc(mw.x, first, bytes);
    src.y = tile_rsrc(mw.y, first, bytes);
    src.z = tile_rsrc(mw.z, first, bytes);
    src.q = tile_rsrc(mw.q, first, bytes);
    const double cxs = tc.cx * tc.inv_s, cys = tc.cy * tc.inv_s, czs = tc.cz * tc.inv_s;
    double r2max = 0.0;
    const int cnt = tid < span ? (span - tid + WG - 1) / WG : 0;
    if (cnt > 0) {
        // two atoms in flight ahead of the one being evaluated; offsets past the thread's
        // last atom are clamped to it (values unused)
        const uint32_t last = (uint32_t)(tid + (cnt - 1) * WG) * 8u;
        uint32_t o = (uint32_t)tid * 8u;
        AtomIn n0 = load_atom(src, o);
        AtomIn n1 = load_atom(src, min(o + WG * 8u, last));
        o += 2 * WG * 8u;
        for (int i = 0; i < cnt; ++i) {
            const AtomIn cur = n0;
            n0 = n1;
            n1 = load_atom(src, min(o, last));
            o += WG * 8u;
            if constexpr (M0 == 0) {               // max |r - c|^2 in FP64, once per atom
                const double dx = cur.x - tc.cx, dy = cur.y - tc.cy, dz = cur.z - tc.cz;
                r2max = fmax(r2max, dx * dx + dy * dy + dz * dz);
            }
            // centred and scaled in FP64 (one rounding), then cast
            const F px = (F)fma(cur.x, tc.inv_s, -cxs);
            const F py = (F)fma(cur.y, tc.inv_s, -cys);
            const F pz = (F)fma(cur.z, tc.inv_s, -czs);
            const F r2 = px * px + py * py + pz * pz;
            F ir, r;
            if constexpr (sizeof(F) == 4) {
                ir = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
                r = r2 * ir;
            } else {
                r = sqrt(r2);
                ir = r > 0.0 ? 1.0 / r : 0.0;
            }
            atom_block<F, L, M0, M1>(acc, pz * ir, px * ir, py * ir, r, (F)cur.q);
        }
    }
    const int64_t nt = mw.ntiles;
    if constexpr (sizeof(F) == 4) {
        float* hi = P.part_f + mw.part_off + (int64_t)tc.tile * nh(L);
        float* lo = P.part_f + mw.part_off + (nt + tc.tile) * nh(L);
        reduce_write_f32<NA>(acc, smem, L, M0, hi, lo);
    } else {
        reduce_write_f64<NA>(acc, smem, L, M0, P.part_d + mw.part_off + (int64_t)tc.tile * nh(L));
    }
    if constexpr (M0 == 0) {                       // max |r|^2 of the tile (FP64)
        double* red = reinterpret_cast<double*>(smem);
        red[tid] = r2max;
        __syncthreads();
        for (int s = WG / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
            __syncthreads();
        }
        if (tid == 0) P.r2_part[mw.r2_off + tc.tile] = red[0];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ dispatch over (L, block)
template <typename F, int L, int B>
__device__ __forceinline__ void dispatch_block(const TileCtx& tc, const DevPlan& P, char* smem)
{
    constexpr int BUDGET = sizeof(F) == 4 ? BUDGET_F32 : BUDGET_F64;
    constexpr Partition part = make_partition(L, BUDGET);
    if constexpr (B < part.nb) {
        if (tc.blk == B) {
            tile_item<F, L, part.start[B], part.start[B + 1] - 1>(tc, P, smem);
            return;
        }
        dispatch_block<F, L, B + 1>(tc, P, smem);
    }
}

// Fixed-order merge of the tile partials of one molecule; unscale to physical moments.
__device__ inline void finalize_moments(const DevPlan& P, int mol, char* smem)
{
    const MolWork& mw = P.mols[mol];
    const int tid = threadIdx.x;
    const int L = mw.L, NHl = nh(L);
    double* spow = reinterpret_cast<double*>(smem);       // s^l, l = 0..L
    double* red = spow + (LMAX + 2);                      // [WG]
    if (tid == 0) {
        const double s = mw.meta[4];
        spow[0] = 1.0;
        for (int l = 1; l <= L; ++l) spow[l] = spow[l - 1] * s;
    }
    double r2 = 0.0;
    for (int t = tid; t < mw.ntiles; t += WG) r2 = fmax(r2, P.r2_part[mw.r2_off + t]);
    red[tid] = r2;
    __syncthreads();
    for (int s = WG / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    const double r2max = red[0];
    __syncthreads();
    // Tile partials.  Up to FIN_SERIAL_MAX tiles, one thread per harmonic sums them in tile
    // order; beyond, FIN_H harmonics at a time: thread (hl, g) sums the tiles t = g, g + FIN_G,
    // ... of harmonic h0 + hl (four tiles' loads in flight before they are added), then the
    // FIN_G group sums are added in group order.  A fixed order per molecule, whatever else
    // shares the launch; a molecule of thousands of tiles no longer waits on one dependent
    // chain of loads per harmonic.
    constexpr int FIN_H = 32, FIN_G = WG / FIN_H, FIN_SERIAL_MAX = 256;
    const int hl = tid % FIN_H, g = tid / FIN_H;
    const int64_t nt = mw.ntiles;
    if (nt <= FIN_SERIAL_MAX) {
        // few tiles (every molecule of a typical batch): one thread per harmonic, tiles in order
        for (int h = tid; h < NHl; h += WG) {
            double v;
            if (mw.prec == TCM_F32C) {
                const float* hi = P.part_f + mw.part_off;
                const float* lo = P.part_f + mw.part_off + nt * NHl;
                float H = 0.0f, Lo = 0.0f;
                for (int64_t t = 0; t < nt; ++t) df_add(H, Lo, hi[t * NHl + h], lo[t * NHl + h]);
                v = (double)H + (double)Lo;
            } else {
                const double* pd = P.part_d + mw.part_off;
                v = 0.0;
                for (int64_t t = 0; t < nt; ++t) v += pd[t * NHl + h];
            }
            mw.Q[h] = v * P.invk[h] * spow[l_of(h)];
        }
    }
    for (int h0 = 0; nt > FIN_SERIAL_MAX && h0 < NHl; h0 += FIN_H) {
        const int h = h0 + hl;
        if (mw.prec == TCM_F32C) {
            const float* hi = P.part_f + mw.part_off;
            const float* lo = P.part_f + mw.part_off + nt * NHl;
            float H = 0.0f, Lo = 0.0f;
            if (h < NHl) {
                int64_t t = g;
                for (; t + 3 * FIN_G < nt; t += 4 * FIN_G) {
                    float a[4], b[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        a[u] = hi[(t + u * FIN_G) * NHl + h];
                        b[u] = lo[(t + u * FIN_G) * NHl + h];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) df_add(H, Lo, a[u], b[u]);
                }
                for (; t < nt; t += FIN_G) df_add(H, Lo, hi[t * NHl + h], lo[t * NHl + h]);
            }
            float* rf = reinterpret_cast<float*>(red);     // [WG] highs, then [WG] lows
            rf[tid] = H;
            rf[WG + tid] = Lo;
            __syncthreads();
            if (g == 0 && h < NHl) {
                for (int q = 1; q < FIN_G; ++q) df_add(H, Lo, rf[q * FIN_H + hl], rf[WG + q * FIN_H + hl]);
                mw.Q[h] = ((double)H + (double)Lo) * P.invk[h] * spow[l_of(h)];
            }
        } else {
            const double* pd = P.part_d + mw.part_off;
            double v = 0.0;
            if (h < NHl) {
                int64_t t = g;
                for (; t + 3 * FIN_G < nt; t += 4 * FIN_G) {
                    double a[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) a[u] = pd[(t + u * FIN_G) * NHl + h];
#pragma unroll
                    for (int u = 0; u < 4; ++u) v += a[u];
                }
                for (; t < nt; t += FIN_G) v += pd[t * NHl + h];
            }
            red[tid] = v;
            __syncthreads();
            if (g == 0 && h < NHl) {
                for (int q = 1; q < FIN_G; ++q) v += red[q * FIN_H + hl];
                mw.Q[h] = v * P.invk[h] * spow[l_of(h)];
            }
        }
        __syncthreads();
    }
    if (tid == 0) mw.meta[3] = sqrt(r2max);
    __syncthreads();
}

template <typename F, int L>
__device__ __forceinline__ void tile_item_entry(const DevPlan& P, int mol, int j, char* smem)
{
    // the statistics launch that precedes this one has written the centre and scale
    const MolWork& mw = P.mols[mol];
    TileCtx tc;
    tc.mw = &mw;
    tc.tile = j / mw.nblk;
    tc.blk = j % mw.nblk;
    tc.cx = mw.meta[0];
    tc.cy = mw.meta[1];
    tc.cz = mw.meta[2];
    tc.inv_s = 1.0 / mw.meta[4];
    dispatch_block<F, L, 0>(tc, P, smem);
}

// Tile kernel over the items [begin, end) of the molecules of one (precision, L) group: one
// workgroup per item (the grid is the item count), so the hardware dispatcher hands out the
// items as slots free up -- in blockIdx order, i.e. in decreasing cost, so the last items to
// start are the cheapest -- and the workgroups of concurrently running launches (the groups of
// other orders on forked streams) interleave with these as the slots free up.  The listing puts
// the m-blocks of one tile on one XCD (positions b with the same b mod 8, back to back) and
// may hold empty positions (molecule -1).  The order does not touch any result: each item
// writes its own partial slot and the partials are merged in tile order afterwards.
template <typename F, int L>
__global__ __launch_bounds__(WG) void tcm_tiles(DevPlan P, int begin, int end)
{
    __shared__ __align__(16) char smem[TILE_SMEM_BYTES];
    const int item = begin + (int)blockIdx.x;
    if (item >= end) return;
    const int j = item - P.n_stats;
    const int mol = __builtin_amdgcn_readfirstlane(P.tile_items[2 * j]);
    if (mol < 0) return;                                 // a padding position of the listing
    tile_item_entry<F, L>(P, mol, __builtin_amdgcn_readfirstlane(P.tile_items[2 * j + 1]), smem);
}

template <typename F, int L>
hipError_t launch_tile_kernel(const DevPlan& P, int begin, int end, hipStream_t s)
{
    if (end <= begin) return hipSuccess;
    hipLaunchKernelGGL((tcm_tiles<F, L>), dim3(end - begin), dim3(WG), 0, s, P, begin, end);
    return hipGetLastError();
}

#define TCM_TILE_CASE(F, LL) \
    case LL:                 \
        return launch_tile_kernel<F, LL>(P, begin, end, s);

}  // namespace tcm
