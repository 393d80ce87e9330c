// Statistics (a0) and pair (a3-a5) kernels of libtcm, the clear kernel, and the launchers.
#include "tcm_device.h"

namespace tcm {

// ------------------------------------------------------------------ STATS items
// Partial sums of x, y, z and the bounding box of one chunk of STATS_CHUNK atoms (HBM bound:
// 24 B/atom).  Every thread issues the loads of all its STATS_PER_THREAD atoms at once; the
// chunk's nine values are reduced within each wavefront by shuffles and across the four
// wavefronts in a fixed order.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fmin(v, __shfl_xor(v, d, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ void stats_item(const DevPlan& P, int mol, int chunk, char* smem)
{
    const MolWork& mw = P.mols[mol];
    const int tid = threadIdx.x;
    const int64_t first = (int64_t)chunk * STATS_CHUNK;
    const int span = (int)min(mw.n - first, (int64_t)STATS_CHUNK);
    const uint32_t bytes = (uint32_t)span * 8u;
    const rsrc_t rx = tile_rsrc(mw.x, first, bytes), ry = tile_rsrc(mw.y, first, bytes),
                 rz = tile_rsrc(mw.z, first, bytes);
    double x[STATS_PER_THREAD], y[STATS_PER_THREAD], z[STATS_PER_THREAD];
    const uint32_t last = span > 0 ? (uint32_t)(span - 1) * 8u : 0u;
#pragma unroll
    for (int j = 0; j < STATS_PER_THREAD; ++j) {     // past the chunk's end: clamped, masked below
        const uint32_t off = min((uint32_t)(tid + j * WG) * 8u, last);
        x[j] = span > 0 ? bload(rx, off) : 0.0;
        y[j] = span > 0 ? bload(ry, off) : 0.0;
        z[j] = span > 0 ? bload(rz, off) : 0.0;
    }
    double v[9] = {0, 0, 0, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int j = 0; j < STATS_PER_THREAD; ++j) {
        if (tid + j * WG >= span) break;
        v[0] += x[j]; v[1] += y[j]; v[2] += z[j];
        v[3] = fmin(v[3], x[j]); v[4] = fmin(v[4], y[j]); v[5] = fmin(v[5], z[j]);
        v[6] = fmax(v[6], x[j]); v[7] = fmax(v[7], y[j]); v[8] = fmax(v[8], z[j]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = wave_sum(v[k]);
#pragma unroll
    for (int k = 3; k < 6; ++k) v[k] = wave_min(v[k]);
#pragma unroll
    for (int k = 6; k < 9; ++k) v[k] = wave_max(v[k]);
    double* red = reinterpret_cast<double*>(smem);   // [WG / 64][9]
    const int wave = tid >> 6;
    if ((tid & 63) == 0)
        for (int k = 0; k < 9; ++k) red[wave * 9 + k] = v[k];
    __syncthreads();
    if (tid < 9) {
        double a = red[tid];
        for (int w = 1; w < WG / 64; ++w) {
            const double b = red[w * 9 + tid];
            a = tid < 3 ? a + b : tid < 6 ? fmin(a, b) : fmax(a, b);
        }
        P.stats_part[(mw.stats_off + chunk) * 10 + tid] = a;
    }
    __syncthreads();
}

// An item covering a run of consecutive chunks (molecules with more chunks than the planner's
// item cap): the same record over all of the run's atoms.
__device__ __forceinline__ void stats_run(const DevPlan& P, int mol, int item, char* smem)
{
    const MolWork& mw = P.mols[mol];
    const int tid = threadIdx.x;
    // the molecule's chunks of STATS_CHUNK atoms, split over its nstats items in runs of
    // consecutive chunks (one chunk per item unless the planner capped the item count)
    const int64_t nch = (mw.n + STATS_CHUNK - 1) / STATS_CHUNK;
    double v[9] = {0, 0, 0, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    auto chunk_stats = [&](int64_t chunk) __attribute__((always_inline)) {
        const int64_t first = chunk * STATS_CHUNK;
        const int span = (int)min(mw.n - first, (int64_t)STATS_CHUNK);   // >= 1
        const uint32_t bytes = (uint32_t)span * 8u;
        const rsrc_t rx = tile_rsrc(mw.x, first, bytes), ry = tile_rsrc(mw.y, first, bytes),
                     rz = tile_rsrc(mw.z, first, bytes);
        double x[STATS_PER_THREAD], y[STATS_PER_THREAD], z[STATS_PER_THREAD];
        const uint32_t last = (uint32_t)(span - 1) * 8u;
#pragma unroll
        for (int j = 0; j < STATS_PER_THREAD; ++j) {     // past the chunk's end: clamped, masked below
            const uint32_t off = min((uint32_t)(tid + j * WG) * 8u, last);
            x[j] = bload(rx, off);
            y[j] = bload(ry, off);
            z[j] = bload(rz, off);
        }
#pragma unroll
        for (int j = 0; j < STATS_PER_THREAD; ++j) {
            if (tid + j * WG >= span) break;
            v[0] += x[j]; v[1] += y[j]; v[2] += z[j];
            v[3] = fmin(v[3], x[j]); v[4] = fmin(v[4], y[j]); v[5] = fmin(v[5], z[j]);
            v[6] = fmax(v[6], x[j]); v[7] = fmax(v[7], y[j]); v[8] = fmax(v[8], z[j]);
        }
    };
    const int64_t per = (nch + mw.nstats - 1) / mw.nstats;
    const int64_t c1 = min(nch, (int64_t)(item + 1) * per);
    for (int64_t chunk = (int64_t)item * per; chunk < c1; ++chunk) chunk_stats(chunk);
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = wave_sum(v[k]);
#pragma unroll
    for (int k = 3; k < 6; ++k) v[k] = wave_min(v[k]);
#pragma unroll
    for (int k = 6; k < 9; ++k) v[k] = wave_max(v[k]);
    double* red = reinterpret_cast<double*>(smem);   // [WG / 64][9]
    const int wave = tid >> 6;
    if ((tid & 63) == 0)
        for (int k = 0; k < 9; ++k) red[wave * 9 + k] = v[k];
    __syncthreads();
    if (tid < 9) {
        double a = red[tid];
        for (int w = 1; w < WG / 64; ++w) {
            const double b = red[w * 9 + tid];
            a = tid < 3 ? a + b : tid < 6 ? fmin(a, b) : fmax(a, b);
        }
        P.stats_part[(mw.stats_off + item) * 10 + tid] = a;
    }
    __syncthreads();
}

// Centre (the given one, else the centroid) and scale s >= max |r_i - c| of one molecule from
// its chunk records: one workgroup per molecule, each thread merges a strided subset of the
// records, then a fixed-order tree over the threads.
__device__ __forceinline__ void stats_finalize(const DevPlan& P, int mol, char* smem)
{
    const MolWork& mw = P.mols[mol];
    const int tid = threadIdx.x;
    double v[9] = {0, 0, 0, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int c = tid; c < mw.nstats; c += WG) {
        const double* r = P.stats_part + (mw.stats_off + c) * 10;
        for (int k = 0; k < 3; ++k) v[k] += r[k];
        for (int k = 3; k < 6; ++k) v[k] = fmin(v[k], r[k]);
        for (int k = 6; k < 9; ++k) v[k] = fmax(v[k], r[k]);
    }
    double* red = reinterpret_cast<double*>(smem);   // [9][WG]
    for (int k = 0; k < 9; ++k) red[k * WG + tid] = v[k];
    __syncthreads();
    for (int s = WG / 2; s > 0; s >>= 1) {
        if (tid < s) {
            for (int k = 0; k < 3; ++k) red[k * WG + tid] += red[k * WG + tid + s];
            for (int k = 3; k < 6; ++k) red[k * WG + tid] = fmin(red[k * WG + tid], red[k * WG + tid + s]);
            for (int k = 6; k < 9; ++k) red[k * WG + tid] = fmax(red[k * WG + tid], red[k * WG + tid + s]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        double c[3];
        if (mw.has_centre || mw.n == 0) {
            c[0] = mw.centre[0]; c[1] = mw.centre[1]; c[2] = mw.centre[2];
        } else {
            c[0] = red[0] / (double)mw.n; c[1] = red[WG] / (double)mw.n; c[2] = red[2 * WG] / (double)mw.n;
        }
        double s2 = 0.0;
        if (mw.n > 0)
            for (int d = 0; d < 3; ++d) {
                const double e = fmax(fabs(red[(6 + d) * WG] - c[d]), fabs(c[d] - red[(3 + d) * WG]));
                s2 += e * e;
            }
        double s = sqrt(s2);
        if (!(s > 0.0)) s = 1.0;
        mw.meta[0] = c[0]; mw.meta[1] = c[1]; mw.meta[2] = c[2];
        mw.meta[4] = s;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ PAIR items
// The LDS layout of the pair kernels is sized for the largest order Lm of the launch's pairs;
// a pair's summation order -- and its energy, bit for bit -- depends only on its own order, not
// on Lm or on how many pairs share the launch.
constexpr int PAIR_WG = 256;             // the force kernel and the scan tensor kernel

__device__ void rot_phase(double* v, int L, const double* cs /*[Lm+1][2]*/)
{
    // (Re, Im) of each m > 0 rotated by m*angle: Q_lm -> e^{i m angle} Q_lm
    const int NHl = nh(L);
    for (int h = threadIdx.x; h < NHl; h += PAIR_WG) {
        const int l = l_of(h), off = h - l * l;
        if (off & 1) {                         // Re part of m = (off+1)/2
            const int m = (off + 1) >> 1;
            const double c = cs[2 * m], s = cs[2 * m + 1];
            const double re = v[h], im = v[h + 1];
            v[h] = c * re - s * im;
            v[h + 1] = s * re + c * im;
        }
    }
}

// out = D v (or D^{-1} v) per order l from the compressed tables: row i's nonzero columns are
// max(0, jb + 4k), k < cnt (the header, codes and slot layout are those the runtime writes).
// Every row has K = l/2 + 1 value slots, those past cnt holding zeros, so the products run
// over all K slots: the value loads then depend only on (l, i), not on the row's code, and
// are issued together with it (the zero slots add exact zeros to the partial sums; their
// columns are clamped into the row).
__device__ __forceinline__ void rot_row(const double* tab, int l, int i, bool inverse, int& jb, const double*& val)
{
    const int n = 2 * l + 1, K = l / 2 + 1;
    const double* blk = tab + rot_block_offset(l);
    const int code = (int)blk[(inverse ? n : 0) + i];
    jb = (code & 0xffff) - 1;
    val = blk + 2 * n + (inverse ? K * n : 0) + i;
}

__device__ void rot_matvec(const double* tab, const double* in, double* out, int L, bool inverse)
{
    const int NHl = nh(L);
    for (int h = threadIdx.x; h < NHl; h += PAIR_WG) {
        const int l = l_of(h), i = h - l * l, n = 2 * l + 1, K = l / 2 + 1;
        int jb;
        const double* val;
        rot_row(tab, l, i, inverse, jb, val);
        const double* v = in + l * l;
        // two partial sums (even and odd slots), four slots' loads in flight at a time
        double s0 = 0.0, s1 = 0.0;
        for (int k = 0; k < K; k += 4) {
            double d[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) d[u] = k + u < K ? val[(k + u) * n] : 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double x = d[u] * v[min(n - 1, max(0, jb + 4 * (k + u)))];
                if (u & 1) s1 += x; else s0 += x;
            }
        }
        out[h] = s0 + s1;
    }
}

// cos / sin of m * (gamma, beta, alpha), the ZYZ Euler angles of the unit quaternion
// q = (w, x, y, z) (R = Rz(alpha) Ry(beta) Rz(gamma)), for m = this thread's index <= L.
__device__ inline void euler_phases(const double* quat, int m, int Lm, double* scs /*[3][Lm+1][2]*/)
{
    const double qn = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    const double w = quat[0] / qn, x = quat[1] / qn, y = quat[2] / qn, z = quat[3] / qn;
    // With r1 = |(w, z)| and r2 = |(x, y)|: e^{i a+} = (w + i z)/r1, e^{i a-} = (y - i x)/r2 (the
    // angles atan2(z, w) and atan2(-x, y); either is free, taken as 0, when its modulus vanishes,
    // since the rotation then depends only on the other), gamma = a+ - a-, alpha = a+ + a-, and
    // beta = 2 atan2(r2, r1): e^{i beta} = (r1^2 - r2^2 + 2 i r1 r2) / (r1^2 + r2^2).
    const double r1 = sqrt(w * w + z * z), r2 = sqrt(x * x + y * y);
    double pc = 1.0, ps = 0.0, mc = 1.0, ms = 0.0;
    if (r1 > 0.0) { pc = w / r1; ps = z / r1; }
    if (r2 > 0.0) { mc = y / r2; ms = -x / r2; }
    const double rr = r1 * r1 + r2 * r2;
    const double e[3][2] = {{pc * mc + ps * ms, ps * mc - pc * ms},       // gamma
                            {(r1 * r1 - r2 * r2) / rr, 2.0 * r1 * r2 / rr}, // beta
                            {pc * mc - ps * ms, ps * mc + pc * ms}};      // alpha
    for (int k = 0; k < 3; ++k) {
        // e^{i m angle} by binary powering (at most 2 log2(m) complex products)
        double c = 1.0, s = 0.0, bc = e[k][0], bs = e[k][1];
        for (int t = m; t > 0; t >>= 1) {
            if (t & 1) {
                const double nc = c * bc - s * bs;
                s = c * bs + s * bc;
                c = nc;
            }
            const double nb = bc * bc - bs * bs;
            bs = 2.0 * bc * bs;
            bc = nb;
        }
        scs[(k * (Lm + 1) + m) * 2] = c;
        scs[(k * (Lm + 1) + m) * 2 + 1] = s;
    }
}

// Q' = Z(alpha) D^{-1} Z(beta) D Z(gamma) Q in place on v (t: temporary of nh(L)), D = the
// representation of a +90 degree rotation about x, Z(phi) = diag(e^{i m phi}); every thread
// of the workgroup takes part.
__device__ inline void rotate_moments(const double* rot, double* v, double* t, int L, int Lm, const double* scs)
{
    rot_phase(v, L, scs);
    __syncthreads();
    rot_matvec(rot, v, t, L, false);
    __syncthreads();
    rot_phase(t, L, scs + 2 * (Lm + 1));
    __syncthreads();
    rot_matvec(rot, t, v, L, true);
    __syncthreads();
    rot_phase(v, L, scs + 4 * (Lm + 1));
    __syncthreads();
}

// rotate_moments on two tables at once (each with its own angles): every table row is loaded
// once for both, and each table's arithmetic is exactly that of rotate_moments.  NT threads
// take part (a whole workgroup of NT threads).
template <int NT>
__device__ void rot_phase2(double* va, double* vb, int L, const double* ca, const double* cb)
{
    const int NHl = nh(L);
    for (int e = threadIdx.x; e < 2 * NHl; e += NT) {
        const bool b = e >= NHl;
        const int h = b ? e - NHl : e;
        const int l = l_of(h), off = h - l * l;
        if (off & 1) {
            const int m = (off + 1) >> 1;
            const double* cs = b ? cb : ca;
            double* v = b ? vb : va;
            const double c = cs[2 * m], s = cs[2 * m + 1];
            const double re = v[h], im = v[h + 1];
            v[h] = c * re - s * im;
            v[h + 1] = s * re + c * im;
        }
    }
}

template <int NT>
__device__ void rot_matvec2(const double* tab, const double* ina, const double* inb, double* outa, double* outb,
                            int L, bool inverse)
{
    const int NHl = nh(L);
    for (int h = threadIdx.x; h < NHl; h += NT) {
        const int l = l_of(h), i = h - l * l, n = 2 * l + 1, K = l / 2 + 1;
        int jb;
        const double* val;
        rot_row(tab, l, i, inverse, jb, val);
        const double* va = ina + l * l;
        const double* vb = inb + l * l;
        double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
        for (int k = 0; k < K; k += 4) {
            double d[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) d[u] = k + u < K ? val[(k + u) * n] : 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = min(n - 1, max(0, jb + 4 * (k + u)));
                if (u & 1) {
                    a1 += d[u] * va[j];
                    b1 += d[u] * vb[j];
                } else {
                    a0 += d[u] * va[j];
                    b0 += d[u] * vb[j];
                }
            }
        }
        outa[h] = a0 + a1;
        outb[h] = b0 + b1;
    }
}

template <int NT>
__device__ inline void rotate_moments2(const double* rot, double* va, double* vb, double* ta, double* tb, int L,
                                       int Lm, const double* ca, const double* cb)
{
    rot_phase2<NT>(va, vb, L, ca, cb);
    __syncthreads();
    rot_matvec2<NT>(rot, va, vb, ta, tb, L, false);
    __syncthreads();
    rot_phase2<NT>(ta, tb, L, ca + 2 * (Lm + 1), cb + 2 * (Lm + 1));
    __syncthreads();
    rot_matvec2<NT>(rot, ta, tb, va, vb, L, true);
    __syncthreads();
    rot_phase2<NT>(va, vb, L, ca + 4 * (Lm + 1), cb + 4 * (Lm + 1));
    __syncthreads();
}

// Contraction in the frame where R lies along the z axis.  Rotating A, B and R together leaves
// eq. (9) unchanged; with R = |R| t, t = +-z, the irregular harmonics of t vanish for M != 0 and
// I_{L'0}(t) = (+-1)^{L'} L'!, so with a, b the moments of A and B rotated into that frame and
// divided by f R^l,
//     U = (1/R) sum_{l1, l2} (-1)^{l2} (+-1)^{l1+l2} (l1+l2)! sum_{m >= 0} w_m (-1)^m Re(a_{l1 m} conj(b_{l2 m}))
// (w_0 = 1, w_m = 2; b_{l,-m} = (-1)^m conj(b_lm) folds m < 0 in): O(L^3) after two O(L^3)
// rotations, the pose of B folded into its rotation.  The square truncation keeps l1, l2 <= L;
// the triangular one (TCM_TRIANGULAR) only l1 + l2 <= L.  The frame rotation is the quaternion
// taking n = R/|R| to t = sign(n_z) z, (1 + n.t, n x t) normalised (1 + |n_z| >= 1, so it is
// well conditioned for every direction).
//
// The pair launches take the pairs PAIR_LANES (64) at a time, one pair per lane: every loop
// index (order, row, slot, m) is then the same in all lanes of a wavefront, the rotation-table
// rows are the same for every lane (scalar loads, scalar operands), and the vector units do the
// arithmetic of 64 pairs per instruction.  A group runs to the largest order of its pairs (the
// launch lists pairs by decreasing order, so groups are nearly uniform); a lane whose pair has a
// lower order skips what it does not need.  The work of a pair is small (O(L^3)), so the kernels
// are written for latency: every load a workgroup needs is issued before the first is used.
//   tcm_pairs_rot    (group, l, side), highest orders first: the order-l block of one side's
//                    table rotated into the frame where R lies along z (B's pose folded in; the
//                    Euler phases come from the plan, computed by the host), scaled by
//                    R^-l / f_lm, written to the plan's scratch [side][h][pair];
//   tcm_pairs_sum_w<N> (group, m), one wavefront, largest order up to SW_L, or tcm_pairs_sum_m
//                    (group, m), four wavefronts, larger orders: for each pair the m-term of the
//                    axial contraction;
//   tcm_pairs_final  (pair): U = (sum over m) / R and the status (eq. 2 checked by the m = 0
//                    contraction, which stores |R| or the failure in a check row).
// Each pair's arithmetic is its own lane's, in a fixed order: a result does not depend on the
// other pairs of the launch, nor on which of the two contraction paths the launch takes.
constexpr int ROT_PAD = 4;        // zero rows after an LDS vector: the slots past a row's count read there
constexpr int ROT_WAVES = 4;      // wavefronts of a rotation workgroup (even: a wavefront's m share a parity)

// The largest order of the workgroup's group of pairs: the plan's largest when every group
// reaches it (no load), else from the plan.
__device__ __forceinline__ int group_order(const DevPlan& P)
{
    return P.gorder_uniform ? P.pair_lmax : P.gorder[blockIdx.x];
}

// The pair's |R| for U = u / |R|, or its status when it fails: eq. 2 (|R| > a_A + a_B, strict)
// unless TCM_UNCHECKED (TCM_EDOMAIN), a zero R (TCM_EINVAL); stored in the last row of pum.
__device__ __forceinline__ double pair_check(const PairWork& pw)
{
    const double Rn = sqrt(pw.R[0] * pw.R[0] + pw.R[1] * pw.R[1] + pw.R[2] * pw.R[2]);
    if (!(Rn > 0.0)) return (double)TCM_EINVAL;
    if (!(pw.flags & TCM_UNCHECKED) && !(Rn > pw.metaA[3] + pw.metaB[3])) return (double)TCM_EDOMAIN;
    return Rn;
}

// Largest of v over the wavefront (the same value in every lane).
__device__ __forceinline__ int wave_max(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ void cmul(double& c, double& s, double bc, double bs)
{
    const double t = c * bc - s * bs;
    s = c * bs + s * bc;
    c = t;
}

// x^N by squaring (N fixed at compile time): a chain of about log2 N products, not N.
template <int N>
__device__ __forceinline__ double pow_ct(double x)
{
    if constexpr (N == 0) {
        return 1.0;
    } else if constexpr (N == 1) {
        return x;
    } else {
        const double h = pow_ct<N / 2>(x);
        return (N & 1) ? h * h * x : h * h;
    }
}

// e^{i w phi} and e^{i W phi} from e^{i phi} (W a power of two, w < W): a wavefront w of W
// walks m = w, w + W, ...; the powers by repeated squaring, e^{i w phi} as the product of those
// of w's bits (fewer dependent products than one step at a time).
template <int W>
__device__ __forceinline__ void phase_walk(double ec, double es, int w, double& c0, double& s0, double& cs,
                                          double& ss)
{
    static_assert((W & (W - 1)) == 0, "W is a power of two");
    c0 = 1.0; s0 = 0.0;
    cs = ec; ss = es;                                    // e^{i b phi}, b = 1, 2, 4, ...
#pragma unroll
    for (int b = 1; b < W; b <<= 1) {
        if (w & b) cmul(c0, s0, cs, ss);
        const double c2 = cs * cs - ss * ss;
        ss = 2.0 * cs * ss;
        cs = c2;
    }
}

// One row of D or D^-1 (row-by-row tables: the code, then K values) applied to the LDS vector
// v[j][lane]: the row is the same for every lane (scalar loads); slot 0 reads column max(0, jb),
// slot k > 0 column jb + 4k (at most n + 3: the rows past n are zero, as are the values past the
// row's count), jb the first column of the row's class (rot_class_jb, computed, so that the
// LDS reads do not wait for the table).  The sum over the slots in order, even and odd slots in
// two partial sums.
using cdptr = const __attribute__((address_space(4))) double*;

template <int K>
__device__ __forceinline__ double rot_row_lanes(cdptr row, const double* v, int jb)
{
    const double* vb = v + jb * PAIR_LANES;
    double s0 = row[1] * v[max(0, jb) * PAIR_LANES], s1 = 0.0;
#pragma unroll
    for (int k = 1; k < K; ++k) {
        const double t = row[1 + k] * vb[4 * k * PAIR_LANES];
        if (k & 1) s1 += t; else s0 += t;
    }
    return s0 + s1;
}

// The order-l work of one (group, side): wavefront wv takes the units m = wv, wv + W, ... (the
// rows of Re and Im of m), at most U of them; the rows of Z(beta) D are kept in registers until
// every wavefront has read the vector, then written over it.
template <int l>
__device__ __forceinline__ void rot_order(const DevPlan& P, int begin, int end, int side, double* sv)
{
    constexpr int n = 2 * l + 1, K = l / 2 + 1, W = ROT_WAVES, U = (l + W) / W;
    const int lane = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int g0 = begin + (int)blockIdx.x * PAIR_LANES;
    const int p = min(g0 + lane, end - 1);
    const PairWork& pw = P.pairs[p];
    // loads: the pair's order, frame and order-l moments
    const int Lp = pw.L;
    const size_t st = P.npairs;
    const double* fr = P.frame + (size_t)side * FRAME_N * st + p;
    double ec[3], es[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ec[k] = fr[(2 * k) * st];
        es[k] = fr[(2 * k + 1) * st];
    }
    const double ir = fr[6 * st];
    const bool act = g0 + lane < end && Lp >= l;
    double qr[U], qi[U];
    const double* qall = side ? P.qb_all : P.qa_all;
    if (qall) {                                          // one table for every pair: order l is in it
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int m = min(wv + u * W, l);
            qr[u] = qall[l * l + (m == 0 ? 0 : 2 * m - 1)];
            qi[u] = qall[l * l + (m == 0 ? 0 : 2 * m)];
        }
    } else {
        const double* Q = (side ? pw.QB : pw.QA) + (act ? l * l : 0);   // order l exists when act
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int m = act ? min(wv + u * W, l) : 0;
            qr[u] = Q[m == 0 ? 0 : 2 * m - 1];
            qi[u] = Q[m == 0 ? 0 : 2 * m];
        }
    }
    double* v = sv + lane;
    if (wv == 0)
#pragma unroll
        for (int j = n; j < n + ROT_PAD; ++j) v[j * PAIR_LANES] = 0.0;
    // Z(gamma) R^-l on the wavefront's units (e^{i m phi} by successive products along its walk)
    const double sc = pow_ct<l>(ir);
    double c0, s0, cst, sst;
    phase_walk<W>(ec[0], es[0], wv, c0, s0, cst, sst);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int m = wv + u * W;
        if (m > l) break;
        const double re = act ? qr[u] * sc : 0.0, im = act ? qi[u] * sc : 0.0;
        if (m == 0) {
            v[0] = re;
        } else {
            v[(2 * m - 1) * PAIR_LANES] = c0 * re - s0 * im;
            v[2 * m * PAIR_LANES] = s0 * re + c0 * im;
        }
        cmul(c0, s0, cst, sst);
    }
    __syncthreads();
    // Z(beta) D; the wavefront's m all have the parity of wv (W is even)
    const int jc = rot_class_jb(false, wv, l), js = rot_class_jb(true, wv, l);
    cdptr Dr = (cdptr)P.rotr + rot_block_offset(l);
    cdptr Di = Dr + n * (K + 1);
    double r0[U], r1[U];
    phase_walk<W>(ec[1], es[1], wv, c0, s0, cst, sst);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int m = wv + u * W;
        if (m > l) break;
        if (m == 0) {
            r0[u] = rot_row_lanes<K>(Dr, v, jc);
        } else {
            const double re = rot_row_lanes<K>(Dr + (2 * m - 1) * (K + 1), v, jc);
            const double im = rot_row_lanes<K>(Dr + 2 * m * (K + 1), v, js);
            r0[u] = c0 * re - s0 * im;
            r1[u] = s0 * re + c0 * im;
        }
        cmul(c0, s0, cst, sst);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int m = wv + u * W;
        if (m > l) break;
        if (m == 0) {
            v[0] = r0[u];
        } else {
            v[(2 * m - 1) * PAIR_LANES] = r0[u];
            v[2 * m * PAIR_LANES] = r1[u];
        }
    }
    __syncthreads();
    // Z(alpha) D^-1, then 1/f_lm; out to the scratch [side][h][pair] with streaming stores (the
    // scratch, 2 (L+1)^2 doubles per pair, is read once, by the next launch)
    cdptr invf = (cdptr)P.invf + l * l;
    double* out = P.prot + ((size_t)side * nh(P.pair_lmax) + l * l) * st + p;
    phase_walk<W>(ec[2], es[2], wv, c0, s0, cst, sst);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int m = wv + u * W;
        if (m > l) break;
        if (m == 0) {
            const double a0 = rot_row_lanes<K>(Di, v, jc) * invf[0];
            if (act) __builtin_nontemporal_store(a0, out);
        } else {
            const double re = rot_row_lanes<K>(Di + (2 * m - 1) * (K + 1), v, jc);
            const double im = rot_row_lanes<K>(Di + 2 * m * (K + 1), v, js);
            const double f = invf[2 * m - 1];
            if (act) {
                __builtin_nontemporal_store((c0 * re - s0 * im) * f, out + (2 * m - 1) * st);
                __builtin_nontemporal_store((s0 * re + c0 * im) * f, out + 2 * m * st);
            }
        }
        cmul(c0, s0, cst, sst);
    }
}

// Binary dispatch of the block's (uniform) order onto the instantiations LO .. HI.
template <int LO, int HI>
__device__ __forceinline__ void rot_dispatch(int l, const DevPlan& P, int begin, int end, int side, double* sv)
{
    if constexpr (LO == HI) {
        rot_order<LO>(P, begin, end, side, sv);
    } else {
        constexpr int MID = (LO + HI) / 2;
        if (l <= MID) rot_dispatch<LO, MID>(l, P, begin, end, side, sv);
        else rot_dispatch<MID + 1, HI>(l, P, begin, end, side, sv);
    }
}

// Orders 0 .. LHI (a launch whose largest order is above 16 takes the second instantiation).
template <int LHI>
__global__ __launch_bounds__(PAIR_LANES * ROT_WAVES) void tcm_pairs_rot(DevPlan P, int begin, int end)
{
    extern __shared__ __align__(16) double sv[];       // v [2 pair_lmax + 1 + ROT_PAD][64]
    const int l = P.pair_lmax - (int)blockIdx.y;         // highest orders first
    if (l > group_order(P)) return;                      // beyond the group's largest order
    rot_dispatch<0, LHI>(l, P, begin, end, (int)blockIdx.z, sv);
}
template __global__ void tcm_pairs_rot<16>(DevPlan, int, int);
template __global__ void tcm_pairs_rot<LMAX>(DevPlan, int, int);

// In the frame where R lies along t = +-z (I_{L'0}(t) = (+-1)^{L'} L'!, every other M zero) and
// with a, b the rotated moments divided by f R^l,
//     U = (1/R) sum_m w_m (-1)^m T_m,   T_m = sum_{l1, l2 >= m} (-1)^{l2} (+-1)^{l1+l2} (l1+l2)! Re(a_{l1 m} conj b_{l2 m})
// (w_0 = 1, w_m = 2; square truncation l1, l2 <= L, triangular l1 + l2 <= L).  Both contraction
// paths add the same terms in the same order, so that a pair's result does not depend on which
// one its launch takes.  With a and b signed, (+-1)^{l1} and (-+1)^{l2}, and j = l2 - m:
//     d_j = sum_{l1 = m, m+1, ...} (l1 + l2)! a_{l1 m}    (a chain of fused multiply-adds from 0),
//     e_j = fma(Re d_j, Re b_{l2 m}, Im d_j Im b_{l2 m})   (e_j = Re d_j Re b_{l2 m} for m = 0),
//     T_m = (S_0 + S_1) + (S_2 + S_3),   S_r = sum of e_j over j = r mod 4, in increasing j,
//     U = [(V_0 + V_1) + (V_2 + V_3)] / R,   V_r = sum of w_m (-1)^m T_m over m = r mod 4, in
// increasing m.  The four partial sums and the independent d_j keep several multiply-add chains
// in flight: a dependent FP64 multiply-add waits about forty clocks for its predecessor.
// Terms past a pair's order are exact zeros, so the group's largest order does not change them.

// Largest order below N (N = 17 or 25): one wavefront per (group, m).  The a_{l1 m} and b_{l2 m}
// of its 64 pairs (l1, l2 = m .. m + N - 1) are held in registers, zero past the group's largest
// order (the terms they add are exact zeros), and the factorials (2m)! .. (2m + 2N - 2)! in
// scalar registers; every loop is unrolled, and the d_j of four consecutive j are formed together
// (eight multiply-add chains).  The terms and their order are those of the larger-order path.
constexpr int SW_L = 24;                                 // the largest order of the register path

template <int N, bool IM, bool MASK>
__device__ __forceinline__ double sw_sum(const double* ar, const double* ai, const double* br, const double* bi,
                                         cdptr f2, int tl)
{
#pragma clang fp contract(off)                           // e_j, S_r and T_m exactly as written
    constexpr int JB = 4;
    double S[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j0 = 0; j0 < N; j0 += JB) {
        double dr[JB], di[JB];
#pragma unroll
        for (int jj = 0; jj < JB; ++jj) dr[jj] = di[jj] = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
            for (int jj = 0; jj < JB; ++jj) {
                if (j0 + jj >= N) continue;
                double f = f2[k + j0 + jj];
                if (MASK) f = k + j0 + jj <= tl ? f : 0.0;
                dr[jj] = fma(f, ar[k], dr[jj]);
                if (IM) di[jj] = fma(f, ai[k], di[jj]);
            }
#pragma unroll
        for (int jj = 0; jj < JB; ++jj) {
            const int j = j0 + jj;
            if (j >= N) continue;
            S[j & 3] += IM ? fma(dr[jj], br[j], di[jj] * bi[j]) : dr[jj] * br[j];
        }
    }
    return (S[0] + S[1]) + (S[2] + S[3]);
}

template <int N>
__global__ __launch_bounds__(PAIR_LANES) void tcm_pairs_sum_w(DevPlan P, int begin, int end)
{
    static_assert(2 * (N - 1) + 2 * (N - 1) < FACT_N, "the factorials read stay in the table");
    const int lane = threadIdx.x;
    const int g0 = begin + (int)blockIdx.x * PAIR_LANES;
    const int m = blockIdx.y;
    const int p = min(g0 + lane, end - 1);
    const bool valid = g0 + lane < end;
    const size_t st = P.npairs;
    // loads: the group's largest order; the pair's order, flags and sign of R_z; a and b of m
    const int gL = group_order(P);
    if (m > gL) return;                                  // past the group's largest order
    const PairWork& pw = P.pairs[p];
    const int Lp = pw.L;
    const bool tri = (pw.flags & TCM_TRIANGULAR) != 0;
    const double sg = P.frame[7 * st + p];
    const double* A = P.prot + p;
    const double* B = P.prot + (size_t)nh(P.pair_lmax) * st + p;
    double ar[N], ai[N], br[N], bi[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int l = m + k;
        ar[k] = ai[k] = br[k] = bi[k] = 0.0;
        if (l <= gL) {
            const size_t h = m == 0 ? (size_t)l * l : (size_t)l * l + 2 * m - 1;
            ar[k] = A[h * st];
            br[k] = B[h * st];
            if (m > 0) {
                ai[k] = A[(h + 1) * st];
                bi[k] = B[(h + 1) * st];
            }
        }
    }
    // (+-1)^{l1} on a, (-+1)^{l2} on b; zero past the pair's order
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int l = m + k;
        const bool ok = valid && l <= Lp;
        const double s1 = ((l & 1) && sg < 0.0) ? -1.0 : 1.0;
        const double s2 = ((l & 1) && sg > 0.0) ? -1.0 : 1.0;
        ar[k] = ok ? s1 * ar[k] : 0.0;
        ai[k] = ok ? s1 * ai[k] : 0.0;
        br[k] = ok ? s2 * br[k] : 0.0;
        bi[k] = ok ? s2 * bi[k] : 0.0;
    }
    const bool mask = __any(valid && tri);               // some lane truncates triangularly
    const int tl = tri ? Lp - 2 * m : 2 * LMAX;
    const cdptr f2 = (cdptr)P.fact + 2 * m;
    double T;
    if (m == 0)
        T = mask ? sw_sum<N, false, true>(ar, ai, br, bi, f2, tl) : sw_sum<N, false, false>(ar, ai, br, bi, f2, tl);
    else
        T = mask ? sw_sum<N, true, true>(ar, ai, br, bi, f2, tl) : sw_sum<N, true, false>(ar, ai, br, bi, f2, tl);
    if (valid) {
        const double wt = m == 0 ? 1.0 : 2.0;
        P.pum[(size_t)m * st + p] = (m & 1) ? -wt * T : wt * T;
        if (m == 0) P.pum[(size_t)(P.pair_lmax + 1) * st + p] = pair_check(pw);
    }
}
template __global__ void tcm_pairs_sum_w<17>(DevPlan, int, int);
template __global__ void tcm_pairs_sum_w<25>(DevPlan, int, int);

// Orders above SW_L: one workgroup per (group, m).  The signed a_{l1 m} and b_{l2 m} are staged
// in LDS, wavefront w forms d_j for j = w, w + W, ..., and wavefront 0 forms T_m from them and
// writes the signed, weighted T_m for tcm_pairs_final.
__global__ __launch_bounds__(PAIR_LANES * PAIR_WAVES) void tcm_pairs_sum_m(DevPlan P, int begin, int end)
{
    extern __shared__ __align__(16) double sb[];       // fact [2 LMAX + 2], a then d, b: [pair_lmax + 1][2][64]
    constexpr int W = PAIR_WAVES, UN = (LMAX + W) / W;  // k or j of a wavefront: wv + u W, u < UN
    const int lane = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int tid = wv * PAIR_LANES + lane;
    const int g0 = begin + (int)blockIdx.x * PAIR_LANES;
    const int m = blockIdx.y, Lm = P.pair_lmax;
    const int p = min(g0 + lane, end - 1);
    const bool valid = g0 + lane < end;
    const PairWork& pw = P.pairs[p];
    const size_t st = P.npairs;
    double* fs = sb;
    double* sa = sb + 2 * LMAX + 2 + lane;               // a_{m+k, m}, later d_{m+j}: [k][re, im][64]
    double* sbv = sa + (size_t)2 * (Lm + 1) * PAIR_LANES;  // b_{m+j, m}: [j][re, im][64]
    // loads: factorials, the pair's order, flags and sign of R_z, a and b of the wavefront's rows
    const int gL = group_order(P);
    if (m > gL) return;                                  // past the group's largest order
    const int C = gL - m;
    const double fv = P.fact[min(tid, 2 * LMAX + 1)];
    const int Lp = pw.L;
    const bool tri = (pw.flags & TCM_TRIANGULAR) != 0;
    const double sg = P.frame[7 * st + p];
    const double* A = P.prot + p;
    const double* B = P.prot + (size_t)nh(Lm) * st + p;
    double ar[UN], ai[UN], br[UN], bi[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
        const int k = wv + u * W, l = m + k;
        ar[u] = ai[u] = br[u] = bi[u] = 0.0;
        if (k <= C) {
            const size_t h = m == 0 ? (size_t)l * l : (size_t)l * l + 2 * m - 1;
            ar[u] = A[h * st];
            br[u] = B[h * st];
            if (m > 0) {
                ai[u] = A[(h + 1) * st];
                bi[u] = B[(h + 1) * st];
            }
        }
    }
    if (tid < 2 * LMAX + 2) fs[tid] = fv;
#pragma unroll
    for (int u = 0; u < UN; ++u) {
        const int k = wv + u * W, l = m + k;
        const bool ok = valid && l <= Lp;
        const double s1 = ((l & 1) && sg < 0.0) ? -1.0 : 1.0;
        const double s2 = ((l & 1) && sg > 0.0) ? -1.0 : 1.0;
        if (k <= C) {
            sa[(2 * k) * PAIR_LANES] = ok ? s1 * ar[u] : 0.0;
            sa[(2 * k + 1) * PAIR_LANES] = ok ? s1 * ai[u] : 0.0;
            sbv[(2 * k) * PAIR_LANES] = ok ? s2 * br[u] : 0.0;
            sbv[(2 * k + 1) * PAIR_LANES] = ok ? s2 * bi[u] : 0.0;
        }
    }
    __syncthreads();
    // d_{m+j} for the wavefront's j = wv + u W, all together (2 UN chains; the j past C read a
    // clamped factorial and are not used): a term counts where k + j <= tl (triangular:
    // l1 + l2 <= Lp)
    const int tl = tri ? Lp - 2 * m : 2 * LMAX;
    double dr[UN], di[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) dr[u] = di[u] = 0.0;
#pragma unroll 2
    for (int k = 0; k <= C; ++k) {
        const double a_r = sa[(2 * k) * PAIR_LANES], a_i = sa[(2 * k + 1) * PAIR_LANES];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int j = wv + u * W;
            const double f = k + j <= tl ? fs[min(2 * m + k + j, 2 * LMAX + 1)] : 0.0;
            dr[u] = fma(f, a_r, dr[u]);
            di[u] = fma(f, a_i, di[u]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UN; ++u) {
        const int j = wv + u * W;
        if (j <= C) {
            sa[(2 * j) * PAIR_LANES] = dr[u];
            sa[(2 * j + 1) * PAIR_LANES] = di[u];
        }
    }
    __syncthreads();
    if (wv == 0 && valid) {
#pragma clang fp contract(off)                           // e_j, S_r and T_m exactly as written
        double S[4] = {0.0, 0.0, 0.0, 0.0};
        for (int j0 = 0; j0 <= C; j0 += 4)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 + r;
                if (j > C) break;
                const double* d = sa + (size_t)(2 * j) * PAIR_LANES;
                const double* b = sbv + (size_t)(2 * j) * PAIR_LANES;
                S[r] += m > 0 ? fma(d[0], b[0], d[PAIR_LANES] * b[PAIR_LANES]) : d[0] * b[0];
            }
        const double T = (S[0] + S[1]) + (S[2] + S[3]);
        const double wt = m == 0 ? 1.0 : 2.0;
        P.pum[(size_t)m * st + p] = (m & 1) ? -wt * T : wt * T;
        if (m == 0) P.pum[(size_t)(Lm + 1) * st + p] = pair_check(pw);
    }
}

// U = (1/R) sum_{m = 0..L} (the m-terms of tcm_pairs_sum_w or tcm_pairs_sum_m) and the status
// (from the check row of pum); every load issued at once (rows past the pair's order are read
// and not added).
// N: rows loaded, N - 1 >= the launch's largest order (17, 25 or LMAX + 1).
template <int N>
__global__ __launch_bounds__(PAIR_LANES) void tcm_pairs_final(DevPlan P, int begin, int end)
{
    const int p = begin + (int)blockIdx.x * PAIR_LANES + (int)threadIdx.x;
    if (p >= end) return;
    const double* pum = P.pum + p;
    const size_t st = P.npairs;
    const int Lm = P.pair_lmax;
    double t[N];
#pragma unroll
    for (int m = 0; m < N; ++m) t[m] = pum[(size_t)min(m, Lm) * st];
    const double rn = pum[(size_t)(Lm + 1) * st];
    const PairWork& pw = P.pairs[p];
    const int Lp = pw.L, out = pw.out;
    if (!(rn > 0.0)) {
        P.status[out] = (int32_t)rn;
        P.U[out] = __builtin_nan("");
        return;
    }
    {
#pragma clang fp contract(off)
        double V[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < N; ++m) V[m & 3] += m <= Lp ? t[m] : 0.0;   // (adding zero changes nothing)
        P.U[out] = ((V[0] + V[1]) + (V[2] + V[3])) / rn;
        P.status[out] = TCM_OK;
    }
}

// Adaptive truncation: per pair, the smallest order L' <= L whose rigorous bound of the
// truncation error meets tol -- square S_A S_B / (R (1-a-b)) [(a/(1-b))^{L'+1} + (b/(1-a))^{L'+1}],
// triangular S_A S_B t^{L'+1} / (R (1-t)), t = a + b, with a = a_A/R, b = a_B/R and S = sum |q|
// (meta[5] of each molecule) -- by running products of the ratios (no power per order), L when
// none does.  Lout[out] and bout[out] receive the order and its bound (infinite outside the
// domain of eq. 2, where the pair keeps L); the plan's own pair records keep the requested
// orders, so that a plan runs the choice again from them on every replay.
__global__ __launch_bounds__(WG) void tcm_pairs_choose(DevPlan P, int begin, int end, double tol, int32_t* Lout,
                                                       double* bout)
{
    const int p = begin + (int)blockIdx.x * WG + (int)threadIdx.x;
    int L = -1;
    if (p < end) {
        const PairWork& pw = P.pairs[p];
        const double R = sqrt(pw.R[0] * pw.R[0] + pw.R[1] * pw.R[1] + pw.R[2] * pw.R[2]);
        const double al = pw.metaA[3] / R, be = pw.metaB[3] / R;
        L = pw.L;
        double b = __builtin_inf();
        if (al + be < 1.0) {
            const double pre = pw.metaA[5] * pw.metaB[5] / (R * (1.0 - al - be));
            const bool tri = (pw.flags & TCM_TRIANGULAR) != 0;
            const double r1 = tri ? al + be : al / (1.0 - be), r2 = tri ? 0.0 : be / (1.0 - al);
            double p1 = r1, p2 = r2;
            for (int l = 0;; ++l, p1 *= r1, p2 *= r2) {
                b = pre * (p1 + p2);
                if (b <= tol || l == pw.L) {
                    L = l;
                    break;
                }
            }
        }
        Lout[pw.out] = L;
        bout[pw.out] = b;
    }
}

// Regrouping after the order choice: the pairs listed again by decreasing chosen order (Lc[out],
// which the copies carry as their order), so that a group of PAIR_LANES pairs runs to (about)
// the orders its pairs need.  cnt[0 .. LMAX] counts
// the pairs of each order (zeroed before), cnt[LMAX + 1 ..] are the placement cursors.  Each
// workgroup counts its pairs per order in LDS and takes its places with one global atomic per
// order (one per pair put thousands of atomics on a few addresses: 0.25 ms for 32k pairs).  The
// place of a pair within its order is taken by atomics (any order: a pair's arithmetic is its
// own lane's and its result goes to U[out], so its value does not depend on where it lands).
__global__ __launch_bounds__(WG) void tcm_pairs_count(DevPlan P, int npairs, const int32_t* Lc, int32_t* cnt)
{
    __shared__ int h[LMAX + 1];
    const int tid = (int)threadIdx.x;
    if (tid <= LMAX) h[tid] = 0;
    __syncthreads();
    const int p = (int)blockIdx.x * WG + tid;
    if (p < npairs) atomicAdd(&h[Lc[P.pairs[p].out]], 1);
    __syncthreads();
    if (tid <= LMAX && h[tid] > 0) atomicAdd(&cnt[tid], h[tid]);
}

__global__ __launch_bounds__(WG) void tcm_pairs_regroup(DevPlan P, int npairs, const int32_t* Lc, int32_t* cnt,
                                                        PairWork* pairs2, double* frame2)
{
    __shared__ int h[LMAX + 1], base[LMAX + 1];
    const int tid = (int)threadIdx.x;
    if (tid <= LMAX) h[tid] = 0;
    __syncthreads();
    const int p = (int)blockIdx.x * WG + tid;
    PairWork w{};
    int r = 0;                                           // the pair's rank among the workgroup's of its order
    if (p < npairs) {
        w = P.pairs[p];
        w.L = Lc[w.out];
        r = atomicAdd(&h[w.L], 1);
    }
    __syncthreads();
    if (tid <= LMAX && h[tid] > 0) {
        int b = 0;
        for (int L = LMAX; L > tid; --L) b += cnt[L];
        base[tid] = b + atomicAdd(&cnt[LMAX + 1 + tid], h[tid]);
    }
    __syncthreads();
    if (p >= npairs) return;
    const int q = base[w.L] + r;
    pairs2[q] = w;
    const size_t st = (size_t)npairs;
#pragma unroll
    for (int c = 0; c < 2 * FRAME_N; ++c) frame2[c * st + q] = P.frame[c * st + p];
}

__global__ __launch_bounds__(WG) void tcm_pairs_group_orders(const PairWork* pairs2, int npairs, int32_t* gorder)
{
    const int g = (int)(blockIdx.x * WG + threadIdx.x);
    if (g * PAIR_LANES < npairs) gorder[g] = pairs2[g * PAIR_LANES].L;    // the first is the largest
}

// ------------------------------------------------------------------ translation scan
// Regrouping eq. (9) by L' = l1 + l2 and M = m1 + m2 (the geometric factor depends on them
// only) gives, for B translated without rotation,
//     U(R) = (1/R) sum_{L'} (rho/R)^{L'} [Re(conj(I_{L'0}) G_{L'0}) + 2 sum_{M>0} Re(conj(I_{L'M}) G_{L'M})]
// with the pair tensor G_{L'M} = sum_{l1+l2=L', m1+m2=M} (-1)^{l2} a_{l1 m1} b_{l2 m2},
// a = Q^A / (f rho^l), b = Q^B / (f rho^l) (f = sqrt((l+m)!(l-m)!), rho = a_A + a_B, so that
// rho/R < 1 inside the domain of eq. (2)), I the factorial-scaled irregular harmonics of R/|R|
// (the pair kernel's recurrences), and G_{L',-M} = (-1)^M conj(G_{L'M}) folding M < 0 in.
//
// With t = rho/R and u = -t (n_x + i n_y), the recurrences of I give
//     t^{L'} I_{L'M} = (2L'-1)!! u^M p_{L'M},   p_{MM} = 1, p_{M-1,M} = 0,
//     p_{L'M} = (n_z t) p_{L'-1,M} - gamma_{L'M} t^2 p_{L'-2,M},
//     gamma_{L'M} = ((L'-1)^2 - M^2) / ((2L'-1)(2L'-3)),
// so that U R = sum_M Re(conj(u^M) sum_{L'} p_{L'M} Gt_{L'M}) with Gt = w_M (2L'-1)!! G
// (w_0 = 1, w_M = 2).  The table holds one row {Re Gt, Im Gt, gamma, 0} per (L', M),
// column by column (M = 0 .. Lt, L' = M .. Lt; Lt = 2L for the square truncation l1, l2 <= L,
// Lt = L for the triangular one l1 + l2 <= L, whose terms are exactly those with L' <= L): each
// position then costs five FP64 operations per row, the rows read with wave-uniform loads.
// G costs O(L^4) once.

// first row of column M in a table over L' <= Lt
__host__ __device__ constexpr int scan_col_start(int Lt, int M) { return M * (Lt + 1) - M * (M - 1) / 2; }
__host__ __device__ constexpr int scan_rows(int Lt) { return (Lt + 1) * (Lt + 2) / 2; }

// One wave per table row: lanes take the (l1, m1) terms of G_{L'M}, a butterfly sums them.
// Every workgroup rotates and scales its own copy of the moment tables in LDS.
__global__ __launch_bounds__(PAIR_WG) void tcm_scan_tensor(const double* QA, const double* QB, int L, int Lt, double rho,
                                                           const double* invf, const double* rot, int has_rot,
                                                           double q0, double q1, double q2, double q3, double* T)
{
    extern __shared__ __align__(16) double sm[];        // sA, sB, sT [nh(L)], scs [3][L+1][2]
    const int tid = threadIdx.x, NHl = nh(L);
    double* sA = sm;
    double* sB = sA + NHl;
    double* sT = sB + NHl;
    double* scs = sT + NHl;
    const double quat[4] = {q0, q1, q2, q3};
    if (has_rot && tid <= L) euler_phases(quat, tid, L, scs);
    for (int h = tid; h < NHl; h += PAIR_WG) {
        sA[h] = QA[h];
        sB[h] = QB[h];
    }
    __syncthreads();
    if (has_rot) rotate_moments(rot, sB, sT, L, L, scs);
    for (int h = tid; h < NHl; h += PAIR_WG) {
        const double sc = invf[h] * pow(rho, -(double)l_of(h));
        sA[h] *= sc;
        sB[h] *= sc;
    }
    __syncthreads();
    const int e = __builtin_amdgcn_readfirstlane(blockIdx.x * (PAIR_WG / 64) + tid / 64);
    if (e >= scan_rows(Lt)) return;
    int M = 0;
    while (M < Lt && scan_col_start(Lt, M + 1) <= e) ++M;
    const int Lp = M + (e - scan_col_start(Lt, M));
    // a_{l m} for any m: m < 0 through a_{l,-m} = (-1)^m conj(a_lm)
    auto get = [&](const double* v, int l, int m, double& re, double& im) {
        const int am = m < 0 ? -m : m;
        if (am == 0) { re = v[l * l]; im = 0.0; return; }
        re = v[l * l + 2 * am - 1];
        im = v[l * l + 2 * am];
        if (m < 0) {
            im = -im;
            if (am & 1) { re = -re; im = -im; }
        }
    };
    const int l1lo = Lp - L > 0 ? Lp - L : 0, l1hi = Lp < L ? Lp : L;
    const int W = 2 * L + 1, nterm = (l1hi - l1lo + 1) * W;
    double gr = 0.0, gi = 0.0;
    for (int k = tid & 63; k < nterm; k += 64) {
        const int l1 = l1lo + k / W, m1 = k % W - L, l2 = Lp - l1, m2 = M - m1;
        if (m1 < -l1 || m1 > l1 || m2 < -l2 || m2 > l2) continue;
        double ar, ai, br, bi;
        get(sA, l1, m1, ar, ai);
        get(sB, l2, m2, br, bi);
        const double sg = (l2 & 1) ? -1.0 : 1.0;
        gr += sg * (ar * br - ai * bi);
        gi += sg * (ar * bi + ai * br);
    }
    gr = wave_sum(gr);
    gi = wave_sum(gi);
    if ((tid & 63) == 0) {
        double kap = 1.0;                                // (2L'-1)!!
        for (int j = 3; j <= 2 * Lp - 1; j += 2) kap *= j;
        const double w = (M == 0 ? 1.0 : 2.0) * kap;
        const double gam = Lp >= M + 2 ? ((Lp - 1.0) * (Lp - 1.0) - (double)M * M) / ((2.0 * Lp - 1.0) * (2.0 * Lp - 3.0))
                                       : 0.0;
        double* row = T + 4 * (size_t)e;
        row[0] = w * gr;
        row[1] = w * gi;
        row[2] = gam;
        row[3] = 0.0;
    }
}

// SCAN_NP positions per thread (k, k + WG, ...: each a coalesced run of the workgroup), so
// that every table row loaded into SGPRs feeds SCAN_NP positions' arithmetic.
constexpr int SCAN_NP = 2;

__global__ __launch_bounds__(WG) void tcm_scan_eval(const double* __restrict__ T, int Lt, double rho, double aA,
                                                    double aB, int unchecked, const double* __restrict__ R,
                                                    int64_t nR, double* __restrict__ U, int32_t* __restrict__ status)
{
    const int64_t k0 = blockIdx.x * (int64_t)(WG * SCAN_NP) + threadIdx.x;
    double x[SCAN_NP], y[SCAN_NP], ur[SCAN_NP], ui[SCAN_NP], ir[SCAN_NP], acc[SCAN_NP], wr[SCAN_NP], wi[SCAN_NP];
    int st[SCAN_NP];
#pragma unroll
    for (int j = 0; j < SCAN_NP; ++j) {
        const int64_t k = k0 + j * WG;
        st[j] = TCM_EINVAL;
        x[j] = y[j] = ur[j] = ui[j] = ir[j] = 0.0;
        if (k < nR) {
            const double Rx = R[3 * k], Ry = R[3 * k + 1], Rz = R[3 * k + 2];
            const double Rn = sqrt(Rx * Rx + Ry * Ry + Rz * Rz);
            if (Rn > 0.0 && (unchecked || Rn > aA + aB)) {
                st[j] = TCM_OK;
                ir[j] = 1.0 / Rn;
                const double t = rho * ir[j];
                x[j] = Rz * ir[j] * t;
                y[j] = t * t;
                ur[j] = -t * Rx * ir[j];
                ui[j] = -t * Ry * ir[j];
            } else if (Rn > 0.0) {
                st[j] = TCM_EDOMAIN;
            }
        }
        acc[j] = 0.0;
        wr[j] = 1.0;                                     // u^M
        wi[j] = 0.0;
    }
    const int L2 = Lt;
    // the table is read-only here and the same for every lane: constant address space, so
    // that its loads are scalar loads into SGPRs
    using crow = const __attribute__((address_space(4))) double*;
    crow row = (crow)T;
    for (int M = 0; M <= L2; ++M) {
        double Sr[SCAN_NP], Si[SCAN_NP], p1[SCAN_NP], p2[SCAN_NP];
#pragma unroll
        for (int j = 0; j < SCAN_NP; ++j) {
            if (M > 0) {
                const double tr = wr[j] * ur[j] - wi[j] * ui[j];
                wi[j] = wr[j] * ui[j] + wi[j] * ur[j];
                wr[j] = tr;
            }
            Sr[j] = row[0];
            Si[j] = row[1];
            p1[j] = 1.0;
            p2[j] = 0.0;
        }
        row += 4;
        int Lp = M + 1;
        for (; Lp < L2; Lp += 2, row += 8) {            // two rows per trip
            const double g0 = row[0], g1 = row[1], c0 = row[2], h0 = row[4], h1 = row[5], c1 = row[6];
#pragma unroll
            for (int j = 0; j < SCAN_NP; ++j) {
                const double pa = x[j] * p1[j] - (c0 * y[j]) * p2[j];
                Sr[j] += pa * g0;
                Si[j] += pa * g1;
                const double pb = x[j] * pa - (c1 * y[j]) * p1[j];
                Sr[j] += pb * h0;
                Si[j] += pb * h1;
                p2[j] = pa;
                p1[j] = pb;
            }
        }
        if (Lp == L2) {
            const double g0 = row[0], g1 = row[1], c0 = row[2];
#pragma unroll
            for (int j = 0; j < SCAN_NP; ++j) {
                const double p = x[j] * p1[j] - (c0 * y[j]) * p2[j];
                Sr[j] += p * g0;
                Si[j] += p * g1;
            }
            row += 4;
        }
#pragma unroll
        for (int j = 0; j < SCAN_NP; ++j) acc[j] += wr[j] * Sr[j] + wi[j] * Si[j];
    }
#pragma unroll
    for (int j = 0; j < SCAN_NP; ++j) {
        const int64_t k = k0 + j * WG;
        if (k < nR) {
            U[k] = st[j] == TCM_OK ? acc[j] * ir[j] : __builtin_nan("");
            status[k] = st[j];
        }
    }
}

hipError_t launch_scan(const double* QA, const double* QB, int L, int triangular, double rho, double aA, double aB,
                       int unchecked, const double* invf, const double* rot, const double* quat, double* T,
                       const double* R, int64_t nR, double* U, int32_t* status, hipStream_t s)
{
    const int has_rot = quat && !(quat[0] > 0 && quat[1] == 0 && quat[2] == 0 && quat[3] == 0);
    const double q[4] = {quat ? quat[0] : 1.0, quat ? quat[1] : 0.0, quat ? quat[2] : 0.0, quat ? quat[3] : 0.0};
    const size_t tb = sizeof(double) * (3 * (size_t)nh(L) + 6 * (L + 1));
    const int waves = PAIR_WG / 64;
    const int Lt = triangular ? L : 2 * L;
    hipLaunchKernelGGL(tcm_scan_tensor, dim3((unsigned)((scan_rows(Lt) + waves - 1) / waves)), dim3(PAIR_WG), tb, s,
                       QA, QB, L, Lt, rho, invf, rot, has_rot, q[0], q[1], q[2], q[3], T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nR <= 0) return e;
    const int64_t blocks = (nR + WG * SCAN_NP - 1) / (WG * SCAN_NP);
    hipLaunchKernelGGL(tcm_scan_eval, dim3((unsigned)blocks), dim3(WG), 0, s, T, Lt, rho, aA, aB, unchecked, R, nR,
                       U, status);
    return hipGetLastError();
}

// ------------------------------------------------------------------ forces and torques
// With a = Q^A / (f R^l), b = Q^B / (f R^l) (f = sqrt((l+m)!(l-m)!), B posed) and the
// factorial-scaled irregular harmonics I of n = R/|R| (the pair kernel's recurrences), eq. (9)
// reads U = (1/R) Re sum (-1)^{l2} a_{l1 m1} b_{l2 m2} conj(I_{l1+l2, m1+m2}).  The solid
// harmonics I_{L'M}(R)/R^{L'+1} obey unit ladders: d/dz -> -I_{L'+1,M}, (d/dx + i d/dy) ->
// I_{L'+1,M+1}, (d/dx - i d/dy) -> -I_{L'+1,M-1}, so with
//     S = sum (-1)^{l2} a b conj(I_{L'+1, M+1}),   Z = sum (-1)^{l2} a b conj(I_{L'+1, M})
// the gradient of U in R is (Re S, -Im S, -Re Z) / R^2 and the force on B is its negative.
// Rotating B about its centre by a small angle about axis k moves each moment by the
// generator J_k = (k x r).grad acting on its harmonic: J_z b_lm = i m b_lm,
// J_+ b_lm = i (l+m+1) b_{l,m+1}, J_- b_lm = i (l-m+1) b_{l,m-1} (J_x = (J_+ + J_-)/2,
// J_y = (J_+ - J_-)/(2i)); the torque on B is tau_B = -(1/R) Re sum W (J b) with
// W_{l2 m2} = sum (-1)^{l2} a conj(I_{L'M}) (U = (1/R) Re sum b W), and likewise for A with
// V_{l1 m1} = sum (-1)^{l2} b conj(I_{L'M}).
//
// All of it is evaluated in the frame where R lies along t = +-z (the pair kernel's frame:
// A and B rotated there, B's pose folded in), where I_{L'M}(t) = delta_{M0} (+-1)^{L'} L'!:
// Z keeps the M = 0 terms and S the M = -1 terms,
//     S = sum (-1)^{l2} (+-1)^{L'+1} (L'+1)! sum_{k>=0} (-1)^{k+1} (a_{l1 k} conj(b_{l2,k+1}) + conj(a_{l1,k+1}) b_{l2 k}),
// W_{l2 m2} = (-1)^{l2} sum_{l1} (+-1)^{L'} L'! a_{l1,-m2}, V_{l1 m1} = sum_{l2} (-1)^{l2} (+-1)^{L'} L'! b_{l2,-m1}:
// O(L^3) in all.  Forces and torques are rotated back to the lab frame at the end.
//
// Per-atom forces at fixed centres: with What = W / R^{l+1} (the coefficients of U in the
// moments of eq. (8) divided by f) and the factorial-scaled regular harmonics Rh of the
// atom's position about its centre (d/dz Rh_lm = Rh_{l-1,m}, (d/dx + i d/dy) Rh_lm =
// Rh_{l-1,m+1}, (d/dx - i d/dy) Rh_lm = -Rh_{l-1,m-1}), the force on atom i is
//     F_i = -q_i sum_{l' < L, m' >= 0} (Re(X Rh), Im(Y Rh), Re(Z Rh))_{l' m'},
// X = P - N, Y = P + N, Z = w_m' What_{l'+1, m'}, P = What_{l'+1, m'-1} (m' = 0:
// -conj(What_{l'+1, 1})), N = What_{l'+1, m'+1} (m' >= 1, else 0), w = 1 (m' = 0) or 2.  The
// tables hold the rotated frame's What, so the atoms are rotated into that frame (with B's
// pose) and their forces rotated back.
constexpr int FT_NSUM = 10;        // U, Z, Re S, Im S, dU/dtheta_B (3), dU/dtheta_A (3)
constexpr int ATAB_ROW = 8;        // Xr Xi Yr Yi Zr Zi c1 c2
constexpr int ATAB_HDR = 36;       // per side: position rotation [9], output rotation [9]

__host__ __device__ constexpr int nrows(int L) { return (L + 1) * (L + 2) / 2; }
__host__ __device__ constexpr int atab_rows(int L) { return L * (L + 1) / 2; }
__host__ __device__ constexpr size_t ft_smem_bytes(int Lm)
{
    // sA, sB, tA, tB [nh], spow [Lm+3], fac [2Lm+2], scsA, scsB [6(Lm+1)], qq [8], rot [9],
    // red [waves][FT_NSUM]
    return sizeof(double) * (4 * (size_t)nh(Lm) + (Lm + 3) + (2 * Lm + 2) + 12 * (Lm + 1) + 8 + 9 +
                             (PAIR_WG / 64) * FT_NSUM);
}

// Entry (l, m) of a real-packed table for any m in [-l, l] (v_{l,-m} = (-1)^m conj(v_lm)).
__device__ __forceinline__ void cget(const double* v, int l, int m, double& re, double& im)
{
    const int am = m < 0 ? -m : m;
    if (am > l) { re = 0.0; im = 0.0; return; }
    if (am == 0) { re = v[l * l]; im = 0.0; return; }
    re = v[l * l + 2 * am - 1];
    im = v[l * l + 2 * am];
    if (m < 0) {
        im = -im;
        if (am & 1) { re = -re; im = -im; }
    }
}

// (J_x v, J_y v, J_z v) at (l, m) for a real-packed table v (complex, interleaved in j[6]).
__device__ __forceinline__ void jvec(const double* v, int l, int m, double* j)
{
    double br, bi, dr, di, ur, ui;
    cget(v, l, m, br, bi);
    cget(v, l, m - 1, dr, di);
    cget(v, l, m + 1, ur, ui);
    const double cp = l + m + 1, cm = l - m + 1;
    // J_x = (i/2)(cp v_{m+1} + cm v_{m-1}),  J_y = (1/2)(cp v_{m+1} - cm v_{m-1}),  J_z = i m v
    const double sr = cp * ur + cm * dr, si = cp * ui + cm * di;
    j[0] = -0.5 * si;
    j[1] = 0.5 * sr;
    j[2] = 0.5 * (cp * ur - cm * dr);
    j[3] = 0.5 * (cp * ui - cm * di);
    j[4] = -m * bi;
    j[5] = m * br;
}

__device__ inline void quat_to_matrix(const double* q, double* M)
{
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    M[0] = 1 - 2 * (y * y + z * z); M[1] = 2 * (x * y - w * z);     M[2] = 2 * (x * z + w * y);
    M[3] = 2 * (x * y + w * z);     M[4] = 1 - 2 * (x * x + z * z); M[5] = 2 * (y * z - w * x);
    M[6] = 2 * (x * z - w * y);     M[7] = 2 * (y * z + w * x);     M[8] = 1 - 2 * (x * x + y * y);
}

// One workgroup per pair: FT[out][10] = (U, F_B, tau_A, tau_B) and the pair's status;
// wscr (when not null) gets
// What (side B) then Vhat (side A), nrows(L) complex each, for the per-atom tables atab
// (when not null: ATAB_HDR doubles of rotations, then side A then side B, atab_rows(L) rows of
// ATAB_ROW doubles each).
__device__ __forceinline__ void pair_ft_item(const DevPlan& P, int p, char* smem, double* FT, double* wscr,
                                             double* atab)
{
    const PairWork& pw = P.pairs[p];
    const int tid = threadIdx.x;
    const int L = pw.L, NHl = nh(L);
    const double Rx = pw.R[0], Ry = pw.R[1], Rz = pw.R[2];
    const double Rn = sqrt(Rx * Rx + Ry * Ry + Rz * Rz);
    const double aA = pw.metaA[3], aB = pw.metaB[3];
    double* out = FT + (size_t)FT_NSUM * pw.out;
    if (!(Rn > 0.0) || (!(pw.flags & TCM_UNCHECKED) && !(Rn > aA + aB))) {
        if (tid < FT_NSUM) out[tid] = __builtin_nan("");
        if (tid == 0) P.status[pw.out] = (Rn > 0.0) ? TCM_EDOMAIN : TCM_EINVAL;
        return;
    }
    const int Lm = P.pair_lmax;
    double* sA = reinterpret_cast<double*>(smem);
    double* sB = sA + nh(Lm);
    double* tA = sB + nh(Lm);
    double* tB = tA + nh(Lm);
    double* spow = tB + nh(Lm);              // R^-k, k <= L + 2
    double* fac = spow + (Lm + 3);           // (+-1)^k k!, k <= 2L + 1
    double* scsA = fac + (2 * Lm + 2);
    double* scsB = scsA + 6 * (Lm + 1);
    double* qq = scsB + 6 * (Lm + 1);        // frame quaternion, then B's
    double* rot = qq + 8;                    // frame rotation matrix
    double* red = rot + 9;                   // [waves][FT_NSUM]
    if (tid == 0) {
        const double ir = 1.0 / Rn;
        spow[0] = 1.0;
        for (int l = 1; l <= L + 2; ++l) spow[l] = spow[l - 1] * ir;
        const double nx = Rx * ir, ny = Ry * ir, nz = Rz * ir, sg = nz < 0.0 ? -1.0 : 1.0;
        double w = 1.0 + sg * nz, x = sg * ny, y = -sg * nx;
        const double qn = sqrt(w * w + x * x + y * y);
        w /= qn; x /= qn; y /= qn;
        qq[0] = w; qq[1] = x; qq[2] = y; qq[3] = 0.0;
        if (pw.has_rot) {
            const double* q = pw.quat;
            qq[4] = w * q[0] - x * q[1] - y * q[2];
            qq[5] = w * q[1] + x * q[0] + y * q[3];
            qq[6] = w * q[2] - x * q[3] + y * q[0];
            qq[7] = w * q[3] + x * q[2] - y * q[1];
        } else {
            qq[4] = w; qq[5] = x; qq[6] = y; qq[7] = 0.0;
        }
        quat_to_matrix(qq, rot);
        fac[0] = 1.0;
        for (int k = 1; k <= 2 * L + 1; ++k) fac[k] = fac[k - 1] * (sg * k);
    }
    __syncthreads();
    if (tid <= L) {
        euler_phases(qq, tid, Lm, scsA);
        euler_phases(qq + 4, tid, Lm, scsB);
    }
    for (int h = tid; h < NHl; h += PAIR_WG) {
        const double sc = spow[l_of(h)];
        sA[h] = pw.QA[h] * sc;
        sB[h] = pw.QB[h] * sc;
    }
    __syncthreads();
    rotate_moments2<PAIR_WG>(P.rot, sA, sB, tA, tB, L, Lm, scsA, scsB);
    for (int h = tid; h < NHl; h += PAIR_WG) {
        sA[h] *= P.invf[h];
        sB[h] *= P.invf[h];
    }
    __syncthreads();
    double acc[FT_NSUM];
    for (int k = 0; k < FT_NSUM; ++k) acc[k] = 0.0;
    const int nr = nrows(L);
    for (int r = tid; r < 2 * nr; r += PAIR_WG) {
        const bool sideB = r < nr;
        const int rr = sideB ? r : r - nr;
        int l = 0;
        while ((l + 1) * (l + 2) / 2 <= rr) ++l;
        const int m = rr - l * (l + 1) / 2;
        const double w = m == 0 ? 1.0 : 2.0;
        double j[6];
        const double sm = (m & 1) ? -1.0 : 1.0;  // v_{l,-m} = (-1)^m conj(v_{l m})
        const int om = m == 0 ? 0 : 2 * m - 1;    // offset of (Re, Im) of m in an order's block
        if (sideB) {                         // W_{l m} = (-1)^l sum_{l1 >= m} fac[l1+l] a_{l1,-m}
            double Wr = 0.0, Wi = 0.0;
            for (int l1 = m; l1 <= L; ++l1) {
                const double ar = sm * sA[l1 * l1 + om], ai = m == 0 ? 0.0 : -sm * sA[l1 * l1 + om + 1];
                Wr += fac[l1 + l] * ar;
                Wi += fac[l1 + l] * ai;
            }
            if (l & 1) { Wr = -Wr; Wi = -Wi; }
            double br, bi;
            cget(sB, l, m, br, bi);
            acc[0] += w * (br * Wr - bi * Wi);
            jvec(sB, l, m, j);
            for (int d = 0; d < 3; ++d) acc[4 + d] += w * (Wr * j[2 * d] - Wi * j[2 * d + 1]);
            if (wscr) {
                wscr[2 * rr] = Wr * spow[l + 1];
                wscr[2 * rr + 1] = Wi * spow[l + 1];
            }
        } else {                             // V_{l m} = sum_{l2 >= m} (-1)^{l2} fac[l+l2] b_{l2,-m}; Z, S rows
            double Vr = 0.0, Vi = 0.0, zr = 0.0, zi = 0.0, pr = 0.0, pi = 0.0, qr = 0.0, qi = 0.0;
            double ar, ai, ur, ui;           // a_{l m}, a_{l,m+1}
            cget(sA, l, m, ar, ai);
            cget(sA, l, m + 1, ur, ui);
            for (int l2 = m; l2 <= L; ++l2) {
                const double* bl = sB + l2 * l2;
                const double br = bl[om], bi = m == 0 ? 0.0 : bl[om + 1];     // b_{l2 m}
                const double f0 = (l2 & 1) ? -fac[l + l2] : fac[l + l2];
                const double f1 = (l2 & 1) ? -fac[l + l2 + 1] : fac[l + l2 + 1];
                Vr += f0 * (sm * br);         // b_{l2,-m}
                Vi += f0 * (-sm * bi);
                zr += f1 * br;                // sum f1 conj(b_{l2 m})
                zi -= f1 * bi;
                qr += f1 * br;                // sum f1 b_{l2 m} (for conj(a_{l,m+1}) b_{l2 m})
                qi += f1 * bi;
                if (m + 1 <= l2) {            // conj(b_{l2,m+1})
                    pr += f1 * bl[2 * m + 1];
                    pi -= f1 * bl[2 * m + 2];
                }
            }
            jvec(sA, l, m, j);
            for (int d = 0; d < 3; ++d) acc[7 + d] += w * (Vr * j[2 * d] - Vi * j[2 * d + 1]);
            const double zt = ar * zr - ai * zi;                  // Re(a_{l m} sum f1 conj(b_{l2 m}))
            acc[1] += (m & 1) ? -w * zt : w * zt;
            // S row: (-1)^{m+1} (a_{l m} sum f1 conj(b_{l2,m+1}) + conj(a_{l,m+1}) sum f1 b_{l2 m})
            double sr = ar * pr - ai * pi, si = ar * pi + ai * pr;
            sr += ur * qr + ui * qi;
            si += ur * qi - ui * qr;
            if (m & 1) { acc[2] += sr; acc[3] += si; } else { acc[2] -= sr; acc[3] -= si; }
            if (wscr) {
                wscr[2 * (nr + rr)] = Vr * spow[l + 1];
                wscr[2 * (nr + rr) + 1] = Vi * spow[l + 1];
            }
        }
    }
    for (int k = 0; k < FT_NSUM; ++k) acc[k] = wave_sum(acc[k]);
    if ((tid & 63) == 0)
        for (int k = 0; k < FT_NSUM; ++k) red[(tid >> 6) * FT_NSUM + k] = acc[k];
    __syncthreads();                         // red is in LDS: the barrier orders it (a device-scope
                                             // fence here would write back and drop the L2 per pair)
    if (tid == 0) {
        double t[FT_NSUM];
        for (int k = 0; k < FT_NSUM; ++k) {
            t[k] = 0.0;
            for (int wv = 0; wv < PAIR_WG / 64; ++wv) t[k] += red[wv * FT_NSUM + k];
        }
        const double ir = spow[1], ir2 = spow[2];
        // rotated frame: F_B = -(Re S, -Im S, -Z) / R^2, tau = -dU/dtheta / R
        const double fp[3] = {-t[2] * ir2, t[3] * ir2, t[1] * ir2};
        const double ta[3] = {-t[7] * ir, -t[8] * ir, -t[9] * ir};
        const double tb[3] = {-t[4] * ir, -t[5] * ir, -t[6] * ir};
        out[0] = t[0] * ir;
        P.status[pw.out] = TCM_OK;
        for (int d = 0; d < 3; ++d) {         // lab = rot^T rotated
            out[1 + d] = rot[d] * fp[0] + rot[3 + d] * fp[1] + rot[6 + d] * fp[2];
            out[4 + d] = rot[d] * ta[0] + rot[3 + d] * ta[1] + rot[6 + d] * ta[2];
            out[7 + d] = rot[d] * tb[0] + rot[3 + d] * tb[1] + rot[6 + d] * tb[2];
        }
        if (atab) {                          // rotations for the per-atom kernel
            double mb[9];
            quat_to_matrix(qq + 4, mb);
            for (int k = 0; k < 9; ++k) {
                atab[k] = rot[k];             // A: positions into the frame
                atab[18 + k] = mb[k];         // B: pose, then into the frame
            }
            for (int r2 = 0; r2 < 3; ++r2)
                for (int c2 = 0; c2 < 3; ++c2) {
                    atab[9 + 3 * r2 + c2] = rot[3 * c2 + r2];    // forces back: rot^T
                    atab[27 + 3 * r2 + c2] = rot[3 * c2 + r2];
                }
        }
    }
    if (!atab || !wscr || L == 0) return;
    // per-atom tables, column by column (m' = 0 .. L-1, l' = m' .. L-1)
    const int na = atab_rows(L);
    double* tabs = atab + ATAB_HDR;
    for (int e = tid; e < 2 * na; e += PAIR_WG) {
        const int side = e < na ? 0 : 1;     // 0: A (Vhat), 1: B (What)
        const int k = side ? e - na : e;
        int mp = 0;
        while ((mp + 1) * L - (mp + 1) * mp / 2 <= k) ++mp;
        const int lp = mp + (k - (mp * L - mp * (mp - 1) / 2));
        const double* Wt = wscr + (side ? 0 : 2 * nr);
        auto W = [&](int l, int mm, double& re, double& im) {   // packed rows (l, m >= 0), any m
            const int am = mm < 0 ? -mm : mm;
            if (am > l) { re = 0.0; im = 0.0; return; }
            re = Wt[2 * (l * (l + 1) / 2 + am)];
            im = Wt[2 * (l * (l + 1) / 2 + am) + 1];
            if (mm < 0) {
                im = -im;
                if (am & 1) { re = -re; im = -im; }
            }
        };
        double Pr, Pi, Nr = 0.0, Ni = 0.0, Zr, Zi;
        W(lp + 1, mp - 1, Pr, Pi);
        if (mp >= 1) W(lp + 1, mp + 1, Nr, Ni);
        W(lp + 1, mp, Zr, Zi);
        const double wz = mp == 0 ? 1.0 : 2.0;
        double* row = tabs + (size_t)ATAB_ROW * (side * na + k);
        row[0] = Pr - Nr;
        row[1] = Pi - Ni;
        row[2] = Pr + Nr;
        row[3] = Pi + Ni;
        row[4] = wz * Zr;
        row[5] = wz * Zi;
        if (lp == mp) {                      // diagonal: Rh_mm = -(x + i y)/(2m) Rh_{m-1,m-1}
            row[6] = 0.0;
            row[7] = mp > 0 ? -1.0 / (2.0 * mp) : 0.0;
        } else {                             // Rh_lm = ((2l-1) z Rh_{l-1} - r^2 Rh_{l-2}) / ((l+m)(l-m))
            const double den = (double)(lp + mp) * (lp - mp);
            row[6] = (2.0 * lp - 1.0) / den;
            row[7] = 1.0 / den;
        }
    }
}

// F[i][3] = -q_i sum over the table rows of (Re(X Rh), Im(Y Rh), Re(Z Rh)) with Rh the
// factorial-scaled regular harmonics of M (x_i - c), rotated back by M's second half.  A
// workgroup takes 64 atoms; its four wavefronts split the m columns (column m holds L - m rows)
// in snake order (waves 0 1 2 3 3 2 1 0 0 1 ...), each following the diagonal recurrence up to
// its last column, and the four partial sums are added in wave order.  The table rows are the
// same for every lane (scalar loads).
__global__ __launch_bounds__(WG) void tcm_atom_forces(const double* __restrict__ T, int L,
                                                      const double* __restrict__ X, const double* __restrict__ Y,
                                                      const double* __restrict__ Zc, const double* __restrict__ Q,
                                                      int64_t n, const double* __restrict__ centre,
                                                      const double* __restrict__ mats, double* __restrict__ F)
{
    __shared__ double part[WG / 64][3][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar table loads
    const int64_t k = blockIdx.x * (int64_t)64 + lane;
    const bool live = k < n;
    using crow = const __attribute__((address_space(4))) double*;
    crow M = (crow)mats;                     // [9] into the table's frame, [9] back to the lab
    const int64_t kk = live ? k : 0;
    const double dx = X[kk] - centre[0], dy = Y[kk] - centre[1], dz = Zc[kk] - centre[2];
    const double x = M[0] * dx + M[1] * dy + M[2] * dz;
    const double y = M[3] * dx + M[4] * dy + M[5] * dz;
    const double z = M[6] * dx + M[7] * dy + M[8] * dz;
    const double r2 = x * x + y * y + z * z;
    crow tab = (crow)T;
    double fx = 0.0, fy = 0.0, fz = 0.0, dr = 1.0, di = 0.0;       // Rh_mm
    for (int m = 0; m < L; ++m) {
        crow row = tab + (size_t)ATAB_ROW * (m * L - m * (m - 1) / 2);   // column m's diagonal row
        if (m > 0) {
            const double c2 = row[7];
            const double tr = (x * dr - y * di) * c2;
            di = (x * di + y * dr) * c2;
            dr = tr;
        }
        const int g = m % 8;
        if ((g < 4 ? g : 7 - g) != wave) continue;
        double p1r = dr, p1i = di, p2r = 0.0, p2i = 0.0;
        fx += row[0] * p1r - row[1] * p1i;
        fy += row[2] * p1i + row[3] * p1r;
        fz += row[4] * p1r - row[5] * p1i;
        row += ATAB_ROW;
        for (int l = m + 1; l < L; ++l, row += ATAB_ROW) {
            const double a = row[6] * z, b = row[7] * r2;
            const double pr = a * p1r - b * p2r, pi = a * p1i - b * p2i;
            p2r = p1r; p2i = p1i; p1r = pr; p1i = pi;
            fx += row[0] * pr - row[1] * pi;
            fy += row[2] * pi + row[3] * pr;
            fz += row[4] * pr - row[5] * pi;
        }
    }
    part[wave][0][lane] = fx;
    part[wave][1][lane] = fy;
    part[wave][2][lane] = fz;
    __syncthreads();
    if (wave == 0 && live) {
        double f[3];
        for (int d = 0; d < 3; ++d) f[d] = ((part[0][d][lane] + part[1][d][lane]) + part[2][d][lane]) + part[3][d][lane];
        const double q = -Q[k];
        F[3 * k] = q * (M[9] * f[0] + M[10] * f[1] + M[11] * f[2]);
        F[3 * k + 1] = q * (M[12] * f[0] + M[13] * f[1] + M[14] * f[2]);
        F[3 * k + 2] = q * (M[15] * f[0] + M[16] * f[1] + M[17] * f[2]);
    }
}

// ------------------------------------------------------------------ kernels
// One workgroup per item (the grid is the item count): no claim counters, the hardware
// dispatcher balances the items; the steps of a run are ordered by launch boundaries only
// (no device-side waits).
__global__ __launch_bounds__(WG) void tcm_stats(DevPlan P, int begin, int end)
{
    __shared__ __align__(16) char smem[9 * (WG / 64) * sizeof(double)];
    const int item = begin + (int)blockIdx.x;
    if (item >= end) return;
    const int mol = __builtin_amdgcn_readfirstlane(P.stats_items[2 * item]);
    const int k = __builtin_amdgcn_readfirstlane(P.stats_items[2 * item + 1]);
    const MolWork& mw = P.mols[mol];
    // one chunk per item unless the molecule has more chunks than the planner's item cap
    if ((mw.n + STATS_CHUNK - 1) / STATS_CHUNK <= mw.nstats)
        stats_item(P, mol, k, smem);
    else
        stats_run(P, mol, k, smem);
}

__global__ __launch_bounds__(WG) void tcm_stats_finalize(DevPlan P, int mol_begin, int mol_end)
{
    __shared__ __align__(16) char smem[9 * WG * sizeof(double)];
    const int mol = mol_begin + (int)blockIdx.x;
    if (mol < mol_end) stats_finalize(P, mol, smem);
}

__global__ __launch_bounds__(WG) void tcm_moments_finalize(DevPlan P)
{
    __shared__ __align__(16) double smem[(LMAX + 2) + WG];
    if ((int)blockIdx.x < P.nmol) finalize_moments(P, blockIdx.x, reinterpret_cast<char*>(smem));
}


// Calibration of the vector ALU: 16 independent FMA chains per thread (a = a * b + c), so the
// sustained rate of plain (non-packed) FMA instructions is measured without latency limits.
template <typename T>
__global__ __launch_bounds__(WG) void tcm_alu_probe(T* out, int iters, T b, T c)
{
    T a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = (T)(threadIdx.x + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) a[k] = a[k] * b + c;
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += a[k];
    out[blockIdx.x * (int64_t)WG + threadIdx.x] = s;
}

hipError_t launch_alu_probe(int prec, void* out, int blocks, int iters, hipStream_t s)
{
    if (prec == 1)
        hipLaunchKernelGGL(tcm_alu_probe<float>, dim3(blocks), dim3(WG), 0, s, (float*)out, iters, 0.999f, 0.001f);
    else
        hipLaunchKernelGGL(tcm_alu_probe<double>, dim3(blocks), dim3(WG), 0, s, (double*)out, iters, 0.999, 0.001);
    return hipGetLastError();
}

// out[0] = sum |q_i| over n charges: one workgroup, each thread a strided subset in index
// order, then a fixed-order tree (the same value on every run).
__global__ __launch_bounds__(WG) void tcm_abs_sum(const double* q, int64_t n, double* out)
{
    __shared__ double red[WG];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += WG) a += fabs(q[i]);
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = WG / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

hipError_t launch_abs_sum(const double* q, int64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(tcm_abs_sum, dim3(1), dim3(WG), 0, s, q, n, out);
    return hipGetLastError();
}

// dst[k][0..7] = src[k][0..7] for k < K (one thread per value): the per-molecule records of
// many molecules gathered for one read-back.
__global__ __launch_bounds__(WG) void tcm_gather8(const double* const* src, int64_t K, double* dst)
{
    const int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x;
    if (i < 8 * K) dst[i] = src[i >> 3][i & 7];
}

hipError_t launch_gather8(const double* const* src, int64_t K, double* dst, hipStream_t s)
{
    if (K <= 0) return hipSuccess;
    const int64_t blocks = (8 * K + WG - 1) / WG;
    hipLaunchKernelGGL(tcm_gather8, dim3((unsigned)blocks), dim3(WG), 0, s, src, K, dst);
    return hipGetLastError();
}

__global__ __launch_bounds__(PAIR_WG) void tcm_pairs_ft(DevPlan P, int begin, int end, double* FT, double* wscr,
                                                        double* atab)
{
    extern __shared__ __align__(16) char smem[];         // ft_smem_bytes(P.pair_lmax)
    const int item = begin + (int)blockIdx.x;
    if (item < end) pair_ft_item(P, item, smem, FT, wscr, atab);
}

// Clears the run's device-side flags (a kernel, not a memset, so that it can sit in a
// captured graph).
__global__ void tcm_clear(int32_t* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <typename F>
struct NumBlocksTable {
    int v[LMAX + 1];
    constexpr NumBlocksTable() : v()
    {
        for (int L = 0; L <= LMAX; ++L) v[L] = num_blocks(L, sizeof(F) == 4 ? BUDGET_F32 : BUDGET_F64);
    }
};

int num_blocks_for(int prec, int L)
{
    static constexpr NumBlocksTable<float> t32{};
    static constexpr NumBlocksTable<double> t64{};
    if (L < 0 || L > LMAX) return 0;
    return prec == TCM_F32C ? t32.v[L] : t64.v[L];
}

hipError_t launch_clear(int32_t* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int grid = (int)((n + 255) / 256);
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(tcm_clear, dim3(grid), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_stats(const DevPlan& P, int begin, int end, hipStream_t s)
{
    if (end <= begin) return hipSuccess;
    hipLaunchKernelGGL(tcm_stats, dim3(end - begin), dim3(WG), 0, s, P, begin, end);
    return hipGetLastError();
}

hipError_t launch_stats_finalize(const DevPlan& P, int mol_begin, int mol_end, hipStream_t s)
{
    if (mol_end <= mol_begin) return hipSuccess;
    hipLaunchKernelGGL(tcm_stats_finalize, dim3(mol_end - mol_begin), dim3(WG), 0, s, P, mol_begin, mol_end);
    return hipGetLastError();
}

hipError_t launch_moments_finalize(const DevPlan& P, hipStream_t s)
{
    if (P.nmol <= 0) return hipSuccess;
    hipLaunchKernelGGL(tcm_moments_finalize, dim3(P.nmol), dim3(WG), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_pairs_ft(const DevPlan& P, int begin, int end, double* FT, double* wscr, double* atab,
                           hipStream_t s)
{
    if (end <= begin) return hipSuccess;
    hipLaunchKernelGGL(tcm_pairs_ft, dim3(end - begin), dim3(PAIR_WG), ft_smem_bytes(P.pair_lmax), s, P, begin, end,
                       FT, wscr, atab);
    return hipGetLastError();
}

hipError_t launch_atom_forces(const double* atab, int side, int L, const double* x, const double* y, const double* z,
                              const double* q, int64_t n, const double* centre, double* F, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 63) / 64;    // 64 atoms per workgroup
    const double* T = atab + ATAB_HDR + (size_t)ATAB_ROW * atab_rows(L) * side;
    hipLaunchKernelGGL(tcm_atom_forces, dim3((unsigned)blocks), dim3(WG), 0, s, T, L, x, y, z, q, n, centre,
                       atab + 18 * side, F);
    return hipGetLastError();
}

// The pairs [begin, end) of the plan (listed by decreasing order): rotation, per-m terms,
// final sums (three launches, ordered on s).
hipError_t launch_pairs(const DevPlan& P, int begin, int end, hipStream_t s)
{
    if (end <= begin) return hipSuccess;
    const int Lm = P.pair_lmax;
    const unsigned groups = (unsigned)((end - begin + PAIR_LANES - 1) / PAIR_LANES);
    const size_t rot_lds = sizeof(double) * (2 * (size_t)Lm + 1 + ROT_PAD) * PAIR_LANES;
    hipError_t e;
    if (Lm <= 16)
        hipLaunchKernelGGL(tcm_pairs_rot<16>, dim3(groups, Lm + 1, 2), dim3(PAIR_LANES, ROT_WAVES), rot_lds, s, P,
                           begin, end);
    else
        hipLaunchKernelGGL(tcm_pairs_rot<LMAX>, dim3(groups, Lm + 1, 2), dim3(PAIR_LANES, ROT_WAVES), rot_lds, s, P,
                           begin, end);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (Lm <= 16) {
        hipLaunchKernelGGL(tcm_pairs_sum_w<17>, dim3(groups, Lm + 1), dim3(PAIR_LANES), 0, s, P, begin, end);
    } else if (Lm <= SW_L) {
        hipLaunchKernelGGL(tcm_pairs_sum_w<25>, dim3(groups, Lm + 1), dim3(PAIR_LANES), 0, s, P, begin, end);
    } else {
        const size_t sum_lds = sizeof(double) * (2 * LMAX + 2 + 4 * ((size_t)Lm + 1) * PAIR_LANES);
        hipLaunchKernelGGL(tcm_pairs_sum_m, dim3(groups, Lm + 1), dim3(PAIR_LANES, PAIR_WAVES), sum_lds, s, P, begin,
                           end);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const dim3 fg((unsigned)((end - begin + PAIR_LANES - 1) / PAIR_LANES));
    if (Lm <= 16)
        hipLaunchKernelGGL(tcm_pairs_final<17>, fg, dim3(PAIR_LANES), 0, s, P, begin, end);
    else if (Lm <= SW_L)
        hipLaunchKernelGGL(tcm_pairs_final<SW_L + 1>, fg, dim3(PAIR_LANES), 0, s, P, begin, end);
    else
        hipLaunchKernelGGL(tcm_pairs_final<LMAX + 1>, fg, dim3(PAIR_LANES), 0, s, P, begin, end);
    return hipGetLastError();
}

hipError_t launch_pairs_choose(const DevPlan& P, int begin, int end, double tol, int32_t* Lout, double* bout,
                               hipStream_t s)
{
    if (end <= begin) return hipSuccess;
    hipLaunchKernelGGL(tcm_pairs_choose, dim3((unsigned)((end - begin + WG - 1) / WG)), dim3(WG), 0, s, P, begin, end,
                       tol, Lout, bout);
    return hipGetLastError();
}

hipError_t launch_pairs_regroup(const DevPlan& P, int npairs, const int32_t* Lc, int32_t* cnt, PairWork* pairs2,
                                double* frame2, int32_t* gorder2, hipStream_t s)
{
    if (npairs <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((npairs + WG - 1) / WG);
    hipError_t e;
    if ((e = launch_clear(cnt, 2 * (LMAX + 1), s)) != hipSuccess) return e;
    hipLaunchKernelGGL(tcm_pairs_count, dim3(grid), dim3(WG), 0, s, P, npairs, Lc, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(tcm_pairs_regroup, dim3(grid), dim3(WG), 0, s, P, npairs, Lc, cnt, pairs2, frame2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int groups = (npairs + PAIR_LANES - 1) / PAIR_LANES;
    hipLaunchKernelGGL(tcm_pairs_group_orders, dim3((unsigned)((groups + WG - 1) / WG)), dim3(WG), 0, s, pairs2,
                       npairs, gorder2);
    return hipGetLastError();
}

hipError_t launch_tiles_f32_a(int L, const DevPlan& P, int begin, int end, hipStream_t s);
hipError_t launch_tiles_f32_b(int L, const DevPlan& P, int begin, int end, hipStream_t s);
hipError_t launch_tiles_f32_c(int L, const DevPlan& P, int begin, int end, hipStream_t s);
hipError_t launch_tiles_f32_d(int L, const DevPlan& P, int begin, int end, hipStream_t s);
hipError_t launch_tiles_f64_a(int L, const DevPlan& P, int begin, int end, hipStream_t s);
hipError_t launch_tiles_f64_b(int L, const DevPlan& P, int begin, int end, hipStream_t s);
hipError_t launch_tiles_f64_c(int L, const DevPlan& P, int begin, int end, hipStream_t s);
hipError_t launch_tiles_f64_d(int L, const DevPlan& P, int begin, int end, hipStream_t s);

hipError_t launch_tiles(int prec, int L, const DevPlan& P, int begin, int end, hipStream_t s)
{
    if (end <= begin) return hipSuccess;
    if (prec == TCM_F32C) {
        if (L <= 12) return launch_tiles_f32_a(L, P, begin, end, s);
        if (L <= 20) return launch_tiles_f32_b(L, P, begin, end, s);
        if (L <= 26) return launch_tiles_f32_c(L, P, begin, end, s);
        return launch_tiles_f32_d(L, P, begin, end, s);
    }
    if (L <= 12) return launch_tiles_f64_a(L, P, begin, end, s);
    if (L <= 20) return launch_tiles_f64_b(L, P, begin, end, s);
    if (L <= 26) return launch_tiles_f64_c(L, P, begin, end, s);
    return launch_tiles_f64_d(L, P, begin, end, s);
}

}  // namespace tcm
