// Internal definitions shared by the HIP kernels and the host runtime of libtcm.
//
// Work decomposition of one batch: a sequence of launches, ordered by launch boundaries, each
// with one workgroup per item
//   a0 STATS      (molecule, chunk)         centroid sums + bounding box of a chunk of atoms
//      STATS_FIN  (molecule)                centre and scale of each molecule
//   a1 TILE       (molecule, tile, m-block) eq. (8) moments of 256*kper atoms for one m-block;
//                                            one launch per (precision, L) group
//   a2 MOM_FIN    (molecule)                fixed-order merge of the tile partials, unscaling
//   a3-a5 PAIR    (pair)                    rotation, geometric factors, eq. (9) contraction
// A plan's launches are captured once into a HIP graph and replayed, or issued directly with
// each (precision, L) group on a stream of its own.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tcm {

constexpr int LMAX = 32;           // largest multipole order the library accepts
constexpr int WG = 256;            // threads per workgroup (4 wave64s)
constexpr int STATS_PER_THREAD = 8;
constexpr int STATS_CHUNK = WG * STATS_PER_THREAD;   // atoms per STATS item

__host__ __device__ constexpr int nh(int L) { return (L + 1) * (L + 1); }

// Per molecule whose moments are computed in this batch.
struct MolWork {
    const double* x;               // FP64 SoA coordinates and charges (device)
    const double* y;
    const double* z;
    const double* q;
    int64_t n;
    int32_t L;                     // order computed (moment table (L+1)^2)
    int32_t prec;                  // 0 = FP64 path, 1 = FP32 compensated path
    int32_t kper;                  // atoms per thread per tile
    int32_t nblk;                  // m-blocks for (prec, L)
    int32_t ntiles;
    int32_t nstats;
    int32_t has_centre;
    int32_t pad0;
    double centre[3];              // used when has_centre
    double* Q;                     // out: (L+1)^2 FP64 packed moments
    double* meta;                  // out: [0..2] centre, [3] radius, [4] scale
    int64_t part_off;              // element offset of the tile partials
    int64_t stats_off;             // record offset of the STATS partials (10 doubles each)
    int64_t r2_off;                // offset of the per-tile max |r|^2 partials
};

// Per requested pair energy.
struct PairWork {
    const double* QA;              // packed FP64 moments, order >= L
    const double* QB;
    const double* metaA;           // meta[3] = radius of A (eq. (2))
    const double* metaB;
    int32_t depA;                  // molecule index in this batch to wait for, or -1
    int32_t depB;
    int32_t L;
    int32_t flags;                 // TCM_UNCHECKED skips the eq. (2) test
    double R[3];                   // c_B - c_A
    double quat[4];                // active rotation of B about c_B, (w, x, y, z)
    int32_t has_rot;
    int32_t out;                   // index into U / status
};

struct DevPlan {
    const MolWork* mols;
    const PairWork* pairs;
    const int32_t* stats_items;    // [n_stats][2]: (molecule, chunk) of each STATS item
    const int32_t* tile_items;     // [n_tiles][2]: (molecule, tile * nblk + m-block) of each
                                   // TILE item, each group's items in decreasing cost
    int32_t nmol;
    int32_t npairs;                // pairs are listed in decreasing cost (largest L first)
    int32_t pair_lmax;             // largest L of the pairs (sizes the pair kernel's LDS)
    int32_t pad1;
    int32_t n_stats;
    int32_t n_tiles;
    int32_t* err;                  // [1] device-side error flag (reserved), cleared before each run
    // scratch
    float* part_f;                 // FP32 path tile partials (hi block, then lo block)
    double* part_d;                // FP64 path tile partials
    double* stats_part;            // STATS partials, 10 doubles per item
    double* r2_part;               // per-tile max |r|^2 (FP64)
    double* prot;                  // pair launches: rotated moments [2][nh(pair_lmax)][npairs]
    double* pum;                   // pair launches: per-m partial energies [pair_lmax+1][npairs], then
                                   // per pair |R| or its failure status (a negative code)
    // outputs
    double* U;
    int32_t* status;
    // FP64 coefficient tables (device)
    const double* invk;            // 1/k_lm of the normalised recurrence, per packed index
    const double* invf;            // 1/sqrt((l+m)!(l-m)!), per packed index
    const double* rot;             // rotation tables (D and D^{-1} per l, compressed by sparsity)
    const double* rotr;            // the same, row by row (rot + rot_tables_len())
    const double* fact;            // k!, k < FACT_N
    const double* frame;           // per pair and side, [2][FRAME_N][npairs]: see side_frame
    int32_t* gorder;               // largest order of each group of PAIR_LANES pairs
    int32_t gorder_uniform;        // 1: every group's largest order is pair_lmax (gorder not read)
    const double* qa_all;          // the A (B) table of every pair of the launch when they share
    const double* qb_all;          // one (its order is then at least pair_lmax), else null
};

// The first column of the rotation-table rows of one class: a 90 degree rotation about x maps
// the real functions of one type (cos, sin) and m parity onto one type and parity, whose
// packed columns are max(0, jb + 4k).  Row of type sin_row and order m at degree l: jb = 2p - 1
// when m and l have the same parity, else 2 (p = 1) or 4 (p = 0), with p = l mod 2 for cos rows
// and (l + 1) mod 2 for sin rows.  The table builder checks every row against it.
__host__ __device__ constexpr int rot_class_jb(bool sin_row, int m, int l)
{
    const bool same = ((m ^ l) & 1) == 0;
    const int p = sin_row ? ((l + 1) & 1) : (l & 1);
    return same ? 2 * p - 1 : (p ? 2 : 4);
}

// Entries of the device factorial table (k! for k < FACT_N; the register contraction reads up
// to (2 L + 2 (N - 1))! with N - 1 >= L, the entries past (2 L)! only against zero moments).
constexpr int FACT_N = 128;

// Pair launches take the pairs PAIR_LANES at a time, one pair per lane of a wavefront.
constexpr int PAIR_LANES = 64;
constexpr int PAIR_WAVES = 4;      // wavefronts of a pair workgroup (threadIdx.y)

// Frame of one side of a pair for the axial form of eq. (9): the rotation that takes R/|R| to
// s z (s = the sign of R_z; side 1: applied after B's pose, the pose first), as e^{i gamma},
// e^{i beta}, e^{i alpha} of its ZYZ Euler angles (rotation = Rz(alpha) Ry(beta) Rz(gamma)),
// then 1/|R| and s.  No angles are formed: the shortest rotation taking n = R/|R| to s z is the
// quaternion (1 + s n_z, s n_y, -s n_x, 0) normalised; for a unit quaternion (w, x, y, z) with
// r1 = |(w, z)| and r2 = |(x, y)|, e^{i a+} = (w + i z)/r1 and e^{i a-} = (y - i x)/r2 (the angle
// taken as 0 when its modulus vanishes), gamma = a+ - a-, alpha = a+ + a-, and
// e^{i beta} = (r1 + i r2)^2 / (r1^2 + r2^2).  Computed by the host when a plan is built.
constexpr int FRAME_N = 8;
__host__ __device__ inline void side_frame(const double R[3], const double quat[4], bool pose, double f[FRAME_N])
{
    const double Rn = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    const double ir = Rn > 0.0 ? 1.0 / Rn : 0.0;
    const double nx = R[0] * ir, ny = R[1] * ir, nz = R[2] * ir;
    const double sg = nz < 0.0 ? -1.0 : 1.0;
    double w = 1.0 + sg * nz, x = sg * ny, y = -sg * nx, z = 0.0;
    const double qn = sqrt(w * w + x * x + y * y);
    w /= qn; x /= qn; y /= qn;
    if (pose) {                                  // frame * pose
        const double a = w * quat[0] - x * quat[1] - y * quat[2];
        const double b = w * quat[1] + x * quat[0] + y * quat[3];
        const double c = w * quat[2] - x * quat[3] + y * quat[0];
        const double d = w * quat[3] + x * quat[2] - y * quat[1];
        const double pn = sqrt(a * a + b * b + c * c + d * d);
        w = a / pn; x = b / pn; y = c / pn; z = d / pn;
    }
    const double r1 = sqrt(w * w + z * z), r2 = sqrt(x * x + y * y);
    double pc = 1.0, ps = 0.0, mc = 1.0, ms = 0.0;
    if (r1 > 0.0) { pc = w / r1; ps = z / r1; }
    if (r2 > 0.0) { mc = y / r2; ms = -x / r2; }
    const double rr = r1 * r1 + r2 * r2;
    f[0] = pc * mc + ps * ms; f[1] = ps * mc - pc * ms;          // gamma
    f[2] = (r1 * r1 - r2 * r2) / rr; f[3] = 2.0 * r1 * r2 / rr;    // beta
    f[4] = pc * mc - ps * ms; f[5] = ps * mc + pc * ms;          // alpha
    f[6] = ir;
    f[7] = sg;
}

// Packed index helpers (layout of every moment table at the boundary):
//   m = 0: l*l ; m > 0: Re at l*l + 2m - 1, Im at l*l + 2m.
__host__ __device__ inline int l_of(int h)
{
    int l = (int)sqrtf((float)h);             // exact after the corrections (h <= 2^24)
    if (l * l > h) --l;
    if ((l + 1) * (l + 1) <= h) ++l;
    return l;
}

// Offset of order l's block in the rotation tables: a header of LMAX + 1 offsets, then per
// order l' (n = 2l'+1, K = l'/2 + 1 value slots per row) 2n row codes and 2Kn values, i.e.
// sum_{l' < l} 2 (2l'+1)(l'/2 + 2) after the header, in closed form.
__host__ __device__ constexpr int rot_block_offset(int l)
{
    const int p = l / 2;                       // pairs of orders (2a, 2a+1), a < p
    int s = 16 * (p - 1) * p * (2 * p - 1) / 6 + 20 * p * (p - 1) + 16 * p;
    if (l & 1) s += 8 * p * p + 18 * p + 4;    // the even order 2p
    return (LMAX + 1) + s;
}

// Doubles of order l's block in the rotation tables (2n row codes, 2Kn values), and of the
// tables for all orders.  The device copy holds the tables twice: slot by slot as described
// above, then row by row (same header and block offsets; in block l, row i of D at i (K+1) and
// row i of D^{-1} at (n + i)(K+1), each the row's code followed by its K values, zero past its
// count), the layout the pair launches read with scalar loads.
__host__ __device__ constexpr int rot_block_len(int l) { return 2 * (2 * l + 1) * (l / 2 + 2); }
__host__ __device__ constexpr int rot_tables_len() { return rot_block_offset(LMAX + 1); }

// m-block partition of the (l, m >= 0) harmonics for the moment tile.  Accumulator cost
// of the m-chain is (L-m+1) values (times 2 for m > 0: real and imaginary parts).
__host__ __device__ constexpr int chain_cost(int L, int m) { return (L - m + 1) * (m > 0 ? 2 : 1); }

__host__ __device__ constexpr int total_cost(int L)
{
    int t = 0;
    for (int m = 0; m <= L; ++m) t += chain_cost(L, m);
    return t;
}

// Partition of m = 0..L into contiguous m-blocks so that no block holds more than `budget`
// accumulators; each block takes up to an even share of the remaining cost.
struct Partition {
    int nb;
    int start[LMAX + 2];
};

__host__ __device__ constexpr Partition make_partition(int L, int budget)
{
    Partition p{};
    const int total = total_cost(L);
    for (int nb = (total + budget - 1) / budget;; ++nb) {
        int m = 0, blk = 0, remaining = total;
        bool ok = true;
        while (m <= L) {
            if (blk == nb) { ok = false; break; }
            p.start[blk] = m;
            int share = (remaining + (nb - blk) - 1) / (nb - blk);
            if (share > budget) share = budget;
            int used = 0;
            const int m0 = m;
            while (m <= L && (m == m0 || used + chain_cost(L, m) <= share)) {
                used += chain_cost(L, m);
                ++m;
            }
            if (used > budget) ok = false;
            remaining -= used;
            ++blk;
        }
        if (ok) {
            p.nb = blk;
            p.start[blk] = L + 1;
            return p;
        }
    }
}

__host__ __device__ constexpr int num_blocks(int L, int budget) { return make_partition(L, budget).nb; }
__host__ __device__ constexpr int block_start(int L, int budget, int b) { return make_partition(L, budget).start[b]; }

constexpr int BUDGET_F32 = 160;    // FP32 accumulators per thread per m-block
constexpr int BUDGET_F64 = 64;     // FP64 accumulators per thread per m-block

}  // namespace tcm
