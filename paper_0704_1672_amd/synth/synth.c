/*
 * synth.c -- deterministic synthetic inputs for the two-centre multipole workloads.
 *
 * This module holds no arithmetic of the multipole method itself (no harmonics, moments
 * or energies): only random numbers and the geometry recipes that place point charges.
 * Both the FP64 oracle and the HIP path read its output, so neither side generates
 * its own inputs.
 *
 * Random numbers: xoshiro256** seeded through splitmix64 (Blackman and Vigna's published
 * definitions).  A stream is identified by (seed, stream); streams are independent of
 * thread scheduling, so a batch of fragments generated in parallel is reproducible.
 *   uniform  : 53-bit doubles in [0, 1)
 *   normal   : Box-Muller
 *   ball     : direction = normalised triple of normals, radius = R U^{1/3}
 *   chain    : 3-D random walk with fixed step, excluded volume checked with a hashed cell
 *              list (cell edge = exclusion radius) against every earlier bead except the
 *              predecessor; up to max_trials trials per step, after which the last trial
 *              is accepted and counted as a violation
 *   quat     : uniform on S^3 (Shoemake's subgroup algorithm)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x)
{
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t xoshiro_next(rng_t *r)
{
    uint64_t *s = r->s;
    uint64_t result = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
}

static void rng_init(rng_t *r, uint64_t seed, uint64_t stream)
{
    uint64_t x = seed ^ (0xd1b54a32d192ed03ULL * (stream + 1));
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}

static double uni(rng_t *r) { return (double)(xoshiro_next(r) >> 11) * 0x1.0p-53; }

/* Box-Muller, one normal per call (the second is discarded to keep streams simple). */
static double nrm(rng_t *r)
{
    double u1 = 1.0 - uni(r); /* (0, 1] */
    double u2 = uni(r);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

static void unit_vec(rng_t *r, double *v)
{
    for (;;) {
        double a = nrm(r), b = nrm(r), c = nrm(r);
        double s = sqrt(a * a + b * b + c * c);
        if (s > 1e-12) { v[0] = a / s; v[1] = b / s; v[2] = c / s; return; }
    }
}

/* ---- exported scalar streams ------------------------------------------------- */
void synth_uniform(uint64_t seed, uint64_t stream, int64_t n, double lo, double hi, double *out)
{
    rng_t r; rng_init(&r, seed, stream);
    for (int64_t i = 0; i < n; ++i) out[i] = lo + (hi - lo) * uni(&r);
}

void synth_normal(uint64_t seed, uint64_t stream, int64_t n, double mu, double sigma, double *out)
{
    rng_t r; rng_init(&r, seed, stream);
    for (int64_t i = 0; i < n; ++i) out[i] = mu + sigma * nrm(&r);
}

void synth_unit_vectors(uint64_t seed, uint64_t stream, int64_t n, double *out)
{
    rng_t r; rng_init(&r, seed, stream);
    for (int64_t i = 0; i < n; ++i) unit_vec(&r, out + 3 * i);
}

/* Unit quaternions (w, x, y, z) uniform on S^3. */
void synth_quaternions(uint64_t seed, uint64_t stream, int64_t n, double *out)
{
    rng_t r; rng_init(&r, seed, stream);
    for (int64_t i = 0; i < n; ++i) {
        double u1 = uni(&r), u2 = uni(&r), u3 = uni(&r);
        double a = sqrt(1.0 - u1), b = sqrt(u1);
        out[4 * i + 0] = b * cos(2.0 * M_PI * u3);
        out[4 * i + 1] = a * sin(2.0 * M_PI * u2);
        out[4 * i + 2] = a * cos(2.0 * M_PI * u2);
        out[4 * i + 3] = b * sin(2.0 * M_PI * u3);
    }
}

/* n points uniform in a ball of radius R about c; charges uniform in [qlo, qhi]. */
void synth_ball(uint64_t seed, uint64_t stream, int64_t n, double R, const double *c,
                double qlo, double qhi, double *xyz, double *q)
{
    rng_t r; rng_init(&r, seed, stream);
    for (int64_t i = 0; i < n; ++i) {
        double v[3];
        unit_vec(&r, v);
        double rad = R * cbrt(uni(&r));
        for (int d = 0; d < 3; ++d) xyz[3 * i + d] = c[d] + rad * v[d];
        q[i] = qlo + (qhi - qlo) * uni(&r);
    }
}

/* ---- excluded-volume random-walk chain --------------------------------------- */
typedef struct {
    int64_t *key_x, *key_y, *key_z;  /* cell coordinates, INT64_MIN = empty slot */
    int64_t *head;                   /* first bead in the cell */
    uint64_t mask;
} cellmap_t;

static uint64_t cell_hash(int64_t x, int64_t y, int64_t z)
{
    uint64_t h = (uint64_t)x * 0x9e3779b97f4a7c15ULL ^ (uint64_t)y * 0xc2b2ae3d27d4eb4fULL ^
                 (uint64_t)z * 0x165667b19e3779f9ULL;
    h ^= h >> 29;
    return h * 0xbf58476d1ce4e5b9ULL;
}

static int64_t *cell_slot(cellmap_t *m, int64_t x, int64_t y, int64_t z, int create)
{
    uint64_t i = cell_hash(x, y, z) & m->mask;
    for (;;) {
        if (m->key_x[i] == INT64_MIN) {
            if (!create) return NULL;
            m->key_x[i] = x; m->key_y[i] = y; m->key_z[i] = z; m->head[i] = -1;
            return &m->head[i];
        }
        if (m->key_x[i] == x && m->key_y[i] == y && m->key_z[i] == z) return &m->head[i];
        i = (i + 1) & m->mask;
    }
}

/* Returns the number of steps whose excluded-volume check failed every trial, or -1 on
 * allocation failure.  Beads start at the origin; charges N(0, sigma) with the mean
 * subtracted (net charge zero in FP64). */
int64_t synth_chain(uint64_t seed, uint64_t stream, int64_t n, double step, double excl,
                    int max_trials, double sigma, double *xyz, double *q)
{
    if (n <= 0) return 0;
    rng_t r; rng_init(&r, seed, stream);
    uint64_t cap = 16;
    while (cap < (uint64_t)n * 2) cap <<= 1;
    cellmap_t m;
    m.mask = cap - 1;
    m.key_x = (int64_t *)malloc(cap * sizeof(int64_t));
    m.key_y = (int64_t *)malloc(cap * sizeof(int64_t));
    m.key_z = (int64_t *)malloc(cap * sizeof(int64_t));
    m.head = (int64_t *)malloc(cap * sizeof(int64_t));
    int64_t *next = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!m.key_x || !m.key_y || !m.key_z || !m.head || !next) {
        free(m.key_x); free(m.key_y); free(m.key_z); free(m.head); free(next);
        return -1;
    }
    for (uint64_t i = 0; i < cap; ++i) m.key_x[i] = INT64_MIN;
    const double inv = 1.0 / excl, ex2 = excl * excl;
    int64_t violations = 0;
    xyz[0] = xyz[1] = xyz[2] = 0.0;
    {
        int64_t *h = cell_slot(&m, 0, 0, 0, 1);
        next[0] = *h; *h = 0;
    }
    for (int64_t i = 1; i < n; ++i) {
        double cand[3] = {xyz[3 * (i - 1)], xyz[3 * (i - 1) + 1], xyz[3 * (i - 1) + 2]};
        int ok = 0;
        for (int t = 0; t < max_trials && !ok; ++t) {
            double v[3];
            unit_vec(&r, v);
            for (int d = 0; d < 3; ++d) cand[d] = xyz[3 * (i - 1) + d] + step * v[d];
            int64_t cx = (int64_t)floor(cand[0] * inv), cy = (int64_t)floor(cand[1] * inv),
                    cz = (int64_t)floor(cand[2] * inv);
            ok = 1;
            for (int dx = -1; dx <= 1 && ok; ++dx)
                for (int dy = -1; dy <= 1 && ok; ++dy)
                    for (int dz = -1; dz <= 1 && ok; ++dz) {
                        int64_t *h = cell_slot(&m, cx + dx, cy + dy, cz + dz, 0);
                        if (!h) continue;
                        for (int64_t j = *h; j >= 0; j = next[j]) {
                            if (j == i - 1) continue;
                            double ax = xyz[3 * j] - cand[0], ay = xyz[3 * j + 1] - cand[1],
                                   az = xyz[3 * j + 2] - cand[2];
                            if (ax * ax + ay * ay + az * az < ex2) { ok = 0; break; }
                        }
                    }
        }
        if (!ok) ++violations;
        for (int d = 0; d < 3; ++d) xyz[3 * i + d] = cand[d];
        int64_t *h = cell_slot(&m, (int64_t)floor(cand[0] * inv), (int64_t)floor(cand[1] * inv),
                               (int64_t)floor(cand[2] * inv), 1);
        next[i] = *h; *h = i;
    }
    free(m.key_x); free(m.key_y); free(m.key_z); free(m.head); free(next);
    /* charges */
    double mean = 0.0;
    for (int64_t i = 0; i < n; ++i) { q[i] = sigma * nrm(&r); mean += q[i]; }
    mean /= (double)n;
    for (int64_t i = 0; i < n; ++i) q[i] -= mean;
    return violations;
}

/* ---- many chains in parallel: fragment f uses stream (stream0 + f) --------------- */
typedef struct {
    uint64_t seed, stream0;
    int64_t nfrag;
    const int64_t *counts, *offsets;
    double step, excl, sigma;
    int max_trials;
    double *xyz, *q;
    int64_t *viol;
    int64_t next_frag;
    pthread_mutex_t lock;
} chains_job_t;

static void *chains_worker(void *arg)
{
    chains_job_t *j = (chains_job_t *)arg;
    for (;;) {
        pthread_mutex_lock(&j->lock);
        int64_t f = j->next_frag++;
        pthread_mutex_unlock(&j->lock);
        if (f >= j->nfrag) return NULL;
        int64_t off = j->offsets[f];
        j->viol[f] = synth_chain(j->seed, j->stream0 + (uint64_t)f, j->counts[f], j->step, j->excl,
                                 j->max_trials, j->sigma, j->xyz + 3 * off, j->q + off);
    }
}

int synth_chains(uint64_t seed, uint64_t stream0, int64_t nfrag, const int64_t *counts,
                 const int64_t *offsets, double step, double excl, int max_trials, double sigma,
                 int nthreads, double *xyz, double *q, int64_t *viol)
{
    chains_job_t j;
    j.seed = seed; j.stream0 = stream0; j.nfrag = nfrag; j.counts = counts; j.offsets = offsets;
    j.step = step; j.excl = excl; j.sigma = sigma; j.max_trials = max_trials;
    j.xyz = xyz; j.q = q; j.viol = viol; j.next_frag = 0;
    pthread_mutex_init(&j.lock, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    int started = 0;
    for (int t = 0; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, chains_worker, &j) == 0) ++started;
    if (started == 0) chains_worker(&j);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&j.lock);
    for (int64_t f = 0; f < nfrag; ++f)
        if (viol[f] < 0) return -1;
    return 0;
}
