/*
 * tcm_oracle.c -- plain, slow, single-threaded FP64 CPU oracle for the two-centre
 * multipole (TCM) method of Solov'yov, Yakubovich, Solov'yov and Greiner,
 * "Two center multipole expansion method: application to macromolecular systems".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load this
 * file: only the tests, the smoke check and the benchmark's CPU-baseline leg use it.  It
 * shares no code, header, table or constant with the HIP implementation.
 *
 * What it computes, in the paper's order and notation:
 *   - eq. (1)  direct pairwise Coulomb energy            -> oracle_coulomb
 *   - eq. (2)  separation condition |R0| > |r_i^A|+|r_j^B| -> oracle_radius (a = max |r_i|)
 *   - eq. (8)  multipole moments Q_lm about a centre      -> oracle_moments
 *   - eq. (6)  3j symbols (general Racah formula)         -> oracle_threej
 *   - eq. (9)  truncated two-centre energy, square truncation l1,l2 <= Lmax
 *                                                          -> oracle_energy
 *              or triangular truncation l1+l2 <= Lmax      -> oracle_energy_shape
 * plus test helpers that are not in the paper: the rigid pose of a molecule
 * (oracle_pose), rigorous truncation-error bounds for both truncation shapes
 * (oracle_trunc_bound, oracle_trunc_bound_tri), the first-order sensitivity of eq. (9) to
 * perturbations of the moments (oracle_energy_sensitivity, the scale of the rounding error
 * of a reduced-precision moment pass), and the
 * forces the paper names as the other use of its final expression (section I):
 *   - -grad_R0 of eq. (9), term by term                   -> oracle_energy_grad
 *   - the coefficients of eq. (9) as a linear function of one molecule's moments
 *                                                          -> oracle_energy_coeffs
 *   - per-atom forces at fixed centres, through eq. (8)   -> oracle_atom_forces
 *
 * Conventions (the paper is silent; readings listed in the design notes):
 *   - Y_lm carries the Condon-Shortley phase; Y_{l,-m} = (-1)^m conj(Y_lm).
 *   - Complex moment arrays are interleaved (re, im) and indexed by l*l + l + m,
 *     m in [-l, l], so an order-L table holds (L+1)^2 complex numbers.
 *   - Units: eq. (1) has no prefactor, so energies are (charge)^2 / length.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (no contraction of a*b+c
 * into fused operations, so every rounding is the one the C source spells out).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_LMAX 64            /* largest order the oracle accepts for moments */
#define ORACLE_FACT_MAX 300       /* long double factorial table length             */

/* ---------------------------------------------------------------------------------
 * Neumaier (improved Kahan-Babuska) compensated summation.  Every long sum in the
 * oracle goes through it so that the oracle's own rounding error stays near 1 ulp.
 * ------------------------------------------------------------------------------- */
typedef struct { double s, c; } nsum_t;

static void nsum_add(nsum_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_value(const nsum_t *a) { return a->s + a->c; }

/* ---------------------------------------------------------------------------------
 * Factorials n! for 0 <= n < ORACLE_FACT_MAX in long double (x87 80-bit: 64-bit
 * mantissa, exponent range to ~1e4932, so 299! ~ 1e612 is representable).
 * ------------------------------------------------------------------------------- */
static long double g_fact[ORACLE_FACT_MAX];
static int g_fact_ready = 0;

static void fact_init(void)
{
    if (g_fact_ready) return;
    g_fact[0] = 1.0L;
    for (int i = 1; i < ORACLE_FACT_MAX; ++i) g_fact[i] = g_fact[i - 1] * (long double)i;
    g_fact_ready = 1;
}

static long double fact(int n) { return g_fact[n]; }

/* ---------------------------------------------------------------------------------
 * Fully normalised associated Legendre functions Pbar_l^m(cos theta), m >= 0, with the
 * Condon-Shortley phase, normalised so that Y_lm(theta, phi) = Pbar_l^m(cos theta) e^{i m phi}
 * is orthonormal on the sphere.  Textbook stable upward recurrence:
 *   Pbar_0^0 = 1/sqrt(4 pi)
 *   Pbar_m^m = -sqrt((2m+1)/(2m)) sin(theta) Pbar_{m-1}^{m-1}
 *   Pbar_{m+1}^m = sqrt(2m+3) cos(theta) Pbar_m^m
 *   Pbar_l^m = a_lm (cos(theta) Pbar_{l-1}^m - b_lm Pbar_{l-2}^m),
 *       a_lm = sqrt((4l^2-1)/(l^2-m^2)),  b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
 * Output index: l*(l+1)/2 + m.
 * ------------------------------------------------------------------------------- */
static void legendre_normalised(int L, double ct, double st, double *P)
{
    P[0] = 1.0 / sqrt(4.0 * M_PI);
    for (int m = 1; m <= L; ++m) {
        int i = m * (m + 1) / 2 + m, j = (m - 1) * m / 2 + (m - 1);
        P[i] = -sqrt((2.0 * m + 1.0) / (2.0 * m)) * st * P[j];
    }
    for (int m = 0; m < L; ++m) {
        int i = (m + 1) * (m + 2) / 2 + m, j = m * (m + 1) / 2 + m;
        P[i] = sqrt(2.0 * m + 3.0) * ct * P[j];
    }
    for (int m = 0; m <= L; ++m) {
        for (int l = m + 2; l <= L; ++l) {
            double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            double b = sqrt((((double)l - 1.0) * (l - 1.0) - (double)m * m) /
                            (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
            P[l * (l + 1) / 2 + m] =
                a * (ct * P[(l - 1) * l / 2 + m] - b * P[(l - 2) * (l - 1) / 2 + m]);
        }
    }
}

/* Y_lm(theta, phi) for any m in [-l, l] (exported for the library-routine pin tests). */
int oracle_ylm(int l, int m, double theta, double phi, double *re, double *im)
{
    if (l < 0 || l > 4 * ORACLE_LMAX || m < -l || m > l || !re || !im) return -1;
    double *P = (double *)malloc(sizeof(double) * (size_t)(l + 1) * (l + 2) / 2);
    if (!P) return -3;
    legendre_normalised(l, cos(theta), sin(theta), P);
    int am = m < 0 ? -m : m;
    double p = P[l * (l + 1) / 2 + am];
    double yr = p * cos(am * phi), yi = p * sin(am * phi);
    if (m < 0) {                             /* Y_{l,-m} = (-1)^m conj(Y_lm) */
        double s = (am & 1) ? -1.0 : 1.0;
        yr = s * yr;
        yi = -s * yi;
    }
    *re = yr;
    *im = yi;
    free(P);
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Wigner 3j symbol (j1 j2 j3; m1 m2 m3) by the general Racah formula:
 *   (-1)^{j1-j2-m3} sqrt(Delta) sqrt((j1+m1)!(j1-m1)!(j2+m2)!(j2-m2)!(j3+m3)!(j3-m3)!)
 *   * sum_k (-1)^k / [k! (j3-j2+k+m1)! (j3-j1+k-m2)! (j1+j2-j3-k)! (j1-k-m1)! (j2-k+m2)!],
 *   Delta = (j1+j2-j3)!(j1-j2+j3)!(-j1+j2+j3)!/(j1+j2+j3+1)!.
 * Integer arguments only (all angular momenta in eq. (9) are integers).  Evaluated in
 * long double; the sum has a single term in the stretched case j3 = j1 + j2 that eq. (9)
 * uses.  Returns 0 outside the selection rules.
 * ------------------------------------------------------------------------------- */
double oracle_threej(int j1, int j2, int j3, int m1, int m2, int m3)
{
    fact_init();
    if (m1 + m2 + m3 != 0) return 0.0;
    if (j1 < 0 || j2 < 0 || j3 < 0) return 0.0;
    if (abs(m1) > j1 || abs(m2) > j2 || abs(m3) > j3) return 0.0;
    if (j3 > j1 + j2 || j3 < abs(j1 - j2)) return 0.0;
    if (j1 + j2 + j3 + 1 >= ORACLE_FACT_MAX) return NAN;
    long double delta = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) /
                        fact(j1 + j2 + j3 + 1);
    long double pref = sqrtl(delta) *
                       sqrtl(fact(j1 + m1) * fact(j1 - m1)) *
                       sqrtl(fact(j2 + m2) * fact(j2 - m2)) *
                       sqrtl(fact(j3 + m3) * fact(j3 - m3));
    int kmin = 0, kmax = j1 + j2 - j3;
    if (j2 - j3 - m1 > kmin) kmin = j2 - j3 - m1;
    if (j1 - j3 + m2 > kmin) kmin = j1 - j3 + m2;
    if (j1 - m1 < kmax) kmax = j1 - m1;
    if (j2 + m2 < kmax) kmax = j2 + m2;
    long double sum = 0.0L;
    for (int k = kmin; k <= kmax; ++k) {
        long double den = fact(k) * fact(j3 - j2 + k + m1) * fact(j3 - j1 + k - m2) *
                          fact(j1 + j2 - j3 - k) * fact(j1 - k - m1) * fact(j2 - k + m2);
        sum += ((k & 1) ? -1.0L : 1.0L) / den;
    }
    int e = j1 - j2 - m3;
    long double sign = (((e % 2) + 2) % 2) ? -1.0L : 1.0L;
    return (double)(sign * pref * sum);
}

/* Unweighted centroid of n points (eq. (1) lets the centre be "any suitable point"). */
int oracle_centroid(const double *xyz, int64_t n, double *c_out)
{
    if (!xyz || !c_out || n <= 0) return -1;
    for (int d = 0; d < 3; ++d) {
        nsum_t s = {0.0, 0.0};
        for (int64_t i = 0; i < n; ++i) nsum_add(&s, xyz[3 * i + d]);
        c_out[d] = nsum_value(&s) / (double)n;
    }
    return 0;
}

/* Radius a = max_i |R_i - c|: the quantity eq. (2) bounds. */
double oracle_radius(const double *xyz, int64_t n, const double *c)
{
    double a = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double dx = xyz[3 * i] - c[0], dy = xyz[3 * i + 1] - c[1], dz = xyz[3 * i + 2] - c[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r > a) a = r;
    }
    return a;
}

/* ---------------------------------------------------------------------------------
 * eq. (8): Q_lm = sum_i q_i r_i^l sqrt(4 pi / (2l+1)) Y_lm(theta_i, phi_i), r_i = R_i - c,
 * for 0 <= l <= L and -l <= m <= l.  Output Q: 2*(L+1)^2 doubles, (re, im) interleaved at
 * complex index l*l + l + m.  Optional Qabs (same layout, real only, (L+1)^2 doubles):
 * sum_i |q_i| |r_i^l sqrt(4pi/(2l+1)) Y_lm| -- the absolute-value sums used to state the
 * conditioning of a moment.  An atom at the centre contributes q_i to Q_00 only (0^0 = 1).
 * ------------------------------------------------------------------------------- */
int oracle_moments(const double *xyz, const double *q, int64_t n, const double *c, int L,
                   double *Q, double *Qabs)
{
    if (!xyz || !q || !c || !Q || n < 0 || L < 0 || L > ORACLE_LMAX) return -1;
    int nc = (L + 1) * (L + 1);
    nsum_t *acc = (nsum_t *)calloc((size_t)2 * nc, sizeof(nsum_t));
    nsum_t *aab = (nsum_t *)calloc((size_t)nc, sizeof(nsum_t));
    double *P = (double *)malloc(sizeof(double) * (size_t)(L + 1) * (L + 2) / 2);
    double *rl = (double *)malloc(sizeof(double) * (size_t)(L + 1));
    if (!acc || !aab || !P || !rl) { free(acc); free(aab); free(P); free(rl); return -3; }
    for (int64_t i = 0; i < n; ++i) {
        double dx = xyz[3 * i] - c[0], dy = xyz[3 * i + 1] - c[1], dz = xyz[3 * i + 2] - c[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r == 0.0) {
            nsum_add(&acc[0], q[i]);
            nsum_add(&aab[0], fabs(q[i]));
            continue;
        }
        double ctr = dz / r;
        if (ctr > 1.0) ctr = 1.0;
        if (ctr < -1.0) ctr = -1.0;
        double theta = acos(ctr), phi = atan2(dy, dx);
        legendre_normalised(L, cos(theta), sin(theta), P);
        rl[0] = 1.0;
        for (int l = 1; l <= L; ++l) rl[l] = rl[l - 1] * r;
        for (int l = 0; l <= L; ++l) {
            double racah = sqrt(4.0 * M_PI / (2.0 * l + 1.0));
            for (int m = 0; m <= l; ++m) {
                double p = P[l * (l + 1) / 2 + m];
                double w = q[i] * rl[l] * racah * p;
                double yr = w * cos(m * phi), yi = w * sin(m * phi);
                int k = l * l + l + m;
                nsum_add(&acc[2 * k], yr);
                nsum_add(&acc[2 * k + 1], yi);
                nsum_add(&aab[k], fabs(w));
                if (m > 0) {                 /* Y_{l,-m} = (-1)^m conj(Y_lm) */
                    double s = (m & 1) ? -1.0 : 1.0;
                    int kn = l * l + l - m;
                    nsum_add(&acc[2 * kn], s * yr);
                    nsum_add(&acc[2 * kn + 1], -s * yi);
                    nsum_add(&aab[kn], fabs(w));
                }
            }
        }
    }
    for (int k = 0; k < 2 * nc; ++k) Q[k] = nsum_value(&acc[k]);
    if (Qabs)
        for (int k = 0; k < nc; ++k) Qabs[k] = nsum_value(&aab[k]);
    free(acc); free(aab); free(P); free(rl);
    return 0;
}

/* ---------------------------------------------------------------------------------
 * eq. (9) summed literally with the summation rule stated after it:
 *   U = sum_{l1,l2=0..L} sum_{m1,m2} (-1)^{l1+M} R0^{-(L'+1)}
 *       sqrt(4 pi (2L')! / ((2l1)! (2l2)!)) (l1 l2 L'; m1 m2 -M) Q^A_{l1m1} Q^B_{l2m2}
 *       conj(Y_{L'M}(Theta_R0, Phi_R0)),      L' = l1 + l2, M = m1 + m2.
 * R = c_B - c_A.  QA, QB: complex tables (layout of oracle_moments) of order >= L, given
 * with their orders LA, LB.  Outputs: U_re, U_im (the sum is real up to rounding),
 * optional terms[(L+1)^2] = Re of the partial sum for each (l1, l2) at index l1*(L+1)+l2,
 * optional abs_sum = sum of |term| (the scale against which rounding is judged).
 *
 * shape selects which (l1, l2) blocks the sum keeps.  The limits printed under eq. (9) are
 * garbled ("l1, l2 = 0" and "l1 + l2 = L" under L_max); the text after it and eq. (11) loop
 * l1 and l2 each to L_max (shape 0, square, the reading used everywhere by default); the
 * other reading keeps the blocks of total order l1 + l2 <= L_max (shape 1, triangular), whose
 * dropped blocks are exactly the (L'+1)-th and higher orders of the expansion of eq. (3).
 * Blocks a shape drops are not summed and their terms[] entries are 0.
 * ------------------------------------------------------------------------------- */
int oracle_energy_shape(const double *QA, int LA, const double *QB, int LB, const double *R, int L,
                        int shape, double *U_re, double *U_im, double *terms, double *abs_sum)
{
    fact_init();
    if (!QA || !QB || !R || !U_re || L < 0 || L > LA || L > LB || 2 * L > 4 * ORACLE_LMAX)
        return -1;
    if (shape != 0 && shape != 1) return -1;
    double Rn = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    if (!(Rn > 0.0)) return -1;
    double ctr = R[2] / Rn;
    if (ctr > 1.0) ctr = 1.0;
    if (ctr < -1.0) ctr = -1.0;
    double Theta = acos(ctr), Phi = atan2(R[1], R[0]);
    int L2 = 2 * L;
    double *P = (double *)malloc(sizeof(double) * (size_t)(L2 + 1) * (L2 + 2) / 2);
    if (!P) return -3;
    legendre_normalised(L2, cos(Theta), sin(Theta), P);
    nsum_t sre = {0, 0}, sim = {0, 0}, sab = {0, 0};
    for (int l1 = 0; l1 <= L; ++l1) {
        for (int l2 = 0; l2 <= L; ++l2) {
            int Lp = l1 + l2;
            if (shape == 1 && Lp > L) {
                if (terms) terms[l1 * (L + 1) + l2] = 0.0;
                continue;
            }
            double coef = (double)sqrtl(4.0L * (long double)M_PI * fact(2 * Lp) /
                                        (fact(2 * l1) * fact(2 * l2)));
            double rpow = pow(Rn, -(double)(Lp + 1));
            nsum_t tre = {0, 0};
            for (int m1 = -l1; m1 <= l1; ++m1) {
                const double *a = QA + 2 * (l1 * l1 + l1 + m1);
                for (int m2 = -l2; m2 <= l2; ++m2) {
                    const double *b = QB + 2 * (l2 * l2 + l2 + m2);
                    int M = m1 + m2;
                    double tj = oracle_threej(l1, l2, Lp, m1, m2, -M);
                    if (tj == 0.0) continue;
                    /* conj(Y_{L'M}(Theta, Phi)) */
                    int aM = M < 0 ? -M : M;
                    double p = P[Lp * (Lp + 1) / 2 + aM];
                    double yr = p * cos(aM * Phi), yi = p * sin(aM * Phi);
                    if (M < 0) {
                        double s = (aM & 1) ? -1.0 : 1.0;
                        yr = s * yr;
                        yi = -s * yi;
                    }
                    yi = -yi; /* conjugate */
                    double sgn = (((l1 + M) % 2) + 2) % 2 ? -1.0 : 1.0;
                    double f = sgn * rpow * coef * tj;
                    /* f * a * b * y */
                    double abr = a[0] * b[0] - a[1] * b[1];
                    double abi = a[0] * b[1] + a[1] * b[0];
                    double tr = f * (abr * yr - abi * yi);
                    double ti = f * (abr * yi + abi * yr);
                    nsum_add(&sre, tr);
                    nsum_add(&sim, ti);
                    nsum_add(&tre, tr);
                    nsum_add(&sab, sqrt(tr * tr + ti * ti));
                }
            }
            if (terms) terms[l1 * (L + 1) + l2] = nsum_value(&tre);
        }
    }
    *U_re = nsum_value(&sre);
    if (U_im) *U_im = nsum_value(&sim);
    if (abs_sum) *abs_sum = nsum_value(&sab);
    free(P);
    return 0;
}

/* eq. (9) with the square truncation l1, l2 <= L (the reading used by default). */
int oracle_energy(const double *QA, int LA, const double *QB, int LB, const double *R, int L,
                  double *U_re, double *U_im, double *terms, double *abs_sum)
{
    return oracle_energy_shape(QA, LA, QB, LB, R, L, 0, U_re, U_im, terms, abs_sum);
}

/* ---------------------------------------------------------------------------------
 * First-order sensitivity of eq. (9) to errors in the moments.  Eq. (9) is bilinear in the
 * two tables, U = sum_t f_t Q^A_{l1m1} Q^B_{l2m2} with f_t the factor of each term (sign,
 * R0 power, square root, 3j symbol, conj Y).  If every moment is perturbed by at most a
 * multiple e of its absolute sum, |dQ_lm| <= e Abar_lm with Abar_lm = sum_i |q_i|
 * |r_i^l sqrt(4 pi/(2l+1)) Y_lm| (the Qabs output of oracle_moments), then to first order
 *   |dU| <= e * sum_t |f_t| (Abar^A_{l1m1} |Q^B_{l2m2}| + |Q^A_{l1m1}| Abar^B_{l2m2}).
 * This returns that sum (without e) over the terms the truncation shape keeps.  QA, QB:
 * complex tables as for oracle_energy; AbarA, AbarB: real tables of the same orders.
 * ------------------------------------------------------------------------------- */
int oracle_energy_sensitivity(const double *QA, const double *AbarA, int LA, const double *QB,
                              const double *AbarB, int LB, const double *R, int L, int shape,
                              double *out)
{
    fact_init();
    if (!QA || !QB || !AbarA || !AbarB || !R || !out || L < 0 || L > LA || L > LB ||
        2 * L > 4 * ORACLE_LMAX || (shape != 0 && shape != 1))
        return -1;
    double Rn = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    if (!(Rn > 0.0)) return -1;
    double ctr = R[2] / Rn;
    if (ctr > 1.0) ctr = 1.0;
    if (ctr < -1.0) ctr = -1.0;
    double Theta = acos(ctr);
    int L2 = 2 * L;
    double *P = (double *)malloc(sizeof(double) * (size_t)(L2 + 1) * (L2 + 2) / 2);
    if (!P) return -3;
    legendre_normalised(L2, cos(Theta), sin(Theta), P);
    nsum_t acc = {0, 0};
    for (int l1 = 0; l1 <= L; ++l1) {
        for (int l2 = 0; l2 <= L; ++l2) {
            int Lp = l1 + l2;
            if (shape == 1 && Lp > L) continue;
            double coef = (double)sqrtl(4.0L * (long double)M_PI * fact(2 * Lp) /
                                        (fact(2 * l1) * fact(2 * l2)));
            double rpow = pow(Rn, -(double)(Lp + 1));
            for (int m1 = -l1; m1 <= l1; ++m1) {
                int ka = l1 * l1 + l1 + m1;
                double qa = hypot(QA[2 * ka], QA[2 * ka + 1]);
                for (int m2 = -l2; m2 <= l2; ++m2) {
                    int kb = l2 * l2 + l2 + m2;
                    int M = m1 + m2;
                    double tj = oracle_threej(l1, l2, Lp, m1, m2, -M);
                    if (tj == 0.0) continue;
                    int aM = M < 0 ? -M : M;
                    /* |conj Y_{L'M}| = |Pbar_{L'}^{|M|}| */
                    double f = fabs(rpow * coef * tj * P[Lp * (Lp + 1) / 2 + aM]);
                    double qb = hypot(QB[2 * kb], QB[2 * kb + 1]);
                    nsum_add(&acc, f * (AbarA[ka] * qb + qa * AbarB[kb]));
                }
            }
        }
    }
    *out = nsum_value(&acc);
    free(P);
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Derivatives of the solid harmonics for the forces (not printed in the paper; textbook
 * calculus on its eq. (8) and eq. (9) ingredients).
 *
 * For a direction theta, three tables over l <= L, 0 <= m <= l (index l*(l+1)/2 + m):
 *   P = Pbar_l^m(cos theta)                      (legendre_normalised)
 *   S = Pbar_l^m(cos theta) / sin(theta), m >= 1 (the same three-term recurrence in l,
 *       started from Pbar_m^m / sin = -sqrt((2m+1)/(2m)) Pbar_{m-1}^{m-1}: no division, so
 *       it holds on the axis too)
 *   D = d Pbar_l^m / d theta:  m = 0: sqrt(l(l+1)) Pbar_l^1;
 *       m >= 1: (sqrt((l-m)(l+m+1)) Pbar_l^{m+1} - sqrt((l+m)(l-m+1)) Pbar_l^{m-1}) / 2
 *       (Condon-Shortley phase).
 * ------------------------------------------------------------------------------- */
static void legendre_derivs(int L, double ct, double st, double *P, double *S, double *D)
{
    legendre_normalised(L, ct, st, P);
    for (int k = 0; k < (L + 1) * (L + 2) / 2; ++k) S[k] = 0.0;
    for (int m = 1; m <= L; ++m) {
        int i = m * (m + 1) / 2 + m, j = (m - 1) * m / 2 + (m - 1);
        S[i] = -sqrt((2.0 * m + 1.0) / (2.0 * m)) * P[j];
        if (m + 1 <= L) S[(m + 1) * (m + 2) / 2 + m] = sqrt(2.0 * m + 3.0) * ct * S[i];
        for (int l = m + 2; l <= L; ++l) {
            double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            double b = sqrt((((double)l - 1.0) * (l - 1.0) - (double)m * m) /
                            (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
            S[l * (l + 1) / 2 + m] = a * (ct * S[(l - 1) * l / 2 + m] - b * S[(l - 2) * (l - 1) / 2 + m]);
        }
    }
    for (int l = 0; l <= L; ++l) {
        for (int m = 0; m <= l; ++m) {
            double up = m + 1 <= l ? P[l * (l + 1) / 2 + m + 1] : 0.0;
            if (m == 0)
                D[l * (l + 1) / 2] = sqrt((double)l * (l + 1)) * up;
            else
                D[l * (l + 1) / 2 + m] = 0.5 * (sqrt((double)(l - m) * (l + m + 1)) * up -
                                                sqrt((double)(l + m) * (l - m + 1)) * P[l * (l + 1) / 2 + m - 1]);
        }
    }
}

/* Gradient of g = r^p Y_lm(theta, phi) (any m in [-l, l]) at the point (r, theta, phi), as
 * 3 complex components (re, im interleaved) in out[6]:
 *   grad g = r^{p-1} e^{i m phi} [ p Pbar r_hat + dPbar/dtheta theta_hat + i m (Pbar/sin) phi_hat ],
 * with negative m through Y_{l,-m} = (-1)^m conj(Y_lm).  The tables P, S, D are those of the
 * point's theta (order >= l).  p = l gives the regular solid harmonic (up to the factor
 * sqrt(4 pi/(2l+1))), p = -(l+1) the irregular one. */
static void grad_solid(int l, int m, int p, double r, double theta, double phi, const double *P,
                       const double *S, const double *D, double *out)
{
    int am = m < 0 ? -m : m;
    int k = l * (l + 1) / 2 + am;
    double ct = cos(theta), st = sin(theta), cp = cos(phi), sp = sin(phi);
    double rh[3] = {st * cp, st * sp, ct}, th[3] = {ct * cp, ct * sp, -st}, ph[3] = {-sp, cp, 0.0};
    double rp = (p - 1 == 0) ? 1.0 : pow(r, (double)(p - 1));
    double er = cos(am * phi), ei = sin(am * phi);
    for (int d = 0; d < 3; ++d) {
        /* v = p P rh + D th + i m S ph  (m >= 0 part) */
        double vr = p * P[k] * rh[d] + D[k] * th[d];
        double vi = am > 0 ? am * S[k] * ph[d] : 0.0;
        double gr = rp * (vr * er - vi * ei), gi = rp * (vr * ei + vi * er);
        if (m < 0) {
            double sg = (am & 1) ? -1.0 : 1.0;
            gr = sg * gr;
            gi = -sg * gi;
        }
        out[2 * d] = gr;
        out[2 * d + 1] = gi;
    }
}

/* ---------------------------------------------------------------------------------
 * grad_R0 of eq. (9): the same literal sum as oracle_energy with R0^{-(L'+1)} conj(Y_{L'M})
 * replaced by its gradient in R0 (the moments held fixed: B translated rigidly).  The force
 * on B is -grad, the force on A +grad.  Output grad[3].
 * ------------------------------------------------------------------------------- */
int oracle_energy_grad(const double *QA, int LA, const double *QB, int LB, const double *R, int L,
                       double *grad)
{
    fact_init();
    if (!QA || !QB || !R || !grad || L < 0 || L > LA || L > LB || 2 * L > 4 * ORACLE_LMAX) return -1;
    double Rn = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    if (!(Rn > 0.0)) return -1;
    double ctr = R[2] / Rn;
    if (ctr > 1.0) ctr = 1.0;
    if (ctr < -1.0) ctr = -1.0;
    double Theta = acos(ctr), Phi = atan2(R[1], R[0]);
    int L2 = 2 * L, nt = (L2 + 1) * (L2 + 2) / 2;
    double *P = (double *)malloc(sizeof(double) * 3 * (size_t)nt);
    if (!P) return -3;
    double *S = P + nt, *D = S + nt;
    legendre_derivs(L2, cos(Theta), sin(Theta), P, S, D);
    nsum_t g[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int l1 = 0; l1 <= L; ++l1) {
        for (int l2 = 0; l2 <= L; ++l2) {
            int Lp = l1 + l2;
            double coef = (double)sqrtl(4.0L * (long double)M_PI * fact(2 * Lp) /
                                        (fact(2 * l1) * fact(2 * l2)));
            for (int m1 = -l1; m1 <= l1; ++m1) {
                const double *a = QA + 2 * (l1 * l1 + l1 + m1);
                for (int m2 = -l2; m2 <= l2; ++m2) {
                    const double *b = QB + 2 * (l2 * l2 + l2 + m2);
                    int M = m1 + m2;
                    double tj = oracle_threej(l1, l2, Lp, m1, m2, -M);
                    if (tj == 0.0) continue;
                    double gy[6];
                    grad_solid(Lp, M, -(Lp + 1), Rn, Theta, Phi, P, S, D, gy);
                    double sgn = (((l1 + M) % 2) + 2) % 2 ? -1.0 : 1.0;
                    double f = sgn * coef * tj;
                    double abr = a[0] * b[0] - a[1] * b[1];
                    double abi = a[0] * b[1] + a[1] * b[0];
                    for (int d = 0; d < 3; ++d) {
                        /* Re(f a b conj(gy_d)) */
                        nsum_add(&g[d], f * (abr * gy[2 * d] + abi * gy[2 * d + 1]));
                    }
                }
            }
        }
    }
    for (int d = 0; d < 3; ++d) grad[d] = nsum_value(&g[d]);
    free(P);
    return 0;
}

/* ---------------------------------------------------------------------------------
 * eq. (9) is bilinear in the two moment tables.  side = 1: W with U = Re sum_{l2 m2}
 * W_{l2 m2} Q^B_{l2 m2}, i.e. W_{l2 m2} = sum_{l1 m1} (the eq. (9) factor) Q^A_{l1 m1}
 * R0^{-(L'+1)} conj(Y_{L'M}); side = 0: the same with the roles of the tables exchanged
 * (U = Re sum V_{l1 m1} Q^A_{l1 m1}).  Output: 2 (L+1)^2 doubles, layout of oracle_moments.
 * ------------------------------------------------------------------------------- */
int oracle_energy_coeffs(const double *QA, int LA, const double *QB, int LB, const double *R, int L,
                         int side, double *W)
{
    fact_init();
    if (!QA || !QB || !R || !W || L < 0 || L > LA || L > LB || 2 * L > 4 * ORACLE_LMAX) return -1;
    double Rn = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    if (!(Rn > 0.0)) return -1;
    double ctr = R[2] / Rn;
    if (ctr > 1.0) ctr = 1.0;
    if (ctr < -1.0) ctr = -1.0;
    double Theta = acos(ctr), Phi = atan2(R[1], R[0]);
    int L2 = 2 * L, nc = (L + 1) * (L + 1);
    double *P = (double *)malloc(sizeof(double) * (size_t)(L2 + 1) * (L2 + 2) / 2);
    nsum_t *acc = (nsum_t *)calloc((size_t)2 * nc, sizeof(nsum_t));
    if (!P || !acc) { free(P); free(acc); return -3; }
    legendre_normalised(L2, cos(Theta), sin(Theta), P);
    for (int l1 = 0; l1 <= L; ++l1) {
        for (int l2 = 0; l2 <= L; ++l2) {
            int Lp = l1 + l2;
            double coef = (double)sqrtl(4.0L * (long double)M_PI * fact(2 * Lp) /
                                        (fact(2 * l1) * fact(2 * l2)));
            double rpow = pow(Rn, -(double)(Lp + 1));
            for (int m1 = -l1; m1 <= l1; ++m1) {
                for (int m2 = -l2; m2 <= l2; ++m2) {
                    int M = m1 + m2;
                    double tj = oracle_threej(l1, l2, Lp, m1, m2, -M);
                    if (tj == 0.0) continue;
                    int aM = M < 0 ? -M : M;
                    double p = P[Lp * (Lp + 1) / 2 + aM];
                    double yr = p * cos(aM * Phi), yi = p * sin(aM * Phi);
                    if (M < 0) {
                        double s = (aM & 1) ? -1.0 : 1.0;
                        yr = s * yr;
                        yi = -s * yi;
                    }
                    yi = -yi; /* conjugate */
                    double sgn = (((l1 + M) % 2) + 2) % 2 ? -1.0 : 1.0;
                    double f = sgn * rpow * coef * tj;
                    /* coefficient of the other table's entry: f * Q_this * conj(Y) */
                    const double *o = side ? QA + 2 * (l1 * l1 + l1 + m1) : QB + 2 * (l2 * l2 + l2 + m2);
                    int k = side ? l2 * l2 + l2 + m2 : l1 * l1 + l1 + m1;
                    nsum_add(&acc[2 * k], f * (o[0] * yr - o[1] * yi));
                    nsum_add(&acc[2 * k + 1], f * (o[0] * yi + o[1] * yr));
                }
            }
        }
    }
    for (int k = 0; k < 2 * nc; ++k) W[k] = nsum_value(&acc[k]);
    free(P);
    free(acc);
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Per-atom forces at fixed centres: with U = Re sum_{lm} W_lm Q_lm (oracle_energy_coeffs)
 * and Q_lm = sum_i q_i r_i^l sqrt(4 pi/(2l+1)) Y_lm(r_i) (eq. (8)), the force on atom i is
 *   F_i = -dU/dR_i = -q_i Re sum_{lm} W_lm sqrt(4 pi/(2l+1)) grad(r^l Y_lm)(r_i),
 * r_i = xyz_i - c (the rigid pose, if any, already applied to xyz).  W: order L, layout of
 * oracle_moments.  Output F[n][3].
 * ------------------------------------------------------------------------------- */
int oracle_atom_forces(const double *W, int L, const double *xyz, const double *q, int64_t n, const double *c,
                       double *F)
{
    if (!W || !xyz || !q || !c || !F || n < 0 || L < 0 || L > ORACLE_LMAX) return -1;
    int nt = (L + 1) * (L + 2) / 2;
    double *P = (double *)malloc(sizeof(double) * 3 * (size_t)nt);
    if (!P) return -3;
    double *S = P + nt, *D = S + nt;
    for (int64_t i = 0; i < n; ++i) {
        double dx = xyz[3 * i] - c[0], dy = xyz[3 * i + 1] - c[1], dz = xyz[3 * i + 2] - c[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        double theta = 0.0, phi = 0.0;
        if (r > 0.0) {
            double ctr = dz / r;
            if (ctr > 1.0) ctr = 1.0;
            if (ctr < -1.0) ctr = -1.0;
            theta = acos(ctr);
            phi = atan2(dy, dx);
        }
        legendre_derivs(L, cos(theta), sin(theta), P, S, D);
        nsum_t f[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int l = 1; l <= L; ++l) {                 /* l = 0 is constant */
            if (r == 0.0 && l > 1) break;              /* grad r^l Y_lm vanishes at 0 for l > 1 */
            double racah = sqrt(4.0 * M_PI / (2.0 * l + 1.0));
            for (int m = -l; m <= l; ++m) {
                double g[6];
                grad_solid(l, m, l, r, theta, phi, P, S, D, g);
                const double *w = W + 2 * (l * l + l + m);
                for (int d = 0; d < 3; ++d) nsum_add(&f[d], racah * (w[0] * g[2 * d] - w[1] * g[2 * d + 1]));
            }
        }
        for (int d = 0; d < 3; ++d) F[3 * i + d] = -q[i] * nsum_value(&f[d]);
    }
    free(P);
    return 0;
}

/* eq. (1): U = sum_i sum_j q_i q_j / |R_j^B - R_i^A| over absolute positions. */
double oracle_coulomb(const double *xyzA, const double *qA, int64_t nA,
                      const double *xyzB, const double *qB, int64_t nB)
{
    nsum_t s = {0.0, 0.0};
    for (int64_t i = 0; i < nA; ++i) {
        for (int64_t j = 0; j < nB; ++j) {
            double dx = xyzB[3 * j] - xyzA[3 * i];
            double dy = xyzB[3 * j + 1] - xyzA[3 * i + 1];
            double dz = xyzB[3 * j + 2] - xyzA[3 * i + 2];
            nsum_add(&s, qA[i] * qB[j] / sqrt(dx * dx + dy * dy + dz * dz));
        }
    }
    return nsum_value(&s);
}

/* ---------------------------------------------------------------------------------
 * Rigid pose (not in the paper, whose scan only translates B): out_i = c_new + Rot(quat)
 * (x_i - c_old), with Rot the active rotation of the normalised unit quaternion
 * quat = (w, x, y, z).  The oracle obtains a posed molecule's moments by recomputing
 * eq. (8) on these coordinates.
 * ------------------------------------------------------------------------------- */
int oracle_pose(const double *xyz, int64_t n, const double *c_old, const double *quat,
                const double *c_new, double *out)
{
    if (!xyz || !c_old || !quat || !c_new || !out || n < 0) return -1;
    double qn = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    if (!(qn > 0.0)) return -1;
    double w = quat[0] / qn, x = quat[1] / qn, y = quat[2] / qn, z = quat[3] / qn;
    double M[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
                   2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                   2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
    for (int64_t i = 0; i < n; ++i) {
        double d[3] = {xyz[3 * i] - c_old[0], xyz[3 * i + 1] - c_old[1], xyz[3 * i + 2] - c_old[2]};
        for (int r = 0; r < 3; ++r)
            out[3 * i + r] = c_new[r] + M[3 * r] * d[0] + M[3 * r + 1] * d[1] + M[3 * r + 2] * d[2];
    }
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Rigorous bound on |U_coulomb - U_L| for the square truncation l1, l2 <= L (derived for
 * the test suite, not printed in the paper).  With alpha = aA/R, beta = aB/R and S = sum|q|:
 * the (l1, l2) term of the double Taylor series of 1/|R + r_B - r_A| is bounded by
 * C(l1+l2, l1) aA^l1 aB^l2 / R^{l1+l2+1}; summing the terms outside the square gives
 *   |dU| <= SA SB / (R (1-alpha-beta)) [ (alpha/(1-beta))^{L+1} + (beta/(1-alpha))^{L+1} ].
 * Requires alpha + beta < 1 (eq. (2)); returns +inf otherwise.
 * ------------------------------------------------------------------------------- */
double oracle_trunc_bound(double SA, double SB, double aA, double aB, double R, int L)
{
    double al = aA / R, be = aB / R;
    if (!(al + be < 1.0)) return INFINITY;
    double t1 = pow(al / (1.0 - be), L + 1), t2 = pow(be / (1.0 - al), L + 1);
    return SA * SB / (R * (1.0 - al - be)) * (t1 + t2);
}

/* ---------------------------------------------------------------------------------
 * The same for the triangular truncation l1 + l2 <= L (oracle_energy_shape, shape 1): the
 * dropped terms are the bidegree (l1, l2) Taylor terms with l1 + l2 = n > L, whose bounds
 * sum to C(n, l1) alpha^l1 beta^l2 summed over l1 = (alpha + beta)^n, so with t = alpha + beta
 *   |dU| <= SA SB / R * sum_{n > L} t^n = SA SB t^{L+1} / (R (1 - t)).
 * Requires t < 1 (eq. (2)); returns +inf otherwise.
 * ------------------------------------------------------------------------------- */
double oracle_trunc_bound_tri(double SA, double SB, double aA, double aB, double R, int L)
{
    double t = aA / R + aB / R;
    if (!(t < 1.0)) return INFINITY;
    return SA * SB * pow(t, L + 1) / (R * (1.0 - t));
}
