/*
 * ACE oracle: a plain, slow CPU implementation of the ACE count estimator in
 * FP64 and exact integers.  TEST INFRASTRUCTURE ONLY: it is called by the
 * tests, by the smoke check and by the benchmark's CPU-baseline leg, never by
 * the library.  It shares no code with the HIP path.
 *
 * What it computes, in the paper's order (Luo & Shrivastava, "Arrays of
 * (locality-sensitive) Count Estimators", arXiv 1706.06664):
 *
 *   projection  p_ic = sum_t x_it w_tc                      (Sec. 2.1, SRP)
 *   bit         h = [p > 0]                                 (Sec. 2.1; sign(0) read as 0)
 *   meta-hash   H_j(x) = sum_k h_{j,k}(x) 2^k              (Sec. 3.2, K-bit concatenation)
 *   insert      A_j[H_j(x)]++ for every table j             (Alg. 1, pre-processing phase)
 *   running sum S2_j = sum_b A_j[b]^2, grown by 2c+1 per    (Sec. 3.4.1, Eq. dynadd:
 *               increment of a count c                        n mu = sum_j S2_j / L)
 *   delete      A_j[H_j(x)]--, S2_j shrinks by 2c-1         (Sec. 3.4.1, Eq. dynsub)
 *   score       T(q) = sum_j A_j[H_j(q)], s = T / L         (Alg. 1, query phase)
 *   threshold   mu - alpha (Alg. 1) or mu_s - sigma_s of     (Sec. 5.3)
 *               the scored set
 *
 * Readings of points the paper leaves open (sign of zero, bit order,
 * pre-increment count in the running mean, strict vs non-strict comparison,
 * population sigma) are listed beside the functions that take them.
 *
 * Floating point: x and w are FP32; their product is exact in FP64, and the
 * sum over t runs in ascending t with one FP64 rounding per addition.  The
 * returned margin m_ic = gamma_d * sum_t |x_it w_tc| with
 * gamma_d = d u / (1 - d u), u = 2^-53, bounds the error of that sum
 * (standard bound for recursive summation, Higham, Accuracy and Stability of
 * Numerical Algorithms, 2nd ed., Sec. 3.1).  Bits with |p| <= m are reported
 * as ambiguous: the sign of the exact sum is not certain there.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

static double gamma_n(int n) {
    const double u = ldexp(1.0, -53);
    return (double)n * u / (1.0 - (double)n * u);
}

/* Dense projection P = X W in FP64 plus the rounding margin M (Sec. 2.1). */
void ace_oracle_project(const float* X, int64_t n, int32_t d, const float* W, int32_t ncols,
                        double* P, double* M) {
    const double g = gamma_n(d);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        for (int32_t c = 0; c < ncols; c++) {
            double p = 0.0, a = 0.0;
            for (int32_t t = 0; t < d; t++) {
                double prod = (double)X[i * d + t] * (double)W[(int64_t)t * ncols + c];
                p += prod;
                a += fabs(prod);
            }
            P[i * ncols + c] = p;
            if (M) M[i * ncols + c] = g * a;
        }
    }
}

/*
 * Hash every row into L K-bit codes (Sec. 2.1 and 3.2).
 * W is [d][K*L] row-major; column c = j*K + k is the SRP vector of bit k of
 * table j (bit k of the code is the k-th concatenated SRP bit; any fixed
 * order is a bijection of bucket labels and leaves counts and scores alone).
 * codes: [n][L].  amb (optional): [n][L], bit k set when |p| <= margin.
 */
void ace_oracle_hash(const float* X, int64_t n, int32_t d, const float* W, int32_t K, int32_t L,
                     uint16_t* codes, uint16_t* amb) {
    const int32_t ncols = K * L;
    const double g = gamma_n(d);
#pragma omp parallel
    {
        double* p = (double*)malloc(sizeof(double) * (size_t)ncols);
        double* a = (double*)malloc(sizeof(double) * (size_t)ncols);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; i++) {
            const float* x = X + i * d;
            for (int32_t c = 0; c < ncols; c++) { p[c] = 0.0; a[c] = 0.0; }
            for (int32_t t = 0; t < d; t++) {
                const double xt = (double)x[t];
                const float* wrow = W + (int64_t)t * ncols;
                for (int32_t c = 0; c < ncols; c++) {
                    double prod = xt * (double)wrow[c];
                    p[c] += prod;
                    a[c] += fabs(prod);
                }
            }
            for (int32_t j = 0; j < L; j++) {
                uint32_t code = 0, am = 0;
                for (int32_t k = 0; k < K; k++) {
                    const int32_t c = j * K + k;
                    if (p[c] > 0.0) code |= 1u << k;           /* sign(0) -> bit 0 */
                    if (fabs(p[c]) <= g * a[c]) am |= 1u << k;
                }
                codes[i * L + j] = (uint16_t)code;
                if (amb) amb[i * L + j] = (uint16_t)am;
            }
        }
        free(p);
        free(a);
    }
}

/*
 * Counting phase of Alg. 1 with the running statistics of Sec. 3.4.1.
 * counts: int64 [L][2^K]; S2: int64 [L]; S3: u64 [L][2] (lo, hi of an
 * unsigned 128-bit sum of cubes, kept for the per-table variance).
 * Points are taken in order; per table the count c before the increment is
 * read first, so S2 grows by (c+1)^2 - c^2 = 2c+1 (Eq. dynadd uses the
 * pre-increment count; that keeps sum_j S2_j / (n L) equal to the mean score
 * of the inserted points).
 */
void ace_oracle_insert(const uint16_t* codes, int64_t n, int32_t K, int32_t L,
                       int64_t* counts, int64_t* S2, uint64_t* S3, int64_t* n_total) {
    const int64_t B = (int64_t)1 << K;
    for (int64_t i = 0; i < n; i++) {
        for (int32_t j = 0; j < L; j++) {
            const int64_t b = codes[i * L + j];
            const int64_t c = counts[j * B + b];
            S2[j] += 2 * c + 1;
            u128 s3 = ((u128)S3[2 * j + 1] << 64) | S3[2 * j];
            s3 += (u128)(3 * c * c + 3 * c + 1);
            S3[2 * j] = (uint64_t)s3;
            S3[2 * j + 1] = (uint64_t)(s3 >> 64);
            counts[j * B + b] = c + 1;
        }
        *n_total += 1;
    }
}

/*
 * Short counters (Sec. 3.4 keeps each count in a 16-bit integer).  With a cap, a count
 * that already equals the cap keeps its value and the increment is dropped (a saturating
 * counter).  S2 and S3 follow the stored counts, so sum_j S2_j / (n L) is the mean of the
 * stored-count scores of the inserted points.  Returns the number of dropped increments.
 * Inserting only, the stored count of a bucket is min(true count, cap) in any order.
 */
int64_t ace_oracle_insert_capped(const uint16_t* codes, int64_t n, int32_t K, int32_t L, int64_t cap,
                                 int64_t* counts, int64_t* S2, uint64_t* S3, int64_t* n_total) {
    const int64_t B = (int64_t)1 << K;
    int64_t dropped = 0;
    for (int64_t i = 0; i < n; i++) {
        for (int32_t j = 0; j < L; j++) {
            int64_t* a = &counts[j * B + codes[i * L + j]];
            if (*a >= cap) {
                dropped++;
                continue;
            }
            const int64_t before = *a, after = before + 1;
            S2[j] += after * after - before * before;
            u128 cube = ((u128)S3[2 * j + 1] << 64) | S3[2 * j];
            cube += (u128)(after * after * after - before * before * before);
            S3[2 * j] = (uint64_t)cube;
            S3[2 * j + 1] = (uint64_t)(cube >> 64);
            *a = after;
        }
        *n_total += 1;
    }
    return dropped;
}

/*
 * Deletion (Sec. 3.4.1, Eq. dynsub): decrement each table's count, S2 shrinks
 * by c^2 - (c-1)^2 = 2c-1 with c the count before the decrement.  A point
 * whose bucket is empty in some table cannot have been inserted; such a point
 * is skipped whole and counted in the return value.
 */
int64_t ace_oracle_delete(const uint16_t* codes, int64_t n, int32_t K, int32_t L,
                          int64_t* counts, int64_t* S2, uint64_t* S3, int64_t* n_total) {
    const int64_t B = (int64_t)1 << K;
    int64_t rejected = 0;
    for (int64_t i = 0; i < n; i++) {
        int ok = 1;
        for (int32_t j = 0; j < L; j++)
            if (counts[j * B + codes[i * L + j]] < 1) ok = 0;
        if (!ok) { rejected++; continue; }
        for (int32_t j = 0; j < L; j++) {
            const int64_t b = codes[i * L + j];
            const int64_t c = counts[j * B + b];
            S2[j] -= 2 * c - 1;
            u128 s3 = ((u128)S3[2 * j + 1] << 64) | S3[2 * j];
            s3 -= (u128)(3 * c * c - 3 * c + 1);
            S3[2 * j] = (uint64_t)s3;
            S3[2 * j + 1] = (uint64_t)(s3 >> 64);
            counts[j * B + b] = c - 1;
        }
        *n_total -= 1;
    }
    return rejected;
}

/* Query phase of Alg. 1: T(q) = sum_j A_j[H_j(q)] (the score is T / L). */
void ace_oracle_score(const uint16_t* codes, int64_t n, int32_t K, int32_t L,
                      const int64_t* counts, int64_t* T) {
    const int64_t B = (int64_t)1 << K;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        int64_t t = 0;
        for (int32_t j = 0; j < L; j++) t += counts[j * B + codes[i * L + j]];
        T[i] = t;
    }
}

/*
 * Moments of a scored set: m, sum T, sum T^2 (the last as lo/hi of an
 * unsigned 128-bit integer).  Accumulates into the given totals.
 */
void ace_oracle_moments(const int64_t* T, int64_t n, int64_t* m, int64_t* sumT, uint64_t* sumT2) {
    u128 s2 = ((u128)sumT2[1] << 64) | sumT2[0];
    for (int64_t i = 0; i < n; i++) {
        *m += 1;
        *sumT += T[i];
        s2 += (u128)T[i] * (u128)T[i];
    }
    sumT2[0] = (uint64_t)s2;
    sumT2[1] = (uint64_t)(s2 >> 64);
}

typedef struct {
    int64_t n, m_scored;
    double mu, mu_scored, sigma, sigma_table, tau;
    int32_t mode, pad;
} ace_oracle_thresh;

/*
 * Threshold statistics (Alg. 1 and Sec. 5.3).
 *   mu       = sum_j S2_j / (n L): the mean score of the inserted points.
 *   mu_s     = sum T / (m L) over the scored set.
 *   sigma_s  = sqrt(m sum T^2 - (sum T)^2) / (m L): population std of the
 *              scored set's scores (the numerator is an exact integer).
 *   sigma_t  = (1/L) sum_j sqrt(n S3_j - S2_j^2) / n: the mean over tables of
 *              the std of the per-table count seen by the inserted points;
 *              by the triangle inequality it bounds the inserted set's sigma.
 * mode 0 (scored):  tau = mu_s - alpha sigma_s
 * mode 1 (const):   tau = mu - alpha
 * mode 2 (table):   tau = mu - alpha sigma_t
 * Returns 0, or 4 when a needed set is empty.
 */
int ace_oracle_threshold(int64_t n, int32_t L, const int64_t* S2, const uint64_t* S3,
                         int64_t m, int64_t sumT, const uint64_t* sumT2,
                         int32_t mode, double alpha, ace_oracle_thresh* out) {
    memset(out, 0, sizeof(*out));
    out->n = n;
    out->m_scored = m;
    out->mode = mode;
    i128 s2tot = 0;
    for (int32_t j = 0; j < L; j++) s2tot += S2[j];
    out->mu = n > 0 ? (double)s2tot / ((double)n * (double)L) : 0.0;
    if (m > 0) {
        const u128 st2 = ((u128)sumT2[1] << 64) | sumT2[0];
        const i128 num = (i128)m * (i128)st2 - (i128)sumT * (i128)sumT;
        out->mu_scored = (double)sumT / ((double)m * (double)L);
        out->sigma = sqrt((double)num) / ((double)m * (double)L);
    }
    if (n > 0) {
        double acc = 0.0;
        for (int32_t j = 0; j < L; j++) {
            const u128 s3 = ((u128)S3[2 * j + 1] << 64) | S3[2 * j];
            const i128 v = (i128)n * (i128)s3 - (i128)S2[j] * (i128)S2[j];
            acc += sqrt((double)v) / (double)n;
        }
        out->sigma_table = acc / (double)L;
    }
    if (mode == 0) {
        if (m == 0) return 4;
        out->tau = out->mu_scored - alpha * out->sigma;
    } else if (mode == 1) {
        if (n == 0) return 4;
        out->tau = out->mu - alpha;
    } else {
        if (n == 0) return 4;
        out->tau = out->mu - alpha * out->sigma_table;
    }
    return 0;
}

/*
 * Flags: mode 1 (Alg. 1) reports s <= tau; modes 0 and 2 report s < tau
 * ("less than", Sec. 5.3).  s = T / L is compared as T against L tau.
 */
void ace_oracle_flags(const int64_t* T, int64_t n, int32_t L, double tau, int32_t mode, uint8_t* flags) {
    const double lim = (double)L * tau;
    for (int64_t i = 0; i < n; i++) {
        const double t = (double)T[i];
        flags[i] = (uint8_t)(mode == 1 ? (t <= lim) : (t < lim));
    }
}

/*
 * The statistic ACE estimates (Sec. 3, Eq. thescore): S(q, D) = sum_i p(q, x_i)^K
 * with p the SRP collision probability 1 - arccos(cos-sim)/pi (Sec. 2.1, Eq. srp).
 * A zero vector has no angle.  Its SRP bit is always 0 under the sign(0) -> 0
 * reading, so it matches a nonzero vector's bit with probability 1/2 and
 * another zero vector's always: p = 0.5 and p = 1 for those pairs.
 */
void ace_oracle_exact_score(const float* Q, int64_t nq, const float* X, int64_t n, int32_t d, int32_t K,
                            double* S) {
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < nq; a++) {
        const float* q = Q + a * d;
        double qq = 0.0;
        for (int32_t t = 0; t < d; t++) qq += (double)q[t] * (double)q[t];
        double s = 0.0;
        for (int64_t i = 0; i < n; i++) {
            const float* x = X + i * d;
            double xx = 0.0, qx = 0.0;
            for (int32_t t = 0; t < d; t++) {
                xx += (double)x[t] * (double)x[t];
                qx += (double)q[t] * (double)x[t];
            }
            double p;
            if (qq == 0.0 && xx == 0.0) {
                p = 1.0;
            } else if (qq == 0.0 || xx == 0.0) {
                p = 0.5;
            } else {
                double cs = qx / (sqrt(qq) * sqrt(xx));
                if (cs > 1.0) cs = 1.0;
                if (cs < -1.0) cs = -1.0;
                p = 1.0 - acos(cs) / 3.14159265358979323846;
            }
            s += pow(p, (double)K);
        }
        S[a] = s;
    }
}
