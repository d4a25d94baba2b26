/*
 * Host driver that runs every oracle routine under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by test_oracle_sanitizers.py on the CPU).
 * It covers the edge cases the routines must handle: K = 16 and K = 1, a single table,
 * zero rows, n = 0, a capped insert that saturates, a deletion of a point never
 * inserted, every threshold mode on empty and non-empty sets.  Exit status 0 only if the
 * sanitizers stay silent and the invariants checked here hold (sum of each table's counts
 * equals the points inserted; the scores equal a recount).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n, m_scored;
    double mu, mu_scored, sigma, sigma_table, tau;
    int32_t mode, pad;
} thresh_t;

void ace_oracle_project(const float* X, int64_t n, int32_t d, const float* W, int32_t ncols, double* P, double* M);
void ace_oracle_hash(const float* X, int64_t n, int32_t d, const float* W, int32_t K, int32_t L, uint16_t* codes,
                     uint16_t* amb);
void ace_oracle_insert(const uint16_t* codes, int64_t n, int32_t K, int32_t L, int64_t* counts, int64_t* S2,
                       uint64_t* S3, int64_t* n_total);
int64_t ace_oracle_insert_capped(const uint16_t* codes, int64_t n, int32_t K, int32_t L, int64_t cap,
                                 int64_t* counts, int64_t* S2, uint64_t* S3, int64_t* n_total);
int64_t ace_oracle_delete(const uint16_t* codes, int64_t n, int32_t K, int32_t L, int64_t* counts, int64_t* S2,
                          uint64_t* S3, int64_t* n_total);
void ace_oracle_score(const uint16_t* codes, int64_t n, int32_t K, int32_t L, const int64_t* counts, int64_t* T);
void ace_oracle_moments(const int64_t* T, int64_t n, int64_t* m, int64_t* sumT, uint64_t* sumT2);
int ace_oracle_threshold(int64_t n, int32_t L, const int64_t* S2, const uint64_t* S3, int64_t m, int64_t sumT,
                         const uint64_t* sumT2, int32_t mode, double alpha, thresh_t* out);
void ace_oracle_flags(const int64_t* T, int64_t n, int32_t L, double tau, int32_t mode, uint8_t* flags);
void ace_oracle_exact_score(const float* Q, int64_t nq, const float* X, int64_t n, int32_t d, int32_t K, double* S);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static float uniform_pm1(void) {
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (float)((double)(state >> 11) / 9007199254740992.0 * 2.0 - 1.0);
}

#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                  \
        }                                                              \
    } while (0)

static int run(int64_t n, int32_t d, int32_t K, int32_t L) {
    const int64_t B = (int64_t)1 << K;
    float* X = malloc(sizeof(float) * (size_t)(n ? n : 1) * d);
    float* W = malloc(sizeof(float) * (size_t)d * K * L);
    for (int64_t i = 0; i < n * d; i++) X[i] = uniform_pm1();
    for (int64_t i = 0; i < (int64_t)d * K * L; i++) W[i] = uniform_pm1();
    if (n > 2)
        for (int32_t t = 0; t < d; t++) X[1 * d + t] = 0.f;  /* a zero row */
    double* P = malloc(sizeof(double) * (size_t)(n ? n : 1) * K * L);
    double* M = malloc(sizeof(double) * (size_t)(n ? n : 1) * K * L);
    ace_oracle_project(X, n, d, W, K * L, P, M);
    uint16_t* codes = calloc((size_t)(n ? n : 1) * L, sizeof(uint16_t));
    uint16_t* amb = calloc((size_t)(n ? n : 1) * L, sizeof(uint16_t));
    ace_oracle_hash(X, n, d, W, K, L, codes, amb);
    for (int64_t i = 0; i < n * L; i++) CHECK(codes[i] < B);

    int64_t* counts = calloc((size_t)L * B, sizeof(int64_t));
    int64_t* S2 = calloc((size_t)L, sizeof(int64_t));
    uint64_t* S3 = calloc((size_t)L * 2, sizeof(uint64_t));
    int64_t nt = 0;
    ace_oracle_insert(codes, n, K, L, counts, S2, S3, &nt);
    CHECK(nt == n);
    for (int32_t j = 0; j < L; j++) {
        int64_t s = 0;
        for (int64_t b = 0; b < B; b++) s += counts[j * B + b];
        CHECK(s == n);
    }
    int64_t* T = calloc((size_t)(n ? n : 1), sizeof(int64_t));
    ace_oracle_score(codes, n, K, L, counts, T);
    for (int64_t i = 0; i < n; i++) {
        int64_t t = 0;
        for (int32_t j = 0; j < L; j++) t += counts[j * B + codes[i * L + j]];
        CHECK(T[i] == t && T[i] >= L);
    }
    int64_t m = 0, sumT = 0;
    uint64_t sumT2[2] = {0, 0};
    ace_oracle_moments(T, n, &m, &sumT, sumT2);
    thresh_t th;
    for (int32_t mode = 0; mode < 3; mode++) {
        const int rc = ace_oracle_threshold(nt, L, S2, S3, m, sumT, sumT2, mode, 1.0, &th);
        CHECK(rc == (n == 0 ? 4 : 0));
        uint8_t* flags = calloc((size_t)(n ? n : 1), 1);
        ace_oracle_flags(T, n, L, th.tau, mode, flags);
        free(flags);
    }
    /* a point never inserted is rejected whole; inserted points delete back to zero */
    if (n > 0) {
        uint16_t* other = malloc(sizeof(uint16_t) * (size_t)L);
        for (int32_t j = 0; j < L; j++) other[j] = (uint16_t)((codes[j] + 1) & (B - 1));
        int64_t present = 1;
        for (int32_t j = 0; j < L; j++) present &= counts[j * B + other[j]] > 0;
        const int64_t rej = ace_oracle_delete(other, 1, K, L, counts, S2, S3, &nt);
        CHECK(rej == (present ? 0 : 1));
        if (present) ace_oracle_insert(other, 1, K, L, counts, S2, S3, &nt);
        free(other);
    }
    CHECK(ace_oracle_delete(codes, n, K, L, counts, S2, S3, &nt) == 0);
    CHECK(nt == 0);
    for (int64_t i = 0; i < (int64_t)L * B; i++) CHECK(counts[i] == 0);
    for (int32_t j = 0; j < L; j++) CHECK(S2[j] == 0 && S3[2 * j] == 0 && S3[2 * j + 1] == 0);
    /* saturating short counters with a small cap */
    const int64_t dropped = ace_oracle_insert_capped(codes, n, K, L, 2, counts, S2, S3, &nt);
    CHECK(dropped >= 0 && nt == n);
    for (int64_t i = 0; i < (int64_t)L * B; i++) CHECK(counts[i] <= 2);
    /* exact statistic with zero rows on both sides */
    double* S = malloc(sizeof(double) * (size_t)(n ? n : 1));
    ace_oracle_exact_score(X, n, X, n, d, K, S);
    for (int64_t i = 0; i < n; i++) CHECK(S[i] >= 1.0 - 1e-12);
    free(S);
    free(X); free(W); free(P); free(M); free(codes); free(amb); free(counts); free(S2); free(S3); free(T);
    return 0;
}

int main(void) {
    static const int32_t shapes[][4] = {{37, 13, 16, 5}, {1, 1, 1, 1}, {0, 4, 3, 2}, {300, 7, 10, 20}, {64, 33, 15, 3}};
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); s++) {
        if (run(shapes[s][0], shapes[s][1], shapes[s][2], shapes[s][3])) {
            fprintf(stderr, "shape %zu failed\n", s);
            return 1;
        }
    }
    printf("oracle sanitizer run ok\n");
    return 0;
}
