/* Host-only harness that drives every entry point of the CPU oracle
 * (oracle/cashash_oracle.c, oracle/geometry_oracle.c) over small seeded
 * inputs -- empty and one-point images, self pairs, query subsets, the
 * epipolar band, tau, k above the candidate count, degenerate geometry --
 * so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * reports any out-of-bounds access, leak or undefined operation.  It checks
 * only invariants that hold for any input; the oracle's values are pinned
 * elsewhere. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/cashash_oracle.h"

int32_t oracle_subset_size(int32_t n, int32_t num, int32_t den);
void oracle_top_scale(const float* scale, int32_t n, int32_t m, int32_t* rows);
void oracle_floyd8(const uint32_t* r, int32_t n, int32_t* out);
void oracle_fundamental_batch(int32_t n_pairs, const float* q, const float* t, const int64_t* off,
                              const uint32_t* rand, int32_t n_hyp, double thr, int32_t min_matches,
                              double* F, int32_t* n_inliers, int32_t* best_h, int32_t* status);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32(void) { /* xorshift64* */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 2685821657736338717ull) >> 32);
}
static double next_normal(void) { /* sum of uniforms: plenty for a harness */
    double s = 0.0;
    for (int i = 0; i < 12; ++i) s += next_u32() / 4294967296.0;
    return s - 6.0;
}

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            failures++;                                                   \
        }                                                                 \
    } while (0)

int main(void) {
    enum { M = 6 };
    const int32_t nf[M] = {0, 1, 37, 64, 130, 300};
    uint8_t* desc[M];
    uint64_t* codes[M];
    uint8_t* keys[M];
    float* kp[M];
    for (int m = 0; m < M; ++m) {
        desc[m] = malloc((size_t)nf[m] * 128 + 1);
        codes[m] = malloc((size_t)nf[m] * 16 + 8);
        keys[m] = malloc((size_t)nf[m] * 6 + 1);
        kp[m] = malloc((size_t)nf[m] * 8 + 4);
        for (int64_t i = 0; i < (int64_t)nf[m] * 128; ++i) desc[m][i] = (uint8_t)(next_u32() % 120);
        for (int64_t i = 0; i < (int64_t)nf[m] * 2; ++i) kp[m][i] = (float)(next_u32() % 1000);
    }
    /* duplicated rows in the largest image: ties of distance and Hamming */
    memcpy(desc[5] + 128 * 7, desc[5] + 128 * 3, 128);
    double* rc = malloc(sizeof(double) * 128 * 128);
    double* rb = malloc(sizeof(double) * 48 * 128);
    for (int i = 0; i < 128 * 128; ++i) rc[i] = next_normal();
    for (int i = 0; i < 48 * 128; ++i) rb[i] = (i / 128) % 8 < 2 ? next_normal() : 0.0; /* coarse keys */
    oracle_build_codes(M, (const uint8_t* const*)desc, nf, rc, rb, codes, keys);

    int32_t pairs[][2] = {{5, 4}, {4, 5}, {5, 5}, {0, 5}, {5, 0}, {1, 5}, {5, 1}, {2, 3}, {3, 2}, {1, 1}, {0, 0}};
    const int64_t P = sizeof pairs / sizeof pairs[0];
    int64_t total = 0;
    for (int64_t p = 0; p < P; ++p) total += nf[pairs[p][0]];
    int32_t* out = malloc(sizeof(int32_t) * 3 * (size_t)(total + 1));
    double* F = malloc(sizeof(double) * 9 * (size_t)P);
    for (int64_t p = 0; p < P; ++p)
        for (int i = 0; i < 9; ++i) F[9 * p + i] = (i == 5) ? -1.0 : (i == 7) ? 1.0 : 0.0; /* rectified */
    const int32_t ks[] = {1, 2, 10, 64};
    const int32_t taus[] = {128, 40, 0};
    for (int ki = 0; ki < 4; ++ki)
        for (int ti = 0; ti < 3; ++ti)
            for (int epi = 0; epi < 2; ++epi) {
                oracle_params prm = {ks[ki], 4, 5, taus[ti]};
                oracle_match_pairs(M, (const uint8_t* const*)desc, (const uint64_t* const*)codes,
                                   (const uint8_t* const*)keys, nf, P, &pairs[0][0], &prm,
                                   epi ? (const float* const*)kp : NULL, epi ? F : NULL, 200.0, out, out + total,
                                   out + 2 * total);
                for (int64_t i = 0; i < total; ++i) {
                    const int32_t idx = out[i], d1 = out[total + i], d2 = out[2 * total + i];
                    CHECK(idx >= -1 && d1 >= -1 && d2 >= -1);
                    CHECK(d2 == -1 || d1 <= d2);
                    CHECK(idx == -1 || (d1 >= 0 && d2 >= 0 && 25ll * d1 < 16ll * d2));
                }
            }
    /* query subsets of one pair */
    {
        int32_t sel[] = {299, 0, 7, 3, 150};
        int32_t o[3][5];
        oracle_params prm = {10, 4, 5, 128};
        oracle_match_pair(desc[5], codes[5], keys[5], nf[5], desc[4], codes[4], keys[4], nf[4], &prm, kp[5], kp[4],
                          F, 4.0, sel, 5, o[0], o[1], o[2]);
        oracle_match_pair(desc[5], codes[5], keys[5], nf[5], desc[0], codes[0], keys[0], nf[0], &prm, NULL, NULL,
                          NULL, 0.0, sel, 5, o[0], o[1], o[2]);
        for (int i = 0; i < 5; ++i) CHECK(o[0][i] == -1 && o[1][i] == -1 && o[2][i] == -1);
    }
    /* geometry: subsets, Floyd sampling, fundamental matrices */
    {
        float sc[301];
        for (int i = 0; i < 301; ++i) sc[i] = (float)(next_u32() % 17) - 3.0f;
        sc[5] = -0.0f;
        sc[9] = 0.0f;
        for (int n = 0; n <= 301; n += 43) {
            const int32_t mm = oracle_subset_size(n, 1, 5);
            int32_t* rows = malloc(sizeof(int32_t) * (size_t)(mm + 1));
            oracle_top_scale(sc, n, mm, rows);
            for (int i = 1; i < mm; ++i) CHECK(rows[i - 1] < rows[i]);
            free(rows);
        }
        for (int n = 8; n < 40; ++n) {
            uint32_t r[8];
            int32_t o8[8];
            for (int i = 0; i < 8; ++i) r[i] = next_u32();
            oracle_floyd8(r, n, o8);
            for (int i = 0; i < 8; ++i) {
                CHECK(o8[i] >= 0 && o8[i] < n);
                for (int j = 0; j < i; ++j) CHECK(o8[i] != o8[j]);
            }
        }
        enum { NP = 4, NM = 40, NH = 16 };
        const int32_t counts[NP] = {NM, 7, 20, 0};
        int64_t off[NP + 1] = {0};
        for (int p = 0; p < NP; ++p) off[p + 1] = off[p] + counts[p];
        float* q = malloc(sizeof(float) * 2 * (size_t)(off[NP] + 1));
        float* t = malloc(sizeof(float) * 2 * (size_t)(off[NP] + 1));
        for (int64_t i = 0; i < off[NP]; ++i) {
            q[2 * i] = (float)(next_u32() % 1920);
            q[2 * i + 1] = (float)(next_u32() % 1080);
            t[2 * i] = q[2 * i] + 30.0f;
            t[2 * i + 1] = q[2 * i + 1] + (float)(next_u32() % 3);
        }
        for (int64_t i = off[2]; i < off[3]; ++i) { /* coincident points: degenerate */
            q[2 * i] = q[2 * i + 1] = 5.0f;
            t[2 * i] = t[2 * i + 1] = 9.0f;
        }
        uint32_t rnd[NH * 8];
        for (int i = 0; i < NH * 8; ++i) rnd[i] = next_u32();
        double Fo[9 * NP];
        int32_t inl[NP], bh[NP], stt[NP];
        oracle_fundamental_batch(NP, q, t, off, rnd, NH, 2.0, 16, Fo, inl, bh, stt);
        for (int p = 0; p < NP; ++p) CHECK(stt[p] >= 0 && stt[p] <= 3);
        CHECK(stt[1] == 1 && stt[3] == 1);
        free(q);
        free(t);
    }
    for (int m = 0; m < M; ++m) {
        free(desc[m]);
        free(codes[m]);
        free(keys[m]);
        free(kp[m]);
    }
    free(rc);
    free(rb);
    free(out);
    free(F);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle harness ok\n");
    return 0;
}
