/*
 * CPU oracle for CasHash pairwise matching.  TEST INFRASTRUCTURE ONLY: see
 * cashash_oracle.h.  Each function follows the paper's steps in order, with
 * no blocking or fusion; OpenMP only splits independent queries or pairs.
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -shared -fPIC -lm.
 */
#include "cashash_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int32_t oracle_num_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Mean of the set, kept as integer sums so that centring is exact:
 * N * (x - mean) = N * x - S. */
void oracle_column_sums(int32_t n_images, const uint8_t* const* desc, const int32_t* n_feat,
                        int64_t* S, int64_t* n_tot) {
    for (int i = 0; i < ORACLE_DIM; ++i) S[i] = 0;
    int64_t n = 0;
    for (int32_t m = 0; m < n_images; ++m) {
        for (int64_t r = 0; r < n_feat[m]; ++r)
            for (int i = 0; i < ORACLE_DIM; ++i) S[i] += desc[m][r * ORACLE_DIM + i];
        n += n_feat[m];
    }
    *n_tot = n;
}

/* Charikar hashing ("The Improved Parallel Calculation of Hashing Code"):
 * bit = [r . (x - mean) > 0], evaluated as [r . (N x - S) > 0] (N > 0 keeps the
 * sign).  The inner product is one binary64 fused multiply-add chain over
 * components 0..127; an exact zero gives bit 0. */
static int sign_bit(const double* r, const double* c) {
    double p = 0.0;
    for (int i = 0; i < ORACLE_DIM; ++i) p = fma(r[i], c[i], p);
    return p > 0.0;
}

void oracle_project(const uint8_t* x, int64_t n, const int64_t* S, int64_t n_tot,
                    const double* r_code, const double* r_bucket,
                    uint64_t* codes, uint8_t* keys) {
#pragma omp parallel for schedule(static)
    for (int64_t d = 0; d < n; ++d) {
        double c[ORACLE_DIM];
        for (int i = 0; i < ORACLE_DIM; ++i)
            c[i] = (double)(n_tot * (int64_t)x[d * ORACLE_DIM + i] - S[i]);
        /* Step 2 code: n = 128 bits */
        uint64_t w[2] = {0, 0};
        for (int j = 0; j < ORACLE_CODE_BITS; ++j)
            if (sign_bit(r_code + (int64_t)j * ORACLE_DIM, c)) w[j >> 6] |= (uint64_t)1 << (j & 63);
        codes[d * 2 + 0] = w[0];
        codes[d * 2 + 1] = w[1];
        /* Step 1 keys: m = 8 bits per table, 6 tables */
        for (int t = 0; t < ORACLE_TABLES; ++t) {
            unsigned key = 0;
            for (int b = 0; b < ORACLE_KEY_BITS; ++b)
                if (sign_bit(r_bucket + ((int64_t)t * ORACLE_KEY_BITS + b) * ORACLE_DIM, c)) key |= 1u << b;
            keys[d * ORACLE_TABLES + t] = (uint8_t)key;
        }
    }
}

void oracle_build_codes(int32_t n_images, const uint8_t* const* desc, const int32_t* n_feat,
                        const double* r_code, const double* r_bucket,
                        uint64_t* const* codes, uint8_t* const* keys) {
    int64_t S[ORACLE_DIM], n_tot;
    oracle_column_sums(n_images, desc, n_feat, S, &n_tot);
    for (int32_t m = 0; m < n_images; ++m)
        oracle_project(desc[m], n_feat[m], S, n_tot, r_code, r_bucket, codes[m], keys[m]);
}

/* ---------------- matching ---------------- */

typedef struct {
    int32_t ham;
    int32_t j;
} ranked_t;

static int cmp_ranked(const void* a, const void* b) {
    const ranked_t* x = (const ranked_t*)a;
    const ranked_t* y = (const ranked_t*)b;
    if (x->ham != y->ham) return x->ham < y->ham ? -1 : 1;
    return (x->j > y->j) - (x->j < y->j);
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

static int popcount64(uint64_t v) {
    int c = 0;
    while (v) {
        v &= v - 1;
        ++c;
    }
    return c;
}

/* Eq. 1-2: distance of candidate (x', y') to the epipolar line
 * (a, b, c) = F (x, y, 1) of the query, compared without division or square
 * root as e^2 <= d^2 (a^2 + b^2), with the absolute value Eq. 2 omits. */
static int within_band(const double* F, double x, double y, double xp, double yp, double d) {
    double a = (F[0] * x + F[1] * y) + F[2];
    double b = (F[3] * x + F[4] * y) + F[5];
    double c = (F[6] * x + F[7] * y) + F[8];
    double e = (a * xp + b * yp) + c;
    return e * e <= (d * d) * (a * a + b * b);
}

/* Bucket lists of the train image for every table: ascending indices j with
 * key_t(j) == v, stored as start[t][v] .. start[t][v+1] into ids[t][*]. */
static void build_buckets(const uint8_t* keys_t, int32_t n_t, int32_t* start, int32_t* ids) {
    for (int t = 0; t < ORACLE_TABLES; ++t) {
        int32_t* st = start + t * 257;
        int32_t* id = ids + (int64_t)t * n_t;
        int32_t cnt[256];
        memset(cnt, 0, sizeof cnt);
        for (int32_t j = 0; j < n_t; ++j) cnt[keys_t[(int64_t)j * ORACLE_TABLES + t]]++;
        st[0] = 0;
        for (int v = 0; v < 256; ++v) st[v + 1] = st[v] + cnt[v];
        int32_t fill[256];
        memcpy(fill, st, sizeof fill);
        for (int32_t j = 0; j < n_t; ++j) id[fill[keys_t[(int64_t)j * ORACLE_TABLES + t]]++] = j;
    }
}

typedef struct {
    const uint8_t *desc_q, *desc_t;
    const uint64_t *codes_q, *codes_t;
    const uint8_t *keys_q, *keys_t;
    int32_t n_q, n_t;
    const oracle_params* prm;
    const float *kp_q, *kp_t;
    const double* F;
    double max_px;
    const int32_t *start, *ids;
} pair_ctx;

/* One query through Steps 1-4.  Scratch: seen[n_t] holds, per train point,
 * the stamp of the last query that collected it; cand[n_t], dist[n_t]. */
static void match_one(const pair_ctx* P, int32_t q, int32_t stamp, int32_t* seen, ranked_t* cand,
                      int32_t* dist, int32_t* out_idx, int32_t* out_d1, int32_t* out_d2) {
    const int32_t n_t = P->n_t;
    /* Step 1: union of same-key candidates over the tables (a set). */
    int32_t n_u = 0;
    for (int t = 0; t < ORACLE_TABLES; ++t) {
        int v = P->keys_q[(int64_t)q * ORACLE_TABLES + t];
        const int32_t* st = P->start + t * 257;
        const int32_t* id = P->ids + (int64_t)t * n_t;
        for (int32_t s = st[v]; s < st[v + 1]; ++s) {
            int32_t j = id[s];
            if (seen[j] == stamp) continue;
            seen[j] = stamp;
            cand[n_u].j = j;
            n_u++;
        }
    }
    /* Epipolar constraint (geometry-aware step 3), then Step 2 Hamming
     * distances with the optional tau filter of the ranking section. */
    int32_t n_c = 0;
    const uint64_t* cq = P->codes_q + (int64_t)q * 2;
    for (int32_t u = 0; u < n_u; ++u) {
        int32_t j = cand[u].j;
        if (P->kp_q) {
            double x = P->kp_q[(int64_t)q * 2], y = P->kp_q[(int64_t)q * 2 + 1];
            double xp = P->kp_t[(int64_t)j * 2], yp = P->kp_t[(int64_t)j * 2 + 1];
            if (!within_band(P->F, x, y, xp, yp, P->max_px)) continue;
        }
        const uint64_t* cj = P->codes_t + (int64_t)j * 2;
        int32_t h = popcount64(cq[0] ^ cj[0]) + popcount64(cq[1] ^ cj[1]);
        if (h > P->prm->tau) continue;
        cand[n_c].ham = h;
        cand[n_c].j = j;
        n_c++;
    }
    /* Step 3: the k smallest (Hamming distance, index). */
    qsort(cand, (size_t)n_c, sizeof(ranked_t), cmp_ranked);
    int32_t n_k = n_c < P->prm->k ? n_c : P->prm->k;
    /* Step 4: exact squared Euclidean distances and the ratio test. */
    int32_t best_j = -1, best_d = 0;
    const uint8_t* a = P->desc_q + (int64_t)q * ORACLE_DIM;
    for (int32_t s = 0; s < n_k; ++s) {
        const uint8_t* b = P->desc_t + (int64_t)cand[s].j * ORACLE_DIM;
        int32_t d = 0;
        for (int i = 0; i < ORACLE_DIM; ++i) {
            int32_t diff = (int32_t)a[i] - (int32_t)b[i];
            d += diff * diff;
        }
        dist[s] = d;
        if (best_j < 0 || d < best_d || (d == best_d && cand[s].j < best_j)) {
            best_d = d;
            best_j = cand[s].j;
        }
    }
    qsort(dist, (size_t)n_k, sizeof(int32_t), cmp_i32);
    int32_t d1 = n_k >= 1 ? dist[0] : -1;
    int32_t d2 = n_k >= 2 ? dist[1] : -1;
    int64_t num = P->prm->ratio_num, den = P->prm->ratio_den;
    int ok = n_k >= 2 && den * den * (int64_t)d1 < num * num * (int64_t)d2;
    *out_idx = ok ? best_j : -1;
    *out_d1 = d1;
    *out_d2 = d2;
}

static void match_range(const pair_ctx* P, const int32_t* q_idx, int64_t lo, int64_t hi,
                        int32_t* match_idx, int32_t* d1sq, int32_t* d2sq) {
    int32_t n_alloc = P->n_t > 0 ? P->n_t : 1;
    int32_t* seen = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_alloc);
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_alloc);
    ranked_t* cand = (ranked_t*)malloc(sizeof(ranked_t) * (size_t)n_alloc);
    for (int32_t j = 0; j < n_alloc; ++j) seen[j] = -1;
    int32_t stamp = 0;
    for (int64_t s = lo; s < hi; ++s, ++stamp) {
        int32_t q = q_idx ? q_idx[s] : (int32_t)s;
        match_one(P, q, stamp, seen, cand, dist, match_idx + s, d1sq + s, d2sq + s);
    }
    free(seen);
    free(dist);
    free(cand);
}

static int32_t* alloc_buckets_ids(int32_t n_t) {
    return (int32_t*)malloc(sizeof(int32_t) * (size_t)ORACLE_TABLES * (size_t)(n_t > 0 ? n_t : 1));
}

void oracle_match_pair(const uint8_t* desc_q, const uint64_t* codes_q, const uint8_t* keys_q, int32_t n_q,
                       const uint8_t* desc_t, const uint64_t* codes_t, const uint8_t* keys_t, int32_t n_t,
                       const oracle_params* prm,
                       const float* kp_q, const float* kp_t, const double* F, double max_px,
                       const int32_t* q_idx, int32_t n_sel,
                       int32_t* match_idx, int32_t* d1sq, int32_t* d2sq) {
    int32_t start[ORACLE_TABLES * 257];
    int32_t* ids = alloc_buckets_ids(n_t);
    build_buckets(keys_t, n_t, start, ids);
    pair_ctx P = {desc_q, desc_t, codes_q, codes_t, keys_q, keys_t, n_q, n_t, prm,
                  kp_q, kp_t, F, max_px, start, ids};
    int64_t n = q_idx ? n_sel : n_q;
    const int64_t chunk = 256;
    int64_t n_chunks = (n + chunk - 1) / chunk;
#pragma omp parallel for schedule(dynamic)
    for (int64_t c = 0; c < n_chunks; ++c) {
        int64_t lo = c * chunk, hi = lo + chunk < n ? lo + chunk : n;
        match_range(&P, q_idx, lo, hi, match_idx, d1sq, d2sq);
    }
    free(ids);
}

void oracle_match_pairs(int32_t n_images, const uint8_t* const* desc, const uint64_t* const* codes,
                        const uint8_t* const* keys, const int32_t* n_feat,
                        int64_t n_pairs, const int32_t* pairs, const oracle_params* prm,
                        const float* const* kp, const double* F, double max_px,
                        int32_t* match_idx, int32_t* d1sq, int32_t* d2sq) {
    (void)n_images;
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_pairs + 1));
    off[0] = 0;
    for (int64_t p = 0; p < n_pairs; ++p) off[p + 1] = off[p] + n_feat[pairs[2 * p]];
#pragma omp parallel for schedule(dynamic)
    for (int64_t p = 0; p < n_pairs; ++p) {
        int32_t qi = pairs[2 * p], ti = pairs[2 * p + 1];
        int32_t start[ORACLE_TABLES * 257];
        int32_t* ids = alloc_buckets_ids(n_feat[ti]);
        build_buckets(keys[ti], n_feat[ti], start, ids);
        pair_ctx P = {desc[qi], desc[ti], codes[qi], codes[ti], keys[qi], keys[ti],
                      n_feat[qi], n_feat[ti], prm,
                      kp ? kp[qi] : NULL, kp ? kp[ti] : NULL, F ? F + 9 * p : NULL, max_px, start, ids};
        match_range(&P, NULL, 0, n_feat[qi], match_idx + off[p], d1sq + off[p], d2sq + off[p]);
        free(ids);
    }
    free(off);
}
