/*
 * CPU oracle for Cascade Hashing (CasHash) pairwise SIFT matching.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-step-at-a-time
 * statement of what the matching method computes, used to check the GPU
 * library's outputs and as a timed CPU baseline.  It shares no code, header,
 * table or helper with the GPU library and must never be called by it.
 *
 * Method (paper, "Review of Cascade Hashing", Steps 1-4; "The Improved
 * Parallel Calculation of Hashing Code"; "Improved Parallel Euclidean
 * Distance Calculation"; "Improved Parallel Hashing Ranking"; Eq. 1-2 of the
 * geometry-aware section):
 *   codes   : sign bits of mean-centred random projections (Charikar LSH),
 *             128 code bits and 6 tables of 8-bit bucket keys per descriptor;
 *   Step 1  : candidates of a query = union over tables of the train points
 *             whose key equals the query's key in that table;
 *   (Eq.1-2): optionally keep only candidates within max_px of the query's
 *             epipolar line in the train image;
 *   Step 2-3: Hamming distance of 128-bit codes; keep the k candidates with
 *             smallest (Hamming distance, candidate index); optionally drop
 *             candidates with Hamming distance above tau first;
 *   Step 4  : exact squared Euclidean distances to those k, nearest accepted
 *             if it passes Lowe's ratio test (integer compare).
 *
 * Floating point: projections in IEEE binary64 as one fused multiply-add
 * chain in ascending component order; epipolar test in binary64 with no
 * contraction.  Build with -ffp-contract=off.
 */
#ifndef CASHASH_ORACLE_H
#define CASHASH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_DIM 128
#define ORACLE_CODE_BITS 128
#define ORACLE_TABLES 6
#define ORACLE_KEY_BITS 8

typedef struct {
    int32_t k;          /* number of Hamming-ranked candidates kept (>= 1) */
    int32_t ratio_num;  /* ratio test: den^2 * D1 < num^2 * D2 */
    int32_t ratio_den;
    int32_t tau;        /* drop candidates with Hamming distance > tau; 128 keeps all */
} oracle_params;

/* Column sums S[i] = sum of component i over every descriptor of every image,
 * and the descriptor count n_tot. */
void oracle_column_sums(int32_t n_images, const uint8_t* const* desc, const int32_t* n_feat,
                        int64_t* S /*[128]*/, int64_t* n_tot);

/* Codes and keys of n descriptors x[n][128] given the set's column sums.
 * r_code: [128][128] rows; r_bucket: [6][8][128] rows (row-major float64).
 * codes[n][2]: bit j of the code is row j, stored in word j>>6 at bit j&63.
 * keys[n][6]: bit b of key t is the sign of bucket row (t, b). */
void oracle_project(const uint8_t* x, int64_t n, const int64_t* S, int64_t n_tot,
                    const double* r_code, const double* r_bucket,
                    uint64_t* codes, uint8_t* keys);

/* Whole-set codes: column sums over all images, then every image's codes. */
void oracle_build_codes(int32_t n_images, const uint8_t* const* desc, const int32_t* n_feat,
                        const double* r_code, const double* r_bucket,
                        uint64_t* const* codes, uint8_t* const* keys);

/* Match queries of image Q against train image T.
 * q_idx: list of n_sel query indices to evaluate (NULL = all n_q, in order);
 * outputs are written at positions 0..n_sel-1 (or 0..n_q-1).
 * kp_q / kp_t / F: keypoints (float32 [n][2]) and row-major F (line in T =
 * F * (x, y, 1)); pass kp_q == NULL for plain matching.
 * match_idx: nearest candidate index or -1; d1sq: smallest squared distance
 * over the kept candidates or -1 if none; d2sq: second smallest (counting
 * multiplicity) or -1 if fewer than two. */
void oracle_match_pair(const uint8_t* desc_q, const uint64_t* codes_q, const uint8_t* keys_q, int32_t n_q,
                       const uint8_t* desc_t, const uint64_t* codes_t, const uint8_t* keys_t, int32_t n_t,
                       const oracle_params* prm,
                       const float* kp_q, const float* kp_t, const double* F, double max_px,
                       const int32_t* q_idx, int32_t n_sel,
                       int32_t* match_idx, int32_t* d1sq, int32_t* d2sq);

/* Match a list of (query image, train image) pairs; outputs are flat, pair p
 * at offset sum over p' < p of n_feat[pairs[p'][0]].  kp == NULL for plain
 * matching, else kp[m] per image and F[p*9..] per pair.  Pairs are processed
 * in parallel with OpenMP (OMP_NUM_THREADS). */
void oracle_match_pairs(int32_t n_images, const uint8_t* const* desc, const uint64_t* const* codes,
                        const uint8_t* const* keys, const int32_t* n_feat,
                        int64_t n_pairs, const int32_t* pairs, const oracle_params* prm,
                        const float* const* kp, const double* F, double max_px,
                        int32_t* match_idx, int32_t* d1sq, int32_t* d2sq);

/* Threads OpenMP will use (1 if built without OpenMP). */
int32_t oracle_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
