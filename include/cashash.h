/*
 * cashash.h -- C ABI of the MI355X (gfx950) Cascade Hashing matcher.
 *
 * The library computes, for 128-d uint8 SIFT descriptors, the hot path of
 * GPU-accelerated Cascade Hashing image matching (Xu, Sun, Tao, "GPU
 * Accelerated Cascade Hashing Image Matching for Large Scale 3D
 * Reconstruction"):
 *   - hashing codes: Charikar sign random projections of mean-centred
 *     descriptors ("The Improved Parallel Calculation of Hashing Code"),
 *     128-bit remapping codes (Step 2, n = 128) and six 8-bit lookup keys
 *     (Step 1, m = 8, multiple tables);
 *   - matching of a query image I against a train image J ("Review of
 *     Cascade Hashing", Steps 1-4): union of same-key candidates over the
 *     tables, Hamming ranking to the top k, exact squared Euclidean distance
 *     ("Improved Parallel Euclidean Distance Calculation") and Lowe's ratio
 *     test;
 *   - the geometry-guided variant (Eq. 1-2): candidates restricted to a band
 *     of max_px pixels around the query's epipolar line before ranking;
 *   - the threshold tau of "Improved Parallel Hashing Ranking".
 *
 * Every step runs in hand-written HIP kernels on the current HIP device.
 * No function throws; every int-returning function returns CASHASH_OK (0) or
 * a negative error code, and cashash_last_error() gives the message.  On
 * error the contents of output buffers are unspecified.
 *
 * Buffers.  The caller owns every buffer.  Arrays of per-image pointers
 * (desc, codes, keys, kp) are host arrays; the pointers inside them, and the
 * per-query output arrays, are device pointers when cfg.mem ==
 * CASHASH_MEM_DEVICE and host pointers when cfg.mem == CASHASH_MEM_HOST (the
 * library then streams images to the device in blocks it schedules under
 * cfg.device_budget_bytes and copies results back; beyond the budget it keeps
 * two output areas of up to 2^25 queries x 12 bytes, 400 MB each, in device
 * memory and in pinned host memory).  The pair list and the
 * fundamental matrices are always host memory.  Calls are synchronous: when
 * a call returns, its outputs are complete.  The library keeps no pointer to
 * caller memory after a call returns.  One context per host thread.
 */
#ifndef CASHASH_H
#define CASHASH_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CASHASH_OK 0
#define CASHASH_E_INVAL (-1)          /* null pointer, bad size or bad index */
#define CASHASH_E_NOMEM (-2)          /* device or pinned host allocation failed, or budget too small */
#define CASHASH_E_DEVICE (-3)         /* a HIP call failed */
#define CASHASH_E_UNSAFE_MATRIX (-4)  /* a projection row is too long for the fast-path margin proof */
#define CASHASH_E_LIMIT (-5)          /* n_feat > 65535, k outside 1..64, or another hard limit */
#define CASHASH_E_IO (-6)             /* a file could not be opened, read or written, or has a bad header */

#define CASHASH_MODE_BATCHED_BF16X2 0      /* BF16 hi+lo MFMA projection; all pairs in one persistent launch */
#define CASHASH_MODE_PLAIN_FP32_PER_PAIR 1 /* FP32 VALU projection; one launch set per image pair */

#define CASHASH_MEM_HOST 0
#define CASHASH_MEM_DEVICE 1

#define CASHASH_DIM 128
#define CASHASH_TABLES 6
#define CASHASH_MAX_FEAT 65535
#define CASHASH_MAX_K 64

typedef struct {
    int32_t k;                   /* Hamming-ranked candidates kept per query, 1..64 (default 10) */
    int32_t ratio_num;           /* ratio test den^2 * D1 < num^2 * D2 on squared distances */
    int32_t ratio_den;           /*   (default 4 / 5, i.e. 0.8); both > 0 */
    int32_t max_hamming;         /* tau: candidates with Hamming distance > tau are dropped; 128 = off */
    double margin_coef;          /* fast projection trusted iff |v| > margin_coef*|x| + 2^-20*|bias| + 2^-26;
                                    otherwise recomputed in binary64 (default 1e-3) */
    int32_t mode;                /* CASHASH_MODE_* */
    int32_t mem;                 /* CASHASH_MEM_* : where image data and outputs live */
    int64_t device_budget_bytes; /* host-memory mode: device bytes for resident images (0 = 1/4 of free) */
    void* stream;                /* hipStream_t to run on, or NULL for a library-owned stream */
} cashash_config;

typedef struct {
    int32_t n_images;
    const uint8_t* const* desc; /* desc[m]: n_feat[m] x 128 uint8, row-major, row = feature index */
    const int32_t* n_feat;      /* host array, 0..65535 per image */
} cashash_images;

typedef struct {
    int64_t pairs, queries;
    int64_t bucket_entries;         /* sum over queries of the six same-key bucket sizes */
    int64_t union_size;             /* sum over queries of the candidate-set size (after the band) */
    int64_t ranked;                 /* sum over queries of the kept top-k size min(k, candidates) */
    int64_t near_margin_recomputes; /* projections recomputed in binary64 */
    int64_t h2d_bytes, d2h_bytes, image_loads;
    int64_t tile_queries;           /* matcher launch shape used: queries per work item, */
    int64_t blocks_per_cu;          /*   persistent blocks per compute unit (0 in the plain form) */
    int64_t graph_replayed;         /* 1 if the batched matcher ran as a replay of a captured HIP graph */
    double ms_codes, ms_match;      /* wall time of the call */
    int64_t disk_bytes;             /* disk level: bytes read from the set and codes files */
    int64_t group_loads;            /* disk level: groups read into host memory */
} cashash_stats;

/* Fill cfg with the defaults above. */
void cashash_default_config(cashash_config* cfg);

typedef struct cashash_ctx cashash_ctx; /* opaque: device buffers, streams, graphs, tuning */

/* Create a context on the current HIP device.
 * r_code: host float64 [128][128], row j gives code bit j.
 * r_bucket: host float64 [6][8][128], row (t, b) gives bit b of key t.
 * Both are copied.  cfg may be NULL (defaults).
 * Errors: E_INVAL (null out / matrices, bad ratio or mode), E_LIMIT (k not in
 * 1..64, max_hamming not in 0..128), E_UNSAFE_MATRIX (some row has
 * 5e-5 * |row|_2 >= margin_coef, or a non-finite entry: the fast
 * projection's rounding bound would not stay below the margin), E_DEVICE. */
int cashash_create(cashash_ctx** out, const double* r_code, const double* r_bucket,
                   const cashash_config* cfg);

/* Replace the configuration (same checks as cashash_create). */
int cashash_set_config(cashash_ctx* ctx, const cashash_config* cfg);

/* Release every resource of ctx (NULL is a no-op). */
void cashash_destroy(cashash_ctx* ctx);

/* Codes and keys of every descriptor of the image set (the paper's hash-code
 * module).  The mean used for centring is the mean over ALL descriptors of
 * `images`.  Output per image m (buffers of the caller, on the side given by
 * cfg.mem):
 *   codes_out[m]: uint64 [n_feat[m]][2]; bit j (row j of r_code) is bit j&63
 *                 of word j>>6; bit = [r_j . (x - mean) > 0], exact zero -> 0.
 *   keys_out[m] : uint8 [n_feat[m]][6]; bit b of byte t is row (t, b).
 * Every bit equals the sign of the binary64 fused multiply-add chain over
 * components 0..127 of r_j . (N x - S), with S the column sums and N the
 * descriptor count.  stats may be NULL. */
int cashash_build_codes(cashash_ctx* ctx, const cashash_images* images,
                        uint64_t* const* codes_out, uint8_t* const* keys_out, cashash_stats* stats);

/* Match each (query image, train image) pair (Steps 1-4).
 * codes / keys: as produced by cashash_build_codes for these images.
 * pairs: host int32 [n_pairs][2] = (query, train); q == t is allowed.
 * Outputs, flat over pairs: pair p occupies n_feat[pairs[p][0]] entries
 * starting at the sum of n_feat[pairs[p'][0]] over p' < p.  Per query q:
 *   match_idx: train index of the nearest kept candidate if the ratio test
 *              passes, else -1 (fewer than two candidates never pass);
 *   d1sq     : smallest squared Euclidean distance over the kept candidates,
 *              -1 if none;
 *   d2sq     : second smallest (counting multiplicity), -1 if fewer than two.
 * Kept candidates: the k smallest (Hamming distance, train index) of the set
 * union of the train points that share a key with q in any table, after
 * dropping Hamming distance > max_hamming.  Ties in the nearest distance go
 * to the smaller index.  stats may be NULL. */
int cashash_match_pairs(cashash_ctx* ctx, const cashash_images* images,
                        const uint64_t* const* codes, const uint8_t* const* keys,
                        int64_t n_pairs, const int32_t* pairs,
                        int32_t* match_idx, int32_t* d1sq, int32_t* d2sq, cashash_stats* stats);

/* cashash_match_pairs with the epipolar constraint of Eq. 1-2 applied to the
 * candidate set before ranking: candidate (x', y') of query (x, y) is kept iff
 * e^2 <= max_px^2 (a^2 + b^2), where (a, b, c) = F (x, y, 1) and
 * e = a x' + b y' + c, evaluated in binary64 without contraction in this
 * order: a = (F0 x + F1 y) + F2, b = (F3 x + F4 y) + F5, c = (F6 x + F7 y) + F8,
 * e = (a x' + b y') + c.
 * kp_xy[m]: float32 [n_feat[m]][2] keypoints (side given by cfg.mem).
 * F: host float64 [n_pairs][9] row-major.  max_px >= 0 and finite. */
int cashash_match_pairs_epipolar(cashash_ctx* ctx, const cashash_images* images,
                                 const uint64_t* const* codes, const uint8_t* const* keys,
                                 const float* const* kp_xy, int64_t n_pairs, const int32_t* pairs,
                                 const double* F, double max_px,
                                 int32_t* match_idx, int32_t* d1sq, int32_t* d2sq,
                                 cashash_stats* stats);

/* ---- Allocation-free matching ---------------------------------------------
 * For callers that cannot allocate device memory during a call: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * Same arguments, outputs and errors as cashash_match_pairs, with
 * cfg.mem == CASHASH_MEM_DEVICE.  Every device buffer of the call (bucket
 * tables, uploaded image and pair tables, work items, work counters,
 * statistics) is taken from one static device array of
 * CASHASH_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds from
 * its first context until the process ends; the call makes no device or
 * pinned allocation (its planning uses ordinary host memory), runs its launch
 * eagerly (no graph) with the cached or default launch shape (no tuning),
 * and clears the counters it needs before use.  Scratch bytes used, each
 * piece rounded up to 256:
 *     sum over distinct train images t of (6*257*4 + 144*n_feat[t])
 *   + 72*n_images + 4*n_train + 96*n_pairs + 16*tiles + 2048 + 64,
 * tiles = sum over pairs of ceil(n_feat[query] / tile queries) (at most 32
 * queries per tile).  A call needing more returns CASHASH_E_LIMIT before any
 * device work.  All calls on one GPU share its array: calls that overlap in
 * time on one GPU (from two threads or two contexts) race and must not be
 * issued. */
#define CASHASH_NOALLOC_SCRATCH_BYTES (32LL << 20)
int cashash_match_pairs_noalloc(cashash_ctx* ctx, const cashash_images* images,
                                const uint64_t* const* codes, const uint8_t* const* keys,
                                int64_t n_pairs, const int32_t* pairs,
                                int32_t* match_idx, int32_t* d1sq, int32_t* d2sq, cashash_stats* stats);

/* Message for the last nonzero return on this thread ("" if none). */
const char* cashash_last_error(void);

/* Host logic of CASHASH_MEM_HOST matching, exposed for inspection and tests
 * (no device call): plan the block schedule ("Three-Level Data Scheduling
 * Strategy", matching subsection) for images of img_bytes[m] device bytes and
 * the given pairs, with blocks of at most slot_bytes.  Images used by some
 * pair are packed in index order into blocks; block pairs are visited as
 * (i, i+1) .. (i, last), then (i, i), for i = 0, 1, ...; at most three blocks
 * are resident.  Outputs: number of steps and blocks, block and image loads
 * under that order, and optionally steps_out[4*s..] = (bi, bk, first, end)
 * positions into order_out (n_pairs pair indices in visiting order).
 * Errors: E_INVAL, E_NOMEM (an image alone exceeds slot_bytes). */
int cashash_plan_schedule(int32_t n_images, const int64_t* img_bytes, int64_t n_pairs, const int32_t* pairs,
                          int64_t slot_bytes, int64_t* n_steps, int64_t* n_blocks, int64_t* block_loads,
                          int64_t* image_loads, int64_t* steps_out, int64_t max_steps, int64_t* order_out);

/* Kernel-only timing of the last call's dominant kernel (the matcher), in
 * milliseconds, measured with HIP events on the stream it ran on, and the
 * number of launches it covered. */
int cashash_last_kernel_ms(cashash_ctx* ctx, double* ms, int64_t* launches);

/* ---- Geometry-aware two-stage matching ("Image Matching with Geometry-aware
 * Cascade Hashing on GPU", first stage and guided second stage) -----------
 *
 * Stage 1 matches the largest-scale fraction (default one fifth) of every
 * image's features over the given pairs; a pair with at least min_matches
 * stage-1 matches gets a fundamental matrix estimated from them and is
 * accepted iff at least two thirds of its matches are inliers of that
 * matrix; stage 2 matches all features of the accepted pairs with the
 * epipolar band of Eq. 1-2 around the estimated matrix.  The paper leaves
 * the estimator open; this library uses RANSAC over Hartley-normalised
 * eight-point hypotheses with a least-squares refit on the best hypothesis's
 * inliers, in binary64 with every sum taken sequentially in match order:
 *   - hypothesis h draws 8 distinct match indices by Floyd's algorithm from
 *     rand8[h][0..7]: for j = n-8 .. n-1, v = floor(r (j+1) / 2^32), and j
 *     instead if v was already drawn;
 *   - its matrix is the null vector (f8 = 1) of the 8 x 9 design matrix
 *     [u x, u y, u, v x, v y, v, x, y, 1] of the normalised sample (Gaussian
 *     elimination, partial pivoting), made rank 2 by removing the component
 *     along the eigenvector of F^T F with the smallest eigenvalue (cyclic
 *     Jacobi, 6 sweeps), mapped back to pixels (F = T_t^T F T_q);
 *   - a match is an inlier iff its train point lies within thr_px of the
 *     query point's epipolar line, tested exactly as the band of
 *     cashash_match_pairs_epipolar;
 *   - the best hypothesis has the most inliers (lowest index on ties); the
 *     refit takes the smallest eigenvector of A^T A over its inliers (cyclic
 *     Jacobi, 10 sweeps), rank 2, pixels, and counts inliers again.
 * These calls need cfg.mem == CASHASH_MEM_DEVICE (else E_INVAL); per-image
 * arrays hold device pointers, per-pair results are host arrays. */

#define CASHASH_GEO_ACCEPT 0        /* guided matching runs for the pair */
#define CASHASH_GEO_FEW_MATCHES 1   /* fewer than max(min_matches, 8) stage-1 matches */
#define CASHASH_GEO_DEGENERATE 2    /* coincident points or no hypothesis with >= 8 inliers */
#define CASHASH_GEO_FEW_INLIERS 3   /* 3 * inliers < 2 * matches after the refit */
#define CASHASH_GEO_MAX_MATCHES 8192 /* query points per image in cashash_estimate_fundamental */

typedef struct {
    int32_t frac_num, frac_den; /* stage-1 subset: ceil(n frac_num / frac_den) features (default 1 / 5) */
    int32_t min_matches;        /* default 16 */
    int32_t n_hyp;              /* RANSAC hypotheses, 1..2^20 (default 256) */
    double ransac_px;           /* inlier distance to the epipolar line, px (default 2.0) */
    double band_px;             /* stage-2 band half-width d of Eq. 1 (default 4.0) */
    const uint32_t* rand8;      /* host uint32 [n_hyp][8] uniform draws (required; default NULL) */
} cashash_geometric_config;

/* Fill g with the defaults above. */
void cashash_default_geometric_config(cashash_geometric_config* g);

/* ceil(n frac_num / frac_den), or -1 unless n >= 0 and 0 < frac_num <= frac_den.
 * Host only. */
int64_t cashash_subset_size(int32_t n, int32_t frac_num, int32_t frac_den);

/* Stage-1 subset of each image: rows_out[m] (device int32
 * [cashash_subset_size(n_feat[m], ..)]) receives the indices of the largest
 * scales[m] values (device float32 [n_feat[m]]), ordered by the IEEE-754
 * total order (so -0 < +0; NaN with the sign bit clear ranks above +inf),
 * lower index first on ties, written in ascending index order.
 * Errors: E_INVAL (host mode, null or misaligned pointer, bad fraction),
 * E_LIMIT (n_feat > 65535), E_DEVICE. */
int cashash_select_top_scale(cashash_ctx* ctx, int32_t n_images, const float* const* scales, const int32_t* n_feat,
                             int32_t frac_num, int32_t frac_den, int32_t* const* rows_out);

/* Row gather per image m: out row j = input row rows[m][j], j < n_rows[m],
 * for each field whose input and output arrays are both given (desc 128 B,
 * codes 2 x uint64, keys 6 B, kp 2 x float32; pass NULL for both to skip a
 * field).  All pointers inside the arrays are device pointers; alignment as
 * for matching (desc 16, codes 8, keys 2, kp 4 bytes).
 * Errors: E_INVAL (host mode, null or misaligned buffer, a row outside
 * 0..n_feat[m]-1; the other rows are copied), E_DEVICE. */
int cashash_gather_rows(cashash_ctx* ctx, int32_t n_images, const int32_t* n_feat, const int32_t* n_rows,
                        const int32_t* const* rows, const uint8_t* const* desc, const uint64_t* const* codes,
                        const uint8_t* const* keys, const float* const* kp, uint8_t* const* desc_out,
                        uint64_t* const* codes_out, uint8_t* const* keys_out, float* const* kp_out);

/* Fundamental matrix of each pair from its matches.  match_idx: device, the
 * flat match_idx output of cashash_match_pairs for the same n_feat and pairs
 * (pair p's slots follow those of the pairs before it; a slot >= 0 is a
 * match of that query point).  kp_xy[m]: device float32 [n_feat[m]][2].
 * Matches are taken in ascending query order.  Outputs, host [n_pairs]:
 * F_out [n_pairs][9] row-major (zeros unless a refit ran), n_matches,
 * n_inliers (of the refit matrix), best_hyp (the best hypothesis, -1 if
 * none was solvable or none ran; may be NULL) and status (CASHASH_GEO_*).
 * Errors: E_INVAL (host mode, null pointer, pair out of range, bad n_hyp or
 * threshold, a match index outside its train image), E_LIMIT (a query
 * image with more than CASHASH_GEO_MAX_MATCHES points), E_DEVICE. */
int cashash_estimate_fundamental(cashash_ctx* ctx, int32_t n_images, const int32_t* n_feat,
                                 const float* const* kp_xy, int64_t n_pairs, const int32_t* pairs,
                                 const int32_t* match_idx, const uint32_t* rand8, int32_t n_hyp, double thr_px,
                                 int32_t min_matches, double* F_out, int32_t* n_matches, int32_t* n_inliers,
                                 int32_t* best_hyp, int32_t* status);

/* The two stages over device-resident images: subset selection, row gather
 * and stage-1 matching into library-owned device memory, fundamental
 * matrices, then cashash_match_pairs_epipolar (band g->band_px) over the
 * accepted pairs.  Outputs: per pair (host) F_out [n_pairs][9], n_matches,
 * n_inliers, status as cashash_estimate_fundamental; per query (device) the
 * flat layout of cashash_match_pairs over ALL pairs, with every slot of a
 * pair that was not accepted set to -1.  stats: those of stage 2, with pairs
 * and queries counted over all pairs and ms_match the whole call.
 * Errors: as the calls it is made of. */
int cashash_match_pairs_geometric(cashash_ctx* ctx, const cashash_images* images, const uint64_t* const* codes,
                                  const uint8_t* const* keys, const float* const* kp_xy, const float* const* scales,
                                  int64_t n_pairs, const int32_t* pairs, const cashash_geometric_config* g,
                                  double* F_out, int32_t* n_matches, int32_t* n_inliers, int32_t* status,
                                  int32_t* match_idx, int32_t* d1sq, int32_t* d2sq, cashash_stats* stats);

/* ---- Disk level of the data scheduling ("Three-Level Data Scheduling
 * Strategy": disk -> host memory -> GPU) ------------------------------------
 *
 * The image set lives in a file; groups of images are read into host memory
 * under host_budget_bytes while a second thread reads the next group ahead,
 * and each group (pair of groups) goes through the host-memory path, which
 * streams blocks to the device under cfg.device_budget_bytes.  These calls
 * need cfg.mem == CASHASH_MEM_HOST (else E_INVAL).  Files, little-endian,
 * headers padded to 64 bytes:
 *   set file    "CASHSET1", int64 n_images, int64 flags (bit 0: keypoints),
 *               int64 prefix sums of the feature counts [n_images + 1], then
 *               at the next multiple of 64 bytes uint8 descriptors [N][128]
 *               (N = total features) and, if flagged, float32 keypoints [N][2]
 *   codes file  "CASHCOD1", int64 n_images, int64 N; at byte 64 uint64 codes
 *               [N][2], then uint8 keys [N][6]
 *   output file "CASHOUT1", int64 n_pairs, int64 T (total queries); at byte 64
 *               int32 match_idx [T], d1sq [T], d2sq [T] in the flat layout of
 *               cashash_match_pairs
 *   progress    "CASHPRG1", uint64 plan hash, int64 n_steps; at byte 64 one
 *               byte per group pair, 1 once its outputs are written and synced
 * File errors return CASHASH_E_IO. */

/* Write the set file of host images (kp_xy may be NULL). */
int cashash_set_write(const char* path, const cashash_images* images, const float* const* kp_xy);

/* Codes and keys of every descriptor of the set file (as cashash_build_codes
 * over the whole set: centred on the mean of all N descriptors) into
 * codes_path.  Two passes over groups of consecutive images, each group at
 * most host_budget_bytes / 2 of descriptors: column sums, then codes.
 * stats: disk_bytes, group_loads, near_margin_recomputes, h2d/d2h bytes. */
int cashash_build_codes_disk(cashash_ctx* ctx, const char* set_path, const char* codes_path,
                             int64_t host_budget_bytes, cashash_stats* stats);

/* Match the pairs of a set file against its codes file, writing out_path.
 * Groups hold at most host_budget_bytes / 3 (descriptors, codes and keys);
 * group pairs are visited in the scheduler's order ((i, i+1) .. (i, last),
 * then (i, i)) with two groups in progress and one read ahead.  After each
 * group pair its outputs are written and synced, then its byte in the
 * progress file (progress_path may be NULL: no resume and no syncing).
 * Outputs are written by a second thread while the next group pair runs.  A call with the same
 * set, pairs and budget skips the group pairs already marked, so an
 * interrupted run resumes where it stopped; any other progress file is reset.
 * max_steps > 0 stops after that many group pairs (0 = run to the end);
 * *steps_left (may be NULL) receives the number still to do.  The outputs
 * equal cashash_match_pairs over the same images and pairs. */
int cashash_match_pairs_disk(cashash_ctx* ctx, const char* set_path, const char* codes_path, int64_t n_pairs,
                             const int32_t* pairs, const char* out_path, const char* progress_path,
                             int64_t host_budget_bytes, int64_t max_steps, int64_t* steps_left,
                             cashash_stats* stats);

/* Device time of the last cashash_match_pairs_geometric call's four parts,
 * in milliseconds (HIP events on its stream): subset selection and gather,
 * stage-1 matching, fundamental matrices, stage 2 (fills included). */
int cashash_last_geometric_ms(cashash_ctx* ctx, double* ms4);

#ifdef __cplusplus
}
#endif
#endif
