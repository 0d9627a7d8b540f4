/* CPU oracle for the first stage of geometry-aware CasHash matching --
 * TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
 * baseline; never linked into the GPU library).
 *
 * Sec. 3.1 of the paper: the largest-scale fifth of each image's features is
 * matched first; a pair with at least 16 such matches gets a fundamental
 * matrix estimated from them, and it goes on to guided matching only if at
 * least two thirds of those matches are inliers of that matrix.  The paper
 * names no estimator beyond "GPU fundamental matrix estimation"; the one
 * written here is RANSAC over Hartley-normalised eight-point hypotheses with
 * a least-squares refit on the best hypothesis's inliers:
 *
 *   subset      the ceil(n num / den) features of largest scale (IEEE total
 *               order of the float32 scale), lower index first on ties,
 *               listed in ascending index order
 *   sampling    eight distinct match indices per hypothesis by Floyd's
 *               algorithm, driven by eight given uniform 32-bit draws
 *   hypothesis  null vector of the 8x9 design matrix by Gaussian elimination
 *               with partial pivoting; rank 2 by removing the component along
 *               the eigenvector of F^T F with the smallest eigenvalue (cyclic
 *               Jacobi, fixed sweep count); back to pixel coordinates
 *   inlier      distance of the train point to the query point's epipolar
 *               line at most thr, tested as e^2 <= thr^2 (a^2 + b^2) (Eq. 2)
 *   best        most inliers, lowest hypothesis index on ties
 *   refit       smallest eigenvector of A^T A over the best's inliers (cyclic
 *               Jacobi), rank 2, pixel coordinates; inliers counted again
 *   accept      n >= min_matches and 3 * inliers >= 2 * n
 *
 * All arithmetic is binary64 in the order written (compiled without fp
 * contraction); every sum runs sequentially in list order.
 *
 * Parity status: pinned (numpy sorting, SVD and eigh special cases,
 * noise-free correspondences of known cameras, planted outliers, Floyd's
 * closed forms).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define JACOBI_SWEEPS_3 6
#define JACOBI_SWEEPS_9 10
#define SQRT2 1.4142135623730951

enum { GEO_ACCEPT = 0, GEO_FEW_MATCHES = 1, GEO_DEGENERATE = 2, GEO_FEW_INLIERS = 3 };

/* ---- subset by scale ---------------------------------------------------- */

static uint32_t order_key(float s) {
    uint32_t b;
    memcpy(&b, &s, sizeof b);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

typedef struct { uint32_t key; int32_t idx; } KeyIdx;

static int by_scale_desc(const void* a, const void* b) {
    const KeyIdx* x = (const KeyIdx*)a;
    const KeyIdx* y = (const KeyIdx*)b;
    if (x->key != y->key) return x->key > y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

static int by_int(const void* a, const void* b) {
    const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return x < y ? -1 : (x > y);
}

int32_t oracle_subset_size(int32_t n, int32_t num, int32_t den) {
    return (int32_t)(((int64_t)n * num + den - 1) / den);
}

/* rows[0..m) = the m largest-scale feature indices, ascending. */
void oracle_top_scale(const float* scale, int32_t n, int32_t m, int32_t* rows) {
    if (m <= 0) return;
    KeyIdx* a = (KeyIdx*)malloc(sizeof(KeyIdx) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) { a[i].key = order_key(scale[i]); a[i].idx = i; }
    qsort(a, (size_t)n, sizeof(KeyIdx), by_scale_desc);
    for (int32_t i = 0; i < m; ++i) rows[i] = a[i].idx;
    qsort(rows, (size_t)m, sizeof(int32_t), by_int);
    free(a);
}

/* ---- sampling ------------------------------------------------------------ */

/* Floyd's algorithm for 8 distinct values of [0, n), n >= 8: for
 * j = n-8 .. n-1 draw v uniform in [0, j] as floor(r (j+1) / 2^32); if v is
 * already taken, take j. */
void oracle_floyd8(const uint32_t* r, int32_t n, int32_t* out) {
    for (int i = 0; i < 8; ++i) {
        const int32_t j = n - 8 + i;
        int32_t v = (int32_t)(((uint64_t)r[i] * (uint64_t)(j + 1)) >> 32);
        for (int a = 0; a < i; ++a)
            if (out[a] == v) { v = j; break; }
        out[i] = v;
    }
}

/* ---- linear algebra ------------------------------------------------------- */

/* Cyclic Jacobi on the symmetric n x n matrix A (row-major), accumulating the
 * rotations into V (columns become eigenvectors; pass V = I).  Each rotation
 * of plane (p, q), p < q in row-major order, uses the symmetric Schur pair
 *   theta = (a_qq - a_pp) / (2 a_pq),  t = sign(theta) / (|theta| + sqrt(theta^2 + 1)),
 *   c = 1 / sqrt(t^2 + 1),  s = t c   (sign(0) = +1)
 * and is applied as A <- A J (columns p, q), then A <- J^T A (rows p, q),
 * then V <- V J, where J_pp = J_qq = c, J_pq = s, J_qp = -s.  A plane whose
 * a_pq is exactly zero is skipped. */
void oracle_jacobi(int32_t n, double* A, double* V, int32_t sweeps) {
    for (int32_t sw = 0; sw < sweeps; ++sw)
        for (int32_t p = 0; p < n - 1; ++p)
            for (int32_t q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (apq == 0.0) continue;
                const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
                if (theta < 0.0) t = -t;
                const double c = 1.0 / sqrt(t * t + 1.0);
                const double s = t * c;
                for (int32_t k = 0; k < n; ++k) {
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int32_t k = 0; k < n; ++k) {
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int32_t k = 0; k < n; ++k) {
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
}

/* Index of the smallest diagonal entry (first one on ties). */
static int32_t min_diag(int32_t n, const double* A) {
    int32_t m = 0;
    for (int32_t i = 1; i < n; ++i)
        if (A[i * n + i] < A[m * n + m]) m = i;
    return m;
}

/* Null vector of the 8 x 9 matrix A (row-major, overwritten) with f[8] = 1:
 * forward elimination with partial pivoting over columns 0..7 (largest |a|,
 * first row on ties), then back substitution.  Returns 0 if a pivot is 0. */
int32_t oracle_null8(double* A, double* f) {
    for (int c = 0; c < 8; ++c) {
        int p = c;
        double best = fabs(A[c * 9 + c]);
        for (int r = c + 1; r < 8; ++r)
            if (fabs(A[r * 9 + c]) > best) { best = fabs(A[r * 9 + c]); p = r; }
        if (best == 0.0) return 0;
        if (p != c)
            for (int k = c; k < 9; ++k) {
                const double tmp = A[c * 9 + k];
                A[c * 9 + k] = A[p * 9 + k];
                A[p * 9 + k] = tmp;
            }
        for (int r = c + 1; r < 8; ++r) {
            const double g = A[r * 9 + c] / A[c * 9 + c];
            for (int k = c + 1; k < 9; ++k) A[r * 9 + k] = A[r * 9 + k] - g * A[c * 9 + k];
        }
    }
    f[8] = 1.0;
    for (int c = 7; c >= 0; --c) {
        double acc = 0.0;
        for (int k = c + 1; k < 9; ++k) acc = acc + A[c * 9 + k] * f[k];
        f[c] = -(acc / A[c * 9 + c]);
    }
    return 1;
}

/* F <- F (I - v v^T), v the eigenvector of F^T F with the smallest
 * eigenvalue: the nearest rank-2 matrix in Frobenius norm. */
void oracle_rank2(double* F) {
    double M[9], V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            M[i * 3 + j] = (F[i] * F[j] + F[3 + i] * F[3 + j]) + F[6 + i] * F[6 + j];
    oracle_jacobi(3, M, V, JACOBI_SWEEPS_3);
    const int32_t m = min_diag(3, M);
    const double v0 = V[m], v1 = V[3 + m], v2 = V[6 + m];
    for (int i = 0; i < 3; ++i) {
        const double w = (F[3 * i] * v0 + F[3 * i + 1] * v1) + F[3 * i + 2] * v2;
        F[3 * i + 0] = F[3 * i + 0] - w * v0;
        F[3 * i + 1] = F[3 * i + 1] - w * v1;
        F[3 * i + 2] = F[3 * i + 2] - w * v2;
    }
}

/* ---- normalisation ------------------------------------------------------ */

typedef struct { double s, cx, cy; } Norm;

/* Hartley: centroid to the origin, mean distance to the centroid sqrt(2).
 * Returns 0 if all points coincide. */
static int normalise(const float* pts, int32_t n, Norm* N) {
    double sx = 0.0, sy = 0.0;
    for (int32_t i = 0; i < n; ++i) { sx = sx + (double)pts[2 * i]; sy = sy + (double)pts[2 * i + 1]; }
    const double cx = sx / (double)n, cy = sy / (double)n;
    double sd = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        const double dx = (double)pts[2 * i] - cx, dy = (double)pts[2 * i + 1] - cy;
        sd = sd + sqrt(dx * dx + dy * dy);
    }
    if (!(sd > 0.0)) return 0;
    N->s = SQRT2 / (sd / (double)n);
    N->cx = cx;
    N->cy = cy;
    return 1;
}

/* Design row of the constraint p'^T F p = 0 (p in the query image, p' in the
 * train image, F row-major), in normalised coordinates. */
static void design_row(const Norm* Nq, const Norm* Nt, const float* q, const float* t, double* a) {
    const double x = Nq->s * ((double)q[0] - Nq->cx), y = Nq->s * ((double)q[1] - Nq->cy);
    const double u = Nt->s * ((double)t[0] - Nt->cx), v = Nt->s * ((double)t[1] - Nt->cy);
    a[0] = u * x; a[1] = u * y; a[2] = u;
    a[3] = v * x; a[4] = v * y; a[5] = v;
    a[6] = x;     a[7] = y;     a[8] = 1.0;
}

/* F = T_t^T Fn T_q with T = [[s, 0, -s cx], [0, s, -s cy], [0, 0, 1]]. */
static void denormalise(const double* Fn, const Norm* Nq, const Norm* Nt, double* F) {
    const double txq = -(Nq->s * Nq->cx), tyq = -(Nq->s * Nq->cy);
    const double txt = -(Nt->s * Nt->cx), tyt = -(Nt->s * Nt->cy);
    double G[9];
    for (int i = 0; i < 3; ++i) {
        G[3 * i + 0] = Fn[3 * i + 0] * Nq->s;
        G[3 * i + 1] = Fn[3 * i + 1] * Nq->s;
        G[3 * i + 2] = (Fn[3 * i + 0] * txq + Fn[3 * i + 1] * tyq) + Fn[3 * i + 2];
    }
    for (int j = 0; j < 3; ++j) {
        F[j] = Nt->s * G[j];
        F[3 + j] = Nt->s * G[3 + j];
        F[6 + j] = (txt * G[j] + tyt * G[3 + j]) + G[6 + j];
    }
}

/* Eq. 1-2 with d = thr: the train point lies within thr of the query point's
 * epipolar line F p. */
int32_t oracle_is_inlier(const double* F, const float* q, const float* t, double thr) {
    const double x = (double)q[0], y = (double)q[1];
    const double la = (F[0] * x + F[1] * y) + F[2];
    const double lb = (F[3] * x + F[4] * y) + F[5];
    const double lc = (F[6] * x + F[7] * y) + F[8];
    const double e = (la * (double)t[0] + lb * (double)t[1]) + lc;
    return e * e <= (thr * thr) * (la * la + lb * lb);
}

static int32_t count_inliers(const double* F, const float* q, const float* t, int32_t n, double thr) {
    int32_t c = 0;
    for (int32_t i = 0; i < n; ++i) c += oracle_is_inlier(F, q + 2 * i, t + 2 * i, thr);
    return c;
}

/* Eigenvector of the smallest eigenvalue of the symmetric 9x9 matrix. */
static void smallest_eigvec9(double* A, double* f) {
    double V[81];
    for (int i = 0; i < 81; ++i) V[i] = (i % 10 == 0) ? 1.0 : 0.0;
    oracle_jacobi(9, A, V, JACOBI_SWEEPS_9);
    const int32_t m = min_diag(9, A);
    for (int i = 0; i < 9; ++i) f[i] = V[i * 9 + m];
}

/* RANSAC over normalised eight-point hypotheses for one pair's matches
 * (q[i], t[i]), i < n, float32 pixel coordinates.  rand holds 8 draws per
 * hypothesis.  Writes F (zeros unless at least one hypothesis was solved),
 * the refit's inlier count and the best hypothesis; returns the status. */
int32_t oracle_fundamental(const float* q, const float* t, int32_t n, const uint32_t* rand, int32_t n_hyp,
                           double thr, int32_t min_matches, double* F_out, int32_t* n_inliers, int32_t* best_h) {
    for (int i = 0; i < 9; ++i) F_out[i] = 0.0;
    *n_inliers = 0;
    *best_h = -1;
    if (n < min_matches || n < 8) return GEO_FEW_MATCHES;
    Norm Nq, Nt;
    if (!normalise(q, n, &Nq) || !normalise(t, n, &Nt)) return GEO_DEGENERATE;
    int32_t best_cnt = -1;
    double best_F[9];
    for (int32_t h = 0; h < n_hyp; ++h) {
        int32_t idx[8];
        oracle_floyd8(rand + 8 * (size_t)h, n, idx);
        double A[72], f[9], Fh[9];
        for (int r = 0; r < 8; ++r) design_row(&Nq, &Nt, q + 2 * idx[r], t + 2 * idx[r], A + 9 * r);
        if (!oracle_null8(A, f)) continue;
        oracle_rank2(f);
        denormalise(f, &Nq, &Nt, Fh);
        const int32_t c = count_inliers(Fh, q, t, n, thr);
        if (c > best_cnt) {
            best_cnt = c;
            *best_h = h;
            memcpy(best_F, Fh, sizeof best_F);
        }
    }
    if (best_cnt < 8) return GEO_DEGENERATE;
    /* least-squares refit on the best hypothesis's inliers */
    double N[81] = {0};
    for (int32_t i = 0; i < n; ++i) {
        if (!oracle_is_inlier(best_F, q + 2 * i, t + 2 * i, thr)) continue;
        double a[9];
        design_row(&Nq, &Nt, q + 2 * i, t + 2 * i, a);
        for (int r = 0; r < 9; ++r)
            for (int c = r; c < 9; ++c) N[r * 9 + c] = N[r * 9 + c] + a[r] * a[c];
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < r; ++c) N[r * 9 + c] = N[c * 9 + r];
    double f[9];
    smallest_eigvec9(N, f);
    oracle_rank2(f);
    denormalise(f, &Nq, &Nt, F_out);
    *n_inliers = count_inliers(F_out, q, t, n, thr);
    return 3 * (int64_t)(*n_inliers) >= 2 * (int64_t)n ? GEO_ACCEPT : GEO_FEW_INLIERS;
}

/* oracle_fundamental over many pairs (OpenMP over pairs).  Pair p's matches
 * are q[off[p] .. off[p+1]) and t[same]. */
void oracle_fundamental_batch(int32_t n_pairs, const float* q, const float* t, const int64_t* off,
                              const uint32_t* rand, int32_t n_hyp, double thr, int32_t min_matches,
                              double* F, int32_t* n_inliers, int32_t* best_h, int32_t* status) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t p = 0; p < n_pairs; ++p) {
        const int64_t o = off[p];
        status[p] = oracle_fundamental(q + 2 * o, t + 2 * o, (int32_t)(off[p + 1] - o), rand, n_hyp, thr,
                                       min_matches, F + 9 * (size_t)p, n_inliers + p, best_h + p);
    }
}
