// Geometry-aware first stage on gfx950 (Sec. 3.1 of the paper): the
// largest-scale fifth of each image's features is matched first, a
// fundamental matrix is estimated from each pair's matches, and only pairs
// whose matches are mostly inliers of it go on to epipolar-guided matching
// (Eq. 1-2).  The paper does not spell out its estimator; this one is RANSAC
// over Hartley-normalised eight-point hypotheses with a least-squares refit:
//
//   subset      ceil(n num / den) largest scales (IEEE total order of the
//               float32 value), lower index first on ties, ascending order
//   sampling    Floyd's algorithm over the pair's match list, one 32-bit
//               uniform draw per pick: v = floor(r (j + 1) / 2^32) for
//               j = n-8 .. n-1, replaced by j if already taken
//   hypothesis  null vector (f8 = 1) of the 8 x 9 design matrix of the
//               normalised sample by Gaussian elimination with partial
//               pivoting; rank 2 by F <- F (I - v v^T), v the eigenvector of
//               F^T F with the smallest eigenvalue (cyclic Jacobi, 6 sweeps);
//               back to pixels with F <- T_t^T F T_q
//   inlier      e^2 <= thr^2 (a^2 + b^2) with (a, b, c) = F (x, y, 1) and
//               e = a x' + b y' + c (the band test of Eq. 2)
//   best        most inliers, lowest hypothesis index on ties
//   refit       smallest eigenvector of A^T A over the best's inliers (cyclic
//               Jacobi, 10 sweeps), rank 2, pixels; inliers counted again
//   accept      n >= min_matches and 3 inliers >= 2 n
//
// Every step is binary64 in the order written (the library is compiled
// without fp contraction), and every sum runs sequentially in match order, so
// results are reproducible bit for bit.  Jacobi rotations use the symmetric
// Schur pair theta = (a_qq - a_pp) / (2 a_pq), t = sign(theta) / (|theta| +
// sqrt(theta^2 + 1)), c = 1 / sqrt(t^2 + 1), s = t c, applied to columns p, q,
// then rows p, q, then to the accumulated eigenvectors; planes with a_pq == 0
// are skipped.
#include "cashash_device.h"
#include "cashash_launch.h"

namespace cashash {

namespace {

constexpr double kSqrt2 = 1.4142135623730951;
enum { kAccept = 0, kFewMatches = 1, kDegenerate = 2, kFewInliers = 3 };

// IEEE total order of a float32 as an unsigned key (larger key, larger value).
__device__ __forceinline__ uint32_t scale_key(float s) {
    const uint32_t b = __float_as_uint(s);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Exclusive rank of `flag` among the block's 256 threads, in thread order,
// and the block's total.  wtot: 4 words of LDS.  Contains two barriers.
__device__ __forceinline__ uint32_t block_rank(bool flag, uint32_t* wtot, uint32_t* total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long b = __ballot(flag);
    if (lane == 0) wtot[wv] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t r = (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
    for (int w = 0; w < wv; ++w) r += wtot[w];
    *total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
    __syncthreads();
    return r;
}

}  // namespace

// ---------------------------------------------------------------- top scale
// One block per image.  Radix select over the 32-bit order keys, eight bits
// per pass from the top: each pass histograms the keys that share the digits
// chosen so far and picks the bin holding the rem-th largest.  The threshold
// key T and the number rem of keys equal to T that are taken come out of the
// fourth pass; a final pass writes, in index order, every key above T and the
// first rem keys equal to T.
__global__ __launch_bounds__(256) void top_scale_kernel(const SelectImg* __restrict__ imgs) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_pick[2];
    __shared__ uint32_t wtot[4];
    const SelectImg im = imgs[blockIdx.x];
    if (im.m <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63;
    uint32_t prefix = 0, pmask = 0, rem = (uint32_t)im.m;
    for (int shift = 24; shift >= 0; shift -= 8) {
        hist[tid] = 0;
        __syncthreads();
        for (int i = tid; i < im.n; i += 256) {
            const uint32_t k = scale_key(im.scale[i]);
            if ((k & pmask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid < 64) {
            // lane l holds bins 255-4l .. 252-4l, descending
            const int b0 = 255 - 4 * lane;
            const uint32_t h0 = hist[b0], h1 = hist[b0 - 1], h2 = hist[b0 - 2], h3 = hist[b0 - 3];
            const uint32_t sum = h0 + h1 + h2 + h3;
            uint32_t inc = sum;
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t v = __shfl_up(inc, d);
                if (lane >= d) inc += v;
            }
            const unsigned long long hit = __ballot(inc >= rem);
            if (lane == __ffsll((long long)hit) - 1) {
                uint32_t acc = inc - sum;
                int b = b0;
                if (acc + h0 < rem) {
                    acc += h0;
                    b = b0 - 1;
                    if (acc + h1 < rem) {
                        acc += h1;
                        b = b0 - 2;
                        if (acc + h2 < rem) {
                            acc += h2;
                            b = b0 - 3;
                        }
                    }
                }
                s_pick[0] = (uint32_t)b;
                s_pick[1] = rem - acc;
            }
        }
        __syncthreads();
        prefix |= s_pick[0] << shift;
        pmask |= 255u << shift;
        rem = s_pick[1];
    }
    uint32_t base = 0, base_eq = 0;
    for (int c0 = 0; c0 < im.n; c0 += 256) {
        const int i = c0 + tid;
        const uint32_t k = i < im.n ? scale_key(im.scale[i]) : 0u;
        const bool eq = i < im.n && k == prefix;
        uint32_t n_eq, n_take;
        const uint32_t eq_rank = base_eq + block_rank(eq, wtot, &n_eq);
        const bool take = (i < im.n && k > prefix) || (eq && eq_rank < rem);
        const uint32_t pos = base + block_rank(take, wtot, &n_take);
        if (take && pos < (uint32_t)im.m) im.rows_out[pos] = i;
        base += n_take;
        base_eq += n_eq;
    }
}

// ---------------------------------------------------------------- row gather
// 8 threads per row: each copies 16 descriptor bytes; threads 0-2 of the row
// also copy the code, the keys and the keypoint.  Rows outside the source
// image set bit 0 of *err and are skipped.
__global__ __launch_bounds__(256) void gather_rows_kernel(const GatherImg* __restrict__ imgs,
                                                          const RowChunk* __restrict__ chunks, int n_chunks,
                                                          unsigned* __restrict__ err) {
    const int rr = threadIdx.x >> 3, part = threadIdx.x & 7;
    for (int c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const RowChunk ch = chunks[c];
        if (rr >= ch.nr) continue;
        const GatherImg g = imgs[ch.img];
        const int j = ch.r0 + rr;
        const int32_t src = g.rows[j];
        if (src < 0 || src >= g.n) {
            if (part == 0) atomicOr(err, 1u);
            continue;
        }
        if (g.o_desc)
            reinterpret_cast<uint4*>(g.o_desc + (size_t)j * kDim)[part] =
                reinterpret_cast<const uint4*>(g.desc + (size_t)src * kDim)[part];
        if (part == 0 && g.o_codes) {
            g.o_codes[2 * (size_t)j] = g.codes[2 * (size_t)src];
            g.o_codes[2 * (size_t)j + 1] = g.codes[2 * (size_t)src + 1];
        }
        if (part == 1 && g.o_keys) {
            const uint16_t* s = reinterpret_cast<const uint16_t*>(g.keys + (size_t)src * kTables);
            uint16_t* d = reinterpret_cast<uint16_t*>(g.o_keys + (size_t)j * kTables);
            d[0] = s[0];
            d[1] = s[1];
            d[2] = s[2];
        }
        if (part == 2 && g.o_kp) {
            g.o_kp[2 * (size_t)j] = g.kp[2 * (size_t)src];
            g.o_kp[2 * (size_t)j + 1] = g.kp[2 * (size_t)src + 1];
        }
    }
}

// ---------------------------------------------------------------- fundamental matrix
namespace {

struct Norm2 {
    double s, cx, cy;
};

// Normalised coordinates of a pixel point.
__device__ __forceinline__ double nx(const Norm2& N, float x) { return N.s * ((double)x - N.cx); }
__device__ __forceinline__ double ny(const Norm2& N, float y) { return N.s * ((double)y - N.cy); }

// Eq. 2 band test with d^2 = dd.
__device__ __forceinline__ bool inlier(const double (&F)[9], float4 m, double dd) {
    const double x = (double)m.x, y = (double)m.y;
    const double la = (F[0] * x + F[1] * y) + F[2];
    const double lb = (F[3] * x + F[4] * y) + F[5];
    const double lc = (F[6] * x + F[7] * y) + F[8];
    const double e = (la * (double)m.z + lb * (double)m.w) + lc;
    return e * e <= dd * (la * la + lb * lb);
}

// One symmetric Schur rotation's (c, s) for plane (p, q).
__device__ __forceinline__ void schur(double app, double aqq, double apq, double& c, double& s) {
    const double theta = (aqq - app) / (2.0 * apq);
    double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
    if (theta < 0.0) t = -t;
    c = 1.0 / sqrt(t * t + 1.0);
    s = t * c;
}

// F <- F (I - v v^T) with v the eigenvector of F^T F of the smallest
// eigenvalue; 3 x 3 cyclic Jacobi held in registers.
__device__ __forceinline__ void rank2(double (&F)[9]) {
    double M[3][3], V[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            M[i][j] = (F[i] * F[j] + F[3 + i] * F[3 + j]) + F[6 + i] * F[6 + j];
            V[i][j] = i == j ? 1.0 : 0.0;
        }
#pragma unroll 1
    for (int sw = 0; sw < kJacobiSweeps3; ++sw) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = p + 1; q < 3; ++q) {
                if (M[p][q] == 0.0) continue;
                double c, s;
                schur(M[p][p], M[q][q], M[p][q], c, s);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double akp = M[k][p], akq = M[k][q];
                    M[k][p] = c * akp - s * akq;
                    M[k][q] = s * akp + c * akq;
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double apk = M[p][k], aqk = M[q][k];
                    M[p][k] = c * apk - s * aqk;
                    M[q][k] = s * apk + c * aqk;
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    // smallest diagonal entry, first on ties.  The entries pass through an
    // empty asm so the selects below stay register selects (otherwise the
    // compiler turns them into one indexed load and keeps M, V in scratch).
    double d0 = M[0][0], d1 = M[1][1], d2 = M[2][2];
    double w00 = V[0][0], w10 = V[1][0], w20 = V[2][0], w01 = V[0][1], w11 = V[1][1], w21 = V[2][1];
    double w02 = V[0][2], w12 = V[1][2], w22 = V[2][2];
    asm volatile("" : "+v"(d0), "+v"(d1), "+v"(d2), "+v"(w00), "+v"(w10), "+v"(w20));
    asm volatile("" : "+v"(w01), "+v"(w11), "+v"(w21), "+v"(w02), "+v"(w12), "+v"(w22));
    double dmin = d0, v0 = w00, v1 = w10, v2 = w20;
    if (d1 < dmin) {
        dmin = d1;
        v0 = w01;
        v1 = w11;
        v2 = w21;
    }
    if (d2 < dmin) {
        v0 = w02;
        v1 = w12;
        v2 = w22;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double w = (F[3 * i] * v0 + F[3 * i + 1] * v1) + F[3 * i + 2] * v2;
        F[3 * i + 0] = F[3 * i + 0] - w * v0;
        F[3 * i + 1] = F[3 * i + 1] - w * v1;
        F[3 * i + 2] = F[3 * i + 2] - w * v2;
    }
}

// Normalised-coordinate matrix back to pixels: F = T_t^T Fn T_q with
// T = [[s, 0, -s cx], [0, s, -s cy], [0, 0, 1]].
__device__ __forceinline__ void to_pixels(const double (&Fn)[9], const Norm2& Q, const Norm2& T, double (&F)[9]) {
    const double txq = -(Q.s * Q.cx), tyq = -(Q.s * Q.cy);
    const double txt = -(T.s * T.cx), tyt = -(T.s * T.cy);
    double G[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        G[3 * i + 0] = Fn[3 * i + 0] * Q.s;
        G[3 * i + 1] = Fn[3 * i + 1] * Q.s;
        G[3 * i + 2] = (Fn[3 * i + 0] * txq + Fn[3 * i + 1] * tyq) + Fn[3 * i + 2];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F[j] = T.s * G[j];
        F[3 + j] = T.s * G[3 + j];
        F[6 + j] = (txt * G[j] + tyt * G[3 + j]) + G[6 + j];
    }
}

// Design row of p'^T F p = 0 for normalised (x, y) <-> (u, v), F row-major.
__device__ __forceinline__ void design_row(double x, double y, double u, double v, double* a) {
    a[0] = u * x;
    a[1] = u * y;
    a[2] = u;
    a[3] = v * x;
    a[4] = v * y;
    a[5] = v;
    a[6] = x;
    a[7] = y;
    a[8] = 1.0;
}

// Null vector of the 8 x 9 matrix with f8 = 1 (partial pivoting, first row
// of the largest |a| on ties); false if a pivot is exactly zero.
__device__ __forceinline__ bool null8(double (&A)[8][9], double (&f)[9]) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        double best = fabs(A[c][c]);
        int p = c;
#pragma unroll
        for (int r = c + 1; r < 8; ++r) {
            const double v = fabs(A[r][c]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (best == 0.0) return false;
#pragma unroll
        for (int r = c + 1; r < 8; ++r)
            if (p == r) {
#pragma unroll
                for (int k = c; k < 9; ++k) {
                    const double t = A[c][k];
                    A[c][k] = A[r][k];
                    A[r][k] = t;
                }
            }
#pragma unroll
        for (int r = c + 1; r < 8; ++r) {
            const double g = A[r][c] / A[c][c];
#pragma unroll
            for (int k = c + 1; k < 9; ++k) A[r][k] = A[r][k] - g * A[c][k];
        }
    }
    f[8] = 1.0;
#pragma unroll
    for (int c = 7; c >= 0; --c) {
        double acc = 0.0;
#pragma unroll
        for (int k = c + 1; k < 9; ++k) acc = acc + A[c][k] * f[k];
        f[c] = -(acc / A[c][c]);
    }
    return true;
}

}  // namespace

// One block of 256 threads per pair.  The pair's stage-1 matches are
// compacted (ascending query order) into LDS as (x, y, x', y'); thread 0
// computes the two normalisations; each thread runs hypotheses h = tid,
// tid + 256, ... entirely in registers and counts their inliers against the
// LDS list; the block picks the best; 45 threads accumulate the upper
// triangle of A^T A over its inliers, each sequentially in match order;
// wave 0 runs the 9 x 9 Jacobi with one lane per row / column of each
// rotation; thread 0 finishes the refit and the block counts its inliers.
__global__ __launch_bounds__(256) void fundamental_kernel(const GeoImg* __restrict__ imgs,
                                                          const GeoPair* __restrict__ pairs,
                                                          const int32_t* __restrict__ match_idx,
                                                          const uint32_t* __restrict__ rnd, GeoParams prm,
                                                          GeoOut out, unsigned* __restrict__ err) {
    extern __shared__ __attribute__((aligned(16))) uint8_t dyn[];
    float4* pts = reinterpret_cast<float4*>(dyn);
    uint8_t* flag = dyn + (size_t)16 * prm.cap;
    __shared__ double sA[81], sV[81], sF[9], s_norm[6];
    __shared__ uint32_t wtot[4];
    __shared__ unsigned long long s_best[4];
    __shared__ int32_t s_ok;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t p = blockIdx.x;
    const GeoPair pr = pairs[p];
    const GeoImg Q = imgs[pr.qi], T = imgs[pr.ti];

    // stage-1 matches, ascending query order
    uint32_t n = 0;
    for (int c0 = 0; c0 < Q.n; c0 += 256) {
        const int q = c0 + tid;
        int32_t m = q < Q.n ? match_idx[pr.out + q] : -1;
        if (m >= T.n) {
            atomicOr(err, 2u);
            m = -1;
        }
        uint32_t tot;
        const uint32_t pos = n + block_rank(m >= 0, wtot, &tot);
        if (m >= 0 && pos < (uint32_t)prm.cap)
            pts[pos] = make_float4(Q.kp[2 * q], Q.kp[2 * q + 1], T.kp[2 * m], T.kp[2 * m + 1]);
        n += tot;
    }
    auto finish = [&](int st, int ni, int bh) {
        out.n_matches[p] = (int32_t)n;
        out.n_inliers[p] = ni;
        out.best_h[p] = bh;
        out.status[p] = st;
    };
    if (n > (uint32_t)prm.cap) {
        if (tid == 0) {
            atomicOr(err, 4u);
            for (int i = 0; i < 9; ++i) out.F[9 * p + i] = 0.0;
            finish(kDegenerate, 0, -1);
        }
        return;
    }
    if ((int)n < prm.min_matches || n < 8) {
        if (tid < 9) out.F[9 * p + tid] = 0.0;
        if (tid == 0) finish(kFewMatches, 0, -1);
        return;
    }
    __syncthreads();

    // Hartley normalisation of both point sets (sequential sums)
    if (tid == 0) {
        double sx = 0.0, sy = 0.0, su = 0.0, sv = 0.0;
        for (uint32_t i = 0; i < n; ++i) {
            const float4 m = pts[i];
            sx = sx + (double)m.x;
            sy = sy + (double)m.y;
            su = su + (double)m.z;
            sv = sv + (double)m.w;
        }
        const double dn = (double)n;
        const double cx = sx / dn, cy = sy / dn, cu = su / dn, cv = sv / dn;
        double dq = 0.0, dt = 0.0;
        for (uint32_t i = 0; i < n; ++i) {
            const float4 m = pts[i];
            const double dx = (double)m.x - cx, dy = (double)m.y - cy;
            const double du = (double)m.z - cu, dv = (double)m.w - cv;
            dq = dq + sqrt(dx * dx + dy * dy);
            dt = dt + sqrt(du * du + dv * dv);
        }
        s_ok = (dq > 0.0) && (dt > 0.0);
        s_norm[0] = kSqrt2 / (dq / dn);
        s_norm[1] = cx;
        s_norm[2] = cy;
        s_norm[3] = kSqrt2 / (dt / dn);
        s_norm[4] = cu;
        s_norm[5] = cv;
    }
    __syncthreads();
    if (!s_ok) {
        if (tid < 9) out.F[9 * p + tid] = 0.0;
        if (tid == 0) finish(kDegenerate, 0, -1);
        return;
    }
    const Norm2 NQ{s_norm[0], s_norm[1], s_norm[2]}, NT{s_norm[3], s_norm[4], s_norm[5]};
    const double dd = prm.thr * prm.thr;

    // hypotheses: pixel-space matrix of hypothesis h, false if unsolvable
    auto hypothesis = [&](int h, double (&Fh)[9]) -> bool {
        int idx[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int j = (int)n - 8 + i;
            int v = (int)(((uint64_t)rnd[8 * (size_t)h + i] * (uint64_t)(j + 1)) >> 32);
#pragma unroll
            for (int a = 0; a < i; ++a)
                if (idx[a] == v) v = j;
            idx[i] = v;
        }
        double A[8][9];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const float4 m = pts[idx[r]];
            design_row(nx(NQ, m.x), ny(NQ, m.y), nx(NT, m.z), ny(NT, m.w), A[r]);
        }
        double f[9];
        if (!null8(A, f)) return false;
        rank2(f);
        to_pixels(f, NQ, NT, Fh);
        return true;
    };
    int best_c = -1, best_h = 0x7FFFFFFF;
    for (int h = tid; h < prm.n_hyp; h += 256) {
        double Fh[9];
        if (!hypothesis(h, Fh)) continue;
        int cnt = 0;
        for (uint32_t i = 0; i < n; ++i) cnt += inlier(Fh, pts[i], dd) ? 1 : 0;
        if (cnt > best_c) {
            best_c = cnt;
            best_h = h;
        }
    }
    // block argmax of (count, -h); the winning thread rebuilds its matrix
    unsigned long long key = ((unsigned long long)(uint32_t)(best_c + 1) << 32) | (uint32_t)(0x7FFFFFFF - best_h);
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(key, d);
        key = o > key ? o : key;
    }
    if (lane == 0) s_best[wv] = key;
    __syncthreads();
    unsigned long long top = s_best[0];
    for (int w = 1; w < 4; ++w) top = s_best[w] > top ? s_best[w] : top;
    const int bc = (int)(top >> 32) - 1;
    const int bh = 0x7FFFFFFF - (int)(uint32_t)(top & 0xFFFFFFFFull);
    if (bc < 8) {
        if (tid < 9) out.F[9 * p + tid] = 0.0;
        if (tid == 0) finish(kDegenerate, 0, bc >= 0 ? bh : -1);
        return;
    }
    if (best_h == bh) {
        double Fh[9];
        hypothesis(bh, Fh);
#pragma unroll
        for (int i = 0; i < 9; ++i) sF[i] = Fh[i];
    }
    __syncthreads();

    // refit: inlier flags of the best hypothesis, then A^T A (upper triangle,
    // one thread per entry, sequential over matches)
    {
        double F[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) F[i] = sF[i];
        for (uint32_t i = tid; i < n; i += 256) flag[i] = inlier(F, pts[i], dd) ? 1 : 0;
    }
    __syncthreads();
    if (tid < 45) {
        int r = 0, k = tid;
        while (k >= 9 - r) {
            k -= 9 - r;
            ++r;
        }
        const int c = r + k;
        double acc = 0.0;
        for (uint32_t i = 0; i < n; ++i) {
            if (!flag[i]) continue;
            const float4 m = pts[i];
            double a[9];
            design_row(nx(NQ, m.x), ny(NQ, m.y), nx(NT, m.z), ny(NT, m.w), a);
            double ar = a[0], ac = a[0];
#pragma unroll
            for (int j = 1; j < 9; ++j) {
                ar = r == j ? a[j] : ar;
                ac = c == j ? a[j] : ac;
            }
            acc = acc + ar * ac;
        }
        sA[r * 9 + c] = acc;
        sA[c * 9 + r] = acc;
    }
    if (tid < 81) sV[tid] = (tid % 10 == 0) ? 1.0 : 0.0;
    __syncthreads();
    if (wv == 0) {
        const int k = lane < 9 ? lane : 0;
        for (int sw = 0; sw < kJacobiSweeps9; ++sw)
            for (int pp = 0; pp < 8; ++pp)
                for (int qq = pp + 1; qq < 9; ++qq) {
                    const double apq = sA[pp * 9 + qq];
                    if (apq == 0.0) continue;
                    double c, s;
                    schur(sA[pp * 9 + pp], sA[qq * 9 + qq], apq, c, s);
                    if (lane < 9) {
                        const double akp = sA[k * 9 + pp], akq = sA[k * 9 + qq];
                        sA[k * 9 + pp] = c * akp - s * akq;
                        sA[k * 9 + qq] = s * akp + c * akq;
                    }
                    wave_sync();
                    if (lane < 9) {
                        const double apk = sA[pp * 9 + k], aqk = sA[qq * 9 + k];
                        sA[pp * 9 + k] = c * apk - s * aqk;
                        sA[qq * 9 + k] = s * apk + c * aqk;
                        const double vkp = sV[k * 9 + pp], vkq = sV[k * 9 + qq];
                        sV[k * 9 + pp] = c * vkp - s * vkq;
                        sV[k * 9 + qq] = s * vkp + c * vkq;
                    }
                    wave_sync();
                }
        if (lane == 0) {
            int m = 0;
            for (int i = 1; i < 9; ++i)
                if (sA[i * 9 + i] < sA[m * 9 + m]) m = i;
            double f[9], F[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = sV[i * 9 + m];
            rank2(f);
            to_pixels(f, NQ, NT, F);
#pragma unroll
            for (int i = 0; i < 9; ++i) sF[i] = F[i];
        }
    }
    __syncthreads();
    double F[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) F[i] = sF[i];
    uint32_t cnt = 0;
    for (uint32_t i = tid; i < n; i += 256) cnt += inlier(F, pts[i], dd) ? 1u : 0u;
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d);
    if (lane == 0) wtot[wv] = cnt;
    __syncthreads();
    if (tid < 9) out.F[9 * p + tid] = sF[tid];
    if (tid == 0) {
        const int ni = (int)(wtot[0] + wtot[1] + wtot[2] + wtot[3]);
        finish(3ll * ni >= 2ll * (long long)n ? kAccept : kFewInliers, ni, bh);
    }
}

hipError_t launch_top_scale(hipStream_t s, const SelectImg* imgs, int n_images) {
    if (n_images <= 0) return hipSuccess;
    hipLaunchKernelGGL(top_scale_kernel, dim3(n_images), dim3(256), 0, s, imgs);
    return hipGetLastError();
}

hipError_t launch_gather_rows(hipStream_t s, const GatherImg* imgs, const RowChunk* chunks, int n_chunks,
                              unsigned* err) {
    if (n_chunks <= 0) return hipSuccess;
    const int grid = n_chunks < 65536 ? n_chunks : 65536;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(grid), dim3(256), 0, s, imgs, chunks, n_chunks, err);
    return hipGetLastError();
}

size_t fundamental_lds_bytes(int cap) { return (size_t)cap * 17; }

hipError_t launch_fundamental(hipStream_t s, const GeoImg* imgs, const GeoPair* pairs, int64_t n_pairs,
                              const int32_t* match_idx, const uint32_t* rnd, const GeoParams& prm, const GeoOut& out,
                              unsigned* err) {
    if (n_pairs <= 0) return hipSuccess;
    const size_t lds = (fundamental_lds_bytes(prm.cap) + 15) & ~size_t(15);
    if (lds > 65536) {
        // dynamic LDS beyond 64 KB has to be allowed explicitly
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fundamental_kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fundamental_kernel, dim3((unsigned)n_pairs), dim3(256), lds, s, imgs, pairs, match_idx, rnd,
                       prm, out, err);
    return hipGetLastError();
}

}  // namespace cashash
