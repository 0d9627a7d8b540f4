// HIP kernels of the CasHash matcher for gfx950 (MI355X).
//
// Hash codes ("The Improved Parallel Calculation of Hashing Code"): the
// paper's one-block-per-(point, bit) reduction is replaced by a dense
// contraction on the matrix cores: descriptors (uint8, exact in bf16) times
// the projection rows split into bf16 hi + lo parts, fp32 accumulate.  A
// projection whose value lies within a proven rounding margin of zero is
// recomputed in binary64 exactly as the reference definition does it.
//
// Matching ("Review of Cascade Hashing", Steps 1-4; "Improved Parallel
// Hashing Ranking"; Eq. 1-2): one wavefront per query.  Train images are
// pre-sorted into per-table buckets whose entries carry code, keys and index,
// so a query's candidates are six contiguous runs.  The paper's per-query
// index table (a histogram over Hamming distance) is kept: a 129-bin counting
// pass in LDS finds the Hamming threshold of the k-th candidate, and ties are
// resolved by two more 256-bin counting passes over the candidate index
// (a radix select on the key (Hamming distance, index)).  Distances use
// v_dot4_u32_u8 and are exact.
#include "cashash_internal.h"

namespace cashash {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d);
        if (lane >= d) v += t;
    }
    return v;
}

// ------------------------------------------------------------------ utilities

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n, unsigned long long v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ column sums
// One block per chunk of <= 2048 rows.  Thread t reads the 16-byte column
// group t % 8 of rows t / 8, t / 8 + 32, ...; partial column totals meet in
// LDS and each column is added to the int64 sums with one atomic.
__global__ __launch_bounds__(256) void colsum_kernel(const ImgDev* __restrict__ imgs,
                                                     const RowChunk* __restrict__ chunks,
                                                     unsigned long long* __restrict__ S) {
    __shared__ uint32_t part[32][kDim + 1];
    const RowChunk ch = chunks[blockIdx.x];
    const uint8_t* base = imgs[ch.img].desc + (int64_t)ch.r0 * kDim;
    const int g = threadIdx.x & 7, rl = threadIdx.x >> 3;
    uint32_t s[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) s[c] = 0;
    for (int r = rl; r < ch.nr; r += 32) {
        const uint4 w = *reinterpret_cast<const uint4*>(base + (int64_t)r * kDim + g * 16);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) s[a * 4 + b] += (ws[a] >> (8 * b)) & 0xFFu;
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) part[rl][g * 16 + c] = s[c];
    __syncthreads();
    if (threadIdx.x < kDim) {
        uint32_t tot = 0;
        for (int r = 0; r < 32; ++r) tot += part[r][threadIdx.x];
        atomicAdd(&S[threadIdx.x], (unsigned long long)tot);
    }
}

// bias_j = (r_j . S) / N in binary64, rounded once to fp32 for the fast path.
__global__ void bias_kernel(const double* __restrict__ R, const unsigned long long* __restrict__ S,
                            double n_tot, float* __restrict__ bias) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kRows) return;
    double acc = 0.0;
    for (int i = 0; i < kDim; ++i) acc = fma(R[j * kDim + i], (double)S[i], acc);
    bias[j] = (float)(acc / n_tot);
}

// ------------------------------------------------------------------ projection
__device__ __forceinline__ uint32_t bf16_pair(uint32_t w, int sh) {
    const float f0 = (float)((w >> sh) & 0xFFu);
    const float f1 = (float)((w >> (sh + 8)) & 0xFFu);
    return (__float_as_uint(f0) >> 16) | (__float_as_uint(f1) & 0xFFFF0000u);
}

__device__ __forceinline__ bf16x8 bytes_to_bf16x8(uint2 w) {
    union {
        uint4 u;
        bf16x8 v;
    } cv;
    cv.u = make_uint4(bf16_pair(w.x, 0), bf16_pair(w.x, 16), bf16_pair(w.y, 0), bf16_pair(w.y, 16));
    return cv.v;
}

__device__ __forceinline__ bf16x8 load_frag(const uint4* __restrict__ frag, int idx) {
    union {
        uint4 u;
        bf16x8 v;
    } cv;
    cv.u = frag[idx];
    return cv.v;
}

// Writes the fast bits and the near-margin mask of one descriptor.
__device__ __forceinline__ void store_code(const CodeOut& o, int row, uint64_t w0, uint64_t w1, uint64_t w2,
                                           uint64_t m0, uint64_t m1, uint64_t m2, uint64_t* __restrict__ near) {
    o.codes[2 * (int64_t)row] = w0;
    o.codes[2 * (int64_t)row + 1] = w1;
    uint16_t* kp = reinterpret_cast<uint16_t*>(o.keys + 6 * (int64_t)row);
    kp[0] = (uint16_t)(w2 & 0xFFFFu);
    kp[1] = (uint16_t)((w2 >> 16) & 0xFFFFu);
    kp[2] = (uint16_t)((w2 >> 32) & 0xFFFFu);
    uint64_t* nm = near + 3 * (o.flat + row);
    nm[0] = m0;
    nm[1] = m1;
    nm[2] = m2;
}

// BF16 hi+lo split on MFMA.  One wave per tile of 16 descriptors: for each of
// the 11 row tiles, D[16 rows][16 desc] = sum over 4 k-steps of
// (R_hi + R_lo)[rows][32 k] x X^T[32 k][desc] with v_mfma_f32_16x16x32_bf16.
// Lane l holds descriptor l % 16 and rows 4 (l / 16) .. +3 of each row tile.
__global__ __launch_bounds__(256) void proj_mfma_kernel(const ImgDev* __restrict__ imgs,
                                                        const CodeOut* __restrict__ outs,
                                                        const RowChunk* __restrict__ tiles, int n_tiles,
                                                        const uint4* __restrict__ frag,
                                                        const float* __restrict__ bias, float margin_coef,
                                                        uint64_t* __restrict__ near) {
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int n_waves = (gridDim.x * blockDim.x) >> 6;
    for (int tile = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; tile < n_tiles; tile += n_waves) {
        const RowChunk tc = tiles[tile];
        const bool live = n < tc.nr;
        const uint8_t* x = imgs[tc.img].desc + (int64_t)(tc.r0 + (live ? n : 0)) * kDim;
        bf16x8 xb[4];
        uint32_t sq = 0;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const uint2 w = live ? *reinterpret_cast<const uint2*>(x + 32 * ks + 8 * g) : make_uint2(0u, 0u);
            sq = __builtin_amdgcn_udot4(w.x, w.x, sq, false);
            sq = __builtin_amdgcn_udot4(w.y, w.y, sq, false);
            xb[ks] = bytes_to_bf16x8(w);
        }
        sq += __shfl_xor(sq, 16);
        sq += __shfl_xor(sq, 32);
        const float base_margin = margin_coef * sqrtf((float)sq) + 0x1p-26f;
        uint64_t w[3] = {0, 0, 0}, m[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int n_rt = k < 2 ? 4 : kRowTiles - 8;
#pragma unroll 1
            for (int rw = 0; rw < n_rt; ++rw) {
                const int rt = 4 * k + rw;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        load_frag(frag, ((0 * kRowTiles + rt) * 4 + ks) * 64 + lane), xb[ks], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        load_frag(frag, ((1 * kRowTiles + rt) * 4 + ks) * 64 + lane), xb[ks], acc, 0, 0, 0);
                }
                const float4 b = reinterpret_cast<const float4*>(bias)[rt * 4 + g];
                const float bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float v = acc[i] - bv[i];
                    const float M = base_margin + 0x1p-20f * fabsf(bv[i]);
                    const bool nr = !(fabsf(v) > M);
                    const bool bit = !nr && v > 0.f;
                    const int pos = 16 * rw + 4 * g + i;
                    w[k] |= (uint64_t)bit << pos;
                    m[k] |= (uint64_t)nr << pos;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            w[k] |= __shfl_xor(w[k], 16);
            w[k] |= __shfl_xor(w[k], 32);
            m[k] |= __shfl_xor(m[k], 16);
            m[k] |= __shfl_xor(m[k], 32);
        }
        if (g == 0 && live) store_code(outs[tc.img], tc.r0 + n, w[0], w[1], w[2], m[0], m[1], m[2], near);
    }
}

// Plain FP32 form: one thread per descriptor, 176 fp32 FMA chains over the
// descriptor held in registers; the rows are wave-uniform scalar loads.
__global__ __launch_bounds__(256) void proj_fp32_kernel(const ImgDev* __restrict__ imgs,
                                                        const CodeOut* __restrict__ outs,
                                                        const RowChunk* __restrict__ tiles, int n_tiles,
                                                        const float* __restrict__ R32,
                                                        const float* __restrict__ bias, float margin_coef,
                                                        uint64_t* __restrict__ near) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int tile = t >> 4, n = t & 15;
    if (tile >= n_tiles) return;
    const RowChunk tc = tiles[tile];
    if (n >= tc.nr) return;
    const uint4* xp = reinterpret_cast<const uint4*>(imgs[tc.img].desc + (int64_t)(tc.r0 + n) * kDim);
    float xf[kDim];
    uint32_t sq = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint4 w = xp[c];
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            sq = __builtin_amdgcn_udot4(ws[a], ws[a], sq, false);
#pragma unroll
            for (int b = 0; b < 4; ++b) xf[c * 16 + a * 4 + b] = (float)((ws[a] >> (8 * b)) & 0xFFu);
        }
    }
    const float base_margin = margin_coef * sqrtf((float)sq) + 0x1p-26f;
    uint64_t w[3] = {0, 0, 0}, m[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int rows = k < 2 ? 64 : kRows - 128;
        for (int rr = 0; rr < rows; ++rr) {
            const int r = 64 * k + rr;
            const float* rp = R32 + r * kDim;
            float acc = 0.f;
#pragma unroll
            for (int i = 0; i < kDim; ++i) acc = fmaf(rp[i], xf[i], acc);
            const float bv = bias[r];
            const float v = acc - bv;
            const float M = base_margin + 0x1p-20f * fabsf(bv);
            const bool nr = !(fabsf(v) > M);
            const bool bit = !nr && v > 0.f;
            w[k] |= (uint64_t)bit << rr;
            m[k] |= (uint64_t)nr << rr;
        }
    }
    store_code(outs[tc.img], tc.r0 + n, w[0], w[1], w[2], m[0], m[1], m[2], near);
}

// Binary64 recompute of near-margin projections: the same fused
// multiply-add chain over components 0..127 of r_j . (N x - S) that defines
// the codes; N x_i - S_i is an exact integer in binary64.  One thread per
// descriptor; every thread that recomputes is the only writer of its code.
__global__ __launch_bounds__(256) void fixup_kernel(const ImgDev* __restrict__ imgs,
                                                    const CodeOut* __restrict__ outs,
                                                    const RowChunk* __restrict__ tiles, int n_tiles,
                                                    const uint64_t* __restrict__ near,
                                                    const double* __restrict__ R,
                                                    const unsigned long long* __restrict__ S, double n_tot,
                                                    unsigned long long* __restrict__ counter) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int tile = t >> 4, n = t & 15;
    uint32_t cnt = 0;
    if (tile < n_tiles) {
        const RowChunk tc = tiles[tile];
        if (n < tc.nr) {
            const CodeOut o = outs[tc.img];
            const int row = tc.r0 + n;
            const uint64_t* nm = near + 3 * (o.flat + row);
            uint64_t mk[3] = {nm[0], nm[1], nm[2]};
            cnt = __popcll(mk[0]) + __popcll(mk[1]) + __popcll(mk[2]);
            if (cnt) {
                const uint8_t* x = imgs[tc.img].desc + (int64_t)row * kDim;
                uint64_t wd[3] = {o.codes[2 * (int64_t)row], o.codes[2 * (int64_t)row + 1], 0};
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    while (mk[k]) {
                        const int bitpos = __ffsll((unsigned long long)mk[k]) - 1;
                        mk[k] &= mk[k] - 1;
                        const int r = 64 * k + bitpos;
                        const double* rr = R + r * kDim;
                        double p = 0.0;
                        for (int i = 0; i < kDim; ++i) {
                            const double c = n_tot * (double)x[i] - (double)S[i];
                            p = fma(rr[i], c, p);
                        }
                        if (p > 0.0) wd[k] |= (uint64_t)1 << bitpos;
                    }
                }
                o.codes[2 * (int64_t)row] = wd[0];
                o.codes[2 * (int64_t)row + 1] = wd[1];
                if (wd[2]) {
                    uint8_t* kb = o.keys + 6 * (int64_t)row;
                    for (int tb = 0; tb < kTables; ++tb) kb[tb] = (uint8_t)(kb[tb] | ((wd[2] >> (8 * tb)) & 0xFFu));
                }
            }
        }
    }
    // wave total -> one atomic per wave
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(counter, (unsigned long long)cnt);
}

// ------------------------------------------------------------------ bucket tables
// One wave per (train image, table): counting sort of the 8-bit keys into 256
// buckets, stable (ascending index inside a bucket).  Ranks inside a 64-wide
// chunk come from eight key-bit ballots.
template <bool EPI>
__global__ __launch_bounds__(64) void bucket_kernel(const ImgDev* __restrict__ imgs,
                                                    const TableOut* __restrict__ touts,
                                                    const int32_t* __restrict__ train_list) {
    using Ent = typename EntOf<EPI>::T;
    __shared__ uint32_t cnt[256];
    const int lane = threadIdx.x;
    const int m = train_list[blockIdx.x / kTables];
    const int t = blockIdx.x % kTables;
    const ImgDev im = imgs[m];
    const TableOut to = touts[m];
    const int n = im.n;
#pragma unroll
    for (int i = 0; i < 4; ++i) cnt[4 * lane + i] = 0;
    __syncthreads();
    for (int c = 0; c < n; c += 64) {
        const int j = c + lane;
        if (j < n) atomicAdd(&cnt[im.keys[6 * (int64_t)j + t]], 1u);
    }
    __syncthreads();
    uint32_t a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = cnt[4 * lane + i];
    const uint32_t tot = a[0] + a[1] + a[2] + a[3];
    const uint32_t incl = wave_incl_scan(tot, lane);
    uint32_t run = incl - tot;
    uint32_t* off = to.off + t * kOffStride;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        off[4 * lane + i] = run;
        cnt[4 * lane + i] = run;
        run += a[i];
    }
    if (lane == 63) off[256] = incl;
    __syncthreads();
    Ent* out = reinterpret_cast<Ent*>(to.ent) + (int64_t)t * n;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int c = 0; c < n; c += 64) {
        const int j = c + lane;
        const bool valid = j < n;
        const uint32_t key = valid ? im.keys[6 * (int64_t)j + t] : 0u;
        uint64_t eq = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool kb = (key >> b) & 1u;
            const uint64_t bm = __ballot(kb);
            eq &= kb ? bm : ~bm;
        }
        const uint32_t rank = __popcll(eq & lt_mask);
        uint32_t pos = 0;
        if (valid) pos = cnt[key] + rank;
        __syncthreads();
        if (valid) {
            const uint16_t* kp = reinterpret_cast<const uint16_t*>(im.keys + 6 * (int64_t)j);
            Ent e;
            e.c0 = im.codes[2 * (int64_t)j];
            e.c1 = im.codes[2 * (int64_t)j + 1];
            e.kid = (uint64_t)kp[0] | ((uint64_t)kp[1] << 16) | ((uint64_t)kp[2] << 32) | ((uint64_t)j << 48);
            if constexpr (EPI) {
                e.x = im.kp[2 * (int64_t)j];
                e.y = im.kp[2 * (int64_t)j + 1];
            }
            out[pos] = e;
            if (rank == 0) cnt[key] = pos + (uint32_t)__popcll(eq);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ matching

// Smallest bin d of a 256-bin LDS histogram whose cumulative count reaches
// `need` (need >= 1 and <= total); *below = count of bins < d.
__device__ __forceinline__ uint32_t hist_select(const uint32_t* hist, uint32_t need, int lane, uint32_t* below) {
    const uint4 h = reinterpret_cast<const uint4*>(hist)[lane];
    const uint32_t s0 = h.x, s1 = s0 + h.y, s2 = s1 + h.z, s3 = s2 + h.w;
    const uint32_t incl = wave_incl_scan(s3, lane);
    const uint32_t ex = incl - s3;
    const bool has = incl >= need;
    const uint32_t i = (ex + s0 >= need) ? 0u : (ex + s1 >= need) ? 1u : (ex + s2 >= need) ? 2u : 3u;
    const uint32_t bl = ex + (i == 0 ? 0u : i == 1 ? s0 : i == 2 ? s1 : s2);
    const uint64_t m = __ballot(has);
    const int L = __ffsll((unsigned long long)m) - 1;
    *below = uniform(__shfl(bl, L));
    return uniform(__shfl(4u * (uint32_t)lane + i, L));
}

__device__ __forceinline__ void clear_hist(uint32_t* hist, int lane) {
    reinterpret_cast<uint4*>(hist)[lane] = make_uint4(0u, 0u, 0u, 0u);
    wave_sync();
}

// Per-query view of the six bucket runs: bucket start of table t (b0..b5) and
// prefix sums of the bucket sizes (P1..P6), plus the query's code and keys and
// its epipolar line.  Passed by value so every field stays in registers.
struct QueryRuns {
    uint64_t qc0, qc1, qk;
    uint32_t b0, b1, b2, b3, b4, b5;
    uint32_t P1, P2, P3, P4, P5, P6;
    double la, lb, lc;
};

// Candidate e of the concatenated six bucket runs -> packed key
// (Hamming << 16 | index), or ~0u if it repeats an earlier table's candidate,
// falls outside the epipolar band or exceeds tau.  n_union counts the
// candidates that survive the union and the band.
template <bool EPI>
__device__ __forceinline__ uint32_t key_at(uint32_t e, const typename EntOf<EPI>::T* __restrict__ ent, int32_t n_t,
                                           const QueryRuns r, int32_t tau, double dd, uint32_t& n_union) {
    using Ent = typename EntOf<EPI>::T;
    if (e >= r.P6) return ~0u;
    const uint32_t t = (uint32_t)(e >= r.P1) + (e >= r.P2) + (e >= r.P3) + (e >= r.P4) + (e >= r.P5);
    const uint32_t Pt = t == 0 ? 0u : t == 1 ? r.P1 : t == 2 ? r.P2 : t == 3 ? r.P3 : t == 4 ? r.P4 : r.P5;
    const uint32_t bt = t == 0 ? r.b0 : t == 1 ? r.b1 : t == 2 ? r.b2 : t == 3 ? r.b3 : t == 4 ? r.b4 : r.b5;
    const Ent* ep = ent + (int64_t)t * n_t + (bt + (e - Pt));
    const uint64_t kid = ep->kid;
    bool dup = false;
#pragma unroll
    for (int u = 0; u < kTables - 1; ++u) dup |= (u < (int)t) && (((kid ^ r.qk) >> (8 * u)) & 0xFFu) == 0;
    if (dup) return ~0u;
    if constexpr (EPI) {
        const double xp = (double)ep->x, yp = (double)ep->y;
        const double ev = (r.la * xp + r.lb * yp) + r.lc;
        if (!(ev * ev <= dd * (r.la * r.la + r.lb * r.lb))) return ~0u;
    }
    ++n_union;
    const uint32_t h = (uint32_t)(__popcll(ep->c0 ^ r.qc0) + __popcll(ep->c1 ^ r.qc1));
    if ((int32_t)h > tau) return ~0u;
    return (h << 16) | (uint32_t)(kid >> 48);
}

template <bool EPI>
__global__ __launch_bounds__(256) void match_kernel(const ImgDev* __restrict__ imgs,
                                                    const PairDev* __restrict__ pairs,
                                                    const Item* __restrict__ items, int32_t n_items,
                                                    uint32_t* __restrict__ counter, MatchParams prm,
                                                    int32_t* __restrict__ o_idx, int32_t* __restrict__ o_d1,
                                                    int32_t* __restrict__ o_d2,
                                                    unsigned long long* __restrict__ stats) {
    using Ent = typename EntOf<EPI>::T;
    __shared__ __attribute__((aligned(16))) uint32_t s_hist[kWavesPerBlock][256];
    __shared__ uint32_t s_list[kWavesPerBlock][kListCap];
    __shared__ uint32_t s_sel[kWavesPerBlock][kMaxK];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t* hist = s_hist[wv];
    uint32_t* list = s_list[wv];
    uint32_t* sel = s_sel[wv];
    const int part = lane & 3;
    uint64_t st_bucket = 0, st_ranked = 0;
    uint32_t st_union = 0;
    uint64_t st_union64 = 0;

    int32_t it = (int32_t)(blockIdx.x * kWavesPerBlock + wv);
    for (;;) {
        if (counter) {
            uint32_t v = 0;
            if (lane == 0) v = atomicAdd(counter, 1u);
            it = (int32_t)uniform(__shfl(v, 0));
        }
        if (it >= n_items) break;
        const Item item = items[it];
        const PairDev& pr = pairs[item.pair];
        const ImgDev Q = imgs[pr.qi];
        const ImgDev T = imgs[pr.ti];
        const Ent* ent = reinterpret_cast<const Ent*>(T.ent);
        const int32_t n_t = T.n;
        const double dd = prm.max_px * prm.max_px;
        double F[9];
        if constexpr (EPI) {
#pragma unroll
            for (int i = 0; i < 9; ++i) F[i] = pr.F[i];
        }
        for (int32_t q = item.q0; q < item.q0 + item.nq; ++q) {
            // ---- Step 1: the query's bucket in each table
            QueryRuns qr;
            qr.qc0 = Q.codes[2 * (int64_t)q];
            qr.qc1 = Q.codes[2 * (int64_t)q + 1];
            const uint16_t* kq = reinterpret_cast<const uint16_t*>(Q.keys + 6 * (int64_t)q);
            qr.qk = (uint64_t)kq[0] | ((uint64_t)kq[1] << 16) | ((uint64_t)kq[2] << 32);
            uint32_t bs[kTables], ln[kTables];
#pragma unroll
            for (int t = 0; t < kTables; ++t) {
                const uint32_t v = (uint32_t)((qr.qk >> (8 * t)) & 0xFFu);
                bs[t] = T.off[t * kOffStride + v];
                ln[t] = T.off[t * kOffStride + v + 1] - bs[t];
            }
            qr.b0 = bs[0]; qr.b1 = bs[1]; qr.b2 = bs[2]; qr.b3 = bs[3]; qr.b4 = bs[4]; qr.b5 = bs[5];
            qr.P1 = ln[0];
            qr.P2 = qr.P1 + ln[1];
            qr.P3 = qr.P2 + ln[2];
            qr.P4 = qr.P3 + ln[3];
            qr.P5 = qr.P4 + ln[4];
            qr.P6 = qr.P5 + ln[5];
            const uint32_t total = qr.P6;
            qr.la = qr.lb = qr.lc = 0.0;
            if constexpr (EPI) {
                const double x = (double)Q.kp[2 * (int64_t)q], y = (double)Q.kp[2 * (int64_t)q + 1];
                qr.la = (F[0] * x + F[1] * y) + F[2];
                qr.lb = (F[3] * x + F[4] * y) + F[5];
                qr.lc = (F[6] * x + F[7] * y) + F[8];
            }
            st_bucket += total;

            // ---- Steps 1-3 pass 1: union, Hamming, tau; index table over H
            clear_hist(hist, lane);
            uint32_t n_valid = 0;
            for (uint32_t base = 0; base < total; base += 64) {
                const uint32_t key = key_at<EPI>(base + lane, ent, n_t, qr, prm.tau, dd, st_union);
                const bool keep = key != ~0u;
                const uint64_t mk = __ballot(keep);
                if (keep) {
                    atomicAdd(&hist[key >> 16], 1u);
                    const uint32_t slot = n_valid + mbcnt64(mk);
                    if (slot < (uint32_t)kListCap) list[slot] = key;
                }
                n_valid += (uint32_t)__popcll(mk);
            }
            wave_sync();
            const bool in_list = n_valid <= (uint32_t)kListCap;
            const uint32_t span = in_list ? n_valid : total;
            uint32_t dummy = 0;
#define CAND(e) (in_list ? ((e) < n_valid ? list[(e)] : ~0u) : key_at<EPI>((e), ent, n_t, qr, prm.tau, dd, dummy))

            const uint32_t kk = n_valid < (uint32_t)prm.k ? n_valid : (uint32_t)prm.k;
            st_ranked += kk;
            int32_t r_idx = -1, r_d1 = -1, r_d2 = -1;
            if (kk > 0) {
                // ---- Step 3: threshold of the kk-th key by counting passes
                uint32_t below;
                const uint32_t hs = hist_select(hist, kk, lane, &below);
                uint32_t need = kk - below;
                uint32_t ties = uniform(hist[hs]);
                uint32_t bound;
                if (ties == need) {
                    bound = (hs + 1) << 16;
                } else {
                    clear_hist(hist, lane);
                    for (uint32_t base = 0; base < span; base += 64) {
                        const uint32_t key = CAND(base + lane);
                        if ((key >> 16) == hs) atomicAdd(&hist[(key >> 8) & 0xFFu], 1u);
                    }
                    wave_sync();
                    const uint32_t d1 = hist_select(hist, need, lane, &below);
                    need -= below;
                    ties = uniform(hist[d1]);
                    const uint32_t prefix = (hs << 16) | (d1 << 8);
                    if (ties == need) {
                        bound = prefix + 256u;
                    } else {
                        clear_hist(hist, lane);
                        for (uint32_t base = 0; base < span; base += 64) {
                            const uint32_t key = CAND(base + lane);
                            if ((key >> 8) == (prefix >> 8)) atomicAdd(&hist[key & 0xFFu], 1u);
                        }
                        wave_sync();
                        const uint32_t d2 = hist_select(hist, need, lane, &below);
                        bound = (prefix | d2) + 1u;
                    }
                }
                // compaction: the kk keys below the bound
                uint32_t nsel = 0;
                for (uint32_t base = 0; base < span; base += 64) {
                    const uint32_t key = CAND(base + lane);
                    const bool keep = key < bound;
                    const uint64_t mk = __ballot(keep);
                    const uint32_t slot = nsel + mbcnt64(mk);
                    if (keep && slot < (uint32_t)kMaxK) sel[slot] = key & 0xFFFFu;
                    nsel += (uint32_t)__popcll(mk);
                }
                wave_sync();

                // ---- Step 4: exact squared distances, 4 lanes per candidate
                const uint8_t* qa = Q.desc + (int64_t)q * kDim + part * 32;
                const uint4 a0 = reinterpret_cast<const uint4*>(qa)[0];
                const uint4 a1 = reinterpret_cast<const uint4*>(qa)[1];
                const uint32_t av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
                uint32_t aa = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) aa = __builtin_amdgcn_udot4(av[i], av[i], aa, false);
                uint64_t best = ~0ull;
                uint32_t sec = ~0u;
                for (uint32_t r0 = 0; r0 < kk; r0 += 16) {
                    const uint32_t s = r0 + (uint32_t)(lane >> 2);
                    const bool act = s < kk;
                    uint32_t j = 0, dp = 0;
                    if (act) {
                        j = min(sel[s], (uint32_t)(n_t - 1));  // ids come from the train image's tables
                        const uint4* bp = reinterpret_cast<const uint4*>(T.desc + (int64_t)j * kDim + part * 32);
                        const uint4 b0 = bp[0], b1 = bp[1];
                        const uint32_t bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
                        uint32_t ab = 0, bb = 0;
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            ab = __builtin_amdgcn_udot4(av[i], bv[i], ab, false);
                            bb = __builtin_amdgcn_udot4(bv[i], bv[i], bb, false);
                        }
                        dp = aa + bb - 2u * ab;
                    }
                    uint32_t d = dp + __shfl_xor(dp, 1);
                    d += __shfl_xor(d, 2);
                    if (act && part == 0) {
                        const uint64_t c = ((uint64_t)d << 32) | j;
                        if (c < best) {
                            sec = min(sec, (uint32_t)(best >> 32));
                            best = c;
                        } else {
                            sec = min(sec, d);
                        }
                    }
                }
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const uint64_t ob = __shfl_xor(best, off);
                    const uint32_t os = __shfl_xor(sec, off);
                    const uint32_t hi = max((uint32_t)(best >> 32), (uint32_t)(ob >> 32));
                    sec = min(min(sec, os), hi);
                    best = min(best, ob);
                }
                const int64_t D1 = (int64_t)(best >> 32);
                r_d1 = (int32_t)D1;
                if (kk >= 2) {
                    const int64_t D2 = (int64_t)sec;
                    r_d2 = (int32_t)D2;
                    if (prm.den2 * D1 < prm.num2 * D2) r_idx = (int32_t)(uint32_t)best;
                }
            }
#undef CAND
            if (lane == 0) {
                const int64_t o = pr.out + q;
                o_idx[o] = r_idx;
                o_d1[o] = r_d1;
                o_d2[o] = r_d2;
            }
        }
        if (!counter) break;
    }
    // statistics: bucket entries (uniform per wave) and union sizes (per lane)
    st_union64 = st_union;
    for (int d = 32; d >= 1; d >>= 1) st_union64 += __shfl_xor(st_union64, d);
    if (lane == 0 && stats) {
        atomicAdd(&stats[0], (unsigned long long)st_bucket);
        atomicAdd(&stats[1], (unsigned long long)st_union64);
        atomicAdd(&stats[2], (unsigned long long)st_ranked);
    }
}

// ------------------------------------------------------------------ launchers
#define CH_LAUNCH(...)                                  \
    do {                                                \
        hipLaunchKernelGGL(__VA_ARGS__);                \
        hipError_t e_ = hipGetLastError();              \
        if (e_ != hipSuccess) return e_;                \
    } while (0)

hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, int64_t n, unsigned long long v) {
    if (n <= 0) return hipSuccess;
    CH_LAUNCH(fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipSuccess;
}

hipError_t launch_fill_u32(hipStream_t s, uint32_t* p, int64_t n, uint32_t v) {
    if (n <= 0) return hipSuccess;
    CH_LAUNCH(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipSuccess;
}

hipError_t launch_colsum(hipStream_t s, const ImgDev* imgs, const RowChunk* chunks, int n_chunks,
                         unsigned long long* S) {
    if (n_chunks <= 0) return hipSuccess;
    CH_LAUNCH(colsum_kernel, dim3(n_chunks), dim3(256), 0, s, imgs, chunks, S);
    return hipSuccess;
}

hipError_t launch_bias(hipStream_t s, const double* R, const unsigned long long* S, double n_tot, float* bias) {
    CH_LAUNCH(bias_kernel, dim3(1), dim3(192), 0, s, R, S, n_tot, bias);
    return hipSuccess;
}

hipError_t launch_proj_mfma(hipStream_t s, int grid, const ImgDev* imgs, const CodeOut* outs, const RowChunk* tiles,
                            int n_tiles, const uint4* frag, const float* bias, float margin, uint64_t* near) {
    if (n_tiles <= 0) return hipSuccess;
    CH_LAUNCH(proj_mfma_kernel, dim3(grid), dim3(256), 0, s, imgs, outs, tiles, n_tiles, frag, bias, margin, near);
    return hipSuccess;
}

hipError_t launch_proj_fp32(hipStream_t s, const ImgDev* imgs, const CodeOut* outs, const RowChunk* tiles,
                            int n_tiles, const float* R32, const float* bias, float margin, uint64_t* near) {
    if (n_tiles <= 0) return hipSuccess;
    const int64_t threads = (int64_t)n_tiles * 16;
    CH_LAUNCH(proj_fp32_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, imgs, outs, tiles, n_tiles,
              R32, bias, margin, near);
    return hipSuccess;
}

hipError_t launch_fixup(hipStream_t s, const ImgDev* imgs, const CodeOut* outs, const RowChunk* tiles, int n_tiles,
                        const uint64_t* near, const double* R, const unsigned long long* S, double n_tot,
                        unsigned long long* counter) {
    if (n_tiles <= 0) return hipSuccess;
    const int64_t threads = (int64_t)n_tiles * 16;
    CH_LAUNCH(fixup_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, imgs, outs, tiles, n_tiles, near,
              R, S, n_tot, counter);
    return hipSuccess;
}

hipError_t launch_bucket(hipStream_t s, bool epi, const ImgDev* imgs, const TableOut* touts, const int32_t* train_list,
                         int n_train) {
    if (n_train <= 0) return hipSuccess;
    if (epi)
        CH_LAUNCH(bucket_kernel<true>, dim3(n_train * kTables), dim3(64), 0, s, imgs, touts, train_list);
    else
        CH_LAUNCH(bucket_kernel<false>, dim3(n_train * kTables), dim3(64), 0, s, imgs, touts, train_list);
    return hipSuccess;
}

hipError_t launch_match(hipStream_t s, bool epi, int grid, const ImgDev* imgs, const PairDev* pairs, const Item* items,
                        int32_t n_items, uint32_t* counter, const MatchParams& prm, int32_t* o_idx, int32_t* o_d1,
                        int32_t* o_d2, unsigned long long* stats) {
    if (n_items <= 0 || grid <= 0) return hipSuccess;
    if (epi)
        CH_LAUNCH(match_kernel<true>, dim3(grid), dim3(64 * kWavesPerBlock), 0, s, imgs, pairs, items, n_items,
                  counter, prm, o_idx, o_d1, o_d2, stats);
    else
        CH_LAUNCH(match_kernel<false>, dim3(grid), dim3(64 * kWavesPerBlock), 0, s, imgs, pairs, items, n_items,
                  counter, prm, o_idx, o_d1, o_d2, stats);
    return hipSuccess;
}

}  // namespace cashash
