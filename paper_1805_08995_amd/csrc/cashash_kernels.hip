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

// Loads through pointers known to address global memory (pointers read from
// device tables would otherwise be treated as generic and use flat loads).
template <class T>
__device__ __forceinline__ T gload(const T* p) {
#if __HIP_DEVICE_COMPILE__
    return *(const __attribute__((address_space(1))) T*)(p);
#else
    return *p;  // host pass: parsed only, never run
#endif
}
typedef unsigned long long u64x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ ulonglong2 gload(const ulonglong2* p) {
    const u64x2_t v = gload(reinterpret_cast<const u64x2_t*>(p));
    return make_ulonglong2(v.x, v.y);
}
__device__ __forceinline__ uint4 gload(const uint4* p) {
    const u32x4_t v = gload(reinterpret_cast<const u32x4_t*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 gload(const float2* p) {
    const f32x2_t v = gload(reinterpret_cast<const f32x2_t*>(p));
    return make_float2(v.x, v.y);
}
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

// Work items from the per-pair tile table: item i belongs to the last entry
// whose first tile is <= i (binary search); its queries are tile (i - first)
// of that pair's query image, qt per tile.
__global__ void make_items_kernel(const PairTiles* __restrict__ pt, int32_t n_pt, const PairDev* __restrict__ pairs,
                                  const ImgDev* __restrict__ imgs, int32_t qt, Item* __restrict__ items,
                                  int32_t n_items) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    int32_t lo = 0, hi = n_pt - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (pt[mid].first <= i) lo = mid; else hi = mid - 1;
    }
    const int32_t p = pt[lo].pair;
    const int32_t q0 = (i - pt[lo].first) * qt;
    const int32_t nq = imgs[pairs[p].qi].n;
    items[i] = Item{p, q0, min(qt, nq - q0), 0};
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

// Writes the fast bits of one descriptor (near-margin bits are 0 until the
// binary64 recompute) and appends it to the near list if any row is flagged:
// one atomic per wavefront reserves the wave's slots.
__device__ __forceinline__ void store_code(const CodeOut& o, int img, int row, bool live, uint64_t w0, uint64_t w1,
                                           uint64_t w2, uint64_t m0, uint64_t m1, uint64_t m2,
                                           NearEntry* __restrict__ near, unsigned int* __restrict__ near_count) {
    if (live) {
        o.codes[2 * (int64_t)row] = w0;
        o.codes[2 * (int64_t)row + 1] = w1;
        uint16_t* kp = reinterpret_cast<uint16_t*>(o.keys + 6 * (int64_t)row);
        kp[0] = (uint16_t)(w2 & 0xFFFFu);
        kp[1] = (uint16_t)((w2 >> 16) & 0xFFFFu);
        kp[2] = (uint16_t)((w2 >> 32) & 0xFFFFu);
    }
    const bool flagged = live && (m0 | m1 | m2) != 0;
    const uint64_t fm = __ballot(flagged);
    if (fm == 0) return;
    uint32_t base = 0;
    if ((threadIdx.x & 63) == (uint32_t)(__ffsll((unsigned long long)fm) - 1))
        base = atomicAdd(near_count, (unsigned int)__popcll(fm));
    base = __builtin_amdgcn_readlane(base, __ffsll((unsigned long long)fm) - 1);
    if (flagged) {
        NearEntry& e = near[base + mbcnt64(fm)];
        e.img = img;
        e.row = row;
        e.mask[0] = m0;
        e.mask[1] = m1;
        e.mask[2] = m2;
    }
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
                                                        NearEntry* __restrict__ near,
                                                        unsigned int* __restrict__ near_count) {
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
        store_code(outs[tc.img], tc.img, tc.r0 + n, g == 0 && live, w[0], w[1], w[2], m[0], m[1], m[2], near,
                   near_count);
    }
}

// Plain FP32 form: one thread per descriptor, 176 fp32 FMA chains over the
// descriptor held in registers; the rows are wave-uniform scalar loads.
__global__ __launch_bounds__(256) void proj_fp32_kernel(const ImgDev* __restrict__ imgs,
                                                        const CodeOut* __restrict__ outs,
                                                        const RowChunk* __restrict__ tiles, int n_tiles,
                                                        const float* __restrict__ R32,
                                                        const float* __restrict__ bias, float margin_coef,
                                                        NearEntry* __restrict__ near,
                                                        unsigned int* __restrict__ near_count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int tile = min(t >> 4, n_tiles - 1), n = t & 15;
    const RowChunk tc = tiles[tile];
    const bool live = (t >> 4) < n_tiles && n < tc.nr;
    const uint4* xp = reinterpret_cast<const uint4*>(imgs[tc.img].desc + (int64_t)(tc.r0 + (live ? n : 0)) * kDim);
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
    store_code(outs[tc.img], tc.img, tc.r0 + n, live, w[0], w[1], w[2], m[0], m[1], m[2], near, near_count);
}

// Binary64 recompute of near-margin projections: the same fused
// multiply-add chain over components 0..127 of r_j . (N x - S) that defines
// the codes; N x_i - S_i is an exact integer in binary64.  One thread per
// listed descriptor (grid-stride); it is the only writer of that code.
__global__ __launch_bounds__(256) void fixup_kernel(const ImgDev* __restrict__ imgs,
                                                    const CodeOut* __restrict__ outs,
                                                    const NearEntry* __restrict__ near,
                                                    const unsigned int* __restrict__ near_count,
                                                    const double* __restrict__ R,
                                                    const unsigned long long* __restrict__ S, double n_tot,
                                                    unsigned long long* __restrict__ counter) {
    const uint32_t n_near = *near_count;
    uint32_t cnt = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_near; i += gridDim.x * blockDim.x) {
        const NearEntry e = near[i];
        const CodeOut o = outs[e.img];
        const int64_t row = e.row;
        uint64_t mk[3] = {e.mask[0], e.mask[1], e.mask[2]};
        cnt += (uint32_t)(__popcll(mk[0]) + __popcll(mk[1]) + __popcll(mk[2]));
        const uint8_t* x = imgs[e.img].desc + row * kDim;
        uint64_t wd[3] = {o.codes[2 * row], o.codes[2 * row + 1], 0};
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
        o.codes[2 * row] = wd[0];
        o.codes[2 * row + 1] = wd[1];
        if (wd[2]) {
            uint8_t* kb = o.keys + 6 * row;
            for (int tb = 0; tb < kTables; ++tb) kb[tb] = (uint8_t)(kb[tb] | ((wd[2] >> (8 * tb)) & 0xFFu));
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
    ulonglong2* out_code = reinterpret_cast<ulonglong2*>(to.ent) + (int64_t)t * n;
    uint64_t* out_kid = reinterpret_cast<uint64_t*>(to.ent + (size_t)kTables * n * 16) + (int64_t)t * n;
    float2* out_kp = reinterpret_cast<float2*>(to.ent + (size_t)kTables * n * 24) + (int64_t)t * n;
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
            out_code[pos] = make_ulonglong2(im.codes[2 * (int64_t)j], im.codes[2 * (int64_t)j + 1]);
            out_kid[pos] = (uint64_t)kp[0] | ((uint64_t)kp[1] << 16) | ((uint64_t)kp[2] << 32) | ((uint64_t)j << 48);
            if constexpr (EPI) out_kp[pos] = make_float2(im.kp[2 * (int64_t)j], im.kp[2 * (int64_t)j + 1]);
            if (rank == 0) cnt[key] = pos + (uint32_t)__popcll(eq);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ matching

// x as seen through a DPP pattern; lanes whose source is outside their row,
// or whose row is masked off, receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
    return __builtin_amdgcn_update_dpp(0u, x, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive prefix sum over the 64 lanes with DPP row shifts and row
// broadcasts (no LDS round trip).
__device__ __forceinline__ uint32_t wave_scan_dpp(uint32_t x) {
    x += dpp<0x111, 0xf>(x);  // row_shr:1
    x += dpp<0x112, 0xf>(x);  // row_shr:2
    x += dpp<0x114, 0xf>(x);  // row_shr:4
    x += dpp<0x118, 0xf>(x);  // row_shr:8
    x += dpp<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    return (uint64_t)readlane((uint32_t)v, l) | ((uint64_t)readlane((uint32_t)(v >> 32), l) << 32);
}
__device__ __forceinline__ double readlane_f64(double v, int l) { return __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(v), l)); }

// Smallest bin d of the 256-bin LDS index table whose cumulative count
// reaches `need` (1 <= need <= total); *below = count in bins < d.
__device__ __forceinline__ uint32_t hist_select(const uint32_t* hist, uint32_t need, int lane, uint32_t* below) {
    const uint4 h = reinterpret_cast<const uint4*>(hist)[lane];
    const uint32_t s0 = h.x, s1 = s0 + h.y, s2 = s1 + h.z, s3 = s2 + h.w;
    const uint32_t incl = wave_scan_dpp(s3);
    const uint32_t ex = incl - s3;
    const uint32_t i = (ex + s0 >= need) ? 0u : (ex + s1 >= need) ? 1u : (ex + s2 >= need) ? 2u : 3u;
    const uint32_t bl = ex + (i == 0 ? 0u : i == 1 ? s0 : i == 2 ? s1 : s2);
    const uint64_t m = __ballot(incl >= need);
    const int L = __ffsll((unsigned long long)m) - 1;
    *below = readlane(bl, L);
    return readlane(4u * (uint32_t)lane + i, L);
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
    uint32_t P1, P2, P3, P4, P5, P6;
    const uint32_t* cofs;  // LDS: C_t = t * n_t + b_t - P_t, candidate e of table t sits at entry e + C_t
    double la, lb, lc;
};

// Train image tables, struct of arrays (see ent_bytes).
struct TrainView {
    const ulonglong2* code;
    const uint64_t* kid;
    const float2* kp;
    int32_t n;
};

// Candidate e of the concatenated six bucket runs -> packed key
// (Hamming << 16 | index), or ~0u if e is past the runs, repeats an earlier
// table's candidate, falls outside the epipolar band or exceeds tau.  The
// loads are unconditional (a clamped position) so several calls can have
// their loads in flight together.  n_union counts candidates that survive
// the union and the band.
// Table t and entry position of candidate e of the concatenated runs; lanes
// past the runs get candidate 0's position (a valid address).
__device__ __forceinline__ uint32_t entry_pos(uint32_t e, const QueryRuns& r, uint32_t& t) {
    const uint32_t ec = e < r.P6 ? e : 0u;
    t = (uint32_t)(ec >= r.P1) + (ec >= r.P2) + (ec >= r.P3) + (ec >= r.P4) + (ec >= r.P5);
    return ec + r.cofs[t];
}

// Eq. 1-2: the candidate's keypoint lies within the band around the
// query's epipolar line.
__device__ __forceinline__ bool in_band(const TrainView& tv, uint32_t pos, const QueryRuns& r, double dd) {
    const float2 p = gload(tv.kp + pos);
    const double xp = (double)p.x, yp = (double)p.y;
    const double ev = (r.la * xp + r.lb * yp) + r.lc;
    return ev * ev <= dd * (r.la * r.la + r.lb * r.lb);
}

// Entry (t, pos) -> packed key (Hamming << 16 | index), or ~0u if it repeats
// an earlier table's candidate or exceeds tau.  `live` masks lanes with no
// candidate; n_union counts candidates that survive the union.
__device__ __forceinline__ uint32_t entry_key(const TrainView& tv, uint32_t t, uint32_t pos, bool live,
                                              const QueryRuns& r, int32_t tau, uint32_t& n_union) {
    const ulonglong2 c = gload(tv.code + pos);
    const uint64_t kid = gload(tv.kid + pos);
    // union: drop the candidate if it shares an earlier table's key with the
    // query (it was already collected there).  Zero bytes of x = keys ^ qkeys
    // are found with the carry-free test ((x & 0x7f..) + 0x7f..) | x.
    const uint64_t x = (kid ^ r.qk) & 0xFFFFFFFFFFFFull;
    const uint64_t zb = ~(((x & 0x7F7F7F7F7F7Full) + 0x7F7F7F7F7F7Full) | x) & 0x808080808080ull;
    const bool dup = (zb & ((1ull << (8u * t)) - 1ull)) != 0;
    bool ok = live && !dup;
    n_union += ok ? 1u : 0u;
    const uint32_t h = (uint32_t)(__popcll(c.x ^ r.qc0) + __popcll(c.y ^ r.qc1));
    ok = ok && (int32_t)h <= tau;
    return ok ? ((h << 16) | (uint32_t)(kid >> 48)) : ~0u;
}

// Candidate e of the concatenated six bucket runs -> packed key, or ~0u if e
// is past the runs, outside the epipolar band, a repeat or above tau.
template <bool EPI>
__device__ __forceinline__ uint32_t key_at(uint32_t e, const TrainView& tv, const QueryRuns& r, int32_t tau,
                                           double dd, uint32_t& n_union) {
    uint32_t t;
    const uint32_t pos = entry_pos(e, r, t);
    bool live = e < r.P6;
    if constexpr (EPI) live = live && in_band(tv, pos, r, dd);
    return entry_key(tv, t, pos, live, r, tau, n_union);
}

// The first C chunks of 64 candidates into register slots, all loads issued
// together (slots >= C keep ~0u).
template <bool EPI, int C, int NS>
__device__ __forceinline__ void gather_chunks(uint32_t (&kr)[NS], int lane, const TrainView& tv, const QueryRuns& r,
                                              int32_t tau, double dd, uint32_t& n_union) {
#pragma unroll
    for (int u = 0; u < C; ++u) kr[u] = key_at<EPI>(64u * u + (uint32_t)lane, tv, r, tau, dd, n_union);
}

// One wavefront per tile of <= kMaxTile consecutive queries of one pair.
//  setup    : lane l loads query l's code, keys and six bucket ranges at once;
//             each query's values are then broadcast with readlane.
//  Steps 1-3: per query, the six bucket runs are read four 64-wide chunks at
//             a time (union by first-table dedupe, Hamming, tau, band); the
//             index table (histogram over Hamming distance) is built in LDS
//             and scanned to find the Hamming distance H* of the k-th
//             candidate; ties at H* are broken by index by counting with
//             ballots over a binary search of index bits.
//  Step 4   : the tile's kept (query, candidate) pairs are measured together,
//             4 lanes per pair with v_dot4_u32_u8; lane l then takes query l's
//             distances, picks the nearest and second nearest and applies the
//             ratio test, and the tile's outputs are stored coalesced.
template <bool EPI, int NS>
__global__ __launch_bounds__(256) void match_kernel(const ImgDev* __restrict__ imgs,
                                                    const PairDev* __restrict__ pairs,
                                                    const Item* __restrict__ items, int32_t n_items,
                                                    uint32_t* __restrict__ counter, MatchParams prm,
                                                    int32_t* __restrict__ o_idx, int32_t* __restrict__ o_d1,
                                                    int32_t* __restrict__ o_d2,
                                                    unsigned long long* __restrict__ stats) {
    __shared__ __attribute__((aligned(16))) uint32_t s_hist[kWavesPerBlock][256];
    __shared__ __attribute__((aligned(16))) uint32_t s_list[kWavesPerBlock][kListCap];
    __shared__ __attribute__((aligned(16))) uint32_t s_sel[kWavesPerBlock][kSelCap];
    __shared__ __attribute__((aligned(16))) uint32_t s_cofs[kWavesPerBlock][kMaxTile * 8];  // per query: C_0..C_5
    const int lane = threadIdx.x & 63;
    const int wv = (int)uniform(threadIdx.x >> 6);
    uint32_t* hist = s_hist[wv];
    uint32_t* list = s_list[wv];
    uint32_t* sel = s_sel[wv];
    uint32_t* cofs = s_cofs[wv];
    const int part = lane & 3;
    uint64_t st_bucket = 0, st_ranked = 0;
    uint32_t st_union = 0;
    const double dd = prm.max_px * prm.max_px;

    // XCD of this wavefront: its segment of the work list is the one whose
    // train images stay in this XCD's L2
    const uint32_t home = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kSegments - 1);
    int32_t it = (int32_t)(blockIdx.x * kWavesPerBlock + wv);
    int32_t cur = 0, end = 0;
    for (;;) {
        if (counter) {
            if (cur >= end) {
                for (int sx = 0; sx < kSegments; ++sx) {
                    const uint32_t x = (home + (uint32_t)sx) & (kSegments - 1);
                    const int32_t s0 = prm.seg[x], s1 = prm.seg[x + 1];
                    if (s0 >= s1) continue;
                    uint32_t v = 0;
                    if (lane == 0) v = atomicAdd(counter + x * kCounterStride, (uint32_t)prm.grab);
                    v = readlane(v, 0);
                    if ((int64_t)s0 + v < (int64_t)s1) {
                        cur = s0 + (int32_t)v;
                        end = min(cur + prm.grab, s1);
                        break;
                    }
                }
                if (cur >= end) break;  // every segment is exhausted
            }
            it = cur++;
        }
        if (it >= n_items) break;
        const Item item = items[it];
        const PairDev& pr = pairs[item.pair];
        const ImgDev Q = imgs[pr.qi];
        const ImgDev T = imgs[pr.ti];
        TrainView tv;
        tv.n = T.n;
        tv.code = reinterpret_cast<const ulonglong2*>(T.ent);
        tv.kid = reinterpret_cast<const uint64_t*>(T.ent + (size_t)kTables * T.n * 16);
        tv.kp = reinterpret_cast<const float2*>(T.ent + (size_t)kTables * T.n * 24);
        const int nq = (int)uniform((uint32_t)item.nq);
        const int32_t q0 = (int32_t)uniform((uint32_t)item.q0);

        // ---- setup, one lane per query of the tile
        const int64_t lq = q0 + min(lane, nq - 1);
        const uint64_t v_qc0 = gload(Q.codes + 2 * lq), v_qc1 = gload(Q.codes + 2 * lq + 1);
        const uint16_t* kq = reinterpret_cast<const uint16_t*>(Q.keys + 6 * lq);
        const uint64_t v_qk = (uint64_t)gload(kq) | ((uint64_t)gload(kq + 1) << 16) | ((uint64_t)gload(kq + 2) << 32);
        uint32_t v_P[kTables];
        {
            uint32_t acc = 0, cu[kTables];
#pragma unroll
            for (int t = 0; t < kTables; ++t) {
                const uint32_t v = (uint32_t)((v_qk >> (8 * t)) & 0xFFu);
                const uint32_t b = gload(T.off + t * kOffStride + v);
                cu[t] = (uint32_t)t * (uint32_t)T.n + b - acc;  // entry of candidate e of table t: e + cu[t]
                acc += gload(T.off + t * kOffStride + v + 1) - b;
                v_P[t] = acc;
            }
            // the previous tile's readers are done (the finalize step ended with a wave sync)
            if (lane < kMaxTile) {
                uint4* cw = reinterpret_cast<uint4*>(cofs + 8 * lane);
                cw[0] = make_uint4(cu[0], cu[1], cu[2], cu[3]);
                cw[1] = make_uint4(cu[4], cu[5], 0u, 0u);
            }
            wave_sync();
        }
        double v_la = 0.0, v_lb = 0.0, v_lc = 0.0;
        if constexpr (EPI) {
            const double x = (double)gload(Q.kp + 2 * lq), y = (double)gload(Q.kp + 2 * lq + 1);
            v_la = (pr.F[0] * x + pr.F[1] * y) + pr.F[2];
            v_lb = (pr.F[3] * x + pr.F[4] * y) + pr.F[5];
            v_lc = (pr.F[6] * x + pr.F[7] * y) + pr.F[8];
        }
        uint32_t my_kk = 0, my_off = 0, sel_n = 0;
        const uint32_t jbits = tv.n > 1 ? 32u - (uint32_t)__clz(tv.n - 1) : 0u;

        for (int qi = 0; qi < nq; ++qi) {
            QueryRuns qr;
            {
                // the query's code and keys: wave-uniform addresses, scalar loads
                const int64_t q = (int64_t)q0 + qi;
                qr.qc0 = Q.codes[2 * q];
                qr.qc1 = Q.codes[2 * q + 1];
                const uint16_t* kqq = reinterpret_cast<const uint16_t*>(Q.keys + 6 * q);
                qr.qk = (uint64_t)kqq[0] | ((uint64_t)kqq[1] << 16) | ((uint64_t)kqq[2] << 32);
            }
            qr.P1 = readlane(v_P[0], qi); qr.P2 = readlane(v_P[1], qi); qr.P3 = readlane(v_P[2], qi);
            qr.P4 = readlane(v_P[3], qi); qr.P5 = readlane(v_P[4], qi); qr.P6 = readlane(v_P[5], qi);
            qr.cofs = cofs + 8 * qi;
            if constexpr (EPI) {
                qr.la = readlane_f64(v_la, qi);
                qr.lb = readlane_f64(v_lb, qi);
                qr.lc = readlane_f64(v_lc, qi);
            } else {
                qr.la = qr.lb = qr.lc = 0.0;
            }
            const uint32_t total = qr.P6;
            st_bucket += total;

            // ---- Steps 1-3, gather: union, Hamming, tau, band; index table
            clear_hist(hist, lane);
            uint32_t n_valid = 0;
            constexpr uint32_t kRegCap = 64u * NS;
            uint32_t kr[NS];  // candidate keys held in registers (up to kRegCap)
#pragma unroll
            for (int u = 0; u < NS; ++u) kr[u] = ~0u;
            bool in_regs = true;
            bool gathered = false;
            if (total == 0) {
                gathered = true;  // no candidate: nothing to read (the image may have no entries)
            } else if constexpr (EPI) {
                // band first: only keypoints are read for every bucket entry;
                // the ~1% inside the band are compacted (table, position) into
                // the LDS list and only they are read in full
                uint32_t n_surv = 0;
                for (uint32_t base = 0; base < total; base += 128) {
                    uint32_t t0, t1;
                    const uint32_t e0 = base + lane, e1 = base + 64u + lane;
                    const uint32_t p0 = entry_pos(e0, qr, t0), p1 = entry_pos(e1, qr, t1);
                    const bool ok0 = e0 < total && in_band(tv, p0, qr, dd);
                    const bool ok1 = e1 < total && in_band(tv, p1, qr, dd);
                    const uint64_t m0 = __ballot(ok0);
                    const uint32_t s0 = n_surv + mbcnt64(m0);
                    if (ok0 && s0 < (uint32_t)kListCap) list[s0] = (t0 << 24) | p0;
                    n_surv += (uint32_t)__popcll(m0);
                    const uint64_t m1 = __ballot(ok1);
                    const uint32_t s1 = n_surv + mbcnt64(m1);
                    if (ok1 && s1 < (uint32_t)kListCap) list[s1] = (t1 << 24) | p1;
                    n_surv += (uint32_t)__popcll(m1);
                }
                wave_sync();
                if (n_surv <= kRegCap && n_surv <= (uint32_t)kListCap) {
                    const uint32_t slots = (n_surv + 63u) >> 6;
#pragma unroll
                    for (int u = 0; u < NS; ++u) {
                        if ((uint32_t)u < slots) {
                            const uint32_t i = 64u * u + lane;
                            const bool live = i < n_surv;
                            const uint32_t packed = live ? list[i] : 0u;
                            kr[u] = entry_key(tv, packed >> 24, live ? (packed & 0xFFFFFFu) : 0u, live, qr, prm.tau,
                                              st_union);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < NS; ++u) {
                        const bool keep = kr[u] != ~0u;
                        if (keep) atomicAdd(&hist[kr[u] >> 16], 1u);
                        n_valid += (uint32_t)__popcll(__ballot(keep));
                    }
                    gathered = true;
                }
                wave_sync();
            }
            if (!gathered) {
                if (total <= kRegCap) {
                    // common case: every bucket entry of the query fits the
                    // register slots; exactly ceil(total / 64) chunks are read
                    const uint32_t nch = (total + 63u) >> 6;
                    switch (nch) {
#define GATHER_CASE(C)                                                                            \
    case C:                                                                                       \
        if constexpr (C <= NS) gather_chunks<EPI, C, NS>(kr, lane, tv, qr, prm.tau, dd, st_union); \
        break;
                        GATHER_CASE(1)
                        GATHER_CASE(2)
                        GATHER_CASE(3)
                        GATHER_CASE(4)
                        GATHER_CASE(5)
                        GATHER_CASE(6)
                        GATHER_CASE(7)
                        GATHER_CASE(8)
#undef GATHER_CASE
                        default:
                            break;
                    }
#pragma unroll
                    for (int u = 0; u < NS; ++u) {
                        if ((uint32_t)u < nch) {
                            const bool keep = kr[u] != ~0u;
                            if (keep) atomicAdd(&hist[kr[u] >> 16], 1u);
                            n_valid += (uint32_t)__popcll(__ballot(keep));
                        }
                    }
                } else {
                    for (uint32_t base = 0; base < total; base += 256) {
                        uint32_t kv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            kv[u] = key_at<EPI>(base + 64u * u + lane, tv, qr, prm.tau, dd, st_union);
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const bool keep = kv[u] != ~0u;
                            const uint64_t mk = __ballot(keep);
                            const uint32_t slot = n_valid + mbcnt64(mk);
                            if (keep) {
                                atomicAdd(&hist[kv[u] >> 16], 1u);
                                if (slot < (uint32_t)kListCap) list[slot] = kv[u];
                            }
                            n_valid += (uint32_t)__popcll(mk);
                        }
                    }
                    in_regs = n_valid <= kRegCap && n_valid <= (uint32_t)kListCap;
                    wave_sync();
                    if (in_regs) {
#pragma unroll
                        for (int u = 0; u < NS; ++u) {
                            const uint32_t e = 64u * u + lane;
                            kr[u] = e < n_valid ? list[e] : ~0u;
                        }
                    }
                }
            }
            wave_sync();
            const uint32_t kk = n_valid < (uint32_t)prm.k ? n_valid : (uint32_t)prm.k;
            st_ranked += kk;
            if (lane == qi) {
                my_kk = kk;
                my_off = sel_n;
            }
            if (kk == 0) continue;
            const bool in_list = n_valid <= (uint32_t)kListCap;
            const uint32_t span = in_list ? n_valid : total;
            uint32_t dummy = 0;
            // number of candidate keys in [lo, hi), counted with ballots
#define COUNT_RANGE(lo, hi, c)                                                                        \
    do {                                                                                              \
        c = 0;                                                                                        \
        if (in_regs) {                                                                                \
            _Pragma("unroll") for (int u = 0; u < NS; ++u) c +=                                \
                (uint32_t)__popcll(__ballot(kr[u] >= (lo) && kr[u] < (hi)));                          \
        } else {                                                                                      \
            for (uint32_t base = 0; base < span; base += 64) {                                        \
                const uint32_t e = base + lane;                                                       \
                const uint32_t key = in_list ? (e < n_valid ? list[e] : ~0u)                          \
                                             : key_at<EPI>(e, tv, qr, prm.tau, dd, dummy);            \
                c += (uint32_t)__popcll(__ballot(key >= (lo) && key < (hi)));                         \
            }                                                                                         \
        }                                                                                             \
    } while (0)

            // ---- Step 3: Hamming distance H* of the kk-th candidate from the index table
            uint32_t below;
            const uint32_t hs = hist_select(hist, kk, lane, &below);
            const uint32_t need = kk - below;
            const uint32_t ties = readlane(hist[hs], 0);
            uint32_t tkey;  // kept candidates: key <= tkey
            if (ties == need) {
                tkey = ((hs + 1u) << 16) - 1u;
            } else if (ties <= 64) {
                // few ties: gather their indices (the index table is no longer
                // needed) and rank each one against the others
                const uint32_t lo = hs << 16, hi = lo + 0x10000u;
                uint32_t nt = 0;
                if (in_regs) {
#pragma unroll
                    for (int u = 0; u < NS; ++u) {
                        const bool tie = kr[u] >= lo && kr[u] < hi;
                        const uint64_t mk = __ballot(tie);
                        const uint32_t slot = nt + mbcnt64(mk);
                        if (tie && slot < 256u) hist[slot] = kr[u] & 0xFFFFu;
                        nt += (uint32_t)__popcll(mk);
                    }
                } else {
                    for (uint32_t base = 0; base < span; base += 64) {
                        const uint32_t e = base + lane;
                        const uint32_t key = in_list ? (e < n_valid ? list[e] : ~0u)
                                                     : key_at<EPI>(e, tv, qr, prm.tau, dd, dummy);
                        const bool tie = key >= lo && key < hi;
                        const uint64_t mk = __ballot(tie);
                        const uint32_t slot = nt + mbcnt64(mk);
                        if (tie && slot < 256u) hist[slot] = key & 0xFFFFu;
                        nt += (uint32_t)__popcll(mk);
                    }
                }
                wave_sync();
                const uint32_t jl = (uint32_t)lane < ties ? hist[lane] : ~0u;
                uint32_t rank = 0;
                for (uint32_t m = 0; m < ties; ++m) rank += hist[m] < jl ? 1u : 0u;
                const uint64_t pick = __ballot((uint32_t)lane < ties && rank == need - 1u);
                tkey = lo | readlane(jl, __ffsll((unsigned long long)pick) - 1);
            } else {
                // many ties: the need-th smallest index among them, by counting
                // with ballots over a binary search of the index bits
                const uint32_t lo = hs << 16;
                uint32_t J = 0;
                for (int b = (int)jbits - 1; b >= 0; --b) {
                    const uint32_t J2 = J | (1u << b);
                    uint32_t cnt;
                    COUNT_RANGE(lo, lo | J2, cnt);
                    if (cnt < need) J = J2;
                }
                tkey = lo | J;
            }
            // compaction of the kept candidates into the tile list
            if (in_regs) {
#pragma unroll
                for (int u = 0; u < NS; ++u) {
                    const bool keep = kr[u] <= tkey;
                    const uint64_t mk = __ballot(keep);
                    const uint32_t slot = sel_n + mbcnt64(mk);
                    if (keep && slot < (uint32_t)kSelCap) sel[slot] = ((uint32_t)qi << 16) | (kr[u] & 0xFFFFu);
                    sel_n += (uint32_t)__popcll(mk);
                }
            } else {
                for (uint32_t base = 0; base < span; base += 64) {
                    const uint32_t e = base + lane;
                    const uint32_t key = in_list ? (e < n_valid ? list[e] : ~0u)
                                                 : key_at<EPI>(e, tv, qr, prm.tau, dd, dummy);
                    const bool keep = key <= tkey;
                    const uint64_t mk = __ballot(keep);
                    const uint32_t slot = sel_n + mbcnt64(mk);
                    if (keep && slot < (uint32_t)kSelCap) sel[slot] = ((uint32_t)qi << 16) | (key & 0xFFFFu);
                    sel_n += (uint32_t)__popcll(mk);
                }
            }
            wave_sync();
        }
#undef COUNT_RANGE
        if (sel_n > (uint32_t)kSelCap) sel_n = kSelCap;  // cannot happen when nq * k <= kSelCap

        // ---- Step 4: squared distances of all kept pairs of the tile, 4 lanes per pair
        for (uint32_t p0 = 0; p0 < sel_n; p0 += 32) {
            uint32_t dpv[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t p = p0 + 16u * h + (uint32_t)(lane >> 2);
                const bool act = p < sel_n;
                const uint32_t e = act ? sel[p] : 0u;
                const uint32_t qi = e >> 16;
                const uint32_t j = min(e & 0xFFFFu, (uint32_t)(tv.n - 1));
                const uint4* ap = reinterpret_cast<const uint4*>(Q.desc + (int64_t)(q0 + (int)qi) * kDim + part * 32);
                const uint4* bp = reinterpret_cast<const uint4*>(T.desc + (int64_t)j * kDim + part * 32);
                const uint4 a0 = gload(ap), a1 = gload(ap + 1), b0 = gload(bp), b1 = gload(bp + 1);
                const uint32_t av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
                const uint32_t bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
                uint32_t aa = 0, ab = 0, bb = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    aa = __builtin_amdgcn_udot4(av[i], av[i], aa, false);
                    ab = __builtin_amdgcn_udot4(av[i], bv[i], ab, false);
                    bb = __builtin_amdgcn_udot4(bv[i], bv[i], bb, false);
                }
                dpv[h] = aa + bb - 2u * ab;  // sum over this lane's 32 components of (a - b)^2
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint32_t d = dpv[h] + dpp<0xB1, 0xf>(dpv[h]);  // quad_perm [1,0,3,2]
                d += dpp<0x4E, 0xf>(d);                        // quad_perm [2,3,0,1]
                const uint32_t p = p0 + 16u * h + (uint32_t)(lane >> 2);
                if (part == 0 && p < sel_n) list[p] = d;
            }
        }
        wave_sync();

        // ---- nearest, second nearest and ratio test, one lane per query
        if (lane < nq) {
            uint64_t best = ~0ull;
            uint32_t sec = ~0u;
            for (uint32_t s = 0; s < my_kk; ++s) {
                const uint32_t d = list[my_off + s];
                const uint32_t j = sel[my_off + s] & 0xFFFFu;
                const uint64_t c = ((uint64_t)d << 32) | j;
                if (c < best) {
                    sec = min(sec, (uint32_t)(best >> 32));
                    best = c;
                } else {
                    sec = min(sec, d);
                }
            }
            int32_t r_idx = -1, r_d1 = -1, r_d2 = -1;
            if (my_kk >= 1) r_d1 = (int32_t)(best >> 32);
            if (my_kk >= 2) {
                r_d2 = (int32_t)sec;
                if (prm.den2 * (int64_t)r_d1 < prm.num2 * (int64_t)r_d2) r_idx = (int32_t)(uint32_t)best;
            }
            const int64_t o = pr.out + q0 + lane;
            o_idx[o] = r_idx;
            o_d1[o] = r_d1;
            o_d2[o] = r_d2;
        }
        wave_sync();
        if (!counter) break;
    }
    // statistics: bucket entries and ranked counts (uniform), union sizes (per lane)
    uint64_t u64 = st_union;
    for (int d = 32; d >= 1; d >>= 1) u64 += __shfl_xor(u64, d);
    if (lane == 0 && stats) {
        atomicAdd(&stats[0], (unsigned long long)st_bucket);
        atomicAdd(&stats[1], (unsigned long long)u64);
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

hipError_t launch_make_items(hipStream_t s, const PairTiles* pt, int32_t n_pt, const PairDev* pairs,
                             const ImgDev* imgs, int32_t qt, Item* items, int32_t n_items) {
    if (n_items <= 0) return hipSuccess;
    CH_LAUNCH(make_items_kernel, dim3((unsigned)((n_items + 255) / 256)), dim3(256), 0, s, pt, n_pt, pairs, imgs, qt,
              items, n_items);
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
                            int n_tiles, const uint4* frag, const float* bias, float margin, NearEntry* near,
                            unsigned int* near_count) {
    if (n_tiles <= 0) return hipSuccess;
    CH_LAUNCH(proj_mfma_kernel, dim3(grid), dim3(256), 0, s, imgs, outs, tiles, n_tiles, frag, bias, margin, near,
              near_count);
    return hipSuccess;
}

hipError_t launch_proj_fp32(hipStream_t s, const ImgDev* imgs, const CodeOut* outs, const RowChunk* tiles,
                            int n_tiles, const float* R32, const float* bias, float margin, NearEntry* near,
                            unsigned int* near_count) {
    if (n_tiles <= 0) return hipSuccess;
    const int64_t threads = (int64_t)n_tiles * 16;
    CH_LAUNCH(proj_fp32_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, imgs, outs, tiles, n_tiles,
              R32, bias, margin, near, near_count);
    return hipSuccess;
}

hipError_t launch_fixup(hipStream_t s, int grid, const ImgDev* imgs, const CodeOut* outs, const NearEntry* near,
                        const unsigned int* near_count, const double* R, const unsigned long long* S, double n_tot,
                        unsigned long long* counter) {
    CH_LAUNCH(fixup_kernel, dim3(grid), dim3(256), 0, s, imgs, outs, near, near_count, R, S, n_tot, counter);
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

hipError_t launch_match(hipStream_t s, bool epi, int ns, int grid, const ImgDev* imgs, const PairDev* pairs,
                        const Item* items, int32_t n_items, uint32_t* counter, const MatchParams& prm, int32_t* o_idx,
                        int32_t* o_d1, int32_t* o_d2, unsigned long long* stats) {
    if (n_items <= 0 || grid <= 0) return hipSuccess;
    const dim3 g(grid), b(64 * kWavesPerBlock);
    if (epi && ns > 4)
        CH_LAUNCH((match_kernel<true, 8>), g, b, 0, s, imgs, pairs, items, n_items, counter, prm, o_idx, o_d1, o_d2, stats);
    else if (epi)
        CH_LAUNCH((match_kernel<true, 4>), g, b, 0, s, imgs, pairs, items, n_items, counter, prm, o_idx, o_d1, o_d2, stats);
    else if (ns > 4)
        CH_LAUNCH((match_kernel<false, 8>), g, b, 0, s, imgs, pairs, items, n_items, counter, prm, o_idx, o_d1, o_d2,
                  stats);
    else
        CH_LAUNCH((match_kernel<false, 4>), g, b, 0, s, imgs, pairs, items, n_items, counter, prm, o_idx, o_d1, o_d2,
                  stats);
    return hipSuccess;
}

}  // namespace cashash
