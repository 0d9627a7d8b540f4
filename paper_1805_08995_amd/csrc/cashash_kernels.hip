// HIP kernels of the hash-code and bucket-table steps for gfx950 (MI355X).
//
// Hash codes ("The Improved Parallel Calculation of Hashing Code"): the
// paper's one-block-per-(point, bit) reduction is replaced by a dense
// contraction on the matrix cores: descriptors (uint8, exact in bf16) times
// the projection rows split into bf16 hi + lo parts, fp32 accumulate.  A
// projection whose value lies within a proven rounding margin of zero is
// recomputed in binary64 exactly as the reference definition does it.
// Bucket tables: per train image and table, a stable counting sort of the
// 8-bit keys whose entries carry code, keys and index (Step 1 lookup runs).
#include <algorithm>

#include "cashash_device.h"

namespace cashash {

// ------------------------------------------------------------------ utilities

// Control words of the binary64 recompute (jobs per row, overflow flag),
// cleared by block 0 of the projection kernel (256 threads) before use.
constexpr int kNearCtlWords = 256;

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
// binary64 recompute) and, if any row is flagged, appends it to the
// wavefront's own segment of the near list (seg[cnt ..]); cnt is the
// wave-uniform fill of that segment.  No atomics: each wave owns its segment.
__device__ __forceinline__ void store_code(const CodeOut& o, int img, int row, bool live, uint64_t w0, uint64_t w1,
                                           uint64_t w2, uint64_t m0, uint64_t m1, uint64_t m2,
                                           NearEntry* __restrict__ seg, uint32_t& cnt) {
    if (live) {
        gstore(reinterpret_cast<ulonglong2*>(o.codes) + row, make_ulonglong2(w0, w1));
        uint16_t* kp = reinterpret_cast<uint16_t*>(o.keys + 6 * (int64_t)row);
        gstore(kp, (uint16_t)(w2 & 0xFFFFu));
        gstore(kp + 1, (uint16_t)((w2 >> 16) & 0xFFFFu));
        gstore(kp + 2, (uint16_t)((w2 >> 32) & 0xFFFFu));
    }
    const bool flagged = live && (m0 | m1 | m2) != 0;
    const uint64_t fm = __ballot(flagged);
    if (fm == 0) return;
    if (flagged) {
        NearEntry& e = seg[cnt + mbcnt64(fm)];
        e.img = img;
        e.row = row;
        e.mask[0] = m0;
        e.mask[1] = m1;
        e.mask[2] = m2;
    }
    cnt += (uint32_t)__popcll(fm);
}

// BF16 hi+lo split on MFMA.  One wave per group of kProjTB tiles of 16
// descriptors: for each of the 11 row tiles, D[16 rows][16 desc] = sum over
// 4 k-steps of (R_hi + R_lo)[rows][32 k] x X^T[32 k][desc] with
// v_mfma_f32_16x16x32_bf16.  Each fragment of R is loaded once per group and
// applied to every tile of it.  Lane l holds descriptor l % 16 of each tile
// and rows 4 (l / 16) .. +3 of each row tile.
__global__ __launch_bounds__(256) void proj_mfma_kernel(const ImgDev* __restrict__ imgs,
                                                        const CodeOut* __restrict__ outs,
                                                        const RowChunk* __restrict__ tiles, int n_tiles,
                                                        const uint4* __restrict__ frag,
                                                        const float* __restrict__ bias, float margin_coef,
                                                        NearEntry* __restrict__ near,
                                                        uint32_t* __restrict__ seg_count, uint32_t seg_cap,
                                                        uint32_t* __restrict__ near_ctl) {
    if (blockIdx.x == 0) near_ctl[threadIdx.x] = 0u;  // the recompute's control words (kNearCtlWords)
    constexpr int TB = kProjTB;
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int n_waves = (gridDim.x * blockDim.x) >> 6;
    const int wave = (int)uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    NearEntry* seg = near + (size_t)wave * seg_cap;
    uint32_t cnt = 0;
    for (int t0 = wave * TB; t0 < n_tiles; t0 += n_waves * TB) {
        RowChunk tc[TB];
        bool live[TB];
        bf16x8 xb[TB][4];
        float base_margin[TB];
#pragma unroll
        for (int b = 0; b < TB; ++b) {
            const bool in = t0 + b < n_tiles;
            tc[b] = tiles[in ? t0 + b : t0];
            live[b] = in && n < tc[b].nr;
            const uint8_t* x = imgs[tc[b].img].desc + (int64_t)(tc[b].r0 + (live[b] ? n : 0)) * kDim;
            uint32_t sq = 0;
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const uint2 w = live[b] ? gload(reinterpret_cast<const uint2*>(x + 32 * ks + 8 * g)) : make_uint2(0u, 0u);
                sq = __builtin_amdgcn_udot4(w.x, w.x, sq, false);
                sq = __builtin_amdgcn_udot4(w.y, w.y, sq, false);
                xb[b][ks] = bytes_to_bf16x8(w);
            }
            sq += __shfl_xor(sq, 16);
            sq += __shfl_xor(sq, 32);
            base_margin[b] = margin_coef * sqrtf((float)sq) + 0x1p-26f;
        }
        // this lane's bits, packed: row 16 rw + 4 g + i of row block k at bit
        // 16 (k & 1) + 4 rw + i of word k >> 1 (its own g only)
        uint32_t pw[TB][2], pm[TB][2];
#pragma unroll
        for (int b = 0; b < TB; ++b) pw[b][0] = pw[b][1] = pm[b][0] = pm[b][1] = 0u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int n_rt = k < 2 ? 4 : kRowTiles - 8;
#pragma unroll 1
            for (int rw = 0; rw < n_rt; ++rw) {
                const int rt = 4 * k + rw;
                f32x4 acc[TB];
#pragma unroll
                for (int b = 0; b < TB; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const bf16x8 fh = load_frag(frag, ((0 * kRowTiles + rt) * 4 + ks) * 64 + lane);
                    const bf16x8 fl = load_frag(frag, ((1 * kRowTiles + rt) * 4 + ks) * 64 + lane);
#pragma unroll
                    for (int b = 0; b < TB; ++b) {
                        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh, xb[b][ks], acc[b], 0, 0, 0);
                        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fl, xb[b][ks], acc[b], 0, 0, 0);
                    }
                }
                const float4 bq = reinterpret_cast<const float4*>(bias)[rt * 4 + g];
                const float bv[4] = {bq.x, bq.y, bq.z, bq.w};
#pragma unroll
                for (int b = 0; b < TB; ++b)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float v = acc[b][i] - bv[i];
                        const float M = base_margin[b] + 0x1p-20f * fabsf(bv[i]);
                        const bool nr = !(fabsf(v) > M);
                        const bool bit = !nr && v > 0.f;
                        const int pos = 16 * (k & 1) + 4 * rw + i;
                        pw[b][k >> 1] |= (uint32_t)bit << pos;
                        pm[b][k >> 1] |= (uint32_t)nr << pos;
                    }
            }
        }
        // unpack to rows 16 rw + 4 g + i (g: this lane's row group)
        auto unpack = [&](uint32_t p16) {
            uint64_t r = 0;
#pragma unroll
            for (int rw = 0; rw < 4; ++rw) r |= (uint64_t)((p16 >> (4 * rw)) & 0xFu) << (16 * rw + 4 * g);
            return r;
        };
#pragma unroll
        for (int b = 0; b < TB; ++b) {
            uint64_t w[3] = {unpack(pw[b][0] & 0xFFFFu), unpack(pw[b][0] >> 16), unpack(pw[b][1])};
            uint64_t m[3] = {unpack(pm[b][0] & 0xFFFFu), unpack(pm[b][0] >> 16), unpack(pm[b][1])};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                w[k] |= __shfl_xor(w[k], 16);
                w[k] |= __shfl_xor(w[k], 32);
                m[k] |= __shfl_xor(m[k], 16);
                m[k] |= __shfl_xor(m[k], 32);
            }
            store_code(outs[tc[b].img], tc[b].img, tc[b].r0 + n, g == 0 && live[b], w[0], w[1], w[2], m[0], m[1],
                       m[2], seg, cnt);
        }
    }
    if (lane == 0) seg_count[wave] = cnt;
}

// Plain FP32 form: one thread per descriptor, 176 fp32 FMA chains over the
// descriptor held in registers; the rows are wave-uniform scalar loads.
__global__ __launch_bounds__(256) void proj_fp32_kernel(const ImgDev* __restrict__ imgs,
                                                        const CodeOut* __restrict__ outs,
                                                        const RowChunk* __restrict__ tiles, int n_tiles,
                                                        const float* __restrict__ R32,
                                                        const float* __restrict__ bias, float margin_coef,
                                                        NearEntry* __restrict__ near,
                                                        uint32_t* __restrict__ seg_count,
                                                        uint32_t* __restrict__ near_ctl) {
    if (blockIdx.x == 0) near_ctl[threadIdx.x] = 0u;  // the recompute's control words (kNearCtlWords)
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
    // one 64-entry segment per wavefront
    const int wave = t >> 6;
    uint32_t cnt = 0;
    store_code(outs[tc.img], tc.img, tc.r0 + n, live, w[0], w[1], w[2], m[0], m[1], m[2], near + (size_t)wave * 64,
               cnt);
    if ((t & 63) == 0) seg_count[wave] = cnt;
}

// ------------------------------------------------------------------ binary64 recompute
// Near-margin projections are recomputed with the same fused multiply-add
// chain over components 0..127 of r_j . (N x - S) that defines the codes
// (N x_i - S_i is an exact integer in binary64).  A recompute is a job
// (near-list entry, row j).  The jobs are grouped by row first, so that the
// wavefront evaluating 64 of them reads one row of R, with wave-uniform
// (scalar) loads, and only the descriptors differ per lane:
//   near_sort  : per block of kSortSegs near-list segments, count the jobs
//                of each row, reserve their places in the row's region of
//                the job list (one atomic per block and row), place them;
//                clear the result bits of the entries;
//   near_eval  : one wavefront per 64 jobs of one row; a positive value ORs
//                the row's bit into the entry's result bits;
//   near_apply : the result bits ORed into each entry's code and keys (one
//                thread per entry, the only writer of that descriptor).
// A row region holds cap_r jobs.  If some row has more, near_eval takes its
// spread form instead: the jobs of each segment are spread over the lanes
// as they come (any row per lane, rows read with vector loads); the results
// are the same.  Block sizes measured on 800k descriptors (190k jobs):
// 32 segments per near_sort block (fewer blocks: longer passes; more: more
// row reservations), 8 per near_apply block (about one entry per thread).
constexpr int kSortSegs = 32;
constexpr int kApplySegs = 8;

struct NearJob {
    uint32_t entry;       // near-list index sg * seg_cap + i
    uint32_t pad;
    const uint8_t* x;     // the descriptor
};

constexpr int kNearOverflow = kRows;  // control word: some row has more jobs than its region

// The near-list entries of a block's SEGS segments from s0 on, flattened:
// s_pre[j] is the number of entries in segments s0 .. s0 + j - 1.
template <int SEGS>
__device__ __forceinline__ uint32_t near_entry_of(const uint32_t* s_pre, uint32_t i, uint32_t s0, uint32_t seg_cap) {
    uint32_t j = 0;
#pragma unroll
    for (uint32_t step = SEGS / 2; step >= 1; step >>= 1)
        if (s_pre[j + step] <= i) j += step;
    return (s0 + j) * seg_cap + (i - s_pre[j]);
}

template <int SEGS>
__device__ __forceinline__ void near_block_prefix(uint32_t* s_pre, const uint32_t* seg_count, uint32_t s0,
                                                  uint32_t n_seg) {
    static_assert(SEGS >= 2 && SEGS <= 64 && (SEGS & (SEGS - 1)) == 0, "SEGS: a power of two up to 64");
    if (threadIdx.x < 64) {
        const uint32_t t = threadIdx.x;
        const uint32_t c = (t < SEGS && s0 + t < n_seg) ? seg_count[s0 + t] : 0u;
        const uint32_t incl = wave_incl_scan(c, (int)t);
        if (t < SEGS) s_pre[t + 1] = incl;
        if (t == 0) s_pre[0] = 0;
    }
}

__global__ __launch_bounds__(256) void near_sort_kernel(const ImgDev* __restrict__ imgs,
                                                        const NearEntry* __restrict__ near,
                                                        const uint32_t* __restrict__ seg_count, uint32_t seg_cap,
                                                        uint32_t n_seg, unsigned long long* __restrict__ res,
                                                        uint32_t* __restrict__ ctl, NearJob* __restrict__ jobs,
                                                        uint32_t cap_r, unsigned long long* __restrict__ counter) {
    __shared__ uint32_t s_pre[kSortSegs + 1];
    __shared__ uint32_t s_hist[kRows];
    __shared__ uint32_t s_tot[4];
    const uint32_t s0 = blockIdx.x * kSortSegs;
    near_block_prefix<kSortSegs>(s_pre, seg_count, s0, n_seg);
    for (int r = threadIdx.x; r < kRows; r += blockDim.x) s_hist[r] = 0;
    __syncthreads();
    const uint32_t n_ent = s_pre[kSortSegs];
    // pass 1: jobs per row; result bits cleared
    uint32_t tot = 0;
    for (uint32_t i = threadIdx.x; i < n_ent; i += blockDim.x) {
        const uint32_t e = near_entry_of<kSortSegs>(s_pre, i, s0, seg_cap);
        const NearEntry ne = near[e];
#pragma unroll
        for (int w = 0; w < 3; ++w) {
            res[3 * (size_t)e + w] = 0ull;
            for (uint64_t m = ne.mask[w]; m; m &= m - 1) {
                atomicAdd(&s_hist[64 * w + __ffsll((unsigned long long)m) - 1], 1u);
                ++tot;
            }
        }
    }
    tot += __shfl_xor(tot, 1);
    tot += __shfl_xor(tot, 2);
    tot += __shfl_xor(tot, 4);
    tot += __shfl_xor(tot, 8);
    tot += __shfl_xor(tot, 16);
    tot += __shfl_xor(tot, 32);
    if ((threadIdx.x & 63) == 0) s_tot[threadIdx.x >> 6] = tot;
    __syncthreads();
    // reserve each row's places (s_hist becomes the row's next free place)
    for (int r = threadIdx.x; r < kRows; r += blockDim.x) {
        const uint32_t h = s_hist[r];
        uint32_t b = 0;
        if (h) {
            b = atomicAdd(&ctl[r], h);
            if (b + h > cap_r) ctl[kNearOverflow] = 1u;
        }
        s_hist[r] = b;
    }
    if (threadIdx.x == 0) {
        const uint32_t t = s_tot[0] + s_tot[1] + s_tot[2] + s_tot[3];
        if (t) atomicAdd(counter, (unsigned long long)t);
    }
    __syncthreads();
    // pass 2: place the jobs
    for (uint32_t i = threadIdx.x; i < n_ent; i += blockDim.x) {
        const uint32_t e = near_entry_of<kSortSegs>(s_pre, i, s0, seg_cap);
        const NearEntry ne = near[e];
        const uint8_t* x = imgs[ne.img].desc + (int64_t)ne.row * kDim;
#pragma unroll
        for (int w = 0; w < 3; ++w)
            for (uint64_t m = ne.mask[w]; m; m &= m - 1) {
                const int r = 64 * w + __ffsll((unsigned long long)m) - 1;
                const uint32_t pos = atomicAdd(&s_hist[r], 1u);
                if (pos < cap_r) jobs[(size_t)r * cap_r + pos] = NearJob{e, 0u, x};
            }
    }
}

// The binary64 chain of one descriptor x (per lane) against row rp: c_i =
// N x_i - S_i exactly, then p = fma(r_i, c_i, p) for i = 0 .. 127.
__device__ __forceinline__ double near_chain_q(double p, uint4 xv, const double rv[16], const double* s_S, int q,
                                               double n_tot) {
    const uint32_t xw[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
            const int ci = 16 * q + 4 * a + bb;
            const double c = n_tot * (double)((xw[a] >> (8 * bb)) & 0xFFu) - s_S[ci];
            p = fma(rv[4 * a + bb], c, p);
        }
    return p;
}

// Row rp the same for the whole wavefront (scalar loads).  The descriptor is
// loaded whole; the scheduling barriers keep the conversions of each group
// of 16 components next to their multiply-adds (hoisting all 128 would need
// 256 registers).
__device__ __forceinline__ double near_chain_uniform(const uint8_t* x, const double* __restrict__ rp,
                                                     const double* s_S, double n_tot) {
    const uint4* xp = reinterpret_cast<const uint4*>(x);
    uint4 xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xv[q] = gload(xp + q);
    double p = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        double rv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) rv[i] = rp[16 * q + i];
        p = near_chain_q(p, xv[q], rv, s_S, q, n_tot);
        __builtin_amdgcn_sched_barrier(0);
    }
    return p;
}

// Row rp per lane (vector loads, 16 components at a time).
__device__ __forceinline__ double near_chain_lane(const uint8_t* x, const double* rp, const double* s_S,
                                                  double n_tot) {
    const uint4* xp = reinterpret_cast<const uint4*>(x);
    const double2* rr = reinterpret_cast<const double2*>(rp);
    double p = 0.0;
#pragma unroll 1
    for (int q = 0; q < 8; ++q) {
        double rv[16];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const double2 v = rr[8 * q + i];
            rv[2 * i] = v.x;
            rv[2 * i + 1] = v.y;
        }
        p = near_chain_q(p, gload(xp + q), rv, s_S, q, n_tot);
        __builtin_amdgcn_sched_barrier(0);
    }
    return p;
}

// The spread form of the recompute, used when some row has more jobs than
// its region holds: per segment, the (entry, row) jobs of up to 64 entries
// are spread over the lanes 64 at a time, whichever entry they belong to.
__device__ __forceinline__ void near_eval_spread(const ImgDev* __restrict__ imgs, const NearEntry* __restrict__ near,
                                                 const uint32_t* __restrict__ seg_count, uint32_t seg_cap,
                                                 uint32_t n_seg, const double* __restrict__ R, const double* s_S,
                                                 double n_tot, unsigned long long* __restrict__ res, uint32_t* s_fb,
                                                 int lane, uint32_t wave, uint32_t n_waves) {
    for (uint32_t sg = wave; sg < n_seg; sg += n_waves) {
        const uint32_t ns = uniform(seg_count[sg]);
        for (uint32_t base = 0; base < ns; base += 64) {
            const uint32_t i = base + (uint32_t)lane;
            const bool has = i < ns;
            NearEntry e{};
            if (has) e = near[(size_t)sg * seg_cap + i];
            const uint32_t pc = has ? (uint32_t)(__popcll(e.mask[0]) + __popcll(e.mask[1]) + __popcll(e.mask[2])) : 0u;
            const uint32_t incl = wave_incl_scan(pc, lane);
            const uint32_t total = uniform(__shfl(incl, 63));
            s_fb[lane] = incl;
            wave_sync();
            for (uint32_t j0 = 0; j0 < total; j0 += 64) {
                const uint32_t j = j0 + (uint32_t)lane;
                const bool act = j < total;
                // owner: the first entry whose inclusive prefix exceeds j
                uint32_t L = 0;
#pragma unroll
                for (uint32_t step = 32; step >= 1; step >>= 1)
                    if (s_fb[L + step - 1] <= j) L += step;
                L = act ? L : 0u;
                const uint32_t start = L ? s_fb[L - 1] : 0u;
                uint32_t kth = act ? j - start : 0u;
                const uint64_t m0 = __shfl(e.mask[0], (int)L), m1 = __shfl(e.mask[1], (int)L),
                               m2 = __shfl(e.mask[2], (int)L);
                const int img = __shfl(e.img, (int)L), row = __shfl(e.row, (int)L);
                // the kth set bit of the owner's 176-bit mask
                int word = 0;
                uint64_t w = m0;
                const uint32_t c0 = (uint32_t)__popcll(m0), c1 = (uint32_t)__popcll(m1);
                if (kth >= c0) {
                    kth -= c0;
                    word = 1;
                    w = m1;
                    if (kth >= c1) {
                        kth -= c1;
                        word = 2;
                        w = m2;
                    }
                }
                for (uint32_t t = 0; t < kth; ++t) w &= w - 1;
                const int bitpos = w ? __ffsll((unsigned long long)w) - 1 : 0;
                if (act) {
                    const int r = 64 * word + bitpos;
                    const double p =
                        near_chain_lane(imgs[img].desc + (int64_t)row * kDim, R + (size_t)r * kDim, s_S, n_tot);
                    if (p > 0.0)
                        atomicOr(&res[3 * ((size_t)sg * seg_cap + base + L) + word], 1ull << bitpos);
                }
            }
            wave_sync();  // s_fb is rewritten by the next batch
        }
    }
}

__global__ __launch_bounds__(256) void near_eval_kernel(const NearJob* __restrict__ jobs, uint32_t cap_r,
                                                        const uint32_t* __restrict__ ctl,
                                                        const double* __restrict__ R,
                                                        const unsigned long long* __restrict__ S, double n_tot,
                                                        unsigned long long* __restrict__ res,
                                                        const ImgDev* __restrict__ imgs,
                                                        const NearEntry* __restrict__ near,
                                                        const uint32_t* __restrict__ seg_count, uint32_t seg_cap,
                                                        uint32_t n_seg) {
    __shared__ double s_S[kDim];
    __shared__ uint32_t s_pre[kRows + 1];  // first 64-job chunk of each row
    __shared__ uint32_t s_n[kRows];        // jobs of each row
    __shared__ uint32_t s_fb[4][64];       // spread form: per wave, inclusive prefix of jobs per entry
    for (int i = threadIdx.x; i < kDim; i += blockDim.x) s_S[i] = (double)S[i];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t wave = uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const bool overflow = uniform(ctl[kNearOverflow]) != 0u;
    if (!overflow && threadIdx.x < 64) {
        // lane l: rows 3l .. 3l + 2
        uint32_t c[3], sum = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int r = 3 * lane + a;
            const uint32_t n = r < kRows ? min(ctl[r], cap_r) : 0u;
            if (r < kRows) s_n[r] = n;
            c[a] = (n + 63) >> 6;
            sum += c[a];
        }
        const uint32_t incl = wave_incl_scan(sum, lane);
        uint32_t run = incl - sum;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int r = 3 * lane + a;
            if (r < kRows) s_pre[r] = run;
            run += c[a];
        }
        if (lane == 63) s_pre[kRows] = incl;
    }
    __syncthreads();
    if (overflow) {
        near_eval_spread(imgs, near, seg_count, seg_cap, n_seg, R, s_S, n_tot, res, s_fb[wv], lane, wave, n_waves);
        return;
    }
    const uint32_t n_chunks = uniform(s_pre[kRows]);
    for (uint32_t ch = wave; ch < n_chunks; ch += n_waves) {
        // the row: the last one whose first chunk is <= ch
        uint32_t r = 0;
#pragma unroll
        for (uint32_t step = 128; step >= 1; step >>= 1)
            if (r + step < kRows && s_pre[r + step] <= ch) r += step;
        r = uniform(r);
        const uint32_t j = 64 * (ch - s_pre[r]) + (uint32_t)lane;
        if (j < s_n[r]) {
            const NearJob jb = jobs[(size_t)r * cap_r + j];
            const double p = near_chain_uniform(jb.x, R + (size_t)r * kDim, s_S, n_tot);
            if (p > 0.0) atomicOr(&res[3 * (size_t)jb.entry + (r >> 6)], 1ull << (r & 63));
        }
    }
}

__global__ __launch_bounds__(256) void near_apply_kernel(const CodeOut* __restrict__ outs,
                                                         const NearEntry* __restrict__ near,
                                                         const uint32_t* __restrict__ seg_count, uint32_t seg_cap,
                                                         uint32_t n_seg, const unsigned long long* __restrict__ res) {
    __shared__ uint32_t s_pre[kApplySegs + 1];
    const uint32_t s0 = blockIdx.x * kApplySegs;
    near_block_prefix<kApplySegs>(s_pre, seg_count, s0, n_seg);
    __syncthreads();
    const uint32_t n_ent = s_pre[kApplySegs];
    for (uint32_t i = threadIdx.x; i < n_ent; i += blockDim.x) {
        const uint32_t e = near_entry_of<kApplySegs>(s_pre, i, s0, seg_cap);
        const uint64_t b0 = res[3 * (size_t)e], b1 = res[3 * (size_t)e + 1], b2 = res[3 * (size_t)e + 2];
        if (!(b0 | b1 | b2)) continue;
        const NearEntry ne = near[e];
        const CodeOut o = outs[ne.img];
        const int64_t row = ne.row;
        if (b0 | b1) {
            o.codes[2 * row] |= b0;
            o.codes[2 * row + 1] |= b1;
        }
        if (b2) {
            uint8_t* kb = o.keys + 6 * row;
            for (int tb = 0; tb < kTables; ++tb) kb[tb] = (uint8_t)(kb[tb] | ((b2 >> (8 * tb)) & 0xFFu));
        }
    }
}

// ------------------------------------------------------------------ bucket tables
// One block of kBucketWaves wavefronts per (train image, table): a stable
// counting sort of the 8-bit keys into 256 buckets (ascending index inside a
// bucket).  Wave w owns a contiguous slice of the entries: it counts its
// slice's keys, the block scans the bucket totals and gives each wave its
// start inside every bucket, then each wave scatters its slice in order.
// Ranks inside a 64-wide chunk come from eight key-bit ballots.
template <bool EPI>
__global__ __launch_bounds__(64 * kBucketWaves) void bucket_kernel(const ImgDev* __restrict__ imgs,
                                                                   const TableOut* __restrict__ touts,
                                                                   const int32_t* __restrict__ train_list) {
    __shared__ uint32_t cnt[kBucketWaves][256];  // per-wave counts, then per-wave write positions
    __shared__ uint32_t wsum[4];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int m = train_list[blockIdx.x / kTables];
    const int t = blockIdx.x % kTables;
    const ImgDev im = imgs[m];
    const TableOut to = touts[m];
    const int n = im.n;
    // this wave's slice [lo, hi), a whole number of 64-entry chunks
    const int per = ((n + 64 * kBucketWaves - 1) / (64 * kBucketWaves)) * 64;
    const int lo = min(n, wv * per), hi = min(n, lo + per);
#pragma unroll
    for (int i = 0; i < 4; ++i) cnt[wv][4 * lane + i] = 0;
    __syncthreads();
#pragma unroll 4
    for (int j = lo + lane; j < hi; j += 64) atomicAdd(&cnt[wv][gload(im.keys + 6 * (int64_t)j + t)], 1u);
    __syncthreads();
    // thread b < 256 of the block owns bucket b
    static_assert(64 * kBucketWaves >= 256, "a thread per bucket");
    const int bk = threadIdx.x;
    uint32_t c[kBucketWaves], tot = 0, incl = 0;
    if (bk < 256) {
#pragma unroll
        for (int w = 0; w < kBucketWaves; ++w) {
            c[w] = cnt[w][bk];
            tot += c[w];
        }
        incl = wave_incl_scan(tot, lane);
        if (lane == 63) wsum[wv] = incl;
    }
    __syncthreads();
    if (bk < 256) {
        uint32_t start = incl - tot;
        for (int w = 0; w < wv; ++w) start += wsum[w];
        uint32_t* off = to.off + t * kOffStride;
        gstore(off + bk, start);
        if (bk == 255) gstore(off + 256, start + tot);
#pragma unroll
        for (int w = 0; w < kBucketWaves; ++w) {
            cnt[w][bk] = start;
            start += c[w];
        }
    }
    __syncthreads();
    ulonglong2* out_code = reinterpret_cast<ulonglong2*>(to.ent) + (int64_t)t * n;
    uint64_t* out_kid = reinterpret_cast<uint64_t*>(to.ent + (size_t)kTables * n * 16) + (int64_t)t * n;
    float2* out_kp = reinterpret_cast<float2*>(to.ent + (size_t)kTables * n * 24) + (int64_t)t * n;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t* wc = cnt[wv];
    for (int c0 = lo; c0 < hi; c0 += 64) {
        const int j = c0 + lane;
        const bool valid = j < hi;
        const uint32_t key = valid ? gload(im.keys + 6 * (int64_t)j + t) : 0u;
        uint64_t eq = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool kb = (key >> b) & 1u;
            const uint64_t bm = __ballot(kb);
            eq &= kb ? bm : ~bm;
        }
        const uint32_t rank = __popcll(eq & lt_mask);
        uint32_t pos = 0;
        if (valid) pos = wc[key] + rank;
        wave_sync();  // every lane has read its bucket's position before the first lane advances it
        if (valid) {
            const uint16_t* kp = reinterpret_cast<const uint16_t*>(im.keys + 6 * (int64_t)j);
            gstore(out_code + pos, gload(reinterpret_cast<const ulonglong2*>(im.codes) + j));
            gstore(out_kid + pos, (uint64_t)gload(kp) | ((uint64_t)gload(kp + 1) << 16) |
                                      ((uint64_t)gload(kp + 2) << 32) | ((uint64_t)j << 48));
            if constexpr (EPI) gstore(out_kp + pos, gload(reinterpret_cast<const float2*>(im.kp) + j));
            if (rank == 0) wc[key] = pos + (uint32_t)__popcll(eq);
        }
        wave_sync();
    }
}

// ------------------------------------------------------------------ launchers
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
                            uint32_t* seg_count, uint32_t seg_cap, void* near_work) {
    if (n_tiles <= 0) return hipSuccess;
    CH_LAUNCH(proj_mfma_kernel, dim3(grid), dim3(256), 0, s, imgs, outs, tiles, n_tiles, frag, bias, margin, near,
              seg_count, seg_cap, static_cast<uint32_t*>(near_work));
    return hipSuccess;
}

hipError_t launch_proj_fp32(hipStream_t s, const ImgDev* imgs, const CodeOut* outs, const RowChunk* tiles,
                            int n_tiles, const float* R32, const float* bias, float margin, NearEntry* near,
                            uint32_t* seg_count, void* near_work) {
    if (n_tiles <= 0) return hipSuccess;
    const int64_t threads = (int64_t)n_tiles * 16;
    CH_LAUNCH(proj_fp32_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, imgs, outs, tiles, n_tiles,
              R32, bias, margin, near, seg_count, static_cast<uint32_t*>(near_work));
    return hipSuccess;
}

uint32_t near_row_cap(uint64_t n_cap) {
    const uint64_t c = std::max<uint64_t>(64, (n_cap + kRows - 1) / kRows);
    return (uint32_t)((c + 63) & ~uint64_t(63));
}

// Work area: control words, result bits (3 words per near-list place), jobs.
size_t near_work_bytes(uint64_t n_cap) {
    const size_t res = ((size_t)n_cap * 24 + 255) & ~size_t(255);
    return (size_t)kNearCtlWords * 4 + res + (size_t)kRows * near_row_cap(n_cap) * sizeof(NearJob);
}

hipError_t launch_near_recompute(hipStream_t s, int eval_grid, const ImgDev* imgs, const CodeOut* outs, const NearEntry* near,
                        const uint32_t* seg_count, uint32_t seg_cap, uint32_t n_seg, const double* R,
                        const unsigned long long* S, double n_tot, void* work, unsigned long long* counter) {
    if (n_seg == 0) return hipSuccess;
    const uint64_t n_cap = (uint64_t)n_seg * seg_cap;
    const uint32_t cap_r = near_row_cap(n_cap);
    uint32_t* ctl = static_cast<uint32_t*>(work);
    unsigned long long* res = reinterpret_cast<unsigned long long*>(ctl + kNearCtlWords);
    NearJob* jobs = reinterpret_cast<NearJob*>(reinterpret_cast<uint8_t*>(res) +
                                               (((size_t)n_cap * 24 + 255) & ~size_t(255)));
    const unsigned blocks = (n_seg + kSortSegs - 1) / kSortSegs;
    const unsigned ablocks = (n_seg + kApplySegs - 1) / kApplySegs;
    CH_LAUNCH(near_sort_kernel, dim3(blocks), dim3(256), 0, s, imgs, near, seg_count, seg_cap, n_seg, res, ctl, jobs,
              cap_r, counter);
    CH_LAUNCH(near_eval_kernel, dim3(eval_grid), dim3(256), 0, s, jobs, cap_r, ctl, R, S, n_tot, res, imgs, near,
              seg_count, seg_cap, n_seg);
    CH_LAUNCH(near_apply_kernel, dim3(ablocks), dim3(256), 0, s, outs, near, seg_count, seg_cap, n_seg, res);
    return hipSuccess;
}

hipError_t launch_bucket(hipStream_t s, bool epi, const ImgDev* imgs, const TableOut* touts, const int32_t* train_list,
                         int n_train) {
    if (n_train <= 0) return hipSuccess;
    if (epi)
        CH_LAUNCH(bucket_kernel<true>, dim3(n_train * kTables), dim3(64 * kBucketWaves), 0, s, imgs, touts, train_list);
    else
        CH_LAUNCH(bucket_kernel<false>, dim3(n_train * kTables), dim3(64 * kBucketWaves), 0, s, imgs, touts,
                  train_list);
    return hipSuccess;
}

}  // namespace cashash
