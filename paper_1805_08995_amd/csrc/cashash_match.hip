// The CasHash matcher for gfx950 (MI355X): "Review of Cascade Hashing",
// Steps 1-4, "Improved Parallel Hashing Ranking" and Eq. 1-2.
//
// One wavefront per tile of up to 32 consecutive queries of one pair.  Train
// images are pre-sorted into per-table buckets whose entries carry code, keys
// and index, so a query's candidates are six contiguous runs read 64 at a
// time.  The paper's per-query index table (a histogram over Hamming
// distance) is built in LDS and scanned with DPP to find the Hamming distance
// of the k-th candidate; ties there are broken by index.  The tile's kept
// candidates are measured together with v_dot4_u32_u8 (exact), then the
// ratio test runs one lane per query.  All pairs run in one persistent launch
// with per-XCD work segments.
#include "cashash_device.h"

namespace cashash {

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

// x as seen through a DPP pattern; lanes with no source receive ~0u.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_hi(uint32_t x) {
    return __builtin_amdgcn_update_dpp(~0u, x, CTRL, ROW_MASK, 0xf, false);
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Minimum over the 64 lanes (the same prefix pattern as wave_scan_dpp; lane
// 63 ends with the minimum of all).
__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
    x = min(x, dpp_hi<0x111, 0xf>(x));
    x = min(x, dpp_hi<0x112, 0xf>(x));
    x = min(x, dpp_hi<0x114, 0xf>(x));
    x = min(x, dpp_hi<0x118, 0xf>(x));
    x = min(x, dpp_hi<0x142, 0xa>(x));
    x = min(x, dpp_hi<0x143, 0xc>(x));
    return readlane(x, 63);
}
__device__ __forceinline__ uint32_t readfirstlane_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    return (uint64_t)readlane((uint32_t)v, l) | ((uint64_t)readlane((uint32_t)(v >> 32), l) << 32);
}
__device__ __forceinline__ double readlane_f64(double v, int l) { return __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(v), l)); }

// Smallest bin d of the 256-bin LDS index table whose cumulative count
// reaches `need` (1 <= need <= total); *below = count in bins < d, *in_bin =
// count in bin d.  Lane l holds bins 4l .. 4l+3.  READOUT (the plain
// kernels): after the scan only the lane that crosses `need` is read out
// (readlane) and the bin inside it is picked with scalar arithmetic; else
// every lane picks its candidate bin and the crossing lane's is read (the
// band kernels, which rarely rank and schedule better with this form).
template <bool READOUT>
__device__ __forceinline__ uint32_t hist_select(const uint32_t* hist, uint32_t need, int lane, uint32_t* below,
                                                uint32_t* in_bin) {
    const uint4 h = reinterpret_cast<const uint4*>(hist)[lane];
    if constexpr (READOUT) {
        const uint32_t s3 = h.x + h.y + h.z + h.w;
        const uint32_t incl = wave_scan_dpp(s3);
        const uint64_t m = __ballot(incl >= need);
        const int L = __ffsll((unsigned long long)m) - 1;
        uint32_t b = readlane(incl - s3, L);
        const uint32_t c0 = readlane(h.x, L), c1 = readlane(h.y, L), c2 = readlane(h.z, L), c3 = readlane(h.w, L);
        uint32_t d = 4u * (uint32_t)L, c = c0;
        if (b + c0 < need) {
            b += c0;
            ++d;
            c = c1;
            if (b + c1 < need) {
                b += c1;
                ++d;
                c = c2;
                if (b + c2 < need) {
                    b += c2;
                    ++d;
                    c = c3;
                }
            }
        }
        *below = b;
        *in_bin = c;
        return d;
    } else {
        const uint32_t s0 = h.x, s1 = s0 + h.y, s2 = s1 + h.z, s3 = s2 + h.w;
        const uint32_t incl = wave_scan_dpp(s3);
        const uint32_t ex = incl - s3;
        const uint32_t i = (ex + s0 >= need) ? 0u : (ex + s1 >= need) ? 1u : (ex + s2 >= need) ? 2u : 3u;
        const uint32_t bl = ex + (i == 0 ? 0u : i == 1 ? s0 : i == 2 ? s1 : s2);
        const uint64_t m = __ballot(incl >= need);
        const int L = __ffsll((unsigned long long)m) - 1;
        *below = readlane(bl, L);
        const uint32_t d = readlane(4u * (uint32_t)lane + i, L);
        *in_bin = readlane(hist[d], 0);
        return d;
    }
}

__device__ __forceinline__ void clear_hist(uint32_t* hist, int lane) {
    reinterpret_cast<uint4*>(hist)[lane] = make_uint4(0u, 0u, 0u, 0u);
    wave_sync();
}

// Per-query view of the six bucket runs concatenated in table order, plus the
// query's code and keys and its epipolar line.  Passed by value so every
// field stays in registers.  Two layouts of the run table qtab (LDS, per
// query), both giving for candidate e its entry position e + C (C = t * n +
// b_t - start of its run, of table t) and 8t (the shift that masks the keys
// of tables >= t in the union test):
//  by table (most kernels): P1..P5 are the run starts of tables 1..5 and P6
//    the number of bucket entries; the number of starts at or below e is its
//    table t, and qtab[t] = C.
//  by ordinal (the 4- and 6-slot plain kernels): P1..P5 are the starts of the
//    non-empty runs after the first non-empty one (~0u for the other runs),
//    whose count at or below e is the ordinal o of e's run among the
//    non-empty runs, and qtab[o] = (16 C << 6) | 8t.  qtab[8 + 2u .. 9 + 2u]
//    holds the 64-bit mask of those starts inside chunk u (bit j: a start at
//    candidate 64u + j + 1), so a lane finds its ordinal with mbcnt, and
//    bits 3(u-1) .. 3u-1 of qtab[6] count the starts at or below 64u.
// In both, the query's key bytes 0-3 sit in qtab[7] and bytes 4-5 in bits
// 16-31 of qtab[6].
struct QueryRuns {
    uint64_t qc0, qc1, qk;
    uint32_t P1, P2, P3, P4, P5, P6;
    const uint32_t* qtab;
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
// Entry position of candidate e of the concatenated runs; cw receives 8t in
// its low 6 bits.  Lanes past the runs get candidate 0's position (a valid
// address).
template <bool ORD>
__device__ __forceinline__ uint32_t entry_pos(uint32_t e, const QueryRuns& r, uint32_t& cw) {
    const uint32_t ec = e < r.P6 ? e : 0u;
    const uint32_t o = (uint32_t)(ec >= r.P1) + (ec >= r.P2) + (ec >= r.P3) + (ec >= r.P4) + (ec >= r.P5);
    if constexpr (ORD) {
        cw = r.qtab[o];
        return ec + (cw >> 10);
    } else {
        cw = 8u * o;
        return ec + r.qtab[o];
    }
}

// Eq. 1-2: the candidate's keypoint lies within the band around the
// query's epipolar line.
__device__ __forceinline__ bool band_ok(float2 p, const QueryRuns& r, double dd) {
    const double xp = (double)p.x, yp = (double)p.y;
    const double ev = (r.la * xp + r.lb * yp) + r.lc;
    return ev * ev <= dd * (r.la * r.la + r.lb * r.lb);
}
__device__ __forceinline__ bool in_band(const TrainView& tv, uint32_t pos, const QueryRuns& r, double dd) {
    return band_ok(gload(tv.kp + pos), r, dd);
}

// popcount(x) + acc as one v_bcnt_u32_b32 (a dependent chain keeps the
// compiler from splitting a 128-bit count into two halves and an add).
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// Loaded entry (code c, keys and index kid) of a run of table t -> packed
// key (Hamming << 16 | index), or ~0u if it repeats an earlier table's
// candidate or exceeds tau.  The low 6 bits of cw hold 8t.  `live` masks
// lanes with no candidate; n_union counts candidates that survive the union.
// CHAIN selects hand-picked instructions for the union test and a chained
// count (the plain kernels); the band kernels, where few entries get here,
// keep the compiler's own, which schedules better there.  FILT = false
// (tau = 128, no filter): no tau test and no union count here (the caller
// counts the union from the valid keys).
template <bool CHAIN, bool FILT>
__device__ __forceinline__ uint32_t loaded_key(ulonglong2 c, uint64_t kid, uint32_t cw, bool live,
                                               const QueryRuns& r, int32_t tau, uint32_t& n_union) {
    // union: drop the candidate if it shares an earlier table's key with the
    // query (it was already collected there): a zero byte among bytes
    // 0 .. t-1 of keys ^ query keys.  Bytes t.. are forced to 0xFF with
    // fm = ~0 << 8t, then the exact zero-byte test (v - 0x01..) & ~v & 0x80..
    // runs on bytes 0-3 and on byte 4 (table 4's key, only below t = 5).
    const uint64_t fm = ~0ull << (cw & 63u);
    bool dup;
    if constexpr (CHAIN) {
        // bitop3 truth tables: 0xBE = (a ^ b) | c, 0x20 = a & ~b & c
        const uint32_t y = __builtin_amdgcn_bitop3_b32((uint32_t)kid, (uint32_t)r.qk, (uint32_t)fm, 0xBE);
        const uint32_t y4 =
            __builtin_amdgcn_bitop3_b32((uint32_t)(kid >> 32), (uint32_t)(r.qk >> 32), (uint32_t)(fm >> 32), 0xBE);
        const uint32_t zl = __builtin_amdgcn_bitop3_b32(y - 0x01010101u, y, 0x80808080u, 0x20);
        const uint32_t zh = __builtin_amdgcn_bitop3_b32(y4 - 1u, y4, 0x80u, 0x20);
        dup = (zl | zh) != 0u;
    } else {
        const uint32_t y = ((uint32_t)kid ^ (uint32_t)r.qk) | (uint32_t)fm;
        const uint32_t y4 = ((uint32_t)(kid >> 32) ^ (uint32_t)(r.qk >> 32)) | (uint32_t)(fm >> 32);
        dup = (((y - 0x01010101u) & ~y) | ((y4 - 0x01010101u) & ~y4 & 0xFFu)) & 0x80808080u;
    }
    bool ok = live && !dup;
    if constexpr (FILT) n_union += ok ? 1u : 0u;
    uint32_t h;
    if constexpr (CHAIN) {
        h = (uint32_t)__popc((uint32_t)c.x ^ (uint32_t)r.qc0);
        h = bcnt_acc((uint32_t)(c.x >> 32) ^ (uint32_t)(r.qc0 >> 32), h);
        h = bcnt_acc((uint32_t)c.y ^ (uint32_t)r.qc1, h);
        h = bcnt_acc((uint32_t)(c.y >> 32) ^ (uint32_t)(r.qc1 >> 32), h);
    } else {
        h = (uint32_t)(__popcll(c.x ^ r.qc0) + __popcll(c.y ^ r.qc1));
    }
    if constexpr (FILT) ok = ok && (int32_t)h <= tau;
    return ok ? ((h << 16) | (uint32_t)(kid >> 48)) : ~0u;
}

// The same for the entry at pos, loaded here.
template <bool CHAIN, bool FILT>
__device__ __forceinline__ uint32_t entry_key(const TrainView& tv, uint32_t cw, uint32_t pos, bool live,
                                              const QueryRuns& r, int32_t tau, uint32_t& n_union) {
    return loaded_key<CHAIN, FILT>(gload(tv.code + pos), gload(tv.kid + pos), cw, live, r, tau, n_union);
}

// Candidate e of the concatenated six bucket runs -> packed key, or ~0u if e
// is past the runs, outside the epipolar band, a repeat or above tau.
template <bool EPI, bool ORD, bool FILT>
__device__ __forceinline__ uint32_t key_at(uint32_t e, const TrainView& tv, const QueryRuns& r, int32_t tau,
                                           double dd, uint32_t& n_union) {
    uint32_t cw;
    const uint32_t pos = entry_pos<ORD>(e, r, cw);
    bool live = e < r.P6;
    if constexpr (EPI) live = live && in_band(tv, pos, r, dd);
    return entry_key<!EPI, FILT>(tv, cw, pos, live, r, tau, n_union);
}

// The first C chunks of 64 candidates into register slots, all loads issued
// together (slots >= C keep ~0u).
template <bool EPI, bool FILT, int C, int NS>
__device__ __forceinline__ void gather_chunks(uint32_t (&kr)[NS], int lane, const TrainView& tv, const QueryRuns& r,
                                              int32_t tau, double dd, uint32_t& n_union) {
#pragma unroll
    for (int u = 0; u < C; ++u) kr[u] = key_at<EPI, false, FILT>(64u * u + (uint32_t)lane, tv, r, tau, dd, n_union);
}

// The same for the plain form when the runs fit 256 candidates: the run
// ordinal of chunk u's lanes comes from the chunk's start mask with mbcnt
// (o0 = starts at or below 64u, carried from chunk to chunk), and only the
// last chunk can hold lanes past the runs.  Positions of all C chunks are
// found first so that their loads are in flight together.
template <bool FILT, int C, int NS>
__device__ __forceinline__ void gather_chunks_mask(uint32_t (&kr)[NS], int lane, const TrainView& tv,
                                                   const QueryRuns& r, int32_t tau, uint32_t& n_union) {
    uint32_t cw[C], boff[C];  // run word; byte offset of the entry's code (16 bytes per entry)
    const uint32_t pre = C > 1 ? readfirstlane_u32(r.qtab[6]) : 0u;  // uniform: o0 below is scalar work
#pragma unroll
    for (int u = 0; u < C; ++u) {
        const uint2 sm = *reinterpret_cast<const uint2*>(r.qtab + 8 + 2 * u);
        const uint32_t o0 = u == 0 ? 0u : (pre >> (3 * (u - 1))) & 7u;
        const uint32_t o = __builtin_amdgcn_mbcnt_hi(sm.y, __builtin_amdgcn_mbcnt_lo(sm.x, o0));
        const uint32_t e = 64u * u + (uint32_t)lane;
        const bool live = u + 1 < C || e < r.P6;
        cw[u] = r.qtab[live ? o : 0u];
        boff[u] = (cw[u] >> 6) + (live ? e << 4 : 0u);
    }
    ulonglong2 c[C];
    uint64_t kid[C];
#pragma unroll
    for (int u = 0; u < C; ++u) {
        c[u] = gload(reinterpret_cast<const ulonglong2*>(reinterpret_cast<const char*>(tv.code) + boff[u]));
        kid[u] = gload(reinterpret_cast<const uint64_t*>(reinterpret_cast<const char*>(tv.kid) + (boff[u] >> 1)));
    }
#pragma unroll
    for (int u = 0; u < C; ++u)
        kr[u] = loaded_key<true, FILT>(c[u], kid[u], cw[u], u + 1 < C || 64u * u + (uint32_t)lane < r.P6, r, tau,
                                       n_union);
}

// Resident blocks per CU each instantiation is compiled for (4 waves per
// block): the register budget that keeps 7, 6 or 5 wavefronts per SIMD.  The
// band kernel runs 7 (72 registers, a few spilled outside its band pass; its
// shorter LDS lists let 7 blocks share a CU's LDS): the extra wavefronts hide
// more of its keypoint-load latency.  The 8-slot kernels run 6 (80 registers);
// the 6-slot ones 5, as their 28.8 KB of LDS per block allows.
template <bool EPI, int NS>
constexpr int kMatchMinBlocks = NS == 4 ? (EPI ? 7 : 6) : (NS == 8 ? 6 : 5);

// One wavefront per tile of <= kMaxTile consecutive queries of one pair.
//  setup    : lane l loads query l's keys and six bucket ranges at once and
//             leaves its run table (and keys) in LDS; the run starts are
//             broadcast per query with LDS permutes.
//  Steps 1-3: per query, the six bucket runs are read in 64-wide chunks, all
//             of a query's chunks in flight together when they fit the
//             register slots (union by first-table dedupe, Hamming, tau,
//             band); the index table (histogram over Hamming distance) is
//             built in LDS and scanned to find the Hamming distance H* of
//             the k-th candidate; ties at H* are broken by index (up to 64
//             ranked directly, more by ballot counting over a binary search
//             of the index bits).
//  Step 4   : the tile's kept (query, candidate) pairs are measured together,
//             4 lanes per pair with v_dot4_u32_u8; lane l then takes query l's
//             distances, picks the nearest and second nearest and applies the
//             ratio test, and the tile's outputs are stored coalesced.
// FILT = false: the plain kernels' form for tau = 128 (no Hamming filter).
template <bool EPI, int NS, bool FILT>
__global__ __launch_bounds__(256, (kMatchMinBlocks<EPI, NS>)) void match_kernel(const ImgDev* __restrict__ imgs,
                                                    const PairDev* __restrict__ pairs,
                                                    const Item* __restrict__ items, int32_t n_items,
                                                    uint32_t* __restrict__ counter, MatchParams prm,
                                                    int32_t* __restrict__ o_idx, int32_t* __restrict__ o_d1,
                                                    int32_t* __restrict__ o_d2,
                                                    unsigned long long* __restrict__ stats) {
    __shared__ __attribute__((aligned(16))) uint32_t s_hist[kWavesPerBlock][256];
    // candidate list and tile list capacities (the band kernel's are shorter)
    constexpr int kLC = EPI ? kListCapEpi : kListCap;
    constexpr int kSC = EPI ? kSelCapEpi : kSelCap;
    __shared__ __attribute__((aligned(16))) uint32_t s_list[kWavesPerBlock][kLC];
    __shared__ __attribute__((aligned(16))) uint32_t s_sel[kWavesPerBlock][kSC];
    // run words per query, plus the chunk start masks (4- and 6-slot plain
    // kernels)
    // or the epipolar line (band kernel)
    constexpr bool kMask = (NS == 4 || NS == 6) && !EPI;
    constexpr int kQS = kMask ? 8 + 2 * NS : (EPI ? 14 : 8);
    __shared__ __attribute__((aligned(16))) uint32_t s_qtab[kWavesPerBlock][kMaxTile * kQS];
    // arguments needed only when work is grabbed or a tile is finished, kept
    // in LDS rather than in scalar registers (the kernel is short of them)
    struct Rare {
        int32_t* o_idx;
        int32_t* o_d1;
        int32_t* o_d2;
        unsigned long long* stats;
        uint32_t* counter;
        int64_t num2, den2;
        int32_t seg[kSegments + 1];
        int32_t grab;
    };
    __shared__ Rare s_rare;
    if (threadIdx.x == 0) {
        s_rare.o_idx = o_idx;
        s_rare.o_d1 = o_d1;
        s_rare.o_d2 = o_d2;
        s_rare.stats = stats;
        s_rare.counter = counter;
        s_rare.num2 = prm.num2;
        s_rare.den2 = prm.den2;
        for (int i = 0; i <= kSegments; ++i) s_rare.seg[i] = prm.seg[i];
        s_rare.grab = prm.grab;
    }
    __syncthreads();
    const bool persistent = counter != nullptr;
    const int lane = threadIdx.x & 63;
    const int wv = (int)uniform(threadIdx.x >> 6);
    uint32_t* hist = s_hist[wv];
    uint32_t* list = s_list[wv];
    uint32_t* sel = s_sel[wv];
    uint32_t* qtab = s_qtab[wv];
    const int part = lane & 3;
    uint64_t st_bucket = 0, st_ranked = 0;
    uint64_t st_valid = 0;  // no Hamming filter: the union is the valid keys, counted per query (uniform)
    uint32_t st_union = 0;
    const double dd = prm.max_px * prm.max_px;

    // XCD of this wavefront: its segment of the work list is the one whose
    // train images stay in this XCD's L2
    const uint32_t home = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kSegments - 1);
    int32_t it = (int32_t)(blockIdx.x * kWavesPerBlock + wv);
    int32_t cur = 0, end = 0;
    for (;;) {
        if (persistent) {
            if (cur >= end) {
                for (int sx = 0; sx < kSegments; ++sx) {
                    const uint32_t x = (home + (uint32_t)sx) & (kSegments - 1);
                    const int32_t s0 = s_rare.seg[x], s1 = s_rare.seg[x + 1];
                    if (s0 >= s1) continue;
                    uint32_t v = 0;
                    const int32_t grab = s_rare.grab;
                    if (lane == 0) v = atomicAdd(s_rare.counter + x * kCounterStride, (uint32_t)grab);
                    v = readlane(v, 0);
                    if ((int64_t)s0 + v < (int64_t)s1) {
                        cur = s0 + (int32_t)v;
                        end = min(cur + grab, s1);
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
        // v_P[0..4]: the run starts P1..P5 (see QueryRuns); v_P[5]: bucket entries
        uint32_t v_P[kTables];
        {
            // the previous tile's readers are done (the finalize step ended with a wave sync)
            uint32_t* qt = qtab + kQS * lane;
            const bool own = lane < kMaxTile;
            if constexpr (kMask) {
                if (own) {
#pragma unroll
                    for (int i = 0; i < NS / 2; ++i) reinterpret_cast<uint4*>(qt + 8)[i] = make_uint4(0u, 0u, 0u, 0u);
                }
            }
            uint32_t acc = 0, cnt = 0, cu[kTables];  // entries and non-empty runs before table t
            uint32_t pre = 0;                         // run starts at or below 64, 128, ... (3 bits each)
#pragma unroll
            for (int t = 0; t < kTables; ++t) {
                const uint32_t v = (uint32_t)((v_qk >> (8 * t)) & 0xFFu);
                const uint32_t b = gload(T.off + t * kOffStride + v);
                const uint32_t len = gload(T.off + t * kOffStride + v + 1) - b;
                const uint32_t start = acc;
                cu[t] = (uint32_t)t * (uint32_t)T.n + b - start;  // candidate e of run t: entry e + cu[t]
                if constexpr (kMask) {
                    if (t > 0) v_P[t - 1] = (len != 0 && cnt != 0) ? start : ~0u;
                    if (len != 0) {
                        if (own) qt[cnt] = (cu[t] << 10) | (8u * (uint32_t)t);
                        if (own && cnt != 0 && start <= 64u * NS)
                            atomicOr(qt + 8 + ((start - 1u) >> 5), 1u << ((start - 1u) & 31u));
                        if (cnt != 0) {
#pragma unroll
                            for (int bnd = 1; bnd < NS; ++bnd) pre += (uint32_t)(start <= 64u * bnd) << (3 * (bnd - 1));
                        }
                        ++cnt;
                    }
                } else if (t > 0) {
                    v_P[t - 1] = start;
                }
                acc += len;
            }
            v_P[kTables - 1] = acc;
            // the query's keys: bytes 0-3 in qt[7], bytes 4-5 in the high half of qt[6]
            const uint32_t khi = (uint32_t)(v_qk >> 32) << 16;
            if constexpr (!kMask) {
                if (own) {
                    reinterpret_cast<uint4*>(qt)[0] = make_uint4(cu[0], cu[1], cu[2], cu[3]);
                    reinterpret_cast<uint4*>(qt)[1] = make_uint4(cu[4], cu[5], khi, (uint32_t)v_qk);
                }
            } else if (own) {
                reinterpret_cast<uint2*>(qt + 6)[0] = make_uint2(pre | khi, (uint32_t)v_qk);
            }
            wave_sync();
        }
        if constexpr (EPI) {
            // the query's epipolar line F x, kept in its run table (words
            // 8-13) rather than in registers for the whole tile
            const double x = (double)gload(Q.kp + 2 * lq), y = (double)gload(Q.kp + 2 * lq + 1);
            const double la = (pr.F[0] * x + pr.F[1] * y) + pr.F[2];
            const double lb = (pr.F[3] * x + pr.F[4] * y) + pr.F[5];
            const double lc = (pr.F[6] * x + pr.F[7] * y) + pr.F[8];
            if (lane < kMaxTile) {
                double* ql = reinterpret_cast<double*>(qtab + kQS * lane + 8);
                ql[0] = la;
                ql[1] = lb;
                ql[2] = lc;
            }
            wave_sync();
        }
        uint32_t sel_n = 0;
        const uint32_t jbits = tv.n > 1 ? 32u - (uint32_t)__clz(tv.n - 1) : 0u;

        // plain kernels: the next query's code (a wave-uniform address) is
        // loaded while the current query is ranked
        uint64_t nc0 = 0, nc1 = 0;
        const ulonglong2* qcodes = reinterpret_cast<const ulonglong2*>(Q.codes);
        if constexpr (!EPI) {
            const ulonglong2 c = gload(qcodes + q0);
            nc0 = c.x;
            nc1 = c.y;
        }
        for (int qi = 0; qi < nq; ++qi) {
            QueryRuns qr;
            {
                // the query's code; its keys: from the run table, where the
                // tile setup left them
                if constexpr (EPI) {
                    const ulonglong2 c = gload(qcodes + ((int64_t)q0 + qi));
                    qr.qc0 = c.x;
                    qr.qc1 = c.y;
                } else {
                    qr.qc0 = nc0;
                    qr.qc1 = nc1;
                }
                const uint2 kw = *reinterpret_cast<const uint2*>(qtab + kQS * qi + 6);
                qr.qk = (uint64_t)kw.y | ((uint64_t)(kw.x >> 16) << 32);
            }
            // run boundaries P1..P5 only meet per-lane compares: broadcast into
            // vector registers (the kernel is short of scalar registers);
            // P6 bounds the loops and stays scalar.  The masked plain kernels
            // find runs by the chunk masks and need P1..P5 only when the runs
            // exceed their register slots: there a copy of the query's view
            // with them (runs_keyed) is made where it is read, so that no
            // register holds them across the common path.
            auto bounds = [&]() {
                qr.P1 = __shfl(v_P[0], qi); qr.P2 = __shfl(v_P[1], qi); qr.P3 = __shfl(v_P[2], qi);
                qr.P4 = __shfl(v_P[3], qi); qr.P5 = __shfl(v_P[4], qi);
            };
            auto runs_keyed = [&]() -> QueryRuns {
                if constexpr (kMask) {
                    QueryRuns q = qr;
                    q.P1 = __shfl(v_P[0], qi); q.P2 = __shfl(v_P[1], qi); q.P3 = __shfl(v_P[2], qi);
                    q.P4 = __shfl(v_P[3], qi); q.P5 = __shfl(v_P[4], qi);
                    return q;
                } else {
                    return qr;
                }
            };
            if constexpr (!kMask && !EPI) bounds();
            qr.P6 = readlane(v_P[5], qi);
            qr.qtab = qtab + kQS * qi;
            if constexpr (EPI) {
                const double* ql = reinterpret_cast<const double*>(qtab + kQS * qi + 8);
                qr.la = ql[0];
                qr.lb = ql[1];
                qr.lc = ql[2];
            } else {
                qr.la = qr.lb = qr.lc = 0.0;
            }
            const uint32_t total = qr.P6;
            st_bucket += total;

            // ---- Steps 1-3, gather: union, Hamming, tau, band; index table
            // (the histogram over Hamming distance; built during the gather,
            // except on the band path, where few candidates survive and it is
            // built only when more than k do)
            uint32_t n_valid = 0;
            constexpr uint32_t kRegCap = 64u * NS;
            uint32_t kr[NS];  // candidate keys held in registers (up to kRegCap)
#pragma unroll
            for (int u = 0; u < NS; ++u) kr[u] = ~0u;
            uint32_t n_slots = 0;  // register slots that hold candidates (the rest stay ~0u)
            // the 8-slot kernel and the band kernel (whose slots hold only
            // the band's few survivors) skip empty slots in the ranking and
            // compaction loops; the 4-slot plain kernel keeps no slot count
            // (its slots are nearly always full, and the count would take it
            // past 80 VGPRs, the limit for six wavefronts per SIMD)
            constexpr bool kSkipEmpty = NS > 4 || EPI;
            // ties needing at most this many picks are ranked by repeated
            // wave minima (plain kernels, keys in registers)
            constexpr uint32_t kMinRounds = 4u;
            bool in_regs = true;
            bool gathered = false;
            bool hist_built = true;  // false: the index table still has to be built from kr
            if (total == 0) {
                gathered = true;  // no candidate: nothing to read (the image may have no entries)
            } else if constexpr (EPI) {
                // band first: only keypoints are read for every bucket entry;
                // the ~1% inside the band are compacted (table, position) into
                // the LDS list and only they are read in full
                // The pass walks the six runs one by one, so a run's table t
                // is known and its entries are consecutive: first the leading
                // 64 entries of all six runs with their keypoint loads in
                // flight together, then the rest of any longer run.  (The
                // survivors' order differs from the concatenated order; their
                // keys are ranked by (H, index), which does not depend on it.)
                uint32_t n_surv = 0;
                uint32_t rb[kTables], rl[kTables];  // run start in the table; run length
                {
                    // uniform per query: scalar registers (readlane of the
                    // per-lane starts, the run table read once)
                    const uint32_t st[kTables + 1] = {0u, readlane(v_P[0], qi), readlane(v_P[1], qi),
                                                      readlane(v_P[2], qi), readlane(v_P[3], qi),
                                                      readlane(v_P[4], qi), qr.P6};
#pragma unroll
                    for (int t = 0; t < kTables; ++t) {
                        rl[t] = st[t + 1] - st[t];
                        rb[t] = readfirstlane_u32(qr.qtab[t]) + st[t];
                    }
                }
                // Eq. 1-2 for 64 keypoints at once: the compare's lane mask
                // itself (no branch), ANDed with the run's lanes (a vector
                // compare: cheaper here than building the mask from the run
                // length with scalar shifts).  Lanes past the run read the
                // entries after it, unclamped: at most 64 entries past the
                // keypoints of the last table, inside the 512 bytes the
                // tables of a band call keep at their end; their results are
                // masked out
                const double rhs = dd * (qr.la * qr.la + qr.lb * qr.lb);
                // keypoint of entry pos: a 32-bit byte offset from the table's
                // base (the scalar-base load form, no 64-bit address per lane)
                auto kp_at = [&](uint32_t pos) {
                    return reinterpret_cast<const float2*>(reinterpret_cast<const char*>(tv.kp) + (pos << 3));
                };
                auto band_chunk = [&](int t, uint32_t i0, float2 kp, uint32_t pos) {
                    const double xp = (double)kp.x, yp = (double)kp.y;
                    const double ev = (qr.la * xp + qr.lb * yp) + qr.lc;
                    const bool in_run = i0 + (uint32_t)lane < rl[t];
                    const bool in_band = ev * ev <= rhs;
                    const uint64_t mk = __builtin_amdgcn_ballot_w64(in_band) & __builtin_amdgcn_ballot_w64(in_run);
                    if (mk != 0) {  // wave-uniform; most chunks have no survivor
                        const uint32_t sl = n_surv + mbcnt64(mk);
                        // a lane's own survival from its compares, not from
                        // its bit of mk (no 64-bit shift and test per lane)
                        if (in_band && in_run && sl < (uint32_t)kLC)
                            list[sl] = ((8u * (uint32_t)t) << 24) | pos;
                        n_surv += (uint32_t)__popcll(mk);
                    }
                };
                {
                    uint32_t ps[kTables];
                    float2 kp[kTables];
#pragma unroll
                    for (int t = 0; t < kTables; ++t) ps[t] = rb[t] + (uint32_t)lane;
#pragma unroll
                    for (int t = 0; t < kTables; ++t) kp[t] = gload(kp_at(ps[t]));
#pragma unroll
                    for (int t = 0; t < kTables; ++t) band_chunk(t, 0u, kp[t], ps[t]);
                }
#pragma unroll
                for (int t = 0; t < kTables; ++t) {
                    const uint32_t len = readfirstlane_u32(rl[t]);
                    for (uint32_t i0 = 64; i0 < len; i0 += 64) {
                        const uint32_t pos = rb[t] + i0 + (uint32_t)lane;
                        band_chunk(t, i0, gload(kp_at(pos)), pos);
                    }
                }
                wave_sync();
                if (n_surv <= kRegCap && n_surv <= (uint32_t)kLC) {
                    const uint32_t slots = (n_surv + 63u) >> 6;
                    n_slots = slots;
#pragma unroll
                    for (int u = 0; u < NS; ++u) {
                        if ((uint32_t)u < slots) {
                            const uint32_t i = 64u * u + lane;
                            const bool live = i < n_surv;
                            const uint32_t packed = live ? list[i] : 0u;
                            kr[u] = entry_key<false, true>(tv, packed >> 24, live ? (packed & 0xFFFFFFu) : 0u, live, qr, prm.tau,
                                              st_union);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < NS; ++u)
                        if (!kSkipEmpty || (uint32_t)u < slots) n_valid += (uint32_t)__popcll(__ballot(kr[u] != ~0u));
                    gathered = true;  // the index table is built only if ranking is needed
                }
                wave_sync();
            }
            if (gathered) {
                hist_built = false;
            } else {
                if constexpr (EPI) bounds();  // the band kernel's only path that reads them
                clear_hist(hist, lane);
                if (total <= kRegCap) {
                    // common case: every bucket entry of the query fits the
                    // register slots; exactly ceil(total / 64) chunks are read
                    const uint32_t nch = (total + 63u) >> 6;
                    n_slots = nch;
                    switch (nch) {
#define GATHER_CASE(C)                                                                            \
    case C:                                                                                       \
        if constexpr (C <= NS && kMask) gather_chunks_mask<FILT, C, NS>(kr, lane, tv, qr, prm.tau, st_union); \
        else if constexpr (C <= NS) gather_chunks<EPI, FILT, C, NS>(kr, lane, tv, qr, prm.tau, dd, st_union); \
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
                            // a valid key is below 129 << 16 (the empty key is ~0u); tested
                            // this way, the compiler does not rebuild ~0u for the other lanes
                            const bool keep = kr[u] < (129u << 16);
                            n_valid += (uint32_t)__popcll(__ballot(keep));
                            if (keep) atomicAdd(&hist[kr[u] >> 16], 1u);
                        }
                    }
                } else {
                    const QueryRuns qb = runs_keyed();  // the only path that can leave in_regs false
                    for (uint32_t base = 0; base < total; base += 256) {
                        uint32_t kv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            kv[u] = key_at<EPI, kMask, FILT>(base + 64u * u + lane, tv, qb, prm.tau, dd, st_union);
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const bool keep = kv[u] != ~0u;
                            const uint64_t mk = __ballot(keep);
                            const uint32_t slot = n_valid + mbcnt64(mk);
                            if (keep) {
                                atomicAdd(&hist[kv[u] >> 16], 1u);
                                if (slot < (uint32_t)kLC) list[slot] = kv[u];
                            }
                            n_valid += (uint32_t)__popcll(mk);
                        }
                    }
                    in_regs = n_valid <= kRegCap && n_valid <= (uint32_t)kLC;
                    wave_sync();
                    if (in_regs) {
                        n_slots = (n_valid + 63u) >> 6;
#pragma unroll
                        for (int u = 0; u < NS; ++u) {
                            const uint32_t e = 64u * u + lane;
                            if (!kSkipEmpty || (uint32_t)u < n_slots) kr[u] = e < n_valid ? list[e] : ~0u;
                        }
                    }
                }
            }
            wave_sync();
            if constexpr (!EPI) {
                const ulonglong2 c = gload(qcodes + ((int64_t)q0 + min(qi + 1, nq - 1)));
                nc0 = c.x;
                nc1 = c.y;
            }
            if constexpr (!FILT) st_valid += n_valid;
            const uint32_t kk = n_valid < (uint32_t)prm.k ? n_valid : (uint32_t)prm.k;
            st_ranked += kk;
            // the query's kept count and first tile-list slot, for the ratio
            // test; word 7 of its run table (its key bytes) is only read
            // when the query starts
            if (lane == 0) qtab[kQS * qi + 7] = kk | (sel_n << 16);
            if (kk == 0) continue;
            const bool in_list = n_valid <= (uint32_t)kLC;
            const uint32_t span = in_list ? n_valid : total;
            uint32_t dummy = 0;
            // number of candidate keys in [lo, hi), counted with ballots
#define COUNT_RANGE(lo, hi, c)                                                                        \
    do {                                                                                              \
        c = 0;                                                                                        \
        if (in_regs) {                                                                                \
            _Pragma("unroll") for (int u = 0; u < NS; ++u) if (!kSkipEmpty || (uint32_t)u < n_slots) c += \
                (uint32_t)__popcll(__ballot(kr[u] >= (lo) && kr[u] < (hi)));                          \
        } else {                                                                                      \
            for (uint32_t base = 0; base < span; base += 64) {                                        \
                const uint32_t e = base + lane;                                                       \
                const uint32_t key = in_list ? (e < n_valid ? list[e] : ~0u)                          \
                                             : key_at<EPI, kMask, FILT>(e, tv, runs_keyed(), prm.tau, dd, dummy);  \
                c += (uint32_t)__popcll(__ballot(key >= (lo) && key < (hi)));                         \
            }                                                                                         \
        }                                                                                             \
    } while (0)

            uint32_t tkey;  // kept candidates: key <= tkey
            if (n_valid <= (uint32_t)prm.k) {
                tkey = 0xFFFFFFFEu;  // every valid candidate is kept; no ranking needed
            } else {
                if (!hist_built) {
                    clear_hist(hist, lane);
#pragma unroll
                    for (int u = 0; u < NS; ++u)
                        if ((!kSkipEmpty || (uint32_t)u < n_slots) && kr[u] != ~0u) atomicAdd(&hist[kr[u] >> 16], 1u);
                    wave_sync();
                }
                // ---- Step 3: Hamming distance H* of the kk-th candidate from the index table
                uint32_t below;
                uint32_t ties;  // candidates at Hamming distance H*
                const uint32_t hs = hist_select<!EPI>(hist, kk, lane, &below, &ties);
                const uint32_t need = kk - below;
                if (ties == need) {
                    tkey = ((hs + 1u) << 16) - 1u;
                } else if (!EPI && in_regs && need <= kMinRounds) {
                    // few ties needed: the need-th smallest key at or above
                    // H* << 16, by rounds of a wave minimum over the keys at
                    // or above a bound (keys below it, and the ~0u of empty
                    // slots, wrap to values above every key in range); keys
                    // are distinct, and the first `ties` keys at or above
                    // the bound are the ties, so each round finds the next
                    uint32_t bnd = hs << 16, cur = 0;
                    for (uint32_t rd = 0; rd < need; ++rd) {
                        uint32_t m = ~0u;
#pragma unroll
                        for (int u = 0; u < NS; ++u)
                            if (!kSkipEmpty || (uint32_t)u < n_slots) m = min(m, kr[u] - bnd);
                        cur = bnd + wave_min(m);
                        bnd = cur + 1u;
                    }
                    tkey = cur;
                } else if (ties <= 64) {
                    // few ties: gather their indices (the index table is no longer
                    // needed) and rank each one against the others
                    const uint32_t lo = hs << 16, hi = lo + 0x10000u;
                    uint32_t nt = 0;
                    if (in_regs) {
#pragma unroll
                        for (int u = 0; u < NS; ++u) {
                            if (kSkipEmpty && (uint32_t)u >= n_slots) break;
                            const bool tie = kr[u] >= lo && kr[u] < hi;
                            const uint64_t mk = __ballot(tie);
                            // the index table counted exactly these keys: nt < ties <= 64
                            // (the band kernels keep a guard; their code schedules better with it)
                            const uint32_t slot = nt + mbcnt64(mk);
                            if (tie && (!EPI || slot < 256u)) hist[slot] = kr[u] & 0xFFFFu;
                            nt += (uint32_t)__popcll(mk);
                        }
                    } else {
                        for (uint32_t base = 0; base < span; base += 64) {
                            const uint32_t e = base + lane;
                            const uint32_t key = in_list ? (e < n_valid ? list[e] : ~0u)
                                                         : key_at<EPI, kMask, FILT>(e, tv, runs_keyed(), prm.tau, dd, dummy);
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
            }
            // compaction of the kept candidates into the tile list
            if (in_regs) {
#pragma unroll
                for (int u = 0; u < NS; ++u) {
                    if (kSkipEmpty && (uint32_t)u >= n_slots) break;
                    // exactly kk <= k keys are kept per query and the host sizes
                    // tiles so that nq * k <= kSC: the slot is in range
                    const bool keep = kr[u] <= tkey;
                    const uint64_t mk = __ballot(keep);
                    const uint32_t slot = sel_n + mbcnt64(mk);
                    if (keep && (!EPI || slot < (uint32_t)kSC)) sel[slot] = ((uint32_t)qi << 16) | (kr[u] & 0xFFFFu);
                    sel_n += (uint32_t)__popcll(mk);
                }
            } else {
                for (uint32_t base = 0; base < span; base += 64) {
                    const uint32_t e = base + lane;
                    const uint32_t key = in_list ? (e < n_valid ? list[e] : ~0u)
                                                 : key_at<EPI, kMask, FILT>(e, tv, runs_keyed(), prm.tau, dd, dummy);
                    const bool keep = key <= tkey;
                    const uint64_t mk = __ballot(keep);
                    const uint32_t slot = sel_n + mbcnt64(mk);
                    if (keep && slot < (uint32_t)kSC) sel[slot] = ((uint32_t)qi << 16) | (key & 0xFFFFu);
                    sel_n += (uint32_t)__popcll(mk);
                }
            }
            wave_sync();
        }
#undef COUNT_RANGE
        if (sel_n > (uint32_t)kSC) sel_n = kSC;  // cannot happen when nq * k <= kSC

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
            const uint32_t kw = qtab[kQS * lane + 7];
            const uint32_t my_kk = kw & 0xFFFFu, my_off = kw >> 16;
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
                if (s_rare.den2 * (int64_t)r_d1 < s_rare.num2 * (int64_t)r_d2) r_idx = (int32_t)(uint32_t)best;
            }
            const int64_t o = pr.out + q0 + lane;
            gstore(s_rare.o_idx + o, r_idx);
            gstore(s_rare.o_d1 + o, r_d1);
            gstore(s_rare.o_d2 + o, r_d2);
        }
        wave_sync();
        if (!persistent) break;
    }
    // statistics: bucket entries and ranked counts (uniform), union sizes (per lane)
    uint64_t u64 = st_union;
    for (int d = 32; d >= 1; d >>= 1) u64 += __shfl_xor(u64, d);
    u64 += st_valid;
    if (lane == 0 && s_rare.stats) {
        atomicAdd(&s_rare.stats[0], (unsigned long long)st_bucket);
        atomicAdd(&s_rare.stats[1], (unsigned long long)u64);
        atomicAdd(&s_rare.stats[2], (unsigned long long)st_ranked);
    }
}

// ------------------------------------------------------------------ launcher
hipError_t launch_match(hipStream_t s, bool epi, int ns, int grid, const ImgDev* imgs, const PairDev* pairs,
                        const Item* items, int32_t n_items, uint32_t* counter, const MatchParams& prm, int32_t* o_idx,
                        int32_t* o_d1, int32_t* o_d2, unsigned long long* stats) {
    if (n_items <= 0 || grid <= 0) return hipSuccess;
    const dim3 g(grid), b(64 * kWavesPerBlock);
    const bool filt = prm.tau < kCodeBits;  // a Hamming filter is set
#define CH_MATCH(E, N, F) \
    CH_LAUNCH((match_kernel<E, N, F>), g, b, 0, s, imgs, pairs, items, n_items, counter, prm, o_idx, o_d1, o_d2, stats)
    if (epi)
        CH_MATCH(true, 4, true);  // the band pass keeps only its survivors in the slots
    else if (ns > 6 && filt)
        CH_MATCH(false, 8, true);
    else if (ns > 6)
        CH_MATCH(false, 8, false);
    else if (ns > 4 && filt)
        CH_MATCH(false, 6, true);
    else if (ns > 4)
        CH_MATCH(false, 6, false);
    else if (filt)
        CH_MATCH(false, 4, true);
    else
        CH_MATCH(false, 4, false);
#undef CH_MATCH
    return hipSuccess;
}

}  // namespace cashash
