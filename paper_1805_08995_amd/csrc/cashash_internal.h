// Device-side data layouts shared by the host runtime and the kernels of the
// CasHash matcher (gfx950).  Nothing here is part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cashash {

constexpr int kDim = 128;          // SIFT dimension d
constexpr int kTables = 6;         // lookup tables (Step 1)
constexpr int kKeyBits = 8;        // m bits per lookup key
constexpr int kCodeBits = 128;     // n bits of the remapping code (Step 2)
constexpr int kRows = kCodeBits + kTables * kKeyBits;  // 176 projection rows
constexpr int kRowTiles = kRows / 16;                   // 11 MFMA row tiles
constexpr int kOffStride = 257;    // bucket offsets per table (256 keys + end)
constexpr int kMaxK = 64;
constexpr int kListCap = 512;      // per-wave LDS candidate list (u32 keys); reused for tile distances
constexpr int kSelCap = 384;       // per-wave LDS list of a query tile's kept candidates
// The band kernel's shorter lists: more than kRegCap = 256 band survivors
// take its fallback path, and its tiles keep at most 320 candidates (32
// queries at k = 10, fewer queries for larger k).  Less LDS per block, so that
// seven blocks fit a compute unit.
constexpr int kListCapEpi = 320;
constexpr int kSelCapEpi = 320;
// A query's candidate keys are held in NS 64-wide register slots (NS = 4, 6
// or 8, a template parameter of the matcher); queries with more candidates
// use the LDS list.  Plain-form pairs run 4 slots up to kLargeTrain train
// points, 6 up to kHugeTrain and 8 above (fewer slots: fewer registers, more
// resident waves).  The band (epipolar) form always runs 4 slots: only the
// survivors of its band pass fill them.
constexpr int kLargeTrain = 9000;
constexpr int kHugeTrain = 14000;  // plain form: above it, 8 slots; above kLargeTrain, 6
constexpr int kWavesPerBlock = 4;  // matcher block = 4 waves
constexpr int kMaxTile = 32;       // queries per matcher work item (one per lane of the tile setup)
constexpr int kBucketWaves = 8;    // wavefronts per (train image, table) counting sort
constexpr int kProjTB = 4;         // 16-descriptor tiles per projection wavefront group (one fragment load each)

// Per-image view.  desc/codes/keys/kp are the caller's (or staged) buffers;
// off/ent are the bucket tables the library builds for train images.
struct ImgDev {
    const uint8_t* desc;   // [n][128]
    const uint64_t* codes; // [n][2]
    const uint8_t* keys;   // [n][6]
    const float* kp;       // [n][2] or null
    const uint32_t* off;   // [6][257] bucket start offsets, or null
    const uint8_t* ent;    // [6][n] bucket-ordered entries, or null
    int32_t n;
    int32_t pad;
};

// Writable per-image outputs of the code builder.
struct CodeOut {
    uint64_t* codes;   // [n][2]
    uint8_t* keys;     // [n][6]
    int64_t pad;
};

// A descriptor with at least one projection inside the rounding margin: its
// image, row and 176-bit mask of the rows to recompute in binary64.
struct NearEntry {
    int32_t img;
    int32_t row;
    uint64_t mask[3];
};

// Writable bucket tables of one train image.
struct TableOut {
    uint32_t* off;     // [6][257]
    uint8_t* ent;      // bucket-ordered entries, ent_bytes(n, epi)
};

// Bucket-ordered entries of a train image, struct of arrays over the six
// tables: for table t and position s (entries of one bucket contiguous, in
// ascending index order)
//   code[t][s] : the point's 128-bit code (16 B)
//   kid[t][s]  : its six keys in bytes 0..5 and its index in bits 48..63
//   kp[t][s]   : its keypoint (epipolar form only)
// laid out one after another from TableOut::ent / ImgDev::ent.
inline __host__ __device__ size_t ent_bytes(int n, bool epi) { return (size_t)kTables * n * (epi ? 32 : 24); }

struct PairDev {
    int32_t qi, ti;     // query image, train image
    int64_t out;        // first output slot of this pair
    double F[9];        // row-major fundamental matrix (epipolar form)
};

struct Item {           // a tile of consecutive queries of one pair (nq <= kMaxTile, nq * k <= kSelCap or kSelCapEpi)
    int32_t pair;
    int32_t q0;
    int32_t nq;
    int32_t pad;
};

struct PairTiles {      // pair `pair`'s query tiles are items [first, first + count)
    int32_t pair;
    int32_t first;
};

struct RowChunk {       // rows [r0, r0 + nr) of image img
    int32_t img;
    int32_t r0;
    int32_t nr;
    int32_t pad;
};

constexpr int kSegments = 8;       // one work segment per XCD
constexpr int kCounterStride = 64; // u32 elements between work counters (one 256-byte line each)

struct MatchParams {
    int32_t k;
    int32_t tau;
    int64_t num2;       // ratio_num^2
    int64_t den2;       // ratio_den^2
    double max_px;
    // persistent scheduling: items [seg[x], seg[x+1]) are segment x, handed
    // out `grab` at a time from counter x; a wave starts on its own XCD's
    // segment and moves to the others when it is exhausted
    int32_t seg[kSegments + 1];
    int32_t grab;
};

struct ProjParams {
    float margin_coef;
    int32_t n_tiles;
    double n_tot;       // descriptor count of the set, as binary64
};

// Bf16 hi/lo fragments of the 176 projection rows, pre-arranged so that lane
// l of a wave loads its 8 values for (part, row tile, k step) as one 16-byte
// vector: frag[part][rt][ks][l][i] = part(R[16 rt + l % 16][32 ks + 8 (l / 16) + i]).
constexpr int kFragBytes = 2 * kRowTiles * 4 * 64 * 16;

// ---- geometry-aware first stage (Sec. 3.1) ---------------------------------

// Top-scale selection of one image: rows_out[0..m) receives the m largest
// scales' indices in ascending index order.
struct SelectImg {
    const float* scale;  // [n]
    int32_t* rows_out;   // [m]
    int32_t n, m;
};

// Row gather of one image: out row j = in row rows[j]; a null output pointer
// skips that field.
struct GatherImg {
    const uint8_t* desc;    // [n][128]
    const uint64_t* codes;  // [n][2]
    const uint8_t* keys;    // [n][6]
    const float* kp;        // [n][2]
    const int32_t* rows;    // [m]
    uint8_t* o_desc;
    uint64_t* o_codes;
    uint8_t* o_keys;
    float* o_kp;
    int32_t n, m;
};

// Keypoints of an image the stage-1 matches index.
struct GeoImg {
    const float* kp;  // [n][2]
    int32_t n;
    int32_t pad;
};

struct GeoPair {
    int32_t qi, ti;
    int64_t out;      // first stage-1 output slot of the pair (n of qi slots)
};

struct GeoParams {
    int32_t n_hyp;        // hypotheses (rows of the 8-draw table)
    int32_t min_matches;  // fewer stage-1 matches: not estimated
    double thr;           // inlier distance to the epipolar line, px
    int32_t cap;          // matches held in LDS per pair (>= every pair's query count)
    int32_t pad;
};

struct GeoOut {
    double* F;            // [P][9]
    int32_t* n_matches;   // [P]
    int32_t* n_inliers;   // [P]
    int32_t* best_h;      // [P]
    int32_t* status;      // [P]
};

constexpr int kGeoMaxMatches = 8192;  // LDS list of one pair's stage-1 matches (16 B each)
constexpr int kJacobiSweeps3 = 6;
constexpr int kJacobiSweeps9 = 10;

}  // namespace cashash
