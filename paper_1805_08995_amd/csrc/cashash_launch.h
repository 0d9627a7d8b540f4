// Host-side launchers of the device kernels (defined in cashash_kernels.hip).
#pragma once
#include "cashash_internal.h"

namespace cashash {
hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, int64_t n, unsigned long long v);
hipError_t launch_fill_u32(hipStream_t s, uint32_t* p, int64_t n, uint32_t v);
hipError_t launch_make_items(hipStream_t s, const PairTiles* pt, int32_t n_pt, const PairDev* pairs,
                             const ImgDev* imgs, int32_t qt, Item* items, int32_t n_items);
hipError_t launch_colsum(hipStream_t s, const ImgDev* imgs, const RowChunk* chunks, int n_chunks,
                         unsigned long long* S);
hipError_t launch_bias(hipStream_t s, const double* R, const unsigned long long* S, double n_tot, float* bias);
// Projection: wavefront w appends its near-margin descriptors to
// near[w * seg_cap ..] and writes their number to seg_count[w] (the fp32 form
// has one 64-entry segment per wavefront of its grid).  near_work: the work
// area of the recompute that follows (the projection clears its control
// words).
hipError_t launch_proj_mfma(hipStream_t s, int grid, const ImgDev* imgs, const CodeOut* outs, const RowChunk* tiles,
                            int n_tiles, const uint4* frag, const float* bias, float margin, NearEntry* near,
                            uint32_t* seg_count, uint32_t seg_cap, void* near_work);
hipError_t launch_proj_fp32(hipStream_t s, const ImgDev* imgs, const CodeOut* outs, const RowChunk* tiles,
                            int n_tiles, const float* R32, const float* bias, float margin, NearEntry* near,
                            uint32_t* seg_count, void* near_work);
// Binary64 recompute of the near list's flagged projections (three launches).
// work: near_work_bytes(n_seg * seg_cap) bytes of device scratch, the one
// given to the projection launch just before.
uint32_t near_row_cap(uint64_t n_cap);
size_t near_work_bytes(uint64_t n_cap);
hipError_t launch_near_recompute(hipStream_t s, int eval_grid, const ImgDev* imgs, const CodeOut* outs, const NearEntry* near,
                        const uint32_t* seg_count, uint32_t seg_cap, uint32_t n_seg, const double* R,
                        const unsigned long long* S, double n_tot, void* work, unsigned long long* counter);
hipError_t launch_bucket(hipStream_t s, bool epi, const ImgDev* imgs, const TableOut* touts,
                         const int32_t* train_list, int n_train);
hipError_t launch_match(hipStream_t s, bool epi, int ns, int grid, const ImgDev* imgs, const PairDev* pairs, const Item* items,
                        int32_t n_items, uint32_t* counter, const MatchParams& prm, int32_t* o_idx, int32_t* o_d1,
                        int32_t* o_d2, unsigned long long* stats);
}  // namespace cashash

// Geometry-aware first stage (defined in cashash_geometry.hip).
namespace cashash {
hipError_t launch_top_scale(hipStream_t s, const SelectImg* imgs, int n_images);
hipError_t launch_gather_rows(hipStream_t s, const GatherImg* imgs, const RowChunk* chunks, int n_chunks,
                              unsigned* err);
size_t fundamental_lds_bytes(int cap);
hipError_t launch_fundamental(hipStream_t s, const GeoImg* imgs, const GeoPair* pairs, int64_t n_pairs,
                              const int32_t* match_idx, const uint32_t* rnd, const GeoParams& prm, const GeoOut& out,
                              unsigned* err);
}  // namespace cashash
