// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fe.h"

namespace fe {

// One image as the device sees it (batch table entry).
struct ImgDev {
  const uint8_t* data;
  uint32_t width, height, stride;
  uint32_t tiles_x, tiles_y;    // top-level tiles per row / column
  uint32_t groups_x, groups_y;  // workgroup super-tiles per row / column
  uint32_t wg_first;            // first logical workgroup of this image
  // the 2 x 2 level's parameters for this image, read when
  // FinishArgs::per_image is set: FE_PHASE2 / FE_IDENTITY_ONLY flags and
  // the MSE threshold of the listed 4 x 4 ranges
  uint32_t fine_flags;
  uint32_t fine_thr;
  uint64_t tile_first;          // global index of this image's first tile
};
static_assert(sizeof(ImgDev) == 56, "image table entry");

// Per-workgroup encoder parameters (EncodeArgs::wg_params): the MSE
// thresholds of levels 1..L-1, then FE_PHASE2 / FE_IDENTITY_ONLY flags.
constexpr int kWgParamWords = 8;

// One workgroup's block of top tiles, expanded from the image table by the
// prep kernel so that a workgroup starts with a single 32-byte load.
struct BlockDesc {
  const uint8_t* data;  // image
  uint64_t tg0;         // global index of the block's first tile
  uint32_t stride;      // image row pitch (bytes)
  uint32_t wh;          // (width - 1) | (height - 1) << 16
  uint32_t t0;          // first tile of the block: tx0 | ty0 << 16
  uint32_t sblk;        // record-slot block (see EncodeArgs::staging)
};

// Per-call encoder constants (passed by value).
struct EncodeArgs {
  const ImgDev* imgs;
  const uint32_t* wg_first;  // per image: first logical workgroup (sorted)
  const BlockDesc* blocks;   // per logical workgroup
  uint32_t n_imgs;
  uint32_t n_wg;       // logical workgroups over all images
  uint32_t phase2;     // run Technique 1
  uint32_t identity_only;   // phase 1 fits the identity isometry only
  uint32_t thr[4];     // MSE thresholds of levels 1..L-1
  // when not NULL, kWgParamWords words per logical workgroup that replace
  // thr, phase2 and identity_only for that workgroup (callers that mix
  // parameter sets in one launch)
  const uint32_t* wg_params;
  // Record slots, one group of NT * cells per workgroup block (NT tiles),
  // cell-major inside it: the record of Morton cell c of the block's tile t
  // is at sblk * NT * cells + c * NT + t, so the one-record tiles of a block
  // (cell 0) lie side by side.
  uint4* staging;
  uint64_t* masks;     // per tile: bit c set when cell c holds a record
  // Trees that reach 2 x 2 ranges (the kernel's EXT form): the 4 x 4 level
  // is tested against thr[L-1] instead of being stored, record cells are
  // 2 x 2 units, and each failed 4 x 4 range is appended to fine_list
  // (count in *fine_count) for the 2 x 2 level: x | y << 16, the record
  // slot of its first child, its tile's global index, m | cell << 8.
  uint4* fine_list;
  uint32_t* fine_count;
};

constexpr int kChunkTiles = 256;  // tiles per scatter workgroup

// Tile shape of the encode kernel: GX x GY top tiles per workgroup.
struct TileShape {
  int gx, gy;
};

// Supported tile shapes for (b_max, levels); the first is the default.
int encode_shapes(int b_max, int levels, TileShape* out, int max_out);

// Launch the fused encode kernel for (b_max, levels, shape).  Returns
// hipErrorInvalidValue when the combination is not instantiated.
hipError_t launch_mns_tiles(int b_max, int levels, TileShape shape, const EncodeArgs& args,
                            hipStream_t stream);
// The EXT form for trees that continue to 2 x 2 (levels = the fused levels,
// b_max -> 4; default tile shape only).
hipError_t launch_mns_tiles_ext(int b_max, int levels, TileShape shape, const EncodeArgs& args,
                                hipStream_t stream);

hipError_t launch_zero_u32(uint32_t* p, size_t n, hipStream_t stream);

// Expand the image table into one BlockDesc per logical workgroup for a
// block of gx x gy tiles of side b_max.
hipError_t launch_block_prep(const ImgDev* imgs, uint32_t n_imgs, uint32_t n_wg, int b_max, int gx, int gy,
                             BlockDesc* blocks, hipStream_t stream);

// Count records per chunk of tiles, scan the chunk counts, and copy the
// records from staging into stream order; writes per-image offsets and the
// total (offsets[n_imgs]).  chunk_sum needs ceil(tiles / kChunkTiles)
// entries, chunk_base one more.
// Records are read from the block-grouped, cell-major slots written by the
// encode kernel for tile shape `shape`; an image's blocks are numbered from
// its wg_first in row-major block order.
// chunk_img[c] is the image holding tile c * kChunkTiles (NULL when there
// is one image).
hipError_t launch_scatter(const ImgDev* imgs, uint32_t n_imgs, const uint32_t* chunk_img, uint64_t total_tiles,
                          int cells, TileShape shape, const uint64_t* masks, uint32_t* chunk_sum,
                          uint64_t* chunk_base, const uint4* staging, uint4* out, uint64_t cap, uint64_t* offsets,
                          hipStream_t stream);

hipError_t launch_downsample(const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                             uint8_t* out, hipStream_t stream);

hipError_t launch_range_moments(const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                                int block, const uint32_t* xy, uint32_t count, uint32_t* mom,
                                hipStream_t stream);

// Decoder.
struct DecodeArgs {
  const uint4* recs;
  uint64_t n;
  uint32_t width, height, b_max, pad;
};
hipError_t launch_decode_check(const DecodeArgs& a, uint32_t* bad, hipStream_t stream);
// The 2 x 2 level of trees that reach 2 x 2 ranges: for each 4 x 4 range
// the fused kernel listed (EXT form), phase 2 over its four 2 x 2 children
// and, where that fails, the children's phase-1 records (the last level).
struct FinishArgs {
  const ImgDev* imgs;
  uint32_t n_imgs;
  const uint4* list;
  const uint32_t* count;
  uint32_t level;       // 1-based level of the listed 4 x 4 ranges
  uint32_t thr;         // their MSE threshold (phase 2)
  uint32_t phase2, identity_only;
  uint32_t per_image;   // take thr / phase2 / identity_only from each range's image entry
  // record slots per block: nt whole-tile slots, then cells per tile (a
  // listed range that is a whole tile stores its phase-2 record in the former)
  uint32_t nt, cells;
  uint4* staging;
  uint64_t* masks;
};
hipError_t launch_fine_finish(const FinishArgs& a, uint64_t max_entries, hipStream_t stream);

// Native check of a.recs (count into *bad) and the records zoomed by z into out.
hipError_t launch_decode_zoom(const DecodeArgs& a, uint32_t z, uint4* out, uint32_t* bad, hipStream_t stream);
hipError_t launch_decode_fill(uint8_t* dst, const uint8_t* src, uint32_t w, uint32_t h,
                              hipStream_t stream);
hipError_t launch_decode_iter(const DecodeArgs& a, const uint8_t* cur, uint8_t* nxt,
                              hipStream_t stream);
// Tile-ordered decoder: tile_start[t] = first record of top tile t (n at
// the end); bit 0 of *flag is set when the stream is not tile-ordered with
// co-centred domains (the tile kernel must not run then), bit 1 when it has
// blocks of 2 x 2 pieces (the small-piece kernel must run too).
hipError_t launch_decode_tile_setup(const DecodeArgs& a, uint32_t* tile_start, uint32_t* flag,
                                    hipStream_t stream);
// Decode plan (64 x 64-pixel blocks): per block 256 cell -> piece bytes and
// 256 piece slots of 8 bytes, built once per call from tile_start; the
// transforms of 2 x 2 pieces go to small_list (count in *small_count, which
// the caller zeroes; at most n entries).
size_t decode_plan_blocks(uint32_t w, uint32_t h);
hipError_t launch_decode_plan(const DecodeArgs& a, const uint32_t* tile_start, uint8_t* cells, uint2* pieces,
                              uint32_t* small_list, uint32_t* small_count, hipStream_t stream);
hipError_t launch_decode_tile_iter(const DecodeArgs& a, const uint8_t* cells, const uint2* pieces,
                                   const uint8_t* cur, uint8_t* nxt, hipStream_t stream);
// One iteration of the listed 2 x 2 pieces (after the plan).
hipError_t launch_decode_small(const DecodeArgs& a, const uint32_t* small_list, const uint32_t* small_count,
                               const uint8_t* cur, uint8_t* nxt, hipStream_t stream);

// Bitstream packing (Sec. 3.3, 3.4): chunk_bits / chunk_base hold
// pack_chunks(n) words (at least one), *total receives the stream length in
// bits (header included), *bad the number of transforms whose fields do not
// fit their codes; out holds cap_words 64-bit words.
size_t pack_chunks(uint64_t n);
hipError_t launch_pack(const uint4* t, uint64_t n, int L, int b_min, bool iso, uint64_t header_word,
                       uint64_t* chunk_bits, uint64_t* chunk_base, uint64_t* total, uint32_t* bad,
                       unsigned long long* out, uint64_t cap_words, hipStream_t stream);

// Exhaustive search (one image).  Plans, the 2x2 phase planes, per-level
// domain sums, the MFMA search of a list of ranges (best key per range),
// and the per-range finalisation into records / next-level ranges.
struct FsPlan {
  uint32_t B, nu, nv;      // block side; domain origins per row / column
  uint32_t pitch, prow;    // phase-plane pitch (bytes) and rows
  size_t plane_bytes;      // all four planes
  uint64_t ndom;           // nu * nv
};
constexpr uint64_t kFsMaxDomains = 1u << 20;   // domain index must fit the 64-bit best key

FsPlan fs_plan(uint32_t w, uint32_t h, uint32_t B);
size_t fs_frag_bytes(uint32_t B, uint32_t R);
hipError_t fs_planes(const FsPlan& pl, const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                     uint8_t* planes, hipStream_t s);
// Local search (Sec. 2): best surrounding step-1 domain of each listed range
// (identity only), as a best key for fs_finalize.
hipError_t ls_search(const FsPlan& pl, const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                     const uint8_t* planes, const uint32_t* sd, const double* qd, const uint32_t* xy, uint32_t R,
                     uint64_t* best, hipStream_t stream);
hipError_t fs_domain_sums(const FsPlan& pl, uint32_t w, uint32_t h, const uint8_t* planes, uint32_t* sd,
                          double* qd, hipStream_t s);
hipError_t fs_search(const FsPlan& pl, const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                     const uint8_t* planes, const uint32_t* sd, const double* qd, const uint32_t* xy, uint32_t R,
                     uint8_t* frag, uint32_t* sr, double* alpha, double* beta, uint64_t* best, hipStream_t s);
hipError_t fs_finalize(const FsPlan& pl, const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                       const uint8_t* planes, const uint32_t* xy, uint32_t R, const uint64_t* best, int level,
                       int last, uint32_t thr, uint32_t b_max, uint32_t b_min, uint4* staging, uint64_t* masks,
                       uint32_t* next_xy, uint32_t* next_count, hipStream_t s);
hipError_t fs_report(const FsPlan& pl, const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                     const uint8_t* planes, const uint32_t* xy, uint32_t R, const uint64_t* best, uint32_t* out,
                     hipStream_t s);
hipError_t fs_level1(uint32_t w, uint32_t h, uint32_t b_max, uint32_t* xy, hipStream_t s);

}  // namespace fe
