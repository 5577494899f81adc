// The encode launch sequence shared by the eager calls, recorded plans and
// the allocation-free entry point (host only).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fe.h"
#include "fe_internal.h"

namespace fe {

// Geometry of one encode call over a list of images.
struct EncodeGeom {
  bool ext = false;       // tree down to 2 x 2: EXT form, then the 2 x 2 level
  int L = 0;              // fused levels
  int bmax = 0;
  TileShape shape{0, 0};
  int cells = 0;          // record cells per top tile
  uint64_t tiles = 0;     // top tiles of all images
  uint32_t wgs = 0;       // workgroup blocks
  size_t chunks = 0;      // ordering chunks of kChunkTiles tiles
  uint64_t slots = 0;     // 16-byte record slots
  uint64_t fine_max = 0;  // 2 x 2 level: entries of the 4 x 4 range list
};

// Device buffers of one encode call (sizes from EncodeGeom).
struct EncodeBufs {
  const ImgDev* table;   // image table: n ImgDev, their wg_first words, chunk images
  BlockDesc* blocks;     // wgs
  uint4* staging;        // slots
  uint64_t* masks;       // tiles
  uint32_t* chunk_sum;   // chunks
  uint64_t* chunk_base;  // chunks + 1
  uint4* fine_list;      // fine_max (ext)
  uint32_t* fine_count;  // 1 (ext)
};

// Tile shape, sizes and table entries (table[0, n_imgs)) of an encode of
// imgs (validated by the caller).  Allocates nothing.
fe_status encode_geometry(fe_ctx* ctx, const fe_image_desc* imgs, uint32_t n_imgs, const fe_params* p,
                          ImgDev* table, EncodeGeom& g);

// [block prep], [4 x 4 count cleared], fused encode, [2 x 2 level], ordering
// into d_out / offsets, all on stream s.  ctx (may be NULL) times the
// launches while its timing is on.
fe_status encode_launch(fe_ctx* ctx, const EncodeGeom& g, const EncodeBufs& b, uint32_t n_imgs, const fe_params* p,
                        bool prep, fe_transform* d_out, size_t cap, uint64_t* offsets, hipStream_t s);

// Wait for s and read the stream length offsets[n_imgs] into *n_out;
// FE_ERR_CAPACITY when it exceeds cap.
fe_status read_count(fe_ctx* ctx, const uint64_t* offsets, uint32_t n_imgs, size_t cap, size_t* n_out,
                     hipStream_t s);

int ctx_device(const fe_ctx* ctx);

// The allocation-free encode's static scratch of the current device: its
// address (taken with hipGetSymbolAddress once per device, at context
// creation) and size.
fe_status static_scratch_init(int device);
fe_status static_scratch(int device, uint8_t** ptr, size_t* bytes);

// Write the single-image table entry `v` to dst (a kernel, so that the call
// copies nothing from the host).
hipError_t launch_table_fill(const ImgDev& v, ImgDev* dst, hipStream_t s);

}  // namespace fe
