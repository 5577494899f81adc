// Host side of the C ABI: contexts, scratch management and the launch
// sequences of encode / batch encode / decode / the stand-alone steps.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fe.h"
#include "fe_common.h"
#include "fe_encode_seq.h"
#include "fe_internal.h"

struct fe_ctx {
  int device = 0;
  // pinned staging of the image table, two buffers used in turn, so that a
  // new table waits only for the copy out of the table before the last
  hipEvent_t table_ready[2] = {nullptr, nullptr};   // copy out of h_table[k] finished
  fe::ImgDev* h_table[2] = {nullptr, nullptr};
  size_t h_table_n[2] = {0, 0};
  int table_cur = 0;                  // the buffer the device table was copied from
  size_t table_slots = 0;             // size of the table on the device (0: none)
  uint64_t table_gen = 0;             // bumped whenever the device table changes
  bool blocks_valid = false;          // block descriptors built from ...
  uint64_t blocks_gen = 0;            // ... this table generation,
  int blocks_key[3] = {0, 0, 0};      // ... b_max and tile shape
  hipEvent_t blocks_ready = nullptr;  // recorded after the last block-descriptor build
  uint64_t* h_scalars = nullptr;      // pinned read-back words
  fe::ImgDev* d_table = nullptr;
  size_t d_table_n = 0;
  uint4* staging = nullptr;
  size_t staging_n = 0;
  uint64_t* masks = nullptr;
  size_t masks_n = 0;
  uint32_t* chunk_sum = nullptr;
  size_t chunk_n = 0;
  uint64_t* chunk_base = nullptr;
  size_t chunk_base_n = 0;
  fe::BlockDesc* blocks = nullptr;
  size_t blocks_n = 0;
  // exhaustive search scratch
  uint8_t* fs_planes = nullptr;
  size_t fs_planes_n = 0;
  uint32_t* fs_sd = nullptr;
  size_t fs_sd_n = 0;
  double* fs_qd = nullptr;
  size_t fs_qd_n = 0;
  uint32_t* fs_xy[2] = {nullptr, nullptr};
  size_t fs_xy_n[2] = {0, 0};
  uint8_t* fs_frag = nullptr;
  size_t fs_frag_n = 0;
  uint32_t* fs_sr = nullptr;
  size_t fs_sr_n = 0;
  double* fs_alpha = nullptr;
  size_t fs_alpha_n = 0;
  double* fs_beta = nullptr;
  size_t fs_beta_n = 0;
  uint64_t* fs_best = nullptr;
  size_t fs_best_n = 0;
  uint64_t* offsets = nullptr;
  size_t offsets_n = 0;
  uint32_t* flags = nullptr;          // small device counters
  uint8_t* tmp_img = nullptr;
  size_t tmp_n = 0;
  uint32_t* dec_tiles = nullptr;      // decoder: first record of each top tile
  size_t dec_tiles_n = 0;
  uint8_t* dec_cells = nullptr;       // decoder plan: cell -> piece per block
  size_t dec_cells_n = 0;
  uint2* dec_pieces = nullptr;        // decoder plan: pieces per block
  size_t dec_pieces_n = 0;
  uint64_t* pack_chunk = nullptr;     // bitstream: chunk sums, then chunk bases
  size_t pack_chunk_n = 0;
  uint4* zoom_recs = nullptr;         // zoom decoding: the scaled transforms
  size_t zoom_recs_n = 0;
  uint32_t* dec_small = nullptr;      // decoder: transforms of 2 x 2 pieces, then their count
  size_t dec_small_n = 0;
  uint4* fine_list = nullptr;         // b_min = 2: the 4 x 4 ranges that go on to 2 x 2
  size_t fine_list_n = 0;
  uint32_t* fine_count = nullptr;
  size_t fine_count_n = 0;
  bool last_decode_tiled = false;     // which decoder the last fe_decode ran
  int decode_mode = FE_DECODE_AUTO;
  fe::TileShape shape_override[33][5] = {};
  // kernel timing (fe_timing_enable)
  bool timing = false;
  uint32_t timing_mask = ~0u;         // slots timed while timing is on (fe_timing_select)
  static constexpr int kTimingCap = 4096;
  hipEvent_t* ev = nullptr;           // 2 * kTimingCap events
  int ev_slot[kTimingCap] = {};
  int ev_used = 0;
};

// A recorded batch encode (hipGraph) with its own scratch.
struct fe_plan {
  int device = 0;
  uint32_t n_imgs = 0;
  fe::ImgDev* d_table = nullptr;
  fe::BlockDesc* blocks = nullptr;
  uint4* staging = nullptr;
  uint64_t* masks = nullptr;
  uint32_t* chunk_sum = nullptr;
  uint64_t* chunk_base = nullptr;
  uint4* fine_list = nullptr;     // trees down to 2 x 2: the listed 4 x 4 ranges
  uint32_t* fine_count = nullptr;
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // event-record nodes around the encode and ordering kernels: they record
  // the plan's own events, or a pair of the context's timing events while
  // timing is enabled
  fe_ctx* ctx = nullptr;
  hipEvent_t own[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphNode_t tnode[4] = {nullptr, nullptr, nullptr, nullptr};
  bool timed = false;        // all four nodes found
  bool on_ctx = false;       // nodes currently point at context events
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

fe_status hip_fail(hipError_t e, const char* what) {
  return fe::fail(e == hipErrorOutOfMemory ? FE_ERR_OOM : FE_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define FE_HIP(call, what)                      \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Grow a device buffer to hold n elements (contents not kept).
template <typename T>
fe_status ensure(T*& p, size_t& cap, size_t n, const char* what) {
  if (n <= cap && p) return FE_OK;
  if (p) {
    (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  size_t want = std::max<size_t>(n, 1);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), want * sizeof(T));
  if (e != hipSuccess) {
    p = nullptr;
    return hip_fail(e, what);
  }
  cap = want;
  return FE_OK;
}

// Bracket a launch with timing events when timing is on.
struct Timed {
  fe_ctx* c;
  hipStream_t s;
  int idx = -1;
  Timed(fe_ctx* ctx, int slot, hipStream_t stream) : c(ctx), s(stream) {
    if (!c || !c->timing || !c->ev || c->ev_used >= fe_ctx::kTimingCap || !((c->timing_mask >> slot) & 1u)) return;
    idx = c->ev_used++;
    c->ev_slot[idx] = slot;
    (void)hipEventRecord(c->ev[2 * idx], s);
  }
  ~Timed() {
    if (idx >= 0) (void)hipEventRecord(c->ev[2 * idx + 1], s);
  }
};

// Calls whose tiles fill fewer default-shape workgroups than this (the
// chip's compute units) use the smallest shape instead.
constexpr uint64_t kSmallCallGroups = 256;

fe::TileShape pick_shape(fe_ctx* ctx, int b_max, int L) {
  fe::TileShape o = ctx->shape_override[b_max][L];
  if (o.gx > 0) return o;
  fe::TileShape shapes[8];
  const int k = fe::encode_shapes(b_max, L, shapes, 8);
  return k > 0 ? shapes[0] : fe::TileShape{0, 0};
}

// Host image of the device table: the n ImgDev entries, then their
// wg_first words, then one word per chunk of kChunkTiles tiles naming the
// image that holds the chunk's first tile.  Returns the size in ImgDev slots.
size_t table_words(const fe::ImgDev* src, size_t n, uint64_t tiles, std::vector<fe::ImgDev>& host) {
  const size_t chunks = (size_t)((tiles + fe::kChunkTiles - 1) / fe::kChunkTiles);
  const size_t words = n + chunks;
  const size_t slots = n + (words * sizeof(uint32_t) + sizeof(fe::ImgDev) - 1) / sizeof(fe::ImgDev);
  host.assign(slots, fe::ImgDev{});
  memcpy(host.data(), src, n * sizeof(fe::ImgDev));
  uint32_t* w = reinterpret_cast<uint32_t*>(host.data() + n);
  for (size_t k = 0; k < n; ++k) w[k] = src[k].wg_first;
  size_t k = 0;
  for (size_t c = 0; c < chunks; ++c) {
    const uint64_t t = (uint64_t)c * fe::kChunkTiles;
    while (k + 1 < n && src[k + 1].tile_first <= t) ++k;
    w[n + c] = (uint32_t)k;
  }
  return slots;
}

// Copy the table (see table_words) to the device through the pinned
// staging buffer (one copy).  A table equal to the one already on the
// device (the pinned buffer still holds it) is not copied again.
fe_status upload_table(fe_ctx* ctx, const fe::ImgDev* src, size_t n, uint64_t tiles, hipStream_t s) {
  std::vector<fe::ImgDev> host;
  const size_t slots = table_words(src, n, tiles, host);
  const int cur = ctx->table_cur;
  if (ctx->table_slots == slots && ctx->d_table && ctx->h_table[cur] &&
      memcmp(ctx->h_table[cur], host.data(), slots * sizeof(fe::ImgDev)) == 0) {
    // already on the device; order this stream after its copy
    FE_HIP(hipStreamWaitEvent(s, ctx->table_ready[cur], 0), "wait for table copy");
    return FE_OK;
  }
  // the other buffer: its copy (the table before the last) is done long ago
  const int nb = cur ^ 1;
  FE_HIP(hipEventSynchronize(ctx->table_ready[nb]), "wait for an earlier table copy");
  if (slots > ctx->h_table_n[nb]) {
    if (ctx->h_table[nb]) (void)hipHostFree(ctx->h_table[nb]);
    ctx->h_table[nb] = nullptr;
    ctx->h_table_n[nb] = 0;
    FE_HIP(hipHostMalloc(reinterpret_cast<void**>(&ctx->h_table[nb]), slots * sizeof(fe::ImgDev), hipHostMallocDefault),
           "pinned image table");
    ctx->h_table_n[nb] = slots;
  }
  ctx->table_slots = 0;   // invalid until the copy is enqueued
  ++ctx->table_gen;
  fe_status st = ensure(ctx->d_table, ctx->d_table_n, slots, "device image table");
  if (st != FE_OK) return st;
  memcpy(ctx->h_table[nb], host.data(), slots * sizeof(fe::ImgDev));
  FE_HIP(hipMemcpyAsync(ctx->d_table, ctx->h_table[nb], slots * sizeof(fe::ImgDev), hipMemcpyHostToDevice, s),
         "image table copy");
  FE_HIP(hipEventRecord(ctx->table_ready[nb], s), "table event");
  ctx->table_cur = nb;
  ctx->table_slots = slots;
  return FE_OK;
}

// Device pointers into a table built by table_words.
inline const uint32_t* table_wg_first(const fe::ImgDev* d, size_t n) {
  return reinterpret_cast<const uint32_t*>(d + n);
}
inline const uint32_t* table_chunk_img(const fe::ImgDev* d, size_t n) { return table_wg_first(d, n) + n; }

// Arguments of a batch encode (fe_encode_batch, fe_plan_create).
fe_status check_batch(const fe_image_desc* h_imgs, uint32_t n_imgs, const fe_params* p, const fe_transform* d_out,
                      const uint64_t* d_offsets) {
  if (!h_imgs || !d_out || !d_offsets || n_imgs == 0) return fe::fail(FE_ERR_INVALID, "NULL argument");
  fe_status st = fe::check_params(p);
  if (st != FE_OK) return st;
  if (p->flags & (FE_FULL_SEARCH | FE_LOCAL_SEARCH)) return fe::fail(FE_ERR_INVALID, "batch encode runs MNS only");
  if ((uintptr_t)d_out & 15) return fe::fail(FE_ERR_INVALID, "output must be 16-byte aligned");
  for (uint32_t k = 0; k < n_imgs; ++k) {
    if (!h_imgs[k].data || h_imgs[k].reserved) return fe::fail(FE_ERR_INVALID, "image %u: bad descriptor", k);
    if ((st = fe::check_shape(h_imgs[k].width, h_imgs[k].height, h_imgs[k].stride, p->b_max)) != FE_OK) return st;
    if ((uintptr_t)h_imgs[k].data & 3) return fe::fail(FE_ERR_SHAPE, "image %u must be 4-byte aligned", k);
  }
  return FE_OK;
}

// Image table of a batch for `shape`: per image its tiles, workgroup blocks,
// first workgroup and first tile.  Returns the totals.
fe_status build_table(const fe_image_desc* imgs, uint32_t n_imgs, const fe_params* p, fe::TileShape shape,
                      fe::ImgDev* table, uint64_t& tiles, uint32_t& wgs) {
  tiles = 0;
  wgs = 0;
  for (uint32_t k = 0; k < n_imgs; ++k) {
    fe::ImgDev& d = table[k];
    d = fe::ImgDev{};
    d.data = imgs[k].data;
    d.width = imgs[k].width;
    d.height = imgs[k].height;
    d.stride = imgs[k].stride;
    d.tiles_x = d.width / p->b_max;
    d.tiles_y = d.height / p->b_max;
    d.groups_x = (d.tiles_x + shape.gx - 1) / shape.gx;
    d.groups_y = (d.tiles_y + shape.gy - 1) / shape.gy;
    d.wg_first = wgs;
    d.tile_first = tiles;
    const uint64_t g = (uint64_t)d.groups_x * d.groups_y;
    if (wgs + g > 0x7fffffffull) return fe::fail(FE_ERR_SHAPE, "batch too large (workgroups)");
    wgs += (uint32_t)g;
    tiles += (uint64_t)d.tiles_x * d.tiles_y;
  }
  return FE_OK;
}

// Tile shape of an encode call with L fused levels.  The context's choice
// (or the default); but a call too small to give the default shape a
// workgroup per CU (a single 512 x 512 image, say) takes the shape with the
// fewest tiles per workgroup, unless the caller set one.  Trees down to
// 2 x 2 (ext) use the shapes their EXT form is built for: the default, or
// the smallest of 16 -> 4 (4 x 2) and 8 -> 4 (4 x 4).
fe::TileShape choose_shape(fe_ctx* ctx, const fe_image_desc* imgs, uint32_t n_imgs, const fe_params* p, int L,
                           bool ext) {
  const int bmax = (int)p->b_max;
  fe::TileShape cand[16];
  const int k = fe::encode_shapes(bmax, L, cand, 16);
  if (k <= 0) return fe::TileShape{0, 0};
  fe::TileShape shape = ext ? cand[0] : pick_shape(ctx, bmax, L);
  if (!ext && ctx->shape_override[bmax][L].gx > 0) return shape;
  uint64_t all_tiles = 0;
  for (uint32_t i = 0; i < n_imgs; ++i) all_tiles += (uint64_t)(imgs[i].width / p->b_max) * (imgs[i].height / p->b_max);
  if (all_tiles / (uint64_t)(cand[0].gx * cand[0].gy) >= kSmallCallGroups) return shape;
  shape = cand[0];
  for (int i = 1; i < k; ++i)
    if (cand[i].gx * cand[i].gy < shape.gx * shape.gy) shape = cand[i];
  if (ext && !((bmax == 16 && shape.gx == 4 && shape.gy == 2) || (bmax == 8 && shape.gx == 4 && shape.gy == 4)))
    shape = cand[0];
  return shape;
}

}  // namespace

namespace fe {

fe_status encode_geometry(fe_ctx* ctx, const fe_image_desc* imgs, uint32_t n_imgs, const fe_params* p,
                          ImgDev* table, EncodeGeom& g) {
  // b_min = 2: the fused kernel runs the tree down to 4 x 4 (its EXT form)
  // and the 2 x 2 level follows in a kernel of its own
  g.ext = p->b_min < 4;
  g.L = levels_of(p->b_max, g.ext ? 4u : p->b_min);   // fused levels
  g.bmax = (int)p->b_max;
  g.shape = choose_shape(ctx, imgs, n_imgs, p, g.L, g.ext);
  if (g.shape.gx <= 0) return fail(FE_ERR_INVALID, "no kernel for b_max=%d with %d levels", g.bmax, g.L);
  g.cells = 1 << (2 * (g.L - 1 + (g.ext ? 1 : 0)));
  fe_status st = build_table(imgs, n_imgs, p, g.shape, table, g.tiles, g.wgs);
  if (st != FE_OK) return st;
  g.chunks = (size_t)((g.tiles + kChunkTiles - 1) / kChunkTiles);
  g.slots = (uint64_t)g.wgs * (uint64_t)(g.shape.gx * g.shape.gy) * (uint64_t)(g.cells + 1);
  g.fine_max = g.ext ? g.tiles * (uint64_t)(g.bmax / 4) * (uint64_t)(g.bmax / 4) : 0;
  // the 2 x 2 level's list names each child's record slot in 32 bits
  if (g.ext && g.slots >= (1ull << 32))
    return fail(FE_ERR_SHAPE, "batch too large for 2 x 2 ranges (%llu record slots, at most 2^32)",
                (unsigned long long)g.slots);
  return FE_OK;
}

fe_status encode_launch(fe_ctx* ctx, const EncodeGeom& g, const EncodeBufs& b, uint32_t n_imgs, const fe_params* p,
                        bool prep, fe_transform* d_out, size_t cap, uint64_t* offsets, hipStream_t s) {
  if (prep) FE_HIP(launch_block_prep(b.table, n_imgs, g.wgs, g.bmax, g.shape.gx, g.shape.gy, b.blocks, s), "prep launch");
  EncodeArgs a{};
  a.imgs = b.table;
  a.wg_first = table_wg_first(b.table, n_imgs);
  a.blocks = b.blocks;
  a.n_imgs = n_imgs;
  a.n_wg = g.wgs;
  a.phase2 = (p->flags & FE_PHASE2) ? 1u : 0u;
  a.identity_only = (p->flags & FE_IDENTITY_ONLY) ? 1u : 0u;
  for (int l = 0; l < 4; ++l) a.thr[l] = l < (int)p->n_thr ? p->mse_thr[l] : 0u;
  a.staging = b.staging;
  a.masks = b.masks;
  if (g.ext) {
    a.fine_list = b.fine_list;
    a.fine_count = b.fine_count;
    FE_HIP(launch_zero_u32(b.fine_count, 1, s), "zero 4 x 4 count");   // a kernel, not a memset
  }
  {
    Timed t(ctx, FE_TIMING_ENCODE, s);
    if (!g.ext) {
      FE_HIP(launch_mns_tiles(g.bmax, g.L, g.shape, a, s), "encode kernel launch");
    } else {
      FE_HIP(launch_mns_tiles_ext(g.bmax, g.L, g.shape, a, s), "encode kernel launch");
      FinishArgs f{};
      f.imgs = b.table;
      f.n_imgs = n_imgs;
      f.list = b.fine_list;
      f.count = b.fine_count;
      f.level = (uint32_t)g.L;
      f.thr = p->mse_thr[g.L - 1];
      f.phase2 = a.phase2;
      f.identity_only = a.identity_only;
      f.nt = (uint32_t)(g.shape.gx * g.shape.gy);
      f.cells = (uint32_t)g.cells;
      f.staging = b.staging;
      f.masks = b.masks;
      FE_HIP(launch_fine_finish(f, g.fine_max, s), "2 x 2 level launch");
    }
  }
  {
    Timed t(ctx, FE_TIMING_SCATTER, s);
    FE_HIP(launch_scatter(b.table, n_imgs, n_imgs > 1 ? table_chunk_img(b.table, n_imgs) : nullptr, g.tiles, g.cells,
                          g.shape, b.masks, b.chunk_sum, b.chunk_base, b.staging, reinterpret_cast<uint4*>(d_out),
                          (uint64_t)cap, offsets, s),
           "scatter kernel launch");
  }
  return FE_OK;
}

fe_status read_count(fe_ctx* ctx, const uint64_t* offsets, uint32_t n_imgs, size_t cap, size_t* n_out,
                     hipStream_t s) {
  FE_HIP(hipMemcpyAsync(ctx->h_scalars, offsets + n_imgs, sizeof(uint64_t), hipMemcpyDeviceToHost, s),
         "count read-back");
  FE_HIP(hipStreamSynchronize(s), "encode");
  *n_out = (size_t)ctx->h_scalars[0];
  if (*n_out > cap) return fail(FE_ERR_CAPACITY, "output holds %zu transforms, %zu needed", cap, *n_out);
  return FE_OK;
}

int ctx_device(const fe_ctx* ctx) { return ctx->device; }

}  // namespace fe

namespace {

// Shared MNS encode of a list of images with common parameters.
fe_status encode_images(fe_ctx* ctx, const fe_image_desc* imgs, uint32_t n_imgs, const fe_params* p,
                        fe_transform* d_out, size_t cap, uint64_t* d_offsets, size_t* n_out, hipStream_t s) {
  std::vector<fe::ImgDev> table(n_imgs);
  fe::EncodeGeom g;
  fe_status st = fe::encode_geometry(ctx, imgs, n_imgs, p, table.data(), g);
  if (st != FE_OK) return st;
  // record slots: one group of NT * cells per workgroup block
  if ((st = ensure(ctx->staging, ctx->staging_n, (size_t)g.slots, "record staging")) != FE_OK) return st;
  if ((st = ensure(ctx->masks, ctx->masks_n, (size_t)g.tiles, "tile masks")) != FE_OK) return st;
  if ((st = ensure(ctx->chunk_sum, ctx->chunk_n, g.chunks, "chunk sums")) != FE_OK) return st;
  if ((st = ensure(ctx->chunk_base, ctx->chunk_base_n, g.chunks + 1, "chunk bases")) != FE_OK) return st;
  const size_t blocks_cap = ctx->blocks_n;
  if ((st = ensure(ctx->blocks, ctx->blocks_n, (size_t)g.wgs, "block descriptors")) != FE_OK) return st;
  if (ctx->blocks_n != blocks_cap) ctx->blocks_valid = false;   // reallocated
  uint64_t* offsets = d_offsets;
  if (!offsets) {
    if ((st = ensure(ctx->offsets, ctx->offsets_n, (size_t)n_imgs + 1, "offsets")) != FE_OK) return st;
    offsets = ctx->offsets;
  }
  if (g.ext) {
    if ((st = ensure(ctx->fine_list, ctx->fine_list_n, (size_t)g.fine_max, "4 x 4 range list")) != FE_OK) return st;
    if ((st = ensure(ctx->fine_count, ctx->fine_count_n, 1, "4 x 4 range count")) != FE_OK) return st;
  }
  if ((st = upload_table(ctx, table.data(), n_imgs, g.tiles, s)) != FE_OK) return st;

  // block descriptors: rebuilt unless they were built from this very table
  // and shape (the buffer is only written here)
  if (!ctx->blocks_valid || ctx->blocks_gen != ctx->table_gen || ctx->blocks_key[0] != g.bmax ||
      ctx->blocks_key[1] != g.shape.gx || ctx->blocks_key[2] != g.shape.gy) {
    ctx->blocks_valid = false;
    FE_HIP(fe::launch_block_prep(ctx->d_table, n_imgs, g.wgs, g.bmax, g.shape.gx, g.shape.gy, ctx->blocks, s),
           "prep launch");
    FE_HIP(hipEventRecord(ctx->blocks_ready, s), "blocks event");
    ctx->blocks_valid = true;
    ctx->blocks_gen = ctx->table_gen;
    ctx->blocks_key[0] = g.bmax;
    ctx->blocks_key[1] = g.shape.gx;
    ctx->blocks_key[2] = g.shape.gy;
  } else {
    FE_HIP(hipStreamWaitEvent(s, ctx->blocks_ready, 0), "wait for block descriptors");
  }
  const fe::EncodeBufs b{ctx->d_table, ctx->blocks, ctx->staging, ctx->masks, ctx->chunk_sum, ctx->chunk_base,
                         ctx->fine_list, ctx->fine_count};
  if ((st = fe::encode_launch(ctx, g, b, n_imgs, p, false, d_out, cap, offsets, s)) != FE_OK) return st;
  if (n_out) return fe::read_count(ctx, offsets, n_imgs, cap, n_out, s);
  return FE_OK;
}

// Scratch for the exhaustive search of up to R ranges of side B.
fe_status fs_reserve(fe_ctx* ctx, const fe::FsPlan& pl, uint32_t R) {
  fe_status st;
  if ((st = ensure(ctx->fs_sd, ctx->fs_sd_n, (size_t)pl.ndom, "domain sums")) != FE_OK) return st;
  if ((st = ensure(ctx->fs_qd, ctx->fs_qd_n, (size_t)pl.ndom, "domain Q")) != FE_OK) return st;
  if ((st = ensure(ctx->fs_frag, ctx->fs_frag_n, fe::fs_frag_bytes(pl.B, R), "A fragments")) != FE_OK) return st;
  if ((st = ensure(ctx->fs_sr, ctx->fs_sr_n, (size_t)R, "range sums")) != FE_OK) return st;
  if ((st = ensure(ctx->fs_alpha, ctx->fs_alpha_n, (size_t)R, "range alpha")) != FE_OK) return st;
  if ((st = ensure(ctx->fs_beta, ctx->fs_beta_n, (size_t)R, "range beta")) != FE_OK) return st;
  if ((st = ensure(ctx->fs_best, ctx->fs_best_n, (size_t)R, "best keys")) != FE_OK) return st;
  return FE_OK;
}

fe_status fs_check(uint32_t w, uint32_t h, uint32_t b_max, uint32_t b_min) {
  if (b_max > 16) return fe::fail(FE_ERR_INVALID, "exhaustive search supports b_max <= 16");
  const fe::FsPlan pl = fe::fs_plan(w, h, b_min);
  if (pl.ndom >= fe::kFsMaxDomains)
    return fe::fail(FE_ERR_SHAPE, "exhaustive search: %llu domain origins exceed the limit of %llu",
                    (unsigned long long)pl.ndom, (unsigned long long)fe::kFsMaxDomains);
  return FE_OK;
}

// Exhaustive-search quadtree of one image: per level, MFMA search of every
// listed range, exact finalisation, children queued on the device; the
// host reads each level's child count.
fe_status encode_full_search(fe_ctx* ctx, const uint8_t* d_img, uint32_t w, uint32_t h, uint32_t stride,
                             const fe_params* p, fe_transform* d_out, size_t cap, size_t* n_out, hipStream_t s) {
  fe_status st = fs_check(w, h, p->b_max, p->b_min);
  if (st != FE_OK) return st;
  const int L = fe::levels_of(p->b_max, p->b_min);
  const int cells = 1 << (2 * (L - 1));
  const uint64_t tiles = (uint64_t)(w / p->b_max) * (h / p->b_max);
  const size_t max_ranges = (size_t)tiles * cells;
  const fe::FsPlan pl0 = fe::fs_plan(w, h, p->b_max);
  if ((st = ensure(ctx->fs_planes, ctx->fs_planes_n, pl0.plane_bytes, "phase planes")) != FE_OK) return st;
  for (int b = 0; b < 2; ++b)
    if ((st = ensure(ctx->fs_xy[b], ctx->fs_xy_n[b], max_ranges, "range lists")) != FE_OK) return st;
  if ((st = ensure(ctx->staging, ctx->staging_n, (size_t)tiles * (cells + 1), "record staging")) != FE_OK) return st;
  if ((st = ensure(ctx->masks, ctx->masks_n, (size_t)tiles, "tile masks")) != FE_OK) return st;
  const size_t chunks = (size_t)((tiles + fe::kChunkTiles - 1) / fe::kChunkTiles);
  if ((st = ensure(ctx->chunk_sum, ctx->chunk_n, chunks, "chunk sums")) != FE_OK) return st;
  if ((st = ensure(ctx->chunk_base, ctx->chunk_base_n, chunks + 1, "chunk bases")) != FE_OK) return st;
  if ((st = ensure(ctx->offsets, ctx->offsets_n, 2, "offsets")) != FE_OK) return st;
  fe::ImgDev im{};
  im.data = d_img;
  im.width = w;
  im.height = h;
  im.stride = stride;
  im.tiles_x = w / p->b_max;
  im.tiles_y = h / p->b_max;
  im.groups_x = im.tiles_x;
  im.groups_y = im.tiles_y;
  im.wg_first = 0;
  im.tile_first = 0;
  if ((st = upload_table(ctx, &im, 1, tiles, s)) != FE_OK) return st;
  FE_HIP(fe::launch_zero_u32(reinterpret_cast<uint32_t*>(ctx->masks), (size_t)tiles * 2, s), "zero masks");
  FE_HIP(fe::fs_planes(pl0, d_img, w, h, stride, ctx->fs_planes, s), "phase planes");
  FE_HIP(fe::fs_level1(w, h, p->b_max, ctx->fs_xy[0], s), "level-1 ranges");
  uint32_t R = (uint32_t)tiles;
  for (int lev = 1; lev <= L && R > 0; ++lev) {
    const uint32_t B = p->b_max >> (lev - 1);
    const fe::FsPlan pl = fe::fs_plan(w, h, B);
    if ((st = fs_reserve(ctx, pl, R)) != FE_OK) return st;
    const uint32_t* xy = ctx->fs_xy[(lev - 1) & 1];
    uint32_t* nxt = ctx->fs_xy[lev & 1];
    FE_HIP(fe::fs_domain_sums(pl, w, h, ctx->fs_planes, ctx->fs_sd, ctx->fs_qd, s), "domain sums");
    {
      Timed t(ctx, FE_TIMING_FULLSEARCH, s);
      if (p->flags & FE_LOCAL_SEARCH)
        FE_HIP(fe::ls_search(pl, d_img, w, h, stride, ctx->fs_planes, ctx->fs_sd, ctx->fs_qd, xy, R, ctx->fs_best, s),
               "local search launch");
      else
        FE_HIP(fe::fs_search(pl, d_img, w, h, stride, ctx->fs_planes, ctx->fs_sd, ctx->fs_qd, xy, R, ctx->fs_frag,
                             ctx->fs_sr, ctx->fs_alpha, ctx->fs_beta, ctx->fs_best, s),
               "search launch");
    }
    FE_HIP(fe::launch_zero_u32(ctx->flags, 1, s), "zero count");
    const bool last = lev == L;
    FE_HIP(fe::fs_finalize(pl, d_img, w, h, stride, ctx->fs_planes, xy, R, ctx->fs_best, lev, last ? 1 : 0,
                           last ? 0u : p->mse_thr[lev - 1], p->b_max, p->b_min, ctx->staging, ctx->masks, nxt,
                           ctx->flags, s),
           "finalize launch");
    if (last) break;
    FE_HIP(hipMemcpyAsync(ctx->h_scalars, ctx->flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "count");
    FE_HIP(hipStreamSynchronize(s), "level");
    R = (uint32_t)(ctx->h_scalars[0] & 0xffffffffu);
  }
  // records sit tile-major (blocks of one tile)
  FE_HIP(fe::launch_scatter(ctx->d_table, 1, nullptr, tiles, cells, fe::TileShape{1, 1}, ctx->masks, ctx->chunk_sum,
                            ctx->chunk_base, ctx->staging,
                            reinterpret_cast<uint4*>(d_out), (uint64_t)cap, ctx->offsets, s),
         "scatter launch");
  FE_HIP(hipMemcpyAsync(ctx->h_scalars, ctx->offsets + 1, sizeof(uint64_t), hipMemcpyDeviceToHost, s), "count");
  FE_HIP(hipStreamSynchronize(s), "encode");
  *n_out = (size_t)ctx->h_scalars[0];
  if (*n_out > cap) return fe::fail(FE_ERR_CAPACITY, "output holds %zu transforms, %zu needed", cap, *n_out);
  return FE_OK;
}

}  // namespace

extern "C" {

fe_status fe_create(int device, fe_ctx** out) {
  fe::clear_error();
  if (!out) return fe::fail(FE_ERR_INVALID, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0) return fe::fail(FE_ERR_DEVICE, "no HIP device available");
  if (device < 0 || device >= count) return fe::fail(FE_ERR_DEVICE, "device %d out of range (%d)", device, count);
  hipDeviceProp_t prop;
  FE_HIP(hipGetDeviceProperties(&prop, device), "device properties");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fe::fail(FE_ERR_DEVICE, "device %d is %s, this library is built for gfx950", device, prop.gcnArchName);
  DeviceGuard g(device);
  fe_ctx* c = new fe_ctx();
  c->device = device;
  hipError_t e1 = hipEventCreateWithFlags(&c->table_ready[0], hipEventDisableTiming);
  if (e1 == hipSuccess) e1 = hipEventCreateWithFlags(&c->table_ready[1], hipEventDisableTiming);
  if (e1 == hipSuccess) e1 = hipEventCreateWithFlags(&c->blocks_ready, hipEventDisableTiming);
  hipError_t e2 = hipHostMalloc(reinterpret_cast<void**>(&c->h_scalars), 64, hipHostMallocDefault);
  hipError_t e3 = hipMalloc(reinterpret_cast<void**>(&c->flags), 64);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
    fe_destroy(c);
    return fe::fail(FE_ERR_OOM, "context allocation failed");
  }
  // the allocation-free encode's scratch: its address on this device
  if (fe_status st = fe::static_scratch_init(device); st != FE_OK) {
    fe_destroy(c);
    return st;
  }
  *out = c;
  return FE_OK;
}

void fe_destroy(fe_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  for (int k = 0; k < 2; ++k) {
    if (c->table_ready[k]) (void)hipEventDestroy(c->table_ready[k]);
    if (c->h_table[k]) (void)hipHostFree(c->h_table[k]);
  }
  if (c->blocks_ready) (void)hipEventDestroy(c->blocks_ready);
  if (c->h_scalars) (void)hipHostFree(c->h_scalars);
  (void)hipFree(c->d_table);
  (void)hipFree(c->staging);
  (void)hipFree(c->masks);
  (void)hipFree(c->chunk_sum);
  (void)hipFree(c->chunk_base);
  (void)hipFree(c->blocks);
  (void)hipFree(c->fs_planes);
  (void)hipFree(c->fs_sd);
  (void)hipFree(c->fs_qd);
  (void)hipFree(c->fs_xy[0]);
  (void)hipFree(c->fs_xy[1]);
  (void)hipFree(c->fs_frag);
  (void)hipFree(c->fs_sr);
  (void)hipFree(c->fs_alpha);
  (void)hipFree(c->fs_beta);
  (void)hipFree(c->fs_best);
  (void)hipFree(c->offsets);
  (void)hipFree(c->flags);
  (void)hipFree(c->tmp_img);
  (void)hipFree(c->dec_tiles);
  (void)hipFree(c->dec_cells);
  (void)hipFree(c->dec_pieces);
  (void)hipFree(c->pack_chunk);
  (void)hipFree(c->zoom_recs);
  (void)hipFree(c->fine_list);
  (void)hipFree(c->dec_small);
  (void)hipFree(c->fine_count);
  if (c->ev) {
    for (int i = 0; i < 2 * fe_ctx::kTimingCap; ++i)
      if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    delete[] c->ev;
  }
  delete c;
}

fe_status fe_downsample(fe_ctx* ctx, const uint8_t* d_img, uint32_t w, uint32_t h, uint32_t stride,
                        uint8_t* d_out, void* stream) {
  fe::clear_error();
  if (!ctx || !d_img || !d_out) return fe::fail(FE_ERR_INVALID, "NULL argument");
  if (w < 2 || h < 2 || (w & 1) || (h & 1)) return fe::fail(FE_ERR_SHAPE, "sides must be even and >= 2");
  if (stride < w || stride % 4 || ((uintptr_t)d_img & 3))
    return fe::fail(FE_ERR_SHAPE, "stride must be >= width, a multiple of 4, and the image 4-byte aligned");
  DeviceGuard g(ctx->device);
  FE_HIP(fe::launch_downsample(d_img, w, h, stride, d_out, (hipStream_t)stream), "downsample launch");
  return FE_OK;
}

fe_status fe_range_moments(fe_ctx* ctx, const uint8_t* d_img, uint32_t w, uint32_t h, uint32_t stride,
                           uint32_t block, const uint32_t* d_xy, uint32_t count, uint32_t* d_moments,
                           void* stream) {
  fe::clear_error();
  if (!ctx || !d_img || (count && (!d_xy || !d_moments))) return fe::fail(FE_ERR_INVALID, "NULL argument");
  if (block != 4 && block != 8 && block != 16 && block != 32)
    return fe::fail(FE_ERR_INVALID, "block must be 4, 8, 16 or 32");
  fe_status st = fe::check_shape(w, h, stride, block);
  if (st != FE_OK) return st;
  DeviceGuard g(ctx->device);
  FE_HIP(fe::launch_range_moments(d_img, w, h, stride, (int)block, d_xy, count, d_moments, (hipStream_t)stream),
         "moments launch");
  return FE_OK;
}

fe_status fe_encode(fe_ctx* ctx, const uint8_t* d_img, uint32_t w, uint32_t h, uint32_t stride,
                    const fe_params* p, fe_transform* d_out, size_t cap, size_t* n_out, void* stream) {
  fe::clear_error();
  if (!ctx || !d_img || !d_out || !n_out) return fe::fail(FE_ERR_INVALID, "NULL argument");
  fe_status st = fe_validate(w, h, stride, p);
  if (st != FE_OK) return st;
  if ((uintptr_t)d_img & 3) return fe::fail(FE_ERR_SHAPE, "image must be 4-byte aligned");
  if ((uintptr_t)d_out & 15) return fe::fail(FE_ERR_INVALID, "output must be 16-byte aligned");
  DeviceGuard g(ctx->device);
  if (p->flags & (FE_FULL_SEARCH | FE_LOCAL_SEARCH)) {
    if (p->b_min < 4) return fe::fail(FE_ERR_INVALID, "the exhaustive and local searches need b_min >= 4");
    return encode_full_search(ctx, d_img, w, h, stride, p, d_out, cap, n_out, (hipStream_t)stream);
  }
  fe_image_desc one{d_img, w, h, stride, 0};
  return encode_images(ctx, &one, 1, p, d_out, cap, nullptr, n_out, (hipStream_t)stream);
}

fe_status fe_encode_batch(fe_ctx* ctx, const fe_image_desc* h_imgs, uint32_t n_imgs, const fe_params* p,
                          fe_transform* d_out, size_t cap, uint64_t* d_offsets, size_t* n_out, void* stream) {
  fe::clear_error();
  if (!ctx) return fe::fail(FE_ERR_INVALID, "NULL argument");
  fe_status st = check_batch(h_imgs, n_imgs, p, d_out, d_offsets);
  if (st != FE_OK) return st;
  DeviceGuard g(ctx->device);
  return encode_images(ctx, h_imgs, n_imgs, p, d_out, cap, d_offsets, n_out, (hipStream_t)stream);
}

namespace {

// The decoder after argument checks; a.recs holds n 16-byte transforms on
// the device, the current device is ctx's.
fe_status decode_body(fe_ctx* ctx, const fe::DecodeArgs& a, uint32_t iters, const uint8_t* d_start, uint8_t* d_out,
                      hipStream_t s) {
  const uint64_t n = a.n;
  const uint32_t w = a.width, h = a.height, b_max = a.b_max;
  // Tile-ordered decoding needs whole top tiles, room for a domain of the
  // top size, word-aligned rows and a stream that partitions every tile in
  // stream order with co-centred domains (checked on the device below).
  bool tiled_shape = ctx->decode_mode == FE_DECODE_AUTO && n > 0 && w % b_max == 0 && h % b_max == 0 && w >= 2 * b_max && h >= 2 * b_max &&
                           ((uintptr_t)d_out & 3) == 0;
  const size_t ntiles = (size_t)(w / b_max) * (h / b_max);
  const size_t nblk = fe::decode_plan_blocks(w, h);
  if (tiled_shape) {
    fe_status st = ensure(ctx->dec_tiles, ctx->dec_tiles_n, ntiles + 1, "tile starts");
    if (st == FE_OK) st = ensure(ctx->dec_cells, ctx->dec_cells_n, nblk * 256, "decode plan cells");
    if (st == FE_OK) st = ensure(ctx->dec_pieces, ctx->dec_pieces_n, nblk * 256, "decode plan pieces");
    if (st == FE_OK) st = ensure(ctx->dec_small, ctx->dec_small_n, (size_t)n + 1, "decode 2 x 2 list");
    if (st != FE_OK) {
      // no room for the plan: the per-record decoder needs none
      (void)hipGetLastError();
      fe::clear_error();
      tiled_shape = false;
    }
  }
  FE_HIP(fe::launch_zero_u32(ctx->flags, 2, s), "zero flags");
  FE_HIP(fe::launch_decode_check(a, ctx->flags, s), "check launch");
  if (tiled_shape) FE_HIP(fe::launch_decode_tile_setup(a, ctx->dec_tiles, ctx->flags + 1, s), "tile setup");
  FE_HIP(hipMemcpyAsync(ctx->h_scalars, ctx->flags, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s),
         "flag read-back");
  FE_HIP(hipStreamSynchronize(s), "transform check");
  const uint32_t bad = (uint32_t)(ctx->h_scalars[0] & 0xffffffffu);
  if (bad) return fe::fail(FE_ERR_INVALID, "%u transforms are out of range for a %ux%u image", bad, w, h);
  const uint32_t tflags = (uint32_t)(ctx->h_scalars[0] >> 32);
  const bool tiled = tiled_shape && (tflags & 1u) == 0u;
  const bool small = tiled && (tflags & 2u) != 0u;   // 2 x 2 pieces: their kernel runs beside the tiles
  fe_status st = ensure(ctx->tmp_img, ctx->tmp_n, (size_t)w * h, "decode buffer");
  if (st != FE_OK) return st;
  uint8_t* buf[2] = {d_out, ctx->tmp_img};
  const int s0 = (int)(iters & 1u);   // iterate t lives in buf[s0 ^ (t & 1)]; t = iters in d_out
  FE_HIP(fe::launch_decode_fill(buf[1 - s0], d_start, w, h, s), "fill");
  FE_HIP(fe::launch_decode_fill(buf[s0], d_start, w, h, s), "fill");
  ctx->last_decode_tiled = tiled;
  uint32_t* small_count = tiled ? ctx->dec_small + n : nullptr;
  if (tiled && iters) {
    FE_HIP(fe::launch_zero_u32(small_count, 1, s), "zero 2 x 2 count");
    FE_HIP(fe::launch_decode_plan(a, ctx->dec_tiles, ctx->dec_cells, ctx->dec_pieces, ctx->dec_small, small_count, s),
           "plan");
  }
  for (uint32_t t = 0; t < iters; ++t) {
    Timed tm(ctx, FE_TIMING_DECODE, s);
    const uint8_t* cur = buf[s0 ^ (int)(t & 1u)];
    uint8_t* nxt = buf[s0 ^ (int)((t + 1) & 1u)];
    if (tiled) {
      FE_HIP(fe::launch_decode_tile_iter(a, ctx->dec_cells, ctx->dec_pieces, cur, nxt, s), "decode launch");
      if (small) FE_HIP(fe::launch_decode_small(a, ctx->dec_small, small_count, cur, nxt, s), "2 x 2 launch");
    }
    else
      FE_HIP(fe::launch_decode_iter(a, cur, nxt, s), "decode launch");
  }
  return FE_OK;
}

}  // namespace

fe_status fe_decode(fe_ctx* ctx, const fe_transform* d_t, size_t n, uint32_t w, uint32_t h, uint32_t b_max,
                    uint32_t iters, const uint8_t* d_start, uint8_t* d_out, void* stream) {
  fe::clear_error();
  if (!ctx || !d_out || (n && !d_t)) return fe::fail(FE_ERR_INVALID, "NULL argument");
  if (!fe::is_pow2(b_max) || b_max < 4 || b_max > 32) return fe::fail(FE_ERR_INVALID, "bad b_max %u", b_max);
  if (w < 2 || h < 2 || w > 65536 || h > 65536) return fe::fail(FE_ERR_SHAPE, "bad image size %ux%u", w, h);
  if ((uintptr_t)d_t & 15) return fe::fail(FE_ERR_INVALID, "transforms must be 16-byte aligned");
  DeviceGuard g(ctx->device);
  const fe::DecodeArgs a{reinterpret_cast<const uint4*>(d_t), (uint64_t)n, w, h, b_max, 0};
  return decode_body(ctx, a, iters, d_start, d_out, (hipStream_t)stream);
}

fe_status fe_decode_zoom(fe_ctx* ctx, const fe_transform* d_t, size_t n, uint32_t w, uint32_t h, uint32_t b_max,
                         uint32_t zoom, uint32_t iters, const uint8_t* d_start, uint8_t* d_out, void* stream) {
  fe::clear_error();
  if (!ctx || !d_out || (n && !d_t)) return fe::fail(FE_ERR_INVALID, "NULL argument");
  if (!fe::is_pow2(b_max) || b_max < 4 || b_max > 32) return fe::fail(FE_ERR_INVALID, "bad b_max %u", b_max);
  if (!fe::is_pow2(zoom) || zoom * b_max > 32)
    return fe::fail(FE_ERR_INVALID, "zoom %u: it must be a power of two with zoom * b_max <= 32", zoom);
  if (w < 2 || h < 2 || (uint64_t)w * zoom > 65536 || (uint64_t)h * zoom > 65536)
    return fe::fail(FE_ERR_SHAPE, "bad image size %ux%u at zoom %u", w, h, zoom);
  if ((uintptr_t)d_t & 15) return fe::fail(FE_ERR_INVALID, "transforms must be 16-byte aligned");
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  fe_status st = ensure(ctx->zoom_recs, ctx->zoom_recs_n, std::max<size_t>(n, 1), "zoomed transforms");
  if (st != FE_OK) return st;
  const fe::DecodeArgs native{reinterpret_cast<const uint4*>(d_t), (uint64_t)n, w, h, b_max, 0};
  FE_HIP(fe::launch_zero_u32(ctx->flags, 2, s), "zero flags");
  FE_HIP(fe::launch_decode_zoom(native, zoom, ctx->zoom_recs, ctx->flags, s), "zoom launch");
  FE_HIP(hipMemcpyAsync(ctx->h_scalars, ctx->flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "flag read-back");
  FE_HIP(hipStreamSynchronize(s), "transform check");
  const uint32_t bad = (uint32_t)(ctx->h_scalars[0] & 0xffffffffu);
  if (bad) return fe::fail(FE_ERR_INVALID, "%u transforms are out of range for a %ux%u image", bad, w, h);
  const fe::DecodeArgs a{ctx->zoom_recs, (uint64_t)n, w * zoom, h * zoom, b_max * zoom, 0};
  return decode_body(ctx, a, iters, d_start, d_out, s);
}

size_t fe_pack_bound(size_t n) { return 8 + ((33 * (uint64_t)n + 63) / 64) * 8; }

fe_status fe_pack(fe_ctx* ctx, const fe_transform* d_t, size_t n, uint32_t w, uint32_t h, uint32_t b_max,
                  uint32_t b_min, uint32_t flags, uint8_t* d_out, size_t cap, uint64_t* n_bits, void* stream) {
  fe::clear_error();
  if (!ctx || !d_out || !n_bits || (n && !d_t)) return fe::fail(FE_ERR_INVALID, "NULL argument");
  if (((uintptr_t)d_out & 7) || ((uintptr_t)d_t & 15)) return fe::fail(FE_ERR_INVALID, "misaligned buffer");
  if (flags & ~FE_PACK_ISOMETRY) return fe::fail(FE_ERR_INVALID, "unknown pack flags 0x%x", flags);
  if (!fe::is_pow2(b_max) || !fe::is_pow2(b_min) || b_min < 2 || b_max < 4 || b_max > 32 || b_min > b_max ||
      fe::levels_of(b_max, b_min) > 4)
    return fe::fail(FE_ERR_INVALID, "bad block sizes %u, %u", b_max, b_min);
  if (w % b_max || h % b_max || w < 2 * b_max || h < 2 * b_max || w > 65536 || h > 65536)
    return fe::fail(FE_ERR_SHAPE, "image %ux%u does not tile with b_max %u", w, h, b_max);
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const int L = fe::levels_of(b_max, b_min);
  const size_t ntiles = (size_t)(w / b_max) * (h / b_max);
  const size_t chunks = std::max<size_t>(fe::pack_chunks(n), 1);
  fe_status st = ensure(ctx->dec_tiles, ctx->dec_tiles_n, ntiles + 1, "tile starts");
  if (st == FE_OK) st = ensure(ctx->pack_chunk, ctx->pack_chunk_n, 2 * chunks, "pack chunk sums");
  if (st != FE_OK) return st;
  // the stream's structure (encoder order, co-centred domains) and fields
  fe::DecodeArgs a{reinterpret_cast<const uint4*>(d_t), (uint64_t)n, w, h, b_max, 0};
  FE_HIP(fe::launch_zero_u32(ctx->flags, 4, s), "zero flags");
  if (n) {
    FE_HIP(fe::launch_decode_check(a, ctx->flags, s), "check launch");
    FE_HIP(fe::launch_decode_tile_setup(a, ctx->dec_tiles, ctx->flags + 1, s), "order check");
  }
  const uint64_t header = (uint64_t)(w - 1) | ((uint64_t)(h - 1) << 16) |
                          ((uint64_t)(31 - __builtin_clz(b_max)) << 32) | ((uint64_t)(31 - __builtin_clz(b_min)) << 35) |
                          ((uint64_t)((flags & FE_PACK_ISOMETRY) ? 1 : 0) << 38);
  uint64_t* total = reinterpret_cast<uint64_t*>(ctx->flags + 2);
  FE_HIP(fe::launch_pack(reinterpret_cast<const uint4*>(d_t), (uint64_t)n, L, (int)b_min,
                         (flags & FE_PACK_ISOMETRY) != 0, header, ctx->pack_chunk, ctx->pack_chunk + chunks, total,
                         ctx->flags, reinterpret_cast<unsigned long long*>(d_out), (uint64_t)(cap / 8), s),
         "pack launch");
  FE_HIP(hipMemcpyAsync(ctx->h_scalars, ctx->flags, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s), "pack read-back");
  FE_HIP(hipStreamSynchronize(s), "pack");
  const uint32_t bad = (uint32_t)(ctx->h_scalars[0] & 0xffffffffu);
  const uint32_t disorder = (uint32_t)(ctx->h_scalars[0] >> 32) & 1u;   // bit 1 (2 x 2 blocks) is fine here
  const uint64_t bits = ctx->h_scalars[1];
  if (bad) return fe::fail(FE_ERR_INVALID, "%u transforms have fields their codes cannot hold", bad);
  if (disorder) return fe::fail(FE_ERR_INVALID, "the stream is not in encoder order with co-centred domains");
  *n_bits = bits;
  const uint64_t need = (bits + 63) / 64 * 8;
  if (need > cap) return fe::fail(FE_ERR_CAPACITY, "the file needs %llu bytes, cap is %zu", (unsigned long long)need, cap);
  return FE_OK;
}

fe_status fe_decode_set_mode(fe_ctx* ctx, int mode) {
  fe::clear_error();
  if (!ctx) return fe::fail(FE_ERR_INVALID, "NULL context");
  if (mode != FE_DECODE_AUTO && mode != FE_DECODE_RECORDS) return fe::fail(FE_ERR_INVALID, "bad decode mode %d", mode);
  ctx->decode_mode = mode;
  return FE_OK;
}

int fe_decode_last(const fe_ctx* ctx) { return ctx && ctx->last_decode_tiled ? FE_DECODE_TILES : FE_DECODE_RECORDS; }

int fe_tile_shapes(uint32_t b_max, uint32_t b_min, uint32_t* gx, uint32_t* gy, int max_out) {
  if (!fe::is_pow2(b_max) || !fe::is_pow2(b_min) || b_min < 4 || b_max > 32 || b_min > b_max) return 0;
  fe::TileShape shapes[16];
  const int k = fe::encode_shapes((int)b_max, fe::levels_of(b_max, b_min), shapes, 16);
  for (int i = 0; i < k && i < max_out; ++i) {
    if (gx) gx[i] = (uint32_t)shapes[i].gx;
    if (gy) gy[i] = (uint32_t)shapes[i].gy;
  }
  return k;
}

fe_status fe_set_tile_shape(fe_ctx* ctx, uint32_t b_max, uint32_t b_min, uint32_t gx, uint32_t gy) {
  fe::clear_error();
  if (!ctx) return fe::fail(FE_ERR_INVALID, "NULL context");
  const int n = fe_tile_shapes(b_max, b_min, nullptr, nullptr, 0);
  if (n == 0) return fe::fail(FE_ERR_INVALID, "no kernel for b_max=%u b_min=%u", b_max, b_min);
  const int L = fe::levels_of(b_max, b_min);
  if (gx == 0 && gy == 0) {
    ctx->shape_override[b_max][L] = fe::TileShape{0, 0};
    return FE_OK;
  }
  fe::TileShape shapes[16];
  const int k = fe::encode_shapes((int)b_max, L, shapes, 16);
  for (int i = 0; i < k; ++i) {
    if ((uint32_t)shapes[i].gx == gx && (uint32_t)shapes[i].gy == gy) {
      ctx->shape_override[b_max][L] = shapes[i];
      return FE_OK;
    }
  }
  return fe::fail(FE_ERR_INVALID, "tile shape %ux%u is not built for b_max=%u b_min=%u", gx, gy, b_max, b_min);
}

fe_status fe_get_tile_shape(fe_ctx* ctx, uint32_t b_max, uint32_t b_min, uint32_t* gx, uint32_t* gy) {
  fe::clear_error();
  if (!ctx || !gx || !gy) return fe::fail(FE_ERR_INVALID, "NULL argument");
  if (fe_tile_shapes(b_max, b_min, nullptr, nullptr, 0) == 0)
    return fe::fail(FE_ERR_INVALID, "no kernel for b_max=%u b_min=%u", b_max, b_min);
  const fe::TileShape t = pick_shape(ctx, (int)b_max, fe::levels_of(b_max, b_min));
  *gx = (uint32_t)t.gx;
  *gy = (uint32_t)t.gy;
  return FE_OK;
}

fe_status fe_autotune(fe_ctx* ctx, const fe_image_desc* h_imgs, uint32_t n_imgs, const fe_params* p,
                      fe_transform* d_out, size_t cap, uint64_t* d_offsets, uint32_t reps, uint32_t* gx,
                      uint32_t* gy, double* ms, void* stream) {
  fe::clear_error();
  if (!ctx || !gx || !gy || !ms || reps == 0) return fe::fail(FE_ERR_INVALID, "bad arguments");
  fe_status st = fe::check_params(p);
  if (st != FE_OK) return st;
  if (p->b_min < 4) return fe::fail(FE_ERR_INVALID, "b_min 2 has no tile shapes to tune");
  const int L = fe::levels_of(p->b_max, p->b_min);
  fe::TileShape shapes[16];
  const int k = fe::encode_shapes((int)p->b_max, L, shapes, 16);
  const bool was_timing = ctx->timing;
  // two rounds over the shapes, each shape keeping its better mean: the
  // first launches after the device has idled run slower, and a single
  // round would charge that to the first shape
  double mean_of[16];
  for (int i = 0; i < k; ++i) mean_of[i] = 1e30;
  for (int round = 0; round < 2 && st == FE_OK; ++round) {
    for (int i = 0; i < k; ++i) {
      ctx->shape_override[p->b_max][L] = shapes[i];
      st = fe_encode_batch(ctx, h_imgs, n_imgs, p, d_out, cap, d_offsets, nullptr, stream);   // warm-up
      if (st != FE_OK) break;
      double t_ms[FE_TIMING_SLOTS];
      uint64_t cnt[FE_TIMING_SLOTS];
      if ((st = fe_timing_read(ctx, t_ms, cnt, FE_TIMING_SLOTS)) != FE_OK) break;
      if ((st = fe_timing_enable(ctx, 1)) != FE_OK) break;
      for (uint32_t r = 0; r < reps && st == FE_OK; ++r)
        st = fe_encode_batch(ctx, h_imgs, n_imgs, p, d_out, cap, d_offsets, nullptr, stream);
      if (st != FE_OK) break;
      if ((st = fe_timing_read(ctx, t_ms, cnt, FE_TIMING_SLOTS)) != FE_OK) break;
      const double mean = cnt[FE_TIMING_ENCODE] ? t_ms[FE_TIMING_ENCODE] / (double)cnt[FE_TIMING_ENCODE] : 1e30;
      mean_of[i] = std::min(mean_of[i], mean);
    }
  }
  double best = 1e30;
  fe::TileShape best_shape{0, 0};
  for (int i = 0; i < k; ++i)
    if (mean_of[i] < best) {
      best = mean_of[i];
      best_shape = shapes[i];
    }
  ctx->timing = was_timing;
  if (st != FE_OK) {
    ctx->shape_override[p->b_max][L] = fe::TileShape{0, 0};
    return st;
  }
  ctx->shape_override[p->b_max][L] = best_shape;
  *gx = (uint32_t)best_shape.gx;
  *gy = (uint32_t)best_shape.gy;
  *ms = best;
  return FE_OK;
}

fe_status fe_full_search_ranges(fe_ctx* ctx, const uint8_t* d_img, uint32_t w, uint32_t h, uint32_t stride,
                                uint32_t block, const uint32_t* d_xy, uint32_t count, uint32_t* d_out, void* stream) {
  fe::clear_error();
  if (!ctx || !d_img || (count && (!d_xy || !d_out))) return fe::fail(FE_ERR_INVALID, "NULL argument");
  if (block != 4 && block != 8 && block != 16) return fe::fail(FE_ERR_INVALID, "block must be 4, 8 or 16");
  fe_status st = fe::check_shape(w, h, stride, block);
  if (st != FE_OK) return st;
  if ((st = fs_check(w, h, block, block)) != FE_OK) return st;
  if (count == 0) return FE_OK;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const fe::FsPlan pl = fe::fs_plan(w, h, block);
  if ((st = ensure(ctx->fs_planes, ctx->fs_planes_n, pl.plane_bytes, "phase planes")) != FE_OK) return st;
  if ((st = fs_reserve(ctx, pl, count)) != FE_OK) return st;
  FE_HIP(fe::fs_planes(pl, d_img, w, h, stride, ctx->fs_planes, s), "phase planes");
  FE_HIP(fe::fs_domain_sums(pl, w, h, ctx->fs_planes, ctx->fs_sd, ctx->fs_qd, s), "domain sums");
  {
    Timed t(ctx, FE_TIMING_FULLSEARCH, s);
    FE_HIP(fe::fs_search(pl, d_img, w, h, stride, ctx->fs_planes, ctx->fs_sd, ctx->fs_qd, d_xy, count, ctx->fs_frag,
                         ctx->fs_sr, ctx->fs_alpha, ctx->fs_beta, ctx->fs_best, s),
           "search launch");
  }
  FE_HIP(fe::fs_report(pl, d_img, w, h, stride, ctx->fs_planes, d_xy, count, ctx->fs_best, d_out, s), "report");
  return FE_OK;
}

fe_status fe_timing_enable(fe_ctx* ctx, int enable) {
  fe::clear_error();
  if (!ctx) return fe::fail(FE_ERR_INVALID, "NULL context");
  DeviceGuard g(ctx->device);
  if (enable && !ctx->ev) {
    ctx->ev = new hipEvent_t[2 * fe_ctx::kTimingCap]();
    // timestamps only: no system-scope fence (cache writeback) when an
    // event completes, which would add to the bracketed kernel's time
    for (int i = 0; i < 2 * fe_ctx::kTimingCap; ++i)
      FE_HIP(hipEventCreateWithFlags(&ctx->ev[i], hipEventDisableSystemFence), "timing events");
  }
  ctx->timing = enable != 0;
  return FE_OK;
}

fe_status fe_timing_select(fe_ctx* ctx, uint32_t slot_mask) {
  fe::clear_error();
  if (!ctx) return fe::fail(FE_ERR_INVALID, "NULL context");
  ctx->timing_mask = slot_mask;
  return FE_OK;
}

fe_status fe_timing_read(fe_ctx* ctx, double* ms, uint64_t* launches, uint32_t n) {
  fe::clear_error();
  if (!ctx || (n && (!ms || !launches)) || n > FE_TIMING_SLOTS) return fe::fail(FE_ERR_INVALID, "bad arguments");
  DeviceGuard g(ctx->device);
  for (uint32_t k = 0; k < n; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (int i = 0; i < ctx->ev_used; ++i) {
    FE_HIP(hipEventSynchronize(ctx->ev[2 * i + 1]), "timing event");
    float t = 0.f;
    FE_HIP(hipEventElapsedTime(&t, ctx->ev[2 * i], ctx->ev[2 * i + 1]), "timing elapsed");
    const int slot = ctx->ev_slot[i];
    if (slot >= 0 && (uint32_t)slot < n) {
      ms[slot] += t;
      launches[slot] += 1;
    }
  }
  ctx->ev_used = 0;
  return FE_OK;
}

// ---------------------------------------------------------------- plans
}  // extern "C"

namespace {

// Nodes of a linear graph in dependency order (empty if not a chain).
std::vector<hipGraphNode_t> chain_of(hipGraph_t g) {
  std::vector<hipGraphNode_t> out;
  size_t nroots = 0;
  if (hipGraphGetRootNodes(g, nullptr, &nroots) != hipSuccess || nroots != 1) return {};
  hipGraphNode_t cur = nullptr;
  if (hipGraphGetRootNodes(g, &cur, &nroots) != hipSuccess) return {};
  while (cur) {
    out.push_back(cur);
    size_t nd = 0;
    if (hipGraphNodeGetDependentNodes(cur, nullptr, &nd) != hipSuccess || nd > 1) return {};
    hipGraphNode_t next = nullptr;
    if (nd == 1 && hipGraphNodeGetDependentNodes(cur, &next, &nd) != hipSuccess) return {};
    cur = nd == 1 ? next : nullptr;
  }
  return out;
}

// Splice event-record nodes into a copy of the plan's chain
// [[zero count], encode, [2 x 2 level], order...]: own[0] just before the
// encode kernel (after the count's clearing, or as a root), own[1] and
// own[2] between the encode kernels and the first ordering kernel, own[3]
// after the last.  Instantiates the copy.  Returns false (and leaves the
// plan untouched) if any step fails.
bool add_timing_nodes(fe_plan* pl, size_t i_enc, size_t i_ord) {
  hipGraph_t g = nullptr;
  if (hipGraphClone(&g, pl->graph) != hipSuccess) return false;
  bool ok = false;
  do {
    // chain positions: the encode kernels are c[i_enc] .. c[i_ord - 1], the
    // ordering kernels c[i_ord] ..
    std::vector<hipGraphNode_t> c = chain_of(g);
    if (i_ord <= i_enc || c.size() <= i_ord) break;
    hipGraphNode_t enc = c[i_enc], enc_end = c[i_ord - 1], ord = c[i_ord], last = c.back();
    hipGraphNode_t n[4] = {};
    if (i_enc > 0) {
      if (hipGraphAddEventRecordNode(&n[0], g, &c[i_enc - 1], 1, pl->own[0]) != hipSuccess) break;
    } else {
      if (hipGraphAddEventRecordNode(&n[0], g, nullptr, 0, pl->own[0]) != hipSuccess) break;
    }
    if (hipGraphAddDependencies(g, &n[0], &enc, 1) != hipSuccess) break;
    if (hipGraphAddEventRecordNode(&n[1], g, &enc_end, 1, pl->own[1]) != hipSuccess) break;
    if (hipGraphAddEventRecordNode(&n[2], g, &enc_end, 1, pl->own[2]) != hipSuccess) break;
    if (hipGraphAddDependencies(g, &n[1], &ord, 1) != hipSuccess) break;
    if (hipGraphAddDependencies(g, &n[2], &ord, 1) != hipSuccess) break;
    if (hipGraphAddEventRecordNode(&n[3], g, &last, 1, pl->own[3]) != hipSuccess) break;
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) break;
    // node handles of the instantiated copy are those of `g`
    for (int k = 0; k < 4; ++k) pl->tnode[k] = n[k];
    (void)hipGraphDestroy(pl->graph);
    pl->graph = g;
    pl->exec = ex;
    ok = true;
  } while (false);
  if (!ok) (void)hipGraphDestroy(g);
  return ok;
}

}  // namespace

extern "C" {

fe_status fe_plan_create(fe_ctx* ctx, const fe_image_desc* h_imgs, uint32_t n_imgs, const fe_params* p,
                         fe_transform* d_out, size_t cap, uint64_t* d_offsets, fe_plan** out) {
  fe::clear_error();
  if (!ctx || !out) return fe::fail(FE_ERR_INVALID, "NULL argument");
  *out = nullptr;
  fe_status st = check_batch(h_imgs, n_imgs, p, d_out, d_offsets);
  if (st != FE_OK) return st;
  DeviceGuard g(ctx->device);
  std::vector<fe::ImgDev> table(n_imgs);
  fe::EncodeGeom geo;
  if ((st = fe::encode_geometry(ctx, h_imgs, n_imgs, p, table.data(), geo)) != FE_OK) return st;
  const bool ext = geo.ext;
  const uint64_t tiles = geo.tiles;
  const uint32_t wgs = geo.wgs;
  fe_plan* pl = new fe_plan();
  pl->device = ctx->device;
  pl->n_imgs = n_imgs;
  // device table: the ImgDev entries, their wg_first words, chunk images
  std::vector<fe::ImgDev> host;
  const size_t slots = table_words(table.data(), n_imgs, tiles, host);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&pl->d_table), slots * sizeof(fe::ImgDev));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&pl->blocks), std::max<size_t>(wgs, 1) * sizeof(fe::BlockDesc));
  if (e == hipSuccess)
    e = hipMalloc(reinterpret_cast<void**>(&pl->staging), std::max<size_t>((size_t)geo.slots, 1) * 16);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&pl->masks), std::max<size_t>(tiles, 1) * 8);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&pl->chunk_sum), std::max<size_t>(geo.chunks, 1) * 4);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&pl->chunk_base), (geo.chunks + 1) * 8);
  if (e == hipSuccess && ext) e = hipMalloc(reinterpret_cast<void**>(&pl->fine_list), std::max<uint64_t>(geo.fine_max, 1) * 16);
  if (e == hipSuccess && ext) e = hipMalloc(reinterpret_cast<void**>(&pl->fine_count), 4);
  if (e == hipSuccess) e = hipMemcpy(pl->d_table, host.data(), slots * sizeof(fe::ImgDev), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->capture, hipStreamNonBlocking);
  for (int k = 0; k < 4 && e == hipSuccess; ++k) e = hipEventCreate(&pl->own[k]);
  if (e != hipSuccess) {
    fe_plan_destroy(pl);
    return hip_fail(e, "plan allocation");
  }
  pl->ctx = ctx;
  // The block descriptors depend only on the images' addresses and sides,
  // which a plan fixes: they are built once, here, not in every replay.
  e = fe::launch_block_prep(pl->d_table, n_imgs, wgs, geo.bmax, geo.shape.gx, geo.shape.gy, pl->blocks, pl->capture);
  if (e == hipSuccess) e = hipStreamSynchronize(pl->capture);
  if (e != hipSuccess) {
    fe_plan_destroy(pl);
    return hip_fail(e, "plan block descriptors");
  }
  // record the launch sequence once; replays re-read the images in place.
  // Chain: [zero count], encode, [2 x 2 level], ordering; the count is
  // cleared by a kernel, not a memset node.
  e = hipStreamBeginCapture(pl->capture, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const fe::EncodeBufs b{pl->d_table, pl->blocks, pl->staging, pl->masks, pl->chunk_sum, pl->chunk_base,
                           pl->fine_list, pl->fine_count};
    const fe_status ls = fe::encode_launch(nullptr, geo, b, n_imgs, p, false, d_out, cap, d_offsets, pl->capture);
    e = hipStreamEndCapture(pl->capture, &pl->graph);
    if (ls != FE_OK && e == hipSuccess) e = hipErrorLaunchFailure;
  }
  if (e != hipSuccess) {
    fe_plan_destroy(pl);
    return hip_fail(e, "plan capture");
  }
  // The capture is a chain: [zero count], encode, [2 x 2 level], then the
  // ordering kernels.  If timing is on, a copy of it gets event-record nodes
  // before and after the encode kernels and after the last ordering kernel;
  // if that fails, or timing is off, the plain chain is used and launches
  // are not timed.
  pl->timed = ctx->timing && (ext ? add_timing_nodes(pl, 1, 3) : add_timing_nodes(pl, 0, 1));
  if (!pl->timed) {
    e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      fe_plan_destroy(pl);
      return hip_fail(e, "plan instantiate");
    }
  }
  *out = pl;
  return FE_OK;
}

fe_status fe_plan_launch(fe_plan* pl, void* stream) {
  fe::clear_error();
  if (!pl) return fe::fail(FE_ERR_INVALID, "NULL plan");
  DeviceGuard g(pl->device);
  fe_ctx* c = pl->ctx;
  if (pl->timed) {
    // point the event nodes at two fresh pairs of the context's timing
    // events (a node update takes effect from the next launch on)
    if (c && c->timing && c->ev && c->ev_used + 2 <= fe_ctx::kTimingCap) {
      const int i = c->ev_used++, j = c->ev_used++;
      c->ev_slot[i] = FE_TIMING_ENCODE;
      c->ev_slot[j] = FE_TIMING_SCATTER;
      const hipEvent_t evs[4] = {c->ev[2 * i], c->ev[2 * i + 1], c->ev[2 * j], c->ev[2 * j + 1]};
      for (int k = 0; k < 4; ++k)
        FE_HIP(hipGraphExecEventRecordNodeSetEvent(pl->exec, pl->tnode[k], evs[k]), "plan timing node");
      pl->on_ctx = true;
    } else if (pl->on_ctx) {
      for (int k = 0; k < 4; ++k)
        FE_HIP(hipGraphExecEventRecordNodeSetEvent(pl->exec, pl->tnode[k], pl->own[k]), "plan timing node");
      pl->on_ctx = false;
    }
  }
  FE_HIP(hipGraphLaunch(pl->exec, (hipStream_t)stream), "plan launch");
  return FE_OK;
}

void fe_plan_destroy(fe_plan* pl) {
  if (!pl) return;
  DeviceGuard g(pl->device);
  if (pl->capture) (void)hipStreamSynchronize(pl->capture);
  (void)hipDeviceSynchronize();   // no replay may still use the buffers
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->capture) (void)hipStreamDestroy(pl->capture);
  for (hipEvent_t ev : pl->own)
    if (ev) (void)hipEventDestroy(ev);
  for (void* q : {(void*)pl->d_table, (void*)pl->blocks, (void*)pl->staging, (void*)pl->masks,
                  (void*)pl->chunk_sum, (void*)pl->chunk_base, (void*)pl->fine_list, (void*)pl->fine_count})
    if (q) (void)hipFree(q);
  delete pl;
}

}  // extern "C"
