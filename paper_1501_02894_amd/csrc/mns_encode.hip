// Fused MNS quadtree encoder for gfx950.
//
// One workgroup (256 lanes, 4 waves) owns a GX x GY block of top-level
// B_max tiles of one image and runs the whole quadtree of those tiles:
//
//   1. stage: the pixels of the union of the tiles' co-centred 2B x 2B
//      domains (which contains every range and every descendant's domain)
//      are read once from HBM into LDS; the 2 x 2 round-half-up mean image
//      H0 of that region and its transpose are formed in LDS on the fly
//      (Sec. 3, the four-neighbour mean filter).
//   2. per level l (B = B_max >> (l-1)), the workgroup's list of ranges is
//      fitted one range per lane: sums of packed-u8 dot products
//      (v_dot4_u32_u8) over row pairs of the range and of the domain window
//      / its transpose give Sum r, Sum r^2, Sum d, Sum d^2 and the 8
//      isometric Sum r T_e(d), and the lane fits (e, k, m) exactly in fp64
//      (Sec. 3).  Long lists are dealt round the waves in groups of 64;
//      a list of at most 64 ranges has its rows spread over the waves, whose
//      partial sums meet in LDS before one wave fits it.
//   3. phase 2 (Sec. 3.1-3.3): in the same lanes, the parents that failed at
//      level l-1 are decided from the identity moments of their four
//      children, which are exactly the level-l ranges just computed (four
//      consecutive lanes, exchanged by DPP).
//   4. accepted ranges are written as 16-byte records into per-tile slots
//      indexed by the Morton code of their top-left B_min cell; failed ranges
//      are compacted (wave ballot + prefix, one LDS atomic per wave) into the
//      workgroup's parent list, which every wave reads after a barrier: entry
//      e of the next level is child e mod 4 (Z order) of parent e / 4.
//
// After the workgroup finishes, its tiles' occupancy masks are published;
// the ordering kernels (order.hip) pack the records into the depth-first
// stream (tiles in raster order, Morton order inside a tile).
#include <algorithm>

#include "fe_device.h"
#include "fe_internal.h"

namespace fe {
namespace {

template <int BMAX, int L, int GX, int GY>
struct Geo {
  static constexpr int BMAXV = BMAX;
  static constexpr int GXV = GX;
  static constexpr int BMIN = BMAX >> (L - 1);
  static constexpr int NT = GX * GY;                          // tiles per workgroup
  static constexpr int LOG_GX = Log2<GX>::value;
  static constexpr int CELLS = 1 << (2 * (L - 1));
  // failed ranges of one level, at most NT 4^(L-2) (level L-1)
  static constexpr int PCAP = NT * CELLS / 4 > 0 ? NT * CELLS / 4 : 1;
  static constexpr int TW = GX * BMAX, TH = GY * BMAX;        // tile block in pixels
  // Tile pixels in LDS tile after tile, each tile row-major (pitch BMAX
  // bytes), tiles TSTRIDE bytes apart: one dword more than a tile, so that
  // the same row of different tiles falls in different banks.
  static constexpr int TPITCH = BMAX;                         // tile pixel row pitch (bytes)
  static constexpr int TSTRIDE = BMAX * BMAX + 4;             // tile stride (bytes)
  // The staged region is the union of the tiles' co-centred domains,
  // (GX + 1) x (GY + 1) tiles, with its origin rounded down to 8 pixels.
  // For b_max >= 16 the origin X0 - b_max / 2 (or its clamp to the image) is
  // a multiple of 8 already, so the bounds are exact.
  static constexpr bool EXACT = BMAX >= 16;
  static constexpr int RWA = EXACT ? (GX + 1) * BMAX : ((GX + 1) * BMAX + 6 + 7) & ~7;  // region width bound (px)
  static constexpr int RHA = EXACT ? (GY + 1) * BMAX : (GY + 1) * BMAX + 8;             // region height bound (px)
  static constexpr int HW = RWA / 2, HH = RHA / 2;            // H0 region bounds
  static constexpr int HH4 = (HH + 3) & ~3;                   // H0 rows, multiple of 4
  // Row pitches of H0 and H0^T: an odd number of dwords, so that the rows
  // a range's window spans start in different banks.
  static constexpr int odd_pitch(int w) { return ((w / 4 + 1) & 1) ? w + 4 : w + 8; }
  static constexpr int HP = EXACT ? odd_pitch(HW) : HW + 8;   // H0 row pitch
  static constexpr int TP = EXACT ? odd_pitch(HH4) : HH4 + 8; // H0^T row pitch
  static constexpr int IMG_W = NT * TSTRIDE / 4 + 4;          // dwords
  static constexpr int H0_W = HH4 * HP / 4 + 4;
  static constexpr int H0T_W = HW * TP / 4 + 4;
  static_assert(NT % 4 == 0 && NT <= 256, "tiles per workgroup: a multiple of 4, at most one per lane");
  // Moments of a short list, summed over the waves.  Below b_max = 32 only
  // the top level has short lists (its list is the block's tiles, at most
  // NT), and they are summed before that level writes its failed ranges, so
  // the sums share their words with the lists of failed ranges.
  static constexpr bool SHARE = BMAX <= 16;
  static constexpr int PW = SHARE ? (NT <= 64 ? NT : 1) : 64;    // sums per moment
  static constexpr int LIST_W = SHARE ? (2 * PCAP > 12 * PW ? 2 * PCAP : 12 * PW) : 2 * PCAP + 12 * PW;
};

struct Region {
  int W, H;            // image sides
  int ax0, ay0;        // H0 region origin (pixels), multiples of 8
  int X0, Y0;          // tile block origin (pixels)
  int tiles_x;
  uint64_t tg0;        // global index of the block's first tile
};

// Geometry of one block of top tiles and of its staged region.
struct BlockGeo {
  Region rg;
  const uint8_t* data;
  uint32_t stride;
  int gx, gy;            // tiles of the block inside the image
  int n8, hrows;         // region: 8-pixel column groups, row pairs
  int tx_end, ty_end;    // end of the tile block (pixels)
  uint32_t sblk;         // record-slot block
};

// A workgroup's thresholds and flags (workgroup-uniform): the call's, or
// its own words when the call mixes parameter sets.  Selected by value, not
// indexed, so that they stay in scalar registers.
struct LevelParams {
  uint32_t t0, t1, t2, t3;
  bool phase2, identity_only;
  __device__ __forceinline__ uint32_t thr(int l) const { return l == 0 ? t0 : l == 1 ? t1 : l == 2 ? t2 : t3; }
};

__device__ __forceinline__ LevelParams level_params(const EncodeArgs& a, uint32_t wg) {
  LevelParams p;
  if (a.wg_params) {
    const uint32_t* w = a.wg_params + (size_t)wg * kWgParamWords;
    p.t0 = w[0];
    p.t1 = w[1];
    p.t2 = w[2];
    p.t3 = w[3];
    p.phase2 = (w[4] & FE_PHASE2) != 0;
    p.identity_only = (w[4] & FE_IDENTITY_ONLY) != 0;
  } else {
    p.t0 = a.thr[0];
    p.t1 = a.thr[1];
    p.t2 = a.thr[2];
    p.t3 = a.thr[3];
    p.phase2 = a.phase2 != 0;
    p.identity_only = a.identity_only != 0;
  }
  return p;
}

template <int BMAX, int GX, int GY>
__device__ __forceinline__ BlockGeo block_geo(const BlockDesc& d) {
  BlockGeo b;
  b.rg.W = (int)(d.wh & 0xffffu) + 1;
  b.rg.H = (int)(d.wh >> 16) + 1;
  const int tx0 = (int)(d.t0 & 0xffffu), ty0 = (int)(d.t0 >> 16);
  b.rg.tiles_x = b.rg.W / BMAX;
  b.gx = min(GX, b.rg.tiles_x - tx0);
  b.gy = min(GY, b.rg.H / BMAX - ty0);
  b.rg.tg0 = d.tg0;
  b.rg.X0 = tx0 * BMAX;
  b.rg.Y0 = ty0 * BMAX;
  // union of the tiles' co-centred domains (it contains every range and
  // every descendant's domain), origin rounded down to 8 pixels
  const int rx0 = clampi(b.rg.X0 - BMAX / 2, 0, b.rg.W - 2 * BMAX);
  const int rx1 = clampi((tx0 + b.gx - 1) * BMAX - BMAX / 2, 0, b.rg.W - 2 * BMAX) + 2 * BMAX;
  const int ry0 = clampi(b.rg.Y0 - BMAX / 2, 0, b.rg.H - 2 * BMAX);
  const int ry1 = clampi((ty0 + b.gy - 1) * BMAX - BMAX / 2, 0, b.rg.H - 2 * BMAX) + 2 * BMAX;
  b.rg.ax0 = rx0 & ~7;
  b.rg.ay0 = ry0 & ~7;
  b.n8 = (rx1 - b.rg.ax0 + 7) >> 3;
  b.hrows = (ry1 - b.rg.ay0) >> 1;
  b.tx_end = b.rg.X0 + b.gx * BMAX;
  b.ty_end = b.rg.Y0 + b.gy * BMAX;
  b.data = d.data;
  b.stride = d.stride;
  b.sblk = d.sblk;
  return b;
}

// Image words read through the global address space (global_load rather
// than flat_load, which would also occupy the LDS counter).
typedef __attribute__((address_space(1))) const uint32_t gu32;

// Word 3 of a raw buffer resource on gfx9-family chips (gfx950 included):
// 32-bit data format, no swizzle, no index stride.
constexpr int kBufferWord3 = 0x00020000;

// Region staging.  A group is 8 x 8 pixels of the region (column group c8,
// rows 8 g .. 8 g + 7), i.e. a 4 x 4 block of H0; lane `tid` owns groups
// tid + 256 * it.  load() reads the lane's groups from the image into
// registers; store() writes them to LDS: the tile pixels, H0 as dwords, and
// its transpose as dwords after a 4 x 4 byte transpose in registers.
template <class G>
struct Stage {
  static constexpr int NC8 = G::RWA / 8;
  static constexpr int NG = (G::HH4 / 4 * NC8 + 255) / 256;
  uint32_t v[NG][8][2];

  __device__ __forceinline__ static bool owns(const BlockGeo& b, int idx, int& g, int& c8) {
    g = idx / NC8;
    c8 = idx - g * NC8;
    return 4 * g < b.hrows && c8 < b.n8;
  }

  __device__ __forceinline__ void load(const BlockGeo& b, int tid) {
    if constexpr (G::BMAXV >= 16) {
      // Through a buffer resource based at the region origin, row r of a
      // group is the scalar offset r * stride: no per-row address arithmetic
      // in vector registers.  Needs every region offset below 2^31.
      if ((uint64_t)G::RHA * b.stride < (1ull << 31)) {
        const uint8_t* org = b.data + (size_t)b.rg.ay0 * b.stride + b.rg.ax0;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t*>(org), (short)0, (int)((uint32_t)G::RHA * b.stride), kBufferWord3);
#pragma unroll
        for (int it = 0; it < NG; ++it) {
          int g, c8;
          if (!owns(b, tid + 256 * it, g, c8)) continue;
          const uint32_t voff = (uint32_t)(8 * g) * b.stride + 8u * (uint32_t)c8;
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, (uint32_t)r * b.stride, 0);
            v[it][r][0] = w[0];
            v[it][r][1] = w[1];
          }
        }
        return;
      }
    }
#pragma unroll
    for (int it = 0; it < NG; ++it) {
      int g, c8;
      if (!owns(b, tid + 256 * it, g, c8)) continue;
      const int x = b.rg.ax0 + 8 * c8;
      const uint8_t* row0 = b.data + (size_t)(b.rg.ay0 + 8 * g) * b.stride + x;
      if constexpr (G::BMAXV >= 16) {
        // the region spans multiples of 8 pixels inside the image in both
        // directions, so every group is whole
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const gu32* p = (const gu32*)(row0 + (size_t)r * b.stride);
          v[it][r][0] = p[0];
          v[it][r][1] = p[1];
        }
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          v[it][r][0] = v[it][r][1] = 0u;
          if (8 * g + r < 2 * b.hrows) {
            const gu32* p = (const gu32*)(row0 + (size_t)r * b.stride);
            if (x + 8 <= b.rg.W) {
              v[it][r][0] = p[0];
              v[it][r][1] = p[1];
            } else if (x < b.rg.W) {
              v[it][r][0] = p[0];
            }
          }
        }
      }
    }
  }

  __device__ __forceinline__ void store(const BlockGeo& b, int tid, uint32_t* s_img, uint32_t* s_h0,
                                        uint32_t* s_h0t) const {
#pragma unroll
    for (int it = 0; it < NG; ++it) {
      int g, c8;
      if (!owns(b, tid + 256 * it, g, c8)) continue;
      const int x = b.rg.ax0 + 8 * c8;
      const uint32_t(&w)[8][2] = v[it];
      // tile pixels.  For b_max >= 8 the tile block starts at a multiple of
      // 8 pixels from the region origin in both directions and spans a
      // multiple of 8, so a group lies wholly inside or outside it; for
      // b_max = 4 tile edges are multiples of 4 and rows/halves are tested.
      if constexpr (G::BMAXV >= 8) {
        const int gy0 = b.rg.ay0 + 8 * g;
        if (gy0 >= b.rg.Y0 && gy0 < b.ty_end && x >= b.rg.X0 && x < b.tx_end) {
          // inside the tile block, so non-negative
          const uint32_t px = (uint32_t)(x - b.rg.X0), py = (uint32_t)(gy0 - b.rg.Y0);
          const uint32_t t = (py / G::BMAXV) * G::GXV + px / G::BMAXV;
          uint32_t* dst = s_img + t * (G::TSTRIDE / 4) + (py % G::BMAXV) * (G::TPITCH / 4) + (px % G::BMAXV) / 4;
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            dst[r * (G::TPITCH / 4)] = w[r][0];
            dst[r * (G::TPITCH / 4) + 1] = w[r][1];
          }
        }
      } else {
        // 4 x 4 tiles: one row of four pixels per tile and dword
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int y = b.rg.ay0 + 8 * g + r;
          if (y < b.rg.Y0 || y >= b.ty_end) continue;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int xx = x + 4 * h;
            if (xx >= b.rg.X0 && xx < b.tx_end) {
              const int t = ((y - b.rg.Y0) >> 2) * G::GXV + ((xx - b.rg.X0) >> 2);
              s_img[t * (G::TSTRIDE / 4) + ((y - b.rg.Y0) & 3)] = w[r][h];
            }
          }
        }
      }
      // 2x2 means: H0 rows 4g .. 4g+3, columns 4 c8 .. 4 c8 + 3
      uint32_t hrow[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        hrow[q] = mean2x2_x4(w[2 * q][0], w[2 * q][1], w[2 * q + 1][0], w[2 * q + 1][1]);
        s_h0[(4 * g + q) * (G::HP / 4) + c8] = hrow[q];
      }
      // transpose the 4x4 byte block: H0T rows 4 c8 .. 4 c8 + 3, columns 4g..
      const uint32_t u0 = __builtin_amdgcn_perm(hrow[1], hrow[0], 0x05010400u);
      const uint32_t u1 = __builtin_amdgcn_perm(hrow[1], hrow[0], 0x07030602u);
      const uint32_t w0 = __builtin_amdgcn_perm(hrow[3], hrow[2], 0x05010400u);
      const uint32_t w1 = __builtin_amdgcn_perm(hrow[3], hrow[2], 0x07030602u);
      s_h0t[(4 * c8 + 0) * (G::TP / 4) + g] = __builtin_amdgcn_perm(w0, u0, 0x05040100u);
      s_h0t[(4 * c8 + 1) * (G::TP / 4) + g] = __builtin_amdgcn_perm(w0, u0, 0x07060302u);
      s_h0t[(4 * c8 + 2) * (G::TP / 4) + g] = __builtin_amdgcn_perm(w1, u1, 0x05040100u);
      s_h0t[(4 * c8 + 3) * (G::TP / 4) + g] = __builtin_amdgcn_perm(w1, u1, 0x07060302u);
    }
  }
};

template <int BMAX, int L, int GX, int GY>
struct Lds {
  using G = Geo<BMAX, L, GX, GY>;
  uint32_t img[G::IMG_W];
  uint32_t h0[G::H0_W];
  uint32_t h0t[G::H0T_W];
  uint32_t top[G::NT];             // level-1 list: the block's tiles inside the image
  // failed ranges of two consecutive levels (list entries), and the
  // moments of a short list summed over the waves (see Geo::SHARE)
  uint32_t lists[G::LIST_W];
  uint32_t cnt[L + 1];             // per level: ranges that failed (parents of the next list)
  unsigned long long mask[G::NT];
  __device__ __forceinline__ uint32_t* par(int k) { return lists + k * G::PCAP; }
  __device__ __forceinline__ uint32_t* part(int j) { return lists + (G::SHARE ? 0 : 2 * G::PCAP) + j * G::PW; }
};

// DPP: every lane of a quad reads quad lane Q's value, or the sum over its quad.
template <int Q>
__device__ __forceinline__ int quad_bcast(int v) {
  return __builtin_amdgcn_update_dpp(0, v, Q * 0x55, 0xF, 0xF, false);
}
__device__ __forceinline__ int quad_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  return v + __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
}

// A range of the list: its place inside the workgroup's block of tiles.
// List entries hold x | y << 8 (pixels from the block's first tile) | the
// Morton code of its top-left B_min cell inside its tile << 16, and in the
// lists of failed ranges also its phase-1 mean m << 24.  Entry e of a level
// below the top is child e mod 4 (Z order) of failed range e / 4 above.
struct RangeRef {
  int xr, yr;   // relative to the block's first tile
  int cell;     // Morton code of the top-left B_min cell in its tile
  int m;        // the parent's mean (levels below the top)
};

template <int BB, int BMAX, int BMIN>
__device__ __forceinline__ RangeRef range_ref(const uint32_t* top, const uint32_t* ppar, int e) {
  RangeRef r;
  if constexpr (BB == BMAX) {
    const uint32_t t = top[e];
    r.xr = (int)(t & 0xffu);
    r.yr = (int)((t >> 8) & 0xffu);
    r.cell = 0;
    r.m = 0;
  } else {
    constexpr int CL = (BB / BMIN) * (BB / BMIN);   // cells covered by one range of this level
    const uint32_t pe = ppar[e >> 2];
    const int c = e & 3;
    r.xr = (int)(pe & 0xffu) + (c & 1) * BB;
    r.yr = (int)((pe >> 8) & 0xffu) + (c >> 1) * BB;
    r.cell = (int)((pe >> 16) & 0xffu) + c * CL;
    r.m = (int)(pe >> 24);
  }
  return r;
}

// LDS offsets of a range's pixels, of its co-centred domain window in H0
// and of that window in H0^T.
template <class G, int BB>
struct Window {
  int dx, dy;            // domain origin (pixels, in the image)
  int roff, doff, toff;
  __device__ __forceinline__ Window(const RangeRef& r, const Region& rg) {
    dx = clampi(rg.X0 + r.xr - BB / 2, 0, rg.W - 2 * BB);
    dy = clampi(rg.Y0 + r.yr - BB / 2, 0, rg.H - 2 * BB);
    const int wx = (dx - rg.ax0) >> 1, wy = (dy - rg.ay0) >> 1;
    constexpr int LB = Log2<G::BMAXV>::value;
    roff = ((r.yr >> LB) * G::GXV + (r.xr >> LB)) * G::TSTRIDE + (r.yr & (G::BMAXV - 1)) * G::TPITCH +
           (r.xr & (G::BMAXV - 1));
    doff = wy * G::HP + wx;
    toff = wx * G::TP + wy;
  }
};

// Record slot, inside its block's slots, of the record at Morton cell
// `cell` (record-cell units) of the tile at column tx, row ty of the block:
// a record that covers the whole tile goes to the block's first NT slots
// (tile after tile, so that the many unsplit tiles of an image fill whole
// lines), the records of a split tile to that tile's own CE slots after
// them, indexed by cell (so a split tile's records share lines too).
template <int GX, int NT, int CE>
__device__ __forceinline__ uint32_t rec_slot(int tx, int ty, int cell, bool whole) {
  const uint32_t t = (uint32_t)ty * GX + (uint32_t)tx;
  return whole ? t : (uint32_t)NT + t * (uint32_t)CE + (uint32_t)cell;
}

// The quadtree of one block, the four waves sharing each level's list.
// Uses only LDS data staged for the block; writes records to staging and
// tile masks.
//
// Every range is fitted by exactly one lane.  A level's moments come from
// one of two layouts:
//  - a list of more than 64 ranges is cut into groups of 64, dealt round the
//    four waves; a lane sums every row of its range;
//  - a list of at most 64 ranges is one group whose rows are spread over the
//    waves (and, when the list is short, over teams of lanes inside each
//    wave, reduced by DPP); the waves add their partial moments into LDS and,
//    after a barrier, one wave fits the whole list, a lane per range.
// The fit is phase 1 (Sec. 3); from level 2 on, the list holds the four
// children (Z order) of each range that failed the level above in four
// consecutive lanes, so the same lanes also decide the parent's Technique 1
// (Sec. 3.1-3.3) by DPP exchanges inside their quad.  Accepted ranges are
// written at once; failed ones are compacted (ballot prefix, one LDS atomic
// per wave) into the parent list of the next level.  A barrier ends each
// level.
template <int BMAX, int L, int GX, int GY, bool EXT>
__device__ __forceinline__ void process_block(const EncodeArgs& a, const LevelParams& P, const BlockGeo& bg,
                                              Lds<BMAX, L, GX, GY>& sm, uint32_t rot) {
  using G = Geo<BMAX, L, GX, GY>;
  // record cells per tile: B_min cells, or 2 x 2 cells when the tree goes on
  // to 2 x 2 (EXT), whose Morton codes are those of the B_min cells times 4
  constexpr int CE = EXT ? 4 * G::CELLS : G::CELLS;
  constexpr int CSH = EXT ? 2 : 0;
  constexpr int LOG_BMAX = Log2<BMAX>::value;
  const Region& rg = bg.rg;
  const int tid = threadIdx.x;
  unsigned long long* s_mask = sm.mask;
  uint4* const rec_base = a.staging + (uint64_t)bg.sblk * (uint64_t)(G::NT * (CE + 1));   // the block's record slots
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave - (int)rot) & 3;   // this wave's rank in the block

  // ranges in the current list (workgroup-uniform); level 1: the block's
  // tiles inside the image, listed by the kernel before its barrier
  int n = bg.gx * bg.gy;
  for (int lev = 1; lev <= L; ++lev) {
    const uint32_t* ppar = sm.par((lev - 1) & 1);   // parents of this level's ranges
    uint32_t* npar = sm.par(lev & 1);               // this level's failed ranges
    uint32_t* nfail = &sm.cnt[lev];                 // zeroed by the kernel
    const bool last = lev == L && !EXT;   // EXT: the 4 x 4 level is tested too
    const int B = BMAX >> (lev - 1);

    auto level_pass = [&](auto bconst) {
      constexpr int BB = decltype(bconst)::value;
      constexpr bool ALIGNED = BB >= 16;
      constexpr int RP = BB / 2;                           // row pairs of a range
      constexpr double NN = (double)(BB * BB);
      using W = Window<G, BB>;
      // 64 n^2 t of this level; a forced level accepts every range
      const double thr64 = last ? __builtin_inf() : 64.0 * NN * NN * (double)P.thr(lev - 1);

      // Fit, Technique 1, records and compaction for list entry e, lane =
      // e mod 64, given the range's moments in acc.
      auto finish = [&](int e, bool valid, uint32_t (&acc)[12]) {
        const RangeRef r = range_ref<BB, BMAX, G::BMIN>(sm.top, ppar, min(e, n - 1));
        if (P.identity_only) {   // every isometry scores as the identity: the fit keeps e = 0
#pragma unroll
          for (int j = 5; j < 12; ++j) acc[j] = acc[4];
        }
        const Fit1 f = fit_phase1_terms<BB>(acc, thr64);
        const int tx = r.xr >> LOG_BMAX, ty = r.yr >> LOG_BMAX;

        // ---- Technique 1 for the parent of this quad of children
        bool dead = false;   // the parent was stored by phase 2
        if constexpr (BB < BMAX) {
          if (P.phase2) {
            constexpr int LOGNB = 2 * Log2<BB>::value;
            int c1, c2, delta;
            phase2_consts(lev - 1, c1, c2, delta);
            const double thr2 = 400.0 * NN * NN * (double)P.thr(lev - 2);
            const int c = e & 3;
            const int m = r.m;
            int O = (int)((2u * acc[0] + (uint32_t)(BB * BB)) >> (LOGNB + 1));
            const int O0 = quad_bcast<0>(O), O1 = quad_bcast<1>(O), O2 = quad_bcast<2>(O);
            if (c == 3) O = 4 * m - O0 - O1 - O2;   // eq. (1)
            const double P0 = NN * (double)acc[4] - f.srsd;
            const double f1 = (double)(c1 * c1) * f.Q - (double)(40 * c1) * P0;
            const double f2 = (double)(c2 * c2) * f.Q - (double)(40 * c2) * P0;
            const bool use2 = f2 < f1;
            const double dm = (double)(O * (BB * BB) - (int)acc[0]);
            const double S = (use2 ? f2 : f1) + 400.0 * (f.R + dm * dm);
            const bool okc = (uint32_t)(O - m + delta) <= (uint32_t)(2 * delta) && (uint32_t)O <= 255u && S < thr2;
            const int all = quad_sum(okc ? 1 : 0);
            const int bits = quad_sum((use2 ? 1 : 0) << c);
            dead = valid && all == 4;
            if (dead && c == 0) {
              const int pxr = r.xr, pyr = r.yr;   // child 0 shares its parent's corner
              constexpr int PB = 2 * BB;
              const int PX = rg.X0 + pxr, PY = rg.Y0 + pyr;
              const int pdx = clampi(PX - PB / 2, 0, rg.W - 2 * PB);
              const int pdy = clampi(PY - PB / 2, 0, rg.H - 2 * PB);
              const int cell = r.cell << CSH;
              rec_base[rec_slot<GX, G::NT, CE>(tx, ty, cell, PB == BMAX)] =
                  make_record(PX, PY, pdx, pdy, lev - 2, 1, 0, bits, m, O0 - m, O1 - m, O2 - m);
              atomicOr(&s_mask[ty * GX + tx], 1ull << cell);
            }
          }
        }

        // ---- store accepted ranges; compact failures into the next list
        const bool live = valid && !dead;
        const bool fail = live && !f.accept;
        if (live && f.accept) {
          const W w(r, rg);
          const int cell = r.cell << CSH;
          rec_base[rec_slot<GX, G::NT, CE>(tx, ty, cell, BB == BMAX)] = make_record(rg.X0 + r.xr, rg.Y0 + r.yr, w.dx, w.dy, lev - 1, 0,
                                                                 (int)f.e, (int)f.k, (int)f.lum, 0, 0, 0);
          atomicOr(&s_mask[ty * GX + tx], 1ull << cell);
        }
        const uint64_t bal = __ballot(fail);
        if (!bal) return;
        const int first = (int)__builtin_ctzll(bal);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        const uint32_t ent = (uint32_t)r.xr | ((uint32_t)r.yr << 8) | ((uint32_t)r.cell << 16);
        if constexpr (EXT) {
          if (lev == L) {
            // failed 4 x 4 ranges go on to the 2 x 2 level, through the
            // global list (one atomic per wave)
            uint32_t base = 0;
            if (lane == first) base = atomicAdd(a.fine_count, (uint32_t)__popcll(bal));
            base = (uint32_t)__shfl((int)base, first);
            if (fail) {
              const int cell = r.cell << CSH;
              const uint64_t tg = rg.tg0 + (uint64_t)((uint32_t)ty * (uint32_t)rg.tiles_x + (uint32_t)tx);
              a.fine_list[base + rank] =
                  make_uint4((uint32_t)(rg.X0 + r.xr) | ((uint32_t)(rg.Y0 + r.yr) << 16),
                             (uint32_t)((rec_base - a.staging) + rec_slot<GX, G::NT, CE>(tx, ty, cell, false)), (uint32_t)tg,
                             f.lum | ((uint32_t)cell << 8));
            }
            return;
          }
        }
        uint32_t q0 = 0;
        if (lane == first) q0 = atomicAdd(nfail, (uint32_t)__popcll(bal));
        q0 = (uint32_t)__shfl((int)q0, first);
        if (fail) npar[q0 + rank] = ent | (f.lum << 24);
      };

      // A short list has its rows spread over the waves at the top level
      // (every block starts with one) and for ranges of 16 x 16 and larger;
      // smaller ranges take too few rows for the split to pay.
      constexpr bool TOP_SHORT = BB == BMAX && G::NT <= 64 && BB >= 8;
      constexpr bool SPLIT_OK = BB >= 8 && (BB == BMAX || BB >= 16);
      if (!TOP_SHORT && (n > 64 || !SPLIT_OK)) {
        // groups of 64 ranges, one lane per range over all its rows (lanes
        // beyond the list repeat its last range and store nothing)
        for (int g = wr; g * 64 < n; g += 4) {
          const int e = g * 64 + lane;
          const bool valid = e < n;
          const W w(range_ref<BB, BMAX, G::BMIN>(sm.top, ppar, min(e, n - 1)), rg);
          // dword-aligned row starts; every window row shares its byte shift
          const uint32_t* r0 = sm.img + (w.roff >> 2);
          const uint32_t* d0 = sm.h0 + (w.doff >> 2);
          const uint32_t* t0 = sm.h0t + (w.toff >> 2);
          const uint32_t shd = (uint32_t)w.doff & 3u, sht = (uint32_t)w.toff & 3u;
          constexpr int RW = G::TPITCH / 4, HW4 = G::HP / 4, TW4 = G::TP / 4;
          uint32_t acc[12];
#pragma unroll
          for (int j = 0; j < 12; ++j) acc[j] = 0u;
          // small ranges unrolled whole; larger ones a row pair at a time
          // (their loads would otherwise all be hoisted into registers)
          if constexpr (RP <= 2) {
#pragma unroll
            for (int i = 0; i < RP; ++i)
              accumulate_rows_sh<BB, ALIGNED>(r0 + i * RW, r0 + (BB - 1 - i) * RW, d0 + i * HW4,
                                              d0 + (BB - 1 - i) * HW4, t0 + i * TW4, t0 + (BB - 1 - i) * TW4, shd,
                                              sht, acc);
          } else {
#pragma unroll 1
            for (int i = 0; i < RP; ++i)
              accumulate_rows_sh<BB, ALIGNED>(r0 + i * RW, r0 + (BB - 1 - i) * RW, d0 + i * HW4,
                                              d0 + (BB - 1 - i) * HW4, t0 + i * TW4, t0 + (BB - 1 - i) * TW4, shd,
                                              sht, acc);
          }
          finish(e, valid, acc);
        }
      } else {
        // one short list: rows spread over sw waves and over teams of tin
        // lanes (tin x sw <= RP, powers of two), partial sums added in LDS
        int p2 = 1;
        while (p2 < n) p2 <<= 1;
        const int tin = min(RP, 64 / p2);
        const int sw = min(4, RP / tin);
        if (wr < sw) {
          const int logt = __builtin_ctz((unsigned)tin);
          const int e = lane >> logt, t = lane & (tin - 1);
          const W w(range_ref<BB, BMAX, G::BMIN>(sm.top, ppar, min(e, n - 1)), rg);
          const int i0 = wr * tin + t, step = sw * tin;
          constexpr int RW = G::TPITCH / 4, HW4 = G::HP / 4, TW4 = G::TP / 4;
          const uint32_t shd = (uint32_t)w.doff & 3u, sht = (uint32_t)w.toff & 3u;
          const uint32_t* ra = sm.img + (w.roff >> 2) + i0 * RW;
          const uint32_t* rb = sm.img + (w.roff >> 2) + (BB - 1 - i0) * RW;
          const uint32_t* da = sm.h0 + (w.doff >> 2) + i0 * HW4;
          const uint32_t* db = sm.h0 + (w.doff >> 2) + (BB - 1 - i0) * HW4;
          const uint32_t* ta = sm.h0t + (w.toff >> 2) + i0 * TW4;
          const uint32_t* tb = sm.h0t + (w.toff >> 2) + (BB - 1 - i0) * TW4;
          uint32_t acc[12];
#pragma unroll
          for (int j = 0; j < 12; ++j) acc[j] = 0u;
          for (int i = i0; i < RP; i += step) {
            accumulate_rows_sh<BB, ALIGNED>(ra, rb, da, db, ta, tb, shd, sht, acc);
            ra += step * RW;
            rb -= step * RW;
            da += step * HW4;
            db -= step * HW4;
            ta += step * TW4;
            tb -= step * TW4;
          }
          team_reduce(acc, tin);
          if (e < n && t == 0) {
#pragma unroll
            for (int j = 0; j < 12; ++j) atomicAdd(sm.part(j) + e, acc[j]);
          }
        }
        __syncthreads();   // the list's moments are complete
        if (wr == 0) {
          const bool valid = lane < n;
          uint32_t acc[12];
#pragma unroll
          for (int j = 0; j < 12; ++j) {
            acc[j] = lane < G::PW ? sm.part(j)[lane] : 0u;   // zero beyond the list
            // zero again for the next short list (with SHARE there is none,
            // and the words go on to hold this level's failed ranges)
            if (!G::SHARE && lane < G::PW) sm.part(j)[lane] = 0u;
          }
          finish(lane, valid, acc);
        }
      }
    };
    if constexpr (BMAX >= 32) { if (B == 32) level_pass(std::integral_constant<int, 32>{}); }
    if constexpr (BMAX >= 16 && G::BMIN <= 16) { if (B == 16) level_pass(std::integral_constant<int, 16>{}); }
    if constexpr (BMAX >= 8 && G::BMIN <= 8) { if (B == 8) level_pass(std::integral_constant<int, 8>{}); }
    if constexpr (G::BMIN <= 4) { if (B == 4) level_pass(std::integral_constant<int, 4>{}); }
    __syncthreads();   // the next level's parents and their count are complete
    n = (int)(4u * *nfail);
    if (last || n == 0) break;
  }

  // ---- publish the block's tiles' occupancy masks (complete after the
  // barrier that ended the last level)
  for (int t = tid; t < G::NT; t += 256) {
    const int tx = t & (GX - 1), ty = t >> G::LOG_GX;
    if (tx < bg.gx && ty < bg.gy)
      a.masks[rg.tg0 + (uint64_t)((uint32_t)ty * (uint32_t)rg.tiles_x + (uint32_t)tx)] = s_mask[t];
  }
}

template <int BMAX, int L, int GX, int GY>
__device__ __forceinline__ void block_start(const BlockGeo& bg, Lds<BMAX, L, GX, GY>& sm, int tid) {
  using G = Geo<BMAX, L, GX, GY>;
  for (int t = tid; t < G::NT; t += 256) sm.mask[t] = 0ull;
  for (int t = tid; t < 12 * G::PW; t += 256) sm.part(0)[t] = 0u;
  if (tid <= L) sm.cnt[tid] = 0u;
  // level-1 list: the block's tiles inside the image, row-major (gx gy <= NT <= 256)
  if (tid < bg.gx * bg.gy) {
    const int ty = tid / bg.gx, tx = tid - ty * bg.gx;
    sm.top[tid] = (uint32_t)(tx * BMAX) | ((uint32_t)(ty * BMAX) << 8);
  }
}

template <int BMAX, int L, int GX, int GY, bool EXT>
__global__ __launch_bounds__(256) void mns_tiles_kernel(EncodeArgs a) {
  using G = Geo<BMAX, L, GX, GY>;
  __shared__ Lds<BMAX, L, GX, GY> sm;
  const int tid = threadIdx.x;
  // XCD-aware order: consecutive logical blocks share an XCD (and its L2).
  const uint32_t per = (a.n_wg + 7u) >> 3;
  const uint32_t wg = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  if (wg >= a.n_wg) return;
  const BlockGeo bg = block_geo<BMAX, GX, GY>(a.blocks[wg]);
  Stage<G> st;
  st.load(bg, tid);
  st.store(bg, tid, sm.img, sm.h0, sm.h0t);
  block_start(bg, sm, tid);
  const LevelParams P = level_params(a, wg);
  __syncthreads();
  process_block<BMAX, L, GX, GY, EXT>(a, P, bg, sm, wg & 3u);
}

// One lane per logical workgroup: find its image (binary search over the
// sorted first-workgroup indices) and its block of tiles.
__global__ __launch_bounds__(256) void block_prep_kernel(const ImgDev* imgs, uint32_t n_imgs, uint32_t n_wg,
                                                        int b_max, int gx, int gy, BlockDesc* blocks) {
  const uint32_t wg = blockIdx.x * 256u + threadIdx.x;
  if (wg >= n_wg) return;
  int lo = 0, hi = (int)n_imgs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (imgs[mid].wg_first <= wg) lo = mid; else hi = mid - 1;
  }
  const ImgDev im = imgs[lo];
  const uint32_t local = wg - im.wg_first;
  const uint32_t gyi = local / im.groups_x, gxi = local - gyi * im.groups_x;
  const uint32_t tx0 = gxi * (uint32_t)gx, ty0 = gyi * (uint32_t)gy;
  BlockDesc d;
  d.data = im.data;
  d.tg0 = im.tile_first + (uint64_t)ty0 * im.tiles_x + tx0;
  d.stride = im.stride;
  d.wh = (im.width - 1u) | ((im.height - 1u) << 16);
  d.t0 = tx0 | (ty0 << 16);
  d.sblk = wg;
  blocks[wg] = d;
}

}  // namespace

// ---------------------------------------------------------------- launchers
template <int BMAX, int L, int GX, int GY, bool EXT = false>
static hipError_t launch_one(const EncodeArgs& a, hipStream_t s) {
  const uint32_t grid = ((a.n_wg + 7u) >> 3) << 3;
  hipLaunchKernelGGL((mns_tiles_kernel<BMAX, L, GX, GY, EXT>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Tile shapes (GX x GY top tiles per workgroup) instantiated per
// (b_max, levels); the first entry is the default.
#define FE_SHAPES(X)                                                                    \
  X(4, 1, 16, 16) X(4, 1, 32, 8)                                                        \
  X(8, 1, 16, 8) X(8, 1, 8, 8) X(8, 2, 8, 8) X(8, 2, 16, 4) X(8, 2, 4, 4) X(8, 2, 8, 4)  \
  X(16, 1, 8, 4) X(16, 1, 4, 4) X(16, 2, 8, 4) X(16, 2, 4, 4) X(16, 2, 8, 2)             \
  X(16, 3, 8, 8) X(16, 3, 8, 7) X(16, 3, 8, 6) X(16, 3, 8, 4) X(16, 3, 4, 4)             \
  X(16, 3, 16, 2) X(16, 3, 8, 2) X(16, 3, 4, 2) X(16, 3, 16, 4)                         \
  X(32, 1, 4, 2) X(32, 1, 2, 2) X(32, 2, 4, 2) X(32, 2, 2, 2) X(32, 3, 4, 2)             \
  X(32, 3, 2, 2) X(32, 4, 4, 4) X(32, 4, 4, 2) X(32, 4, 2, 2) X(32, 4, 8, 1) X(32, 4, 4, 1)

int encode_shapes(int b_max, int levels, TileShape* out, int max_out) {
  int k = 0;
#define FE_LIST(BM, LV, GX_, GY_) \
  if (b_max == BM && levels == LV && k < max_out) out[k++] = TileShape{GX_, GY_};
  FE_SHAPES(FE_LIST)
#undef FE_LIST
  return k;
}

hipError_t launch_mns_tiles(int b_max, int levels, TileShape shape, const EncodeArgs& a, hipStream_t s) {
#define FE_LAUNCH(BM, LV, GX_, GY_) \
  if (b_max == BM && levels == LV && shape.gx == GX_ && shape.gy == GY_) return launch_one<BM, LV, GX_, GY_>(a, s);
  FE_SHAPES(FE_LAUNCH)
#undef FE_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_mns_tiles_ext(int b_max, int levels, TileShape shape, const EncodeArgs& a, hipStream_t s) {
  // the default shapes of 16 -> 4, 8 -> 4 and 4 -> 4, and the smallest of
  // the first two (for calls with few tiles)
  if (b_max == 16 && levels == 3 && shape.gx == 8 && shape.gy == 8) return launch_one<16, 3, 8, 8, true>(a, s);
  if (b_max == 16 && levels == 3 && shape.gx == 4 && shape.gy == 2) return launch_one<16, 3, 4, 2, true>(a, s);
  if (b_max == 8 && levels == 2 && shape.gx == 8 && shape.gy == 8) return launch_one<8, 2, 8, 8, true>(a, s);
  if (b_max == 8 && levels == 2 && shape.gx == 4 && shape.gy == 4) return launch_one<8, 2, 4, 4, true>(a, s);
  if (b_max == 4 && levels == 1 && shape.gx == 16 && shape.gy == 16) return launch_one<4, 1, 16, 16, true>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_block_prep(const ImgDev* imgs, uint32_t n_imgs, uint32_t n_wg, int b_max, int gx, int gy,
                             BlockDesc* blocks, hipStream_t s) {
  if (n_wg == 0) return hipSuccess;
  hipLaunchKernelGGL(block_prep_kernel, dim3((n_wg + 255) / 256), dim3(256), 0, s, imgs, n_imgs, n_wg, b_max, gx,
                     gy, blocks);
  return hipGetLastError();
}

}  // namespace fe
