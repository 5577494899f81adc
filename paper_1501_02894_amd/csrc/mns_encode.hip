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
//      cut into passes of 64 lanes, a team of T lanes per range, and the
//      passes are dealt round the four waves: the team sums packed-u8 dot
//      products (v_dot4_u32_u8)
//      over row pairs of the range and of the domain window / its transpose,
//      giving Sum r, Sum r^2, Sum d, Sum d^2 and the 8 isometric Sum r T_e(d);
//      a DPP butterfly leaves the totals in every lane, and every lane fits
//      (e, k, m) exactly in fp64 (Sec. 3).
//   3. phase 2 (Sec. 3.1-3.3): in the same pass, the parents that failed at
//      level l-1 are decided from the identity moments of their four
//      children, which are exactly the level-l ranges just computed.
//   4. accepted ranges are written as 16-byte records into per-tile slots
//      indexed by the Morton code of their top-left B_min cell; failed ranges
//      are compacted (wave ballot + prefix, one LDS atomic per pass) into the
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
  static constexpr int BMIN = BMAX >> (L - 1);
  static constexpr int NT = GX * GY;                          // tiles per workgroup
  static constexpr int LOG_GX = Log2<GX>::value;
  static constexpr int CELLS = 1 << (2 * (L - 1));
  // failed ranges of one level, at most NT 4^(L-2) (level L-1)
  static constexpr int PCAP = NT * CELLS / 4 > 0 ? NT * CELLS / 4 : 1;
  static constexpr int TW = GX * BMAX, TH = GY * BMAX;        // tile block in pixels
  static constexpr int TPITCH = TW + 4;                       // tile pixel row pitch (bytes)
  static constexpr int RWA = ((GX + 1) * BMAX + 6 + 7) & ~7;  // region width bound (px)
  static constexpr int RHA = (GY + 1) * BMAX + 8;             // region height bound (px)
  static constexpr int HW = RWA / 2, HH = RHA / 2;            // H0 region bounds
  static constexpr int HP = HW + 8;                           // H0 row pitch
  static constexpr int TP = ((HH + 3) & ~3) + 8;              // H0^T row pitch
  static constexpr int IMG_W = TH * TPITCH / 4 + 4;           // dwords
  static constexpr int HH4 = (HH + 3) & ~3;                   // H0 rows, multiple of 4
  static constexpr int H0_W = HH4 * HP / 4 + 4;
  static constexpr int H0T_W = HW * TP / 4 + 4;
  static_assert(NT % 4 == 0 && NT <= 256, "tiles per workgroup: a multiple of 4, at most one per lane");
};

struct Region {
  int W, H;            // image sides
  int ax0, ay0;        // H0 region origin (pixels), multiples of 8
  int X0, Y0;          // tile block origin (pixels)
  int tiles_x;
  uint64_t tg0;        // global index of the block's first tile
};

// List entry: bits 0-7 cell x, 8-15 cell y (in B_min units inside the tile),
// bits 16+ tile index t = tly * GX + tlx inside the workgroup's block.
template <int BMAX, int BMIN, int LOG_GX>
__device__ __forceinline__ void range_xy(uint32_t meta, const Region& r, int& X, int& Y) {
  const int t = (int)(meta >> 16);
  X = r.X0 + (t & ((1 << LOG_GX) - 1)) * BMAX + (int)(meta & 0xffu) * BMIN;
  Y = r.Y0 + (t >> LOG_GX) * BMAX + (int)((meta >> 8) & 0xffu) * BMIN;
}

template <int LOG_GX>
__device__ __forceinline__ uint64_t tile_global(uint32_t meta, const Region& r) {
  const int t = (int)(meta >> 16);
  return r.tg0 + (uint64_t)((uint32_t)(t >> LOG_GX) * (uint32_t)r.tiles_x + (uint32_t)(t & ((1 << LOG_GX) - 1)));
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ int morton(uint32_t meta) {
  const int cx = meta & 0xff, cy = (meta >> 8) & 0xff;
  int code = 0;
#pragma unroll
  for (int bit = 0; bit < 3; ++bit) {
    code |= ((cx >> bit) & 1) << (2 * bit);
    code |= ((cy >> bit) & 1) << (2 * bit + 1);
  }
  return code;
}

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

// Region staging.  A group is 8 x 8 pixels of the region (column group c8,
// rows 8 g .. 8 g + 7), i.e. a 4 x 4 block of H0; lane `tid` owns groups
// tid + 256 * it.  H0 is written as dwords, and its transpose as dwords
// after a 4 x 4 byte transpose in registers.
template <class G>
struct Stage {
  static constexpr int NC8 = G::RWA / 8;
  static constexpr int NG = (G::HH4 / 4 * NC8 + 255) / 256;

  __device__ __forceinline__ static void run(const BlockGeo& b, int tid, uint32_t* s_img, uint32_t* s_h0,
                                             uint32_t* s_h0t) {
#pragma unroll
    for (int it = 0; it < NG; ++it) {
      const int idx = tid + 256 * it;
      const int g = idx / NC8, c8 = idx - g * NC8;
      if (4 * g >= b.hrows || c8 >= b.n8) continue;
      const int x = b.rg.ax0 + 8 * c8;
      uint32_t v[8][2];
      const uint8_t* row0 = b.data + (size_t)(b.rg.ay0 + 8 * g) * b.stride + x;
      if constexpr (G::BMAXV >= 16) {
        // the region spans multiples of 8 pixels inside the image in both
        // directions, so every group is whole
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const gu32* p = (const gu32*)(row0 + (size_t)r * b.stride);
          v[r][0] = p[0];
          v[r][1] = p[1];
        }
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          v[r][0] = v[r][1] = 0u;
          if (8 * g + r < 2 * b.hrows) {
            const gu32* p = (const gu32*)(row0 + (size_t)r * b.stride);
            if (x + 8 <= b.rg.W) {
              v[r][0] = p[0];
              v[r][1] = p[1];
            } else if (x < b.rg.W) {
              v[r][0] = p[0];
            }
          }
        }
      }
      // tile pixels.  For b_max >= 8 the tile block starts at a multiple of
      // 8 pixels from the region origin in both directions and spans a
      // multiple of 8, so a group lies wholly inside or outside it; for
      // b_max = 4 tile edges are multiples of 4 and rows/halves are tested.
      if constexpr (G::BMAXV >= 8) {
        const int gy0 = b.rg.ay0 + 8 * g;
        if (gy0 >= b.rg.Y0 && gy0 < b.ty_end && x >= b.rg.X0 && x < b.tx_end) {
          uint32_t* dst = s_img + (gy0 - b.rg.Y0) * (G::TPITCH / 4) + ((x - b.rg.X0) >> 2);
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            dst[r * (G::TPITCH / 4)] = v[r][0];
            dst[r * (G::TPITCH / 4) + 1] = v[r][1];
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int y = b.rg.ay0 + 8 * g + r;
          if (y < b.rg.Y0 || y >= b.ty_end) continue;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int xx = x + 4 * h;
            if (xx >= b.rg.X0 && xx < b.tx_end)
              s_img[(y - b.rg.Y0) * (G::TPITCH / 4) + ((xx - b.rg.X0) >> 2)] = v[r][h];
          }
        }
      }
      // 2x2 means: H0 rows 4g .. 4g+3, columns 4 c8 .. 4 c8 + 3
      uint32_t hrow[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        hrow[q] = mean2x2_x4(v[2 * q][0], v[2 * q][1], v[2 * q + 1][0], v[2 * q + 1][1]);
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
  uint32_t par[2][G::PCAP];        // failed ranges of two consecutive levels, meta | m << 24
  uint32_t cnt[L + 1];             // per level: ranges that failed (parents of the next list)
  unsigned long long mask[G::NT];
};

// Lane `src` of the wave's value v.
__device__ __forceinline__ int lane_read(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }

// VALU instructions of one level pass of the compiled kernel by range side:
// per moment iteration (one row pair of a range per lane) and per pass (the
// fits, phase 2, record stores and compaction, whatever T is).
template <int BB>
struct PassCost;
template <>
struct PassCost<32> { static constexpr int it = 250, pass = 220; };
template <>
struct PassCost<16> { static constexpr int it = 127, pass = 200; };
template <>
struct PassCost<8> { static constexpr int it = 79, pass = 300; };
template <>
struct PassCost<4> { static constexpr int it = 49, pass = 280; };

// Team size T (lanes per range, a power of two up to min(BB/2, 16)) for a
// workgroup list of n ranges of side BB.  The top level splits its tiles
// evenly over the four waves and fills their lanes.  Lower levels take the T
// of least VALU work in total, ceil(n T / 64) passes of ceil(BB / 2T)
// moment iterations plus the per-pass work: small teams when the list is
// long, large ones when a short list would otherwise leave lanes idle.
template <int BB>
__device__ __forceinline__ int team_size(int n, bool top) {
  constexpr int TMAX = BB / 2 < 16 ? BB / 2 : 16;
  if (top) {
    const int nw = (n + 3) >> 2;
    int T = 1;
    while (T < TMAX && nw * T * 2 <= 64) T *= 2;
    return T;
  }
  int best_t = 1, best = 0x7fffffff;
  for (int T = 1, lg = 0; T <= TMAX; T *= 2, ++lg) {
    const int c = ((n * T + 63) >> 6) * ((BB / 2 + T - 1) / T * PassCost<BB>::it + PassCost<BB>::pass + 12 * lg);
    if (c < best) {
      best = c;
      best_t = T;
    }
  }
  return best_t;
}

// The quadtree of one block, the four waves sharing each level's list.  Uses
// only LDS data staged for the block; writes records to staging and tile
// masks.
//
// Per level the list is cut into passes of 64 lanes, a team of T lanes per
// range, and pass p goes to wave (p + rot) mod 4: the team accumulates the
// range's moments and reduces them so that every lane of the team holds the
// totals; every lane then fits the range.  From level 2 on the list holds
// the four children (Z order) of each range that failed the level above, in
// consecutive teams of one pass (4T divides 64), so the same pass also runs
// the parent's phase 2 (Technique 1) across the four teams.  Accepted ranges
// are written at once; failed ones are compacted (ballot prefix, one LDS
// atomic per pass) into the parent list of the next level, whose entry e is
// then child e mod 4 of parent e / 4.  A barrier ends each level.
// Record slot of Morton cell `cell` of tile t (row-major in a block of GX
// tiles per row) inside its block: one row of the block's tiles at a time,
// and inside a row cell-major, so that the records of one cell of a tile
// row are adjacent (the level pass writes them together) and a tile row's
// records sit in one span (the ordering kernel reads them together).
template <int GX>
__device__ __forceinline__ uint32_t rec_slot(uint32_t t, int cell, int cells) {
  return (t / GX) * (uint32_t)(GX * cells) + (uint32_t)cell * GX + t % GX;
}

template <int BMAX, int L, int GX, int GY, bool EXT>
__device__ __forceinline__ void process_block(const EncodeArgs& a, const BlockGeo& bg, Lds<BMAX, L, GX, GY>& sm,
                                              uint32_t rot) {
  using G = Geo<BMAX, L, GX, GY>;
  // record cells per tile: B_min cells, or 2 x 2 cells when the tree goes on
  // to 2 x 2 (EXT), whose Morton codes are those of the B_min cells times 4
  constexpr int CE = EXT ? 4 * G::CELLS : G::CELLS;
  constexpr int CSH = EXT ? 2 : 0;
  const Region& rg = bg.rg;
  const int gx = bg.gx, gy = bg.gy;
  const int tid = threadIdx.x;
  const uint32_t* s_img = sm.img;
  const uint32_t* s_h0 = sm.h0;
  const uint32_t* s_h0t = sm.h0t;
  unsigned long long* s_mask = sm.mask;
  const uint64_t slot0 = (uint64_t)bg.sblk * (uint64_t)(G::NT * CE);   // the block's record slots
  const int wave = tid >> 6, lane = tid & 63;
  const int p0 = (wave - (int)rot) & 3;   // this wave's first pass of a level

  // ranges in the current list (workgroup-uniform); level 1: the block's
  // tiles inside the image, listed by the kernel before its barrier
  int n = gx * gy;
  for (int lev = 1; lev <= L; ++lev) {
    const uint32_t* ppar = sm.par[(lev - 1) & 1];   // parents of this level's ranges
    uint32_t* npar = sm.par[lev & 1];               // this level's failed ranges
    uint32_t* nfail = &sm.cnt[lev];                 // zeroed by the kernel
    const bool last = lev == L && !EXT;   // EXT: the 4 x 4 level is tested too
    const uint32_t thr = last ? 0u : a.thr[lev - 1];
    const int B = BMAX >> (lev - 1);

    auto level_pass = [&](auto bconst) {
      constexpr int BB = decltype(bconst)::value;
      constexpr bool ALIGNED = BB >= 16;
      const int T = team_size<BB>(n, BB == BMAX);
      const int logT = __builtin_ctz((unsigned)T);
      const int passes = (n * T + 63) >> 6;
      for (int p = p0; p < passes; p += 4) {
        const int idx = p * 64 + lane;
        const int e = idx >> logT, t = idx & (T - 1);
        const bool valid = e < n;
        // ---- moments of range e (the team's rows t, t + T, ...)
        uint32_t acc[12];
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[j] = 0u;
        uint32_t meta = 0, pe = 0;
        int X = 0, Y = 0;
        if (valid) {
          if constexpr (BB == BMAX) {
            meta = sm.top[e];
          } else {
            // child e mod 4 (Z order) of the failed parent e / 4
            constexpr uint32_t side = (uint32_t)(BB / G::BMIN);   // in B_min cells
            pe = ppar[e >> 2];
            const uint32_t c = (uint32_t)e & 3u;
            meta = (pe & 0x00ff0000u) | ((((pe >> 8) & 0xffu) + (c >> 1) * side) << 8) | ((pe & 0xffu) + (c & 1u) * side);
          }
          range_xy<BMAX, G::BMIN, G::LOG_GX>(meta, rg, X, Y);
          const int dx = clampi(X - BB / 2, 0, rg.W - 2 * BB);
          const int dy = clampi(Y - BB / 2, 0, rg.H - 2 * BB);
          const int rx = X - rg.X0, ry = Y - rg.Y0;
          const int wx = (dx - rg.ax0) >> 1, wy = (dy - rg.ay0) >> 1;
          for (int i = t; i < BB / 2; i += T)
            accumulate_row_pair<BB, ALIGNED>(s_img, ry * G::TPITCH + rx, G::TPITCH, s_h0, wy * G::HP + wx,
                                             G::HP, s_h0t, wx * G::TP + wy, G::TP, i, acc);
        }
        team_reduce(acc, T);   // butterfly: every lane of the team holds the totals
        if (a.identity_only) {  // every isometry scores as the identity: the fit keeps e = 0
#pragma unroll
          for (int j = 5; j < 12; ++j) acc[j] = acc[4];
        }
        const uint32_t fit = fit_phase1<BB>(acc, last, thr);

        // ---- phase 2 of the parent of this group of four children
        bool dead = false;   // the parent was stored by phase 2
        if constexpr (BB < BMAX) {
          if (a.phase2) {
            constexpr int LOGNB = 2 * Log2<BB>::value;
            constexpr double NB = (double)(BB * BB);
            int c1, c2, delta;
            phase2_consts(lev - 1, c1, c2, delta);
            const double thr2 = (400.0 * NB * NB) * (double)a.thr[lev - 2];
            const int c = e & 3;
            const int g0 = lane - c * T;               // lane of child 0 (same t)
            const int m = (int)(pe >> 24);
            int O = (int)((2u * acc[0] + (uint32_t)(BB * BB)) >> (LOGNB + 1));
            const int O0 = lane_read(O, g0), O1 = lane_read(O, g0 + T), O2 = lane_read(O, g0 + 2 * T);
            if (c == 3) O = 4 * m - O0 - O1 - O2;   // eq. (1)
            const double dsr = (double)acc[0], dsd = (double)acc[2];
            const double Q = NB * (double)acc[3] - dsd * dsd;
            const double P = NB * (double)acc[4] - dsr * dsd;
            const double R = NB * (double)acc[1] - dsr * dsr;
            const double f1 = (double)(c1 * c1) * Q - (double)(40 * c1) * P;
            const double f2 = (double)(c2 * c2) * Q - (double)(40 * c2) * P;
            const bool use2 = f2 < f1;
            const double dm = (double)O * NB - dsr;
            const double S = (use2 ? f2 : f1) + 400.0 * R + 400.0 * (dm * dm);
            const bool okc = valid && O - m <= delta && m - O <= delta && O >= 0 && O <= 255 && S < thr2;
            const uint64_t okb = __ballot(okc), u2b = __ballot(valid && use2);
            const uint64_t pat = 1ull | (1ull << T) | (1ull << (2 * T)) | (1ull << (3 * T));
            dead = valid && ((okb >> g0) & pat) == pat;
            if (dead && c == 0 && t == 0) {
              const uint64_t ub = u2b >> g0;
              const int bits = (int)((ub & 1ull) | (((ub >> T) & 1ull) << 1) | (((ub >> (2 * T)) & 1ull) << 2) |
                                     (((ub >> (3 * T)) & 1ull) << 3));
              const uint32_t pmeta = pe & 0x00ffffffu;
              int PX, PY;
              range_xy<BMAX, G::BMIN, G::LOG_GX>(pmeta, rg, PX, PY);
              constexpr int PB = 2 * BB;
              const int pdx = clampi(PX - PB / 2, 0, rg.W - 2 * PB);
              const int pdy = clampi(PY - PB / 2, 0, rg.H - 2 * PB);
              const int cell = morton(pmeta) << CSH;
              a.staging[slot0 + rec_slot<GX>((pmeta >> 16) & 0xffu, cell, CE)] =
                  make_record(PX, PY, pdx, pdy, lev - 2, 1, 0, bits, m, O0 - m, O1 - m, O2 - m);
              atomicOr(&s_mask[pmeta >> 16], 1ull << cell);
            }
          }
        }

        // ---- store accepted ranges; compact failures into the next lists
        const bool lead = valid && t == 0 && !dead;
        bool fail = false;
        if (lead) {
          if (fit & kFitAccept) {
            const int dx = clampi(X - BB / 2, 0, rg.W - 2 * BB);
            const int dy = clampi(Y - BB / 2, 0, rg.H - 2 * BB);
            const int cell = morton(meta) << CSH;
            a.staging[slot0 + rec_slot<GX>((meta >> 16) & 0xffu, cell, CE)] =
                make_record(X, Y, dx, dy, lev - 1, 0, (int)((fit >> 11) & 7u), (int)((fit >> 8) & 7u),
                            (int)(fit & 0xffu), 0, 0, 0);
            atomicOr(&s_mask[meta >> 16], 1ull << cell);
          } else {
            fail = true;
          }
        }
        const uint64_t bal = __ballot(fail);
        if constexpr (EXT) {
          if (lev == L) {
            // failed 4 x 4 ranges go on to the 2 x 2 level, through the
            // global list (one atomic per wave)
            if (bal) {
              const int first = (int)__builtin_ctzll(bal);
              uint32_t base = 0;
              if (lane == first) base = atomicAdd(a.fine_count, (uint32_t)__popcll(bal));
              base = (uint32_t)__shfl((int)base, first);
              if (fail) {
                const uint32_t q = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                const int cell = morton(meta) << CSH;
                a.fine_list[q] = make_uint4((uint32_t)X | ((uint32_t)Y << 16),
                                            (uint32_t)(slot0 + rec_slot<GX>((meta >> 16) & 0xffu, cell, CE)),
                                            (uint32_t)tile_global<G::LOG_GX>(meta, rg),
                                            (fit & 0xffu) | ((uint32_t)cell << 8));
              }
            }
            continue;
          }
        }
        if (bal) {
          const int first = (int)__builtin_ctzll(bal);
          uint32_t q0 = 0;
          if (lane == first) q0 = atomicAdd(nfail, (uint32_t)__popcll(bal));
          q0 = (uint32_t)__shfl((int)q0, first);
          if (fail)
            npar[q0 + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] =
                meta | ((fit & 0xffu) << 24);
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
  for (int t = tid; t < G::NT; t += 256)
    if ((t & (GX - 1)) < gx && (t >> G::LOG_GX) < gy) a.masks[tile_global<G::LOG_GX>((uint32_t)t << 16, rg)] = s_mask[t];
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
  Stage<G>::run(bg, tid, sm.img, sm.h0, sm.h0t);
  for (int t = tid; t < G::NT; t += 256) sm.mask[t] = 0ull;
  if (tid <= L) sm.cnt[tid] = 0u;
  // level-1 list: the block's tiles inside the image, row-major (gx gy <= NT <= 256)
  if (tid < bg.gx * bg.gy) sm.top[tid] = (uint32_t)((tid / bg.gx) * GX + tid % bg.gx) << 16;
  __syncthreads();
  process_block<BMAX, L, GX, GY, EXT>(a, bg, sm, wg & 3u);
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
  X(16, 3, 8, 8) X(16, 3, 8, 4) X(16, 3, 4, 4) X(16, 3, 16, 2) X(16, 3, 8, 2)            \
  X(16, 3, 4, 2) X(16, 3, 16, 4)                                                        \
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
