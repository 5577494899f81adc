// Iterated decoding (Sec. 1: the stored contractive maps are applied to any
// start image until their attractor is reached).  Jacobi iteration: every
// pixel of iterate t+1 is computed from iterate t, ping-ponging two images.
//
// One wave per transform.  A phase-1 transform covers B x B pixels; lane l
// handles pixels p = l, l + 64, ...: it forms the domain value feeding p --
// the round-half-up 2 x 2 mean of the iterate at the isometry's source
// position -- the wave sums those values (the source positions are a
// permutation of the domain, so the sum is Sum d), and each lane writes
// clamp(floor((k (n d_p - Sum d) + 8 n m + 4 n) / (8 n)), 0, 255).
// A phase-2 transform gives each of its four sub-blocks a 16-lane row with
// the sub-block's own co-centred domain, contrast c/20 and luminance O_c
// (O_3 from eq. (1), Sec. 3.3).
#include "fe_device.h"
#include "fe_internal.h"

namespace fe {
namespace {

struct Fields {
  int x, y, dx, dy, level, flags, iso, s_idx, lum, d0, d1, d2;
};

__device__ __forceinline__ Fields unpack(uint4 w) {
  Fields f;
  f.x = (int)(w.x & 0xffffu);
  f.y = (int)(w.x >> 16);
  f.dx = (int)(w.y & 0xffffu);
  f.dy = (int)(w.y >> 16);
  f.level = (int)(w.z & 0xffu);
  f.flags = (int)((w.z >> 8) & 0xffu);
  f.iso = (int)((w.z >> 16) & 0xffu);
  f.s_idx = (int)(w.z >> 24);
  f.lum = (int)(w.w & 0xffu);
  f.d0 = (int)(int8_t)((w.w >> 8) & 0xffu);
  f.d1 = (int)(int8_t)((w.w >> 16) & 0xffu);
  f.d2 = (int)(int8_t)(w.w >> 24);
  return f;
}

__device__ __forceinline__ int log2i(int v) { return 31 - __builtin_clz((unsigned)v); }

// Source position of pixel (i, j) under isometry e (table of fe.h).
__device__ __forceinline__ void iso_src(int e, int i, int j, int B, int& si, int& sj) {
  int a = i, b = j;
  if (e & 4) { a = j; b = i; }
  const bool flip_first = (e & 4) ? (e & 1) : (e & 2);
  const bool flip_second = (e & 4) ? (e & 2) : (e & 1);
  si = flip_first ? B - 1 - a : a;
  sj = flip_second ? B - 1 - b : b;
}

__device__ __forceinline__ int mean4(const uint8_t* img, int W, int x, int y) {
  const uint8_t* p = img + (size_t)y * W + x;
  return (p[0] + p[1] + p[W] + p[W + 1] + 2) >> 2;
}

// Non-zero when a transform cannot be applied inside the image.
__device__ __forceinline__ bool bad_record(const Fields& f, int W, int H, int bmax) {
  if (f.flags > 1 || bmax < 4) return true;
  if (f.level > 3) return true;
  const int B = bmax >> f.level;
  if (B < 2 || (f.x % B) || (f.y % B) || f.x + B > W || f.y + B > H) return true;
  if (f.flags == 0) {
    if (f.iso > 7 || f.s_idx > 7) return true;
    if (f.dx + 2 * B > W || f.dy + 2 * B > H) return true;
    if (f.d0 || f.d1 || f.d2) return true;
    return false;
  }
  if (B < 4 || f.level > 2 || f.iso != 0 || f.s_idx > 15) return true;
  const int O0 = f.lum + f.d0, O1 = f.lum + f.d1, O2 = f.lum + f.d2;
  const int O3 = 4 * f.lum - O0 - O1 - O2;
  if (O0 < 0 || O0 > 255 || O1 < 0 || O1 > 255 || O2 < 0 || O2 > 255 || O3 < 0 || O3 > 255) return true;
  return W < B || H < B;
}

__global__ __launch_bounds__(256) void check_kernel(DecodeArgs a, uint32_t* bad) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  if (bad_record(unpack(a.recs[i]), (int)a.width, (int)a.height, (int)a.b_max)) atomicAdd(bad, 1u);
}

// Zoom (the maps are resolution independent, Sec. 1): check each transform
// against the native image, then write it with range and domain origins
// multiplied by z.  Levels, contrasts and luminances do not change; the
// result is decoded as a z W x z H image with top blocks of z b_max, where
// the co-centred domains stay co-centred (the clamp commutes with the
// scaling).  A transform that fails the native check is counted and written
// with its fields masked, never decoded.
__global__ __launch_bounds__(256) void zoom_kernel(DecodeArgs a, uint32_t z, uint4* __restrict__ out,
                                                   uint32_t* bad) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const uint4 w = a.recs[i];
  if (bad_record(unpack(w), (int)a.width, (int)a.height, (int)a.b_max)) atomicAdd(bad, 1u);
  const uint32_t x = (w.x & 0xffffu) * z, y = (w.x >> 16) * z;
  const uint32_t dx = (w.y & 0xffffu) * z, dy = (w.y >> 16) * z;
  out[i] = make_uint4((x & 0xffffu) | ((y & 0xffffu) << 16), (dx & 0xffffu) | ((dy & 0xffffu) << 16), w.z, w.w);
}

// 16 bytes per lane: one 16-byte copy when both pointers allow it, else
// byte by byte.
__global__ __launch_bounds__(256) void fill_kernel(uint8_t* dst, const uint8_t* src, uint64_t n) {
  const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16u;
  if (i >= n) return;
  const bool wide = i + 16u <= n && ((uintptr_t)dst & 15u) == 0 && (!src || ((uintptr_t)src & 15u) == 0);
  if (wide) {
    *reinterpret_cast<uint4*>(dst + i) =
        src ? *reinterpret_cast<const uint4*>(src + i) : make_uint4(0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u);
    return;
  }
  const uint64_t end = i + 16u < n ? i + 16u : n;
  for (uint64_t k = i; k < end; ++k) dst[k] = src ? src[k] : (uint8_t)128;
}

template <int WIDTH>
__device__ __forceinline__ int group_sum(int v) {
#pragma unroll
  for (int off = WIDTH / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WIDTH);
  return v;
}

__global__ __launch_bounds__(256) void iter_kernel(DecodeArgs a, const uint8_t* __restrict__ cur,
                                                  uint8_t* __restrict__ nxt) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave = ((uint64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const uint64_t nwaves = (uint64_t)gridDim.x * 4;
  const int W = (int)a.width, H = (int)a.height;
  for (uint64_t r = wave; r < a.n; r += nwaves) {
    const Fields f = unpack(a.recs[r]);
    const int B = (int)a.b_max >> f.level;
    if (f.flags == 0) {
      const int n = B * B, logn = log2i(n);
      int dv[16];
      int sum = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int p = lane + 64 * k;
        dv[k] = 0;
        if (p < n) {
          const int i = p >> log2i(B), j = p & (B - 1);
          int si, sj;
          iso_src(f.iso, i, j, B, si, sj);
          dv[k] = mean4(cur, W, f.dx + 2 * sj, f.dy + 2 * si);
          sum += dv[k];
        }
      }
      sum = group_sum<64>(sum);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int p = lane + 64 * k;
        if (p < n) {
          const int i = p >> log2i(B), j = p & (B - 1);
          const int num = f.s_idx * (n * dv[k] - sum) + 8 * n * f.lum + 4 * n;
          const int v = num < 0 ? 0 : min(num >> (3 + logn), 255);
          nxt[(size_t)(f.y + i) * W + f.x + j] = (uint8_t)v;
        }
      }
    } else {
      const int b = B >> 1, nb = b * b, lognb = log2i(nb), logb = log2i(b);
      const int c = lane >> 4, l16 = lane & 15;
      const int cx = f.x + (c & 1) * b, cy = f.y + (c >> 1) * b;
      const int cdx = clampi(cx - b / 2, 0, W - 2 * b), cdy = clampi(cy - b / 2, 0, H - 2 * b);
      const int O0 = f.lum + f.d0, O1 = f.lum + f.d1, O2 = f.lum + f.d2;
      const int O = c == 0 ? O0 : (c == 1 ? O1 : (c == 2 ? O2 : 4 * f.lum - O0 - O1 - O2));
      int c1, c2, delta;
      phase2_consts(f.level + 1, c1, c2, delta);
      const int cv = ((f.s_idx >> c) & 1) ? c2 : c1;
      int dv[16];
      int sum = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int p = l16 + 16 * k;
        dv[k] = 0;
        if (p < nb) {
          const int i = p >> logb, j = p & (b - 1);
          dv[k] = mean4(cur, W, cdx + 2 * j, cdy + 2 * i);
          sum += dv[k];
        }
      }
      sum = group_sum<16>(sum);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int p = l16 + 16 * k;
        if (p < nb) {
          const int i = p >> logb, j = p & (b - 1);
          const int num = cv * (nb * dv[k] - sum) + 20 * nb * O + 10 * nb;
          const int v = num < 0 ? 0 : min((num >> lognb) / 20, 255);
          nxt[(size_t)(cy + i) * W + cx + j] = (uint8_t)v;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- tiles
// Tile-ordered decoding.  Streams whose records partition every top tile in
// order (consecutive Morton intervals of 2 x 2-pixel cells, y bit above x,
// tiles in raster order), use the co-centred domains and map blocks of at
// least 4 x 4 pixels are decoded one block of 128 x 128 pixels per
// workgroup: the block's domain region of the iterate is reduced to H0 in
// LDS once, every record's domain sum comes from there, and the output is
// written four pixels at a time.  Any other stream uses iter_kernel.

__device__ __forceinline__ int cell_morton(int cx, int cy) {
  int code = 0;
#pragma unroll
  for (int bit = 0; bit < 4; ++bit) code |= (((cx >> bit) & 1) << (2 * bit)) | (((cy >> bit) & 1) << (2 * bit + 1));
  return code;
}

__device__ __forceinline__ int cocentred(int p, int B, int extent) { return clampi(p - B / 2, 0, extent - 2 * B); }

// One lane per record: the first record of each tile, and whether the
// stream meets the conditions above: bit 0 of *flag is set when the stream
// is not in encoder order with co-centred domains, bit 1 when it maps
// blocks under 4 x 4 pixels (the 2 x 2 level: phase-1 ranges of side 2,
// phase-2 ranges of side 4), which the tile decoder does not take.
__global__ __launch_bounds__(256) void tile_setup_kernel(DecodeArgs a, uint32_t* tile_start, uint32_t* flag) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int W = (int)a.width, H = (int)a.height, bm = (int)a.b_max;
  const int tiles_x = W / bm, ntiles = tiles_x * (H / bm), cells = (bm / 2) * (bm / 2);
  auto info = [&](uint64_t k, int& tile, int& key, int& end, bool& centred) {
    const Fields f = unpack(a.recs[k]);
    const int B = bm >> f.level;
    tile = (f.y / bm) * tiles_x + f.x / bm;
    key = cell_morton((f.x % bm) >> 1, (f.y % bm) >> 1);
    end = key + (B >> 1) * (B >> 1);
    centred = f.dx == cocentred(f.x, B, W) && f.dy == cocentred(f.y, B, H);
  };
  {
    const Fields f = unpack(a.recs[i]);
    const int B = bm >> f.level;
    if (B < 4 || (f.flags != 0 && B < 8)) atomicOr(flag, 2u);
  }
  int tile, key, end;
  bool centred;
  info(i, tile, key, end, centred);
  bool ok = centred;
  bool first = true;
  if (i == 0) {
    ok = ok && tile == 0 && key == 0;
  } else {
    int tp, kp, ep;
    bool cp;
    info(i - 1, tp, kp, ep, cp);
    if (tile == tp) {
      ok = ok && key == ep;
      first = false;
    } else {
      ok = ok && tile == tp + 1 && key == 0 && ep == cells;
    }
  }
  if (i == a.n - 1) ok = ok && end == cells && tile == ntiles - 1;
  if (!ok) atomicOr(flag, 1u);
  if (first && tile >= 0 && tile < ntiles) tile_start[tile] = (uint32_t)i;
  if (i == a.n - 1) tile_start[ntiles] = (uint32_t)a.n;
}

// A decode plan splits the image into blocks of 64 x 64 pixels (partial at
// the right and bottom edges).  Each block's transforms become pieces: a
// phase-1 transform is one piece, a phase-2 transform four (one per
// sub-block, with its own domain, contrast and luminance, Sec. 3.3).  Every
// piece is an aligned square of side b >= 4 inside the block, so a block
// holds at most 256 pieces, and each 4 x 4-pixel cell of the block lies in
// exactly one.  Per block the plan stores the piece index of each cell
// (256 bytes) and up to 256 pieces of 8 bytes:
//   word 0: wx | wy << 6 | e << 12 | c << 15 | phase2 << 20 | log2(b / 4) << 21
//   word 1: L = 8 n m + 4 n (phase 1) or 20 n O_c + 10 n (phase 2), n = b^2,
// with (wx, wy) the domain origin in the block's H0 region (below) and c the
// contrast numerator (k of k/8, or the set's value of c/20).  Everything in
// the plan is fixed by the stream; only Sum d changes between iterations.
constexpr int kDecTile = 64;                 // block side (pixels)
constexpr int kDecCells = (kDecTile / 4) * (kDecTile / 4);
constexpr int kDecSpare = kDecCells - 1;        // plan slot of the cells of 2 x 2 blocks
constexpr uint32_t kDecSkip = 1u << 23;         // piece word-0 flag: cell left to the small-piece kernel

struct DecRegion {
  int X0, Y0, bw, bh;   // block origin and size (pixels)
  int ax0, ay0;         // origin of the staged region (multiple of 8)
  int n8x, n8y;         // 8 x 8-pixel groups staged per side
};

// The staged region is the union of the co-centred domains of the block's
// top tiles (every piece's domain lies inside it), origin rounded down to 8.
__device__ __forceinline__ DecRegion dec_region(int blk, int W, int H, int bm) {
  DecRegion r;
  const int nbx = (W + kDecTile - 1) / kDecTile;
  r.X0 = (blk % nbx) * kDecTile;
  r.Y0 = (blk / nbx) * kDecTile;
  r.bw = min(kDecTile, W - r.X0);
  r.bh = min(kDecTile, H - r.Y0);
  const int rx0 = clampi(r.X0 - bm / 2, 0, W - 2 * bm);
  const int rx1 = clampi(r.X0 + r.bw - bm - bm / 2, 0, W - 2 * bm) + 2 * bm;
  const int ry0 = clampi(r.Y0 - bm / 2, 0, H - 2 * bm);
  const int ry1 = clampi(r.Y0 + r.bh - bm - bm / 2, 0, H - 2 * bm) + 2 * bm;
  r.ax0 = rx0 & ~7;
  r.ay0 = ry0 & ~7;
  r.n8x = (rx1 - r.ax0 + 7) >> 3;
  r.n8y = (ry1 - r.ay0 + 7) >> 3;
  return r;
}

// One workgroup per block: gather the block's transforms (one run of
// consecutive records per tile row), expand them into pieces and the cell
// map.  Runs once per decode call.
__global__ __launch_bounds__(256) void dec_plan_kernel(DecodeArgs a, const uint32_t* __restrict__ tile_start,
                                                       uint8_t* __restrict__ cells, uint2* __restrict__ pieces,
                                                       uint32_t* __restrict__ small_list,
                                                       uint32_t* __restrict__ small_count) {
  __shared__ uint32_t s_run0[kDecTile / 4], s_runs[kDecTile / 4 + 1], s_count, s_small;
  __shared__ uint8_t s_cell[kDecCells];
  const int tid = threadIdx.x, blk = blockIdx.x;
  const int W = (int)a.width, H = (int)a.height, bm = (int)a.b_max;
  const DecRegion g = dec_region(blk, W, H, bm);
  const int tiles_x = W / bm, gxn = g.bw / bm, gyn = g.bh / bm;
  const int t0x = g.X0 / bm, t0y = g.Y0 / bm;
  if (tid < gyn) {
    const int t0 = (t0y + tid) * tiles_x + t0x;
    s_run0[tid] = tile_start[t0];
    s_runs[tid + 1] = tile_start[t0 + gxn] - tile_start[t0];
  }
  if (tid == 0) {
    s_count = 0;
    s_small = 0;
  }
  __syncthreads();
  if (tid == 0) {
    s_runs[0] = 0;
    for (int k = 0; k < gyn; ++k) s_runs[k + 1] += s_runs[k];
  }
  __syncthreads();
  const int nrec = (int)s_runs[gyn];
  uint2* out = pieces + (size_t)blk * kDecCells;
  for (int j = tid; j < nrec; j += 256) {
    int row = 0;
    while (row + 1 < gyn && (int)s_runs[row + 1] <= j) ++row;
    const uint32_t ri = s_run0[row] + (uint32_t)(j - (int)s_runs[row]);
    const Fields f = unpack(a.recs[ri]);
    const int B = bm >> f.level;
    if (B < 4 || (f.flags != 0 && B < 8)) {
      // a block of 2 x 2 pieces: listed for the small-piece kernel; its
      // cell points at the block's spare slot, which tells the tile kernel
      // to leave the cell alone
      small_list[atomicAdd(small_count, 1u)] = ri;
      s_small = 1;
      s_cell[((f.y - g.Y0) >> 2) * (kDecTile / 4) + ((f.x - g.X0) >> 2)] = (uint8_t)kDecSpare;
      continue;
    }
    const int np = f.flags ? 4 : 1, b = f.flags ? B / 2 : B;
    const uint32_t p0 = atomicAdd(&s_count, (uint32_t)np);
    int c1 = 0, c2 = 0, delta = 0;
    if (f.flags) phase2_consts(f.level + 1, c1, c2, delta);
    const int lb = log2i(b) - 2, n = b * b;
    for (int c = 0; c < np; ++c) {
      const int px = f.x + (f.flags ? (c & 1) * b : 0), py = f.y + (f.flags ? (c >> 1) * b : 0);
      uint32_t w0, w1;
      if (f.flags == 0) {
        const int wx = (f.dx - g.ax0) >> 1, wy = (f.dy - g.ay0) >> 1;
        w0 = (uint32_t)wx | (uint32_t)wy << 6 | (uint32_t)f.iso << 12 | (uint32_t)f.s_idx << 15 | (uint32_t)lb << 21;
        w1 = (uint32_t)(8 * n * f.lum + 4 * n);
      } else {
        const int wx = (cocentred(px, b, W) - g.ax0) >> 1, wy = (cocentred(py, b, H) - g.ay0) >> 1;
        const int O0 = f.lum + f.d0, O1 = f.lum + f.d1, O2 = f.lum + f.d2;
        const int O = c == 0 ? O0 : (c == 1 ? O1 : (c == 2 ? O2 : 4 * f.lum - O0 - O1 - O2));
        const int cv = ((f.s_idx >> c) & 1) ? c2 : c1;
        w0 = (uint32_t)wx | (uint32_t)wy << 6 | (uint32_t)cv << 15 | 1u << 20 | (uint32_t)lb << 21;
        w1 = (uint32_t)(20 * n * O + 10 * n);
      }
      const uint32_t p = p0 + (uint32_t)c;
      out[p] = make_uint2(w0, w1);
      const int cx0 = (px - g.X0) >> 2, cy0 = (py - g.Y0) >> 2, cs = b >> 2;
      for (int k = 0; k < cs * cs; ++k) s_cell[(cy0 + k / cs) * (kDecTile / 4) + cx0 + k % cs] = (uint8_t)p;
    }
  }
  __syncthreads();
  cells[(size_t)blk * kDecCells + tid] = s_cell[tid];
  // with a 2 x 2 block in it, the block has at most 255 pieces, so the
  // spare slot is free: a piece that only marks its cells
  if (tid == 0 && s_small) out[kDecSpare] = make_uint2(kDecSkip, 0u);
}

template <int BMAX>
struct DecGeo {
  static constexpr int NG8 = (kDecTile + BMAX + 6 + 7) / 8;   // max 8-pixel groups per region side
  static constexpr int HS = 4 * NG8;                          // H0 entries per region side
  static constexpr int HP = HS + 4;                           // H0 row pitch (bytes)
};

// Four H0 bytes starting at column `col` of row `row` (any alignment).
__device__ __forceinline__ uint32_t h0_quad(const uint32_t* t, int pitch_words, int row, int col) {
  const int w = row * pitch_words + (col >> 2);
  return __builtin_amdgcn_alignbyte(t[w + 1], t[w], (uint32_t)(col & 3));
}

// One Jacobi iteration over one block: stage the region's H0 and its
// transpose, every lane adds its cell's quarter-by-quarter share of its
// piece's domain sum (the piece's b x b domain block split into 4 x 4
// sub-blocks, one per cell of the piece), then writes its cell's 16 pixels.
template <int BMAX>
__global__ __launch_bounds__(256) void dec_iter_kernel(DecodeArgs a, uint32_t n_blk,
                                                       const uint8_t* __restrict__ cells,
                                                       const uint2* __restrict__ pieces,
                                                       const uint8_t* __restrict__ cur, uint8_t* __restrict__ nxt) {
  using D = DecGeo<BMAX>;
  constexpr int PW = D::HP / 4;
  __shared__ uint32_t s_h0[D::HS * PW + 1], s_h0t[D::HS * PW + 1];
  __shared__ uint32_t s_sd[kDecCells];
  const int tid = threadIdx.x;
  // XCD-aware order: consecutive blocks (one band of block rows) share an XCD
  const uint32_t per = (n_blk + 7u) >> 3;
  const uint32_t blk = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  if (blk >= n_blk) return;
  const int W = (int)a.width, H = (int)a.height;
  const DecRegion g = dec_region((int)blk, W, H, BMAX);
  // Every load below is unconditional, with clamped addresses, so that all
  // of them are in flight together: the lane's cell byte, its staging group
  // (a group outside the region loads a clamped one and stores nothing),
  // then its piece, which needs the cell byte only.  A cell outside a
  // partial block reads the block's own (unused) plan slot.
  const int cx = tid & (kDecTile / 4 - 1), cy = tid / (kDecTile / 4);
  const bool live = 4 * cx < g.bw && 4 * cy < g.bh;
  const uint32_t p = cells[(size_t)blk * kDecCells + tid];
  // ---- stage: one 8 x 8-pixel group per lane -> 4 x 4 H0 and H0^T
  const int gx0 = tid % D::NG8, gy0 = tid / D::NG8;
  const bool stage = gy0 < g.n8y && gx0 < g.n8x;
  const int gx = min(gx0, g.n8x - 1), gy = min(gy0, g.n8y - 1);
  const int x = g.ax0 + 8 * gx;        // x < W; x + 4 == W when the group sticks out
  const int second = x + 8 <= W ? 1 : 0;
  uint32_t v[8][2];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int y = min(g.ay0 + 8 * gy + r, H - 1);   // rows past the image feed no domain
    const uint32_t* src = reinterpret_cast<const uint32_t*>(cur + (size_t)y * W + x);
    v[r][0] = src[0];
    v[r][1] = src[second];                          // columns past the image feed no domain
  }
  __builtin_amdgcn_sched_barrier(0);     // keep the staging loads ahead of the piece load
  const uint2 pc = pieces[(size_t)blk * kDecCells + p];
  uint32_t hr[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) hr[q] = mean2x2_x4(v[2 * q][0], v[2 * q][1], v[2 * q + 1][0], v[2 * q + 1][1]);
  // a lane without a group writes the spare word past the tables (no branch,
  // so the loads above stay ahead of everything that waits for them)
  const int o_h0 = stage ? (4 * gy) * PW + gx : D::HS * PW;
  const int o_h0t = stage ? (4 * gx) * PW + gy : D::HS * PW;
  const int step = stage ? PW : 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) s_h0[o_h0 + q * step] = hr[q];
  const uint32_t u0 = __builtin_amdgcn_perm(hr[1], hr[0], 0x05010400u);
  const uint32_t u1 = __builtin_amdgcn_perm(hr[1], hr[0], 0x07030602u);
  const uint32_t w0 = __builtin_amdgcn_perm(hr[3], hr[2], 0x05010400u);
  const uint32_t w1 = __builtin_amdgcn_perm(hr[3], hr[2], 0x07030602u);
  s_h0t[o_h0t + 0 * step] = __builtin_amdgcn_perm(w0, u0, 0x05040100u);
  s_h0t[o_h0t + 1 * step] = __builtin_amdgcn_perm(w0, u0, 0x07060302u);
  s_h0t[o_h0t + 2 * step] = __builtin_amdgcn_perm(w1, u1, 0x05040100u);
  s_h0t[o_h0t + 3 * step] = __builtin_amdgcn_perm(w1, u1, 0x07060302u);
  s_sd[tid] = 0u;
  __syncthreads();
  // ---- the piece's fields and this cell's place in it
  const int wx = (int)(pc.x & 63u), wy = (int)((pc.x >> 6) & 63u);
  const int e = (int)((pc.x >> 12) & 7u), cnum = (int)((pc.x >> 15) & 31u);
  const bool ph2 = (pc.x >> 20) & 1u;
  const int lb = (int)((pc.x >> 21) & 3u) + 2, b = 1 << lb;
  const int rx = (4 * cx) & (b - 1), ry = (4 * cy) & (b - 1);
  if (live) {
    uint32_t acc = 0u;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc = __builtin_amdgcn_udot4(h0_quad(s_h0, PW, wy + ry + r, wx + rx), 0x01010101u, acc, false);
    atomicAdd(&s_sd[p], acc);
  }
  __syncthreads();
  if (!live || (pc.x & kDecSkip)) return;
  // ---- output: clamp((c (n d - Sum d) + L) >> shift) per pixel, divided by
  // 20 for a phase-2 piece
  const int shift = ph2 ? 2 * lb : 3 + 2 * lb;
  const int K = cnum << (2 * lb);
  const int C = (int)pc.y - cnum * (int)s_sd[p];
  // source rows / columns: for e < 4 row i of the range reads H0 row si with
  // columns running forward or backward; for e >= 4 it reads H0^T row sj
  const bool tr = e >= 4;
  const bool flip_row = tr ? (e & 1) : (e & 2);     // on the index that follows the range column
  const bool flip_col = tr ? (e & 2) : (e & 1);
  const uint32_t* tab = tr ? s_h0t : s_h0;
  const int base_row = tr ? wx : wy, base_col = tr ? wy : wx;
  uint8_t* dst = nxt + (size_t)(g.Y0 + 4 * cy) * W + g.X0 + 4 * cx;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = ry + r;
    uint32_t q;
    if (ph2) {
      q = h0_quad(s_h0, PW, wy + i, wx + rx);
    } else {
      // e < 4: row si = i or b-1-i, columns rx.. (or mirrored, reversed);
      // e >= 4: H0^T row sj = i or b-1-i, columns likewise
      const int srow = (tr ? flip_col : flip_row) ? b - 1 - i : i;
      const bool rev = tr ? flip_row : flip_col;
      const int scol = rev ? b - 4 - rx : rx;
      q = h0_quad(tab, PW, base_row + srow, base_col + scol);
      if (rev) q = __builtin_amdgcn_perm(0u, q, 0x00010203u);
    }
    uint32_t word = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int d = (int)((q >> (8 * k)) & 0xffu);
      const int num = K * d + C;
      uint32_t v = num < 0 ? 0u : (uint32_t)num >> shift;
      if (ph2) v /= 20u;
      word |= min(v, 255u) << (8 * k);
    }
    *reinterpret_cast<uint32_t*>(dst + (size_t)r * W) = word;
  }
}

// The 2 x 2 pieces of a tile-decoded stream, one iteration: four lanes per
// listed transform, one per 2 x 2 piece (a phase-2 range of side 4 has four
// sub-blocks; a phase-1 2 x 2 range is one piece, taken by the first lane).
// A 2 x 2 piece's domain lies at an odd origin (x - 1), so its means are
// formed from the iterate's pixels; the arithmetic is the per-record
// decoder's.
constexpr unsigned kSmallGroups = 2048;

__global__ __launch_bounds__(256) void small_iter_kernel(DecodeArgs a, const uint32_t* __restrict__ list,
                                                         const uint32_t* __restrict__ count,
                                                         const uint8_t* __restrict__ cur, uint8_t* __restrict__ nxt) {
  const int W = (int)a.width, H = (int)a.height;
  const uint64_t nl = 4ull * *count;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < nl; i += (uint64_t)gridDim.x * 256u) {
    const Fields f = unpack(a.recs[list[i >> 2]]);
    const int c = (int)(i & 3u);
    if (!f.flags && c != 0) continue;
    int c1 = 0, c2 = 0, delta = 0;
    if (f.flags) phase2_consts(f.level + 1, c1, c2, delta);
    {
      const int px = f.x + (f.flags ? 2 * (c & 1) : 0), py = f.y + (f.flags ? 2 * (c >> 1) : 0);
      const int ox = f.flags ? cocentred(px, 2, W) : f.dx, oy = f.flags ? cocentred(py, 2, H) : f.dy;
      int d[2][2], sum = 0;
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
        for (int j2 = 0; j2 < 2; ++j2) {
          d[i2][j2] = mean4(cur, W, ox + 2 * j2, oy + 2 * i2);
          sum += d[i2][j2];
        }
      int O = f.lum, k = f.s_idx;
      if (f.flags) {
        const int O0 = f.lum + f.d0, O1 = f.lum + f.d1, O2 = f.lum + f.d2;
        O = c == 0 ? O0 : (c == 1 ? O1 : (c == 2 ? O2 : 4 * f.lum - O0 - O1 - O2));
        k = ((f.s_idx >> c) & 1) ? c2 : c1;
      }
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
        for (int j2 = 0; j2 < 2; ++j2) {
          int si = i2, sj = j2;
          if (!f.flags) iso_src(f.iso, i2, j2, 2, si, sj);
          // selects, not an indexed load: the four means stay in registers
          const int dv = si ? (sj ? d[1][1] : d[1][0]) : (sj ? d[0][1] : d[0][0]);
          int v;
          if (!f.flags) {
            const int num = k * (4 * dv - sum) + 32 * f.lum + 16;
            v = num < 0 ? 0 : min(num >> 5, 255);
          } else {
            const int num = k * (4 * dv - sum) + 80 * O + 40;
            v = num < 0 ? 0 : min((num >> 2) / 20, 255);
          }
          nxt[(size_t)(py + i2) * W + px + j2] = (uint8_t)v;
        }
    }
  }
}

}  // namespace

hipError_t launch_decode_check(const DecodeArgs& a, uint32_t* bad, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(check_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, bad);
  return hipGetLastError();
}

hipError_t launch_decode_zoom(const DecodeArgs& a, uint32_t z, uint4* out, uint32_t* bad, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(zoom_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, z, out, bad);
  return hipGetLastError();
}

hipError_t launch_decode_fill(uint8_t* dst, const uint8_t* src, uint32_t w, uint32_t h, hipStream_t s) {
  const uint64_t n = (uint64_t)w * h;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 4095) / 4096)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_decode_tile_setup(const DecodeArgs& a, uint32_t* tile_start, uint32_t* flag, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(tile_setup_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, tile_start, flag);
  return hipGetLastError();
}

size_t decode_plan_blocks(uint32_t w, uint32_t h) {
  return (size_t)((w + kDecTile - 1) / kDecTile) * ((h + kDecTile - 1) / kDecTile);
}

hipError_t launch_decode_plan(const DecodeArgs& a, const uint32_t* tile_start, uint8_t* cells, uint2* pieces,
                              uint32_t* small_list, uint32_t* small_count, hipStream_t s) {
  const unsigned grid = (unsigned)decode_plan_blocks(a.width, a.height);
  hipLaunchKernelGGL(dec_plan_kernel, dim3(grid), dim3(256), 0, s, a, tile_start, cells, pieces, small_list,
                     small_count);
  return hipGetLastError();
}

hipError_t launch_decode_small(const DecodeArgs& a, const uint32_t* small_list, const uint32_t* small_count,
                               const uint8_t* cur, uint8_t* nxt, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const uint64_t want = (4 * a.n + 255) / 256;
  const unsigned grid = (unsigned)(want < kSmallGroups ? want : kSmallGroups);
  hipLaunchKernelGGL(small_iter_kernel, dim3(grid), dim3(256), 0, s, a, small_list, small_count, cur, nxt);
  return hipGetLastError();
}

hipError_t launch_decode_tile_iter(const DecodeArgs& a, const uint8_t* cells, const uint2* pieces,
                                   const uint8_t* cur, uint8_t* nxt, hipStream_t s) {
  const uint32_t n_blk = (uint32_t)decode_plan_blocks(a.width, a.height);
  const unsigned grid = 8u * ((n_blk + 7u) >> 3);
  switch (a.b_max) {
    case 32: hipLaunchKernelGGL(dec_iter_kernel<32>, dim3(grid), dim3(256), 0, s, a, n_blk, cells, pieces, cur, nxt); break;
    case 16: hipLaunchKernelGGL(dec_iter_kernel<16>, dim3(grid), dim3(256), 0, s, a, n_blk, cells, pieces, cur, nxt); break;
    case 8: hipLaunchKernelGGL(dec_iter_kernel<8>, dim3(grid), dim3(256), 0, s, a, n_blk, cells, pieces, cur, nxt); break;
    case 4: hipLaunchKernelGGL(dec_iter_kernel<4>, dim3(grid), dim3(256), 0, s, a, n_blk, cells, pieces, cur, nxt); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_decode_iter(const DecodeArgs& a, const uint8_t* cur, uint8_t* nxt, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  uint64_t waves = a.n < (1u << 20) ? a.n : (1u << 20);
  const unsigned grid = (unsigned)((waves + 3) / 4);
  hipLaunchKernelGGL(iter_kernel, dim3(grid), dim3(256), 0, s, a, cur, nxt);
  return hipGetLastError();
}

}  // namespace fe
