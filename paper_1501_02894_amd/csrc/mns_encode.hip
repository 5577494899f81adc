// Fused MNS quadtree encoder for gfx950.
//
// One workgroup (256 lanes, 4 waves) owns a GX x GY block of top-level
// B_max tiles of one image and runs the whole quadtree of those tiles:
//
//   1. stage: the pixels of the union of the tiles' co-centred 2B x 2B
//      domains (which contains every range and every descendant's domain)
//      are read once from HBM with 8-byte coalesced loads into LDS; the 2 x 2
//      round-half-up mean image H0 of that region and its transpose are
//      formed in LDS on the fly (Sec. 3: "mean filter to four neighbor
//      pixels").
//   2. per level l (B = B_max >> (l-1)): every listed range is processed by a
//      team of T lanes (T chosen so the list fills the workgroup); each lane
//      sums packed-u8 dot products (v_dot4_u32_u8) over row pairs (i, B-1-i)
//      of the range and of the domain window / its transpose, giving Sum r,
//      Sum r^2, Sum d, Sum d^2 and the 8 isometric Sum r T_e(d); DPP team
//      reduction; the team leader fits (e, k, m) exactly in int64 (Sec. 3).
//   3. phase 2 (Sec. 3.1-3.3): the parents that failed at level l-1 are
//      decided from the identity moments of their four children, which are
//      exactly the level-l ranges just computed.
//   4. accepted ranges are written as 16-byte records into per-tile slots
//      indexed by the Morton code of their top-left B_min cell; failed ranges
//      are compacted (wave ballot + prefix) into the parent list and their
//      four children into the next level's list.
//
// After the workgroup finishes, its tiles' occupancy masks and record
// counts are published; a second kernel orders the records into the
// depth-first stream (tiles in raster order, Morton order inside a tile).
#include "fe_device.h"
#include "fe_internal.h"

namespace fe {
namespace {

template <int BMAX, int L, int GX, int GY>
struct Geo {
  static constexpr int BMIN = BMAX >> (L - 1);
  static constexpr int NT = GX * GY;
  static constexpr int CELLS = 1 << (2 * (L - 1));
  static constexpr int CAP = NT * CELLS;                      // deepest list bound
  static constexpr int PCAP = CAP / 4 > 0 ? CAP / 4 : 1;      // parent list bound
  static constexpr int RWA = ((GX + 1) * BMAX + 6 + 7) & ~7;  // region width bound (px)
  static constexpr int RHA = (GY + 1) * BMAX + 8;             // region height bound (px)
  static constexpr int RP = RWA + 4;                          // image row pitch (bytes)
  static constexpr int HW = RWA / 2, HH = RHA / 2;            // H0 region bounds
  static constexpr int HP = HW + 8;                           // H0 row pitch
  static constexpr int TP = ((HH + 3) & ~3) + 8;              // H0^T row pitch
  static constexpr int IMG_W = RHA * RP / 4 + 4;              // dwords
  static constexpr int H0_W = HH * HP / 4 + 4;
  static constexpr int H0T_W = HW * TP / 4 + 4;
};

struct Region {
  int W, H;            // image sides
  int ax0, ay0;        // region origin (pixels), multiples of 8
  int tx0, ty0, gx;    // first tile of the block, tiles per block row
  int tiles_x;
  uint64_t tile_first;
};

template <int BMAX, int BMIN>
__device__ __forceinline__ void range_xy(uint32_t meta, const Region& r, int& X, int& Y) {
  const int tile = (int)(meta >> 16);
  const int tly = tile / r.gx, tlx = tile - tly * r.gx;
  X = (r.tx0 + tlx) * BMAX + (int)(meta & 0xffu) * BMIN;
  Y = (r.ty0 + tly) * BMAX + (int)((meta >> 8) & 0xffu) * BMIN;
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

// Stream compaction over the workgroup: returns the exclusive position of
// this lane's flag within the current 256-lane chunk, and the chunk total.
__device__ __forceinline__ uint32_t block_prefix(bool flag, uint32_t* s_wsum, uint32_t& total) {
  const uint64_t bal = __ballot(flag);
  const uint32_t lane_pre =
      __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s_wsum[wave] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t v = s_wsum[w];
    off += (w < wave) ? v : 0u;
    tot += v;
  }
  __syncthreads();
  total = tot;
  return off + lane_pre;
}

template <int BMAX, int L, int GX, int GY>
__global__ __launch_bounds__(256) void mns_tiles_kernel(EncodeArgs a) {
  using G = Geo<BMAX, L, GX, GY>;
  __shared__ uint32_t s_img[G::IMG_W];
  __shared__ uint32_t s_h0[G::H0_W];
  __shared__ uint32_t s_h0t[G::H0T_W];
  __shared__ uint32_t s_meta[2][G::CAP];
  __shared__ uint32_t s_fit[G::CAP];
  __shared__ uint32_t s_mom[5][G::CAP];
  __shared__ uint32_t s_pmeta[G::PCAP];
  __shared__ uint32_t s_pm[G::PCAP];
  __shared__ unsigned long long s_mask[G::NT];
  __shared__ uint32_t s_wsum[4];

  // XCD-aware order: consecutive logical blocks share an XCD (and its L2).
  const uint32_t per = (a.n_wg + 7u) >> 3;
  const uint32_t wg = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  if (wg >= a.n_wg) return;
  int lo = 0, hi = (int)a.n_imgs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.imgs[mid].wg_first <= wg) lo = mid; else hi = mid - 1;
  }
  const ImgDev im = a.imgs[lo];
  const uint32_t local = wg - im.wg_first;
  const int gyi = (int)(local / im.groups_x), gxi = (int)(local - (uint32_t)gyi * im.groups_x);
  Region rg;
  rg.W = (int)im.width;
  rg.H = (int)im.height;
  rg.tx0 = gxi * GX;
  rg.ty0 = gyi * GY;
  rg.gx = min(GX, (int)im.tiles_x - rg.tx0);
  const int gy = min(GY, (int)im.tiles_y - rg.ty0);
  rg.tiles_x = (int)im.tiles_x;
  rg.tile_first = im.tile_first;
  const int ntiles = rg.gx * gy;
  const int tid = threadIdx.x;

  // ---- 1. stage the region and its 2x2 mean image
  const int rx0 = clampi(rg.tx0 * BMAX - BMAX / 2, 0, rg.W - 2 * BMAX);
  const int rx1 = clampi((rg.tx0 + rg.gx - 1) * BMAX - BMAX / 2, 0, rg.W - 2 * BMAX) + 2 * BMAX;
  const int ry0 = clampi(rg.ty0 * BMAX - BMAX / 2, 0, rg.H - 2 * BMAX);
  const int ry1 = clampi((rg.ty0 + gy - 1) * BMAX - BMAX / 2, 0, rg.H - 2 * BMAX) + 2 * BMAX;
  rg.ax0 = rx0 & ~7;
  rg.ay0 = ry0 & ~7;
  const int n8 = (rx1 - rg.ax0 + 7) >> 3;
  const int hrows = (ry1 - rg.ay0) >> 1;
  uint8_t* h0t_b = reinterpret_cast<uint8_t*>(s_h0t);
  for (int idx = tid; idx < hrows * n8; idx += 256) {
    const int hr = idx / n8, c8 = idx - hr * n8;
    const int x = rg.ax0 + 8 * c8;
    const uint8_t* p0 = im.data + (size_t)(rg.ay0 + 2 * hr) * im.stride + x;
    const uint8_t* p1 = p0 + im.stride;
    uint32_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    if (x + 8 <= rg.W) {
      const uint2 u = *reinterpret_cast<const uint2*>(p0);
      const uint2 v = *reinterpret_cast<const uint2*>(p1);
      a0 = u.x; a1 = u.y; b0 = v.x; b1 = v.y;
    } else if (x < rg.W) {
      a0 = *reinterpret_cast<const uint32_t*>(p0);
      b0 = *reinterpret_cast<const uint32_t*>(p1);
    }
    s_img[(2 * hr) * (G::RP / 4) + 2 * c8] = a0;
    s_img[(2 * hr) * (G::RP / 4) + 2 * c8 + 1] = a1;
    s_img[(2 * hr + 1) * (G::RP / 4) + 2 * c8] = b0;
    s_img[(2 * hr + 1) * (G::RP / 4) + 2 * c8 + 1] = b1;
    const uint32_t h = mean2x2_x4(a0, a1, b0, b1);
    s_h0[hr * (G::HP / 4) + c8] = h;
    h0t_b[(4 * c8 + 0) * G::TP + hr] = (uint8_t)h;
    h0t_b[(4 * c8 + 1) * G::TP + hr] = (uint8_t)(h >> 8);
    h0t_b[(4 * c8 + 2) * G::TP + hr] = (uint8_t)(h >> 16);
    h0t_b[(4 * c8 + 3) * G::TP + hr] = (uint8_t)(h >> 24);
  }
  for (int t = tid; t < G::NT; t += 256) s_mask[t] = 0ull;
  for (int t = tid; t < ntiles; t += 256) s_meta[0][t] = (uint32_t)t << 16;
  __syncthreads();

  int n = ntiles;  // ranges in the current list (uniform)
  for (int lev = 1; lev <= L; ++lev) {
    const int cb = (lev - 1) & 1;
    const bool last = lev == L;
    const uint32_t thr = last ? 0u : a.thr[lev - 1];
    const int B = BMAX >> (lev - 1);

    // ---- 2. moments + phase-1 fit of the listed ranges
    auto moments_fit = [&](auto bconst) {
      constexpr int BB = decltype(bconst)::value;
      constexpr bool ALIGNED = BB >= 16;
      int T = 1;
      while (T < BB / 2 && T < 16 && n * (T * 2) <= 256) T *= 2;
      const int logT = __builtin_ctz((unsigned)T);
      for (int base = 0; base < n * T; base += 256) {
        const int idx = base + tid;
        const int e = idx >> logT, t = idx & (T - 1);
        uint32_t acc[12];
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[j] = 0u;
        if (e < n) {
          int X, Y;
          range_xy<BMAX, G::BMIN>(s_meta[cb][e], rg, X, Y);
          const int dx = clampi(X - BB / 2, 0, rg.W - 2 * BB);
          const int dy = clampi(Y - BB / 2, 0, rg.H - 2 * BB);
          const int rx = X - rg.ax0, ry = Y - rg.ay0;
          const int wx = (dx - rg.ax0) >> 1, wy = (dy - rg.ay0) >> 1;
          for (int i = t; i < BB / 2; i += T)
            accumulate_row_pair<BB, ALIGNED>(s_img, ry * G::RP + rx, G::RP, s_h0, wy * G::HP + wx, G::HP,
                                             s_h0t, wx * G::TP + wy, G::TP, i, acc);
        }
        team_reduce(acc, T);
        if (e < n && t == 0) {
          s_fit[e] = fit_phase1<BB>(acc, last, thr);
          s_mom[0][e] = acc[0];
          s_mom[1][e] = acc[1];
          s_mom[2][e] = acc[2];
          s_mom[3][e] = acc[3];
          s_mom[4][e] = acc[4];
        }
      }
    };
    if constexpr (BMAX >= 32) { if (B == 32) moments_fit(std::integral_constant<int, 32>{}); }
    if constexpr (BMAX >= 16 && G::BMIN <= 16) { if (B == 16) moments_fit(std::integral_constant<int, 16>{}); }
    if constexpr (BMAX >= 8 && G::BMIN <= 8) { if (B == 8) moments_fit(std::integral_constant<int, 8>{}); }
    if constexpr (G::BMIN <= 4) { if (B == 4) moments_fit(std::integral_constant<int, 4>{}); }
    __syncthreads();

    // ---- 3. phase 2 of the parents that failed at level lev-1
    if (lev >= 2 && a.phase2) {
      const int np = n >> 2;
      auto phase2 = [&](auto bconst) {
        constexpr int BB = decltype(bconst)::value;   // child side
        for (int p = tid; p < np; p += 256) {
          uint32_t mom[4][5];
#pragma unroll
          for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int s = 0; s < 5; ++s) mom[c][s] = s_mom[s][4 * p + c];
          const int m = (int)s_pm[p];
          int O[4];
          uint32_t bits;
          const bool ok = fit_phase2<BB>(mom, m, lev - 1, a.thr[lev - 2], O, bits);
          if (ok) {
            const uint32_t pmeta = s_pmeta[p];
            int X, Y;
            range_xy<BMAX, G::BMIN>(pmeta, rg, X, Y);
            const int PB = 2 * BB;
            const int dx = clampi(X - PB / 2, 0, rg.W - 2 * PB);
            const int dy = clampi(Y - PB / 2, 0, rg.H - 2 * PB);
            const uint4 rec = make_record(X, Y, dx, dy, lev - 2, 1, 0, (int)bits, m, O[0] - m, O[1] - m,
                                          O[2] - m);
            const int tile = (int)(pmeta >> 16);
            const int tly = tile / rg.gx, tlx = tile - tly * rg.gx;
            const uint64_t tg = rg.tile_first + (uint64_t)(rg.ty0 + tly) * rg.tiles_x + (rg.tx0 + tlx);
            const int cell = morton(pmeta);
            a.staging[tg * G::CELLS + cell] = rec;
            atomicOr(&s_mask[tile], 1ull << cell);
#pragma unroll
            for (int c = 0; c < 4; ++c) s_fit[4 * p + c] |= kFitDead;
          }
        }
      };
      if constexpr (BMAX >= 32 && G::BMIN <= 16) { if (B == 16) phase2(std::integral_constant<int, 16>{}); }
      if constexpr (BMAX >= 16 && G::BMIN <= 8) { if (B == 8) phase2(std::integral_constant<int, 8>{}); }
      if constexpr (BMAX >= 8 && G::BMIN <= 4) { if (B == 4) phase2(std::integral_constant<int, 4>{}); }
      __syncthreads();
    }

    // ---- 4. store accepted ranges; compact failures into the next level
    uint32_t nfail = 0;
    for (int base = 0; base < n; base += 256) {
      const int e = base + tid;
      bool fail = false;
      uint32_t meta = 0, fit = 0;
      if (e < n) {
        meta = s_meta[cb][e];
        fit = s_fit[e];
        if (!(fit & kFitDead)) {
          if (fit & kFitAccept) {
            int X, Y;
            range_xy<BMAX, G::BMIN>(meta, rg, X, Y);
            const int dx = clampi(X - B / 2, 0, rg.W - 2 * B);
            const int dy = clampi(Y - B / 2, 0, rg.H - 2 * B);
            const uint4 rec = make_record(X, Y, dx, dy, lev - 1, 0, (int)((fit >> 11) & 7u),
                                          (int)((fit >> 8) & 7u), (int)(fit & 0xffu), 0, 0, 0);
            const int tile = (int)(meta >> 16);
            const int tly = tile / rg.gx, tlx = tile - tly * rg.gx;
            const uint64_t tg = rg.tile_first + (uint64_t)(rg.ty0 + tly) * rg.tiles_x + (rg.tx0 + tlx);
            const int cell = morton(meta);
            a.staging[tg * G::CELLS + cell] = rec;
            atomicOr(&s_mask[tile], 1ull << cell);
          } else {
            fail = true;
          }
        }
      }
      uint32_t total;
      const uint32_t q = nfail + block_prefix(fail, s_wsum, total);
      if (fail) {
        s_pmeta[q] = meta;
        s_pm[q] = fit & 0xffu;
        const uint32_t half = (uint32_t)(B / 2 / G::BMIN);
        const uint32_t cx = meta & 0xffu, cy = (meta >> 8) & 0xffu, tile = meta & 0xffff0000u;
#pragma unroll
        for (uint32_t c = 0; c < 4; ++c)
          s_meta[cb ^ 1][4 * q + c] = tile | ((cy + (c >> 1) * half) << 8) | (cx + (c & 1u) * half);
      }
      nfail += total;
    }
    __syncthreads();
    n = (int)(4 * nfail);
    if (last || n == 0) break;
  }

  // ---- publish per-tile occupancy and counts
  for (int t = tid; t < ntiles; t += 256) {
    const int tly = t / rg.gx, tlx = t - tly * rg.gx;
    const uint64_t tg = rg.tile_first + (uint64_t)(rg.ty0 + tly) * rg.tiles_x + (rg.tx0 + tlx);
    const unsigned long long mk = s_mask[t];
    a.masks[tg] = mk;
    atomicAdd(&a.chunk_sum[tg / kChunkTiles], (uint32_t)__popcll(mk));
  }
}

__global__ void zero_u32_kernel(uint32_t* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// One workgroup per kChunkTiles consecutive tiles (global order = image,
// then tile raster).  Record k of tile t goes to the stream position
// (records of all earlier tiles) + (rank of its Morton cell among t's).
__global__ __launch_bounds__(256) void scatter_kernel(const ImgDev* imgs, uint32_t n_imgs,
                                                     uint64_t total_tiles, int cells,
                                                     const uint64_t* masks, const uint32_t* chunk_sum,
                                                     const uint4* staging, uint4* out, uint64_t cap,
                                                     uint64_t* offsets) {
  __shared__ unsigned long long s_red[256];
  __shared__ uint32_t s_scan[256];
  __shared__ unsigned long long s_tbase[kChunkTiles];
  const int tid = threadIdx.x;
  const uint64_t c0 = (uint64_t)blockIdx.x * kChunkTiles;
  unsigned long long acc = 0;
  for (uint32_t i = tid; i < blockIdx.x; i += 256) acc += chunk_sum[i];
  s_red[tid] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) s_red[tid] += s_red[tid + s];
    __syncthreads();
  }
  const unsigned long long base = s_red[0];
  constexpr int PER = kChunkTiles / 256;
  unsigned long long mk[PER];
  uint32_t tsum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const uint64_t tile = c0 + (uint64_t)tid * PER + j;
    mk[j] = tile < total_tiles ? masks[tile] : 0ull;
    tsum += (uint32_t)__popcll(mk[j]);
  }
  s_scan[tid] = tsum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t v = tid >= off ? s_scan[tid - off] : 0u;
    __syncthreads();
    s_scan[tid] += v;
    __syncthreads();
  }
  unsigned long long pos = base + s_scan[tid] - tsum;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const uint64_t tile = c0 + (uint64_t)tid * PER + j;
    s_tbase[tid * PER + j] = pos;
    unsigned long long m = mk[j];
    while (m) {
      const int b = __builtin_ctzll(m);
      m &= m - 1;
      if (pos < cap) out[pos] = staging[tile * (uint64_t)cells + b];
      ++pos;
    }
  }
  __syncthreads();
  for (uint32_t k = tid; k < n_imgs; k += 256) {
    const uint64_t tf = imgs[k].tile_first;
    if (tf >= c0 && tf < c0 + kChunkTiles) offsets[k] = s_tbase[tf - c0];
  }
  if (blockIdx.x == gridDim.x - 1 && tid == 255) offsets[n_imgs] = pos;
}

}  // namespace

// ---------------------------------------------------------------- launchers
template <int BMAX, int L, int GX, int GY>
static hipError_t launch_one(const EncodeArgs& a, hipStream_t s) {
  const uint32_t grid = ((a.n_wg + 7u) >> 3) << 3;
  hipLaunchKernelGGL((mns_tiles_kernel<BMAX, L, GX, GY>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Tile shapes (GX x GY top tiles per workgroup) instantiated per
// (b_max, levels); the first entry is the default.
#define FE_SHAPES(X)                                                     \
  X(4, 1, 16, 16) X(4, 1, 32, 8)                                         \
  X(8, 1, 16, 8) X(8, 1, 8, 8) X(8, 2, 8, 8) X(8, 2, 16, 4) X(8, 2, 4, 4) \
  X(16, 1, 8, 4) X(16, 1, 4, 4) X(16, 2, 8, 4) X(16, 2, 4, 4)            \
  X(16, 3, 8, 4) X(16, 3, 4, 4) X(16, 3, 16, 2) X(16, 3, 8, 2)           \
  X(32, 1, 4, 2) X(32, 2, 4, 2) X(32, 3, 4, 2) X(32, 3, 2, 2)            \
  X(32, 4, 4, 2) X(32, 4, 2, 2) X(32, 4, 8, 1)

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

hipError_t launch_zero_u32(uint32_t* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_scatter(const ImgDev* imgs, uint32_t n_imgs, uint64_t total_tiles, int cells,
                          const uint64_t* masks, const uint32_t* chunk_sum, const uint4* staging, uint4* out,
                          uint64_t cap, uint64_t* offsets, hipStream_t s) {
  const unsigned grid = (unsigned)((total_tiles + kChunkTiles - 1) / kChunkTiles);
  hipLaunchKernelGGL(scatter_kernel, dim3(grid), dim3(256), 0, s, imgs, n_imgs, total_tiles, cells, masks,
                     chunk_sum, staging, out, cap, offsets);
  return hipGetLastError();
}

}  // namespace fe
