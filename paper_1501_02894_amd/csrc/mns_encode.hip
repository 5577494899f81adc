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
  static constexpr int NT = GX * GY;                          // tiles per workgroup
  static constexpr int NTW = NT / 4;                          // tiles per wave
  static constexpr int CELLS = 1 << (2 * (L - 1));
  static constexpr int CAPW = NTW * CELLS;                    // per-wave deepest list bound
  static constexpr int PCAPW = CAPW / 4 > 0 ? CAPW / 4 : 1;   // per-wave parent list bound
  static constexpr int TW = GX * BMAX, TH = GY * BMAX;        // tile block in pixels
  static constexpr int TPITCH = TW + 4;                       // tile pixel row pitch (bytes)
  static constexpr int RWA = ((GX + 1) * BMAX + 6 + 7) & ~7;  // region width bound (px)
  static constexpr int RHA = (GY + 1) * BMAX + 8;             // region height bound (px)
  static constexpr int HW = RWA / 2, HH = RHA / 2;            // H0 region bounds
  static constexpr int HP = HW + 8;                           // H0 row pitch
  static constexpr int TP = ((HH + 3) & ~3) + 8;              // H0^T row pitch
  static constexpr int IMG_W = TH * TPITCH / 4 + 4;           // dwords
  static constexpr int H0_W = HH * HP / 4 + 4;
  static constexpr int H0T_W = HW * TP / 4 + 4;
  static_assert(NT % 4 == 0, "tiles per workgroup must split over 4 waves");
};

struct Region {
  int W, H;            // image sides
  int ax0, ay0;        // H0 region origin (pixels), multiples of 8
  int X0, Y0;          // tile block origin (pixels)
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

__device__ __forceinline__ uint64_t tile_global(uint32_t meta, const Region& r) {
  const int tile = (int)(meta >> 16);
  const int tly = tile / r.gx, tlx = tile - tly * r.gx;
  return r.tile_first + (uint64_t)(r.ty0 + tly) * r.tiles_x + (uint64_t)(r.tx0 + tlx);
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

// Make this wave's LDS writes visible to its own later reads (the lanes of
// one wave exchange data through LDS; no other wave is involved).  The
// fences are restricted to LDS so that outstanding global stores (records)
// are not waited for.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int BMAX, int L, int GX, int GY>
__global__ __launch_bounds__(256) void mns_tiles_kernel(EncodeArgs a) {
  using G = Geo<BMAX, L, GX, GY>;
  __shared__ uint32_t s_img[G::IMG_W];
  __shared__ uint32_t s_h0[G::H0_W];
  __shared__ uint32_t s_h0t[G::H0T_W];
  __shared__ uint32_t s_meta[4][2][G::CAPW];
  __shared__ uint32_t s_fit[4][G::CAPW];
  __shared__ uint32_t s_mom[4][5][G::CAPW];
  __shared__ uint32_t s_pmeta[4][G::PCAPW];
  __shared__ uint32_t s_pm[4][G::PCAPW];
  __shared__ unsigned long long s_mask[G::NT];

  // XCD-aware order: consecutive logical blocks share an XCD (and its L2).
  const uint32_t per = (a.n_wg + 7u) >> 3;
  const uint32_t wg = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  if (wg >= a.n_wg) return;
  // image of this block: the number of images starting at or before it,
  // counted with independent vector loads (no dependent search chain)
  int lo = -1;
  for (uint32_t k0 = 0; k0 < a.n_imgs; k0 += 64u) {
    const uint32_t k = k0 + (threadIdx.x & 63u);
    lo += (int)__popcll(__ballot(k < a.n_imgs && a.wg_first[k] <= wg));
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
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
  rg.X0 = rg.tx0 * BMAX;
  rg.Y0 = rg.ty0 * BMAX;
  const int ntiles = rg.gx * gy;
  const int tid = threadIdx.x;

  // ---- 1. stage the tile pixels and the 2x2 mean image of the domain region
  const int rx0 = clampi(rg.X0 - BMAX / 2, 0, rg.W - 2 * BMAX);
  const int rx1 = clampi((rg.tx0 + rg.gx - 1) * BMAX - BMAX / 2, 0, rg.W - 2 * BMAX) + 2 * BMAX;
  const int ry0 = clampi(rg.Y0 - BMAX / 2, 0, rg.H - 2 * BMAX);
  const int ry1 = clampi((rg.ty0 + gy - 1) * BMAX - BMAX / 2, 0, rg.H - 2 * BMAX) + 2 * BMAX;
  rg.ax0 = rx0 & ~7;
  rg.ay0 = ry0 & ~7;
  const int n8 = (rx1 - rg.ax0 + 7) >> 3;
  const int hrows = (ry1 - rg.ay0) >> 1;
  const int tx_end = rg.X0 + rg.gx * BMAX, ty_end = rg.Y0 + gy * BMAX;
  uint8_t* h0t_b = reinterpret_cast<uint8_t*>(s_h0t);
  for (int idx = tid; idx < hrows * n8; idx += 256) {
    const int hr = idx / n8, c8 = idx - hr * n8;
    const int x = rg.ax0 + 8 * c8, y = rg.ay0 + 2 * hr;
    const uint32_t* p0 = reinterpret_cast<const uint32_t*>(im.data + (size_t)y * im.stride + x);
    const uint32_t* p1 = reinterpret_cast<const uint32_t*>(im.data + (size_t)(y + 1) * im.stride + x);
    uint32_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    if (x + 8 <= rg.W) {
      a0 = p0[0]; a1 = p0[1]; b0 = p1[0]; b1 = p1[1];
    } else if (x < rg.W) {
      a0 = p0[0]; b0 = p1[0];
    }
    // tile pixels (dword granularity: tile edges are multiples of 4)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int xx = x + 4 * h;
      if (xx >= rg.X0 && xx < tx_end) {
        const int col = (xx - rg.X0) >> 2;
        if (y >= rg.Y0 && y < ty_end) s_img[(y - rg.Y0) * (G::TPITCH / 4) + col] = h ? a1 : a0;
        if (y + 1 >= rg.Y0 && y + 1 < ty_end) s_img[(y + 1 - rg.Y0) * (G::TPITCH / 4) + col] = h ? b1 : b0;
      }
    }
    const uint32_t hv = mean2x2_x4(a0, a1, b0, b1);
    s_h0[hr * (G::HP / 4) + c8] = hv;
    h0t_b[(4 * c8 + 0) * G::TP + hr] = (uint8_t)hv;
    h0t_b[(4 * c8 + 1) * G::TP + hr] = (uint8_t)(hv >> 8);
    h0t_b[(4 * c8 + 2) * G::TP + hr] = (uint8_t)(hv >> 16);
    h0t_b[(4 * c8 + 3) * G::TP + hr] = (uint8_t)(hv >> 24);
  }
  for (int t = tid; t < G::NT; t += 256) s_mask[t] = 0ull;
  __syncthreads();

  // ---- 2. each wave runs the quadtree of its own tiles, independently
  const int wave = tid >> 6, lane = tid & 63;
  const int t_first = wave * G::NTW;
  const int my_tiles = max(0, min(G::NTW, ntiles - t_first));
  if (my_tiles == 0) return;
  uint32_t* w_meta0 = s_meta[wave][0];
  uint32_t* w_meta1 = s_meta[wave][1];
  uint32_t* w_fit = s_fit[wave];
  uint32_t* w_pmeta = s_pmeta[wave];
  uint32_t* w_pm = s_pm[wave];
  if (lane < my_tiles) w_meta0[lane] = (uint32_t)(t_first + lane) << 16;
  wave_sync();

  int n = my_tiles;  // ranges in the current list (wave-uniform)
  for (int lev = 1; lev <= L; ++lev) {
    uint32_t* cur = (lev & 1) ? w_meta0 : w_meta1;
    uint32_t* nxt = (lev & 1) ? w_meta1 : w_meta0;
    const bool last = lev == L;
    const uint32_t thr = last ? 0u : a.thr[lev - 1];
    const int B = BMAX >> (lev - 1);

    // moments + phase-1 fit of the listed ranges (team of T lanes per range)
    auto moments_fit = [&](auto bconst) {
      constexpr int BB = decltype(bconst)::value;
      constexpr bool ALIGNED = BB >= 16;
      int T = 1;
      while (T < BB / 2 && T < 16 && n * (T * 2) <= 64) T *= 2;
      const int logT = __builtin_ctz((unsigned)T);
      for (int base = 0; base < n * T; base += 64) {
        const int idx = base + lane;
        const int e = idx >> logT, t = idx & (T - 1);
        uint32_t acc[12];
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[j] = 0u;
        if (e < n) {
          int X, Y;
          range_xy<BMAX, G::BMIN>(cur[e], rg, X, Y);
          const int dx = clampi(X - BB / 2, 0, rg.W - 2 * BB);
          const int dy = clampi(Y - BB / 2, 0, rg.H - 2 * BB);
          const int rx = X - rg.X0, ry = Y - rg.Y0;
          const int wx = (dx - rg.ax0) >> 1, wy = (dy - rg.ay0) >> 1;
          for (int i = t; i < BB / 2; i += T)
            accumulate_row_pair<BB, ALIGNED>(s_img, ry * G::TPITCH + rx, G::TPITCH, s_h0, wy * G::HP + wx,
                                             G::HP, s_h0t, wx * G::TP + wy, G::TP, i, acc);
        }
        team_reduce(acc, T);
        if (e < n && t == 0) {
          w_fit[e] = fit_phase1<BB>(acc, last, thr);
#pragma unroll
          for (int s = 0; s < 5; ++s) s_mom[wave][s][e] = acc[s];
        }
      }
    };
    if constexpr (BMAX >= 32) { if (B == 32) moments_fit(std::integral_constant<int, 32>{}); }
    if constexpr (BMAX >= 16 && G::BMIN <= 16) { if (B == 16) moments_fit(std::integral_constant<int, 16>{}); }
    if constexpr (BMAX >= 8 && G::BMIN <= 8) { if (B == 8) moments_fit(std::integral_constant<int, 8>{}); }
    if constexpr (G::BMIN <= 4) { if (B == 4) moments_fit(std::integral_constant<int, 4>{}); }
    wave_sync();

    // phase 2 of the parents that failed at level lev-1 (their children are
    // exactly the ranges just fitted, four per parent in Z order)
    if (lev >= 2 && a.phase2) {
      const int np = n >> 2;
      auto phase2 = [&](auto bconst) {
        constexpr int BB = decltype(bconst)::value;   // child side
        for (int p = lane; p < np; p += 64) {
          uint32_t mom[4][5];
#pragma unroll
          for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int s = 0; s < 5; ++s) mom[c][s] = s_mom[wave][s][4 * p + c];
          const int m = (int)w_pm[p];
          int O[4];
          uint32_t bits;
          if (fit_phase2<BB>(mom, m, lev - 1, a.thr[lev - 2], O, bits)) {
            const uint32_t pmeta = w_pmeta[p];
            int X, Y;
            range_xy<BMAX, G::BMIN>(pmeta, rg, X, Y);
            const int PB = 2 * BB;
            const int dx = clampi(X - PB / 2, 0, rg.W - 2 * PB);
            const int dy = clampi(Y - PB / 2, 0, rg.H - 2 * PB);
            const int cell = morton(pmeta);
            a.staging[tile_global(pmeta, rg) * G::CELLS + cell] =
                make_record(X, Y, dx, dy, lev - 2, 1, 0, (int)bits, m, O[0] - m, O[1] - m, O[2] - m);
            atomicOr(&s_mask[pmeta >> 16], 1ull << cell);
#pragma unroll
            for (int c = 0; c < 4; ++c) w_fit[4 * p + c] |= kFitDead;
          }
        }
      };
      if constexpr (BMAX >= 32 && G::BMIN <= 16) { if (B == 16) phase2(std::integral_constant<int, 16>{}); }
      if constexpr (BMAX >= 16 && G::BMIN <= 8) { if (B == 8) phase2(std::integral_constant<int, 8>{}); }
      if constexpr (BMAX >= 8 && G::BMIN <= 4) { if (B == 4) phase2(std::integral_constant<int, 4>{}); }
      wave_sync();
    }

    // store accepted ranges; compact failures (ballot prefix) into the
    // parent list and their children into the next level's list
    uint32_t nfail = 0;
    for (int base = 0; base < n; base += 64) {
      const int e = base + lane;
      bool fail = false;
      uint32_t meta = 0, fit = 0;
      if (e < n) {
        meta = cur[e];
        fit = w_fit[e];
        if (!(fit & kFitDead)) {
          if (fit & kFitAccept) {
            int X, Y;
            range_xy<BMAX, G::BMIN>(meta, rg, X, Y);
            const int dx = clampi(X - B / 2, 0, rg.W - 2 * B);
            const int dy = clampi(Y - B / 2, 0, rg.H - 2 * B);
            const int cell = morton(meta);
            a.staging[tile_global(meta, rg) * G::CELLS + cell] =
                make_record(X, Y, dx, dy, lev - 1, 0, (int)((fit >> 11) & 7u), (int)((fit >> 8) & 7u),
                            (int)(fit & 0xffu), 0, 0, 0);
            atomicOr(&s_mask[meta >> 16], 1ull << cell);
          } else {
            fail = true;
          }
        }
      }
      const uint64_t bal = __ballot(fail);
      const uint32_t q = nfail + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      if (fail) {
        w_pmeta[q] = meta;
        w_pm[q] = fit & 0xffu;
        const uint32_t half = (uint32_t)(B / 2 / G::BMIN);
        const uint32_t cx = meta & 0xffu, cy = (meta >> 8) & 0xffu, tile = meta & 0xffff0000u;
#pragma unroll
        for (uint32_t c = 0; c < 4; ++c)
          nxt[4 * q + c] = tile | ((cy + (c >> 1) * half) << 8) | (cx + (c & 1u) * half);
      }
      nfail += (uint32_t)__popcll(bal);
    }
    wave_sync();
    n = (int)(4 * nfail);
    if (last || n == 0) break;
  }

  // ---- publish the wave's tiles' occupancy masks
  wave_sync();
  if (lane < my_tiles) {
    const uint32_t meta = (uint32_t)(t_first + lane) << 16;
    a.masks[tile_global(meta, rg)] = s_mask[t_first + lane];
  }
}

__global__ void zero_u32_kernel(uint32_t* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Records per chunk of kChunkTiles tiles (one lane per tile).
__global__ __launch_bounds__(kChunkTiles) void chunk_count_kernel(const uint64_t* masks, uint64_t total_tiles,
                                                                 uint32_t* chunk_sum) {
  __shared__ uint32_t s_w[kChunkTiles / 64];
  const uint64_t tile = (uint64_t)blockIdx.x * kChunkTiles + threadIdx.x;
  uint32_t c = tile < total_tiles ? (uint32_t)__popcll(masks[tile]) : 0u;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kChunkTiles / 64; ++w) t += s_w[w];
    chunk_sum[blockIdx.x] = t;
  }
}

// Exclusive scan of the chunk counts (one workgroup): chunk_base[c] =
// records of all chunks before c; chunk_base[n] = total.
__global__ __launch_bounds__(1024) void chunk_scan_kernel(const uint32_t* chunk_sum, uint32_t n,
                                                         uint64_t* chunk_base) {
  __shared__ unsigned long long s_w[16];
  __shared__ unsigned long long s_carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (uint32_t c0 = 0; c0 < n; c0 += 1024) {
    const uint32_t c = c0 + tid;
    const unsigned long long v = c < n ? chunk_sum[c] : 0ull;
    unsigned long long incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned long long u = __shfl_up(incl, off);
      if (lane >= off) incl += u;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    unsigned long long pre = s_carry;
    for (int w = 0; w < wave; ++w) pre += s_w[w];
    if (c < n) chunk_base[c] = pre + incl - v;
    __syncthreads();
    if (tid == 1023) s_carry = pre + incl;
    __syncthreads();
  }
  if (tid == 0) chunk_base[n] = s_carry;
}

// One workgroup per kChunkTiles consecutive tiles (global order = image,
// then tile raster).  Stream position of a record = records of all earlier
// tiles + rank of its Morton cell among its tile's cells.  The workgroup
// scans its tiles' counts, then copies its contiguous output range with one
// record per lane (coalesced writes), locating each record's tile by binary
// search over the tile bases.
__global__ __launch_bounds__(256) void scatter_kernel(const ImgDev* imgs, uint32_t n_imgs,
                                                     uint64_t total_tiles, int cells,
                                                     const uint64_t* masks, const uint64_t* chunk_base,
                                                     const uint4* staging, uint4* out, uint64_t cap,
                                                     uint64_t* offsets) {
  __shared__ uint32_t s_wsum[4];
  __shared__ uint32_t s_tbase[kChunkTiles + 1];
  __shared__ unsigned long long s_mk[kChunkTiles];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t c0 = (uint64_t)blockIdx.x * kChunkTiles;
  const unsigned long long base = chunk_base[blockIdx.x];
  constexpr int PER = kChunkTiles / 256;
  uint32_t cnt[PER];
  uint32_t tsum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const uint64_t tile = c0 + (uint64_t)tid * PER + j;
    const unsigned long long m = tile < total_tiles ? masks[tile] : 0ull;
    s_mk[tid * PER + j] = m;
    cnt[j] = (uint32_t)__popcll(m);
    tsum += cnt[j];
  }
  // exclusive scan of tsum over the 256 lanes
  uint32_t incl = tsum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  if (lane == 63) s_wsum[wave] = incl;
  __syncthreads();
  uint32_t wpre = 0, total = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    wpre += w < wave ? s_wsum[w] : 0u;
    total += s_wsum[w];
  }
  uint32_t pos = wpre + incl - tsum;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    s_tbase[tid * PER + j] = pos;
    pos += cnt[j];
  }
  if (tid == 0) s_tbase[kChunkTiles] = total;
  __syncthreads();
  for (uint32_t r = tid; r < total; r += 256) {
    int lo = 0, hi = kChunkTiles - 1;      // last tile with base <= r
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_tbase[mid] <= r) lo = mid; else hi = mid - 1;
    }
    unsigned long long m = s_mk[lo];
    for (uint32_t k = r - s_tbase[lo]; k > 0; --k) m &= m - 1;
    const int cell = __builtin_ctzll(m);
    const unsigned long long o = base + r;
    if (o < cap) out[o] = staging[(c0 + lo) * (uint64_t)cells + cell];
  }
  for (uint32_t k = tid; k < n_imgs; k += 256) {
    const uint64_t tf = imgs[k].tile_first;
    if (tf >= c0 && tf < c0 + kChunkTiles) offsets[k] = base + s_tbase[tf - c0];
  }
  if (blockIdx.x == gridDim.x - 1 && tid == 0) offsets[n_imgs] = base + total;
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
                          const uint64_t* masks, uint32_t* chunk_sum, uint64_t* chunk_base, const uint4* staging,
                          uint4* out, uint64_t cap, uint64_t* offsets, hipStream_t s) {
  const unsigned grid = (unsigned)((total_tiles + kChunkTiles - 1) / kChunkTiles);
  hipLaunchKernelGGL(chunk_count_kernel, dim3(grid), dim3(kChunkTiles), 0, s, masks, total_tiles, chunk_sum);
  hipLaunchKernelGGL(chunk_scan_kernel, dim3(1), dim3(1024), 0, s, chunk_sum, grid, chunk_base);
  hipLaunchKernelGGL(scatter_kernel, dim3(grid), dim3(256), 0, s, imgs, n_imgs, total_tiles, cells, masks,
                     chunk_base, staging, out, cap, offsets);
  return hipGetLastError();
}

}  // namespace fe
