// Stream order (Sec. 3.3 stores the transforms depth first): the records
// that the fused encoder left in per-tile slots, indexed by Morton cell, are
// packed into one stream per image -- tiles in raster order, cells in
// Morton order inside a tile, images one after another -- with each
// image's first position in `offsets`.
#include <algorithm>

#include "fe_device.h"
#include "fe_internal.h"

namespace fe {
namespace {

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

// Images a chunk of kChunkTiles tiles can touch: every image has at least
// 2 x 2 top tiles.
constexpr int kChunkImgs = kChunkTiles / 4 + 1;

// Up to this many chunks the ordering runs as one kernel whose workgroups
// count the records before their chunk themselves (at most 16 k masks each).
constexpr unsigned kSmallChunks = 64;

// Up to this many chunks each workgroup adds up the per-chunk counts before
// its chunk itself (at most 4 k words) instead of a separate scan.
constexpr unsigned kSumChunks = 4096;

// Workgroups of the ordering kernel at most; each loops over its chunks.
constexpr unsigned kScatterGroups = 16384;

// Records copied per pass of a chunk.
constexpr int kPass = 1024;

// Per-lane share (of 256 lanes) of the record counts in p[0, n): U loads
// in flight per round, addresses clamped, so that no load waits for the one
// before it.  A lane's share (and a wave's) stays below 2^32: at most
// n / 256 entries (n <= kSumChunks chunk counts of at most 256 * 64 records
// each, or at most 64 * 256 masks of at most 64 records each).
__device__ __forceinline__ uint32_t count_of(uint32_t v) { return v; }
__device__ __forceinline__ uint32_t count_of(uint64_t mask) { return (uint32_t)__popcll(mask); }
template <int U, typename T>
__device__ __forceinline__ uint32_t lane_sum(const T* p, uint64_t n, int tid) {
  uint32_t acc = 0;
  for (uint64_t i0 = 0; i0 < n; i0 += 256u * U) {
    T x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = i0 + (uint64_t)tid + 256u * (uint64_t)u;
      x[u] = p[i < n ? i : n - 1u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += i0 + (uint64_t)tid + 256u * (uint64_t)u < n ? count_of(x[u]) : 0u;
  }
  return acc;
}

// One workgroup per kChunkTiles consecutive tiles (global order = image,
// then tile raster).  Stream position of a record = records of all earlier
// tiles + rank of its Morton cell among its tile's cells.  One lane per
// tile: the tile's mask, its first slot and its record count; a scan of the
// counts gives every tile's first position.  Then, per pass of kPass
// records, each tile lane lists the slots of its records that fall in the
// pass (lowest cell first), and the workgroup copies the pass with one
// record per lane (coalesced writes).
//
// PREFIX says where the records before a chunk come from (the variants have
// no branches around their first loads, which would make the compiler wait
// for each load before the next): kPrefixMasks counts them from the masks
// (few chunks), kPrefixSums adds up the per-chunk counts, kPrefixBase reads
// them from the scan of those counts.  MULTI: several images (chunk_img
// gives each chunk's first one); otherwise one image, entry 0.
constexpr int kPrefixMasks = 0, kPrefixSums = 1, kPrefixBase = 2;
template <int PREFIX, bool MULTI>
__global__ __launch_bounds__(256) void scatter_kernel(const ImgDev* imgs, uint32_t n_imgs,
                                                     const uint32_t* chunk_img, uint64_t total_tiles,
                                                     uint32_t n_chunks, int cells, int gx, int gy,
                                                     const uint64_t* masks, const uint32_t* chunk_sum,
                                                     const uint64_t* chunk_base, const uint4* staging, uint4* out,
                                                     uint64_t cap, uint64_t* offsets) {
  static_assert(kChunkTiles == 256, "one tile per lane");
  __shared__ uint32_t s_wsum[4];
  __shared__ uint32_t s_tbase[kChunkTiles];
  __shared__ unsigned long long s_rslot[kPass];
  __shared__ unsigned long long s_tf[kChunkImgs];      // the chunk's images: first tile,
  __shared__ uint32_t s_tx[kChunkImgs], s_gx[kChunkImgs], s_wf[kChunkImgs];   // tiles / blocks per row, first block
  __shared__ uint32_t s_red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // a workgroup orders chunk blockIdx.x, then every gridDim.x-th chunk after
  // it (fewer, longer-lived workgroups: short ones are bound by their launch)
  for (uint32_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
  const uint64_t c0 = (uint64_t)chunk * kChunkTiles;
  // the loads that depend on nothing are issued first (the chunk's first
  // image, the counts before the chunk, this lane's tile mask), so that the
  // image entries, which wait for the first, are the only second round trip
  uint32_t k0 = 0;
  if constexpr (MULTI) k0 = chunk_img[chunk];
  const uint64_t tile = c0 + (uint64_t)tid;
  const bool has_tile = tile < total_tiles;
  unsigned long long base = 0;   // kPrefixMasks / kPrefixSums: read after the barrier below
  uint32_t acc = 0;
  // the records of all earlier tiles: from the scan, from the per-chunk
  // counts (one round of loads, added up once the image entries are on
  // their way), or (few chunks) from the masks
  constexpr int U = kSumChunks / 256;
  uint32_t cs[U];
  if constexpr (PREFIX == kPrefixBase) base = chunk_base[chunk];
  if constexpr (PREFIX == kPrefixSums) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = (uint32_t)tid + 256u * (uint32_t)u;
      cs[u] = chunk_sum[i < chunk ? i : 0u];
    }
  }
  if constexpr (PREFIX == kPrefixMasks) acc = lane_sum<8>(masks, c0, tid);
  const unsigned long long m_raw = masks[has_tile ? tile : 0u];
  const int nk = (int)min<uint32_t>((uint32_t)kChunkImgs, n_imgs - k0);
  const ImgDev im = imgs[k0 + (uint32_t)min(tid, nk - 1)];
  if constexpr (PREFIX == kPrefixSums) {
#pragma unroll
    for (int u = 0; u < U; ++u) acc += (uint32_t)tid + 256u * (uint32_t)u < chunk ? cs[u] : 0u;
  }
  if constexpr (PREFIX != kPrefixBase) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += (uint32_t)__shfl_xor((int)acc, off);
    if (lane == 0) s_red[wave] = acc;
  }
  if (tid < nk) {
    s_tf[tid] = im.tile_first;
    s_tx[tid] = im.tiles_x;
    s_gx[tid] = im.groups_x;
    s_wf[tid] = im.wg_first;
  }
  __syncthreads();
  if constexpr (PREFIX != kPrefixBase) base = (unsigned long long)s_red[0] + s_red[1] + s_red[2] + s_red[3];
  const int nt = gx * gy;
  unsigned long long m = 0ull, slot = 0ull;
  uint32_t stride = 0;   // slots between cells of the tile
  if (has_tile) {
    m = m_raw;
    // the tile's image: the last of the chunk's images starting at or before it
    int k = 0;
    while (k + 1 < nk && s_tf[k + 1] <= tile) ++k;
    const uint32_t local = (uint32_t)(tile - s_tf[k]);
    const uint32_t ty = local / s_tx[k], tx = local - ty * s_tx[k];
    const uint32_t by = ty / (uint32_t)gy, bx = tx / (uint32_t)gx;
    const uint64_t blk = (uint64_t)s_wf[k] + (uint64_t)by * s_gx[k] + bx;
    // the block's slots: one whole-tile slot per tile, then each tile's
    // cells; a tile whose only record covers it (mask 1) uses the former
    const uint64_t t = (uint64_t)(ty - by * (uint32_t)gy) * (uint64_t)gx + (tx - bx * (uint32_t)gx);
    const uint64_t blk0 = blk * (uint64_t)nt * (uint64_t)(cells + 1);
    slot = m == 1ull ? blk0 + t : blk0 + (uint64_t)nt + t * (uint64_t)cells;
    stride = m == 1ull ? 0u : 1u;
  }
  const uint32_t cnt = (uint32_t)__popcll(m);
  // exclusive scan of the counts over the 256 lanes
  uint32_t incl = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  if (lane == 63) s_wsum[wave] = incl;
  __syncthreads();
  uint32_t pos = incl - cnt, total = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    pos += w < wave ? s_wsum[w] : 0u;
    total += s_wsum[w];
  }
  s_tbase[tid] = pos;
  for (uint32_t r0 = 0; r0 < total; r0 += kPass) {
    // this tile's records inside [r0, r0 + kPass)
    if (cnt && pos < r0 + kPass && pos + cnt > r0) {
      unsigned long long mm = m;
      uint32_t r = pos;
      for (; r < r0; ++r) mm &= mm - 1;
      for (; mm && r < r0 + kPass; ++r) {
        s_rslot[r - r0] = slot + (unsigned long long)__builtin_ctzll(mm) * stride;
        mm &= mm - 1;
      }
    }
    __syncthreads();
    const uint32_t n = min<uint32_t>((uint32_t)kPass, total - r0);
    // all loads first (index clamped into the pass), then the stores; named
    // values, not an array, which the compiler would place in scratch
    static_assert(kPass == 4 * 256, "four records per lane");
    const uint32_t ra = (uint32_t)tid, rb = ra + 256u, rc = ra + 512u, rd = ra + 768u;
    const uint4 va = staging[s_rslot[ra < n ? ra : n - 1u]];
    const uint4 vb = staging[s_rslot[rb < n ? rb : n - 1u]];
    const uint4 vc = staging[s_rslot[rc < n ? rc : n - 1u]];
    const uint4 vd = staging[s_rslot[rd < n ? rd : n - 1u]];
    const unsigned long long o = base + r0 + ra;
    if (ra < n && o < cap) out[o] = va;
    if (rb < n && o + 256u < cap) out[o + 256u] = vb;
    if (rc < n && o + 512u < cap) out[o + 512u] = vc;
    if (rd < n && o + 768u < cap) out[o + 768u] = vd;
    __syncthreads();
  }
  // the first position of every image that starts in this chunk (all of
  // them are among the chunk's image entries)
  if (tid < nk) {
    const uint64_t tf = s_tf[tid];
    if (tf >= c0 && tf < c0 + kChunkTiles) offsets[k0 + (uint32_t)tid] = base + s_tbase[tf - c0];
  }
  if (chunk == n_chunks - 1 && tid == 0) offsets[n_imgs] = base + total;
  __syncthreads();   // the LDS arrays are reused by the next chunk
  }
}

}  // namespace

hipError_t launch_zero_u32(uint32_t* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

template <int PREFIX>
static void launch_scatter_as(unsigned sgrid, const ImgDev* imgs, uint32_t n_imgs, const uint32_t* chunk_img,
                              uint64_t total_tiles, unsigned grid, int cells, TileShape shape, const uint64_t* masks,
                              const uint32_t* chunk_sum, const uint64_t* chunk_base, const uint4* staging, uint4* out,
                              uint64_t cap, uint64_t* offsets, hipStream_t s) {
  if (chunk_img)
    hipLaunchKernelGGL((scatter_kernel<PREFIX, true>), dim3(sgrid), dim3(256), 0, s, imgs, n_imgs, chunk_img,
                       total_tiles, grid, cells, shape.gx, shape.gy, masks, chunk_sum, chunk_base, staging, out, cap,
                       offsets);
  else
    hipLaunchKernelGGL((scatter_kernel<PREFIX, false>), dim3(sgrid), dim3(256), 0, s, imgs, n_imgs, chunk_img,
                       total_tiles, grid, cells, shape.gx, shape.gy, masks, chunk_sum, chunk_base, staging, out, cap,
                       offsets);
}

hipError_t launch_scatter(const ImgDev* imgs, uint32_t n_imgs, const uint32_t* chunk_img, uint64_t total_tiles,
                          int cells, TileShape shape, const uint64_t* masks, uint32_t* chunk_sum,
                          uint64_t* chunk_base, const uint4* staging, uint4* out, uint64_t cap, uint64_t* offsets,
                          hipStream_t s) {
  const unsigned grid = (unsigned)((total_tiles + kChunkTiles - 1) / kChunkTiles);
  const unsigned sgrid = grid < kScatterGroups ? grid : kScatterGroups;
  if (grid <= kSmallChunks) {
    // one kernel: each chunk counts the records before it from the masks
    launch_scatter_as<kPrefixMasks>(sgrid, imgs, n_imgs, chunk_img, total_tiles, grid, cells, shape, masks, nullptr,
                                    nullptr, staging, out, cap, offsets, s);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(chunk_count_kernel, dim3(grid), dim3(kChunkTiles), 0, s, masks, total_tiles, chunk_sum);
  if (grid <= kSumChunks) {
    // each chunk adds up the counts of the chunks before it
    launch_scatter_as<kPrefixSums>(sgrid, imgs, n_imgs, chunk_img, total_tiles, grid, cells, shape, masks, chunk_sum,
                                   nullptr, staging, out, cap, offsets, s);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(chunk_scan_kernel, dim3(1), dim3(1024), 0, s, chunk_sum, grid, chunk_base);
  launch_scatter_as<kPrefixBase>(sgrid, imgs, n_imgs, chunk_img, total_tiles, grid, cells, shape, masks, nullptr,
                                 chunk_base, staging, out, cap, offsets, s);
  return hipGetLastError();
}

}  // namespace fe
