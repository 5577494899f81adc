// The 2 x 2 level of quadtrees that reach the paper's smallest ranges
// (Sec. 3.3: four levels, 16 x 16 down to 2 x 2).
//
// The fused encoder runs such a tree from B_max down to 4 x 4 (its EXT
// form): it tests the 4 x 4 level against its threshold like any other
// level and lists the 4 x 4 ranges that fail.  This kernel takes that list,
// four lanes per listed range, one per 2 x 2 child (Z order).  A 2 x 2
// child at x has its co-centred domain at x - 1, an odd origin, so its
// domain means are formed here from the image's pixels (16 bytes per child,
// read through the L2), not from the fused encoder's H0.
//
// Each lane forms its child's moments (Sum r, Sum r^2, Sum d, Sum d^2 and
// the eight Sum r T_e(d)) and phase-1 fit (the last level, always stored;
// Sec. 3).  The four lanes exchange their identity moments and each decides
// Technique 1 for the parent (Sec. 3.1-3.3) with the level's contrast set
// and eq. (1); if it holds, the first lane stores the parent's phase-2
// record in the parent's first cell, otherwise every lane stores its child.
// Occupancy bits go to the tile masks with one 64-bit atomic OR per range
// (the fused encoder has already written its own bits).
#include "fe_device.h"
#include "fe_internal.h"

namespace fe {
namespace {

constexpr unsigned kFinishGroups = 2048;

__global__ __launch_bounds__(256) void fine_finish_kernel(FinishArgs a) {
  const uint32_t count = *a.count;
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  // lanes 4 e .. 4 e + 3 of a wave take listed range e: a lane's group of
  // four stays together through the loop (the stride is a multiple of 64)
  for (uint64_t gid = (uint64_t)blockIdx.x * 256u + threadIdx.x; gid < 4ull * count; gid += stride) {
    const uint4 ent = a.list[gid >> 2];
    const int c = (int)(gid & 3u);
    const uint32_t tile = ent.z;
    // the tile's image: the last one whose first tile is at or before it
    int lo = 0, hi = (int)a.n_imgs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.imgs[mid].tile_first <= tile) lo = mid; else hi = mid - 1;
    }
    const ImgDev im = a.imgs[lo];
    const uint32_t flags = a.per_image ? im.fine_flags : (a.phase2 ? FE_PHASE2 : 0u) | (a.identity_only ? FE_IDENTITY_ONLY : 0u);
    const uint32_t thr = a.per_image ? im.fine_thr : a.thr;
    const int W = (int)im.width, H = (int)im.height;
    const int px = (int)(ent.x & 0xffffu), py = (int)(ent.x >> 16);
    const int cx = px + 2 * (c & 1), cy = py + 2 * (c >> 1);
    const int ox = clampi(cx - 1, 0, W - 4), oy = clampi(cy - 1, 0, H - 4);
    const uint8_t* img = im.data;
    const size_t st = im.stride;
    uint32_t r[2][2], d[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        r[i][j] = img[(size_t)(cy + i) * st + (size_t)(cx + j)];
        const uint8_t* q = img + (size_t)(oy + 2 * i) * st + (size_t)(ox + 2 * j);
        d[i][j] = ((uint32_t)q[0] + q[1] + q[st] + q[st + 1] + 2u) >> 2;
      }
    }
    uint32_t acc[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) acc[j] = 0u;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const uint32_t v = r[i][j];
        const int i2 = 1 - i, j2 = 1 - j;
        acc[0] += v;
        acc[1] += v * v;
        acc[2] += d[i][j];
        acc[3] += d[i][j] * d[i][j];
        acc[4] += v * d[i][j];     // T_0: d[i][j]
        acc[5] += v * d[i][j2];    // T_1: d[i][1-j]
        acc[6] += v * d[i2][j];    // T_2: d[1-i][j]
        acc[7] += v * d[i2][j2];   // T_3: d[1-i][1-j]
        acc[8] += v * d[j][i];     // T_4: d[j][i]
        acc[9] += v * d[j2][i];    // T_5: d[1-j][i]
        acc[10] += v * d[j][i2];   // T_6: d[j][1-i]
        acc[11] += v * d[j2][i2];  // T_7: d[1-j][1-i]
      }
    }
    if (flags & FE_IDENTITY_ONLY) {
#pragma unroll
      for (int j = 5; j < 12; ++j) acc[j] = acc[4];
    }
    const uint32_t fit = fit_phase1<2>(acc, true, 0u);
    const int m = (int)(ent.w & 0xffu);
    const int cell0 = (int)((ent.w >> 8) & 0xffu);
    // Technique 1 for the parent from the four children's identity moments
    bool dead = false;
    int O[4] = {0, 0, 0, 0};
    uint32_t bits = 0;
    if (flags & FE_PHASE2) {
      uint32_t mom[4][5];
      const int g0 = (int)(threadIdx.x & 63u) & ~3;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int j = 0; j < 5; ++j) mom[k][j] = (uint32_t)__shfl((int)acc[j], g0 + k);
      }
      dead = fit_phase2<2>(mom, m, (int)a.level, thr, O, bits);
    }
    if (dead) {
      // a listed range that is a whole top tile (trees 4 -> 2) keeps its
      // record in its block's whole-tile slot, not at its first child's
      uint64_t pslot = ent.y;
      if (a.level == 1) {
        const uint64_t per = (uint64_t)a.nt * (a.cells + 1u);
        const uint64_t blk = pslot / per;
        pslot = blk * per + (pslot - blk * per - a.nt) / a.cells;
      }
      if (c == 0)
        a.staging[pslot] = make_record(px, py, clampi(px - 2, 0, W - 8), clampi(py - 2, 0, H - 8), (int)a.level - 1,
                                       1, 0, (int)bits, m, O[0] - m, O[1] - m, O[2] - m);
    } else {
      a.staging[(uint64_t)ent.y + (uint64_t)c] =
          make_record(cx, cy, ox, oy, (int)a.level, 0, (int)((fit >> 11) & 7u), (int)((fit >> 8) & 7u),
                      (int)(fit & 0xffu), 0, 0, 0);
    }
    // the parent's cell alone, or its four children's: one atomic per range
    if (c == 0)
      atomicOr(reinterpret_cast<unsigned long long*>(a.masks + tile), (dead ? 1ull : 0xfull) << cell0);
  }
}

}  // namespace

hipError_t launch_fine_finish(const FinishArgs& a, uint64_t max_entries, hipStream_t s) {
  if (max_entries == 0) return hipSuccess;
  const uint64_t want = (4 * max_entries + 255) / 256;
  const unsigned groups = (unsigned)(want < kFinishGroups ? want : kFinishGroups);
  hipLaunchKernelGGL(fine_finish_kernel, dim3(groups), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace fe
