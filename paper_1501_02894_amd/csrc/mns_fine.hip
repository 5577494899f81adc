// MNS quadtree down to the paper's smallest ranges, 2 x 2 (Sec. 3.3: four
// levels, 16 x 16 to 2 x 2).
//
// A 2 x 2 range at x has its co-centred domain at x - 1, so the 2 x 2 means
// of its domain lie on another pixel phase than the H0 image the fused
// encoder stages, and a 2 x 2 range is half a packed dword wide.  This
// encoder therefore works on pixels.  One wave owns one top tile: it stages
// the tile's 2 B_max x 2 B_max domain region (which holds the tile and every
// descendant's co-centred domain) in LDS and forms each range's domain block
// (the 2 x 2 means, at whichever phase) from those pixels once.
//
// Per level (B = B_max >> (l - 1)), a team of T = min(64, B^2) lanes takes
// one range, B^2 / T pixels per lane: each lane adds r, r^2, d, d^2 and the
// eight isometric products r T_e(d) of its pixels, a butterfly over the team
// gives the totals and the phase-1 fit is the fused encoder's (Sec. 3).
// Phase 2 (Sec. 3.1-3.3) of the ranges that failed one level up is decided
// from the identity moments of their children, which this level has just
// formed (every child of a failed range is listed, four in a row).  Accepted
// ranges go to the tile's record slots by the Morton code of their top-left
// 2 x 2 cell; the ordering kernels then pack the slots into stream order.
#include "fe_device.h"
#include "fe_internal.h"

namespace fe {
namespace {

constexpr int kFineWaves = 4;

template <int BMAX>
struct FineLds {
  static constexpr int R = 2 * BMAX;                   // staged region side (px)
  static constexpr int MAXE = (BMAX / 2) * (BMAX / 2);  // ranges of one level at most
  uint8_t px[R * R];
  uint8_t dblk[256];           // domain blocks of the ranges of one pass
  uint16_t list[2][MAXE];      // ranges: lx | ly << 8, pixels inside the tile
  uint32_t fit[MAXE];          // phase-1 fit word per range
  uint32_t mom[MAXE][5];       // identity moments per range (phase 2 of the parents)
  uint16_t par[MAXE / 4];      // failed ranges of the level above, in list order
  uint32_t pfit[MAXE / 4];     // their phase-1 fit words
  uint32_t dead[MAXE / 4];     // 1 when phase 2 stored that parent
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off);
  return v;
}

template <int BITS>
__device__ __forceinline__ int morton2(int cx, int cy) {
  int code = 0;
#pragma unroll
  for (int b = 0; b < BITS; ++b) code |= (((cx >> b) & 1) << (2 * b)) | (((cy >> b) & 1) << (2 * b + 1));
  return code;
}

struct Tile {
  int X, Y;         // tile origin (pixels)
  int rx, ry;       // staged region origin (pixels)
  uint64_t slot0;   // first record slot of the tile
};

// One level of side B over the wave's list list[buf][0 .. nc).  Returns the
// number of ranges listed for the next level (in list[buf ^ 1]).
template <int BMAX, int B>
__device__ __forceinline__ int fine_level(FineLds<BMAX>& S, const FineArgs& a, const Tile& t, int buf, int nc,
                                          uint64_t& mask) {
  constexpr int R = 2 * BMAX;
  constexpr int LMAX = Log2<BMAX>::value;               // levels BMAX .. 2
  constexpr int level = Log2<BMAX / B>::value + 1;      // 1-based
  constexpr bool last = level == LMAX;
  constexpr int N = B * B, T = N < 64 ? N : 64, PX = N / T, RP = 64 / T;
  constexpr int CELL_BITS = LMAX - 1;
  const int lane = threadIdx.x & 63, sub = lane & (T - 1);
  const int W = (int)a.w, H = (int)a.h;
  const bool p2 = level > 1 && a.phase2 != 0;

  // moments and phase-1 fit of every listed range; each pass first writes
  // its ranges' B x B domain blocks d (2 x 2 means) to dblk, then reads
  // them under the eight isometries
  const bool iso = a.identity_only == 0;
  for (int base = 0; base < nc; base += RP) {
    const int idx = base + lane / T;
    const bool valid = idx < nc;
    const int db = (lane / T) * N;   // this range's block in dblk
    uint32_t acc[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) acc[j] = 0u;
    uint32_t rv[PX];
    if (valid) {
      const uint32_t ent = S.list[buf][idx];
      const int x = t.X + (int)(ent & 0xffu), y = t.Y + (int)(ent >> 8);
      const int qx = x - t.rx, qy = y - t.ry;
      const int ox = clampi(x - B / 2, 0, W - 2 * B) - t.rx, oy = clampi(y - B / 2, 0, H - 2 * B) - t.ry;
#pragma unroll
      for (int u = 0; u < PX; ++u) {
        const int q = sub + T * u;
        const int i = q / B, j = q % B;
        const int o = (oy + 2 * i) * R + ox + 2 * j;
        const uint32_t d = ((uint32_t)S.px[o] + S.px[o + 1] + S.px[o + R] + S.px[o + R + 1] + 2u) >> 2;
        S.dblk[db + q] = (uint8_t)d;
        rv[u] = S.px[(qy + i) * R + qx + j];
        acc[0] += rv[u];
        acc[1] += rv[u] * rv[u];
        acc[2] += d;
        acc[3] += d * d;
        acc[4] += rv[u] * d;          // T_0: d[i][j]
      }
    }
    wave_lds_sync();
    if (valid && iso) {
      auto dm = [&](int i, int j) -> uint32_t { return S.dblk[db + i * B + j]; };
#pragma unroll
      for (int u = 0; u < PX; ++u) {
        const int q = sub + T * u;
        const int i = q / B, j = q % B, i2 = B - 1 - i, j2 = B - 1 - j;
        const uint32_t r = rv[u];
        acc[5] += r * dm(i, j2);      // T_1: d[i][B-1-j]
        acc[6] += r * dm(i2, j);      // T_2: d[B-1-i][j]
        acc[7] += r * dm(i2, j2);     // T_3: d[B-1-i][B-1-j]
        acc[8] += r * dm(j, i);       // T_4: d[j][i]
        acc[9] += r * dm(j2, i);      // T_5: d[B-1-j][i]
        acc[10] += r * dm(j, i2);     // T_6: d[j][B-1-i]
        acc[11] += r * dm(j2, i2);    // T_7: d[B-1-j][B-1-i]
      }
    }
    wave_lds_sync();   // dblk is rewritten by the next pass
    // totals over the team: DPP inside rows of 16 lanes, then across rows
    team_reduce(acc, T < 16 ? T : 16);
#pragma unroll
    for (int off = 16; off < T; off <<= 1) {
#pragma unroll
      for (int j = 0; j < 12; ++j) acc[j] += __shfl_xor(acc[j], off);
    }
    if (valid && sub == 0) {
      if (!iso) {
#pragma unroll
        for (int j = 5; j < 12; ++j) acc[j] = acc[4];
      }
      S.fit[idx] = fit_phase1<B>(acc, last, last ? 0u : a.thr[level - 1]);
      if (p2) {
#pragma unroll
        for (int j = 0; j < 5; ++j) S.mom[idx][j] = acc[j];
      }
    }
  }
  wave_lds_sync();

  // phase 2 of the parents: children 4p .. 4p + 3 belong to parent p
  uint64_t bits = 0;
  if constexpr (level > 1) {
    if (p2) {
      const int np = nc >> 2;
      if (lane < np) {
        uint32_t mom[4][5];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
          for (int j = 0; j < 5; ++j) mom[c][j] = S.mom[4 * lane + c][j];
        }
        const int m = (int)(S.pfit[lane] & 0xffu);
        int O[4];
        uint32_t cbits;
        const bool ok = fit_phase2<B>(mom, m, level - 1, a.thr[level - 2], O, cbits);
        S.dead[lane] = ok ? 1u : 0u;
        if (ok) {
          const uint32_t pe = S.par[lane];
          const int plx = (int)(pe & 0xffu), ply = (int)(pe >> 8);
          const int x = t.X + plx, y = t.Y + ply;
          const int cell = morton2<CELL_BITS>(plx >> 1, ply >> 1);
          a.staging[t.slot0 + (uint64_t)cell] =
              make_record(x, y, clampi(x - B, 0, W - 4 * B), clampi(y - B, 0, H - 4 * B), level - 2, 1, 0,
                          (int)cbits, m, O[0] - m, O[1] - m, O[2] - m);
          bits |= 1ull << cell;
        }
      }
      wave_lds_sync();
    }
  }

  // store the accepted ranges; list the children of the failed ones
  bool fail = false;
  if (lane < nc) {
    const bool dead = p2 && S.dead[lane >> 2] != 0u;
    if (!dead) {
      const uint32_t f = S.fit[lane];
      if (f & kFitAccept) {
        const uint32_t ent = S.list[buf][lane];
        const int lx = (int)(ent & 0xffu), ly = (int)(ent >> 8);
        const int x = t.X + lx, y = t.Y + ly;
        const int cell = morton2<CELL_BITS>(lx >> 1, ly >> 1);
        a.staging[t.slot0 + (uint64_t)cell] =
            make_record(x, y, clampi(x - B / 2, 0, W - 2 * B), clampi(y - B / 2, 0, H - 2 * B), level - 1, 0,
                        (int)((f >> 11) & 7u), (int)((f >> 8) & 7u), (int)(f & 0xffu), 0, 0, 0);
        bits |= 1ull << cell;
      } else {
        fail = !last;
      }
    }
  }
  mask |= wave_or(bits);
  if constexpr (last) {
    return 0;
  } else {
    const uint64_t fb = __ballot(fail);
    if (fail) {
      const int pos = __popcll(fb & ((1ull << lane) - 1ull));
      const uint32_t ent = S.list[buf][lane];
      S.par[pos] = (uint16_t)ent;
      S.pfit[pos] = S.fit[lane];
      constexpr int h = B / 2;
      const int lx = (int)(ent & 0xffu), ly = (int)(ent >> 8);
#pragma unroll
      for (int c = 0; c < 4; ++c)
        S.list[buf ^ 1][4 * pos + c] = (uint16_t)((lx + (c & 1) * h) | ((ly + (c >> 1) * h) << 8));
    }
    wave_lds_sync();
    return 4 * __popcll(fb);
  }
}

template <int BMAX, int B>
__device__ __forceinline__ void fine_levels(FineLds<BMAX>& S, const FineArgs& a, const Tile& t, int buf, int nc,
                                            uint64_t& mask) {
  const int next = fine_level<BMAX, B>(S, a, t, buf, nc, mask);
  if constexpr (B > 2) {
    if (next > 0) fine_levels<BMAX, B / 2>(S, a, t, buf ^ 1, next, mask);
  }
}

template <int BMAX>
__global__ __launch_bounds__(64 * kFineWaves) void mns_fine_kernel(FineArgs a) {
  constexpr int R = 2 * BMAX;
  constexpr int CELLS = (BMAX / 2) * (BMAX / 2);
  __shared__ FineLds<BMAX> s_lds[kFineWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t tile = blockIdx.x * kFineWaves + (uint32_t)wave;
  if (tile >= a.tiles) return;   // waves never wait on each other
  FineLds<BMAX>& S = s_lds[wave];
  const int W = (int)a.w, H = (int)a.h;
  Tile t;
  t.X = (int)(tile % a.tiles_x) * BMAX;
  t.Y = (int)(tile / a.tiles_x) * BMAX;
  t.rx = clampi(t.X - BMAX / 2, 0, W - 2 * BMAX);
  t.ry = clampi(t.Y - BMAX / 2, 0, H - 2 * BMAX);
  t.slot0 = (uint64_t)tile * CELLS;
  if constexpr (BMAX >= 8) {
    // rx is a multiple of 4 (X - BMAX / 2 or W - 2 BMAX), as are the
    // stride and the image address: whole dwords
    uint32_t* px4 = reinterpret_cast<uint32_t*>(S.px);
    for (int k = lane; k < R * R / 4; k += 64) {
      const int row = k / (R / 4), c4 = k % (R / 4);
      px4[k] = *reinterpret_cast<const uint32_t*>(a.img + (size_t)(t.ry + row) * a.stride + (size_t)(t.rx + 4 * c4));
    }
  } else {
    for (int k = lane; k < R * R; k += 64) S.px[k] = a.img[(size_t)(t.ry + k / R) * a.stride + (size_t)(t.rx + k % R)];
  }
  if (lane == 0) S.list[0][0] = 0;
  wave_lds_sync();
  uint64_t mask = 0;
  fine_levels<BMAX, BMAX>(S, a, t, 0, 1, mask);
  if (lane == 0) a.masks[tile] = mask;
}

template <int BMAX>
hipError_t launch_fine(const FineArgs& a, hipStream_t s) {
  const unsigned groups = (unsigned)((a.tiles + kFineWaves - 1) / kFineWaves);
  hipLaunchKernelGGL(mns_fine_kernel<BMAX>, dim3(groups), dim3(64 * kFineWaves), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mns_fine(int b_max, const FineArgs& a, hipStream_t s) {
  if (a.tiles == 0) return hipSuccess;
  switch (b_max) {
    case 4: return launch_fine<4>(a, s);
    case 8: return launch_fine<8>(a, s);
    case 16: return launch_fine<16>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fe
