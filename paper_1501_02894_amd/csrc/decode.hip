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
  if (B < 4 || (f.x % B) || (f.y % B) || f.x + B > W || f.y + B > H) return true;
  if (f.flags == 0) {
    if (f.iso > 7 || f.s_idx > 7) return true;
    if (f.dx + 2 * B > W || f.dy + 2 * B > H) return true;
    if (f.d0 || f.d1 || f.d2) return true;
    return false;
  }
  if (B < 8 || f.level > 2 || f.iso != 0 || f.s_idx > 15) return true;
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

__global__ __launch_bounds__(256) void fill_kernel(uint8_t* dst, const uint8_t* src, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src ? src[i] : (uint8_t)128;
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

}  // namespace

hipError_t launch_decode_check(const DecodeArgs& a, uint32_t* bad, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(check_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, bad);
  return hipGetLastError();
}

hipError_t launch_decode_fill(uint8_t* dst, const uint8_t* src, uint32_t w, uint32_t h, hipStream_t s) {
  const uint64_t n = (uint64_t)w * h;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
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
