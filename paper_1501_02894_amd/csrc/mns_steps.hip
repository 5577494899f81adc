// Stand-alone steps of the MNS path: the domain-pyramid downsample (Sec. 3,
// 2 x 2 mean filter) and the moments of an explicit list of ranges against
// their co-centred domains.  The encoder fuses both into its tile kernel;
// these entry points run the same arithmetic on their own.
#include "fe_device.h"
#include "fe_internal.h"

namespace fe {
namespace {

// Each lane forms four H0 pixels (an 8 x 2 pixel group) with two 8-byte
// row reads when the group lies inside the image, else byte by byte.
__global__ __launch_bounds__(256) void downsample_kernel(const uint8_t* img, uint32_t w, uint32_t h,
                                                        uint32_t stride, uint8_t* out) {
  const uint32_t hw = w >> 1, hh = h >> 1;
  const uint32_t groups = (hw + 3) >> 2;
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)groups * hh) return;
  const uint32_t j = (uint32_t)(idx / groups), g = (uint32_t)(idx - (uint64_t)j * groups);
  const uint32_t x = 8 * g;
  const uint8_t* p0 = img + (size_t)(2 * j) * stride + x;
  const uint8_t* p1 = p0 + stride;
  uint8_t* o = out + (size_t)j * hw + 4 * g;
  if (x + 8 <= w) {
    const uint32_t* q0 = reinterpret_cast<const uint32_t*>(p0);
    const uint32_t* q1 = reinterpret_cast<const uint32_t*>(p1);
    const uint32_t v = mean2x2_x4(q0[0], q0[1], q1[0], q1[1]);
    o[0] = (uint8_t)v;
    o[1] = (uint8_t)(v >> 8);
    o[2] = (uint8_t)(v >> 16);
    o[3] = (uint8_t)(v >> 24);
  } else {
    for (uint32_t i = 0; 4 * g + i < hw && i < 4; ++i) {
      const uint32_t s = p0[2 * i] + p0[2 * i + 1] + p1[2 * i] + p1[2 * i + 1] + 2u;
      o[i] = (uint8_t)(s >> 2);
    }
  }
}

// One wave per range.  The range is copied into LDS, the B x B domain
// window (2 x 2 means of the 2B x 2B co-centred domain) and its transpose
// are formed in LDS at the same byte alignment they have inside the
// encoder's H0, and the team/row-pair accumulation of the encoder is run.
template <int B>
__global__ __launch_bounds__(256) void range_moments_kernel(const uint8_t* img, uint32_t w, uint32_t h,
                                                           uint32_t stride, const uint32_t* xy,
                                                           uint32_t count, uint32_t* mom) {
  constexpr int RP = B + 4;             // range pitch
  constexpr int HP = B + 12;            // window pitch (room for a 0..3 byte shift)
  constexpr int IMG_W = B * RP / 4 + 4;
  constexpr int H0_W = B * HP / 4 + 4;
  __shared__ uint32_t s_img[4][IMG_W];
  __shared__ uint32_t s_h0[4][H0_W];
  __shared__ uint32_t s_h0t[4][H0_W];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t r = (uint64_t)blockIdx.x * 4 + wave;
  if (r >= count) return;   // whole wave leaves together
  const uint32_t v = xy[r];
  const int x = (int)(v & 0xffffu), y = (int)(v >> 16);
  const bool ok = (x % B == 0) && (y % B == 0) && x + B <= (int)w && y + B <= (int)h &&
                  (int)w >= 2 * B && (int)h >= 2 * B;
  uint32_t acc[12];
#pragma unroll
  for (int j = 0; j < 12; ++j) acc[j] = 0u;
  if (ok) {
    const int dx = clampi(x - B / 2, 0, (int)w - 2 * B);
    const int dy = clampi(y - B / 2, 0, (int)h - 2 * B);
    const int sx = (dx >> 1) & 3, sy = (dy >> 1) & 3;   // byte alignment inside H0 / H0^T rows
    uint8_t* ib = reinterpret_cast<uint8_t*>(s_img[wave]);
    uint8_t* hb = reinterpret_cast<uint8_t*>(s_h0[wave]);
    uint8_t* tb = reinterpret_cast<uint8_t*>(s_h0t[wave]);
    for (int p = lane; p < B * B; p += 64) {
      const int i = p / B, j = p - (p / B) * B;
      ib[i * RP + j] = img[(size_t)(y + i) * stride + x + j];
      const uint8_t* q = img + (size_t)(dy + 2 * i) * stride + dx + 2 * j;
      const uint32_t s = q[0] + q[1] + q[stride] + q[stride + 1] + 2u;
      hb[i * HP + sx + j] = (uint8_t)(s >> 2);
      tb[j * HP + sy + i] = (uint8_t)(s >> 2);
    }
    // the exchange is within one wave: complete the LDS writes, no barrier
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    constexpr int T = B / 2 < 16 ? B / 2 : 16;
    if (lane < T) {
      for (int i = lane; i < B / 2; i += T)
        accumulate_row_pair<B, (B >= 16)>(s_img[wave], 0, RP, s_h0[wave], sx, HP, s_h0t[wave], sy, HP, i, acc);
    }
  }
  constexpr int T = B / 2 < 16 ? B / 2 : 16;
  team_reduce(acc, T);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < 12; ++j) mom[12 * r + j] = acc[j];
  }
}

}  // namespace

hipError_t launch_downsample(const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride, uint8_t* out,
                             hipStream_t s) {
  const uint64_t work = (uint64_t)((w / 2 + 3) / 4) * (h / 2);
  if (work == 0) return hipSuccess;
  hipLaunchKernelGGL(downsample_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, img, w, h,
                     stride, out);
  return hipGetLastError();
}

hipError_t launch_range_moments(const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride, int block,
                                const uint32_t* xy, uint32_t count, uint32_t* mom, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const dim3 grid((count + 3) / 4), blk(256);
  switch (block) {
    case 4: hipLaunchKernelGGL(range_moments_kernel<4>, grid, blk, 0, s, img, w, h, stride, xy, count, mom); break;
    case 8: hipLaunchKernelGGL(range_moments_kernel<8>, grid, blk, 0, s, img, w, h, stride, xy, count, mom); break;
    case 16: hipLaunchKernelGGL(range_moments_kernel<16>, grid, blk, 0, s, img, w, h, stride, xy, count, mom); break;
    case 32: hipLaunchKernelGGL(range_moments_kernel<32>, grid, blk, 0, s, img, w, h, stride, xy, count, mom); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fe
