// Allocation-free MNS encode of one image (fe_encode_noalloc).
//
// For callers that cannot allocate device memory during the call (code
// under HIP graph capture, tight serving loops): every scratch buffer of the
// encode -- image table entry, block descriptors, record slots, tile masks,
// ordering counts, the 2 x 2 level's range list -- is carved out of one
// file-scope device array.  Each GPU holds its own copy of the array, at its
// own address, for the life of the process; the address is taken once per
// device with hipGetSymbolAddress when a context is created there, and only
// that address is used on the host.  Every call on one GPU shares the
// array: calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fe.h"
#include "fe_common.h"
#include "fe_encode_seq.h"
#include "fe_internal.h"

namespace fe {
namespace {

constexpr size_t kStaticScratchBytes = 32u << 20;   // 32 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

std::mutex g_mu;
uint8_t* g_ptr[kMaxDevices] = {};

__global__ void table_fill_kernel(ImgDev v, ImgDev* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}

size_t align256(size_t v) { return (v + 255u) & ~(size_t)255u; }

}  // namespace

fe_status static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(FE_ERR_DEVICE, "device %d: no static scratch slot", device);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return FE_OK;
  // the caller made `device` current
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(FE_ERR_DEVICE, "static scratch address on device %d: %s", device, hipGetErrorString(e));
  g_ptr[device] = static_cast<uint8_t*>(p);
  return FE_OK;
}

fe_status static_scratch(int device, uint8_t** ptr, size_t* bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= kMaxDevices || !g_ptr[device])
    return fail(FE_ERR_DEVICE, "no static scratch on device %d (create a context there first)", device);
  *ptr = g_ptr[device];
  *bytes = kStaticScratchBytes;
  return FE_OK;
}

hipError_t launch_table_fill(const ImgDev& v, ImgDev* dst, hipStream_t s) {
  hipLaunchKernelGGL(table_fill_kernel, dim3(1), dim3(64), 0, s, v, dst);
  return hipGetLastError();
}

}  // namespace fe

extern "C" fe_status fe_encode_noalloc(fe_ctx* ctx, const uint8_t* d_img, uint32_t w, uint32_t h, uint32_t stride,
                                       const fe_params* p, fe_transform* d_out, size_t cap, uint64_t* d_offsets,
                                       size_t* n_out, void* stream) {
  fe::clear_error();
  if (!ctx || !d_img || !d_out || !d_offsets) return fe::fail(FE_ERR_INVALID, "NULL argument");
  fe_status st = fe_validate(w, h, stride, p);
  if (st != FE_OK) return st;
  if (p->flags & (FE_FULL_SEARCH | FE_LOCAL_SEARCH))
    return fe::fail(FE_ERR_INVALID, "the allocation-free encode runs MNS only");
  if ((uintptr_t)d_img & 3) return fe::fail(FE_ERR_SHAPE, "image must be 4-byte aligned");
  if ((uintptr_t)d_out & 15) return fe::fail(FE_ERR_INVALID, "output must be 16-byte aligned");
  if ((uintptr_t)d_offsets & 7) return fe::fail(FE_ERR_INVALID, "offsets must be 8-byte aligned");
  const int device = fe::ctx_device(ctx);
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != device && hipSetDevice(device) != hipSuccess) return fe::fail(FE_ERR_DEVICE, "cannot select device %d", device);
  struct Restore {
    int prev, dev;
    ~Restore() {
      if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
    }
  } restore{prev, device};

  uint8_t* base = nullptr;
  size_t limit = 0;
  if ((st = fe::static_scratch(device, &base, &limit)) != FE_OK) return st;
  const fe_image_desc one{d_img, w, h, stride, 0};
  fe::ImgDev entry;
  fe::EncodeGeom g;
  if ((st = fe::encode_geometry(ctx, &one, 1, p, &entry, g)) != FE_OK) return st;

  // carve the scratch: each buffer 256-byte aligned
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = fe::align256(off + (bytes ? bytes : 1));
    return at;
  };
  const size_t o_table = take(sizeof(fe::ImgDev));
  const size_t o_blocks = take((size_t)g.wgs * sizeof(fe::BlockDesc));
  const size_t o_staging = take((size_t)g.slots * 16u);
  const size_t o_masks = take((size_t)g.tiles * 8u);
  const size_t o_csum = take(g.chunks * 4u);
  const size_t o_cbase = take((g.chunks + 1) * 8u);
  const size_t o_fine = take(g.ext ? (size_t)g.fine_max * 16u : 0u);
  const size_t o_fcount = take(4u);
  if (off > limit)
    return fe::fail(FE_ERR_CAPACITY, "a %ux%u image at b_max=%u, b_min=%u needs %zu bytes of static scratch; the limit is %zu",
                    w, h, p->b_max, p->b_min, off, limit);
  const fe::EncodeBufs b{reinterpret_cast<fe::ImgDev*>(base + o_table),
                         reinterpret_cast<fe::BlockDesc*>(base + o_blocks),
                         reinterpret_cast<uint4*>(base + o_staging),
                         reinterpret_cast<uint64_t*>(base + o_masks),
                         reinterpret_cast<uint32_t*>(base + o_csum),
                         reinterpret_cast<uint64_t*>(base + o_cbase),
                         reinterpret_cast<uint4*>(base + o_fine),
                         reinterpret_cast<uint32_t*>(base + o_fcount)};
  const hipStream_t s = (hipStream_t)stream;
  const hipError_t e = fe::launch_table_fill(entry, const_cast<fe::ImgDev*>(b.table), s);
  if (e != hipSuccess) return fe::fail(FE_ERR_DEVICE, "table launch: %s", hipGetErrorString(e));
  if ((st = fe::encode_launch(ctx, g, b, 1, p, true, d_out, cap, d_offsets, s)) != FE_OK) return st;
  if (n_out) return fe::read_count(ctx, d_offsets, 1, cap, n_out, s);
  return FE_OK;
}
