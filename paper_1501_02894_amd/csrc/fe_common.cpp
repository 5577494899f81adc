// Host-only parts of the C ABI: status text, per-thread error text and the
// validation of encode requests.  No HIP dependency (builds with g++).
#include <stdarg.h>
#include <stdio.h>

#include <string>

#include "fe.h"
#include "fe_common.h"

namespace fe {

static thread_local std::string g_error;

fe_status fail(fe_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return s;
}

void clear_error() { g_error.clear(); }

bool is_pow2(uint32_t v) { return v != 0 && (v & (v - 1)) == 0; }

int levels_of(uint32_t b_max, uint32_t b_min) {
  int L = 1;
  while ((b_min << (L - 1)) < b_max) ++L;
  return L;
}

fe_status check_params(const fe_params* p) {
  if (!p) return fail(FE_ERR_INVALID, "params is NULL");
  if (!is_pow2(p->b_max) || !is_pow2(p->b_min))
    return fail(FE_ERR_INVALID, "b_max (%u) and b_min (%u) must be powers of two", p->b_max, p->b_min);
  if (p->b_min < 2 || p->b_min > p->b_max || p->b_max < 4 || p->b_max > 32)
    return fail(FE_ERR_INVALID, "need 2 <= b_min <= b_max, 4 <= b_max <= 32 (got %u, %u)", p->b_min, p->b_max);
  const int L = levels_of(p->b_max, p->b_min);
  if (L > 4) return fail(FE_ERR_INVALID, "%u -> %u is %d levels; two level bits hold four", p->b_max, p->b_min, L);
  if (p->n_thr != (uint32_t)(L - 1))
    return fail(FE_ERR_INVALID, "n_thr must be %d (one per level except the last), got %u", L - 1, p->n_thr);
  if (p->flags & ~(FE_PHASE2 | FE_FULL_SEARCH | FE_IDENTITY_ONLY | FE_LOCAL_SEARCH))
    return fail(FE_ERR_INVALID, "unknown flags 0x%x", p->flags);
  if ((p->flags & (FE_FULL_SEARCH | FE_LOCAL_SEARCH)) && (p->flags & FE_IDENTITY_ONLY))
    return fail(FE_ERR_INVALID, "FE_IDENTITY_ONLY applies to the co-centred (MNS) search only");
  if ((p->flags & FE_FULL_SEARCH) && (p->flags & FE_LOCAL_SEARCH))
    return fail(FE_ERR_INVALID, "FE_FULL_SEARCH and FE_LOCAL_SEARCH exclude each other");
  return FE_OK;
}

fe_status check_shape(uint32_t w, uint32_t h, uint32_t stride, uint32_t b_max) {
  if (w == 0 || h == 0 || w % b_max || h % b_max)
    return fail(FE_ERR_SHAPE, "image %ux%u: sides must be positive multiples of b_max=%u", w, h, b_max);
  if (w < 2 * b_max || h < 2 * b_max)
    return fail(FE_ERR_SHAPE, "image %ux%u: sides must be at least 2*b_max=%u", w, h, 2 * b_max);
  if (w > 65536 || h > 65536) return fail(FE_ERR_SHAPE, "image %ux%u: sides above 65536", w, h);
  if (stride < w || stride % 4)
    return fail(FE_ERR_SHAPE, "stride %u must be >= width %u and a multiple of 4", stride, w);
  return FE_OK;
}

}  // namespace fe

extern "C" {

const char* fe_last_error(void) { return fe::g_error.c_str(); }

const char* fe_status_string(fe_status s) {
  switch (s) {
    case FE_OK: return "FE_OK";
    case FE_ERR_INVALID: return "FE_ERR_INVALID";
    case FE_ERR_SHAPE: return "FE_ERR_SHAPE";
    case FE_ERR_CAPACITY: return "FE_ERR_CAPACITY";
    case FE_ERR_DEVICE: return "FE_ERR_DEVICE";
    case FE_ERR_OOM: return "FE_ERR_OOM";
    case FE_ERR_BUSY: return "FE_ERR_BUSY";
  }
  return "FE_ERR_UNKNOWN";
}

int fe_version(void) { return 10000; }

fe_status fe_validate(uint32_t width, uint32_t height, uint32_t stride, const fe_params* params) {
  fe::clear_error();
  fe_status s = fe::check_params(params);
  if (s != FE_OK) return s;
  return fe::check_shape(width, height, stride, params->b_max);
}

size_t fe_max_transforms(uint32_t width, uint32_t height, uint32_t b_min) {
  if (b_min == 0) return 0;
  return (size_t)(width / b_min) * (size_t)(height / b_min);
}

}  // extern "C"
