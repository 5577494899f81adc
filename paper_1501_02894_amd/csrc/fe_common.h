// Host-only helpers shared by the C-ABI implementation files.
#pragma once

#include <stdint.h>

#include "fe.h"

namespace fe {

// Record `fmt` as this thread's last error and return `s`.
fe_status fail(fe_status s, const char* fmt, ...);
void clear_error();

bool is_pow2(uint32_t v);
int levels_of(uint32_t b_max, uint32_t b_min);   // L = log2(b_max / b_min) + 1
fe_status check_params(const fe_params* p);
fe_status check_shape(uint32_t w, uint32_t h, uint32_t stride, uint32_t b_max);

}  // namespace fe
