// Parser of the compressed file (Sec. 3.3; Technique 2, Sec. 3.4), on the
// host: the codes have data-dependent lengths (a code's length is known only
// once its phase and level bits are read, and Technique 2 makes the level
// bits depend on the block before), so the file is read in one sequential
// pass.  The layout is stated beside fe_pack in fe.h.
#include <cstdint>
#include <cstring>

#include "fe.h"
#include "fe_common.h"

namespace {

struct Reader {
  const uint8_t* data;
  uint64_t n_bits;
  uint64_t pos = 0;
  bool ok = true;

  uint32_t get(int width) {
    if (pos + (uint64_t)width > n_bits) {
      ok = false;
      return 0;
    }
    uint32_t v = 0;
    for (int b = 0; b < width; ++b, ++pos) v |= (uint32_t)((data[pos >> 3] >> (pos & 7)) & 1u) << b;
    return v;
  }
};

int clamp_origin(int p, int B, int extent) {
  const int v = p - B / 2, hi = extent - 2 * B;
  return v < 0 ? 0 : (v > hi ? hi : v);
}

}  // namespace

fe_status fe_unpack(const uint8_t* h_bits, uint64_t n_bits, fe_transform* h_out, size_t cap, size_t* n_out,
                    fe_stream_info* info) {
  fe::clear_error();
  if (!n_out || (n_bits && !h_bits) || (cap && !h_out)) return fe::fail(FE_ERR_INVALID, "NULL argument");
  *n_out = 0;
  Reader rd{h_bits, n_bits};
  const uint32_t W = rd.get(16) + 1, H = rd.get(16) + 1;
  const uint32_t b_max = 1u << rd.get(3), b_min = 1u << rd.get(3);
  const uint32_t iso = rd.get(1);
  const uint32_t reserved = rd.get(25);
  if (!rd.ok) return fe::fail(FE_ERR_INVALID, "the file is shorter than its header");
  if (reserved) return fe::fail(FE_ERR_INVALID, "reserved header bits are set");
  if (b_min < 2 || b_max < 4 || b_max > 32 || b_min > b_max || fe::levels_of(b_max, b_min) > 4 || W % b_max ||
      H % b_max || W < 2 * b_max || H < 2 * b_max)
    return fe::fail(FE_ERR_INVALID, "header: %ux%u image with blocks %u -> %u does not tile", W, H, b_max, b_min);
  if (info) *info = fe_stream_info{W, H, b_max, b_min, iso ? FE_PACK_ISOMETRY : 0u};
  const int L = fe::levels_of(b_max, b_min);
  const uint32_t tiles_x = W / b_max, tiles = tiles_x * (H / b_max);
  const uint32_t cells = 1u << (2 * (L - 1));
  uint32_t tile = 0, cell = 0;
  int prev_child = -1;   // child index of the previous block if it lies at the last level
  size_t count = 0;
  while (tile < tiles) {
    const uint32_t p2 = rd.get(1);
    uint32_t level;
    if (L >= 2 && prev_child >= 0 && prev_child < 3)
      level = (uint32_t)(L - 1);   // Technique 2: a sibling of the last-level block before
    else
      level = rd.get(2);
    if (!rd.ok) return fe::fail(FE_ERR_INVALID, "the file ends inside transform %zu", count);
    if (level >= (uint32_t)L) return fe::fail(FE_ERR_INVALID, "transform %zu: level %u of %d", count, level, L);
    const uint32_t B = b_max >> level;
    const uint32_t span = (B / b_min) * (B / b_min);
    if (cell % span) return fe::fail(FE_ERR_INVALID, "transform %zu does not fit the next free cell", count);
    uint32_t lx = 0, ly = 0;   // Morton decode, x bit below y bit
    for (int b = 0; b < L - 1; ++b) {
      lx |= ((cell >> (2 * b)) & 1u) << b;
      ly |= ((cell >> (2 * b + 1)) & 1u) << b;
    }
    const uint32_t x = (tile % tiles_x) * b_max + lx * b_min, y = (tile / tiles_x) * b_max + ly * b_min;
    fe_transform t;
    std::memset(&t, 0, sizeof t);
    t.x = (uint16_t)x;
    t.y = (uint16_t)y;
    t.dx = (uint16_t)clamp_origin((int)x, (int)B, (int)W);
    t.dy = (uint16_t)clamp_origin((int)y, (int)B, (int)H);
    t.level = (uint8_t)level;
    t.lum = (uint8_t)rd.get(8);
    if (!p2) {
      t.s_idx = (uint8_t)rd.get(3);
      t.iso = iso ? (uint8_t)rd.get(3) : 0;
    } else {
      if ((int)level >= L - 1 || level > 2)
        return fe::fail(FE_ERR_INVALID, "transform %zu: phase 2 at level %u", count, level);
      t.flags = FE_TRANSFORM_PHASE2;
      const int M = level == 0 ? 5 : 6;
      for (int c = 0; c < 3; ++c) {
        const uint32_t v = rd.get(M);
        const int mag = (int)(v >> 1);
        t.dlum[c] = (int8_t)((v & 1u) ? -mag : mag);
      }
      t.s_idx = (uint8_t)rd.get(4);
    }
    if (!rd.ok) return fe::fail(FE_ERR_INVALID, "the file ends inside transform %zu", count);
    if (count < cap) h_out[count] = t;
    ++count;
    prev_child = (L >= 2 && (int)level == L - 1) ? (int)(((y / b_min) & 1u) * 2 + ((x / b_min) & 1u)) : -1;
    cell += span;
    if (cell == cells) {
      ++tile;
      cell = 0;
    }
  }
  *n_out = count;
  if (count > cap) return fe::fail(FE_ERR_CAPACITY, "the file holds %zu transforms, cap is %zu", count, cap);
  return FE_OK;
}
