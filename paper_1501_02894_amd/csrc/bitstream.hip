// The compressed file (Sec. 3.3; Technique 2, Sec. 3.4): one variable-length
// code per transform, in stream order, behind a 64-bit header.
//
// A code is, least significant bit first: the phase bit (1 = phase 2), the
// 0-based level in 2 bits (left out for a last-level block that is not the
// top-left child of its parent, Technique 2), the luminance byte, then
//   phase 1: the contrast k in 3 bits, and the isometry in 3 more bits when
//            the stream stores isometries (14 or 17 bits in all);
//   phase 2: O_1..O_3 - O_i as M-bit sign (1 = negative) and magnitude,
//            M = 5 at level 1 and 6 below, then the 4 contrast bits
//            (30 or 33 bits in all).
// Header: W - 1 (16 bits), H - 1 (16), log2 B_max (3), log2 B_min (3), the
// isometry flag (1), 25 zero bits.
//
// Packing is a prefix sum of code lengths: per chunk of 1024 transforms the
// code lengths are summed, one workgroup scans the chunk sums, and every
// transform then ORs its code into the zeroed stream at its bit offset
// (at most two 64-bit words, with 64-bit atomics).
#include <algorithm>

#include "fe_device.h"
#include "fe_internal.h"

namespace fe {
namespace {

constexpr int kPackChunk = 1024;

struct Code {
  uint64_t bits;
  int len;
  bool ok;
};

// The code of transform w (fe_transform words) in a quadtree of L levels.
__device__ __forceinline__ Code make_code(uint4 w, int L, int b_min, bool iso) {
  const int x = (int)(w.x & 0xffffu), y = (int)(w.x >> 16);
  const int level = (int)(w.z & 0xffu), flags = (int)((w.z >> 8) & 0xffu);
  const int e = (int)((w.z >> 16) & 0xffu), s = (int)(w.z >> 24);
  const int lum = (int)(w.w & 0xffu);
  Code c{0ull, 0, level < L && flags <= 1};
  auto put = [&](uint32_t v, int width) {
    c.bits |= (uint64_t)v << c.len;
    c.len += width;
  };
  put((uint32_t)flags & 1u, 1);
  const int child = ((y / b_min) & 1) * 2 + ((x / b_min) & 1);
  if (!(L >= 2 && level == L - 1 && child != 0)) put((uint32_t)level & 3u, 2);
  put((uint32_t)lum, 8);
  if (flags == 0) {
    c.ok = c.ok && s < 8 && e < 8 && (iso || e == 0);
    put((uint32_t)s & 7u, 3);
    if (iso) put((uint32_t)e & 7u, 3);
  } else {
    // phase 2 stands for a parent at level 1..3 (0-based 0..2), never the last
    const int M = level == 0 ? 5 : 6;
    c.ok = c.ok && level <= 2 && level < L - 1 && e == 0 && s < 16;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int d = (int)(int8_t)((w.w >> (8 + 8 * k)) & 0xffu);
      const int mag = d < 0 ? -d : d;
      c.ok = c.ok && mag <= (1 << (M - 1)) - 1;
      put((uint32_t)(d < 0 ? 1 : 0) | ((uint32_t)(mag & ((1 << (M - 1)) - 1)) << 1), M);
    }
    put((uint32_t)s & 15u, 4);
  }
  return c;
}

// Chunk sums of code lengths; counts transforms whose fields do not fit.
__global__ __launch_bounds__(256) void pack_count_kernel(const uint4* __restrict__ t, uint64_t n, int L, int b_min,
                                                         int iso, uint64_t* __restrict__ chunk_bits,
                                                         uint32_t* __restrict__ bad) {
  __shared__ uint64_t s_w[4];
  const uint64_t c0 = (uint64_t)blockIdx.x * kPackChunk;
  uint64_t acc = 0;
  uint32_t nbad = 0;
#pragma unroll
  for (int u = 0; u < kPackChunk / 256; ++u) {
    const uint64_t i = c0 + threadIdx.x + 256u * (uint64_t)u;
    if (i < n) {
      const Code c = make_code(t[i], L, b_min, iso != 0);
      acc += (uint64_t)c.len;
      nbad += c.ok ? 0u : 1u;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  if (nbad) atomicAdd(bad, nbad);
  __syncthreads();
  if (threadIdx.x == 0) chunk_bits[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// Exclusive scan of the chunk sums (one workgroup of 1024 lanes); the total
// stream length, header included, goes to *total.
__global__ __launch_bounds__(1024) void pack_scan_kernel(const uint64_t* __restrict__ chunk_bits, uint32_t n,
                                                         uint64_t* __restrict__ chunk_base, uint64_t header,
                                                         uint64_t* __restrict__ total) {
  __shared__ uint64_t s_w[16];
  __shared__ uint64_t s_carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_carry = header;
  __syncthreads();
  for (uint32_t b = 0; b < n; b += 1024) {
    const uint32_t c = b + (uint32_t)tid;
    const uint64_t v = c < n ? chunk_bits[c] : 0ull;
    uint64_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t o = __shfl_up(incl, off);
      if (lane >= off) incl += o;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint64_t pre = s_carry;
    for (int k = 0; k < wave; ++k) pre += s_w[k];
    if (c < n) chunk_base[c] = pre + incl - v;
    __syncthreads();
    if (tid == 1023) s_carry = pre + incl;
    __syncthreads();
  }
  if (tid == 0) *total = s_carry;
}

// Zero the words the stream occupies (at most cap_words), reading its
// length from *total.
__global__ __launch_bounds__(256) void pack_zero_kernel(unsigned long long* __restrict__ out, uint64_t cap_words,
                                                        const uint64_t* __restrict__ total) {
  const uint64_t words = min<uint64_t>((*total + 63u) >> 6, cap_words);
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < words; i += (uint64_t)gridDim.x * 256u)
    out[i] = 0ull;
}

// OR every code into place; the first workgroup also writes the header.
// Words at or beyond cap_words are not touched (the host reports the
// capacity error from the total).
__global__ __launch_bounds__(256) void pack_write_kernel(const uint4* __restrict__ t, uint64_t n, int L, int b_min,
                                                         int iso, const uint64_t* __restrict__ chunk_base,
                                                         uint64_t header_word, unsigned long long* __restrict__ out,
                                                         uint64_t cap_words) {
  __shared__ uint32_t s_w[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t c0 = (uint64_t)blockIdx.x * kPackChunk;
  if (blockIdx.x == 0 && tid == 0 && cap_words > 0) atomicOr(&out[0], (unsigned long long)header_word);
  Code code[kPackChunk / 256];
  uint32_t mine = 0;   // this lane's four codes, consecutive transforms 4 tid .. 4 tid + 3
#pragma unroll
  for (int u = 0; u < kPackChunk / 256; ++u) {
    const uint64_t i = c0 + 4u * (uint64_t)tid + (uint64_t)u;
    code[u] = i < n ? make_code(t[i], L, b_min, iso != 0) : Code{0ull, 0, true};
    mine += (uint32_t)code[u].len;
  }
  // exclusive scan of the lanes' sums (4 transforms per lane, in order)
  uint32_t incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) s_w[wave] = incl;
  __syncthreads();
  uint32_t pre = incl - mine;
  for (int k = 0; k < wave; ++k) pre += s_w[k];
  uint64_t pos = chunk_base[blockIdx.x] + pre;
#pragma unroll
  for (int u = 0; u < kPackChunk / 256; ++u) {
    const Code c = code[u];
    if (c.len > 0) {
      const uint64_t wi = pos >> 6;
      const int sh = (int)(pos & 63u);
      if (wi < cap_words) atomicOr(&out[wi], (unsigned long long)(c.bits << sh));
      if (sh + c.len > 64 && wi + 1 < cap_words) atomicOr(&out[wi + 1], (unsigned long long)(c.bits >> (64 - sh)));
    }
    pos += (uint64_t)c.len;
  }
}

}  // namespace

size_t pack_chunks(uint64_t n) { return (size_t)((n + kPackChunk - 1) / kPackChunk); }

hipError_t launch_pack(const uint4* t, uint64_t n, int L, int b_min, bool iso, uint64_t header_word,
                       uint64_t* chunk_bits, uint64_t* chunk_base, uint64_t* total, uint32_t* bad,
                       unsigned long long* out, uint64_t cap_words, hipStream_t s) {
  const unsigned chunks = (unsigned)pack_chunks(n);
  if (chunks) {
    hipLaunchKernelGGL(pack_count_kernel, dim3(chunks), dim3(256), 0, s, t, n, L, b_min, iso ? 1 : 0, chunk_bits,
                       bad);
  }
  hipLaunchKernelGGL(pack_scan_kernel, dim3(1), dim3(1024), 0, s, chunk_bits, chunks, chunk_base, (uint64_t)64,
                     total);
  const uint64_t zero_blocks = std::min<uint64_t>((cap_words + 255) / 256, 4096);
  if (zero_blocks)
    hipLaunchKernelGGL(pack_zero_kernel, dim3((unsigned)zero_blocks), dim3(256), 0, s, out, cap_words, total);
  if (chunks) {
    hipLaunchKernelGGL(pack_write_kernel, dim3(chunks), dim3(256), 0, s, t, n, L, b_min, iso ? 1 : 0, chunk_base,
                       header_word, out, cap_words);
  } else if (cap_words) {
    hipLaunchKernelGGL(pack_write_kernel, dim3(1), dim3(256), 0, s, t, (uint64_t)0, L, b_min, iso ? 1 : 0,
                       chunk_base, header_word, out, cap_words);
  }
  return hipGetLastError();
}

}  // namespace fe
