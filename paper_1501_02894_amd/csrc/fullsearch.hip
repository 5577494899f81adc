// Exhaustive range-domain search (Sec. 1: every 2B x 2B block at step 1 is
// a candidate domain, (W-2B+1)(H-2B+1) of them), the baseline that the
// no-search coder replaces.  Same domain reduction (2 x 2 round-half-up
// means), same isometries, contrast grid and scaled error S = 64 n E as
// no-search; the best candidate minimises (S, domain index v*(W-2B+1)+u,
// isometry), k the lowest on ties.
//
// Sum r T_e(D) over all range x domain pairs is a dense contraction, done
// with int8 MFMA on centred values: A holds, per range, 8 copies permuted
// by the inverse isometries (r - 128), B the domain windows (D - 128)
// gathered from the four 2 x 2 phase images (implicit im2col), and
//   Sum r T_e(D) = G + 128 Sum r + 128 Sum D - 16384 n   (G the i32 MFMA sum).
// The epilogue screens every (range, domain) pair with an exact bound on
// the best error reachable from its largest correlation and evaluates the
// survivors exactly; per range the best (f, domain, isometry) is kept as a
// 64-bit key and combined with atomicMin.
#include "fe_device.h"
#include "fe_internal.h"

namespace fe {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kStripsPerBlock = 32;   // domain rows per workgroup
constexpr int kIdxBits = 23;          // domain * 8 + isometry
constexpr int64_t kFBias = 1ll << 40; // -f < 2^40 for every block size <= 32

// Key of a candidate: (f + 2^40) << 23 | (domain * 8 + e); smaller is better.
__device__ __forceinline__ uint64_t cand_key(int64_t f, uint32_t dom, int e) {
  return ((uint64_t)(f + kFBias) << kIdxBits) | ((uint64_t)dom << 3) | (uint64_t)e;
}

// Inverse isometry: rotations by 90 degrees (5, 6) swap; the rest are
// involutions.
__device__ __forceinline__ int iso_inverse(int e) { return e == 5 ? 6 : (e == 6 ? 5 : e); }

// Source position of pixel (i, j) under isometry e (table of fe.h).
__device__ __forceinline__ void iso_src(int e, int i, int j, int B, int& si, int& sj) {
  int a = i, b = j;
  if (e & 4) { a = j; b = i; }
  const bool flip_first = (e & 4) ? (e & 1) : (e & 2);
  const bool flip_second = (e & 4) ? (e & 2) : (e & 1);
  si = flip_first ? B - 1 - a : a;
  sj = flip_second ? B - 1 - b : b;
}

// Row rho of a 32-row A fragment holds (local range, isometry) such that in
// the 32x32 accumulator layout lane group g (= lane / 32) owns, in its 16
// registers j, local range 2g + j / 8 and isometry j % 8.
__device__ __forceinline__ void frag_row(int rho, int& lr, int& e) {
  lr = 2 * ((rho >> 2) & 1) + (rho >> 4);
  e = 4 * ((rho >> 3) & 1) + (rho & 3);
}

// ------------------------------------------------------------------ prep
// Four 2x2-mean phase images: plane (p, q)[y][x] = round-half-up mean of
// I[2y+q .. 2y+q+1][2x+p .. 2x+p+1] where the 2x2 group lies in the image;
// zero elsewhere (padding read by the last strips, never used).
__global__ __launch_bounds__(256) void fs_planes_kernel(const uint8_t* img, uint32_t w, uint32_t h,
                                                       uint32_t stride, uint8_t* planes, uint32_t pitch,
                                                       uint32_t prow) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t per_plane = (uint64_t)pitch * prow;
  if (i >= 4 * per_plane) return;
  const uint32_t pl = (uint32_t)(i / per_plane);
  const uint32_t rem = (uint32_t)(i - (uint64_t)pl * per_plane);
  const uint32_t y = rem / pitch, x = rem - y * pitch;
  const uint32_t p = pl & 1u, q = pl >> 1;
  const uint32_t ix = 2 * x + p, iy = 2 * y + q;
  uint8_t v = 0;
  if (ix + 1 < w && iy + 1 < h) {
    const uint8_t* a = img + (size_t)iy * stride + ix;
    v = (uint8_t)((a[0] + a[1] + a[stride] + a[stride + 1] + 2u) >> 2);
  }
  planes[i] = v;
}

struct FsGeo {
  uint32_t w, h, B, nu, nv;     // nu = W-2B+1, nv = H-2B+1
  uint32_t pitch, prow;         // plane pitch (bytes) and rows
  const uint8_t* planes;
};

__device__ __forceinline__ const uint8_t* domain_origin_ptr(const FsGeo& g, uint32_t u, uint32_t v) {
  const uint32_t pl = (u & 1u) + 2 * (v & 1u);
  return g.planes + (size_t)pl * g.pitch * g.prow + (size_t)(v >> 1) * g.pitch + (u >> 1);
}

// K8: Sum D and Q = n Sum D^2 - (Sum D)^2 of every domain.
__global__ __launch_bounds__(256) void fs_domain_sums_kernel(FsGeo g, uint32_t* sd, double* q) {
  const uint32_t d = blockIdx.x * 256 + threadIdx.x;
  if (d >= g.nu * g.nv) return;
  const uint32_t v = d / g.nu, u = d - v * g.nu;
  const uint8_t* o = domain_origin_ptr(g, u, v);
  uint32_t s = 0, s2 = 0;
  for (uint32_t i = 0; i < g.B; ++i)
    for (uint32_t j = 0; j < g.B; ++j) {
      const uint32_t x = o[(size_t)i * g.pitch + j];
      s += x;
      s2 += x * x;
    }
  sd[d] = s;
  const double n = (double)(g.B * g.B), ds = (double)s;
  q[d] = n * (double)s2 - ds * ds;
}

// Per range: Sum r, and alpha / beta of P = n G + alpha + beta Sum D.
__global__ __launch_bounds__(256) void fs_range_sums_kernel(const uint8_t* img, uint32_t stride, uint32_t B,
                                                           const uint32_t* xy, uint32_t R, uint32_t* sr,
                                                           double* alpha, double* beta) {
  const uint32_t r = blockIdx.x * 256 + threadIdx.x;
  if (r >= R) return;
  const uint32_t x = xy[r] & 0xffffu, y = xy[r] >> 16;
  uint32_t s = 0;
  for (uint32_t i = 0; i < B; ++i)
    for (uint32_t j = 0; j < B; ++j) s += img[(size_t)(y + i) * stride + x + j];
  sr[r] = s;
  const double n = (double)(B * B);
  alpha[r] = 128.0 * n * (double)s - 16384.0 * n * n;
  beta[r] = 128.0 * n - (double)s;
}

// A fragments: frag[F][c][lane] = BYTES bytes, row rho = lane % 32 of
// fragment F (ranges 4F .. 4F+3), K indices of chunk c for lane group
// lane / 32: [KC_STEP c + BYTES (lane / 32), + BYTES).  Entry = r at the
// inverse-isometry source of pixel q, minus 128.
template <int B>
__global__ __launch_bounds__(256) void fs_build_a_kernel(const uint8_t* img, uint32_t stride, const uint32_t* xy,
                                                        uint32_t R, uint32_t nfrag, uint8_t* frag) {
  constexpr int K = B * B;
  constexpr int BYTES = B == 4 ? 8 : 16;
  constexpr int KCS = 2 * BYTES;              // K per chunk
  constexpr int KC = K / KCS;                 // chunks
  const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;   // (F, c, lane)
  if (t >= (uint64_t)nfrag * KC * 64) return;
  const uint32_t lane = (uint32_t)(t & 63u), c = (uint32_t)((t >> 6) % KC), F = (uint32_t)((t >> 6) / KC);
  int lr, e;
  frag_row((int)(lane & 31u), lr, e);
  const uint32_t r = 4 * F + (uint32_t)lr;
  uint8_t out[BYTES];
  const int einv = iso_inverse(e);
  for (int b = 0; b < BYTES; ++b) {
    uint8_t val = 0;   // (128 - 128) for padding ranges
    if (r < R) {
      const int q = KCS * (int)c + BYTES * (int)(lane >> 5) + b;
      const int i = q / B, j = q - (q / B) * B;
      int si, sj;
      iso_src(einv, i, j, B, si, sj);
      const uint32_t x = xy[r] & 0xffffu, y = xy[r] >> 16;
      val = (uint8_t)((int)img[(size_t)(y + si) * stride + x + sj] - 128);
    }
    out[b] = val;
  }
  uint8_t* dst = frag + t * BYTES;
  for (int b = 0; b < BYTES; ++b) dst[b] = out[b];
}

// ------------------------------------------------------------------ GEMM
// Workgroup: 4 waves x NF A fragments (32 rows = 4 ranges each) against
// kStripsPerBlock domain rows of 32 domains of one parity class.
template <int B, int NF>
struct FsCfg {
  static constexpr int K = B * B;
  static constexpr int BYTES = B == 4 ? 8 : 16;
  static constexpr int KCS = 2 * BYTES;
  static constexpr int KC = K / KCS;
  static constexpr int LROWS = kStripsPerBlock + B - 1;   // staged plane rows
  static constexpr int LP = 32 + B + 12;                  // staged row pitch (bytes), multiple of 4
  // The staged rows are held four times, copy k shifted left by k bytes, so
  // that every lane reads its window's words aligned.  Copies lie 8 mod 32
  // dwords apart: lanes col = 4w + k of a half-wave then hit 32 distinct
  // banks.
  static constexpr int CW = ((LROWS * (LP / 4) + 23) / 32) * 32 + 8;   // dwords per copy
};

template <int B, int NF>
__global__ __launch_bounds__(256) void fs_gemm_kernel(FsGeo g, const uint8_t* frag, uint32_t nfrag, uint32_t R,
                                                     const double* alpha, const double* beta, const uint32_t* sd,
                                                     const double* qd, uint64_t* best, uint32_t xblocks,
                                                     uint32_t tblocks) {
  using C = FsCfg<B, NF>;
  __shared__ uint32_t s_pl[4 * C::CW];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, grp = lane >> 5, col = lane & 31;
  // domain block: parity class, block of plane rows, block of 32 columns
  uint32_t db = blockIdx.y;
  const uint32_t cls = db % 4u;
  db /= 4u;
  const uint32_t tb = db % tblocks, xb = db / tblocks;
  const uint32_t p = cls & 1u, q = cls >> 1;
  const uint32_t ncols = (g.nu + 1u - p) / 2u;   // u = 2x + p <= W - 2B
  const uint32_t nrows = (g.nv + 1u - q) / 2u;   // v = 2t + q <= H - 2B
  const uint32_t t0 = tb * kStripsPerBlock, x0 = xb * 32u;
  if (t0 >= nrows || x0 >= ncols) return;
  const uint8_t* plane = g.planes + (size_t)cls * g.pitch * g.prow;
  // stage plane rows t0 .. t0 + LROWS - 1, columns x0 .. x0 + LP - 1, in
  // four copies shifted by 0..3 bytes: a lane reads two aligned words of a
  // row (the pitch and x0 are multiples of 4) and forms the word of every
  // copy from them.  The last words of a row read up to 7 bytes past it,
  // inside the plane's padded pitch, and are never used.
  for (int i = tid; i < C::LROWS * (C::LP / 4); i += 256) {
    const int r = i / (C::LP / 4), c4 = i - r * (C::LP / 4);
    uint32_t w0 = 0, w1 = 0;
    const uint32_t row = t0 + (uint32_t)r;
    if (row < g.prow) {
      const uint32_t* s = reinterpret_cast<const uint32_t*>(plane + (size_t)row * g.pitch + x0) + c4;
      w0 = s[0];
      w1 = s[1];
    }
    // staged centred: d - 128 == d ^ 0x80 as int8
#pragma unroll
    for (int k = 0; k < 4; ++k)
      s_pl[k * C::CW + r * (C::LP / 4) + c4] = __builtin_amdgcn_alignbyte(w1, w0, (uint32_t)k) ^ 0x80808080u;
  }
  __syncthreads();
  // this lane's copy and word column: every window row starts word-aligned
  const uint32_t* s_col = s_pl + (col & 3) * C::CW + (col >> 2);

  // A fragments of this wave (registers)
  const uint32_t F0 = (blockIdx.x * 4u + (uint32_t)wave) * NF;
  v4i afr[NF][C::KC];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int c = 0; c < C::KC; ++c) {
      v4i a = {0, 0, 0, 0};
      if (F0 + f < nfrag) {
        const uint8_t* src = frag + (((size_t)(F0 + f) * C::KC + c) * 64 + lane) * C::BYTES;
        if constexpr (C::BYTES == 16) {
          a = *reinterpret_cast<const v4i*>(src);
        } else {
          const uint2 u = *reinterpret_cast<const uint2*>(src);
          a.x = (int)u.x;
          a.y = (int)u.y;
        }
      }
      afr[f][c] = a;
    }
  // per-lane ranges: 2 per fragment (local ranges 2 grp, 2 grp + 1)
  constexpr int NR = 2 * NF;
  double al[NR], be[NR], thr[NR];
  uint64_t bk[NR];
  bool rv[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const uint32_t r = 4 * (F0 + k / 2) + 2 * grp + (k & 1);
    rv[k] = r < R;
    al[k] = rv[k] ? alpha[r] : 0.0;
    be[k] = rv[k] ? beta[r] : 0.0;
    bk[k] = ((uint64_t)kFBias << kIdxBits);
    // screen against the best candidate other workgroups have published so
    // far: it is a real candidate, so a pair whose bound is strictly worse
    // cannot win, and ties still pass the screen
    const int64_t fs = rv[k] ? (int64_t)(best[r] >> kIdxBits) - kFBias : 0;
    thr[k] = fs < 0 ? -(double)fs : 0.0;
  }
  const double n = (double)(B * B);
  const uint32_t xcol = x0 + (uint32_t)col;
  const bool dvalid = xcol < ncols;
  const uint32_t u = 2 * xcol + p;
  // The domain sums of strip t + 1 are loaded while strip t is searched, so
  // that no strip waits for its own; a lane without a domain there reads
  // domain 0 and ignores it.
  const uint32_t dom0 = dvalid ? (2 * t0 + q) * g.nu + u : 0u;
  uint32_t sd_next = sd[dom0];
  double qd_next = qd[dom0];
  for (int t = 0; t < kStripsPerBlock; ++t) {
    const uint32_t trow = t0 + (uint32_t)t;
    if (trow >= nrows) break;                       // uniform over the workgroup
    const uint32_t v = 2 * trow + q;
    const uint32_t dom = v * g.nu + u;
    const double dsd = dvalid ? (double)sd_next : 0.0;
    const double dq = dvalid ? qd_next : 0.0;
    const bool more = dvalid && t + 1 < kStripsPerBlock && trow + 1 < nrows;
    const uint32_t dom_next = more ? dom + 2 * g.nu : 0u;
    sd_next = sd[dom_next];
    qd_next = qd[dom_next];
    v16i acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[f][j] = 0;
#pragma unroll
    for (int c = 0; c < C::KC; ++c) {
      // B fragment: column col, K [KCS c + BYTES grp, + BYTES) of the domain
      // whose window starts at staged row t, column col
      v4i bfr = {0, 0, 0, 0};
      if constexpr (B == 16) {
        const int row = t + 2 * c + grp;           // K q0 = 32c + 16 grp -> row q0 / 16
        const uint32_t* w = s_col + row * (C::LP / 4);
        bfr.x = (int)w[0];
        bfr.y = (int)w[1];
        bfr.z = (int)w[2];
        bfr.w = (int)w[3];
      } else if constexpr (B == 8) {
        const int row = t + 4 * c + 2 * grp;       // q0 = 32c + 16 grp -> rows q0 / 8, +1
        const uint32_t* w = s_col + row * (C::LP / 4);
        bfr.x = (int)w[0];
        bfr.y = (int)w[1];
        bfr.z = (int)w[C::LP / 4];
        bfr.w = (int)w[C::LP / 4 + 1];
      } else {
        const int row = t + 2 * grp;               // q0 = 8 grp -> rows 2 grp, +1
        const uint32_t* w = s_col + row * (C::LP / 4);
        bfr.x = (int)w[0];
        bfr.y = (int)w[C::LP / 4];
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        if constexpr (B == 4) {
          const long av = (long)(uint32_t)afr[f][c].x | ((long)(uint32_t)afr[f][c].y << 32);
          const long bv = (long)(uint32_t)bfr.x | ((long)(uint32_t)bfr.y << 32);
          acc[f] = __builtin_amdgcn_mfma_i32_32x32x16_i8(av, bv, acc[f], 0, 0, 0);
        } else {
          acc[f] = __builtin_amdgcn_mfma_i32_32x32x32_i8(afr[f][c], bfr, acc[f], 0, 0, 0);
        }
      }
    }
    // epilogue: per (range, domain) the largest correlation decides the
    // isometry; screen by the bound f >= -64 P^2 / Q, then evaluate exactly
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int f = k / 2, s = k & 1;
      int gmax = acc[f][8 * s];
#pragma unroll
      for (int j = 1; j < 8; ++j) gmax = max(gmax, acc[f][8 * s + j]);
      const double P = n * (double)gmax + al[k] + be[k] * dsd;
      const bool pass = dvalid && rv[k] && P > 0.0 && 64.0 * P * P * (1.0 + 0x1p-40) >= thr[k] * dq;
      if (pass) {
        const double P16 = 16.0 * P;
        int kk = (7.0 * dq < P16) ? 4 : 0;
        kk += ((double)(2 * kk + 3) * dq < P16) ? 2 : 0;
        kk += ((double)(2 * kk + 1) * dq < P16) ? 1 : 0;
        const double fv = (double)(kk * kk) * dq - (double)(16 * kk) * P;
        // Only a candidate at least as good as the threshold can lower the
        // range's minimum key: the threshold is -f of a real candidate (this
        // lane's best, or the key already published for the range), whose
        // key any worse f exceeds.  So the isometry and the key are formed
        // for those few alone.
        if (fv <= -thr[k]) {
          int e = 7;
#pragma unroll
          for (int j = 7; j >= 0; --j)
            if (acc[f][8 * s + j] == gmax) e = j;
          if (kk == 0) e = 0;
          const uint64_t key = cand_key((int64_t)fv, dom, e);
          if (key < bk[k]) {
            bk[k] = key;
            thr[k] = -fv;
          }
        }
      }
    }
  }
  // best over the 32 domain columns of each range, then across workgroups
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    uint64_t kv = bk[k];
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
      const uint64_t o = __shfl_xor(kv, off, 32);
      kv = o < kv ? o : kv;
    }
    if (col == 0 && rv[k]) {
      const uint32_t r = 4 * (F0 + k / 2) + 2 * grp + (k & 1);
      atomicMin(reinterpret_cast<unsigned long long*>(&best[r]), (unsigned long long)kv);
    }
  }
}

// ------------------------------------------------------------------ local search
// Local search (Sec. 2): the candidates of a B x B range at (x, y) are the
// 2B x 2B blocks that contain it, step-1 origins x - B <= u <= x and
// y - B <= v <= y inside the image ((B+1)^2 away from the borders), with the
// identity only.  One wave per range: every lane holds the range's rows in
// registers, scores candidates lane, lane + 64, ... exactly in integers
// (Sum r d from the phase planes, Sum d and Q of the domain from the domain
// sums), and the wave keeps the least key, so that the finalisation of the
// exhaustive search applies unchanged.
template <int B>
__global__ __launch_bounds__(256) void ls_search_kernel(FsGeo g, const uint8_t* __restrict__ img, uint32_t stride,
                                                       const uint32_t* __restrict__ sd, const double* __restrict__ qd,
                                                       const uint32_t* __restrict__ xy, uint32_t R,
                                                       uint64_t* __restrict__ best) {
  constexpr int Q4 = B / 4;
  constexpr int64_t N = B * B;
  const int lane = threadIdx.x & 63;
  const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= R) return;   // the whole wave: nothing below synchronises the workgroup
  const int x = (int)(xy[r] & 0xffffu), y = (int)(xy[r] >> 16);
  uint32_t rr[B][Q4];
  uint32_t srs = 0;
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int q = 0; q < Q4; ++q) {
      rr[i][q] = *reinterpret_cast<const uint32_t*>(img + (size_t)(y + i) * stride + x + 4 * q);
      srs = __builtin_amdgcn_udot4(rr[i][q], 0x01010101u, srs, false);
    }
  const int64_t sr = (int64_t)srs;
  const int u0 = max(0, x - B), u1 = min(x, (int)g.w - 2 * B);
  const int v0 = max(0, y - B), v1 = min(y, (int)g.h - 2 * B);
  const int cu = u1 - u0 + 1, nc = cu * (v1 - v0 + 1);
  uint64_t key = ~0ull;
  for (int c = lane; c < nc; c += 64) {
    const int v = v0 + c / cu, u = u0 + c % cu;
    const uint32_t dom = (uint32_t)v * g.nu + (uint32_t)u;
    const uint8_t* o = domain_origin_ptr(g, (uint32_t)u, (uint32_t)v);
    const uint32_t sh = (uint32_t)((uintptr_t)o & 3u);
    const uint32_t* a = reinterpret_cast<const uint32_t*>((uintptr_t)o & ~(uintptr_t)3);
    const uint32_t pw = g.pitch / 4;
    uint32_t srd = 0;
#pragma unroll
    for (int i = 0; i < B; ++i) {
      uint32_t w[Q4 + 1];
#pragma unroll
      for (int q = 0; q <= Q4; ++q) w[q] = a[(size_t)i * pw + q];
#pragma unroll
      for (int q = 0; q < Q4; ++q)
        srd = __builtin_amdgcn_udot4(rr[i][q], __builtin_amdgcn_alignbyte(w[q + 1], w[q], sh), srd, false);
    }
    const int64_t d = (int64_t)sd[dom];
    const int64_t Q = (int64_t)qd[dom];
    const int64_t P = N * (int64_t)srd - sr * d;
    int k = 0;
#pragma unroll
    for (int j = 0; j < 7; ++j) k += ((int64_t)(2 * j + 1) * Q < 16 * P) ? 1 : 0;
    const int64_t f = (int64_t)(k * k) * Q - (int64_t)(16 * k) * P;
    const uint64_t kk = cand_key(f, dom, 0);
    key = kk < key ? kk : key;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o2 = __shfl_xor(key, off);
    key = o2 < key ? o2 : key;
  }
  if (lane == 0) best[r] = key;
}

// ------------------------------------------------------------------ finalize
// Per range: decode the best key, recompute Sum r T_e(D) exactly, derive k,
// m and S, store the record (accepted, or forced at the last level) or
// queue the four children (Z order) for the next level.
__global__ __launch_bounds__(256) void fs_finalize_kernel(FsGeo g, const uint8_t* img, uint32_t stride,
                                                         const uint32_t* xy, uint32_t R, const uint64_t* best,
                                                         int level, int last, uint32_t thr, uint32_t b_max,
                                                         uint32_t b_min, uint32_t tiles_x, uint4* staging,
                                                         unsigned long long* masks, uint32_t* next_xy,
                                                         uint32_t* next_count) {
  const uint32_t r = blockIdx.x * 256 + threadIdx.x;
  if (r >= R) return;
  const uint32_t B = g.B, n = B * B;
  const uint32_t x = xy[r] & 0xffffu, y = xy[r] >> 16;
  const uint64_t key = best[r];
  const uint32_t idx = (uint32_t)(key & ((1u << kIdxBits) - 1u));
  const uint32_t dom = idx >> 3;
  const int e = (int)(idx & 7u);
  const uint32_t dv = dom / g.nu, du = dom - dv * g.nu;
  const uint8_t* o = domain_origin_ptr(g, du, dv);
  int64_t sr = 0, srr = 0, sd = 0, sdd = 0, srd = 0;
  for (uint32_t i = 0; i < B; ++i)
    for (uint32_t j = 0; j < B; ++j) {
      const int64_t rv = img[(size_t)(y + i) * stride + x + j];
      int si, sj;
      iso_src(e, (int)i, (int)j, (int)B, si, sj);
      const int64_t dvl = o[(size_t)si * g.pitch + sj];
      const int64_t dd = o[(size_t)i * g.pitch + j];
      sr += rv;
      srr += rv * rv;
      sd += dd;
      sdd += dd * dd;
      srd += rv * dvl;
    }
  const int64_t N = n;
  const int64_t Q = N * sdd - sd * sd, P = N * srd - sr * sd, Rr = N * srr - sr * sr;
  int k = 0;
  for (int j = 0; j < 7; ++j) k += ((int64_t)(2 * j + 1) * Q < 16 * P) ? 1 : 0;
  const int64_t f = (int64_t)(k * k) * Q - (int64_t)(16 * k) * P;
  const int64_t m = (2 * sr + N) / (2 * N);
  const int64_t dm = N * m - sr;
  const int64_t S = f + 64 * Rr + 64 * dm * dm;
  const bool accept = last || S < 64 * N * N * (int64_t)thr;
  if (accept) {
    const uint32_t tx = x / b_max, ty = y / b_max;
    const uint32_t lx = (x % b_max) / b_min, ly = (y % b_max) / b_min;
    uint32_t cell = 0;
    for (int bit = 0; bit < 3; ++bit) cell |= (((lx >> bit) & 1u) << (2 * bit)) | (((ly >> bit) & 1u) << (2 * bit + 1));
    const uint32_t L = 31 - __builtin_clz(b_max / b_min) + 1;
    const uint64_t tile = (uint64_t)ty * tiles_x + tx;
    // slots of one-tile blocks: the whole-tile record, then one per cell
    staging[tile * ((1ull << (2 * (L - 1))) + 1) + (B == b_max ? 0u : 1u + cell)] =
        make_record((int)x, (int)y, (int)du, (int)dv, level - 1, 0, e, k, (int)m, 0, 0, 0);
    atomicOr(&masks[tile], 1ull << cell);
  } else {
    const uint32_t q0 = atomicAdd(next_count, 4u);
    const uint32_t b = B / 2;
    next_xy[q0 + 0] = x | (y << 16);
    next_xy[q0 + 1] = (x + b) | (y << 16);
    next_xy[q0 + 2] = x | ((y + b) << 16);
    next_xy[q0 + 3] = (x + b) | ((y + b) << 16);
  }
}

__global__ void fs_level1_kernel(uint32_t w, uint32_t h, uint32_t b_max, uint32_t* xy) {
  const uint32_t tiles_x = w / b_max, n = tiles_x * (h / b_max);
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t ty = i / tiles_x, tx = i - ty * tiles_x;
  xy[i] = (tx * b_max) | ((ty * b_max) << 16);
}

// Exact best match of explicit ranges (no quadtree): one thread per range
// walks the best key's candidate (for parity checks of sampled ranges).
__global__ __launch_bounds__(256) void fs_report_kernel(FsGeo g, const uint8_t* img, uint32_t stride,
                                                       const uint32_t* xy, uint32_t R, const uint64_t* best,
                                                       uint32_t* out) {
  const uint32_t r = blockIdx.x * 256 + threadIdx.x;
  if (r >= R) return;
  const uint32_t B = g.B, n = B * B;
  const uint32_t x = xy[r] & 0xffffu, y = xy[r] >> 16;
  const uint64_t key = best[r];
  const uint32_t idx = (uint32_t)(key & ((1u << kIdxBits) - 1u));
  const uint32_t dom = idx >> 3;
  const int e = (int)(idx & 7u);
  const uint32_t dv = dom / g.nu, du = dom - dv * g.nu;
  const uint8_t* o = domain_origin_ptr(g, du, dv);
  int64_t sr = 0, srr = 0, sd = 0, sdd = 0, srd = 0;
  for (uint32_t i = 0; i < B; ++i)
    for (uint32_t j = 0; j < B; ++j) {
      const int64_t rv = img[(size_t)(y + i) * stride + x + j];
      int si, sj;
      iso_src(e, (int)i, (int)j, (int)B, si, sj);
      const int64_t dvl = o[(size_t)si * g.pitch + sj];
      const int64_t dd = o[(size_t)i * g.pitch + j];
      sr += rv;
      srr += rv * rv;
      sd += dd;
      sdd += dd * dd;
      srd += rv * dvl;
    }
  const int64_t N = n;
  const int64_t Q = N * sdd - sd * sd, P = N * srd - sr * sd, Rr = N * srr - sr * sr;
  int k = 0;
  for (int j = 0; j < 7; ++j) k += ((int64_t)(2 * j + 1) * Q < 16 * P) ? 1 : 0;
  const int64_t f = (int64_t)(k * k) * Q - (int64_t)(16 * k) * P;
  const int64_t m = (2 * sr + N) / (2 * N);
  const int64_t dm = N * m - sr;
  const int64_t S = f + 64 * Rr + 64 * dm * dm;
  out[4 * r + 0] = dom;
  out[4 * r + 1] = (uint32_t)e | ((uint32_t)k << 8) | ((uint32_t)m << 16);
  out[4 * r + 2] = (uint32_t)((uint64_t)S & 0xffffffffu);
  out[4 * r + 3] = (uint32_t)((uint64_t)S >> 32);
}

}  // namespace

// ------------------------------------------------------------------ host side
FsPlan fs_plan(uint32_t w, uint32_t h, uint32_t B) {
  FsPlan pl;
  pl.B = B;
  pl.nu = w - 2 * B + 1;
  pl.nv = h - 2 * B + 1;
  pl.pitch = (w / 2 + 64 + 3) & ~3u;
  pl.prow = h / 2 + 1 + kStripsPerBlock;
  pl.plane_bytes = (size_t)4 * pl.pitch * pl.prow;
  pl.ndom = (uint64_t)pl.nu * pl.nv;
  return pl;
}

static FsGeo geo_of(const FsPlan& pl, uint32_t w, uint32_t h, const uint8_t* planes) {
  FsGeo g;
  g.w = w;
  g.h = h;
  g.B = pl.B;
  g.nu = pl.nu;
  g.nv = pl.nv;
  g.pitch = pl.pitch;
  g.prow = pl.prow;
  g.planes = planes;
  return g;
}

hipError_t fs_planes(const FsPlan& pl, const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride, uint8_t* planes,
                     hipStream_t s) {
  const uint64_t n = pl.plane_bytes;
  hipLaunchKernelGGL(fs_planes_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, img, w, h, stride,
                     planes, pl.pitch, pl.prow);
  return hipGetLastError();
}

hipError_t fs_domain_sums(const FsPlan& pl, uint32_t w, uint32_t h, const uint8_t* planes, uint32_t* sd, double* qd,
                          hipStream_t s) {
  const FsGeo g = geo_of(pl, w, h, planes);
  hipLaunchKernelGGL(fs_domain_sums_kernel, dim3((unsigned)((pl.ndom + 255) / 256)), dim3(256), 0, s, g, sd, qd);
  return hipGetLastError();
}

template <int B, int NF>
static hipError_t fs_search_t(const FsPlan& pl, const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                              const uint8_t* planes, const uint32_t* sd, const double* qd, const uint32_t* xy,
                              uint32_t R, uint8_t* frag, uint32_t* sr, double* alpha, double* beta, uint64_t* best,
                              hipStream_t s) {
  using C = FsCfg<B, NF>;
  const uint32_t nfrag = (R + 3) / 4;
  const uint64_t at = (uint64_t)nfrag * C::KC * 64;
  hipLaunchKernelGGL(fs_build_a_kernel<B>, dim3((unsigned)((at + 255) / 256)), dim3(256), 0, s, img, stride, xy, R,
                     nfrag, frag);
  hipLaunchKernelGGL(fs_range_sums_kernel, dim3((R + 255) / 256), dim3(256), 0, s, img, stride, (uint32_t)B, xy, R,
                     sr, alpha, beta);
  // seed each range's best with its local-search result (the surrounding
  // step-1 domains, identity only): a real candidate whose key the search
  // below either improves or reproduces for that domain, so the minimum is
  // unchanged, while the search's screen starts from a tight threshold
  const FsGeo g = geo_of(pl, w, h, planes);
  hipLaunchKernelGGL(ls_search_kernel<B>, dim3((R + 3) / 4), dim3(256), 0, s, g, img, stride, sd, qd, xy, R, best);
  const uint32_t maxcols = (pl.nu + 1) / 2, maxrows = (pl.nv + 1) / 2;
  const uint32_t xblocks = (maxcols + 31) / 32, tblocks = (maxrows + kStripsPerBlock - 1) / kStripsPerBlock;
  const uint32_t rgroups = (nfrag + 4 * NF - 1) / (4 * NF);
  hipLaunchKernelGGL((fs_gemm_kernel<B, NF>), dim3(rgroups, 4 * xblocks * tblocks), dim3(256), 0, s, g, frag, nfrag,
                     R, alpha, beta, sd, qd, best, xblocks, tblocks);
  return hipGetLastError();
}

size_t fs_frag_bytes(uint32_t B, uint32_t R) {
  const size_t nfrag = (R + 3) / 4;
  return nfrag * 32 * (size_t)B * B;   // 32 rows (4 ranges x 8 isometries) of K = B^2 bytes each
}

hipError_t fs_search(const FsPlan& pl, const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                     const uint8_t* planes, const uint32_t* sd, const double* qd, const uint32_t* xy, uint32_t R,
                     uint8_t* frag, uint32_t* sr, double* alpha, double* beta, uint64_t* best, hipStream_t s) {
  if (R == 0) return hipSuccess;
  // A fragments per wave: two at B = 16 (152 VGPRs, three waves per SIMD);
  // one at B = 8 and 4, whose epilogue is long against their short MFMA
  // chains, so that eight waves per SIMD hide its latency (60 and 54 VGPRs;
  // on C2 99 and 92 us against 134 and 115 us with four fragments)
  switch (pl.B) {
    case 16: return fs_search_t<16, 2>(pl, img, w, h, stride, planes, sd, qd, xy, R, frag, sr, alpha, beta, best, s);
    case 8: return fs_search_t<8, 1>(pl, img, w, h, stride, planes, sd, qd, xy, R, frag, sr, alpha, beta, best, s);
    case 4: return fs_search_t<4, 1>(pl, img, w, h, stride, planes, sd, qd, xy, R, frag, sr, alpha, beta, best, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t ls_search(const FsPlan& pl, const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                     const uint8_t* planes, const uint32_t* sd, const double* qd, const uint32_t* xy, uint32_t R,
                     uint64_t* best, hipStream_t s) {
  if (R == 0) return hipSuccess;
  const FsGeo g = geo_of(pl, w, h, planes);
  const dim3 grid((R + 3) / 4);
  switch (pl.B) {
    case 16: hipLaunchKernelGGL(ls_search_kernel<16>, grid, dim3(256), 0, s, g, img, stride, sd, qd, xy, R, best); break;
    case 8: hipLaunchKernelGGL(ls_search_kernel<8>, grid, dim3(256), 0, s, g, img, stride, sd, qd, xy, R, best); break;
    case 4: hipLaunchKernelGGL(ls_search_kernel<4>, grid, dim3(256), 0, s, g, img, stride, sd, qd, xy, R, best); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t fs_finalize(const FsPlan& pl, const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                       const uint8_t* planes, const uint32_t* xy, uint32_t R, const uint64_t* best, int level,
                       int last, uint32_t thr, uint32_t b_max, uint32_t b_min, uint4* staging, uint64_t* masks,
                       uint32_t* next_xy, uint32_t* next_count, hipStream_t s) {
  if (R == 0) return hipSuccess;
  const FsGeo g = geo_of(pl, w, h, planes);
  hipLaunchKernelGGL(fs_finalize_kernel, dim3((R + 255) / 256), dim3(256), 0, s, g, img, stride, xy, R, best, level,
                     last, thr, b_max, b_min, w / b_max, staging, reinterpret_cast<unsigned long long*>(masks),
                     next_xy, next_count);
  return hipGetLastError();
}

hipError_t fs_report(const FsPlan& pl, const uint8_t* img, uint32_t w, uint32_t h, uint32_t stride,
                     const uint8_t* planes, const uint32_t* xy, uint32_t R, const uint64_t* best, uint32_t* out,
                     hipStream_t s) {
  if (R == 0) return hipSuccess;
  const FsGeo g = geo_of(pl, w, h, planes);
  hipLaunchKernelGGL(fs_report_kernel, dim3((R + 255) / 256), dim3(256), 0, s, g, img, stride, xy, R, best, out);
  return hipGetLastError();
}

hipError_t fs_level1(uint32_t w, uint32_t h, uint32_t b_max, uint32_t* xy, hipStream_t s) {
  const uint32_t n = (w / b_max) * (h / b_max);
  hipLaunchKernelGGL(fs_level1_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w, h, b_max, xy);
  return hipGetLastError();
}

}  // namespace fe
