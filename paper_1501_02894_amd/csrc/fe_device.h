// Device helpers of the MNS encoder: packed-u8 moment accumulation from LDS,
// team reductions over DPP, and the exact integer fits of phase 1 and phase 2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fe {

template <int V>
struct Log2 {
  static constexpr int value = 1 + Log2<V / 2>::value;
};
template <>
struct Log2<1> {
  static constexpr int value = 0;
};

__device__ __forceinline__ uint32_t dot4(uint32_t a, uint32_t b, uint32_t acc) {
  return __builtin_amdgcn_udot4(a, b, acc, false);
}

// Sum over lanes of aligned power-of-two teams (T <= 16, within a DPP row).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_read(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

template <int N>
__device__ __forceinline__ void team_reduce(uint32_t (&a)[N], int T) {
  if (T >= 2) {
#pragma unroll
    for (int j = 0; j < N; ++j) a[j] += dpp_read<0xB1>(a[j]);   // quad_perm 1,0,3,2
  }
  if (T >= 4) {
#pragma unroll
    for (int j = 0; j < N; ++j) a[j] += dpp_read<0x4E>(a[j]);   // quad_perm 2,3,0,1
  }
  if (T >= 8) {
#pragma unroll
    for (int j = 0; j < N; ++j) a[j] += dpp_read<0x141>(a[j]);  // row_half_mirror
  }
  if (T >= 16) {
#pragma unroll
    for (int j = 0; j < N; ++j) a[j] += dpp_read<0x140>(a[j]);  // row_mirror
  }
}

// Q dwords of the LDS row starting at byte address p (4-byte aligned when
// ALIGNED).
template <int Q, bool ALIGNED>
__device__ __forceinline__ void lds_row_at(const uint8_t* p, uint32_t (&o)[Q]) {
  if constexpr (ALIGNED) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
    for (int q = 0; q < Q; ++q) o[q] = w[q];
  } else {
    const uint32_t sh = (uint32_t)(uintptr_t)p & 3u;
    const uint32_t* w = reinterpret_cast<const uint32_t*>(p - sh);
    uint32_t v[Q + 1];
#pragma unroll
    for (int q = 0; q <= Q; ++q) v[q] = w[q];
#pragma unroll
    for (int q = 0; q < Q; ++q) o[q] = __builtin_amdgcn_alignbyte(v[q + 1], v[q], sh);
  }
}

// Moment slots: 0 Sum r, 1 Sum r^2, 2 Sum d, 3 Sum d^2, 4+e Sum r T_e(d).
//
// Adds the contribution of range rows i and B-1-i, given by the LDS byte
// addresses of their first pixels: range rows ra, rb (dword aligned), rows i
// and B-1-i of the B x B domain window d (da, db) and of its transpose
// (ta, tb), dT[i][j] = d[j][i].
//
// With rrev the range with each row reversed, the eight isometries of the
// table T_e(d)[i][j] = d[i][j], d[i][B-1-j], d[B-1-i][j], d[B-1-i][B-1-j],
// d[j][i], d[B-1-j][i], d[j][B-1-i], d[B-1-j][B-1-i] give, per row i
// (i' = B-1-i):  e0 r_i.d_i, e1 rrev_i.d_i, e2 r_i.d_i', e3 rrev_i.d_i',
// e4 r_i.dT_i, e5 rrev_i.dT_i, e6 r_i.dT_i', e7 rrev_i.dT_i'.
template <int Q>
__device__ __forceinline__ void accumulate_words(const uint32_t (&ra)[Q], const uint32_t (&rb)[Q],
                                                 const uint32_t (&da)[Q], const uint32_t (&db)[Q],
                                                 const uint32_t (&ta)[Q], const uint32_t (&tb)[Q],
                                                 uint32_t (&a)[12]) {
  const uint32_t ones = 0x01010101u;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const uint32_t xa = ra[q], xb = rb[q];
    const uint32_t ya = __builtin_bswap32(ra[Q - 1 - q]);   // rrev_i, dword q
    const uint32_t yb = __builtin_bswap32(rb[Q - 1 - q]);
    a[0] = dot4(xa, ones, dot4(xb, ones, a[0]));
    a[1] = dot4(xa, xa, dot4(xb, xb, a[1]));
    a[2] = dot4(da[q], ones, dot4(db[q], ones, a[2]));
    a[3] = dot4(da[q], da[q], dot4(db[q], db[q], a[3]));
    a[4] = dot4(xa, da[q], dot4(xb, db[q], a[4]));
    a[5] = dot4(ya, da[q], dot4(yb, db[q], a[5]));
    a[6] = dot4(xa, db[q], dot4(xb, da[q], a[6]));
    a[7] = dot4(ya, db[q], dot4(yb, da[q], a[7]));
    a[8] = dot4(xa, ta[q], dot4(xb, tb[q], a[8]));
    a[9] = dot4(ya, ta[q], dot4(yb, tb[q], a[9]));
    a[10] = dot4(xa, tb[q], dot4(xb, ta[q], a[10]));
    a[11] = dot4(ya, tb[q], dot4(yb, ta[q], a[11]));
  }
}

template <int B, bool ALIGNED>
__device__ __forceinline__ void accumulate_rows(const uint8_t* rap, const uint8_t* rbp, const uint8_t* dap,
                                                const uint8_t* dbp, const uint8_t* tap, const uint8_t* tbp,
                                                uint32_t (&a)[12]) {
  constexpr int Q = B / 4;
  uint32_t ra[Q], rb[Q], da[Q], db[Q], ta[Q], tb[Q];
  lds_row_at<Q, true>(rap, ra);
  lds_row_at<Q, true>(rbp, rb);
  lds_row_at<Q, ALIGNED>(dap, da);
  lds_row_at<Q, ALIGNED>(dbp, db);
  lds_row_at<Q, ALIGNED>(tap, ta);
  lds_row_at<Q, ALIGNED>(tbp, tb);
  accumulate_words<Q>(ra, rb, da, db, ta, tb, a);
}

// Q dwords of an LDS row that starts sh bytes (0..3) after the dword w.
template <int Q, bool ALIGNED>
__device__ __forceinline__ void lds_row_sh(const uint32_t* w, uint32_t sh, uint32_t (&o)[Q]) {
  if constexpr (ALIGNED) {
#pragma unroll
    for (int q = 0; q < Q; ++q) o[q] = w[q];
  } else {
    uint32_t v[Q + 1];
#pragma unroll
    for (int q = 0; q <= Q; ++q) v[q] = w[q];
#pragma unroll
    for (int q = 0; q < Q; ++q) o[q] = __builtin_amdgcn_alignbyte(v[q + 1], v[q], sh);
  }
}

// accumulate_rows for windows whose rows all share one byte shift: the
// range rows ra, rb and the dword before each window row (da, db: H0, shd
// bytes in; ta, tb: H0^T, sht bytes in), so that the shifts and aligned
// addresses are formed once per range rather than once per row.
template <int B, bool ALIGNED>
__device__ __forceinline__ void accumulate_rows_sh(const uint32_t* rap, const uint32_t* rbp, const uint32_t* dap,
                                                   const uint32_t* dbp, const uint32_t* tap, const uint32_t* tbp,
                                                   uint32_t shd, uint32_t sht, uint32_t (&a)[12]) {
  constexpr int Q = B / 4;
  uint32_t ra[Q], rb[Q], da[Q], db[Q], ta[Q], tb[Q];
  lds_row_sh<Q, true>(rap, 0u, ra);
  lds_row_sh<Q, true>(rbp, 0u, rb);
  lds_row_sh<Q, ALIGNED>(dap, shd, da);
  lds_row_sh<Q, ALIGNED>(dbp, shd, db);
  lds_row_sh<Q, ALIGNED>(tap, sht, ta);
  lds_row_sh<Q, ALIGNED>(tbp, sht, tb);
  accumulate_words<Q>(ra, rb, da, db, ta, tb, a);
}

// The same for the range at byte offset r_off of `img` (row pitch rp), the
// domain window at byte offset d_off of `h0` (pitch hp) and its transpose at
// byte offset t_off of `h0t` (pitch tp).
template <int B, bool ALIGNED>
__device__ __forceinline__ void accumulate_row_pair(const uint32_t* img, int r_off, int rp,
                                                    const uint32_t* h0, int d_off, int hp,
                                                    const uint32_t* h0t, int t_off, int tp, int i,
                                                    uint32_t (&a)[12]) {
  const int ia = i, ib = B - 1 - i;
  const uint8_t* im = reinterpret_cast<const uint8_t*>(img);
  const uint8_t* hd = reinterpret_cast<const uint8_t*>(h0);
  const uint8_t* ht = reinterpret_cast<const uint8_t*>(h0t);
  accumulate_rows<B, ALIGNED>(im + r_off + ia * rp, im + r_off + ib * rp, hd + d_off + ia * hp, hd + d_off + ib * hp,
                              ht + t_off + ia * tp, ht + t_off + ib * tp, a);
}

// Phase-1 fit packed as: bits 0-7 m, 8-10 k, 11-13 e, bit 14 accept.
constexpr uint32_t kFitAccept = 1u << 14;
constexpr uint32_t kFitDead = 1u << 15;   // set when the parent was stored by phase 2

// Best (e, k/8) and luminance m of a B x B range from its moments, and
// whether the scaled collage error S = 64 n E is below 64 n^2 t (or the
// level is forced).  f(P) = min_k (k^2 Q - 16 k P) is non-increasing in P
// and strictly decreasing where the minimising k is >= 1, so the best
// isometry is the lowest e of maximal Sum r T_e(d) unless that P gives
// k = 0, in which case every isometry scores 0 and e = 0.
//
// The arithmetic is float64 but exact: every operand and every partial
// result is an integer of magnitude below 2^53 (n <= 1024, sums of 8-bit
// pixels: products below 2^37, k^2 Q and 16 k P below 2^44); the threshold
// 64 n^2 t is t times a power of two, hence exact too.
template <int B>
__device__ __forceinline__ uint32_t fit_phase1(const uint32_t (&m)[12], bool forced, uint32_t t) {
  constexpr int LOGN = 2 * Log2<B>::value;
  constexpr double N = (double)(B * B);
  uint32_t best = m[4];
  int e = 0;
#pragma unroll
  for (int j = 1; j < 8; ++j) {
    if (m[4 + j] > best) {
      best = m[4 + j];
      e = j;
    }
  }
  const double sr = (double)m[0], srr = (double)m[1], sd = (double)m[2], sdd = (double)m[3];
  const double Q = N * sdd - sd * sd;
  const double P = N * (double)best - sr * sd;
  const double P16 = 16.0 * P;
  // k = #{j in 0..6 : (2j+1) Q < 16 P}; the predicate is monotone in j, so
  // three tests of a binary search find the count
  int k = (7.0 * Q < P16) ? 4 : 0;
  k += ((double)(2 * k + 3) * Q < P16) ? 2 : 0;
  k += ((double)(2 * k + 1) * Q < P16) ? 1 : 0;
  if (k == 0) e = 0;
  const double kd = (double)k;
  const double f = (kd * kd) * Q - (16.0 * kd) * P;
  const uint32_t lum = (2u * m[0] + (uint32_t)(B * B)) >> (LOGN + 1);
  const double R = N * srr - sr * sr;
  const double dm = (double)lum * N - sr;
  const double S = f + 64.0 * R + 64.0 * (dm * dm);
  const bool acc = forced || S < (64.0 * N * N) * (double)t;
  return lum | ((uint32_t)k << 8) | ((uint32_t)e << 11) | (acc ? kFitAccept : 0u);
}

// The same phase-1 fit for the fused encoder, which also hands the terms
// Technique 1 reuses to its caller.  The best isometry is found with one
// key per isometry, Sum r T_e(d) << 3 | (7 - e) (every sum is below 2^27,
// B <= 32), whose maximum is the largest sum at the lowest e.  `thr64` is
// 64 n^2 t as a double, or +infinity at a forced level; every other
// quantity is the exact integer arithmetic of fit_phase1.
struct Fit1 {
  double Q, R, srsd;   // n Sum d^2 - (Sum d)^2, n Sum r^2 - (Sum r)^2, Sum r Sum d
  uint32_t lum, k, e;
  bool accept;
};

template <int B>
__device__ __forceinline__ Fit1 fit_phase1_terms(const uint32_t (&m)[12], double thr64) {
  constexpr int LOGN = 2 * Log2<B>::value;
  constexpr double N = (double)(B * B);
  uint32_t key[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) key[j] = (m[4 + j] << 3) | (uint32_t)(7 - j);
  const uint32_t k012 = max(max(key[0], key[1]), key[2]);
  const uint32_t k345 = max(max(key[3], key[4]), key[5]);
  const uint32_t top = max(max(k012, k345), max(key[6], key[7]));
  Fit1 r;
  const double sr = (double)m[0], sd = (double)m[2];
  r.srsd = sr * sd;
  r.Q = N * (double)m[3] - sd * sd;
  r.R = N * (double)m[1] - sr * sr;
  const double P = N * (double)(top >> 3) - r.srsd;
  const double P16 = 16.0 * P;
  // k = #{j in 0..6 : (2j+1) Q < 16 P}, a monotone predicate: three tests
  uint32_t k = (7.0 * r.Q < P16) ? 4u : 0u;
  k += ((double)(2 * k + 3) * r.Q < P16) ? 2u : 0u;
  k += ((double)(2 * k + 1) * r.Q < P16) ? 1u : 0u;
  r.k = k;
  r.e = k ? 7u - (top & 7u) : 0u;
  const double f = (double)(k * k) * r.Q - (double)(16 * k) * P;
  r.lum = (2u * m[0] + (uint32_t)(B * B)) >> (LOGN + 1);
  const double dm = (double)((int)(r.lum << LOGN) - (int)m[0]);
  const double S = f + 64.0 * (r.R + dm * dm);
  r.accept = S < thr64;
  return r;
}

// Phase-2 contrast sets (twentieths) and mean-difference bounds per level
// 1..3: {.2,.5}, {.4,.65}, {.5,.9}; 5-bit (level 1) and 6-bit (levels 2, 3)
// signed differences.
__device__ __forceinline__ void phase2_consts(int level, int& c1, int& c2, int& delta) {
  c1 = level == 1 ? 4 : (level == 2 ? 8 : 10);
  c2 = level == 1 ? 10 : (level == 2 ? 13 : 18);
  delta = level == 1 ? 15 : 31;
}

// Technique 1 for one parent whose four children (side b, Z order) have
// identity moments mom[c] = {Sum r, Sum r^2, Sum d, Sum d^2, Sum r d}.
// Returns accept; fills O_0..O_2 (O_3 by eq. (1)) and the contrast bits.
// float64, exact as in fit_phase1 (c <= 18, n_b <= 256: every partial
// result below 2^44; a threshold above 2^53 exceeds every S, so its
// rounding cannot change the comparison).
template <int b>
__device__ __forceinline__ bool fit_phase2(const uint32_t (&mom)[4][5], int m, int level, uint32_t t,
                                           int (&O)[4], uint32_t& bits) {
  constexpr int LOGNB = 2 * Log2<b>::value;
  constexpr double NB = (double)(b * b);
  int c1, c2, delta;
  phase2_consts(level, c1, c2, delta);
#pragma unroll
  for (int c = 0; c < 3; ++c) O[c] = (int)((2u * mom[c][0] + (uint32_t)(b * b)) >> (LOGNB + 1));
  O[3] = 4 * m - O[0] - O[1] - O[2];
  bool ok = O[3] >= 0 && O[3] <= 255;
#pragma unroll
  for (int c = 0; c < 4; ++c) ok = ok && (O[c] - m <= delta) && (m - O[c] <= delta);
  const double thr = (400.0 * NB * NB) * (double)t;
  const double a1 = (double)(c1 * c1), b1 = (double)(40 * c1);
  const double a2 = (double)(c2 * c2), b2 = (double)(40 * c2);
  bits = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double sr = (double)mom[c][0], srr = (double)mom[c][1], sd = (double)mom[c][2];
    const double sdd = (double)mom[c][3], srd = (double)mom[c][4];
    const double Q = NB * sdd - sd * sd;
    const double P = NB * srd - sr * sd;
    const double R = NB * srr - sr * sr;
    const double f1 = a1 * Q - b1 * P;
    const double f2 = a2 * Q - b2 * P;
    const bool use2 = f2 < f1;
    const double dm = (double)O[c] * NB - sr;
    const double S = (use2 ? f2 : f1) + 400.0 * R + 400.0 * (dm * dm);
    ok = ok && S < thr;
    bits |= (use2 ? 1u : 0u) << c;
  }
  return ok;
}

// Record words (little-endian fe_transform).
__device__ __forceinline__ uint4 make_record(int x, int y, int dx, int dy, int level, int flags,
                                             int iso, int s_idx, int lum, int d0, int d1, int d2) {
  uint4 w;
  w.x = (uint32_t)x | ((uint32_t)y << 16);
  w.y = (uint32_t)dx | ((uint32_t)dy << 16);
  w.z = (uint32_t)level | ((uint32_t)flags << 8) | ((uint32_t)iso << 16) | ((uint32_t)s_idx << 24);
  w.w = (uint32_t)lum | (((uint32_t)d0 & 0xffu) << 8) | (((uint32_t)d1 & 0xffu) << 16) |
        (((uint32_t)d2 & 0xffu) << 24);
  return w;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Four round-half-up 2x2 means of an 8-wide, 2-row pixel group:
// a0/a1 = row 0 pixels 0-3 / 4-7, b0/b1 = row 1.  Column pairs are first
// averaged down (v_lerp_u8, per byte floor((a + b) / 2)); with u_e, u_o the
// averages of the even and odd column of an output pixel and c_e, c_o the
// bits they dropped ((a ^ b) & 1), the mean (sum + 2) >> 2 equals
// (u_e + (c_e & c_o) + u_o + 1) >> 1, a second v_lerp_u8 with rounding bit
// 1 (u_e + 1 cannot overflow: c_e = 1 implies u_e <= 254).
__device__ __forceinline__ uint32_t mean2x2_x4(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1) {
  const uint32_t u0 = __builtin_amdgcn_lerp(a0, b0, 0u), u1 = __builtin_amdgcn_lerp(a1, b1, 0u);
  const uint32_t x0 = a0 ^ b0, x1 = a1 ^ b1;
  constexpr uint32_t EVEN = 0x06040200u, ODD = 0x07050301u;   // bytes 0, 2 of lo, then of hi
  const uint32_t ue = __builtin_amdgcn_perm(u1, u0, EVEN), uo = __builtin_amdgcn_perm(u1, u0, ODD);
  const uint32_t cc = __builtin_amdgcn_perm(x1, x0, EVEN) & __builtin_amdgcn_perm(x1, x0, ODD) & 0x01010101u;
  return __builtin_amdgcn_lerp(ue + cc, uo, 0x01010101u);
}

}  // namespace fe
