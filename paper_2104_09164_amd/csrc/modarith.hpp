// Exact 64-bit modular arithmetic for CDNA4 (gfx950) device code.
//
// Residues are uint64 words for primes q < 2^61.  gfx950 has no 64x64-bit
// multiply; the compiler builds 64-bit products from v_mad_u64_u32 /
// v_mul_lo_u32 / v_mul_hi_u32, which run at or near full VALU rate there.
//
//  * Shoup multiplication by a constant w with companion w' = floor(w 2^64/q):
//    x*w - mulhi(x, w')*q lies in [0, 2q) for any 64-bit x.  Used for NTT
//    twiddles and every per-prime constant.
//  * Montgomery reduction (R = 2^64) of 128-bit sums of products: keys,
//    plaintexts and base-conversion constants are stored premultiplied by R,
//    so a lazily accumulated sum of up to floor((2^64-1)/q) products needs one
//    reduction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint64_t u64;
typedef uint32_t u32;

struct u128v { u64 lo, hi; };

__device__ __forceinline__ u128v mul_wide(u64 a, u64 b) {
  u128v r; r.lo = a * b; r.hi = __umul64hi(a, b); return r;
}
__device__ __forceinline__ void acc_wide(u128v& s, u64 a, u64 b) {
  u64 lo = a * b, hi = __umul64hi(a, b);
  s.lo += lo; s.hi += hi + (s.lo < lo);
}
// x in [0, 2q) -> [0, q)
__device__ __forceinline__ u64 csub(u64 x, u64 q) { return x >= q ? x - q : x; }
__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) { return csub(a + b, q); }          // a, b < q
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }  // a, b < q
// Shoup: [0, 2q) for any x
__device__ __forceinline__ u64 shoup_lazy(u64 x, u64 w, u64 wsh, u64 q) {
  return x * w - __umul64hi(x, wsh) * q;
}
__device__ __forceinline__ u64 shoup(u64 x, u64 w, u64 wsh, u64 q) { return csub(shoup_lazy(x, w, wsh, q), q); }
// Shoup product with a three-term quotient estimate: the low x 32-bit
// partial product and the carries of the middle terms are dropped, so the
// quotient is low by at most 2 and the result lies in [0, 4q) for any 64-bit
// x (q < 2^61 keeps 8q below 2^64).  One v_mad_u64_u32 and two v_mul_hi_u32
// instead of the four-product carry chain of the exact high half.
__device__ __forceinline__ u64 shoup_lazy4(u64 x, u64 w, u64 wsh, u64 q) {
  const u32 x0 = (u32)x, x1 = (u32)(x >> 32), s0 = (u32)wsh, s1 = (u32)(wsh >> 32);
  const u64 mid = (u64)__umulhi(x1, s0) + (u64)__umulhi(x0, s1);
  const u64 qh = (u64)x1 * s1 + mid;
  return x * w - qh * q;
}
// X + (x w mod q) for X < 2^64 - 4q: the Shoup product of shoup_lazy4 with
// the subtraction of qh q folded into the low-64-bit accumulation chain as
// + qh (2^64 - q):  t = x0 w0 + X + qh0 nq0 (two v_mad_u64_u32), high word
// + lo32 of the four cross products.  nq = 2^64 - q.  Result X + T with T in
// [0, 4q) (exact as an integer while X + 4q < 2^64).
__device__ __forceinline__ u64 add_shoup4(u64 X, u64 x, u64 w, u64 wsh, u64 nq) {
  const u32 x0 = (u32)x, x1 = (u32)(x >> 32), s0 = (u32)wsh, s1 = (u32)(wsh >> 32);
  const u32 w0 = (u32)w, w1 = (u32)(w >> 32), n0 = (u32)nq, n1 = (u32)(nq >> 32);
  const u64 qh = (u64)x1 * s1 + ((u64)__umulhi(x1, s0) + (u64)__umulhi(x0, s1));
  const u32 h0 = (u32)qh, h1 = (u32)(qh >> 32);
  u64 t = (u64)x0 * w0 + X;
  t = (u64)h0 * n0 + t;
  const u32 hi = (u32)(t >> 32) + x1 * w0 + x0 * w1 + h1 * n0 + h0 * n1;
  return ((u64)hi << 32) | (u32)t;
}
// x mod q up to a small multiple: [0, 4q) for any 64-bit x, from the Shoup
// product by 1 (companion mu = floor(2^64/q)).  When q > 2^32, mu fits 32
// bits and one 32-bit high product of the top word estimates the quotient:
// qh = floor(x1 mu / 2^32) <= floor(x/q) <= qh + 2 (the dropped x0 mu / 2^64
// and the rounding of mu each cost less than 1), so x - qh q is in [0, 3q).
// reduce_lazy's q > 2^32 path on its own, for callers whose primes are all
// above 2^32 (no branch on mu in the loop).
__device__ __forceinline__ u64 reduce_lazy_wide(u64 x, u64 q, u64 mu) {
  const u32 qh = __umulhi((u32)(x >> 32), (u32)mu);
  return x - (u64)qh * q;
}
__device__ __forceinline__ u64 reduce_lazy(u64 x, u64 q, u64 mu) {
  if (mu >> 32) return shoup_lazy4(x, 1, mu, q);
  return reduce_lazy_wide(x, q, mu);
}

// x < 2m (m <= 2^63): x - m if x >= m; negm = 2^64 - m supplied from memory so
// that the difference is one 64-bit add (v_lshl_add_u64) instead of a
// subtract-with-borrow pair.
__device__ __forceinline__ u64 csub_neg(u64 x, u64 negm) {
  const u64 d = x + negm;
  return (int64_t)d < 0 ? x : d;
}
// x < 2m (m <= 2^62): x - m if x >= m, by the sign of the 64-bit difference.
__device__ __forceinline__ u64 csub_signed(u64 x, u64 m) {
  const u64 d = x - m;
  return (int64_t)d < 0 ? x : d;
}
// Montgomery REDC of s < q 2^64: s 2^-64 mod q in [0, q).  qneg = -q^{-1} mod 2^64.
__device__ __forceinline__ u64 redc(u128v s, u64 q, u64 qneg) {
  u64 m = s.lo * qneg;
  u64 t = s.hi + __umul64hi(m, q) + (s.lo != 0);
  return csub(t, q);
}
// x mod q for any 64-bit x, with mu = floor(2^64 / q) (q >= 2^20).
__device__ __forceinline__ u64 reduce64(u64 x, u64 q, u64 mu) {
  u64 r = x - __umul64hi(x, mu) * q;   // in [0, 3q) at most: floor error <= 2
  r = csub(r, q);
  return csub(r, q);
}
