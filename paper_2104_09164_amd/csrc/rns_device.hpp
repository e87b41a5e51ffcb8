// Device helpers shared by the RNS kernel files (rns_kernels.hip,
// ext_sums.hip): block size, the NTT-domain automorphism, the XCD-aware grid
// decode, the key inner product and the inner-sum accumulation.
#pragma once
#include "he_internal.hpp"
#include "modarith.hpp"

namespace {

constexpr int BS = 256;

__device__ __forceinline__ u32 brev_n(u32 x, u32 logn) { return __builtin_bitreverse32(x) >> (32 - logn); }

// NTT-domain automorphism X -> X^g: output position k reads input position perm(k).
__device__ __forceinline__ u32 galois_perm(u32 k, u32 g, u32 logn) {
  const u32 two_n_mask = (2u << logn) - 1;
  const u32 e = 2 * brev_n(k, logn) + 1;
  const u32 e2 = (e * g) & two_n_mask;
  return brev_n((e2 - 1) >> 1, logn);
}

// XCD-aware decode of a 1-D grid of inner x T workgroups.  Workgroups are
// dealt to the 8 XCDs round-robin by id, so id L runs on XCD L mod 8.  When T
// is a multiple of 8, the `inner` workgroups that share one tile's operands
// (the items or steps of a batch) all land on that tile's XCD, back to back,
// and read the shared words from its L2; otherwise inner index fastest.
__device__ __forceinline__ void xcd_decode(u32 L, u32 inner, u32 T, u32& i, u32& tile) {
  if (T & 7) {
    i = L % inner;
    tile = L / inner;
    return;
  }
  const u32 r = L >> 3;
  i = r % inner;
  tile = (r / inner) * 8 + (L & 7);
}

// Key inner product of one item: u_b = sum_j x_j ksk_{b,j}, u_a = sum_j x_j ksk_{a,j}
// with Shoup products by the key words (companions kbs / kas), the sum
// folded into the product's low-word chain (add_shoup4).  LAZY (q < 2^58):
// at most 8 terms below 4q each, so the sum stays below 32q; otherwise it is
// kept below 4q after every term.  The outputs are left lazy for their
// consumers: Q-limbs (below 32q) are read only as u + q - conv by a Shoup
// product, which takes any 64-bit input; P-limbs feed the inverse NTT, which
// takes inputs below 4q (reduce_lazy brings a lazy sum there).
constexpr u64 kLazyKS = 1ull << 58;
template <int BETA, bool LAZY>
__device__ __forceinline__ void ks_dot(const u64 (&x)[BETA], const u64 (&kb)[BETA], const u64 (&kbs)[BETA],
                                       const u64 (&ka)[BETA], const u64 (&kas)[BETA], const PrimeConst& P,
                                       bool p_limb, u64& ob, u64& oa) {
  u64 sb = 0, sa = 0;
#pragma unroll
  for (int j = 0; j < BETA; ++j) {
    sb = add_shoup4(sb, x[j], kb[j], kbs[j], P.nq);
    sa = add_shoup4(sa, x[j], ka[j], kas[j], P.nq);
    if (!LAZY) {
      sb = csub_neg(sb, P.nq4);
      sa = csub_neg(sa, P.nq4);
    }
  }
  if (LAZY && p_limb) {
    sb = reduce_lazy(sb, P.q, P.mu);
    sa = reduce_lazy(sa, P.q, P.mu);
  }
  ob = sb;
  oa = sa;
}

// Inner-sum accumulation of products pt (.) x, pt with its Shoup companion
// ps: each product is in [0, 4q).  LAZY (q < 2^55): plain 64-bit sums — at
// most 65 terms (the baby-step limit) stay below 260 q < 2^64 — reduced once
// at the end; otherwise the sum is kept below 4q after every term.
constexpr u64 kLazyMP = 1ull << 55;
template <bool LAZY>
__device__ __forceinline__ u64 mp_add(u64 acc, u64 x, u64 pt, u64 ps, const PrimeConst& k) {
  const u64 p = shoup_lazy4(x, pt, ps, k.q);
  return LAZY ? acc + p : csub_neg(acc + p, k.nq4);
}
template <bool LAZY>
__device__ __forceinline__ u64 mp_final(u64 acc, const PrimeConst& k) {
  if (LAZY) acc = reduce_lazy(acc, k.q, k.mu);   // -> [0, 4q)
  return csub_neg(csub_neg(acc, k.nq2), k.nq);
}

// Key inner product of the fused kernels for 2^55 <= q < 2^60 and at most 4
// digits: the products (each in [0, 4q)) summed without reduction (below 16q
// < 2^64), then one conditional subtraction of 8q (below 8q, so that the lift
// of c0, below 2q, can still be added).  The fused kernels' consumers take any
// 64-bit input and reduce at the end, so no other reduction is needed.
template <int BETA>
__device__ __forceinline__ void ks_dot_mid(const u64 (&x)[BETA], const u64 (&kb)[BETA], const u64 (&kbs)[BETA],
                                           const u64 (&ka)[BETA], const u64 (&kas)[BETA], const PrimeConst& P,
                                           u64& ob, u64& oa) {
  static_assert(BETA <= 4, "the lazy sum of at most 4 products stays below 16q");
  u64 sb = 0, sa = 0;
#pragma unroll
  for (int j = 0; j < BETA; ++j) {
    sb = add_shoup4(sb, x[j], kb[j], kbs[j], P.nq);
    sa = add_shoup4(sa, x[j], ka[j], kas[j], P.nq);
  }
  ob = csub_signed(sb, P.q << 3);
  oa = csub_signed(sa, P.q << 3);
}
// Inner sums of the fused kernels for 2^55 <= q < 2^60: products (each below
// 4q) added without reduction; the caller brings the running sum below 3q
// by reduce_lazy_wide before every third product (at most 3q + 3 * 4q =
// 15q < 2^64); closed by mp_final<true>.
constexpr u64 kMidQ = 1ull << 60;
__device__ __forceinline__ u64 mp_add_mid(u64 acc, u64 x, u64 pt, u64 ps, const PrimeConst& k) {
  return acc + shoup_lazy4(x, pt, ps, k.q);
}

// Exact column sums for primes below 2^50 (the fused kernels): a value r
// (below 2^56) and a word b (below 2^50, given as its 28-bit columns b0, b1)
// are multiplied as r = a1 2^28 + a0 by four 32 x 32 -> 64-bit multiply-adds
// into column sums C0 += a0 b0, C1 += a0 b1 + a1 b0, C2 += a1 b1; the sum
// C0 + C1 2^28 + C2 2^56 is reduced mod q once at the end.
constexpr u64 kLow28 = (1ull << 28) - 1;
constexpr u64 kWideQ = 1ull << 50;
__device__ __forceinline__ void col_mad(u64 (&c)[3], u64 r, u64 b0, u64 b1) {
  const u32 a0 = (u32)(r & kLow28), a1 = (u32)(r >> 28);
  c[0] = (u64)a0 * (u32)b0 + c[0];
  c[1] = (u64)a0 * (u32)b1 + c[1];
  c[1] = (u64)a1 * (u32)b0 + c[1];
  c[2] = (u64)a1 * (u32)b1 + c[2];
}
// C0 + C1 2^28 + C2 2^56 mod q, lazily: below 11 q (any 64-bit columns).
__device__ __forceinline__ u64 col_lazy(const u64 (&c)[3], const PrimeConst& P) {
  return reduce_lazy(c[0], P.q, P.mu) + shoup_lazy4(c[1], P.t28, P.t28_sh, P.q) +
         shoup_lazy4(c[2], P.t56, P.t56_sh, P.q);
}
// The same in [0, q).
__device__ __forceinline__ u64 col_final(const u64 (&c)[3], const PrimeConst& P) {
  const u64 v = reduce_lazy(col_lazy(c, P), P.q, P.mu);
  return csub_neg(csub_neg(v, P.nq2), P.nq);
}

inline int ok() { return hipGetLastError() == hipSuccess ? HE_OK : HE_EDEVICE; }

}  // namespace
