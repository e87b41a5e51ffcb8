// RNS kernels of hybrid key switching, BSGS inner sums, squaring and rescale.
//
// Every kernel is HBM-streaming: one thread per coefficient index k, 256
// threads per block, consecutive threads on consecutive words of a limb-poly
// (limb-major [.][limb][N] layouts), so each wavefront reads and writes
// contiguous 512-byte runs.  Per-prime constants come from small device tables
// (broadcast loads).  Arithmetic: Shoup products by constants, keys and
// plaintexts (stored with their companions, sums kept lazily below a bound),
// and lazy 128-bit sums of products closed by one Montgomery reduction for
// the base conversions and the tensor.
#include "rns_kernels.hpp"
#include "modarith.hpp"
#include "rns_device.hpp"

namespace {

__global__ void __launch_bounds__(BS) k_copy_polys(PolyBatch pb, u32 N) {
  const u32 b = blockIdx.y, r = blockIdx.z;
  if (pb.prime[r] == 0xFF) return;
  const u64* src = pb.src[b] + (size_t)(pb.src_off + r) * N;
  u64* dst = pb.dst[b] + (size_t)(pb.dst_off + r) * N;
  for (u32 k = blockIdx.x * BS + threadIdx.x; k < N; k += gridDim.x * BS) dst[k] = src[k];
}

// Lazy sum of up to 8 Shoup products (each in [0, 4q)) into acc: below 32q
// for q < 2^59 (reduced once by conv_final); otherwise kept below 4q.
template <bool LAZY>
__device__ __forceinline__ u64 conv_add(u64 acc, u64 v, const u64* __restrict__ pair, const PrimeConst& P) {
  acc = add_shoup4(acc, v, pair[0], pair[1], P.nq);
  return LAZY ? acc : csub_neg(acc, P.nq4);
}
template <bool LAZY>
__device__ __forceinline__ u64 conv_final(u64 acc, const PrimeConst& P) {
  if (LAZY) acc = reduce_lazy(acc, P.q, P.mu);
  return csub_neg(csub_neg(acc, P.nq2), P.nq);
}

// grid: (N/BS, beta, B); A = digit size alpha (the last digit may hold fewer limbs)
template <int A>
__global__ void __launch_bounds__(BS) k_modup_conv(const u64* __restrict__ coef, u64* __restrict__ ext,
                                                   const PrimeConst* __restrict__ pc, const u64* __restrict__ hatinv,
                                                   const u64* __restrict__ hatmod, u32 N, u32 l, u32 nq, u32 np,
                                                   u32 dnum) {
  const u32 k = blockIdx.x * BS + threadIdx.x;
  const u32 j = blockIdx.y, b = blockIdx.z;
  const u32 ne = l + 1 + np, nt = nq + np;
  const u32 lo = j * A, hi = min((j + 1) * A, l + 1), cnt = hi - lo;
  const size_t tab = ((size_t)l * dnum + j) * A;
  u64 v[A];
#pragma unroll
  for (int i = 0; i < A; ++i) {
    v[i] = 0;
    if ((u32)i < cnt) {
      const u64 q = pc[lo + i].q;
      const u64 x = coef[((size_t)b * (l + 1) + lo + i) * N + k];
      v[i] = shoup(x, hatinv[(tab + i) * 2], hatinv[(tab + i) * 2 + 1], q);
    }
  }
  u64* out = ext + ((size_t)b * dnum + j) * ne * N;
  // dnum here is the allocation stride of digits per item (maximum digits)
  for (u32 t = 0; t < ne; ++t) {
    if (t >= lo && t < hi) continue;
    const u32 pr = t <= l ? t : nq + (t - l - 1);
    const PrimeConst P = pc[pr];
    u64 s = 0;
    if (P.q < (1ull << 59)) {
#pragma unroll
      for (int i = 0; i < A; ++i)
        if ((u32)i < cnt) s = conv_add<true>(s, v[i], hatmod + 2 * ((tab + i) * nt + pr), P);
      s = conv_final<true>(s, P);
    } else {
#pragma unroll
      for (int i = 0; i < A; ++i)
        if ((u32)i < cnt) s = conv_add<false>(s, v[i], hatmod + 2 * ((tab + i) * nt + pr), P);
      s = conv_final<false>(s, P);
    }
    out[(size_t)t * N + k] = s;
  }
}

// 1-D grid over S x (N/BS, ne) tiles: the steps of a tile share its extended
// digits (xcd_decode).  The automorphism moves to the output side: with
// k' = perm_{g^{-1}}(k), u_s[k'] = sum_j d_j[k] ksk_{s,j}[k'] equals
// sum_j d_j[perm_g(k')] ksk_{s,j}[k'], so every step reads the same
// (unpermuted) digit words of a tile, from L2 after the first step, and
// gathers its key and scatters its output within the same aligned groups.
// BETA = digits at this level.
template <int BETA, bool LAZY>
__device__ __forceinline__ void ks_inner_body(const u64* __restrict__ ext, u32 ext_items, const OwnMap& own,
                                              const u64* __restrict__ key, u64* __restrict__ u, const PrimeConst& P,
                                              u32 N, u32 l, u32 nt, u32 ne, u32 pr, u32 dstride, u32 nitems,
                                              u32 alpha, u32 s, u32 k, u32 ko, u32 t) {
  const size_t kw = (size_t)dstride * 2 * nt * N;          // companions follow the key words
  u64 kb[BETA], kbs[BETA], ka[BETA], kas[BETA];
#pragma unroll
  for (int j = 0; j < BETA; ++j) {
    const size_t ob = (((size_t)j * 2 + 0) * nt + pr) * N + ko, oa = (((size_t)j * 2 + 1) * nt + pr) * N + ko;
    kb[j] = key[ob];
    kbs[j] = key[kw + ob];
    ka[j] = key[oa];
    kas[j] = key[kw + oa];
  }
  const u32 own_digit = t <= l ? t / alpha : 0xFFFFFFFFu;
  u64* ub = u + (size_t)s * nitems * 2 * ne * N;
  const u64* es = ext + (size_t)s * ext_items * dstride * ne * N;
  const u64* obase = own.base ? own.base + s * own.os : nullptr;
  for (u32 b = 0; b < nitems; ++b) {
    const u64* e = es + ((size_t)b * dstride) * ne * N + (size_t)t * N + k;
    const u64* src = obase ? obase + b * own.ob : own.ptr[b];
    u64 x[BETA];
#pragma unroll
    for (int j = 0; j < BETA; ++j) x[j] = (u32)j == own_digit ? src[(size_t)t * N + k] : e[(size_t)j * ne * N];
    u64 rb, ra;
    ks_dot<BETA, LAZY>(x, kb, kbs, ka, kas, P, t > l, rb, ra);
    u64* o = ub + ((size_t)b * 2 * ne + t) * N + ko;
    o[0] = rb;
    o[(size_t)ne * N] = ra;
  }
}

template <int BETA>
__global__ void __launch_bounds__(BS) k_ks_inner_steps(const u64* __restrict__ ext, u32 ext_items, OwnMap own,
                                                       StepKeys keys, u64* __restrict__ u,
                                                       const PrimeConst* __restrict__ pc, u32 N, u32 logn, u32 l,
                                                       u32 nq, u32 np, u32 dstride, u32 nitems, u32 alpha,
                                                       u32 nsteps) {
  const u32 ne = l + 1 + np, nt = nq + np, nkb = N / BS;
  u32 s, tile;
  xcd_decode(blockIdx.x, nsteps, nkb * ne, s, tile);
  const u32 k = (tile % nkb) * BS + threadIdx.x, t = tile / nkb;
  const u32 pr = t <= l ? t : nq + (t - l - 1);
  const PrimeConst P = pc[pr];
  const u32 ko = galois_perm(k, keys.galois_inv[s], logn);    // output (and key) position
  if (P.q < kLazyKS)
    ks_inner_body<BETA, true>(ext, ext_items, own, keys.key[s], u, P, N, l, nt, ne, pr, dstride, nitems, alpha, s, k,
                              ko, t);
  else
    ks_inner_body<BETA, false>(ext, ext_items, own, keys.key[s], u, P, N, l, nt, ne, pr, dstride, nitems, alpha, s,
                               k, ko, t);
}

// grid: (N/BS, l+1, S B), item z = s B + b
__global__ void __launch_bounds__(BS) k_ks_final_steps(const u64* __restrict__ u, const u64* __restrict__ conv,
                                                       StepKeys keys, Items add0, OutMap om,
                                                       const PrimeConst* __restrict__ pc, const u64* __restrict__ md,
                                                       u32 N, u32 logn, u32 l, u32 np, u32 nq, u32 B) {
  const u32 k = blockIdx.x * BS + threadIdx.x;
  const u32 i = blockIdx.y, z = blockIdx.z, s = z / B, b = z % B;
  const u32 ne = l + 1 + np;
  const u64 q = pc[i].q;
  const u64* pinv = md + 2 * np + 2 * (size_t)np * nq;   // [nq][2]
  const u64 w = pinv[2 * i], wsh = pinv[2 * i + 1];
  const size_t ui = ((size_t)z * 2 * ne + i) * N + k;
  const size_t ci = ((size_t)z * 2 * (l + 1) + i) * N + k;
  u64 r0 = shoup(u[ui] + q - conv[ci], w, wsh, q);
  const u64 r1 = shoup(u[ui + (size_t)ne * N] + q - conv[ci + (size_t)(l + 1) * N], w, wsh, q);
  r0 = add_mod(r0, add0.p[b][(size_t)i * N + galois_perm(k, keys.galois[s], logn)], q);
  u64* out = om.base ? om.base + s * om.os + b * om.ob : om.ptr[z];
  out[(size_t)i * N + k] = r0;
  out[(size_t)(l + 1 + i) * N + k] = r1;
}

// 1-D grid over B x (N/BS, l+1, n2/JC) tiles (items of a tile share its
// plaintext words).  One thread: coefficient k of limb li of item b, giant
// sums jc JC .. jc JC + JC - 1; the baby-step values r_i are formed in
// registers from the key-switch buffers and consumed at once.
template <int JC, bool LAZY>
__device__ __forceinline__ void ks_final_mp_body(const u64* __restrict__ u, const u64* __restrict__ conv,
                                                 const StepKeys& keys, const Items& in, const u64* __restrict__ pts,
                                                 u64* __restrict__ sums, const PrimeConst& pk,
                                                 const u64* __restrict__ md, u32 N, u32 logn, u32 l, u32 np,
                                                 u32 nq, u32 n1, u32 n2, u32 b, u32 k, u32 li, u32 jc) {
  const u32 B = in.n, ne = l + 1 + np;
  const u64 q = pk.q;
  const u64* pinv = md + 2 * np + 2 * (size_t)np * nq;   // [nq][2]
  const u64 w = pinv[2 * li], wsh = pinv[2 * li + 1];
  const size_t csz = (size_t)2 * (l + 1) * N;
  const size_t comp = (size_t)n1 * n2 * (l + 1) * N;  // companions follow the m diagonals
  const u64* x = in.p[b];
  u64 r0 = x[(size_t)li * N + k], r1 = x[(size_t)(l + 1 + li) * N + k];
  u64 t0[JC], t1[JC];
#pragma unroll
  for (int jj = 0; jj < JC; ++jj) t0[jj] = t1[jj] = 0;
  for (u32 i = 0; i < n1; ++i) {
    if (i > 0) {
      const u32 z = (i - 1) * B + b;
      const size_t ui = ((size_t)z * 2 * ne + li) * N + k;
      const size_t ci = ((size_t)z * 2 * (l + 1) + li) * N + k;
      r0 = shoup(u[ui] + q - conv[ci], w, wsh, q);
      r1 = shoup(u[ui + (size_t)ne * N] + q - conv[ci + (size_t)(l + 1) * N], w, wsh, q);
      r0 = add_mod(r0, x[(size_t)li * N + galois_perm(k, keys.galois[i - 1], logn)], q);
    }
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) {
      const size_t o = ((size_t)(n1 * (jc * JC + jj) + i) * (l + 1) + li) * N + k;
      const u64 pt = pts[o], ps = pts[comp + o];
      t0[jj] = mp_add<LAZY>(t0[jj], r0, pt, ps, pk);
      t1[jj] = mp_add<LAZY>(t1[jj], r1, pt, ps, pk);
    }
  }
#pragma unroll
  for (int jj = 0; jj < JC; ++jj) {
    u64* o = sums + ((size_t)(jc * JC + jj) * B + b) * csz;
    o[(size_t)li * N + k] = mp_final<LAZY>(t0[jj], pk);
    o[(size_t)(l + 1 + li) * N + k] = mp_final<LAZY>(t1[jj], pk);
  }
}

template <int JC>
__global__ void __launch_bounds__(BS) k_ks_final_mp(const u64* __restrict__ u, const u64* __restrict__ conv,
                                                    StepKeys keys, Items in, const u64* __restrict__ pts,
                                                    u64* __restrict__ sums, const PrimeConst* __restrict__ pc,
                                                    const u64* __restrict__ md, u32 N, u32 logn, u32 l, u32 np, u32 nq,
                                                    u32 n1, u32 n2) {
  const u32 nkb = N / BS;
  u32 b, tile;
  xcd_decode(blockIdx.x, in.n, nkb * (l + 1) * (n2 / JC), b, tile);
  const u32 k = (tile % nkb) * BS + threadIdx.x;
  const u32 li = (tile / nkb) % (l + 1), jc = tile / (nkb * (l + 1));
  const PrimeConst pk = pc[li];
  if (pk.q < kLazyMP)
    ks_final_mp_body<JC, true>(u, conv, keys, in, pts, sums, pk, md, N, logn, l, np, nq, n1, n2, b, k, li, jc);
  else
    ks_final_mp_body<JC, false>(u, conv, keys, in, pts, sums, pk, md, N, logn, l, np, nq, n1, n2, b, k, li, jc);
}

// Lazy-ModDown inner sums over Q_l u P.  With u holding the extended
// key-switch inner products of baby steps i = 1 .. n1-1 (step s = i - 1):
//   r_0 = (P c0, P c1),  r_i = (P c0[perm_{g_i}] + u_b, u_a)  (P x is 0 on the P-limbs),
//   sqp[j][b] = sum_i pts[n1 j + i] (.) r_i,  limb t of ne = l+1+K.
// The extended rotations exist only in registers.  One thread: coefficient
// k of limb t of item b, giant sums jc JC .. jc JC + JC - 1.  u's Q-limbs are
// lazy (below 32q, or 4q for q >= 2^58); adding the lazy P c0 product (below
// 2q) stays below 2^64 and the plaintext product takes any 64-bit input.
template <int JC, bool LAZY>
__device__ __forceinline__ void ext_mp_body(const u64* __restrict__ u, const StepKeys& keys, const Items& in,
                                            const u64* __restrict__ pts, u64* __restrict__ sqp, const PrimeConst& pk,
                                            u64 pw, u64 pws, u32 N, u32 logn, u32 l, u32 ne, u32 n1, u32 n2, u32 b,
                                            u32 k, u32 t, u32 jc) {
  const u32 B = in.n;
  const bool qlimb = t <= l;
  const u64 q = pk.q;
  const size_t comp = (size_t)n1 * n2 * ne * N;   // companions follow the m diagonals
  const u64* x = in.p[b];
  u64 t0[JC], t1[JC];
#pragma unroll
  for (int jj = 0; jj < JC; ++jj) t0[jj] = t1[jj] = 0;
  if (qlimb) {
    const u64 r0 = shoup(x[(size_t)t * N + k], pw, pws, q), r1 = shoup(x[(size_t)(l + 1 + t) * N + k], pw, pws, q);
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) {
      const size_t o = ((size_t)n1 * (jc * JC + jj) * ne + t) * N + k;
      const u64 pt = pts[o], ps = pts[comp + o];
      t0[jj] = mp_add<LAZY>(t0[jj], r0, pt, ps, pk);
      t1[jj] = mp_add<LAZY>(t1[jj], r1, pt, ps, pk);
    }
  }
  for (u32 i = 1; i < n1; ++i) {
    const size_t ui = ((size_t)((i - 1) * B + b) * 2 * ne + t) * N + k;
    u64 r0 = u[ui];
    const u64 r1 = u[ui + (size_t)ne * N];
    if (qlimb) r0 += shoup_lazy(x[(size_t)t * N + galois_perm(k, keys.galois[i - 1], logn)], pw, pws, q);
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) {
      const size_t o = (((size_t)n1 * (jc * JC + jj) + i) * ne + t) * N + k;
      const u64 pt = pts[o], ps = pts[comp + o];
      t0[jj] = mp_add<LAZY>(t0[jj], r0, pt, ps, pk);
      t1[jj] = mp_add<LAZY>(t1[jj], r1, pt, ps, pk);
    }
  }
#pragma unroll
  for (int jj = 0; jj < JC; ++jj) {
    u64* o = sqp + ((size_t)(jc * JC + jj) * B + b) * 2 * ne * N;
    o[(size_t)t * N + k] = mp_final<LAZY>(t0[jj], pk);
    o[(size_t)(ne + t) * N + k] = mp_final<LAZY>(t1[jj], pk);
  }
}

// 1-D grid over B x (N/BS, ne, n2/JC) tiles: the items of a tile share its
// plaintext words (xcd_decode).
template <int JC>
__global__ void __launch_bounds__(BS) k_ext_mp(const u64* __restrict__ u, StepKeys keys, Items in,
                                               const u64* __restrict__ pts, u64* __restrict__ sqp,
                                               const PrimeConst* __restrict__ pc, const u64* __restrict__ md,
                                               u32 N, u32 logn, u32 l, u32 np, u32 nq, u32 n1, u32 n2) {
  const u32 nkb = N / BS, ne = l + 1 + np;
  u32 b, tile;
  xcd_decode(blockIdx.x, in.n, nkb * ne * (n2 / JC), b, tile);
  const u32 k = (tile % nkb) * BS + threadIdx.x;
  const u32 t = (tile / nkb) % ne, jc = tile / (nkb * ne);
  const u32 pr = t <= l ? t : nq + (t - l - 1);
  const PrimeConst pk = pc[pr];
  const u64* pmod = md + 2 * np + 2 * (size_t)np * nq + 2 * (size_t)nq;   // [nq][2] P mod q_i
  const u64 pw = t <= l ? pmod[2 * t] : 0, pws = t <= l ? pmod[2 * t + 1] : 0;
  if (pk.q < kLazyMP)
    ext_mp_body<JC, true>(u, keys, in, pts, sqp, pk, pw, pws, N, logn, l, ne, n1, n2, b, k, t, jc);
  else
    ext_mp_body<JC, false>(u, keys, in, pts, sqp, pk, pw, pws, N, logn, l, ne, n1, n2, b, k, t, jc);
}

// ModDown output of Z extended ciphertexts: out(z) = (y_Q - conv) P^{-1} over
// limbs i <= l (NTT domain), y = [Z][2][ne][N] (Q-limbs in [0, q)), conv =
// [Z][2][l+1][N]; out(z) at om (base + z ob, or ptr[z]); + bias on c0 when
// non-null.  grid: (N/BS, l+1, Z)
__global__ void __launch_bounds__(BS) k_moddown_final(const u64* __restrict__ y, const u64* __restrict__ conv,
                                                      OutMap om, const u64* __restrict__ bias,
                                                      const PrimeConst* __restrict__ pc, const u64* __restrict__ md,
                                                      u32 N, u32 l, u32 np, u32 nq) {
  const u32 k = blockIdx.x * BS + threadIdx.x;
  const u32 i = blockIdx.y, z = blockIdx.z;
  const u32 ne = l + 1 + np;
  const u64 q = pc[i].q;
  const u64* pinv = md + 2 * np + 2 * (size_t)np * nq;   // [nq][2]
  const u64 w = pinv[2 * i], wsh = pinv[2 * i + 1];
  const size_t yi = ((size_t)z * 2 * ne + i) * N + k;
  const size_t ci = ((size_t)z * 2 * (l + 1) + i) * N + k;
  u64* o = om.base ? om.base + z * om.ob : om.ptr[z];
  u64 r0 = shoup(y[yi] + q - conv[ci], w, wsh, q);
  if (bias) r0 = add_mod(r0, bias[(size_t)i * N + k], q);
  o[(size_t)i * N + k] = r0;
  o[(size_t)(l + 1 + i) * N + k] = shoup(y[yi + (size_t)ne * N] + q - conv[ci + (size_t)(l + 1) * N], w, wsh, q);
}

// grid: (N/BS, l+1, B).  One thread: coefficient k of limb i of item b, all
// J giant steps summed in registers (modular sums are exact, so the order of
// the terms does not change the result).
__global__ void __launch_bounds__(BS) k_ks_final_sum(const u64* __restrict__ u, const u64* __restrict__ conv,
                                                     StepKeys keys, const u64* __restrict__ sums,
                                                     const u64* __restrict__ bias, OutMap om,
                                                     const PrimeConst* __restrict__ pc, const u64* __restrict__ md,
                                                     u32 N, u32 logn, u32 l, u32 np, u32 nq, u32 B, u32 J) {
  const u32 k = blockIdx.x * BS + threadIdx.x;
  const u32 i = blockIdx.y, b = blockIdx.z;
  const u32 ne = l + 1 + np;
  const u64 q = pc[i].q;
  const u64* pinv = md + 2 * np + 2 * (size_t)np * nq;   // [nq][2]
  const u64 w = pinv[2 * i], wsh = pinv[2 * i + 1];
  const size_t csz = (size_t)2 * (l + 1) * N;
  const u64* s0 = sums + (size_t)b * csz;
  u64 r0 = s0[(size_t)i * N + k], r1 = s0[(size_t)(l + 1 + i) * N + k];
  for (u32 j = 1; j <= J; ++j) {
    const u32 z = (j - 1) * B + b;
    const size_t ui = ((size_t)z * 2 * ne + i) * N + k;
    const size_t ci = ((size_t)z * 2 * (l + 1) + i) * N + k;
    const u64* sj = sums + ((size_t)j * B + b) * csz;
    r0 = add_mod(r0, shoup(u[ui] + q - conv[ci], w, wsh, q), q);
    r0 = add_mod(r0, sj[(size_t)i * N + galois_perm(k, keys.galois[j - 1], logn)], q);
    r1 = add_mod(r1, shoup(u[ui + (size_t)ne * N] + q - conv[ci + (size_t)(l + 1) * N], w, wsh, q), q);
  }
  if (bias) r0 = add_mod(r0, bias[(size_t)i * N + k], q);
  u64* out = om.base ? om.base + b * om.ob : om.ptr[b];
  out[(size_t)i * N + k] = r0;
  out[(size_t)(l + 1 + i) * N + k] = r1;
}

// grid: (N/BS, 2, B); K = number of special primes
template <int K>
__global__ void __launch_bounds__(BS) k_moddown_conv(const u64* __restrict__ u, u64* __restrict__ conv,
                                                     const PrimeConst* __restrict__ pc,
                                                     const u64* __restrict__ md, u32 N, u32 l, u32 nq) {
  const u32 k = blockIdx.x * BS + threadIdx.x;
  const u32 p = blockIdx.y, b = blockIdx.z;
  const u32 ne = l + 1 + K;
  const u64* phatinv = md;                     // [K][2]
  const u64* phatmod = md + 2 * K;             // [K][nq][2]
  const u64* src = u + ((size_t)b * 2 + p) * ne * N;
  u64 v[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const u64 q = pc[nq + kk].q;
    v[kk] = shoup(src[(size_t)(l + 1 + kk) * N + k], phatinv[2 * kk], phatinv[2 * kk + 1], q);
  }
  u64* dst = conv + ((size_t)b * 2 + p) * (l + 1) * N;
  for (u32 i = 0; i <= l; ++i) {
    const PrimeConst P = pc[i];
    u64 s = 0;
    if (P.q < (1ull << 59)) {
#pragma unroll
      for (int kk = 0; kk < K; ++kk) s = conv_add<true>(s, v[kk], phatmod + 2 * ((size_t)kk * nq + i), P);
      s = conv_final<true>(s, P);
    } else {
#pragma unroll
      for (int kk = 0; kk < K; ++kk) s = conv_add<false>(s, v[kk], phatmod + 2 * ((size_t)kk * nq + i), P);
      s = conv_final<false>(s, P);
    }
    dst[(size_t)i * N + k] = s;
  }
}

// grid: (N/BS, l+1, B)
__global__ void __launch_bounds__(BS) k_ks_final(const u64* __restrict__ u, const u64* __restrict__ conv,
                                                 FinalArgs fa, const u64* __restrict__ bias,
                                                 const PrimeConst* __restrict__ pc, const u64* __restrict__ md,
                                                 u32 N, u32 logn, u32 l, u32 nq, u32 np, u32 galois) {
  const u32 k = blockIdx.x * BS + threadIdx.x;
  const u32 i = blockIdx.y, b = blockIdx.z;
  const u32 ne = l + 1 + np;
  const u64 q = pc[i].q;
  const u64* pinv = md + 2 * np + 2 * (size_t)np * nq;   // [nq][2]
  const u64 w = pinv[2 * i], wsh = pinv[2 * i + 1];
  const size_t ui = ((size_t)b * 2 * ne + i) * N + k;
  const size_t ci = ((size_t)b * 2 * (l + 1) + i) * N + k;
  u64 r0 = shoup(u[ui] + q - conv[ci], w, wsh, q);
  u64 r1 = shoup(u[ui + (size_t)ne * N] + q - conv[ci + (size_t)(l + 1) * N], w, wsh, q);
  const size_t o0 = (size_t)i * N + k, o1 = (size_t)(l + 1 + i) * N + k;
  if (fa.add0[b]) {
    const u32 ks = galois != 1 ? galois_perm(k, galois, logn) : k;
    r0 = add_mod(r0, fa.add0[b][(size_t)i * N + ks], q);
  }
  if (fa.add1[b]) r1 = add_mod(r1, fa.add1[b][o0], q);
  if (fa.acc[b]) {
    r0 = add_mod(r0, fa.acc[b][o0], q);
    r1 = add_mod(r1, fa.acc[b][o1], q);
  }
  if (bias) r0 = add_mod(r0, bias[o0], q);
  fa.out[b][o0] = r0;
  fa.out[b][o1] = r1;
}

// 1-D grid over B x (N/BS, l+1, n2/JC) tiles: the items of a tile share its
// plaintext words (xcd_decode).  One product per giant sum: s_j = pts[j] (.) in.
template <int JC>
__global__ void __launch_bounds__(BS) k_multplain(Items in, const u64* __restrict__ pts, u64* __restrict__ s,
                                                  const PrimeConst* __restrict__ pc, u32 N, u32 l, u32 n2, u32 pl) {
  const u32 nkb = N / BS;
  u32 b, tile;
  xcd_decode(blockIdx.x, in.n, nkb * (l + 1) * (n2 / JC), b, tile);
  const u32 k = (tile % nkb) * BS + threadIdx.x;
  const u32 li = (tile / nkb) % (l + 1), jc = tile / (nkb * (l + 1));
  const PrimeConst pk = pc[li];
  const size_t csz = (size_t)2 * (l + 1) * N, comp = (size_t)n2 * pl * N;
  const u64 r0 = in.p[b][(size_t)li * N + k], r1 = in.p[b][(size_t)(l + 1 + li) * N + k];
#pragma unroll
  for (int jj = 0; jj < JC; ++jj) {
    const size_t o = ((size_t)(jc * JC + jj) * pl + li) * N + k;
    const u64 pt = pts[o], ps = pts[comp + o];
    u64* out = s + ((size_t)(jc * JC + jj) * in.n + b) * csz;
    out[(size_t)li * N + k] = mp_final<false>(shoup_lazy4(r0, pt, ps, pk.q), pk);
    out[(size_t)(l + 1 + li) * N + k] = mp_final<false>(shoup_lazy4(r1, pt, ps, pk.q), pk);
  }
}

// Plaintext multiply-accumulate for R requests over T ciphertext terms each
// (the inner sums of a multi-input linear transform): term t of request r at
// x + (r T + t) csz; for output o = g n_out + j < NG n_out,
//   s(r, o) = sum_{t < T} pts[o][t] (.) term(r, t)   (both polynomials),
// written at s + (g R n_out + r n_out + j) csz (giant-major, the layout the
// step-batched giant key switch reads).  pts = [NG n_out][T][l+1][N] then
// companions.  Each thread keeps RC requests' sums, so a plaintext word is
// loaded once per RC requests.  1-D grid over n_o x (N/BS, l+1) tiles.
constexpr int RC = 8;
template <bool LAZY>
__device__ __forceinline__ void mp_acc_body(const u64* __restrict__ x, const u64* __restrict__ pts,
                                            u64* __restrict__ s, const PrimeConst& pk, u32 N, u32 l, u32 R, u32 T,
                                            u32 n_out, u32 n_o, u32 o, u32 k, u32 li) {
  const size_t csz = (size_t)2 * (l + 1) * N;
  const size_t comp = (size_t)n_o * T * (l + 1) * N;
  const u32 g = o / n_out, j = o % n_out;
  for (u32 r0 = 0; r0 < R; r0 += RC) {
    const u32 rn = min((u32)RC, R - r0);
    u64 a0[RC], a1[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) a0[r] = a1[r] = 0;
    for (u32 t = 0; t < T; ++t) {
      const size_t po = (((size_t)o * T + t) * (l + 1) + li) * N + k;
      const u64 pt = pts[po], ps = pts[comp + po];
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        if ((u32)r >= rn) break;
        const u64* xt = x + ((size_t)(r0 + r) * T + t) * csz;
        a0[r] = mp_add<LAZY>(a0[r], xt[(size_t)li * N + k], pt, ps, pk);
        a1[r] = mp_add<LAZY>(a1[r], xt[(size_t)(l + 1 + li) * N + k], pt, ps, pk);
      }
    }
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      if ((u32)r >= rn) break;
      u64* out = s + ((size_t)g * R * n_out + (size_t)(r0 + r) * n_out + j) * csz;
      out[(size_t)li * N + k] = mp_final<LAZY>(a0[r], pk);
      out[(size_t)(l + 1 + li) * N + k] = mp_final<LAZY>(a1[r], pk);
    }
  }
}

__global__ void __launch_bounds__(BS) k_mp_acc(const u64* __restrict__ x, const u64* __restrict__ pts,
                                               u64* __restrict__ s, const PrimeConst* __restrict__ pc, u32 N, u32 l,
                                               u32 R, u32 T, u32 n_out, u32 n_o) {
  const u32 nkb = N / BS;
  u32 o, tile;
  xcd_decode(blockIdx.x, n_o, nkb * (l + 1), o, tile);
  const u32 k = (tile % nkb) * BS + threadIdx.x, li = tile / nkb;
  const PrimeConst pk = pc[li];
  if (pk.q < kLazyMP) mp_acc_body<true>(x, pts, s, pk, N, l, R, T, n_out, n_o, o, k, li);
  else mp_acc_body<false>(x, pts, s, pk, N, l, R, T, n_out, n_o, o, k, li);
}

// grid: (N/BS, l+1, B)
__global__ void __launch_bounds__(BS) k_tensor(Items in, u64* __restrict__ d01, u64* __restrict__ d2,
                                               const PrimeConst* __restrict__ pc, u32 N, u32 l) {
  const u32 k = blockIdx.x * BS + threadIdx.x;
  const u32 i = blockIdx.y, b = blockIdx.z;
  const PrimeConst P = pc[i];
  const u64 c0 = in.p[b][(size_t)i * N + k], c1 = in.p[b][(size_t)(l + 1 + i) * N + k];
  const u64 c0m = shoup(c0, P.rmod, P.rmod_sh, P.q), c1m = shoup(c1, P.rmod, P.rmod_sh, P.q);
  const u64 x00 = redc(mul_wide(c0m, c0), P.q, P.qneg);
  const u64 x01 = redc(mul_wide(c0m, c1), P.q, P.qneg);
  const u64 x11 = redc(mul_wide(c1m, c1), P.q, P.qneg);
  u64* o = d01 + (size_t)b * 2 * (l + 1) * N;
  o[(size_t)i * N + k] = x00;
  o[(size_t)(l + 1 + i) * N + k] = add_mod(x01, x01, P.q);
  d2[((size_t)b * (l + 1) + i) * N + k] = x11;
}

// grid: (N/BS, l, 2B)
__global__ void __launch_bounds__(BS) k_rescale_reduce(const u64* __restrict__ last, u64* __restrict__ red,
                                                       const PrimeConst* __restrict__ pc, u32 N, u32 l) {
  const u32 k = blockIdx.x * BS + threadIdx.x;
  const u32 i = blockIdx.y, bp = blockIdx.z;
  red[((size_t)bp * l + i) * N + k] = reduce64(last[((size_t)bp * (l + 1) + l) * N + k], pc[i].q, pc[i].mu);
}

// grid: (N/BS, l, 2B)
__global__ void __launch_bounds__(BS) k_rescale_final(Items in, const u64* __restrict__ red, Items out,
                                                      const PrimeConst* __restrict__ pc,
                                                      const u64* __restrict__ rs, u32 N, u32 l, u32 nq) {
  const u32 k = blockIdx.x * BS + threadIdx.x;
  const u32 i = blockIdx.y, b = blockIdx.z >> 1, p = blockIdx.z & 1;
  const u64 q = pc[i].q;
  const u64* w = rs + ((size_t)l * nq + i) * 2;
  const u64 x = in.p[b][((size_t)p * (l + 1) + i) * N + k];
  const u64 y = red[(((size_t)b * 2 + p) * l + i) * N + k];
  out.p[b][((size_t)p * l + i) * N + k] = shoup(x + q - y, w[0], w[1], q);
}

// grid: (N/BS, 2(l+1), B)
__global__ void __launch_bounds__(BS) k_add(Items a, Items b_, Items out, const PrimeConst* __restrict__ pc, u32 N,
                                            u32 l) {
  const u32 k = blockIdx.x * BS + threadIdx.x;
  const u32 r = blockIdx.y, b = blockIdx.z;
  const u64 q = pc[r % (l + 1)].q;
  const size_t o = (size_t)r * N + k;
  out.p[b][o] = add_mod(a.p[b][o], b_.p[b][o], q);
}

// grid: (N/BS, l+1, B)
__global__ void __launch_bounds__(BS) k_add_plain(Items ct, const u64* __restrict__ poly,
                                                  const PrimeConst* __restrict__ pc, u32 N) {
  const u32 k = blockIdx.x * BS + threadIdx.x;
  const u32 i = blockIdx.y, b = blockIdx.z;
  const size_t o = (size_t)i * N + k;
  ct.p[b][o] = add_mod(ct.p[b][o], poly[o], pc[i].q);
}

// grid: (N/BS, nitems, npoly)
// comp = floor(w 2^64 / q) by restoring long division of w 2^64 (w < q < 2^61:
// the running remainder stays below 2q < 2^62).  grid (N/BS, level+1, m).
__global__ void __launch_bounds__(BS) k_shoup_companion(const u64* __restrict__ pts, u64* __restrict__ comp,
                                                        const PrimeConst* __restrict__ pc, u32 N, u32 nlimbs,
                                                        u32 l, u32 nq) {
  const u32 k = blockIdx.x * BS + threadIdx.x, r = blockIdx.y, i = blockIdx.z;
  const size_t o = ((size_t)i * nlimbs + r) * N + k;
  const u64 q = pc[r <= l ? r : nq + (r - l - 1)].q;
  u64 rem = pts[o], quo = 0;
  for (int bit = 63; bit >= 0; --bit) {
    rem <<= 1;
    quo <<= 1;
    if (rem >= q) {
      rem -= q;
      quo |= 1;
    }
  }
  comp[o] = quo;
}


}  // namespace

int launch_copy_polys(he_ctx* c, const PolyBatch& pb) {
  if (!pb.nitems || !pb.npoly) return HE_OK;
  u32 nv = 0;
  for (u32 r = 0; r < pb.npoly; ++r) nv += pb.prime[r] != 0xFF;
  TraceScope ts(c, TK_COPY, 2.0 * nv * pb.nitems * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_copy_polys, dim3(c->N / BS / 4, pb.nitems, pb.npoly), dim3(BS), c->stream, pb, c->N);
  return ok();
}

int launch_modup_conv(he_ctx* c, u32 l, u32 nitems, const u64* coef, u64* ext) {
  const u32 beta = digits_at(c, l), ne = l + 1 + c->np;
  TraceScope ts(c, TK_MODUP_CONV, (double)nitems * ((l + 1) + (beta * ne - (l + 1))) * (8.0 * (double)c->N));
  const dim3 grid(c->N / BS, digits_at(c, l), nitems);
#define HE_LAUNCH_UP(A)                                                                                           \
  HE_LAUNCH(ts, (k_modup_conv<A>), grid, dim3(BS), c->stream, coef, ext, c->d_pc, c->d_modup_hatinv,               \
            c->d_modup_hatmod, c->N, l, c->nq, c->np, c->dnum)
  switch (c->alpha) {
    case 1: HE_LAUNCH_UP(1); break;
    case 2: HE_LAUNCH_UP(2); break;
    case 3: HE_LAUNCH_UP(3); break;
    case 4: HE_LAUNCH_UP(4); break;
    case 5: HE_LAUNCH_UP(5); break;
    case 6: HE_LAUNCH_UP(6); break;
    case 7: HE_LAUNCH_UP(7); break;
    case 8: HE_LAUNCH_UP(8); break;
    default: return HE_EPARAM;
  }
#undef HE_LAUNCH_UP
  return ok();
}

int launch_ks_final_sum(he_ctx* c, u32 l, u32 B, u32 S, const u64* u, const u64* conv, const StepKeys& keys,
                        const u64* sums, const u64* bias, const OutMap& om) {
  // per item: s_0 (2 polys), per step u and conv (2 + 2) and s_j.c0, 2 polys written
  TraceScope ts(c, TK_KS_FINAL_SUM,
                ((double)B * (4.0 + 5.0 * S) * (l + 1) + (bias ? l + 1 : 0)) * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_ks_final_sum, dim3(c->N / BS, l + 1, B), dim3(BS), c->stream, u, conv, keys, sums, bias, om,
                     c->d_pc, c->d_moddown, c->N, c->log_n, l, c->np, c->nq, B, S);
  return ok();
}

int launch_ks_inner_steps(he_ctx* c, u32 l, u32 B, u32 S, const u64* ext, u32 ext_items, const OwnMap& own,
                          const StepKeys& keys, u64* u) {
  const u32 beta = digits_at(c, l), ne = l + 1 + c->np;
  // digits: once per item when the steps share them (hoisted), once per (step, item) otherwise;
  // keys: value and Shoup companion per word
  const double digits = (double)(ext_items ? S : 1) * B * beta * ne;
  TraceScope ts(c, TK_KS_INNER_STEPS, (digits + (double)S * (4.0 * beta * ne + 2.0 * B * ne)) * (8.0 * (double)c->N));
  dim3 grid(S * (c->N / BS) * ne);
#define HE_LAUNCH_KS(BT)                                                                                          \
  HE_LAUNCH(ts, (k_ks_inner_steps<BT>), grid, dim3(BS), c->stream, ext, ext_items, own, keys, u, c->d_pc, c->N,     \
            c->log_n, l, c->nq, c->np, c->dnum, B, c->alpha, S)
  switch (beta) {
    case 1: HE_LAUNCH_KS(1); break;
    case 2: HE_LAUNCH_KS(2); break;
    case 3: HE_LAUNCH_KS(3); break;
    case 4: HE_LAUNCH_KS(4); break;
    case 5: HE_LAUNCH_KS(5); break;
    case 6: HE_LAUNCH_KS(6); break;
    case 7: HE_LAUNCH_KS(7); break;
    case 8: HE_LAUNCH_KS(8); break;
    default: return HE_EPARAM;
  }
#undef HE_LAUNCH_KS
  return ok();
}

int launch_ks_final_steps(he_ctx* c, u32 l, u32 B, u32 S, const u64* u, const u64* conv, const StepKeys& keys,
                          const Items& add0, const OutMap& om) {
  // per item: u and conv (2 polys each) and add0.c0 read, 2 polys written
  TraceScope ts(c, TK_KS_FINAL_STEPS, (double)S * B * 7.0 * (l + 1) * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_ks_final_steps, dim3(c->N / BS, l + 1, S * B), dim3(BS), c->stream, u, conv, keys, add0, om,
                     c->d_pc, c->d_moddown, c->N, c->log_n, l, c->np, c->nq, B);
  return ok();
}

int launch_ks_final_multplain(he_ctx* c, u32 l, u32 B, u32 n1, u32 n2, const u64* u, const u64* conv,
                              const StepKeys& keys, const Items& in, const u64* pts, u64* s) {
  const u32 jc = n2 >= 8 ? 8 : (n2 >= 4 ? 4 : (n2 >= 2 ? 2 : 1));
  if (n2 % jc) return HE_EINVAL;
  // per item: the input ciphertext, u and conv of every baby step (2 + 2 polys)
  // and its rotated c0 source limb, the n2 sums written; plaintexts once
  TraceScope ts(c, TK_KS_FINAL_MP,
                ((double)B * (2.0 + 5.0 * (n1 - 1) + 2.0 * n2) * (l + 1) + 2.0 * n1 * n2 * (l + 1)) *
                    (8.0 * (double)c->N));
  dim3 grid(B * (n2 / jc) * (c->N / BS) * (l + 1));
#define HE_LAUNCH_MP(J)                                                                                           \
  HE_LAUNCH(ts, (k_ks_final_mp<J>), grid, dim3(BS), c->stream, u, conv, keys, in, pts, s, c->d_pc,           \
                     c->d_moddown, c->N, c->log_n, l, c->np, c->nq, n1, n2)
  switch (jc) {
    case 8: HE_LAUNCH_MP(8); break;
    case 4: HE_LAUNCH_MP(4); break;
    case 2: HE_LAUNCH_MP(2); break;
    default: HE_LAUNCH_MP(1); break;
  }
#undef HE_LAUNCH_MP
  return ok();
}

int launch_moddown_conv(he_ctx* c, u32 l, u32 nitems, const u64* u, u64* conv) {
  TraceScope ts(c, TK_MODDOWN_CONV, (double)nitems * (2.0 * c->np + 2.0 * (l + 1)) * (8.0 * (double)c->N));
  const dim3 grid(c->N / BS, 2, nitems);
#define HE_LAUNCH_DN(K) \
  HE_LAUNCH(ts, (k_moddown_conv<K>), grid, dim3(BS), c->stream, u, conv, c->d_pc, c->d_moddown, c->N, l, c->nq)
  switch (c->np) {
    case 1: HE_LAUNCH_DN(1); break;
    case 2: HE_LAUNCH_DN(2); break;
    case 3: HE_LAUNCH_DN(3); break;
    case 4: HE_LAUNCH_DN(4); break;
    case 5: HE_LAUNCH_DN(5); break;
    case 6: HE_LAUNCH_DN(6); break;
    case 7: HE_LAUNCH_DN(7); break;
    case 8: HE_LAUNCH_DN(8); break;
    default: return HE_EPARAM;
  }
#undef HE_LAUNCH_DN
  return ok();
}

int launch_ks_final(he_ctx* c, u32 l, u32 nitems, const u64* u, const u64* conv, u32 galois, const FinalArgs& fa,
                    const u64* bias) {
  double per = 6.0 * (l + 1);                      // u and conv (2 polys each) read, 2 polys written
  if (fa.add0[0]) per += l + 1;
  if (fa.add1[0]) per += l + 1;
  if (fa.acc[0]) per += 2.0 * (l + 1);
  TraceScope ts(c, TK_KS_FINAL, ((double)nitems * per + (bias ? l + 1 : 0)) * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_ks_final, dim3(c->N / BS, l + 1, nitems), dim3(BS), c->stream, u, conv, fa, bias, c->d_pc,
                     c->d_moddown, c->N, c->log_n, l, c->nq, c->np, galois);
  return ok();
}

int launch_multplain(he_ctx* c, u32 l, u32 n2, const Items& in, const u64* pts, u32 pl, u64* s) {
  TraceScope ts(c, TK_MULTPLAIN, ((double)in.n * (1 + n2) * 2.0 * (l + 1) + 2.0 * n2 * (l + 1)) * (8.0 * (double)c->N));
  const u32 jc = n2 >= 8 ? 8 : (n2 >= 4 ? 4 : (n2 >= 2 ? 2 : 1));
  if (n2 % jc || pl < l + 1) return HE_EINVAL;
  dim3 grid(in.n * (n2 / jc) * (c->N / BS) * (l + 1));
#define HE_LAUNCH_M1(J) \
  HE_LAUNCH(ts, (k_multplain<J>), grid, dim3(BS), c->stream, in, pts, s, c->d_pc, c->N, l, n2, pl)
  switch (jc) {
    case 8: HE_LAUNCH_M1(8); break;
    case 4: HE_LAUNCH_M1(4); break;
    case 2: HE_LAUNCH_M1(2); break;
    default: HE_LAUNCH_M1(1); break;
  }
#undef HE_LAUNCH_M1
  return ok();
}

int launch_ext_multplain(he_ctx* c, u32 l, u32 B, u32 n1, u32 n2, const u64* u, const StepKeys& keys,
                         const Items& in, const u64* pts, u64* sqp) {
  const u32 jc = n2 >= 8 ? 8 : (n2 >= 4 ? 4 : (n2 >= 2 ? 2 : 1));
  if (n2 % jc) return HE_EINVAL;
  const double ne = l + 1 + c->np;
  // per item: c0 and c1 (plus c0 again, permuted, per baby step), u of every
  // baby step (2 polys over Q_l u P), the n2 sums written over Q_l u P;
  // plaintexts (value + companion) once
  TraceScope ts(c, TK_EXT_MP,
                ((double)B * (2.0 * (l + 1) + (n1 - 1) * (2.0 * ne + (l + 1)) + 2.0 * n2 * ne) + 2.0 * n1 * n2 * ne) *
                    (8.0 * (double)c->N));
  dim3 grid(B * (n2 / jc) * (c->N / BS) * (u32)ne);
#define HE_LAUNCH_XM(J)                                                                                           \
  HE_LAUNCH(ts, (k_ext_mp<J>), grid, dim3(BS), c->stream, u, keys, in, pts, sqp, c->d_pc, c->d_moddown, c->N,  \
            c->log_n, l, c->np, c->nq, n1, n2)
  switch (jc) {
    case 8: HE_LAUNCH_XM(8); break;
    case 4: HE_LAUNCH_XM(4); break;
    case 2: HE_LAUNCH_XM(2); break;
    default: HE_LAUNCH_XM(1); break;
  }
#undef HE_LAUNCH_XM
  return ok();
}

int launch_moddown_final(he_ctx* c, u32 l, u32 Z, const u64* y, const u64* conv, const OutMap& om,
                         const u64* bias) {
  if (!om.base && Z > HE_MAXB) return HE_EINVAL;
  TraceScope ts(c, TK_MODDOWN_FINAL, ((double)Z * 6.0 + (bias ? 1.0 : 0.0)) * (l + 1) * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_moddown_final, dim3(c->N / BS, l + 1, Z), dim3(BS), c->stream, y, conv, om, bias, c->d_pc,
            c->d_moddown, c->N, l, c->np, c->nq);
  return ok();
}

int launch_mp_acc(he_ctx* c, u32 l, u32 R, u32 T, u32 n_out, u32 NG, const u64* x, const u64* pts, u64* s) {
  if (!R || !T || T > 64 || !n_out || !NG) return HE_EINVAL;
  const u32 n_o = NG * n_out;
  // every term of every request once, plaintexts (value + companion) once, the sums
  TraceScope ts(c, TK_MP_ACC,
                ((double)R * T * 2.0 + (double)n_o * T * 2.0 + (double)R * n_o * 2.0) * (l + 1) * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_mp_acc, dim3(n_o * (c->N / BS) * (l + 1)), dim3(BS), c->stream, x, pts, s, c->d_pc, c->N, l, R, T,
            n_out, n_o);
  return ok();
}

int launch_tensor(he_ctx* c, u32 l, const Items& in, u64* d01, u64* d2) {
  TraceScope ts(c, TK_TENSOR, (double)in.n * 5.0 * (l + 1) * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_tensor, dim3(c->N / BS, l + 1, in.n), dim3(BS), c->stream, in, d01, d2, c->d_pc, c->N, l);
  return ok();
}

int launch_rescale_reduce(he_ctx* c, u32 l, u32 nitems, const u64* last, u64* red) {
  TraceScope ts(c, TK_RESCALE_REDUCE, (double)nitems * (2.0 + 2.0 * l) * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_rescale_reduce, dim3(c->N / BS, l, 2 * nitems), dim3(BS), c->stream, last, red, c->d_pc, c->N, l);
  return ok();
}

int launch_rescale_final(he_ctx* c, u32 l, const Items& in, const u64* red, const Items& out) {
  TraceScope ts(c, TK_RESCALE_FINAL, (double)in.n * 6.0 * l * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_rescale_final, dim3(c->N / BS, l, 2 * in.n), dim3(BS), c->stream, in, red, out, c->d_pc,
                     c->d_rescale, c->N, l, c->nq);
  return ok();
}

int launch_add(he_ctx* c, u32 l, const Items& a, const Items& b, const Items& out) {
  TraceScope ts(c, TK_ADD, (double)a.n * 6.0 * (l + 1) * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_add, dim3(c->N / BS, 2 * (l + 1), a.n), dim3(BS), c->stream, a, b, out, c->d_pc, c->N, l);
  return ok();
}

int launch_add_plain(he_ctx* c, u32 l, const Items& ct, const u64* poly) {
  TraceScope ts(c, TK_ADD_PLAIN, ((double)ct.n * 2.0 + 1.0) * (l + 1) * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_add_plain, dim3(c->N / BS, l + 1, ct.n), dim3(BS), c->stream, ct, poly, c->d_pc, c->N);
  return ok();
}

int launch_shoup_companion(he_ctx* c, u32 m, u32 nlimbs, u32 l, const u64* pts, u64* comp) {
  TraceScope ts(c, TK_SHOUP_COMPANION, 2.0 * m * nlimbs * (8.0 * (double)c->N));
  HE_LAUNCH(ts, k_shoup_companion, dim3(c->N / BS, nlimbs, m), dim3(BS), c->stream, pts, comp, c->d_pc, c->N, nlimbs,
            l, c->nq);
  return ok();
}

