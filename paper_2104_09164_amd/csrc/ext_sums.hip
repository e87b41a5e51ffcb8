// Fused lazy-ModDown inner sums (the baby steps' key inner products and the
// MultPlain inner sums over Q_l u P in one pass; also the plain sums of the
// hoisted rotate-and-sum groups), in three forms: every request's sums in
// registers of one thread (k_ks_ext_fused), a single request with
// values-only key and plaintext streams (k_ks_ext_one), or the key and
// plaintext words of a tile shared through LDS by the threads of several
// requests (k_ks_ext_lds, ext_sums_lds.hip).  All compute the same words.
#include "rns_kernels.hpp"
#include "modarith.hpp"
#include "rns_device.hpp"

namespace {

// Fused baby steps of the lazy-ModDown form: the key inner product of every
// baby step and the inner sums over Q_l u P in one pass, so the per-step
// products never reach memory.  Output position x of step i needs the digits
// and c0 at y = perm_{g_i}(x) (the automorphism, gathered: an aligned block
// of 256 positions maps onto another aligned block, and the 64 lanes of a
// wave touch 8 whole 64-byte lines) and the key and plaintext words at x:
//   u_i(x) = sum_j d_j(y) ksk_{i,j}(x),   r_i(x) = (P c0(y) + u_b, u_a),
//   sqp[j][b](x) = sum_i pts[n1 j + i](x) r_i(x),   r_0 = (P c0, P c1).
// The arithmetic and its order are those of k_ks_inner_steps followed by
// k_ext_mp (same lazy bounds), so the results are the same words.
// One thread: position x of limb t for G items (keys and plaintext words
// loaded once per step for the G items), all JC = n2 giant sums.
// 1-D grid over item groups x (N/BS, ne) tiles: the groups of a tile run
// back to back on one XCD and share its key and plaintext words in L2.
template <int BETA, int JC, int G, bool LKS, bool LMP>
__device__ __forceinline__ void ks_ext_fused_body(const u64* __restrict__ ext, const OwnMap& own,
                                                  const StepKeys& keys, const Items& in, const u64* __restrict__ pts,
                                                  u64* __restrict__ sqp, const PrimeConst& P, u64 pw, u64 pws, u32 N,
                                                  u32 logn, u32 l, u32 nt, u32 ne, u32 pr, u32 dstride, u32 alpha,
                                                  u32 n1, u32 b0, u32 gn, u32 x, u32 t) {
  const u32 B = in.n;
  const bool qlimb = t <= l;
  const u64 q = P.q;
  const size_t comp = (size_t)n1 * JC * ne * N;    // plaintext companions follow the m = n1 JC diagonals
  const size_t kw = (size_t)dstride * 2 * nt * N;  // key companions follow the key words
  const u32 own_digit = qlimb ? t / alpha : 0xFFFFFFFFu;
  u64 a0[G][JC], a1[G][JC];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) a0[g][jj] = a1[g][jj] = 0;
  if (qlimb) {
    u64 pt[JC], ps[JC];
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) {
      const size_t o = ((size_t)n1 * jj * ne + t) * N + x;
      pt[jj] = pts ? pts[o] : 1;                   // no plaintexts: a plain sum (x 1, companion mu)
      ps[jj] = pts ? pts[comp + o] : P.mu;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if ((u32)g >= gn) break;
      const u64* c = in.p[b0 + g];
      const u64 r0 = shoup(c[(size_t)t * N + x], pw, pws, q), r1 = shoup(c[(size_t)(l + 1 + t) * N + x], pw, pws, q);
#pragma unroll
      for (int jj = 0; jj < JC; ++jj) {
        a0[g][jj] = mp_add<LMP>(a0[g][jj], r0, pt[jj], ps[jj], P);
        a1[g][jj] = mp_add<LMP>(a1[g][jj], r1, pt[jj], ps[jj], P);
      }
    }
  }
  for (u32 i = 1; i < n1; ++i) {
    const u32 y = galois_perm(x, keys.galois[i - 1], logn);
    const u64* key = keys.key[i - 1];
    u64 kb[BETA], kbs[BETA], ka[BETA], kas[BETA];
#pragma unroll
    for (int j = 0; j < BETA; ++j) {
      const size_t ob = (((size_t)j * 2 + 0) * nt + pr) * N + x, oa = (((size_t)j * 2 + 1) * nt + pr) * N + x;
      kb[j] = key[ob];
      kbs[j] = key[kw + ob];
      ka[j] = key[oa];
      kas[j] = key[kw + oa];
    }
    u64 pt[JC], ps[JC];
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) {
      const size_t o = (((size_t)n1 * jj + i) * ne + t) * N + x;
      pt[jj] = pts ? pts[o] : 1;
      ps[jj] = pts ? pts[comp + o] : P.mu;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if ((u32)g >= gn) break;
      const u32 b = b0 + g;
      const u64* e = ext + ((size_t)b * dstride * ne + t) * N + y;
      const u64* src = own.ptr[b];
      u64 d[BETA];
#pragma unroll
      for (int j = 0; j < BETA; ++j) d[j] = (u32)j == own_digit ? src[(size_t)t * N + y] : e[(size_t)j * ne * N];
      u64 r0, r1;
      ks_dot<BETA, LKS>(d, kb, kbs, ka, kas, P, !qlimb, r0, r1);
      if (qlimb) r0 += shoup_lazy(in.p[b][(size_t)t * N + y], pw, pws, q);
#pragma unroll
      for (int jj = 0; jj < JC; ++jj) {
        a0[g][jj] = mp_add<LMP>(a0[g][jj], r0, pt[jj], ps[jj], P);
        a1[g][jj] = mp_add<LMP>(a1[g][jj], r1, pt[jj], ps[jj], P);
      }
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if ((u32)g >= gn) break;
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) {
      u64* o = sqp + ((size_t)jj * B + b0 + g) * 2 * ne * N;
      o[(size_t)t * N + x] = mp_final<LMP>(a0[g][jj], P);
      o[(size_t)(ne + t) * N + x] = mp_final<LMP>(a1[g][jj], P);
    }
  }
}

// W > 0: compiled for W waves per SIMD (the register budget that allows);
// W = 0: the compiler's own allocation.
template <int BETA, int JC, int G, int W>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(W > 0 ? W : 1, W > 0 ? W : 8)))
k_ks_ext_fused(const u64* __restrict__ ext, OwnMap own, StepKeys keys,
                                                     Items in, const u64* __restrict__ pts, u64* __restrict__ sqp,
                                                     const PrimeConst* __restrict__ pc, const u64* __restrict__ md,
                                                     u32 N, u32 logn, u32 l, u32 nq, u32 np, u32 dstride, u32 alpha,
                                                     u32 n1) {
  const u32 nkb = N / BS, ne = l + 1 + np, nt = nq + np;
  const u32 ngroups = (in.n + G - 1) / G;
  u32 grp, tile;
  xcd_decode(blockIdx.x, ngroups, nkb * ne, grp, tile);
  const u32 x = (tile % nkb) * BS + threadIdx.x, t = tile / nkb;
  const u32 pr = t <= l ? t : nq + (t - l - 1);
  const PrimeConst P = pc[pr];
  const u64* pmod = md + 2 * np + 2 * (size_t)np * nq + 2 * (size_t)nq;   // [nq][2] P mod q_i
  const u64 pw = t <= l ? pmod[2 * t] : 0, pws = t <= l ? pmod[2 * t + 1] : 0;
  const u32 b0 = grp * G, gn = min((u32)G, in.n - b0);
  const bool lks = P.q < kLazyKS, lmp = P.q < kLazyMP;
  if (lks && lmp)
    ks_ext_fused_body<BETA, JC, G, true, true>(ext, own, keys, in, pts, sqp, P, pw, pws, N, logn, l, nt, ne, pr,
                                               dstride, alpha, n1, b0, gn, x, t);
  else if (lks)
    ks_ext_fused_body<BETA, JC, G, true, false>(ext, own, keys, in, pts, sqp, P, pw, pws, N, logn, l, nt, ne, pr,
                                                dstride, alpha, n1, b0, gn, x, t);
  else
    ks_ext_fused_body<BETA, JC, G, false, false>(ext, own, keys, in, pts, sqp, P, pw, pws, N, logn, l, nt, ne, pr,
                                                 dstride, alpha, n1, b0, gn, x, t);
}


// Small batches (below ks_fuse_min_batch): the same sums with one request and
// position per thread, so the register budget allows a high occupancy.  A
// small batch is bound by the key and plaintext streams (read once per
// request from HBM, the other requests of a tile finding them in L2), so on
// the primes below 2^50 (COL) they are read as
// values only, without their Shoup companions (half the bytes), and both the
// key sums and the inner sums are exact 28-bit column sums: digit d and key
// word k (both below q < 2^50) split into 28-bit columns, four multiply-adds
// per product into K0 < 8 2^56, K1 < 8 2^51, K2 < 8 2^44 over at most 8
// digits, reduced lazily (col_lazy, below 11 q; with the lift of c0, below
// 2q, r < 13 q < 2^54) and multiplied into the inner column sums as in the
// LDS-shared form.  Other primes take the register form's Shoup products.
// The words written are in [0, q): the same words as every other form.
template <int BETA, int JC, bool COL, bool LKS, bool LMP>
__device__ __forceinline__ void ks_ext_one_body(const u64* __restrict__ ext, const OwnMap& own, const StepKeys& keys,
                                                const Items& in, const u64* __restrict__ pts, u64* __restrict__ sqp,
                                                const PrimeConst& P, u64 pw, u64 pws, u32 N, u32 logn, u32 l, u32 nt,
                                                u32 ne, u32 pr, u32 dstride, u32 alpha, u32 n1, u32 b, u32 x, u32 t) {
  const u32 B = in.n;
  const bool qlimb = t <= l;
  const u64 q = P.q;
  const size_t comp = (size_t)n1 * JC * ne * N;    // plaintext companions follow the m = n1 JC diagonals
  const size_t kw = (size_t)dstride * 2 * nt * N;  // key companions follow the key words
  const u32 own_digit = qlimb ? t / alpha : 0xFFFFFFFFu;
  u64 a0[JC], a1[JC];                              // Shoup inner sums
  u64 w0[COL ? JC : 1][3], w1[COL ? JC : 1][3];    // column inner sums
#pragma unroll
  for (int jj = 0; jj < JC; ++jj) a0[jj] = a1[jj] = 0;
#pragma unroll
  for (int jj = 0; jj < (COL ? JC : 1); ++jj)
    w0[jj][0] = w0[jj][1] = w0[jj][2] = w1[jj][0] = w1[jj][1] = w1[jj][2] = 0;
  // plaintext word of giant sum jj at step i (value; companion unless COL)
  auto pt_of = [&](int jj, u32 i, u64& v, u64& c) {
    const size_t o = (((size_t)n1 * jj + i) * ne + t) * N + x;
    v = pts ? pts[o] : 1;                          // no plaintexts: a plain sum (x 1, companion mu)
    c = COL ? 0 : (pts ? pts[comp + o] : P.mu);
  };
  auto inner = [&](int jj, u64 r0, u64 r1, u64 pt, u64 ps) {
    if (COL) {
      col_mad(w0[jj], r0, pt & kLow28, pt >> 28);
      col_mad(w1[jj], r1, pt & kLow28, pt >> 28);
    } else {
      a0[jj] = mp_add<LMP>(a0[jj], r0, pt, ps, P);
      a1[jj] = mp_add<LMP>(a1[jj], r1, pt, ps, P);
    }
  };
  if (qlimb) {
    const u64* c = in.p[b];
    const u64 r0 = shoup(c[(size_t)t * N + x], pw, pws, q), r1 = shoup(c[(size_t)(l + 1 + t) * N + x], pw, pws, q);
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) {
      u64 pt, ps;
      pt_of(jj, 0, pt, ps);
      inner(jj, r0, r1, pt, ps);
    }
  }
  const u64* e = ext + ((size_t)b * dstride * ne + t) * N;
  const u64* src = own.ptr[b] + (size_t)t * N;
  for (u32 i = 1; i < n1; ++i) {
    const u32 y = galois_perm(x, keys.galois[i - 1], logn);
    const u64* key = keys.key[i - 1];
    u64 d[BETA];
#pragma unroll
    for (int j = 0; j < BETA; ++j) d[j] = (u32)j == own_digit ? src[y] : e[(size_t)j * ne * N + y];
    u64 r0, r1;
    if (COL) {
      u64 kb[3] = {0, 0, 0}, ka[3] = {0, 0, 0};
#pragma unroll
      for (int j = 0; j < BETA; ++j) {
        const u64 vb = key[(((size_t)j * 2 + 0) * nt + pr) * N + x], va = key[(((size_t)j * 2 + 1) * nt + pr) * N + x];
        col_mad(kb, d[j], vb & kLow28, vb >> 28);
        col_mad(ka, d[j], va & kLow28, va >> 28);
      }
      r0 = col_lazy(kb, P);
      r1 = col_lazy(ka, P);
    } else {
      u64 kb[BETA], kbs[BETA], ka[BETA], kas[BETA];
#pragma unroll
      for (int j = 0; j < BETA; ++j) {
        const size_t ob = (((size_t)j * 2 + 0) * nt + pr) * N + x, oa = (((size_t)j * 2 + 1) * nt + pr) * N + x;
        kb[j] = key[ob];
        kbs[j] = key[kw + ob];
        ka[j] = key[oa];
        kas[j] = key[kw + oa];
      }
      ks_dot<BETA, LKS>(d, kb, kbs, ka, kas, P, !qlimb, r0, r1);
    }
    if (qlimb) r0 += shoup_lazy(in.p[b][(size_t)t * N + y], pw, pws, q);
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) {
      u64 pt, ps;
      pt_of(jj, i, pt, ps);
      inner(jj, r0, r1, pt, ps);
    }
  }
#pragma unroll
  for (int jj = 0; jj < JC; ++jj) {
    u64* o = sqp + ((size_t)jj * B + b) * 2 * ne * N;
    o[(size_t)t * N + x] = COL ? col_final(w0[jj], P) : mp_final<LMP>(a0[jj], P);
    o[(size_t)(ne + t) * N + x] = COL ? col_final(w1[jj], P) : mp_final<LMP>(a1[jj], P);
  }
}

// 1-D grid of B requests x (N / BS, ne) tiles (xcd_decode: the requests of a
// tile run back to back on one XCD and find its key and plaintext words in
// L2).
template <int BETA, int JC>
__global__ void __launch_bounds__(BS) k_ks_ext_one(const u64* __restrict__ ext, OwnMap own, StepKeys keys, Items in,
                                                   const u64* __restrict__ pts, u64* __restrict__ sqp,
                                                   const PrimeConst* __restrict__ pc, const u64* __restrict__ md,
                                                   u32 N, u32 logn, u32 l, u32 nq, u32 np, u32 dstride, u32 alpha,
                                                   u32 n1) {
  const u32 nkb = N / BS, ne = l + 1 + np, nt = nq + np;
  u32 b, tile;
  xcd_decode(blockIdx.x, in.n, nkb * ne, b, tile);
  const u32 x = (tile % nkb) * BS + threadIdx.x, t = tile / nkb;
  const u32 pr = t <= l ? t : nq + (t - l - 1);
  const PrimeConst P = pc[pr];
  const u64* pmod = md + 2 * np + 2 * (size_t)np * nq + 2 * (size_t)nq;   // [nq][2] P mod q_i
  const u64 pw = t <= l ? pmod[2 * t] : 0, pws = t <= l ? pmod[2 * t + 1] : 0;
#define HE_ONE_BODY(C, K, M)                                                                                    \
  ks_ext_one_body<BETA, JC, C, K, M>(ext, own, keys, in, pts, sqp, P, pw, pws, N, logn, l, nt, ne, pr, dstride, \
                                     alpha, n1, b, x, t)
  if (P.q < kWideQ)
    HE_ONE_BODY(true, true, true);
  else if (P.q < kLazyMP)
    HE_ONE_BODY(false, true, true);
  else if (P.q < kLazyKS)
    HE_ONE_BODY(false, true, false);
  else
    HE_ONE_BODY(false, false, false);
#undef HE_ONE_BODY
}

}  // namespace

int launch_ks_ext_fused(he_ctx* c, u32 l, u32 B, u32 n1, u32 n2, const u64* ext, const OwnMap& own,
                        const StepKeys& keys, const Items& in, const u64* pts, u64* sqp, u64* lift) {
  const u32 beta = digits_at(c, l), ne = l + 1 + c->np, S = n1 - 1;
  if (n1 < 2 || S > HE_MAX_STEPS || !(n2 == 1 || n2 == 2 || n2 == 4 || n2 == 8) || B != in.n || (!pts && n2 != 1))
    return HE_EINVAL;
  // keys once per step, each item's digits and input once, plaintexts once, the sums written
  TraceScope ts(c, TK_KS_EXT_FUSED,
                ((double)S * 4.0 * beta * ne + (double)B * (beta * ne + 2.0 * (l + 1) + 2.0 * n2 * ne) +
                 (pts ? 2.0 * n1 * n2 * ne : 0.0)) * (8.0 * (double)c->N));
  // the LDS-shared form with W requests per workgroup, W halved (down to 4)
  // while the batch does not fill it (idle waves still share the tile
  // loads); smaller batches the small-batch kernel or the register form
  u32 W = (u32)c->ks_fuse_lds;
  while (W > 4 && B < W) W /= 2;
  if (W && B >= (u32)c->ks_fuse_min_batch)
    return launch_ks_ext_lds(c, l, B, n1, n2, ext, own, keys, in, pts, sqp, beta, ne, W, lift, ts);
  if (W && c->ks_fuse_one) {
    // batches below ks_fuse_min_batch: one request and position per thread,
    // values-only streams below 2^50 (ks_fuse_lds = 0 keeps the register form)
    dim3 grid1(B * (c->N / BS) * ne);
#define HE_LAUNCH_ONE(BT, J)                                                                                      \
  HE_LAUNCH(ts, (k_ks_ext_one<BT, J>), grid1, dim3(BS), c->stream, ext, own, keys, in, pts, sqp, c->d_pc,        \
            c->d_moddown, c->N, c->log_n, l, c->nq, c->np, c->dnum, c->alpha, n1)
#define HE_ONE_J(BT)                                                                        \
  switch (n2) {                                                                             \
    case 8: HE_LAUNCH_ONE(BT, 8); break;                                                    \
    case 4: HE_LAUNCH_ONE(BT, 4); break;                                                    \
    case 2: HE_LAUNCH_ONE(BT, 2); break;                                                    \
    default: HE_LAUNCH_ONE(BT, 1); break;                                                   \
  }
    switch (beta) {
      case 1: HE_ONE_J(1); break;
      case 2: HE_ONE_J(2); break;
      case 3: HE_ONE_J(3); break;
      case 4: HE_ONE_J(4); break;
      case 5: HE_ONE_J(5); break;
      case 6: HE_ONE_J(6); break;
      case 7: HE_ONE_J(7); break;
      case 8: HE_ONE_J(8); break;
      default: return HE_EPARAM;
    }
#undef HE_ONE_J
#undef HE_LAUNCH_ONE
    return ok();
  }
  // items per thread: by default G n2 <= 16 accumulator pairs (each key and
  // plaintext word loaded is used G times); knob ks_fuse_g halves G
  // (fewer registers), knob ks_fuse_waves = 3 compiles for 3 waves per SIMD.
  const u32 Gd = n2 == 8 ? 2 : (n2 == 4 ? 4 : 8);
  const u32 G = c->ks_fuse_g ? Gd / 2 : Gd;
  const bool w3 = c->ks_fuse_waves == 3;
  dim3 grid(((B + G - 1) / G) * (c->N / BS) * ne);
#define HE_LAUNCH_FX(BT, J, GG)                                                                                   \
  do {                                                                                                            \
    if (w3)                                                                                                       \
      HE_LAUNCH(ts, (k_ks_ext_fused<BT, J, GG, 3>), grid, dim3(BS), c->stream, ext, own, keys, in, pts, sqp,      \
                c->d_pc, c->d_moddown, c->N, c->log_n, l, c->nq, c->np, c->dnum, c->alpha, n1);                   \
    else                                                                                                          \
      HE_LAUNCH(ts, (k_ks_ext_fused<BT, J, GG, 0>), grid, dim3(BS), c->stream, ext, own, keys, in, pts, sqp,      \
                c->d_pc, c->d_moddown, c->N, c->log_n, l, c->nq, c->np, c->dnum, c->alpha, n1);                   \
  } while (0)
#define HE_FX_J(BT)                                                            \
  switch (n2) {                                                                \
    case 8: if (G == 1) HE_LAUNCH_FX(BT, 8, 1); else HE_LAUNCH_FX(BT, 8, 2); break;  \
    case 4: if (G == 2) HE_LAUNCH_FX(BT, 4, 2); else HE_LAUNCH_FX(BT, 4, 4); break;  \
    case 2: if (G == 4) HE_LAUNCH_FX(BT, 2, 4); else HE_LAUNCH_FX(BT, 2, 8); break;  \
    default: if (G == 4) HE_LAUNCH_FX(BT, 1, 4); else HE_LAUNCH_FX(BT, 1, 8); break; \
  }
  switch (beta) {
    case 1: HE_FX_J(1); break;
    case 2: HE_FX_J(2); break;
    case 3: HE_FX_J(3); break;
    case 4: HE_FX_J(4); break;
    case 5: HE_FX_J(5); break;
    case 6: HE_FX_J(6); break;
    case 7: HE_FX_J(7); break;
    case 8: HE_FX_J(8); break;
    default: return HE_EPARAM;
  }
#undef HE_FX_J
#undef HE_LAUNCH_FX
  return ok();
}

