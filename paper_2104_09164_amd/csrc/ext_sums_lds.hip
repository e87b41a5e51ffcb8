// LDS-shared form of the fused lazy-ModDown inner sums (knob ks_fuse_lds):
// the same words as k_ks_ext_fused (ext_sums.hip), with each baby step's key
// and plaintext words shared through LDS by the threads of several requests.
#include "rns_kernels.hpp"
#include "modarith.hpp"
#include "rns_device.hpp"

namespace {

// The same sums with the key and plaintext words shared through LDS.  A
// workgroup covers 64 consecutive positions x of limb t for W requests (wave
// g serves request b0 + g), so a thread keeps only its own 2 JC sums in
// registers and the kernel runs at a higher
// occupancy than the register form.  Baby step i's words of the tile (4 beta
// key words and 2 JC plaintext words per position) are loaded once per
// workgroup into an LDS buffer, double-buffered: the loads of step i + 1 are
// issued before step i is computed and stored to LDS after it, with one
// barrier per step that every thread reaches.  Digits are gathered at y =
// perm_{g_i}(x) per request as in the register form, and so is the lift P c0
// mod q, formed once per position by k_lift_c0 (the register form multiplies
// c0(y) by P at every step); the sums are the register form's up to the
// representative of each lazy term, and the words written (in [0, q)) are
// the same.
// Words per position per step (4 per digit: key b, its companion, key a,
// its companion; 2 per giant sum: plaintext and companion), key rows each
// wave moves (W waves: wave w moves kind w mod 4 of the digits j = w / 4,
// w / 4 + W / 4, ...) and plaintext rows each wave moves.
constexpr int lds_nw(int beta, int jc) { return 4 * beta + 2 * jc; }
constexpr int lds_kr(int beta, int w) { return (beta + w / 4 - 1) / (w / 4); }
constexpr int lds_pr(int jc, int w) { return (2 * jc + w - 1) / w; }
constexpr int lds_st(int beta, int jc, int w) { return lds_kr(beta, w) + lds_pr(jc, w); }

// Tile rows of one step: row 4 j + k holds the key words of digit j (k = 0:
// b, 1: b companion, 2: a, 3: a companion); row 4 beta + 2 jj + {0, 1} the
// plaintext word and companion of giant sum jj.  The wave index is read into
// a scalar register, so every branch on a row is uniform over the wave.
template <int BETA, int JC, int W, int MODE>
__device__ __forceinline__ void lds_tile_load(u64 (&st)[lds_st(BETA, JC, W)], u32 w, u32 i,
                                              const u64* __restrict__ key, const u64* __restrict__ pts,
                                              const PrimeConst& P, u32 N, u32 ne, u32 nt, u32 pr, u32 t, u32 n1,
                                              size_t kw, size_t comp, u32 x) {
  constexpr int KR = lds_kr(BETA, W), PRW = lds_pr(JC, W);
  if (i > 0) {
    const u32 k = w & 3, j0 = w >> 2;
    const u64* kp = key + (k & 1 ? kw : 0) + ((size_t)(k >> 1) * nt + pr) * N + x;
#pragma unroll
    for (int r = 0; r < KR; ++r) {
      const u32 j = j0 + (W / 4) * r;
      if (j < (u32)BETA) st[r] = kp[(size_t)j * 2 * nt * N];
    }
  }
#pragma unroll
  for (int r = 0; r < PRW; ++r) {
    const u32 pw = w + W * r;                          // plaintext row (of 2 JC)
    if (pw < 2 * JC) {
      const u32 jj = pw >> 1;
      if (MODE == 3) {
        // 28-bit columns of the plaintext word: low 28 bits (row 2 jj), the rest (row 2 jj + 1)
        const u64 v = pts ? pts[(((size_t)n1 * jj + i) * ne + t) * N + x] : 1;
        st[KR + r] = pw & 1 ? v >> 28 : v & kLow28;
      } else if (!pts) {
        st[KR + r] = pw & 1 ? P.mu : 1;                // no plaintexts: a plain sum (x 1, companion mu)
      } else {
        st[KR + r] = pts[(pw & 1 ? comp : 0) + (((size_t)n1 * jj + i) * ne + t) * N + x];
      }
    }
  }
}
template <int BETA, int JC, int W>
__device__ __forceinline__ void lds_tile_store(const u64 (&st)[lds_st(BETA, JC, W)], u32 w, u32 i, u64 (*buf)[64],
                                               u32 p) {
  constexpr int KR = lds_kr(BETA, W), PRW = lds_pr(JC, W);
  if (i > 0) {
    const u32 k = w & 3, j0 = w >> 2;
#pragma unroll
    for (int r = 0; r < KR; ++r) {
      const u32 j = j0 + (W / 4) * r;
      if (j < (u32)BETA) buf[4 * j + k][p] = st[r];
    }
  }
#pragma unroll
  for (int r = 0; r < PRW; ++r) {
    const u32 pw = w + W * r;
    if (pw < 2 * JC) buf[4 * BETA + pw][p] = st[KR + r];
  }
}


// MODE 0: q < 2^55 (key sums lazy, inner sums lazy); 1: q < 2^60 with at
// most 4 digits (ks_dot_mid, mp_add_mid); 2: any other prime (every sum kept
// below 4q after each term); 3: q < 2^50, inner sums as exact integer column
// sums: r (lazy key sum plus lift, below 33 q < 2^55.1) and the plaintext word
// (below 2^50) split into 28-bit columns, r = a1 2^28 + a0, pt = b1 2^28 +
// b0; per product four multiply-adds into C0 += a0 b0 (< 2^56 per term),
// C1 += a0 b1 + a1 b0 (< 2^55.2), C2 += a1 b1 (< 2^49.1), each below 2^63
// over at most 65 terms; at the end C0 + C1 2^28 + C2 2^56 reduced mod q.
// The inner sum is the same integer as the modular one, so the words agree.
template <int BETA, int JC, int W, int MODE>
__device__ __forceinline__ void ks_ext_lds_body(const u64* __restrict__ ext, const OwnMap& own,
                                                const StepKeys& keys, const Items& in, const u64* __restrict__ pts,
                                                u64* __restrict__ sqp, const PrimeConst& P, u64 pw, u64 pws, u32 N,
                                                u32 logn, u32 l, u32 nt, u32 ne, u32 pr, u32 dstride, u32 alpha,
                                                u32 n1, u32 b0, u32 x0, u32 t, u64 (*sh)[lds_nw(BETA, JC)][64],
                                                const u64* __restrict__ c0p, u32 w) {
  // w: the wave within its block's W (uniform), serving request b0 + w
  const u32 B = in.n;
  const u32 p = threadIdx.x & 63;
  const u32 x = x0 + p, b = b0 + w;
  const bool active = b < B;                          // idle waves still move tiles and reach barriers
  const bool qlimb = t <= l;
  const u64 q = P.q;
  const size_t comp = (size_t)n1 * JC * ne * N;       // plaintext companions follow the m = n1 JC diagonals
  const size_t kw = (size_t)dstride * 2 * nt * N;     // key companions follow the key words
  const u32 own_digit = qlimb ? t / alpha : 0xFFFFFFFFu;
  u64 a0[JC], a1[JC];
#pragma unroll
  for (int jj = 0; jj < JC; ++jj) a0[jj] = a1[jj] = 0;
  constexpr bool COLS = MODE == 3;
  u64 w0[COLS ? JC : 1][3], w1[COLS ? JC : 1][3];   // MODE 3 column sums
#pragma unroll
  for (int jj = 0; jj < (COLS ? JC : 1); ++jj)
    w0[jj][0] = w0[jj][1] = w0[jj][2] = w1[jj][0] = w1[jj][1] = w1[jj][2] = 0;
  u64 st[lds_st(BETA, JC, W)];
  lds_tile_load<BETA, JC, W, MODE>(st, w, 0, nullptr, pts, P, N, ne, nt, pr, t, n1, kw, comp, x);
  lds_tile_store<BETA, JC, W>(st, w, 0, sh[0], p);
  // gathered words of the next baby step (digits at its automorphism of x,
  // and c0 there), issued one step ahead so that their latency hides behind
  // the current step's products
  const u64* e_base = ext + ((size_t)b * dstride * ne + t) * N;
  const u64* own_base = active ? own.ptr[b] + (size_t)t * N : nullptr;
  // the lift P c0 mod q of the request, formed for every position by k_lift_c0
  const u64* c0_base = active && qlimb ? c0p + ((size_t)b * (l + 1) + t) * N : nullptr;
  u64 dn[BETA], cn = 0;
  // with step i's tile in sh[i & 1]: issue the gathers and the tile loads of
  // step i + 1 (before step i is computed), then store that tile to the other
  // buffer (after)
  auto issue = [&](u32 i) {
    if (active && i + 1 < n1) {
      const u32 yn = galois_perm(x, keys.galois[i], logn);
#pragma unroll
      for (int j = 0; j < BETA; ++j) dn[j] = (u32)j == own_digit ? own_base[yn] : e_base[(size_t)j * ne * N + yn];
      if (qlimb) cn = c0_base[yn];
    }
    if (i + 1 < n1)
      lds_tile_load<BETA, JC, W, MODE>(st, w, i + 1, keys.key[i], pts, P, N, ne, nt, pr, t, n1, kw, comp, x);
  };
  auto retire = [&](u32 i) {
    if (i + 1 < n1) lds_tile_store<BETA, JC, W>(st, w, i + 1, sh[(i + 1) & 1], p);
  };
  // step 0 (kept out of the loop, so that the compiler never merges its
  // operands with the later steps'): the unrotated term (P c0, P c1) on the
  // Q-limbs
  __syncthreads();
  issue(0);
  if (active && qlimb) {
    const u64 (*cur)[64] = sh[0];
    const u64 r0 = c0_base[x], r1 = shoup(in.p[b][(size_t)(l + 1 + t) * N + x], pw, pws, q);
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) {
      const u64 pt = cur[4 * BETA + 2 * jj][p], ps = cur[4 * BETA + 2 * jj + 1][p];
      if (COLS) {
        col_mad(w0[jj], r0, pt, ps);
        col_mad(w1[jj], r1, pt, ps);
      } else if (MODE == 1) {
        a0[jj] = mp_add_mid(a0[jj], r0, pt, ps, P);
        a1[jj] = mp_add_mid(a1[jj], r1, pt, ps, P);
      } else {
        a0[jj] = mp_add<MODE == 0>(a0[jj], r0, pt, ps, P);
        a1[jj] = mp_add<MODE == 0>(a1[jj], r1, pt, ps, P);
      }
    }
  }
  retire(0);
  for (u32 i = 1; i < n1; ++i) {
    __syncthreads();                                  // step i's tile is in sh[i & 1]; sh[(i + 1) & 1] is free
    u64 d[BETA], c0y = cn;
#pragma unroll
    for (int j = 0; j < BETA; ++j) d[j] = dn[j];
    issue(i);
    const u64 (*cur)[64] = sh[i & 1];
    if (active) {
      {
        u64 kb[BETA], kbs[BETA], ka[BETA], kas[BETA];
#pragma unroll
        for (int j = 0; j < BETA; ++j) {
          kb[j] = cur[4 * j][p];
          kbs[j] = cur[4 * j + 1][p];
          ka[j] = cur[4 * j + 2][p];
          kas[j] = cur[4 * j + 3][p];
        }
        u64 r0, r1;
        if (MODE == 1) {
          if constexpr (BETA <= 4) ks_dot_mid<BETA>(d, kb, kbs, ka, kas, P, r0, r1);
        } else {
          ks_dot<BETA, MODE == 0 || MODE == 3>(d, kb, kbs, ka, kas, P, false, r0, r1);
        }
        if (qlimb) r0 += c0y;                          // below q, read for this step's automorphism
        if (MODE == 1 && i % 3 == 0) {
          // the inner sums of MODE 1 (q >= 2^55): reduced before every third
          // product, in one uniform branch per step
#pragma unroll
          for (int jj = 0; jj < JC; ++jj) {
            a0[jj] = reduce_lazy_wide(a0[jj], P.q, P.mu);
            a1[jj] = reduce_lazy_wide(a1[jj], P.q, P.mu);
          }
        }
#pragma unroll
        for (int jj = 0; jj < JC; ++jj) {
          const u64 pt = cur[4 * BETA + 2 * jj][p], ps = cur[4 * BETA + 2 * jj + 1][p];
          if (MODE == 3) {
            col_mad(w0[jj], r0, pt, ps);
            col_mad(w1[jj], r1, pt, ps);
          } else if (MODE == 1) {
            a0[jj] = mp_add_mid(a0[jj], r0, pt, ps, P);
            a1[jj] = mp_add_mid(a1[jj], r1, pt, ps, P);
          } else {
            a0[jj] = mp_add<MODE == 0>(a0[jj], r0, pt, ps, P);
            a1[jj] = mp_add<MODE == 0>(a1[jj], r1, pt, ps, P);
          }
        }
      }
    }
    retire(i);
  }
  if (!active) return;
#pragma unroll
  for (int jj = 0; jj < JC; ++jj) {
    u64* o = sqp + ((size_t)jj * B + b) * 2 * ne * N;
    if (COLS) {
      o[(size_t)t * N + x] = col_final(w0[jj], P);
      o[(size_t)(ne + t) * N + x] = col_final(w1[jj], P);
    } else {
      o[(size_t)t * N + x] = mp_final<MODE != 2>(a0[jj], P);
      o[(size_t)(ne + t) * N + x] = mp_final<MODE != 2>(a1[jj], P);
    }
  }
}

// 1-D grid over request groups of W x (tiles, ne) (xcd_decode: the groups of
// a tile run back to back on one XCD and share its words in L2).  A tile is
// one 64-position block (H = 1) or two (H = 2), each served by its own W
// waves with its own LDS tiles.  With `orbit` (the blocks in the order of the
// cycles of P, the block map of galois[0]: block X reads P(X) at the first
// step) the tiles run on one XCD, in order, follow those cycles: since
// galois[s] = galois[0]^(s+1), block P(X) reads at step i the block X reads
// at step i + 1, so the workgroups running together on an XCD read each
// other's gathers of the step before from L2, and a digit block comes from
// HBM about once per run of tiles instead of once per step.  H = 2 pairs X
// with P(X) in one workgroup (entries 2k, 2k + 1 of an orbit table whose
// cycles all have even length).
template <int BETA, int JC, int W, int H>
__global__ void __launch_bounds__(64 * W * H) __attribute__((amdgpu_waves_per_eu(4)))
k_ks_ext_lds(const u64* __restrict__ ext, OwnMap own, StepKeys keys, Items in, const u64* __restrict__ pts,
             u64* __restrict__ sqp, const PrimeConst* __restrict__ pc, const u64* __restrict__ md, u32 N, u32 logn,
             u32 l, u32 nq, u32 np, u32 dstride, u32 alpha, u32 n1, const u64* __restrict__ c0p,
             const uint16_t* __restrict__ orbit) {
  __shared__ u64 sh[H][2][lds_nw(BETA, JC)][64];
  const u32 npb = N / 64, ntile = npb / H, ne = l + 1 + np, nt = nq + np;
  const u32 ngroups = (in.n + W - 1) / W;
  u32 grp, tile;
  xcd_decode(blockIdx.x, ngroups, ntile * ne, grp, tile);
  const u32 wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const u32 h = wv / W, w = wv % W;                   // block h of the tile, wave w of its W
  u32 blk = tile % ntile;
  if (orbit) {
    // tile u of a limb runs on XCD u mod 8 as its (u / 8)-th: XCD x takes the
    // x-th eighth of the orbit order
    const u32 idx = (blk % 8) * (ntile / 8) + blk / 8;
    blk = orbit[H * idx + h];
  }
  const u32 x0 = blk * 64, t = tile / ntile;
  const u32 pr = t <= l ? t : nq + (t - l - 1);
  const PrimeConst P = pc[pr];
  const u64* pmod = md + 2 * np + 2 * (size_t)np * nq + 2 * (size_t)nq;   // [nq][2] P mod q_i
  const u64 pw = t <= l ? pmod[2 * t] : 0, pws = t <= l ? pmod[2 * t + 1] : 0;
  const u32 b0 = grp * W;
#define HE_LDS_BODY(M)                                                                                              \
  ks_ext_lds_body<BETA, JC, W, M>(ext, own, keys, in, pts, sqp, P, pw, pws, N, logn, l, nt, ne, pr, dstride, alpha, \
                                  n1, b0, x0, t, sh[h], c0p, w)
  if (P.q < kWideQ)
    HE_LDS_BODY(3);
  else if (P.q < kLazyMP)
    HE_LDS_BODY(0);
  else if (BETA <= 4 && P.q < kMidQ)
    HE_LDS_BODY(1);
  else
    HE_LDS_BODY(2);
#undef HE_LDS_BODY
}

// The lift of c0 by P on the Q-limbs, P c0 mod q_t in [0, q_t), for every
// request b, limb t <= l and position x, at lift + (b (l + 1) + t) N + x:
// each baby step reads it at its automorphism of x, where the inner sums
// would otherwise form the product there once per step.  Grid (N / 256,
// l + 1, B).
__global__ void __launch_bounds__(256) k_lift_c0(Items in, u64* __restrict__ lift,
                                                 const PrimeConst* __restrict__ pc, const u64* __restrict__ md,
                                                 u32 N, u32 l, u32 nq, u32 np) {
  const u32 x = blockIdx.x * 256 + threadIdx.x, t = blockIdx.y, b = blockIdx.z;
  const u64* pmod = md + 2 * np + 2 * (size_t)np * nq + 2 * (size_t)nq;   // [nq][2] P mod q_i
  lift[((size_t)b * (l + 1) + t) * N + x] = shoup(in.p[b][(size_t)t * N + x], pmod[2 * t], pmod[2 * t + 1], pc[t].q);
}

}  // namespace

int launch_ks_ext_lds(he_ctx* c, u32 l, u32 B, u32 n1, u32 n2, const u64* ext, const OwnMap& own,
                      const StepKeys& keys, const Items& in, const u64* pts, u64* sqp, u32 beta, u32 ne, u32 W,
                      u64* lift, TraceScope& ts) {
  if (!lift) return HE_EINVAL;
  {
    TraceScope tl(c, TK_LIFT_C0, (double)B * (l + 1) * 16.0 * (double)c->N);
    HE_LAUNCH(tl, k_lift_c0, dim3(c->N / 256, l + 1, B), dim3(256), c->stream, in, lift, c->d_pc, c->d_moddown,
              c->N, l, c->nq, c->np);
  }
  const u64* c0p = lift;
  // the LDS-shared form: W requests (waves) per block, 64 positions, one
  // block per workgroup or (knob ks_fuse_pair, W <= 8, a run of powers of one
  // automorphism whose block cycles have even length) a pair of blocks; the
  // blocks dealt to the XCDs along the automorphism's cycles (knob
  // ks_fuse_orbit, a run of powers of one automorphism)
  const u32 H = c->ks_fuse_pair && keys.orbit && keys.orbit_even && W <= 8 ? 2 : 1;
  const uint16_t* orbit = keys.orbit && (c->ks_fuse_orbit || H == 2) ? keys.orbit : nullptr;
  dim3 grid_l(((B + W - 1) / W) * (c->N / 64 / H) * ne);
#define HE_LAUNCH_LX(BT, J, WW, HH)                                                                               \
  HE_LAUNCH(ts, (k_ks_ext_lds<BT, J, WW, HH>), grid_l, dim3(64 * WW * HH), c->stream, ext, own, keys, in, pts,    \
            sqp, c->d_pc, c->d_moddown, c->N, c->log_n, l, c->nq, c->np, c->dnum, c->alpha, n1, c0p, orbit)
#define HE_LX_W(BT, J)                                                                      \
  do {                                                                                      \
    if (W == 16) HE_LAUNCH_LX(BT, J, 16, 1);                                                \
    else if (W == 8 && H == 2) HE_LAUNCH_LX(BT, J, 8, 2);                                   \
    else if (W == 8) HE_LAUNCH_LX(BT, J, 8, 1);                                             \
    else if (H == 2) HE_LAUNCH_LX(BT, J, 4, 2);                                             \
    else HE_LAUNCH_LX(BT, J, 4, 1);                                                         \
  } while (0)
#define HE_LX_J(BT)                                                                         \
  switch (n2) {                                                                             \
    case 8: HE_LX_W(BT, 8); break;                                                          \
    case 4: HE_LX_W(BT, 4); break;                                                          \
    case 2: HE_LX_W(BT, 2); break;                                                          \
    default: HE_LX_W(BT, 1); break;                                                         \
  }
  switch (beta) {
    case 1: HE_LX_J(1); break;
    case 2: HE_LX_J(2); break;
    case 3: HE_LX_J(3); break;
    case 4: HE_LX_J(4); break;
    case 5: HE_LX_J(5); break;
    case 6: HE_LX_J(6); break;
    case 7: HE_LX_J(7); break;
    case 8: HE_LX_J(8); break;
    default: return HE_EPARAM;
  }
#undef HE_LX_J
#undef HE_LX_W
#undef HE_LAUNCH_LX
  return ok();
}
