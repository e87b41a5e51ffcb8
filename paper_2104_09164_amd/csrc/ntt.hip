// Negacyclic number-theoretic transform for gfx950.
//
// Forward: Cooley-Tukey, decimation in time, bit-reversed output order
// (position k holds a(psi^(2 brev(k) + 1))); stage s = 0..logN-1 pairs
// (j, j + N/2^(s+1)) with twiddle psi^brev(2^s + (j >> (logN - s))).
// Inverse: the Gentleman-Sande mirror image with psi^-brev(.), then N^{-1}.
// Lazy butterflies in the style of Harvey: the twiddle product uses a
// three-term Shoup quotient (result in [0, 4q)), values stay below 8q
// (forward) / 4q (inverse) between stages, and outputs are fully reduced to
// [0, q) on the way out.  Twiddles are stored as (w, w') pairs so one 16-byte
// load fetches both.
//
// Decomposition.  logN stages split into phases of LP stages.  A phase
// works on tiles of COLS independent sub-transforms of length 2^LP held in
// LDS: phase A (stages 0..LA-1) on columns j = k 2^LB + lo (stride 2^LB),
// phase B (stages LA..logN-1) on contiguous rows j = hi 2^LB + k.  For
// logN <= 13 a single phase covers the whole polynomial.  Inside a phase each
// thread loads 2^r elements of one radix-2^r butterfly group from LDS into
// registers, runs r stages there, and writes back; passes of r = 3..5 stages
// cover the phase.  HBM is touched once per phase (coalesced tile copies).
// The hot path is HBM/VALU balanced on MI355X: a 64x64-bit modular multiply
// is ~9 VALU ops (v_mad_u64_u32 is full rate on gfx950).
#include <algorithm>
#include "he_internal.hpp"
#include "modarith.hpp"

namespace {

__host__ __device__ constexpr int npasses(int lp) { return lp <= 5 ? 1 : (lp <= 10 ? 2 : 3); }
__host__ __device__ constexpr int pass_bits(int lp, int p) {
  return lp / npasses(lp) + (p < lp % npasses(lp) ? 1 : 0);
}
__host__ __device__ constexpr int pass_start(int lp, int p) {
  int s = 0;
  for (int i = 0; i < p; ++i) s += pass_bits(lp, i);
  return s;
}

__device__ __forceinline__ const u64* item_src(const PolyBatch& pb, u32 b) {
  return pb.stride ? pb.src[0] + (size_t)b * pb.stride : pb.src[b];
}
__device__ __forceinline__ u64* item_dst(const PolyBatch& pb, u32 b) {
  return pb.stride ? pb.dst[0] + (size_t)b * (pb.dst_stride ? pb.dst_stride : pb.stride) : pb.dst[b];
}

// Primes below 2^57 take the forward butterflies without the per-stage
// conditional subtraction (room for the lazy bound growth up to N = 2^17).
constexpr u64 kLazyQ = 1ull << 57;

// LDS padding: one spare word every 16 to spread strided accesses over banks.
__device__ __forceinline__ u32 pidx(u32 i) { return i + (i >> 4); }

template <int LOGN, int S0, int LP, int COLS, int NT, bool INV>
struct Phase {
  static constexpr int TILE = COLS << LP;
  static constexpr bool ROWS = S0 > 0;       // phase B layout (contiguous sub-transforms)

  // tile-local linear index of (col, k)
  __device__ static __forceinline__ u32 local(u32 col, u32 k) {
    return ROWS ? (col << LP) + k : k * COLS + col;
  }
  // global word offset within the polynomial of tile-local index i
  __device__ static __forceinline__ u32 gaddr(u32 sub0, u32 i) {
    if (ROWS) return (sub0 << LP) + i;
    return (i / COLS) * (1u << (LOGN - LP)) + sub0 + (i % COLS);
  }

  // Forward stages S0+U .. S0+U+RB-1 on one radix-2^RB group.  CSUB-free
  // form (NOCSUB, primes below kLazyQ): X is not brought below 4q, so the
  // bound grows by 4q per stage, from below 8q at the input to below
  // (8 + 4 logN) q <= 76 q < 2^64 after the last stage; the final pass
  // reduces it.  Otherwise values stay below 8q between stages.
  template <int U, int RB, bool NOCSUB>
  __device__ static __forceinline__ void fwd_stages(u64 (&x)[1 << RB], const ulonglong2* __restrict__ tw,
                                                    const PrimeConst& k, u32 hi, u32 kt) {
    constexpr int R = 1 << RB;
    const u64 q4 = 4 * k.q;
#pragma unroll
    for (int uu = 0; uu < RB; ++uu) {
      const int s = S0 + U + uu;
      const int half = R >> (uu + 1);
#pragma unroll
      for (int blk = 0; blk < (1 << uu); ++blk) {
        const u32 ti = (1u << s) + (hi << (U + uu)) + (kt << uu) + blk;
        const ulonglong2 wp = tw[ti];
#pragma unroll
        for (int e = 0; e < half; ++e) {
          const int m0 = blk * 2 * half + e, m1 = m0 + half;
          const u64 X = NOCSUB ? x[m0] : csub_neg(x[m0], k.nq4);     // < 4q (CSUB form)
          const u64 S = add_shoup4(X, x[m1], wp.x, wp.y, k.nq);      // X + T, T < 4q
          x[m0] = S;
          x[m1] = 2 * X + q4 - S;                                   // X + 4q - T > 0 (mod 2^64 wrap exact)
        }
      }
    }
  }

  // Output word of the phase: reduced to [0, q) (and scaled by N^{-1} for the
  // inverse) when final_, else the lazy value as is.
  template <bool NOCSUB>
  __device__ static __forceinline__ u64 out_word(u64 a, const PrimeConst& k, int final_) {
    if (!final_) return a;
    if (INV) return csub_neg(csub_neg(a, k.nq2), k.nq);   // N^{-1} already applied at stage 0
    if (NOCSUB) return csub_neg(csub_neg(reduce_lazy(a, k.q, k.mu), k.nq2), k.nq);   // lazy value below 76q
    return csub_neg(csub_neg(csub_neg(a, k.nq4), k.nq2), k.nq);
  }

  // One pass of RB stages.  FROM_G: the group is read straight from the
  // phase's source in HBM instead of the LDS tile; TO_G: written straight to
  // the destination (with out_word) instead of back to LDS.  Both are used by
  // the column phase, whose groups are coalesced rows of COLS words.
  template <int U, int RB, bool NOCSUB, bool FROM_G = false, bool TO_G = false>
  __device__ static __forceinline__ void pass(u64* lds, const ulonglong2* __restrict__ tw, const PrimeConst& k,
                                              u32 sub0, const u64* src = nullptr, u64* dst = nullptr,
                                              int final_ = 0) {
    const u64 q = k.q;
    constexpr int R = 1 << RB;
    constexpr int KL = 1 << (LP - U - RB);
    constexpr int KT = 1 << U;
    constexpr int GROUPS = COLS * KL * KT;
    for (int g = threadIdx.x; g < GROUPS; g += NT) {
      u32 kl, col, kt;
      // Lane order.  Columns layout: column fastest (stride 1 word).  Rows
      // layout: k bits fastest (kl, then kt: stride 1 or 2^r words, 17 after
      // padding), rows last; a row-fastest order would put 256-word strides
      // between lanes and serialise on two bank groups.
      if (!ROWS) { col = g % COLS; u32 t = g / COLS; kl = t % KL; kt = t / KL; }
      else { kl = g % KL; u32 t = g / KL; kt = t % KT; col = t / KT; }
      const u32 hi = ROWS ? sub0 + col : 0;
      u64 x[R];
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const u32 li = local(col, kt * (R * KL) + m * KL + kl);
        x[m] = FROM_G ? src[gaddr(sub0, li)] : lds[pidx(li)];
      }
      const u64 q4 = 4 * q;
      if (!INV) {
        fwd_stages<U, RB, NOCSUB>(x, tw, k, hi, kt);
      } else {
#pragma unroll
        for (int uu = RB - 1; uu >= 0; --uu) {
          const int s = S0 + U + uu;
          const int half = R >> (uu + 1);
#pragma unroll
          for (int blk = 0; blk < (1 << uu); ++blk) {
            const u32 ti = (1u << s) + (hi << (U + uu)) + (kt << uu) + blk;
            const ulonglong2 wp = tw[ti];
#pragma unroll
            for (int e = 0; e < half; ++e) {
              const int m0 = blk * 2 * half + e, m1 = m0 + half;
              const u64 A = x[m0], B = x[m1];                            // < 4q
              if (s == 0) {
                // last stage of the inverse: N^{-1} folded into both outputs
                // (the phase holding stage 0 is always the final one)
                x[m0] = shoup_lazy4(A + B, k.ninv, k.ninv_sh, q);        // < 4q
                x[m1] = shoup_lazy4(A + q4 - B, k.w0ni, k.w0ni_sh, q);   // < 4q
              } else {
                x[m0] = csub_neg(A + B, k.nq4);                          // < 4q
                x[m1] = shoup_lazy4(A + q4 - B, wp.x, wp.y, q);          // < 4q
              }
            }
          }
        }
      }
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const u32 li = local(col, kt * (R * KL) + m * KL + kl);
        if (TO_G) dst[gaddr(sub0, li)] = out_word<NOCSUB>(x[m], k, final_);
        else lds[pidx(li)] = x[m];
      }
    }
  }

  template <int P, bool NOCSUB>
  __device__ static __forceinline__ void passes_fwd(u64* lds, const ulonglong2* tw, const PrimeConst& k, u32 sub0) {
    if constexpr (P < npasses(LP)) {
      pass<pass_start(LP, P), pass_bits(LP, P), NOCSUB>(lds, tw, k, sub0);
      __syncthreads();
      passes_fwd<P + 1, NOCSUB>(lds, tw, k, sub0);
    }
  }
  template <int P>
  __device__ static __forceinline__ void passes_inv(u64* lds, const ulonglong2* tw, const PrimeConst& k, u32 sub0) {
    if constexpr (P >= 0) {
      pass<pass_start(LP, P), pass_bits(LP, P), false>(lds, tw, k, sub0);
      __syncthreads();
      passes_inv<P - 1>(lds, tw, k, sub0);
    }
  }

  // Tile in (16-byte pairs; COLS and 2^LP are even, so pairs never straddle
  // a row), the phase's stages, tile out.  final_: reduce to [0, q) (and
  // scale by N^{-1} for the inverse) on the way out.
  template <bool NOCSUB>
  __device__ static __forceinline__ void body(u64* lds, const u64* src, u64* dst, const ulonglong2* __restrict__ tw,
                                              const PrimeConst& k, u32 sub0, int final_) {
    if constexpr (!ROWS && npasses(LP) == 2) {
      // column phase: first pass from HBM, second pass to HBM, LDS only in between
      constexpr int P0 = INV ? 1 : 0, P1 = INV ? 0 : 1;
      pass<pass_start(LP, P0), pass_bits(LP, P0), NOCSUB, true, false>(lds, tw, k, sub0, src);
      __syncthreads();
      pass<pass_start(LP, P1), pass_bits(LP, P1), NOCSUB, false, true>(lds, tw, k, sub0, nullptr, dst, final_);
      return;
    }
    const u64 q = k.q;
    if constexpr (ROWS && npasses(LP) == 2 && (!INV || pass_bits(LP, 1) <= 3)) {
      // row phase: first pass straight from HBM; the last pass goes back
      // through LDS so the tile leaves in full 16-byte rows.  Lanes of the
      // forward's first pass read runs of 2^(LP-RB) consecutive words; the
      // inverse starts with the last stages, whose lanes sit 2^RB words apart,
      // so it reads directly only when that gap is at most 8 words (64 bytes).
      constexpr int P0 = INV ? 1 : 0, P1 = INV ? 0 : 1;
      pass<pass_start(LP, P0), pass_bits(LP, P0), NOCSUB, true, false>(lds, tw, k, sub0, src);
      __syncthreads();
      pass<pass_start(LP, P1), pass_bits(LP, P1), NOCSUB>(lds, tw, k, sub0);
      __syncthreads();
    } else {
      for (u32 i = 2 * threadIdx.x; i < (u32)TILE; i += 2 * NT) {
        const ulonglong2 v = *(const ulonglong2*)(src + gaddr(sub0, i));
        lds[pidx(i)] = v.x;
        lds[pidx(i + 1)] = v.y;
      }
      __syncthreads();
      if (!INV) passes_fwd<0, NOCSUB>(lds, tw, k, sub0);
      else passes_inv<npasses(LP) - 1>(lds, tw, k, sub0);
    }
    ulonglong2 v;
    if (final_) {
      for (u32 i = 2 * threadIdx.x; i < (u32)TILE; i += 2 * NT) {
        v.x = out_word<NOCSUB>(lds[pidx(i)], k, 1);
        v.y = out_word<NOCSUB>(lds[pidx(i + 1)], k, 1);
        *(ulonglong2*)(dst + gaddr(sub0, i)) = v;
      }
    } else {
      for (u32 i = 2 * threadIdx.x; i < (u32)TILE; i += 2 * NT) {
        v.x = lds[pidx(i)];
        v.y = lds[pidx(i + 1)];
        *(ulonglong2*)(dst + gaddr(sub0, i)) = v;
      }
    }
  }
};

// Radix-2^RB butterflies on a register array x[m], m = the RB index bits of
// the stages s0 .. s0+RB-1 (most significant first); `prefix` = the index bits
// above them, so the twiddle of sub-stage uu, block blk is
// psi^brev(2^(s0+uu) + prefix 2^uu + blk).
template <int RB, bool INV>
__device__ __forceinline__ void reg_pass(u64 (&x)[1 << RB], const ulonglong2* __restrict__ tw, const PrimeConst& k,
                                         u32 s0, u32 prefix) {
  constexpr int R = 1 << RB;
  const u64 q = k.q, q4 = 4 * q;
  if (!INV) {
#pragma unroll
    for (int uu = 0; uu < RB; ++uu) {
      const int half = R >> (uu + 1);
#pragma unroll
      for (int blk = 0; blk < (1 << uu); ++blk) {
        const ulonglong2 wp = tw[(1u << (s0 + uu)) + (prefix << uu) + blk];
#pragma unroll
        for (int e = 0; e < half; ++e) {
          const int m0 = blk * 2 * half + e, m1 = m0 + half;
          const u64 X = csub_neg(x[m0], k.nq4);
          const u64 S = add_shoup4(X, x[m1], wp.x, wp.y, k.nq);
          x[m0] = S;
          x[m1] = 2 * X + q4 - S;
        }
      }
    }
  } else {
#pragma unroll
    for (int uu = RB - 1; uu >= 0; --uu) {
      const int half = R >> (uu + 1);
#pragma unroll
      for (int blk = 0; blk < (1 << uu); ++blk) {
        const ulonglong2 wp = tw[(1u << (s0 + uu)) + (prefix << uu) + blk];
#pragma unroll
        for (int e = 0; e < half; ++e) {
          const int m0 = blk * 2 * half + e, m1 = m0 + half;
          const u64 A = x[m0], B = x[m1];
          x[m0] = csub_neg(A + B, k.nq4);
          x[m1] = shoup_lazy4(A + q4 - B, wp.x, wp.y, q);
        }
      }
    }
  }
}

// Single-pass transform for N = 2^15: one 1024-thread workgroup per
// limb-poly holds the whole polynomial in registers (32 words per thread);
// index j = a 2^10 + b 2^5 + c.  Pass 1 (stages 0-4, bits of a) runs in
// thread (b, c), pass 2 (stages 5-9, bits of b) in thread (a, c), pass 3
// (stages 10-14, bits of c) in thread (a, b).  The two transposes go through
// LDS in two rounds, each round moving the words of the threads that keep
// the preserved index's top bit (c for the first, a for the second): those
// threads write all 32 words and read back 32, reusing one register array,
// so no thread ever holds more than 32 words.  HBM sees one read and one
// write of every word.  Grid: (item, poly), polynomials of one prime adjacent.
constexpr int T1_A = 32 * 16 + 16;       // transpose 1 slab: [a][b][c mod 16]
constexpr int T2_ROW = 33, T2_SLAB = 32 * T2_ROW;   // transpose 2: [a mod 16][b][c], rows padded

template <bool INV>
__global__ void __launch_bounds__(1024) k_ntt15(PolyBatch pb, const u64* __restrict__ tw_all,
                                                const PrimeConst* __restrict__ pc) {
  constexpr u32 N = 1u << 15;
  __shared__ u64 lds[32 * T1_A > 16 * T2_SLAB ? 32 * T1_A : 16 * T2_SLAB];
  const u32 b_item = blockIdx.x, r = blockIdx.y;
  const u32 pr = pb.prime[r];
  const PrimeConst k = pc[pr];
  const ulonglong2* tw = (const ulonglong2*)(tw_all + (size_t)pr * 4 * N + (INV ? 2 * N : 0));
  const u32 row = pb.row[r];
  const u64* src = item_src(pb, b_item) + (size_t)(pb.src_off + row) * N;
  u64* dst = item_dst(pb, b_item) + (size_t)(pb.dst_off + row) * N;
  const u32 t = threadIdx.x, hi5 = t >> 5, lo5 = t & 31;
  const u32 c_half = lo5 >> 4, cl = lo5 & 15, a_half = t >> 9, al = hi5 & 15;
  u64 x[32];
  if (!INV) {
    // thread (b, c) = (hi5, lo5): x[a] = word a 2^10 + t (coalesced)
#pragma unroll
    for (int a = 0; a < 32; ++a) x[a] = src[a * 1024 + t];
    reg_pass<5, false>(x, tw, k, 0, 0);
    // transpose 1 (c preserved): (b, c) holds a  ->  (a, c) holds b
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h) __syncthreads();
      if (c_half == (u32)h) {
#pragma unroll
        for (int a = 0; a < 32; ++a) lds[a * T1_A + hi5 * 16 + cl] = x[a];
      }
      __syncthreads();
      if (c_half == (u32)h) {
#pragma unroll
        for (int bb = 0; bb < 32; ++bb) x[bb] = lds[hi5 * T1_A + bb * 16 + cl];
      }
    }
    reg_pass<5, false>(x, tw, k, 5, hi5);                   // thread (a, c): prefix a
    // transpose 2 (a preserved): (a, c) holds b  ->  (a, b) holds c
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      __syncthreads();
      if (a_half == (u32)h) {
#pragma unroll
        for (int bb = 0; bb < 32; ++bb) lds[al * T2_SLAB + bb * T2_ROW + lo5] = x[bb];
      }
      __syncthreads();
      if (a_half == (u32)h) {
#pragma unroll
        for (int cc = 0; cc < 32; ++cc) x[cc] = lds[al * T2_SLAB + lo5 * T2_ROW + cc];
      }
    }
    reg_pass<5, false>(x, tw, k, 10, t);                    // thread (a, b): prefix a 2^5 + b = t
#pragma unroll
    for (int cc = 0; cc < 32; cc += 2) {
      ulonglong2 v;
      v.x = csub_neg(csub_neg(csub_neg(x[cc], k.nq4), k.nq2), k.nq);
      v.y = csub_neg(csub_neg(csub_neg(x[cc + 1], k.nq4), k.nq2), k.nq);
      *(ulonglong2*)(dst + t * 32 + cc) = v;
    }
  } else {
    // thread (a, b) = (hi5, lo5): x[c] = word t 2^5 + c
#pragma unroll
    for (int cc = 0; cc < 32; cc += 2) {
      const ulonglong2 v = *(const ulonglong2*)(src + t * 32 + cc);
      x[cc] = v.x;
      x[cc + 1] = v.y;
    }
    reg_pass<5, true>(x, tw, k, 10, t);
    // transpose 2 back (a preserved): (a, b) holds c  ->  (a, c) holds b
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      __syncthreads();
      if (a_half == (u32)h) {
#pragma unroll
        for (int cc = 0; cc < 32; ++cc) lds[al * T2_SLAB + lo5 * T2_ROW + cc] = x[cc];
      }
      __syncthreads();
      if (a_half == (u32)h) {
#pragma unroll
        for (int bb = 0; bb < 32; ++bb) x[bb] = lds[al * T2_SLAB + bb * T2_ROW + lo5];
      }
    }
    reg_pass<5, true>(x, tw, k, 5, hi5);                    // thread (a, c)
    // transpose 1 back (c preserved): (a, c) holds b  ->  (b, c) holds a
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      __syncthreads();
      if (c_half == (u32)h) {
#pragma unroll
        for (int bb = 0; bb < 32; ++bb) lds[hi5 * T1_A + bb * 16 + cl] = x[bb];
      }
      __syncthreads();
      if (c_half == (u32)h) {
#pragma unroll
        for (int a = 0; a < 32; ++a) x[a] = lds[a * T1_A + hi5 * 16 + cl];
      }
    }
    reg_pass<5, true>(x, tw, k, 0, 0);                      // thread (b, c)
#pragma unroll
    for (int a = 0; a < 32; ++a)
      dst[a * 1024 + t] = csub_neg(csub_neg(shoup_lazy4(x[a], k.ninv, k.ninv_sh, k.q), k.nq2), k.nq);
  }
}

// One launch = one phase over every (tile, poly, item).  read_src: load from
// pb.src (first phase) else from pb.dst.  final_: reduce to [0, q) (and scale
// by N^{-1} for the inverse) on the way out.
template <int LOGN, int S0, int LP, int COLS, int NT, bool INV>
__global__ void __launch_bounds__(NT) k_ntt_phase(PolyBatch pb, const u64* __restrict__ tw_all,
                                                  const PrimeConst* __restrict__ pc, int read_src, int final_) {
  using Ph = Phase<LOGN, S0, LP, COLS, NT, INV>;
  constexpr int TILE = Ph::TILE;
  __shared__ u64 lds[TILE + TILE / 16];
  // grid (tile, item, poly): all items of one limb are adjacent, so the twiddle
  // table of that prime is reused from L2 across the batch; 2^k tiles per
  // polynomial keep tile t on XCD t mod 8, which then needs 1/8 of the table.
  const u32 tile = blockIdx.x, b = blockIdx.y, r = blockIdx.z;
  const u32 pr = pb.prime[r];
  const u32 N = 1u << LOGN;
  const PrimeConst k = pc[pr];
  const u64 q = k.q;
  const ulonglong2* tw = (const ulonglong2*)(tw_all + (size_t)pr * 4 * N + (INV ? 2 * N : 0));
  const u32 row = pb.row[r];
  u64* dst = item_dst(pb, b) + (size_t)(pb.dst_off + row) * N;
  const u64* src = read_src ? item_src(pb, b) + (size_t)(pb.src_off + row) * N : dst;
  const u32 sub0 = tile * COLS;
  // the whole body is specialised on the butterfly form, so no load is
  // shared (and hoisted) across the two
  if (!INV && q < kLazyQ) Ph::template body<true>(lds, src, dst, tw, k, sub0, final_);
  else Ph::template body<false>(lds, src, dst, tw, k, sub0, final_);
}

u32 valid_polys(const PolyBatch& pb) { return pb.npoly * pb.nitems; }   // rows are compacted

template <int LOGN, int S0, int LP, int COLS, int NT, bool INV>
void launch_phase(he_ctx* c, const PolyBatch& pb, int read_src, int final_) {
  const int kind = LP == LOGN ? (INV ? TK_NTT_ONE_INV : TK_NTT_ONE_FWD)
                              : (S0 == 0 ? (INV ? TK_NTT_INV_A : TK_NTT_FWD_A) : (INV ? TK_NTT_INV_B : TK_NTT_FWD_B));
  TraceScope ts(c, kind, 16.0 * (double)valid_polys(pb) * (double)(1u << LOGN));
  dim3 grid((1u << (LOGN - LP)) / COLS, pb.nitems, pb.npoly);
  HE_LAUNCH(ts, (k_ntt_phase<LOGN, S0, LP, COLS, NT, INV>), grid, dim3(NT), c->stream, pb, c->d_tw, c->d_pc,
                     read_src, final_);
}

// Single phase for logN <= 13, two phases (LA = ceil(logN/2)) above.  With
// the knob ntt_chunk_mb > 0 the two-phase transform runs phase A then phase B
// on chunks of that many MiB of polynomials, so that the intermediate written
// by phase A can still be in the Infinity Cache when phase B reads it back.

// Phase A (columns) with COLS sub-transforms per tile; phase B (rows) with
// CB.  Column tiles want >= 16 so each row segment is a full 128-byte line;
// row tiles are contiguous at any width, and narrower ones give more,
// smaller workgroups.
template <int LOGN, int COLS>
void phase_a(he_ctx* c, const PolyBatch& ch, bool inv, int read_src, int final_) {
  constexpr int LA = (LOGN + 1) / 2;
  constexpr int NTA = ((COLS << LA) / 16) > 512 ? 512 : ((COLS << LA) / 16);
  if (!inv) launch_phase<LOGN, 0, LA, COLS, NTA, false>(c, ch, read_src, final_);
  else launch_phase<LOGN, 0, LA, COLS, NTA, true>(c, ch, read_src, final_);
}
template <int LOGN, int CB>
void phase_b(he_ctx* c, const PolyBatch& ch, bool inv, int read_src, int final_) {
  constexpr int LA = (LOGN + 1) / 2, LB = LOGN - LA;
  constexpr int NTB = ((CB << LB) / 16) > 512 ? 512 : ((CB << LB) / 16);
  if (!inv) launch_phase<LOGN, LA, LB, CB, NTB, false>(c, ch, read_src, final_);
  else launch_phase<LOGN, LA, LB, CB, NTB, true>(c, ch, read_src, final_);
}
template <int LOGN>
void ntt_two_phase(he_ctx* c, const PolyBatch& ch, bool inv) {
  const int ca = (int)c->ntt_cols, cb = c->ntt_cols_b ? (int)c->ntt_cols_b : ca;
  auto a = [&](int read_src, int final_) {
    if (ca == 8) phase_a<LOGN, 8>(c, ch, inv, read_src, final_);
    else if (ca == 32) phase_a<LOGN, 32>(c, ch, inv, read_src, final_);
    else phase_a<LOGN, 16>(c, ch, inv, read_src, final_);
  };
  auto b = [&](int read_src, int final_) {
    if (cb == 8) phase_b<LOGN, 8>(c, ch, inv, read_src, final_);
    else if (cb == 32) phase_b<LOGN, 32>(c, ch, inv, read_src, final_);
    else phase_b<LOGN, 16>(c, ch, inv, read_src, final_);
  };
  if (!inv) {
    a(1, 0);
    b(0, 1);
  } else {
    b(1, 0);
    a(0, 1);
  }
}

template <int LOGN>
void ntt_dispatch(he_ctx* c, const PolyBatch& pb, bool inv) {
  if constexpr (LOGN == 15) {
    if (c->ntt_single_pass) {
      TraceScope ts(c, inv ? TK_NTT15_INV : TK_NTT15_FWD, 16.0 * (double)valid_polys(pb) * (double)(1u << LOGN));
      dim3 grid(pb.nitems, pb.npoly);
      if (!inv) HE_LAUNCH(ts, (k_ntt15<false>), grid, dim3(1024), c->stream, pb, c->d_tw, c->d_pc);
      else HE_LAUNCH(ts, (k_ntt15<true>), grid, dim3(1024), c->stream, pb, c->d_tw, c->d_pc);
      return;
    }
  }
  if constexpr (LOGN <= 13) {
    constexpr int NT = LOGN >= 12 ? 256 : 128;
    if (!inv) launch_phase<LOGN, 0, LOGN, 1, NT, false>(c, pb, 1, 1);
    else launch_phase<LOGN, 0, LOGN, 1, NT, true>(c, pb, 1, 1);
  } else {
    const size_t poly_bytes = (size_t)8 << LOGN;
    u32 per = pb.npoly;
    if (c->ntt_chunk_mb > 0) {
      per = (u32)(((size_t)c->ntt_chunk_mb << 20) / (poly_bytes * pb.nitems));
      if (per < 1) per = 1;
    }
    for (u32 r0 = 0; r0 < pb.npoly; r0 += per) {
      PolyBatch ch = pb;
      ch.npoly = std::min(per, pb.npoly - r0);
      for (u32 r = 0; r < ch.npoly; ++r) {
        ch.prime[r] = pb.prime[r0 + r];
        ch.row[r] = pb.row[r0 + r];
      }
      ntt_two_phase<LOGN>(c, ch, inv);     // tile widths: knobs ntt_cols, ntt_cols_b
    }
  }
}

}  // namespace

int launch_ntt(he_ctx* c, const PolyBatch& in, bool inverse) {
  // Compact the grid to the rows that are transformed: skipped rows would
  // otherwise occupy workgroup slots that exit at once.
  PolyBatch pb = in;
  u32 n = 0;
  for (u32 r = 0; r < in.npoly; ++r)
    if (in.prime[r] != 0xFF) {
      pb.prime[n] = in.prime[r];
      pb.row[n++] = (uint8_t)r;
    }
  pb.npoly = n;
  if (pb.nitems == 0 || pb.npoly == 0) return HE_OK;
  switch (c->log_n) {
    case 10: ntt_dispatch<10>(c, pb, inverse); break;
    case 11: ntt_dispatch<11>(c, pb, inverse); break;
    case 12: ntt_dispatch<12>(c, pb, inverse); break;
    case 13: ntt_dispatch<13>(c, pb, inverse); break;
    case 14: ntt_dispatch<14>(c, pb, inverse); break;
    case 15: ntt_dispatch<15>(c, pb, inverse); break;
    case 16: ntt_dispatch<16>(c, pb, inverse); break;
    case 17: ntt_dispatch<17>(c, pb, inverse); break;
    default: return HE_EPARAM;
  }
  return hipGetLastError() == hipSuccess ? HE_OK : HE_EDEVICE;
}
