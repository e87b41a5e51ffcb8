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

  template <int U, int RB>
  __device__ static __forceinline__ void pass(u64* lds, const ulonglong2* __restrict__ tw, const PrimeConst& k,
                                              u32 sub0) {
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
      for (int m = 0; m < R; ++m) x[m] = lds[pidx(local(col, kt * (R * KL) + m * KL + kl))];
      const u64 q4 = 4 * q;
      if (!INV) {
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
              const u64 X = csub_neg(x[m0], k.nq4);                      // < 4q
              const u64 S = add_shoup4(X, x[m1], wp.x, wp.y, k.nq);      // X + T < 8q
              x[m0] = S;
              x[m1] = 2 * X + q4 - S;                                   // X + 4q - T in (0, 8q)
            }
          }
        }
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
              x[m0] = csub_neg(A + B, k.nq4);                            // < 4q
              x[m1] = shoup_lazy4(A + q4 - B, wp.x, wp.y, q);            // < 4q
            }
          }
        }
      }
#pragma unroll
      for (int m = 0; m < R; ++m) lds[pidx(local(col, kt * (R * KL) + m * KL + kl))] = x[m];
    }
  }

  template <int P>
  __device__ static __forceinline__ void passes_fwd(u64* lds, const ulonglong2* tw, const PrimeConst& k, u32 sub0) {
    if constexpr (P < npasses(LP)) {
      pass<pass_start(LP, P), pass_bits(LP, P)>(lds, tw, k, sub0);
      __syncthreads();
      passes_fwd<P + 1>(lds, tw, k, sub0);
    }
  }
  template <int P>
  __device__ static __forceinline__ void passes_inv(u64* lds, const ulonglong2* tw, const PrimeConst& k, u32 sub0) {
    if constexpr (P >= 0) {
      pass<pass_start(LP, P), pass_bits(LP, P)>(lds, tw, k, sub0);
      __syncthreads();
      passes_inv<P - 1>(lds, tw, k, sub0);
    }
  }
};

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
  if (pr == 0xFF) return;
  const u32 N = 1u << LOGN;
  const PrimeConst k = pc[pr];
  const u64 q = k.q;
  const ulonglong2* tw = (const ulonglong2*)(tw_all + (size_t)pr * 4 * N + (INV ? 2 * N : 0));
  const u64* src = read_src ? pb.src[b] + (size_t)(pb.src_off + r) * N : pb.dst[b] + (size_t)(pb.dst_off + r) * N;
  u64* dst = pb.dst[b] + (size_t)(pb.dst_off + r) * N;
  const u32 sub0 = tile * COLS;
  // Tile copy in 16-byte pairs (COLS and 2^LP are even, so pairs never straddle a row).
  for (u32 i = 2 * threadIdx.x; i < (u32)TILE; i += 2 * NT) {
    const ulonglong2 v = *(const ulonglong2*)(src + Ph::gaddr(sub0, i));
    lds[pidx(i)] = v.x;
    lds[pidx(i + 1)] = v.y;
  }
  __syncthreads();
  if (!INV) Ph::template passes_fwd<0>(lds, tw, k, sub0);
  else Ph::template passes_inv<npasses(LP) - 1>(lds, tw, k, sub0);
  ulonglong2 v;
  if (final_) {
    if (!INV) {
      for (u32 i = 2 * threadIdx.x; i < (u32)TILE; i += 2 * NT) {
        v.x = csub_neg(csub_neg(csub_neg(lds[pidx(i)], k.nq4), k.nq2), k.nq);
        v.y = csub_neg(csub_neg(csub_neg(lds[pidx(i + 1)], k.nq4), k.nq2), k.nq);
        *(ulonglong2*)(dst + Ph::gaddr(sub0, i)) = v;
      }
    } else {
      for (u32 i = 2 * threadIdx.x; i < (u32)TILE; i += 2 * NT) {
        v.x = csub_neg(csub_neg(shoup_lazy4(lds[pidx(i)], k.ninv, k.ninv_sh, q), k.nq2), k.nq);
        v.y = csub_neg(csub_neg(shoup_lazy4(lds[pidx(i + 1)], k.ninv, k.ninv_sh, q), k.nq2), k.nq);
        *(ulonglong2*)(dst + Ph::gaddr(sub0, i)) = v;
      }
    }
  } else {
    for (u32 i = 2 * threadIdx.x; i < (u32)TILE; i += 2 * NT) {
      v.x = lds[pidx(i)];
      v.y = lds[pidx(i + 1)];
      *(ulonglong2*)(dst + Ph::gaddr(sub0, i)) = v;
    }
  }
}

template <int LOGN, int S0, int LP, int COLS, int NT, bool INV>
void launch_phase(he_ctx* c, const PolyBatch& pb, int read_src, int final_) {
  dim3 grid((1u << (LOGN - LP)) / COLS, pb.nitems, pb.npoly);
  hipLaunchKernelGGL((k_ntt_phase<LOGN, S0, LP, COLS, NT, INV>), grid, dim3(NT), 0, c->stream, pb, c->d_tw, c->d_pc,
                     read_src, final_);
}

// Single phase for logN <= 13, two phases (LA = ceil(logN/2)) above.  With
// the knob ntt_chunk_mb > 0 the two-phase transform runs phase A then phase B
// on chunks of that many MiB of polynomials, so that the intermediate written
// by phase A can still be in the Infinity Cache when phase B reads it back.

template <int LOGN, int COLS>
void ntt_two_phase(he_ctx* c, const PolyBatch& ch, bool inv) {
  constexpr int LA = (LOGN + 1) / 2, LB = LOGN - LA;
  constexpr int NTA = ((COLS << LA) / 16) > 512 ? 512 : ((COLS << LA) / 16);
  constexpr int NTB = ((COLS << LB) / 16) > 512 ? 512 : ((COLS << LB) / 16);
  if (!inv) {
    launch_phase<LOGN, 0, LA, COLS, NTA, false>(c, ch, 1, 0);
    launch_phase<LOGN, LA, LB, COLS, NTB, false>(c, ch, 0, 1);
  } else {
    launch_phase<LOGN, LA, LB, COLS, NTB, true>(c, ch, 1, 0);
    launch_phase<LOGN, 0, LA, COLS, NTA, true>(c, ch, 0, 1);
  }
}

template <int LOGN>
void ntt_dispatch(he_ctx* c, const PolyBatch& pb, bool inv) {
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
      ch.src_off = pb.src_off + r0;
      ch.dst_off = pb.dst_off + r0;
      for (u32 r = 0; r < ch.npoly; ++r) ch.prime[r] = pb.prime[r0 + r];
      // tile width: sub-transforms per workgroup (knob ntt_cols)
      if (c->ntt_cols == 8) ntt_two_phase<LOGN, 8>(c, ch, inv);
      else if (c->ntt_cols == 32) ntt_two_phase<LOGN, 32>(c, ch, inv);
      else ntt_two_phase<LOGN, 16>(c, ch, inv);
    }
  }
}

}  // namespace

int launch_ntt(he_ctx* c, const PolyBatch& pb, bool inverse) {
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
