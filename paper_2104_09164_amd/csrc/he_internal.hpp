// Internal structures of the HIP library behind include/he.h.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>
#include <map>
#include <vector>
#include "../../include/he.h"

typedef uint64_t u64;
typedef uint32_t u32;

#define HE_MAXB HE_MAX_BATCH
#define HE_MAXP HE_MAX_PRIMES
#define HE_MAX_POLYS 256      // limb-polys per item in one transform launch

// Per-prime constants, device resident (one array indexed by prime number:
// 0..L for q_i, L+1..L+K for p_k).
struct PrimeConst {
  u64 q;
  u64 qneg;        // -q^{-1} mod 2^64 (Montgomery)
  u64 mu;          // floor(2^64 / q) (Barrett-style reduce64)
  u64 ninv, ninv_sh;   // N^{-1} mod q and its Shoup companion
  u64 w0ni, w0ni_sh;   // inverse stage-0 twiddle psi^{-N/2} times N^{-1}, and its companion
  u64 rmod, rmod_sh;   // 2^64 mod q and its Shoup companion (to Montgomery form)
  u64 nq, nq2, nq4;    // 2^64 - q, 2^64 - 2q, 2^64 - 4q
  u64 t28, t28_sh;     // 2^28 mod q and its Shoup companion (28-bit column sums)
  u64 t56, t56_sh;     // 2^56 mod q and its Shoup companion
};

// Twiddle tables of prime i at tw + i * 4N, as (w, Shoup companion) pairs:
//   [0,2N)   (psi^brev(k), ...)   forward Cooley-Tukey twiddles (bit-reversed)
//   [2N,4N)  (psi^-brev(k), ...)  inverse Gentleman-Sande twiddles
// Forward output order: position k holds the evaluation at psi^(2 brev(k) + 1).

// A batch of limb-poly transforms: item b, poly r (0 <= r < npoly) reads
// src[b] + (src_off + r) * N and writes dst[b] + (dst_off + r) * N with prime
// prime[r]; prime[r] == 0xFF skips the poly.
struct PolyBatch {
  u64* src[HE_MAXB];
  u64* dst[HE_MAXB];
  u32 src_off, dst_off, npoly, nitems;
  uint8_t prime[HE_MAX_POLYS];   // prime index of poly row r; 0xFF = skip the row
  uint8_t row[HE_MAX_POLYS];     // NTT launches only: grid row -> poly row (rows compacted)
  size_t stride = 0;             // NTT launches: when nonzero, item b is at src[0] + b * stride and
  size_t dst_stride = 0;         // dst[0] + b * (dst_stride ? dst_stride : stride) (any number of
                                 // items; the pointer lists are then unused beyond [0])
};

// Kernel classes of the tracer (he_trace_read aggregates per class).
enum TraceKind {
  TK_NTT_FWD_A, TK_NTT_FWD_B, TK_NTT_INV_B, TK_NTT_INV_A, TK_NTT_ONE_FWD, TK_NTT_ONE_INV, TK_NTT15_FWD, TK_NTT15_INV,
  TK_MODUP_CONV, TK_KS_INNER_STEPS, TK_MODDOWN_CONV, TK_KS_FINAL, TK_KS_FINAL_STEPS, TK_KS_FINAL_MP, TK_KS_FINAL_SUM,
  TK_EXT_MP, TK_KS_EXT_FUSED, TK_MODDOWN_FINAL, TK_MP_ACC, TK_MULTPLAIN, TK_TENSOR, TK_RESCALE_REDUCE, TK_RESCALE_FINAL, TK_ADD, TK_ADD_PLAIN, TK_COPY, TK_SHOUP_COMPANION, TK_LIFT_C0,
  TK_CLIENT_FFT, TK_CLIENT_ELEM,
  TK_COUNT
};
const char* trace_name(int kind);

struct TraceRec {
  int kind;
  hipEvent_t a, b;
  double bytes;
};

struct Tracer {
  bool on = false;
  std::vector<hipEvent_t> pool;   // created when tracing is switched on
  size_t next = 0;
  std::vector<TraceRec> recs;
  uint64_t dropped = 0;           // launches not recorded (pool exhausted)
};

struct KeySlot {
  int32_t step;
  u32 galois;
  u64* dev;         // [dnum][2][L+1+K][N] NTT form, then their Shoup companions (same shape)
  // The N/64 blocks of 64 positions in the order of the cycles of P, the
  // block map of this key's automorphism (block X reads block P(X)): each
  // cycle X, P(X), P^2(X), ... in turn (device memory).  orbit_even: every
  // cycle has even length, so that entries 2k, 2k + 1 are a pair (X, P(X)).
  const uint16_t* orbit = nullptr;
  bool orbit_even = false;
};

struct he_ctx {
  u32 log_n, N;
  u32 nq, np, alpha, dnum;   // L+1, K
  std::vector<u64> primes;    // q_0..q_L, p_0..p_{K-1}
  hipStream_t stream = nullptr;
  int device = 0;

  // device tables (library-owned)
  PrimeConst* d_pc = nullptr;
  u64* d_tw = nullptr;
  // ModUp conversion: for level l, digit j, source i (< alpha), target prime t:
  //   hatinv[l][j][i] (+ shoup): (Q_D / q_i)^{-1} mod q_i
  //   hatmod[l][j][i][t]: ((Q_D / q_i) mod t) * 2^64 mod t (Montgomery form)
  u64* d_modup_hatinv = nullptr;   // [nq][dnum][alpha][2]
  u64* d_modup_hatmod = nullptr;   // [nq][dnum][alpha][nt]
  // ModDown: phatinv[k] (+shoup) = (P/p_k)^{-1} mod p_k; phatmod[k][i] = ((P/p_k) mod q_i) 2^64 mod q_i;
  // pinv[i] (+shoup) = P^{-1} mod q_i
  u64* d_moddown = nullptr;        // [np][2] | [np][nq] | [nq][2]
  // Rescale: qlinv[l][i] (+shoup) = q_l^{-1} mod q_i, i < l
  u64* d_rescale = nullptr;        // [nq][nq][2]
  uint16_t* d_orbits = nullptr;    // block-orbit tables of the rotation keys (KeySlot::orbit)
  std::vector<PrimeConst> h_pc;

  // execution knobs (bit-preserving)
  int64_t ntt_chunk_mb = 0;
  int64_t ntt_cols = 16;      // sub-transforms per NTT workgroup tile: 8, 16 or 32
  int64_t ntt_cols_b = 0;     // the same for the row phase (0 = ntt_cols)
  int64_t ntt_single_pass = 0;
  int64_t ks_fuse = 1;          // lazy-ModDown baby steps: inner product fused into the inner sums
  int64_t ks_fuse_g = 0;        // fused extended sums: 1 = half the items per thread
  int64_t ks_fuse_waves = 0;    // fused extended sums: 3 = compiled for 3 waves per SIMD
  int64_t ks_fuse_min_batch = 3;  // fused extended sums: smallest batch that takes the LDS-shared form
  int64_t ks_fuse_pair = 0;       // LDS-shared form: pairs of blocks along the automorphism per workgroup
  int64_t ks_fuse_orbit = 1;      // LDS-shared form: blocks dealt to each XCD along the automorphism's cycles
  int64_t ks_fuse_one = 1;        // a batch of one: its own kernel (values-only streams below 2^50)
  int64_t ks_fuse_lds = 8;      // fused extended sums: 4, 8 or 16 = LDS-shared form with that many requests per
                                // workgroup (8 measured fastest), 0 = the register form

  Tracer tr;

  // workspace
  uint8_t* ws = nullptr;
  size_t ws_bytes = 0;
  u32 ws_batch = 0, ws_n1 = 0, ws_n2 = 0;

  // keys
  bool have_relin = false;
  u64* relin_dev = nullptr;
  std::vector<KeySlot> rot;
};

struct he_dense {
  he_ctx* ctx;
  u32 level, m, n, n1, n2;
  double pt_scale, bias_scale;
  u32 pl;      // limbs per diagonal: level+1, or level+1+K over Q_l u P (lazy-ModDown evaluation)
  u32 rs_bits; // rotate-and-sum: 0 sequential, else hoisted groups of this many bits
  u64* pts;    // [m][pl][N], NTT form, then their Shoup companions floor(w 2^64 / q), same shape
  u64* bias;   // [level+1][N], NTT form, or null
};

struct he_linear {
  he_ctx* ctx;
  u32 level, n_out, n_giant, n_in, n_baby;
  double pt_scale;
  int32_t baby[64], giant[64];   // rotation amounts (giant[0] = 0)
  u64* pts;    // [n_giant][n_out][n_in][n_baby][level+1][N], NTT form, then their Shoup companions
};

// ---------------------------------------------------------------- helpers
static inline u32 nt_of(const he_ctx* c) { return c->nq + c->np; }
static inline size_t limb_bytes(const he_ctx* c) { return (size_t)c->N * sizeof(u64); }
// prime index of extended limb t in basis q_0..q_l, p_0..p_{K-1}
static inline u32 ext_prime(const he_ctx* c, u32 l, u32 t) { return t <= l ? t : c->nq + (t - l - 1); }
static inline u32 digits_at(const he_ctx* c, u32 l) { return (l + 1 + c->alpha - 1) / c->alpha; }

// Records a HIP failure (call site + error string) for he_last_error().
void note_hip_error(const char* where, hipError_t e);
#define HE_HIP(call)                                    \
  do {                                                  \
    hipError_t he_e_ = (call);                          \
    if (he_e_ != hipSuccess) {                          \
      note_hip_error(#call, he_e_);                     \
      return HE_EDEVICE;                                \
    }                                                   \
  } while (0)

// Brackets one kernel launch with HIP events on the context stream while
// tracing is on (and the stream is not being captured into a graph);
// `bytes` = algorithmic bytes of the launch (each word read or written once).
// With the tracer on (and the stream not capturing), a scope owns two pool
// events that the launch inside it carries in its dispatch packet
// (hipExtLaunchKernelGGL): they are stamped when the kernel starts and ends,
// so the traced time is the kernel's own execution time.
struct TraceScope {
  he_ctx* c;
  int kind;
  double bytes;
  hipEvent_t a = nullptr, b = nullptr;
  TraceScope(he_ctx* ctx, int k, double b);
  ~TraceScope();
};

// Launch on `stream`, carrying the scope's events when it has them.
#define HE_LAUNCH(ts, kernel, grid, block, stream, ...)                                              \
  do {                                                                                              \
    if ((ts).a)                                                                                     \
      hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, (ts).a, (ts).b, 0, __VA_ARGS__);        \
    else                                                                                            \
      hipLaunchKernelGGL(kernel, grid, block, 0, stream, __VA_ARGS__);                              \
  } while (0)

// Looks up the calling GPU's copy of the no-allocation scratch array (ops.hip);
// called by he_ctx_create with that GPU current.
void noalloc_scratch_init(int device);

// kernel launchers (ntt.hip)
int launch_ntt(he_ctx* c, const PolyBatch& pb, bool inverse);
// kernel launchers (rns_kernels.hip) are declared in rns_kernels.hpp
