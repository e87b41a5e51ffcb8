// Context set-up, table generation, device uploads and the non-evaluation
// entry points of include/he.h.
#include <cstdio>
#include <cstring>
#include <new>
#include <algorithm>
#include "rns_kernels.hpp"

typedef unsigned __int128 u128;

namespace {

// ---------------------------------------------------------- host number theory
u64 mul_mod(u64 a, u64 b, u64 m) { return (u64)((u128)a * b % m); }
u64 pow_mod(u64 b, u64 e, u64 m) {
  u64 r = 1 % m;
  for (b %= m; e; e >>= 1, b = mul_mod(b, b, m))
    if (e & 1) r = mul_mod(r, b, m);
  return r;
}
u64 inv_mod(u64 a, u64 m) { return pow_mod(a % m, m - 2, m); }   // m prime
u64 shoup_of(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

// Deterministic Miller-Rabin for 64-bit integers (first twelve prime bases).
bool is_prime64(u64 n) {
  if (n < 2) return false;
  static const u64 small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (u64 p : small) {
    if (n % p == 0) return n == p;
  }
  u64 d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  for (u64 a : small) {
    u64 x = pow_mod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool composite = true;
    for (int r = 1; r < s; ++r) {
      x = mul_mod(x, x, n);
      if (x == n - 1) { composite = false; break; }
    }
    if (composite) return false;
  }
  return true;
}

// A primitive 2N-th root of unity mod q: the (q-1)/2N-th power of a quadratic
// non-residue (Euler's criterion) has order exactly 2N since 2N is a power of two.
u64 root_2n(u64 q, u32 N) {
  for (u64 x = 3;; ++x) {
    if (pow_mod(x, (q - 1) / 2, q) != q - 1) continue;
    return pow_mod(x, (q - 1) / (2 * (u64)N), q);
  }
}

u32 bitrev(u32 x, u32 bits) {
  u32 r = 0;
  for (u32 i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

// -q^{-1} mod 2^64 by Newton iteration (each step doubles the correct bits).
u64 neg_inv64(u64 q) {
  u64 x = q;
  for (int i = 0; i < 6; ++i) x *= 2 - q * x;
  return (u64)0 - x;
}

PrimeConst make_pc(u64 q, u32 N) {
  PrimeConst p;
  p.q = q;
  p.qneg = neg_inv64(q);
  p.mu = ~(u64)0 / q;
  p.rmod = (u64)(((u128)1 << 64) % q);
  p.rmod_sh = shoup_of(p.rmod, q);
  p.t28 = (u64)(((u128)1 << 28) % q);
  p.t28_sh = shoup_of(p.t28, q);
  p.t56 = (u64)(((u128)1 << 56) % q);
  p.t56_sh = shoup_of(p.t56, q);
  p.ninv = inv_mod(N, q);
  p.ninv_sh = shoup_of(p.ninv, q);
  p.nq = (u64)0 - q;
  p.nq2 = (u64)0 - 2 * q;
  p.nq4 = (u64)0 - 4 * q;
  return p;
}

template <class T>
int upload(he_ctx* c, T** dptr, const std::vector<T>& h) {
  (void)c;
  HE_HIP(hipMalloc((void**)dptr, h.size() * sizeof(T)));
  HE_HIP(hipMemcpy(*dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return HE_OK;
}

int build_tables(he_ctx* c) {
  const u32 N = c->N, nt = nt_of(c);
  c->h_pc.resize(nt);
  std::vector<u64> tw((size_t)nt * 4 * N);
  for (u32 i = 0; i < nt; ++i) {
    const u64 q = c->primes[i];
    c->h_pc[i] = make_pc(q, N);
    const u64 psi = root_2n(q, N), ipsi = inv_mod(psi, q);
    std::vector<u64> pw(N), ipw(N);
    pw[0] = ipw[0] = 1;
    for (u32 k = 1; k < N; ++k) { pw[k] = mul_mod(pw[k - 1], psi, q); ipw[k] = mul_mod(ipw[k - 1], ipsi, q); }
    c->h_pc[i].w0ni = mul_mod(ipw[N / 2], c->h_pc[i].ninv, q);   // brev(1) = N/2
    c->h_pc[i].w0ni_sh = shoup_of(c->h_pc[i].w0ni, q);
    u64* t = tw.data() + (size_t)i * 4 * N;
    for (u32 k = 0; k < N; ++k) {
      const u32 e = bitrev(k, c->log_n);
      t[2 * k] = pw[e];
      t[2 * k + 1] = shoup_of(pw[e], q);
      t[2 * N + 2 * k] = ipw[e];
      t[2 * N + 2 * k + 1] = shoup_of(ipw[e], q);
    }
  }
  int rc;
  if ((rc = upload(c, &c->d_pc, c->h_pc))) return rc;
  if ((rc = upload(c, &c->d_tw, tw))) return rc;

  // ModUp: for every level l and digit j, D = [j alpha, min((j+1) alpha, l+1)).
  const u32 nq = c->nq, np = c->np, A = c->alpha, dn = c->dnum;
  std::vector<u64> hinv((size_t)nq * dn * A * 2, 0), hmod((size_t)nq * dn * A * nt * 2, 0);
  for (u32 l = 0; l < nq; ++l)
    for (u32 j = 0; j < dn; ++j) {
      const u32 lo = j * A, hi = std::min((j + 1) * A, l + 1);
      for (u32 i = lo; i < hi; ++i) {
        const u64 qi = c->primes[i];
        u64 inv = 1;
        for (u32 i2 = lo; i2 < hi; ++i2)
          if (i2 != i) inv = mul_mod(inv, inv_mod(c->primes[i2] % qi, qi), qi);
        const size_t e = ((size_t)l * dn + j) * A + (i - lo);
        hinv[2 * e] = inv;
        hinv[2 * e + 1] = shoup_of(inv, qi);
        for (u32 t = 0; t < nt; ++t) {
          const u64 m = c->primes[t];
          u64 h = 1 % m;
          for (u32 i2 = lo; i2 < hi; ++i2)
            if (i2 != i) h = mul_mod(h, c->primes[i2] % m, m);
          hmod[2 * (e * nt + t)] = h;                    // (Q_D / q_i) mod p_t and its Shoup companion
          hmod[2 * (e * nt + t) + 1] = shoup_of(h, m);
        }
      }
    }
  if ((rc = upload(c, &c->d_modup_hatinv, hinv))) return rc;
  if ((rc = upload(c, &c->d_modup_hatmod, hmod))) return rc;

  // ModDown.
  // [np][2] (P/p_k)^{-1} mod p_k; [np][nq][2] (P/p_k) mod q_i; [nq][2] P^{-1} mod q_i;
  // [nq][2] P mod q_i (Shoup pairs)
  std::vector<u64> md((size_t)np * 2 + (size_t)np * nq * 2 + (size_t)nq * 4);
  for (u32 k = 0; k < np; ++k) {
    const u64 pk = c->primes[nq + k];
    u64 inv = 1;
    for (u32 k2 = 0; k2 < np; ++k2)
      if (k2 != k) inv = mul_mod(inv, inv_mod(c->primes[nq + k2] % pk, pk), pk);
    md[2 * k] = inv;
    md[2 * k + 1] = shoup_of(inv, pk);
    for (u32 i = 0; i < nq; ++i) {
      const u64 qi = c->primes[i];
      u64 h = 1;
      for (u32 k2 = 0; k2 < np; ++k2)
        if (k2 != k) h = mul_mod(h, c->primes[nq + k2] % qi, qi);
      md[2 * np + 2 * ((size_t)k * nq + i)] = h;
      md[2 * np + 2 * ((size_t)k * nq + i) + 1] = shoup_of(h, qi);
    }
  }
  for (u32 i = 0; i < nq; ++i) {
    const u64 qi = c->primes[i];
    u64 P = 1;
    for (u32 k = 0; k < np; ++k) P = mul_mod(P, c->primes[nq + k] % qi, qi);
    const u64 pinv = inv_mod(P, qi);
    md[2 * np + 2 * (size_t)np * nq + 2 * i] = pinv;
    md[2 * np + 2 * (size_t)np * nq + 2 * i + 1] = shoup_of(pinv, qi);
    md[2 * np + 2 * (size_t)np * nq + 2 * (size_t)nq + 2 * i] = P;
    md[2 * np + 2 * (size_t)np * nq + 2 * (size_t)nq + 2 * i + 1] = shoup_of(P, qi);
  }
  if ((rc = upload(c, &c->d_moddown, md))) return rc;

  // Rescale: q_l^{-1} mod q_i for i < l.
  std::vector<u64> rs((size_t)nq * nq * 2, 0);
  for (u32 l = 1; l < nq; ++l)
    for (u32 i = 0; i < l; ++i) {
      const u64 qi = c->primes[i], inv = inv_mod(c->primes[l] % qi, qi);
      rs[((size_t)l * nq + i) * 2] = inv;
      rs[((size_t)l * nq + i) * 2 + 1] = shoup_of(inv, qi);
    }
  return upload(c, &c->d_rescale, rs);
}

void free_tables(he_ctx* c) {
  for (auto& e : c->tr.pool) hipEventDestroy(e);
  c->tr.pool.clear();
  hipFree(c->d_pc);
  hipFree(c->d_tw);
  hipFree(c->d_modup_hatinv);
  hipFree(c->d_modup_hatmod);
  hipFree(c->d_moddown);
  hipFree(c->d_rescale);
  hipFree(c->d_orbits);
  c->d_orbits = nullptr;
}

// Position map of the NTT-domain automorphism X -> X^g (output position k
// reads input position perm(k)), on the host.
u32 host_galois_perm(u32 k, u32 g, u32 logn) {
  auto brev = [logn](u32 v) {
    u32 r = 0;
    for (u32 i = 0; i < logn; ++i) r |= ((v >> i) & 1u) << (logn - 1 - i);
    return r;
  };
  const u64 two_n = 2ull << logn;
  const u64 e = (2ull * brev(k) + 1) * g % two_n;
  return brev((u32)((e - 1) >> 1));
}

// The blocks of 64 positions in the order of the cycles of the block map P
// of the automorphism g (blocks map to blocks: X reads P(X)), each cycle X,
// P(X), P^2(X), ... in turn; returns whether every cycle has even length.
bool block_orbits(u32 logn, u32 g, std::vector<uint16_t>& out) {
  const u32 npb = (1u << logn) / 64;
  std::vector<u32> P(npb);
  for (u32 b = 0; b < npb; ++b) P[b] = host_galois_perm(b * 64, g, logn) / 64;
  std::vector<char> seen(npb, 0);
  out.clear();
  bool even = true;
  for (u32 b = 0; b < npb; ++b) {
    if (seen[b]) continue;
    size_t len = 0;
    for (u32 x = b; !seen[x]; x = P[x], ++len) {
      seen[x] = 1;
      out.push_back((uint16_t)x);
    }
    even = even && len % 2 == 0;
  }
  return even;
}

PolyBatch one_item(u64* p, u32 npoly, u32 period, u32 first_prime) {
  PolyBatch pb;
  std::memset(&pb, 0, sizeof(pb));
  pb.src[0] = pb.dst[0] = p;
  pb.nitems = 1;
  pb.npoly = npoly;
  for (u32 r = 0; r < npoly; ++r) pb.prime[r] = (uint8_t)(first_prime + r % period);
  return pb;
}

}  // namespace

thread_local char g_last_error[256] = "";

static const char* kTraceNames[TK_COUNT] = {
    "ntt_fwd_phaseA", "ntt_fwd_phaseB", "ntt_inv_phaseB", "ntt_inv_phaseA", "ntt_fwd_onepass", "ntt_inv_onepass",
    "ntt15_fwd", "ntt15_inv", "modup_conv", "ks_inner_steps", "moddown_conv", "ks_final", "ks_final_steps",
    "ks_final_multplain", "ks_final_sum", "ext_multplain", "ks_inner_ext_multplain", "moddown_final", "multplain_accumulate", "multplain", "tensor", "rescale_reduce", "rescale_final", "add",
    "add_plain", "copy_polys", "shoup_companion", "lift_c0", "client_fft", "client_elementwise"};

const char* trace_name(int kind) { return kind >= 0 && kind < TK_COUNT ? kTraceNames[kind] : "?"; }

static bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

TraceScope::TraceScope(he_ctx* ctx, int k, double by) : c(ctx), kind(k), bytes(by) {
  if (!c->tr.on || capturing(c->stream)) return;
  if (c->tr.next + 2 > c->tr.pool.size()) { ++c->tr.dropped; return; }
  a = c->tr.pool[c->tr.next++];
  b = c->tr.pool[c->tr.next++];
}

TraceScope::~TraceScope() {
  if (a) c->tr.recs.push_back({kind, a, b, bytes});
}

static int trace_enable(he_ctx* c, bool on) {
  if (on && c->tr.pool.empty()) {
    c->tr.pool.resize(16384);
    for (auto& e : c->tr.pool) HE_HIP(hipEventCreate(&e));
  }
  c->tr.on = on;
  c->tr.next = 0;
  c->tr.recs.clear();
  c->tr.dropped = 0;
  return HE_OK;
}

void note_hip_error(const char* where, hipError_t e) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", where, hipGetErrorString(e));
}

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* he_last_error(void) { return g_last_error; }

const char* he_strerror(int code) {
  switch (code) {
    case HE_OK: return "ok";
    case HE_EINVAL: return "invalid argument or shape";
    case HE_EPARAM: return "invalid ring parameters";
    case HE_ENOKEY: return "missing evaluation key";
    case HE_ELEVEL: return "level mismatch or rescale at level 0";
    case HE_ESCALE: return "scale mismatch";
    case HE_ENOMEM: return "buffer too small";
    case HE_EDEVICE: return "HIP runtime error";
    case HE_ESTATE: return "context not ready (workspace not bound or keys not loaded)";
    default: return "unknown error";
  }
}

int he_gen_primes(uint32_t log_n, uint32_t bits, uint32_t count, const uint64_t* taken, uint32_t n_taken,
                  uint64_t* out) {
  if (!out || (n_taken && !taken) || bits < 20 || bits > 61 || log_n < 1 || log_n > 17) return HE_EINVAL;
  const u64 two_n = 2ull << log_n;
  u64 c = (1ull << bits) + 1;
  for (u32 got = 0; got < count;) {
    if (c <= two_n) return HE_EPARAM;
    c -= two_n;
    bool used = false;
    for (u32 i = 0; i < n_taken; ++i) used |= taken[i] == c;
    for (u32 i = 0; i < got; ++i) used |= out[i] == c;
    if (!used && is_prime64(c)) out[got++] = c;
  }
  return HE_OK;
}

int he_ctx_create(const he_params* pr, void* stream, he_ctx** out) {
  if (!pr || !out || !pr->q || (pr->n_p && !pr->p)) return HE_EINVAL;
  if (pr->log_n < 10 || pr->log_n > 17) return HE_EPARAM;
  if (pr->n_q < 1 || pr->n_p < 1 || pr->n_q + pr->n_p > HE_MAX_PRIMES) return HE_EPARAM;
  if (pr->alpha < 1 || pr->alpha > pr->n_p || pr->alpha > 8 || pr->n_p > 8) return HE_EPARAM;
  const u32 dnum = (pr->n_q + pr->alpha - 1) / pr->alpha;
  if (dnum > 8 || dnum * (pr->n_q + pr->n_p) > HE_MAX_POLYS) return HE_EPARAM;
  const u64 two_n = 2ull << pr->log_n;
  std::vector<u64> primes(pr->q, pr->q + pr->n_q);
  primes.insert(primes.end(), pr->p, pr->p + pr->n_p);
  for (size_t i = 0; i < primes.size(); ++i) {
    const u64 q = primes[i];
    if (q >= (1ull << 61) || q % two_n != 1 || !is_prime64(q)) return HE_EPARAM;
    for (size_t j = 0; j < i; ++j)
      if (primes[j] == q) return HE_EPARAM;
  }
  he_ctx* c = new (std::nothrow) he_ctx;
  if (!c) return HE_ENOMEM;
  c->log_n = pr->log_n;
  c->N = 1u << pr->log_n;
  c->nq = pr->n_q;
  c->np = pr->n_p;
  c->alpha = pr->alpha;
  c->dnum = dnum;
  c->primes = primes;
  c->stream = (hipStream_t)stream;
  g_last_error[0] = 0;
  int rc = HE_OK;
  {
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) { note_hip_error("hipGetDevice", e); rc = HE_EDEVICE; }
  }
  if (!rc) noalloc_scratch_init(c->device);
  if (!rc) rc = build_tables(c);
  if (rc) {
    free_tables(c);
    delete c;
    return rc;
  }
  *out = c;
  return HE_OK;
}

int he_ctx_destroy(he_ctx* c) {
  if (!c) return HE_EINVAL;
  hipStreamSynchronize(c->stream);
  free_tables(c);
  delete c;
  return HE_OK;
}

int he_ctx_set_stream(he_ctx* c, void* stream) {
  if (!c) return HE_EINVAL;
  c->stream = (hipStream_t)stream;
  return HE_OK;
}

size_t he_ct_bytes(const he_ctx* c, uint32_t level) {
  return c ? (size_t)2 * (level + 1) * c->N * sizeof(u64) : 0;
}

size_t he_key_bytes(const he_ctx* c, uint32_t n_rot) {
  return c ? (size_t)(1 + n_rot) * 2 * c->dnum * 2 * nt_of(c) * c->N * sizeof(u64) : 0;
}

size_t he_dense_bytes_ex(const he_ctx* c, uint32_t level, uint32_t m, int has_bias, uint32_t flags) {
  if (!c) return 0;
  const size_t pl = level + 1 + ((flags & HE_DENSE_QP) ? c->np : 0);
  return (2 * (size_t)m * pl + (has_bias ? level + 1 : 0)) * c->N * sizeof(u64);
}

size_t he_dense_bytes(const he_ctx* c, uint32_t level, uint32_t m, int has_bias) {
  return he_dense_bytes_ex(c, level, m, has_bias, 0);
}

int he_load_keys(he_ctx* c, const uint64_t* relin, uint32_t n_rot, const int32_t* steps, const uint64_t* const* rot,
                 void* key_dev, size_t key_bytes) {
  if (!c || !key_dev || (n_rot && (!steps || !rot))) return HE_EINVAL;
  if (key_bytes < he_key_bytes(c, n_rot)) return HE_ENOMEM;
  for (u32 u = 0; u < n_rot; ++u)
    if (!rot[u]) return HE_EINVAL;
  const size_t words = (size_t)c->dnum * 2 * nt_of(c) * c->N;
  const u32 npoly = c->dnum * 2 * nt_of(c);
  u64* base = (u64*)key_dev;
  c->have_relin = false;
  c->relin_dev = nullptr;
  c->rot.clear();
  auto put = [&](u64* dst, const u64* src) -> int {
    if (hipMemcpyAsync(dst, src, words * sizeof(u64), hipMemcpyHostToDevice, c->stream) != hipSuccess) return HE_EDEVICE;
    PolyBatch pb = one_item(dst, npoly, nt_of(c), 0);
    int rc = launch_ntt(c, pb, false);
    if (rc) return rc;
    // Shoup companions of every key word, limb t over prime t of q_0..q_L, p_0..p_{K-1}
    return launch_shoup_companion(c, c->dnum * 2, nt_of(c), nt_of(c) - 1, dst, dst + words);
  };
  int rc;
  if (relin) {
    if ((rc = put(base, relin))) return rc;
    c->relin_dev = base;
    c->have_relin = true;
  }
  const u64 two_n = 2ull * c->N;
  for (u32 u = 0; u < n_rot; ++u) {
    u64* dst = base + (size_t)(1 + u) * 2 * words;
    if ((rc = put(dst, rot[u]))) return rc;
    const int64_t half = c->N / 2;
    const u64 r = (u64)(((steps[u] % half) + half) % half);
    c->rot.push_back({steps[u], (u32)pow_mod(5, r, two_n), dst});
  }
  // the block-orbit tables of the keys' automorphisms, for the block order
  // of the fused extended sums (a key that starts a run of baby steps)
  if (hipStreamSynchronize(c->stream) != hipSuccess) return HE_EDEVICE;
  hipFree(c->d_orbits);
  c->d_orbits = nullptr;
  const size_t npb = c->N / 64;
  if (npb >= 16 && !c->rot.empty()) {
    std::vector<uint16_t> all(c->rot.size() * npb), one;
    std::vector<char> even(c->rot.size());
    for (size_t u = 0; u < c->rot.size(); ++u) {
      even[u] = block_orbits(c->log_n, c->rot[u].galois, one);
      std::copy(one.begin(), one.end(), all.begin() + u * npb);
    }
    HE_HIP(hipMalloc((void**)&c->d_orbits, all.size() * sizeof(uint16_t)));
    HE_HIP(hipMemcpy(c->d_orbits, all.data(), all.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    for (size_t u = 0; u < c->rot.size(); ++u) {
      c->rot[u].orbit = c->d_orbits + u * npb;
      c->rot[u].orbit_even = even[u] != 0;
    }
  }
  return HE_OK;
}

int he_dense_load_ex(he_ctx* c, uint32_t level, uint32_t m, uint32_t n, uint32_t n1, const uint64_t* pt_diag,
                     const uint64_t* bias, double pt_scale, double bias_scale, uint32_t flags, void* dev, size_t bytes,
                     he_dense** out) {
  const u32 rs_bits = (flags >> HE_DENSE_RS_SHIFT) & 0xFF;
  if (!c || !pt_diag || !dev || !out || (flags & ~(uint32_t)(HE_DENSE_QP | (0xFFu << HE_DENSE_RS_SHIFT))) ||
      rs_bits > HE_DENSE_RS_MAX)
    return HE_EINVAL;
  auto pow2 = [](u32 v) { return v && !(v & (v - 1)); };
  if (level >= c->nq) return HE_ELEVEL;
  if (!pow2(m) || !pow2(n) || !pow2(n1) || n % m || m % n1 || (c->N / 2) % n) return HE_EINVAL;
  if (bytes < he_dense_bytes_ex(c, level, m, bias != nullptr, flags)) return HE_ENOMEM;
  const u32 pl = level + 1 + ((flags & HE_DENSE_QP) ? c->np : 0);
  const size_t limb = c->N, per = (size_t)pl * limb;
  u64* d = (u64*)dev;
  if (hipMemcpyAsync(d, pt_diag, (size_t)m * per * sizeof(u64), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return HE_EDEVICE;
  for (u32 k0 = 0; k0 < m; k0 += HE_MAXB) {
    PolyBatch pb;
    std::memset(&pb, 0, sizeof(pb));
    pb.nitems = std::min<u32>(HE_MAXB, m - k0);
    pb.npoly = pl;
    for (u32 b = 0; b < pb.nitems; ++b) pb.src[b] = pb.dst[b] = d + (size_t)(k0 + b) * per;
    for (u32 r = 0; r < pl; ++r) pb.prime[r] = (uint8_t)ext_prime(c, level, r);
    int rc = launch_ntt(c, pb, false);
    if (rc) return rc;
  }
  int rc = launch_shoup_companion(c, m, pl, level, d, d + (size_t)m * per);
  if (rc) return rc;
  u64* db = nullptr;
  if (bias) {
    db = d + (size_t)2 * m * per;
    const size_t bper = (size_t)(level + 1) * limb;
    if (hipMemcpyAsync(db, bias, bper * sizeof(u64), hipMemcpyHostToDevice, c->stream) != hipSuccess) return HE_EDEVICE;
    PolyBatch pb = one_item(db, level + 1, level + 1, 0);
    int rc = launch_ntt(c, pb, false);
    if (rc) return rc;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return HE_EDEVICE;
  he_dense* h = new (std::nothrow) he_dense;
  if (!h) return HE_ENOMEM;
  *h = he_dense{c, level, m, n, n1, m / n1, pt_scale, bias_scale, pl, rs_bits, d, db};
  *out = h;
  return HE_OK;
}

int he_dense_load(he_ctx* c, uint32_t level, uint32_t m, uint32_t n, uint32_t n1, const uint64_t* pt_diag,
                  const uint64_t* bias, double pt_scale, double bias_scale, void* dev, size_t bytes, he_dense** out) {
  return he_dense_load_ex(c, level, m, n, n1, pt_diag, bias, pt_scale, bias_scale, 0, dev, bytes, out);
}

size_t he_linear_bytes(const he_ctx* c, uint32_t level, uint32_t n_out, uint32_t n_giant, uint32_t n_in,
                       uint32_t n_baby) {
  return c ? 2 * (size_t)n_out * n_giant * n_in * n_baby * (level + 1) * c->N * sizeof(u64) : 0;
}

int he_linear_load(he_ctx* c, uint32_t level, uint32_t n_out, uint32_t n_giant, uint32_t n_in, uint32_t n_baby,
                   const int32_t* baby, const int32_t* giant, const uint64_t* pts, double pt_scale, void* dev,
                   size_t bytes, he_linear** out) {
  if (!c || !baby || !giant || !pts || !dev || !out) return HE_EINVAL;
  if (level >= c->nq) return HE_ELEVEL;
  if (!n_out || !n_giant || !n_in || !n_baby || n_giant > 64 || n_baby > 64 || n_in * n_baby > HE_MAXB ||
      giant[0] != 0)
    return HE_EINVAL;
  if (bytes < he_linear_bytes(c, level, n_out, n_giant, n_in, n_baby)) return HE_ENOMEM;
  const size_t m = (size_t)n_out * n_giant * n_in * n_baby, per = (size_t)(level + 1) * c->N;
  u64* d = (u64*)dev;
  if (hipMemcpyAsync(d, pts, m * per * sizeof(u64), hipMemcpyHostToDevice, c->stream) != hipSuccess) return HE_EDEVICE;
  for (size_t k0 = 0; k0 < m; k0 += HE_MAXB) {
    PolyBatch pb;
    std::memset(&pb, 0, sizeof(pb));
    pb.nitems = (u32)std::min<size_t>(HE_MAXB, m - k0);
    pb.npoly = level + 1;
    for (u32 b = 0; b < pb.nitems; ++b) pb.src[b] = pb.dst[b] = d + (k0 + b) * per;
    for (u32 r = 0; r <= level; ++r) pb.prime[r] = (uint8_t)r;
    int rc = launch_ntt(c, pb, false);
    if (rc) return rc;
  }
  int rc = launch_shoup_companion(c, (u32)m, level + 1, level, d, d + m * per);
  if (rc) return rc;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return HE_EDEVICE;
  he_linear* h = new (std::nothrow) he_linear;
  if (!h) return HE_ENOMEM;
  h->ctx = c;
  h->level = level;
  h->n_out = n_out;
  h->n_giant = n_giant;
  h->n_in = n_in;
  h->n_baby = n_baby;
  h->pt_scale = pt_scale;
  for (u32 b = 0; b < n_baby; ++b) h->baby[b] = baby[b];
  for (u32 g = 0; g < n_giant; ++g) h->giant[g] = giant[g];
  h->pts = d;
  *out = h;
  return HE_OK;
}

int he_linear_free(he_linear* t) {
  if (!t) return HE_EINVAL;
  delete t;
  return HE_OK;
}

int he_dense_free(he_dense* d) {
  if (!d) return HE_EINVAL;
  delete d;
  return HE_OK;
}

int he_ct_from_coeff_dev(he_ctx* c, const uint64_t* coeff, uint32_t level, double scale, he_ct* ct) {
  if (!c || !coeff || !ct || !ct->dev) return HE_EINVAL;
  if (level >= c->nq) return HE_ELEVEL;
  PolyBatch pb = one_item(ct->dev, 2 * (level + 1), level + 1, 0);
  pb.src[0] = (u64*)coeff;
  int rc = launch_ntt(c, pb, false);
  if (rc) return rc;
  ct->level = level;
  ct->scale = scale;
  return HE_OK;
}

int he_ct_to_coeff_dev(he_ctx* c, const he_ct* ct, uint64_t* coeff) {
  if (!c || !coeff || !ct || !ct->dev) return HE_EINVAL;
  if (ct->level >= c->nq) return HE_ELEVEL;
  PolyBatch pb = one_item(coeff, 2 * (ct->level + 1), ct->level + 1, 0);
  pb.src[0] = ct->dev;
  return launch_ntt(c, pb, true);
}

int he_ct_import(he_ctx* c, const uint64_t* host, uint32_t level, double scale, he_ct* ct) {
  if (!c || !host || !ct || !ct->dev) return HE_EINVAL;
  if (level >= c->nq) return HE_ELEVEL;
  if (hipMemcpyAsync(ct->dev, host, he_ct_bytes(c, level), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return HE_EDEVICE;
  int rc = he_ct_from_coeff_dev(c, ct->dev, level, scale, ct);
  if (rc) return rc;
  return hipStreamSynchronize(c->stream) == hipSuccess ? HE_OK : HE_EDEVICE;
}

int he_ct_export(he_ctx* c, const he_ct* ct, uint64_t* host) {
  if (!c || !host || !ct || !ct->dev) return HE_EINVAL;
  if (!c->ws) return HE_ESTATE;
  if (ct->level >= c->nq) return HE_ELEVEL;
  u64* tmp = (u64*)c->ws;   // the first region of the workspace is at least one ciphertext
  int rc = he_ct_to_coeff_dev(c, ct, tmp);
  if (rc) return rc;
  if (hipMemcpyAsync(host, tmp, he_ct_bytes(c, ct->level), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return HE_EDEVICE;
  return hipStreamSynchronize(c->stream) == hipSuccess ? HE_OK : HE_EDEVICE;
}

int he_ntt(he_ctx* c, uint32_t n_items, uint64_t* const* items, uint32_t first_prime, uint32_t limbs, int inverse) {
  if (!c || !items || n_items > HE_MAXB || limbs == 0 || limbs > HE_MAX_POLYS) return HE_EINVAL;
  if (first_prime + limbs > nt_of(c)) return HE_EINVAL;
  PolyBatch pb;
  std::memset(&pb, 0, sizeof(pb));
  pb.nitems = n_items;
  pb.npoly = limbs;
  for (u32 b = 0; b < n_items; ++b) {
    if (!items[b]) return HE_EINVAL;
    pb.src[b] = pb.dst[b] = items[b];
  }
  for (u32 r = 0; r < limbs; ++r) pb.prime[r] = (uint8_t)(first_prime + r);
  return launch_ntt(c, pb, inverse != 0);
}

int he_ctx_set_knob(he_ctx* c, const char* key, int64_t value) {
  if (!c || !key || value < 0) return HE_EINVAL;
  if (!std::strcmp(key, "ntt_chunk_mb")) { c->ntt_chunk_mb = value; return HE_OK; }
  if (!std::strcmp(key, "ntt_cols")) {
    if (value != 8 && value != 16 && value != 32) return HE_EINVAL;
    c->ntt_cols = value;
    return HE_OK;
  }
  if (!std::strcmp(key, "ntt_cols_b")) {
    if (value != 0 && value != 8 && value != 16 && value != 32) return HE_EINVAL;
    c->ntt_cols_b = value;
    return HE_OK;
  }
  if (!std::strcmp(key, "ntt_single_pass")) {
    if (value > 1) return HE_EINVAL;
    c->ntt_single_pass = value;
    return HE_OK;
  }
  if (!std::strcmp(key, "ks_fuse")) {
    if (value > 1) return HE_EINVAL;
    c->ks_fuse = value;
    return HE_OK;
  }
  if (!std::strcmp(key, "ks_fuse_g")) {
    if (value > 1) return HE_EINVAL;
    c->ks_fuse_g = value;
    return HE_OK;
  }
  if (!std::strcmp(key, "ks_fuse_waves")) {
    if (value != 0 && value != 3) return HE_EINVAL;
    c->ks_fuse_waves = value;
    return HE_OK;
  }
  if (!std::strcmp(key, "ks_fuse_min_batch")) {
    if (value < 1 || value > HE_MAXB) return HE_EINVAL;
    c->ks_fuse_min_batch = value;
    return HE_OK;
  }
  if (!std::strcmp(key, "ks_fuse_pair")) {
    if (value > 1) return HE_EINVAL;
    c->ks_fuse_pair = value;
    return HE_OK;
  }
  if (!std::strcmp(key, "ks_fuse_orbit")) {
    if (value > 1) return HE_EINVAL;
    c->ks_fuse_orbit = value;
    return HE_OK;
  }
  if (!std::strcmp(key, "ks_fuse_one")) {
    if (value > 1) return HE_EINVAL;
    c->ks_fuse_one = value;
    return HE_OK;
  }
  if (!std::strcmp(key, "ks_fuse_lds")) {
    if (value != 0 && value != 4 && value != 8 && value != 16) return HE_EINVAL;
    c->ks_fuse_lds = value;
    return HE_OK;
  }
  if (!std::strcmp(key, "trace")) {
    if (value > 1) return HE_EINVAL;
    return trace_enable(c, value == 1);
  }
  return HE_EINVAL;
}

int he_trace_read(he_ctx* c, he_trace_entry* out, uint32_t capacity, uint32_t* count) {
  if (!c || !count || (capacity && !out)) return HE_EINVAL;
  HE_HIP(hipStreamSynchronize(c->stream));
  uint64_t n[TK_COUNT] = {0};
  double ms[TK_COUNT] = {0}, by[TK_COUNT] = {0};
  for (const TraceRec& r : c->tr.recs) {
    float t = 0;
    HE_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ++n[r.kind];
    ms[r.kind] += t;
    by[r.kind] += r.bytes;
  }
  uint32_t k = 0;
  for (int i = 0; i < TK_COUNT; ++i) {
    if (!n[i]) continue;
    if (k < capacity) out[k] = he_trace_entry{trace_name(i), n[i], ms[i], by[i]};
    ++k;
  }
  *count = k;
  c->tr.next = 0;
  c->tr.recs.clear();
  return c->tr.dropped ? HE_ENOMEM : HE_OK;
}

int he_ctx_get_knob(const he_ctx* c, const char* key, int64_t* value) {
  if (!c || !key || !value) return HE_EINVAL;
  if (!std::strcmp(key, "ntt_chunk_mb")) { *value = c->ntt_chunk_mb; return HE_OK; }
  if (!std::strcmp(key, "ntt_cols")) { *value = c->ntt_cols; return HE_OK; }
  if (!std::strcmp(key, "ntt_cols_b")) { *value = c->ntt_cols_b; return HE_OK; }
  if (!std::strcmp(key, "ntt_single_pass")) { *value = c->ntt_single_pass; return HE_OK; }
  if (!std::strcmp(key, "ks_fuse")) { *value = c->ks_fuse; return HE_OK; }
  if (!std::strcmp(key, "ks_fuse_g")) { *value = c->ks_fuse_g; return HE_OK; }
  if (!std::strcmp(key, "ks_fuse_waves")) { *value = c->ks_fuse_waves; return HE_OK; }
  if (!std::strcmp(key, "ks_fuse_lds")) { *value = c->ks_fuse_lds; return HE_OK; }
  if (!std::strcmp(key, "ks_fuse_min_batch")) { *value = c->ks_fuse_min_batch; return HE_OK; }
  if (!std::strcmp(key, "ks_fuse_pair")) { *value = c->ks_fuse_pair; return HE_OK; }
  if (!std::strcmp(key, "ks_fuse_orbit")) { *value = c->ks_fuse_orbit; return HE_OK; }
  if (!std::strcmp(key, "ks_fuse_one")) { *value = c->ks_fuse_one; return HE_OK; }
  if (!std::strcmp(key, "trace")) { *value = c->tr.on ? 1 : 0; return HE_OK; }
  return HE_EINVAL;
}

struct he_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int he_graph_begin(he_ctx* c) {
  if (!c) return HE_EINVAL;
  if (!c->stream) return HE_ESTATE;
  return hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) == hipSuccess ? HE_OK : HE_EDEVICE;
}

int he_graph_end(he_ctx* c, he_graph** out) {
  if (!c || !out) return HE_EINVAL;
  *out = nullptr;
  if (!c->stream) return HE_ESTATE;
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(c->stream, &g) != hipSuccess || !g) {
    if (g) hipGraphDestroy(g);
    (void)hipGetLastError();
    return HE_EDEVICE;
  }
  hipGraphExec_t e = nullptr;
  if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(g);
    (void)hipGetLastError();
    return HE_EDEVICE;
  }
  *out = new he_graph{g, e};
  return HE_OK;
}

int he_graph_launch(he_ctx* c, const he_graph* g) {
  if (!c || !g) return HE_EINVAL;
  return hipGraphLaunch(g->exec, c->stream) == hipSuccess ? HE_OK : HE_EDEVICE;
}

int he_graph_free(he_graph* g) {
  if (!g) return HE_EINVAL;
  hipGraphExecDestroy(g->exec);
  hipGraphDestroy(g->graph);
  delete g;
  return HE_OK;
}

int he_sync(he_ctx* c) {
  if (!c) return HE_EINVAL;
  return hipStreamSynchronize(c->stream) == hipSuccess ? HE_OK : HE_EDEVICE;
}

}  // extern "C"
