// Evaluation entry points of include/he.h: rotation (hybrid key switching,
// hoisted), square with relinearisation, rescale, add and the dense layer in
// baby-step/giant-step form.  Host code only: every step below is one or more
// kernel launches on the context stream; nothing is computed on the CPU.
#include <cmath>
#include <cstring>
#include <mutex>
#include "rns_kernels.hpp"

// Scratch of the no-allocation rescale (he_rescale_batch_noalloc): one array
// per GPU, held until the process ends.  Host code never passes `scratch`
// itself to a kernel or a copy (in host code the name is a host-side stand-in);
// it uses the device address hipGetSymbolAddress returned for that GPU.
static __device__ __align__(256) uint64_t scratch[HE_NOALLOC_SCRATCH_BYTES / sizeof(uint64_t)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices];    // device address of `scratch` per GPU
int g_noalloc_rc[kMaxDevices];       // HE_OK, or the error its look-up returned
bool g_noalloc_done[kMaxDevices];
}  // namespace

// Called by he_ctx_create with `device` current: looks up that GPU's copy of
// `scratch` once.
void noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_done[device]) return;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) {
    note_hip_error("hipGetSymbolAddress(scratch)", e);
    g_noalloc_rc[device] = HE_EDEVICE;
  } else {
    g_noalloc_ptr[device] = p;
    g_noalloc_rc[device] = HE_OK;
  }
  g_noalloc_done[device] = true;
}

namespace {

// Workspace regions for a batch of up to B ciphertexts (sizes in limb-polys,
// computed at the top level L so that the layout does not depend on the level).
struct WS {
  u64 *rtmp, *coef, *ext, *u, *conv, *d01, *d2, *red, *giant, *z0, *z1;
};

// Rotation steps per step-batched key switch: the baby steps of the widest
// layer (hoisted, sharing one ModUp) or its giant steps (one ModUp each).
u32 ks_group(u32 n1) { return n1 > 2 ? std::min<u32>(n1 - 1, HE_MAX_STEPS) : 1; }
u32 giant_group(u32 n2) { return n2 > 2 ? std::min<u32>(n2 - 1, HE_MAX_STEPS) : 1; }

size_t ws_words(const he_ctx* c, u32 B, u32 n1, u32 n2, WS* w) {
  const size_t N = c->N, L1 = c->nq, E = c->nq + c->np;
  const size_t csz = 2 * L1 * N;
  size_t off = 0;
  auto take = [&](u64** p, size_t words) {
    if (w) *p = (u64*)(c->ws) + off;
    off += (words + 31) & ~(size_t)31;   // keep 256-byte alignment
  };
  WS dummy;
  WS& x = w ? *w : dummy;
  // coef and ext hold the ModUp of every giant step (GJ steps of B items);
  // u and conv every step of one step-batched key switch.  The n2 B
  // lazy-ModDown inner sums over Q u P go to ext (the digits are dead by then)
  // or, from the fused kernel that still reads the digits, to u; conv holds
  // their conversions.
  const size_t GJ = giant_group(n2), G = std::max<size_t>(ks_group(n1), GJ), J2 = n2 ? n2 : 1;
  take(&x.rtmp, B * csz);
  take(&x.coef, GJ * B * L1 * N);
  take(&x.ext, std::max(GJ * c->dnum, 2 * J2) * B * E * N);
  take(&x.u, std::max(G, J2) * B * 2 * E * N);
  take(&x.conv, std::max(G, J2) * B * csz);
  take(&x.d01, B * csz);
  take(&x.d2, B * L1 * N);
  take(&x.red, B * csz);
  take(&x.giant, B * (n2 ? n2 : 1) * csz);
  take(&x.z0, B * csz);
  take(&x.z1, B * csz);
  return off;
}

WS carve(he_ctx* c) {
  WS w;
  ws_words(c, c->ws_batch, c->ws_n1, c->ws_n2, &w);
  return w;
}

bool same_scale(double a, double b) { return std::fabs(a - b) <= std::ldexp(std::fabs(a), -30); }

const KeySlot* find_rot(const he_ctx* c, u32 galois) {
  for (const KeySlot& k : c->rot)
    if (k.galois == galois) return &k;
  return nullptr;
}

u32 galois_of(const he_ctx* c, int64_t step) {
  const int64_t half = c->N / 2;
  u64 r = (u64)(((step % half) + half) % half);
  u64 g = 1, b = 5, m = 2ull * c->N;
  for (; r; r >>= 1, b = b * b % m)
    if (r & 1) g = g * b % m;
  return (u32)g;
}

// g^{-1} mod 2N: the group of odd residues mod 2N has order N, so g^{N-1}.
u32 galois_inverse(const he_ctx* c, u32 g) {
  const u64 m = 2ull * c->N;
  u64 r = 1, b = g;
  for (u64 e = c->N - 1; e; e >>= 1, b = b * b % m)
    if (e & 1) r = r * b % m;
  return (u32)r;
}

PolyBatch batch_of(u32 nitems) {
  PolyBatch pb;
  std::memset(&pb, 0, sizeof(pb));
  pb.nitems = nitems;
  return pb;
}

// ModUp of the c1 polynomials (NTT form) of B items at level l into w.ext
// (all digits, NTT form): INTT to coefficients, fast base conversion of each
// digit, NTT of the converted limbs.  A digit's own limbs are the source's
// limbs unchanged; the inner product reads them from the source.
int modup(he_ctx* c, u32 l, u32 B, u64* const* c1, const WS& w) {
  const size_t N = c->N;
  const u32 ne = l + 1 + c->np, beta = digits_at(c, l);
  PolyBatch pb = batch_of(B);
  pb.npoly = l + 1;
  for (u32 b = 0; b < B; ++b) {
    pb.src[b] = c1[b];
    pb.dst[b] = w.coef + (size_t)b * (l + 1) * N;
  }
  for (u32 r = 0; r <= l; ++r) pb.prime[r] = (uint8_t)r;
  int rc = launch_ntt(c, pb, true);
  if (!rc) rc = launch_modup_conv(c, l, B, w.coef, w.ext);
  if (rc) return rc;
  PolyBatch nt = batch_of(B);
  nt.npoly = beta * ne;
  for (u32 b = 0; b < B; ++b) nt.src[b] = nt.dst[b] = w.ext + (size_t)b * c->dnum * ne * N;
  for (u32 j = 0; j < beta; ++j) {
    const u32 lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, l + 1);
    for (u32 t = 0; t < ne; ++t)
      nt.prime[j * ne + t] = (t >= lo && t < hi) ? 0xFF : (uint8_t)ext_prime(c, l, t);
  }
  return launch_ntt(c, nt, false);
}

// ModUp of BB items whose c1 polynomials are at c1_base + z c1_stride (the
// giant-step inputs): as modup, items z = 0 .. BB-1 of coef / ext.
int modup_strided(he_ctx* c, u32 l, u32 BB, const u64* c1_base, size_t c1_stride, const WS& w) {
  const size_t N = c->N;
  const u32 ne = l + 1 + c->np, beta = digits_at(c, l);
  PolyBatch pb = batch_of(BB);
  pb.npoly = l + 1;
  pb.src[0] = (u64*)c1_base;
  pb.dst[0] = w.coef;
  pb.stride = c1_stride;
  pb.dst_stride = (size_t)(l + 1) * N;
  for (u32 r = 0; r <= l; ++r) pb.prime[r] = (uint8_t)r;
  int rc = launch_ntt(c, pb, true);
  if (!rc) rc = launch_modup_conv(c, l, BB, w.coef, w.ext);
  if (rc) return rc;
  PolyBatch nt = batch_of(BB);
  nt.npoly = beta * ne;
  nt.src[0] = nt.dst[0] = w.ext;
  nt.stride = (size_t)c->dnum * ne * N;
  for (u32 j = 0; j < beta; ++j) {
    const u32 lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, l + 1);
    for (u32 t = 0; t < ne; ++t)
      nt.prime[j * ne + t] = (t >= lo && t < hi) ? 0xFF : (uint8_t)ext_prime(c, l, t);
  }
  return launch_ntt(c, nt, false);
}

OwnMap own_of(u32 B, u64* const* c1) {
  OwnMap own;
  std::memset(&own, 0, sizeof(own));
  for (u32 b = 0; b < B; ++b) own.ptr[b] = c1[b];
  return own;
}

// Key switch of the digits in w.ext (own limbs from c1) with `key`
// (automorphism `galois` on the digits), ModDown, combined into fa.out.
int ks_core(he_ctx* c, u32 l, u32 B, const WS& w, u64* const* c1, const u64* key, u32 galois, const FinalArgs& fa,
            const u64* bias) {
  const size_t N = c->N;
  const u32 ne = l + 1 + c->np;
  StepKeys sk;
  sk.key[0] = key;
  sk.galois[0] = galois;
  sk.galois_inv[0] = galois_inverse(c, galois);
  int rc = launch_ks_inner_steps(c, l, B, 1, w.ext, 0, own_of(B, c1), sk, w.u);
  if (rc) return rc;
  PolyBatch pi = batch_of(B);
  pi.npoly = 2 * ne;
  for (u32 b = 0; b < B; ++b) pi.src[b] = pi.dst[b] = w.u + (size_t)b * 2 * ne * N;
  for (u32 r = 0; r < 2 * ne; ++r) pi.prime[r] = (r % ne) > l ? (uint8_t)ext_prime(c, l, r % ne) : 0xFF;
  if ((rc = launch_ntt(c, pi, true))) return rc;
  if ((rc = launch_moddown_conv(c, l, B, w.u, w.conv))) return rc;
  PolyBatch pf = batch_of(B);
  pf.npoly = 2 * (l + 1);
  for (u32 b = 0; b < B; ++b) pf.src[b] = pf.dst[b] = w.conv + (size_t)b * 2 * (l + 1) * N;
  for (u32 r = 0; r < 2 * (l + 1); ++r) pf.prime[r] = (uint8_t)(r % (l + 1));
  if ((rc = launch_ntt(c, pf, false))) return rc;
  return launch_ks_final(c, l, B, w.u, w.conv, galois, fa, bias);
}

// S rotation steps of the same B items (digits of their c1 already in w.ext
// from one ModUp): one launch per stage for all S B key switches.
// Everything of a step-batched key switch but the epilogue: u (NTT form,
// P-limbs included) and conv (NTT form) of every (step, item) in w.u / w.conv.
int ks_steps_inner(he_ctx* c, u32 l, u32 B, u32 S, const WS& w, const OwnMap& own, u32 ext_items,
                   const StepKeys& keys) {
  const size_t N = c->N;
  const u32 ne = l + 1 + c->np;
  int rc = launch_ks_inner_steps(c, l, B, S, w.ext, ext_items, own, keys, w.u);
  if (rc) return rc;
  PolyBatch pi = batch_of(S * B);
  pi.npoly = 2 * ne;
  pi.src[0] = pi.dst[0] = w.u;
  pi.stride = (size_t)2 * ne * N;
  for (u32 r = 0; r < 2 * ne; ++r) pi.prime[r] = (r % ne) > l ? (uint8_t)ext_prime(c, l, r % ne) : 0xFF;
  if ((rc = launch_ntt(c, pi, true))) return rc;
  if ((rc = launch_moddown_conv(c, l, S * B, w.u, w.conv))) return rc;
  PolyBatch pf = batch_of(S * B);
  pf.npoly = 2 * (l + 1);
  pf.src[0] = pf.dst[0] = w.conv;
  pf.stride = (size_t)2 * (l + 1) * N;
  for (u32 r = 0; r < 2 * (l + 1); ++r) pf.prime[r] = (uint8_t)(r % (l + 1));
  return launch_ntt(c, pf, false);
}

// ModDown of Z ciphertexts over Q_l u P (y = [Z][2][l+1+K][N], NTT form, limbs
// in [0, q)) into om (+ bias on c0): inverse NTT of the P-limbs in place,
// conversion to Q_l (conv, coefficient form), its NTT, and the combine.
int moddown_items(he_ctx* c, u32 l, u32 Z, u64* y, u64* conv, const OutMap& om, const u64* bias) {
  const size_t N = c->N;
  const u32 ne = l + 1 + c->np;
  PolyBatch pi = batch_of(Z);
  pi.npoly = 2 * ne;
  pi.src[0] = pi.dst[0] = y;
  pi.stride = (size_t)2 * ne * N;
  for (u32 r = 0; r < 2 * ne; ++r) pi.prime[r] = (r % ne) > l ? (uint8_t)ext_prime(c, l, r % ne) : 0xFF;
  int rc = launch_ntt(c, pi, true);
  if (!rc) rc = launch_moddown_conv(c, l, Z, y, conv);
  if (rc) return rc;
  PolyBatch pf = batch_of(Z);
  pf.npoly = 2 * (l + 1);
  pf.src[0] = pf.dst[0] = conv;
  pf.stride = (size_t)2 * (l + 1) * N;
  for (u32 r = 0; r < 2 * (l + 1); ++r) pf.prime[r] = (uint8_t)(r % (l + 1));
  if ((rc = launch_ntt(c, pf, false))) return rc;
  return launch_moddown_final(c, l, Z, y, conv, om, bias);
}

int ks_steps(he_ctx* c, u32 l, u32 B, u32 S, const WS& w, u64* const* c1, const StepKeys& keys, const Items& add0,
             const OutMap& om) {
  int rc = ks_steps_inner(c, l, B, S, w, own_of(B, c1), 0, keys);
  return rc ? rc : launch_ks_final_steps(c, l, B, S, w.u, w.conv, keys, add0, om);
}

FinalArgs no_final() {
  FinalArgs fa;
  std::memset(&fa, 0, sizeof(fa));
  return fa;
}

// Pointers, levels and scales of a batched call (no workspace involved).
int check_items(const he_ctx* c, u32 n, const he_ct* in, const he_ct* out, u32 n_out) {
  if (!c || !in || !out || n == 0 || n > HE_MAXB) return HE_EINVAL;
  for (u32 b = 0; b < n; ++b) {
    if (!in[b].dev) return HE_EINVAL;
    if (in[b].level >= c->nq || in[b].level != in[0].level) return HE_ELEVEL;
    if (!same_scale(in[b].scale, in[0].scale)) return HE_ESCALE;
  }
  for (u32 b = 0; b < n_out; ++b)
    if (!out[b].dev) return HE_EINVAL;
  return HE_OK;
}

int check_batch(const he_ctx* c, u32 n, const he_ct* in, const he_ct* out, u32 n_out) {
  if (!c || !in || !out || n == 0 || n > HE_MAXB) return HE_EINVAL;
  if (!c->ws) return HE_ESTATE;
  if (n > c->ws_batch) return HE_ENOMEM;
  for (u32 b = 0; b < n; ++b) {
    if (!in[b].dev) return HE_EINVAL;
    if (in[b].level >= c->nq || in[b].level != in[0].level) return HE_ELEVEL;
    if (!same_scale(in[b].scale, in[0].scale)) return HE_ESCALE;
  }
  for (u32 b = 0; b < n_out; ++b)
    if (!out[b].dev) return HE_EINVAL;
  return HE_OK;
}

int copy_ct(he_ctx* c, u32 l, const u64* src, u64* dst) {
  if (src == dst) return HE_OK;
  return hipMemcpyAsync(dst, src, (size_t)2 * (l + 1) * c->N * sizeof(u64), hipMemcpyDeviceToDevice, c->stream) ==
                 hipSuccess
             ? HE_OK
             : HE_EDEVICE;
}

// Rescale of n ciphertexts at level l > 0 (checked by the caller) with its
// scratch regions: rtmp [n][2][l+1][N] (the inverse NTT of the last limbs, at
// their positions), red [n][2][l][N] (those limbs reduced mod q_i, NTT form)
// and, when an output aliases its input, z0 [n][2][l][N] (staging).
int rescale_items(he_ctx* c, u32 n, const he_ct* in, he_ct* out, u64* rtmp, u64* red, u64* z0) {
  int rc;
  const u32 l = in[0].level;
  const size_t N = c->N;
  // INTT of the last limb of both polynomials into rtmp ([B][2][l+1][N] layout).
  PolyBatch pb = batch_of(n);
  pb.npoly = 2 * (l + 1);
  for (u32 b = 0; b < n; ++b) {
    pb.src[b] = in[b].dev;
    pb.dst[b] = rtmp + (size_t)b * 2 * (l + 1) * N;
  }
  for (u32 r = 0; r < 2 * (l + 1); ++r) pb.prime[r] = (r % (l + 1)) == l ? (uint8_t)l : 0xFF;
  if ((rc = launch_ntt(c, pb, true))) return rc;
  if ((rc = launch_rescale_reduce(c, l, n, rtmp, red))) return rc;
  PolyBatch pr = batch_of(n);
  pr.npoly = 2 * l;
  for (u32 b = 0; b < n; ++b) pr.src[b] = pr.dst[b] = red + (size_t)b * 2 * l * N;
  for (u32 r = 0; r < 2 * l; ++r) pr.prime[r] = (uint8_t)(r % l);
  if ((rc = launch_ntt(c, pr, false))) return rc;
  Items ii, oo;
  ii.n = oo.n = n;
  bool alias = false;
  for (u32 b = 0; b < n; ++b) {
    ii.p[b] = in[b].dev;
    alias |= out[b].dev == in[b].dev;
  }
  // An in-place rescale moves c1 down by one limb: stage through z0.
  for (u32 b = 0; b < n; ++b) oo.p[b] = alias ? z0 + (size_t)b * 2 * l * N : out[b].dev;
  if ((rc = launch_rescale_final(c, l, ii, red, oo))) return rc;
  if (alias)
    for (u32 b = 0; b < n; ++b)
      if (hipMemcpyAsync(out[b].dev, oo.p[b], (size_t)2 * l * N * sizeof(u64), hipMemcpyDeviceToDevice, c->stream) !=
          hipSuccess)
        return HE_EDEVICE;
  for (u32 b = 0; b < n; ++b) {
    out[b].level = l - 1;
    out[b].scale = in[b].scale / (double)c->primes[l];
  }
  return HE_OK;
}

}  // namespace

extern "C" {

size_t he_workspace_bytes(const he_ctx* c, uint32_t max_batch, uint32_t max_n1, uint32_t max_n2) {
  if (!c) return 0;
  return ws_words(c, max_batch ? max_batch : 1, max_n1, max_n2, nullptr) * sizeof(u64);
}

int he_ctx_bind(he_ctx* c, void* ws, size_t bytes, uint32_t max_batch, uint32_t max_n1, uint32_t max_n2) {
  if (!c || !ws || max_batch == 0 || max_batch > HE_MAXB || ((uintptr_t)ws & 255)) return HE_EINVAL;
  if (bytes < he_workspace_bytes(c, max_batch, max_n1, max_n2)) return HE_ENOMEM;
  c->ws = (uint8_t*)ws;
  c->ws_bytes = bytes;
  c->ws_batch = max_batch;
  c->ws_n1 = max_n1;
  c->ws_n2 = max_n2;
  return HE_OK;
}

int he_rotate_hoisted_batch(he_ctx* c, uint32_t n, const he_ct* in, uint32_t n_steps, const int32_t* steps,
                            he_ct* out) {
  int rc = check_batch(c, n, in, out, n * n_steps);
  if (rc) return rc;
  if (n_steps && !steps) return HE_EINVAL;
  const u32 l = in[0].level;
  std::vector<const KeySlot*> keys(n_steps);
  for (u32 s = 0; s < n_steps; ++s) {
    const u32 g = galois_of(c, steps[s]);
    keys[s] = g == 1 ? nullptr : find_rot(c, g);
    if (g != 1 && !keys[s]) return HE_ENOKEY;
    for (u32 b = 0; b < n; ++b)
      if (g != 1 && out[b * n_steps + s].dev == in[b].dev) return HE_EINVAL;
  }
  const WS w = carve(c);
  const size_t N = c->N;
  bool need_modup = false;
  for (u32 s = 0; s < n_steps; ++s) need_modup |= keys[s] != nullptr;
  u64* c1[HE_MAXB];
  for (u32 b = 0; b < n; ++b) c1[b] = in[b].dev + (size_t)(l + 1) * N;
  if (need_modup && (rc = modup(c, l, n, c1, w))) return rc;
  Items add0;
  add0.n = n;
  for (u32 b = 0; b < n; ++b) add0.p[b] = in[b].dev;
  // keyed steps in groups that fit the workspace and the output pointer table
  const u32 group = std::max<u32>(1, std::min<u32>(ks_group(c->ws_n1), HE_MAXB / n));
  std::vector<u32> keyed;
  for (u32 s = 0; s < n_steps; ++s) {
    for (u32 b = 0; b < n; ++b) {
      out[b * n_steps + s].level = l;
      out[b * n_steps + s].scale = in[b].scale;
    }
    if (keys[s]) {
      keyed.push_back(s);
      continue;
    }
    for (u32 b = 0; b < n; ++b)
      if ((rc = copy_ct(c, l, in[b].dev, out[b * n_steps + s].dev))) return rc;
  }
  for (size_t g0 = 0; g0 < keyed.size(); g0 += group) {
    const u32 S = (u32)std::min<size_t>(group, keyed.size() - g0);
    StepKeys sk;
    OutMap om;
    std::memset(&om, 0, sizeof(om));
    for (u32 i = 0; i < S; ++i) {
      const u32 s = keyed[g0 + i];
      sk.key[i] = keys[s]->dev;
      sk.galois[i] = keys[s]->galois;
      sk.galois_inv[i] = galois_inverse(c, keys[s]->galois);
      for (u32 b = 0; b < n; ++b) om.ptr[i * n + b] = out[b * n_steps + s].dev;
    }
    if ((rc = ks_steps(c, l, n, S, w, c1, sk, add0, om))) return rc;
  }
  return HE_OK;
}

int he_rotate_hoisted(he_ctx* c, const he_ct* in, uint32_t n_steps, const int32_t* steps, he_ct* out) {
  return he_rotate_hoisted_batch(c, 1, in, n_steps, steps, out);
}

int he_rotate(he_ctx* c, const he_ct* in, int32_t step, he_ct* out) {
  return he_rotate_hoisted_batch(c, 1, in, 1, &step, out);
}

int he_square_batch(he_ctx* c, uint32_t n, const he_ct* in, he_ct* out) {
  int rc = check_batch(c, n, in, out, n);
  if (rc) return rc;
  if (!c->have_relin) return HE_ENOKEY;
  const u32 l = in[0].level;
  const size_t N = c->N;
  const WS w = carve(c);
  Items it;
  it.n = n;
  for (u32 b = 0; b < n; ++b) it.p[b] = in[b].dev;
  if ((rc = launch_tensor(c, l, it, w.d01, w.d2))) return rc;
  u64* c1[HE_MAXB];
  for (u32 b = 0; b < n; ++b) c1[b] = w.d2 + (size_t)b * (l + 1) * N;
  if ((rc = modup(c, l, n, c1, w))) return rc;
  FinalArgs fa = no_final();
  for (u32 b = 0; b < n; ++b) {
    fa.out[b] = out[b].dev;
    fa.add0[b] = w.d01 + (size_t)b * 2 * (l + 1) * N;
    fa.add1[b] = w.d01 + (size_t)b * 2 * (l + 1) * N + (size_t)(l + 1) * N;
  }
  if ((rc = ks_core(c, l, n, w, c1, c->relin_dev, 1, fa, nullptr))) return rc;
  for (u32 b = 0; b < n; ++b) {
    out[b].level = l;
    out[b].scale = in[b].scale * in[b].scale;
  }
  return HE_OK;
}

int he_square(he_ctx* c, const he_ct* in, he_ct* out) { return he_square_batch(c, 1, in, out); }

int he_rescale_batch(he_ctx* c, uint32_t n, const he_ct* in, he_ct* out) {
  int rc = check_batch(c, n, in, out, n);
  if (rc) return rc;
  if (in[0].level == 0) return HE_ELEVEL;
  const WS w = carve(c);
  return rescale_items(c, n, in, out, w.rtmp, w.red, w.z0);
}

int he_rescale_batch_noalloc(he_ctx* c, uint32_t n, const he_ct* in, he_ct* out) {
  int rc = check_items(c, n, in, out, n);
  if (rc) return rc;
  const u32 l = in[0].level;
  if (l == 0) return HE_ELEVEL;
  const int dev = c->device;
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (dev < 0 || dev >= kMaxDevices || !g_noalloc_done[dev]) return HE_ESTATE;
    if (g_noalloc_rc[dev]) return g_noalloc_rc[dev];
    base = g_noalloc_ptr[dev];
  }
  bool alias = false;
  for (u32 b = 0; b < n; ++b) alias |= out[b].dev == in[b].dev;
  const size_t N = c->N;
  const size_t rtmp_w = (size_t)n * 2 * (l + 1) * N, red_w = (size_t)n * 2 * l * N;
  const size_t need = (rtmp_w + red_w + (alias ? red_w : 0)) * sizeof(u64);
  if (need > HE_NOALLOC_SCRATCH_BYTES) return HE_ENOMEM;
  u64* rtmp = (u64*)base;
  u64* red = rtmp + rtmp_w;
  return rescale_items(c, n, in, out, rtmp, red, red + red_w);
}

int he_rescale(he_ctx* c, const he_ct* in, he_ct* out) { return he_rescale_batch(c, 1, in, out); }

int he_add(he_ctx* c, const he_ct* a, const he_ct* b, he_ct* out) {
  if (!c || !a || !b || !out || !a->dev || !b->dev || !out->dev) return HE_EINVAL;
  if (a->level != b->level || a->level >= c->nq) return HE_ELEVEL;
  if (!same_scale(a->scale, b->scale)) return HE_ESCALE;
  Items x, y, o;
  x.n = y.n = o.n = 1;
  x.p[0] = a->dev;
  y.p[0] = b->dev;
  o.p[0] = out->dev;
  int rc = launch_add(c, a->level, x, y, o);
  if (rc) return rc;
  out->level = a->level;
  out->scale = a->scale;
  return HE_OK;
}

int he_eval_dense_batch(he_ctx* c, uint32_t n, const he_ct* in, const he_dense* d, he_ct* out) {
  int rc = check_batch(c, n, in, out, n);
  if (rc) return rc;
  if (!d || d->ctx != c) return HE_EINVAL;
  const u32 l = d->level;
  if (in[0].level != l) return HE_ELEVEL;
  const u32 n1 = d->n1, n2 = d->n2;
  if (n1 > std::max<u32>(c->ws_n1, 1) || n2 > std::max<u32>(c->ws_n2, 1)) return HE_ENOMEM;
  if (n1 > 1 && n1 - 1 > ks_group(c->ws_n1)) return HE_ENOMEM;   // all baby steps in one step-batched switch
  const double out_scale = in[0].scale * d->pt_scale;
  if (d->bias && !same_scale(d->bias_scale, out_scale)) return HE_ESCALE;
  for (u32 b = 0; b < n; ++b)
    if (out[b].dev == in[b].dev) return HE_EINVAL;
  // Rotation keys for every step, looked up before anything is enqueued.
  std::vector<u32> rs_steps;
  for (u32 t = d->n / 2; t >= d->m && t > 0; t /= 2) rs_steps.push_back(t);
  std::vector<const KeySlot*> baby(n1, nullptr), giant(n2, nullptr), rsk(rs_steps.size(), nullptr);
  for (u32 i = 1; i < n1; ++i)
    if (!(baby[i] = find_rot(c, galois_of(c, i)))) return HE_ENOKEY;   // i < n1 <= 64 < N/2: never the identity
  for (u32 j = 1; j < n2; ++j)
    if (galois_of(c, (int64_t)n1 * j) != 1 && !(giant[j] = find_rot(c, galois_of(c, (int64_t)n1 * j)))) return HE_ENOKEY;
  // Hoisted rotate-and-sum (rs_bits > 0): groups of rs_bits bits of the shift
  // index from the most significant; group g sums rho^{k t_g}, 0 < k < 2^b_g.
  const bool rs_hoisted = d->rs_bits > 0 && !rs_steps.empty();
  std::vector<u32> grp_bits, grp_shift;
  std::vector<StepKeys> grp_keys;
  if (rs_hoisted) {
    u32 left = 0;
    while ((d->m << left) < d->n) ++left;
    while (left > 0) {
      const u32 b = std::min<u32>(d->rs_bits, left);
      left -= b;
      const u32 t = d->m << left;
      StepKeys sk;
      std::memset(&sk, 0, sizeof(sk));
      for (u32 k = 1; k < (1u << b); ++k) {       // k t < n <= N/2: never the identity
        const KeySlot* ks = find_rot(c, galois_of(c, (int64_t)k * t));
        if (!ks) return HE_ENOKEY;
        sk.key[k - 1] = ks->dev;
        sk.galois[k - 1] = ks->galois;
        sk.galois_inv[k - 1] = galois_inverse(c, ks->galois);
        if (k == 1) {                              // step k rotates by k t: galois[k-1] = galois[0]^k
          sk.orbit = ks->orbit;
          sk.orbit_even = ks->orbit_even;
        }
      }
      grp_bits.push_back(b);
      grp_shift.push_back(t);
      grp_keys.push_back(sk);
    }
  } else {
    for (size_t u = 0; u < rs_steps.size(); ++u)
      if (galois_of(c, rs_steps[u]) != 1 && !(rsk[u] = find_rot(c, galois_of(c, rs_steps[u])))) return HE_ENOKEY;
  }

  const size_t N = c->N, csz = (size_t)2 * (l + 1) * N;
  const WS w = carve(c);
  Items inI;
  inI.n = n;
  for (u32 b = 0; b < n; ++b) inI.p[b] = in[b].dev;

  // Baby steps: one hoisted ModUp, n1 - 1 key switches.
  u64* c1in[HE_MAXB];
  for (u32 b = 0; b < n; ++b) c1in[b] = in[b].dev + (size_t)(l + 1) * N;
  if (n1 > 1) {
    // Baby steps i = 1 .. n1-1 (all below N/2, so each has a key): one hoisted
    // ModUp, then one step-batched key switch whose epilogue forms each
    // rotated ciphertext in registers and folds it straight into the inner
    // sums s_j (giant region [n2][B][csz]); the rotations are never stored.
    // The workspace holds ks_group(max_n1) >= n1 - 1 steps.
    if ((rc = modup(c, l, n, c1in, w))) return rc;
    const u32 S = n1 - 1;
    StepKeys sk;
    for (u32 i = 0; i < S; ++i) {
      sk.key[i] = baby[i + 1]->dev;
      sk.galois[i] = baby[i + 1]->galois;
      sk.galois_inv[i] = galois_inverse(c, baby[i + 1]->galois);
    }
    sk.orbit = baby[1]->orbit;                     // baby step i rotates by i: galois[i] = galois[0]^(i+1)
    sk.orbit_even = baby[1]->orbit_even;
    if (d->pl > l + 1) {
      // lazy ModDown: the inner products stay over Q_l u P; the inner sums
      // are formed there (the extended rotations only in registers) into
      // the dead digit region, then each sum is brought down once
      // (fused: the inner products stay in registers; the sums go to w.u,
      // free in this form, since the digits in w.ext are read throughout)
      u64* sqp = w.ext;
      if (c->ks_fuse && n2 <= 8) {
        sqp = w.u;
        if ((rc = launch_ks_ext_fused(c, l, n, n1, n2, w.ext, own_of(n, c1in), sk, inI, d->pts, sqp, w.conv)))
          return rc;
      } else {
        if ((rc = launch_ks_inner_steps(c, l, n, S, w.ext, 0, own_of(n, c1in), sk, w.u))) return rc;
        if ((rc = launch_ext_multplain(c, l, n, n1, n2, w.u, sk, inI, d->pts, w.ext))) return rc;
      }
      OutMap om;
      std::memset(&om, 0, sizeof(om));
      om.base = w.giant;
      om.ob = csz;
      if ((rc = moddown_items(c, l, n2 * n, sqp, w.conv, om, nullptr))) return rc;
    } else {
      if ((rc = ks_steps_inner(c, l, n, S, w, own_of(n, c1in), 0, sk))) return rc;
      if ((rc = launch_ks_final_multplain(c, l, n, n1, n2, w.u, w.conv, sk, inI, d->pts, w.giant))) return rc;
    }
  } else if ((rc = launch_multplain(c, l, n2, inI, d->pts, d->pl, w.giant))) {
    return rc;                                     // n1 = 1: s_j = pts[j] (.) in (= ModDown(pts[j] (.) P in))
  }

  // Giant steps then rotate-and-sum, each a full key switch; the last one
  // writes the caller's output and adds the bias.
  // giant region [n2][B][csz]: s_j of item b at giant + (j n + b) csz
  u32 total = (n2 - 1) + (rs_hoisted ? 0u : (u32)rs_steps.size());
  u64* cur[HE_MAXB];
  for (u32 b = 0; b < n; ++b) cur[b] = w.giant + (size_t)b * csz;
  bool giants_batched = n2 > 1 && n2 - 1 <= giant_group(c->ws_n2);
  for (u32 j = 1; j < n2; ++j) giants_batched = giants_batched && giant[j];
  if (giants_batched) {
    // Every giant step at once: ModUp of all s_j (j >= 1), one step-batched
    // key switch (own digits per (j, b)), and an epilogue that sums
    // s_0 + rho(s_1) + ... per item.  Equal to the in-order accumulation.
    const u32 J = n2 - 1;
    if ((rc = modup_strided(c, l, J * n, w.giant + (size_t)n * csz + (size_t)(l + 1) * N, csz, w))) return rc;
    StepKeys sk;
    for (u32 j = 0; j < J; ++j) {
      sk.key[j] = giant[j + 1]->dev;
      sk.galois[j] = giant[j + 1]->galois;
      sk.galois_inv[j] = galois_inverse(c, giant[j + 1]->galois);
    }
    OwnMap own;
    std::memset(&own, 0, sizeof(own));
    own.base = w.giant + (size_t)n * csz + (size_t)(l + 1) * N;
    own.os = (size_t)n * csz;
    own.ob = csz;
    if ((rc = ks_steps_inner(c, l, n, J, w, own, n, sk))) return rc;
    const bool last = rs_steps.empty();
    OutMap om;
    std::memset(&om, 0, sizeof(om));
    for (u32 b = 0; b < n; ++b) om.ptr[b] = last ? out[b].dev : w.z0 + (size_t)b * csz;
    if ((rc = launch_ks_final_sum(c, l, n, J, w.u, w.conv, sk, w.giant, last ? d->bias : nullptr, om))) return rc;
    if (last) {
      for (u32 b = 0; b < n; ++b) {
        out[b].level = l;
        out[b].scale = out_scale;
      }
      return HE_OK;
    }
    for (u32 b = 0; b < n; ++b) cur[b] = w.z0 + (size_t)b * csz;
    total = rs_hoisted ? 0u : (u32)rs_steps.size();
  }
  u32 done = 0;
  auto step = [&](const KeySlot* key, u64* const* src, bool accumulate_in_place) -> int {
    ++done;
    const bool last = done == total && !rs_hoisted;
    u64* dst[HE_MAXB];
    for (u32 b = 0; b < n; ++b) {
      if (last) dst[b] = out[b].dev;
      else if (accumulate_in_place) dst[b] = cur[b];
      else dst[b] = (cur[b] == w.z0 + (size_t)b * csz) ? w.z1 + (size_t)b * csz : w.z0 + (size_t)b * csz;
    }
    FinalArgs fa = no_final();
    for (u32 b = 0; b < n; ++b) {
      fa.out[b] = dst[b];
      fa.add0[b] = src[b];
      fa.acc[b] = cur[b];
    }
    const u64* bias = last ? d->bias : nullptr;
    int r;
    if (key) {
      u64* c1[HE_MAXB];
      for (u32 b = 0; b < n; ++b) c1[b] = src[b] + (size_t)(l + 1) * N;
      if ((r = modup(c, l, n, c1, w))) return r;
      if ((r = ks_core(c, l, n, w, c1, key->dev, key->galois, fa, bias))) return r;
    } else {
      // rotation by a multiple of N/2 is the identity: dst = cur + src
      Items a, s, o;
      a.n = s.n = o.n = n;
      for (u32 b = 0; b < n; ++b) { a.p[b] = cur[b]; s.p[b] = (u64*)src[b]; o.p[b] = dst[b]; }
      if ((r = launch_add(c, l, a, s, o))) return r;
      if (bias && (r = launch_add_plain(c, l, o, bias))) return r;
    }
    for (u32 b = 0; b < n; ++b) cur[b] = dst[b];
    return HE_OK;
  };
  for (u32 j = 1; j < n2 && !giants_batched; ++j) {
    u64* src[HE_MAXB];
    for (u32 b = 0; b < n; ++b) src[b] = w.giant + ((size_t)j * n + b) * csz;
    if ((rc = step(giant[j], src, true))) return rc;
  }
  for (size_t u = 0; u < rs_steps.size() && !rs_hoisted; ++u) {
    u64* src[HE_MAXB];
    for (u32 b = 0; b < n; ++b) src[b] = cur[b];
    if ((rc = step(rsk[u], src, false))) return rc;
  }
  for (size_t g = 0; g < grp_bits.size(); ++g) {
    // one hoisted group: ModUp of cur's c1, the 2^b - 1 rotations' inner
    // products summed with P cur in registers (extended basis), one ModDown
    const bool last = g + 1 == grp_bits.size();
    u64* c1[HE_MAXB];
    Items ci;
    ci.n = n;
    for (u32 b = 0; b < n; ++b) {
      c1[b] = cur[b] + (size_t)(l + 1) * N;
      ci.p[b] = cur[b];
    }
    if ((rc = modup(c, l, n, c1, w))) return rc;
    if ((rc = launch_ks_ext_fused(c, l, n, 1u << grp_bits[g], 1, w.ext, own_of(n, c1), grp_keys[g], ci, nullptr,
                                  w.u, w.conv)))
      return rc;
    OutMap om;
    std::memset(&om, 0, sizeof(om));
    for (u32 b = 0; b < n; ++b)
      om.ptr[b] = last ? out[b].dev
                       : ((cur[b] == w.z0 + (size_t)b * csz) ? w.z1 + (size_t)b * csz : w.z0 + (size_t)b * csz);
    if ((rc = moddown_items(c, l, n, w.u, w.conv, om, last ? d->bias : nullptr))) return rc;
    for (u32 b = 0; b < n; ++b) cur[b] = om.ptr[b];
  }
  if (total == 0 && !rs_hoisted) {
    Items o;
    o.n = n;
    for (u32 b = 0; b < n; ++b) {
      if ((rc = copy_ct(c, l, cur[b], out[b].dev))) return rc;
      o.p[b] = out[b].dev;
    }
    if (d->bias && (rc = launch_add_plain(c, l, o, d->bias))) return rc;
  }
  for (u32 b = 0; b < n; ++b) {
    out[b].level = l;
    out[b].scale = out_scale;
  }
  return HE_OK;
}

int he_eval_dense(he_ctx* c, const he_ct* in, const he_dense* d, he_ct* out) {
  return he_eval_dense_batch(c, 1, in, d, out);
}

size_t he_linear_scratch_bytes(const he_ctx* c, uint32_t level, uint32_t n_in, uint32_t n_baby) {
  return c ? (size_t)n_in * n_baby * 2 * (level + 1) * c->N * sizeof(u64) : 0;
}

int he_eval_linear_batch(he_ctx* c, uint32_t n_req, const he_ct* in, const he_linear* t, void* scratch,
                         size_t scratch_bytes, he_ct* out) {
  if (!t || t->ctx != c || n_req == 0) return HE_EINVAL;
  const u32 n_in = t->n_in, n_out = t->n_out, NB = t->n_baby, NG = t->n_giant, l = t->level;
  const u32 I = n_req * n_in, M = n_req * n_out, T = n_in * NB;
  if (I > HE_MAXB || M > HE_MAXB) return HE_ENOMEM;
  int rc = check_batch(c, I, in, out, M);
  if (rc) return rc;
  if (in[0].level != l) return HE_ELEVEL;
  if (M > c->ws_batch) return HE_ENOMEM;
  if (NG > std::max<u32>(c->ws_n2, 1) || (NG > 1 && NG - 1 > giant_group(c->ws_n2))) return HE_ENOMEM;
  for (u32 j = 0; j < M; ++j)
    for (u32 i = 0; i < I; ++i)
      if (out[j].dev == in[i].dev) return HE_EINVAL;
  const size_t N = c->N, csz = (size_t)2 * (l + 1) * N;
  if (!scratch || scratch_bytes < (size_t)I * NB * csz * sizeof(u64)) return HE_ENOMEM;
  // keys, checked before anything is enqueued
  std::vector<int32_t> bsteps;
  std::vector<u32> bslot(NB, 0xFFFFFFFFu);
  for (u32 b = 0; b < NB; ++b)
    if (galois_of(c, t->baby[b]) != 1) {
      bslot[b] = (u32)bsteps.size();
      bsteps.push_back(t->baby[b]);
    }
  StepKeys sk;
  std::memset(&sk, 0, sizeof(sk));
  for (u32 g = 1; g < NG; ++g) {
    const KeySlot* k = find_rot(c, galois_of(c, t->giant[g]));
    if (galois_of(c, t->giant[g]) == 1 || !k) return HE_ENOKEY;   // giant[g] must be a real rotation
    sk.key[g - 1] = k->dev;
    sk.galois[g - 1] = k->galois;
    sk.galois_inv[g - 1] = galois_inverse(c, k->galois);
  }
  for (int32_t st : bsteps)
    if (!find_rot(c, galois_of(c, st))) return HE_ENOKEY;
  const WS w = carve(c);
  u64* x = (u64*)scratch;   // term (item, b) of input item = r n_in + i at x + (item NB + b) csz
  // 1. baby rotations of every input (one hoisted ModUp per input, step-batched key switches);
  //    the unrotated terms are copied next to them
  if (!bsteps.empty()) {
    std::vector<he_ct> rot(I * bsteps.size());
    for (u32 it = 0; it < I; ++it)
      for (u32 b = 0; b < NB; ++b)
        if (bslot[b] != 0xFFFFFFFFu) rot[it * bsteps.size() + bslot[b]].dev = x + ((size_t)it * NB + b) * csz;
    if ((rc = he_rotate_hoisted_batch(c, I, in, (u32)bsteps.size(), bsteps.data(), rot.data()))) return rc;
  }
  for (u32 it = 0; it < I; ++it)
    for (u32 b = 0; b < NB; ++b)
      if (bslot[b] == 0xFFFFFFFFu && (rc = copy_ct(c, l, in[it].dev, x + ((size_t)it * NB + b) * csz))) return rc;
  // 2. inner sums s[g][r n_out + j] = sum_{i, b} pt[g][j][i][b] (.) rho^{baby b}(in[r n_in + i]),
  //    at giant + (g M + r n_out + j) csz (the layout of the dense layer's giant region)
  if ((rc = launch_mp_acc(c, l, n_req, T, n_out, NG, x, t->pts, w.giant))) return rc;
  // 3. out[m] = s[0][m] + sum_{g >= 1} rho^{giant g}(s[g][m]): every giant step of every output in
  //    one step-batched key switch (one ModUp per (g, m)), summed in one epilogue
  if (NG == 1) {
    for (u32 m = 0; m < M; ++m)
      if ((rc = copy_ct(c, l, w.giant + (size_t)m * csz, out[m].dev))) return rc;
  } else {
    const u32 J = NG - 1;
    u64* c1base = w.giant + (size_t)M * csz + (size_t)(l + 1) * N;
    if ((rc = modup_strided(c, l, J * M, c1base, csz, w))) return rc;
    OwnMap own;
    std::memset(&own, 0, sizeof(own));
    own.base = c1base;
    own.os = (size_t)M * csz;
    own.ob = csz;
    if ((rc = ks_steps_inner(c, l, M, J, w, own, M, sk))) return rc;
    OutMap om;
    std::memset(&om, 0, sizeof(om));
    for (u32 m = 0; m < M; ++m) om.ptr[m] = out[m].dev;
    if ((rc = launch_ks_final_sum(c, l, M, J, w.u, w.conv, sk, w.giant, nullptr, om))) return rc;
  }
  for (u32 m = 0; m < M; ++m) {
    out[m].level = l;
    out[m].scale = in[0].scale * t->pt_scale;
  }
  return HE_OK;
}

int he_eval_linear(he_ctx* c, const he_ct* in, const he_linear* t, void* scratch, size_t scratch_bytes,
                   he_ct* out) {
  return he_eval_linear_batch(c, 1, in, t, scratch, scratch_bytes, out);
}

}  // extern "C"
