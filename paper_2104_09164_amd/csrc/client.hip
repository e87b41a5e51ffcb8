// Client side of the protocol on the device: CKKS encoding (inverse
// canonical embedding, scaling, rounding, RNS), public-key encryption with
// caller-supplied random polynomials, decryption and decoding (exact
// centred CRT lift, canonical embedding).  The parties that hold pk and sk
// run these (Results, "Time requirement of secure action recognition",
// steps (iii) encryption and (v) decryption); the evaluation path never
// calls them.
//
// Embedding.  Slot j lives at zeta^(e_j), e_j = 5^j mod 2N, zeta = exp(i pi/N);
// the conjugate slot at zeta^(-e_j).  Every odd exponent t = 2u + 1 mod 2N is
// one of +-e_j, so with w_u = z_j at u = (e_j - 1)/2 and conj(z_j) at
// u = N - 1 - (e_j - 1)/2:
//   encode:  m_k = (1/N) Re( zeta^-k  sum_u w_u exp(-2 pi i u k / N) )
//   decode:  z_j = sum_k (m_k zeta^k) exp(+2 pi i u k / N)  at u = (e_j - 1)/2.
// Both are one length-N complex FFT in double precision: Stockham passes of
// radix 8 (one radix-2 or radix-4 pass first when 3 does not divide
// log2 N), self-sorting, natural order in and out; each pass is an HBM
// streaming kernel over the whole batch, consecutive threads reading
// consecutive complex words, 8 points per thread in registers.
//
// Encryption and decryption are limb-local (one thread per coefficient per
// limb): residues of the small polynomials, forward NTTs (the library's
// transforms), and products with pk / s kept in Montgomery form.
#include "rns_kernels.hpp"
#include "modarith.hpp"

#include <cmath>
#include <cstring>
#include <vector>

struct he_client {
  he_ctx* ctx = nullptr;
  u32 max_batch = 0;
  u64* pk = nullptr;       // [2][L+1][N] NTT form, Montgomery form (x 2^64 mod q_i)
  u64* sk = nullptr;       // [L+1][N] NTT form, Montgomery form
  double2* tw = nullptr;   // [N] exp(-2 pi i k / N)
  double2* twist = nullptr;  // [N] zeta^k = exp(i pi k / N)
  u32* pos = nullptr;      // [N/2] (e_j - 1) / 2
  u64* garner = nullptr;   // [nq][nq][2]: q_j^{-1} mod q_i and its Shoup companion (j < i)
  double2* fa = nullptr;   // [max_batch][N] FFT ping-pong buffers
  double2* fb = nullptr;
  u64* res = nullptr;      // [max_batch][3][L+1][N] encryption: residues of (v, m + e0, e1)
};

namespace {

constexpr int BS = 256;

inline int ok() { return hipGetLastError() == hipSuccess ? HE_OK : HE_EDEVICE; }

__device__ __forceinline__ u64 signed_residue(int64_t x, const PrimeConst& P) {
  const u64 r = reduce64(x < 0 ? (u64)(-x) : (u64)x, P.q, P.mu);
  return (x < 0 && r) ? P.q - r : r;
}

// grid (N/BS, nl): out[i][k] = s[k] mod q_i
__global__ void __launch_bounds__(BS) k_cl_signed_rns(const int64_t* __restrict__ s, u64* __restrict__ out,
                                                      const PrimeConst* __restrict__ pc, u32 N) {
  const u32 k = blockIdx.x * BS + threadIdx.x, i = blockIdx.y;
  out[(size_t)i * N + k] = signed_residue(s[k], pc[i]);
}

// grid (N/BS, rows): x <- x 2^64 mod q (row r over prime r mod period)
__global__ void __launch_bounds__(BS) k_cl_to_mont(u64* __restrict__ x, const PrimeConst* __restrict__ pc, u32 N,
                                                   u32 period) {
  const u32 k = blockIdx.x * BS + threadIdx.x, r = blockIdx.y;
  const PrimeConst P = pc[r % period];
  u64* p = x + (size_t)r * N + k;
  *p = shoup(*p, P.rmod, P.rmod_sh, P.q);
}

// grid (N/2/BS, n): w[b][pos_j] = z_j, w[b][N-1-pos_j] = conj(z_j)
__global__ void __launch_bounds__(BS) k_cl_scatter(const double2* __restrict__ z, double2* __restrict__ w,
                                                   const u32* __restrict__ pos, u32 N) {
  const u32 j = blockIdx.x * BS + threadIdx.x, b = blockIdx.y;
  const double2 v = z[(size_t)b * (N / 2) + j];
  const u32 u = pos[j];
  double2* o = w + (size_t)b * N;
  o[u] = v;
  o[N - 1 - u] = make_double2(v.x, -v.y);
}

// In-register DFT of R = 2, 4 or 8 points, natural order in and out:
// V_t = sum_s v_s exp(-+2 pi i s t / R), by radix-2 Stockham passes over the
// register array (all indices compile-time after unrolling).
template <int R>
__device__ __forceinline__ void dft_regs(double2 (&v)[R], bool inverse) {
  constexpr double h = 0.70710678118654752440;   // cos(pi/4)
  const double2 w8[8] = {{1.0, 0.0}, {h, -h}, {0.0, -1.0}, {-h, -h}, {-1.0, 0.0}, {-h, h}, {0.0, 1.0}, {h, h}};
#pragma unroll
  for (int ns = 1; ns < R; ns *= 2) {
    double2 o[R];
#pragma unroll
    for (int jj = 0; jj < R / 2; ++jj) {
      const int k = jj & (ns - 1);
      double2 w = w8[k * (8 / (2 * ns))];   // exp(-2 pi i k / (2 ns))
      if (inverse) w.y = -w.y;
      const double2 a = v[jj], b = v[jj + R / 2];
      const double2 t = make_double2(b.x * w.x - b.y * w.y, b.x * w.y + b.y * w.x);
      const int d = (jj / ns) * 2 * ns + k;
      o[d] = make_double2(a.x + t.x, a.y + t.y);
      o[d + ns] = make_double2(a.x - t.x, a.y - t.y);
    }
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = o[m];
  }
}

// One Stockham radix-R pass (R = 2^LR) after sub-transforms of length
// ns = 2^lns; grid (N/R/BS, n).  Thread j: v_t = x[j + t N/R] times the
// twiddle W^(t (j mod ns)), W = exp(-+2 pi i / (R ns)); R-point DFT; V_t to
// y[(j / ns) R ns + (j mod ns) + t ns].  Passes whose radices multiply to N,
// with ns the product of the radices before, give the DFT in natural order
// (sign - forward, + inverse, unnormalised).
template <int LR>
__global__ void __launch_bounds__(BS) k_cl_fft_pass(const double2* __restrict__ x, double2* __restrict__ y,
                                                    const double2* __restrict__ tw, u32 N, u32 logn, u32 lns,
                                                    int inverse) {
  constexpr int R = 1 << LR;
  const u32 j = blockIdx.x * BS + threadIdx.x, bi = blockIdx.y;
  const u32 stride = N >> LR, k = j & ((1u << lns) - 1);
  if (j >= stride) return;   // N / R < BS for the smallest rings
  const double2* xi = x + (size_t)bi * N;
  double2* yo = y + (size_t)bi * N;
  const u32 tsh = logn - LR - lns;   // W^(t k) = exp(-2 pi i (t k 2^tsh) / N)
  double2 v[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const double2 a = xi[j + t * stride];
    if (t == 0) {
      v[t] = a;
    } else {
      double2 w = tw[(size_t)(t * k) << tsh];
      if (inverse) w.y = -w.y;
      v[t] = make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
    }
  }
  dft_regs<R>(v, inverse != 0);
  const u32 o = ((j >> lns) << (lns + LR)) | k;
#pragma unroll
  for (int t = 0; t < R; ++t) yo[o + (t << lns)] = v[t];
}

// grid (N/BS, n): M_k = round_half_away(scale Re(zeta^-k V_k) / N), residues
// over q_0..q_{nl-1}: pt[b][i][k].
__global__ void __launch_bounds__(BS) k_cl_round(const double2* __restrict__ V, const double2* __restrict__ twist,
                                                 u64* __restrict__ pt, const PrimeConst* __restrict__ pc, u32 N,
                                                 u32 nl, double scale_over_n) {
  const u32 k = blockIdx.x * BS + threadIdx.x, b = blockIdx.y;
  const double2 v = V[(size_t)b * N + k], t = twist[k];
  const double m = (t.x * v.x + t.y * v.y) * scale_over_n;   // Re(conj(t) v) scale / N
  const double r = round(m);                                 // half away from zero
  const int64_t M = (int64_t)r;
  u64* o = pt + (size_t)b * nl * N + k;
  for (u32 i = 0; i < nl; ++i) o[(size_t)i * N] = signed_residue(M, pc[i]);
}

// grid (N/BS, nl, n): residues of v, m + e0, e1 over q_i into res[b][0..2][i].
__global__ void __launch_bounds__(BS) k_cl_enc_lift(const u64* __restrict__ pt, const int32_t* __restrict__ noise,
                                                    u64* __restrict__ res, const PrimeConst* __restrict__ pc,
                                                    u32 N, u32 nl) {
  const u32 k = blockIdx.x * BS + threadIdx.x, i = blockIdx.y, b = blockIdx.z;
  const PrimeConst P = pc[i];
  const int32_t* nz = noise + (size_t)b * 3 * N;
  const size_t plane = (size_t)nl * N;
  u64* r = res + (size_t)b * 3 * plane + (size_t)i * N + k;
  r[0] = signed_residue(nz[k], P);
  r[plane] = add_mod(pt[(size_t)b * plane + (size_t)i * N + k], signed_residue(nz[N + k], P), P.q);
  r[2 * plane] = signed_residue(nz[2 * N + k], P);
}

// grid (N/BS, nl, n), NTT domain: c0 = v b + (m + e0), c1 = v a + e1.
__global__ void __launch_bounds__(BS) k_cl_enc_combine(const u64* __restrict__ res, const u64* __restrict__ pk,
                                                       Items out, const PrimeConst* __restrict__ pc, u32 N, u32 nl,
                                                       u32 nq) {
  const u32 k = blockIdx.x * BS + threadIdx.x, i = blockIdx.y, b = blockIdx.z;
  const PrimeConst P = pc[i];
  const size_t plane = (size_t)nl * N, at = (size_t)i * N + k;
  const u64* r = res + (size_t)b * 3 * plane + at;
  const u64 v = r[0];
  const u64 vb = redc(mul_wide(v, pk[at]), P.q, P.qneg);
  const u64 va = redc(mul_wide(v, pk[(size_t)nq * N + at]), P.q, P.qneg);
  out.p[b][at] = add_mod(vb, r[plane], P.q);
  out.p[b][plane + at] = add_mod(va, r[2 * plane], P.q);
}

// grid (N/BS, nl, n), NTT domain: m = c0 + c1 s.
__global__ void __launch_bounds__(BS) k_cl_dec_mul(Items in, const u64* __restrict__ sk, u64* __restrict__ pt,
                                                   const PrimeConst* __restrict__ pc, u32 N, u32 nl) {
  const u32 k = blockIdx.x * BS + threadIdx.x, i = blockIdx.y, b = blockIdx.z;
  const PrimeConst P = pc[i];
  const size_t plane = (size_t)nl * N, at = (size_t)i * N + k;
  const u64 c0 = in.p[b][at], c1 = in.p[b][plane + at];
  pt[(size_t)b * plane + at] = add_mod(c0, redc(mul_wide(c1, sk[at]), P.q, P.qneg), P.q);
}

// Exact centred lift of one coefficient from its residues x_i (i < nl) and
// the product with zeta^k / scale.  Mixed-radix (Garner) digits a_i of
// X = sum_i a_i q_0...q_{i-1} in [0, Q); the digits of Q - X follow by
// complementing (q_i - 1 - a_i) and adding 1 with carries.  The smaller of X
// and Q - X (compared digit by digit from the top) is the magnitude of the
// centred value, evaluated by Horner in double (its relative error is a few
// units in the last place whatever the size of Q).
template <int MAXL>
__global__ void __launch_bounds__(BS) k_cl_dec_lift(const u64* __restrict__ pt, double2* __restrict__ w,
                                                    const u64* __restrict__ garner, const double2* __restrict__ twist,
                                                    const PrimeConst* __restrict__ pc, u32 N, u32 nl, u32 nq,
                                                    double inv_scale) {
  const u32 k = blockIdx.x * BS + threadIdx.x, b = blockIdx.y;
  const u64* x = pt + (size_t)b * nl * N + k;
  constexpr int U = MAXL <= 16 ? MAXL : 1;   // register-resident digits up to 16 limbs
  u64 a[MAXL], d[MAXL];
#pragma unroll U
  for (int i = 0; i < MAXL; ++i) {
    if (i < (int)nl) {
      const PrimeConst P = pc[i];
      u64 t = x[(size_t)i * N];
#pragma unroll U
      for (int j = 0; j < i; ++j) {
        const u64* g = garner + ((size_t)i * nq + j) * 2;
        t = sub_mod(t, reduce64(a[j], P.q, P.mu), P.q);
        t = shoup(t, g[0], g[1], P.q);
      }
      a[i] = t;
    }
  }
  u32 carry = 1;
#pragma unroll U
  for (int i = 0; i < MAXL; ++i) {
    if (i < (int)nl) {
      const u64 q = pc[i].q;
      u64 v = q - 1 - a[i] + carry;
      carry = v == q;
      d[i] = carry ? 0 : v;
    }
  }
  bool neg = false;   // X > Q/2: the centred value is -(Q - X)
#pragma unroll U
  for (int i = MAXL - 1; i >= 0; --i) {
    if (i < (int)nl && a[i] != d[i]) {
      neg = a[i] > d[i];
      break;
    }
  }
  double val = 0.0;
#pragma unroll U
  for (int i = MAXL - 1; i >= 0; --i)
    if (i < (int)nl) val = val * (double)pc[i].q + (double)(neg ? d[i] : a[i]);
  const double m = (neg ? -val : val) * inv_scale;
  const double2 t = twist[k];
  w[(size_t)b * N + k] = make_double2(m * t.x, m * t.y);
}

// grid (N/2/BS, n): z[b][j] = vals[b][pos_j]
__global__ void __launch_bounds__(BS) k_cl_gather(const double2* __restrict__ vals, double2* __restrict__ z,
                                                  const u32* __restrict__ pos, u32 N) {
  const u32 j = blockIdx.x * BS + threadIdx.x, b = blockIdx.y;
  z[(size_t)b * (N / 2) + j] = vals[(size_t)b * N + pos[j]];
}

u32 grid_x(u32 work) { return (work + BS - 1) / BS; }

// Length-N FFT of n vectors starting in cl->fa; returns the buffer holding
// the result (fa or fb).  log2 N = 3 a + b: one radix-2^b pass (b > 0), then
// a radix-8 passes.
int fft(he_client* cl, u32 n, bool inverse, double2** result) {
  he_ctx* c = cl->ctx;
  double2 *x = cl->fa, *y = cl->fb;
  u32 lns = 0;
  while (lns < c->log_n) {
    const u32 rem = (c->log_n - lns) % 3, lr = (lns == 0 && rem) ? rem : 3;
    TraceScope ts(c, TK_CLIENT_FFT, (double)n * c->N * 32.0);
    const dim3 g(grid_x(c->N >> lr), n);
    if (lr == 1)
      HE_LAUNCH(ts, k_cl_fft_pass<1>, g, dim3(BS), c->stream, x, y, cl->tw, c->N, c->log_n, lns, (int)inverse);
    else if (lr == 2)
      HE_LAUNCH(ts, k_cl_fft_pass<2>, g, dim3(BS), c->stream, x, y, cl->tw, c->N, c->log_n, lns, (int)inverse);
    else
      HE_LAUNCH(ts, k_cl_fft_pass<3>, g, dim3(BS), c->stream, x, y, cl->tw, c->N, c->log_n, lns, (int)inverse);
    std::swap(x, y);
    lns += lr;
  }
  *result = x;
  return ok();
}

// Forward NTT (inverse = false) or INTT of `rows` limb-polys per item, items
// at base + b stride, row r over prime r mod period.
int ntt_rows(he_ctx* c, u64* base, u32 n, size_t stride, u32 rows, u32 period, bool inverse) {
  PolyBatch pb;
  std::memset(&pb, 0, sizeof(pb));
  pb.nitems = n;
  pb.npoly = rows;
  pb.src[0] = pb.dst[0] = base;
  pb.stride = stride;
  for (u32 r = 0; r < rows; ++r) pb.prime[r] = (uint8_t)(r % period);
  return launch_ntt(c, pb, inverse);
}

int upload_ntt_mont(he_client* cl, u64* dst, u32 rows) {
  he_ctx* c = cl->ctx;
  int rc = ntt_rows(c, dst, 1, 0, rows, c->nq, false);
  if (rc) return rc;
  hipLaunchKernelGGL(k_cl_to_mont, dim3(c->N / BS, rows), dim3(BS), 0, c->stream, dst, c->d_pc, c->N, c->nq);
  return ok();
}

template <typename T>
int dev_alloc(T** p, size_t count) {
  HE_HIP(hipMalloc((void**)p, count * sizeof(T)));
  return HE_OK;
}

u64 mulmod_host(u64 a, u64 b, u64 q) { return (u64)((unsigned __int128)a * b % q); }
u64 powmod_host(u64 a, u64 e, u64 q) {
  u64 r = 1;
  for (a %= q; e; e >>= 1, a = mulmod_host(a, a, q))
    if (e & 1) r = mulmod_host(r, a, q);
  return r;
}

}  // namespace

extern "C" {

int he_client_destroy(he_client* cl) {
  if (!cl) return HE_EINVAL;
  if (cl->ctx) hipStreamSynchronize(cl->ctx->stream);
  for (void* p : {(void*)cl->pk, (void*)cl->sk, (void*)cl->tw, (void*)cl->twist, (void*)cl->pos, (void*)cl->garner,
                  (void*)cl->fa, (void*)cl->fb, (void*)cl->res})
    if (p) hipFree(p);
  delete cl;
  return HE_OK;
}

int he_client_create(he_ctx* c, uint32_t max_batch, const uint64_t* pk_host, const int64_t* sk_host,
                     he_client** out) {
  if (!c || !out || max_batch == 0 || max_batch > HE_MAXB) return HE_EINVAL;
  *out = nullptr;
  const u32 N = c->N, nq = c->nq;
  if (sk_host)
    for (u32 k = 0; k < N; ++k)
      if (sk_host[k] < -1 || sk_host[k] > 1) return HE_EINVAL;
  if (pk_host)
    for (u32 r = 0; r < 2 * nq; ++r)
      for (u32 k = 0; k < N; ++k)
        if (pk_host[(size_t)r * N + k] >= c->primes[r % nq]) return HE_EINVAL;
  he_client* cl = new he_client;
  cl->ctx = c;
  cl->max_batch = max_batch;
  int rc = HE_OK;
  auto fail = [&](int e) { he_client_destroy(cl); return e; };

  // host tables: FFT twiddles, the twist zeta^k, slot positions, Garner inverses
  std::vector<double2> tw(N), twist(N);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (u32 k = 0; k < N; ++k) {
    const long double a = -2.0L * pi * (long double)k / (long double)N;
    tw[k] = make_double2((double)cosl(a), (double)sinl(a));
  }
  for (u32 k = 0; k < N; ++k) {
    const long double a = pi * (long double)k / (long double)N;
    twist[k] = make_double2((double)cosl(a), (double)sinl(a));
  }
  std::vector<u32> pos(N / 2);
  u64 e = 1;
  for (u32 j = 0; j < N / 2; ++j) {
    pos[j] = (u32)((e - 1) / 2);
    e = e * 5 % (2ull * N);
  }
  std::vector<u64> garner((size_t)nq * nq * 2, 0);
  for (u32 i = 0; i < nq; ++i)
    for (u32 j = 0; j < i; ++j) {
      const u64 q = c->primes[i];
      const u64 inv = powmod_host(c->primes[j] % q, q - 2, q);
      garner[((size_t)i * nq + j) * 2] = inv;
      garner[((size_t)i * nq + j) * 2 + 1] = (u64)(((unsigned __int128)inv << 64) / q);
    }

  if ((rc = dev_alloc(&cl->tw, N)) || (rc = dev_alloc(&cl->twist, N)) || (rc = dev_alloc(&cl->pos, N / 2)) ||
      (rc = dev_alloc(&cl->garner, garner.size())) || (rc = dev_alloc(&cl->fa, (size_t)max_batch * N)) ||
      (rc = dev_alloc(&cl->fb, (size_t)max_batch * N)))
    return fail(rc);
  if (hipMemcpyAsync(cl->tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(cl->twist, twist.data(), twist.size() * sizeof(double2), hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(cl->pos, pos.data(), pos.size() * sizeof(u32), hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(cl->garner, garner.data(), garner.size() * sizeof(u64), hipMemcpyHostToDevice, c->stream))
    return fail(HE_EDEVICE);

  const size_t limbs_words = (size_t)nq * N;
  if (pk_host) {
    if ((rc = dev_alloc(&cl->pk, 2 * limbs_words)) || (rc = dev_alloc(&cl->res, (size_t)max_batch * 3 * limbs_words)))
      return fail(rc);
    if (hipMemcpyAsync(cl->pk, pk_host, 2 * limbs_words * sizeof(u64), hipMemcpyHostToDevice, c->stream))
      return fail(HE_EDEVICE);
    if ((rc = upload_ntt_mont(cl, cl->pk, 2 * nq))) return fail(rc);
  }
  if (sk_host) {
    int64_t* s_dev = nullptr;
    if ((rc = dev_alloc(&cl->sk, limbs_words)) || (rc = dev_alloc(&s_dev, N))) {
      if (s_dev) hipFree(s_dev);
      return fail(rc);
    }
    if (hipMemcpyAsync(s_dev, sk_host, (size_t)N * sizeof(int64_t), hipMemcpyHostToDevice, c->stream)) {
      hipFree(s_dev);
      return fail(HE_EDEVICE);
    }
    hipLaunchKernelGGL(k_cl_signed_rns, dim3(N / BS, nq), dim3(BS), 0, c->stream, s_dev, cl->sk, c->d_pc, N);
    rc = ok();
    if (!rc) rc = upload_ntt_mont(cl, cl->sk, nq);
    hipStreamSynchronize(c->stream);
    hipFree(s_dev);
    if (rc) return fail(rc);
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(HE_EDEVICE);
  *out = cl;
  return HE_OK;
}

int he_encode(he_client* cl, uint32_t n, const double* slots, double scale, uint32_t level, uint64_t* pt) {
  if (!cl || ((!slots || !pt) && n) || n > cl->max_batch) return HE_EINVAL;
  if (((uintptr_t)slots & 15) || ((uintptr_t)pt & 7)) return HE_EINVAL;
  he_ctx* c = cl->ctx;
  if (level >= c->nq) return HE_ELEVEL;
  if (!(scale > 0.0) || !std::isfinite(scale)) return HE_EINVAL;
  if (n == 0) return HE_OK;
  const u32 N = c->N;
  {
    TraceScope ts(c, TK_CLIENT_ELEM, (double)n * N * 24.0);
    HE_LAUNCH(ts, k_cl_scatter, dim3(grid_x(N / 2), n), dim3(BS), c->stream, (const double2*)slots, cl->fa, cl->pos,
              N);
  }
  double2* V = nullptr;
  int rc = fft(cl, n, false, &V);
  if (rc) return rc;
  TraceScope ts(c, TK_CLIENT_ELEM, (double)n * N * (32.0 + 8.0 * (level + 1)));
  HE_LAUNCH(ts, k_cl_round, dim3(N / BS, n), dim3(BS), c->stream, V, cl->twist, pt, c->d_pc, N, level + 1,
            scale / (double)N);
  return ok();
}

int he_encrypt(he_client* cl, uint32_t n, const uint64_t* pt, const int32_t* noise, uint32_t level, double scale,
               he_ct* out) {
  if (!cl || ((!pt || !noise || !out) && n) || n > cl->max_batch) return HE_EINVAL;
  he_ctx* c = cl->ctx;
  if (level >= c->nq) return HE_ELEVEL;
  if (!cl->pk) return HE_ENOKEY;
  if (n == 0) return HE_OK;
  const u32 N = c->N, nl = level + 1;
  Items o;
  o.n = n;
  for (u32 b = 0; b < n; ++b) {
    if (!out[b].dev) return HE_EINVAL;
    o.p[b] = out[b].dev;
  }
  {
    TraceScope ts(c, TK_CLIENT_ELEM, (double)n * ((double)nl * N * 8.0 * 4.0 + 12.0 * N));
    HE_LAUNCH(ts, k_cl_enc_lift, dim3(N / BS, nl, n), dim3(BS), c->stream, pt, noise, cl->res, c->d_pc, N, nl);
  }
  int rc = ntt_rows(c, cl->res, n, (size_t)3 * nl * N, 3 * nl, nl, false);
  if (rc) return rc;
  {
    TraceScope ts(c, TK_CLIENT_ELEM, (double)n * nl * N * 8.0 * 5.0 + 2.0 * nl * N * 8.0);
    HE_LAUNCH(ts, k_cl_enc_combine, dim3(N / BS, nl, n), dim3(BS), c->stream, cl->res, cl->pk, o, c->d_pc, N, nl,
              c->nq);
  }
  if ((rc = ok())) return rc;
  for (u32 b = 0; b < n; ++b) {
    out[b].level = level;
    out[b].scale = scale;
  }
  return HE_OK;
}

int he_decrypt(he_client* cl, uint32_t n, const he_ct* in, uint64_t* pt) {
  if (!cl || ((!in || !pt) && n) || n > cl->max_batch) return HE_EINVAL;
  he_ctx* c = cl->ctx;
  if (!cl->sk) return HE_ENOKEY;
  if (n == 0) return HE_OK;
  const u32 level = in[0].level;
  if (level >= c->nq) return HE_ELEVEL;
  Items it;
  it.n = n;
  for (u32 b = 0; b < n; ++b) {
    if (!in[b].dev) return HE_EINVAL;
    if (in[b].level != level) return HE_ELEVEL;
    it.p[b] = in[b].dev;
  }
  const u32 N = c->N, nl = level + 1;
  {
    TraceScope ts(c, TK_CLIENT_ELEM, (double)n * nl * N * 8.0 * 3.0 + (double)nl * N * 8.0);
    HE_LAUNCH(ts, k_cl_dec_mul, dim3(N / BS, nl, n), dim3(BS), c->stream, it, cl->sk, pt, c->d_pc, N, nl);
  }
  int rc = ok();
  if (rc) return rc;
  return ntt_rows(c, pt, n, (size_t)nl * N, nl, nl, true);
}

int he_decode(he_client* cl, uint32_t n, const uint64_t* pt, uint32_t level, double scale, double* slots) {
  if (!cl || ((!pt || !slots) && n) || n > cl->max_batch) return HE_EINVAL;
  if (((uintptr_t)slots & 15) || ((uintptr_t)pt & 7)) return HE_EINVAL;
  he_ctx* c = cl->ctx;
  if (level >= c->nq) return HE_ELEVEL;
  if (!(scale > 0.0) || !std::isfinite(scale)) return HE_EINVAL;
  if (n == 0) return HE_OK;
  const u32 N = c->N, nl = level + 1;
  {
    TraceScope ts(c, TK_CLIENT_ELEM, (double)n * N * (8.0 * nl + 16.0));
    const dim3 g(N / BS, n);
    if (nl <= 4)
      HE_LAUNCH(ts, k_cl_dec_lift<4>, g, dim3(BS), c->stream, pt, cl->fa, cl->garner, cl->twist, c->d_pc, N, nl,
                c->nq, 1.0 / scale);
    else if (nl <= 8)
      HE_LAUNCH(ts, k_cl_dec_lift<8>, g, dim3(BS), c->stream, pt, cl->fa, cl->garner, cl->twist, c->d_pc, N, nl,
                c->nq, 1.0 / scale);
    else if (nl <= 16)
      HE_LAUNCH(ts, k_cl_dec_lift<16>, g, dim3(BS), c->stream, pt, cl->fa, cl->garner, cl->twist, c->d_pc, N, nl,
                c->nq, 1.0 / scale);
    else
      HE_LAUNCH(ts, k_cl_dec_lift<HE_MAXP>, g, dim3(BS), c->stream, pt, cl->fa, cl->garner, cl->twist, c->d_pc, N,
                nl, c->nq, 1.0 / scale);
  }
  double2* vals = nullptr;
  int rc = fft(cl, n, true, &vals);
  if (rc) return rc;
  TraceScope ts(c, TK_CLIENT_ELEM, (double)n * N * 16.0);
  HE_LAUNCH(ts, k_cl_gather, dim3(grid_x(N / 2), n), dim3(BS), c->stream, vals, (double2*)slots, cl->pos, N);
  return ok();
}

}  // extern "C"
