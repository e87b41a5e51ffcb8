// Launchers of the RNS kernels (rns_kernels.hip).  All run on c->stream.
#pragma once
#include "he_internal.hpp"

// Per-item pointer list (one entry per ciphertext of a batch).
struct Items {
  u32 n = 0;
  u64* p[HE_MAXB];
};

// Copies polys: item b, poly r: dst[b] + (dst_off + r) N <- src[b] + (src_off + r) N
// for every r < npoly with prime[r] != 0xFF.
int launch_copy_polys(he_ctx* c, const PolyBatch& pb);

// ModUp conversion at level l: coef = [B][l+1][N] coefficient form (item
// stride (l+1) N); ext = [B][beta][l+1+K][N]; writes every limb of every digit
// except the digit's own limbs (coefficient form; those stay in the source).
int launch_modup_conv(he_ctx* c, u32 l, u32 nitems, const u64* coef, u64* ext);


// ModDown conversion: u = [B][2][l+1+K][N] with the P-limbs already in
// coefficient form; conv = [B][2][l+1][N] coefficient form.
int launch_moddown_conv(he_ctx* c, u32 l, u32 nitems, const u64* u, u64* conv);

// Final combine of a key switch at level l (NTT domain), item b:
//   out.c0[i] = acc.c0[i] + add0.c0[perm_g(.)][i] + (u_b[i] - conv_b[i]) P^{-1}
//   out.c1[i] = acc.c1[i] + add1[i]                + (u_a[i] - conv_a[i]) P^{-1}
// add0 (a ciphertext whose c0 is permuted by galois), add1 (a polynomial),
// acc (a ciphertext): null entries are skipped.  bias (one polynomial, shared)
// is added to c0 when non-null.
struct FinalArgs {
  u64* out[HE_MAXB];
  const u64* add0[HE_MAXB];
  const u64* add1[HE_MAXB];
  const u64* acc[HE_MAXB];
};
int launch_ks_final(he_ctx* c, u32 l, u32 nitems, const u64* u, const u64* conv, u32 galois, const FinalArgs& fa,
                    const u64* bias);

// Several rotation steps of the same B items in one set of launches (the
// hoisted form: the digits in ext are shared by every step).  Item (s, b) of
// the u / conv workspaces is s B + b.
#define HE_MAX_STEPS 64
struct StepKeys {
  const u64* key[HE_MAX_STEPS];   // key of step s ([dnum][2][L+1+K][N] NTT form, then Shoup companions)
  u32 galois[HE_MAX_STEPS];       // its Galois element g
  u32 galois_inv[HE_MAX_STEPS];   // g^{-1} mod 2N
  // When galois[s] = galois[0]^(s+1) for every s (a run of baby steps or a
  // hoisted rotate-and-sum group): the block orbits of galois[0]'s key
  // (KeySlot::orbit, orbit_even), else null.
  const uint16_t* orbit = nullptr;
  u32 orbit_even = 0;
};
// Source c1 (NTT form) of item (s, b), whose digits' own limbs the inner
// product reads: base + s os + b ob when base is set, else ptr[b] (same for every s).
struct OwnMap {
  u64* ptr[HE_MAXB];
  const u64* base;
  size_t os, ob;
};
// u[s B + b] = key-switch inner product of item (s, b) with key s:
//   u[.][p][t][k'] = sum_j ext[.][j][t][perm_g(k')] * key[j][p][prime(t)][k'],  p in {b, a},
// left lazy: Q-limbs below 32 q_t (read by the epilogues as u + q - conv),
// P-limbs below 4 p_t (inputs of the inverse NTT).  Digits: ext item
// s ext_items + b (ext_items = 0: the steps share item b's digits, the
// hoisted form; = B: one ModUp per (s, b)).
int launch_ks_inner_steps(he_ctx* c, u32 l, u32 B, u32 S, const u64* ext, u32 ext_items, const OwnMap& own,
                          const StepKeys& keys, u64* u);
// Output ciphertext of item (s, b): base + s os + b ob when base is set, else ptr[s B + b] (S B <= HE_MAXB).
struct OutMap {
  u64* ptr[HE_MAXB];
  u64* base;
  size_t os, ob;
};
// ModDown output of Z extended ciphertexts y = [Z][2][l+1+K][N] whose
// conversions (NTT form) are in conv = [Z][2][l+1][N]: out(z) = (y_Q - conv)
// P^{-1} (+ bias on c0 when non-null), out(z) = om.base + z om.ob, or
// om.ptr[z] (Z <= HE_MAXB).
int launch_moddown_final(he_ctx* c, u32 l, u32 Z, const u64* y, const u64* conv, const OutMap& om,
                         const u64* bias);

// Rotation outputs: out(s, b).c0 = add0.p[b].c0[perm_{g_s}(.)] + (u_b - conv_b) P^{-1},
//                   out(s, b).c1 =                               (u_a - conv_a) P^{-1}.
int launch_ks_final_steps(he_ctx* c, u32 l, u32 B, u32 S, const u64* u, const u64* conv, const StepKeys& keys,
                          const Items& add0, const OutMap& om);
// Giant-step sum of B items with J = S steps, om item b (base + b ob or ptr[b]) =
//   s_0(b) + sum_{j=1..J} rho^{g_j}(s_j(b)) (+ bias on c0):
//   s_j(b) = sums + (j B + b) csz, and the key switch of (j, b) in u / conv item (j-1) B + b.
int launch_ks_final_sum(he_ctx* c, u32 l, u32 B, u32 S, const u64* u, const u64* conv, const StepKeys& keys,
                        const u64* sums, const u64* bias, const OutMap& om);

// Baby steps folded into the inner sums: with u / conv holding the key
// switches of baby steps i = 1 .. n1-1 (step s = i - 1) of items b < B,
//   s[j][b] = sum_{i < n1} pts[n1 j + i] (.) r_i(b),   r_0(b) = in.p[b],
//   r_i(b) = the rotation of in.p[b] by i (as launch_ks_final_steps computes it),
// without writing the rotated ciphertexts.  s = [n2][B][2][l+1][N].
int launch_ks_final_multplain(he_ctx* c, u32 l, u32 B, u32 n1, u32 n2, const u64* u, const u64* conv,
                              const StepKeys& keys, const Items& in, const u64* pts, u64* s);

// Inner sums with one baby step (n1 = 1), item b, j < n2:
//   s[j][b] = pts[j] (.) in.p[b]   (both polynomials), s = [n2][B][2][l+1][N];
// pts in NTT form followed by their Shoup companions (he_dense layout), pl
// limbs per diagonal (l+1, or l+1+K for diagonals over Q_l u P: the first
// l+1 are used).
int launch_multplain(he_ctx* c, u32 l, u32 n2, const Items& in, const u64* pts, u32 pl, u64* s);

// Lazy-ModDown inner sums: with u holding the extended key-switch inner
// products of baby steps i = 1 .. n1-1 (step s = i - 1) of items b < B,
//   sqp[j][b] = sum_{i < n1} pts[n1 j + i] (.) r_i(b) over Q_l u P,
//   r_0 = (P c0, P c1), r_i = (P sigma_i(c0) + u_b, u_a),
// pts = [m][l+1+K][N] then companions; sqp = [n2][B][2][l+1+K][N], every limb in [0, q).
int launch_ext_multplain(he_ctx* c, u32 l, u32 B, u32 n1, u32 n2, const u64* u, const StepKeys& keys,
                         const Items& in, const u64* pts, u64* sqp);
// The same inner sums fused with the baby steps' key inner products (digits
// of item b in ext as for launch_ks_inner_steps with ext_items = 0, own limbs
// from own.ptr[b]): one launch, no per-step products in memory.  n1 >= 2,
// n2 in {1, 2, 4, 8}, keys = the n1 - 1 baby steps.  pts = null (n2 = 1): the
// plain sum sqp[b] = sum_{i < n1} r_i(b) (a hoisted rotate-and-sum group).
// Batches of ks_fuse_min_batch or more take the LDS-shared form, smaller ones
// the small-batch kernel (knob ks_fuse_one), else the register form.
// lift: B (l + 1) N words of scratch, free during the call, that the
// LDS-shared form fills with P c0 mod q on the Q-limbs (required there).
// The LDS-shared form of launch_ks_ext_fused (ext_sums_lds.hip) with W
// requests per workgroup (4, 8 or 16), launched inside its trace scope.
int launch_ks_ext_lds(he_ctx* c, u32 l, u32 B, u32 n1, u32 n2, const u64* ext, const OwnMap& own,
                      const StepKeys& keys, const Items& in, const u64* pts, u64* sqp, u32 beta, u32 ne, u32 W,
                      u64* lift, TraceScope& ts);
int launch_ks_ext_fused(he_ctx* c, u32 l, u32 B, u32 n1, u32 n2, const u64* ext, const OwnMap& own,
                        const StepKeys& keys, const Items& in, const u64* pts, u64* sqp, u64* lift);


// Inner sums of a multi-input linear transform for R requests: term t < T of
// request r at x + (r T + t) csz; for o = g n_out + j < NG n_out,
// s(r, o) = sum_t pts[o][t] (.) term(r, t) (both polynomials) at
// s + (g R n_out + r n_out + j) csz.  pts = [NG n_out][T][l+1][N] then
// companions.  T <= 64.
int launch_mp_acc(he_ctx* c, u32 l, u32 R, u32 T, u32 n_out, u32 NG, const u64* x, const u64* pts, u64* s);

// comp[i][r][k] = floor(pts[i][r][k] 2^64 / q) for m arrays of nlimbs limbs,
// limb r over prime r for r <= l, else p_{r-l-1} (the Shoup companions of
// plaintext and key words; exact long division).
int launch_shoup_companion(he_ctx* c, u32 m, u32 nlimbs, u32 l, const u64* pts, u64* comp);

// Tensor for squaring: d01 = [B][2][l+1] (c0^2, 2 c0 c1), d2 = [B][l+1] (c1^2).
int launch_tensor(he_ctx* c, u32 l, const Items& in, u64* d01, u64* d2);

// Rescale helpers.  last = [B][2][l+1][N] whose limb l holds c_l in coefficient form;
// red = [B][2][l][N] receives c_l mod q_i (coefficient form).
int launch_rescale_reduce(he_ctx* c, u32 l, u32 nitems, const u64* last, u64* red);
// out(b) = (in(b) - red) * q_l^{-1} over limbs i < l (NTT domain).
int launch_rescale_final(he_ctx* c, u32 l, const Items& in, const u64* red, const Items& out);

// out = a + b (ciphertexts at level l).
int launch_add(he_ctx* c, u32 l, const Items& a, const Items& b, const Items& out);
// c0(b) += poly (a plaintext at level l, NTT form).
int launch_add_plain(he_ctx* c, u32 l, const Items& ct, const u64* poly);
