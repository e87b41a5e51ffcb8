/* he.h -- C ABI of the MI355X library for encrypted dense-network inference
 * over RNS-CKKS (homomorphic evaluation of y = W x + b and x^2 on slot-packed
 * ciphertexts).
 *
 * Paper: "Secure Human Action Recognition by Encrypted Neural Network
 * Inference", Methods.  The cloud holds only evaluation keys and the
 * cleartext model, receives encrypted inputs and returns one encrypted result;
 * it never holds the secret key and never decrypts (Methods, "Threat model";
 * Results, the three-party protocol).  Hence no evaluation call takes a key
 * of the parties, samples randomness, encrypts or decrypts.  The client
 * section at the end (he_client_*) serves the parties that do: it keeps pk
 * and/or sk in an object of its own, apart from the evaluation context.
 *
 * Conventions shared by every call
 * --------------------------------
 * Return value: 0 (HE_OK) or a negative HE_E* code; he_strerror() names it.
 * Argument checks run synchronously on the host before anything is enqueued;
 * a failed check enqueues nothing and leaves every output untouched.
 *
 * Ring: R_Q = Z_Q[X]/(X^N + 1), N = 2^log_n, 2^10 <= N <= 2^17, N/2 slots.
 * Primes: q_0..q_L (ciphertext modulus chain) and p_0..p_{K-1} (special
 * primes of hybrid key switching), all distinct, prime, = 1 mod 2N, < 2^61.
 * Decomposition: digits of alpha consecutive q-primes starting at q_0,
 * dnum = ceil((L+1)/alpha), alpha <= K.
 *
 * Interchange format (host <-> library): COEFFICIENT form, limb-major, every
 * residue in [0, q).  A polynomial over primes r_0..r_{m-1} is
 * uint64[m][N]; a ciphertext at level l is uint64[2][l+1][N] = (c0, c1) with
 * decryption c0 + c1*s mod Q_l.  Coefficient form is the unique
 * representation, so outputs can be compared bit for bit with any other
 * implementation of the same steps.
 *
 * Device format: ciphertexts live in caller-owned device memory (he_ct.dev)
 * in the library's internal NTT (evaluation) form, same [2][l+1][N] shape.
 * The caller owns ALL device memory (ciphertexts, key storage, plaintext
 * storage, workspace); the library owns only its host tables and small
 * device tables allocated by he_ctx_create and freed by he_ctx_destroy.
 *
 * Streams: every evaluation call enqueues on the context's HIP stream and
 * returns without waiting; device faults surface at he_sync / he_ct_export.
 *
 * Rotations: rho^r rotates the slot vector LEFT by r (Methods,
 * "Single-channel homomorphic convolutions"); slot j sits at the root
 * zeta^(5^j mod 2N), so rho^r is the automorphism X -> X^(5^(r mod N/2)).
 * Key switching is the hybrid RNS method: ModUp of each digit, inner product
 * with the key, ModDown (Methods, "Algorithmic and cryptographic
 * optimizations": RNS variant of CKKS, hoisting).
 *
 * Not thread-safe per context: calls on one he_ctx must not overlap.
 */
#ifndef HE_H_
#define HE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HE_OK        0
#define HE_EINVAL   (-1)   /* null pointer, bad shape (m does not divide n, ...) */
#define HE_EPARAM   (-2)   /* bad ring parameters */
#define HE_ENOKEY   (-3)   /* missing rotation key / relinearisation key */
#define HE_ELEVEL   (-4)   /* rescale at level 0, operands at different levels */
#define HE_ESCALE   (-5)   /* operand scales differ by more than 2^-30 relative */
#define HE_ENOMEM   (-6)   /* workspace, key or plaintext buffer too small */
#define HE_EDEVICE  (-7)   /* HIP runtime error */
#define HE_ESTATE   (-8)   /* context not bound to a workspace / keys not loaded */

#define HE_MAX_BATCH 64    /* ciphertexts per batched call */
#define HE_MAX_PRIMES 64   /* L+1+K */

typedef struct he_ctx he_ctx;
typedef struct he_dense he_dense;

/* A ciphertext handle.  dev: caller-owned device buffer of at least
 * he_ct_bytes(ctx, level) bytes holding [2][level+1][N] words in NTT form.
 * scale: the CKKS scaling factor (IEEE double), tracked by every call. */
typedef struct {
  uint64_t* dev;
  uint32_t level;
  double scale;
} he_ct;

typedef struct {
  uint32_t log_n;         /* N = 2^log_n */
  uint32_t n_q;           /* L + 1 */
  const uint64_t* q;      /* q_0..q_L */
  uint32_t n_p;           /* K */
  const uint64_t* p;      /* p_0..p_{K-1} */
  uint32_t alpha;         /* primes per digit (1 <= alpha <= K) */
} he_params;

const char* he_strerror(int code);
/* Text of the last HIP runtime failure seen by this thread (the failing call
 * and hipGetErrorString), or "" if none; valid until the next library call
 * on the same thread. */
const char* he_last_error(void);

/* Prime selection helper (parameter set-up, host only): the `count` largest
 * primes 2^bits + 1 - k*2N (k >= 1) that are not listed in taken[0..n_taken),
 * in descending order, written to out[0..count).  bits in [20, 61]. */
int he_gen_primes(uint32_t log_n, uint32_t bits, uint32_t count, const uint64_t* taken, uint32_t n_taken,
                  uint64_t* out);

/* Validates params (HE_EPARAM on failure), builds NTT, base-conversion and
 * rescale tables, uploads them.  hip_stream: a hipStream_t (NULL = default
 * stream).  *out receives the handle. */
int he_ctx_create(const he_params* params, void* hip_stream, he_ctx** out);
int he_ctx_destroy(he_ctx* ctx);
int he_ctx_set_stream(he_ctx* ctx, void* hip_stream);

/* Graph capture of a sequence of calls (the batching of the method's
 * Discussion, many requests per launch sequence, replayed at one launch per
 * sequence).  he_graph_begin starts capturing the context's stream
 * (thread-local capture mode): every later call on this context until
 * he_graph_end records its kernels and copies into a HIP graph instead of
 * running them; he_graph_end ends the capture and instantiates the graph
 * into *out (caller-owned, freed with he_graph_free).  he_graph_launch runs
 * it on the context's current stream; it reads and writes the same device
 * buffers as the captured calls did, which the caller keeps allocated and
 * at the same levels and scales.  The captured calls must allocate nothing
 * (workspace bound before) and issue no memset; the tracer is inactive while
 * capturing.  HE_ESTATE when the context uses the legacy default stream
 * (which cannot be captured), HE_EDEVICE when the runtime refuses the capture
 * or a captured call failed (the capture is then discarded). */
typedef struct he_graph he_graph;
int he_graph_begin(he_ctx* ctx);
int he_graph_end(he_ctx* ctx, he_graph** out);
int he_graph_launch(he_ctx* ctx, const he_graph* graph);
int he_graph_free(he_graph* graph);

/* Sizes in bytes of caller-owned device buffers. */
size_t he_ct_bytes(const he_ctx* ctx, uint32_t level);
/* Key storage for the relinearisation key plus n_rot rotation keys. */
size_t he_key_bytes(const he_ctx* ctx, uint32_t n_rot);
/* Workspace for batched calls of up to max_batch ciphertexts and dense
 * layers with baby-step count <= max_n1 (at most 65) and giant-step count
 * <= max_n2.  The key-switch buffers hold min(max_n1 - 1, 64) rotation steps
 * of max_batch ciphertexts at once (one launch per stage for all of them);
 * hoisted rotations beyond that run in groups. */
size_t he_workspace_bytes(const he_ctx* ctx, uint32_t max_batch, uint32_t max_n1, uint32_t max_n2);
/* Plaintext storage of one dense layer (m diagonals at `level`, + bias). */
size_t he_dense_bytes(const he_ctx* ctx, uint32_t level, uint32_t m, int has_bias);

/* Binds caller-owned scratch (device, 256-byte aligned).  No evaluation call
 * allocates device memory; all temporaries live here.  The limits passed to
 * he_workspace_bytes are recorded and enforced (HE_ENOMEM beyond them). */
int he_ctx_bind(he_ctx* ctx, void* workspace_dev, size_t bytes, uint32_t max_batch, uint32_t max_n1,
                uint32_t max_n2);

/* Uploads evaluation keys (host, coefficient form) into caller-owned device
 * storage key_dev (>= he_key_bytes(ctx, n_rot)), converting to the internal
 * form.  Each key: uint64[dnum][2][L+1+K][N] = per digit (b_j, a_j) over
 * q_0..q_L then p_0..p_{K-1}, with b_j = -a_j s + e_j + g_j s' and gadget
 * g_j = P (Q/Q_j) [(Q/Q_j)^{-1}]_{Q_j}.  relin (s' = s^2) may be NULL if
 * he_square is never called.  rot[u] is the key of the left rotation by
 * steps[u] (s' = s(X^(5^steps[u]))).  Stored per key: the NTT form, then
 * the Shoup companions floor(w 2^64 / q) of its words (2x the host size).
 * Synchronous; replaces earlier keys. */
int he_load_keys(he_ctx* ctx, const uint64_t* relin, uint32_t n_rot, const int32_t* steps,
                 const uint64_t* const* rot, void* key_dev, size_t key_bytes);

/* Uploads one dense layer y = W x + b (W: m x n, m | n, n | N/2, powers of
 * two, n1 | m) in the baby-step/giant-step form (Methods, "Algorithmic and
 * cryptographic optimizations", baby-step strategy with
 * rho^(a+b) = rho^a o rho^b):
 *   pt_diag: host uint64[m][level+1][N], coefficient form; entry k = n1*j + i
 *            encodes the k-th hybrid diagonal d_k[s] = W[s mod m][(s+k) mod n]
 *            pre-rotated by -n1*j and replicated with period n, at scale
 *            pt_scale, over q_0..q_level only (level-aware encoding).
 *   bias:    host uint64[level+1][N] (the bias replicated with period m, at
 *            scale bias_scale) or NULL.
 * dev: caller-owned device storage >= he_dense_bytes(ctx, level, m, bias!=0):
 *      the diagonals in NTT form, their Shoup companions floor(w 2^64 / q)
 *      (same shape), then the bias in NTT form.
 * *out receives a host handle (free with he_dense_free). Synchronous. */
int he_dense_load(he_ctx* ctx, uint32_t level, uint32_t m, uint32_t n, uint32_t n1, const uint64_t* pt_diag,
                  const uint64_t* bias, double pt_scale, double bias_scale, void* dev, size_t bytes,
                  he_dense** out);
int he_dense_free(he_dense* d);

/* Lazy-ModDown form of a dense layer (double hoisting; an evaluation order
 * the paper does not use, chosen per layer as a plan parameter because it
 * changes the rounding).  With flags = HE_DENSE_QP, pt_diag is
 * uint64[m][level+1+K][N]: the same integer diagonals reduced over
 * q_0..q_level then p_0..p_{K-1}.  he_eval_dense(_batch) then keeps every
 * baby-step rotation over Q_level u P without its ModDown,
 *   r_0 = (P c0, P c1),  r_i = (P sigma_i(c0) + u_b, u_a)  ((u_b, u_a): the
 *   key-switch inner product of c1 for step i over Q_level u P),
 * forms s_j = ModDown(sum_i MultPlain(r_i, pt_{n1 j + i})) (both
 * polynomials; one ModDown per inner sum instead of one per baby step), and
 * continues with the giant steps, rotate-and-sum and bias as above.  The
 * bias stays uint64[level+1][N].
 * flags |= HE_DENSE_RS(b), 1 <= b <= HE_DENSE_RS_MAX: the rotate-and-sum is
 * hoisted (the paper's hoisting applied to it; also a plan parameter, as it
 * changes the rounding): the n/m shifted copies are summed over the log2(n/m)
 * bits of the shift index in groups of b bits, most significant first; a group
 * of b' bits with base shift t sets z <- ModDown(sum_{k < 2^b'} rho^{k t}(z)),
 * every rotation of the group from one ModUp of z and kept over Q_level u P
 * until that single ModDown (so keys for the amounts k t are needed).  b = 1
 * gives exactly the sequential steps.  flags = 0 is he_dense_load /
 * he_dense_bytes; other bits: HE_EINVAL.  dev: the diagonals (NTT form), their
 * Shoup companions, then the bias, as above. */
#define HE_DENSE_QP 1u
#define HE_DENSE_RS_SHIFT 8
#define HE_DENSE_RS_MAX 6
#define HE_DENSE_RS(b) ((uint32_t)(b) << HE_DENSE_RS_SHIFT)
size_t he_dense_bytes_ex(const he_ctx* ctx, uint32_t level, uint32_t m, int has_bias, uint32_t flags);
int he_dense_load_ex(he_ctx* ctx, uint32_t level, uint32_t m, uint32_t n, uint32_t n1, const uint64_t* pt_diag,
                     const uint64_t* bias, double pt_scale, double bias_scale, uint32_t flags, void* dev,
                     size_t bytes, he_dense** out);

/* Multi-input linear transform in baby-step/giant-step form: the paper's
 * multi-channel homomorphic convolution (Methods, "Single-channel homomorphic
 * convolutions" and the multi-channel equation after it, in the baby-step
 * strategy of "Algorithmic and cryptographic optimizations": rotate each
 * input by the kernel offsets, multiply by plaintexts pre-rotated by the
 * channel offsets, sum, rotate by the channel offsets, sum):
 *   out[j] = sum_{g < n_giant} rho^{giant[g]}( sum_{i < n_in} sum_{b < n_baby}
 *                                pt[g][j][i][b] (.) rho^{baby[b]}(in[i]) ),   j < n_out.
 * baby: rotation amounts (0 = the input itself); giant[0] must be 0, the other
 * giant amounts non-trivial rotations.  n_in n_baby <= 64, n_giant <= 64.
 * pts: host uint64[n_giant][n_out][n_in][n_baby][level+1][N], coefficient
 * form, encoded at pt_scale over q_0..q_level.  dev: caller-owned device
 * storage >= he_linear_bytes(...): the plaintexts in NTT form, then their
 * Shoup companions.  *out: host handle (free with he_linear_free).
 * Synchronous. */
typedef struct he_linear he_linear;
size_t he_linear_bytes(const he_ctx* ctx, uint32_t level, uint32_t n_out, uint32_t n_giant, uint32_t n_in,
                       uint32_t n_baby);
int he_linear_load(he_ctx* ctx, uint32_t level, uint32_t n_out, uint32_t n_giant, uint32_t n_in, uint32_t n_baby,
                   const int32_t* baby, const int32_t* giant, const uint64_t* pts, double pt_scale, void* dev,
                   size_t bytes, he_linear** out);
int he_linear_free(he_linear* t);
/* Caller-owned scratch for he_eval_linear, per request: every input under
 * every baby rotation (he_linear_scratch_bytes(ctx, level, n_in, n_baby)
 * bytes, device). */
size_t he_linear_scratch_bytes(const he_ctx* ctx, uint32_t level, uint32_t n_in, uint32_t n_baby);
/* Evaluates the transform on in[0..n_in) (equal level = the plaintexts' level,
 * equal scale) into out[0..n_out) (scale in.scale * pt_scale; outputs must
 * not alias inputs).  scratch holds every term (the rotated and the unrotated
 * inputs).  The workspace bound with he_ctx_bind must have
 * max_batch >= n_in, n_out and max_n2 >= n_giant (HE_ENOMEM otherwise); keys
 * for every nonzero rotation amount (HE_ENOKEY).  The baby rotations of all
 * inputs share one ModUp per input; all giant steps of all outputs form one
 * step-batched key switch. */
int he_eval_linear(he_ctx* ctx, const he_ct* in, const he_linear* t, void* scratch, size_t scratch_bytes,
                   he_ct* out);
/* The same for n_req requests sharing the plaintexts (read once per batch):
 * in[r n_in + i], out[r n_out + j]; scratch >= n_req he_linear_scratch_bytes;
 * n_req n_in and n_req n_out <= the bound max_batch.  Each output equals its
 * single-request evaluation bit for bit. */
int he_eval_linear_batch(he_ctx* ctx, uint32_t n_req, const he_ct* in, const he_linear* t, void* scratch,
                         size_t scratch_bytes, he_ct* out);

/* Ciphertext import/export: the encrypted input a user sends to the cloud and
 * the single encrypted result it returns (Methods, "Data encryption": one
 * ciphertext holds the whole padded, replicated input; Results, the three-party
 * protocol: the cloud returns one ciphertext to the monitoring service).
 * he_ct_import: coeff_host = host uint64[2][level+1][N] coefficient residues,
 * each below its prime (not checked: larger words give unspecified residues),
 * level <= L (HE_ELEVEL otherwise); scale is stored as given.  The caller sets
 * inout->dev (>= he_ct_bytes(ctx, level), device, caller-owned); the call
 * converts to NTT form into it and writes inout->level and inout->scale.
 * Blocking (returns after the stream has finished the conversion).
 * he_ct_export: writes host coefficient form [2][level+1][N] to coeff_host
 * (caller-owned); needs a bound workspace (HE_ESTATE; the conversion is
 * staged there); blocking (synchronises the stream, so device faults of
 * earlier calls surface here as HE_EDEVICE).  The _dev variants take
 * caller-owned device coefficient buffers of the same layout and are
 * asynchronous (enqueued on the context's stream; the caller keeps the
 * buffers alive until the stream reaches them). */
int he_ct_import(he_ctx* ctx, const uint64_t* coeff_host, uint32_t level, double scale, he_ct* inout);
int he_ct_export(he_ctx* ctx, const he_ct* ct, uint64_t* coeff_host);
int he_ct_from_coeff_dev(he_ctx* ctx, const uint64_t* coeff_dev, uint32_t level, double scale, he_ct* inout);
int he_ct_to_coeff_dev(he_ctx* ctx, const he_ct* ct, uint64_t* coeff_dev);

/* Dense layer: baby steps rho^i(in) for i < n1 with ONE shared ModUp
 * (hoisting), inner sums s_j = sum_i MultPlain(rho^i(in), pt_{n1 j + i}),
 * giant steps z = s_0 + sum_{j>=1} rho^(n1 j)(s_j) in increasing j,
 * rotate-and-sum z += rho^t(z) for t = n/2, n/4, ..., m, then + bias.
 * No rescale (lazy rescaling: the caller rescales once).
 * out->scale = in->scale * pt_scale; out->level = in->level.
 * Needs rotation keys for every step used.  out->dev must not alias in->dev. */
int he_eval_dense(he_ctx* ctx, const he_ct* in, const he_dense* layer, he_ct* out);
/* Square with relinearisation: the activation between dense layers (Methods,
 * "Non-convolutional layers": the activation is a polynomial of degree 2;
 * x^2 here, a x^2 + b x + c folded into the neighbouring dense layers by the
 * caller).  (c0^2, 2 c0 c1, c1^2), then the hybrid key switch of c1^2 with
 * the relinearisation key (s' = s^2; ModUp of its digits, inner product,
 * ModDown), added to (c0^2, 2 c0 c1).  out->scale = in->scale^2, out->level =
 * in->level; no rescale (lazy rescaling, the caller rescales once).
 * in, out: caller-owned device ciphertexts at one level (out->dev sized for
 * it; out may not alias in).  HE_ENOKEY without a relinearisation key,
 * HE_ESTATE without a bound workspace, HE_EINVAL for null pointers. */
int he_square(he_ctx* ctx, const he_ct* in, he_ct* out);
/* Left slot rotation by step, rho^step (Methods, "Single-channel homomorphic
 * convolutions": rho rotates the slot vector left; rotations use the
 * rotation key of that amount, the hybrid RNS key switch of "Algorithmic and
 * cryptographic optimizations"): ModUp(c1), automorphism X -> X^(5^step) of
 * every extended digit, key inner product over Q_l u P, ModDown, plus the
 * automorphism of c0.  step = 0 mod N/2 copies.  Scale and level unchanged.
 * HE_ENOKEY if no key for step was loaded; out must not alias in. */
int he_rotate(he_ctx* ctx, const he_ct* in, int32_t step, he_ct* out);
/* Hoisted rotations of one ciphertext by steps[0..n_steps) (Methods,
 * "Algorithmic and cryptographic optimizations", hoisting: the decomposition
 * and base extension of c1 are common to every rotation of one ciphertext, so
 * they are computed once): one ModUp shared by all; out[u] =
 * rho^steps[u](in), bit-identical to he_rotate(in, steps[u]).  out: n_steps
 * caller-owned device ciphertexts at in's level, none aliasing in. */
int he_rotate_hoisted(he_ctx* ctx, const he_ct* in, uint32_t n_steps, const int32_t* steps, he_ct* out);
/* Rescale by q_level (Methods, "Algorithmic and cryptographic
 * optimizations", lazy rescaling: once per dense layer and once per square):
 * c_i <- (c_i - (c_level mod q_i)) q_level^{-1} mod q_i (floor form, c_level
 * the coefficient-form residue in [0, q_level)), level - 1, scale / q_level.
 * out may alias in.  HE_ELEVEL at level 0. */
int he_rescale(he_ctx* ctx, const he_ct* in, he_ct* out);
/* Limb-wise sum of two ciphertexts at equal level and scale (the sums of the
 * convolution and dense equations of Methods, "Single-channel homomorphic
 * convolutions").  HE_ELEVEL for different levels, HE_ESCALE for scales
 * further apart than 2^-30 relative; out may alias a or b. */
int he_add(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct* out);

/* Batched forms: n <= HE_MAX_BATCH independent ciphertexts (e.g. from
 * different requests) in one set of launches; keys and plaintexts are read
 * once per batch.  in[i], out[i] obey the single-call rules; all in[i] share
 * one level and one scale.  Results are bit-identical to n single calls. */
int he_eval_dense_batch(he_ctx* ctx, uint32_t n, const he_ct* in, const he_dense* layer, he_ct* out);
int he_square_batch(he_ctx* ctx, uint32_t n, const he_ct* in, he_ct* out);
int he_rescale_batch(he_ctx* ctx, uint32_t n, const he_ct* in, he_ct* out);
/* out[i * n_steps + u] = rho^steps[u](in[i]). */
int he_rotate_hoisted_batch(he_ctx* ctx, uint32_t n, const he_ct* in, uint32_t n_steps, const int32_t* steps,
                            he_ct* out);

/* Rescale that allocates nothing and needs no bound workspace, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  Same arguments, checks
 * and results as he_rescale_batch (bit for bit), except that its temporaries
 * live in a library-owned static device array of HE_NOALLOC_SCRATCH_BYTES per
 * GPU (held until the process ends): n (2 (l+1) + 2 l) N words, plus 2 l N n
 * more when an output aliases its input, at the inputs' level l; HE_ENOMEM
 * beyond the array.  The array is shared by every call on that GPU (all
 * contexts, all streams): calls that overlap on one GPU race and must be
 * ordered by the caller.  HE_ESTATE if no context was created on this GPU. */
#define HE_NOALLOC_SCRATCH_BYTES (64u << 20)
int he_rescale_batch_noalloc(he_ctx* ctx, uint32_t n, const he_ct* in, he_ct* out);

/* Kernel-level entry: negacyclic NTT (inverse != 0: INTT) in place on
 * n_items device buffers, each holding `limbs` consecutive limb-polys for
 * primes first_prime .. first_prime + limbs - 1 (indices into q_0..q_L,
 * p_0..p_{K-1}).  Forward output is the library's NTT order; the inverse
 * maps it back to coefficients.  items: host array of device pointers. */
int he_ntt(he_ctx* ctx, uint32_t n_items, uint64_t* const* items, uint32_t first_prime, uint32_t limbs,
           int inverse);

/* Execution knobs: launch shapes and scheduling choices that never change a
 * result bit (the arithmetic and its reduction points are fixed).  Set by the
 * autotuner.  Keys:
 *   "ntt_chunk_mb"  two-phase NTT: run both phases per chunk of this many MiB
 *                   of polynomials (0 = each phase over the whole batch)
 *   "ntt_cols"      two-phase NTT: sub-transforms per workgroup tile, 8, 16
 *                   (default) or 32
 *   "ntt_cols_b"    the same for the second (row) phase alone: 8, 16, 32, or
 *                   0 (default) = as "ntt_cols"
 *   "ntt_single_pass"  N = 2^15: 1 = one register-resident launch per
 *                   transform (one HBM pass), 0 (default) = two phases
 *   "ks_fuse"       lazy-ModDown dense layers with n2 <= 8: 1 (default) = the
 *                   baby steps' key inner products computed inside the
 *                   inner-sum kernel (never stored), 0 = two launches
 *   "ks_fuse_g"     fused lazy-ModDown inner sums: 1 = half the default
 *                   number of requests per thread (fewer registers), 0
 *                   (default) = 8 / 8 / 4 / 2 requests for 1 / 2 / 4 / 8
 *                   giant sums
 *   "ks_fuse_waves" fused lazy-ModDown inner sums: 3 = the kernel compiled for
 *                   three waves per SIMD, 0 (default) = the compiler's choice
 *   "ks_fuse_lds"   fused lazy-ModDown inner sums: 4, 8 (default) or 16 = the
 *                   form that shares each baby step's key and plaintext words
 *                   through LDS among that many requests per workgroup (a
 *                   wave per request, one position per thread; halved down to
 *                   4 while a batch does not fill it); 0 = the register form
 *                   (requests per thread: ks_fuse_g)
 *   "ks_fuse_min_batch"  smallest batch that takes the LDS-shared form
 *                   (1..64, default 3; smaller batches ks_fuse_one's kernel or
 *                   the register form)
 *   "ks_fuse_orbit" LDS-shared form: 1 (default) = the position blocks
 *                   dealt to each XCD in the order of the cycles of the first
 *                   step's automorphism on blocks (block X reads block P(X)),
 *                   so that the workgroups running together read each
 *                   other's gathers of the step before from L2; 0 = in
 *                   address order
 *   "ks_fuse_one"   batches below ks_fuse_min_batch (with ks_fuse_lds set):
 *                   1 (default) = their own kernel (one request and position
 *                   per thread; on primes below 2^50 the key and plaintext
 *                   words read without their Shoup companions, the key sums
 *                   as exact column sums), 0 = the register form
 *   "ks_fuse_pair"  LDS-shared form with 4 or 8 requests: 1 = each
 *                   workgroup serves two position blocks, X and P(X), so that
 *                   one block's gathers are the other's of the step before;
 *                   0 (default) = one block per workgroup
 *   "trace"         1 = bracket every kernel launch with HIP events on the
 *                   context stream (not while the stream is being captured
 *                   into a graph); read with he_trace_read.  0 = off.
 * Returns HE_EINVAL for an unknown key or a negative value. */
int he_ctx_set_knob(he_ctx* ctx, const char* key, int64_t value);
int he_ctx_get_knob(const he_ctx* ctx, const char* key, int64_t* value);

/* Per-kernel-class totals of the launches traced since the last read
 * (knob "trace"): launches, summed event time in ms, and algorithmic bytes
 * (every word a launch must read or write, counted once).  Synchronises the
 * stream, then resets the trace.  Writes up to `capacity` entries, sets
 * *count to the number of classes seen; HE_ENOMEM if launches were dropped
 * because more than 8192 were traced between reads.  `kernel` points to a
 * static string. */
typedef struct {
  const char* kernel;
  uint64_t launches;
  double ms;
  double bytes;
} he_trace_entry;
int he_trace_read(he_ctx* ctx, he_trace_entry* out, uint32_t capacity, uint32_t* count);

/* Waits for all work enqueued on the context's stream. */
int he_sync(he_ctx* ctx);

/* ----------------------------------------------------------- client side
 * Encoding, encryption, decryption and decoding on the device for the
 * parties that hold keys (the protocol's parties: end-users encrypt with pk,
 * the monitoring service decrypts with sk; Results, "Time requirement of
 * secure action recognition", steps (iii) and (v); Methods, threat model).
 * The evaluation entry points above never take pk or sk.  All calls enqueue
 * on the context's stream and return without waiting.
 *
 * Slots: z in C^(N/2), element j at zeta^(5^j mod 2N), zeta = exp(i pi/N)
 * (the ordering under which rho^r rotates left by r); the plaintext of z at
 * scale D is the integer polynomial with coefficients
 *   M_k = round(D (2/N) Re sum_j z_j zeta^(-5^j k))   (half away from zero),
 * reduced mod each q_i.  Device slot arrays: [n][N/2] complex numbers, each
 * as two doubles (re, im), 16-byte aligned.  Device plaintext arrays:
 * [n][level+1][N] coefficient residues (uint64, item stride (level+1) N
 * words).  HE_EINVAL for misaligned device arrays, n > max_batch, a null
 * array with n > 0, or a scale that is not positive and finite; n = 0 is a
 * no-op. */
typedef struct he_client he_client;
/* pk_host: [2][L+1][N] coefficient residues (b, a) with b = -a s + e, or
 * NULL (no encryption); sk_host: the N secret coefficients in {-1, 0, 1}, or
 * NULL (no decryption); HE_EINVAL for a residue >= its prime or a secret
 * coefficient outside {-1, 0, 1}.  Both are copied to library-owned device memory in
 * NTT form; with scratch for batches of up to max_batch requests
 * (1 <= max_batch <= HE_MAX_BATCH). */
int he_client_create(he_ctx* ctx, uint32_t max_batch, const uint64_t* pk_host, const int64_t* sk_host,
                     he_client** out);
/* Waits for the context's stream, frees the client's device memory.  Destroy
 * every client before its context. */
int he_client_destroy(he_client* cl);
/* Encodes n slot vectors at `scale` into plaintexts over q_0..q_level.  The
 * caller keeps scale * max |z_j| below 2^62 (M_k then fits a signed 64-bit
 * word; larger values give unspecified residues).  The embedding is a
 * double-precision FFT: while |scale m_k| < 2^52 a coefficient can differ by
 * 1 from an exact evaluation of the sum, when its value lies within rounding
 * of a half; above 2^52 the scaled value itself carries the FP64 spacing
 * (2^(e - 52) at magnitude 2^e) and the difference is a few such units. */
int he_encode(he_client* cl, uint32_t n, const double* slots_dev, double scale, uint32_t level,
              uint64_t* pt_dev);
/* Public-key encryption at `level` (pk restricted to q_0..q_level):
 *   c0 = v b + e0 + m,  c1 = v a + e1  (mod q_i),
 * with the random polynomials given by the caller: noise_dev [n][3][N]
 * signed 32-bit coefficients (v, e0, e1), v ternary and e0, e1 small.
 * pt_dev: [n][level+1][N] coefficient residues (he_encode's output);
 * out[r].dev receives ciphertext r (NTT form), level and scale are set.
 * HE_ENOKEY without pk. */
int he_encrypt(he_client* cl, uint32_t n, const uint64_t* pt_dev, const int32_t* noise_dev, uint32_t level,
               double scale, he_ct* out);
/* m = c0 + c1 s (mod q_i, i <= level) of n ciphertexts at one level, as
 * coefficient residues [n][level+1][N] in pt_dev.  HE_ENOKEY without sk. */
int he_decrypt(he_client* cl, uint32_t n, const he_ct* in, uint64_t* pt_dev);
/* Slots of n plaintexts over q_0..q_level at `scale`: each coefficient is
 * lifted exactly to its centred integer in (-Q/2, Q/2] (mixed-radix digits,
 * Q = q_0...q_level), divided by scale, and evaluated at the slot roots by a
 * double-precision FFT.  Writes [n][N/2] complex slots to slots_dev. */
int he_decode(he_client* cl, uint32_t n, const uint64_t* pt_dev, uint32_t level, double scale, double* slots_dev);

#ifdef __cplusplus
}
#endif
#endif /* HE_H_ */
