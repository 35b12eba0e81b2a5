/*
 * neujeans.h - C ABI of the MI355X (gfx950) library for the fused CinS-conv +
 * CoeffToSlot hot path of NeuJeans (Ju et al., arXiv 2312.04356).
 *
 * Scheme: RNS-CKKS over R = Z[X]/(X^N + 1) (Sec. 2.1-2.4).  Ciphertext moduli
 * q_0..q_L, special moduli p_0..p_{alpha-1}; hybrid key switching with digits of
 * alpha consecutive ciphertext primes (dnum = ceil((L+1)/alpha) at the top level,
 * Table 4).  All primes are = 1 mod 2N and below 2^50.
 *
 * Memory and ownership
 *   - Ciphertext and plaintext buffers are caller-owned DEVICE memory of uint64_t
 *     canonical residues (each word in [0, prime)).  A level-l ciphertext is
 *     [2][l+1][N] (polynomial, limb, coefficient), limb-major, contiguous.  The
 *     library never frees them.
 *   - Device ciphertexts are kept in the library's evaluation form (is_ntt = 1):
 *     every homomorphic call requires and produces that form.  nj_to_coeff /
 *     nj_to_eval convert in place to and from coefficient form (natural order),
 *     the form in which results are compared with other implementations.
 *   - Host arrays passed in are borrowed for the duration of the call.
 *   - Contexts, keys and plans are library-owned; free them with their destroy call.
 *
 * Streams: every device call enqueues on the given hipStream_t (passed as void*,
 * NULL = default stream) and does not synchronise the device, except where noted.
 * Arguments are validated on the host before anything is enqueued.
 *
 * Errors: every call returns nj_status (0 = NJ_OK, negative = error) and never
 * throws; nj_last_error() gives a thread-local message for the last failure.
 */
#ifndef NEUJEANS_H
#define NEUJEANS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NJ_OK = 0,
    NJ_EINVAL = -1,       /* bad argument (null pointer, size, form, unknown id) */
    NJ_ELEVEL = -2,       /* level out of range or mismatched between operands */
    NJ_ESCALE = -3,       /* scale mismatch */
    NJ_ENOKEY = -4,       /* a needed switching key (Galois element) was not generated */
    NJ_EDEVICE = -5,      /* HIP runtime error (message from hipGetErrorString) */
    NJ_ENOMEM = -6,       /* device allocation failed */
    NJ_EUNSUPPORTED = -7  /* parameters outside what the kernels implement */
} nj_status;

typedef struct nj_ctx nj_ctx;   /* ring, primes, transform tables, secret, keys, scratch */
typedef struct nj_plan nj_plan; /* one or more BSGS linear transforms with their diagonals */

typedef struct {
    int log_n;           /* N = 2^log_n, 10 <= log_n <= 16 */
    int n_q;             /* number of ciphertext primes, top level L = n_q - 1, n_q <= 32 */
    int alpha;           /* number of special primes = ciphertext primes per digit, 1..16 */
    const uint64_t *q;   /* host [n_q]: q_0..q_L */
    const uint64_t *p;   /* host [alpha]: p_0..p_{alpha-1} */
    double scale;        /* Delta, the message scale of encoded inputs */
} nj_params;

typedef struct {
    uint64_t *data;      /* device [2][level+1][N] */
    int level;
    int is_ntt;          /* 1 = evaluation form (required by homomorphic calls) */
    double scale;
} nj_ct;

const char *nj_last_error(void);

/* ------------------------------------------------------------ parameters */

/* Prime chain rule: scan t = k*2N + 1 downward from below 2^bits, skip `exclude`,
 * return the first `count` primes (Miller-Rabin, deterministic below 2^64).
 * out: host [count].  NJ_EINVAL if bits > 50 or not enough primes exist. */
nj_status nj_gen_primes(int log_n, int bits, int count, const uint64_t *exclude, int n_exclude, uint64_t *out);

/* Creates a context on the current HIP device: validates primes, builds transform
 * tables and basis-conversion constants, allocates no ciphertext scratch yet.
 * NJ_EUNSUPPORTED (before any device work) for n_q > 32, alpha > 16 or more than 8
 * key-switching digits ceil(n_q / alpha). */
nj_status nj_ctx_create(const nj_params *params, nj_ctx **out);
void nj_ctx_destroy(nj_ctx *ctx);

/* Secret key s, host int8 [N] with entries in {-1, 0, 1} (sparse ternary, Table 4 h). */
nj_status nj_set_secret(nj_ctx *ctx, const int8_t *s);

/* Switching key to s from s' = s(X^g) (rotation / conjugation keys; Sec. 2.1 HRot)
 * or from s' = s^2 when galois_elt == 0 (relinearisation).  Randomness is an input:
 *   a: host uint64 [dnum][L+1+alpha][N], uniform residues in coefficient form,
 *      limbs ordered q_0..q_L, p_0..p_{alpha-1};
 *   e: host int64 [dnum][N], small errors.
 * key_j = (-a_j s + e_j + P g_j s', a_j) with g_j = 1 mod the primes of digit j,
 * 0 mod all others.  Synchronous.  Replaces an existing key for the same element. */
nj_status nj_gen_switch_key(nj_ctx *ctx, uint32_t galois_elt, const uint64_t *a, const int64_t *e);

/* Galois element of a left rotation of the slots by r: 5^r mod 2N. */
uint32_t nj_galois_elt(const nj_ctx *ctx, int r);

/* ------------------------------------------------------------ transforms */

/* In-place negacyclic transform of n_limbs limbs of N words at `data`, limb i taken
 * modulo prime prime_idx[i] (host array; index < n_q selects q_i, n_q + k selects p_k). */
nj_status nj_ntt_limbs(nj_ctx *ctx, uint64_t *data, const int *prime_idx, int n_limbs, int inverse, void *stream);

/* In-place conversion of n_polys level-l polynomials [n_polys][l+1][N] between
 * coefficient form and evaluation form. */
nj_status nj_to_eval(nj_ctx *ctx, uint64_t *data, int level, int n_polys, void *stream);
nj_status nj_to_coeff(nj_ctx *ctx, uint64_t *data, int level, int n_polys, void *stream);

/* ------------------------------------------------------------ encryption */

/* Secret-key encryption at `level` (Sec. 2.1 Enc): (c0, c1) = (-a s + e + m, a).
 *   m: device [(level+1)][N] plaintext residues, coefficient form;
 *   a: host [(level+1)][N] uniform residues (coefficient form); e: host int64 [N].
 * out->data: device [2][level+1][N]; the result is in evaluation form. */
nj_status nj_encrypt_sk(nj_ctx *ctx, const uint64_t *m, int level, const uint64_t *a, const int64_t *e,
                        double scale, nj_ct *out, void *stream);
/* Switching keys in and out of the context (saving and restoring a key set).  A key is
 * nj_key_words(ctx) = dnum * 2 * (L+1+alpha) * N words: [dnum][2][L+1+alpha][N], digit j's
 * (b_j, a_j) over q_0..q_L, p_0..p_{alpha-1}, evaluation form; its values are tied to the
 * context's primes and secret, so only a context of the same parameters and secret can
 * use it.  Galois element 0 is the relinearisation key.
 *   export: NJ_ENOKEY if the context holds no key for g; import: adds or replaces it;
 *   both NJ_EINVAL when words != nj_key_words(ctx).  Synchronous (wait for the device).
 *   nj_key_list: the Galois elements held (up to max of them into gs), their count in n. */
size_t nj_key_words(const nj_ctx *ctx);
nj_status nj_key_export(nj_ctx *ctx, uint32_t galois_elt, uint64_t *host, size_t words);
nj_status nj_key_import(nj_ctx *ctx, uint32_t galois_elt, const uint64_t *host, size_t words);
nj_status nj_key_list(const nj_ctx *ctx, uint32_t *gs, int max, int *n);

/* Public key (Sec. 2.1 KeyGen): pk = (-a s + e, a) over q_0..q_L, kept on the device
 * (evaluation form) until the context is destroyed; a new call replaces it.
 *   a: host [(L+1)][N] uniform residues (coefficient form); e: host int64 [N].
 * Needs the secret (nj_set_secret).  Synchronous. */
nj_status nj_gen_public_key(nj_ctx *ctx, const uint64_t *a, const int64_t *e);
/* Public-key encryption at `level` (Sec. 2.1 Enc(m; pk)):
 * (c0, c1) = (v pk0 + e0 + m, v pk1 + e1) on the first level+1 limbs of pk.
 *   m: device [(level+1)][N] plaintext residues, coefficient form;
 *   v, e0, e1: host int64 [N] small polynomials (v ternary, e0 and e1 errors).
 * out->data: device [2][level+1][N], evaluation form; out->scale = scale.
 * NJ_EINVAL without a public key; NJ_ELEVEL for a level outside 0..L. */
nj_status nj_encrypt_pk(nj_ctx *ctx, const uint64_t *m, int level, const int64_t *v, const int64_t *e0,
                        const int64_t *e1, double scale, nj_ct *out, void *stream);

/* Decryption polynomial c0 + c1 s (Sec. 2.1 Dec): out device [(level+1)][N], coefficient form. */
nj_status nj_decrypt(nj_ctx *ctx, const nj_ct *in, uint64_t *out, void *stream);

/* Plaintext encoding on the host (Sec. 2.2 Slot encoding; Sec. 3.3.1 real CinS):
 *   z: complex slots as interleaved doubles [N/2][2];  out: host int64 [N], the
 *   rounded coefficients round_half_even(scale * f). */
nj_status nj_encode_slots(int log_n, const double *z, double scale, int64_t *out);
/* Real CinS: chans host double [C][2l] (C = N / (2l)), slices of 2l reals each. */
nj_status nj_encode_cins(int log_n, const double *chans, int slice_len2, double scale, int64_t *out);
/* Inverse of nj_encode_slots on centred integer coefficients: z out [N/2][2]. */
nj_status nj_decode_slots(int log_n, const double *coeffs, double scale, double *z);
/* Signed coefficients -> device residues [(level+1)][N] (coefficient form).  Synchronous. */
nj_status nj_upload_plain(nj_ctx *ctx, const int64_t *coeffs, int level, uint64_t *dst, void *stream);

/* ------------------------------------------------------- homomorphic ops */

/* HRot (Sec. 2.1): slots rotated left by r = automorphism 5^r then key switching.  A
 * rotation by a multiple of N/2 slots is the identity (g = 1, below). */
nj_status nj_rotate(nj_ctx *ctx, const nj_ct *in, int r, nj_ct *out, void *stream);
/* Automorphism X -> X^g followed by hybrid key switching back to s (ModUp, key
 * inner product, ModDown).  Needs the key of g (NJ_ENOKEY otherwise), except g = 1,
 * the identity, which copies in to out.  NJ_EINVAL for an even g or g >= 2N.  in and
 * out may alias. */
nj_status nj_apply_galois(nj_ctx *ctx, const nj_ct *in, uint32_t galois_elt, nj_ct *out, void *stream);
/* nj_apply_galois for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): the same kernels and the
 * same result word for word, with the scratch in a fixed 160 MiB (20 Mi words) device
 * array of the library instead of the context's growable arena.  No hipMalloc, hipFree
 * or other allocating call is made.  The array exists once per GPU for the process's
 * lifetime (its address is looked up when a context is created on that GPU); every call
 * on one GPU shares it, so calls that may overlap on one GPU (different streams or
 * threads, any context) race and must be serialised by the caller.  Nothing in it needs
 * clearing between calls.  NJ_EUNSUPPORTED when the key switch needs more scratch than
 * the array holds (ModUp digits, inner products and ModDown limbs at level l: about
 * (2(l+1) + dnum_l (l+1+alpha) + 2(l+1+alpha) + 2 alpha + 3(l+1)) N words) or while live
 * profiling is on; otherwise the errors of nj_apply_galois. */
nj_status nj_apply_galois_noalloc(nj_ctx *ctx, const nj_ct *in, uint32_t galois_elt, nj_ct *out, void *stream);
/* Key switching of one polynomial d (evaluation form, level l): (out0, out1) with
 * out0 + out1 s ~ d s', using the key of galois_elt (0 = relinearisation key). */
nj_status nj_keyswitch(nj_ctx *ctx, const uint64_t *d, int level, uint32_t galois_elt, uint64_t *out0, uint64_t *out1,
                       void *stream);
/* PMult (Sec. 2.1): both polynomials times a plaintext pt, device [(level+1)][N] in
 * evaluation form (nj_to_eval of its coefficients).  out may alias in.  The plaintext's
 * scale is not known to the call: out->scale = in->scale, and the caller multiplies in
 * the plaintext's own scale. */
nj_status nj_pmult(nj_ctx *ctx, const nj_ct *in, const uint64_t *pt, nj_ct *out, void *stream);
/* HAdd / HSub (Sec. 2.1): out = a + b or a - b.  Same level (else NJ_ELEVEL) and the
 * same scale up to a relative 1e-9 (else NJ_ESCALE).  out may alias a or b. */
nj_status nj_add(nj_ctx *ctx, const nj_ct *a, const nj_ct *b, nj_ct *out, void *stream);
nj_status nj_sub(nj_ctx *ctx, const nj_ct *a, const nj_ct *b, nj_ct *out, void *stream);
/* Rescale (Sec. 2.4): divide by q_l with rounding, level l -> l-1. */
/* Level drop: the first level+1 limbs of each polynomial of `in` (level <= in->level),
 * an exact change of modulus Q_l -> Q_level with the scale unchanged.  out must not
 * alias in unless level == in->level. */
nj_status nj_drop_level(nj_ctx *ctx, const nj_ct *in, int level, nj_ct *out, void *stream);
nj_status nj_rescale(nj_ctx *ctx, const nj_ct *in, nj_ct *out, void *stream);
/* ModRaise (Sec. 2.4): level-0 ciphertext lifted (centred) to `level`. */
nj_status nj_modraise(nj_ctx *ctx, const nj_ct *in, int level, nj_ct *out, void *stream);

/* ---------------------------------------------------------------- plans */

/* A plan holds n_lt BSGS linear transforms (Sec. 2.6).  Transform t acts at level
 * level0 - t on slot-rotation unit u_t with diagonal offsets j*u_t and baby size n1_t. */
int nj_plan_count(const nj_plan *plan);
/* Galois elements whose keys the plan needs; returns the count (writes at most max). */
int nj_plan_galois(const nj_plan *plan, uint32_t *out, int max);
/* Diagonal offsets of transform t, in the order used by nj_plan_set_diagonal. */
int nj_plan_offsets(const nj_plan *plan, int t, int32_t *out, int max);
/* Replaces diagonal `idx` of transform t with host residues [(level_t+1)][N] in
 * coefficient form (already baby-step giant-step pre-rotated). Synchronous.  In a
 * block conv plan idx = (ob bi + ib) n_diag + d addresses diagonal d of block (ob, ib). */
nj_status nj_plan_set_diagonal(nj_ctx *ctx, nj_plan *plan, int t, int idx, const uint64_t *coeffs);
/* Lazy giant steps (on = 1): the giant rotations of every transform of the plan sum
 * their key inner products over Q_l u P and share one ModDown (the BSGS outer sum is
 * linear); a different rounding of the same result, so parity holds per setting.
 * Single-ciphertext and batched transforms only (block and mixed-level transforms
 * return NJ_EUNSUPPORTED). */
nj_status nj_plan_set_lazy(nj_plan *plan, int on);
/* Hoisted baby steps of transform t (t = -1: every transform of the plan) (on = 1, the
 * default): the baby rotations share one ModUp of c1 and apply the automorphism to its
 * extended digits; off, every baby rotation is its own key switch.  Used by
 * nj_conv2d_cins, nj_coeff_to_slot and nj_time_plan (block transforms always hoist).
 * Different low bits, so parity holds per setting. */
nj_status nj_plan_set_hoist(nj_plan *plan, int t, int on);
void nj_plan_destroy(nj_plan *plan);

/* Fused conv2d + StoC2 plan (Sec. 3.3, Sec. 4, Algorithm 1): C = N/W^2
 * channels per ciphertext, W = smallest power of two >= w0 + (f-1)/2.
 *   weights: host double [C][C][f][f] (out, in, row, col), cross-correlation with
 *   'same' zero padding.  Diagonals K' = S'K^, encoded at scale q_1 for level 1.
 *   n1 = baby steps (0 = ceil(sqrt(C))). */
nj_status nj_conv_plan_create(nj_ctx *ctx, int w0, int f, const double *weights, int n1, nj_plan **out);

/* CoeffToSlot plan (Sec. 2.4): T_{N/2}^{-1}'s stages in `groups` consecutive groups
 * at levels L, L-1, ...; each group's diagonals encoded at the scale of the prime
 * its rescale drops; the 1/2 of the real split folded into the last group. */
nj_status nj_cts_plan_create(nj_ctx *ctx, int groups, nj_plan **out);
/* The same with the baby-step count of each group chosen: n1 host [groups] (0 = the
 * default ceil(sqrt(#diagonals)), else any positive count; Sec. 2.6 leaves the BSGS
 * split free).  Different splits give different low bits, so parity holds per split. */
nj_status nj_cts_plan_create_split(nj_ctx *ctx, int groups, const int *n1, nj_plan **out);
/* Cost-model features (as nj_plan_features) of each group of that CoeffToSlot plan at its
 * level, baby steps hoisted or not, without building or uploading its diagonals: f host
 * [groups][7].  n1 as for nj_cts_plan_create_split (may be null). */
nj_status nj_cts_plan_features(nj_ctx *ctx, int groups, const int *n1, int hoist, float *f);

/* BSGS evaluation of transform t of the plan on `in`, no rescale.  The input level may
 * be the transform's level or any lower one (the first l+1 limbs of each diagonal are
 * used); out->scale = in->scale * the diagonals' encoding scale.
 * hoist = 1: baby-step rotations share one ModUp of c1. */
nj_status nj_plan_apply(nj_ctx *ctx, const nj_plan *plan, int t, const nj_ct *in, nj_ct *out, int hoist, void *stream);

/* Fused conv (Algorithm 1): BSGS with the K' diagonals, rescale.  Input at any level
 * l in 1..the plan's level, output at l-1 with scale in->scale * s_plan / q_l, where
 * s_plan is the plan's encoding scale (q at the plan's level: exact when l equals it). */
nj_status nj_conv2d_cins(nj_ctx *ctx, const nj_plan *conv, const nj_ct *in, nj_ct *out, void *stream);

/* CoeffToSlot (Algorithm 1, before EvalMod): ModRaise of the level-0 input to L,
 * each group's BSGS + rescale, then Re = ct + conj(ct), Im = -X^{N/2}(ct - conj(ct)).
 * re/im: device [2][L-groups+1][N]. */
nj_status nj_coeff_to_slot(nj_ctx *ctx, const nj_plan *cts, const nj_ct *in, nj_ct *re, nj_ct *im, void *stream);

/* --------------------------------------------------------- batched calls */

/* Batches: in->data (and each output's data) holds n ciphertexts of the same level
 * back to back, [n][2][l+1][N].  The library processes sub-batches of up to 8 in
 * which every switching-key word and every plaintext-diagonal word is read once
 * for all ciphertexts (key switches grouped by Galois element).  Results are
 * bit-identical to n separate calls.  Outputs must not alias inputs. */
nj_status nj_apply_galois_batch(nj_ctx *ctx, const nj_ct *in, int n, uint32_t galois_elt, nj_ct *out, void *stream);
nj_status nj_conv2d_cins_batch(nj_ctx *ctx, const nj_plan *conv, const nj_ct *in, int n, nj_ct *out, void *stream);
nj_status nj_coeff_to_slot_batch(nj_ctx *ctx, const nj_plan *cts, const nj_ct *in, int n, nj_ct *re, nj_ct *im,
                                 void *stream);

/* ------------------------------------------------------------ conv variants */

/* One tap of a convolution (Sec. 3.3): out[out_ch][y][x] += w * in[in_ch][y+dy][x+dx],
 * zero outside the w0 x w0 image.  A 3x3 'same' conv is the taps dy, dx in -1..1; a
 * pointwise conv the single tap (0, 0); a depthwise conv the taps with
 * out_ch == in_ch; a stride-2 conv the taps of its polyphase decomposition on the
 * four phase images of each input channel (phase (a, b) = rows a::2, columns b::2,
 * stored as channel 4 i + 2 b + a), with offsets floor((u - p)/2) (nj_conv_taps). */
typedef struct {
    int32_t out_ch, in_ch, dy, dx;
    double w;
} nj_tap;

/* Conv plan from a tap list (Sec. 3.3, block convs Sec. 3.3.4).  Layout: W = smallest
 * power of two >= w0 + max |dy|, |dx|; l = W^2/2 slots per channel; C = N/W^2
 * channels per ciphertext; channel block b of c_in (c_out) lives in input (output)
 * ciphertext b, bi = ceil(c_in/C) inputs, bo = ceil(c_out/C) outputs.
 *   fuse = 1: diagonals of K^' = S'K^ (conv fused with StoC2, all C offsets);
 *   fuse = 0: diagonals of K^ only (CinS-slot output, e.g. depthwise: one diagonal,
 *             one PMult, no rotation), only offsets nonzero in some block.
 *   n1 = baby steps (0 = ceil(sqrt(#offsets))); level = level the plan consumes
 *   (1..L), diagonals encoded at scale q_level; the plan also serves any lower level.
 * Errors: NJ_EINVAL for taps outside the channel ranges or |offset| >= W, or all-zero
 * weights; NJ_EUNSUPPORTED if W^2 > N. */
nj_status nj_conv_plan_create_taps(nj_ctx *ctx, int w0, int c_in, int c_out, const nj_tap *taps, int n_taps,
                                   int fuse, int n1, int level, nj_plan **out);
/* A conv layer (Sec. 3.3): weights [c_out][c_in][f][f] (depthwise: [c][f][f]), odd f,
 * 'same' zero padding (f-1)/2, stride 1 or 2 (Sec. 5: a stride-2 conv is the sum over the
 * four phases (a, b) of unit-stride convs of the phase images I_i[a::2, b::2], stored as
 * input channel 4 i + 2 b + a at width w0/2; the kernel tap (u, v) reads phase
 * ((u-p) mod 2, (v-p) mod 2) at offset (floor((u-p)/2), floor((v-p)/2))); fuse = 1 merges
 * StoC2 into the kernel matrix (Sec. 4). */
typedef struct {
    int w0;         /* input image width (stride 2: even; the output is w0/2 wide) */
    int c_in, c_out;
    int f;          /* kernel width, odd */
    int stride;     /* 1 or 2 */
    int depthwise;  /* 1: one kernel per channel (c_in == c_out) */
    int fuse;       /* 1: fused with StoC2 */
} nj_conv_desc;
/* The taps of such a layer (host only): taps may be null to get the count in *n_taps;
 * else at most max_taps are written.  NJ_EINVAL for bad shapes or a short buffer. */
nj_status nj_conv_taps(int c_in, int c_out, int f, int stride, int depthwise, const double *weights, nj_tap *taps,
                       int max_taps, int *n_taps);
/* The plan of a conv layer: nj_conv_plan_create_taps of its taps (inputs of a stride-2
 * layer in the phase layout above, 4 c_in channels at w0/2). */
nj_status nj_conv_plan_create_layer(nj_ctx *ctx, const nj_conv_desc *desc, const double *weights, int n1, int level,
                                    nj_plan **out);
/* Slot permutations of the downsampling flows (Sec. 5, Algorithm 2, Appendix B) as BSGS
 * transforms (0/1 diagonals encoded at scale q_level, so a transform + rescale keeps the
 * scale), applied after ModEval to one half of a CoeffToSlot output: half 0 the real
 * part (slot j = coefficient rev(j)), half 1 the imaginary part (N/2 + rev(j)), images in
 * the fused conv's coefficient layout (coefficient (y W + x) C + rev_C(c) = pixel (y, x)
 * of channel c, W^2 C = N):
 *   kind 0, decompose: one ciphertext (W, C) -> (W/2, 4C) holding the phase images,
 *     channel 4 i + 2 b + a = I_i[a::2, b::2] (the input layout of a stride-2 conv
 *     plan); one block, W - 1 diagonals; apply with nj_conv2d_cins;
 *   kind 1, densify: four ciphertexts (W, C) of stride-1 conv outputs -> one (W/2, 4C),
 *     channel 4 i + m = even pixels of channel i of input m; a block plan (bi = 4, bo = 1)
 *     applied with nj_conv2d_block.
 * n1 = baby steps (0 = ceil(sqrt(#diagonals))).  NJ_EINVAL for a layout with W^2 C != N. */
nj_status nj_downsample_plan_create(nj_ctx *ctx, int kind, int W, int C, int half, int n1, int level, nj_plan **out);
/* A fully connected layer y = W x fused with the whole StoC (Sec. 4.2.1: slot encoding is
 * CinS with l = 1): weights [n_out][n_in] (host), n' = the smallest power of two >= n_in,
 * n_out (<= N/2).  The input ciphertext is slot-encoded with period n': slots j, j + n',
 * ... hold x_{j mod n'} (real, 0 for n_in <= j mod n' < n').  nj_conv2d_cins applies it
 * (input level 1..level, output one level lower, scale kept): the output's coefficient
 * k N / (2 n') holds y_k for k < n_out (times the scale), the other coefficients 0.  n'
 * cyclic diagonals (n1 = baby steps, 0 = ceil(sqrt(n'))).  NJ_EUNSUPPORTED if n' > N/2. */
nj_status nj_fc_plan_create(nj_ctx *ctx, int n_in, int n_out, const double *weights, int n1, int level,
                            nj_plan **out);
/* Layout of a conv plan: W, C, l, bi, bo (any pointer may be null).  Returns the
 * plan's level, -1 for a null or empty plan. */
int nj_plan_layout(const nj_plan *plan, int *W, int *C, int *ell, int *bi, int *bo);
/* Block conv (Sec. 3.3.4): bi ciphertexts contiguous from in->data ([bi][2][l+1][N],
 * l in 1..the plan's level) -> bo contiguous outputs [bo][2][l][N] at level l-1 after
 * the rescale, scale as for nj_conv2d_cins.  Baby steps hoisted once per input, giant
 * steps once per output block.  Outputs must not overlap the inputs. */
nj_status nj_conv2d_block(nj_ctx *ctx, const nj_plan *conv, const nj_ct *in, nj_ct *out, void *stream);

/* ------------------------------------------------------------ batched jobs */

/* One job (Algorithm 1, conv then bootstrapping's first step, at the ciphertext's own
 * level): conv with plan `conv` on bi input ciphertexts contiguous at in.data (level
 * 1..the plan's level) -> rescale -> level drop to 0 -> ModRaise -> CoeffToSlot with
 * the batch's plan -> real split into bo Re and bo Im ciphertexts, contiguous at
 * re.data and im.data ([bo][2][L-g+1][N], g = number of CoeffToSlot groups).  The
 * library fills in the level, form and scale of re and im. */
typedef struct {
    const nj_plan *conv;
    nj_ct in;
    nj_ct re, im;
} nj_job;

/* Runs the jobs on `stream` using the context scratch.
 *   mode 0, plain: one job after another, each step as the single-job calls run it.
 *   mode 1, batched: each conv on the fused single-ciphertext path, the rescale
 *     computing only the limb the level drop keeps (and, for plans with lazy giant steps
 *     at N >= 8192, the conv itself only the limbs 0 and l that rescale reads: the
 *     giant steps' ModUp digits, inner products and ModDown are restricted to them),
 *     the jobs spread over the worker
 *     streams as in mode 2 (convs at low levels leave much of the GPU idle); then every
 *     conv output (all at one level after ModRaise) goes through batched CoeffToSlot on
 *     `stream`, which reads each rotation key and plaintext diagonal once for up to 8
 *     ciphertexts.
 *   mode 2, concurrent: each job as in mode 0, the jobs spread over the context's
 *     worker streams (nj_batch_workers, default 4) by longest-first assignment, each
 *     worker with its own part of the scratch (workers x the plain scratch); the
 *     workers fork from `stream` and join back into it, so work queued on `stream`
 *     afterwards sees every output.
 *   mode 3, batched across levels: as mode 1, but single-block jobs of one conv plan
 *     run together across their levels (each baby and giant rotation key read once for
 *     up to 16 jobs; ModUp and ModDown batched per level, with unfused transforms);
 *     jobs of a plan with lazy giant steps (nj_plan_set_lazy) run one at a time.
 * All modes give bit-identical outputs.  Errors: NJ_EINVAL (bad plan or job),
 * NJ_ELEVEL (input level outside 1..plan level), NJ_ENOKEY, NJ_ENOMEM. */
nj_status nj_batch_run(nj_ctx *ctx, const nj_plan *cts, nj_job *jobs, int n_jobs, int mode, void *stream);
/* Worker streams of modes 1 and 2 (1..4; NJ_EINVAL otherwise).  Streams run at the default
 * priority.  Concurrent calls on one context must not overlap (they share the
 * workers and the scratch). */
nj_status nj_batch_workers(nj_ctx *ctx, int n_streams);

/* Persistent batched execution: a schedule captured once into a HIP graph that owns
 * its scratch memory; nj_batch_launch replays it with no host work per job.
 * nj_batch_create captures mode 1, nj_batch_create_mode the given mode (0 to 3; a
 * mode-2 graph holds the workers' branches).  Capture computes nothing; the jobs'
 * buffers, plans and keys must stay in place for the batch's lifetime.  Replays on
 * one batch must not overlap. */
typedef struct nj_batch nj_batch;
nj_status nj_batch_create(nj_ctx *ctx, const nj_plan *cts, nj_job *jobs, int n_jobs, nj_batch **out);
nj_status nj_batch_create_mode(nj_ctx *ctx, const nj_plan *cts, nj_job *jobs, int n_jobs, int mode, nj_batch **out);
nj_status nj_batch_launch(nj_batch *batch, void *stream);
void nj_batch_destroy(nj_batch *batch);

/* ------------------------------------------------- bootstrapping after CoeffToSlot */

/* HMult (Sec. 2.1): tensor product at l = min(levels), relinearisation with the key of
 * Galois element 0 (s^2 -> s), rescale -> level l-1, scale s_a s_b / q_l.  out may not
 * alias the inputs. */
nj_status nj_hmult(nj_ctx *ctx, const nj_ct *a, const nj_ct *b, nj_ct *out, void *stream);
/* c * in at a lower `level`: the first level+2 limbs times the integer
 * round(c * scale * q_{level+1} / in->scale), rescale; out->scale = scale. */
nj_status nj_mul_const(nj_ctx *ctx, const nj_ct *in, double c, int level, double scale, nj_ct *out, void *stream);
/* Adds c to every slot (round(c * ct->scale) to the constant coefficient), in place. */
nj_status nj_add_const(nj_ctx *ctx, nj_ct *ct, double c, void *stream);
/* Chebyshev interpolant (first-kind nodes) of cos(2 pi (K x - 1/4) / 2^r) on [-1, 1]:
 * coeffs [degree+1], host. */
nj_status nj_cheb_interpolate(int degree, double K, int r, double *coeffs);
/* ModEval (Sec. 2.4; Algorithm 1): for a CoeffToSlot output whose slots hold
 * t = m + (q_0 / scale) I, returns m ~ (P / 2 pi) sin(2 pi t / P), P = q_0 / scale:
 * x = t / (K P) (the input read at scale K q_0), one integer multiply bringing the
 * scale near 2^48, the degree-63 Chebyshev series of cos(2 pi (K x - 1/4) / 8)
 * (coeffs [64], or null for the library's interpolant) by baby steps T_1..T_7 and giant
 * steps T_8/T_16/T_32 with every constant encoded at its term's exact scale, then r = 3
 * double angles.  Uses 11 levels (input level >= 12); needs the relinearisation key.
 * |I| must stay below K. */
nj_status nj_eval_mod(nj_ctx *ctx, const nj_ct *in, int K, int r, const double *coeffs, int n_coeffs, nj_ct *out,
                      void *stream);
/* Evaluation order of ModEval's Chebyshev baby-step sums sum_j c_j T_j (Sec. 2.4 leaves
 * the evaluation to prior work; both orders give the same message up to rounding noise):
 *   order 0 (default): each term c_j T_j is a constant multiply at its own scale followed
 *     by its own rescale to the sum's level, then the terms are added;
 *   order 1: the integers round(c_j tau q / s_j) times T_j are accumulated at one level and
 *     the sum is rescaled once (fewer rescales; different low bits).
 * Applies to every later nj_eval_mod / nj_slot_activation / nj_conv_act_layer /
 * nj_bootstrap call on the context.  NJ_EINVAL for another order. */
nj_status nj_eval_order(nj_ctx *ctx, int order);
/* Re + i Im (i = X^{N/2} on the slots); same level (NJ_ELEVEL) and scale (NJ_ESCALE,
 * as nj_add). */
nj_status nj_combine(nj_ctx *ctx, const nj_ct *re, const nj_ct *im, nj_ct *out, void *stream);
/* StoC1 = S_{l <- 1} = S_{l/2} ... S_1 (Algorithm 1, the StoC stages left after fusing
 * StoC2 into the next conv) in `groups` stage groups at levels level, level-1, ...;
 * diagonals encoded at each group's q.  nj_stoc1 applies it (input at `level`), output
 * at level - groups with the input's scale. */
nj_status nj_stoc1_plan_create(nj_ctx *ctx, int ell, int groups, int level, nj_plan **out);
nj_status nj_stoc1(nj_ctx *ctx, const nj_plan *plan, const nj_ct *in, nj_ct *out, void *stream);

/* ------------------------------------------- Algorithm 1 and bootstrapping */

/* The zero-padding masks of Algorithm 1 (Sec. 4; the flattened conv of Sec. 2.5.1 leaves
 * values at padding positions): for CinS images of w0 x w0 pixels padded to W x W, C per
 * ciphertext (W^2 C = N = 2^log_n), mask_re[j] / mask_im[j] (N/2 doubles each, host) are
 * 1 where slot j of the real / imaginary CoeffToSlot output holds an output pixel and 0
 * where it holds padding.  Coefficient k of the fused conv's output holds padded pixel
 * floor(k / C) (row-major in W x W); CoeffToSlot leaves coefficient rev(j) in real slot j
 * and N/2 + rev(j) in imaginary slot j (bit reversal over log_n - 1 bits).  Host only. */
nj_status nj_layer_masks(int log_n, int W, int C, int w0, double *mask_re, double *mask_im);
/* Algorithm 1 after CoeffToSlot: ModEval (as nj_eval_mod) of re and im (same level l);
 * if masks are given, PMult by mask_re / mask_im and rescale (masks: device plaintexts in
 * evaluation form, [l - 10][N] = the ModEval output's limbs, the slot masks encoded at
 * scale q_{l-11} so the scale is kept); the activation: act 0 none, act 1 the square of
 * AESPA (Sec. 2.5.2) by HMult with relinearisation; Re + i Im (nj_combine), dropped to
 * the StoC1 plan's first level (an error if below it); StoC1 -> out (level and scale
 * set).  Needs the relinearisation key and the StoC1 plan's rotation keys. */
nj_status nj_slot_activation(nj_ctx *ctx, int K, int r, const double *coeffs, int n_coeffs, const uint64_t *mask_re,
                             const uint64_t *mask_im, int act, const nj_plan *stoc1, const nj_ct *re, const nj_ct *im,
                             nj_ct *out, void *stream);
/* Algorithm 2's slot-domain part (Sec. 5): nj_slot_activation with the decomposition of
 * each half (nj_downsample_plan_create kind 0, dec_re for half 0 and dec_im for half 1,
 * both at one level l <= the activated level: the halves are dropped to l first, each
 * plan consumes a level) between the activation and Re + i Im; `stoc1` is then the StoC1
 * plan of the phase layout (l/4).  dec_re = dec_im = null is nj_slot_activation. */
nj_status nj_slot_activation_decompose(nj_ctx *ctx, int K, int r, const double *coeffs, int n_coeffs,
                                       const uint64_t *mask_re, const uint64_t *mask_im, int act,
                                       const nj_plan *dec_re, const nj_plan *dec_im, const nj_plan *stoc1,
                                       const nj_ct *re, const nj_ct *im, nj_ct *out, void *stream);
/* Algorithm 1, one layer: conv2d_cins (fused with StoC2; conv may be null, then `in` is
 * a level-0 ciphertext) -> level 0 -> ModRaise + CoeffToSlot (nj_coeff_to_slot) ->
 * nj_slot_activation.  `out` is the next layer's CinS input (the StoC2 stages left are
 * fused into the next conv). */
nj_status nj_conv_act_layer(nj_ctx *ctx, const nj_plan *conv, const nj_plan *cts, int K, int r, const double *coeffs,
                            int n_coeffs, const uint64_t *mask_re, const uint64_t *mask_im, int act,
                            const nj_plan *stoc1, const nj_ct *in, nj_ct *out, void *stream);
/* Bootstrapping (Sec. 2.4) of a level-0 ciphertext: ModRaise, CoeffToSlot, ModEval of
 * Re and Im, Re + i Im, StoC1: nj_conv_act_layer without conv, masks or activation. */
nj_status nj_bootstrap(nj_ctx *ctx, const nj_plan *cts, int K, int r, const double *coeffs, int n_coeffs,
                       const nj_plan *stoc1, const nj_ct *in, nj_ct *out, void *stream);

/* ------------------------------------------------------------ plan selection */

/* Timing mode for latency measurement: after nj_timing_keys(ctx, pool) with pool > 0,
 * a Galois element without a switching key uses one of `pool` key-sized buffers of
 * random residues (element g -> buffer g mod pool), so candidate plans can be timed
 * without generating their keys; a pool larger than the last-level cache (16 x 100 MB
 * at N = 2^16) keeps the key traffic of the real transform.  Results computed with
 * these buffers are not valid ciphertexts; real keys always take precedence.
 * pool = 0 leaves timing mode and frees the buffers. Synchronous. */
nj_status nj_timing_keys(nj_ctx *ctx, int pool);

/* A conv-kind plan with a given BSGS structure and random diagonals, for timing: unit
 * u slots, n_off diagonal offsets j (diagonal j*u, any representatives), baby size n1
 * (0 = ceil(sqrt(#offsets))), bi x bo blocks, encoded for `level`. */
nj_status nj_plan_create_random(nj_ctx *ctx, int level, int u, const int32_t *offsets, int n_off, int n1, int bi,
                                int bo, uint64_t seed, nj_plan **out);

/* Median time in ms (HIP events on the null stream, one warm-up run, then `reps`) of
 * transform t of the plan at `level` (<= its level) on random ciphertexts, run as the
 * library runs it: single-ciphertext hoisted BSGS for one block, block BSGS otherwise
 * (no rescale).  Synchronous. */
nj_status nj_time_plan(nj_ctx *ctx, const nj_plan *plan, int t, int level, int reps, float *ms);

/* Cost-model features of transform t at `level` (the plan features of the learned cost
 * model): f[0] = limbs (level+1); f[1] = diagonals per block (channels of a fused conv);
 * f[2] = log2(N/2 / u), u the slot stride of its rotations (image size); f[3] = baby steps
 * (BSGS split); f[4] = hoisted baby rotations, bi (babies - 1), or 0 when not hoisted
 * (hoist count); f[5] = DFT stages merged into the transform (fusion depth: log2 C for a
 * conv fused with StoC2, the stage count of a CoeffToSlot or StoC1 group); f[6] = bo. */
nj_status nj_plan_features(const nj_plan *plan, int t, int level, float *f);


/* Learned cost model (plan selection by predicted latency): 7 features -> 64 -> 64 -> 1,
 * FP32, ReLU.  Parameters (NJ_MLP_PARAMS floats): W1 [7][64], b1 [64], W2 [64][64]
 * (row = input unit), b2 [64], w3 [64], b3.  Created with He-uniform weights from a
 * seeded generator and zero biases; training standardises features and target on the
 * training set and predictions undo it.  All host arrays; synchronous calls. */
#define NJ_MLP_FEATURES 7
#define NJ_MLP_HIDDEN 64
#define NJ_MLP_PARAMS (7 * 64 + 64 + 64 * 64 + 64 + 64 + 1)
typedef struct nj_mlp nj_mlp;
nj_status nj_mlp_create(uint64_t seed, nj_mlp **out);
void nj_mlp_destroy(nj_mlp *mlp);
nj_status nj_mlp_set_params(nj_mlp *mlp, const float *params); /* also resets the Adam state */
nj_status nj_mlp_get_params(const nj_mlp *mlp, float *params);
/* The standardisation a trained model applies (for saving and restoring it with the
 * parameters): norm host [NJ_MLP_NORM] = feature means [7], feature scales [7], target
 * mean, target scale.  A new model has means 0 and scales 1.  Set: NJ_EINVAL for a
 * scale <= 0. */
#define NJ_MLP_NORM (2 * 7 + 2)
nj_status nj_mlp_get_norm(const nj_mlp *mlp, float *norm);
nj_status nj_mlp_set_norm(nj_mlp *mlp, const float *norm);
/* Gradient of mean((f(x_i) - y_i)^2) over the n samples X [n][7], y [n] with respect
 * to every parameter (raw inputs, no standardisation), and the loss. */
nj_status nj_mlp_grad(nj_mlp *mlp, const float *X, const float *y, int n, float *grad, float *loss);
/* Adam (lr, beta 0.9 / 0.999, eps 1e-8) on minibatches of `batch` samples, shuffled
 * each epoch by a seeded generator; final_loss (may be null) = training MSE in
 * standardised target units. */
nj_status nj_mlp_train(nj_mlp *mlp, const float *X, const float *y, int n, int epochs, int batch, float lr,
                       uint64_t seed, float *final_loss);
nj_status nj_mlp_predict(nj_mlp *mlp, const float *X, int n, float *out);

/* Autotuner (plan selection, Sec. 2.6's BSGS split and hoisting): picks the baby-step
 * count n1, the hoisting mode and (when lazy is non-null) the giant steps' ModDown of
 * transform t of a plan at `level` (1 <= level <= the transform's).  Candidates: n1 = 0
 * (the default split) and the powers of two within a factor 4 of sqrt(#diagonals), each
 * hoisted or not (block transforms: hoisted only).  With model (may be null) and
 * shortlist > 0, the model ranks the candidates by their features (nj_plan_features of
 * each split) and only its `shortlist` best are timed; otherwise every candidate is.
 * The default split, hoisted, is always timed, so the choice is never slower than the
 * default as measured.  Each candidate is timed as nj_time_plan times it (reps runs,
 * median), on a plan of the same diagonal offsets with random diagonals, so the rotation
 * keys must be present or timing mode on (nj_timing_keys); with lazy non-null every
 * timed split of a single-block transform is timed both with the plan's own giant-step
 * ModDown and with the other form (nj_plan_set_lazy: one ModDown for all giant steps,
 * or one per step).  Outputs: n1 (0 = default), hoist (1/0), lazy (1/0; may be null:
 * the plan's own form only), the choice's time in ms, and the default's time with the
 * plan's own form (default_ms may be null).  The plan itself is not changed: rebuild it
 * with the chosen n1 (plan constructors take n1) and apply nj_plan_set_hoist and
 * nj_plan_set_lazy.  Synchronous; allocates the candidate plans one at a time. */
nj_status nj_tune_split(nj_ctx *ctx, const nj_plan *plan, int t, int level, const nj_mlp *model, int shortlist,
                        int reps, int *n1, int *hoist, int *lazy, float *ms, float *default_ms);

/* ------------------------------------------------------------ profiling */

/* Live kernel timing for roofline reports: when enabled, the library records HIP
 * events on the launch stream around every launch of the kernel families below
 * and accumulates each launch's algorithmic HBM bytes (every input word read once,
 * every output word written once).  kind: 0/1 NTT 4096-word tile pass forward/inverse,
 * 2/3 NTT column pass forward/inverse, 4 basis conversion, 5 key inner product,
 * 6 plaintext multiply-accumulate, 7 other, 8 forward tile pass fused with the
 * ModDown combine. */
nj_status nj_prof_enable(nj_ctx *ctx, int on);
/* Synchronises the device, then returns launches, total ms and total bytes of `kind`
 * recorded since the last reset; reset = 1 clears the records. */
nj_status nj_prof_read(nj_ctx *ctx, int kind, int *launches, double *total_ms, double *total_bytes, int reset);

#ifdef __cplusplus
}
#endif
#endif
