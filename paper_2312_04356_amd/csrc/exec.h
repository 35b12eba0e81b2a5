// Internal executor helpers shared by the C ABI files: scratch arena, key switching
// of one or many polynomials, BSGS transforms, rescale / ModRaise.
#pragma once

#include "internal.h"

namespace nj {
namespace ex {

inline hipStream_t S(void *s) { return (hipStream_t)s; }

// Bump allocator over the context scratch buffer.
struct Arena {
    uint64_t *p;
    size_t left;
    uint64_t *take(size_t w)
    {
        if (w > left) return nullptr;
        uint64_t *r = p;
        p += w;
        left -= w;
        return r;
    }
};

// Buffers for K jobs at level l: polynomials to switch d [K][l+1], their
// coefficient form [K][l+1], extended digits [K][dnum][l+1+alpha], inner
// products [K][2][l+1+alpha], special-prime limbs [K][2][alpha], converted limbs
// [K][2][l+1] (all x N words).
struct MultiBufs {
    uint64_t *d, *coef, *ext, *u, *pc, *conv;
};

constexpr int kGiantChunk = 8;  // giant-step key switches per batch in a single-ciphertext transform
constexpr int kMaxWorkers = 4;  // worker streams: hardware queues per process on the target (GPU_MAX_HW_QUEUES)
// creates the context's kMaxWorkers worker streams and their events if not yet made
nj_status workers_ready(nj_ctx *c);
constexpr int kBatch = 8;       // ciphertexts per sub-batch of the batched calls

Arena arena_for(nj_ctx *c, size_t words, bool &ok);
const uint64_t *key_of(const nj_ctx *c, uint32_t g);
int galois_of_rot(const nj_ctx *c, long long r);
nj_status check_ct(const nj_ctx *c, const nj_ct *ct, const char *what);
LimbTab ct_limbs(int l);

// scratch words of one key switch at level l (apply_galois with in == out, ks_one)
size_t ks_words(const nj_ctx *c, int l);
// out = (tau_g(c0), tau_g(c1)) switched back to s; in and out may alias
nj_status apply_galois(nj_ctx *c, int l, const uint64_t *in, uint32_t g, uint64_t *out, Arena A, hipStream_t s);

size_t multi_words(const nj_ctx *c, int l, int K);
bool multi_bufs(const nj_ctx *c, int l, int K, Arena &A, MultiBufs &M);
// ModUp of K polynomials at d + z dstride N (dstride in limbs, l+1 when packed)
// (tiles = false: at N >= 8192 the converted limbs are left after their column pass,
// for the fused key inner product)
// (gt: job z's polynomial is read through X -> X^g[z], N >= 8192; zoff: job z's
// polynomial at d + zoff[z] N instead of d + z dstride N)
// (drop: only the targets a rescale followed by a drop to level 0 needs, Q limbs 0 and l
// and the special primes)
nj_status modup_multi(nj_ctx *c, int l, int K, const uint64_t *d, MultiBufs &M, hipStream_t s, int dstride = -1,
                      bool tiles = true, const GalTab *gt = nullptr, const int *zoff = nullptr, bool drop = false);
// whether ModUp leaves the tile pass to the key inner product (launch_ntt_ip)
bool fuse_ip(const nj_ctx *c, int l);
// ModEval of Re and Im evaluated together (packed) when N >= 8192
nj_status eval_mod_pair(nj_ctx *c, const nj_ct *re, const nj_ct *im, int K, int r, const double *coeffs,
                        int n_coeffs, nj_ct *out_re, nj_ct *out_im, void *stream);
// one key switch of tau_g(d): out = (ModDown_0 + add read through X -> X^g_add, ModDown_1)
// (conj: the output is replaced by the real/imaginary split with add's ciphertext, see
// MdConj; N >= 8192)
nj_status ks_one(nj_ctx *c, int l, const uint64_t *d, uint32_t g, const uint64_t *key, const uint64_t *add,
                 uint32_t g_add, uint64_t *out, MultiBufs &M, hipStream_t s, const MdConj *conj = nullptr);
// as ks_multi, on digits of tau_g(d) that modup_multi left column-passed (tiles =
// false); kj.d[z] is d itself, read through X -> X^g[z] for the own limbs
nj_status ks_fused(nj_ctx *c, int l, int K, const KeyJobs &kj, const MdJobs &mj, int sum, const uint64_t *acc,
                   MultiBufs &M, hipStream_t s, const MdConj *conj = nullptr);
// K key switches on ModUp'ed digits (M.ext): key inner products, then ks_down
nj_status ks_multi(nj_ctx *c, int l, int K, const KeyJobs &kj, const MdJobs &mj, int sum, const uint64_t *acc,
                   MultiBufs &M, hipStream_t s);
// ModDown of K jobs' inner products (M.u) and the combine into their outputs
// (p_tiled: the inner products already left their special-prime rows in M.pc after the
// first 12 stages of the inverse transform; N >= 8192.  acc: the previous value added
// (sum = 0: for K = 1 it may be any ciphertext, else it must be the outputs).
// last_out, one job, N >= 8192: the output's last limb also leaves through the first
// 12 stages of its inverse transform into last_out [2][N], for rescale(last_pre))
// drop: only output limbs 0 and l (the fused one-job combine, no last_out or conj, l >= 2;
// the inner products' Q rows 0 and l and special-prime rows are all it reads)
nj_status ks_down(nj_ctx *c, int l, int K, const MdJobs &mj, int sum, const uint64_t *acc, MultiBufs &M,
                  hipStream_t s, bool p_tiled = false, uint64_t *last_out = nullptr, const MdConj *conj = nullptr,
                  bool drop = false, const KeyJobs *ipq = nullptr);

// inner_g += diag_dg (.) baby_b for each entry, any number of baby and giant steps
struct MacEntry {
    int g, b, dg;
};
nj_status mac_general(nj_ctx *c, int l, const std::vector<const uint64_t *> &baby, int ng,
                      const std::vector<MacEntry> &ent, const uint64_t *diag, int dl, uint64_t *inner, hipStream_t s);

nj_lt_t at_level(const nj_lt_t &lt, int l);
size_t bsgs_words(const nj_ctx *c, const nj_lt_t &lt);
// (last_out [2][N]: when the transform ends in a one-job ModDown it also writes its last
// limb after the first pass of an inverse transform there and sets *last_done)
// (drop: out goes on to a rescale and a drop to level 0; with lazy giant steps at N >= 8192
// only its limbs 0 and l are computed, the others are left undefined)
nj_status bsgs_apply(nj_ctx *c, const nj_lt_t &lt, const uint64_t *in, uint64_t *out, int hoist, Arena A,
                     hipStream_t s, uint64_t *last_out = nullptr, bool *last_done = nullptr, bool drop = false);
// bsgs_apply into y, then rescale into out (which may be x); the rescale's first pass
// rides on the transform's last ModDown where it can
nj_status bsgs_rescale(nj_ctx *c, const nj_lt_t &lt, const uint64_t *x, uint64_t *y, uint64_t *out, Arena A,
                       hipStream_t s);
size_t bsgs_batch_words(const nj_ctx *c, const nj_lt_t &lt, int K);
nj_status bsgs_apply_batch(nj_ctx *c, const nj_lt_t &lt, int K, const uint64_t *in, uint64_t *out, Arena A,
                           hipStream_t s);
nj_status apply_galois_batch(nj_ctx *c, int l, int K, const uint64_t *in, uint32_t g, uint64_t *out, Arena A,
                             hipStream_t s);
size_t block_words(const nj_ctx *c, const nj_lt_t &lt);
nj_status block_bsgs_apply(nj_ctx *c, const nj_lt_t &lt, const uint64_t *in, uint64_t *out, Arena A, hipStream_t s);

// rescale [2][l+1] -> [2][l]; n_out < l keeps only the first n_out limbs of the result
// (rescale followed by a level drop, computing only the kept limbs)
// n_polys > 2 (several ciphertexts packed at level l) needs N >= 8192
nj_status rescale(nj_ctx *c, int l, const uint64_t *in, uint64_t *out, Arena A, hipStream_t s, int n_out = -1,
                  int n_polys = 2, uint64_t *last_pre = nullptr);
// rescale of K packed ciphertexts [K][2][l+1] -> [K][2][l] (one set of launches when N >= 8192)
nj_status rescale_batch(nj_ctx *c, int l, int K, const uint64_t *in, uint64_t *out, Arena A, hipStream_t s);
nj_status modraise(nj_ctx *c, const uint64_t *in, int top, uint64_t *out, Arena A, hipStream_t s);
nj_status conj_split(nj_ctx *c, int l, const uint64_t *x, uint64_t *re, uint64_t *im, Arena A, hipStream_t s);

// ModRaise + CoeffToSlot + real split of n level-0 ciphertexts [n][2][1][N]
size_t cts_batch_words(const nj_ctx *c, const nj_plan *p, int Kmax);
nj_status cts_batch(nj_ctx *c, const nj_plan *p, const uint64_t *in, int n, uint64_t *const *re, uint64_t *const *im,
                    Arena A, hipStream_t s);
size_t cts_single_words(const nj_ctx *c, const nj_plan *p);
nj_status cts_single(nj_ctx *c, const nj_plan *p, const uint64_t *in, uint64_t *re, uint64_t *im, Arena A,
                     hipStream_t s);

}  // namespace ex
}  // namespace nj
