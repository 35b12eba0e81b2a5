// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "../../include/neujeans.h"
#include "modarith.h"

#define NJ_MAX_LIMBS 256  // limbs addressed by one launch (3 KiB limb table in the kernel arguments)

namespace nj {

// Per-launch limb -> prime table, passed by value in kernel arguments.
struct LimbTab {
    int n;
    int pidx[NJ_MAX_LIMBS];  // prime index of each launched limb
    int off[NJ_MAX_LIMBS];   // limb offset from the base pointer, in units of N words
    int soff[NJ_MAX_LIMBS];  // offset of the limb in an optional separate source buffer
};

// Per-prime constants resident in device memory (indexed by prime index).
struct PrimeInfo {
    Mod m;
    double ninv, ninvq;  // N^{-1} mod t and its Shoup companion
    double half;         // floor(t/2), for centred lifts
};

void set_error(const std::string &msg);
nj_status fail(nj_status code, const std::string &msg);
nj_status hip_fail(hipError_t e, const char *what);

#define NJ_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t _e = (call);                                                      \
        if (_e != hipSuccess) return ::nj::hip_fail(_e, #call);                      \
    } while (0)

// Basis-conversion constants of one ModUp digit at one level: from the digit's
// primes (m of them) to every other prime of Q_l u P.
struct BconvTab {
    int m;                 // primes in the digit
    int n_out;             // targets
    double *hat_inv;       // device [m]:  (D/q_a)^{-1} mod q_a
    double *hat;           // device [m][n_out]: (D/q_a) mod target
    int in_pidx[16];       // host copies
    std::vector<int> out_pidx;
    std::vector<int> out_limb;  // position of each target inside the extended array
};

struct Key {
    uint64_t *d = nullptr;  // device [dnum][2][L+1+alpha][N], evaluation form
};

// Many key switches at once (kernel arguments).
#define NJ_MAX_JOBS 16
struct BconvShared {  // per-digit tables of one basis conversion (ModUp digits, or the P basis)
    int nd;
    int m[4], n_out[4], in_off0[4];
    const double *hat_inv[4], *hat[4];
    int in_pidx[4][16];
    int out_pidx[4][48], out_off[4][48];
};
struct BconvPtrs {  // per job: input limbs base, output limbs base
    const uint64_t *in[2 * NJ_MAX_JOBS];
    uint64_t *out[2 * NJ_MAX_JOBS];
};
struct KeyJobs {
    const uint64_t *ext[NJ_MAX_JOBS], *d[NJ_MAX_JOBS], *key[NJ_MAX_JOBS];
    uint32_t g[NJ_MAX_JOBS];
};
__device__ __forceinline__ uint32_t brev_n(uint32_t x, int bits) { return __brev(x) >> (32 - bits); }

// Evaluation-form word k holds a(psi^(2 rev(k) + 1)); the word that X -> X^g moves to
// position k is the one at exponent (2 rev(k) + 1) g mod 2N.
__device__ __forceinline__ int galois_src2(int k, uint32_t g, int logN)
{
    const uint32_t N = 1u << logN;
    uint32_t e = 2u * brev_n((uint32_t)k, logN) + 1u;
    uint32_t eg = (uint32_t)(((uint64_t)e * g) & (2u * N - 1u));
    return (int)brev_n((eg - 1u) >> 1, logN);
}

// Output limb t of a key inner product at level l: t < l+1 is q_t, else p_(t-l-1); kl
// = the key's limb of t; own = the digit t belongs to (-1 for special primes).
// Sums need their operands at one scale: equal up to a relative 1e-9 (scales computed
// by the same sequence of steps are equal exactly).
inline bool same_scale(double a, double b) { return std::fabs(a - b) <= 1e-9 * std::fmax(std::fabs(a), std::fabs(b)); }

struct IpRow {
    size_t t, ne, nk, kl;
    int own;
};

__device__ __forceinline__ IpRow ip_row(int t, int level, int L, int alpha)
{
    IpRow r;
    r.t = t;
    r.ne = level + 1 + alpha;
    r.nk = L + 1 + alpha;
    r.kl = t <= level ? t : L + 1 + (t - level - 1);
    r.own = t <= level ? t / alpha : -1;
    return r;
}

// Raw buffer access (gfx9 buffer resource: base, size in bytes): a per-thread 32-bit
// byte offset plus a wave-uniform offset held in a scalar register, so strided loads
// of a column need no per-load 64-bit address arithmetic.  Accesses past `bytes` read
// 0 and write nothing.
typedef unsigned int nj_u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ uint64_t buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    const nj_u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return ((uint64_t)v.y << 32) | v.x;
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint64_t x)
{
    nj_u32x2 v;
    v.x = (uint32_t)x, v.y = (uint32_t)(x >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
}

// Real/imaginary split fused into a one-job ModDown combine: with the combined value
// xc of the conjugation key switch, re = x + xc and im = -X^{N/2} (x - xc) are written
// instead of xc (kernel argument; x null = off).
struct MdConj {
    const uint64_t *x;
    uint64_t *re, *im;
};
struct GalTab {  // Galois element of each job (1 = none)
    uint32_t g[NJ_MAX_JOBS];
};
struct MdJobs {
    const uint64_t *add[NJ_MAX_JOBS];
    uint32_t g_add[NJ_MAX_JOBS];
    uint64_t *out[NJ_MAX_JOBS];
};
struct AutoJobs {
    const uint64_t *in[NJ_MAX_JOBS];
    uint64_t *out[NJ_MAX_JOBS];
    uint32_t g[NJ_MAX_JOBS];
};

#define NJ_MAX_BABY 16
#define NJ_MAX_GIANT 16
// BSGS accumulation plan (kernel argument): d_of[g][b] = diagonal index or -1.
// Key inner products of jobs at different levels sharing one key (the top-level key
// serves every level: its digit j, limb t words do not depend on the level).
struct KeyJobsX {
    const uint64_t *ext[NJ_MAX_JOBS];  // extended digits [nd_z][l_z+1+alpha][N]
    const uint64_t *d[NJ_MAX_JOBS];    // own-digit limbs [l_z+1][N], read through X -> X^g[z]
    uint64_t *u[NJ_MAX_JOBS];          // output [2][l_z+1+alpha][N]
    uint32_t g[NJ_MAX_JOBS];
    int lv[NJ_MAX_JOBS];               // level l_z
};

// one residue per ciphertext prime (an integer constant reduced mod q_0..q_63)
struct LimbConsts {
    double v[64];
};

struct MacPlan {
    int nb, ng;
    int dl;  // limbs per stored diagonal (the plan's encoding level + 1)
    const uint64_t *baby[NJ_MAX_BABY];
    int d_of[NJ_MAX_GIANT][NJ_MAX_BABY];
};

struct Scratch {
    uint64_t *buf = nullptr;
    size_t words = 0;
};

// Live kernel timing: HIP events recorded on the launch stream around each
// launch of the profiled kernel families, with the launch's algorithmic bytes.
struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double bytes;
};
enum ProfKind {
    PROF_NTT_TILE = 0,  // forward tile pass; +1 for the inverse
    PROF_NTT_TILE_INV,
    PROF_NTT_COL,       // forward column pass; +1 for the inverse
    PROF_NTT_COL_INV,
    PROF_BCONV,
    PROF_KEYIP,
    PROF_PMAC,
    PROF_OTHER,
    PROF_NTT_MD,  // forward tile pass fused with the ModDown combine
    PROF_KINDS
};

}  // namespace nj

struct nj_ctx {
    int log_n, N, n_q, L, alpha, dnum, n_primes;
    double scale;
    int device;
    std::vector<uint64_t> primes;  // q_0..q_L, p_0..p_{alpha-1}
    nj::PrimeInfo *d_info = nullptr;
    std::vector<nj::PrimeInfo> info;
    double *d_tw = nullptr, *d_twq = nullptr, *d_itw = nullptr, *d_itwq = nullptr;  // [n_primes][N]
    // ModUp tables [level][digit]; ModDown tables [level]
    std::vector<std::vector<nj::BconvTab>> modup;
    std::vector<nj::BconvTab> moddown;
    // the same conversions with only the targets a rescale followed by a drop to level 0
    // reads: Q limbs 0 and l (and, for ModUp, the special primes)
    std::vector<std::vector<nj::BconvTab>> modup_drop;
    std::vector<nj::BconvTab> moddown_drop;
    // per level: device [l+1] N^-1 (D_j/q_i)^-1 mod q_i (i in digit j), the ModUp inputs'
    // factor folded into their inverse transform; and [n_primes] N^-1 (P/p_a)^-1 mod p_a
    std::vector<double *> d_upscale;
    double *d_downscale = nullptr;
    std::vector<double> pinv_q;   // P^{-1} mod q_i (host)
    std::vector<double> pmod;     // P mod every prime (host), 0 for the p's
    double *d_pinv = nullptr, *d_pinvq = nullptr;  // [n_q] P^{-1} mod q_i and companion
    double *d_qlinv = nullptr, *d_qlinvq = nullptr;  // [n_q][n_q]: q_l^{-1} mod q_i
    uint64_t *d_primes = nullptr;                     // [n_primes]
    double *d_pmod = nullptr;                         // [L+1+alpha] P mod each key limb's prime
    // secret key in evaluation form [n_primes][N]
    std::vector<int8_t> s;
    uint64_t *d_s = nullptr;
    uint64_t *d_pk = nullptr;  // public key [2][L+1][N], evaluation form (nj_gen_public_key)
    std::map<uint32_t, nj::Key> keys;
    std::vector<uint64_t *> timing_keys;  // latency measurement: random key buffers for missing elements
    nj::Scratch scratch;
    // ModEval's Chebyshev baby-step sums: 0 = one constant multiply and rescale per
    // term, 1 = integer multiples accumulated at one level and rescaled once (nj_eval_order)
    int eval_order = 0;
    // intermediate ciphertexts of the composite calls (Algorithm 1, bootstrapping)
    uint64_t *layer_buf = nullptr;
    size_t layer_words = 0;
    // worker streams of the concurrent job schedule (nj_batch_run mode 2), made on
    // first use at the default priority, with a fork event and one join event each
    int batch_workers = 4;
    std::vector<hipStream_t> workers;
    std::vector<hipEvent_t> worker_done;
    hipEvent_t fork_ev = nullptr;
    // live profiling (nj_prof_*)
    bool prof = false;
    std::vector<nj::ProfRec> prof_recs;
    std::vector<hipEvent_t> ev_pool;
};

#include <hip/hip_ext.h>

namespace nj {
// Records events around a launch when profiling is on (no-op otherwise).
struct ProfScope {
    nj_ctx *c;
    ProfRec r;
    hipStream_t s;
    ProfScope(const nj_ctx *cc, int kind, double bytes, hipStream_t st);
    ~ProfScope();
};

// Events for one profiled launch (pushed into the context's records), or false.
bool prof_events(const nj_ctx *c, int kind, double bytes, hipEvent_t *a, hipEvent_t *b);

// Kernel launch; when profiling, hipExtLaunchKernelGGL has the dispatch itself
// timestamp its start and end into two events (kernel time only, no host gaps).
template <typename F, typename... Args>
inline hipError_t launch(const nj_ctx *c, int kind, double bytes, F kernel, dim3 grid, dim3 block, hipStream_t s,
                         Args... args)
{
    hipEvent_t a, b;
    if (c->prof && prof_events(c, kind, bytes, &a, &b))
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    return hipGetLastError();
}
}  // namespace nj

struct nj_lt_t {
    int level, u, n1, n_diag;
    std::vector<int> js;                 // offsets j (diagonal j*u)
    std::vector<int> g_of, i_of;         // BSGS split j = g n1 + i
    std::vector<int> babies, giants;
    uint64_t *d_diag = nullptr;          // [bo][bi][n_diag][dl][N] evaluation form
    int dl = 0;                          // limbs per diagonal: encoded at level dl-1, usable at any level below
    double scale = 0.0;                  // encoding scale of the diagonals
    int bi = 1, bo = 1;                  // block conv: input / output ciphertexts
    bool lazy = false;                   // giant steps share one ModDown
    bool hoist = true;                   // baby steps share one ModUp of c1
    int stages = 0;                      // DFT butterfly stages merged into the transform (fusion depth)
    std::vector<char> nz;                // [bo][bi][n_diag] nonzero diagonals (empty = all)
};

struct nj_plan {
    int kind;  // 0 conv, 1 CoeffToSlot, 2 StoC1
    int N = 0;
    std::vector<nj_lt_t> lts;
    // conv layout
    int W = 0, C = 0, ell = 0, w0 = 0, f = 0;
    int c_in = 0, c_out = 0;
};

namespace nj {

// ---------------------------------------------------------------- kernels.hip
hipError_t launch_ntt(const nj_ctx *c, uint64_t *data, const LimbTab &lt, bool inverse, hipStream_t s,
                      const uint64_t *src = nullptr);
// (gt: limb b of job off[b] / L1 is read from src through X -> X^g[job])
hipError_t launch_intt_scaled(const nj_ctx *c, uint64_t *data, const uint64_t *src, const LimbTab &lt,
                              const double *scale, hipStream_t s, const GalTab *gt = nullptr, int L1 = 0);
hipError_t launch_rescale_fused(const nj_ctx *c, int level, const uint64_t *in, uint64_t *out, int n_out,
                                uint64_t *last, uint64_t *lifted, hipStream_t s, int n_polys = 2, bool last_tiled = false);
hipError_t launch_ntt_tiles(const nj_ctx *c, uint64_t *data, const LimbTab &lt, hipStream_t s);
hipError_t launch_bconv_col(const nj_ctx *c, const BconvShared &sh, const BconvPtrs &jp, int n_jobs, hipStream_t s);
// key inner products fused with the extended digits' forward tile pass (N >= 8192,
// 1..4 digits, every g = 1): per job u_base + z 2 ne N, or (sum) one output summed over
// the jobs; accumulate adds to the output's previous value
hipError_t launch_ntt_ip(const nj_ctx *c, int level, const KeyJobs &kj, int n_jobs, uint64_t *u, int sum,
                         int accumulate, hipStream_t s, uint64_t *pout = nullptr, int skip = 0);
// (pout given: the special-prime rows skip u and leave through the first 12 stages of
// ModDown's inverse transform, job z's halves at rows (2 z + p) alpha + a of pout;
// skip > 0: Q limbs 1..skip are not computed, skip = l - 1 keeping Q limbs 0 and l)
// special-prime rows of n_jobs key inner products whose digits are extended and in
// evaluation form (KeyJobs as for launch_key_ip_multi): the products pass through the
// first 12 stages of ModDown's inverse transform into pout, job z's halves at rows
// (2 z + p) alpha + a (N >= 8192, 1..4 digits, alpha <= 8)
hipError_t launch_key_ip_ptile(const nj_ctx *c, int level, const KeyJobs &kj, int n_jobs, uint64_t *pout,
                               hipStream_t s);
// centred lift of n_polys limbs (prime src_pidx, coefficient form, src + z N) into
// primes 0..n_out-1 with the column pass applied, out [n_polys][n_out][N] (N >= 8192)
hipError_t launch_lift_col(const nj_ctx *c, const uint64_t *src, int src_pidx, int n_polys, int n_out, uint64_t *out,
                           hipStream_t s);
hipError_t launch_intt_cols_scaled(const nj_ctx *c, uint64_t *data, const LimbTab &lt, const double *scale,
                                   hipStream_t s);
// (acc0: job 0's previous value read from there instead of its output; last_out, one
// job: the last limb also leaves through the first 12 stages of its inverse transform
// into last_out [2][N], for launch_rescale_fused(last_tiled))
// skip > 0 (with cols_done, no last_out or conj): only output limbs 0 and 1 + skip ..
// the plain combine of launch_ntt_moddown (no accumulation, converted limbs column-passed)
// with the jobs' Q-limb key inner products computed inside it from extended
// evaluation-form digits (KeyJobs as for launch_key_ip_multi; N >= 8192, 1..4 digits)
hipError_t launch_key_ip_moddown(const nj_ctx *c, int level, int K, const uint64_t *conv, const KeyJobs &kj,
                                 const MdJobs &mj, hipStream_t s);
hipError_t launch_ntt_moddown(const nj_ctx *c, int level, int K, uint64_t *conv, const uint64_t *u_base,
                              const MdJobs &mj, int acc, int cols_done, hipStream_t s, const uint64_t *acc0 = nullptr,
                              uint64_t *last_out = nullptr, const MdConj *conj = nullptr, int skip = 0);
hipError_t launch_ntt_fast(const nj_ctx *c, uint64_t *data, const uint64_t *src, const LimbTab &lt, bool inverse,
                           hipStream_t s);
// out = a op b per limb (op 0 add, 1 sub, 2 mul), evaluation form
hipError_t launch_elementwise(const nj_ctx *c, int op, const uint64_t *a, const uint64_t *b, uint64_t *out,
                              const LimbTab &lt, hipStream_t s);
// out limb i = in limb i read through X -> X^g (evaluation form, contiguous limbs)
hipError_t launch_automorph(const nj_ctx *c, const uint64_t *in, uint64_t *out, uint32_t g, int n_limbs,
                            hipStream_t s);
hipError_t launch_lift_last(const nj_ctx *c, const uint64_t *src, int src_pidx, int n_out, uint64_t *dst,
                            hipStream_t s);
hipError_t launch_rescale_combine(const nj_ctx *c, int level, const uint64_t *a, const uint64_t *lifted, uint64_t *out,
                                  hipStream_t s,
                                  int n_out = -1);
hipError_t launch_pmac(const nj_ctx *c, int level, const uint64_t *ct, const uint64_t *pt, uint64_t *acc, int first,
                       hipStream_t s);
hipError_t launch_monomial_half(const nj_ctx *c, int level, const uint64_t *in, uint64_t *out, hipStream_t s);
// re = x + xc, im = -X^{N/2} (x - xc) over both polynomials (re, im must not alias x, xc)
hipError_t launch_conj_split(const nj_ctx *c, int level, const uint64_t *x, const uint64_t *xc, uint64_t *re,
                             uint64_t *im, hipStream_t s);
hipError_t launch_signed_to_rns(const nj_ctx *c, const int64_t *coeffs, const LimbTab &lt, uint64_t *out,
                                hipStream_t s, const uint64_t *d_primes);
hipError_t launch_keygen_combine(const nj_ctx *c, int digit, uint64_t *b, const uint64_t *a, const uint64_t *e,
                                 const uint64_t *s_eval, const uint64_t *sp_eval, const double *d_pmod, hipStream_t s);


// ------------------------------------------------------------------- ksw.hip
hipError_t launch_bconv_multi(const nj_ctx *c, const BconvShared &sh, const BconvPtrs &jp, int n_jobs, hipStream_t s);
// key inner products of n_jobs jobs into u_base + z 2 ne N, output limbs 0..rows-1 (rows
// < 0: all l + 1 + alpha; rows = l + 1: the Q limbs alone)
hipError_t launch_key_ip_multi(const nj_ctx *c, int level, const KeyJobs &kj, int n_jobs, uint64_t *u_base,
                               hipStream_t s, int rows = -1);
hipError_t launch_moddown_multi(const nj_ctx *c, int level, const MdJobs &mj, int n_jobs, int sum,
                                const uint64_t *u_base, const uint64_t *conv_base, const uint64_t *acc, hipStream_t s);
hipError_t launch_automorph_multi(const nj_ctx *c, const AutoJobs &aj, int n_jobs, int n_limbs, hipStream_t s);
hipError_t launch_key_ip_shared(const nj_ctx *c, int level, const KeyJobs &kj, int n_jobs, const uint64_t *key,
                                uint64_t *u_base, hipStream_t s,
                                int accumulate = 0);
hipError_t launch_bsgs_mac_multi(const nj_ctx *c, int level, const MacPlan &mp, int n_ct, size_t bstride,
                                 size_t istride, const uint64_t *diag, uint64_t *inner, int n_diag, hipStream_t s);
// inner[g] = sum_b baby_b (.) diag[d_of[g][b]] for every giant g; inner [ng][2][l+1][N]
hipError_t launch_tensor(const nj_ctx *c, const uint64_t *a, size_t astride, const uint64_t *b, size_t bstride,
                         uint64_t *d01, uint64_t *d2, int level, hipStream_t s);
hipError_t launch_mul_int(const nj_ctx *c, const uint64_t *in, size_t istride, uint64_t *out, int n_limbs,
                          const LimbConsts &kc, hipStream_t s, int accumulate = 0, int n_polys = 2);
hipError_t launch_add_int(const nj_ctx *c, uint64_t *poly, int n_limbs, const LimbConsts &kc, hipStream_t s);
hipError_t launch_zero(const nj_ctx *c, uint64_t *p, size_t words, hipStream_t s);
hipError_t launch_key_ip_sum(const nj_ctx *c, int level, const KeyJobs &kj, int n_jobs, uint64_t *u, int accumulate,
                             hipStream_t s);
// (skip > 0: limbs 1..skip left out)
hipError_t launch_automorph_acc(const nj_ctx *c, const AutoJobs &aj, int n_jobs, int n_limbs, uint64_t *out,
                                size_t ostride, int mode, hipStream_t s, int skip = 0);
hipError_t launch_key_ip_mixed(const nj_ctx *c, const KeyJobsX &kj, int n_jobs, const uint64_t *key, hipStream_t s);
hipError_t launch_bsgs_mac(const nj_ctx *c, int level, const MacPlan &mp, const uint64_t *diag, uint64_t *inner,
                           int n_diag, hipStream_t s,
                           int accumulate = 0);

// --------------------------------------------------------------- noalloc.hip
// looks up (once per device, the device current) the static scratch of
// nj_apply_galois_noalloc
hipError_t noalloc_init(int device);

// ------------------------------------------------------------------- ctx.hip
LimbTab limbs_q(int level);                       // q_0..q_l
LimbTab limbs_ext(const nj_ctx *c, int level);    // q_0..q_l, p_0..p_{alpha-1}
uint64_t *scratch_get(nj_ctx *c, size_t words);   // ctx-owned, grows on demand (synchronises)
int n_digits(const nj_ctx *c, int level);

// ------------------------------------------------------------------ encode.cpp
void special_idft(int n, std::vector<double> &re, std::vector<double> &im);   // slots -> V^{-1} z
void special_dft(int n, std::vector<double> &re, std::vector<double> &im);    // V w -> slots
void encode_slots(int N, const double *z_re, const double *z_im, double scale, int64_t *out);
void encode_cins(int N, const double *chans, int slice2, double scale, int64_t *out);
void decode_slots(int N, const double *coeffs, double scale, double *z_re, double *z_im);
nj_status build_conv_diagonals(int N, int w0, int f, const double *weights, int n1, nj_lt_t &lt,
                               std::vector<std::vector<double>> &dre, std::vector<std::vector<double>> &dim);
nj_status build_cts_diagonals(int N, int groups, const int *n1s, std::vector<nj_lt_t> &lts,
                              std::vector<std::vector<std::vector<double>>> &dre,
                              std::vector<std::vector<std::vector<double>>> &dim);
nj_status build_block_diagonals(int N, int W, int c_in, int c_out, const nj_tap *taps, int n_taps, int fuse, int n1,
                                nj_lt_t &lt, std::vector<std::vector<double>> &dre,
                                std::vector<std::vector<double>> &dim);
nj_status build_fc_diagonals(int N, int n_in, int n_out, const double *W, int n1, nj_lt_t &lt,
                             std::vector<std::vector<double>> &dre, std::vector<std::vector<double>> &dim);
nj_status build_downsample_diagonals(int N, int kind, int W, int C, int half, int n1, nj_lt_t &lt,
                                     std::vector<std::vector<double>> &dre, std::vector<std::vector<double>> &dim);
nj_status build_stoc1_diagonals(int N, int ell, int groups, std::vector<nj_lt_t> &lts,
                                std::vector<std::vector<std::vector<double>>> &dre,
                                std::vector<std::vector<std::vector<double>>> &dim);
void cheb_interpolate_cos(int degree, double K, int r, double *c);
// encode a transform's complex diagonals at `scale` into its level's primes, NTT, keep on device
nj_status upload_plan_diagonals(nj_ctx *c, nj_lt_t &lt, const std::vector<std::vector<double>> &re,
                                const std::vector<std::vector<double>> &im, double scale);
void bsgs_split(nj_lt_t &lt, int n);

}  // namespace nj
