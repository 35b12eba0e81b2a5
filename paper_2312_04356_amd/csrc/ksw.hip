// Hybrid key switching and BSGS accumulation kernels (gfx950).  Every key switch runs
// as a batch of jobs (one job being the plain case): ModUp's basis conversion
// (k_bconv_multi; at N >= 8192 the fused conversion + column pass in ntt.hip), key inner
// products (k_key_ip_multi / _sum / _shared / _mixed: one job per key, a sum over jobs,
// one key for many ciphertexts, one key for jobs at mixed levels), the ModDown combine
// (k_moddown_multi, or fused into the tile pass in ntt.hip) and the automorphisms.
//
//  * k_bsgs_mac: every giant step's inner sum sum_i baby_i (.) diag_{g,i} in one pass:
//    each baby and each diagonal word is read once.
#include <algorithm>

#include "internal.h"

namespace nj {

constexpr int kBT = 256;


// ------------------------------------------------------- key inner product

// Key inner product terms of one key switch at output limb t: for digit j the input
// word (the digit's own limb d when j is t's digit, else the extended digit j), read
// through X -> X^g at src, and the two key words.  ND = number of digits: for ND > 0
// all 3 ND loads are issued before any is used; ND = 0 is the generic loop.
template <int ND>
__device__ __forceinline__ void ip_load(const IpRow &r, const uint64_t *ext, const uint64_t *d, const uint64_t *key,
                                        int src, int k, size_t N, uint64_t *rx, uint64_t *rb, uint64_t *ra)
{
#pragma unroll
    for (int j = 0; j < ND; j++) {
        const uint64_t *xp = j == r.own ? d + r.t * N : ext + ((size_t)j * r.ne + r.t) * N;
        rx[j] = xp[src];
        rb[j] = key[(((size_t)j * 2 + 0) * r.nk + r.kl) * N + k];
        ra[j] = key[(((size_t)j * 2 + 1) * r.nk + r.kl) * N + k];
    }
}

// a0 += sum_j x_j b_j, a1 += sum_j x_j a_j (lazy products in (-t, t), no reduction)
template <int ND>
__device__ __forceinline__ void ip_acc(const uint64_t *rx, const uint64_t *rb, const uint64_t *ra, double &a0,
                                       double &a1, Mod m)
{
#pragma unroll
    for (int j = 0; j < ND; j++) {
        const double x = u2d(rx[j]);
        a0 += mul_lazy(x, u2d(rb[j]), m);
        a1 += mul_lazy(x, u2d(ra[j]), m);
    }
}

// generic digit count: one digit at a time, reduced after every 8 terms (start 0)
__device__ __forceinline__ void ip_generic(const IpRow &r, const uint64_t *ext, const uint64_t *d,
                                           const uint64_t *key, int src, int k, size_t N, int n_digits, double &a0,
                                           double &a1, Mod m)
{
    for (int j = 0; j < n_digits; j++) {
        const uint64_t *xp = j == r.own ? d + r.t * N : ext + ((size_t)j * r.ne + r.t) * N;
        const double x = u2d(xp[src]);
        a0 += mul_lazy(x, u2d(key[(((size_t)j * 2 + 0) * r.nk + r.kl) * N + k]), m);
        a1 += mul_lazy(x, u2d(key[(((size_t)j * 2 + 1) * r.nk + r.kl) * N + k]), m);
        if ((j & 7) == 7) a0 = reduce(a0, m), a1 = reduce(a1, m);
    }
}

// one key switch: (a0, a1) = sum over digits, reduced to [0, t)
template <int ND>
__device__ __forceinline__ void ip_one(const IpRow &r, const uint64_t *ext, const uint64_t *d, const uint64_t *key,
                                       int src, int k, size_t N, int n_digits, double &a0, double &a1, Mod m)
{
    a0 = 0.0, a1 = 0.0;
    if constexpr (ND > 0) {
        uint64_t rx[ND], rb[ND], ra[ND];
        ip_load<ND>(r, ext, d, key, src, k, N, rx, rb, ra);
        ip_acc<ND>(rx, rb, ra, a0, a1, m);
    } else {
        ip_generic(r, ext, d, key, src, k, N, n_digits, a0, a1, m);
    }
    a0 = reduce(a0, m), a1 = reduce(a1, m);
}

// returns EXPR with the compile-time digit count ND: 1..4 unrolled, 0 = generic loop
#define NJ_ND_SWITCH(nd, EXPR)                   \
    switch (nd) {                                \
    case 1: { constexpr int ND = 1; return EXPR; } \
    case 2: { constexpr int ND = 2; return EXPR; } \
    case 3: { constexpr int ND = 3; return EXPR; } \
    case 4: { constexpr int ND = 4; return EXPR; } \
    default: { constexpr int ND = 0; return EXPR; } \
    }

// ------------------------------------------------------------------- BSGS

// Loads are issued for every static slot b < NBM from an address that is always in
// bounds (babies beyond nb read baby nb-1, absent diagonals read another diagonal of
// the same giant step) and masked to zero afterwards, so a wave has a whole giant
// step's words in flight at once instead of waiting on one data-dependent load at a time.
template <int NBM>
__device__ __forceinline__ void load_babies(const MacPlan &mp, size_t zoff, size_t o0, size_t o1, double *b0,
                                            double *b1)
{
    uint64_t r0[NBM], r1[NBM];
#pragma unroll
    for (int b = 0; b < NBM; b++) {
        const uint64_t *bp = mp.baby[b < mp.nb ? b : mp.nb - 1] + zoff;
        r0[b] = bp[o0];
        r1[b] = bp[o1];
    }
#pragma unroll
    for (int b = 0; b < NBM; b++) {
        b0[b] = b < mp.nb ? u2d(r0[b]) : 0.0;
        b1[b] = b < mp.nb ? u2d(r1[b]) : 0.0;
    }
}

// w[b] = word o of diagonal d_of[g][b] (diagonals dstride words apart), zero where
// absent; false if giant step g has no diagonal at all
template <int NBM>
__device__ __forceinline__ bool load_giant(const MacPlan &mp, int g, const uint64_t *diag, size_t dstride, size_t o,
                                           double *w)
{
    int any = -1;
#pragma unroll
    for (int b = 0; b < NBM; b++)
        if (b < mp.nb && mp.d_of[g][b] >= 0) any = mp.d_of[g][b];
    if (any < 0) return false;
    uint64_t r[NBM];
#pragma unroll
    for (int b = 0; b < NBM; b++) {
        const int d = b < mp.nb ? mp.d_of[g][b] : -1;
        r[b] = diag[(size_t)(d < 0 ? any : d) * dstride + o];
    }
#pragma unroll
    for (int b = 0; b < NBM; b++) {
        const int d = b < mp.nb ? mp.d_of[g][b] : -1;
        w[b] = d < 0 ? 0.0 : u2d(r[b]);
    }
    return true;
}

// sum_b x[b] w[b] mod t from a start value in [0, t): products are lazy, in (-t, t),
// and the sum is reduced after every 7 of them, so it stays below 8t <= 2^53
template <int NBM>
__device__ __forceinline__ double mac_row(double a, const double *x, const double *w, Mod m)
{
#pragma unroll
    for (int b = 0; b < NBM; b++) {
        a += mul_lazy(x[b], w[b], m);
        if (b % 7 == 6 && b + 1 < NBM) a = reduce(a, m);
    }
    return reduce(a, m);
}

template <int NBM>
__global__ __launch_bounds__(kBT) void k_bsgs_mac(MacPlan mp, const uint64_t *diag, uint64_t *inner, int level,
                                                 int accumulate, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, i = blockIdx.y;
    const int k = blockIdx.x * kBT + threadIdx.x;
    if (k >= N) return;
    const Mod m = info[i].m;
    const size_t L1 = level + 1, o = (size_t)i * N + k;
    double b0[NBM], b1[NBM];
    load_babies<NBM>(mp, 0, o, L1 * N + o, b0, b1);
    for (int g = 0; g < mp.ng; g++) {
        uint64_t *o0 = inner + (size_t)g * 2 * L1 * N + o, *o1 = o0 + L1 * N;
        double w[NBM];
        const bool any = load_giant<NBM>(mp, g, diag, (size_t)mp.dl * N, o, w);
        const double a0 = accumulate ? u2d(*o0) : 0.0, a1 = accumulate ? u2d(*o1) : 0.0;
        if (!any) {
            if (!accumulate) *o0 = 0, *o1 = 0;
            continue;
        }
        *o0 = d2u(mac_row<NBM>(a0, b0, w, m));
        *o1 = d2u(mac_row<NBM>(a1, b1, w, m));
    }
}

// --------------------------------------------------- many key switches at once
//
// k_bconv_multi: basis conversion for many (job, digit) pairs sharing the digit
// tables (blockIdx.z = job * nd + digit).  MMAX bounds the digit size: all MMAX input
// loads are issued at once from in-bounds limbs (slots past the digit re-read its last
// limb and are zeroed after scaling), and the block's chunk of 8 targets is unrolled
// (targets past n_out predicated), so the scalar table reads of all 8 can be batched.
template <int MMAX>
__global__ __launch_bounds__(kBT) void k_bconv_multi(BconvShared sh, BconvPtrs jp, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN;
    const int job = blockIdx.z / sh.nd, j = blockIdx.z % sh.nd;
    const int k = blockIdx.x * kBT + threadIdx.x;
    const int o0 = blockIdx.y * 8, n_out = sh.n_out[j], m = sh.m[j];
    if (k >= N || o0 >= n_out) return;
    const uint64_t *in = jp.in[job];
    uint64_t *out = jp.out[job];
    const double *hat_inv = sh.hat_inv[j], *hat = sh.hat[j];
    uint64_t raw[MMAX];
#pragma unroll
    for (int a = 0; a < MMAX; a++) raw[a] = in[(size_t)(sh.in_off0[j] + (a < m ? a : m - 1)) * N + k];
    double v[MMAX];
#pragma unroll
    for (int a = 0; a < MMAX; a++) {
        const int aa = a < m ? a : m - 1;
        const double x = mul_canon(u2d(raw[a]), hat_inv[aa], info[sh.in_pidx[j][aa]].m);
        v[a] = a < m ? x : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int o = o0 + q;
        if (o < n_out) {
            const Mod mt = info[sh.out_pidx[j][o]].m;
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < MMAX; a++) {
                acc += mul_lazy(v[a], hat[(a < m ? a : 0) * n_out + o], mt);
                if ((a & 7) == 7) acc = reduce(acc, mt);
            }
            out[(size_t)sh.out_off[j][o] * N + k] = d2u(reduce(acc, mt));
        }
    }
}

hipError_t launch_bconv_multi(const nj_ctx *c, const BconvShared &sh, const BconvPtrs &jp, int n_jobs, hipStream_t s)
{
    if (n_jobs == 0) return hipSuccess;
    int max_out = 0, mmax = 0;
    double bytes = 0;
    for (int j = 0; j < sh.nd; j++) {
        max_out = max(max_out, sh.n_out[j]);
        mmax = max(mmax, sh.m[j]);
        bytes += 8.0 * c->N * (sh.m[j] + sh.n_out[j]) * n_jobs;
    }
    dim3 grid((c->N + kBT - 1) / kBT, (max_out + 7) / 8, n_jobs * sh.nd);
    if (mmax <= 2) return launch(c, PROF_BCONV, bytes, k_bconv_multi<2>, grid, dim3(kBT), s, sh, jp, c->d_info, c->log_n);
    if (mmax <= 4) return launch(c, PROF_BCONV, bytes, k_bconv_multi<4>, grid, dim3(kBT), s, sh, jp, c->d_info, c->log_n);
    if (mmax <= 8) return launch(c, PROF_BCONV, bytes, k_bconv_multi<8>, grid, dim3(kBT), s, sh, jp, c->d_info, c->log_n);
    return launch(c, PROF_BCONV, bytes, k_bconv_multi<16>, grid, dim3(kBT), s, sh, jp, c->d_info, c->log_n);
}

// key inner products of many jobs (blockIdx.z = job); u of job z at u_base + z * 2 ne N
template <int ND>
__global__ __launch_bounds__(kBT) void k_key_ip_multi(KeyJobs kj, uint64_t *u_base, int n_digits, int level, int L,
                                                     int alpha, int nq, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN;
    const int t = blockIdx.y, z = blockIdx.z;
    const int pidx = t <= level ? t : nq + (t - level - 1);
    const Mod m = info[pidx].m;
    const int k = blockIdx.x * kBT + threadIdx.x;
    if (k >= N) return;
    const IpRow r = ip_row(t, level, L, alpha);
    const uint32_t g = kj.g[z];
    const int src = g == 1u ? k : galois_src2(k, g, logN);
    double a0, a1;
    ip_one<ND>(r, kj.ext[z], kj.d[z], kj.key[z], src, k, N, n_digits, a0, a1, m);
    uint64_t *u = u_base + (size_t)z * 2 * r.ne * N;
    u[(size_t)t * N + k] = d2u(a0);
    u[(r.ne + t) * N + k] = d2u(a1);
}

// lazy giant steps: sum over the jobs (each its own key) of the key inner products,
// written to u [2][ne][N] or added to it (accumulate)
// For ND in 1..3 two jobs are loaded together (6 ND words in flight) and the running
// sum, in [0, t) after each reduction, takes at most 2 ND <= 6 lazy terms before the
// next; for ND = 4 one job at a time (4 terms); the generic loop reduces every 8 terms.
template <int ND>
__global__ __launch_bounds__(kBT) void k_key_ip_sum(KeyJobs kj, int n_jobs, uint64_t *u, int accumulate, int n_digits,
                                                   int level, int L, int alpha, int nq, const PrimeInfo *info,
                                                   int logN)
{
    const int N = 1 << logN;
    const int t = blockIdx.y;
    const int pidx = t <= level ? t : nq + (t - level - 1);
    const Mod m = info[pidx].m;
    const int k = blockIdx.x * kBT + threadIdx.x;
    if (k >= N) return;
    const IpRow r = ip_row(t, level, L, alpha);
    const size_t o0 = (size_t)t * N + k, o1 = (r.ne + t) * N + k;
    double acc0 = accumulate ? u2d(u[o0]) : 0.0, acc1 = accumulate ? u2d(u[o1]) : 0.0;
    if constexpr (ND > 0) {
        constexpr int ZU = ND <= 3 ? 2 : 1;
        int z = 0;
        for (; z + ZU <= n_jobs; z += ZU) {
            uint64_t rx[ZU][ND], rb[ZU][ND], ra[ZU][ND];
#pragma unroll
            for (int q = 0; q < ZU; q++) {
                const uint32_t g = kj.g[z + q];
                const int src = g == 1u ? k : galois_src2(k, g, logN);
                ip_load<ND>(r, kj.ext[z + q], kj.d[z + q], kj.key[z + q], src, k, N, rx[q], rb[q], ra[q]);
            }
#pragma unroll
            for (int q = 0; q < ZU; q++) ip_acc<ND>(rx[q], rb[q], ra[q], acc0, acc1, m);
            acc0 = reduce(acc0, m), acc1 = reduce(acc1, m);
        }
        for (; z < n_jobs; z++) {
            const uint32_t g = kj.g[z];
            const int src = g == 1u ? k : galois_src2(k, g, logN);
            uint64_t rx[ND], rb[ND], ra[ND];
            ip_load<ND>(r, kj.ext[z], kj.d[z], kj.key[z], src, k, N, rx, rb, ra);
            ip_acc<ND>(rx, rb, ra, acc0, acc1, m);
            acc0 = reduce(acc0, m), acc1 = reduce(acc1, m);
        }
    } else {
        for (int z = 0; z < n_jobs; z++) {
            const uint32_t g = kj.g[z];
            const int src = g == 1u ? k : galois_src2(k, g, logN);
            double a0, a1;
            ip_one<0>(r, kj.ext[z], kj.d[z], kj.key[z], src, k, N, n_digits, a0, a1, m);
            acc0 = add_mod(reduce(acc0, m), a0, m), acc1 = add_mod(reduce(acc1, m), a1, m);
        }
    }
    u[o0] = d2u(reduce(acc0, m));
    u[o1] = d2u(reduce(acc1, m));
}

hipError_t launch_key_ip_sum(const nj_ctx *c, int level, const KeyJobs &kj, int n_jobs, uint64_t *u, int accumulate,
                             hipStream_t s)
{
    const int nd = n_digits(c, level), ne = level + 1 + c->alpha;
    dim3 grid((c->N + kBT - 1) / kBT, ne);
    NJ_ND_SWITCH(nd, launch(c, PROF_KEYIP, 8.0 * c->N * ne * (3.0 * nd * n_jobs + 2.0 * (1 + accumulate)),
                            k_key_ip_sum<ND>, grid, dim3(kBT), s, kj, n_jobs, u, accumulate, nd, level, c->L,
                            c->alpha, c->n_q, c->d_info, c->log_n));
}

hipError_t launch_key_ip_multi(const nj_ctx *c, int level, const KeyJobs &kj, int n_jobs, uint64_t *u_base,
                               hipStream_t s, int rows)
{
    const int nd = n_digits(c, level), ne = level + 1 + c->alpha;
    if (rows < 0) rows = ne;
    if (rows < 1 || rows > ne) return hipErrorInvalidValue;
    dim3 grid((c->N + kBT - 1) / kBT, rows, n_jobs);
    NJ_ND_SWITCH(nd, launch(c, PROF_KEYIP, 8.0 * c->N * rows * (3.0 * nd + 2.0) * n_jobs, k_key_ip_multi<ND>, grid,
                            dim3(kBT), s, kj, u_base, nd, level, c->L, c->alpha, c->n_q, c->d_info, c->log_n));
}

// ModDown combine of many jobs.  sum == 0: job z writes out[z] (blockIdx.z = 2 job + half),
// adding the previous out[z] when acc is non-null; sum == 1: out[0] = acc + sum over jobs
// (blockIdx.z = half).  Job z's u at u_base + z 2 ne N,
// its converted limbs at conv_base + z 2 (l+1) N, its c0 (read through X -> X^g_add[z]) at add[z].
__global__ __launch_bounds__(kBT) void k_moddown_multi(MdJobs mj, int n_jobs, int sum, const uint64_t *u_base,
                                                      const uint64_t *conv_base, const uint64_t *acc, int level,
                                                      int ne, const double *pinv, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, i = blockIdx.y;
    const int k = blockIdx.x * kBT + threadIdx.x;
    if (k >= N) return;
    const Mod m = info[i].m;
    const int L1 = level + 1;
    const int p = sum ? blockIdx.z : (blockIdx.z & 1);
    const int z0 = sum ? 0 : (blockIdx.z >> 1), z1 = sum ? n_jobs : z0 + 1;
    double r = 0.0;
    for (int z = z0; z < z1; z++) {
        const uint64_t *u = u_base + (size_t)z * 2 * ne * N, *cv = conv_base + (size_t)z * 2 * L1 * N;
        double t = mul_canon(sub_mod(u2d(u[((size_t)p * ne + i) * N + k]), u2d(cv[((size_t)p * L1 + i) * N + k]), m),
                             pinv[i], m);
        if (p == 0 && mj.add[z]) {
            const uint32_t g = mj.g_add[z];
            const int src = g <= 1u ? k : galois_src2(k, g, logN);
            t = add_mod(t, u2d(mj.add[z][(size_t)i * N + src]), m);
        }
        r = add_mod(r, t, m);
    }
    const size_t o = ((size_t)p * L1 + i) * N + k;
    if (sum) {
        if (acc) r = add_mod(r, u2d(acc[o]), m);
        mj.out[0][o] = d2u(r);
    } else {
        if (acc) r = add_mod(r, u2d(mj.out[z0][o]), m);  // accumulate into the job's own output
        mj.out[z0][o] = d2u(r);
    }
}

hipError_t launch_moddown_multi(const nj_ctx *c, int level, const MdJobs &mj, int n_jobs, int sum,
                                const uint64_t *u_base, const uint64_t *conv_base, const uint64_t *acc, hipStream_t s)
{
    dim3 grid((c->N + kBT - 1) / kBT, level + 1, sum ? 2 : 2 * n_jobs);
    const double bytes = 8.0 * c->N * (level + 1) * (n_jobs * 5.0 + (sum ? 2.0 : 2.0 * n_jobs) + (acc ? 2.0 : 0.0));
    return launch(c, PROF_OTHER, bytes, k_moddown_multi, grid, dim3(kBT), s, mj, n_jobs, sum, u_base, conv_base, acc,
                  level, level + 1 + c->alpha, c->d_pinv, c->d_info, c->log_n);
}

// Key inner products of many ciphertexts with ONE key (batched execution): each key
// word is read once and applied to every ciphertext's extended digits.  Job z reads
// its digits at kj.ext[z] (own-digit limbs at kj.d[z]) through X -> X^kj.g[z] and writes
// u_base + z 2 ne N.
__global__ __launch_bounds__(kBT) void k_key_ip_shared(KeyJobs kj, int n_jobs, const uint64_t *key, uint64_t *u_base,
                                                      int accumulate, int n_digits, int level, int L, int alpha,
                                                      int nq, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN;
    const int t = blockIdx.y;
    const int ne = level + 1 + alpha, nk = L + 1 + alpha;
    const int pidx = t <= level ? t : nq + (t - level - 1);
    const int kl = t <= level ? t : L + 1 + (t - level - 1);
    const int own = t <= level ? t / alpha : -1;
    const Mod m = info[pidx].m;
    const int k = blockIdx.x * kBT + threadIdx.x;
    if (k >= N) return;
    double kb[8], ka[8];  // dnum <= 8 digits per level on this path
#pragma unroll
    for (int j = 0; j < 8; j++) {
        if (j < n_digits) {
            kb[j] = u2d(key[(((size_t)j * 2 + 0) * nk + kl) * N + k]);
            ka[j] = u2d(key[(((size_t)j * 2 + 1) * nk + kl) * N + k]);
        }
    }
    for (int z = 0; z < n_jobs; z++) {
        const uint32_t g = kj.g[z];
        const int src = g == 1u ? k : galois_src2(k, g, logN);
        const uint64_t *ext = kj.ext[z], *d = kj.d[z];
        uint64_t *u = u_base + (size_t)z * 2 * ne * N;
        const size_t o0 = (size_t)t * N + k, o1 = ((size_t)ne + t) * N + k;
        // with accumulate, the running sum counts as one of the (<= 8) lazy terms
        double acc0 = accumulate ? u2d(u[o0]) : 0.0, acc1 = accumulate ? u2d(u[o1]) : 0.0;
#pragma unroll
        for (int j = 0; j < 7; j++) {
            if (j < n_digits) {
                const uint64_t *xp = j == own ? d + (size_t)t * N : ext + ((size_t)j * ne + t) * N;
                double x = u2d(xp[src]);
                acc0 += mul_lazy(x, kb[j], m);
                acc1 += mul_lazy(x, ka[j], m);
            }
        }
        if (n_digits == 8) {
            const uint64_t *xp = own == 7 ? d + (size_t)t * N : ext + ((size_t)7 * ne + t) * N;
            double x = u2d(xp[src]);
            acc0 = reduce(acc0, m) + mul_lazy(x, kb[7], m);
            acc1 = reduce(acc1, m) + mul_lazy(x, ka[7], m);
        }
        u[o0] = d2u(reduce(acc0, m));
        u[o1] = d2u(reduce(acc1, m));
    }
}

hipError_t launch_key_ip_shared(const nj_ctx *c, int level, const KeyJobs &kj, int n_jobs, const uint64_t *key,
                                uint64_t *u_base, hipStream_t s, int accumulate)
{
    const int nd = n_digits(c, level), ne = level + 1 + c->alpha;
    if (nd > 8) return hipErrorInvalidValue;
    dim3 grid((c->N + kBT - 1) / kBT, ne);
    return launch(c, PROF_KEYIP, 8.0 * c->N * ne * (2.0 * nd + n_jobs * (nd + 2.0 + 2.0 * accumulate)),
                  k_key_ip_shared, grid, dim3(kBT), s, kj, n_jobs, key, u_base, accumulate, nd, level, c->L, c->alpha,
                  c->n_q, c->d_info, c->log_n);
}

// c0 parts of the lazy giant steps: out (+)= tau_{g_z}(in_z) over l+1 limbs, per job
// (mode 0 / 1, out_z at out + z ostride) or summed over the jobs into out (mode 2 / 3)
__global__ __launch_bounds__(kBT) void k_automorph_acc(AutoJobs aj, int n_jobs, uint64_t *out, size_t ostride,
                                                      int mode, const PrimeInfo *info, int logN, int skip)
{
    const int N = 1 << logN, i = blockIdx.y == 0 ? 0 : (int)blockIdx.y + skip;
    const int k = blockIdx.x * kBT + threadIdx.x;
    if (k >= N) return;
    const Mod m = info[i].m;
    const size_t o = (size_t)i * N;
    if (mode < 2) {
        const int z = blockIdx.z;
        const int src = aj.g[z] <= 1u ? k : galois_src2(k, aj.g[z], logN);
        double v = u2d(aj.in[z][o + src]);
        if (mode == 1) v = add_mod(v, u2d(out[z * ostride + o + k]), m);
        out[z * ostride + o + k] = d2u(v);
        return;
    }
    double v = mode == 3 ? u2d(out[o + k]) : 0.0;
    for (int z = 0; z < n_jobs; z++) {
        const int src = aj.g[z] <= 1u ? k : galois_src2(k, aj.g[z], logN);
        v = add_mod(v, u2d(aj.in[z][o + src]), m);
    }
    out[o + k] = d2u(v);
}

hipError_t launch_automorph_acc(const nj_ctx *c, const AutoJobs &aj, int n_jobs, int n_limbs, uint64_t *out,
                                size_t ostride, int mode, hipStream_t s, int skip)
{
    if (skip < 0 || skip > std::max(0, n_limbs - 2)) return hipErrorInvalidValue;
    n_limbs -= skip;  // limb 0, then limbs 1 + skip ..
    dim3 grid((c->N + kBT - 1) / kBT, n_limbs, mode < 2 ? n_jobs : 1);
    const double words = (double)n_limbs * c->N * (mode < 2 ? n_jobs * (mode ? 3.0 : 2.0) : n_jobs + (mode == 3 ? 2.0 : 1.0));
    return launch(c, PROF_OTHER, 8.0 * words, k_automorph_acc, grid, dim3(kBT), s, aj, n_jobs, out, ostride, mode,
                  c->d_info, c->log_n, skip);
}

// Mixed-level form of k_key_ip_shared: grid row t is Q limb t for t <= lmax, special
// prime t - lmax - 1 after; job z skips Q limbs above its level l_z, and its limb index
// inside its own [l_z+1+alpha] layout is t (Q) or l_z+1+a (special prime a).
__global__ __launch_bounds__(kBT) void k_key_ip_mixed(KeyJobsX kj, int n_jobs, const uint64_t *key, int lmax,
                                                     int ndmax, int L, int alpha, int nq, const PrimeInfo *info,
                                                     int logN)
{
    const int N = 1 << logN;
    const int t = blockIdx.y;
    const bool isq = t <= lmax;
    const int a = t - lmax - 1;
    const int pidx = isq ? t : nq + a;
    const int kl = isq ? t : L + 1 + a;
    const int own = isq ? t / alpha : -1;
    const int nk = L + 1 + alpha;
    const Mod m = info[pidx].m;
    const int k = blockIdx.x * kBT + threadIdx.x;
    if (k >= N) return;
    double kb[8], ka[8];  // dnum <= 8 digits per level on this path
#pragma unroll
    for (int j = 0; j < 8; j++) {
        if (j < ndmax) {
            kb[j] = u2d(key[(((size_t)j * 2 + 0) * nk + kl) * N + k]);
            ka[j] = u2d(key[(((size_t)j * 2 + 1) * nk + kl) * N + k]);
        }
    }
    for (int z = 0; z < n_jobs; z++) {
        const int lz = kj.lv[z];
        if (isq && t > lz) continue;
        const int ne = lz + 1 + alpha, loc = isq ? t : lz + 1 + a, nd = (lz + alpha) / alpha;
        const uint32_t g = kj.g[z];
        const int src = g == 1u ? k : galois_src2(k, g, logN);
        const uint64_t *ext = kj.ext[z], *d = kj.d[z];
        double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            if (j < nd) {
                const uint64_t *xp = j == own ? d + (size_t)loc * N : ext + ((size_t)j * ne + loc) * N;
                double x = u2d(xp[src]);
                acc0 += mul_lazy(x, kb[j], m);
                acc1 += mul_lazy(x, ka[j], m);
            }
        }
        uint64_t *u = kj.u[z];
        u[(size_t)loc * N + k] = d2u(reduce(acc0, m));
        u[((size_t)ne + loc) * N + k] = d2u(reduce(acc1, m));
    }
}

hipError_t launch_key_ip_mixed(const nj_ctx *c, const KeyJobsX &kj, int n_jobs, const uint64_t *key, hipStream_t s)
{
    int lmax = 0;
    double words = 0.0;
    for (int z = 0; z < n_jobs; z++) {
        lmax = std::max(lmax, kj.lv[z]);
        const int ne = kj.lv[z] + 1 + c->alpha;
        words += (double)ne * (n_digits(c, kj.lv[z]) + 2.0);
    }
    const int ndmax = n_digits(c, lmax), ne = lmax + 1 + c->alpha;
    if (ndmax > 8) return hipErrorInvalidValue;
    dim3 grid((c->N + kBT - 1) / kBT, ne);
    return launch(c, PROF_KEYIP, 8.0 * c->N * (2.0 * ndmax * ne + words), k_key_ip_mixed, grid, dim3(kBT), s, kj,
                  n_jobs, key, lmax, ndmax, c->L, c->alpha, c->n_q, c->d_info, c->log_n);
}

// BSGS multiply-accumulate for many ciphertexts sharing one transform: blockIdx.z =
// chunk of up to 4 giant steps whose diagonal words (<= 4 x 16) stay in registers
// while the ciphertexts' baby steps stream past.  Ciphertext z's baby b is at
// mp.baby[b] + z * bstride, its inner sums at inner + z * istride (giant-major).
template <int GCH, int NBM>
__global__ __launch_bounds__(kBT) void k_bsgs_mac_multi(MacPlan mp, int n_ct, size_t bstride, size_t istride,
                                                       const uint64_t *diag, uint64_t *inner, int level,
                                                       const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, i = blockIdx.y;
    const int k = blockIdx.x * kBT + threadIdx.x;
    if (k >= N) return;
    const Mod m = info[i].m;
    const size_t L1 = level + 1;
    const int g0 = blockIdx.z * GCH;
    const size_t o = (size_t)i * N + k;
    double w[GCH][NBM];
    bool any[GCH];
#pragma unroll
    for (int gg = 0; gg < GCH; gg++) {
        any[gg] = g0 + gg < mp.ng && load_giant<NBM>(mp, g0 + gg, diag, (size_t)mp.dl * N, o, w[gg]);
        if (!any[gg])
#pragma unroll
            for (int b = 0; b < NBM; b++) w[gg][b] = 0.0;
    }
    for (int z = 0; z < n_ct; z++) {
        double b0[NBM], b1[NBM];
        load_babies<NBM>(mp, (size_t)z * bstride, o, L1 * N + o, b0, b1);
        uint64_t *oz = inner + (size_t)z * istride + o;
#pragma unroll
        for (int gg = 0; gg < GCH; gg++) {
            const int g = g0 + gg;
            if (g >= mp.ng) break;
            oz[(size_t)g * 2 * L1 * N] = any[gg] ? d2u(mac_row<NBM>(0.0, b0, w[gg], m)) : 0;
            oz[(size_t)(g * 2 + 1) * L1 * N] = any[gg] ? d2u(mac_row<NBM>(0.0, b1, w[gg], m)) : 0;
        }
    }
}

hipError_t launch_bsgs_mac_multi(const nj_ctx *c, int level, const MacPlan &mp, int n_ct, size_t bstride,
                                 size_t istride, const uint64_t *diag, uint64_t *inner, int n_diag, hipStream_t s)
{
    const double bytes = 8.0 * c->N * (level + 1) * (n_diag + n_ct * (2.0 * mp.nb + 2.0 * mp.ng));
    if (mp.nb <= 8) {
        dim3 grid((c->N + kBT - 1) / kBT, level + 1, (mp.ng + 7) / 8);
        return launch(c, PROF_PMAC, bytes, k_bsgs_mac_multi<8, 8>, grid, dim3(kBT), s, mp, n_ct, bstride, istride,
                      diag, inner, level, c->d_info, c->log_n);
    }
    dim3 grid((c->N + kBT - 1) / kBT, level + 1, (mp.ng + 3) / 4);
    return launch(c, PROF_PMAC, bytes, k_bsgs_mac_multi<4, 16>, grid, dim3(kBT), s, mp, n_ct, bstride, istride, diag,
                  inner, level, c->d_info, c->log_n);
}

// out[z] = in[z] read through X -> X^g[z], l+1 limbs per job (blockIdx.z = job)
__global__ __launch_bounds__(kBT) void k_automorph_multi(AutoJobs aj, int n_limbs, int logN)
{
    const int N = 1 << logN, z = blockIdx.z, i = blockIdx.y;
    const int k = blockIdx.x * kBT + threadIdx.x;
    if (k >= N) return;
    aj.out[z][(size_t)i * N + k] = aj.in[z][(size_t)i * N + galois_src2(k, aj.g[z], logN)];
}

hipError_t launch_automorph_multi(const nj_ctx *c, const AutoJobs &aj, int n_jobs, int n_limbs, hipStream_t s)
{
    dim3 grid((c->N + kBT - 1) / kBT, n_limbs, n_jobs);
    return launch(c, PROF_OTHER, 16.0 * c->N * n_limbs * n_jobs, k_automorph_multi, grid, dim3(kBT), s, aj, n_limbs,
                  c->log_n);
}

hipError_t launch_bsgs_mac(const nj_ctx *c, int level, const MacPlan &mp, const uint64_t *diag, uint64_t *inner,
                           int n_diag, hipStream_t s, int accumulate)
{
    if (mp.nb < 1 || mp.nb > NJ_MAX_BABY || mp.ng < 0 || mp.ng > NJ_MAX_GIANT) return hipErrorInvalidValue;
    dim3 grid((c->N + kBT - 1) / kBT, level + 1);
    const double bytes = 8.0 * c->N * (level + 1) * (2.0 * mp.nb + n_diag + (2.0 + 2 * accumulate) * mp.ng);
    if (mp.nb <= 4)
        return launch(c, PROF_PMAC, bytes, k_bsgs_mac<4>, grid, dim3(kBT), s, mp, diag, inner, level, accumulate,
                      c->d_info, c->log_n);
    if (mp.nb <= 8)
        return launch(c, PROF_PMAC, bytes, k_bsgs_mac<8>, grid, dim3(kBT), s, mp, diag, inner, level, accumulate,
                      c->d_info, c->log_n);
    return launch(c, PROF_PMAC, bytes, k_bsgs_mac<16>, grid, dim3(kBT), s, mp, diag, inner, level, accumulate,
                  c->d_info, c->log_n);
}

}  // namespace nj
