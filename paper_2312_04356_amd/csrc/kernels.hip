// HIP kernels (gfx950) of the RNS-CKKS hot path and their host launchers.
//
// Layout: every polynomial limb is N contiguous uint64 residues; a LimbTab lists,
// per launched limb, the prime it is taken modulo and its offset (in units of N)
// from the base pointer.  Evaluation form = output of the negacyclic forward
// transform below: word k holds a(psi^(2 rev(k) + 1)) with rev the log2(N)-bit
// reversal and psi the context's primitive 2N-th root of the limb's prime.
#include "internal.h"

namespace nj {

constexpr int kThreads = 256;
constexpr int kTile = 4096;  // elements staged in LDS by one NTT workgroup (32 KiB as FP64)

__device__ __forceinline__ uint32_t bitrev(uint32_t x, int bits) { return __brev(x) >> (32 - bits); }

// ------------------------------------------------------------------ NTT
//
// Forward: Cooley-Tukey stages m = 1, 2, ..., N/2 (stride t = N/2m), twiddle
// psi^rev(m+i) for butterfly block i; inverse: Gentleman-Sande stages in the
// reverse order with psi^-rev(h+i), then a factor N^-1.  N = N1 * T with
// T = min(N, 4096): the first log2(N1) stages only couple words with the same
// index mod T ("columns", pass A); the remaining ones stay inside contiguous
// T-word blocks (pass B).  Each pass stages a 4096-word tile in LDS.

template <bool INV>
__global__ __launch_bounds__(kThreads) void k_ntt_cols(uint64_t *data, LimbTab lt, const double *tw,
                                                       const double *twq, const PrimeInfo *info, int logN)
{
    __shared__ double s[kTile];
    const int N = 1 << logN, N1 = N >> 12, TC = kTile / N1;
    const int limb = blockIdx.y, pidx = lt.pidx[limb];
    const Mod m = info[pidx].m;
    uint64_t *a = data + (size_t)lt.off[limb] * N;
    const double *W = tw + (size_t)pidx * N, *Wq = twq + (size_t)pidx * N;
    const int col0 = blockIdx.x * TC;
    for (int e = threadIdx.x; e < kTile; e += kThreads) {
        int c = e % TC, r = e / TC;
        s[e] = u2d(a[(size_t)r * kTile + col0 + c]);
    }
    __syncthreads();
    if (!INV) {
        for (int mm = 1; mm < N1; mm <<= 1) {
            const int tr = N1 / (2 * mm);
            for (int b = threadIdx.x; b < kTile / 2; b += kThreads) {
                int c = b % TC, p = b / TC, i = p / tr, j = p % tr;
                int r1 = 2 * i * tr + j, r2 = r1 + tr;
                double U = s[r1 * TC + c];
                double V = mul_shoup(s[r2 * TC + c], W[mm + i], Wq[mm + i], m);
                s[r1 * TC + c] = add_mod(U, V, m);
                s[r2 * TC + c] = sub_mod(U, V, m);
            }
            __syncthreads();
        }
    } else {
        for (int h = N1 / 2; h >= 1; h >>= 1) {
            const int tr = N1 / (2 * h);
            for (int b = threadIdx.x; b < kTile / 2; b += kThreads) {
                int c = b % TC, p = b / TC, i = p / tr, j = p % tr;
                int r1 = 2 * i * tr + j, r2 = r1 + tr;
                double U = s[r1 * TC + c], V = s[r2 * TC + c];
                s[r1 * TC + c] = add_mod(U, V, m);
                s[r2 * TC + c] = mul_shoup(sub_mod(U, V, m), W[h + i], Wq[h + i], m);
            }
            __syncthreads();
        }
        const double ni = info[pidx].ninv, niq = info[pidx].ninvq;
        for (int e = threadIdx.x; e < kTile; e += kThreads) s[e] = mul_shoup(s[e], ni, niq, m);
        __syncthreads();
    }
    for (int e = threadIdx.x; e < kTile; e += kThreads) {
        int c = e % TC, r = e / TC;
        a[(size_t)r * kTile + col0 + c] = d2u(s[e]);
    }
}

template <bool INV>
__global__ __launch_bounds__(kThreads) void k_ntt_rows(uint64_t *data, LimbTab lt, const double *tw,
                                                       const double *twq, const PrimeInfo *info, int logN)
{
    __shared__ double s[kTile];
    const int N = 1 << logN, T = N < kTile ? N : kTile, N1 = N / T;
    const int limb = blockIdx.y, pidx = lt.pidx[limb];
    const Mod m = info[pidx].m;
    const int b = blockIdx.x;  // tile index within the limb
    uint64_t *a = data + (size_t)lt.off[limb] * N + (size_t)b * T;
    const double *W = tw + (size_t)pidx * N, *Wq = twq + (size_t)pidx * N;
    for (int e = threadIdx.x; e < T; e += kThreads) s[e] = u2d(a[e]);
    __syncthreads();
    if (!INV) {
        for (int mm = N1; mm < N; mm <<= 1) {
            const int t = N / (2 * mm);
            for (int p = threadIdx.x; p < T / 2; p += kThreads) {
                int i = p / t, j = p % t, x1 = 2 * i * t + j, x2 = x1 + t;
                int wi = mm + b * (mm / N1) + i;
                double U = s[x1], V = mul_shoup(s[x2], W[wi], Wq[wi], m);
                s[x1] = add_mod(U, V, m);
                s[x2] = sub_mod(U, V, m);
            }
            __syncthreads();
        }
    } else {
        for (int h = N / 2; h >= N1; h >>= 1) {
            const int t = N / (2 * h);
            for (int p = threadIdx.x; p < T / 2; p += kThreads) {
                int i = p / t, j = p % t, x1 = 2 * i * t + j, x2 = x1 + t;
                int wi = h + b * (h / N1) + i;
                double U = s[x1], V = s[x2];
                s[x1] = add_mod(U, V, m);
                s[x2] = mul_shoup(sub_mod(U, V, m), W[wi], Wq[wi], m);
            }
            __syncthreads();
        }
        if (N1 == 1) {
            const double ni = info[pidx].ninv, niq = info[pidx].ninvq;
            for (int e = threadIdx.x; e < T; e += kThreads) s[e] = mul_shoup(s[e], ni, niq, m);
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < T; e += kThreads) a[e] = d2u(s[e]);
}

hipError_t launch_ntt(const nj_ctx *c, uint64_t *data, const LimbTab &lt, bool inverse, hipStream_t s,
                      const uint64_t *src)
{
    if (lt.n == 0) return hipSuccess;
    if (c->N >= kTile) return launch_ntt_fast(c, data, src, lt, inverse, s);
    if (src) {  // generic kernels work in place
        for (int i = 0; i < lt.n; i++) {
            hipError_t e = hipMemcpyAsync(data + (size_t)lt.off[i] * c->N, src + (size_t)lt.soff[i] * c->N,
                                          (size_t)c->N * 8, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
        }
    }
    const int N = c->N, T = N < kTile ? N : kTile, N1 = N / T;
    dim3 grid(N1, lt.n);
    if (!inverse) {
        if (N1 > 1)
            hipLaunchKernelGGL(k_ntt_cols<false>, grid, dim3(kThreads), 0, s, data, lt, c->d_tw, c->d_twq, c->d_info,
                               c->log_n);
        hipLaunchKernelGGL(k_ntt_rows<false>, grid, dim3(kThreads), 0, s, data, lt, c->d_tw, c->d_twq, c->d_info,
                           c->log_n);
    } else {
        hipLaunchKernelGGL(k_ntt_rows<true>, grid, dim3(kThreads), 0, s, data, lt, c->d_itw, c->d_itwq, c->d_info,
                           c->log_n);
        if (N1 > 1)
            hipLaunchKernelGGL(k_ntt_cols<true>, grid, dim3(kThreads), 0, s, data, lt, c->d_itw, c->d_itwq, c->d_info,
                               c->log_n);
    }
    return hipGetLastError();
}

// --------------------------------------------------------- elementwise ops

__global__ void k_elementwise(int op, const uint64_t *a, const uint64_t *b, uint64_t *out, LimbTab lt,
                              const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, limb = blockIdx.y;
    const Mod m = info[lt.pidx[limb]].m;
    const size_t base = (size_t)lt.off[limb] * N;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
        double x = u2d(a[base + k]), y = u2d(b[base + k]), r;
        if (op == 0) r = add_mod(x, y, m);
        else if (op == 1) r = sub_mod(x, y, m);
        else r = mul_canon(x, y, m);
        out[base + k] = d2u(r);
    }
}

hipError_t launch_elementwise(const nj_ctx *c, int op, const uint64_t *a, const uint64_t *b, uint64_t *out,
                              const LimbTab &lt, hipStream_t s)
{
    if (lt.n == 0) return hipSuccess;
    dim3 grid((c->N + kThreads - 1) / kThreads, lt.n);
    hipLaunchKernelGGL(k_elementwise, grid, dim3(kThreads), 0, s, op, a, b, out, lt, c->d_info, c->log_n);
    return hipGetLastError();
}

// ------------------------------------------------------------ automorphism
//
// In evaluation form X -> X^g permutes words: out[k] = in[k'] where the
// evaluation exponent of k' is g times that of k (mod 2N).

__device__ __forceinline__ int galois_src(int k, uint32_t g, int logN)
{
    const uint32_t N = 1u << logN;
    uint32_t e = 2u * bitrev((uint32_t)k, logN) + 1u;
    uint32_t eg = (uint32_t)(((uint64_t)e * g) & (2u * N - 1u));
    return (int)bitrev((eg - 1u) >> 1, logN);
}

__global__ void k_automorph(const uint64_t *in, uint64_t *out, uint32_t g, int n_limbs, int logN)
{
    const int N = 1 << logN;
    const size_t base = (size_t)blockIdx.y * N;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x)
        out[base + k] = in[base + galois_src(k, g, logN)];
}

hipError_t launch_automorph(const nj_ctx *c, const uint64_t *in, uint64_t *out, uint32_t g, int n_limbs,
                            hipStream_t s)
{
    if (n_limbs == 0) return hipSuccess;
    dim3 grid((c->N + kThreads - 1) / kThreads, n_limbs);
    hipLaunchKernelGGL(k_automorph, grid, dim3(kThreads), 0, s, in, out, g, n_limbs, c->log_n);
    return hipGetLastError();
}

// ------------------------------------------------- rescale / ModRaise lifts
//
// src: one limb (coefficient form) modulo prime src_pidx; for each target limb i
// (prime i, offsets 0..n_out-1) write the centred lift of src reduced mod q_i.

__global__ void k_lift(const uint64_t *src, int src_pidx, int n_out, uint64_t *dst, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, i = blockIdx.y;
    const Mod ms = info[src_pidx].m, mt = info[i].m;
    const double half = info[src_pidx].half;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
        double v = u2d(src[k]);
        double r = v > half ? v - ms.t : v;  // centred, |r| < 2^49
        dst[(size_t)i * N + k] = d2u(reduce(r, mt));
    }
}

hipError_t launch_lift_last(const nj_ctx *c, const uint64_t *src, int src_pidx, int n_out, uint64_t *dst,
                            hipStream_t s)
{
    if (n_out == 0) return hipSuccess;
    dim3 grid((c->N + kThreads - 1) / kThreads, n_out);
    hipLaunchKernelGGL(k_lift, grid, dim3(kThreads), 0, s, src, src_pidx, n_out, dst, c->d_info, c->log_n);
    return hipGetLastError();
}

// out_i = (a_i - lifted_i) * q_l^{-1} mod q_i for i < l  (one polynomial)
__global__ void k_rescale_combine(const uint64_t *a, const uint64_t *lifted, uint64_t *out, int level,
                                  const double *qlinv, const double *qlinvq, int nq, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, i = blockIdx.y;
    const Mod m = info[i].m;
    const double w = qlinv[level * nq + i], wq = qlinvq[level * nq + i];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
        double x = sub_mod(u2d(a[(size_t)i * N + k]), u2d(lifted[(size_t)i * N + k]), m);
        out[(size_t)i * N + k] = d2u(mul_shoup(x, w, wq, m));
    }
}

hipError_t launch_rescale_combine(const nj_ctx *c, int level, const uint64_t *a, const uint64_t *lifted, uint64_t *out,
                                  hipStream_t s, int n_out)
{
    dim3 grid((c->N + kThreads - 1) / kThreads, n_out < 0 ? level : n_out);
    hipLaunchKernelGGL(k_rescale_combine, grid, dim3(kThreads), 0, s, a, lifted, out, level, c->d_qlinv, c->d_qlinvq,
                       c->n_q, c->d_info, c->log_n);
    return hipGetLastError();
}

// ------------------------------------------- plaintext multiply-accumulate
//
// acc[p][i] (+)= ct[p][i] * pt[i] for both polynomials p of a level-l ciphertext.

__global__ void k_pmac(const uint64_t *ct, const uint64_t *pt, uint64_t *acc, int level, int first,
                       const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, row = blockIdx.y, i = row % (level + 1);
    const Mod m = info[i].m;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
        double r = mul_canon(u2d(ct[(size_t)row * N + k]), u2d(pt[(size_t)i * N + k]), m);
        if (!first) r = add_mod(r, u2d(acc[(size_t)row * N + k]), m);
        acc[(size_t)row * N + k] = d2u(r);
    }
}

hipError_t launch_pmac(const nj_ctx *c, int level, const uint64_t *ct, const uint64_t *pt, uint64_t *acc, int first,
                       hipStream_t s)
{
    dim3 grid((c->N + kThreads - 1) / kThreads, 2 * (level + 1));
    ProfScope ps(c, PROF_PMAC, 8.0 * c->N * (level + 1) * (first ? 5.0 : 7.0), s);
    hipLaunchKernelGGL(k_pmac, grid, dim3(kThreads), 0, s, ct, pt, acc, level, first, c->d_info, c->log_n);
    return hipGetLastError();
}

// ----------------------------------------------- multiplication by -X^{N/2}
//
// In evaluation form -X^{N/2} is the word-wise constant -(psi^{N/2})^(2 rev(k)+1),
// i.e. -i_t when rev(k) is even and +i_t when odd, i_t = psi^{N/2} = tw[1].

__global__ void k_monomial_half(const uint64_t *in, uint64_t *out, int level, const double *tw,
                                const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, row = blockIdx.y, i = row % (level + 1);
    const Mod m = info[i].m;
    const double it = tw[(size_t)i * N + 1];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
        double r = mul_canon(u2d(in[(size_t)row * N + k]), it, m);
        if ((bitrev((uint32_t)k, logN) & 1u) == 0u) r = r == 0.0 ? 0.0 : m.t - r;
        out[(size_t)row * N + k] = d2u(r);
    }
}

hipError_t launch_monomial_half(const nj_ctx *c, int level, const uint64_t *in, uint64_t *out, hipStream_t s)
{
    dim3 grid((c->N + kThreads - 1) / kThreads, 2 * (level + 1));
    hipLaunchKernelGGL(k_monomial_half, grid, dim3(kThreads), 0, s, in, out, level, c->d_tw, c->d_info, c->log_n);
    return hipGetLastError();
}

// The real/imaginary split after the conjugation key switch, one pass over both inputs:
// re = x + xc, im = -X^{N/2} (x - xc) (the monomial product as in k_monomial_half).
__global__ void k_conj_split(const uint64_t *x, const uint64_t *xc, uint64_t *re, uint64_t *im, int level,
                             const double *tw, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, row = blockIdx.y, i = row % (level + 1);
    const Mod m = info[i].m;
    const double it = tw[(size_t)i * N + 1];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
        const size_t o = (size_t)row * N + k;
        const double a = u2d(x[o]), b = u2d(xc[o]);
        re[o] = d2u(add_mod(a, b, m));
        double r = mul_canon(sub_mod(a, b, m), it, m);
        if ((bitrev((uint32_t)k, logN) & 1u) == 0u) r = r == 0.0 ? 0.0 : m.t - r;
        im[o] = d2u(r);
    }
}

hipError_t launch_conj_split(const nj_ctx *c, int level, const uint64_t *x, const uint64_t *xc, uint64_t *re,
                             uint64_t *im, hipStream_t s)
{
    dim3 grid((c->N + kThreads - 1) / kThreads, 2 * (level + 1));
    hipLaunchKernelGGL(k_conj_split, grid, dim3(kThreads), 0, s, x, xc, re, im, level, c->d_tw, c->d_info, c->log_n);
    return hipGetLastError();
}

// --------------------------------------------------------- key generation

__global__ void k_signed_to_rns(const int64_t *x, LimbTab lt, uint64_t *out, const uint64_t *primes, int logN)
{
    const int N = 1 << logN, limb = blockIdx.y;
    const int64_t t = (int64_t)primes[lt.pidx[limb]];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
        int64_t r = x[k] % t;
        out[(size_t)lt.off[limb] * N + k] = (uint64_t)(r < 0 ? r + t : r);
    }
}

// b[t] = e[t] - a[t] s[t] + (t in digit j ? (P mod t) sp[t] : 0) over all top-level key limbs
__global__ void k_keygen_combine(uint64_t *b, const uint64_t *a, const uint64_t *e, const uint64_t *s,
                                 const uint64_t *sp, const double *pmod, int digit, int alpha, int L, int nq,
                                 const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, t = blockIdx.y;
    const int pidx = t <= L ? t : nq + (t - L - 1);
    const Mod m = info[pidx].m;
    const bool in_digit = t <= L && t / alpha == digit;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
        const size_t o = (size_t)t * N + k;
        double r = sub_mod(u2d(e[o]), mul_canon(u2d(a[o]), u2d(s[(size_t)pidx * N + k]), m), m);
        if (in_digit) r = add_mod(r, mul_canon(pmod[t], u2d(sp[(size_t)pidx * N + k]), m), m);
        b[o] = d2u(r);
    }
}

hipError_t launch_signed_to_rns(const nj_ctx *c, const int64_t *coeffs, const LimbTab &lt, uint64_t *out,
                                hipStream_t s, const uint64_t *d_primes)
{
    if (lt.n == 0) return hipSuccess;
    dim3 grid((c->N + kThreads - 1) / kThreads, lt.n);
    hipLaunchKernelGGL(k_signed_to_rns, grid, dim3(kThreads), 0, s, coeffs, lt, out, d_primes, c->log_n);
    return hipGetLastError();
}

hipError_t launch_keygen_combine(const nj_ctx *c, int digit, uint64_t *b, const uint64_t *a, const uint64_t *e,
                                 const uint64_t *s_eval, const uint64_t *sp_eval, const double *d_pmod, hipStream_t s)
{
    dim3 grid((c->N + kThreads - 1) / kThreads, c->L + 1 + c->alpha);
    hipLaunchKernelGGL(k_keygen_combine, grid, dim3(kThreads), 0, s, b, a, e, s_eval, sp_eval, d_pmod, digit,
                       c->alpha, c->L, c->n_q, c->d_info, c->log_n);
    return hipGetLastError();
}

}  // namespace nj
