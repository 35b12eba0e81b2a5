// Elementwise kernels of the bootstrapping steps after CoeffToSlot: the ciphertext
// tensor product of HMult, multiplication by an integer constant (per-limb residues),
// and adding a constant to the slots (the constant polynomial in evaluation form is the
// same residue in every word).
#include "internal.h"

namespace nj {

namespace {
constexpr int kT = 256;
}

// d0 = a0 b0, d1 = a0 b1 + a1 b0 into d01 [2][l+1][N]; d2 = a1 b1 into d2 [l+1][N].
// a, b are ciphertexts at levels >= l (second polynomial at +astride / +bstride words).
__global__ __launch_bounds__(kT) void k_tensor(const uint64_t *a, size_t astride, const uint64_t *b, size_t bstride,
                                               uint64_t *d01, uint64_t *d2, int level, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, i = blockIdx.y;
    const int k = blockIdx.x * kT + threadIdx.x;
    if (k >= N) return;
    const Mod m = info[i].m;
    const size_t o = (size_t)i * N + k, L1 = level + 1;
    const double x0 = u2d(a[o]), x1 = u2d(a[astride + o]), y0 = u2d(b[o]), y1 = u2d(b[bstride + o]);
    d01[o] = d2u(mul_canon(x0, y0, m));
    d01[L1 * N + o] = d2u(reduce(mul_lazy(x0, y1, m) + mul_lazy(x1, y0, m), m));
    d2[o] = d2u(mul_canon(x1, y1, m));
}

// out [P][n_limbs][N] (+)= in (limbs 0..n_limbs-1 of polynomial p at +p istride, P =
// gridDim.z) times the integer whose residue mod q_i is kc.v[i]
__global__ __launch_bounds__(kT) void k_mul_int(const uint64_t *in, size_t istride, uint64_t *out, int n_limbs,
                                                LimbConsts kc, int accumulate, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, i = blockIdx.y, p = blockIdx.z;
    const int k = blockIdx.x * kT + threadIdx.x;
    if (k >= N) return;
    const Mod m = info[i].m;
    const double x = u2d(in[p * istride + (size_t)i * N + k]);
    const size_t o = ((size_t)p * n_limbs + i) * N + k;
    double r = mul_canon(x, kc.v[i], m);
    if (accumulate) r = add_mod(r, u2d(out[o]), m);
    out[o] = d2u(r);
}

// limbs 0..n_limbs-1 of poly (in place) += kc.v[i] (mod q_i)
__global__ __launch_bounds__(kT) void k_add_int(uint64_t *poly, LimbConsts kc, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, i = blockIdx.y;
    const int k = blockIdx.x * kT + threadIdx.x;
    if (k >= N) return;
    const Mod m = info[i].m;
    const size_t o = (size_t)i * N + k;
    poly[o] = d2u(add_mod(u2d(poly[o]), kc.v[i], m));
}

__global__ __launch_bounds__(kT) void k_zero(uint64_t *p, size_t words)
{
    const size_t w = (size_t)blockIdx.x * kT + threadIdx.x;
    if (w < words) p[w] = 0;
}

hipError_t launch_tensor(const nj_ctx *c, const uint64_t *a, size_t astride, const uint64_t *b, size_t bstride,
                         uint64_t *d01, uint64_t *d2, int level, hipStream_t s)
{
    dim3 grid((c->N + kT - 1) / kT, level + 1);
    return launch(c, PROF_OTHER, 8.0 * c->N * (level + 1) * 7.0, k_tensor, grid, dim3(kT), s, a, astride, b, bstride,
                  d01, d2, level, c->d_info, c->log_n);
}

hipError_t launch_mul_int(const nj_ctx *c, const uint64_t *in, size_t istride, uint64_t *out, int n_limbs,
                          const LimbConsts &kc, hipStream_t s, int accumulate, int n_polys)
{
    dim3 grid((c->N + kT - 1) / kT, n_limbs, n_polys);
    return launch(c, PROF_OTHER, 8.0 * c->N * n_limbs * (accumulate ? 3.0 : 2.0) * n_polys, k_mul_int, grid, dim3(kT),
                  s, in, istride, out, n_limbs, kc, accumulate, c->d_info, c->log_n);
}

hipError_t launch_add_int(const nj_ctx *c, uint64_t *poly, int n_limbs, const LimbConsts &kc, hipStream_t s)
{
    dim3 grid((c->N + kT - 1) / kT, n_limbs);
    return launch(c, PROF_OTHER, 8.0 * c->N * n_limbs * 2.0, k_add_int, grid, dim3(kT), s, poly, kc, c->d_info,
                  c->log_n);
}

hipError_t launch_zero(const nj_ctx *c, uint64_t *p, size_t words, hipStream_t s)
{
    dim3 grid((unsigned)((words + kT - 1) / kT));
    return launch(c, PROF_OTHER, 8.0 * words, k_zero, grid, dim3(kT), s, p, words);
}

}  // namespace nj
