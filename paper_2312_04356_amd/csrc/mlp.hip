// Learned cost model for plan selection: a 7 -> 64 -> 64 -> 1 FP32 MLP with ReLU that
// predicts the (standardised) log latency of a BSGS transform from its structure.
// Training runs on the GPU: one wavefront per chunk of samples computes forward and
// backward passes with parameters in LDS and gradients in registers, per-chunk partial
// gradients are reduced in a fixed order (deterministic) and applied with Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

using nj::fail;

namespace {

constexpr int F = NJ_MLP_FEATURES, H = NJ_MLP_HIDDEN;
// parameter layout: W1 [F][H], b1 [H], W2 [H][H] (row = input unit), b2 [H], w3 [H], b3
constexpr int OW1 = 0, OB1 = OW1 + F * H, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;
constexpr int P = OB3 + 1;
static_assert(P == NJ_MLP_PARAMS, "parameter count");
constexpr int kChunk = 64;  // samples per wavefront

__device__ __forceinline__ float wave_sum(float v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Thread j of the wavefront owns hidden unit j of both layers.  Forward (and, when
// `grad` is set, backward) over samples [blockIdx.x * kChunk, +kChunk) of X [n][F];
// partial gradients of mean((out - y)^2) go to grad + blockIdx.x * P, the chunk's
// summed squared error to sse[blockIdx.x]; predictions to pred when non-null.
__global__ __launch_bounds__(64) void k_mlp_chunk(const float *params, const float *X, const float *y, int n,
                                                  float inv_n, float *grad, float *sse, float *pred)
{
    __shared__ float sW2[H][H + 1];
    __shared__ float sh1[H], sdh2[H];
    const int j = threadIdx.x;
    for (int i = 0; i < H; i++) sW2[i][j] = params[OW2 + i * H + j];
    float w1[F];
#pragma unroll
    for (int k = 0; k < F; k++) w1[k] = params[OW1 + k * H + j];
    const float b1 = params[OB1 + j], b2 = params[OB2 + j], w3 = params[OW3 + j], b3 = params[OB3];
    float gW1[F] = {}, gW2[H] = {};  // gW2[i] = dL/dW2[i][j]
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, err2 = 0.f;
    __syncthreads();
    const int s0 = blockIdx.x * kChunk, s1 = min(n, s0 + kChunk);
    for (int smp = s0; smp < s1; smp++) {
        float x[F];
#pragma unroll
        for (int k = 0; k < F; k++) x[k] = X[(size_t)smp * F + k];
        float a1 = b1;
#pragma unroll
        for (int k = 0; k < F; k++) a1 += w1[k] * x[k];
        const float h1 = a1 > 0.f ? a1 : 0.f;
        sh1[j] = h1;
        __syncthreads();
        float a2 = b2;
#pragma unroll 8
        for (int i = 0; i < H; i++) a2 += sW2[i][j] * sh1[i];
        const float h2 = a2 > 0.f ? a2 : 0.f;
        const float out = wave_sum(w3 * h2) + b3;
        if (pred && j == 0) pred[smp] = out;
        if (grad) {
            const float e = out - y[smp];
            err2 += e * e;
            const float dout = 2.f * e * inv_n;
            gw3 += dout * h2;
            gb3 += dout;
            const float dh2 = a2 > 0.f ? dout * w3 : 0.f;
            gb2 += dh2;
#pragma unroll 8
            for (int i = 0; i < H; i++) gW2[i] += sh1[i] * dh2;
            sdh2[j] = dh2;
            __syncthreads();
            float dh1 = 0.f;
#pragma unroll 8
            for (int q = 0; q < H; q++) dh1 += sW2[j][q] * sdh2[q];
            dh1 = a1 > 0.f ? dh1 : 0.f;
            gb1 += dh1;
#pragma unroll
            for (int k = 0; k < F; k++) gW1[k] += x[k] * dh1;
        }
        __syncthreads();
    }
    if (!grad) return;
    float *g = grad + (size_t)blockIdx.x * P;
#pragma unroll
    for (int k = 0; k < F; k++) g[OW1 + k * H + j] = gW1[k];
    g[OB1 + j] = gb1;
    for (int i = 0; i < H; i++) g[OW2 + i * H + j] = gW2[i];
    g[OB2 + j] = gb2;
    g[OW3 + j] = gw3;
    if (j == 0) {
        g[OB3] = gb3;
        sse[blockIdx.x] = err2;
    }
}

// gradient = sum of the chunks' partials (fixed order); Adam step when lr > 0, else the
// gradient is written to out_grad
__global__ void k_mlp_adam(const float *partial, int n_chunks, float *params, float *m, float *v, float lr, float b1,
                           float b2, float eps, float c1, float c2, float *out_grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float g = 0.f;
    for (int c = 0; c < n_chunks; c++) g += partial[(size_t)c * P + p];
    if (out_grad) out_grad[p] = g;
    if (lr <= 0.f) return;
    const float mm = b1 * m[p] + (1.f - b1) * g, vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm, v[p] = vv;
    params[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double unit(uint64_t &s) { return (double)(splitmix(s) >> 11) * 0x1.0p-53; }

}  // namespace

struct nj_mlp {
    float *d_params = nullptr, *d_m = nullptr, *d_v = nullptr;
    float mean[F], stdv[F], y_mean = 0.f, y_std = 1.f;
    int step = 0;
};

namespace {

nj_status run_chunks(nj_mlp *m, const float *dX, const float *dy, int n, float *dgrad, float *dsse, float *dpred,
                     hipStream_t s)
{
    const int chunks = (n + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_mlp_chunk, dim3(chunks), dim3(64), 0, s, m->d_params, dX, dy, n, 1.f / (float)n, dgrad,
                       dsse, dpred);
    NJ_HIP(hipGetLastError());
    return NJ_OK;
}

std::vector<float> standardise(const nj_mlp *m, const float *X, int n)
{
    std::vector<float> Z((size_t)n * F);
    for (int i = 0; i < n; i++)
        for (int k = 0; k < F; k++) Z[(size_t)i * F + k] = (X[(size_t)i * F + k] - m->mean[k]) / m->stdv[k];
    return Z;
}

template <class T>
struct DevBuf {
    T *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t n) { return hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)); }
};

}  // namespace

extern "C" {

nj_status nj_mlp_create(uint64_t seed, nj_mlp **out)
{
    if (!out) return fail(NJ_EINVAL, "nj_mlp_create: null output");
    nj_mlp *m = new nj_mlp();
    for (int k = 0; k < F; k++) m->mean[k] = 0.f, m->stdv[k] = 1.f;
    if (hipMalloc(&m->d_params, P * 4) != hipSuccess || hipMalloc(&m->d_m, P * 4) != hipSuccess ||
        hipMalloc(&m->d_v, P * 4) != hipSuccess) {
        nj_mlp_destroy(m);
        return fail(NJ_ENOMEM, "nj_mlp_create: device memory");
    }
    // He-uniform weights (bound sqrt(6 / fan_in)), zero biases, from a seeded splitmix64
    std::vector<float> h(P, 0.f);
    uint64_t s = seed;
    const double a1 = std::sqrt(6.0 / F), a2 = std::sqrt(6.0 / H);
    for (int i = 0; i < F * H; i++) h[OW1 + i] = (float)((2 * unit(s) - 1) * a1);
    for (int i = 0; i < H * H; i++) h[OW2 + i] = (float)((2 * unit(s) - 1) * a2);
    for (int i = 0; i < H; i++) h[OW3 + i] = (float)((2 * unit(s) - 1) * a2);
    if (nj_mlp_set_params(m, h.data())) {
        nj_mlp_destroy(m);
        return NJ_EDEVICE;
    }
    *out = m;
    return NJ_OK;
}

void nj_mlp_destroy(nj_mlp *m)
{
    if (!m) return;
    if (m->d_params) (void)hipFree(m->d_params);
    if (m->d_m) (void)hipFree(m->d_m);
    if (m->d_v) (void)hipFree(m->d_v);
    delete m;
}

nj_status nj_mlp_set_params(nj_mlp *m, const float *params)
{
    if (!m || !params) return fail(NJ_EINVAL, "nj_mlp_set_params: null argument");
    NJ_HIP(hipMemcpy(m->d_params, params, P * 4, hipMemcpyHostToDevice));
    std::vector<float> z(P, 0.f);
    NJ_HIP(hipMemcpy(m->d_m, z.data(), P * 4, hipMemcpyHostToDevice));
    NJ_HIP(hipMemcpy(m->d_v, z.data(), P * 4, hipMemcpyHostToDevice));
    m->step = 0;
    return NJ_OK;
}

nj_status nj_mlp_get_norm(const nj_mlp *m, float *norm)
{
    if (!m || !norm) return fail(NJ_EINVAL, "nj_mlp_get_norm: null argument");
    for (int k = 0; k < F; k++) norm[k] = m->mean[k], norm[F + k] = m->stdv[k];
    norm[2 * F] = m->y_mean, norm[2 * F + 1] = m->y_std;
    return NJ_OK;
}

nj_status nj_mlp_set_norm(nj_mlp *m, const float *norm)
{
    if (!m || !norm) return fail(NJ_EINVAL, "nj_mlp_set_norm: null argument");
    for (int k = 0; k < F; k++)
        if (!(norm[F + k] > 0.f)) return fail(NJ_EINVAL, "nj_mlp_set_norm: feature scales must be positive");
    if (!(norm[2 * F + 1] > 0.f)) return fail(NJ_EINVAL, "nj_mlp_set_norm: target scale must be positive");
    for (int k = 0; k < F; k++) m->mean[k] = norm[k], m->stdv[k] = norm[F + k];
    m->y_mean = norm[2 * F], m->y_std = norm[2 * F + 1];
    return NJ_OK;
}

nj_status nj_mlp_get_params(const nj_mlp *m, float *params)
{
    if (!m || !params) return fail(NJ_EINVAL, "nj_mlp_get_params: null argument");
    NJ_HIP(hipMemcpy(params, m->d_params, P * 4, hipMemcpyDeviceToHost));
    return NJ_OK;
}

nj_status nj_mlp_grad(nj_mlp *m, const float *X, const float *y, int n, float *grad, float *loss)
{
    if (!m || !X || !y || !grad || n < 1) return fail(NJ_EINVAL, "nj_mlp_grad: bad arguments");
    const int chunks = (n + kChunk - 1) / kChunk;
    DevBuf<float> dX, dy, dpart, dsse, dg;
    NJ_HIP(dX.alloc((size_t)n * F));
    NJ_HIP(dy.alloc(n));
    NJ_HIP(dpart.alloc((size_t)chunks * P));
    NJ_HIP(dsse.alloc(chunks));
    NJ_HIP(dg.alloc(P));
    NJ_HIP(hipMemcpy(dX.p, X, (size_t)n * F * 4, hipMemcpyHostToDevice));
    NJ_HIP(hipMemcpy(dy.p, y, (size_t)n * 4, hipMemcpyHostToDevice));
    nj_status st = run_chunks(m, dX.p, dy.p, n, dpart.p, dsse.p, nullptr, 0);
    if (st) return st;
    hipLaunchKernelGGL(k_mlp_adam, dim3((P + 255) / 256), dim3(256), 0, 0, dpart.p, chunks, m->d_params, m->d_m,
                       m->d_v, 0.f, 0.f, 0.f, 0.f, 1.f, 1.f, dg.p);
    NJ_HIP(hipGetLastError());
    NJ_HIP(hipMemcpy(grad, dg.p, P * 4, hipMemcpyDeviceToHost));
    if (loss) {
        std::vector<float> sse(chunks);
        NJ_HIP(hipMemcpy(sse.data(), dsse.p, chunks * 4, hipMemcpyDeviceToHost));
        double t = 0;
        for (float v : sse) t += v;
        *loss = (float)(t / n);
    }
    return NJ_OK;
}

nj_status nj_mlp_train(nj_mlp *m, const float *X, const float *y, int n, int epochs, int batch, float lr,
                       uint64_t seed, float *final_loss)
{
    if (!m || !X || !y || n < 2 || epochs < 1 || batch < 1 || !(lr > 0.f)) return fail(NJ_EINVAL, "nj_mlp_train: bad arguments");
    // feature and target standardisation from the training set
    for (int k = 0; k < F; k++) {
        double s = 0, s2 = 0;
        for (int i = 0; i < n; i++) s += X[(size_t)i * F + k], s2 += (double)X[(size_t)i * F + k] * X[(size_t)i * F + k];
        const double mu = s / n, var = std::max(s2 / n - mu * mu, 0.0);
        m->mean[k] = (float)mu, m->stdv[k] = var > 1e-12 ? (float)std::sqrt(var) : 1.f;
    }
    double s = 0, s2 = 0;
    for (int i = 0; i < n; i++) s += y[i], s2 += (double)y[i] * y[i];
    m->y_mean = (float)(s / n);
    m->y_std = (float)std::max(std::sqrt(std::max(s2 / n - (s / n) * (s / n), 0.0)), 1e-6);
    std::vector<float> Z = standardise(m, X, n), t(n);
    for (int i = 0; i < n; i++) t[i] = (y[i] - m->y_mean) / m->y_std;
    const int bmax = std::min(batch, n), chunks = (bmax + kChunk - 1) / kChunk;
    DevBuf<float> dX, dy, dpart, dsse;
    NJ_HIP(dX.alloc((size_t)n * F));
    NJ_HIP(dy.alloc(n));
    NJ_HIP(dpart.alloc((size_t)chunks * P));
    NJ_HIP(dsse.alloc(chunks));
    std::vector<int> perm(n);
    std::vector<float> Zp((size_t)n * F), tp(n);
    uint64_t rs = seed;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int ep = 0; ep < epochs; ep++) {
        for (int i = 0; i < n; i++) perm[i] = i;
        for (int i = n - 1; i > 0; i--) std::swap(perm[i], perm[splitmix(rs) % (uint64_t)(i + 1)]);
        for (int i = 0; i < n; i++) {
            std::memcpy(&Zp[(size_t)i * F], &Z[(size_t)perm[i] * F], F * 4);
            tp[i] = t[perm[i]];
        }
        NJ_HIP(hipMemcpy(dX.p, Zp.data(), (size_t)n * F * 4, hipMemcpyHostToDevice));
        NJ_HIP(hipMemcpy(dy.p, tp.data(), (size_t)n * 4, hipMemcpyHostToDevice));
        for (int b0 = 0; b0 + 1 < n; b0 += bmax) {
            const int nb = std::min(bmax, n - b0);
            nj_status st = run_chunks(m, dX.p + (size_t)b0 * F, dy.p + b0, nb, dpart.p, dsse.p, nullptr, 0);
            if (st) return st;
            m->step++;
            const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
            hipLaunchKernelGGL(k_mlp_adam, dim3((P + 255) / 256), dim3(256), 0, 0, dpart.p, (nb + kChunk - 1) / kChunk,
                               m->d_params, m->d_m, m->d_v, lr, b1, b2, eps, c1, c2, (float *)nullptr);
            NJ_HIP(hipGetLastError());
        }
    }
    if (final_loss) {  // mean squared error over the whole set, standardised target units
        std::vector<float> pred(n);
        DevBuf<float> dp;
        NJ_HIP(dp.alloc(n));
        NJ_HIP(hipMemcpy(dX.p, Z.data(), (size_t)n * F * 4, hipMemcpyHostToDevice));
        nj_status st = run_chunks(m, dX.p, nullptr, n, nullptr, nullptr, dp.p, 0);
        if (st) return st;
        NJ_HIP(hipMemcpy(pred.data(), dp.p, (size_t)n * 4, hipMemcpyDeviceToHost));
        double e = 0;
        for (int i = 0; i < n; i++) e += (double)(pred[i] - t[i]) * (pred[i] - t[i]);
        *final_loss = (float)(e / n);
    }
    return NJ_OK;
}

nj_status nj_mlp_predict(nj_mlp *m, const float *X, int n, float *out)
{
    if (!m || !X || !out || n < 1) return fail(NJ_EINVAL, "nj_mlp_predict: bad arguments");
    std::vector<float> Z = standardise(m, X, n);
    DevBuf<float> dX, dp;
    NJ_HIP(dX.alloc((size_t)n * F));
    NJ_HIP(dp.alloc(n));
    NJ_HIP(hipMemcpy(dX.p, Z.data(), (size_t)n * F * 4, hipMemcpyHostToDevice));
    nj_status st = run_chunks(m, dX.p, nullptr, n, nullptr, nullptr, dp.p, 0);
    if (st) return st;
    NJ_HIP(hipMemcpy(out, dp.p, (size_t)n * 4, hipMemcpyDeviceToHost));
    for (int i = 0; i < n; i++) out[i] = out[i] * m->y_std + m->y_mean;
    return NJ_OK;
}

}  // extern "C"
