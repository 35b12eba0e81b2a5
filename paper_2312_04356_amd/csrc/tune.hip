// Latency measurement for plan selection: random-content switching keys and plans
// with the structure of a real transform (the work of a BSGS transform does not depend
// on the values), event-timed runs, and the cost-model features of a transform.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "exec.h"

using namespace nj;
using namespace nj::ex;

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// rows of `row_limbs` limbs: limb t of a row is a residue mod q_t for t < q_limbs and
// mod p_{t - q_limbs} after; word = hash(seed, row, t, k) mod prime
__global__ void k_fill_random(uint64_t *dst, int row_limbs, int q_limbs, int nq, const uint64_t *primes, uint64_t seed,
                              int logN)
{
    const int N = 1 << logN, t = blockIdx.y, row = blockIdx.z;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const uint64_t q = primes[t < q_limbs ? t : nq + (t - q_limbs)];
    const size_t w = ((size_t)row * row_limbs + t) * N + k;
    dst[w] = mix64(seed * 0x9E3779B97F4A7C15ull + w) % q;
}

hipError_t fill_random(const nj_ctx *c, uint64_t *dst, int rows, int row_limbs, int q_limbs, uint64_t seed,
                       hipStream_t s)
{
    if (rows < 1) return hipSuccess;
    dim3 grid((c->N + 255) / 256, row_limbs, rows);
    hipLaunchKernelGGL(k_fill_random, grid, dim3(256), 0, s, dst, row_limbs, q_limbs, c->n_q, c->d_primes, seed,
                       c->log_n);
    return hipGetLastError();
}

int ilog2(int x)
{
    int r = 0;
    while ((1 << (r + 1)) <= x) r++;
    return r;
}

}  // namespace

extern "C" {

nj_status nj_timing_keys(nj_ctx *c, int pool)
{
    if (!c || pool < 0 || pool > 256) return fail(NJ_EINVAL, "nj_timing_keys: pool must be 0..256");
    NJ_HIP(hipDeviceSynchronize());
    for (auto *k : c->timing_keys) (void)hipFree(k);
    c->timing_keys.clear();
    const int nk = c->L + 1 + c->alpha;
    const size_t words = (size_t)c->dnum * 2 * nk * c->N;
    for (int i = 0; i < pool; i++) {
        uint64_t *k = nullptr;
        if (hipMalloc(&k, words * 8) != hipSuccess) {
            nj_timing_keys(c, 0);
            return fail(NJ_ENOMEM, "nj_timing_keys: device memory");
        }
        c->timing_keys.push_back(k);
        NJ_HIP(fill_random(c, k, c->dnum * 2, nk, c->L + 1, 0x5EED0000ull + i, 0));
    }
    NJ_HIP(hipDeviceSynchronize());
    return NJ_OK;
}

nj_status nj_plan_create_random(nj_ctx *c, int level, int u, const int32_t *offsets, int n_off, int n1, int bi, int bo,
                                uint64_t seed, nj_plan **out)
{
    if (!c || !offsets || n_off < 1 || !out || u < 1 || n1 < 0 || bi < 1 || bo < 1 || (c->N / 2) % u)
        return fail(NJ_EINVAL, "nj_plan_create_random: bad arguments");
    if (level < 1 || level > c->L) return fail(NJ_ELEVEL, "nj_plan_create_random: need 1 <= level <= L");
    const int n = c->N / 2, m = n / u;
    nj_plan *p = new nj_plan();
    p->kind = 0;
    p->N = c->N;
    p->lts.resize(1);
    nj_lt_t &lt = p->lts[0];
    lt.level = level, lt.u = u, lt.n1 = n1, lt.bi = bi, lt.bo = bo;
    std::vector<int> js;
    for (int i = 0; i < n_off; i++) js.push_back((((offsets[i] % m) + m + m / 2) % m) - m / 2);  // centred
    std::sort(js.begin(), js.end());
    js.erase(std::unique(js.begin(), js.end()), js.end());
    lt.js = js;
    bsgs_split(lt, n);
    lt.dl = level + 1, lt.scale = (double)c->primes[level];
    lt.stages = ilog2(m);  // the structure of a conv fused with StoC2 on C = n / u channels
    p->ell = u, p->C = m, p->c_in = m * bi, p->c_out = m * bo;
    for (p->W = 1; p->W * p->W < 2 * u; p->W *= 2) {}
    const size_t count = (size_t)bo * bi * lt.n_diag;
    if (hipMalloc(&lt.d_diag, count * lt.dl * c->N * 8) != hipSuccess) {
        delete p;
        return fail(NJ_ENOMEM, "nj_plan_create_random: device memory");
    }
    hipError_t e = fill_random(c, lt.d_diag, (int)count, lt.dl, lt.dl, seed, 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        nj_plan_destroy(p);
        return fail(NJ_EDEVICE, hipGetErrorString(e));
    }
    *out = p;
    return NJ_OK;
}

nj_status nj_time_plan(nj_ctx *c, const nj_plan *p, int t, int level, int reps, float *ms)
{
    if (!c || !p || t < 0 || t >= (int)p->lts.size() || reps < 1 || !ms)
        return fail(NJ_EINVAL, "nj_time_plan: bad arguments");
    if (level < 0 || level > p->lts[t].level) return fail(NJ_ELEVEL, "nj_time_plan: level above the transform's");
    const nj_lt_t lt = at_level(p->lts[t], level);
    const bool blk = lt.bi != 1 || lt.bo != 1;
    const size_t N = c->N, clen = 2 * N * (level + 1);
    uint64_t *x = nullptr, *y = nullptr;
    NJ_HIP(hipMalloc(&x, clen * lt.bi * 8));
    if (hipMalloc(&y, clen * lt.bo * 8) != hipSuccess) {
        (void)hipFree(x);
        return fail(NJ_ENOMEM, "nj_time_plan: device memory");
    }
    auto done = [&](nj_status st) {
        (void)hipDeviceSynchronize();
        (void)hipFree(x), (void)hipFree(y);
        return st;
    };
    if (fill_random(c, x, 2 * lt.bi, level + 1, level + 1, 77, 0) != hipSuccess) return done(fail(NJ_EDEVICE, "fill"));
    bool ok;
    Arena A = arena_for(c, blk ? block_words(c, lt) : bsgs_words(c, lt), ok);
    if (!ok) return done(fail(NJ_ENOMEM, "scratch"));
    hipEvent_t a, b;
    NJ_HIP(hipEventCreate(&a));
    NJ_HIP(hipEventCreate(&b));
    std::vector<float> times;
    nj_status st = NJ_OK;
    for (int r = 0; r <= reps && !st; r++) {
        (void)hipEventRecord(a, 0);
        st = blk ? block_bsgs_apply(c, lt, x, y, A, 0) : bsgs_apply(c, lt, x, y, lt.hoist ? 1 : 0, A, 0);
        (void)hipEventRecord(b, 0);
        (void)hipEventSynchronize(b);
        float v = 0.f;
        (void)hipEventElapsedTime(&v, a, b);
        if (r > 0) times.push_back(v);  // the first run warms up
    }
    (void)hipEventDestroy(a), (void)hipEventDestroy(b);
    if (st) return done(st);
    std::sort(times.begin(), times.end());
    *ms = times[times.size() / 2];
    return done(NJ_OK);
}

nj_status nj_plan_features(const nj_plan *p, int t, int level, float *f)
{
    if (!p || t < 0 || t >= (int)p->lts.size() || !f) return fail(NJ_EINVAL, "nj_plan_features: bad arguments");
    const nj_lt_t &lt = p->lts[t];
    const int n = p->N / 2;
    const bool hoisted = lt.hoist || lt.bi != 1 || lt.bo != 1;  // block transforms always hoist
    f[0] = (float)(level + 1);                                  // level
    f[1] = (float)lt.n_diag;                                    // channels: diagonals per block
    f[2] = (float)ilog2(n / lt.u);                              // slot stride of the rotations (image size)
    f[3] = (float)lt.babies.size();                             // BSGS split: baby steps
    f[4] = hoisted ? (float)(lt.bi * ((int)lt.babies.size() - 1)) : 0.f;  // hoisted baby rotations
    f[5] = (float)lt.stages;                                    // fusion depth: DFT stages merged in
    f[6] = (float)lt.bo;                                        // output blocks (giant rotations per step)
    return NJ_OK;
}

}  // extern "C"
