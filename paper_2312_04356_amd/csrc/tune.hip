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

// Cost-model features of a transform at `level` (see nj_plan_features)
void lt_features(const nj_lt_t &lt, int N, int level, float *f)
{
    const int n = N / 2;
    const bool hoisted = lt.hoist || lt.bi != 1 || lt.bo != 1;  // block transforms always hoist
    f[0] = (float)(level + 1);                                  // level
    f[1] = (float)lt.n_diag;                                    // channels: diagonals per block
    f[2] = (float)ilog2(n / lt.u);                              // slot stride of the rotations (image size)
    f[3] = (float)lt.babies.size();                             // BSGS split: baby steps
    f[4] = hoisted ? (float)(lt.bi * ((int)lt.babies.size() - 1)) : 0.f;  // hoisted baby rotations
    f[5] = (float)lt.stages;                                    // fusion depth: DFT stages merged in
    f[6] = (float)lt.bo;                                        // output blocks (giant rotations per step)
}

// baby-step counts the tuner tries: 0 (the library's default split) and the powers of
// two within a factor 4 of sqrt(#diagonals), at most the diagonal count
std::vector<int> split_candidates(int n_diag)
{
    std::vector<int> out{0};
    const double r = std::sqrt((double)n_diag);
    for (int k = 0; k < 12; k++) {
        const int v = 1 << k;
        if (r / 4 <= v && v <= 4 * r && v <= std::max(1, n_diag)) out.push_back(v);
    }
    return out;
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
    lt_features(p->lts[t], p->N, level, f);
    return NJ_OK;
}

nj_status nj_tune_split(nj_ctx *c, const nj_plan *p, int t, int level, const nj_mlp *model, int shortlist, int reps,
                        int *n1_out, int *hoist_out, int *lazy_out, float *ms_out, float *default_ms)
{
    if (!c || !p || t < 0 || t >= (int)p->lts.size() || reps < 1 || shortlist < 0 || !n1_out || !hoist_out || !ms_out)
        return fail(NJ_EINVAL, "nj_tune_split: bad arguments");
    if (p->N != c->N) return fail(NJ_EINVAL, "nj_tune_split: plan of another ring");
    const nj_lt_t &src = p->lts[t];
    if (level < 1 || level > src.level) return fail(NJ_ELEVEL, "nj_tune_split: need 1 <= level <= the transform's");
    const bool blk = src.bi != 1 || src.bo != 1;  // block transforms always hoist
    const int n = c->N / 2;
    struct Cand {
        int n1;
        bool hoist;
        float score, ms;
    };
    std::vector<Cand> cands;
    for (int n1 : split_candidates(src.n_diag))
        for (int h = 1; h >= (blk ? 1 : 0); h--) cands.push_back(Cand{n1, h != 0, 0.f, -1.f});
    // the model ranks the candidates by predicted latency (features of each split,
    // computed without building it); without a model every candidate is timed
    std::vector<int> order(cands.size());
    for (size_t i = 0; i < cands.size(); i++) order[i] = (int)i;
    if (model && shortlist > 0) {
        std::vector<float> X(cands.size() * NJ_MLP_FEATURES), y(cands.size());
        for (size_t i = 0; i < cands.size(); i++) {
            nj_lt_t lt = src;
            lt.d_diag = nullptr;
            lt.n1 = cands[i].n1, lt.hoist = cands[i].hoist;
            bsgs_split(lt, n);
            lt_features(lt, c->N, level, &X[i * NJ_MLP_FEATURES]);
        }
        nj_status st = nj_mlp_predict(const_cast<nj_mlp *>(model), X.data(), (int)cands.size(), y.data());
        if (st) return st;
        for (size_t i = 0; i < cands.size(); i++) cands[i].score = y[i];
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cands[a].score < cands[b].score; });
    }
    // timed: the shortlist (or every candidate) and always the default split, hoisted
    std::vector<int> timed;
    for (int i : order)
        if (!model || shortlist == 0 || (int)timed.size() < shortlist) timed.push_back(i);
    for (size_t i = 0; i < cands.size(); i++)
        if (cands[i].n1 == 0 && cands[i].hoist && std::find(timed.begin(), timed.end(), (int)i) == timed.end())
            timed.push_back((int)i);
    // each timed split with the plan's own giant-step ModDown and, when asked for
    // (lazy_out), with the other (one ModDown per giant step, or one for all); block
    // transforms have only per-step ModDowns
    std::vector<int32_t> offs(src.js.begin(), src.js.end());
    int best = -1;
    bool best_lazy = src.lazy;
    float best_ms = 0.f;
    for (int i : timed)
        for (int v = 0; v < (lazy_out && !blk ? 2 : 1); v++) {
            const bool lz = v ? !src.lazy : src.lazy;
            nj_plan *q = nullptr;
            nj_status st = nj_plan_create_random(c, level, src.u, offs.data(), (int)offs.size(), cands[i].n1, src.bi,
                                                 src.bo, 0x7u + (uint64_t)i, &q);
            if (st) return st;
            q->lts[0].stages = src.stages, q->lts[0].hoist = cands[i].hoist, q->lts[0].lazy = lz;
            float ms = 0.f;
            st = nj_time_plan(c, q, 0, level, reps, &ms);
            nj_plan_destroy(q);
            if (st) return st;
            if (v == 0) cands[i].ms = ms;  // the plan's own setting (the default's time)
            if (best < 0 || ms < best_ms) best = i, best_lazy = lz, best_ms = ms;
        }
    *n1_out = cands[best].n1, *hoist_out = cands[best].hoist ? 1 : 0, *ms_out = best_ms;
    if (lazy_out) *lazy_out = best_lazy ? 1 : 0;
    if (default_ms)
        for (const Cand &k : cands)
            if (k.n1 == 0 && k.hoist) *default_ms = k.ms;
    return NJ_OK;
}

}  // extern "C"
