// Plan construction: fused conv (K' = S'K^), tap-list / block convs and CoeffToSlot
// stage groups, encoded as integer plaintexts and kept on the device in evaluation form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <set>

#include "internal.h"

using namespace nj;

namespace nj {

// encode complex diagonals at `scale`, reduce into the level's primes, transform.
// re.size() diagonals (lt.n_diag per block); empty ones are zero and stay zero.
nj_status upload_plan_diagonals(nj_ctx *c, nj_lt_t &lt, const std::vector<std::vector<double>> &re,
                           const std::vector<std::vector<double>> &im, double scale)
{
    const size_t N = c->N, plen = N * (lt.level + 1), count = re.size();
    lt.dl = lt.level + 1;
    lt.scale = scale;
    NJ_HIP(hipMalloc(&lt.d_diag, plen * count * 8));
    int64_t *tmp = nullptr;
    NJ_HIP(hipMalloc(&tmp, N * 8));
    std::vector<int64_t> coeffs(N);
    for (size_t d = 0; d < count; d++) {
        uint64_t *dst = lt.d_diag + d * plen;
        if (re[d].empty()) {
            NJ_HIP(hipMemset(dst, 0, plen * 8));
            continue;
        }
        encode_slots(c->N, re[d].data(), im[d].data(), scale, coeffs.data());
        NJ_HIP(hipMemcpy(tmp, coeffs.data(), N * 8, hipMemcpyHostToDevice));
        NJ_HIP(launch_signed_to_rns(c, tmp, limbs_q(lt.level), dst, 0, c->d_primes));
        NJ_HIP(launch_ntt(c, dst, limbs_q(lt.level), false, 0));
    }
    NJ_HIP(hipDeviceSynchronize());
    NJ_HIP(hipFree(tmp));
    return NJ_OK;
}

}  // namespace nj

int plan_galois_impl(const nj_plan *p, std::vector<uint32_t> &gs)
{
    std::set<uint32_t> s;
    const long long n = p->N / 2;
    auto gal = [&](long long r) {
        long long rr = ((r % n) + n) % n;
        uint64_t g = 1, b = 5, e = (uint64_t)rr, m = 2ull * p->N;
        for (; e; e >>= 1, b = b * b % m)
            if (e & 1) g = g * b % m;
        return (uint32_t)g;
    };
    for (const auto &lt : p->lts) {
        for (int i : lt.babies)
            if (i) s.insert(gal((long long)i * lt.u));
        for (int g : lt.giants)
            if (g) s.insert(gal((long long)g * lt.n1 * lt.u));
    }
    if (p->kind == 1) s.insert(2u * p->N - 1u);
    gs.assign(s.begin(), s.end());
    return (int)gs.size();
}

extern "C" {

nj_status nj_conv_plan_create(nj_ctx *c, int w0, int f, const double *weights, int n1, nj_plan **out)
{
    if (!c || !weights || !out || w0 < 1 || f < 1) return fail(NJ_EINVAL, "nj_conv_plan_create: bad arguments");
    if (c->L < 1) return fail(NJ_ELEVEL, "nj_conv_plan_create: needs at least two ciphertext primes");
    nj_plan *p = new nj_plan();
    p->kind = 0;
    p->N = c->N;
    p->lts.resize(1);
    nj_lt_t &lt = p->lts[0];
    lt.level = 1;
    std::vector<std::vector<double>> re, im;
    nj_status st = build_conv_diagonals(c->N, w0, f, weights, n1, lt, re, im);
    if (st) {
        delete p;
        return st;
    }
    p->ell = lt.u;
    p->C = (c->N / 2) / lt.u;
    p->w0 = w0;
    p->f = f;
    p->c_in = p->c_out = p->C;
    for (p->W = 1; p->W * p->W < 2 * lt.u; p->W *= 2) {}
    st = upload_plan_diagonals(c, lt, re, im, (double)c->primes[1]);
    if (st) {
        nj_plan_destroy(p);
        return st;
    }
    *out = p;
    return NJ_OK;
}

nj_status nj_conv_plan_create_taps(nj_ctx *c, int w0, int c_in, int c_out, const nj_tap *taps, int n_taps, int fuse,
                                   int n1, int level, nj_plan **out)
{
    if (!c || !taps || !out || w0 < 1 || c_in < 1 || c_out < 1 || n_taps < 1 || n1 < 0)
        return fail(NJ_EINVAL, "nj_conv_plan_create_taps: bad arguments");
    if (level < 1 || level > c->L) return fail(NJ_ELEVEL, "nj_conv_plan_create_taps: need 1 <= level <= L");
    int reach = 0;
    for (int t = 0; t < n_taps; t++) reach = std::max(reach, std::max(std::abs(taps[t].dy), std::abs(taps[t].dx)));
    int W = 1;
    while (W < w0 + reach) W *= 2;
    if (W * W > c->N) return fail(NJ_EUNSUPPORTED, "nj_conv_plan_create_taps: padded image larger than N");
    nj_plan *p = new nj_plan();
    p->kind = 0;
    p->N = c->N;
    p->lts.resize(1);
    nj_lt_t &lt = p->lts[0];
    lt.level = level;
    std::vector<std::vector<double>> re, im;
    nj_status st = build_block_diagonals(c->N, W, c_in, c_out, taps, n_taps, fuse ? 1 : 0, n1, lt, re, im);
    if (st) {
        delete p;
        return st;
    }
    p->W = W, p->ell = lt.u, p->C = (c->N / 2) / lt.u, p->w0 = w0, p->f = 0;
    p->c_in = c_in, p->c_out = c_out;
    st = upload_plan_diagonals(c, lt, re, im, (double)c->primes[level]);
    if (st) {
        nj_plan_destroy(p);
        return st;
    }
    *out = p;
    return NJ_OK;
}

nj_status nj_conv_taps(int c_in, int c_out, int f, int stride, int depthwise, const double *weights, nj_tap *taps,
                       int max_taps, int *n_taps)
{
    if (!weights || !n_taps || c_in < 1 || c_out < 1 || f < 1 || f % 2 == 0 || (stride != 1 && stride != 2) ||
        (depthwise && c_in != c_out))
        return fail(NJ_EINVAL, "nj_conv_taps: bad arguments");
    const int p = (f - 1) / 2;
    const long long need = (long long)(depthwise ? c_out : c_out * c_in) * f * f;
    *n_taps = (int)need;
    if (!taps) return NJ_OK;
    if (max_taps < need) return fail(NJ_EINVAL, "nj_conv_taps: tap buffer too small");
    auto fdiv = [](int a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); };  // floor(a / 2)
    int k = 0;
    for (int o = 0; o < c_out; o++)
        for (int i = depthwise ? o : 0; i < (depthwise ? o + 1 : c_in); i++)
            for (int u = 0; u < f; u++)
                for (int v = 0; v < f; v++) {
                    nj_tap t;
                    t.out_ch = o;
                    t.w = depthwise ? weights[((size_t)o * f + u) * f + v] : weights[(((size_t)o * c_in + i) * f + u) * f + v];
                    if (stride == 1) {
                        t.in_ch = i, t.dy = u - p, t.dx = v - p;
                    } else {  // phase (a, b) = (u - p, v - p) mod 2 of input channel i: channel 4 i + 2 b + a
                        t.dy = fdiv(u - p), t.dx = fdiv(v - p);
                        const int a = (u - p) - 2 * t.dy, b = (v - p) - 2 * t.dx;
                        t.in_ch = 4 * i + 2 * b + a;
                    }
                    taps[k++] = t;
                }
    return NJ_OK;
}

nj_status nj_conv_plan_create_layer(nj_ctx *c, const nj_conv_desc *d, const double *weights, int n1, int level,
                                    nj_plan **out)
{
    if (!c || !d || !weights || !out) return fail(NJ_EINVAL, "nj_conv_plan_create_layer: null argument");
    if (d->stride == 2 && d->w0 % 2) return fail(NJ_EINVAL, "nj_conv_plan_create_layer: stride 2 needs an even width");
    int n = 0;
    nj_status st = nj_conv_taps(d->c_in, d->c_out, d->f, d->stride, d->depthwise, weights, nullptr, 0, &n);
    if (st) return st;
    std::vector<nj_tap> taps(n);
    if ((st = nj_conv_taps(d->c_in, d->c_out, d->f, d->stride, d->depthwise, weights, taps.data(), n, &n))) return st;
    const int w_in = d->stride == 2 ? d->w0 / 2 : d->w0, ci = d->stride == 2 ? 4 * d->c_in : d->c_in;
    return nj_conv_plan_create_taps(c, w_in, ci, d->c_out, taps.data(), n, d->fuse, n1, level, out);
}

nj_status nj_downsample_plan_create(nj_ctx *c, int kind, int W, int C, int half, int n1, int level, nj_plan **out)
{
    if (!c || !out || n1 < 0) return fail(NJ_EINVAL, "nj_downsample_plan_create: bad arguments");
    if (level < 1 || level > c->L) return fail(NJ_ELEVEL, "nj_downsample_plan_create: need 1 <= level <= L");
    nj_plan *p = new nj_plan();
    p->kind = 0;
    p->N = c->N;
    p->lts.resize(1);
    nj_lt_t &lt = p->lts[0];
    lt.level = level;
    std::vector<std::vector<double>> re, im;
    nj_status st = build_downsample_diagonals(c->N, kind, W, C, half, n1, lt, re, im);
    if (st) {
        delete p;
        return st;
    }
    p->W = W / 2, p->C = 4 * C, p->ell = (W / 2) * (W / 2) / 2, p->w0 = 0, p->f = 0;
    p->c_in = kind == 0 ? C : 4 * C, p->c_out = 4 * C;
    st = upload_plan_diagonals(c, lt, re, im, (double)c->primes[level]);
    if (st) {
        nj_plan_destroy(p);
        return st;
    }
    *out = p;
    return NJ_OK;
}

nj_status nj_fc_plan_create(nj_ctx *c, int n_in, int n_out, const double *weights, int n1, int level, nj_plan **out)
{
    if (!c || !weights || !out || n1 < 0) return fail(NJ_EINVAL, "nj_fc_plan_create: bad arguments");
    if (level < 1 || level > c->L) return fail(NJ_ELEVEL, "nj_fc_plan_create: need 1 <= level <= L");
    nj_plan *p = new nj_plan();
    p->kind = 0;
    p->N = c->N;
    p->lts.resize(1);
    nj_lt_t &lt = p->lts[0];
    lt.level = level;
    std::vector<std::vector<double>> re, im;
    nj_status st = build_fc_diagonals(c->N, n_in, n_out, weights, n1, lt, re, im);
    if (st) {
        delete p;
        return st;
    }
    p->W = 1, p->C = c->N / 2, p->ell = 1, p->w0 = 1, p->f = 1, p->c_in = n_in, p->c_out = n_out;
    st = upload_plan_diagonals(c, lt, re, im, (double)c->primes[level]);
    if (st) {
        nj_plan_destroy(p);
        return st;
    }
    *out = p;
    return NJ_OK;
}

int nj_plan_layout(const nj_plan *p, int *W, int *C, int *ell, int *bi, int *bo)
{
    if (!p || p->lts.empty()) return -1;
    if (W) *W = p->W;
    if (C) *C = p->C;
    if (ell) *ell = p->ell;
    if (bi) *bi = p->lts[0].bi;
    if (bo) *bo = p->lts[0].bo;
    return p->lts[0].level;
}

nj_status nj_cts_plan_create(nj_ctx *c, int groups, nj_plan **out) { return nj_cts_plan_create_split(c, groups, nullptr, out); }

nj_status nj_cts_plan_features(nj_ctx *c, int groups, const int *n1, int hoist, float *f)
{
    if (!c || !f) return fail(NJ_EINVAL, "nj_cts_plan_features: null argument");
    if (groups < 1 || groups > c->L) return fail(NJ_ELEVEL, "nj_cts_plan_features: need 1 <= groups <= L");
    nj_plan p;
    p.kind = 1;
    p.N = c->N;
    std::vector<std::vector<std::vector<double>>> re, im;
    nj_status st = build_cts_diagonals(c->N, groups, n1, p.lts, re, im);
    if (st) return st;
    for (int g = 0; g < groups; g++) {
        p.lts[g].level = c->L - g;
        p.lts[g].hoist = hoist != 0;
        if ((st = nj_plan_features(&p, g, c->L - g, f + 7 * g))) return st;
    }
    return NJ_OK;
}

nj_status nj_cts_plan_create_split(nj_ctx *c, int groups, const int *n1, nj_plan **out)
{
    if (!c || !out) return fail(NJ_EINVAL, "nj_cts_plan_create: null argument");
    if (groups < 1 || groups > c->L) return fail(NJ_ELEVEL, "nj_cts_plan_create: need 1 <= groups <= L");
    if (n1)
        for (int g = 0; g < groups; g++)
            if (n1[g] < 0 || n1[g] > c->N / 2) return fail(NJ_EINVAL, "nj_cts_plan_create_split: bad baby-step count");
    nj_plan *p = new nj_plan();
    p->kind = 1;
    p->N = c->N;
    std::vector<std::vector<std::vector<double>>> re, im;
    nj_status st = build_cts_diagonals(c->N, groups, n1, p->lts, re, im);
    if (st) {
        delete p;
        return st;
    }
    for (int g = 0; g < groups; g++) {
        nj_lt_t &lt = p->lts[g];
        lt.level = c->L - g;
        st = upload_plan_diagonals(c, lt, re[g], im[g], (double)c->primes[lt.level]);
        if (st) {
            nj_plan_destroy(p);
            return st;
        }
    }
    *out = p;
    return NJ_OK;
}

}  // extern "C"
