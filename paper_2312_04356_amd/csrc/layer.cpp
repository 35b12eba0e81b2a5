// Algorithm 1 (default conv2d and activation, Sec. 4) as library calls: the zero-
// padding masks, the slot-domain tail after CoeffToSlot (ModEval of Re and Im, masks,
// activation, Re + i Im, StoC1), the whole layer from a CinS input, and bootstrapping
// (the same chain without conv, masks and activation).  The composite calls run the
// library's own entry points in stream order; their intermediate ciphertexts live in a
// context-owned buffer of full-size ciphertext slots, apart from the scratch the inner
// calls use.
#include <algorithm>
#include <string>

#include "exec.h"
#include "internal.h"

using namespace nj;

namespace {

// slot i of the context's layer buffer (2 (L+1) N words each), n slots guaranteed
uint64_t *layer_slot(nj_ctx *c, int n, int i)
{
    const size_t words = 2 * (size_t)c->N * (c->L + 1);
    if (c->layer_words < words * n) {
        if (c->layer_buf) {
            (void)hipDeviceSynchronize();
            (void)hipFree(c->layer_buf);
            c->layer_buf = nullptr;
            c->layer_words = 0;
        }
        if (hipMalloc(&c->layer_buf, words * n * 8) != hipSuccess) return nullptr;
        c->layer_words = words * n;
    }
    return c->layer_buf + words * i;
}

nj_ct slot_ct(uint64_t *d) { return nj_ct{d, 0, 1, 0.0}; }

constexpr int kTailSlots = 6;   // nj_slot_activation uses slots 0..5
constexpr int kLayerSlots = 9;  // nj_conv_act_layer adds 6..8

uint32_t brev(uint32_t x, int bits)
{
    uint32_t r = 0;
    for (int i = 0; i < bits; i++) r = (r << 1) | ((x >> i) & 1u);
    return r;
}

}  // namespace

extern "C" {

nj_status nj_layer_masks(int log_n, int W, int C, int w0, double *mask_re, double *mask_im)
{
    if (log_n < 2 || log_n > 20 || W < 1 || C < 1 || w0 < 1 || w0 > W || !mask_re || !mask_im)
        return fail(NJ_EINVAL, "nj_layer_masks: bad arguments");
    const long long N = 1ll << log_n;
    if ((long long)W * W * C != N) return fail(NJ_EINVAL, "nj_layer_masks: W^2 C must equal N");
    const uint32_t n2 = (uint32_t)(N / 2);
    auto out_pixel = [&](long long k) {
        const long long p = k / C;  // padded pixel of coefficient k
        return (p / W < w0 && p % W < w0) ? 1.0 : 0.0;
    };
    for (uint32_t j = 0; j < n2; j++) {
        const uint32_t k = brev(j, log_n - 1);
        mask_re[j] = out_pixel(k);
        mask_im[j] = out_pixel((long long)n2 + k);
    }
    return NJ_OK;
}

nj_status nj_slot_activation(nj_ctx *c, int K, int r, const double *coeffs, int n_coeffs, const uint64_t *mask_re,
                             const uint64_t *mask_im, int act, const nj_plan *stoc1, const nj_ct *re, const nj_ct *im,
                             nj_ct *out, void *stream)
{
    return nj_slot_activation_decompose(c, K, r, coeffs, n_coeffs, mask_re, mask_im, act, nullptr, nullptr, stoc1, re,
                                        im, out, stream);
}

nj_status nj_slot_activation_decompose(nj_ctx *c, int K, int r, const double *coeffs, int n_coeffs,
                                       const uint64_t *mask_re, const uint64_t *mask_im, int act,
                                       const nj_plan *dec_re, const nj_plan *dec_im, const nj_plan *stoc1,
                                       const nj_ct *re, const nj_ct *im, nj_ct *out, void *stream)
{
    if (!c || !re || !im || !out || !stoc1) return fail(NJ_EINVAL, "nj_slot_activation: null argument");
    if ((dec_re == nullptr) != (dec_im == nullptr))
        return fail(NJ_EINVAL, "nj_slot_activation_decompose: give both decomposition plans or none");
    if (re->level != im->level) return fail(NJ_ELEVEL, "nj_slot_activation: Re and Im must share a level");
    if (act != 0 && act != 1) return fail(NJ_EINVAL, "nj_slot_activation: act must be 0 (none) or 1 (square)");
    if ((mask_re == nullptr) != (mask_im == nullptr)) return fail(NJ_EINVAL, "nj_slot_activation: give both masks or none");
    if (!layer_slot(c, kTailSlots, 0)) return fail(NJ_ENOMEM, "nj_slot_activation: layer buffers");
    nj_ct s[kTailSlots];
    for (int i = 0; i < kTailSlots; i++) s[i] = slot_ct(layer_slot(c, kTailSlots, i));
    nj_status st;
    if ((st = ex::eval_mod_pair(c, re, im, K, r, coeffs, n_coeffs, &s[0], &s[1], stream))) return st;
    nj_ct *cr = &s[0], *ci = &s[1];
    if (mask_re) {  // masks encoded at q_l: PMult then rescale by q_l leaves the scale as it was
        const double sc = cr->scale;
        if ((st = nj_pmult(c, cr, mask_re, &s[2], stream)) || (st = nj_rescale(c, &s[2], &s[3], stream))) return st;
        if ((st = nj_pmult(c, ci, mask_im, &s[2], stream)) || (st = nj_rescale(c, &s[2], &s[4], stream))) return st;
        s[3].scale = s[4].scale = sc;
        cr = &s[3], ci = &s[4];
    }
    if (act == 1) {  // the square (Sec. 2.5.2): HMult, relinearisation, rescale
        nj_ct *dr = cr == &s[0] ? &s[3] : &s[0], *di = cr == &s[0] ? &s[4] : &s[1];
        if ((st = nj_hmult(c, cr, cr, dr, stream)) || (st = nj_hmult(c, ci, ci, di, stream))) return st;
        cr = dr, ci = di;
    }
    if (dec_re) {  // Algorithm 2: each half rearranged into the phase images (transform + rescale)
        nj_ct *dr = cr == &s[0] ? &s[3] : &s[0], *di = cr == &s[0] ? &s[4] : &s[1];
        const int pl = dec_re->lts.empty() ? -1 : dec_re->lts[0].level;
        if (pl < 1 || dec_im->lts.empty() || dec_im->lts[0].level != pl)
            return fail(NJ_EINVAL, "nj_slot_activation_decompose: bad decomposition plans");
        if (cr->level < pl) return fail(NJ_ELEVEL, "nj_slot_activation_decompose: plans above the activated level");
        if (cr->level > pl) {
            if ((st = nj_drop_level(c, cr, pl, dr, stream)) || (st = nj_drop_level(c, ci, pl, di, stream))) return st;
            std::swap(cr, dr), std::swap(ci, di);
        }
        if ((st = nj_conv2d_cins(c, dec_re, cr, dr, stream)) || (st = nj_conv2d_cins(c, dec_im, ci, di, stream)))
            return st;
        cr = dr, ci = di;
    }
    if ((st = nj_combine(c, cr, ci, &s[2], stream))) return st;
    nj_ct *z = &s[2];
    const int pl = stoc1->kind == 2 && !stoc1->lts.empty() ? stoc1->lts[0].level : -1;
    if (pl < 0) return fail(NJ_EINVAL, "nj_slot_activation: not a StoC1 plan");
    if (z->level < pl) return fail(NJ_ELEVEL, "nj_slot_activation: the StoC1 plan starts above the combined level");
    if (z->level > pl) {
        if ((st = nj_drop_level(c, z, pl, &s[5], stream))) return st;
        z = &s[5];
    }
    return nj_stoc1(c, stoc1, z, out, stream);
}

nj_status nj_conv_act_layer(nj_ctx *c, const nj_plan *conv, const nj_plan *cts, int K, int r, const double *coeffs,
                            int n_coeffs, const uint64_t *mask_re, const uint64_t *mask_im, int act,
                            const nj_plan *stoc1, const nj_ct *in, nj_ct *out, void *stream)
{
    if (!c || !cts || !in || !out) return fail(NJ_EINVAL, "nj_conv_act_layer: null argument");
    if (!layer_slot(c, kLayerSlots, 0)) return fail(NJ_ENOMEM, "nj_conv_act_layer: layer buffers");
    nj_ct y = slot_ct(layer_slot(c, kLayerSlots, 6)), re = slot_ct(layer_slot(c, kLayerSlots, 7)),
          im = slot_ct(layer_slot(c, kLayerSlots, 8));
    nj_status st;
    const nj_ct *x0 = in;
    if (conv) {
        if ((st = nj_conv2d_cins(c, conv, in, &y, stream))) return st;
        if (y.level > 0) {  // the conv output enters ModRaise at level 0
            nj_ct y0 = slot_ct(layer_slot(c, kLayerSlots, 7));
            if ((st = nj_drop_level(c, &y, 0, &y0, stream))) return st;
            NJ_HIP(hipMemcpyAsync(y.data, y0.data, 2 * (size_t)c->N * 8, hipMemcpyDeviceToDevice, ex::S(stream)));
            y.level = 0, y.scale = y0.scale;
        }
        x0 = &y;
    }
    if ((st = nj_coeff_to_slot(c, cts, x0, &re, &im, stream))) return st;
    return nj_slot_activation(c, K, r, coeffs, n_coeffs, mask_re, mask_im, act, stoc1, &re, &im, out, stream);
}

nj_status nj_bootstrap(nj_ctx *c, const nj_plan *cts, int K, int r, const double *coeffs, int n_coeffs,
                       const nj_plan *stoc1, const nj_ct *in, nj_ct *out, void *stream)
{
    return nj_conv_act_layer(c, nullptr, cts, K, r, coeffs, n_coeffs, nullptr, nullptr, 0, stoc1, in, out, stream);
}

}  // extern "C"
