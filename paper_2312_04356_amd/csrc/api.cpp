// C ABI entry points: key generation, encryption, hybrid key switching, rotations,
// rescale, ModRaise, BSGS linear transforms, the fused conv and CoeffToSlot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>

#include "exec.h"

using namespace nj;

int plan_galois_impl(const nj_plan *p, std::vector<uint32_t> &gs);

namespace nj {
namespace ex {



size_t ks_words(const nj_ctx *c, int l) { return multi_words(c, l, 1) + (size_t)c->N * (l + 1); }

const uint64_t *key_of(const nj_ctx *c, uint32_t g)
{
    auto it = c->keys.find(g);
    if (it != c->keys.end()) return it->second.d;
    if (!c->timing_keys.empty()) return c->timing_keys[g % c->timing_keys.size()];
    return nullptr;
}

// N >= 8192 with at most 4 digits: ModUp stops after the column pass and the key inner
// product runs the extended digits' tile pass itself (jobs with g = 1)
bool fuse_ip(const nj_ctx *c, int l) { return c->N >= 8192 && c->alpha <= 8 && n_digits(c, l) <= 4; }

nj_status ks_fused(nj_ctx *c, int l, int K, const KeyJobs &kj, const MdJobs &mj, int sum, const uint64_t *acc,
                   MultiBufs &M, hipStream_t s, const MdConj *conj)
{
    NJ_HIP(launch_ntt_ip(c, l, kj, K, M.u, 0, 0, s, M.pc));
    return ks_down(c, l, K, mj, sum, acc, M, s, true, nullptr, conj);
}

// One key switch of tau_g(d) (d in evaluation form, level l) with `key`: ModUp,
// inner product, ModDown, and out = (ModDown_0 + add read through X -> X^g_add,
// ModDown_1) (add may be null).  The single-job case of the batched path, so it runs
// the same kernels; where the inner product runs the digits' tile pass the
// automorphism rides on ModUp's inverse transform and on the own-limb reads.
nj_status ks_one(nj_ctx *c, int l, const uint64_t *d, uint32_t g, const uint64_t *key, const uint64_t *add,
                 uint32_t g_add, uint64_t *out, MultiBufs &M, hipStream_t s, const MdConj *conj)
{
    const bool f = fuse_ip(c, l);
    if (conj && !f) return fail(NJ_EUNSUPPORTED, "key switch: the fused split needs the fused inner product");
    if (!f && g != 1u) {  // the automorphism first, into M.d
        AutoJobs aj;
        aj.in[0] = d, aj.out[0] = M.d, aj.g[0] = g;
        NJ_HIP(launch_automorph_multi(c, aj, 1, l + 1, s));
        d = M.d, g = 1;
    }
    GalTab gt;
    gt.g[0] = g;
    nj_status st = modup_multi(c, l, 1, d, M, s, -1, !f, f && g != 1u ? &gt : nullptr);
    if (st) return st;
    KeyJobs kj;
    MdJobs mj;
    kj.ext[0] = M.ext, kj.d[0] = d, kj.g[0] = g, kj.key[0] = key;
    mj.add[0] = add, mj.g_add[0] = g_add, mj.out[0] = out;
    return f ? ks_fused(c, l, 1, kj, mj, 0, nullptr, M, s, conj) : ks_multi(c, l, 1, kj, mj, 0, nullptr, M, s);
}

// (tau_g(c0), tau_g(c1)) switched back to s; in and out may alias.
nj_status apply_galois(nj_ctx *c, int l, const uint64_t *in, uint32_t g, uint64_t *out, Arena A, hipStream_t s)
{
    if (g % 2 == 0 || g >= 2u * (uint32_t)c->N) return fail(NJ_EINVAL, "Galois element must be odd and below 2N");
    if (g == 1) {  // X -> X: the identity (a rotation by a multiple of N/2 slots), no key switch
        if (out != in) NJ_HIP(hipMemcpyAsync(out, in, 2 * (size_t)c->N * (l + 1) * 8, hipMemcpyDeviceToDevice, s));
        return NJ_OK;
    }
    const uint64_t *key = key_of(c, g);
    if (!key) return fail(NJ_ENOKEY, "no switching key for Galois element " + std::to_string(g));
    MultiBufs M;
    if (!multi_bufs(c, l, 1, A, M)) return fail(NJ_ENOMEM, "scratch too small");
    const size_t N = c->N, plen = N * (l + 1);
    const uint64_t *c0 = in;
    if (in == out) {  // the combine reads c0 at permuted positions while writing out
        uint64_t *cp = A.take(plen);
        if (!cp) return fail(NJ_ENOMEM, "scratch too small");
        NJ_HIP(hipMemcpyAsync(cp, in, plen * 8, hipMemcpyDeviceToDevice, s));
        c0 = cp;
    }
    return ks_one(c, l, in + plen, g, key, c0, g, out, M, s);
}

int galois_of_rot(const nj_ctx *c, long long r) { return (int)nj_galois_elt(c, (int)(((r % (c->N / 2)) + c->N / 2) % (c->N / 2))); }


size_t multi_words(const nj_ctx *c, int l, int K)
{
    const size_t N = c->N, ne = l + 1 + c->alpha, nd = n_digits(c, l);
    return N * K * (2 * (l + 1) + nd * ne + 2 * ne + 2 * c->alpha + 2 * (l + 1));
}

bool multi_bufs(const nj_ctx *c, int l, int K, Arena &A, MultiBufs &M)
{
    const size_t N = c->N, ne = l + 1 + c->alpha, nd = n_digits(c, l);
    M.d = A.take(N * K * (l + 1));
    M.coef = A.take(N * K * (l + 1));
    M.ext = A.take(N * K * nd * ne);
    M.u = A.take(N * K * 2 * ne);
    M.pc = A.take(N * K * 2 * c->alpha);
    M.conv = A.take(N * K * 2 * (l + 1));
    return M.conv != nullptr;
}

// ModUp of K polynomials stored at d + z dstride N (evaluation form; dstride in limbs,
// l+1 when packed) into ext + z dnum ne N.
nj_status modup_multi(nj_ctx *c, int l, int K, const uint64_t *d, MultiBufs &M, hipStream_t s, int dstride,
                      bool tiles, const GalTab *gt, const int *zoff, bool drop)
{
    const auto &tabs = drop ? c->modup_drop[l] : c->modup[l];
    const int N = c->N, ne = l + 1 + c->alpha, nd = n_digits(c, l);
    // N >= 8192: the conversion's input factors ride on the inverse transform, and the
    // conversion runs fused with its outputs' column pass
    const bool fused = N >= 8192 && c->alpha <= 8;
    if (gt && !fused) return fail(NJ_EUNSUPPORTED, "ModUp through an automorphism needs N >= 8192");
    auto intt = [&](const LimbTab &t) {
        return fused ? launch_intt_scaled(c, M.coef, d, t, c->d_upscale[l], s, gt, l + 1)
                     : launch_ntt(c, M.coef, t, true, s, d);
    };
    if (dstride < 0) dstride = l + 1;
    LimbTab lt;
    lt.n = 0;
    for (int z = 0; z < K; z++)
        for (int i = 0; i <= l; i++) {
            lt.pidx[lt.n] = i, lt.off[lt.n] = z * (l + 1) + i, lt.soff[lt.n] = (zoff ? zoff[z] : z * dstride) + i;
            if (++lt.n == NJ_MAX_LIMBS) {
                NJ_HIP(intt(lt));
                lt.n = 0;
            }
        }
    NJ_HIP(intt(lt));
    for (int j0 = 0; j0 < nd; j0 += 4) {
        BconvShared sh;
        sh.nd = std::min(4, nd - j0);
        for (int jj = 0; jj < sh.nd; jj++) {
            const int j = j0 + jj;
            const BconvTab &bt = tabs[j];
            sh.m[jj] = bt.m, sh.n_out[jj] = bt.n_out, sh.in_off0[jj] = j * c->alpha;
            sh.hat_inv[jj] = bt.hat_inv, sh.hat[jj] = bt.hat;
            for (int a = 0; a < bt.m; a++) sh.in_pidx[jj][a] = bt.in_pidx[a];
            for (int o = 0; o < bt.n_out; o++) sh.out_pidx[jj][o] = bt.out_pidx[o], sh.out_off[jj][o] = j * ne + bt.out_limb[o];
        }
        BconvPtrs jp;
        for (int z = 0; z < K; z++) jp.in[z] = M.coef + (size_t)z * (l + 1) * N, jp.out[z] = M.ext + (size_t)z * nd * ne * N;
        NJ_HIP(fused ? launch_bconv_col(c, sh, jp, K, s) : launch_bconv_multi(c, sh, jp, K, s));
    }
    if (fused && !tiles) return NJ_OK;  // the key inner product runs the tile pass
    auto ntt = [&](const LimbTab &t) { return fused ? launch_ntt_tiles(c, M.ext, t, s) : launch_ntt(c, M.ext, t, false, s); };
    lt.n = 0;
    for (int z = 0; z < K; z++)
        for (int j = 0; j < nd; j++) {
            const BconvTab &bt = tabs[j];
            for (int o = 0; o < bt.n_out; o++) {
                lt.pidx[lt.n] = bt.out_pidx[o];
                lt.off[lt.n] = (z * nd + j) * ne + bt.out_limb[o];
                if (++lt.n == NJ_MAX_LIMBS) {
                    NJ_HIP(ntt(lt));
                    lt.n = 0;
                }
            }
        }
    NJ_HIP(ntt(lt));
    return NJ_OK;
}

// K key switches from already-extended digits: inner products, ModDown, combine.
// sum = 0: job z writes mj.out[z]; sum = 1: mj.out[0] = acc + sum of all jobs.
nj_status ks_down(nj_ctx *c, int l, int K, const MdJobs &mj, int sum, const uint64_t *acc, MultiBufs &M,
                  hipStream_t s, bool p_tiled, uint64_t *last_out, const MdConj *conj, bool drop, const KeyJobs *ipq);

nj_status ks_multi(nj_ctx *c, int l, int K, const KeyJobs &kj, const MdJobs &mj, int sum, const uint64_t *acc,
                   MultiBufs &M, hipStream_t s)
{
    if (fuse_ip(c, l)) {  // special-prime rows straight into ModDown's inverse tile pass
        NJ_HIP(launch_key_ip_ptile(c, l, kj, K, M.pc, s));
        if (!sum && !acc)  // the Q limbs' products inside the ModDown combine
            return ks_down(c, l, K, mj, 0, nullptr, M, s, true, nullptr, nullptr, false, &kj);
        NJ_HIP(launch_key_ip_multi(c, l, kj, K, M.u, s, l + 1));
        return ks_down(c, l, K, mj, sum, acc, M, s, true);
    }
    NJ_HIP(launch_key_ip_multi(c, l, kj, K, M.u, s));
    return ks_down(c, l, K, mj, sum, acc, M, s);
}

// ModDown of K jobs' inner products (M.u) and the combine into their outputs (ipq: the
// Q limbs' inner products are computed inside the combine from these jobs' extended
// evaluation-form digits instead of read from M.u; plain combine only).
nj_status ks_down(nj_ctx *c, int l, int K, const MdJobs &mj, int sum, const uint64_t *acc, MultiBufs &M,
                  hipStream_t s, bool p_tiled, uint64_t *last_out, const MdConj *conj, bool drop, const KeyJobs *ipq)
{
    const int N = c->N, ne = l + 1 + c->alpha, al = c->alpha;
    const bool fused = N >= 8192 && al <= 8;  // as in modup_multi
    if (p_tiled && !fused) return fail(NJ_EUNSUPPORTED, "ModDown: pre-transformed special-prime rows need N >= 8192");
    const bool one = !sum && N >= 4096 && K == 1;  // the fused combine of one job
    if (drop && (sum || !fused || last_out || conj || l < 2))
        return fail(NJ_EUNSUPPORTED, "ModDown: limbs 0 and l only with the fused combine, no hand-off, level >= 2");
    if (last_out && !(one && fused)) return fail(NJ_EUNSUPPORTED, "ModDown: the rescale hand-off needs one job, N >= 8192");
    if (ipq && (sum || acc || last_out || conj || drop || !fused || !fuse_ip(c, l)))
        return fail(NJ_EUNSUPPORTED, "ModDown: inner products in the combine need the plain fused combine");
    if (conj && !one) return fail(NJ_EUNSUPPORTED, "ModDown: the fused split needs one job, N >= 4096");
    // one job with a previous value held elsewhere: the fused combine reads it there
    const uint64_t *acc0 = one && acc && acc != mj.out[0] ? acc : nullptr;
    if (acc && !sum && K == 1 && acc != mj.out[0] && !one)
        NJ_HIP(hipMemcpyAsync(mj.out[0], acc, 2 * (size_t)(l + 1) * N * 8, hipMemcpyDeviceToDevice, s));
    auto intt = [&](const LimbTab &t) {
        if (p_tiled) return launch_intt_cols_scaled(c, M.pc, t, c->d_downscale, s);
        return fused ? launch_intt_scaled(c, M.pc, M.u, t, c->d_downscale, s) : launch_ntt(c, M.pc, t, true, s, M.u);
    };
    LimbTab lp;
    lp.n = 0;
    for (int z = 0; z < K; z++)
        for (int p = 0; p < 2; p++)
            for (int a = 0; a < al; a++) {
                lp.pidx[lp.n] = c->n_q + a, lp.off[lp.n] = (2 * z + p) * al + a;
                lp.soff[lp.n] = (2 * z + p) * ne + l + 1 + a;
                if (++lp.n == NJ_MAX_LIMBS) {
                    NJ_HIP(intt(lp));
                    lp.n = 0;
                }
            }
    NJ_HIP(intt(lp));
    const BconvTab &bt = drop ? c->moddown_drop[l] : c->moddown[l];
    BconvShared sh;
    sh.nd = 1;
    sh.m[0] = bt.m, sh.n_out[0] = bt.n_out, sh.in_off0[0] = 0, sh.hat_inv[0] = bt.hat_inv, sh.hat[0] = bt.hat;
    for (int a = 0; a < bt.m; a++) sh.in_pidx[0][a] = bt.in_pidx[a];
    for (int o = 0; o < bt.n_out; o++) sh.out_pidx[0][o] = bt.out_pidx[o], sh.out_off[0][o] = bt.out_limb[o];
    BconvPtrs jp;
    for (int h = 0; h < 2 * K; h++) jp.in[h] = M.pc + (size_t)h * al * N, jp.out[h] = M.conv + (size_t)h * (l + 1) * N;
    NJ_HIP(fused ? launch_bconv_col(c, sh, jp, 2 * K, s) : launch_bconv_multi(c, sh, jp, 2 * K, s));
    if (ipq) {
        NJ_HIP(launch_key_ip_moddown(c, l, K, M.conv, *ipq, mj, s));
        return NJ_OK;
    }
    if (!sum && N >= 4096) {  // the combine runs inside the transform's tile pass
        NJ_HIP(launch_ntt_moddown(c, l, K, M.conv, M.u, mj, acc != nullptr, fused, s, acc0, last_out, conj,
                                  drop ? l - 1 : 0));
        return NJ_OK;
    }
    auto ntt = [&](const LimbTab &t) { return fused ? launch_ntt_tiles(c, M.conv, t, s) : launch_ntt(c, M.conv, t, false, s); };
    LimbTab lq;
    lq.n = 0;
    for (int h = 0; h < 2 * K; h++)
        for (int i = 0; i <= l; i++) {
            lq.pidx[lq.n] = i, lq.off[lq.n] = h * (l + 1) + i;
            if (++lq.n == NJ_MAX_LIMBS) {
                NJ_HIP(ntt(lq));
                lq.n = 0;
            }
        }
    NJ_HIP(ntt(lq));
    NJ_HIP(launch_moddown_multi(c, l, mj, K, sum, M.u, M.conv, acc, s));
    return NJ_OK;
}

// Multiply-accumulate of one ciphertext's BSGS transform in passes of at most 16 giant
// x 16 baby steps (later baby passes accumulate): inner_g = sum over entries (g, b, dg)
// of diag_dg (.) baby_b.  With no babies the giant steps' inner sums are zero.
nj_status mac_general(nj_ctx *c, int l, const std::vector<const uint64_t *> &baby, int ng,
                      const std::vector<MacEntry> &ent, const uint64_t *diag, int dl, uint64_t *inner, hipStream_t s)
{
    const size_t clen = 2 * (size_t)c->N * (l + 1);
    const int nb = (int)baby.size();
    if (nb == 0 || ent.empty()) {  // every diagonal zero: every inner sum is the zero ciphertext
        if (ng > 0) NJ_HIP(launch_zero(c, inner, (size_t)ng * clen, s));
        return NJ_OK;
    }
    for (int g0 = 0; g0 < ng; g0 += NJ_MAX_GIANT) {
        const int gn = std::min(NJ_MAX_GIANT, ng - g0);
        for (int b0 = 0; b0 == 0 || b0 < nb; b0 += NJ_MAX_BABY) {
            MacPlan mp;
            mp.nb = std::max(0, std::min(NJ_MAX_BABY, nb - b0)), mp.ng = gn, mp.dl = dl;
            for (int b = 0; b < mp.nb; b++) mp.baby[b] = baby[b0 + b];
            for (int g = 0; g < NJ_MAX_GIANT; g++)
                for (int b = 0; b < NJ_MAX_BABY; b++) mp.d_of[g][b] = -1;
            int used = 0;
            for (const MacEntry &e : ent)
                if (e.g >= g0 && e.g < g0 + gn && e.b >= b0 && e.b < b0 + mp.nb) mp.d_of[e.g - g0][e.b - b0] = e.dg, used++;
            NJ_HIP(launch_bsgs_mac(c, l, mp, diag, inner + g0 * clen, used, s, b0 > 0));
        }
    }
    return NJ_OK;
}

// key switches batched per launch in a BSGS transform (baby steps, or a chunk of giant steps)
int bsgs_jobs(const nj_lt_t &lt)
{
    return std::min(kGiantChunk, std::max(1, std::max((int)lt.babies.size() - 1, (int)lt.giants.size())));
}

size_t bsgs_words(const nj_ctx *c, const nj_lt_t &lt)
{
    const size_t N = c->N, l = lt.level, ne = l + 1 + c->alpha;
    return N * 2 * (l + 1) * (lt.babies.size() + lt.giants.size()) + multi_words(c, l, bsgs_jobs(lt)) +
           (lt.lazy ? N * (2 * ne + l + 1) : 0);
}

// sum_d diag_d (.) (in <<< j_d u), baby-step giant-step; out must not alias in.
nj_status bsgs_apply(nj_ctx *c, const nj_lt_t &lt, const uint64_t *in, uint64_t *out, int hoist, Arena A,
                     hipStream_t s, uint64_t *last_out, bool *last_done, bool drop)
{
    if (last_done) *last_done = false;
    const int l = lt.level, n = c->N / 2;
    const size_t N = c->N, clen = 2 * N * (l + 1);
    const int nb = (int)lt.babies.size(), ng = (int)lt.giants.size();
    std::vector<const uint64_t *> baby(nb);
    std::vector<uint64_t *> baby_buf(nb);
    for (int b = 0; b < nb; b++) baby_buf[b] = A.take(clen);
    uint64_t *inner = A.take(clen * ng);
    if (!inner) return fail(NJ_ENOMEM, "scratch too small");
    for (size_t b = 0; b < lt.babies.size(); b++)
        if (lt.babies[b] != 0 && !key_of(c, galois_of_rot(c, (long long)lt.babies[b] * lt.u)))
            return fail(NJ_ENOKEY, "missing baby-step rotation key");
    for (int gg : lt.giants)
        if (gg != 0 && !key_of(c, galois_of_rot(c, (long long)gg * lt.n1 * lt.u)))
            return fail(NJ_ENOKEY, "missing giant-step rotation key");
    MultiBufs M;
    if (!multi_bufs(c, l, bsgs_jobs(lt), A, M)) return fail(NJ_ENOMEM, "scratch too small");
    const size_t nd = n_digits(c, l), ne = l + 1 + c->alpha, plen = N * (l + 1);
    // baby steps: the input's rotations as batches of key switches
    std::vector<int> todo;
    for (int b = 0; b < nb; b++) {
        baby[b] = lt.babies[b] == 0 ? in : baby_buf[b];
        if (lt.babies[b] != 0) todo.push_back(b);
    }
    nj_status st;
    if (hoist && !todo.empty() && (st = modup_multi(c, l, 1, in + plen, M, s))) return st;
    for (size_t c0 = 0; c0 < todo.size(); c0 += kGiantChunk) {
        const int K = (int)std::min((size_t)kGiantChunk, todo.size() - c0);
        KeyJobs kj;
        MdJobs mj;
        AutoJobs aj;
        GalTab gt;
        for (int z = 0; z < K; z++) {
            const int b = todo[c0 + z];
            const uint32_t g = galois_of_rot(c, (long long)lt.babies[b] * lt.u);
            if (hoist) {  // one ModUp of c1; X -> X^g applied to the extended digits
                kj.ext[z] = M.ext, kj.d[z] = in + plen, kj.g[z] = g;
            } else if (fuse_ip(c, l)) {  // ModUp of each tau_g(c1), read through X -> X^g
                gt.g[z] = g;
                kj.ext[z] = M.ext + (size_t)z * nd * ne * N, kj.d[z] = in + plen, kj.g[z] = g;
            } else {  // ModUp of each tau_g(c1)
                aj.in[z] = in + plen, aj.out[z] = M.d + (size_t)z * plen, aj.g[z] = g;
                kj.ext[z] = M.ext + (size_t)z * nd * ne * N, kj.d[z] = M.d + (size_t)z * plen, kj.g[z] = 1;
            }
            kj.key[z] = key_of(c, g);
            mj.add[z] = in, mj.g_add[z] = g, mj.out[z] = baby_buf[b];
        }
        if (!hoist && fuse_ip(c, l)) {
            if ((st = modup_multi(c, l, K, in + plen, M, s, 0, false, &gt))) return st;
        } else if (!hoist) {
            NJ_HIP(launch_automorph_multi(c, aj, K, l + 1, s));
            if ((st = modup_multi(c, l, K, M.d, M, s))) return st;
        }
        st = !hoist && fuse_ip(c, l) ? ks_fused(c, l, K, kj, mj, 0, nullptr, M, s) : ks_multi(c, l, K, kj, mj, 0, nullptr, M, s);
        if (st) return st;
    }
    // every giant step's inner sum
    std::vector<MacEntry> ent;
    for (int d = 0; d < lt.n_diag; d++)
        if (lt.nz.empty() || lt.nz[d])
            ent.push_back(MacEntry{
                (int)(std::lower_bound(lt.giants.begin(), lt.giants.end(), lt.g_of[d]) - lt.giants.begin()),
                (int)(std::lower_bound(lt.babies.begin(), lt.babies.end(), lt.i_of[d]) - lt.babies.begin()), d});
    if ((st = mac_general(c, l, baby, ng, ent, lt.d_diag, lt.dl, inner, s))) return st;
    // out = inner_0 + sum_g rot(inner_g, g n1 u): the rotations run as batches of key
    // switches whose ModDown combine also sums them (exact modular sums)
    const uint64_t *acc = nullptr;
    for (int g = 0; g < ng; g++)
        if (lt.giants[g] == 0) acc = inner + (size_t)g * clen;
    std::vector<int> gl;
    for (int g = 0; g < ng; g++)
        if (lt.giants[g] != 0) gl.push_back(g);
    if (gl.empty()) {
        if (acc) NJ_HIP(hipMemcpyAsync(out, acc, clen * 8, hipMemcpyDeviceToDevice, s));
        return NJ_OK;
    }
    if (lt.lazy) {  // key inner products summed over Q_l u P, one ModDown
        uint64_t *usum = A.take(2 * ne * N), *c0sum = A.take(plen);
        if (!c0sum) return fail(NJ_ENOMEM, "scratch too small");
        // drop: the output goes on to a rescale and a drop to level 0, which read only its
        // Q limbs 0 and l; the giant steps' digits, inner products, c0 sums and ModDown
        // are computed for those limbs (and the special primes) alone
        const bool dr = drop && fuse_ip(c, l) && l >= 2 && !last_out;
        const int skip = dr ? l - 1 : 0;
        for (size_t c0 = 0; c0 < gl.size(); c0 += kGiantChunk) {
            const int K = (int)std::min((size_t)kGiantChunk, gl.size() - c0);
            const bool f = fuse_ip(c, l);  // fused: tau_ge rides on ModUp and the own-limb reads
            KeyJobs kj;
            AutoJobs aj, ac;
            GalTab gt;
            int zoff[NJ_MAX_JOBS];  // limb offset of each giant's c1 from inner + plen
            for (int z = 0; z < K; z++) {
                const int g = gl[c0 + z];
                const uint32_t ge = galois_of_rot(c, (long long)lt.giants[g] * lt.n1 * lt.u);
                const uint64_t *x = inner + (size_t)g * clen;
                aj.in[z] = x + plen, aj.out[z] = M.d + (size_t)z * plen, aj.g[z] = ge;
                ac.in[z] = x, ac.out[z] = nullptr, ac.g[z] = ge;
                kj.ext[z] = M.ext + (size_t)z * nd * ne * N, kj.d[z] = M.d + (size_t)z * plen, kj.g[z] = 1;
                if (f) kj.d[z] = x + plen, kj.g[z] = ge, gt.g[z] = ge, zoff[z] = g * 2 * (l + 1);
                kj.key[z] = key_of(c, ge);
            }
            if (f) {
                if ((st = modup_multi(c, l, K, inner + plen, M, s, -1, false, &gt, zoff, dr))) return st;
            } else {
                NJ_HIP(launch_automorph_multi(c, aj, K, l + 1, s));
                if ((st = modup_multi(c, l, K, M.d, M, s, -1, !f))) return st;
            }
            const bool last = c0 + K == gl.size();  // its special-prime rows go on to ModDown's inverse transform
            NJ_HIP(f ? launch_ntt_ip(c, l, kj, K, usum, 1, c0 ? 1 : 0, s, last ? M.pc : nullptr, skip)
                     : launch_key_ip_sum(c, l, kj, K, usum, c0 ? 1 : 0, s));
            NJ_HIP(launch_automorph_acc(c, ac, K, l + 1, c0sum, 0, c0 ? 3 : 2, s, skip));
        }
        MultiBufs M1 = M;
        M1.u = usum;
        MdJobs mj;
        mj.add[0] = c0sum, mj.g_add[0] = 1, mj.out[0] = out;
        const bool hand = last_out && N >= 8192 && c->alpha <= 8;  // the rescale's first pass rides along
        if (hand && last_done) *last_done = true;
        return ks_down(c, l, 1, mj, 0, acc, M1, s, fuse_ip(c, l), hand ? last_out : nullptr, nullptr, dr);
    }
    for (size_t c0 = 0; c0 < gl.size(); c0 += kGiantChunk) {
        const int K = (int)std::min((size_t)kGiantChunk, gl.size() - c0);
        const bool f = fuse_ip(c, l);  // fused: tau_ge rides on ModUp and the own-limb reads
        KeyJobs kj;
        MdJobs mj;
        AutoJobs aj;
        GalTab gt;
        int zoff[NJ_MAX_JOBS];
        for (int z = 0; z < K; z++) {
            const int g = gl[c0 + z];
            const uint32_t ge = galois_of_rot(c, (long long)lt.giants[g] * lt.n1 * lt.u);
            const uint64_t *x = inner + (size_t)g * clen;
            aj.in[z] = x + plen, aj.out[z] = M.d + (size_t)z * plen, aj.g[z] = ge;
            kj.ext[z] = M.ext + (size_t)z * nd * ne * N, kj.d[z] = M.d + (size_t)z * plen, kj.g[z] = 1;
            if (f) kj.d[z] = x + plen, kj.g[z] = ge, gt.g[z] = ge, zoff[z] = g * 2 * (l + 1);
            kj.key[z] = key_of(c, ge);
            mj.add[z] = x, mj.g_add[z] = ge;
        }
        mj.out[0] = out;
        if (f) {
            if ((st = modup_multi(c, l, K, inner + plen, M, s, -1, false, &gt, zoff))) return st;
        } else {
            NJ_HIP(launch_automorph_multi(c, aj, K, l + 1, s));
            if ((st = modup_multi(c, l, K, M.d, M, s, -1, !f))) return st;
        }
        st = f ? ks_fused(c, l, K, kj, mj, 1, acc, M, s) : ks_multi(c, l, K, kj, mj, 1, acc, M, s);
        if (st) return st;
        acc = out;
    }
    (void)n;
    return NJ_OK;
}

// ------------------------------------------------------------ batched execution
//
// K ciphertexts (contiguous, [K][2][l+1][N]) through one BSGS transform: every key
// and every diagonal word is read once for the whole batch.  Baby steps hoisted.

// the multi-ciphertext multiply-accumulate holds at most 16 x 16 steps; larger splits
// run the transform one ciphertext at a time
bool batch_mac_fits(const nj_lt_t &lt) { return lt.babies.size() <= NJ_MAX_BABY && lt.giants.size() <= NJ_MAX_GIANT; }

size_t bsgs_batch_words(const nj_ctx *c, const nj_lt_t &lt, int K)
{
    const size_t N = c->N, l = lt.level, clen = 2 * N * (l + 1);
    if (!batch_mac_fits(lt)) return bsgs_words(c, lt);
    return clen * K * (lt.babies.size() + lt.giants.size()) + multi_words(c, l, K) +
           (lt.lazy ? N * K * (2 * (l + 1 + c->alpha) + l + 1) : 0);
}

nj_status bsgs_apply_batch(nj_ctx *c, const nj_lt_t &lt, int K, const uint64_t *in, uint64_t *out, Arena A,
                           hipStream_t s)
{
    const int l = lt.level;
    const size_t N = c->N, clen = 2 * N * (l + 1), plen = N * (l + 1);
    const int nb = (int)lt.babies.size(), ng = (int)lt.giants.size();
    if (K < 1 || K > NJ_MAX_JOBS) return fail(NJ_EINVAL, "batch size out of range");
    if (!batch_mac_fits(lt)) {
        for (int z = 0; z < K; z++) {
            nj_status st = bsgs_apply(c, lt, in + z * clen, out + z * clen, 1, A, s);
            if (st) return st;
        }
        return NJ_OK;
    }
    for (int b : lt.babies)
        if (b != 0 && !key_of(c, galois_of_rot(c, (long long)b * lt.u))) return fail(NJ_ENOKEY, "missing baby-step key");
    for (int g : lt.giants)
        if (g != 0 && !key_of(c, galois_of_rot(c, (long long)g * lt.n1 * lt.u)))
            return fail(NJ_ENOKEY, "missing giant-step key");
    uint64_t *baby_all = A.take(clen * K * nb);   // [nb][K][clen], slot 0 unused (the input is baby 0)
    uint64_t *inner_all = A.take(clen * K * ng);  // [K][ng][clen]
    MultiBufs M;
    if (!inner_all || !multi_bufs(c, l, K, A, M)) return fail(NJ_ENOMEM, "scratch too small");
    const size_t nd = n_digits(c, l), ne = l + 1 + c->alpha;
    nj_status st;
    // baby steps: one ModUp per ciphertext, then one shared-key inner product per rotation
    if (nb > 1 && (st = modup_multi(c, l, K, in + plen, M, s, 2 * (l + 1)))) return st;
    for (int b = 0; b < nb; b++) {
        if (lt.babies[b] == 0) continue;
        const uint32_t g = galois_of_rot(c, (long long)lt.babies[b] * lt.u);
        KeyJobs kj;
        MdJobs mj;
        for (int z = 0; z < K; z++) {
            kj.ext[z] = M.ext + (size_t)z * nd * ne * N, kj.d[z] = in + z * clen + plen, kj.g[z] = g;
            mj.add[z] = in + z * clen, mj.g_add[z] = g, mj.out[z] = baby_all + ((size_t)b * K + z) * clen;
        }
        NJ_HIP(launch_key_ip_shared(c, l, kj, K, key_of(c, g), M.u, s));
        if ((st = ks_down(c, l, K, mj, 0, nullptr, M, s))) return st;
    }
    // inner sums of every giant step of every ciphertext
    MacPlan mp;
    mp.nb = nb, mp.ng = ng, mp.dl = lt.dl;
    for (int b = 0; b < nb; b++) mp.baby[b] = lt.babies[b] == 0 ? in : baby_all + (size_t)b * K * clen;
    for (int g = 0; g < NJ_MAX_GIANT; g++)
        for (int b = 0; b < NJ_MAX_BABY; b++) mp.d_of[g][b] = -1;
    for (int d = 0; d < lt.n_diag; d++) {
        const int g = (int)(std::lower_bound(lt.giants.begin(), lt.giants.end(), lt.g_of[d]) - lt.giants.begin());
        const int b = (int)(std::lower_bound(lt.babies.begin(), lt.babies.end(), lt.i_of[d]) - lt.babies.begin());
        mp.d_of[g][b] = d;
    }
    NJ_HIP(launch_bsgs_mac_multi(c, l, mp, K, clen, ng * clen, lt.d_diag, inner_all, lt.n_diag, s));
    // giant steps: out_z = inner_{z,0} + sum_g rot(inner_{z,g})
    bool have = false;
    for (int g = 0; g < ng; g++)
        if (lt.giants[g] == 0) {
            NJ_HIP(hipMemcpy2DAsync(out, clen * 8, inner_all + (size_t)g * clen, ng * clen * 8, clen * 8, K,
                                    hipMemcpyDeviceToDevice, s));
            have = true;
        }
    uint64_t *usum = nullptr, *c0sum = nullptr;
    if (lt.lazy) {
        usum = A.take(N * K * 2 * ne), c0sum = A.take(N * K * (l + 1));
        if (!c0sum) return fail(NJ_ENOMEM, "scratch too small");
    }
    // fused (N >= 8192): tau_ge rides on ModUp's inverse transform and on the own-limb
    // reads, and the key inner product (one key, one job per ciphertext) runs the digits'
    // tile pass; the last giant step's special-prime rows go on to ModDown's inverse
    // transform there
    const bool f = fuse_ip(c, l);
    int g_last = -1;
    for (int g = 0; g < ng; g++)
        if (lt.giants[g] != 0) g_last = g;
    bool first = true;
    for (int g = 0; g < ng; g++) {
        if (lt.giants[g] == 0) continue;
        const uint32_t ge = galois_of_rot(c, (long long)lt.giants[g] * lt.n1 * lt.u);
        AutoJobs aj, ac;
        KeyJobs kj;
        MdJobs mj;
        GalTab gt;
        int zoff[NJ_MAX_JOBS];  // limb offset of each ciphertext's c1 of this giant step from inner_all + plen
        for (int z = 0; z < K; z++) {
            const uint64_t *x = inner_all + ((size_t)z * ng + g) * clen;
            aj.in[z] = x + plen, aj.out[z] = M.d + (size_t)z * plen, aj.g[z] = ge;
            ac.in[z] = x, ac.out[z] = nullptr, ac.g[z] = ge;
            kj.ext[z] = M.ext + (size_t)z * nd * ne * N, kj.d[z] = M.d + (size_t)z * plen, kj.g[z] = 1;
            kj.key[z] = key_of(c, ge);
            if (f) kj.d[z] = x + plen, kj.g[z] = ge, gt.g[z] = ge, zoff[z] = (z * ng + g) * 2 * (l + 1);
            mj.add[z] = x, mj.g_add[z] = ge, mj.out[z] = out + z * clen;
        }
        if (f) {
            if ((st = modup_multi(c, l, K, inner_all + plen, M, s, -1, false, &gt, zoff))) return st;
        } else {
            NJ_HIP(launch_automorph_multi(c, aj, K, l + 1, s));
            if ((st = modup_multi(c, l, K, M.d, M, s))) return st;
        }
        if (lt.lazy) {  // per ciphertext: inner products and rotated c0 parts summed
            if (f)
                NJ_HIP(launch_ntt_ip(c, l, kj, K, usum, 0, first ? 0 : 1, s, g == g_last ? M.pc : nullptr));
            else
                NJ_HIP(launch_key_ip_shared(c, l, kj, K, key_of(c, ge), usum, s, first ? 0 : 1));
            NJ_HIP(launch_automorph_acc(c, ac, K, l + 1, c0sum, plen, first ? 0 : 1, s));
            first = false;
            continue;
        }
        if (f) {
            if ((st = ks_fused(c, l, K, kj, mj, 0, have ? out : nullptr, M, s))) return st;
        } else {
            NJ_HIP(launch_key_ip_shared(c, l, kj, K, key_of(c, ge), M.u, s));
            if ((st = ks_down(c, l, K, mj, 0, have ? out : nullptr, M, s))) return st;
        }
        have = true;
    }
    if (lt.lazy && !first) {  // one ModDown per ciphertext
        MultiBufs M1 = M;
        M1.u = usum;
        MdJobs mj;
        for (int z = 0; z < K; z++) mj.add[z] = c0sum + z * plen, mj.g_add[z] = 1, mj.out[z] = out + z * clen;
        if ((st = ks_down(c, l, K, mj, 0, have ? out : nullptr, M1, s, f))) return st;
    }
    return NJ_OK;
}

// K key switches tau_g of contiguous ciphertexts [K][2][l+1] sharing one key
nj_status apply_galois_batch(nj_ctx *c, int l, int K, const uint64_t *in, uint32_t g, uint64_t *out, Arena A,
                             hipStream_t s)
{
    if (g % 2 == 0 || g >= 2u * (uint32_t)c->N) return fail(NJ_EINVAL, "Galois element must be odd and below 2N");
    if (g == 1) {  // the identity, as in apply_galois
        if (out != in)
            NJ_HIP(hipMemcpyAsync(out, in, (size_t)K * 2 * c->N * (l + 1) * 8, hipMemcpyDeviceToDevice, s));
        return NJ_OK;
    }
    const uint64_t *key = key_of(c, g);
    if (!key) return fail(NJ_ENOKEY, "no switching key for Galois element " + std::to_string(g));
    if (K < 1 || K > NJ_MAX_JOBS) return fail(NJ_EINVAL, "batch size out of range");
    if (in == out) return fail(NJ_EINVAL, "batched key switching needs separate input and output");
    const size_t N = c->N, clen = 2 * N * (l + 1), plen = N * (l + 1), nd = n_digits(c, l), ne = l + 1 + c->alpha;
    MultiBufs M;
    if (!multi_bufs(c, l, K, A, M)) return fail(NJ_ENOMEM, "scratch too small");
    AutoJobs aj;
    KeyJobs kj;
    MdJobs mj;
    for (int z = 0; z < K; z++) {
        aj.in[z] = in + z * clen + plen, aj.out[z] = M.d + (size_t)z * plen, aj.g[z] = g;
        kj.ext[z] = M.ext + (size_t)z * nd * ne * N, kj.d[z] = M.d + (size_t)z * plen, kj.g[z] = 1;
        mj.add[z] = in + z * clen, mj.g_add[z] = g, mj.out[z] = out + z * clen;
    }
    NJ_HIP(launch_automorph_multi(c, aj, K, l + 1, s));
    nj_status st = modup_multi(c, l, K, M.d, M, s);
    if (st) return st;
    NJ_HIP(launch_key_ip_shared(c, l, kj, K, key, M.u, s));
    return ks_down(c, l, K, mj, 0, nullptr, M, s);
}

// a transform applied at ciphertext level l <= its plan's: same diagonals (their first
// l+1 limbs are the residues of the same integer plaintexts), keys serve every level
nj_lt_t at_level(const nj_lt_t &lt, int l)
{
    nj_lt_t a = lt;
    a.level = l;
    return a;
}

// ------------------------------------------------------------------ block conv
//
// Block matrix-vector product of a blocked conv (Sec. 3.3.4): bi input ciphertexts
// [bi][2][l+1][N] -> bo outputs [bo][2][l+1][N], out_ob = sum_ib K^(ob,ib) in_ib.
// Baby steps are hoisted once per input (shared-key inner products over the inputs),
// each output block's giant-step inner sums run over all its nonzero input blocks in
// multiply-accumulate passes of at most 16 babies, and each giant rotation is one
// shared-key key switch over the output blocks, accumulated into the outputs.
size_t block_words(const nj_ctx *c, const nj_lt_t &lt)
{
    const size_t N = c->N, l = lt.level, clen = 2 * N * (l + 1);
    const int K = std::min(std::max(lt.bi, lt.bo), kBatch);
    return clen * (lt.bi * lt.babies.size() + lt.bo * lt.giants.size()) + multi_words(c, l, K);
}

nj_status block_bsgs_apply(nj_ctx *c, const nj_lt_t &lt, const uint64_t *in, uint64_t *out, Arena A, hipStream_t s)
{
    if (lt.lazy) return fail(NJ_EUNSUPPORTED, "block transforms run giant steps with one ModDown each");
    const int l = lt.level, bi = lt.bi, bo = lt.bo, nd = lt.n_diag;
    const size_t N = c->N, clen = 2 * N * (l + 1), plen = N * (l + 1);
    const int nb = (int)lt.babies.size(), ng = (int)lt.giants.size();
    for (int b : lt.babies)
        if (b != 0 && !key_of(c, galois_of_rot(c, (long long)b * lt.u))) return fail(NJ_ENOKEY, "missing baby-step key");
    for (int g : lt.giants)
        if (g != 0 && !key_of(c, galois_of_rot(c, (long long)g * lt.n1 * lt.u)))
            return fail(NJ_ENOKEY, "missing giant-step key");
    uint64_t *baby_all = A.take(clen * bi * nb);   // [nb][bi][clen], baby 0 is the input itself
    uint64_t *inner_all = A.take(clen * bo * ng);  // [bo][ng][clen]
    MultiBufs M;
    if (!baby_all || !inner_all || !multi_bufs(c, l, std::min(std::max(bi, bo), kBatch), A, M))
        return fail(NJ_ENOMEM, "scratch too small");
    const size_t ndig = n_digits(c, l), ne = l + 1 + c->alpha;
    nj_status st;
    // baby steps of every input, kBatch inputs per ModUp
    for (int z0 = 0; nb > 1 && z0 < bi; z0 += kBatch) {
        const int K = std::min(kBatch, bi - z0);
        const uint64_t *x = in + z0 * clen;
        if ((st = modup_multi(c, l, K, x + plen, M, s, 2 * (l + 1)))) return st;
        for (int b = 0; b < nb; b++) {
            if (lt.babies[b] == 0) continue;
            const uint32_t g = galois_of_rot(c, (long long)lt.babies[b] * lt.u);
            KeyJobs kj;
            MdJobs mj;
            for (int z = 0; z < K; z++) {
                kj.ext[z] = M.ext + (size_t)z * ndig * ne * N, kj.d[z] = x + z * clen + plen, kj.g[z] = g;
                mj.add[z] = x + z * clen, mj.g_add[z] = g, mj.out[z] = baby_all + ((size_t)b * bi + z0 + z) * clen;
            }
            NJ_HIP(launch_key_ip_shared(c, l, kj, K, key_of(c, g), M.u, s));
            if ((st = ks_down(c, l, K, mj, 0, nullptr, M, s))) return st;
        }
    }
    // inner sums: output block ob, giant g = sum over (ib, baby) of diag (.) baby
    std::vector<int> gidx(nd), bidx(nd);
    for (int d = 0; d < nd; d++) {
        gidx[d] = (int)(std::lower_bound(lt.giants.begin(), lt.giants.end(), lt.g_of[d]) - lt.giants.begin());
        bidx[d] = (int)(std::lower_bound(lt.babies.begin(), lt.babies.end(), lt.i_of[d]) - lt.babies.begin());
    }
    auto nonzero = [&](int ob, int ib, int d) { return lt.nz.empty() || lt.nz[((size_t)ob * bi + ib) * nd + d]; };
    for (int ob = 0; ob < bo; ob++) {
        std::vector<int> ibs;
        for (int ib = 0; ib < bi; ib++)
            for (int d = 0; d < nd; d++)
                if (nonzero(ob, ib, d)) {
                    ibs.push_back(ib);
                    break;
                }
        const uint64_t *dbase = lt.d_diag + (size_t)ob * bi * nd * lt.dl * N;
        uint64_t *inner = inner_all + (size_t)ob * ng * clen;
        std::vector<const uint64_t *> bs;
        std::vector<MacEntry> ent;
        for (int ib : ibs) {
            const int b0 = (int)bs.size();
            for (int b = 0; b < nb; b++)
                bs.push_back(lt.babies[b] == 0 ? in + ib * clen : baby_all + ((size_t)b * bi + ib) * clen);
            for (int d = 0; d < nd; d++)
                if (nonzero(ob, ib, d)) ent.push_back(MacEntry{gidx[d], b0 + bidx[d], ib * nd + d});
        }
        if ((st = mac_general(c, l, bs, ng, ent, dbase, lt.dl, inner, s))) return st;
    }
    // giant steps
    bool have = false;
    for (int g = 0; g < ng; g++)
        if (lt.giants[g] == 0) {
            NJ_HIP(hipMemcpy2DAsync(out, clen * 8, inner_all + (size_t)g * clen, ng * clen * 8, clen * 8, bo,
                                    hipMemcpyDeviceToDevice, s));
            have = true;
        }
    for (int g = 0; g < ng; g++) {
        if (lt.giants[g] == 0) continue;
        const uint32_t ge = galois_of_rot(c, (long long)lt.giants[g] * lt.n1 * lt.u);
        for (int z0 = 0; z0 < bo; z0 += kBatch) {
            const int K = std::min(kBatch, bo - z0);
            AutoJobs aj;
            KeyJobs kj;
            MdJobs mj;
            for (int z = 0; z < K; z++) {
                const uint64_t *x = inner_all + ((size_t)(z0 + z) * ng + g) * clen;
                aj.in[z] = x + plen, aj.out[z] = M.d + (size_t)z * plen, aj.g[z] = ge;
                kj.ext[z] = M.ext + (size_t)z * ndig * ne * N, kj.d[z] = M.d + (size_t)z * plen, kj.g[z] = 1;
                mj.add[z] = x, mj.g_add[z] = ge, mj.out[z] = out + (z0 + z) * clen;
            }
            NJ_HIP(launch_automorph_multi(c, aj, K, l + 1, s));
            if ((st = modup_multi(c, l, K, M.d, M, s))) return st;
            NJ_HIP(launch_key_ip_shared(c, l, kj, K, key_of(c, ge), M.u, s));
            if ((st = ks_down(c, l, K, mj, 0, have ? out : nullptr, M, s))) return st;
        }
        have = true;
    }
    return NJ_OK;
}

// rescale of a ciphertext [2][l+1] -> [2][l]; out must not alias in
nj_status rescale(nj_ctx *c, int l, const uint64_t *in, uint64_t *out, Arena A, hipStream_t s, int n_out,
                  int n_polys, uint64_t *last_pre)
{
    const size_t N = c->N;
    if (n_out < 0) n_out = l;
    if (last_pre && (N < 8192 || n_polys != 2)) return fail(NJ_EUNSUPPORTED, "rescale: hand-off needs N >= 8192");
    if (N >= 8192) {  // the lifted limbs stay in out, transformed and combined in place
        uint64_t *last = last_pre ? last_pre : A.take(n_polys * N);
        if (!last) return fail(NJ_ENOMEM, "scratch too small");
        NJ_HIP(launch_rescale_fused(c, l, in, out, n_out, last, out, s, n_polys, last_pre != nullptr));
        return NJ_OK;
    }
    if (n_polys != 2) return fail(NJ_EUNSUPPORTED, "rescale: packed ciphertexts need N >= 8192");
    uint64_t *last = A.take(2 * N), *lifted = A.take(N * l);
    if (!lifted) return fail(NJ_ENOMEM, "scratch too small");
    for (int p = 0; p < 2; p++)
        NJ_HIP(hipMemcpyAsync(last + p * N, in + ((size_t)p * (l + 1) + l) * N, N * 8, hipMemcpyDeviceToDevice, s));
    LimbTab lt;
    lt.n = 2;
    lt.pidx[0] = lt.pidx[1] = l;
    lt.off[0] = 0, lt.off[1] = 1;
    NJ_HIP(launch_ntt(c, last, lt, true, s));
    for (int p = 0; p < 2; p++) {
        NJ_HIP(launch_lift_last(c, last + p * N, l, n_out, lifted, s));
        NJ_HIP(launch_ntt(c, lifted, limbs_q(n_out - 1), false, s));
        NJ_HIP(launch_rescale_combine(c, l, in + (size_t)p * (l + 1) * N, lifted, out + (size_t)p * n_out * N, s,
                                      n_out));
    }
    return NJ_OK;
}

nj_status rescale_batch(nj_ctx *c, int l, int K, const uint64_t *in, uint64_t *out, Arena A, hipStream_t s)
{
    if (c->N >= 8192) return rescale(c, l, in, out, A, s, -1, 2 * K);
    const size_t cl = 2 * (size_t)c->N * (l + 1), cl1 = 2 * (size_t)c->N * l;
    for (int z = 0; z < K; z++) {
        nj_status st = rescale(c, l, in + z * cl, out + z * cl1, A, s);
        if (st) return st;
    }
    return NJ_OK;
}

nj_status modraise(nj_ctx *c, const uint64_t *in, int top, uint64_t *out, Arena A, hipStream_t s)
{
    const size_t N = c->N;
    uint64_t *tmp = A.take(2 * N);
    if (!tmp) return fail(NJ_ENOMEM, "scratch too small");
    LimbTab lt;
    lt.n = 2;
    lt.pidx[0] = lt.pidx[1] = 0;
    lt.off[0] = 0, lt.off[1] = 1;
    lt.soff[0] = 0, lt.soff[1] = 1;
    NJ_HIP(launch_ntt(c, tmp, lt, true, s, in));  // coefficient form of both level-0 limbs
    LimbTab lo;
    lo.n = 2 * (top + 1);
    for (int k = 0; k < lo.n; k++) lo.pidx[k] = k % (top + 1), lo.off[k] = k;
    if (N >= 8192) {  // lift fused with the column pass, then the tile pass
        NJ_HIP(launch_lift_col(c, tmp, 0, 2, top + 1, out, s));
        NJ_HIP(launch_ntt_tiles(c, out, lo, s));
        return NJ_OK;
    }
    for (int p = 0; p < 2; p++) NJ_HIP(launch_lift_last(c, tmp + p * N, 0, top + 1, out + (size_t)p * (top + 1) * N, s));
    NJ_HIP(launch_ntt(c, out, lo, false, s));
    return NJ_OK;
}

LimbTab ct_limbs(int l)
{
    LimbTab t;
    t.n = 2 * (l + 1);
    for (int k = 0; k < t.n; k++) t.pidx[k] = k % (l + 1), t.off[k] = k;
    return t;
}

nj_status conj_split(nj_ctx *c, int l, const uint64_t *x, uint64_t *re, uint64_t *im, Arena A, hipStream_t s)
{
    const size_t clen = 2 * (size_t)c->N * (l + 1);
    if (fuse_ip(c, l)) {  // the split runs inside the conjugation's ModDown combine
        const uint32_t g = 2 * c->N - 1;
        const uint64_t *key = key_of(c, g);
        if (!key) return fail(NJ_ENOKEY, "no switching key for the conjugation");
        MultiBufs M;
        if (!multi_bufs(c, l, 1, A, M)) return fail(NJ_ENOMEM, "scratch too small");
        const MdConj cj{x, re, im};
        return ks_one(c, l, x + clen / 2, g, key, x, g, nullptr, M, s, &cj);
    }
    uint64_t *cj = A.take(clen);
    if (!cj) return fail(NJ_ENOMEM, "scratch too small");
    nj_status st = apply_galois(c, l, x, 2 * c->N - 1, cj, A, s);
    if (st) return st;
    NJ_HIP(launch_conj_split(c, l, x, cj, re, im, s));
    return NJ_OK;
}

nj_status check_ct(const nj_ctx *c, const nj_ct *ct, const char *what)
{
    if (!ct || !ct->data) return fail(NJ_EINVAL, std::string(what) + ": null ciphertext");
    if (ct->level < 0 || ct->level > c->L) return fail(NJ_ELEVEL, std::string(what) + ": level out of range");
    if (!ct->is_ntt) return fail(NJ_EINVAL, std::string(what) + ": ciphertext must be in evaluation form");
    return NJ_OK;
}

Arena arena_for(nj_ctx *c, size_t words, bool &ok)
{
    uint64_t *p = scratch_get(c, words);
    ok = p != nullptr;
    return Arena{p, ok ? words : 0};
}

hipError_t upload_signed(nj_ctx *c, const int64_t *host, int n_rows, const LimbTab &lt, uint64_t *dst, uint64_t *tmp,
                         hipStream_t s)
{
    (void)n_rows;
    hipError_t e = hipMemcpyAsync(tmp, host, (size_t)c->N * 8, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return launch_signed_to_rns(c, (const int64_t *)tmp, lt, dst, s, c->d_primes);
}

size_t cts_batch_words(const nj_ctx *c, const nj_plan *p, int Kmax)
{
    const int lo = c->L - (int)p->lts.size();
    const size_t N = c->N, ctop = 2 * N * (c->L + 1), cout = 2 * N * (lo + 1);
    size_t need = 0;
    for (const auto &lt : p->lts) need = std::max(need, bsgs_batch_words(c, lt, Kmax));
    need = std::max(need, Kmax * cout + multi_words(c, lo, Kmax));
    return need + 2 * Kmax * ctop + N * (c->L + 2);
}

// ModRaise + CoeffToSlot + real split of n level-0 ciphertexts (contiguous [n][2][1][N]),
// kBatch at a time; ciphertext z's outputs go to re[z], im[z].
nj_status cts_batch(nj_ctx *c, const nj_plan *p, const uint64_t *in, int n, uint64_t *const *re, uint64_t *const *im,
                    Arena A, hipStream_t s)
{
    const int Kmax = std::min(n, kBatch), lo = c->L - (int)p->lts.size();
    const size_t N = c->N, ctop = 2 * N * (c->L + 1), cin = 2 * N, cout = 2 * N * (lo + 1);
    uint64_t *x = A.take(Kmax * ctop), *y = A.take(Kmax * ctop);
    if (!y) return fail(NJ_ENOMEM, "scratch too small");
    nj_status st;
    for (int z0 = 0; z0 < n; z0 += kBatch) {
        const int K = std::min(kBatch, n - z0);
        for (int z = 0; z < K; z++)
            if ((st = modraise(c, in + (z0 + z) * cin, c->L, x + z * ctop, A, s))) return st;
        int l = c->L;
        for (const auto &lt : p->lts) {
            if (lt.level != l) return fail(NJ_ELEVEL, "CoeffToSlot: plan levels do not follow the context's top level");
            if ((st = bsgs_apply_batch(c, lt, K, x, y, A, s))) return st;
            if ((st = rescale_batch(c, l, K, y, x, A, s))) return st;
            l--;
        }
        // real split of every ciphertext: one batch of conjugations
        Arena B = A;
        uint64_t *cj = B.take(K * cout);
        if ((st = apply_galois_batch(c, l, K, x, 2 * c->N - 1, cj, B, s))) return st;
        for (int z = 0; z < K; z++) NJ_HIP(launch_conj_split(c, l, x + z * cout, cj + z * cout, re[z0 + z], im[z0 + z], s));
    }
    return NJ_OK;
}

// One BSGS transform then a rescale: x -> y (scratch) -> out (level l-1).  When the
// transform's last step is a one-job ModDown (lazy giant steps, N >= 8192) it also
// runs the first pass of the rescale's inverse transform.
nj_status bsgs_rescale(nj_ctx *c, const nj_lt_t &lt, const uint64_t *x, uint64_t *y, uint64_t *out, Arena A,
                       hipStream_t s)
{
    uint64_t *last = c->N >= 8192 ? A.take(2 * (size_t)c->N) : nullptr;
    if (c->N >= 8192 && !last) return fail(NJ_ENOMEM, "scratch too small");
    bool done = false;
    nj_status st = bsgs_apply(c, lt, x, y, lt.hoist ? 1 : 0, A, s, last, &done);
    if (st) return st;
    return rescale(c, lt.level, y, out, A, s, -1, 2, done ? last : nullptr);
}

size_t cts_single_words(const nj_ctx *c, const nj_plan *p)
{
    const size_t N = c->N, top = c->L, clen = 2 * N * (top + 1);
    size_t need = 0;
    for (const auto &lt : p->lts) need = std::max(need, bsgs_words(c, lt));
    return std::max(need, ks_words(c, c->L) + clen) + 2 * clen + N * (top + 2);
}

// ModRaise + CoeffToSlot + real split of one level-0 ciphertext [2][1][N]
nj_status cts_single(nj_ctx *c, const nj_plan *p, const uint64_t *in, uint64_t *re, uint64_t *im, Arena A,
                     hipStream_t s)
{
    const size_t N = c->N, clen = 2 * N * (c->L + 1);
    uint64_t *x = A.take(clen), *y = A.take(clen);
    if (!y) return fail(NJ_ENOMEM, "scratch too small");
    nj_status st = modraise(c, in, c->L, x, A, s);
    if (st) return st;
    int l = c->L;
    for (const auto &lt : p->lts) {
        if (lt.level != l) return fail(NJ_ELEVEL, "CoeffToSlot: plan levels do not follow the context's top level");
        if ((st = bsgs_rescale(c, lt, x, y, x, A, s))) return st;
        l--;
    }
    return conj_split(c, l, x, re, im, A, s);
}

}  // namespace ex
}  // namespace nj

using namespace nj::ex;

extern "C" {

nj_status nj_set_secret(nj_ctx *c, const int8_t *sk)
{
    if (!c || !sk) return fail(NJ_EINVAL, "nj_set_secret: null argument");
    c->s.assign(sk, sk + c->N);
    std::vector<int64_t> s64(c->N);
    for (int i = 0; i < c->N; i++) {
        if (sk[i] < -1 || sk[i] > 1) return fail(NJ_EINVAL, "nj_set_secret: entries must be -1, 0 or 1");
        s64[i] = sk[i];
    }
    if (!c->d_s) NJ_HIP(hipMalloc(&c->d_s, (size_t)c->n_primes * c->N * 8));
    int64_t *tmp = nullptr;
    NJ_HIP(hipMalloc(&tmp, (size_t)c->N * 8));
    NJ_HIP(hipMemcpy(tmp, s64.data(), (size_t)c->N * 8, hipMemcpyHostToDevice));
    LimbTab lt;
    lt.n = c->n_primes;
    for (int i = 0; i < lt.n; i++) lt.pidx[i] = i, lt.off[i] = i;
    NJ_HIP(launch_signed_to_rns(c, tmp, lt, c->d_s, 0, c->d_primes));
    NJ_HIP(launch_ntt(c, c->d_s, lt, false, 0));
    NJ_HIP(hipDeviceSynchronize());
    NJ_HIP(hipFree(tmp));
    return NJ_OK;
}

nj_status nj_gen_switch_key(nj_ctx *c, uint32_t g, const uint64_t *a, const int64_t *e)
{
    if (!c || !a || !e) return fail(NJ_EINVAL, "nj_gen_switch_key: null argument");
    if (!c->d_s) return fail(NJ_EINVAL, "nj_gen_switch_key: secret not set");
    if (g != 0 && (g % 2 == 0 || g >= 2u * c->N)) return fail(NJ_EINVAL, "nj_gen_switch_key: bad Galois element");
    const size_t N = c->N, nk = c->L + 1 + c->alpha;
    uint64_t *key = nullptr;
    auto it = c->keys.find(g);
    if (it != c->keys.end()) key = it->second.d;
    else {
        NJ_HIP(hipMalloc(&key, (size_t)c->dnum * 2 * nk * N * 8));
        c->keys[g].d = key;
    }
    uint64_t *sp = nullptr, *ebuf = nullptr;
    int64_t *etmp = nullptr;
    NJ_HIP(hipMalloc(&sp, (size_t)c->n_primes * N * 8));
    NJ_HIP(hipMalloc(&ebuf, nk * N * 8));
    NJ_HIP(hipMalloc(&etmp, N * 8));
    LimbTab all;
    all.n = c->n_primes;
    for (int i = 0; i < all.n; i++) all.pidx[i] = i, all.off[i] = i;
    if (g == 0) NJ_HIP(launch_elementwise(c, 2, c->d_s, c->d_s, sp, all, 0));
    else NJ_HIP(launch_automorph(c, c->d_s, sp, g, c->n_primes, 0));
    LimbTab kl;
    kl.n = (int)nk;
    for (int t = 0; t < (int)nk; t++) kl.pidx[t] = t <= c->L ? t : c->n_q + (t - c->L - 1), kl.off[t] = t;
    for (int j = 0; j < c->dnum; j++) {
        uint64_t *bj = key + ((size_t)j * 2 + 0) * nk * N, *aj = key + ((size_t)j * 2 + 1) * nk * N;
        NJ_HIP(hipMemcpy(aj, a + (size_t)j * nk * N, nk * N * 8, hipMemcpyHostToDevice));
        NJ_HIP(launch_ntt(c, aj, kl, false, 0));
        NJ_HIP(hipMemcpy(etmp, e + (size_t)j * N, N * 8, hipMemcpyHostToDevice));
        NJ_HIP(launch_signed_to_rns(c, etmp, kl, ebuf, 0, c->d_primes));
        NJ_HIP(launch_ntt(c, ebuf, kl, false, 0));
        NJ_HIP(launch_keygen_combine(c, j, bj, aj, ebuf, c->d_s, sp, c->d_pmod, 0));
    }
    NJ_HIP(hipDeviceSynchronize());
    (void)hipFree(sp), (void)hipFree(ebuf), (void)hipFree(etmp);
    return NJ_OK;
}

nj_status nj_ntt_limbs(nj_ctx *c, uint64_t *data, const int *prime_idx, int n_limbs, int inverse, void *stream)
{
    if (!c || !data || !prime_idx || n_limbs < 0) return fail(NJ_EINVAL, "nj_ntt_limbs: bad arguments");
    for (int base = 0; base < n_limbs; base += NJ_MAX_LIMBS) {
        LimbTab lt;
        lt.n = std::min(NJ_MAX_LIMBS, n_limbs - base);
        for (int i = 0; i < lt.n; i++) {
            int p = prime_idx[base + i];
            if (p < 0 || p >= c->n_primes) return fail(NJ_EINVAL, "nj_ntt_limbs: prime index out of range");
            lt.pidx[i] = p, lt.off[i] = base + i;
        }
        NJ_HIP(launch_ntt(c, data, lt, inverse != 0, S(stream)));
    }
    return NJ_OK;
}

static nj_status convert(nj_ctx *c, uint64_t *data, int level, int n_polys, bool inverse, void *stream)
{
    if (!c || !data || level < 0 || level > c->L || n_polys < 1) return fail(NJ_EINVAL, "conversion: bad arguments");
    for (int p = 0; p < n_polys; p++)
        NJ_HIP(launch_ntt(c, data + (size_t)p * (level + 1) * c->N, limbs_q(level), inverse, S(stream)));
    return NJ_OK;
}
nj_status nj_to_eval(nj_ctx *c, uint64_t *data, int level, int n_polys, void *stream)
{
    return convert(c, data, level, n_polys, false, stream);
}
nj_status nj_to_coeff(nj_ctx *c, uint64_t *data, int level, int n_polys, void *stream)
{
    return convert(c, data, level, n_polys, true, stream);
}

nj_status nj_upload_plain(nj_ctx *c, const int64_t *coeffs, int level, uint64_t *dst, void *stream)
{
    if (!c || !coeffs || !dst || level < 0 || level > c->L) return fail(NJ_EINVAL, "nj_upload_plain: bad arguments");
    bool ok;
    Arena A = arena_for(c, c->N, ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    NJ_HIP(upload_signed(c, coeffs, 1, limbs_q(level), dst, A.take(c->N), S(stream)));
    NJ_HIP(hipStreamSynchronize(S(stream)));  // the host array is borrowed only for the call
    return NJ_OK;
}

nj_status nj_encrypt_sk(nj_ctx *c, const uint64_t *m, int level, const uint64_t *a, const int64_t *e, double scale,
                        nj_ct *out, void *stream)
{
    if (!c || !m || !a || !e || !out || !out->data) return fail(NJ_EINVAL, "nj_encrypt_sk: null argument");
    if (level < 0 || level > c->L) return fail(NJ_ELEVEL, "nj_encrypt_sk: level out of range");
    if (!c->d_s) return fail(NJ_EINVAL, "nj_encrypt_sk: secret not set");
    const size_t N = c->N, plen = N * (level + 1);
    hipStream_t s = S(stream);
    bool ok;
    Arena A = arena_for(c, 2 * plen + N, ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    uint64_t *mt = A.take(plen), *et = A.take(plen), *tmp = A.take(N);
    uint64_t *c0 = out->data, *c1 = out->data + plen;
    NJ_HIP(hipMemcpyAsync(c1, a, plen * 8, hipMemcpyHostToDevice, s));
    NJ_HIP(launch_ntt(c, c1, limbs_q(level), false, s));
    NJ_HIP(hipMemcpyAsync(mt, m, plen * 8, hipMemcpyDeviceToDevice, s));
    NJ_HIP(launch_ntt(c, mt, limbs_q(level), false, s));
    NJ_HIP(upload_signed(c, e, 1, limbs_q(level), et, tmp, s));
    NJ_HIP(launch_ntt(c, et, limbs_q(level), false, s));
    NJ_HIP(launch_elementwise(c, 2, c1, c->d_s, c0, limbs_q(level), s));
    NJ_HIP(launch_elementwise(c, 1, et, c0, c0, limbs_q(level), s));
    NJ_HIP(launch_elementwise(c, 0, c0, mt, c0, limbs_q(level), s));
    NJ_HIP(hipStreamSynchronize(s));  // the host arrays a and e are borrowed only for the call
    out->level = level;
    out->is_ntt = 1;
    out->scale = scale;
    return NJ_OK;
}

size_t nj_key_words(const nj_ctx *c)
{
    return c ? (size_t)c->dnum * 2 * (c->L + 1 + c->alpha) * c->N : 0;
}

nj_status nj_key_export(nj_ctx *c, uint32_t g, uint64_t *host, size_t words)
{
    if (!c || !host) return fail(NJ_EINVAL, "nj_key_export: null argument");
    if (words != nj_key_words(c)) return fail(NJ_EINVAL, "nj_key_export: buffer size must be nj_key_words");
    auto it = c->keys.find(g);
    if (it == c->keys.end()) return fail(NJ_ENOKEY, "nj_key_export: no key for this Galois element");
    NJ_HIP(hipDeviceSynchronize());  // work still writing the key finishes first
    NJ_HIP(hipMemcpy(host, it->second.d, words * 8, hipMemcpyDeviceToHost));
    return NJ_OK;
}

nj_status nj_key_import(nj_ctx *c, uint32_t g, const uint64_t *host, size_t words)
{
    if (!c || !host) return fail(NJ_EINVAL, "nj_key_import: null argument");
    if (words != nj_key_words(c)) return fail(NJ_EINVAL, "nj_key_import: buffer size must be nj_key_words");
    if (g != 0 && (g % 2 == 0 || g >= 2u * c->N)) return fail(NJ_EINVAL, "nj_key_import: bad Galois element");
    uint64_t *key = nullptr;
    auto it = c->keys.find(g);
    if (it != c->keys.end()) key = it->second.d;
    else {
        NJ_HIP(hipMalloc(&key, words * 8));
        c->keys[g].d = key;
    }
    NJ_HIP(hipDeviceSynchronize());  // no queued work still reads the key being replaced
    NJ_HIP(hipMemcpy(key, host, words * 8, hipMemcpyHostToDevice));
    return NJ_OK;
}

nj_status nj_key_list(const nj_ctx *c, uint32_t *gs, int max, int *n)
{
    if (!c || !n || (max > 0 && !gs)) return fail(NJ_EINVAL, "nj_key_list: bad arguments");
    int k = 0;
    for (const auto &kv : c->keys) {
        if (k < max) gs[k] = kv.first;
        k++;
    }
    *n = k;
    return NJ_OK;
}

nj_status nj_gen_public_key(nj_ctx *c, const uint64_t *a, const int64_t *e)
{
    if (!c || !a || !e) return fail(NJ_EINVAL, "nj_gen_public_key: null argument");
    if (!c->d_s) return fail(NJ_EINVAL, "nj_gen_public_key: secret not set");
    const size_t N = c->N, plen = N * (c->L + 1);
    if (!c->d_pk) NJ_HIP(hipMalloc(&c->d_pk, 2 * plen * 8));
    uint64_t *b = c->d_pk, *ak = c->d_pk + plen, *et = nullptr, *tmp = nullptr;
    NJ_HIP(hipMalloc(&et, plen * 8));
    if (hipMalloc(&tmp, N * 8) != hipSuccess) {
        (void)hipFree(et);
        return fail(NJ_ENOMEM, "nj_gen_public_key: device memory");
    }
    const LimbTab lq = limbs_q(c->L);
    hipError_t err = hipMemcpy(ak, a, plen * 8, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = launch_ntt(c, ak, lq, false, 0);
    if (err == hipSuccess) err = upload_signed(c, e, 1, lq, et, tmp, 0);
    if (err == hipSuccess) err = launch_ntt(c, et, lq, false, 0);
    if (err == hipSuccess) err = launch_elementwise(c, 2, ak, c->d_s, b, lq, 0);  // a s
    if (err == hipSuccess) err = launch_elementwise(c, 1, et, b, b, lq, 0);       // e - a s
    if (err == hipSuccess) err = hipDeviceSynchronize();
    (void)hipFree(et), (void)hipFree(tmp);
    if (err != hipSuccess) return fail(NJ_EDEVICE, hipGetErrorString(err));
    return NJ_OK;
}

nj_status nj_encrypt_pk(nj_ctx *c, const uint64_t *m, int level, const int64_t *v, const int64_t *e0, const int64_t *e1,
                        double scale, nj_ct *out, void *stream)
{
    if (!c || !m || !v || !e0 || !e1 || !out || !out->data) return fail(NJ_EINVAL, "nj_encrypt_pk: null argument");
    if (level < 0 || level > c->L) return fail(NJ_ELEVEL, "nj_encrypt_pk: level out of range");
    if (!c->d_pk) return fail(NJ_EINVAL, "nj_encrypt_pk: no public key (nj_gen_public_key)");
    const size_t N = c->N, plen = N * (level + 1), ptop = N * (c->L + 1);
    hipStream_t s = S(stream);
    bool ok;
    Arena A = arena_for(c, 3 * plen + N, ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    uint64_t *vt = A.take(plen), *et = A.take(plen), *mt = A.take(plen), *tmp = A.take(N);
    uint64_t *c0 = out->data, *c1 = out->data + plen;
    const LimbTab lq = limbs_q(level);
    // the first level+1 limbs of each key polynomial are that polynomial at `level`
    NJ_HIP(upload_signed(c, v, 1, lq, vt, tmp, s));
    NJ_HIP(launch_ntt(c, vt, lq, false, s));
    NJ_HIP(hipMemcpyAsync(mt, m, plen * 8, hipMemcpyDeviceToDevice, s));
    NJ_HIP(launch_ntt(c, mt, lq, false, s));
    NJ_HIP(launch_elementwise(c, 2, c->d_pk, vt, c0, lq, s));          // v pk0
    NJ_HIP(launch_elementwise(c, 0, c0, mt, c0, lq, s));               // + m
    NJ_HIP(launch_elementwise(c, 2, c->d_pk + ptop, vt, c1, lq, s));   // v pk1
    NJ_HIP(upload_signed(c, e0, 1, lq, et, tmp, s));
    NJ_HIP(launch_ntt(c, et, lq, false, s));
    NJ_HIP(launch_elementwise(c, 0, c0, et, c0, lq, s));               // + e0
    NJ_HIP(hipStreamSynchronize(s));  // tmp is reused for e1 and the host arrays are borrowed only for the call
    NJ_HIP(upload_signed(c, e1, 1, lq, et, tmp, s));
    NJ_HIP(launch_ntt(c, et, lq, false, s));
    NJ_HIP(launch_elementwise(c, 0, c1, et, c1, lq, s));               // + e1
    NJ_HIP(hipStreamSynchronize(s));
    out->level = level;
    out->is_ntt = 1;
    out->scale = scale;
    return NJ_OK;
}

nj_status nj_decrypt(nj_ctx *c, const nj_ct *in, uint64_t *out, void *stream)
{
    if (!c || !out) return fail(NJ_EINVAL, "nj_decrypt: null argument");
    nj_status st = check_ct(c, in, "nj_decrypt");
    if (st) return st;
    if (!c->d_s) return fail(NJ_EINVAL, "nj_decrypt: secret not set");
    const int l = in->level;
    const size_t plen = (size_t)c->N * (l + 1);
    NJ_HIP(launch_elementwise(c, 2, in->data + plen, c->d_s, out, limbs_q(l), S(stream)));
    NJ_HIP(launch_elementwise(c, 0, out, in->data, out, limbs_q(l), S(stream)));
    NJ_HIP(launch_ntt(c, out, limbs_q(l), true, S(stream)));
    return NJ_OK;
}

nj_status nj_encode_slots(int log_n, const double *z, double scale, int64_t *out)
{
    if (!z || !out || log_n < 2 || log_n > 20) return fail(NJ_EINVAL, "nj_encode_slots: bad arguments");
    const int N = 1 << log_n, n = N / 2;
    std::vector<double> re(n), im(n);
    for (int j = 0; j < n; j++) re[j] = z[2 * j], im[j] = z[2 * j + 1];
    encode_slots(N, re.data(), im.data(), scale, out);
    return NJ_OK;
}

nj_status nj_encode_cins(int log_n, const double *chans, int slice_len2, double scale, int64_t *out)
{
    if (!chans || !out || log_n < 2 || log_n > 20 || slice_len2 < 2 || (1 << log_n) % slice_len2 ||
        (slice_len2 & (slice_len2 - 1)))
        return fail(NJ_EINVAL, "nj_encode_cins: bad arguments");
    encode_cins(1 << log_n, chans, slice_len2, scale, out);
    return NJ_OK;
}

nj_status nj_decode_slots(int log_n, const double *coeffs, double scale, double *z)
{
    if (!coeffs || !z || log_n < 2 || log_n > 20) return fail(NJ_EINVAL, "nj_decode_slots: bad arguments");
    const int N = 1 << log_n, n = N / 2;
    std::vector<double> re(n), im(n);
    decode_slots(N, coeffs, scale, re.data(), im.data());
    for (int j = 0; j < n; j++) z[2 * j] = re[j], z[2 * j + 1] = im[j];
    return NJ_OK;
}

nj_status nj_apply_galois(nj_ctx *c, const nj_ct *in, uint32_t g, nj_ct *out, void *stream)
{
    nj_status st = check_ct(c, in, "nj_apply_galois");
    if (st) return st;
    if (!out || !out->data) return fail(NJ_EINVAL, "nj_apply_galois: null output");
    bool ok;
    Arena A = arena_for(c, ks_words(c, in->level), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    st = apply_galois(c, in->level, in->data, g, out->data, A, S(stream));
    if (st) return st;
    out->level = in->level, out->is_ntt = 1, out->scale = in->scale;
    return NJ_OK;
}

nj_status nj_rotate(nj_ctx *c, const nj_ct *in, int r, nj_ct *out, void *stream)
{
    if (!c) return fail(NJ_EINVAL, "nj_rotate: null context");
    return nj_apply_galois(c, in, nj_galois_elt(c, r), out, stream);
}

nj_status nj_keyswitch(nj_ctx *c, const uint64_t *d, int level, uint32_t g, uint64_t *out0, uint64_t *out1,
                       void *stream)
{
    if (!c || !d || !out0 || !out1) return fail(NJ_EINVAL, "nj_keyswitch: null argument");
    if (level < 0 || level > c->L) return fail(NJ_ELEVEL, "nj_keyswitch: level out of range");
    const uint64_t *key = key_of(c, g);
    if (!key) return fail(NJ_ENOKEY, "nj_keyswitch: no key for that element");
    const size_t plen = (size_t)c->N * (level + 1);
    bool ok;
    Arena A = arena_for(c, ks_words(c, level) + 2 * plen, ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    uint64_t *pair = A.take(2 * plen);
    MultiBufs M;
    if (!pair || !multi_bufs(c, level, 1, A, M)) return fail(NJ_ENOMEM, "scratch");
    nj_status st = ks_one(c, level, d, 1, key, nullptr, 0, pair, M, S(stream));
    if (st) return st;
    NJ_HIP(hipMemcpyAsync(out0, pair, plen * 8, hipMemcpyDeviceToDevice, S(stream)));
    NJ_HIP(hipMemcpyAsync(out1, pair + plen, plen * 8, hipMemcpyDeviceToDevice, S(stream)));
    return NJ_OK;
}

nj_status nj_pmult(nj_ctx *c, const nj_ct *in, const uint64_t *pt, nj_ct *out, void *stream)
{
    nj_status st = check_ct(c, in, "nj_pmult");
    if (st) return st;
    if (!pt || !out || !out->data) return fail(NJ_EINVAL, "nj_pmult: null argument");
    NJ_HIP(launch_pmac(c, in->level, in->data, pt, out->data, 1, S(stream)));
    out->level = in->level, out->is_ntt = 1, out->scale = in->scale;
    return NJ_OK;
}

static nj_status addsub(nj_ctx *c, int op, const nj_ct *a, const nj_ct *b, nj_ct *out, void *stream, const char *nm)
{
    nj_status st = check_ct(c, a, nm);
    if (st) return st;
    if ((st = check_ct(c, b, nm))) return st;
    if (a->level != b->level) return fail(NJ_ELEVEL, std::string(nm) + ": operands at different levels");
    if (!same_scale(a->scale, b->scale)) return fail(NJ_ESCALE, std::string(nm) + ": operands at different scales");
    if (!out || !out->data) return fail(NJ_EINVAL, std::string(nm) + ": null output");
    NJ_HIP(launch_elementwise(c, op, a->data, b->data, out->data, ct_limbs(a->level), S(stream)));
    out->level = a->level, out->is_ntt = 1, out->scale = a->scale;
    return NJ_OK;
}
nj_status nj_add(nj_ctx *c, const nj_ct *a, const nj_ct *b, nj_ct *out, void *stream)
{
    return addsub(c, 0, a, b, out, stream, "nj_add");
}
nj_status nj_sub(nj_ctx *c, const nj_ct *a, const nj_ct *b, nj_ct *out, void *stream)
{
    return addsub(c, 1, a, b, out, stream, "nj_sub");
}

nj_status nj_rescale(nj_ctx *c, const nj_ct *in, nj_ct *out, void *stream)
{
    nj_status st = check_ct(c, in, "nj_rescale");
    if (st) return st;
    if (in->level < 1) return fail(NJ_ELEVEL, "nj_rescale: level 0 cannot be rescaled");
    if (!out || !out->data || out->data == in->data) return fail(NJ_EINVAL, "nj_rescale: output must not alias input");
    bool ok;
    Arena A = arena_for(c, (size_t)c->N * (in->level + 2), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    st = rescale(c, in->level, in->data, out->data, A, S(stream));
    if (st) return st;
    out->level = in->level - 1, out->is_ntt = 1, out->scale = in->scale / (double)c->primes[in->level];
    return NJ_OK;
}

nj_status nj_drop_level(nj_ctx *c, const nj_ct *in, int level, nj_ct *out, void *stream)
{
    nj_status st = check_ct(c, in, "nj_drop_level");
    if (st) return st;
    if (level < 0 || level > in->level) return fail(NJ_ELEVEL, "nj_drop_level: level must be in 0..input level");
    if (!out || !out->data || (out->data == in->data && level != in->level))
        return fail(NJ_EINVAL, "nj_drop_level: bad output");
    const size_t N = c->N;
    if (out->data != in->data)
        NJ_HIP(hipMemcpy2DAsync(out->data, (level + 1) * N * 8, in->data, (in->level + 1) * N * 8, (level + 1) * N * 8, 2,
                                hipMemcpyDeviceToDevice, S(stream)));
    out->level = level, out->is_ntt = in->is_ntt, out->scale = in->scale;
    return NJ_OK;
}

nj_status nj_modraise(nj_ctx *c, const nj_ct *in, int level, nj_ct *out, void *stream)
{
    nj_status st = check_ct(c, in, "nj_modraise");
    if (st) return st;
    if (in->level != 0) return fail(NJ_ELEVEL, "nj_modraise: input must be at level 0");
    if (level < 0 || level > c->L) return fail(NJ_ELEVEL, "nj_modraise: target level out of range");
    if (!out || !out->data || out->data == in->data) return fail(NJ_EINVAL, "nj_modraise: output must not alias input");
    bool ok;
    Arena A = arena_for(c, 2 * (size_t)c->N, ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    st = modraise(c, in->data, level, out->data, A, S(stream));
    if (st) return st;
    out->level = level, out->is_ntt = 1, out->scale = in->scale;
    return NJ_OK;
}

// ------------------------------------------------------------------- plans

int nj_plan_count(const nj_plan *p) { return p ? (int)p->lts.size() : 0; }

int nj_plan_galois(const nj_plan *p, uint32_t *out, int max)
{
    if (!p) return 0;
    std::vector<uint32_t> gs;
    plan_galois_impl(p, gs);
    for (int i = 0; i < (int)gs.size() && i < max; i++) out[i] = gs[i];
    return (int)gs.size();
}

int nj_plan_offsets(const nj_plan *p, int t, int32_t *out, int max)
{
    if (!p || t < 0 || t >= (int)p->lts.size()) return 0;
    const nj_lt_t &lt = p->lts[t];
    for (int i = 0; i < lt.n_diag && i < max; i++) out[i] = lt.js[i];
    return lt.n_diag;
}

nj_status nj_plan_set_diagonal(nj_ctx *c, nj_plan *p, int t, int idx, const uint64_t *coeffs)
{
    if (!c || !p || !coeffs || t < 0 || t >= (int)p->lts.size()) return fail(NJ_EINVAL, "nj_plan_set_diagonal: bad arguments");
    nj_lt_t &lt = p->lts[t];
    if (idx < 0 || idx >= lt.n_diag * lt.bi * lt.bo) return fail(NJ_EINVAL, "nj_plan_set_diagonal: index out of range");
    if (!lt.nz.empty()) lt.nz[idx] = 1;
    const size_t plen = (size_t)c->N * lt.dl;
    uint64_t *dst = lt.d_diag + (size_t)idx * plen;
    NJ_HIP(hipMemcpy(dst, coeffs, plen * 8, hipMemcpyHostToDevice));
    NJ_HIP(launch_ntt(c, dst, limbs_q(lt.dl - 1), false, 0));
    NJ_HIP(hipDeviceSynchronize());
    return NJ_OK;
}

nj_status nj_plan_set_lazy(nj_plan *p, int on)
{
    if (!p) return fail(NJ_EINVAL, "nj_plan_set_lazy: null plan");
    for (auto &lt : p->lts) lt.lazy = on != 0;
    return NJ_OK;
}

nj_status nj_plan_set_hoist(nj_plan *p, int t, int on)
{
    if (!p || t < -1 || t >= (int)p->lts.size()) return fail(NJ_EINVAL, "nj_plan_set_hoist: bad arguments");
    for (int i = 0; i < (int)p->lts.size(); i++)
        if (t < 0 || i == t) p->lts[i].hoist = on != 0;
    return NJ_OK;
}

void nj_plan_destroy(nj_plan *p)
{
    if (!p) return;
    (void)hipDeviceSynchronize();
    for (auto &lt : p->lts)
        if (lt.d_diag) (void)hipFree(lt.d_diag);
    delete p;
}

nj_status nj_plan_apply(nj_ctx *c, const nj_plan *p, int t, const nj_ct *in, nj_ct *out, int hoist, void *stream)
{
    if (!c || !p || t < 0 || t >= (int)p->lts.size()) return fail(NJ_EINVAL, "nj_plan_apply: bad arguments");
    nj_status st = check_ct(c, in, "nj_plan_apply");
    if (st) return st;
    if (p->lts[t].bi != 1 || p->lts[t].bo != 1)
        return fail(NJ_EINVAL, "nj_plan_apply: block plans run through nj_conv2d_block");
    if (in->level > p->lts[t].level) return fail(NJ_ELEVEL, "nj_plan_apply: ciphertext above the transform's level");
    if (!out || !out->data || out->data == in->data) return fail(NJ_EINVAL, "nj_plan_apply: output must not alias input");
    const nj_lt_t lt = at_level(p->lts[t], in->level);
    bool ok;
    Arena A = arena_for(c, bsgs_words(c, lt), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    st = bsgs_apply(c, lt, in->data, out->data, hoist, A, S(stream));
    if (st) return st;
    out->level = lt.level, out->is_ntt = 1, out->scale = in->scale * lt.scale;
    return NJ_OK;
}

nj_status nj_conv2d_cins(nj_ctx *c, const nj_plan *p, const nj_ct *in, nj_ct *out, void *stream)
{
    if (!c || !p || p->kind != 0 || p->lts.empty()) return fail(NJ_EINVAL, "nj_conv2d_cins: not a conv plan");
    nj_status st = check_ct(c, in, "nj_conv2d_cins");
    if (st) return st;
    if (p->lts[0].bi != 1 || p->lts[0].bo != 1)
        return fail(NJ_EINVAL, "nj_conv2d_cins: block plans run through nj_conv2d_block");
    if (in->level < 1 || in->level > p->lts[0].level)
        return fail(NJ_ELEVEL, "nj_conv2d_cins: input level must be in 1..the plan's level");
    const nj_lt_t lt = at_level(p->lts[0], in->level);
    if (!out || !out->data || out->data == in->data) return fail(NJ_EINVAL, "nj_conv2d_cins: output must not alias input");
    const size_t clen = 2 * (size_t)c->N * (lt.level + 1);
    bool ok;
    Arena A = arena_for(c, clen + bsgs_words(c, lt) + (size_t)c->N * (lt.level + 2), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    uint64_t *y = A.take(clen);
    st = bsgs_rescale(c, lt, in->data, y, out->data, A, S(stream));
    if (st) return st;
    out->level = lt.level - 1, out->is_ntt = 1, out->scale = in->scale * lt.scale / (double)c->primes[lt.level];
    return NJ_OK;
}

nj_status nj_coeff_to_slot(nj_ctx *c, const nj_plan *p, const nj_ct *in, nj_ct *re, nj_ct *im, void *stream)
{
    if (!c || !p || p->kind != 1 || p->lts.empty()) return fail(NJ_EINVAL, "nj_coeff_to_slot: not a CoeffToSlot plan");
    nj_status st = check_ct(c, in, "nj_coeff_to_slot");
    if (st) return st;
    if (in->level != 0) return fail(NJ_ELEVEL, "nj_coeff_to_slot: input must be at level 0");
    if (!re || !im || !re->data || !im->data) return fail(NJ_EINVAL, "nj_coeff_to_slot: null output");
    bool ok;
    Arena A = arena_for(c, cts_single_words(c, p), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    if ((st = cts_single(c, p, in->data, re->data, im->data, A, S(stream)))) return st;
    re->level = im->level = c->L - (int)p->lts.size();
    re->is_ntt = im->is_ntt = 1;
    re->scale = im->scale = in->scale;
    return NJ_OK;
}

// ------------------------------------------------------------ batched calls

static nj_status check_batch(const nj_ctx *c, const nj_ct *in, int n, const nj_ct *out, const char *nm)
{
    nj_status st = check_ct(c, in, nm);
    if (st) return st;
    if (n < 1) return fail(NJ_EINVAL, std::string(nm) + ": batch size must be positive");
    if (!out || !out->data || out->data == in->data) return fail(NJ_EINVAL, std::string(nm) + ": bad output");
    return NJ_OK;
}

nj_status nj_apply_galois_batch(nj_ctx *c, const nj_ct *in, int n, uint32_t g, nj_ct *out, void *stream)
{
    nj_status st = check_batch(c, in, n, out, "nj_apply_galois_batch");
    if (st) return st;
    const int l = in->level, Kmax = std::min(n, kBatch);
    const size_t clen = 2 * (size_t)c->N * (l + 1);
    bool ok;
    Arena A = arena_for(c, multi_words(c, l, Kmax), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    for (int z0 = 0; z0 < n; z0 += kBatch) {
        const int K = std::min(kBatch, n - z0);
        st = apply_galois_batch(c, l, K, in->data + z0 * clen, g, out->data + z0 * clen, A, S(stream));
        if (st) return st;
    }
    out->level = l, out->is_ntt = 1, out->scale = in->scale;
    return NJ_OK;
}

nj_status nj_conv2d_cins_batch(nj_ctx *c, const nj_plan *p, const nj_ct *in, int n, nj_ct *out, void *stream)
{
    if (!c || !p || p->kind != 0 || p->lts.empty()) return fail(NJ_EINVAL, "nj_conv2d_cins_batch: not a conv plan");
    nj_status st = check_batch(c, in, n, out, "nj_conv2d_cins_batch");
    if (st) return st;
    if (p->lts[0].bi != 1 || p->lts[0].bo != 1)
        return fail(NJ_EINVAL, "nj_conv2d_cins_batch: block plans run through nj_conv2d_block");
    if (in->level < 1 || in->level > p->lts[0].level)
        return fail(NJ_ELEVEL, "nj_conv2d_cins_batch: input level must be in 1..the plan's level");
    const nj_lt_t lt = at_level(p->lts[0], in->level);
    const int l = lt.level, Kmax = std::min(n, kBatch);
    const size_t N = c->N, clen = 2 * N * (l + 1), clen_out = 2 * N * l;
    bool ok;
    Arena A = arena_for(c, Kmax * clen + bsgs_batch_words(c, lt, Kmax) + N * (l + 2), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    uint64_t *y = A.take(Kmax * clen);
    hipStream_t s = S(stream);
    for (int z0 = 0; z0 < n; z0 += kBatch) {
        const int K = std::min(kBatch, n - z0);
        if ((st = bsgs_apply_batch(c, lt, K, in->data + z0 * clen, y, A, s))) return st;
        if ((st = rescale_batch(c, l, K, y, out->data + z0 * clen_out, A, s))) return st;
    }
    out->level = l - 1, out->is_ntt = 1, out->scale = in->scale * lt.scale / (double)c->primes[l];
    return NJ_OK;
}

nj_status nj_coeff_to_slot_batch(nj_ctx *c, const nj_plan *p, const nj_ct *in, int n, nj_ct *re, nj_ct *im,
                                 void *stream)
{
    if (!c || !p || p->kind != 1 || p->lts.empty()) return fail(NJ_EINVAL, "nj_coeff_to_slot_batch: not a CoeffToSlot plan");
    nj_status st = check_batch(c, in, n, re, "nj_coeff_to_slot_batch");
    if (st) return st;
    if (in->level != 0) return fail(NJ_ELEVEL, "nj_coeff_to_slot_batch: input must be at level 0");
    if (!im || !im->data || im->data == re->data) return fail(NJ_EINVAL, "nj_coeff_to_slot_batch: bad output");
    const int lo = c->L - (int)p->lts.size();
    const size_t cout = 2 * (size_t)c->N * (lo + 1);
    std::vector<uint64_t *> rp(n), ip(n);
    for (int z = 0; z < n; z++) rp[z] = re->data + z * cout, ip[z] = im->data + z * cout;
    bool ok;
    Arena A = arena_for(c, cts_batch_words(c, p, std::min(n, kBatch)), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    if ((st = cts_batch(c, p, in->data, n, rp.data(), ip.data(), A, S(stream)))) return st;
    re->level = im->level = lo;
    re->is_ntt = im->is_ntt = 1;
    re->scale = im->scale = in->scale;
    return NJ_OK;
}

nj_status nj_conv2d_block(nj_ctx *c, const nj_plan *p, const nj_ct *in, nj_ct *out, void *stream)
{
    if (!c || !p || p->kind != 0 || p->lts.empty()) return fail(NJ_EINVAL, "nj_conv2d_block: not a conv plan");
    nj_status st = check_batch(c, in, p->lts[0].bi, out, "nj_conv2d_block");
    if (st) return st;
    if (in->level < 1 || in->level > p->lts[0].level)
        return fail(NJ_ELEVEL, "nj_conv2d_block: input level must be in 1..the plan's level");
    const nj_lt_t lt = at_level(p->lts[0], in->level);
    const int l = lt.level;
    const size_t N = c->N, clen = 2 * N * (l + 1), clen_out = 2 * N * l;
    if (out->data < in->data + lt.bi * clen && in->data < out->data + lt.bo * clen_out)
        return fail(NJ_EINVAL, "nj_conv2d_block: outputs overlap the inputs");
    bool ok;
    Arena A = arena_for(c, lt.bo * clen + block_words(c, lt) + N * (l + 2), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    uint64_t *y = A.take(lt.bo * clen);
    hipStream_t s = S(stream);
    if ((st = block_bsgs_apply(c, lt, in->data, y, A, s))) return st;
    if ((st = rescale_batch(c, l, lt.bo, y, out->data, A, s))) return st;
    out->level = l - 1, out->is_ntt = 1, out->scale = in->scale * lt.scale / (double)c->primes[l];
    return NJ_OK;
}

}  // extern "C"
