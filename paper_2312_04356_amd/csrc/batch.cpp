// Jobs of conv -> rescale -> level drop -> ModRaise -> CoeffToSlot -> real split at
// uneven levels: a plain schedule (one job after another), a batched schedule (each conv
// on the fused single-ciphertext path, then CoeffToSlot batched over every conv output,
// where every output is at one level), the batched schedule with the convs of one plan
// grouped across levels (each rotation key read once for the group, at the price of
// unfused transforms), a concurrent schedule, and HIP-graph replays of each.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "exec.h"

using namespace nj;
using namespace nj::ex;

struct nj_batch {
    nj_ctx *c = nullptr;
    uint64_t *buf = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// ------------------------------------------------ one transform, uneven levels

struct MixJob {
    int level;
    const uint64_t *in;  // [2][level+1][N]
    uint64_t *out;       // [2][level+1][N], before the rescale
};

struct Grp {
    int l, z0, K;
    MultiBufs M;
};

// runs of equal level in a level-sorted job list
std::vector<Grp> level_groups(const std::vector<MixJob> &jobs)
{
    std::vector<Grp> g;
    for (int z = 0; z < (int)jobs.size(); z++) {
        if (g.empty() || jobs[z].level != g.back().l) g.push_back(Grp{jobs[z].level, z, 0, {}});
        g.back().K++;
    }
    return g;
}

// limb offset of an arena pointer from the arena base, in units of N words
int limb_off(const nj_ctx *c, const uint64_t *base, const uint64_t *p) { return (int)((p - base) / c->N); }

// NTT launches over the limbs of every level group at once (tables flushed at
// NJ_MAX_LIMBS limbs); each group's limbs are given by `each(g, push)`.  The inverse
// transforms read their limbs from separate source offsets, the forward ones work in
// place.
template <class F>
hipError_t ntt_all(const nj_ctx *c, uint64_t *base, bool inverse, hipStream_t s, F each, int n_groups)
{
    const uint64_t *src = inverse ? base : nullptr;
    LimbTab lt;
    lt.n = 0;
    hipError_t e = hipSuccess;
    auto push = [&](int pidx, int off, int soff) {
        lt.pidx[lt.n] = pidx, lt.off[lt.n] = off, lt.soff[lt.n] = soff;
        if (++lt.n == NJ_MAX_LIMBS) {
            if (e == hipSuccess) e = launch_ntt(c, base, lt, inverse, s, src);
            lt.n = 0;
        }
    };
    for (int g = 0; g < n_groups; g++) each(g, push);
    if (e == hipSuccess && lt.n) e = launch_ntt(c, base, lt, inverse, s, src);
    return e;
}

// ModUp of every group's K polynomials at M.d (packed [K][l+1]) into M.ext; the iNTT
// and NTT launches span all groups, the basis conversions run per level.
nj_status modup_mixed(nj_ctx *c, std::vector<Grp> &gr, uint64_t *base, hipStream_t s)
{
    const size_t N = c->N;
    NJ_HIP(ntt_all(c, base, true, s, [&](int g, auto push) {
        const Grp &q = gr[g];
        for (int z = 0; z < q.K; z++)
            for (int i = 0; i <= q.l; i++)
                push(i, limb_off(c, base, q.M.coef) + z * (q.l + 1) + i, limb_off(c, base, q.M.d) + z * (q.l + 1) + i);
    }, (int)gr.size()));
    for (const Grp &q : gr) {
        const int nd = n_digits(c, q.l), ne = q.l + 1 + c->alpha;
        for (int j0 = 0; j0 < nd; j0 += 4) {
            BconvShared sh;
            sh.nd = std::min(4, nd - j0);
            for (int jj = 0; jj < sh.nd; jj++) {
                const int j = j0 + jj;
                const BconvTab &bt = c->modup[q.l][j];
                sh.m[jj] = bt.m, sh.n_out[jj] = bt.n_out, sh.in_off0[jj] = j * c->alpha;
                sh.hat_inv[jj] = bt.hat_inv, sh.hat[jj] = bt.hat;
                for (int a = 0; a < bt.m; a++) sh.in_pidx[jj][a] = bt.in_pidx[a];
                for (int o = 0; o < bt.n_out; o++)
                    sh.out_pidx[jj][o] = bt.out_pidx[o], sh.out_off[jj][o] = j * ne + bt.out_limb[o];
            }
            BconvPtrs jp;
            for (int z = 0; z < q.K; z++)
                jp.in[z] = q.M.coef + (size_t)z * (q.l + 1) * N, jp.out[z] = q.M.ext + (size_t)z * nd * ne * N;
            NJ_HIP(launch_bconv_multi(c, sh, jp, q.K, s));
        }
    }
    NJ_HIP(ntt_all(c, base, false, s, [&](int g, auto push) {
        const Grp &q = gr[g];
        const int nd = n_digits(c, q.l), ne = q.l + 1 + c->alpha;
        for (int z = 0; z < q.K; z++)
            for (int j = 0; j < nd; j++) {
                const BconvTab &bt = c->modup[q.l][j];
                for (int o = 0; o < bt.n_out; o++)
                    push(bt.out_pidx[o], limb_off(c, base, q.M.ext) + (z * nd + j) * ne + bt.out_limb[o], 0);
            }
    }, (int)gr.size()));
    return NJ_OK;
}

// ModDown of every group's inner products (M.u) and the combine into mj[g]'s outputs
// (accumulating into them when acc); iNTT / NTT launches span all groups.
nj_status ks_down_mixed(nj_ctx *c, std::vector<Grp> &gr, const std::vector<MdJobs> &mj, bool acc, uint64_t *base,
                        hipStream_t s)
{
    const size_t N = c->N;
    const int al = c->alpha;
    NJ_HIP(ntt_all(c, base, true, s, [&](int g, auto push) {
        const Grp &q = gr[g];
        const int ne = q.l + 1 + al;
        for (int z = 0; z < q.K; z++)
            for (int p = 0; p < 2; p++)
                for (int a = 0; a < al; a++)
                    push(c->n_q + a, limb_off(c, base, q.M.pc) + (2 * z + p) * al + a,
                         limb_off(c, base, q.M.u) + (2 * z + p) * ne + q.l + 1 + a);
    }, (int)gr.size()));
    for (const Grp &q : gr) {
        const BconvTab &bt = c->moddown[q.l];
        BconvShared sh;
        sh.nd = 1;
        sh.m[0] = bt.m, sh.n_out[0] = bt.n_out, sh.in_off0[0] = 0, sh.hat_inv[0] = bt.hat_inv, sh.hat[0] = bt.hat;
        for (int a = 0; a < bt.m; a++) sh.in_pidx[0][a] = bt.in_pidx[a];
        for (int o = 0; o < bt.n_out; o++) sh.out_pidx[0][o] = bt.out_pidx[o], sh.out_off[0][o] = o;
        BconvPtrs jp;
        for (int h = 0; h < 2 * q.K; h++)
            jp.in[h] = q.M.pc + (size_t)h * al * N, jp.out[h] = q.M.conv + (size_t)h * (q.l + 1) * N;
        NJ_HIP(launch_bconv_multi(c, sh, jp, 2 * q.K, s));
    }
    NJ_HIP(ntt_all(c, base, false, s, [&](int g, auto push) {
        const Grp &q = gr[g];
        for (int h = 0; h < 2 * q.K; h++)
            for (int i = 0; i <= q.l; i++) push(i, limb_off(c, base, q.M.conv) + h * (q.l + 1) + i, 0);
    }, (int)gr.size()));
    for (size_t g = 0; g < gr.size(); g++)
        NJ_HIP(launch_moddown_multi(c, gr[g].l, mj[g], gr[g].K, 0, gr[g].M.u, gr[g].M.conv,
                                    acc ? mj[g].out[0] : nullptr, s));
    return NJ_OK;
}

size_t mixed_words(const nj_ctx *c, const nj_lt_t &lt, const std::vector<MixJob> &jobs)
{
    const size_t N = c->N, nb = lt.babies.size(), ng = lt.giants.size();
    size_t w = 0;
    for (const Grp &g : level_groups(jobs)) w += multi_words(c, g.l, g.K);
    for (const MixJob &j : jobs) w += 2 * N * (j.level + 1) * (nb + ng);
    return w;
}

// sum_d diag_d (.) (in_z <<< j_d u) for up to NJ_MAX_JOBS ciphertexts sorted by level
// (each at most the plan's level).  Baby steps hoisted per ciphertext; each baby and
// giant rotation is one mixed-level shared-key inner product over all jobs, with ModUp
// and ModDown batched per level group; the multiply-accumulate runs per ciphertext.
nj_status bsgs_apply_mixed(nj_ctx *c, const nj_lt_t &lt, const std::vector<MixJob> &jobs, Arena A, hipStream_t s)
{
    const int n = (int)jobs.size(), nb = (int)lt.babies.size(), ng = (int)lt.giants.size(), nd = lt.n_diag;
    const size_t N = c->N;
    if (n < 1 || n > NJ_MAX_JOBS) return fail(NJ_EINVAL, "mixed transform: 1..16 ciphertexts");
    if (lt.lazy) return fail(NJ_EUNSUPPORTED, "mixed-level transforms run giant steps with one ModDown each");
    for (int b : lt.babies)
        if (b != 0 && !key_of(c, galois_of_rot(c, (long long)b * lt.u))) return fail(NJ_ENOKEY, "missing baby-step key");
    for (int g : lt.giants)
        if (g != 0 && !key_of(c, galois_of_rot(c, (long long)g * lt.n1 * lt.u)))
            return fail(NJ_ENOKEY, "missing giant-step key");
    std::vector<Grp> gr = level_groups(jobs);
    uint64_t *base = A.p;  // every buffer below is N-word aligned from here
    std::vector<int> grp_of(n), idx_in(n);
    for (int q = 0; q < (int)gr.size(); q++) {
        if (!multi_bufs(c, gr[q].l, gr[q].K, A, gr[q].M)) return fail(NJ_ENOMEM, "scratch too small");
        for (int i = 0; i < gr[q].K; i++) grp_of[gr[q].z0 + i] = q, idx_in[gr[q].z0 + i] = i;
    }
    std::vector<std::vector<uint64_t *>> baby(n, std::vector<uint64_t *>(nb, nullptr));
    std::vector<uint64_t *> inner(n);
    for (int z = 0; z < n; z++) {
        const size_t clen = 2 * N * (jobs[z].level + 1);
        for (int b = 0; b < nb; b++) baby[z][b] = A.take(clen);
        inner[z] = A.take(clen * ng);
        if (!inner[z]) return fail(NJ_ENOMEM, "scratch too small");
    }
    auto ne_of = [&](int l) { return (size_t)(l + 1 + c->alpha); };
    auto ext_of = [&](int z) {
        const Grp &g = gr[grp_of[z]];
        return g.M.ext + (size_t)idx_in[z] * n_digits(c, g.l) * ne_of(g.l) * N;
    };
    auto u_of = [&](int z) { return gr[grp_of[z]].M.u + (size_t)idx_in[z] * 2 * ne_of(jobs[z].level) * N; };
    nj_status st;
    // baby steps
    if (nb > 1) {
        for (Grp &g : gr) {
            const size_t plen = N * (g.l + 1);
            for (int i = 0; i < g.K; i++)
                NJ_HIP(hipMemcpyAsync(g.M.d + i * plen, jobs[g.z0 + i].in + plen, plen * 8, hipMemcpyDeviceToDevice, s));
        }
        if ((st = modup_mixed(c, gr, base, s))) return st;
        for (int b = 0; b < nb; b++) {
            if (lt.babies[b] == 0) continue;
            const uint32_t ge = galois_of_rot(c, (long long)lt.babies[b] * lt.u);
            KeyJobsX kj;
            for (int z = 0; z < n; z++) {
                kj.ext[z] = ext_of(z), kj.d[z] = jobs[z].in + N * (jobs[z].level + 1), kj.u[z] = u_of(z);
                kj.g[z] = ge, kj.lv[z] = jobs[z].level;
            }
            NJ_HIP(launch_key_ip_mixed(c, kj, n, key_of(c, ge), s));
            std::vector<MdJobs> mj(gr.size());
            for (size_t q = 0; q < gr.size(); q++)
                for (int i = 0; i < gr[q].K; i++)
                    mj[q].add[i] = jobs[gr[q].z0 + i].in, mj[q].g_add[i] = ge, mj[q].out[i] = baby[gr[q].z0 + i][b];
            if ((st = ks_down_mixed(c, gr, mj, false, base, s))) return st;
        }
    }
    // every giant step's inner sum, one ciphertext at a time
    std::vector<int> gidx(nd), bidx(nd);
    for (int d = 0; d < nd; d++) {
        gidx[d] = (int)(std::lower_bound(lt.giants.begin(), lt.giants.end(), lt.g_of[d]) - lt.giants.begin());
        bidx[d] = (int)(std::lower_bound(lt.babies.begin(), lt.babies.end(), lt.i_of[d]) - lt.babies.begin());
    }
    std::vector<MacEntry> ent;
    for (int d = 0; d < nd; d++)
        if (lt.nz.empty() || lt.nz[d]) ent.push_back(MacEntry{gidx[d], bidx[d], d});
    for (int z = 0; z < n; z++) {
        std::vector<const uint64_t *> bs(nb);
        for (int b = 0; b < nb; b++) bs[b] = lt.babies[b] == 0 ? jobs[z].in : baby[z][b];
        if ((st = mac_general(c, jobs[z].level, bs, ng, ent, lt.d_diag, lt.dl, inner[z], s))) return st;
    }
    // giant steps, accumulated into the outputs
    bool have = false;
    for (int g = 0; g < ng; g++)
        if (lt.giants[g] == 0) {
            for (int z = 0; z < n; z++) {
                const size_t clen = 2 * N * (jobs[z].level + 1);
                NJ_HIP(hipMemcpyAsync(jobs[z].out, inner[z] + (size_t)g * clen, clen * 8, hipMemcpyDeviceToDevice, s));
            }
            have = true;
        }
    for (int g = 0; g < ng; g++) {
        if (lt.giants[g] == 0) continue;
        const uint32_t ge = galois_of_rot(c, (long long)lt.giants[g] * lt.n1 * lt.u);
        for (Grp &q : gr) {
            const size_t plen = N * (q.l + 1), clen = 2 * plen;
            AutoJobs aj;
            for (int i = 0; i < q.K; i++)
                aj.in[i] = inner[q.z0 + i] + (size_t)g * clen + plen, aj.out[i] = q.M.d + i * plen, aj.g[i] = ge;
            NJ_HIP(launch_automorph_multi(c, aj, q.K, q.l + 1, s));
        }
        if ((st = modup_mixed(c, gr, base, s))) return st;
        KeyJobsX kj;
        for (int z = 0; z < n; z++) {
            const Grp &q = gr[grp_of[z]];
            kj.ext[z] = ext_of(z), kj.d[z] = q.M.d + idx_in[z] * N * (q.l + 1), kj.u[z] = u_of(z);
            kj.g[z] = 1, kj.lv[z] = jobs[z].level;
        }
        NJ_HIP(launch_key_ip_mixed(c, kj, n, key_of(c, ge), s));
        std::vector<MdJobs> mj(gr.size());
        for (size_t q = 0; q < gr.size(); q++) {
            const size_t clen = 2 * N * (gr[q].l + 1);
            for (int i = 0; i < gr[q].K; i++)
                mj[q].add[i] = inner[gr[q].z0 + i] + (size_t)g * clen, mj[q].g_add[i] = ge,
                mj[q].out[i] = jobs[gr[q].z0 + i].out;
        }
        if ((st = ks_down_mixed(c, gr, mj, have, base, s))) return st;
        have = true;
    }
    return NJ_OK;
}

// ----------------------------------------------------------------- job lists

int job_bi(const nj_job &j) { return j.conv->lts[0].bi; }
int job_bo(const nj_job &j) { return j.conv->lts[0].bo; }

nj_status check_jobs(nj_ctx *c, const nj_plan *cts, const nj_job *jobs, int n)
{
    if (!c || !cts || cts->kind != 1 || cts->lts.empty()) return fail(NJ_EINVAL, "batch: not a CoeffToSlot plan");
    if (!jobs || n < 1) return fail(NJ_EINVAL, "batch: no jobs");
    for (int z = 0; z < n; z++) {
        const nj_job &j = jobs[z];
        if (!j.conv || j.conv->kind != 0 || j.conv->lts.empty()) return fail(NJ_EINVAL, "batch: job without a conv plan");
        nj_status st = check_ct(c, &j.in, "batch job input");
        if (st) return st;
        if (j.in.level < 1 || j.in.level > j.conv->lts[0].level)
            return fail(NJ_ELEVEL, "batch: job input level must be in 1..its plan's level");
        if (!j.re.data || !j.im.data) return fail(NJ_EINVAL, "batch: job without outputs");
    }
    return NJ_OK;
}

// Work units of the batched schedule: single-block jobs of one plan sorted by level,
// at most NJ_MAX_JOBS per unit; block jobs one per unit.
std::vector<std::vector<int>> make_units(const nj_job *jobs, int n)
{
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (jobs[a].conv != jobs[b].conv) return jobs[a].conv < jobs[b].conv;
        return jobs[a].in.level < jobs[b].in.level;
    });
    std::vector<std::vector<int>> units;
    for (int z : order) {
        const bool blk = job_bi(jobs[z]) != 1 || job_bo(jobs[z]) != 1;
        if (blk || units.empty() || (int)units.back().size() == NJ_MAX_JOBS ||
            jobs[units.back()[0]].conv != jobs[z].conv || job_bi(jobs[units.back()[0]]) != 1 ||
            job_bo(jobs[units.back()[0]]) != 1)
            units.push_back({});
        units.back().push_back(z);
    }
    return units;
}

std::vector<MixJob> unit_jobs(const nj_job *jobs, const std::vector<int> &u)
{
    std::vector<MixJob> mj;
    for (int z : u) mj.push_back(MixJob{jobs[z].in.level, jobs[z].in.data, nullptr});
    return mj;
}

// worker streams (defined with the concurrent schedule below)
int n_workers(const nj_ctx *c, int n);
template <class Run>
nj_status on_workers(nj_ctx *c, const std::vector<double> &cost, size_t per, Arena A0, hipStream_t s, Run run);

// one job's conv -> rescale -> level drop: its bo level-0 outputs at out [bo][2][1][N]
size_t conv_words(nj_ctx *c, const nj_job &j)
{
    const size_t N = c->N;
    const nj_lt_t lt = at_level(j.conv->lts[0], j.in.level);
    const size_t l = lt.level;
    return lt.bo * 2 * N * (l + 1) + (lt.bi == 1 && lt.bo == 1 ? bsgs_words(c, lt) : block_words(c, lt)) + N * (l + 2);
}

nj_status conv_to_pool(nj_ctx *c, const nj_job &j, uint64_t *out, Arena A, hipStream_t s)
{
    const size_t N = c->N;
    const nj_lt_t lt = at_level(j.conv->lts[0], j.in.level);
    const size_t clen = 2 * N * (lt.level + 1);
    uint64_t *y = A.take(lt.bo * clen);
    if (!y) return fail(NJ_ENOMEM, "scratch too small");
    // only the limbs the rescale and the level drop read
    nj_status st = lt.bi == 1 && lt.bo == 1 ? bsgs_apply(c, lt, j.in.data, y, lt.hoist ? 1 : 0, A, s, nullptr, nullptr, true)
                                            : block_bsgs_apply(c, lt, j.in.data, y, A, s);
    for (int ob = 0; ob < lt.bo && !st; ob++) st = rescale(c, lt.level, y + ob * clen, out + ob * 2 * N, A, s, 1);
    return st;
}

// relative cost of a job's conv (key switches x limbs), to balance the workers
double conv_cost(const nj_job &j)
{
    const nj_lt_t lt = at_level(j.conv->lts[0], j.in.level);
    return (double)(lt.level + 1) * ((double)lt.babies.size() * lt.bi + (double)lt.giants.size() * lt.bo);
}

size_t conv_worker_words(nj_ctx *c, const nj_job *jobs, int n)
{
    size_t w = 0;
    for (int z = 0; z < n; z++) w = std::max(w, conv_words(c, jobs[z]));
    return (w + 255) / 256 * 256;
}

size_t batched_words(nj_ctx *c, const nj_plan *cts, const nj_job *jobs, int n, bool mixed)
{
    const size_t N = c->N;
    size_t outs = 0, phase1 = 0;
    for (int z = 0; z < n; z++) outs += job_bo(jobs[z]);
    if (!mixed) phase1 = conv_worker_words(c, jobs, n) * n_workers(c, n);
    for (const auto &u : mixed ? make_units(jobs, n) : std::vector<std::vector<int>>()) {
        const nj_job &j0 = jobs[u[0]];
        size_t w = 0;
        int lmax = 0;
        if (job_bi(j0) != 1 || job_bo(j0) != 1) {
            const nj_lt_t lt = at_level(j0.conv->lts[0], j0.in.level);
            lmax = lt.level;
            w = lt.bo * 2 * N * (lt.level + 1) + block_words(c, lt);
        } else if (j0.conv->lts[0].lazy) {  // one job at a time (conv_to_pool)
            for (int z : u) w = std::max(w, conv_words(c, jobs[z]));
        } else {
            std::vector<MixJob> mj = unit_jobs(jobs, u);
            for (const MixJob &m : mj) w += 2 * N * (m.level + 1), lmax = std::max(lmax, m.level);
            w += mixed_words(c, j0.conv->lts[0], mj);
        }
        phase1 = std::max(phase1, w + N * (lmax + 2));
    }
    const size_t phase2 = cts_batch_words(c, cts, (int)std::min<size_t>(outs, kBatch));
    return outs * 2 * N + std::max(phase1, phase2);
}

// mode 3's conv phase: single-block jobs of one plan together across their levels,
// block jobs one at a time; the level-0 outputs into pool
nj_status convs_across_levels(nj_ctx *c, const nj_job *jobs, int n, const std::vector<size_t> &off, uint64_t *pool,
                              Arena A, hipStream_t s)
{
    const size_t N = c->N;
    nj_status st;
    for (const auto &u : make_units(jobs, n)) {
        Arena B = A;
        const nj_job &j0 = jobs[u[0]];
        if (job_bi(j0) != 1 || job_bo(j0) != 1) {
            const nj_lt_t lt = at_level(j0.conv->lts[0], j0.in.level);
            const size_t clen = 2 * N * (lt.level + 1);
            uint64_t *y = B.take(lt.bo * clen);
            if (!y) return fail(NJ_ENOMEM, "scratch too small");
            if ((st = block_bsgs_apply(c, lt, j0.in.data, y, B, s))) return st;
            for (int ob = 0; ob < lt.bo; ob++)
                if ((st = rescale(c, lt.level, y + ob * clen, pool + (off[u[0]] + ob) * 2 * N, B, s, 1))) return st;
            continue;
        }
        if (j0.conv->lts[0].lazy) {  // the mixed-level path has no lazy giant steps: one job at a time
            for (int z : u)
                if ((st = conv_to_pool(c, jobs[z], pool + off[z] * 2 * N, B, s))) return st;
            continue;
        }
        std::vector<MixJob> mj = unit_jobs(jobs, u);
        for (MixJob &m : mj)
            if (!(m.out = B.take(2 * N * (m.level + 1)))) return fail(NJ_ENOMEM, "scratch too small");
        if ((st = bsgs_apply_mixed(c, j0.conv->lts[0], mj, B, s))) return st;
        for (size_t i = 0; i < u.size(); i++)
            if ((st = rescale(c, mj[i].level, mj[i].out, pool + off[u[i]] * 2 * N, B, s, 1))) return st;
    }
    return NJ_OK;
}

nj_status run_batched(nj_ctx *c, const nj_plan *cts, const nj_job *jobs, int n, bool mixed, Arena A, hipStream_t s)
{
    const size_t N = c->N, clo = 2 * N * (c->L - cts->lts.size() + 1);
    std::vector<size_t> off(n + 1, 0);
    for (int z = 0; z < n; z++) off[z + 1] = off[z] + job_bo(jobs[z]);
    uint64_t *pool = A.take(off[n] * 2 * N);  // level-0 conv outputs [outs][2][1][N]
    if (!pool) return fail(NJ_ENOMEM, "scratch too small");
    nj_status st;
    if (!mixed) {  // every conv on its fused path, the jobs spread over the worker streams
        std::vector<double> cost(n);
        for (int z = 0; z < n; z++) cost[z] = conv_cost(jobs[z]);
        st = on_workers(c, cost, conv_worker_words(c, jobs, n), A, s, [&](int z, Arena B, hipStream_t w) {
            return conv_to_pool(c, jobs[z], pool + off[z] * 2 * N, B, w);
        });
        if (st) return st;
    } else if ((st = convs_across_levels(c, jobs, n, off, pool, A, s))) {
        return st;
    }
    std::vector<uint64_t *> re(off[n]), im(off[n]);
    for (int z = 0; z < n; z++)
        for (int ob = 0; ob < job_bo(jobs[z]); ob++)
            re[off[z] + ob] = jobs[z].re.data + ob * clo, im[off[z] + ob] = jobs[z].im.data + ob * clo;
    return cts_batch(c, cts, pool, (int)off[n], re.data(), im.data(), A, s);
}

size_t plain_words(nj_ctx *c, const nj_plan *cts, const nj_job *jobs, int n)
{
    const size_t N = c->N;
    size_t w = 0;
    for (int z = 0; z < n; z++) {
        const nj_lt_t lt = at_level(jobs[z].conv->lts[0], jobs[z].in.level);
        const size_t l = lt.level, bo = lt.bo;
        const size_t conv = (lt.bi == 1 && bo == 1 ? bsgs_words(c, lt) : block_words(c, lt)) + N * (l + 2);
        w = std::max(w, bo * 2 * N * (2 * l + 2) + std::max(conv, cts_single_words(c, cts)));
    }
    return w;
}

// one job after another; each step as the single-job calls run it
nj_status run_plain(nj_ctx *c, const nj_plan *cts, const nj_job *jobs, int n, Arena A0, hipStream_t s)
{
    const size_t N = c->N, clo = 2 * N * (c->L - cts->lts.size() + 1);
    nj_status st;
    for (int z = 0; z < n; z++) {
        Arena A = A0;
        const nj_job &j = jobs[z];
        const nj_lt_t lt = at_level(j.conv->lts[0], j.in.level);
        const int l = lt.level, bo = lt.bo;
        const size_t clen = 2 * N * (l + 1), clen1 = 2 * N * l;
        uint64_t *y = A.take(bo * clen), *r = A.take(bo * clen1), *lo = A.take(bo * 2 * N);
        if (!lo) return fail(NJ_ENOMEM, "scratch too small");
        if (lt.bi == 1 && bo == 1) {  // as nj_conv2d_cins: the rescale's first pass rides on the last ModDown
            if ((st = bsgs_rescale(c, lt, j.in.data, y, r, A, s))) return st;
        } else {  // as nj_conv2d_block
            if ((st = block_bsgs_apply(c, lt, j.in.data, y, A, s))) return st;
            if ((st = rescale_batch(c, l, bo, y, r, A, s))) return st;
        }
        for (int ob = 0; ob < bo; ob++) {
            NJ_HIP(hipMemcpy2DAsync(lo + ob * 2 * N, N * 8, r + ob * clen1, l * N * 8, N * 8, 2, hipMemcpyDeviceToDevice,
                                    s));
        }
        for (int ob = 0; ob < bo; ob++)
            if ((st = cts_single(c, cts, lo + ob * 2 * N, j.re.data + ob * clo, j.im.data + ob * clo, A, s))) return st;
    }
    return NJ_OK;
}

// ------------------------------------------------ concurrent plain schedule
//
// Mode 2: every job runs as in the plain schedule (so the outputs are bit-identical),
// but the jobs are spread over worker streams, each with its own part of the scratch:
// the latency-bound kernels of different jobs (transform tile passes, the fused key
// inner products at two waves per SIMD, ModDown combines) then fill the GPU together.
// The workers fork from the caller's stream and join back into it through events, so
// the schedule also captures into one HIP graph.


// estimated relative cost of a job, to balance the workers: key switches x limbs of
// its conv, plus the CoeffToSlot every output block runs at the top levels
double job_cost(const nj_plan *cts, const nj_job &j)
{
    const nj_lt_t lt = at_level(j.conv->lts[0], j.in.level);
    const double conv = (double)(lt.level + 1) * ((double)lt.babies.size() * lt.bi + (double)lt.giants.size() * lt.bo);
    double ct = 0;
    for (const auto &g : cts->lts) ct += (double)(g.level + 1) * (double)(g.babies.size() + g.giants.size());
    return conv + lt.bo * ct;
}


size_t worker_words(nj_ctx *c, const nj_plan *cts, const nj_job *jobs, int n)
{
    return (plain_words(c, cts, jobs, n) + 255) / 256 * 256;  // each worker's part 2 KiB aligned
}

int n_workers(const nj_ctx *c, int n) { return std::max(1, std::min(std::min(c->batch_workers, kMaxWorkers), n)); }

// Runs run(z, arena, stream) for every job z on the worker streams: longest-processing-
// time assignment by cost (the costliest job to the least-loaded worker), each worker
// with `per` words of A0; the workers fork from s and join back into it.
template <class Run>
nj_status on_workers(nj_ctx *c, const std::vector<double> &cost, size_t per, Arena A0, hipStream_t s, Run run)
{
    nj_status st = workers_ready(c);
    if (st) return st;
    const int n = (int)cost.size(), W = n_workers(c, n);
    if (A0.left < per * W) return fail(NJ_ENOMEM, "scratch too small");
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<double> load(W, 0.0);
    std::vector<std::vector<int>> part(W);
    for (int z : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        part[k].push_back(z);
        load[k] += cost[z];
    }
    NJ_HIP(hipEventRecord(c->fork_ev, s));
    for (int k = 0; k < W; k++) NJ_HIP(hipStreamWaitEvent(c->workers[k], c->fork_ev, 0));
    for (int k = 0; k < W && !st; k++)
        for (int z : part[k]) {
            st = run(z, Arena{A0.p + (size_t)k * per, per}, c->workers[k]);
            if (st) break;
        }
    // the workers always join back, also after an error, so no stream is left forked
    for (int k = 0; k < W; k++) {
        NJ_HIP(hipEventRecord(c->worker_done[k], c->workers[k]));
        NJ_HIP(hipStreamWaitEvent(s, c->worker_done[k], 0));
    }
    return st;
}

nj_status run_concurrent(nj_ctx *c, const nj_plan *cts, const nj_job *jobs, int n, Arena A0, hipStream_t s)
{
    std::vector<double> cost(n);
    for (int z = 0; z < n; z++) cost[z] = job_cost(cts, jobs[z]);
    return on_workers(c, cost, worker_words(c, cts, jobs, n), A0, s,
                      [&](int z, Arena B, hipStream_t w) { return run_plain(c, cts, &jobs[z], 1, B, w); });
}

size_t schedule_words(nj_ctx *c, const nj_plan *cts, const nj_job *jobs, int n, int mode)
{
    if (mode == 2) return worker_words(c, cts, jobs, n) * n_workers(c, n);
    return mode ? batched_words(c, cts, jobs, n, mode == 3) : plain_words(c, cts, jobs, n);
}

nj_status run_schedule(nj_ctx *c, const nj_plan *cts, const nj_job *jobs, int n, int mode, Arena A, hipStream_t s)
{
    if (mode == 2) return run_concurrent(c, cts, jobs, n, A, s);
    return mode ? run_batched(c, cts, jobs, n, mode == 3, A, s) : run_plain(c, cts, jobs, n, A, s);
}

void set_outputs(nj_ctx *c, const nj_plan *cts, const nj_job *jobs, int n)
{
    for (int z = 0; z < n; z++) {
        nj_job &j = const_cast<nj_job &>(jobs[z]);
        const nj_lt_t &lt = j.conv->lts[0];
        j.re.level = j.im.level = c->L - (int)cts->lts.size();
        j.re.is_ntt = j.im.is_ntt = 1;
        j.re.scale = j.im.scale = j.in.scale * lt.scale / (double)c->primes[j.in.level];
    }
}

}  // namespace

// the context's worker streams (default priority) and their fork/join events, made once
nj_status nj::ex::workers_ready(nj_ctx *c)
{
    while ((int)c->workers.size() < kMaxWorkers) {
        hipStream_t w;
        hipEvent_t e;
        NJ_HIP(hipStreamCreateWithFlags(&w, hipStreamNonBlocking));
        c->workers.push_back(w);
        NJ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->worker_done.push_back(e);
    }
    if (!c->fork_ev) NJ_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    return NJ_OK;
}

extern "C" {

nj_status nj_batch_run(nj_ctx *c, const nj_plan *cts, nj_job *jobs, int n, int mode, void *stream)
{
    nj_status st = check_jobs(c, cts, jobs, n);
    if (st) return st;
    if (mode < 0 || mode > 3)
        return fail(NJ_EINVAL, "nj_batch_run: mode must be 0 (plain), 1 (batched), 2 (concurrent) or 3 (batched, "
                               "convs grouped across levels)");
    bool ok;
    Arena A = arena_for(c, schedule_words(c, cts, jobs, n, mode), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    st = run_schedule(c, cts, jobs, n, mode, A, S(stream));
    if (st) return st;
    set_outputs(c, cts, jobs, n);
    return NJ_OK;
}

nj_status nj_batch_workers(nj_ctx *c, int n)
{
    if (!c || n < 1 || n > kMaxWorkers) return fail(NJ_EINVAL, "nj_batch_workers: 1..4 worker streams");
    c->batch_workers = n;
    return NJ_OK;
}

nj_status nj_batch_create(nj_ctx *c, const nj_plan *cts, nj_job *jobs, int n, nj_batch **out)
{
    return nj_batch_create_mode(c, cts, jobs, n, 1, out);
}

nj_status nj_batch_create_mode(nj_ctx *c, const nj_plan *cts, nj_job *jobs, int n, int mode, nj_batch **out)
{
    nj_status st = check_jobs(c, cts, jobs, n);
    if (st) return st;
    if (!out) return fail(NJ_EINVAL, "nj_batch_create: null output");
    if (mode < 0 || mode > 3) return fail(NJ_EINVAL, "nj_batch_create: mode must be 0, 1, 2 or 3");
    if ((mode == 1 || mode == 2) && (st = workers_ready(c))) return st;  // streams made before capture
    const size_t words = schedule_words(c, cts, jobs, n, mode);
    nj_batch *b = new nj_batch();
    b->c = c;
    auto bail = [&](nj_status e) {
        nj_batch_destroy(b);
        return e;
    };
    if (hipMalloc(&b->buf, words * 8) != hipSuccess) return bail(fail(NJ_ENOMEM, "nj_batch_create: device memory"));
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(NJ_EDEVICE, "nj_batch_create: stream"));
    const bool prof = c->prof;
    c->prof = false;  // no event records inside the graph
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        c->prof = prof;
        return bail(fail(NJ_EDEVICE, "nj_batch_create: stream capture"));
    }
    st = run_schedule(c, cts, jobs, n, mode, Arena{b->buf, words}, b->cap);
    const hipError_t e = hipStreamEndCapture(b->cap, &b->graph);
    c->prof = prof;
    if (st) return bail(st);
    if (e != hipSuccess) return bail(fail(NJ_EDEVICE, std::string("nj_batch_create: capture: ") + hipGetErrorString(e)));
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
        return bail(fail(NJ_EDEVICE, "nj_batch_create: graph instantiation"));
    set_outputs(c, cts, jobs, n);
    *out = b;
    return NJ_OK;
}

nj_status nj_batch_launch(nj_batch *b, void *stream)
{
    if (!b || !b->exec) return fail(NJ_EINVAL, "nj_batch_launch: no batch");
    NJ_HIP(hipGraphLaunch(b->exec, S(stream)));
    return NJ_OK;
}

void nj_batch_destroy(nj_batch *b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->buf) (void)hipFree(b->buf);
    delete b;
}

}  // extern "C"
