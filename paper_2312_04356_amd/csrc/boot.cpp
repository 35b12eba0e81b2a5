// Bootstrapping after CoeffToSlot (Sec. 2.4, Algorithm 1): HMult with relinearisation,
// integer-constant multiplication, ModEval by a scale-exact Chebyshev evaluation and
// double angles, Re + i Im, and StoC1 = S_{l <- 1}.
//
// Scale rules (every integer constant is a fixed function of float64 scales):
//   HMult: scale s_a s_b / q_l.  const_mult(ct, c, lam, tau): level lam + 1, times the
//   integer round(c tau q_{lam+1} / s), rescale -> (lam, tau).  add_const: + round(c s).
// ModEval: x = t / (K P) is the input read at scale K q_0; one integer multiply and
// rescale bring the scale near 2^48; Chebyshev series of degree 63 by baby steps
// T_1..T_7 and giant steps T_8, T_16, T_32 (T_2j = 2 T_j^2 - 1, T_{a+b} = 2 T_a T_b -
// T_{a-b}, Chebyshev division p = q T_G + r); then D(y) = 2 y^2 - 1 r times; the result
// read at scale s_y 2 pi s_0 / q_0 is the message.
#include <hip/hip_runtime.h>

#include <cmath>
#include <initializer_list>
#include <vector>

#include "exec.h"

using namespace nj;
using namespace nj::ex;

namespace {

constexpr int kChebDegree = 63;

struct Cx {
    uint64_t *d = nullptr;  // [K][2][l+1][N], evaluation form (K ciphertexts packed)
    int l = 0;
    double s = 0.0;
};

// Scratch of the parts of one ModEval that run on worker streams: the Chebyshev basis
// products T3, then T5, T6, T7 (slots 0..3, kBranchSlots each), the quotient of the
// series' top division (slot 4, kTreeSlots), and one key-switch arena per worker.
constexpr int kBranchSlots = 8, kTreeSlots = 24, kBranchWorkers = 3;
struct BranchMem {
    Arena slots[5];
    Arena ks[kBranchWorkers];
};

// Ciphertext buffers of one evaluation: fixed-size slots (K level-lmax ciphertexts
// each) from an arena with a free list; the key-switch scratch is a separate arena.
// Every operation applies to the K packed ciphertexts at once (K > 1 needs N >= 8192).
// Independent products can run as branches: an Ev on a worker stream with its own slots
// and scratch, forked after the values it reads are enqueued and joined before its
// result is used, so every value is computed by the same kernels as in one stream.
class Ev {
  public:
    Ev(nj_ctx *c, int lmax, Arena cts, Arena ks, hipStream_t s, int K = 1)
        : c(c), N(c->N), lmax(lmax), K(K), cts(cts), ks(ks), s(s)
    {
        relin = key_of(c, 0);
        if (!relin) err = fail(NJ_ENOKEY, "no relinearisation key (Galois element 0)");
    }
    nj_ctx *c;
    size_t N;
    int lmax, K;
    Arena cts, ks;
    hipStream_t s;
    int wid = -1;  // worker stream of a branch
    nj_status err = NJ_OK;
    const uint64_t *relin = nullptr;
    std::vector<uint64_t *> free_;

    Ev branch(int w, Arena slots, Arena kscratch) const
    {
        Ev b(c, lmax, slots, kscratch, c->workers[w], K);
        b.wid = w;
        for (int j = 0; j < 33; j++) b.T[j] = T[j];
        return b;
    }
    void fork(std::initializer_list<Ev *> bs)
    {
        check(hipEventRecord(c->fork_ev, s));
        for (Ev *b : bs) check(hipStreamWaitEvent(b->s, c->fork_ev, 0));
    }
    void join(Ev &b)
    {
        check(hipEventRecord(c->worker_done[b.wid], b.s));
        check(hipStreamWaitEvent(s, c->worker_done[b.wid], 0));
        check(b.err);
    }

    static size_t slots_needed() { return 48; }
    size_t slot_words() const { return (size_t)K * 2 * N * (lmax + 1); }
    size_t cstride(int l) const { return 2 * N * (l + 1); }  // words between packed ciphertexts
    bool ok() const { return err == NJ_OK; }
    void check(hipError_t e)
    {
        if (e != hipSuccess && err == NJ_OK) err = fail(NJ_EDEVICE, hipGetErrorString(e));
    }
    void check(nj_status st)
    {
        if (st != NJ_OK && err == NJ_OK) err = st;
    }

    Cx alloc(int l, double sc)
    {
        Cx x;
        x.l = l, x.s = sc;
        if (!free_.empty()) {
            x.d = free_.back();
            free_.pop_back();
        } else if (!(x.d = cts.take(slot_words()))) {
            if (err == NJ_OK) err = fail(NJ_ENOMEM, "ModEval: ciphertext pool exhausted");
        }
        return x;
    }
    void release(Cx &x)
    {
        if (x.d) free_.push_back(x.d);
        x.d = nullptr;
    }
    LimbConsts residues(long long k, int n_limbs) const
    {
        LimbConsts kc;
        for (int i = 0; i < n_limbs; i++) {
            const long long q = (long long)c->primes[i];
            long long r = k % q;
            if (r < 0) r += q;
            kc.v[i] = (double)r;
        }
        return kc;
    }
    // x rescaled by q_l into o (both packed)
    void rescale_into(const Cx &x, Cx &o, Arena A) { check(rescale(c, x.l, x.d, o.d, A, s, -1, 2 * K)); }

    Cx add(const Cx &a, const Cx &b, int op)  // op 0: a + b, 1: a - b (same level)
    {
        Cx o = alloc(a.l, a.s);
        if (!ok()) return o;
        LimbTab lt;
        lt.n = 2 * K * (a.l + 1);
        for (int k = 0; k < lt.n; k++) lt.pidx[k] = k % (a.l + 1), lt.off[k] = k;
        check(launch_elementwise(c, op, a.d, b.d, o.d, lt, s));
        return o;
    }
    void add_const(Cx &x, double v)
    {
        const long long k = (long long)std::nearbyint(v * x.s);
        for (int z = 0; z < K && ok(); z++)
            check(launch_add_int(c, x.d + z * cstride(x.l), x.l + 1, residues(k, x.l + 1), s));
    }
    Cx zero(int l, double sc)
    {
        Cx o = alloc(l, sc);
        if (ok()) check(launch_zero(c, o.d, K * cstride(l), s));
        return o;
    }
    // tensor product, relinearisation, rescale
    Cx hmult(const Cx &a, const Cx &b)
    {
        const int l = std::min(a.l, b.l);
        Cx t = alloc(l, 0.0), d2 = alloc(l, 0.0);  // t [K][2][l+1], d2 [K][l+1]
        Cx o = alloc(l - 1, a.s * b.s / (double)c->primes[l]);
        if (!ok()) return o;
        for (int z = 0; z < K; z++)
            check(launch_tensor(c, a.d + z * cstride(a.l), N * (a.l + 1), b.d + z * cstride(b.l), N * (b.l + 1),
                                t.d + z * cstride(l), d2.d + z * N * (l + 1), l, s));
        Arena A = ks;
        MultiBufs M;  // the batched key-switch path: its fused kernels, one job per ciphertext
        if (!multi_bufs(c, l, K, A, M)) {
            check(fail(NJ_ENOMEM, "ModEval: key-switch scratch"));
            return o;
        }
        const bool f = fuse_ip(c, l);
        check(modup_multi(c, l, K, d2.d, M, s, -1, !f));
        const size_t nd = n_digits(c, l), ne = l + 1 + c->alpha;
        KeyJobs kj;
        MdJobs mj;
        for (int z = 0; z < K; z++) {
            kj.ext[z] = M.ext + z * nd * ne * N, kj.d[z] = d2.d + z * N * (l + 1), kj.key[z] = relin, kj.g[z] = 1;
            mj.add[z] = nullptr, mj.g_add[z] = 1, mj.out[z] = t.d + z * cstride(l);
        }
        check(f ? ks_fused(c, l, K, kj, mj, 0, t.d, M, s) : ks_multi(c, l, K, kj, mj, 0, t.d, M, s));  // t += the switched d2
        rescale_into(t, o, A);
        release(t), release(d2);
        return o;
    }
    // c * x at level lam with recorded scale tau; d == nullptr when the constant is 0
    Cx const_mult(const Cx &x, double v, int lam, double tau)
    {
        const long long k = (long long)std::nearbyint(v * tau * (double)c->primes[lam + 1] / x.s);
        Cx o;
        if (k == 0 || !ok()) return o;
        Cx t = alloc(lam + 1, 0.0);
        o = alloc(lam, tau);
        if (!ok()) return o;
        check(launch_mul_int(c, x.d, N * (x.l + 1), t.d, lam + 2, residues(k, lam + 2), s, 0, 2 * K));
        rescale_into(t, o, ks);
        release(t);
        return o;
    }
    Cx sq_minus1(const Cx &a)  // 2 a^2 - 1
    {
        Cx p = hmult(a, a);
        Cx o = add(p, p, 0);
        release(p);
        add_const(o, -1.0);
        return o;
    }
    Cx prod_minus(const Cx &a, const Cx &b, const Cx &cc)  // 2 a b - c
    {
        Cx p = hmult(a, b);
        Cx c2 = const_mult(cc, 1.0, p.l, p.s);
        Cx p2 = add(p, p, 0);
        Cx o = add(p2, c2, 1);
        release(p), release(c2), release(p2);
        return o;
    }

    Cx T[33];
    // bm: T3 alongside T4, then T5, T6, T7 alongside T8, on worker streams
    void basis(const Cx &x, const BranchMem *bm = nullptr)
    {
        T[1] = x;
        T[2] = sq_minus1(T[1]);
        if (!bm) {
            T[3] = prod_minus(T[1], T[2], T[1]);
            T[4] = sq_minus1(T[2]);
            T[5] = prod_minus(T[2], T[3], T[1]);
            T[6] = sq_minus1(T[3]);
            T[7] = prod_minus(T[3], T[4], T[1]);
            T[8] = sq_minus1(T[4]);
        } else {
            Ev b3 = branch(0, bm->slots[0], bm->ks[0]);
            fork({&b3});
            const Cx t3 = b3.prod_minus(T[1], T[2], T[1]);
            T[4] = sq_minus1(T[2]);
            join(b3);
            T[3] = t3;
            Ev b5 = branch(0, bm->slots[1], bm->ks[0]), b6 = branch(1, bm->slots[2], bm->ks[1]),
               b7 = branch(2, bm->slots[3], bm->ks[2]);
            fork({&b5, &b6, &b7});
            const Cx t5 = b5.prod_minus(T[2], T[3], T[1]);
            const Cx t6 = b6.sq_minus1(T[3]);
            const Cx t7 = b7.prod_minus(T[3], T[4], T[1]);
            T[8] = sq_minus1(T[4]);
            join(b5), join(b6), join(b7);
            T[5] = t5, T[6] = t6, T[7] = t7;
        }
        T[16] = sq_minus1(T[8]);
        T[32] = sq_minus1(T[16]);
    }

    // bm (the top call): the quotient of the top division on a worker stream alongside
    // the remainder
    Cx eval(const std::vector<double> &cf, int lam, double tau, const BranchMem *bm = nullptr)
    {
        const int d = (int)cf.size() - 1;
        if (d < 8 && c->eval_order == 0) {
            // each term c_j T_j brought to level lam, scale tau by its own constant multiply
            // and rescale, then the terms summed
            Cx acc;
            for (int j = 1; j <= d; j++) {
                if (cf[j] == 0.0) continue;
                Cx t = const_mult(T[j], cf[j], lam, tau);
                if (!t.d) continue;
                if (!acc.d) {
                    acc = t;
                } else {
                    Cx sum = add(acc, t, 0);
                    release(acc), release(t);
                    acc = sum;
                }
            }
            if (!acc.d) acc = zero(lam, tau);
            add_const(acc, cf[0]);
            return acc;
        }
        if (d < 8) {
            // sum_j k_j T_j at level lam + 1, k_j = round(c_j tau q_{lam+1} / s_j) (every term
            // then at scale tau q_{lam+1}), accumulated in place; one rescale for the sum
            const double ql = (double)c->primes[lam + 1];
            Cx acc;
            for (int j = 1; j <= d; j++) {
                if (cf[j] == 0.0) continue;
                const long long k = (long long)std::nearbyint(cf[j] * tau * ql / T[j].s);
                if (k == 0) continue;
                if (!acc.d) acc = alloc(lam + 1, 0.0);
                if (!ok()) return acc;
                check(launch_mul_int(c, T[j].d, N * (T[j].l + 1), acc.d, lam + 2, residues(k, lam + 2), s,
                                     acc.s != 0.0 ? 1 : 0, 2 * K));
                acc.s = tau * ql;
            }
            if (!acc.d) {
                acc = zero(lam, tau);
            } else {
                Cx o = alloc(lam, tau);
                if (ok()) rescale_into(acc, o, ks);
                release(acc);
                acc = o;
            }
            add_const(acc, cf[0]);
            return acc;
        }
        const int G = d >= 32 ? 32 : (d >= 16 ? 16 : 8);
        std::vector<double> q(d - G + 1, 0.0), r(cf.begin(), cf.begin() + G);
        q[0] = cf[G];
        for (int j = 1; j <= d - G; j++) {
            q[j] = 2.0 * cf[G + j];
            r[G - j] -= cf[G + j];
        }
        const double tau_q = tau * (double)c->primes[lam + 1] / T[G].s;
        Cx Q, rr;
        if (bm) {
            Ev bq = branch(0, bm->slots[4], bm->ks[0]);
            fork({&bq});
            Q = bq.eval(q, lam + 1, tau_q);
            rr = eval(r, lam, tau);
            join(bq);
        } else {
            Q = eval(q, lam + 1, tau_q);
        }
        Cx prod = hmult(Q, T[G]);
        release(Q);  // (a branch's slot joins this free list: the branch is done)
        if (!bm) rr = eval(r, lam, tau);
        Cx o = add(prod, rr, 0);
        o.s = tau;
        release(prod), release(rr);
        return o;
    }
};

size_t eval_ks_words(const nj_ctx *c, int l0, int K)
{
    return std::max(ks_words(c, l0), multi_words(c, l0, K)) + (size_t)c->N * (l0 + 3) * K;
}

size_t eval_mod_words(const nj_ctx *c, int l0, int K = 1)
{
    const size_t slot = K * 2 * (size_t)c->N * (l0 + 1);
    return (Ev::slots_needed() + 4 * kBranchSlots + kTreeSlots) * slot + (1 + kBranchWorkers) * eval_ks_words(c, l0, K);
}

// ModEval of K ciphertexts in[z] (level l0, scale s0) evaluated together (packed; K > 1
// needs N >= 8192): out[z] at level l0 - 11
nj_status eval_mod(nj_ctx *c, int K, const uint64_t *const *in, int l0, double s0, double Kr, const double *cf,
                   uint64_t *const *out, double *out_scale, Arena A, hipStream_t s)
{
    const size_t N = c->N, slot = K * 2 * N * (l0 + 1), pool = Ev::slots_needed() * slot;
    nj_status st = workers_ready(c);
    if (st) return st;
    uint64_t *ctsbuf = A.take(pool);
    if (!ctsbuf) return fail(NJ_ENOMEM, "scratch");
    BranchMem bm;  // the worker streams' slots and key-switch scratch
    for (int i = 0; i < 5; i++) {
        const size_t w = (i < 4 ? kBranchSlots : kTreeSlots) * slot;
        bm.slots[i] = Arena{A.take(w), w};
        if (!bm.slots[i].p) return fail(NJ_ENOMEM, "scratch");
    }
    for (int k = 0; k < kBranchWorkers; k++) {
        const size_t w = eval_ks_words(c, l0, K);
        bm.ks[k] = Arena{A.take(w), w};
        if (!bm.ks[k].p) return fail(NJ_ENOMEM, "scratch");
    }
    Ev ev(c, l0, Arena{ctsbuf, pool}, A, s, K);
    if (!ev.ok()) return ev.err;
    const double q0 = (double)c->primes[0];
    const double sx = Kr * q0;  // the same integers read as x = t / (K P)
    const long long k = (long long)std::nearbyint(std::ldexp(1.0, 48) * (double)c->primes[l0] / sx);
    Cx t = ev.alloc(l0, 0.0), x = ev.alloc(l0 - 1, sx * (double)k / (double)c->primes[l0]);
    if (!ev.ok()) return ev.err;
    for (int z = 0; z < K; z++)
        ev.check(launch_mul_int(c, in[z], N * (l0 + 1), t.d + z * ev.cstride(l0), l0 + 1, ev.residues(k, l0 + 1), s));
    ev.rescale_into(t, x, ev.ks);
    ev.release(t);
    ev.basis(x, &bm);
    const int lam = x.l - 7;
    Cx g = ev.eval(std::vector<double>(cf, cf + kChebDegree + 1), lam, (double)c->primes[lam], &bm);
    for (int i = 0; i < 3; i++) {
        Cx h = ev.sq_minus1(g);
        ev.release(g);
        g = h;
    }
    if (!ev.ok()) return ev.err;
    for (int z = 0; z < K; z++)
        NJ_HIP(hipMemcpyAsync(out[z], g.d + z * ev.cstride(g.l), 2 * N * (g.l + 1) * 8, hipMemcpyDeviceToDevice, s));
    *out_scale = g.s * (2.0 * M_PI) * s0 / q0;
    return NJ_OK;
}

constexpr int kEvalModLevels = 11;

}  // namespace

extern "C" {

nj_status nj_hmult(nj_ctx *c, const nj_ct *a, const nj_ct *b, nj_ct *out, void *stream)
{
    nj_status st = check_ct(c, a, "nj_hmult");
    if (st || (st = check_ct(c, b, "nj_hmult"))) return st;
    const int l = std::min(a->level, b->level);
    if (l < 1) return fail(NJ_ELEVEL, "nj_hmult: needs level >= 1");
    if (!out || !out->data) return fail(NJ_EINVAL, "nj_hmult: null output");
    const size_t N = c->N;
    bool ok;
    Arena A = arena_for(c, 4 * 2 * N * (l + 1) + ks_words(c, l) + N * (l + 3), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    uint64_t *buf = A.take(4 * 2 * N * (l + 1));
    Ev ev(c, l, Arena{buf, 4 * 2 * N * (l + 1)}, A, S(stream));
    if (!ev.ok()) return ev.err;
    Cx x{a->data, a->level, a->scale}, y{b->data, b->level, b->scale};
    Cx o = ev.hmult(x, y);
    if (!ev.ok()) return ev.err;
    NJ_HIP(hipMemcpyAsync(out->data, o.d, 2 * N * l * 8, hipMemcpyDeviceToDevice, S(stream)));
    out->level = l - 1, out->is_ntt = 1, out->scale = o.s;
    return NJ_OK;
}

nj_status nj_mul_const(nj_ctx *c, const nj_ct *in, double v, int level, double scale, nj_ct *out, void *stream)
{
    nj_status st = check_ct(c, in, "nj_mul_const");
    if (st) return st;
    if (level < 0 || level >= in->level) return fail(NJ_ELEVEL, "nj_mul_const: target level must be below the input's");
    if (!out || !out->data || !(scale > 0.0)) return fail(NJ_EINVAL, "nj_mul_const: bad output or scale");
    const size_t N = c->N;
    const int l = in->level;
    bool ok;
    Arena A = arena_for(c, 4 * 2 * N * (l + 1) + N * (l + 3), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    uint64_t *buf = A.take(4 * 2 * N * (l + 1));
    Ev ev(c, l, Arena{buf, 4 * 2 * N * (l + 1)}, A, S(stream));
    ev.err = NJ_OK;  // no key needed
    Cx x{in->data, in->level, in->scale};
    Cx o = ev.const_mult(x, v, level, scale);
    if (!ev.ok()) return ev.err;
    if (!o.d) {
        Cx z = ev.zero(level, scale);
        if (!ev.ok()) return ev.err;
        o = z;
    }
    NJ_HIP(hipMemcpyAsync(out->data, o.d, 2 * N * (level + 1) * 8, hipMemcpyDeviceToDevice, S(stream)));
    out->level = level, out->is_ntt = 1, out->scale = scale;
    return NJ_OK;
}

nj_status nj_add_const(nj_ctx *c, nj_ct *ct, double v, void *stream)
{
    nj_status st = check_ct(c, ct, "nj_add_const");
    if (st) return st;
    const long long k = (long long)std::nearbyint(v * ct->scale);
    LimbConsts kc;
    for (int i = 0; i <= ct->level; i++) {
        const long long q = (long long)c->primes[i];
        long long r = k % q;
        kc.v[i] = (double)(r < 0 ? r + q : r);
    }
    NJ_HIP(launch_add_int(c, ct->data, ct->level + 1, kc, S(stream)));
    return NJ_OK;
}

nj_status nj_cheb_interpolate(int degree, double K, int r, double *coeffs)
{
    if (degree < 1 || degree > 1023 || !coeffs || r < 0 || r > 16) return fail(NJ_EINVAL, "nj_cheb_interpolate: bad arguments");
    cheb_interpolate_cos(degree, K, r, coeffs);
    return NJ_OK;
}

nj_status nj_eval_order(nj_ctx *c, int order)
{
    if (!c) return fail(NJ_EINVAL, "nj_eval_order: null context");
    if (order != 0 && order != 1) return fail(NJ_EINVAL, "nj_eval_order: order must be 0 or 1");
    c->eval_order = order;
    return NJ_OK;
}

nj_status nj_eval_mod(nj_ctx *c, const nj_ct *in, int K, int r, const double *coeffs, int n_coeffs, nj_ct *out,
                      void *stream)
{
    nj_status st = check_ct(c, in, "nj_eval_mod");
    if (st) return st;
    if (K < 1 || r != 3 || (coeffs && n_coeffs != kChebDegree + 1))
        return fail(NJ_EUNSUPPORTED, "nj_eval_mod: supports r = 3 double angles and 64 Chebyshev coefficients");
    if (in->level < kEvalModLevels + 1) return fail(NJ_ELEVEL, "nj_eval_mod: needs input level >= 12");
    if (!out || !out->data || out->data == in->data) return fail(NJ_EINVAL, "nj_eval_mod: bad output");
    std::vector<double> cf(kChebDegree + 1);
    if (coeffs) std::copy(coeffs, coeffs + kChebDegree + 1, cf.begin());
    else cheb_interpolate_cos(kChebDegree, (double)K, r, cf.data());
    bool ok;
    Arena A = arena_for(c, eval_mod_words(c, in->level), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    double sc = 0.0;
    const uint64_t *ins[1] = {in->data};
    uint64_t *outs[1] = {out->data};
    if ((st = eval_mod(c, 1, ins, in->level, in->scale, (double)K, cf.data(), outs, &sc, A, S(stream)))) return st;
    out->level = in->level - kEvalModLevels, out->is_ntt = 1, out->scale = sc;
    return NJ_OK;
}

}  // extern "C"

// ModEval of Re and Im together (one packed evaluation, N >= 8192; else one after the
// other): the same results as two nj_eval_mod calls
nj_status nj::ex::eval_mod_pair(nj_ctx *c, const nj_ct *re, const nj_ct *im, int K, int r, const double *coeffs,
                                int n_coeffs, nj_ct *out_re, nj_ct *out_im, void *stream)
{
    nj_status st;
    if (c->N < 8192) {
        if ((st = nj_eval_mod(c, re, K, r, coeffs, n_coeffs, out_re, stream))) return st;
        return nj_eval_mod(c, im, K, r, coeffs, n_coeffs, out_im, stream);
    }
    st = check_ct(c, re, "nj_eval_mod");
    if (st || (st = check_ct(c, im, "nj_eval_mod"))) return st;
    if (re->level != im->level || re->scale != im->scale) return fail(NJ_ELEVEL, "eval_mod_pair: Re and Im differ");
    if (K < 1 || r != 3 || (coeffs && n_coeffs != kChebDegree + 1))
        return fail(NJ_EUNSUPPORTED, "nj_eval_mod: supports r = 3 double angles and 64 Chebyshev coefficients");
    if (re->level < kEvalModLevels + 1) return fail(NJ_ELEVEL, "nj_eval_mod: needs input level >= 12");
    if (!out_re || !out_im || !out_re->data || !out_im->data) return fail(NJ_EINVAL, "eval_mod_pair: bad output");
    std::vector<double> cf(kChebDegree + 1);
    if (coeffs) std::copy(coeffs, coeffs + kChebDegree + 1, cf.begin());
    else cheb_interpolate_cos(kChebDegree, (double)K, r, cf.data());
    bool ok;
    Arena A = arena_for(c, eval_mod_words(c, re->level, 2), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    const uint64_t *ins[2] = {re->data, im->data};
    uint64_t *outs[2] = {out_re->data, out_im->data};
    double sc = 0.0;
    if ((st = eval_mod(c, 2, ins, re->level, re->scale, (double)K, cf.data(), outs, &sc, A, S(stream)))) return st;
    out_re->level = out_im->level = re->level - kEvalModLevels;
    out_re->is_ntt = out_im->is_ntt = 1;
    out_re->scale = out_im->scale = sc;
    return NJ_OK;
}

extern "C" {

nj_status nj_combine(nj_ctx *c, const nj_ct *re, const nj_ct *im, nj_ct *out, void *stream)
{
    nj_status st = check_ct(c, re, "nj_combine");
    if (st || (st = check_ct(c, im, "nj_combine"))) return st;
    if (re->level != im->level) return fail(NJ_ELEVEL, "nj_combine: Re and Im must share a level");
    if (!same_scale(re->scale, im->scale)) return fail(NJ_ESCALE, "nj_combine: Re and Im at different scales");
    if (!out || !out->data || out->data == re->data || out->data == im->data) return fail(NJ_EINVAL, "nj_combine: bad output");
    // the monomial kernel multiplies by -X^{N/2}, so Re - (-X^{N/2} Im) = Re + i Im
    NJ_HIP(launch_monomial_half(c, im->level, im->data, out->data, S(stream)));
    NJ_HIP(launch_elementwise(c, 1, re->data, out->data, out->data, ct_limbs(re->level), S(stream)));
    out->level = re->level, out->is_ntt = 1, out->scale = re->scale;
    return NJ_OK;
}

nj_status nj_stoc1_plan_create(nj_ctx *c, int ell, int groups, int level, nj_plan **out)
{
    if (!c || !out) return fail(NJ_EINVAL, "nj_stoc1_plan_create: null argument");
    if (level - groups + 1 < 1 || level > c->L) return fail(NJ_ELEVEL, "nj_stoc1_plan_create: levels out of range");
    nj_plan *p = new nj_plan();
    p->kind = 2;
    p->N = c->N;
    p->ell = ell;
    std::vector<std::vector<std::vector<double>>> re, im;
    nj_status st = build_stoc1_diagonals(c->N, ell, groups, p->lts, re, im);
    if (st) {
        delete p;
        return st;
    }
    for (int g = 0; g < groups; g++) {
        nj_lt_t &lt = p->lts[g];
        lt.level = level - g;
        st = upload_plan_diagonals(c, lt, re[g], im[g], (double)c->primes[lt.level]);
        if (st) {
            nj_plan_destroy(p);
            return st;
        }
    }
    *out = p;
    return NJ_OK;
}

nj_status nj_stoc1(nj_ctx *c, const nj_plan *p, const nj_ct *in, nj_ct *out, void *stream)
{
    if (!c || !p || p->kind != 2 || p->lts.empty()) return fail(NJ_EINVAL, "nj_stoc1: not a StoC1 plan");
    nj_status st = check_ct(c, in, "nj_stoc1");
    if (st) return st;
    if (in->level != p->lts[0].level) return fail(NJ_ELEVEL, "nj_stoc1: input must be at the plan's first level");
    if (!out || !out->data || out->data == in->data) return fail(NJ_EINVAL, "nj_stoc1: bad output");
    const size_t N = c->N, clen = 2 * N * (in->level + 1);
    size_t need = 0;
    for (const auto &lt : p->lts) need = std::max(need, bsgs_words(c, lt));
    bool ok;
    Arena A = arena_for(c, 2 * clen + need + N * (in->level + 2), ok);
    if (!ok) return fail(NJ_ENOMEM, "scratch");
    uint64_t *x = A.take(clen), *y = A.take(clen);
    NJ_HIP(hipMemcpyAsync(x, in->data, clen * 8, hipMemcpyDeviceToDevice, S(stream)));
    int l = in->level;
    for (const auto &lt : p->lts) {
        if ((st = bsgs_rescale(c, lt, x, y, x, A, S(stream)))) return st;
        l--;
    }
    NJ_HIP(hipMemcpyAsync(out->data, x, 2 * N * (l + 1) * 8, hipMemcpyDeviceToDevice, S(stream)));
    out->level = l, out->is_ntt = 1, out->scale = in->scale;
    return NJ_OK;
}

}  // extern "C"
