// Context construction: primes, roots, transform tables, RNS basis-conversion
// constants (hybrid key switching, Table 4 dnum), secret and switching keys.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "internal.h"

namespace nj {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
nj_status fail(nj_status code, const std::string &msg)
{
    g_err = msg;
    return code;
}
nj_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? NJ_ENOMEM : NJ_EDEVICE;
}

// ----------------------------------------------------------- host integers

typedef unsigned __int128 u128;
static uint64_t hmul(uint64_t a, uint64_t b, uint64_t t) { return (uint64_t)((u128)a * b % t); }
static uint64_t hpow(uint64_t a, uint64_t e, uint64_t t)
{
    uint64_t r = 1;
    a %= t;
    for (; e; e >>= 1, a = hmul(a, a, t))
        if (e & 1) r = hmul(r, a, t);
    return r;
}
static uint64_t hinv(uint64_t a, uint64_t t) { return hpow(a % t, t - 2, t); }

static bool miller_rabin(uint64_t n)
{
    if (n < 2) return false;
    static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t p : small) {
        if (n % p == 0) return n == p;
    }
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) d >>= 1, s++;
    for (uint64_t a : small) {
        uint64_t x = hpow(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (int r = 1; r < s && witness; r++) {
            x = hmul(x, x, n);
            if (x == n - 1) witness = false;
        }
        if (witness) return false;
    }
    return true;
}

static uint32_t rev_bits(uint32_t x, int bits)
{
    uint32_t r = 0;
    for (int i = 0; i < bits; i++) r = (r << 1) | ((x >> i) & 1u);
    return r;
}

// A primitive 2N-th root of unity mod t: x^((t-1)/2N) has order 2N iff its N-th power is -1.
static uint64_t root_2n(uint64_t t, int N)
{
    for (uint64_t x = 3;; x += 2) {
        uint64_t y = hpow(x, (t - 1) / (2 * (uint64_t)N), t);
        if (hpow(y, (uint64_t)N, t) == t - 1) return y;
    }
}

LimbTab limbs_q(int level)
{
    LimbTab lt;
    lt.n = level + 1;
    for (int i = 0; i <= level; i++) lt.pidx[i] = i, lt.off[i] = i;
    return lt;
}

LimbTab limbs_ext(const nj_ctx *c, int level)
{
    LimbTab lt;
    lt.n = level + 1 + c->alpha;
    for (int i = 0; i <= level; i++) lt.pidx[i] = i, lt.off[i] = i;
    for (int k = 0; k < c->alpha; k++) lt.pidx[level + 1 + k] = c->n_q + k, lt.off[level + 1 + k] = level + 1 + k;
    return lt;
}

int n_digits(const nj_ctx *c, int level) { return (level + 1 + c->alpha - 1) / c->alpha; }

uint64_t *scratch_get(nj_ctx *c, size_t words)
{
    if (c->scratch.words >= words) return c->scratch.buf;
    if (c->scratch.buf) {
        (void)hipDeviceSynchronize();
        (void)hipFree(c->scratch.buf);
        c->scratch.buf = nullptr;
        c->scratch.words = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, words * sizeof(uint64_t)) != hipSuccess) return nullptr;
    c->scratch.buf = (uint64_t *)p;
    c->scratch.words = words;
    return c->scratch.buf;
}

// Device upload helper
template <typename T>
static hipError_t upload(T **dst, const std::vector<T> &src)
{
    hipError_t e = hipMalloc((void **)dst, src.size() * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Basis-conversion table from primes `from` (prime indices) to primes `to`.
static hipError_t make_bconv(const nj_ctx *c, const std::vector<int> &from, const std::vector<int> &to,
                             const std::vector<int> &to_limb, BconvTab &bt)
{
    const int m = (int)from.size(), n_out = (int)to.size();
    bt.m = m;
    bt.n_out = n_out;
    bt.out_pidx = to;
    bt.out_limb = to_limb;
    std::vector<double> hinv_d(2 * m), hat((size_t)m * n_out);
    for (int a = 0; a < m; a++) {
        bt.in_pidx[a] = from[a];
        uint64_t qa = c->primes[from[a]], prod = 1;
        for (int b = 0; b < m; b++)
            if (b != a) prod = hmul(prod, c->primes[from[b]] % qa, qa);
        uint64_t iv = hinv(prod, qa);
        hinv_d[a] = (double)iv;
        hinv_d[m + a] = (double)iv / (double)qa;
        for (int o = 0; o < n_out; o++) {
            uint64_t t = c->primes[to[o]], pr = 1;
            for (int b = 0; b < m; b++)
                if (b != a) pr = hmul(pr, c->primes[from[b]] % t, t);
            hat[(size_t)a * n_out + o] = (double)pr;
        }
    }
    hipError_t e = upload(&bt.hat_inv, hinv_d);
    if (e != hipSuccess) return e;
    return upload(&bt.hat, hat);
}

}  // namespace nj

using namespace nj;

extern "C" {

const char *nj_last_error(void) { return nj::g_err.c_str(); }

nj_status nj_gen_primes(int log_n, int bits, int count, const uint64_t *exclude, int n_exclude, uint64_t *out)
{
    if (!out || count < 0 || bits > 50 || bits < 20 || log_n < 1 || log_n > 20 || (n_exclude > 0 && !exclude))
        return fail(NJ_EINVAL, "nj_gen_primes: bad arguments");
    const uint64_t m = 2ull << log_n;
    uint64_t k = ((1ull << bits) - 2) / m;
    int got = 0;
    for (; got < count && k > 0; k--) {
        uint64_t t = k * m + 1;
        bool skip = false;
        for (int i = 0; i < n_exclude && !skip; i++) skip = exclude[i] == t;
        for (int i = 0; i < got && !skip; i++) skip = out[i] == t;
        if (!skip && miller_rabin(t)) out[got++] = t;
    }
    return got == count ? NJ_OK : fail(NJ_EINVAL, "nj_gen_primes: not enough primes");
}

uint32_t nj_galois_elt(const nj_ctx *c, int r)
{
    const int n = c->N / 2;
    int rr = ((r % n) + n) % n;
    return (uint32_t)hpow(5, (uint64_t)rr, 2 * (uint64_t)c->N);
}

nj_status nj_ctx_create(const nj_params *P, nj_ctx **out)
{
    if (!P || !out || !P->q || !P->p) return fail(NJ_EINVAL, "nj_ctx_create: null argument");
    if (P->log_n < 10 || P->log_n > 16) return fail(NJ_EUNSUPPORTED, "nj_ctx_create: log_n must be 10..16");
    // the basis-conversion tables of a launch hold digits of at most 16 primes and 48
    // targets each (BconvShared): n_q <= 32 keeps every ModUp digit (n_q + alpha - m
    // targets) and ModDown (n_q targets) inside them
    if (P->n_q < 1 || P->n_q > 32 || P->alpha < 1 || P->alpha > 16)
        return fail(NJ_EUNSUPPORTED, "nj_ctx_create: prime counts out of range (1 <= n_q <= 32, 1 <= alpha <= 16)");
    // the shared-key inner products hold every digit's key words of one limb in registers
    if ((P->n_q + P->alpha - 1) / P->alpha > 8)
        return fail(NJ_EUNSUPPORTED, "nj_ctx_create: more than 8 key-switching digits (dnum = ceil(n_q / alpha))");
    nj_ctx *c = new nj_ctx();
    c->log_n = P->log_n;
    c->N = 1 << P->log_n;
    c->n_q = P->n_q;
    c->L = P->n_q - 1;
    c->alpha = P->alpha;
    c->dnum = (c->L + 1 + c->alpha - 1) / c->alpha;
    c->n_primes = P->n_q + P->alpha;
    c->scale = P->scale;
    (void)hipGetDevice(&c->device);
    for (int i = 0; i < P->n_q; i++) c->primes.push_back(P->q[i]);
    for (int i = 0; i < P->alpha; i++) c->primes.push_back(P->p[i]);
    const uint64_t two_n = 2ull * c->N;
    for (int i = 0; i < c->n_primes; i++) {
        uint64_t t = c->primes[i];
        if (t >= (1ull << 50) || t < (1ull << 30) || t % two_n != 1 || !miller_rabin(t)) {
            delete c;
            return fail(NJ_EUNSUPPORTED, "nj_ctx_create: every prime must be 1 mod 2N, prime, in [2^30, 2^50)");
        }
        for (int j = 0; j < i; j++)
            if (c->primes[j] == t) {
                delete c;
                return fail(NJ_EINVAL, "nj_ctx_create: repeated prime");
            }
    }
    const int N = c->N, np = c->n_primes;
    // per-prime constants and transform tables
    std::vector<double> tw((size_t)np * N), twq((size_t)np * N), itw((size_t)np * N), itwq((size_t)np * N);
    c->info.resize(np);
    for (int i = 0; i < np; i++) {
        uint64_t t = c->primes[i];
        double td = (double)t;
        uint64_t psi = root_2n(t, N), ipsi = hinv(psi, t);
        // psi^k and psi^-k for k < N
        std::vector<uint64_t> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (int k = 1; k < N; k++) pw[k] = hmul(pw[k - 1], psi, t), ipw[k] = hmul(ipw[k - 1], ipsi, t);
        for (int k = 0; k < N; k++) {
            uint32_t r = rev_bits((uint32_t)k, c->log_n);
            tw[(size_t)i * N + k] = (double)pw[r];
            twq[(size_t)i * N + k] = (double)pw[r] / td;
            itw[(size_t)i * N + k] = (double)ipw[r];
            itwq[(size_t)i * N + k] = (double)ipw[r] / td;
        }
        uint64_t ni = hinv((uint64_t)N, t);
        c->info[i].m.t = td;
        c->info[i].m.ti = 1.0 / td;
        c->info[i].ninv = (double)ni;
        c->info[i].ninvq = (double)ni / td;
        c->info[i].half = (double)(t / 2);
    }
    hipError_t e;
    if ((e = upload(&c->d_tw, tw)) != hipSuccess || (e = upload(&c->d_twq, twq)) != hipSuccess ||
        (e = upload(&c->d_itw, itw)) != hipSuccess || (e = upload(&c->d_itwq, itwq)) != hipSuccess ||
        (e = upload(&c->d_info, c->info)) != hipSuccess) {
        nj_ctx_destroy(c);
        return hip_fail(e, "nj_ctx_create: table upload");
    }
    // ModUp tables: every level, every digit
    c->modup.resize(c->n_q);
    for (int l = 0; l <= c->L; l++) {
        int nd = n_digits(c, l);
        c->modup[l].resize(nd);
        for (int j = 0; j < nd; j++) {
            int lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, l + 1);
            std::vector<int> from, to, to_limb;
            for (int a = lo; a < hi; a++) from.push_back(a);
            for (int tpos = 0; tpos < l + 1 + c->alpha; tpos++) {
                if (tpos >= lo && tpos < hi) continue;
                to.push_back(tpos <= l ? tpos : c->n_q + (tpos - l - 1));
                to_limb.push_back(tpos);
            }
            if ((e = make_bconv(c, from, to, to_limb, c->modup[l][j])) != hipSuccess) {
                nj_ctx_destroy(c);
                return hip_fail(e, "nj_ctx_create: ModUp tables");
            }
        }
    }
    // ModDown tables: P -> Q_l
    c->moddown.resize(c->n_q);
    for (int l = 0; l <= c->L; l++) {
        std::vector<int> from, to, to_limb;
        for (int k = 0; k < c->alpha; k++) from.push_back(c->n_q + k);
        for (int i = 0; i <= l; i++) to.push_back(i), to_limb.push_back(i);
        if ((e = make_bconv(c, from, to, to_limb, c->moddown[l])) != hipSuccess) {
            nj_ctx_destroy(c);
            return hip_fail(e, "nj_ctx_create: ModDown tables");
        }
    }
    // the conversions restricted to Q limbs 0 and l (key switches whose output is rescaled
    // and dropped to level 0)
    c->modup_drop.resize(c->n_q);
    c->moddown_drop.resize(c->n_q);
    for (int l = 0; l <= c->L; l++) {
        const int nd = n_digits(c, l);
        c->modup_drop[l].resize(nd);
        for (int j = 0; j < nd; j++) {
            const int lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, l + 1);
            std::vector<int> from, to, to_limb;
            for (int a = lo; a < hi; a++) from.push_back(a);
            for (int tpos = 0; tpos < l + 1 + c->alpha; tpos++) {
                if ((tpos >= lo && tpos < hi) || (tpos > 0 && tpos < l)) continue;
                to.push_back(tpos <= l ? tpos : c->n_q + (tpos - l - 1));
                to_limb.push_back(tpos);
            }
            if ((e = make_bconv(c, from, to, to_limb, c->modup_drop[l][j])) != hipSuccess) {
                nj_ctx_destroy(c);
                return hip_fail(e, "nj_ctx_create: ModUp tables");
            }
        }
        std::vector<int> from, to, to_limb;
        for (int k = 0; k < c->alpha; k++) from.push_back(c->n_q + k);
        to.push_back(0), to_limb.push_back(0);
        if (l > 0) to.push_back(l), to_limb.push_back(l);
        if ((e = make_bconv(c, from, to, to_limb, c->moddown_drop[l])) != hipSuccess) {
            nj_ctx_destroy(c);
            return hip_fail(e, "nj_ctx_create: ModDown tables");
        }
    }
    // basis-conversion input factors folded into the inverse transforms' N^-1
    {
        auto fac = [&](const std::vector<int> &digit, int a) {  // N^-1 (D/q_a)^-1 mod q_a
            const uint64_t qa = c->primes[digit[a]];
            uint64_t prod = 1;
            for (size_t b = 0; b < digit.size(); b++)
                if ((int)b != a) prod = hmul(prod, c->primes[digit[b]] % qa, qa);
            return (double)hmul(hinv((uint64_t)c->N % qa, qa), hinv(prod, qa), qa);
        };
        c->d_upscale.assign(c->n_q, nullptr);
        for (int l = 0; l <= c->L; l++) {
            std::vector<double> sc(l + 1);
            for (int j = 0; j * c->alpha <= l; j++) {
                std::vector<int> digit;
                for (int a = j * c->alpha; a < std::min((j + 1) * c->alpha, l + 1); a++) digit.push_back(a);
                for (size_t a = 0; a < digit.size(); a++) sc[digit[a]] = fac(digit, (int)a);
            }
            if ((e = upload(&c->d_upscale[l], sc)) != hipSuccess) {
                nj_ctx_destroy(c);
                return hip_fail(e, "nj_ctx_create: ModUp factors");
            }
        }
        std::vector<int> pd;
        for (int k = 0; k < c->alpha; k++) pd.push_back(c->n_q + k);
        std::vector<double> sc(np, 0.0);
        for (int k = 0; k < c->alpha; k++) sc[c->n_q + k] = fac(pd, k);
        if ((e = upload(&c->d_downscale, sc)) != hipSuccess) {
            nj_ctx_destroy(c);
            return hip_fail(e, "nj_ctx_create: ModDown factors");
        }
    }
    // P mod every prime, P^-1 mod q_i, q_l^-1 mod q_i
    std::vector<double> pinv(2 * c->n_q), qlinv((size_t)c->n_q * c->n_q, 0.0), qlinvq((size_t)c->n_q * c->n_q, 0.0);
    c->pmod.assign(np, 0.0);
    for (int i = 0; i < np; i++) {
        uint64_t t = c->primes[i], pm = 1;
        for (int k = 0; k < c->alpha; k++) pm = hmul(pm, c->primes[c->n_q + k] % t, t);
        c->pmod[i] = (double)pm;
        if (i < c->n_q) {
            uint64_t iv = hinv(pm, t);
            pinv[i] = (double)iv;
            pinv[c->n_q + i] = (double)iv / (double)t;
        }
    }
    for (int l = 1; l <= c->L; l++)
        for (int i = 0; i < l; i++) {
            uint64_t t = c->primes[i], iv = hinv(c->primes[l] % t, t);
            qlinv[(size_t)l * c->n_q + i] = (double)iv;
            qlinvq[(size_t)l * c->n_q + i] = (double)iv / (double)t;
        }
    std::vector<double> pinv_a(pinv.begin(), pinv.begin() + c->n_q), pinv_b(pinv.begin() + c->n_q, pinv.end());
    std::vector<double> pmod_key(c->L + 1 + c->alpha, 0.0);
    for (int t = 0; t <= c->L; t++) pmod_key[t] = c->pmod[t];
    if ((e = upload(&c->d_primes, c->primes)) != hipSuccess || (e = upload(&c->d_pmod, pmod_key)) != hipSuccess) {
        nj_ctx_destroy(c);
        return hip_fail(e, "nj_ctx_create: constants upload");
    }
    if ((e = upload(&c->d_pinv, pinv_a)) != hipSuccess || (e = upload(&c->d_pinvq, pinv_b)) != hipSuccess ||
        (e = upload(&c->d_qlinv, qlinv)) != hipSuccess || (e = upload(&c->d_qlinvq, qlinvq)) != hipSuccess) {
        nj_ctx_destroy(c);
        return hip_fail(e, "nj_ctx_create: constants upload");
    }
    // the device address of the no-allocation entry point's static scratch, looked up
    // once per device while it is current; a failure only disables that entry point,
    // which reports it
    (void)noalloc_init(c->device);
    *out = c;
    return NJ_OK;
}

void nj_ctx_destroy(nj_ctx *c)
{
    if (!c) return;
    (void)hipDeviceSynchronize();
    auto fr = [](void *p) {
        if (p) (void)hipFree(p);
    };
    fr(c->d_tw), fr(c->d_twq), fr(c->d_itw), fr(c->d_itwq), fr(c->d_info);
    fr(c->d_pinv), fr(c->d_pinvq), fr(c->d_qlinv), fr(c->d_qlinvq), fr(c->d_s), fr(c->d_pk), fr(c->d_primes), fr(c->d_pmod);
    for (auto &lv : c->modup)
        for (auto &b : lv) fr(b.hat_inv), fr(b.hat);
    for (auto &b : c->moddown) fr(b.hat_inv), fr(b.hat);
    for (auto &b : c->moddown_drop) fr(b.hat_inv), fr(b.hat);
    for (auto &v : c->modup_drop)
        for (auto &b : v) fr(b.hat_inv), fr(b.hat);
    for (auto *p : c->d_upscale) fr(p);
    fr(c->layer_buf);
    fr(c->d_downscale);
    for (auto &kv : c->keys) fr(kv.second.d);
    for (auto *k : c->timing_keys) fr(k);
    fr(c->scratch.buf);
    for (auto &r : c->prof_recs) (void)hipEventDestroy(r.a), (void)hipEventDestroy(r.b);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    for (auto w : c->workers) (void)hipStreamDestroy(w);
    for (auto e : c->worker_done) (void)hipEventDestroy(e);
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    delete c;
}

}  // extern "C"
