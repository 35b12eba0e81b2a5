/*
 * Oracle: plain, slow, obviously-correct CPU RNS-CKKS integer arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the HIP path.
 *
 * Conventions (all polynomials are in coefficient form, natural order):
 *   ring R_t = Z_t[X]/(X^n + 1) for each prime t;  a "limb" is n residues in [0,t).
 *   Level-l ciphertext moduli are q_0..q_l; the special (key-switching) moduli are
 *   p_0..p_{alpha-1}.  An "extended" array holds the limbs q_0..q_l followed by
 *   p_0..p_{alpha-1}.  Key-switching keys hold every top-level limb
 *   q_0..q_L, p_0..p_{alpha-1}.
 *   Digits (hybrid key switching, dnum digits at the top level) are consecutive
 *   alpha-groups of ciphertext primes: D_j = {q_{j*alpha} .. q_{min((j+1)alpha,l+1)-1}}.
 *
 * Products use unsigned __int128 and the % operator; there is no lazy reduction,
 * no precomputed quotient and no vectorisation.  Polynomial products use a
 * textbook negacyclic number-theoretic transform (weighted cyclic transform,
 * iterative radix-2 Cooley-Tukey) as a multiplication primitive only.
 *
 * Threads: loops over independent limbs (and digits x limbs) are split over
 * OpenMP threads; each limb is still computed by one thread in the order written,
 * so the results do not depend on the thread count (or_set_threads).
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ scalars */

uint64_t or_mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

/* threads used by the limb loops (n <= 0: the OpenMP default, every host core) */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }
int or_get_threads(void) { return omp_get_max_threads(); }
static uint64_t addm(uint64_t a, uint64_t b, uint64_t q) { uint64_t s = a + b; return s >= q ? s - q : s; }
static uint64_t subm(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + (q - b); }
static uint64_t negm(uint64_t a, uint64_t q) { return a ? q - a : 0; }

uint64_t or_powmod(uint64_t a, uint64_t e, uint64_t q)
{
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = or_mulmod(r, a, q);
        a = or_mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}

/* inverse modulo a prime (Fermat) */
static uint64_t invm(uint64_t a, uint64_t q) { return or_powmod(a % q, q - 2, q); }

/* signed integer -> residue */
static uint64_t from_i64(int64_t v, uint64_t q)
{
    if (v >= 0) return (uint64_t)v % q;
    uint64_t m = (uint64_t)(-(v + 1)) + 1; /* |v| without overflow */
    return negm(m % q, q);
}

/* Miller-Rabin, deterministic for all n < 2^64 with the first twelve prime bases. */
int or_is_prime(uint64_t n)
{
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    uint64_t d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; r++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = or_powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int k = 1; k < r; k++) {
            x = or_mulmod(x, x, n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

/*
 * Prime chain rule: scan t = k*2n + 1 downward from the largest such t below
 * 2^bits and take the first `count` primes not listed in `exclude`.
 * Returns the number of primes written.
 */
int or_gen_primes(int log_n, int bits, int count, const uint64_t *exclude, int n_ex, uint64_t *out)
{
    uint64_t m = 2ull << log_n;
    uint64_t k = ((1ull << bits) - 2) / m;
    int got = 0;
    while (got < count && k > 0) {
        uint64_t t = k * m + 1;
        k--;
        int skip = 0;
        for (int i = 0; i < n_ex; i++) if (exclude[i] == t) skip = 1;
        for (int i = 0; i < got; i++) if (out[i] == t) skip = 1;
        if (skip || !or_is_prime(t)) continue;
        out[got++] = t;
    }
    return got;
}

/* psi: g^((q-1)/2n) for the smallest quadratic non-residue g; then psi^n = -1. */
uint64_t or_find_psi(int n, uint64_t q)
{
    for (uint64_t g = 2;; g++) {
        if (or_powmod(g, (q - 1) / 2, q) == q - 1) return or_powmod(g, (q - 1) / (2 * (uint64_t)n), q);
    }
}

/* ------------------------------------------------ number-theoretic transform */

static void bit_reverse_permute(uint64_t *a, int n)
{
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
    }
}

/* cyclic length-n transform with primitive n-th root w: A_k = sum_i a_i w^(ik) */
static void cyclic_ntt(uint64_t *a, int n, uint64_t w, uint64_t q)
{
    uint64_t *wp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n / 2 > 0 ? n / 2 : 1));
    wp[0] = 1;
    for (int j = 1; j < n / 2; j++) wp[j] = or_mulmod(wp[j - 1], w, q);
    bit_reverse_permute(a, n);
    for (int len = 2; len <= n; len <<= 1) {
        int step = n / len;
        for (int i = 0; i < n; i += len) {
            for (int j = 0; j < len / 2; j++) {
                uint64_t u = a[i + j];
                uint64_t v = or_mulmod(a[i + j + len / 2], wp[j * step], q);
                a[i + j] = addm(u, v, q);
                a[i + j + len / 2] = subm(u, v, q);
            }
        }
    }
    free(wp);
}

/* negacyclic forward transform: A_k = sum_i a_i psi^i w^(ik), w = psi^2 */
void or_ntt_fwd(uint64_t *a, int n, uint64_t q)
{
    uint64_t psi = or_find_psi(n, q), pw = 1;
    for (int i = 0; i < n; i++) { a[i] = or_mulmod(a[i], pw, q); pw = or_mulmod(pw, psi, q); }
    cyclic_ntt(a, n, or_mulmod(psi, psi, q), q);
}

/* inverse of or_ntt_fwd */
void or_ntt_inv(uint64_t *a, int n, uint64_t q)
{
    uint64_t psi = or_find_psi(n, q);
    uint64_t psi_inv = invm(psi, q);
    cyclic_ntt(a, n, or_mulmod(psi_inv, psi_inv, q), q);
    uint64_t ninv = invm((uint64_t)n, q), pw = ninv;
    for (int i = 0; i < n; i++) { a[i] = or_mulmod(a[i], pw, q); pw = or_mulmod(pw, psi_inv, q); }
}

/* c = a * b in Z_q[X]/(X^n+1) (c may alias a or b) */
void or_polymul(const uint64_t *a, const uint64_t *b, uint64_t *c, int n, uint64_t q)
{
    uint64_t *ta = (uint64_t *)malloc(sizeof(uint64_t) * n), *tb = (uint64_t *)malloc(sizeof(uint64_t) * n);
    memcpy(ta, a, sizeof(uint64_t) * n);
    memcpy(tb, b, sizeof(uint64_t) * n);
    or_ntt_fwd(ta, n, q);
    or_ntt_fwd(tb, n, q);
    for (int i = 0; i < n; i++) ta[i] = or_mulmod(ta[i], tb[i], q);
    or_ntt_inv(ta, n, q);
    memcpy(c, ta, sizeof(uint64_t) * n);
    free(ta);
    free(tb);
}

/* c = a * s for a small signed integer polynomial s (given as int64) */
static void polymul_small(const uint64_t *a, const int64_t *s, uint64_t *c, int n, uint64_t q)
{
    uint64_t *ts = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (int i = 0; i < n; i++) ts[i] = from_i64(s[i], q);
    or_polymul(a, ts, c, n, q);
    free(ts);
}

/* ------------------------------------------------------------ automorphism */

/* out(X) = a(X^g), g odd: coefficient i moves to i*g mod 2n, negated when it lands in [n, 2n). */
void or_automorph(const uint64_t *a, uint64_t *out, int n, uint64_t g, uint64_t q)
{
    uint64_t two_n = 2 * (uint64_t)n;
    for (int i = 0; i < n; i++) {
        uint64_t e = (uint64_t)i * g % two_n;
        if (e < (uint64_t)n) out[e] = a[i];
        else out[e - n] = negm(a[i], q);
    }
}

/* out = a * X^k (k in [0, 2n)) */
void or_monomial(const uint64_t *a, uint64_t *out, int n, int k, uint64_t q)
{
    for (int i = 0; i < n; i++) {
        int e = (i + k) % (2 * n);
        if (e < n) out[e] = a[i];
        else out[e - n] = negm(a[i], q);
    }
}

/* --------------------------------------------------------------- RNS ring */

typedef struct {
    int n;          /* ring degree */
    int L;          /* top level: ciphertext primes q_0..q_L */
    int alpha;      /* special primes p_0..p_{alpha-1} = primes per digit */
    const uint64_t *q;
    const uint64_t *p;
} or_ring;

/* prime of extended limb index t at level l (0..l -> q, l+1.. -> p) */
static uint64_t ext_prime(const or_ring *R, int l, int t) { return t <= l ? R->q[t] : R->p[t - l - 1]; }
/* index of that limb inside a top-level key array */
static int key_limb(const or_ring *R, int l, int t) { return t <= l ? t : R->L + 1 + (t - l - 1); }

static int n_digits(const or_ring *R, int l) { return (l + 1 + R->alpha - 1) / R->alpha; }

/*
 * ModUp of digit j at level l: fast basis conversion from the digit's primes D_j
 * to every other prime of Q_l u P, without correction:
 *   y_t = sum_{i in D_j} [x_i * (D_j/q_i)^{-1}]_{q_i} * (D_j/q_i)  mod t
 * limbs of D_j itself are copied.  x: [(l+1)][n]; ext: [(l+1+alpha)][n].
 */
void or_modup_digit(const or_ring *R, int l, int j, const uint64_t *x, uint64_t *ext)
{
    int n = R->n, lo = j * R->alpha, hi = (j + 1) * R->alpha;
    if (hi > l + 1) hi = l + 1;
    int m = hi - lo;
    /* v_a = [x_a * (D_j/q_a)^{-1}]_{q_a} for every coefficient */
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)m * n);
#pragma omp parallel for schedule(static)
    for (int a = 0; a < m; a++) {
        uint64_t qa = R->q[lo + a], prod = 1;
        for (int b = 0; b < m; b++) if (b != a) prod = or_mulmod(prod, R->q[lo + b] % qa, qa);
        uint64_t hat_inv = invm(prod, qa);
        for (int k = 0; k < n; k++) v[(size_t)a * n + k] = or_mulmod(x[(size_t)(lo + a) * n + k], hat_inv, qa);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < l + 1 + R->alpha; t++) {
        uint64_t pt = ext_prime(R, l, t), hat_t[64];
        if (t >= lo && t < hi) { memcpy(ext + (size_t)t * n, x + (size_t)t * n, sizeof(uint64_t) * n); continue; }
        for (int a = 0; a < m; a++) { /* (D_j/q_a) mod t */
            uint64_t prod = 1;
            for (int b = 0; b < m; b++) if (b != a) prod = or_mulmod(prod, R->q[lo + b] % pt, pt);
            hat_t[a] = prod;
        }
        for (int k = 0; k < n; k++) {
            uint64_t acc = 0;
            for (int a = 0; a < m; a++) acc = addm(acc, or_mulmod(v[(size_t)a * n + k] % pt, hat_t[a], pt), pt);
            ext[(size_t)t * n + k] = acc;
        }
    }
    free(v);
}

/* all digits: ext_all [n_digits(l)][(l+1+alpha)][n] */
void or_modup(const or_ring *R, int l, const uint64_t *x, uint64_t *ext_all)
{
    size_t stride = (size_t)(l + 1 + R->alpha) * R->n;
    for (int j = 0; j < n_digits(R, l); j++) or_modup_digit(R, l, j, x, ext_all + j * stride);
}

/*
 * ModDown: u over Q_l u P  ->  (u - conv_P->Q(u_P)) * P^{-1} over Q_l, with
 *   conv_i = sum_k [u_{p_k} (P/p_k)^{-1}]_{p_k} (P/p_k)  mod q_i.
 */
void or_moddown(const or_ring *R, int l, const uint64_t *u, uint64_t *out)
{
    int n = R->n, al = R->alpha;
    uint64_t *hat_inv = (uint64_t *)malloc(sizeof(uint64_t) * al);
    for (int a = 0; a < al; a++) {
        uint64_t pa = R->p[a], prod = 1;
        for (int b = 0; b < al; b++) if (b != a) prod = or_mulmod(prod, R->p[b] % pa, pa);
        hat_inv[a] = invm(prod, pa);
    }
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * al * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int a = 0; a < al; a++)
        for (int k = 0; k < n; k++) v[(size_t)a * n + k] = or_mulmod(u[(size_t)(l + 1 + a) * n + k], hat_inv[a], R->p[a]);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i <= l; i++) {
        uint64_t qi = R->q[i], Pmod = 1;
        uint64_t *hat_i = (uint64_t *)malloc(sizeof(uint64_t) * al);
        for (int a = 0; a < al; a++) {
            uint64_t prod = 1;
            for (int b = 0; b < al; b++) if (b != a) prod = or_mulmod(prod, R->p[b] % qi, qi);
            hat_i[a] = prod;
            Pmod = or_mulmod(Pmod, R->p[a] % qi, qi);
        }
        uint64_t Pinv = invm(Pmod, qi);
        for (int k = 0; k < n; k++) {
            uint64_t acc = 0;
            for (int a = 0; a < al; a++) acc = addm(acc, or_mulmod(v[(size_t)a * n + k] % qi, hat_i[a], qi), qi);
            out[(size_t)i * n + k] = or_mulmod(subm(u[(size_t)i * n + k], acc, qi), Pinv, qi);
        }
        free(hat_i);
    }
    free(v);
    free(hat_inv);
}

/*
 * Key inner product + ModDown from already-extended digits.
 * ext_all: [n_digits(l)][(l+1+alpha)][n] (the ModUp of the polynomial to switch);
 * if g != 1 each extended limb is first mapped by the automorphism X -> X^g
 * (hoisted rotation).  key: [n_digits(L)][2][(L+1+alpha)][n].
 * out0/out1: [(l+1)][n].
 */
/* key inner product (u0, u1) = sum_j tau_g(ext_j) (b_j, a_j) over Q_l u P, coefficient form */
void or_key_ip(const or_ring *R, int l, const uint64_t *ext_all, uint64_t g, const uint64_t *key, uint64_t *u0,
               uint64_t *u1)
{
    int n = R->n, ne = l + 1 + R->alpha, nk = R->L + 1 + R->alpha;
    size_t stride = (size_t)ne * n;
    memset(u0, 0, stride * sizeof(uint64_t));
    memset(u1, 0, stride * sizeof(uint64_t));
    for (int j = 0; j < n_digits(R, l); j++) {
        const uint64_t *kb = key + ((size_t)j * 2 + 0) * nk * n;
        const uint64_t *ka = key + ((size_t)j * 2 + 1) * nk * n;
#pragma omp parallel for schedule(dynamic, 1)
        for (int t = 0; t < ne; t++) {
            uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * n), *prd = (uint64_t *)malloc(sizeof(uint64_t) * n);
            uint64_t pt = ext_prime(R, l, t);
            const uint64_t *y = ext_all + j * stride + (size_t)t * n;
            if (g != 1) { or_automorph(y, tmp, n, g, pt); y = tmp; }
            int kl = key_limb(R, l, t);
            or_polymul(y, kb + (size_t)kl * n, prd, n, pt);
            for (int k = 0; k < n; k++) u0[(size_t)t * n + k] = addm(u0[(size_t)t * n + k], prd[k], pt);
            or_polymul(y, ka + (size_t)kl * n, prd, n, pt);
            for (int k = 0; k < n; k++) u1[(size_t)t * n + k] = addm(u1[(size_t)t * n + k], prd[k], pt);
            free(tmp); free(prd);
        }
    }
}

void or_keyswitch_ext(const or_ring *R, int l, const uint64_t *ext_all, uint64_t g, const uint64_t *key,
                      uint64_t *out0, uint64_t *out1)
{
    size_t stride = (size_t)(l + 1 + R->alpha) * R->n;
    uint64_t *u0 = (uint64_t *)malloc(stride * sizeof(uint64_t));
    uint64_t *u1 = (uint64_t *)malloc(stride * sizeof(uint64_t));
    or_key_ip(R, l, ext_all, g, key, u0, u1);
    or_moddown(R, l, u0, out0);
    or_moddown(R, l, u1, out1);
    free(u0); free(u1);
}

/* plain (non-hoisted) key switch of d: ModUp -> inner product -> ModDown */
void or_keyswitch(const or_ring *R, int l, const uint64_t *d, const uint64_t *key, uint64_t *out0, uint64_t *out1)
{
    size_t sz = (size_t)n_digits(R, l) * (l + 1 + R->alpha) * R->n;
    uint64_t *ext = (uint64_t *)malloc(sizeof(uint64_t) * sz);
    or_modup(R, l, d, ext);
    or_keyswitch_ext(R, l, ext, 1, key, out0, out1);
    free(ext);
}

/*
 * Key-switching key from s' to s (both small integer polynomials):
 *   b_j = -a_j s + e_j + P g_j s'  (mod every top-level prime),  key_j = (b_j, a_j),
 * where g_j is 1 modulo the primes of top-level digit j and 0 modulo all others.
 * a: [dnum][(L+1+alpha)][n] uniform residues;  e: [dnum][n].
 */
void or_switch_key(const or_ring *R, const int64_t *s, const int64_t *sp, const uint64_t *a, const int64_t *e,
                   uint64_t *key)
{
    int n = R->n, L = R->L, nk = L + 1 + R->alpha, dn = n_digits(R, L);
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int j = 0; j < dn; j++) {
        for (int t = 0; t < nk; t++) {
            uint64_t *prd = (uint64_t *)malloc(sizeof(uint64_t) * n);
            uint64_t pt = t <= L ? R->q[t] : R->p[t - L - 1];
            const uint64_t *aj = a + ((size_t)j * nk + t) * n;
            uint64_t *b = key + (((size_t)j * 2 + 0) * nk + t) * n;
            uint64_t *ak = key + (((size_t)j * 2 + 1) * nk + t) * n;
            memcpy(ak, aj, sizeof(uint64_t) * n);
            polymul_small(aj, s, prd, n, pt);
            int in_digit = (t <= L) && (t / R->alpha == j);
            uint64_t Pmod = 1;
            for (int k = 0; k < R->alpha; k++) Pmod = or_mulmod(Pmod, R->p[k] % pt, pt);
            for (int k = 0; k < n; k++) {
                uint64_t v = subm(from_i64(e[(size_t)j * n + k], pt), prd[k], pt);
                if (in_digit) v = addm(v, or_mulmod(Pmod, from_i64(sp[k], pt), pt), pt);
                b[k] = v;
            }
            free(prd);
        }
    }
}

/* -------------------------------------------------------- ciphertext level */

/* rescale one polynomial: a_i' = (a_i - r) q_l^{-1} mod q_i, r = centred [a]_{q_l}; in [(l+1)][n], out [l][n] */
void or_rescale(const or_ring *R, int l, const uint64_t *a, uint64_t *out)
{
    int n = R->n;
    uint64_t ql = R->q[l];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < l; i++) {
        uint64_t qi = R->q[i], inv = invm(ql % qi, qi);
        for (int k = 0; k < n; k++) {
            uint64_t v = a[(size_t)l * n + k];
            uint64_t r = (v > ql / 2) ? negm((ql - v) % qi, qi) : v % qi; /* centred lift of v, mod q_i */
            out[(size_t)i * n + k] = or_mulmod(subm(a[(size_t)i * n + k], r, qi), inv, qi);
        }
    }
}

/* ModRaise of one polynomial from level 0 to level L: every limb gets the centred lift of [a]_{q_0} */
void or_modraise(const or_ring *R, int L, const uint64_t *a0, uint64_t *out)
{
    int n = R->n;
    uint64_t q0 = R->q[0];
#pragma omp parallel for schedule(static)
    for (int i = 0; i <= L; i++) {
        uint64_t qi = R->q[i];
        for (int k = 0; k < n; k++) {
            uint64_t v = a0[k];
            out[(size_t)i * n + k] = (v > q0 / 2) ? negm((q0 - v) % qi, qi) : v % qi;
        }
    }
}

/* secret-key encryption at level l: (c0, c1) = (-a s + e + m, a); ct [2][(l+1)][n] */
void or_encrypt_sk(const or_ring *R, int l, const int64_t *s, const uint64_t *m, const uint64_t *a, const int64_t *e,
                   uint64_t *ct)
{
    int n = R->n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i <= l; i++) {
        uint64_t qi = R->q[i], *prd = (uint64_t *)malloc(sizeof(uint64_t) * n);
        polymul_small(a + (size_t)i * n, s, prd, n, qi);
        for (int k = 0; k < n; k++) {
            ct[(size_t)i * n + k] = addm(subm(from_i64(e[k], qi), prd[k], qi), m[(size_t)i * n + k], qi);
            ct[((size_t)(l + 1) + i) * n + k] = a[(size_t)i * n + k];
        }
        free(prd);
    }
}

/* Public-key encryption (Sec. 2.1: Enc(m; pk) with pk = (-a s + e, a), an encryption of
 * zero at the top level): ct = (v pk0 + e0 + m, v pk1 + e1) at level l, from the first
 * l+1 limbs of pk [2][L+1][n], small signed v, e0, e1 [n]; ct [2][(l+1)][n]. */
void or_encrypt_pk(const or_ring *R, int l, const uint64_t *pk, const uint64_t *m, const int64_t *v, const int64_t *e0,
                   const int64_t *e1, uint64_t *ct)
{
    int n = R->n, L1 = R->L + 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i <= l; i++) {
        uint64_t qi = R->q[i], *p0 = (uint64_t *)malloc(sizeof(uint64_t) * n), *p1 = (uint64_t *)malloc(sizeof(uint64_t) * n);
        polymul_small(pk + (size_t)i * n, v, p0, n, qi);
        polymul_small(pk + ((size_t)L1 + i) * n, v, p1, n, qi);
        for (int k = 0; k < n; k++) {
            ct[(size_t)i * n + k] = addm(addm(p0[k], from_i64(e0[k], qi), qi), m[(size_t)i * n + k], qi);
            ct[((size_t)(l + 1) + i) * n + k] = addm(p1[k], from_i64(e1[k], qi), qi);
        }
        free(p0), free(p1);
    }
}

/* decryption polynomial c0 + c1 s at level l; out [(l+1)][n] */
void or_decrypt(const or_ring *R, int l, const int64_t *s, const uint64_t *ct, uint64_t *out)
{
    int n = R->n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i <= l; i++) {
        uint64_t qi = R->q[i], *prd = (uint64_t *)malloc(sizeof(uint64_t) * n);
        polymul_small(ct + ((size_t)(l + 1) + i) * n, s, prd, n, qi);
        for (int k = 0; k < n; k++) out[(size_t)i * n + k] = addm(ct[(size_t)i * n + k], prd[k], qi);
        free(prd);
    }
}

/* per-limb product of a level-l polynomial with a plaintext: out_i = a_i * pt_i */
void or_poly_pmult(const or_ring *R, int l, const uint64_t *a, const uint64_t *pt, uint64_t *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i <= l; i++) or_polymul(a + (size_t)i * R->n, pt + (size_t)i * R->n, out + (size_t)i * R->n, R->n, R->q[i]);
}

/* per-limb automorphism of a level-l polynomial */
void or_poly_automorph(const or_ring *R, int l, const uint64_t *a, uint64_t g, uint64_t *out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i <= l; i++) or_automorph(a + (size_t)i * R->n, out + (size_t)i * R->n, R->n, g, R->q[i]);
}

/* per-limb multiplication by X^k */
void or_poly_monomial(const or_ring *R, int l, const uint64_t *a, int k, uint64_t *out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i <= l; i++) or_monomial(a + (size_t)i * R->n, out + (size_t)i * R->n, R->n, k, R->q[i]);
}
