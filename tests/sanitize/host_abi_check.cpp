// The library's host-only entry points run under AddressSanitizer and
// UndefinedBehaviorSanitizer (built and run by tests/test_sanitizers.py, no GPU needed):
// slot and CinS encoders and the decoder, prime generation, conv tap lists, Chebyshev
// coefficients, layer masks and the context's parameter refusals, with their error paths.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "neujeans.h"

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                                \
        }                                                                            \
    } while (0)

int main()
{
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    // slots -> coefficients -> slots
    for (int log_n : {4, 10, 12}) {
        const int N = 1 << log_n;
        std::vector<double> z(N), back(N), cd(N);
        std::vector<int64_t> c(N);
        for (double &v : z) v = u(rng);
        CHECK(nj_encode_slots(log_n, z.data(), std::ldexp(1.0, 30), c.data()) == NJ_OK);
        for (int k = 0; k < N; k++) cd[k] = (double)c[k];
        CHECK(nj_decode_slots(log_n, cd.data(), std::ldexp(1.0, 30), back.data()) == NJ_OK);
        double err = 0;
        for (int k = 0; k < N; k++) err = std::fmax(err, std::fabs(back[k] - z[k]));
        CHECK(err < 1e-6);
    }
    CHECK(nj_encode_slots(1, nullptr, 1.0, nullptr) == NJ_EINVAL);
    CHECK(nj_last_error() != nullptr);
    // real CinS: C channels of 2l reals
    {
        const int log_n = 12, N = 1 << log_n, l2 = 64, C = N / l2;
        std::vector<double> ch((size_t)C * l2);
        for (double &v : ch) v = u(rng);
        std::vector<int64_t> out(N);
        CHECK(nj_encode_cins(log_n, ch.data(), l2, std::ldexp(1.0, 30), out.data()) == NJ_OK);
        CHECK(nj_encode_cins(log_n, ch.data(), 48, 1.0, out.data()) == NJ_EINVAL);  // not a power of two
    }
    // primes p = 1 mod 2N below 2^bits, distinct from an excluded list
    {
        std::vector<uint64_t> q(6), p(3);
        CHECK(nj_gen_primes(12, 50, 6, nullptr, 0, q.data()) == NJ_OK);
        CHECK(nj_gen_primes(12, 50, 3, q.data(), 6, p.data()) == NJ_OK);
        for (uint64_t x : q) CHECK(x % 8192 == 1 && x < (1ull << 50));
        for (uint64_t x : p)
            for (uint64_t y : q) CHECK(x != y);
        CHECK(nj_gen_primes(12, 62, 1, nullptr, 0, q.data()) == NJ_EINVAL);
    }
    // conv tap lists: counts first, then the taps; short buffers are refused
    {
        struct Case {
            int c_in, c_out, f, stride, dw;
        } cases[] = {{16, 16, 3, 1, 0}, {64, 128, 3, 2, 0}, {16, 16, 3, 1, 1}, {64, 128, 1, 2, 0}, {3, 64, 7, 2, 0}};
        for (const Case &k : cases) {
            const size_t nw = k.dw ? (size_t)k.c_in * k.f * k.f : (size_t)k.c_out * k.c_in * k.f * k.f;
            std::vector<double> w(nw);
            for (double &v : w) v = u(rng);
            int n = 0;
            CHECK(nj_conv_taps(k.c_in, k.c_out, k.f, k.stride, k.dw, w.data(), nullptr, 0, &n) == NJ_OK && n > 0);
            std::vector<nj_tap> taps(n);
            int n2 = 0;
            CHECK(nj_conv_taps(k.c_in, k.c_out, k.f, k.stride, k.dw, w.data(), taps.data(), n, &n2) == NJ_OK);
            CHECK(n2 == n);
            for (const nj_tap &t : taps) CHECK(t.out_ch >= 0 && t.out_ch < k.c_out && t.in_ch >= 0);
            if (n > 1) CHECK(nj_conv_taps(k.c_in, k.c_out, k.f, k.stride, k.dw, w.data(), taps.data(), n - 1, &n2) ==
                             NJ_EINVAL);
        }
        double w1 = 1.0;
        int n = 0;
        CHECK(nj_conv_taps(1, 1, 2, 1, 0, &w1, nullptr, 0, &n) == NJ_EINVAL);  // even kernel width
    }
    // Chebyshev interpolant and layer masks
    {
        std::vector<double> cf(64);
        CHECK(nj_cheb_interpolate(63, 32.0, 3, cf.data()) == NJ_OK);
        CHECK(nj_cheb_interpolate(-1, 32.0, 3, cf.data()) == NJ_EINVAL);
        const int log_n = 12, n = 1 << (log_n - 1);
        std::vector<double> re(n), im(n);
        CHECK(nj_layer_masks(log_n, 32, 4, 16, re.data(), im.data()) == NJ_OK);
        double ones = 0;
        for (int j = 0; j < n; j++) ones += re[j] + im[j];
        CHECK(ones == 4.0 * 16 * 16);
    }
    // parameter sets the kernels do not implement are refused before any device work
    {
        std::vector<uint64_t> q(64, 0), p(16, 0);
        nj_params prm{16, 64, 8, q.data(), p.data(), std::ldexp(1.0, 40)};
        nj_ctx *ctx = nullptr;
        CHECK(nj_ctx_create(&prm, &ctx) == NJ_EUNSUPPORTED && ctx == nullptr);
        prm.n_q = 17, prm.alpha = 1;  // 17 digits
        CHECK(nj_ctx_create(&prm, &ctx) == NJ_EUNSUPPORTED && ctx == nullptr);
        CHECK(nj_ctx_create(nullptr, &ctx) == NJ_EINVAL);
    }
    std::printf("host ABI checks passed\n");
    return 0;
}
