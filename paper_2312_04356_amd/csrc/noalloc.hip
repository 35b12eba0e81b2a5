// Key switching for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops that forbid allocation): nj_apply_galois with its scratch in
// a fixed device array of this file instead of the context's growable arena.
#include <hip/hip_runtime.h>

#include <mutex>

#include "exec.h"

using namespace nj;
using namespace nj::ex;

// 20 Mi words = 160 MiB per GPU: one key switch at any level of N = 2^16 with 24
// ciphertext primes and 8 special primes needs 296 N = 19.4 Mi words (apply_galois'
// ModUp digits, inner products, ModDown limbs and the copy of c0 when in == out).
#define NJ_NOALLOC_WORDS (20u << 20)
#define NJ_NOALLOC_DEVICES 64

static __device__ __align__(256) uint64_t scratch[NJ_NOALLOC_WORDS];

namespace nj {

static std::mutex g_noalloc_mu;
static uint64_t *g_noalloc_ptr[NJ_NOALLOC_DEVICES];
static hipError_t g_noalloc_err[NJ_NOALLOC_DEVICES];
static bool g_noalloc_done[NJ_NOALLOC_DEVICES];

// Device address of `scratch` on `device` (which must be current): the symbol's host
// name is not a device address, so the address is looked up once per device and kept.
hipError_t noalloc_init(int device)
{
    if (device < 0 || device >= NJ_NOALLOC_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_done[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_noalloc_err[device] = e;
        g_noalloc_ptr[device] = e == hipSuccess ? static_cast<uint64_t *>(p) : nullptr;
        g_noalloc_done[device] = true;
    }
    return g_noalloc_err[device];
}

}  // namespace nj

extern "C" nj_status nj_apply_galois_noalloc(nj_ctx *c, const nj_ct *in, uint32_t g, nj_ct *out, void *stream)
{
    nj_status st = check_ct(c, in, "nj_apply_galois_noalloc");
    if (st) return st;
    if (!out || !out->data) return fail(NJ_EINVAL, "nj_apply_galois_noalloc: null output");
    if (c->prof)
        return fail(NJ_EUNSUPPORTED, "nj_apply_galois_noalloc: live profiling is on (it creates HIP events)");
    const size_t need = ks_words(c, in->level);
    if (need > NJ_NOALLOC_WORDS)
        return fail(NJ_EUNSUPPORTED, "nj_apply_galois_noalloc: this key switch needs " + std::to_string(need) +
                                         " scratch words, the static buffer holds " +
                                         std::to_string((size_t)NJ_NOALLOC_WORDS));
    if (g % 2 == 0 || g >= 2u * (uint32_t)c->N)
        return fail(NJ_EINVAL, "nj_apply_galois_noalloc: Galois element must be odd and below 2N");
    if (g != 1 && !key_of(c, g)) return fail(NJ_ENOKEY, "nj_apply_galois_noalloc: no switching key for that element");
    if (c->device < 0 || c->device >= NJ_NOALLOC_DEVICES)
        return fail(NJ_EUNSUPPORTED, "nj_apply_galois_noalloc: device index out of range");
    uint64_t *ptr;
    hipError_t e;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        ptr = g_noalloc_ptr[c->device];
        e = g_noalloc_done[c->device] ? g_noalloc_err[c->device] : hipErrorNotInitialized;
    }
    if (!ptr) return hip_fail(e, "nj_apply_galois_noalloc: static scratch address");
    Arena A{ptr, (size_t)NJ_NOALLOC_WORDS};
    st = apply_galois(c, in->level, in->data, g, out->data, A, S(stream));
    if (st) return st;
    out->level = in->level, out->is_ntt = 1, out->scale = in->scale;
    return NJ_OK;
}
