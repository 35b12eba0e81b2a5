// Live kernel timing with HIP events (used for roofline reports).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace nj {

static hipEvent_t take_event(nj_ctx *c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(const nj_ctx *cc, int kind, double bytes, hipStream_t st) : c(const_cast<nj_ctx *>(cc)), s(st)
{
    r.kind = kind;
    r.bytes = bytes;
    r.a = r.b = nullptr;
    if (!c->prof) return;
    r.a = take_event(c);
    r.b = take_event(c);
    if (r.a) (void)hipEventRecord(r.a, s);
}

bool prof_events(const nj_ctx *cc, int kind, double bytes, hipEvent_t *a, hipEvent_t *b)
{
    nj_ctx *c = const_cast<nj_ctx *>(cc);
    ProfRec r;
    r.kind = kind;
    r.bytes = bytes;
    r.a = take_event(c);
    r.b = take_event(c);
    if (!r.a || !r.b) return false;
    c->prof_recs.push_back(r);
    *a = r.a, *b = r.b;
    return true;
}

ProfScope::~ProfScope()
{
    if (!c->prof || !r.a || !r.b) return;
    (void)hipEventRecord(r.b, s);
    c->prof_recs.push_back(r);
}

}  // namespace nj

using namespace nj;

extern "C" {

nj_status nj_prof_enable(nj_ctx *c, int on)
{
    if (!c) return fail(NJ_EINVAL, "nj_prof_enable: null context");
    c->prof = on != 0;
    return NJ_OK;
}

nj_status nj_prof_read(nj_ctx *c, int kind, int *launches, double *total_ms, double *total_bytes, int reset)
{
    if (!c || !launches || !total_ms || !total_bytes || kind < 0 || kind >= PROF_KINDS)
        return fail(NJ_EINVAL, "nj_prof_read: bad arguments");
    NJ_HIP(hipDeviceSynchronize());
    int n = 0;
    double ms = 0.0, by = 0.0;
    for (const ProfRec &r : c->prof_recs) {
        if (r.kind != kind) continue;
        float t = 0.f;
        NJ_HIP(hipEventElapsedTime(&t, r.a, r.b));
        n++, ms += t, by += r.bytes;
    }
    *launches = n, *total_ms = ms, *total_bytes = by;
    if (reset) {
        std::vector<ProfRec> keep;
        for (const ProfRec &r : c->prof_recs) {
            if (r.kind == kind) c->ev_pool.push_back(r.a), c->ev_pool.push_back(r.b);
            else keep.push_back(r);
        }
        c->prof_recs.swap(keep);
    }
    return NJ_OK;
}

}  // extern "C"
