// Per-kernel timing with HIP events (wandqs_profile / wandqs_profile_stats).
#include <cstdio>
#include <cstring>

#include "wq_common.h"

namespace wq {
namespace {

int class_of(Prof& p, const char* name) {
    for (size_t i = 0; i < p.names.size(); ++i)
        if (p.names[i] == name) return (int)i;
    p.names.emplace_back(name);
    p.launches.push_back(0);
    p.ms.push_back(0.0);
    p.bytes.push_back(0.0);
    return (int)p.names.size() - 1;
}

bool grow(Prof& p, int n) {
    for (int k = 0; k < n; ++k) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return false;
        p.all_ev.push_back(e);
        p.free_ev.push_back(e);
    }
    return true;
}

}  // namespace

ProfScope::ProfScope(wandqs_ctx* c, const char* name, double bytes) : c_(c), bytes_(bytes) {
    Prof& p = c->prof;
    if (!p.on) return;
    if (p.free_ev.size() < 2) prof_harvest(c);
    if (p.free_ev.size() < 2 && !grow(p, 512)) return;
    cls_ = class_of(p, name);
    a_ = p.free_ev.back();
    p.free_ev.pop_back();
    b_ = p.free_ev.back();
    p.free_ev.pop_back();
}

ProfScope::~ProfScope() {
    if (cls_ < 0) return;
    c_->prof.pending.push_back(ProfPending{cls_, a_, b_, bytes_});
}

void prof_harvest(wandqs_ctx* c) {
    Prof& p = c->prof;
    if (p.pending.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (const ProfPending& q : p.pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
            p.ms[q.cls] += ms;
            p.launches[q.cls] += 1;
            p.bytes[q.cls] += q.bytes;
        }
        p.free_ev.push_back(q.a);
        p.free_ev.push_back(q.b);
    }
    p.pending.clear();
}

void prof_reset(wandqs_ctx* c, bool on) {
    Prof& p = c->prof;
    prof_harvest(c);
    p.names.clear();
    p.launches.clear();
    p.ms.clear();
    p.bytes.clear();
    p.on = on;
    if (on && p.all_ev.empty()) grow(p, 2048);
    if (!on) {
        for (hipEvent_t e : p.all_ev) (void)hipEventDestroy(e);
        p.all_ev.clear();
        p.free_ev.clear();
    }
}

}  // namespace wq

extern "C" {

wandqs_status wandqs_profile(wandqs_ctx* c, int32_t enable) {
    if (!c) return WANDQS_E_INVALID;
    wq::prof_reset(c, enable != 0);
    return WANDQS_OK;
}

wandqs_status wandqs_profile_stats(wandqs_ctx* c, wandqs_kernel_stat* out, int32_t max,
                                   int32_t* n) {
    if (!c || !n || max < 0 || (max > 0 && !out)) return WANDQS_E_INVALID;
    wq::prof_harvest(c);
    const wq::Prof& p = c->prof;
    *n = (int32_t)p.names.size();
    for (int32_t i = 0; i < *n && i < max; ++i) {
        std::memset(&out[i], 0, sizeof(out[i]));
        std::snprintf(out[i].name, sizeof(out[i].name), "%s", p.names[i].c_str());
        out[i].launches = p.launches[i];
        out[i].total_ms = p.ms[i];
        out[i].alg_bytes = p.bytes[i];
    }
    return WANDQS_OK;
}

}  // extern "C"
