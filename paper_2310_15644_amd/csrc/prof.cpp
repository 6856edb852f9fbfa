// HIP-event timing of library launches (measurement support, off by default).
#include <vector>

#include "efie_internal.h"

namespace efie {
namespace {
struct Rec {
    int id;
    hipEvent_t a, b;
    double work;
};
bool g_on = false;
std::vector<hipEvent_t> g_pool;
std::vector<Rec> g_pending;
hipEvent_t g_open[PROF_COUNT];
bool g_is_open[PROF_COUNT] = {};
double g_ms[PROF_COUNT] = {};
double g_work[PROF_COUNT] = {};
int64_t g_n[PROF_COUNT] = {};

hipEvent_t take() {
    if (g_pool.empty()) {
        hipEvent_t e;
        EFIE_HIP_CHECK(hipEventCreate(&e));
        return e;
    }
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
}

void drain() {
    for (auto& r : g_pending) {
        EFIE_HIP_CHECK(hipEventSynchronize(r.b));
        float ms = 0.f;
        EFIE_HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
        g_ms[r.id] += ms;
        g_work[r.id] += r.work;
        g_n[r.id] += 1;
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_pending.clear();
}
}  // namespace

void prof_begin(int id, hipStream_t s) {
    if (!g_on) return;
    hipEvent_t e = take();
    EFIE_HIP_CHECK(hipEventRecord(e, s));
    g_open[id] = e;
    g_is_open[id] = true;
}

void prof_end(int id, hipStream_t s, double work) {
    if (!g_on || !g_is_open[id]) return;
    hipEvent_t e = take();
    EFIE_HIP_CHECK(hipEventRecord(e, s));
    g_pending.push_back({id, g_open[id], e, work});
    g_is_open[id] = false;
    if (g_pending.size() > 4096) drain();
}
}  // namespace efie

extern "C" int efie_prof_enable(int on) {
    return efie::guarded([&]() {
        efie::g_on = on != 0;
        return int(EFIE_OK);
    });
}

extern "C" int efie_prof_reset(void) {
    return efie::guarded([&]() {
        efie::drain();
        for (int i = 0; i < efie::PROF_COUNT; ++i) {
            efie::g_ms[i] = 0.0;
            efie::g_work[i] = 0.0;
            efie::g_n[i] = 0;
        }
        return int(EFIE_OK);
    });
}

extern "C" int efie_prof_read(int id, int64_t* launches, double* total_ms, double* total_work) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(id >= 0 && id < efie::PROF_COUNT && launches && total_ms, EFIE_ERR_ARG, "prof_read: bad argument");
        efie::drain();
        *launches = efie::g_n[id];
        *total_ms = efie::g_ms[id];
        if (total_work) *total_work = efie::g_work[id];
        return int(EFIE_OK);
    });
}
