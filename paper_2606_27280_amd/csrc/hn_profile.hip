// Optional per-kernel event timing for measurement sessions.
#include <string.h>

#include <mutex>
#include <unordered_map>
#include <vector>

#include "hn_internal.h"

namespace hn {
namespace {

struct Rec {
    const char *tag;
    hipEvent_t a, b;
};
struct Session {
    std::vector<Rec> recs;
};
std::mutex g_mu;
std::unordered_map<void *, Session> g_sessions;

}  // namespace

ProfScope::ProfScope(hipStream_t s, const char *tag) : stream_(s), tag_(tag) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_sessions.empty()) return;
    auto it = g_sessions.find((void *)s);
    if (it == g_sessions.end()) return;
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    active_ = hipEventRecord(a_, s) == hipSuccess;
}

ProfScope::~ProfScope() {
    if (!active_) return;
    if (hipEventRecord(b_, stream_) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_sessions.find((void *)stream_);
    if (it != g_sessions.end()) it->second.recs.push_back(Rec{tag_, a_, b_});
}

}  // namespace hn

using namespace hn;

extern "C" int hn_profile_begin(void *stream) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    g_sessions[stream];
    return HN_OK;
}

extern "C" int hn_profile_end(void *stream, const char **names, double *ms, int64_t *counts,
                              int32_t max, int32_t *n_out) {
    clear_error();
    std::vector<Rec> recs;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_sessions.find(stream);
        if (it == g_sessions.end()) return fail(HN_ERR_INVALID_ARG, "no profile session");
        recs.swap(it->second.recs);
        g_sessions.erase(it);
    }
    HN_HIP(hipStreamSynchronize((hipStream_t)stream));
    int32_t n = 0;
    for (const Rec &r : recs) {
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, r.a, r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
        int32_t j = 0;
        while (j < n && strcmp(names[j], r.tag) != 0) ++j;
        if (j == n) {
            if (n >= max) continue;
            names[n] = r.tag;
            ms[n] = 0.0;
            counts[n] = 0;
            ++n;
        }
        ms[j] += t;
        counts[j] += 1;
    }
    if (n_out) *n_out = n;
    return HN_OK;
}
