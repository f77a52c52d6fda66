// Optional per-kernel timing: when enabled, every kernel launch of the
// library is bracketed by two HIP events recorded on the launch's own stream;
// mm_profile_summary() waits for them and reports count and total time per
// kernel family.  Off by default; costs two event records per launch when on.
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace starmm {

namespace {

struct Rec {
    const char* name;
    hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t st) : name_(name), st_(st), a_(nullptr) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    a_ = get_event();
    if (a_) hipEventRecord((hipEvent_t)a_, st_);
}

ProfScope::~ProfScope() {
    if (!a_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = get_event();
    if (!b) return;
    hipEventRecord(b, st_);
    g_recs.push_back(Rec{name_, (hipEvent_t)a_, b});
}

}  // namespace starmm

using namespace starmm;

extern "C" {

void mm_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
}

void mm_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& r : g_recs) {
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
}

int64_t mm_profile_summary(char* buf, size_t len) {
    std::map<std::string, std::pair<int64_t, double>> agg;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto& r : g_recs) {
            hipEventSynchronize(r.b);
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
            auto& v = agg[r.name];
            v.first += 1;
            v.second += ms;
        }
    }
    std::string out = "{";
    bool first = true;
    for (auto& kv : agg) {
        char tmp[256];
        std::snprintf(tmp, sizeof tmp, "%s\"%s\": [%lld, %.6f]", first ? "" : ", ", kv.first.c_str(),
                      (long long)kv.second.first, kv.second.second);
        out += tmp;
        first = false;
    }
    out += "}";
    if (buf && len > 0) {
        std::strncpy(buf, out.c_str(), len - 1);
        buf[len - 1] = 0;
    }
    return (int64_t)out.size();
}

}  // extern "C"
