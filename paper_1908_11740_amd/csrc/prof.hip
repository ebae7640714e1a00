// Opt-in per-kernel timer: when enabled, every library launch is bracketed
// by a pair of hipEvents on the stream it is launched on; sj_prof_collect()
// folds the elapsed times into per-kernel totals.  Off by default (no events
// are recorded then).
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sj_internal.hpp"
#include "sj_prof.hpp"

namespace sj {
namespace {

struct Rec {
    std::string name;
    hipEvent_t a, b;
};

struct Tot {
    double ms = 0;
    int64_t calls = 0;
};

std::mutex mu;
bool enabled = false;
bool paused = false;
std::vector<hipEvent_t> pool;
std::vector<Rec> pending;
std::vector<std::pair<std::string, Tot>> totals;

hipEvent_t take() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

Tot& slot(const std::string& n) {
    for (auto& t : totals)
        if (t.first == n) return t.second;
    totals.emplace_back(n, Tot{});
    return totals.back().second;
}

}  // namespace

bool prof_pause(bool p) {
    std::lock_guard<std::mutex> lk(mu);
    const bool old = paused;
    paused = p;
    return old;
}

ProfRange::ProfRange(const char* name, hipStream_t s) : name_(name), s_(s), a_(nullptr) {
    std::lock_guard<std::mutex> lk(mu);
    if (!enabled || paused) return;
    a_ = take();
    if (a_ && hipEventRecord((hipEvent_t)a_, s) != hipSuccess) a_ = nullptr;
}

ProfRange::~ProfRange() {
    if (!a_) return;
    std::lock_guard<std::mutex> lk(mu);
    hipEvent_t b = take();
    if (!b || hipEventRecord(b, s_) != hipSuccess) return;
    pending.push_back(Rec{name_, (hipEvent_t)a_, b});
}

}  // namespace sj

extern "C" {

void sj_prof_enable(int on) {
    std::lock_guard<std::mutex> lk(sj::mu);
    sj::enabled = on != 0;
    sj::totals.clear();
    for (auto& r : sj::pending) {
        sj::pool.push_back(r.a);
        sj::pool.push_back(r.b);
    }
    sj::pending.clear();
}

int sj_prof_collect(void) {
    std::lock_guard<std::mutex> lk(sj::mu);
    for (auto& r : sj::pending) {
        (void)hipEventSynchronize(r.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            sj::Tot& t = sj::slot(r.name);
            t.ms += ms;
            t.calls += 1;
        }
        sj::pool.push_back(r.a);
        sj::pool.push_back(r.b);
    }
    sj::pending.clear();
    return (int)sj::totals.size();
}

const char* sj_prof_name(int i) {
    std::lock_guard<std::mutex> lk(sj::mu);
    if (i < 0 || i >= (int)sj::totals.size()) return "";
    return sj::totals[i].first.c_str();
}

double sj_prof_total_ms(int i) {
    std::lock_guard<std::mutex> lk(sj::mu);
    if (i < 0 || i >= (int)sj::totals.size()) return 0.0;
    return sj::totals[i].second.ms;
}

int64_t sj_prof_calls(int i) {
    std::lock_guard<std::mutex> lk(sj::mu);
    if (i < 0 || i >= (int)sj::totals.size()) return 0;
    return sj::totals[i].second.calls;
}

}  // extern "C"
