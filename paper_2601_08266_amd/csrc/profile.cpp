// Optional per-kernel timing: when enabled, every instrumented launch is
// bracketed by two hipEvents recorded on the launch stream; reading the
// totals waits for the events and sums their elapsed times per kernel name.
// Everything here exists only between fsi_profile_enable(1) and
// fsi_profile_enable(0): disabling destroys the events and the totals.
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "profile.hpp"

namespace fsi {

namespace {

struct Pending {
    int slot;
    hipEvent_t start, stop;
};

struct Registry {
    std::mutex mu;
    bool enabled = false;
    std::vector<std::string> names;
    std::vector<double> total_ms;
    std::vector<int64_t> count;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
};

Registry &reg()
{
    static Registry r;
    return r;
}

int slot_of(Registry &r, const char *name)
{
    for (size_t i = 0; i < r.names.size(); ++i)
        if (r.names[i] == name) return (int)i;
    r.names.emplace_back(name);
    r.total_ms.push_back(0.0);
    r.count.push_back(0);
    return (int)r.names.size() - 1;
}

hipEvent_t take_event(Registry &r)
{
    if (!r.pool.empty()) {
        hipEvent_t e = r.pool.back();
        r.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int drain(Registry &r)
{
    int rc = FSI_OK;
    for (auto &p : r.pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.stop) != hipSuccess ||
            hipEventElapsedTime(&ms, p.start, p.stop) != hipSuccess)
            rc = FSI_ERR_HIP;
        r.total_ms[p.slot] += ms;
        r.count[p.slot] += 1;
        r.pool.push_back(p.start);
        r.pool.push_back(p.stop);
    }
    r.pending.clear();
    return rc;
}

}  // namespace

bool profiling_enabled()
{
    Registry &r = reg();
    std::lock_guard<std::mutex> lk(r.mu);
    return r.enabled;
}

ProfileScope::ProfileScope(const char *name, hipStream_t st) : st_(st)
{
    Registry &r = reg();
    std::lock_guard<std::mutex> lk(r.mu);
    if (!r.enabled) return;
    slot_ = slot_of(r, name);
    start_ = take_event(r);
    stop_ = take_event(r);
    if (start_ && stop_ && hipEventRecord(start_, st_) == hipSuccess) active_ = true;
}

ProfileScope::~ProfileScope()
{
    if (!active_) return;
    Registry &r = reg();
    std::lock_guard<std::mutex> lk(r.mu);
    if (hipEventRecord(stop_, st_) == hipSuccess) r.pending.push_back({slot_, start_, stop_});
}

}  // namespace fsi

using namespace fsi;

extern "C" __attribute__((visibility("default"))) int fsi_profile_enable(int on)
{
    Registry &r = reg();
    std::lock_guard<std::mutex> lk(r.mu);
    int rc = drain(r);
    if (!on) {
        for (hipEvent_t e : r.pool) (void)hipEventDestroy(e);
        std::vector<hipEvent_t>().swap(r.pool);
        std::vector<std::string>().swap(r.names);
        std::vector<double>().swap(r.total_ms);
        std::vector<int64_t>().swap(r.count);
        r.enabled = false;
        return rc;
    }
    for (size_t i = 0; i < r.total_ms.size(); ++i) {
        r.total_ms[i] = 0.0;
        r.count[i] = 0;
    }
    if (r.pool.size() < 512) {
        for (int i = 0; i < 512; ++i) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) {
                set_error("hipEventCreate failed");
                return FSI_ERR_HIP;
            }
            r.pool.push_back(e);
        }
    }
    r.enabled = on != 0;
    return rc;
}

extern "C" __attribute__((visibility("default"))) int fsi_profile_read(const char *kernel,
                                                                       double *total_ms,
                                                                       int64_t *launches)
{
    Registry &r = reg();
    std::lock_guard<std::mutex> lk(r.mu);
    int rc = drain(r);
    if (total_ms) *total_ms = 0.0;
    if (launches) *launches = 0;
    if (kernel == nullptr) return FSI_ERR_ARG;
    for (size_t i = 0; i < r.names.size(); ++i)
        if (r.names[i] == kernel) {
            if (total_ms) *total_ms = r.total_ms[i];
            if (launches) *launches = r.count[i];
        }
    return rc;
}
