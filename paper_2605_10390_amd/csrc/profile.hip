// Event-pair recorder behind include/fs_profile.h.  Host code only.
#include "fs_profile.h"
#include "fs_internal.hpp"

#include <mutex>
#include <vector>

namespace fs {

namespace {
struct Record {
    int kind;
    uint64_t keys;
    hipEvent_t begin, end;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Record> g_records;
std::vector<hipEvent_t> g_pool;
// calls on this thread that must not create events (the allocation-free
// entry point) hold a ProfileSuspend
thread_local int g_suspended = 0;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void recycle_all() {
    for (auto& r : g_records) {
        g_pool.push_back(r.begin);
        g_pool.push_back(r.end);
    }
    g_records.clear();
}
}  // namespace

bool profiling() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_on;
}

ProfileSuspend::ProfileSuspend() { ++g_suspended; }
ProfileSuspend::~ProfileSuspend() { --g_suspended; }

void profile_mark(int kind, uint64_t keys, hipStream_t s, hipEvent_t* begin_out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || g_suspended) {
        *begin_out = nullptr;
        return;
    }
    hipEvent_t b = take_event();
    if (b && hipEventRecord(b, s) != hipSuccess) {
        g_pool.push_back(b);
        b = nullptr;
    }
    *begin_out = b;
    (void)kind;
    (void)keys;
}

void profile_close(int kind, uint64_t keys, hipStream_t s, hipEvent_t begin) {
    if (!begin) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t e = take_event();
    if (!e || hipEventRecord(e, s) != hipSuccess) {
        g_pool.push_back(begin);
        if (e) g_pool.push_back(e);
        return;
    }
    g_records.push_back(Record{kind, keys, begin, e});
}

}  // namespace fs

extern "C" int fs_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(fs::g_mu);
    const int prev = fs::g_on ? 1 : 0;
    if (on) fs::recycle_all();
    fs::g_on = on != 0;
    return prev;
}

extern "C" int fs_profile_read(int kind, uint64_t* launches, uint64_t* keys, double* total_ms) {
    if (kind < 0 || kind >= FS_KERNEL_KINDS) return -1;
    std::lock_guard<std::mutex> lk(fs::g_mu);
    uint64_t c = 0, k = 0;
    double ms = 0.0;
    for (auto& r : fs::g_records) {
        if (r.kind != kind) continue;
        if (hipEventSynchronize(r.end) != hipSuccess) return -1;
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.begin, r.end) != hipSuccess) return -1;
        ++c;
        k += r.keys;
        ms += t;
    }
    if (launches) *launches = c;
    if (keys) *keys = k;
    if (total_ms) *total_ms = ms;
    return 0;
}
