// Per-kernel HIP-event timing for libcola launches (a diagnostic, off by default).
//
// While enabled, every launcher brackets its kernel with an event pair recorded on the launch
// stream; cola_profiler_read synchronises the recorded events and reports total milliseconds
// and launch counts per kernel kind.  Events come from a pool that is reused across reads.

#include <mutex>
#include <vector>

#include "cola_internal.h"

namespace cola {

namespace {

const char* const kKindNames[PROF_NUM_KINDS] = {
    "fill", "cic_deposit", "fft_z_r2c", "fft_y_forward", "fft_x_forward", "fft_x_green",
    "fft_y_split", "fft_y_inverse", "fft_z_c2r", "gather_kick_drift", "gather_force",
    "ic_kernels", "fft_x_inverse_mult", "pk_bin", "copy", "other", "gather_kick", "pk_deposit", "cic_sort", "cic_tile",
    "lc_conv3", "lc_conv3_wgrad", "lc_other", "fof", "pk_alias", "fft_z_c2r3"};

struct Record {
    int kind;
    long tag;
    hipEvent_t start, stop;
};

struct Profiler {
    std::mutex mu;
    bool enabled = false;
    std::vector<hipEvent_t> pool;
    std::vector<Record> records;
    int depth = 0;  // nested scopes record only the outermost launch
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

Profiler& prof() {
    static Profiler p;
    return p;
}

}  // namespace

ProfScope::ProfScope(int kind, hipStream_t st, long tag) : kind_(kind), tag_(tag), st_(st) {
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.enabled) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    counted_ = true;
    if (p.depth++ > 0) return;
    start_ = p.get();
    if (start_) (void)hipEventRecord(start_, st_);
}

ProfScope::~ProfScope() {
    if (!counted_) return;
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    --p.depth;
    if (!p.enabled || !start_) return;
    hipEvent_t stop = p.get();
    if (!stop) return;
    (void)hipEventRecord(stop, st_);
    p.records.push_back({kind_, tag_, start_, stop});
}

}  // namespace cola

using namespace cola;

extern "C" {

int cola_profiler_enable(int on) {
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    for (auto& r : p.records) {
        p.pool.push_back(r.start);
        p.pool.push_back(r.stop);
    }
    p.records.clear();
    p.depth = 0;
    p.enabled = on != 0;
    return COLA_OK;
}

int cola_profiler_num_kinds(void) { return PROF_NUM_KINDS; }

const char* cola_profiler_kind_name(int kind) {
    if (kind < 0 || kind >= PROF_NUM_KINDS) return "";
    return kKindNames[kind];
}

int cola_profiler_read(int32_t n_kinds, double* total_ms, int64_t* launches) {
    if (!total_ms || !launches || n_kinds < 1) return COLA_ERR_INVALID_ARG;
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    for (int k = 0; k < n_kinds; ++k) {
        total_ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto& r : p.records) {
        if (hipEventSynchronize(r.stop) != hipSuccess) return COLA_ERR_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return COLA_ERR_HIP;
        if (r.kind < n_kinds) {
            total_ms[r.kind] += ms;
            launches[r.kind] += 1;
        }
        p.pool.push_back(r.start);
        p.pool.push_back(r.stop);
    }
    p.records.clear();
    return COLA_OK;
}

int cola_profiler_read_groups(int32_t cap, int32_t* kinds, int64_t* tags, double* total_ms, int64_t* launches) {
    if (cap < 1 || !kinds || !tags || !total_ms || !launches) return COLA_ERR_INVALID_ARG;
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    int n = 0;
    for (auto& r : p.records) {
        if (hipEventSynchronize(r.stop) != hipSuccess) return COLA_ERR_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return COLA_ERR_HIP;
        int i = 0;
        while (i < n && !(kinds[i] == r.kind && tags[i] == r.tag)) ++i;
        if (i == n) {
            if (n == cap) return COLA_ERR_INVALID_ARG;
            kinds[i] = r.kind;
            tags[i] = r.tag;
            total_ms[i] = 0.0;
            launches[i] = 0;
            ++n;
        }
        total_ms[i] += ms;
        launches[i] += 1;
    }
    for (auto& r : p.records) {
        p.pool.push_back(r.start);
        p.pool.push_back(r.stop);
    }
    p.records.clear();
    return n;
}

}  // extern "C"
