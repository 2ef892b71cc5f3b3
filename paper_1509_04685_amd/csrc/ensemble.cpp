// Mock ensembles (Sec. 2.3, Sec. 1): several shape classes of seeded realizations run through
// the library's batched entry points, either eagerly or as one captured hipGraph with each class
// on its own stream so that independent classes overlap on the GPU.

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cola_internal.h"

namespace {

struct GraphCache {
    std::mutex mu;
    std::map<std::string, hipGraphExec_t> execs;
    std::vector<hipStream_t> streams;
};

GraphCache& cache() {
    static GraphCache c;
    return c;
}

template <class T>
void put(std::string& key, const T& v) {
    key.append(reinterpret_cast<const char*>(&v), sizeof(T));
}

std::string make_key(int n_classes, const cola_ensemble_class* cls, const cola_cosmology* cosmo) {
    std::string key;
    put(key, *cosmo);
    put(key, n_classes);
    for (int c = 0; c < n_classes; ++c) {
        const cola_ensemble_class& e = cls[c];
        put(key, e.prob);
        for (int r = 0; r < e.prob.n_real; ++r) put(key, e.seeds[r]);
        for (int d = 0; d < 3; ++d) {
            put(key, e.parts->x[d]);
            put(key, e.parts->p[d]);
            put(key, e.parts->psi1[d]);
            put(key, e.parts->psi2[d]);
        }
        put(key, e.ws);
        put(key, e.ws_bytes);
        put(key, e.n_out);
        for (int k = 0; k < e.n_out; ++k) put(key, e.a_out[k]);
        put(key, e.n_pk);
        put(key, e.n_bins);
        put(key, e.k_mean);
        put(key, e.pk);
        put(key, e.n_modes);
        put(key, e.net);
        put(key, e.lc_ws);
        put(key, e.lc_ws_bytes);
        if (e.net) {  // the host-side scales are baked into the captured launches
            put(key, e.net->params);
            put(key, e.net->packed);
            for (int i = 0; i < 4; ++i) put(key, e.net->in_scale[i]);
            put(key, e.net->out_scale);
            put(key, e.net->out_scale_slope);
            put(key, e.net->out_band);
            put(key, e.net->n_knots);
            for (int i = 0; i < 8; ++i) {
                put(key, e.net->knot_a[i]);
                put(key, e.net->knot_v[i]);
            }
            put(key, e.net->n_gknots);
            put(key, e.net->gknot_u);
            put(key, e.net->gknot_t);
        }
    }
    return key;
}

int node_of(const std::vector<double>& a, double a_out) {
    int j = 0;
    for (size_t i = 0; i < a.size(); ++i)
        if (a[i] <= a_out * (1.0 + 1e-12)) j = (int)i;
    return j;
}

// The class's steps to node j: plain, or corrected by the class's network.
int advance(cola_ensemble_class& e, const cola_cosmology* cosmo, int j, hipStream_t st) {
    if (e.net)
        return cola_step_lc(&e.prob, cosmo, e.parts->node, j, e.parts, e.net, e.lc_ws, e.lc_ws_bytes, e.ws,
                            e.ws_bytes, st);
    return cola_step(&e.prob, cosmo, e.parts->node, j, e.parts, e.ws, e.ws_bytes, st);
}

int run_class(cola_ensemble_class& e, const cola_cosmology* cosmo, hipStream_t st) {
    int s = cola_ic_2lpt(&e.prob, cosmo, e.seeds, e.parts, e.ws, e.ws_bytes, st);
    if (s != COLA_OK) return s;
    std::vector<double> a = cola::time_nodes(e.prob);
    const long nb = (long)e.n_bins * e.prob.n_real;
    for (int k = 0; k < e.n_out; ++k) {
        int j = node_of(a, e.a_out[k]);
        if (j > e.parts->node || (e.net && e.parts->force_node != j)) {
            // a corrected class always steps (even to its own node) so that the corrected force
            // of node j is cached for an output between nodes
            s = advance(e, cosmo, j, st);
            if (s != COLA_OK) return s;
        }
        s = cola_power_spectrum(&e.prob, cosmo, e.parts, e.a_out[k], e.n_pk, e.n_bins, e.k_mean + k * nb,
                                e.pk + k * nb, e.n_modes + k * nb, e.ws, e.ws_bytes, st);
        if (s != COLA_OK) return s;
    }
    if (e.parts->node < e.prob.n_steps - 1) s = advance(e, cosmo, e.prob.n_steps - 1, st);
    return s;
}

int validate(int n_classes, const cola_ensemble_class* cls, const cola_cosmology* cosmo) {
    if (n_classes < 1 || !cls || !cosmo) return COLA_ERR_INVALID_ARG;
    for (int c = 0; c < n_classes; ++c) {
        const cola_ensemble_class& e = cls[c];
        if (!e.seeds || !e.parts || !e.ws || e.n_out < 0 || (e.n_out > 0 && (!e.a_out || !e.k_mean || !e.pk || !e.n_modes)))
            return COLA_ERR_INVALID_ARG;
        size_t need = cola_workspace_bytes(&e.prob, e.n_out > 0 ? e.n_pk : 0);
        if (need == 0) return COLA_ERR_INVALID_ARG;
        if (e.ws_bytes < need) return COLA_ERR_WORKSPACE_TOO_SMALL;
        if (e.net) {
            if (!e.lc_ws) return COLA_ERR_INVALID_ARG;
            const size_t lneed = cola_lc_workspace_bytes(e.prob.n_part * e.prob.pm_factor, e.net->channels,
                                                         e.prob.n_real, 0);
            if (lneed == 0) return COLA_ERR_UNSUPPORTED_SIZE;
            if (e.lc_ws_bytes < lneed) return COLA_ERR_WORKSPACE_TOO_SMALL;
            for (int c2 = 0; c2 < c; ++c2)
                if (cls[c2].lc_ws == e.lc_ws) return COLA_ERR_INVALID_ARG;  // classes run concurrently
        }
        for (int k = 1; k < e.n_out; ++k)
            if (!(e.a_out[k] > e.a_out[k - 1])) return COLA_ERR_INVALID_ARG;
        for (int c2 = 0; c2 < c; ++c2)
            if (cls[c2].ws == e.ws) return COLA_ERR_INVALID_ARG;  // classes run concurrently
    }
    return COLA_OK;
}

}  // namespace

extern "C" {

int cola_ensemble_run(int32_t n_classes, cola_ensemble_class* classes, const cola_cosmology* cosmo, int32_t mode,
                      void* stream) {
    int s = validate(n_classes, classes, cosmo);
    if (s != COLA_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (mode == 0) {
        for (int c = 0; c < n_classes; ++c)
            if ((s = run_class(classes[c], cosmo, st)) != COLA_OK) return s;
        return COLA_OK;
    }
    if (mode != 1) return COLA_ERR_INVALID_ARG;
    GraphCache& gc = cache();
    std::lock_guard<std::mutex> lock(gc.mu);
    const std::string key = make_key(n_classes, classes, cosmo);
    auto it = gc.execs.find(key);
    if (it == gc.execs.end()) {
        // streams[0] is the capture origin (the caller's stream may be the legacy default stream,
        // which cannot be captured); streams[1..] carry one class each.
        while ((int)gc.streams.size() < n_classes + 1) {
            hipStream_t ns = nullptr;
            hipError_t e = hipStreamCreateWithFlags(&ns, hipStreamNonBlocking);
            if (e != hipSuccess) return cola::hip_fail(e, "hipStreamCreateWithFlags");
            gc.streams.push_back(ns);
        }
        hipStream_t origin = gc.streams[0];
        hipEvent_t fork = nullptr;
        std::vector<hipEvent_t> joins(n_classes, nullptr);
        hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (e != hipSuccess) return cola::hip_fail(e, "hipEventCreateWithFlags");
        for (auto& j : joins)
            if ((e = hipEventCreateWithFlags(&j, hipEventDisableTiming)) != hipSuccess)
                return cola::hip_fail(e, "hipEventCreateWithFlags");
        hipGraph_t graph = nullptr;
        if ((e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return cola::hip_fail(e, "hipStreamBeginCapture");
        int status = COLA_OK;
        if ((e = hipEventRecord(fork, origin)) != hipSuccess) status = cola::hip_fail(e, "hipEventRecord(fork)");
        for (int c = 0; c < n_classes && status == COLA_OK; ++c) {
            hipStream_t cs = gc.streams[c + 1];
            if ((e = hipStreamWaitEvent(cs, fork, 0)) != hipSuccess) {
                status = cola::hip_fail(e, "hipStreamWaitEvent(fork)");
                break;
            }
            status = run_class(classes[c], cosmo, cs);
            if (status == COLA_OK && (e = hipEventRecord(joins[c], cs)) != hipSuccess)
                status = cola::hip_fail(e, "hipEventRecord(join)");
            if (status == COLA_OK && (e = hipStreamWaitEvent(origin, joins[c], 0)) != hipSuccess)
                status = cola::hip_fail(e, "hipStreamWaitEvent(join)");
        }
        e = hipStreamEndCapture(origin, &graph);
        if (status == COLA_OK && e != hipSuccess) status = cola::hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        if (status == COLA_OK && (e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess)
            status = cola::hip_fail(e, "hipGraphInstantiate");
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipEventDestroy(fork);
        for (auto& j : joins) (void)hipEventDestroy(j);
        if (status != COLA_OK) return status;
        it = gc.execs.emplace(key, exec).first;
    }
    hipError_t e = hipGraphLaunch(it->second, st);
    if (e != hipSuccess) return cola::hip_fail(e, "hipGraphLaunch");
    return COLA_OK;
}

int cola_ensemble_release(void) {
    GraphCache& gc = cache();
    std::lock_guard<std::mutex> lock(gc.mu);
    for (auto& kv : gc.execs) (void)hipGraphExecDestroy(kv.second);
    gc.execs.clear();
    for (auto s : gc.streams) (void)hipStreamDestroy(s);
    gc.streams.clear();
    return COLA_OK;
}

}  // extern "C"
