// C-ABI entry points of the learned coarse-mesh force correction and of the particle-field helpers
// its training uses.  Validation on the host first; nothing is queued on an error return.

#include <cmath>

#include "cola_internal.h"
#include "lc_internal.h"

namespace cola {

namespace {
constexpr int kMaxLcMesh = 1536;
}

bool lc_mesh_ok(int n) { return n >= 16 && n <= kMaxLcMesh && n % 16 == 0; }

LcWsLayout lc_ws_layout(int n, int C, int n_real, bool training) {
    LcWsLayout L;
    const size_t V = (size_t)n * n * n;
    const size_t act = lc_align(V * C * 2);
    L.x0_stride = (long)V * 8;
    size_t off = 0;
    L.x0 = off; off += lc_align(V * 16 * (size_t)n_real);
    L.a1 = off; off += act;
    L.a2 = off; off += act;
    L.t = off; off += lc_align(V * 12);
    if (training) {
        L.z1 = off; off += act;
        L.z2 = off; off += act;
        L.dz1 = off; off += act;
        L.dz2 = off; off += act;
    }
    L.total = off;
    return L;
}

LcActs lc_carve(void* ws, const LcWsLayout& L) {
    char* b = static_cast<char*>(ws);
    LcActs A;
    A.x0 = reinterpret_cast<uint16_t*>(b + L.x0);
    A.a1 = reinterpret_cast<uint16_t*>(b + L.a1);
    A.a2 = reinterpret_cast<uint16_t*>(b + L.a2);
    A.t = reinterpret_cast<float*>(b + L.t);
    const bool tr = L.z1 != 0;
    A.z1 = tr ? reinterpret_cast<uint16_t*>(b + L.z1) : nullptr;
    A.z2 = tr ? reinterpret_cast<uint16_t*>(b + L.z2) : nullptr;
    A.dz1 = tr ? reinterpret_cast<uint16_t*>(b + L.dz1) : nullptr;
    A.dz2 = tr ? reinterpret_cast<uint16_t*>(b + L.dz2) : nullptr;
    return A;
}

int lc_check_net(const cola_lc_net* net, bool training) {
    if (!net || !net->params || !net->packed) return COLA_ERR_INVALID_ARG;
    if (net->channels != 16 && net->channels != 32) return COLA_ERR_INVALID_ARG;
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(net->in_scale[i])) return COLA_ERR_NONFINITE;
    if (!std::isfinite(net->out_scale) || !std::isfinite(net->out_scale_slope) || !std::isfinite(net->out_band))
        return COLA_ERR_NONFINITE;
    if (net->n_knots != 0 && (net->n_knots < 2 || net->n_knots > 8)) return COLA_ERR_INVALID_ARG;
    for (int i = 0; i < net->n_knots; ++i) {
        if (!std::isfinite(net->knot_a[i]) || !std::isfinite(net->knot_v[i])) return COLA_ERR_NONFINITE;
        if (i > 0 && !(net->knot_a[i] > net->knot_a[i - 1])) return COLA_ERR_INVALID_ARG;
    }
    if (net->n_gknots != 0 && (net->n_gknots < 2 || net->n_gknots > 10)) return COLA_ERR_INVALID_ARG;
    const int rows = net->n_knots >= 2 ? net->n_knots : 1;
    for (int j = 0; j < net->n_gknots; ++j) {
        if (!std::isfinite(net->gknot_u[j])) return COLA_ERR_NONFINITE;
        if (j > 0 && !(net->gknot_u[j] > net->gknot_u[j - 1])) return COLA_ERR_INVALID_ARG;
        for (int i = 0; i < rows; ++i)
            if (!std::isfinite(net->gknot_t[i][j])) return COLA_ERR_NONFINITE;
    }
    if (training && (!net->grads || !net->adam_m || !net->adam_v)) return COLA_ERR_INVALID_ARG;
    return COLA_OK;
}

LcParams lc_params_of(const cola_lc_net* net) {
    const int C = net->channels;
    const LcOffsets o = lc_offsets(C);
    const LcPackedOffsets q = lc_packed_offsets(C);
    const char* pk = static_cast<const char*>(net->packed);
    LcParams P;
    P.C = C;
    P.w1 = net->params + o.w1;
    P.b1 = net->params + o.b1;
    P.w2 = net->params + o.w2;
    P.b2 = net->params + o.b2;
    P.w3 = net->params + o.w3;
    P.b3 = net->params + o.b3;
    P.wb1 = reinterpret_cast<const uint16_t*>(pk + q.wb1);
    P.wb2 = reinterpret_cast<const uint16_t*>(pk + q.wb2);
    P.wt2 = reinterpret_cast<const uint16_t*>(pk + q.wt2);
    return P;
}

}  // namespace cola

using namespace cola;

#define LC_TRY(expr)                                         \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(_e, #expr);    \
    } while (0)

namespace {

hipError_t repack(const cola_lc_net* net, hipStream_t st) {
    const LcOffsets o = lc_offsets(net->channels);
    const LcPackedOffsets q = lc_packed_offsets(net->channels);
    char* pk = static_cast<char*>(net->packed);
    return lc_pack_weights(net->params + o.w1, net->params + o.w2, net->channels,
                           reinterpret_cast<uint16_t*>(pk + q.wb1), reinterpret_cast<uint16_t*>(pk + q.wb2),
                           reinterpret_cast<uint16_t*>(pk + q.wt2), st);
}

bool ptrs3(const float* const p[3]) { return p && p[0] && p[1] && p[2]; }

}  // namespace

extern "C" {

int64_t cola_lc_param_count(int32_t channels) {
    if (channels != 16 && channels != 32) return 0;
    return lc_offsets(channels).total;
}

size_t cola_lc_packed_bytes(int32_t channels) {
    if (channels != 16 && channels != 32) return 0;
    return lc_packed_offsets(channels).total;
}

size_t cola_lc_workspace_bytes(int32_t n_mesh, int32_t channels, int32_t n_real, int32_t training) {
    if (!lc_mesh_ok(n_mesh) || (channels != 16 && channels != 32) || n_real < 1) return 0;
    return lc_ws_layout(n_mesh, channels, n_real, training != 0).total;
}

int cola_lc_pack(const cola_lc_net* net, void* stream) {
    int s;
    if ((s = lc_check_net(net, false)) != COLA_OK) return s;
    (void)hipGetLastError();
    LC_TRY(repack(net, static_cast<hipStream_t>(stream)));
    return COLA_OK;
}

int cola_lc_forward(const cola_lc_net* net, int32_t n_mesh, const float* delta, const float* g[3], float* df[3],
                    int32_t accumulate, int32_t training, void* ws, size_t ws_bytes, void* stream) {
    int s;
    if ((s = lc_check_net(net, false)) != COLA_OK) return s;
    if (!lc_mesh_ok(n_mesh)) return COLA_ERR_UNSUPPORTED_SIZE;
    if (!delta || !ptrs3(g) || !df || !df[0] || !df[1] || !df[2] || !ws) return COLA_ERR_INVALID_ARG;
    const LcWsLayout L = lc_ws_layout(n_mesh, net->channels, 1, training != 0);
    if (ws_bytes < L.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const LcActs A = lc_carve(ws, L);
    const LcParams P = lc_params_of(net);
    ws_forget(ws);
    (void)hipGetLastError();
    LC_TRY(lc_pack(delta, g, n_mesh, n_mesh, net->in_scale, A.x0, st));
    LC_TRY(lc_forward(P, A, n_mesh, net->out_scale, net->out_band, df, n_mesh, accumulate ? 1 : 0, training != 0,
                      st));
    return COLA_OK;
}

int cola_lc_backward(const cola_lc_net* net, int32_t n_mesh, const float* d_df, void* ws, size_t ws_bytes,
                     void* stream) {
    int s;
    if ((s = lc_check_net(net, false)) != COLA_OK) return s;
    if (!net->grads) return COLA_ERR_INVALID_ARG;
    if (!lc_mesh_ok(n_mesh)) return COLA_ERR_UNSUPPORTED_SIZE;
    if (!d_df || !ws) return COLA_ERR_INVALID_ARG;
    const LcWsLayout L = lc_ws_layout(n_mesh, net->channels, 1, true);
    if (ws_bytes < L.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const LcActs A = lc_carve(ws, L);
    const LcParams P = lc_params_of(net);
    const LcOffsets o = lc_offsets(net->channels);
    LcGrads G{net->grads + o.w1, net->grads + o.b1, net->grads + o.w2,
              net->grads + o.b2, net->grads + o.w3, net->grads + o.b3};
    (void)hipGetLastError();
    LC_TRY(lc_backward(P, A, G, n_mesh, net->out_scale, net->out_band, d_df, st));
    return COLA_OK;
}

int cola_lc_loss(int32_t n_mesh, double box, const float* pos[3], int64_t n, const float* df[3], const float* g1[3],
                 const float* g3[3], double* stats, float* d_df, void* stream) {
    if (!std::isfinite(box)) return COLA_ERR_NONFINITE;
    if (n_mesh < 2 || n_mesh > kMaxLcMesh || !(box > 0.0) || n < 1) return COLA_ERR_INVALID_ARG;
    if (!ptrs3(pos) || !ptrs3(df) || !ptrs3(g1) || !ptrs3(g3) || !stats || !d_df) return COLA_ERR_INVALID_ARG;
    (void)hipGetLastError();
    LC_TRY(lc_loss(pos, n, n_mesh, box, df, g1, g3, stats, d_df, static_cast<hipStream_t>(stream)));
    return COLA_OK;
}

int cola_lc_adam(const cola_lc_net* net, int32_t t, float lr, float beta1, float beta2, float eps, void* stream) {
    int s;
    if ((s = lc_check_net(net, true)) != COLA_OK) return s;
    if (t < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return COLA_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    LC_TRY(lc_adam(net->params, net->grads, net->adam_m, net->adam_v, lc_offsets(net->channels).total, lr, beta1,
                   beta2, eps, t, st));
    LC_TRY(repack(net, st));
    return COLA_OK;
}

// Three mesh buffers (S, A, B), the interleaved force mesh F and the twiddle table: the step's
// force passes (pm_force_interleaved) on a caller's positions or density.
struct FieldsWs {
    float2 *S, *A, *B, *tw;
    float* F;
    long frow;
};
static size_t fields_f_bytes(int n) { return (size_t)n * n * force_row3(n) * sizeof(float); }
static FieldsWs carve_fields(void* ws, const Mesh3& g) {
    char* b = static_cast<char*>(ws);
    const size_t mb = lc_align(g.bytes());
    FieldsWs w;
    w.S = reinterpret_cast<float2*>(b);
    w.A = reinterpret_cast<float2*>(b + mb);
    w.B = reinterpret_cast<float2*>(b + 2 * mb);
    w.F = reinterpret_cast<float*>(b + 3 * mb);
    w.tw = reinterpret_cast<float2*>(b + 3 * mb + lc_align(fields_f_bytes(g.n)));
    w.frow = force_row3(g.n);
    return w;
}

size_t cola_pm_fields_workspace_bytes(int32_t n_mesh) {
    if (!fft_size_ok(n_mesh) || n_mesh > kMaxLcMesh) return 0;
    const Mesh3 g = make_mesh(n_mesh);
    return 3 * lc_align(g.bytes()) + lc_align(fields_f_bytes(n_mesh)) + lc_align((size_t)n_mesh * sizeof(float2));
}

int cola_pm_fields(int32_t n_mesh, double box, const float* pos[3], int64_t n, float* delta, float* g[3],
                   float* acc[3], void* ws, size_t ws_bytes, void* stream) {
    if (!fft_size_ok(n_mesh) || n_mesh > kMaxLcMesh) return COLA_ERR_UNSUPPORTED_SIZE;
    if (!std::isfinite(box)) return COLA_ERR_NONFINITE;
    if (!(box > 0.0) || n < 1 || !ptrs3(pos) || !ws) return COLA_ERR_INVALID_ARG;
    if (g && !(g[0] && g[1] && g[2])) return COLA_ERR_INVALID_ARG;
    if (acc && !(acc[0] && acc[1] && acc[2])) return COLA_ERR_INVALID_ARG;
    if (ws_bytes < cola_pm_fields_workspace_bytes(n_mesh)) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Mesh3 gm = make_mesh(n_mesh);
    const FieldsWs w = carve_fields(ws, gm);
    const long row = 2L * gm.nzp;
    float* s_real = reinterpret_cast<float*>(w.S);
    const double cells = (double)n_mesh * n_mesh * n_mesh;
    ws_forget(ws);
    (void)hipGetLastError();
    LC_TRY(launch_twiddles(w.tw, n_mesh, st));
    LC_TRY(launch_fill(s_real, 2L * gm.total_c(), 0.0f, st));
    LC_TRY(cic_deposit_absolute(pos, n, n_mesh, (float)(n_mesh / box), row, s_real, st));
    LC_TRY(density_finish(s_real, row, n_mesh, (float)(cells / (double)n), -1.0f, st));
    if (delta) LC_TRY(mesh_unpad(s_real, row, n_mesh, delta, st));
    LC_TRY(fft_zy_forward(s_real, row, 0, w.A, 0, gm, w.tw, 1, 1.0f, 0.0f, st));
    LC_TRY(pm_force_interleaved(w.A, w.B, w.S, w.F, w.frow, 0, 0, gm, w.tw, (float)(2.0 * M_PI / box), 1, st));
    if (g) LC_TRY(mesh_unpad3(w.F, w.frow, n_mesh, g, st));
    if (acc) LC_TRY(gather_absolute(pos, n, n_mesh, box, w.F, w.frow, acc, st));
    return COLA_OK;
}

int cola_mesh_force(int32_t n_mesh, double box, const float* delta, float* g[3], void* ws, size_t ws_bytes,
                    void* stream) {
    if (!fft_size_ok(n_mesh) || n_mesh > kMaxLcMesh) return COLA_ERR_UNSUPPORTED_SIZE;
    if (!std::isfinite(box)) return COLA_ERR_NONFINITE;
    if (!(box > 0.0) || !delta || !ptrs3(g) || !ws) return COLA_ERR_INVALID_ARG;
    if (ws_bytes < cola_pm_fields_workspace_bytes(n_mesh)) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Mesh3 gm = make_mesh(n_mesh);
    const FieldsWs w = carve_fields(ws, gm);
    ws_forget(ws);
    (void)hipGetLastError();
    LC_TRY(launch_twiddles(w.tw, n_mesh, st));
    LC_TRY(fft_zy_forward(delta, n_mesh, 0, w.A, 0, gm, w.tw, 1, 1.0f, 0.0f, st));
    LC_TRY(pm_force_interleaved(w.A, w.B, w.S, w.F, w.frow, 0, 0, gm, w.tw, (float)(2.0 * M_PI / box), 1, st));
    LC_TRY(mesh_unpad3(w.F, w.frow, n_mesh, g, st));
    return COLA_OK;
}

int cola_positions(const cola_problem* prob, const cola_particles* in, float* pos[3], void* stream) {
    if (!prob || !in || !pos || !pos[0] || !pos[1] || !pos[2]) return COLA_ERR_INVALID_ARG;
    if (!(prob->box > 0.0) || prob->n_part < 2 || prob->pm_factor < 1 || prob->n_real < 1) return COLA_ERR_INVALID_ARG;
    for (int d = 0; d < 3; ++d)
        if (!in->x[d]) return COLA_ERR_INVALID_ARG;
    const long npr = (long)prob->n_part * prob->n_part * prob->n_part;
    const double qoff = 0.5 * prob->box / ((double)prob->n_part * prob->pm_factor);
    const float* x[3] = {in->x[0], in->x[1], in->x[2]};
    (void)hipGetLastError();
    LC_TRY(lc_positions(x, npr, prob->n_real, prob->n_part, prob->box, qoff, pos, static_cast<hipStream_t>(stream)));
    return COLA_OK;
}

int cola_mfma_selftest(const uint16_t* a, const uint16_t* b, float* d, void* stream) {
    if (!a || !b || !d) return COLA_ERR_INVALID_ARG;
    (void)hipGetLastError();
    LC_TRY(lc_mfma_selftest(a, b, d, static_cast<hipStream_t>(stream)));
    return COLA_OK;
}

}  // extern "C"
