// C ABI of the Active Flux library (declared in include/af.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "af.h"
#include "af_internal.h"

namespace {

thread_local int g_last_hip = 0;

constexpr int kDiagPartials = 1024;

}  // namespace

struct af_ctx {
    af_config cfg;
    hipStream_t stream;
    int device;
    size_t N;
    size_t elem;           // bytes per state element
    void* state2;          // second state for ping-ponging (16 planes)
    void* state3;          // third state, only for af_time_steps
    void* scratch;         // path scratch
    unsigned* status;      // device status bits
    double* partials;      // diagnostics partials
    double* diag_out;      // 9 doubles on the device
    hipEvent_t ev[4];      // [0], [1]: owned; [2], [3]: slots for per-launch timing events
    bool f32;              // AF_F32 context: float perturbation planes about cfg.bg
    void* comp;            // AF_F32: 4 float compensation planes of the average update
    const void* traj[2];   // AF_F32: the buffers of the trajectory the compensation belongs to
    void* adj_scratch;     // AF_F64: forward intermediates and reverse accumulators of af_step_adjoint
    int variant;           // 0: fused LDS-tiled kernel, 1: multi-kernel path, 2: two-launch split
};

#define AF_HIP(x)                                       \
    do {                                                \
        hipError_t e_ = (x);                            \
        if (e_ != hipSuccess) {                         \
            g_last_hip = (int)e_;                       \
            return AF_ERR_HIP;                          \
        }                                               \
    } while (0)

namespace {

void planes_of(const af_state* s, void* out[16]) {
    for (int k = 0; k < 4; ++k) {
        out[k] = s->avg[k];
        out[4 + k] = s->V[k];
        out[8 + k] = s->EV[k];
        out[12 + k] = s->EH[k];
    }
}

void planes_of_buffer(void* base, size_t N, size_t elem, void* out[16]) {
    for (int k = 0; k < 16; ++k) out[k] = (char*)base + (size_t)k * N * elem;
}

bool state_ok(const af_state* s) {
    if (!s) return false;
    void* p[16];
    planes_of(s, p);
    for (int k = 0; k < 16; ++k)
        if (!p[k]) return false;
    return true;
}

af_status status_from_bits(unsigned b) {
    if (b & af::SB_NONPHYS) return AF_ERR_NONPHYSICAL;
    if (b & af::SB_CFL) return AF_ERR_ACOUSTIC_CFL;
    if (b & af::SB_FOOT) return AF_ERR_FOOT;
    return AF_OK;
}

hipError_t launch_step(af_ctx* c, void* const in[16], void* const out[16], double dt, bool timed) {
    af::StepArgs a;
    a.nx = c->cfg.nx;
    a.ny = c->cfg.ny;
    a.h = c->cfg.h;
    a.gamma = c->cfg.gamma;
    a.dt = dt;
    a.scheme = (c->cfg.flags & AF_SCHEME_RB) ? 1 : 0;
    for (int k = 0; k < 16; ++k) { a.in[k] = in[k]; a.out[k] = out[k]; }
    a.scratch = c->scratch;
    a.status = c->status;
    a.stream = c->stream;
    a.ev_begin = timed ? c->ev[2] : nullptr;
    a.ev_end = timed ? c->ev[3] : nullptr;
    a.variant = c->variant;
    for (int k = 0; k < 4; ++k) a.bg[k] = c->cfg.bg[k];
    a.comp = c->comp;
    if (c->f32) return af::launch_step_fused_f32(a);
    if (c->variant == 1) return af::launch_step_multi_f64(a);
    if (c->variant == 2) return af::launch_step_split_f64(a);
    return af::launch_step_fused_f64(a);
}

hipError_t copy_state(af_ctx* c, void* const dst[16], void* const src[16]) {
    for (int k = 0; k < 16; ++k) {
        hipError_t e = hipMemcpyAsync(dst[k], src[k], c->N * c->elem, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// AF_F32: the Kahan compensation belongs to one trajectory; a state that is neither
// of the two buffers of the previous call starts a new one (compensation zeroed).
hipError_t follow_trajectory(af_ctx* c, const void* a, const void* b) {
    if (!c->f32) return hipSuccess;
    const bool same = (a == c->traj[0] || a == c->traj[1]);
    c->traj[0] = a;
    c->traj[1] = b;
    if (same) return hipSuccess;
    return hipMemsetAsync(c->comp, 0, 4 * c->N * sizeof(float), c->stream);
}

af_status read_status(af_ctx* c, unsigned* bits) {
    unsigned h = 0;
    AF_HIP(hipMemcpyAsync(&h, c->status, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
    AF_HIP(hipStreamSynchronize(c->stream));
    if (h) AF_HIP(hipMemsetAsync(c->status, 0, sizeof(unsigned), c->stream));
    *bits = h;
    return AF_OK;
}

}  // namespace

extern "C" {

const char* af_status_string(af_status s) {
    switch (s) {
        case AF_OK: return "ok";
        case AF_ERR_ARG: return "invalid argument";
        case AF_ERR_HIP: return "HIP runtime error";
        case AF_ERR_ACOUSTIC_CFL: return "acoustic CFL c dt / h exceeds 1/2";
        case AF_ERR_FOOT: return "convective foot moved one cell or more";
        case AF_ERR_NONPHYSICAL: return "non-physical state (rho <= 0, p <= 0 or NaN)";
        case AF_ERR_UNSUPPORTED: return "operation not supported for this precision";
        default: return "unknown status";
    }
}

int32_t af_last_hip_error(void) { return g_last_hip; }

af_status af_init(const af_config* cfg, void* hip_stream, af_ctx** out) {
    if (!cfg || !out) return AF_ERR_ARG;
    *out = nullptr;
    if (cfg->nx < 4 || cfg->ny < 4 || !(cfg->h > 0.0) || !(cfg->gamma > 1.0) || !std::isfinite(cfg->h) ||
        !std::isfinite(cfg->gamma))
        return AF_ERR_ARG;
    if (cfg->precision != AF_F64 && cfg->precision != AF_F32) return AF_ERR_ARG;
    if (cfg->precision == AF_F32 && (!(cfg->bg[0] > 0.0) || !(cfg->bg[3] > 0.0))) return AF_ERR_ARG;
    af_ctx* c = new (std::nothrow) af_ctx();
    if (!c) return AF_ERR_ARG;
    std::memset(c, 0, sizeof(*c));
    c->cfg = *cfg;
    c->stream = (hipStream_t)hip_stream;
    c->N = (size_t)cfg->nx * cfg->ny;
    c->f32 = cfg->precision == AF_F32;
    c->elem = c->f32 ? sizeof(float) : sizeof(double);
    hipError_t e = hipGetDevice(&c->device);
    const char* v = getenv("AF_VARIANT");
    c->variant = 0;
    if (v && std::strcmp(v, "multi") == 0) c->variant = 1;
    if (v && std::strcmp(v, "split") == 0) c->variant = 2;
    size_t sbytes = 16;
    if (c->variant == 1) sbytes = af::scratch_bytes_multi_f64(cfg->nx, cfg->ny);
    if (c->variant == 2) sbytes = af::scratch_bytes_split_f64(cfg->nx, cfg->ny);
    if (c->f32) c->variant = 0;
    if (e == hipSuccess && c->f32) e = af::prepare_fused_f32();
    if (e == hipSuccess && c->f32) e = hipMalloc(&c->comp, 4 * c->N * sizeof(float));
    if (e == hipSuccess && c->f32) e = hipMemsetAsync(c->comp, 0, 4 * c->N * sizeof(float), c->stream);
    if (e == hipSuccess && !c->f32 && c->variant == 0) e = af::prepare_fused_f64();
    if (e == hipSuccess && c->variant == 2) e = af::prepare_split_f64();
    if (e == hipSuccess) e = hipMalloc(&c->state2, 16 * c->N * c->elem);
    if (e == hipSuccess) e = hipMalloc(&c->scratch, sbytes);
    if (e == hipSuccess) e = hipMalloc((void**)&c->status, sizeof(unsigned));
    if (e == hipSuccess) e = hipMalloc((void**)&c->partials, kDiagPartials * 9 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&c->diag_out, 9 * sizeof(double));
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreate(&c->ev[k]);
    if (e == hipSuccess) e = hipMemsetAsync(c->status, 0, sizeof(unsigned), c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        af_destroy(c);
        return AF_ERR_HIP;
    }
    *out = c;
    return AF_OK;
}

void af_destroy(af_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->state2) (void)hipFree(c->state2);
    if (c->state3) (void)hipFree(c->state3);
    if (c->scratch) (void)hipFree(c->scratch);
    if (c->status) (void)hipFree(c->status);
    if (c->partials) (void)hipFree(c->partials);
    if (c->diag_out) (void)hipFree(c->diag_out);
    if (c->comp) (void)hipFree(c->comp);
    if (c->adj_scratch) (void)hipFree(c->adj_scratch);
    for (int k = 0; k < 2; ++k)
        if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    delete c;
}

af_status af_step_out(af_ctx* c, const af_state* in, af_state* out, double dt) {
    if (!c || !state_ok(in) || !state_ok(out) || !(dt > 0.0) || !std::isfinite(dt)) return AF_ERR_ARG;
    void *pi[16], *po[16];
    planes_of(in, pi);
    planes_of(out, po);
    AF_HIP(follow_trajectory(c, pi[0], po[0]));
    AF_HIP(launch_step(c, pi, po, dt, false));
    if (c->cfg.flags & AF_CHECK) {
        unsigned bits;
        af_status s = read_status(c, &bits);
        if (s != AF_OK) return s;
        return status_from_bits(bits);
    }
    return AF_OK;
}

af_status af_step(af_ctx* c, af_state* inout, double dt, int32_t nsteps) {
    if (!c || !state_ok(inout) || !(dt > 0.0) || !std::isfinite(dt) || nsteps < 1) return AF_ERR_ARG;
    void *a[16], *b[16];
    planes_of(inout, a);
    planes_of_buffer(c->state2, c->N, c->elem, b);
    AF_HIP(follow_trajectory(c, a[0], b[0]));
    const bool check = (c->cfg.flags & AF_CHECK) != 0;
    for (int s = 0; s < nsteps; ++s) {
        void** src = (s & 1) ? b : a;
        void** dst = (s & 1) ? a : b;
        AF_HIP(launch_step(c, src, dst, dt, false));
        if (check) {
            unsigned bits;
            af_status st = read_status(c, &bits);
            if (st != AF_OK) return st;
            if (bits) {
                if (s & 1) AF_HIP(copy_state(c, a, b));   // keep the last good state in *inout
                AF_HIP(hipStreamSynchronize(c->stream));
                return status_from_bits(bits);
            }
        }
    }
    if (nsteps & 1) AF_HIP(copy_state(c, a, b));
    return AF_OK;
}

af_status af_read_status(af_ctx* c, af_status* status) {
    if (!c || !status) return AF_ERR_ARG;
    unsigned bits;
    af_status s = read_status(c, &bits);
    if (s != AF_OK) return s;
    *status = status_from_bits(bits);
    return AF_OK;
}

af_status af_step_adjoint(af_ctx* c, const af_state* primal_n, const af_state* cot_np1, af_state* cot_n,
                          double dt) {
    if (!c || !state_ok(primal_n) || !state_ok(cot_np1) || !state_ok(cot_n) || !(dt > 0.0)) return AF_ERR_ARG;
    if (c->f32 || (c->cfg.flags & AF_SCHEME_RB)) return AF_ERR_UNSUPPORTED;
    if (!c->adj_scratch) AF_HIP(hipMalloc(&c->adj_scratch, af::scratch_bytes_adjoint_f64(c->cfg.nx, c->cfg.ny)));
    af::StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nx = c->cfg.nx;
    a.ny = c->cfg.ny;
    a.h = c->cfg.h;
    a.gamma = c->cfg.gamma;
    a.dt = dt;
    planes_of(primal_n, a.in);
    a.scratch = c->adj_scratch;
    a.status = c->status;
    a.stream = c->stream;
    void *p1[16], *p0[16];
    planes_of(cot_np1, p1);
    planes_of(cot_n, p0);
    AF_HIP(af::launch_adjoint_f64(a, p1, p0));
    return AF_OK;
}

af_status af_diagnostics(af_ctx* c, const af_state* s, double dt, af_diag* out) {
    if (!c || !state_ok(s) || !out) return AF_ERR_ARG;
    void* p[16];
    planes_of(s, p);
    AF_HIP(af::launch_diag(p, c->f32, c->cfg.bg, c->cfg.nx, c->cfg.ny, c->cfg.h, c->cfg.gamma, c->partials,
                           kDiagPartials, c->diag_out, c->stream));
    double h[9];
    AF_HIP(hipMemcpyAsync(h, c->diag_out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    AF_HIP(hipStreamSynchronize(c->stream));
    const double A = c->cfg.h * c->cfg.h;
    out->mass = h[0] * A;
    out->momx = h[1] * A;
    out->momy = h[2] * A;
    out->energy = h[3] * A;
    out->entropy = h[4] * A;
    out->min_rho = h[5];
    out->min_p = h[6];
    out->max_speed = h[7];
    out->max_acoustic_r = h[8] * dt / c->cfg.h;
    return AF_OK;
}

af_status af_time_steps(af_ctx* c, const af_state* s, double dt, int32_t nsteps, double* total_ms,
                        double* kernel_ms) {
    if (!c || !state_ok(s) || nsteps < 1 || nsteps > 4096 || !total_ms || !kernel_ms || !(dt > 0.0))
        return AF_ERR_ARG;
    if (!c->state3) AF_HIP(hipMalloc(&c->state3, 16 * c->N * c->elem));
    void *src[16], *a[16], *b[16];
    planes_of(s, src);
    planes_of_buffer(c->state3, c->N, c->elem, a);
    planes_of_buffer(c->state2, c->N, c->elem, b);
    AF_HIP(copy_state(c, a, src));
    // one event pair around every launch of the dominant kernel, on the context stream
    std::vector<hipEvent_t> ev(2 * (size_t)nsteps, nullptr);
    hipError_t e = hipSuccess;
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    if (e == hipSuccess) e = hipEventRecord(c->ev[0], c->stream);
    for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
        void** x = (k & 1) ? b : a;
        void** y = (k & 1) ? a : b;
        c->ev[2] = ev[2 * k];
        c->ev[3] = ev[2 * k + 1];
        e = launch_step(c, x, y, dt, true);
    }
    c->ev[2] = c->ev[3] = nullptr;
    if (e == hipSuccess) e = hipEventRecord(c->ev[1], c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(c->ev[1]);
    float ms = 0.f;
    double ksum = 0.0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
    *total_ms = ms;
    for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
        float km = 0.f;
        e = hipEventElapsedTime(&km, ev[2 * k], ev[2 * k + 1]);
        ksum += km;
    }
    *kernel_ms = ksum / nsteps;
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        return AF_ERR_HIP;
    }
    return AF_OK;
}

const char* af_dominant_kernel(af_ctx* c) {
    if (c && c->f32) return "af::k_fused<float, PolPert<float>, 32, 8, 512, 0, true>";
    if (c && c->variant == 1) return "af_step multi-kernel sequence";
    if (c && c->variant == 2) return "af::k_points_update<32, 8, 512, 0>";
    return "af::k_fused<32, 8, 512, 0>";
}

}  // extern "C"
