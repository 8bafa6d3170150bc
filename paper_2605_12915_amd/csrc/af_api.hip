// C ABI of the Active Flux library (declared in include/af.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <new>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "af.h"
#include "af_batch.h"
#include "af_internal.h"

namespace af {

// Zero fill by a kernel rather than hipMemsetAsync, so that a caller may capture the
// enclosing call into a hipGraph (memset nodes are avoided in captured work).
__global__ void k_zero(unsigned long long* p, size_t n) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = 0ull;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 8;   // every buffer zeroed here is a whole number of 8-byte words
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s,
                       (unsigned long long*)p, n);
    return hipGetLastError();
}

}  // namespace af

namespace {

thread_local int g_last_hip = 0;

constexpr int kDiagPartials = 4096;   // blocks of the first reduction pass

}  // namespace

struct af_ctx {
    af_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    size_t N = 0;
    size_t elem = 0;               // bytes per state element
    void* state2 = nullptr;        // second state for ping-ponging (16 planes)
    void* state3 = nullptr;        // third state, only for af_time_steps
    void* scratch = nullptr;       // path scratch
    unsigned* status = nullptr;    // device status bits
    double* partials = nullptr;    // diagnostics partials
    double* diag_out = nullptr;    // af::kDiagVals doubles on the device
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // [0], [1] owned; [2], [3] per-launch timing slots
    bool f32 = false;              // AF_F32 context: float perturbation planes about cfg.bg
    void* comp = nullptr;          // AF_F32: 4 float compensation planes of the average update
    const void* traj_out = nullptr;  // AF_F32: buffer holding the output the compensation belongs to
    void* comp_t = nullptr;        // AF_F32: af_time_steps' own compensation planes
    void* snap = nullptr;          // AF_CHECK: the input state (and compensation) kept for a rollback
    void* adj_scratch = nullptr;   // AF_F64: forward intermediates and reverse accumulators of af_step_adjoint
    int variant = 0;               // 0: fused LDS-tiled kernel, 1: multi-kernel path, 2: two-launch split
    // ---- batching form (af_init_batch) ----
    int nbatch = 0;                          // 0 for a single-grid context
    std::vector<af_config> bcfg;
    std::vector<af::BatchInst> binst;        // host copy of the descriptors
    std::vector<af::BatchInst> bup;          // descriptors as last uploaded
    int force_cfg = -1;                      // AF_BATCH_TILE: fixed tile configuration, no tuning
    std::string tune_cache;                  // AF_BATCH_TUNE_CACHE: file of earlier tuning results
    std::string tune_key;                    // this batch's line key in that file
    bool tuned_from_cache = false;
    std::string kname;                       // af_dominant_kernel's text for batch contexts
    af::BatchInst* d_binst = nullptr;
    std::vector<void*> bbufs;                // per-instance partner states and compensation planes
    std::vector<const void*> btraj;          // per-instance state of the current trajectory
    std::vector<void*> bsnap;                // AF_CHECK: per-instance copy of the input and compensation
    int2* d_work = nullptr;
    int nwork = 0, tune_cfg = -1, grid = 0;
    double tune_ms[af::kNumBatchCfgs] = {};
    hipStream_t cap = nullptr;               // internal stream for graph capture and replay
    hipEvent_t bev[2] = {nullptr, nullptr};
    std::map<int, hipGraphExec_t> graphs;    // nsteps -> instantiated graph
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

// true if the two states have a plane pointer in common (an output that must not alias)
bool share_plane(const af_state* a, const af_state* b) {
    void *pa[16], *pb[16];
    planes_of(a, pa);
    planes_of(b, pb);
    for (int k = 0; k < 16; ++k)
        for (int q = 0; q < 16; ++q)
            if (pa[k] == pb[q]) return true;
    return false;
}

af_status status_from_bits(unsigned b) {
    if (b & af::SB_NONPHYS) return AF_ERR_NONPHYSICAL;
    if (b & af::SB_CFL) return AF_ERR_ACOUSTIC_CFL;
    if (b & af::SB_FOOT) return AF_ERR_FOOT;
    if (b & af::SB_FOOTPRINT) return AF_ERR_FOOTPRINT;
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
    if (c->variant == 3) return af::launch_step_fc_f64(a);
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

// AF_F32: the Kahan compensation belongs to one trajectory.  A call continues it only
// when its input is the buffer that holds the previous call's output; any other input
// (including the previous input again) starts a new trajectory with zeroed compensation.
hipError_t follow_trajectory(af_ctx* c, const void* in, const void* out) {
    if (!c->f32) return hipSuccess;
    const bool same = in == c->traj_out;
    c->traj_out = out;
    if (same) return hipSuccess;
    return af::launch_zero(c->comp, 4 * c->N * sizeof(float), c->stream);
}

// AF_CHECK rollback buffer: 16 state planes plus, for AF_F32, the 4 compensation planes.
hipError_t ensure_snap(af_ctx* c) {
    if (c->snap) return hipSuccess;
    return hipMalloc(&c->snap, 16 * c->N * c->elem + (c->f32 ? 4 * c->N * sizeof(float) : 0));
}

void* snap_comp(af_ctx* c) { return (char*)c->snap + 16 * c->N * c->elem; }

af_status read_status(af_ctx* c, unsigned* bits) {
    unsigned h = 0;
    AF_HIP(hipMemcpyAsync(&h, c->status, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
    AF_HIP(hipStreamSynchronize(c->stream));
    if (h) AF_HIP(hipMemsetAsync(c->status, 0, sizeof(unsigned), c->stream));
    *bits = h;
    return AF_OK;
}


// ---------------------------------------------------------------------------
// Batching form
// ---------------------------------------------------------------------------
// Point-update scheme of a batch (all its grids share it; af_init_batch checks).
static int batch_scheme(const af_ctx* c) { return (c->cfg.flags & AF_SCHEME_RB) ? 1 : 0; }

// Work list of (instance, tile) for tile configuration `cfg`.
hipError_t batch_build_work(af_ctx* c, int cfg) {
    const af::BatchTileCfg t = af::kBatchCfgs[cfg];
    std::vector<int2> w;
    for (int q = 0; q < c->nbatch; ++q) {
        af::BatchInst& d = c->binst[q];
        d.tiles_x = (d.nx + t.tx - 1) / t.tx;
        d.ntiles = d.tiles_x * ((d.ny + t.ty - 1) / t.ty);
        for (int k = 0; k < d.ntiles; ++k) w.push_back(make_int2(q, k));
    }
    if (c->d_work) { hipError_t e = hipFree(c->d_work); if (e != hipSuccess) return e; c->d_work = nullptr; }
    hipError_t e = hipMalloc((void**)&c->d_work, w.size() * sizeof(int2));
    if (e == hipSuccess) e = hipMemcpy(c->d_work, w.data(), w.size() * sizeof(int2), hipMemcpyHostToDevice);
    c->nwork = (int)w.size();
    int per_cu = 1;
    if (e == hipSuccess) e = af::batch_occupancy(cfg, batch_scheme(c), &per_cu);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, c->device);
    c->grid = t.direct ? c->nwork : (per_cu > 0 ? per_cu : 1) * prop.multiProcessorCount;
    return e;
}

// Upload the descriptors when they changed (new state pointers, dt, tile shape).
// Synchronous: the host vector may change again on the next call.
hipError_t batch_upload(af_ctx* c, hipStream_t s) {
    const size_t bytes = c->nbatch * sizeof(af::BatchInst);
    if (c->bup.size() == c->binst.size() && std::memcmp(c->bup.data(), c->binst.data(), bytes) == 0)
        return hipSuccess;
    hipError_t e = hipMemcpyAsync(c->d_binst, c->binst.data(), bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) c->bup = c->binst;
    return e;
}

// Autotuner: time every tile configuration on the batch itself (a copy of the
// caller's states stepped between two library-owned buffers), keep the fastest.
hipError_t batch_tune(af_ctx* c) {
    std::vector<af::BatchInst> saved = c->binst;
    std::vector<void*> tmp;
    hipError_t e = hipSuccess;
    for (int q = 0; q < c->nbatch && e == hipSuccess; ++q) {
        af::BatchInst& d = c->binst[q];
        const size_t N = (size_t)d.nx * d.ny;
        void *t1 = nullptr, *t2 = nullptr;
        e = hipMalloc(&t1, 16 * N * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&t2, 4 * N * sizeof(float));
        if (e == hipSuccess) e = hipMemsetAsync(t2, 0, 4 * N * sizeof(float), c->stream);
        tmp.push_back(t1);
        tmp.push_back(t2);
        for (int k = 0; k < 16 && e == hipSuccess; ++k)
            e = hipMemcpyAsync(d.S[1][k], saved[q].S[0][k], N * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
        for (int k = 0; k < 16; ++k) {
            d.S[0][k] = d.S[1][k];
            d.S[1][k] = (float*)t1 + (size_t)k * N;
        }
        d.comp = (float*)t2;
    }
    int best = 0;
    for (int cfg = 0; cfg < af::kNumBatchCfgs && e == hipSuccess; ++cfg) {
        e = batch_build_work(c, cfg);
        if (e == hipSuccess) e = batch_upload(c, c->stream);
        const int warm = 2, reps = 4;
        for (int r = 0; r < warm && e == hipSuccess; ++r)
            e = af::launch_batch(cfg, batch_scheme(c), c->d_binst, c->d_work, c->nwork, r & 1, c->status, c->grid,
                                 c->stream);
        if (e == hipSuccess) e = hipEventRecord(c->ev[0], c->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            e = af::launch_batch(cfg, batch_scheme(c), c->d_binst, c->d_work, c->nwork, r & 1, c->status, c->grid,
                                 c->stream);
        if (e == hipSuccess) e = hipEventRecord(c->ev[1], c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(c->ev[1]);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
        c->tune_ms[cfg] = ms / reps;
        if (c->tune_ms[cfg] < c->tune_ms[best]) best = cfg;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    for (void* p : tmp)
        if (p) (void)hipFree(p);
    c->binst = saved;
    if (e == hipSuccess) {
        c->tune_cfg = best;
        e = batch_build_work(c, best);
    }
    // the tuning runs leave status bits of scratch data: clear them
    if (e == hipSuccess) e = hipMemsetAsync(c->status, 0, sizeof(unsigned), c->stream);
    return e;
}

// Tuning cache.  One line per tuned batch: its key, the chosen candidate and the
// per-step times of all candidates.  The key identifies the device (architecture and
// compute units), the candidate table, the point update and the grid sizes in order:
// any change there tunes afresh.  A missing, unreadable or malformed file is ignored
// (the batch is tuned and the line appended); lines with another key are skipped.
uint64_t fnv1a(uint64_t h, uint64_t v) {
    for (int b = 0; b < 8; ++b) {
        h ^= (v >> (8 * b)) & 0xff;
        h *= 0x100000001b3ull;
    }
    return h;
}

std::string batch_tune_key(const af_ctx* c) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    for (char& ch : arch)
        if (ch == ' ') ch = '_';
    uint64_t h = 0xcbf29ce484222325ull;
    for (int k = 0; k < af::kNumBatchCfgs; ++k) {
        const af::BatchTileCfg t = af::kBatchCfgs[k];
        h = fnv1a(h, ((uint64_t)t.tx << 48) ^ ((uint64_t)t.ty << 32) ^ ((uint64_t)t.nt << 8) ^ (t.direct ? 4u : 0u) ^
                         (uint64_t)t.minw ^ ((uint64_t)t.rw << 16));
    }
    for (const af::BatchInst& d : c->binst) h = fnv1a(h, ((uint64_t)(uint32_t)d.nx << 32) | (uint32_t)d.ny);
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%s/%d/s%d/n%d/%016llx", arch.c_str(), cus, batch_scheme(c), c->nbatch,
                  (unsigned long long)h);
    return buf;
}

bool batch_tune_lookup(af_ctx* c) {
    std::FILE* f = std::fopen(c->tune_cache.c_str(), "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char key[200];
        int cfg = -1, used = 0;
        if (std::sscanf(line, "%199s %d%n", key, &cfg, &used) != 2 || c->tune_key != key) continue;
        if (cfg < 0 || cfg >= af::kNumBatchCfgs) continue;
        double ms[af::kNumBatchCfgs];
        const char* q = line + used;
        int k = 0;
        for (; k < af::kNumBatchCfgs; ++k) {
            int m = 0;
            if (std::sscanf(q, "%lf%n", &ms[k], &m) != 1) break;
            q += m;
        }
        if (k != af::kNumBatchCfgs) continue;
        c->tune_cfg = cfg;              // the last matching line wins
        for (k = 0; k < af::kNumBatchCfgs; ++k) c->tune_ms[k] = ms[k];
        found = true;
    }
    std::fclose(f);
    return found;
}

void batch_tune_store(const af_ctx* c) {
    std::FILE* f = std::fopen(c->tune_cache.c_str(), "a");
    if (!f) return;
    std::string line = c->tune_key + " " + std::to_string(c->tune_cfg);
    for (int k = 0; k < af::kNumBatchCfgs; ++k) {
        char t[40];
        std::snprintf(t, sizeof(t), " %.6f", c->tune_ms[k]);
        line += t;
    }
    line += "\n";
    std::fputs(line.c_str(), f);
    std::fclose(f);
}

// Instantiated graphs are kept per nsteps; past kMaxGraphs distinct values the cache
// is emptied (a caller cycling through many step counts should not grow it forever).
constexpr size_t kMaxGraphs = 16;

hipError_t batch_graph(af_ctx* c, int nsteps, hipGraphExec_t* out) {
    auto it = c->graphs.find(nsteps);
    if (it != c->graphs.end()) { *out = it->second; return hipSuccess; }
    if (c->graphs.size() >= kMaxGraphs) {
        hipError_t e = hipStreamSynchronize(c->cap);   // no replay may still be running
        if (e != hipSuccess) return e;
        for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
        c->graphs.clear();
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    for (int k = 0; k < nsteps && e == hipSuccess; ++k)
        e = af::launch_batch(c->tune_cfg, batch_scheme(c), c->d_binst, c->d_work, c->nwork, k & 1, c->status, c->grid,
                             c->cap);
    if (e == hipSuccess && (nsteps & 1)) e = af::launch_batch_copy(c->d_binst, c->nbatch, c->cap);
    hipError_t e2 = hipStreamEndCapture(c->cap, &g);
    if (e == hipSuccess) e = e2;
    hipGraphExec_t x = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e == hipSuccess) { c->graphs[nsteps] = x; *out = x; }
    return e;
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
        case AF_ERR_SCRATCH: return "grid larger than the static scratch of the allocation-free entry point";
        case AF_ERR_FOOTPRINT: return "foot-centred update: disk about a foot leaves the half-cell footprint";
        default: return "unknown status";
    }
}

int32_t af_last_hip_error(void) { return g_last_hip; }

// Largest grid a context accepts: 2^31 cells (275 GB of FP64 state, more than one GPU
// holds with a second state), which keeps every byte count in size_t and every launch
// within HIP's 2^32 work-items per grid dimension.
constexpr uint64_t kMaxCells = uint64_t(1) << 31;

af_status af_init(const af_config* cfg, void* hip_stream, af_ctx** out) {
    if (!cfg || !out) return AF_ERR_ARG;
    *out = nullptr;
    if (cfg->nx < 4 || cfg->ny < 4 || !(cfg->h > 0.0) || !(cfg->gamma > 1.0) || !std::isfinite(cfg->h) ||
        !std::isfinite(cfg->gamma))
        return AF_ERR_ARG;
    if ((uint64_t)cfg->nx * (uint64_t)cfg->ny > kMaxCells) return AF_ERR_ARG;
    if (cfg->precision != AF_F64 && cfg->precision != AF_F32) return AF_ERR_ARG;
    if (cfg->precision == AF_F32 && (!(cfg->bg[0] > 0.0) || !(cfg->bg[3] > 0.0))) return AF_ERR_ARG;
    if ((cfg->flags & AF_SCHEME_FC) && (cfg->flags & AF_SCHEME_RB)) return AF_ERR_ARG;
    if ((cfg->flags & AF_SCHEME_FC) && cfg->precision != AF_F64) return AF_ERR_UNSUPPORTED;
    af_ctx* c = new (std::nothrow) af_ctx();
    if (!c) return AF_ERR_ARG;
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
    if (c->f32) c->variant = 0;   // the FP32 form has the fused kernel only
    if (cfg->flags & AF_SCHEME_FC) c->variant = 3;   // the foot-centred update: multi-kernel path
    size_t sbytes = 16;
    if (c->variant == 1) sbytes = af::scratch_bytes_multi_f64(cfg->nx, cfg->ny);
    if (c->variant == 3) sbytes = af::scratch_bytes_fc_f64(cfg->nx, cfg->ny);
    if (c->variant == 2) sbytes = af::scratch_bytes_split_f64(cfg->nx, cfg->ny);
    if (e == hipSuccess && c->f32) e = af::prepare_fused_f32();
    if (e == hipSuccess && c->f32) e = hipMalloc(&c->comp, 4 * c->N * sizeof(float));
    if (e == hipSuccess && c->f32) e = af::launch_zero(c->comp, 4 * c->N * sizeof(float), c->stream);
    if (e == hipSuccess && !c->f32 && c->variant == 0) e = af::prepare_fused_f64();
    if (e == hipSuccess && !c->f32) e = af::prepare_adjoint_f64();
    if (e == hipSuccess && c->variant == 2) e = af::prepare_split_f64();
    if (e == hipSuccess) e = hipMalloc(&c->state2, 16 * c->N * c->elem);
    if (e == hipSuccess) e = hipMalloc(&c->scratch, sbytes);
    if (e == hipSuccess) e = hipMalloc((void**)&c->status, sizeof(unsigned));
    if (e == hipSuccess) e = hipMalloc((void**)&c->partials, kDiagPartials * af::kDiagVals * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&c->diag_out, af::kDiagVals * sizeof(double));
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
    if (c->cap) (void)hipStreamSynchronize(c->cap);
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
    if (c->comp_t) (void)hipFree(c->comp_t);
    if (c->snap) (void)hipFree(c->snap);
    for (void* p : c->bsnap) (void)hipFree(p);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    for (void* p : c->bbufs) (void)hipFree(p);
    if (c->d_binst) (void)hipFree(c->d_binst);
    if (c->d_work) (void)hipFree(c->d_work);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    for (int k = 0; k < 2; ++k)
        if (c->bev[k]) (void)hipEventDestroy(c->bev[k]);
    for (int k = 0; k < 2; ++k)
        if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    delete c;
}

af_status af_step_out(af_ctx* c, const af_state* in, af_state* out, double dt) {
    if (!c || !state_ok(in) || !state_ok(out) || !(dt > 0.0) || !std::isfinite(dt)) return AF_ERR_ARG;
    if (share_plane(in, out)) return AF_ERR_ARG;
    if (c->nbatch) return AF_ERR_UNSUPPORTED;
    void *pi[16], *po[16];
    planes_of(in, pi);
    planes_of(out, po);
    const bool check = (c->cfg.flags & AF_CHECK) != 0;
    AF_HIP(follow_trajectory(c, pi[0], po[0]));
    // AF_CHECK on an AF_F32 context: keep the compensation for a rollback
    if (check && c->f32) {
        AF_HIP(ensure_snap(c));
        AF_HIP(hipMemcpyAsync(snap_comp(c), c->comp, 4 * c->N * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    }
    AF_HIP(launch_step(c, pi, po, dt, false));
    if (check) {
        unsigned bits;
        af_status s = read_status(c, &bits);
        if (s != AF_OK) return s;
        if (bits && c->f32) {
            AF_HIP(hipMemcpyAsync(c->comp, snap_comp(c), 4 * c->N * sizeof(float), hipMemcpyDeviceToDevice,
                                  c->stream));
            AF_HIP(hipStreamSynchronize(c->stream));
        }
        return status_from_bits(bits);
    }
    return AF_OK;
}

af_status af_step(af_ctx* c, af_state* inout, double dt, int32_t nsteps) {
    if (!c || !state_ok(inout) || !(dt > 0.0) || !std::isfinite(dt) || nsteps < 1) return AF_ERR_ARG;
    if (c->nbatch) return AF_ERR_UNSUPPORTED;
    void *a[16], *b[16];
    planes_of(inout, a);
    planes_of_buffer(c->state2, c->N, c->elem, b);
    // the result ends in *inout: it is the buffer that continues the trajectory
    AF_HIP(follow_trajectory(c, a[0], a[0]));
    const bool check = (c->cfg.flags & AF_CHECK) != 0;
    void* snap[16] = {};
    if (check) {
        // rollback copy: the input (overwritten from step 1 on) and the compensation
        AF_HIP(ensure_snap(c));
        planes_of_buffer(c->snap, c->N, c->elem, snap);
        if (nsteps > 1) AF_HIP(copy_state(c, snap, a));
        if (c->f32)
            AF_HIP(hipMemcpyAsync(snap_comp(c), c->comp, 4 * c->N * sizeof(float), hipMemcpyDeviceToDevice,
                                  c->stream));
    }
    for (int s = 0; s < nsteps; ++s) {
        void** src = (s & 1) ? b : a;
        void** dst = (s & 1) ? a : b;
        AF_HIP(launch_step(c, src, dst, dt, false));
        if (check) {
            unsigned bits;
            af_status st = read_status(c, &bits);
            if (st != AF_OK) return st;
            if (bits) {
                // *inout returns to the input of the call (step 0 writes the partner
                // buffer only, so it is untouched when step 0 fails)
                if (s > 0) AF_HIP(copy_state(c, a, snap));
                if (c->f32)
                    AF_HIP(hipMemcpyAsync(c->comp, snap_comp(c), 4 * c->N * sizeof(float), hipMemcpyDeviceToDevice,
                                          c->stream));
                AF_HIP(hipStreamSynchronize(c->stream));
                return status_from_bits(bits);
            }
        }
    }
    if (nsteps & 1) AF_HIP(copy_state(c, a, b));
    return AF_OK;
}

af_status af_reset_trajectory(af_ctx* c) {
    if (!c) return AF_ERR_ARG;
    c->traj_out = nullptr;
    if (c->nbatch)
        for (auto& t : c->btraj) t = nullptr;
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
    if (!c || !state_ok(primal_n) || !state_ok(cot_np1) || !state_ok(cot_n) || !(dt > 0.0) || !std::isfinite(dt))
        return AF_ERR_ARG;
    if (share_plane(cot_n, cot_np1) || share_plane(cot_n, primal_n)) return AF_ERR_ARG;
    if (c->f32 || c->nbatch || c->variant == 3) return AF_ERR_UNSUPPORTED;
    if (!c->adj_scratch) AF_HIP(hipMalloc(&c->adj_scratch, af::scratch_bytes_adjoint_f64(c->cfg.nx, c->cfg.ny)));
    af::StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nx = c->cfg.nx;
    a.ny = c->cfg.ny;
    a.h = c->cfg.h;
    a.gamma = c->cfg.gamma;
    a.dt = dt;
    a.scheme = (c->cfg.flags & AF_SCHEME_RB) ? 1 : 0;
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

af_status af_step_adjoint_noalloc(const af_config* cfg, void* hip_stream, const af_state* primal_n,
                                  const af_state* cot_np1, af_state* cot_n, double dt) {
    if (!cfg || !state_ok(primal_n) || !state_ok(cot_np1) || !state_ok(cot_n) || !(dt > 0.0) || !std::isfinite(dt))
        return AF_ERR_ARG;
    if (cfg->nx < 4 || cfg->ny < 4 || !(cfg->h > 0.0) || !(cfg->gamma > 1.0) || !std::isfinite(cfg->h) ||
        !std::isfinite(cfg->gamma))
        return AF_ERR_ARG;
    if (share_plane(cot_n, cot_np1) || share_plane(cot_n, primal_n)) return AF_ERR_ARG;
    if (cfg->precision != AF_F64 || (cfg->flags & AF_SCHEME_FC)) return AF_ERR_UNSUPPORTED;
    if ((uint64_t)cfg->nx * (uint64_t)cfg->ny > af::kNoallocMaxCells) return AF_ERR_SCRATCH;
    af::StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nx = cfg->nx;
    a.ny = cfg->ny;
    a.h = cfg->h;
    a.gamma = cfg->gamma;
    a.dt = dt;
    a.scheme = (cfg->flags & AF_SCHEME_RB) ? 1 : 0;
    a.stream = (hipStream_t)hip_stream;
    planes_of(primal_n, a.in);
    void *p1[16], *p0[16];
    planes_of(cot_np1, p1);
    planes_of(cot_n, p0);
    AF_HIP(af::launch_adjoint_noalloc(a, p1, p0));
    if (cfg->flags & AF_CHECK) {
        void* sp = nullptr;
        AF_HIP(af::noalloc_scratch_ptr(&sp));
        unsigned h = 0;
        AF_HIP(hipMemcpyAsync(&h, sp, sizeof(unsigned), hipMemcpyDeviceToHost, a.stream));
        AF_HIP(hipStreamSynchronize(a.stream));
        return status_from_bits(h);
    }
    return AF_OK;
}

af_status af_diagnostics(af_ctx* c, const af_state* s, double dt, af_diag* out) {
    if (!c || !state_ok(s) || !out) return AF_ERR_ARG;
    if (c->nbatch) return AF_ERR_UNSUPPORTED;
    void* p[16];
    planes_of(s, p);
    AF_HIP(af::launch_diag(p, c->f32, c->cfg.bg, c->cfg.nx, c->cfg.ny, c->cfg.h, c->cfg.gamma, c->partials,
                           kDiagPartials, c->diag_out, c->stream));
    double h[af::kDiagVals];
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
    out->vorticity = h[9] * 0.5 * c->cfg.h;
    out->enstrophy = h[10];
    return AF_OK;
}

af_status af_time_steps(af_ctx* c, const af_state* s, double dt, int32_t nsteps, double* total_ms,
                        double* kernel_ms) {
    if (!c || !state_ok(s) || nsteps < 1 || nsteps > 4096 || !total_ms || !kernel_ms || !(dt > 0.0))
        return AF_ERR_ARG;
    if (c->nbatch) return AF_ERR_UNSUPPORTED;
    if (!c->state3) AF_HIP(hipMalloc(&c->state3, 16 * c->N * c->elem));
    if (c->f32 && !c->comp_t) AF_HIP(hipMalloc(&c->comp_t, 4 * c->N * sizeof(float)));
    void *src[16], *a[16], *b[16];
    planes_of(s, src);
    planes_of_buffer(c->state3, c->N, c->elem, a);
    planes_of_buffer(c->state2, c->N, c->elem, b);
    AF_HIP(copy_state(c, a, src));
    // the timed steps use their own compensation planes: the caller's trajectory is
    // left as it was
    void* comp_saved = c->comp;
    if (c->f32) {
        AF_HIP(af::launch_zero(c->comp_t, 4 * c->N * sizeof(float), c->stream));
        c->comp = c->comp_t;
    }
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
    c->comp = comp_saved;
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


af_status af_init_batch(const af_config* cfgs, int32_t n, void* hip_stream, af_ctx** out) {
    if (!cfgs || !out || n < 1 || n > 4096) return AF_ERR_ARG;
    *out = nullptr;
    uint64_t total = 0;
    for (int q = 0; q < n; ++q) {
        const af_config& cf = cfgs[q];
        if (cf.nx < 4 || cf.ny < 4 || !(cf.h > 0.0) || !(cf.gamma > 1.0) || !std::isfinite(cf.h) ||
            !std::isfinite(cf.gamma))
            return AF_ERR_ARG;
        total += (uint64_t)cf.nx * (uint64_t)cf.ny;
        if (total > kMaxCells) return AF_ERR_ARG;
        if (cf.precision != AF_F32 || (cf.flags & AF_SCHEME_FC)) return AF_ERR_UNSUPPORTED;
        if (!(cf.bg[0] > 0.0) || !(cf.bg[3] > 0.0)) return AF_ERR_ARG;
        if ((cf.flags & AF_SCHEME_RB) != (cfgs[0].flags & AF_SCHEME_RB)) return AF_ERR_UNSUPPORTED;   // one scheme per batch
    }
    af_ctx* c = new (std::nothrow) af_ctx();
    if (!c) return AF_ERR_ARG;
    c->cfg = cfgs[0];
    c->stream = (hipStream_t)hip_stream;
    c->f32 = true;
    c->elem = sizeof(float);
    c->nbatch = n;
    c->bcfg.assign(cfgs, cfgs + n);
    c->binst.resize(n);
    c->btraj.assign(n, nullptr);
    if (const char* v = std::getenv("AF_BATCH_TILE")) {
        const int k = std::atoi(v);
        if (k >= 0 && k < af::kNumBatchCfgs) c->force_cfg = k;
    }
    if (const char* v = std::getenv("AF_BATCH_TUNE_CACHE"))
        if (*v) c->tune_cache = v;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&c->bev[k], hipEventDisableTiming);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreate(&c->ev[k]);
    if (e == hipSuccess) e = hipMalloc((void**)&c->status, sizeof(unsigned));
    if (e == hipSuccess) e = hipMemsetAsync(c->status, 0, sizeof(unsigned), c->stream);
    if (e == hipSuccess) e = hipMalloc((void**)&c->d_binst, n * sizeof(af::BatchInst));
    for (int q = 0; q < n && e == hipSuccess; ++q) {
        const af_config& cf = cfgs[q];
        af::BatchInst& d = c->binst[q];
        std::memset(&d, 0, sizeof(d));
        d.nx = cf.nx;
        d.ny = cf.ny;
        d.pol = af::pert_pol_f32(cf.bg, cf.gamma);
        const size_t N = (size_t)cf.nx * cf.ny;
        void *b = nullptr, *cp = nullptr;
        e = hipMalloc(&b, 16 * N * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&cp, 4 * N * sizeof(float));
        if (e == hipSuccess) e = hipMemsetAsync(cp, 0, 4 * N * sizeof(float), c->stream);
        c->bbufs.push_back(b);
        c->bbufs.push_back(cp);
        for (int k = 0; k < 16; ++k) d.S[1][k] = (float*)b + (size_t)k * N;
        d.comp = (float*)cp;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        af_destroy(c);
        return AF_ERR_HIP;
    }
    *out = c;
    return AF_OK;
}

af_status af_step_batch(af_ctx* c, af_state* states, const double* dts, int32_t nsteps) {
    if (!c || !states || !dts || nsteps < 1 || nsteps > 65536) return AF_ERR_ARG;
    if (c->nbatch < 1) return AF_ERR_UNSUPPORTED;
    for (int q = 0; q < c->nbatch; ++q) {
        if (!state_ok(&states[q]) || !(dts[q] > 0.0) || !std::isfinite(dts[q])) return AF_ERR_ARG;
    }
    for (int q = 0; q < c->nbatch; ++q) {
        af::BatchInst& d = c->binst[q];
        void* p[16];
        planes_of(&states[q], p);
        for (int k = 0; k < 16; ++k) d.S[0][k] = (float*)p[k];
        d.lam1 = (float)(dts[q] / c->bcfg[q].h);
        d.lam0 = (float)(0.5 * dts[q] / c->bcfg[q].h);
        if (c->btraj[q] != p[0]) {   // a new trajectory: fresh compensation
            AF_HIP(af::launch_zero(d.comp, 4 * (size_t)d.nx * d.ny * sizeof(float), c->stream));
            c->btraj[q] = p[0];
        }
    }
    if (c->tune_cfg < 0) {
        if (c->force_cfg >= 0) {
            AF_HIP(batch_build_work(c, c->force_cfg));
            c->tune_cfg = c->force_cfg;
        } else {
            if (!c->tune_cache.empty()) {
                c->tune_key = batch_tune_key(c);
                c->tuned_from_cache = batch_tune_lookup(c);
            }
            if (c->tuned_from_cache) {
                AF_HIP(batch_build_work(c, c->tune_cfg));
            } else {
                AF_HIP(batch_tune(c));
                if (!c->tune_cache.empty()) batch_tune_store(c);
            }
        }
    }
    AF_HIP(batch_upload(c, c->stream));
    hipGraphExec_t gx = nullptr;
    AF_HIP(batch_graph(c, nsteps, &gx));
    const bool check = (c->cfg.flags & AF_CHECK) != 0;
    // AF_CHECK: copy every grid's input and compensation for a rollback
    auto snap_copy = [&](bool restore) -> hipError_t {
        for (int q = 0; q < c->nbatch; ++q) {
            const af::BatchInst& d = c->binst[q];
            const size_t N = (size_t)d.nx * d.ny;
            float* sp = (float*)c->bsnap[q];
            for (int k = 0; k < 16; ++k) {
                void* dst = restore ? (void*)d.S[0][k] : (void*)(sp + k * N);
                const void* src = restore ? (const void*)(sp + k * N) : (const void*)d.S[0][k];
                hipError_t e = hipMemcpyAsync(dst, src, N * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
                if (e != hipSuccess) return e;
            }
            void* dst = restore ? (void*)d.comp : (void*)(sp + 16 * N);
            const void* src = restore ? (const void*)(sp + 16 * N) : (const void*)d.comp;
            hipError_t e = hipMemcpyAsync(dst, src, 4 * N * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    if (check) {
        if (c->bsnap.empty()) {
            for (int q = 0; q < c->nbatch; ++q) {
                void* p = nullptr;
                const size_t N = (size_t)c->binst[q].nx * c->binst[q].ny;
                hipError_t e = hipMalloc(&p, 20 * N * sizeof(float));
                if (e != hipSuccess) {
                    for (void* x : c->bsnap) (void)hipFree(x);
                    c->bsnap.clear();
                    g_last_hip = (int)e;
                    return AF_ERR_HIP;
                }
                c->bsnap.push_back(p);
            }
        }
        AF_HIP(snap_copy(false));
    }
    // order the replay after the caller's stream and make the caller's stream wait for it
    AF_HIP(hipEventRecord(c->bev[0], c->stream));
    AF_HIP(hipStreamWaitEvent(c->cap, c->bev[0], 0));
    AF_HIP(hipGraphLaunch(gx, c->cap));
    AF_HIP(hipEventRecord(c->bev[1], c->cap));
    AF_HIP(hipStreamWaitEvent(c->stream, c->bev[1], 0));
    if (check) {
        unsigned bits;
        af_status st = read_status(c, &bits);
        if (st != AF_OK) return st;
        if (bits) {
            // every grid returns to the input of the call
            AF_HIP(snap_copy(true));
            AF_HIP(hipStreamSynchronize(c->stream));
        }
        return status_from_bits(bits);
    }
    return AF_OK;
}

int32_t af_batch_info(af_ctx* c, char* buf, int32_t buflen) {
    if (!c || c->nbatch < 1 || !buf || buflen < 1) return -1;
    std::string s = "{\"instances\": " + std::to_string(c->nbatch) + ", \"work_items\": " + std::to_string(c->nwork) +
                    ", \"grid\": " + std::to_string(c->grid) + ", \"chosen\": ";
    if (c->tune_cfg >= 0) {
        const af::BatchTileCfg t = af::kBatchCfgs[c->tune_cfg];
        s += "[" + std::to_string(t.tx) + ", " + std::to_string(t.ty) + ", " + std::to_string(t.nt) + "]";
        s += std::string(", \"mode\": \"") + (t.direct ? "direct" : "persistent") + "\", \"min_waves\": " +
             std::to_string(t.minw) + ", \"target_rows\": " + std::to_string(t.rw);
    } else {
        s += "null";
    }
    s += std::string(", \"tuned_from_cache\": ") + (c->tuned_from_cache ? "true" : "false");
    s += ", \"candidates\": [";
    for (int k = 0; k < af::kNumBatchCfgs; ++k) {
        const af::BatchTileCfg t = af::kBatchCfgs[k];
        char tmp[200];
        std::snprintf(tmp, sizeof(tmp),
                      "%s{\"tile\": [%d, %d, %d], \"mode\": \"%s\", \"min_waves\": %d, \"target_rows\": %d, "
                      "\"ms_per_step\": %.6f}",
                      k ? ", " : "", t.tx, t.ty, t.nt, t.direct ? "direct" : "persistent", t.minw, t.rw, c->tune_ms[k]);
        s += tmp;
    }
    s += "]}";
    const int32_t n = (int32_t)s.size();
    std::strncpy(buf, s.c_str(), (size_t)buflen);
    buf[buflen - 1] = '\0';
    return n;
}

const char* af_dominant_kernel(af_ctx* c) {
    if (c && c->nbatch) {
        if (c->tune_cfg < 0) return "af::k_fused_batch (tile not chosen yet)";
        const af::BatchTileCfg t = af::kBatchCfgs[c->tune_cfg];
        c->kname = std::string(t.direct ? "af::k_fused_batch_direct<" : "af::k_fused_batch<") + std::to_string(t.tx) +
                   ", " + std::to_string(t.ty) + ", " + std::to_string(t.nt) +
                   (t.direct ? ", " + std::to_string(t.minw) : std::string()) + ", " +
                   std::to_string(batch_scheme(c)) + (t.direct ? ", " + std::to_string(t.rw) : std::string()) + ">";
        return c->kname.c_str();
    }
    const bool rb = c && (c->cfg.flags & AF_SCHEME_RB);
    if (c && c->f32)
        return rb ? "af::k_fused<float, af::PolPert<float>, 31, 10, 512, 1, true, 4, 32, true>"
                  : "af::k_fused<float, af::PolPert<float>, 31, 10, 512, 0, true, 4, 32, true>";
    if (c && c->variant == 3) return "af::k_fc_points";
    if (c && c->variant == 1) return "af_step multi-kernel sequence";
    if (c && c->variant == 2) return rb ? "af::k_points_update<32, 8, 512, 1>" : "af::k_points_update<32, 8, 512, 0>";
    return rb ? "af::k_fused<double, af::PolAbs<double>, 31, 10, 512, 1, false, 1, 32, true>"
              : "af::k_fused<double, af::PolAbs<double>, 31, 10, 512, 0, false, 1, 32, true>";
}

}  // extern "C"
