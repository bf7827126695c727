// api.cpp -- host side of the C ABI declared in include/moto.h: plans,
// workspace layouts, argument checks, and the host loops of the iterative
// drivers (eigen-solve, descent, saddle search) that queue the device
// kernels and poll the device convergence flags.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "kernels.hpp"
#include "moto.h"

using namespace moto;

struct moto_plan_s {
    moto_hamiltonian h;
    Geo g;
    CoefD k;
    double hest;
    int ns;
    int64_t* pinned;  // host read-back buffer (hipHostMalloc)
    // autotuned frame-layout HVP variants, keyed by (dtype, batch, n_vec)
    struct Tune {
        int dt, batch, nvec, variant;
    } tune[32];
    int n_tune;
    // instantiated HIP graphs of the eigen-solver's iteration chunk, keyed by
    // everything baked into the captured kernel arguments
    struct GraphEntry {
        hipGraphExec_t exec;
        const void* ws;
        const void* mask;
        long long key[8];
        int valid;
    } graphs[4];
    int next_graph;
    // private stream the graphs are captured on (capture is not possible on
    // the legacy default stream a caller may pass); replays use the caller's
    hipStream_t cap_stream;
    long long graph_replays;  // replays of captured iteration chunks (diagnostic)
    // shell table of a Hamiltonian with more than three shells (k.gen points here)
    GenShells gen;
};

namespace {

constexpr size_t kAlign = 256;
inline size_t al(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

#define HIP_TRY(expr)                               \
    do {                                            \
        if ((expr) != hipSuccess) return MOTO_EHIP; \
    } while (0)

size_t energy_ws(const moto_plan p, int batch) { return al(sizeof(double) * NPART * (size_t)batch * p->g.tiles); }

// Eigen-solve workspace layout (offsets in bytes from the workspace base)
// for a population of P solves (P = 1: one solve); every region holds the P
// members back to back.
struct EigLayout {
    size_t mT, cT, c64, S, HS, Xsave, part, G, ctrl, flag, info, total;
    int mb, n2, nblk_g, nblk_u, nblk_o;
    long long s_ms, part_ms, g_ms;  // per-member strides (elements, doubles, doubles)
};

EigLayout eig_layout(const moto_plan p, moto_dtype hvp, int k, int guard, int P = 1) {
    EigLayout L;
    const size_t N = p->g.N;
    const size_t es = hvp == MOTO_F64 ? sizeof(double) : sizeof(float);
    L.mb = k + guard;
    L.n2 = 2 * (int)N;
    L.nblk_g = gram_blocks(L.n2);
    L.nblk_u = update_blocks(L.n2, hvp == MOTO_F64, L.mb);
    L.nblk_o = (int)((N + NT - 1) / NT);
    L.s_ms = 3LL * L.mb * L.n2;
    size_t part = sizeof(double) * NPART * (size_t)p->g.tiles;
    part = std::max(part, sizeof(double) * (size_t)L.nblk_g * (2 * MAXS * (MAXS + 1) / 2));
    part = std::max(part, sizeof(double) * (size_t)L.nblk_u * MAXB);
    part = std::max(part, sizeof(double) * ((size_t)L.nblk_o * MAXB * 3 + MAXB));
    part = al(part);
    L.part_ms = (long long)(part / sizeof(double));
    const size_t gsz = al(sizeof(double) * 2 * MAXS * (MAXS + 1) / 2);
    L.g_ms = (long long)(gsz / sizeof(double));
    const size_t Pz = (size_t)P;
    size_t o = 0;
    L.mT = o;
    o += al(Pz * es * 3 * N);
    L.cT = o;
    o += al(Pz * es * N);
    L.c64 = o;
    o += al(Pz * sizeof(double) * N);
    L.S = o;
    o += al(Pz * es * (size_t)L.s_ms);
    L.HS = o;
    o += al(Pz * es * (size_t)L.s_ms);
    L.Xsave = o;
    o += al(Pz * es * (size_t)L.mb * 3 * N);
    L.part = o;
    o += Pz * part;
    L.G = o;
    o += Pz * gsz;
    L.ctrl = o;
    o += al(Pz * sizeof(EigCtrl));
    L.flag = o;
    o += al(sizeof(int));
    L.info = o;
    o += al(sizeof(moto_info) * Pz);
    L.total = o;
    return L;
}

// Default guard: k for k <= 4 (at least 2), then max(4, ceil(k/2)), within
// the widest block.  Measured on the 128x128 k = 4 state: guard 2, 3, 4, 8 ->
// 303, 249, 236, 196 iterations and 56, 50, 50, 70 ms; wider guards cost more
// per iteration than they save in iterations.
// Default guard (block vectors beyond the k wanted): 2 for k <= 2, 2k for
// k = 3, 4, max(4, ceil(k / 2)) above, at most MAXB - k.  With k = 4 on a
// 128x128 three-shell skyrmion state the wanted pairs sit against a band of
// close levels: guard 8 converges within 200 iterations (198), guard 4 needs
// 237 (at 0.7 of the time per iteration).
int resolve_guard(int k, int guard) {
    if (guard >= 0) return guard;
    int g = k <= 2 ? 2 : k <= 4 ? 2 * k : (k + 1) / 2;
    if (k > 4 && g < 4) g = 4;
    if (k + g > MAXB) g = MAXB - k;
    return g < 0 ? 0 : g;
}

bool hvp_ok(moto_dtype d) { return d == MOTO_F32 || d == MOTO_F64; }

int tuned_variant(const moto_plan p, moto_dtype dt, int batch, int nvec) {
    for (int i = 0; i < p->n_tune; ++i)
        if (p->tune[i].dt == (int)dt && p->tune[i].batch == batch && p->tune[i].nvec == nvec) return p->tune[i].variant;
    return -1;
}

// Offsets of the first ns shells of the triangular lattice (every lattice
// vector dx a1 + dy a2, |.|^2 = dx^2 + dx dy + dy^2, grouped by length in
// increasing order), copied from the compile-time table the kernels use,
// and the halo they need (largest |dx|, |dy|).
bool shell_table(int ns, GenShells* t) {
    if (ns < 1 || ns > GEN_MAX_SHELLS) return false;
    const ShellGeom& G = kShellGeom;
    int R = 0;
    for (int s = 0; s <= ns; ++s) t->start[s] = G.start[s];
    for (int o = 0; o < G.start[ns]; ++o) {
        t->dx[o] = G.dx[o];
        t->dy[o] = G.dy[o];
        R = std::max(R, std::max(std::abs((int)G.dx[o]), std::abs((int)G.dy[o])));
    }
    t->ns = ns;
    t->n_off = G.start[ns];
    t->R = R;
    for (int s = 0; s < GEN_MAX_SHELLS; ++s) t->cJ[s] = 0.0;
    return R <= GEN_RMAX;
}

// Read back n bytes of device memory through the plan's pinned buffer.
// true while the caller's stream is being captured into a graph (the library
// then queues plain launches: a replay of its own graph cannot be captured)
bool stream_capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return cs != hipStreamCaptureStatusNone;
}

moto_status readback(moto_plan p, const void* dev, size_t n, void* host, hipStream_t st) {
    HIP_TRY(hipMemcpyAsync(p->pinned, dev, n, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(host, p->pinned, n);
    return MOTO_OK;
}

}  // namespace

extern "C" {

const char* moto_status_string(moto_status s) {
    switch (s) {
        case MOTO_OK: return "ok";
        case MOTO_EINVAL: return "invalid argument";
        case MOTO_EHIP: return "HIP runtime error";
        case MOTO_EWORKSPACE: return "workspace too small";
        case MOTO_EUNSUPPORTED:
            return "outside the GPU scope (more than 36 exchange shells, DMI beyond the first shell, or a call "
                   "limited to three shells)";
        default: return "unknown status";
    }
}

moto_status moto_plan_create(const moto_hamiltonian* h, moto_plan* out) {
    if (!h || !out) return MOTO_EINVAL;
    *out = nullptr;
    if (h->Lx < 1 || h->Ly < 1 || h->n_shells < 1 || h->n_shells > MOTO_MAX_SHELLS || h->reserved != 0)
        return MOTO_EINVAL;
    if ((int64_t)h->Lx * h->Ly > (int64_t)1 << 28) return MOTO_EINVAL;
    for (int s = 0; s < MOTO_MAX_SHELLS; ++s) {
        if (!std::isfinite(h->J[s]) || !std::isfinite(h->D[s])) return MOTO_EINVAL;
        if (s >= 1 && h->D[s] != 0.0) return MOTO_EUNSUPPORTED;
    }
    if (!std::isfinite(h->K) || !std::isfinite(h->B[0]) || !std::isfinite(h->B[1]) || !std::isfinite(h->B[2]))
        return MOTO_EINVAL;
    moto_plan p = new (std::nothrow) moto_plan_s;
    if (!p) return MOTO_EINVAL;
    p->h = *h;
    p->g = make_geo(h->Lx, h->Ly);
    p->ns = h->n_shells;
    for (int s = 0; s < 3; ++s) p->k.cJ[s] = s < h->n_shells ? -2.0 * h->J[s] : 0.0;
    p->k.cD = 2.0 * h->D[0];
    p->k.cK = -2.0 * h->K;
    for (int a = 0; a < 3; ++a) p->k.B[a] = h->B[a];
    if (!shell_table(h->n_shells, &p->gen)) {
        delete p;
        return MOTO_EUNSUPPORTED;
    }
    for (int s = 0; s < h->n_shells; ++s) p->gen.cJ[s] = -2.0 * h->J[s];
    p->k.gen = h->n_shells > 3 ? &p->gen : nullptr;
    double sj = 0.0, sd = 0.0;
    for (int s = 0; s < h->n_shells; ++s) {
        const int cnt = p->gen.start[s + 1] - p->gen.start[s];
        sj += cnt * std::fabs(h->J[s]);
        sd += cnt * std::fabs(h->D[s]);
    }
    p->hest = 4.0 * (sj + sd) + 4.0 * std::fabs(h->K) +
              std::sqrt(h->B[0] * h->B[0] + h->B[1] * h->B[1] + h->B[2] * h->B[2]);
    p->pinned = nullptr;
    p->n_tune = 0;
    p->next_graph = 0;
    p->cap_stream = nullptr;
    p->graph_replays = 0;
    for (auto& ge : p->graphs) ge.valid = 0;
    if (hipHostMalloc((void**)&p->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        delete p;
        return MOTO_EHIP;
    }
    *out = p;
    return MOTO_OK;
}

moto_status moto_plan_destroy(moto_plan p) {
    if (!p) return MOTO_EINVAL;
    for (auto& ge : p->graphs)
        if (ge.valid) (void)hipGraphExecDestroy(ge.exec);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->pinned) (void)hipHostFree(p->pinned);
    delete p;
    return MOTO_OK;
}

double moto_hessian_norm_bound(moto_plan p) { return p ? p->hest : 0.0; }
int32_t moto_n_params(moto_plan p) { return p ? 2 * p->ns + 4 : 0; }

// ---------------------------------------------------------------------------
size_t moto_energy_grad_workspace(moto_plan p, int32_t batch) {
    if (!p || batch < 1) return 0;
    return energy_ws(p, batch);
}

int64_t moto_plan_graph_replays(moto_plan p) { return p ? p->graph_replays : -1; }

namespace {
// energy/gradient kernels with their per-tile partials in `part` (at least
// energy_ws(p, batch) bytes), then the fixed-order reduction of E and dE/dtheta
moto_status energy_grad_into(moto_plan p, moto_dtype dt, int batch, const void* m, const uint8_t* mask, double* E,
                             void* grad, void* c, void* F, double* dE_dtheta, double* part, hipStream_t st) {
    HIP_TRY(launch_energy_grad(p->g, p->k, dt == MOTO_F64, batch, m, mask, grad, c, F, part, st));
    if (E || dE_dtheta) HIP_TRY(launch_reduce_partials(part, batch, p->g.tiles, p->ns, E, dE_dtheta, st));
    return MOTO_OK;
}
}  // namespace

moto_status moto_energy_grad(moto_plan p, moto_dtype dt, int32_t batch, const void* m, const uint8_t* mask,
                             double* E, void* grad, void* c, void* F, double* dE_dtheta, void* ws,
                             size_t ws_bytes, moto_stream stream) {
    if (!p || !m || batch < 1 || !hvp_ok(dt)) return MOTO_EINVAL;
    if (p->k.gen && dE_dtheta) return MOTO_EUNSUPPORTED;
    if (!ws || ws_bytes < energy_ws(p, batch)) return MOTO_EWORKSPACE;
    return energy_grad_into(p, dt, batch, m, mask, E, grad, c, F, dE_dtheta, (double*)ws, (hipStream_t)stream);
}

moto_status moto_energy_grad_noalloc(moto_plan p, moto_dtype dt, int32_t batch, const void* m, const uint8_t* mask,
                                     double* E, void* grad, void* c, void* F, double* dE_dtheta, moto_stream stream) {
    if (!p || !m || batch < 1 || !hvp_ok(dt)) return MOTO_EINVAL;
    if (p->k.gen && dE_dtheta) return MOTO_EUNSUPPORTED;
    if (energy_ws(p, batch) > ENERGY_SCRATCH_BYTES) return MOTO_EWORKSPACE;
    double* part = nullptr;
    HIP_TRY(energy_scratch(&part));
    return energy_grad_into(p, dt, batch, m, mask, E, grad, c, F, dE_dtheta, part, (hipStream_t)stream);
}

moto_status moto_tangent_hvp(moto_plan p, moto_dtype dt, moto_layout layout, int32_t batch, const void* m,
                             const void* c, const uint8_t* mask, int32_t n_vec, const void* V, void* W,
                             moto_stream stream) {
    if (!p || !m || !c || !V || !W || batch < 1 || n_vec < 0 || !hvp_ok(dt)) return MOTO_EINVAL;
    if (layout != MOTO_AMBIENT && layout != MOTO_FRAME) return MOTO_EINVAL;
    if (V == W) return MOTO_EINVAL;
    if (n_vec == 0) return MOTO_OK;
    HIP_TRY(launch_tangent_hvp(p->g, p->k, dt == MOTO_F64, layout == MOTO_FRAME, batch, m, c, mask, n_vec, V, W,
                               nullptr, (hipStream_t)stream, tuned_variant(p, dt, batch, n_vec)));
    return MOTO_OK;
}

int32_t moto_tangent_hvp_variants(void) { return HVP_NVARIANTS; }

moto_status moto_plan_set_hvp_variant(moto_plan p, moto_dtype dt, int32_t batch, int32_t n_vec, int32_t variant) {
    if (!p || !hvp_ok(dt) || batch < 1 || n_vec < 1 || !hvp_variant_ok(variant, p->g, dt == MOTO_F64)) return MOTO_EINVAL;
    if (p->k.gen) return MOTO_EUNSUPPORTED;
    int slot = -1;
    for (int i = 0; i < p->n_tune; ++i)
        if (p->tune[i].dt == (int)dt && p->tune[i].batch == batch && p->tune[i].nvec == n_vec) slot = i;
    if (slot < 0) slot = p->n_tune < 32 ? p->n_tune++ : 31;
    p->tune[slot] = {(int)dt, batch, n_vec, variant};
    return MOTO_OK;
}

const char* moto_tangent_hvp_variant_name(int32_t v) { return hvp_variant_name(v); }

moto_status moto_tangent_hvp_autotune(moto_plan p, moto_dtype dt, int32_t batch, const void* m, const void* c,
                                      const uint8_t* mask, int32_t n_vec, const void* V, void* W, int32_t reps,
                                      int32_t* chosen, float* times_ms, moto_stream stream) {
    if (!p || !m || !c || !V || !W || batch < 1 || n_vec < 1 || !hvp_ok(dt) || V == W) return MOTO_EINVAL;
    if (p->k.gen) return MOTO_EUNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = dt == MOTO_F64;
    if (reps < 1) reps = 3;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int best = -1;
    float best_t = 0.0f;
    for (int v = 0; v < HVP_NVARIANTS; ++v) {
        if (times_ms) times_ms[v] = -1.0f;
        if (!hvp_variant_ok(v, p->g, f64)) continue;
        HIP_TRY(launch_hvp_frame(v, p->g, p->k, f64, batch, m, c, mask, n_vec, V, W, nullptr, st));  // warm-up
        HIP_TRY(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r)
            HIP_TRY(launch_hvp_frame(v, p->g, p->k, f64, batch, m, c, mask, n_vec, V, W, nullptr, st));
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        ms /= reps;
        if (times_ms) times_ms[v] = ms;
        if (best < 0 || ms < best_t) {
            best = v;
            best_t = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int slot = -1;
    for (int i = 0; i < p->n_tune; ++i)
        if (p->tune[i].dt == (int)dt && p->tune[i].batch == batch && p->tune[i].nvec == n_vec) slot = i;
    if (slot < 0) {
        slot = p->n_tune < 32 ? p->n_tune++ : 31;
    }
    p->tune[slot] = {(int)dt, batch, n_vec, best};
    if (chosen) *chosen = best;
    return MOTO_OK;
}

moto_status moto_hessian_apply(moto_plan p, moto_dtype dt, int32_t batch, int32_t n_vec, const void* V, void* W,
                               moto_stream stream) {
    if (!p || !V || !W || batch < 1 || n_vec < 0 || !hvp_ok(dt) || V == W) return MOTO_EINVAL;
    if (p->k.gen) return MOTO_EUNSUPPORTED;
    if (n_vec == 0) return MOTO_OK;
    HIP_TRY(launch_hessian_apply(p->g, p->k, dt == MOTO_F64, batch, n_vec, V, W, (hipStream_t)stream));
    return MOTO_OK;
}

moto_status moto_param_mixed(moto_plan p, moto_dtype dt, int32_t batch, const void* m, const void* U, double* out,
                             void* ws, size_t ws_bytes, moto_stream stream) {
    if (!p || !m || !U || !out || batch < 1 || !hvp_ok(dt)) return MOTO_EINVAL;
    if (p->k.gen) return MOTO_EUNSUPPORTED;
    if (!ws || ws_bytes < energy_ws(p, batch)) return MOTO_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_param_mixed(p->g, dt == MOTO_F64, batch, m, U, (double*)ws, st));
    HIP_TRY(launch_reduce_partials((double*)ws, batch, p->g.tiles, p->ns, nullptr, out, st));
    return MOTO_OK;
}

moto_status moto_param_grad_apply(moto_plan p, moto_dtype dt, int32_t batch, const void* m, const double* w,
                                  void* out, moto_stream stream) {
    if (!p || !m || !w || !out || batch < 1 || !hvp_ok(dt)) return MOTO_EINVAL;
    if (p->k.gen) return MOTO_EUNSUPPORTED;
    HIP_TRY(launch_param_grad_apply(p->g, p->ns, dt == MOTO_F64, batch, m, w, out, (hipStream_t)stream));
    return MOTO_OK;
}

moto_status moto_topological_charge(moto_plan p, int32_t batch, const double* m, double* Q, void* ws,
                                    size_t ws_bytes, moto_stream stream) {
    if (!p || !m || !Q || batch < 1) return MOTO_EINVAL;
    if (!ws || ws_bytes < energy_ws(p, batch)) return MOTO_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_topo_charge(p->g, batch, m, (double*)ws, st));
    HIP_TRY(launch_reduce_partials((double*)ws, batch, p->g.tiles, p->ns, Q, nullptr, st));
    return MOTO_OK;
}

// ---------------------------------------------------------------------------
void moto_default_eig_opts(moto_dtype hvp, moto_eig_opts* o) {
    if (!o) return;
    o->tol = hvp == MOTO_F64 ? 1e-10 : 1e-5;
    o->max_iter = 200;
    o->guard = -1;
    o->warm = 0;
    o->check_every = 8;
    o->seed = 0x2509262690ull;
    o->use_graph = 1;
    o->flags = 0;
}

size_t moto_min_modes_workspace(moto_plan p, moto_dtype hvp, int32_t k, int32_t guard) {
    if (!p || k < 1 || !hvp_ok(hvp)) return 0;
    return eig_layout(p, hvp, k, resolve_guard(k, guard)).total;
}

// Capture one chunk of launches into an instantiated graph stored in the
// plan's cache (round robin over four slots).  Returns nullptr, with the
// runtime's sticky error cleared, when capture or instantiation fails.
extern "C++" {
template <class F>
static hipGraphExec_t capture_chunk(moto_plan p, F& launches, const long long* key, const void* ws,
                                    const void* mask) {
    if (!p->cap_stream && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        p->cap_stream = nullptr;
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    const hipError_t ce = launches(p->cap_stream);
    const hipError_t ee = hipStreamEndCapture(p->cap_stream, &graph);
    hipGraphExec_t exec = nullptr;
    if (ce == hipSuccess && ee == hipSuccess && graph &&
        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
        exec = nullptr;
    if (graph) (void)hipGraphDestroy(graph);
    if (!exec) {
        (void)hipGetLastError();
        return nullptr;
    }
    auto& slot = p->graphs[p->next_graph];
    p->next_graph = (p->next_graph + 1) % 4;
    if (slot.valid) (void)hipGraphExecDestroy(slot.exec);
    slot.exec = exec;
    slot.ws = ws;
    slot.mask = mask;
    std::memcpy(slot.key, key, sizeof(slot.key));
    slot.valid = 1;
    return exec;
}
}  // extern "C++"

// P independent solves on lattices of the plan's geometry (P = 1: one solve).
// m [P][3][N], mask [P][N] or null, evals [P][k], V [P][k][3][N], resid [P][k]
// or null, info host [P] or null.
static moto_status min_modes_pop_impl(moto_plan p, moto_dtype hvp, int P, const double* m, const uint8_t* mask,
                                      int k, const moto_eig_opts* o, double* evals, double* V, double* resid,
                                      moto_info* info, char* ws, size_t ws_bytes, hipStream_t st,
                                      const double* c64_in) {
    const int guard = resolve_guard(k, o->guard);
    const bool async = (o->flags & MOTO_ASYNC) != 0;
    const EigLayout L = eig_layout(p, hvp, k, guard, P);
    if (L.mb > MAXB || L.mb > L.n2) return MOTO_EINVAL;
    if (ws_bytes < L.total) return MOTO_EWORKSPACE;
    const bool f64 = hvp == MOTO_F64;
    const int N = p->g.N;
    double* c64 = (double*)(ws + L.c64);
    double* part = (double*)(ws + L.part);
    EigCtrl* ctrl = (EigCtrl*)(ws + L.ctrl);
    int* all_done = (int*)(ws + L.flag);
    // c_i = m_i . g_i at m (FP64)
    if (c64_in) {
        HIP_TRY(hipMemcpyAsync(c64, c64_in, sizeof(double) * N * (size_t)P, hipMemcpyDeviceToDevice, st));
    } else {
        HIP_TRY(launch_energy_grad(p->g, p->k, true, P, m, nullptr, nullptr, c64, nullptr, part, st));
    }
    // the spins are staged in the workspace in the HVP precision (a copy in
    // FP64), so that a captured iteration chunk refers to workspace memory
    // only and stays valid for any caller's m
    const void* mT = ws + L.mT;
    const void* cT = c64;
    if (!f64) {
        HIP_TRY(launch_f64_to_f32(m, (float*)(ws + L.mT), 3 * (size_t)N * P, st));
        HIP_TRY(launch_f64_to_f32(c64, (float*)(ws + L.cT), (size_t)N * P, st));
        cT = ws + L.cT;
    } else {
        HIP_TRY(hipMemcpyAsync(ws + L.mT, m, sizeof(double) * 3 * (size_t)N * P, hipMemcpyDeviceToDevice, st));
    }
    EigArgs a;
    a.n2 = L.n2;
    a.mb = L.mb;
    a.k = k;
    a.max_iter = o->max_iter;
    a.tol_abs = o->tol * p->hest;
    a.drop = f64 ? 1e-13 : 1e-9;
    a.P = P;
    a.s_ms = P > 1 ? L.s_ms : 0;
    a.part_ms = P > 1 ? L.part_ms : 0;
    a.g_ms = P > 1 ? L.g_ms : 0;
    a.mask = mask;
    a.Nsite = (int)p->g.N;
    a.mask_ms = P > 1 ? (long long)p->g.N : 0;
    // The vector row kernels skip the rows of inactive sites, so in a masked
    // population most of their P x nblk workgroups find nothing to do: cap
    // the grids at 4096 (Grams) and 2048 (updates) workgroups over the
    // members (64 x 128x128 with a disc of 241 sites: +13 % outer iterations
    // per second; a single member keeps its full grid, a quarter of which
    // measured 7 % slower)
    int nbg = L.nblk_g, nbu = L.nblk_u;
    if (mask && !rows_on_matrix_cores(f64, L.mb)) {
        nbg = std::max(1, std::min(nbg, (4096 + P - 1) / P));
        nbu = std::max(1, std::min(nbu, (2048 + P - 1) / P));
    }
    void* S = ws + L.S;
    void* HS = ws + L.HS;
    const size_t es = f64 ? sizeof(double) : sizeof(float);
    void* Wslot = (char*)S + es * (size_t)L.mb * L.n2;
    void* HWslot = (char*)HS + es * (size_t)L.mb * L.n2;
    // the HVP of the whole population is one batched launch; it stops once
    // every member is done
    const int* hv_done = P > 1 ? all_done : &ctrl->done;
    const long long vbs = L.s_ms;
    const int warm = o->warm;
    const int hv_var = tuned_variant(p, hvp, P, L.mb);
    double* G = (double*)(ws + L.G);
    auto control = [&](int first, hipStream_t s) -> hipError_t {
        hipError_t e = launch_eig_control(a, part, nbu, ctrl, first, s);
        if (e == hipSuccess && P > 1) e = launch_eig_all_done(a, ctrl, all_done, s);
        return e;
    };
    HIP_TRY(launch_eig_init(f64, a, S, m, warm == 1 ? V : nullptr, warm == 1 ? k : 0, ws + L.Xsave, warm == 2,
                            mask, N, o->seed, ctrl, st));
    HIP_TRY(launch_check_finite(m, c64, N, P, ctrl, st));
    if (P > 1) HIP_TRY(launch_eig_all_done(a, ctrl, all_done, st));
    // start: orthonormal X; HX = H X; Rayleigh-Ritz on span(X); W = HX - X Lam
    for (int pass = 0; pass < 2; ++pass) HIP_TRY(launch_orth(f64, a, 0, S, part, nbg, G, ctrl, st));
    HIP_TRY(launch_tangent_hvp(p->g, p->k, f64, true, P, mT, cT, mask, L.mb, S, HS, hv_done, st, hv_var, vbs));
    HIP_TRY(launch_gram(f64, a, L.mb, S, HS, part, nbg, G, ctrl, st));
    HIP_TRY(launch_rr(a, L.mb, G, ctrl, st));
    HIP_TRY(launch_update(f64, a, L.mb, S, HS, part, nbu, ctrl, st));
    HIP_TRY(control(1, st));
    const int every = o->check_every > 0 ? o->check_every : 8;
    const int max_chunks = o->max_iter / every + 2;
    auto chunk_launches = [&](hipStream_t s) -> hipError_t {
        for (int it = 0; it < every; ++it) {
            for (int pass = 0; pass < 2; ++pass) {
                hipError_t e = launch_orth(f64, a, 1 + pass, S, part, nbg, G, ctrl, s);
                if (e != hipSuccess) return e;
            }
            hipError_t e = launch_tangent_hvp(p->g, p->k, f64, true, P, mT, cT, mask, L.mb, Wslot, HWslot, hv_done,
                                              s, hv_var, vbs);
            if (e == hipSuccess) e = launch_gram(f64, a, -1, S, HS, part, nbg, G, ctrl, s);
            if (e == hipSuccess) e = launch_rr(a, -1, G, ctrl, s);
            if (e == hipSuccess) e = launch_update(f64, a, -1, S, HS, part, nbu, ctrl, s);
            if (e == hipSuccess) e = control(0, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    // one iteration chunk as a HIP graph, captured once per key on the plan's
    // private stream and replayed on the caller's; any capture failure falls
    // back to plain launches
    hipGraphExec_t gexec = nullptr;
    if (o->use_graph && !stream_capturing(st)) {
        long long key[8];
        double tolbits = a.tol_abs;
        std::memcpy(&key[0], &tolbits, sizeof(double));
        key[1] = (long long)hvp;
        key[2] = L.mb;
        key[3] = k;
        key[4] = every;
        key[5] = o->max_iter;
        key[6] = hv_var;
        key[7] = N + ((long long)P << 32);
        for (auto& ge : p->graphs)
            if (ge.valid && ge.ws == (const void*)ws && ge.mask == (const void*)mask &&
                std::memcmp(ge.key, key, sizeof(key)) == 0)
                gexec = ge.exec;
        if (!gexec) gexec = capture_chunk(p, chunk_launches, key, ws, mask);
    }
    const int* done_dev = P > 1 ? all_done : &ctrl->done;
    auto one_chunk = [&]() -> hipError_t {
        if (!gexec) return chunk_launches(st);
        p->graph_replays += 1;
        return hipGraphLaunch(gexec, st);
    };
    // with host synchronisation the done flag is read before each chunk (a
    // read-back queued behind a running chunk, to overlap the round trip,
    // measured slower: the chunk's kernels then start with gaps)
    for (int chunk = 0; chunk < max_chunks; ++chunk) {
        if (!async) {
            int hdr[1];
            moto_status rs = readback(p, done_dev, sizeof(hdr), hdr, st);
            if (rs != MOTO_OK) return rs;
            if (hdr[0]) break;
        }
        HIP_TRY(one_chunk());
    }
    HIP_TRY(launch_eig_output(f64, a, S, m, N, V, part, ctrl, evals, resid, ws + L.Xsave, st));
    if (async) {
        // outcome straight into the caller's device array; no synchronisation
        if (info) HIP_TRY(launch_eig_gather_info(P, ctrl, info, st));
    } else if (info) {
        // status, iterations and HVP columns of every member, gathered and
        // read back at once (P <= MOTO_MAX_POPULATION fits the pinned buffer)
        HIP_TRY(launch_eig_gather_info(P, ctrl, (moto_info*)(ws + L.info), st));
        moto_status rs = readback(p, ws + L.info, sizeof(moto_info) * (size_t)P, info, st);
        if (rs != MOTO_OK) return rs;
    } else {
        HIP_TRY(hipStreamSynchronize(st));
    }
    return MOTO_OK;
}

static moto_status min_modes_impl(moto_plan p, moto_dtype hvp, const double* m, const uint8_t* mask, int k,
                                  const moto_eig_opts* o, double* evals, double* V, double* resid, moto_info* info,
                                  char* ws, size_t ws_bytes, hipStream_t st, const double* c64_in) {
    return min_modes_pop_impl(p, hvp, 1, m, mask, k, o, evals, V, resid, info, ws, ws_bytes, st, c64_in);
}

moto_status moto_min_modes(moto_plan p, moto_dtype hvp, const double* m, const uint8_t* mask, int32_t k,
                           const moto_eig_opts* opts, double* evals, double* V, double* resid, moto_info* info,
                           void* ws, size_t ws_bytes, moto_stream stream) {
    if (!p || !m || !V || !evals || k < 1 || !hvp_ok(hvp)) return MOTO_EINVAL;
    moto_eig_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_eig_opts(hvp, &o);
    if (o.max_iter < 0 || !(o.tol >= 0.0) || o.warm < 0 || o.warm > 2 || (o.flags & ~MOTO_ASYNC)) return MOTO_EINVAL;
    if (!ws) return MOTO_EWORKSPACE;
    return min_modes_impl(p, hvp, m, mask, k, &o, evals, V, resid, info, (char*)ws, ws_bytes,
                          (hipStream_t)stream, nullptr);
}

size_t moto_min_modes_population_workspace(moto_plan p, moto_dtype hvp, int32_t P, int32_t k, int32_t guard) {
    if (!p || k < 1 || P < 1 || P > MOTO_MAX_POPULATION || !hvp_ok(hvp)) return 0;
    return eig_layout(p, hvp, k, resolve_guard(k, guard), P).total;
}

moto_status moto_min_modes_population(moto_plan p, moto_dtype hvp, int32_t P, const double* m,
                                      const uint8_t* mask, int32_t k, const moto_eig_opts* opts, double* evals,
                                      double* V, double* resid, moto_info* info, void* ws, size_t ws_bytes,
                                      moto_stream stream) {
    if (!p || !m || !V || !evals || k < 1 || P < 1 || P > MOTO_MAX_POPULATION || !hvp_ok(hvp)) return MOTO_EINVAL;
    moto_eig_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_eig_opts(hvp, &o);
    if (o.max_iter < 0 || !(o.tol >= 0.0) || o.warm < 0 || o.warm > 2 || (o.flags & ~MOTO_ASYNC)) return MOTO_EINVAL;
    if (!ws) return MOTO_EWORKSPACE;
    return min_modes_pop_impl(p, hvp, P, m, mask, k, &o, evals, V, resid, info, (char*)ws, ws_bytes,
                              (hipStream_t)stream, nullptr);
}

// ---------------------------------------------------------------------------
// Thick-restart Lanczos (second inner solver)
// ---------------------------------------------------------------------------
void moto_default_lanczos_opts(moto_dtype hvp, moto_lanczos_opts* o) {
    if (!o) return;
    o->tol = hvp == MOTO_F64 ? 1e-10 : 1e-5;
    o->m_max = 32;
    o->keep = 0;
    o->max_restarts = 200;
    o->warm = 0;
    o->seed = 0x2509262690ull;
    o->use_graph = 1;
    o->block = 0;
}

namespace {
struct LzLayout {
    size_t mT, cT, c64, Q, part, ctrl, total;
    int n2, nblk;
};

// the basis holds m_max + LZ_MAXBLK columns whatever the block size, so that
// the workspace size depends on the depth alone
LzLayout lz_layout(const moto_plan p, moto_dtype hvp, int m_max) {
    LzLayout L;
    const size_t N = p->g.N;
    const size_t es = hvp == MOTO_F64 ? sizeof(double) : sizeof(float);
    L.n2 = 2 * (int)N;
    L.nblk = lz_blocks(L.n2);
    const int nblk_o = (int)((N + NT - 1) / NT);
    size_t o = 0;
    L.mT = o;
    o += al(es * 3 * N);
    L.cT = o;
    o += al(es * N);
    L.c64 = o;
    o += al(sizeof(double) * N);
    L.Q = o;
    o += al(es * (size_t)(m_max + LZ_MAXBLK) * L.n2);
    size_t part = sizeof(double) * NPART * (size_t)p->g.tiles;
    part = std::max(part, sizeof(double) * (size_t)L.nblk * (LZ_NCOL + 1));
    part = std::max(part, sizeof(double) * ((size_t)nblk_o * MAXB * 3 + MAXB));
    L.part = o;
    o += al(part);
    L.ctrl = o;
    o += al(sizeof(LzCtrl));
    L.total = o;
    return L;
}

int lz_keep(int k, int m_max, int keep) { return keep > 0 ? keep : std::max(k + 2, m_max / 2); }
int lz_block(int block) { return block > 0 ? block : 2; }
}  // namespace

size_t moto_min_modes_lanczos_workspace(moto_plan p, moto_dtype hvp, int32_t m_max) {
    if (!p || !hvp_ok(hvp) || m_max < 3 || m_max > LZ_MAXM) return 0;
    return lz_layout(p, hvp, m_max).total;
}

moto_status moto_min_modes_lanczos(moto_plan p, moto_dtype hvp, const double* m, const uint8_t* mask, int32_t k,
                                   const moto_lanczos_opts* opts, double* evals, double* V, double* resid,
                                   moto_info* info, void* ws_, size_t ws_bytes, moto_stream stream) {
    if (!p || !m || !V || !evals || k < 1 || k > MAXB || !hvp_ok(hvp)) return MOTO_EINVAL;
    moto_lanczos_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_lanczos_opts(hvp, &o);
    const int keep = lz_keep(k, o.m_max, o.keep);
    const int b = lz_block(o.block);
    if (o.m_max < 3 || o.m_max > LZ_MAXM || b > LZ_MAXBLK || o.block < 0 || keep < k || keep + b > o.m_max ||
        !(o.tol >= 0.0) || o.max_restarts < 0 || o.warm < 0 || o.warm > 1)
        return MOTO_EINVAL;
    if (o.m_max + b > 2 * p->g.N) return MOTO_EINVAL;  // the Krylov basis must fit the space
    char* ws = (char*)ws_;
    const LzLayout L = lz_layout(p, hvp, o.m_max);
    if (!ws) return MOTO_EWORKSPACE;
    if (ws_bytes < L.total) return MOTO_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = hvp == MOTO_F64;
    const int N = p->g.N;
    double* c64 = (double*)(ws + L.c64);
    double* part = (double*)(ws + L.part);
    LzCtrl* ctrl = (LzCtrl*)(ws + L.ctrl);
    void* Q = ws + L.Q;
    const size_t es = f64 ? sizeof(double) : sizeof(float);
    HIP_TRY(launch_energy_grad(p->g, p->k, true, 1, m, nullptr, nullptr, c64, nullptr, part, st));
    // spins staged in the workspace (see min_modes_pop_impl)
    const void* mT = ws + L.mT;
    const void* cT = c64;
    if (!f64) {
        HIP_TRY(launch_f64_to_f32(m, (float*)(ws + L.mT), 3 * (size_t)N, st));
        HIP_TRY(launch_f64_to_f32(c64, (float*)(ws + L.cT), (size_t)N, st));
        cT = ws + L.cT;
    } else {
        HIP_TRY(hipMemcpyAsync(ws + L.mT, m, sizeof(double) * 3 * (size_t)N, hipMemcpyDeviceToDevice, st));
    }
    const int hv_var = tuned_variant(p, hvp, 1, 1);
    HIP_TRY(launch_lz_init(f64, N, b, Q, m, o.warm ? V : nullptr, o.warm ? k : 0, mask, o.seed, ctrl, o.m_max, st));
    HIP_TRY(launch_check_finite(m, c64, N, ctrl, st));
    const double tol_abs = o.tol * p->hest;
    // one cycle from kept column j0: re-orthonormalise the b columns j0.. (the
    // start block, or the residual block after a restart), then the steps
    // j0 .. m_max-1, each an HVP of column j into column j + b
    auto cycle = [&](int j0, hipStream_t s) -> hipError_t {
        for (int l = 0; l < b; ++l) {
            hipError_t e = launch_lz_orth(f64, L.n2, Q, j0 + l, -1, part, L.nblk, ctrl, s);
            if (e != hipSuccess) return e;
        }
        for (int j = j0; j < o.m_max; ++j) {
            hipError_t e = launch_tangent_hvp(p->g, p->k, f64, true, 1, mT, cT, mask, 1, (char*)Q + es * j * L.n2,
                                              (char*)Q + es * (j + b) * L.n2, &ctrl->done, s, hv_var);
            if (e == hipSuccess) e = launch_lz_orth(f64, L.n2, Q, j + b, j, part, L.nblk, ctrl, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    // the cycles after the first repeat the same launches (from column keep):
    // captured once as a HIP graph and replayed
    hipGraphExec_t gexec = nullptr;
    if (o.use_graph) {
        long long key[8];
        std::memcpy(&key[0], &tol_abs, sizeof(double));
        key[1] = (long long)hvp + 1000;  // distinct from the eigen-solver keys
        key[2] = o.m_max;
        key[3] = keep;
        key[4] = k;
        key[5] = -b;
        key[6] = hv_var;
        key[7] = N;
        for (auto& ge : p->graphs)
            if (ge.valid && ge.ws == (const void*)ws && ge.mask == (const void*)mask &&
                std::memcmp(ge.key, key, sizeof(key)) == 0)
                gexec = ge.exec;
        if (!gexec) {
            auto cyc = [&](hipStream_t s) { return cycle(keep, s); };
            gexec = capture_chunk(p, cyc, key, ws, mask);
        }
    }
    int hdr[6] = {0, 0, 0, 0, 0, keep};  // done, status, restarts, m_eff, m_max, nkeep
    for (int c = 0; c <= o.max_restarts + 1; ++c) {
        if (c == 0)
            HIP_TRY(cycle(0, st));
        else if (gexec && hdr[5] == keep) {
            HIP_TRY(hipGraphLaunch(gexec, st));
            p->graph_replays += 1;
        }
        else
            HIP_TRY(cycle(hdr[5], st));  // a breakdown kept fewer Ritz vectors than `keep`
        HIP_TRY(launch_lz_rr_restart(f64, L.n2, b, Q, k, keep, tol_abs, o.max_restarts, o.m_max, L.nblk, mask, N,
                                     o.seed, ctrl, st));
        moto_status rs = readback(p, ctrl, sizeof(hdr), hdr, st);
        if (rs != MOTO_OK) return rs;
        if (hdr[0]) break;
    }
    EigArgs a;
    a.n2 = L.n2;
    a.mb = k;
    a.k = k;
    a.max_iter = 0;
    a.tol_abs = tol_abs;
    a.drop = 0.0;
    HIP_TRY(launch_eig_output(f64, a, Q, m, N, V, part, &ctrl->out, evals, resid, nullptr, st));
    EigCtrl hc;
    moto_status rs = readback(p, &ctrl->out, 32, &hc, st);
    if (rs != MOTO_OK) return rs;
    if (info) {
        info->status = hc.status;
        info->iters = hc.iters;
        info->n_hvp = hc.n_hvp;
    }
    return MOTO_OK;
}

// ---------------------------------------------------------------------------
void moto_default_step_opts(moto_step_opts* o) {
    if (!o) return;
    o->rule = 0;
    o->mem = 8;
    o->theta_max = 0.1;
    o->alpha0 = 0.0;
    o->sy_min = 1e-12;
    o->tau_F = 1e-6;
}

size_t moto_step_state_bytes(moto_plan p, int32_t mem) {
    if (!p || mem < 1 || mem > 16) return 0;
    return step_state_bytes(p->g.N, mem);
}

static bool fill_step_args(moto_plan p, const moto_step_opts* o, int k_reflect, StepArgs* a) {
    if (o->rule < 0 || o->rule > 2) return false;
    if (o->mem < 1 || o->mem > 16 || !(o->theta_max > 0.0) || k_reflect < 0 || k_reflect > 4) return false;
    a->N = p->g.N;
    a->mem = o->rule == 2 ? 1 : o->mem;  // CG keeps one (s, y) pair
    a->rule = o->rule;
    a->k_reflect = k_reflect;
    a->theta_max = o->theta_max;
    a->alpha0 = o->alpha0 > 0.0 ? o->alpha0 : 1.0 / p->hest;
    a->sy_min = o->sy_min;
    a->tau_F = o->tau_F;
    return true;
}

moto_status moto_reflected_step(moto_plan p, double* m, const double* F, const double* V, int32_t k_reflect,
                                const moto_step_opts* opts, void* state, double* out, moto_stream stream) {
    if (!p || !m || !F || !state || !out || (k_reflect > 0 && !V)) return MOTO_EINVAL;
    moto_step_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_step_opts(&o);
    StepArgs a;
    if (!fill_step_args(p, &o, k_reflect, &a)) return MOTO_EINVAL;
    HIP_TRY(launch_step(a, m, F, V, state, out, (hipStream_t)stream));
    return MOTO_OK;
}

// ---------------------------------------------------------------------------
void moto_default_descend_opts(moto_dtype hvp, moto_descend_opts* o) {
    if (!o) return;
    o->eta = 0.1;
    o->tau_F = 1e-6;
    o->max_iter = 5000;
    o->check_every = 16;
    moto_default_step_opts(&o->step);
    moto_default_eig_opts(hvp, &o->eig);
    o->flags = 0;
    o->reserved = 0;
}

// Descent / search workspace: [energy partials][F 3N][out 2][state][eig ws][V k_max 3N][evals]
struct DrvLayout {
    size_t epart, F, out, state, eig, V, ev, total;
};

static DrvLayout drv_layout(moto_plan p, moto_dtype hvp, int mem, int kmax, int guard) {
    DrvLayout L;
    const size_t N = p->g.N;
    size_t o = 0;
    L.epart = o;
    o += energy_ws(p, 1);
    L.F = o;
    o += al(sizeof(double) * 3 * N);
    L.out = o;
    o += al(sizeof(double) * 4);
    L.state = o;
    o += al(step_state_bytes((int)N, mem));
    L.eig = o;
    o += al(eig_layout(p, hvp, kmax, resolve_guard(kmax, guard)).total);
    L.V = o;
    o += al(sizeof(double) * 3 * N * (size_t)kmax);
    L.ev = o;
    o += al(sizeof(double) * 2 * (size_t)kmax);
    L.total = o;
    return L;
}

size_t moto_descend_workspace(moto_plan p, moto_dtype hvp, const moto_descend_opts* o) {
    if (!p || !hvp_ok(hvp)) return 0;
    moto_descend_opts d;
    if (o)
        d = *o;
    else
        moto_default_descend_opts(hvp, &d);
    if (d.step.mem < 1 || d.step.mem > 16) return 0;
    return drv_layout(p, hvp, d.step.mem, 1, d.eig.guard).total;
}

moto_status moto_descend(moto_plan p, moto_dtype hvp, double* m, const double* v1, int32_t sign,
                         const moto_descend_opts* opts, moto_descend_result* res, void* ws, size_t ws_bytes,
                         moto_stream stream) {
    if (!p || !m || !v1 || !res || (sign != 1 && sign != -1) || !hvp_ok(hvp)) return MOTO_EINVAL;
    moto_descend_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_descend_opts(hvp, &o);
    if (!(o.eta > 0.0) || o.max_iter < 0 || (o.flags & ~MOTO_ASYNC)) return MOTO_EINVAL;
    const bool async = (o.flags & MOTO_ASYNC) != 0;
    o.step.tau_F = o.tau_F;
    StepArgs a;
    if (!fill_step_args(p, &o.step, 0, &a)) return MOTO_EINVAL;
    const DrvLayout L = drv_layout(p, hvp, o.step.mem, 1, o.eig.guard);
    if (!ws || ws_bytes < L.total) return MOTO_EWORKSPACE;
    char* w = (char*)ws;
    hipStream_t st = (hipStream_t)stream;
    const int N = p->g.N;
    double* F = (double*)(w + L.F);
    double* out = (double*)(w + L.out);
    double* part = (double*)(w + L.epart);
    HIP_TRY(launch_zero(w + L.state, step_state_bytes(N, o.step.mem), st));
    HIP_TRY(launch_zero(out, sizeof(double) * 4, st));
    HIP_TRY(launch_seed_rotate(N, m, v1, sign * o.eta, part, st));
    const int every = o.check_every > 0 ? o.check_every : 16;
    int it = 0;
    double ho[2] = {0.0, 0.0};
    while (it < o.max_iter) {
        // the step kernels return at once after the stop test has passed, so
        // the steps queued past it (all of them with MOTO_ASYNC) change nothing
        const int n = async ? o.max_iter : std::min(every, o.max_iter - it);
        for (int q = 0; q < n; ++q) {
            HIP_TRY(launch_energy_grad(p->g, p->k, true, 1, m, nullptr, nullptr, nullptr, F, part, st));
            HIP_TRY(launch_step(a, m, F, nullptr, w + L.state, out, st));
        }
        it += n;
        if (async) break;
        moto_status rs = readback(p, out, sizeof(ho), ho, st);
        if (rs != MOTO_OK) return rs;
        if (ho[1] != 0.0 || !std::isfinite(ho[0])) break;
    }
    // final quantities at the relaxed state
    double* E = (double*)(w + L.ev);
    HIP_TRY(launch_energy_grad(p->g, p->k, true, 1, m, nullptr, nullptr, nullptr, F, part, st));
    HIP_TRY(launch_reduce_partials(part, 1, p->g.tiles, p->ns, E, nullptr, st));
    // lambda_1 at the relaxed state
    moto_eig_opts eo = o.eig;
    eo.warm = 0;
    eo.flags = async ? MOTO_ASYNC : 0;
    double lam = 0.0;
    moto_info inf;
    moto_status rs = min_modes_impl(p, hvp, m, nullptr, 1, &eo, E + 1, (double*)(w + L.V), nullptr,
                                    async ? nullptr : &inf, w + L.eig, ws_bytes - L.eig, st, nullptr);
    if (rs != MOTO_OK) return rs;
    HIP_TRY(launch_topo_charge(p->g, 1, m, part, st));
    double Qd[1];
    HIP_TRY(launch_reduce_partials(part, 1, p->g.tiles, p->ns, (double*)(w + L.out) + 2, nullptr, st));
    if (async) {
        HIP_TRY(launch_descend_result(w + L.state, N, o.step.mem, out, E, out + 2, (moto_descend_result*)res, st));
        return MOTO_OK;
    }
    double hv[4];
    rs = readback(p, w + L.ev, 2 * sizeof(double), hv, st);
    if (rs != MOTO_OK) return rs;
    rs = readback(p, (double*)(w + L.out) + 2, sizeof(double), Qd, st);
    if (rs != MOTO_OK) return rs;
    lam = hv[1];
    // ||F|| at the final point: the step state holds it when stopped; otherwise
    // recompute through one stop-only test
    res->converged = ho[1] != 0.0 ? 1 : 0;
    res->iters = it;
    res->E = hv[0];
    res->Q = Qd[0];
    res->fnorm = ho[0];
    res->lambda1 = lam;
    {
        // exact step count from the state header
        int hdr[5];
        rs = readback(p, w + L.state, sizeof(hdr), hdr, st);
        if (rs != MOTO_OK) return rs;
        res->iters = hdr[4];
    }
    return MOTO_OK;
}

// ---------------------------------------------------------------------------
void moto_default_search_opts(moto_dtype hvp, moto_search_opts* o) {
    if (!o) return;
    o->tau_F = 1e-6;
    o->tau_lam = 0.0;
    o->k = 1;
    o->k_cert = 2;
    o->k_reflect = 1;
    o->max_outer = 5000;
    moto_default_step_opts(&o->step);
    moto_default_eig_opts(hvp, &o->eig);
}

size_t moto_saddle_search_workspace(moto_plan p, moto_dtype hvp, const moto_search_opts* o) {
    if (!p || !hvp_ok(hvp)) return 0;
    moto_search_opts d;
    if (o)
        d = *o;
    else
        moto_default_search_opts(hvp, &d);
    if (d.step.mem < 1 || d.step.mem > 16 || d.k < 1) return 0;
    const int kmax = std::max(d.k, std::max(d.k_cert, 2));
    return drv_layout(p, hvp, d.step.mem, kmax, d.eig.guard).total;
}

moto_status moto_saddle_search(moto_plan p, moto_dtype hvp, double* m, const uint8_t* mask,
                               const moto_search_opts* opts, moto_search_result* res, double* evals_out,
                               double* V_out, void* ws, size_t ws_bytes, moto_stream stream) {
    if (!p || !m || !res || !hvp_ok(hvp)) return MOTO_EINVAL;
    moto_search_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_search_opts(hvp, &o);
    if (o.k < 1 || o.k_reflect < 0 || o.k_reflect > o.k || o.k_reflect > 4 || o.max_outer < 0) return MOTO_EINVAL;
    const int kc = std::max(o.k_cert, 2);
    const int kmax = std::max(o.k, kc);
    o.step.tau_F = o.tau_F;
    StepArgs a;
    if (!fill_step_args(p, &o.step, o.k_reflect, &a)) return MOTO_EINVAL;
    const DrvLayout L = drv_layout(p, hvp, o.step.mem, kmax, o.eig.guard);
    if (!ws || ws_bytes < L.total) return MOTO_EWORKSPACE;
    char* w = (char*)ws;
    hipStream_t st = (hipStream_t)stream;
    const int N = p->g.N;
    double* F = (double*)(w + L.F);
    double* out = (double*)(w + L.out);
    double* part = (double*)(w + L.epart);
    double* V = (double*)(w + L.V);
    double* ev = (double*)(w + L.ev);
    double* c64 = (double*)(w + L.eig) ;  // scratch only before the first eigen call (not used)
    (void)c64;
    HIP_TRY(hipMemsetAsync(w + L.state, 0, step_state_bytes(N, o.step.mem), st));
    HIP_TRY(hipMemsetAsync(out, 0, sizeof(double) * 2, st));
    const double tau_lam = o.tau_lam > 0.0 ? o.tau_lam : (hvp == MOTO_F64 ? 1e-6 : 1e-4) * p->hest;
    int it = 0;
    int64_t n_hvp = 0;
    double ho[2] = {INFINITY, 0.0};
    bool nan = false;
    for (it = 0; it <= o.max_outer; ++it) {
        HIP_TRY(launch_energy_grad(p->g, p->k, true, 1, m, mask, nullptr, nullptr, F, part, st));
        moto_eig_opts eo = o.eig;
        eo.warm = it == 0 ? 0 : 2;
        eo.flags = 0;  // the driver reads the outcome on the host
        moto_info inf;
        moto_status rs = min_modes_impl(p, hvp, m, mask, o.k, &eo, ev, V, nullptr, &inf, w + L.eig,
                                        ws_bytes - L.eig, st, nullptr);
        if (rs != MOTO_OK) return rs;
        n_hvp += inf.n_hvp;
        if (inf.status == MOTO_NAN) {
            nan = true;
            break;
        }
        if (it == o.max_outer) {
            // last iterate: evaluate ||F_mmf|| without moving (tau = +inf)
            StepArgs a2 = a;
            a2.tau_F = INFINITY;
            HIP_TRY(launch_step(a2, m, F, V, w + L.state, out, st));
        } else {
            HIP_TRY(launch_step(a, m, F, V, w + L.state, out, st));
        }
        rs = readback(p, out, sizeof(ho), ho, st);
        if (rs != MOTO_OK) return rs;
        if (ho[1] != 0.0 || !std::isfinite(ho[0])) break;
    }
    // certification at the final point
    moto_eig_opts eo = o.eig;
    eo.warm = 0;
    eo.seed = o.eig.seed + 1;
    eo.flags = 0;
    moto_info inf;
    moto_status rs = min_modes_impl(p, hvp, m, mask, kc, &eo, ev, V, nullptr, &inf, w + L.eig, ws_bytes - L.eig,
                                    st, nullptr);
    if (rs != MOTO_OK) return rs;
    n_hvp += inf.n_hvp;
    HIP_TRY(launch_energy_grad(p->g, p->k, true, 1, m, mask, nullptr, nullptr, F, part, st));
    HIP_TRY(launch_reduce_partials(part, 1, p->g.tiles, p->ns, out + 2, nullptr, st));
    double hv[3];
    rs = readback(p, out + 2, sizeof(double), hv, st);
    if (rs != MOTO_OK) return rs;
    double lam[2];
    rs = readback(p, ev, sizeof(lam), lam, st);
    if (rs != MOTO_OK) return rs;
    int status;
    const bool conv = std::isfinite(ho[0]) && ho[0] <= o.tau_F;
    if (nan || !std::isfinite(ho[0]) || !std::isfinite(lam[0]) || !std::isfinite(lam[1]) || inf.status == MOTO_NAN)
        status = MOTO_NAN;
    else if (!conv || inf.status != MOTO_CONVERGED)
        // an unconverged certifying solve only bounds the eigenvalues from
        // above: no SADDLE / HIGHER_INDEX verdict from it
        status = MOTO_NOT_CONVERGED;
    else if (lam[0] < -tau_lam && lam[1] > tau_lam)
        status = MOTO_SADDLE;
    else if (lam[1] < -tau_lam)
        status = MOTO_HIGHER_INDEX;
    else
        status = MOTO_DEGENERATE;
    {
        int hdr[5];
        rs = readback(p, w + L.state, sizeof(hdr), hdr, st);
        if (rs != MOTO_OK) return rs;
        res->iters = hdr[4];
    }
    res->status = status;
    res->n_hvp = n_hvp;
    res->E = hv[0];
    res->fnorm = ho[0];
    res->lambda1 = lam[0];
    res->lambda2 = lam[1];
    if (evals_out) HIP_TRY(hipMemcpyAsync(evals_out, ev, sizeof(double) * kc, hipMemcpyDeviceToDevice, st));
    if (V_out) HIP_TRY(hipMemcpyAsync(V_out, V, sizeof(double) * 3 * (size_t)N * kc, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return MOTO_OK;
}

// ---------------------------------------------------------------------------
// Searches over a population (lock step)
// ---------------------------------------------------------------------------
namespace {
// [energy partials P][F P 3N][out P x 2][step states P][eig population ws]
// [V P kmax 3N][evals P kmax][E P][info P]
struct PopSearchLayout {
    size_t epart, F, out, state, eig, V, ev, E, total;
    size_t state_b;
};

PopSearchLayout pop_search_layout(moto_plan p, moto_dtype hvp, int P, int mem, int kmax, int guard) {
    PopSearchLayout L;
    const size_t N = p->g.N, Pz = (size_t)P;
    size_t o = 0;
    L.epart = o;
    o += energy_ws(p, P);
    L.F = o;
    o += al(sizeof(double) * 3 * N * Pz);
    L.out = o;
    o += al(sizeof(double) * 2 * Pz);
    L.state_b = al(step_state_bytes((int)N, mem));
    L.state = o;
    o += L.state_b * Pz;
    L.eig = o;
    o += al(eig_layout(p, hvp, kmax, resolve_guard(kmax, guard), P).total);
    L.V = o;
    o += al(sizeof(double) * 3 * N * (size_t)kmax * Pz);
    L.ev = o;
    o += al(sizeof(double) * (size_t)kmax * Pz);
    L.E = o;
    o += al(sizeof(double) * Pz);
    L.total = o;
    return L;
}

bool pop_search_opts_ok(const moto_search_opts& o) {
    return o.k >= 1 && o.k_reflect >= 0 && o.k_reflect <= o.k && o.k_reflect <= 4 && o.max_outer >= 0 &&
           std::max(o.k, std::max(o.k_cert, 2)) + resolve_guard(std::max(o.k, std::max(o.k_cert, 2)), o.eig.guard) <=
               MAXB;
}
}  // namespace

size_t moto_saddle_search_population_workspace(moto_plan p, moto_dtype hvp, int32_t P, const moto_search_opts* opts) {
    if (!p || !hvp_ok(hvp) || P < 1 || P > MOTO_MAX_POPULATION) return 0;
    moto_search_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_search_opts(hvp, &o);
    if (!pop_search_opts_ok(o) || o.step.mem < 1 || o.step.mem > 16) return 0;
    const int kmax = std::max(o.k, std::max(o.k_cert, 2));
    return pop_search_layout(p, hvp, P, o.step.mem, kmax, o.eig.guard).total;
}

moto_status moto_saddle_search_population(moto_plan p, moto_dtype hvp, int32_t P, double* m, const uint8_t* mask,
                                          const moto_search_opts* opts, moto_search_result* res, double* evals_out,
                                          double* V_out, void* ws, size_t ws_bytes, moto_stream stream) {
    if (!p || !m || !res || !hvp_ok(hvp) || P < 1 || P > MOTO_MAX_POPULATION) return MOTO_EINVAL;
    moto_search_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_search_opts(hvp, &o);
    if (!pop_search_opts_ok(o)) return MOTO_EINVAL;
    const int kc = std::max(o.k_cert, 2);
    const int kmax = std::max(o.k, kc);
    o.step.tau_F = o.tau_F;
    StepArgs a;
    if (!fill_step_args(p, &o.step, o.k_reflect, &a)) return MOTO_EINVAL;
    const PopSearchLayout L = pop_search_layout(p, hvp, P, o.step.mem, kmax, o.eig.guard);
    if (!ws || ws_bytes < L.total) return MOTO_EWORKSPACE;
    char* w = (char*)ws;
    hipStream_t st = (hipStream_t)stream;
    const size_t N = p->g.N, N3 = 3 * N;
    double* F = (double*)(w + L.F);
    double* out = (double*)(w + L.out);
    double* part = (double*)(w + L.epart);
    double* V = (double*)(w + L.V);
    double* ev = (double*)(w + L.ev);
    double* E = (double*)(w + L.E);
    char* eigw = w + L.eig;
    const size_t eig_bytes = L.V - L.eig;
    HIP_TRY(hipMemsetAsync(w + L.state, 0, L.state_b * (size_t)P, st));
    HIP_TRY(hipMemsetAsync(out, 0, sizeof(double) * 2 * (size_t)P, st));
    const double tau_lam = o.tau_lam > 0.0 ? o.tau_lam : (hvp == MOTO_F64 ? 1e-6 : 1e-4) * p->hest;
    std::vector<int> done(P, 0), iters(P, 0), nanm(P, 0);
    std::vector<double> ho(2 * (size_t)P, 0.0), fnorm(P, INFINITY);
    std::vector<long long> n_hvp(P, 0);
    std::vector<moto_info> inf(P);
    for (int it = 0; it <= o.max_outer; ++it) {
        HIP_TRY(launch_energy_grad(p->g, p->k, true, P, m, mask, nullptr, nullptr, F, part, st));
        moto_eig_opts eo = o.eig;
        eo.warm = it == 0 ? 0 : 2;
        eo.flags = 0;  // the driver reads the outcome on the host
        moto_status rs = min_modes_pop_impl(p, hvp, P, m, mask, o.k, &eo, ev, V, nullptr, inf.data(), eigw,
                                            eig_bytes, st, nullptr);
        if (rs != MOTO_OK) return rs;
        int active = 0;
        for (int y = 0; y < P; ++y) {
            if (done[y]) continue;
            n_hvp[y] += inf[y].n_hvp;
            if (inf[y].status == MOTO_NAN) {
                nanm[y] = 1;
                done[y] = 1;
                // its state stops it: the population step below leaves it alone
                HIP_TRY(launch_step_stop(w + L.state, (int)N, a.mem, L.state_b, y, st));
                continue;
            }
            ++active;
        }
        if (active == 0) break;
        {
            // every member in one set of launches; members that met tau_F or
            // failed are stopped in their step state and left alone
            StepArgs ay = a;
            if (it == o.max_outer) ay.tau_F = INFINITY;  // last iterate: ||F_mmf|| without moving
            HIP_TRY(launch_step_population(ay, P, o.k, m, F, V, w + L.state, L.state_b, out, st));
        }
        rs = readback(p, out, sizeof(double) * 2 * (size_t)P, ho.data(), st);
        if (rs != MOTO_OK) return rs;
        int left = 0;
        for (int y = 0; y < P; ++y) {
            if (done[y]) continue;
            fnorm[y] = ho[2 * y];
            if (ho[2 * y + 1] != 0.0 || !std::isfinite(ho[2 * y])) done[y] = 1;
            else ++left;
        }
        if (left == 0) break;
    }
    // certification of every member at its final point
    moto_eig_opts eo = o.eig;
    eo.warm = 0;
    eo.seed = o.eig.seed + 1;
    eo.flags = 0;
    moto_status rs = min_modes_pop_impl(p, hvp, P, m, mask, kc, &eo, ev, V, nullptr, inf.data(), eigw, eig_bytes, st,
                                        nullptr);
    if (rs != MOTO_OK) return rs;
    HIP_TRY(launch_energy_grad(p->g, p->k, true, P, m, mask, nullptr, nullptr, F, part, st));
    HIP_TRY(launch_reduce_partials(part, P, p->g.tiles, p->ns, E, nullptr, st));
    std::vector<double> hE(P), hev((size_t)P * kc);
    rs = readback(p, E, sizeof(double) * (size_t)P, hE.data(), st);
    if (rs != MOTO_OK) return rs;
    const int cap = 4096 / (int)(sizeof(double) * kc);  // members per read-back of the pinned buffer
    for (int y0 = 0; y0 < P; y0 += cap) {
        const int ny = std::min(P - y0, cap);
        rs = readback(p, ev + (size_t)y0 * kc, sizeof(double) * kc * (size_t)ny, hev.data() + (size_t)y0 * kc, st);
        if (rs != MOTO_OK) return rs;
    }
    for (int y = 0; y < P; ++y) {
        int hdr[5];
        rs = readback(p, w + L.state + L.state_b * (size_t)y, sizeof(hdr), hdr, st);
        if (rs != MOTO_OK) return rs;
        iters[y] = hdr[4];
        const double l1 = hev[(size_t)y * kc], l2 = hev[(size_t)y * kc + 1];
        const bool conv = std::isfinite(fnorm[y]) && fnorm[y] <= o.tau_F;
        int status;
        if (nanm[y] || !std::isfinite(fnorm[y]) || !std::isfinite(l1) || !std::isfinite(l2) ||
            inf[y].status == MOTO_NAN)
            status = MOTO_NAN;
        else if (!conv || inf[y].status != MOTO_CONVERGED)
            status = MOTO_NOT_CONVERGED;
        else if (l1 < -tau_lam && l2 > tau_lam)
            status = MOTO_SADDLE;
        else if (l2 < -tau_lam)
            status = MOTO_HIGHER_INDEX;
        else
            status = MOTO_DEGENERATE;
        res[y].status = status;
        res[y].iters = iters[y];
        res[y].n_hvp = n_hvp[y] + inf[y].n_hvp;
        res[y].E = hE[y];
        res[y].fnorm = fnorm[y];
        res[y].lambda1 = l1;
        res[y].lambda2 = l2;
    }
    if (evals_out) HIP_TRY(hipMemcpyAsync(evals_out, ev, sizeof(double) * kc * (size_t)P, hipMemcpyDeviceToDevice, st));
    if (V_out) HIP_TRY(hipMemcpyAsync(V_out, V, sizeof(double) * N3 * kc * (size_t)P, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return MOTO_OK;
}

// ---------------------------------------------------------------------------
// Batched searches (one persistent launch)
// ---------------------------------------------------------------------------
static moto_status check_ham(const moto_hamiltonian* h, bool need_size) {
    if (!h) return MOTO_EINVAL;
    if (need_size && (h->Lx < 1 || h->Ly < 1)) return MOTO_EINVAL;
    if (h->n_shells < 1 || h->n_shells > MOTO_MAX_SHELLS || h->reserved != 0) return MOTO_EINVAL;
    for (int s = 0; s < MOTO_MAX_SHELLS; ++s) {
        if (!std::isfinite(h->J[s]) || !std::isfinite(h->D[s])) return MOTO_EINVAL;
        if (s >= 3 && s < h->n_shells && h->J[s] != 0.0) return MOTO_EUNSUPPORTED;
        if (s >= 1 && h->D[s] != 0.0) return MOTO_EUNSUPPORTED;
    }
    if (h->n_shells > 3) return MOTO_EUNSUPPORTED;
    return MOTO_OK;
}

struct BatchHostLayout {
    size_t Ls, tiles, order, moff, woff, res0, total;
    std::vector<long long> m_off, ws_off;
};

static bool batch_layout_host(int32_t n, const int32_t* L, int mem, BatchHostLayout* o) {
    size_t p = 0;
    o->Ls = p;
    p += al(sizeof(int) * (size_t)n);
    o->tiles = p;
    p += al(sizeof(int) * (size_t)n);
    o->order = p;
    p += al(sizeof(int) * (size_t)n);
    o->moff = p;
    p += al(sizeof(long long) * (size_t)n);
    o->woff = p;
    p += al(sizeof(long long) * (size_t)n);
    o->res0 = p;
    o->m_off.resize(n);
    o->ws_off.resize(n);
    long long mo = 0;
    for (int i = 0; i < n; ++i) {
        if (L[i] < 5 || L[i] > 4096) return false;
        o->m_off[i] = mo;
        mo += 3LL * L[i] * L[i];
        o->ws_off[i] = (long long)(p - o->res0);
        p += al(batch_search_bytes(L[i] * L[i], mem));
    }
    o->total = p;
    return true;
}

size_t moto_saddle_search_batched_workspace(int32_t n, const int32_t* L, const moto_search_opts* o) {
    if (n < 1 || !L) return 0;
    moto_search_opts d;
    if (o)
        d = *o;
    else
        moto_default_search_opts(MOTO_F32, &d);
    if (d.step.mem < 1 || d.step.mem > 16) return 0;
    BatchHostLayout bl;
    if (!batch_layout_host(n, L, d.step.mem, &bl)) return 0;
    return bl.total;
}

// the batched launch with explicit tile shapes; ev0 / ev1 (optional) are
// recorded around the kernel alone
static moto_status batched_impl(const moto_hamiltonian* h, int32_t n, const int32_t* L, double* m_all,
                                const uint8_t* mask_all, const int32_t* tiles, const moto_search_opts* opts,
                                moto_search_result* res, void* ws, size_t ws_bytes, hipStream_t st,
                                hipEvent_t ev0, hipEvent_t ev1) {
    moto_status cs = check_ham(h, false);
    if (cs != MOTO_OK) return cs;
    if (n < 1 || !L || !m_all || !res) return MOTO_EINVAL;
    moto_search_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_search_opts(MOTO_F32, &o);
    if (o.k < 1 || o.k > 2 || o.k_cert > 2 || o.k_reflect != 1 || o.max_outer < 0 || o.step.rule != 0 ||
        o.step.mem < 1 || o.step.mem > 16 || !(o.step.theta_max > 0.0) || o.eig.max_iter < 0)
        return MOTO_EINVAL;
    std::vector<int> tl(n, MOTO_TILE_32x8);
    if (tiles)
        for (int i = 0; i < n; ++i) {
            if (tiles[i] < MOTO_TILE_32x8 || tiles[i] > MOTO_TILE_64x4) return MOTO_EINVAL;
            tl[i] = tiles[i];
        }
    BatchHostLayout bl;
    if (!batch_layout_host(n, L, o.step.mem, &bl)) return MOTO_EINVAL;
    if (!ws || ws_bytes < bl.total) return MOTO_EWORKSPACE;
    // largest lattices first
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return L[a] > L[b]; });
    char* w = (char*)ws;
    HIP_TRY(hipMemcpyAsync(w + bl.Ls, L, sizeof(int) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + bl.tiles, tl.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + bl.order, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + bl.moff, bl.m_off.data(), sizeof(long long) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + bl.woff, bl.ws_off.data(), sizeof(long long) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));  // the host descriptor arrays are local
    double sj = 0.0, sd = 0.0;
    for (int s = 0; s < h->n_shells; ++s) {
        sj += 6.0 * std::fabs(h->J[s]);
        sd += 6.0 * std::fabs(h->D[s]);
    }
    const double hest = 4.0 * (sj + sd) + 4.0 * std::fabs(h->K) +
                        std::sqrt(h->B[0] * h->B[0] + h->B[1] * h->B[1] + h->B[2] * h->B[2]);
    BatchArgs a;
    for (int s = 0; s < 3; ++s) a.k.cJ[s] = s < h->n_shells ? -2.0 * h->J[s] : 0.0;
    a.k.cD = 2.0 * h->D[0];
    a.k.cK = -2.0 * h->K;
    for (int c = 0; c < 3; ++c) a.k.B[c] = h->B[c];
    a.hest = hest;
    a.tau_F = o.tau_F;
    a.tau_lam = o.tau_lam > 0.0 ? o.tau_lam : 1e-4 * hest;
    a.theta_max = o.step.theta_max;
    a.alpha0 = o.step.alpha0 > 0.0 ? o.step.alpha0 : 1.0 / hest;
    a.sy_min = o.step.sy_min;
    a.eig_tol_abs = o.eig.tol * hest;
    a.drop = 1e-9;
    a.kk = o.k;
    a.k_cert = 2;
    a.mem = o.step.mem;
    a.max_outer = o.max_outer;
    a.eig_max_iter = o.eig.max_iter;
    a.n = n;
    a.seed = o.eig.seed;
    if (ev0) HIP_TRY(hipEventRecord(ev0, st));
    HIP_TRY(launch_batched_search(a, m_all, mask_all, (const int*)(w + bl.Ls), (const int*)(w + bl.tiles),
                                  (const int*)(w + bl.order), (const long long*)(w + bl.moff),
                                  (const long long*)(w + bl.woff), w + bl.res0, res, n, st));
    if (ev1) HIP_TRY(hipEventRecord(ev1, st));
    return MOTO_OK;
}

moto_status moto_saddle_search_batched(const moto_hamiltonian* h, int32_t n, const int32_t* L, double* m_all,
                                       const uint8_t* mask_all, const int32_t* tiles, const moto_search_opts* opts,
                                       moto_search_result* res, void* ws, size_t ws_bytes, moto_stream stream) {
    return batched_impl(h, n, L, m_all, mask_all, tiles, opts, res, ws, ws_bytes, (hipStream_t)stream, nullptr,
                        nullptr);
}

// Autotuner of the batched searches' tile shapes, per lattice-size bucket
// (sides 8 apart): up to BATCH_TUNE_SAMPLE members of each bucket run
// BATCH_TUNE_STEPS outer steps from copies of their starts with every shape;
// the fastest kernel time wins for the whole bucket.
namespace {
constexpr int BATCH_TUNE_SAMPLE = 4;
constexpr int BATCH_TUNE_STEPS = 2;
constexpr int BATCH_TUNE_BUCKET = 8;
size_t batch_tune_extra(int32_t n, const int32_t* L) {
    size_t m = 0, k = 0;
    for (int i = 0; i < n; ++i) {
        m += 3ull * L[i] * L[i];
        k += (size_t)L[i] * L[i];
    }
    return al(sizeof(double) * m) + al(k) + al(sizeof(moto_search_result) * (size_t)n);
}
}  // namespace

size_t moto_saddle_search_batched_autotune_workspace(int32_t n, const int32_t* L, const moto_search_opts* o) {
    const size_t b = moto_saddle_search_batched_workspace(n, L, o);
    return b == 0 ? 0 : b + batch_tune_extra(n, L);
}

moto_status moto_saddle_search_batched_autotune(const moto_hamiltonian* h, int32_t n, const int32_t* L,
                                                const double* m_all, const uint8_t* mask_all,
                                                const moto_search_opts* opts, int32_t* tiles, void* ws,
                                                size_t ws_bytes, moto_stream stream) {
    if (!h || n < 1 || !L || !m_all || !tiles) return MOTO_EINVAL;
    const size_t base = moto_saddle_search_batched_workspace(n, L, opts);
    if (base == 0) return MOTO_EINVAL;
    if (!ws || ws_bytes < base + batch_tune_extra(n, L)) return MOTO_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    moto_search_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_search_opts(MOTO_F32, &o);
    o.max_outer = BATCH_TUNE_STEPS;
    std::vector<long long> off(n);
    long long acc = 0;
    for (int i = 0; i < n; ++i) {
        off[i] = acc;
        acc += 3LL * L[i] * L[i];
    }
    char* w = (char*)ws;
    double* mcopy = (double*)(w + base);
    uint8_t* kcopy = (uint8_t*)(w + base + al(sizeof(double) * (size_t)acc));
    moto_search_result* rcopy = (moto_search_result*)(w + base + al(sizeof(double) * (size_t)acc) + al((size_t)acc / 3));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MOTO_EHIP;
    }
    moto_status rs = MOTO_OK;
    for (int i = 0; i < n; ++i) tiles[i] = MOTO_TILE_32x8;
    int maxb = 0;
    for (int i = 0; i < n; ++i) maxb = std::max(maxb, L[i] / BATCH_TUNE_BUCKET);
    for (int bk = 0; bk <= maxb && rs == MOTO_OK; ++bk) {
        std::vector<int> mem;
        for (int i = 0; i < n; ++i)
            if (L[i] / BATCH_TUNE_BUCKET == bk) mem.push_back(i);
        if (mem.empty()) continue;
        const int ns = std::min((int)mem.size(), BATCH_TUNE_SAMPLE);
        std::vector<int32_t> Ls(ns), tl(ns);
        for (int q = 0; q < ns; ++q) Ls[q] = L[mem[q]];
        float best = 0.0f;
        int best_tile = MOTO_TILE_32x8;
        for (int t = MOTO_TILE_32x8; t <= MOTO_TILE_64x4 && rs == MOTO_OK; ++t) {
            // fresh copies of the sampled starts (the search moves them)
            long long o2 = 0;
            for (int q = 0; q < ns; ++q) {
                const size_t nn = 3ull * Ls[q] * Ls[q];
                if (hipMemcpyAsync(mcopy + o2, m_all + off[mem[q]], sizeof(double) * nn, hipMemcpyDeviceToDevice,
                                   st) != hipSuccess ||
                    (mask_all && hipMemcpyAsync(kcopy + o2 / 3, mask_all + off[mem[q]] / 3, nn / 3,
                                                hipMemcpyDeviceToDevice, st) != hipSuccess)) {
                    rs = MOTO_EHIP;
                    break;
                }
                o2 += (long long)nn;
            }
            if (rs != MOTO_OK) break;
            for (int q = 0; q < ns; ++q) tl[q] = t;
            rs = batched_impl(h, ns, Ls.data(), mcopy, mask_all ? kcopy : nullptr, tl.data(), &o, rcopy, ws, base, st,
                              e0, e1);
            if (rs != MOTO_OK) break;
            float ms = 0.0f;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rs = MOTO_EHIP;
                break;
            }
            if (t == MOTO_TILE_32x8 || ms < best) {
                best = ms;
                best_tile = t;
            }
        }
        for (int i : mem) tiles[i] = best_tile;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rs;
}

// ---------------------------------------------------------------------------
// Explorer objectives
// ---------------------------------------------------------------------------
void moto_default_explorer_opts(moto_dtype hvp, moto_explorer_opts* o) {
    if (!o) return;
    o->k = 2;
    o->reserved = 0;
    o->Q_target = std::nan("");
    moto_default_eig_opts(hvp, &o->eig);
}

namespace {
// [eig population ws][mask copies P N][c P N][energy / charge partials]
// [E P][Q P + 1][evals P k][V P k 3N][l1 partials][D P (P + A)]
struct ExpLayout {
    size_t eig, mask, c, part, E, Q, ev, V, l1, D, total;
};

ExpLayout exp_layout(moto_plan p, moto_dtype hvp, int P, int A, int k, int guard) {
    ExpLayout L;
    const size_t N = p->g.N, Pz = (size_t)P, Qz = (size_t)(P + A);
    size_t o = 0;
    L.eig = o;
    o += eig_layout(p, hvp, k, resolve_guard(k, guard), P).total;
    L.mask = o;
    o += al(Pz * N);
    L.c = o;
    o += al(sizeof(double) * Pz * N);
    L.part = o;
    o += energy_ws(p, P + 1);
    L.E = o;
    o += al(sizeof(double) * Pz);
    L.Q = o;
    o += al(sizeof(double) * (Pz + 1));
    L.ev = o;
    o += al(sizeof(double) * Pz * k);
    L.V = o;
    o += al(sizeof(double) * Pz * k * 3 * N);
    L.l1 = o;
    o += al(sizeof(double) * (size_t)l1_chunks(3LL * (long long)N) * Pz * Qz);
    L.D = o;
    o += al(sizeof(double) * Pz * Qz);
    L.total = o;
    return L;
}

bool explorer_args_ok(moto_plan p, moto_dtype hvp, int P, int A, const moto_explorer_opts& o) {
    if (!p || !hvp_ok(hvp) || P < 1 || P > MOTO_MAX_POPULATION || A < 0 || A > MOTO_MAX_ARCHIVE) return false;
    if (o.k < 2 || o.k + resolve_guard(o.k, o.eig.guard) > MAXB) return false;
    if (o.eig.max_iter < 0 || !(o.eig.tol >= 0.0) || o.eig.warm != 0) return false;
    return true;
}
}  // namespace

size_t moto_explorer_workspace(moto_plan p, moto_dtype hvp, int32_t P, int32_t n_archive,
                               const moto_explorer_opts* opts) {
    moto_explorer_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_explorer_opts(hvp, &o);
    if (!explorer_args_ok(p, hvp, P, n_archive, o)) return 0;
    return exp_layout(p, hvp, P, n_archive, o.k, o.eig.guard).total;
}

moto_status moto_explorer_objectives(moto_plan p, moto_dtype hvp, int32_t P, const double* x0, const uint8_t* mask,
                                     const double* delta, int32_t n_archive, const double* archive,
                                     const moto_explorer_opts* opts, double* x_out, moto_explorer_result* res,
                                     double* evals, double* V, double* D, void* ws, size_t ws_bytes,
                                     moto_stream stream) {
    moto_explorer_opts o;
    if (opts)
        o = *opts;
    else
        moto_default_explorer_opts(hvp, &o);
    if (!explorer_args_ok(p, hvp, P, n_archive, o)) return MOTO_EINVAL;
    if (!x0 || !delta || !x_out || !res || (n_archive > 0 && !archive)) return MOTO_EINVAL;
    const ExpLayout L = exp_layout(p, hvp, P, n_archive, o.k, o.eig.guard);
    if (!ws || ws_bytes < L.total) return MOTO_EWORKSPACE;
    char* w = (char*)ws;
    hipStream_t st = (hipStream_t)stream;
    const int N = p->g.N;
    const int k = o.k;
    uint8_t* mrep = mask ? (uint8_t*)(w + L.mask) : nullptr;
    double* c = (double*)(w + L.c);
    double* part = (double*)(w + L.part);
    double* E = (double*)(w + L.E);
    double* Qv = (double*)(w + L.Q);
    double* ev = evals ? evals : (double*)(w + L.ev);
    double* Vb = V ? V : (double*)(w + L.V);
    double* Db = D ? D : (double*)(w + L.D);
    // candidates (and one copy of the mask per candidate for the batched HVP)
    HIP_TRY(launch_candidates(N, P, x0, mask, delta, x_out, mrep, st));
    // energies and c = m . g of every candidate
    HIP_TRY(launch_energy_grad(p->g, p->k, true, P, x_out, nullptr, nullptr, c, nullptr, part, st));
    HIP_TRY(launch_reduce_partials(part, P, p->g.tiles, p->ns, E, nullptr, st));
    // topological charges of the candidates, then of x0
    HIP_TRY(launch_topo_charge(p->g, P, x_out, part, st));
    HIP_TRY(launch_reduce_partials(part, P, p->g.tiles, p->ns, Qv, nullptr, st));
    HIP_TRY(launch_topo_charge(p->g, 1, x0, part, st));
    HIP_TRY(launch_reduce_partials(part, 1, p->g.tiles, p->ns, Qv + P, nullptr, st));
    // l1 distances to S u A
    HIP_TRY(launch_l1(3LL * N, P, n_archive, x_out, archive, (double*)(w + L.l1), Db, st));
    // the k lowest modes of every candidate, in lock step
    moto_eig_opts eo = o.eig;
    eo.flags = 0;
    moto_status rs = min_modes_pop_impl(p, hvp, P, x_out, mrep, k, &eo, ev, Vb, nullptr, nullptr, w + L.eig,
                                        L.mask - L.eig, st, c);
    if (rs != MOTO_OK) return rs;
    const EigLayout EL = eig_layout(p, hvp, k, resolve_guard(k, o.eig.guard), P);
    const EigCtrl* ctrl = (const EigCtrl*)(w + L.eig + EL.ctrl);
    HIP_TRY(launch_explorer_finish(P, n_archive, k, Db, E, ev, Qv, Qv + P, o.Q_target, ctrl, res, st));
    return MOTO_OK;
}

}  // extern "C"

