// C ABI of libic.so (declared and documented in include/ic.h): argument
// checks, workspace layout, host<->device copies and the per-call launch
// sequence.  All device work is in ic_device.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "ic_internal.h"

namespace ic {

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int tiles(int n, int t) { return (n + t - 1) / t; }

}  // namespace

// Default z extent of a stage block.  Blocks run in rounds of `cap` resident
// blocks (three 512-thread blocks per compute unit in FP32, two in FP64, as
// LDS and registers allow); a block marches tz planes plus three halo
// planes.  The extent with the fewest rounds x planes wins (ties: the larger
// extent, fewer halo re-reads).  ic_set_tile overrides it.
int choose_tz(const ic_params &p) {
    const long cap = 256L * (p.prec == IC_FP64 ? 2 : 3);
    int best = 32;
    long best_cost = -1;
    for (int tz = 32; tz >= TZ_MIN; tz /= 2) {
        const long blocks = (long)tiles(p.nx, TX) * tiles(p.ny, TY) * tiles(p.nz, tz);
        const long cost = (blocks + cap - 1) / cap * ((tz < p.nz ? tz : p.nz) + 3);
        if (best_cost < 0 || cost < best_cost) {
            best = tz;
            best_cost = cost;
        }
    }
    return best;
}

int nblocks_total(const ic_params &p) {
    return tiles(p.nx, TX) * tiles(p.ny, TY) * tiles(p.nz, TZ_MIN);
}

int nblocks_of(const ic_ctx *c) { return c->nblk[0] * c->nblk[1] * c->nblk[2]; }

// Walks the workspace layout; with base == nullptr it only measures.
static size_t layout(const ic_params &p, char *base, Workspace *ws) {
    const size_t ncell = (size_t)p.nx * p.ny * p.nz;
    const size_t esz = p.prec == IC_FP64 ? 8 : 4;
    const size_t N = p.max_particles > 0 ? (size_t)p.max_particles : 1;
    const size_t nblk = (size_t)nblocks_total(p);
    const int pmax = p.nx > p.ny ? (p.nx > p.nz ? p.nx : p.nz) : (p.ny > p.nz ? p.ny : p.nz);
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *ptr = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return ptr;
    };
    Workspace w{};
    for (int i = 0; i < 4; ++i) w.A[i] = take(ncell * esz);
    for (int i = 0; i < 4; ++i) w.B[i] = take(ncell * esz);
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 9; ++i) w.N[k][i] = p.kT > 0.0 ? take(ncell * esz) : nullptr;
    auto d3 = [&]() { return (double *)take(3 * N * sizeof(double)); };
    auto d1 = [&]() { return (double *)take(N * sizeof(double)); };
    w.q = d3(); w.u = d3(); w.me = d1(); w.eps = d1(); w.ks = d1(); w.qeq = d3(); w.fext = d3();
    w.qh = d3(); w.jv_old = d3(); w.F = d3(); w.Vt = d3(); w.du = d3(); w.mf = d3();
    w.omega = (double *)take(2 * N * sizeof(double)); w.jv_new = d3();   // two stages' Omega
    w.pk.bc = (int32_t *)take(3 * N * sizeof(int32_t));
    w.pk.bf = (int32_t *)take(3 * N * sizeof(int32_t));
    w.pk.wc = (double *)take(9 * N * sizeof(double));
    w.pk.wf = (double *)take(9 * N * sizeof(double));
    w.blk_count = (int32_t *)take((nblk + 1) * sizeof(int32_t));
    w.blk_off = (int32_t *)take((nblk + 1) * sizeof(int32_t));
    w.blk_cursor = (int32_t *)take((nblk + 1) * sizeof(int32_t));
    w.blk_list = (int32_t *)take(N * MAX_BLOCKS_PER_PARTICLE * sizeof(int32_t));
    w.blk_key = (int32_t *)take(N * MAX_BLOCKS_PER_PARTICLE * sizeof(int32_t));
    auto i1 = [&]() { return (int32_t *)take(N * sizeof(int32_t)); };
    w.cl_parent = i1(); w.cl_root = i1(); w.cl_cnt = i1();
    w.cl_off = (int32_t *)take((N + 1) * sizeof(int32_t));
    w.cl_cursor = i1(); w.cl_list = i1();
    w.sum_f = d3(); w.sum_l = d3();
    w.prof = (double *)take((size_t)IC_MAX_MODES * pmax * sizeof(double));
    w.red = (double *)take(4 * 1024 * sizeof(double));
    w.flag = (int32_t *)take(sizeof(int32_t) * 4);
    w.st = (StepState *)take(sizeof(StepState));
    if (ws) *ws = w;
    return off;
}

size_t workspace_bytes(const ic_params &p, size_t *) { return layout(p, nullptr, nullptr); }

static size_t adj_layout(const ic_params &p, char *base, AdjWorkspace *aw) {
    const size_t ncell = (size_t)p.nx * p.ny * p.nz;
    const size_t esz = p.prec == IC_FP64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *ptr = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return ptr;
    };
    AdjWorkspace w{};
    for (int i = 0; i < 4; ++i) w.L2[i] = take(ncell * esz);
    for (int i = 0; i < 4; ++i) w.L1[i] = take(ncell * esz);
    for (int i = 0; i < 4; ++i) w.acc[i] = take(ncell * esz);
    for (int i = 0; i < 3; ++i) w.murf[i] = take(ncell * esz);
    w.mur = take(ncell * esz);
    w.partial = (double *)take((size_t)IC_MAX_MODES * adjoint_blocks(p) * sizeof(double));
    const size_t N = (size_t)(p.max_particles > 0 ? p.max_particles : 0);
    auto d3 = [&]() { return (double *)take(3 * N * sizeof(double)); };
    auto d1 = [&]() { return (double *)take(N * sizeof(double)); };
    w.plqh = d3(); w.plF = d3(); w.plVt = d3(); w.plmf = d3();
    w.pdme = d1(); w.pdeps = d1(); w.pdks = d1();
    w.pq = d3();
    if (aw) *aw = w;
    return off;
}

size_t adjoint_workspace_bytes(const ic_params &p) { return adj_layout(p, nullptr, nullptr); }
void carve_adjoint(const ic_params &p, char *base, AdjWorkspace &aw) { adj_layout(p, base, &aw); }

void carve_workspace(const ic_params &p, char *base, Workspace &ws) { layout(p, base, &ws); }

hipEvent_t prof_event(ic_ctx *c) {
    if (!c->profiling) return nullptr;
    if (c->ev_pool.empty()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
}

void prof_push(ic_ctx *c, hipEvent_t a, hipEvent_t b) {
    if (a && b)
        c->ev_pending.emplace_back(a, b);
    else {
        if (a) c->ev_pool.push_back(a);
        if (b) c->ev_pool.push_back(b);
    }
}

}  // namespace ic

using namespace ic;

namespace {

int fail(ic_ctx *c, int code, const char *msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(ic_ctx *c, hipError_t e, const char *where) {
    if (c) {
        c->err = std::string(where) + ": " + hipGetErrorString(e);
    }
    return IC_E_HIP;
}

int check_params(const ic_params *p, ic_ctx *c) {
    if (!p) return fail(c, IC_E_ARG, "params is NULL");
    if (p->nx < 4 || p->ny < 4 || p->nz < 4)
        return fail(c, IC_E_ARG, "grid must have at least 4 cells per side");
    if ((double)p->nx * p->ny * p->nz > 2147483647.0)
        return fail(c, IC_E_ARG, "grid larger than 2^31 cells");
    if (p->prec != IC_FP32 && p->prec != IC_FP64) return fail(c, IC_E_ARG, "prec must be IC_FP32 or IC_FP64");
    // the stage kernel addresses a field with 32-bit byte offsets
    if ((double)p->nx * p->ny * p->nz * (p->prec == IC_FP64 ? 8.0 : 4.0) >= 4294967296.0)
        return fail(c, IC_E_ARG, "one field must be smaller than 4 GiB");
    if (!(p->h > 0) || !(p->rho0 > 0) || !(p->cf > 0) || !(p->dt > 0))
        return fail(c, IC_E_ARG, "h, rho0, cf and dt must be positive");
    if (!(p->eta >= 0) || !(p->zeta >= 0) || !(p->kT >= 0))
        return fail(c, IC_E_ARG, "eta, zeta and kT must be non-negative");
    if (!isfinite(p->h + p->rho0 + p->cf + p->dt + p->eta + p->zeta + p->kT))
        return fail(c, IC_E_ARG, "parameters must be finite");
    if (p->max_particles < 0) return fail(c, IC_E_ARG, "max_particles must be >= 0");
    if (p->cf * p->dt / p->h > 0.5) return fail(c, IC_E_UNSTABLE, "cf dt / h > 0.5");
    const double nu_l = (4.0 * p->eta / 3.0 + p->zeta) / p->rho0;
    if (nu_l * p->dt / (p->h * p->h) > 0.2)
        return fail(c, IC_E_UNSTABLE, "(4 eta/3 + zeta)/rho0 dt/h^2 > 0.2");
    return IC_OK;
}

int check_bound(ic_ctx *c) {
    if (!c) return IC_E_ARG;
    if (!c->bound) return fail(c, IC_E_STATE, "fields and workspace are not bound");
    return IC_OK;
}

// Device flags: [0] a step found m_e + m_f <= 0, [1] a reversed step got a
// non-finite particle position, [2] a step met a non-finite particle
// position, velocity or impulse (a NaN or inf in the fields or particles).
int take_flag(ic_ctx *c) {
    int32_t flag[3] = {0, 0, 0};
    hipError_t e = hipMemcpyAsync(flag, c->ws.flag, sizeof(flag), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "flag readback");
    if (flag[0] || flag[1] || flag[2]) {
        const int32_t zero[3] = {0, 0, 0};
        e = hipMemcpyAsync(c->ws.flag, zero, sizeof(zero), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "flag reset");
        if (flag[2])
            return fail(c, IC_E_ARG,
                        "non-finite state: a step met a non-finite particle position, velocity "
                        "or impulse (NaN or inf in the fields or particles)");
        if (flag[0]) return fail(c, IC_E_MASS, "a step found m_e + m_f <= 0");
        return fail(c, IC_E_ARG, "a reversed step got a non-finite particle position");
    }
    return IC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Ensembles: several contexts' steps captured into one HIP graph.
// ---------------------------------------------------------------------------
struct ic_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<ic_ctx *> ctxs;
    int64_t nsteps = 0;
    ic::Batch *batch = nullptr;   // batched steps' device tables (or none: one chain per context)
};


extern "C" {

// ic_step's graph: RUN_STEPS steps, each taking its noise from the step
// before and drawing the next one's, captured from the eager schedule on a
// private stream and replayed on the context stream.  Everything the
// captured launches bake in is in the signature; a change recaptures.
static const int64_t RUN_STEPS = 4;

static std::vector<char> run_signature(const ic_ctx *c) {
    std::vector<char> s;
    auto put = [&s](const void *p, size_t n) {
        s.insert(s.end(), (const char *)p, (const char *)p + n);
    };
    put(&c->np, sizeof c->np);
    put(&c->tz, sizeof c->tz);
    put(c->nblk, sizeof c->nblk);
    put(c->f, sizeof c->f);
    put(&c->ws, sizeof c->ws);
    put(&c->side, sizeof c->side);
    put(&c->forcing.nmodes, sizeof c->forcing.nmodes);
    put(c->forcing.modes, sizeof(ic_mode) * (size_t)c->forcing.nmodes);
    return s;
}

static void drop_run_graph(ic_ctx *c) {
    if (c->run_exec) (void)hipGraphExecDestroy(c->run_exec);
    if (c->run_graph) (void)hipGraphDestroy(c->run_graph);
    c->run_exec = nullptr;
    c->run_graph = nullptr;
    c->run_sig.clear();
}

static hipError_t capture_run_graph(ic_ctx *c) {
    drop_run_graph(c);
    hipStream_t origin = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&origin, hipStreamNonBlocking);
    bool capturing = false;
    if (e == hipSuccess) {
        e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal);
        capturing = e == hipSuccess;
    }
    const hipStream_t own = c->stream;
    c->stream = origin;
    for (int64_t s = 0; s < RUN_STEPS && e == hipSuccess; ++s) e = launch_step(c, true, false, false);
    c->stream = own;
    if (capturing) {
        const hipError_t e2 = hipStreamEndCapture(origin, &c->run_graph);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&c->run_exec, c->run_graph, nullptr, nullptr, 0);
    if (origin) (void)hipStreamDestroy(origin);
    if (e == hipSuccess)
        c->run_sig = run_signature(c);
    else
        drop_run_graph(c);
    return e;
}

int ic_create(const ic_params *p, void *stream, ic_ctx **out) {
    if (!out) return IC_E_ARG;
    *out = nullptr;
    const int rc = check_params(p, nullptr);
    if (rc != IC_OK) return rc;
    ic_ctx *c = new (std::nothrow) ic_ctx();
    if (!c) return IC_E_ARG;
    c->p = *p;
    c->stream = (hipStream_t)stream;
    c->device = 0;
    (void)hipGetDevice(&c->device);
    c->ncu = 0;
    if (hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess ||
        c->ncu <= 0)
        c->ncu = 256;
    c->bound = false;
    c->adj_bound = false;
    c->np = 0;
    c->step = 0;
    c->nsamples = 0;
    c->forcing.nmodes = 0;
    c->tz = choose_tz(*p);
    c->nblk[0] = (p->nx + TX - 1) / TX;
    c->nblk[1] = (p->ny + TY - 1) / TY;
    c->nblk[2] = (p->nz + c->tz - 1) / c->tz;
    int pmax = p->nx > p->ny ? p->nx : p->ny;
    if (p->nz > pmax) pmax = p->nz;
    c->prof_stride = pmax;
    c->profiling = false;
    c->prof_ms = 0.0;
    c->prof_launches = 0;
    c->side = nullptr;
    c->ev_fork = c->ev_part = c->ev_noise = nullptr;
    c->run_graph = nullptr;
    c->run_exec = nullptr;
    c->noise_ready = -1;
    *out = c;
    return IC_OK;
}

int ic_destroy(ic_ctx *c) {
    if (!c) return IC_OK;
    if (c->run_exec) (void)hipStreamSynchronize(c->stream);
    drop_run_graph(c);
    if (!c->ev_pending.empty()) (void)hipStreamSynchronize(c->stream);
    for (auto &pr : c->ev_pending) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    for (hipEvent_t e : {c->ev_fork, c->ev_part, c->ev_noise})
        if (e) (void)hipEventDestroy(e);
    delete c;
    return IC_OK;
}

int ic_profile(ic_ctx *c, int32_t enable) {
    if (!c) return IC_E_ARG;
    c->profiling = enable != 0;
    return IC_OK;
}

int ic_profile_read(ic_ctx *c, double *stage_ms, int64_t *launches) {
    if (!c) return IC_E_ARG;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "profile sync");
    for (auto &pr : c->ev_pending) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, pr.first, pr.second);
        if (e != hipSuccess) return hip_fail(c, e, "profile elapsed");
        c->prof_ms += ms;
        c->prof_launches += 1;
        c->ev_pool.push_back(pr.first);
        c->ev_pool.push_back(pr.second);
    }
    c->ev_pending.clear();
    if (stage_ms) *stage_ms = c->prof_ms;
    if (launches) *launches = c->prof_launches;
    c->prof_ms = 0.0;
    c->prof_launches = 0;
    return IC_OK;
}

int ic_workspace_size(const ic_params *p, size_t *bytes) {
    if (!bytes) return IC_E_ARG;
    const int rc = check_params(p, nullptr);
    if (rc != IC_OK) return rc;
    *bytes = workspace_bytes(*p);
    return IC_OK;
}

int ic_bind(ic_ctx *c, void *drho, void *gx, void *gy, void *gz, void *workspace,
            size_t workspace_bytes_) {
    if (!c) return IC_E_ARG;
    if (!drho || !gx || !gy || !gz || !workspace) return fail(c, IC_E_ARG, "NULL buffer");
    if (((uintptr_t)workspace & 255) != 0) return fail(c, IC_E_ARG, "workspace not 256-byte aligned");
    if (workspace_bytes_ < workspace_bytes(c->p)) return fail(c, IC_E_ARG, "workspace too small");
    if (!c->side) {
        // side stream and its events, created with the first binding
        hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_part, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_noise, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (c->side) (void)hipStreamDestroy(c->side);
            for (hipEvent_t *ev : {&c->ev_fork, &c->ev_part, &c->ev_noise}) {
                if (*ev) (void)hipEventDestroy(*ev);
                *ev = nullptr;
            }
            c->side = nullptr;
            return hip_fail(c, e, "bind: side stream");
        }
    }
    c->f[0] = drho;
    c->f[1] = gx;
    c->f[2] = gy;
    c->f[3] = gz;
    carve_workspace(c->p, (char *)workspace, c->ws);
    c->np = 0;
    c->nsamples = 0;
    c->forcing.nmodes = 0;
    hipError_t e = hipMemsetAsync(c->ws.flag, 0, 4 * sizeof(int32_t), c->stream);
    // binning counters start at zero; the scan kernel re-zeroes them after use
    if (e == hipSuccess)
        e = hipMemsetAsync(c->ws.blk_count, 0, (nblocks_total(c->p) + 1) * sizeof(int32_t), c->stream);
    if (e == hipSuccess) e = launch_set_step(c);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "bind");
    c->bound = true;
    c->noise_ready = -1;
    return IC_OK;
}

int ic_set_particles(ic_ctx *c, int32_t n, const double *q, const double *u, const double *me,
                     const double *eps, const double *ks, const double *qeq, const double *fext) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    if (n < 0) return fail(c, IC_E_ARG, "n < 0");
    if (n > c->p.max_particles) return fail(c, IC_E_CAPACITY, "n > max_particles");
    if (n > 0 && (!q || !me || !eps)) return fail(c, IC_E_ARG, "q, me and eps are required");
    const ic_params &p = c->p;
    const double V = 8.0 * p.h * p.h * p.h;
    const double L[3] = {p.nx * p.h, p.ny * p.h, p.nz * p.h};
    double max_eps = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a)
            if (!isfinite(q[3 * i + a])) return fail(c, IC_E_ARG, "non-finite position");
        if (!isfinite(me[i]) || !isfinite(eps[i])) return fail(c, IC_E_ARG, "non-finite particle property");
        if (!(me[i] + p.rho0 * V > 0.0)) return fail(c, IC_E_MASS, "particle mass m_e + rho0 V <= 0");
        if (!(p.cf * p.cf + eps[i] >= 0.0)) return fail(c, IC_E_MASS, "c_p^2 = cf^2 + eps < 0");
        if (eps[i] > max_eps) max_eps = eps[i];
    }
    if (sqrt(p.cf * p.cf + max_eps) * p.dt / p.h > 0.5)
        return fail(c, IC_E_UNSTABLE, "particle sound speed gives c dt / h > 0.5");
    std::vector<double> hq(3 * (size_t)n), hzero(3 * (size_t)n, 0.0), hks((size_t)n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double x = fmod(q[3 * i + a], L[a]);
            if (x < 0) x += L[a];
            if (x >= L[a]) x -= L[a];
            hq[3 * i + a] = x;
        }
    if (ks)
        for (int i = 0; i < n; ++i) hks[i] = ks[i];
    const Workspace &w = c->ws;
    const size_t b3 = 3 * (size_t)n * sizeof(double), b1 = (size_t)n * sizeof(double);
    hipError_t e = hipSuccess;
    auto cp = [&](void *dst, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
    };
    cp(w.q, hq.data(), b3);
    cp(w.me, me, b1);
    cp(w.eps, eps, b1);
    cp(w.ks, hks.data(), b1);
    cp(w.qeq, qeq ? qeq : hq.data(), b3);
    cp(w.fext, fext ? fext : hzero.data(), b3);
    cp(w.sum_f, hzero.data(), b3);
    cp(w.sum_l, hzero.data(), b3);
    if (u) cp(w.u, u, b3);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_particles copy");
    c->np = n;
    c->nsamples = 0;
    if (!u && n > 0) {
        e = launch_init_velocity(c);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "initial velocity");
    }
    return IC_OK;
}

int ic_get_particles(ic_ctx *c, double *q, double *u) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    const size_t b3 = 3 * (size_t)c->np * sizeof(double);
    hipError_t e = hipSuccess;
    if (q && b3) e = hipMemcpyAsync(q, c->ws.q, b3, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && u && b3) e = hipMemcpyAsync(u, c->ws.u, b3, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "get_particles");
    return take_flag(c);
}

int ic_set_forcing(ic_ctx *c, int32_t nmodes, const ic_mode *modes) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    if (nmodes < 0 || nmodes > IC_MAX_MODES) return fail(c, IC_E_ARG, "nmodes out of range");
    if (nmodes > 0 && !modes) return fail(c, IC_E_ARG, "modes is NULL");
    const ic_params &p = c->p;
    const int n_of[3] = {p.nx, p.ny, p.nz};
    std::vector<double> prof((size_t)IC_MAX_MODES * c->prof_stride, 0.0);
    for (int m = 0; m < nmodes; ++m) {
        const ic_mode &md = modes[m];
        if (md.axis < 0 || md.axis > 2) return fail(c, IC_E_ARG, "mode axis must be 0, 1 or 2");
        if (md.shape != IC_MODE_COS && md.shape != IC_MODE_PLANE) return fail(c, IC_E_ARG, "bad mode shape");
        if (!isfinite(md.x0 + md.amp + md.omega + md.phase)) return fail(c, IC_E_ARG, "non-finite mode");
        const int n = n_of[md.axis];
        double *pr = prof.data() + (size_t)m * c->prof_stride;
        if (md.shape == IC_MODE_PLANE) {
            long i0 = (long)floor(md.x0 / p.h + 0.5);
            i0 %= n;
            if (i0 < 0) i0 += n;
            pr[i0] = 1.0;
        } else {
            const double L = n * p.h;
            for (int i = 0; i < n; ++i) pr[i] = cos(2.0 * M_PI * md.m * (i * p.h - md.x0) / L);
        }
        c->forcing.modes[m] = md;
    }
    hipError_t e = hipMemcpyAsync(c->ws.prof, prof.data(), prof.size() * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_forcing");
    c->forcing.nmodes = nmodes;
    return IC_OK;
}

int ic_set_step(ic_ctx *c, int64_t n) {
    if (!c) return IC_E_ARG;
    if (n < 0) return fail(c, IC_E_ARG, "step must be >= 0");
    c->step = n;
    c->noise_ready = -1;
    if (c->bound) {
        hipError_t e = launch_set_step(c);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "set step");
    }
    return IC_OK;
}

int ic_set_tile(ic_ctx *c, int32_t tz) {
    if (!c) return IC_E_ARG;
    if (tz != 4 && tz != 8 && tz != 16 && tz != 32) return fail(c, IC_E_ARG, "tz must be 4, 8, 16 or 32");
    c->tz = tz;
    c->nblk[2] = (c->p.nz + tz - 1) / tz;
    return IC_OK;
}

int ic_get_tile(ic_ctx *c, int32_t *tz) {
    if (!c || !tz) return IC_E_ARG;
    *tz = c->tz;
    return IC_OK;
}

int ic_get_step(ic_ctx *c, int64_t *n) {
    if (!c || !n) return IC_E_ARG;
    *n = c->step;
    return IC_OK;
}

int ic_step(ic_ctx *c, int64_t nsteps) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    if (nsteps < 0) return fail(c, IC_E_ARG, "nsteps < 0");
    // The side stream pays for its event round trips only on large grids;
    // small grids are launch-latency-bound and step on one stream, drawing
    // each step's noise in line.  On large grids a step draws the next one's
    // noise in the background, except FP64 steps launched one by one (beside
    // FP64 stages launched from the host the FP64 noise kernel cost more
    // than it hid; inside the graph it hides).
    const bool overlap = (double)c->p.nx * c->p.ny * c->p.nz >= 1048576.0;
    const bool noise = c->p.kT > 0.0;
    const bool eager_ahead = c->p.prec != IC_FP64;
    hipError_t e = hipSuccess;
    auto one = [&](bool ahead) {
        const bool first = !(noise && c->noise_ready == c->step);
        e = launch_step(c, overlap, first, !ahead);
        if (e != hipSuccess) return;
        c->step += 1;
        if (c->np > 0) c->nsamples += 1;
        c->noise_ready = noise && overlap && ahead ? c->step : -1;
    };
    int64_t s = 0;
    if (overlap && !c->profiling && nsteps >= RUN_STEPS + 1) {
        if (noise && c->noise_ready != c->step) {
            one(true);
            ++s;
        }
        if (e == hipSuccess && (!c->run_exec || c->run_sig != run_signature(c)) &&
            capture_run_graph(c) != hipSuccess)
            (void)hipGetLastError();   // no graph: the steps below are launched one by one
        for (; e == hipSuccess && c->run_exec && s + RUN_STEPS <= nsteps; s += RUN_STEPS) {
            e = hipGraphLaunch(c->run_exec, c->stream);
            if (e != hipSuccess) break;
            c->step += RUN_STEPS;
            if (c->np > 0) c->nsamples += RUN_STEPS;
            c->noise_ready = noise ? c->step : -1;
        }
        if (e != hipSuccess) return hip_fail(c, e, "step graph");
    }
    for (; s < nsteps; ++s) {
        one(eager_ahead);
        if (e != hipSuccess) return hip_fail(c, e, "step launch");
    }
    return IC_OK;
}

int ic_step_prepare(ic_ctx *c) {
    const int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    const bool overlap = (double)c->p.nx * c->p.ny * c->p.nz >= 1048576.0;
    if (!overlap || c->profiling || (c->run_exec && c->run_sig == run_signature(c))) return IC_OK;
    if (capture_run_graph(c) != hipSuccess)
        (void)hipGetLastError();   // ic_step captures again, or launches one by one
    return IC_OK;
}

// True when p is device memory the kernels can read and write directly.
static bool is_device_pointer(const void *p) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();   // unregistered host memory reports an error
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

int ic_interpolate(ic_ctx *c, int32_t n, const double *q, int32_t kind, const void *field,
                   double *out) {
    if (!c) return IC_E_ARG;
    if (n < 0) return fail(c, IC_E_ARG, "n < 0");
    if (kind < IC_CELL || kind > IC_FACES) return fail(c, IC_E_ARG, "bad kind");
    if (n == 0) return IC_OK;
    if (!q || !field || !out) return fail(c, IC_E_ARG, "NULL pointer");
    const bool q_dev = is_device_pointer(q), out_dev = is_device_pointer(out);
    if (q_dev && out_dev) {
        hipError_t e = launch_interpolate(c, n, q, kind, field, out);
        if (e != hipSuccess) return hip_fail(c, e, "interpolate launch");
        return IC_OK;
    }
    // host positions or results: staged through one device buffer
    const size_t nq = 3 * (size_t)n, no = (kind == IC_FACES ? 3 : 1) * (size_t)n;
    double *tmp = nullptr;
    hipError_t e = hipMalloc((void **)&tmp, (nq + no) * sizeof(double));
    if (e != hipSuccess) return hip_fail(c, e, "interpolate staging");
    const double *qd = q;
    double *od = out_dev ? out : tmp + nq;
    if (!q_dev) {
        e = hipMemcpyAsync(tmp, q, nq * sizeof(double), hipMemcpyHostToDevice, c->stream);
        qd = tmp;
    }
    if (e == hipSuccess) e = launch_interpolate(c, n, qd, kind, field, od);
    if (e == hipSuccess && !out_dev)
        e = hipMemcpyAsync(out, od, no * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    const hipError_t ef = hipFree(tmp);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return hip_fail(c, e, "interpolate");
    return IC_OK;
}

int ic_interpolate_noalloc(ic_ctx *c, int32_t n, const double *q, int32_t kind,
                           const void *field, double *out) {
    if (!c) return IC_E_ARG;
    if (n < 0) return fail(c, IC_E_ARG, "n < 0");
    if (n > IC_NOALLOC_MAX_POINTS)
        return fail(c, IC_E_ARG,
                    "n > IC_NOALLOC_MAX_POINTS: the static staging buffer of "
                    "ic_interpolate_noalloc holds 16384 positions (use ic_interpolate)");
    if (kind < IC_CELL || kind > IC_FACES) return fail(c, IC_E_ARG, "bad kind");
    if (n == 0) return IC_OK;
    if (!q || !field || !out) return fail(c, IC_E_ARG, "NULL pointer");
    const bool q_dev = is_device_pointer(q), out_dev = is_device_pointer(out);
    hipError_t e;
    if (q_dev && out_dev)
        e = launch_interpolate(c, n, q, kind, field, out);
    else
        e = launch_interpolate_noalloc(c, n, q, q_dev, kind, field, out, out_dev);
    if (e != hipSuccess) return hip_fail(c, e, "interpolate (no allocation)");
    return IC_OK;
}

int ic_spread(ic_ctx *c, int32_t n, const double *q, const double *f, int32_t kind, void *field) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    if (n < 0) return fail(c, IC_E_ARG, "n < 0");
    if (n > c->p.max_particles) return fail(c, IC_E_CAPACITY, "n > max_particles");
    if (kind < IC_CELL || kind > IC_FACE_Z) return fail(c, IC_E_ARG, "bad kind");
    if (n == 0) return IC_OK;
    if (!q || !f || !field) return fail(c, IC_E_ARG, "NULL pointer");
    hipError_t e = launch_spread(c, n, q, f, kind, field);
    if (e != hipSuccess) return hip_fail(c, e, "spread launch");
    return IC_OK;
}

int ic_avg_force(ic_ctx *c, double *f_out, double *lambda_out, int64_t *nsamples, int32_t reset) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    const size_t n3 = 3 * (size_t)c->np;
    std::vector<double> sf(n3), sl(n3);
    hipError_t e = hipSuccess;
    if (n3) {
        e = hipMemcpyAsync(sf.data(), c->ws.sum_f, n3 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sl.data(), c->ws.sum_l, n3 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "avg_force readback");
    const double inv = c->nsamples > 0 ? 1.0 / (double)c->nsamples : 0.0;
    for (size_t i = 0; i < n3; ++i) {
        if (f_out) f_out[i] = sf[i] * inv;
        if (lambda_out) lambda_out[i] = sl[i] * inv;
    }
    if (nsamples) *nsamples = c->nsamples;
    if (reset) {
        std::vector<double> z(n3, 0.0);
        if (n3) {
            e = hipMemcpyAsync(c->ws.sum_f, z.data(), n3 * sizeof(double), hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->ws.sum_l, z.data(), n3 * sizeof(double), hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "avg_force reset");
        }
        c->nsamples = 0;
    }
    return take_flag(c);
}

int ic_conserved(ic_ctx *c, double out[4]) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    if (!out) return fail(c, IC_E_ARG, "out is NULL");
    double s[4];
    hipError_t e = launch_conserved(c, s);
    if (e != hipSuccess) return hip_fail(c, e, "conserved");
    const double h3 = c->p.h * c->p.h * c->p.h;
    for (int k = 0; k < 4; ++k) out[k] = h3 * s[k];
    if (c->np > 0) {
        const size_t n = (size_t)c->np;
        std::vector<double> u(3 * n), me(n);
        e = hipMemcpyAsync(u.data(), c->ws.u, 3 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(me.data(), c->ws.me, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "conserved particles");
        for (size_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) out[1 + a] += me[i] * u[3 * i + a];
    }
    return take_flag(c);
}

double ic_eps_from_kappa_ratio(double cf, double kappa_ratio) {
    return cf * cf * (1.0 / kappa_ratio - 1.0);
}

const char *ic_strerror(int code) {
    switch (code) {
        case IC_OK: return "ok";
        case IC_E_ARG: return "invalid argument";
        case IC_E_UNSTABLE: return "time step beyond the stability limit";
        case IC_E_MASS: return "non-positive mass or negative squared sound speed";
        case IC_E_STATE: return "call out of order";
        case IC_E_HIP: return "HIP runtime error";
        case IC_E_CAPACITY: return "too many particles";
        default: return "unknown error";
    }
}

const char *ic_last_error(const ic_ctx *c) { return c ? c->err.c_str() : "no context"; }

int ic_adjoint_workspace_size(const ic_params *p, size_t *bytes) {
    if (!bytes) return IC_E_ARG;
    const int rc = check_params(p, nullptr);
    if (rc != IC_OK) return rc;
    *bytes = adjoint_workspace_bytes(*p);
    return IC_OK;
}

int ic_bind_adjoint(ic_ctx *c, void *workspace, size_t bytes) {
    if (!c) return IC_E_ARG;
    if (!workspace && bytes == 0) {   // unbind: the caller is about to free it
        c->adj_bound = false;
        c->adj = AdjWorkspace{};
        return IC_OK;
    }
    if (!workspace) return fail(c, IC_E_ARG, "NULL adjoint workspace");
    if (((uintptr_t)workspace & 255) != 0) return fail(c, IC_E_ARG, "adjoint workspace not 256-byte aligned");
    if (bytes < adjoint_workspace_bytes(c->p)) return fail(c, IC_E_ARG, "adjoint workspace too small");
    carve_adjoint(c->p, (char *)workspace, c->adj);
    hipError_t e = hipMemsetAsync(c->adj.partial, 0,
                                  (size_t)IC_MAX_MODES * adjoint_blocks(c->p) * sizeof(double), c->stream);
    const size_t pb = (size_t)c->p.max_particles * sizeof(double);
    for (double *g : {c->adj.pdme, c->adj.pdeps, c->adj.pdks})
        if (e == hipSuccess && pb) e = hipMemsetAsync(g, 0, pb, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "bind adjoint");
    c->adj_bound = true;
    return IC_OK;
}

int ic_adjoint_step(ic_ctx *c, int64_t n, const void *drho, const void *gx, const void *gy,
                    const void *gz, void *ldrho, void *lgx, void *lgy, void *lgz) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    if (!c->adj_bound) return fail(c, IC_E_STATE, "adjoint workspace not bound");
    if (c->p.kT != 0.0) return fail(c, IC_E_STATE, "adjoint needs kT = 0");
    if (c->np != 0) return fail(c, IC_E_STATE, "adjoint needs a particle-free context");
    if (n < 0) return fail(c, IC_E_ARG, "step must be >= 0");
    if (!drho || !gx || !gy || !gz || !ldrho || !lgx || !lgy || !lgz)
        return fail(c, IC_E_ARG, "NULL field");
    const void *const Un[4] = {drho, gx, gy, gz};
    void *const lam[4] = {ldrho, lgx, lgy, lgz};
    hipError_t e = launch_adjoint_step(c, n, Un, lam, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint step");
    return IC_OK;
}

int ic_adjoint_step_particles(ic_ctx *c, int64_t n, const void *drho, const void *gx,
                              const void *gy, const void *gz, const double *q, const double *u,
                              void *ldrho, void *lgx, void *lgy, void *lgz, double *lq, double *lu,
                              const double *lF) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    if (!c->adj_bound) return fail(c, IC_E_STATE, "adjoint workspace not bound");
    if (c->p.kT != 0.0) return fail(c, IC_E_STATE, "adjoint needs kT = 0");
    if (n < 0) return fail(c, IC_E_ARG, "step must be >= 0");
    if (!drho || !gx || !gy || !gz || !ldrho || !lgx || !lgy || !lgz)
        return fail(c, IC_E_ARG, "NULL field");
    if (c->np > 0 && (!q || !u || !lq || !lu)) return fail(c, IC_E_ARG, "NULL particle array");
    const void *const Un[4] = {drho, gx, gy, gz};
    void *const lam[4] = {ldrho, lgx, lgy, lgz};
    const AdjParticles pp{q, u, lq, lu, lF};
    hipError_t e = launch_adjoint_step(c, n, Un, lam, &pp);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint step");
    return IC_OK;
}

int ic_adjoint_particle_grad(ic_ctx *c, double *dme, double *deps, double *dks, int32_t reset) {
    if (!c) return IC_E_ARG;
    if (!c->adj_bound) return fail(c, IC_E_STATE, "adjoint workspace not bound");
    const size_t b = (size_t)c->np * sizeof(double);
    hipError_t e = hipSuccess;
    double *host[3] = {dme, deps, dks};
    double *dev[3] = {c->adj.pdme, c->adj.pdeps, c->adj.pdks};
    for (int k = 0; k < 3; ++k)
        if (e == hipSuccess && host[k] && b)
            e = hipMemcpyAsync(host[k], dev[k], b, hipMemcpyDeviceToHost, c->stream);
    if (reset) {
        const size_t pb = (size_t)c->p.max_particles * sizeof(double);
        for (int k = 0; k < 3; ++k)
            if (e == hipSuccess && pb) e = hipMemsetAsync(dev[k], 0, pb, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint particle gradients");
    return take_flag(c);
}

int ic_get_state(ic_ctx *c, void *drho, void *gx, void *gy, void *gz, double *q, double *u) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    const size_t fb = (size_t)c->p.nx * c->p.ny * c->p.nz * (c->p.prec == IC_FP64 ? 8 : 4);
    void *dst[4] = {drho, gx, gy, gz};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 4 && e == hipSuccess; ++i)
        if (dst[i]) e = hipMemcpyAsync(dst[i], c->f[i], fb, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "get_state");
    return ic_copy_particles(c, q, u);
}

int ic_set_state(ic_ctx *c, const void *drho, const void *gx, const void *gy, const void *gz,
                 const double *q, const double *u) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    const size_t fb = (size_t)c->p.nx * c->p.ny * c->p.nz * (c->p.prec == IC_FP64 ? 8 : 4);
    const void *src[4] = {drho, gx, gy, gz};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 4 && e == hipSuccess; ++i)
        if (src[i]) e = hipMemcpyAsync(c->f[i], src[i], fb, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_state");
    rc = ic_load_particles(c, q, u);
    if (rc != IC_OK) return rc;
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_state");
    return IC_OK;
}

int ic_copy_particles(ic_ctx *c, double *q, double *u) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    const size_t b3 = 3 * (size_t)c->np * sizeof(double);
    hipError_t e = hipSuccess;
    if (q && b3) e = hipMemcpyAsync(q, c->ws.q, b3, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && u && b3) e = hipMemcpyAsync(u, c->ws.u, b3, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy_particles");
    return IC_OK;
}

int ic_load_particles(ic_ctx *c, const double *q, const double *u) {
    int rc = check_bound(c);
    if (rc != IC_OK) return rc;
    const size_t n3 = 3 * (size_t)c->np, b3 = n3 * sizeof(double);
    hipError_t e = hipSuccess;
    if (q && b3) {
        // positions index the grid: checked and wrapped on the host
        std::vector<double> hq(n3);
        e = hipMemcpyAsync(hq.data(), q, b3, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "load_particles");
        const double L[3] = {c->p.nx * c->p.h, c->p.ny * c->p.h, c->p.nz * c->p.h};
        for (size_t i = 0; i < n3; ++i) {
            if (!isfinite(hq[i])) return fail(c, IC_E_ARG, "non-finite position");
            const double Li = L[i % 3];
            double x = fmod(hq[i], Li);
            if (x < 0) x += Li;
            if (x >= Li) x -= Li;
            hq[i] = x;
        }
        e = hipMemcpyAsync(c->ws.q, hq.data(), b3, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e == hipSuccess && u && b3) e = hipMemcpyAsync(c->ws.u, u, b3, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "load_particles");
    return IC_OK;
}

int ic_adjoint_drive(ic_ctx *c, double *grad, int32_t reset) {
    if (!c || !grad) return IC_E_ARG;
    if (!c->adj_bound) return fail(c, IC_E_STATE, "adjoint workspace not bound");
    const int nb = adjoint_blocks(c->p);
    std::vector<double> part((size_t)IC_MAX_MODES * nb);
    hipError_t e = hipMemcpyAsync(part.data(), c->adj.partial, part.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint drive read");
    for (int m = 0; m < c->forcing.nmodes; ++m) {
        double sum = 0.0;
        for (int b = 0; b < nb; ++b) sum += part[(size_t)m * nb + b];
        grad[m] = sum;
    }
    if (reset) {
        e = hipMemsetAsync(c->adj.partial, 0, part.size() * sizeof(double), c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "adjoint drive reset");
    }
    return IC_OK;
}

int ic_graph_create(ic_ctx *const *ctxs, int32_t n, int64_t nsteps, ic_graph **out) {
    if (!out) return IC_E_ARG;
    *out = nullptr;
    if (!ctxs || n <= 0 || nsteps <= 0) return IC_E_ARG;
    for (int32_t i = 0; i < n; ++i) {
        if (!ctxs[i]) return IC_E_ARG;
        if (!ctxs[i]->bound) return fail(ctxs[i], IC_E_STATE, "graph: context not bound");
        if (ctxs[i]->profiling) return fail(ctxs[i], IC_E_STATE, "graph: profiling is on");
        for (int32_t j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(ctxs[i], IC_E_ARG, "graph: context listed twice");
    }
    ic_graph *g = new (std::nothrow) ic_graph();
    if (!g) return IC_E_ARG;
    g->ctxs.assign(ctxs, ctxs + n);
    g->nsteps = nsteps;
    // One large grid: capture the eager schedule itself (prologue and next
    // step's noise on the context's side stream, forked from and joined into
    // the captured origin stream), which the single-stream batched step
    // cannot overlap.
    const ic_params &p0 = ctxs[0]->p;
    const bool single_large = n == 1 && (double)p0.nx * p0.ny * p0.nz >= 1048576.0;
    if (!single_large && batch_supported(ctxs, n)) {
        const hipError_t eb = batch_create(ctxs, n, &g->batch);
        if (eb != hipSuccess) {
            delete g;
            return hip_fail(ctxs[0], eb, "graph: batch tables");
        }
    }
    // one branch stream per context, forked from and joined into an origin
    // stream that is captured (default priorities throughout)
    hipStream_t origin = nullptr;
    std::vector<hipStream_t> br(n, nullptr);
    std::vector<hipEvent_t> join(n, nullptr);
    hipEvent_t fork = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&origin, hipStreamNonBlocking);
    for (int32_t i = 0; i < n && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    bool capturing = false;
    if (e == hipSuccess) {
        e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal);
        capturing = e == hipSuccess;
    }
    if (e == hipSuccess && g->batch) {
        // batched: each kernel of a step once for every context
        for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s) e = batch_step(g->batch, origin);
    } else if (e == hipSuccess && single_large) {
        ic_ctx *c = ctxs[0];
        const hipStream_t own = c->stream;
        c->stream = origin;
        for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s)
            e = launch_step(c, true, s == 0, s == nsteps - 1);
        c->stream = own;
    } else if (e == hipSuccess) {
        e = hipEventRecord(fork, origin);
        for (int32_t i = 0; i < n && e == hipSuccess; ++i) {
            ic_ctx *c = ctxs[i];
            e = hipStreamWaitEvent(br[i], fork, 0);
            const hipStream_t own = c->stream;
            c->stream = br[i];
            // single-stream steps: a second stream forked from the branch
            // stream would nest one capture join inside another
            for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s)
                e = launch_step(c, false, true, true);
            c->stream = own;
            if (e == hipSuccess) e = hipEventRecord(join[i], br[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(origin, join[i], 0);
        }
    }
    if (capturing) {
        const hipError_t e2 = hipStreamEndCapture(origin, &g->graph);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (fork) (void)hipEventDestroy(fork);
    for (int32_t i = 0; i < n; ++i) {
        if (join[i]) (void)hipEventDestroy(join[i]);
        if (br[i]) (void)hipStreamDestroy(br[i]);
    }
    if (origin) (void)hipStreamDestroy(origin);
    if (e != hipSuccess) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        batch_destroy(g->batch);
        delete g;
        return hip_fail(ctxs[0], e, "graph capture");
    }
    *out = g;
    return IC_OK;
}

int ic_graph_launch(ic_graph *g, void *stream) {
    if (!g || !g->exec) return IC_E_ARG;
    const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(g->ctxs[0], e, "graph launch");
    for (ic_ctx *c : g->ctxs) {
        c->step += g->nsteps;
        if (c->np > 0) c->nsamples += g->nsteps;
        c->noise_ready = -1;   // the graph's steps reuse the noise sets
    }
    return IC_OK;
}

int ic_graph_destroy(ic_graph *g) {
    if (!g) return IC_E_ARG;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    batch_destroy(g->batch);
    delete g;
    return IC_OK;
}

}  // extern "C"
