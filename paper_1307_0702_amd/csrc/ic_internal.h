// Internal declarations shared by the C-ABI layer and the HIP kernels of
// libic.so.  Not part of the public interface (include/ic.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "ic.h"

namespace ic {

// Stage-kernel tile: TX cells along x (one half-wave row each), TY rows along
// y, marching over up to tz planes along z (tz chosen per grid, see
// choose_tz).  One thread per (x, y) column.
constexpr int TX = 32;
constexpr int TY = 16;
constexpr int STAGE_THREADS = TX * TY;
// Largest number of stencil blocks one particle's influence box can touch
// (at most 3 tiles per axis).
constexpr int MAX_BLOCKS_PER_PARTICLE = 27;

// Per-particle kernel data at q^{n+1/2}, fixed during the three RK stages
// (App. A, substep 3): first index of the 3 cell-centred and of the 3
// face-shifted kernel points along each axis, and their weights phi.
struct PartKernel {
    int32_t *bc;     // [N][3] first cell index of the cell stencil
    int32_t *bf;     // [N][3] first face index of the face stencil
    double *wc;      // [N][3][3] phi at the cell points, per axis
    double *wf;      // [N][3][3] phi at the face points, per axis
};

// Per-step scalars kept on the device, so that a captured step replays with
// the right step number and drive amplitudes: k_step_begin reads `step`,
// publishes it in `cur` and the amplitudes of the three stage times, then
// advances `step`.
struct StepState {
    int64_t step;                   // next step to run
    uint32_t cur;                   // step in flight (low 32 bits: Philox counter word)
    uint32_t pad;
    double amp[3][IC_MAX_MODES];    // p_ext amplitude at t^n, t^{n+1}, t^{n+1/2}
};

// Smallest z extent of a stage block; the workspace is sized for it, so any
// allowed extent (4, 8, 16, 32) can be chosen after creation.
constexpr int TZ_MIN = 4;

// Device workspace carved out of the caller's buffer.
struct Workspace {
    void *A[4];          // stage buffer U~ (drho, gx, gy, gz)
    void *B[4];          // stage buffer U^{n+1/2}
    // stochastic increments of the three stages (x, y, z each), kT > 0 only;
    // two sets: step n uses set n & 1, so the next step's set can be filled
    // while this step runs
    void *N[2][9];
    // persistent particle state, [N][3] or [N]
    double *q, *u, *me, *eps, *ks, *qeq, *fext;
    // per-step particle data (omega: [2][N], the Omega of two consecutive
    // RK stages)
    double *qh, *jv_old, *F, *Vt, *du, *mf, *omega, *jv_new;
    PartKernel pk;
    // binning of particles into stage blocks
    int32_t *blk_count, *blk_off, *blk_cursor, *blk_list, *blk_key;
    // clusters of particles with intersecting influence boxes ([N] each,
    // cl_off [N + 1]): union-find forest, roots, member counts and offsets
    // per root, fill cursors, members grouped by root
    int32_t *cl_parent, *cl_root, *cl_cnt, *cl_off, *cl_cursor, *cl_list;
    // accumulators
    double *sum_f, *sum_l;
    // forcing profiles [IC_MAX_MODES][pmax]
    double *prof;
    // reductions and flags: flag[0] m_e + m_f <= 0 in a step, flag[1] a
    // non-finite position given to a reversed step, flag[2] a non-finite
    // particle position, velocity or impulse in a step
    double *red;
    int32_t *flag;
    StepState *st;
};

// Adjoint workspace (ic_bind_adjoint): adjoint stage states, the
// accumulator of dL/dU^n, the face-density adjoints and the per-block
// partial sums of the drive-amplitude gradient (one block per 256 cells).
struct AdjWorkspace {
    void *L2[4], *L1[4], *acc[4], *murf[3], *mur;
    double *partial;   // [IC_MAX_MODES][adjoint_blocks]
    // per particle, [N][3]: dL/dq^{n+1/2}, dL/dF^{n+1/2}, dL/dV~, dL/dm_f of
    // the step being reversed; [N]: dL/dm_e, dL/deps_pf, dL/dk_s accumulated
    // over reversed steps until read with reset
    double *plqh, *plF, *plVt, *plmf, *pdme, *pdeps, *pdks;
    double *pq;   // [N][3] the caller's q^n, wrapped into the box
};
// Particle arrays of one reversed step (device, [N][3]): the state q^n, u^n
// before the step, the adjoints lq, lu (in: after the step, out: before) and
// an optional seed dL/dF^{n+1/2}.
struct AdjParticles {
    const double *q, *u;
    double *lq, *lu;
    const double *lF;
};
// z extent of a block of the adjoint's momentum pass (tiles of 32 x 8
// columns): minimises rounds of resident blocks (4 per CU in FP32, 2 in
// FP64, 256 CUs) times planes marched (the extent plus the two planes of the
// prologue); ties go to the larger extent.
constexpr int ADJ_TZ_MIN = 2;
inline int adjoint_tz(const ic_params &p) {
    const long cols = (long)((p.nx + 31) / 32) * ((p.ny + 7) / 8);
    const long cap = 256L * (p.prec == IC_FP64 ? 2 : 4);
    int best = 32;
    long best_cost = -1;
    for (int tz = 32; tz >= ADJ_TZ_MIN; tz /= 2) {
        const long blocks = cols * ((p.nz + tz - 1) / tz);
        const long cost = ((blocks + cap - 1) / cap) * ((tz < p.nz ? tz : p.nz) + 2);
        if (best_cost < 0 || cost < best_cost) {
            best = tz;
            best_cost = cost;
        }
    }
    return best;
}
// Partial-sum slots per mode: at least one per block of the momentum pass at
// the smallest z extent, and never fewer than one per 256 cells.
inline int adjoint_blocks(const ic_params &p) {
    const long cells = ((long)p.nx * p.ny * p.nz + 255) / 256;
    const long tiles = (long)((p.nx + 31) / 32) * ((p.ny + 7) / 8) *
                       ((p.nz + ADJ_TZ_MIN - 1) / ADJ_TZ_MIN);
    return (int)(cells > tiles ? cells : tiles);
}
size_t adjoint_workspace_bytes(const ic_params &p);
void carve_adjoint(const ic_params &p, char *base, AdjWorkspace &aw);

struct Forcing {
    int nmodes;
    ic_mode modes[IC_MAX_MODES];
};

}  // namespace ic

struct ic_ctx {
    ic_params p;
    hipStream_t stream;
    int device;
    int ncu;   // compute units of the device (one background noise block each)
    bool bound;
    void *f[4];
    ic::Workspace ws;
    int32_t np;
    int64_t step;
    int64_t nsamples;
    ic::Forcing forcing;
    int nblk[3];
    int tz;
    int prof_stride;
    std::string err;
    // stage-kernel timing (ic_profile)
    bool profiling;
    std::vector<hipEvent_t> ev_pool;   // free events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    double prof_ms;
    int64_t prof_launches;
    // side stream: particle prologue and next-step noise run beside the
    // fluid stages (default priority); fork / join events
    hipStream_t side;
    hipEvent_t ev_fork, ev_part, ev_noise;
    // reverse mode (ic_bind_adjoint)
    bool adj_bound;
    ic::AdjWorkspace adj;
    // ic_step's own graph of a few steps (grids of >= 2^20 cells), replayed
    // while the launch arguments it captured (run_sig) still hold
    hipGraph_t run_graph;
    hipGraphExec_t run_exec;
    std::vector<char> run_sig;
    // step whose noise increments the previous step already drew (-1: none)
    int64_t noise_ready;
};

namespace ic {

size_t workspace_bytes(const ic_params &p, size_t *offsets_out = nullptr);
int choose_tz(const ic_params &p);
void carve_workspace(const ic_params &p, char *base, Workspace &ws);
int nblocks_total(const ic_params &p);      // at the smallest z extent (workspace sizing)
int nblocks_of(const ic_ctx *c);            // at the context's z extent

// Launchers (ic_device.hip).  Each returns hipSuccess or the launch error.
// One IC step.  overlap: run the particle prologue and the next step's noise
// on the side stream (eager stepping only, never under graph capture); then
// first: the step's noise is not yet generated (first step of a call), last:
// do not generate the next step's noise.  Without overlap every step runs on
// the context stream and generates its own noise.
hipError_t launch_step(ic_ctx *c, bool overlap, bool first, bool last);
hipError_t launch_interpolate(ic_ctx *c, int n, const double *q, int kind, const void *field,
                              double *out);
// Batched ensemble steps (ic_graph_create): every kernel of a step runs once
// for all n contexts.  Supported when the contexts share a precision and
// none holds more particles than one workgroup clusters (512).
struct Batch;
bool batch_supported(ic_ctx *const *ctxs, int n);
hipError_t batch_create(ic_ctx *const *ctxs, int n, Batch **out);   // device tables (hipMalloc)
hipError_t batch_step(const Batch *b, hipStream_t s);              // one step of every context
void batch_destroy(Batch *b);
// ic_interpolate_noalloc: positions / results in host memory (flags false)
// are staged through the library's static device buffer; synchronises the
// context stream.  n <= IC_NOALLOC_MAX_POINTS.
hipError_t launch_interpolate_noalloc(ic_ctx *c, int n, const double *q, bool q_dev, int kind,
                                      const void *field, double *out, bool out_dev);
hipError_t launch_spread(ic_ctx *c, int n, const double *q, const double *f, int kind,
                         void *field);
hipError_t launch_init_velocity(ic_ctx *c);
hipError_t launch_conserved(ic_ctx *c, double *host_out);
hipError_t launch_set_step(ic_ctx *c);      // device step counter := c->step
// Reverse of step n from the state U^n (device fields): lam (device, in:
// dL/dU^{n+1}, out: dL/dU^n); drive gradient added to the adjoint partials.
// pp: the particle arrays, or nullptr for a particle-free context.
hipError_t launch_adjoint_step(ic_ctx *c, int64_t n, const void *const Un[4], void *const lam[4],
                               const AdjParticles *pp);

// Event pair around one stage launch when profiling (nullptr otherwise).
hipEvent_t prof_event(ic_ctx *c);
void prof_push(ic_ctx *c, hipEvent_t a, hipEvent_t b);

}  // namespace ic
