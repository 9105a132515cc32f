// HIP kernels of the inertial-coupling step for gfx950 and their launchers.
//
// Method: Balboa Usabiaga & Delgado-Buscalioni, arXiv:1307.0702, App. A
// ("Temporal discretization", substeps 1-7; SSP-RK3 stages with the noise
// combinations W_A -/+ sqrt(3) W_B, W_A and the stage pressures).
//
// Layout: state fields are SoA arrays, x fastest; face i+1/2 of a vector
// component belongs to cell i.  The density array holds rho - rho0.
//
// The fluid stage (the hot loop, three sweeps per step) is one kernel per RK
// stage: each block owns a TX x TY column of cells and marches it along z,
// keeping one plane of momentum, velocity and fluxes and two of density in
// LDS.  Every value is read from HBM once per sweep (plus a ring one or two
// cells wide), the next plane is prefetched into registers while the current
// one is computed, and every flux is computed once (plus a one-cell ring of
// halo fluxes).  The stochastic increments of a step are drawn once, by the
// noise kernel, from a counter-based Philox generator keyed by (seed; cell,
// step, call, replica), and each stage reads its combination.  The particle
// terms run as one wave per cluster of particles whose kernels may touch the
// same points, members in ascending id.  There are no float atomics in the
// forward step, so its results are bitwise reproducible.  Data a sweep
// touches once streams past L2 (non-temporal), which keeps L2 for the halo
// the neighbouring blocks re-read; the next step's noise is drawn in the
// background of the step in flight by one block per CU.
#include <math.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "ic_internal.h"

// Multiply-adds are fused only where one source expression holds both (not
// across statements), so the code a kernel body compiles to does not depend
// on the kernel it is inlined into: the batched ensemble kernels then give
// the single-context kernels' results bit for bit.
#pragma clang fp contract(on)

// Argument tables of the batched ensemble kernels live in global memory that
// no kernel writes: declared constant (address space 4), their loads are
// scalar and may be repeated at any point, as kernel arguments are.
#define IC_CONST __attribute__((address_space(4)))

namespace ic {
namespace {

// A table entry viewed through an ordinary reference (the compiler still sees
// where it points).
template <typename X>
__device__ __forceinline__ const X &from_const(const IC_CONST X &r) {
    return *(const X *)&r;
}

// ---------------------------------------------------------------------------
// 3-point function of Roma and Peskin (App. A, "Spatial discretization").
// ---------------------------------------------------------------------------
__device__ __forceinline__ double phi3(double r) {
    r = fabs(r);
    if (r <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * r * r)) * (1.0 / 3.0);
    if (r <= 1.5) {
        const double s = 1.0 - r;
        return (5.0 - 3.0 * r - sqrt(1.0 - 3.0 * s * s)) * (1.0 / 6.0);
    }
    return 0.0;
}

// Weight of point d (0..2) among the three kernel points along one axis from
// coordinate q (cell centres at i h, faces at (i + 1/2) h), and the first
// (wrapped) point index.
__device__ __forceinline__ int axis_point(double q, double inv_h, int n, bool face, int d,
                                          double *w) {
    const double x = q * inv_h - (face ? 0.5 : 0.0);
    const double nearest = floor(x + 0.5);
    *w = phi3(x - (nearest - 1.0 + d));
    int f = (int)nearest - 1;
    if (f < 0) f += n;
    if (f >= n) f -= n;
    return f;
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ double wrap_pos(double q, double L) {
    double r = q - L * floor(q / L);
    if (r >= L) r -= L;  // q/L rounding can leave r == L
    return r;
}

__device__ __forceinline__ double min_image(double d, double L) {
    return d - L * floor(d / L + 0.5);
}

// ---------------------------------------------------------------------------
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// Coefficients of the FP64 Box-Muller series (highest power first).  They
// reach the kernels as arguments, so every Horner step reads its coefficient
// from scalar registers; written as literals, each step first copied its
// 64-bit constant into a vector register pair (two extra VALU instructions
// per step; with the branch-free quarter-turn selection below, the FP64
// noise kernel went from 0.81 to 0.71 ms at 256^3).  bm_poly() fills them on
// the host with the values the series below state.
struct BMPoly {
    double ln[11];   // 1/21, 1/19, ..., 1/3, 1
    double sn[7];    // -1/15!, 1/13!, ..., -1/3!
    double cs[8];    // 1/16!, -1/14!, ..., 1/4!, -1/2!
};

template <typename T>
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, T &z0, T &z1,
                                           const BMPoly &P);
// FP64 Box-Muller on the 24-bit grid of the uniforms: u = m 2^-24 with m odd.
// ln u = (e - 24) ln 2 + ln f for m = f 2^e, f in [1/sqrt2, sqrt2), with
// ln f = 2 atanh(s), s = (f - 1)/(f + 1), |s| < 0.172, from its power series
// (terms to s^21, truncation below 1e-17 relative).
__device__ __forceinline__ double ln_grid24(uint32_t m, const BMPoly &P) {
    int e = 31 - __builtin_clz(m);
    double f = __builtin_ldexp((double)m, -e);     // [1, 2)
    if (f > 1.4142135623730951) {
        f *= 0.5;
        e += 1;
    }
    const double s = (f - 1.0) / (f + 1.0), z = s * s;
    double p = P.ln[0];
#pragma unroll
    for (int i = 1; i < 11; ++i) p = fma(p, z, P.ln[i]);
    return (double)(e - 24) * 0.6931471805599453 + 2.0 * s * p;
}

// cos and sin of the angle 2 pi n 2^-24: exact reduction to the nearest
// quarter turn in integers, then the Taylor series of sin (to th^15) and cos
// (to th^16) on |th| <= pi/4 (truncation below 7e-17).
__device__ __forceinline__ void sincos_grid24(uint32_t n, double &sn, double &cs,
                                              const BMPoly &P) {
    const uint32_t q = (n + (1u << 21)) >> 22;      // nearest quarter turn, 0..4
    const int j = (int)n - (int)(q << 22);           // [-2^21, 2^21]
    const double th = (double)j * (6.283185307179586 * 0x1p-24);
    const double z = th * th;
    double ps = P.sn[0];
#pragma unroll
    for (int i = 1; i < 7; ++i) ps = fma(ps, z, P.sn[i]);
    const double s0 = fma(th * z, ps, th);
    double pc = P.cs[0];
#pragma unroll
    for (int i = 1; i < 8; ++i) pc = fma(pc, z, P.cs[i]);
    const double c0 = fma(z, pc, 1.0);
    // quarter turn q: odd q swaps sin and cos; sin changes sign for q = 2, 3
    // and cos for q = 1, 2 (q = 4 is the full turn).  Selects, not a switch:
    // the lanes of a wave take different quarters.
    const double sv = (q & 1u) ? c0 : s0, cv = (q & 1u) ? s0 : c0;
    sn = (q & 2u) ? -sv : sv;
    cs = ((q + 1u) & 2u) ? -cv : cv;
}

template <>
__device__ __forceinline__ void box_muller<double>(uint32_t a, uint32_t b, double &z0,
                                                   double &z1, const BMPoly &P) {
    // uniforms ((x >> 9) + 1/2) 2^-23 = (2 (x >> 9) + 1) 2^-24
    const double r = sqrt(-2.0 * ln_grid24(2u * (a >> 9) + 1u, P));
    double s, c;
    sincos_grid24(2u * (b >> 9) + 1u, s, c, P);
    z0 = r * c;
    z1 = r * s;
}
template <>
__device__ __forceinline__ void box_muller<float>(uint32_t a, uint32_t b, float &z0, float &z1,
                                                  const BMPoly &) {
    const float u1 = ((float)(a >> 9) + 0.5f) * 0x1p-23f, u2 = ((float)(b >> 9) + 0.5f) * 0x1p-23f;
    // v_log_f32 is log2 (argument >= 2^-24, never denormal); v_sin/v_cos take
    // the angle in turns.
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
    z0 = r * __builtin_amdgcn_cosf(u2);
    z1 = r * __builtin_amdgcn_sinf(u2);
}

struct NoiseKey {
    uint32_t k0, k1, step, replica;
};

enum { SEL_ALL = 0, SEL_DIAG = 1, SEL_EDGE = 2 };

// The normals W_A and W_B of one cell and step, ordered xx, yy, zz, xy, xz,
// yz.  Philox calls: 0 -> A_xx A_yy A_zz A_xy, 1 -> A_xz A_yz B_xz B_yz,
// 2 -> B_xx B_yy B_zz B_xy (Box-Muller on word pairs (x,y) and (z,w)).
// SEL_DIAG fills the xx, yy, zz entries only, SEL_EDGE xy, xz, yz only.
template <typename T, int SEL>
__device__ __forceinline__ void cell_normals(uint32_t cell, const NoiseKey &nk, T A[6], T B[6],
                                             const BMPoly &P) {
    constexpr bool diag = SEL != SEL_EDGE, edge = SEL != SEL_DIAG;
    const U4 r0 = philox(cell, nk.step, 0u, nk.replica, nk.k0, nk.k1);
    if (diag) box_muller<T>(r0.x, r0.y, A[0], A[1], P);
    box_muller<T>(r0.z, r0.w, A[2], A[3], P);
    if (edge) {
        const U4 r1 = philox(cell, nk.step, 1u, nk.replica, nk.k0, nk.k1);
        box_muller<T>(r1.x, r1.y, A[4], A[5], P);
        box_muller<T>(r1.z, r1.w, B[4], B[5], P);
    }
    const U4 r2 = philox(cell, nk.step, 2u, nk.replica, nk.k0, nk.k1);
    if (diag) box_muller<T>(r2.x, r2.y, B[0], B[1], P);
    box_muller<T>(r2.z, r2.w, B[2], B[3], P);
}

// Discrete Landau-Lifshitz stress of one cell from its normals (Sec. IV B):
// diagonal sd Z_aa + st (Z_xx + Z_yy + Z_zz) at the centre, off-diagonal
// so Z_ab on the edges; sd = sqrt(2 eta kT) sqrt(2) / sqrt(h^3 dt),
// st = (sqrt(zeta kT / 3) - sqrt(2 eta kT) / 3) sqrt(2) / sqrt(h^3 dt),
// so = sqrt(2 eta kT) / sqrt(h^3 dt).
template <typename T>
__device__ __forceinline__ void ll_stress(const T Z[6], T sd, T st, T so, T S[6]) {
    const T tr = st * (Z[0] + Z[1] + Z[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) S[c] = sd * Z[c] + tr;
#pragma unroll
    for (int c = 3; c < 6; ++c) S[c] = so * Z[c];
}

template <typename T>
__device__ __forceinline__ T fast_rcp(T x);
template <>
__device__ __forceinline__ float fast_rcp<float>(float x) {
    return __builtin_amdgcn_rcpf(x);
}
template <>
__device__ __forceinline__ double fast_rcp<double>(double x) {
    return 1.0 / x;
}

// ---------------------------------------------------------------------------
// Fluid RK stage (App. A, SSP-RK3; fluxes of Sec. IV B with the conservative
// staggered discretisation given in the design notes).
// ---------------------------------------------------------------------------
template <typename T>
struct StageArgs {
    const T *in[4];   // stage input U^s
    const T *un[4];   // U^n (stages 2 and 3)
    T *out[4];
    int nx, ny, nz, tz, gx, gy, gz;
    uint32_t fbytes;  // bytes of one field (< 2^32)
    T rho0, cf2, eta, lam, inv_h, dt_h, dt, ra, rb;
    // stochastic increment of this stage (x, y, z) in the two noise sets,
    // NOISE only; step n reads set n & 1 (StepState.cur)
    const T *noise[2][3];
    const StepState *st;
    int full;         // every tile whole (nx, ny multiples of TX, TY)
    // imposed pressure: sum_m amp[m] * prof[m][coord(maxis[m])], amp at this
    // stage's time (StepState, device)
    int nmodes;
    int maxis[IC_MAX_MODES];
    const double *amp;
    const double *prof;
    int pstride;
};

constexpr int PX = TX + 3;  // local x in [-1, TX+1]
constexpr int PY = TY + 3;  // local y in [-1, TY+1]
constexpr int PS = PX * PY;

__device__ __forceinline__ int lidx(int lx, int ly) { return (ly + 1) * PX + (lx + 1); }

// Raw buffer access: a 32-bit per-thread byte offset inside a plane (VGPR)
// plus a uniform plane offset (SGPR), so that loads and stores need no
// per-access 64-bit address arithmetic.  Flags word of the gfx9 family.
//
// Cache policy: the stage sweep's stencil input is read by neighbouring
// blocks too (halo planes, ring columns), so it goes through L2 normally
// (CP_LOAD).  Data touched once per launch streams non-temporally (CP_NT):
// the stage outputs (no one reads them in the same launch, and the next
// sweep reads them whole from HBM), the pointwise U^n of the RK combination,
// and the noise increments (written once per step, read once per stage).
// Kept out of L2, they leave it to the re-read halo: at 256^3 the FP32 step
// went from 0.975 to 0.896 ms, the FP64 step from 2.12 to 2.00 ms.
constexpr int CP_LOAD = 0, CP_NT = 2;   // the nt bit of the cache-policy operand
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}
template <typename T, int CP = CP_LOAD>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, CP));
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, CP));
    }
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                       uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff,
                                          CP_NT);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                       uint32_t soff) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff,
                                          CP_NT);
}

// Kernels on the step's critical path (stage sweeps, particle passes) raise
// their waves' issue priority, so that the next step's noise kernel, which
// shares the CUs with them and is ALU-bound, takes the issue slots they leave
// idle rather than the ones they would use.
__device__ __forceinline__ void critical_path() { __builtin_amdgcn_s_setprio(3); }

// Imposed pressure at cell (x, y, z).  The particle pressure S Omega and the
// spread force S F are added after the sweep (k_cl_stage): both enter the
// stage output linearly.
// Split as p_ext(x, y) + p_ext(z): the x and y parts are fixed for a column,
// the z part is uniform over a plane.
template <typename T>
__device__ __forceinline__ T ext_pressure_xy(const StageArgs<T> &a, int x, int y) {
    T s = 0;
    for (int m = 0; m < a.nmodes; ++m) {
        const int ax = a.maxis[m];
        if (ax != 2) s += (T)a.amp[m] * (T)a.prof[m * a.pstride + (ax == 0 ? x : y)];
    }
    return s;
}
template <typename T>
__device__ __forceinline__ T ext_pressure_z(const StageArgs<T> &a, int z) {
    T s = 0;
    for (int m = 0; m < a.nmodes; ++m)
        if (a.maxis[m] == 2) s += (T)a.amp[m] * (T)a.prof[m * a.pstride + z];
    return s;
}

// One RK stage over a tile of TX x TY columns, marching over planes k of
// [z0, z1).  LDS holds only plane k: momentum and velocity on the region
// [-1, W] x [-1, Wy], density of planes k and k+1 on [-1, W+1] x [-1, Wy+1]
// (two alternating buffers) and the six x/y fluxes of plane k.  Values of
// plane k+1 that plane k needs (g and v at the same column) come from the
// registers that also commit plane k+1, and the zz flux of plane k+1 is
// taken one iteration later, so the z-momentum of plane k is written in
// iteration k+1.  Each thread owns one column; waves 0-3 also own one side
// each of the momentum ring (+x column, -x column, +y row, -y row, computing
// the fluxes the tile's own faces need there) and wave 4 the rest of the
// density ring.  Register sets for planes k+1 and k+2 alternate, so every
// load is issued one iteration before its use.
// Workgroups go to the 8 XCDs round-robin; tile index of workgroup b among
// nblk that gives each XCD a contiguous run of tiles (x fastest), so tiles
// sharing halo lines share one L2.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
    const int per = nblk / 8, rem = nblk % 8, xcd = b % 8, idx = b / 8;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

constexpr int STAGE_LDS = 14 * PS;   // elements of LDS a stage tile uses

// One RK stage over tile t of the context's grid; lds holds STAGE_LDS
// elements.
template <typename T, int STAGE, bool NOISE, bool FULL>
__device__ __forceinline__ void stage_body(const StageArgs<T> &a, int t, T *lds) {
    T(*s_G)[PS] = reinterpret_cast<T(*)[PS]>(lds);
    T(*s_V)[PS] = reinterpret_cast<T(*)[PS]>(lds + 3 * PS);
    T(*s_P)[PS] = reinterpret_cast<T(*)[PS]>(lds + 6 * PS);
    T(*s_F)[PS] = reinterpret_cast<T(*)[PS]>(lds + 8 * PS);

    const int nx = a.nx, ny = a.ny, nz = a.nz, tz = a.tz;
    const uint32_t pbytes = (uint32_t)nx * (uint32_t)ny * (uint32_t)sizeof(T);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int bx = t % a.gx, by = (t / a.gx) % a.gy, bz = t / (a.gx * a.gy);
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * tz;   // z0 is even (tz is)
    // FULL: every tile is whole (nx, ny multiples of TX, TY)
    const int W = FULL ? TX : min(TX, nx - x0), Wy = FULL ? TY : min(TY, ny - y0);
    const int z1 = min(z0 + tz, nz);
    const T rho0 = a.rho0, half = (T)0.5, quarter = (T)0.25;

    __amdgpu_buffer_rsrc_t rin[4], run[4], rnn[3], rout[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        rin[c] = make_rsrc(a.in[c], a.fbytes);
        rout[c] = make_rsrc(a.out[c], a.fbytes);
        if (STAGE != 0) run[c] = make_rsrc(a.un[c], a.fbytes);
    }
    if (NOISE) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            rnn[c] = make_rsrc((a.st->cur & 1u) ? a.noise[1][c] : a.noise[0][c], a.fbytes);
    }
    auto soff = [&](int p) -> uint32_t { return (uint32_t)wrap(p, nz) * pbytes; };

    // own column
    const int lx = tid % TX, ly = tid / TX;
    const bool own = FULL || (lx < W && ly < Wy);
    const int lo = lidx(lx, ly);
    const int xo = x0 + lx, yo = y0 + ly;
    const uint32_t vo = own ? (uint32_t)(yo * nx + xo) * (uint32_t)sizeof(T) : 0u;
    // momentum ring (waves 0-3) and the rest of the density ring (wave 4)
    bool r1 = false, r1f = false, r2 = false;
    int r1x = 0, r1y = 0, r2x = 0, r2y = 0;
    if (wave < 2) {
        if (lane < Wy + 2) {
            r1 = true;
            r1x = wave == 0 ? W : -1;
            r1y = lane - 1;
            r1f = lane >= 1 && lane <= Wy;
        }
    } else if (wave < 4) {
        if (lane < W) {
            r1 = true;
            r1f = true;
            r1x = lane;
            r1y = wave == 2 ? Wy : -1;
        }
    } else if (wave == 4) {
        if (lane < Wy + 3) {
            r2 = true;
            r2x = W + 1;
            r2y = lane - 1;
        } else if (lane < Wy + W + 5) {
            r2 = true;
            r2x = lane - (Wy + 3) - 1;
            r2y = Wy + 1;
        }
    }
    const int l1 = lidx(r1x, r1y), l2 = lidx(r2x, r2y);
    const int g1x = wrap(x0 + r1x, nx), g1y = wrap(y0 + r1y, ny);
    const T pex_own = own ? ext_pressure_xy(a, xo, yo) : (T)0;
    const T pex_r1 = r1 ? ext_pressure_xy(a, g1x, g1y) : (T)0;
    const uint32_t v1 = r1 ? (uint32_t)(g1y * nx + g1x) * (uint32_t)sizeof(T) : 0u;
    const uint32_t v2 =
        r2 ? (uint32_t)(wrap(y0 + r2y, ny) * nx + wrap(x0 + r2x, nx)) * (uint32_t)sizeof(T) : 0u;

    // Register set for plane p: momentum of p and density of p+1 at the own
    // column and the ring position, and density of p+1 on the density ring.
    struct Set {
        T g[3], rn, g1[3], rn1, rn2;
    };
    auto load_set = [&](Set &S, int p) {
        const uint32_t sg = soff(p), sr = soff(p + 1);
        if (own) {
#pragma unroll
            for (int c = 0; c < 3; ++c) S.g[c] = bload<T>(rin[1 + c], vo, sg);
            S.rn = bload<T>(rin[0], vo, sr);
        }
        if (r1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) S.g1[c] = bload<T>(rin[1 + c], v1, sg);
            S.rn1 = bload<T>(rin[0], v1, sr);
        }
        if (r2) S.rn2 = bload<T>(rin[0], v2, sr);
    };
    Set SO, SE;   // used by odd / even iterations k (planes k+1 even / odd)

    // v = g / rho_face at a column with density r (plane p), its +x and +y
    // neighbours and density rz of plane p+1 above it
    auto vel = [&](const T g[3], T r, T rxp, T ryp, T rz, T v[3]) {
        v[0] = g[0] * fast_rcp<T>(rho0 + half * (r + rxp));
        v[1] = g[1] * fast_rcp<T>(rho0 + half * (r + ryp));
        v[2] = g[2] * fast_rcp<T>(rho0 + half * (r + rz));
    };

    // ---- prologue: plane z0-1 into G/V, density z0-1 and z0 into P
    {
        const uint32_t sr = soff(z0 - 1);
        if (own) s_P[1][lo] = bload<T>(rin[0], vo, sr);
        if (r1) s_P[1][l1] = bload<T>(rin[0], v1, sr);
        if (r2) s_P[1][l2] = bload<T>(rin[0], v2, sr);
    }
    load_set(SE, z0 - 1);
    __syncthreads();
    {
        const T *P = s_P[1];
        if (own) {
            T v[3];
            vel(SE.g, P[lo], P[lo + 1], P[lo + PX], SE.rn, v);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                s_G[c][lo] = SE.g[c];
                s_V[c][lo] = v[c];
            }
            s_P[0][lo] = SE.rn;
        }
        if (r1) {
            T v[3];
            vel(SE.g1, P[l1], P[l1 + 1], P[l1 + PX], SE.rn1, v);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                s_G[c][l1] = SE.g1[c];
                s_V[c][l1] = v[c];
            }
            s_P[0][l1] = SE.rn1;
        }
        if (r2) s_P[0][l2] = SE.rn2;
    }
    load_set(SO, z0);
    load_set(SE, z0 + 1);
    __syncthreads();

    // carried values
    T vzm = 0, gzm = 0;           // own column: vz, gz of plane k-1
    T vzm1 = 0;                   // ring position: vz of plane k-1
    T Pzz_m = 0, Pxz_m = 0, Pyz_m = 0;   // own column: zz flux at k-1, xz/yz at k-1/2
    T lag_d = 0, lag_u = 0, lag_n = 0;   // z-momentum of plane k-1 waiting for Pzz(k)
    const T dth = a.dt_h;

    auto fin_gz = [&](int kz, T Pzz_k) {
        // z-momentum of plane kz = k-1, now that the zz flux of plane k is known
        const T d = lag_d - dth * (Pzz_k - Pzz_m);
        const T v = STAGE == 0 ? lag_u + d : a.ra * lag_n + a.rb * (lag_u + d);
        bstore(v, rout[3], vo, soff(kz));
    };

    // One plane.  ODD: parity of k (fixes the buffer roles); PREP: k = z0-1,
    // which only prepares carried values.
    auto iteration = [&](auto odd_c, auto prep_c, const int k, Set &S) {
        constexpr bool ODD = decltype(odd_c)::value, PREP = decltype(prep_c)::value;
        const T *Pk = s_P[ODD ? 1 : 0];     // density of plane k
        const T *P1 = s_P[ODD ? 0 : 1];     // density of plane k+1
        T *Pw = s_P[ODD ? 1 : 0];           // receives density of plane k+2
        const T *gx = s_G[0], *gy = s_G[1], *gz = s_G[2];
        const T *vx = s_V[0], *vy = s_V[1], *vz = s_V[2];
        const int zk = k;                   // k in [z0-1, z1)
        const T pez = PREP ? (T)0 : ext_pressure_z(a, wrap(zk, nz));
        // ---- phase B: velocities of plane k+1, fluxes of plane k
        T vn[3] = {0, 0, 0}, vn1[3] = {0, 0, 0};
        T un[4] = {0, 0, 0, 0}, nn[3] = {0, 0, 0}, mflux = 0, Pxz = 0, Pyz = 0;
        // FP64: the pointwise loads go out after the barrier, just before
        // their use, so they are not held across the flux phase
        constexpr bool EARLY = sizeof(T) == 4;
        if (EARLY && !PREP && own) {
            const uint32_t su = soff(zk);
            if (STAGE != 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) un[c] = bload<T, CP_NT>(run[c], vo, su);
            }
            if (NOISE) {
#pragma unroll
                for (int c = 0; c < 3; ++c) nn[c] = bload<T, CP_NT>(rnn[c], vo, su);
            }
        }
        if (own) {
            const int l = lo;
            vel(S.g, P1[l], P1[l + 1], P1[l + PX], S.rn, vn);
            const T viz_x = a.eta * ((vn[0] - vx[l]) + (vz[l + 1] - vz[l])) * a.inv_h;
            const T viz_y = a.eta * ((vn[1] - vy[l]) + (vz[l + PX] - vz[l])) * a.inv_h;
            Pxz = quarter * (gx[l] + S.g[0]) * (vz[l] + vz[l + 1]) - viz_x;
            Pyz = quarter * (gy[l] + S.g[1]) * (vz[l] + vz[l + PX]) - viz_y;
            if (!PREP) {
                const T pi = a.cf2 * Pk[l] + (pex_own + pez);
                const T dvx = vx[l] - vx[l - 1], dvy = vy[l] - vy[l - PX], dvz = vz[l] - vzm;
                const T ldiv = a.lam * ((dvx + dvy + dvz) * a.inv_h);
                const T Pzz = pi + quarter * (gz[l] + gzm) * (vz[l] + vzm) -
                              (2 * a.eta * dvz * a.inv_h + ldiv);
                if (k > z0) fin_gz(k - 1, Pzz);
                Pzz_m = Pzz;
                const T pxx = pi + quarter * (gx[l] + gx[l - 1]) * (vx[l] + vx[l - 1]) -
                              (2 * a.eta * dvx * a.inv_h + ldiv);
                const T pyy = pi + quarter * (gy[l] + gy[l - PX]) * (vy[l] + vy[l - PX]) -
                              (2 * a.eta * dvy * a.inv_h + ldiv);
                const T vxy = a.eta * ((vx[l + PX] - vx[l]) + (vy[l + 1] - vy[l])) * a.inv_h;
                s_F[0][l] = pxx;
                s_F[1][l] = pyy;
                s_F[2][l] = quarter * (gx[l] + gx[l + PX]) * (vy[l] + vy[l + 1]) - vxy;
                s_F[3][l] = quarter * (gy[l] + gy[l + 1]) * (vx[l] + vx[l + PX]) - vxy;
                s_F[4][l] = quarter * (gz[l] + gz[l + 1]) * (vx[l] + vn[0]) - viz_x;
                s_F[5][l] = quarter * (gz[l] + gz[l + PX]) * (vy[l] + vn[1]) - viz_y;
                mflux = (gx[l] - gx[l - 1]) + (gy[l] - gy[l - PX]) + (gz[l] - gzm);
            }
            vzm = vz[l];
            gzm = gz[l];
        }
        if (r1) {
            const int l = l1;
            vel(S.g1, P1[l], P1[l + 1], P1[l + PX], S.rn1, vn1);
            if (!PREP && r1f) {
                if (wave == 0) {            // +x column: centre flux xx
                    const T pi = a.cf2 * Pk[l] + (pex_r1 + pez);
                    const T dvx = vx[l] - vx[l - 1];
                    const T div = (dvx + (vy[l] - vy[l - PX]) + (vz[l] - vzm1)) * a.inv_h;
                    s_F[0][l] = pi + quarter * (gx[l] + gx[l - 1]) * (vx[l] + vx[l - 1]) -
                                (2 * a.eta * dvx * a.inv_h + a.lam * div);
                } else if (wave == 2) {     // +y row: centre flux yy
                    const T pi = a.cf2 * Pk[l] + (pex_r1 + pez);
                    const T dvy = vy[l] - vy[l - PX];
                    const T div = ((vx[l] - vx[l - 1]) + dvy + (vz[l] - vzm1)) * a.inv_h;
                    s_F[1][l] = pi + quarter * (gy[l] + gy[l - PX]) * (vy[l] + vy[l - PX]) -
                                (2 * a.eta * dvy * a.inv_h + a.lam * div);
                } else if (wave == 1) {     // -x column: edge fluxes yx, zx
                    const T vxy = a.eta * ((vx[l + PX] - vx[l]) + (vy[l + 1] - vy[l])) * a.inv_h;
                    const T viz_x = a.eta * ((vn1[0] - vx[l]) + (vz[l + 1] - vz[l])) * a.inv_h;
                    s_F[3][l] = quarter * (gy[l] + gy[l + 1]) * (vx[l] + vx[l + PX]) - vxy;
                    s_F[4][l] = quarter * (gz[l] + gz[l + 1]) * (vx[l] + vn1[0]) - viz_x;
                } else {                    // -y row: edge fluxes xy, zy
                    const T vxy = a.eta * ((vx[l + PX] - vx[l]) + (vy[l + 1] - vy[l])) * a.inv_h;
                    const T viz_y = a.eta * ((vn1[1] - vy[l]) + (vz[l + PX] - vz[l])) * a.inv_h;
                    s_F[2][l] = quarter * (gx[l] + gx[l + PX]) * (vy[l] + vy[l + 1]) - vxy;
                    s_F[5][l] = quarter * (gz[l] + gz[l + PX]) * (vy[l] + vn1[1]) - viz_y;
                }
            }
            vzm1 = vz[l];
        }
        __syncthreads();

        // ---- phase X: update of plane k (z-momentum: of plane k-1, done
        // above), then plane k+1 into G/V and density of plane k+2 into P
        if (own) {
            if (!PREP) {
                if (!EARLY) {
                    const uint32_t su = soff(zk);
                    if (STAGE != 0) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) un[c] = bload<T, CP_NT>(run[c], vo, su);
                    }
                    if (NOISE) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) nn[c] = bload<T, CP_NT>(rnn[c], vo, su);
                    }
                }
                const int l = lo;
                // own column of plane k: only this thread writes it below
                const T us[4] = {Pk[l], s_G[0][l], s_G[1][l], s_G[2][l]};
                T d[3];
                d[0] = -dth * mflux;
                d[1] = -dth * ((s_F[0][l + 1] - s_F[0][l]) + (s_F[2][l] - s_F[2][l - PX]) + (Pxz - Pxz_m));
                d[2] = -dth * ((s_F[1][l + PX] - s_F[1][l]) + (s_F[3][l] - s_F[3][l - 1]) + (Pyz - Pyz_m));
                lag_d = -dth * ((s_F[4][l] - s_F[4][l - 1]) + (s_F[5][l] - s_F[5][l - PX]));
                if (NOISE) {
                    d[1] += nn[0];
                    d[2] += nn[1];
                    lag_d += nn[2];
                }
                lag_u = us[3];
                lag_n = un[3];
                const uint32_t so = soff(zk);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T v = STAGE == 0 ? us[c] + d[c] : a.ra * un[c] + a.rb * (us[c] + d[c]);
                    bstore(v, rout[c], vo, so);
                }
            }
            Pxz_m = Pxz;
            Pyz_m = Pyz;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                s_G[c][lo] = S.g[c];
                s_V[c][lo] = vn[c];
            }
            Pw[lo] = S.rn;
        }
        if (r1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                s_G[c][l1] = S.g1[c];
                s_V[c][l1] = vn1[c];
            }
            Pw[l1] = S.rn1;
        }
        if (r2) Pw[l2] = S.rn2;
        if (k + 3 <= z1) load_set(S, k + 3);
        __syncthreads();
    };
    using T1 = std::integral_constant<bool, true>;
    using F0 = std::integral_constant<bool, false>;
    iteration(T1{}, T1{}, z0 - 1, SO);
    for (int k = z0; k < z1; k += 2) {
        iteration(F0{}, F0{}, k, SE);
        if (k + 1 < z1) iteration(T1{}, F0{}, k + 1, SO);
    }
    // ---- tail: zz flux of plane z1 finishes the z-momentum of plane z1-1
    if (own) {
        const int l = lo;
        const T *Pz = s_P[z1 & 1];
        const T *gz = s_G[2], *vx = s_V[0], *vy = s_V[1], *vz = s_V[2];
        const T pi = a.cf2 * Pz[l] + (pex_own + ext_pressure_z(a, wrap(z1, nz)));
        const T dvz = vz[l] - vzm;
        const T div = ((vx[l] - vx[l - 1]) + (vy[l] - vy[l - PX]) + dvz) * a.inv_h;
        const T Pzz = pi + quarter * (gz[l] + gzm) * (vz[l] + vzm) -
                      (2 * a.eta * dvz * a.inv_h + a.lam * div);
        fin_gz(z1 - 1, Pzz);
    }
}

#define IC_STAGE_ATTRS                   \
    __global__ __launch_bounds__(STAGE_THREADS) \
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 4)))

template <typename T, int STAGE, bool NOISE, bool FULL>
IC_STAGE_ATTRS void stage_kernel(const StageArgs<T> a) {
    __shared__ T s_lds[STAGE_LDS];
    critical_path();
    stage_body<T, STAGE, NOISE, FULL>(a, xcd_tile(blockIdx.x, a.gx * a.gy * a.gz), s_lds);
}

// One RK stage over the tiles of many contexts at once (ensembles): block b
// runs tile tile[b] of context member[b] with that context's arguments
// (args[member]); noise and whole-tile specialisation per context.
template <typename T, int STAGE>
IC_STAGE_ATTRS void stage_kernel_batched(const IC_CONST StageArgs<T> *args,
                                         const IC_CONST int32_t *member,
                                         const IC_CONST int32_t *tile) {
    __shared__ T s_lds[STAGE_LDS];
    const StageArgs<T> &a = from_const(args[member[blockIdx.x]]);
    const int t = tile[blockIdx.x];
    if (a.noise[0][0]) {
        if (a.full)
            stage_body<T, STAGE, true, true>(a, t, s_lds);
        else
            stage_body<T, STAGE, true, false>(a, t, s_lds);
    } else {
        if (a.full)
            stage_body<T, STAGE, false, true>(a, t, s_lds);
        else
            stage_body<T, STAGE, false, false>(a, t, s_lds);
    }
}
#undef IC_STAGE_ATTRS

// ---------------------------------------------------------------------------
// Stochastic increments of one step.  The stochastic flux enters each RK
// stage linearly and does not depend on the state, so its increment
// N(W) = -(dt/h) div(-Sigma(W)) is computed once per step for W_A and W_B
// and written as N1 = N(W_A) - sqrt(3) N(W_B), N2 = N(W_A) + sqrt(3) N(W_B),
// N3 = N(W_A) for the three stages (App. A, weak third-order combinations).
// Same column march as the stage kernel; ring cells draw only the normals
// their neighbours need.
// ---------------------------------------------------------------------------
template <typename T>
struct NoiseArgs {
    T *out[2][9];             // the two noise sets; step m writes set m & 1
    int nx, ny, nz, tz, gx, gy, gz;
    T dt_h, sd, st, so, s3;
    NoiseKey nk;              // step word taken from *step at run time
    const StepState *step;
    uint32_t ahead;           // 0: noise of the step in flight, 1: of the next step
    BMPoly poly;              // FP64 Box-Muller series (unused in FP32)
};

// Tile of the noise kernel: 32 x NY columns, NY = NTY<T> (32 in FP32, 16
// in FP64, whose registers and LDS are twice as wide) when the noise runs on
// its own, NBG = 8 for the next step's noise run in the background (below).
// Waves 0-3 also take one side each of the ring of cells whose stresses the
// tile's faces need (+x column: xx, +y row: yy, -x column: xy and xz, -y row:
// xy and yz), so each SIMD carries one ring wave (NY >= 8: four waves).
constexpr int NTX = 32, NPX = NTX + 2;
template <typename T>
constexpr int NTY = sizeof(T) == 4 ? 32 : 16;
constexpr int NBG = 8;

__device__ __forceinline__ int nidx(int lx, int ly) { return (ly + 1) * NPX + (lx + 1); }

// Noise of tile t (of a.gx x a.gy x a.gz tiles of 32 x NY columns); s_S
// holds the current plane's stresses [W_A, W_B][xx, yy, xy, xz, yz].  The
// values do not depend on the tile shape.
template <typename T, int NY>
__device__ __forceinline__ void noise_body(const NoiseArgs<T> &args, int t,
                                           T (*s_S)[5][NPX * (NY + 2)]) {
    NoiseArgs<T> a = args;
    const uint32_t m = args.step->cur + args.ahead;
    a.nk.step = m;
    T *const *out = (m & 1u) ? args.out[1] : args.out[0];
    const int nx = a.nx, ny = a.ny, nz = a.nz, tz = a.tz;
    const int plane = nx * ny;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int bx = t % a.gx, by = (t / a.gx) % a.gy, bz = t / (a.gx * a.gy);
    const int x0 = bx * NTX, y0 = by * NY, z0 = bz * tz;
    const int W = min(NTX, nx - x0), Wy = min(NY, ny - y0), z1 = min(z0 + tz, nz);
    const int lx = tid % NTX, ly = tid / NTX;
    const bool own = lx < W && ly < Wy;
    const int li = nidx(lx, ly);
    const int own_xy = own ? (y0 + ly) * nx + x0 + lx : 0;
    // ring cell of waves 0-3
    int h_x = 0, h_y = 0;
    bool ring = false;
    if (wave == 0 && lane < Wy) { ring = true; h_x = W; h_y = lane; }
    else if (wave == 1 && lane < W) { ring = true; h_x = lane; h_y = Wy; }
    else if (wave == 2 && lane < Wy) { ring = true; h_x = -1; h_y = lane; }
    else if (wave == 3 && lane < W) { ring = true; h_x = lane; h_y = -1; }
    const int h_l = nidx(h_x, h_y);
    const int h_xy = wrap(y0 + h_y, ny) * nx + wrap(x0 + h_x, nx);

    // own stresses: planes k and k+1 (all components), plane k-1 (xz, yz)
    T SAc[6] = {0, 0, 0, 0, 0, 0}, SBc[6] = {0, 0, 0, 0, 0, 0};
    T SAp[6] = {0, 0, 0, 0, 0, 0}, SBp[6] = {0, 0, 0, 0, 0, 0};
    if (own) {
        T A[6] = {0, 0, 0, 0, 0, 0}, B[6] = {0, 0, 0, 0, 0, 0};
        cell_normals<T, SEL_EDGE>((uint32_t)(wrap(z0 - 1, nz) * plane + own_xy), a.nk, A, B, args.poly);
        ll_stress(A, a.sd, a.st, a.so, SAp);
        ll_stress(B, a.sd, a.st, a.so, SBp);
        cell_normals<T, SEL_ALL>((uint32_t)(z0 * plane + own_xy), a.nk, A, B, args.poly);
        ll_stress(A, a.sd, a.st, a.so, SAc);
        ll_stress(B, a.sd, a.st, a.so, SBc);
    }
    for (int k = z0; k < z1; ++k) {
        T SAn[6] = {0, 0, 0, 0, 0, 0}, SBn[6] = {0, 0, 0, 0, 0, 0};
        if (own) {
            T A[6], B[6];
            cell_normals<T, SEL_ALL>((uint32_t)(wrap(k + 1, nz) * plane + own_xy), a.nk, A, B, args.poly);
            ll_stress(A, a.sd, a.st, a.so, SAn);
            ll_stress(B, a.sd, a.st, a.so, SBn);
            const int l = li;
            s_S[0][0][l] = SAc[0]; s_S[0][1][l] = SAc[1]; s_S[0][2][l] = SAc[3];
            s_S[0][3][l] = SAc[4]; s_S[0][4][l] = SAc[5];
            s_S[1][0][l] = SBc[0]; s_S[1][1][l] = SBc[1]; s_S[1][2][l] = SBc[3];
            s_S[1][3][l] = SBc[4]; s_S[1][4][l] = SBc[5];
        }
        if (ring) {
            T A[6] = {0, 0, 0, 0, 0, 0}, B[6] = {0, 0, 0, 0, 0, 0}, SA[6], SB[6];
            const uint32_t hc = (uint32_t)(k * plane + h_xy);
            if (wave < 2)
                cell_normals<T, SEL_DIAG>(hc, a.nk, A, B, args.poly);
            else
                cell_normals<T, SEL_EDGE>(hc, a.nk, A, B, args.poly);
            ll_stress(A, a.sd, a.st, a.so, SA);
            ll_stress(B, a.sd, a.st, a.so, SB);
            const int l = h_l;
            if (wave == 0) {
                s_S[0][0][l] = SA[0]; s_S[1][0][l] = SB[0];
            } else if (wave == 1) {
                s_S[0][1][l] = SA[1]; s_S[1][1][l] = SB[1];
            } else if (wave == 2) {
                s_S[0][2][l] = SA[3]; s_S[1][2][l] = SB[3];
                s_S[0][3][l] = SA[4]; s_S[1][3][l] = SB[4];
            } else {
                s_S[0][2][l] = SA[3]; s_S[1][2][l] = SB[3];
                s_S[0][4][l] = SA[5]; s_S[1][4][l] = SB[5];
            }
        }
        __syncthreads();
        if (own) {
            const int l = li;
            T N[2][3];
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                const T *Sc = w == 0 ? SAc : SBc, *Sp = w == 0 ? SAp : SBp, *Sn = w == 0 ? SAn : SBn;
                const T *xx = s_S[w][0], *yy = s_S[w][1], *xy = s_S[w][2], *xz = s_S[w][3],
                        *yz = s_S[w][4];
                N[w][0] = a.dt_h * ((xx[l + 1] - xx[l]) + (xy[l] - xy[l - NPX]) + (Sc[4] - Sp[4]));
                N[w][1] = a.dt_h * ((yy[l + NPX] - yy[l]) + (xy[l] - xy[l - 1]) + (Sc[5] - Sp[5]));
                N[w][2] = a.dt_h * ((Sn[2] - Sc[2]) + (xz[l] - xz[l - 1]) + (yz[l] - yz[l - NPX]));
            }
            const int g = k * plane + own_xy;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                // streamed past L2 (read once per stage, much later)
                __builtin_nontemporal_store(N[0][c] - a.s3 * N[1][c], &out[c][g]);
                __builtin_nontemporal_store(N[0][c] + a.s3 * N[1][c], &out[3 + c][g]);
                __builtin_nontemporal_store(N[0][c], &out[6 + c][g]);
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            SAp[c] = SAc[c]; SBp[c] = SBc[c];
            SAc[c] = SAn[c]; SBc[c] = SBn[c];
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(NTX * NTY<T>) void noise_kernel(const NoiseArgs<T> args) {
    __shared__ T s_S[2][5][NPX * (NTY<T> + 2)];
    noise_body<T, NTY<T>>(args, xcd_tile(blockIdx.x, args.gx * args.gy * args.gz), s_S);
}

// The next step's noise in the background of the step in flight: one
// 256-thread block per CU (one wave per SIMD, 56 VGPRs) walks the 32 x 8
// tiles.  Its waves keep the default issue priority below the stage and
// particle kernels, so they run in the issue slots those latency-bound
// kernels leave idle, and a CU gives up one stage block to them instead of
// two for a 1024-thread tile.  Measured at 256^3 (FP32 ms per step): 1.022
// with one 32 x 32 tile per block, 0.973 like this; 224 or 288 blocks
// (some CUs without one or with two) 1.008 and 1.010, 160 blocks 1.18 (the
// noise then outlasts the step).
template <typename T>
__global__ __launch_bounds__(NTX * NBG) void noise_kernel_bg(const NoiseArgs<T> args) {
    __shared__ T s_S[2][5][NPX * (NBG + 2)];
    const int nt = args.gx * args.gy * args.gz;
    for (int t = blockIdx.x; t < nt; t += gridDim.x) noise_body<T, NBG>(args, t, s_S);
}

// Noise of many contexts in one launch: block b draws tile tile[b] of
// context member[b].
template <typename T>
__global__ __launch_bounds__(NTX * NTY<T>) void noise_kernel_batched(
    const IC_CONST NoiseArgs<T> *args, const IC_CONST int32_t *member,
    const IC_CONST int32_t *tile) {
    __shared__ T s_S[2][5][NPX * (NTY<T> + 2)];
    noise_body<T, NTY<T>>(from_const(args[member[blockIdx.x]]), tile[blockIdx.x], s_S);
}

// ---------------------------------------------------------------------------
// Per-step scalars (StepState).  One wave: every lane reads the step before
// lane 0 advances it.
// ---------------------------------------------------------------------------
struct DriveArgs {
    int nmodes;
    double dt;
    double amp[IC_MAX_MODES], omega[IC_MAX_MODES], phase[IC_MAX_MODES];
};

__device__ __forceinline__ void step_begin_body(StepState *st, const DriveArgs &d) {
    const int lane = threadIdx.x;
    const int64_t n = st->step;
    // stage times t^n, t^n + dt, t^n + dt/2 (App. A, stage pressures)
    if (lane < 3 * IC_MAX_MODES) {
        const int stage = lane / IC_MAX_MODES, m = lane % IC_MAX_MODES;
        const double tn = (double)n * d.dt;
        const double t = stage == 0 ? tn : (stage == 1 ? tn + d.dt : tn + 0.5 * d.dt);
        st->amp[stage][m] = m < d.nmodes ? d.amp[m] * sin(d.omega[m] * t + d.phase[m]) : 0.0;
    }
    __syncthreads();
    if (lane == 0) {
        st->cur = (uint32_t)(n & 0xFFFFFFFF);
        st->step = n + 1;
    }
}

__global__ __launch_bounds__(64) void k_step_begin(StepState *st, const DriveArgs d) {
    step_begin_body(st, d);
}

// One block per context.
__global__ __launch_bounds__(64) void k_step_begin_batched(StepState *const IC_CONST *st,
                                                           const IC_CONST DriveArgs *d) {
    step_begin_body(st[blockIdx.x], from_const(d[blockIdx.x]));
}

__global__ void k_set_step(StepState *st, int64_t n) {
    if (threadIdx.x == 0) st->step = n;
}

// ---------------------------------------------------------------------------
// Particle kernels: one 64-lane wave per particle.  Lanes 0..17 hold the 18
// kernel weights (3 axes x {cell, face} x 3 points) and lanes 18..23 the
// first point indices; 27-point sums are reduced with a fixed butterfly, so
// results do not depend on timing.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct Grid {
    int nx, ny, nz;
    double h, inv_h, rho0;
};

struct WaveKernel {
    double w;   // lanes 0..17
    int first;  // lanes 18..23
};

__device__ __forceinline__ WaveKernel wave_kernel(const Grid &G, const double q[3]) {
    const int lane = threadIdx.x & 63;
    const int n[3] = {G.nx, G.ny, G.nz};
    WaveKernel k{0.0, 0};
    if (lane < 24) {
        const int ax = lane < 18 ? lane / 6 : (lane - 18) % 3;
        const bool face = lane < 18 ? (lane % 6) >= 3 : lane >= 21;
        const int d = lane < 18 ? lane % 3 : 0;
        double w;
        const int f = axis_point(q[ax], G.inv_h, n[ax], face, d, &w);
        if (lane < 18)
            k.w = w;
        else
            k.first = f;
    }
    return k;
}

// Weight and element index of kernel point pt (0..26, x fastest) of location
// kind (0 cell, 1+a face a), and the index of the next point along axis nb
// (-1: none).  Every lane of the wave must call it.
__device__ __forceinline__ void wave_point(const Grid &G, const WaveKernel &k, int kind, int pt,
                                           size_t *idx, double *w, int nb = -1,
                                           size_t *idx_nb = nullptr) {
    const int d[3] = {pt % 3, (pt / 3) % 3, pt / 9};
    const int n[3] = {G.nx, G.ny, G.nz};
    double wt = 1.0;
    int c[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const bool face = kind == ax + 1;
        wt *= __shfl(k.w, ax * 6 + (face ? 3 : 0) + d[ax], 64);
        c[ax] = wrap(__shfl(k.first, 18 + (face ? 3 : 0) + ax, 64) + d[ax], n[ax]);
    }
    *idx = ((size_t)c[2] * G.ny + c[1]) * G.nx + c[0];
    *w = wt;
    if (nb >= 0) {
        c[nb] = c[nb] + 1 == n[nb] ? 0 : c[nb] + 1;
        *idx_nb = ((size_t)c[2] * G.ny + c[1]) * G.nx + c[0];
    }
}

// Sums over the 81 (component, point) pairs of the face kernels at q:
// sv[a] = J_a (g^a / rho_face^a) and, if sm, sm[a] = J_a rho_face^a.
template <typename T>
__device__ __forceinline__ void wave_face_sums(const Grid &G, const T *const f[4], const double q[3],
                                               double sv[3], double *sm) {
    const int lane = threadIdx.x & 63;
    const WaveKernel k = wave_kernel(G, q);
    double av[3] = {0, 0, 0}, am[3] = {0, 0, 0};
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int item = lane + 64 * it;
        const bool valid = item < 81;
        const int itm = valid ? item : 0;
        const int ax = itm / 27, pt = itm % 27;
        size_t i, j;
        double w;
        wave_point(G, k, ax + 1, pt, &i, &w, ax, &j);
        if (valid) {
            const double rf = G.rho0 + 0.5 * ((double)f[0][i] + (double)f[0][j]);
            av[ax] += w * ((double)f[1 + ax][i] / rf);
            am[ax] += w * rf;
        }
    }
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        sv[ax] = wave_sum(av[ax]);
        if (sm) sm[ax] = wave_sum(am[ax]);
    }
}

template <typename T>
struct PartArgs {
    Grid G;
    const T *f[4];
    int np;
    double dt, V, L[3];
    double *q, *u, *me, *eps, *ks, *qeq, *fext;
    double *qh, *jv_old, *F, *Vt, *du, *mf, *omega, *jv_new;
    int32_t *bc, *bf;
    double *wc, *wf;
    double *sum_f, *sum_l;
    int32_t *flag;
};

// Substeps 1-2 and the kernel data at q^{n+1/2} (App. A).
template <typename T>
__device__ __forceinline__ void pre_body(const PartArgs<T> &a, int p) {
    const int lane = threadIdx.x & 63;
    double q[3] = {a.q[3 * p], a.q[3 * p + 1], a.q[3 * p + 2]};
    // A non-finite position or velocity (NaN or inf in the fields) would
    // reach the integer point indices of the kernel: it is replaced by 0 and
    // reported through flag[2].
    bool bad = false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
        if (!isfinite(q[ax])) {
            bad = true;
            q[ax] = 0.0;
        }
    double U[3];
    wave_face_sums<T>(a.G, a.f, q, U, nullptr);           // J^n v^n at q^n
    double qh[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        qh[ax] = wrap_pos(q[ax] + 0.5 * a.dt * U[ax], a.L[ax]);
        if (!isfinite(qh[ax])) {
            bad = true;
            qh[ax] = 0.0;
        }
    }
    if (bad && lane == 0) a.flag[2] = 1;
    double jv[3];
    wave_face_sums<T>(a.G, a.f, qh, jv, nullptr);         // J^{n+1/2} v^n
    const WaveKernel k = wave_kernel(a.G, qh);
    // Omega of the first RK stage: eps V J(rho^n - rho0) at q^{n+1/2}
    double om;
    {
        size_t i;
        double w;
        wave_point(a.G, k, 0, lane < 27 ? lane : 0, &i, &w);
        om = wave_sum(lane < 27 ? w * (double)a.f[0][i] : 0.0);
    }
    if (lane < 18) {
        const int ax = lane / 6, d = lane % 3;
        if ((lane % 6) < 3)
            a.wc[9 * p + 3 * ax + d] = k.w;
        else
            a.wf[9 * p + 3 * ax + d] = k.w;
    } else if (lane < 24) {
        if (lane < 21)
            a.bc[3 * p + lane - 18] = k.first;
        else
            a.bf[3 * p + lane - 21] = k.first;
    } else if (lane < 27) {
        const int ax = lane - 24;
        if (ax == 0) a.omega[p] = a.eps[p] * a.V * om;
        a.qh[3 * p + ax] = qh[ax];
        a.jv_old[3 * p + ax] = jv[ax];
        a.F[3 * p + ax] = -a.ks[p] * min_image(qh[ax] - a.qeq[3 * p + ax], a.L[ax]) +
                          a.fext[3 * p + ax];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_pre(const PartArgs<T> a) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    critical_path();
    pre_body(a, p);
}

// Waves of many contexts in one launch: wave w handles particle
// local[w] of context member[w] (member < 0: no work).
struct WaveMap {
    const IC_CONST int32_t *member, *local;
    int nwaves;
};

template <typename T>
__global__ __launch_bounds__(256) void k_pre_batched(const IC_CONST PartArgs<T> *args,
                                                     const WaveMap map) {
    const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= map.nwaves) return;
    pre_body(from_const(args[map.member[w]]), map.local[w]);
}

// Kernel data for standalone spreading at caller positions.
__global__ __launch_bounds__(256) void k_weights(const Grid G, int np, const double *q, double *qh,
                                                 int32_t *bc, int32_t *bf, double *wc, double *wf) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= np) return;
    const int lane = threadIdx.x & 63;
    const double L[3] = {G.nx * G.h, G.ny * G.h, G.nz * G.h};
    const double x[3] = {wrap_pos(q[3 * p], L[0]), wrap_pos(q[3 * p + 1], L[1]),
                         wrap_pos(q[3 * p + 2], L[2])};
    const WaveKernel k = wave_kernel(G, x);
    if (lane < 18) {
        const int ax = lane / 6, d = lane % 3;
        if ((lane % 6) < 3)
            wc[9 * p + 3 * ax + d] = k.w;
        else
            wf[9 * p + 3 * ax + d] = k.w;
    } else if (lane < 24) {
        if (lane < 21)
            bc[3 * p + lane - 18] = k.first;
        else
            bf[3 * p + lane - 21] = k.first;
    } else if (lane < 27) {
        qh[3 * p + lane - 24] = x[lane - 24];
    }
}

// u := J v at the particle positions (no-slip initial velocity).
template <typename T>
__global__ __launch_bounds__(256) void k_init_u(const PartArgs<T> a) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    const int lane = threadIdx.x & 63;
    const double q[3] = {a.q[3 * p], a.q[3 * p + 1], a.q[3 * p + 2]};
    double U[3];
    wave_face_sums<T>(a.G, a.f, q, U, nullptr);
    if (lane < 3) a.u[3 * p + lane] = U[lane];
}

// Standalone J of a caller field.
template <typename T>
__global__ __launch_bounds__(256) void k_interp(const Grid G, int np, const double *q, int kind,
                                                const T *field, double *out) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= np) return;
    const int lane = threadIdx.x & 63;
    const double L[3] = {G.nx * G.h, G.ny * G.h, G.nz * G.h};
    double qq[3] = {wrap_pos(q[3 * p], L[0]), wrap_pos(q[3 * p + 1], L[1]),
                    wrap_pos(q[3 * p + 2], L[2])};
    // a non-finite position gives NaN (it never reaches the point indices)
    const bool bad = !(isfinite(qq[0]) && isfinite(qq[1]) && isfinite(qq[2]));
    if (bad) qq[0] = qq[1] = qq[2] = 0.0;
    const double nan_or_0 = bad ? __builtin_nan("") : 0.0;
    const WaveKernel k = wave_kernel(G, qq);
    if (kind != IC_FACES) {
        size_t i;
        double w;
        wave_point(G, k, kind, lane < 27 ? lane : 0, &i, &w);
        double s = lane < 27 ? w * (double)field[i] : 0.0;
        s = wave_sum(s);
        if (lane == 0) out[p] = s + nan_or_0;
        return;
    }
    // three consecutive face fields (x, y, z components), out [n][3]
    const size_t ncell = (size_t)G.nx * G.ny * G.nz;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        size_t i;
        double w;
        wave_point(G, k, 1 + ax, lane < 27 ? lane : 0, &i, &w);
        double s = lane < 27 ? w * (double)field[ax * ncell + i] : 0.0;
        s = wave_sum(s);
        if (lane == 0) out[3 * p + ax] = s + nan_or_0;
    }
}

// ---------------------------------------------------------------------------
// Binning of particles into stage blocks.  A particle is listed for every
// block whose cells, ring of halo cells or extra plane its kernel points
// (within [f-1, f+2] of f = floor(q/h) per axis) can reach; each list is
// sorted by the particle's first plane relative to the block (key) and id.
// ---------------------------------------------------------------------------
struct BinArgs {
    int np, nx, ny, nz, gx, gy, gz, nblk, tz;
    double inv_h;
    const double *qh;
    const int32_t *bc;   // first cell index of each particle's stencil (overlap test)
    int32_t *count, *off, *cursor, *list, *key;
};

// Distinct tile indices (tile size ts) touched by positions f-2 .. f+3.
__device__ __forceinline__ int axis_tiles(int f, int n, int ts, int out[3]) {
    int cnt = 0;
    for (int s = f - 2; s <= f + 3; ++s) {
        const int t = ((s % n) + n) % n / ts;
        bool seen = false;
        for (int c = 0; c < cnt; ++c) seen |= out[c] == t;
        if (!seen && cnt < 3) out[cnt++] = t;
    }
    return cnt;
}

__device__ __forceinline__ int particle_blocks(const BinArgs &b, int p, int out[27]) {
    int tx[3], ty[3], tz[3];
    const double *q = b.qh + 3 * p;
    const int cx = axis_tiles((int)floor(q[0] * b.inv_h), b.nx, TX, tx);
    const int cy = axis_tiles((int)floor(q[1] * b.inv_h), b.ny, TY, ty);
    const int cz = axis_tiles((int)floor(q[2] * b.inv_h), b.nz, b.tz, tz);
    int n = 0;
    for (int k = 0; k < cz; ++k)
        for (int j = 0; j < cy; ++j)
            for (int i = 0; i < cx; ++i) out[n++] = (tz[k] * b.gy + ty[j]) * b.gx + tx[i];
    return n;
}

__global__ __launch_bounds__(256) void k_bin_count(const BinArgs b) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= b.np) return;
    int bl[27];
    const int n = particle_blocks(b, p, bl);
    for (int c = 0; c < n; ++c) atomicAdd(&b.count[bl[c]], 1);
}

// Exclusive scan of count into off (and cursor); re-zeroes count.
__global__ __launch_bounds__(1024) void k_bin_scan(const BinArgs b) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int chunk = (b.nblk + nt - 1) / nt;
    const int lo = min(tid * chunk, b.nblk), hi = min(lo + chunk, b.nblk);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += b.count[i];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < nt; o <<= 1) {
        const int v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int i = lo; i < hi; ++i) {
        const int c = b.count[i];
        b.off[i] = run;
        b.cursor[i] = run;
        b.count[i] = 0;
        run += c;
    }
    if (tid == nt - 1) b.off[b.nblk] = part[nt - 1];
}

__global__ __launch_bounds__(256) void k_bin_fill(const BinArgs b) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= b.np) return;
    int bl[27];
    const int n = particle_blocks(b, p, bl);
    for (int c = 0; c < n; ++c) {
        const int slot = atomicAdd(&b.cursor[bl[c]], 1);
        b.list[slot] = p;
    }
}

// One wave per block list.  The list (filled in arbitrary order) is sorted
// by particle id, then coloured greedily in that order: a candidate takes
// the smallest colour not used by an earlier candidate whose point box
// overlaps its own (|d bc| <= 3 on every axis, periodic), so candidates of
// one colour touch disjoint grid points.  The list is finally ordered by
// (colour, id) and key[] holds the colour.  Lists longer than the LDS buffer
// are sorted by lane 0 and get one colour per candidate.
constexpr int SORT_CAP = 512;

__device__ __forceinline__ bool boxes_overlap(const int a[3], const int b[3], const int n[3]) {
    bool all = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        int d = a[ax] - b[ax];
        if (d < 0) d = -d;
        d = min(d, n[ax] - d);
        all = all && d <= 3;
    }
    return all;
}

__global__ __launch_bounds__(64) void k_bin_sort(const BinArgs b) {
    __shared__ int32_t sp[SORT_CAP], sq[SORT_CAP], sc[SORT_CAP], sb[SORT_CAP][3];
    const int blk = blockIdx.x;
    const int lane = threadIdx.x;
    const int s0 = b.off[blk], n = b.off[blk + 1] - s0;
    if (n == 0) return;
    if (n > SORT_CAP) {
        if (lane != 0) return;
        for (int m = s0 + 1; m < s0 + n; ++m) {
            const int v = b.list[m];
            int j = m - 1;
            while (j >= s0 && b.list[j] > v) {
                b.list[j + 1] = b.list[j];
                --j;
            }
            b.list[j + 1] = v;
        }
        for (int i = 0; i < n; ++i) b.key[s0 + i] = i;
        return;
    }
    const int nn[3] = {b.nx, b.ny, b.nz};
    for (int i = lane; i < n; i += 64) sq[i] = b.list[s0 + i];
    __syncthreads();
    // rank sort by particle id (ids in one list are distinct)
    for (int i = lane; i < n; i += 64) {
        const int pi = sq[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) rank += sq[j] < pi;
        sp[rank] = pi;
    }
    __syncthreads();
    for (int i = lane; i < n; i += 64) {
        const int pi = sp[i];
        sb[i][0] = b.bc[3 * pi];
        sb[i][1] = b.bc[3 * pi + 1];
        sb[i][2] = b.bc[3 * pi + 2];
    }
    __syncthreads();
    // greedy colouring in id order (the wave takes candidates one at a time)
    for (int i = 0; i < n; ++i) {
        unsigned long long used = 0;
        int far = 0;   // colours >= 64 in use by an overlapping candidate
        for (int j = lane; j < i; j += 64) {
            if (boxes_overlap(sb[i], sb[j], nn)) {
                if (sc[j] < 64) used |= 1ull << sc[j];
                else far = max(far, sc[j] + 1);
            }
        }
        for (int o = 32; o >= 1; o >>= 1) {
            used |= __shfl_xor(used, o, 64);
            far = max(far, __shfl_xor(far, o, 64));
        }
        const int c = ~used ? __builtin_ctzll(~used) : max(64, far);
        if (lane == 0) sc[i] = c;
        __syncthreads();
    }
    // order by (colour, id)
    for (int i = lane; i < n; i += 64) {
        const int ci = sc[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) rank += sc[j] < ci || (sc[j] == ci && j < i);
        b.list[s0 + rank] = sp[i];
        b.key[s0 + rank] = ci;
    }
}

// Binning of a small particle set (at most SB_CAP particles, so no tile
// list exceeds SB_CAP entries, and at most SB_MAXBLK tiles) in one
// workgroup: counts and cursors in LDS, the exclusive scan as in k_bin_scan,
// then each wave sorts and colours whole tile lists exactly as k_bin_sort
// does.  One launch instead of four: on small grids the binning sits on the
// step's critical path, where launch latency dominates it.
constexpr int SB_THREADS = 1024, SB_WAVES = SB_THREADS / 64;
constexpr int SB_CAP = 128;
constexpr int SB_MAXBLK = 4096;

// LDS written by some lanes of a wave, read by others after this point
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(SB_THREADS) void k_bin_small(const BinArgs b) {
    __shared__ int32_t s_cur[SB_MAXBLK];
    __shared__ int32_t s_part[SB_THREADS];
    __shared__ int32_t w_q[SB_WAVES][SB_CAP], w_p[SB_WAVES][SB_CAP], w_c[SB_WAVES][SB_CAP];
    __shared__ int32_t w_b[SB_WAVES][SB_CAP][3];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = b.nblk;
    for (int i = tid; i < nblk; i += SB_THREADS) s_cur[i] = 0;
    __syncthreads();
    for (int p = tid; p < b.np; p += SB_THREADS) {
        int bl[27];
        const int n = particle_blocks(b, p, bl);
        for (int c = 0; c < n; ++c) atomicAdd(&s_cur[bl[c]], 1);
    }
    __syncthreads();
    // exclusive scan of the counts: offsets to memory, cursors in LDS
    const int chunk = (nblk + SB_THREADS - 1) / SB_THREADS;
    const int lo = min(tid * chunk, nblk), hi = min(lo + chunk, nblk);
    int sum = 0;
    for (int i = lo; i < hi; ++i) sum += s_cur[i];
    s_part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < SB_THREADS; o <<= 1) {
        const int v = tid >= o ? s_part[tid - o] : 0;
        __syncthreads();
        s_part[tid] += v;
        __syncthreads();
    }
    int run = s_part[tid] - sum;
    for (int i = lo; i < hi; ++i) {
        const int cnt = s_cur[i];
        b.off[i] = run;
        s_cur[i] = run;
        run += cnt;
    }
    if (tid == SB_THREADS - 1) b.off[nblk] = s_part[SB_THREADS - 1];
    __syncthreads();
    for (int p = tid; p < b.np; p += SB_THREADS) {
        int bl[27];
        const int n = particle_blocks(b, p, bl);
        for (int c = 0; c < n; ++c) b.list[atomicAdd(&s_cur[bl[c]], 1)] = p;
    }
    __syncthreads();
    // each wave: whole tile lists, sorted by id, coloured greedily, ordered
    // by (colour, id)
    const int nn[3] = {b.nx, b.ny, b.nz};
    int32_t *sq = w_q[wave], *sp = w_p[wave], *sc = w_c[wave];
    int32_t(*sb)[3] = w_b[wave];
    for (int blk = wave; blk < nblk; blk += SB_WAVES) {
        const int s0 = b.off[blk], n = b.off[blk + 1] - s0;
        if (n == 0) continue;
        for (int i = lane; i < n; i += 64) sq[i] = b.list[s0 + i];
        wave_lds_sync();
        for (int i = lane; i < n; i += 64) {
            const int pi = sq[i];
            int rank = 0;
            for (int j = 0; j < n; ++j) rank += sq[j] < pi;
            sp[rank] = pi;
        }
        wave_lds_sync();
        for (int i = lane; i < n; i += 64) {
            const int pi = sp[i];
            sb[i][0] = b.bc[3 * pi];
            sb[i][1] = b.bc[3 * pi + 1];
            sb[i][2] = b.bc[3 * pi + 2];
        }
        wave_lds_sync();
        for (int i = 0; i < n; ++i) {
            unsigned long long used = 0;
            int far = 0;
            for (int j = lane; j < i; j += 64) {
                if (boxes_overlap(sb[i], sb[j], nn)) {
                    if (sc[j] < 64) used |= 1ull << sc[j];
                    else far = max(far, sc[j] + 1);
                }
            }
            for (int o = 32; o >= 1; o >>= 1) {
                used |= __shfl_xor(used, o, 64);
                far = max(far, __shfl_xor(far, o, 64));
            }
            const int c = ~used ? __builtin_ctzll(~used) : max(64, far);
            if (lane == 0) sc[i] = c;
            wave_lds_sync();
        }
        for (int i = lane; i < n; i += 64) {
            const int ci = sc[i];
            int rank = 0;
            for (int j = 0; j < n; ++j) rank += sc[j] < ci || (sc[j] == ci && j < i);
            b.list[s0 + rank] = sp[i];
            b.key[s0 + rank] = ci;
        }
        wave_lds_sync();   // before the wave's next list reuses its buffers
    }
}

// Spreading S of caller values onto one field (ic_spread), owner-computes,
// one stage block per workgroup.  The block's candidates arrive ordered by
// (colour, id) from k_bin_sort; candidates of one colour touch disjoint
// points, so each colour is one parallel round over (candidate, point) items
// and every point receives its sums in the same order on every run (no float
// atomics): field += f_p w_p / h^3 over the 27 points of one location kind.
template <typename T>
struct SparseArgs {
    int nx, ny, nz, tz;
    double inv_h3;
    const int32_t *blk_off, *blk_list, *blk_color, *bc, *bf;
    const double *wc, *wf;
    const double *val;   // f[p]
    int kind;            // IC_CELL or IC_FACE_*
    T *field;
};

constexpr int SP_CAP = 64;    // candidates staged in LDS at a time
constexpr int SP_THREADS = 256;   // threads of a sparse block (one stage tile)
constexpr int SP_BATCH = 4;   // items per thread whose loads are issued together

template <typename T>
__global__ __launch_bounds__(SP_THREADS) void k_sparse(const SparseArgs<T> a) {
    __shared__ int32_t s_bc[SP_CAP][3], s_bf[SP_CAP][3], s_col[SP_CAP];
    __shared__ double s_wc[SP_CAP][9], s_wf[SP_CAP][9], s_v[SP_CAP];
    const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const int cb = a.blk_off[blk], ce = a.blk_off[blk + 1];
    if (cb == ce) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int n[3] = {nx, ny, nz};
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * a.tz;
    const int lo[3] = {x0, y0, z0};
    const int wd[3] = {min(TX, nx - x0), min(TY, ny - y0), min(a.tz, nz - z0)};
    const int tid = threadIdx.x;
    const int fa = a.kind - 1;   // face axis, -1: cells
    constexpr int per = 27;

    for (int c0 = cb; c0 < ce; c0 += SP_CAP) {
        const int nc = min(SP_CAP, ce - c0);
        __syncthreads();
        for (int i = tid; i < nc; i += SP_THREADS) {
            const int pid = a.blk_list[c0 + i];
            s_col[i] = a.blk_color[c0 + i];
            for (int d = 0; d < 3; ++d) {
                s_bc[i][d] = a.bc[3 * pid + d];
                s_bf[i][d] = a.bf[3 * pid + d];
            }
            for (int d = 0; d < 9; ++d) {
                s_wc[i][d] = a.wc[9 * pid + d];
                s_wf[i][d] = a.wf[9 * pid + d];
            }
            s_v[i] = a.val[pid];
        }
        __syncthreads();
        for (int r0 = 0; r0 < nc;) {
            // one colour: candidates [r0, r1)
            const int col = s_col[r0];
            int r1 = r0 + 1;
            while (r1 < nc && s_col[r1] == col) ++r1;
            const int items = (r1 - r0) * per;
            for (int base = 0; base < items; base += SP_BATCH * SP_THREADS) {
                size_t gi[SP_BATCH];
                double add[SP_BATCH];
                bool ok[SP_BATCH];
#pragma unroll
                for (int bi = 0; bi < SP_BATCH; ++bi) {
                    const int it = base + bi * SP_THREADS + tid;
                    ok[bi] = false;
                    gi[bi] = 0;
                    add[bi] = 0.0;
                    if (it >= items) continue;
                    const int cq = it / per;
                    const int ci = r0 + cq;
                    const int pt = it - cq * per;
                    // point index along each axis relative to the stencil start
                    const int d[3] = {pt % 3, (pt / 3) % 3, pt / 9};
                    int pos[3];
                    bool in = true;
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax) {
                        const int start = ax == fa ? s_bf[ci][ax] : s_bc[ci][ax];
                        pos[ax] = wrap(start + d[ax], n[ax]);
                        in = in && pos[ax] >= lo[ax] && pos[ax] < lo[ax] + wd[ax];
                    }
                    if (!in) continue;
                    // cell weights on the axes other than the face axis
                    double po = 1.0;
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax)
                        if (ax != fa) po *= s_wc[ci][3 * ax + d[ax]];
                    const double w = fa < 0 ? po : po * s_wf[ci][3 * fa + d[fa]];
                    ok[bi] = true;
                    gi[bi] = ((size_t)pos[2] * ny + pos[1]) * nx + pos[0];
                    add[bi] = s_v[ci] * w * a.inv_h3;
                }
                // the batch's points are distinct: issue every load, then every store
                T old[SP_BATCH];
#pragma unroll
                for (int bi = 0; bi < SP_BATCH; ++bi) old[bi] = ok[bi] ? a.field[gi[bi]] : (T)0;
#pragma unroll
                for (int bi = 0; bi < SP_BATCH; ++bi)
                    if (ok[bi]) a.field[gi[bi]] = (T)((double)old[bi] + add[bi]);
            }
            __syncthreads();
            r0 = r1;
        }
    }
}

// ---------------------------------------------------------------------------
// Particle clusters of one step.  A cluster is a connected component of the
// graph that joins two particles when their influence boxes intersect (the
// 4 x 4 x 4 points [bc-1, bc+2] per axis that a particle's stage terms,
// no-slip correction and gathers reach).  Particles of different clusters
// touch disjoint grid points, so one wave per cluster can update the grid
// with plain read-modify-writes; inside a cluster the wave takes its members
// one after another in ascending id, so every point receives its sums in the
// same order on every run (no float atomics).  Most clusters hold one
// particle.
// Union-find: parent[p] is p or a smaller id; a union hooks the larger root
// onto the smaller one with a compare-and-swap, so the root of a component
// is its smallest id whatever order the unions run in.
// ---------------------------------------------------------------------------
struct ClusterArgs {
    int np;
    int32_t *parent;   // union-find forest
    int32_t *root;     // root of each particle
    int32_t *cnt;      // members of the cluster whose root is p (0 for non-roots)
    int32_t *off;      // exclusive prefix sums of cnt ([np + 1])
    int32_t *cursor;   // fill cursors
    int32_t *list;     // members grouped by root, in fill order
};

__device__ __forceinline__ int uf_find(int32_t *parent, int x) {
    for (;;) {
        const int p = __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p == x) return x;
        x = p;
    }
}

__device__ __forceinline__ void uf_union(int32_t *parent, int a, int b) {
    for (;;) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        int expected = a;
        if (__hip_atomic_compare_exchange_strong(parent + a, &expected, b, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

// One wave per tile list: unions of the listed particles whose influence
// boxes intersect.  Every point of a particle's box lies in a tile the
// particle is listed for, so two intersecting boxes share the tile of a
// common point and every edge of the graph is seen.  Lists longer than
// UNION_CAP are merged whole: a cluster larger than needed is still
// processed correctly, only more serially.
constexpr int UNION_CAP = 256;

__global__ __launch_bounds__(64) void k_bin_union(const BinArgs b, int32_t *parent) {
    __shared__ int32_t s_id[UNION_CAP], s_b[UNION_CAP][3];
    const int blk = blockIdx.x, lane = threadIdx.x;
    const int s0 = b.off[blk], n = b.off[blk + 1] - s0;
    if (n <= 1) return;
    if (n > UNION_CAP) {
        for (int i = 1 + lane; i < n; i += 64) uf_union(parent, b.list[s0], b.list[s0 + i]);
        return;
    }
    for (int i = lane; i < n; i += 64) {
        const int p = b.list[s0 + i];
        s_id[i] = p;
        s_b[i][0] = b.bc[3 * p];
        s_b[i][1] = b.bc[3 * p + 1];
        s_b[i][2] = b.bc[3 * p + 2];
    }
    __syncthreads();
    const int nn[3] = {b.nx, b.ny, b.nz};
    for (int i = 1; i < n; ++i)
        for (int j = lane; j < i; j += 64)
            if (boxes_overlap(s_b[i], s_b[j], nn)) uf_union(parent, s_id[i], s_id[j]);
}

// parent[p] = p, cnt[p] = 0 (before the unions of a step)
__global__ __launch_bounds__(256) void k_cl_init(const ClusterArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.np) return;
    a.parent[p] = p;
    a.cnt[p] = 0;
}

__global__ __launch_bounds__(256) void k_cl_count(const ClusterArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.np) return;
    const int r = uf_find(a.parent, p);
    a.root[p] = r;
    atomicAdd(a.cnt + r, 1);
}

// Exclusive scan of cnt into off and cursor (one workgroup).
__global__ __launch_bounds__(1024) void k_cl_scan(const ClusterArgs a) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int chunk = (a.np + nt - 1) / nt;
    const int lo = min(tid * chunk, a.np), hi = min(lo + chunk, a.np);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += a.cnt[i];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < nt; o <<= 1) {
        const int v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int i = lo; i < hi; ++i) {
        a.off[i] = run;
        a.cursor[i] = run;
        run += a.cnt[i];
    }
    if (tid == nt - 1) a.off[a.np] = part[nt - 1];
}

__global__ __launch_bounds__(256) void k_cl_fill(const ClusterArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.np) return;
    a.list[atomicAdd(a.cursor + a.root[p], 1)] = p;
}

// Clusters of at most CL_SMALL_CAP particles in one workgroup: every pair
// tested directly, the forest and the counts in LDS, then the same root,
// cnt, off and list arrays as the general path (members of a cluster listed
// in ascending id).  One launch instead of seven on small particle sets.
constexpr int CL_SMALL_CAP = 512;

struct ClusterSmallArgs {
    ClusterArgs ca;
    const int32_t *bc;
    int nx, ny, nz;
};

__device__ __forceinline__ void cl_small_body(const ClusterArgs &a, const int32_t *bc, int nx,
                                              int ny, int nz) {
    __shared__ int32_t s_par[CL_SMALL_CAP], s_b[CL_SMALL_CAP][3], s_cnt[CL_SMALL_CAP + 1];
    const int tid = threadIdx.x, np = a.np;
    const int nn[3] = {nx, ny, nz};
    for (int p = tid; p < np; p += blockDim.x) {
        s_par[p] = p;
        s_cnt[p] = 0;
        s_b[p][0] = bc[3 * p];
        s_b[p][1] = bc[3 * p + 1];
        s_b[p][2] = bc[3 * p + 2];
    }
    __syncthreads();
    // hook each particle onto the smallest overlapping id below it, then
    // take minima along the chains until nothing changes (a component's root
    // is its smallest id, as in the general path)
    for (int p = tid; p < np; p += blockDim.x) {
        int m = p;
        for (int q = 0; q < p; ++q)
            if (boxes_overlap(s_b[p], s_b[q], nn)) {
                m = q;
                break;
            }
        s_par[p] = m;
    }
    __syncthreads();
    // min-label propagation over the edges: repeat until stable
    __shared__ int changed;
    for (;;) {
        if (tid == 0) changed = 0;
        __syncthreads();
        for (int p = tid; p < np; p += blockDim.x) {
            int m = s_par[s_par[p]];
            for (int q = 0; q < np; ++q)
                if (q != p && boxes_overlap(s_b[p], s_b[q], nn)) m = min(m, s_par[q]);
            if (m < s_par[p]) {
                s_par[p] = m;
                changed = 1;
            }
        }
        __syncthreads();
        if (!changed) break;
        __syncthreads();
    }
    for (int p = tid; p < np; p += blockDim.x) {
        a.root[p] = s_par[p];
        atomicAdd(&s_cnt[s_par[p]], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int p = 0; p < np; ++p) {
            const int c = s_cnt[p];
            a.off[p] = run;
            a.cnt[p] = c;
            s_cnt[p] = run;
            run += c;
        }
        a.off[np] = run;
        // members in ascending id: one pass in id order
        for (int p = 0; p < np; ++p) a.list[s_cnt[s_par[p]]++] = p;
    }
}

__global__ __launch_bounds__(1024) void k_cl_small(const ClusterSmallArgs a) {
    cl_small_body(a.ca, a.bc, a.nx, a.ny, a.nz);
}

// One workgroup per context.
__global__ __launch_bounds__(1024) void k_cl_small_batched(const IC_CONST ClusterSmallArgs *a) {
    const ClusterSmallArgs &c = from_const(a[blockIdx.x]);
    cl_small_body(c.ca, c.bc, c.nx, c.ny, c.nz);
}

// Next member above `last` of the cluster list[o, o + k) (its smallest id
// greater than last).
__device__ __forceinline__ int cluster_next(const int32_t *list, int o, int k, int last) {
    const int lane = threadIdx.x & 63;
    int best = 0x7fffffff;
    for (int i = lane; i < k; i += 64) {
        const int v = list[o + i];
        if (v > last && v < best) best = v;
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) best = min(best, __shfl_xor(best, s, 64));
    return best;
}

// A wave's view of one particle's kernel data: lanes 0..8 the cell
// weights wc[axis][point], lanes 9..17 the face weights, lanes 18..20 the
// first cell index and 21..23 the first face index per axis.
struct WaveStencil {
    double w;
    int i;
};

__device__ __forceinline__ WaveStencil load_stencil(const int32_t *bc, const int32_t *bf,
                                                    const double *wc, const double *wf, int p) {
    const int lane = threadIdx.x & 63;
    WaveStencil s{0.0, 0};
    if (lane < 9)
        s.w = wc[9 * p + lane];
    else if (lane < 18)
        s.w = wf[9 * p + lane - 9];
    else if (lane < 21)
        s.i = bc[3 * p + lane - 18];
    else if (lane < 24)
        s.i = bf[3 * p + lane - 21];
    return s;
}
__device__ __forceinline__ double st_wc(const WaveStencil &s, int ax, int d) {
    return __shfl(s.w, 3 * ax + d, 64);
}
__device__ __forceinline__ double st_wf(const WaveStencil &s, int ax, int d) {
    return __shfl(s.w, 9 + 3 * ax + d, 64);
}
__device__ __forceinline__ int st_bc(const WaveStencil &s, int ax) { return __shfl(s.i, 18 + ax, 64); }
__device__ __forceinline__ int st_bf(const WaveStencil &s, int ax) { return __shfl(s.i, 21 + ax, 64); }

// Grid updates of one particle become visible to the next member's loads
// (same wave, same workgroup).
__device__ __forceinline__ void member_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Stage terms of one RK stage (App. A, stage pressures; reading R18): for
// each particle, g^a += b [-(dt/h) (P(i+a) - P(i)) + dt F^a w_a / h^3] with
// P = Omega w / h^3, over the 4 x 3 x 3 faces of each component its pressure
// and force reach; and the next stage's Omega = eps V J(drho_next) from the
// density this stage wrote (27 products in the lanes, a butterfly sum).
template <typename T>
struct StagePassArgs {
    int nx, ny, nz, np;
    double inv_h3, b, dt_h, dt, V;
    const int32_t *root, *cnt, *off, *list;
    const int32_t *bc, *bf;
    const double *wc, *wf;
    const double *F, *omega, *eps;
    double *omega_next;   // nullptr after the last stage
    const T *drho_next;
    T *g[3];
};

template <typename T>
__device__ __forceinline__ void stage_terms_of(const StagePassArgs<T> &a, int p) {
    const int lane = threadIdx.x & 63;
    const int n[3] = {a.nx, a.ny, a.nz};
    const WaveStencil s = load_stencil(a.bc, a.bf, a.wc, a.wf, p);
    const double om = a.omega[p];
    const double Fp[3] = {a.F[3 * p], a.F[3 * p + 1], a.F[3 * p + 2]};
    int bcv[3], sh[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        bcv[ax] = st_bc(s, ax);
        int d = bcv[ax] - st_bf(s, ax);   // 0 or 1 up to the period
        if (d < 0) d += n[ax];
        sh[ax] = d;
    }
    size_t gi[2];
    double add[2];
    int cmp[2];
    bool ok[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int item = lane + 64 * it;
        ok[it] = item < 108;
        const int itm = ok[it] ? item : 0;
        const int fa = itm / 36, pt = itm - 36 * fa;
        int d[3];
        if (fa == 0) {
            d[0] = pt % 4; d[1] = (pt / 4) % 3; d[2] = pt / 12;
        } else if (fa == 1) {
            d[0] = pt % 3; d[1] = (pt / 3) % 4; d[2] = pt / 12;
        } else {
            d[0] = pt % 3; d[1] = (pt / 3) % 3; d[2] = pt / 9;
        }
        int pos[3];
        double po = 1.0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            pos[ax] = wrap(bcv[ax] - (ax == fa ? 1 : 0) + d[ax], n[ax]);
            // every lane takes part in the shuffles; the face axis reads
            // point 0 and does not use it
            const double wv = st_wc(s, ax, ax == fa ? 0 : d[ax]);
            if (ax != fa) po *= wv;
        }
        const int dc = d[fa];
        const int of = dc - 1 + sh[fa];
        const double wpos = st_wc(s, fa, dc >= 1 ? dc - 1 : 0);
        const double wnb = st_wc(s, fa, dc <= 2 ? dc : 2);
        const double wff = st_wf(s, fa, (of >= 0 && of <= 2) ? of : 0);
        const double w_pos = dc >= 1 ? po * wpos : 0.0;
        const double w_nb = dc <= 2 ? po * wnb : 0.0;
        const double w_f = (of >= 0 && of <= 2) ? po * wff : 0.0;
        const double dP = om * (w_nb - w_pos) * a.inv_h3;
        const double fw = Fp[fa] * w_f * a.inv_h3;
        gi[it] = ((size_t)pos[2] * a.ny + pos[1]) * a.nx + pos[0];
        add[it] = a.b * (-a.dt_h * dP + a.dt * fw);
        cmp[it] = fa;
    }
    // The next stage's Omega reads the density this stage wrote, which the
    // particle terms do not change: its gather goes out with the momentum
    // loads instead of after the stores.
    double v = 0.0;
    if (a.omega_next) {
        const int l27 = lane < 27 ? lane : 0;
        const int d0 = l27 % 3, d1 = (l27 / 3) % 3, d2 = l27 / 9;
        const double w = st_wc(s, 0, d0) * st_wc(s, 1, d1) * st_wc(s, 2, d2);
        if (lane < 27) {
            const int x = wrap(bcv[0] + d0, a.nx), y = wrap(bcv[1] + d1, a.ny),
                      z = wrap(bcv[2] + d2, a.nz);
            v = w * (double)a.drho_next[((size_t)z * a.ny + y) * a.nx + x];
        }
    }
    T old[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) old[it] = ok[it] ? a.g[cmp[it]][gi[it]] : (T)0;
#pragma unroll
    for (int it = 0; it < 2; ++it)
        if (ok[it]) a.g[cmp[it]][gi[it]] = (T)((double)old[it] + add[it]);
    if (a.omega_next) {
        v = wave_sum(v);
        if (lane == 0) a.omega_next[p] = a.eps[p] * a.V * v;
    }
}

template <typename T>
__device__ __forceinline__ void cl_stage_body(const StagePassArgs<T> &a, int p) {
    if (a.root[p] != p) return;
    const int k = a.cnt[p];
    if (k == 1) {
        stage_terms_of(a, p);
        return;
    }
    const int o = a.off[p];
    int m = p;   // the root is the cluster's smallest id
    for (int i = 0; i < k; ++i) {
        if (i) {
            member_fence();
            m = cluster_next(a.list, o, k, m);
        }
        stage_terms_of(a, m);
    }
}

// At most 96 VGPRs (5 waves per SIMD, no spills): with its density gather
// issued beside the momentum loads the pass would otherwise take 100 and
// drop to 4 waves, which cost more than the shorter chain saves.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_cl_stage(
    const StagePassArgs<T> a) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    critical_path();
    cl_stage_body(a, p);
}

template <typename T>
__global__ __launch_bounds__(256) void k_cl_stage_batched(const IC_CONST StagePassArgs<T> *args,
                                                          const WaveMap map) {
    const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= map.nwaves) return;
    cl_stage_body(from_const(args[map.member[w]]), map.local[w]);
}

// Substeps 4-7 for one cluster per wave (App. A): the impulse and particle
// velocity of every member from the unconstrained state, V~ = J v~,
// m_f = V J rho_face, u^{n+1} = u^n + m_f/(m_e + m_f) (V~ - u^n); then the
// momentum-conserving corrections g += rho_face V S(u^{n+1} - V~) member
// after member; then the full-step positions q^{n+1} = q^n + dt/2
// J^{n+1/2}(v^{n+1} + v^n) and the window sums from the corrected state.
// Reading R6: every member's V~ comes from the uncorrected state.  A
// non-finite V~, m_f or position raises flag[2] (and the position keeps its
// old value); m_e + m_f <= 0 raises flag[0].
template <typename T>
struct PostPassArgs {
    PartArgs<T> pa;
    const int32_t *root, *cnt, *off, *list;
    T *g[3];        // momentum of U^{n+1}, corrected in place
    double inv_h3;
};

template <typename T>
__device__ __forceinline__ void impulse_of(const PartArgs<T> &a, int p) {
    const int lane = threadIdx.x & 63;
    const double qh[3] = {a.qh[3 * p], a.qh[3 * p + 1], a.qh[3 * p + 2]};
    double Vt[3], sm[3];
    wave_face_sums<T>(a.G, a.f, qh, Vt, sm);
    if (lane < 3) {
        const int ax = lane;
        const double me = a.me[p];
        const double mf = a.V * sm[ax];
        const double u = a.u[3 * p + ax];
        double un = u + mf / (me + mf) * (Vt[ax] - u);
        double du = a.V * (un - Vt[ax]);
        if (!isfinite(Vt[ax]) || !isfinite(mf)) {
            a.flag[2] = 1;
            un = u;
            du = 0.0;
        } else if (!(me + mf > 0.0)) {
            a.flag[0] = 1;
        }
        a.Vt[3 * p + ax] = un;  // u^{n+1}
        a.du[3 * p + ax] = du;
        a.mf[3 * p + ax] = mf;
    }
}

template <typename T>
__device__ __forceinline__ void noslip_of(const PostPassArgs<T> &c, int p) {
    const PartArgs<T> &a = c.pa;
    const int lane = threadIdx.x & 63;
    const int n[3] = {a.G.nx, a.G.ny, a.G.nz};
    const WaveStencil s = load_stencil(a.bc, a.bf, a.wc, a.wf, p);
    const T *drho = a.f[0];
    int bcv[3], bfv[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        bcv[ax] = st_bc(s, ax);
        bfv[ax] = st_bf(s, ax);
    }
    size_t gi[2];
    double add[2];
    int cmp[2];
    bool ok[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int item = lane + 64 * it;
        ok[it] = item < 81;
        const int itm = ok[it] ? item : 0;
        const int fa = itm / 27, pt = itm - 27 * fa;
        const int d[3] = {pt % 3, (pt / 3) % 3, pt / 9};
        int pos[3];
        double po = 1.0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            pos[ax] = wrap((ax == fa ? bfv[ax] : bcv[ax]) + d[ax], n[ax]);
            const double wv = st_wc(s, ax, d[ax]);
            if (ax != fa) po *= wv;
        }
        const double wf = st_wf(s, fa, d[fa]);
        int nb[3] = {pos[0], pos[1], pos[2]};
        nb[fa] = nb[fa] + 1 == n[fa] ? 0 : nb[fa] + 1;
        const size_t g = ((size_t)pos[2] * a.G.ny + pos[1]) * a.G.nx + pos[0];
        const size_t j = ((size_t)nb[2] * a.G.ny + nb[1]) * a.G.nx + nb[0];
        double v = 0.0;
        if (ok[it]) {
            const double rf = a.G.rho0 + 0.5 * ((double)drho[g] + (double)drho[j]);
            v = rf * a.du[3 * p + fa] * (po * wf) * c.inv_h3;
        }
        gi[it] = g;
        add[it] = v;
        cmp[it] = fa;
    }
    T old[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) old[it] = ok[it] ? c.g[cmp[it]][gi[it]] : (T)0;
#pragma unroll
    for (int it = 0; it < 2; ++it)
        if (ok[it]) c.g[cmp[it]][gi[it]] = (T)((double)old[it] + add[it]);
}

template <typename T>
__device__ __forceinline__ void final_of(const PartArgs<T> &a, int p) {
    const int lane = threadIdx.x & 63;
    const double qh[3] = {a.qh[3 * p], a.qh[3 * p + 1], a.qh[3 * p + 2]};
    double jv[3];
    wave_face_sums<T>(a.G, a.f, qh, jv, nullptr);
    if (lane < 3) {
        const int ax = lane;
        const double q = a.q[3 * p + ax];
        const double qn = q + 0.5 * a.dt * (jv[ax] + a.jv_old[3 * p + ax]);
        if (isfinite(qn))
            a.q[3 * p + ax] = wrap_pos(qn, a.L[ax]);
        else
            a.flag[2] = 1;
        const double un = a.Vt[3 * p + ax];
        const double F = a.F[3 * p + ax];
        const double lam = a.me[p] * (un - a.u[3 * p + ax]) / a.dt - F;
        a.sum_f[3 * p + ax] += -(F - a.fext[3 * p + ax]);
        a.sum_l[3 * p + ax] += lam;
        a.u[3 * p + ax] = un;
        a.jv_new[3 * p + ax] = jv[ax];
    }
}

// Substeps 4-7 of a particle alone in its cluster: no other particle
// touches its points, so one gather serves all three phases.  Each lane keeps
// its face points' index, weight, face density and momentum from the
// impulse gather, writes the corrected momentum and sums J v^{n+1} from the
// values it wrote, with the same products and sums as a fresh gather.
template <typename T, bool FINAL>
__device__ __forceinline__ void post_single(const PostPassArgs<T> &c, int p) {
    const PartArgs<T> &a = c.pa;
    const int lane = threadIdx.x & 63;
    const double qh[3] = {a.qh[3 * p], a.qh[3 * p + 1], a.qh[3 * p + 2]};
    // lanes 0-2 load their component's particle state with the position, so
    // these loads share one round trip instead of following the gathers
    const int lb = lane < 3 ? lane : 0;
    const double me = a.me[p], u = a.u[3 * p + lb];
    double q = 0.0, jvo = 0.0, Fp = 0.0, fx = 0.0, sf = 0.0, sl = 0.0;
    if (FINAL && lane < 3) {
        q = a.q[3 * p + lb];
        jvo = a.jv_old[3 * p + lb];
        Fp = a.F[3 * p + lb];
        fx = a.fext[3 * p + lb];
        sf = a.sum_f[3 * p + lb];
        sl = a.sum_l[3 * p + lb];
    }
    const WaveKernel k = wave_kernel(a.G, qh);
    size_t gi[2];
    double w[2], rf[2], gt[2];
    int ax[2];
    bool ok[2];
    double av[3] = {0, 0, 0}, am[3] = {0, 0, 0};
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int item = lane + 64 * it;
        ok[it] = item < 81;
        const int itm = ok[it] ? item : 0;
        ax[it] = itm / 27;
        size_t j;
        wave_point(a.G, k, ax[it] + 1, itm % 27, &gi[it], &w[it], ax[it], &j);
        rf[it] = 0.0;
        gt[it] = 0.0;
        if (ok[it]) {
            rf[it] = a.G.rho0 + 0.5 * ((double)a.f[0][gi[it]] + (double)a.f[0][j]);
            gt[it] = (double)a.f[1 + ax[it]][gi[it]];
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (b == ax[it]) {
                    av[b] += w[it] * (gt[it] / rf[it]);
                    am[b] += w[it] * rf[it];
                }
        }
    }
    double Vt[3], sm[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        Vt[b] = wave_sum(av[b]);
        sm[b] = wave_sum(am[b]);
    }
    // substeps 4-5 (lanes 0-2, one component each)
    double du = 0.0, un = 0.0;
    if (lane < 3) {
        const int b = lane;
        const double mf = a.V * sm[b];
        un = u + mf / (me + mf) * (Vt[b] - u);
        du = a.V * (un - Vt[b]);
        if (!isfinite(Vt[b]) || !isfinite(mf)) {
            a.flag[2] = 1;
            un = u;
            du = 0.0;
        } else if (!(me + mf > 0.0)) {
            a.flag[0] = 1;
        }
        a.Vt[3 * p + b] = un;
        a.du[3 * p + b] = du;
        a.mf[3 * p + b] = mf;
    }
    // substep 6 on the kept points, then J v^{n+1} from the written values
    double jvs[3] = {0, 0, 0};
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double dua = __shfl(du, ax[it], 64);
        if (ok[it]) {
            const T gn = (T)(gt[it] + rf[it] * dua * w[it] * c.inv_h3);
            c.g[ax[it]][gi[it]] = gn;
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (b == ax[it]) jvs[b] += w[it] * ((double)gn / rf[it]);
        }
    }
    if (!FINAL) return;
    double jv[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) jv[b] = wave_sum(jvs[b]);
    if (lane < 3) {
        const int b = lane;
        const double qn = q + 0.5 * a.dt * (jv[b] + jvo);
        if (isfinite(qn))
            a.q[3 * p + b] = wrap_pos(qn, a.L[b]);
        else
            a.flag[2] = 1;
        const double lam = me * (un - u) / a.dt - Fp;
        a.sum_f[3 * p + b] = sf + -(Fp - fx);
        a.sum_l[3 * p + b] = sl + lam;
        a.u[3 * p + b] = un;
        a.jv_new[3 * p + b] = jv[b];
    }
}

// FINAL = false: substeps 4-6 only (the reverse mode's recomputation, which
// keeps positions and window sums untouched).
template <typename T, bool FINAL = true>
__device__ __forceinline__ void cl_post_body(const PostPassArgs<T> &c, int p) {
    const PartArgs<T> &a = c.pa;
    if (c.root[p] != p) return;
    const int k = c.cnt[p], o = c.off[p];
    if (k == 1) {
        post_single<T, FINAL>(c, p);
        return;
    }
    int m = p;
    for (int i = 0; i < k; ++i) {
        if (i) m = cluster_next(c.list, o, k, m);
        impulse_of(a, m);
    }
    member_fence();
    m = p;
    for (int i = 0; i < k; ++i) {
        if (i) {
            m = cluster_next(c.list, o, k, m);
        }
        noslip_of(c, m);
        member_fence();
    }
    if (!FINAL) return;
    m = p;
    for (int i = 0; i < k; ++i) {
        if (i) m = cluster_next(c.list, o, k, m);
        final_of(a, m);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cl_post(const PostPassArgs<T> c) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= c.pa.np) return;
    critical_path();
    cl_post_body(c, p);
}

// The last stage's particle terms and substeps 4-7 in one launch: a
// cluster's points are written by its own wave alone, so its substeps 4-7
// can follow its stage terms without waiting for the other clusters (the
// same operations in the same order as k_cl_stage then k_cl_post).
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_cl_last(
    const StagePassArgs<T> a, const PostPassArgs<T> c) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    critical_path();
    cl_stage_body(a, p);
    member_fence();
    cl_post_body(c, p);
}

template <typename T>
__global__ __launch_bounds__(256) void k_cl_noslip(const PostPassArgs<T> c) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= c.pa.np) return;
    cl_post_body<T, false>(c, p);
}

template <typename T>
__global__ __launch_bounds__(256) void k_cl_post_batched(const IC_CONST PostPassArgs<T> *args,
                                                         const WaveMap map) {
    const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= map.nwaves) return;
    cl_post_body(from_const(args[map.member[w]]), map.local[w]);
}

// k_cl_last for every member of an ensemble in one launch.
template <typename T>
__global__ __launch_bounds__(256) void k_cl_last_batched(
    const IC_CONST StagePassArgs<T> *sargs, const IC_CONST PostPassArgs<T> *pargs,
    const WaveMap map) {
    const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= map.nwaves) return;
    const int m = map.member[w], p = map.local[w];
    cl_stage_body(from_const(sargs[m]), p);
    member_fence();
    cl_post_body(from_const(pargs[m]), p);
}

// ---------------------------------------------------------------------------
// Adjoint (reverse mode) of one deterministic, particle-free RK3 step: the
// transpose of the stage increment Delta(U) (conservative staggered flux of
// the stage kernel, App. A) applied to an adjoint state lambda, one cell per
// thread, neighbours read through the caches, arithmetic in the context
// precision.
//   k_adj_tile: the momentum part mu_g (incl. the v = g / rho_face chain), the
//     face-density adjoints mu_rf = d/d rho_face and mu_p (sum of the
//     centre-flux adjoints); writes the momentum components of the RK
//     combination, mu_rf and mu_rpart = c_f^2 mu_p + (sum_a mu_rf_a) / 2,
//     and per-block partial sums of mu_p prof_m (drive-amplitude gradient).
//   k_adj_rho: mu_rho = mu_rpart + (sum_a mu_rf_a[i - e_a]) / 2 and the
//     density component of the RK combination.
// RK combination of the reversed stages (U^{n+1} = U^n/3 + 2/3 (U2 + D(U2)),
// U2 = 3/4 U^n + 1/4 (U1 + D(U1)), U1 = U^n + D(U^n)):
//   ADJ_FIRST (stage 3): out = cs (lam + mu), acc  = ds lam
//   ADJ_MID   (stage 2): out = cs (lam + mu), acc += ds lam
//   ADJ_LAST  (stage 1): out = acc + cs (lam + mu)
// ---------------------------------------------------------------------------
enum AdjMode { ADJ_FIRST = 0, ADJ_MID = 1, ADJ_LAST = 2 };

struct DriveCoef {
    int axis[IC_MAX_MODES];
    double c[IC_MAX_MODES];   // weight of the stage times sin(omega t_s + phase)
};

template <typename T>
struct AdjArgs {
    const T *U[4];      // stage input (drho, gx, gy, gz)
    const T *lam[4];    // adjoint of the stage output
    T *out[4];          // adjoint of the stage input (RK-combined)
    T *acc[4];          // dL/dU^n accumulator
    T *murf[3];         // mu_rf per axis
    T *mur;             // c_f^2 mu_p + (sum_a mu_rf_a) / 2
    int nx, ny, nz;
    int mode;
    double rho0, cf2, eta, lam_b, k, inv_h, cs, ds;   // lam_b = zeta - 2 eta / 3, k = dt / h
    int nmodes, pstride;
    DriveCoef dc;
    const double *prof;
    double *partial;    // [IC_MAX_MODES][nbp], one slot per block
    int nbp;
    int tz, gx, gy, gz; // tiled momentum pass: z extent and tile counts
};

template <typename T>
__device__ __forceinline__ void adj_combine(const AdjArgs<T> &a, int c, int j, T l, T mu) {
    // pointwise and touched once per launch: streamed past L2, which keeps
    // the stencil planes the neighbouring blocks re-read
    const T o = (T)a.cs * (l + mu);
    if (a.mode == ADJ_LAST) {
        __builtin_nontemporal_store(__builtin_nontemporal_load(&a.acc[c][j]) + o, &a.out[c][j]);
    } else {
        __builtin_nontemporal_store(o, &a.out[c][j]);
        const T prev = a.mode == ADJ_MID ? __builtin_nontemporal_load(&a.acc[c][j]) : (T)0;
        __builtin_nontemporal_store(prev + (T)a.ds * l, &a.acc[c][j]);
    }
}

__device__ __forceinline__ void cell_of(int j, int nx, int ny, int &x, int &y, int &z) {
    const int r = j / nx;
    x = j - r * nx;
    z = r / ny;
    y = r - z * ny;
}

// Momentum pass of the transposed stage increment: a tile of ATX x ATY
// columns marches over tz planes in z (adjoint_tz).  LDS holds three planes (k-1, k, k+1)
// of lambda_g, g and v = g / rho_face and three density planes (k, k+1, k+2)
// over the tile plus a one-cell halo, so a cell's neighbour reads come from
// LDS and each velocity is divided out once per point.  lambda_rho is read
// from memory (four values per cell), and the two density values one cell
// beyond the halo that the halo's own velocities need come from registers:
// 40.8 KB of LDS in FP32 (4 blocks per CU), 81.6 KB in FP64 (2).  Per plane
// k: commit the prefetched plane k+1 to LDS (forming its v), issue the loads
// of plane k+2 into registers, barrier, update plane k, barrier.  The march
// is unrolled by three so every LDS slot is a compile-time constant.
constexpr int ATX = 32, ATY = 8, ATHREADS = ATX * ATY;
constexpr int APX = ATX + 2, APY = ATY + 2, APS = APX * APY;   // local x, y in [-1, AT]
constexpr int APTS = (APS + ATHREADS - 1) / ATHREADS;            // halo points per thread

// Reciprocal for the adjoint's v = g / rho_face: the hardware estimate
// (1 ulp) in FP32, a correctly rounded division in FP64.
__device__ __forceinline__ float adj_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double adj_rcp(double x) { return 1.0 / x; }

// FP32: the hint of 3 waves per SIMD lets the compiler use 126 VGPRs without
// scratch, which still runs 4 waves per SIMD (a hint of 4 made it keep 119
// and spill 36 B per lane).
template <typename T>
__global__ __launch_bounds__(ATHREADS)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 2))) void k_adj_tile(const AdjArgs<T> a) {
    using C = T;
    __shared__ __attribute__((aligned(16))) T s_lg[3][3][APS];   // also the reduction scratch
    __shared__ T s_g[3][3][APS], s_v[3][3][APS], s_r[3][APS];
    const int nx = a.nx, ny = a.ny, nz = a.nz, plane = nx * ny;
    int bx, by, bz;
    {
        const int nblk = a.gx * a.gy * a.gz, b = blockIdx.x;
        const int per = nblk / 8, rem = nblk % 8, xcd = b % 8, idx = b / 8;
        const int t = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
        bx = t % a.gx;
        by = (t / a.gx) % a.gy;
        bz = t / (a.gx * a.gy);
    }
    const int x0 = bx * ATX, y0 = by * ATY, z0 = bz * a.tz;
    const int W = min(ATX, nx - x0), Wy = min(ATY, ny - y0), z1 = min(z0 + a.tz, nz);
    const int tid = threadIdx.x, lx = tid % ATX, ly = tid / ATX;
    const bool own = lx < W && ly < Wy;
    const int c0 = (ly + 1) * APX + (lx + 1);
    const int own_xy = own ? (y0 + ly) * nx + x0 + lx : 0;
    const int own_x1 = own ? (y0 + ly) * nx + wrap(x0 + lx + 1, nx) : 0;
    const int own_y1 = own ? wrap(y0 + ly + 1, ny) * nx + x0 + lx : 0;
    const C rho0 = (C)a.rho0, half = (C)0.5, quarter = (C)0.25;
    // this thread's halo points (x in [-1, W], y in [-1, Wy]); points on the
    // high edges also need the density one cell further out
    int pi[APTS], pg[APTS], pgx[APTS], pgy[APTS];
    bool pin[APTS], pex[APTS], pey[APTS];
#pragma unroll
    for (int r = 0; r < APTS; ++r) {
        const int i = tid + r * ATHREADS;
        const int px = i % APX - 1, py = i / APX - 1;
        pi[r] = i;
        pin[r] = i < APS && px <= W && py <= Wy;
        pex[r] = pin[r] && px == W;
        pey[r] = pin[r] && py == Wy;
        const int gx = wrap(x0 + px, nx), gy = wrap(y0 + py, ny);
        pg[r] = pin[r] ? gy * nx + gx : 0;
        pgx[r] = pex[r] ? gy * nx + wrap(x0 + px + 1, nx) : 0;
        pgy[r] = pey[r] ? wrap(y0 + py + 1, ny) * nx + gx : 0;
    }
    T f_lg[APTS][3], f_g[APTS][3], f_rn[APTS], f_rx[APTS], f_ry[APTS];
    // loads of plane z, the density of plane z + 1, and the edge densities of plane z
    auto fetch = [&](int z) {
        const int o0 = wrap(z, nz) * plane, o1 = wrap(z + 1, nz) * plane;
#pragma unroll
        for (int r = 0; r < APTS; ++r) {
            if (pin[r]) {
                f_rn[r] = a.U[0][o1 + pg[r]];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    f_lg[r][c] = a.lam[1 + c][o0 + pg[r]];
                    f_g[r][c] = a.U[1 + c][o0 + pg[r]];
                }
            }
            if (pex[r]) f_rx[r] = a.U[0][o0 + pgx[r]];
            if (pey[r]) f_ry[r] = a.U[0][o0 + pgy[r]];
        }
    };
    // plane z into slot S (the density of plane z is in slot S already; the
    // density of plane z + 1 goes to slot S + 1)
    auto commit = [&](auto S_) {
        constexpr int S = decltype(S_)::value, S1 = (S + 1) % 3;
#pragma unroll
        for (int r = 0; r < APTS; ++r) {
            const int i = pi[r];
            if (pin[r]) {
                s_r[S1][i] = f_rn[r];
                const C r0 = s_r[S][i];
                const C rx = pex[r] ? (C)f_rx[r] : (C)s_r[S][i + 1];
                const C ry = pey[r] ? (C)f_ry[r] : (C)s_r[S][i + APX];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    s_lg[c][S][i] = f_lg[r][c];
                    s_g[c][S][i] = f_g[r][c];
                    const C rnb = c == 0 ? rx : (c == 1 ? ry : (C)f_rn[r]);
                    s_v[c][S][i] = (C)f_g[r][c] * adj_rcp(rho0 + half * (r0 + rnb));
                }
            }
        }
    };
    double dacc[IC_MAX_MODES];
#pragma unroll
    for (int m = 0; m < IC_MAX_MODES; ++m) dacc[m] = 0.0;
    C q_lr[4];   // lambda_rho of the own cell and its +x, +y, +z neighbours

    // update of plane k, whose slot is R (planes k - 1, k + 1 in R - 1, R + 1)
    auto update = [&](auto R_, int k) {
        constexpr int R = decltype(R_)::value;
        constexpr int SK[3] = {(R + 2) % 3, R, (R + 1) % 3};
        auto at = [&](int sa, int s, int sb, int t, int &pl) {
            int d[3] = {0, 0, 0};
            d[sa] += s;
            d[sb] += t;
            pl = SK[d[2] + 1];
            return c0 + d[0] + d[1] * APX;
        };
        auto vat = [&](int c, int sa, int s, int sb, int t) {
            int pl;
            const int i = at(sa, s, sb, t, pl);
            return (C)s_v[c][pl][i];
        };
        auto gat = [&](int c, int sa, int s, int sb, int t) {
            int pl;
            const int i = at(sa, s, sb, t, pl);
            return (C)s_g[c][pl][i];
        };
        auto lgat = [&](int c, int sa, int s, int sb, int t) {
            int pl;
            const int i = at(sa, s, sb, t, pl);
            return (C)s_lg[c][pl][i];
        };
        const C k_ = (C)a.k, eta = (C)a.eta, ih = (C)a.inv_h, lam_b = (C)a.lam_b;
        auto mup_at = [&](int sa, int s) {
            C m = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) m += -k_ * (lgat(c, sa, s, c, -1) - lgat(c, sa, s, c, 0));
            return m;
        };
        const C lr0 = q_lr[0];
        const C lr1[3] = {q_lr[1], q_lr[2], q_lr[3]};
        const C rj = (C)s_r[SK[1]][c0];
        const C rn[3] = {(C)s_r[SK[1]][c0 + 1], (C)s_r[SK[1]][c0 + APX], (C)s_r[SK[2]][c0]};
        const C mu_p = mup_at(0, 0);
        const int j = k * plane + own_xy;
        C murf[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            C mgv = -k_ * (lr0 - lr1[ax]);
            C mvv = 0;
            const C lgm = lgat(ax, ax, -1, ax, 0), lg0 = lgat(ax, ax, 0, ax, 0), lgp = lgat(ax, ax, 1, ax, 0);
            const C mC0 = -k_ * (lgm - lg0);
            const C mC1 = -k_ * (lg0 - lgp);
            const C v0 = vat(ax, ax, 0, ax, 0), vm = vat(ax, ax, -1, ax, 0), vp = vat(ax, ax, 1, ax, 0);
            const C g0 = gat(ax, ax, 0, ax, 0), gm = gat(ax, ax, -1, ax, 0), gp = gat(ax, ax, 1, ax, 0);
            mgv += quarter * (v0 + vm) * mC0 + quarter * (vp + v0) * mC1;
            mvv += quarter * (g0 + gm) * mC0 + quarter * (gp + g0) * mC1;
            mvv += -2 * eta * ih * (mC0 - mC1);
            mvv += -lam_b * (mu_p - mup_at(ax, 1)) * ih;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (b == ax) continue;
                const C mE0 = -k_ * (lgat(ax, b, 0, b, 0) - lgat(ax, b, 1, b, 0));
                const C mEm = -k_ * (lgat(ax, b, -1, b, 0) - lgat(ax, b, 0, b, 0));
                const C Q0 = vat(b, b, 0, ax, 0) + vat(b, ax, 1, b, 0);
                const C Qm = vat(b, b, -1, ax, 0) + vat(b, b, -1, ax, 1);
                mgv += quarter * Q0 * mE0 + quarter * Qm * mEm;
                mvv += -eta * ih * (mEm - mE0);
                const C mF0 = -k_ * (lgat(b, ax, 0, ax, 0) - lgat(b, ax, 1, ax, 0));
                const C mFm = -k_ * (lgat(b, b, -1, ax, 0) - lgat(b, b, -1, ax, 1));
                const C P0 = gat(b, ax, 0, ax, 0) + gat(b, ax, 1, ax, 0);
                const C Pm = gat(b, b, -1, ax, 0) + gat(b, b, -1, ax, 1);
                mvv += quarter * P0 * mF0 + quarter * Pm * mFm;
                mvv += -eta * ih * (mFm - mF0);
            }
            const C irf = adj_rcp(rho0 + half * (rj + rn[ax]));
            adj_combine(a, 1 + ax, j, lg0, mgv + mvv * irf);
            murf[ax] = -mvv * (g0 * irf) * irf;
        }
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) __builtin_nontemporal_store(murf[ax], &a.murf[ax][j]);
        __builtin_nontemporal_store((C)a.cf2 * mu_p + half * (murf[0] + murf[1] + murf[2]), &a.mur[j]);
#pragma unroll
        for (int m = 0; m < IC_MAX_MODES; ++m) {
            if (m >= a.nmodes) break;
            const int ax = a.dc.axis[m];
            dacc[m] += (double)mu_p * a.prof[m * a.pstride + (ax == 0 ? x0 + lx : (ax == 1 ? y0 + ly : k))];
        }
    };
    // one plane of the march: commit plane k + 1 (slot R + 1), prefetch k + 2
    // and the own lambda_rho values of plane k, update plane k (slot R)
    auto iteration = [&](auto R_, int k) {
        constexpr int R = decltype(R_)::value;
        __syncthreads();
        commit(std::integral_constant<int, (R + 1) % 3>{});
        if (k + 2 <= z1) fetch(k + 2);
        if (own) {
            const int o = k * plane;
            q_lr[0] = (C)a.lam[0][o + own_xy];
            q_lr[1] = (C)a.lam[0][o + own_x1];
            q_lr[2] = (C)a.lam[0][o + own_y1];
            q_lr[3] = (C)a.lam[0][wrap(k + 1, nz) * plane + own_xy];
        }
        __syncthreads();
        if (own) update(R_, k);
    };

    // prologue: density of z0 - 1 (slot 2), planes z0 - 1 (slot 2) and z0 (slot 0)
    {
#pragma unroll
        for (int r = 0; r < APTS; ++r)
            if (pin[r]) s_r[2][pi[r]] = a.U[0][wrap(z0 - 1, nz) * plane + pg[r]];
    }
    fetch(z0 - 1);
    __syncthreads();
    commit(std::integral_constant<int, 2>{});
    fetch(z0);
    __syncthreads();
    commit(std::integral_constant<int, 0>{});
    fetch(z0 + 1);
    for (int k = z0; k < z1; k += 3) {
        iteration(std::integral_constant<int, 0>{}, k);
        if (k + 1 < z1) iteration(std::integral_constant<int, 1>{}, k + 1);
        if (k + 2 < z1) iteration(std::integral_constant<int, 2>{}, k + 2);
    }
    if (a.nmodes > 0) {
        // per-block partials in a fixed order; the reduction reuses LDS
        __syncthreads();
        double(*s_red)[ATHREADS / 64] = reinterpret_cast<double(*)[ATHREADS / 64]>(&s_lg[0][0][0]);
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int m = 0; m < IC_MAX_MODES; ++m) {
            if (m >= a.nmodes) break;
            double v = dacc[m];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) s_red[m][wave] = v;
        }
        __syncthreads();
        if (tid < a.nmodes) {
            double sum = 0.0;
            for (int w = 0; w < ATHREADS / 64; ++w) sum += s_red[tid][w];
            a.partial[tid * a.nbp + blockIdx.x] += a.dc.c[tid] * sum;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj_rho(const AdjArgs<T> a) {
    const int ncell = a.nx * a.ny * a.nz;
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= ncell) return;
    int x, y, z;
    cell_of(j, a.nx, a.ny, x, y, z);
    const int jm[3] = {j + (x == 0 ? a.nx - 1 : -1), j + (y == 0 ? a.nx * (a.ny - 1) : -a.nx),
                       j + (z == 0 ? a.nx * a.ny * (a.nz - 1) : -a.nx * a.ny)};
    // every value here is read once: non-temporal, like the stores
    const T mu = __builtin_nontemporal_load(&a.mur[j]) +
                 (T)0.5 * ((__builtin_nontemporal_load(&a.murf[0][jm[0]]) +
                            __builtin_nontemporal_load(&a.murf[1][jm[1]])) +
                           __builtin_nontemporal_load(&a.murf[2][jm[2]]));
    adj_combine(a, 0, j, __builtin_nontemporal_load(&a.lam[0][j]), mu);
}

// ---------------------------------------------------------------------------
// Reverse mode of the particle coupling (App. A substeps 1-2 and 4-7, and the
// particle pressure and spread force inside each RK stage increment), one
// 64-lane wave per particle.  Gathers use the kernel weights and their
// position gradients (phi is C^1, so phi' exists everywhere); scatters into
// the adjoint fields are atomic adds, so the rounding order of the adjoint
// (not its value) can differ from run to run.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dphi3(double r) {
    const double a = fabs(r);
    if (a <= 0.5) return -r / sqrt(1.0 - 3.0 * r * r);
    if (a <= 1.5) {
        const double s = 1.0 - a;
        const double v = 0.5 + s / (2.0 * sqrt(1.0 - 3.0 * s * s));
        return r > 0.0 ? -v : v;
    }
    return 0.0;
}

// Point pt (0..26, x fastest) of the kernel of location kind (0 cell, 1 + a
// face a) at q in the box: element index, grid coordinates, weight w =
// prod phi, its gradient dw/dq and, for a face, the index of the second
// cell of the face density (the next cell along a).
struct KPoint {
    size_t i, nb;
    int c[3];
    double w, dw[3];
};

__device__ __forceinline__ KPoint kpoint(const Grid &G, const double q[3], int kind, int pt) {
    const int n[3] = {G.nx, G.ny, G.nz};
    const int d[3] = {pt % 3, (pt / 3) % 3, pt / 9};
    double ph[3], dph[3];
    KPoint k;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double x = q[ax] * G.inv_h - (kind == ax + 1 ? 0.5 : 0.0);
        const double nearest = floor(x + 0.5);
        const double r = x - (nearest - 1.0 + d[ax]);
        ph[ax] = phi3(r);
        dph[ax] = dphi3(r) * G.inv_h;
        k.c[ax] = wrap((int)nearest - 1 + d[ax], n[ax]);
    }
    k.w = ph[0] * ph[1] * ph[2];
    k.dw[0] = dph[0] * ph[1] * ph[2];
    k.dw[1] = ph[0] * dph[1] * ph[2];
    k.dw[2] = ph[0] * ph[1] * dph[2];
    k.i = ((size_t)k.c[2] * G.ny + k.c[1]) * G.nx + k.c[0];
    k.nb = k.i;
    if (kind > 0) {
        int c2[3] = {k.c[0], k.c[1], k.c[2]};
        const int a = kind - 1;
        c2[a] = c2[a] + 1 == n[a] ? 0 : c2[a] + 1;
        k.nb = ((size_t)c2[2] * G.ny + c2[1]) * G.nx + c2[0];
    }
    return k;
}

template <typename T>
struct AdjPartArgs {
    Grid G;
    int np;
    double dt, V, inv_h3, L[3], cs;   // cs: weight of the reversed RK stage
    const T *Un[4];     // state before the step
    const T *U3[4];     // third stage output before the no-slip correction
    const T *gnew[3];   // momentum after the correction
    const T *Us;        // density of the reversed stage's input
    const T *lin[4];    // adjoint of the reversed stage's output
    T *lam[4];          // adjoint fields receiving the scatters
    const double *q, *u;          // particle state before the step
    double *lq, *lu;              // in: dL/d(q, u) after the step; out: before
    const double *lF;             // dL/dF^{n+1/2} of this step, or nullptr
    const double *me, *eps, *ks, *qeq, *qh, *F, *un, *du, *mf;
    double *lqh, *lFt, *lVt, *lmf, *dme, *deps, *dks;
};

// Positions of a reversed step wrapped into the box (they index the grid); a
// non-finite component becomes 0 and raises flag[1].
__global__ __launch_bounds__(256) void k_adjp_positions(int np, const double *q, double *out,
                                                        double L0, double L1, double L2,
                                                        int32_t *flag) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= 3 * np) return;
    const int ax = i % 3;
    const double L = ax == 0 ? L0 : (ax == 1 ? L1 : L2);
    double x = q[i];
    if (!isfinite(x)) {
        x = 0.0;
        flag[1] = 1;
    }
    out[i] = wrap_pos(x, L);
}

template <typename T>
__device__ __forceinline__ void scatter_face_density(T *lr, const KPoint &k, double v) {
    atomicAdd(lr + k.i, (T)(0.5 * v));
    atomicAdd(lr + k.nb, (T)(0.5 * v));
}

// Substep 7 reversed: q^{n+1} = q^n + dt/2 J(v^{n+1} + v^n) at q^{n+1/2}.
// Scatters the J v^{n+1} part into the adjoint of g^{n+1} and rho^{n+1};
// starts the per-particle accumulators.
template <typename T>
__global__ __launch_bounds__(256) void k_adjp_final(const AdjPartArgs<T> a) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    const int lane = threadIdx.x & 63;
    const double qh[3] = {a.qh[3 * p], a.qh[3 * p + 1], a.qh[3 * p + 2]};
    const double lJ[3] = {0.5 * a.dt * a.lq[3 * p], 0.5 * a.dt * a.lq[3 * p + 1],
                          0.5 * a.dt * a.lq[3 * p + 2]};
    double gq[3] = {0, 0, 0};
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int item = lane + 64 * it;
        if (item < 81) {
            const int ax = item / 27;
            const KPoint k = kpoint(a.G, qh, ax + 1, item % 27);
            const double rf = a.G.rho0 + 0.5 * ((double)a.U3[0][k.i] + (double)a.U3[0][k.nb]);
            const double gn = (double)a.gnew[ax][k.i];
            atomicAdd(a.lam[1 + ax] + k.i, (T)(lJ[ax] * k.w / rf));
            scatter_face_density(a.lam[0], k, -lJ[ax] * k.w * gn / (rf * rf));
#pragma unroll
            for (int b = 0; b < 3; ++b) gq[b] += lJ[ax] * k.dw[b] * (gn / rf);
        }
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) gq[b] = wave_sum(gq[b]);
    if (lane < 3) {
        a.lqh[3 * p + lane] = gq[lane];
        a.lFt[3 * p + lane] = a.lF ? a.lF[3 * p + lane] : 0.0;
    }
}

// Substeps 6 and 5 reversed, gather side: the no-slip correction
// g^{n+1} = g~ + rho_face V S(u^{n+1} - V~) and the particle velocity
// u^{n+1} = u^n + m_f/(m_e + m_f) (V~ - u^n).  Reads the complete adjoint of
// g^{n+1}; keeps dL/dV~ and dL/dm_f for k_adjp_velocity.
template <typename T>
__global__ __launch_bounds__(256) void k_adjp_noslip(const AdjPartArgs<T> a) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    const int lane = threadIdx.x & 63;
    const double qh[3] = {a.qh[3 * p], a.qh[3 * p + 1], a.qh[3 * p + 2]};
    const double du[3] = {a.du[3 * p], a.du[3 * p + 1], a.du[3 * p + 2]};   // V (u^{n+1} - V~)
    double sd[3] = {0, 0, 0}, gq[3] = {0, 0, 0};
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int item = lane + 64 * it;
        if (item < 81) {
            const int ax = item / 27;
            const KPoint k = kpoint(a.G, qh, ax + 1, item % 27);
            const double rf = a.G.rho0 + 0.5 * ((double)a.U3[0][k.i] + (double)a.U3[0][k.nb]);
            const double lg = (double)a.lam[1 + ax][k.i];
            sd[ax] += k.w * lg * rf;
            scatter_face_density(a.lam[0], k, lg * k.w * du[ax] * a.inv_h3);
#pragma unroll
            for (int b = 0; b < 3; ++b) gq[b] += du[ax] * a.inv_h3 * k.dw[b] * lg * rf;
        }
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        sd[b] = wave_sum(sd[b]);
        gq[b] = wave_sum(gq[b]);
    }
    const double me = a.me[p];
    double dme = 0.0, lu_out[3], lVt[3], lmf[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double ldu = a.V * a.inv_h3 * sd[ax];
        const double un = a.un[3 * p + ax], mf = a.mf[3 * p + ax];
        const double Vt = un - du[ax] / a.V;
        const double lun = a.lu[3 * p + ax] + ldu;
        const double mt = me + mf, c = mf / mt;
        lu_out[ax] = lun * (1.0 - c);
        lVt[ax] = c * lun - ldu;
        const double lc = lun * (Vt - a.u[3 * p + ax]);
        lmf[ax] = lc * me / (mt * mt);
        dme -= lc * mf / (mt * mt);
    }
    if (lane < 3) {
        a.lqh[3 * p + lane] += gq[lane];
        a.lVt[3 * p + lane] = lVt[lane];
        a.lmf[3 * p + lane] = lmf[lane];
        a.lu[3 * p + lane] = lu_out[lane];
    }
    if (lane == 0) a.dme[p] += dme;
}

// Substeps 4-5 reversed, scatter side: V~ = J(g~ / rho_face) and
// m_f = V J rho_face at q^{n+1/2}, into the adjoint of the third stage output.
template <typename T>
__global__ __launch_bounds__(256) void k_adjp_velocity(const AdjPartArgs<T> a) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    const int lane = threadIdx.x & 63;
    const double qh[3] = {a.qh[3 * p], a.qh[3 * p + 1], a.qh[3 * p + 2]};
    const double lVt[3] = {a.lVt[3 * p], a.lVt[3 * p + 1], a.lVt[3 * p + 2]};
    const double lm[3] = {a.V * a.lmf[3 * p], a.V * a.lmf[3 * p + 1], a.V * a.lmf[3 * p + 2]};
    double gq[3] = {0, 0, 0};
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int item = lane + 64 * it;
        if (item < 81) {
            const int ax = item / 27;
            const KPoint k = kpoint(a.G, qh, ax + 1, item % 27);
            const double rf = a.G.rho0 + 0.5 * ((double)a.U3[0][k.i] + (double)a.U3[0][k.nb]);
            const double g3 = (double)a.U3[1 + ax][k.i];
            atomicAdd(a.lam[1 + ax] + k.i, (T)(lVt[ax] * k.w / rf));
            scatter_face_density(a.lam[0], k, -lVt[ax] * k.w * g3 / (rf * rf) + lm[ax] * k.w);
#pragma unroll
            for (int b = 0; b < 3; ++b) gq[b] += k.dw[b] * (lVt[ax] * (g3 / rf) + lm[ax] * rf);
        }
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) gq[b] = wave_sum(gq[b]);
    if (lane < 3) a.lqh[3 * p + lane] += gq[lane];
}

// Particle terms of one reversed RK stage increment (weight cs): the stage
// pressure S(eps V J rho_s) and the spread force dt S F, both at q^{n+1/2}.
// mu_p (the adjoint of the cell pressure) is formed from the stage's output
// adjoint; the density part is added to the stage's input adjoint (after
// k_adj_rho wrote it).
template <typename T>
__global__ __launch_bounds__(256) void k_adjp_stage(const AdjPartArgs<T> a) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    const int lane = threadIdx.x & 63;
    const double qh[3] = {a.qh[3 * p], a.qh[3 * p + 1], a.qh[3 * p + 2]};
    const double F[3] = {a.F[3 * p], a.F[3 * p + 1], a.F[3 * p + 2]};
    const double kdt = a.dt * a.G.inv_h;
    const int n[3] = {a.G.nx, a.G.ny, a.G.nz};
    const size_t stride[3] = {1, (size_t)a.G.nx, (size_t)a.G.nx * a.G.ny};
    double sP = 0, sJ = 0, gP[3] = {0, 0, 0}, gJ[3] = {0, 0, 0};
    double sF[3] = {0, 0, 0}, gF[3] = {0, 0, 0};
    KPoint kc;
    kc.w = 0.0;
    kc.i = 0;
    if (lane < 27) {
        kc = kpoint(a.G, qh, 0, lane);
        double mp = 0.0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const size_t im = kc.c[ax] == 0 ? kc.i + (size_t)(n[ax] - 1) * stride[ax] : kc.i - stride[ax];
            mp -= kdt * ((double)a.lin[1 + ax][im] - (double)a.lin[1 + ax][kc.i]);
        }
        const double r = (double)a.Us[kc.i];
        sP = kc.w * mp;
        sJ = kc.w * r;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            gP[b] = kc.dw[b] * mp;
            gJ[b] = kc.dw[b] * r;
        }
    }
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int item = lane + 64 * it;
        if (item < 81) {
            const int ax = item / 27;
            const KPoint k = kpoint(a.G, qh, ax + 1, item % 27);
            const double lg = (double)a.lin[1 + ax][k.i];
            sF[ax] += k.w * lg;
#pragma unroll
            for (int b = 0; b < 3; ++b) gF[b] += F[ax] * k.dw[b] * lg;
        }
    }
    sP = wave_sum(sP);
    sJ = wave_sum(sJ);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        gP[b] = wave_sum(gP[b]);
        gJ[b] = wave_sum(gJ[b]);
        sF[b] = wave_sum(sF[b]);
        gF[b] = wave_sum(gF[b]);
    }
    const double P = sP * a.inv_h3, eps = a.eps[p];
    if (lane < 27) atomicAdd(a.lam[0] + kc.i, (T)(a.cs * eps * a.V * kc.w * P));
    if (lane < 3) {
        const int b = lane;
        a.lqh[3 * p + b] += a.cs * (eps * a.V * (sJ * gP[b] * a.inv_h3 + P * gJ[b]) +
                                    a.dt * a.inv_h3 * gF[b]);
        a.lFt[3 * p + b] += a.cs * a.dt * a.inv_h3 * sF[b];
    }
    if (lane == 0) a.deps[p] += a.cs * a.V * sJ * P;
}

// Substeps 2 and 1 reversed, after the stages: F = -k_s minimg(q^{n+1/2} -
// q_eq) + f_ext, J v^n at q^{n+1/2} (kept for substep 7) and q^{n+1/2} =
// q^n + dt/2 J v^n at q^n; scatters into the adjoint of the state before the
// step and writes dL/dq^n.
template <typename T>
__global__ __launch_bounds__(256) void k_adjp_start(const AdjPartArgs<T> a) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    const int lane = threadIdx.x & 63;
    double lqh[3], lv[3], pos[3];
    double dks = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const double lF = a.lFt[3 * p + b];
        pos[b] = a.qh[3 * p + b];
        lqh[b] = a.lqh[3 * p + b] - a.ks[p] * lF;
        dks -= lF * min_image(pos[b] - a.qeq[3 * p + b], a.L[b]);
        lv[b] = 0.5 * a.dt * a.lq[3 * p + b];
    }
    double lq[3] = {a.lq[3 * p], a.lq[3 * p + 1], a.lq[3 * p + 2]};
    // pass 0: J v^n at q^{n+1/2}; pass 1: J v^n at q^n
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        double gq[3] = {0, 0, 0};
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int item = lane + 64 * it;
            if (item < 81) {
                const int ax = item / 27;
                const KPoint k = kpoint(a.G, pos, ax + 1, item % 27);
                const double rf = a.G.rho0 + 0.5 * ((double)a.Un[0][k.i] + (double)a.Un[0][k.nb]);
                const double g0 = (double)a.Un[1 + ax][k.i];
                atomicAdd(a.lam[1 + ax] + k.i, (T)(lv[ax] * k.w / rf));
                scatter_face_density(a.lam[0], k, -lv[ax] * k.w * g0 / (rf * rf));
#pragma unroll
                for (int b = 0; b < 3; ++b) gq[b] += lv[ax] * k.dw[b] * (g0 / rf);
            }
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) gq[b] = wave_sum(gq[b]);
        if (pass == 0) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                lqh[b] += gq[b];
                lq[b] += lqh[b];
                lv[b] = 0.5 * a.dt * lqh[b];
                pos[b] = a.q[3 * p + b];
            }
        } else {
#pragma unroll
            for (int b = 0; b < 3; ++b) lq[b] += gq[b];
        }
    }
    if (lane < 3) a.lq[3 * p + lane] = lq[lane];
    if (lane == 0) a.dks[p] += dks;
}

// FP64 block partial sums of the four fields (deterministic order).
template <typename T>
__global__ __launch_bounds__(256) void k_sums(const T *f0, const T *f1, const T *f2, const T *f3,
                                              size_t n, double *partial) {
    __shared__ double s[4][256];
    double acc[4] = {0, 0, 0, 0};
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        acc[0] += (double)f0[i];
        acc[1] += (double)f1[i];
        acc[2] += (double)f2[i];
        acc[3] += (double)f3[i];
    }
    for (int c = 0; c < 4; ++c) s[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int c = 0; c < 4; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) partial[4 * blockIdx.x + c] = s[c][0];
}

// ---------------------------------------------------------------------------
// Host-side helpers
// ---------------------------------------------------------------------------
template <typename T>
PartArgs<T> part_args(ic_ctx *c, void *const f[4]) {
    PartArgs<T> a{};
    const ic_params &p = c->p;
    a.G = Grid{p.nx, p.ny, p.nz, p.h, 1.0 / p.h, p.rho0};
    for (int i = 0; i < 4; ++i) a.f[i] = (const T *)f[i];
    a.np = c->np;
    a.dt = p.dt;
    a.V = 8.0 * p.h * p.h * p.h;
    a.L[0] = p.nx * p.h;
    a.L[1] = p.ny * p.h;
    a.L[2] = p.nz * p.h;
    const Workspace &w = c->ws;
    a.q = w.q; a.u = w.u; a.me = w.me; a.eps = w.eps; a.ks = w.ks; a.qeq = w.qeq; a.fext = w.fext;
    a.qh = w.qh; a.jv_old = w.jv_old; a.F = w.F; a.Vt = w.Vt; a.du = w.du; a.mf = w.mf;
    a.omega = w.omega; a.jv_new = w.jv_new;
    a.bc = w.pk.bc; a.bf = w.pk.bf; a.wc = w.pk.wc; a.wf = w.pk.wf;
    a.sum_f = w.sum_f; a.sum_l = w.sum_l; a.flag = w.flag;
    return a;
}

BinArgs bin_args(ic_ctx *c, int np, const double *qh) {
    BinArgs b{};
    b.np = np;
    b.nx = c->p.nx;
    b.ny = c->p.ny;
    b.nz = c->p.nz;
    b.gx = c->nblk[0];
    b.gy = c->nblk[1];
    b.gz = c->nblk[2];
    b.nblk = b.gx * b.gy * b.gz;
    b.tz = c->tz;
    b.inv_h = 1.0 / c->p.h;
    b.qh = qh;
    b.count = c->ws.blk_count;
    b.off = c->ws.blk_off;
    b.cursor = c->ws.blk_cursor;
    b.list = c->ws.blk_list;
    b.key = c->ws.blk_key;
    b.bc = c->ws.pk.bc;
    return b;
}

inline unsigned wave_blocks(int n) { return (unsigned)((n * 64 + 255) / 256); }
inline unsigned thread_blocks(int n) { return (unsigned)((n + 255) / 256); }

void launch_binning(ic_ctx *c, int np, const double *qh, hipStream_t s) {
    const BinArgs b = bin_args(c, np, qh);
    if (np <= SB_CAP && b.nblk <= SB_MAXBLK) {
        hipLaunchKernelGGL(k_bin_small, dim3(1), dim3(SB_THREADS), 0, s, b);
        return;
    }
    hipLaunchKernelGGL(k_bin_count, dim3(thread_blocks(np)), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, b);
    hipLaunchKernelGGL(k_bin_fill, dim3(thread_blocks(np)), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_bin_sort, dim3(b.nblk), dim3(64), 0, s, b);
}

ClusterArgs cluster_args(ic_ctx *c, int np) {
    const Workspace &w = c->ws;
    ClusterArgs a{};
    a.np = np;
    a.parent = w.cl_parent;
    a.root = w.cl_root;
    a.cnt = w.cl_cnt;
    a.off = w.cl_off;
    a.cursor = w.cl_cursor;
    a.list = w.cl_list;
    return a;
}

// Clusters of the particles at q^{n+1/2} (after k_pre wrote the kernel
// data): one workgroup for small sets, else tile binning, unions per tile
// list, then count, scan and fill.
void launch_clusters(ic_ctx *c, int np, hipStream_t s) {
    const ClusterArgs ca = cluster_args(c, np);
    if (np <= CL_SMALL_CAP) {
        hipLaunchKernelGGL(k_cl_small, dim3(1), dim3(1024), 0, s,
                           ClusterSmallArgs{ca, c->ws.pk.bc, c->p.nx, c->p.ny, c->p.nz});
        return;
    }
    const BinArgs b = bin_args(c, np, c->ws.qh);
    hipLaunchKernelGGL(k_cl_init, dim3(thread_blocks(np)), dim3(256), 0, s, ca);
    hipLaunchKernelGGL(k_bin_count, dim3(thread_blocks(np)), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, b);
    hipLaunchKernelGGL(k_bin_fill, dim3(thread_blocks(np)), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_bin_union, dim3(b.nblk), dim3(64), 0, s, b, ca.parent);
    hipLaunchKernelGGL(k_cl_count, dim3(thread_blocks(np)), dim3(256), 0, s, ca);
    hipLaunchKernelGGL(k_cl_scan, dim3(1), dim3(1024), 0, s, ca);
    hipLaunchKernelGGL(k_cl_fill, dim3(thread_blocks(np)), dim3(256), 0, s, ca);
}


// Arguments of one context's step kernels (shared by the eager step and the
// batched ensemble step, so both run the same arithmetic).
DriveArgs drive_args(const ic_ctx *c) {
    DriveArgs d{};
    d.nmodes = c->forcing.nmodes;
    d.dt = c->p.dt;
    for (int m = 0; m < d.nmodes; ++m) {
        d.amp[m] = c->forcing.modes[m].amp;
        d.omega[m] = c->forcing.modes[m].omega;
        d.phase[m] = c->forcing.modes[m].phase;
    }
    return d;
}

BMPoly bm_poly() {
    BMPoly P;
    const double ln[11] = {1.0 / 21, 1.0 / 19, 1.0 / 17, 1.0 / 15, 1.0 / 13, 1.0 / 11,
                           1.0 / 9,  1.0 / 7,  1.0 / 5,  1.0 / 3,  1.0};
    const double sn[7] = {-1.0 / 1307674368000.0, 1.0 / 6227020800.0, -1.0 / 39916800.0,
                          1.0 / 362880.0,         -1.0 / 5040.0,      1.0 / 120.0,
                          -1.0 / 6.0};
    const double cs[8] = {1.0 / 20922789888000.0, -1.0 / 87178291200.0, 1.0 / 479001600.0,
                          -1.0 / 3628800.0,       1.0 / 40320.0,        -1.0 / 720.0,
                          1.0 / 24.0,             -0.5};
    for (int i = 0; i < 11; ++i) P.ln[i] = ln[i];
    for (int i = 0; i < 7; ++i) P.sn[i] = sn[i];
    for (int i = 0; i < 8; ++i) P.cs[i] = cs[i];
    return P;
}

template <typename T>
NoiseArgs<T> noise_args(const ic_ctx *c) {
    const ic_params &p = c->p;
    const Workspace &w = c->ws;
    NoiseArgs<T> na{};
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 9; ++i) na.out[k][i] = (T *)w.N[k][i];
    na.nx = p.nx; na.ny = p.ny; na.nz = p.nz; na.tz = c->tz;
    na.gx = (p.nx + NTX - 1) / NTX; na.gy = (p.ny + NTY<T> - 1) / NTY<T>; na.gz = c->nblk[2];
    const double amp = 1.0 / sqrt(p.h * p.h * p.h * p.dt);
    const double an = sqrt(2.0 * p.eta * p.kT);
    const double bt = sqrt(p.zeta * p.kT / 3.0) - an / 3.0;
    na.dt_h = (T)(p.dt / p.h);
    na.sd = (T)(amp * an * sqrt(2.0));
    na.st = (T)(amp * bt * sqrt(2.0));
    na.so = (T)(amp * an);
    na.s3 = (T)sqrt(3.0);
    na.nk = NoiseKey{(uint32_t)(p.seed & 0xFFFFFFFFu), (uint32_t)(p.seed >> 32), 0u, p.replica};
    na.step = w.st;
    na.ahead = 0;
    na.poly = bm_poly();
    return na;
}

constexpr double RK_A[3] = {0.0, 0.75, 1.0 / 3.0}, RK_B[3] = {1.0, 0.25, 2.0 / 3.0};

// Stage st reads src and writes dst: U -> A -> B -> U.
struct StageBufs {
    void *src[4], *dst[4];
};
inline StageBufs stage_buffers(const ic_ctx *c, int st) {
    StageBufs b;
    for (int i = 0; i < 4; ++i) {
        void *const chain[4] = {c->f[i], c->ws.A[i], c->ws.B[i], c->f[i]};
        b.src[i] = chain[st];
        b.dst[i] = chain[st + 1];
    }
    return b;
}

template <typename T>
StageArgs<T> stage_args(const ic_ctx *c, int st) {
    const ic_params &p = c->p;
    const Workspace &w = c->ws;
    StageArgs<T> a{};
    a.nx = p.nx; a.ny = p.ny; a.nz = p.nz; a.tz = c->tz;
    a.gx = c->nblk[0]; a.gy = c->nblk[1]; a.gz = c->nblk[2];
    a.rho0 = (T)p.rho0;
    a.cf2 = (T)(p.cf * p.cf);
    a.eta = (T)p.eta;
    a.lam = (T)(p.zeta - 2.0 * p.eta / 3.0);
    a.inv_h = (T)(1.0 / p.h);
    a.dt_h = (T)(p.dt / p.h);
    a.dt = (T)p.dt;
    a.fbytes = (uint32_t)((size_t)p.nx * p.ny * p.nz * sizeof(T));
    a.st = w.st;
    a.full = p.nx % TX == 0 && p.ny % TY == 0;
    a.nmodes = c->forcing.nmodes;
    a.prof = w.prof;
    a.pstride = c->prof_stride;
    for (int m = 0; m < a.nmodes; ++m) a.maxis[m] = c->forcing.modes[m].axis;
    const StageBufs sb = stage_buffers(c, st);
    for (int i = 0; i < 4; ++i) {
        a.in[i] = (const T *)sb.src[i];
        a.un[i] = (const T *)c->f[i];
        a.out[i] = (T *)sb.dst[i];
    }
    a.ra = (T)RK_A[st];
    a.rb = (T)RK_B[st];
    const bool noise = p.kT > 0.0;
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 3; ++i) a.noise[k][i] = noise ? (const T *)w.N[k][3 * st + i] : nullptr;
    a.amp = w.st->amp[st];
    return a;
}

// Omega of stage st lives in omega[st & 1]: k_pre writes stage 0's, and the
// particle pass after stage st computes stage st + 1's from the density
// stage st wrote.
template <typename T>
StagePassArgs<T> stage_pass_args(ic_ctx *c, int st) {
    const ic_params &p = c->p;
    const Workspace &w = c->ws;
    const size_t ostride = (size_t)(p.max_particles > 0 ? p.max_particles : 0);
    const ClusterArgs ca = cluster_args(c, c->np);
    const StageBufs sb = stage_buffers(c, st);
    StagePassArgs<T> sp{};
    sp.nx = p.nx; sp.ny = p.ny; sp.nz = p.nz; sp.np = c->np;
    sp.inv_h3 = 1.0 / (p.h * p.h * p.h);
    sp.b = RK_B[st];
    sp.dt_h = p.dt / p.h;
    sp.dt = p.dt;
    sp.V = 8.0 * p.h * p.h * p.h;
    sp.root = ca.root; sp.cnt = ca.cnt; sp.off = ca.off; sp.list = ca.list;
    sp.bc = w.pk.bc; sp.bf = w.pk.bf; sp.wc = w.pk.wc; sp.wf = w.pk.wf;
    sp.F = w.F;
    sp.omega = w.omega + (st & 1) * ostride;
    sp.eps = w.eps;
    sp.omega_next = st < 2 ? w.omega + ((st + 1) & 1) * ostride : nullptr;
    sp.drho_next = (const T *)sb.dst[0];
    for (int i = 0; i < 3; ++i) sp.g[i] = (T *)sb.dst[1 + i];
    return sp;
}

template <typename T>
PostPassArgs<T> post_args(ic_ctx *c) {
    void *U[4] = {c->f[0], c->f[1], c->f[2], c->f[3]};
    const ClusterArgs ca = cluster_args(c, c->np);
    PostPassArgs<T> pp{};
    pp.pa = part_args<T>(c, U);
    pp.root = ca.root; pp.cnt = ca.cnt; pp.off = ca.off; pp.list = ca.list;
    for (int i = 0; i < 3; ++i) pp.g[i] = (T *)c->f[1 + i];
    pp.inv_h3 = 1.0 / (c->p.h * c->p.h * c->p.h);
    return pp;
}

// One step on the context stream.  Beside it, on the side stream: the
// particle prologue (half-step positions, kernel weights, stage-1 Omega,
// clusters), which only reads U^n and is joined before the first particle
// stage term, and (FP32) the noise of the next step, which depends only on
// the key and the step number, joined at the end of the step: the fluid
// stages are memory-bound and the noise kernel ALU-bound.
template <typename T>
hipError_t step_impl(ic_ctx *c, bool overlap, bool first, bool last) {
    const ic_params &p = c->p;
    hipStream_t s = c->stream;
    const Workspace &w = c->ws;
    void *U[4] = {c->f[0], c->f[1], c->f[2], c->f[3]};
    const unsigned nblk_all = (unsigned)(c->nblk[0] * c->nblk[1] * c->nblk[2]);
    const int np = c->np;
    const bool noise = p.kT > 0.0;
    // first: draw this step's noise in line; !last: draw the next step's in
    // the background of this one.  One stream draws in line only.
    if (!overlap) first = last = true;
    const bool ahead = noise && !last;
    const bool side_part = overlap && np > 0;
    const hipStream_t ps = side_part ? c->side : s;   // stream of the particle prologue
    hipError_t err = hipSuccess;
    auto chk = [&](hipError_t e) {
        if (err == hipSuccess) err = e;
    };

    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(64), 0, s, w.st, drive_args(c));
    if (side_part || ahead) {
        chk(hipEventRecord(c->ev_fork, s));
        chk(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    }
    if (np > 0) {
        hipLaunchKernelGGL(k_pre<T>, dim3(wave_blocks(np)), dim3(256), 0, ps, part_args<T>(c, U));
        launch_clusters(c, np, ps);
        if (side_part) chk(hipEventRecord(c->ev_part, c->side));
    }
    if (noise) {
        NoiseArgs<T> na = noise_args<T>(c);
        const dim3 ng(na.gx * na.gy * na.gz), nt(NTX * NTY<T>);
        if (ahead) {
            NoiseArgs<T> bg = na;
            bg.ahead = 1;
            bg.gy = (p.ny + NBG - 1) / NBG;
            const int ntile = bg.gx * bg.gy * bg.gz;
            hipLaunchKernelGGL(noise_kernel_bg<T>, dim3(std::min(ntile, c->ncu)), dim3(NTX * NBG),
                               0, c->side, bg);
            chk(hipEventRecord(c->ev_noise, c->side));
        }
        if (first) {
            na.ahead = 0;
            hipLaunchKernelGGL(noise_kernel<T>, ng, nt, 0, s, na);
        }
    }
    const bool full = p.nx % TX == 0 && p.ny % TY == 0;
    for (int st = 0; st < 3; ++st) {
        const StageArgs<T> a = stage_args<T>(c, st);
        hipEvent_t e0 = prof_event(c), e1 = prof_event(c);
        if (e0) (void)hipEventRecord(e0, s);
#define IC_STAGE(S, N, F) \
    hipLaunchKernelGGL((stage_kernel<T, S, N, F>), dim3(nblk_all), dim3(STAGE_THREADS), 0, s, a)
#define IC_STAGES(F)                                                                        \
    if (noise) {                                                                            \
        if (st == 0) IC_STAGE(0, true, F); else if (st == 1) IC_STAGE(1, true, F); else IC_STAGE(2, true, F); \
    } else {                                                                                \
        if (st == 0) IC_STAGE(0, false, F); else if (st == 1) IC_STAGE(1, false, F); else IC_STAGE(2, false, F); \
    }
        if (full) {
            IC_STAGES(true)
        } else {
            IC_STAGES(false)
        }
#undef IC_STAGES
#undef IC_STAGE
        if (e1) {
            (void)hipEventRecord(e1, s);
            prof_push(c, e0, e1);
        }
        if (np > 0) {
            if (st == 0 && side_part) chk(hipStreamWaitEvent(s, c->ev_part, 0));
            if (st < 2)
                hipLaunchKernelGGL(k_cl_stage<T>, dim3(wave_blocks(np)), dim3(256), 0, s,
                                   stage_pass_args<T>(c, st));
            else
                hipLaunchKernelGGL(k_cl_last<T>, dim3(wave_blocks(np)), dim3(256), 0, s,
                                   stage_pass_args<T>(c, st), post_args<T>(c));
        }
    }
    if (ahead) chk(hipStreamWaitEvent(s, c->ev_noise, 0));
    chk(hipGetLastError());
    return err;
}

// ---------------------------------------------------------------------------
// Batched ensemble step: for n contexts of one precision, every kernel of the
// step runs once for all of them, with per-context arguments in device
// tables and per-block (or per-wave) maps to the context and its tile (or
// particle).  Stage and noise tiles are ordered so that each XCD gets a
// contiguous run of tiles, as in the single-context launches.  Each context
// draws its own noise every step (as a single-stream step does), so a batched
// step is bitwise the single-stream step of every member.
// ---------------------------------------------------------------------------
template <typename T>
struct BatchTables {
    int n = 0;
    StepState **st = nullptr;
    DriveArgs *drive = nullptr;
    NoiseArgs<T> *noise = nullptr;
    int32_t *nmember = nullptr, *ntile = nullptr;
    int nnoise = 0;
    StageArgs<T> *stage[3] = {nullptr, nullptr, nullptr};
    int32_t *tmember = nullptr, *ttile = nullptr;
    int ntiles = 0;
    PartArgs<T> *part = nullptr;
    ClusterSmallArgs *clus = nullptr;
    int nclus = 0;
    StagePassArgs<T> *pass[3] = {nullptr, nullptr, nullptr};
    PostPassArgs<T> *post = nullptr;
    int32_t *wmember = nullptr, *wlocal = nullptr;
    int nwaves = 0;
};

// Host image of the tables, laid out in one buffer and copied to the device.
struct TableImage {
    std::vector<char> bytes;
    template <typename X>
    size_t put(const std::vector<X> &v) {
        const size_t off = (bytes.size() + 255) & ~(size_t)255;
        bytes.resize(off + v.size() * sizeof(X));
        if (!v.empty()) memcpy(bytes.data() + off, v.data(), v.size() * sizeof(X));
        return off;
    }
};

inline int host_xcd_tile(int b, int nblk) {
    const int per = nblk / 8, rem = nblk % 8, xcd = b % 8, idx = b / 8;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Block -> (member, tile) for n members of cnt[m] tiles each, XCD-ordered.
inline void tile_map(const std::vector<int> &cnt, std::vector<int32_t> &member,
                     std::vector<int32_t> &tile) {
    std::vector<int> start(cnt.size() + 1, 0);
    for (size_t m = 0; m < cnt.size(); ++m) start[m + 1] = start[m] + cnt[m];
    const int total = start.back();
    member.resize(total);
    tile.resize(total);
    for (int g = 0; g < total; ++g) {
        const int t = host_xcd_tile(g, total);
        const int m = (int)(std::upper_bound(start.begin(), start.end(), t) - start.begin()) - 1;
        member[g] = m;
        tile[g] = t - start[m];
    }
}

template <typename T>
hipError_t batch_build(ic_ctx *const *ctxs, int n, BatchTables<T> &bt, void **dev) {
    *dev = nullptr;
    TableImage img;
    std::vector<StepState *> st;
    std::vector<DriveArgs> drive;
    std::vector<NoiseArgs<T>> noise;
    std::vector<int> ncnt, tcnt;
    std::vector<StageArgs<T>> stage[3];
    std::vector<PartArgs<T>> part;
    std::vector<ClusterSmallArgs> clus;
    std::vector<StagePassArgs<T>> pass[3];
    std::vector<PostPassArgs<T>> post;
    std::vector<int32_t> wmember, wlocal;
    for (int i = 0; i < n; ++i) {
        ic_ctx *c = ctxs[i];
        st.push_back(c->ws.st);
        drive.push_back(drive_args(c));
        const NoiseArgs<T> na = noise_args<T>(c);
        noise.push_back(na);
        ncnt.push_back(c->p.kT > 0.0 ? na.gx * na.gy * na.gz : 0);
        tcnt.push_back(c->nblk[0] * c->nblk[1] * c->nblk[2]);
        for (int s = 0; s < 3; ++s) stage[s].push_back(stage_args<T>(c, s));
        if (c->np > 0) {
            const int m = (int)part.size();
            void *U[4] = {c->f[0], c->f[1], c->f[2], c->f[3]};
            part.push_back(part_args<T>(c, U));
            clus.push_back(ClusterSmallArgs{cluster_args(c, c->np), c->ws.pk.bc, c->p.nx, c->p.ny,
                                            c->p.nz});
            for (int s = 0; s < 3; ++s) pass[s].push_back(stage_pass_args<T>(c, s));
            post.push_back(post_args<T>(c));
            for (int p = 0; p < c->np; ++p) {
                wmember.push_back(m);
                wlocal.push_back(p);
            }
        }
    }
    std::vector<int32_t> nmember, ntile, tmember, ttile;
    tile_map(ncnt, nmember, ntile);
    tile_map(tcnt, tmember, ttile);
    const size_t o_st = img.put(st), o_drive = img.put(drive), o_noise = img.put(noise);
    const size_t o_nm = img.put(nmember), o_nt = img.put(ntile);
    size_t o_stage[3], o_pass[3];
    for (int s = 0; s < 3; ++s) o_stage[s] = img.put(stage[s]);
    const size_t o_tm = img.put(tmember), o_tt = img.put(ttile);
    const size_t o_part = img.put(part), o_clus = img.put(clus);
    for (int s = 0; s < 3; ++s) o_pass[s] = img.put(pass[s]);
    const size_t o_post = img.put(post), o_wm = img.put(wmember), o_wl = img.put(wlocal);
    char *d = nullptr;
    hipError_t e = hipMalloc((void **)&d, img.bytes.size());
    if (e != hipSuccess) return e;
    e = hipMemcpy(d, img.bytes.data(), img.bytes.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return e;
    }
    *dev = d;
    bt.n = n;
    bt.st = (StepState **)(d + o_st);
    bt.drive = (DriveArgs *)(d + o_drive);
    bt.noise = (NoiseArgs<T> *)(d + o_noise);
    bt.nmember = (int32_t *)(d + o_nm);
    bt.ntile = (int32_t *)(d + o_nt);
    bt.nnoise = (int)nmember.size();
    for (int s = 0; s < 3; ++s) {
        bt.stage[s] = (StageArgs<T> *)(d + o_stage[s]);
        bt.pass[s] = (StagePassArgs<T> *)(d + o_pass[s]);
    }
    bt.tmember = (int32_t *)(d + o_tm);
    bt.ttile = (int32_t *)(d + o_tt);
    bt.ntiles = (int)tmember.size();
    bt.part = (PartArgs<T> *)(d + o_part);
    bt.clus = (ClusterSmallArgs *)(d + o_clus);
    bt.nclus = (int)clus.size();
    bt.post = (PostPassArgs<T> *)(d + o_post);
    bt.wmember = (int32_t *)(d + o_wm);
    bt.wlocal = (int32_t *)(d + o_wl);
    bt.nwaves = (int)wmember.size();
    return hipSuccess;
}

// A device pointer to a table as a constant-address-space pointer.
template <typename X>
inline const IC_CONST X *cst(const X *p) {
    return (const IC_CONST X *)(uintptr_t)p;
}

template <typename T>
hipError_t batch_step(const BatchTables<T> &bt, hipStream_t s) {
    hipLaunchKernelGGL(k_step_begin_batched, dim3(bt.n), dim3(64), 0, s, cst(bt.st), cst(bt.drive));
    if (bt.nnoise > 0)
        hipLaunchKernelGGL(noise_kernel_batched<T>, dim3(bt.nnoise), dim3(NTX * NTY<T>), 0, s,
                           cst(bt.noise), cst(bt.nmember), cst(bt.ntile));
    const WaveMap wm{cst(bt.wmember), cst(bt.wlocal), bt.nwaves};
    if (bt.nwaves > 0) {
        hipLaunchKernelGGL(k_pre_batched<T>, dim3(wave_blocks(bt.nwaves)), dim3(256), 0, s,
                           cst(bt.part), wm);
        hipLaunchKernelGGL(k_cl_small_batched, dim3(bt.nclus), dim3(1024), 0, s, cst(bt.clus));
    }
    for (int st = 0; st < 3; ++st) {
        const dim3 g(bt.ntiles), b(STAGE_THREADS);
        if (st == 0)
            hipLaunchKernelGGL((stage_kernel_batched<T, 0>), g, b, 0, s, cst(bt.stage[0]),
                               cst(bt.tmember), cst(bt.ttile));
        else if (st == 1)
            hipLaunchKernelGGL((stage_kernel_batched<T, 1>), g, b, 0, s, cst(bt.stage[1]),
                               cst(bt.tmember), cst(bt.ttile));
        else
            hipLaunchKernelGGL((stage_kernel_batched<T, 2>), g, b, 0, s, cst(bt.stage[2]),
                               cst(bt.tmember), cst(bt.ttile));
        if (bt.nwaves > 0 && st < 2)
            hipLaunchKernelGGL(k_cl_stage_batched<T>, dim3(wave_blocks(bt.nwaves)), dim3(256), 0, s,
                               cst(bt.pass[st]), wm);
        else if (bt.nwaves > 0)
            hipLaunchKernelGGL(k_cl_last_batched<T>, dim3(wave_blocks(bt.nwaves)), dim3(256), 0, s,
                               cst(bt.pass[2]), cst(bt.post), wm);
    }
    return hipGetLastError();
}

}  // namespace

struct Batch {
    int prec = 0;
    void *dev = nullptr;
    BatchTables<float> f;
    BatchTables<double> d;
};

bool batch_supported(ic_ctx *const *ctxs, int n) {
    for (int i = 0; i < n; ++i) {
        if (ctxs[i]->p.prec != ctxs[0]->p.prec) return false;
        if (ctxs[i]->np > CL_SMALL_CAP) return false;
    }
    return n > 0;
}

hipError_t batch_create(ic_ctx *const *ctxs, int n, Batch **out) {
    *out = nullptr;
    Batch *b = new (std::nothrow) Batch();
    if (!b) return hipErrorOutOfMemory;
    b->prec = ctxs[0]->p.prec;
    const hipError_t e = b->prec == IC_FP64 ? batch_build<double>(ctxs, n, b->d, &b->dev)
                                            : batch_build<float>(ctxs, n, b->f, &b->dev);
    if (e != hipSuccess) {
        delete b;
        return e;
    }
    *out = b;
    return hipSuccess;
}

hipError_t batch_step(const Batch *b, hipStream_t s) {
    return b->prec == IC_FP64 ? batch_step<double>(b->d, s) : batch_step<float>(b->f, s);
}

void batch_destroy(Batch *b) {
    if (!b) return;
    if (b->dev) (void)hipFree(b->dev);
    delete b;
}

namespace {

template <typename T>
hipError_t interp_impl(ic_ctx *c, int n, const double *q, int kind, const void *field,
                       double *out) {
    const Grid G{c->p.nx, c->p.ny, c->p.nz, c->p.h, 1.0 / c->p.h, c->p.rho0};
    hipLaunchKernelGGL(k_interp<T>, dim3(wave_blocks(n)), dim3(256), 0, c->stream, G, n, q, kind,
                       (const T *)field, out);
    return hipGetLastError();
}

template <typename T>
hipError_t spread_impl(ic_ctx *c, int n, const double *q, const double *f, int kind,
                       void *field) {
    const ic_params &p = c->p;
    const Workspace &w = c->ws;
    const Grid G{p.nx, p.ny, p.nz, p.h, 1.0 / p.h, p.rho0};
    hipLaunchKernelGGL(k_weights, dim3(wave_blocks(n)), dim3(256), 0, c->stream, G, n, q, w.qh,
                       w.pk.bc, w.pk.bf, w.pk.wc, w.pk.wf);
    launch_binning(c, n, w.qh, c->stream);
    SparseArgs<T> sa{};
    sa.nx = p.nx; sa.ny = p.ny; sa.nz = p.nz; sa.tz = c->tz;
    sa.inv_h3 = 1.0 / (p.h * p.h * p.h);
    sa.blk_off = w.blk_off; sa.blk_list = w.blk_list; sa.blk_color = w.blk_key;
    sa.bc = w.pk.bc; sa.bf = w.pk.bf; sa.wc = w.pk.wc; sa.wf = w.pk.wf;
    sa.val = f;
    sa.kind = kind;
    sa.field = (T *)field;
    const dim3 grid(c->nblk[0], c->nblk[1], c->nblk[2]);
    hipLaunchKernelGGL(k_sparse<T>, grid, dim3(SP_THREADS), 0, c->stream, sa);
    return hipGetLastError();
}

template <typename T>
hipError_t init_u_impl(ic_ctx *c) {
    void *U[4] = {c->f[0], c->f[1], c->f[2], c->f[3]};
    PartArgs<T> pa = part_args<T>(c, U);
    hipLaunchKernelGGL(k_init_u<T>, dim3(wave_blocks(c->np)), dim3(256), 0, c->stream, pa);
    return hipGetLastError();
}

constexpr int SUM_BLOCKS = 1024;

template <typename T>
hipError_t sums_impl(ic_ctx *c, double *host4) {
    const size_t n = (size_t)c->p.nx * c->p.ny * c->p.nz;
    hipLaunchKernelGGL(k_sums<T>, dim3(SUM_BLOCKS), dim3(256), 0, c->stream, (const T *)c->f[0],
                       (const T *)c->f[1], (const T *)c->f[2], (const T *)c->f[3], n, c->ws.red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    static thread_local double part[4 * SUM_BLOCKS];
    e = hipMemcpyAsync(part, c->ws.red, sizeof(part), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    for (int k = 0; k < 4; ++k) host4[k] = 0.0;
    for (int b = 0; b < SUM_BLOCKS; ++b)
        for (int k = 0; k < 4; ++k) host4[k] += part[4 * b + k];
    return hipSuccess;
}

}  // namespace

// Reverse of one deterministic step (see k_adj_tile and the k_adjp_*
// kernels).  The stage inputs U1, U2 of step n are recomputed from U^n with
// the forward stage kernels into the workspace stage buffers; with
// particles, also the particle prologue at q^n, the third stage output
// (into L1) and the no-slip-corrected momentum (into acc), which the
// reversed substeps 4-7 read before the stage reversal overwrites them.
template <typename T>
hipError_t adjoint_impl(ic_ctx *c, int64_t n, const void *const Un[4], void *const lam[4],
                        const AdjParticles *pp) {
    const ic_params &p = c->p;
    hipStream_t s = c->stream;
    const Workspace &w = c->ws;
    const AdjWorkspace &aw = c->adj;
    const size_t ncell = (size_t)p.nx * p.ny * p.nz;
    const unsigned nb = (unsigned)((ncell + 255) / 256);
    const unsigned nblk_all = (unsigned)(c->nblk[0] * c->nblk[1] * c->nblk[2]);
    const bool full = p.nx % TX == 0 && p.ny % TY == 0;
    const int np = pp ? c->np : 0;
    // every block of the momentum pass owns one partial-sum slot per mode
    const int atz = adjoint_tz(p);
    if ((long)((p.nx + ATX - 1) / ATX) * ((p.ny + ATY - 1) / ATY) * ((p.nz + atz - 1) / atz) >
        adjoint_blocks(p))
        return hipErrorInvalidValue;
    PartArgs<T> pa{};
    if (np > 0) {
        void *f[4] = {const_cast<void *>(Un[0]), const_cast<void *>(Un[1]),
                      const_cast<void *>(Un[2]), const_cast<void *>(Un[3])};
        pa = part_args<T>(c, f);
        hipLaunchKernelGGL(k_adjp_positions, dim3(thread_blocks(3 * np)), dim3(256), 0, s, np, pp->q,
                           aw.pq, p.nx * p.h, p.ny * p.h, p.nz * p.h, w.flag);
        pa.q = aw.pq;
        pa.u = const_cast<double *>(pp->u);
    }
    // particle terms of recomputed stage st, written into the stage output
    // dst (and the next stage's Omega from its density)
    auto stage_particles = [&](int st, void *const *dst) {
        if (np == 0) return;
        StagePassArgs<T> sp = stage_pass_args<T>(c, st);
        sp.drho_next = (const T *)dst[0];
        for (int i = 0; i < 3; ++i) sp.g[i] = (T *)dst[1 + i];
        hipLaunchKernelGGL(k_cl_stage<T>, dim3(wave_blocks(np)), dim3(256), 0, s, sp);
    };

    // stage inputs of step n
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, w.st, (int64_t)n);
    DriveArgs d{};
    d.nmodes = c->forcing.nmodes;
    d.dt = p.dt;
    for (int m = 0; m < d.nmodes; ++m) {
        d.amp[m] = c->forcing.modes[m].amp;
        d.omega[m] = c->forcing.modes[m].omega;
        d.phase[m] = c->forcing.modes[m].phase;
    }
    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(64), 0, s, w.st, d);
    StageArgs<T> a{};
    a.nx = p.nx; a.ny = p.ny; a.nz = p.nz; a.tz = c->tz;
    a.gx = c->nblk[0]; a.gy = c->nblk[1]; a.gz = c->nblk[2];
    a.rho0 = (T)p.rho0;
    a.cf2 = (T)(p.cf * p.cf);
    a.eta = (T)p.eta;
    a.lam = (T)(p.zeta - 2.0 * p.eta / 3.0);
    a.inv_h = (T)(1.0 / p.h);
    a.dt_h = (T)(p.dt / p.h);
    a.dt = (T)p.dt;
    a.fbytes = (uint32_t)(ncell * sizeof(T));
    a.nmodes = c->forcing.nmodes;
    a.prof = w.prof;
    a.pstride = c->prof_stride;
    for (int m = 0; m < a.nmodes; ++m) a.maxis[m] = c->forcing.modes[m].axis;
    for (int i = 0; i < 4; ++i) {
        a.in[i] = (const T *)Un[i];
        a.un[i] = (const T *)Un[i];
        a.out[i] = (T *)w.A[i];
    }
    if (np > 0) {
        hipLaunchKernelGGL(k_pre<T>, dim3(wave_blocks(np)), dim3(256), 0, s, pa);
        launch_clusters(c, np, s);
    }
    a.ra = (T)0.0;
    a.rb = (T)1.0;
    a.amp = w.st->amp[0];
    if (full)
        hipLaunchKernelGGL((stage_kernel<T, 0, false, true>), dim3(nblk_all), dim3(STAGE_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((stage_kernel<T, 0, false, false>), dim3(nblk_all), dim3(STAGE_THREADS), 0, s, a);
    stage_particles(0, w.A);
    for (int i = 0; i < 4; ++i) {
        a.in[i] = (const T *)w.A[i];
        a.out[i] = (T *)w.B[i];
    }
    a.ra = (T)0.75;
    a.rb = (T)0.25;
    a.amp = w.st->amp[1];
    if (full)
        hipLaunchKernelGGL((stage_kernel<T, 1, false, true>), dim3(nblk_all), dim3(STAGE_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((stage_kernel<T, 1, false, false>), dim3(nblk_all), dim3(STAGE_THREADS), 0, s, a);
    stage_particles(1, w.B);

    AdjPartArgs<T> pr{};
    if (np > 0) {
        // third stage into L1, its no-slip-corrected momentum into acc
        for (int i = 0; i < 4; ++i) {
            a.in[i] = (const T *)w.B[i];
            a.out[i] = (T *)aw.L1[i];
        }
        a.ra = (T)(1.0 / 3.0);
        a.rb = (T)(2.0 / 3.0);
        a.amp = w.st->amp[2];
        if (full)
            hipLaunchKernelGGL((stage_kernel<T, 2, false, true>), dim3(nblk_all), dim3(STAGE_THREADS), 0, s, a);
        else
            hipLaunchKernelGGL((stage_kernel<T, 2, false, false>), dim3(nblk_all), dim3(STAGE_THREADS), 0, s, a);
        stage_particles(2, aw.L1);
        for (int i = 1; i < 4; ++i) {
            const hipError_t e = hipMemcpyAsync(aw.acc[i], aw.L1[i], ncell * sizeof(T),
                                                hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
        }
        for (int i = 0; i < 4; ++i) pa.f[i] = (const T *)aw.L1[i];
        {
            // substeps 4-6: impulse from the third stage output, corrections
            // into the copy of its momentum
            PostPassArgs<T> po = post_args<T>(c);
            po.pa = pa;
            for (int i = 0; i < 3; ++i) po.g[i] = (T *)aw.acc[1 + i];
            hipLaunchKernelGGL(k_cl_noslip<T>, dim3(wave_blocks(np)), dim3(256), 0, s, po);
        }
        // substeps 7, 6, 5, 4 reversed
        pr.G = Grid{p.nx, p.ny, p.nz, p.h, 1.0 / p.h, p.rho0};
        pr.np = np;
        pr.dt = p.dt;
        pr.V = 8.0 * p.h * p.h * p.h;
        pr.inv_h3 = 1.0 / (p.h * p.h * p.h);
        pr.L[0] = p.nx * p.h;
        pr.L[1] = p.ny * p.h;
        pr.L[2] = p.nz * p.h;
        for (int i = 0; i < 4; ++i) {
            pr.Un[i] = (const T *)Un[i];
            pr.U3[i] = (const T *)aw.L1[i];
            pr.lam[i] = (T *)lam[i];
        }
        for (int i = 0; i < 3; ++i) pr.gnew[i] = (const T *)aw.acc[1 + i];
        pr.q = aw.pq;
        pr.u = pp->u;
        pr.lq = pp->lq;
        pr.lu = pp->lu;
        pr.lF = pp->lF;
        pr.me = w.me; pr.eps = w.eps; pr.ks = w.ks; pr.qeq = w.qeq; pr.qh = w.qh; pr.F = w.F;
        pr.un = w.Vt; pr.du = w.du; pr.mf = w.mf;
        pr.lqh = aw.plqh; pr.lFt = aw.plF; pr.lVt = aw.plVt; pr.lmf = aw.plmf;
        pr.dme = aw.pdme; pr.deps = aw.pdeps; pr.dks = aw.pdks;
        const dim3 pg(wave_blocks(np));
        hipLaunchKernelGGL(k_adjp_final<T>, pg, dim3(256), 0, s, pr);
        hipLaunchKernelGGL(k_adjp_noslip<T>, pg, dim3(256), 0, s, pr);
        hipLaunchKernelGGL(k_adjp_velocity<T>, pg, dim3(256), 0, s, pr);
    }

    // reverse the three stages: (stage input, adjoint in, adjoint out, cs, ds)
    const double tn = (double)n * p.dt;
    const double ts[3] = {tn, tn + p.dt, tn + 0.5 * p.dt};
    const void *const *Uin[3] = {Un, (const void *const *)w.A, (const void *const *)w.B};
    void *const *Lout[3] = {lam, aw.L1, aw.L2};
    const void *const *Lin[3] = {(const void *const *)aw.L1, (const void *const *)aw.L2,
                                 (const void *const *)lam};
    const double cs[3] = {1.0, 0.25, 2.0 / 3.0}, ds[3] = {1.0, 0.75, 1.0 / 3.0};
    for (int st = 2; st >= 0; --st) {
        AdjArgs<T> x{};
        for (int i = 0; i < 4; ++i) {
            x.U[i] = (const T *)Uin[st][i];
            x.lam[i] = (const T *)Lin[st][i];
            x.out[i] = (T *)Lout[st][i];
            x.acc[i] = (T *)aw.acc[i];
        }
        for (int i = 0; i < 3; ++i) x.murf[i] = (T *)aw.murf[i];
        x.mur = (T *)aw.mur;
        x.nx = p.nx; x.ny = p.ny; x.nz = p.nz;
        x.mode = st == 2 ? ADJ_FIRST : (st == 1 ? ADJ_MID : ADJ_LAST);
        x.rho0 = p.rho0;
        x.cf2 = p.cf * p.cf;
        x.eta = p.eta;
        x.lam_b = p.zeta - 2.0 * p.eta / 3.0;
        x.k = p.dt / p.h;
        x.inv_h = 1.0 / p.h;
        x.cs = cs[st];
        x.ds = ds[st];
        x.nmodes = c->forcing.nmodes;
        x.pstride = c->prof_stride;
        x.prof = w.prof;
        x.partial = aw.partial;
        for (int m = 0; m < c->forcing.nmodes; ++m) {
            const ic_mode &md = c->forcing.modes[m];
            x.dc.axis[m] = md.axis;
            x.dc.c[m] = cs[st] * sin(md.omega * ts[st] + md.phase);
        }
        x.nbp = adjoint_blocks(p);
        x.tz = atz;
        x.gx = (p.nx + ATX - 1) / ATX;
        x.gy = (p.ny + ATY - 1) / ATY;
        x.gz = (p.nz + atz - 1) / atz;
        hipLaunchKernelGGL(k_adj_tile<T>, dim3(x.gx * x.gy * x.gz), dim3(ATHREADS), 0, s, x);
        hipLaunchKernelGGL(k_adj_rho<T>, dim3(nb), dim3(256), 0, s, x);
        if (np > 0) {
            pr.cs = cs[st];
            pr.Us = (const T *)Uin[st][0];
            for (int i = 0; i < 4; ++i) {
                pr.lin[i] = (const T *)Lin[st][i];
                pr.lam[i] = (T *)Lout[st][i];
            }
            hipLaunchKernelGGL(k_adjp_stage<T>, dim3(wave_blocks(np)), dim3(256), 0, s, pr);
        }
    }
    if (np > 0) {
        for (int i = 0; i < 4; ++i) pr.lam[i] = (T *)lam[i];
        hipLaunchKernelGGL(k_adjp_start<T>, dim3(wave_blocks(np)), dim3(256), 0, s, pr);
    }
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, w.st, (int64_t)c->step);
    return hipGetLastError();
}

hipError_t launch_adjoint_step(ic_ctx *c, int64_t n, const void *const Un[4], void *const lam[4],
                               const AdjParticles *pp) {
    return c->p.prec == IC_FP64 ? adjoint_impl<double>(c, n, Un, lam, pp)
                                : adjoint_impl<float>(c, n, Un, lam, pp);
}

hipError_t launch_step(ic_ctx *c, bool overlap, bool first, bool last) {
    return c->p.prec == IC_FP64 ? step_impl<double>(c, overlap, first, last)
                                : step_impl<float>(c, overlap, first, last);
}
hipError_t launch_interpolate(ic_ctx *c, int n, const double *q, int kind, const void *field,
                              double *out) {
    return c->p.prec == IC_FP64 ? interp_impl<double>(c, n, q, kind, field, out)
                                : interp_impl<float>(c, n, q, kind, field, out);
}
hipError_t launch_spread(ic_ctx *c, int n, const double *q, const double *f, int kind,
                         void *field) {
    return c->p.prec == IC_FP64 ? spread_impl<double>(c, n, q, f, kind, field)
                                : spread_impl<float>(c, n, q, f, kind, field);
}
hipError_t launch_init_velocity(ic_ctx *c) {
    return c->p.prec == IC_FP64 ? init_u_impl<double>(c) : init_u_impl<float>(c);
}
hipError_t launch_conserved(ic_ctx *c, double *host_out) {
    return c->p.prec == IC_FP64 ? sums_impl<double>(c, host_out) : sums_impl<float>(c, host_out);
}

hipError_t launch_set_step(ic_ctx *c) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, c->stream, c->ws.st, (int64_t)c->step);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Staging memory of ic_interpolate_noalloc: a file-scope device array (one
// copy on every GPU the library runs on, held until the process ends) in
// place of the temporary allocation of ic_interpolate.  In host code the
// array's name is only a host-side stand-in, never a device address: the
// address is looked up once per GPU with hipGetSymbolAddress, with that GPU
// current, and only the looked-up pointer is passed to copies and kernels.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t SCRATCH_DOUBLES = 6 * (size_t)IC_NOALLOC_MAX_POINTS;  // [n][3] q + [n][3] out
__device__ __align__(256) double scratch[SCRATCH_DOUBLES];
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;                              // guards the lookup table
std::mutex scratch_use[SCRATCH_MAX_DEVICES];        // one staged call per GPU at a time
double *scratch_ptr[SCRATCH_MAX_DEVICES];

hipError_t scratch_address(int device, double **out) {
    *out = nullptr;
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        scratch_ptr[device] = (double *)ptr;
    }
    *out = scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

hipError_t launch_interpolate_noalloc(ic_ctx *c, int n, const double *q, bool q_dev, int kind,
                                      const void *field, double *out, bool out_dev) {
    if (n > IC_NOALLOC_MAX_POINTS) return hipErrorInvalidValue;
    double *scr = nullptr;
    hipError_t e = scratch_address(c->device, &scr);
    if (e != hipSuccess) return e;
    const size_t nq = 3 * (size_t)n, no = (kind == IC_FACES ? 3 : 1) * (size_t)n;
    std::lock_guard<std::mutex> lk(scratch_use[c->device]);
    const double *qd = q_dev ? q : scr;
    double *od = out_dev ? out : scr + 3 * (size_t)IC_NOALLOC_MAX_POINTS;
    if (!q_dev) e = hipMemcpyAsync(scr, q, nq * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_interpolate(c, n, qd, kind, field, od);
    if (e == hipSuccess && !out_dev)
        e = hipMemcpyAsync(out, od, no * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    // the staging memory is free for the next call once the stream is idle
    const hipError_t es = hipStreamSynchronize(c->stream);
    return e != hipSuccess ? e : es;
}

}  // namespace ic
