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
// keeping three planes of density, two of momentum and velocity and one of
// fluxes in LDS, so every value is loaded from HBM once per sweep and every
// flux and every random number is computed once (plus a one-cell ring of
// halo fluxes).  Random numbers are drawn in-kernel from a counter-based
// Philox generator keyed by (seed; cell, step, call, replica).  Particle
// terms enter through per-block candidate lists built once per step (no
// float atomics anywhere, so results are bitwise reproducible).
#include <math.h>

#include "ic_internal.h"

namespace ic {
namespace {

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

// The three kernel points along one axis reached from coordinate q: cell
// centres sit at i h, faces at (i + 1/2) h.  Returns the first (wrapped)
// index and the three weights.
__device__ __forceinline__ int axis_points(double q, double inv_h, int n, bool face,
                                           double w[3]) {
    const double x = q * inv_h - (face ? 0.5 : 0.0);
    const double nearest = floor(x + 0.5);
#pragma unroll
    for (int d = 0; d < 3; ++d) w[d] = phi3(x - (nearest - 1.0 + d));
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

template <typename T>
__device__ __forceinline__ T uniform23(uint32_t w);
template <>
__device__ __forceinline__ float uniform23<float>(uint32_t w) {
    return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}
template <>
__device__ __forceinline__ double uniform23<double>(uint32_t w) {
    return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

template <typename T>
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, T &z0, T &z1);
template <>
__device__ __forceinline__ void box_muller<double>(uint32_t a, uint32_t b, double &z0,
                                                   double &z1) {
    const double u1 = uniform23<double>(a), u2 = uniform23<double>(b);
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z0 = r * c;
    z1 = r * s;
}
template <>
__device__ __forceinline__ void box_muller<float>(uint32_t a, uint32_t b, float &z0, float &z1) {
    const float u1 = uniform23<float>(a), u2 = uniform23<float>(b);
    // v_log_f32 is log2; v_sin_f32 / v_cos_f32 take the angle in turns.
    const float r = __builtin_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
    z0 = r * __builtin_amdgcn_cosf(u2);
    z1 = r * __builtin_amdgcn_sinf(u2);
}

struct NoiseKey {
    uint32_t k0, k1, step, replica;
};

// The six noise components of one cell for an RK stage, Z = W_A + wB W_B,
// ordered xx, yy, zz, xy, xz, yz.  Philox calls: 0 -> A_xx A_yy A_zz A_xy,
// 1 -> A_xz A_yz B_xz B_yz, 2 -> B_xx B_yy B_zz B_xy.
template <typename T, bool WB>
__device__ __forceinline__ void cell_noise(uint32_t cell, const NoiseKey &nk, T wB, T Z[6]) {
    const U4 r0 = philox(cell, nk.step, 0u, nk.replica, nk.k0, nk.k1);
    const U4 r1 = philox(cell, nk.step, 1u, nk.replica, nk.k0, nk.k1);
    box_muller<T>(r0.x, r0.y, Z[0], Z[1]);
    box_muller<T>(r0.z, r0.w, Z[2], Z[3]);
    box_muller<T>(r1.x, r1.y, Z[4], Z[5]);
    if (WB) {
        T b[6];
        box_muller<T>(r1.z, r1.w, b[4], b[5]);
        const U4 r2 = philox(cell, nk.step, 2u, nk.replica, nk.k0, nk.k1);
        box_muller<T>(r2.x, r2.y, b[0], b[1]);
        box_muller<T>(r2.z, r2.w, b[2], b[3]);
#pragma unroll
        for (int c = 0; c < 6; ++c) Z[c] += wB * b[c];
    }
}

// ---------------------------------------------------------------------------
// Fluid RK stage (App. A, SSP-RK3; fluxes of Sec. IV B with the staggered
// discretisation described in ic_oracle's reading and the design notes).
// ---------------------------------------------------------------------------
template <typename T>
struct StageArgs {
    const T *in[4];   // stage input U^s
    const T *un[4];   // U^n (stages 2 and 3)
    T *out[4];
    int nx, ny, nz;
    T rho0, cf2, eta, lam, inv_h, dt_h, dt, ra, rb, wB;
    T sd, st, so;      // stochastic stress amplitudes (diag, trace, off-diagonal)
    NoiseKey nk;
    // particles at q^{n+1/2}
    int np;
    const int32_t *blk_off, *blk_list;
    const int32_t *bc, *bf;
    const double *wc, *wf, *omega, *F;
    double inv_h3;
    // imposed pressure: sum_m mamp[m] * prof[m][coord(maxis[m])]
    int nmodes;
    int maxis[IC_MAX_MODES];
    double mamp[IC_MAX_MODES];
    const double *prof;
    int pstride;
};

constexpr int PX = TX + 3;  // local x in [-1, TX+1]
constexpr int PY = TY + 3;  // local y in [-1, TY+1]
constexpr int PS = PX * PY;

__device__ __forceinline__ int lidx(int lx, int ly) { return (ly + 1) * PX + (lx + 1); }

// Particle pressure sum_p Omega_p w_p / h^3 at cell (x, y, z) and the
// imposed pressure there.
template <typename T>
__device__ __forceinline__ T extra_pressure(const StageArgs<T> &a, int cb, int ce, int x, int y,
                                            int z) {
    double p = 0.0;
    for (int c = cb; c < ce; ++c) {
        const int pid = a.blk_list[c];
        int dz = z - a.bc[3 * pid + 2];
        if (dz < 0) dz += a.nz;
        if (dz >= 3) continue;
        int dx = x - a.bc[3 * pid + 0];
        if (dx < 0) dx += a.nx;
        int dy = y - a.bc[3 * pid + 1];
        if (dy < 0) dy += a.ny;
        if (dx < 3 && dy < 3)
            p += a.omega[pid] * a.wc[9 * pid + 0 + dx] * a.wc[9 * pid + 3 + dy] *
                 a.wc[9 * pid + 6 + dz];
    }
    p *= a.inv_h3;
    for (int m = 0; m < a.nmodes; ++m) {
        const int ax = a.maxis[m];
        const int coord = ax == 0 ? x : (ax == 1 ? y : z);
        p += a.mamp[m] * a.prof[m * a.pstride + coord];
    }
    return (T)p;
}

// Spread external force S_alpha F at the three faces of cell (x, y, z).
template <typename T>
__device__ __forceinline__ void face_force(const StageArgs<T> &a, int cb, int ce, int x, int y,
                                           int z, T f[3]) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int c = cb; c < ce; ++c) {
        const int pid = a.blk_list[c];
        const int32_t *bc = a.bc + 3 * pid, *bf = a.bf + 3 * pid;
        const double *wc = a.wc + 9 * pid, *wf = a.wf + 9 * pid;
        int cz = z - bc[2], fz = z - bf[2];
        if (cz < 0) cz += a.nz;
        if (fz < 0) fz += a.nz;
        if (cz >= 3 && fz >= 3) continue;
        int cx = x - bc[0], fx = x - bf[0], cy = y - bc[1], fy = y - bf[1];
        if (cx < 0) cx += a.nx;
        if (fx < 0) fx += a.nx;
        if (cy < 0) cy += a.ny;
        if (fy < 0) fy += a.ny;
        const double *F = a.F + 3 * pid;
        if (fx < 3 && cy < 3 && cz < 3) s[0] += F[0] * wf[0 + fx] * wc[3 + cy] * wc[6 + cz];
        if (cx < 3 && fy < 3 && cz < 3) s[1] += F[1] * wc[0 + cx] * wf[3 + fy] * wc[6 + cz];
        if (cx < 3 && cy < 3 && fz < 3) s[2] += F[2] * wc[0 + cx] * wc[3 + cy] * wf[6 + fz];
    }
    f[0] = (T)(s[0] * a.inv_h3);
    f[1] = (T)(s[1] * a.inv_h3);
    f[2] = (T)(s[2] * a.inv_h3);
}

template <typename T, int STAGE, bool NOISE>
__global__ __launch_bounds__(STAGE_THREADS) void stage_kernel(const StageArgs<T> a) {
    __shared__ T s_rho[3][PS];
    __shared__ T s_g[2][3][PS];
    __shared__ T s_vx[2][PS], s_vy[2][PS], s_vz[3][PS];
    __shared__ T s_fl[6][PS];  // Pxx, Pyy, Pxy, Pyx, Pzx, Pzy at the current plane

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
    const int W = min(TX, nx - x0), Wy = min(TY, ny - y0), z1 = min(z0 + TZ, nz);
    const int lx = tid % TX, ly = tid / TX;
    const bool own = lx < W && ly < Wy;
    const int gxo = x0 + lx, gyo = y0 + ly;
    const int li = lidx(lx, ly);
    int cb = 0, ce = 0;
    if (a.np > 0) {
        const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        cb = a.blk_off[blk];
        ce = a.blk_off[blk + 1];
    }
    const T rho0 = a.rho0, half = (T)0.5, quarter = (T)0.25;
    const int nrr = (W + 3) * (Wy + 3);  // density region [-1, W+1] x [-1, Wy+1]
    const int nrg = (W + 2) * (Wy + 2);  // momentum/velocity region [-1, W] x [-1, Wy]

    auto gaddr = [&](int lxx, int lyy, int z) {
        const int x = wrap(x0 + lxx, nx), y = wrap(y0 + lyy, ny);
        return (size_t)((z * ny + y) * nx + x);
    };
    auto load_rho = [&](int p) {  // plane p (unwrapped) of density into LDS
        const int z = wrap(p, nz);
        T *dst = s_rho[(p + 3) % 3];
        for (int i = tid; i < nrr; i += STAGE_THREADS) {
            const int lxx = i % (W + 3) - 1, lyy = i / (W + 3) - 1;
            dst[lidx(lxx, lyy)] = a.in[0][gaddr(lxx, lyy, z)];
        }
    };
    // Momentum of plane p into LDS and velocity v = g / rho_face there; needs
    // density of plane p in LDS and reads plane p+1 density for v^z.
    auto load_g_vel = [&](int p) {
        const int z = wrap(p, nz), zp = wrap(p + 1, nz);
        const T *r = s_rho[(p + 3) % 3];
        T *gx = s_g[(p + 2) & 1][0], *gy = s_g[(p + 2) & 1][1], *gz = s_g[(p + 2) & 1][2];
        T *vx = s_vx[(p + 2) & 1], *vy = s_vy[(p + 2) & 1], *vz = s_vz[(p + 3) % 3];
        for (int i = tid; i < nrg; i += STAGE_THREADS) {
            const int lxx = i % (W + 2) - 1, lyy = i / (W + 2) - 1;
            const size_t ga = gaddr(lxx, lyy, z);
            const int l = lidx(lxx, lyy);
            const T g0 = a.in[1][ga], g1 = a.in[2][ga], g2 = a.in[3][ga];
            const T rz = a.in[0][gaddr(lxx, lyy, zp)];
            gx[l] = g0;
            gy[l] = g1;
            gz[l] = g2;
            vx[l] = g0 / (rho0 + half * (r[l] + r[l + 1]));
            vy[l] = g1 / (rho0 + half * (r[l] + r[l + PX]));
            vz[l] = g2 / (rho0 + half * (r[l] + rz));
        }
    };

    // ---- prologue: planes z0-1 and z0 of density, plane z0-1 of momentum
    load_rho(z0 - 1);
    load_rho(z0);
    __syncthreads();
    load_g_vel(z0 - 1);
    T Zc[6] = {0, 0, 0, 0, 0, 0}, Zn[6] = {0, 0, 0, 0, 0, 0};
    if (NOISE && own)
        cell_noise<T, STAGE != 2>((uint32_t)gaddr(lx, ly, wrap(z0 - 1, nz)), a.nk, a.wB, Zc);
    __syncthreads();

    T Pzz_cur = 0, Pxz_prev = 0, Pyz_prev = 0, gz_prev = 0, pex_cur = 0;

    for (int k = z0 - 1; k < z1; ++k) {
        const bool prep = (k == z0 - 1);
        // ---- phase A: density of plane k+2, momentum and velocity of plane k+1
        load_rho(k + 2);
        load_g_vel(k + 1);
        __syncthreads();

        const T *rk = s_rho[(k + 3) % 3], *rk1 = s_rho[(k + 4) % 3];
        const T *gx = s_g[(k + 2) & 1][0], *gy = s_g[(k + 2) & 1][1], *gz = s_g[(k + 2) & 1][2];
        const T *gx1 = s_g[(k + 3) & 1][0], *gy1 = s_g[(k + 3) & 1][1],
                *gz1 = s_g[(k + 3) & 1][2];
        const T *vx = s_vx[(k + 2) & 1], *vy = s_vy[(k + 2) & 1], *vz = s_vz[(k + 3) % 3];
        const T *vx1 = s_vx[(k + 3) & 1], *vy1 = s_vy[(k + 3) & 1], *vz1 = s_vz[(k + 4) % 3];
        const T *vzm = s_vz[(k + 2) % 3];
        const int zk = wrap(k, nz), zk1 = wrap(k + 1, nz);

        // ---- phase B: fluxes
        T Pzz_next = 0, Pxz_cur = 0, Pyz_cur = 0, pex_next = 0;
        if (own) {
            if (NOISE)
                cell_noise<T, STAGE != 2>((uint32_t)gaddr(lx, ly, zk1), a.nk, a.wB, Zn);
            // centre flux zz at plane k+1
            pex_next = extra_pressure(a, cb, ce, gxo, gyo, zk1);
            const int l = li;
            const T div1 = ((vx1[l] - vx1[l - 1]) + (vy1[l] - vy1[l - PX]) + (vz1[l] - vz[l])) *
                           a.inv_h;
            T pzz = a.cf2 * rk1[l] + pex_next + quarter * (gz1[l] + gz[l]) * (vz1[l] + vz[l]) -
                    (2 * a.eta * (vz1[l] - vz[l]) * a.inv_h + a.lam * div1);
            if (NOISE) pzz -= a.sd * Zn[2] + a.st * (Zn[0] + Zn[1] + Zn[2]);
            Pzz_next = pzz;
            // edge fluxes along z at plane k (own column only)
            const T viz_x = a.eta * ((vx1[l] - vx[l]) + (vz[l + 1] - vz[l])) * a.inv_h;
            const T viz_y = a.eta * ((vy1[l] - vy[l]) + (vz[l + PX] - vz[l])) * a.inv_h;
            Pxz_cur = quarter * (gx[l] + gx1[l]) * (vz[l] + vz[l + 1]) - viz_x;
            Pyz_cur = quarter * (gy[l] + gy1[l]) * (vz[l] + vz[l + PX]) - viz_y;
            if (NOISE) {
                Pxz_cur -= a.so * Zc[4];
                Pyz_cur -= a.so * Zc[5];
            }
            if (!prep) {
                const T pi = a.cf2 * rk[l] + pex_cur;
                const T div = ((vx[l] - vx[l - 1]) + (vy[l] - vy[l - PX]) + (vz[l] - vzm[l])) *
                              a.inv_h;
                T pxx = pi + quarter * (gx[l] + gx[l - 1]) * (vx[l] + vx[l - 1]) -
                        (2 * a.eta * (vx[l] - vx[l - 1]) * a.inv_h + a.lam * div);
                T pyy = pi + quarter * (gy[l] + gy[l - PX]) * (vy[l] + vy[l - PX]) -
                        (2 * a.eta * (vy[l] - vy[l - PX]) * a.inv_h + a.lam * div);
                const T vxy = a.eta * ((vx[l + PX] - vx[l]) + (vy[l + 1] - vy[l])) * a.inv_h;
                T pxy = quarter * (gx[l] + gx[l + PX]) * (vy[l] + vy[l + 1]) - vxy;
                T pyx = quarter * (gy[l] + gy[l + 1]) * (vx[l] + vx[l + PX]) - vxy;
                T pzx = quarter * (gz[l] + gz[l + 1]) * (vx[l] + vx1[l]) - viz_x;
                T pzy = quarter * (gz[l] + gz[l + PX]) * (vy[l] + vy1[l]) - viz_y;
                if (NOISE) {
                    const T tr = a.st * (Zc[0] + Zc[1] + Zc[2]);
                    pxx -= a.sd * Zc[0] + tr;
                    pyy -= a.sd * Zc[1] + tr;
                    pxy -= a.so * Zc[3];
                    pyx -= a.so * Zc[3];
                    pzx -= a.so * Zc[4];
                    pzy -= a.so * Zc[5];
                }
                s_fl[0][l] = pxx;
                s_fl[1][l] = pyy;
                s_fl[2][l] = pxy;
                s_fl[3][l] = pyx;
                s_fl[4][l] = pzx;
                s_fl[5][l] = pzy;
            }
        }
        if (!prep) {
            // ring of halo fluxes at plane k: +x column (xx), +y row (yy),
            // -x column (yx, zx), -y row (xy, zy)
            const int nh = 2 * (W + Wy);
            for (int i = tid; i < nh; i += STAGE_THREADS) {
                int hx, hy, type;
                if (i < Wy) {
                    hx = W; hy = i; type = 0;
                } else if (i < Wy + W) {
                    hx = i - Wy; hy = Wy; type = 1;
                } else if (i < 2 * Wy + W) {
                    hx = -1; hy = i - Wy - W; type = 2;
                } else {
                    hx = i - 2 * Wy - W; hy = -1; type = 3;
                }
                const int l = lidx(hx, hy);
                T Z[6] = {0, 0, 0, 0, 0, 0};
                if (NOISE) cell_noise<T, STAGE != 2>((uint32_t)gaddr(hx, hy, zk), a.nk, a.wB, Z);
                if (type <= 1) {
                    const T pe = extra_pressure(a, cb, ce, wrap(x0 + hx, nx), wrap(y0 + hy, ny), zk);
                    const T pi = a.cf2 * rk[l] + pe;
                    const T div = ((vx[l] - vx[l - 1]) + (vy[l] - vy[l - PX]) + (vz[l] - vzm[l])) *
                                  a.inv_h;
                    const T tr = NOISE ? a.st * (Z[0] + Z[1] + Z[2]) : (T)0;
                    if (type == 0) {
                        T pxx = pi + quarter * (gx[l] + gx[l - 1]) * (vx[l] + vx[l - 1]) -
                                (2 * a.eta * (vx[l] - vx[l - 1]) * a.inv_h + a.lam * div);
                        if (NOISE) pxx -= a.sd * Z[0] + tr;
                        s_fl[0][l] = pxx;
                    } else {
                        T pyy = pi + quarter * (gy[l] + gy[l - PX]) * (vy[l] + vy[l - PX]) -
                                (2 * a.eta * (vy[l] - vy[l - PX]) * a.inv_h + a.lam * div);
                        if (NOISE) pyy -= a.sd * Z[1] + tr;
                        s_fl[1][l] = pyy;
                    }
                } else if (type == 2) {
                    const T vxy = a.eta * ((vx[l + PX] - vx[l]) + (vy[l + 1] - vy[l])) * a.inv_h;
                    const T viz_x = a.eta * ((vx1[l] - vx[l]) + (vz[l + 1] - vz[l])) * a.inv_h;
                    T pyx = quarter * (gy[l] + gy[l + 1]) * (vx[l] + vx[l + PX]) - vxy;
                    T pzx = quarter * (gz[l] + gz[l + 1]) * (vx[l] + vx1[l]) - viz_x;
                    if (NOISE) {
                        pyx -= a.so * Z[3];
                        pzx -= a.so * Z[4];
                    }
                    s_fl[3][l] = pyx;
                    s_fl[4][l] = pzx;
                } else {
                    const T vxy = a.eta * ((vx[l + PX] - vx[l]) + (vy[l + 1] - vy[l])) * a.inv_h;
                    const T viz_y = a.eta * ((vy1[l] - vy[l]) + (vz[l + PX] - vz[l])) * a.inv_h;
                    T pxy = quarter * (gx[l] + gx[l + PX]) * (vy[l] + vy[l + 1]) - vxy;
                    T pzy = quarter * (gz[l] + gz[l + PX]) * (vy[l] + vy1[l]) - viz_y;
                    if (NOISE) {
                        pxy -= a.so * Z[3];
                        pzy -= a.so * Z[5];
                    }
                    s_fl[2][l] = pxy;
                    s_fl[5][l] = pzy;
                }
            }
        }
        __syncthreads();

        // ---- phase C: update of plane k
        if (!prep && own) {
            const int l = li;
            T f[3] = {0, 0, 0};
            if (ce > cb) face_force(a, cb, ce, gxo, gyo, zk, f);
            const T drho = -a.dt_h * ((gx[l] - gx[l - 1]) + (gy[l] - gy[l - PX]) + (gz[l] - gz_prev));
            const T dgx = -a.dt_h * ((s_fl[0][l + 1] - s_fl[0][l]) + (s_fl[2][l] - s_fl[2][l - PX]) +
                                     (Pxz_cur - Pxz_prev)) + a.dt * f[0];
            const T dgy = -a.dt_h * ((s_fl[1][l + PX] - s_fl[1][l]) + (s_fl[3][l] - s_fl[3][l - 1]) +
                                     (Pyz_cur - Pyz_prev)) + a.dt * f[1];
            const T dgz = -a.dt_h * ((Pzz_next - Pzz_cur) + (s_fl[4][l] - s_fl[4][l - 1]) +
                                     (s_fl[5][l] - s_fl[5][l - PX])) + a.dt * f[2];
            const size_t g = gaddr(lx, ly, zk);
            const T us[4] = {rk[l], gx[l], gy[l], gz[l]};
            const T d[4] = {drho, dgx, dgy, dgz};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                T v;
                if (STAGE == 0)
                    v = us[c] + d[c];
                else
                    v = a.ra * a.un[c][g] + a.rb * (us[c] + d[c]);
                a.out[c][g] = v;
            }
        }
        if (own) gz_prev = gz[li];
        Pzz_cur = Pzz_next;
        Pxz_prev = Pxz_cur;
        Pyz_prev = Pyz_cur;
        pex_cur = pex_next;
#pragma unroll
        for (int c = 0; c < 6; ++c) Zc[c] = Zn[c];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Particle kernels: one 64-lane wave per particle; the 27-point sums are
// reduced with a fixed butterfly so results do not depend on timing.
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

// Kernel point `pt` (0..26, x fastest) of location `kind` (0 cell, 1+a face
// a) around q: global element index and weight prod phi.
__device__ __forceinline__ void stencil_point(const Grid &G, const double q[3], int kind, int pt,
                                              size_t *idx, double *w) {
    const int d[3] = {pt % 3, (pt / 3) % 3, pt / 9};
    int c[3];
    double wt = 1.0;
    const int n[3] = {G.nx, G.ny, G.nz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        double ww[3];
        const int f = axis_points(q[ax], G.inv_h, n[ax], kind == ax + 1, ww);
        c[ax] = wrap(f + d[ax], n[ax]);
        wt *= ww[d[ax]];
    }
    *idx = ((size_t)c[2] * G.ny + c[1]) * G.nx + c[0];
    *w = wt;
}

// Face neighbour (+1 along axis ax) of element index i.
__device__ __forceinline__ size_t plus_one(const Grid &G, size_t i, int ax) {
    const int x = (int)(i % G.nx), y = (int)((i / G.nx) % G.ny), z = (int)(i / ((size_t)G.nx * G.ny));
    int c[3] = {x, y, z};
    const int n[3] = {G.nx, G.ny, G.nz};
    c[ax] = c[ax] + 1 == n[ax] ? 0 : c[ax] + 1;
    return ((size_t)c[2] * G.ny + c[1]) * G.nx + c[0];
}

// J_alpha (g^alpha / rho_face^alpha) for alpha = 0, 1, 2 at q; every lane of
// the wave gets the result.
template <typename T>
__device__ __forceinline__ void wave_velocity(const Grid &G, const T *const f[4], const double q[3],
                                              double out[3]) {
    const int lane = threadIdx.x & 63;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int item = lane; item < 81; item += 64) {
        const int ax = item / 27, pt = item % 27;
        size_t i;
        double w;
        stencil_point(G, q, ax + 1, pt, &i, &w);
        const size_t j = plus_one(G, i, ax);
        const double rf = G.rho0 + 0.5 * ((double)f[0][i] + (double)f[0][j]);
        acc[ax] += w * ((double)f[1 + ax][i] / rf);
    }
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) out[ax] = wave_sum(acc[ax]);
}

template <typename T>
struct PartArgs {
    Grid G;
    const T *f[4];   // fields read by the kernel
    T *fw[4];        // fields written (correction)
    int np;
    double dt, V, L[3];
    double *q, *u, *me, *eps, *ks, *qeq, *fext;
    double *qh, *jv_old, *F, *Vt, *du, *mf, *omega, *jv_new;
    int32_t *bc, *bf;
    double *wc, *wf;
    double *sum_f, *sum_l;
    int32_t *flag;
};

// Substeps 1-2 and the kernel weights at q^{n+1/2} (App. A).
template <typename T>
__global__ __launch_bounds__(256) void k_pre(const PartArgs<T> a) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    const int lane = threadIdx.x & 63;
    double q[3] = {a.q[3 * p], a.q[3 * p + 1], a.q[3 * p + 2]};
    double U[3];
    wave_velocity<T>(a.G, a.f, q, U);                         // J^n v^n at q^n
    double qh[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) qh[ax] = wrap_pos(q[ax] + 0.5 * a.dt * U[ax], a.L[ax]);
    double jv[3];
    wave_velocity<T>(a.G, a.f, qh, jv);                       // J^{n+1/2} v^n
    if (lane == 0) {
        const int n[3] = {a.G.nx, a.G.ny, a.G.nz};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            a.qh[3 * p + ax] = qh[ax];
            a.jv_old[3 * p + ax] = jv[ax];
            a.F[3 * p + ax] = -a.ks[p] * min_image(qh[ax] - a.qeq[3 * p + ax], a.L[ax]) +
                              a.fext[3 * p + ax];
            a.bc[3 * p + ax] = axis_points(qh[ax], a.G.inv_h, n[ax], false, a.wc + 9 * p + 3 * ax);
            a.bf[3 * p + ax] = axis_points(qh[ax], a.G.inv_h, n[ax], true, a.wf + 9 * p + 3 * ax);
        }
    }
}

// Kernel data for standalone spreading at caller positions.
__global__ void k_weights(const Grid G, int np, const double *q, double *qh, int32_t *bc,
                          int32_t *bf, double *wc, double *wf) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int n[3] = {G.nx, G.ny, G.nz};
    const double L[3] = {G.nx * G.h, G.ny * G.h, G.nz * G.h};
    for (int ax = 0; ax < 3; ++ax) {
        const double x = wrap_pos(q[3 * p + ax], L[ax]);
        qh[3 * p + ax] = x;
        bc[3 * p + ax] = axis_points(x, G.inv_h, n[ax], false, wc + 9 * p + 3 * ax);
        bf[3 * p + ax] = axis_points(x, G.inv_h, n[ax], true, wf + 9 * p + 3 * ax);
    }
}

// Omega_p = eps_p V J_p(rho - rho0) for the stage input density (Sec. III,
// Eq. omega; stage pressures of App. A).
template <typename T>
__global__ __launch_bounds__(256) void k_omega(const PartArgs<T> a, const T *drho) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    if (lane < 27) {
        const int d[3] = {lane % 3, (lane / 3) % 3, lane / 9};
        const int x = wrap(a.bc[3 * p] + d[0], a.G.nx), y = wrap(a.bc[3 * p + 1] + d[1], a.G.ny),
                  z = wrap(a.bc[3 * p + 2] + d[2], a.G.nz);
        const double w = a.wc[9 * p + d[0]] * a.wc[9 * p + 3 + d[1]] * a.wc[9 * p + 6 + d[2]];
        s = w * (double)drho[((size_t)z * a.G.ny + y) * a.G.nx + x];
    }
    s = wave_sum(s);
    if (lane == 0) a.omega[p] = a.eps[p] * a.V * s;
}

// Substeps 4-5 on the unconstrained state: V~ = J v~, m_f = V J rho_face,
// u^{n+1} = u^n + m_f/(m_e+m_f) (V~ - u^n); keeps du = V (u^{n+1} - V~).
template <typename T>
__global__ __launch_bounds__(256) void k_post(const PartArgs<T> a) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    const int lane = threadIdx.x & 63;
    const double qh[3] = {a.qh[3 * p], a.qh[3 * p + 1], a.qh[3 * p + 2]};
    double sv[3] = {0, 0, 0}, sm[3] = {0, 0, 0};
    for (int item = lane; item < 81; item += 64) {
        const int ax = item / 27, pt = item % 27;
        size_t i;
        double w;
        stencil_point(a.G, qh, ax + 1, pt, &i, &w);
        const size_t j = plus_one(a.G, i, ax);
        const double rf = a.G.rho0 + 0.5 * ((double)a.f[0][i] + (double)a.f[0][j]);
        sv[ax] += w * ((double)a.f[1 + ax][i] / rf);
        sm[ax] += w * rf;
    }
    double Vt[3], mf[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        Vt[ax] = wave_sum(sv[ax]);
        mf[ax] = a.V * wave_sum(sm[ax]);
    }
    if (lane == 0) {
        const double me = a.me[p];
        for (int ax = 0; ax < 3; ++ax) {
            if (!(me + mf[ax] > 0.0)) a.flag[0] = 1;
            const double u = a.u[3 * p + ax];
            const double un = u + mf[ax] / (me + mf[ax]) * (Vt[ax] - u);
            a.Vt[3 * p + ax] = un;  // u^{n+1}
            a.du[3 * p + ax] = a.V * (un - Vt[ax]);
            a.mf[3 * p + ax] = mf[ax];
        }
    }
}

// Substep 7 and the window sums: q^{n+1} = q^n + dt/2 J^{n+1/2}(v^{n+1}+v^n).
template <typename T>
__global__ __launch_bounds__(256) void k_final(const PartArgs<T> a) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.np) return;
    const int lane = threadIdx.x & 63;
    const double qh[3] = {a.qh[3 * p], a.qh[3 * p + 1], a.qh[3 * p + 2]};
    double jv[3];
    wave_velocity<T>(a.G, a.f, qh, jv);
    if (lane == 0) {
        for (int ax = 0; ax < 3; ++ax) {
            const double q = a.q[3 * p + ax];
            a.q[3 * p + ax] = wrap_pos(q + 0.5 * a.dt * (jv[ax] + a.jv_old[3 * p + ax]), a.L[ax]);
            const double un = a.Vt[3 * p + ax];
            const double F = a.F[3 * p + ax];
            const double lam = a.me[p] * (un - a.u[3 * p + ax]) / a.dt - F;
            a.sum_f[3 * p + ax] += -(F - a.fext[3 * p + ax]);
            a.sum_l[3 * p + ax] += lam;
            a.u[3 * p + ax] = un;
            a.jv_new[3 * p + ax] = jv[ax];
        }
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
    wave_velocity<T>(a.G, a.f, q, U);
    if (lane == 0)
        for (int ax = 0; ax < 3; ++ax) a.u[3 * p + ax] = U[ax];
}

// Standalone J of a caller field.
template <typename T>
__global__ __launch_bounds__(256) void k_interp(const Grid G, int np, const double *q, int kind,
                                                const T *field, double *out) {
    const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= np) return;
    const int lane = threadIdx.x & 63;
    const double L[3] = {G.nx * G.h, G.ny * G.h, G.nz * G.h};
    const double qq[3] = {wrap_pos(q[3 * p], L[0]), wrap_pos(q[3 * p + 1], L[1]),
                          wrap_pos(q[3 * p + 2], L[2])};
    double s = 0.0;
    if (lane < 27) {
        size_t i;
        double w;
        stencil_point(G, qq, kind, lane, &i, &w);
        s = w * (double)field[i];
    }
    s = wave_sum(s);
    if (lane == 0) out[p] = s;
}

// ---------------------------------------------------------------------------
// Binning of particles into stage blocks (one workgroup).  A particle is
// listed for every block whose cells, ring of halo cells or extra plane its
// kernel points (cell- or face-centred, within [f-1, f+2] of f = floor(q/h)
// per axis) can reach.  Lists are sorted by particle id.
// ---------------------------------------------------------------------------
struct BinArgs {
    int np, nx, ny, nz, gx, gy, gz, nblk;
    double inv_h;
    const double *qh;
    int32_t *count, *off, *cursor, *list;
};

// Distinct tile indices (tile size ts) touched by positions f-2 .. f+3.
__device__ __forceinline__ int axis_tiles(int f, int n, int ts, int out[3]) {
    int cnt = 0;
    for (int s = f - 2; s <= f + 3; ++s) {
        int t = ((s % n) + n) % n / ts;
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
    const int cz = axis_tiles((int)floor(q[2] * b.inv_h), b.nz, TZ, tz);
    int n = 0;
    for (int k = 0; k < cz; ++k)
        for (int j = 0; j < cy; ++j)
            for (int i = 0; i < cx; ++i) out[n++] = (tz[k] * b.gy + ty[j]) * b.gx + tx[i];
    return n;
}

__global__ __launch_bounds__(1024) void k_bin(const BinArgs b) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < b.nblk; i += nt) b.count[i] = 0;
    __syncthreads();
    for (int p = tid; p < b.np; p += nt) {
        int bl[27];
        const int n = particle_blocks(b, p, bl);
        for (int c = 0; c < n; ++c) atomicAdd(&b.count[bl[c]], 1);
    }
    __threadfence_block();
    __syncthreads();
    // exclusive scan of count -> off (contiguous chunk per thread)
    __shared__ int32_t part[1024];
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
        b.off[i] = run;
        b.cursor[i] = run;
        run += b.count[i];
    }
    if (tid == nt - 1) b.off[b.nblk] = part[nt - 1];
    __threadfence_block();
    __syncthreads();
    for (int p = tid; p < b.np; p += nt) {
        int bl[27];
        const int n = particle_blocks(b, p, bl);
        for (int c = 0; c < n; ++c) b.list[atomicAdd(&b.cursor[bl[c]], 1)] = p;
    }
    __threadfence_block();
    __syncthreads();
    for (int i = tid; i < b.nblk; i += nt) {
        const int s0 = b.off[i], s1 = b.off[i + 1];
        for (int m = s0 + 1; m < s1; ++m) {
            const int v = b.list[m];
            int j = m - 1;
            while (j >= s0 && b.list[j] > v) {
                b.list[j + 1] = b.list[j];
                --j;
            }
            b.list[j + 1] = v;
        }
    }
}

// Owner-computes spreading onto faces (or cells) of the blocks that hold
// candidates: field[c] += scale(i) * sum_p val_p w_p(i) / h^3, with
// scale = rho_face of `drho` when drho is given (the momentum correction of
// substep 6) and 1 otherwise.  Each grid point is written by one thread.
template <typename T>
struct SpreadArgs {
    int nx, ny, nz;
    double inv_h3, rho0;
    const int32_t *blk_off, *blk_list, *bc, *bf;
    const double *wc, *wf;
    const double *val;   // val[vstride * p + c]
    int vstride, ncomp, kind0;
    T *fields[3];
    const T *drho;
};

template <typename T>
__global__ __launch_bounds__(STAGE_THREADS) void k_spread_binned(const SpreadArgs<T> a) {
    const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const int cb = a.blk_off[blk], ce = a.blk_off[blk + 1];
    if (cb == ce) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= nx || y >= ny) return;
    const int z1 = min(z0 + TZ, nz);
    const int n[3] = {nx, ny, nz};
    for (int z = z0; z < z1; ++z) {
        const size_t g = ((size_t)z * ny + y) * nx + x;
        const int pos[3] = {x, y, z};
        for (int c = 0; c < a.ncomp; ++c) {
            const int kind = a.kind0 + c;  // 0 cell, 1+a face a
            double s = 0.0;
            bool hit = false;
            for (int ci = cb; ci < ce; ++ci) {
                const int pid = a.blk_list[ci];
                double w = 1.0;
                bool in = true;
                for (int ax = 0; ax < 3; ++ax) {
                    const bool face = kind == ax + 1;
                    int d = pos[ax] - (face ? a.bf[3 * pid + ax] : a.bc[3 * pid + ax]);
                    if (d < 0) d += n[ax];
                    if (d >= 3) {
                        in = false;
                        break;
                    }
                    w *= face ? a.wf[9 * pid + 3 * ax + d] : a.wc[9 * pid + 3 * ax + d];
                }
                if (in) {
                    s += a.val[a.vstride * pid + c] * w;
                    hit = true;
                }
            }
            if (hit) {
                double scale = 1.0;
                if (a.drho != nullptr && kind > 0) {
                    const int ax = kind - 1;
                    int nb[3] = {x, y, z};
                    nb[ax] = nb[ax] + 1 == n[ax] ? 0 : nb[ax] + 1;
                    const size_t j = ((size_t)nb[2] * ny + nb[1]) * nx + nb[0];
                    scale = a.rho0 + 0.5 * ((double)a.drho[g] + (double)a.drho[j]);
                }
                T *fld = a.fields[c];
                fld[g] = (T)((double)fld[g] + scale * s * a.inv_h3);
            }
        }
    }
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
    for (int i = 0; i < 4; ++i) {
        a.f[i] = (const T *)f[i];
        a.fw[i] = (T *)f[i];
    }
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
    b.inv_h = 1.0 / c->p.h;
    b.qh = qh;
    b.count = c->ws.blk_count;
    b.off = c->ws.blk_off;
    b.cursor = c->ws.blk_cursor;
    b.list = c->ws.blk_list;
    return b;
}

inline unsigned wave_blocks(int n) { return (unsigned)((n * 64 + 255) / 256); }

template <typename T>
hipError_t step_impl(ic_ctx *c) {
    const ic_params &p = c->p;
    hipStream_t s = c->stream;
    const Workspace &w = c->ws;
    void *U[4] = {c->f[0], c->f[1], c->f[2], c->f[3]};
    const dim3 grid(c->nblk[0], c->nblk[1], c->nblk[2]);
    const int np = c->np;
    PartArgs<T> pa = part_args<T>(c, U);

    if (np > 0) {
        hipLaunchKernelGGL(k_pre<T>, dim3(wave_blocks(np)), dim3(256), 0, s, pa);
        hipLaunchKernelGGL(k_bin, dim3(1), dim3(1024), 0, s, bin_args(c, np, w.qh));
    }

    StageArgs<T> a{};
    a.nx = p.nx; a.ny = p.ny; a.nz = p.nz;
    a.rho0 = (T)p.rho0;
    a.cf2 = (T)(p.cf * p.cf);
    a.eta = (T)p.eta;
    a.lam = (T)(p.zeta - 2.0 * p.eta / 3.0);
    a.inv_h = (T)(1.0 / p.h);
    a.dt_h = (T)(p.dt / p.h);
    a.dt = (T)p.dt;
    const double amp = 1.0 / sqrt(p.h * p.h * p.h * p.dt);
    const double an = sqrt(2.0 * p.eta * p.kT);
    const double bt = sqrt(p.zeta * p.kT / 3.0) - an / 3.0;
    a.sd = (T)(amp * an * sqrt(2.0));
    a.st = (T)(amp * bt * sqrt(2.0));
    a.so = (T)(amp * an);
    a.nk = NoiseKey{(uint32_t)(p.seed & 0xFFFFFFFFu), (uint32_t)(p.seed >> 32),
                    (uint32_t)(c->step & 0xFFFFFFFF), p.replica};
    a.np = np;
    a.blk_off = w.blk_off;
    a.blk_list = w.blk_list;
    a.bc = w.pk.bc; a.bf = w.pk.bf; a.wc = w.pk.wc; a.wf = w.pk.wf;
    a.omega = w.omega;
    a.F = w.F;
    a.inv_h3 = 1.0 / (p.h * p.h * p.h);
    a.nmodes = c->forcing.nmodes;
    a.prof = w.prof;
    a.pstride = c->prof_stride;
    for (int m = 0; m < a.nmodes; ++m) a.maxis[m] = c->forcing.modes[m].axis;

    const bool noise = p.kT > 0.0;
    const double tn = (double)c->step * p.dt;
    const double tst[3] = {tn, tn + p.dt, tn + 0.5 * p.dt};
    const double ra[3] = {0.0, 0.75, 1.0 / 3.0}, rb[3] = {1.0, 0.25, 2.0 / 3.0};
    const double wB[3] = {-sqrt(3.0), sqrt(3.0), 0.0};
    void *const A[4] = {w.A[0], w.A[1], w.A[2], w.A[3]};
    void *const B[4] = {w.B[0], w.B[1], w.B[2], w.B[3]};
    void *const *src[3] = {U, A, B};
    void *const *dst[3] = {A, B, U};
    for (int st = 0; st < 3; ++st) {
        if (np > 0)
            hipLaunchKernelGGL(k_omega<T>, dim3(wave_blocks(np)), dim3(256), 0, s, pa,
                               (const T *)src[st][0]);
        for (int i = 0; i < 4; ++i) {
            a.in[i] = (const T *)src[st][i];
            a.un[i] = (const T *)U[i];
            a.out[i] = (T *)dst[st][i];
        }
        a.ra = (T)ra[st];
        a.rb = (T)rb[st];
        a.wB = (T)wB[st];
        for (int m = 0; m < a.nmodes; ++m) {
            const ic_mode &md = c->forcing.modes[m];
            a.mamp[m] = md.amp * sin(md.omega * tst[st] + md.phase);
        }
        hipEvent_t e0 = prof_event(c), e1 = prof_event(c);
        if (e0) hipEventRecord(e0, s);
#define IC_STAGE(S, N) hipLaunchKernelGGL((stage_kernel<T, S, N>), grid, dim3(STAGE_THREADS), 0, s, a)
        if (noise) {
            if (st == 0) IC_STAGE(0, true); else if (st == 1) IC_STAGE(1, true); else IC_STAGE(2, true);
        } else {
            if (st == 0) IC_STAGE(0, false); else if (st == 1) IC_STAGE(1, false); else IC_STAGE(2, false);
        }
#undef IC_STAGE
        if (e1) {
            hipEventRecord(e1, s);
            prof_push(c, e0, e1);
        }
    }

    if (np > 0) {
        hipLaunchKernelGGL(k_post<T>, dim3(wave_blocks(np)), dim3(256), 0, s, pa);
        SpreadArgs<T> sa{};
        sa.nx = p.nx; sa.ny = p.ny; sa.nz = p.nz;
        sa.inv_h3 = 1.0 / (p.h * p.h * p.h);
        sa.rho0 = p.rho0;
        sa.blk_off = w.blk_off; sa.blk_list = w.blk_list;
        sa.bc = w.pk.bc; sa.bf = w.pk.bf; sa.wc = w.pk.wc; sa.wf = w.pk.wf;
        sa.val = w.du;
        sa.vstride = 3;
        sa.ncomp = 3;
        sa.kind0 = 1;
        for (int i = 0; i < 3; ++i) sa.fields[i] = (T *)U[1 + i];
        sa.drho = (const T *)U[0];
        hipLaunchKernelGGL(k_spread_binned<T>, grid, dim3(STAGE_THREADS), 0, s, sa);
        hipLaunchKernelGGL(k_final<T>, dim3(wave_blocks(np)), dim3(256), 0, s, pa);
    }
    return hipGetLastError();
}

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
    hipLaunchKernelGGL(k_weights, dim3((n + 255) / 256), dim3(256), 0, c->stream, G, n, q, w.qh,
                       w.pk.bc, w.pk.bf, w.pk.wc, w.pk.wf);
    hipLaunchKernelGGL(k_bin, dim3(1), dim3(1024), 0, c->stream, bin_args(c, n, w.qh));
    SpreadArgs<T> sa{};
    sa.nx = p.nx; sa.ny = p.ny; sa.nz = p.nz;
    sa.inv_h3 = 1.0 / (p.h * p.h * p.h);
    sa.rho0 = p.rho0;
    sa.blk_off = w.blk_off; sa.blk_list = w.blk_list;
    sa.bc = w.pk.bc; sa.bf = w.pk.bf; sa.wc = w.pk.wc; sa.wf = w.pk.wf;
    sa.val = f;
    sa.vstride = 1;
    sa.ncomp = 1;
    sa.kind0 = kind;
    sa.fields[0] = (T *)field;
    sa.drho = nullptr;
    const dim3 grid(c->nblk[0], c->nblk[1], c->nblk[2]);
    hipLaunchKernelGGL(k_spread_binned<T>, grid, dim3(STAGE_THREADS), 0, c->stream, sa);
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

hipError_t launch_step(ic_ctx *c) {
    return c->p.prec == IC_FP64 ? step_impl<double>(c) : step_impl<float>(c);
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

}  // namespace ic
