// rlbm.hip -- HIP (gfx950) kernels and C ABI of the d2v72 relativistic lattice
// Boltzmann method (arXiv:1709.09073).  Interface: include/rlbm.h.
//
// One thread per cell.  The fused step kernel does, per cell:
//   pull streaming with bilinear interpolation                      (Sec. 2.4)
//   moments N^mu, T^{mu nu} through per-direction shell sums
//   Landau frame T^a_b U^b = eps U^a: Newton on the fixed-point form
//     u_i (T^00 - T^0j u_j) = T^i0 - T^ij u_j, started from the exact
//     equilibrium relation |u| = 4M/(3 + sqrt(9 - 8M^2)), M = |T^0i|/T^00  (Eq. eigen-eq)
//   n = gamma (N^0 - u.N)                                            (Eq. density-eq)
//   (n, eps) -> (theta, z): MJ closed form; FD/BE safeguarded Newton on
//     h(mu) = g_2^3/g_3^2 = 2n^3/(pi eps^2), mu = ln z          (Eqs. theta-eq, n-eps-eq)
//   tau: constant or tau_a/theta + tau_b                             (Sec. 3.2)
//   fifth-order equilibrium in separable harmonic form               (Eq. expansion-eq, App. A)
//   Anderson-Witting relaxation f* = f + gamma(1 - v.u)/tau (f^eq - f) (Sec. 2.1)
// and stores f* (SoA, coalesced in x).  Landau, inversion and the radial step of
// the equilibrium run in FP64 in every precision mode; populations, streaming,
// shell sums, angular synthesis and relaxation run in the storage precision.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <new>
#include <type_traits>
#include <vector>

#include "rlbm.h"
#include "rlbm_mlp.h"
#include "rlbm_tables.h"

#ifndef RLBM_STEP_WAVES_PER_SIMD
#define RLBM_STEP_WAVES_PER_SIMD 3   // occupancy target of the FP32 step kernel (register budget 512/3)
#endif
#ifndef RLBM_STEP_WAVES_FDBE
#define RLBM_STEP_WAVES_FDBE 3       // FD/BE fit 3 waves without spills with the shortened FP32-path sums
#endif
#ifndef RLBM_FP32_STAGED
#define RLBM_FP32_STAGED 1      // FP32 populations take the staged pull too (tiles that fit)
#endif
#ifndef RLBM_BATCH_WAVES_MJ
#define RLBM_BATCH_WAVES_MJ 2   // measured: 3 waves spill in the batch kernel and run ~10% slower
#endif
#ifndef RLBM_BATCH_WAVES_FDBE
#define RLBM_BATCH_WAVES_FDBE 2      // the batch kernel spills at 3
#endif
// FP64 populations need about twice the registers: no occupancy target (no spills)
// (the forced / non-equilibrium-wall variant carries a second equilibrium state: 2 waves)
#define RLBM_STEP_BOUNDS(ST, R, FORCED) \
    __launch_bounds__(256, sizeof(R) == 8 ? 1 : (FORCED) ? 2 \
                           : ((ST) == RLBM_MJ ? RLBM_STEP_WAVES_PER_SIMD : RLBM_STEP_WAVES_FDBE))
#define RLBM_BATCH_BOUNDS(ST, R) \
    __launch_bounds__(256, sizeof(R) == 8 ? 1 : ((ST) == RLBM_MJ ? RLBM_BATCH_WAVES_MJ : RLBM_BATCH_WAVES_FDBE))

namespace {

using namespace rlbm_tab;

constexpr double S3H = 0.8660254037844386;   // sqrt(3)/2 rounded to FP64
constexpr double PI_D = 3.141592653589793;

// unit vectors of the 12 directions n*pi/6, exact values
__host__ __device__ constexpr double cdir(int n) {
    return n == 0 ? 1.0 : n == 1 ? S3H : n == 2 ? 0.5 : n == 3 ? 0.0 : n == 4 ? -0.5 : n == 5 ? -S3H
         : n == 6 ? -1.0 : n == 7 ? -S3H : n == 8 ? -0.5 : n == 9 ? 0.0 : n == 10 ? 0.5 : S3H;
}
__host__ __device__ constexpr double sdir(int n) { return cdir((n + 9) % 12); }
// cos(j*phi_n), sin(j*phi_n) from the exact table (j*n taken mod 12)
__host__ __device__ constexpr double cjn(int j, int n) { return cdir((j * n) % 12); }
__host__ __device__ constexpr double sjn(int j, int n) { return sdir((j * n) % 12); }
// x c + acc for a factor c that is a compile-time constant once loops are unrolled (a
// direction cosine, a table entry).  The compiler keeps x * 0 (x may be NaN or
// infinite), so zero and unit factors are spelled out: they cost nothing or one add.
template <typename T>
__device__ __forceinline__ T fma_c(T x, double c, T acc) {
    if (c == 0.0) return acc;
    if (c == 1.0) return acc + x;
    if (c == -1.0) return acc - x;
    return x * (T)c + acc;
}
// index of the pair (j, k), j-major, k = j..5
__host__ __device__ constexpr int pair_index(int j, int k) { return j * 6 - (j * (j - 1)) / 2 + (k - j); }

struct KArgs {
    const void *fin;
    void *fout;
    int nx, ny;
    long long plane;             // nx*ny
    int tx, ty, ntx, ntiles, per_xcd;
    int nty, sw;                 // tile rows; tile columns per strip (tile order below)
    int bc_xlo, bc_xhi, bc_ylo, bc_yhi;
    int tau_mode;
    double tau, tau_a, tau_b;
    double th_wall_lo, th_wall_hi;
    double force_x, force_y;     // momentum-update acceleration (forced kernels)
    double wall_n, wall_theta;   // state imposed on RLBM_BC_WALL_NEQ rows
    int guess;
    const float *mlp;
    unsigned *status;
    unsigned long long *stats;   // [0] Newton iterations, [1] solves (NULL: not collected)
    float *o_mlx, *o_mlt;        // inversion training pairs (moments kernel)
    // init inputs
    const double *i_n, *i_z, *i_theta, *i_ux, *i_uy;
    int given_z;
    // field outputs
    double *o_n, *o_eps, *o_theta, *o_z, *o_ux, *o_uy, *o_qx, *o_qy;
    double *o_pi[4];             // non-equilibrium tensors pi^{x..x} of rank 2..5
    double *o_mom[9];            // raw moments N^0, N^x, N^y, T^00, T^0x, T^0y, T^xx, T^xy, T^yy
};

// ---------------------------------------------------------------- tile mapping
// Tiles are numbered strip by strip: a strip is sw tile columns wide (about
// RLBM_STRIP_CELLS cells for staged-pull launches; the whole grid width, i.e. plain
// row order, for direct-pull ones), swept row by row from top to bottom.  The hardware
// hands consecutive workgroups to the 8 XCDs in turn, so workgroup b runs tile
// (b % 8) * per_xcd + b / 8: each XCD sweeps its own contiguous run of strip rows.  The
// tile above a tile ran sw tiles earlier on the same XCD, so the halo rows they share
// are still in that XCD's L2 even on grids too wide for a whole tile row to stay there.
#ifndef RLBM_STRIP_CELLS
#define RLBM_STRIP_CELLS 1024
#endif

__device__ __forceinline__ void tile_xy(const KArgs &a, int t, int &txi, int &tyi) {
    const int per_strip = a.sw * a.nty;
    const int s = t / per_strip;
    const int r = t - s * per_strip;
    const int w = min(a.sw, a.ntx - s * a.sw);
    tyi = r / w;
    txi = s * a.sw + (r - tyi * w);
}

__device__ __forceinline__ bool cell_of(const KArgs &a, int &x, int &y) {
    const int b = blockIdx.x;
    const int t = (b & 7) * a.per_xcd + (b >> 3);
    if (t >= a.ntiles) return false;
    int txi, tyi;
    tile_xy(a, t, txi, tyi);
    const int lx = threadIdx.x % a.tx;
    const int ly = threadIdx.x / a.tx;
    x = txi * a.tx + lx;
    y = tyi * a.ty + ly;
    return x < a.nx && y < a.ny;
}

__device__ __forceinline__ void neighbours(const KArgs &a, int x, int y, int &xl, int &xr, int &yd, int &yu) {
    xl = x - 1;
    xr = x + 1;
    yd = y - 1;
    yu = y + 1;
    if (xl < 0) xl = (a.bc_xlo == RLBM_BC_PERIODIC) ? a.nx - 1 : 0;
    if (xr >= a.nx) xr = (a.bc_xhi == RLBM_BC_PERIODIC) ? 0 : a.nx - 1;
    if (yd < 0) yd = (a.bc_ylo == RLBM_BC_PERIODIC) ? a.ny - 1 : 0;
    if (yu >= a.ny) yu = (a.bc_yhi == RLBM_BC_PERIODIC) ? 0 : a.ny - 1;
}

// ---------------------------------------------------------------- buffer access
// Populations are read and written with raw buffer instructions: one descriptor per
// direction covers its 6 shell planes, the shell's plane offset is a scalar and
// the cell's offset a 32-bit per-lane value, so no 64-bit per-lane address is formed.
// The host keeps 6 * nx * ny * sizeof(element) below 2^32.
using rsrc_t = __amdgpu_buffer_rsrc_t;

// Cache policy bits of the population loads and stores (bit 1 = non-temporal).  The
// populations a step writes are read only by the next launch, after the whole grid
// has been written, so the stores stream past the caches.
#ifndef RLBM_POP_LOAD_POLICY
#define RLBM_POP_LOAD_POLICY 0
#endif
#ifndef RLBM_POP_STORE_POLICY
#define RLBM_POP_STORE_POLICY 2
#endif
constexpr int LOAD_POLICY = RLBM_POP_LOAD_POLICY;
constexpr int STORE_POLICY = RLBM_POP_STORE_POLICY;

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename S>
__device__ __forceinline__ S bload(rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float bload<float>(rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, LOAD_POLICY));
}
template <>
__device__ __forceinline__ double bload<double>(rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, LOAD_POLICY));
}

template <typename S>
__device__ __forceinline__ void bstore(S v, rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ void bstore<float>(float v, rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, STORE_POLICY);
}
template <>
__device__ __forceinline__ void bstore<double>(double v, rsrc_t r, unsigned voff, unsigned soff) {
    typedef unsigned v2u __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, voff, soff, STORE_POLICY);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// Vector elements are copied to scalars before a bit cast: clang takes
// __builtin_bit_cast of an ext_vector element as a cast of element 0.
__device__ __forceinline__ float u32_as_float(unsigned u) { return __builtin_bit_cast(float, u); }
__device__ __forceinline__ unsigned float_as_u32(float v) { return __builtin_bit_cast(unsigned, v); }
__device__ __forceinline__ double u32_as_double(unsigned lo, unsigned hi) {
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

// A direction block of FP32/FP64 populations holds, per cell, the six shells as
// 16-byte records: FP32 shells 0..3 (record at cell*16) then shells 4..5 (8 bytes at
// 16*P + cell*8); FP64 shells 2j, 2j+1 at 16*j*P + cell*16, j = 0, 1, 2 (P = nx*ny).
template <typename S>
struct Rec;

template <>
struct Rec<float> {
    static __device__ __forceinline__ void load(rsrc_t r, unsigned cell, unsigned P, float (&v)[6]) {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, cell * 16u, 0u, LOAD_POLICY);
        const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(r, cell * 8u, 16u * P, LOAD_POLICY);
        unsigned e0 = a[0], e1 = a[1], e2 = a[2], e3 = a[3], e4 = b[0], e5 = b[1];
        v[0] = u32_as_float(e0);
        v[1] = u32_as_float(e1);
        v[2] = u32_as_float(e2);
        v[3] = u32_as_float(e3);
        v[4] = u32_as_float(e4);
        v[5] = u32_as_float(e5);
    }
    static __device__ __forceinline__ void store(rsrc_t r, unsigned cell, unsigned P, const float (&v)[6]) {
        const u32x4 a = {float_as_u32(v[0]), float_as_u32(v[1]), float_as_u32(v[2]), float_as_u32(v[3])};
        const u32x2 b = {float_as_u32(v[4]), float_as_u32(v[5])};
        __builtin_amdgcn_raw_buffer_store_b128(a, r, cell * 16u, 0u, STORE_POLICY);
        __builtin_amdgcn_raw_buffer_store_b64(b, r, cell * 8u, 16u * P, STORE_POLICY);
    }
};

template <>
struct Rec<double> {
    static __device__ __forceinline__ void load(rsrc_t r, unsigned cell, unsigned P, double (&v)[6]) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, cell * 16u, 16u * (unsigned)j * P, LOAD_POLICY);
            unsigned e0 = a[0], e1 = a[1], e2 = a[2], e3 = a[3];
            v[2 * j] = u32_as_double(e0, e1);
            v[2 * j + 1] = u32_as_double(e2, e3);
        }
    }
    static __device__ __forceinline__ void store(rsrc_t r, unsigned cell, unsigned P, const double (&v)[6]) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const unsigned long long x = __builtin_bit_cast(unsigned long long, v[2 * j]);
            const unsigned long long y = __builtin_bit_cast(unsigned long long, v[2 * j + 1]);
            const u32x4 a = {(unsigned)x, (unsigned)(x >> 32), (unsigned)y, (unsigned)(y >> 32)};
            __builtin_amdgcn_raw_buffer_store_b128(a, r, cell * 16u, 16u * (unsigned)j * P, STORE_POLICY);
        }
    }
};

// ---------------------------------------------------------------- streaming
// Pull of all 72 populations of cell (x, y).  Axis directions shift by one cell;
// the others interpolate bilinearly from (x, y), (xb, y), (x, yb), (xb, yb) with
// xb = x - sgn(v_x), yb = y - sgn(v_y) and weights |vx||vy|, (1-|vx|)|vy|,
// |vx|(1-|vy|), (1-|vx|)(1-|vy|); with |v| components in {1/2, sqrt3/2} these
// pair up into two weights wA = sqrt3/4 and wB = (1 - sqrt3/2)/2.
template <typename S, typename R>
__device__ __forceinline__ void pull(const S *__restrict__ fin, long long plane, int nx, int x, int y, int xl,
                                     int xr, int yd, int yu, R (&f)[72]) {
    const unsigned oc = (unsigned)(y * nx), od = (unsigned)(yd * nx), ou = (unsigned)(yu * nx);
    const unsigned P = (unsigned)plane;
    const R wA = (R)(S3H * 0.5);
    const R wB = (R)((1.0 - S3H) * 0.5);
#pragma unroll
    for (int n = 0; n < 12; ++n) {
        const rsrc_t r = make_rsrc(fin + (long long)(6 * n) * plane, 6u * P * (unsigned)sizeof(S));
        const unsigned xb = cdir(n) > 0.1 ? xl : xr;     // source column x - sgn(v_x)
        const unsigned rb = sdir(n) > 0.1 ? od : ou;     // source row    y - sgn(v_y)
        if (n % 3 == 0) {
            const unsigned src = n == 0 ? oc + xl : n == 3 ? od + x : n == 6 ? oc + xr : ou + x;
            S v[6];
            Rec<S>::load(r, src, P, v);
#pragma unroll
            for (int s = 0; s < 6; ++s) f[6 * n + s] = (R)v[s];
        } else {
            S bb[6], bx[6], cb[6], cx[6];
            Rec<S>::load(r, rb + xb, P, bb);
            Rec<S>::load(r, rb + x, P, bx);
            Rec<S>::load(r, oc + xb, P, cb);
            Rec<S>::load(r, oc + x, P, cx);
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                if (n == 1 || n == 5 || n == 7 || n == 11)   // |v_x| = sqrt3/2, |v_y| = 1/2
                    f[6 * n + s] = wA * ((R)bb[s] + (R)cb[s]) + wB * ((R)bx[s] + (R)cx[s]);
                else                                          // |v_x| = 1/2, |v_y| = sqrt3/2
                    f[6 * n + s] = wA * ((R)bb[s] + (R)bx[s]) + wB * ((R)cb[s] + (R)cx[s]);
            }
        }
    }
}

// ---------------------------------------------------------------- moments
struct Mom {
    double N0, Nx, Ny, T00, T01, T02, T11, T12, T22;
};

// GU: f holds f_i / w_k (the 16-bit deviation path works in those units); the
// weights fold into the constants.
template <int ST, typename R, bool GU = false>
__device__ __forceinline__ Mom moments(const R (&f)[72]) {
    Mom m{-0.0, -0.0, -0.0, -0.0, -0.0, -0.0, -0.0, -0.0, -0.0};   // -0 + x folds to x
    // per direction: a = sum_k f p_k, b = sum_k f p_k^2; opposite directions n and
    // n + 6 share |cos|, |sin|, so their sums (even moments) and differences (odd
    // moments) enter once
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        R a[2] = {0, 0}, b[2] = {0, 0};
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const double w = GU ? W_SHELL[ST][s] : 1.0;
                const R v = f[6 * (n + 6 * h) + s];
                a[h] += v * (R)(P_SHELL[ST][s] * w);
                b[h] += v * (R)(P_SHELL[ST][s] * P_SHELL[ST][s] * w);
            }
        const double SA = (double)a[0] + (double)a[1], DA = (double)a[0] - (double)a[1];
        const double SB = (double)b[0] + (double)b[1], DB = (double)b[0] - (double)b[1];
        const double c = cdir(n), sn = sdir(n);
        m.N0 += SA;
        m.Nx = fma_c(DA, c, m.Nx);
        m.Ny = fma_c(DA, sn, m.Ny);
        m.T00 += SB;
        m.T01 = fma_c(DB, c, m.T01);
        m.T02 = fma_c(DB, sn, m.T02);
        m.T11 = fma_c(SB, c * c, m.T11);
        m.T12 = fma_c(SB, c * sn, m.T12);
        m.T22 = fma_c(SB, sn * sn, m.T22);
    }
    return m;
}

// 1/x from the hardware reciprocal estimate refined by two Newton-Raphson steps
// (each squares the relative error): a short dependency chain without the scaling
// steps of a correctly rounded division, for a positive normal x.
__device__ __forceinline__ double rcp_refined(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
}

// a / b and 1/sqrt(x) for the FP32 and 16-bit population paths (LOOSE): the hardware
// estimates refined by two Newton-Raphson steps, a few ulp of FP64 and far below those
// populations' own rounding, in about half the instructions of the correctly rounded
// forms, which FP64 populations keep.
template <bool LOOSE>
__device__ __forceinline__ double qdiv(double a, double b) {
    if constexpr (LOOSE) return a * rcp_refined(b);
    else return a / b;
}
template <bool LOOSE>
__device__ __forceinline__ double inv_sqrt(double x) {
    if constexpr (LOOSE) {
        double r = __builtin_amdgcn_rsq(x);
        r = r * fma(-0.5 * x * r, r, 1.5);
        return r * fma(-0.5 * x * r, r, 1.5);
    } else {
        return 1.0 / sqrt(x);
    }
}

// ---------------------------------------------------------------- Landau frame
template <bool LOOSE>
__device__ __forceinline__ void landau(const Mom &m, double &ux, double &uy, double &eps, unsigned &flags) {
    const double inv = qdiv<LOOSE>(1.0, m.T00);
    const double mx = m.T01 * inv, my = m.T02 * inv;
    const double M2 = mx * mx + my * my;
    const double sc = qdiv<LOOSE>(4.0, 3.0 + sqrt(fmax(9.0 - 8.0 * M2, 0.0)));
    ux = sc * mx;
    uy = sc * my;
    bool conv = false;
    for (int it = 0; it < 40; ++it) {
        const double e = m.T00 - m.T01 * ux - m.T02 * uy;
        const double Fx = m.T01 - m.T11 * ux - m.T12 * uy - e * ux;
        const double Fy = m.T02 - m.T12 * ux - m.T22 * uy - e * uy;
        const double a = -m.T11 + m.T01 * ux - e, b = -m.T12 + m.T02 * ux;
        const double c = -m.T12 + m.T01 * uy, d = -m.T22 + m.T02 * uy - e;
        const double idet = qdiv<LOOSE>(1.0, a * d - b * c);
        const double dx = (d * Fx - b * Fy) * idet, dy = (a * Fy - c * Fx) * idet;
        ux -= dx;
        uy -= dy;
        if (fabs(dx) + fabs(dy) <= 1e-12) {
            conv = true;
            break;
        }
    }
    if (!conv) flags |= RLBM_FLAG_NOCONV;
    eps = m.T00 - m.T01 * ux - m.T02 * uy;
}

// ---------------------------------------------------------------- g_nu(z)
// g[m] = g_m(e^mu) for m = MLO..MHI (1 <= MLO <= MHI <= 6).  Tables: Taylor in mu
// about tabulated centres using d g_m / d mu = g_{m-1}; BE near mu = 0: series of
// Li_m about mu = 0; far tails: the defining series.
template <int MLO, int MHI>
__device__ __forceinline__ void g_tail(double mu, double xi, double (&g)[7]) {
    const double e = exp(mu);
    double ek[5];
    ek[1] = e;
    ek[2] = e * e;
    ek[3] = ek[2] * e;
    ek[4] = ek[2] * ek[2];
#pragma unroll
    for (int m = MLO; m <= MHI; ++m) {
        double s = 0, sg = 1;
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            s += sg * ek[k] / pow((double)k, (double)m);
            sg *= -xi;
        }
        g[m] = s;
    }
}

// One table centre's coefficients held in registers: columns 0 .. K+4 of its row, the
// ones orders 1..6 read.  The Newton iterates of one cell and its final evaluation
// usually fall on the same centre; with REUSE they then take the row from registers
// instead of reading it again, a dependent load the cell would otherwise wait for
// each time.  (Fermi-Dirac with FP32 or 16-bit populations only: the Bose-Einstein
// kernels have no registers to spare for the row, and the FP64 step, one wave per
// SIMD, ran no faster with it.)
template <int K>
struct GRow {
    static_assert(K + 5 <= NG, "orders 1..6 with K Taylor terms read columns 0 .. K+4 of a row");
    int i;   // centre index held; -1: none
    double c[K + 5];
};

template <bool LOOSE>
using GRowT = GRow<LOOSE ? NT_LOOSE : NT>;

template <bool REUSE, int K>
__device__ __forceinline__ void g_row_fetch(const double (*tab)[NG], int i, GRow<K> &row) {
    if (REUSE && i == row.i) return;
    const double *src = tab[i];
#pragma unroll
    for (int j = 0; j < K + 5; ++j) row.c[j] = src[j];
    row.i = i;
}

template <int MLO, int MHI, int K>
__device__ __forceinline__ void g_table(const GRow<K> &row, double d, double (&g)[7]) {
    double t[K];
    t[0] = 1.0;
#pragma unroll
    for (int k = 1; k < K; ++k) t[k] = t[k - 1] * (d * (1.0 / k));   // d / k off the dependency chain
#pragma unroll
    for (int m = MLO; m <= MHI; ++m) {
        double s = 0;
#pragma unroll
        for (int k = K - 1; k >= 0; --k) s += row.c[6 - m + k] * t[k];
        g[m] = s;
    }
}

// LOOSE (FP32 / 16-bit populations): shortened sums, tail below 1e-11 relative
// (bounded when the tables are generated).
template <int ST, int MLO, int MHI, bool LOOSE = false>
__device__ __forceinline__ void gvals(double mu, double (&g)[7], unsigned &flags, GRowT<LOOSE> &row) {
    constexpr int K = LOOSE ? NT_LOOSE : NT;
    constexpr int NZ = LOOSE ? BE_NZ_LOOSE : BE_NZ;
    // table indices below are formed from mu: keep it finite and inside the tables' reach
    if (!(mu > -40.0)) {
        if (mu != mu) flags |= RLBM_FLAG_NONPOSITIVE;   // NaN
        mu = -40.0;
    }
    if constexpr (ST == RLBM_BE) {
        if (!(mu <= LOG_ZC_BE)) {
            flags |= RLBM_FLAG_CONDENSED;
            mu = LOG_ZC_BE;
        }
    }
    if constexpr (ST == RLBM_FD) {
        if (mu < FD_MU_MIN - 0.5 * FD_DMU) {
            g_tail<MLO, MHI>(mu, 1.0, g);
            return;
        }
        int i = (int)rint((mu - FD_MU_MIN) * (1.0 / FD_DMU));
        if (i > FD_NC - 1) {
            i = FD_NC - 1;
            if (mu > FD_MU_MIN + (FD_NC - 0.5) * FD_DMU) flags |= RLBM_FLAG_RANGE;
        }
        g_row_fetch<LOOSE>(FD_TAB, i, row);
        g_table<MLO, MHI, K>(row, mu - (FD_MU_MIN + i * FD_DMU), g);
    } else {
        if (mu < BE_MU_MIN - 0.5 * BE_DMU) {
            g_tail<MLO, MHI>(mu, -1.0, g);
            return;
        }
        if (mu < BE_MU_SPLIT - 0.5 * BE_DMU) {
            int i = (int)rint((mu - BE_MU_MIN) * (1.0 / BE_DMU));
            if (i > BE_NC - 1) i = BE_NC - 1;
            g_row_fetch<false>(BE_TAB, i, row);
            g_table<MLO, MHI, K>(row, mu - (BE_MU_MIN + i * BE_DMU), g);
            return;
        }
        // Li_m(e^mu) = mu^{m-1}/(m-1)! (H_{m-1} - ln(-mu)) + sum_{k != m-1} zeta(m-k) mu^k / k!
        const double L = log(-mu);
        double t[NZ];
        t[0] = 1.0;
#pragma unroll
        for (int k = 1; k < NZ; ++k) t[k] = t[k - 1] * (mu * (1.0 / k));
#pragma unroll
        for (int m = MLO; m <= MHI; ++m) {
            double s = 0;
#pragma unroll
            for (int k = NZ - 1; k >= 0; --k) s += BE_ZETA[6 - m + k] * t[k];   // zeta(1) stored as 0
            g[m] = s + t[m - 1] * (HARMONIC[m - 1] - L);
        }
    }
}

template <int ST, int MLO, int MHI, bool LOOSE = false>
__device__ __forceinline__ void gvals(double mu, double (&g)[7], unsigned &flags) {
    GRowT<LOOSE> row;
    row.i = -1;
    gvals<ST, MLO, MHI, LOOSE>(mu, g, flags, row);
}

// Newton on mu = ln z leaves an error C dmu^2 after a step dmu, with C = f''/(2 f')
// at most 0.5 for FD and about 0.5/|mu| for BE near mu = 0, so a step below this
// tolerance is applied and ends the solve (no confirming evaluation).  FP64
// populations: 1e-8 (error <= 5e-17); FP32/16-bit populations: 1e-5 (error <= 5e-11,
// far below the populations' own rounding).
template <int ST, bool LOOSE>
__device__ __forceinline__ double newton_tol(double mu) {
    constexpr double t = LOOSE ? 1e-5 : 1e-8;
    return ST == RLBM_BE ? t * fmin(1.0, fabs(mu)) : t;
}

// Solve h(mu) = g_2^3/g_3^2 = r for mu = ln z (FD, BE), safeguarded Newton.
// row: the table row of the last evaluation, for the caller's final evaluation at the root.
template <int ST, bool LOOSE>
__device__ __forceinline__ double invert_h(double r, double mu, unsigned &flags, int &iters, GRowT<LOOSE> &row) {
    double lo = -40.0, hi = (ST == RLBM_BE) ? LOG_ZC_BE : FD_MU_MIN + (FD_NC - 0.5) * FD_DMU;
    if (ST == RLBM_BE && r >= H_ZC_BE) {
        flags |= RLBM_FLAG_CONDENSED;
        return LOG_ZC_BE;
    }
    if (!(mu > lo && mu < hi)) mu = 0.5 * (lo + hi);
    bool conv = false;
    iters = 0;
    for (int it = 0; it < 80; ++it) {
        ++iters;
        double g[7];
        gvals<ST, 1, 3, LOOSE>(mu, g, flags, row);
        double h, dmu;
        if constexpr (LOOSE) {
            // one FP64 reciprocal (1-2 ulp); the step itself only needs single precision: its
            // relative error (~1e-7) adds at most 1e-7 |dmu| to what the step leaves
            const double a = rcp_refined(g[2] * g[3]);
            const double q = g[2] * g[2] * a;
            h = g[2] * q * q;
            const double D = h * (3.0 * g[1] * g[3] * a - 2.0 * q);
            dmu = (double)__fdividef((float)(h - r), (float)D);
        } else {
            const double q = g[2] / g[3];
            h = g[2] * q * q;
            dmu = (h - r) / (h * (3.0 * g[1] / g[2] - 2.0 * q));   // dh/dmu = h (3 g1/g2 - 2 g2/g3)
        }
        const double F = h - r;
        if (F == 0.0 || fabs(dmu) <= newton_tol<ST, LOOSE>(mu)) {   // the error left after this step is O(dmu^2)
            mu -= (F == 0.0) ? 0.0 : dmu;
            conv = true;
            break;
        }
        if (F > 0) hi = mu; else lo = mu;
        double mn = mu - dmu;
        if (!(mn > lo && mn < hi)) mn = 0.5 * (lo + hi);   // safeguard: keep inside the bracket
        mu = mn;
        if (hi - lo <= 4e-16 * fmax(1.0, fabs(mu))) {
            conv = true;
            break;
        }
    }
    if (!conv) flags |= RLBM_FLAG_NOCONV;
    return mu;
}

// Solve g_2(e^mu) = target for mu (FD, BE): fugacity from (n, theta).
template <int ST, bool LOOSE = false>
__device__ __forceinline__ double invert_g2(double target, unsigned &flags) {
    double lo = -40.0, hi = (ST == RLBM_BE) ? LOG_ZC_BE : FD_MU_MIN + (FD_NC - 0.5) * FD_DMU;
    double mu = (ST == RLBM_BE) ? -0.6931471805599453 : 0.0;
    if (ST == RLBM_BE) {
        if (!(target < G2_ZC_BE)) {   // density above the condensation bound at this theta
            flags |= RLBM_FLAG_CONDENSED;
            return LOG_ZC_BE;
        }
    }
    bool conv = false;
    for (int it = 0; it < 80; ++it) {
        double g[7];
        gvals<ST, 1, 2>(mu, g, flags);
        const double F = g[2] - target;
        const double dmu = F / g[1];            // d g_2 / d mu = g_1
        if (F == 0.0 || fabs(dmu) <= newton_tol<ST, LOOSE>(mu)) {
            mu -= (F == 0.0) ? 0.0 : dmu;
            conv = true;
            break;
        }
        if (F > 0) hi = mu; else lo = mu;
        double mn = mu - dmu;
        if (!(mn > lo && mn < hi)) mn = 0.5 * (lo + hi);
        mu = mn;
        if (hi - lo <= 4e-16 * fmax(1.0, fabs(mu))) {
            conv = true;
            break;
        }
    }
    if (!conv) flags |= RLBM_FLAG_NOCONV;
    return mu;
}

// Macroscopic state of a cell: theta, z (or mu), g_1..g_6, u, gamma, n, eps.
struct Macro {
    double n, eps, theta, z, ux, uy, ga;
    double g[7];
};

template <int ST, bool LOOSE>
__device__ __forceinline__ void state_from_moments(const Mom &m, Macro &M, unsigned &flags, const KArgs &a,
                                                   int &iters, double *L_out = nullptr) {
    landau<LOOSE>(m, M.ux, M.uy, M.eps, flags);
    const double u2 = M.ux * M.ux + M.uy * M.uy;
    if (!(u2 < 1.0)) {
        flags |= RLBM_FLAG_SUPERLUMINAL;
        M.ux = M.uy = 0.0;
    }
    M.ga = inv_sqrt<LOOSE>(1.0 - (M.ux * M.ux + M.uy * M.uy));
    M.n = M.ga * (m.N0 - M.ux * m.Nx - M.uy * m.Ny);
    // a NaN or infinite population makes N^0 and T^00 (every p^0 > 0) and so n or eps
    // non-finite; comparisons with NaN are false
    if (!(M.n > 0.0 && M.n < INFINITY) || !(M.eps > 0.0 && M.eps < INFINITY)) {
        flags |= (fabs(M.n) < INFINITY && fabs(M.eps) < INFINITY) ? RLBM_FLAG_NONPOSITIVE : RLBM_FLAG_NONFINITE;
        M.n = (M.n > 0.0 && M.n < INFINITY) ? M.n : 1.0;
        M.eps = (M.eps > 0.0 && M.eps < INFINITY) ? M.eps : 1.0;
    }
    const double r = qdiv<LOOSE>(2.0 * M.n * M.n * M.n, PI_D * M.eps * M.eps);
    if (L_out) *L_out = log(r);
    iters = 0;
    if constexpr (ST == RLBM_MJ) {
        M.theta = qdiv<LOOSE>(M.eps, 2.0 * M.n);
        M.z = r;
#pragma unroll
        for (int k = 1; k <= 6; ++k) M.g[k] = r;
    } else {
        // starting point of the Newton solve: the trained network, or the fixed guess
        double mu0 = (ST == RLBM_BE) ? -0.6931471805599453 : 0.0;
        if (a.guess == RLBM_GUESS_MLP) mu0 = (double)rlbm_mlp::eval(a.mlp, logf((float)r));
        GRowT<LOOSE> row;
        row.i = -1;
        const double mu = invert_h<ST, LOOSE>(r, mu0, flags, iters, row);
        gvals<ST, 1, 6, LOOSE>(mu, M.g, flags, row);
        M.z = exp(mu);
        if constexpr (LOOSE) M.theta = qdiv<LOOSE>(0.5 * M.g[2] * M.eps, M.g[3] * M.n);
        else M.theta = 0.5 * (M.g[2] / M.g[3]) * (M.eps / M.n);
    }
}

// Fugacity and g's from (n, theta) (init, wall cells).
template <int ST>
__device__ __forceinline__ void state_from_n_theta(double n, double theta, Macro &M, unsigned &flags) {
    const double target = n / (2.0 * PI_D * theta * theta);
    M.theta = theta;
    if constexpr (ST == RLBM_MJ) {
        M.z = target;
#pragma unroll
        for (int k = 1; k <= 6; ++k) M.g[k] = target;
    } else {
        const double mu = invert_g2<ST>(target, flags);
        gvals<ST, 1, 6>(mu, M.g, flags);
        M.z = exp(mu);
    }
}

template <int ST>
__device__ __forceinline__ void state_from_z_theta(double z, double theta, Macro &M, unsigned &flags) {
    M.theta = theta;
    M.z = z;
    if constexpr (ST == RLBM_MJ) {
#pragma unroll
        for (int k = 1; k <= 6; ++k) M.g[k] = z;
    } else {
        gvals<ST, 1, 6>(log(z), M.g, flags);
    }
}

// ---------------------------------------------------------------- equilibrium + relaxation
// f^eq_{s,n} = sum_j r_j(s) A_{j,n};  r_j(s) = sum_k E^(j)_{s,k} G_k P_kj(u^2) (FP64),
// A_{j,n} = Re[(u_x + i u_y)^j e^{-i j phi_n}], G_k = k! g_{k+1} theta^{k+1} gamma^k.
// MODE: EQ_SET f <- f^eq; EQ_COLLIDE f <- f + omega_n (f^eq - f) with
// omega_n = gamma (1 - v_n.u) / tau; EQ_NEQ f <- (1 - omega_n)(f - f^eq), the part
// f* - f^eq a collision leaves; EQ_ADD f <- f + f^eq.
// Projector table of expansion order N (5 for every statistic; 2..4 for Maxwell-Juttner).
template <int ST, int N>
__device__ __forceinline__ constexpr double emat(int pair, int shell) {
    if constexpr (N == 5) return EMAT[ST][pair][shell];
    else return EMAT_LO[N - 2][pair][shell];
}

// PKJ[pi][0] + PKJ[pi][1] u^2 + PKJ[pi][2] u^4, with the zero coefficients skipped
__device__ __forceinline__ double poly_u2(int pi, double u2) {
    if (PKJ[pi][2] != 0.0) return (u2 * PKJ[pi][2] + PKJ[pi][1]) * u2 + PKJ[pi][0];
    return fma_c(u2, PKJ[pi][1], PKJ[pi][0]);
}

enum { EQ_SET = 0, EQ_COLLIDE = 1, EQ_NEQ = 2, EQ_ADD = 3 };

// GU: f holds f_i / w_k and receives f^eq_i / w_k (the 1/w_k folds into the projector).
template <int ST, int MODE, typename R, int N = 5, bool GU = false>
__device__ __forceinline__ void equilibrium_relax(const Macro &M, double tau, R (&f)[72]) {
    constexpr bool COLLIDE = MODE == EQ_COLLIDE || MODE == EQ_NEQ;
    static_assert(N == 5 || (ST == RLBM_MJ && N >= 2 && N <= 4), "lower orders are tabulated for MJ");
    const double u2 = M.ux * M.ux + M.uy * M.uy;
    double G[6];
    {
        double th = M.theta, gk = 1.0, fact = 1.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            if (k > 0) fact *= (double)k;
            G[k] = fact * M.g[k + 1] * th * gk;
            th *= M.theta;
            gk *= M.ga;
        }
    }
    double h[21];
#pragma unroll
    for (int j = 0; j <= N; ++j)
#pragma unroll
        for (int k = j; k <= N; ++k) {
            const int pi = pair_index(j, k);
            h[pi] = G[k] * poly_u2(pi, u2);
        }
    // harmonics (u_x + i u_y)^j
    R C[6], S[6];
    {
        double c = 1.0, s = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            C[j] = (R)c;
            S[j] = (R)s;
            const double cn = c * M.ux - s * M.uy;
            s = c * M.uy + s * M.ux;
            c = cn;
        }
    }
    // A_{j,n} for n = 0..5 (n + 6 follows from A_{j,n+6} = (-1)^j A_{j,n})
    R A[6][6];
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        A[0][n] = (R)1;
#pragma unroll
        for (int j = 1; j < 6; ++j) A[j][n] = fma_c(S[j], sjn(j, n), fma_c(C[j], cjn(j, n), (R)-0.0));
    }
    R om[12];
    if constexpr (COLLIDE) {
        const R gt = (R)qdiv<sizeof(R) == 4>(M.ga, tau);
        const R ux = (R)M.ux, uy = (R)M.uy;
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            const R vu = fma_c(uy, sdir(n), fma_c(ux, cdir(n), (R)-0.0));
            om[n] = gt - gt * vu;
            om[n + 6] = gt + gt * vu;
        }
    }
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        R r[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            double acc = 0.0;
            if (j <= N) {
#pragma unroll
                for (int k = j; k <= N; ++k)
                    acc += (emat<ST, N>(pair_index(j, k), s) * (GU ? 1.0 / W_SHELL[ST][s] : 1.0)) * h[pair_index(j, k)];
            }
            r[j] = (R)acc;
        }
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            const R ev = r[0] + r[2] * A[2][n] + r[4] * A[4][n];
            const R od = r[1] * A[1][n] + r[3] * A[3][n] + r[5] * A[5][n];
            const R fe0 = ev + od, fe1 = ev - od;
            R &a = f[6 * n + s];
            R &b = f[6 * (n + 6) + s];
            if constexpr (MODE == EQ_COLLIDE) {
                a = a + om[n] * (fe0 - a);
                b = b + om[n + 6] * (fe1 - b);
            } else if constexpr (MODE == EQ_NEQ) {
                a = (a - fe0) - om[n] * (a - fe0);
                b = (b - fe1) - om[n + 6] * (b - fe1);
            } else if constexpr (MODE == EQ_ADD) {
                a = a + fe0;
                b = b + fe1;
            } else {
                a = fe0;
                b = fe1;
            }
        }
    }
}

template <typename S, typename R>
__device__ __forceinline__ void store(S *__restrict__ fout, long long plane, int off, const R (&f)[72]) {
    const unsigned P = (unsigned)plane;
#pragma unroll
    for (int n = 0; n < 12; ++n) {
        const rsrc_t r = make_rsrc(fout + (long long)(6 * n) * plane, 6u * P * (unsigned)sizeof(S));
        S v[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) v[s] = (S)f[6 * n + s];
        Rec<S>::store(r, (unsigned)off, P, v);
    }
}

// ---------------------------------------------------------------- 16-bit deviation storage
// Per cell: e_i = (f_i / w_k - R_i) / s_k stored as a signed normalized 16-bit integer
// (SNORM16: q = round(32767 e), |e| <= 1), with the reference
// R_{k,n} = rho_k + p_k (alpha cos phi_n + beta sin phi_n) (the direction average of
// f/w per shell plus one p-weighted dipole, least squares) and a scale per shell,
// s_k >= max_n |f_{k,n} / w_k - R_{k,n}|, kept as IEEE half (rounded up).  Fixed point
// gives every value of a shell the same absolute step s_k / 32767, and the per-shell
// scale keeps the inner shells, which carry the density, energy and momentum, at
// their own small residuals.  Buffer layout (192 bytes per cell): 12 direction blocks
// of nx*ny cells x 6 SNORM16 (12 bytes per cell, shells k = 0..5 in order), then nx*ny
// cells x 48 bytes: floats rho_0..rho_5, alpha, beta, then halves s_0..s_5, then 4
// bytes of padding.  A direction's six deviations of a cell are one 12-byte load; a
// cell's side record three 16-byte loads.  The reference is linear in the side values,
// so a pull interpolates the side values with the bilinear weights and the
// deviations with the weights times the source's shell scales.
struct Dev16 {};

constexpr float SNORM16_STEP = 1.0f / 32767.0f;

// deviation k (0..5) of a cell's packed record, as the integer value in float
__device__ __forceinline__ float dev_value(const u32x3 &v, int k) {
    const unsigned u = v[k >> 1];
    return (k & 1) ? (float)((int)u >> 16) : (float)(short)(u & 0xffffu);
}

__device__ __forceinline__ float half_lo(unsigned u) { return (float)__builtin_bit_cast(f16x2, u).x; }
__device__ __forceinline__ float half_hi(unsigned u) { return (float)__builtin_bit_cast(f16x2, u).y; }

struct SideRef {
    float v[8];        // rho_0..rho_5, alpha, beta
    unsigned s[3];     // shell scales as half pairs (s_0, s_1), (s_2, s_3), (s_4, s_5)
    __device__ __forceinline__ float scale(int k) const { return (k & 1) ? half_hi(s[k >> 1]) : half_lo(s[k >> 1]); }
};

__device__ __forceinline__ void load_side(rsrc_t rs, unsigned cell, SideRef &o) {
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(rs, cell * 48u, 0u, LOAD_POLICY);
    const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(rs, cell * 48u, 16u, LOAD_POLICY);
    const u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(rs, cell * 48u, 32u, LOAD_POLICY);
    unsigned a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3], b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3];
    o.v[0] = u32_as_float(a0);
    o.v[1] = u32_as_float(a1);
    o.v[2] = u32_as_float(a2);
    o.v[3] = u32_as_float(a3);
    o.v[4] = u32_as_float(b0);
    o.v[5] = u32_as_float(b1);
    o.v[6] = u32_as_float(b2);
    o.v[7] = u32_as_float(b3);
    o.s[0] = c[0];
    o.s[1] = c[1];
    o.s[2] = c[2];
}

// The populations of direction N of one source cell, decoded to f/w: the reference
// rho_k + p_k (alpha cos phi_N + beta sin phi_N) plus the deviation times the shell's
// step s_k / 32767.  Every pull decodes a source value this way, so the tile-staged
// pull and the direct one give the same bits.
// A source cell's side record ready for decoding: rho_0..rho_5, alpha, beta and the
// code steps s_k / 32767.
struct DecodeRef {
    float v[8];
    float step[6];
};

__device__ __forceinline__ DecodeRef decode_ref(const SideRef &sr) {
    DecodeRef d;
#pragma unroll
    for (int k = 0; k < 8; ++k) d.v[k] = sr.v[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) d.step[k] = sr.scale(k) * SNORM16_STEP;
    return d;
}

template <int ST, int N>
__device__ __forceinline__ void dev_decode(const DecodeRef &d, const u32x3 &q, float (&g)[6]) {
    const float tn = fma_c(d.v[7], sdir(N), fma_c(d.v[6], cdir(N), -0.0f));
#pragma unroll
    for (int k = 0; k < 6; ++k) g[k] = fmaf(d.step[k], dev_value(q, k), fmaf((float)P_SHELL[ST][k], tn, d.v[k]));
}

// Bilinear interpolation of direction N's six shells from the decoded sources at
// (xb, yb), (x, yb), (xb, y), (x, y): the same weights and order as the direct FP32
// pull (used by the 16-bit direct pull and by the staged pull of both formats).
template <int N>
__device__ __forceinline__ void bilinear_direction(const float (&bb)[6], const float (&bx)[6],
                                                   const float (&cb)[6], const float (&cx)[6], float (&f)[72]) {
    const float wA = (float)(S3H * 0.5), wB = (float)((1.0 - S3H) * 0.5);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (N == 1 || N == 5 || N == 7 || N == 11)   // |v_x| = sqrt3/2, |v_y| = 1/2
            f[6 * N + k] = wA * (bb[k] + cb[k]) + wB * (bx[k] + cx[k]);
        else                                          // |v_x| = 1/2, |v_y| = sqrt3/2
            f[6 * N + k] = wA * (bb[k] + bx[k]) + wB * (cb[k] + cx[k]);
    }
}

template <int ST, int N>
__device__ __forceinline__ void dev_tap(const char *base, rsrc_t rs, long long plane, unsigned cell, float (&g)[6]) {
    const rsrc_t r = make_rsrc(base + (long long)N * plane * 12, 12u * (unsigned)plane);
    SideRef sr;
    load_side(rs, cell, sr);
    const u32x3 q = __builtin_amdgcn_raw_buffer_load_b96(r, cell * 12u, 0u, LOAD_POLICY);
    dev_decode<ST, N>(decode_ref(sr), q, g);
}

template <int ST, int N>
__device__ __forceinline__ void dev_pull_direction(const char *base, rsrc_t rs, long long plane, int nx, int x, int y,
                                                   int xl, int xr, int yd, int yu, float (&f)[72]) {
    const unsigned oc = (unsigned)(y * nx), od = (unsigned)(yd * nx), ou = (unsigned)(yu * nx);
    const unsigned xb = cdir(N) > 0.1 ? xl : xr;
    const unsigned rb = sdir(N) > 0.1 ? od : ou;
    if constexpr (N % 3 == 0) {
        const unsigned src = N == 0 ? oc + xl : N == 3 ? od + x : N == 6 ? oc + xr : ou + x;
        float g[6];
        dev_tap<ST, N>(base, rs, plane, src, g);
#pragma unroll
        for (int k = 0; k < 6; ++k) f[6 * N + k] = g[k];
    } else {
        float bb[6], bx[6], cb[6], cx[6];
        dev_tap<ST, N>(base, rs, plane, rb + xb, bb);
        dev_tap<ST, N>(base, rs, plane, rb + x, bx);
        dev_tap<ST, N>(base, rs, plane, oc + xb, cb);
        dev_tap<ST, N>(base, rs, plane, oc + x, cx);
        bilinear_direction<N>(bb, bx, cb, cx, f);
    }
}

// Direct pull of a cell (no staging): every tap decoded from global memory.
template <int ST>
__device__ __forceinline__ void pull_dev(const void *fin, long long plane, int nx, int x, int y, int xl, int xr, int yd,
                                         int yu, float (&f)[72]) {
    const char *base = (const char *)fin;
    const rsrc_t rs = make_rsrc(base + 144LL * plane, 48u * (unsigned)plane);
    dev_pull_direction<ST, 0>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
    dev_pull_direction<ST, 1>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
    dev_pull_direction<ST, 2>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
    dev_pull_direction<ST, 3>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
    dev_pull_direction<ST, 4>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
    dev_pull_direction<ST, 5>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
    dev_pull_direction<ST, 6>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
    dev_pull_direction<ST, 7>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
    dev_pull_direction<ST, 8>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
    dev_pull_direction<ST, 9>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
    dev_pull_direction<ST, 10>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
    dev_pull_direction<ST, 11>(base, rs, plane, nx, x, y, xl, xr, yd, yu, f);
}

// ---------------------------------------------------------------- tile-staged pull
// A workgroup covers a tile of tx x ty cells; its halo tile of (tx + 2) x (ty + 2) source
// cells is read once per direction into LDS (six floats per cell; 16-bit deviations are
// decoded on the way), and every cell then interpolates its direction from LDS.  Each
// source value is read (and decoded) 1.3 to 1.5 times per step (the halo over the
// tile: 324, 340 or 396 cells for 256) instead of up to four times (once per pulling
// cell).  Two LDS buffers alternate between directions, so one barrier per direction
// suffices, and the halo values of the next two (FP32) or three (16-bit) directions
// are in flight during each round.  Halo cell h (row-major in the halo tile) is
// handled by thread h and, for h >= 256, by thread h - 256; tiles with more than 512
// halo cells use the direct pull.
constexpr int STAGED_MAX_HALO = 512;

// source coordinate of a halo position (one step outside the grid at most matters;
// positions further out feed only cells outside the grid and are clamped in bounds)
__device__ __forceinline__ int halo_src(int g, int n, int bc_lo, int bc_hi) {
    if (g < 0) return bc_lo == RLBM_BC_PERIODIC ? n - 1 : 0;
    if (g >= n) return (bc_hi == RLBM_BC_PERIODIC && g == n) ? 0 : n - 1;
    return g;
}

// What the staged pull reads per halo cell and direction, and how it becomes six floats.
template <int ST, typename S>
struct Stage;

template <int ST>
struct Stage<ST, Dev16> {
    using Raw = u32x3;                 // six SNORM16 codes
    using Side = DecodeRef;            // the cell's side record, read once per step
    static __device__ __forceinline__ void side(const void *fin, long long plane, unsigned cell, Side &d) {
        const rsrc_t rs = make_rsrc((const char *)fin + 144LL * plane, 48u * (unsigned)plane);
        SideRef sr;
        load_side(rs, cell, sr);
        d = decode_ref(sr);
    }
    template <int N>
    static __device__ __forceinline__ void load(const void *fin, long long plane, unsigned cell, Raw &q) {
        const rsrc_t r = make_rsrc((const char *)fin + (long long)N * plane * 12, 12u * (unsigned)plane);
        q = __builtin_amdgcn_raw_buffer_load_b96(r, cell * 12u, 0u, LOAD_POLICY);
    }
    template <int N>
    static __device__ __forceinline__ void value(const Side &d, const Raw &q, float (&g)[6]) { dev_decode<ST, N>(d, q, g); }
};

template <int ST>
struct Stage<ST, float> {
    struct Raw {
        float v[6];
    };
    struct Side {};
    static __device__ __forceinline__ void side(const void *, long long, unsigned, Side &) {}
    template <int N>
    static __device__ __forceinline__ void load(const void *fin, long long plane, unsigned cell, Raw &q) {
        const rsrc_t r = make_rsrc((const float *)fin + (long long)(6 * N) * plane, 24u * (unsigned)plane);
        Rec<float>::load(r, cell, (unsigned)plane, q.v);
    }
    template <int N>
    static __device__ __forceinline__ void value(const Side &, const Raw &q, float (&g)[6]) {
#pragma unroll
        for (int k = 0; k < 6; ++k) g[k] = q.v[k];
    }
};

template <int ST, typename S>
struct HaloCell {
    typename Stage<ST, S>::Side side;
    unsigned cell;
    bool valid;
};

// Loads are issued for both halo slots whether or not the slot holds a halo cell (an
// empty slot reads cell 0 and is never written to LDS): with no branch around them the
// compiler can wait for exactly the previous direction's loads and leave the next
// direction's in flight.
template <int ST, typename S, int N>
__device__ __forceinline__ void stage_load(const void *fin, long long plane, const HaloCell<ST, S> (&hc)[2],
                                           typename Stage<ST, S>::Raw (&q)[2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) Stage<ST, S>::template load<N>(fin, plane, hc[j].cell, q[j]);
}

template <int ST, typename S, int N>
__device__ __forceinline__ void stage_write(const HaloCell<ST, S> (&hc)[2], const typename Stage<ST, S>::Raw (&q)[2],
                                            int tid, float *buf) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        if (!hc[j].valid) continue;
        float g[6];
        Stage<ST, S>::template value<N>(hc[j].side, q[j], g);
        float *dst = buf + 6 * (tid + 256 * j);
#pragma unroll
        for (int k = 0; k < 6; k += 2) *reinterpret_cast<float2 *>(dst + k) = make_float2(g[k], g[k + 1]);
    }
}

__device__ __forceinline__ void lds_read_tap(const float *buf, int h, float (&g)[6]) {
    const float *src = buf + 6 * h;
#pragma unroll
    for (int k = 0; k < 6; k += 2) {
        const float2 v = *reinterpret_cast<const float2 *>(src + k);
        g[k] = v.x;
        g[k + 1] = v.y;
    }
}

// Direction N of the cell at halo position (hx, hy) from the staged buffer.
template <int N>
__device__ __forceinline__ void lds_direction(const float *buf, int hw, int hx, int hy, float (&f)[72]) {
    const int xb = cdir(N) > 0.1 ? hx - 1 : (cdir(N) < -0.1 ? hx + 1 : hx);
    const int yb = sdir(N) > 0.1 ? hy - 1 : (sdir(N) < -0.1 ? hy + 1 : hy);
    if constexpr (N % 3 == 0) {
        float g[6];
        lds_read_tap(buf, yb * hw + xb, g);
#pragma unroll
        for (int k = 0; k < 6; ++k) f[6 * N + k] = g[k];
    } else {
        float bb[6], bx[6], cb[6], cx[6];
        lds_read_tap(buf, yb * hw + xb, bb);
        lds_read_tap(buf, yb * hw + hx, bx);
        lds_read_tap(buf, hy * hw + xb, cb);
        lds_read_tap(buf, hy * hw + hx, cx);
        bilinear_direction<N>(bb, bx, cb, cx, f);
    }
}

// Directions whose halo values are in flight while a round works (register cost:
// depth x 2 halo slots x 3 (16-bit deviations) or 6 (FP32) registers).  Measured: FP32
// best at 2 (3: -0.1%), 16-bit deviations at 3 (+0.5 to +1% over 2).
template <typename S>
constexpr int STAGE_AHEAD = std::is_same<S, Dev16>::value ? 3 : 2;

// One direction of the staged pull: q[i] holds direction N + i's halo values (requested
// in earlier rounds); direction N + STAGE_AHEAD<S>'s are requested first.
template <int ST, typename S, int N>
__device__ __forceinline__ void stage_round(const void *fin, long long plane, const HaloCell<ST, S> (&hc)[2], int tid,
                                            float *lds, int nh, int hw, int hx, int hy, bool use,
                                            typename Stage<ST, S>::Raw (&q)[STAGE_AHEAD<S>][2], float (&f)[72]) {
    constexpr int D = STAGE_AHEAD<S>;
    typename Stage<ST, S>::Raw qn[2];
    if constexpr (N + D < 12) stage_load<ST, S, N + D>(fin, plane, hc, qn);
    float *buf = lds + (N & 1) * 6 * nh;
    stage_write<ST, S, N>(hc, q[0], tid, buf);
    __syncthreads();
    if (use) lds_direction<N>(buf, hw, hx, hy, f);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int i = 0; i + 1 < D; ++i) q[i][j] = q[i + 1][j];
        if constexpr (N + D < 12) q[D - 1][j] = qn[j];
    }
}

template <int ST, typename S, int I>
__device__ __forceinline__ void stage_prime(const void *fin, long long plane, const HaloCell<ST, S> (&hc)[2],
                                            typename Stage<ST, S>::Raw (&q)[STAGE_AHEAD<S>][2]) {
    if constexpr (I < STAGE_AHEAD<S>) {
        stage_load<ST, S, I>(fin, plane, hc, q[I]);
        stage_prime<ST, S, I + 1>(fin, plane, hc, q);
    }
}

// Tile-staged pull for the workgroup's tile at (x0, y0) of grid a.  Every thread of the
// workgroup calls it (it holds barriers); `use` says whether this thread's own pull
// position (hx, hy) (halo coordinates, its stencil inside the halo tile) takes the
// staged values.
template <int ST, typename S>
__device__ __forceinline__ void staged_pull(const KArgs &a, int x0, int y0, float *lds, int hx, int hy, bool use,
                                            float (&f)[72]) {
    const int tid = (int)threadIdx.x;
    const int hw = a.tx + 2, nh = hw * (a.ty + 2);
    HaloCell<ST, S> hc[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int h = tid + 256 * j;
        hc[j].valid = h < nh;
        const int hxx = h % hw, hyy = h / hw;
        const int sx = halo_src(x0 - 1 + hxx, a.nx, a.bc_xlo, a.bc_xhi);
        const int sy = halo_src(y0 - 1 + hyy, a.ny, a.bc_ylo, a.bc_yhi);
        hc[j].cell = hc[j].valid ? (unsigned)(sy * a.nx + sx) : 0u;
        Stage<ST, S>::side(a.fin, a.plane, hc[j].cell, hc[j].side);
    }
    typename Stage<ST, S>::Raw q[STAGE_AHEAD<S>][2];
    stage_prime<ST, S, 0>(a.fin, a.plane, hc, q);
    stage_round<ST, S, 0>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
    stage_round<ST, S, 1>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
    stage_round<ST, S, 2>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
    stage_round<ST, S, 3>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
    stage_round<ST, S, 4>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
    stage_round<ST, S, 5>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
    stage_round<ST, S, 6>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
    stage_round<ST, S, 7>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
    stage_round<ST, S, 8>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
    stage_round<ST, S, 9>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
    stage_round<ST, S, 10>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
    stage_round<ST, S, 11>(a.fin, a.plane, hc, tid, lds, nh, hw, hx, hy, use, q, f);
}

// Shell scale kept as an IEEE half no smaller than s: s (1 + 2^-10) + 2^-24 rounds to
// nearest at most 2^-11 s (normal halves) or 2^-25 (subnormals) below itself.
__device__ __forceinline__ _Float16 scale_half(float s) { return (_Float16)fmaf(s, 1.0009765625f, 5.9604645e-8f); }

typedef short s16x2 __attribute__((ext_vector_type(2)));

// Sum over the 12 directions of c_n v_n and s_n v_n from the differences
// d_n = v_n - v_{n+6} of opposite directions (cos phi_n = 1, S3H, 1/2, 0, -1/2, -S3H and
// sin phi_n = 0, 1/2, S3H, 1, S3H, 1/2 for n = 0..5).
__device__ __forceinline__ float dipole_c(const float (&d)[6]) {
    return d[0] + (float)S3H * (d[1] - d[5]) + 0.5f * (d[2] - d[4]);
}
__device__ __forceinline__ float dipole_s(const float (&d)[6]) {
    return d[3] + 0.5f * (d[1] + d[5]) + (float)S3H * (d[2] + d[4]);
}

// The same sums with sqrt(3)/2 carried as two floats (hi + lo), so the constant is
// exact to FP64 and only the arithmetic rounds: these sums feed a correction applied
// in every cell and step, and a constant off by 2e-8 would bias it the same way each
// time.
constexpr float S3H_HI = (float)S3H;
constexpr float S3H_LO = (float)(S3H - (double)S3H_HI);
__device__ __forceinline__ float dipole_c_exact(const float (&d)[6]) {
    const float a = d[1] - d[5];
    return fmaf(S3H_LO, a, fmaf(S3H_HI, a, fmaf(0.5f, d[2] - d[4], d[0])));
}
__device__ __forceinline__ float dipole_s_exact(const float (&d)[6]) {
    const float a = d[2] + d[4];
    return fmaf(S3H_LO, a, fmaf(S3H_HI, a, fmaf(0.5f, d[1] + d[5], d[3])));
}

// x / d with a rounding error of at most about half an ulp, either sign: x times the
// rounded reciprocal c, then one correction by the exact residual x - d q.  (x * c
// alone is off by the relative error of c, the same sign every time: applied to a
// conserved density in every cell and step, that would be a steady drift.)
__device__ __forceinline__ float div_by(float x, float d, float c) {
    const float q = x * c;
    return fmaf(fmaf(-q, d, x), c, q);
}

// Momentum density sum_q f p^0 p^x (weights, momenta and cosines exact) of the decoded
// dipole p~_k (alpha c~_n + beta s~_n) per unit of alpha, where the decoder's p~_k, c~_n,
// s~_n are the shell momenta, cosines and sines rounded to float:
// sum_k W_k P_k^2 p~_k * sum_n c_n c~_n.  (sum_n c_n s~_n vanishes: the rounded values
// keep the table's symmetry; the y sum is the same.)
template <int ST>
constexpr double dipole_moment_norm() {
    double m = 0.0;
    for (int k = 0; k < 6; ++k)
        m += W_SHELL[ST][k] * P_SHELL[ST][k] * P_SHELL[ST][k] * (double)(float)P_SHELL[ST][k];
    double c = 0.0;
    for (int n = 0; n < 12; ++n) c += cdir(n) * (double)(float)cdir(n);
    return m * c;
}

// Encode the populations g = f/w of one cell (post-collision) as 16-bit deviations.
// The reference R_{k,n} = rho_k + p_k (alpha cos phi_n + beta sin phi_n) is the shell
// average plus the least-squares dipole; each shell's deviations are coded against
// its own maximum (a half, rounded up).  After coding, rho_k, alpha and beta are
// corrected so that the decoded populations keep the cell's shell sums (so N^0 and
// T^00) and its momentum density T^{0x}, T^{0y} exactly: the rounding errors of the
// codes would otherwise act as a small random source of those conserved quantities in
// every cell and step.
template <int ST>
__device__ __forceinline__ void store_dev(void *fout, long long plane, int off, const float (&f)[72]) {
    char *base = (char *)fout;
    float g[72];
#pragma unroll
    for (int q = 0; q < 72; ++q) g[q] = f[q];
    float rho[6], shell_sum[6], A = 0.0f, B = 0.0f;
    double pp = 0.0, X = 0.0, Y = 0.0;   // T^{0x}, T^{0y} (weights exact)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        // directions n and n + 6 are opposite: sums e_n = g_n + g_{n+6} enter the
        // average, differences d_n = g_n - g_{n+6} the dipole
        float e[6], d[6];
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            e[n] = g[6 * n + k] + g[6 * (n + 6) + k];
            d[n] = g[6 * n + k] - g[6 * (n + 6) + k];
        }
        const float sum = ((e[0] + e[1]) + (e[2] + e[3])) + (e[4] + e[5]);
        const float sc = dipole_c(d), ss = dipole_s(d);
        shell_sum[k] = sum;
        rho[k] = sum * (1.0f / 12.0f);
        const float p = (float)P_SHELL[ST][k];
        const double wpp = W_SHELL[ST][k] * P_SHELL[ST][k] * P_SHELL[ST][k];
        A = fmaf(p, sc, A);
        B = fmaf(p, ss, B);
        X = fma(wpp, (double)dipole_c_exact(d), X);
        Y = fma(wpp, (double)dipole_s_exact(d), Y);
        pp += P_SHELL[ST][k] * P_SHELL[ST][k];
    }
    // least-squares dipole: sum_n cos^2 = 6 over the 12 directions
    const float inv_den = (float)(1.0 / (6.0 * pp));
    const float alpha = A * inv_den, beta = B * inv_den;
    float smax[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int n = 0; n < 12; ++n) {
        const float tn = fma_c(beta, sdir(n), fma_c(alpha, cdir(n), -0.0f));
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            g[6 * n + k] -= rho[k] + (float)P_SHELL[ST][k] * tn;
            smax[k] = fmaxf(smax[k], fabsf(g[6 * n + k]));
        }
    }
    // per-shell scale (a half, rounded up) and its reciprocal: the hardware reciprocal
    // (1 ulp) may put |e| a hair above 1, where the SNORM16 conversion saturates
    _Float16 sh[6];
    float inv[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        sh[k] = scale_half(smax[k]);
        inv[k] = __builtin_amdgcn_rcpf((float)sh[k]);
    }
    const unsigned uoff = (unsigned)off;
    unsigned code[12][3];
#pragma unroll
    for (int n = 0; n < 12; ++n) {
        const rsrc_t r = make_rsrc(base + (long long)n * plane * 12, 12u * (unsigned)plane);
        u32x3 w;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const s16x2 q = __builtin_amdgcn_cvt_pknorm_i16(g[6 * n + 2 * j] * inv[2 * j],
                                                            g[6 * n + 2 * j + 1] * inv[2 * j + 1]);
            w[j] = code[n][j] = __builtin_bit_cast(unsigned, q);
        }
        __builtin_amdgcn_raw_buffer_store_b96(w, r, uoff * 12u, 0u, STORE_POLICY);
    }
    // the codes' shell sums and dipole sums, and the corrections that restore the
    // cell's conserved densities (the decoder's step is the half scale times 1/32767)
    double DX = 0.0, DY = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        float e[6], d[6];
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            const float a = dev_value(u32x3{code[n][0], code[n][1], code[n][2]}, k);
            const float b = dev_value(u32x3{code[n + 6][0], code[n + 6][1], code[n + 6][2]}, k);
            e[n] = a + b;
            d[n] = a - b;
        }
        const float S = ((e[0] + e[1]) + (e[2] + e[3])) + (e[4] + e[5]);   // integer, exact
        const float step = (float)sh[k] * SNORM16_STEP;
        rho[k] = div_by(fmaf(-step, S, shell_sum[k]), 12.0f, 1.0f / 12.0f);
        const double wpps = W_SHELL[ST][k] * P_SHELL[ST][k] * P_SHELL[ST][k] * (double)step;
        DX = fma(wpps, (double)dipole_c_exact(d), DX);
        DY = fma(wpps, (double)dipole_s_exact(d), DY);
    }
    // the decoded momentum density is alpha * dipole_moment_norm + DX: keep it at X
    constexpr double inv_m3 = 1.0 / dipole_moment_norm<ST>();
    const float alpha_c = (float)((X - DX) * inv_m3), beta_c = (float)((Y - DY) * inv_m3);
    const rsrc_t rs = make_rsrc(base + 144LL * plane, 48u * (unsigned)plane);
    const u32x4 s0 = {float_as_u32(rho[0]), float_as_u32(rho[1]), float_as_u32(rho[2]), float_as_u32(rho[3])};
    const u32x4 s1 = {float_as_u32(rho[4]), float_as_u32(rho[5]), float_as_u32(alpha_c), float_as_u32(beta_c)};
    const f16x2 h01 = {sh[0], sh[1]}, h23 = {sh[2], sh[3]}, h45 = {sh[4], sh[5]};
    const u32x4 s2 = {__builtin_bit_cast(unsigned, h01), __builtin_bit_cast(unsigned, h23),
                      __builtin_bit_cast(unsigned, h45), 0u};
    __builtin_amdgcn_raw_buffer_store_b128(s0, rs, uoff * 48u, 0u, STORE_POLICY);
    __builtin_amdgcn_raw_buffer_store_b128(s1, rs, uoff * 48u, 16u, STORE_POLICY);
    __builtin_amdgcn_raw_buffer_store_b128(s2, rs, uoff * 48u, 32u, STORE_POLICY);
}

__device__ __forceinline__ void report(unsigned *status, unsigned flags) {
    if (flags) atomicOr(status, flags);
}

// ---------------------------------------------------------------- kernels
// One fused update of cell (x, y) of the grid described by a.
// FORCED: the variant for forced flows and RLBM_BC_WALL_NEQ rows (Sec. 3.4).
// Where cell (x, y) pulls from: wall cells (fixed-temperature columns, and for the
// forced variant the non-equilibrium wall rows) take the pull of their fluid neighbour.
struct CellPlan {
    bool wall_lo, wall_hi, neq_lo, neq_hi;
    int xe, ye;
};

template <bool FORCED>
__device__ __forceinline__ CellPlan plan_cell(const KArgs &a, int x, int y) {
    CellPlan c;
    c.wall_lo = (a.bc_xlo == RLBM_BC_WALL_T) && x == 0;
    c.wall_hi = (a.bc_xhi == RLBM_BC_WALL_T) && x == a.nx - 1;
    c.xe = c.wall_lo ? 1 : (c.wall_hi ? a.nx - 2 : x);   // wall cells read their fluid neighbour
    c.neq_lo = c.neq_hi = false;
    c.ye = y;
    if constexpr (FORCED) {
        c.neq_lo = (a.bc_ylo == RLBM_BC_WALL_NEQ) && y == 0;
        c.neq_hi = (a.bc_yhi == RLBM_BC_WALL_NEQ) && y == a.ny - 1;
        c.ye = c.neq_lo ? 1 : (c.neq_hi ? a.ny - 2 : y);   // wall rows update their fluid neighbour first
    }
    return c;
}

template <typename S, typename R, int ST>
__device__ __forceinline__ void pull_cell(const KArgs &a, const CellPlan &c, R (&f)[72]) {
    int xl, xr, yd, yu;
    neighbours(a, c.xe, c.ye, xl, xr, yd, yu);
    if constexpr (std::is_same<S, Dev16>::value) pull_dev<ST>(a.fin, a.plane, a.nx, c.xe, c.ye, xl, xr, yd, yu, f);
    else pull<S, R>((const S *)a.fin, a.plane, a.nx, c.xe, c.ye, xl, xr, yd, yu, f);
}

// Everything after the pull: moments, Landau frame, inversion, tau, equilibrium,
// relaxation (or the wall rules), store.
template <int ST, typename S, typename R, int N = 5, bool FORCED = false>
__device__ __forceinline__ void finish_cell(const KArgs &a, int x, int y, const CellPlan &c, R (&f)[72]) {
    unsigned flags = 0;
    const bool wall_lo = c.wall_lo, wall_hi = c.wall_hi, neq_lo = c.neq_lo, neq_hi = c.neq_hi;
    (void)neq_lo;
    (void)neq_hi;
    const Mom m = moments<ST, R, std::is_same<S, Dev16>::value>(f);
    Macro M;
    int iters;
    state_from_moments<ST, sizeof(R) == 4>(m, M, flags, a, iters);
    if (ST != RLBM_MJ && a.stats) {
        // one atomic per wavefront: sum the lanes' iteration counts first
        unsigned long long it = (unsigned long long)iters;
        if (__activemask() == ~0ull) {
            for (int off = 32; off > 0; off >>= 1) it += __shfl_down(it, off, 64);
            if ((threadIdx.x & 63) == 0) atomicAdd(&a.stats[0], it);
        } else {
            atomicAdd(&a.stats[0], it);   // partial wavefront at a grid edge
        }
    }
    if (wall_lo || wall_hi) {
        // zeroth-order extrapolation of n and u, fixed wall temperature
        const double n = M.n;
        state_from_n_theta<ST>(n, wall_lo ? a.th_wall_lo : a.th_wall_hi, M, flags);
        equilibrium_relax<ST, EQ_SET, R, N, std::is_same<S, Dev16>::value>(M, 1.0, f);
    } else {
        const double tau = (a.tau_mode == RLBM_TAU_CONST) ? a.tau : qdiv<sizeof(R) == 4>(a.tau_a, M.theta) + a.tau_b;
        if constexpr (FORCED) {
            // momentum update: the collision sees u + a tau
            M.ux += a.force_x * tau;
            M.uy += a.force_y * tau;
            if (!(M.ux * M.ux + M.uy * M.uy < 1.0)) {
                flags |= RLBM_FLAG_SUPERLUMINAL;
                M.ux = M.uy = 0.0;
            }
            M.ga = 1.0 / sqrt(1.0 - (M.ux * M.ux + M.uy * M.uy));
            if (neq_lo || neq_hi) {
                // wall row: f^eq(wall_n, wall_theta, u = 0) + (f* - f^eq) of the fluid neighbour
                equilibrium_relax<ST, EQ_NEQ, R, N, std::is_same<S, Dev16>::value>(M, tau, f);
                state_from_n_theta<ST>(a.wall_n, a.wall_theta, M, flags);
                M.ux = M.uy = 0.0;
                M.ga = 1.0;
                equilibrium_relax<ST, EQ_ADD, R, N, std::is_same<S, Dev16>::value>(M, 1.0, f);
            } else {
                equilibrium_relax<ST, EQ_COLLIDE, R, N, std::is_same<S, Dev16>::value>(M, tau, f);
            }
        } else {
            equilibrium_relax<ST, EQ_COLLIDE, R, N, std::is_same<S, Dev16>::value>(M, tau, f);
        }
    }
    if constexpr (std::is_same<S, Dev16>::value) store_dev<ST>(a.fout, a.plane, y * a.nx + x, f);
    else store<S, R>((S *)a.fout, a.plane, y * a.nx + x, f);
    report(a.status, flags);
}

template <int ST, typename S, typename R, int N = 5, bool FORCED = false>
__device__ __forceinline__ void step_cell(const KArgs &a, int x, int y) {
    const CellPlan c = plan_cell<FORCED>(a, x, y);
    R f[72];
    pull_cell<S, R, ST>(a, c, f);
    finish_cell<ST, S, R, N, FORCED>(a, x, y, c, f);
}

// One tile with the staged pull (16-bit deviations or FP32 populations).  All threads
// of the workgroup take part in the staging (its barriers); cells outside the grid stop
// after it.  A wall cell whose fluid neighbour's stencil falls outside the halo tile
// (the high x wall when a tile starts on it) pulls directly, with the same arithmetic.
template <int ST, typename S>
__device__ __forceinline__ void staged_tile(const KArgs &a, int txi, int tyi, float *lds) {
    const int x0 = txi * a.tx, y0 = tyi * a.ty;
    const int lx = (int)threadIdx.x % a.tx, ly = (int)threadIdx.x / a.tx;
    const int x = x0 + lx, y = y0 + ly;
    const bool active = x < a.nx && y < a.ny;
    const CellPlan c = plan_cell<false>(a, x, y);
    const int hx = c.xe - x0 + 1, hy = c.ye - y0 + 1;
    const bool inside = hx >= 1 && hx <= a.tx && hy >= 1 && hy <= a.ty;
    float f[72];
    // 16-bit deviations: the kernel is bound by instruction issue, so the waves of a
    // workgroup in its staged pull (loads, barriers) issue ahead of the others' collision
    // work (measured +2.8% on the FD hot spot; FP32, latency-bound, lost 1-2% with it)
    constexpr bool PRIO = std::is_same<S, Dev16>::value;
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
    staged_pull<ST, S>(a, x0, y0, lds, hx, hy, active && inside, f);
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
    if (!active) return;
    if (!inside) pull_cell<S, float, ST>(a, c, f);
    finish_cell<ST, S, float, 5, false>(a, x, y, c, f);
}

template <int ST, typename S, typename R, int N = 5, bool FORCED = false>
__global__ RLBM_STEP_BOUNDS(ST, R, FORCED) void k_step(KArgs a) {
    int x, y;
    if (!cell_of(a, x, y)) return;
    step_cell<ST, S, R, N, FORCED>(a, x, y);
}

// Staged-pull step (tiles with at most STAGED_MAX_HALO halo cells); dynamic LDS:
// 2 x 6 floats per halo cell.
template <int ST, typename S>
__global__ RLBM_STEP_BOUNDS(ST, float, false) void k_step_staged(KArgs a) {
    extern __shared__ float stage_lds[];
    const int b = blockIdx.x;
    const int t = (b & 7) * a.per_xcd + (b >> 3);
    if (t >= a.ntiles) return;                 // the whole workgroup leaves together
    int txi, tyi;
    tile_xy(a, t, txi, tyi);
    staged_tile<ST, S>(a, txi, tyi, stage_lds);
}

// Many grids in one launch.  The tiles of all grids are numbered consecutively
// (grid g owns tiles tile_base[g] .. tile_base[g+1]-1, tile_grid[t] = g); a
// persistent set of workgroups sweeps them, XCD k taking the contiguous tile
// range [k T/8, (k+1) T/8) so neighbouring tiles share that XCD's L2.  descs holds
// each grid's arguments with in/out buffers for the current parity.
struct Batch {
    int ntiles;
    int per_xcd;        // ceil(ntiles / 8)
    int groups_per_xcd; // workgroups launched per XCD
    int staged;         // staged pull (dynamic LDS sized for the tile)
};

template <int ST, typename S, typename R>
__global__ RLBM_BATCH_BOUNDS(ST, R) void k_step_batch(Batch b, const KArgs *__restrict__ descs,
                                                 const int *__restrict__ tile_grid, const int *__restrict__ tile_base) {
    const int xcd = blockIdx.x & 7;
    const int lane_group = blockIdx.x >> 3;
    const int t_begin = xcd * b.per_xcd;
    const int t_end = min(t_begin + b.per_xcd, b.ntiles);
    for (int t = t_begin + lane_group; t < t_end; t += b.groups_per_xcd) {
        // the grid index is the same for the whole workgroup: keep it (and so every
        // field of its descriptor and every buffer descriptor) in scalar registers
        const int g = __builtin_amdgcn_readfirstlane(tile_grid[t]);
        const KArgs a = descs[g];
        const int lt = t - __builtin_amdgcn_readfirstlane(tile_base[g]);
        int txi, tyi;
        tile_xy(a, lt, txi, tyi);
        if constexpr (!std::is_same<S, double>::value) {
            if (b.staged) {
                extern __shared__ float stage_lds[];
                // no barrier between tiles: the buffers keep alternating by direction
                // parity, so every read of a buffer ends before the next tile's
                // barrier that precedes its rewrite
                staged_tile<ST, S>(a, txi, tyi, stage_lds);
                continue;
            }
        }
        const int x = txi * a.tx + (int)threadIdx.x % a.tx;
        const int y = tyi * a.ty + (int)threadIdx.x / a.tx;
        if (x < a.nx && y < a.ny) step_cell<ST, S, R>(a, x, y);
    }
}

// One workgroup per tile of the batch (workgroup b takes tile (b % 8) per_xcd + b / 8,
// so each XCD sweeps a contiguous range).  Without the persistent loop the kernel
// fits the single-grid register budget (3 waves per SIMD for FP32).
template <int ST, typename S, typename R>
__global__ RLBM_STEP_BOUNDS(ST, R, false) void k_step_tiles(Batch b, const KArgs *__restrict__ descs,
                                                        const int *__restrict__ tile_grid,
                                                        const int *__restrict__ tile_base) {
    const int t = (blockIdx.x & 7) * b.per_xcd + (blockIdx.x >> 3);
    if (t >= b.ntiles) return;
    const int g = __builtin_amdgcn_readfirstlane(tile_grid[t]);
    const KArgs a = descs[g];
    const int lt = t - __builtin_amdgcn_readfirstlane(tile_base[g]);
    int txi, tyi;
    tile_xy(a, lt, txi, tyi);
    if constexpr (!std::is_same<S, double>::value) {
        if (b.staged) {
            extern __shared__ float stage_lds[];
            staged_tile<ST, S>(a, txi, tyi, stage_lds);
            return;
        }
    }
    const int x = txi * a.tx + (int)threadIdx.x % a.tx;
    const int y = tyi * a.ty + (int)threadIdx.x / a.tx;
    if (x < a.nx && y < a.ny) step_cell<ST, S, R>(a, x, y);
}

template <int ST, typename S, typename R>
__global__ __launch_bounds__(256) void k_moments(KArgs a) {
    int x, y;
    if (!cell_of(a, x, y)) return;
    unsigned flags = 0;
    int xl, xr, yd, yu;
    neighbours(a, x, y, xl, xr, yd, yu);
    R f[72];
    if constexpr (std::is_same<S, Dev16>::value) pull_dev<ST>(a.fin, a.plane, a.nx, x, y, xl, xr, yd, yu, f);
    else pull<S, R>((const S *)a.fin, a.plane, a.nx, x, y, xl, xr, yd, yu, f);
    const Mom m = moments<ST, R, std::is_same<S, Dev16>::value>(f);
    Macro M;
    int iters;
    double L;
    state_from_moments<ST, sizeof(R) == 4>(m, M, flags, a, iters, &L);
    const int off = y * a.nx + x;
    if (a.o_mlx) a.o_mlx[off] = (float)L;
    if (a.o_mlt) a.o_mlt[off] = (float)log(M.z);
    const double hE = 3.0 * M.theta * M.g[3] / M.g[2];
    if (a.o_n) a.o_n[off] = M.n;
    if (a.o_eps) a.o_eps[off] = M.eps;
    if (a.o_theta) a.o_theta[off] = M.theta;
    if (a.o_z) a.o_z[off] = M.z;
    if (a.o_ux) a.o_ux[off] = M.ux;
    if (a.o_uy) a.o_uy[off] = M.uy;
    if (a.o_qx) a.o_qx[off] = hE * (M.n * M.ga * M.ux - m.Nx);
    if (a.o_qy) a.o_qy[off] = hE * (M.n * M.ga * M.uy - m.Ny);
    const double raw[9] = {m.N0, m.Nx, m.Ny, m.T00, m.T01, m.T02, m.T11, m.T12, m.T22};
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (a.o_mom[i]) a.o_mom[i][off] = raw[i];
    report(a.status, flags);
}

// sum_i f_i (p_i^x)^r for r = 2..5, in FP64: p^x = p_k cos(phi_n).
template <int ST, typename R, bool GU = false>
__device__ __forceinline__ void px_powers(const R (&f)[72], double (&o)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = 0.0;
#pragma unroll
    for (int n = 0; n < 12; ++n) {
        if (n == 3 || n == 9) continue;   // cos(phi_n) = 0
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double p = P_SHELL[ST][k], v = (double)f[6 * n + k] * (GU ? W_SHELL[ST][k] : 1.0);
            a[0] += v * (p * p);
            a[1] += v * (p * p * p);
            a[2] += v * (p * p * p * p);
            a[3] += v * (p * p * p * p * p);
        }
        const double c = cdir(n);
        o[0] += a[0] * (c * c);
        o[1] += a[1] * (c * c * c);
        o[2] += a[2] * (c * c * c * c);
        o[3] += a[3] * (c * c * c * c * c);
    }
}

// Diagonal x components of the non-equilibrium tensors, pi^{x..x} = sum_i (f_i -
// f^eq_i) (p_i^x)^r for r = 2..5 (Eq. tensors-eq), of the pre-collision populations
// the next step would see; f^eq is the order-N equilibrium of the cell's own state.
template <int ST, typename S, typename R, int N>
__global__ __launch_bounds__(256) void k_noneq(KArgs a) {
    int x, y;
    if (!cell_of(a, x, y)) return;
    unsigned flags = 0;
    int xl, xr, yd, yu;
    neighbours(a, x, y, xl, xr, yd, yu);
    R f[72];
    if constexpr (std::is_same<S, Dev16>::value) pull_dev<ST>(a.fin, a.plane, a.nx, x, y, xl, xr, yd, yu, f);
    else pull<S, R>((const S *)a.fin, a.plane, a.nx, x, y, xl, xr, yd, yu, f);
    const Mom m = moments<ST, R, std::is_same<S, Dev16>::value>(f);
    Macro M;
    int iters;
    state_from_moments<ST, sizeof(R) == 4>(m, M, flags, a, iters);
    double sf[4], se[4];
    px_powers<ST, R, std::is_same<S, Dev16>::value>(f, sf);
    equilibrium_relax<ST, EQ_SET, R, N, std::is_same<S, Dev16>::value>(M, 1.0, f);   // f <- f^eq
    px_powers<ST, R, std::is_same<S, Dev16>::value>(f, se);
    const int off = y * a.nx + x;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (a.o_pi[r]) a.o_pi[r][off] = sf[r] - se[r];
    report(a.status, flags);
}

template <int ST, typename S, typename R, int N = 5>
__global__ __launch_bounds__(256) void k_init(KArgs a) {
    int x, y;
    if (!cell_of(a, x, y)) return;
    unsigned flags = 0;
    const int off = y * a.nx + x;
    Macro M;
    M.ux = a.i_ux[off];
    M.uy = a.i_uy[off];
    const double u2 = M.ux * M.ux + M.uy * M.uy;
    if (!(u2 < 1.0)) {
        flags |= RLBM_FLAG_SUPERLUMINAL;
        M.ux = M.uy = 0.0;
    }
    M.ga = 1.0 / sqrt(1.0 - (M.ux * M.ux + M.uy * M.uy));
    const double th = a.i_theta[off];
    // the largest Anderson-Witting weight gamma (1 - v.u)/tau over the directions is
    // gamma (1 + |u|)/tau; from 2 on the relaxation over-shoots without bound
    const double tau = (a.tau_mode == RLBM_TAU_CONST) ? a.tau : a.tau_a / th + a.tau_b;
    if (!(tau > 0.5 * M.ga * (1.0 + sqrt(M.ux * M.ux + M.uy * M.uy)))) flags |= RLBM_FLAG_UNSTABLE;
    if (a.given_z) state_from_z_theta<ST>(a.i_z[off], th, M, flags);
    else state_from_n_theta<ST>(a.i_n[off], th, M, flags);
    R f[72];
    equilibrium_relax<ST, EQ_SET, R, N, std::is_same<S, Dev16>::value>(M, 1.0, f);
    if constexpr (std::is_same<S, Dev16>::value) store_dev<ST>(a.fout, a.plane, off, f);
    else store<S, R>((S *)a.fout, a.plane, off, f);
    report(a.status, flags);
}

// ---------------------------------------------------------------- host side
using KFn = void (*)(KArgs);

using BFn = void (*)(Batch, const KArgs *, const int *, const int *);

template <int ST>
struct Kern {
    static KFn step(int prec) {
        return prec == RLBM_FP64 ? k_step<ST, double, double>
             : prec == RLBM_FP32 ? k_step<ST, float, float> : k_step<ST, Dev16, float>;
    }
    static KFn staged(int prec) { return prec == RLBM_FP32 ? k_step_staged<ST, float> : k_step_staged<ST, Dev16>; }
    static BFn batch(int prec) {
        return prec == RLBM_FP64 ? k_step_batch<ST, double, double>
             : prec == RLBM_FP32 ? k_step_batch<ST, float, float> : k_step_batch<ST, Dev16, float>;
    }
    static BFn tiles(int prec) {
        return prec == RLBM_FP64 ? k_step_tiles<ST, double, double>
             : prec == RLBM_FP32 ? k_step_tiles<ST, float, float> : k_step_tiles<ST, Dev16, float>;
    }
    static KFn mom(int prec) {
        return prec == RLBM_FP64 ? k_moments<ST, double, double>
             : prec == RLBM_FP32 ? k_moments<ST, float, float> : k_moments<ST, Dev16, float>;
    }
    static KFn init(int prec) {
        return prec == RLBM_FP64 ? k_init<ST, double, double>
             : prec == RLBM_FP32 ? k_init<ST, float, float> : k_init<ST, Dev16, float>;
    }
};

// Maxwell-Juttner kernels of expansion order 2..4 (step, init), FP64 and FP32 storage
template <int N>
KFn pick_lo(int which, int prec) {
    if (which == 0) return prec == RLBM_FP64 ? k_step<RLBM_MJ, double, double, N> : k_step<RLBM_MJ, float, float, N>;
    return prec == RLBM_FP64 ? k_init<RLBM_MJ, double, double, N> : k_init<RLBM_MJ, float, float, N>;
}

KFn pick(int which, int st, int prec);

// forced flow / non-equilibrium walls: order 5, FP64 or FP32 populations
KFn pick_forced(int st, int prec) {
    if (st == RLBM_MJ) return prec == RLBM_FP64 ? k_step<RLBM_MJ, double, double, 5, true> : k_step<RLBM_MJ, float, float, 5, true>;
    if (st == RLBM_FD) return prec == RLBM_FP64 ? k_step<RLBM_FD, double, double, 5, true> : k_step<RLBM_FD, float, float, 5, true>;
    return prec == RLBM_FP64 ? k_step<RLBM_BE, double, double, 5, true> : k_step<RLBM_BE, float, float, 5, true>;
}

bool is_forced(const rlbm_params &p) {
    return p.force[0] != 0.0 || p.force[1] != 0.0 || p.bc[2] == RLBM_BC_WALL_NEQ || p.bc[3] == RLBM_BC_WALL_NEQ;
}

KFn pick_order(int which, int st, int prec, int order) {
    if (order == 5 || which == 1) return pick(which, st, prec);
    if (order == 2) return pick_lo<2>(which, prec);
    if (order == 3) return pick_lo<3>(which, prec);
    return pick_lo<4>(which, prec);
}

template <int ST, int N>
KFn noneq_kernel(int prec) {
    if constexpr (N < 5) return prec == RLBM_FP64 ? k_noneq<ST, double, double, N> : k_noneq<ST, float, float, N>;
    else return prec == RLBM_FP64 ? k_noneq<ST, double, double, N>
              : prec == RLBM_FP32 ? k_noneq<ST, float, float, N> : k_noneq<ST, Dev16, float, N>;
}

KFn pick_noneq(int st, int prec, int order) {
    if (st == RLBM_FD) return noneq_kernel<RLBM_FD, 5>(prec);
    if (st == RLBM_BE) return noneq_kernel<RLBM_BE, 5>(prec);
    return order == 2 ? noneq_kernel<RLBM_MJ, 2>(prec) : order == 3 ? noneq_kernel<RLBM_MJ, 3>(prec)
         : order == 4 ? noneq_kernel<RLBM_MJ, 4>(prec) : noneq_kernel<RLBM_MJ, 5>(prec);
}

KFn pick_staged(int st, int prec) {
    return st == RLBM_MJ ? Kern<RLBM_MJ>::staged(prec) : st == RLBM_FD ? Kern<RLBM_FD>::staged(prec)
                                                        : Kern<RLBM_BE>::staged(prec);
}

// dynamic LDS of the staged pull for tiles of tx x ty, 0 where the direct pull runs:
// FP64 populations, lower orders, forcing, and tiles whose halo exceeds
// STAGED_MAX_HALO cells
size_t staged_lds_bytes(const rlbm_params &p, int tx, int ty) {
    const int nh = (tx + 2) * (ty + 2);
    const bool staged = p.precision == RLBM_DEV16 || (p.precision == RLBM_FP32 && RLBM_FP32_STAGED);
    if (!staged || nh > STAGED_MAX_HALO || p.order != 5 || is_forced(p)) return 0;
    return sizeof(float) * 12 * (size_t)nh;
}

BFn pick_batch(int st, int prec, bool persistent) {
    if (!persistent)
        return st == RLBM_MJ ? Kern<RLBM_MJ>::tiles(prec) : st == RLBM_FD ? Kern<RLBM_FD>::tiles(prec) : Kern<RLBM_BE>::tiles(prec);
    return st == RLBM_MJ ? Kern<RLBM_MJ>::batch(prec) : st == RLBM_FD ? Kern<RLBM_FD>::batch(prec) : Kern<RLBM_BE>::batch(prec);
}

KFn pick(int which, int st, int prec) {
    switch (st) {
        case RLBM_MJ: return which == 0 ? Kern<RLBM_MJ>::step(prec) : which == 1 ? Kern<RLBM_MJ>::mom(prec) : Kern<RLBM_MJ>::init(prec);
        case RLBM_FD: return which == 0 ? Kern<RLBM_FD>::step(prec) : which == 1 ? Kern<RLBM_FD>::mom(prec) : Kern<RLBM_FD>::init(prec);
        default: return which == 0 ? Kern<RLBM_BE>::step(prec) : which == 1 ? Kern<RLBM_BE>::mom(prec) : Kern<RLBM_BE>::init(prec);
    }
}

}  // namespace

struct rlbm_ctx {
    std::vector<rlbm_params> p;     // per grid
    std::vector<KArgs> base;        // per grid, without in/out buffers
    hipStream_t stream;
    unsigned *status;               // device status word
    unsigned long long *stats;      // device inversion counters (collect_stats)
    int64_t stat_steps;             // steps launched with counting on
    int cur;                        // 0: f_a holds the state, 1: f_b
    int64_t steps;
    bool batch;                     // several grids, one persistent launch per step
    int tx, ty;                     // workgroup tile
    // batch tables (device): descs[2][ngrids], tile_grid[ntiles], tile_base[ngrids + 1]
    KArgs *d_descs;
    int *d_tile_grid, *d_tile_base;
    int ntiles_total;
    int batch_groups_per_xcd;
    int persistent;                 // batch: workgroups per XCD (0: one workgroup per tile)
    // replay of captured step chunks
    hipStream_t cap_stream;
    hipGraphExec_t gexec[2];        // GRAPH_CHUNK steps starting from parity 0 / 1
};

namespace {

constexpr int GRAPH_CHUNK = 32;     // even: a replay returns to the starting parity

int validate(const rlbm_params *p) {
    if (!p) return RLBM_EINVAL;
    if (p->nx < 2 || p->ny < 2) return RLBM_EINVAL;
    {
        const long long elem = p->precision == RLBM_FP64 ? 8 : 4;   // DEV16: its 48-byte side records
        const long long span = p->precision == RLBM_DEV16 ? 12 : 6;   // 4-byte planes under one buffer descriptor
        if (span * p->nx * p->ny * elem > 0xFFFFFFFFLL) return RLBM_EINVAL;
    }
    if (p->stats < RLBM_MJ || p->stats > RLBM_BE) return RLBM_EINVAL;
    if (p->order < 2 || p->order > 5) return RLBM_EINVAL;
    if (p->order != 5 && (p->stats != RLBM_MJ || p->precision == RLBM_DEV16))
        return RLBM_ENOTIMPL;   // lower orders: Maxwell-Juttner with FP64 or FP32 populations
    if (p->precision != RLBM_FP64 && p->precision != RLBM_FP32 && p->precision != RLBM_DEV16) return RLBM_EINVAL;
    if (p->tau_mode == RLBM_TAU_CONST) {
        if (!(p->tau > 0.5)) return RLBM_EINVAL;   // gamma (1 + |u|)/2 >= 1/2: unstable for every state
    } else if (p->tau_mode == RLBM_TAU_INV_THETA) {
        if (!(p->tau_a >= 0.0) || !(p->tau_b > 0.0)) return RLBM_EINVAL;
    } else {
        return RLBM_EINVAL;
    }
    for (int i = 0; i < 4; ++i)
        if (p->bc[i] < RLBM_BC_PERIODIC || p->bc[i] > RLBM_BC_WALL_NEQ) return RLBM_EINVAL;
    if (p->bc[0] == RLBM_BC_WALL_NEQ || p->bc[1] == RLBM_BC_WALL_NEQ) return RLBM_EINVAL;   // y sides only
    if (!std::isfinite(p->force[0]) || !std::isfinite(p->force[1])) return RLBM_EINVAL;
    if (is_forced(*p)) {
        if (p->order != 5 || p->precision == RLBM_DEV16) return RLBM_ENOTIMPL;
        if ((p->bc[2] == RLBM_BC_WALL_NEQ || p->bc[3] == RLBM_BC_WALL_NEQ) &&
            (p->ny < 3 || !(p->wall_n > 0.0) || !(p->wall_theta > 0.0)))
            return RLBM_EINVAL;
    }
    if ((p->bc[0] == RLBM_BC_PERIODIC) != (p->bc[1] == RLBM_BC_PERIODIC)) return RLBM_EINVAL;
    if ((p->bc[2] == RLBM_BC_PERIODIC) != (p->bc[3] == RLBM_BC_PERIODIC)) return RLBM_EINVAL;
    if (p->bc[2] == RLBM_BC_WALL_T || p->bc[3] == RLBM_BC_WALL_T) return RLBM_EINVAL;
    if ((p->bc[0] == RLBM_BC_WALL_T || p->bc[1] == RLBM_BC_WALL_T) && p->nx < 4) return RLBM_EINVAL;
    for (int i = 0; i < 2; ++i)
        if (p->bc[i] == RLBM_BC_WALL_T && !(p->theta_wall[i] > 0.0)) return RLBM_EINVAL;
    if (p->guess != RLBM_GUESS_FIXED && p->guess != RLBM_GUESS_MLP) return RLBM_EINVAL;
    if (p->guess == RLBM_GUESS_MLP && !p->mlp) return RLBM_EINVAL;
    if (p->tile_x != 0 || p->tile_y != 0) {
        const int tx = p->tile_x, ty = p->tile_y;
        if (tx < 16 || ty < 1 || tx * ty != 256 || (tx & (tx - 1))) return RLBM_EINVAL;
    }
    if (!p->f_a || !p->f_b || p->f_a == p->f_b) return RLBM_EINVAL;
    return RLBM_OK;
}

bool valid_init(const rlbm_init_fields *init) {
    return init && init->theta && init->ux && init->uy && (init->given_z ? init->z != nullptr : init->n != nullptr);
}

void auto_tile(const rlbm_params &p, int &tx, int &ty) {
    if (p.tile_x > 0) {
        tx = p.tile_x;
        ty = p.tile_y;
        return;
    }
    // Defaults when no tile is given (rlbm_autotune measures instead): 128 x 2 (direct
    // pull) on grids 4096 or more cells wide, where it ran fastest on an 8192-wide grid;
    // otherwise rows of 8, 4 or 2 cells (the staged pull where the halo fits).
    if (p.nx >= 4096 && p.ny >= 2) {
        tx = 128;
        ty = 2;
        return;
    }
    ty = p.ny >= 8 ? 8 : (p.ny >= 4 ? 4 : 2);
    tx = 256 / ty;
}

KArgs make_base(const rlbm_params &p, rlbm_ctx *c) {
    KArgs a{};
    a.nx = p.nx;
    a.ny = p.ny;
    a.plane = (long long)p.nx * p.ny;
    a.bc_xlo = p.bc[0];
    a.bc_xhi = p.bc[1];
    a.bc_ylo = p.bc[2];
    a.bc_yhi = p.bc[3];
    a.tau_mode = p.tau_mode;
    a.tau = p.tau;
    a.tau_a = p.tau_a;
    a.tau_b = p.tau_b;
    a.th_wall_lo = p.theta_wall[0];
    a.th_wall_hi = p.theta_wall[1];
    a.force_x = p.force[0];
    a.force_y = p.force[1];
    a.wall_n = p.wall_n;
    a.wall_theta = p.wall_theta;
    a.guess = p.guess;
    a.mlp = p.mlp;
    a.status = c->status;
    a.stats = p.collect_stats ? c->stats : nullptr;
    return a;
}

// strips: order the tiles in strips (staged-pull launches) or by rows (direct pull,
// whose 128x2 and 256x1 tiles ran 4% slower in strips on an 8192-wide grid, while 64x4
// staged tiles ran 2% faster)
void set_tiles(KArgs &a, int tx, int ty, bool strips = false) {
    a.tx = tx;
    a.ty = ty;
    a.ntx = (a.nx + tx - 1) / tx;
    a.nty = (a.ny + ty - 1) / ty;
    a.ntiles = a.ntx * a.nty;
    a.per_xcd = (a.ntiles + 7) / 8;
    // strip width in tiles (at least one tile; a strip as wide as the grid is row order)
    a.sw = (strips && RLBM_STRIP_CELLS > 0) ? std::min(a.ntx, std::max(1, RLBM_STRIP_CELLS / tx)) : a.ntx;
}

void drop_graphs(rlbm_ctx *c) {
    for (int i = 0; i < 2; ++i)
        if (c->gexec[i]) {
            (void)hipGraphExecDestroy(c->gexec[i]);
            c->gexec[i] = nullptr;
        }
}

void release(rlbm_ctx *c) {
    if (!c) return;
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    (void)hipFree(c->status);
    (void)hipFree(c->stats);
    (void)hipFree(c->d_descs);
    (void)hipFree(c->d_tile_grid);
    (void)hipFree(c->d_tile_base);
    delete c;
}

// (Re)build the tile decomposition of every grid and, for a batch, its device tables.
// Launches still in flight may read the tables and graphs replaced here: wait first.
int configure(rlbm_ctx *c, int tx, int ty) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return RLBM_EHIP;
    drop_graphs(c);
    c->tx = tx;
    c->ty = ty;
    for (auto &a : c->base) set_tiles(a, tx, ty, staged_lds_bytes(c->p[0], tx, ty) > 0);
    if (!c->batch) return RLBM_OK;
    const int ng = (int)c->base.size();
    std::vector<int> tbase(ng + 1, 0);
    for (int g = 0; g < ng; ++g) tbase[g + 1] = tbase[g] + c->base[g].ntiles;
    const int T = tbase[ng];
    std::vector<int> tgrid(T);
    for (int g = 0; g < ng; ++g)
        for (int t = tbase[g]; t < tbase[g + 1]; ++t) tgrid[t] = g;
    std::vector<KArgs> d(2 * ng);
    for (int par = 0; par < 2; ++par)
        for (int g = 0; g < ng; ++g) {
            KArgs a = c->base[g];
            a.fin = par ? c->p[g].f_b : c->p[g].f_a;
            a.fout = par ? c->p[g].f_a : c->p[g].f_b;
            d[par * ng + g] = a;
        }
    (void)hipFree(c->d_tile_grid);
    c->d_tile_grid = nullptr;
    if (hipMalloc(&c->d_tile_grid, sizeof(int) * T) != hipSuccess) return RLBM_EHIP;
    if (!c->d_descs && hipMalloc(&c->d_descs, sizeof(KArgs) * 2 * ng) != hipSuccess) return RLBM_EHIP;
    if (!c->d_tile_base && hipMalloc(&c->d_tile_base, sizeof(int) * (ng + 1)) != hipSuccess) return RLBM_EHIP;
    if (hipMemcpyAsync(c->d_tile_grid, tgrid.data(), sizeof(int) * T, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_tile_base, tbase.data(), sizeof(int) * (ng + 1), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_descs, d.data(), sizeof(KArgs) * 2 * ng, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return RLBM_EHIP;
    c->ntiles_total = T;
    // persistent: c->persistent workgroups per XCD sweep its tile range; 0: one per tile
    const int per_xcd = (T + 7) / 8;
    c->batch_groups_per_xcd = (c->persistent > 0 && c->persistent < per_xcd) ? c->persistent : per_xcd;
    return RLBM_OK;
}

int launch_step(rlbm_ctx *c, hipStream_t s) {
    const rlbm_params &p0 = c->p[0];
    if (c->batch) {
        Batch b;
        b.ntiles = c->ntiles_total;
        b.per_xcd = (c->ntiles_total + 7) / 8;
        b.groups_per_xcd = c->batch_groups_per_xcd;
        const KArgs *descs = c->d_descs + (size_t)c->cur * c->base.size();
        const bool persistent = b.groups_per_xcd < b.per_xcd;
        const size_t lds = staged_lds_bytes(p0, c->tx, c->ty);
        b.staged = lds > 0;
        hipLaunchKernelGGL(pick_batch(p0.stats, p0.precision, persistent), dim3(8 * b.groups_per_xcd), dim3(256), lds, s,
                           b, descs, (const int *)c->d_tile_grid, (const int *)c->d_tile_base);
    } else {
        KArgs a = c->base[0];
        a.fin = c->cur ? p0.f_b : p0.f_a;
        a.fout = c->cur ? p0.f_a : p0.f_b;
        const size_t lds = staged_lds_bytes(p0, c->tx, c->ty);
        if (lds > 0) {
            hipLaunchKernelGGL(pick_staged(p0.stats, p0.precision), dim3(8 * a.per_xcd), dim3(256), lds, s, a);
        } else {
            const KFn k = is_forced(p0) ? pick_forced(p0.stats, p0.precision) : pick_order(0, p0.stats, p0.precision, p0.order);
            hipLaunchKernelGGL(k, dim3(8 * a.per_xcd), dim3(256), 0, s, a);
        }
    }
    c->cur ^= 1;
    c->steps++;
    return hipGetLastError() == hipSuccess ? RLBM_OK : RLBM_EHIP;
}

// Capture GRAPH_CHUNK steps starting at the current parity into an executable graph.
int capture_chunk(rlbm_ctx *c, hipGraphExec_t &out) {
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return RLBM_EHIP;
    const int cur0 = c->cur;
    const int64_t steps0 = c->steps;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return RLBM_EHIP;
    int rc = RLBM_OK;
    for (int i = 0; i < GRAPH_CHUNK && rc == RLBM_OK; ++i) rc = launch_step(c, c->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    c->cur = cur0;          // capturing ran nothing
    c->steps = steps0;
    if (rc != RLBM_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return RLBM_EHIP;
    }
    const hipError_t ei = hipGraphInstantiate(&out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    return ei == hipSuccess ? RLBM_OK : RLBM_EHIP;
}

int finish_init(rlbm_ctx *c, const rlbm_init_fields *init) {
    const rlbm_params &p0 = c->p[0];
    for (size_t g = 0; g < c->base.size(); ++g) {
        KArgs ia = c->base[g];
        set_tiles(ia, 32, 8);
        ia.fout = c->p[g].f_a;
        ia.i_n = init[g].n;
        ia.i_z = init[g].z;
        ia.i_theta = init[g].theta;
        ia.i_ux = init[g].ux;
        ia.i_uy = init[g].uy;
        ia.given_z = init[g].given_z;
        hipLaunchKernelGGL(pick_order(2, p0.stats, p0.precision, p0.order), dim3(8 * ia.per_xcd), dim3(256), 0, c->stream,
                           ia);
    }
    return hipGetLastError() == hipSuccess ? RLBM_OK : RLBM_EHIP;
}

int create(rlbm_ctx **out, int ngrids, const rlbm_params *p, const rlbm_init_fields *init) {
    if (!out) return RLBM_EINVAL;
    *out = nullptr;
    if (ngrids < 1 || !p || !init) return RLBM_EINVAL;
    for (int g = 0; g < ngrids; ++g) {
        int rc = validate(&p[g]);
        if (rc) return rc;
        if (!valid_init(&init[g])) return RLBM_EINVAL;
        const rlbm_params &a = p[g], &b = p[0];
        if (ngrids > 1 && (a.order != 5 || is_forced(a))) return RLBM_ENOTIMPL;   // batches: unforced, order 5
        if (a.stats != b.stats || a.precision != b.precision || a.order != b.order || a.guess != b.guess ||
            a.mlp != b.mlp || a.stream != b.stream || a.tile_x != b.tile_x || a.tile_y != b.tile_y ||
            a.collect_stats != b.collect_stats)
            return RLBM_EINVAL;
    }
    rlbm_ctx *c = new (std::nothrow) rlbm_ctx();
    if (!c) return RLBM_EHIP;
    c->stream = (hipStream_t)p[0].stream;
    c->batch = ngrids > 1;
    if (hipMalloc(&c->status, sizeof(unsigned)) != hipSuccess ||
        hipMalloc(&c->stats, 2 * sizeof(unsigned long long)) != hipSuccess ||
        hipMemsetAsync(c->status, 0, sizeof(unsigned), c->stream) != hipSuccess ||
        hipMemsetAsync(c->stats, 0, 2 * sizeof(unsigned long long), c->stream) != hipSuccess) {
        release(c);
        return RLBM_EHIP;
    }
    c->p.assign(p, p + ngrids);
    for (int g = 0; g < ngrids; ++g) c->base.push_back(make_base(p[g], c));
    int tx, ty;
    auto_tile(p[0], tx, ty);
    if (c->batch && p[0].tile_x == 0) {
        tx = 32;
        ty = 8;
    }
    int rc = configure(c, tx, ty);
    if (!rc) rc = finish_init(c, init);
    if (!rc) {
        // the initial state's stability verdict (RLBM_FLAG_UNSTABLE) decides the call;
        // other bits stay in the status word for rlbm_sync / rlbm_status
        unsigned h = 0;
        if (hipMemcpyAsync(&h, c->status, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            rc = RLBM_EHIP;
        else if (h & RLBM_FLAG_UNSTABLE)
            rc = RLBM_EINVAL;
    }
    if (rc) {
        release(c);
        return rc;
    }
    *out = c;
    return RLBM_OK;
}

}  // namespace

extern "C" {

int rlbm_init(rlbm_ctx **out, const rlbm_params *p, const rlbm_init_fields *init) {
    return create(out, 1, p, init);
}

int rlbm_init_batch(rlbm_ctx **out, int32_t ngrids, const rlbm_params *p, const rlbm_init_fields *init) {
    return create(out, ngrids, p, init);
}

int rlbm_step(rlbm_ctx *c, int64_t nsteps) {
    if (!c || nsteps < 0) return RLBM_EINVAL;
    int64_t left = nsteps;
    if (left >= 2 * GRAPH_CHUNK) {
        // replay captured chunks: one graph launch per GRAPH_CHUNK steps
        hipGraphExec_t &g = c->gexec[c->cur];
        if (!g) {
            int rc = capture_chunk(c, g);
            if (rc) return rc;
        }
        for (; left >= GRAPH_CHUNK; left -= GRAPH_CHUNK) {
            if (hipGraphLaunch(g, c->stream) != hipSuccess) return RLBM_EHIP;
            c->steps += GRAPH_CHUNK;
        }
    }
    for (; left > 0; --left) {
        int rc = launch_step(c, c->stream);
        if (rc) return rc;
    }
    if (c->p[0].collect_stats) c->stat_steps += nsteps;
    return c->p[0].check ? rlbm_sync(c) : RLBM_OK;
}

int rlbm_capture(rlbm_ctx *c) {
    if (!c) return RLBM_EINVAL;
    const int cur0 = c->cur;
    for (int par = 0; par < 2; ++par) {
        c->cur = par;
        if (!c->gexec[par]) {
            int rc = capture_chunk(c, c->gexec[par]);
            if (rc) {
                c->cur = cur0;
                return rc;
            }
        }
    }
    c->cur = cur0;
    return RLBM_OK;
}

int rlbm_configure(rlbm_ctx *c, int32_t tile_x, int32_t tile_y, int32_t persistent) {
    if (!c || tile_x < 16 || tile_y < 1 || tile_x * tile_y != 256 || (tile_x & (tile_x - 1)) || persistent < 0)
        return RLBM_EINVAL;
    c->persistent = persistent;
    return configure(c, tile_x, tile_y);
}

int rlbm_autotune(rlbm_ctx *c, int32_t trial_steps, int32_t *tile_x, int32_t *tile_y) {
    if (!c || trial_steps < 1) return RLBM_EINVAL;
    static const int cand[][3] = {{32, 8, 0}, {64, 4, 0}, {16, 16, 0}, {128, 2, 0}, {256, 1, 0},
                                  {32, 8, 96}, {64, 4, 96}};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return RLBM_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return RLBM_EHIP;
    }
    // three rounds over the candidates, each timed trial_steps steps after one
    // warm-up step; a candidate's time is its best round (clock ramps and other
    // transients only ever add time)
    constexpr int NCAND = sizeof(cand) / sizeof(cand[0]), ROUNDS = 3;
    float tmin[NCAND];
    for (int i = 0; i < NCAND; ++i) tmin[i] = 1e30f;
    int rc = RLBM_OK;
    const int bx0 = c->tx, by0 = c->ty, bp0 = c->persistent;
    for (int round = 0; round < ROUNDS && rc == RLBM_OK; ++round) {
        for (int i = 0; i < NCAND && rc == RLBM_OK; ++i) {
            const int *t = cand[i];
            if (t[2] && !c->batch) continue;
            c->persistent = t[2];
            rc = configure(c, t[0], t[1]);
            if (rc) break;
            rc = launch_step(c, c->stream);   // warm-up
            if (rc) break;
            (void)hipEventRecord(e0, c->stream);
            for (int k = 0; k < trial_steps && rc == RLBM_OK; ++k) rc = launch_step(c, c->stream);
            (void)hipEventRecord(e1, c->stream);
            if (rc || hipEventSynchronize(e1) != hipSuccess) {
                rc = rc ? rc : RLBM_EHIP;
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tmin[i] = fminf(tmin[i], ms);
        }
    }
    int bx = bx0, by = by0, bp = bp0;
    float best = 1e30f;
    for (int i = 0; i < NCAND; ++i)
        if (tmin[i] < best) {
            best = tmin[i];
            bx = cand[i][0];
            by = cand[i][1];
            bp = cand[i][2];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the trial steps counted iterations too: restart the inversion counters (the
    // stream is idle here, and this call is never captured into a graph)
    if (!rc && c->p[0].collect_stats) {
        if (hipMemsetAsync(c->stats, 0, 2 * sizeof(unsigned long long), c->stream) != hipSuccess) rc = RLBM_EHIP;
        c->stat_steps = 0;
    }
    c->persistent = bp;
    if (!rc) rc = configure(c, bx, by);
    if (tile_x) *tile_x = bx;
    if (tile_y) *tile_y = by;
    return rc;
}

int rlbm_moments_grid(rlbm_ctx *c, int32_t g, const rlbm_out_fields *o) {
    if (!c || !o || g < 0 || g >= (int)c->base.size()) return RLBM_EINVAL;
    KArgs a = c->base[g];
    set_tiles(a, 32, 8);
    a.fin = c->cur ? c->p[g].f_b : c->p[g].f_a;
    a.o_n = o->n;
    a.o_eps = o->eps;
    a.o_theta = o->theta;
    a.o_z = o->z;
    a.o_ux = o->ux;
    a.o_uy = o->uy;
    a.o_qx = o->qx;
    a.o_qy = o->qy;
    double *const raw[9] = {o->N0, o->Nx, o->Ny, o->T00, o->T0x, o->T0y, o->Txx, o->Txy, o->Tyy};
    for (int i = 0; i < 9; ++i) a.o_mom[i] = raw[i];
    a.stats = nullptr;
    hipLaunchKernelGGL(pick(1, c->p[0].stats, c->p[0].precision), dim3(8 * a.per_xcd), dim3(256), 0, c->stream, a);
    if (hipGetLastError() != hipSuccess) return RLBM_EHIP;
    return rlbm_sync(c);
}

int rlbm_inversion_stats(rlbm_ctx *c, uint64_t *iterations, uint64_t *solves) {
    if (!c || !iterations || !solves) return RLBM_EINVAL;
    unsigned long long h[2] = {0, 0};
    if (hipMemcpyAsync(h, c->stats, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess) return RLBM_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return RLBM_EHIP;
    uint64_t cells = 0;
    for (const auto &a : c->base) cells += (uint64_t)a.plane;
    *iterations = h[0];
    *solves = (c->p[0].stats == RLBM_MJ) ? 0 : (uint64_t)c->stat_steps * cells;
    return RLBM_OK;
}

int rlbm_inversion_samples(rlbm_ctx *c, float *x, float *t) {
    if (!c || !x || !t) return RLBM_EINVAL;
    KArgs a = c->base[0];
    set_tiles(a, 32, 8);
    a.fin = c->cur ? c->p[0].f_b : c->p[0].f_a;
    a.o_mlx = x;
    a.o_mlt = t;
    a.stats = nullptr;
    hipLaunchKernelGGL(pick(1, c->p[0].stats, c->p[0].precision), dim3(8 * a.per_xcd), dim3(256), 0, c->stream, a);
    if (hipGetLastError() != hipSuccess) return RLBM_EHIP;
    return rlbm_sync(c);
}

int rlbm_moments(rlbm_ctx *c, const rlbm_out_fields *o) { return rlbm_moments_grid(c, 0, o); }

int rlbm_noneq_tensors(rlbm_ctx *c, int32_t g, double *pi_xx, double *pi_xxx, double *pi_xxxx, double *pi_xxxxx) {
    if (!c || g < 0 || g >= (int)c->base.size()) return RLBM_EINVAL;
    KArgs a = c->base[g];
    set_tiles(a, 32, 8);
    a.fin = c->cur ? c->p[g].f_b : c->p[g].f_a;
    a.o_pi[0] = pi_xx;
    a.o_pi[1] = pi_xxx;
    a.o_pi[2] = pi_xxxx;
    a.o_pi[3] = pi_xxxxx;
    a.stats = nullptr;
    hipLaunchKernelGGL(pick_noneq(c->p[0].stats, c->p[0].precision, c->p[0].order), dim3(8 * a.per_xcd), dim3(256), 0,
                       c->stream, a);
    if (hipGetLastError() != hipSuccess) return RLBM_EHIP;
    return rlbm_sync(c);
}

int rlbm_state_index(const rlbm_ctx *c) { return c ? c->cur : -1; }

int64_t rlbm_steps_done(const rlbm_ctx *c) { return c ? c->steps : -1; }

uint32_t rlbm_status(rlbm_ctx *c) {
    if (!c) return 0;
    unsigned h = 0;
    if (hipMemcpyAsync(&h, c->status, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream) != hipSuccess) return 0xffffffffu;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return 0xffffffffu;
    return h;
}

int rlbm_sync(rlbm_ctx *c) {
    if (!c) return RLBM_EINVAL;
    unsigned h = 0;
    if (hipMemcpyAsync(&h, c->status, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream) != hipSuccess) return RLBM_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return RLBM_EHIP;
    if (h) {
        if (hipMemsetAsync(c->status, 0, sizeof(unsigned), c->stream) != hipSuccess) return RLBM_EHIP;
        if (hipStreamSynchronize(c->stream) != hipSuccess) return RLBM_EHIP;
        return (h & RLBM_FLAG_NONFINITE) ? RLBM_ENONFINITE : RLBM_EDOMAIN;
    }
    return RLBM_OK;
}

void rlbm_free(rlbm_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    release(c);
}

const char *rlbm_strerror(int code) {
    switch (code) {
        case RLBM_OK: return "ok";
        case RLBM_EINVAL: return "invalid argument";
        case RLBM_EDOMAIN: return "state outside the method's domain (see rlbm_status bits)";
        case RLBM_EHIP: return "HIP runtime error";
        case RLBM_ENONFINITE: return "non-finite field";
        case RLBM_ENOTIMPL: return "not implemented by the library";
        default: return "unknown status code";
    }
}

}  // extern "C"
