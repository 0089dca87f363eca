// lbcm: hybrid central-moments / BGK lattice Boltzmann step for the coupled
// Cahn-Hilliard--Navier-Stokes equations (De Rosis, Saito, Kaneko, Abe, arXiv:1803.11345),
// written for MI355X (gfx950, wave64).
//
// Data layout in HBM.  Each population set is 9 planes [i][y][x] (x fastest).  Two copies
// ("pairs") of (f, g) live back to back in one workspace; a step reads pair `cur` and writes
// pair 1 - cur.  Streaming is done by pulling: the stored value P[i](x) is the post-collision
// population f*_i(x, t-1) at its origin node, and the post-streaming population of the paper,
// f_i(x, t) = f*_i(x - c_i, t - 1) (Eqs. (4)-(5)), is read at x - c_i.  With walls, a link that
// would come from outside is the same node's opposite post-collision value (half-way
// bounce-back).  Every reader of the state (step, fields, diagnostics) pulls.
//
// The step kernel (k_step) is one fused pass per time step.  A workgroup is one wave of 64
// lanes that owns a band of 64 columns and walks down a segment of rows.  For row y it
//   1. pulls g of row y+1 and sums it into phi(y+1) (plus the two halo columns), kept in a
//      4-row ring in LDS so that the 3x3 phi stencil of row y is available;
//   2. pulls f of row y;
//   3. evaluates grad phi and Lap phi (Eq. (12)), mu, p0, p~ and omega_rho;
//   4. collides f in central moments (Eqs. (15)-(17)) and g with BGK (Eq. (7));
//   5. stores f* and g* of row y at their own node (coalesced, non-temporal).
// Each g value is pulled once per segment (+2 rows of priming), so HBM traffic stays near the
// 36 values per node the step must move.
//
// The central-moment collision never forms the 9x9 matrix: the few pre-collision central
// moments it needs (k3, k4, k5) come from raw moments, and the post-collision populations are
// rebuilt by shifting the post-collision central moments back to raw moments (binomial
// expansion in v) and inverting the raw-moment map of D2Q9, which factorises into the 1-D map
// (m0, m1, m2) -> (f_0, f_+, f_-) = (m0 - m2, (m1 + m2)/2, (m2 - m1)/2) applied along x and y.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>

#include "lbcm.h"

namespace {

constexpr int kDefaultRows = 2;   // rows per tile (one wave row each)
constexpr int kDefaultWx = 8;     // 64-column waves across a tile
template <class S> constexpr int kMaxThreads = sizeof(S) == 8 ? 512 : 1024;
constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;
constexpr int kDiagFields = 7;

// ------------------------------------------------------------------------------------------
// storage.  f is stored shifted by the lattice weights, f_i - w_i (its deviation from the
// resting equilibrium rho = 1, v = 0), in every precision: the moments the collision needs are
// then formed from small numbers and a weak body force is not lost in the rounding of
// O(0.1) populations.  g is stored as is.

constexpr int kBufFlags = 0x00020000;  // word 3 of a raw buffer resource (gfx9 family)
#ifndef LBCM_F_LOAD_AUX
#define LBCM_F_LOAD_AUX 0
#endif
#ifndef LBCM_G_LOAD_AUX
#define LBCM_G_LOAD_AUX 0
#endif
#ifndef LBCM_STORE_AUX
#define LBCM_STORE_AUX 2
#endif
constexpr int kFLoad = LBCM_F_LOAD_AUX;  // cache policy of the f pulls
constexpr int kGLoad = LBCM_G_LOAD_AUX;  // cache policy of the g pulls (re-read as tile halos)
constexpr int kNT = LBCM_STORE_AUX;      // cache policy of the stores (2 = non-temporal)

using rsrc_t = __amdgpu_buffer_rsrc_t;

template <class S> __device__ __forceinline__ rsrc_t make_rsrc(const S *p, uint32_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<S *>(p), (short)0, (int)(n * (uint32_t)sizeof(S)),
                                             kBufFlags);
}

template <class S> struct Io;
template <> struct Io<double> {
    using R = double;
    using V2 = __attribute__((__vector_size__(2 * sizeof(unsigned int)))) unsigned int;
    static __device__ __forceinline__ R ld(const double *p) { return *p; }
    static __device__ __forceinline__ void st(double *p, R v) { __builtin_nontemporal_store(v, p); }
    template <int AUX> static __device__ __forceinline__ R bld(rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, AUX));
    }
    static __device__ __forceinline__ void bst(rsrc_t r, uint32_t voff, uint32_t soff, R v)
    {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, (int)voff, (int)soff, kNT);
    }
};
template <> struct Io<float> {
    using R = float;
    static __device__ __forceinline__ R ld(const float *p) { return *p; }
    static __device__ __forceinline__ void st(float *p, R v) { __builtin_nontemporal_store(v, p); }
    template <int AUX> static __device__ __forceinline__ R bld(rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, AUX));
    }
    static __device__ __forceinline__ void bst(rsrc_t r, uint32_t voff, uint32_t soff, R v)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)voff, (int)soff, kNT);
    }
};

// ------------------------------------------------------------------------------------------
// parameters

struct Geo {
    int nx, ny;
    uint32_t plane;  // nx * ny
    int wx;          // wave columns per tile (tile width 64 * wx)
    int rows;        // rows per tile (one wave row each)
    int nbands, nrows;  // tiles across and down
    int walls;
};

template <class R> struct Phys {
    R a, gamma, Gamma;
    R w_mid, w_half;  // omega_rho = w_mid + w_half * phi
    R w3, wphi;
    R hFx, hFy;       // half of the body force
    int k8_printed;
};

__constant__ double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
__constant__ int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int kCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__constant__ int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// ------------------------------------------------------------------------------------------
// pull of the 9 post-streaming populations of one row.  One buffer resource covers the 9 planes
// of a population set (pb bytes apart); the plane and the row y (uniform across the wave) go in
// the scalar offset of the buffer loads, and each lane supplies the byte offsets of its columns
// x, x - 1 and x + 1 (periodic).  With walls, a link that would
// come from behind a wall takes the node's own opposite post-collision value (the weights of
// opposite directions are equal, so this holds for the shifted f as well).

template <class S, bool WALLS, int AUX>
__device__ __forceinline__ void pull_row(rsrc_t P, uint32_t pb, int nx, int ny, int y, uint32_t cx,
                                         uint32_t cl, uint32_t cr, typename Io<S>::R v[9])
{
    using IO = Io<S>;
    int yd = y - 1;  // source row of the directions with c_y = +1 (2, 5, 6)
    int yu = y + 1;  // source row of the directions with c_y = -1 (4, 7, 8)
    bool bot = false, top = false;
    if (WALLS) {
        bot = yd < 0;
        top = yu >= ny;
    } else {
        if (yd < 0) yd += ny;
        if (yu >= ny) yu -= ny;
    }
    const uint32_t rowb = (uint32_t)nx * (uint32_t)sizeof(S);
    const uint32_t s0 = (uint32_t)y * rowb, sd = (uint32_t)yd * rowb, su = (uint32_t)yu * rowb;
    v[0] = IO::template bld<AUX>(P, cx, s0);
    v[1] = IO::template bld<AUX>(P, cl, pb + s0);
    v[3] = IO::template bld<AUX>(P, cr, 3 * pb + s0);
    if (WALLS && bot) {
        v[2] = IO::template bld<AUX>(P, cx, 4 * pb + s0);
        v[5] = IO::template bld<AUX>(P, cx, 7 * pb + s0);
        v[6] = IO::template bld<AUX>(P, cx, 8 * pb + s0);
    } else {
        v[2] = IO::template bld<AUX>(P, cx, 2 * pb + sd);
        v[5] = IO::template bld<AUX>(P, cl, 5 * pb + sd);
        v[6] = IO::template bld<AUX>(P, cr, 6 * pb + sd);
    }
    if (WALLS && top) {
        v[4] = IO::template bld<AUX>(P, cx, 2 * pb + s0);
        v[7] = IO::template bld<AUX>(P, cx, 5 * pb + s0);
        v[8] = IO::template bld<AUX>(P, cx, 6 * pb + s0);
    } else {
        v[4] = IO::template bld<AUX>(P, cx, 4 * pb + su);
        v[7] = IO::template bld<AUX>(P, cr, 7 * pb + su);
        v[8] = IO::template bld<AUX>(P, cl, 8 * pb + su);
    }
}

// The same pull for one arbitrary node (readers; plain global loads, any y per lane).
template <class S>
__device__ __forceinline__ void pull_node(const S *__restrict__ P, const Geo &geo, size_t n, double v[9])
{
    using IO = Io<S>;
    const int nx = geo.nx, ny = geo.ny;
    const int y = (int)(n / nx), x = (int)(n % nx);
    const int xl = x == 0 ? nx - 1 : x - 1, xr = x == nx - 1 ? 0 : x + 1;
    const size_t N = geo.plane;
    for (int i = 0; i < 9; ++i) {
        int xs = kCX[i] > 0 ? xl : (kCX[i] < 0 ? xr : x);
        int ys = y - kCY[i];
        int ii = i;
        if (ys < 0 || ys >= ny) {
            if (geo.walls) {
                ii = kOpp[i];
                xs = x;
                ys = y;
            } else {
                ys = ys < 0 ? ys + ny : ys - ny;
            }
        }
        v[i] = (double)IO::ld(P + (size_t)ii * N + (size_t)ys * nx + xs);
    }
}

template <class R> __device__ __forceinline__ R sum9(const R v[9])
{
    R s = v[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) s += v[i];
    return s;
}

// ------------------------------------------------------------------------------------------
// populations from central moments, in deviation form.  Input: rho - 1, rho, v and the central
// moments about v of the populations to build, c_pq = sum f (c_x - v_x)^p (c_y - v_y)^q, with
// c20, c02 and c22 given as deviations from their resting values 1/3, 1/3 and 1/9.  Output:
// f_i - w_i.  The central moments are shifted back to raw moments m_pq = sum f c_x^p c_y^q
// (binomial expansion in v), the raw moments of the weights are taken off, and the D2Q9
// raw-moment map is inverted as the tensor product of the 1-D map
// (m0, m1, m2) -> (f_0, f_+, f_-) = (m0 - m2, (m1 + m2)/2, (m2 - m1)/2).

template <class R>
__device__ __forceinline__ void from_central(R rd, R rho, R ux, R uy, R c10, R c01, R c20d, R c02d,
                                             R c11, R c21, R c12, R c22d, R out[9])
{
    const R third = (R)(1.0 / 3.0);
    const R c20 = c20d + third, c02 = c02d + third;
    const R ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
    const R m00 = rd;
    const R m10 = c10 + ux * rho;
    const R m01 = c01 + uy * rho;
    const R m20 = c20d + 2 * ux * c10 + ux2 * rho;
    const R m02 = c02d + 2 * uy * c01 + uy2 * rho;
    const R m11 = c11 + ux * c01 + uy * c10 + uxy * rho;
    const R m21 = c21 + 2 * ux * c11 + uy * c20 + ux2 * c01 + 2 * uxy * c10 + ux2 * uy * rho;
    const R m12 = c12 + 2 * uy * c11 + ux * c02 + uy2 * c10 + 2 * uxy * c01 + ux * uy2 * rho;
    const R m22 = c22d + 2 * ux * c12 + 2 * uy * c21 + ux2 * c02 + uy2 * c20 + 4 * uxy * c11 +
                  2 * ux * uy2 * c10 + 2 * ux2 * uy * c01 + ux2 * uy2 * rho;
    // inverse along x for each y-order q: h_q(0), h_q(+1), h_q(-1)
    const R h0z = m00 - m20, h0p = (R)0.5 * (m10 + m20), h0m = (R)0.5 * (m20 - m10);
    const R h1z = m01 - m21, h1p = (R)0.5 * (m11 + m21), h1m = (R)0.5 * (m21 - m11);
    const R h2z = m02 - m22, h2p = (R)0.5 * (m12 + m22), h2m = (R)0.5 * (m22 - m12);
    // inverse along y
    out[0] = h0z - h2z;             // ( 0,  0)
    out[1] = h0p - h2p;             // (+1,  0)
    out[2] = (R)0.5 * (h1z + h2z);  // ( 0, +1)
    out[3] = h0m - h2m;             // (-1,  0)
    out[4] = (R)0.5 * (h2z - h1z);  // ( 0, -1)
    out[5] = (R)0.5 * (h1p + h2p);  // (+1, +1)
    out[6] = (R)0.5 * (h1m + h2m);  // (-1, +1)
    out[7] = (R)0.5 * (h2m - h1m);  // (-1, -1)
    out[8] = (R)0.5 * (h2p - h1p);  // (+1, -1)
}

// Equilibrium central moments k3..k8 (the list ending in Eq. (16)), k3 and k8 as deviations
// from their resting values 2/3 and 1/9.  rd = rho - 1, ptd = p~ - 1/3.
template <class R>
__device__ __forceinline__ void eq_central(R rd, R rho, R ux, R uy, R ptd, R gamma, R dpx, R dpy, R surf,
                                           R &e3, R &e4, R &e5, R &e6, R &e7, R &e8)
{
    const R third = (R)(1.0 / 3.0);
    const R ux2 = ux * ux, uy2 = uy * uy;
    const R q = rd * third - ptd;  // rho c_s^2 - p~
    e3 = 2 * ptd;
    e4 = gamma * (dpx * dpx - dpy * dpy);
    e5 = gamma * dpx * dpy;
    e6 = -(R)0.5 * uy * e4 - 2 * ux * e5 - rho * uy * ux2 + uy * q;
    e7 = (R)0.5 * ux * e4 - 2 * uy * e5 - rho * ux * uy2 + ux * q;
    e8 = ptd * third - (ux2 + uy2) * q + 3 * rho * ux2 * uy2 - (R)(1.0 / 6.0) * gamma * surf +
         (R)0.5 * e4 * (uy2 - ux2) + 4 * ux * uy * e5;
}

// g equilibrium (Eqs. (9)-(10)): w_i [Gamma mu + phi (3 c.v + 9/2 (c.v)^2 - 3/2 v^2)], i >= 1,
// and g0 = phi - sum_{i>=1}, which is phi - (5/9) Gamma mu - (2/3) phi v^2.
template <class R>
__device__ __forceinline__ void g_equilibrium(R phi, R gmu, R ux, R uy, R out[9])
{
    const R w1 = (R)(1.0 / 9.0), w5 = (R)(1.0 / 36.0);
    const R u2 = ux * ux + uy * uy;
    const R base = gmu - (R)1.5 * phi * u2;
    const R ax = 3 * phi * ux, ay = 3 * phi * uy;
    const R qx = (R)4.5 * phi * ux * ux, qy = (R)4.5 * phi * uy * uy;
    const R sp = ux + uy, sm = ux - uy;
    const R a5 = 3 * phi * sp, a6 = 3 * phi * sm;  // projections on (+1,+1) and (+1,-1)
    const R q5 = (R)4.5 * phi * sp * sp, q6 = (R)4.5 * phi * sm * sm;
    out[1] = w1 * (base + ax + qx);
    out[3] = w1 * (base - ax + qx);
    out[2] = w1 * (base + ay + qy);
    out[4] = w1 * (base - ay + qy);
    out[5] = w5 * (base + a5 + q5);
    out[7] = w5 * (base - a5 + q5);
    out[8] = w5 * (base + a6 + q6);
    out[6] = w5 * (base - a6 + q6);
    out[0] = phi - (R)(5.0 / 9.0) * gmu - (R)(2.0 / 3.0) * phi * u2;
}

// ------------------------------------------------------------------------------------------
// one node: central-moment collision of f (Eq. (17)) and BGK of g (Eq. (7)).
// f and fo hold f_i - w_i.

template <class R> struct Rcp;
template <> struct Rcp<double> {
    static __device__ __forceinline__ double of(double v) { return 1.0 / v; }
};
template <> struct Rcp<float> {
    static __device__ __forceinline__ float of(float v) { return __builtin_amdgcn_rcpf(v); }  // 1 ulp
};

template <class R, bool FORCE>
__device__ __forceinline__ void collide_node(const R f[9], const R g[9], R phi, R dpx, R dpy,
                                             R lap, const Phys<R> &c, R fo[9], R go[9],
                                             R &rho_out)
{
    const R third = (R)(1.0 / 3.0);
    const R rd = sum9(f);  // rho - 1
    const R rho = 1 + rd;
    const R jx = (f[1] + f[5] + f[8]) - (f[3] + f[6] + f[7]);
    const R jy = (f[2] + f[5] + f[6]) - (f[4] + f[7] + f[8]);
    const R irho = Rcp<R>::of(rho);
    const R hFx = FORCE ? c.hFx : (R)0, hFy = FORCE ? c.hFy : (R)0;
    const R ux = (jx + hFx) * irho, uy = (jy + hFy) * irho;
    rho_out = rho;

    // pre-collision second-order central moments about v (m10 = rho ux - F_x/2); the weights'
    // share 1/3 of the diagonal ones cancels against the same share of the equilibria
    const R sxx = (f[1] + f[3]) + (f[5] + f[6]) + (f[7] + f[8]);
    const R syy = (f[2] + f[4]) + (f[5] + f[6]) + (f[7] + f[8]);
    const R sxy = (f[5] - f[6]) + (f[7] - f[8]);
    R kxx = sxx - rho * ux * ux;
    R kyy = syy - rho * uy * uy;
    R kxy = sxy - rho * ux * uy;
    if (FORCE) {
        kxx += 2 * ux * hFx;
        kyy += 2 * uy * hFy;
        kxy += ux * hFy + uy * hFx;
    }
    const R k3 = kxx + kyy, k4 = kxx - kyy, k5 = kxy;

    // thermodynamics: mu, p~ - 1/3, omega_rho
    const R phi2 = phi * phi;
    const R mu = c.a * phi * (phi2 - 1) - c.gamma * lap;
    const R ptd = rd * third + c.a * phi2 * ((R)0.75 * phi2 - (R)0.5) - c.gamma * phi * lap;
    const R wr = c.w_mid + c.w_half * phi;
    const R surf = c.k8_printed ? lap : dpx * dpx + dpy * dpy;

    R e3, e4, e5, e6, e7, e8;
    eq_central(rd, rho, ux, uy, ptd, c.gamma, dpx, dpy, surf, e3, e4, e5, e6, e7, e8);

    const R s3 = k3 + c.w3 * (e3 - k3);
    const R s4 = k4 + wr * (e4 - k4);
    const R s5 = k5 + wr * (e5 - k5);
    R s6 = e6, s7 = e7, s8 = e8;
    if (FORCE) {
        // central moments of Guo's forcing term; k6..k8 relax at rate 1, weight 1/2
        const R Fx = 2 * hFx, Fy = 2 * hFy;
        s6 += (R)0.5 * (Fy * (third - ux * ux) - 2 * Fx * ux * uy);
        s7 += (R)0.5 * (Fx * (third - uy * uy) - 2 * Fy * ux * uy);
        s8 += 2 * ux * uy * (Fx * uy + Fy * ux);
    }
    from_central(rd, rho, ux, uy, hFx, hFy, (R)0.5 * (s3 + s4), (R)0.5 * (s3 - s4), s5, s6, s7, s8, fo);

    R geq[9];
    g_equilibrium(phi, c.Gamma * mu, ux, uy, geq);
#pragma unroll
    for (int i = 0; i < 9; ++i) go[i] = g[i] + c.wphi * (geq[i] - g[i]);
}

// ------------------------------------------------------------------------------------------
// the step kernel.  A workgroup owns a tile of 64 * wx columns by rows_t rows; each of its waves
// owns one 64-column row segment.  Every wave pulls f and g of its own nodes, sums phi into an
// LDS tile with a one-node halo, and the halo is filled by the same pulls one node further out:
// the waves of the first and last tile row also pull g of the rows above and below, and lanes 0
// and 1 of the first wave column pull the two halo columns.  One barrier later every node reads
// its 3x3 phi stencil from LDS, collides and stores f*, g* at its own node (non-temporal).
//
// Every load of a workgroup is issued before its barrier, and workgroups are dispatched in
// row-major tile order, so the waves resident at any moment cover a compact band of rows: the
// HBM sees a few long streams per plane instead of many short ones.  The halo re-reads (one
// extra g row per tile row-pair, two columns per tile) are served by L2 and the MALL.
// Workgroups are dealt round-robin to the 8 XCDs; with a multiple of 8 tiles per tile row the
// tiles above and below a tile land on its XCD, so its halo rows are hits in the same L2.

template <class S, bool WALLS, bool FORCE>
__global__ __launch_bounds__(kMaxThreads<S>) void k_step(const S *__restrict__ fa, const S *__restrict__ ga,
                                                         S *__restrict__ fb, S *__restrict__ gb, Geo geo,
                                                         Phys<typename Io<S>::R> c, int *__restrict__ flag)
{
    using R = typename Io<S>::R;
    using IO = Io<S>;
    constexpr uint32_t E = sizeof(S);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    R *phs = reinterpret_cast<R *>(lds_raw);  // [rows_t + 2][ldw]

    const int nx = geo.nx, ny = geo.ny;
    const int wx = geo.wx, rows_t = geo.rows;
    const int ldw = 64 * wx + 2;
    const int lane = threadIdx.x & 63;
    // wave index made explicitly uniform, so that the row offsets stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wc = wave % wx, wr = wave / wx;  // wave column and row inside the tile
    const int band = blockIdx.x % geo.nbands, rg = blockIdx.x / geo.nbands;
    const int X0 = band * 64 * wx;
    const int X1 = min(X0 + 64 * wx, nx);
    const int y0 = rg * rows_t;
    const int y1 = min(y0 + rows_t, ny);
    const int y = y0 + wr;
    const bool row_ok = y < y1;                       // uniform per wave
    const int xr_ = X0 + wc * 64 + lane;
    const bool col_ok = xr_ < X1;
    const bool valid = row_ok && col_ok;
    const int x = col_ok ? xr_ : X1 - 1;              // clamped for addressing
    const int yy = row_ok ? y : y1 - 1;
    const int xl = x == 0 ? nx - 1 : x - 1;
    const int xr = x == nx - 1 ? 0 : x + 1;
    const uint32_t cx = (uint32_t)x * E, cl = (uint32_t)xl * E, cr = (uint32_t)xr * E;
    const uint32_t pb = geo.plane * E;
    const rsrc_t rfa = make_rsrc(fa, 9 * geo.plane), rga = make_rsrc(ga, 9 * geo.plane);
    const rsrc_t rfb = make_rsrc(fb, 9 * geo.plane), rgb = make_rsrc(gb, 9 * geo.plane);
    const int slot = wc * 64 + lane + 1;              // LDS column of this lane
    const int last = y1 - y0 - 1;                     // last valid tile row

    // own populations; the loads go out at raised wave priority so that the memory pipeline of
    // the CU keeps being fed while other workgroups compute
    __builtin_amdgcn_s_setprio(3);
    R g[9], f[9];
    pull_row<S, WALLS, kFLoad>(rfa, pb, nx, ny, yy, cx, cl, cr, f);
    pull_row<S, WALLS, kGLoad>(rga, pb, nx, ny, yy, cx, cl, cr, g);
    const R phi_own = sum9(g);
    if (valid) phs[(wr + 1) * ldw + slot] = phi_own;

    // halo rows: the first tile row fetches the row above, the last valid one the row below
    auto halo_row = [&](int hy, int hslot_row, int own_slot_row) {
        if (WALLS && (hy < 0 || hy >= ny)) {  // ghost row behind a wall: mirror
            if (col_ok) phs[hslot_row * ldw + slot] = phi_own;
            (void)own_slot_row;
        } else {
            R h[9];
            pull_row<S, WALLS, kGLoad>(rga, pb, nx, ny, hy < 0 ? hy + ny : (hy >= ny ? hy - ny : hy), cx, cl, cr, h);
            if (col_ok) phs[hslot_row * ldw + slot] = sum9(h);
        }
    };
    if (wr == 0) halo_row(y0 - 1, 0, 1);
    if (wr == last) halo_row(y1, last + 2, last + 1);

    // halo columns (x = X0 - 1 on lane 0, x = X1 on lane 1) for this wave's row and, on the
    // first / last tile row, the corner rows
    if (wc == 0 && lane < 2 && wr <= last) {
        const int hx = lane == 0 ? (X0 == 0 ? nx - 1 : X0 - 1) : (X1 == nx ? 0 : X1);
        const int hxl = hx == 0 ? nx - 1 : hx - 1, hxr = hx == nx - 1 ? 0 : hx + 1;
        const uint32_t hcx = (uint32_t)hx * E, hcl = (uint32_t)hxl * E, hcr = (uint32_t)hxr * E;
        const int hs = lane == 0 ? 0 : X1 - X0 + 1;
        R h[9];
        pull_row<S, WALLS, kGLoad>(rga, pb, nx, ny, y, hcx, hcl, hcr, h);
        const R ph = sum9(h);
        phs[(wr + 1) * ldw + hs] = ph;
        for (int side = 0; side < 2; ++side) {
            if (side == 0 && wr != 0) continue;
            if (side == 1 && wr != last) continue;
            const int hy = side == 0 ? y0 - 1 : y1;
            const int srow = side == 0 ? 0 : last + 2;
            if (WALLS && (hy < 0 || hy >= ny)) {
                phs[srow * ldw + hs] = ph;
            } else {
                R h2[9];
                pull_row<S, WALLS, kGLoad>(rga, pb, nx, ny, hy < 0 ? hy + ny : (hy >= ny ? hy - ny : hy), hcx, hcl, hcr, h2);
                phs[srow * ldw + hs] = sum9(h2);
            }
        }
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    if (!row_ok) return;

    const R *rS = phs + wr * ldw, *rC = phs + (wr + 1) * ldw, *rN = phs + (wr + 2) * ldw;
    const R pS = rS[slot], pSW = rS[slot - 1], pSE = rS[slot + 1];
    const R pC = rC[slot], pW = rC[slot - 1], pE = rC[slot + 1];
    const R pN = rN[slot], pNW = rN[slot - 1], pNE = rN[slot + 1];
    const R dpx = ((R)4 * (pE - pW) + (pNE - pNW) + (pSE - pSW)) * (R)(1.0 / 12.0);
    const R dpy = ((R)4 * (pN - pS) + (pNE - pSE) + (pNW - pSW)) * (R)(1.0 / 12.0);
    const R lap = ((R)4 * ((pE + pW) + (pN + pS)) + ((pNE + pNW) + (pSE + pSW)) - (R)20 * pC) *
                  (R)(1.0 / 6.0);

    R fo[9], go[9], rho;
    collide_node<R, FORCE>(f, g, pC, dpx, dpy, lap, c, fo, go, rho);
    const bool bad = !(std::isfinite(rho) && std::isfinite(pC)) && col_ok;
    if (__any(bad) && lane == 0) atomicOr(flag, 1);

    if (col_ok) {
        const uint32_t so = (uint32_t)y * (uint32_t)nx * E;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            IO::bst(rfb, cx, i * pb + so, fo[i]);
            IO::bst(rgb, cx, i * pb + so, go[i]);
        }
    }
}

// ------------------------------------------------------------------------------------------
// initialisation.  k_equilibria computes the equilibria of the given macroscopic planes into
// a post-streaming state (9 + 9 planes, node-local); k_unstream stores them in pull layout:
// P[i](z) = F[i](z + c_i), or F[opp(i)](z) where z + c_i is behind a wall.

__device__ __forceinline__ double plane_at(const double *p, int nx, int ny, bool walls, int x, int y)
{
    x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
    if (walls) {
        y = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
    } else {
        y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
    }
    return p[(size_t)y * nx + x];
}

template <class S>
__global__ void k_equilibria(const double *__restrict__ phi0, const double *__restrict__ rho0,
                             const double *__restrict__ ux0, const double *__restrict__ uy0,
                             S *__restrict__ F, S *__restrict__ G, Geo geo,
                             Phys<typename Io<S>::R> c)
{
    using R = typename Io<S>::R;
    const int nx = geo.nx, ny = geo.ny;
    const size_t N = geo.plane;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(n / nx), x = (int)(n % nx);
        const bool wl = geo.walls != 0;
        double nb[3][3];
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) nb[dy + 1][dx + 1] = plane_at(phi0, nx, ny, wl, x + dx, y + dy);
        const R pC = (R)nb[1][1], pE = (R)nb[1][2], pW = (R)nb[1][0], pN = (R)nb[2][1], pS = (R)nb[0][1];
        const R pNE = (R)nb[2][2], pNW = (R)nb[2][0], pSE = (R)nb[0][2], pSW = (R)nb[0][0];
        const R dpx = ((R)4 * (pE - pW) + (pNE - pNW) + (pSE - pSW)) * (R)(1.0 / 12.0);
        const R dpy = ((R)4 * (pN - pS) + (pNE - pSE) + (pNW - pSW)) * (R)(1.0 / 12.0);
        const R lap = ((R)4 * ((pE + pW) + (pN + pS)) + ((pNE + pNW) + (pSE + pSW)) - (R)20 * pC) *
                      (R)(1.0 / 6.0);
        const R rd = rho0 ? (R)(rho0[n] - 1.0) : (R)0;
        const R rho = 1 + rd;
        const R ux = ux0 ? (R)ux0[n] : (R)0, uy = uy0 ? (R)uy0[n] : (R)0;
        const R phi = pC;
        const R phi2 = phi * phi;
        const R mu = c.a * phi * (phi2 - 1) - c.gamma * lap;
        const R ptd = rd * (R)(1.0 / 3.0) + c.a * phi2 * ((R)0.75 * phi2 - (R)0.5) - c.gamma * phi * lap;
        const R surf = c.k8_printed ? lap : dpx * dpx + dpy * dpy;
        R e3, e4, e5, e6, e7, e8;
        eq_central(rd, rho, ux, uy, ptd, c.gamma, dpx, dpy, surf, e3, e4, e5, e6, e7, e8);
        R fe[9], ge[9];
        from_central(rd, rho, ux, uy, (R)0, (R)0, (R)0.5 * (e3 + e4), (R)0.5 * (e3 - e4), e5, e6, e7, e8, fe);
        g_equilibrium(phi, c.Gamma * mu, ux, uy, ge);
        for (int i = 0; i < 9; ++i) {
            Io<S>::st(F + i * N + n, (S)fe[i]);
            Io<S>::st(G + i * N + n, (S)ge[i]);
        }
    }
}

template <class S>
__global__ void k_unstream(const S *__restrict__ F, S *__restrict__ P, Geo geo)
{
    const int nx = geo.nx, ny = geo.ny;
    const size_t N = geo.plane;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < 9 * N;
         t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / N);
        const size_t n = t % N;
        const int y = (int)(n / nx), x = (int)(n % nx);
        int xs = x + kCX[i], ys = y + kCY[i];
        xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
        size_t src;
        if (ys < 0 || ys >= ny) {
            if (geo.walls) {
                src = (size_t)kOpp[i] * N + n;
            } else {
                ys = ys < 0 ? ys + ny : ys - ny;
                src = (size_t)i * N + (size_t)ys * nx + xs;
            }
        } else {
            src = (size_t)i * N + (size_t)ys * nx + xs;
        }
        P[t] = F[src];
    }
}

// ------------------------------------------------------------------------------------------
// readers: post-streaming populations, macroscopic fields and FP64 reductions (in double).

template <class S>
__global__ void k_fields(const S *__restrict__ f, const S *__restrict__ g, Geo geo, double a,
                         double hFx, double hFy, double *phi, double *rho, double *ux, double *uy,
                         double *p0)
{
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < geo.plane;
         n += (size_t)gridDim.x * blockDim.x) {
        double fv[9], gv[9];
        pull_node<S>(f, geo, n, fv);
        pull_node<S>(g, geo, n, gv);
        const double r = 1.0 + sum9(fv);
        const double ph = sum9(gv);
        const double jx = (fv[1] + fv[5] + fv[8]) - (fv[3] + fv[6] + fv[7]);
        const double jy = (fv[2] + fv[5] + fv[6]) - (fv[4] + fv[7] + fv[8]);
        if (phi) phi[n] = ph;
        if (rho) rho[n] = r;
        if (ux) ux[n] = (jx + hFx) / r;
        if (uy) uy[n] = (jy + hFy) / r;
        if (p0) p0[n] = r / 3.0 + a * (-0.5 * ph * ph + 0.75 * ph * ph * ph * ph);
    }
}

// one post-streaming population plane (which = 0..8: f_i, 9..17: g_i) as FP64
template <class S>
__global__ void k_population(const S *__restrict__ f, const S *__restrict__ g, Geo geo, int which,
                             double *out)
{
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < geo.plane;
         n += (size_t)gridDim.x * blockDim.x) {
        double v[9];
        pull_node<S>(which < 9 ? f : g, geo, n, v);
        out[n] = which < 9 ? v[which] + kW[which] : v[which - 9];
    }
}

template <class S>
__global__ __launch_bounds__(kReduceThreads) void k_diag(const S *__restrict__ f,
                                                         const S *__restrict__ g, Geo geo,
                                                         double hFx, double hFy, double *partial)
{
    double acc[kDiagFields] = {0, 0, 0, 0, 0, 0, 0};  // phi, |phi|, rho, jx, jy, max|u|, nonfinite
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < geo.plane;
         n += (size_t)gridDim.x * blockDim.x) {
        double fv[9], gv[9];
        pull_node<S>(f, geo, n, fv);
        pull_node<S>(g, geo, n, gv);
        const double r = 1.0 + sum9(fv), ph = sum9(gv);
        const double jx = (fv[1] + fv[5] + fv[8]) - (fv[3] + fv[6] + fv[7]) + hFx;
        const double jy = (fv[2] + fv[5] + fv[6]) - (fv[4] + fv[7] + fv[8]) + hFy;
        if (!(std::isfinite(r) && std::isfinite(ph))) {
            acc[6] += 1;
            continue;
        }
        acc[0] += ph;
        acc[1] += fabs(ph);
        acc[2] += r;
        acc[3] += jx;
        acc[4] += jy;
        acc[5] = fmax(acc[5], sqrt(jx * jx + jy * jy) / r);
    }
    __shared__ double red[kDiagFields][kReduceThreads];
    for (int k = 0; k < kDiagFields; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kReduceThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < kDiagFields; ++k)
                red[k][threadIdx.x] = k == 5 ? fmax(red[k][threadIdx.x], red[k][threadIdx.x + s])
                                             : red[k][threadIdx.x] + red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < kDiagFields) partial[blockIdx.x * kDiagFields + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kReduceThreads) void k_diag_finish(const double *partial, int nblocks,
                                                                double *out)
{
    __shared__ double red[kDiagFields][kReduceThreads];
    double acc[kDiagFields] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += kReduceThreads)
        for (int k = 0; k < kDiagFields; ++k) {
            const double v = partial[b * kDiagFields + k];
            acc[k] = k == 5 ? fmax(acc[k], v) : acc[k] + v;
        }
    for (int k = 0; k < kDiagFields; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kReduceThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < kDiagFields; ++k)
                red[k][threadIdx.x] = k == 5 ? fmax(red[k][threadIdx.x], red[k][threadIdx.x + s])
                                             : red[k][threadIdx.x] + red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < kDiagFields) out[threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_clear_int(int *p) { *p = 0; }

}  // namespace

// ==========================================================================================
// host side

struct lbcm_handle {
    lbcm_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    size_t elem = 0;         // bytes per stored value
    size_t pair_bytes = 0;   // bytes of one (f, g) pair
    char *ws = nullptr;      // workspace base
    bool owns_ws = false;
    int cur = 0;             // pair holding the current state
    bool ready = false;
    int64_t step = 0;
    double *diag_partial = nullptr;
    double *diag_out = nullptr;
    int *flag = nullptr;
    std::string err;
};

namespace {

std::string g_create_error;

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

size_t elem_bytes(int precision)
{
    switch (precision) {
    case LBCM_FP64: return 8;
    case LBCM_FP32: return 4;
    default: return 0;
    }
}

const char *check_params(const lbcm_params *p)
{
    if (!p) return "params is NULL";
    if (p->nx < 1 || p->ny < 1) return "nx and ny must be >= 1";
    if (p->bc_y != LBCM_BC_PERIODIC && p->bc_y != LBCM_BC_WALLS) return "bc_y must be 0 or 1";
    if (elem_bytes(p->precision) == 0) return "unsupported precision";
    const double N = (double)p->nx * (double)p->ny;
    if (9.0 * N * (double)elem_bytes(p->precision) > 4294967295.0)
        return "lattice too large: one population set (9 planes) must stay below 4 GiB";
    if (!(p->nu_l > 0) || !(p->nu_g > 0)) return "viscosities must be > 0";
    if (!(p->mobility > 0) || !(p->Gamma > 0)) return "mobility and Gamma must be > 0";
    if (!(p->omega3 > 0 && p->omega3 < 2)) return "omega3 must lie in (0, 2)";
    if (!std::isfinite(p->a) || !std::isfinite(p->gamma) || !std::isfinite(p->force_x) ||
        !std::isfinite(p->force_y))
        return "a, gamma and the force must be finite";
    if (p->k8_variant != 0 && p->k8_variant != 1) return "k8_variant must be 0 or 1";
    if (p->check_every < 0) return "check_every must be >= 0";
    if (p->tile_rows < 0 || p->tile_wx < 0) return "tile_rows and tile_wx must be >= 0";
    return nullptr;
}

size_t pair_bytes_of(const lbcm_params *p)
{
    return align_up(18 * (size_t)p->nx * (size_t)p->ny * elem_bytes(p->precision));
}

size_t tail_bytes() { return align_up(kReduceBlocks * kDiagFields * sizeof(double)) + align_up(kDiagFields * sizeof(double)) + kAlign; }

int fail(lbcm_handle *h, int code, const std::string &msg)
{
    if (h) h->err = msg;
    return code;
}

#define HIP_TRY(h, call)                                                                      \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(h, LBCM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

template <class R> Phys<R> make_phys(const lbcm_params &p)
{
    const double cs2 = 1.0 / 3.0;
    const double wl = 1.0 / (p.nu_l / cs2 + 0.5), wg = 1.0 / (p.nu_g / cs2 + 0.5);
    Phys<R> c;
    c.a = (R)p.a;
    c.gamma = (R)p.gamma;
    c.Gamma = (R)p.Gamma;
    c.w_mid = (R)(0.5 * (wl + wg));
    c.w_half = (R)(0.5 * (wl - wg));
    c.w3 = (R)p.omega3;
    c.wphi = (R)(1.0 / (p.mobility / (p.Gamma * cs2) + 0.5));
    c.hFx = (R)(0.5 * p.force_x);
    c.hFy = (R)(0.5 * p.force_y);
    c.k8_printed = p.k8_variant;
    return c;
}

Geo make_geo(const lbcm_params &p)
{
    Geo g;
    g.nx = p.nx;
    g.ny = p.ny;
    g.plane = (uint32_t)((size_t)p.nx * p.ny);
    const int max_waves = (p.precision == LBCM_FP64 ? 512 : 1024) / 64;
    const int need = (p.nx + 63) / 64;
    g.wx = p.tile_wx > 0 ? p.tile_wx : kDefaultWx;
    if (g.wx > need) g.wx = need;
    if (g.wx > max_waves) g.wx = max_waves;
    int rows = p.tile_rows > 0 ? p.tile_rows : (p.precision == LBCM_FP64 ? 2 : kDefaultRows);
    if (rows > max_waves / g.wx) rows = max_waves / g.wx;
    if (rows > p.ny) rows = p.ny;
    g.rows = rows;
    g.nbands = (p.nx + 64 * g.wx - 1) / (64 * g.wx);
    g.nrows = (p.ny + g.rows - 1) / g.rows;
    g.walls = p.bc_y;
    return g;
}

template <class S> S *pop(lbcm_handle *h, int pair, int set)  // set 0 = f, 1 = g
{
    return reinterpret_cast<S *>(h->ws + (size_t)pair * h->pair_bytes) + (size_t)set * 9 * h->p.nx * (size_t)h->p.ny;
}

int grid_for(size_t n, int threads)
{
    size_t b = (n + threads - 1) / threads;
    if (b > 65535) b = 65535;
    if (b < 1) b = 1;
    return (int)b;
}

template <class S> int launch_steps(lbcm_handle *h, int64_t nsteps)
{
    using R = typename Io<S>::R;
    const Geo geo = make_geo(h->p);
    const Phys<R> c = make_phys<R>(h->p);
    const bool walls = h->p.bc_y == LBCM_BC_WALLS;
    const bool force = h->p.force_x != 0 || h->p.force_y != 0;
    const int64_t nblk = (int64_t)geo.nbands * geo.nrows;
    if (nblk > 0x7fffffff) return fail(h, LBCM_EINVAL, "too many tiles");
    const dim3 grid((unsigned)nblk), block(64 * geo.wx * geo.rows);
    const size_t lds = (size_t)(geo.rows + 2) * (64 * geo.wx + 2) * sizeof(R);
    for (int64_t s = 0; s < nsteps; ++s) {
        const S *fa = pop<S>(h, h->cur, 0), *ga = pop<S>(h, h->cur, 1);
        S *fb = pop<S>(h, 1 - h->cur, 0), *gb = pop<S>(h, 1 - h->cur, 1);
        if (walls) {
            if (force) hipLaunchKernelGGL((k_step<S, true, true>), grid, block, lds, h->stream, fa, ga, fb, gb, geo, c, h->flag);
            else hipLaunchKernelGGL((k_step<S, true, false>), grid, block, lds, h->stream, fa, ga, fb, gb, geo, c, h->flag);
        } else {
            if (force) hipLaunchKernelGGL((k_step<S, false, true>), grid, block, lds, h->stream, fa, ga, fb, gb, geo, c, h->flag);
            else hipLaunchKernelGGL((k_step<S, false, false>), grid, block, lds, h->stream, fa, ga, fb, gb, geo, c, h->flag);
        }
        HIP_TRY(h, hipGetLastError());
        h->cur = 1 - h->cur;
        h->step += 1;
        if (h->p.check_every > 0 && ((s + 1) % h->p.check_every == 0 || s + 1 == nsteps)) {
            int flag = 0;
            HIP_TRY(h, hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            if (flag) return fail(h, LBCM_EDIVERGED, "non-finite rho or phi detected at step " + std::to_string(h->step));
        }
    }
    return LBCM_OK;
}

template <class S>
int do_init(lbcm_handle *h, const double *phi0, const double *rho0, const double *ux0, const double *uy0)
{
    using R = typename Io<S>::R;
    const Geo geo = make_geo(h->p);
    const Phys<R> c = make_phys<R>(h->p);
    // equilibria into the spare pair, then un-stream into pair 0
    S *F = pop<S>(h, 1, 0), *G = pop<S>(h, 1, 1);
    const int gb = grid_for(geo.plane, 256);
    hipLaunchKernelGGL((k_equilibria<S>), dim3(gb), dim3(256), 0, h->stream, phi0, rho0, ux0, uy0, F, G, geo, c);
    HIP_TRY(h, hipGetLastError());
    const int gu = grid_for(9 * (size_t)geo.plane, 256);
    hipLaunchKernelGGL((k_unstream<S>), dim3(gu), dim3(256), 0, h->stream, F, pop<S>(h, 0, 0), geo);
    HIP_TRY(h, hipGetLastError());
    hipLaunchKernelGGL((k_unstream<S>), dim3(gu), dim3(256), 0, h->stream, G, pop<S>(h, 0, 1), geo);
    HIP_TRY(h, hipGetLastError());
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(1), 0, h->stream, h->flag);
    HIP_TRY(h, hipGetLastError());
    h->cur = 0;
    h->step = 0;
    h->ready = true;
    return LBCM_OK;
}

template <class S>
int do_fields(lbcm_handle *h, double *phi, double *rho, double *ux, double *uy, double *p0)
{
    const Geo geo = make_geo(h->p);
    const int gb = grid_for(geo.plane, 256);
    const S *f = pop<S>(h, h->cur, 0), *g = pop<S>(h, h->cur, 1);
    hipLaunchKernelGGL((k_fields<S>), dim3(gb), dim3(256), 0, h->stream, f, g, geo, h->p.a,
                       0.5 * h->p.force_x, 0.5 * h->p.force_y, phi, rho, ux, uy, p0);
    HIP_TRY(h, hipGetLastError());
    return LBCM_OK;
}

template <class S> int do_population(lbcm_handle *h, int which, double *out)
{
    const Geo geo = make_geo(h->p);
    const int gb = grid_for(geo.plane, 256);
    const S *f = pop<S>(h, h->cur, 0), *g = pop<S>(h, h->cur, 1);
    hipLaunchKernelGGL((k_population<S>), dim3(gb), dim3(256), 0, h->stream, f, g, geo, which, out);
    HIP_TRY(h, hipGetLastError());
    return LBCM_OK;
}

template <class S> int do_diag(lbcm_handle *h)
{
    const Geo geo = make_geo(h->p);
    const S *f = pop<S>(h, h->cur, 0), *g = pop<S>(h, h->cur, 1);
    hipLaunchKernelGGL((k_diag<S>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, h->stream, f, g, geo,
                       0.5 * h->p.force_x, 0.5 * h->p.force_y, h->diag_partial);
    HIP_TRY(h, hipGetLastError());
    hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(kReduceThreads), 0, h->stream, h->diag_partial, kReduceBlocks, h->diag_out);
    HIP_TRY(h, hipGetLastError());
    return LBCM_OK;
}

// host-side dispatch on the storage precision
template <class Fn> int dispatch(lbcm_handle *h, Fn &&fn)
{
    switch (h->p.precision) {
    case LBCM_FP64: return fn((double *)nullptr);
    case LBCM_FP32: return fn((float *)nullptr);
    default: return fail(h, LBCM_EINVAL, "unsupported precision");
    }
}

}  // namespace

extern "C" {

size_t lbcm_workspace_size(const lbcm_params *p)
{
    if (check_params(p)) return 0;
    return 2 * pair_bytes_of(p) + tail_bytes();
}

int lbcm_create(const lbcm_params *p, lbcm_handle **out)
{
    if (!out) {
        g_create_error = "out is NULL";
        return LBCM_EINVAL;
    }
    *out = nullptr;
    if (const char *m = check_params(p)) {
        g_create_error = m;
        return LBCM_EINVAL;
    }
    const size_t need = lbcm_workspace_size(p);
    if (p->workspace) {
        if (p->workspace_bytes < need) {
            g_create_error = "workspace too small: need " + std::to_string(need) + " bytes";
            return LBCM_EINVAL;
        }
        if ((uintptr_t)p->workspace % kAlign) {
            g_create_error = "workspace must be 256-byte aligned";
            return LBCM_EINVAL;
        }
    }
    lbcm_handle *h = new (std::nothrow) lbcm_handle();
    if (!h) {
        g_create_error = "out of host memory";
        return LBCM_ENOMEM;
    }
    h->p = *p;
    h->stream = (hipStream_t)p->stream;
    h->elem = elem_bytes(p->precision);
    h->pair_bytes = pair_bytes_of(p);
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipGetDevice: ") + hipGetErrorString(e);
        delete h;
        return LBCM_EHIP;
    }
    if (p->workspace) {
        h->ws = (char *)p->workspace;
    } else {
        e = hipMalloc((void **)&h->ws, need);
        if (e != hipSuccess) {
            g_create_error = std::string("hipMalloc(") + std::to_string(need) + "): " + hipGetErrorString(e);
            (void)hipGetLastError();
            delete h;
            return e == hipErrorOutOfMemory ? LBCM_ENOMEM : LBCM_EHIP;
        }
        h->owns_ws = true;
    }
    char *tail = h->ws + 2 * h->pair_bytes;
    h->diag_partial = (double *)tail;
    tail += align_up(kReduceBlocks * kDiagFields * sizeof(double));
    h->diag_out = (double *)tail;
    tail += align_up(kDiagFields * sizeof(double));
    h->flag = (int *)tail;
    *out = h;
    return LBCM_OK;
}

int lbcm_init_device(lbcm_handle *h, const double *phi0, const double *rho0, const double *ux0, const double *uy0)
{
    if (!h) return LBCM_EINVAL;
    if (!phi0) return fail(h, LBCM_EINVAL, "phi0 is NULL");
    return dispatch(h, [&](auto *tag) { return do_init<std::remove_pointer_t<decltype(tag)>>(h, phi0, rho0, ux0, uy0); });
}

int lbcm_init(lbcm_handle *h, const double *phi0, const double *rho0, const double *ux0, const double *uy0)
{
    if (!h) return LBCM_EINVAL;
    if (!phi0) return fail(h, LBCM_EINVAL, "phi0 is NULL");
    // stage the host planes in pair 0 (overwritten only by the final un-stream of the init)
    const size_t N = (size_t)h->p.nx * h->p.ny;
    double *stage = (double *)h->ws;
    const double *src[4] = {phi0, rho0, ux0, uy0};
    const double *dev[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < 4; ++k) {
        if (!src[k]) continue;
        HIP_TRY(h, hipMemcpyAsync(stage + k * N, src[k], N * sizeof(double), hipMemcpyHostToDevice, h->stream));
        dev[k] = stage + k * N;
    }
    int rc = lbcm_init_device(h, dev[0], dev[1], dev[2], dev[3]);
    if (rc) return rc;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return LBCM_OK;
}

int lbcm_step(lbcm_handle *h, int64_t nsteps)
{
    if (!h) return LBCM_EINVAL;
    if (!h->ready) return fail(h, LBCM_ESTATE, "lbcm_step before lbcm_init");
    if (nsteps < 0) return fail(h, LBCM_EINVAL, "nsteps must be >= 0");
    return dispatch(h, [&](auto *tag) { return launch_steps<std::remove_pointer_t<decltype(tag)>>(h, nsteps); });
}

int lbcm_fields_device(lbcm_handle *h, double *phi, double *rho, double *ux, double *uy, double *p0)
{
    if (!h) return LBCM_EINVAL;
    if (!h->ready) return fail(h, LBCM_ESTATE, "lbcm_fields before lbcm_init");
    return dispatch(h, [&](auto *tag) { return do_fields<std::remove_pointer_t<decltype(tag)>>(h, phi, rho, ux, uy, p0); });
}

int lbcm_fields(lbcm_handle *h, double *phi, double *rho, double *ux, double *uy, double *p0)
{
    if (!h) return LBCM_EINVAL;
    if (!h->ready) return fail(h, LBCM_ESTATE, "lbcm_fields before lbcm_init");
    // one plane at a time through the spare pair (>= 8 bytes per node for every precision)
    const size_t N = (size_t)h->p.nx * h->p.ny;
    double *stage = (double *)(h->ws + (size_t)(1 - h->cur) * h->pair_bytes);
    double *dst[5] = {phi, rho, ux, uy, p0};
    for (int k = 0; k < 5; ++k) {
        if (!dst[k]) continue;
        double *d[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
        d[k] = stage;
        int rc = lbcm_fields_device(h, d[0], d[1], d[2], d[3], d[4]);
        if (rc) return rc;
        HIP_TRY(h, hipMemcpyAsync(dst[k], stage, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    return LBCM_OK;
}

int lbcm_populations(lbcm_handle *h, double *f, double *g)
{
    if (!h) return LBCM_EINVAL;
    if (!h->ready) return fail(h, LBCM_ESTATE, "lbcm_populations before lbcm_init");
    const size_t N = (size_t)h->p.nx * h->p.ny;
    double *stage = (double *)(h->ws + (size_t)(1 - h->cur) * h->pair_bytes);
    for (int k = 0; k < 18; ++k) {
        double *dst = k < 9 ? f : g;
        if (!dst) continue;
        int rc = dispatch(h, [&](auto *tag) { return do_population<std::remove_pointer_t<decltype(tag)>>(h, k, stage); });
        if (rc) return rc;
        HIP_TRY(h, hipMemcpyAsync(dst + (size_t)(k % 9) * N, stage, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    return LBCM_OK;
}

int lbcm_diag(lbcm_handle *h, lbcm_diagnostics *out)
{
    if (!h || !out) return fail(h, LBCM_EINVAL, "NULL argument");
    if (!h->ready) return fail(h, LBCM_ESTATE, "lbcm_diag before lbcm_init");
    int rc = dispatch(h, [&](auto *tag) { return do_diag<std::remove_pointer_t<decltype(tag)>>(h); });
    if (rc) return rc;
    double v[kDiagFields];
    HIP_TRY(h, hipMemcpyAsync(v, h->diag_out, sizeof v, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    out->sum_phi = v[0];
    out->sum_abs_phi = v[1];
    out->sum_rho = v[2];
    out->sum_jx = v[3];
    out->sum_jy = v[4];
    out->max_u = v[5];
    out->nonfinite = (int64_t)v[6];
    out->step = h->step;
    return LBCM_OK;
}

size_t lbcm_state_size(const lbcm_handle *h)
{
    return h ? 18 * (size_t)h->p.nx * h->p.ny * h->elem : 0;
}

int lbcm_get_state(lbcm_handle *h, void *host, size_t bytes)
{
    if (!h || !host) return fail(h, LBCM_EINVAL, "NULL argument");
    if (!h->ready) return fail(h, LBCM_ESTATE, "lbcm_get_state before lbcm_init");
    if (bytes != lbcm_state_size(h)) return fail(h, LBCM_EINVAL, "wrong state size");
    HIP_TRY(h, hipMemcpyAsync(host, h->ws + (size_t)h->cur * h->pair_bytes, bytes, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return LBCM_OK;
}

int lbcm_set_state(lbcm_handle *h, const void *host, size_t bytes, int64_t step)
{
    if (!h || !host) return fail(h, LBCM_EINVAL, "NULL argument");
    if (bytes != lbcm_state_size(h)) return fail(h, LBCM_EINVAL, "wrong state size");
    if (step < 0) return fail(h, LBCM_EINVAL, "step must be >= 0");
    HIP_TRY(h, hipMemcpyAsync(h->ws + (size_t)h->cur * h->pair_bytes, host, bytes, hipMemcpyHostToDevice, h->stream));
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(1), 0, h->stream, h->flag);
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->ready = true;
    h->step = step;
    return LBCM_OK;
}

int lbcm_destroy(lbcm_handle *h)
{
    if (!h) return LBCM_OK;
    int rc = LBCM_OK;
    if (h->owns_ws && h->ws) {
        if (hipStreamSynchronize(h->stream) != hipSuccess) rc = LBCM_EHIP;
        if (hipFree(h->ws) != hipSuccess) rc = LBCM_EHIP;
    }
    delete h;
    return rc;
}

const char *lbcm_last_error(const lbcm_handle *h)
{
    return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
