// lbcm: hybrid central-moments / BGK lattice Boltzmann step for the coupled
// Cahn-Hilliard--Navier-Stokes equations (De Rosis, Saito, Kaneko, Abe, arXiv:1803.11345),
// written for MI355X (gfx950, wave64).
//
// Data layout in HBM.  Each population set (f or g) is 9 planes [i][y][x] (x fastest), packed
// back to back; two copies ("pairs") of (f, g) live in one workspace, a step reads pair `cur`
// and writes pair 1 - cur.  Streaming is done by pulling: the stored value P[i](x) is the
// post-collision population f*_i(x, t-1) at its origin node, and the post-streaming population
// of the paper, f_i(x, t) = f*_i(x - c_i, t - 1) (Eqs. (4)-(5)), is read at x - c_i.  With
// walls, a link that would come from outside is the same node's opposite post-collision value
// (half-way bounce-back).  Every reader of the state (step, fields, diagnostics) pulls.
//
// Storage modes.  f is always stored shifted by the lattice weights, f_i - w_i (its deviation
// from the resting equilibrium rho = 1, v = 0), so that its moments are formed from small
// numbers and a weak body force is not lost in the rounding of O(0.1) values.  g is stored as
// is.  FP64 and FP32 store every plane in that type.  The 16-bit modes store the nine f planes
// and g_1..g_8 (all small) as IEEE half or bfloat16 and keep g_0, which carries phi in [-1, 1],
// in FP32; arithmetic is FP32 in every mode but FP64.
//
// The step kernel (k_step) is one fused pass per time step over 2-D tiles; see its comment.
//
// The central-moment collision never forms the 9x9 matrix of the basis: the few pre-collision
// central moments it needs (k3, k4, k5) come from raw moments, and the post-collision
// populations are rebuilt by shifting the post-collision central moments back to raw moments
// (binomial expansion in v) and inverting the raw-moment map of D2Q9, which factorises into the
// 1-D map (m0, m1, m2) -> (f_0, f_+, f_-) = (m0 - m2, (m1 + m2)/2, (m2 - m1)/2) along x and y.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "lbcm.h"

namespace {

// Default step tiles, in waves of 64 columns across (wx) and wave rows down.  Large lattices are
// bandwidth-bound: there the measured best tiles of the 4096^2 step (FP32 4 x 3, FP64 2 x 4,
// 16-bit storage 4 x 3 with two-row waves); below, where a launch is a latency chain and more
// workgroups pay, 8 x 2.  Large: from kLargeNodes nodes on, for FP32 from kLargeNodes32 (at
// 1024^2 the 4 x 3 tile is 15 % faster than 8 x 2 in FP32, while 16-bit storage gains nothing
// there).
constexpr size_t kLargeNodes = size_t(1) << 22, kLargeNodes32 = size_t(1) << 20;
constexpr int kDefaultWx = 8, kDefaultRows = 2;
constexpr int kLargeWx = 4, kLargeRows = 3;
constexpr int kLargeWx16 = 4, kLargeRows16 = 3;
constexpr int kLargeWx64 = 2, kLargeRows64 = 4;
constexpr int kXcds = 8;         // XCDs of the device, to which workgroups are dealt in turn
constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;
constexpr int kDiagFields = 8;  // phi, |phi|, rho, jx, jy, max|v|, nonfinite, max|dv|

// ------------------------------------------------------------------------------------------
// raw buffer access

constexpr int kBufFlags = 0x00020000;  // word 3 of a raw buffer resource (gfx9 family)
constexpr int kLoadAux = 0;            // cache policy of the pulls (g rows are re-read as halos)
constexpr int kStoreAux = 2;           // cache policy of the stores: non-temporal

using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kBufFlags);
}

// One stored element type: load through a buffer resource into the compute type R, store R.
template <class T> struct Elem;
template <> struct Elem<double> {
    using V2 = __attribute__((__vector_size__(2 * sizeof(unsigned int)))) unsigned int;
    template <class R> static __device__ __forceinline__ R ld(rsrc_t r, uint32_t v, uint32_t s)
    {
        return (R)__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)v, (int)s, kLoadAux));
    }
    template <class R> static __device__ __forceinline__ void st(rsrc_t r, uint32_t v, uint32_t s, R x)
    {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, (double)x), r, (int)v, (int)s, kStoreAux);
    }
};
template <> struct Elem<float> {
    template <class R> static __device__ __forceinline__ R ld(rsrc_t r, uint32_t v, uint32_t s)
    {
        return (R)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)v, (int)s, kLoadAux));
    }
    template <class R> static __device__ __forceinline__ void st(rsrc_t r, uint32_t v, uint32_t s, R x)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, (float)x), r, (int)v, (int)s, kStoreAux);
    }
};
template <> struct Elem<_Float16> {
    template <class R> static __device__ __forceinline__ R ld(rsrc_t r, uint32_t v, uint32_t s)
    {
        return (R)(float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)v, (int)s, kLoadAux));
    }
    template <class R> static __device__ __forceinline__ void st(rsrc_t r, uint32_t v, uint32_t s, R x)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)(float)x), r, (int)v, (int)s,
                                              kStoreAux);
    }
};
template <> struct Elem<__bf16> {
    template <class R> static __device__ __forceinline__ R ld(rsrc_t r, uint32_t v, uint32_t s)
    {
        return (R)(float)__builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)v, (int)s, kLoadAux));
    }
    template <class R> static __device__ __forceinline__ void st(rsrc_t r, uint32_t v, uint32_t s, R x)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (__bf16)(float)x), r, (int)v, (int)s,
                                              kStoreAux);
    }
};

// Storage modes: compute type R, type of the f planes, of g_0 and of g_1..g_8, and the most
// lattice rows each wave of the step kernel updates (two with 16-bit storage, whose loads carry
// half the bytes: two rows per wave keep as many bytes in flight per wave as one FP32 row; used
// on lattices large enough to be bandwidth-bound, see rows_per_wave).
struct ModeF64 { using R = double; using F = double; using G0 = double; using G = double; static constexpr int kRpw = 1; };
struct ModeF32 { using R = float; using F = float; using G0 = float; using G = float; static constexpr int kRpw = 1; };
struct ModeF16 { using R = float; using F = _Float16; using G0 = float; using G = _Float16; static constexpr int kRpw = 2; };
struct ModeB16 { using R = float; using F = __bf16; using G0 = float; using G = __bf16; static constexpr int kRpw = 2; };
static_assert(ModeF64::kRpw == ModeF32::kRpw && ModeB16::kRpw == ModeF16::kRpw, "rows per wave follow the storage width");

// Byte offset of plane i in a set whose plane 0 has element type T0 and planes 1..8 type T.
template <class T0, class T> __device__ __forceinline__ uint32_t plane_off(int i, uint32_t N)
{
    return i == 0 ? 0u : N * (uint32_t)sizeof(T0) + (uint32_t)(i - 1) * N * (uint32_t)sizeof(T);
}
template <class T0, class T> __device__ __forceinline__ uint32_t set_bytes(uint32_t N)
{
    return N * (uint32_t)sizeof(T0) + 8u * N * (uint32_t)sizeof(T);
}

// Runtime description of a set (for the readers and the initialisation, not on the hot path).
enum : int { kKindF64 = 0, kKindF32 = 1, kKindF16 = 2, kKindB16 = 3 };
struct SetView {
    unsigned char *base;
    uint32_t off[9];  // byte offset of each plane
    int kind[9];      // element kind of each plane
};

__device__ __forceinline__ double view_ld(const SetView &v, int i, size_t n)
{
    const unsigned char *p = v.base + v.off[i];
    switch (v.kind[i]) {
    case kKindF64: return ((const double *)p)[n];
    case kKindF32: return (double)((const float *)p)[n];
    case kKindF16: return (double)(float)((const _Float16 *)p)[n];
    default: return (double)(float)((const __bf16 *)p)[n];
    }
}

__device__ __forceinline__ void view_st(const SetView &v, int i, size_t n, double x)
{
    unsigned char *p = v.base + v.off[i];
    switch (v.kind[i]) {
    case kKindF64: ((double *)p)[n] = x; break;
    case kKindF32: ((float *)p)[n] = (float)x; break;
    case kKindF16: ((_Float16 *)p)[n] = (_Float16)(float)x; break;
    default: ((__bf16 *)p)[n] = (__bf16)(float)x; break;
    }
}

__device__ __forceinline__ void view_copy(const SetView &src, int i, size_t ns, const SetView &dst, int j, size_t nd)
{
    const unsigned char *s = src.base + src.off[i];
    unsigned char *d = dst.base + dst.off[j];
    switch (src.kind[i]) {
    case kKindF64: ((double *)d)[nd] = ((const double *)s)[ns]; break;
    case kKindF32: ((float *)d)[nd] = ((const float *)s)[ns]; break;
    default: ((unsigned short *)d)[nd] = ((const unsigned short *)s)[ns]; break;
    }
}

// ------------------------------------------------------------------------------------------
// parameters

struct Geo {
    int nx, ny;
    uint32_t plane;     // nx * ny
    int wx;             // wave columns per tile (tile width 64 * wx)
    int rows;           // wave rows per tile
    int rpw;            // lattice rows per wave row (1 or the mode's kRpw); tile height rows * rpw
    int nbands, nrows;  // tiles across and down
    int walls;
    double ub6, ut6;    // x velocities of the bottom and top walls, divided by 6
    double wgrad;       // wall gradient of phi along the inward normal
};

// Moving walls: a link that comes back from a wall moving along x with speed U gains
// 2 w_j s (c_j . U) / c_s^2 = s c_jx U / 6 (the diagonal links 5, 6 at the bottom, 7, 8 at the
// top; s = 1 for f, the node's phi for g).  Applied wherever populations are pulled.
template <class R>
__device__ __forceinline__ void wall_motion(R v[9], R s, bool bot, bool top, R ub6, R ut6)
{
    if (bot) {
        v[5] += s * ub6;
        v[6] -= s * ub6;
    }
    if (top) {
        v[7] -= s * ut6;
        v[8] += s * ut6;
    }
}

template <class R> struct Phys {
    R a, gamma, Gamma;
    R w_mid, w_half;  // omega_rho = w_mid + w_half * phi
    R w3, wphi;
    R hFx, hFy;       // half of the body force
    R ub6, ut6;       // wall x velocities / 6
    R wgrad;          // wall gradient of phi (inward normal)
    int k8_printed;
};

__constant__ double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
__constant__ int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int kCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__constant__ int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// ------------------------------------------------------------------------------------------
// pull of the 9 post-streaming populations of one row.  One buffer resource covers the 9 planes
// of a set; the plane offset and the row y (uniform across the wave) go in the scalar offset of
// the buffer loads, and each lane supplies the element index of its columns x, x - 1 and x + 1
// (periodic).  With walls, a link that would come from behind a wall takes the node's own
// opposite post-collision value (the weights of opposite directions are equal, so this holds
// for the shifted f as well; plane 0 never bounces, so g_0 keeps its own type).

template <class T0, class T, class R, bool WALLS>
__device__ __forceinline__ void pull_row(rsrc_t P, uint32_t N, int nx, int ny, int y, uint32_t x,
                                         uint32_t xl, uint32_t xr, R v[9])
{
    constexpr uint32_t b0 = sizeof(T0), b = sizeof(T);
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
    const uint32_t rb = (uint32_t)nx * b;
    const uint32_t s0 = (uint32_t)y * rb, sd = (uint32_t)yd * rb, su = (uint32_t)yu * rb;
    const uint32_t cx = x * b, cl = xl * b, cr = xr * b;
    auto po = [&](int i) { return plane_off<T0, T>(i, N); };
    v[0] = Elem<T0>::template ld<R>(P, x * b0, (uint32_t)y * (uint32_t)nx * b0);
    v[1] = Elem<T>::template ld<R>(P, cl, po(1) + s0);
    v[3] = Elem<T>::template ld<R>(P, cr, po(3) + s0);
    if (WALLS && bot) {
        v[2] = Elem<T>::template ld<R>(P, cx, po(4) + s0);
        v[5] = Elem<T>::template ld<R>(P, cx, po(7) + s0);
        v[6] = Elem<T>::template ld<R>(P, cx, po(8) + s0);
    } else {
        v[2] = Elem<T>::template ld<R>(P, cx, po(2) + sd);
        v[5] = Elem<T>::template ld<R>(P, cl, po(5) + sd);
        v[6] = Elem<T>::template ld<R>(P, cr, po(6) + sd);
    }
    if (WALLS && top) {
        v[4] = Elem<T>::template ld<R>(P, cx, po(2) + s0);
        v[7] = Elem<T>::template ld<R>(P, cx, po(5) + s0);
        v[8] = Elem<T>::template ld<R>(P, cx, po(6) + s0);
    } else {
        v[4] = Elem<T>::template ld<R>(P, cx, po(4) + su);
        v[7] = Elem<T>::template ld<R>(P, cr, po(7) + su);
        v[8] = Elem<T>::template ld<R>(P, cl, po(8) + su);
    }
}

// The same pull for one arbitrary node (readers; any y per lane), in double.
__device__ __forceinline__ void pull_node(const SetView &P, const Geo &geo, size_t n, double v[9], bool is_g)
{
    const int nx = geo.nx, ny = geo.ny;
    const int y = (int)(n / nx), x = (int)(n % nx);
    const int xl = x == 0 ? nx - 1 : x - 1, xr = x == nx - 1 ? 0 : x + 1;
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
        v[i] = view_ld(P, ii, (size_t)ys * nx + xs);
    }
    if (geo.walls) {
        double s = 1.0;
        if (is_g) {
            s = 0;
            for (int i = 0; i < 9; ++i) s += v[i];
        }
        wall_motion(v, s, y == 0, y == ny - 1, geo.ub6, geo.ut6);
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
// raw-moment map is inverted as the tensor product of the 1-D map.

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

template <class R> struct Rcp;
template <> struct Rcp<double> {
    static __device__ __forceinline__ double of(double v) { return 1.0 / v; }
};
template <> struct Rcp<float> {
    static __device__ __forceinline__ float of(float v) { return __builtin_amdgcn_rcpf(v); }  // 1 ulp
};

// ------------------------------------------------------------------------------------------
// one node: central-moment collision of f (Eq. (17)) and BGK of g (Eq. (7)).
// f and fo hold f_i - w_i.

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
// the step kernel.  A workgroup owns a tile of 64 * wx columns by rows * RPW lattice rows; each
// of its waves owns a 64-column segment of RPW rows (one node per lane and row; two rows on large
// lattices with 16-bit storage, so that a wave has as many bytes in flight as with FP32 storage
// and one row: 2-4 % faster there).  Every wave pulls f and g of its own nodes, sums phi into an
// LDS tile with a one-node halo, and the halo is filled by the same pulls one node further out:
// the waves of the first and last tile row also pull g of the rows above and below, and lanes 0
// and 1 of the first wave column pull the two halo columns.  One barrier later every node reads
// its 3x3 phi stencil from LDS, collides and stores f*, g* at its own node (non-temporal).
//
// Every load of a workgroup is issued before its barrier (at raised wave priority, f first), and
// workgroups are dispatched in row-major tile order, so the waves resident at any moment cover a
// compact band of rows: the HBM sees a few long streams per plane instead of many short ones.
// The halo re-reads are served by L2 and the MALL.  With a multiple of 8 tiles per tile row the
// tiles above and below a tile are dealt to its XCD, so its halo rows are hits in the same L2.

template <class M> constexpr int kMaxThreads = sizeof(typename M::R) == 8 ? 512 : 1024;

// One tile (band, rg) of one lattice, one lattice row per wave row; called by the kernels with the
// workgroup's LDS.  All threads of the workgroup must call it (it contains the barrier).  The
// two-row tile below computes the same thing; this one is kept separate because written as its
// RPW = 1 case the compiler needs ~35 more scalar registers (100 and more with walls), which
// leaves room for one 1024-thread workgroup per CU instead of two.
template <class M, bool WALLS, bool FORCE>
__device__ __forceinline__ void step_tile_row(const unsigned char *__restrict__ fa, const unsigned char *__restrict__ ga,
                                          unsigned char *__restrict__ fb, unsigned char *__restrict__ gb,
                                          const Geo &geo, const Phys<typename M::R> &c, int *__restrict__ flag,
                                          int band, int rg, typename M::R *phs)
{
    using R = typename M::R;
    using F = typename M::F;
    using G0 = typename M::G0;
    using G = typename M::G;

    const int nx = geo.nx, ny = geo.ny;
    const uint32_t N = geo.plane;
    const int wx = geo.wx, rows_t = geo.rows;
    const int ldw = 64 * wx + 2;
    const int lane = threadIdx.x & 63;
    // wave index made explicitly uniform, so that the row offsets stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wc = wave % wx, wr = wave / wx;  // wave column and row inside the tile
    const int X0 = band * 64 * wx;
    const int X1 = min(X0 + 64 * wx, nx);
    const int y0 = rg * rows_t;
    const int y1 = min(y0 + rows_t, ny);
    const int y = y0 + wr;
    const bool row_ok = y < y1;  // uniform per wave
    const int xr_ = X0 + wc * 64 + lane;
    const bool col_ok = xr_ < X1;
    const bool valid = row_ok && col_ok;
    const int x = col_ok ? xr_ : X1 - 1;  // clamped for addressing
    const int yy = row_ok ? y : y1 - 1;
    const uint32_t xl = x == 0 ? nx - 1 : x - 1;
    const uint32_t xr = x == nx - 1 ? 0 : x + 1;
    const rsrc_t rfa = make_rsrc(fa, set_bytes<F, F>(N));
    const rsrc_t rga = make_rsrc(ga, set_bytes<G0, G>(N));
    const rsrc_t rfb = make_rsrc(fb, set_bytes<F, F>(N));
    const rsrc_t rgb = make_rsrc(gb, set_bytes<G0, G>(N));
    const int slot = wc * 64 + lane + 1;  // LDS column of this lane
    const int last = y1 - y0 - 1;         // last valid tile row
    auto wrap_row = [&](int r) { return r < 0 ? r + ny : (r >= ny ? r - ny : r); };

    // own populations; the loads go out at raised wave priority so that the memory pipeline of
    // the CU keeps being fed while other workgroups compute
    __builtin_amdgcn_s_setprio(3);
    R g[9], f[9];
    pull_row<F, F, R, WALLS>(rfa, N, nx, ny, yy, (uint32_t)x, xl, xr, f);
    pull_row<G0, G, R, WALLS>(rga, N, nx, ny, yy, (uint32_t)x, xl, xr, g);
    const R phi_own = sum9(g);  // the wall corrections of g cancel in the sum
    if (WALLS) {
        const bool bot = yy == 0, top = yy == ny - 1;
        wall_motion(f, (R)1, bot, top, c.ub6, c.ut6);
        wall_motion(g, phi_own, bot, top, c.ub6, c.ut6);
    }
    if (valid) phs[(wr + 1) * ldw + slot] = phi_own;

    // halo rows: the first tile row fetches the row above, the last valid one the row below;
    // behind a wall the ghost row holds the first / last row's phi minus the wall gradient
    auto halo_row = [&](int hy, int srow) {
        if (WALLS && (hy < 0 || hy >= ny)) {
            if (col_ok) phs[srow * ldw + slot] = phi_own - c.wgrad;
        } else {
            R h[9];
            pull_row<G0, G, R, WALLS>(rga, N, nx, ny, wrap_row(hy), (uint32_t)x, xl, xr, h);
            if (col_ok) phs[srow * ldw + slot] = sum9(h);
        }
    };
    if (wr == 0) halo_row(y0 - 1, 0);
    if (wr == last) halo_row(y1, last + 2);

    // halo columns (x = X0 - 1 on lane 0, x = X1 on lane 1) for this wave's row and, on the
    // first / last tile row, the corner rows
    if (wc == 0 && lane < 2 && wr <= last) {
        const uint32_t hx = lane == 0 ? (X0 == 0 ? nx - 1 : X0 - 1) : (X1 == nx ? 0 : X1);
        const uint32_t hxl = hx == 0 ? nx - 1 : hx - 1, hxr = hx == (uint32_t)nx - 1 ? 0 : hx + 1;
        const int hs = lane == 0 ? 0 : X1 - X0 + 1;
        R h[9];
        pull_row<G0, G, R, WALLS>(rga, N, nx, ny, y, hx, hxl, hxr, h);
        const R ph = sum9(h);
        phs[(wr + 1) * ldw + hs] = ph;
        for (int side = 0; side < 2; ++side) {
            if (side == 0 && wr != 0) continue;
            if (side == 1 && wr != last) continue;
            const int hy = side == 0 ? y0 - 1 : y1;
            const int srow = side == 0 ? 0 : last + 2;
            if (WALLS && (hy < 0 || hy >= ny)) {
                phs[srow * ldw + hs] = ph - c.wgrad;
            } else {
                R h2[9];
                pull_row<G0, G, R, WALLS>(rga, N, nx, ny, wrap_row(hy), hx, hxl, hxr, h2);
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
        const uint32_t ux_ = (uint32_t)x, uy_ = (uint32_t)y, unx = (uint32_t)nx;
        constexpr uint32_t bf = sizeof(F), bg0 = sizeof(G0), bg = sizeof(G);
#pragma unroll
        for (int i = 0; i < 9; ++i) Elem<F>::template st<R>(rfb, ux_ * bf, plane_off<F, F>(i, N) + uy_ * unx * bf, fo[i]);
        Elem<G0>::template st<R>(rgb, ux_ * bg0, uy_ * unx * bg0, go[0]);
#pragma unroll
        for (int i = 1; i < 9; ++i)
            Elem<G>::template st<R>(rgb, ux_ * bg, plane_off<G0, G>(i, N) + uy_ * unx * bg, go[i]);
    }
}

// One tile (band, rg) of one lattice with RPW lattice rows per wave row: wave row wr updates the
// rows y0 + RPW * wr + k, k < RPW, of the tile.  All threads of the workgroup must call it.
template <class M, int RPW, bool WALLS, bool FORCE>
__device__ __forceinline__ void step_tile(const unsigned char *__restrict__ fa, const unsigned char *__restrict__ ga,
                                          unsigned char *__restrict__ fb, unsigned char *__restrict__ gb,
                                          const Geo &geo, const Phys<typename M::R> &c, int *__restrict__ flag,
                                          int band, int rg, typename M::R *phs)
{
    using R = typename M::R;
    using F = typename M::F;
    using G0 = typename M::G0;
    using G = typename M::G;
    if constexpr (RPW == 1) {
        step_tile_row<M, WALLS, FORCE>(fa, ga, fb, gb, geo, c, flag, band, rg, phs);
        return;
    }

    const int nx = geo.nx, ny = geo.ny;
    const uint32_t N = geo.plane;
    const int wx = geo.wx;
    const int ldw = 64 * wx + 2;
    const int lane = threadIdx.x & 63;
    // wave index made explicitly uniform, so that the row offsets stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wc = wave % wx, wr = wave / wx;  // wave column and row inside the tile
    const int X0 = band * 64 * wx;
    const int X1 = min(X0 + 64 * wx, nx);
    const int y0 = rg * geo.rows * RPW;
    const int y1 = min(y0 + geo.rows * RPW, ny);
    const int last = y1 - y0 - 1;  // last valid tile row
    const int xr_ = X0 + wc * 64 + lane;
    const bool col_ok = xr_ < X1;
    const int x = col_ok ? xr_ : X1 - 1;  // clamped for addressing
    const uint32_t xl = x == 0 ? nx - 1 : x - 1;
    const uint32_t xr = x == nx - 1 ? 0 : x + 1;
    const rsrc_t rfa = make_rsrc(fa, set_bytes<F, F>(N));
    const rsrc_t rga = make_rsrc(ga, set_bytes<G0, G>(N));
    const rsrc_t rfb = make_rsrc(fb, set_bytes<F, F>(N));
    const rsrc_t rgb = make_rsrc(gb, set_bytes<G0, G>(N));
    const int slot = wc * 64 + lane + 1;  // LDS column of this lane
    auto wrap_row = [&](int r) { return r < 0 ? r + ny : (r >= ny ? r - ny : r); };

    // own populations; the loads go out at raised wave priority so that the memory pipeline of
    // the CU keeps being fed while other workgroups compute
    __builtin_amdgcn_s_setprio(3);
    R g[RPW][9], f[RPW][9];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int tr = wr * RPW + k;
        const int yy = min(y0 + tr, y1 - 1);  // clamped for addressing
        pull_row<F, F, R, WALLS>(rfa, N, nx, ny, yy, (uint32_t)x, xl, xr, f[k]);
        pull_row<G0, G, R, WALLS>(rga, N, nx, ny, yy, (uint32_t)x, xl, xr, g[k]);
    }

    // halo rows: the first tile row fetches the row above, the last valid one the row below;
    // behind a wall the ghost row holds the first / last row's phi minus the wall gradient
    auto halo_row = [&](int hy, int srow, R phi_own) {
        if (WALLS && (hy < 0 || hy >= ny)) {
            if (col_ok) phs[srow * ldw + slot] = phi_own - c.wgrad;
        } else {
            R h[9];
            pull_row<G0, G, R, WALLS>(rga, N, nx, ny, wrap_row(hy), (uint32_t)x, xl, xr, h);
            if (col_ok) phs[srow * ldw + slot] = sum9(h);
        }
    };
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int tr = wr * RPW + k;
        const int yy = min(y0 + tr, y1 - 1);
        const R phi_own = sum9(g[k]);  // the wall corrections of g cancel in the sum
        if (WALLS) {
            const bool bot = yy == 0, top = yy == ny - 1;
            wall_motion(f[k], (R)1, bot, top, c.ub6, c.ut6);
            wall_motion(g[k], phi_own, bot, top, c.ub6, c.ut6);
        }
        if (tr <= last && col_ok) phs[(tr + 1) * ldw + slot] = phi_own;
        if (tr == 0) halo_row(y0 - 1, 0, phi_own);
        if (tr == last) halo_row(y1, last + 2, phi_own);
    }

    // halo columns (x = X0 - 1 on lane 0, x = X1 on lane 1) for this wave's rows and, on the
    // first / last tile row, the corner rows
    if (wc == 0 && lane < 2) {
        const uint32_t hx = lane == 0 ? (X0 == 0 ? nx - 1 : X0 - 1) : (X1 == nx ? 0 : X1);
        const uint32_t hxl = hx == 0 ? nx - 1 : hx - 1, hxr = hx == (uint32_t)nx - 1 ? 0 : hx + 1;
        const int hs = lane == 0 ? 0 : X1 - X0 + 1;
        for (int k = 0; k < RPW; ++k) {
            const int tr = wr * RPW + k;
            if (tr > last) break;
            R h[9];
            pull_row<G0, G, R, WALLS>(rga, N, nx, ny, y0 + tr, hx, hxl, hxr, h);
            const R ph = sum9(h);
            phs[(tr + 1) * ldw + hs] = ph;
            for (int side = 0; side < 2; ++side) {
                if (side == 0 && tr != 0) continue;
                if (side == 1 && tr != last) continue;
                const int hy = side == 0 ? y0 - 1 : y1;
                const int srow = side == 0 ? 0 : last + 2;
                if (WALLS && (hy < 0 || hy >= ny)) {
                    phs[srow * ldw + hs] = ph - c.wgrad;
                } else {
                    R h2[9];
                    pull_row<G0, G, R, WALLS>(rga, N, nx, ny, wrap_row(hy), hx, hxl, hxr, h2);
                    phs[srow * ldw + hs] = sum9(h2);
                }
            }
        }
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);

#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int tr = wr * RPW + k;
        if (tr > last) break;  // uniform per wave
        const int y = y0 + tr;
        const R *rS = phs + tr * ldw, *rC = phs + (tr + 1) * ldw, *rN = phs + (tr + 2) * ldw;
        const R pS = rS[slot], pSW = rS[slot - 1], pSE = rS[slot + 1];
        const R pC = rC[slot], pW = rC[slot - 1], pE = rC[slot + 1];
        const R pN = rN[slot], pNW = rN[slot - 1], pNE = rN[slot + 1];
        const R dpx = ((R)4 * (pE - pW) + (pNE - pNW) + (pSE - pSW)) * (R)(1.0 / 12.0);
        const R dpy = ((R)4 * (pN - pS) + (pNE - pSE) + (pNW - pSW)) * (R)(1.0 / 12.0);
        const R lap = ((R)4 * ((pE + pW) + (pN + pS)) + ((pNE + pNW) + (pSE + pSW)) - (R)20 * pC) *
                      (R)(1.0 / 6.0);

        R fo[9], go[9], rho;
        collide_node<R, FORCE>(f[k], g[k], pC, dpx, dpy, lap, c, fo, go, rho);
        const bool bad = !(std::isfinite(rho) && std::isfinite(pC)) && col_ok;
        if (__any(bad) && lane == 0) atomicOr(flag, 1);

        if (col_ok) {
            const uint32_t ux_ = (uint32_t)x, uy_ = (uint32_t)y, unx = (uint32_t)nx;
            constexpr uint32_t bf = sizeof(F), bg0 = sizeof(G0), bg = sizeof(G);
#pragma unroll
            for (int i = 0; i < 9; ++i) Elem<F>::template st<R>(rfb, ux_ * bf, plane_off<F, F>(i, N) + uy_ * unx * bf, fo[i]);
            Elem<G0>::template st<R>(rgb, ux_ * bg0, uy_ * unx * bg0, go[0]);
#pragma unroll
            for (int i = 1; i < 9; ++i)
                Elem<G>::template st<R>(rgb, ux_ * bg, plane_off<G0, G>(i, N) + uy_ * unx * bg, go[i]);
        }
    }
}

template <class M, int RPW, bool WALLS, bool FORCE>
__global__ __launch_bounds__(kMaxThreads<M>) void
k_step(const unsigned char *__restrict__ fa, const unsigned char *__restrict__ ga,
       unsigned char *__restrict__ fb, unsigned char *__restrict__ gb, Geo geo,
       Phys<typename M::R> c, int *__restrict__ flag)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int band = blockIdx.x % geo.nbands, rg = blockIdx.x / geo.nbands;
    step_tile<M, RPW, WALLS, FORCE>(fa, ga, fb, gb, geo, c, flag, band, rg, reinterpret_cast<typename M::R *>(lds_raw));
}

// ------------------------------------------------------------------------------------------
// batched step: every tile of every box of an ensemble in one launch.  tiles[g] = (box, t) is
// the tile of grid index g: tile t of the box in its row-major order (box < 0: an empty slot,
// whose workgroup returns at once).  Each box has its own size, tile shape (within the launch's
// workgroup size), boundaries, force and physics.  Every wave updates one lattice row,
// in the 16-bit modes too: the small tiles of an ensemble gain nothing from the longer loads in
// flight of two-row waves, and lose the occupancy their registers cost.

template <class R> struct BoxDesc {
    Geo geo;
    Phys<R> c;
    const unsigned char *set[2][2];  // [pair][f or g]
    int *flag;                       // the box's divergence flag (set on a non-finite rho or phi)
    int walls, force;
    int done_off;                    // persistent dataflow launch: first step counter of this box's tiles
};

template <class M>
__global__ __launch_bounds__(kMaxThreads<M>) void k_step_batch(const BoxDesc<typename M::R> *__restrict__ boxes,
                                                               const int2 *__restrict__ tiles, int cur)
{
    using R = typename M::R;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    R *phs = reinterpret_cast<R *>(lds_raw);
    const int2 e = tiles[blockIdx.x];
    if (e.x < 0) return;  // empty slot: the whole workgroup leaves before any barrier
    const BoxDesc<R> &d = boxes[e.x];
    const int band = e.y % d.geo.nbands, rg = e.y / d.geo.nbands;
    const unsigned char *fa = d.set[cur][0], *ga = d.set[cur][1];
    unsigned char *fb = const_cast<unsigned char *>(d.set[1 - cur][0]);
    unsigned char *gb = const_cast<unsigned char *>(d.set[1 - cur][1]);
    int *flag = d.flag;
    if (d.walls) {
        if (d.force) step_tile<M, 1, true, true>(fa, ga, fb, gb, d.geo, d.c, flag, band, rg, phs);
        else step_tile<M, 1, true, false>(fa, ga, fb, gb, d.geo, d.c, flag, band, rg, phs);
    } else {
        if (d.force) step_tile<M, 1, false, true>(fa, ga, fb, gb, d.geo, d.c, flag, band, rg, phs);
        else step_tile<M, 1, false, false>(fa, ga, fb, gb, d.geo, d.c, flag, band, rg, phs);
    }
}

// Divergence flags of an ensemble: out[0] = number of boxes whose flag is set, out[1] = the
// smallest such box index (n if none).  One workgroup of kReduceThreads threads.
template <class R>
__global__ __launch_bounds__(kReduceThreads) void k_batch_flags(const BoxDesc<R> *__restrict__ boxes, int n, int *out)
{
    __shared__ int cnt[kReduceThreads], first[kReduceThreads];
    int c = 0, f = n;
    for (int i = threadIdx.x; i < n; i += kReduceThreads)
        if (*boxes[i].flag) {
            ++c;
            f = min(f, i);
        }
    cnt[threadIdx.x] = c;
    first[threadIdx.x] = f;
    __syncthreads();
    for (int s = kReduceThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            cnt[threadIdx.x] += cnt[threadIdx.x + s];
            first[threadIdx.x] = min(first[threadIdx.x], first[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = cnt[0];
        out[1] = first[0];
    }
}

// ------------------------------------------------------------------------------------------
// persistent ensemble launch: one launch advances every box by nsteps.  Workgroups take work
// items k = step * ntiles + t from a global counter (work stealing over the tiles of all boxes,
// step-major), so a workgroup never holds an item whose step is ahead of an item not yet handed
// out.  Two schedules:
//  - kPersistBarrier: a grid barrier between steps (the launch must be co-resident: it is a
//    cooperative launch of at most the resident number of workgroups);
//  - kPersistDataflow: per-tile step counters; an item (s, t) waits until every tile whose
//    nodes its reads or writes reach (the rows y0 - 2 .. y1 + 1 and columns x0 - 2 .. x1 + 1:
//    the pulls of the phi halo) has finished step s - 1.  Those items have smaller indices, so
//    they were handed out before, to running workgroups; the smallest unfinished item therefore
//    always has its inputs and progress never depends on which workgroups are resident.
// Every wait is bounded: after kSpinLimit polls a workgroup sets ctl->abort and leaves, every
// other wait sees the flag and leaves too, and the host reports the launch as failed.
// Cross-workgroup hand-offs are agent-scope release / acquire pairs (on this device an L2
// write-back and an L2 invalidation of the workgroup's XCD); polls are relaxed loads.

constexpr int kPersistBarrier = 1, kPersistDataflow = 2;
constexpr int kSpinLimit = 1 << 21;

struct PersistCtl {
    unsigned long long next;  // next work item
    unsigned int bar_count;   // grid barrier: arrivals in the current generation
    unsigned int bar_gen;     // grid barrier: generation
    int abort;                // a wait gave up
    int pad[3];
};

__device__ __forceinline__ int relaxed_load(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier over nwg workgroups (all threads of the workgroup call it).  Returns false if a
// wait gave up.
__device__ bool grid_barrier(PersistCtl *c, unsigned nwg, int *ok_lds)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned g = __hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nwg - 1) {
            __hip_atomic_store(&c->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&c->bar_gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            for (int n = 0; __hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g; ++n) {
                if (n >= kSpinLimit || ((n & 255) == 255 && relaxed_load(&c->abort))) {
                    __hip_atomic_store(&c->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *ok_lds = ok;
    }
    __syncthreads();
    return *ok_lds != 0;
}

// Dataflow wait of item (s, tile (band, rg) of box d): lanes 0..24 of wave 0 each poll one tile of
// the 5 x 5 candidate set (tile rows holding rg and rows y0 - 2, y0 - 1, y1, y1 + 1, bands holding
// band and columns x0 - 2, x0 - 1, x1, x1 + 1, wrapped periodically; rows behind a wall skipped).
template <class R>
__device__ bool wait_neighbours(const BoxDesc<R> &d, int band, int rg, int s, const int *done, PersistCtl *c,
                                int *ok_lds)
{
    if (threadIdx.x < 64) {
        int ok = 1;
        const int lane = threadIdx.x;
        if (lane < 25 && s > 0) {
            const Geo &g = d.geo;
            const int h = g.rows * g.rpw, w = 64 * g.wx;
            const int y0 = rg * h, y1 = min(y0 + h, g.ny), x0 = band * w, x1 = min(x0 + w, g.nx);
            const int ri = lane / 5, ci = lane % 5;
            const int ry[5] = {y0, y0 - 2, y0 - 1, y1, y1 + 1};
            const int cx[5] = {x0, x0 - 2, x0 - 1, x1, x1 + 1};
            int yy = ry[ri];
            bool skip = false;
            if (yy < 0 || yy >= g.ny) {
                if (g.walls) skip = true;
                else yy = ((yy % g.ny) + g.ny) % g.ny;
            }
            const int xx = ((cx[ci] % g.nx) + g.nx) % g.nx;
            if (!skip) {
                const int *p = done + d.done_off + (yy / h) * g.nbands + xx / w;
                for (int n = 0; relaxed_load(p) < s; ++n) {
                    if (n >= kSpinLimit || ((n & 255) == 255 && relaxed_load(&c->abort))) {
                        __hip_atomic_store(&c->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
        }
        ok = __all(ok);
        if (lane == 0) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            *ok_lds = ok;
        }
    }
    __syncthreads();
    return *ok_lds != 0;
}

// One tile (box e.x, tile e.y) at step s of a persistent launch; all threads of the workgroup call it.
template <class M>
__device__ __forceinline__ void persist_tile(const BoxDesc<typename M::R> &d, int2 e, int s, int phase0,
                                             typename M::R *phs)
{
    const int band = e.y % d.geo.nbands, rg = e.y / d.geo.nbands;
    const int p = (phase0 + s) & 1;
    const unsigned char *fa = d.set[p][0], *ga = d.set[p][1];
    unsigned char *fb = const_cast<unsigned char *>(d.set[1 - p][0]);
    unsigned char *gb = const_cast<unsigned char *>(d.set[1 - p][1]);
    if (d.walls) {
        if (d.force) step_tile<M, 1, true, true>(fa, ga, fb, gb, d.geo, d.c, d.flag, band, rg, phs);
        else step_tile<M, 1, true, false>(fa, ga, fb, gb, d.geo, d.c, d.flag, band, rg, phs);
    } else {
        if (d.force) step_tile<M, 1, false, true>(fa, ga, fb, gb, d.geo, d.c, d.flag, band, rg, phs);
        else step_tile<M, 1, false, false>(fa, ga, fb, gb, d.geo, d.c, d.flag, band, rg, phs);
    }
    __syncthreads();  // every wave's stores issued and its reads of the phi tile done
}

// Items of the dataflow schedule taken per grab of the global counter (fewer atomics on one
// address); a workgroup runs its items in index order, so the smallest unfinished item is always
// the next one of its holder and the argument for progress holds unchanged.
constexpr int kPersistChunk = 8;

template <class M>
__global__ __launch_bounds__(kMaxThreads<M>) void k_step_persist(const BoxDesc<typename M::R> *__restrict__ boxes,
                                                                 const int2 *__restrict__ tiles, int ntiles, int nsteps,
                                                                 int phase0, int mode, PersistCtl *ctl, int *done,
                                                                 unsigned nwg)
{
    using R = typename M::R;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    R *phs = reinterpret_cast<R *>(lds_raw);
    __shared__ long long item;
    __shared__ int ok_lds;
    if (mode == kPersistBarrier) {
        // workgroup w runs tiles w, w + nwg, ... of every step; a grid barrier between steps
        for (int s = 0; s < nsteps; ++s) {
            if (s > 0 && !grid_barrier(ctl, nwg, &ok_lds)) return;
            for (int t = blockIdx.x; t < ntiles; t += nwg) {
                const int2 e = tiles[t];
                if (e.x >= 0) persist_tile<M>(boxes[e.x], e, s, phase0, phs);
            }
        }
        return;
    }
    const long long total = (long long)nsteps * ntiles;
    for (;;) {
        if (threadIdx.x == 0)
            item = relaxed_load(&ctl->abort) ? total : (long long)atomicAdd(&ctl->next, (unsigned long long)kPersistChunk);
        __syncthreads();
        const long long k0 = item;
        __syncthreads();  // `item` is rewritten by the next grab
        if (k0 >= total) break;
        bool ok = true;
        for (long long k = k0; ok && k < k0 + kPersistChunk && k < total; ++k) {
            const int s = (int)(k / ntiles);
            const int2 e = tiles[k % ntiles];
            if (e.x < 0) continue;
            const BoxDesc<R> &d = boxes[e.x];
            ok = wait_neighbours(d, e.y % d.geo.nbands, e.y / d.geo.nbands, s, done, ctl, &ok_lds);
            if (!ok) break;
            persist_tile<M>(d, e, s, phase0, phs);
            if (threadIdx.x == 0)
                __hip_atomic_store(done + d.done_off + e.y, s + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!ok) break;
    }
}

// Resets the control block and the step counters before a persistent launch (a kernel, not a
// memset, so that the launch sequence stays free of memset nodes).
__global__ void k_persist_reset(PersistCtl *ctl, int *done, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        ctl->next = 0;
        ctl->bar_count = 0;
        ctl->bar_gen = 0;
        ctl->abort = 0;
    }
    for (int j = i; j < n; j += gridDim.x * blockDim.x) done[j] = 0;
}

// ------------------------------------------------------------------------------------------
// initialisation.  k_equilibria computes the equilibria of the given macroscopic planes into
// a post-streaming state (9 + 9 planes, node-local, storage types); k_unstream stores them in
// pull layout: P[i](z) = F[i](z + c_i), or F[opp(i)](z) where z + c_i is behind a wall.

__device__ __forceinline__ double plane_at(const double *p, int nx, int ny, bool walls, double wgrad, int x, int y)
{
    x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
    if (walls) {
        if (y < 0) return p[x] - wgrad;
        if (y >= ny) return p[(size_t)(ny - 1) * nx + x] - wgrad;
    } else {
        y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
    }
    return p[(size_t)y * nx + x];
}

template <class R>
__global__ void k_equilibria(const double *__restrict__ phi0, const double *__restrict__ rho0,
                             const double *__restrict__ ux0, const double *__restrict__ uy0,
                             SetView F, SetView G, Geo geo, Phys<R> c)
{
    const int nx = geo.nx, ny = geo.ny;
    const size_t N = geo.plane;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(n / nx), x = (int)(n % nx);
        const bool wl = geo.walls != 0;
        double nb[3][3];
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) nb[dy + 1][dx + 1] = plane_at(phi0, nx, ny, wl, geo.wgrad, x + dx, y + dy);
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
            view_st(F, i, n, (double)fe[i]);
            view_st(G, i, n, (double)ge[i]);
        }
    }
}

__global__ void k_unstream(SetView F, SetView P, Geo geo, bool is_g)
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
        if (ys < 0 || ys >= ny) {
            if (geo.walls) {
                // the pull returns this value in direction opp(i) with the moving-wall term
                // added: store it without that term
                double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                const int j = kOpp[i];
                double s = 1.0;
                if (is_g) {
                    s = 0;
                    for (int k = 0; k < 9; ++k) s += view_ld(F, k, n);
                }
                wall_motion(v, s, y == 0 && ys < 0, y == ny - 1 && ys >= ny, geo.ub6, geo.ut6);
                view_st(P, i, n, view_ld(F, j, n) - v[j]);
                continue;
            }
            ys = ys < 0 ? ys + ny : ys - ny;
        }
        view_copy(F, i, (size_t)ys * nx + xs, P, i, n);
    }
}

// ------------------------------------------------------------------------------------------
// readers: post-streaming populations, macroscopic fields and FP64 reductions (in double).

__global__ void k_fields(SetView f, SetView g, Geo geo, double a, double hFx, double hFy, double *phi,
                         double *rho, double *ux, double *uy, double *p0)
{
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < geo.plane;
         n += (size_t)gridDim.x * blockDim.x) {
        double fv[9], gv[9];
        pull_node(f, geo, n, fv, false);
        pull_node(g, geo, n, gv, true);
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
__global__ void k_population(SetView f, SetView g, Geo geo, int which, double *out)
{
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < geo.plane;
         n += (size_t)gridDim.x * blockDim.x) {
        double v[9];
        pull_node(which < 9 ? f : g, geo, n, v, which >= 9);
        out[n] = which < 9 ? v[which] + kW[which] : v[which - 9];
    }
}

// max-type fields of the diagnostics (the others are sums)
__device__ __forceinline__ bool diag_is_max(int k) { return k == 5 || k == 7; }

// FP64 reductions of one state (f, g); with have_prev also the largest change of v against the
// previous state (pf), max |v(t) - v(t - 1)|.  Each block writes its kDiagFields partials.
__global__ __launch_bounds__(kReduceThreads) void k_diag(SetView f, SetView g, SetView pf, int have_prev, Geo geo,
                                                         double hFx, double hFy, double *partial)
{
    double acc[kDiagFields] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < geo.plane;
         n += (size_t)gridDim.x * blockDim.x) {
        double fv[9], gv[9];
        pull_node(f, geo, n, fv, false);
        pull_node(g, geo, n, gv, true);
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
        if (have_prev) {
            double qv[9];
            pull_node(pf, geo, n, qv, false);
            const double rp = 1.0 + sum9(qv);
            const double jxp = (qv[1] + qv[5] + qv[8]) - (qv[3] + qv[6] + qv[7]) + hFx;
            const double jyp = (qv[2] + qv[5] + qv[6]) - (qv[4] + qv[7] + qv[8]) + hFy;
            const double dx = jx / r - jxp / rp, dy = jy / r - jyp / rp;
            acc[7] = fmax(acc[7], sqrt(dx * dx + dy * dy));  // fmax drops a NaN of the previous state
        }
    }
    __shared__ double red[kDiagFields][kReduceThreads];
    for (int k = 0; k < kDiagFields; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kReduceThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < kDiagFields; ++k)
                red[k][threadIdx.x] = diag_is_max(k) ? fmax(red[k][threadIdx.x], red[k][threadIdx.x + s])
                                                     : red[k][threadIdx.x] + red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < kDiagFields) partial[blockIdx.x * kDiagFields + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kReduceThreads) void k_diag_finish(const double *partial, int nblocks,
                                                                double *out)
{
    __shared__ double red[kDiagFields][kReduceThreads];
    double acc[kDiagFields] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += kReduceThreads)
        for (int k = 0; k < kDiagFields; ++k) {
            const double v = partial[b * kDiagFields + k];
            acc[k] = diag_is_max(k) ? fmax(acc[k], v) : acc[k] + v;
        }
    for (int k = 0; k < kDiagFields; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kReduceThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < kDiagFields; ++k)
                red[k][threadIdx.x] = diag_is_max(k) ? fmax(red[k][threadIdx.x], red[k][threadIdx.x + s])
                                                     : red[k][threadIdx.x] + red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < kDiagFields) out[threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_clear_int(int *p) { *p = 0; }

// Streaming reference: PLANES planes of n floats read and written to PLANES other planes, one
// element per lane and one launch over all elements (the access pattern of the step kernel
// without its shifted pulls, halo reads and arithmetic), non-temporal stores like the step's.
template <int PLANES>
__global__ __launch_bounds__(512) void k_stream(const float *__restrict__ src, float *__restrict__ dst, uint32_t n)
{
    const uint32_t i = blockIdx.x * 512u + threadIdx.x;
    if (i >= n) return;
    float v[PLANES];
#pragma unroll
    for (int p = 0; p < PLANES; ++p) v[p] = src[(size_t)p * n + i];
#pragma unroll
    for (int p = 0; p < PLANES; ++p) __builtin_nontemporal_store(v[PLANES - 1 - p], &dst[(size_t)p * n + i]);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Device scratch of lbcm_diag_state, the allocation-free diagnostics: the partial sums of
// k_diag (kReduceBlocks blocks of kDiagFields doubles) and the kDiagFields results of
// k_diag_finish, 65,600 bytes whatever the lattice size (the kernels stride over the nodes).
// Every GPU the library runs on holds its own copy until the process ends.  Host code never
// uses this name as an address: it asks the runtime for the copy of the current device
// (scratch_address) and passes that pointer.
constexpr size_t kScratchDoubles = (size_t)kReduceBlocks * kDiagFields + kDiagFields;
static __device__ __align__(256) double scratch[kScratchDoubles];

// ==========================================================================================
// host side

struct lbcm_handle {
    lbcm_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    size_t fset = 0, gset = 0;  // bytes of the f and g sets
    size_t fset_al = 0;         // f set bytes rounded up to the alignment (offset of the g set)
    size_t pair_bytes = 0;      // bytes of one (f, g) pair
    char *ws = nullptr;         // workspace base
    bool owns_ws = false;
    int cur = 0;                // pair holding the current state
    bool ready = false;
    bool prev_ok = false;       // the spare pair holds the state one step before the current one
    int64_t step = 0;
    double *diag_partial = nullptr;
    double *diag_out = nullptr;
    int *flag = nullptr;
    std::string err;
};

namespace {

std::string g_create_error;

// Device address of `scratch` on each device, looked up once per device (with that device
// current) on the first lbcm_diag_state call there.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int dev, double **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// element kinds of the f planes, of g_0 and of g_1..g_8
struct Kinds {
    int f, g0, g;
};
bool kinds_of(int precision, Kinds &k)
{
    switch (precision) {
    case LBCM_FP64: k = {kKindF64, kKindF64, kKindF64}; return true;
    case LBCM_FP32: k = {kKindF32, kKindF32, kKindF32}; return true;
    case LBCM_FP16_SHIFTED: k = {kKindF16, kKindF32, kKindF16}; return true;
    case LBCM_BF16_SHIFTED: k = {kKindB16, kKindF32, kKindB16}; return true;
    default: return false;
    }
}
size_t kind_bytes(int kind) { return kind == kKindF64 ? 8 : (kind == kKindF32 ? 4 : 2); }

void set_sizes(const lbcm_params *p, size_t &fset, size_t &gset)
{
    Kinds k;
    kinds_of(p->precision, k);
    const size_t N = (size_t)p->nx * (size_t)p->ny;
    fset = 9 * N * kind_bytes(k.f);
    gset = N * kind_bytes(k.g0) + 8 * N * kind_bytes(k.g);
}

const char *check_params(const lbcm_params *p)
{
    if (!p) return "params is NULL";
    if (p->nx < 1 || p->ny < 1) return "nx and ny must be >= 1";
    if (p->bc_y != LBCM_BC_PERIODIC && p->bc_y != LBCM_BC_WALLS) return "bc_y must be 0 or 1";
    Kinds k;
    if (!kinds_of(p->precision, k)) return "unsupported precision";
    const double N = (double)p->nx * (double)p->ny;
    const double per_node = std::max(9.0 * (double)kind_bytes(k.f), (double)kind_bytes(k.g0) + 8.0 * kind_bytes(k.g));
    if (N * per_node > 4294967295.0) return "lattice too large: one population set (9 planes) must stay below 4 GiB";
    if (!(p->nu_l > 0) || !(p->nu_g > 0)) return "viscosities must be > 0";
    if (!(p->mobility > 0) || !(p->Gamma > 0)) return "mobility and Gamma must be > 0";
    if (!(p->omega3 > 0 && p->omega3 < 2)) return "omega3 must lie in (0, 2)";
    if (!std::isfinite(p->a) || !std::isfinite(p->gamma) || !std::isfinite(p->force_x) ||
        !std::isfinite(p->force_y))
        return "a, gamma and the force must be finite";
    if (!std::isfinite(p->wall_vx_bottom) || !std::isfinite(p->wall_vx_top) || !std::isfinite(p->wall_gradient))
        return "the wall velocities and the wall gradient must be finite";
    if (p->k8_variant != 0 && p->k8_variant != 1) return "k8_variant must be 0 or 1";
    if (p->check_every < 0) return "check_every must be >= 0";
    if (p->tile_rows < 0 || p->tile_wx < 0) return "tile_rows and tile_wx must be >= 0";
    return nullptr;
}

size_t pair_bytes_of(const lbcm_params *p)
{
    size_t fs, gs;
    set_sizes(p, fs, gs);
    return align_up(fs) + align_up(gs);
}

size_t tail_bytes()
{
    return align_up(kReduceBlocks * kDiagFields * sizeof(double)) + align_up(kDiagFields * sizeof(double)) + kAlign;
}

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
    c.ub6 = (R)(p.wall_vx_bottom / 6.0);
    c.ut6 = (R)(p.wall_vx_top / 6.0);
    c.wgrad = (R)p.wall_gradient;
    c.k8_printed = p.k8_variant;
    return c;
}

bool large_lattice(const lbcm_params &p)
{
    return (size_t)p.nx * p.ny >= (p.precision == LBCM_FP32 ? kLargeNodes32 : kLargeNodes);
}

// Lattice rows per wave of the single-lattice step kernel: two with 16-bit storage on large
// lattices, where the step is bandwidth-bound; one otherwise (on small, latency-bound lattices a
// wave's second row only lengthens the critical path).
int rows_per_wave(const lbcm_params &p)
{
    const bool b16 = p.precision == LBCM_FP16_SHIFTED || p.precision == LBCM_BF16_SHIFTED;
    return b16 && large_lattice(p) ? ModeF16::kRpw : 1;
}

// LDS of one step tile: its phi with a one-node halo
size_t tile_lds_bytes(const Geo &g, size_t elem) { return (size_t)(g.rows * g.rpw + 2) * (64 * g.wx + 2) * elem; }

// geometry of the step tiles; rpw: lattice rows per wave row of the kernel that runs them
Geo make_geo(const lbcm_params &p, int rpw)
{
    Geo g;
    g.nx = p.nx;
    g.ny = p.ny;
    g.plane = (uint32_t)((size_t)p.nx * p.ny);
    const int max_waves = (p.precision == LBCM_FP64 ? 512 : 1024) / 64;
    const int need = (p.nx + 63) / 64;
    g.rpw = rpw;
    const bool f64 = p.precision == LBCM_FP64, large = large_lattice(p);
    const int dwx = !large ? kDefaultWx : f64 ? kLargeWx64 : g.rpw == 2 ? kLargeWx16 : kLargeWx;
    const int drows = !large ? kDefaultRows : f64 ? kLargeRows64 : g.rpw == 2 ? kLargeRows16 : kLargeRows;
    g.wx = p.tile_wx > 0 ? p.tile_wx : dwx;
    if (g.wx > need) g.wx = need;
    if (g.wx > max_waves) g.wx = max_waves;
    int rows = p.tile_rows > 0 ? p.tile_rows : drows;
    if (rows > max_waves / g.wx) rows = max_waves / g.wx;
    if (rows > (p.ny + g.rpw - 1) / g.rpw) rows = (p.ny + g.rpw - 1) / g.rpw;
    g.rows = rows;
    g.nbands = (p.nx + 64 * g.wx - 1) / (64 * g.wx);
    g.nrows = (p.ny + g.rows * g.rpw - 1) / (g.rows * g.rpw);
    g.walls = p.bc_y;
    g.ub6 = p.wall_vx_bottom / 6.0;
    g.ut6 = p.wall_vx_top / 6.0;
    g.wgrad = p.wall_gradient;
    return g;
}

// the single-lattice kernel's geometry (the storage mode's rows per wave)
Geo make_geo(const lbcm_params &p) { return make_geo(p, rows_per_wave(p)); }

unsigned char *set_base(lbcm_handle *h, int pair, int set)  // set 0 = f, 1 = g
{
    return reinterpret_cast<unsigned char *>(h->ws + (size_t)pair * h->pair_bytes + (set ? h->fset_al : 0));
}

SetView view_of(lbcm_handle *h, int pair, int set)
{
    Kinds k;
    kinds_of(h->p.precision, k);
    const size_t N = (size_t)h->p.nx * h->p.ny;
    SetView v;
    v.base = set_base(h, pair, set);
    const int k0 = set ? k.g0 : k.f, k1 = set ? k.g : k.f;
    for (int i = 0; i < 9; ++i) {
        v.kind[i] = i == 0 ? k0 : k1;
        v.off[i] = (uint32_t)(i == 0 ? 0 : N * kind_bytes(k0) + (size_t)(i - 1) * N * kind_bytes(k1));
    }
    return v;
}

int grid_for(size_t n, int threads)
{
    size_t b = (n + threads - 1) / threads;
    if (b > 65535) b = 65535;
    if (b < 1) b = 1;
    return (int)b;
}

// One launch of the step kernel for the tile geometry geo (its rows per wave: 1 or the mode's kRpw).
template <class M, int RPW>
void launch_k_step_rpw(const Geo &geo, const Phys<typename M::R> &c, bool walls, bool force, size_t lds, hipStream_t st,
                       const unsigned char *fa, const unsigned char *ga, unsigned char *fb, unsigned char *gb, int *flag)
{
    const dim3 grid((unsigned)(geo.nbands * geo.nrows)), block(64 * geo.wx * geo.rows);
    if (walls) {
        if (force) hipLaunchKernelGGL((k_step<M, RPW, true, true>), grid, block, lds, st, fa, ga, fb, gb, geo, c, flag);
        else hipLaunchKernelGGL((k_step<M, RPW, true, false>), grid, block, lds, st, fa, ga, fb, gb, geo, c, flag);
    } else {
        if (force) hipLaunchKernelGGL((k_step<M, RPW, false, true>), grid, block, lds, st, fa, ga, fb, gb, geo, c, flag);
        else hipLaunchKernelGGL((k_step<M, RPW, false, false>), grid, block, lds, st, fa, ga, fb, gb, geo, c, flag);
    }
}
template <class M>
void launch_k_step(const Geo &geo, const Phys<typename M::R> &c, bool walls, bool force, size_t lds, hipStream_t st,
                   const unsigned char *fa, const unsigned char *ga, unsigned char *fb, unsigned char *gb, int *flag)
{
    if (geo.rpw == 1) launch_k_step_rpw<M, 1>(geo, c, walls, force, lds, st, fa, ga, fb, gb, flag);
    else launch_k_step_rpw<M, M::kRpw>(geo, c, walls, force, lds, st, fa, ga, fb, gb, flag);
}

template <class M> int launch_steps(lbcm_handle *h, int64_t nsteps)
{
    using R = typename M::R;
    const Geo geo = make_geo(h->p);
    const Phys<R> c = make_phys<R>(h->p);
    const bool walls = h->p.bc_y == LBCM_BC_WALLS;
    const bool force = h->p.force_x != 0 || h->p.force_y != 0;
    const int64_t nblk = (int64_t)geo.nbands * geo.nrows;
    if (nblk > 0x7fffffff) return fail(h, LBCM_EINVAL, "too many tiles");
    if (geo.rpw != 1 && geo.rpw != M::kRpw) return fail(h, LBCM_EINVAL, "tile geometry does not match the storage mode");
    const size_t lds = tile_lds_bytes(geo, sizeof(R));
    for (int64_t s = 0; s < nsteps; ++s) {
        const unsigned char *fa = set_base(h, h->cur, 0), *ga = set_base(h, h->cur, 1);
        unsigned char *fb = set_base(h, 1 - h->cur, 0), *gb = set_base(h, 1 - h->cur, 1);
        launch_k_step<M>(geo, c, walls, force, lds, h->stream, fa, ga, fb, gb, h->flag);
        HIP_TRY(h, hipGetLastError());
        h->cur = 1 - h->cur;
        h->step += 1;
        h->prev_ok = true;
        if (h->p.check_every > 0 && ((s + 1) % h->p.check_every == 0 || s + 1 == nsteps)) {
            int flag = 0;
            HIP_TRY(h, hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            if (flag) return fail(h, LBCM_EDIVERGED, "non-finite rho or phi detected at step " + std::to_string(h->step));
        }
    }
    return LBCM_OK;
}

// Time `trials` launches of the step kernel with tile shape (wx, rows) and rpw rows per wave (1 or
// the mode's kRpw) that read the current pair and write the spare one (the state is left as it
// was).  Returns ms per launch, < 0 on error.
template <class M> float time_tiles(lbcm_handle *h, int wx, int rows, int rpw, int trials)
{
    using R = typename M::R;
    lbcm_params q = h->p;
    q.tile_wx = wx;
    q.tile_rows = rows;
    const Geo geo = make_geo(q, rpw);
    const Phys<R> c = make_phys<R>(q);
    const bool walls = q.bc_y == LBCM_BC_WALLS, force = q.force_x != 0 || q.force_y != 0;
    const size_t lds = tile_lds_bytes(geo, sizeof(R));
    const unsigned char *fa = set_base(h, h->cur, 0), *ga = set_base(h, h->cur, 1);
    unsigned char *fb = set_base(h, 1 - h->cur, 0), *gb = set_base(h, 1 - h->cur, 1);
    h->prev_ok = false;  // the timed launches overwrite the spare pair
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1;
    }
    float ms = -1;
    for (int pass = 0; pass < 2; ++pass) {  // pass 0 warms up
        if (pass == 1 && hipEventRecord(e0, h->stream) != hipSuccess) break;
        for (int s = 0; s < (pass ? trials : 1); ++s)
            launch_k_step<M>(geo, c, walls, force, lds, h->stream, fa, ga, fb, gb, h->flag);
        if (hipGetLastError() != hipSuccess) break;
        if (pass == 1 && hipEventRecord(e1, h->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            ms /= (float)trials;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

int max_waves_of(int precision) { return precision == LBCM_FP64 ? 8 : 16; }

// Candidate tile shapes (wx, rows) for a lattice: wx a power of two up to the lattice width,
// wx * rows == waves (or every split up to waves when waves == 0).
std::vector<std::pair<int, int>> tile_candidates(const lbcm_params &p, int waves)
{
    std::vector<std::pair<int, int>> out;
    const int need = (p.nx + 63) / 64, mw = max_waves_of(p.precision);
    for (int wx = 1; wx <= mw; wx *= 2) {
        if (wx > need && wx > 1) break;
        // wave rows: powers of two, and 3 times them (3 rows is the best height of the large
        // FP32 and 16-bit steps)
        for (int rows : {1, 2, 3, 4, 6, 8, 12, 16}) {
            if (wx * rows > mw) break;
            if (rows > p.ny && rows > 1) break;
            if (waves == 0 || wx * rows == waves) out.push_back({wx, rows});
        }
    }
    if (out.empty()) out.push_back({1, 1});
    return out;
}

template <class M>
int do_init(lbcm_handle *h, const double *phi0, const double *rho0, const double *ux0, const double *uy0)
{
    using R = typename M::R;
    const Geo geo = make_geo(h->p);
    const Phys<R> c = make_phys<R>(h->p);
    // equilibria into the spare pair, then un-stream into pair 0
    const SetView F = view_of(h, 1, 0), G = view_of(h, 1, 1);
    const int gb = grid_for(geo.plane, 256);
    hipLaunchKernelGGL((k_equilibria<R>), dim3(gb), dim3(256), 0, h->stream, phi0, rho0, ux0, uy0, F, G, geo, c);
    HIP_TRY(h, hipGetLastError());
    const int gu = grid_for(9 * (size_t)geo.plane, 256);
    hipLaunchKernelGGL(k_unstream, dim3(gu), dim3(256), 0, h->stream, F, view_of(h, 0, 0), geo, false);
    HIP_TRY(h, hipGetLastError());
    hipLaunchKernelGGL(k_unstream, dim3(gu), dim3(256), 0, h->stream, G, view_of(h, 0, 1), geo, true);
    HIP_TRY(h, hipGetLastError());
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(1), 0, h->stream, h->flag);
    HIP_TRY(h, hipGetLastError());
    h->cur = 0;
    h->step = 0;
    h->ready = true;
    h->prev_ok = false;
    return LBCM_OK;
}

int do_fields(lbcm_handle *h, double *phi, double *rho, double *ux, double *uy, double *p0)
{
    const Geo geo = make_geo(h->p);
    const int gb = grid_for(geo.plane, 256);
    hipLaunchKernelGGL(k_fields, dim3(gb), dim3(256), 0, h->stream, view_of(h, h->cur, 0), view_of(h, h->cur, 1), geo,
                       h->p.a, 0.5 * h->p.force_x, 0.5 * h->p.force_y, phi, rho, ux, uy, p0);
    HIP_TRY(h, hipGetLastError());
    return LBCM_OK;
}

int do_population(lbcm_handle *h, int which, double *out)
{
    const Geo geo = make_geo(h->p);
    const int gb = grid_for(geo.plane, 256);
    hipLaunchKernelGGL(k_population, dim3(gb), dim3(256), 0, h->stream, view_of(h, h->cur, 0), view_of(h, h->cur, 1),
                       geo, which, out);
    HIP_TRY(h, hipGetLastError());
    return LBCM_OK;
}

int do_diag(lbcm_handle *h)
{
    const Geo geo = make_geo(h->p);
    hipLaunchKernelGGL(k_diag, dim3(kReduceBlocks), dim3(kReduceThreads), 0, h->stream, view_of(h, h->cur, 0),
                       view_of(h, h->cur, 1), view_of(h, 1 - h->cur, 0), (int)h->prev_ok, geo, 0.5 * h->p.force_x,
                       0.5 * h->p.force_y, h->diag_partial);
    HIP_TRY(h, hipGetLastError());
    hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(kReduceThreads), 0, h->stream, h->diag_partial, kReduceBlocks,
                       h->diag_out);
    HIP_TRY(h, hipGetLastError());
    return LBCM_OK;
}

// host-side dispatch on the storage mode
template <class Fn> int dispatch(lbcm_handle *h, Fn &&fn)
{
    switch (h->p.precision) {
    case LBCM_FP64: return fn(ModeF64{});
    case LBCM_FP32: return fn(ModeF32{});
    case LBCM_FP16_SHIFTED: return fn(ModeF16{});
    case LBCM_BF16_SHIFTED: return fn(ModeB16{});
    default: return fail(h, LBCM_EINVAL, "unsupported precision");
    }
}

}  // namespace

// ------------------------------------------------------------------------------------------
// ensembles

struct lbcm_batch {
    int n = 0;
    int precision = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    char *arena = nullptr;
    std::vector<lbcm_handle *> box;
    std::vector<int> wx, rows;     // tile shape of each box in the batched launch
    int waves = 16;                // waves per workgroup of the batched launch
    int order = 1;                 // 0: tiles in box order, 1: largest boxes first, 2: one XCD per box
    void *d_desc = nullptr;        // BoxDesc table
    int2 *d_tiles = nullptr;       // grid index -> (box, tile of the box), box -1: empty slot
    int *flag = nullptr;
    int ntiles = 0;                // tiles of all boxes
    int grid = 0;                  // workgroups of the batched launch (tiles and empty slots)
    size_t lds = 0;
    std::vector<int> base_cur;     // pair that was current in each box when the table was built
    int phase = 0;                 // steps taken since the table was built, mod 2
    bool use_graph = true;
    bool graph_ok = false;
    hipGraphExec_t gexec = nullptr;
    int persist = 0;               // 0: one launch per step; kPersistBarrier / kPersistDataflow
    void *d_ctl = nullptr;         // PersistCtl of the persistent launch
    int *d_done = nullptr;         // per-tile step counters of the dataflow schedule
    int ndone = 0;
    int persist_grid = 0;          // workgroups of the persistent launch (resident count)
    std::string err;
};

namespace {

int bfail(lbcm_batch *b, int code, const std::string &msg)
{
    if (b) b->err = msg;
    return code;
}

#define BHIP_TRY(b, call)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return bfail(b, LBCM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

void drop_graph(lbcm_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->graph_ok = false;
}

// (Re)build the descriptor and tile tables from the current state of every box.
template <class M> int build_tables(lbcm_batch *b)
{
    using R = typename M::R;
    std::vector<int> idx(b->n);
    for (int i = 0; i < b->n; ++i) idx[i] = i;
    if (b->order >= 1)
        std::stable_sort(idx.begin(), idx.end(), [&](int u, int v) {
            return (size_t)b->box[u]->p.nx * b->box[u]->p.ny > (size_t)b->box[v]->p.nx * b->box[v]->p.ny;
        });
    std::vector<BoxDesc<R>> desc(b->n);
    std::vector<std::vector<int2>> streams(b->order == 2 ? kXcds : 1);
    std::vector<size_t> load(streams.size(), 0);
    size_t ntiles = 0, lds = 0;
    b->base_cur.assign(b->n, 0);
    for (int i : idx) {
        lbcm_handle *h = b->box[i];
        if (!h->ready) return bfail(b, LBCM_ESTATE, "box " + std::to_string(i) + " is not initialised");
        lbcm_params q = h->p;
        q.tile_wx = b->wx[i];
        q.tile_rows = b->rows[i];
        BoxDesc<R> &d = desc[i];
        d.geo = make_geo(q, 1);  // the batched kernel updates one row per wave in every mode
        if (d.geo.wx * d.geo.rows > b->waves) return bfail(b, LBCM_EINVAL, "tile larger than the workgroup");
        d.c = make_phys<R>(q);
        b->base_cur[i] = h->cur;
        for (int k = 0; k < 2; ++k) {
            d.set[k][0] = set_base(h, h->cur ^ k, 0);
            d.set[k][1] = set_base(h, h->cur ^ k, 1);
        }
        d.flag = h->flag;
        d.done_off = 0;
        d.walls = q.bc_y == LBCM_BC_WALLS;
        d.force = q.force_x != 0 || q.force_y != 0;
        const size_t nt = (size_t)d.geo.nbands * d.geo.nrows;
        ntiles += nt;
        if (ntiles > 0x7fffffff / kXcds) return bfail(b, LBCM_EINVAL, "too many tiles");
        // the least-loaded stream takes the box (with one stream: every box in turn)
        const size_t s = std::min_element(load.begin(), load.end()) - load.begin();
        for (size_t t = 0; t < nt; ++t) streams[s].push_back(make_int2(i, (int)t));
        load[s] += nt;
        lds = std::max(lds, tile_lds_bytes(d.geo, sizeof(R)));
    }
    // grid index g = kXcds k + x runs tile k of stream x: workgroups are dealt to the XCDs in
    // turn, so each stream's tiles run on one XCD (order 2); with one stream the grid is the
    // boxes' tiles back to back
    std::vector<int2> tiles;
    if (streams.size() == 1) {
        tiles = std::move(streams[0]);
    } else {
        const size_t len = *std::max_element(load.begin(), load.end());
        tiles.assign(len * streams.size(), make_int2(-1, 0));
        for (size_t x = 0; x < streams.size(); ++x)
            for (size_t k = 0; k < streams[x].size(); ++k) tiles[k * streams.size() + x] = streams[x][k];
    }
    // step counters of the persistent dataflow schedule: one per tile, box after box
    int ndone = 0;
    for (int i = 0; i < b->n; ++i) {
        desc[i].done_off = ndone;
        ndone += desc[i].geo.nbands * desc[i].geo.nrows;
    }
    drop_graph(b);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_done) (void)hipFree(b->d_done);
    b->d_desc = nullptr;
    b->d_tiles = nullptr;
    b->d_done = nullptr;
    b->persist_grid = 0;
    BHIP_TRY(b, hipMalloc((void **)&b->d_done, (size_t)std::max(ndone, 1) * sizeof(int)));
    b->ndone = ndone;
    if (!b->d_ctl) BHIP_TRY(b, hipMalloc(&b->d_ctl, sizeof(PersistCtl)));
    BHIP_TRY(b, hipMalloc(&b->d_desc, desc.size() * sizeof(BoxDesc<R>)));
    BHIP_TRY(b, hipMalloc((void **)&b->d_tiles, tiles.size() * sizeof(int2)));
    BHIP_TRY(b, hipMemcpyAsync(b->d_desc, desc.data(), desc.size() * sizeof(BoxDesc<R>), hipMemcpyHostToDevice, b->stream));
    BHIP_TRY(b, hipMemcpyAsync(b->d_tiles, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    b->ntiles = (int)ntiles;
    b->grid = (int)tiles.size();
    b->lds = lds;
    b->phase = 0;
    return LBCM_OK;
}

bool tables_stale(lbcm_batch *b)
{
    if (!b->d_desc) return true;
    for (int i = 0; i < b->n; ++i)
        if (b->box[i]->cur != (b->base_cur[i] ^ b->phase)) return true;
    return false;
}

template <class M> void launch_batch(lbcm_batch *b, int phase)
{
    hipLaunchKernelGGL((k_step_batch<M>), dim3(b->grid), dim3(64 * b->waves), b->lds, b->stream,
                       (const BoxDesc<typename M::R> *)b->d_desc, b->d_tiles, phase);
}

void advance_boxes(lbcm_batch *b, int64_t steps)
{
    for (lbcm_handle *h : b->box) {
        h->cur ^= (int)(steps & 1);
        h->step += steps;
        if (steps > 0) h->prev_ok = true;
    }
    b->phase ^= (int)(steps & 1);
}

// Divergence check of an ensemble: synchronises and returns LBCM_EDIVERGED if any box's flag is
// set (the flags are cleared by lbcm_init, lbcm_set_state and lbcm_copy_state of that box).
template <class M> int check_batch(lbcm_batch *b)
{
    hipLaunchKernelGGL((k_batch_flags<typename M::R>), dim3(1), dim3(kReduceThreads), 0, b->stream,
                       (const BoxDesc<typename M::R> *)b->d_desc, b->n, b->flag);
    BHIP_TRY(b, hipGetLastError());
    int v[2] = {0, 0};
    BHIP_TRY(b, hipMemcpyAsync(v, b->flag, sizeof v, hipMemcpyDeviceToHost, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    if (v[0])
        return bfail(b, LBCM_EDIVERGED,
                     "non-finite rho or phi in " + std::to_string(v[0]) + " box(es), the first of them box " +
                         std::to_string(v[1]) + ", by step " + std::to_string(b->box[v[1]]->step));
    return LBCM_OK;
}

// One persistent launch advancing every box by nsteps (1 <= nsteps < 2^30); synchronises to read
// the give-up flag.
template <class M> int persist_launch(lbcm_batch *b, int nsteps)
{
    using R = typename M::R;
    const unsigned threads = 64u * (unsigned)b->waves;
    if (!b->persist_grid) {
        int dev = 0, cus = 0, per_cu = 0;
        BHIP_TRY(b, hipGetDevice(&dev));
        BHIP_TRY(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        BHIP_TRY(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_step_persist<M>, (int)threads,
                                                                 b->lds));
        if (per_cu < 1) return bfail(b, LBCM_EINVAL, "persistent launch: the workgroup does not fit on a CU");
        b->persist_grid = per_cu * cus;
    }
    PersistCtl *ctl = (PersistCtl *)b->d_ctl;
    hipLaunchKernelGGL(k_persist_reset, dim3(grid_for((size_t)b->ndone, 256)), dim3(256), 0, b->stream, ctl, b->d_done,
                       b->ndone);
    BHIP_TRY(b, hipGetLastError());
    const BoxDesc<R> *boxes = (const BoxDesc<R> *)b->d_desc;
    const int2 *tiles = b->d_tiles;
    int ntiles = b->grid, steps = nsteps, phase0 = b->phase, mode = b->persist;
    int *done = b->d_done;
    unsigned nwg = (unsigned)b->persist_grid;
    if (mode == kPersistBarrier) {
        void *args[] = {&boxes, &tiles, &ntiles, &steps, &phase0, &mode, &ctl, &done, &nwg};
        BHIP_TRY(b, hipLaunchCooperativeKernel((const void *)k_step_persist<M>, dim3(nwg), dim3(threads), args, b->lds,
                                               b->stream));
    } else {
        hipLaunchKernelGGL((k_step_persist<M>), dim3(nwg), dim3(threads), b->lds, b->stream, boxes, tiles, ntiles, steps,
                           phase0, mode, ctl, done, nwg);
        BHIP_TRY(b, hipGetLastError());
    }
    advance_boxes(b, nsteps);
    int gave_up = 0;
    BHIP_TRY(b, hipMemcpyAsync(&gave_up, &ctl->abort, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    if (gave_up)
        return bfail(b, LBCM_EHIP, "persistent launch: a wait gave up; the boxes' state is undefined");
    return LBCM_OK;
}

template <class M> int batch_steps(lbcm_batch *b, int64_t nsteps)
{
    if (tables_stale(b)) {
        int rc = build_tables<M>(b);
        if (rc) return rc;
    }
    // divergence checks: every `every` steps (the shortest positive check_every of the boxes)
    // and at the end of the call
    int every = 0;
    for (lbcm_handle *h : b->box)
        if (h->p.check_every > 0) every = every ? std::min(every, h->p.check_every) : h->p.check_every;
    if (b->persist) {
        // one launch per chunk: the whole call, or the steps between two divergence checks
        const int64_t chunk = std::min<int64_t>(every > 0 ? every : nsteps, int64_t(1) << 29);
        for (int64_t s = 0; s < nsteps; s += chunk) {
            const int k = (int)std::min(chunk, nsteps - s);
            if (int rc = persist_launch<M>(b, k)) return rc;
            if (every > 0)
                if (int rc = check_batch<M>(b)) return rc;
        }
        return LBCM_OK;
    }
    int64_t s = 0, since = 0;
    auto checked = [&](int64_t k) -> int {  // k steps were just queued
        advance_boxes(b, k);
        s += k;
        since += k;
        if (every <= 0 || (since < every && s < nsteps)) return LBCM_OK;
        since = 0;
        return check_batch<M>(b);
    };
    if (b->phase == 1 && s < nsteps) {  // get to an even phase for the two-step graph
        launch_batch<M>(b, 1);
        BHIP_TRY(b, hipGetLastError());
        if (int rc = checked(1)) return rc;
    }
    if (b->use_graph && nsteps - s >= 2) {
        if (!b->graph_ok) {
            hipGraph_t g = nullptr;
            BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            launch_batch<M>(b, 0);
            launch_batch<M>(b, 1);
            hipError_t e = hipStreamEndCapture(b->stream, &g);
            if (e != hipSuccess) return bfail(b, LBCM_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return bfail(b, LBCM_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            b->graph_ok = true;
        }
        while (s + 2 <= nsteps) {
            BHIP_TRY(b, hipGraphLaunch(b->gexec, b->stream));
            if (int rc = checked(2)) return rc;
        }
    }
    while (s < nsteps) {
        launch_batch<M>(b, b->phase);
        BHIP_TRY(b, hipGetLastError());
        if (int rc = checked(1)) return rc;
    }
    return LBCM_OK;
}

// ms per batched launch that reads the current pairs and writes the spare ones (state unchanged)
template <class M> float time_batch(lbcm_batch *b, int trials)
{
    if (tables_stale(b) && build_tables<M>(b) != LBCM_OK) return -1;
    for (lbcm_handle *h : b->box) h->prev_ok = false;  // the timed launches overwrite the spare pairs
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1;
    }
    float ms = -1;
    launch_batch<M>(b, b->phase);
    if (hipEventRecord(e0, b->stream) == hipSuccess) {
        for (int t = 0; t < trials; ++t) launch_batch<M>(b, b->phase);
        if (hipGetLastError() == hipSuccess && hipEventRecord(e1, b->stream) == hipSuccess &&
            hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            ms /= (float)trials;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

template <class M> int batch_autotune(lbcm_batch *b, int trials)
{
    // per box size and per workgroup size: the fastest tile split of that many waves
    const int mw = max_waves_of(b->precision);
    float best_ms = -1;
    std::vector<int> best_wx, best_rows;
    int best_waves = 0, best_order = 0;
    for (int waves : {mw / 2, 3 * mw / 4, mw}) {  // 8, 12, 16 waves (FP64: 4, 6, 8)
        std::vector<int> wx(b->n, 1), rows(b->n, 1);
        std::vector<std::pair<std::pair<int, int>, std::pair<int, int>>> memo;  // (nx, ny) -> (wx, rows)
        for (int i = 0; i < b->n; ++i) {
            lbcm_handle *h = b->box[i];
            auto key = std::make_pair(h->p.nx, h->p.ny);
            auto it = std::find_if(memo.begin(), memo.end(), [&](auto &m) { return m.first == key; });
            if (it == memo.end()) {
                float bms = -1;
                std::pair<int, int> bc{1, waves};
                for (auto cand : tile_candidates(h->p, waves)) {
                    const float ms = time_tiles<M>(h, cand.first, cand.second, 1, trials);
                    if (ms < 0) return bfail(b, LBCM_EHIP, "timing a tile shape failed");
                    if (bms < 0 || ms < bms) {
                        bms = ms;
                        bc = cand;
                    }
                }
                memo.push_back({key, bc});
                it = memo.end() - 1;
            }
            wx[i] = it->second.first;
            rows[i] = it->second.second;
        }
        for (int order = 0; order < 3; ++order) {
            b->wx = wx;
            b->rows = rows;
            b->waves = waves;
            b->order = order;
            int rc = build_tables<M>(b);
            if (rc) return rc;
            const float ms = time_batch<M>(b, trials);
            if (ms < 0) return bfail(b, LBCM_EHIP, "timing the batched launch failed");
            if (best_ms < 0 || ms < best_ms) {
                best_ms = ms;
                best_wx = wx;
                best_rows = rows;
                best_waves = waves;
                best_order = order;
            }
        }
    }
    b->wx = best_wx;
    b->rows = best_rows;
    b->waves = best_waves;
    b->order = best_order;
    // the looped single-box launches: the same per-box tiles where the single-lattice kernel is
    // the batched one's (one row per wave); where it has two-row waves (large 16-bit boxes) the
    // fastest tile of that kernel, timed per box size over every split
    std::vector<std::pair<std::pair<int, int>, std::pair<int, int>>> single;  // (nx, ny) -> (wx, rows)
    for (int i = 0; i < b->n; ++i) {
        lbcm_handle *h = b->box[i];
        std::pair<int, int> bc{b->wx[i], b->rows[i]};
        const int rpw = rows_per_wave(h->p);
        if (rpw != 1) {
            auto key = std::make_pair(h->p.nx, h->p.ny);
            auto it = std::find_if(single.begin(), single.end(), [&](auto &m) { return m.first == key; });
            if (it == single.end()) {
                float bms = -1;
                for (auto cand : tile_candidates(h->p, 0)) {
                    const float ms = time_tiles<M>(h, cand.first, cand.second, rpw, trials);
                    if (ms < 0) return bfail(b, LBCM_EHIP, "timing a tile shape failed");
                    if (bms < 0 || ms < bms) {
                        bms = ms;
                        bc = cand;
                    }
                }
                single.push_back({key, bc});
            } else {
                bc = it->second;
            }
        }
        h->p.tile_wx = bc.first;
        h->p.tile_rows = bc.second;
    }
    return build_tables<M>(b);
}

template <class Fn> int bdispatch(lbcm_batch *b, Fn &&fn)
{
    switch (b->precision) {
    case LBCM_FP64: return fn(ModeF64{});
    case LBCM_FP32: return fn(ModeF32{});
    case LBCM_FP16_SHIFTED: return fn(ModeF16{});
    case LBCM_BF16_SHIFTED: return fn(ModeB16{});
    default: return bfail(b, LBCM_EINVAL, "unsupported precision");
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
    set_sizes(p, h->fset, h->gset);
    h->fset_al = align_up(h->fset);
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
    return dispatch(h, [&](auto mode) { return do_init<decltype(mode)>(h, phi0, rho0, ux0, uy0); });
}

int lbcm_init(lbcm_handle *h, const double *phi0, const double *rho0, const double *ux0, const double *uy0)
{
    if (!h) return LBCM_EINVAL;
    if (!phi0) return fail(h, LBCM_EINVAL, "phi0 is NULL");
    // stage the host planes in pair 0 (>= 36 bytes per node in every mode; overwritten only by
    // the final un-stream of the initialisation)
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
    return dispatch(h, [&](auto mode) { return launch_steps<decltype(mode)>(h, nsteps); });
}

int lbcm_fields_device(lbcm_handle *h, double *phi, double *rho, double *ux, double *uy, double *p0)
{
    if (!h) return LBCM_EINVAL;
    if (!h->ready) return fail(h, LBCM_ESTATE, "lbcm_fields before lbcm_init");
    return do_fields(h, phi, rho, ux, uy, p0);
}

int lbcm_fields(lbcm_handle *h, double *phi, double *rho, double *ux, double *uy, double *p0)
{
    if (!h) return LBCM_EINVAL;
    if (!h->ready) return fail(h, LBCM_ESTATE, "lbcm_fields before lbcm_init");
    // one plane at a time through the spare pair (>= 8 bytes per node in every mode)
    const size_t N = (size_t)h->p.nx * h->p.ny;
    double *stage = (double *)(h->ws + (size_t)(1 - h->cur) * h->pair_bytes);
    h->prev_ok = false;  // staged through the spare pair
    double *dst[5] = {phi, rho, ux, uy, p0};
    for (int k = 0; k < 5; ++k) {
        if (!dst[k]) continue;
        double *d[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
        d[k] = stage;
        int rc = do_fields(h, d[0], d[1], d[2], d[3], d[4]);
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
    h->prev_ok = false;  // staged through the spare pair
    for (int k = 0; k < 18; ++k) {
        double *dst = k < 9 ? f : g;
        if (!dst) continue;
        int rc = do_population(h, k, stage);
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
    int rc = do_diag(h);
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
    out->max_du = h->prev_ok ? v[7] : std::nan("");
    return LBCM_OK;
}

size_t lbcm_state_size(const lbcm_handle *h)
{
    return h ? h->fset + h->gset : 0;
}

int lbcm_get_state(lbcm_handle *h, void *host, size_t bytes)
{
    if (!h || !host) return fail(h, LBCM_EINVAL, "NULL argument");
    if (!h->ready) return fail(h, LBCM_ESTATE, "lbcm_get_state before lbcm_init");
    if (bytes != lbcm_state_size(h)) return fail(h, LBCM_EINVAL, "wrong state size");
    HIP_TRY(h, hipMemcpyAsync(host, set_base(h, h->cur, 0), h->fset, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync((char *)host + h->fset, set_base(h, h->cur, 1), h->gset, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return LBCM_OK;
}

int lbcm_set_state(lbcm_handle *h, const void *host, size_t bytes, int64_t step)
{
    if (!h || !host) return fail(h, LBCM_EINVAL, "NULL argument");
    if (bytes != lbcm_state_size(h)) return fail(h, LBCM_EINVAL, "wrong state size");
    if (step < 0) return fail(h, LBCM_EINVAL, "step must be >= 0");
    HIP_TRY(h, hipMemcpyAsync(set_base(h, h->cur, 0), host, h->fset, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(set_base(h, h->cur, 1), (const char *)host + h->fset, h->gset, hipMemcpyHostToDevice,
                              h->stream));
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(1), 0, h->stream, h->flag);
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->ready = true;
    h->prev_ok = false;
    h->step = step;
    return LBCM_OK;
}

int lbcm_copy_state(lbcm_handle *dst, const lbcm_handle *src, int64_t step)
{
    if (!dst || !src) return fail(dst, LBCM_EINVAL, "NULL argument");
    if (!src->ready) return fail(dst, LBCM_ESTATE, "lbcm_copy_state from a lattice before lbcm_init");
    if (step < 0) return fail(dst, LBCM_EINVAL, "step must be >= 0");
    if (dst->p.nx != src->p.nx || dst->p.ny != src->p.ny || dst->p.precision != src->p.precision ||
        dst->fset != src->fset || dst->gset != src->gset)
        return fail(dst, LBCM_EINVAL, "lattices differ in size or precision");
    if (dst->stream != src->stream) HIP_TRY(dst, hipStreamSynchronize(src->stream));
    HIP_TRY(dst, hipMemcpyAsync(set_base(dst, dst->cur, 0), set_base(const_cast<lbcm_handle *>(src), src->cur, 0), dst->fset,
                                hipMemcpyDeviceToDevice, dst->stream));
    HIP_TRY(dst, hipMemcpyAsync(set_base(dst, dst->cur, 1), set_base(const_cast<lbcm_handle *>(src), src->cur, 1), dst->gset,
                                hipMemcpyDeviceToDevice, dst->stream));
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(1), 0, dst->stream, dst->flag);
    HIP_TRY(dst, hipGetLastError());
    dst->ready = true;
    dst->prev_ok = false;
    dst->step = step;
    return LBCM_OK;
}

int64_t lbcm_step_count(const lbcm_handle *h) { return h ? h->step : -1; }

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

int lbcm_stream_probe(const float *src, float *dst, size_t n, int32_t planes, int32_t reps, void *stream, float *ms)
{
    auto err = [](int code, const std::string &m) {
        g_create_error = "lbcm_stream_probe: " + m;
        return code;
    };
    if (!src || !dst || !ms || n < 1 || n > 0xffffffffull || reps < 1 || (planes != 9 && planes != 18))
        return err(LBCM_EINVAL, "need src, dst, ms, 1 <= n < 2^32, reps >= 1 and planes 9 or 18");
    const hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)((n + 511) / 512)), block(512);
    auto launch = [&] {
        if (planes == 18) hipLaunchKernelGGL((k_stream<18>), grid, block, 0, st, src, dst, (uint32_t)n);
        else hipLaunchKernelGGL((k_stream<9>), grid, block, 0, st, src, dst, (uint32_t)n);
    };
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return err(LBCM_EHIP, hipGetErrorString(e));
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return err(LBCM_EHIP, hipGetErrorString(e));
    }
    launch();
    e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return err(LBCM_EHIP, hipGetErrorString(e));
    *ms /= (float)reps;
    return LBCM_OK;
}

int lbcm_diag_state(const lbcm_params *p, const void *f, const void *g, const void *f_prev, int64_t step,
                    lbcm_diagnostics *out)
{
    auto err = [](int code, const std::string &m) {
        g_create_error = "lbcm_diag_state: " + m;
        return code;
    };
    if (const char *m = check_params(p)) return err(LBCM_EINVAL, m);
    if (!f || !g || !out) return err(LBCM_EINVAL, "f, g and out must not be NULL");
    Kinds k;
    kinds_of(p->precision, k);
    const uintptr_t al = kind_bytes(k.f) > kind_bytes(k.g0) ? kind_bytes(k.f) : kind_bytes(k.g0);
    if ((uintptr_t)f % al || (uintptr_t)g % al || (uintptr_t)f_prev % al)
        return err(LBCM_EINVAL, "population sets must be aligned to " + std::to_string(al) + " bytes");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return err(LBCM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return err(LBCM_EINVAL, "device index beyond the scratch table");
    double *ptr = nullptr;
    e = scratch_address(dev, &ptr);
    if (e != hipSuccess) return err(LBCM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    const size_t N = (size_t)p->nx * p->ny;
    auto view = [&](const void *base, bool is_g) {
        SetView v;
        v.base = (unsigned char *)const_cast<void *>(base);
        const int k0 = is_g ? k.g0 : k.f, k1 = is_g ? k.g : k.f;
        for (int i = 0; i < 9; ++i) {
            v.kind[i] = i == 0 ? k0 : k1;
            v.off[i] = (uint32_t)(i == 0 ? 0 : N * kind_bytes(k0) + (size_t)(i - 1) * N * kind_bytes(k1));
        }
        return v;
    };
    const Geo geo = make_geo(*p);
    const hipStream_t st = (hipStream_t)p->stream;
    double *partial = ptr, *res = ptr + (size_t)kReduceBlocks * kDiagFields;
    hipLaunchKernelGGL(k_diag, dim3(kReduceBlocks), dim3(kReduceThreads), 0, st, view(f, false), view(g, true),
                       view(f_prev ? f_prev : f, false), (int)(f_prev != nullptr), geo, 0.5 * p->force_x,
                       0.5 * p->force_y, partial);
    if ((e = hipGetLastError()) != hipSuccess) return err(LBCM_EHIP, std::string("k_diag: ") + hipGetErrorString(e));
    hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(kReduceThreads), 0, st, partial, kReduceBlocks, res);
    if ((e = hipGetLastError()) != hipSuccess)
        return err(LBCM_EHIP, std::string("k_diag_finish: ") + hipGetErrorString(e));
    double v[kDiagFields];
    if ((e = hipMemcpyAsync(v, res, sizeof v, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return err(LBCM_EHIP, std::string("reading the results: ") + hipGetErrorString(e));
    out->sum_phi = v[0];
    out->sum_abs_phi = v[1];
    out->sum_rho = v[2];
    out->sum_jx = v[3];
    out->sum_jy = v[4];
    out->max_u = v[5];
    out->nonfinite = (int64_t)v[6];
    out->step = step;
    out->max_du = f_prev ? v[7] : std::nan("");
    return LBCM_OK;
}

int lbcm_autotune(lbcm_handle *h, int trials)
{
    if (!h) return LBCM_EINVAL;
    if (!h->ready) return fail(h, LBCM_ESTATE, "lbcm_autotune before lbcm_init");
    if (trials < 1) return fail(h, LBCM_EINVAL, "trials must be >= 1");
    return dispatch(h, [&](auto mode) -> int {
        using M = decltype(mode);
        float best = -1;
        std::pair<int, int> bc{h->p.tile_wx, h->p.tile_rows};
        for (auto cand : tile_candidates(h->p, 0)) {
            const float ms = time_tiles<M>(h, cand.first, cand.second, rows_per_wave(h->p), trials);
            if (ms < 0) return fail(h, LBCM_EHIP, "timing a tile shape failed");
            if (best < 0 || ms < best) {
                best = ms;
                bc = cand;
            }
        }
        h->p.tile_wx = bc.first;
        h->p.tile_rows = bc.second;
        return LBCM_OK;
    });
}

int lbcm_info(const lbcm_handle *h, lbcm_params *out)
{
    if (!h || !out) return LBCM_EINVAL;
    *out = h->p;
    out->stream = h->stream;
    return LBCM_OK;
}

int lbcm_tile_rows_per_wave(const lbcm_handle *h, int32_t *rpw)
{
    if (!h || !rpw) return LBCM_EINVAL;
    *rpw = make_geo(h->p).rpw;
    return LBCM_OK;
}

int lbcm_tile_shape(const lbcm_handle *h, int32_t *wx, int32_t *rows)
{
    if (!h || !wx || !rows) return LBCM_EINVAL;
    const Geo g = make_geo(h->p);
    *wx = g.wx;
    *rows = g.rows;
    return LBCM_OK;
}

int lbcm_batch_create(const lbcm_params *boxes, int32_t nboxes, lbcm_batch **out)
{
    if (!out) return LBCM_EINVAL;
    *out = nullptr;
    if (!boxes || nboxes < 1) {
        g_create_error = "need at least one box";
        return LBCM_EINVAL;
    }
    for (int i = 0; i < nboxes; ++i) {
        if (const char *m = check_params(&boxes[i])) {
            g_create_error = "box " + std::to_string(i) + ": " + m;
            return LBCM_EINVAL;
        }
        if (boxes[i].precision != boxes[0].precision || boxes[i].stream != boxes[0].stream) {
            g_create_error = "every box of a batch must have the same precision and stream";
            return LBCM_EINVAL;
        }
    }
    lbcm_batch *b = new (std::nothrow) lbcm_batch();
    if (!b) {
        g_create_error = "out of host memory";
        return LBCM_ENOMEM;
    }
    b->n = nboxes;
    b->precision = boxes[0].precision;
    b->waves = max_waves_of(b->precision);
    b->stream = (hipStream_t)boxes[0].stream;
    auto bail = [&](int code, const std::string &m) {
        g_create_error = m;
        lbcm_batch_destroy(b);
        return code;
    };
    if (!b->stream) {  // graph capture needs a stream of its own
        hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(LBCM_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        b->owns_stream = true;
    }
    std::vector<size_t> off(nboxes);
    size_t total = 0;
    for (int i = 0; i < nboxes; ++i) {
        off[i] = total;
        total += align_up(lbcm_workspace_size(&boxes[i]));
    }
    const size_t flag_off = total;
    total += kAlign;
    hipError_t e = hipMalloc((void **)&b->arena, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return bail(e == hipErrorOutOfMemory ? LBCM_ENOMEM : LBCM_EHIP, std::string("hipMalloc(") + std::to_string(total) + "): " + hipGetErrorString(e));
    }
    b->flag = (int *)(b->arena + flag_off);
    e = hipMemsetAsync(b->flag, 0, sizeof(int), b->stream);
    if (e != hipSuccess) return bail(LBCM_EHIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
    b->box.resize(nboxes, nullptr);
    b->wx.resize(nboxes);
    b->rows.resize(nboxes);
    for (int i = 0; i < nboxes; ++i) {
        lbcm_params q = boxes[i];
        q.stream = b->stream;
        q.workspace = b->arena + off[i];
        q.workspace_bytes = align_up(lbcm_workspace_size(&boxes[i]));
        int rc = lbcm_create(&q, &b->box[i]);
        if (rc) return bail(rc, "box " + std::to_string(i) + ": " + g_create_error);
        // default tile: as wide as the box allows, the rest of the workgroup in rows
        const Geo g = make_geo(q, 1);
        b->wx[i] = g.wx;
        b->rows[i] = std::max(1, b->waves / g.wx);
    }
    *out = b;
    return LBCM_OK;
}

lbcm_handle *lbcm_batch_box(lbcm_batch *b, int32_t i)
{
    return (b && i >= 0 && i < b->n) ? b->box[i] : nullptr;
}

int lbcm_batch_set_graph(lbcm_batch *b, int32_t enable)
{
    if (!b) return LBCM_EINVAL;
    b->use_graph = enable != 0;
    if (!b->use_graph) drop_graph(b);
    return LBCM_OK;
}

int lbcm_batch_set_persistent(lbcm_batch *b, int32_t mode)
{
    if (!b) return LBCM_EINVAL;
    if (mode != 0 && mode != kPersistBarrier && mode != kPersistDataflow)
        return bfail(b, LBCM_EINVAL, "persistent mode must be 0, 1 or 2");
    b->persist = mode;
    b->persist_grid = 0;
    return LBCM_OK;
}

int lbcm_batch_set_order(lbcm_batch *b, int32_t order)
{
    if (!b) return LBCM_EINVAL;
    if (order < 0 || order > 2) return bfail(b, LBCM_EINVAL, "order must be 0, 1 or 2");
    if (order != b->order) {
        b->order = order;
        drop_graph(b);
        if (b->d_desc) (void)hipFree(b->d_desc);  // rebuilt by the next step
        b->d_desc = nullptr;
    }
    return LBCM_OK;
}

int lbcm_batch_autotune(lbcm_batch *b, int32_t trials)
{
    if (!b) return LBCM_EINVAL;
    if (trials < 1) return bfail(b, LBCM_EINVAL, "trials must be >= 1");
    for (int i = 0; i < b->n; ++i)
        if (!b->box[i]->ready) return bfail(b, LBCM_ESTATE, "box " + std::to_string(i) + " is not initialised");
    return bdispatch(b, [&](auto mode) { return batch_autotune<decltype(mode)>(b, trials); });
}

int lbcm_batch_step(lbcm_batch *b, int64_t nsteps)
{
    if (!b) return LBCM_EINVAL;
    if (nsteps < 0) return bfail(b, LBCM_EINVAL, "nsteps must be >= 0");
    return bdispatch(b, [&](auto mode) { return batch_steps<decltype(mode)>(b, nsteps); });
}

int lbcm_batch_step_looped(lbcm_batch *b, int64_t nsteps)
{
    if (!b) return LBCM_EINVAL;
    if (nsteps < 0) return bfail(b, LBCM_EINVAL, "nsteps must be >= 0");
    for (int64_t s = 0; s < nsteps; ++s)
        for (int i = 0; i < b->n; ++i) {
            int rc = lbcm_step(b->box[i], 1);
            if (rc) return bfail(b, rc, "box " + std::to_string(i) + ": " + b->box[i]->err);
        }
    return LBCM_OK;
}

int lbcm_batch_step_looped_streams(lbcm_batch *b, int64_t nsteps, int32_t nstreams)
{
    if (!b) return LBCM_EINVAL;
    if (nsteps < 0) return bfail(b, LBCM_EINVAL, "nsteps must be >= 0");
    if (nstreams < 1 || nstreams > 64) return bfail(b, LBCM_EINVAL, "nstreams must be in [1, 64]");
    if (nstreams == 1) return lbcm_batch_step_looped(b, nsteps);
    std::vector<hipStream_t> side(nstreams, nullptr);
    std::vector<hipEvent_t> done(nstreams, nullptr);
    hipEvent_t fork = nullptr;
    int rc = LBCM_OK;
    auto cleanup = [&]() {
        // the batch's stream has waited for every side stream already; destroying them is safe
        for (auto &e : done)
            if (e) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        for (auto &st : side)
            if (st) (void)hipStreamDestroy(st);
    };
    auto hip_ok = [&](hipError_t e, const char *what) {
        if (e == hipSuccess) return true;
        rc = bfail(b, LBCM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
        return false;
    };
    // streams of default priority (different priorities have hung on these parts)
    bool ok = hip_ok(hipEventCreateWithFlags(&fork, hipEventDisableTiming), "hipEventCreateWithFlags");
    for (int k = 0; ok && k < nstreams; ++k)
        ok = hip_ok(hipStreamCreateWithFlags(&side[k], hipStreamNonBlocking), "hipStreamCreateWithFlags") &&
             hip_ok(hipEventCreateWithFlags(&done[k], hipEventDisableTiming), "hipEventCreateWithFlags");
    for (int64_t s = 0; ok && s < nsteps; ++s) {
        // fork from the batch's stream, box i on side stream i mod nstreams, join back
        ok = hip_ok(hipEventRecord(fork, b->stream), "hipEventRecord");
        for (int k = 0; ok && k < nstreams; ++k) ok = hip_ok(hipStreamWaitEvent(side[k], fork, 0), "hipStreamWaitEvent");
        for (int i = 0; ok && i < b->n; ++i) {
            lbcm_handle *h = b->box[i];
            const hipStream_t own = h->stream;
            h->stream = side[i % nstreams];
            const int r = lbcm_step(h, 1);
            h->stream = own;
            if (r) {
                rc = bfail(b, r, "box " + std::to_string(i) + ": " + h->err);
                ok = false;
            }
        }
        for (int k = 0; k < nstreams && side[k]; ++k) {
            // joined even after an error, so that the batch's stream orders everything queued
            if (!hip_ok(hipEventRecord(done[k], side[k]), "hipEventRecord") ||
                !hip_ok(hipStreamWaitEvent(b->stream, done[k], 0), "hipStreamWaitEvent"))
                ok = false;
        }
    }
    if (!ok && rc == LBCM_OK) rc = LBCM_EHIP;
    if (hipStreamSynchronize(b->stream) != hipSuccess && rc == LBCM_OK) rc = bfail(b, LBCM_EHIP, "hipStreamSynchronize failed");
    cleanup();
    return rc;
}

int lbcm_batch_info(const lbcm_batch *b, int32_t *waves, int32_t *order, int32_t *ntiles, int32_t *wx, int32_t *rows)
{
    if (!b) return LBCM_EINVAL;
    if (waves) *waves = b->waves;
    if (order) *order = b->order;
    if (ntiles) *ntiles = b->ntiles;
    for (int i = 0; i < b->n; ++i) {
        if (wx) wx[i] = b->wx[i];
        if (rows) rows[i] = b->rows[i];
    }
    return LBCM_OK;
}

int lbcm_batch_destroy(lbcm_batch *b)
{
    if (!b) return LBCM_OK;
    int rc = LBCM_OK;
    if (b->stream && hipStreamSynchronize(b->stream) != hipSuccess) rc = LBCM_EHIP;
    drop_graph(b);
    for (lbcm_handle *h : b->box)
        if (h && lbcm_destroy(h) != LBCM_OK) rc = LBCM_EHIP;
    if (b->d_desc && hipFree(b->d_desc) != hipSuccess) rc = LBCM_EHIP;
    if (b->d_tiles && hipFree(b->d_tiles) != hipSuccess) rc = LBCM_EHIP;
    if (b->d_done && hipFree(b->d_done) != hipSuccess) rc = LBCM_EHIP;
    if (b->d_ctl && hipFree(b->d_ctl) != hipSuccess) rc = LBCM_EHIP;
    if (b->arena && hipFree(b->arena) != hipSuccess) rc = LBCM_EHIP;
    if (b->owns_stream && hipStreamDestroy(b->stream) != hipSuccess) rc = LBCM_EHIP;
    delete b;
    return rc;
}

const char *lbcm_batch_last_error(const lbcm_batch *b)
{
    return b ? b->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
