// Learned surrogate of the lattice Boltzmann step: a stack of 3x3 convolutions (circular
// padding, periodic boxes) that maps the macroscopic state (phi, v_x, v_y) to the state K steps
// later, trained on trajectories of the LB solver.  The state also carries the density, which
// holds the pressure field: without it the velocity K steps on is not determined by the state.
//
// Network.  z_l[p] = b_l + sum_t a_l[p + d_t] W_l[t] with tap t = 3 (dy + 1) + (dx + 1) at
// d_t = (dy, dx); a_0 = state, a_{l+1} = relu(z_l), out = state + alpha * z_{L-1} (alpha: a fixed
// per-channel output scale).  Loss: mean over pixels and channels of ((out - target) / alpha)^2.
//
// Precision and units.  Layer 0 (4 real input channels, 36 products per output) runs on the
// matrix cores in FP32 (v_mfma_f32_16x16x4_f32) with FP32 state and weights, so the state enters
// at full precision.  Layers 1 .. L-1 are implicit GEMMs on the MFMA units
// (v_mfma_f32_16x16x32_bf16: BF16 activations and weights, FP32 accumulation); their weights are
// packed to BF16 from the FP32 masters after every update.  Activations are NHWC BF16 [P][C]; the
// last layer's 4 outputs are padded to 32.  Inference from field planes runs the layers in fused
// pairs whose intermediate activation stays in LDS (k_first_pair, k_pair).
//
// Packs.  Wf[t][co][ci] feeds the forward pass (the MFMA A operand takes 8 consecutive K = input
// channels per lane).  Wb[t][ci][co] = W[8 - t][ci][co] feeds the input gradient: tap t of the
// mirrored pack sits at d_t = -d_{8-t}, so the forward kernel run on dZ with it gives
// dX[p] = sum_t dZ[p - d_t] W[t]^T.  The weight gradient dW[t] = sum_p X[p + d_t]^T dZ[p] is a GEMM
// whose K dimension runs over pixels.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "lbcm_net.h"

// dynamic LDS of the convolution kernels (external linkage: an array declared in the anonymous
// namespace would be a zero-sized object of this file)
extern __shared__ __align__(16) __bf16 lbcm_conv_lds[];

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned int)))) unsigned int u32x4;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(2 * sizeof(unsigned int)))) unsigned int u32x2;

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations, not for its
// global loads or stores, so loads issued before it (weights or patches prefetched into registers)
// and earlier output stores stay in flight across it.  (__syncthreads also waits for every
// outstanding global load and store.)
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// raw buffer resource over [p, p + bytes) (gfx9-family word 3); accesses past its end are dropped
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

constexpr int kStateC = 4;        // phi, v_x, v_y, rho (channel order of the state)
constexpr int kFirstRows = 9 * kStateC + 1;  // layer-0 weight rows (tap, channel) and the bias row
constexpr int kOutC = 32;         // padded output channels of the last layer (two groups: the forward's wave split)
constexpr int kThreads = 256;     // four waves
constexpr int kTileH = 8;         // conv tile: 8 rows x 32 columns of one sample
constexpr int kTileW = 32;
constexpr int kPatchH = kTileH + 2, kPatchW = kTileW + 2;
constexpr int kDwPix = 64;        // pixels staged per iteration of the weight-gradient kernel
constexpr int kDwChunk = 4096;    // pixels reduced by one weight-gradient workgroup

__device__ __forceinline__ int tap_dy(int t) { return t / 3 - 1; }
__device__ __forceinline__ int tap_dx(int t) { return t % 3 - 1; }

__device__ __forceinline__ int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// pixel index of p shifted by (dy, dx) inside its sample (circular)
__device__ __forceinline__ uint32_t shift_pix(uint32_t p, int dy, int dx, int H, int W)
{
    const uint32_t hw = (uint32_t)H * W;
    const uint32_t n = p / hw, r = p - n * hw;
    const int y = wrap((int)(r / W) + dy, H), x = wrap((int)(r % W) + dx, W);
    return n * hw + (uint32_t)y * W + (uint32_t)x;
}

__device__ __forceinline__ bf16x8 ld8(const __bf16 *p) { return __builtin_bit_cast(bf16x8, *(const u32x4 *)p); }

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4i16 lds_v4i16;

// One 16 x 32 MFMA operand (16 channels, K = 32 pixels) from a [pixel][channel] LDS block of
// pixel stride ps: lane (r, q) gets channel r of pixels 8q .. 8q + 7.  Its offset o0 is opix ps +
// the block's first channel + och (opix = 8 (lane / 16) + (lane % 16) / 4, och = 4 (lane % 4)); the
// two halves of its eight pixels are read with the transposing load at o0 and o0 + 4 ps.
__device__ __forceinline__ bf16x8 ld_tr(const __bf16 *p, int o0, int ps)
{
    const auto *base = (const __attribute__((address_space(3))) char *)(p);
    const v4i16 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4i16 *)(base + 2 * o0));
    const v4i16 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4i16 *)(base + 2 * (o0 + 4 * ps)));
    typedef short v8i16 __attribute__((ext_vector_type(8)));
    const v8i16 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_bit_cast(bf16x8, v);
}

// wrap v into [0, n) for v in [-1, n + 40] (the rows and columns a tile and its halo touch)
__device__ __forceinline__ int wrap_near(int v, int n)
{
    if (v < 0) v += n;
    if (v >= n) {
        v -= n;
        if (v >= n) v %= n;
    }
    return v;
}

// tile index -> (sample, first row, first column) of an 8 x 32 tile
struct TileCoord {
    int n, y0, x0;
};
__device__ __forceinline__ TileCoord tile_coord(int tile, int H, int W)
{
    const int tx = (W + kTileW - 1) / kTileW, ty = (H + kTileH - 1) / kTileH;
    const int n = tile / (tx * ty), rem = tile % (tx * ty);
    return {n, (rem / tx) * kTileH, (rem % tx) * kTileW};
}

// ------------------------------------------------------------------------------------------
// layer 0 on the matrix cores in FP32 over 8 x 32 tiles: Y[p][co] = bf16(relu(b[co] + sum_{t, ci}
// s[p + d_t][ci] W0[t][ci][co])), a workgroup taking the tiles b, b + G, ... (G the grid) with the
// next tile's patch in flight during the current one.  v_mfma_f32_16x16x4_f32 takes K = 4,
// exactly the state channels of one tap, so each tap is one MFMA per 16-channel x 16-pixel block
// with FP32 products and sums.  Wave w computes tile row w (two 16-pixel blocks) for all C / 16
// channel blocks; its A operands (W0 of 9 taps x C / 16 blocks, one value per lane) stay in
// registers for all tiles.  The state patch (tile plus circular halo) is staged in LDS.  With PLANES the
// patch is read from the four FP64 field planes and converted to the state (phi, v / u_scale,
// (rho - 1) / rho_scale) as k_from_planes does, and the tile's own state goes to s_out (the
// residual of the last layer).

constexpr int kFirstThreads = 64 * kTileH;  // one wave per tile row

struct PlaneIn {
    const double *phi, *ux, *uy, *rho;
    float inv_u, inv_r;
};

template <int C, bool PLANES, bool WIDE>
__global__ __launch_bounds__(kFirstThreads) void k_first(const float *__restrict__ s, PlaneIn pin, float *__restrict__ s_out,
                                                         const float *__restrict__ W0, const float *__restrict__ b0, int ntiles,
                                                         int H, int W, __bf16 *__restrict__ Y, uint8_t *__restrict__ mask_out)
{
    constexpr int NB = C / 16;  // channel blocks
    constexpr int NP = kPatchH * kPatchW;
    static_assert(NP <= kFirstThreads, "one patch pixel per thread");
    __shared__ __align__(16) float sp[NP * kStateC];
    __shared__ __align__(16) uint8_t mstage[kTileH * kTileW * (C / 4)];  // ReLU mask bytes of a tile
    const int lane = threadIdx.x & 63;
    const int row = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, q = lane >> 4;
    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    // A operand of block cb at tap t: lane (r, q) holds W0[t][ci = q][co = 16 cb + r]
    float wa[9][NB];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) wa[t][cb] = W0[(kStateC * t + q) * C + 16 * cb + r];
    // D of a block: lane (r, q) holds channels 16 cb + 4 q + e of pixel r; the sums start at the bias
    float bias[NB][4];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[cb][e] = b0[16 * cb + 4 * q + e];
    // this thread's patch pixel (threads past the patch repeat its last pixel: no branch around
    // the loads, so that their wait counts exactly); with WIDE (box of at least 8 rows and 32
    // columns) the circular halo indices wrap with selects
    const int k = min((int)threadIdx.x, NP - 1), py = k / kPatchW, px = k % kPatchW;
    auto wrap1 = [](int v, int n) {
        if (!WIDE) return wrap_near(v, n);
        const int a = v < 0 ? v + n : v;
        return a >= n ? a - n : a;
    };
    auto load = [&](int t) {
        const TileCoord tc = tile_coord(t, H, W);
        const int gy = wrap1(tc.y0 - 1 + py, H), gx = wrap1(tc.x0 - 1 + px, W);
        const size_t p = ((size_t)tc.n * H + gy) * W + gx;
        f32x4 v;
        if constexpr (PLANES) {
            v[0] = (float)pin.phi[p];
            v[1] = (float)pin.ux[p] * pin.inv_u;
            v[2] = (float)pin.uy[p] * pin.inv_u;
            v[3] = (float)(pin.rho[p] - 1.0) * pin.inv_r;
            // the tile's own pixels (each belongs to exactly one tile)
            if (py >= 1 && py <= kTileH && px >= 1 && px <= kTileW && tc.y0 + py - 1 < H && tc.x0 + px - 1 < W)
                *(f32x4 *)(s_out + p * kStateC) = v;
        } else {
            v = *(const f32x4 *)(s + p * kStateC);
        }
        return v;
    };
    f32x4 pv = load(tile);
    __syncthreads();  // also waits for the weight and bias loads, so that no wait in the loop is for them
    *(f32x4 *)(sp + k * kStateC) = pv;
    lds_barrier();
    // Per tile: the next tile's patch pixel (the last iteration repeats the last tile's), the
    // MFMAs and the output stores, then the patch exchange; LDS-only barriers, so that the output
    // stores stay in flight into the next tile.
    for (; tile < ntiles; tile += gridDim.x) {
        const TileCoord tc = tile_coord(tile, H, W);
        pv = load(min(tile + (int)gridDim.x, ntiles - 1));
        f32x4 acc[2][NB];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int cb = 0; cb < NB; ++cb)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[h][cb][e] = bias[cb][e];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            float x[2];  // B operand: lane (r, q) holds channel q of pixel r of the block
#pragma unroll
            for (int h = 0; h < 2; ++h) x[h] = sp[((row + 1 + tap_dy(t)) * kPatchW + 16 * h + r + 1 + tap_dx(t)) * kStateC + q];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int cb = 0; cb < NB; ++cb) acc[h][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[t][cb], x[h], acc[h][cb], 0, 0, 0);
        }
        // bf16(relu) through a buffer resource over the tile's rows inside the box: a pixel past
        // the right edge gets an offset past it (dropped), rows past the bottom lie past it
        const int rows = min(kTileH, H - tc.y0);
        const size_t tile_px = ((size_t)tc.n * H + tc.y0) * W;
        const rsrc_t ry = make_rsrc(Y + tile_px * C, (uint32_t)rows * W * C * sizeof(__bf16));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int xg = tc.x0 + 16 * h + r;
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                bf16x4 v;
                uint32_t bits = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = (__bf16)fmaxf(acc[h][cb][e], 0.f);
                    bits |= ((float)v[e] > 0.f ? 1u : 0u) << e;
                }
                const int off = xg < W ? ((row * W + xg) * C + 16 * cb + 4 * q) * (int)sizeof(__bf16) : 0x7fffffff;
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), ry, off, 0, 0);
                mstage[(row * kTileW + 16 * h + r) * (C / 4) + 4 * cb + q] = (uint8_t)bits;
            }
        }
        lds_barrier();  // every wave is done with this tile's patch, the mask bytes are in LDS
        {
            // ReLU mask bytes of the training forward (bit e of byte [p][c / 4]): C / 4 bytes per
            // tile pixel (thread t: pixel t), dropped past the box, and all of them without masks
            // (a resource of size 0)
            const rsrc_t rm = make_rsrc(mask_out ? mask_out + tile_px * (C / 4) : nullptr, mask_out ? (uint32_t)rows * W * (C / 4) : 0u);
            const int t = min((int)threadIdx.x, kTileH * kTileW - 1), ty = t / kTileW, tx = t % kTileW;
            const bool ok = (int)threadIdx.x < kTileH * kTileW && tc.x0 + tx < W;
            const int off = ok ? (ty * W + tc.x0 + tx) * (C / 4) : 0x7fffffff;
            if constexpr (C == 64)
                __builtin_amdgcn_raw_buffer_store_b128(*(const u32x4 *)(mstage + t * 16), rm, off, 0, 0);
            else
                __builtin_amdgcn_raw_buffer_store_b64(*(const u32x2 *)(mstage + t * 8), rm, off, 0, 0);
        }
        *(f32x4 *)(sp + k * kStateC) = pv;
        lds_barrier();
    }
}

// layer 0 gradients on the BF16 matrix cores: D[co][col] = sum_p dZ[p][co] B[p][col] with col =
// kStateC t + ci < 36 (B = s[p + d_t][ci], the weight gradient), col 36 (B = 1, the bias gradient)
// and cols 37 .. 47 (B = 0, padding to three 16-column blocks).  Each FP32 state value splits
// exactly into three BF16 parts (hi = bf16(x), mid = bf16(x - hi), lo = x - hi - mid: three 8-bit
// significands hold FP32's 24), so every product with the BF16 dZ is exact and the sums are FP32,
// as with FP32 operands, at three BF16 MFMAs per 32 pixels where the FP32 MFMA took eight.
// v_mfma_f32_16x16x32_bf16 takes one tile row (32 pixels) as its K: lane (r, q) holds A =
// dZ[pixels 8q .. 8q + 7][co0 + r] (transposing LDS reads) and B = one part of B[the same
// pixels][col0 + r].  Workgroup b takes the tiles b, b + G, ... (G = the grid), staging each
// tile's FP32 state patch and dZ in LDS with the next tile's global loads in flight; wave w takes
// tile rows w and w + 4 and keeps all C / 16 x 3 output blocks in registers.  The workgroup's
// sums go to partial row b ([row][col][co], cols < kFirstRows), added in a fixed order by
// k_grad_reduce.  Two workgroups per CU keep twice the tile loads in flight (the loads of the
// next tile are all that overlaps a tile's short MFMA work).
constexpr int kFirstDwBlocks = 512;  // workgroups of k_first_dw at most
constexpr int kFirstCols = 48;       // kFirstRows columns padded to three 16-column blocks

template <int C>
__global__ __launch_bounds__(kThreads) void k_first_dw(const float *__restrict__ s, const __bf16 *__restrict__ dz, int H,
                                                       int W, int ntiles, float *__restrict__ partial)
{
    constexpr int NCB = C / 16, NJ = kFirstCols / 16, PSD = C + 8;  // PSD: LDS pixel stride of dZ
    constexpr int NS = kPatchH * kPatchW * kStateC, NIS = (NS + kThreads - 1) / kThreads;
    constexpr int NZ = kTileH * kTileW * C / 8, NIZ = NZ / kThreads;
    static_assert(NZ % kThreads == 0, "whole dZ chunks per thread");
    static_assert(kTileW == 32 && kTileH == 2 * (kThreads / 64), "a K step is one tile row; each wave takes two");
    __shared__ float sp[NS];
    __shared__ __align__(16) __bf16 sd[kTileH * kTileW * PSD];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, q = lane >> 4;
    // this lane's three B columns: patch offset from the pixel's position, and x m + a = B
    // (m = 1, a = 0: the state value; m = 0: a, 1 for the bias column and 0 for padding)
    int boff[NJ];
    float bm[NJ], ba[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int col = 16 * j + r, t = col / kStateC;
        const bool prod = col < kFirstRows - 1;
        boff[j] = prod ? ((1 + tap_dy(t)) * kPatchW + 1 + tap_dx(t)) * kStateC + col % kStateC : 0;
        bm[j] = prod ? 1.f : 0.f;
        ba[j] = col == kFirstRows - 1 ? 1.f : 0.f;
    }
    // the transposing reads' offsets of this lane (pixel of the first half, times the stride, and channel)
    const int opix = 8 * (lane >> 4) + ((lane & 15) >> 2), och = 4 * (lane & 3);
    f32x4 acc[NCB][NJ];
#pragma unroll
    for (int i = 0; i < NCB; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    float vs[NIS];
    u32x4 vz[NIZ];
    // global loads of one tile (state patch with circular halo; dZ, zero past the box edge)
    auto load = [&](int tile) {
        const TileCoord tc = tile_coord(tile, H, W);
#pragma unroll
        for (int i = 0; i < NIS; ++i) {
            const int k = threadIdx.x + i * kThreads;
            if (k < NS) {
                const int px = k / kStateC, c = k % kStateC;
                const int gy = wrap_near(tc.y0 - 1 + px / kPatchW, H), gx = wrap_near(tc.x0 - 1 + px % kPatchW, W);
                vs[i] = s[(((size_t)tc.n * H + gy) * W + gx) * kStateC + c];
            }
        }
#pragma unroll
        for (int i = 0; i < NIZ; ++i) {
            const int k = threadIdx.x + i * kThreads;
            const int px = k / (C / 8), ch = (k % (C / 8)) * 8;
            const int y = tc.y0 + px / kTileW, xg = tc.x0 + px % kTileW;
            vz[i] = u32x4{0, 0, 0, 0};
            if (y < H && xg < W) vz[i] = *(const u32x4 *)(dz + (((size_t)tc.n * H + y) * W + xg) * C + ch);
        }
    };
    int tile = blockIdx.x;
    if (tile < ntiles) load(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        __syncthreads();  // every wave is done with the previous tile's LDS
#pragma unroll
        for (int i = 0; i < NIS; ++i) {
            const int k = threadIdx.x + i * kThreads;
            if (k < NS) sp[k] = vs[i];
        }
#pragma unroll
        for (int i = 0; i < NIZ; ++i) {
            const int k = threadIdx.x + i * kThreads;
            *(u32x4 *)(sd + (k / (C / 8)) * PSD + (k % (C / 8)) * 8) = vz[i];
        }
        __syncthreads();
        if (tile + (int)gridDim.x < ntiles) load(tile + gridDim.x);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int y = w + (kThreads / 64) * h;  // tile row
            bf16x8 a[NCB], b[3][NJ];
#pragma unroll
            for (int i = 0; i < NCB; ++i) a[i] = ld_tr(sd + y * kTileW * PSD, opix * PSD + 16 * i + och, PSD);
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float v = fmaf(sp[(y * kPatchW + 8 * q + e) * kStateC + boff[j]], bm[j], ba[j]);  // exact: x, 1 or 0
                    const __bf16 hi = (__bf16)v;
                    const float r1 = v - (float)hi;
                    const __bf16 mid = (__bf16)r1;
                    b[0][j][e] = hi;
                    b[1][j][e] = mid;
                    b[2][j][e] = (__bf16)(r1 - (float)mid);
                }
#pragma unroll
            for (int part = 0; part < 3; ++part)
#pragma unroll
                for (int i = 0; i < NCB; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[part][j], acc[i][j], 0, 0, 0);
        }
    }
    // D of block (i, j): lane (r, q) holds co = 16 i + 4 q + e, col = 16 j + r.  Waves 1 .. 3 hand
    // their sums to wave 0 through LDS (over the dZ tile), which adds them in wave order and writes
    // the workgroup's partial row b.
    static_assert((kThreads / 64 - 1) * kFirstRows * C * sizeof(float) <= sizeof(sd), "three waves' sums fit the dZ tile");
    float *red = reinterpret_cast<float *>(sd);
    __syncthreads();  // every wave is done with the last tile
    if (w > 0)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int col = 16 * j + r;
            if (col < kFirstRows)
#pragma unroll
                for (int i = 0; i < NCB; ++i)
#pragma unroll
                    for (int e = 0; e < 4; ++e) red[((w - 1) * kFirstRows + col) * C + 16 * i + 4 * q + e] = acc[i][j][e];
        }
    __syncthreads();
    if (w > 0) return;
    float *out = partial + (size_t)blockIdx.x * kFirstRows * C;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int col = 16 * j + r;
        if (col < kFirstRows)
#pragma unroll
            for (int i = 0; i < NCB; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int o = col * C + 16 * i + 4 * q + e;
                    float v = acc[i][j][e];
#pragma unroll
                    for (int u = 0; u < kThreads / 64 - 1; ++u) v += red[u * kFirstRows * C + o];
                    out[o] = v;
                }
    }
}

// ------------------------------------------------------------------------------------------
// MFMA convolution over 8 x 32 pixel tiles of one sample (layers 1 .. L-1 forward, and the input
// gradient with the mirrored pack).
//
// The workgroup (8 waves) stages the layer's weights once and the 10 x 34 input patch (tile plus
// circular halo) of each tile in dynamic LDS, with pixel strides padded by 32 bytes (weight rows
// by 16) to spread the rows of a fragment over the banks; the next tile's patch is loaded during
// the current tile's MFMAs (WaveSplit below gives each wave its output channels and rows).  A wave keeps its
// weight fragments (9 taps x CIN / 32 K-steps per channel group) in registers for the whole
// launch, as the MFMA A operand, and takes 16 pixels as the B operand, so that each lane ends
// with 4 consecutive output channels of one pixel (one 8-byte store).  Tiles past the grid are
// taken in a grid-stride loop.  Dynamic LDS: ConvLds<CIN, COUT>::bytes.
//
// MODE 0: Y = bf16(relu(bias + conv)), and in the training forward the ReLU mask of Y (bit e of
// byte [p][c / 4]: Y[p][c + e] > 0);  MODE 2: Y = bf16(conv * mask) (the input gradient times the
// ReLU derivative of the layer input, from that mask);  MODE 1: Yf[p][c] = resid[p][c] + alpha_c
// (bias + conv) for c < kStateC (the last layer, FP32);  MODE 3: the same state written to the
// FP64 field planes (phi, v = u_scale v', rho = 1 + rho_scale rho').

constexpr int kConvThreads = 512;

struct OutArgs {
    const float *bias;
    const uint8_t *mask;  // MODE 2: ReLU mask of the forward activation (see mask_out)
    uint8_t *mask_out;    // MODE 0 (training forward): bit e of byte [p][c / 4] = (Y[p][c + e] > 0); null: none
    __bf16 *Y;
    const float *resid;
    float *Yf;
    float alpha0, alpha1, alpha2, alpha3;
    double *phi, *ux, *uy, *rho;  // MODE 3: FP64 field planes
    double u_scale, r_scale;
};

template <int CIN>
struct Patch {
    static constexpr int PS = CIN + 16;  // LDS pixel stride (bf16)
    static constexpr int NV = kPatchH * kPatchW * (CIN / 8), NI = (NV + kConvThreads - 1) / kConvThreads;
    u32x4 v[NI];

    // Branch-free (every thread issues NI loads, the last chunk repeated past NV), so that a wait
    // for these registers counts exactly the memory operations issued after them.  With WIDE (box
    // of at least 8 rows and 32 columns) the circular halo indices stay in [-n, 2n) and wrap with
    // selects; otherwise wrap_near.
    template <bool WIDE>
    __device__ __forceinline__ void load(const __bf16 *__restrict__ X, TileCoord tc, int H, int W)
    {
        const __bf16 *Xn = X + (size_t)tc.n * H * W * CIN;
        auto wrap1 = [](int v, int n) {
            if (!WIDE) return wrap_near(v, n);
            const int a = v < 0 ? v + n : v;
            return a >= n ? a - n : a;
        };
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int k = min((int)threadIdx.x + i * kConvThreads, NV - 1);
            const int px = k / (CIN / 8), ch = (k % (CIN / 8)) * 8;
            const int gy = wrap1(tc.y0 - 1 + px / kPatchW, H), gx = wrap1(tc.x0 - 1 + px % kPatchW, W);
            v[i] = *(const u32x4 *)(Xn + ((size_t)gy * W + gx) * CIN + ch);
        }
    }
    // also branch-free: a thread past NV stores the last chunk again (the same value to the same
    // place), so that no load is sunk into a conditional block and waited for there
    __device__ __forceinline__ void store(__bf16 *patch) const
    {
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int k = min((int)threadIdx.x + i * kConvThreads, NV - 1);
            *(u32x4 *)(patch + (k / (CIN / 8)) * PS + (k % (CIN / 8)) * 8) = v[i];
        }
    }
};

template <int CIN, int COUT>
struct ConvLds {
    static constexpr int PS = Patch<CIN>::PS;        // patch pixel stride (bf16)
    static constexpr int WS = CIN + 8;               // weight row stride (bf16)
    static constexpr int patch_elems = kPatchH * kPatchW * PS;
    static constexpr int weight_elems = 9 * COUT * WS;
    static constexpr int mask_bytes = kTileH * kTileW * (COUT / 4);  // ReLU mask bytes of a tile (training forward)
    static constexpr size_t bytes = (size_t)(patch_elems + weight_elems) * sizeof(__bf16) + mask_bytes;
};

// Work split of a conv layer over the 8 waves (the layers a of the fused pairs keep their own):
// wave w computes GPW channel groups of 16 for HPW of the tile's two 16-pixel column halves over
// RW tile rows.  With HPW = 2 (every layer of the forward pass): one group, both halves,
// row group mg = w % MG, group w / MG.  With GPW = 2, HPW = 1 (the input gradients and the last
// layer of training): half = w % 2, row group (w / 2) % MG, groups [2 pair, 2 pair + 2) for
// pair = (w / 2) / MG; every pixel fragment read from LDS then feeds twice as many MFMAs.  Which
// split each kernel takes was measured (wave_split_groups).
constexpr int wave_split_groups(int cout, int mode) { return (mode == 1 || mode == 2) && cout >= 32 ? 2 : 1; }

template <int COUT, int MODE>
struct WaveSplit {
    static constexpr int NG = COUT / 16, GPW = wave_split_groups(COUT, MODE), HPW = GPW == 2 ? 1 : 2,
                         NPAIR = NG / GPW, MG = (kConvThreads / 64) * HPW / (2 * NPAIR), RW = kTileH / MG;
    static_assert(MG * NPAIR * (2 / HPW) == kConvThreads / 64 && RW * MG == kTileH, "eight waves cover the tile");
    __device__ static int half0(int wave) { return HPW == 2 ? 0 : wave & 1; }
    __device__ static int mg(int wave) { return HPW == 2 ? wave % MG : (wave >> 1) % MG; }
    __device__ static int cbase(int wave) { return 16 * GPW * (HPW == 2 ? wave / MG : (wave >> 1) / MG); }
};

// One output tile of a conv layer from its input patch in LDS (the tile plus a one-pixel halo,
// 10 x 34 pixels, pixel stride CIN + 16), with this wave's A fragments wa[g] (W[t][co = cbase +
// 16 g + r][ci = 32 ks + 8 q .. + 8] in lane (r, q)) and the biases of its output channels.
// Input-stationary order: each pixel fragment of the wave's RW + 2 patch rows (its column half) is
// read from LDS once and applied to every output row (tap dy) and channel group that uses it.
// Stage s covers patch row s (3 horizontal taps x KS fragments); the fragments of stage s + 1 are
// read before the MFMAs of stage s, in a second register buffer.  Every output sums its taps in
// the order t = 0 .. 8 and K-steps within a tap.
// With mstage (MODE 0 of the training forward) the ReLU mask bits of the tile go to LDS,
// mstage[tile pixel][c / 4] (bit e: Y[p][c + e] > 0), for a coalesced store by the caller.
template <int CIN, int COUT, int MODE, bool MASKS = false>
__device__ __forceinline__ void conv_tile(const __bf16 *patch, const bf16x8 (&wa)[WaveSplit<COUT, MODE>::GPW][9][CIN / 32],
                                          const float (&bias)[WaveSplit<COUT, MODE>::GPW][4], TileCoord tc, const OutArgs &o,
                                          int H, int W, uint8_t *mstage = nullptr)
{
    constexpr int PS = CIN + 16, KS = CIN / 32;
    using S = WaveSplit<COUT, MODE>;
    constexpr int RW = S::RW, GPW = S::GPW, HPW = S::HPW;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int half0 = S::half0(wave), mg = S::mg(wave);
    const int cbase = S::cbase(wave);
    const int r = lane & 15, q = lane >> 4;
    f32x4 acc[GPW][RW][HPW];
#pragma unroll
    for (int g = 0; g < GPW; ++g)
#pragma unroll
        for (int rho = 0; rho < RW; ++rho)
#pragma unroll
            for (int h = 0; h < HPW; ++h) acc[g][rho][h] = f32x4{0, 0, 0, 0};
    // stage st: patch row st / HPW, column half half0 + st % HPW
    constexpr int NS = HPW * (RW + 2);
    // two fragment buffers (the next stage read during this one's MFMAs); one for the input
    // gradients, whose two channel groups per wave and mask leave no room for the second (it
    // spilled; the other wave of the SIMD covers the wait: 51.5 -> 49.3 us measured)
    constexpr int NB = MODE == 2 ? 1 : 2;
    bf16x8 fr[NB][3][KS];
    auto load_stage = [&](int st, bf16x8 (&f)[3][KS]) {
        const int py = st / HPW, half = half0 + st % HPW;
#pragma unroll
        for (int dxi = 0; dxi < 3; ++dxi)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                f[dxi][ks] = ld8(patch + ((RW * mg + py) * kPatchW + 16 * half + r + dxi) * PS + 32 * ks + 8 * q);
    };
    // global loads of the epilogue, requested before the MFMAs so that their latency hides behind
    // them (clamped pixels, every lane): MODE 2 the ReLU mask bytes of this lane's outputs, MODE 1
    // and 3 the residual state of its pixels (used by the q = 0 lanes of the first channel group)
    uint32_t mv[GPW][RW][HPW];
    f32x4 rsv[RW][HPW];
    if constexpr (MODE == 1 || MODE == 3) {
#pragma unroll
        for (int rho = 0; rho < RW; ++rho)
#pragma unroll
            for (int h = 0; h < HPW; ++h) {
                const int yy = min(tc.y0 + RW * mg + rho, H - 1), xx = min(tc.x0 + 16 * (half0 + h) + r, W - 1);
                rsv[rho][h] = *(const f32x4 *)(o.resid + (((size_t)tc.n * H + yy) * W + xx) * kStateC);
            }
    }
    if constexpr (MODE == 2) {
#pragma unroll
        for (int g = 0; g < GPW; ++g)
#pragma unroll
            for (int rho = 0; rho < RW; ++rho)
#pragma unroll
                for (int h = 0; h < HPW; ++h) {
                    const int yy = min(tc.y0 + RW * mg + rho, H - 1), xx = min(tc.x0 + 16 * (half0 + h) + r, W - 1);
                    const size_t p = ((size_t)tc.n * H + yy) * W + xx;
                    mv[g][rho][h] = o.mask[p * (COUT / 4) + (cbase + 16 * g + 4 * q) / 4];
                }
    }
    if (NB == 2) load_stage(0, fr[0]);
#pragma unroll
    for (int st = 0; st < NS; ++st) {
        if (NB == 1)
            load_stage(st, fr[0]);
        else if (st + 1 < NS)
            load_stage(st + 1, fr[(st + 1) % NB]);
        const int py = st / HPW, h = st % HPW;
#pragma unroll
        for (int dxi = 0; dxi < 3; ++dxi)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int g = 0; g < GPW; ++g)
#pragma unroll
                    for (int rho = 0; rho < RW; ++rho) {
                        const int dyi = py - rho;  // tap row index dy + 1
                        if (dyi < 0 || dyi > 2) continue;
                        acc[g][rho][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[g][3 * dyi + dxi][ks], fr[st % NB][dxi][ks],
                                                                                 acc[g][rho][h], 0, 0, 0);
                    }
        __builtin_amdgcn_sched_barrier(0);
    }
    // D[co][pixel]: lane (r, q) holds channels cbase + 16 g + 4 q .. + 3 of pixel r of each block
    if constexpr (MODE == 0 || MODE == 2) {
        // BF16 activations (MODE 0: bias + ReLU) or input gradients (MODE 2: times the ReLU mask of
        // the forward activation), stored branch-free through a buffer resource spanning the
        // tile's rows inside the box: a pixel past the right edge gets an offset past the
        // resource, which the hardware drops, and rows past the bottom edge lie past it anyway.
        // (The waits for the next tile's prefetched loads then count exactly, instead of also
        // waiting for these stores.)  The mask loads are issued together, from clamped pixels.
        const int rows = min(kTileH, H - tc.y0);
        const size_t tile_px = ((size_t)tc.n * H + tc.y0) * W;
        const rsrc_t ry = make_rsrc(o.Y + tile_px * COUT, (uint32_t)rows * W * COUT * sizeof(__bf16));
#pragma unroll
        for (int g = 0; g < GPW; ++g)
#pragma unroll
            for (int rho = 0; rho < RW; ++rho)
#pragma unroll
                for (int h = 0; h < HPW; ++h) {
                    const int c0 = cbase + 16 * g + 4 * q;
                    const int xx = tc.x0 + 16 * (half0 + h) + r;
                    const f32x4 &a = acc[g][rho][h];
                    bf16x4 v4;
                    uint32_t bits = 0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float v = a[e] + bias[g][e];
                        v4[e] = (__bf16)(MODE == 2 ? (((mv[g][rho][h] >> e) & 1u) ? v : 0.f) : fmaxf(v, 0.f));
                        bits |= ((float)v4[e] > 0.f ? 1u : 0u) << e;
                    }
                    const int pix = (RW * mg + rho) * W + xx;
                    const int off = xx < W ? (pix * COUT + c0) * (int)sizeof(__bf16) : 0x7fffffff;
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v4), ry, off, 0, 0);
                    if (MASKS) mstage[((RW * mg + rho) * kTileW + 16 * (half0 + h) + r) * (COUT / 4) + c0 / 4] = (uint8_t)bits;
                }
    } else {
        // the last layer: FP32 residual + alpha of the four state channels (MODE 1), or the same
        // written into the FP64 field planes (MODE 3)
        static_assert(MODE == 1 || MODE == 3, "output modes");
#pragma unroll
        for (int g = 0; g < GPW; ++g)
#pragma unroll
            for (int rho = 0; rho < RW; ++rho)
#pragma unroll
                for (int h = 0; h < HPW; ++h) {
                    const int c0 = cbase + 16 * g + 4 * q;
                    const int yy = tc.y0 + RW * mg + rho, xx = tc.x0 + 16 * (half0 + h) + r;
                    if (yy >= H || xx >= W) continue;
                    const size_t p = ((size_t)tc.n * H + yy) * W + xx;
                    const f32x4 &a = acc[g][rho][h];
                    if (c0 == 0) {  // the 4 state channels are those of the q = 0 lanes of the first channel group
                        static_assert(kStateC == 4, "one lane holds the four state channels of a pixel");
                        const f32x4 rs = rsv[rho][h];
                        f32x4 v;
                        v[0] = rs[0] + o.alpha0 * (a[0] + bias[g][0]);
                        v[1] = rs[1] + o.alpha1 * (a[1] + bias[g][1]);
                        v[2] = rs[2] + o.alpha2 * (a[2] + bias[g][2]);
                        v[3] = rs[3] + o.alpha3 * (a[3] + bias[g][3]);
                        if (MODE == 1) {
                            *(f32x4 *)(o.Yf + p * kStateC) = v;
                        } else {
                            o.phi[p] = v[0];
                            o.ux[p] = v[1] * o.u_scale;
                            o.uy[p] = v[2] * o.u_scale;
                            o.rho[p] = 1.0 + v[3] * o.r_scale;
                        }
                    }
                }
    }
}

// A BF16 output tile staged in LDS (pixel stride C + 8) to Y, in whole pixels: 16 bytes per
// thread, consecutive threads on consecutive bytes of a tile row, through a buffer resource
// spanning the tile's rows inside the box (pixels past the right edge get an offset past it,
// which the hardware drops).
template <int C>
__device__ __forceinline__ void stage_store(const __bf16 *ystage, __bf16 *Y, TileCoord tc, int H, int W)
{
    constexpr int NCK = kTileH * kTileW * C / 8;  // 16-byte chunks of the tile
    static_assert(NCK % kConvThreads == 0, "whole chunks per thread");
    const int rows = min(kTileH, H - tc.y0);
    const size_t tile_px = ((size_t)tc.n * H + tc.y0) * W;
    const rsrc_t ry = make_rsrc(Y + tile_px * C, (uint32_t)rows * W * C * sizeof(__bf16));
#pragma unroll
    for (int i = 0; i < NCK / kConvThreads; ++i) {
        const int k = threadIdx.x + i * kConvThreads, px = k / (C / 8), ch = (k % (C / 8)) * 8;
        const int ty = px / kTileW, x = tc.x0 + px % kTileW;
        const u32x4 v = *(const u32x4 *)(ystage + px * (C + 8) + ch);
        const int off = x < W ? ((ty * W + x) * C + ch) * (int)sizeof(__bf16) : 0x7fffffff;
        __builtin_amdgcn_raw_buffer_store_b128(v, ry, off, 0, 0);
    }
}

// WIDE: the box has at least 8 rows and 32 columns (see Patch::load).
template <int CIN, int COUT, int MODE, bool WIDE>
__global__ __launch_bounds__(kConvThreads) void k_conv(const __bf16 *__restrict__ X, const __bf16 *__restrict__ Wp, OutArgs o,
                                                       int ntiles, int H, int W)
{
    using Lds = ConvLds<CIN, COUT>;
    constexpr int WS = Lds::WS;
    static_assert(Lds::PS == Patch<CIN>::PS, "patch stride");
    constexpr int KS = CIN / 32;  // K-steps per tap
    constexpr int GPW = WaveSplit<COUT, MODE>::GPW;
    __bf16 *patch = lbcm_conv_lds, *wl = lbcm_conv_lds + Lds::patch_elems;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, q = lane >> 4;
    const int cbase = WaveSplit<COUT, MODE>::cbase(wave);

    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    // the layer's weights Wp[t][co][ci] go to LDS once per workgroup (coalesced 16-byte loads),
    // then each wave takes its fragments from there
    {
        constexpr int NV = 9 * COUT * CIN / 8, NI = (NV + kConvThreads - 1) / kConvThreads;
        u32x4 v[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int k = threadIdx.x + i * kConvThreads;
            if (k < NV) v[i] = *(const u32x4 *)(Wp + (size_t)k * 8);
        }
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int k = threadIdx.x + i * kConvThreads;
            if (k < NV) *(u32x4 *)(wl + (k / (CIN / 8)) * WS + (k % (CIN / 8)) * 8) = v[i];
        }
    }
    // this lane's output channels: cbase + 16 g + 4 q + e
    float bias[GPW][4];
#pragma unroll
    for (int g = 0; g < GPW; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[g][e] = (MODE != 2) ? o.bias[cbase + 16 * g + 4 * q + e] : 0.f;
    Patch<CIN> pre;
    pre.template load<WIDE>(X, tile_coord(tile, H, W), H, W);
    __syncthreads();  // also waits for the bias loads, so that no wait in the loop is for them
    bf16x8 wa[GPW][9][KS];
#pragma unroll
    for (int g = 0; g < GPW; ++g)
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) wa[g][t][ks] = ld8(wl + (t * COUT + cbase + 16 * g + r) * WS + 32 * ks + 8 * q);

    pre.store(patch);
    lds_barrier();
    // Per tile: the next tile's patch loads (the last iteration repeats the last tile's: no branch
    // around the loads), the MFMAs and output stores, then the patch exchange.  Barriers for LDS
    // only: the wait for the patch registers then counts just the loads, and this tile's output
    // stores, issued after them, stay in flight into the next tile's MFMAs.
    // ReLU mask bytes of the training forward: staged in LDS by conv_tile, then one store of COUT / 4
    // bytes per tile pixel (thread t: pixel t; threads past the tile or pixels past the box get an
    // offset past the resource, which is dropped; without masks the resource is empty)
    uint8_t *mstage = (uint8_t *)(wl + Lds::weight_elems);
    constexpr bool MASKS = MODE == 0;
    for (; tile < ntiles; tile += gridDim.x) {
        const TileCoord tc = tile_coord(tile, H, W);
        pre.template load<WIDE>(X, tile_coord(min(tile + (int)gridDim.x, ntiles - 1), H, W), H, W);
        conv_tile<CIN, COUT, MODE, MASKS>(patch, wa, bias, tc, o, H, W, mstage);
        lds_barrier();  // every wave is done with this tile's patch, the mask bytes are in LDS
        if (MASKS) {
            const int rows = min(kTileH, H - tc.y0);
            const size_t tile_px = ((size_t)tc.n * H + tc.y0) * W;
            const rsrc_t rm = make_rsrc(o.mask_out ? o.mask_out + tile_px * (COUT / 4) : nullptr,
                                        o.mask_out ? (uint32_t)rows * W * (COUT / 4) : 0u);
            const int t = min((int)threadIdx.x, kTileH * kTileW - 1), ty = t / kTileW, tx = t % kTileW;
            const bool ok = (int)threadIdx.x < kTileH * kTileW && tc.x0 + tx < W;
            const int off = ok ? (ty * W + tc.x0 + tx) * (COUT / 4) : 0x7fffffff;
            if constexpr (COUT == 64) {
                const u32x4 m = *(const u32x4 *)(mstage + t * 16);
                __builtin_amdgcn_raw_buffer_store_b128(m, rm, off, 0, 0);
            } else {
                const u32x2 m = *(const u32x2 *)(mstage + t * 8);
                __builtin_amdgcn_raw_buffer_store_b64(m, rm, off, 0, 0);
            }
        }
        pre.store(patch);
        lds_barrier();
    }
}

// ------------------------------------------------------------------------------------------
// Two consecutive 64-channel conv layers in one pass (inference): Z = bf16(relu(ba + conv(X, Wa)))
// and then layer b on Z as k_conv does (MODE 0: bf16 ReLU output; MODE 3: the last layer into the
// FP64 planes), one 8 x 32 output tile per workgroup.  Z never leaves LDS: the workgroup stages
// the 12 x 36 input patch (tile plus a two-pixel circular halo), computes Z on the tile plus a
// one-pixel halo (10 x 34) and runs layer b from there, recomputing the halo ring of Z that the
// neighbouring tiles also compute.  Every output sums its taps in the same order as k_conv, so
// the result equals two k_conv launches bit for bit.
//
// Layer a: wave (mg, ng) computes channels [16 ng, 16 ng + 16) of Z rows [5 mg, 5 mg + 5) at Z
// columns 1 .. 32 (ten 16-pixel blocks, input-stationary as in conv_tile) and of Z column 0
// (mg = 0) or 33 (mg = 1), rows 0 .. 9 (one block whose lanes gather their pixels; lanes 10 .. 15
// repeat row 9 and store nothing).  Each layer's weights are staged in LDS once per workgroup
// (every wave takes its A fragments from there); layer b's are requested together with the patch
// and layer a's, kept in registers across LDS-only barriers, and written to LDS once layer a is
// done, when Z also replaces the patch.  LDS: patch (then Z) and one layer's weights.

struct PairLds {
    static constexpr int C = 64, PS = C + 16, WS = C + 8;
    static constexpr int XH = kTileH + 4, XW = kTileW + 4;  // input patch
    static constexpr int ZH = kTileH + 2, ZW = kTileW + 2;  // intermediate (written over the patch)
    static constexpr int x_elems = XH * XW * PS, z_elems = ZH * ZW * PS;
    static constexpr int w_elems = 9 * C * WS;               // one layer's weights, up to 64 outputs
    static constexpr size_t bytes = (size_t)(x_elems + w_elems) * sizeof(__bf16);
};
static_assert(PairLds::z_elems <= PairLds::x_elems, "Z fits where the patch was");
static_assert(PairLds::ZW == kPatchW && PairLds::ZH == kPatchH, "layer b reads Z as a conv patch");

// One layer's packed weights Wp[t][co][ci] (PACK output channels per tap, of which the first
// COUT are staged) on their way to LDS (rows of CIN padded to CIN + 8), in the
// registers of all threads of the workgroup: load() issues the global loads, store() writes
// them to LDS once they have arrived.
template <int CIN, int COUT, int PACK = COUT>
struct WeightStage {
    static constexpr int WS = CIN + 8;
    static constexpr int NV = 9 * COUT * CIN / 8, NI = (NV + kConvThreads - 1) / kConvThreads;
    u32x4 v[NI];

    __device__ __forceinline__ void load(const __bf16 *__restrict__ Wp)
    {
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int k = threadIdx.x + i * kConvThreads;
            const int t = k / (COUT * CIN / 8), rem = k % (COUT * CIN / 8);  // tap, (co, ci / 8) in it
            if (k < NV) v[i] = *(const u32x4 *)(Wp + ((size_t)t * PACK * CIN / 8 + rem) * 8);
        }
    }
    __device__ __forceinline__ void store(__bf16 *wl) const
    {
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int k = threadIdx.x + i * kConvThreads;
            if (k < NV) *(u32x4 *)(wl + (k / (CIN / 8)) * WS + (k % (CIN / 8)) * 8) = v[i];
        }
    }
};

// A fragments of channel group co / 16 from weights staged in LDS: lane (r, q) takes
// W[t][co][ci = 32 ks + 8 q .. + 8]
template <int CIN, int COUT>
__device__ __forceinline__ void lds_frags(const __bf16 *wl, int co, int q, bf16x8 (&wa)[9][CIN / 32])
{
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int ks = 0; ks < CIN / 32; ++ks) wa[t][ks] = ld8(wl + (t * COUT + co) * (CIN + 8) + 32 * ks + 8 * q);
}


template <int COUT, int MODE, int PACK = COUT>
__global__ __launch_bounds__(kConvThreads) void k_pair(const __bf16 *__restrict__ X, const __bf16 *__restrict__ Wa,
                                                       const float *__restrict__ ba, const __bf16 *__restrict__ Wb, OutArgs o,
                                                       int ntiles, int H, int W)
{
    using L = PairLds;
    constexpr int C = L::C, PS = L::PS, KS = C / 32, XW = L::XW, ZW = L::ZW;
    __bf16 *xs = lbcm_conv_lds, *zs = lbcm_conv_lds, *wl = lbcm_conv_lds + L::x_elems;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, q = lane >> 4;
    const int tile = blockIdx.x;
    if (tile >= ntiles) return;
    const TileCoord tc = tile_coord(tile, H, W);
    const int mg = wave & 1, ng = wave >> 1;
    bf16x8 wa[9][KS];
    float bias[4];
    // every global load at once: the patch, layer a's weights, then layer b's, which stay in
    // registers (in flight) until layer a is done
    WeightStage<C, C> sa;
    WeightStage<C, COUT, PACK> sb;
    {
        constexpr int NV = L::XH * XW * (C / 8), NI = (NV + kConvThreads - 1) / kConvThreads;
        const __bf16 *Xn = X + (size_t)tc.n * H * W * C;
        u32x4 v[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int k = threadIdx.x + i * kConvThreads;
            if (k < NV) {
                const int px = k / (C / 8), ch = (k % (C / 8)) * 8;
                const int gy = wrap(tc.y0 - 2 + px / XW, H), gx = wrap(tc.x0 - 2 + px % XW, W);
                v[i] = *(const u32x4 *)(Xn + ((size_t)gy * W + gx) * C + ch);
            }
        }
        sa.load(Wa);
        sb.load(Wb);
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[e] = ba[16 * ng + 4 * q + e];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int k = threadIdx.x + i * kConvThreads;
            if (k < NV) *(u32x4 *)(xs + (k / (C / 8)) * PS + (k % (C / 8)) * 8) = v[i];
        }
        sa.store(wl);
    }
    lds_barrier();
    lds_frags<C, C>(wl, 16 * ng + r, q, wa);
    // Z rows 5 mg + rho (rho < 5) at Z columns 1 + 16 half + r: X rows 5 mg + rho + dyi, X columns
    // 1 + 16 half + r + dxi; then the edge column of Z
    constexpr int RW = 5, NS = 2 * (RW + 2);
    f32x4 acc[2 * RW + 1];
#pragma unroll
    for (int mi = 0; mi <= 2 * RW; ++mi) acc[mi] = f32x4{0, 0, 0, 0};
    {
        bf16x8 fr[2][3][KS];
        auto load_stage = [&](int st, bf16x8 (&f)[3][KS]) {
            const int xr = RW * mg + (st >> 1), half = st & 1;
#pragma unroll
            for (int dxi = 0; dxi < 3; ++dxi)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) f[dxi][ks] = ld8(xs + (xr * XW + 1 + 16 * half + r + dxi) * PS + 32 * ks + 8 * q);
        };
        load_stage(0, fr[0]);
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            if (st + 1 < NS) load_stage(st + 1, fr[(st + 1) & 1]);
            const int py = st >> 1, half = st & 1;
#pragma unroll
            for (int dxi = 0; dxi < 3; ++dxi)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int rho = 0; rho < RW; ++rho) {
                        const int dyi = py - rho;
                        if (dyi < 0 || dyi > 2) continue;
                        acc[2 * rho + half] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[3 * dyi + dxi][ks], fr[st & 1][dxi][ks],
                                                                                      acc[2 * rho + half], 0, 0, 0);
                    }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const int zr = r < L::ZH ? r : L::ZH - 1, zc = mg ? ZW - 1 : 0;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            acc[2 * RW] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                wa[t][ks], ld8(xs + ((zr + t / 3) * XW + zc + t % 3) * PS + 32 * ks + 8 * q), acc[2 * RW], 0, 0, 0);
    lds_barrier();  // every wave is done with the patch and layer a's weights
    auto zstore = [&](int y, int x, const f32x4 &a) {
        bf16x4 v4;
#pragma unroll
        for (int e = 0; e < 4; ++e) v4[e] = (__bf16)fmaxf(a[e] + bias[e], 0.f);
        *(u32x2 *)(zs + (y * ZW + x) * PS + 16 * ng + 4 * q) = __builtin_bit_cast(u32x2, v4);
    };
#pragma unroll
    for (int mi = 0; mi < 2 * RW; ++mi) zstore(RW * mg + (mi >> 1), 1 + 16 * (mi & 1) + r, acc[mi]);
    if (r < L::ZH) zstore(zr, zc, acc[2 * RW]);
    sb.store(wl);
    // layer b
    constexpr int GPW = WaveSplit<COUT, MODE>::GPW;
    const int cb = WaveSplit<COUT, MODE>::cbase(wave);
    float biasb[GPW][4];
#pragma unroll
    for (int g = 0; g < GPW; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) biasb[g][e] = o.bias[cb + 16 * g + 4 * q + e];
    lds_barrier();
    bf16x8 wb[GPW][9][KS];
#pragma unroll
    for (int g = 0; g < GPW; ++g) lds_frags<C, COUT>(wl, cb + 16 * g + r, q, wb[g]);
    conv_tile<C, COUT, MODE>(zs, wb, biasb, tc, o, H, W);
}

// Layers 0 and 1 in one pass (inference): layer 0 as k_first (FP32 MFMA, the bias as the starting
// sum, taps in order) on the tile plus a one-pixel halo, kept in LDS as bf16(relu), then layer 1
// on it as k_conv does (MODE 0), one 8 x 32 tile per workgroup; bit for bit the result of k_first
// and one k_conv launch.  The FP32 state patch covers the tile plus a two-pixel halo and is read
// from the FP64 field planes (the tile's own state also goes to s_out, the residual of the last
// layer).  The wave split of layer 0 over the 10 x 34 intermediate is that of k_pair's layer a;
// layer 1's weights are requested at the start and staged in LDS once layer 0 is done.
// Dynamic LDS: Z and one layer's weights.
__global__ __launch_bounds__(kConvThreads) void k_first_pair(PlaneIn pin, float *__restrict__ s_out, const float *__restrict__ W0,
                                                             const float *__restrict__ b0, const __bf16 *__restrict__ W1,
                                                             OutArgs o, int ntiles, int H, int W)
{
    using L = PairLds;
    constexpr int C = L::C, KS = C / 32, XH = L::XH, XW = L::XW, ZW = L::ZW;
    __shared__ __align__(16) float sp[XH * XW * kStateC];
    __bf16 *zs = lbcm_conv_lds, *wl = lbcm_conv_lds + L::z_elems;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, q = lane >> 4;
    const int tile = blockIdx.x;
    if (tile >= ntiles) return;
    const TileCoord tc = tile_coord(tile, H, W);
    static_assert(XH * XW <= kConvThreads, "one patch pixel per thread");
    const int mg = wave & 1, ng = wave >> 1;
    float w0[9];  // A operand at tap t: lane (r, q) holds W0[t][ci = q][co = 16 ng + r]
    float bias0[4];
    WeightStage<C, C> s1;  // layer 1's weights, in flight during layer 0
    {
        // every global load at once: this thread's patch pixel first, then both layers' weights
        const int k = threadIdx.x, py = k / XW, px = k % XW;
        size_t p = 0;
        double ph = 0, ux = 0, uy = 0, rh = 1;
        if (k < XH * XW) {
            const int gy = wrap(tc.y0 - 2 + py, H), gx = wrap(tc.x0 - 2 + px, W);
            p = ((size_t)tc.n * H + gy) * W + gx;
            ph = pin.phi[p];
            ux = pin.ux[p];
            uy = pin.uy[p];
            rh = pin.rho[p];
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) w0[t] = W0[(kStateC * t + q) * C + 16 * ng + r];
#pragma unroll
        for (int e = 0; e < 4; ++e) bias0[e] = b0[16 * ng + 4 * q + e];
        s1.load(W1);
        if (k < XH * XW) {
            f32x4 v;
            v[0] = (float)ph;
            v[1] = (float)ux * pin.inv_u;
            v[2] = (float)uy * pin.inv_u;
            v[3] = (float)(rh - 1.0) * pin.inv_r;
            if (py >= 2 && py < 2 + kTileH && px >= 2 && px < 2 + kTileW && tc.y0 + py - 2 < H && tc.x0 + px - 2 < W)
                *(f32x4 *)(s_out + p * kStateC) = v;
            *(f32x4 *)(sp + k * kStateC) = v;
        }
    }
    lds_barrier();
    {
        // Z rows 5 mg + rho at Z columns 1 + 16 half + r, and the edge column of Z (lanes 10 .. 15
        // repeat row 9); Z (zr, zc) reads the patch at (zr + dy + 1, zc + dx + 1)
        constexpr int RW = 5;
        const int zr = r < L::ZH ? r : L::ZH - 1, zc = mg ? ZW - 1 : 0;
        f32x4 acc[2 * RW + 1];
#pragma unroll
        for (int mi = 0; mi <= 2 * RW; ++mi)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[mi][e] = bias0[e];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dyi = t / 3, dxi = t % 3;
#pragma unroll
            for (int mi = 0; mi < 2 * RW; ++mi) {
                const float x = sp[((RW * mg + (mi >> 1) + dyi) * XW + 1 + 16 * (mi & 1) + r + dxi) * kStateC + q];
                acc[mi] = __builtin_amdgcn_mfma_f32_16x16x4f32(w0[t], x, acc[mi], 0, 0, 0);
            }
            const float x = sp[((zr + dyi) * XW + zc + dxi) * kStateC + q];
            acc[2 * RW] = __builtin_amdgcn_mfma_f32_16x16x4f32(w0[t], x, acc[2 * RW], 0, 0, 0);
        }
        auto zstore = [&](int y, int x, const f32x4 &a) {
            bf16x4 v4;
#pragma unroll
            for (int e = 0; e < 4; ++e) v4[e] = (__bf16)fmaxf(a[e], 0.f);
            *(u32x2 *)(zs + (y * ZW + x) * L::PS + 16 * ng + 4 * q) = __builtin_bit_cast(u32x2, v4);
        };
#pragma unroll
        for (int mi = 0; mi < 2 * RW; ++mi) zstore(RW * mg + (mi >> 1), 1 + 16 * (mi & 1) + r, acc[mi]);
        if (r < L::ZH) zstore(zr, zc, acc[2 * RW]);
    }
    s1.store(wl);
    constexpr int GPW = WaveSplit<C, 0>::GPW;
    const int cb = WaveSplit<C, 0>::cbase(wave);
    float bias1[GPW][4];
#pragma unroll
    for (int g = 0; g < GPW; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) bias1[g][e] = o.bias[cb + 16 * g + 4 * q + e];
    lds_barrier();
    bf16x8 wb[GPW][9][KS];
#pragma unroll
    for (int g = 0; g < GPW; ++g) lds_frags<C, C>(wl, cb + 16 * g + r, q, wb[g]);
    conv_tile<C, C, 0>(zs, wb, bias1, tc, o, H, W);
}

// ------------------------------------------------------------------------------------------
// Input gradient of the last layer (training): dX[p][ci] = mask(p, ci) sum_t sum_co Wb[t][ci][co]
// dZ[p + d_t][co] with Wb the mirrored pack (as k_conv's MODE 2), where only the kStateC state
// channels of dZ can be nonzero.  The contraction runs over (tap, state channel), k = kStateC t + co
// < 36 padded to two MFMA K steps of 32, instead of over the 32 padded channels of each tap (nine K
// steps): lane (r, q) of K step s holds taps 8 s + 2 q and 8 s + 2 q + 1 (zero past tap 8), four
// channels each, of weight row ci = 16 g + r (A) and of the pixel r of a 16-pixel block (B).  dZ
// holds only the state channels ([P][kStateC], as the loss writes it).  A workgroup takes the tiles
// b, b + G, ... (G the grid); wave w computes tile row w for every channel group; the dZ patch
// (tile plus circular halo, 8 bytes per pixel) goes through LDS, the next tile's requested during
// this one, and so does the output tile, stored in whole pixels.  Products are exact (BF16 x BF16) and summed in FP32, in another order than a
// per-tap K step would take.
constexpr int kLastDgradBlocks = 1024;  // workgroups of k_last_dgrad at most
template <int C>
__global__ __launch_bounds__(kConvThreads) void k_last_dgrad(const __bf16 *__restrict__ dZ, const __bf16 *__restrict__ Wb,
                                                             const uint8_t *__restrict__ mask, __bf16 *__restrict__ dX, int ntiles,
                                                             int H, int W)
{
    constexpr int NG = C / 16, NPX = kPatchH * kPatchW;
    static_assert(kStateC == 4 && NPX <= kConvThreads && kConvThreads / 64 == kTileH && kTileW == 32,
                  "one patch pixel per thread, one tile row per wave, two 16-pixel blocks per row");
    constexpr int PSY = C + 8;  // pixel stride of the staged output tile (bf16)
    __shared__ u32x2 zp[NPX];  // the patch's state channels, four BF16 per pixel
    __shared__ __align__(16) __bf16 ys[kTileH * kTileW * PSY];  // the output tile
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, q = lane >> 4;
    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    // taps of this lane's two halves of K step s (t >= 9 is padding: read tap 8, use zero)
    auto tap = [&](int s, int h) { return 8 * s + 2 * q + h; };
    bf16x8 wa[NG][2];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            u32x2 v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = tap(s, h);
                const u32x2 x = *(const u32x2 *)(Wb + ((size_t)min(t, 8) * C + 16 * g + r) * kOutC);
                v[h] = t < 9 ? x : u32x2{0, 0};
            }
            wa[g][s] = __builtin_bit_cast(bf16x8, u32x4{v[0][0], v[0][1], v[1][0], v[1][1]});
        }
    auto load = [&](int tl) {
        const TileCoord tc = tile_coord(tl, H, W);
        const int k = min((int)threadIdx.x, NPX - 1);
        const int gy = wrap_near(tc.y0 - 1 + k / kPatchW, H), gx = wrap_near(tc.x0 - 1 + k % kPatchW, W);
        return *(const u32x2 *)(dZ + (((size_t)tc.n * H + gy) * W + gx) * kStateC);
    };
    u32x2 pre = load(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const TileCoord tc = tile_coord(tile, H, W);
        // the ReLU mask bytes of this lane's outputs, requested first (channels 16 g + 4 q .. + 3 of
        // pixel r of block hb in tile row w; clamped into the box)
        uint32_t mv[2][NG];
        const int yy = min(tc.y0 + w, H - 1);
#pragma unroll
        for (int hb = 0; hb < 2; ++hb) {
            const size_t p = ((size_t)tc.n * H + yy) * W + min(tc.x0 + 16 * hb + r, W - 1);
#pragma unroll
            for (int g = 0; g < NG; ++g) mv[hb][g] = mask[p * (C / 4) + 4 * g + q];
        }
        if ((int)threadIdx.x < NPX) zp[threadIdx.x] = pre;
        __syncthreads();
        pre = load(min(tile + (int)gridDim.x, ntiles - 1));
        f32x4 acc[2][NG];
#pragma unroll
        for (int hb = 0; hb < 2; ++hb) {
            bf16x8 b[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                u32x2 v[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int t = min(tap(s, h), 8);
                    const u32x2 x = zp[(w + 1 + tap_dy(t)) * kPatchW + 16 * hb + r + 1 + tap_dx(t)];
                    v[h] = tap(s, h) < 9 ? x : u32x2{0, 0};
                }
                b[s] = __builtin_bit_cast(bf16x8, u32x4{v[0][0], v[0][1], v[1][0], v[1][1]});
            }
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                acc[hb][g] = f32x4{0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < 2; ++s) acc[hb][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[g][s], b[s], acc[hb][g], 0, 0, 0);
            }
        }
        // lane (r, q) holds channels 16 g + 4 q .. + 3 of pixel r of block hb: times the ReLU mask of
        // the layer input, staged in LDS, then stored in whole pixels
#pragma unroll
        for (int hb = 0; hb < 2; ++hb) {
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int c0 = 16 * g + 4 * q;
                const uint32_t m = mv[hb][g];
                bf16x4 v4;
#pragma unroll
                for (int e = 0; e < 4; ++e) v4[e] = (__bf16)(((m >> e) & 1u) ? acc[hb][g][e] : 0.f);
                *(u32x2 *)(ys + (w * kTileW + 16 * hb + r) * PSY + c0) = __builtin_bit_cast(u32x2, v4);
            }
        }
        __syncthreads();
        stage_store<C>(ys, dX, tc, H, W);
        __syncthreads();  // every wave is done with the patch and the staged tile
    }
}

// ------------------------------------------------------------------------------------------
// Weight and bias gradients of the last layer (training), whose output gradient dZ can be nonzero
// only in its kStateC state channels.  dW[t][ci][co] = sum_p X[p + d_t][ci] dZ[p][co] = sum_p
// X[p][ci] dZ[p - d_t][co] (the box is periodic), so the tap shifts dZ instead of X and one GEMM
// covers every tap: M = ci (C / 16 blocks), N = (tap, state channel), col = kStateC t + co < 36 in
// three 16-column blocks, K = the 32 pixels of a tile row.  Lane (r, q) holds A = X[pixels 8q ..
// 8q + 7][ci0 + r] (transposing LDS reads of the unshifted tile) and B = dZ[those pixels - d_t][co]
// of its column (zero past column 35).  db[co] = sum_p dZ[p][co]: thread t sums tile pixel t.  A
// workgroup takes the tiles b, b + G, ... (G the grid), staging the X tile (zero past the box
// edge) and the state channels of dZ on the tile plus its circular halo in LDS, with the next
// tile's loads in flight; wave w takes tile rows w and w + 4.  The waves' sums are added in LDS in
// wave order: partial row b holds dW[t][ci][co < kStateC], bias row b db[co < 64] (zero past
// kStateC), both added in a fixed order by k_grad_reduce.
constexpr int kLastDwBlocks = 512;  // workgroups of k_last_dw at most
template <int C>
__global__ __launch_bounds__(kThreads) void k_last_dw(const __bf16 *__restrict__ X, const __bf16 *__restrict__ dZ, int H, int W,
                                                      int ntiles, float *__restrict__ partial, float *__restrict__ db_partial)
{
    constexpr int NI = C / 16, NJ = 3, NCOL = 9 * kStateC, PSX = C + 8, NPX = kPatchH * kPatchW;
    constexpr int NX = kTileH * kTileW * C / 8, NIX = NX / kThreads;  // 16-byte chunks of the X tile
    constexpr int NIZ = (NPX + kThreads - 1) / kThreads;
    static_assert(kStateC == 4 && NCOL <= 16 * NJ && NX % kThreads == 0, "column blocks and X chunks");
    static_assert(kTileW == 32 && kTileH == 2 * (kThreads / 64) && kThreads == kTileH * kTileW,
                  "a K step is one tile row, each wave takes two, one thread per tile pixel");
    __shared__ __align__(16) __bf16 xs[kTileH * kTileW * PSX];
    __shared__ u32x2 zp[NPX];  // state channels of dZ on the patch, four BF16 per pixel
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, q = lane >> 4;
    const int opix = 8 * (lane >> 4) + ((lane & 15) >> 2), och = 4 * (lane & 3);
    // this lane's B columns: offset of patch pixel p - d_t from that of p, and the state channel
    int zoff[NJ], zco[NJ];
    bool zok[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int col = 16 * j + r, t = min(col / kStateC, 8);
        zok[j] = col < NCOL;
        zoff[j] = (1 - tap_dy(t)) * kPatchW + 1 - tap_dx(t);
        zco[j] = col % kStateC;
    }
    f32x4 acc[NI][NJ];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    float bsum[kStateC] = {0, 0, 0, 0};
    u32x4 vx[NIX];
    u32x2 vz[NIZ];
    auto load = [&](int tile) {
        const TileCoord tc = tile_coord(tile, H, W);
#pragma unroll
        for (int i = 0; i < NIX; ++i) {
            const int k = threadIdx.x + i * kThreads, px = k / (C / 8), ch = (k % (C / 8)) * 8;
            const int y = tc.y0 + px / kTileW, x = tc.x0 + px % kTileW;
            vx[i] = u32x4{0, 0, 0, 0};
            if (y < H && x < W) vx[i] = *(const u32x4 *)(X + (((size_t)tc.n * H + y) * W + x) * C + ch);
        }
#pragma unroll
        for (int i = 0; i < NIZ; ++i) {
            const int k = min((int)threadIdx.x + i * kThreads, NPX - 1);
            const int gy = wrap_near(tc.y0 - 1 + k / kPatchW, H), gx = wrap_near(tc.x0 - 1 + k % kPatchW, W);
            vz[i] = *(const u32x2 *)(dZ + (((size_t)tc.n * H + gy) * W + gx) * kStateC);
        }
    };
    int tile = blockIdx.x;
    if (tile < ntiles) load(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const TileCoord tc = tile_coord(tile, H, W);
        __syncthreads();  // every wave is done with the previous tile's LDS
#pragma unroll
        for (int i = 0; i < NIX; ++i) {
            const int k = threadIdx.x + i * kThreads;
            *(u32x4 *)(xs + (k / (C / 8)) * PSX + (k % (C / 8)) * 8) = vx[i];
        }
#pragma unroll
        for (int i = 0; i < NIZ; ++i) {
            const int k = threadIdx.x + i * kThreads;
            if (k < NPX) zp[k] = vz[i];
        }
        __syncthreads();
        if (tile + (int)gridDim.x < ntiles) load(tile + gridDim.x);
        {
            const int ty = threadIdx.x / kTileW, tx = threadIdx.x % kTileW;
            if (tc.y0 + ty < H && tc.x0 + tx < W) {
                const bf16x4 z = __builtin_bit_cast(bf16x4, zp[(ty + 1) * kPatchW + tx + 1]);
#pragma unroll
                for (int c = 0; c < kStateC; ++c) bsum[c] += (float)z[c];
            }
        }
        const __bf16 *zb = reinterpret_cast<const __bf16 *>(zp);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int y = w + (kThreads / 64) * h;  // tile row
            bf16x8 a[NI], b[NJ];
#pragma unroll
            for (int i = 0; i < NI; ++i) a[i] = ld_tr(xs + y * kTileW * PSX, opix * PSX + 16 * i + och, PSX);
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const __bf16 v = zb[((y * kPatchW + 8 * q + e) + zoff[j]) * kStateC + zco[j]];
                    b[j][e] = zok[j] ? v : (__bf16)0.f;
                }
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int j = 0; j < NJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    // D of block (i, j): lane (r, q) holds ci = 16 i + 4 q + e, col = 16 j + r.  Waves 1 .. 3 and
    // every thread's bias sums go to LDS (over the X tile); wave 0 adds them in order.
    constexpr int NW = kThreads / 64;
    static_assert(((NW - 1) * NCOL * C + kThreads * kStateC) * sizeof(float) <= sizeof(xs), "the sums fit the X tile");
    float *red = reinterpret_cast<float *>(xs), *bred = red + (NW - 1) * NCOL * C;
    __syncthreads();
    if (w > 0)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int col = 16 * j + r;
            if (col < NCOL)
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int e = 0; e < 4; ++e) red[((w - 1) * NCOL + col) * C + 16 * i + 4 * q + e] = acc[i][j][e];
        }
#pragma unroll
    for (int c = 0; c < kStateC; ++c) bred[threadIdx.x * kStateC + c] = bsum[c];
    __syncthreads();
    if (w > 0) return;
    {
        float sb = 0;
        if (lane < kStateC)
            for (int t = 0; t < kThreads; ++t) sb += bred[t * kStateC + lane];
        db_partial[(size_t)blockIdx.x * 64 + lane] = sb;
    }
    float *out = partial + (size_t)blockIdx.x * 9 * C * kStateC;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int col = 16 * j + r;
        if (col < NCOL)
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int ci = 16 * i + 4 * q + e;
                    float v = acc[i][j][e];
#pragma unroll
                    for (int u = 0; u < NW - 1; ++u) v += red[(u * NCOL + col) * C + ci];
                    out[((col / kStateC) * C + ci) * kStateC + col % kStateC] = v;
                }
    }
}

// ------------------------------------------------------------------------------------------
// weight gradient of layers with 32 input channels (64: k_conv_dw_strip below):
// partial[chunk][t][ci][co] = sum over the chunk's pixels p of X[p + d_t][ci] dZ[p][co].  A
// workgroup owns one tap and one chunk; it stages 64 pixels of X (shifted) and dZ in LDS with
// 16-byte loads (pixel stride padded by 16 bytes), then each wave accumulates its share of the
// (ci, co) 16 x 16 tiles with MFMAs whose K dimension is the pixels.

__global__ __launch_bounds__(kThreads) void k_conv_dw(const __bf16 *__restrict__ X, int cin, const __bf16 *__restrict__ dZ,
                                                      int cout, uint32_t P, int H, int W, float *__restrict__ partial)
{
    constexpr int PS = 64 + 8;
    __shared__ __align__(16) __bf16 sx[kDwPix * PS];
    __shared__ __align__(16) __bf16 sz[kDwPix * PS];
    const int t = blockIdx.y;
    const uint32_t chunk = blockIdx.x;
    const uint32_t p_begin = chunk * kDwChunk, p_end = min(P, p_begin + kDwChunk);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int nt = cout / 16, ntiles = (cin / 16) * nt;  // <= 16 tiles, 4 per wave
    f32x4 acc[4];
    for (int i = 0; i < 4; ++i) acc[i] = f32x4{0, 0, 0, 0};
    const int dy = tap_dy(t), dx = tap_dx(t);
    for (uint32_t p0 = p_begin; p0 < p_end; p0 += kDwPix) {
        for (int v = threadIdx.x; v < kDwPix * cin / 8; v += kThreads) {
            const int px = v / (cin / 8), ch = (v % (cin / 8)) * 8;
            const uint32_t p = p0 + px;
            u32x4 val = {0, 0, 0, 0};
            if (p < p_end) val = *(const u32x4 *)(X + (size_t)shift_pix(p, dy, dx, H, W) * cin + ch);
            *(u32x4 *)(sx + px * PS + ch) = val;
        }
        for (int v = threadIdx.x; v < kDwPix * cout / 8; v += kThreads) {
            const int px = v / (cout / 8), ch = (v % (cout / 8)) * 8;
            const uint32_t p = p0 + px;
            u32x4 val = {0, 0, 0, 0};
            if (p < p_end) val = *(const u32x4 *)(dZ + (size_t)p * cout + ch);
            *(u32x4 *)(sz + px * PS + ch) = val;
        }
        __syncthreads();
        for (int s = 0; s < 4; ++s) {
            const int tile = wave * 4 + s;
            if (tile >= ntiles) break;
            const int mi = tile / nt, ni = tile % nt;
#pragma unroll
            for (int kk = 0; kk < kDwPix; kk += 32) {
                bf16x8 a, b;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int px = kk + 8 * q + e;
                    a[e] = sx[px * PS + 16 * mi + r];  // A[ci][pixel]
                    b[e] = sz[px * PS + 16 * ni + r];  // B[pixel][co]
                }
                acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[s], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    float *out = partial + ((size_t)chunk * 9 + t) * cin * cout;
    for (int s = 0; s < 4; ++s) {
        const int tile = wave * 4 + s;
        if (tile >= ntiles) break;
        const int mi = tile / nt, ni = tile % nt;
        for (int e = 0; e < 4; ++e) out[(size_t)(16 * mi + 4 * q + e) * cout + 16 * ni + r] = acc[s][e];
    }
}

// Weight gradient of a layer with 64 input channels (the 64 -> 64 layers; the last layer has
// k_last_dw), all 9 taps in one pass: partial[g][t][ci][co] = sum over the pixels p of work unit
// g of X[p + d_t][ci] dZ[p][co].  A work unit is a run of
// rows of one 32-column strip of one sample, walked row by row.  The pixels are the K dimension
// of the MFMAs while the activations are channel-packed (NHWC); the rows are staged in LDS as they
// are (34 pixels of X from column sx - 1, 32 of dZ, 16-byte copies) and the operands are read
// with the transposing LDS load ds_read_b64_tr_b16: within each 16 lanes, lane 4 i + a receives
// element a of the 8-byte reads of lanes i, i + 4, i + 8, i + 12.  So lane S reads the four
// channels 4 (S % 4) .. + 3 of pixel 8 (S / 16) + 4 h + (S % 16) / 4 for half h of the fragment,
// and lane (r, q) ends with the pixels 8 q .. 8 q + 7 of channel r, the MFMA's K layout; a tap's
// column shift dx is an offset of the pixel.  X rows are kept in a ring of four (row y reads
// y - 1 .. y + 1 while y + 2 is written) and dZ rows in two buffers, so one barrier per row
// suffices; each thread copies one or two 16-byte chunks per row, loaded kDwAhead rows ahead.
// Wave w owns input channels [16 (w % 4), + 16) and the taps [5 (w / 4), min(9, 5 (w / 4) + 5)),
// keeping those taps x COUT / 16 output blocks in registers.  The unit's bias gradient (sum of dZ
// over its pixels) rides along with the dZ staging and goes to db_partial[g][co].

constexpr int kDwStrip = 32;            // strip width: one MFMA K step
constexpr int kDwXPix = kDwStrip + 2;   // staged X pixels per row
constexpr int kDwPSX = 64 + 8;          // LDS pixel stride (bf16) of X
constexpr int kDwThreads = 512;         // eight waves
constexpr int kDwSlots = 4;             // X rows in the LDS ring
constexpr int kDwAhead = 4;             // rows of global loads in flight
constexpr int kDwXChunks = kDwXPix * 8;  // 16-byte chunks of one X row

template <int COUT>
struct DwLds {
    static constexpr int PSZ = COUT + 8;                           // LDS pixel stride of dZ
    static constexpr int x_elems = kDwSlots * kDwXPix * kDwPSX;    // [slot][pixel][ci]
    static constexpr int z_elems = 2 * kDwStrip * PSZ;             // [buffer][pixel][co]
    static constexpr size_t bytes = (size_t)(x_elems + z_elems) * sizeof(__bf16);
};

template <int COUT>
__global__ __launch_bounds__(kDwThreads) void k_conv_dw_strip(const __bf16 *__restrict__ X, const __bf16 *__restrict__ dZ, int H,
                                                              int W, int seg, int units_per_strip, float *__restrict__ partial,
                                                              float *__restrict__ db_partial)
{
    using L = DwLds<COUT>;
    constexpr int NJ = COUT / 16, PSZ = L::PSZ;
    constexpr int ZCH = COUT / 8, NZC = kDwStrip * ZCH;  // 16-byte chunks of a dZ pixel and row
    constexpr int NCH = kDwXChunks + NZC;                // chunks of a row of both
    static_assert(NCH <= 2 * kDwThreads, "one or two chunks per thread");
    __bf16 *xs = lbcm_conv_lds, *zs = lbcm_conv_lds + L::x_elems;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, q = lane >> 4;
    const int cg = w & 3;
    const int nstrips = (W + kDwStrip - 1) / kDwStrip;
    const int strip = blockIdx.x / units_per_strip, part = blockIdx.x % units_per_strip;
    const int n = strip / nstrips, sx = (strip % nstrips) * kDwStrip;
    const int ya = part * seg, yb = min(H, ya + seg);
    const __bf16 *Xn = X + (size_t)n * H * W * 64;
    const __bf16 *Zn = dZ + (size_t)n * H * W * COUT;

    // staging: thread t copies chunk t and, if t + kDwThreads < NCH, chunk t + kDwThreads; chunk c
    // < kDwXChunks is X pixel c / 8 (column sx - 1 + c / 8, wrapped), channels 8 (c % 8) ..; the
    // rest are dZ pixel c' / ZCH (column sx + c' / ZCH), channels 8 (c' % ZCH) .., c' = c - kDwXChunks
    struct Chunk {
        bool x, valid, inside;  // X or dZ; a chunk at all; dZ column inside the box
        int gcol, ch, lds;      // global column, channel, LDS offset within a row (slot/buffer 0)
    };
    auto chunk = [&](int c) {
        Chunk k;
        k.valid = c < NCH;
        c = min(c, NCH - 1);
        k.x = c < kDwXChunks;
        if (k.x) {
            const int j = c / 8;
            k.gcol = wrap(sx - 1 + j, W);
            k.ch = 8 * (c % 8);
            k.lds = j * kDwPSX + k.ch;
            k.inside = true;
        } else {
            const int cz = c - kDwXChunks, j = cz / ZCH;
            k.inside = sx + j < W;
            k.gcol = min(sx + j, W - 1);
            k.ch = 8 * (cz % ZCH);
            k.lds = L::x_elems + j * PSZ + k.ch;
        }
        return k;
    };
    const Chunk c0 = chunk(threadIdx.x), c1 = chunk(threadIdx.x + kDwThreads);
    constexpr bool TWO = NCH > kDwThreads;
    // For the argument y an X chunk loads X row y + 1 and a dZ chunk dZ row y: what iteration
    // y - 1 stores.  No branches around the loads (clamped indices), so that the compiler waits
    // for exactly the row it stores while later rows stay in flight.
    auto load1 = [&](const Chunk &k, int y) {
        const __bf16 *src = k.x ? Xn + ((size_t)wrap(y + 1, H) * W + k.gcol) * 64 + k.ch
                                : Zn + ((size_t)min(y, H - 1) * W + k.gcol) * COUT + k.ch;
        return *(const u32x4 *)src;
    };
    auto slot_off = [&](int yx) { return ((yx - ya + 1) % kDwSlots) * kDwXPix * kDwPSX; };  // yx >= ya - 1
    auto buf_off = [&](int yz) { return ((yz - ya) & 1) * kDwStrip * PSZ; };
    // the bias gradient: a dZ chunk's thread sums its eight channels of its pixel over the stored
    // rows, in row order
    float bsum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    auto store1 = [&](const Chunk &k, int yx, int yz, const u32x4 &v) {
        const bool zero = !k.x && !(k.inside && yz < yb);
        const u32x4 s = zero ? u32x4{0, 0, 0, 0} : v;
        if (k.valid) *(u32x4 *)(lbcm_conv_lds + k.lds + (k.x ? slot_off(yx) : buf_off(yz))) = s;
        if (!k.x && k.valid) {
            const bf16x8 b = __builtin_bit_cast(bf16x8, s);
#pragma unroll
            for (int e = 0; e < 8; ++e) bsum[e] += (float)b[e];
        }
    };
    struct Row {
        u32x4 v0, v1;
    };
    auto load = [&](int y, Row &f) {
        f.v0 = load1(c0, y);
        if (TWO) f.v1 = load1(c1, y);
    };
    auto store = [&](int yx, int yz, const Row &f) {
        store1(c0, yx, yz, f.v0);
        if (TWO) store1(c1, yx, yz, f.v1);
    };

    // this lane's operand offsets (pixel offset of half 0 times the stride, plus the channel)
    const int opix = 8 * (lane >> 4) + ((lane & 15) >> 2), och = 4 * (lane & 3);
    Row fifo[kDwAhead];
    {
        // X rows ya - 1 .. ya + 2 and dZ rows ya, ya + 1 before the loop (each dZ row stored once)
        Row f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            f.v0 = load1(c0, c0.x ? ya - 2 + k : ya + min(k, 1));
            if (TWO) f.v1 = load1(c1, c1.x ? ya - 2 + k : ya + min(k, 1));
            if (c0.x || k < 2) store1(c0, ya - 1 + k, ya + k, f.v0);
            if (TWO && (c1.x || k < 2)) store1(c1, ya - 1 + k, ya + k, f.v1);
        }
    }
    // FIFO slot u: what iteration y stores when y = ya + u (mod kDwAhead), X row y + 3 and dZ row
    // y + 2, requested kDwAhead iterations earlier
#pragma unroll
    for (int u = 0; u < kDwAhead; ++u) load(ya + u + 2, fifo[u]);
    lds_barrier();
    const int yend = ya + (yb - ya + kDwAhead - 1) / kDwAhead * kDwAhead;  // rows past yb add zero
    // the row loop and the output of taps [T0, T0 + NT), compile-time constants of each half of
    // the waves
    auto rows = [&](auto t0c, auto ntc) {
        constexpr int T0 = decltype(t0c)::value, NT = decltype(ntc)::value;
        f32x4 acc[NT][NJ];
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
            for (int jn = 0; jn < NJ; ++jn) acc[i][jn] = f32x4{0, 0, 0, 0};
        // The operands of row y + 1 are read during row y's MFMAs (two register sets): row y + 1
        // needs X rows y .. y + 2 and dZ row y + 1, stored one iteration ahead, while this
        // iteration writes X row y + 3 and dZ row y + 2 into the slot and buffer that row y's
        // operands (read in the previous iteration, before its barrier) came from.
        bf16x8 b[2][NJ], a[2][NT];
        auto operands = [&](int y, bf16x8 (&bo)[NJ], bf16x8 (&ao)[NT]) {
#pragma unroll
            for (int jn = 0; jn < NJ; ++jn) bo[jn] = ld_tr(zs + buf_off(y), opix * PSZ + 16 * jn + och, PSZ);
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                const int t = T0 + i;
                ao[i] = ld_tr(xs + slot_off(y + t / 3 - 1), (opix + t % 3) * kDwPSX + 16 * cg + och, kDwPSX);
            }
        };
        static_assert(kDwAhead % 2 == 0, "the register set of row y is y - ya mod 2");
        operands(ya, b[0], a[0]);
        // every wave's reads of row ya are done before the first iteration overwrites the slot of
        // X row ya - 1 and the buffer of dZ row ya (later iterations get this from their barrier)
        lds_barrier();
        for (int y0 = ya; y0 < yend; y0 += kDwAhead) {
#pragma unroll
            for (int u = 0; u < kDwAhead; ++u) {
                const int y = y0 + u, cur = u & 1;
                operands(y + 1, b[cur ^ 1], a[cur ^ 1]);  // the last iteration reads rows past yend: stored, unused
#pragma unroll
                for (int i = 0; i < NT; ++i)
#pragma unroll
                    for (int jn = 0; jn < NJ; ++jn)
                        acc[i][jn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cur][i], b[cur][jn], acc[i][jn], 0, 0, 0);
                store(y + 3, y + 2, fifo[u]);
                load(y + kDwAhead + 2, fifo[u]);
                lds_barrier();
            }
        }
        // D of block (t, jn): lane (r, q) holds ci = 16 cg + 4 q + e, co = 16 jn + r
        float *out = partial + (size_t)blockIdx.x * 9 * 64 * COUT;
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
            for (int jn = 0; jn < NJ; ++jn)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    out[((size_t)(T0 + i) * 64 + 16 * cg + 4 * q + e) * COUT + 16 * jn + r] = acc[i][jn][e];
    };
    if (w < 4)
        rows(std::integral_constant<int, 0>{}, std::integral_constant<int, 5>{});
    else
        rows(std::integral_constant<int, 5>{}, std::integral_constant<int, 4>{});
    // bias partial of this unit: each dZ chunk thread's sums to LDS (the dZ buffers are free after
    // the last barrier), then thread co adds the 32 pixels' sums of channel co in pixel order
    float *red = (float *)(lbcm_conv_lds + L::x_elems);  // [pixel][COUT]
    static_assert(kDwStrip * COUT * sizeof(float) <= L::z_elems * sizeof(__bf16), "bias sums fit the dZ buffers");
    auto put = [&](const Chunk &k, int c) {
        if (!k.x && k.valid) {
            const int cz = c - kDwXChunks;
#pragma unroll
            for (int e = 0; e < 8; ++e) red[(cz / ZCH) * COUT + k.ch + e] = bsum[e];
        }
    };
    put(c0, threadIdx.x);
    if (TWO && threadIdx.x + kDwThreads < NCH) put(c1, threadIdx.x + kDwThreads);
    __syncthreads();
    if ((int)threadIdx.x < COUT) {
        float sb = 0;
        for (int j = 0; j < kDwStrip; ++j) sb += red[j * COUT + threadIdx.x];
        db_partial[(size_t)blockIdx.x * 64 + threadIdx.x] = sb;
    }
}

// Gradient sums of one layer in one launch, each in a fixed order (two runs give bitwise equal
// gradients):
//   dW[t][ci][co] = sum_c wp[c][t][ci][co] over the nw_rows per-unit partials (padded cin x cout,
//                   written at the real size cin_r x cout_r), in the first ceil(9 cin_r cout_r / 64)
//                   workgroups;
//   db[j] = sum_i bp[i ld_b + j] (j < ncols_b), in the workgroups after them.
// A workgroup owns 64 outputs, one per lane; wave v of its kSumWaves sums the rows v, v + kSumWaves,
// ... in row order with four loads in flight, and the wave sums are then added in a fixed tree.
constexpr int kSumWaves = 16;
__global__ __launch_bounds__(kSumWaves * 64) void k_grad_reduce(const float *__restrict__ wp, int nw_rows, int cin, int cout,
                                                                int cin_r, int cout_r, float *__restrict__ dW,
                                                                const float *__restrict__ bp, int nb_rows, int ld_b, int ncols_b,
                                                                float *__restrict__ db)
{
    __shared__ float red[kSumWaves][64];
    const int l = threadIdx.x & 63, v = threadIdx.x >> 6;
    const int nw = 9 * cin_r * cout_r, wblocks = (nw + 63) / 64;
    const float *src;
    size_t ld;
    int rows, j;
    bool ok;
    float *dst;
    if ((int)blockIdx.x < wblocks) {
        j = blockIdx.x * 64 + l;
        ok = j < nw;
        const int jj = ok ? j : 0;
        const int t = jj / (cin_r * cout_r), rem = jj % (cin_r * cout_r), ci = rem / cout_r, co = rem % cout_r;
        src = wp + ((size_t)t * cin + ci) * cout + co;
        ld = (size_t)9 * cin * cout;
        rows = nw_rows;
        dst = dW;
    } else {
        j = (blockIdx.x - wblocks) * 64 + l;
        ok = j < ncols_b;
        src = bp + (ok ? j : 0);
        ld = (size_t)ld_b;
        rows = nb_rows;
        dst = db;
    }
    float sum = 0;
    if (ok) {
        int i = v;
        for (; i + 3 * kSumWaves < rows; i += 4 * kSumWaves) {
            const float a0 = src[(size_t)i * ld], a1 = src[(size_t)(i + kSumWaves) * ld];
            const float a2 = src[(size_t)(i + 2 * kSumWaves) * ld], a3 = src[(size_t)(i + 3 * kSumWaves) * ld];
            sum += a0;
            sum += a1;
            sum += a2;
            sum += a3;
        }
        for (; i < rows; i += kSumWaves) sum += src[(size_t)i * ld];
    }
    red[v][l] = sum;
    __syncthreads();
#pragma unroll
    for (int k = kSumWaves / 2; k > 0; k >>= 1) {
        if (v < k) red[v][l] += red[v + k][l];
        __syncthreads();
    }
    if (v == 0 && ok) dst[j] = red[0][l];
}

// bias gradient db[co] = sum_p dZ[p][co]: per-block partial sums (then k_grad_reduce)
__global__ __launch_bounds__(256) void k_db_partial(const __bf16 *__restrict__ dZ, int cout, uint32_t P,
                                                    float *__restrict__ partial)
{
    // block b sums pixels [b * 1024, (b+1) * 1024) for all channels; thread = channel + 64 * slice
    __shared__ float red[256];
    const int c = threadIdx.x % 64, slice = threadIdx.x / 64;
    const uint32_t p0 = blockIdx.x * 1024u;
    float s = 0;
    if (c < cout)
        for (uint32_t p = p0 + slice; p < min(P, p0 + 1024u); p += 4) s += (float)dZ[(size_t)p * cout + c];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 64) {
        const float v = red[threadIdx.x] + red[threadIdx.x + 64] + red[threadIdx.x + 128] + red[threadIdx.x + 192];
        partial[(size_t)blockIdx.x * 64 + threadIdx.x] = v;
    }
}

// ------------------------------------------------------------------------------------------
// loss: mean over pixels and the kStateC state channels of ((pred - target) / alpha_c)^2; the
// gradient of the last layer's pre-scale output is 2 (pred - target) / (alpha_c kStateC P), stored
// as [P][kStateC] BF16 (the last layer's gradient kernels read only these channels).
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ pred, const float *__restrict__ target, uint32_t P,
                                              float ia0, float ia1, float ia2, float ia3, __bf16 *__restrict__ dZ,
                                              float *__restrict__ partial)
{
    __shared__ float red[256];
    const float scale = 2.0f / ((float)kStateC * (float)P);
    const float ia[kStateC] = {ia0, ia1, ia2, ia3};
    float s = 0;
    for (uint32_t p = blockIdx.x * 256u + threadIdx.x; p < P; p += gridDim.x * 256u) {
        const f32x4 a = *(const f32x4 *)(pred + (size_t)p * kStateC), b = *(const f32x4 *)(target + (size_t)p * kStateC);
        bf16x4 g;
#pragma unroll
        for (int c = 0; c < kStateC; ++c) {
            const float d = (a[c] - b[c]) * ia[c];
            s += d * d;
            g[c] = (__bf16)(scale * d);
        }
        *(u32x2 *)(dZ + (size_t)p * kStateC) = __builtin_bit_cast(u32x2, g);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------------------------------
// packing and optimiser

// where the weights of one layer >= 1 sit in the parameter vector and in its two packs
struct PackEntry {
    int64_t w_off;                 // first weight W[0][0][0] in the parameter vector
    int nw, cin_r, cout_r, cin, cout;  // 9 cin_r cout_r weights; real and padded channel counts
    __bf16 *Wf, *Wb;
};

// master W[t][ci][co] (ci < cin_r, co < cout_r) -> Wf[t][co][ci] and Wb[t'][ci][co] = W[8 - t'][ci][co]
// in BF16, padded to (cin, cout) with zeros
__global__ void k_pack(const float *__restrict__ Wm, int cin_r, int cout_r, int cin, int cout, __bf16 *__restrict__ Wf,
                       __bf16 *__restrict__ Wb)
{
    const int n = 9 * cin * cout;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int t = i / (cin * cout), rem = i % (cin * cout);
        // forward pack index i = (t, co, ci)
        const int co = rem / cin, ci = rem % cin;
        const float vf = (ci < cin_r && co < cout_r) ? Wm[((size_t)t * cin_r + ci) * cout_r + co] : 0.f;
        Wf[i] = (__bf16)vf;
        // mirrored pack index i = (t', ci, co): Wb[t'][ci][co] = W[8 - t'][ci][co]
        const int ci2 = rem / cout, co2 = rem % cout;
        const int ts = 8 - t;
        const float vb = (ci2 < cin_r && co2 < cout_r) ? Wm[((size_t)ts * cin_r + ci2) * cout_r + co2] : 0.f;
        Wb[i] = (__bf16)vb;
    }
}

// Adam on the FP32 masters; with a pack table (packs already made, their zero padding in place)
// each updated weight of layers 1 .. L-1 is also written to its two BF16 packs, as k_pack would.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       size_t n, float lr, float b1, float b2, float eps, float c1, float c2, const PackEntry *__restrict__ tab,
                       int ntab)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1 - b1) * gi;
        const float vi = b2 * v[i] + (1 - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        for (int k = 0; k < ntab; ++k) {
            const PackEntry e = tab[k];
            const int64_t j = (int64_t)i - e.w_off;
            if (j < 0 || j >= e.nw) continue;
            const int t = (int)(j / (e.cin_r * e.cout_r)), rem = (int)(j % (e.cin_r * e.cout_r));
            const int ci = rem / e.cout_r, co = rem % e.cout_r;
            e.Wf[((size_t)t * e.cout + co) * e.cin + ci] = (__bf16)pi;
            e.Wb[((size_t)(8 - t) * e.cin + ci) * e.cout + co] = (__bf16)pi;
        }
    }
}

// state planes (FP64, [B][H][W] each) -> FP32 [P][4] = (phi, v_x / u_scale, v_y / u_scale,
// (rho - 1) / rho_scale)
__global__ void k_from_planes(const double *__restrict__ phi, const double *__restrict__ ux, const double *__restrict__ uy,
                              const double *__restrict__ rho, float inv_u, float inv_r, uint32_t P, float *__restrict__ s)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        f32x4 v;
        v[0] = (float)phi[p];
        v[1] = (float)ux[p] * inv_u;
        v[2] = (float)uy[p] * inv_u;
        v[3] = (float)(rho[p] - 1.0) * inv_r;
        *(f32x4 *)(s + (size_t)p * kStateC) = v;
    }
}

// A training batch from recorded frames: sample b of the state is frame idx[b] of the FP64 field
// planes frames[c][f][y][x] (c = phi, v_x, v_y, rho), under symmetry k of the square lattice
// (transpose if k & 4, then flip y if k & 2, then flip x if k & 1, velocity components swapped and
// negated with it), converted as k_from_planes does.  The transform only moves and negates
// values, so the result equals transforming the planes first.  One workgroup per 32 x 32 tile of
// one sample: the tile's source pixels are read along source rows (under a transposing symmetry
// consecutive threads take consecutive tile rows, which are consecutive source columns), kept in
// LDS converted, and written along state rows, so both sides stay coalesced.  Coordinates past
// the box are clamped on the read side (branch-free) and skipped on the write side.
constexpr int kGatherTile = 32;
__global__ __launch_bounds__(256) void k_gather_states(const double *__restrict__ frames, int64_t nframes, const int32_t *__restrict__ idx, int k,
                                                       int H, int W, float inv_u, float inv_r, float *__restrict__ s)
{
    constexpr int T = kGatherTile, RPP = 256 / T;  // tile rows per pass of the workgroup
    __shared__ f32x4 tile[T][T + 1];
    const int tiles_x = (W + T - 1) / T, tiles = tiles_x * ((H + T - 1) / T);
    const int b = blockIdx.x / tiles, rem = blockIdx.x % tiles;
    const int ty0 = rem / tiles_x * T, tx0 = rem % tiles_x * T;
    const size_t hw = (size_t)H * W, plane = (size_t)nframes * hw, base = (size_t)idx[b] * hw;
    const bool tr = k & 4;
    const int a = threadIdx.x % T, c = threadIdx.x / T;
#pragma unroll
    for (int m = 0; m < T / RPP; ++m) {
        const int i = tr ? a : c + RPP * m, j = tr ? c + RPP * m : a;  // tile row, tile column
        const int y = min(ty0 + i, H - 1), x = min(tx0 + j, W - 1);
        const int yf = (k & 2) ? H - 1 - y : y, xf = (k & 1) ? W - 1 - x : x;
        const int ys = tr ? xf : yf, xs = tr ? yf : xf;
        const size_t at = base + (size_t)ys * W + xs;
        const double vx = frames[plane + at], vy = frames[2 * plane + at];
        const double ux = tr ? vy : vx, uy = tr ? vx : vy;
        f32x4 v;
        v[0] = (float)frames[at];
        v[1] = (float)((k & 1) ? -ux : ux) * inv_u;
        v[2] = (float)((k & 2) ? -uy : uy) * inv_u;
        v[3] = (float)(frames[3 * plane + at] - 1.0) * inv_r;
        tile[i][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < T / RPP; ++m) {
        const int i = c + RPP * m, y = ty0 + i, x = tx0 + a;
        if (y < H && x < W) *(f32x4 *)(s + (((size_t)b * H + y) * W + x) * kStateC) = tile[i][a];
    }
}

// partial sums, one set per block (FP64), of the check: (phi_a - phi_b)^2, phi_b^2,
// |v_a - v_b|^2 and |v_b|^2 over P points; a and b hold (phi, v_x, v_y) planes
constexpr int kErrBlocks = 256, kErrSums = 4;
__global__ __launch_bounds__(256) void k_err_partial(const double *__restrict__ a, const double *__restrict__ b, uint32_t P,
                                                     double *__restrict__ partial)
{
    __shared__ double red[kErrSums][256];
    double acc[kErrSums] = {0, 0, 0, 0};
    for (uint32_t p = blockIdx.x * 256u + threadIdx.x; p < P; p += gridDim.x * 256u) {
        const double d = a[p] - b[p];
        acc[0] += d * d;
        acc[1] += b[p] * b[p];
#pragma unroll
        for (int c = 1; c < 3; ++c) {
            const double bv = b[(size_t)c * P + p], dv = a[(size_t)c * P + p] - bv;
            acc[2] += dv * dv;
            acc[3] += bv * bv;
        }
    }
#pragma unroll
    for (int k = 0; k < kErrSums; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < kErrSums; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < kErrSums) partial[blockIdx.x * kErrSums + threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace

// ==========================================================================================
// host side

struct lbcm_net {
    int batch = 0, H = 0, W = 0, C = 0, L = 0;
    uint32_t P = 0;
    hipStream_t stream = nullptr;
    int ntiles = 0;                             // 8 x 32 tiles over the batch
    int conv_grid = 0;                          // workgroups of a conv launch (grid-stride over tiles)
    std::vector<int> cin_r, cout_r, cin, cout;  // real and padded channel counts per layer
    std::vector<size_t> w_off, b_off;           // offsets of each layer in the parameter vector
    size_t nparams = 0;
    float alpha[kStateC] = {1.f, 1.f, 1.f, 1.f};  // output scale per state channel
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    std::vector<__bf16 *> Wf, Wb;               // BF16 packs of layers 1 .. L-1
    std::vector<__bf16 *> act;                  // act[l] = input of layer l >= 1 (relu output of layer l - 1)
    std::vector<uint8_t *> mask8;               // ReLU mask of act[l] from the training forward (bit e of byte [p][c / 4]: act > 0)
    __bf16 *dz_a = nullptr, *dz_b = nullptr;    // gradient ping-pong buffers (P x 64)
    __bf16 *dz_last = nullptr;                  // gradient of the last layer's output, state channels (P x kStateC)
    PackEntry *pack_table = nullptr;            // where the Adam update writes the BF16 packs of layers 1 .. L-1
    int32_t *gather_idx = nullptr;              // frame indices of lbcm_net_gather_states (batch)
    float *resid = nullptr, *out = nullptr;     // FP32 [P][kStateC]: input state, output state
    float *dw_partial = nullptr, *db_partial = nullptr, *loss_partial = nullptr, *first_partial = nullptr;
    int loss_blocks = 0;
    int dw_seg = 0, dw_units_per_strip = 0, dw_units = 0;  // work units of k_conv_dw_strip
    bool packed = false;
    std::string err;
};

namespace {

std::string g_net_error;

int nfail(lbcm_net *n, int code, const std::string &m)
{
    if (n) n->err = m;
    return code;
}

#define NHIP(n, call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return nfail(n, LBCM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

int grid_of(size_t n, int threads)
{
    size_t b = (n + threads - 1) / threads;
    return (int)std::max<size_t>(1, std::min<size_t>(b, 65535));
}

// FP64 field planes in and out of one forward pass
struct PlaneIO {
    PlaneIn in;
    double *phi, *ux, *uy, *rho;
    double u_scale, r_scale;
};

// A kernel that uses more than 64 KiB of dynamic LDS must be allowed it explicitly, once per
// device (done[] is the kernel's own record of the devices already set up).
constexpr int kMaxDevices = 64;
int allow_dynamic_lds(lbcm_net *n, const void *kernel, size_t bytes, bool (&done)[kMaxDevices])
{
    int dev = 0;
    NHIP(n, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return nfail(n, LBCM_EHIP, "device index out of range");
    if (!done[dev]) {
        NHIP(n, hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
        done[dev] = true;
    }
    return LBCM_OK;
}

template <int CI, int CO, int MO>
int launch_conv_t(lbcm_net *n, const __bf16 *X, const __bf16 *Wp, const OutArgs &o)
{
    constexpr size_t bytes = ConvLds<CI, CO>::bytes;
    static bool done[kMaxDevices] = {}, done_wide[kMaxDevices] = {};
    const bool wide = n->H >= kTileH && n->W >= kTileW;
    int rc = allow_dynamic_lds(n, wide ? reinterpret_cast<const void *>(&k_conv<CI, CO, MO, true>)
                                       : reinterpret_cast<const void *>(&k_conv<CI, CO, MO, false>),
                               bytes, wide ? done_wide : done);
    if (rc) return rc;
    if (wide)
        hipLaunchKernelGGL((k_conv<CI, CO, MO, true>), dim3(n->conv_grid), dim3(kConvThreads), bytes, n->stream, X, Wp, o, n->ntiles,
                           n->H, n->W);
    else
        hipLaunchKernelGGL((k_conv<CI, CO, MO, false>), dim3(n->conv_grid), dim3(kConvThreads), bytes, n->stream, X, Wp, o, n->ntiles,
                           n->H, n->W);
    NHIP(n, hipGetLastError());
    return LBCM_OK;
}

template <int CO, int MO, int PK = CO>
int launch_pair_t(lbcm_net *n, const __bf16 *X, const __bf16 *Wa, const float *ba, const __bf16 *Wb, const OutArgs &o)
{
    constexpr size_t bytes = PairLds::bytes;
    static bool done[kMaxDevices] = {};
    int rc = allow_dynamic_lds(n, reinterpret_cast<const void *>(&k_pair<CO, MO, PK>), bytes, done);
    if (rc) return rc;
    hipLaunchKernelGGL((k_pair<CO, MO, PK>), dim3(n->ntiles), dim3(kConvThreads), bytes, n->stream, X, Wa, ba, Wb, o, n->ntiles,
                       n->H, n->W);
    NHIP(n, hipGetLastError());
    return LBCM_OK;
}

template <int COUT>
int launch_dw_strip(lbcm_net *n, const __bf16 *X, const __bf16 *dz)
{
    constexpr size_t bytes = DwLds<COUT>::bytes;
    static bool done[kMaxDevices] = {};
    int rc = allow_dynamic_lds(n, reinterpret_cast<const void *>(&k_conv_dw_strip<COUT>), bytes, done);
    if (rc) return rc;
    hipLaunchKernelGGL(k_conv_dw_strip<COUT>, dim3(n->dw_units), dim3(kDwThreads), bytes, n->stream, X, dz, n->H, n->W, n->dw_seg,
                       n->dw_units_per_strip, n->dw_partial, n->db_partial);
    NHIP(n, hipGetLastError());
    return LBCM_OK;
}

int launch_first_pair(lbcm_net *n, const PlaneIO *io, const OutArgs &o)
{
    constexpr size_t bytes = (size_t)(PairLds::z_elems + PairLds::w_elems) * sizeof(__bf16);
    static bool done[kMaxDevices] = {};
    int rc = allow_dynamic_lds(n, reinterpret_cast<const void *>(&k_first_pair), bytes, done);
    if (rc) return rc;
    hipLaunchKernelGGL(k_first_pair, dim3(n->ntiles), dim3(kConvThreads), bytes, n->stream, io->in, n->resid, n->params + n->w_off[0],
                       n->params + n->b_off[0], n->Wf[1], o, n->ntiles, n->H, n->W);
    NHIP(n, hipGetLastError());
    return LBCM_OK;
}

int launch_conv(lbcm_net *n, const __bf16 *X, int cin, const __bf16 *Wp, int cout, int mode, const OutArgs &o)
{
    if (cin == 64 && cout == 64 && mode == 0) return launch_conv_t<64, 64, 0>(n, X, Wp, o);
    if (cin == 64 && cout == 64 && mode == 2) return launch_conv_t<64, 64, 2>(n, X, Wp, o);
    if (cin == 64 && cout == 32 && mode == 1) return launch_conv_t<64, 32, 1>(n, X, Wp, o);
    if (cin == 64 && cout == 32 && mode == 3) return launch_conv_t<64, 32, 3>(n, X, Wp, o);
    if (cin == 32 && cout == 32 && mode == 0) return launch_conv_t<32, 32, 0>(n, X, Wp, o);
    if (cin == 32 && cout == 32 && mode == 1) return launch_conv_t<32, 32, 1>(n, X, Wp, o);
    if (cin == 32 && cout == 32 && mode == 3) return launch_conv_t<32, 32, 3>(n, X, Wp, o);
    if (cin == 32 && cout == 32 && mode == 2) return launch_conv_t<32, 32, 2>(n, X, Wp, o);
    return nfail(n, LBCM_EINVAL, "unsupported channel counts");
}

int pack_all(lbcm_net *n)
{
    for (int l = 1; l < n->L; ++l) {
        hipLaunchKernelGGL(k_pack, dim3(grid_of(9 * (size_t)n->cin[l] * n->cout[l], 256)), dim3(256), 0, n->stream,
                           n->params + n->w_off[l], n->cin_r[l], n->cout_r[l], n->cin[l], n->cout[l], n->Wf[l], n->Wb[l]);
        NHIP(n, hipGetLastError());
    }
    n->packed = true;
    return LBCM_OK;
}


template <int C>
void launch_first(lbcm_net *n, const PlaneIO *io)
{
    // two resident workgroups per CU, each taking several tiles in turn
    const dim3 g(std::min(n->ntiles, 512)), b(kFirstThreads);
    const float *W0 = n->params + n->w_off[0], *b0 = n->params + n->b_off[0];
    const bool wide = n->H >= kTileH && n->W >= kTileW;
    if (io) {
        if (wide)
            hipLaunchKernelGGL((k_first<C, true, true>), g, b, 0, n->stream, nullptr, io->in, n->resid, W0, b0, n->ntiles, n->H, n->W,
                               n->act[1], nullptr);
        else
            hipLaunchKernelGGL((k_first<C, true, false>), g, b, 0, n->stream, nullptr, io->in, n->resid, W0, b0, n->ntiles, n->H,
                               n->W, n->act[1], nullptr);
    } else {
        if (wide)
            hipLaunchKernelGGL((k_first<C, false, true>), g, b, 0, n->stream, n->resid, PlaneIn{}, nullptr, W0, b0, n->ntiles, n->H,
                               n->W, n->act[1], n->mask8[1]);
        else
            hipLaunchKernelGGL((k_first<C, false, false>), g, b, 0, n->stream, n->resid, PlaneIn{}, nullptr, W0, b0, n->ntiles, n->H,
                               n->W, n->act[1], n->mask8[1]);
    }
}

// forward from the FP32 state in n->resid ([P][kStateC]) into n->out, or with io from and into
// FP64 field planes (the input state is then also left in n->resid)
int forward(lbcm_net *n, const PlaneIO *io = nullptr)
{
    if (!n->packed) {
        int rc = pack_all(n);
        if (rc) return rc;
    }
    // output arguments of a launch whose last layer is lb
    auto out_args = [&](int lb) {
        const bool last = lb == n->L - 1;
        OutArgs o{};
        o.bias = n->params + n->b_off[lb];
        o.Y = last ? nullptr : n->act[lb + 1];
        o.mask_out = (last || io) ? nullptr : n->mask8[lb + 1];  // the training forward keeps the ReLU masks
        o.resid = n->resid;
        o.Yf = n->out;
        o.alpha0 = n->alpha[0];
        o.alpha1 = n->alpha[1];
        o.alpha2 = n->alpha[2];
        o.alpha3 = n->alpha[3];
        if (io) {
            o.phi = io->phi;
            o.ux = io->ux;
            o.uy = io->uy;
            o.rho = io->rho;
            o.u_scale = io->u_scale;
            o.r_scale = io->r_scale;
        }
        return o;
    };
    // inference from planes with 64 channels runs the layers in fused pairs (the activation
    // between the two layers of a pair stays in LDS): layers 0 and 1, then 2 and 3, ..., and a
    // last single layer if one is left
    const bool pairs = io && n->C == 64;
    int l = 1;
    if (pairs && n->L > 2) {
        int rc = launch_first_pair(n, io, out_args(1));
        if (rc) return rc;
        l = 2;
    } else {
        if (n->C == 64)
            launch_first<64>(n, io);
        else
            launch_first<32>(n, io);
        NHIP(n, hipGetLastError());
    }
    while (l < n->L) {
        const bool paired = pairs && l + 1 < n->L;
        const int lb = paired ? l + 1 : l;  // the layer that writes the output
        const bool last = lb == n->L - 1;
        const OutArgs o = out_args(lb);
        int rc;
        if (paired)
            // the last layer into the planes: only its first 16 padded output channels (the 4
            // state channels and 12 zero ones) are computed, from its 32-channel weight pack
            rc = last ? launch_pair_t<16, 3, kOutC>(n, n->act[l], n->Wf[l], n->params + n->b_off[l], n->Wf[lb], o)
                      : launch_pair_t<64, 0>(n, n->act[l], n->Wf[l], n->params + n->b_off[l], n->Wf[lb], o);
        else
            rc = launch_conv(n, n->act[l], n->cin[l], n->Wf[l], n->cout[l], last ? (io ? 3 : 1) : 0, o);
        if (rc) return rc;
        l = lb + 1;
    }
    return LBCM_OK;
}

}  // namespace

extern "C" {

int lbcm_net_create(int32_t batch, int32_t height, int32_t width, int32_t channels, int32_t layers, void *stream,
                    lbcm_net **out)
{
    if (!out) return LBCM_EINVAL;
    *out = nullptr;
    const size_t P = (size_t)batch * height * width;
    if (batch < 1 || height < 1 || width < 1 || P > (1ull << 26)) {
        g_net_error = "batch, height and width must be >= 1 with batch * height * width <= 2^26";
        return LBCM_EINVAL;
    }
    if (channels != 32 && channels != 64) {
        g_net_error = "channels must be 32 or 64";
        return LBCM_EINVAL;
    }
    if (layers < 2 || layers > 32) {
        g_net_error = "layers must be in [2, 32]";
        return LBCM_EINVAL;
    }
    lbcm_net *n = new (std::nothrow) lbcm_net();
    if (!n) return LBCM_ENOMEM;
    n->batch = batch;
    n->H = height;
    n->W = width;
    n->C = channels;
    n->L = layers;
    n->P = (uint32_t)P;
    n->stream = (hipStream_t)stream;
    const size_t ntiles = (size_t)batch * ((height + kTileH - 1) / kTileH) * ((width + kTileW - 1) / kTileW);
    n->ntiles = (int)ntiles;
    // one resident workgroup per CU (LDS and two waves per SIMD); more tiles are taken in turn
    n->conv_grid = (int)std::min<size_t>(ntiles, 256);
    for (int l = 0; l < layers; ++l) {
        n->cin_r.push_back(l == 0 ? kStateC : channels);
        n->cout_r.push_back(l == layers - 1 ? kStateC : channels);
        n->cin.push_back(l == 0 ? kStateC : channels);
        n->cout.push_back(l == layers - 1 ? kOutC : channels);
        n->w_off.push_back(n->nparams);
        n->nparams += 9 * (size_t)n->cin_r[l] * n->cout_r[l];
        n->b_off.push_back(n->nparams);
        n->nparams += n->cout[l];  // bias padded to the kernel's output width (zeros past cout_r)
    }
    auto bail = [&](const std::string &m) {
        g_net_error = m;
        lbcm_net_destroy(n);
        return LBCM_ENOMEM;
    };
    auto dmalloc = [&](void **p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; };
    const size_t pb = n->nparams * sizeof(float);
    if (!dmalloc((void **)&n->params, pb) || !dmalloc((void **)&n->grads, pb) || !dmalloc((void **)&n->adam_m, pb) ||
        !dmalloc((void **)&n->adam_v, pb))
        return bail("out of device memory (parameters)");
    if (hipMemsetAsync(n->params, 0, pb, n->stream) != hipSuccess || hipMemsetAsync(n->grads, 0, pb, n->stream) != hipSuccess ||
        hipMemsetAsync(n->adam_m, 0, pb, n->stream) != hipSuccess || hipMemsetAsync(n->adam_v, 0, pb, n->stream) != hipSuccess)
        return bail("hipMemsetAsync failed");
    n->Wf.assign(layers, nullptr);
    n->Wb.assign(layers, nullptr);
    for (int l = 1; l < layers; ++l) {
        const size_t wb = 9 * (size_t)n->cin[l] * n->cout[l] * sizeof(__bf16);
        if (!dmalloc((void **)&n->Wf[l], wb) || !dmalloc((void **)&n->Wb[l], wb)) return bail("out of device memory (packs)");
    }
    n->act.assign(layers, nullptr);
    n->mask8.assign(layers, nullptr);
    for (int l = 1; l < layers; ++l)
        if (!dmalloc((void **)&n->act[l], P * channels * sizeof(__bf16)) || !dmalloc((void **)&n->mask8[l], P * (channels / 4)))
            return bail("out of device memory (activations)");
    if (!dmalloc((void **)&n->dz_a, P * 64 * sizeof(__bf16)) || !dmalloc((void **)&n->dz_b, P * 64 * sizeof(__bf16)) ||
        !dmalloc((void **)&n->dz_last, P * kStateC * sizeof(__bf16)))
        return bail("out of device memory (gradients)");
    {
        std::vector<PackEntry> tab;
        for (int l = 1; l < layers; ++l)
            tab.push_back({(int64_t)n->w_off[l], 9 * n->cin_r[l] * n->cout_r[l], n->cin_r[l], n->cout_r[l], n->cin[l], n->cout[l],
                           n->Wf[l], n->Wb[l]});
        if (!dmalloc((void **)&n->pack_table, tab.size() * sizeof(PackEntry))) return bail("out of device memory (pack table)");
        if (hipMemcpyAsync(n->pack_table, tab.data(), tab.size() * sizeof(PackEntry), hipMemcpyHostToDevice, n->stream) !=
                hipSuccess ||
            hipStreamSynchronize(n->stream) != hipSuccess)
            return bail("pack table copy failed");
    }
    if (!dmalloc((void **)&n->resid, P * kStateC * sizeof(float)) || !dmalloc((void **)&n->out, P * kStateC * sizeof(float)) ||
        !dmalloc((void **)&n->gather_idx, (size_t)batch * sizeof(int32_t)))
        return bail("out of device memory (state)");
    const size_t nchunks = (P + kDwChunk - 1) / kDwChunk;
    {
        // strip work units of the 64-input-channel weight gradient: runs of seg rows, about 256 in all
        const size_t nstrips = (width + kDwStrip - 1) / kDwStrip, rows = (size_t)batch * nstrips * height;
        n->dw_seg = (int)std::max<size_t>(4, (rows + 255) / 256);
        n->dw_units_per_strip = (height + n->dw_seg - 1) / n->dw_seg;
        n->dw_units = (int)((size_t)batch * nstrips * n->dw_units_per_strip);
    }
    // weight partial rows: of the generic and strip kernels (up to 9 x 64 x 64 each) and of the last
    // layer's (9 x 64 x kStateC each); bias partial rows of 64
    const size_t last_rows = std::min<size_t>(ntiles, kLastDwBlocks);
    const size_t wfloats = std::max<size_t>(std::max<size_t>(nchunks, (size_t)n->dw_units) * 9 * 64 * 64, last_rows * 9 * 64 * kStateC);
    if (!dmalloc((void **)&n->dw_partial, wfloats * sizeof(float))) return bail("out of device memory (dW)");
    if (!dmalloc((void **)&n->db_partial,
                 std::max<size_t>(std::max<size_t>((P + 1023) / 1024, (size_t)n->dw_units), last_rows) * 64 * sizeof(float)))
        return bail("out of device memory (db)");
    if (!dmalloc((void **)&n->first_partial, std::min<size_t>(ntiles, kFirstDwBlocks) * kFirstRows * channels * sizeof(float)))
        return bail("out of device memory (first layer)");
    n->loss_blocks = grid_of(P, 256) > 1024 ? 1024 : grid_of(P, 256);
    if (!dmalloc((void **)&n->loss_partial, n->loss_blocks * sizeof(float))) return bail("out of device memory (loss)");
    *out = n;
    return LBCM_OK;
}

size_t lbcm_net_param_count(const lbcm_net *n) { return n ? n->nparams : 0; }

int lbcm_net_set_output_scale(lbcm_net *n, const float *alpha)
{
    if (!n || !alpha) return LBCM_EINVAL;
    for (int c = 0; c < kStateC; ++c)
        if (!(alpha[c] > 0.f) || !std::isfinite(alpha[c])) return nfail(n, LBCM_EINVAL, "output scales must be finite and > 0");
    for (int c = 0; c < kStateC; ++c) n->alpha[c] = alpha[c];
    return LBCM_OK;
}

int lbcm_net_set_params(lbcm_net *n, const float *host, size_t count)
{
    if (!n || !host) return LBCM_EINVAL;
    if (count != n->nparams) return nfail(n, LBCM_EINVAL, "wrong parameter count");
    NHIP(n, hipMemcpyAsync(n->params, host, count * sizeof(float), hipMemcpyHostToDevice, n->stream));
    NHIP(n, hipMemsetAsync(n->adam_m, 0, count * sizeof(float), n->stream));
    NHIP(n, hipMemsetAsync(n->adam_v, 0, count * sizeof(float), n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    n->packed = false;
    return LBCM_OK;
}

int lbcm_net_get_params(lbcm_net *n, float *host, size_t count)
{
    if (!n || !host) return LBCM_EINVAL;
    if (count != n->nparams) return nfail(n, LBCM_EINVAL, "wrong parameter count");
    NHIP(n, hipMemcpyAsync(host, n->params, count * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    return LBCM_OK;
}

int lbcm_net_get_grads(lbcm_net *n, float *host, size_t count)
{
    if (!n || !host) return LBCM_EINVAL;
    if (count != n->nparams) return nfail(n, LBCM_EINVAL, "wrong parameter count");
    NHIP(n, hipMemcpyAsync(host, n->grads, count * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    return LBCM_OK;
}

int lbcm_net_forward(lbcm_net *n, const float *in, float *out)
{
    if (!n || !in) return LBCM_EINVAL;
    NHIP(n, hipMemcpyAsync(n->resid, in, (size_t)n->P * kStateC * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    int rc = forward(n);
    if (rc) return rc;
    if (out) NHIP(n, hipMemcpyAsync(out, n->out, (size_t)n->P * kStateC * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    return LBCM_OK;
}

int lbcm_net_forward_planes(lbcm_net *n, const double *phi, const double *ux, const double *uy, const double *rho, double u_scale,
                            double rho_scale, double *phi_out, double *ux_out, double *uy_out, double *rho_out)
{
    if (!n || !phi || !ux || !uy || !rho || !phi_out || !ux_out || !uy_out || !rho_out || !(u_scale > 0) || !(rho_scale > 0))
        return LBCM_EINVAL;
    const PlaneIO io{{phi, ux, uy, rho, (float)(1.0 / u_scale), (float)(1.0 / rho_scale)}, phi_out, ux_out, uy_out, rho_out,
                     u_scale, rho_scale};
    return forward(n, &io);
}

int lbcm_net_state_from_planes(lbcm_net *n, const double *phi, const double *ux, const double *uy, const double *rho,
                               double u_scale, double rho_scale, float *state)
{
    if (!n || !phi || !ux || !uy || !rho || !state || !(u_scale > 0) || !(rho_scale > 0)) return LBCM_EINVAL;
    hipLaunchKernelGGL(k_from_planes, dim3(grid_of(n->P, 256)), dim3(256), 0, n->stream, phi, ux, uy, rho, (float)(1.0 / u_scale),
                       (float)(1.0 / rho_scale), n->P, state);
    NHIP(n, hipGetLastError());
    return LBCM_OK;
}

int lbcm_net_gather_states(lbcm_net *n, const double *frames, int64_t nframes, const int32_t *frame_index, int32_t symmetry,
                           double u_scale, double rho_scale, float *state)
{
    if (!n || !frames || !frame_index || !state || !(u_scale > 0) || !(rho_scale > 0)) return LBCM_EINVAL;
    if (symmetry < 0 || symmetry > 7) return nfail(n, LBCM_EINVAL, "symmetry must be in [0, 7]");
    if ((symmetry & 4) && n->H != n->W) return nfail(n, LBCM_EINVAL, "a transposing symmetry needs a square box");
    for (int b = 0; b < n->batch; ++b)
        if (frame_index[b] < 0 || frame_index[b] >= nframes) return nfail(n, LBCM_EINVAL, "frame index out of range");
    NHIP(n, hipMemcpyAsync(n->gather_idx, frame_index, (size_t)n->batch * sizeof(int32_t), hipMemcpyHostToDevice, n->stream));
    const int tiles = ((n->H + kGatherTile - 1) / kGatherTile) * ((n->W + kGatherTile - 1) / kGatherTile);
    hipLaunchKernelGGL(k_gather_states, dim3(n->batch * tiles), dim3(256), 0, n->stream, frames, nframes, n->gather_idx, symmetry,
                       n->H, n->W, (float)(1.0 / u_scale), (float)(1.0 / rho_scale), state);
    NHIP(n, hipGetLastError());
    return LBCM_OK;
}

int lbcm_net_backward(lbcm_net *n, const float *target, float *loss)
{
    if (!n || !target) return LBCM_EINVAL;
    const uint32_t P = n->P;
    const int L = n->L;
    hipLaunchKernelGGL(k_loss, dim3(n->loss_blocks), dim3(256), 0, n->stream, n->out, target, P, 1.f / n->alpha[0],
                       1.f / n->alpha[1], 1.f / n->alpha[2], 1.f / n->alpha[3], n->dz_last, n->loss_partial);
    NHIP(n, hipGetLastError());
    __bf16 *dz = n->dz_last, *dn = n->dz_a;
    const int nchunks = (int)((P + kDwChunk - 1) / kDwChunk);
    const int dbb = (int)((P + 1023) / 1024);
    for (int l = L - 1; l >= 1; --l) {
        // weight and bias gradients of layer l from its input act[l] and dz (gradient of its output)
        // (partial rows of the padded shape wcin x wcout, and bias partial rows)
        int parts = nchunks, db_rows = 0, wcout = n->cout[l];
        if (dz == n->dz_last) {
            // the last layer: only the state channels of dz
            parts = db_rows = std::min(n->ntiles, kLastDwBlocks);
            wcout = kStateC;
            if (n->cin[l] == 64)
                hipLaunchKernelGGL(k_last_dw<64>, dim3(parts), dim3(kThreads), 0, n->stream, n->act[l], dz, n->H, n->W, n->ntiles,
                                   n->dw_partial, n->db_partial);
            else
                hipLaunchKernelGGL(k_last_dw<32>, dim3(parts), dim3(kThreads), 0, n->stream, n->act[l], dz, n->H, n->W, n->ntiles,
                                   n->dw_partial, n->db_partial);
        } else if (n->cin[l] == 64 && n->cout[l] == 64) {
            parts = db_rows = n->dw_units;  // the strip kernel leaves one bias partial per work unit
            const int rc = launch_dw_strip<64>(n, n->act[l], dz);
            if (rc) return rc;
        } else {
            hipLaunchKernelGGL(k_conv_dw, dim3(nchunks, 9), dim3(kThreads), 0, n->stream, n->act[l], n->cin[l], dz, n->cout[l], P,
                               n->H, n->W, n->dw_partial);
            NHIP(n, hipGetLastError());
            hipLaunchKernelGGL(k_db_partial, dim3(dbb), dim3(256), 0, n->stream, dz, n->cout[l], P, n->db_partial);
            db_rows = dbb;
        }
        NHIP(n, hipGetLastError());
        const int wblocks = (9 * n->cin_r[l] * n->cout_r[l] + 63) / 64, bblocks = (n->cout[l] + 63) / 64;
        hipLaunchKernelGGL(k_grad_reduce, dim3(wblocks + bblocks), dim3(kSumWaves * 64), 0, n->stream, n->dw_partial, parts,
                           n->cin[l], wcout, n->cin_r[l], n->cout_r[l], n->grads + n->w_off[l], n->db_partial, db_rows, 64,
                           n->cout[l], n->grads + n->b_off[l]);
        NHIP(n, hipGetLastError());
        // gradient of the layer input times the ReLU derivative of that input (act[l] > 0); the last
        // layer's contracts over (tap, state channel) only
        if (dz == n->dz_last) {
            const dim3 g(std::min(n->ntiles, kLastDgradBlocks)), b(kConvThreads);
            if (n->cin[l] == 64)
                hipLaunchKernelGGL(k_last_dgrad<64>, g, b, 0, n->stream, dz, n->Wb[l], n->mask8[l], dn, n->ntiles, n->H, n->W);
            else
                hipLaunchKernelGGL(k_last_dgrad<32>, g, b, 0, n->stream, dz, n->Wb[l], n->mask8[l], dn, n->ntiles, n->H, n->W);
            NHIP(n, hipGetLastError());
        } else {
            OutArgs o{};
            o.mask = n->mask8[l];
            o.Y = dn;
            int rc = launch_conv(n, dz, n->cout[l], n->Wb[l], n->cin[l], 2, o);
            if (rc) return rc;
        }
        __bf16 *spare = dz == n->dz_last ? n->dz_b : dz;  // the next layer's input gradient goes to a 64-channel buffer
        dz = dn;
        dn = spare;
    }
    // layer 0 gradients (its 36 x C weights and C biases are contiguous in the vector)
    const int fblocks = std::min(n->ntiles, kFirstDwBlocks);
    if (n->C == 64)
        hipLaunchKernelGGL(k_first_dw<64>, dim3(fblocks), dim3(kThreads), 0, n->stream, n->resid, dz, n->H, n->W, n->ntiles,
                           n->first_partial);
    else
        hipLaunchKernelGGL(k_first_dw<32>, dim3(fblocks), dim3(kThreads), 0, n->stream, n->resid, dz, n->H, n->W, n->ntiles,
                           n->first_partial);
    NHIP(n, hipGetLastError());
    hipLaunchKernelGGL(k_grad_reduce, dim3((kFirstRows * n->C + 63) / 64), dim3(kSumWaves * 64), 0, n->stream, nullptr, 0, 0, 0, 0,
                       0, nullptr, n->first_partial, fblocks, kFirstRows * n->C, kFirstRows * n->C, n->grads + n->w_off[0]);
    NHIP(n, hipGetLastError());
    if (loss) {
        std::vector<float> part(n->loss_blocks);
        NHIP(n, hipMemcpyAsync(part.data(), n->loss_partial, part.size() * sizeof(float), hipMemcpyDeviceToHost, n->stream));
        NHIP(n, hipStreamSynchronize(n->stream));
        double s = 0;
        for (float v : part) s += v;
        *loss = (float)(s / ((double)kStateC * P));
    }
    return LBCM_OK;
}

int lbcm_net_adam(lbcm_net *n, float lr, float beta1, float beta2, float eps, int64_t t)
{
    if (!n || t < 1) return LBCM_EINVAL;
    const float c1 = 1.f - std::pow(beta1, (float)t), c2 = 1.f - std::pow(beta2, (float)t);
    // packs already made: update them in the same pass; otherwise the next forward makes them
    const int ntab = n->packed ? n->L - 1 : 0;
    hipLaunchKernelGGL(k_adam, dim3(grid_of(n->nparams, 256)), dim3(256), 0, n->stream, n->params, n->grads, n->adam_m, n->adam_v,
                       n->nparams, lr, beta1, beta2, eps, c1, c2, n->pack_table, ntab);
    NHIP(n, hipGetLastError());
    return LBCM_OK;
}

int lbcm_net_destroy(lbcm_net *n)
{
    if (!n) return LBCM_OK;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    else (void)hipDeviceSynchronize();
    auto f = [](void *p) { if (p) (void)hipFree(p); };
    f(n->params);
    f(n->grads);
    f(n->adam_m);
    f(n->adam_v);
    for (auto p : n->Wf) f(p);
    for (auto p : n->Wb) f(p);
    for (auto p : n->act) f(p);
    for (auto p : n->mask8) f(p);
    f(n->dz_a);
    f(n->dz_b);
    f(n->dz_last);
    f(n->pack_table);
    f(n->resid);
    f(n->out);
    f(n->gather_idx);
    f(n->dw_partial);
    f(n->db_partial);
    f(n->first_partial);
    f(n->loss_partial);
    delete n;
    return LBCM_OK;
}

const char *lbcm_net_last_error(const lbcm_net *n) { return n ? n->err.c_str() : g_net_error.c_str(); }

}  // extern "C"

// ==========================================================================================
// hybrid driver: surrogate jumps checked against the lattice Boltzmann step

struct lbcm_hybrid {
    lbcm_handle *lat = nullptr;      // the caller's lattice: holds the state between windows
    lbcm_handle *scratch = nullptr;  // private lattice of the same size for the checks
    lbcm_net *net = nullptr;
    int K = 0, J = 0;
    double u_scale = 1, rho_scale = 1, threshold = 0, vthreshold = 0;
    uint32_t P = 0;
    double *start = nullptr, *a = nullptr, *b = nullptr;  // (phi, v_x, v_y, rho) planes
    double *lb = nullptr;                                 // the check's lattice Boltzmann fields (same planes)
    double *err_partial = nullptr;
    double *err_host = nullptr;       // pinned copy of the partial sums
    hipEvent_t err_ready = nullptr;   // recorded after that copy
    int64_t cooldown = 0;  // plain windows still to run after failed checks
    int streak = 0;        // consecutive failed checks
    int audit_every = 0;   // every audit_every-th window is an audit (0: none)
    int64_t windows = 0;   // windows run so far (plain, checked and audited)
    // Within one lbcm_hybrid_advance call, after an accepted check: the next window starts from
    // the check's lattice fields (lb, equal to those of the caller's lattice after the copy), and
    // its first `spec_done` jumps were launched before the decision, the last into spec_cur.
    bool start_ready = false;
    int spec_done = 0;
    double *spec_cur = nullptr;
    lbcm_hybrid_stats st{};
    std::string err;
};

namespace {

std::string g_hybrid_error;

int hfail(lbcm_hybrid *h, int code, const std::string &m)
{
    h->err = m;
    return code;
}

#define HCALL(h, call, what, errfn, obj)                                                      \
    do {                                                                                      \
        int rc_ = (call);                                                                     \
        if (rc_ != LBCM_OK) return hfail(h, rc_, std::string(what) + ": " + errfn(obj));     \
    } while (0)
#define HLAT(h, call, what) HCALL(h, call, what, lbcm_last_error, h->lat)
#define HSCR(h, call, what) HCALL(h, call, what, lbcm_last_error, h->scratch)
#define HNET(h, call, what) HCALL(h, call, what, lbcm_net_last_error, h->net)

double *plane(double *base, uint32_t P, int k) { return base + (size_t)k * P; }

// the four check sums of k_err_partial, read back (synchronises)
// the check's FP64 partial sums: k_err_partial, then an asynchronous copy into pinned host memory
// and an event; wait_sums waits for that event only (work queued after it keeps the GPU busy)
int launch_sums(lbcm_hybrid *h, const double *x, const double *ref)
{
    hipStream_t s = h->net->stream;
    hipLaunchKernelGGL(k_err_partial, dim3(kErrBlocks), dim3(256), 0, s, x, ref, h->P, h->err_partial);
    if (hipGetLastError() != hipSuccess) return hfail(h, LBCM_EHIP, "k_err_partial launch failed");
    if (hipMemcpyAsync(h->err_host, h->err_partial, kErrSums * kErrBlocks * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipEventRecord(h->err_ready, s) != hipSuccess)
        return hfail(h, LBCM_EHIP, "queueing the error sums failed");
    return LBCM_OK;
}

int wait_sums(lbcm_hybrid *h, double (&sum)[kErrSums])
{
    if (hipEventSynchronize(h->err_ready) != hipSuccess) return hfail(h, LBCM_EHIP, "reading the error sums failed");
    for (int k = 0; k < kErrSums; ++k) sum[k] = 0;
    for (int i = 0; i < kErrBlocks; ++i)
        for (int k = 0; k < kErrSums; ++k) sum[k] += h->err_host[i * kErrSums + k];
    return LBCM_OK;
}

// relative L2 difference ||x - ref|| / ||ref||; a non-finite state on either side counts as an
// infinite error (rejected)
double rel_l2(double d2, double r2)
{
    if (!std::isfinite(d2) || !std::isfinite(r2)) return INFINITY;
    return r2 > 0 ? std::sqrt(d2 / r2) : (d2 > 0 ? INFINITY : 0.0);
}

// jumps of the next window launched before a check's decision (they hide the wait for it)
constexpr int kSpecJumps = 2;

// one window of J * K lattice steps; `more`: another window follows in this advance call
int hybrid_window(lbcm_hybrid *h, bool more)
{
    const uint32_t P = h->P;
    const int64_t span = (int64_t)h->J * h->K;
    const int64_t index = h->windows++;
    if (h->cooldown > 0) {  // plain lattice Boltzmann window after failed checks
        h->start_ready = false;
        h->spec_done = 0;
        HLAT(h, lbcm_step(h->lat, span), "lbcm_step");
        h->st.lb_steps_run += span;
        h->st.steps += span;
        h->cooldown -= 1;
        return LBCM_OK;
    }
    const bool audit = h->audit_every > 0 && (index + 1) % h->audit_every == 0;
    if (audit) more = false;  // no speculative jumps after an audit: the next window reads the lattice
    auto pl = [&](double *base, int k) { return plane(base, P, k); };
    auto jump = [&](double *in, double *outp) {
        return lbcm_net_forward_planes(h->net, pl(in, 0), pl(in, 1), pl(in, 2), pl(in, 3), h->u_scale, h->rho_scale, pl(outp, 0),
                                       pl(outp, 1), pl(outp, 2), pl(outp, 3));
    };
    double *cur, *x = h->a, *y = h->b;
    int done = 0;
    if (h->start_ready) {
        cur = h->lb;
        if (h->spec_done > 0) {
            cur = h->spec_cur;
            done = h->spec_done;
            x = cur;
            y = cur == h->a ? h->b : h->a;
        }
    } else {
        HLAT(h, lbcm_fields_device(h->lat, pl(h->start, 0), pl(h->start, 3), pl(h->start, 1), pl(h->start, 2), nullptr),
             "lbcm_fields_device");
        cur = h->start;
    }
    h->start_ready = false;
    h->spec_done = 0;
    for (int j = done; j < h->J - 1; ++j) {  // J - 1 surrogate jumps
        HNET(h, jump(cur, y), "lbcm_net_forward_planes");
        cur = y;
        std::swap(x, y);
    }
    // the last jump of the window both ways: the surrogate into y, K lattice steps on the scratch
    // lattice from equilibrium populations of the same state
    HNET(h, jump(cur, y), "lbcm_net_forward_planes");
    if (audit) {
        // audit: the caller's lattice, which still holds the window's starting populations, runs
        // the whole window with the lattice Boltzmann step; the network's state after its J jumps
        // is compared with that result (the error accumulated over the window).  The lattice keeps
        // the exact result whatever the outcome; a failure backs off like a failed check.
        HLAT(h, lbcm_step(h->lat, span), "lbcm_step");
        HLAT(h, lbcm_fields_device(h->lat, pl(h->lb, 0), pl(h->lb, 3), pl(h->lb, 1), pl(h->lb, 2), nullptr),
             "lbcm_fields_device");
        int rc = launch_sums(h, y, h->lb);
        if (rc) return rc;
        double sum[kErrSums];
        rc = wait_sums(h, sum);
        if (rc) return rc;
        const double e = rel_l2(sum[0], sum[1]), ev = rel_l2(sum[2], sum[3]);
        h->st.audits += 1;
        h->st.max_audited_error = std::max(h->st.max_audited_error, e);
        h->st.max_audited_velocity_error = std::max(h->st.max_audited_velocity_error, ev);
        h->st.lb_steps_run += span;
        h->st.steps += span;
        if (e <= h->threshold && (h->vthreshold <= 0 || ev <= h->vthreshold)) {
            h->streak = 0;
        } else {
            h->st.failed_audits += 1;
            h->streak = std::min(h->streak + 1, 5);
            h->cooldown = (int64_t)1 << (h->streak - 1);
        }
        return LBCM_OK;
    }
    HSCR(h, lbcm_init_device(h->scratch, pl(cur, 0), pl(cur, 3), pl(cur, 1), pl(cur, 2)), "lbcm_init_device");
    HSCR(h, lbcm_step(h->scratch, h->K), "lbcm_step");
    HSCR(h, lbcm_fields_device(h->scratch, pl(h->lb, 0), pl(h->lb, 3), pl(h->lb, 1), pl(h->lb, 2), nullptr),
         "lbcm_fields_device");
    int rc = launch_sums(h, y, h->lb);
    if (rc) return rc;
    // the next window's first jumps, from the check's lattice state, while the sums travel; kept
    // only if the check accepts (x and y are free once the sums are queued)
    const int spec = more ? std::min(kSpecJumps, h->J - 1) : 0;
    double *sc = h->lb;
    for (int j = 0; j < spec; ++j) {
        double *o = (j & 1) ? h->b : h->a;
        HNET(h, jump(sc, o), "lbcm_net_forward_planes");
        sc = o;
    }
    double sum[kErrSums];
    rc = wait_sums(h, sum);
    if (rc) return rc;
    const double e = rel_l2(sum[0], sum[1]), ev = rel_l2(sum[2], sum[3]);
    h->st.checks += 1;
    h->st.last_error = e;
    h->st.max_error = std::max(h->st.max_error, e);
    h->st.last_velocity_error = ev;
    const bool ok = e <= h->threshold && (h->vthreshold <= 0 || ev <= h->vthreshold);
    if (!ok) {
        // rejected: the caller's lattice still holds the window's starting populations; run the
        // window with the plain step from there, then 2^(k-1) more plain windows (at most 16)
        // after k failures in a row; the speculative jumps are dropped
        h->st.failed_checks += 1;
        HLAT(h, lbcm_step(h->lat, span), "lbcm_step");
        h->st.lb_steps_run += h->K + span;
        h->streak = std::min(h->streak + 1, 5);
        h->cooldown = (int64_t)1 << (h->streak - 1);
    } else {
        HLAT(h, lbcm_copy_state(h->lat, h->scratch, lbcm_step_count(h->lat) + span), "lbcm_copy_state");
        h->st.jumps += h->J - 1;
        h->st.lb_steps_run += h->K;
        h->st.max_accepted_error = std::max(h->st.max_accepted_error, e);
        h->st.max_accepted_velocity_error = std::max(h->st.max_accepted_velocity_error, ev);
        h->streak = 0;
        h->start_ready = more;
        h->spec_done = spec;
        h->spec_cur = sc;
    }
    h->st.steps += span;
    return LBCM_OK;
}

}  // namespace

extern "C" {

int lbcm_hybrid_create(lbcm_handle *lattice, lbcm_net *net, int32_t steps_per_jump, int32_t jumps_per_check, double u_scale,
                       double rho_scale, double threshold, double velocity_threshold, lbcm_hybrid **out)
{
    if (!out) return LBCM_EINVAL;
    *out = nullptr;
    lbcm_params p;
    if (!lattice || !net || lbcm_info(lattice, &p) != LBCM_OK) {
        g_hybrid_error = "lattice and network are required";
        return LBCM_EINVAL;
    }
    if (steps_per_jump < 1 || jumps_per_check < 1 || !(u_scale > 0) || !(rho_scale > 0) || !(threshold >= 0) ||
        std::isnan(velocity_threshold)) {
        g_hybrid_error = "steps_per_jump and jumps_per_check must be >= 1, u_scale and rho_scale > 0, threshold >= 0";
        return LBCM_EINVAL;
    }
    if (p.bc_y != LBCM_BC_PERIODIC || net->batch != 1 || net->H != p.ny || net->W != p.nx) {
        g_hybrid_error = "the network must be built for one periodic box of the lattice's size";
        return LBCM_EINVAL;
    }
    if ((hipStream_t)p.stream != net->stream) {
        g_hybrid_error = "the lattice and the network must use the same stream";
        return LBCM_EINVAL;
    }
    lbcm_hybrid *h = new (std::nothrow) lbcm_hybrid();
    if (!h) return LBCM_ENOMEM;
    h->lat = lattice;
    h->net = net;
    h->K = steps_per_jump;
    h->J = jumps_per_check;
    h->u_scale = u_scale;
    h->rho_scale = rho_scale;
    h->threshold = threshold;
    h->vthreshold = velocity_threshold;
    h->P = net->P;
    lbcm_params ps = p;  // the scratch lattice: same size, physics and stream; its own memory
    ps.workspace = nullptr;
    ps.workspace_bytes = 0;
    ps.check_every = 0;
    if (lbcm_create(&ps, &h->scratch) != LBCM_OK) {
        g_hybrid_error = std::string("scratch lattice: ") + lbcm_last_error(nullptr);
        delete h;
        return LBCM_ENOMEM;
    }
    const size_t pb = (size_t)h->P * sizeof(double);
    if (hipMalloc((void **)&h->start, 4 * pb) != hipSuccess || hipMalloc((void **)&h->a, 4 * pb) != hipSuccess ||
        hipMalloc((void **)&h->b, 4 * pb) != hipSuccess || hipMalloc((void **)&h->lb, 4 * pb) != hipSuccess ||
        hipMalloc((void **)&h->err_partial, kErrSums * kErrBlocks * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&h->err_host, kErrSums * kErrBlocks * sizeof(double)) != hipSuccess ||
        hipEventCreateWithFlags(&h->err_ready, hipEventDisableTiming) != hipSuccess) {
        g_hybrid_error = "out of device memory";
        lbcm_hybrid_destroy(h);
        return LBCM_ENOMEM;
    }
    *out = h;
    return LBCM_OK;
}

int lbcm_hybrid_advance(lbcm_hybrid *h, int64_t windows)
{
    if (!h || windows < 0) return LBCM_EINVAL;
    h->start_ready = false;  // the caller may have changed the lattice since the last call
    h->spec_done = 0;
    for (int64_t w = 0; w < windows; ++w) {
        int rc = hybrid_window(h, w + 1 < windows);
        if (rc) return rc;
    }
    return LBCM_OK;
}

int lbcm_hybrid_set_audit(lbcm_hybrid *h, int32_t every)
{
    if (!h) return LBCM_EINVAL;
    if (every < 0) return hfail(h, LBCM_EINVAL, "audit period must be >= 0");
    h->audit_every = every;
    return LBCM_OK;
}

int lbcm_hybrid_get_stats(const lbcm_hybrid *h, lbcm_hybrid_stats *out)
{
    if (!h || !out) return LBCM_EINVAL;
    *out = h->st;
    return LBCM_OK;
}

int lbcm_hybrid_destroy(lbcm_hybrid *h)
{
    if (!h) return LBCM_OK;
    if (h->net && h->net->stream) (void)hipStreamSynchronize(h->net->stream);
    else (void)hipDeviceSynchronize();
    for (void *q : {(void *)h->start, (void *)h->a, (void *)h->b, (void *)h->lb, (void *)h->err_partial})
        if (q) (void)hipFree(q);
    if (h->err_host) (void)hipHostFree(h->err_host);
    if (h->err_ready) (void)hipEventDestroy(h->err_ready);
    if (h->scratch) lbcm_destroy(h->scratch);
    delete h;
    return LBCM_OK;
}

const char *lbcm_hybrid_last_error(const lbcm_hybrid *h) { return h ? h->err.c_str() : g_hybrid_error.c_str(); }

}  // extern "C"
