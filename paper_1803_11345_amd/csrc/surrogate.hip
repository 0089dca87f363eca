// Learned surrogate of the lattice Boltzmann step: a stack of 3x3 convolutions (circular
// padding, periodic boxes) that maps the macroscopic state (phi, v_x, v_y) to the state K steps
// later, trained on trajectories of the LB solver.  Forward and backward passes are implicit GEMMs
// on the MFMA units of gfx950 (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation).
//
// Tensors.  Activations are NHWC in BF16 with the channel count padded to a multiple of 32 (the K
// step of one MFMA); the three state channels are padded to 32 on input and 16 on output.  Master
// weights are FP32, W[l][t][ci][co] with t = 3 (dy + 1) + (dx + 1) the tap at (dy, dx); each
// iteration packs them to BF16 twice: Wf[t][co][ci] for the forward pass (the MFMA B operand wants
// 8 consecutive input channels per lane) and Wb[t][ci][co] = W[8 - t][ci][co] for the input
// gradient: tap t of the mirrored pack sits at d_t = -d_{8-t}, so running the forward kernel on dZ
// with it gives sum_t dZ[p - d_t] W[t].
//
// One convolution layer computes Y[p][co] = b[co] + sum_t sum_ci X[p + d_t][ci] W[t][ci][co] for
// every pixel p of every sample; its input gradient dX[p][ci] = sum_t sum_co dZ[p - d_t][co]
// W[t][ci][co] is the same kernel on the mirrored pack; its weight gradient
// dW[t][ci][co] = sum_p X[p + d_t][ci] dZ[p][co] is a GEMM whose K dimension runs over pixels.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbcm_net.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned int)))) unsigned int u32x4;

constexpr int kStateC = 3;      // phi, v_x, v_y
constexpr int kInC = 32;        // padded input channels of the first layer
constexpr int kOutC = 32;       // padded output channels of the last layer (a K step of the input gradient)
constexpr int kConvThreads = 256;
constexpr int kPixPerWave = 32;  // two 16-row MFMA tiles
constexpr int kDwPix = 64;       // pixels staged per iteration of the weight-gradient kernel
constexpr int kDwChunk = 4096;   // pixels reduced by one weight-gradient workgroup

__device__ __forceinline__ int tap_dy(int t) { return t / 3 - 1; }
__device__ __forceinline__ int tap_dx(int t) { return t % 3 - 1; }

// pixel index of p shifted by (dy, dx) inside its sample (circular)
__device__ __forceinline__ uint32_t shift_pix(uint32_t p, int dy, int dx, int H, int W)
{
    const uint32_t hw = (uint32_t)H * W;
    const uint32_t n = p / hw, r = p - n * hw;
    int y = (int)(r / W) + dy, x = (int)(r % W) + dx;
    y = y < 0 ? y + H : (y >= H ? y - H : y);
    x = x < 0 ? x + W : (x >= W ? x - W : x);
    return n * hw + (uint32_t)y * W + (uint32_t)x;
}

__device__ __forceinline__ bf16x8 ld8(const __bf16 *p) { return __builtin_bit_cast(bf16x8, *(const u32x4 *)p); }

// ------------------------------------------------------------------------------------------
// convolution (forward, or input gradient with the mirrored pack).
// Each wave computes 32 pixels x Cout output channels (Cout <= 64: up to 4 N-tiles of 16).
// mode 0: out = bf16(act(bias + conv)); mode 1: out_f32[p][c] = resid[p][c] + bias + conv for
// c < kStateC (the last layer).  relu: 1 applies max(0, .).  mask (may be NULL): the result is
// multiplied by [mask > 0] (the ReLU derivative of the layer input, for the input gradient).

template <int NT>
__global__ __launch_bounds__(kConvThreads) void k_conv(const __bf16 *__restrict__ X, int cin, const __bf16 *__restrict__ Wp,
                                                       const float *__restrict__ bias, int cout, int sign, int relu,
                                                       const __bf16 *__restrict__ mask, int mode, __bf16 *__restrict__ Y,
                                                       const float *__restrict__ resid, float *__restrict__ Yf,
                                                       uint32_t P, int H, int W)
{
    const int lane = threadIdx.x & 63;
    const uint32_t wave = blockIdx.x * (kConvThreads / 64) + (threadIdx.x >> 6);
    const uint32_t m0 = wave * kPixPerWave;
    if (m0 >= P) return;  // P is a multiple of 32 (checked on the host)
    const int r = lane & 15, q = lane >> 4;  // row / column inside a tile, K group
    f32x4 acc[2][NT];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    for (int t = 0; t < 9; ++t) {
        const int dy = sign * tap_dy(t), dx = sign * tap_dx(t);
        const uint32_t pa = shift_pix(m0 + r, dy, dx, H, W), pb = shift_pix(m0 + 16 + r, dy, dx, H, W);
        const __bf16 *Wt = Wp + (size_t)t * cout * cin;
        for (int kc = 0; kc < cin; kc += 32) {
            const int k = kc + 8 * q;
            const bf16x8 a0 = ld8(X + (size_t)pa * cin + k);
            const bf16x8 a1 = ld8(X + (size_t)pb * cin + k);
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const bf16x8 b = ld8(Wt + (size_t)(16 * j + r) * cin + k);
                acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b, acc[0][j], 0, 0, 0);
                acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b, acc[1][j], 0, 0, 0);
            }
        }
    }
    // D layout: lane holds rows 4q..4q+3 of column r of each 16x16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int c = 16 * j + r;
            const float bc = bias ? bias[c] : 0.f;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t p = m0 + 16 * i + 4 * q + e;
                float v = acc[i][j][e] + bc;
                if (mode == 1) {
                    if (c < kStateC) Yf[(size_t)p * kStateC + c] = resid[(size_t)p * kStateC + c] + v;
                } else {
                    if (mask && !((float)mask[(size_t)p * cout + c] > 0.f)) v = 0.f;
                    if (relu) v = fmaxf(v, 0.f);
                    Y[(size_t)p * cout + c] = (__bf16)v;
                }
            }
        }
}

// ------------------------------------------------------------------------------------------
// weight gradient: partial[chunk][t][ci][co] = sum over the chunk's pixels p of
// X[p + d_t][ci] dZ[p][co].  A workgroup (4 waves) owns one tap and one chunk of pixels; it stages
// 64 pixels of X (shifted) and dZ in LDS with 16-byte loads, then each wave accumulates its share
// of the (ci, co) 16x16 tiles with MFMAs whose K dimension is the pixels.

__global__ __launch_bounds__(kConvThreads) void k_conv_dw(const __bf16 *__restrict__ X, int cin, const __bf16 *__restrict__ dZ,
                                                          int cout, uint32_t P, int H, int W, float *__restrict__ partial)
{
    __shared__ __align__(16) __bf16 sx[kDwPix * 64];
    __shared__ __align__(16) __bf16 sz[kDwPix * 64];
    const int t = blockIdx.y;
    const uint32_t chunk = blockIdx.x;
    const uint32_t p_begin = chunk * kDwChunk, p_end = min(P, p_begin + kDwChunk);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int mt = cin / 16, nt = cout / 16, ntiles = mt * nt;  // <= 16 tiles, 4 per wave
    f32x4 acc[4];
    for (int i = 0; i < 4; ++i) acc[i] = f32x4{0, 0, 0, 0};
    const int dy = tap_dy(t), dx = tap_dx(t);
    for (uint32_t p0 = p_begin; p0 < p_end; p0 += kDwPix) {
        // stage: 64 pixels x cin of X shifted, 64 x cout of dZ; 8 bf16 per thread per load
        for (int v = threadIdx.x; v < kDwPix * cin / 8; v += kConvThreads) {
            const int px = v / (cin / 8), ch = (v % (cin / 8)) * 8;
            const uint32_t p = p0 + px;
            u32x4 val = {0, 0, 0, 0};
            if (p < p_end) val = *(const u32x4 *)(X + (size_t)shift_pix(p, dy, dx, H, W) * cin + ch);
            *(u32x4 *)(sx + px * cin + ch) = val;
        }
        for (int v = threadIdx.x; v < kDwPix * cout / 8; v += kConvThreads) {
            const int px = v / (cout / 8), ch = (v % (cout / 8)) * 8;
            const uint32_t p = p0 + px;
            u32x4 val = {0, 0, 0, 0};
            if (p < p_end) val = *(const u32x4 *)(dZ + (size_t)p * cout + ch);
            *(u32x4 *)(sz + px * cout + ch) = val;
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
                    a[e] = sx[px * cin + 16 * mi + r];  // A[ci][pixel]
                    b[e] = sz[px * cout + 16 * ni + r]; // B[pixel][co]
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

// sum of the per-chunk partials in chunk order (deterministic), into the real-size gradient
// dW[t][ci][co] (ci < cin_r, co < cout_r) of the padded partials
__global__ void k_dw_reduce(const float *__restrict__ partial, int nchunks, int cin, int cout, int cin_r, int cout_r,
                            float *__restrict__ dW)
{
    const int n = 9 * cin_r * cout_r;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int t = i / (cin_r * cout_r), rem = i % (cin_r * cout_r), ci = rem / cout_r, co = rem % cout_r;
        float s = 0;
        for (int c = 0; c < nchunks; ++c) s += partial[(((size_t)c * 9 + t) * cin + ci) * cout + co];
        dW[i] = s;
    }
}

// bias gradient db[co] = sum_p dZ[p][co]: per-block partial sums, then a fixed-order sum
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

__global__ void k_db_reduce(const float *__restrict__ partial, int nblocks, int cout_r, float *__restrict__ db)
{
    const int c = threadIdx.x;
    if (c >= cout_r) return;
    float s = 0;
    for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * 64 + c];
    db[c] = s;
}

// ------------------------------------------------------------------------------------------
// loss: mean over pixels and the three state channels of (pred - target)^2; the gradient of the
// last layer's output is 2 (pred - target) / (3 P), stored padded to kOutC channels.
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ pred, const float *__restrict__ target, uint32_t P,
                                              __bf16 *__restrict__ dZ, float *__restrict__ partial)
{
    __shared__ float red[256];
    const float scale = 2.0f / (3.0f * (float)P);
    float s = 0;
    for (uint32_t p = blockIdx.x * 256u + threadIdx.x; p < P; p += gridDim.x * 256u) {
        for (int c = 0; c < kOutC; ++c) {
            float g = 0;
            if (c < kStateC) {
                const float d = pred[(size_t)p * kStateC + c] - target[(size_t)p * kStateC + c];
                s += d * d;
                g = scale * d;
            }
            dZ[(size_t)p * kOutC + c] = (__bf16)g;
        }
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

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       size_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1 - b1) * gi;
        const float vi = b2 * v[i] + (1 - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// FP32 state [P][3] -> BF16 [P][kInC] (zero padded)
__global__ void k_in_pack(const float *__restrict__ s, uint32_t P, __bf16 *__restrict__ x)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x)
        for (int c = 0; c < kInC; ++c) x[(size_t)p * kInC + c] = (__bf16)(c < kStateC ? s[(size_t)p * kStateC + c] : 0.f);
}

// state planes (FP64, [B][H][W] each) -> FP32 [P][3] with the velocity divided by u_scale, and back
__global__ void k_from_planes(const double *__restrict__ phi, const double *__restrict__ ux, const double *__restrict__ uy,
                              float inv_u, uint32_t P, float *__restrict__ s)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        s[(size_t)p * 3 + 0] = (float)phi[p];
        s[(size_t)p * 3 + 1] = (float)ux[p] * inv_u;
        s[(size_t)p * 3 + 2] = (float)uy[p] * inv_u;
    }
}

__global__ void k_to_planes(const float *__restrict__ s, double u_scale, uint32_t P, double *__restrict__ phi,
                            double *__restrict__ ux, double *__restrict__ uy)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        phi[p] = s[(size_t)p * 3 + 0];
        ux[p] = s[(size_t)p * 3 + 1] * u_scale;
        uy[p] = s[(size_t)p * 3 + 2] * u_scale;
    }
}

// partial sums of (a - b)^2 and b^2 over P points, one pair per block (FP64)
constexpr int kErrBlocks = 256;
__global__ __launch_bounds__(256) void k_err_partial(const double *__restrict__ a, const double *__restrict__ b, uint32_t P,
                                                     double *__restrict__ partial)
{
    __shared__ double r0[256], r1[256];
    double d2 = 0, b2 = 0;
    for (uint32_t p = blockIdx.x * 256u + threadIdx.x; p < P; p += gridDim.x * 256u) {
        const double d = a[p] - b[p];
        d2 += d * d;
        b2 += b[p] * b[p];
    }
    r0[threadIdx.x] = d2;
    r1[threadIdx.x] = b2;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            r0[threadIdx.x] += r0[threadIdx.x + k];
            r1[threadIdx.x] += r1[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = r0[0];
        partial[2 * blockIdx.x + 1] = r1[0];
    }
}

}  // namespace

// ==========================================================================================
// host side

struct lbcm_net {
    int batch = 0, H = 0, W = 0, C = 0, L = 0;
    uint32_t P = 0;
    hipStream_t stream = nullptr;
    std::vector<int> cin_r, cout_r, cin, cout;  // real and padded channel counts per layer
    std::vector<size_t> w_off, b_off;           // offsets of each layer in the parameter vector
    size_t nparams = 0;
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    std::vector<__bf16 *> Wf, Wb;
    std::vector<__bf16 *> act;                  // act[0] = packed input, act[l + 1] = output of layer l (l < L - 1)
    __bf16 *dz_a = nullptr, *dz_b = nullptr;    // gradient ping-pong buffers (P x C)
    float *resid = nullptr, *out = nullptr;     // FP32 [P][3]
    float *dw_partial = nullptr, *db_partial = nullptr, *loss_partial = nullptr;
    int loss_blocks = 0;
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

int launch_conv(lbcm_net *n, const __bf16 *X, int cin, const __bf16 *Wp, const float *bias, int cout, int sign, int relu,
                const __bf16 *mask, int mode, __bf16 *Y, const float *resid, float *Yf)
{
    const uint32_t waves = n->P / kPixPerWave;
    const dim3 grid((waves + kConvThreads / 64 - 1) / (kConvThreads / 64)), block(kConvThreads);
    switch (cout / 16) {
    case 1: hipLaunchKernelGGL(k_conv<1>, grid, block, 0, n->stream, X, cin, Wp, bias, cout, sign, relu, mask, mode, Y, resid, Yf, n->P, n->H, n->W); break;
    case 2: hipLaunchKernelGGL(k_conv<2>, grid, block, 0, n->stream, X, cin, Wp, bias, cout, sign, relu, mask, mode, Y, resid, Yf, n->P, n->H, n->W); break;
    case 4: hipLaunchKernelGGL(k_conv<4>, grid, block, 0, n->stream, X, cin, Wp, bias, cout, sign, relu, mask, mode, Y, resid, Yf, n->P, n->H, n->W); break;
    default: return nfail(n, LBCM_EINVAL, "unsupported channel count");
    }
    NHIP(n, hipGetLastError());
    return LBCM_OK;
}

int pack_all(lbcm_net *n)
{
    for (int l = 0; l < n->L; ++l) {
        hipLaunchKernelGGL(k_pack, dim3(grid_of(9 * (size_t)n->cin[l] * n->cout[l], 256)), dim3(256), 0, n->stream,
                           n->params + n->w_off[l], n->cin_r[l], n->cout_r[l], n->cin[l], n->cout[l], n->Wf[l], n->Wb[l]);
        NHIP(n, hipGetLastError());
    }
    n->packed = true;
    return LBCM_OK;
}

// forward from the FP32 state in n->resid ([P][3]); result in n->out
int forward(lbcm_net *n)
{
    if (!n->packed) {
        int rc = pack_all(n);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_in_pack, dim3(grid_of(n->P, 256)), dim3(256), 0, n->stream, n->resid, n->P, n->act[0]);
    NHIP(n, hipGetLastError());
    for (int l = 0; l < n->L; ++l) {
        const bool last = l == n->L - 1;
        int rc = launch_conv(n, n->act[l], n->cin[l], n->Wf[l], n->params + n->b_off[l], n->cout[l], 1, last ? 0 : 1, nullptr,
                             last ? 1 : 0, last ? nullptr : n->act[l + 1], n->resid, n->out);
        if (rc) return rc;
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
    if (batch < 1 || height < 1 || width < 1 || P % kPixPerWave || P > 0xffffffffull / 64) {
        g_net_error = "batch * height * width must be a positive multiple of 32 (and below 2^26)";
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
    for (int l = 0; l < layers; ++l) {
        n->cin_r.push_back(l == 0 ? kStateC : channels);
        n->cout_r.push_back(l == layers - 1 ? kStateC : channels);
        n->cin.push_back(l == 0 ? kInC : channels);
        n->cout.push_back(l == layers - 1 ? kOutC : channels);
        n->w_off.push_back(n->nparams);
        n->nparams += 9 * (size_t)n->cin_r[l] * n->cout_r[l];
        n->b_off.push_back(n->nparams);
        n->nparams += n->cout_r[l] + (n->cout[l] - n->cout_r[l]);  // bias padded to cout (zeros)
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
    for (int l = 0; l < layers; ++l) {
        const size_t wb = 9 * (size_t)n->cin[l] * n->cout[l] * sizeof(__bf16);
        if (!dmalloc((void **)&n->Wf[l], wb) || !dmalloc((void **)&n->Wb[l], wb)) return bail("out of device memory (packs)");
    }
    n->act.assign(layers, nullptr);
    if (!dmalloc((void **)&n->act[0], P * kInC * sizeof(__bf16))) return bail("out of device memory (input)");
    for (int l = 1; l < layers; ++l)
        if (!dmalloc((void **)&n->act[l], P * channels * sizeof(__bf16))) return bail("out of device memory (activations)");
    if (!dmalloc((void **)&n->dz_a, P * 64 * sizeof(__bf16)) || !dmalloc((void **)&n->dz_b, P * 64 * sizeof(__bf16)))
        return bail("out of device memory (gradients)");
    if (!dmalloc((void **)&n->resid, P * kStateC * sizeof(float)) || !dmalloc((void **)&n->out, P * kStateC * sizeof(float)))
        return bail("out of device memory (state)");
    const size_t nchunks = (P + kDwChunk - 1) / kDwChunk;
    if (!dmalloc((void **)&n->dw_partial, nchunks * 9 * 64 * 64 * sizeof(float))) return bail("out of device memory (dW)");
    if (!dmalloc((void **)&n->db_partial, ((P + 1023) / 1024) * 64 * sizeof(float))) return bail("out of device memory (db)");
    n->loss_blocks = grid_of(P, 256) > 1024 ? 1024 : grid_of(P, 256);
    if (!dmalloc((void **)&n->loss_partial, n->loss_blocks * sizeof(float))) return bail("out of device memory (loss)");
    *out = n;
    return LBCM_OK;
}

size_t lbcm_net_param_count(const lbcm_net *n) { return n ? n->nparams : 0; }

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

int lbcm_net_forward_planes(lbcm_net *n, const double *phi, const double *ux, const double *uy, double u_scale,
                            double *phi_out, double *ux_out, double *uy_out)
{
    if (!n || !phi || !ux || !uy || !phi_out || !ux_out || !uy_out || !(u_scale > 0)) return LBCM_EINVAL;
    hipLaunchKernelGGL(k_from_planes, dim3(grid_of(n->P, 256)), dim3(256), 0, n->stream, phi, ux, uy, (float)(1.0 / u_scale),
                       n->P, n->resid);
    NHIP(n, hipGetLastError());
    int rc = forward(n);
    if (rc) return rc;
    hipLaunchKernelGGL(k_to_planes, dim3(grid_of(n->P, 256)), dim3(256), 0, n->stream, n->out, u_scale, n->P, phi_out,
                       ux_out, uy_out);
    NHIP(n, hipGetLastError());
    return LBCM_OK;
}

int lbcm_net_state_from_planes(lbcm_net *n, const double *phi, const double *ux, const double *uy, double u_scale,
                               float *state)
{
    if (!n || !phi || !ux || !uy || !state || !(u_scale > 0)) return LBCM_EINVAL;
    hipLaunchKernelGGL(k_from_planes, dim3(grid_of(n->P, 256)), dim3(256), 0, n->stream, phi, ux, uy, (float)(1.0 / u_scale),
                       n->P, state);
    NHIP(n, hipGetLastError());
    return LBCM_OK;
}

int lbcm_net_backward(lbcm_net *n, const float *target, float *loss)
{
    if (!n || !target) return LBCM_EINVAL;
    const uint32_t P = n->P;
    const int L = n->L;
    hipLaunchKernelGGL(k_loss, dim3(n->loss_blocks), dim3(256), 0, n->stream, n->out, target, P, n->dz_a, n->loss_partial);
    NHIP(n, hipGetLastError());
    __bf16 *dz = n->dz_a, *dn = n->dz_b;
    const int nchunks = (int)((P + kDwChunk - 1) / kDwChunk);
    const int dbb = (int)((P + 1023) / 1024);
    for (int l = L - 1; l >= 0; --l) {
        // weight and bias gradients of layer l from its input act[l] and dz (gradient of its output)
        hipLaunchKernelGGL(k_conv_dw, dim3(nchunks, 9), dim3(kConvThreads), 0, n->stream, n->act[l], n->cin[l], dz, n->cout[l],
                           P, n->H, n->W, n->dw_partial);
        NHIP(n, hipGetLastError());
        hipLaunchKernelGGL(k_dw_reduce, dim3(grid_of(9 * (size_t)n->cin_r[l] * n->cout_r[l], 256)), dim3(256), 0, n->stream,
                           n->dw_partial, nchunks, n->cin[l], n->cout[l], n->cin_r[l], n->cout_r[l], n->grads + n->w_off[l]);
        NHIP(n, hipGetLastError());
        hipLaunchKernelGGL(k_db_partial, dim3(dbb), dim3(256), 0, n->stream, dz, n->cout[l], P, n->db_partial);
        NHIP(n, hipGetLastError());
        hipLaunchKernelGGL(k_db_reduce, dim3(1), dim3(64), 0, n->stream, n->db_partial, dbb, n->cout[l], n->grads + n->b_off[l]);
        NHIP(n, hipGetLastError());
        if (l == 0) break;
        // gradient of the layer input, times the ReLU derivative of that input (act[l] > 0)
        int rc = launch_conv(n, dz, n->cout[l], n->Wb[l], nullptr, n->cin[l], 1, 0, n->act[l], 0, dn, nullptr, nullptr);
        if (rc) return rc;
        std::swap(dz, dn);
    }
    if (loss) {
        std::vector<float> part(n->loss_blocks);
        NHIP(n, hipMemcpyAsync(part.data(), n->loss_partial, part.size() * sizeof(float), hipMemcpyDeviceToHost, n->stream));
        NHIP(n, hipStreamSynchronize(n->stream));
        double s = 0;
        for (float v : part) s += v;
        *loss = (float)(s / (3.0 * P));
    }
    return LBCM_OK;
}

int lbcm_net_adam(lbcm_net *n, float lr, float beta1, float beta2, float eps, int64_t t)
{
    if (!n || t < 1) return LBCM_EINVAL;
    const float c1 = 1.f - std::pow(beta1, (float)t), c2 = 1.f - std::pow(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(grid_of(n->nparams, 256)), dim3(256), 0, n->stream, n->params, n->grads, n->adam_m, n->adam_v,
                       n->nparams, lr, beta1, beta2, eps, c1, c2);
    NHIP(n, hipGetLastError());
    n->packed = false;
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
    f(n->dz_a);
    f(n->dz_b);
    f(n->resid);
    f(n->out);
    f(n->dw_partial);
    f(n->db_partial);
    f(n->loss_partial);
    delete n;
    return LBCM_OK;
}

const char *lbcm_net_last_error(const lbcm_net *n) { return n ? n->err.c_str() : g_net_error.c_str(); }

}  // extern "C"

// ==========================================================================================
// hybrid driver: surrogate jumps checked against the lattice Boltzmann step

struct lbcm_hybrid {
    lbcm_handle *lat = nullptr;
    lbcm_net *net = nullptr;
    int K = 0, J = 0;
    double u_scale = 1, threshold = 0;
    uint32_t P = 0;
    double *start = nullptr, *a = nullptr, *b = nullptr, *lbphi = nullptr;  // 3 planes each (lbphi: 1)
    double *err_partial = nullptr;
    bool cooldown = false;
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

#define HCALL(h, call, what)                                                                   \
    do {                                                                                       \
        int rc_ = (call);                                                                      \
        if (rc_ != LBCM_OK) return hfail(h, rc_, std::string(what) + ": " + lbcm_last_error(h->lat) + lbcm_net_last_error(h->net)); \
    } while (0)

double *plane(double *base, uint32_t P, int k) { return base + (size_t)k * P; }

// relative L2 difference of two device planes: ||x - ref|| / ||ref|| (FP64, synchronises)
int phi_error(lbcm_hybrid *h, const double *x, const double *ref, double *out)
{
    hipStream_t s = h->net->stream;
    hipLaunchKernelGGL(k_err_partial, dim3(kErrBlocks), dim3(256), 0, s, x, ref, h->P, h->err_partial);
    if (hipGetLastError() != hipSuccess) return hfail(h, LBCM_EHIP, "k_err_partial launch failed");
    double part[2 * kErrBlocks];
    if (hipMemcpyAsync(part, h->err_partial, sizeof(part), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return hfail(h, LBCM_EHIP, "reading the error sums failed");
    double d2 = 0, r2 = 0;
    for (int i = 0; i < kErrBlocks; ++i) {
        d2 += part[2 * i];
        r2 += part[2 * i + 1];
    }
    *out = r2 > 0 ? std::sqrt(d2 / r2) : (d2 > 0 ? INFINITY : 0.0);
    return LBCM_OK;
}

// one window of J * K lattice steps
int hybrid_window(lbcm_hybrid *h)
{
    const uint32_t P = h->P;
    const int64_t span = (int64_t)h->J * h->K;
    if (h->cooldown) {  // plain lattice Boltzmann window after a failed check
        HCALL(h, lbcm_step(h->lat, span), "lbcm_step");
        h->st.lb_steps_run += span;
        h->st.steps += span;
        h->cooldown = false;
        return LBCM_OK;
    }
    double *x = h->a, *y = h->b;
    HCALL(h, lbcm_fields_device(h->lat, plane(h->start, P, 0), nullptr, plane(h->start, P, 1), plane(h->start, P, 2), nullptr),
          "lbcm_fields_device");
    const double *cur = h->start;
    for (int j = 0; j < h->J - 1; ++j) {  // J - 1 surrogate jumps
        HCALL(h, lbcm_net_forward_planes(h->net, plane((double *)cur, P, 0), plane((double *)cur, P, 1), plane((double *)cur, P, 2),
                                         h->u_scale, plane(y, P, 0), plane(y, P, 1), plane(y, P, 2)),
              "lbcm_net_forward_planes");
        cur = y;
        std::swap(x, y);
    }
    // the last jump of the window by both: the surrogate into y, the lattice from the same state
    HCALL(h, lbcm_net_forward_planes(h->net, plane((double *)cur, P, 0), plane((double *)cur, P, 1), plane((double *)cur, P, 2),
                                     h->u_scale, plane(y, P, 0), plane(y, P, 1), plane(y, P, 2)),
          "lbcm_net_forward_planes");
    HCALL(h, lbcm_init_device(h->lat, plane((double *)cur, P, 0), nullptr, plane((double *)cur, P, 1), plane((double *)cur, P, 2)),
          "lbcm_init_device");
    HCALL(h, lbcm_step(h->lat, h->K), "lbcm_step");
    HCALL(h, lbcm_fields_device(h->lat, h->lbphi, nullptr, nullptr, nullptr, nullptr), "lbcm_fields_device");
    double e = 0;
    int rc = phi_error(h, plane(y, P, 0), h->lbphi, &e);
    if (rc) return rc;
    h->st.checks += 1;
    h->st.last_error = e;
    h->st.max_error = std::max(h->st.max_error, e);
    if (!(e <= h->threshold)) {
        // rejected: redo the window with the lattice Boltzmann step from its starting fields
        h->st.failed_checks += 1;
        HCALL(h, lbcm_init_device(h->lat, plane(h->start, P, 0), nullptr, plane(h->start, P, 1), plane(h->start, P, 2)),
              "lbcm_init_device");
        HCALL(h, lbcm_step(h->lat, span), "lbcm_step");
        h->st.lb_steps_run += h->K + span;
        h->cooldown = true;
    } else {
        h->st.jumps += h->J - 1;
        h->st.lb_steps_run += h->K;
    }
    h->st.steps += span;
    return LBCM_OK;
}

}  // namespace

extern "C" {

int lbcm_hybrid_create(lbcm_handle *lattice, lbcm_net *net, int32_t steps_per_jump, int32_t jumps_per_check, double u_scale,
                       double threshold, lbcm_hybrid **out)
{
    if (!out) return LBCM_EINVAL;
    *out = nullptr;
    lbcm_params p;
    if (!lattice || !net || lbcm_info(lattice, &p) != LBCM_OK) {
        g_hybrid_error = "lattice and network are required";
        return LBCM_EINVAL;
    }
    if (steps_per_jump < 1 || jumps_per_check < 1 || !(u_scale > 0) || !(threshold >= 0)) {
        g_hybrid_error = "steps_per_jump and jumps_per_check must be >= 1, u_scale > 0, threshold >= 0";
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
    h->threshold = threshold;
    h->P = net->P;
    const size_t pb = (size_t)h->P * sizeof(double);
    if (hipMalloc((void **)&h->start, 3 * pb) != hipSuccess || hipMalloc((void **)&h->a, 3 * pb) != hipSuccess ||
        hipMalloc((void **)&h->b, 3 * pb) != hipSuccess || hipMalloc((void **)&h->lbphi, pb) != hipSuccess ||
        hipMalloc((void **)&h->err_partial, 2 * kErrBlocks * sizeof(double)) != hipSuccess) {
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
    for (int64_t w = 0; w < windows; ++w) {
        int rc = hybrid_window(h);
        if (rc) return rc;
    }
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
    for (void *q : {(void *)h->start, (void *)h->a, (void *)h->b, (void *)h->lbphi, (void *)h->err_partial})
        if (q) (void)hipFree(q);
    delete h;
    return LBCM_OK;
}

const char *lbcm_hybrid_last_error(const lbcm_hybrid *h) { return h ? h->err.c_str() : g_hybrid_error.c_str(); }

}  // extern "C"
