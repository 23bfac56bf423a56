// mlp.hip -- BF16 matrix-core kernels of the flow-map surrogate network.
//
// The surrogate is a fully connected network 64 -> 256 -> 256 -> 256 -> 256 -> 2 with
// the tanh form of GELU after each hidden layer (Hendrycks & Gimpel, 2016).  Weights
// and activations are bfloat16, products accumulate in FP32 on the gfx950 matrix
// cores (v_mfma_f32_32x32x16_bf16), and the optimiser keeps FP32 master weights.
//
// One GEMM kernel serves every product:
//   C[M x N] = sum_k A(i, k) B(k, j),  A(i, k) = A[i*sai + k*sak], B(k, j) = B[k*sbk + j*sbj]
// Each wave owns a 32-row band and NB 32-column blocks of C; a block is 4 waves
// (128 rows).  A k-step of 16 feeds one 32x32x16 MFMA per column block.  Operand
// fragments are loaded straight from global memory (weights and activation tiles
// stay in L2); with a unit k-stride a lane's eight bf16 values are one 16-byte load.
#include "lp_internal.h"

namespace lp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr float kC0 = 0.7978845608028654f;  // sqrt(2/pi)
constexpr float kC1 = 0.044715f;

__device__ inline float gelu(float x)
{
    return 0.5f * x * (1.f + tanhf(kC0 * (x + kC1 * x * x * x)));
}

__device__ inline float gelu_grad(float x)
{
    const float t = tanhf(kC0 * (x + kC1 * x * x * x));
    return 0.5f * (1.f + t) + 0.5f * x * (1.f - t * t) * kC0 * (1.f + 3.f * kC1 * x * x);
}

__device__ inline uint16_t bf16_bits(float f)
{
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu))
        return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ inline float bf16_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// eight consecutive-k values of A(i, .) or B(., j) as an MFMA operand
__device__ inline bf16x8 frag(const uint16_t *p, int64_t kstride)
{
    if (kstride == 1)
        return *reinterpret_cast<const bf16x8 *>(p);
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e)
        v[e] = __builtin_bit_cast(__bf16, p[e * kstride]);
    return v;
}

}  // namespace

namespace {

template <int EPI, int NB>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t row0 = (int64_t)blockIdx.x * 128 + wave * 32;
    if (row0 >= g.M)  // a 32-row band past the end (M is a multiple of 32)
        return;
    const int64_t col0 = (int64_t)blockIdx.y * (32 * NB);
    const int64_t k_lo = (int64_t)blockIdx.z * g.kchunk;
    const int64_t k_hi = k_lo + g.kchunk < g.K ? k_lo + g.kchunk : g.K;
    f32x16 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
        acc[b] = f32x16{0.f};
    const int r = lane & 31, kh = (lane >> 5) * 8;
    const uint16_t *Ar = g.A + (row0 + r) * g.sai;
    for (int64_t k0 = k_lo; k0 < k_hi; k0 += 16) {
        const bf16x8 a = frag(Ar + (k0 + kh) * g.sak, g.sak);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const bf16x8 bb = frag(g.B + (k0 + kh) * g.sbk + (col0 + b * 32 + r) * g.sbj, g.sbk);
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc[b], 0, 0, 0);
        }
    }
    // accumulator layout: value v of lane l is C[8 (v/4) + 4 (l/32) + v%4][l%32]
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int64_t j = col0 + b * 32 + r;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t i = row0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const float c = acc[b][v];
            if constexpr (EPI == kEpiHidden) {
                const float z = c + g.bias[j];
                if (g.Z)
                    g.Z[i * g.ldc + j] = z;
                g.H[i * g.ldc + j] = bf16_bits(gelu(z));
            } else if constexpr (EPI == kEpiOut) {
                if (j < g.nvalid)
                    g.Y[i * g.ldy + j] = c + g.bias[j];
            } else if constexpr (EPI == kEpiBackData) {
                const float dz = c * gelu_grad(g.Zin[i * g.ldc + j]);
                g.dZ[i * g.ldc + j] = dz;
                g.H[i * g.ldc + j] = bf16_bits(dz);
            } else {
                atomicAdd(&g.Y[i * g.ldy + j], c);
            }
        }
    }
}

// dY = (Y - T) / B on the two outputs, zero on the padding columns; also bf16 copy
__global__ void k_loss_grad(const float *Y, const float *T, int64_t B, int ldy, float inv_b,
                            float *dZ, uint16_t *dZq, float *loss)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= B * ldy)
        return;
    const int64_t row = i / ldy;
    const int col = (int)(i % ldy);
    float d = 0.f;
    if (col < 2) {
        const float e = Y[row * ldy + col] - T[row * 2 + col];
        d = e * inv_b;
        atomicAdd(loss, 0.5f * e * e * inv_b);
    }
    dZ[i] = d;
    dZq[i] = bf16_bits(d);
}

// column sums of dZ [B x N] (bias gradients)
__global__ void k_colsum(const float *dZ, int64_t B, int N, float *db)
{
    const int j = blockIdx.x;
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < B; i += blockDim.x)
        s += dZ[i * N + j];
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_xor(s, off, 64);
    __shared__ float ws[4];
    if ((threadIdx.x & 63) == 0)
        ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        db[j] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Adam on an FP32 master tensor [K x N]; also writes the bf16 copies W [K x N] and
// W^T [N x K].  Columns >= nvalid (output padding) stay zero.
__global__ void k_adam(float *W, const float *G, float *m, float *v, int K, int N, int nvalid,
                       float lr, float b1, float b2, float eps, float c1, float c2, uint16_t *Wb,
                       uint16_t *WT)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)K * N)
        return;
    const int k = (int)(i / N), j = (int)(i % N);
    float w = W[i];
    if (j < nvalid && G) {
        const float g = G[i];
        const float mm = b1 * m[i] + (1.f - b1) * g;
        const float vv = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mm;
        v[i] = vv;
        w -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
        W[i] = w;
    }
    const uint16_t h = bf16_bits(j < nvalid ? w : 0.f);
    if (Wb)
        Wb[i] = h;
    if (WT)
        WT[(int64_t)j * K + k] = h;
}

__global__ void k_fill_f32(float *p, float v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_to_bf16(const float *x, int64_t n, uint16_t *y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = bf16_bits(x[i]);
}

// ---------------------------------------------------------------- fused inference
// The whole network on one tile of 256 rows per block, activations in registers.
// Each layer is computed transposed, H^T = W^T A^T, so the weights are the matrix
// core's A operand (read from LDS, where the block stages one layer at a time) and
// the activations its B operand: lane l keeps 8 consecutive features of row
// (l mod 32) for each k-step.  The accumulator of the 32x32x16 product leaves lane
// l with features 8(v/4) + 4(l/32) + (v mod 4) of that row; two permlane32 swaps per
// 32-feature block move each half-wave's missing four features across, which is
// exactly the next layer's B-operand layout.  GELU in the sigmoid form
// x / (1 + exp(-2u)), u = sqrt(2/pi) (x + 0.044715 x^3), on the hardware exp2 and
// reciprocal; bf16 rounding by the round-to-nearest-even convert.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kFusedRows = 256;      // rows per tile: 8 waves x 32
constexpr int kFusedThreads = 512;
constexpr int kLdsStride = 256 + 8;  // bf16 per staged weight row (padding against bank conflicts)

__device__ inline float gelu_sigmoid(float x)
{
    constexpr float kLog2e = 1.4426950408889634f;
    const float t = x * x;
    const float m = x * fmaf(t, -2.f * kC0 * kC1 * kLog2e, -2.f * kC0 * kLog2e);
    return x * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(m));
}

__device__ inline uint32_t pack_bf16(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{a, b}, bf16x2_t));
}

// One 32-feature output block nb of a layer with K inputs (16-wide k-steps in `in`):
// the accumulator starts from the biases of the features the lane holds and takes the
// K/16 products in k order.
template <int K>
__device__ inline f32x16 fused_block(const uint16_t *wl, const float *bl, int r, int h, int nb,
                                     const bf16x8 (&in)[16])
{
    f32x16 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 b = *reinterpret_cast<const float4 *>(bl + nb * 32 + 8 * q + 4 * h);
        acc[4 * q + 0] = b.x;
        acc[4 * q + 1] = b.y;
        acc[4 * q + 2] = b.z;
        acc[4 * q + 3] = b.w;
    }
#pragma unroll
    for (int s = 0; s < K / 16; ++s) {
        const bf16x8 w =
            *reinterpret_cast<const bf16x8 *>(wl + (nb * 32 + r) * kLdsStride + 16 * s + 8 * h);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, in[s], acc, 0, 0, 0);
    }
    return acc;
}

// GELU + bf16 of one output block, then the half-wave exchange into the next layer's
// two operands for these 32 features
__device__ inline void block_epilogue(const f32x16 &acc, bf16x8 &o0, bf16x8 &o1)
{
    float g[16];
#pragma unroll
    for (int v = 0; v < 16; ++v)
        g[v] = gelu_sigmoid(acc[v]);
    uint32_t P[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        P[j] = pack_bf16(g[2 * j], g[2 * j + 1]);
    // lanes 32-63 of the first register trade places with lanes 0-31 of the second
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        auto lo = __builtin_amdgcn_permlane32_swap(P[j], P[j + 2], false, false);
        P[j] = lo[0];
        P[j + 2] = lo[1];
        auto hi = __builtin_amdgcn_permlane32_swap(P[j + 4], P[j + 6], false, false);
        P[j + 4] = hi[0];
        P[j + 6] = hi[1];
    }
    o0 = __builtin_bit_cast(bf16x8, u32x4_t{P[0], P[1], P[2], P[3]});
    o1 = __builtin_bit_cast(bf16x8, u32x4_t{P[4], P[5], P[6], P[7]});
}

// A hidden layer of 256 outputs, block by block: the epilogue of one block is written
// beside the products of the next, so that the wave's GELU arithmetic runs while the
// matrix core works (the products of a block depend only on the layer's inputs), and
// only two accumulators are live instead of eight.
template <int K>
__device__ inline void hidden_layer(const uint16_t *wl, const float *bl, int r, int h,
                                    bf16x8 (&in)[16])
{
    bf16x8 out[16];
    f32x16 cur = fused_block<K>(wl, bl, r, h, 0, in);
#pragma unroll
    for (int nb = 1; nb < 8; ++nb) {
        const f32x16 next = fused_block<K>(wl, bl, r, h, nb, in);
        block_epilogue(cur, out[2 * nb - 2], out[2 * nb - 1]);
        cur = next;
    }
    block_epilogue(cur, out[14], out[15]);
#pragma unroll
    for (int s = 0; s < 16; ++s)
        in[s] = out[s];
}

__device__ inline void stage_layer(uint16_t *wl, float *bl, const uint16_t *WT, const float *bias,
                                   int N, int K)
{
    __syncthreads();  // every wave is done with the previous layer's weights
    const int chunks = N * K / 8;
    for (int c = threadIdx.x; c < chunks; c += kFusedThreads) {
        const int n = c / (K / 8), kk = (c % (K / 8)) * 8;
        *reinterpret_cast<u32x4_t *>(wl + n * kLdsStride + kk) =
            *reinterpret_cast<const u32x4_t *>(WT + (size_t)n * K + kk);
    }
    for (int c = threadIdx.x; c < N; c += kFusedThreads)
        bl[c] = bias[c];
    __syncthreads();
}

__global__ __launch_bounds__(kFusedThreads) void k_mlp_fused(MlpFusedArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    uint16_t *wl = reinterpret_cast<uint16_t *>(lds);
    float *bl = reinterpret_cast<float *>(lds + 256 * kLdsStride * sizeof(uint16_t));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 31, h = lane >> 5;
    const int64_t ntile = (a.rows + kFusedRows - 1) / kFusedRows;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t row = tile * kFusedRows + wave * 32 + r;
        const bool live = row < a.rows;
        bf16x8 in[16];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            in[s] = live ? *reinterpret_cast<const bf16x8 *>(a.X + row * 64 + 16 * s + 8 * h)
                         : bf16x8{};
        stage_layer(wl, bl, a.WT[0], a.bias[0], 256, 64);
        hidden_layer<64>(wl, bl, r, h, in);
#pragma unroll 1
        for (int l = 1; l < 4; ++l) {
            stage_layer(wl, bl, a.WT[l], a.bias[l], 256, 256);
            hidden_layer<256>(wl, bl, r, h, in);
        }
        stage_layer(wl, bl, a.WT[4], a.bias[4], 32, 256);
        const f32x16 y = fused_block<256>(wl, bl, r, h, 0, in);
        // outputs 0 and 1 of the row sit in values 0 and 1 of the lower half-wave
        if (live && h == 0) {
            a.Y[row * 2 + 0] = y[0];
            a.Y[row * 2 + 1] = y[1];
        }
    }
}

}  // namespace

hipError_t launch_mlp_fused(const MlpFusedArgs &a, hipStream_t s)
{
    if (a.rows <= 0)
        return hipSuccess;
    if (a.rows % 32)
        return hipErrorInvalidValue;
    const size_t lds = 256 * kLdsStride * sizeof(uint16_t) + 256 * sizeof(float);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_mlp_fused,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        attr = true;
    }
    int cus = 0, dev = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    const int64_t ntile = (a.rows + kFusedRows - 1) / kFusedRows;
    const uint32_t grid = (uint32_t)(ntile < cus ? ntile : cus);
    hipLaunchKernelGGL(k_mlp_fused, dim3(grid), dim3(kFusedThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_gemm(int epi, const GemmArgs &g, hipStream_t s)
{
    if (g.M % 32 || g.K % 16 || g.kchunk % 16 || g.kchunk <= 0)
        return hipErrorInvalidValue;
    const int nb = g.N >= 128 ? 4 : 1;
    if (g.N % (32 * nb))
        return hipErrorInvalidValue;
    const dim3 grid((uint32_t)((g.M + 127) / 128), (uint32_t)(g.N / (32 * nb)),
                    (uint32_t)((g.K + g.kchunk - 1) / g.kchunk));
#define LP_G(E, NBV) hipLaunchKernelGGL((k_gemm<E, NBV>), grid, dim3(256), 0, s, g)
    if (nb == 4) {
        switch (epi) {
        case kEpiHidden: LP_G(kEpiHidden, 4); break;
        case kEpiOut: LP_G(kEpiOut, 4); break;
        case kEpiBackData: LP_G(kEpiBackData, 4); break;
        case kEpiAccum: LP_G(kEpiAccum, 4); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (epi) {
        case kEpiHidden: LP_G(kEpiHidden, 1); break;
        case kEpiOut: LP_G(kEpiOut, 1); break;
        case kEpiBackData: LP_G(kEpiBackData, 1); break;
        case kEpiAccum: LP_G(kEpiAccum, 1); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef LP_G
    return hipGetLastError();
}

hipError_t launch_loss_grad(const float *Y, const float *T, int64_t B, int ldy, float *dZ,
                            uint16_t *dZq, float *loss, hipStream_t s)
{
    const int64_t n = B * ldy;
    hipLaunchKernelGGL(k_loss_grad, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, Y, T, B,
                       ldy, 1.f / (float)B, dZ, dZq, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const float *dZ, int64_t B, int N, float *db, hipStream_t s)
{
    hipLaunchKernelGGL(k_colsum, dim3(N), dim3(256), 0, s, dZ, B, N, db);
    return hipGetLastError();
}

hipError_t launch_adam(float *W, const float *G, float *m, float *v, int K, int N, int nvalid,
                       float lr, float b1, float b2, float eps, int t, uint16_t *Wb, uint16_t *WT,
                       hipStream_t s)
{
    const int64_t n = (int64_t)K * N;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, W, G, m, v, K,
                       N, nvalid, lr, b1, b2, eps, c1, c2, Wb, WT);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s)
{
    int64_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_f32, dim3((uint32_t)(b > 4096 ? 4096 : (b ? b : 1))), dim3(256), 0,
                       s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *x, int64_t n, uint16_t *y, hipStream_t s)
{
    int64_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_to_bf16, dim3((uint32_t)(b > 4096 ? 4096 : (b ? b : 1))), dim3(256), 0,
                       s, x, n, y);
    return hipGetLastError();
}

}  // namespace lp
