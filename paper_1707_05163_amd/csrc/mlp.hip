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

}  // namespace

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
