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
// core's A operand (read from LDS, where the block streams them half a layer at a time) and
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
constexpr int kStride256 = 256 + 8;  // bf16 per staged weight row of a 256-input layer
constexpr int kStride64 = 64 + 8;    // the same for the 64-input first layer (the 8 bf16 of
                                     // padding put 16 consecutive rows on distinct banks)
constexpr int kHalfRows = 128;       // weight rows (output features) per LDS buffer

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

// One step of the network on a wave's 32 rows: the products of one 32-feature output
// block with K inputs (weights from LDS rows of STRIDE bf16 at w, biases at b; the
// accumulator starts from the biases of the features the lane holds and takes the K/16
// products in k order), written beside the epilogue of the block before (prev): GELU
// and bf16 of its 16 values, then the half-wave exchange into the next layer's two
// operands o0, o1 for those 32 features.  Left to itself the compiler issues all the
// products first and the epilogue after them; here the step is cut into one piece per
// product, fenced so that nothing moves across: the weights of the product three
// ahead are read from LDS, the product is issued, and a share of the epilogue follows
// while the matrix core works.  At a layer's first block the previous block is the
// previous layer's last one (CROSS): its outputs are this layer's inputs for k-steps
// K/16 - 2 and K/16 - 1 (o0 and o1 alias in[] there), so those two products come last.
template <int K, int STRIDE, bool PREV, bool CROSS>
__device__ inline f32x16 step(const uint16_t *w, const float *b, int r, int h,
                              const bf16x8 (&in)[16], const f32x16 &prev, bf16x8 &o0,
                              bf16x8 &o1)
{
    constexpr int kSteps = K / 16, kAhead = 3, kLate = CROSS ? 2 : 0, kPer = 16 / kSteps;
    static_assert(!CROSS || PREV, "a layer's first block follows the previous layer's last");
    f32x16 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 v = *reinterpret_cast<const float4 *>(b + 8 * q + 4 * h);
        acc[4 * q + 0] = v.x;
        acc[4 * q + 1] = v.y;
        acc[4 * q + 2] = v.z;
        acc[4 * q + 3] = v.w;
    }
    const uint16_t *wr = w + r * STRIDE + 8 * h;
    bf16x8 wq[kSteps];
#pragma unroll
    for (int i = 0; i < kAhead && i < kSteps; ++i)
        wq[i] = *reinterpret_cast<const bf16x8 *>(wr + 16 * i);
    __builtin_amdgcn_sched_barrier(0);
    float g[16];
    uint32_t P[8];
#pragma unroll
    for (int i = 0; i < kSteps; ++i) {
        if (i + kAhead < kSteps)
            wq[i + kAhead] = *reinterpret_cast<const bf16x8 *>(wr + 16 * (i + kAhead));
        if (i < kSteps - kLate)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq[i], in[i], acc, 0, 0, 0);
        if constexpr (PREV) {
#pragma unroll
            for (int v = i * kPer; v < (i + 1) * kPer; ++v) {
                g[v] = gelu_sigmoid(prev[v]);
                if (v & 1)
                    P[v >> 1] = pack_bf16(g[v - 1], g[v]);
                // lanes 32-63 of the first register trade places with lanes 0-31 of the
                // second, once both are packed
                if (v == 7 || v == 15) {
                    const int j0 = v == 7 ? 0 : 4;
#pragma unroll
                    for (int j = j0; j < j0 + 2; ++j) {
                        auto x = __builtin_amdgcn_permlane32_swap(P[j], P[j + 2], false, false);
                        P[j] = x[0];
                        P[j + 2] = x[1];
                    }
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (PREV) {
        o0 = __builtin_bit_cast(bf16x8, u32x4_t{P[0], P[1], P[2], P[3]});
        o1 = __builtin_bit_cast(bf16x8, u32x4_t{P[4], P[5], P[6], P[7]});
    }
    if constexpr (CROSS) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq[kSteps - 2], o0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq[kSteps - 1], o1, acc, 0, 0, 0);
    }
    return acc;
}

typedef __attribute__((address_space(3))) void *lds_ptr_t;

// Rows [0, R) of a row-major [R x K] bf16 matrix at src, loaded straight into LDS rows
// of STRIDE bf16 at dst without passing through registers: K/8 lanes carry a row, 16
// bytes each.  Such a load writes its lanes' 16-byte pieces one after the other from
// one wave-uniform LDS address, so each row is one load with the lanes of the other
// rows switched off.  Row n0 + q of a group of G rows starts 16 q bytes past
// n0 STRIDE*2 + q K*2 (the padding of the rows before it); that shift goes into the
// load's immediate offset, which the hardware adds to the global address as well (the
// lanes' pointers are moved back by it).  The LDS address is then the same for the G
// loads of a group, and their immediates differ, so the compiler can never fold the
// G masked loads into one.  Wave w takes rows w R/8 .. (w + 1) R/8 - 1.  The loads
// count as the wave's vector-memory operations until the data is in LDS.
template <int Q, int G>
__device__ inline void load_row_group(const uint16_t *p, lds_ptr_t d, int g)
{
    if constexpr (Q < G) {
        if (g == Q)
            __builtin_amdgcn_global_load_lds(p, d, 16, 16 * Q, 0);
        load_row_group<Q + 1, G>(p, d, g);
    }
}

template <int R, int K, int STRIDE>
__device__ inline void load_rows_to_lds(uint16_t *dst, const uint16_t *src, int wave, int lane)
{
    constexpr int L = K / 8, G = 64 / L, kPerWave = R / 8;
    static_assert(kPerWave % G == 0, "whole groups of rows per wave");
    static_assert(STRIDE * 2 - K * 2 == 16, "16 bytes of padding per row");
    const int g = lane / L, c = lane % L;
#pragma unroll
    for (int i = 0; i < kPerWave; i += G) {
        const int n0 = wave * kPerWave + i;
        const uint16_t *p = src + (size_t)(n0 + g) * K + c * 8 - 8 * g;
        const lds_ptr_t d = (lds_ptr_t)(reinterpret_cast<char *>(dst) + n0 * STRIDE * 2);
        load_row_group<0, G>(p, d, g);
    }
}

// The wave's own loads into LDS have landed; after the barrier every wave's have, and
// every wave is done reading the buffer that the loads issued next overwrite.
__device__ inline void chunk_sync()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
}

// Weights stream through two LDS buffers in eight chunks per tile: the first layer
// (buffer 0), then each 256-input layer as output features 0-127 (buffer 1) and
// 128-255 (buffer 0), then the output layer (buffer 1).  Each chunk's loads are issued
// one chunk ahead, right after the barrier that frees their buffer, so they run while
// the matrix core works on the other buffer.  Eight chunks per tile keep every
// chunk's buffer the same from tile to tile, so each access names its buffer at
// compile time (and the compiler waits for loads into one buffer only before reading
// that one).
__global__ __launch_bounds__(kFusedThreads) void k_mlp_fused(MlpFusedArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t buf0[kHalfRows * kStride256];
    __shared__ __attribute__((aligned(16))) uint16_t buf1[kHalfRows * kStride256];
    __shared__ __attribute__((aligned(16))) float bl[4 * 256 + 32];
    static_assert(256 * kStride64 <= kHalfRows * kStride256, "first layer fits one buffer");
    const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t ntile = (a.rows + kFusedRows - 1) / kFusedRows;
    for (int c = threadIdx.x; c < 4 * 256 + 32; c += kFusedThreads)
        bl[c] = c < 1024 ? a.bias[c >> 8][c & 255] : a.bias[4][c - 1024];
    load_rows_to_lds<256, 64, kStride64>(buf0, a.WT[0], wave, lane);  // grid <= tiles
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t row = tile * kFusedRows + wave * 32 + r;
        const bool live = row < a.rows;
        bf16x8 in[16], out[16];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            in[s] = live ? *reinterpret_cast<const bf16x8 *>(a.X + row * 64 + 16 * s + 8 * h)
                         : bf16x8{};
        chunk_sync();
        load_rows_to_lds<128, 256, kStride256>(buf1, a.WT[1], wave, lane);
        // first layer, 64 inputs, weights in buffer 0
        f32x16 cur = step<64, kStride64, false, false>(buf0, bl, r, h, in, f32x16{}, out[0], out[1]);
#pragma unroll
        for (int nb = 1; nb < 8; ++nb)
            cur = step<64, kStride64, true, false>(buf0 + nb * 32 * kStride64, bl + nb * 32, r, h,
                                                   in, cur, out[2 * nb - 2], out[2 * nb - 1]);
        // 256-input layers: output features 0-127 from buffer 1, 128-255 from buffer 0
#pragma unroll 1
        for (int l = 1; l < 4; ++l) {
            chunk_sync();
            load_rows_to_lds<128, 256, kStride256>(buf0, a.WT[l] + 128 * 256, wave, lane);
            const float *bias = bl + 256 * l;
#pragma unroll
            for (int s = 0; s < 14; ++s)
                in[s] = out[s];
            cur = step<256, kStride256, true, true>(buf1, bias, r, h, in, cur, in[14], in[15]);
#pragma unroll
            for (int nb = 1; nb < 4; ++nb)
                cur = step<256, kStride256, true, false>(buf1 + nb * 32 * kStride256, bias + nb * 32,
                                                         r, h, in, cur, out[2 * nb - 2],
                                                         out[2 * nb - 1]);
            chunk_sync();
            if (l < 3)
                load_rows_to_lds<128, 256, kStride256>(buf1, a.WT[l + 1], wave, lane);
            else
                load_rows_to_lds<32, 256, kStride256>(buf1, a.WT[4], wave, lane);
#pragma unroll
            for (int nb = 4; nb < 8; ++nb)
                cur = step<256, kStride256, true, false>(buf0 + (nb - 4) * 32 * kStride256,
                                                         bias + nb * 32, r, h, in, cur,
                                                         out[2 * nb - 2], out[2 * nb - 1]);
        }
        // output layer, weights in buffer 1; the next tile's first layer goes to buffer 0
        chunk_sync();
        if (tile + gridDim.x < ntile)
            load_rows_to_lds<256, 64, kStride64>(buf0, a.WT[0], wave, lane);
#pragma unroll
        for (int s = 0; s < 14; ++s)
            in[s] = out[s];
        const f32x16 y = step<256, kStride256, true, true>(buf1, bl + 1024, r, h, in, cur, in[14],
                                                           in[15]);
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
    int cus = 0, dev = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    const int64_t ntile = (a.rows + kFusedRows - 1) / kFusedRows;
    const uint32_t grid = (uint32_t)(ntile < cus ? ntile : cus);
    hipLaunchKernelGGL(k_mlp_fused, dim3(grid), dim3(kFusedThreads), 0, s, a);
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
