// terrain_mlp.hip -- the learned warm start: a 12 -> 64 -> 64 -> 3 SiLU MLP
// that predicts each contact's initial impulses (lambda_n, lambda_t1,
// lambda_t2) / (m_eff g dt) in the contact frame.
//
//   k_mlp_bf16    inference on MFMA (v_mfma_f32_32x32x16_bf16): one wave per 32
//                 contacts, weights and activations in BF16, FP32 accumulate
//   k_mlp_f32     the same network in FP32 on the vector ALU (reference)
//   k_learned_lam lambda^0 = frame x output x scale, projected onto the bounds
//   k_mlp_train   FP32 forward + backward of 0.5 mean ||y - label||^2 on
//                 MFMA (FP32), per-block gradient partials reduced in fixed order
//   k_adam        Adam update
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "terrain_internal.h"

namespace trk {

namespace {

constexpr int kIn = 12, kH = 64, kOut = 3;
// offsets of the flat parameter vector
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kOut * kH, oScale = ob3 + kOut;
constexpr int kNP = oScale;  // trainable parameters (in_scale is fixed)
static_assert(oScale + kIn == kMlpParams, "parameter layout");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ inline float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float dsilu(float z)
{
    float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// SiLU of the BF16 inference: the hardware reciprocal (about 1 ulp) in place
// of a full division
__device__ inline float silu_fast(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

}  // namespace

// ---------------------------------------------------------------------------
// BF16 MFMA inference.  Each wave works alone on tiles of 32 contacts (no
// block barrier after the weights are staged): the block's weights sit in LDS
// as B operands, the input tile is read from global memory straight into the
// A operand (the next tile's rows in flight meanwhile), and one per-wave LDS
// tile turns each layer's D layout into the next layer's A layout.
//   layer 1: X[32 x 16] (12 inputs padded) . W1^T[16 x 64]: 2 N-tiles x 1 K-step
//   layer 2: H1[32 x 64] . W2^T[64 x 64]: 2 N-tiles x 4 K-steps
//   layer 3: H2[32 x 64] . W3^T[64 x 32] (3 of 32 columns used): 4 K-steps
// Operand layouts of v_mfma_f32_32x32x16_bf16 (A 32x16, B 16x32, D 32x32):
//   A[i][k] -> lane i + 32 (k / 8), element k % 8
//   B[k][j] -> lane j + 32 (k / 8), element k % 8
//   D[i][j] -> lane j + 32 ((i / 4) % 2), element (i % 4) + 4 (i / 8)
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kMlpWaves = 4;
constexpr int kHPitch = kH + 8;    // BF16 rows of 64 + 8 (16-byte aligned)

__device__ inline void wave_sync()
{
    // the LDS operations of one wave run in order; keep the compiler from
    // moving them across this point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp_bf16(const float* __restrict__ W, const float* __restrict__ feat,
                                                              float* __restrict__ out, const uint32_t* d_n, int64_t cap)
{
    // B operands: row j holds the weights into unit j (W1 padded to K = 16,
    // W3 padded to 32 rows), so lane (j, half) reads 8 consecutive K values
    __shared__ __attribute__((aligned(16))) __bf16 w1s[kH][16];
    __shared__ __attribute__((aligned(16))) __bf16 w2s[kH][kHPitch];
    __shared__ __attribute__((aligned(16))) __bf16 w3s[32][kHPitch];
    __shared__ __attribute__((aligned(16))) __bf16 hts[kMlpWaves][32][kHPitch];
    const int tid = threadIdx.x;
    for (int t = tid; t < kH * 16; t += blockDim.x) {
        const int j = t / 16, k = t % 16;
        w1s[j][k] = (__bf16)(k < kIn ? W[oW1 + j * kIn + k] : 0.0f);
    }
    for (int t = tid; t < kH * kH; t += blockDim.x) w2s[t / kH][t % kH] = (__bf16)W[oW2 + t];
    for (int t = tid; t < 32 * kH; t += blockDim.x) {
        const int j = t / kH, k = t % kH;
        w3s[j][k] = (__bf16)(j < kOut ? W[oW3 + j * kH + k] : 0.0f);
    }
    __syncthreads();  // the only block barrier: the weights are read-only afterwards

    const int wave = tid >> 6, lane = tid & 63;
    const int half = lane >> 5, col = lane & 31;
    const float bias1[2] = {W[ob1 + col], W[ob1 + 32 + col]};
    const float bias2[2] = {W[ob2 + col], W[ob2 + 32 + col]};
    const float bias3 = col < kOut ? W[ob3 + col] : 0.0f;
    float scl[8];  // scales of this lane's input columns 8 half .. 8 half + 7
    for (int q = 0; q < 8; ++q) scl[q] = half * 8 + q < kIn ? W[oScale + half * 8 + q] : 0.0f;

    const uint64_t n = d_n ? (uint64_t)min((uint64_t)*d_n, (uint64_t)cap) : (uint64_t)cap;
    const uint64_t ntiles = (n + 31) / 32;
    const uint64_t nwaves = (uint64_t)gridDim.x * kMlpWaves;
    __bf16(*ht)[kHPitch] = hts[wave];
    auto brow = [&](const __bf16* row, int k0) { return *reinterpret_cast<const bf16x8*>(row + k0 + half * 8); };
    // the input row of a tile: lane (col, half) holds features 8 half .. 8 half + 7
    // (only 8 .. 11 of the second half are inside the 12)
    auto load_x = [&](uint64_t tile, float4& x0, float4& x1) {
        const uint64_t c = tile * 32 + col;
        x0 = make_float4(0.f, 0.f, 0.f, 0.f);
        x1 = x0;
        if (tile < ntiles && c < n) {
            const float4* f = reinterpret_cast<const float4*>(feat + c * kIn);
            x0 = f[2 * half];
            if (half == 0) x1 = f[1];
        }
    };
    // D tile (+ bias, SiLU) -> BF16 rows of ht, N-tile nt
    auto store_h = [&](const floatx16& acc, float bias, int nt) {
        for (int e = 0; e < 16; ++e) {
            const int i = (e & 3) + 8 * (e >> 2) + 4 * half;
            ht[i][nt * 32 + col] = (__bf16)silu_fast(acc[e] + bias);
        }
    };
    uint64_t tile = (uint64_t)blockIdx.x * kMlpWaves + wave;
    float4 x0, x1;
    load_x(tile, x0, x1);
    for (; tile < ntiles; tile += nwaves) {
        bf16x8 A;
        A[0] = (__bf16)(x0.x * scl[0]); A[1] = (__bf16)(x0.y * scl[1]);
        A[2] = (__bf16)(x0.z * scl[2]); A[3] = (__bf16)(x0.w * scl[3]);
        A[4] = (__bf16)(x1.x * scl[4]); A[5] = (__bf16)(x1.y * scl[5]);
        A[6] = (__bf16)(x1.z * scl[6]); A[7] = (__bf16)(x1.w * scl[7]);
        load_x(tile + nwaves, x0, x1);  // the next tile's rows, in flight meanwhile
        // layer 1
        floatx16 d0 = {}, d1 = {};
        d0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, brow(w1s[col], 0), d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, brow(w1s[32 + col], 0), d1, 0, 0, 0);
        store_h(d0, bias1[0], 0);
        store_h(d1, bias1[1], 1);
        wave_sync();
        // layer 2 (its A operands read before the tile is overwritten)
        bf16x8 A2[4];
        for (int ks = 0; ks < 4; ++ks) A2[ks] = brow(ht[col], ks * 16);
        wave_sync();
        d0 = {}; d1 = {};
        for (int ks = 0; ks < 4; ++ks) {
            d0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A2[ks], brow(w2s[col], ks * 16), d0, 0, 0, 0);
            d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A2[ks], brow(w2s[32 + col], ks * 16), d1, 0, 0, 0);
        }
        store_h(d0, bias2[0], 0);
        store_h(d1, bias2[1], 1);
        wave_sync();
        // layer 3: columns 0..2 of D are the outputs
        for (int ks = 0; ks < 4; ++ks) A2[ks] = brow(ht[col], ks * 16);
        floatx16 d3 = {};
        for (int ks = 0; ks < 4; ++ks)
            d3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A2[ks], brow(w3s[col], ks * 16), d3, 0, 0, 0);
        if (col < kOut)
            for (int e = 0; e < 16; ++e) {
                const int i = (e & 3) + 8 * (e >> 2) + 4 * half;
                const uint64_t c = tile * 32 + i;
                if (c < n) out[c * kOut + col] = d3[e] + bias3;
            }
        wave_sync();  // the tile is rewritten by the next iteration
    }
}

// FP32 reference inference: one thread per contact
__global__ __launch_bounds__(256) void k_mlp_f32(const float* __restrict__ W, const float* __restrict__ feat,
                                                 float* __restrict__ out, const uint32_t* d_n, int64_t cap)
{
    __shared__ float w[kMlpParams];
    for (int t = threadIdx.x; t < kMlpParams; t += blockDim.x) w[t] = W[t];
    __syncthreads();
    uint64_t n = d_n ? (uint64_t)min((uint64_t)*d_n, (uint64_t)cap) : (uint64_t)cap;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (uint64_t)gridDim.x * blockDim.x) {
        float x0[kIn], h1[kH];
        for (int k = 0; k < kIn; ++k) x0[k] = feat[c * kIn + k] * w[oScale + k];
        for (int o = 0; o < kH; ++o) {
            float z = w[ob1 + o];
            for (int k = 0; k < kIn; ++k) z += w[oW1 + o * kIn + k] * x0[k];
            h1[o] = silu(z);
        }
        float y[kOut] = {w[ob3], w[ob3 + 1], w[ob3 + 2]};
        for (int o = 0; o < kH; ++o) {
            float z = w[ob2 + o];
            for (int k = 0; k < kH; ++k) z += w[oW2 + o * kH + k] * h1[k];
            float h = silu(z);
            for (int q = 0; q < kOut; ++q) y[q] += w[oW3 + q * kH + o] * h;
        }
        for (int q = 0; q < kOut; ++q) out[c * kOut + q] = y[q];
    }
}

void launch_mlp_infer(const float* W, const float* feat, float* out, const uint32_t* d_n, int64_t cap, bool bf16,
                      hipStream_t s)
{
    if (cap <= 0) return;
    if (bf16) {
        // one round of resident blocks, each wave looping over tiles
        static int resident = 0;
        if (!resident) {
            int dev = 0, per_cu = 0;
            (void)hipGetDevice(&dev);
            hipDeviceProp_t pr;
            (void)hipGetDeviceProperties(&pr, dev);
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mlp_bf16, 64 * kMlpWaves, 0);
            resident = std::max(1, per_cu) * pr.multiProcessorCount;
        }
        int64_t tiles = (cap + 31) / 32;
        int grid = (int)std::min<int64_t>((tiles + kMlpWaves - 1) / kMlpWaves, resident);
        hipLaunchKernelGGL(k_mlp_bf16, dim3(grid), dim3(64 * kMlpWaves), 0, s, W, feat, out, d_n, cap);
    } else {
        int grid = (int)std::min<int64_t>((cap + 255) / 256, 2048);
        hipLaunchKernelGGL(k_mlp_f32, dim3(grid), dim3(256), 0, s, W, feat, out, d_n, cap);
    }
}

// ---------------------------------------------------------------------------
// lambda^0 of the learned start (colour order): world impulse from the
// previous-step impulse plus the network output in the contact frame, projected
// onto {ln >= lo, |lt| <= mu |ln|}
// ---------------------------------------------------------------------------
__global__ void k_learned_lam(DevBuffers b, StepParams p, int64_t cap)
{
    uint32_t nc = b.cnt->n_raw < (uint64_t)cap ? b.cnt->n_raw : (uint32_t)cap;
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc || b.cnt->overflow) return;
    float4 f1 = b.frm1[c], f2 = b.frm2[c], a = b.r0[c], q = b.r2[c];
    // residual form: the output corrects the previous-step impulse in the
    // contact frame (inputs 3-5), so a zero output is the previous-step start
    const float* fc = b.feat + (size_t)c * 12;
    float y0 = fc[3] + b.mlp_out[3 * (size_t)c], y1 = fc[4] + b.mlp_out[3 * (size_t)c + 1],
          y2 = fc[5] + b.mlp_out[3 * (size_t)c + 2];
    float ls = f1.w;
    float ln = y0 * ls;
    float t0 = (y1 * f1.x + y2 * f2.x) * ls, t1 = (y1 * f1.y + y2 * f2.y) * ls, t2 = (y1 * f1.z + y2 * f2.z) * ls;
    if (!(isfinite(ln) && isfinite(t0) && isfinite(t1) && isfinite(t2))) {
        int u = b.envs[(uint32_t)b.pid[__float_as_int(q.w)] / p.id_cap].unit;
        atomicOr(&b.ustats[u].learn_bad, 1u);
        ln = 0.f; t0 = t1 = t2 = 0.f;
    }
    ln = fmaxf(ln, q.y);
    float tn = a.x * t0 + a.y * t1 + a.z * t2;
    t0 -= tn * a.x; t1 -= tn * a.y; t2 -= tn * a.z;
    float lim = p.mu * fabsf(ln);
    float m2 = t0 * t0 + t1 * t1 + t2 * t2;
    if (m2 > lim * lim) {
        float sc = m2 > 0.f ? lim * rsqrtf(m2) : 0.f;
        t0 *= sc; t1 *= sc; t2 *= sc;
    }
    b.lamL[c] = make_float4(ln, t0, t1, t2);
}

void launch_learned_lam(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s)
{
    hipLaunchKernelGGL(k_learned_lam, dim3((unsigned)((z.C + 255) / 256)), dim3(256), 0, s, b, p, z.C);
}

// ---------------------------------------------------------------------------
// training: forward + backward of 0.5 mean ||y - label||^2 in FP32 on MFMA
// (v_mfma_f32_32x32x2f32, FP32 products and sums).  Each wave takes tiles of
// 32 samples; a block's 4 waves take R tiles each (128 R samples, R from 1
// to 4 so that a call fills the 256 CUs where the batch allows).  Per tile:
//   layer 1   Z1[32 x 64] = X[32 x 12] . W1^T          2 N-tiles x 6 K-steps
//   layer 2   Z2 = H1 . W2^T                           2 N-tiles x 32 K-steps
//   layer 3   y = H2 . W3^T (3 outputs: vector ALU)
//   backward  gZ2 = (gy . W3) o silu'(Z2) (vector ALU)
//             gZ1 = (gZ2 . W2) o silu'(Z1)             2 N-tiles x 32 K-steps
//   gradients dW2 += gZ2^T . H1  (64 x 64, K = 32 samples: 2 x 2 tiles x 16)
//             dW1 += gZ1^T . X   (64 x 12 of one 32-wide N-tile: 2 tiles x 16)
//             dW3, the biases and the loss on the vector ALU
// The gradient accumulators stay in registers across a wave's tiles; the
// block's waves add theirs in LDS in a fixed order and write the block's
// partial to part[block][kNP] (loss at part[.][kNP]).
// Operand layouts (A 32x2, B 2x32, D 32x32): A[i][k] -> lane i + 32 k,
// B[k][j] -> lane j + 32 k, D[i][j] -> lane j + 32 ((i / 4) % 2), element
// (i % 4) + 4 (i / 8).
// ---------------------------------------------------------------------------
constexpr int kTrainWaves = 4;
constexpr int kTP = kH + 1;  // LDS pitch of the 64-wide rows

// tiles per wave and blocks of a batch of B samples
__host__ __device__ constexpr int train_tiles(int64_t B)
{
    return B > (int64_t)3 * kTrainWaves * 32 * 256 ? 4 : (B > (int64_t)kTrainWaves * 32 * 256 ? 2 : 1);
}
__host__ __device__ constexpr int64_t train_blocks(int64_t B)
{
    return (B + (int64_t)kTrainWaves * 32 * train_tiles(B) - 1) / ((int64_t)kTrainWaves * 32 * train_tiles(B));
}

__device__ inline floatx16 mfma32(float a, float b, floatx16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(64 * kTrainWaves) void k_mlp_train(const float* __restrict__ W,
                                                                const float* __restrict__ feat,
                                                                const float* __restrict__ label, int64_t B,
                                                                int tiles, float* __restrict__ part)
{
    __shared__ float w[kMlpParams];
    __shared__ float xs[kTrainWaves][32][kIn + 1];
    __shared__ float h1s[kTrainWaves][32][kTP];
    __shared__ float h2s[kTrainWaves][32][kTP];  // H2, then gZ2
    __shared__ float g1s[kTrainWaves][32][kTP];  // gZ1
    __shared__ float gys[kTrainWaves][32][kOut];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, col = lane & 31, half = lane >> 5;
    for (int k = t; k < kMlpParams; k += blockDim.x) w[k] = W[k];
    __syncthreads();
    const float inv_b = 1.0f / (float)B;
    floatx16 dW2[2][2], dW1[2];
    for (int m = 0; m < 2; ++m) {
        dW1[m] = floatx16{};
        for (int n = 0; n < 2; ++n) dW2[m][n] = floatx16{};
    }
    float dW3[kOut] = {0.0f, 0.0f, 0.0f}, db1[2] = {0.0f, 0.0f}, db2[2] = {0.0f, 0.0f}, db3 = 0.0f, loss = 0.0f;
    for (int r = 0; r < tiles; ++r) {
        const int64_t s0 = (((int64_t)blockIdx.x * tiles + r) * kTrainWaves + wave) * 32;
        for (int e = lane; e < 32 * kIn; e += 64) {
            const int i = e / kIn, k = e % kIn;
            const int64_t sm = s0 + i;
            xs[wave][i][k] = sm < B ? feat[sm * kIn + k] * w[oScale + k] : 0.0f;
        }
        __syncthreads();
        // layer 1: Z1 in registers (D layout), H1 into LDS
        floatx16 z1[2], z2[2];
        for (int n = 0; n < 2; ++n) {
            floatx16 acc = {};
            for (int kk = 0; kk < kIn / 2; ++kk) {
                const int k = 2 * kk + half;
                acc = mfma32(xs[wave][col][k], w[oW1 + (n * 32 + col) * kIn + k], acc);
            }
            const float bias = w[ob1 + n * 32 + col];
            for (int e = 0; e < 16; ++e) {
                const int i = (e & 3) + 8 * (e >> 2) + 4 * half;
                const float zz = acc[e] + bias;
                z1[n][e] = zz;
                h1s[wave][i][n * 32 + col] = silu(zz);
            }
        }
        __syncthreads();
        // layer 2: Z2 in registers, H2 into LDS
        for (int n = 0; n < 2; ++n) {
            floatx16 acc = {};
            for (int kk = 0; kk < kH / 2; ++kk) {
                const int k = 2 * kk + half;
                acc = mfma32(h1s[wave][col][k], w[oW2 + (n * 32 + col) * kH + k], acc);
            }
            const float bias = w[ob2 + n * 32 + col];
            for (int e = 0; e < 16; ++e) {
                const int i = (e & 3) + 8 * (e >> 2) + 4 * half;
                const float zz = acc[e] + bias;
                z2[n][e] = zz;
                h2s[wave][i][n * 32 + col] = silu(zz);
            }
        }
        __syncthreads();
        // layer 3 and the error: sample col, the two lane halves summing half
        // of H2's columns each
        {
            float y[kOut] = {0.0f, 0.0f, 0.0f};
            for (int k = half * 32; k < half * 32 + 32; ++k) {
                const float h = h2s[wave][col][k];
                for (int q = 0; q < kOut; ++q) y[q] += w[oW3 + q * kH + k] * h;
            }
            const int64_t sm = s0 + col;
            for (int q = 0; q < kOut; ++q) {
                y[q] += __shfl_xor(y[q], 32);
                const float e = sm < B ? (y[q] + w[ob3 + q]) - label[sm * kOut + q] : 0.0f;
                if (half == 0) {
                    gys[wave][col][q] = e * inv_b;
                    loss += 0.5f * e * e;
                }
            }
        }
        __syncthreads();
        // dW3 (row q, column lane), db3
        for (int i = 0; i < 32; ++i) {
            const float h = h2s[wave][i][lane];
            for (int q = 0; q < kOut; ++q) dW3[q] += gys[wave][i][q] * h;
        }
        if (lane < kOut)
            for (int i = 0; i < 32; ++i) db3 += gys[wave][i][lane];
        __syncthreads();
        // gZ2 = (gy . W3) o silu'(Z2), into h2s
        for (int n = 0; n < 2; ++n)
            for (int e = 0; e < 16; ++e) {
                const int i = (e & 3) + 8 * (e >> 2) + 4 * half, j = n * 32 + col;
                float gh = 0.0f;
                for (int q = 0; q < kOut; ++q) gh += gys[wave][i][q] * w[oW3 + q * kH + j];
                const float g = gh * dsilu(z2[n][e]);
                h2s[wave][i][j] = g;
                db2[n] += g;
            }
        __syncthreads();
        // dW2 += gZ2^T . H1
        for (int m = 0; m < 2; ++m)
            for (int n = 0; n < 2; ++n)
                for (int kk = 0; kk < 16; ++kk) {
                    const int i = 2 * kk + half;
                    dW2[m][n] = mfma32(h2s[wave][i][m * 32 + col], h1s[wave][i][n * 32 + col], dW2[m][n]);
                }
        // gZ1 = (gZ2 . W2) o silu'(Z1), into g1s
        for (int n = 0; n < 2; ++n) {
            floatx16 acc = {};
            for (int kk = 0; kk < kH / 2; ++kk) {
                const int o = 2 * kk + half;
                acc = mfma32(h2s[wave][col][o], w[oW2 + o * kH + n * 32 + col], acc);
            }
            for (int e = 0; e < 16; ++e) {
                const int i = (e & 3) + 8 * (e >> 2) + 4 * half;
                const float g = acc[e] * dsilu(z1[n][e]);
                g1s[wave][i][n * 32 + col] = g;
                db1[n] += g;
            }
        }
        __syncthreads();
        // dW1 += gZ1^T . X (columns col < 12 of one N-tile)
        for (int m = 0; m < 2; ++m)
            for (int kk = 0; kk < 16; ++kk) {
                const int i = 2 * kk + half;
                dW1[m] = mfma32(g1s[wave][i][m * 32 + col], col < kIn ? xs[wave][i][col] : 0.0f, dW1[m]);
            }
        __syncthreads();  // the wave's buffers are rewritten by its next tile
    }
    // the block's partial: the waves add theirs in order
    float* red = &h1s[0][0][0];
    for (int wv = 0; wv < kTrainWaves; ++wv) {
        if (wave == wv) {
            auto put = [&](int idx, float v) { red[idx] = wv == 0 ? v : red[idx] + v; };
            for (int m = 0; m < 2; ++m)
                for (int e = 0; e < 16; ++e) {
                    const int o = m * 32 + (e & 3) + 8 * (e >> 2) + 4 * half;
                    for (int n = 0; n < 2; ++n) put(oW2 + o * kH + n * 32 + col, dW2[m][n][e]);
                    if (col < kIn) put(oW1 + o * kIn + col, dW1[m][e]);
                }
            for (int q = 0; q < kOut; ++q) put(oW3 + q * kH + lane, dW3[q]);
            for (int n = 0; n < 2; ++n) {
                const float v1 = db1[n] + __shfl_xor(db1[n], 32), v2 = db2[n] + __shfl_xor(db2[n], 32);
                if (half == 0) {
                    put(ob1 + n * 32 + col, v1);
                    put(ob2 + n * 32 + col, v2);
                }
            }
            if (lane < kOut) put(ob3 + lane, db3);
            float l = loss;
            for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o);
            if (lane == 0) put(kNP, l * inv_b);
        }
        __syncthreads();
    }
    float* out = part + (size_t)blockIdx.x * (kNP + 1);
    for (int k = t; k <= kNP; k += blockDim.x) out[k] = red[k];
}

// the blocks' partials summed in a fixed order: 64 parameters per block of
// 1024 threads, 16 groups each summing every 16th partial (64 consecutive
// parameters per load: coalesced), then the 16 group sums in group order
constexpr int kRedGroups = 16;
__global__ __launch_bounds__(64 * kRedGroups) void k_grad_reduce(const float* __restrict__ part, int nblocks,
                                                                   float* __restrict__ grad, float* loss)
{
    __shared__ float gs[kRedGroups][64];
    const int j = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int pidx = blockIdx.x * 64 + j;
    float g = 0.0f;
    if (pidx <= kNP)
        for (int b = grp; b < nblocks; b += kRedGroups) g += part[(size_t)b * (kNP + 1) + pidx];
    gs[grp][j] = g;
    __syncthreads();
    if (grp == 0 && pidx <= kNP) {
        float t = 0.0f;
        for (int k = 0; k < kRedGroups; ++k) t += gs[k][j];
        if (pidx < kNP) grad[pidx] = t;
        else if (loss) *loss = t;
    }
}

__global__ void k_adam(float* W, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    float gk = g[k];
    float mk = b1 * m[k] + (1.0f - b1) * gk;
    float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    W[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

int64_t mlp_grad_scratch(int64_t B) { return train_blocks(B) * (int64_t)(kNP + 1); }
int mlp_trainable() { return kNP; }

void launch_mlp_grad(const float* W, const float* feat, const float* label, int64_t B, float* grad, float* loss,
                     float* scratch, hipStream_t s)
{
    const int nb = (int)train_blocks(B);
    hipLaunchKernelGGL(k_mlp_train, dim3(nb), dim3(64 * kTrainWaves), 0, s, W, feat, label, B, train_tiles(B),
                       scratch);
    hipLaunchKernelGGL(k_grad_reduce, dim3((kNP + 1 + 63) / 64), dim3(64 * kRedGroups), 0, s, scratch, nb, grad, loss);
}

void launch_adam(float* W, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps, int t,
                 hipStream_t s)
{
    float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, W, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

}  // namespace trk

// ---------------------------------------------------------------------------
// Loss gradient without allocation: the per-block gradient partials live in a
// file-scope device array of fixed size instead of a caller workspace.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kNoAllocMaxBatch = TR_MLP_NOALLOC_MAX_BATCH;
constexpr int64_t kNoAllocFloats = trk::train_blocks(kNoAllocMaxBatch) * (int64_t)(trk::kNP + 1);
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel: the device address of each GPU's copy comes from
// hipGetSymbolAddress on that GPU.
static __device__ __align__(256) float g_train_scratch[kNoAllocFloats];

std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy (looked up once per device, with the
// device current).  nullptr on failure.
float* train_scratch_ptr(int dev)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_train_scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" int mlp_loss_grad_noalloc(const float* weights, const float* feat, const float* label, int64_t B,
                                     float* grad, float* loss, void* stream)
{
    if (!weights || !feat || !label || !grad || B <= 0) return TR_E_INVAL;
    if (B > kNoAllocMaxBatch) return TR_E_CAPACITY;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TR_E_DEVICE;
    float* scratch = train_scratch_ptr(dev);
    if (!scratch) return TR_E_DEVICE;
    trk::launch_mlp_grad(weights, feat, label, B, grad, loss, scratch, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? TR_OK : TR_E_DEVICE;
}
