// qw_mlp_kernels.hip -- kernels of the surrogate network (a multilayer
// perceptron with GELU activations): a bfloat16 matrix product on the gfx950
// matrix cores with FP32 accumulation and fused epilogues, plus the small
// elementwise and reduction kernels of training.
//
// Every product is C[m][n] = sum_k A[m][k] B[n][k] with both operands stored
// K-contiguous (row-major A, row-major B = the transpose of the right
// factor), so each lane fetches 8 consecutive bfloat16 (16 bytes) of a row
// for every v_mfma_f32_32x32x16_bf16.  A workgroup of 4 waves owns a 64 x 64
// tile of C, each wave a 32 x 32 block accumulated over K in steps of 16.
// The network's layers, their gradients and the weight gradients are all
// such products: the epilogues store whichever layout (row-major and/or
// transposed, FP32 and/or bfloat16) the next product reads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qw_mlp_launch.hpp"

namespace qwm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr float kInvSqrt2 = 0.70710678118654752440f;
constexpr float kInvSqrt2Pi = 0.39894228040143267794f;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * kInvSqrt2)); }
__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * kInvSqrt2)) + z * kInvSqrt2Pi * expf(-0.5f * z * z);
}

// 16 bytes of a K-contiguous row, zero outside the matrix
__device__ __forceinline__ bf16x8 load_row8(const __bf16* base, int row, int rows, int ld, int k)
{
    if (row >= rows) return bf16x8{};
    return *reinterpret_cast<const bf16x8*>(base + (size_t)row * ld + k);
}

// Output element (i, j) of a 32 x 32 block held by lane l in accumulator r:
// j = l mod 32, i = 8 (r / 4) + 4 (l / 32) + r mod 4.
template <int EPI>
__global__ __launch_bounds__(256) void gemm_nt(GemmArgs g)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int split = EPI == EPI_PARTIAL ? (int)blockIdx.z % g.ksplit : 0;
    const int net = EPI == EPI_PARTIAL ? (int)blockIdx.z / g.ksplit : (int)blockIdx.z;
    const int m0 = blockIdx.x * 64 + (w >> 1) * 32;
    const int n0 = blockIdx.y * 64 + (w & 1) * 32;
    const __bf16* A = g.A + net * g.sA;
    const __bf16* B = g.B + net * g.sB;
    const int kl = 8 * (lane >> 5);
    const int kbeg = EPI == EPI_PARTIAL ? split * g.k_chunk : 0;
    const int kend = EPI == EPI_PARTIAL ? min(g.K, kbeg + g.k_chunk) : g.K;

    // K in chunks of 64 through LDS, double-buffered: the workgroup loads the
    // A and B tiles of a chunk (64 rows x 128 bytes each) row-contiguously,
    // 16 bytes per lane, eight lanes per row, while the waves' products run
    // on the chunk before; each wave then reads its MFMA operands (8 values
    // of a row, as before) from LDS.  The products run in the same order as
    // a direct K loop in steps of 16.
    __shared__ __bf16 sA[2][64][72], sB[2][64][72];  // row stride 144 bytes
    const int lr = threadIdx.x >> 3, ls = (threadIdx.x & 7) * 8;
    const int mt = blockIdx.x * 64, nt = blockIdx.y * 64;
    bf16x8 ga[2], gb[2];
    auto gload = [&](int kc) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bool kin = kc + ls < kend;
            ga[h] = kin ? load_row8(A, mt + lr + 32 * h, g.M, g.lda, kc + ls) : bf16x8{};
            gb[h] = kin ? load_row8(B, nt + lr + 32 * h, g.N, g.ldb, kc + ls) : bf16x8{};
        }
    };
    f32x16 acc = {};
    const int wa = (w >> 1) * 32 + (lane & 31), wb = (w & 1) * 32 + (lane & 31);
    int buf = 0;
    if (kbeg < kend) gload(kbeg);
    for (int kc = kbeg; kc < kend; kc += 64) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            *reinterpret_cast<bf16x8*>(&sA[buf][lr + 32 * h][ls]) = ga[h];
            *reinterpret_cast<bf16x8*>(&sB[buf][lr + 32 * h][ls]) = gb[h];
        }
        __syncthreads();
        if (kc + 64 < kend) gload(kc + 64);
        const int steps = min(4, (kend - kc) / 16);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (u < steps) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sA[buf][wa][16 * u + kl]);
                const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sB[buf][wb][16 * u + kl]);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
            }
        }
        buf ^= 1;
    }

    const int n = n0 + (lane & 31);
    const int mb = m0 + 4 * (lane >> 5);
    const bool ncol = n < g.N;
    float* Cf = g.Cf ? g.Cf + net * g.sCf : nullptr;
    __bf16* Cb = g.Cb ? g.Cb + net * g.sCb : nullptr;
    __bf16* Ct = g.Ct ? g.Ct + net * g.sCt : nullptr;
    const float bias = (g.bias && ncol) ? g.bias[net * g.sbias + n] : 0.0f;
    float sq = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float out[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int m = mb + 8 * q + s;
            const bool in = ncol && m < g.M;
            const float c = acc[4 * q + s];
            float o = 0.0f;
            if constexpr (EPI == EPI_F32) {
                if (in) Cf[(size_t)m * g.ldcf + n] = c;
            } else if constexpr (EPI == EPI_PARTIAL) {
                if (in) g.Cp[net * g.sCp_net + ((size_t)split * g.M + m) * g.N + n] = c;
            } else if constexpr (EPI == EPI_HIDDEN) {
                const float z = c + bias;
                if (in && Cf) Cf[(size_t)m * g.ldcf + n] = z;
                o = in ? gelu(z) : 0.0f;
            } else if constexpr (EPI == EPI_OUT) {
                const float y = c + bias;
                if (in) Cf[(size_t)m * g.ldcf + n] = y;
                if (g.T) {
                    const float d = in ? y - g.T[(size_t)m * g.ldt + n] : 0.0f;
                    sq += d * d;
                    o = g.gscale * d;
                }
            } else if constexpr (EPI == EPI_GELU_BWD) {
                o = in ? c * gelu_grad(g.Z[net * g.sZ + (size_t)m * g.ldz + n]) : 0.0f;
            }
            out[s] = o;
            if (Cb && m < g.Mpad && n < g.ldcb) Cb[(size_t)m * g.ldcb + n] = (__bf16)o;
        }
        // transposed copy: the 4 consecutive rows of this lane are contiguous
        const int m = mb + 8 * q;
        if (Ct && n < g.nct && m < g.Mpad) {
            bf16x4 v = {(__bf16)out[0], (__bf16)out[1], (__bf16)out[2], (__bf16)out[3]};
            *reinterpret_cast<bf16x4*>(Ct + (size_t)n * g.ldct + m) = v;
        }
    }
    if constexpr (EPI == EPI_OUT) {
        if (g.loss_part) {
            __shared__ float red[256];
            red[threadIdx.x] = sq;
            __syncthreads();
            for (int s = 128; s > 0; s >>= 1) {
                if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
                __syncthreads();
            }
            if (threadIdx.x == 0) g.loss_part[net * g.sLoss + blockIdx.x * gridDim.y + blockIdx.y] = red[0];
        }
    }
}

// normalised input, zero-padded to kInPad columns and Mpad rows, in both layouts
__global__ __launch_bounds__(256) void prep_input(const float* x, int B, int n_in, int Mpad, const float* shift,
                                                  const float* scale, __bf16* xb, __bf16* xt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Mpad * kInPad) return;
    const int m = i / kInPad, c = i - m * kInPad;
    float v = 0.0f;
    if (m < B && c < n_in) v = (x[(size_t)m * n_in + c] - shift[c]) * scale[c];
    const __bf16 h = (__bf16)v;
    xb[i] = h;
    xt[(size_t)c * Mpad + m] = h;
}

// out[net][r] = sum over m < M of in[net][r][m] (bfloat16 rows, FP32 sum, fixed order)
__global__ __launch_bounds__(256) void row_sums(const __bf16* in, long long s_in, int ld, int M, float* out,
                                                long long s_out)
{
    __shared__ float red[256];
    const int r = blockIdx.x, net = blockIdx.y;
    const __bf16* row = in + net * s_in + (size_t)r * ld;
    float s = 0.0f;
    for (int m = threadIdx.x; m < M; m += 256) s += (float)row[m];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[net * s_out + r] = red[0];
}

// Adam on the FP32 master parameters of every net (update = 1), or only the
// refresh of the bfloat16 copies (update = 0); the copies go to W[out][in_pad]
// and Wt[in][out_pad] of each layer.
__global__ __launch_bounds__(256) void adam(AdamArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int net = blockIdx.y;
    if (i >= a.n) return;
    const size_t at = (size_t)net * a.n + i;
    float p = a.p[at];
    if (a.update) {
        const float g = a.g[at];
        const float m = a.b1 * a.m[at] + (1.0f - a.b1) * g;
        const float v = a.b2 * a.v[at] + (1.0f - a.b2) * g * g;
        a.m[at] = m;
        a.v[at] = v;
        p -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
        a.p[at] = p;
    }
    for (int l = 0; l < a.n_layers; ++l) {
        const LayerMap& L = a.layer[l];
        const int o = i - L.p_off;
        if (o >= 0 && o < L.n_out * L.n_in) {
            const int r = o / L.n_in, c = o - r * L.n_in;
            const __bf16 h = (__bf16)p;
            a.wb[net * a.s_wb + L.wb_off + (size_t)r * L.ld_wb + c] = h;
            a.wt[net * a.s_wt + L.wt_off + (size_t)c * L.ld_wt + r] = h;
            break;
        }
    }
}

__global__ __launch_bounds__(256) void fill_zero_u32(uint32_t* p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// loss[net] = sum of the per-workgroup squared errors / (B n_out)
__global__ void loss_finish(const float* part, long long s_part, int n_part, float inv_count, float* loss)
{
    if (threadIdx.x == 0) {
        const int net = blockIdx.x;
        float s = 0.0f;
        for (int i = 0; i < n_part; ++i) s += part[net * s_part + i];
        loss[net] = s * inv_count;
    }
}

// ensemble mean and spread of the mapped outputs y oscale + oshift: the
// spread is the largest over the outputs of the standard deviation across
// the nets times the output's weight swt
__global__ __launch_bounds__(256) void ensemble(const float* y, long long s_net, int ld, int B, int n_out, int nets,
                                                const float* oshift, const float* oscale, const float* swt,
                                                float* mean, float* spread)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= B) return;
    float worst = 0.0f;
    for (int o = 0; o < n_out; ++o) {
        const float sh = oshift[o], sc = oscale[o];
        float s = 0.0f;
        for (int k = 0; k < nets; ++k) s += y[k * s_net + (size_t)m * ld + o] * sc + sh;
        const float mu = s / nets;
        float q = 0.0f;
        for (int k = 0; k < nets; ++k) {
            const float d = y[k * s_net + (size_t)m * ld + o] * sc + sh - mu;
            q += d * d;
        }
        mean[(size_t)m * n_out + o] = mu;
        const float sd = (nets > 1 ? sqrtf(q / (nets - 1)) : 0.0f) * swt[o];
        worst = sd > worst ? sd : worst;
    }
    spread[m] = worst;
}

// ---------------------------------------------------------------------------
hipError_t launch_gemm(int epi, const GemmArgs& g, int nets, int ncover, hipStream_t s)
{
    const dim3 grid((g.Mpad + 63) / 64, (ncover + 63) / 64, nets), block(256);
    switch (epi) {
    case EPI_F32: hipLaunchKernelGGL(gemm_nt<EPI_F32>, grid, block, 0, s, g); break;
    case EPI_HIDDEN: hipLaunchKernelGGL(gemm_nt<EPI_HIDDEN>, grid, block, 0, s, g); break;
    case EPI_OUT: hipLaunchKernelGGL(gemm_nt<EPI_OUT>, grid, block, 0, s, g); break;
    case EPI_GELU_BWD: hipLaunchKernelGGL(gemm_nt<EPI_GELU_BWD>, grid, block, 0, s, g); break;
    case EPI_PARTIAL: {
        if (g.ksplit < 1 || g.k_chunk < 16 || g.k_chunk % 16 != 0) return hipErrorInvalidValue;
        const dim3 gridp(grid.x, grid.y, nets * g.ksplit);
        hipLaunchKernelGGL(gemm_nt<EPI_PARTIAL>, gridp, block, 0, s, g);
        break;
    }
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// fixed-order sum of the split-K parts
__global__ __launch_bounds__(256) void ksum(const float* part, long long s_part_net, int ksplit, int M, int N,
                                            float* C, long long s_c, int ldc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int net = blockIdx.y;
    if (i >= M * N) return;
    const float* p = part + net * s_part_net + i;
    float acc = 0.0f;
    for (int sp = 0; sp < ksplit; ++sp) acc += p[(size_t)sp * M * N];
    const int m = i / N, n = i - m * N;
    C[net * s_c + (size_t)m * ldc + n] = acc;
}

// ksum and row_sums in one launch: workgroups [0, nk) of each net do the
// split-K sum, the next `rows` workgroups the row sums (same arithmetic)
__global__ __launch_bounds__(256) void ksum_rows(const float* part, long long s_part_net, int ksplit, int M, int N,
                                                 float* C, long long s_c, int ldc, int nk, const __bf16* in,
                                                 long long s_in, int ld, int Mrows, float* out, long long s_out)
{
    __shared__ float red[256];
    const int net = blockIdx.y;
    if ((int)blockIdx.x < nk) {
        const int i = blockIdx.x * blockDim.x + threadIdx.x;
        if (i >= M * N) return;
        const float* p = part + net * s_part_net + i;
        float acc = 0.0f;
        for (int sp = 0; sp < ksplit; ++sp) acc += p[(size_t)sp * M * N];
        const int m = i / N, n = i - m * N;
        C[net * s_c + (size_t)m * ldc + n] = acc;
        return;
    }
    const int r = blockIdx.x - nk;
    const __bf16* row = in + net * s_in + (size_t)r * ld;
    float sum = 0.0f;
    for (int m = threadIdx.x; m < Mrows; m += 256) sum += (float)row[m];
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[net * s_out + r] = red[0];
}

hipError_t launch_ksum_rows(const float* part, long long s_part_net, int ksplit, int M, int N, float* C,
                            long long s_c, int ldc, const __bf16* in, long long s_in, int ld, int rows, int Mrows,
                            float* out, long long s_out, int nets, hipStream_t s)
{
    const int nk = (M * N + 255) / 256;
    hipLaunchKernelGGL(ksum_rows, dim3(nk + rows, nets), dim3(256), 0, s, part, s_part_net, ksplit, M, N, C, s_c, ldc,
                       nk, in, s_in, ld, Mrows, out, s_out);
    return hipGetLastError();
}

hipError_t launch_ksum(const float* part, long long s_part_net, int ksplit, int M, int N, float* C, long long s_c,
                       int ldc, int nets, hipStream_t s)
{
    hipLaunchKernelGGL(ksum, dim3((M * N + 255) / 256, nets), dim3(256), 0, s, part, s_part_net, ksplit, M, N, C, s_c,
                       ldc);
    return hipGetLastError();
}

hipError_t launch_prep_input(const float* x, int B, int n_in, int Mpad, const float* shift, const float* scale,
                             __bf16* xb, __bf16* xt, hipStream_t s)
{
    const int n = Mpad * kInPad;
    hipLaunchKernelGGL(prep_input, dim3((n + 255) / 256), dim3(256), 0, s, x, B, n_in, Mpad, shift, scale, xb, xt);
    return hipGetLastError();
}

hipError_t launch_row_sums(const __bf16* in, long long s_in, int ld, int rows, int M, float* out, long long s_out,
                           int nets, hipStream_t s)
{
    hipLaunchKernelGGL(row_sums, dim3(rows, nets), dim3(256), 0, s, in, s_in, ld, M, out, s_out);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs& a, int nets, hipStream_t s)
{
    hipLaunchKernelGGL(adam, dim3((a.n + 255) / 256, nets), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<uint32_t*>(p), n);
    return hipGetLastError();
}

hipError_t launch_loss_finish(const float* part, long long s_part, int n_part, float inv_count, float* loss,
                              int nets, hipStream_t s)
{
    hipLaunchKernelGGL(loss_finish, dim3(nets), dim3(64), 0, s, part, s_part, n_part, inv_count, loss);
    return hipGetLastError();
}

hipError_t launch_ensemble(const float* y, long long s_net, int ld, int B, int n_out, int nets, const float* oshift,
                           const float* oscale, const float* swt, float* mean, float* spread, hipStream_t s)
{
    hipLaunchKernelGGL(ensemble, dim3((B + 255) / 256), dim3(256), 0, s, y, s_net, ld, B, n_out, nets, oshift, oscale,
                       swt, mean, spread);
    return hipGetLastError();
}

}  // namespace qwm
