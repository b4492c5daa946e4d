// qw_mlp_launch.hpp -- interface between the surrogate network's host engine
// (qw_mlp.cpp) and its kernels (qw_mlp_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qwm {

constexpr int kInPad = 16;   // input features and outputs are padded to one K step of the product
constexpr int kMaxLayers = 17;

enum { EPI_F32 = 0, EPI_HIDDEN = 1, EPI_OUT = 2, EPI_GELU_BWD = 3, EPI_PARTIAL = 4 };

// C[m][n] = sum_k A[m][k] B[n][k]; operands bfloat16, K-contiguous, K a
// multiple of 16, leading dimensions multiples of 8; per-net strides in
// elements (blockIdx.z = net).  Epilogues:
//   EPI_F32       Cf = C
//   EPI_HIDDEN    z = C + bias -> Cf (if set); h = gelu(z) -> Cb, Ct (if set)
//   EPI_OUT       y = C + bias -> Cf; with T: d = y - T, g = gscale d -> Cb, Ct,
//                 per-workgroup sums of d^2 -> loss_part
//   EPI_GELU_BWD  g = C gelu'(Z) -> Cb, Ct
//   EPI_PARTIAL   split-K part: blockIdx.z = net ksplit + split sums k in
//                 [split k_chunk, (split + 1) k_chunk) into the dense M x N
//                 slice Cp + net sCp_net + split M N (summed by launch_ksum)
// Cb rows [M, Mpad) and columns [N, ldcb) are written as zeros, likewise
// Ct rows [N, nct) and columns [M, Mpad): the padding the next product reads.
struct GemmArgs {
    const __bf16* A;
    long long sA;
    int lda;
    const __bf16* B;
    long long sB;
    int ldb;
    int M, N, K, Mpad;
    const float* bias;
    long long sbias;
    float* Cf;
    long long sCf;
    int ldcf;
    __bf16* Cb;
    long long sCb;
    int ldcb;
    __bf16* Ct;
    long long sCt;
    int ldct, nct;
    const float* Z;
    long long sZ;
    int ldz;
    const float* T;
    int ldt;
    float* loss_part;
    long long sLoss;
    float gscale;
    int ksplit, k_chunk;  // EPI_PARTIAL only
    float* Cp;
    long long sCp_net;
};

// where one layer's weights sit in the flat FP32 parameters and in the
// bfloat16 copies
struct LayerMap {
    int p_off, n_out, n_in;
    int wb_off, ld_wb;  // W[out][ld_wb]
    int wt_off, ld_wt;  // Wt[in][ld_wt]
};

struct AdamArgs {
    float* p;
    float* m;
    float* v;
    const float* g;
    int n;  // parameters per net
    int update;
    float lr, b1, b2, eps, c1, c2;  // c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t)
    __bf16* wb;
    __bf16* wt;
    long long s_wb, s_wt;
    int n_layers;
    LayerMap layer[kMaxLayers];
};

hipError_t launch_gemm(int epi, const GemmArgs& g, int nets, int ncover, hipStream_t s);
// C[net][m][ldc] = sum over split (in order) of part[net][split][m][N]
hipError_t launch_ksum(const float* part, long long s_part_net, int ksplit, int M, int N, float* C, long long s_c,
                       int ldc, int nets, hipStream_t s);
// launch_ksum and launch_row_sums(in, s_in, ld, rows, Mrows, out, s_out) as one launch
hipError_t launch_ksum_rows(const float* part, long long s_part_net, int ksplit, int M, int N, float* C,
                            long long s_c, int ldc, const __bf16* in, long long s_in, int ld, int rows, int Mrows,
                            float* out, long long s_out, int nets, hipStream_t s);
hipError_t launch_prep_input(const float* x, int B, int n_in, int Mpad, const float* shift, const float* scale,
                             __bf16* xb, __bf16* xt, hipStream_t s);
hipError_t launch_row_sums(const __bf16* in, long long s_in, int ld, int rows, int M, float* out, long long s_out,
                           int nets, hipStream_t s);
hipError_t launch_adam(const AdamArgs& a, int nets, hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_loss_finish(const float* part, long long s_part, int n_part, float inv_count, float* loss,
                              int nets, hipStream_t s);
hipError_t launch_ensemble(const float* y, long long s_net, int ld, int B, int n_out, int nets, const float* oshift,
                           const float* oscale, const float* swt, float* mean, float* spread, hipStream_t s);

}  // namespace qwm
