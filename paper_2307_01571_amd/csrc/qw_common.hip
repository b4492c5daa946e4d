// qw_common.hip -- precision-independent reduction kernels.  All sums run in
// double in a fixed order, so results are bitwise reproducible run to run.
#include "qw_launch.hpp"

namespace qw {

// Fixed-order workgroup sums (kRedThreads threads): out[q] = sum over
// b < n of x[b stride + q] for q < nq, where thread t adds b = t, t + T,
// t + 2T, ... in turn and a pairwise tree then combines the T threads'
// sums.  red: kRedGroup x kRedThreads doubles of shared memory; out may be
// shared or global memory (written by threads 0 .. nq-1 of each group).
constexpr int kRedThreads = 256;
constexpr int kRedGroup = 8;

__device__ void block_sums(const double* x, long long stride, int n, int nq, double* out, double* red)
{
    const int t = threadIdx.x;
    for (int q0 = 0; q0 < nq; q0 += kRedGroup) {
        const int g = min(kRedGroup, nq - q0);
        double s[kRedGroup];
#pragma unroll
        for (int j = 0; j < kRedGroup; ++j) s[j] = 0.0;
        for (int b = t; b < n; b += kRedThreads) {
            const double* p = x + (size_t)b * stride + q0;
#pragma unroll
            for (int j = 0; j < kRedGroup; ++j)
                if (j < g) s[j] += p[j];
        }
#pragma unroll
        for (int j = 0; j < kRedGroup; ++j) red[j * kRedThreads + t] = s[j];
        __syncthreads();
        for (int w = kRedThreads / 2; w > 0; w >>= 1) {
            if (t < w) {
#pragma unroll
                for (int j = 0; j < kRedGroup; ++j) red[j * kRedThreads + t] += red[j * kRedThreads + t + w];
            }
            __syncthreads();
        }
        if (t < g) out[q0 + t] = red[t * kRedThreads];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kRedThreads) void sum_rows(const double* rownorm, int ny, double* out)
{
    __shared__ double red[kRedGroup * kRedThreads];
    block_sums(rownorm, 1, ny, 1, out, red);
}

// results = [norm, P_n (B), P_n^+ (B), P_n^- (B), P_flip, P_neg] from the
// row sums of |psi|^2 and the per-workgroup column partials
// [window sums (3B), total, flip, positive-energy].  One workgroup of
// kRedThreads threads; acc (at least 3B + 4 doubles) and red are its shared
// scratch.
__device__ void obs_finish_body(const double* rownorm, int ny, const double* partial, int nblocks, int stride,
                                int n_max, double* results, double* acc, double* red)
{
    const int nb = 2 * n_max + 1;
    const int nacc = 3 * nb + 3;
    block_sums(partial, stride, nblocks, nacc, acc, red);
    block_sums(rownorm, 1, ny, 1, acc + nacc, red);
    if (threadIdx.x == 0) {
        const double norm = acc[nacc];
        const double tot = acc[3 * nb];
        results[0] = norm;
        for (int q = 0; q < 3 * nb; ++q) results[1 + q] = acc[q] / tot;
        results[1 + 3 * nb] = acc[3 * nb + 1] / tot;
        results[2 + 3 * nb] = 1.0 - acc[3 * nb + 2] / tot;
    }
}

__global__ __launch_bounds__(kRedThreads) void obs_finish(const double* rownorm, int ny, const double* partial,
                                                          int nblocks, int stride, int n_max, double* results)
{
    __shared__ double acc[128];
    __shared__ double red[kRedGroup * kRedThreads];
    obs_finish_body(rownorm, ny, partial, nblocks, stride, n_max, results, acc, red);
}

// batched: one workgroup per instance
__global__ __launch_bounds__(kRedThreads) void batch_sum_rows(const BatchInst* inst)
{
    __shared__ double red[kRedGroup * kRedThreads];
    const BatchInst& I = inst[blockIdx.x];
    block_sums(I.row.rownorm, 1, I.row.ny, 1, I.scalars, red);
}

__global__ __launch_bounds__(kRedThreads) void batch_obs_finish(const BatchInst* inst, int stride, int n_max)
{
    __shared__ double acc[128];
    __shared__ double red[kRedGroup * kRedThreads];
    const BatchInst& I = inst[blockIdx.x];
    obs_finish_body(I.row.rownorm, I.row.ny, I.col.partial, I.ntile_col, stride, n_max, I.scalars + 8, acc, red);
}

__global__ void clock_set(StepClock* t, double t0, double dt, long long k)
{
    if (threadIdx.x == 0) {
        t->t0 = t0;
        t->dt = dt;
        t->k_base = k;
    }
}

__global__ void clock_advance(StepClock* t, long long steps)
{
    if (threadIdx.x == 0) t->k_base += steps;
}

hipError_t launch_sum_rows(const double* rownorm, int ny, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_rows, dim3(1), dim3(kRedThreads), 0, s, rownorm, ny, out);
    return hipGetLastError();
}

hipError_t launch_obs_finish(const double* rownorm, int ny, const double* partial, int nblocks, int stride,
                             int n_max, double* results, hipStream_t s)
{
    hipLaunchKernelGGL(obs_finish, dim3(1), dim3(kRedThreads), 0, s, rownorm, ny, partial, nblocks, stride, n_max,
                       results);
    return hipGetLastError();
}

hipError_t launch_batch_sum_rows(const BatchInst* inst, int n, hipStream_t s)
{
    hipLaunchKernelGGL(batch_sum_rows, dim3(n), dim3(kRedThreads), 0, s, inst);
    return hipGetLastError();
}

hipError_t launch_batch_obs_finish(const BatchInst* inst, int n, int stride, int n_max, hipStream_t s)
{
    hipLaunchKernelGGL(batch_obs_finish, dim3(n), dim3(kRedThreads), 0, s, inst, stride, n_max);
    return hipGetLastError();
}

hipError_t launch_clock_set(StepClock* t, double t0, double dt, long long k, hipStream_t s)
{
    hipLaunchKernelGGL(clock_set, dim3(1), dim3(64), 0, s, t, t0, dt, k);
    return hipGetLastError();
}

hipError_t launch_clock_advance(StepClock* t, long long steps, hipStream_t s)
{
    hipLaunchKernelGGL(clock_advance, dim3(1), dim3(64), 0, s, t, steps);
    return hipGetLastError();
}

}  // namespace qw
