// qw_common.hip -- precision-independent reduction kernels.  All sums run in
// double in a fixed order, so results are bitwise reproducible run to run.
#include "qw_launch.hpp"

namespace qw {

__global__ void sum_rows(const double* rownorm, int ny, double* out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < ny; ++i) s += rownorm[i];
        out[0] = s;
    }
}

// results = [norm, P_n (B), P_n^+ (B), P_n^- (B), P_flip, P_neg] from the
// row sums of |psi|^2 and the per-workgroup column partials
// [window sums (3B), total, flip, positive-energy].  One workgroup of 128
// threads; acc is its shared scratch.
__device__ void obs_finish_body(const double* rownorm, int ny, const double* partial, int nblocks, int stride,
                                int n_max, double* results, double* acc)
{
    const int nb = 2 * n_max + 1;
    const int nacc = 3 * nb + 3;
    const int i = threadIdx.x;
    if (i < nacc) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * stride + i];
        acc[i] = s;
    }
    __syncthreads();
    if (i == 0) {
        double norm = 0.0;
        for (int y = 0; y < ny; ++y) norm += rownorm[y];
        const double tot = acc[3 * nb];
        results[0] = norm;
        for (int q = 0; q < 3 * nb; ++q) results[1 + q] = acc[q] / tot;
        results[1 + 3 * nb] = acc[3 * nb + 1] / tot;
        results[2 + 3 * nb] = 1.0 - acc[3 * nb + 2] / tot;
    }
}

__global__ __launch_bounds__(128) void obs_finish(const double* rownorm, int ny, const double* partial, int nblocks,
                                                  int stride, int n_max, double* results)
{
    __shared__ double acc[128];
    obs_finish_body(rownorm, ny, partial, nblocks, stride, n_max, results, acc);
}

// batched: one workgroup per instance
__global__ __launch_bounds__(64) void batch_sum_rows(const BatchInst* inst)
{
    const BatchInst& I = inst[blockIdx.x];
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int y = 0; y < I.row.ny; ++y) s += I.row.rownorm[y];
        I.scalars[0] = s;
    }
}

__global__ __launch_bounds__(128) void batch_obs_finish(const BatchInst* inst, int stride, int n_max)
{
    __shared__ double acc[128];
    const BatchInst& I = inst[blockIdx.x];
    obs_finish_body(I.row.rownorm, I.row.ny, I.col.partial, I.ntile_col, stride, n_max, I.scalars + 8, acc);
}

__global__ void batch_set_time(BatchTime* t, double t0, double dt, long long k)
{
    if (threadIdx.x == 0) {
        t->t0 = t0;
        t->dt = dt;
        t->k_base = k;
    }
}

__global__ void batch_advance(BatchTime* t, long long steps)
{
    if (threadIdx.x == 0) t->k_base += steps;
}

hipError_t launch_sum_rows(const double* rownorm, int ny, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_rows, dim3(1), dim3(64), 0, s, rownorm, ny, out);
    return hipGetLastError();
}

hipError_t launch_obs_finish(const double* rownorm, int ny, const double* partial, int nblocks, int stride,
                             int n_max, double* results, hipStream_t s)
{
    hipLaunchKernelGGL(obs_finish, dim3(1), dim3(128), 0, s, rownorm, ny, partial, nblocks, stride, n_max, results);
    return hipGetLastError();
}

hipError_t launch_batch_sum_rows(const BatchInst* inst, int n, hipStream_t s)
{
    hipLaunchKernelGGL(batch_sum_rows, dim3(n), dim3(64), 0, s, inst);
    return hipGetLastError();
}

hipError_t launch_batch_obs_finish(const BatchInst* inst, int n, int stride, int n_max, hipStream_t s)
{
    hipLaunchKernelGGL(batch_obs_finish, dim3(n), dim3(128), 0, s, inst, stride, n_max);
    return hipGetLastError();
}

hipError_t launch_batch_set_time(BatchTime* t, double t0, double dt, long long k, hipStream_t s)
{
    hipLaunchKernelGGL(batch_set_time, dim3(1), dim3(64), 0, s, t, t0, dt, k);
    return hipGetLastError();
}

hipError_t launch_batch_advance(BatchTime* t, long long steps, hipStream_t s)
{
    hipLaunchKernelGGL(batch_advance, dim3(1), dim3(64), 0, s, t, steps);
    return hipGetLastError();
}

}  // namespace qw
