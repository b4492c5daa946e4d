// qw_batch.inl -- batched form of the split-operator passes: one launch per
// pass advances every instance of a batch, whatever its grid.  Included by
// qw_kernels_f32.hip and qw_kernels_f64.hip after qw_kernels.inl.
//
// Every work item is one tile of one instance: 256 threads over RPW rows
// (row pass) or TX columns (column pass) of a line length N, with
// RPW = TX = 256 / (2 N / E).  With E elements per lane a tile always covers
// 128 E cells, so the items of all instances cost the same and a launch
// balances itself.  The launch is persistent when asked: fewer workgroups
// than items, each walking its own strided share of the list.  The step loop
// kernel runs many middle steps in one cooperative launch, with grid-wide
// barriers between the column and row phases.
//
// The transform of each length comes in schedule variants (the same E,
// other radix orders); the hot modes (ROW_MID, COL_PROP) take the variant
// the batch's autotuner picked per length, the others the default plan.
#pragma once
#include "qw_kernels.inl"
#include "qw_batch_loop.hpp"

// Row passes at three workgroups per CU: the middle row pass then fits 168
// VGPRs with a 20-byte spill and runs faster than at two workgroups with
// 172 (96 instances of 256^2 to 1024^2: FP32 724.6 -> 632.5 us per launch,
// FP64 1655 -> 1392 us).
// The step-loop kernels, which hold both passes' bodies, stay at two: at
// three they spill 124-152 bytes per lane and run slower (one workgroup per
// instance, 512 instances of 64^2: 41.4 -> 49.8 us per step).
#ifndef QW_WPE_BATCH_ROW
#define QW_WPE_BATCH_ROW 3
#endif
#ifndef QW_WPE_BATCH_COL
#define QW_WPE_BATCH_COL 2
#endif

namespace qw {

// Schedule variants per precision: X(lg, variant, radices...).  Variant 0 is
// the single-instance plan of that length, so a batch on its defaults does
// the same arithmetic as the single-instance kernels.  The including file
// names its precision's list as QW_BATCH_VARIANTS.
#define QW_BATCH_VARIANTS_float(X)                                                      \
    X(6, 0, 16, 4) X(6, 1, 4, 16) X(6, 2, 8, 8)                                         \
    X(7, 0, 16, 8) X(7, 1, 8, 16) X(7, 2, 4, 4, 8)                                      \
    X(8, 0, 16, 16) X(8, 1, 4, 4, 16) X(8, 2, 8, 8, 4)                                  \
    X(9, 0, 16, 8, 4) X(9, 1, 8, 8, 8) X(9, 2, 4, 8, 16) X(9, 3, 16, 16, 2)             \
    X(10, 0, 16, 16, 4) X(10, 1, 16, 8, 8) X(10, 2, 4, 16, 16) X(10, 3, 8, 8, 16)       \
    X(11, 0, 16, 16, 8) X(11, 1, 8, 16, 16) X(11, 2, 16, 8, 16)

#define QW_BATCH_VARIANTS_double(X)                                                     \
    X(6, 0, 8, 8) X(6, 1, 4, 4, 4)                                                      \
    X(7, 0, 8, 4, 4) X(7, 1, 4, 4, 8) X(7, 2, 4, 8, 4)                                  \
    X(8, 0, 8, 8, 4) X(8, 1, 4, 8, 8) X(8, 2, 8, 4, 8)                                  \
    X(9, 0, 8, 8, 8) X(9, 1, 8, 4, 4, 4)                                                \
    X(10, 0, 8, 8, 4, 4) X(10, 1, 4, 4, 8, 8) X(10, 2, 8, 4, 8, 4)

template <typename T>
struct batch_family;
template <>
struct batch_family<float> {
    static constexpr int E = 16, lg_min = 6, lg_max = 11;
};
template <>
struct batch_family<double> {
    static constexpr int E = 8, lg_min = 6, lg_max = 10;
};

// tile geometry of the batched kernels for length N
template <typename T, int N>
struct bshape {
    static constexpr int E = batch_family<T>::E;
    static constexpr int NT = N / E;
    static constexpr int L = 2 * NT;
    static constexpr int LINES = kBatchThreads / L;  // rows (RPW) or columns (TX) per tile
    static constexpr int LLR = lds_len<T, N>::value + QW_LDS_EXTRA_ROW;
    static constexpr int LLC = lds_len<T, N>::value + QW_LDS_EXTRA_COL;
    static constexpr int lds_row = LINES * 2 * LLR;
    static constexpr int lds_col = LINES * 2 * LLC;
    static_assert(L <= kBatchThreads, "a line must fit one batched workgroup");
};

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <typename T, int LG>
constexpr int batch_lds_row()
{
    if constexpr (LG < batch_family<T>::lg_min) return 0;
    else return cmax(bshape<T, (1 << LG)>::lds_row, batch_lds_row<T, LG - 1>());
}
template <typename T, int LG>
constexpr int batch_lds_col()
{
    if constexpr (LG < batch_family<T>::lg_min) return 0;
    else return cmax(bshape<T, (1 << LG)>::lds_col, batch_lds_col<T, LG - 1>());
}

constexpr bool batch_hot_row(int mode) { return mode == ROW_MID; }
constexpr bool batch_hot_col(int mode) { return mode == COL_PROP; }

// dispatch one tile to the body of its length and schedule variant
template <typename T, int MODE>
__device__ __forceinline__ void batch_row_tile(int lg, int var, const RowArgs& a, int tile, cx<T>* lds, int tid)
{
    switch (lg * kBatchMaxVariants + var) {
#define QW_X(LG, V, ...)                                                                                   \
    case LG * kBatchMaxVariants + V:                                                                      \
        if constexpr (V == 0 || batch_hot_row(MODE)) {                                                    \
            using B = bshape<T, (1 << LG)>;                                                               \
            row_tile<T, (1 << LG), B::E, sched<__VA_ARGS__>, B::LINES, B::LLR, MODE>(a, tile, lds, tid);        \
        }                                                                                                  \
        return;
        QW_BATCH_VARIANTS(QW_X)
#undef QW_X
    default: return;
    }
}

template <typename T, int MODE>
__device__ __forceinline__ void batch_col_tile(int lg, int var, const ColArgs& a, int tile, cx<T>* lds, int tid)
{
    switch (lg * kBatchMaxVariants + var) {
#define QW_X(LG, V, ...)                                                                                   \
    case LG * kBatchMaxVariants + V:                                                                      \
        if constexpr (V == 0 || batch_hot_col(MODE)) {                                                    \
            using B = bshape<T, (1 << LG)>;                                                               \
            col_tile<T, (1 << LG), B::E, sched<__VA_ARGS__>, B::LINES, B::LLC, MODE>(a, tile, lds, tid);        \
        }                                                                                                  \
        return;
        QW_BATCH_VARIANTS(QW_X)
#undef QW_X
    default: return;
    }
}

// The items are split into 8 contiguous ranges, one per XCD (workgroups are
// dealt round-robin to the XCDs); the workgroups of one XCD stride through
// its range, so tiles that share cache lines meet in the same L2.
struct item_range {
    int it, end, step;
};
__device__ __forceinline__ item_range batch_items(int n_items)
{
    if ((gridDim.x & 7) != 0) return {(int)blockIdx.x, n_items, (int)gridDim.x};
    const int per = gridDim.x >> 3, xcd = blockIdx.x & 7, w = blockIdx.x >> 3;
    const int chunk = (n_items + 7) >> 3;
    const int lo = xcd * chunk;
    const int hi = lo + chunk < n_items ? lo + chunk : n_items;
    return {lo + w, hi, per};
}

template <typename T, int MODE>
__device__ __forceinline__ void batch_row_item(const BatchLaunch& b, int it, cx<T>* lds, int tid)
{
    const uint32_t e = b.items[it];
    const BatchInst& I = b.inst[e >> 16];
    RowArgs a = I.row;
    a.src = b.src + I.off;
    a.dst = b.dst + I.off;
    if constexpr (MODE == ROW_FIRST || MODE == ROW_MID || MODE == ROW_LAST) {
        a.t0 = b.time->t0;
        a.dt = b.time->dt;
        a.k = (b.use_counter ? b.time->k_base : 0) + b.j;
        a.tau_frac = b.tau_frac;
    }
    int var = 0;
    if constexpr (batch_hot_row(MODE)) {
        a.twx = I.tw_row;
        var = I.row_var;
    }
    batch_row_tile<T, MODE>(I.lgx, var, a, (int)(e & 0xffffu), lds, tid);
}

template <typename T, int MODE>
__device__ __forceinline__ void batch_col_item(const BatchLaunch& b, int it, cx<T>* lds, int tid)
{
    const uint32_t e = b.items[it];
    const BatchInst& I = b.inst[e >> 16];
    ColArgs a = I.col;
    a.psi = b.src + I.off;
    int var = 0;
    if constexpr (batch_hot_col(MODE)) {
        a.twy = I.tw_col;
        var = I.col_var;
    }
    batch_col_tile<T, MODE>(I.lgy, var, a, (int)(e & 0xffffu), lds, tid);
}

// PERSIST = false: one item per workgroup (grid = items rounded up to a
// multiple of 8).  PERSIST = true: any grid, each workgroup loops.
template <typename T, int MODE, bool PERSIST>
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(QW_WPE_BATCH_ROW))) void batch_row(
    BatchLaunch b)
{
    __shared__ cx<T> lds[batch_lds_row<T, batch_family<T>::lg_max>()];
    const item_range r = batch_items(b.n_items);
    if constexpr (!PERSIST) {
        if (r.it < r.end) batch_row_item<T, MODE>(b, r.it, lds, threadIdx.x);
    } else {
        for (int it = r.it; it < r.end; it += r.step) {
            // an opaque thread index keeps the lane-dependent addresses of
            // the passes inside the loop instead of in registers across it
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            batch_row_item<T, MODE>(b, it, lds, tid);
            __syncthreads();  // LDS is reused by the next item
        }
    }
}

template <typename T, int MODE, bool PERSIST>
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(QW_WPE_BATCH_COL))) void batch_col(
    BatchLaunch b)
{
    __shared__ cx<T> lds[batch_lds_col<T, batch_family<T>::lg_max>()];
    const item_range r = batch_items(b.n_items);
    if constexpr (!PERSIST) {
        if (r.it < r.end) batch_col_item<T, MODE>(b, r.it, lds, threadIdx.x);
    } else {
        for (int it = r.it; it < r.end; it += r.step) {
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            batch_col_item<T, MODE>(b, it, lds, tid);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// persistent step loop: `steps` middle steps (column pass, then middle row
// pass) in one cooperative launch, a grid-wide barrier between the phases
// ---------------------------------------------------------------------------
#ifndef QW_WPE_BATCH_LOOP
#define QW_WPE_BATCH_LOOP 2
#endif

__device__ __forceinline__ unsigned sync_load(unsigned* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// thread 0: wait until *p >= want; false once the wait runs past spin_ticks
// or another workgroup has recorded a failure (then records one itself)
__device__ __forceinline__ bool sync_wait(unsigned* p, unsigned want, BatchSync* s, unsigned long long spin_ticks)
{
    const unsigned long long start = (unsigned long long)wall_clock64();
    while (sync_load(p) < want) {
        if (sync_load(&s->failed.v) != 0u || (unsigned long long)wall_clock64() - start > spin_ticks) {
            __hip_atomic_store(&s->failed.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    return true;
}

// Grid-wide barrier number k (1, 2, ...).  The launch is cooperative, so
// every workgroup is resident.  Arrivals are counted per group of
// gridDim.x / 8 workgroups; the last arrival of a group counts the group in
// globally, waits for all 8 and then lets its group pass, so each polled
// word has at most one group's workgroups on it (one counter polled by
// every workgroup, with every wave writing back L2, cost 135 against 46 us
// per step of eight 256^2 instances).  Ordering, all at agent scope: a
// workgroup's stores are complete (every wave waits for its own) before
// thread 0 arrives with a release; the group's last arrival acquires them
// with that same read-modify-write and releases them with its global
// arrival; the last group's release is acquired by each group's last
// arrival before it releases its group, and each workgroup acquires after
// its wait, so the next phase sees what the previous one wrote from every
// XCD.  Every wait is bounded by
// spin_ticks of the constant-rate wall clock: past it, or once another
// workgroup has recorded a failure, the workgroup records the failure
// (sticky, read by the host) and the loop ends.
__device__ __forceinline__ bool loop_barrier(BatchSync* s, unsigned k, unsigned long long spin_ticks, int* flag)
{
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached L2
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned g = blockIdx.x & 7u, per = gridDim.x >> 3;
        const unsigned n = __hip_atomic_fetch_add(&s->group_arrived[g].v, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (n == k * per) {
            __hip_atomic_fetch_add(&s->arrived.v, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            ok = sync_wait(&s->arrived.v, 8u * k, s, spin_ticks);
            if (ok) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(&s->group_pass[g].v, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            ok = sync_wait(&s->group_pass[g].v, k, s, spin_ticks);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the CU's L1 and the XCD's L2 drop stale lines
        *flag = ok;
    }
    __syncthreads();
    return *flag != 0;
}

// Every workgroup leaves through here; the last one to leave zeroes the
// counters for the next launch on the stream.  A workgroup counts itself out
// only after its last wait, so no wait can see the reset.
__device__ __forceinline__ void loop_depart(BatchSync* s)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned d = __hip_atomic_fetch_add(&s->departed.v, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (d + 1 == gridDim.x) {
            __hip_atomic_store(&s->arrived.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int g = 0; g < 8; ++g) {
                __hip_atomic_store(&s->group_arrived[g].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&s->group_pass[g].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __hip_atomic_store(&s->departed.v, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Middle steps j0 .. j0 + steps - 1 (rows.j = j0, absolute step indices):
// per step every workgroup walks its share of the column items, meets the
// others at the barrier, walks its share of the row items, and meets them
// again before the next step.  The items, their order within a phase and
// the tile bodies are those of the one-launch-per-pass kernels, so the
// results are the same bit for bit.
template <typename T>
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(QW_WPE_BATCH_LOOP))) void batch_loop(
    BatchLaunch cols, BatchLaunch rows, int steps, BatchSync* sync, unsigned long long spin_ticks)
{
    constexpr int LG = batch_family<T>::lg_max;
    __shared__ cx<T> lds[cmax(batch_lds_row<T, LG>(), batch_lds_col<T, LG>())];
    __shared__ int flag;
    const item_range cr = batch_items(cols.n_items), rr = batch_items(rows.n_items);
    const int j0 = rows.j;
    unsigned k = 0;
    for (int s = 0; s < steps; ++s) {
        for (int it = cr.it; it < cr.end; it += cr.step) {
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            batch_col_item<T, COL_PROP>(cols, it, lds, tid);
            __syncthreads();
        }
        if (!loop_barrier(sync, ++k, spin_ticks, &flag)) break;
        BatchLaunch r = rows;
        r.j = j0 + s;
        for (int it = rr.it; it < rr.end; it += rr.step) {
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            batch_row_item<T, ROW_MID>(r, it, lds, tid);
            __syncthreads();
        }
        if (s + 1 == steps) break;
        if (!loop_barrier(sync, ++k, spin_ticks, &flag)) break;
    }
    loop_depart(sync);
}

// One workgroup per instance: middle steps j0 .. j0 + steps - 1 of instance
// blockIdx.x, its column items, then its row items, per step.  An
// instance's data dependences stay inside its workgroup, so the barrier
// after each item (workgroup-scope release and acquire) is the only one and
// the launch needs no co-residency; the items, their order and the tile
// bodies are those of the per-pass kernels, so the results are the same bit
// for bit.  ranges[i] = (first row item, end, first column item, end).
template <typename T>
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(QW_WPE_BATCH_LOOP))) void
batch_inst_loop(BatchLaunch cols, BatchLaunch rows, const BatchInstItems* ranges, int steps)
{
    constexpr int LG = batch_family<T>::lg_max;
    __shared__ cx<T> lds[cmax(batch_lds_row<T, LG>(), batch_lds_col<T, LG>())];
    const BatchInstItems q = ranges[blockIdx.x];
    const int j0 = rows.j;
    for (int s = 0; s < steps; ++s) {
        for (int it = q.col_first; it < q.col_end; ++it) {
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            batch_col_item<T, COL_PROP>(cols, it, lds, tid);
            __syncthreads();
        }
        BatchLaunch r = rows;
        r.j = j0 + s;
        for (int it = q.row_first; it < q.row_end; ++it) {
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            batch_row_item<T, ROW_MID>(r, it, lds, tid);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <typename T>
int batch_variant(int lg, int v, int* radices, int max_radices)
{
#define QW_X(LG, V, ...)                                                  \
    if (lg == LG && v == V) {                                             \
        const int r[] = {__VA_ARGS__};                                    \
        const int n = (int)(sizeof(r) / sizeof(r[0]));                    \
        for (int i = 0; i < n && i < max_radices; ++i) radices[i] = r[i]; \
        return n;                                                         \
    }
    QW_BATCH_VARIANTS(QW_X)
#undef QW_X
    return 0;
}

template <typename T>
int batch_tiles(int lg)
{
    // tiles of 256 threads per 2^lg lines of this length: lines / LINES
    const int l = 2 * (1 << lg) / batch_family<T>::E;
    return l > kBatchThreads ? -1 : kBatchThreads / l;
}

template <typename T>
hipError_t launch_batch_twiddles(void* tw, int lg, int v, hipStream_t st)
{
#define QW_X(LG, V, ...)                                                                                     \
    if (lg == LG && v == V) {                                                                               \
        constexpr int N = 1 << LG;                                                                           \
        static_assert(tw_len<1, __VA_ARGS__>::value <= 2 * N, "twiddle table larger than its slot");         \
        hipLaunchKernelGGL((twiddle_table<T, N, sched<__VA_ARGS__>>), dim3((2 * N + 255) / 256), dim3(256), 0, \
                           st, reinterpret_cast<cx<T>*>(tw));                                               \
        return hipGetLastError();                                                                            \
    }
    QW_BATCH_VARIANTS(QW_X)
#undef QW_X
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_batch_row(int mode, int grid, bool persist, const BatchLaunch& b, hipStream_t st)
{
    const dim3 g(grid), blk(kBatchThreads);
    if (persist) {
        if (mode != ROW_MID) return hipErrorInvalidValue;
        hipLaunchKernelGGL((batch_row<T, ROW_MID, true>), g, blk, 0, st, b);
        return hipGetLastError();
    }
    switch (mode) {
    case ROW_FIRST: hipLaunchKernelGGL((batch_row<T, ROW_FIRST, false>), g, blk, 0, st, b); break;
    case ROW_MID: hipLaunchKernelGGL((batch_row<T, ROW_MID, false>), g, blk, 0, st, b); break;
    case ROW_LAST: hipLaunchKernelGGL((batch_row<T, ROW_LAST, false>), g, blk, 0, st, b); break;
    case ROW_FWD_NORM: hipLaunchKernelGGL((batch_row<T, ROW_FWD_NORM, false>), g, blk, 0, st, b); break;
    case ROW_INV_SCALE: hipLaunchKernelGGL((batch_row<T, ROW_INV_SCALE, false>), g, blk, 0, st, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_col(int mode, int grid, bool persist, const BatchLaunch& b, hipStream_t st)
{
    const dim3 g(grid), blk(kBatchThreads);
    if (persist) {
        if (mode != COL_PROP) return hipErrorInvalidValue;
        hipLaunchKernelGGL((batch_col<T, COL_PROP, true>), g, blk, 0, st, b);
        return hipGetLastError();
    }
    switch (mode) {
    case COL_PROP: hipLaunchKernelGGL((batch_col<T, COL_PROP, false>), g, blk, 0, st, b); break;
    case COL_INV: hipLaunchKernelGGL((batch_col<T, COL_INV, false>), g, blk, 0, st, b); break;
    case COL_OBS: hipLaunchKernelGGL((batch_col<T, COL_OBS, false>), g, blk, 0, st, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// workgroups of the step loop that fit one CU (0 if the query fails)
template <typename T>
int batch_loop_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_loop<T>, kBatchThreads, 0) != hipSuccess) return 0;
    return nb;
}

template <typename T>
hipError_t launch_batch_inst_loop(int n_inst, const BatchLaunch& cols, const BatchLaunch& rows,
                                  const BatchInstItems* ranges, int steps, hipStream_t st)
{
    hipLaunchKernelGGL((batch_inst_loop<T>), dim3(n_inst), dim3(kBatchThreads), 0, st, cols, rows, ranges, steps);
    return hipGetLastError();
}

// one cooperative launch: the runtime refuses a grid that cannot be resident at once
template <typename T>
hipError_t launch_batch_loop(int grid, const BatchLaunch& cols, const BatchLaunch& rows, int steps, BatchSync* sync,
                             unsigned long long spin_ticks, hipStream_t st)
{
    BatchLaunch c = cols, r = rows;
    void* args[] = {&c, &r, &steps, &sync, &spin_ticks};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&batch_loop<T>), dim3(grid), dim3(kBatchThreads),
                                      args, 0, st);
}

}  // namespace qw

#define QW_DEFINE_BATCH_LAUNCHERS(T, SUF)                                                              \
    namespace qw {                                                                                     \
    int batch_lg_min_##SUF() { return batch_family<T>::lg_min; }                                       \
    int batch_lg_max_##SUF() { return batch_family<T>::lg_max; }                                       \
    int batch_variant_##SUF(int lg, int v, int* r, int m) { return batch_variant<T>(lg, v, r, m); }    \
    int batch_tiles_##SUF(int lg) { return batch_tiles<T>(lg); }                                       \
    hipError_t launch_batch_twiddles_##SUF(void* tw, int lg, int v, hipStream_t s)                     \
    {                                                                                                  \
        return launch_batch_twiddles<T>(tw, lg, v, s);                                                 \
    }                                                                                                  \
    hipError_t launch_batch_row_##SUF(int mode, int grid, bool persist, const BatchLaunch& b, hipStream_t s) \
    {                                                                                                  \
        return launch_batch_row<T>(mode, grid, persist, b, s);                                         \
    }                                                                                                  \
    hipError_t launch_batch_col_##SUF(int mode, int grid, bool persist, const BatchLaunch& b, hipStream_t s) \
    {                                                                                                  \
        return launch_batch_col<T>(mode, grid, persist, b, s);                                         \
    }                                                                                                  \
    int batch_loop_blocks_per_cu_##SUF() { return batch_loop_blocks_per_cu<T>(); }                     \
    hipError_t launch_batch_loop_##SUF(int grid, const BatchLaunch& c, const BatchLaunch& r, int steps, \
                                       BatchSync* sync, unsigned long long ticks, hipStream_t s)        \
    {                                                                                                  \
        return launch_batch_loop<T>(grid, c, r, steps, sync, ticks, s);                                \
    }                                                                                                  \
    hipError_t launch_batch_inst_loop_##SUF(int n, const BatchLaunch& c, const BatchLaunch& r,          \
                                            const BatchInstItems* q, int steps, hipStream_t s)         \
    {                                                                                                  \
        return launch_batch_inst_loop<T>(n, c, r, q, steps, s);                                        \
    }                                                                                                  \
    }
