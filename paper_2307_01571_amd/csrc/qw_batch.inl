// qw_batch.inl -- batched form of the split-operator passes: one launch per
// pass advances every instance of a batch, whatever its grid.  Included by
// qw_kernels_f32.hip and qw_kernels_f64.hip after qw_kernels.inl.
//
// Every work item is one tile of one instance: 256 threads over RPW rows
// (row pass) or TX columns (column pass) of a line length N, with
// RPW = TX = 256 / (2 N / E).  With E elements per lane a tile always covers
// 128 E cells, so the items of all instances cost the same and a launch
// balances itself.  The launch is persistent when asked: fewer workgroups
// than items, each walking its own strided share of the list.
//
// The transform of each length comes in schedule variants (the same E,
// other radix orders); the hot modes (ROW_MID, COL_PROP) take the variant
// the batch's autotuner picked per length, the others the default plan.
#pragma once
#include "qw_kernels.inl"

#ifndef QW_WPE_BATCH_ROW
#define QW_WPE_BATCH_ROW 2
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
    }
