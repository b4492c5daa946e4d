// qw_batch_loop.hpp -- interface of the batched form's step loop: the
// barrier counters it keeps in the batch workspace and its per-precision
// launchers (defined in qw_batch_f32.hip and qw_batch_f64.hip).
#pragma once
#include "qw_launch.hpp"

namespace qw {

// Counters of the step loop's grid-wide barrier (one per batch, in its
// workspace; zero between launches).  The workgroups form 8 groups
// (blockIdx mod 8, one per XCD under round-robin dispatch); every word that
// is polled or counted sits in a 256-byte slot of its own.
struct BatchSyncSlot {
    unsigned v;
    unsigned pad_[63];
};
struct BatchSync {
    BatchSyncSlot arrived;           // the groups' last arrivals, over the launch's barriers
    BatchSyncSlot departed;          // workgroups that have left the running launch
    BatchSyncSlot failed;            // sticky: a barrier wait ran past its limit (read and cleared by the host)
    BatchSyncSlot group_arrived[8];  // arrivals within each group
    BatchSyncSlot group_pass[8];     // barrier index each group may pass
};

// an instance's work items: rows [row_first, row_end) of the row list,
// columns [col_first, col_end) of the column list
struct BatchInstItems {
    int row_first, row_end, col_first, col_end;
};

// step-loop workgroups that fit one CU (0 if the query fails); one
// cooperative launch of grid workgroups running `steps` middle steps from
// rows.j, each wait bounded by spin_ticks of the wall clock; or one launch
// of one workgroup per instance (n of them) running its own steps
#define QW_DECLARE_LOOP_LAUNCHERS(SUF)                                                                    \
    int batch_loop_blocks_per_cu_##SUF();                                                                 \
    hipError_t launch_batch_loop_##SUF(int grid, const BatchLaunch& cols, const BatchLaunch& rows, int steps, \
                                       BatchSync* sync, unsigned long long spin_ticks, hipStream_t s);     \
    hipError_t launch_batch_inst_loop_##SUF(int n, const BatchLaunch& cols, const BatchLaunch& rows,        \
                                            const BatchInstItems* ranges, int steps, hipStream_t s);
QW_DECLARE_LOOP_LAUNCHERS(f32)
QW_DECLARE_LOOP_LAUNCHERS(f64)
#undef QW_DECLARE_LOOP_LAUNCHERS

}  // namespace qw
