// qw_launch.hpp -- interface between the host engine (qw_api.cpp) and the
// kernel translation units.  Plain structs of pointers and scalars, passed
// by value as kernel arguments.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qw {

enum { ROW_FIRST = 0, ROW_MID = 1, ROW_LAST = 2, ROW_FWD_NORM = 3, ROW_INV_SCALE = 4 };
enum { COL_PROP = 0, COL_INV = 1, COL_OBS = 2, COL_MAPS = 3 };

// same values as the QW_BEAM_* constants of the public header
constexpr int QW_BEAM_NONE_ = 0;
constexpr int QW_BEAM_STANDING_PARAXIAL_ = 1;
constexpr int QW_BEAM_UNIFORM_ = 2;
constexpr int QW_BEAM_GAUSSIAN_FULL_ = 3;

// Full Gaussian-beam standing wave, evaluated per cell (double), in a box
// whose y coordinate stands for the lab point y + vy t.
struct FullBeam {
    double a0, kl, w0, xr, eps;  // eps = 1/(kl w0), xr = kl w0^2/2
    double x_min, dx, y_min, dy;
    double vy;
    int longitudinal;
};

// Device-resident time of a propagation.  A graph-captured chunk of steps
// takes t0, dt and the base k_base of the step index from here and advances
// k_base by its length at its end, so one captured chunk replays for every
// chunk of a run.  (Batched form: V is taken at t0 + k dt with
// k = (use_counter ? k_base : 0) + j.)
struct StepClock {
    double t0, dt;
    long long k_base;
    long long pad_;
};

struct RowArgs {
    const void* src;          // [ny][nx][4] complex T
    void* dst;                // may equal src (in place)
    const void* twx;          // per-pass twiddles of the x transform (2 nx entries)
    const void* beam_x;       // nx field factors (X0, X1)
    const void* beam_y;       // ny field factors (Y0, Y1)
    double* rownorm;          // ROW_FWD_NORM: ny row sums of |psi|^2
    const double* scale_src;  // ROW_INV_SCALE: sum of |phi|^2 of the packet
    double t0, dt;            // the field is taken at t0 + k dt ...
    long long k;
    double tau_frac;          // ... and V acts for tau_frac * dt
    double omega, t_ramp, ramp_k, c;  // ramp_k = pi / (2 t_ramp)
    int beam_mode;
    int ny;
    FullBeam full;            // beam_mode == QW_BEAM_GAUSSIAN_FULL_
    const StepClock* clock;   // if set (graph replays): t0 and dt from here, k offset by clock->k_base
    int one_block;            // ROW_MID: 0 both Dirac blocks, 1 block A only, 2 block B only
};

struct ColArgs {
    void* psi;
    const void* twy;   // per-pass twiddles of the y transform (2 ny entries)
    const void* ktab;  // COL_PROP: kinetic table, (nx/2+1) x (ny/2+1) pairs (cos(E dt), sin(E dt)/E)/(nx ny);
                       // with a frame (nx/2+1) x ny pairs of pairs, see kinetic_table_frame
    int nx;
    int frame;         // 1: moving box and/or gauge shift (a_m) -- the frame kinetic table
    double a_m;        // constant gauge vector potential along y (kinetic p_y = p_y + a_m)
    double dkx, dky, c, dt, inv_cells;
    double* partial;  // COL_OBS: per-workgroup sums, partial_stride doubles each;
                      // COL_MAPS: [ny][nx][3] per-cell (|phi|^2, |c+|^2, |c-|^2)
    int partial_stride;
    int band_ref, band_half, window, n_max, spin0;
    int one_block;     // COL_PROP: 0 both Dirac blocks, 1 block A only, 2 block B only
};

struct BeamArgs {
    int mode, longitudinal, nx, ny;
    double x_min, y_min, lx, ly, a0, kl, w0, ux, uy;
};

struct KineticArgs {
    int nx, ny;
    double dkx, dky, c, dt, inv_cells;
    double vy, a_m;  // frame (kinetic_table_frame only)
};

struct PacketArgs {
    int nx, ny, spin;
    double dkx, dky, c, p0x, p0y, x0, y0, sigma_x, x_min, y_min;
    double a_m;  // gauge shift: p0 is kinetic, the grid momentum canonical
};

// ---------------------------------------------------------------------------
// Batched form: independent instances, each with its own grid, field and
// packet, advanced by one launch per pass.  A launch walks a list of work
// items (instance, tile); every tile is one 256-thread workgroup's worth of
// lines of that instance, whatever its length.
// ---------------------------------------------------------------------------
constexpr int kBatchThreads = 256;
constexpr int kBatchMaxVariants = 4;  // schedule variants per transform length

struct BatchInst {
    RowArgs row;           // row pass arguments (state pointers and time set per launch)
    ColArgs col;           // column pass arguments (state pointer set per launch)
    const void* tw_row;    // twiddles of the tuned schedules used by ROW_MID ...
    const void* tw_col;    // ... and COL_PROP (the other modes use the default plan's)
    double* scalars;       // [0] packet norm, [8 ..) observables
    long long off;         // byte offset of the instance's state from the batch base
    int lgx, lgy;          // log2 nx, log2 ny
    int row_var, col_var;  // tuned schedule variants (0 = default plan)
    int ntile_col;         // column tiles (partials for the observables)
    int pad_;
};

struct BatchLaunch {
    const BatchInst* __restrict__ inst;
    const uint32_t* __restrict__ items;  // (instance << 16) | tile
    int n_items;
    int j;            // step index (plus k_base when use_counter)
    int use_counter;
    int pad_;
    char* src;        // state bases; dst may equal src
    char* dst;
    const StepClock* time;
    double tau_frac;
};

// Per-precision entry points (qw_kernels_f32.hip, qw_kernels_f64.hip).
// n is the transform length (nx for rows, ny for columns).
#define QW_DECLARE_LAUNCHERS(SUF)                                                          \
    hipError_t launch_row_##SUF(int mode, int nx, const RowArgs& a, hipStream_t s);       \
    hipError_t launch_col_##SUF(int mode, int ny, const ColArgs& a, hipStream_t s);       \
    int col_blocks_##SUF(int nx, int ny);                                                 \
    int plan_radices_##SUF(int n, int* radices, int max_radices);                         \
    hipError_t launch_twiddles_##SUF(void* tw, int n, hipStream_t s);                     \
    hipError_t launch_beam_tables_##SUF(void* bx, void* by, const BeamArgs& b, hipStream_t s); \
    hipError_t launch_packet_##SUF(void* psi, double* rownorm, const PacketArgs& e, hipStream_t s); \
    hipError_t launch_kinetic_table_##SUF(void* ktab, const KineticArgs& k, hipStream_t s);          \
    hipError_t launch_kinetic_table_frame_##SUF(void* ktab, const KineticArgs& k, hipStream_t s);    \
    /* batched form (qw_batch_*.hip): lengths 2^lg, lg_min <= lg <= lg_max; schedule variant v */  \
    int batch_lg_min_##SUF();                                                                    \
    int batch_lg_max_##SUF();                                                                    \
    int batch_variant_##SUF(int lg, int v, int* radices, int max_radices);                       \
    int batch_tiles_##SUF(int lg);                                                               \
    hipError_t launch_batch_twiddles_##SUF(void* tw, int lg, int v, hipStream_t s);              \
    hipError_t launch_batch_row_##SUF(int mode, int grid, bool persist, const BatchLaunch& b, hipStream_t s); \
    hipError_t launch_batch_col_##SUF(int mode, int grid, bool persist, const BatchLaunch& b, hipStream_t s);
QW_DECLARE_LAUNCHERS(f32)
QW_DECLARE_LAUNCHERS(f64)
#undef QW_DECLARE_LAUNCHERS

// precision-independent kernels (qw_common.hip)
// out[0] = sum of rownorm[0..ny) in a fixed order
hipError_t launch_sum_rows(const double* rownorm, int ny, double* out, hipStream_t s);
// observables: results[0..3B+3) from the row norms and the column partials
hipError_t launch_obs_finish(const double* rownorm, int ny, const double* partial, int nblocks, int stride,
                             int n_max, double* results, hipStream_t s);
// batched: per instance, scalars[0] = sum of its row norms
hipError_t launch_batch_sum_rows(const BatchInst* inst, int n, hipStream_t s);
// batched: per instance, scalars[8 ..] = observables from its rows and column partials
hipError_t launch_batch_obs_finish(const BatchInst* inst, int n, int stride, int n_max, hipStream_t s);
// batched time: set (t0, dt, k_base), or advance k_base
hipError_t launch_clock_set(StepClock* t, double t0, double dt, long long k, hipStream_t s);
hipError_t launch_clock_advance(StepClock* t, long long steps, hipStream_t s);

}  // namespace qw
