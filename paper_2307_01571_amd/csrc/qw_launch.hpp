// qw_launch.hpp -- interface between the host engine (qw_api.cpp) and the
// kernel translation units.  Plain structs of pointers and scalars, passed
// by value as kernel arguments.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qw {

enum { ROW_FIRST = 0, ROW_MID = 1, ROW_LAST = 2, ROW_FWD_NORM = 3, ROW_INV_SCALE = 4 };
enum { COL_PROP = 0, COL_INV = 1, COL_OBS = 2 };

// same values as the QW_BEAM_* constants of the public header
constexpr int QW_BEAM_NONE_ = 0;
constexpr int QW_BEAM_STANDING_PARAXIAL_ = 1;
constexpr int QW_BEAM_UNIFORM_ = 2;

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
};

struct ColArgs {
    void* psi;
    const void* twy;   // per-pass twiddles of the y transform (2 ny entries)
    const void* ktab;  // COL_PROP: kinetic table, (nx/2+1) x (ny/2+1) pairs (cos(E dt), sin(E dt)/E)/(nx ny)
    int nx;
    double dkx, dky, c, dt, inv_cells;
    double* partial;  // COL_OBS: per-workgroup sums, partial_stride doubles each
    int partial_stride;
    int band_ref, band_half, window, n_max, spin0;
};

struct BeamArgs {
    int mode, longitudinal, nx, ny;
    double x_min, y_min, lx, ly, a0, kl, w0, ux, uy;
};

struct KineticArgs {
    int nx, ny;
    double dkx, dky, c, dt, inv_cells;
};

struct PacketArgs {
    int nx, ny, spin;
    double dkx, dky, c, p0x, p0y, x0, y0, sigma_x, x_min, y_min;
};

// Per-precision entry points (qw_kernels_f32.hip, qw_kernels_f64.hip).
// n is the transform length (nx for rows, ny for columns).
#define QW_DECLARE_LAUNCHERS(SUF)                                                          \
    hipError_t launch_row_##SUF(int mode, int nx, const RowArgs& a, hipStream_t s);       \
    hipError_t launch_col_##SUF(int mode, int ny, const ColArgs& a, hipStream_t s);       \
    int col_blocks_##SUF(int nx, int ny);                                                 \
    hipError_t launch_twiddles_##SUF(void* tw, int n, hipStream_t s);                     \
    hipError_t launch_beam_tables_##SUF(void* bx, void* by, const BeamArgs& b, hipStream_t s); \
    hipError_t launch_packet_##SUF(void* psi, double* rownorm, const PacketArgs& e, hipStream_t s); \
    hipError_t launch_kinetic_table_##SUF(void* ktab, const KineticArgs& k, hipStream_t s);
QW_DECLARE_LAUNCHERS(f32)
QW_DECLARE_LAUNCHERS(f64)
#undef QW_DECLARE_LAUNCHERS

// precision-independent kernels (qw_common.hip)
// out[0] = sum of rownorm[0..ny) in a fixed order
hipError_t launch_sum_rows(const double* rownorm, int ny, double* out, hipStream_t s);
// observables: results[0..3B+3) from the row norms and the column partials
hipError_t launch_obs_finish(const double* rownorm, int ny, const double* partial, int nblocks, int stride,
                             int n_max, double* results, hipStream_t s);

}  // namespace qw
