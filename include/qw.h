/*
 * qw.h -- C ABI of the MI355X split-operator propagator for the 2D Dirac
 * equation (libqw.so, HIP for gfx950).
 *
 * What it computes (Ge, Ahrens, Shen, "Two-dimensional simulation of the
 * spin-flip in the Kapitza-Dirac effect"):
 *   - the four-component Dirac spinor Psi(x, y) on a periodic nx x ny grid,
 *     Hamiltonian H = c alpha.(p + A) + beta c^2 in atomic units
 *     (Sec. II.B, Eq. 5, standard representation, m = hbar = 1);
 *   - the standing-wave vector potential of two counter-propagating Gaussian
 *     beams (Sec. II.A, Eq. 1-4) in its paraxial form, evaluated on the GPU;
 *   - time steps Psi(t + dt) = U(t + dt, t) Psi(t) by the FFT split-operator
 *     method (Sec. II.D, Eq. 15), in the symmetric order
 *     V(t_k, dt/2) F^-1 K(dt) F V(t_{k+1}, dt/2) with t_k = t0 + k dt;
 *   - the Gaussian initial packet (Sec. II.C, Eq. 12-14) and the band and
 *     spin-resolved probabilities (Sec. III.B, Eq. 18-19).
 *
 * Conventions shared by every call:
 *   - grid points x_i = x_min + i lx / nx (likewise y); momenta
 *     p = (2 pi / lx) k with k in [-nx/2, nx/2) (the Nyquist column is -nx/2);
 *   - psi is caller-owned device memory, contiguous [ny][nx][4] complex
 *     (interleaved re, im), complex128 for QW_F64, complex64 for QW_F32;
 *   - the workspace is caller-owned device memory of at least
 *     qw_workspace_bytes() bytes, 256-byte aligned, alive until qw_destroy;
 *   - the library allocates no device memory; qw_ctx itself is host memory
 *     owned by the library and released by qw_destroy;
 *   - every call that takes hip_stream enqueues only on that stream
 *     (a hipStream_t; NULL is the legacy default stream) and returns without
 *     waiting, except qw_observables, which waits for its own results;
 *   - every function returns QW_OK (0) or a negative QW_E_* code, never
 *     throws and never exits; argument errors are reported before anything
 *     is enqueued; qw_last_error(ctx) describes the last failure;
 *   - a context (likewise a batch) is not thread-safe: calls on one context
 *     from several host threads must be serialised by the caller; distinct
 *     contexts are independent.  Work enqueued on different streams for the
 *     same context or workspace (its tables, step clock and scratch plane)
 *     must not overlap on the device.
 */
#ifndef QW_H
#define QW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    QW_OK = 0,
    QW_E_ARG = -1,       /* null pointer, bad enum, non-finite parameter */
    QW_E_SIZE = -2,      /* grid size not a power of two in [8, 4096] */
    QW_E_WORKSPACE = -3, /* workspace too small or misaligned */
    QW_E_DEVICE = -4,    /* a HIP call failed (sticky device errors included) */
    QW_E_NUMERIC = -5,   /* a non-finite observable (outputs still written) */
    QW_E_STATE = -6      /* call out of order (e.g. stepping before qw_set_beam) */
};

enum { QW_F64 = 0, QW_F32 = 1 };

enum {
    QW_BEAM_NONE = 0,              /* A = 0: free evolution */
    QW_BEAM_STANDING_PARAXIAL = 1, /* standing wave, see qw_beam */
    QW_BEAM_UNIFORM = 2,           /* constant A = (ux, uy) */
    QW_BEAM_GAUSSIAN_FULL = 3      /* the full two-beam Gaussian standing wave, see qw_beam */
};

typedef struct qw_ctx_s *qw_ctx;

/* Grid and arithmetic type.  nx, ny: powers of two, 8 <= n <= 4096.
 * lx, ly > 0 box lengths; c > 0 the speed of light (137.036 in atomic units).
 * precision QW_F64: all arithmetic in double.  QW_F32: state, FFT
 * butterflies and spinor updates in float; the kinetic phase E(p) dt and
 * the field phase k_L x are formed and reduced modulo 2 pi in double before
 * the float sin/cos; norms and probabilities are summed in double. */
typedef struct {
    int32_t nx, ny;
    double x_min, y_min, lx, ly;
    double c;
    int32_t precision;
} qw_grid;

/* Vector potential.  QW_BEAM_STANDING_PARAXIAL (Sec. II.A, Eq. 1-4 in the
 * paraxial limit x << x_R, z = 0):
 *   A_y = a0 exp(-y^2/w0^2) cos(k_L x) cos(w t) f(t)
 *   A_x = a0 (2 y / (k_L w0^2)) exp(-y^2/w0^2) sin(k_L x) cos(w t) f(t)
 * QW_BEAM_GAUSSIAN_FULL (Sec. II.A, Eq. 1a, 1b, 2, 3 and 4 as printed, with
 * r^2 = y^2): the sum over d = +1, -1 of
 *   A_x,d = -2 d a0 (w0/w) eps (y/w) exp(-y^2/w^2) cos(phi_d + atan(d x/x_R))
 *   A_y,d = -a0 (w0/w) exp(-y^2/w^2) sin(phi_d),
 *   phi_d = w t - d k_L x + atan(d x/x_R) - d x y^2/(x_R w^2),
 *   w = w0 sqrt(1 + x^2/x_R^2), x_R = k_L w0^2/2, eps = 1/(k_L w0),
 * times f(t), evaluated per cell at the lab point of the cell (see qw_frame).
 * Both: k_L = 2 pi / lambda_l, w = c k_L, and the switch-on
 * f(t) = sin^2(pi t / (2 T_r)) for t < T_r = ramp_periods * lambda_l / c,
 * else 1 (ramp_periods = 0: no ramp).  longitudinal = 0 drops A_x.
 * QW_BEAM_UNIFORM uses the constant (ux, uy) and ignores the rest. */
typedef struct {
    int32_t mode;
    double a0, lambda_l, w0, ramp_periods;
    int32_t longitudinal;
    double ux, uy;
} qw_beam;

/* Frame of the simulation (Sec. II.D): the box moves along y with velocity
 * vy -- box row y stands for the lab point y + vy t, so the box follows a
 * packet moving with vy -- and a constant vector potential a_m along y is
 * added (the paper's gauge shift between canonical and kinetic momentum:
 * the grid momentum p is canonical, the kinetic momentum is p + a_m e_y).
 * In box coordinates H = c alpha.(p + a_m e_y + A(x, y + vy t, t)) + beta c^2
 * - vy p_y; the scalar -vy p_y joins the kinetic propagator as the phase
 * exp(i vy p_y dt).  |vy| < c; a moving box (vy != 0) needs a field that is
 * evaluated per cell (QW_BEAM_NONE, QW_BEAM_UNIFORM or QW_BEAM_GAUSSIAN_FULL).
 * Default: vy = a_m = 0 (the lab frame, no gauge shift). */
typedef struct {
    double vy, a_m;
} qw_frame;

/* Initial packet (Sec. II.C, Eq. 12-13):
 *   phi(p) = exp(-|p - p0|^2 / (4 s_p^2)) u^s(p) exp(-i p.r0),  s_p = 1/(2 sigma_x),
 * with u^s the unit-normalised positive-energy bispinor of Eq. 9 in the
 * x-polarised basis chi^+ = (1, 1)/sqrt2 (spin = +1) or chi^- = (1, -1)/sqrt2
 * (spin = -1); psi = sum_p phi(p) exp(i p.r), normalised to sum |psi|^2 = 1.
 * With a gauge shift a_m (qw_frame), p0 is the kinetic momentum: the packet
 * sits at grid momentum p0 - a_m e_y with the bispinors of p + a_m e_y. */
typedef struct {
    double p0x, p0y, x0, y0, sigma_x;
    int32_t spin;
} qw_packet;

/* Observables (Sec. III.B, Eq. 18-19).  With dk = 2 pi / lx, diffraction
 * order n collects the momentum columns k (signed index) with
 * |k - band_ref_idx - 2 n band_half_idx| <= window_idx, i.e. a window about
 * p_ref + 2 n k_L (p_ref = band_ref_idx dk, k_L = band_half_idx dk).
 * 0 <= window_idx < band_half_idx, 0 <= n_max <= 16, spin0 = +1 or -1. */
typedef struct {
    int32_t band_ref_idx, band_half_idx, window_idx, n_max, spin0;
} qw_obs_spec;

/* Bytes of workspace a grid needs (twiddle and field tables, reduction
 * partials and one state-sized plane for qw_observables). */
int qw_workspace_bytes(const qw_grid *g, size_t *bytes);

/* Validate the grid, bind the workspace and enqueue the twiddle-table
 * kernel on hip_stream.  On success *out is a new context. */
int qw_init_grid(qw_ctx *out, const qw_grid *g, void *workspace, size_t ws_bytes, void *hip_stream);

/* Set the vector potential (host-only; the field tables are rebuilt on the
 * stream of the next call that needs them). */
int qw_set_beam(qw_ctx h, const qw_beam *b);

/* Set the frame (host-only; takes effect for the next calls).  The kinetic
 * table, packets and observables of a context follow its current frame. */
int qw_set_frame(qw_ctx h, const qw_frame *f);

/* Write the normalised initial packet into psi (several kernels). */
int qw_init_packet(qw_ctx h, void *psi, const qw_packet *e, void *hip_stream);

/* n >= 0 split-operator steps of size dt from t0, in place on psi.
 * dt may be negative (backward propagation); dt = 0 and n = 0 leave psi as is
 * (n = 0 enqueues nothing).  2n + 1 kernels: one row pass V(t0, dt/2) F_x,
 * then n column passes F_y^-1 K(dt) F_y interleaved with n - 1 row passes
 * F_x V(t_k, dt) F_x^-1, and a last row pass V(t_n, dt/2) F_x^-1.
 * With timing off and hip_stream not being captured by the caller, the
 * middle passes of the two Dirac blocks (A = (psi1, psi4), B = (psi3, psi2),
 * which the propagators never couple) run as two chains of per-block
 * launches, A on hip_stream and B on a stream of the library's own, forked
 * from hip_stream after the first row pass and joined to it before the
 * last; for n > 64 they run as replays of one HIP graph of 64 (column, row)
 * pass pairs per block, whose row passes read t_k from a step clock in the
 * workspace.  The graph is captured on streams of the library's own at the
 * first such call and again whenever psi, the beam or the frame differ from
 * that capture's (graph, streams and events live until qw_destroy).  With
 * timing on, or under the caller's capture, every pass covers both blocks on
 * hip_stream.  The results are the same bit for bit either way.
 * In FP32 the kinetic table carries, besides 1/(nx ny), the factor that
 * undoes the transforms' mean loss of norm (qw_transform_gain). */
int qw_step_n(qw_ctx h, void *psi, int64_t n, double t0, double dt, void *hip_stream);

/* Observables of psi (not modified) into out_host (host memory), laid out as
 *   [norm, P_n (B), P_n^+ (B), P_n^- (B), P_flip, P_neg],  B = 2 n_max + 1,
 * out_len >= 3B + 3.  norm = sum_cells |psi|^2; every P is a ratio to
 * sum_p |phi(p)|^2: P_n = window sum of |phi|^2, P_n^s = window sum of
 * |<u^s(p)|phi(p)>|^2 (bispinors of the kinetic momentum p + a_m e_y),
 * P_flip = sum over all p of |<u^{-spin0}|phi>|^2,
 * P_neg = 1 - sum_p (|c^+|^2 + |c^-|^2) (the negative-energy share).
 * Waits for hip_stream.  Returns QW_E_NUMERIC if any output is not finite. */
int qw_observables(qw_ctx h, const void *psi, const qw_obs_spec *o, double *out_host, int32_t out_len,
                   void *hip_stream);

/* Momentum-space maps of psi (not modified): out (device memory, out_len >=
 * 3 nx ny doubles) receives for every momentum cell, laid out [ky][kx][3] in
 * the transform's order (index k stands for the signed k < n/2 ? k : k - n),
 * (|phi(p)|^2, |<u^+(p)|phi(p)>|^2, |<u^-(p)|phi(p)>|^2) with phi the
 * unnormalised forward transform (Eq. 14, 18-19; bispinors of the kinetic
 * momentum).  Asynchronous. */
int qw_momentum_maps(qw_ctx h, const void *psi, double *out, int64_t out_len, void *hip_stream);

/* Per-kernel timing for profiling: with enable = 1, every later launch of a
 * row or column pass by qw_step_n is bracketed by HIP events on its stream.
 * qw_kernel_times waits for the stream and writes
 *   out[0] = row-pass launches, out[1] = their total ms,
 *   out[2] = column-pass launches, out[3] = their total ms  (out_len >= 4),
 * then clears the counters.  Enabling adds event records between launches. */
int qw_kernel_timing(qw_ctx h, int enable);
int qw_kernel_times(qw_ctx h, double *out, int32_t out_len, void *hip_stream);

/* Mean squared-norm gain of one transform of length n (a power of two, 8 ..
 * 4096) in the given precision, as the library models it: in FP32 each
 * rotation constant and twiddle is the nearest float of its cos and of its
 * sin (phase within half a unit in the last place), so its squared
 * magnitude falls a little short of 1; averaged over each pass's inputs the
 * passes' gains multiply.  The step loop multiplies K(dt) by
 * 1/(gain(nx) gain(ny)), which keeps the norm of a float step on average.
 * QW_F64: 1.  Host arithmetic only (no device work); batch_variant < 0
 * takes the single-instance plan, v >= 0 the batched schedule variant v. */
int qw_transform_gain(int32_t n, int32_t precision, int32_t batch_variant, double *gain);

/* Message of the last failure on h (or of the last failed qw_init_grid when
 * h is NULL).  Valid until the next call on h. */
const char *qw_last_error(qw_ctx h);

/* Release the context (not the caller's psi or workspace).  NULL is a no-op. */
void qw_destroy(qw_ctx h);

/* ---------------------------------------------------------------------------
 * Batched form: many independent instances -- each with its own grid, field
 * and packet, all of one precision -- advanced together.  Every pass of a
 * step is one kernel launch over the tiles of all instances, the step loop
 * replays a captured HIP graph, and the transform schedules are picked per
 * line length by a built-in autotuner.  The physics of each instance is
 * exactly that of the single-instance calls above (same kernels' bodies).
 *
 * Batched instances use the lab frame (no qw_frame) and the table-driven
 * fields (QW_BEAM_NONE, QW_BEAM_STANDING_PARAXIAL, QW_BEAM_UNIFORM).
 *
 * Batch state: the instances' psi arrays back to back in one caller-owned
 * device buffer, instance i at byte offset offsets[i] (256-byte aligned),
 * each laid out as psi above.  Limits: 1 <= n <= 65535 instances; nx, ny
 * powers of two in [64, 2048] for QW_F32 and [64, 1024] for QW_F64.
 * The batch workspace (caller-owned device memory, 256-byte aligned) holds
 * the tables, the work lists, the reduction scratch and one plane the size
 * of the batch state.
 * ------------------------------------------------------------------------- */
typedef struct qw_batch_s *qw_batch;

typedef struct {
    qw_grid grid;
    qw_beam beam;
} qw_instance;

/* Sizes for n instances: offsets[i] (n entries, may be NULL), total state
 * bytes and workspace bytes (either may be NULL).  Host-only. */
int qw_batch_layout(const qw_instance *inst, int32_t n, int64_t *offsets, size_t *state_bytes, size_t *ws_bytes);

/* Validate the instances, bind the workspace and build every table on
 * hip_stream (waits for it).  On success *out is a new batch.  The schedule
 * variant of every length starts at 0 (the single-instance plan), the
 * launch at one workgroup per tile with 64-step graph chunks. */
int qw_batch_init(qw_batch *out, const qw_instance *inst, int32_t n, void *workspace, size_t ws_bytes,
                  void *hip_stream);

/* Write each instance's normalised initial packet (packets: n entries). */
int qw_batch_init_packets(qw_batch b, void *psi, const qw_packet *packets, void *hip_stream);

/* n >= 0 steps of every instance from t0 with step dt, in place, with the
 * same sequence as qw_step_n; asynchronous.  The middle steps run as
 * replays of a captured graph of graph_steps (column pass, row pass) pairs
 * whose step index comes from a device counter, or, with the step loop on
 * (qw_batch_set_loop), as persistent launches of up to graph_steps (64 when
 * 0) steps each; the rest are direct launches, and so is everything while
 * timing is on or while the caller captures hip_stream itself. */
int qw_batch_step_n(qw_batch b, void *psi, int64_t n, double t0, double dt, void *hip_stream);

/* Observables of every instance (specs: n entries, one n_max for all) into
 * out_host: instance i at out_host[i (3B + 3)], laid out as qw_observables;
 * out_len >= n (3B + 3).  Waits for hip_stream. */
int qw_batch_observables(qw_batch b, const void *psi, const qw_obs_spec *specs, double *out_host, int32_t out_len,
                         void *hip_stream);

/* Schedules.  qw_batch_schedule writes the radices of variant v for line
 * length 2^log2n into radices (up to max_radices) and returns their count
 * (0: no such variant) or a negative error.  qw_batch_set_schedule picks
 * variant v for the row (pass = 0) or column (pass = 1) transforms of that
 * length in the step's middle passes. */
int qw_batch_schedule(qw_batch b, int32_t log2n, int32_t v, int32_t *radices, int32_t max_radices);
int qw_batch_set_schedule(qw_batch b, int32_t log2n, int32_t pass, int32_t v);

/* Launch shape: wg_per_cu = 0 launches one workgroup per tile; k > 0 a
 * persistent grid of k workgroups per compute unit that loop over the
 * tiles (row and column pass separately); graph_steps = 0 launches every
 * step directly. */
int qw_batch_set_launch(qw_batch b, int32_t row_wg_per_cu, int32_t col_wg_per_cu, int32_t graph_steps);

/* Step loop (the batched form's persistent launches).  wg_per_cu = 0 (the
 * default) turns it off.  k > 0: qw_batch_step_n runs its middle steps in
 * cooperative launches of k workgroups per compute unit (at most the number
 * that fit one CU, *max_wg_per_cu when not NULL; the grid never exceeds the
 * work items), each advancing up to graph_steps steps: every workgroup
 * walks its share of the column tiles, all meet at a grid-wide barrier,
 * then the row tiles, and a barrier again.  QW_LOOP_INSTANCE: launches of
 * one workgroup per instance, each running its instance's column and row
 * tiles for up to graph_steps steps with no grid-wide barrier (for batches
 * of many small grids).  The arithmetic and the results are those of the
 * one-launch-per-pass path, bit for bit.  wait_limit_s (0: 2 s; at most
 * 60) bounds each barrier wait; a wait past it ends the launch early and
 * leaves psi invalid, and the next qw_batch_observables returns QW_E_DEVICE
 * saying so.  Returns QW_E_DEVICE for k > 0 if the device has no
 * cooperative launches.  wg_per_cu = -1 only reports *max_wg_per_cu. */
#define QW_LOOP_INSTANCE (-2)
int qw_batch_set_loop(qw_batch b, int32_t wg_per_cu, double wait_limit_s, int32_t *max_wg_per_cu);

/* Autotuner: times, on a copy of psi in the workspace (psi is not
 * modified), every schedule variant of every line length of the batch for
 * the row and column passes, then the launch shapes, and keeps the fastest
 * of each.  reps launches per candidate.  report (optional, report_len
 * doubles) receives rows of 4 values (kind, a, b, microseconds per launch):
 * kind 0 row schedule (a = log2n, b = variant), 1 column schedule,
 * 2 row launch (a = wg_per_cu), 3 column launch, 4 middle steps (a = the
 * step loop's wg_per_cu, 0 for the graph replays, QW_LOOP_INSTANCE;
 * microseconds per step, graph_steps (64 when 0) steps per launch);
 * *n_rows their count.  Kind 4 keeps the step loop only where it is
 * faster; QW_LOOP_INSTANCE is a candidate only when no instance has more
 * than 16 tiles per step (row and column tiles; 16 for 128^2 FP32).
 * Waits for hip_stream. */
int qw_batch_autotune(qw_batch b, const void *psi, double dt, int32_t reps, double *report, int32_t report_len,
                      int32_t *n_rows, void *hip_stream);

/* Per-kernel timing, as qw_kernel_timing / qw_kernel_times (graphs are not
 * used while timing is on). */
int qw_batch_kernel_timing(qw_batch b, int enable);
int qw_batch_kernel_times(qw_batch b, double *out, int32_t out_len, void *hip_stream);

/* Message of the last failure on b (or of the last failed qw_batch_init or
 * qw_batch_layout when b is NULL). */
const char *qw_batch_last_error(qw_batch b);

/* Release the batch (graphs, events, host memory; not psi or workspace). */
void qw_batch_destroy(qw_batch b);

#ifdef __cplusplus
}
#endif
#endif /* QW_H */
