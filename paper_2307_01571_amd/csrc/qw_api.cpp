// qw_api.cpp -- host engine behind the C ABI of include/qw.h: argument
// validation, workspace carving, table set-up and the launch sequence of the
// split-operator step (direct launches, or replays of one captured chunk of
// the step loop).  No device memory is allocated here; every launch and
// replay goes to the caller's stream.
#include "qw.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "qw_host.hpp"
#include "qw_launch.hpp"

namespace {

using qwh::align_up;
using qwh::kAlign;
using qwh::kPartialStride;

// workspace layout (byte offsets from the start, each 256-aligned)
struct Layout {
    size_t scalars;   // 256 doubles: [0] packet norm, [8..) observables results
    size_t twx, twy;  // twiddle tables
    size_t bx, by;    // field tables
    size_t ktab;      // kinetic table, (nx/2+1)(ny/2+1) complex
    size_t rownorm;   // ny doubles
    size_t partial;   // column-pass workgroups x kPartialStride doubles
    size_t plane;     // one state-sized array
    size_t total;
};

Layout make_layout(const qw_grid& g)
{
    const size_t cs = g.precision == QW_F32 ? 8 : 16;  // bytes per complex
    const int nblk_max = g.nx;                         // column workgroups never exceed nx
    Layout L;
    size_t o = 0;
    L.scalars = o;
    o = align_up(o + 256 * sizeof(double));
    L.twx = o;  // per-pass twiddles: 2 nx entries
    o = align_up(o + 2 * (size_t)g.nx * cs);
    L.twy = o;
    o = align_up(o + 2 * (size_t)g.ny * cs);
    L.bx = o;
    o = align_up(o + (size_t)g.nx * cs);
    L.by = o;
    o = align_up(o + (size_t)g.ny * cs);
    L.ktab = o;  // room for either table: (nx/2+1)(ny/2+1) pairs, or (nx/2+1) ny pairs of pairs in a frame
    o = align_up(o + (size_t)(g.nx / 2 + 1) * g.ny * 2 * cs);
    L.rownorm = o;
    o = align_up(o + (size_t)g.ny * sizeof(double));
    L.partial = o;
    o = align_up(o + (size_t)nblk_max * kPartialStride * sizeof(double));
    L.plane = o;
    o = align_up(o + (size_t)g.nx * g.ny * 4 * cs);
    L.total = o;
    return L;
}

struct TimedLaunch {
    hipEvent_t a, b;
    int kind;  // 0 row, 1 column
};

}  // namespace

struct qw_ctx_s {
    qw_grid g{};
    qw_beam b{};
    bool beam_set = false;
    bool tables_dirty = true;
    bool ktab_valid = false;
    double ktab_dt = 0.0;  // time step the kinetic table was built for
    qw_frame frame{};      // moving box and gauge shift (zero: lab frame)
    qw_frame ktab_frame{}; // frame the kinetic table was built for
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Layout lay{};
    int device = 0;
    std::string err;
    bool timing = false;
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
    // the step loop's captured chunk (it works on the workspace plane): valid
    // for exec_psi and the beam/frame state of args_version
    hipStream_t cap = nullptr;
    // the middle passes of the two Dirac blocks run as two chains: block A on
    // the caller's stream (or cap), block B on side (or cap_side), forked from
    // and joined back into the first by the events
    hipStream_t side = nullptr, cap_side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr, cap_fork = nullptr, cap_join = nullptr;
    hipGraphExec_t exec = nullptr;
    // recorded on the caller's stream after the replays of each call: the
    // executable graph is destroyed only once its last replay has finished
    hipEvent_t exec_done = nullptr;
    const void* exec_psi = nullptr;
    unsigned long long args_version = 0, exec_version = 0;
};

namespace {

thread_local std::string g_init_error;

int fail(qw_ctx h, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    else g_init_error = buf;
    return code;
}

int hip_fail(qw_ctx h, hipError_t e, const char* what)
{
    return fail(h, QW_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int check_grid(const qw_grid* g)
{
    if (!g) return fail(nullptr, QW_E_ARG, "grid is NULL");
    std::string msg;
    const int rc = qwh::check_grid(*g, 8, 4096, &msg);
    if (rc != QW_OK) return fail(nullptr, rc, "%s", msg.c_str());
    return QW_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool f32(const qw_ctx h) { return h->g.precision == QW_F32; }

hipError_t launch_row(qw_ctx h, int mode, const qw::RowArgs& a, hipStream_t s)
{
    return f32(h) ? qw::launch_row_f32(mode, h->g.nx, a, s) : qw::launch_row_f64(mode, h->g.nx, a, s);
}

hipError_t launch_col(qw_ctx h, int mode, const qw::ColArgs& a, hipStream_t s)
{
    return f32(h) ? qw::launch_col_f32(mode, h->g.ny, a, s) : qw::launch_col_f64(mode, h->g.ny, a, s);
}

int col_blocks(qw_ctx h) { return f32(h) ? qw::col_blocks_f32(h->g.nx, h->g.ny) : qw::col_blocks_f64(h->g.nx, h->g.ny); }

hipEvent_t pooled_event(qw_ctx h)
{
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    // timing-only events: no system-scope fence at record time, so the
    // bracket does not add a cache writeback to the launch it measures
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) == hipSuccess) return e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// bracket a launch with events when timing is on
template <typename F>
hipError_t timed(qw_ctx h, int kind, hipStream_t s, F&& launch)
{
    if (!h->timing) return launch();
    TimedLaunch t{pooled_event(h), pooled_event(h), kind};
    if (!t.a || !t.b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(t.a, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(t.b, s);
    h->timed.push_back(t);
    return e;
}

int ensure_tables(qw_ctx h, hipStream_t s)
{
    if (!h->tables_dirty) return QW_OK;
    const qw::BeamArgs a = qwh::beam_args(h->g, h->b);
    void* bx = h->ws + h->lay.bx;
    void* by = h->ws + h->lay.by;
    hipError_t e = f32(h) ? qw::launch_beam_tables_f32(bx, by, a, s) : qw::launch_beam_tables_f64(bx, by, a, s);
    if (e != hipSuccess) return hip_fail(h, e, "field table kernel");
    h->tables_dirty = false;
    return QW_OK;
}

// the kinetic table depends on dt only (and the grid): rebuild when dt changes
int ensure_kinetic_table(qw_ctx h, double dt, hipStream_t s)
{
    if (h->ktab_valid && h->ktab_dt == dt && h->ktab_frame.vy == h->frame.vy && h->ktab_frame.a_m == h->frame.a_m)
        return QW_OK;
    qw::KineticArgs k = qwh::kinetic_args(h->g, dt);
    if (f32(h)) {
        // the float transforms' mean loss of norm, undone in K (see transform_gain_f32)
        int rx[8], ry[8];
        const int nrx = qw::plan_radices_f32(h->g.nx, rx, 8), nry = qw::plan_radices_f32(h->g.ny, ry, 8);
        k.inv_cells *= qwh::kinetic_norm_factor(true, rx, nrx, ry, nry);
    }
    void* kt = h->ws + h->lay.ktab;
    hipError_t e;
    if (qwh::frame_active(h->frame)) {
        k.vy = h->frame.vy;
        k.a_m = h->frame.a_m;
        e = f32(h) ? qw::launch_kinetic_table_frame_f32(kt, k, s) : qw::launch_kinetic_table_frame_f64(kt, k, s);
    } else {
        e = f32(h) ? qw::launch_kinetic_table_f32(kt, k, s) : qw::launch_kinetic_table_f64(kt, k, s);
    }
    if (e != hipSuccess) return hip_fail(h, e, "kinetic table kernel");
    h->ktab_valid = true;
    h->ktab_dt = dt;
    h->ktab_frame = h->frame;
    return QW_OK;
}

qw::RowArgs row_args(qw_ctx h, const void* src, void* dst)
{
    qw::RowArgs a{};
    a.src = src;
    a.dst = dst;
    a.twx = h->ws + h->lay.twx;
    a.beam_x = h->ws + h->lay.bx;
    a.beam_y = h->ws + h->lay.by;
    a.rownorm = reinterpret_cast<double*>(h->ws + h->lay.rownorm);
    a.scale_src = reinterpret_cast<const double*>(h->ws + h->lay.scalars);
    qwh::row_field(h->g, h->b, h->beam_set, &a, h->frame.vy);
    return a;
}

qw::ColArgs col_args(qw_ctx h, void* psi)
{
    qw::ColArgs a{};
    a.psi = psi;
    a.twy = h->ws + h->lay.twy;
    a.ktab = h->ws + h->lay.ktab;
    qwh::col_grid(h->g, &a);
    a.partial = reinterpret_cast<double*>(h->ws + h->lay.partial);
    a.frame = qwh::frame_active(h->frame) ? 1 : 0;
    a.a_m = h->frame.a_m;
    return a;
}

// middle steps per captured chunk of the step loop
constexpr int kGraphSteps = 64;

// the library's streams and events of the step loop, created once per
// context with its device current (default priority, non-blocking)
hipError_t ensure_streams(qw_ctx h)
{
    if (h->cap) return hipSuccess;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != h->device) e = hipSetDevice(h->device);
    for (hipStream_t* st : {&h->cap, &h->side, &h->cap_side})
        if (e == hipSuccess) e = hipStreamCreateWithFlags(st, hipStreamNonBlocking);
    for (hipEvent_t* ev : {&h->exec_done, &h->fork_ev, &h->join_ev, &h->cap_fork, &h->cap_join})
        if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    if (prev != h->device) (void)hipSetDevice(prev);
    return e;
}

// Middle steps j0 .. j0 + count - 1 (column pass, then the row pass V(t_k, dt)
// with k = the step) and, if final_col, the column pass of the last step,
// as two chains: block A on a, block B on b, b forked from a before and a
// joined to b after (the blocks never couple, so the chains are independent
// and one chain's kernels fill the GPU while the other's start or drain).
hipError_t enqueue_middle(qw_ctx h, hipStream_t a, hipStream_t b, hipEvent_t fork, hipEvent_t join, qw::RowArgs r,
                          qw::ColArgs c, int64_t j0, int64_t count, bool final_col)
{
    hipError_t e = hipEventRecord(fork, a);
    if (e == hipSuccess) e = hipStreamWaitEvent(b, fork, 0);
    r.tau_frac = 1.0;  // V(t_k, dt/2) V(t_k, dt/2) = V(t_k, dt)
    for (int64_t j = 0; j < count && e == hipSuccess; ++j) {
        r.k = j0 + j;
        for (int blk = 1; blk <= 2 && e == hipSuccess; ++blk) {
            hipStream_t st = blk == 1 ? a : b;
            c.one_block = r.one_block = blk;
            e = launch_col(h, qw::COL_PROP, c, st);
            if (e == hipSuccess) e = launch_row(h, qw::ROW_MID, r, st);
        }
    }
    for (int blk = 1; blk <= 2 && final_col && e == hipSuccess; ++blk) {
        c.one_block = blk;
        e = launch_col(h, qw::COL_PROP, c, blk == 1 ? a : b);
    }
    if (e == hipSuccess) e = hipEventRecord(join, b);
    if (e == hipSuccess) e = hipStreamWaitEvent(a, join, 0);
    return e;
}

// the step loop's device clock: 4 doubles at the end of the 256-double
// scalars slot ([0] packet norm, [8, 8 + 3B + 3) observables, B <= 33)
constexpr int kClockSlot = 248;
static_assert(8 + 3 * (2 * qwh::kMaxNmax + 1) + 3 <= kClockSlot, "observables overlap the step clock");
static_assert(kClockSlot + sizeof(qw::StepClock) / sizeof(double) <= 256, "step clock outside the scalars slot");

qw::StepClock* step_clock(qw_ctx h)
{
    return reinterpret_cast<qw::StepClock*>(reinterpret_cast<double*>(h->ws + h->lay.scalars) + kClockSlot);
}

// Destroys the captured chunk after waiting for its last replay: a caller
// may change the beam or the state array, or destroy the context, while
// replays it enqueued are still running, and an executable graph must not
// be released under a running replay.
void drop_graph(qw_ctx h)
{
    if (h->exec) {
        if (h->exec_done) (void)hipEventSynchronize(h->exec_done);
        (void)hipGraphExecDestroy(h->exec);
    }
    h->exec = nullptr;
    h->exec_psi = nullptr;
}

// One chunk of kGraphSteps middle steps (column pass, then the row pass
// V(t_k, dt) with k read from the device clock) and the clock's advance,
// captured on the library's own stream; recaptured when the state array it
// works on (the workspace plane), the beam or the frame change.  r and c are the step loop's argument blocks.
hipError_t ensure_graph(qw_ctx h, void* psi, qw::RowArgs r, const qw::ColArgs& c)
{
    if (h->exec && h->exec_psi == psi && h->exec_version == h->args_version) return hipSuccess;
    drop_graph(h);
    hipError_t e = ensure_streams(h);
    if (e != hipSuccess) return e;
    qw::StepClock* clk = step_clock(h);
    r.clock = clk;
    r.t0 = 0.0;
    r.dt = 0.0;
    e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = enqueue_middle(h, h->cap, h->cap_side, h->cap_fork, h->cap_join, r, c, 0, kGraphSteps, false);
    if (le == hipSuccess) le = qw::launch_clock_advance(clk, kGraphSteps, h->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->cap, &g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->exec = nullptr;
        return e;
    }
    h->exec_psi = psi;
    h->exec_version = h->args_version;
    return hipSuccess;
}

}  // namespace

extern "C" {

int qw_workspace_bytes(const qw_grid* g, size_t* bytes)
{
    int rc = check_grid(g);
    if (rc != QW_OK) return rc;
    if (!bytes) return fail(nullptr, QW_E_ARG, "bytes is NULL");
    *bytes = make_layout(*g).total;
    return QW_OK;
}

int qw_init_grid(qw_ctx* out, const qw_grid* g, void* workspace, size_t ws_bytes, void* hip_stream)
{
    if (!out) return fail(nullptr, QW_E_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_grid(g);
    if (rc != QW_OK) return rc;
    Layout lay = make_layout(*g);
    if (!workspace) return fail(nullptr, QW_E_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(nullptr, QW_E_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    if (ws_bytes < lay.total)
        return fail(nullptr, QW_E_WORKSPACE, "workspace has %zu bytes, the grid needs %zu", ws_bytes, lay.total);
    int ws_device = 0;
    {
        std::string msg;
        const int drc = qwh::device_of(workspace, &ws_device, &msg);
        if (drc != QW_OK) return fail(nullptr, drc, "%s", msg.c_str());
    }
    qw_ctx h = new (std::nothrow) qw_ctx_s;
    if (!h) return fail(nullptr, QW_E_DEVICE, "out of host memory");
    h->g = *g;
    h->ws = static_cast<char*>(workspace);
    h->ws_bytes = ws_bytes;
    h->lay = lay;
    h->device = ws_device;
    hipStream_t s = as_stream(hip_stream);
    hipError_t e = f32(h) ? qw::launch_twiddles_f32(h->ws + lay.twx, g->nx, s)
                          : qw::launch_twiddles_f64(h->ws + lay.twx, g->nx, s);
    if (e == hipSuccess)
        e = f32(h) ? qw::launch_twiddles_f32(h->ws + lay.twy, g->ny, s)
                   : qw::launch_twiddles_f64(h->ws + lay.twy, g->ny, s);
    if (e != hipSuccess) {
        fail(nullptr, QW_E_DEVICE, "twiddle kernel: %s", hipGetErrorString(e));
        delete h;
        return QW_E_DEVICE;
    }
    // field tables start as A = 0 until qw_set_beam
    h->b.mode = QW_BEAM_NONE;
    rc = ensure_tables(h, s);
    if (rc != QW_OK) {
        g_init_error = h->err;
        delete h;
        return rc;
    }
    *out = h;
    return QW_OK;
}

int qw_set_beam(qw_ctx h, const qw_beam* b)
{
    if (!h) return fail(nullptr, QW_E_ARG, "context is NULL");
    if (!b) return fail(h, QW_E_ARG, "beam is NULL");
    std::string msg;
    const int rc = qwh::check_beam(*b, &msg);
    if (rc != QW_OK) return fail(h, rc, "%s", msg.c_str());
    h->b = *b;
    h->beam_set = true;
    h->tables_dirty = true;
    ++h->args_version;
    return QW_OK;
}

int qw_set_frame(qw_ctx h, const qw_frame* f)
{
    if (!h) return fail(nullptr, QW_E_ARG, "context is NULL");
    if (!f) return fail(h, QW_E_ARG, "frame is NULL");
    std::string msg;
    const int rc = qwh::check_frame(*f, h->g.c, &msg);
    if (rc != QW_OK) return fail(h, rc, "%s", msg.c_str());
    h->frame = *f;
    ++h->args_version;
    return QW_OK;
}

int qw_init_packet(qw_ctx h, void* psi, const qw_packet* e, void* hip_stream)
{
    if (!h) return fail(nullptr, QW_E_ARG, "context is NULL");
    if (!psi || !e) return fail(h, QW_E_ARG, "psi or packet is NULL");
    std::string msg;
    const int rc = qwh::check_packet(*e, &msg);
    if (rc != QW_OK) return fail(h, rc, "%s", msg.c_str());
    hipStream_t s = as_stream(hip_stream);
    const qw::PacketArgs p = qwh::packet_args(h->g, *e, h->frame.a_m);
    double* rownorm = reinterpret_cast<double*>(h->ws + h->lay.rownorm);
    double* total = reinterpret_cast<double*>(h->ws + h->lay.scalars);
    hipError_t err = f32(h) ? qw::launch_packet_f32(psi, rownorm, p, s) : qw::launch_packet_f64(psi, rownorm, p, s);
    if (err == hipSuccess) err = qw::launch_sum_rows(rownorm, h->g.ny, total, s);
    if (err == hipSuccess) err = launch_col(h, qw::COL_INV, col_args(h, psi), s);
    if (err == hipSuccess) err = launch_row(h, qw::ROW_INV_SCALE, row_args(h, psi, psi), s);
    if (err != hipSuccess) return hip_fail(h, err, "packet kernels");
    return QW_OK;
}

int qw_step_n(qw_ctx h, void* psi, int64_t n, double t0, double dt, void* hip_stream)
{
    if (!h) return fail(nullptr, QW_E_ARG, "context is NULL");
    if (!psi) return fail(h, QW_E_ARG, "psi is NULL");
    if (n < 0) return fail(h, QW_E_ARG, "n = %lld is negative", (long long)n);
    {
        // the propagation runs through the workspace plane: psi must not overlap the workspace
        const char* p = static_cast<const char*>(psi);
        const size_t state = (size_t)h->g.nx * h->g.ny * 4 * (f32(h) ? 8 : 16);
        if (p < h->ws + h->ws_bytes && p + state > h->ws) return fail(h, QW_E_ARG, "psi overlaps the workspace");
    }
    if (!qwh::finite_all({t0, dt})) return fail(h, QW_E_ARG, "t0 and dt must be finite");
    if (!h->beam_set) return fail(h, QW_E_STATE, "qw_set_beam has not been called");
    if (n == 0) return QW_OK;
    if (h->frame.vy != 0.0 && h->b.mode == QW_BEAM_STANDING_PARAXIAL)
        return fail(h, QW_E_STATE, "a moving box needs a field evaluated per cell, not the paraxial tables");
    {
        std::string msg;
        const int rc = qwh::check_phases(h->g, h->b, true, n, t0, dt, &msg, &h->frame);
        if (rc != QW_OK) return fail(h, rc, "%s", msg.c_str());
    }
    hipStream_t s = as_stream(hip_stream);
    int rc = ensure_tables(h, s);
    if (rc == QW_OK) rc = ensure_kinetic_table(h, dt, s);
    if (rc != QW_OK) return rc;
    // Between its first and last row pass a propagation keeps the state in
    // the workspace plane, in the split layout of the middle passes: the first
    // row pass reads psi and writes the plane, the last reads the plane and
    // writes psi.
    void* plane = h->ws + h->lay.plane;
    qw::RowArgs r = row_args(h, plane, plane);
    r.t0 = t0;
    r.dt = dt;
    qw::ColArgs c = col_args(h, plane);
    c.dt = dt;
    hipError_t e;
    // V(t0, dt/2) then F_x
    r.k = 0;
    r.tau_frac = 0.5;
    {
        qw::RowArgs f = r;
        f.src = psi;
        e = timed(h, 0, s, [&] { return launch_row(h, qw::ROW_FIRST, f, s); });
    }
    int64_t k0 = 1;
    // a caller capturing its own stream (or a stream whose state cannot be
    // queried), or per-launch timing, gets plain launches on the caller's
    // stream; otherwise the two blocks' chains (enqueue_middle), replayed as
    // a captured chunk for every kGraphSteps steps
    hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
    bool chains = !h->timing;
    if (chains && hipStreamIsCapturing(s, &cap_status) != hipSuccess) {
        (void)hipGetLastError();
        chains = false;
    }
    chains = chains && cap_status == hipStreamCaptureStatusNone;
    if (e == hipSuccess && chains) e = ensure_streams(h);
    const bool replay = chains && n - 1 >= kGraphSteps;
    if (e == hipSuccess && replay) {
        // middle steps 1 .. chunks kGraphSteps as replays of one captured chunk
        qw::StepClock* clk = step_clock(h);
        e = qw::launch_clock_set(clk, t0, dt, 1, s);
        if (e == hipSuccess) e = ensure_graph(h, plane, r, c);
        const int64_t chunks = (n - 1) / kGraphSteps;
        for (int64_t q = 0; q < chunks && e == hipSuccess; ++q) e = hipGraphLaunch(h->exec, s);
        if (e == hipSuccess) e = hipEventRecord(h->exec_done, s);
        k0 += chunks * kGraphSteps;
    }
    if (e == hipSuccess && chains) {
        // the remaining middle steps and the last column pass, then R_last
        e = enqueue_middle(h, s, h->side, h->fork_ev, h->join_ev, r, c, k0, n - k0, true);
        r.k = n;
        r.tau_frac = 0.5;
        r.dst = psi;
        if (e == hipSuccess) e = launch_row(h, qw::ROW_LAST, r, s);
        k0 = n + 1;
    }
    for (int64_t k = k0; k <= n && e == hipSuccess; ++k) {
        e = timed(h, 1, s, [&] { return launch_col(h, qw::COL_PROP, c, s); });
        if (e != hipSuccess) break;
        r.k = k;
        if (k < n) {
            r.tau_frac = 1.0;  // V(t_k, dt/2) V(t_k, dt/2) = V(t_k, dt)
            e = timed(h, 0, s, [&] { return launch_row(h, qw::ROW_MID, r, s); });
        } else {
            r.tau_frac = 0.5;
            r.dst = psi;
            e = timed(h, 0, s, [&] { return launch_row(h, qw::ROW_LAST, r, s); });
        }
    }
    if (e != hipSuccess) return hip_fail(h, e, "step kernels");
    return QW_OK;
}

int qw_observables(qw_ctx h, const void* psi, const qw_obs_spec* o, double* out_host, int32_t out_len,
                   void* hip_stream)
{
    if (!h) return fail(nullptr, QW_E_ARG, "context is NULL");
    if (!psi || !o || !out_host) return fail(h, QW_E_ARG, "psi, spec or out is NULL");
    {
        std::string msg;
        const int rc = qwh::check_obs(*o, &msg);
        if (rc != QW_OK) return fail(h, rc, "%s", msg.c_str());
    }
    const int nb = 2 * o->n_max + 1;
    if (out_len < 3 * nb + 3) return fail(h, QW_E_ARG, "out_len %d < %d", out_len, 3 * nb + 3);
    hipStream_t s = as_stream(hip_stream);
    void* plane = h->ws + h->lay.plane;
    double* rownorm = reinterpret_cast<double*>(h->ws + h->lay.rownorm);
    double* results = reinterpret_cast<double*>(h->ws + h->lay.scalars) + 8;
    qw::ColArgs c = col_args(h, plane);
    c.band_ref = o->band_ref_idx;
    c.band_half = o->band_half_idx;
    c.window = o->window_idx;
    c.n_max = o->n_max;
    c.spin0 = o->spin0;
    hipError_t e = launch_row(h, qw::ROW_FWD_NORM, row_args(h, psi, plane), s);
    if (e == hipSuccess) e = launch_col(h, qw::COL_OBS, c, s);
    if (e == hipSuccess)
        e = qw::launch_obs_finish(rownorm, h->g.ny, c.partial, col_blocks(h), kPartialStride, o->n_max, results, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, results, sizeof(double) * (3 * nb + 3), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "observables");
    for (int i = 0; i < 3 * nb + 3; ++i)
        if (!std::isfinite(out_host[i])) return fail(h, QW_E_NUMERIC, "observable %d is not finite", i);
    return QW_OK;
}

int qw_momentum_maps(qw_ctx h, const void* psi, double* out, int64_t out_len, void* hip_stream)
{
    if (!h) return fail(nullptr, QW_E_ARG, "context is NULL");
    if (!psi || !out) return fail(h, QW_E_ARG, "psi or out is NULL");
    const int64_t need = (int64_t)h->g.nx * h->g.ny * 3;
    if (out_len < need) return fail(h, QW_E_ARG, "out_len %lld < %lld", (long long)out_len, (long long)need);
    hipStream_t s = as_stream(hip_stream);
    void* plane = h->ws + h->lay.plane;
    qw::ColArgs c = col_args(h, plane);
    c.partial = out;
    hipError_t e = launch_row(h, qw::ROW_FWD_NORM, row_args(h, psi, plane), s);
    if (e == hipSuccess) e = launch_col(h, qw::COL_MAPS, c, s);
    if (e != hipSuccess) return hip_fail(h, e, "momentum maps");
    return QW_OK;
}

int qw_transform_gain(int32_t n, int32_t precision, int32_t batch_variant, double* gain)
{
    if (!gain) return fail(nullptr, QW_E_ARG, "gain is NULL");
    if (precision != QW_F32 && precision != QW_F64) return fail(nullptr, QW_E_ARG, "unknown precision %d", precision);
    const bool single = batch_variant < 0;
    const bool sp = precision == QW_F32;
    int r[16];
    int cnt = 0;
    if (n >= 2 && (n & (n - 1)) == 0) {
        const int lg = qwh::ilog2(n);
        cnt = single ? (sp ? qw::plan_radices_f32(n, r, 16) : qw::plan_radices_f64(n, r, 16))
                     : (sp ? qw::batch_variant_f32(lg, batch_variant, r, 16)
                           : qw::batch_variant_f64(lg, batch_variant, r, 16));
    }
    if (cnt <= 0) return fail(nullptr, QW_E_ARG, "no %s transform of length %d", single ? "plan" : "schedule variant", n);
    *gain = sp ? qwh::transform_gain_f32(r, cnt) : 1.0;
    return QW_OK;
}

int qw_kernel_timing(qw_ctx h, int enable)
{
    if (!h) return fail(nullptr, QW_E_ARG, "context is NULL");
    h->timing = enable != 0;
    return QW_OK;
}

int qw_kernel_times(qw_ctx h, double* out, int32_t out_len, void* hip_stream)
{
    if (!h) return fail(nullptr, QW_E_ARG, "context is NULL");
    if (!out || out_len < 4) return fail(h, QW_E_ARG, "out needs 4 doubles");
    hipError_t e = hipStreamSynchronize(as_stream(hip_stream));
    if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
    double cnt[2] = {0, 0}, ms[2] = {0, 0};
    for (auto& t : h->timed) {
        float v = 0.f;
        if (hipEventElapsedTime(&v, t.a, t.b) == hipSuccess) {
            cnt[t.kind] += 1;
            ms[t.kind] += v;
        }
        h->event_pool.push_back(t.a);
        h->event_pool.push_back(t.b);
    }
    h->timed.clear();
    out[0] = cnt[0];
    out[1] = ms[0];
    out[2] = cnt[1];
    out[3] = ms[1];
    return QW_OK;
}

const char* qw_last_error(qw_ctx h)
{
    if (!h) return g_init_error.c_str();
    return h->err.c_str();
}

void qw_destroy(qw_ctx h)
{
    if (!h) return;
    drop_graph(h);  // waits for the last replay
    if (h->side) (void)hipStreamSynchronize(h->side);
    for (hipEvent_t ev : {h->exec_done, h->fork_ev, h->join_ev, h->cap_fork, h->cap_join})
        if (ev) (void)hipEventDestroy(ev);
    for (hipStream_t st : {h->cap, h->side, h->cap_side})
        if (st) (void)hipStreamDestroy(st);
    for (auto& t : h->timed) {
        // timing brackets still pending on a stream: wait for them first
        (void)hipEventSynchronize(t.b);
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : h->event_pool) (void)hipEventDestroy(e);
    delete h;
}

}  // extern "C"
