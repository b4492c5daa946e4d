// qw_batch.cpp -- host engine of the batched form (qw_batch_* in qw.h):
// layout of the batch state and workspace, the work lists, the tables, the
// launch sequence with its captured step-loop graph, and the autotuner.
// No device memory is allocated here; every launch goes to the caller's
// stream, or to the library's own capture stream while a graph is recorded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "qw.h"
#include "qw_host.hpp"
#include "qw_batch_loop.hpp"
#include "qw_launch.hpp"

namespace {

using qwh::align_up;
using qwh::ilog2;
using qwh::kPartialStride;

constexpr int kScalarsPerInst = 128;  // [0] packet norm, [8 .. 8 + 3B + 3) observables
constexpr int kMaxInstances = 65535;
constexpr int kDefaultGraphSteps = 64;
constexpr int kMaxLg = 12;
// the autotuner times the instance loop only for batches whose instances
// have at most this many tiles per step (a 128^2 FP32 instance has 16)
constexpr int kInstLoopTiles = 16;

struct Prec {
    bool f32;
    size_t cs;  // bytes per complex
    int lg_min, lg_max;
    int variant(int lg, int v, int* r, int m) const
    {
        return f32 ? qw::batch_variant_f32(lg, v, r, m) : qw::batch_variant_f64(lg, v, r, m);
    }
    int lines_per_tile(int lg) const { return f32 ? qw::batch_tiles_f32(lg) : qw::batch_tiles_f64(lg); }
    hipError_t twiddles(void* tw, int lg, int v, hipStream_t s) const
    {
        return f32 ? qw::launch_batch_twiddles_f32(tw, lg, v, s) : qw::launch_batch_twiddles_f64(tw, lg, v, s);
    }
    hipError_t row(int mode, int grid, bool persist, const qw::BatchLaunch& b, hipStream_t s) const
    {
        return f32 ? qw::launch_batch_row_f32(mode, grid, persist, b, s)
                   : qw::launch_batch_row_f64(mode, grid, persist, b, s);
    }
    hipError_t col(int mode, int grid, bool persist, const qw::BatchLaunch& b, hipStream_t s) const
    {
        return f32 ? qw::launch_batch_col_f32(mode, grid, persist, b, s)
                   : qw::launch_batch_col_f64(mode, grid, persist, b, s);
    }
    int loop_blocks_per_cu() const
    {
        return f32 ? qw::batch_loop_blocks_per_cu_f32() : qw::batch_loop_blocks_per_cu_f64();
    }
    hipError_t loop(int grid, const qw::BatchLaunch& c, const qw::BatchLaunch& r, int steps, qw::BatchSync* sync,
                    unsigned long long ticks, hipStream_t s) const
    {
        return f32 ? qw::launch_batch_loop_f32(grid, c, r, steps, sync, ticks, s)
                   : qw::launch_batch_loop_f64(grid, c, r, steps, sync, ticks, s);
    }
    hipError_t inst_loop(int n, const qw::BatchLaunch& c, const qw::BatchLaunch& r, const qw::BatchInstItems* q,
                         int steps, hipStream_t s) const
    {
        return f32 ? qw::launch_batch_inst_loop_f32(n, c, r, q, steps, s)
                   : qw::launch_batch_inst_loop_f64(n, c, r, q, steps, s);
    }
    hipError_t beam(void* bx, void* by, const qw::BeamArgs& a, hipStream_t s) const
    {
        return f32 ? qw::launch_beam_tables_f32(bx, by, a, s) : qw::launch_beam_tables_f64(bx, by, a, s);
    }
    hipError_t kinetic(void* kt, const qw::KineticArgs& k, hipStream_t s) const
    {
        return f32 ? qw::launch_kinetic_table_f32(kt, k, s) : qw::launch_kinetic_table_f64(kt, k, s);
    }
    hipError_t packet(void* psi, double* rownorm, const qw::PacketArgs& e, hipStream_t s) const
    {
        return f32 ? qw::launch_packet_f32(psi, rownorm, e, s) : qw::launch_packet_f64(psi, rownorm, e, s);
    }
};

Prec prec_of(int precision)
{
    const bool f = precision == QW_F32;
    return Prec{f, f ? 8u : 16u, f ? qw::batch_lg_min_f32() : qw::batch_lg_min_f64(),
                f ? qw::batch_lg_max_f32() : qw::batch_lg_max_f64()};
}

int n_variants(const Prec& p, int lg)
{
    int r[8];
    int v = 0;
    while (v < qw::kBatchMaxVariants && p.variant(lg, v, r, 8) > 0) ++v;
    return v;
}

// Byte offsets of everything in the batch workspace, and the work lists.
struct BatchLayout {
    std::vector<int64_t> state_off;
    size_t state_bytes = 0;
    size_t time = 0, sync = 0, inst_items = 0, desc = 0, row_items = 0, col_items = 0, scalars = 0, rownorm = 0, partial = 0, plane = 0;
    std::map<std::pair<int, int>, size_t> tw;             // (lg, variant) -> twiddle table
    std::vector<size_t> bx, by;                           // per instance field tables
    std::map<std::tuple<int, int, double, double, double>, size_t> ktab;  // (nx, ny, lx, ly, c) -> table
    std::vector<size_t> ktab_of;                          // per instance
    std::vector<int> row_base, col_tile_base;             // per instance: first row / first column tile
    std::vector<uint32_t> row_items_h, col_items_h;       // (instance << 16) | tile, grouped by length
    std::vector<qw::BatchInstItems> inst_items_h;         // per instance: its ranges in the two lists
    std::map<int, std::pair<int, int>> row_range, col_range;  // lg -> [first, end) in the lists
    int n_rows = 0, n_col_tiles = 0;
    size_t total = 0;
};

int make_batch_layout(const qw_instance* inst, int n, BatchLayout* L, std::string* msg)
{
    if (!inst) {
        *msg = "instances is NULL";
        return QW_E_ARG;
    }
    if (n < 1 || n > kMaxInstances) {
        *msg = "instance count " + std::to_string(n) + " is not in [1, " + std::to_string(kMaxInstances) + "]";
        return QW_E_ARG;
    }
    const int precision = inst[0].grid.precision;
    if (precision != QW_F32 && precision != QW_F64) {
        *msg = "instance 0: precision is neither QW_F64 nor QW_F32";
        return QW_E_ARG;
    }
    const Prec p = prec_of(precision);
    for (int i = 0; i < n; ++i) {
        std::string m;
        int rc = qwh::check_grid(inst[i].grid, 1 << p.lg_min, 1 << p.lg_max, &m);
        if (rc == QW_OK && inst[i].grid.precision != precision) {
            m = "all instances must share one precision";
            rc = QW_E_ARG;
        }
        if (rc == QW_OK) rc = qwh::check_beam(inst[i].beam, &m);
        if (rc == QW_OK && inst[i].beam.mode == QW_BEAM_GAUSSIAN_FULL) {
            m = "batched instances take the table-driven fields (not QW_BEAM_GAUSSIAN_FULL)";
            rc = QW_E_ARG;
        }
        if (rc != QW_OK) {
            *msg = "instance " + std::to_string(i) + ": " + m;
            return rc;
        }
    }
    // state
    L->state_off.resize(n);
    size_t o = 0;
    for (int i = 0; i < n; ++i) {
        L->state_off[i] = (int64_t)o;
        o = align_up(o + (size_t)inst[i].grid.nx * inst[i].grid.ny * 4 * p.cs);
    }
    L->state_bytes = o;
    // work lists, grouped by length, longest first
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto by_len = [&](bool rows) {
        std::vector<int> v = order;
        std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
            return rows ? inst[a].grid.nx > inst[b].grid.nx : inst[a].grid.ny > inst[b].grid.ny;
        });
        return v;
    };
    L->row_base.assign(n, 0);
    L->col_tile_base.assign(n, 0);
    int rb = 0, cb = 0;
    for (int i = 0; i < n; ++i) {
        L->row_base[i] = rb;
        rb += inst[i].grid.ny;
        L->col_tile_base[i] = cb;
        const int tx = p.lines_per_tile(ilog2(inst[i].grid.ny));
        cb += (inst[i].grid.nx + tx - 1) / tx;
    }
    L->n_rows = rb;
    L->n_col_tiles = cb;
    L->inst_items_h.assign(n, qw::BatchInstItems{});
    for (int i : by_len(true)) {
        const int lg = ilog2(inst[i].grid.nx), rpw = p.lines_per_tile(lg);
        auto it = L->row_range.find(lg);
        if (it == L->row_range.end()) L->row_range[lg] = {(int)L->row_items_h.size(), 0};
        L->inst_items_h[i].row_first = (int)L->row_items_h.size();
        for (int t = 0; t < (inst[i].grid.ny + rpw - 1) / rpw; ++t) L->row_items_h.push_back(((uint32_t)i << 16) | t);
        L->inst_items_h[i].row_end = (int)L->row_items_h.size();
        L->row_range[lg].second = (int)L->row_items_h.size();
    }
    for (int i : by_len(false)) {
        const int lg = ilog2(inst[i].grid.ny), tx = p.lines_per_tile(lg);
        auto it = L->col_range.find(lg);
        if (it == L->col_range.end()) L->col_range[lg] = {(int)L->col_items_h.size(), 0};
        L->inst_items_h[i].col_first = (int)L->col_items_h.size();
        // Column tiles in groups that share 128-byte lines of a row (a cell
        // is 4 complex values), the groups taken alternately from the left
        // and the right: consecutive items run on one XCD at nearly the same
        // time, and columns x and nx - x read the same rows of the kinetic
        // table (indexed by |kx|), which then come from that XCD's L2.
        const int T = (inst[i].grid.nx + tx - 1) / tx;
        const int per_line = std::max(1, (int)(128 / (4 * p.cs)) / tx);
        const int J = (T + per_line - 1) / per_line;
        for (int q = 0; q < J; ++q) {
            const int j = (q & 1) ? J - 1 - (q >> 1) : (q >> 1);
            for (int u = 0; u < per_line && j * per_line + u < T; ++u)
                L->col_items_h.push_back(((uint32_t)i << 16) | (uint32_t)(j * per_line + u));
        }
        L->inst_items_h[i].col_end = (int)L->col_items_h.size();
        L->col_range[lg].second = (int)L->col_items_h.size();
    }
    // workspace
    size_t w = 0;
    auto take = [&](size_t bytes) {
        const size_t at = w;
        w = align_up(w + bytes);
        return at;
    };
    L->time = take(sizeof(qw::StepClock));
    L->sync = take(sizeof(qw::BatchSync));
    L->inst_items = take(sizeof(qw::BatchInstItems) * (size_t)n);
    L->desc = take(sizeof(qw::BatchInst) * (size_t)n);
    L->row_items = take(sizeof(uint32_t) * L->row_items_h.size());
    L->col_items = take(sizeof(uint32_t) * L->col_items_h.size());
    L->scalars = take(sizeof(double) * kScalarsPerInst * (size_t)n);
    L->rownorm = take(sizeof(double) * (size_t)L->n_rows);
    L->partial = take(sizeof(double) * kPartialStride * (size_t)L->n_col_tiles);
    std::vector<int> lgs;
    for (auto& r : L->row_range) lgs.push_back(r.first);
    for (auto& r : L->col_range) lgs.push_back(r.first);
    for (int lg : lgs) {
        const int nv = n_variants(p, lg);
        for (int v = 0; v < nv; ++v)
            if (!L->tw.count({lg, v})) L->tw[{lg, v}] = take(2 * (size_t)(1 << lg) * p.cs);
    }
    L->bx.resize(n);
    L->by.resize(n);
    L->ktab_of.resize(n);
    for (int i = 0; i < n; ++i) {
        const qw_grid& g = inst[i].grid;
        L->bx[i] = take((size_t)g.nx * p.cs);
        L->by[i] = take((size_t)g.ny * p.cs);
        const auto key = std::make_tuple(g.nx, g.ny, g.lx, g.ly, g.c);
        auto it = L->ktab.find(key);
        if (it == L->ktab.end()) it = L->ktab.emplace(key, take((size_t)(g.nx / 2 + 1) * (g.ny / 2 + 1) * p.cs)).first;
        L->ktab_of[i] = it->second;
    }
    L->plane = take(L->state_bytes);
    L->total = w;
    return QW_OK;
}

struct Timed {
    hipEvent_t a, b;
    int kind;
};

}  // namespace

struct qw_batch_s {
    int n = 0;
    Prec p{};
    std::vector<qw_instance> inst;
    BatchLayout lay;
    std::vector<qw::BatchInst> desc;  // host copy of the device descriptors
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int device = 0;
    int n_cu = 256;
    int row_var[kMaxLg + 1] = {};
    int col_var[kMaxLg + 1] = {};
    int row_wg_per_cu = 0, col_wg_per_cu = 0, graph_steps = kDefaultGraphSteps;
    // step loop: 0 off, k > 0 grid-wide loop with k workgroups per CU,
    // QW_LOOP_INSTANCE one workgroup per instance; the bound of a barrier
    // wait in wall-clock ticks
    int loop_wg_per_cu = 0;
    double wall_khz = 1e5;
    unsigned long long spin_ticks = 200000000ull;
    bool ktab_valid = false;
    double ktab_dt = 0.0;
    // captured step-loop graph and what it was captured for
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    // recorded on the caller's stream after the replays of each call (see drop_graph)
    hipEvent_t exec_done = nullptr;
    void* exec_psi = nullptr;
    int exec_steps = 0, exec_rw = -1, exec_cw = -1;
    bool desc_dirty = false;
    bool timing = false;
    std::vector<Timed> timed;
    std::vector<hipEvent_t> pool;
    std::string err;
};

namespace {

thread_local std::string g_batch_error;

int bfail(qw_batch b, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    else g_batch_error = buf;
    return code;
}

int bhip(qw_batch b, hipError_t e, const char* what)
{
    return bfail(b, QW_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

qw::StepClock* dev_time(qw_batch b) { return reinterpret_cast<qw::StepClock*>(b->ws + b->lay.time); }
qw::BatchSync* dev_sync(qw_batch b) { return reinterpret_cast<qw::BatchSync*>(b->ws + b->lay.sync); }
qw::BatchInst* dev_desc(qw_batch b) { return reinterpret_cast<qw::BatchInst*>(b->ws + b->lay.desc); }

// Destroys the captured step loop after waiting for its last replay, which
// the caller may not have waited for (a new schedule, launch shape or state
// array, or qw_batch_destroy, can follow a qw_batch_step_n directly).
void drop_graph(qw_batch b)
{
    if (b->exec) {
        if (b->exec_done) (void)hipEventSynchronize(b->exec_done);
        (void)hipGraphExecDestroy(b->exec);
    }
    b->exec = nullptr;
    b->exec_psi = nullptr;
}

// point every descriptor's tuned tables at the current variants
void apply_variants(qw_batch b)
{
    for (int i = 0; i < b->n; ++i) {
        qw::BatchInst& d = b->desc[i];
        d.row_var = b->row_var[d.lgx];
        d.col_var = b->col_var[d.lgy];
        d.tw_row = b->ws + b->lay.tw.at({d.lgx, d.row_var});
        d.tw_col = b->ws + b->lay.tw.at({d.lgy, d.col_var});
    }
    b->desc_dirty = true;
    b->ktab_valid = false;  // the kinetic tables carry the schedules' norm factors
}

// copy the host descriptors to the workspace; waits, so the host copy may change afterwards
hipError_t upload_desc(qw_batch b, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(dev_desc(b), b->desc.data(), sizeof(qw::BatchInst) * b->n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) b->desc_dirty = false;
    return e;
}

int grid_of(qw_batch b, int n_items, int wg_per_cu)
{
    if (wg_per_cu <= 0) return (n_items + 7) / 8 * 8;  // one workgroup per tile
    const int g = wg_per_cu * b->n_cu;
    return std::max(8, std::min(g, (n_items + 7) / 8 * 8) / 8 * 8);
}

qw::BatchLaunch launch_rows(qw_batch b, char* src, char* dst, int first = 0, int end = -1)
{
    qw::BatchLaunch l{};
    l.inst = dev_desc(b);
    l.items = reinterpret_cast<const uint32_t*>(b->ws + b->lay.row_items) + first;
    l.n_items = (end < 0 ? (int)b->lay.row_items_h.size() : end) - first;
    l.src = src;
    l.dst = dst;
    l.time = dev_time(b);
    return l;
}

qw::BatchLaunch launch_cols(qw_batch b, char* psi, int first = 0, int end = -1)
{
    qw::BatchLaunch l{};
    l.inst = dev_desc(b);
    l.items = reinterpret_cast<const uint32_t*>(b->ws + b->lay.col_items) + first;
    l.n_items = (end < 0 ? (int)b->lay.col_items_h.size() : end) - first;
    l.src = psi;
    l.dst = psi;
    l.time = dev_time(b);
    return l;
}

hipEvent_t pooled_event(qw_batch b)
{
    if (!b->pool.empty()) {
        hipEvent_t e = b->pool.back();
        b->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <typename F>
hipError_t timed(qw_batch b, int kind, hipStream_t s, F&& launch)
{
    if (!b->timing) return launch();
    Timed t{pooled_event(b), pooled_event(b), kind};
    if (!t.a || !t.b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(t.a, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(t.b, s);
    if (e == hipSuccess) b->timed.push_back(t);
    return e;
}

hipError_t row_pass(qw_batch b, int mode, qw::BatchLaunch l, hipStream_t s)
{
    const bool persist = mode == qw::ROW_MID && b->row_wg_per_cu > 0;
    return b->p.row(mode, grid_of(b, l.n_items, persist ? b->row_wg_per_cu : 0), persist, l, s);
}

hipError_t col_pass(qw_batch b, int mode, qw::BatchLaunch l, hipStream_t s)
{
    const bool persist = mode == qw::COL_PROP && b->col_wg_per_cu > 0;
    return b->p.col(mode, grid_of(b, l.n_items, persist ? b->col_wg_per_cu : 0), persist, l, s);
}

int ensure_ktab(qw_batch b, double dt, hipStream_t s)
{
    if (b->ktab_valid && b->ktab_dt == dt) return QW_OK;
    for (auto& kv : b->lay.ktab) {
        const auto& key = kv.first;
        qw_grid g{};
        g.nx = std::get<0>(key);
        g.ny = std::get<1>(key);
        g.lx = std::get<2>(key);
        g.ly = std::get<3>(key);
        g.c = std::get<4>(key);
        qw::KineticArgs k = qwh::kinetic_args(g, dt);
        // the mean loss of norm of the float transforms of the middle passes'
        // schedules, undone in K (see transform_gain_f32)
        const int lgx = ilog2(g.nx), lgy = ilog2(g.ny);
        int rx[16], ry[16];
        const int nrx = b->p.variant(lgx, b->row_var[lgx], rx, 16), nry = b->p.variant(lgy, b->col_var[lgy], ry, 16);
        k.inv_cells *= qwh::kinetic_norm_factor(b->p.f32, rx, nrx, ry, nry);
        const hipError_t e = b->p.kinetic(b->ws + kv.second, k, s);
        if (e != hipSuccess) return bhip(b, e, "kinetic table kernel");
    }
    b->ktab_valid = true;
    b->ktab_dt = dt;
    return QW_OK;
}

// one (column pass, middle row pass) pair; j = step index, from the device
// counter when use_counter
hipError_t middle_step(qw_batch b, char* psi, int j, bool use_counter, hipStream_t s)
{
    hipError_t e = timed(b, 1, s, [&] { return col_pass(b, qw::COL_PROP, launch_cols(b, psi), s); });
    if (e != hipSuccess) return e;
    qw::BatchLaunch r = launch_rows(b, psi, psi);
    r.j = j;
    r.use_counter = use_counter ? 1 : 0;
    r.tau_frac = 1.0;  // V(t_k, dt/2) V(t_k, dt/2) = V(t_k, dt)
    return timed(b, 0, s, [&] { return row_pass(b, qw::ROW_MID, r, s); });
}

// graph of graph_steps middle steps reading the step index from the device
// counter, then advancing it; captured on the library's own stream
hipError_t ensure_graph(qw_batch b, char* psi)
{
    if (b->exec && b->exec_psi == psi && b->exec_steps == b->graph_steps && b->exec_rw == b->row_wg_per_cu &&
        b->exec_cw == b->col_wg_per_cu)
        return hipSuccess;
    drop_graph(b);
    hipError_t e = hipSuccess;
    if (!b->cap) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess && !b->exec_done) e = hipEventCreateWithFlags(&b->exec_done, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int j = 0; j < b->graph_steps && le == hipSuccess; ++j) le = middle_step(b, psi, j, true, b->cap);
    if (le == hipSuccess) le = qw::launch_clock_advance(dev_time(b), b->graph_steps, b->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->exec = nullptr;
        return e;
    }
    b->exec_psi = psi;
    b->exec_steps = b->graph_steps;
    b->exec_rw = b->row_wg_per_cu;
    b->exec_cw = b->col_wg_per_cu;
    return hipSuccess;
}

// steps k .. k + count - 1 as one step-loop launch
hipError_t loop_launch(qw_batch b, char* psi, int64_t k, int count, hipStream_t s)
{
    const qw::BatchLaunch c = launch_cols(b, psi);
    qw::BatchLaunch r = launch_rows(b, psi, psi);
    r.j = (int)k;
    r.use_counter = 0;
    r.tau_frac = 1.0;
    if (b->loop_wg_per_cu == QW_LOOP_INSTANCE)
        return b->p.inst_loop(b->n, c, r, reinterpret_cast<const qw::BatchInstItems*>(b->ws + b->lay.inst_items),
                              count, s);
    const int items = std::max(c.n_items, r.n_items);
    const int grid = std::max(8, std::min(b->loop_wg_per_cu * b->n_cu, (items + 7) / 8 * 8) / 8 * 8);
    return b->p.loop(grid, c, r, count, dev_sync(b), b->spin_ticks, s);
}

// Middle steps k .. end - 1 (the device clock holds t0, dt and k_base = k).
// fast: step-loop launches when the loop is on, else graph replays of
// graph_steps steps while enough remain; the rest, and everything when not
// fast, as direct launches.
hipError_t run_middle(qw_batch b, char* psi, int64_t k, int64_t end, bool fast, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (fast && b->loop_wg_per_cu != 0) {
        const int chunk = b->graph_steps > 0 ? b->graph_steps : kDefaultGraphSteps;
        for (; k < end && e == hipSuccess; k += chunk)
            e = loop_launch(b, psi, k, (int)std::min<int64_t>(chunk, end - k), s);
        return e;
    }
    if (fast && b->graph_steps > 0 && end - k >= b->graph_steps) {
        e = ensure_graph(b, psi);
        const int64_t chunks = (end - k) / b->graph_steps;
        for (int64_t c = 0; c < chunks && e == hipSuccess; ++c) e = hipGraphLaunch(b->exec, s);
        if (e == hipSuccess) e = hipEventRecord(b->exec_done, s);
        k += chunks * b->graph_steps;
    }
    for (; k < end && e == hipSuccess; ++k) e = middle_step(b, psi, (int)k, false, s);
    return e;
}

int check_psi(qw_batch b, const void* psi)
{
    if (!b) return bfail(nullptr, QW_E_ARG, "batch is NULL");
    if (!psi) return bfail(b, QW_E_ARG, "psi is NULL");
    if (reinterpret_cast<uintptr_t>(psi) % qwh::kAlign != 0)
        return bfail(b, QW_E_ARG, "psi must be %zu-byte aligned", qwh::kAlign);
    return QW_OK;
}

}  // namespace

extern "C" {

int qw_batch_layout(const qw_instance* inst, int32_t n, int64_t* offsets, size_t* state_bytes, size_t* ws_bytes)
{
    BatchLayout L;
    std::string msg;
    const int rc = make_batch_layout(inst, n, &L, &msg);
    if (rc != QW_OK) return bfail(nullptr, rc, "%s", msg.c_str());
    if (offsets) std::copy(L.state_off.begin(), L.state_off.end(), offsets);
    if (state_bytes) *state_bytes = L.state_bytes;
    if (ws_bytes) *ws_bytes = L.total;
    return QW_OK;
}

int qw_batch_init(qw_batch* out, const qw_instance* inst, int32_t n, void* workspace, size_t ws_bytes,
                  void* hip_stream)
{
    if (!out) return bfail(nullptr, QW_E_ARG, "out is NULL");
    *out = nullptr;
    BatchLayout L;
    std::string msg;
    int rc = make_batch_layout(inst, n, &L, &msg);
    if (rc != QW_OK) return bfail(nullptr, rc, "%s", msg.c_str());
    if (!workspace) return bfail(nullptr, QW_E_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % qwh::kAlign != 0)
        return bfail(nullptr, QW_E_WORKSPACE, "workspace must be %zu-byte aligned", qwh::kAlign);
    if (ws_bytes < L.total)
        return bfail(nullptr, QW_E_WORKSPACE, "workspace has %zu bytes, the batch needs %zu", ws_bytes, L.total);
    int ws_device = 0;
    {
        std::string msg;
        const int drc = qwh::device_of(workspace, &ws_device, &msg);
        if (drc != QW_OK) return bfail(nullptr, drc, "%s", msg.c_str());
    }
    qw_batch b = new (std::nothrow) qw_batch_s;
    if (!b) return bfail(nullptr, QW_E_DEVICE, "out of host memory");
    b->n = n;
    b->p = prec_of(inst[0].grid.precision);
    b->inst.assign(inst, inst + n);
    b->lay = std::move(L);
    b->ws = static_cast<char*>(workspace);
    b->ws_bytes = ws_bytes;
    b->device = ws_device;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && cu > 0)
        b->n_cu = cu;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device) == hipSuccess && khz > 0)
        b->wall_khz = khz;
    b->spin_ticks = (unsigned long long)(2.0 * 1e3 * b->wall_khz);
    hipStream_t s = as_stream(hip_stream);
    const BatchLayout& Y = b->lay;
    // descriptors
    b->desc.assign(n, qw::BatchInst{});
    for (int i = 0; i < n; ++i) {
        const qw_grid& g = inst[i].grid;
        qw::BatchInst& d = b->desc[i];
        d.lgx = ilog2(g.nx);
        d.lgy = ilog2(g.ny);
        d.off = Y.state_off[i];
        d.scalars = reinterpret_cast<double*>(b->ws + Y.scalars) + (size_t)kScalarsPerInst * i;
        d.ntile_col = (g.nx + b->p.lines_per_tile(d.lgy) - 1) / b->p.lines_per_tile(d.lgy);
        qw::RowArgs& r = d.row;
        r.twx = b->ws + Y.tw.at({d.lgx, 0});
        r.beam_x = b->ws + Y.bx[i];
        r.beam_y = b->ws + Y.by[i];
        r.rownorm = reinterpret_cast<double*>(b->ws + Y.rownorm) + Y.row_base[i];
        r.scale_src = d.scalars;
        qwh::row_field(g, inst[i].beam, true, &r);
        qw::ColArgs& c = d.col;
        c.twy = b->ws + Y.tw.at({d.lgy, 0});
        c.ktab = b->ws + Y.ktab_of[i];
        qwh::col_grid(g, &c);
        c.partial = reinterpret_cast<double*>(b->ws + Y.partial) + (size_t)kPartialStride * Y.col_tile_base[i];
    }
    apply_variants(b);
    hipError_t e = hipSuccess;
    for (auto& kv : Y.tw)
        if (e == hipSuccess) e = b->p.twiddles(b->ws + kv.second, kv.first.first, kv.first.second, s);
    for (int i = 0; i < n && e == hipSuccess; ++i)
        e = b->p.beam(b->ws + Y.bx[i], b->ws + Y.by[i], qwh::beam_args(inst[i].grid, inst[i].beam), s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + Y.row_items, Y.row_items_h.data(), sizeof(uint32_t) * Y.row_items_h.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + Y.col_items, Y.col_items_h.data(), sizeof(uint32_t) * Y.col_items_h.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + Y.inst_items, Y.inst_items_h.data(), sizeof(qw::BatchInstItems) * n,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = qw::launch_clock_set(dev_time(b), 0.0, 0.0, 0, s);
    if (e == hipSuccess) e = hipMemsetAsync(dev_sync(b), 0, sizeof(qw::BatchSync), s);
    if (e == hipSuccess) e = upload_desc(b, s);  // waits for the stream
    if (e != hipSuccess) {
        bfail(nullptr, QW_E_DEVICE, "batch set-up: %s", hipGetErrorString(e));
        delete b;
        return QW_E_DEVICE;
    }
    *out = b;
    return QW_OK;
}

int qw_batch_init_packets(qw_batch b, void* psi, const qw_packet* packets, void* hip_stream)
{
    int rc = check_psi(b, psi);
    if (rc != QW_OK) return rc;
    if (!packets) return bfail(b, QW_E_ARG, "packets is NULL");
    for (int i = 0; i < b->n; ++i) {
        std::string msg;
        rc = qwh::check_packet(packets[i], &msg);
        if (rc != QW_OK) return bfail(b, rc, "packet %d: %s", i, msg.c_str());
    }
    hipStream_t s = as_stream(hip_stream);
    char* base = static_cast<char*>(psi);
    hipError_t e = b->desc_dirty ? upload_desc(b, s) : hipSuccess;
    for (int i = 0; i < b->n && e == hipSuccess; ++i)
        e = b->p.packet(base + b->lay.state_off[i], b->desc[i].row.rownorm,
                        qwh::packet_args(b->inst[i].grid, packets[i]), s);
    if (e == hipSuccess) e = qw::launch_batch_sum_rows(dev_desc(b), b->n, s);
    if (e == hipSuccess) e = col_pass(b, qw::COL_INV, launch_cols(b, base), s);
    if (e == hipSuccess) e = row_pass(b, qw::ROW_INV_SCALE, launch_rows(b, base, base), s);
    if (e != hipSuccess) return bhip(b, e, "packet kernels");
    return QW_OK;
}

int qw_batch_step_n(qw_batch b, void* psi, int64_t n, double t0, double dt, void* hip_stream)
{
    int rc = check_psi(b, psi);
    if (rc != QW_OK) return rc;
    if (n < 0) return bfail(b, QW_E_ARG, "n = %lld is negative", (long long)n);
    if (n > (int64_t)1 << 30) return bfail(b, QW_E_ARG, "n = %lld exceeds 2^30", (long long)n);
    if (!qwh::finite_all({t0, dt})) return bfail(b, QW_E_ARG, "t0 and dt must be finite");
    if (n == 0) return QW_OK;
    for (int i = 0; i < b->n; ++i) {
        std::string msg;
        rc = qwh::check_phases(b->inst[i].grid, b->inst[i].beam, true, n, t0, dt, &msg);
        if (rc != QW_OK) return bfail(b, rc, "instance %d: %s", i, msg.c_str());
    }
    hipStream_t s = as_stream(hip_stream);
    char* base = static_cast<char*>(psi);
    hipError_t e = b->desc_dirty ? upload_desc(b, s) : hipSuccess;
    if (e != hipSuccess) return bhip(b, e, "descriptor upload");
    rc = ensure_ktab(b, dt, s);
    if (rc != QW_OK) return rc;
    // the graph replays start at step 1
    e = qw::launch_clock_set(dev_time(b), t0, dt, 1, s);
    // V(t0, dt/2) then F_x
    qw::BatchLaunch r = launch_rows(b, base, base);
    r.j = 0;
    r.tau_frac = 0.5;
    if (e == hipSuccess) e = timed(b, 0, s, [&] { return row_pass(b, qw::ROW_FIRST, r, s); });
    // a caller capturing its own stream (or a stream whose state cannot be
    // queried) gets the plain launches
    bool fast = !b->timing;
    hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
    if (fast && hipStreamIsCapturing(s, &cap_status) != hipSuccess) {
        (void)hipGetLastError();
        fast = false;
    }
    fast = fast && cap_status == hipStreamCaptureStatusNone;
    if (e == hipSuccess) e = run_middle(b, base, 1, n, fast, s);
    if (e == hipSuccess) e = timed(b, 1, s, [&] { return col_pass(b, qw::COL_PROP, launch_cols(b, base), s); });
    r.j = (int)n;
    if (e == hipSuccess) e = timed(b, 0, s, [&] { return row_pass(b, qw::ROW_LAST, r, s); });
    if (e != hipSuccess) return bhip(b, e, "batched step kernels");
    return QW_OK;
}

int qw_batch_observables(qw_batch b, const void* psi, const qw_obs_spec* specs, double* out_host, int32_t out_len,
                         void* hip_stream)
{
    int rc = check_psi(b, psi);
    if (rc != QW_OK) return rc;
    if (!specs || !out_host) return bfail(b, QW_E_ARG, "specs or out is NULL");
    const int n_max = specs[0].n_max;
    for (int i = 0; i < b->n; ++i) {
        std::string msg;
        rc = qwh::check_obs(specs[i], &msg);
        if (rc == QW_OK && specs[i].n_max != n_max) {
            msg = "every instance must use the same n_max";
            rc = QW_E_ARG;
        }
        if (rc != QW_OK) return bfail(b, rc, "spec %d: %s", i, msg.c_str());
    }
    const int per = 3 * (2 * n_max + 1) + 3;
    if ((int64_t)out_len < (int64_t)per * b->n) return bfail(b, QW_E_ARG, "out_len %d < %d", out_len, per * b->n);
    for (int i = 0; i < b->n; ++i) {
        qw::ColArgs& c = b->desc[i].col;
        c.band_ref = specs[i].band_ref_idx;
        c.band_half = specs[i].band_half_idx;
        c.window = specs[i].window_idx;
        c.n_max = n_max;
        c.spin0 = specs[i].spin0;
    }
    hipStream_t s = as_stream(hip_stream);
    char* src = static_cast<char*>(const_cast<void*>(psi));
    char* plane = b->ws + b->lay.plane;
    hipError_t e = upload_desc(b, s);
    if (e == hipSuccess) e = row_pass(b, qw::ROW_FWD_NORM, launch_rows(b, src, plane), s);
    if (e == hipSuccess) e = col_pass(b, qw::COL_OBS, launch_cols(b, plane), s);
    if (e == hipSuccess) e = qw::launch_batch_obs_finish(dev_desc(b), b->n, kPartialStride, n_max, s);
    std::vector<double> all((size_t)kScalarsPerInst * b->n);
    if (e == hipSuccess)
        e = hipMemcpyAsync(all.data(), b->ws + b->lay.scalars, sizeof(double) * all.size(), hipMemcpyDeviceToHost, s);
    qw::BatchSync sync{};
    if (e == hipSuccess) e = hipMemcpyAsync(&sync, dev_sync(b), sizeof sync, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bhip(b, e, "batched observables");
    if (sync.failed.v) {
        e = hipMemsetAsync(&dev_sync(b)->failed.v, 0, sizeof(unsigned), s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return bhip(b, e, "step loop status reset");
        return bfail(b, QW_E_DEVICE,
                     "a step-loop barrier wait ran past its limit: the launch ended early and psi is not valid");
    }
    bool finite = true;
    for (int i = 0; i < b->n; ++i)
        for (int q = 0; q < per; ++q) {
            const double v = all[(size_t)kScalarsPerInst * i + 8 + q];
            out_host[(size_t)per * i + q] = v;
            finite = finite && std::isfinite(v);
        }
    if (!finite) return bfail(b, QW_E_NUMERIC, "an observable is not finite");
    return QW_OK;
}

int qw_batch_schedule(qw_batch b, int32_t log2n, int32_t v, int32_t* radices, int32_t max_radices)
{
    if (!b) return bfail(nullptr, QW_E_ARG, "batch is NULL");
    if (!radices || max_radices < 0) return bfail(b, QW_E_ARG, "radices is NULL");
    if (log2n < b->p.lg_min || log2n > b->p.lg_max || v < 0) return 0;
    int r[16];
    const int cnt = b->p.variant(log2n, v, r, 16);
    for (int i = 0; i < cnt && i < max_radices; ++i) radices[i] = r[i];
    return cnt;
}

int qw_batch_set_schedule(qw_batch b, int32_t log2n, int32_t pass, int32_t v)
{
    if (!b) return bfail(nullptr, QW_E_ARG, "batch is NULL");
    if (pass != 0 && pass != 1) return bfail(b, QW_E_ARG, "pass must be 0 (rows) or 1 (columns)");
    if (log2n < b->p.lg_min || log2n > b->p.lg_max) return bfail(b, QW_E_ARG, "no batched length 2^%d", log2n);
    if (v < 0 || v >= n_variants(b->p, log2n))
        return bfail(b, QW_E_ARG, "length 2^%d has no schedule variant %d", log2n, v);
    if (!b->lay.tw.count({log2n, v})) return QW_OK;  // no instance has this length
    (pass == 0 ? b->row_var : b->col_var)[log2n] = v;
    apply_variants(b);
    return QW_OK;
}

int qw_batch_set_launch(qw_batch b, int32_t row_wg_per_cu, int32_t col_wg_per_cu, int32_t graph_steps)
{
    if (!b) return bfail(nullptr, QW_E_ARG, "batch is NULL");
    if (row_wg_per_cu < 0 || row_wg_per_cu > 64 || col_wg_per_cu < 0 || col_wg_per_cu > 64)
        return bfail(b, QW_E_ARG, "workgroups per CU must be in [0, 64]");
    if (graph_steps < 0 || graph_steps > 4096) return bfail(b, QW_E_ARG, "graph_steps must be in [0, 4096]");
    b->row_wg_per_cu = row_wg_per_cu;
    b->col_wg_per_cu = col_wg_per_cu;
    b->graph_steps = graph_steps;
    return QW_OK;
}

int qw_batch_set_loop(qw_batch b, int32_t wg_per_cu, double wait_limit_s, int32_t* max_wg_per_cu)
{
    if (!b) return bfail(nullptr, QW_E_ARG, "batch is NULL");
    if (!(wait_limit_s >= 0.0 && wait_limit_s <= 60.0)) return bfail(b, QW_E_ARG, "wait_limit_s must be in [0, 60]");
    int coop = 0;
    hipError_t e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, b->device);
    if (e != hipSuccess) return bhip(b, e, "device attribute");
    const int fit = b->p.loop_blocks_per_cu();
    if (max_wg_per_cu) *max_wg_per_cu = coop ? fit : 0;
    if (wg_per_cu == -1) return QW_OK;
    if (wg_per_cu == QW_LOOP_INSTANCE) {
        b->loop_wg_per_cu = wg_per_cu;
        return QW_OK;
    }
    if (wg_per_cu < 0) return bfail(b, QW_E_ARG, "wg_per_cu must be -1, QW_LOOP_INSTANCE, 0 or positive");
    if (wg_per_cu > 0 && !coop) return bfail(b, QW_E_DEVICE, "the device has no cooperative launches");
    if (wg_per_cu > fit)
        return bfail(b, QW_E_ARG, "wg_per_cu = %d: at most %d step-loop workgroups fit one CU", wg_per_cu, fit);
    b->loop_wg_per_cu = wg_per_cu;
    b->spin_ticks = (unsigned long long)((wait_limit_s > 0.0 ? wait_limit_s : 2.0) * 1e3 * b->wall_khz);
    return QW_OK;
}

int qw_batch_autotune(qw_batch b, const void* psi, double dt, int32_t reps, double* report, int32_t report_len,
                      int32_t* n_rows, void* hip_stream)
{
    int rc = check_psi(b, psi);
    if (rc != QW_OK) return rc;
    if (reps < 1 || reps > 10000) return bfail(b, QW_E_ARG, "reps must be in [1, 10000]");
    if (!qwh::finite_all({dt})) return bfail(b, QW_E_ARG, "dt must be finite");
    if (report_len > 0 && !report) return bfail(b, QW_E_ARG, "report is NULL");
    // the middle-step candidates run (reps + 1) chunks of steps
    const int chunk = b->graph_steps > 0 ? b->graph_steps : kDefaultGraphSteps;
    for (int i = 0; i < b->n; ++i) {
        std::string msg;
        rc = qwh::check_phases(b->inst[i].grid, b->inst[i].beam, true, (int64_t)(reps + 1) * chunk + 1, 0.0, dt, &msg);
        if (rc != QW_OK) return bfail(b, rc, "instance %d: %s", i, msg.c_str());
    }
    hipStream_t s = as_stream(hip_stream);
    char* plane = b->ws + b->lay.plane;
    const bool was_timing = b->timing;
    b->timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipError_t e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    if (e == hipSuccess) e = hipMemcpyAsync(plane, psi, b->lay.state_bytes, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) rc = ensure_ktab(b, dt, s);
    if (e == hipSuccess && rc == QW_OK) e = qw::launch_clock_set(dev_time(b), 0.0, dt, 0, s);
    int rows = 0;
    auto put = [&](double kind, double a, double v, double us) {
        if (report && (rows + 1) * 4 <= report_len) {
            report[4 * rows + 0] = kind;
            report[4 * rows + 1] = a;
            report[4 * rows + 2] = v;
            report[4 * rows + 3] = us;
        }
        ++rows;
    };
    // microseconds per launch of f, averaged over reps after one warm-up
    auto time_it = [&](auto&& f) -> double {
        hipError_t le = f();
        if (le == hipSuccess) le = hipEventRecord(ev0, s);
        for (int i = 0; i < reps && le == hipSuccess; ++i) le = f();
        if (le == hipSuccess) le = hipEventRecord(ev1, s);
        if (le == hipSuccess) le = hipEventSynchronize(ev1);
        float ms = 0.f;
        if (le == hipSuccess) le = hipEventElapsedTime(&ms, ev0, ev1);
        if (le != hipSuccess) {
            e = le;
            return 1e30;
        }
        return 1e3 * (double)ms / reps;
    };
    const int save_rw = b->row_wg_per_cu, save_cw = b->col_wg_per_cu;
    b->row_wg_per_cu = 0;
    b->col_wg_per_cu = 0;
    // schedules, per pass and length, on the tiles of that length only
    for (int pass = 0; pass < 2 && e == hipSuccess && rc == QW_OK; ++pass) {
        const auto& ranges = pass == 0 ? b->lay.row_range : b->lay.col_range;
        int* var = pass == 0 ? b->row_var : b->col_var;
        for (auto& kv : ranges) {
            const int lg = kv.first;
            double best = 1e30;
            int best_v = 0;
            for (int v = 0; v < n_variants(b->p, lg) && e == hipSuccess; ++v) {
                var[lg] = v;
                apply_variants(b);
                e = upload_desc(b, s);
                if (e != hipSuccess) break;
                double us;
                if (pass == 0) {
                    qw::BatchLaunch l = launch_rows(b, plane, plane, kv.second.first, kv.second.second);
                    l.j = 1;
                    l.tau_frac = 1.0;
                    us = time_it([&] { return row_pass(b, qw::ROW_MID, l, s); });
                } else {
                    const qw::BatchLaunch l = launch_cols(b, plane, kv.second.first, kv.second.second);
                    us = time_it([&] { return col_pass(b, qw::COL_PROP, l, s); });
                }
                put(pass, lg, v, us);
                if (us < best) {
                    best = us;
                    best_v = v;
                }
            }
            var[lg] = best_v;
        }
    }
    if (e == hipSuccess) {
        apply_variants(b);
        e = upload_desc(b, s);
    }
    // launch shapes over the whole batch
    const int shapes[] = {0, 1, 2, 4, 8};
    int best_rw = 0, best_cw = 0;
    for (int pass = 0; pass < 2 && e == hipSuccess && rc == QW_OK; ++pass) {
        double best = 1e30;
        for (int w : shapes) {
            double us;
            if (pass == 0) {
                b->row_wg_per_cu = w;
                qw::BatchLaunch l = launch_rows(b, plane, plane);
                l.j = 1;
                l.tau_frac = 1.0;
                us = time_it([&] { return row_pass(b, qw::ROW_MID, l, s); });
            } else {
                b->col_wg_per_cu = w;
                const qw::BatchLaunch l = launch_cols(b, plane);
                us = time_it([&] { return col_pass(b, qw::COL_PROP, l, s); });
            }
            if (e != hipSuccess) break;
            put(2 + pass, w, 0, us);
            if (us < best) {
                best = us;
                (pass == 0 ? best_rw : best_cw) = w;
            }
        }
    }
    b->row_wg_per_cu = e == hipSuccess ? best_rw : save_rw;
    b->col_wg_per_cu = e == hipSuccess ? best_cw : save_cw;
    // middle steps with the chosen shapes: graph replays (0) against the step
    // loop at every workgroup count per CU that fits, per step over chunks
    const int save_loop = b->loop_wg_per_cu;
    int best_loop = 0;
    if (e == hipSuccess && rc == QW_OK) {
        int coop = 0;
        if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, b->device) != hipSuccess) coop = 0;
        const int fit = coop ? b->p.loop_blocks_per_cu() : 0;
        std::vector<int> cand;
        for (int w = 0; w <= fit; ++w) cand.push_back(w);
        // one workgroup per instance walks the instance's tiles one after
        // another: timed only where no instance has more than kInstLoopTiles
        int most = 0;
        for (const auto& q : b->lay.inst_items_h)
            most = std::max(most, q.row_end - q.row_first + q.col_end - q.col_first);
        if (most <= kInstLoopTiles) cand.push_back(QW_LOOP_INSTANCE);
        double best = 1e30;
        for (int w : cand) {
            if (e != hipSuccess) break;
            b->loop_wg_per_cu = w;
            e = qw::launch_clock_set(dev_time(b), 0.0, dt, 1, s);
            if (e != hipSuccess) break;
            const double us = time_it([&] { return run_middle(b, plane, 1, 1 + chunk, true, s); }) / chunk;
            if (e != hipSuccess) break;
            put(4, w, 0, us);
            if (us < best) {
                best = us;
                best_loop = w;
            }
        }
    }
    b->loop_wg_per_cu = e == hipSuccess ? best_loop : save_loop;
    b->timing = was_timing;
    drop_graph(b);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (rc != QW_OK) return rc;
    if (e != hipSuccess) return bhip(b, e, "autotune");
    if (n_rows) *n_rows = rows;
    return QW_OK;
}

int qw_batch_kernel_timing(qw_batch b, int enable)
{
    if (!b) return bfail(nullptr, QW_E_ARG, "batch is NULL");
    b->timing = enable != 0;
    return QW_OK;
}

int qw_batch_kernel_times(qw_batch b, double* out, int32_t out_len, void* hip_stream)
{
    if (!b) return bfail(nullptr, QW_E_ARG, "batch is NULL");
    if (!out || out_len < 4) return bfail(b, QW_E_ARG, "out needs 4 doubles");
    hipError_t e = hipStreamSynchronize(as_stream(hip_stream));
    if (e != hipSuccess) return bhip(b, e, "stream synchronize");
    double cnt[2] = {0, 0}, ms[2] = {0, 0};
    for (auto& t : b->timed) {
        float v = 0.f;
        if (hipEventElapsedTime(&v, t.a, t.b) == hipSuccess) {
            cnt[t.kind] += 1;
            ms[t.kind] += v;
        }
        b->pool.push_back(t.a);
        b->pool.push_back(t.b);
    }
    b->timed.clear();
    out[0] = cnt[0];
    out[1] = ms[0];
    out[2] = cnt[1];
    out[3] = ms[1];
    return QW_OK;
}

const char* qw_batch_last_error(qw_batch b)
{
    if (!b) return g_batch_error.c_str();
    return b->err.c_str();
}

void qw_batch_destroy(qw_batch b)
{
    if (!b) return;
    drop_graph(b);  // waits for the last replay
    if (b->exec_done) (void)hipEventDestroy(b->exec_done);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (auto& t : b->timed) {
        (void)hipEventSynchronize(t.b);  // a pending timing bracket
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : b->pool) (void)hipEventDestroy(e);
    delete b;
}

}  // extern "C"
