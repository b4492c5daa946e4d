// qw_kernels.inl -- the HIP kernels of the split-operator step, templated on the
// arithmetic type T (float or double) and the transform lengths.  Included by
// qw_kernels_f32.hip and qw_kernels_f64.hip, which instantiate one precision
// each.
//
// Data layout in HBM: psi[ny][nx][4] complex T, x fastest.  Between the
// kernels of one qw_step_n call the array holds the mixed representation
// (kx, y): row passes transform along x, column passes along y.
//
//   row pass    (one workgroup = RPW whole rows):
//       load row -> [F_x^-1] -> V(t, tau) -> [F_x] -> store
//   column pass (one workgroup = TX whole columns):
//       load columns -> F_y -> K(dt)/(nx ny) -> F_y^-1 -> store
//
// Each pass reads and writes the state once: 64 B per cell per pass in FP32,
// 128 B in FP64.
#pragma once
#include "qw_device.hpp"
#include "qw_launch.hpp"

// Tuning constants (measured best on MI355X at 2048^2):
//  - per-lane-group LDS buffer padding in elements (row / column passes);
//  - columns per workgroup once a column needs >= 128 lanes;
//  - minimum waves per SIMD the register allocation must allow: 3 for the
//    float passes (at most 168 VGPRs: three 256-lane workgroups per CU), 2
//    for the double row passes (two 256-lane workgroups per CU, no spills),
//    4 for the double column passes.
#ifndef QW_LDS_EXTRA_ROW
#define QW_LDS_EXTRA_ROW 8
#endif
#ifndef QW_LDS_EXTRA_COL
#define QW_LDS_EXTRA_COL 4
#endif
#ifndef QW_TX_COL
#define QW_TX_COL 1
#endif
#ifndef QW_WPE_ROW
#define QW_WPE_ROW 3
#endif
#ifndef QW_WPE_ROW_F64
#define QW_WPE_ROW_F64 2
#endif
#ifndef QW_WPE_COL
#define QW_WPE_COL 3
#endif
#ifndef QW_WPE_COL_F64
#define QW_WPE_COL_F64 4
#endif
// twiddle prefetch in the column passes (it fits the float column pass's
// 168 VGPRs without spilling)
#ifndef QW_TW_PREFETCH_COL
#define QW_TW_PREFETCH_COL 1
#endif

namespace qw {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kTwoPi = 6.28318530717958647692528676655900577;

// ---------------------------------------------------------------------------
// transform plans: elements per thread E and the radix schedule per length
// ---------------------------------------------------------------------------
template <typename T, int N>
struct plan;

#define QW_PLAN(TYPE, NN, EE, ...)                 \
    template <>                                     \
    struct plan<TYPE, NN> {                         \
        static constexpr int E = EE;                \
        using S = sched<__VA_ARGS__>;               \
    };

QW_PLAN(float, 8, 8, 8)
QW_PLAN(float, 16, 16, 16)
QW_PLAN(float, 32, 16, 8, 4)
QW_PLAN(float, 64, 16, 16, 4)
QW_PLAN(float, 128, 16, 16, 8)
QW_PLAN(float, 256, 16, 16, 16)
QW_PLAN(float, 512, 16, 16, 8, 4)
QW_PLAN(float, 1024, 16, 16, 16, 4)
QW_PLAN(float, 2048, 16, 16, 16, 8)
QW_PLAN(float, 4096, 16, 16, 16, 16)
QW_PLAN(double, 8, 8, 8)
QW_PLAN(double, 16, 8, 4, 4)
QW_PLAN(double, 32, 8, 8, 4)
QW_PLAN(double, 64, 8, 8, 8)
QW_PLAN(double, 128, 8, 8, 4, 4)
QW_PLAN(double, 256, 8, 8, 8, 4)
QW_PLAN(double, 512, 8, 8, 8, 8)
QW_PLAN(double, 1024, 8, 8, 8, 4, 4)
QW_PLAN(double, 2048, 8, 8, 8, 8, 4)
QW_PLAN(double, 4096, 8, 8, 8, 8, 8)
#undef QW_PLAN

// Lanes come in pairs over the same cells: lane 2q + 0 holds spin block A as
// (top, bot) = (psi1, psi4), lane 2q + 1 block B as (top, bot) = (psi3, psi2).
// Each lane loads one contiguous half cell -- (psi1, psi2) or (psi3, psi4) --
// and the pair swaps its second values, so every load and store instruction
// of a wave covers contiguous memory.  A line of length N takes L = 2 N/E
// lanes and each lane keeps 2 E complex values in registers.
template <typename T, int N, typename S = typename plan<T, N>::S>
struct tw_len_of;
template <typename T, int N, int... R>
struct tw_len_of<T, N, sched<R...>> {
    static constexpr int value = tw_len<1, R...>::value;
};

template <typename T, int N>
struct shape {
    static constexpr int E = plan<T, N>::E;
    static constexpr int NT = N / E;                                  // lanes per line and block
    static constexpr int L = 2 * NT;                                  // lanes per line
    static constexpr int RPW = L >= 256 ? 1 : 256 / L;                // rows per workgroup
    static constexpr int RT = NT >= 256 ? 1 : 256 / NT;               // rows of one block per middle row tile
    static constexpr int TX = L >= 512 ? 1 : (L >= 128 ? QW_TX_COL : 256 / L);  // columns per workgroup
    // columns of one block per middle column tile: two, so a tile reads whole
    // lines of the split layout (one-column tiles halve the double column
    // pass's rate at 2048^2: 152 -> 240 us)
    static constexpr int CT = 2 * TX;
    // per-lane-group LDS buffer strides (elements); the extra elements move
    // the groups' buffers onto different banks
    static constexpr int LLR = lds_len<T, N>::value + QW_LDS_EXTRA_ROW;
    static constexpr int LLC = lds_len<T, N>::value + QW_LDS_EXTRA_COL;
};

// ---------------------------------------------------------------------------
// scalar helpers
// ---------------------------------------------------------------------------
// time factor of the standing wave: f(t) cos(w t), f = sin^2(pi t / (2 T_r)) for t < T_r
__device__ __forceinline__ double field_time_factor(int mode, double t, double omega, double t_ramp, double ramp_k)
{
    if (mode != QW_BEAM_STANDING_PARAXIAL_) return 1.0;
    double f = 1.0, s, c;
    if (t_ramp > 0.0 && t < t_ramp) {
        sincos_phase(ramp_k * t, s, c);
        f = s * s;
    }
    sincos_phase(omega * t, s, c);
    return f * c;
}

// Interaction propagator coefficients for A = (ax, ay) acting for tau:
// C = cos(th), S = sin(th)/|A| = (c tau) sin(th)/th with th = c |A| tau.
// SERIES 2 (th^2 <= 0.01) and 1 (th^2 <= 0.49, which covers every field of
// interest at these time steps): the even series in th^2, short or long,
// with no sqrt and no division, exact at |A| = 0.  SERIES 0: the reduced
// sin/cos and one division.  The choice is made once per row from a bound
// on |A|, so each variant is straight-line.
template <int SERIES, typename T>
__device__ __forceinline__ void interaction_coeffs(T ax, T ay, T ctau, T& C, T& S)
{
    const T a2 = fmx(ax, ax, ay * ay);
    if constexpr (SERIES == 2) {
        T sc;
        cos_sinc_short(ctau * ctau * a2, C, sc);
        S = ctau * sc;
    } else if constexpr (SERIES == 1) {
        T sc;
        cos_sinc_series(ctau * ctau * a2, C, sc);
        S = ctau * sc;
    } else {
        const T amag = sqrt(a2);
        T sn;
        sincos_small(ctau * amag, sn, C);
        S = amag > (T)0 ? sn / amag : ctau;
    }
}

template <int SERIES, typename T, int E, int NT>
__device__ __forceinline__ void apply_interaction(cx<T> (&v)[2][E], const cx<T>* bxt, int t, T ax_row, T ay_row,
                                                  T ctau)
{
    asm volatile("" ::: "memory");  // table loads stay here, not in the transform above
    int tt = t;
    asm volatile("" : "+v"(tt));
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const cx<T> xb = bxt[tt + NT * m];
        const T ax = ax_row * xb.im, ay = ay_row * xb.re;
        T C, Sn;
        interaction_coeffs<SERIES>(ax, ay, ctau, C, Sn);
        block_prop0(v[0][m], v[1][m], C, Sn * ax, Sn * ay);
    }
}

// The full Gaussian-beam standing wave (Sec. II.A, Eq. 1-4) at z = 0, per
// cell in double.  With Phi = kL x - G + x y^2/(xR w^2), G = atan(x/xR), the
// sums over the two beams d = +-1 of Eq. 1b and 1a are
//   A_y = -2 A0 (w0/w) exp(-y^2/w^2) sin(w t) cos(Phi),
//   A_x = -4 A0 eps (w0/w) (y/w) exp(-y^2/w^2) sin(w t) sin(Phi - G),
// times the switch-on f(t); y is the lab coordinate of the row.
template <typename T, int E, int NT>
__device__ __forceinline__ void apply_full_beam(cx<T> (&v)[2][E], const RowArgs& a, int y, int t, double tk, T ctau)
{
    const FullBeam& b = a.full;
    double st, ct;
    sincos_phase(a.omega * tk, st, ct);
    if (a.t_ramp > 0.0 && tk < a.t_ramp) {
        double rs, rc;
        sincos_phase(a.ramp_k * tk, rs, rc);
        st *= rs * rs;
    }
    const double yl = b.y_min + b.dy * (double)y + b.vy * tk;
    const double y2 = yl * yl;
    int tt = t;
    asm volatile("" : "+v"(tt));
#pragma unroll 2
    for (int m = 0; m < E; ++m) {
        const double x = b.x_min + b.dx * (double)(tt + NT * m);
        const double q = x / b.xr;
        const double u = 1.0 + q * q;               // (w/w0)^2
        const double w2 = b.w0 * b.w0 * u;
        const double g = atan(q);
        const double env = exp(-y2 / w2) / sqrt(u) * st;
        const double phi = b.kl * x - g + x * y2 / (b.xr * w2);
        double sp, cp, s1, c1;
        sincos_phase(phi, sp, cp);
        sincos_phase(phi - g, s1, c1);
        const T ay = (T)(-2.0 * b.a0 * env * cp);
        const T ax = b.longitudinal ? (T)(-4.0 * b.a0 * b.eps * env * (yl / sqrt(w2)) * s1) : (T)0;
        T C, Sn;
        interaction_coeffs<0>(ax, ay, ctau, C, Sn);
        block_prop0(v[0][m], v[1][m], C, Sn * ax, Sn * ay);
    }
}

__device__ __forceinline__ int signed_idx(int k, int n) { return k < n / 2 ? k : k - n; }

// ---------------------------------------------------------------------------
// State layouts.  LAY_ABI is the boundary's psi[ny][nx][4].  LAY_SPLIT is the
// layout a propagation keeps between its first and last row pass: the two
// Dirac blocks in separate planes (block A = (psi1, psi4) first, block B =
// (psi3, psi2) second, each a "block cell" of two complex values), and each
// 128-byte line of a plane holding an LX x LY patch of block cells:
//   byte(b, y, x) = b nx ny BC + ((y / LY) (nx / LX) + x / LX) 128 + ((y % LY) LX + x % LX) BC.
// LX = 2 in both precisions, so a column workgroup of two columns of one
// block moves whole lines (float: 2 x 4 patches; double: 2 x 2).  A row
// workgroup of two rows of one block moves whole lines in double and half
// lines in float, whose other halves the partner tile (the next two rows)
// moves on the same XCD at the same time (row_pass).  No lane swaps the
// halves of a cell.
// ---------------------------------------------------------------------------
enum { LAY_ABI = 0, LAY_SPLIT = 1 };

template <typename T>
struct split_geom {
    static constexpr int BC = 2 * (int)sizeof(cx<T>);  // bytes per block cell
    static constexpr int LY = sizeof(T) == sizeof(float) ? 4 : 2;  // block cells along y per line
    static constexpr int LX = 128 / (BC * LY);                     // block cells along x per line
};

template <typename T>
__device__ __forceinline__ uint32_t split_off(int b, int y, int x, int nx, int ny)
{
    using G = split_geom<T>;
    return (uint32_t)b * (uint32_t)nx * (uint32_t)ny * G::BC +
           ((uint32_t)(y / G::LY) * (uint32_t)(nx / G::LX) + (uint32_t)(x / G::LX)) * 128u +
           (uint32_t)(((y % G::LY) * G::LX + (x % G::LX)) * G::BC);
}

// ---------------------------------------------------------------------------
// row pass
// ---------------------------------------------------------------------------
// One tile of RPW rows of length N (transform with E elements per lane and
// the radix schedule SCH, LDS stride LL per lane group), threads
// 0 .. RPW 2 N/E - 1.  lds holds RPW 2 LL elements.  IN and OUT are the
// layouts read and written.  With both LAY_SPLIT the tile is RT rows of one
// block (RT = shape::RT: 1 when a row takes 256 or more lanes; else lane
// 2q + r: row parity r); otherwise RPW rows of both blocks (lane 2q + b:
// block b).  Lane 2q + j uses LDS group 2 s + j (lane t: group 0 if RT = 1).
template <typename T, int N, int E, typename SCH, int RPW, int LL, int MODE, int BEAM = 0, int IN = LAY_ABI,
          int OUT = LAY_ABI, bool ONE = false>
__device__ __forceinline__ void row_tile(const RowArgs& a, int tile, cx<T>* lds, int tid)
{
    constexpr int NT = N / E, L = 2 * NT;
    constexpr bool SPLIT_MAP = IN == LAY_SPLIT && OUT == LAY_SPLIT;
    constexpr int RT = SPLIT_MAP ? shape<T, N>::RT : 2 * RPW;
    using G = split_geom<T>;
    const int lo = RT >= 2 ? tid & 1 : 0;
    const int q = RT >= 2 ? tid >> 1 : tid;
    const int s = q / NT;
    const int t = q - s * NT;
    int blk, y;
    if constexpr (SPLIT_MAP) {
        const int tpb = (a.ny + RT - 1) / RT;  // tiles per block
        blk = ONE ? a.one_block - 1 : (tile >= tpb ? 1 : 0);
        y = (ONE ? tile : tile - blk * tpb) * RT + 2 * s + lo;
    } else {
        blk = lo;  // 0: (psi1, psi4), 1: (psi3, psi2)
        y = tile * RPW + s;
    }
    const bool live = y < a.ny;
    cx<T>* lb = lds + (2 * s + lo) * LL;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.twx);
    // byte offsets: lane (y, t, block) plus m NT cells per element; a
    // non-live row is pointed past the array (reads zero, writes dropped)
    constexpr uint32_t CB = 4 * sizeof(cx<T>);  // bytes per cell
    const uint32_t bytes = (uint32_t)a.ny * N * CB;
    const uint32_t lane = live ? ((uint32_t)y * N + t) * CB + blk * (CB / 2) : bytes;
    // split layout: element m at x = t + NT m; linear in m when NT is a whole number of lines
    constexpr bool SPLIT_LINEAR = NT % G::LX == 0;
    const uint32_t slane = live ? split_off<T>(blk, y, t, N, a.ny) : bytes;
    constexpr uint32_t SSTEP = (uint32_t)(NT / G::LX) * 128u;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.src, bytes);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(a.dst, bytes);

    cx<T> v[2][E];
    if constexpr (IN == LAY_ABI) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            cx<T> f;
            bload2((cx<T>*)nullptr, rs, lane, m * NT * CB, v[0][m], f);
            v[1][m] = swap_lane_pair(f);
        }
    } else if constexpr (SPLIT_LINEAR) {
#pragma unroll
        for (int m = 0; m < E; ++m) bload2((cx<T>*)nullptr, rs, slane, m * SSTEP, v[0][m], v[1][m]);
    } else {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const uint32_t o = live ? split_off<T>(blk, y, t + NT * m, N, a.ny) : bytes;
            bload2((cx<T>*)nullptr, rs, o, 0, v[0][m], v[1][m]);
        }
    }

    if constexpr (MODE == ROW_FWD_NORM) {
        // sum |psi|^2 of this row in double (fixed tree over the row's lanes)
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < E; ++m)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                acc += (double)v[c][m].re * (double)v[c][m].re + (double)v[c][m].im * (double)v[c][m].im;
        double* red = reinterpret_cast<double*>(lds);
        red[tid] = acc;
        __syncthreads();
        const int l = tid - s * L;
        for (int w = L / 2; w > 0; w >>= 1) {
            if (l < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (l == 0 && live) a.rownorm[y] = red[tid];
        __syncthreads();
    }

    if constexpr (MODE == ROW_MID || MODE == ROW_LAST || MODE == ROW_INV_SCALE)
        fft<T, N, E, 2, true>(SCH{}, v, t, tw, lb);

    if constexpr ((MODE == ROW_FIRST || MODE == ROW_MID || MODE == ROW_LAST) && BEAM == 1) {
        // interaction propagator V(t, tau) with the full beam evaluated per cell
        const double tk = a.t0 + (double)a.k * a.dt;
        apply_full_beam<T, E, NT>(v, a, live ? y : 0, t, tk, (T)(a.c * a.tau_frac * a.dt));
    } else if constexpr (MODE == ROW_FIRST || MODE == ROW_MID || MODE == ROW_LAST) {
        // interaction propagator V(t, tau) with A evaluated from the field tables;
        // |A|^2 <= s(t)^2 (Y0^2 + Y1^2) on this row bounds the angle
        const double tk = a.t0 + (double)a.k * a.dt;
        const T sfac = (T)field_time_factor(a.beam_mode, tk, a.omega, a.t_ramp, a.ramp_k);
        const T ctau = (T)(a.c * a.tau_frac * a.dt);
        const cx<T>* bxt = reinterpret_cast<const cx<T>*>(a.beam_x);
        const cx<T> yb = reinterpret_cast<const cx<T>*>(a.beam_y)[live ? y : 0];
        const T ay_row = sfac * yb.re, ax_row = sfac * yb.im;
        const T bound = ctau * ctau * (ay_row * ay_row + ax_row * ax_row);
        if (bound <= (T)0.01) apply_interaction<2, T, E, NT>(v, bxt, t, ax_row, ay_row, ctau);
        else if (bound <= (T)0.49) apply_interaction<1, T, E, NT>(v, bxt, t, ax_row, ay_row, ctau);
        else apply_interaction<0, T, E, NT>(v, bxt, t, ax_row, ay_row, ctau);
    }

    if constexpr (MODE == ROW_INV_SCALE) {
        // normalise the initial packet: sum |psi|^2 = nx ny sum |phi|^2
        const T sc = (T)(1.0 / sqrt(a.scale_src[0] * (double)N * (double)a.ny));
#pragma unroll
        for (int m = 0; m < E; ++m)
#pragma unroll
            for (int c = 0; c < 2; ++c) v[c][m] = scale(v[c][m], sc);
    }

    if constexpr (MODE == ROW_FIRST || MODE == ROW_MID || MODE == ROW_FWD_NORM)
        fft<T, N, E, 2, false>(SCH{}, v, t, tw, lb);

    if constexpr (OUT == LAY_ABI) {
#pragma unroll
        for (int m = 0; m < E; ++m) bstore2(v[0][m], swap_lane_pair(v[1][m]), rd, lane, m * NT * CB);
    } else if constexpr (SPLIT_LINEAR) {
#pragma unroll
        for (int m = 0; m < E; ++m) bstore2(v[0][m], v[1][m], rd, slane, m * SSTEP);
    } else {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const uint32_t o = live ? split_off<T>(blk, y, t + NT * m, N, a.ny) : bytes;
            bstore2(v[0][m], v[1][m], rd, o, 0);
        }
    }
}

// ONE: the launch covers the block a.one_block only (a separate symbol, so a
// kernel trace tells the per-block launches from the whole-state ones)
// lane groups (one per row and block, NT lanes and one LDS buffer each) and
// threads of a row-pass workgroup: the middle passes take RT rows of one
// block, the others RPW rows of both blocks
template <typename T, int N, int MODE>
struct row_wg {
    using S = shape<T, N>;
    static constexpr int groups = MODE == ROW_MID ? S::RT : 2 * S::RPW;
    static constexpr int threads = groups * S::NT;
};

template <typename T, int N, int MODE, int BEAM = 0, bool ONE = false>
__global__ __launch_bounds__((row_wg<T, N, MODE>::threads)) __attribute__((
    amdgpu_waves_per_eu(sizeof(T) == sizeof(float) ? QW_WPE_ROW : QW_WPE_ROW_F64))) void row_pass(RowArgs a)
{
    using S = shape<T, N>;
    __shared__ cx<T> lds[row_wg<T, N, MODE>::groups * S::LLR];
    if (a.clock) {  // a replayed chunk of steps: its time is kept on the device
        a.t0 = a.clock->t0;
        a.dt = a.clock->dt;
        a.k += a.clock->k_base;
    }
    // a propagation keeps the split layout from its first row pass to its last
    constexpr int IN = (MODE == ROW_MID || MODE == ROW_LAST) ? LAY_SPLIT : LAY_ABI;
    constexpr int OUT = (MODE == ROW_FIRST || MODE == ROW_MID) ? LAY_SPLIT : LAY_ABI;
    // Passes that read or write the split layout: when a tile has fewer rows
    // (RT rows of one block in the middle passes, RPW rows of both blocks in
    // the first and last) than a line of the split layout (LY), the GR = LY /
    // rows tiles GR P .. GR P + GR - 1 share every line.  Workgroups are
    // dealt round-robin to the 8 XCDs, so the group goes to the workgroups
    // an XCD receives one after the other (blockIdx b, b + 8, ...): they run
    // together, and the lines they share meet in that XCD's L2.  Each XCD
    // takes a contiguous run of groups (rows 2048^2 FP32: 57.8 -> 56.8 us
    // against groups dealt round-robin).
    constexpr int TROWS = (IN == LAY_SPLIT && OUT == LAY_SPLIT) ? S::RT : S::RPW;
    int tile = blockIdx.x;
    if constexpr ((IN == LAY_SPLIT || OUT == LAY_SPLIT) && split_geom<T>::LY > TROWS) {
        constexpr int GR = split_geom<T>::LY / TROWS;
        if (gridDim.x % (8 * GR) == 0) {
            const int x = blockIdx.x & 7, i = blockIdx.x >> 3;
            const int per = gridDim.x / (8 * GR);  // groups per XCD
            tile = GR * (x * per + i / GR) + i % GR;
        }
    }
    row_tile<T, N, S::E, typename plan<T, N>::S, S::RPW, S::LLR, MODE, BEAM, IN, OUT, ONE>(a, tile, lds, threadIdx.x);
}

// ---------------------------------------------------------------------------
// column pass
// ---------------------------------------------------------------------------
// The kinetic step of a column at signed x index kxs, element m at
// y = t + NT m, in the order (top, bot) of block blk, 1/(nx ny) included.
template <typename T, int N, int E, int FRAME>
__device__ __forceinline__ void apply_kinetic(cx<T> (&v)[2][E], const ColArgs& a, int blk, int kxs, int t)
{
    constexpr int NT = N / E;
    const double c = a.c;
    const double px = a.dkx * (double)kxs;
    const T sgn = blk ? (T)-1 : (T)1;  // sign of the sigma_z term in each lane's order
    const T ka = sgn * (T)(c * c);
    const T kx = (T)(c * px);
    if constexpr (FRAME == 1) {
        // in a frame: K(p + a_m e_y, dt) exp(i vy p_y dt) / (nx ny), from the frame
        // table at (|kx|, ky): ((cos(E dt), sin(E dt)/E)/(nx ny), (cos, sin)(vy p_y dt)),
        // E of the kinetic momentum (px, py + a_m)
        const cx2<T>* kt = reinterpret_cast<const cx2<T>*>(a.ktab) + (size_t)(kxs < 0 ? -kxs : kxs) * N;
        asm volatile("" ::: "memory");
        int tt = t;
        asm volatile("" : "+v"(tt));
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int ky = tt + NT * m;
            const double pyk = a.dky * (double)signed_idx(ky, N) + a.a_m;
            const cx2<T> q = kt[ky];
            block_prop(v[0][m], v[1][m], q.a.re, q.a.im * ka, q.a.im * kx, q.a.im * (T)(c * pyk));
            v[0][m] = mul(v[0][m], q.b);
            v[1][m] = mul(v[1][m], q.b);
        }
    } else {
        // kinetic propagator K(p, dt) = cos(E dt) - i sin(E dt) H0(p)/E, times 1/(nx ny):
        // the table holds (cos(E dt), sin(E dt)/E)/(nx ny) at (|kx|, |ky|) (E depends on
        // |p| only); the matrix entries are (a, bx, by) = sin(E dt)/E (c^2, c px, c py)
        const int ny2 = N / 2 + 1;
        const cx<T>* kt = reinterpret_cast<const cx<T>*>(a.ktab) + (size_t)(kxs < 0 ? -kxs : kxs) * ny2;
        const T ky = (T)(c * a.dky);
        asm volatile("" ::: "memory");
        int tt = t;
        asm volatile("" : "+v"(tt));
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int kys = signed_idx(tt + NT * m, N);
            const cx<T> cq = kt[kys < 0 ? -kys : kys];
            block_prop(v[0][m], v[1][m], cq.re, cq.im * ka, cq.im * kx, cq.im * ky * (T)kys);
        }
    }
}

// One tile of columns of length N: TX columns of both blocks (LAY_ABI) or
// CT = shape::CT columns of one block (LAY_SPLIT), NT lanes and one LDS
// buffer of LL elements per column and block.
template <typename T, int N, int E, typename SCH, int TX, int LL, int MODE, int FRAME = 0, int LAY = LAY_ABI,
          bool ONE = false>
__device__ __forceinline__ void col_tile(const ColArgs& a, int tile, cx<T>* lds, int tid)
{
    constexpr int NT = N / E, L = 2 * NT;
    using G = split_geom<T>;
    // LAY_ABI: lane order block fastest, then the column within the tile, then
    // t, so a wave reads TX whole cells of each of several rows.  LAY_SPLIT: a
    // tile is CT columns of one block, lane order column then t.  Lane j (mod
    // CT) uses LDS group j either way (CT = 2 TX for LAY_ABI).
    constexpr int CT = LAY == LAY_SPLIT ? shape<T, N>::CT : 2 * TX;
    const int grp = tid & (CT - 1);
    const int t = tid / CT;
    int blk, x;
    if constexpr (LAY == LAY_SPLIT) {
        // Tile order: when a tile has fewer columns than a line (LX), the LXT
        // tiles that share the lines of CW = LX columns follow each other.
        // In a launch of both blocks, the column groups u = 2j and 2j + 1 are
        // group j of blocks A and B; group j is the (j/2)-th group from the
        // left for even j, from the right for odd j.  Tiles that follow each
        // other run on one XCD at nearly the same time, so the lines they
        // share, and the rows of the kinetic table they read (indexed by
        // |kx|, shared by columns x and nx - x and by both blocks), come from
        // that XCD's L2.
        constexpr int LXT = G::LX > CT ? G::LX / CT : 1;
        constexpr int CW = CT * LXT;
        const int c = tile % LXT, u = tile / LXT;
        const int tpb = (a.nx + CW - 1) / CW;  // column groups per block
        int j;
        if constexpr (ONE) {
            blk = a.one_block - 1;
            j = u;
        } else {
            blk = u & 1;
            j = u >> 1;
        }
        x = ((j & 1) ? tpb - 1 - (j >> 1) : (j >> 1)) * CW + c * CT + grp;
    } else {
        blk = tid & 1;
        x = tile * TX + (grp >> 1);
    }
    const bool live = x < a.nx;
    cx<T>* lb = lds + grp * LL;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.twy);
    constexpr uint32_t CB = 4 * sizeof(cx<T>);  // bytes per cell
    const uint32_t bytes = (uint32_t)a.nx * N * CB;
    const uint32_t lane = live ? ((uint32_t)t * a.nx + x) * CB + blk * (CB / 2) : bytes;
    const uint32_t mstride = (uint32_t)NT * a.nx * CB;  // bytes between a lane's elements
    // split layout: element m at y = t + NT m; linear in m when NT is a whole number of lines
    constexpr bool SPLIT_LINEAR = NT % G::LY == 0;
    const uint32_t slane = live ? split_off<T>(blk, t, x, a.nx, N) : bytes;
    // wave-uniform (a scalar offset of the buffer instructions)
    const uint32_t sstep =
        __builtin_amdgcn_readfirstlane((uint32_t)(NT / G::LY) * (uint32_t)(a.nx / G::LX) * 128u);
    const __amdgpu_buffer_rsrc_t rp = make_rsrc(a.psi, bytes);

    cx<T> v[2][E];
    if constexpr (LAY == LAY_ABI) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            cx<T> f;
            bload2((cx<T>*)nullptr, rp, lane, m * mstride, v[0][m], f);
            v[1][m] = swap_lane_pair(f);
        }
    } else if constexpr (SPLIT_LINEAR) {
#pragma unroll
        for (int m = 0; m < E; ++m) bload2((cx<T>*)nullptr, rp, slane, m * sstep, v[0][m], v[1][m]);
    } else {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const uint32_t o = live ? split_off<T>(blk, t + NT * m, x, a.nx, N) : bytes;
            bload2((cx<T>*)nullptr, rp, o, 0, v[0][m], v[1][m]);
        }
    }

    if constexpr (MODE == COL_INV) {
        fft<T, N, E, 2, true, QW_TW_PREFETCH_COL>(SCH{}, v, t, tw, lb);
    } else {
        fft<T, N, E, 2, false, QW_TW_PREFETCH_COL>(SCH{}, v, t, tw, lb);
    }

    const double c = a.c;
    const int kxs = signed_idx(live ? x : 0, a.nx);
    const double px = a.dkx * (double)kxs;

    if constexpr (MODE == COL_PROP) {
        apply_kinetic<T, N, E, FRAME>(v, a, blk, kxs, t);
        fft<T, N, E, 2, true, QW_TW_PREFETCH_COL>(SCH{}, v, t, tw, lb);
    }

    if constexpr ((MODE == COL_PROP || MODE == COL_INV) && LAY == LAY_ABI) {
#pragma unroll
        for (int m = 0; m < E; ++m) bstore2(v[0][m], swap_lane_pair(v[1][m]), rp, lane, m * mstride);
    } else if constexpr (MODE == COL_PROP || MODE == COL_INV) {
        if constexpr (SPLIT_LINEAR) {
#pragma unroll
            for (int m = 0; m < E; ++m) bstore2(v[0][m], v[1][m], rp, slane, m * sstep);
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const uint32_t o = live ? split_off<T>(blk, t + NT * m, x, a.nx, N) : bytes;
                bstore2(v[0][m], v[1][m], rp, o, 0);
            }
        }
    }

    if constexpr (MODE == COL_OBS || MODE == COL_MAPS) {
        // spin projections onto the unit bispinors u^+-(p) (Eq. 9, 18):
        //   c^s = sqrt((E + c^2)/(2E)) (aA + s aB)/sqrt2,
        //   aA = phi1 + k (px - i py) phi4,  aB = phi2 + k (px + i py) phi3,  k = c/(E + c^2)
        // Block A lanes hold (phi1, phi4), block B lanes (phi3, phi2); each
        // forms its own aA or aB and takes the partner's by a lane shuffle.
        double sw = 0.0, sp = 0.0, sm = 0.0;
        const double sg = blk ? -1.0 : 1.0;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int kys = signed_idx(t + NT * m, N);
            const double py = a.dky * (double)kys + a.a_m;  // kinetic momentum
            const double en = c * sqrt(c * c + px * px + py * py);
            const double kk = c / (en + c * c);
            const double tr = v[0][m].re, ti = v[0][m].im, br = v[1][m].re, bi = v[1][m].im;
            // u = phi1 or phi2, w = phi4 or phi3:  u + k (px - i sg py) w
            const double ur = blk ? br : tr, ui = blk ? bi : ti, wr = blk ? tr : br, wi = blk ? ti : bi;
            const double ar = ur + kk * (px * wr + sg * py * wi), ai = ui + kk * (px * wi - sg * py * wr);
            const double or_ = __shfl_xor(ar, 1), oi = __shfl_xor(ai, 1);
            if constexpr (MODE == COL_MAPS) {
                // per cell: the pair's two lanes hold the two blocks of one cell
                const double wl = tr * tr + ti * ti + br * br + bi * bi;
                const double wo = __shfl_xor(wl, 1);
                if (live && blk == 0) {
                    const double nn = (en + c * c) / (4.0 * en);
                    const double pr = ar + or_, pi = ai + oi, mr = ar - or_, mi = ai - oi;
                    double* out = a.partial + ((size_t)(t + NT * m) * a.nx + x) * 3;
                    out[0] = wl + wo;
                    out[1] = nn * (pr * pr + pi * pi);
                    out[2] = nn * (mr * mr + mi * mi);
                }
                continue;
            }
            if (live) {
                sw += tr * tr + ti * ti + br * br + bi * bi;
                if (blk == 0) {
                    const double nn = (en + c * c) / (4.0 * en);
                    const double pr = ar + or_, pi = ai + oi, mr = ar - or_, mi = ai - oi;
                    sp += nn * (pr * pr + pi * pi);
                    sm += nn * (mr * mr + mi * mi);
                }
            }
        }
        if constexpr (MODE == COL_MAPS) return;
        __syncthreads();  // LDS reused for the reduction
        double* red = reinterpret_cast<double*>(lds);
        constexpr int nthr = TX * L;
        red[tid] = sw;
        red[nthr + tid] = sp;
        red[2 * nthr + tid] = sm;
        __syncthreads();
        // fold the lanes of each column (index = (t TX + cl) 2 + blk) onto t = 0, blk = 0
        for (int w = nthr / 2; w >= 2 * TX; w >>= 1) {
            if (tid < w) {
#pragma unroll
                for (int q = 0; q < 3; ++q) red[q * nthr + tid] += red[q * nthr + tid + w];
            }
            __syncthreads();
        }
        if (tid == 0) {
            const int nb = 2 * a.n_max + 1;
            double* out = a.partial + (size_t)tile * a.partial_stride;
            for (int i = 0; i < 3 * nb + 3; ++i) out[i] = 0.0;
            for (int qc = 0; qc < TX; ++qc) {
                const int xq = tile * TX + qc;
                if (xq >= a.nx) break;
                const double w = red[2 * qc] + red[2 * qc + 1];
                const double wp = red[nthr + 2 * qc], wm = red[2 * nthr + 2 * qc];
                const int ks = signed_idx(xq, a.nx);
                // nearest order centre, then the window test
                const int d0 = ks - a.band_ref + a.band_half;
                const int twom = 2 * a.band_half;
                const int n = d0 >= 0 ? d0 / twom : -((-d0 + twom - 1) / twom);
                int dd = ks - a.band_ref - twom * n;
                dd = dd < 0 ? -dd : dd;
                if (dd <= a.window && n >= -a.n_max && n <= a.n_max) {
                    out[n + a.n_max] += w;
                    out[nb + n + a.n_max] += wp;
                    out[2 * nb + n + a.n_max] += wm;
                }
                out[3 * nb] += w;
                out[3 * nb + 1] += (a.spin0 >= 0 ? wm : wp);
                out[3 * nb + 2] += wp + wm;
            }
        }
    }
}

// lane groups (one per column and block) and threads of a column-pass
// workgroup: the propagation's passes take CT columns of one block, the
// others TX columns of both blocks
template <typename T, int N, int MODE>
struct col_wg {
    using S = shape<T, N>;
    static constexpr int groups = MODE == COL_PROP ? S::CT : 2 * S::TX;
    static constexpr int threads = groups * S::NT;
};

template <typename T, int N, int MODE, int FRAME = 0, bool ONE = false>
__global__ __launch_bounds__((col_wg<T, N, MODE>::threads)) __attribute__((
    amdgpu_waves_per_eu(sizeof(T) == sizeof(float) ? QW_WPE_COL : QW_WPE_COL_F64))) void col_pass(ColArgs a)
{
    using S = shape<T, N>;
    __shared__ cx<T> lds[col_wg<T, N, MODE>::groups * S::LLC];
    // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so
    // give each XCD a contiguous run of tiles -- neighbouring tiles share
    // cache lines (or kinetic table rows) and then meet in the same L2
    const int tile = (gridDim.x & 7) == 0 ? (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    // the propagation's column passes run on the split layout (see row_pass)
    constexpr int LAY = MODE == COL_PROP ? LAY_SPLIT : LAY_ABI;
    col_tile<T, N, S::E, typename plan<T, N>::S, S::TX, S::LLC, MODE, FRAME, LAY, ONE>(a, tile, lds, threadIdx.x);
}

// ---------------------------------------------------------------------------
// tables
// ---------------------------------------------------------------------------
// per-pass twiddles of the plan for length N (layout in fft_pass), in double
template <int NS, int R, int... Rest>
__device__ void fill_pass_twiddles(cx<double>* tmp, int i, int off)
{
    if constexpr (NS > 1) {
        if (i >= off && i < off + NS * R) {
            const int jm = (i - off) / R, r = (i - off) % R;
            double s, c;
            sincospi(2.0 * (double)(jm * r) / (double)(NS * R), &s, &c);
            tmp[0] = cx<double>{c, -s};
        }
    }
    if constexpr (sizeof...(Rest) > 0) fill_pass_twiddles<NS * R, Rest...>(tmp, i, off + (NS > 1 ? NS * R : 0));
}

template <typename T, int... R>
__device__ void pass_twiddle(sched<R...>, cx<T>* tw, int i)
{
    cx<double> v{1.0, 0.0};
    fill_pass_twiddles<1, R...>(&v, i, 0);
    // each of c and s rounded to nearest (see the rotation constants)
    tw[i] = cx<T>{(T)v.re, (T)v.im};
}

template <typename T, int N, typename SCH = typename plan<T, N>::S>
__global__ void twiddle_table(cx<T>* tw)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2 * N) pass_twiddle<T>(SCH{}, tw, i);
}

// field tables: beam_x[i] = (X0, X1) and beam_y[j] = (Y0, Y1) with
// A_y = s(t) Y0(y) X0(x), A_x = s(t) Y1(y) X1(x)
template <typename T>
__global__ void beam_tables(cx<T>* bx, cx<T>* by, BeamArgs b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < b.nx) {
        T x0 = 1, x1 = 1;
        if (b.mode == QW_BEAM_STANDING_PARAXIAL_) {
            const double x = b.x_min + b.lx * (double)i / (double)b.nx;
            x0 = (T)cos(b.kl * x);
            x1 = (T)sin(b.kl * x);
        }
        bx[i] = cx<T>{x0, x1};
    }
    if (i < b.ny) {
        T y0 = 0, y1 = 0;
        if (b.mode == QW_BEAM_STANDING_PARAXIAL_) {
            const double y = b.y_min + b.ly * (double)i / (double)b.ny;
            const double env = exp(-(y * y) / (b.w0 * b.w0));
            y0 = (T)(b.a0 * env);
            y1 = b.longitudinal ? (T)(b.a0 * (2.0 * y / (b.kl * b.w0 * b.w0)) * env) : (T)0;
        } else if (b.mode == QW_BEAM_UNIFORM_) {
            y0 = (T)b.uy;
            y1 = (T)b.ux;
        }
        by[i] = cx<T>{y0, y1};
    }
}

// kinetic table: for |kx| <= nx/2, |ky| <= ny/2 the pair
// (cos(E dt), sin(E dt)/E) / (nx ny) with E = c sqrt(c^2 + p^2), evaluated in
// double (phase E dt in double, reduced in double) and rounded to T
template <typename T>
__global__ void kinetic_table(cx<T>* kt, KineticArgs k)
{
    const int nx2 = k.nx / 2 + 1, ny2 = k.ny / 2 + 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx2 * ny2) return;
    const int ix = i / ny2, iy = i - ix * ny2;
    const double px = k.dkx * (double)ix, py = k.dky * (double)iy;
    const double en = k.c * sqrt(k.c * k.c + px * px + py * py);
    double s, c;
    sincos_phase(en * k.dt, s, c);
    kt[i] = cx<T>{(T)(c * k.inv_cells), (T)(s / en * k.inv_cells)};
}

// kinetic table in a frame: for |kx| <= nx/2 and every ky (signed order),
// ((cos(E dt), sin(E dt)/E)/(nx ny), (cos, sin)(vy py dt)) with py the
// canonical momentum and E = c sqrt(c^2 + px^2 + (py + a_m)^2); phases in
// double, reduced in double
template <typename T>
__global__ void kinetic_table_frame(cx2<T>* kt, KineticArgs k)
{
    const int nx2 = k.nx / 2 + 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx2 * k.ny) return;
    const int ix = i / k.ny, iy = i - ix * k.ny;
    const double px = k.dkx * (double)ix;
    const double py = k.dky * (double)(iy < k.ny / 2 ? iy : iy - k.ny);
    const double pk = py + k.a_m;
    const double en = k.c * sqrt(k.c * k.c + px * px + pk * pk);
    double s, c, fs, fc;
    sincos_phase(en * k.dt, s, c);
    sincos_phase(k.vy * py * k.dt, fs, fc);
    kt[i] = cx2<T>{cx<T>{(T)(c * k.inv_cells), (T)(s / en * k.inv_cells)}, cx<T>{(T)fc, (T)fs}};
}

// ---------------------------------------------------------------------------
// initial packet in momentum space: phi(p) = g(p) u^s(p) exp(i p.(r_min - r0)),
// one workgroup per momentum row ky; row sums of |phi|^2 to rownorm[ky]
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void packet_momentum(cx<T>* psi, double* rownorm, PacketArgs e)
{
    __shared__ double red[256];
    const int ky = blockIdx.x;
    const double c = e.c;
    const double py = e.dky * (double)signed_idx(ky, e.ny);
    const double sp = 1.0 / (2.0 * e.sigma_x);
    const double r2 = 0.70710678118654752440;
    const double chi1 = r2, chi2 = e.spin >= 0 ? r2 : -r2;
    double acc = 0.0;
    for (int kx = threadIdx.x; kx < e.nx; kx += blockDim.x) {
        const double px = e.dkx * (double)signed_idx(kx, e.nx);
        const double pk = py + e.a_m;  // kinetic p_y
        const double dx = px - e.p0x, dy = pk - e.p0y;
        const double amp = exp(-(dx * dx + dy * dy) / (4.0 * sp * sp));
        const double en = c * sqrt(c * c + px * px + pk * pk);
        const double nrm = sqrt((en + c * c) / (2.0 * en));
        const double kk = c / (en + c * c);
        double sn, cs;
        sincos(px * (e.x_min - e.x0) + py * (e.y_min - e.y0), &sn, &cs);
        // u = nrm (chi1, chi2, k (px - i py) chi2, k (px + i py) chi1), kinetic momentum
        const double u1 = nrm * chi1, u2 = nrm * chi2;
        const double u3r = nrm * kk * px * chi2, u3i = -nrm * kk * pk * chi2;
        const double u4r = nrm * kk * px * chi1, u4i = nrm * kk * pk * chi1;
        const double ar = amp * cs, ai = amp * sn;
        cx<T>* q = psi + ((size_t)ky * e.nx + kx) * 4;
        q[0] = cx<T>{(T)(u1 * ar), (T)(u1 * ai)};
        q[1] = cx<T>{(T)(u2 * ar), (T)(u2 * ai)};
        q[2] = cx<T>{(T)(u3r * ar - u3i * ai), (T)(u3r * ai + u3i * ar)};
        q[3] = cx<T>{(T)(u4r * ar - u4i * ai), (T)(u4r * ai + u4i * ar)};
        acc += amp * amp;  // |u| = 1
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) rownorm[ky] = red[0];
}

// ---------------------------------------------------------------------------
// launchers (host side)
// ---------------------------------------------------------------------------
template <typename T, int N>
hipError_t row_launch_n(int mode, const RowArgs& a, hipStream_t st)
{
    using S = shape<T, N>;
    // ROW_MID tiles are RT rows of one block (of both blocks, or of one)
    const int nb = a.one_block ? 1 : 2;
    const dim3 grid(mode == ROW_MID ? nb * ((a.ny + S::RT - 1) / S::RT) : (a.ny + S::RPW - 1) / S::RPW),
        block(mode == ROW_MID ? row_wg<T, N, ROW_MID>::threads : S::RPW * S::L);
    if (a.beam_mode == QW_BEAM_GAUSSIAN_FULL_) {
        switch (mode) {
        case ROW_FIRST: hipLaunchKernelGGL((row_pass<T, N, ROW_FIRST, 1>), grid, block, 0, st, a); break;
        case ROW_MID:
            if (a.one_block) hipLaunchKernelGGL((row_pass<T, N, ROW_MID, 1, true>), grid, block, 0, st, a);
            else hipLaunchKernelGGL((row_pass<T, N, ROW_MID, 1>), grid, block, 0, st, a);
            break;
        case ROW_LAST: hipLaunchKernelGGL((row_pass<T, N, ROW_LAST, 1>), grid, block, 0, st, a); break;
        case ROW_FWD_NORM: hipLaunchKernelGGL((row_pass<T, N, ROW_FWD_NORM>), grid, block, 0, st, a); break;
        case ROW_INV_SCALE: hipLaunchKernelGGL((row_pass<T, N, ROW_INV_SCALE>), grid, block, 0, st, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (mode) {
    case ROW_FIRST: hipLaunchKernelGGL((row_pass<T, N, ROW_FIRST>), grid, block, 0, st, a); break;
    case ROW_MID:
        if (a.one_block) hipLaunchKernelGGL((row_pass<T, N, ROW_MID, 0, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((row_pass<T, N, ROW_MID>), grid, block, 0, st, a);
        break;
    case ROW_LAST: hipLaunchKernelGGL((row_pass<T, N, ROW_LAST>), grid, block, 0, st, a); break;
    case ROW_FWD_NORM: hipLaunchKernelGGL((row_pass<T, N, ROW_FWD_NORM>), grid, block, 0, st, a); break;
    case ROW_INV_SCALE: hipLaunchKernelGGL((row_pass<T, N, ROW_INV_SCALE>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int N>
hipError_t col_launch_n(int mode, const ColArgs& a, hipStream_t st)
{
    using S = shape<T, N>;
    // COL_PROP tiles are CT columns of one block (of both blocks, or of one)
    const int nb = a.one_block ? 1 : 2;
    const dim3 grid(mode == COL_PROP ? nb * ((a.nx + S::CT - 1) / S::CT) : (a.nx + S::TX - 1) / S::TX),
        block(mode == COL_PROP ? col_wg<T, N, COL_PROP>::threads : S::TX * S::L);
    switch (mode) {
    case COL_PROP:
        if (a.frame && a.one_block) hipLaunchKernelGGL((col_pass<T, N, COL_PROP, 1, true>), grid, block, 0, st, a);
        else if (a.frame) hipLaunchKernelGGL((col_pass<T, N, COL_PROP, 1>), grid, block, 0, st, a);
        else if (a.one_block) hipLaunchKernelGGL((col_pass<T, N, COL_PROP, 0, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((col_pass<T, N, COL_PROP>), grid, block, 0, st, a);
        break;
    case COL_INV: hipLaunchKernelGGL((col_pass<T, N, COL_INV>), grid, block, 0, st, a); break;
    case COL_OBS: hipLaunchKernelGGL((col_pass<T, N, COL_OBS>), grid, block, 0, st, a); break;
    case COL_MAPS: hipLaunchKernelGGL((col_pass<T, N, COL_MAPS>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define QW_SIZE_SWITCH(n, CALL)        \
    switch (n) {                       \
    case 8: return CALL(8);            \
    case 16: return CALL(16);          \
    case 32: return CALL(32);          \
    case 64: return CALL(64);          \
    case 128: return CALL(128);        \
    case 256: return CALL(256);        \
    case 512: return CALL(512);        \
    case 1024: return CALL(1024);      \
    case 2048: return CALL(2048);      \
    case 4096: return CALL(4096);      \
    default: break;                    \
    }

template <typename T>
hipError_t launch_row(int mode, int nx, const RowArgs& a, hipStream_t st)
{
#define QW_CALL(NN) row_launch_n<T, NN>(mode, a, st)
    QW_SIZE_SWITCH(nx, QW_CALL)
#undef QW_CALL
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_col(int mode, int ny, const ColArgs& a, hipStream_t st)
{
#define QW_CALL(NN) col_launch_n<T, NN>(mode, a, st)
    QW_SIZE_SWITCH(ny, QW_CALL)
#undef QW_CALL
    return hipErrorInvalidValue;
}

template <int... R>
int sched_radices(sched<R...>, int* radices, int max_radices)
{
    const int r[] = {R...};
    const int n = (int)(sizeof(r) / sizeof(r[0]));
    for (int i = 0; i < n && i < max_radices; ++i) radices[i] = r[i];
    return n;
}

// the radices of the transform plan of length n (0: no plan)
template <typename T>
int plan_radices(int n, int* radices, int max_radices)
{
#define QW_CALL(NN) sched_radices(typename plan<T, NN>::S{}, radices, max_radices)
    QW_SIZE_SWITCH(n, QW_CALL)
#undef QW_CALL
    return 0;
}

template <typename T>
int col_blocks(int nx, int ny)
{
#define QW_CALL(NN) (nx + shape<T, NN>::TX - 1) / shape<T, NN>::TX
    QW_SIZE_SWITCH(ny, QW_CALL)
#undef QW_CALL
    return -1;
}

template <typename T, int N>
hipError_t twiddles_n(void* tw, hipStream_t st)
{
    static_assert(tw_len_of<T, N>::value <= 2 * N, "twiddle table larger than its slot");
    hipLaunchKernelGGL((twiddle_table<T, N>), dim3((2 * N + 255) / 256), dim3(256), 0, st,
                       reinterpret_cast<cx<T>*>(tw));
    return hipGetLastError();
}

// per-pass twiddles for length n into 2n entries at tw
template <typename T>
hipError_t launch_twiddles(void* tw, int n, hipStream_t st)
{
#define QW_CALL(NN) twiddles_n<T, NN>(tw, st)
    QW_SIZE_SWITCH(n, QW_CALL)
#undef QW_CALL
    return hipErrorInvalidValue;
}

#undef QW_SIZE_SWITCH

template <typename T>
hipError_t launch_beam_tables(void* bx, void* by, const BeamArgs& b, hipStream_t st)
{
    const int n = b.nx > b.ny ? b.nx : b.ny;
    hipLaunchKernelGGL(beam_tables<T>, dim3((n + 255) / 256), dim3(256), 0, st, reinterpret_cast<cx<T>*>(bx),
                       reinterpret_cast<cx<T>*>(by), b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_kinetic_table(void* kt, const KineticArgs& k, hipStream_t st)
{
    const int n = (k.nx / 2 + 1) * (k.ny / 2 + 1);
    hipLaunchKernelGGL(kinetic_table<T>, dim3((n + 255) / 256), dim3(256), 0, st, reinterpret_cast<cx<T>*>(kt), k);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_kinetic_table_frame(void* kt, const KineticArgs& k, hipStream_t st)
{
    const int n = (k.nx / 2 + 1) * k.ny;
    hipLaunchKernelGGL(kinetic_table_frame<T>, dim3((n + 255) / 256), dim3(256), 0, st, reinterpret_cast<cx2<T>*>(kt),
                       k);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_packet(void* psi, double* rownorm, const PacketArgs& e, hipStream_t st)
{
    hipLaunchKernelGGL(packet_momentum<T>, dim3(e.ny), dim3(256), 0, st, reinterpret_cast<cx<T>*>(psi), rownorm, e);
    return hipGetLastError();
}

}  // namespace qw

#define QW_DEFINE_LAUNCHERS(T, SUF)                                                                           \
    namespace qw {                                                                                           \
    hipError_t launch_row_##SUF(int mode, int nx, const RowArgs& a, hipStream_t s)                          \
    {                                                                                                        \
        return launch_row<T>(mode, nx, a, s);                                                                \
    }                                                                                                        \
    hipError_t launch_col_##SUF(int mode, int ny, const ColArgs& a, hipStream_t s)                          \
    {                                                                                                        \
        return launch_col<T>(mode, ny, a, s);                                                                \
    }                                                                                                        \
    int col_blocks_##SUF(int nx, int ny) { return col_blocks<T>(nx, ny); }                                   \
    int plan_radices_##SUF(int n, int* r, int m) { return plan_radices<T>(n, r, m); }                         \
    hipError_t launch_twiddles_##SUF(void* tw, int n, hipStream_t s) { return launch_twiddles<T>(tw, n, s); } \
    hipError_t launch_beam_tables_##SUF(void* bx, void* by, const BeamArgs& b, hipStream_t s)               \
    {                                                                                                        \
        return launch_beam_tables<T>(bx, by, b, s);                                                          \
    }                                                                                                        \
    hipError_t launch_packet_##SUF(void* psi, double* rownorm, const PacketArgs& e, hipStream_t s)          \
    {                                                                                                        \
        return launch_packet<T>(psi, rownorm, e, s);                                                         \
    }                                                                                                        \
    hipError_t launch_kinetic_table_##SUF(void* kt, const KineticArgs& k, hipStream_t s)                     \
    {                                                                                                        \
        return launch_kinetic_table<T>(kt, k, s);                                                            \
    }                                                                                                        \
    hipError_t launch_kinetic_table_frame_##SUF(void* kt, const KineticArgs& k, hipStream_t s)               \
    {                                                                                                        \
        return launch_kinetic_table_frame<T>(kt, k, s);                                                      \
    }                                                                                                        \
    }
