// qw_host.hpp -- host-side helpers shared by the single-instance engine
// (qw_api.cpp) and the batched engine (qw_batch.cpp): argument checks and
// the translation of the public structs into kernel arguments.
#pragma once
#include <cmath>
#include <cstdio>
#include <initializer_list>
#include <string>

#include "qw.h"
#include "qw_launch.hpp"

namespace qwh {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kMaxNmax = 16;
constexpr int kPartialStride = 3 * (2 * kMaxNmax + 1) + 3;  // doubles per column-pass workgroup
constexpr size_t kAlign = 256;
// the in-kernel phase reduction (Cody-Waite, three parts of pi/2) is exact
// for |x| < 2^20 pi/2; the callers keep every phase below this bound
constexpr double kMaxPhase = 1.6e6;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

inline bool finite_all(std::initializer_list<double> v)
{
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

// The device of a device-accessible allocation (device, managed or unified
// memory); anything else -- host memory, an unknown pointer -- is refused.
inline int device_of(const void* p, int* device, std::string* msg)
{
    hipPointerAttribute_t attr{};
    const hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *msg = std::string("workspace is not device memory (pointer attributes: ") + hipGetErrorString(e) + ")";
        return QW_E_ARG;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged && attr.type != hipMemoryTypeUnified) {
        *msg = "workspace is not device memory (memory type " + std::to_string((int)attr.type) + ")";
        return QW_E_ARG;
    }
    *device = attr.device;
    return QW_OK;
}

inline bool is_pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

inline int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// Each check returns QW_OK or an error code with *msg set.
inline int check_grid(const qw_grid& g, int lo, int hi, std::string* msg)
{
    char buf[256];
    if (g.precision != QW_F32 && g.precision != QW_F64) {
        snprintf(buf, sizeof buf, "precision %d is neither QW_F64 nor QW_F32", g.precision);
        *msg = buf;
        return QW_E_ARG;
    }
    if (!is_pow2_in(g.nx, lo, hi) || !is_pow2_in(g.ny, lo, hi)) {
        snprintf(buf, sizeof buf, "nx=%d ny=%d: each must be a power of two in [%d, %d]", g.nx, g.ny, lo, hi);
        *msg = buf;
        return QW_E_SIZE;
    }
    if (!finite_all({g.x_min, g.y_min, g.lx, g.ly, g.c}) || !(g.lx > 0) || !(g.ly > 0) || !(g.c > 0)) {
        *msg = "box and c must be finite with lx, ly, c > 0";
        return QW_E_ARG;
    }
    return QW_OK;
}

inline bool standing(int mode) { return mode == QW_BEAM_STANDING_PARAXIAL || mode == QW_BEAM_GAUSSIAN_FULL; }

inline int check_beam(const qw_beam& b, std::string* msg)
{
    if (b.mode != QW_BEAM_NONE && b.mode != QW_BEAM_STANDING_PARAXIAL && b.mode != QW_BEAM_UNIFORM &&
        b.mode != QW_BEAM_GAUSSIAN_FULL) {
        *msg = "unknown beam mode " + std::to_string(b.mode);
        return QW_E_ARG;
    }
    if (standing(b.mode) && (!finite_all({b.a0, b.lambda_l, b.w0, b.ramp_periods}) || !(b.lambda_l > 0) ||
                             !(b.w0 > 0) || b.ramp_periods < 0)) {
        *msg = "standing wave needs finite a0, lambda_l > 0, w0 > 0, ramp_periods >= 0";
        return QW_E_ARG;
    }
    if (b.mode == QW_BEAM_UNIFORM && !finite_all({b.ux, b.uy})) {
        *msg = "uniform field must be finite";
        return QW_E_ARG;
    }
    return QW_OK;
}

inline int check_packet(const qw_packet& e, std::string* msg)
{
    if (!finite_all({e.p0x, e.p0y, e.x0, e.y0, e.sigma_x}) || !(e.sigma_x > 0) || (e.spin != 1 && e.spin != -1)) {
        *msg = "packet needs finite values, sigma_x > 0 and spin = +1 or -1";
        return QW_E_ARG;
    }
    return QW_OK;
}

inline int check_obs(const qw_obs_spec& o, std::string* msg)
{
    if (o.n_max < 0 || o.n_max > kMaxNmax) {
        *msg = "n_max must be in [0, " + std::to_string(kMaxNmax) + "]";
        return QW_E_ARG;
    }
    if (o.band_half_idx <= 0 || o.window_idx < 0 || o.window_idx >= o.band_half_idx) {
        *msg = "need band_half_idx > 0 and 0 <= window_idx < band_half_idx";
        return QW_E_ARG;
    }
    if (o.spin0 != 1 && o.spin0 != -1) {
        *msg = "spin0 must be +1 or -1";
        return QW_E_ARG;
    }
    return QW_OK;
}

inline int check_frame(const qw_frame& f, double c, std::string* msg)
{
    if (!finite_all({f.vy, f.a_m}) || !(std::fabs(f.vy) < c)) {
        *msg = "frame needs finite vy and a_m with |vy| < c";
        return QW_E_ARG;
    }
    return QW_OK;
}

inline bool frame_active(const qw_frame& f) { return f.vy != 0.0 || f.a_m != 0.0; }

// the phases w t, E dt and vy p_y dt of a run of n steps must stay in the
// exact range of the in-kernel reduction
inline int check_phases(const qw_grid& g, const qw_beam& b, bool beam_on, int64_t n, double t0, double dt,
                        std::string* msg, const qw_frame* f = nullptr)
{
    char buf[256];
    if (beam_on && standing(b.mode)) {
        const double om = g.c * 2.0 * kPi / b.lambda_l;
        const double tmax = std::fmax(std::fabs(t0), std::fabs(t0 + (double)n * dt));
        if (om * tmax > kMaxPhase) {
            snprintf(buf, sizeof buf, "|omega t| = %g exceeds %g", om * tmax, kMaxPhase);
            *msg = buf;
            return QW_E_ARG;
        }
    }
    const double px = 0.5 * g.nx * 2.0 * kPi / g.lx;
    const double py = 0.5 * g.ny * 2.0 * kPi / g.ly + (f ? std::fabs(f->a_m) : 0.0);
    const double emax = g.c * std::sqrt(g.c * g.c + px * px + py * py);
    if (f && std::fabs(f->vy) * py * std::fabs(dt) > kMaxPhase) {
        *msg = "|vy p_y dt| exceeds the phase range";
        return QW_E_ARG;
    }
    if (emax * std::fabs(dt) > kMaxPhase) {
        snprintf(buf, sizeof buf, "|E dt| = %g exceeds %g", emax * std::fabs(dt), kMaxPhase);
        *msg = buf;
        return QW_E_ARG;
    }
    return QW_OK;
}

inline qw::BeamArgs beam_args(const qw_grid& g, const qw_beam& b)
{
    qw::BeamArgs a{};
    a.mode = b.mode;
    a.longitudinal = b.longitudinal;
    a.nx = g.nx;
    a.ny = g.ny;
    a.x_min = g.x_min;
    a.y_min = g.y_min;
    a.lx = g.lx;
    a.ly = g.ly;
    a.a0 = b.a0;
    a.kl = b.mode == QW_BEAM_STANDING_PARAXIAL ? 2.0 * kPi / b.lambda_l : 0.0;
    a.w0 = b.w0;
    a.ux = b.ux;
    a.uy = b.uy;
    return a;
}

// Mean squared-norm gain of one float transform with the given radices.  The
// per-pass twiddles and the radix-8/16 rotation constants are float pairs
// (c, s), each rounded to nearest, with c^2 + s^2 a little under 1.  A pass
// of radix R and stride ns multiplies input r of butterfly j by the twiddle
// exp(-+2 pi i (j mod ns) r / (ns R)) and then by the butterfly's rotation
// constants, which for input r are w16^(q s), s = 0..3, with q = r mod 4
// (R = 16), or w16^(2 q s) with q = r mod 2 (R = 8), each on a quarter of
// its energy; R = 2, 4 use only +-1 and +-i.  Averaged over the inputs, the
// passes' gains multiply.  Forward and inverse transforms use conjugate
// pairs of the same magnitudes.  Built with QW_F32_SPLIT_ROTATIONS = 1 the
// rotation constants are hi + lo float pairs, exact to about 2^-48, and only
// the twiddles lose norm.
#ifndef QW_F32_SPLIT_ROTATIONS
#define QW_F32_SPLIT_ROTATIONS 0
#endif
inline double transform_gain_f32(const int* radices, int count)
{
    auto mag2 = [](double angle) {
        const double c = (double)(float)std::cos(angle), s = (double)(float)std::sin(angle);
        return c * c + s * s;
    };
    auto w16 = [&](int j) {
        return (j & 3) == 0 || QW_F32_SPLIT_ROTATIONS ? 1.0 : mag2(2.0 * kPi * (j & 15) / 16.0);
    };
    double gain = 1.0;
    int ns = 1;
    for (int p = 0; p < count; ++p) {
        const int R = radices[p];
        double sum = 0.0;
        for (int r = 0; r < R; ++r) {
            double rot = 1.0;
            if (R == 8 || R == 16) {
                const int q = R == 16 ? (r & 3) : (r & 1);
                rot = 0.0;
                for (int s = 0; s < 4; ++s) rot += w16((R == 16 ? 1 : 2) * q * s);
                rot *= 0.25;
            }
            double tw = 1.0;
            if (ns > 1) {
                tw = 0.0;
                for (int jm = 0; jm < ns; ++jm) tw += mag2(2.0 * kPi * (double)jm * r / ((double)ns * R));
                tw /= ns;
            }
            sum += tw * rot;
        }
        gain *= sum / R;
        ns *= R;
    }
    return gain;
}

// The factor the kinetic table carries besides 1/(nx ny) so that a float
// step keeps the norm on average: a step makes two transforms of each
// length, so its squared-norm gain is (gx gy)^2 and the amplitude factor
// 1/(gx gy) undoes it.  FP64 rotations are exact to 1e-16: factor 1.
inline double kinetic_norm_factor(bool f32, const int* rx, int nrx, const int* ry, int nry)
{
    if (!f32) return 1.0;
    return 1.0 / (transform_gain_f32(rx, nrx) * transform_gain_f32(ry, nry));
}

inline qw::KineticArgs kinetic_args(const qw_grid& g, double dt)
{
    qw::KineticArgs k{};
    k.nx = g.nx;
    k.ny = g.ny;
    k.dkx = 2.0 * kPi / g.lx;
    k.dky = 2.0 * kPi / g.ly;
    k.c = g.c;
    k.dt = dt;
    k.inv_cells = 1.0 / ((double)g.nx * (double)g.ny);
    return k;
}

inline qw::PacketArgs packet_args(const qw_grid& g, const qw_packet& e, double a_m = 0.0)
{
    qw::PacketArgs p{};
    p.nx = g.nx;
    p.ny = g.ny;
    p.spin = e.spin;
    p.dkx = 2.0 * kPi / g.lx;
    p.dky = 2.0 * kPi / g.ly;
    p.c = g.c;
    p.p0x = e.p0x;
    p.p0y = e.p0y;
    p.x0 = e.x0;
    p.y0 = e.y0;
    p.sigma_x = e.sigma_x;
    p.x_min = g.x_min;
    p.y_min = g.y_min;
    p.a_m = a_m;
    return p;
}

// field and grid parts of the row-pass arguments (tables and state set by the caller)
inline void row_field(const qw_grid& g, const qw_beam& b, bool beam_on, qw::RowArgs* a, double vy = 0.0)
{
    a->beam_mode = beam_on ? b.mode : QW_BEAM_NONE;
    if (standing(b.mode)) {
        a->omega = g.c * 2.0 * kPi / b.lambda_l;
        a->t_ramp = b.ramp_periods * b.lambda_l / g.c;
        a->ramp_k = a->t_ramp > 0 ? kPi / (2.0 * a->t_ramp) : 0.0;
    }
    if (b.mode == QW_BEAM_GAUSSIAN_FULL) {
        qw::FullBeam& f = a->full;
        f.a0 = b.a0;
        f.kl = 2.0 * kPi / b.lambda_l;
        f.w0 = b.w0;
        f.xr = 0.5 * f.kl * b.w0 * b.w0;
        f.eps = 1.0 / (f.kl * b.w0);
        f.x_min = g.x_min;
        f.dx = g.lx / g.nx;
        f.y_min = g.y_min;
        f.dy = g.ly / g.ny;
        f.vy = vy;
        f.longitudinal = b.longitudinal;
    }
    a->c = g.c;
    a->ny = g.ny;
}

// grid parts of the column-pass arguments
inline void col_grid(const qw_grid& g, qw::ColArgs* a)
{
    a->nx = g.nx;
    a->dkx = 2.0 * kPi / g.lx;
    a->dky = 2.0 * kPi / g.ly;
    a->c = g.c;
    a->inv_cells = 1.0 / ((double)g.nx * (double)g.ny);
    a->partial_stride = kPartialStride;
}

}  // namespace qwh
