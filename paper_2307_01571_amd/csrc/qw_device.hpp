// qw_device.hpp -- device building blocks for the split-operator passes on gfx950:
// complex arithmetic, radix-2/4/8/16 register butterflies, the Stockham
// transform staged through LDS, and the closed-form 2x2 block propagators.
//
// Block structure (Sec. II.B, Eq. 5 with p_z = A_z = 0, standard
// representation): H = c alpha.(p + A) + beta c^2 never couples (psi1, psi4)
// with (psi2, psi3).  Both the kinetic propagator exp(-i H0 dt) and the
// interaction propagator exp(-i c alpha.A dt) therefore act as two 2x2
// blocks, and each is cos(phase) I - i sin(phase) M/|M| because
// H0^2 = E^2 I and (alpha.A)^2 = |A|^2 I.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// No implicit contraction of a * b + c into fused multiply-adds in the
// kernels: where a fused operation is wanted it is written out (fmx below).
// The rounding of every result then follows the source alone, so kernels
// that run the same arithmetic in different tile shapes or state layouts
// (single-instance and batched passes) produce identical bits.
#pragma clang fp contract(off)

namespace qw {

__device__ __forceinline__ float fmx(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmx(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__device__ __forceinline__ cx<T> add(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> sub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> mul(cx<T> a, cx<T> b)
{
    return {fmx(a.re, b.re, -(a.im * b.im)), fmx(a.re, b.im, a.im * b.re)};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot90(cx<T> a)
{
    return INV ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

// ---------------------------------------------------------------------------
// Buffer addressing (gfx9 raw buffers): one 128-bit resource in SGPRs, a
// 32-bit per-lane byte offset and a wave-uniform scalar offset.  The state
// arrays are at most 1 GiB, so 32-bit offsets cover them; accesses past
// num_records read zero and drop writes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ cx<float> bload(cx<float>*, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ cx<double> bload(cx<double>*, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
typedef int qw_v2i __attribute__((ext_vector_type(2)));
typedef int qw_v4i __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void bstore(cx<float> v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(qw_v2i, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(cx<double> v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(qw_v4i, v), r, voff, soff, 0);
}

// Two consecutive complex values (16 B in float, 32 B in double) at one
// lane offset: half a cell.  The 128-bit loads and stores move whole structs
// by bit cast (taking the vector apart element by element has been seen to
// narrow the load to its first dword).
template <typename T>
struct cx2 {
    cx<T> a, b;
};
__device__ __forceinline__ void bload2(cx<float>*, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                       cx<float>& a, cx<float>& b)
{
    const cx2<float> h = __builtin_bit_cast(cx2<float>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    a = h.a;
    b = h.b;
}
__device__ __forceinline__ void bload2(cx<double>*, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                       cx<double>& a, cx<double>& b)
{
    a = __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    b = __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, soff, 0));
}
__device__ __forceinline__ void bstore2(cx<float> a, cx<float> b, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                        uint32_t soff)
{
    // the vector is built from the four values (a bit cast of a cx2 temporary
    // can be folded into one 16-byte read across two array elements, which
    // keeps a register array in scratch memory)
    const qw_v4i d = {__builtin_bit_cast(int, a.re), __builtin_bit_cast(int, a.im), __builtin_bit_cast(int, b.re),
                      __builtin_bit_cast(int, b.im)};
    __builtin_amdgcn_raw_buffer_store_b128(d, r, voff, soff, 0);
}
__device__ __forceinline__ void bstore2(cx<double> a, cx<double> b, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                        uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(qw_v4i, a), r, voff, soff, 0);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(qw_v4i, b), r, voff + 16, soff, 0);
}

// Exchange a value with the neighbouring lane (lanes 2q <-> 2q+1) by DPP
// quad permutation [1, 0, 3, 2].
__device__ __forceinline__ int swap_lane_pair(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true); }
__device__ __forceinline__ float swap_lane_pair(float v)
{
    return __builtin_bit_cast(float, swap_lane_pair(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double swap_lane_pair(double v)
{
    const long long u = __builtin_bit_cast(long long, v);
    const int lo = swap_lane_pair((int)(u & 0xffffffffLL)), hi = swap_lane_pair((int)(u >> 32));
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <typename T>
__device__ __forceinline__ cx<T> swap_lane_pair(cx<T> v)
{
    return cx<T>{swap_lane_pair(v.re), swap_lane_pair(v.im)};
}

// ---------------------------------------------------------------------------
// sin and cos of a phase given in double.  x = k pi/2 + r with pi/2 split in
// three parts of which the first two have 33-bit mantissas (so k P1 and k P2
// are exact for |k| < 2^20), |r| <= pi/4, then the Taylor series of sin and
// cos about 0: to r^17 / r^18 in double (truncation < 1e-17), to r^11 / r^12
// in float (truncation < 1e-9).  Quadrant k mod 4 selects and signs.
// ---------------------------------------------------------------------------
constexpr double kPio2a = 1.5707963267341256;      // 0x1.921fb544p+0
constexpr double kPio2b = 6.077100506303966e-11;   // 0x1.0b4611a6p-34
constexpr double kPio2c = 2.0222662487959506e-21;
constexpr double kTwoOverPi = 0.6366197723675814;

__device__ __forceinline__ double reduce_quadrant(double x, int& q)
{
    const double k = rint(x * kTwoOverPi);
    double r = fma(-k, kPio2a, x);
    r = fma(-k, kPio2b, r);
    r = fma(-k, kPio2c, r);
    q = (int)(long long)k & 3;
    return r;
}

template <typename T>
__device__ __forceinline__ void quadrant(int q, T sr, T cr, T& s, T& c)
{
    const bool swap = q & 1;
    const T a = swap ? cr : sr, b = swap ? sr : cr;
    s = (q == 1 || q == 0) ? a : -a;
    c = (q == 0 || q == 3) ? b : -b;
}

__device__ __forceinline__ void sincos_phase(double x, double& s, double& c)
{
    int q;
    const double r = reduce_quadrant(x, q);
    const double r2 = r * r;
    double ps = 2.8114572543455206e-15;  // 1/17!
    ps = fma(ps, r2, -7.647163731819816e-13);
    ps = fma(ps, r2, 1.6059043836821613e-10);
    ps = fma(ps, r2, -2.505210838544172e-08);
    ps = fma(ps, r2, 2.7557319223985893e-06);
    ps = fma(ps, r2, -0.0001984126984126984);
    ps = fma(ps, r2, 0.008333333333333333);
    ps = fma(ps, r2, -0.16666666666666666);
    const double sr = fma(ps * r2, r, r);
    double pc = 1.5619206968586225e-16;  // 1/18!
    pc = fma(pc, r2, -4.779477332387385e-14);
    pc = fma(pc, r2, 1.1470745597729725e-11);
    pc = fma(pc, r2, -2.08767569878681e-09);
    pc = fma(pc, r2, 2.755731922398589e-07);
    pc = fma(pc, r2, -2.48015873015873e-05);
    pc = fma(pc, r2, 0.001388888888888889);
    pc = fma(pc, r2, -0.041666666666666664);
    pc = fma(pc, r2, 0.5);
    const double cr = fma(-pc, r2, 1.0);
    quadrant(q, sr, cr, s, c);
}

__device__ __forceinline__ void sincos_phase(double x, float& s, float& c)
{
    int q;
    const float r = (float)reduce_quadrant(x, q);
    const float r2 = r * r;
    float ps = -2.505210838544172e-08f;  // -1/11!
    ps = fmaf(ps, r2, 2.7557319223985893e-06f);
    ps = fmaf(ps, r2, -0.0001984126984126984f);
    ps = fmaf(ps, r2, 0.008333333333333333f);
    ps = fmaf(ps, r2, -0.16666666666666666f);
    const float sr = fmaf(ps * r2, r, r);
    float pc = 2.08767569878681e-09f;  // 1/12!
    pc = fmaf(pc, r2, -2.755731922398589e-07f);
    pc = fmaf(pc, r2, 2.48015873015873e-05f);
    pc = fmaf(pc, r2, -0.001388888888888889f);
    pc = fmaf(pc, r2, 0.041666666666666664f);
    pc = fmaf(pc, r2, -0.5f);
    const float cr = fmaf(pc, r2, 1.0f);
    quadrant(q, sr, cr, s, c);
}

// float-only sin/cos for |x| < ~4e3: the same quadrant reduction with pi/2
// split in three floats (12-bit first two parts, so k P1 and k P2 are exact
// for |k| < 2^12) and the float polynomials above
__device__ __forceinline__ void sincos_small(float x, float& s, float& c)
{
    const float k = rintf(x * 0.6366197466850281f);
    float r = fmaf(-k, 1.5703125f, x);
    r = fmaf(-k, 0.0004837512969970703f, r);
    r = fmaf(-k, 7.549790126404332e-08f, r);
    const int q = (int)k & 3;
    const float r2 = r * r;
    float ps = -2.505210838544172e-08f;
    ps = fmaf(ps, r2, 2.7557319223985893e-06f);
    ps = fmaf(ps, r2, -0.0001984126984126984f);
    ps = fmaf(ps, r2, 0.008333333333333333f);
    ps = fmaf(ps, r2, -0.16666666666666666f);
    const float sr = fmaf(ps * r2, r, r);
    float pc = 2.08767569878681e-09f;
    pc = fmaf(pc, r2, -2.755731922398589e-07f);
    pc = fmaf(pc, r2, 2.48015873015873e-05f);
    pc = fmaf(pc, r2, -0.001388888888888889f);
    pc = fmaf(pc, r2, 0.041666666666666664f);
    pc = fmaf(pc, r2, -0.5f);
    const float cr = fmaf(pc, r2, 1.0f);
    quadrant(q, sr, cr, s, c);
}
__device__ __forceinline__ void sincos_small(double x, double& s, double& c) { sincos_phase(x, s, c); }

// cos(th) and sin(th)/th for th^2 <= 0.01 with the series cut early:
// float to th^4 (truncation < 2e-9), double to th^10 (< 3e-21).
__device__ __forceinline__ void cos_sinc_short(float t2, float& C, float& Sc)
{
    C = fmaf(fmaf(0.041666666666666664f, t2, -0.5f), t2, 1.0f);
    Sc = fmaf(fmaf(0.008333333333333333f, t2, -0.16666666666666666f), t2, 1.0f);
}
__device__ __forceinline__ void cos_sinc_short(double t2, double& C, double& Sc)
{
    double c = -2.755731922398589e-07;  // -1/10!
    c = fma(c, t2, 2.48015873015873e-05);
    c = fma(c, t2, -0.001388888888888889);
    c = fma(c, t2, 0.041666666666666664);
    c = fma(c, t2, -0.5);
    C = fma(c, t2, 1.0);
    double s = -2.505210838544172e-08;  // -1/11!
    s = fma(s, t2, 2.7557319223985893e-06);
    s = fma(s, t2, -0.0001984126984126984);
    s = fma(s, t2, 0.008333333333333333);
    s = fma(s, t2, -0.16666666666666666);
    Sc = fma(s, t2, 1.0);
}

// cos(th) and sin(th)/th as even series in th^2 for th^2 <= 0.49 (|th| <= 0.7):
// float keeps terms to th^10 (truncation < 3e-11), double to th^18 (< 1e-21).
__device__ __forceinline__ void cos_sinc_series(float t2, float& C, float& Sc)
{
    float c = -2.755731922398589e-07f;  // -1/10!
    c = fmaf(c, t2, 2.48015873015873e-05f);
    c = fmaf(c, t2, -0.001388888888888889f);
    c = fmaf(c, t2, 0.041666666666666664f);
    c = fmaf(c, t2, -0.5f);
    C = fmaf(c, t2, 1.0f);
    float s = -2.505210838544172e-08f;  // -1/11!
    s = fmaf(s, t2, 2.7557319223985893e-06f);
    s = fmaf(s, t2, -0.0001984126984126984f);
    s = fmaf(s, t2, 0.008333333333333333f);
    s = fmaf(s, t2, -0.16666666666666666f);
    Sc = fmaf(s, t2, 1.0f);
}
__device__ __forceinline__ void cos_sinc_series(double t2, double& C, double& Sc)
{
    double c = 1.5619206968586225e-16;  // 1/18!
    c = fma(c, t2, -4.779477332387385e-14);
    c = fma(c, t2, 1.1470745597729725e-11);
    c = fma(c, t2, -2.08767569878681e-09);
    c = fma(c, t2, 2.755731922398589e-07);
    c = fma(c, t2, -2.48015873015873e-05);
    c = fma(c, t2, 0.001388888888888889);
    c = fma(c, t2, -0.041666666666666664);
    c = fma(c, t2, 0.5);
    C = fma(-c, t2, 1.0);
    double s = 8.22063524662433e-18;  // 1/19!
    s = fma(s, t2, -2.8114572543455206e-15);
    s = fma(s, t2, 7.647163731819816e-13);
    s = fma(s, t2, -1.6059043836821613e-10);
    s = fma(s, t2, 2.505210838544172e-08);
    s = fma(s, t2, -2.7557319223985893e-06);
    s = fma(s, t2, 0.0001984126984126984);
    s = fma(s, t2, -0.008333333333333333);
    s = fma(s, t2, 0.16666666666666666);
    Sc = fma(-s, t2, 1.0);
}

// ---------------------------------------------------------------------------
// Register DFTs.  Forward: X[k] = sum_n x[n] exp(-2 pi i n k / R); inverse
// uses exp(+...), unnormalised.  Radix 8 and 16 split as Q x 4 with the
// inner twiddles exp(-+2 pi i q s / R) as literal constants.
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b)
{
    cx<T> s = add(a, b), d = sub(a, b);
    a = s;
    b = d;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T>& x0, cx<T>& x1, cx<T>& x2, cx<T>& x3)
{
    cx<T> s02 = add(x0, x2), d02 = sub(x0, x2);
    cx<T> s13 = add(x1, x3), d13 = rot90<T, INV>(sub(x1, x3));
    x0 = add(s02, s13);
    x2 = sub(s02, s13);
    x1 = add(d02, d13);
    x3 = sub(d02, d13);
}

// cos/sin(2 pi j / 16), j = 0..15 (literal constants)
struct tw16 {
    static constexpr double c[16] = {1.0,
                                     0.92387953251128675613,
                                     0.70710678118654752440,
                                     0.38268343236508977173,
                                     0.0,
                                     -0.38268343236508977173,
                                     -0.70710678118654752440,
                                     -0.92387953251128675613,
                                     -1.0,
                                     -0.92387953251128675613,
                                     -0.70710678118654752440,
                                     -0.38268343236508977173,
                                     0.0,
                                     0.38268343236508977173,
                                     0.70710678118654752440,
                                     0.92387953251128675613};
    static constexpr double s[16] = {0.0,
                                     0.38268343236508977173,
                                     0.70710678118654752440,
                                     0.92387953251128675613,
                                     1.0,
                                     0.92387953251128675613,
                                     0.70710678118654752440,
                                     0.38268343236508977173,
                                     0.0,
                                     -0.38268343236508977173,
                                     -0.70710678118654752440,
                                     -0.92387953251128675613,
                                     -1.0,
                                     -0.92387953251128675613,
                                     -0.70710678118654752440,
                                     -0.38268343236508977173};
};

// In float the rotations are the nearest float of each of c and s: the
// phase of every pair is then within half a unit in the last place of the
// exact one.  Their squared magnitudes fall short of 1 (by 3e-8 for j = 2
// mod 4, 6e-8 for odd j), a small loss of norm in every transform that is
// the same from step to step; the step loop takes it out on average through
// its kinetic table (the host's transform-gain model of the kinetic step).
// Pairs chosen for c^2 + s^2 closest to 1 instead carry phase errors of up
// to about 1.3 units in the last place of one sign, which the band
// probabilities pick up coherently, step after step.
// The loss differs from bin to bin, and not evenly in +-k (2048 points: bins
// +1 and -1 lose 0.7e-7 and 1.9e-7 per round trip), so the momentum
// distribution drifts linearly in the step count: bins +80 and -80 (the
// orders +-k_L of a 2048-point row over 80 wavelengths) part by 0.6% per
// 1e5 steps.  With QW_F32_SPLIT_ROTATIONS = 1 each float constant is a pair
// hi + lo (lo the float nearest the rest of the double value), and the lo
// products enter the sum before the hi products are rounded, so the
// constant is exact to about 2^-48 (a lo product added after the rounding is mostly lost: it
// reaches half a unit in the last place only near the top of a binade).
// That costs 2 FMAs per real product, about 3% of the 2048^2 FP32 step.
#ifndef QW_F32_SPLIT_ROTATIONS
#define QW_F32_SPLIT_ROTATIONS 0
#endif
// multiply by exp(-+2 pi i j / 16) with j a compile-time constant
template <typename T, bool INV, int J>
__device__ __forceinline__ cx<T> tw16mul(cx<T> a)
{
    constexpr int j = J & 15;
    if constexpr (j == 0) return a;
    else if constexpr (j == 4) return rot90<T, INV>(a);
    else if constexpr (j == 8) return cx<T>{-a.re, -a.im};
    else if constexpr (j == 12) return rot90<T, !INV>(a);
    else {
        const T c = (T)tw16::c[j];
        const T sj = (T)tw16::s[j];
        const T s = INV ? sj : -sj;
        if constexpr (sizeof(T) == sizeof(float) && QW_F32_SPLIT_ROTATIONS) {
            const T cl = (T)(tw16::c[j] - (double)c);
            const T slj = (T)(tw16::s[j] - (double)sj);
            const T sl = INV ? slj : -slj;
            return cx<T>{fmx(a.re, c, fmx(-a.im, s, fmx(a.re, cl, -(a.im * sl)))),
                         fmx(a.re, s, fmx(a.im, c, fmx(a.re, sl, a.im * cl)))};
        }
        return cx<T>{fmx(a.re, c, -(a.im * s)), fmx(a.re, s, a.im * c)};
    }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cx<T>* x)
{
    if constexpr (R == 1) {
    } else if constexpr (R == 2) {
        dft2<T, INV>(x[0], x[1]);
    } else if constexpr (R == 4) {
        dft4<T, INV>(x[0], x[1], x[2], x[3]);
    } else if constexpr (R == 8) {
        // n = q + 2 l (q < 2, l < 4), k = s + 4 u (s < 4, u < 2)
        dft4<T, INV>(x[0], x[2], x[4], x[6]);
        dft4<T, INV>(x[1], x[3], x[5], x[7]);
        // twiddle exp(-+2 pi i q s / 8) = w16^(2 q s) on the q = 1 row
        x[3] = tw16mul<T, INV, 2>(x[3]);
        x[5] = tw16mul<T, INV, 4>(x[5]);
        x[7] = tw16mul<T, INV, 6>(x[7]);
        cx<T> y[8];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            cx<T> a = x[2 * s], b = x[2 * s + 1];
            y[s] = add(a, b);
            y[s + 4] = sub(a, b);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = y[k];
    } else if constexpr (R == 16) {
        // n = q + 4 l (q, l < 4), k = s + 4 u (s, u < 4)
        cx<T> y[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            cx<T> a = x[q], b = x[q + 4], c = x[q + 8], d = x[q + 12];
            dft4<T, INV>(a, b, c, d);  // index s = 0..3
            y[4 * q + 0] = a;
            y[4 * q + 1] = b;
            y[4 * q + 2] = c;
            y[4 * q + 3] = d;
        }
        // twiddles w16^(q s)
        y[4 * 1 + 1] = tw16mul<T, INV, 1>(y[5]);
        y[4 * 1 + 2] = tw16mul<T, INV, 2>(y[6]);
        y[4 * 1 + 3] = tw16mul<T, INV, 3>(y[7]);
        y[4 * 2 + 1] = tw16mul<T, INV, 2>(y[9]);
        y[4 * 2 + 2] = tw16mul<T, INV, 4>(y[10]);
        y[4 * 2 + 3] = tw16mul<T, INV, 6>(y[11]);
        y[4 * 3 + 1] = tw16mul<T, INV, 3>(y[13]);
        y[4 * 3 + 2] = tw16mul<T, INV, 6>(y[14]);
        y[4 * 3 + 3] = tw16mul<T, INV, 9>(y[15]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            cx<T> a = y[s], b = y[4 + s], c = y[8 + s], d = y[12 + s];
            dft4<T, INV>(a, b, c, d);  // index u = 0..3
            x[s] = a;
            x[s + 4] = b;
            x[s + 8] = c;
            x[s + 12] = d;
        }
    } else {
        static_assert(R == 16, "radix must be 1, 2, 4, 8 or 16");
    }
}

// ---------------------------------------------------------------------------
// Stockham transform of length N over a group of NT = N/E threads.
//
// Ownership: before and after every pass, thread t of a sequence holds the
// elements at positions t + NT m, m = 0..E-1.  A pass of radix R with
// stride NS takes the butterflies j = t + NT b (b < E/R), whose inputs
// j + r N/R are exactly the thread's slots b + r E/R, applies the twiddles
// w^(r (j mod NS)) with w = exp(-+2 pi i / (NS R)), does the radix-R DFT and
// writes output r to position (j / NS) NS R + (j mod NS) + r NS.  Between
// passes the outputs go through LDS; after the last pass (NS R = N) every
// output position equals an input position of the same thread, so the
// result is already in natural order in the same slots.
// ---------------------------------------------------------------------------
template <int... R>
struct sched {};

// LDS padding: one extra element every 2^sh elements breaks the
// power-of-two strides of the exchanges.  Measured on MI355X: every 32
// elements for 8-byte (float) elements, every 8 for 16-byte (double)
// elements, whose stride-8 writes of the first exchange otherwise land on
// the same banks (2048^2 FP64: rows 207 -> 190 us, columns 173 -> 164 us).
#ifndef QW_LDS_PADSH_F32
#define QW_LDS_PADSH_F32 5
#endif
#ifndef QW_LDS_PADSH_F64
#define QW_LDS_PADSH_F64 3
#endif
template <typename T>
struct lds_pad {
    static constexpr int sh = sizeof(T) == sizeof(float) ? QW_LDS_PADSH_F32 : QW_LDS_PADSH_F64;
};
template <typename T>
__device__ __forceinline__ constexpr int lpad(int i) { return i + (i >> lds_pad<T>::sh); }
template <typename T, int N>
struct lds_len {
    static constexpr int value = N + (N >> lds_pad<T>::sh);
};

// Twiddles are stored per pass: for a pass (NS, R) with NS > 1 the entries
// tw[jm R + r] = exp(-2 pi i jm r / (NS R)), jm < NS, r < R, follow the
// previous passes' entries (sum of NS R over passes < 2N).  A butterfly reads
// its R entries from one base: R/2 (float) or R (double) 16-byte loads with
// immediate offsets.
template <typename T, int N, int E, bool INV, int NS, int R>
__device__ __forceinline__ void load_twiddles(cx<T> (&w)[E / R][R], int t, const cx<T>* __restrict__ tw)
{
    constexpr int NT = N / E;
    if constexpr (NS > 1) {
        // keep these loads and their offsets here: hoisting or sharing them
        // across passes would hold every pass's twiddles in registers
        asm volatile("" ::: "memory");
        int tt = t;
        asm volatile("" : "+v"(tt));
#pragma unroll
        for (int b = 0; b < E / R; ++b) {
            const int jm = (tt + NT * b) & (NS - 1);
            const cx2<T>* tp = reinterpret_cast<const cx2<T>*>(tw + jm * R);
#pragma unroll
            for (int r = 0; r < R; r += 2) {
                const cx2<T> pr = tp[r / 2];
                w[b][r] = INV ? conj(pr.a) : pr.a;
                w[b][r + 1] = INV ? conj(pr.b) : pr.b;
            }
        }
    }
}

template <typename T, int N, int E, int NC, bool INV, int NS, int R>
__device__ __forceinline__ void fft_pass(cx<T> (&v)[NC][E], const cx<T> (&w)[E / R][R])
{
    constexpr int B = E / R;
    static_assert(E % R == 0, "radix must divide the per-thread element count");
#pragma unroll
    for (int b = 0; b < B; ++b) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            cx<T> x[R];
#pragma unroll
            for (int r = 0; r < R; ++r) x[r] = v[c][b + r * B];
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) x[r] = mul(x[r], w[b][r]);
            }
            dft<T, R, INV>(x);
#pragma unroll
            for (int r = 0; r < R; ++r) v[c][b + r * B] = x[r];
        }
    }
}

template <int R, int... Rest>
struct first_of {
    static constexpr int value = R;
};

// entries the per-pass twiddle table of a schedule needs
template <int NS, int R, int... Rest>
struct tw_len {
    static constexpr int value = (NS > 1 ? NS * R : 0) + tw_len<NS * R, Rest...>::value;
};
template <int NS, int R>
struct tw_len<NS, R> {
    static constexpr int value = NS > 1 ? NS * R : 0;
};

// Move one component from pass-output order to the next pass's slots via LDS.
template <typename T, int N, int E, int NS, int R>
__device__ __forceinline__ void fft_exchange(cx<T> (&vc)[E], int t, cx<T>* lds)
{
    constexpr int NT = N / E;
    constexpr int B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + NT * b;
        const int base = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lpad<T>(base + r * NS)] = vc[b + r * B];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) vc[m] = lds[lpad<T>(t + NT * m)];
    __syncthreads();
}

// Runs the passes.  With PF the twiddles of pass p+1 are loaded before pass
// p's LDS exchange, so their latency hides behind it.
#ifndef QW_TW_PREFETCH
#define QW_TW_PREFETCH 1
#endif
template <typename T, int N, int E, int NC, bool INV, bool PF, int NS, int R, int... Rest>
__device__ __forceinline__ void fft_run(cx<T> (&v)[NC][E], const cx<T> (&w)[E / R][R], int t,
                                        const cx<T>* __restrict__ tw, cx<T>* lds)
{
    fft_pass<T, N, E, NC, INV, NS, R>(v, w);
    if constexpr (sizeof...(Rest) > 0) {
        constexpr int R2 = first_of<Rest...>::value;
        const cx<T>* tw2 = tw + (NS > 1 ? NS * R : 0);
        cx<T> w2[E / R2][R2];
        if constexpr (PF) load_twiddles<T, N, E, INV, NS * R, R2>(w2, t, tw2);
#pragma unroll
        for (int c = 0; c < NC; ++c) fft_exchange<T, N, E, NS, R>(v[c], t, lds);
        if constexpr (!PF) load_twiddles<T, N, E, INV, NS * R, R2>(w2, t, tw2);
        fft_run<T, N, E, NC, INV, PF, NS * R, Rest...>(v, w2, t, tw2, lds);
    }
}

// PF: prefetch each pass's twiddles before the previous exchange (hides
// their latency; holds them in registers across the exchange)
template <typename T, int N, int E, int NC, bool INV, bool PF = QW_TW_PREFETCH, int R0, int... R>
__device__ __forceinline__ void fft(sched<R0, R...>, cx<T> (&v)[NC][E], int t, const cx<T>* __restrict__ tw,
                                    cx<T>* lds)
{
    cx<T> w0[E / R0][R0];  // the first pass (stride 1) has no twiddles
    fft_run<T, N, E, NC, INV, PF, 1, R0, R...>(v, w0, t, tw, lds);
}

// ---------------------------------------------------------------------------
// 2x2 block propagator  P = C I - i (a sigma_z + bx sigma_x + by sigma_y)
// acting on (top, bot).  In the order (psi1, psi4) block A takes the
// coefficients as given; block B in the order (psi2, psi3) takes -by, which
// in the order (psi3, psi2) used by the kernels becomes (C, -a, bx, by):
//   top' = (C - i a) top + (-by - i bx) bot
//   bot' = ( by - i bx) top + (C + i a) bot
// Kinetic: C = cos(E dt), (a, bx, by) = sin(E dt)/E (c^2, c px, c py).
// Interaction: C = cos(c|A| dt), a = 0, (bx, by) = sin(c|A| dt)/|A| (Ax, Ay).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void block_prop(cx<T>& top, cx<T>& bot, T C, T a, T bx, T by)
{
    const cx<T> t = {fmx(bx, bot.im, fmx(-by, bot.re, fmx(a, top.im, C * top.re))),
                     fmx(-bx, bot.re, fmx(-by, bot.im, fmx(-a, top.re, C * top.im)))};
    const cx<T> b = {fmx(-a, bot.im, fmx(C, bot.re, fmx(bx, top.im, by * top.re))),
                     fmx(a, bot.re, fmx(C, bot.im, fmx(-bx, top.re, by * top.im)))};
    top = t;
    bot = b;
}

// the same with a = 0 (the interaction propagator)
template <typename T>
__device__ __forceinline__ void block_prop0(cx<T>& top, cx<T>& bot, T C, T bx, T by)
{
    const cx<T> t = {fmx(bx, bot.im, fmx(-by, bot.re, C * top.re)), fmx(-bx, bot.re, fmx(-by, bot.im, C * top.im))};
    const cx<T> b = {fmx(C, bot.re, fmx(bx, top.im, by * top.re)), fmx(C, bot.im, fmx(-bx, top.re, by * top.im))};
    top = t;
    bot = b;
}

}  // namespace qw
