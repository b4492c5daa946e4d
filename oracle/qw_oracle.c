/*
 * qw_oracle.c -- TEST INFRASTRUCTURE ONLY (the oracle).
 *
 * A plain, slow, double-precision CPU implementation of the FFT
 * split-operator propagation of the four-component Dirac spinor on a
 * periodic 2D grid in a standing-wave vector potential, written from the
 * paper (Ge, Ahrens, Shen, "Two-dimensional simulation of the spin-flip in
 * the Kapitza-Dirac effect"):
 *   - Hamiltonian H = c alpha.(p + A) + beta c^2 in atomic units
 *     (Sec. II.B, Eq. 5, standard/Dirac representation);
 *   - bispinors u^s(p) with the x-polarised basis chi^{+-} (Eq. 9-10),
 *     energy E(p) (Eq. 11);
 *   - Gaussian packet in momentum space (Sec. II.C, Eq. 12-13) and the
 *     Fourier pair Eq. 14, discretised;
 *   - one split-operator step Psi(t+dt) = U(t+dt,t) Psi(t) (Sec. II.D, Eq. 15),
 *     taken in the symmetric (Strang) order V/2 - K - V/2;
 *   - the spin projections c^s = <u^s|phi> (Sec. III.B, Eq. 18) and the
 *     momentum density |phi|^2 (Eq. 19), summed over diffraction bands.
 *
 * Everything is explicit: 4x4 complex matrices (no block decomposition), a
 * textbook iterative radix-2 Cooley-Tukey FFT with twiddles taken directly
 * from cos/sin, and sums in a fixed order so results do not depend on the
 * thread count.  Only the tests, the smoke check and the benchmark's CPU
 * baseline load this library.  It shares no code with the HIP library.
 */
#include "qw_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double OR_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------ */
/* threads                                                                   */
/* ------------------------------------------------------------------------ */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* FFT: textbook iterative radix-2 decimation in time                        */
/* Forward: X[k] = sum_j x[j] exp(-2 pi i j k / n)  (sign = -1)             */
/* Inverse: unnormalised, exp(+2 pi i j k / n)      (sign = +1)             */
/* ------------------------------------------------------------------------ */
static int is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }

int or_fft1d(double *data, int n, int sign)
{
    cplx *a = (cplx *)data;
    if (!is_pow2(n) || (sign != 1 && sign != -1)) return -1;
    /* bit-reversal permutation */
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    /* butterflies of growing length, twiddle exp(sign 2 pi i k / len) */
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2;
        for (int k = 0; k < half; k++) {
            double ang = sign * 2.0 * OR_PI * (double)k / (double)len;
            cplx w = cos(ang) + I * sin(ang);
            for (int i = 0; i < n; i += len) {
                cplx u = a[i + k];
                cplx v = a[i + k + half] * w;
                a[i + k] = u + v;
                a[i + k + half] = u - v;
            }
        }
    }
    return 0;
}

/* 2D transform of a [ny][nx][ncomp] array: rows (x) then columns (y), each
 * component separately.  sign=-1 forward (unnormalised), sign=+1 inverse
 * including the 1/(nx ny) factor, so inverse(forward(x)) = x.  */
int or_dft2(double *data, int nx, int ny, int ncomp, int sign)
{
    cplx *psi = (cplx *)data;
    if (!is_pow2(nx) || !is_pow2(ny) || ncomp < 1) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|:bad)
    for (int y = 0; y < ny; y++) {
        cplx *line = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
        for (int c = 0; c < ncomp; c++) {
            for (int x = 0; x < nx; x++) line[x] = psi[((size_t)y * nx + x) * ncomp + c];
            bad |= or_fft1d((double *)line, nx, sign);
            for (int x = 0; x < nx; x++) psi[((size_t)y * nx + x) * ncomp + c] = line[x];
        }
        free(line);
    }
#pragma omp parallel for schedule(static) reduction(|:bad)
    for (int x = 0; x < nx; x++) {
        cplx *line = (cplx *)malloc(sizeof(cplx) * (size_t)ny);
        for (int c = 0; c < ncomp; c++) {
            for (int y = 0; y < ny; y++) line[y] = psi[((size_t)y * nx + x) * ncomp + c];
            bad |= or_fft1d((double *)line, ny, sign);
            for (int y = 0; y < ny; y++) psi[((size_t)y * nx + x) * ncomp + c] = line[y];
        }
        free(line);
    }
    if (sign == 1) {
        double s = 1.0 / ((double)nx * (double)ny);
        size_t tot = (size_t)nx * ny * ncomp;
        for (size_t i = 0; i < tot; i++) psi[i] *= s;
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Grid coordinates (Eq. 14 discretised on a periodic box)                   */
/* ------------------------------------------------------------------------ */
static double coord(double lo, double len, int n, int i) { return lo + len * (double)i / (double)n; }

/* signed FFT index: 0..n/2-1 stay, n/2..n-1 map to -n/2..-1 (Nyquist is -n/2) */
static int signed_index(int k, int n) { return k < n / 2 ? k : k - n; }

static double momentum(double len, int n, int k) { return 2.0 * OR_PI * (double)signed_index(k, n) / len; }

/* ------------------------------------------------------------------------ */
/* Dirac matrices, standard representation (Eq. 5)                           */
/*   beta = diag(1, 1, -1, -1),  alpha_k = [[0, sigma_k], [sigma_k, 0]]      */
/* ------------------------------------------------------------------------ */
static void pauli(int k, cplx s[2][2])
{
    if (k == 0) { s[0][0] = 0; s[0][1] = 1;  s[1][0] = 1; s[1][1] = 0; }   /* sigma_x */
    if (k == 1) { s[0][0] = 0; s[0][1] = -I; s[1][0] = I; s[1][1] = 0; }   /* sigma_y */
    if (k == 2) { s[0][0] = 1; s[0][1] = 0;  s[1][0] = 0; s[1][1] = -1; }  /* sigma_z */
}

static void dirac_alpha(int k, cplx m[4][4])
{
    cplx s[2][2];
    pauli(k, s);
    memset(m, 0, sizeof(cplx) * 16);
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            m[i][j + 2] = s[i][j];
            m[i + 2][j] = s[i][j];
        }
}

static void dirac_beta(cplx m[4][4])
{
    memset(m, 0, sizeof(cplx) * 16);
    m[0][0] = 1; m[1][1] = 1; m[2][2] = -1; m[3][3] = -1;
}

/* Free Hamiltonian H0(p) = c (alpha_x px + alpha_y py) + beta c^2, m = hbar = 1. */
static void hamiltonian0(double px, double py, double c, cplx h[4][4])
{
    cplx ax[4][4], ay[4][4], b[4][4];
    dirac_alpha(0, ax);
    dirac_alpha(1, ay);
    dirac_beta(b);
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) h[i][j] = c * (ax[i][j] * px + ay[i][j] * py) + b[i][j] * c * c;
}

/* Energy E(p) = sqrt(m^2 c^4 + c^2 p^2) (Eq. 11), m = 1. */
static double energy(double px, double py, double c) { return sqrt(c * c * c * c + c * c * (px * px + py * py)); }

/* Kinetic propagator exp(-i H0 tau) = cos(E tau) I - i sin(E tau) H0/E,
 * exact because H0^2 = E^2 I. */
static void kinetic_prop(double px, double py, double c, double tau, cplx k[4][4])
{
    cplx h[4][4];
    hamiltonian0(px, py, c, h);
    double e = energy(px, py, c);
    double ce = cos(e * tau), se = sin(e * tau);
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) k[i][j] = (i == j ? ce : 0.0) - I * se * h[i][j] / e;
}

/* Interaction propagator exp(-i c alpha.A tau) = cos(th) I - i (sin(th)/|A|) alpha.A,
 * th = c |A| tau, exact because (alpha.A)^2 = |A|^2 I.  At |A| = 0 the factor
 * sin(th)/|A| takes its limit c tau; below th = 1e-4 its Taylor series. */
static void interaction_prop(double ax_, double ay_, double c, double tau, cplx v[4][4])
{
    cplx ax[4][4], ay[4][4];
    dirac_alpha(0, ax);
    dirac_alpha(1, ay);
    double amag = sqrt(ax_ * ax_ + ay_ * ay_);
    double th = c * amag * tau;
    double s;
    if (fabs(th) < 1e-4) s = c * tau * (1.0 - th * th / 6.0 + th * th * th * th / 120.0);
    else s = sin(th) / amag;
    double ct = cos(th);
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) v[i][j] = (i == j ? ct : 0.0) - I * s * (ax[i][j] * ax_ + ay[i][j] * ay_);
}

static void apply4(cplx m[4][4], cplx *psi)
{
    cplx o[4];
    for (int i = 0; i < 4; i++) {
        o[i] = 0;
        for (int j = 0; j < 4; j++) o[i] += m[i][j] * psi[j];
    }
    for (int i = 0; i < 4; i++) psi[i] = o[i];
}

/* ------------------------------------------------------------------------ */
/* Vector potential                                                          */
/* Standing wave of two counter-propagating Gaussian beams (Sec. II.A,       */
/* Eq. 1-4) in the paraxial limit x << x_R at z = 0:                         */
/*   A_y = A0 exp(-y^2/w0^2) cos(kL x) cos(w t) f(t)                         */
/*   A_x = A0 (2y/(kL w0^2)) exp(-y^2/w0^2) sin(kL x) cos(w t) f(t)          */
/* with kL = 2 pi / lambda, w = c kL, and the ramp f(t) = sin^2(pi t/(2 Tr))  */
/* for t < Tr = ramp_periods * (lambda / c), else 1.                          */
/* ------------------------------------------------------------------------ */
static double ramp(const or_beam *b, double c, double t)
{
    double tr = b->ramp_periods * (b->lambda_l / c);
    if (tr > 0.0 && t < tr) {
        double s = sin(OR_PI * t / (2.0 * tr));
        return s * s;
    }
    return 1.0;
}

/* ------------------------------------------------------------------------ */
/* The full Gaussian-beam standing wave (Sec. II.A, Eq. 1a/1b, 2, 3, 4):      */
/* for d = +1, -1 and r^2 = y^2 (the z = 0 plane),                            */
/*   A_x,d = -2 d A0 (w0/w) eps (y/w) exp(-r^2/w^2) cos(phi1_d)               */
/*   A_y,d = -A0 (w0/w) exp(-r^2/w^2) sin(phi_d)                              */
/*   phi_d  = w t - d kL x + atan(d x / xR) - d x r^2 / (xR w^2)              */
/*   phi1_d = phi_d + atan(d x / xR)                                          */
/*   w(x) = w0 sqrt(1 + x^2/xR^2),  xR = kL w0^2 / 2,  eps = 1/(kL w0),       */
/* summed over d and multiplied by the switch-on f(t).                        */
/* ------------------------------------------------------------------------ */
static void gaussian_full(const or_beam *b, double c, double x, double y, double t, double *out_ax, double *out_ay)
{
    double kl = 2.0 * OR_PI / b->lambda_l;
    double om = c * kl;
    double w0 = b->w0;
    double eps = 1.0 / (kl * w0);
    double xr = 0.5 * kl * w0 * w0;
    double w = w0 * sqrt(1.0 + (x * x) / (xr * xr));
    double r2 = y * y;
    double env = (w0 / w) * exp(-r2 / (w * w));
    double ax = 0.0, ay = 0.0;
    for (int d = -1; d <= 1; d += 2) {
        double phi = om * t - d * kl * x + atan(d * x / xr) - d * x * r2 / (xr * w * w);
        double phi1 = phi + atan(d * x / xr);
        ay += -b->a0 * env * sin(phi);
        ax += -2.0 * d * b->a0 * env * eps * (y / w) * cos(phi1);
    }
    double f = ramp(b, c, t);
    *out_ax = b->longitudinal ? ax * f : 0.0;
    *out_ay = ay * f;
}

void or_beam_eval(const or_beam *b, double c, double x, double y, double t, double *out_ax, double *out_ay)
{
    double ax = 0.0, ay = 0.0;
    if (b->mode == OR_BEAM_GAUSSIAN_FULL) {
        gaussian_full(b, c, x, y, t, out_ax, out_ay);
        return;
    }
    if (b->mode == OR_BEAM_UNIFORM) {
        ax = b->ux;
        ay = b->uy;
    } else if (b->mode == OR_BEAM_STANDING_PARAXIAL) {
        double kl = 2.0 * OR_PI / b->lambda_l;
        double om = c * kl;
        double env = exp(-(y * y) / (b->w0 * b->w0));
        double tt = cos(om * t) * ramp(b, c, t);
        ay = b->a0 * env * cos(kl * x) * tt;
        if (b->longitudinal) ax = b->a0 * (2.0 * y / (kl * b->w0 * b->w0)) * env * sin(kl * x) * tt;
    }
    *out_ax = ax;
    *out_ay = ay;
}

/* ------------------------------------------------------------------------ */
/* Split-operator steps (Eq. 15): V(t_k, dt/2) F^-1 K(dt) F V(t_{k+1}, dt/2)  */
/* in application order V(t_k,dt/2) first.  t_k = t0 + k dt.                  */
/* ------------------------------------------------------------------------ */
/* In a frame (vy, a_m) the box coordinate y stands for the lab point y + vy t,
 * the Hamiltonian in box coordinates is H(p + a_m e_y, A(x, y + vy t, t)) - vy p_y,
 * and the scalar -vy p_y, diagonal in momentum space, joins the kinetic part:
 * exp(-i (H0(p + a_m e_y) - vy p_y) tau) = exp(i vy p_y tau) K(p + a_m e_y, tau). */
static void apply_interaction(const or_grid *g, const or_beam *b, const or_frame *f, cplx *psi, double t, double tau)
{
#pragma omp parallel for schedule(static)
    for (int iy = 0; iy < g->ny; iy++) {
        double y = coord(g->y_min, g->ly, g->ny, iy) + f->vy * t;
        for (int ix = 0; ix < g->nx; ix++) {
            double x = coord(g->x_min, g->lx, g->nx, ix);
            double ax, ay;
            cplx v[4][4];
            or_beam_eval(b, g->c, x, y, t, &ax, &ay);
            interaction_prop(ax, ay, g->c, tau, v);
            apply4(v, psi + ((size_t)iy * g->nx + ix) * 4);
        }
    }
}

static void apply_kinetic(const or_grid *g, const or_frame *f, cplx *phi, double tau)
{
#pragma omp parallel for schedule(static)
    for (int ky = 0; ky < g->ny; ky++) {
        double py = momentum(g->ly, g->ny, ky);
        cplx shift = cexp(I * f->vy * py * tau);
        for (int kx = 0; kx < g->nx; kx++) {
            double px = momentum(g->lx, g->nx, kx);
            cplx k[4][4];
            kinetic_prop(px, py + f->a_m, g->c, tau, k);
            for (int i = 0; i < 4; i++)
                for (int j = 0; j < 4; j++) k[i][j] *= shift;
            apply4(k, phi + ((size_t)ky * g->nx + kx) * 4);
        }
    }
}

int or_step_n_frame(const or_grid *g, const or_beam *b, const or_frame *f, double *data, long n, double t0,
                    double dt)
{
    cplx *psi = (cplx *)data;
    if (!is_pow2(g->nx) || !is_pow2(g->ny) || n < 0) return -1;
    for (long k = 0; k < n; k++) {
        double tk = t0 + (double)k * dt;
        double tk1 = t0 + (double)(k + 1) * dt;
        apply_interaction(g, b, f, psi, tk, 0.5 * dt);
        or_dft2(data, g->nx, g->ny, 4, -1);
        apply_kinetic(g, f, psi, dt);
        or_dft2(data, g->nx, g->ny, 4, +1);
        apply_interaction(g, b, f, psi, tk1, 0.5 * dt);
    }
    return 0;
}

int or_step_n(const or_grid *g, const or_beam *b, double *data, long n, double t0, double dt)
{
    const or_frame lab = {0.0, 0.0};
    return or_step_n_frame(g, b, &lab, data, n, t0, dt);
}

/* ------------------------------------------------------------------------ */
/* Bispinors (Eq. 9-10), normalised to unit length                           */
/*   u^s(p) ~ ( chi^s , c sigma.p chi^s / (E + c^2) ),                       */
/*   chi^+ = (1, 1)/sqrt2, chi^- = (1, -1)/sqrt2 (x-polarised basis).         */
/* ------------------------------------------------------------------------ */
void or_spinor(double px, double py, double c, int s, double *out)
{
    cplx *u = (cplx *)out;
    cplx sx[2][2], sy[2][2];
    pauli(0, sx);
    pauli(1, sy);
    double r2 = 1.0 / sqrt(2.0);
    cplx chi[2] = {r2, (s >= 0 ? r2 : -r2)};
    double e = energy(px, py, c);
    double pre = sqrt((e + c * c) / (2.0 * c * c));
    for (int i = 0; i < 2; i++) {
        cplx sp = 0;
        for (int j = 0; j < 2; j++) sp += (sx[i][j] * px + sy[i][j] * py) * chi[j];
        u[i] = pre * chi[i];
        u[i + 2] = pre * c * sp / (e + c * c);
    }
    double nn = 0.0;
    for (int i = 0; i < 4; i++) nn += creal(u[i] * conj(u[i]));
    nn = sqrt(nn);
    for (int i = 0; i < 4; i++) u[i] /= nn;
}

/* ------------------------------------------------------------------------ */
/* Initial packet (Eq. 12-14):                                               */
/*   phi(p) = g(p) u^s(p) exp(-i p.r0),  g = exp(-|p - p0|^2 / (4 sp^2)),     */
/*   sp = 1/(2 sigma_x);  psi(r_j) = sum_p phi(p) exp(i p.r_j), normalised    */
/*   to sum_cells |psi|^2 = 1.                                                */
/* ------------------------------------------------------------------------ */
/* In a frame with gauge shift a_m the grid momentum p is canonical; the
 * packet is centred on the kinetic momentum p0, i.e. on p = p0 - a_m e_y, and
 * its bispinors are those of the kinetic momentum p + a_m e_y. */
int or_init_packet_frame(const or_grid *g, const or_packet *e, const or_frame *f, double *data)
{
    cplx *psi = (cplx *)data;
    if (!is_pow2(g->nx) || !is_pow2(g->ny) || !(e->sigma_x > 0)) return -1;
    double sp = 1.0 / (2.0 * e->sigma_x);
    for (int ky = 0; ky < g->ny; ky++) {
        double py = momentum(g->ly, g->ny, ky);
        for (int kx = 0; kx < g->nx; kx++) {
            double px = momentum(g->lx, g->nx, kx);
            double dpx = px - e->p0x, dpy = py + f->a_m - e->p0y;
            double amp = exp(-(dpx * dpx + dpy * dpy) / (4.0 * sp * sp));
            /* exp(i p.(r_j - r0)) with r_j = r_min + j d: the r_min - r0 part
             * is a per-momentum phase, the j d part is the inverse DFT kernel */
            double ph = px * (g->x_min - e->x0) + py * (g->y_min - e->y0);
            cplx u[4];
            or_spinor(px, py + f->a_m, g->c, e->spin, (double *)u);
            for (int i = 0; i < 4; i++) psi[((size_t)ky * g->nx + kx) * 4 + i] = amp * u[i] * cexp(I * ph);
        }
    }
    or_dft2(data, g->nx, g->ny, 4, +1);
    double nn = 0.0;
    for (size_t i = 0; i < (size_t)g->nx * g->ny * 4; i++) nn += creal(psi[i] * conj(psi[i]));
    if (!(nn > 0)) return -1;
    double s = 1.0 / sqrt(nn);
    for (size_t i = 0; i < (size_t)g->nx * g->ny * 4; i++) psi[i] *= s;
    return 0;
}

int or_init_packet(const or_grid *g, const or_packet *e, double *data)
{
    const or_frame lab = {0.0, 0.0};
    return or_init_packet_frame(g, e, &lab, data);
}

/* ------------------------------------------------------------------------ */
/* Observables (Eq. 18-19).  phi = forward DFT2(psi).  Diffraction order n    */
/* collects the momentum columns within a closed window of half-width h      */
/* grid steps about p_ref + 2 n kL, with p_ref = r dk and kL = m dk (h < m,   */
/* so the one-photon sidebands at odd multiples of kL are never counted).     */
/* out = [norm, P_n (B), P_n^+ (B), P_n^- (B), P_flip, P_neg], B = 2 n_max+1. */
/* ------------------------------------------------------------------------ */
#define OR_NO_BAND (-(1 << 30))

static long floor_div(long a, long b)
{
    long q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q--;
    return q;
}

int or_band_index(int kx_signed, int ref_idx, int half_idx, int window_idx)
{
    /* nearest order centre, then the window test */
    long n = floor_div((long)kx_signed - ref_idx + half_idx, 2L * half_idx);
    long d = (long)kx_signed - ref_idx - 2L * half_idx * n;
    if (d < 0) d = -d;
    return d <= window_idx ? (int)n : OR_NO_BAND;
}

int or_observables(const or_grid *g, const double *data, const or_obs_spec *o, double *out, int out_len)
{
    const or_frame lab = {0.0, 0.0};
    return or_observables_frame(g, data, o, &lab, out, out_len);
}

/* With a gauge shift a_m the projections use the bispinors of the kinetic
 * momentum p + a_m e_y; the diffraction windows are on p_x (unchanged). */
int or_observables_frame(const or_grid *g, const double *data, const or_obs_spec *o, const or_frame *f, double *out,
                         int out_len)
{
    const cplx *psi = (const cplx *)data;
    int nb = 2 * o->n_max + 1;
    if (o->n_max < 0 || o->band_half_idx <= 0 || o->window_idx < 0 || o->window_idx >= o->band_half_idx ||
        out_len < 3 * nb + 3)
        return -1;
    size_t cells = (size_t)g->nx * g->ny;
    cplx *phi = (cplx *)malloc(sizeof(cplx) * cells * 4);
    if (!phi) return -1;
    memcpy(phi, psi, sizeof(cplx) * cells * 4);
    or_dft2((double *)phi, g->nx, g->ny, 4, -1);

    /* per-row partial sums, then a fixed-order sum over rows */
    int nacc = 3 * nb + 3; /* [P_n, P+_n, P-_n, total, flip, positive] */
    double *part = (double *)calloc((size_t)g->ny * nacc, sizeof(double));
    double *rnorm = (double *)calloc((size_t)g->ny, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int ky = 0; ky < g->ny; ky++) {
        double *acc = part + (size_t)ky * nacc;
        double py = momentum(g->ly, g->ny, ky);
        for (int kx = 0; kx < g->nx; kx++) {
            double px = momentum(g->lx, g->nx, kx);
            const cplx *q = phi + ((size_t)ky * g->nx + kx) * 4;
            cplx up[4], um[4];
            or_spinor(px, py + f->a_m, g->c, +1, (double *)up);
            or_spinor(px, py + f->a_m, g->c, -1, (double *)um);
            double w = 0.0;
            cplx cp = 0, cm = 0;
            for (int i = 0; i < 4; i++) {
                w += creal(q[i] * conj(q[i]));
                cp += conj(up[i]) * q[i];
                cm += conj(um[i]) * q[i];
            }
            double wp = creal(cp * conj(cp)), wm = creal(cm * conj(cm));
            int n = or_band_index(signed_index(kx, g->nx), o->band_ref_idx, o->band_half_idx, o->window_idx);
            if (n >= -o->n_max && n <= o->n_max) {
                acc[n + o->n_max] += w;
                acc[nb + n + o->n_max] += wp;
                acc[2 * nb + n + o->n_max] += wm;
            }
            acc[3 * nb] += w;
            acc[3 * nb + 1] += (o->spin0 >= 0 ? wm : wp);
            acc[3 * nb + 2] += wp + wm;
        }
        double r = 0.0;
        for (int kx = 0; kx < g->nx; kx++) {
            const cplx *p = psi + ((size_t)ky * g->nx + kx) * 4;
            for (int i = 0; i < 4; i++) r += creal(p[i] * conj(p[i]));
        }
        rnorm[ky] = r;
    }
    double *sum = (double *)calloc((size_t)nacc, sizeof(double));
    double norm = 0.0;
    for (int ky = 0; ky < g->ny; ky++) {
        for (int a = 0; a < nacc; a++) sum[a] += part[(size_t)ky * nacc + a];
        norm += rnorm[ky];
    }
    double tot = sum[3 * nb];
    out[0] = norm;
    for (int i = 0; i < 3 * nb; i++) out[1 + i] = sum[i] / tot;
    out[1 + 3 * nb] = sum[3 * nb + 1] / tot;
    out[2 + 3 * nb] = 1.0 - sum[3 * nb + 2] / tot;
    free(sum);
    free(part);
    free(rnorm);
    free(phi);
    int finite = 1;
    for (int i = 0; i < 3 * nb + 3; i++) finite &= isfinite(out[i]);
    return finite ? 0 : -5;
}

/* ------------------------------------------------------------------------ */
/* Matrix accessors for the self-tests (row-major 4x4 complex)               */
/* ------------------------------------------------------------------------ */
void or_hamiltonian0(double px, double py, double c, double *out)
{
    cplx h[4][4];
    hamiltonian0(px, py, c, h);
    memcpy(out, h, sizeof(h));
}

void or_kinetic_matrix(double px, double py, double c, double tau, double *out)
{
    cplx k[4][4];
    kinetic_prop(px, py, c, tau, k);
    memcpy(out, k, sizeof(k));
}

void or_interaction_matrix(double ax, double ay, double c, double tau, double *out)
{
    cplx v[4][4];
    interaction_prop(ax, ay, c, tau, v);
    memcpy(out, v, sizeof(v));
}

double or_energy(double px, double py, double c) { return energy(px, py, c); }
