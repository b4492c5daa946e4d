/*
 * qw_oracle.h -- TEST INFRASTRUCTURE ONLY.  Interface of the plain FP64 CPU
 * oracle of the Dirac FFT split-operator method.  The oracle's own types: it
 * includes nothing from the HIP library and the HIP library includes nothing
 * from here.
 *
 * Arrays are [ny][nx][4] complex128 (interleaved re, im), row-major, x fastest.
 */
#ifndef QW_ORACLE_H
#define QW_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_BEAM_NONE = 0, OR_BEAM_STANDING_PARAXIAL = 1, OR_BEAM_UNIFORM = 2, OR_BEAM_GAUSSIAN_FULL = 3 };

typedef struct {
    int nx, ny;                  /* powers of two */
    double x_min, y_min, lx, ly; /* periodic box [x_min, x_min + lx) x [y_min, y_min + ly) */
    double c;                    /* speed of light in atomic units */
} or_grid;

typedef struct {
    int mode;            /* OR_BEAM_* */
    double a0;           /* amplitude of A (momentum units) */
    double lambda_l;     /* laser wavelength */
    double w0;           /* beam waist */
    double ramp_periods; /* sin^2 switch-on length in laser periods; 0 = none */
    int longitudinal;    /* 1: include the longitudinal A_x component */
    double ux, uy;       /* OR_BEAM_UNIFORM only: constant A */
} or_beam;

/* Frame of the simulation: the box moves along y with velocity vy (box
 * coordinate y is the lab coordinate y - vy t), and a constant vector
 * potential a_m along y is added to the field (a gauge shift between the
 * canonical grid momentum p and the kinetic momentum p + a_m e_y). */
typedef struct {
    double vy;
    double a_m;
} or_frame;

typedef struct {
    double p0x, p0y;  /* central kinetic momentum */
    double x0, y0;    /* central position */
    double sigma_x;   /* position-density standard deviation */
    int spin;         /* +1: chi+ (spin +x), -1: chi- */
} or_packet;

typedef struct {
    int band_ref_idx;  /* p_ref = band_ref_idx * (2 pi / lx) */
    int band_half_idx; /* kL    = band_half_idx * (2 pi / lx) */
    int window_idx;    /* order n counts columns with |k - ref - 2 n half| <= window_idx */
    int n_max;         /* bands -n_max..n_max are reported */
    int spin0;         /* initial spin; P_flip sums |<u^{-spin0}|phi>|^2 */
} or_obs_spec;

void or_set_threads(int n);
int or_get_threads(void);

int or_fft1d(double *data, int n, int sign);
int or_dft2(double *data, int nx, int ny, int ncomp, int sign);

void or_beam_eval(const or_beam *b, double c, double x, double y, double t, double *ax, double *ay);
int or_step_n(const or_grid *g, const or_beam *b, double *psi, long n, double t0, double dt);
int or_step_n_frame(const or_grid *g, const or_beam *b, const or_frame *f, double *psi, long n, double t0,
                    double dt);
void or_spinor(double px, double py, double c, int s, double *u_out);
int or_init_packet(const or_grid *g, const or_packet *e, double *psi);
int or_init_packet_frame(const or_grid *g, const or_packet *e, const or_frame *f, double *psi);
int or_band_index(int kx_signed, int ref_idx, int half_idx, int window_idx); /* -(1<<30): none */
int or_observables(const or_grid *g, const double *psi, const or_obs_spec *o, double *out, int out_len);
int or_observables_frame(const or_grid *g, const double *psi, const or_obs_spec *o, const or_frame *f, double *out,
                         int out_len);

void or_hamiltonian0(double px, double py, double c, double *out16c);
void or_kinetic_matrix(double px, double py, double c, double tau, double *out16c);
void or_interaction_matrix(double ax, double ay, double c, double tau, double *out16c);
double or_energy(double px, double py, double c);

#ifdef __cplusplus
}
#endif
#endif
