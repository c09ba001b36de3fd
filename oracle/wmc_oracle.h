/*
 * Plain FP64 serial reference ("oracle") of the Wavelet Monte Carlo dynamics sweep
 * (Dyer & Ball, "Wavelet Monte Carlo dynamics", arXiv:1611.09160).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call this
 * library: only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * use it. It shares no code, header, table generator or helper with the HIP library.
 *
 * What it computes, in the paper's order and notation:
 *   - wavelet moves (Sec. IV, App. D "Generating a wavelet"): radius lambda with
 *     P(lambda) ~ lambda^-4, centre b uniform in a ball of radius lambda around a
 *     uniformly picked particle, isotropic polarisation p, amplitude A_w = A0 lambda/sqrt(n),
 *     displacement A_w w((r-b)/lambda, p) with the tapered wavelet w = (1-|x|) p x x;
 *   - Metropolis acceptance min(1, exp(-dU/kT)) with no Jacobian term (Sec. IV);
 *   - lambda recycling after a rejection (App. D "Parameter recycling");
 *   - plane-wave moves for periodic boxes (Sec. V, App. D "Generating a plane wave"):
 *     amplitude A_F = (2/k) sqrt(dU_est/(mu N)), discrete k-cube plus quasi-continuous
 *     shell, P_F from R, k recycling by permuting and sign-flipping components;
 *   - plane waves in an infinite system (Sec. V "Distributions of wavevectors", App. D
 *     "Choosing k for an infinite system"): |k| from P(k) ~ k^2 I(k lambda_max) by a tabulated
 *     inverse CDF, isotropic k-hat, P_F = (lambda_min/lambda_max)^3 (Eq. "P(Fourier) infinite"),
 *     |k| kept and k-hat redrawn after a rejection;
 *   - time advanced only on accepted moves (Eqs. "Time step per wavelet", "dt w+F").
 * Variants the paper names or implies, selected in wo_params:
 *   - Glauber acceptance 1/(1 + exp(dU/kT)) (Sec. IV "Choosing the wavelet amplitude", last
 *     paragraph, which anticipates it);
 *   - the exact-rotation wavelet map: each member rotated about the axis p through b by the
 *     angle A (1 - |x|) / lambda, which equals x + A w(x) to first order and is an exact
 *     involution (p -> -p) with unit Jacobian, so "no Jacobian needed" (Sec. IV) holds exactly;
 *   - uniform centring for homogeneous periodic systems (Sec. IV "Distribution of wavelet
 *     radii", last paragraph): b uniform in the box, A_w = A0 lambda / sqrt(<n>) with
 *     <n> = (4 pi/3) lambda^3 N / L^3 (the printed A_w is dimensionally garbled; this is the
 *     form that keeps P_b A_w^2 of the anchored scheme).
 * The serial paper loop is replayed in the coloured cell schedule of the GPU path
 * (levels of octave bands, cells of side >= 2 lambda_hi + r_int, 8 colours, per-cell
 * trial counts by stochastic rounding, per-cell retry chains), drawing every random
 * number from the same counter-based Philox4x32-10 streams. The schedule is a reading
 * of the paper, which is serial: it fixes neither the cells, nor the colours, nor the
 * per-cell trial counts, only the distributions the moves are drawn from.
 */
#ifndef WMC_ORACLE_H
#define WMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WO_MAX_LEVELS 16

enum { WO_BOND_NONE = 0, WO_BOND_FENE = 1, WO_BOND_HARMONIC = 2 };

typedef struct {
    int32_t periodic;        /* 1: cubic periodic box of side box_L; 0: infinite system */
    int32_t plane_waves;     /* 1: add plane-wave moves (periodic only) */
    int32_t wavelets;        /* 1: wavelet levels on (0 only for plane-wave-only checks) */
    int32_t pad0;
    double box_L;            /* default box side (per-system override possible) */
    double lambda_min;       /* smallest wavelet radius */
    double lambda_max;       /* largest wavelet radius (per-system override possible) */
    double band_ratio;       /* ratio lambda_hi/lambda_lo of one level band, in (1, 2] */
    double A0;               /* dimensionless amplitude, Eq. "Wavelet amplitude" */
    double kT;               /* thermal energy */
    int32_t bond_type;       /* WO_BOND_* */
    int32_t wca;             /* 1: WCA between all pairs, bonded ones included */
    double k_bond;           /* FENE k, or harmonic k in U = (k/2) r^2 */
    double R0;               /* FENE maximum extension */
    double sigma, eps;       /* WCA parameters */
    double r_int_harmonic;   /* halo width used with harmonic bonds (> 0) */
    int32_t n_layers;        /* half-width of the discrete k cube (15 in the paper) */
    int32_t retry_cap;       /* max attempts of one recycling chain (64) */
    uint64_t seed;           /* Philox key */
    int32_t accept_rule;     /* WO_ACCEPT_METROPOLIS (Eq. "Metropolis test") or WO_ACCEPT_GLAUBER */
    int32_t wavelet_map;     /* WO_MAP_LINEAR (x + A w, as printed) or WO_MAP_ROTATION (exact) */
    int32_t centring;        /* WO_CENTRE_ANCHOR (Eq. "PDF for b") or WO_CENTRE_UNIFORM (periodic) */
    int32_t pad1;
} wo_params;

enum { WO_ACCEPT_METROPOLIS = 0, WO_ACCEPT_GLAUBER = 1 };
enum { WO_MAP_LINEAR = 0, WO_MAP_ROTATION = 1 };
enum { WO_CENTRE_ANCHOR = 0, WO_CENTRE_UNIFORM = 1 };
#define WO_K_SHELLS 16

typedef struct {
    int64_t sweeps;
    int64_t trials[WO_MAX_LEVELS];      /* trial centres drawn */
    int64_t hits[WO_MAX_LEVELS];        /* trials whose centre fell inside their cell */
    int64_t attempts[WO_MAX_LEVELS];    /* Metropolis tests */
    int64_t accepts[WO_MAX_LEVELS];
    int64_t caps[WO_MAX_LEVELS];        /* chains ended by the retry cap */
    int64_t redraws[WO_MAX_LEVELS];     /* centre redraws that missed during retries */
    int64_t bead_updates[WO_MAX_LEVELS];/* sum of n over attempts */
    int64_t pw_chains, pw_attempts, pw_accepts, pw_k0, pw_caps, pw_bead_updates;
    int64_t violations;                 /* bonds longer than the halo width (harmonic) */
    int64_t accepted_total;             /* wavelet + plane-wave accepted chains */
    int64_t accepted_bead_updates;      /* beads displaced by accepted moves (k = 0: none) */
    /* plane-wave tests and accepts per |k| shell: periodic floor(|l|) (l the lattice index),
     * infinite floor(|k| lambda_max), both capped at WO_K_SHELLS - 1 */
    int64_t pw_shell_attempts[WO_K_SHELLS];
    int64_t pw_shell_accepts[WO_K_SHELLS];
} wo_obs;

typedef struct {
    int32_t kind;        /* 0 wavelet attempt, 1 cell summary, 2 plane-wave attempt */
    int32_t system, sweep, level, cell, trial, retry, n, accepted, extra;
    double dU, thr;      /* energy change and threshold -kT ln u */
} wo_trace_rec;

typedef struct {
    double lo, hi, p, T;     /* band, probability mass, expected chain starts per sweep */
    double h;                /* cell side (periodic) */
    int32_t ncell;           /* cells per axis (periodic) */
    int32_t pad;
    double r_int;
} wo_level_info;

typedef struct {
    double P_F, R, N_k, P_cube, W_cube, W_cont, W_corner, P_k0, dt;
    int32_t n_levels, n_modes;
} wo_system_info;

/* lifecycle; positions are [N][3] host FP64; sys_box_L / sys_lambda_max may be NULL */
int wo_init(void** out, const wo_params* p, int32_t n_systems, const int64_t* sys_bead_offset,
            const double* sys_box_L, const double* sys_lambda_max, int64_t n_chains,
            const int64_t* chain_offset, const double* pos_xyz, int64_t trace_capacity);
int wo_sweep(void* ctx, int64_t n_sweeps);
int wo_positions(void* ctx, double* out_xyz);
int wo_set_positions(void* ctx, const double* xyz);
int wo_set_sweep(void* ctx, int64_t sweep);
int wo_observables(void* ctx, wo_obs* out);
int wo_system_tau(void* ctx, double* out);
int wo_chain_rg2(void* ctx, double* out);
int wo_chain_com(void* ctx, double* out);  /* [n_chains][3] centre of mass, unwrapped positions */
int64_t wo_trace(void* ctx, wo_trace_rec* out, int64_t max);
int wo_get_level_info(void* ctx, int32_t system, wo_level_info* out, int32_t max);
int wo_get_system_info(void* ctx, int32_t system, wo_system_info* out);
int wo_cell_ids(void* ctx, int32_t system, int64_t sweep, int32_t level, int32_t* out);
int wo_cube_weights(void* ctx, int32_t system, double* out);
int wo_shell_table(void* ctx, int32_t system, double* out, int32_t max);
/* infinite system: s(t) = x v at t = i/M, v = 1 - t^3 the tail probability G(x)/G(0) */
int wo_inf_table(void* ctx, int32_t system, double* out, int32_t max);
/* |k| lambda_max of an infinite-system plane wave from its tail probability v in (0, 1] */
double wo_inf_k_of_v(void* ctx, int32_t system, double v);
double wo_G(double x);
const char* wo_last_error(void* ctx);
void wo_free(void* ctx);

/* building blocks exposed for the closed-form pins */
void wo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double wo_inv_cbrt(double x);
double wo_phit(double q);
double wo_I(double x);
double wo_J6(double x);
double wo_M(int m);
void wo_wavelet(const double x[3], const double p[3], double out[3]);
double wo_u_fene(double r2, double k, double R0);
double wo_u_wca(double r2, double sigma, double eps);
/* draw n doubles of one trial stream (system, sweep, tag, cell, t, r, j) */
void wo_stream_doubles(uint64_t seed, int32_t system, int64_t sweep, int32_t tag, int64_t cell,
                       int64_t t, int32_t r, int32_t j, int32_t n, double* out_co, double* out_oc);
/* lambda of a level band from one uniform in [0,1) */
double wo_draw_lambda(double u, double lo, double hi);

#ifdef __cplusplus
}
#endif
#endif
