/*
 * wmc.h - C ABI of the MI355X (gfx950) Wavelet Monte Carlo dynamics sweep.
 *
 * Method: Dyer & Ball, "Wavelet Monte Carlo dynamics: a new algorithm for simulating the
 * hydrodynamics of interacting Brownian particles" (arXiv:1611.09160). Bead-spring
 * polymers evolve by Metropolis-tested, spatially correlated moves:
 *   - vector-wavelet moves (Sec. IV, App. D "Generating a wavelet"): radius lambda with PDF
 *     ~ lambda^-4 on [lambda_min, lambda_max] (Eq. "PDF for lambda"), centre b uniform in a
 *     ball of radius lambda around a uniformly picked bead (Eq. "PDF for b"), isotropic
 *     polarisation p, amplitude A_w = A0 lambda / sqrt(n) (Eq. "Wavelet amplitude"),
 *     displacement A_w w((r - b)/lambda, p) with the tapered wavelet
 *     w(x, p) = (1 - |x|) p x x (Eqs. "Oseen as <ww>", "Tapered wavelet");
 *   - plane-wave moves in periodic boxes (Sec. V): displacement A_F cos(k.r + Phi) e-hat on
 *     every bead, e-hat perpendicular to k (Eq. "Oseen as <FF>"), A_F = (2/k) sqrt(dU_est/(mu N))
 *     (Eq. "Fourier strain energy"), k from the periodic lattice (Eq. "Prob of k_l"),
 *     made with probability P_F (Eq. "P(Fourier)");
 *   - acceptance min(1, exp(-dU/kT)) (Eq. "Metropolis test"), lambda / k recycling after a
 *     rejection and time advanced by dt per accepted move (App. D, Eqs. "Time step per
 *     wavelet", "dt w+F").
 * Interactions (Sec. II): FENE bonds (Eq. "FENE potential") or harmonic bonds, and WCA
 * between all pairs, bonded ones included (Eq. "WCA potential").
 *
 * Every random number comes from counter-based Philox4x32-10 streams keyed by
 * (seed; system, sweep, level or plane-wave tag, cell or chain, trial, retry, try), so a run
 * is reproducible and resumable from (positions, sweep counter, seed).
 *
 * Conventions
 *  - All functions return 0 on success or a negative WMC_E* code; the message is kept in
 *    the context (wmc_last_error). No exception crosses the ABI.
 *  - Host arrays are owned by the caller and only read (or written, for outputs) during
 *    the call. The device arena is owned by the caller (e.g. a torch uint8 tensor on the
 *    GPU) and must stay allocated until wmc_free; the library places all its device
 *    state inside it and allocates no device memory of its own.
 *  - hip_stream is a hipStream_t (NULL = the legacy default stream). wmc_sweep is
 *    asynchronous on that stream; wmc_positions(to_device=1) too; the other calls
 *    synchronise the stream before returning host data.
 *  - Positions are FP64, [N][3] row-major (x, y, z per bead), unwrapped (a bead's
 *    coordinates are never folded back into the box; minimum image is applied to every
 *    difference).
 *  - Beads are numbered 0..N-1. System s owns beads [sys_bead_offset[s],
 *    sys_bead_offset[s+1]); chain c owns beads [chain_offset[c], chain_offset[c+1]) and
 *    bonds join consecutive beads of one chain; chains may not cross systems.
 */
#ifndef WMC_H
#define WMC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    WMC_OK = 0,
    WMC_EINVAL = -1,     /* bad argument or parameter */
    WMC_ESTATE = -2,     /* initial state has infinite energy (overstretched bond, overlap) */
    WMC_EARENA = -3,     /* device arena missing or too small */
    WMC_EHIP = -4,       /* a HIP runtime call failed */
    WMC_ECAPACITY = -5,  /* a per-cell list overflowed its capacity during a sweep (the cell's
                            remaining moves were skipped; the sweep is not a valid sample) */
    WMC_ESCHEDULE = -6   /* a dependency wait between cells hit its bound (the cell was skipped;
                            the sweep is not a valid sample) */
};

enum { WMC_BOND_NONE = 0, WMC_BOND_FENE = 1, WMC_BOND_HARMONIC = 2 };
enum { WMC_FP64 = 0, WMC_MIXED = 1 };
/* acceptance test: Metropolis min(1, e^(-dU/kT)) (Eq. "Metropolis test"), or Glauber
 * 1/(1 + e^(dU/kT)) (anticipated at the end of Sec. IV "Choosing the wavelet amplitude") */
enum { WMC_ACCEPT_METROPOLIS = 0, WMC_ACCEPT_GLAUBER = 1 };
/* wavelet displacement: the linear map r + A w((r - b)/lambda, p) as printed (Eq. "Oseen as
 * <ww>"), or the exact rotation of r about the axis p through b by the angle
 * A (1 - |x|)/lambda, equal to it to first order, an exact involution (p -> -p) with unit
 * Jacobian, so that no Jacobian term is needed in the test (Sec. IV) */
enum { WMC_MAP_LINEAR = 0, WMC_MAP_ROTATION = 1 };
/* wavelet centres: uniform around a uniformly picked bead (Eq. "PDF for b"), or uniform in a
 * homogeneous periodic box with A_w = A0 lambda / sqrt(<n>), <n> = (4 pi/3) lambda^3 N/L^3 (Sec. IV
 * "Distribution of wavelet radii", last paragraph; the printed amplitude is read this way) */
enum { WMC_CENTRE_ANCHOR = 0, WMC_CENTRE_UNIFORM = 1 };
#define WMC_K_SHELLS 16

#define WMC_MAX_LEVELS 16

typedef struct wmc_ctx wmc_ctx;

/* Run parameters (Sec. II units: lengths in sigma, energies in epsilon). */
typedef struct {
    int32_t periodic;        /* 1: cubic periodic box; 0: infinite system (single system only) */
    int32_t plane_waves;     /* 1: plane-wave moves, Sec. V: the periodic lattice of k, or in an
                                infinite system k from P(k) ~ k^2 I(k lambda_max) (Eq. "PDF of k")
                                with P_F = (lambda_min/lambda_max)^3 (Eq. "P(Fourier) infinite") */
    int32_t wavelets;        /* 1: wavelet moves (0 only for plane-wave-only checks) */
    int32_t precision;       /* WMC_FP64, or WMC_MIXED: FP32 tile offsets, displacements,
                                distances and energy terms, FP64 positions, an FP64 recheck of
                                every decision within the FP32 error bound */
    double box_L;            /* box side, used when sys_box_L is NULL */
    double lambda_min;       /* smallest wavelet radius; sets a = lambda_min / lambda_a */
    double lambda_max;       /* largest wavelet radius (<= L/2), used when sys_lambda_max is NULL */
    double band_ratio;       /* lambda_hi / lambda_lo of one level band, in (1, 2] (2 = octaves) */
    double A0;               /* dimensionless move amplitude (Eq. "Wavelet amplitude") */
    double kT;               /* thermal energy */
    int32_t bond_type;       /* WMC_BOND_* */
    int32_t wca;             /* 1: WCA between all pairs */
    double k_bond;           /* FENE k, or harmonic k of U = (k/2) r^2 */
    double R0;               /* FENE maximum bond length */
    double sigma, eps;       /* WCA parameters */
    double r_int_harmonic;   /* interaction halo used with harmonic bonds (> longest bond) */
    int32_t n_layers;        /* half-width of the discrete k cube (App. D, 15) */
    int32_t retry_cap;       /* attempts per recycling chain before giving up (64) */
    uint64_t seed;           /* Philox key */
    int32_t accept_rule;     /* WMC_ACCEPT_* */
    int32_t wavelet_map;     /* WMC_MAP_* */
    int32_t centring;        /* WMC_CENTRE_* (UNIFORM needs a periodic box) */
    int32_t mixed_verify;    /* WMC_MIXED, 1: also evaluate every FP32-tile test in FP64 and
                                count those whose FP32 error exceeds the recheck margin (the
                                decisions are unchanged; slower, for validation) */
} wmc_params;

/* Counters summed over systems (wmc_observables). */
typedef struct {
    int64_t sweeps;
    int64_t trials[WMC_MAX_LEVELS];       /* trial centres drawn */
    int64_t hits[WMC_MAX_LEVELS];         /* trials whose centre fell in their cell */
    int64_t attempts[WMC_MAX_LEVELS];     /* Metropolis tests */
    int64_t accepts[WMC_MAX_LEVELS];
    int64_t caps[WMC_MAX_LEVELS];         /* chains ended by the retry cap */
    int64_t redraws[WMC_MAX_LEVELS];      /* centre redraws that missed during retries */
    int64_t bead_updates[WMC_MAX_LEVELS]; /* sum over attempts of the beads displaced */
    int64_t pw_chains, pw_attempts, pw_accepts, pw_k0, pw_caps, pw_bead_updates;
    int64_t violations;                   /* bonds found longer than the halo width */
    int64_t accepted_total;               /* accepted chains, wavelet + plane wave */
    int64_t rechecks;                     /* WMC_MIXED: decisions re-evaluated in FP64 */
    int64_t overflows;                    /* cell lists that exceeded capacity (must be 0) */
    int64_t grid_rebuilds;                /* neighbour-grid rebuilds */
    int64_t wait_timeouts;                /* dependency waits between cells that hit their bound
                                             (must be 0; the pass then ran out of order) */
    int64_t fallback_cells;               /* cells of LDS-tile levels whose halo did not fit the
                                             tile, run on the global-list path instead */
    int64_t accepted_bead_updates;        /* beads displaced by accepted moves (a k = 0 plane
                                             wave displaces none) */
    /* plane-wave tests and accepts per |k| shell (Fig. "k acceptance prob"): periodic
     * floor(|l|) of the lattice index l, infinite floor(|k| lambda_max), capped at 15 */
    int64_t pw_shell_attempts[WMC_K_SHELLS];
    int64_t pw_shell_accepts[WMC_K_SHELLS];
    int64_t member_rechecks;              /* WMC_MIXED: FP32 support tests re-evaluated in FP64 */
    int64_t margin_checks;                /* mixed_verify: tests evaluated in both precisions */
    int64_t margin_fails;                 /* ... whose |dU32 - dU64| exceeded the margin (must be 0) */
    double margin_max_ratio;              /* ... largest |dU32 - dU64| / margin seen */
} wmc_obs;

/* One trace record per Metropolis test (kind 0 wavelet, 2 plane wave) and per cell phase
 * (kind 1: trial = trial count, retry = |S_c|, n = 0, accepted = hits). */
typedef struct {
    int32_t kind, system, sweep, level, cell, trial, retry, n, accepted, extra;
    double dU, thr;
} wmc_trace_rec;

/* Bytes of device arena wmc_init needs for this problem (same arguments as wmc_init). */
int wmc_arena_bytes(const wmc_params* p, int32_t n_systems, const int64_t* sys_bead_offset,
                    const double* sys_box_L, const double* sys_lambda_max, int64_t n_chains,
                    const int64_t* chain_offset, int64_t trace_capacity, size_t* out_bytes);

/* The launch plan wmc_init would make for this problem if cell_blocks and pw_blocks workgroups of
 * its cell-group and plane-wave kernels could be co-resident, with launches capped at
 * cell_launch_max / pw_launch_max workgroups. Host only: no device is touched. Every index the
 * kernels derive from the plan (block maps, cooperative group tables, per-workgroup result slots,
 * barrier words, list slices, global list slots, cell flags) is checked; report (caller-owned,
 * report_bytes) receives "ok" or the first violation, then a summary. Returns 0, WMC_EINVAL for a
 * violation or bad arguments. (An inspection of the schedule the paper leaves to the
 * implementation, Sec. VII's parallel execution of non-overlapping moves.) */
int wmc_launch_plan(const wmc_params* p, int32_t n_systems, const int64_t* sys_bead_offset,
                    const double* sys_box_L, const double* sys_lambda_max, int64_t n_chains,
                    const int64_t* chain_offset, const double* pos_xyz, int32_t cell_blocks,
                    int32_t pw_blocks, int32_t cell_launch_max, int32_t pw_launch_max, char* report,
                    size_t report_bytes);

/* Set up the problem of Sec. II: N_b-bead chains with FENE (Eq. "FENE potential") or harmonic
 * bonds and WCA pairs (Eq. "WCA potential") in periodic boxes or an infinite system. Validates
 * the parameters, builds the per-system schedule tables (levels of Eq. "PDF for lambda", P_F of
 * Eqs. "P(Fourier)" / "P(Fourier) infinite", the k tables of App. D, dt of Eqs. "Time step per
 * wavelet" / "dt w+F"), copies the positions [N][3] (host, FP64, caller-owned, read only) into
 * the device arena and checks that the initial energy is finite. sys_box_L / sys_lambda_max may
 * be NULL (then params.box_L / params.lambda_max apply to every system). trace_capacity > 0
 * reserves room for that many trace records. Errors: WMC_EINVAL (parameters, topology),
 * WMC_ESTATE (an overstretched FENE bond or two beads of one system at the same point, whose
 * energy is infinite), WMC_EARENA (arena missing or smaller than wmc_arena_bytes), WMC_EHIP.
 * *out is set even on failure (for wmc_last_error) and must be freed with wmc_free. */
int wmc_init(wmc_ctx** out, const wmc_params* p, int32_t n_systems, const int64_t* sys_bead_offset,
             const double* sys_box_L, const double* sys_lambda_max, int64_t n_chains,
             const int64_t* chain_offset, const double* pos_xyz, int64_t trace_capacity,
             void* device_arena, size_t arena_bytes, void* hip_stream);

/* Size of the library-held device arena that wmc_init_static uses (one per device). */
#define WMC_STATIC_ARENA_BYTES (16u << 20)

/* wmc_init without a caller-supplied arena, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops or harnesses that forbid hipMalloc). The
 * context lives in a device array of WMC_STATIC_ARENA_BYTES that the library holds per device
 * until the process ends; no call allocates device memory (no hipMalloc, hipFree or allocating
 * library routine). Arguments as wmc_init, on the current device. Errors:
 *   WMC_EARENA  the problem needs more than WMC_STATIC_ARENA_BYTES (wmc_arena_bytes), or the
 *               device's array is held by a live context made here (at most one per device;
 *               wmc_free releases it);
 *   others      as wmc_init.
 * wmc_init clears the part of the array the problem uses; the array keeps the last context's
 * contents otherwise. All such contexts of a process on one device share that device's array:
 * the guard above admits one at a time, and calls on it that overlap in time (two host threads
 * sweeping it on different streams) race on the array, as they would on any arena. */
int wmc_init_static(wmc_ctx** out, const wmc_params* p, int32_t n_systems, const int64_t* sys_bead_offset,
                    const double* sys_box_L, const double* sys_lambda_max, int64_t n_chains,
                    const int64_t* chain_offset, const double* pos_xyz, int64_t trace_capacity,
                    void* hip_stream);

/* Run n_sweeps sweeps, asynchronously on hip_stream. One sweep = every wavelet level band
 * in colour phases, then the plane-wave chains (Sec. IV-V as summarised above). */
int wmc_sweep(wmc_ctx* c, int64_t n_sweeps, void* hip_stream);

/* The state of Sec. II: bead positions r_i, [N][3] FP64 unwrapped, copied to out_xyz (caller-owned)
 * in host memory (to_device = 0, synchronous) or device memory (to_device = 1, asynchronous on
 * hip_stream). */
int wmc_positions(wmc_ctx* c, double* out_xyz, int32_t to_device, void* hip_stream);

/* Replace the positions (host [N][3]) and set the sweep counter (which keys the streams). */
int wmc_set_state(wmc_ctx* c, const double* pos_xyz, int64_t sweep, void* hip_stream);

/* Counters of the moves (synchronises the device): per wavelet level the trials, hits, Metropolis
 * tests and accepts whose ratio is the acceptance of Fig. "wavelet acceptance plot", per |k| shell
 * the plane-wave tests and accepts of Fig. "k acceptance prob", and the bead-updates that measure
 * the cost per move (Sec. IV "Computational cost"). out is filled in every case. Returns
 * WMC_ECAPACITY when a cell list overflowed (overflows > 0) and WMC_ESCHEDULE when a dependency
 * wait hit its bound (wait_timeouts > 0) since wmc_init: the sweeps concerned are then not
 * valid samples of the method. */
int wmc_observables(wmc_ctx* c, wmc_obs* out);

/* Physical time per system in units of tau (Eq. "Unit of Time"): dt x accepted chains. */
int wmc_system_tau(wmc_ctx* c, double* out /* [n_systems] */);

/* Mean-square radius of gyration of every chain (Eq. "Radius of gyration"). */
int wmc_chain_rg2(wmc_ctx* c, double* out /* [n_chains] */);

/* Centre of mass of every chain from the unwrapped positions (Sec. VI.B), host [n_chains][3]. */
int wmc_chain_com(wmc_ctx* c, double* out);

/* Squared displacement of every chain's centre of mass since the positions of wmc_init or the
 * last wmc_set_state, host [n_chains]; <.>/(6 t) over chains is D of Sec. VI.B. */
int wmc_chain_msd(wmc_ctx* c, double* out);

/* Move up to max trace records to out (host) and clear the trace; returns the count in
 * *n_out. Records are in completion order; sort by (sweep, system, level, cell, trial, retry). */
int wmc_trace(wmc_ctx* c, wmc_trace_rec* out, int64_t max, int64_t* n_out);

/* Schedule constants of one system, for inspection: per level (lo, hi, p, T, h, ncell) and
 * (P_F, R, N_k, P_cube, P_k0, dt). levels_out holds 6 doubles per level. */
int wmc_system_info(wmc_ctx* c, int32_t system, double* levels_out, int32_t* n_levels,
                    double* pw_out /* 6 doubles */);

/* Cell index of every bead of one system in the grid of (sweep, level) at the current
 * positions (the cell a wavelet centre at that point would belong to). out is host [N_s]. */
int wmc_cell_ids(wmc_ctx* c, int32_t system, int64_t sweep, int32_t level, int32_t* out);

/* Philox4x32-10 on the device for n consecutive counters starting at ctr (ctr[0] is
 * incremented), key fixed; out is host [n][4]. For cross-checking the generator. */
int wmc_philox(const uint32_t ctr[4], const uint32_t key[2], int64_t n, uint32_t* out,
               void* device_scratch, size_t scratch_bytes, void* hip_stream);

/* Kernel timing. With timing on, wmc_sweep records HIP events on its stream around every
 * kernel class; wmc_kernel_times synchronises and returns, per class, the summed duration
 * (ms) and the number of launches since timing was switched on. Classes: 0 neighbour-grid
 * build (4 kernels), 1 + l the colour phases of level l (l < WMC_MAX_LEVELS), 17 plane waves. */
#define WMC_TIMING_CLASSES 18
int wmc_set_timing(wmc_ctx* c, int32_t enable);
int wmc_kernel_times(wmc_ctx* c, double* ms_out, int64_t* launches_out);

/* Launch tuning (an implementation choice the paper leaves open: how the concurrent moves of
 * Sec. VII are scheduled on the device; results stay those of the method). Per level, LDS-tile
 * cells run as one dependency-ordered pass ("flow") or one launch per colour ("colours"), with a
 * kernel variant at least the planned one ("V64" < "V256" < "V1024": tile capacity and threads per
 * cell) and, for V64 passes, 64 or 256 threads per cell; global-list cells run as cooperative cell
 * groups ("groups": "on") or one workgroup per cell ("off"); plane waves likewise.
 *
 * wmc_tune: from the current state, times trial_sweeps sweeps (after one untimed sweep) for each
 * candidate choice of every level at once, keeps the fastest per level, and restores the state
 * (positions, sweep counter, counters, trace) exactly as it was. It allocates a device copy of the
 * context's arena while it runs (freed before it returns). json_out (caller-owned, json_bytes)
 * receives the chosen settings with their times as
 *   {"trial_sweeps": k, "levels": [{"level": 0, "cells": "tile", "pass": "flow", "variant": "V64",
 *    "width": 256, "groups": "on", "ms_per_sweep": t}, ...], "plane_wave_groups": "on", ...}
 * ("cells": which kinds of cell the level has, "tile", "global" or "tile+global"; informative).
 * Periodic systems with wavelet moves only; WMC_EINVAL otherwise or when json_out is too small.
 * wmc_set_tuning: applies such a JSON text (fields may be omitted: the plan's choice; unknown
 * values: WMC_EINVAL, nothing applied). wmc_get_tuning: the settings in force, same format. */
int wmc_tune(wmc_ctx* c, int32_t trial_sweeps, char* json_out, size_t json_bytes);
int wmc_set_tuning(wmc_ctx* c, const char* json);
int wmc_get_tuning(wmc_ctx* c, char* json_out, size_t json_bytes);

const char* wmc_last_error(const wmc_ctx* c);
void wmc_free(wmc_ctx* c);

#ifdef __cplusplus
}
#endif
#endif
