/* Oracle internals (test infrastructure only; see wmc_oracle.h). */
#ifndef WO_INTERNAL_H
#define WO_INTERNAL_H
#include <stdint.h>
#include "wmc_oracle.h"

#define WO_PI 3.14159265358979323846

/* one counter-based Philox4x32-10 stream; each double uses half a block */
typedef struct {
    uint32_t ctr[4];
    uint32_t key[2];
    uint32_t next;     /* index of the next double */
    int64_t cached;    /* block index held in w, or -1 */
    uint32_t w[4];
} wo_stream;

void wo_stream_init(wo_stream* s, uint64_t seed, int32_t system, int64_t sweep, int32_t tag,
                    int64_t cell, int64_t t, int32_t r, int32_t j);
uint64_t wo_next_bits(wo_stream* s);   /* 53 random bits */
double wo_next_co(wo_stream* s);       /* uniform in [0,1) */
double wo_next_oc(wo_stream* s);       /* uniform in (0,1] */
int64_t wo_next_index(wo_stream* s, int64_t n); /* uniform in {0..n-1} */

typedef struct {
    int64_t b0, b1, N;
    double L, lmax;
    int32_t n_levels;
    wo_level_info lev[WO_MAX_LEVELS];
    wo_system_info info;
    double* cube_w;     /* [n_modes] weight I(|k| lmax) of each cube mode */
    double* cube_cdf;   /* [n_modes] running sum of cube_w */
    double* shell_s;    /* [n_shell + 1] s = x_s/x at u = i/n_shell */
    int32_t n_shell;
    double x_s;
    double* inf_s;      /* infinite system: [n_inf + 1] s = x v at t = i/n_inf, v = 1 - t^3 */
    int32_t n_inf;
    int64_t accepted;
    /* linked-cell list for pair search (the cell index method), periodic systems only */
    int32_t nc;          /* cells per axis, 0 = no list (scan every bead) */
    double cg, invcg;    /* cell side >= r_cut + twice the largest plane-wave amplitude */
    int64_t* head;       /* [nc^3] first bead of each cell, -1 if empty */
} wo_system;

typedef struct {
    wo_params p;
    int32_t nsys;
    wo_system* sys;
    int64_t N;
    double *x, *y, *z;
    uint8_t* bond_next;      /* bead i bonded to bead i+1 */
    int64_t n_chains;
    int64_t* chain_off;
    int64_t sweep;
    wo_obs obs;
    double rc2, r_int;
    /* scratch */
    int64_t *S, *H, *M;
    int64_t* mark;
    int64_t *cnext, *cprev, *ccell;  /* per bead: linked-cell neighbours and its cell */
    int64_t* seen;                    /* per bead stamp for de-duplicating candidates */
    int64_t seen_stamp;
    int64_t mark_stamp;
    double *nx, *ny, *nz;
    wo_trace_rec* trace;
    int64_t trace_cap, trace_n;
    char err[256];
} wo_ctx;

/* tables */
int wo_build_system_tables(wo_ctx* c, wo_system* s, const wo_system* donor);
void wo_free_system_tables(wo_system* s);

#endif
