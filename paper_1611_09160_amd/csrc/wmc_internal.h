// Internal layout shared by the host and device translation units of libwmc.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/wmc.h"

namespace wmc {

constexpr double kPi = 3.14159265358979323846;

// Philox stream tags (third counter word, high byte)
constexpr int TAG_META = 16;     // + level: per-cell trial count draw
constexpr int TAG_SHIFT = 32;    // + level: grid shift
constexpr int TAG_PWCOUNT = 48;  // plane-wave chain count
constexpr int TAG_PW = 49;       // plane-wave chains

// counter slots (uint64)
constexpr int CNT_LEVEL = 0;     // [level*8 + k], k: trials hits attempts accepts caps redraws beads
constexpr int CNT_PW = 128;      // chains attempts accepts k0 caps beads
constexpr int CNT_VIOL = 136;
constexpr int CNT_OVERFLOW = 137;
constexpr int CNT_RECHECK = 138;
constexpr int CNT_REBUILD = 139;
constexpr int CNT_ACCEPTED = 140;
constexpr int CNT_FLOWWAIT = 141;   // dependency waits that hit their spin limit (must be 0)
constexpr int CNT_ACC_BEADS = 143;  // beads displaced by accepted moves, wavelet and plane wave
constexpr int CNT_FALLBACK = 142;   // LDS-tile cells whose halo did not fit: run on the global-list path
constexpr int CNT_SHELL = 144;      // [2 * shell + accepted]: plane-wave tests per |k| shell
constexpr int CNT_MEMBER_RECHECK = 176;  // FP32-tile support tests re-evaluated in FP64
constexpr int CNT_MARGIN_CHECK = 177;    // mixed_verify: tests evaluated in both precisions
constexpr int CNT_MARGIN_FAIL = 178;     // ... whose FP32 error exceeded the recheck margin
constexpr int CNT_MARGIN_RATIO = 179;    // ... largest error / margin, as FP32 bits (atomic max)
constexpr int CNT_TOTAL = 184;

// Cooperative launches: groups of co-resident workgroups, each group on one (system, cell) of a
// colour phase or on one system's plane waves. A group owns workgroups [first, first + size)
// of the launch and the same range of per-workgroup result slots; its barrier counters are
// gbar[2 (1 + group index) ..].
struct CoopGroup {
    int32_t sys, local, first, size;
};
// The colour phases one cell-group launch runs in order: colour col[i] with its group table
// goff[i] int32 entries past the first colour's. Several colours share a launch only when their tables hold the same groups
// (system, first workgroup, size), so each group runs its system's colours back to back and
// never waits for another system.
struct CoopColours {
    int32_t n;
    int32_t col[8];
    int32_t goff[8];
};
// Group and launch sizes: a barrier costs more the more workgroups of a group arrive, and every
// arriving workgroup writes back its L2, so a launch is also capped in total.
#ifndef WMC_CELL_GROUP_MAX
#define WMC_CELL_GROUP_MAX 16
#endif
#ifndef WMC_CELL_LAUNCH_MAX
#define WMC_CELL_LAUNCH_MAX 256
#endif
#ifndef WMC_PW_GROUP_MAX
#define WMC_PW_GROUP_MAX 128
#endif
#ifndef WMC_PW_LAUNCH_MAX
#define WMC_PW_LAUNCH_MAX 512
#endif
constexpr int COOP_SLOTS = 1024;      // workgroups of one cooperative launch at most
constexpr int CELL_GROUP_MAX = WMC_CELL_GROUP_MAX;    // workgroups per cell group
constexpr int CELL_LAUNCH_MAX = WMC_CELL_LAUNCH_MAX;  // workgroups per cell-group launch
constexpr int CELL_GROUP_BEADS = 1024;                // beads per workgroup of a cell group
constexpr int PW_GROUP_MAX = WMC_PW_GROUP_MAX;        // workgroups per plane-wave group
constexpr int PW_LAUNCH_MAX = WMC_PW_LAUNCH_MAX;      // workgroups per plane-wave launch
constexpr int PW_GROUP_BEADS = 256;                   // beads per workgroup of a plane-wave group
constexpr int COOP_LIST_CAP = 4096;  // list entries one workgroup of a cell group holds (LDS)

// kernel variants of the cell phase: threads per workgroup and LDS list capacities
enum Variant { V64 = 0, V256 = 1, V1024 = 2 };

struct SysDesc {
    int64_t b0, b1;
    int32_t N, n_levels;
    double L, invL, lmax, dt;
    // plane waves
    double PF, P_cube, W_cube, x_s, ks, invks;
    int64_t cube_off;      // offset of this system's cube CDF in the table pool
    int64_t shell_off;     // offset of its shell table (periodic) or of the infinite-system table
    int32_t n_modes, n_shell;
    // neighbour grid
    int32_t nf, pad0;
    double g, invg;
    int64_t fine_off;      // first fine cell of this system
    int32_t lvl_off, pad1; // index of level 0 in the level table
};

struct LevelDesc {
    double lo, hi, p, T, h, invh, half, r_int;
    int32_t n;             // cells per axis (periodic)
    int32_t variant;
    int32_t identity;      // the cell holds every bead (n == 1)
    int32_t use_global;    // reach and member lists in global slots
    int64_t slot_base;     // first global slot of this (system, level)
    int64_t flag_base;     // first done-flag of this (system, level)'s cells
};

struct DevParams {
    int32_t periodic, plane_waves, wavelets, precision;
    int32_t bond_type, wca, retry_cap, n_layers;
    int32_t accept_rule, wavelet_map, centring, mixed_verify;
    double A0, kT, k_bond, R0, R02, sigma2, eps, rc2, rc, r_int;
    uint32_t seed_lo, seed_hi;
    int32_t nsys, pad;
};

struct DevPtrs {
    double *x, *y, *z;          // positions (unwrapped)
    double *xb, *yb, *zb;       // positions at the last neighbour-grid build
    uint8_t* bond_next;         // bead i bonded to bead i+1
    int32_t* sys_id;            // system of each bead
    int32_t* tag;               // member index of a bead during a test, else -1
    const SysDesc* sys;
    const LevelDesc* lev;
    int32_t *fcount, *fstart, *fidx, *fcell;
    int32_t* fblock;            // per-chunk sums of the grid scan
    unsigned long long* drift;  // per system, bits of the max drift since the grid build
    unsigned long long* drift_col;  // per (system, colour): drift published by that colour phase
    double* cell_drift;         // per (system, level, cell): largest drift of the beads it moved
    unsigned long long* cnt;    // CNT_* counters
    unsigned long long* sys_acc;// accepted chains per system
    wmc_trace_rec* trace;
    unsigned long long* trace_n;
    int64_t trace_cap;
    const double* cube_cdf;
    const double* shell_s;
    int32_t* slot_S;            // global reach lists, slot_len entries per slot
    int32_t* slot_M;            // global member lists
    double* slot_MX;            // global member positions (3 * slot_len per slot)
    int64_t slot_len;
    double* pw_new;             // plane-wave trial positions [3N]
    unsigned* gbar;             // grid barrier: arrivals, generation
    int32_t* cell_done;         // per (system, level, cell): epoch of its last completed pass
    unsigned long long* flow_ctr;  // per level: cells handed out by the dependency-ordered kernel
    int32_t* coop_i;            // per-workgroup counts of the cooperative kernels [COOP_SLOTS]
    double* coop_d;             // per-workgroup partial results [5][COOP_SLOTS]
    double* igrid;              // infinite-system grid of the current level: o[3], n[3], k0[3]
    double* com_ref;            // per chain: centre of mass at the reference positions [3 n_chains]
    int64_t total_fine;
};

// kernel launchers (device translation unit)
void launch_fine_build(const DevParams& P, const DevPtrs& D, int64_t N, hipStream_t st);
void launch_bbox(const DevParams& P, const DevPtrs& D, int level, int64_t sweep, hipStream_t st);
void launch_phase(int variant, const DevParams& P, const DevPtrs& D, int level, int colour, int64_t sweep,
                  const int32_t* bmap, int nblocks, hipStream_t st);
// One level pass of LDS-tile cells in dependency order (all colours in one launch).
struct FlowArgs {
    int32_t colour_end[8];   // items [colour_end[c-1], colour_end[c]) have colour c
    int32_t nitems;
    int32_t epoch;           // value a completed cell publishes; never reused within a context
    unsigned long long qbase;  // flow_ctr[level] before this launch
};
// width64: threads per cell of the smallest tile variant (0: 256 up to 4,096 cells, else 64)
void launch_level_flow(int variant, const DevParams& P, const DevPtrs& D, int level, int64_t sweep,
                       const int32_t* items, const FlowArgs& fa, int width64, hipStream_t st);
void launch_pw(const DevParams& P, const DevPtrs& D, int64_t sweep, int nsys, hipStream_t st);
bool launch_pw_coop(const DevParams& P, const DevPtrs& D, int64_t sweep, const CoopGroup* groups,
                    const int32_t* wg_group, int nwg, hipStream_t st);
bool launch_cell_coop(const DevParams& P, const DevPtrs& D, int level, const CoopColours& cc, int64_t sweep,
                      const CoopGroup* groups, const int32_t* wg_group, int nwg, hipStream_t st);
int cell_coop_blocks();
int pw_coop_blocks();
void launch_rg2(const DevPtrs& D, const int64_t* chain_off, int64_t n_chains, double* out, hipStream_t st);
// mode 0: centre of mass [3 n] to out; 1: the same into D.com_ref; 2: |com - com_ref|^2 [n] to out
void launch_com(const DevPtrs& D, const int64_t* chain_off, int64_t n_chains, int mode, double* out, hipStream_t st);
void launch_cell_ids(const DevParams& P, const DevPtrs& D, int sys, int level, int64_t sweep, int64_t n, int32_t* out,
                     hipStream_t st);
void launch_philox(const uint32_t* ctr, const uint32_t* key, int64_t n, uint32_t* out, hipStream_t st);
// Device address of the library-held arena on `device` (the current device), looked up once per
// device; nullptr with *err set when the lookup fails.
constexpr int kMaxDevices = 64;
void* static_arena(int device, hipError_t* err);

}  // namespace wmc
