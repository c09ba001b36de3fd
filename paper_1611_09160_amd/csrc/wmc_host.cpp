// Host side of libwmc: schedule constants, device arena layout and the C ABI (include/wmc.h).
//
// Schedule constants per system (Dyer & Ball, arXiv:1611.09160):
//   levels   bands [lo, lo*band_ratio) from lambda_min up to lambda_max, probability mass
//            p = (lo^-3 - hi^-3)/(lambda_min^-3 - lambda_max^-3) (Eq. "PDF for lambda"), expected
//            chain starts per sweep T = N (1 - P_F) p; periodic cells: the largest even count n
//            with L/n >= (2 hi + r_int)(1 + 1e-9), else a single cell.
//   P_F      Eq. "P(Fourier)" with R = (L/lambda_max)^3 M6 N_k / (6 pi^2) (Sec. V.C); N_k normalises
//            P(k_l) ~ I(|k_l| lambda_max) (Eq. "Prob of k_l") over the discrete cube of App. D plus
//            the quasi-continuous shell outside it.
//   dt       Eq. "dt w+F" with plane waves, Eq. "Time step per wavelet" without.
// I(x) = int_x^inf q^3 phi~(q)^2 dq and J6(x) = int_x^inf q^6 phi~(q)^2 dq are integrated here
// with 20-point Gauss-Legendre panels of width 1/2 plus asymptotic tails beyond Q = 4096.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>
#include <cctype>
#include <cstdio>
#include <cstdlib>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "wmc_internal.h"

using namespace wmc;

struct wmc_ctx {
    wmc_params p;
    DevParams P;
    DevPtrs D;
    int32_t nsys;
    int64_t N, n_chains;
    std::vector<SysDesc> sys;
    std::vector<LevelDesc> lev;
    std::vector<std::vector<double>> level_out;  // per system: 6 doubles per level
    std::vector<std::vector<double>> pw_out;     // per system: 6 doubles
    int max_levels;
    int phase_variant[WMC_MAX_LEVELS];
    std::vector<int32_t> bmap_host;
    int64_t bmap_off[WMC_MAX_LEVELS][8];  // every cell of the colour
    int32_t bmap_n[WMC_MAX_LEVELS][8];
    int64_t tile_off[WMC_MAX_LEVELS][8];  // LDS-tile cells (run by the dependency-ordered pass)
    int32_t tile_n[WMC_MAX_LEVELS][8];
    int64_t glob_off[WMC_MAX_LEVELS][8];  // global-list cells (cooperative groups or k_phase)
    int32_t glob_n[WMC_MAX_LEVELS][8];
    unsigned long long flow_handed[WMC_MAX_LEVELS] = {0};  // cells handed out per level so far
    int32_t flow_epoch = 0;
    // launch choices (wmc_tune / wmc_set_tuning), 0 = the plan's: tile levels run one
    // dependency-ordered pass (1) or one launch per colour (2), with a kernel variant of at least
    // the plan's (variant + 1) and, for the smallest, 64 or 256 threads per cell; global-list
    // levels use their cell groups (1) or one workgroup per cell (2); plane waves likewise
    int tune_pass[WMC_MAX_LEVELS] = {0};
    int tune_variant[WMC_MAX_LEVELS] = {0};
    int tune_width[WMC_MAX_LEVELS] = {0};
    int tune_groups[WMC_MAX_LEVELS] = {0};
    int tune_pw = 0;
    int32_t* bmap_dev;
    // cooperative groups (int32 table: CoopGroup records, then the workgroup -> group map)
    std::vector<int32_t> coop_host;
    int32_t* coop_dev;
    int64_t cgrp_off[WMC_MAX_LEVELS][8], cwg_off[WMC_MAX_LEVELS][8];
    int32_t cwg_n[WMC_MAX_LEVELS][8];     // workgroups of the cell-group launch (0: none)
    bool cmerge[WMC_MAX_LEVELS];          // every colour of the level in one cell-group launch
    int64_t pgrp_off = 0, pwg_off = 0;
    int32_t pwg_n = 0;                    // workgroups of the plane-wave group launch (0: none)
    int64_t* chain_off_dev;
    double* rg2_dev;
    int64_t sweep;
    // kernel timing: event pairs per class, summed lazily
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    double t_ms[WMC_TIMING_CLASSES] = {0};
    int64_t t_n[WMC_TIMING_CLASSES] = {0};
    char* arena;
    size_t arena_bytes;
    size_t arena_used = 0;  // bytes from `arena` (256-B aligned) the context's sub-arrays occupy
    int static_dev = -1;  // device whose library-held arena this context uses (wmc_init_static), else -1
    std::string err;
};

namespace {

// ------------------------------------------------------------------ tapered wavelet
double phit(double q) {
    // phi~(q) = 4 pi int_0^1 r^2 phi(r) sin(qr)/(qr) dr with phi = r^2/2 - r^3/3 - 1/6: for
    // small q by its power series, else the closed form 4 pi q^-6 (5q sin q - (q^2-8) cos q - 8)
    if (q < 2.5) {
        double q2 = q * q, s = 0.0, pw = 1.0, fact = 1.0;
        for (int n = 0; n < 28; ++n) {
            double a = (double)(2 * n);
            double moment = 0.5 / (a + 5.0) - 1.0 / (3.0 * (a + 6.0)) - 1.0 / (6.0 * (a + 3.0));
            s += ((n & 1) ? -1.0 : 1.0) * moment * pw / fact;
            pw *= q2;
            fact *= (a + 2.0) * (a + 3.0);
        }
        return 4.0 * kPi * s;
    }
    double c = cos(q), sn = sin(q), q2 = q * q;
    return 4.0 * kPi * (5.0 * q * sn - (q2 - 8.0) * c - 8.0) / (q2 * q2 * q2);
}

struct Quad {
    static constexpr int NP = 20;
    static constexpr double W = 0.5, QMAX = 4096.0;
    double x[NP], w[NP];
    std::vector<double> tailI, tailJ;  // int_{iW}^{QMAX}
    Quad() {
        for (int i = 0; i < NP; ++i) {
            double z = cos(kPi * (i + 0.75) / (NP + 0.5)), dp = 1.0;
            for (int it = 0; it < 200; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= NP; ++k) {
                    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = NP * (p0 - z * p1) / (1.0 - z * z);
                double step = p1 / dp;
                z -= step;
                if (fabs(step) < 1e-17) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
        int n = (int)(QMAX / W);
        tailI.assign(n + 1, 0.0);
        tailJ.assign(n + 1, 0.0);
        for (int i = n - 1; i >= 0; --i) {
            double a, b;
            segment(i * W, (i + 1) * W, a, b);
            tailI[i] = tailI[i + 1] + a;
            tailJ[i] = tailJ[i + 1] + b;
        }
    }
    void segment(double a, double b, double& vi, double& vj) const {
        double m = 0.5 * (a + b), hw = 0.5 * (b - a);
        vi = vj = 0.0;
        for (int i = 0; i < NP; ++i) {
            double q = m + hw * x[i], f = phit(q), f2 = f * f, q3 = q * q * q;
            vi += w[i] * q3 * f2;
            vj += w[i] * q3 * q3 * f2;
        }
        vi *= hw;
        vj *= hw;
    }
    static double asymI(double Q) { return 2.0 * kPi * kPi / (Q * Q * Q * Q); }
    static double asymJ(double Q) {
        double p2 = kPi * kPi;
        return 8.0 * p2 / Q - 4.0 * p2 * sin(2.0 * Q) / (Q * Q) + (24.0 - 36.0 * cos(2.0 * Q)) * p2 / (Q * Q * Q);
    }
    void IJ(double xq, double& I, double& J) const {
        if (xq >= QMAX) {
            I = asymI(xq);
            J = asymJ(xq);
            return;
        }
        int i = (int)floor(xq / W);
        double vi = 0.0, vj = 0.0;
        if ((i + 1) * W > xq) segment(xq, (i + 1) * W, vi, vj);
        I = vi + tailI[i + 1] + asymI(QMAX);
        J = vj + tailJ[i + 1] + asymJ(QMAX);
    }
    double I(double xq) const {
        double a, b;
        IJ(xq, a, b);
        return a;
    }
    // G(x) = int_x^inf t^2 I(t) dt = (J6(x) - x^3 I(x)) / 3
    double G(double xq) const {
        double a, b;
        IJ(xq, a, b);
        return (b - xq * xq * xq * a) / 3.0;
    }
};

const Quad& quad() {
    static Quad q;
    return q;
}

double M3() { return 2.0 * kPi * kPi / 105.0 * (9.0 - 8.0 * log(2.0)); }
double M4() { return 8.0 * kPi * kPi * kPi / 105.0; }
double M6() { return 8.0 * kPi * kPi * kPi / 5.0; }

struct PWTables {
    std::vector<double> cdf, shell;
    double W_cube = 0, W_cont = 0, W_corner = 0, x_s = 0;
};

PWTables build_pw(double L, double lmax, int NL) {
    const Quad& Q = quad();
    PWTables t;
    const int D = 2 * NL + 1;
    const double ks = 2.0 * kPi / L;
    std::vector<double> byl2(3 * NL * NL + 1);
    for (size_t v = 0; v < byl2.size(); ++v) byl2[v] = Q.I(ks * sqrt((double)v) * lmax);
    t.cdf.resize((size_t)D * D * D);
    double run = 0.0, corner = 0.0, edge = (NL + 0.5) * (NL + 0.5);
    size_t i = 0;
    for (int a = -NL; a <= NL; ++a)
        for (int b = -NL; b <= NL; ++b)
            for (int c = -NL; c <= NL; ++c, ++i) {
                int l2 = a * a + b * b + c * c;
                run += byl2[l2];
                t.cdf[i] = run;
                if ((double)l2 > edge) corner += byl2[l2];
            }
    t.W_cube = run;
    t.W_corner = corner;
    t.x_s = ks * (NL + 0.5) * lmax;
    double Lk = L / (2.0 * kPi);
    t.W_cont = Lk * Lk * Lk * 4.0 * kPi / (lmax * lmax * lmax) * Q.G(t.x_s);
    // shell: s = x_s / x at u = i/M where u = 1 - G(x)/G(x_s) (bisection on s)
    const int M = 4096;
    t.shell.assign(M + 1, 0.0);
    t.shell[0] = 1.0;
    double G0 = Q.G(t.x_s);
    for (int k = 1; k < M; ++k) {
        double want = (1.0 - (double)k / M) * G0, lo = 0.0, hi = t.shell[k - 1];
        for (int it = 0; it < 60; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= 0.0 || Q.G(t.x_s / mid) < want) lo = mid; else hi = mid;
        }
        t.shell[k] = 0.5 * (lo + hi);
    }
    return t;
}

// Infinite system (Sec. V "Distributions of wavevectors"): P(k) = N_k k^2 I(k lmax) with
// N_k = 3 lmax^3/M6, so x = k lmax has the tail probability v = G(x)/G(0). Its inverse is tabulated
// as s = x v at t = i/M with v = 1 - t^3 (s is smooth at both ends; s -> 2 pi^2/G(0) as v -> 0),
// each point solved by bisection on G.
PWTables build_inf_table() {
    const Quad& Q = quad();
    PWTables t;
    const int M = 4096;
    const double G0 = Q.G(0.0);
    t.shell.assign(M + 1, 0.0);
    double x = 0.0;
    for (int i = 1; i < M; ++i) {
        const double ti = (double)i / M, v = 1.0 - ti * ti * ti, want = v * G0;
        double lo = x, hi = x + 0.5;
        while (Q.G(hi) > want) hi *= 2.0;
        for (int it = 0; it < 80; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (Q.G(mid) > want) lo = mid; else hi = mid;
        }
        x = 0.5 * (lo + hi);
        t.shell[i] = x * v;
    }
    t.shell[M] = 2.0 * kPi * kPi / G0;
    return t;
}

#define HIPCHK(c, expr)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            (c)->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " #expr; \
            return WMC_EHIP;                                                             \
        }                                                                                \
    } while (0)

struct Layout {
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t off = (total + 255) & ~(size_t)255;
        total = off + bytes;
        return off;
    }
};

// everything the arena holds, computed identically by wmc_arena_bytes and wmc_init
struct Plan {
    int64_t N = 0, total_fine = 0, slots = 0, slot_len = 0, pool_cube = 0, pool_shell = 0, n_chains = 0, bmap = 0, coop_ints = 0, flags = 0;
    int nsys = 0, total_levels = 0;
    size_t off_x, off_xb, off_bond, off_sysid, off_tag, off_fcount, off_fstart, off_fidx, off_fcell, off_drift, off_driftcol,
        off_celldrift, off_comref,
        off_cnt, off_sysacc, off_fblock, off_gbar, off_coop, off_cooptab, off_flags, off_flowctr, off_trace, off_tracen, off_cube, off_shell, off_slotS, off_slotM, off_slotMX, off_pw,
        off_igrid, off_sys, off_lev, off_bmap, off_choff, off_rg2;
    size_t bytes = 0;
};

}  // namespace

static int validate(wmc_ctx* c, const wmc_params* p, int32_t nsys, const int64_t* so, const double* sL,
                    const double* sl, int64_t n_chains, const int64_t* co) {
    auto fail = [&](const char* m) {
        if (c) c->err = m;
        return WMC_EINVAL;
    };
    if (!p || !so || !co) return fail("null argument");
    if (nsys < 1 || nsys > 4096) return fail("n_systems must be in 1..4096");
    if (!(p->lambda_min > 0.0)) return fail("lambda_min must be positive");
    if (!(p->band_ratio > 1.0 && p->band_ratio <= 2.0)) return fail("band_ratio must lie in (1, 2]");
    if (!(p->A0 > 0.0) || !(p->kT > 0.0)) return fail("A0 and kT must be positive");
    if (p->bond_type < 0 || p->bond_type > 2) return fail("bad bond_type");
    if (p->bond_type == WMC_BOND_FENE && !(p->R0 > 0.0)) return fail("FENE needs R0 > 0");
    if (p->bond_type == WMC_BOND_HARMONIC && !(p->r_int_harmonic > 0.0)) return fail("harmonic bonds need r_int_harmonic > 0");
    if (p->wca && !(p->sigma > 0.0)) return fail("WCA needs sigma > 0");
    if (p->retry_cap < 1 || p->retry_cap > 255) return fail("retry_cap must be in 1..255");
    if (p->plane_waves && p->periodic && (p->n_layers < 1 || p->n_layers > 60)) return fail("n_layers must be in 1..60");
    if (p->accept_rule < 0 || p->accept_rule > 1) return fail("bad accept_rule");
    if (p->wavelet_map < 0 || p->wavelet_map > 1) return fail("bad wavelet_map");
    if (p->centring < 0 || p->centring > 1) return fail("bad centring");
    if (p->centring == WMC_CENTRE_UNIFORM && !p->periodic) return fail("uniform centres need a periodic box");
    if (p->mixed_verify < 0 || p->mixed_verify > 1) return fail("mixed_verify must be 0 or 1");
    if (!p->periodic && nsys != 1) return fail("an infinite system runs as a single system");
    if (so[0] != 0) return fail("sys_bead_offset[0] must be 0");
    for (int s = 0; s < nsys; ++s) {
        if (so[s + 1] <= so[s]) return fail("every system needs at least one bead");
        double L = sL ? sL[s] : p->box_L, lm = sl ? sl[s] : p->lambda_max;
        if (!(lm > p->lambda_min)) return fail("lambda_max must exceed lambda_min");
        if (p->periodic && !(L > 0.0)) return fail("periodic box needs box_L > 0");
        if (p->periodic && lm > 0.5 * L) return fail("lambda_max must not exceed L/2");
    }
    if (so[nsys] > 0x3FFFFFFF) return fail("too many beads (at most 2^30 - 1)");
    if (!p->periodic && so[nsys] > 8192) return fail("an infinite system is limited to 8192 beads");
    if (co[0] != 0 || co[n_chains] != so[nsys]) return fail("chain_offset must cover all beads");
    int s = 0;
    for (int64_t ch = 0; ch < n_chains; ++ch) {
        if (co[ch + 1] <= co[ch]) return fail("empty chain");
        while (co[ch] >= so[s + 1]) ++s;
        if (co[ch + 1] > so[s + 1]) return fail("a chain crosses a system boundary");
    }
    return 0;
}

static double r_int_of(const wmc_params* p) {
    double rc = p->wca ? pow(2.0, 1.0 / 6.0) * p->sigma : 0.0;
    if (p->bond_type == WMC_BOND_FENE) return std::max(p->R0, rc);
    if (p->bond_type == WMC_BOND_HARMONIC) return std::max(p->r_int_harmonic, rc);
    return rc;
}

// per-system schedule (levels, neighbour grid, pw tables) and the arena plan
static int plan_systems(wmc_ctx* c, const wmc_params* p, int32_t nsys, const int64_t* so, const double* sL,
                        const double* sl, int64_t n_chains, int64_t trace_cap, Plan& pl,
                        std::vector<SysDesc>* sys_out, std::vector<LevelDesc>* lev_out,
                        std::vector<PWTables>* pw_pool, std::vector<int>* pw_index) {
    pl.nsys = nsys;
    pl.N = so[nsys];
    pl.n_chains = n_chains;
    const double r_int = r_int_of(p);
    const double rc = p->wca ? pow(2.0, 1.0 / 6.0) * p->sigma : 0.0;
    std::vector<SysDesc> sys(nsys);
    std::vector<LevelDesc> lev;
    std::map<double, int> pw_by_ratio;
    int64_t fine = 0, slots = 0, cube_pool = 0, shell_pool = 0, slot_len = 0, flags = 0;
    const double lam_a = 2.0 / kPi * M4() / M3();
    for (int s = 0; s < nsys; ++s) {
        SysDesc& d = sys[s];
        memset(&d, 0, sizeof(d));
        d.b0 = so[s];
        d.b1 = so[s + 1];
        d.N = (int32_t)(d.b1 - d.b0);
        d.L = p->periodic ? (sL ? sL[s] : p->box_L) : 0.0;
        d.invL = p->periodic ? 1.0 / d.L : 0.0;
        d.lmax = sl ? sl[s] : p->lambda_max;
        // plane-wave tables, shared by systems with equal L / lambda_max
        double PF = 0.0;
        if (p->periodic && p->plane_waves) {
            double ratio = d.L / d.lmax;
            int idx;
            auto it = pw_by_ratio.find(ratio);
            if (it == pw_by_ratio.end()) {
                idx = pw_pool ? (int)pw_pool->size() : (int)pw_by_ratio.size();
                if (pw_pool) pw_pool->push_back(build_pw(d.L, d.lmax, p->n_layers));
                pw_by_ratio[ratio] = idx;
            } else {
                idx = it->second;
            }
            int64_t nm = (int64_t)(2 * p->n_layers + 1) * (2 * p->n_layers + 1) * (2 * p->n_layers + 1);
            d.n_modes = (int32_t)nm;
            d.n_shell = 4096;
            d.cube_off = (int64_t)idx * nm;
            d.shell_off = (int64_t)idx * 4097;
            cube_pool = std::max(cube_pool, (int64_t)(idx + 1) * nm);
            shell_pool = std::max(shell_pool, (int64_t)(idx + 1) * 4097);
            if (pw_pool) {
                const PWTables& t = (*pw_pool)[idx];
                double Wtot = t.W_cube + t.W_cont - t.W_corner;
                double Nk = 1.0 / Wtot;
                double R = (d.L / d.lmax) * (d.L / d.lmax) * (d.L / d.lmax) * M6() * Nk / (6.0 * kPi * kPi);
                double rat = d.lmax / p->lambda_min;
                PF = 1.0 / (1.0 + R * (rat * rat * rat - 1.0));
                d.P_cube = t.W_cube / Wtot;
                d.W_cube = t.W_cube;
                d.x_s = t.x_s;
                if (pw_index) pw_index->push_back(idx);
                if (c) c->pw_out.push_back({PF, R, Nk, d.P_cube, M3() * Nk, 0.0});
            }
            d.ks = 2.0 * kPi / d.L;
            d.invks = d.L / (2.0 * kPi);
        } else if (p->plane_waves) {
            // infinite system: one table, P_F = (lambda_min/lambda_max)^3 (Eq. "P(Fourier) infinite")
            if (pw_pool && pw_pool->empty()) pw_pool->push_back(build_inf_table());
            const double q = p->lambda_min / d.lmax;
            PF = q * q * q;
            d.n_shell = 4096;
            d.shell_off = 0;
            shell_pool = std::max<int64_t>(shell_pool, 4097);
            if (c) c->pw_out.push_back({PF, 1.0, 3.0 * d.lmax * d.lmax * d.lmax / M6(), 0.0, 0.0, 0.0});
        } else if (c) {
            c->pw_out.push_back({0.0, 0.0, 0.0, 0.0, 0.0, 0.0});
        }
        d.PF = PF;
        double dt = 6.0 * p->A0 * p->A0 * M4() * lam_a * lam_a / (8.0 * kPi * kPi * kPi * (double)d.N);
        if (!p->plane_waves) {
            double q = p->lambda_min / d.lmax;
            dt *= (1.0 - q) / (1.0 - q * q * q);
        }
        d.dt = dt;
        if (c) c->pw_out.back()[5] = dt;
        // neighbour grid: cells of side >= max(r_cut, 1) + 0.4
        if (p->periodic) {
            double gmin = std::max(rc, 1.0) + 0.4;
            int nf = std::max(1, (int)floor(d.L / gmin));
            nf = std::min(nf, 512);
            d.nf = nf;
            d.g = d.L / nf;
            d.invg = 1.0 / d.g;
            d.fine_off = fine;
            fine += (int64_t)nf * nf * nf;
        }
        // levels
        d.lvl_off = (int32_t)lev.size();
        double norm = 1.0 / (p->lambda_min * p->lambda_min * p->lambda_min) - 1.0 / (d.lmax * d.lmax * d.lmax);
        double lo = p->lambda_min;
        int nl = 0;
        std::vector<double> lout;
        while (nl < WMC_MAX_LEVELS) {
            double hi = lo * p->band_ratio;
            bool last = false;
            if (hi > d.lmax || d.lmax - hi < 1e-9 * d.lmax) {
                hi = d.lmax;
                last = true;
            }
            LevelDesc L;
            memset(&L, 0, sizeof(L));
            L.lo = lo;
            L.hi = hi;
            L.p = (1.0 / (lo * lo * lo) - 1.0 / (hi * hi * hi)) / norm;
            L.T = (double)d.N * (1.0 - PF) * L.p;
            L.r_int = r_int;
            int64_t cells_per_colour;
            if (p->periodic) {
                int n = (int)floor(d.L / ((2.0 * hi + r_int) * (1.0 + 1e-9)));
                if (n % 2) n -= 1;
                if (n < 2) n = 1;
                L.n = n;
                L.h = d.L / n;
                cells_per_colour = n >= 2 ? (int64_t)(n / 2) * (n / 2) * (n / 2) : 1;
                if ((int64_t)n * n * n > 0xFFFFFF) {
                    if (c) c->err = "too many cells in one level";
                    return WMC_EINVAL;
                }
            } else {
                L.n = 0;
                L.h = (2.0 * hi + r_int) * (1.0 + 1e-9);
                cells_per_colour = 0;
            }
            L.invh = 1.0 / L.h;
            L.half = 0.5 * L.h;
            // kernel variant from the expected reach-list size
            double region = p->periodic ? pow(L.h + 2.0 * hi, 3.0) : 0.0;
            double expect = p->periodic ? std::min((double)d.N, (double)d.N / (d.L * d.L * d.L) * region) : (double)d.N;
            if (p->periodic && L.n == 1) {
                L.identity = 1;
                L.use_global = 1;
                L.variant = V1024;
            } else if (p->periodic && (L.n == 2 || 2.0 * expect > 8192.0)) {
                L.use_global = 1;
                L.variant = V1024;
            } else if (!p->periodic) {
                L.variant = d.N <= 512 ? V64 : (d.N <= 4096 ? V256 : V1024);
            } else if (std::min((double)d.N, 4.0 * expect) <= 512.0) {
                L.variant = V64;
            } else if (std::min((double)d.N, 2.5 * expect) <= 4096.0) {
                L.variant = V256;
            } else {
                L.variant = V1024;
            }
            if (L.use_global) {
                L.slot_base = slots;
                slots += cells_per_colour;
                slot_len = std::max(slot_len, (int64_t)d.N);
            }
            L.flag_base = flags;
            if (p->periodic) flags += (int64_t)std::max(L.n, 1) * std::max(L.n, 1) * std::max(L.n, 1);
            lev.push_back(L);
            lout.insert(lout.end(), {L.lo, L.hi, L.p, L.T, L.h, (double)L.n});
            ++nl;
            if (last) break;
            lo = hi;
        }
        if (nl == WMC_MAX_LEVELS && lev.back().hi < d.lmax) {
            if (c) c->err = "too many levels: raise band_ratio";
            return WMC_EINVAL;
        }
        d.n_levels = nl;
        if (c) c->level_out.push_back(lout);
    }
    pl.total_fine = fine;
    pl.slots = slots;
    pl.slot_len = slot_len;
    pl.flags = flags;
    pl.pool_cube = cube_pool;
    pl.pool_shell = shell_pool;
    pl.total_levels = (int)lev.size();
    // block maps: one entry (system, local cell) per workgroup of each (level, colour) launch;
    // phases holding global-list cells may run them as cooperative groups
    int64_t bm = 0, gphases = 0;
    for (int l = 0; l < WMC_MAX_LEVELS; ++l)
        for (int col = 0; col < 8; ++col) {
            bool glob = false;
            for (int s = 0; s < nsys; ++s)
                if (p->periodic && l < sys[s].n_levels) {
                    const LevelDesc& L = lev[sys[s].lvl_off + l];
                    int64_t ncol = L.n >= 2 ? (int64_t)(L.n / 2) * (L.n / 2) * (L.n / 2) : (col == 0 ? 1 : 0);
                    bm += ncol;
                    if (ncol > 0 && L.use_global) glob = true;
                }
            gphases += glob ? 1 : 0;
        }
    pl.bmap = bm;
    pl.coop_ints = 4 * (bm + nsys) + (int64_t)COOP_SLOTS * (gphases + 1);
    // arena layout
    Layout lay;
    const int64_t N = pl.N;
    pl.off_x = lay.add(3 * N * 8);
    pl.off_xb = lay.add(3 * N * 8);
    pl.off_bond = lay.add(N);
    pl.off_sysid = lay.add(N * 4);
    pl.off_tag = lay.add(N * 4);
    pl.off_fcount = lay.add((fine + 1) * 4);
    pl.off_fstart = lay.add((fine + 1) * 4);
    pl.off_fidx = lay.add(N * 4);
    pl.off_fcell = lay.add(N * 4);
    pl.off_fblock = lay.add((fine / 4096 + 2) * 4);
    pl.off_drift = lay.add(nsys * 8);
    pl.off_driftcol = lay.add(8 * nsys * 8);
    pl.off_cnt = lay.add(CNT_TOTAL * 8);
    pl.off_sysacc = lay.add(nsys * 8);
    pl.off_trace = lay.add(std::max<int64_t>(trace_cap, 0) * sizeof(wmc_trace_rec));
    pl.off_tracen = lay.add(8);
    pl.off_cube = lay.add(cube_pool * 8);
    pl.off_shell = lay.add(shell_pool * 8);
    pl.off_slotS = lay.add(slots * slot_len * 4);
    pl.off_slotM = lay.add(slots * slot_len * 4);
    pl.off_slotMX = lay.add(slots * slot_len * 3 * 8);
    pl.off_pw = lay.add(p->plane_waves ? 3 * N * 8 : 8);
    pl.off_igrid = lay.add(16 * 8);
    pl.off_gbar = lay.add(2 * (1 + COOP_SLOTS) * 4);
    pl.off_coop = lay.add(COOP_SLOTS * 4 + 5 * COOP_SLOTS * 8);
    pl.off_cooptab = lay.add(pl.coop_ints * 4);
    pl.off_flags = lay.add(std::max<int64_t>(pl.flags, 1) * 4);
    pl.off_celldrift = lay.add(std::max<int64_t>(pl.flags, 1) * 8);
    pl.off_flowctr = lay.add(WMC_MAX_LEVELS * 8);
    pl.off_sys = lay.add(nsys * sizeof(SysDesc));
    pl.off_lev = lay.add(lev.size() * sizeof(LevelDesc));
    pl.off_bmap = lay.add(std::max<int64_t>(bm, 1) * 3 * 2 * 4);
    pl.off_choff = lay.add((n_chains + 1) * 8);
    pl.off_rg2 = lay.add(std::max<int64_t>(n_chains, 1) * 3 * 8);
    pl.off_comref = lay.add(std::max<int64_t>(n_chains, 1) * 3 * 8);
    pl.bytes = lay.total + 256;
    if (sys_out) *sys_out = sys;
    if (lev_out) *lev_out = lev;
    return 0;
}

extern "C" int wmc_arena_bytes(const wmc_params* p, int32_t n_systems, const int64_t* so, const double* sL,
                               const double* sl, int64_t n_chains, const int64_t* co, int64_t trace_capacity,
                               size_t* out_bytes) {
    int rc = validate(nullptr, p, n_systems, so, sL, sl, n_chains, co);
    if (rc) return rc;
    Plan pl;
    rc = plan_systems(nullptr, p, n_systems, so, sL, sl, n_chains, trace_capacity, pl, nullptr, nullptr, nullptr,
                      nullptr);
    if (rc) return rc;
    *out_bytes = pl.bytes;
    return 0;
}

extern "C" int wmc_launch_plan(const wmc_params* p, int32_t nsys, const int64_t* so, const double* sL,
                               const double* sl, int64_t n_chains, const int64_t* co, const double* pos,
                               int32_t cell_blocks, int32_t pw_blocks, int32_t cell_launch_max,
                               int32_t pw_launch_max, char* report, size_t report_bytes);

// Group sizes of the cooperative launches, from each system's bead count: a cell group gets one
// workgroup per CELL_GROUP_BEADS beads (at most CELL_GROUP_MAX, and enough that a workgroup's
// slice of the reach list fits its LDS list), a plane-wave group one per PW_GROUP_BEADS (at most
// PW_GROUP_MAX). Sizes shrink proportionally when the sum exceeds what can be co-resident; a
// launch is planned only if it fits and some group has more than one workgroup.
static bool size_groups(std::vector<int>& G, const std::vector<int64_t>& Ns, int per, int gmax, int cap,
                        int64_t slice_cap) {
    int64_t T = 0;
    int top = 0;
    for (size_t i = 0; i < Ns.size(); ++i) {
        G[i] = (int)std::min<int64_t>(gmax, std::max<int64_t>(1, (Ns[i] + per - 1) / per));
        T += G[i];
    }
    if (T > cap) {
        int64_t T2 = 0;
        for (size_t i = 0; i < Ns.size(); ++i) {
            G[i] = (int)std::max<int64_t>(1, (int64_t)G[i] * cap / T);
            T2 += G[i];
        }
        T = T2;
    }
    for (size_t i = 0; i < Ns.size(); ++i) {
        if (slice_cap > 0 && (Ns[i] + G[i] - 1) / G[i] > slice_cap) return false;
        top = std::max(top, G[i]);
    }
    return cap > 0 && T <= cap && top > 1;
}

// Launch slots of a group launch. The dispatcher deals a cooperative launch's workgroups to the
// 8 XCDs in turn, so workgroups whose launch indices agree mod 8 share an XCD and its L2. Each
// group takes the indices of one residue class (largest groups first, least-loaded class), so
// its barriers write back and invalidate one L2 and no other group's lines. Entry w of the map
// is (group | rank << 16), or -1 for a slot no group uses. When the padded launch would exceed
// cap, groups take consecutive slots instead. Returns the launch size.
static int map_groups(const std::vector<int>& G, int cap, std::vector<int32_t>& map) {
    const int ng = (int)G.size();
    std::vector<int> order(ng), cls(ng);
    for (int g = 0; g < ng; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return G[a] > G[b]; });
    int load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int g : order) {
        int r = 0;
        for (int q = 1; q < 8; ++q)
            if (load[q] < load[r]) r = q;
        cls[g] = r;
        load[r] += G[g];
    }
    int top = 0;
    for (int q = 0; q < 8; ++q) top = std::max(top, load[q]);
    map.clear();
    if (8 * top <= cap) {
        map.assign((size_t)8 * top, -1);
        int next[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int g = 0; g < ng; ++g)
            for (int k = 0; k < G[g]; ++k) map[(size_t)cls[g] + 8 * (size_t)next[cls[g]]++] = g | (k << 16);
        while (!map.empty() && map.back() < 0) map.pop_back();
    } else {
        for (int g = 0; g < ng; ++g)
            for (int k = 0; k < G[g]; ++k) map.push_back(g | (k << 16));
    }
    return (int)map.size();
}

static void build_groups(wmc_ctx* c, int64_t capacity_ints, int ccap, int pcap) {
    c->coop_host.clear();
    auto& H = c->coop_host;
    std::vector<int32_t> tiles;
    for (int l = 0; l < WMC_MAX_LEVELS; ++l)
        for (int col = 0; col < 8; ++col) {
            c->cwg_n[l][col] = 0;
            c->tile_n[l][col] = 0;
            std::vector<std::pair<int32_t, int32_t>> glob;
            tiles.clear();
            for (int32_t e = 0; e < c->bmap_n[l][col]; ++e) {
                const int32_t s = c->bmap_host[2 * (c->bmap_off[l][col] + e)];
                const int32_t k = c->bmap_host[2 * (c->bmap_off[l][col] + e) + 1];
                if (c->lev[c->sys[s].lvl_off + l].use_global) {
                    glob.push_back({s, k});
                } else {
                    tiles.push_back(s);
                    tiles.push_back(k);
                }
            }
            c->tile_off[l][col] = (int64_t)c->bmap_host.size() / 2;
            c->tile_n[l][col] = (int32_t)(tiles.size() / 2);
            c->bmap_host.insert(c->bmap_host.end(), tiles.begin(), tiles.end());
            c->glob_off[l][col] = (int64_t)c->bmap_host.size() / 2;
            c->glob_n[l][col] = (int32_t)glob.size();
            for (auto& e : glob) c->bmap_host.insert(c->bmap_host.end(), {e.first, e.second});
            if (glob.empty()) continue;
            std::vector<int64_t> Ns(glob.size());
            for (size_t i = 0; i < glob.size(); ++i) Ns[i] = c->sys[glob[i].first].N;
            std::vector<int> G(glob.size());
            if (!size_groups(G, Ns, CELL_GROUP_BEADS, CELL_GROUP_MAX, ccap, COOP_LIST_CAP)) continue;
            int first = 0;
            c->cgrp_off[l][col] = (int64_t)H.size();
            for (size_t i = 0; i < glob.size(); ++i) {
                H.insert(H.end(), {glob[i].first, glob[i].second, first, G[i]});
                first += G[i];
            }
            std::vector<int32_t> wmap;
            const int nwg = map_groups(G, ccap, wmap);
            c->cwg_off[l][col] = (int64_t)H.size();
            H.insert(H.end(), wmap.begin(), wmap.end());
            c->cwg_n[l][col] = nwg;
        }
    // a level's colours share one launch when each colour with global-list cells has a group
    // launch over the same groups (system, first workgroup, size) as the first such colour
    for (int l = 0; l < WMC_MAX_LEVELS; ++l) {
        c->cmerge[l] = false;
        int c0 = -1, ncol = 0;
        bool ok = true;
        for (int col = 0; col < 8 && ok; ++col) {
            if (c->glob_n[l][col] <= 0) continue;
            ++ncol;
            if (c->cwg_n[l][col] <= 0) {
                ok = false;
            } else if (c0 < 0) {
                c0 = col;
            } else {
                ok = c->glob_n[l][col] == c->glob_n[l][c0] && c->cwg_n[l][col] == c->cwg_n[l][c0];
                for (int32_t i = 0; ok && i < c->glob_n[l][col]; ++i) {
                    const int32_t* a = &H[c->cgrp_off[l][c0] + 4 * i];
                    const int32_t* b = &H[c->cgrp_off[l][col] + 4 * i];
                    ok = a[0] == b[0] && a[2] == b[2] && a[3] == b[3];
                }
            }
        }
        c->cmerge[l] = ok && ncol > 1;
    }
    c->pwg_n = 0;
    if (c->P.periodic && c->P.plane_waves) {
        std::vector<int64_t> Ns(c->nsys);
        for (int s = 0; s < c->nsys; ++s) Ns[s] = c->sys[s].N;
        std::vector<int> G(c->nsys);
        if (size_groups(G, Ns, PW_GROUP_BEADS, PW_GROUP_MAX, pcap, 0)) {
            int first = 0;
            c->pgrp_off = (int64_t)H.size();
            for (int s = 0; s < c->nsys; ++s) {
                H.insert(H.end(), {s, 0, first, G[s]});
                first += G[s];
            }
            std::vector<int32_t> wmap;
            const int nwg = map_groups(G, pcap, wmap);
            c->pwg_off = (int64_t)H.size();
            H.insert(H.end(), wmap.begin(), wmap.end());
            c->pwg_n = nwg;
        }
    }
    if ((int64_t)H.size() > capacity_ints) {  // cannot happen: the layout bounds the table
        H.clear();
        for (int l = 0; l < WMC_MAX_LEVELS; ++l) {
            for (int col = 0; col < 8; ++col) c->cwg_n[l][col] = 0;
            c->cmerge[l] = false;
        }
        c->pwg_n = 0;
    }
}

// Launch plan of a context (host only): per periodic LDS-tile level the kernel variant raised until
// the densest windows fit its lists, the block maps of every (level, colour), and the cooperative
// groups of the global-list cells and of the plane waves for launches of at most ccap / pcap
// co-resident workgroups.
static void plan_launches(wmc_ctx* c, const wmc_params* p, const double* pos, const Plan& pl, int ccap, int pcap) {
    const int nsys = c->nsys;
    // capacities from the actual clustering: a dilute chain puts most of its beads into one
    // cell's reach, far above the uniform-density estimate the plan used. A tile that does not
    // fit LDS falls back to the global path, whose reach and member lists live in LDS too and
    // must not overflow. Per periodic LDS-tile level the beads are binned at a quarter of the
    // cell side; the largest periodic box window as wide as a cell's reach (cell + 2 lambda_hi)
    // and as wide as a wavelet (2 lambda_hi) bound those lists for any shifted cell and any
    // centre, and the variant is raised until both fit with a 12.5% margin.
    if (p->periodic) {
        const int caps[3] = {1024, 4096, 8192}, capm[3] = {256, 1024, 4096};  // global-path lists per variant
        for (int s = 0; s < nsys; ++s) {
            const SysDesc& d = c->sys[s];
            for (int l = 0; l < d.n_levels; ++l) {
                LevelDesc& L = c->lev[d.lvl_off + l];
                if (L.use_global || L.n < 4) continue;
                const int m = 4 * L.n;
                const double inv_bin = 4.0 * L.invh;
                std::vector<int32_t> cnt((size_t)m * m * m, 0);
                for (int64_t i = d.b0; i < d.b1; ++i) {
                    int q[3];
                    for (int ax = 0; ax < 3; ++ax) {
                        double v = pos[3 * i + ax];
                        v -= d.L * floor(v * d.invL);
                        q[ax] = std::min(m - 1, std::max(0, (int)(v * inv_bin)));
                    }
                    ++cnt[q[0] + (size_t)m * (q[1] + (size_t)m * q[2])];
                }
                // largest count over periodic windows of w bins per axis (separable sliding sums)
                auto window_max = [&](int w) {
                    w = std::max(1, std::min(m, w));
                    std::vector<int32_t> a = cnt, b((size_t)m * m * m);
                    for (int ax = 0; ax < 3; ++ax) {
                        const size_t stride = ax == 0 ? 1 : (ax == 1 ? (size_t)m : (size_t)m * m);
                        for (int u = 0; u < m; ++u)
                            for (int v = 0; v < m; ++v) {
                                const size_t base = ax == 0 ? (size_t)m * (u + (size_t)m * v)
                                                  : (ax == 1 ? (size_t)u + (size_t)m * m * v : (size_t)u + (size_t)m * v);
                                int64_t run = 0;
                                for (int k = 0; k < w; ++k) run += a[base + stride * (size_t)(k % m)];
                                for (int k = 0; k < m; ++k) {
                                    b[base + stride * (size_t)k] = (int32_t)run;
                                    run += a[base + stride * (size_t)((k + w) % m)] - a[base + stride * (size_t)k];
                                }
                            }
                        std::swap(a, b);
                    }
                    int64_t worst = 0;
                    for (int32_t v : a) worst = std::max<int64_t>(worst, v);
                    return worst + worst / 8;
                };
                const int64_t need_s = window_max((int)ceil((L.h + 2.0 * L.hi) * inv_bin) + 1);
                const int64_t need_m = window_max((int)ceil(2.0 * L.hi * inv_bin) + 1);
                while (L.variant < V1024 && (need_s > caps[L.variant] || need_m > capm[L.variant])) L.variant += 1;
            }
        }
    }
    // block maps
    c->max_levels = 0;
    for (auto& s : c->sys) c->max_levels = std::max(c->max_levels, (int)s.n_levels);
    c->bmap_host.clear();
    for (int l = 0; l < WMC_MAX_LEVELS; ++l) {
        c->phase_variant[l] = V64;
        for (int col = 0; col < 8; ++col) {
            c->bmap_off[l][col] = (int64_t)c->bmap_host.size() / 2;
            int32_t cnt = 0;
            for (int s = 0; s < nsys && p->periodic; ++s) {
                if (l >= c->sys[s].n_levels) continue;
                const LevelDesc& L = c->lev[c->sys[s].lvl_off + l];
                c->phase_variant[l] = std::max(c->phase_variant[l], L.variant);
                int64_t ncol = L.n >= 2 ? (int64_t)(L.n / 2) * (L.n / 2) * (L.n / 2) : (col == 0 ? 1 : 0);
                for (int64_t k = 0; k < ncol; ++k) {
                    c->bmap_host.push_back(s);
                    c->bmap_host.push_back((int32_t)k);
                    ++cnt;
                }
            }
            c->bmap_n[l][col] = cnt;
        }
        if (!p->periodic && l < c->max_levels) c->phase_variant[l] = c->lev[l].variant;
    }
    build_groups(c, pl.coop_ints, ccap, pcap);
}

// Every index the kernels derive from a launch plan, checked on the host: block-map entries, the
// cooperative group tables (workgroup ranges, per-workgroup result slots, barrier words, list
// slices), the workgroup -> (group, rank) maps, global list slots and cell flags. Returns an empty
// string when all hold, else the first violation.
static std::string check_plan(const wmc_ctx* c, const Plan& pl, int ccap, int pcap) {
    char buf[256];
    auto bad = [&](const char* what, long a, long b, long d) {
        snprintf(buf, sizeof(buf), "%s (%ld, %ld, %ld)", what, a, b, d);
        return std::string(buf);
    };
    const auto& H = c->coop_host;
    if ((int64_t)H.size() > pl.coop_ints) return bad("group table exceeds its arena", (long)H.size(), (long)pl.coop_ints, 0);
    if ((int64_t)c->bmap_host.size() > 3 * 2 * std::max<int64_t>(pl.bmap, 1)) return bad("block map exceeds its arena", (long)c->bmap_host.size(), (long)pl.bmap, 0);
    auto ncol_of = [&](const LevelDesc& L, int col) -> int64_t {
        return L.n >= 2 ? (int64_t)(L.n / 2) * (L.n / 2) * (L.n / 2) : (col == 0 ? 1 : 0);
    };
    // group table at goff with ng groups and the map at woff with nwg entries
    auto check_groups = [&](int64_t goff, int ng, int64_t woff, int nwg, int gmax, int cap, int64_t slice_cap,
                            const char* kind) -> std::string {
        if (nwg > cap) return bad(kind, nwg, cap, -1);
        if (ng > COOP_SLOTS - 1) return bad("more groups than barrier words", ng, COOP_SLOTS - 1, 0);
        int first = 0;
        std::vector<int> size(ng);
        for (int g = 0; g < ng; ++g) {
            const int32_t* e = &H[goff + 4 * g];
            if (e[0] < 0 || e[0] >= c->nsys) return bad("group system out of range", g, e[0], c->nsys);
            if (e[2] != first) return bad("group slots not consecutive", g, e[2], first);
            if (e[3] < 1 || e[3] > gmax) return bad("group size out of range", g, e[3], gmax);
            if (slice_cap > 0 && (c->sys[e[0]].N + e[3] - 1) / e[3] > slice_cap)
                return bad("list slice exceeds the workgroup's list", g, c->sys[e[0]].N, e[3]);
            first += e[3];
            size[g] = e[3];
        }
        if (first > cap || first > COOP_SLOTS) return bad("group slots exceed the launch", first, cap, COOP_SLOTS);
        std::vector<std::vector<int>> seen(ng);
        for (int g = 0; g < ng; ++g) seen[g].assign(size[g], 0);
        for (int w = 0; w < nwg; ++w) {
            const int32_t e = H[woff + w];
            if (e < 0) continue;
            const int g = e & 0xFFFF, r = e >> 16;
            if (g >= ng || r >= size[g]) return bad("map entry names no group rank", w, g, r);
            if (seen[g][r]++) return bad("group rank mapped twice", w, g, r);
        }
        for (int g = 0; g < ng; ++g)
            for (int r = 0; r < size[g]; ++r)
                if (!seen[g][r]) return bad("group rank without a workgroup", g, r, nwg);
        return std::string();
    };
    for (int l = 0; l < WMC_MAX_LEVELS; ++l) {
        for (int col = 0; col < 8; ++col) {
            for (int kind = 0; kind < 2; ++kind) {
                const int64_t off = kind ? c->glob_off[l][col] : c->tile_off[l][col];
                const int32_t n = kind ? c->glob_n[l][col] : c->tile_n[l][col];
                for (int32_t e = 0; e < n; ++e) {
                    const int32_t sy = c->bmap_host[2 * (off + e)], loc = c->bmap_host[2 * (off + e) + 1];
                    if (sy < 0 || sy >= c->nsys || l >= c->sys[sy].n_levels) return bad("block map system", l, col, sy);
                    const LevelDesc& L = c->lev[c->sys[sy].lvl_off + l];
                    if (loc < 0 || loc >= ncol_of(L, col)) return bad("block map cell", l, col, loc);
                    if (kind == 0 && (L.use_global || L.n < 4)) return bad("tile cell on a level without tiles", l, sy, L.n);
                    if (kind == 1 && !L.use_global) return bad("global-list cell on a tile level", l, sy, L.n);
                    if (kind == 1 && (L.slot_base + loc >= pl.slots || pl.slot_len < c->sys[sy].N))
                        return bad("global list slot out of range", l, sy, loc);
                    if (L.variant > c->phase_variant[l]) return bad("level variant above its launch's", l, sy, L.variant);
                }
            }
            if (c->cwg_n[l][col] > 0) {
                const std::string e = check_groups(c->cgrp_off[l][col], c->glob_n[l][col], c->cwg_off[l][col],
                                                   c->cwg_n[l][col], CELL_GROUP_MAX, ccap, COOP_LIST_CAP, "cell launch above cap");
                if (!e.empty()) return e + " level " + std::to_string(l) + " colour " + std::to_string(col);
                for (int32_t g = 0; g < c->glob_n[l][col]; ++g) {
                    const int32_t* ge = &H[c->cgrp_off[l][col] + 4 * g];
                    if (ge[0] != c->bmap_host[2 * (c->glob_off[l][col] + g)] || ge[1] != c->bmap_host[2 * (c->glob_off[l][col] + g) + 1])
                        return bad("group does not match its block-map cell", l, col, g);
                }
            }
        }
        if (c->cmerge[l]) {
            int c0 = -1;
            for (int col = 0; col < 8; ++col) {
                if (c->glob_n[l][col] <= 0) continue;
                if (c->cwg_n[l][col] <= 0) return bad("merged colour without a group launch", l, col, 0);
                if (c0 < 0) { c0 = col; continue; }
                if (c->glob_n[l][col] != c->glob_n[l][c0] || c->cwg_n[l][col] != c->cwg_n[l][c0]) return bad("merged colours differ", l, col, c0);
                for (int32_t g = 0; g < c->glob_n[l][col]; ++g)
                    for (int q : {0, 2, 3})
                        if (H[c->cgrp_off[l][col] + 4 * g + q] != H[c->cgrp_off[l][c0] + 4 * g + q]) return bad("merged group differs", l, col, g);
            }
        }
    }
    if (c->pwg_n > 0) {
        const std::string e = check_groups(c->pgrp_off, c->nsys, c->pwg_off, c->pwg_n, PW_GROUP_MAX, pcap, 0, "plane-wave launch above cap");
        if (!e.empty()) return e + " (plane waves)";
    }
    for (int s = 0; s < c->nsys; ++s)
        for (int l = 0; l < c->sys[s].n_levels; ++l) {
            const LevelDesc& L = c->lev[c->sys[s].lvl_off + l];
            const int64_t n = std::max(L.n, 1);
            if (c->P.periodic && L.flag_base + n * n * n > std::max<int64_t>(pl.flags, 1)) return bad("cell flags out of range", s, l, L.flag_base);
        }
    return std::string();
}

extern "C" int wmc_launch_plan(const wmc_params* p, int32_t nsys, const int64_t* so, const double* sL,
                               const double* sl, int64_t n_chains, const int64_t* co, const double* pos,
                               int32_t cell_blocks, int32_t pw_blocks, int32_t cell_launch_max,
                               int32_t pw_launch_max, char* report, size_t report_bytes) {
    wmc_ctx c;
    auto put = [&](const std::string& m) {
        if (report && report_bytes) {
            strncpy(report, m.c_str(), report_bytes - 1);
            report[report_bytes - 1] = 0;
        }
    };
    int rc = validate(&c, p, nsys, so, sL, sl, n_chains, co);
    if (rc) {
        put(c.err);
        return rc;
    }
    if (!pos || cell_blocks < 0 || pw_blocks < 0) {
        put("null positions or negative limits");
        return WMC_EINVAL;
    }
    c.p = *p;
    c.nsys = nsys;
    c.N = so[nsys];
    c.n_chains = n_chains;
    memset(&c.P, 0, sizeof(c.P));
    c.P.periodic = p->periodic;
    c.P.plane_waves = p->plane_waves;
    Plan pl;
    std::vector<PWTables> pool;
    std::vector<int> pidx;
    rc = plan_systems(&c, p, nsys, so, sL, sl, n_chains, 0, pl, &c.sys, &c.lev, &pool, &pidx);
    if (rc) {
        put(c.err);
        return rc;
    }
    const int ccap = p->periodic ? std::min(cell_blocks, cell_launch_max) : 0;
    const int pcap = std::min(pw_blocks, pw_launch_max);
    plan_launches(&c, p, pos, pl, ccap, pcap);
    const std::string err = check_plan(&c, pl, ccap, pcap);
    int groups = 0, cell_launches = 0, widest = 0;
    for (int l = 0; l < WMC_MAX_LEVELS; ++l)
        for (int col = 0; col < 8; ++col)
            if (c.cwg_n[l][col] > 0) {
                ++cell_launches;
                groups += c.glob_n[l][col];
                widest = std::max(widest, (int)c.cwg_n[l][col]);
            }
    char buf[512];
    snprintf(buf, sizeof(buf),
             "%s; systems %d beads %lld arena %zu bytes; cell-group launches %d (groups %d, widest %d workgroups); "
             "plane-wave group launch %d workgroups",
             err.empty() ? "ok" : err.c_str(), nsys, (long long)c.N, pl.bytes, cell_launches, groups, widest, c.pwg_n);
    put(buf);
    return err.empty() ? 0 : WMC_EINVAL;
}

extern "C" int wmc_init(wmc_ctx** out, const wmc_params* p, int32_t nsys, const int64_t* so, const double* sL,
                        const double* sl, int64_t n_chains, const int64_t* co, const double* pos, int64_t trace_cap,
                        void* arena, size_t arena_bytes, void* stream) {
    if (!out) return WMC_EINVAL;
    wmc_ctx* c = new wmc_ctx();
    *out = c;
    int rc = validate(c, p, nsys, so, sL, sl, n_chains, co);
    if (rc) return rc;
    if (!pos) {
        c->err = "null positions";
        return WMC_EINVAL;
    }
    c->p = *p;
    c->nsys = nsys;
    c->N = so[nsys];
    c->n_chains = n_chains;
    c->sweep = 0;
    Plan pl;
    std::vector<PWTables> pool;
    std::vector<int> pidx;
    rc = plan_systems(c, p, nsys, so, sL, sl, n_chains, trace_cap, pl, &c->sys, &c->lev, &pool, &pidx);
    if (rc) return rc;
    const int64_t N = c->N;
    // host-side checks of the initial state (before any device work): finite energy needs every
    // FENE bond shorter than R0 (Eq. "FENE potential") and, with WCA, no two beads of a system at the
    // same point (Eq. "WCA potential" diverges at r = 0)
    if (p->wca) {
        for (int s = 0; s < nsys; ++s) {
            std::vector<std::array<double, 3>> w((size_t)(so[s + 1] - so[s]));
            for (int64_t i = so[s]; i < so[s + 1]; ++i)
                for (int a = 0; a < 3; ++a) {
                    double v = pos[3 * i + a];
                    if (p->periodic) v -= c->sys[s].L * floor(v * c->sys[s].invL);
                    w[(size_t)(i - so[s])][a] = v;
                }
            std::sort(w.begin(), w.end());
            if (std::adjacent_find(w.begin(), w.end()) != w.end()) {
                c->err = "two beads of one system at the same point (infinite WCA energy)";
                return WMC_ESTATE;
            }
        }
    }
    std::vector<uint8_t> bond(N, 0);
    for (int64_t ch = 0; ch < n_chains; ++ch)
        for (int64_t i = co[ch]; i + 1 < co[ch + 1]; ++i) bond[i] = 1;
    for (int s = 0; s < nsys; ++s)
        for (int64_t i = so[s]; i + 1 < so[s + 1]; ++i) {
            if (!bond[i] || p->bond_type != WMC_BOND_FENE) continue;
            double d[3];
            for (int a = 0; a < 3; ++a) {
                d[a] = pos[3 * (i + 1) + a] - pos[3 * i + a];
                if (p->periodic) d[a] -= c->sys[s].L * rint(d[a] * c->sys[s].invL);
            }
            if ((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2] >= p->R0 * p->R0) {
                c->err = "initial FENE bond overstretched";
                return WMC_ESTATE;
            }
        }
    if (!arena || arena_bytes < pl.bytes) {
        c->err = "device arena missing or smaller than wmc_arena_bytes";
        return WMC_EARENA;
    }
    char* base = (char*)(((uintptr_t)arena + 255) & ~(uintptr_t)255);
    c->arena = base;
    c->arena_bytes = arena_bytes;
    c->arena_used = pl.bytes - 256;
    hipStream_t st = (hipStream_t)stream;
    // device parameters
    DevParams& P = c->P;
    memset(&P, 0, sizeof(P));
    P.periodic = p->periodic;
    P.plane_waves = p->plane_waves;
    P.wavelets = p->wavelets;
    P.accept_rule = p->accept_rule;
    P.mixed_verify = p->mixed_verify;
    P.wavelet_map = p->wavelet_map;
    P.centring = p->centring;
    P.precision = p->precision;
    P.bond_type = p->bond_type;
    P.wca = p->wca;
    P.retry_cap = p->retry_cap;
    P.n_layers = p->n_layers;
    P.A0 = p->A0;
    P.kT = p->kT;
    P.k_bond = p->k_bond;
    P.R0 = p->R0;
    P.R02 = p->R0 * p->R0;
    P.sigma2 = p->sigma * p->sigma;
    P.eps = p->eps;
    P.rc2 = pow(2.0, 1.0 / 3.0) * p->sigma * p->sigma;
    P.rc = p->wca ? pow(2.0, 1.0 / 6.0) * p->sigma : 0.0;
    P.r_int = r_int_of(p);
    P.seed_lo = (uint32_t)p->seed;
    P.seed_hi = (uint32_t)(p->seed >> 32);
    P.nsys = nsys;
    // pointers
    DevPtrs& D = c->D;
    memset(&D, 0, sizeof(D));
    D.x = (double*)(base + pl.off_x);
    D.y = D.x + N;
    D.z = D.x + 2 * N;
    D.xb = (double*)(base + pl.off_xb);
    D.yb = D.xb + N;
    D.zb = D.xb + 2 * N;
    D.bond_next = (uint8_t*)(base + pl.off_bond);
    D.sys_id = (int32_t*)(base + pl.off_sysid);
    D.tag = (int32_t*)(base + pl.off_tag);
    D.fcount = (int32_t*)(base + pl.off_fcount);
    D.fstart = (int32_t*)(base + pl.off_fstart);
    D.fidx = (int32_t*)(base + pl.off_fidx);
    D.fcell = (int32_t*)(base + pl.off_fcell);
    D.fblock = (int32_t*)(base + pl.off_fblock);
    D.drift = (unsigned long long*)(base + pl.off_drift);
    D.drift_col = (unsigned long long*)(base + pl.off_driftcol);
    D.cell_drift = (double*)(base + pl.off_celldrift);
    D.com_ref = (double*)(base + pl.off_comref);
    D.cnt = (unsigned long long*)(base + pl.off_cnt);
    D.sys_acc = (unsigned long long*)(base + pl.off_sysacc);
    D.trace = trace_cap > 0 ? (wmc_trace_rec*)(base + pl.off_trace) : nullptr;
    D.trace_n = (unsigned long long*)(base + pl.off_tracen);
    D.trace_cap = trace_cap;
    D.cube_cdf = (const double*)(base + pl.off_cube);
    D.shell_s = (const double*)(base + pl.off_shell);
    D.slot_S = (int32_t*)(base + pl.off_slotS);
    D.slot_M = (int32_t*)(base + pl.off_slotM);
    D.slot_MX = (double*)(base + pl.off_slotMX);
    D.slot_len = pl.slot_len;
    D.pw_new = (double*)(base + pl.off_pw);
    D.igrid = (double*)(base + pl.off_igrid);
    D.gbar = (unsigned*)(base + pl.off_gbar);
    D.coop_i = (int32_t*)(base + pl.off_coop);
    D.coop_d = (double*)(base + pl.off_coop + COOP_SLOTS * 4);
    c->coop_dev = (int32_t*)(base + pl.off_cooptab);
    D.cell_done = (int32_t*)(base + pl.off_flags);
    D.flow_ctr = (unsigned long long*)(base + pl.off_flowctr);
    D.sys = (const SysDesc*)(base + pl.off_sys);
    D.lev = (const LevelDesc*)(base + pl.off_lev);
    D.total_fine = pl.total_fine;
    c->bmap_dev = (int32_t*)(base + pl.off_bmap);
    c->chain_off_dev = (int64_t*)(base + pl.off_choff);
    c->rg2_dev = (double*)(base + pl.off_rg2);
    // host staging
    std::vector<double> soa(3 * N);
    for (int64_t i = 0; i < N; ++i)
        for (int a = 0; a < 3; ++a) soa[a * N + i] = pos[3 * i + a];
    std::vector<int32_t> sysid(N), tag(N, -1);
    for (int s = 0; s < nsys; ++s)
        for (int64_t i = so[s]; i < so[s + 1]; ++i) sysid[i] = s;
    std::vector<double> cube(pl.pool_cube), shell(pl.pool_shell);
    for (size_t k = 0; k < pool.size(); ++k) {
        std::copy(pool[k].cdf.begin(), pool[k].cdf.end(), cube.begin() + k * pool[k].cdf.size());
        std::copy(pool[k].shell.begin(), pool[k].shell.end(), shell.begin() + k * 4097);
    }
    plan_launches(c, p, pos, pl, p->periodic ? std::min(cell_coop_blocks(), CELL_LAUNCH_MAX) : 0,
                  std::min(pw_coop_blocks(), PW_LAUNCH_MAX));
    HIPCHK(c, hipMemsetAsync(base, 0, pl.bytes - 256, st));
    HIPCHK(c, hipMemcpyAsync(D.x, soa.data(), 3 * N * 8, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(D.bond_next, bond.data(), N, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(D.sys_id, sysid.data(), N * 4, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(D.tag, tag.data(), N * 4, hipMemcpyHostToDevice, st));
    if (!cube.empty()) HIPCHK(c, hipMemcpyAsync((void*)D.cube_cdf, cube.data(), cube.size() * 8, hipMemcpyHostToDevice, st));
    if (!shell.empty())
        HIPCHK(c, hipMemcpyAsync((void*)D.shell_s, shell.data(), shell.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync((void*)D.sys, c->sys.data(), nsys * sizeof(SysDesc), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync((void*)D.lev, c->lev.data(), c->lev.size() * sizeof(LevelDesc), hipMemcpyHostToDevice, st));
    if (!c->bmap_host.empty())
        HIPCHK(c, hipMemcpyAsync(c->bmap_dev, c->bmap_host.data(), c->bmap_host.size() * 4, hipMemcpyHostToDevice, st));
    if (!c->coop_host.empty())
        HIPCHK(c, hipMemcpyAsync(c->coop_dev, c->coop_host.data(), c->coop_host.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->chain_off_dev, co, (n_chains + 1) * 8, hipMemcpyHostToDevice, st));
    launch_com(D, c->chain_off_dev, n_chains, 1, nullptr, st);  // reference centres of mass
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    return 0;
}

// devices whose library-held arena a live context occupies
static std::mutex g_static_mu;
static bool g_static_busy[kMaxDevices] = {false};

extern "C" int wmc_init_static(wmc_ctx** out, const wmc_params* p, int32_t nsys, const int64_t* so,
                               const double* sL, const double* sl, int64_t n_chains, const int64_t* co,
                               const double* pos, int64_t trace_cap, void* stream) {
    if (!out) return WMC_EINVAL;
    size_t need = 0;
    int rc = wmc_arena_bytes(p, nsys, so, sL, sl, n_chains, co, trace_cap, &need);
    if (rc) {
        wmc_ctx* c = new wmc_ctx();
        *out = c;
        validate(c, p, nsys, so, sL, sl, n_chains, co);
        if (c->err.empty()) c->err = "invalid problem";
        return rc;
    }
    if (need > (size_t)WMC_STATIC_ARENA_BYTES) {
        wmc_ctx* c = new wmc_ctx();
        *out = c;
        c->err = "problem needs " + std::to_string(need) + " bytes of device arena, more than the " +
                 std::to_string((size_t)WMC_STATIC_ARENA_BYTES) + " bytes of the library-held arena";
        return WMC_EARENA;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) e = hipErrorInvalidDevice;
    if (e != hipSuccess) {
        wmc_ctx* c = new wmc_ctx();
        *out = c;
        c->err = std::string("HIP error: ") + hipGetErrorString(e) + " at hipGetDevice";
        return WMC_EHIP;
    }
    {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static_busy[dev]) {
            wmc_ctx* c = new wmc_ctx();
            *out = c;
            c->err = "the library-held arena of this device is in use by another context (wmc_free it first)";
            return WMC_EARENA;
        }
        g_static_busy[dev] = true;
    }
    void* base = static_arena(dev, &e);
    if (!base) {
        {
            std::lock_guard<std::mutex> lock(g_static_mu);
            g_static_busy[dev] = false;
        }
        wmc_ctx* c = new wmc_ctx();
        *out = c;
        c->err = std::string("HIP error: ") + hipGetErrorString(e) + " at hipGetSymbolAddress";
        return WMC_EHIP;
    }
    rc = wmc_init(out, p, nsys, so, sL, sl, n_chains, co, pos, trace_cap, base, (size_t)WMC_STATIC_ARENA_BYTES,
                  stream);
    if (*out) (*out)->static_dev = dev;  // wmc_free releases the arena, also after a failed init
    return rc;
}

static hipEvent_t take_event(wmc_ctx* c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// record an event pair around the launches of one kernel class when timing is on
struct Timed {
    wmc_ctx* c;
    int cls;
    hipStream_t st;
    hipEvent_t a = nullptr;
    Timed(wmc_ctx* c_, int cls_, hipStream_t st_) : c(c_), cls(cls_), st(st_) {
        if (c->timing && (a = take_event(c))) (void)hipEventRecord(a, st);
    }
    ~Timed() {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (!b) return;
        (void)hipEventRecord(b, st);
        c->ev_pending.push_back({cls, {a, b}});
    }
};

static void drain_events(wmc_ctx* c) {
    for (auto& p : c->ev_pending) {
        float ms = 0.0f;
        (void)hipEventSynchronize(p.second.second);
        if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
            c->t_ms[p.first] += ms;
            c->t_n[p.first] += 1;
        }
        c->ev_pool.push_back(p.second.first);
        c->ev_pool.push_back(p.second.second);
    }
    c->ev_pending.clear();
}

extern "C" int wmc_sweep(wmc_ctx* c, int64_t n_sweeps, void* stream) {
    if (!c) return WMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    for (int64_t k = 0; k < n_sweeps; ++k) {
        const int64_t sw = c->sweep;
        for (int l = 0; c->p.wavelets && l < c->max_levels; ++l) {
            if (c->P.periodic) {
                {
                    Timed t(c, 0, st);
                    launch_fine_build(c->P, c->D, c->N, st);
                }
                // LDS-tile cells of every colour in one dependency-ordered pass (their tile lists
                // are consecutive in the block map, colour by colour)
                FlowArgs fa;
                fa.nitems = 0;
                for (int col = 0; col < 8; ++col) {
                    fa.nitems += c->tile_n[l][col];
                    fa.colour_end[col] = fa.nitems;
                }
                const int tv = c->tune_variant[l] > 0 ? std::max(c->phase_variant[l], c->tune_variant[l] - 1)
                                                      : c->phase_variant[l];
                if (fa.nitems > 0 && c->tune_pass[l] == 2) {
                    // one launch per colour: the colour phases in order
                    for (int col = 0; col < 8; ++col) {
                        if (c->tile_n[l][col] <= 0) continue;
                        Timed t(c, 1 + l, st);
                        launch_phase(tv, c->P, c->D, l, col, sw, c->bmap_dev + 2 * c->tile_off[l][col],
                                     c->tile_n[l][col], st);
                    }
                } else if (fa.nitems > 0) {
                    Timed t(c, 1 + l, st);
                    fa.epoch = ++c->flow_epoch;
                    fa.qbase = c->flow_handed[l];
                    c->flow_handed[l] += (unsigned long long)fa.nitems;
                    launch_level_flow(tv, c->P, c->D, l, sw, c->bmap_dev + 2 * c->tile_off[l][0], fa,
                                      c->tune_width[l], st);
                }
                // global-list cells colour by colour: cooperative groups, else one workgroup each;
                // every colour in one group launch when their groups agree
                bool merged = false;
                const bool groups = c->tune_groups[l] != 2;
                if (c->cmerge[l] && groups) {
                    CoopColours cc;
                    cc.n = 0;
                    int c0 = -1;
                    for (int col = 0; col < 8; ++col) {
                        if (c->glob_n[l][col] <= 0) continue;
                        if (c0 < 0) c0 = col;
                        cc.col[cc.n] = col;
                        cc.goff[cc.n] = (int32_t)(c->cgrp_off[l][col] - c->cgrp_off[l][c0]);
                        ++cc.n;
                    }
                    Timed t(c, 1 + l, st);
                    merged = launch_cell_coop(c->P, c->D, l, cc, sw, (const CoopGroup*)(c->coop_dev + c->cgrp_off[l][c0]),
                                              c->coop_dev + c->cwg_off[l][c0], c->cwg_n[l][c0], st);
                }
                for (int col = 0; col < 8 && !merged; ++col) {
                    if (c->glob_n[l][col] <= 0) continue;
                    Timed t(c, 1 + l, st);
                    CoopColours cc;
                    cc.n = 1;
                    cc.col[0] = col;
                    cc.goff[0] = 0;
                    if (c->cwg_n[l][col] > 0 && groups &&
                        launch_cell_coop(c->P, c->D, l, cc, sw, (const CoopGroup*)(c->coop_dev + c->cgrp_off[l][col]),
                                         c->coop_dev + c->cwg_off[l][col], c->cwg_n[l][col], st))
                        continue;
                    launch_phase(c->phase_variant[l], c->P, c->D, l, col, sw, c->bmap_dev + 2 * c->glob_off[l][col],
                                 c->glob_n[l][col], st);
                }
            } else {
                launch_bbox(c->P, c->D, l, sw, st);
                for (int col = 0; col < 8; ++col) {
                    Timed t(c, 1 + l, st);
                    launch_phase(c->phase_variant[l], c->P, c->D, l, col, sw, nullptr, 64, st);
                }
            }
        }
        if (!c->P.periodic && c->P.plane_waves) {
            // infinite system: one workgroup, every pair of beads (no neighbour grid)
            Timed t(c, 17, st);
            launch_pw(c->P, c->D, sw, c->nsys, st);
        } else if (c->P.plane_waves) {
            {
                Timed t(c, 0, st);
                launch_fine_build(c->P, c->D, c->N, st);
            }
            Timed t(c, 17, st);
            // groups of workgroups per system when they fit one cooperative launch, otherwise one
            // workgroup per system
            if (!(c->pwg_n > 0 && c->tune_pw != 2 && launch_pw_coop(c->P, c->D, sw, (const CoopGroup*)(c->coop_dev + c->pgrp_off),
                                                 c->coop_dev + c->pwg_off, c->pwg_n, st)))
                launch_pw(c->P, c->D, sw, c->nsys, st);
        }
        c->sweep++;
        if (c->ev_pending.size() > 4096) drain_events(c);
    }
    HIPCHK(c, hipGetLastError());
    return 0;
}

extern "C" int wmc_set_timing(wmc_ctx* c, int32_t enable) {
    if (!c) return WMC_EINVAL;
    drain_events(c);
    c->timing = enable != 0;
    for (int i = 0; i < WMC_TIMING_CLASSES; ++i) {
        c->t_ms[i] = 0.0;
        c->t_n[i] = 0;
    }
    return 0;
}

extern "C" int wmc_kernel_times(wmc_ctx* c, double* ms_out, int64_t* n_out) {
    if (!c) return WMC_EINVAL;
    drain_events(c);
    for (int i = 0; i < WMC_TIMING_CLASSES; ++i) {
        if (ms_out) ms_out[i] = c->t_ms[i];
        if (n_out) n_out[i] = c->t_n[i];
    }
    return 0;
}

// ------------------------------------------------------------------- launch tuning
namespace {
const char* kVariantName[3] = {"V64", "V256", "V1024"};

// the current launch choices as JSON (times per level appended when given)
std::string tuning_json(const wmc_ctx* c, const std::vector<double>* level_ms, double pw_ms, int trial_sweeps) {
    std::string s = "{\"trial_sweeps\": " + std::to_string(trial_sweeps) + ", \"levels\": [";
    for (int l = 0; l < c->max_levels; ++l) {
        const int v = c->tune_variant[l] > 0 ? std::max(c->phase_variant[l], c->tune_variant[l] - 1) : c->phase_variant[l];
        int ntile = 0, nglob = 0;
        for (int col = 0; col < 8; ++col) {
            ntile += c->tile_n[l][col];
            nglob += c->glob_n[l][col];
        }
        char buf[360];
        snprintf(buf, sizeof(buf),
                 "%s{\"level\": %d, \"cells\": \"%s\", \"pass\": \"%s\", \"variant\": \"%s\", \"width\": %d, "
                 "\"groups\": \"%s\"",
                 l ? ", " : "", l, ntile && nglob ? "tile+global" : (ntile ? "tile" : "global"),
                 c->tune_pass[l] == 2 ? "colours" : "flow", kVariantName[v], c->tune_width[l],
                 c->tune_groups[l] == 2 ? "off" : "on");
        s += buf;
        if (level_ms) {
            snprintf(buf, sizeof(buf), ", \"ms_per_sweep\": %.4f", (*level_ms)[l]);
            s += buf;
        }
        s += "}";
    }
    s += std::string("], \"plane_wave_groups\": \"") + (c->tune_pw == 2 ? "off" : "on") + "\"";
    if (level_ms) {
        char buf[64];
        snprintf(buf, sizeof(buf), ", \"plane_wave_ms_per_sweep\": %.4f", pw_ms);
        s += buf;
    }
    return s + "}";
}

// value of "key" in a flat JSON object text (a string without its quotes, or a number), or ""
std::string json_field(const std::string& obj, const char* key) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return "";
    p = obj.find(':', p + k.size());
    if (p == std::string::npos) return "";
    ++p;
    while (p < obj.size() && (obj[p] == ' ' || obj[p] == '\n' || obj[p] == '\t')) ++p;
    if (p < obj.size() && obj[p] == '"') {
        const size_t e = obj.find('"', p + 1);
        return e == std::string::npos ? "" : obj.substr(p + 1, e - p - 1);
    }
    size_t e = p;
    while (e < obj.size() && (isalnum((unsigned char)obj[e]) || obj[e] == '-' || obj[e] == '.')) ++e;
    return obj.substr(p, e - p);
}

struct SavedState {
    void* snap = nullptr;
    int64_t sweep;
    int32_t epoch;
    unsigned long long handed[WMC_MAX_LEVELS];
};
int save_state(wmc_ctx* c, SavedState& s) {
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, hipMalloc(&s.snap, c->arena_used));
    HIPCHK(c, hipMemcpy(s.snap, c->arena, c->arena_used, hipMemcpyDeviceToDevice));
    s.sweep = c->sweep;
    s.epoch = c->flow_epoch;
    memcpy(s.handed, c->flow_handed, sizeof(s.handed));
    return 0;
}
// the device arena and the host counters that index it, as saved (the flow epoch keeps growing:
// an epoch value is never reused within a context)
int restore_state(wmc_ctx* c, const SavedState& s) {
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, hipMemcpy(c->arena, s.snap, c->arena_used, hipMemcpyDeviceToDevice));
    c->sweep = s.sweep;
    memcpy(c->flow_handed, s.handed, sizeof(s.handed));
    return 0;
}
}  // namespace

extern "C" int wmc_tune(wmc_ctx* c, int32_t trial_sweeps, char* json_out, size_t json_bytes) {
    if (!c || trial_sweeps < 1 || trial_sweeps > 1000) return WMC_EINVAL;
    if (!c->P.periodic || !c->p.wavelets) {
        c->err = "wmc_tune: periodic systems with wavelet moves only";
        return WMC_EINVAL;
    }
    struct Cand {
        int pass, variant, width, groups;
    };
    const int NL = c->max_levels;
    std::vector<std::vector<Cand>> cand(NL);
    int K = 1;
    for (int l = 0; l < NL; ++l) {
        int ntile = 0, nglob = 0, ngrp = 0;
        for (int col = 0; col < 8; ++col) {
            ntile += c->tile_n[l][col];
            nglob += c->glob_n[l][col];
            ngrp += c->cwg_n[l][col];
        }
        std::vector<Cand> tile, glob;
        if (ntile > 0) {
            for (int pass = 1; pass <= 2; ++pass)
                for (int v = c->phase_variant[l]; v <= V1024; ++v) {
                    if (v == V64 && pass == 1) {
                        tile.push_back({pass, v + 1, 64, 0});
                        tile.push_back({pass, v + 1, 256, 0});
                    } else {
                        tile.push_back({pass, v + 1, 0, 0});
                    }
                }
        } else {
            tile.push_back({0, 0, 0, 0});
        }
        glob.push_back({0, 0, 0, 0});
        if (nglob > 0 && ngrp > 0) glob.push_back({0, 0, 0, 2});
        for (const Cand& a : tile)
            for (const Cand& b : glob) cand[l].push_back({a.pass, a.variant, a.width, b.groups});
        K = std::max(K, (int)cand[l].size());
    }
    const int npw = c->pwg_n > 0 ? 2 : 1;
    K = std::max(K, npw);
    SavedState st0;
    int rc = save_state(c, st0);
    if (rc) return rc;
    const bool timing0 = c->timing;
    std::vector<std::vector<double>> ms(NL, std::vector<double>(K, 1e300));
    std::vector<double> pwms(K, 1e300);
    for (int k = 0; k < K && rc == 0; ++k) {
        for (int l = 0; l < NL; ++l) {
            const Cand& q = cand[l][k % cand[l].size()];
            c->tune_pass[l] = q.pass;
            c->tune_variant[l] = q.variant;
            c->tune_width[l] = q.width;
            c->tune_groups[l] = q.groups;
        }
        c->tune_pw = (k % npw) ? 2 : 0;
        if ((rc = restore_state(c, st0))) break;
        // one untimed sweep, then the timed ones, all from the saved state
        if ((rc = wmc_sweep(c, 1, nullptr))) break;
        wmc_set_timing(c, 1);
        if ((rc = wmc_sweep(c, trial_sweeps, nullptr))) break;
        double t[WMC_TIMING_CLASSES];
        wmc_kernel_times(c, t, nullptr);
        for (int l = 0; l < NL; ++l)
            if (k < (int)cand[l].size()) ms[l][k] = t[1 + l] / trial_sweeps;
        if (k < npw) pwms[k] = t[17] / trial_sweeps;
    }
    if (rc == 0) {
        std::vector<double> best_ms(NL);
        for (int l = 0; l < NL; ++l) {
            int b = 0;
            for (int k = 1; k < (int)cand[l].size(); ++k)
                if (ms[l][k] < ms[l][b]) b = k;
            c->tune_pass[l] = cand[l][b].pass;
            c->tune_variant[l] = cand[l][b].variant;
            c->tune_width[l] = cand[l][b].width;
            c->tune_groups[l] = cand[l][b].groups;
            best_ms[l] = ms[l][b];
        }
        const int bp = (npw > 1 && pwms[1] < pwms[0]) ? 1 : 0;
        c->tune_pw = bp ? 2 : 0;
        rc = restore_state(c, st0);
        const std::string js = tuning_json(c, &best_ms, pwms[bp], trial_sweeps);
        if (json_out && json_bytes > 0) {
            strncpy(json_out, js.c_str(), json_bytes - 1);
            json_out[json_bytes - 1] = '\0';
            if (js.size() >= json_bytes && rc == 0) {
                c->err = "wmc_tune: json_out too small";
                rc = WMC_EINVAL;
            }
        }
    } else {
        restore_state(c, st0);
    }
    (void)hipFree(st0.snap);
    wmc_set_timing(c, timing0 ? 1 : 0);
    return rc;
}

extern "C" int wmc_set_tuning(wmc_ctx* c, const char* json) {
    if (!c || !json) return WMC_EINVAL;
    const std::string s(json);
    int pass[WMC_MAX_LEVELS] = {0}, var[WMC_MAX_LEVELS] = {0}, width[WMC_MAX_LEVELS] = {0}, grp[WMC_MAX_LEVELS] = {0};
    size_t p = s.find("\"levels\"");
    if (p == std::string::npos) {
        c->err = "wmc_set_tuning: no \"levels\" array";
        return WMC_EINVAL;
    }
    const size_t end = s.find(']', p);
    for (size_t o = s.find('{', p); o != std::string::npos && o < end; o = s.find('{', o + 1)) {
        const size_t e = s.find('}', o);
        if (e == std::string::npos) break;
        const std::string obj = s.substr(o, e - o + 1);
        const std::string ls = json_field(obj, "level");
        char* endp = nullptr;
        const long l = strtol(ls.c_str(), &endp, 10);
        if (ls.empty() || *endp || l < 0 || l >= WMC_MAX_LEVELS) {
            c->err = "wmc_set_tuning: bad level in " + obj;
            return WMC_EINVAL;
        }
        const std::string ps = json_field(obj, "pass"), vs = json_field(obj, "variant"),
                          ws = json_field(obj, "width"), gs = json_field(obj, "groups");
        pass[l] = ps == "colours" ? 2 : (ps == "flow" || ps.empty() ? 1 : -1);
        var[l] = vs.empty() ? 0 : (vs == "V64" ? 1 : vs == "V256" ? 2 : vs == "V1024" ? 3 : -1);
        width[l] = ws.empty() || ws == "0" ? 0 : (ws == "64" ? 64 : ws == "256" ? 256 : -1);
        grp[l] = gs == "off" ? 2 : (gs == "on" || gs.empty() ? 0 : -1);
        if (pass[l] < 0 || var[l] < 0 || width[l] < 0 || grp[l] < 0) {
            c->err = "wmc_set_tuning: bad value in " + obj;
            return WMC_EINVAL;
        }
        if (pass[l] == 1) pass[l] = 0;
    }
    const std::string pw = json_field(s, "plane_wave_groups");
    if (!pw.empty() && pw != "on" && pw != "off") {
        c->err = "wmc_set_tuning: bad plane_wave_groups";
        return WMC_EINVAL;
    }
    for (int l = 0; l < WMC_MAX_LEVELS; ++l) {
        c->tune_pass[l] = pass[l];
        c->tune_variant[l] = var[l];
        c->tune_width[l] = width[l];
        c->tune_groups[l] = grp[l];
    }
    c->tune_pw = pw == "off" ? 2 : 0;
    return 0;
}

extern "C" int wmc_get_tuning(wmc_ctx* c, char* json_out, size_t json_bytes) {
    if (!c || !json_out || json_bytes == 0) return WMC_EINVAL;
    const std::string js = tuning_json(c, nullptr, 0.0, 0);
    strncpy(json_out, js.c_str(), json_bytes - 1);
    json_out[json_bytes - 1] = '\0';
    if (js.size() >= json_bytes) {
        c->err = "wmc_get_tuning: json_out too small";
        return WMC_EINVAL;
    }
    return 0;
}

extern "C" int wmc_positions(wmc_ctx* c, double* out, int32_t to_device, void* stream) {
    if (!c || !out) return WMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = c->N;
    if (to_device) {
        // interleave SoA -> [N][3] with strided copies
        for (int a = 0; a < 3; ++a)
            HIPCHK(c, hipMemcpy2DAsync(out + a, 3 * sizeof(double), c->D.x + a * N, sizeof(double), sizeof(double), N,
                                       hipMemcpyDeviceToDevice, st));
        return 0;
    }
    std::vector<double> soa(3 * N);
    HIPCHK(c, hipMemcpyAsync(soa.data(), c->D.x, 3 * N * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    for (int64_t i = 0; i < N; ++i)
        for (int a = 0; a < 3; ++a) out[3 * i + a] = soa[a * N + i];
    return 0;
}

extern "C" int wmc_set_state(wmc_ctx* c, const double* pos, int64_t sweep, void* stream) {
    if (!c || !pos) return WMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = c->N;
    std::vector<double> soa(3 * N);
    for (int64_t i = 0; i < N; ++i)
        for (int a = 0; a < 3; ++a) soa[a * N + i] = pos[3 * i + a];
    HIPCHK(c, hipMemcpyAsync(c->D.x, soa.data(), 3 * N * 8, hipMemcpyHostToDevice, st));
    launch_com(c->D, c->chain_off_dev, c->n_chains, 1, nullptr, st);  // new reference centres of mass
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    c->sweep = sweep;
    return 0;
}

extern "C" int wmc_observables(wmc_ctx* c, wmc_obs* o) {
    if (!c || !o) return WMC_EINVAL;
    HIPCHK(c, hipDeviceSynchronize());
    std::vector<unsigned long long> cnt(CNT_TOTAL);
    HIPCHK(c, hipMemcpy(cnt.data(), c->D.cnt, CNT_TOTAL * 8, hipMemcpyDeviceToHost));
    memset(o, 0, sizeof(*o));
    o->sweeps = c->sweep;
    for (int l = 0; l < WMC_MAX_LEVELS; ++l) {
        const unsigned long long* C = cnt.data() + CNT_LEVEL + l * 8;
        o->trials[l] = C[0];
        o->hits[l] = C[1];
        o->attempts[l] = C[2];
        o->accepts[l] = C[3];
        o->caps[l] = C[4];
        o->redraws[l] = C[5];
        o->bead_updates[l] = C[6];
    }
    const unsigned long long* W = cnt.data() + CNT_PW;
    o->pw_chains = W[0];
    o->pw_attempts = W[1];
    o->pw_accepts = W[2];
    o->pw_k0 = W[3];
    o->pw_caps = W[4];
    o->pw_bead_updates = W[5];
    o->violations = cnt[CNT_VIOL];
    o->overflows = cnt[CNT_OVERFLOW];
    o->rechecks = cnt[CNT_RECHECK];
    o->grid_rebuilds = cnt[CNT_REBUILD];
    o->accepted_total = cnt[CNT_ACCEPTED];
    o->wait_timeouts = cnt[CNT_FLOWWAIT];
    o->fallback_cells = cnt[CNT_FALLBACK];
    o->accepted_bead_updates = cnt[CNT_ACC_BEADS];
    for (int k = 0; k < WMC_K_SHELLS; ++k) {
        o->pw_shell_attempts[k] = cnt[CNT_SHELL + 2 * k];
        o->pw_shell_accepts[k] = cnt[CNT_SHELL + 2 * k + 1];
    }
    o->member_rechecks = cnt[CNT_MEMBER_RECHECK];
    o->margin_checks = cnt[CNT_MARGIN_CHECK];
    o->margin_fails = cnt[CNT_MARGIN_FAIL];
    {
        float r;
        const uint32_t bits = (uint32_t)cnt[CNT_MARGIN_RATIO];
        memcpy(&r, &bits, 4);
        o->margin_max_ratio = r;
    }
    if (o->overflows > 0) {
        c->err = "a cell list overflowed its capacity: the sweeps since wmc_init are not valid samples";
        return WMC_ECAPACITY;
    }
    if (o->wait_timeouts > 0) {
        c->err = "a dependency wait between cells hit its bound: the sweeps since wmc_init are not valid samples";
        return WMC_ESCHEDULE;
    }
    return 0;
}

extern "C" int wmc_system_tau(wmc_ctx* c, double* out) {
    if (!c || !out) return WMC_EINVAL;
    HIPCHK(c, hipDeviceSynchronize());
    std::vector<unsigned long long> acc(c->nsys);
    HIPCHK(c, hipMemcpy(acc.data(), c->D.sys_acc, c->nsys * 8, hipMemcpyDeviceToHost));
    for (int s = 0; s < c->nsys; ++s) out[s] = c->sys[s].dt * (double)acc[s];
    return 0;
}

extern "C" int wmc_chain_rg2(wmc_ctx* c, double* out) {
    if (!c || !out) return WMC_EINVAL;
    HIPCHK(c, hipDeviceSynchronize());
    launch_rg2(c->D, c->chain_off_dev, c->n_chains, c->rg2_dev, nullptr);
    HIPCHK(c, hipMemcpy(out, c->rg2_dev, c->n_chains * 8, hipMemcpyDeviceToHost));
    return 0;
}

extern "C" int wmc_chain_com(wmc_ctx* c, double* out) {
    if (!c || !out) return WMC_EINVAL;
    HIPCHK(c, hipDeviceSynchronize());
    launch_com(c->D, c->chain_off_dev, c->n_chains, 0, c->rg2_dev, nullptr);
    HIPCHK(c, hipMemcpy(out, c->rg2_dev, c->n_chains * 3 * 8, hipMemcpyDeviceToHost));
    return 0;
}

extern "C" int wmc_chain_msd(wmc_ctx* c, double* out) {
    if (!c || !out) return WMC_EINVAL;
    HIPCHK(c, hipDeviceSynchronize());
    launch_com(c->D, c->chain_off_dev, c->n_chains, 2, c->rg2_dev, nullptr);
    HIPCHK(c, hipMemcpy(out, c->rg2_dev, c->n_chains * 8, hipMemcpyDeviceToHost));
    return 0;
}

extern "C" int wmc_trace(wmc_ctx* c, wmc_trace_rec* out, int64_t max, int64_t* n_out) {
    if (!c || !n_out) return WMC_EINVAL;
    HIPCHK(c, hipDeviceSynchronize());
    unsigned long long n = 0;
    HIPCHK(c, hipMemcpy(&n, c->D.trace_n, 8, hipMemcpyDeviceToHost));
    int64_t have = std::min<int64_t>((int64_t)n, c->D.trace_cap);
    int64_t take = std::min<int64_t>(have, max);
    if (take > 0) HIPCHK(c, hipMemcpy(out, c->D.trace, take * sizeof(wmc_trace_rec), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemset(c->D.trace_n, 0, 8));
    *n_out = take;
    if ((int64_t)n > c->D.trace_cap) {
        c->err = "trace overflowed; records were dropped";
        return WMC_ECAPACITY;
    }
    return 0;
}

extern "C" int wmc_system_info(wmc_ctx* c, int32_t system, double* levels_out, int32_t* n_levels, double* pw_out) {
    if (!c || system < 0 || system >= c->nsys) return WMC_EINVAL;
    const std::vector<double>& l = c->level_out[system];
    if (levels_out) std::copy(l.begin(), l.end(), levels_out);
    if (n_levels) *n_levels = (int32_t)(l.size() / 6);
    if (pw_out) std::copy(c->pw_out[system].begin(), c->pw_out[system].end(), pw_out);
    return 0;
}

extern "C" int wmc_cell_ids(wmc_ctx* c, int32_t system, int64_t sweep, int32_t level, int32_t* out) {
    if (!c || !out || system < 0 || system >= c->nsys || level < 0 || level >= c->sys[system].n_levels)
        return WMC_EINVAL;
    if (!c->P.periodic) launch_bbox(c->P, c->D, level, sweep, nullptr);
    int32_t* dev = c->D.fcell;  // reused as scratch: rebuilt at the next grid build
    launch_cell_ids(c->P, c->D, system, level, sweep, c->sys[system].N, dev, nullptr);
    HIPCHK(c, hipMemcpy(out, dev, c->sys[system].N * 4, hipMemcpyDeviceToHost));
    return 0;
}

extern "C" int wmc_philox(const uint32_t ctr[4], const uint32_t key[2], int64_t n, uint32_t* out, void* scratch,
                          size_t scratch_bytes, void* stream) {
    if (!ctr || !key || !out || n <= 0 || !scratch || scratch_bytes < (size_t)n * 16) return WMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    launch_philox(ctr, key, n, (uint32_t*)scratch, st);
    if (hipMemcpyAsync(out, scratch, n * 16, hipMemcpyDeviceToHost, st) != hipSuccess) return WMC_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return WMC_EHIP;
    return 0;
}

extern "C" const char* wmc_last_error(const wmc_ctx* c) { return c ? c->err.c_str() : "no context"; }

extern "C" void wmc_free(wmc_ctx* c) {
    if (!c) return;
    drain_events(c);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_busy[c->static_dev] = false;
    }
    delete c;
}
