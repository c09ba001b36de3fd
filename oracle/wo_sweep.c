/*
 * Oracle: the sweep, replayed serially in FP64 (test infrastructure only).
 *
 * One sweep of one system, in order:
 *  for each level band (ascending lambda):
 *    grid shift u from stream (tag 32+l); periodic grid of side h = L/n, or for an
 *    infinite system the cells of the lattice h (k + u) that cover the bounding box of the
 *    positions (colour = parity of k, stream key = k mod 256 per axis);
 *    for colour 0..7, for each cell of that colour in ascending id:
 *      S_c = particles within hi of the cell, H_c = within hi + r_int (ascending id);
 *      K_c = stochastic rounding of T_l |S_c| / N (stream tag 16+l);
 *      for each trial t < K_c (stream tag l, cell, t):
 *        lambda in the band (App. D), anchor a uniform in S_c, V uniform in the unit
 *        ball by rejection (App. D), b = r_a + lambda V; b outside the cell: next t;
 *        else a recycling chain with this lambda: p = V'/|V'| (App. D), n = number of
 *        particles within lambda of b, A_w = A0 lambda / sqrt(n) (Eq. "Wavelet amplitude"),
 *        displacement A_w w((r-b)/lambda, p) (Eqs. "Oseen as <ww>", "Tapered wavelet"),
 *        dU over the bonds and WCA pairs the members touch, Metropolis test
 *        (Eq. "Metropolis test"); after a rejection the same lambda is reused with a
 *        new anchor, b (redrawn until it lies in the cell) and p (App. D recycling),
 *        up to retry_cap attempts.
 *  plane waves: H_F = stochastic rounding of N P_F chains; periodic k from the cube or the
 *  quasi-continuous shell (App. D), infinite |k| from its tabulated inverse CDF and k-hat
 *  isotropic (App. D); phase Phi and e-hat perpendicular to k,
 *  displacement A_F cos(k.r + Phi) e-hat on every particle (Eq. "Oseen as <FF>"),
 *  A_F = 2 A0 / (k sqrt(5 N)) (Eq. "Fourier strain energy" with dU_est/mu = A0^2 M6/(2pi)^3),
 *  k = 0 accepted without displacement; a rejection permutes and sign-flips k (periodic) or
 *  redraws k-hat (infinite).
 *  Variants (wmc_oracle.h): Glauber acceptance, the exact-rotation map, uniform centring.
 *  time advances by dt per accepted chain (App. D, last paragraph).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "wo_internal.h"

#define TAG_SHIFT 32
#define TAG_META 16
#define TAG_PWCOUNT 48
#define TAG_PW 49

static void trace_push(wo_ctx* c, int kind, int sys, int level, int64_t cell, int64_t trial,
                       int retry, int64_t n, int acc, int extra, double dU, double thr) {
    if (c->trace_n >= c->trace_cap) return;
    wo_trace_rec* r = &c->trace[c->trace_n++];
    r->kind = kind;
    r->system = sys;
    r->sweep = (int32_t)c->sweep;
    r->level = level;
    r->cell = (int32_t)cell;
    r->trial = (int32_t)trial;
    r->retry = retry;
    r->n = (int32_t)n;
    r->accepted = acc;
    r->extra = extra;
    r->dU = dU;
    r->thr = thr;
}

/* ---------------------------------------------------------------- potentials ------ */
static double u_bond(const wo_ctx* c, double r2) {
    if (c->p.bond_type == WO_BOND_FENE) {
        double R02 = c->p.R0 * c->p.R0;
        if (r2 >= R02) return INFINITY;
        return -0.5 * c->p.k_bond * R02 * log(1.0 - r2 / R02);
    }
    if (c->p.bond_type == WO_BOND_HARMONIC) return 0.5 * c->p.k_bond * r2;
    return 0.0;
}

static double u_pair(const wo_ctx* c, double r2) {
    if (r2 >= c->rc2) return 0.0;
    if (r2 <= 0.0) return INFINITY;
    double s2 = c->p.sigma * c->p.sigma / r2;
    double s6 = s2 * s2 * s2;
    return 4.0 * c->p.eps * (s6 * s6 - s6 + 0.25);
}

/* Acceptance threshold on dU for a uniform u in (0, 1]: Metropolis (Eq. "Metropolis test")
 * accepts with probability min(1, exp(-dU/kT)), i.e. iff dU <= -kT ln u; Glauber accepts
 * with probability 1/(1 + exp(dU/kT)), i.e. iff dU <= kT ln((1 - u)/u). (1 - u is exact for
 * u = m 2^-53.) */
static double threshold(const wo_ctx* c, double u) {
    if (c->p.accept_rule == WO_ACCEPT_GLAUBER) return c->p.kT * (log(1.0 - u) - log(u));
    return -c->p.kT * log(u);
}

/* ------------------------------------------------------------------ geometry ------ */
typedef struct {
    int periodic;
    double L, invL;
    double o[3];
    double h, invh, half;
    int64_t n[3];
    int64_t k0[3];   /* infinite system: lattice index of local cell 0 along each axis */
    double hi, rh;
} grid_t;

static double minimg(const grid_t* g, double d) {
    if (g->periodic) d = d - g->L * rint(d * g->invL);
    return d;
}

static double pair_r2(const wo_ctx* c, const wo_system* s, double ax, double ay, double az,
                      double bx, double by, double bz) {
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    if (c->p.periodic) {
        double L = s->L, invL = 1.0 / s->L;
        dx = dx - L * rint(dx * invL);
        dy = dy - L * rint(dy * invL);
        dz = dz - L * rint(dz * invL);
    }
    return (dx * dx + dy * dy) + dz * dz;
}

static void make_grid(wo_ctx* c, wo_system* s, int sysid, int level, grid_t* g) {
    const wo_level_info* lv = &s->lev[level];
    wo_stream st;
    wo_stream_init(&st, c->p.seed, sysid, c->sweep, TAG_SHIFT + level, 0, 0, 0, 0);
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = wo_next_co(&st);
    g->periodic = c->p.periodic;
    g->hi = lv->hi;
    g->rh = lv->hi + lv->r_int;
    g->h = lv->h;
    g->invh = 1.0 / lv->h;
    g->half = 0.5 * lv->h;
    if (c->p.periodic) {
        g->L = s->L;
        g->invL = 1.0 / s->L;
        for (int a = 0; a < 3; ++a) {
            g->o[a] = lv->h * u[a];
            g->n[a] = lv->ncell;
            g->k0[a] = 0;
        }
    } else {
        g->L = 0.0;
        g->invL = 0.0;
        double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t i = s->b0; i < s->b1; ++i) {
            double v[3] = {c->x[i], c->y[i], c->z[i]};
            for (int a = 0; a < 3; ++a) {
                if (v[a] < mn[a]) mn[a] = v[a];
                if (v[a] > mx[a]) mx[a] = v[a];
            }
        }
        /* cells of the fixed lattice h (k + u), k integer, that cover the bounding box grown by
         * hi: the lattice, the colour of a cell (parity of k) and its stream key do not depend
         * on the positions, so the sweep is the same mixture of moves from every state */
        for (int a = 0; a < 3; ++a) {
            int64_t kmin = (int64_t)floor((mn[a] - lv->hi) * g->invh - u[a]);
            int64_t kmax = (int64_t)floor((mx[a] + lv->hi) * g->invh - u[a]);
            g->k0[a] = kmin;
            g->o[a] = ((double)kmin + u[a]) * lv->h;
            g->n[a] = kmax - kmin + 1;
        }
    }
}

/* colour of a cell: parity of its lattice index along each axis */
static int cell_colour(const grid_t* g, const int64_t ic[3]) {
    return (int)(((g->k0[0] + ic[0]) & 1) | (((g->k0[1] + ic[1]) & 1) << 1) | (((g->k0[2] + ic[2]) & 1) << 2));
}

/* stream key of a cell: its index (periodic), or its lattice index modulo 256 per axis
 * (infinite system; distinct for systems spanning fewer than 256 cells per axis) */
static int64_t cell_key(const grid_t* g, const int64_t ic[3]) {
    if (g->periodic) return ic[0] + g->n[0] * (ic[1] + g->n[1] * ic[2]);
    return ((g->k0[0] + ic[0]) & 255) | (((g->k0[1] + ic[1]) & 255) << 8) | (((g->k0[2] + ic[2]) & 255) << 16);
}

static int64_t cell_of_point(const grid_t* g, double bx, double by, double bz) {
    double b[3] = {bx, by, bz};
    int64_t ic[3];
    for (int a = 0; a < 3; ++a) {
        double v = b[a];
        if (g->periodic) v = v - g->L * floor(v * g->invL);
        int64_t i = (int64_t)floor((v - g->o[a]) * g->invh);
        if (g->periodic) {
            i %= g->n[a];
            if (i < 0) i += g->n[a];
        } else if (i < 0 || i >= g->n[a]) {
            return -1;
        }
        ic[a] = i;
    }
    return ic[0] + g->n[0] * (ic[1] + g->n[1] * ic[2]);
}

static double dist2_cell(const grid_t* g, const int64_t ic[3], double x, double y, double z) {
    double v[3] = {x, y, z}, acc[3];
    for (int a = 0; a < 3; ++a) {
        double cen = g->o[a] + ((double)ic[a] + 0.5) * g->h;
        double d = minimg(g, v[a] - cen);
        double e = fabs(d) - g->half;
        if (e < 0.0) e = 0.0;
        acc[a] = e * e;
    }
    return (acc[0] + acc[1]) + acc[2];
}

/* ------------------------------------------------------ linked cells (pair search) -- */
static int64_t cl_cell(const wo_system* s, double x, double y, double z) {
    double v[3] = {x, y, z};
    int64_t c[3];
    for (int a = 0; a < 3; ++a) {
        double w = v[a] - s->L * floor(v[a] / s->L);
        int64_t i = (int64_t)floor(w * s->invcg);
        if (i >= s->nc) i = s->nc - 1;
        if (i < 0) i = 0;
        c[a] = i;
    }
    return c[0] + s->nc * (c[1] + s->nc * c[2]);
}

static void cl_insert(wo_ctx* c, wo_system* s, int64_t i, int64_t cell) {
    c->ccell[i] = cell;
    c->cprev[i] = -1;
    c->cnext[i] = s->head[cell];
    if (s->head[cell] >= 0) c->cprev[s->head[cell]] = i;
    s->head[cell] = i;
}

static void cl_remove(wo_ctx* c, wo_system* s, int64_t i) {
    int64_t cell = c->ccell[i];
    if (c->cprev[i] >= 0) c->cnext[c->cprev[i]] = c->cnext[i];
    else s->head[cell] = c->cnext[i];
    if (c->cnext[i] >= 0) c->cprev[c->cnext[i]] = c->cprev[i];
}

/* keep the list in step with a bead's new position */
static void cl_moved(wo_ctx* c, wo_system* s, int64_t i) {
    if (!s->nc) return;
    int64_t cell = cl_cell(s, c->x[i], c->y[i], c->z[i]);
    if (cell == c->ccell[i]) return;
    cl_remove(c, s, i);
    cl_insert(c, s, i, cell);
}

static void cl_build(wo_ctx* c, wo_system* s) {
    if (!s->nc) return;
    int64_t nc3 = (int64_t)s->nc * s->nc * s->nc;
    for (int64_t k = 0; k < nc3; ++k) s->head[k] = -1;
    for (int64_t i = s->b0; i < s->b1; ++i) cl_insert(c, s, i, cl_cell(s, c->x[i], c->y[i], c->z[i]));
}

/* call fn(m) once for every bead within the 27 cells around each of the points p and q
 * (every bead within r_cut of p or of q), or for every bead of the system without a list */
typedef void (*cand_fn)(wo_ctx* c, wo_system* s, int64_t m, void* arg);
static void cl_candidates(wo_ctx* c, wo_system* s, const double p[3], const double q[3], cand_fn fn, void* arg) {
    if (!s->nc) {
        for (int64_t m = s->b0; m < s->b1; ++m) fn(c, s, m, arg);
        return;
    }
    int64_t stamp = ++c->seen_stamp;
    const double* pts[2] = {p, q};
    for (int w = 0; w < 2; ++w) {
        int64_t cc = cl_cell(s, pts[w][0], pts[w][1], pts[w][2]);
        int64_t cx = cc % s->nc, cy = (cc / s->nc) % s->nc, cz = cc / ((int64_t)s->nc * s->nc);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t ex = (cx + dx + s->nc) % s->nc, ey = (cy + dy + s->nc) % s->nc, ez = (cz + dz + s->nc) % s->nc;
                    for (int64_t m = s->head[ex + s->nc * (ey + s->nc * ez)]; m >= 0; m = c->cnext[m]) {
                        if (c->seen[m] == stamp) continue;
                        c->seen[m] = stamp;
                        fn(c, s, m, arg);
                    }
                }
    }
}

/* ------------------------------------------------------------ one cell phase ----- */
static int draw_centre(wo_ctx* c, wo_stream* st, const grid_t* g, int64_t cell, int64_t nS,
                       double lam, int64_t* anchor, double b[3]) {
    int64_t a = c->S[wo_next_index(st, nS)];
    double vx, vy, vz, ss;
    do {
        vx = 2.0 * wo_next_co(st) - 1.0;
        vy = 2.0 * wo_next_co(st) - 1.0;
        vz = 2.0 * wo_next_co(st) - 1.0;
        ss = (vx * vx + vy * vy) + vz * vz;
    } while (ss > 1.0);
    b[0] = c->x[a] + lam * vx;
    b[1] = c->y[a] + lam * vy;
    b[2] = c->z[a] + lam * vz;
    *anchor = a;
    return cell_of_point(g, b[0], b[1], b[2]) == cell;
}

/* uniform centring: b uniform in the cell (homogeneous variant, Sec. IV "Distribution of
 * wavelet radii"); returns whether b rounds into the cell */
static int draw_uniform_centre(wo_stream* st, const grid_t* g, int64_t cell, const int64_t ic[3], double b[3]) {
    for (int a = 0; a < 3; ++a) b[a] = g->o[a] + ((double)ic[a] + wo_next_co(st)) * g->h;
    return cell_of_point(g, b[0], b[1], b[2]) == cell;
}

static void draw_direction(wo_stream* st, double p[3]) {
    double vx, vy, vz, ss;
    do {
        vx = 2.0 * wo_next_co(st) - 1.0;
        vy = 2.0 * wo_next_co(st) - 1.0;
        vz = 2.0 * wo_next_co(st) - 1.0;
        ss = (vx * vx + vy * vy) + vz * vz;
    } while (ss > 1.0 || ss == 0.0);
    double nrm = sqrt(ss);
    p[0] = vx / nrm;
    p[1] = vy / nrm;
    p[2] = vz / nrm;
}

typedef struct {
    int64_t j, stamp;
    double jx, jy, jz, kx, ky, kz, acc;
} pair_arg;

static void pair_nonmember(wo_ctx* c, wo_system* s, int64_t m, void* vp) {
    pair_arg* a = (pair_arg*)vp;
    if (m == a->j || c->mark[m] == a->stamp) return;
    double r2o = pair_r2(c, s, a->jx, a->jy, a->jz, c->x[m], c->y[m], c->z[m]);
    double r2n = pair_r2(c, s, a->kx, a->ky, a->kz, c->x[m], c->y[m], c->z[m]);
    if (r2o < c->rc2 || r2n < c->rc2) a->acc += u_pair(c, r2n) - u_pair(c, r2o);
}

/* one Metropolis test of a wavelet move; returns 1 if accepted (positions updated) */
static int wavelet_attempt(wo_ctx* c, wo_system* s, int sysid, int level, int64_t key,
                           int64_t t, int r, int64_t nS, double lam, int64_t anchor,
                           const double b[3], const double p[3], double u_acc) {
    double L = s->L, invL = c->p.periodic ? 1.0 / s->L : 0.0;
    int per = c->p.periodic;
    double lam2 = lam * lam;
    int64_t stamp = ++c->mark_stamp;
    int64_t n = 0;
    /* members: S_c in ascending id within lambda of b, plus the anchor */
    for (int64_t q = 0; q < nS; ++q) {
        int64_t j = c->S[q];
        double d[3] = {c->x[j] - b[0], c->y[j] - b[1], c->z[j] - b[2]};
        if (per)
            for (int a = 0; a < 3; ++a) d[a] = d[a] - L * rint(d[a] * invL);
        double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
        if (d2 <= lam2 || j == anchor) {
            c->M[n] = j;
            c->mark[j] = stamp;
            double xr[3] = {d[0] / lam, d[1] / lam, d[2] / lam};
            /* displacement computed below once n is known; stash scaled offsets */
            c->nx[j] = xr[0];
            c->ny[j] = xr[1];
            c->nz[j] = xr[2];
            ++n;
        }
    }
    /* amplitude: Eq. "Wavelet amplitude" with the local count n; uniform centring uses the mean
     * count <n> = (4 pi/3) lambda^3 N / L^3 of the homogeneous system instead */
    double A;
    if (c->p.centring == WO_CENTRE_UNIFORM)
        A = c->p.A0 * lam / sqrt((4.0 * WO_PI / 3.0) * lam * lam * lam * (double)s->N / (L * L * L));
    else
        A = c->p.A0 * lam / sqrt((double)n);
    for (int64_t q = 0; q < n; ++q) {
        int64_t j = c->M[q];
        double xr[3] = {c->nx[j], c->ny[j], c->nz[j]}, w[3];
        double rr = sqrt((xr[0] * xr[0] + xr[1] * xr[1]) + xr[2] * xr[2]);
        if (c->p.wavelet_map == WO_MAP_ROTATION) {
            /* rotation of x about the axis p through b by the angle a = (A/lambda)(1 - |x|),
             * Rodrigues' formula: x' - x = sin a (p x x) + (1 - cos a)(p (p.x) - x), with
             * 1 - cos a = 2 sin^2(a/2); to first order in a it is A (1 - |x|) p x x */
            double a = rr < 1.0 ? (A / lam) * (1.0 - rr) : 0.0;
            double sa = sin(a), hs = sin(0.5 * a), omc = 2.0 * hs * hs;
            double pd = (p[0] * xr[0] + p[1] * xr[1]) + p[2] * xr[2];
            w[0] = lam * (sa * (p[1] * xr[2] - p[2] * xr[1]) + omc * (p[0] * pd - xr[0]));
            w[1] = lam * (sa * (p[2] * xr[0] - p[0] * xr[2]) + omc * (p[1] * pd - xr[1]));
            w[2] = lam * (sa * (p[0] * xr[1] - p[1] * xr[0]) + omc * (p[2] * pd - xr[2]));
        } else {
            double f = rr < 1.0 ? A * (1.0 - rr) : 0.0;
            w[0] = f * (p[1] * xr[2] - p[2] * xr[1]);
            w[1] = f * (p[2] * xr[0] - p[0] * xr[2]);
            w[2] = f * (p[0] * xr[1] - p[1] * xr[0]);
        }
        c->nx[j] = c->x[j] + w[0];
        c->ny[j] = c->y[j] + w[1];
        c->nz[j] = c->z[j] + w[2];
    }
    /* energy change: bonds and WCA pairs with at least one member, each once */
    double dU = 0.0, rint2 = c->r_int * c->r_int;
    for (int64_t q = 0; q < n; ++q) {
        int64_t j = c->M[q];
        double jx = c->x[j], jy = c->y[j], jz = c->z[j];
        double kx = c->nx[j], ky = c->ny[j], kz = c->nz[j];
        if (c->p.bond_type != WO_BOND_NONE) {
            int64_t part[2] = {-1, -1};
            if (j + 1 < s->b1 && c->bond_next[j]) part[0] = j + 1;
            if (j > s->b0 && c->bond_next[j - 1]) part[1] = j - 1;
            for (int e = 0; e < 2; ++e) {
                int64_t m = part[e];
                if (m < 0) continue;
                int mem = c->mark[m] == stamp;
                if (mem && m < j) continue;
                double r2o = pair_r2(c, s, jx, jy, jz, c->x[m], c->y[m], c->z[m]);
                double r2n = mem ? pair_r2(c, s, kx, ky, kz, c->nx[m], c->ny[m], c->nz[m])
                                 : pair_r2(c, s, kx, ky, kz, c->x[m], c->y[m], c->z[m]);
                if (r2o > rint2) c->obs.violations++;
                dU += u_bond(c, r2n) - u_bond(c, r2o);
            }
        }
        if (c->p.wca) {
            /* pairs with non-members near the old or new position of j */
            pair_arg pa = {j, stamp, jx, jy, jz, kx, ky, kz, 0.0};
            double po[3] = {jx, jy, jz}, pn[3] = {kx, ky, kz};
            cl_candidates(c, s, po, pn, pair_nonmember, &pa);
            dU += pa.acc;
            /* pairs of two members, each once */
            for (int64_t q2 = q + 1; q2 < n; ++q2) {
                int64_t m = c->M[q2];
                double r2o = pair_r2(c, s, jx, jy, jz, c->x[m], c->y[m], c->z[m]);
                double r2n = pair_r2(c, s, kx, ky, kz, c->nx[m], c->ny[m], c->nz[m]);
                if (r2o < c->rc2 || r2n < c->rc2) dU += u_pair(c, r2n) - u_pair(c, r2o);
            }
        }
    }
    double thr = threshold(c, u_acc);
    int acc = dU <= thr;
    c->obs.attempts[level]++;
    c->obs.bead_updates[level] += n;
    trace_push(c, 0, sysid, level, key, t, r, n, acc, (int)anchor, dU, thr);
    if (acc) {
        for (int64_t q = 0; q < n; ++q) {
            int64_t j = c->M[q];
            c->x[j] = c->nx[j];
            c->y[j] = c->ny[j];
            c->z[j] = c->nz[j];
            cl_moved(c, s, j);
        }
        c->obs.accepts[level]++;
        c->obs.accepted_bead_updates += n;
    }
    return acc;
}

static void process_cell(wo_ctx* c, wo_system* s, int sysid, int level, const grid_t* g,
                         int64_t cell, const int64_t ic[3]) {
    const wo_level_info* lv = &s->lev[level];
    int64_t nS = 0;
    double hi2 = g->hi * g->hi;
    for (int64_t j = s->b0; j < s->b1; ++j)
        if (dist2_cell(g, ic, c->x[j], c->y[j], c->z[j]) <= hi2) c->S[nS++] = j;
    /* number of trials: stochastic rounding of T_l |S_c| / N (anchored centres), or of T_l times
     * the cell's share of the box volume, T_l / n^3 (uniform centres) */
    const int uni = c->p.centring == WO_CENTRE_UNIFORM;
    double mu = uni ? lv->T / ((double)g->n[0] * (double)g->n[1] * (double)g->n[2])
                    : (lv->T * (double)nS) / (double)s->N;
    int64_t K = (int64_t)floor(mu);
    wo_stream ms;
    const int64_t key = cell_key(g, ic);
    wo_stream_init(&ms, c->p.seed, sysid, c->sweep, TAG_META + level, key, 0, 0, 0);
    if (wo_next_co(&ms) < mu - (double)K) K += 1;
    if (K > 0xFFFFF) { K = 0xFFFFF; c->obs.violations++; }
    int64_t hits = 0;
    for (int64_t t = 0; t < K; ++t) {
        wo_stream st;
        wo_stream_init(&st, c->p.seed, sysid, c->sweep, level, key, t, 0, 0);
        double lam = wo_draw_lambda(wo_next_co(&st), lv->lo, lv->hi);
        int64_t anchor = -1;
        double b[3];
        c->obs.trials[level]++;
        if (uni ? !draw_uniform_centre(&st, g, cell, ic, b) : !draw_centre(c, &st, g, cell, nS, lam, &anchor, b))
            continue;
        c->obs.hits[level]++;
        ++hits;
        for (int r = 0;;) {
            double p[3];
            draw_direction(&st, p);
            double u_acc = wo_next_oc(&st);
            if (wavelet_attempt(c, s, sysid, level, key, t, r, nS, lam, anchor, b, p, u_acc)) {
                s->accepted++;
                c->obs.accepted_total++;
                break;
            }
            if (++r >= c->p.retry_cap) { c->obs.caps[level]++; break; }
            int found = 0;
            for (int j = 0; j < 4096; ++j) {
                wo_stream_init(&st, c->p.seed, sysid, c->sweep, level, key, t, r, j);
                if (uni ? draw_uniform_centre(&st, g, cell, ic, b) : draw_centre(c, &st, g, cell, nS, lam, &anchor, b)) {
                    found = 1;
                    break;
                }
                c->obs.redraws[level]++;
            }
            if (!found) { c->obs.caps[level]++; break; }
        }
    }
    trace_push(c, 1, sysid, level, key, K, (int)nS, 0, (int)hits, 0, 0.0, 0.0);
}

/* ------------------------------------------------------------- plane waves -------- */
static const int PERM[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

static void sample_k(wo_ctx* c, wo_system* s, wo_stream* st, int l[3]) {
    int NL = c->p.n_layers, D = 2 * NL + 1;
    if (wo_next_co(st) < s->info.P_cube) {
        double target = wo_next_co(st) * s->info.W_cube;
        int64_t lo = 0, hi = (int64_t)s->info.n_modes - 1;
        while (lo < hi) { /* smallest i with cdf[i] > target */
            int64_t mid = (lo + hi) / 2;
            if (s->cube_cdf[mid] > target) hi = mid; else lo = mid + 1;
        }
        int64_t i = lo;
        l[0] = (int)(i / ((int64_t)D * D)) - NL;
        l[1] = (int)((i / D) % D) - NL;
        l[2] = (int)(i % D) - NL;
        return;
    }
    double invks = s->L / (2.0 * WO_PI);
    for (int tries = 0;; ++tries) {
        if (tries >= 100000) { /* bounded like the GPU path; not reached with valid tables */
            l[0] = NL + 1;
            l[1] = 0;
            l[2] = 0;
            return;
        }
        double us = wo_next_co(st) * s->n_shell;
        int64_t i = (int64_t)floor(us);
        double fr = us - (double)i;
        double sv = s->shell_s[i] + fr * (s->shell_s[i + 1] - s->shell_s[i]);
        double v[3];
        draw_direction(st, v);
        if (!(sv > 1e-12)) continue;
        double kmag = (s->x_s / sv) / s->lmax;
        int ok = 1, inside = 1;
        for (int a = 0; a < 3; ++a) {
            double la = rint(kmag * v[a] * invks);
            if (fabs(la) > 1048576.0) ok = 0;
            l[a] = ok ? (int)la : 0;
            if (abs(l[a]) > NL) inside = 0;
        }
        if (ok && !inside) return;
    }
}

typedef struct {
    int64_t j;
    double acc;
} pw_arg;

static void pw_pair(wo_ctx* c, wo_system* s, int64_t m, void* vp) {
    pw_arg* a = (pw_arg*)vp;
    int64_t j = a->j;
    if (m <= j) return;
    double r2o = pair_r2(c, s, c->x[j], c->y[j], c->z[j], c->x[m], c->y[m], c->z[m]);
    double r2n = pair_r2(c, s, c->nx[j], c->ny[j], c->nz[j], c->nx[m], c->ny[m], c->nz[m]);
    if (r2o < c->rc2 || r2n < c->rc2) a->acc += u_pair(c, r2n) - u_pair(c, r2o);
}

/* one Metropolis test of the plane wave of wavevector k (nonzero); shell is its |k| shell and
 * extra its trace tag */
static int pw_attempt(wo_ctx* c, wo_system* s, int sysid, int64_t h, int r, const double k[3], int shell,
                      int extra, double Phi, double psi, double u_acc) {
    double kmag = sqrt((k[0] * k[0] + k[1] * k[1]) + k[2] * k[2]);
    double kh[3] = {k[0] / kmag, k[1] / kmag, k[2] / kmag};
    int ax = 0;
    for (int a = 1; a < 3; ++a)
        if (fabs(kh[a]) < fabs(kh[ax])) ax = a;
    double ref[3] = {0.0, 0.0, 0.0};
    ref[ax] = 1.0;
    double e1[3] = {kh[1] * ref[2] - kh[2] * ref[1], kh[2] * ref[0] - kh[0] * ref[2],
                    kh[0] * ref[1] - kh[1] * ref[0]};
    double n1 = sqrt((e1[0] * e1[0] + e1[1] * e1[1]) + e1[2] * e1[2]);
    for (int a = 0; a < 3; ++a) e1[a] = e1[a] / n1;
    double e2[3] = {kh[1] * e1[2] - kh[2] * e1[1], kh[2] * e1[0] - kh[0] * e1[2],
                    kh[0] * e1[1] - kh[1] * e1[0]};
    double cp = cos(psi), sp = sin(psi);
    double e[3] = {cp * e1[0] + sp * e2[0], cp * e1[1] + sp * e2[1], cp * e1[2] + sp * e2[2]};
    double AF = 2.0 * c->p.A0 / (kmag * sqrt(5.0 * (double)s->N));
    for (int64_t j = s->b0; j < s->b1; ++j) {
        double ph = ((k[0] * c->x[j] + k[1] * c->y[j]) + k[2] * c->z[j]) + Phi;
        double f = AF * cos(ph);
        c->nx[j] = c->x[j] + f * e[0];
        c->ny[j] = c->y[j] + f * e[1];
        c->nz[j] = c->z[j] + f * e[2];
    }
    double dU = 0.0;
    if (c->p.bond_type != WO_BOND_NONE) {
        for (int64_t j = s->b0; j + 1 < s->b1; ++j) {
            if (!c->bond_next[j]) continue;
            double r2o = pair_r2(c, s, c->x[j], c->y[j], c->z[j], c->x[j + 1], c->y[j + 1], c->z[j + 1]);
            double r2n = pair_r2(c, s, c->nx[j], c->ny[j], c->nz[j], c->nx[j + 1], c->ny[j + 1], c->nz[j + 1]);
            dU += u_bond(c, r2n) - u_bond(c, r2o);
        }
    }
    if (c->p.wca) {
        /* every pair j < m within r_cut before or after the move; both beads move by at most
         * A_F, and the cell side exceeds r_cut + 2 A_F, so the 27 cells around j hold them */
        for (int64_t j = s->b0; j < s->b1; ++j) {
            pw_arg pa = {j, 0.0};
            double po[3] = {c->x[j], c->y[j], c->z[j]};
            cl_candidates(c, s, po, po, pw_pair, &pa);
            dU += pa.acc;
        }
    }
    double thr = threshold(c, u_acc);
    int acc = dU <= thr;
    c->obs.pw_attempts++;
    c->obs.pw_bead_updates += s->N;
    c->obs.pw_shell_attempts[shell]++;
    if (acc) c->obs.pw_shell_accepts[shell]++;
    trace_push(c, 2, sysid, -1, h, 0, r, s->N, acc, extra, dU, thr);
    if (acc) {
        c->obs.accepted_bead_updates += s->N;
        for (int64_t j = s->b0; j < s->b1; ++j) {
            c->x[j] = c->nx[j];
            c->y[j] = c->ny[j];
            c->z[j] = c->nz[j];
        }
        cl_build(c, s);
        c->obs.pw_accepts++;
    }
    return acc;
}

/* x = |k| lambda_max of an infinite-system plane wave from its tail probability v in (0, 1]
 * (App. D "Choosing k for an infinite system": the tabulated inverse, interpolated) */
static double inf_x_of_v(const wo_system* s, double v) {
    double t = cbrt(1.0 - v), u = t * (double)s->n_inf;
    int64_t i = (int64_t)floor(u);
    if (i >= s->n_inf) i = s->n_inf - 1;
    double fr = u - (double)i;
    double sv = s->inf_s[i] + fr * (s->inf_s[i + 1] - s->inf_s[i]);
    return sv / v;
}

static void plane_waves(wo_ctx* c, wo_system* s, int sysid) {
    const int per = c->p.periodic;
    wo_stream cs;
    wo_stream_init(&cs, c->p.seed, sysid, c->sweep, TAG_PWCOUNT, 0, 0, 0, 0);
    double mu = (double)s->N * s->info.P_F;
    int64_t HF = (int64_t)floor(mu);
    if (wo_next_co(&cs) < mu - (double)HF) HF += 1;
    for (int64_t h = 0; h < HF; ++h) {
        c->obs.pw_chains++;
        wo_stream st;
        wo_stream_init(&st, c->p.seed, sysid, c->sweep, TAG_PW, 0, h, 0, 0);
        /* periodic: a lattice mode l (App. D "Choosing k for a periodic system");
         * infinite: |k| lambda_max = x from its tail probability, direction isotropic */
        int l[3] = {0, 0, 0};
        double x = 0.0, kh[3] = {0.0, 0.0, 0.0};
        if (per) {
            sample_k(c, s, &st, l);
        } else {
            x = inf_x_of_v(s, wo_next_oc(&st));
            draw_direction(&st, kh);
        }
        for (int r = 0;;) {
            double Phi = 2.0 * WO_PI * wo_next_co(&st);
            double psi = 2.0 * WO_PI * wo_next_co(&st);
            double u_acc = wo_next_oc(&st);
            int zero = per ? (l[0] == 0 && l[1] == 0 && l[2] == 0) : x == 0.0;
            if (zero) {
                /* k = 0: no displacement, deemed accepted (Sec. V "Choosing plane wave amplitude") */
                c->obs.pw_k0++;
                c->obs.pw_accepts++;
                s->accepted++;
                c->obs.accepted_total++;
                trace_push(c, 2, sysid, -1, h, 0, r, 0, 1, per ? (512 << 20) | (512 << 10) | 512 : 0, 0.0,
                           threshold(c, u_acc));
                break;
            }
            double k[3];
            int shell, extra;
            if (per) {
                double ks = 2.0 * WO_PI / s->L;
                for (int a = 0; a < 3; ++a) k[a] = ks * (double)l[a];
                double lm = sqrt(((double)l[0] * (double)l[0] + (double)l[1] * (double)l[1]) + (double)l[2] * (double)l[2]);
                shell = lm < WO_K_SHELLS - 1 ? (int)lm : WO_K_SHELLS - 1;
                extra = (int)((((uint32_t)(l[0] + 512) & 0x3FFu) << 20) | (((uint32_t)(l[1] + 512) & 0x3FFu) << 10) |
                              ((uint32_t)(l[2] + 512) & 0x3FFu));
            } else {
                double km = x / s->lmax;
                for (int a = 0; a < 3; ++a) k[a] = km * kh[a];
                shell = x < WO_K_SHELLS - 1 ? (int)x : WO_K_SHELLS - 1;
                extra = shell;
            }
            if (pw_attempt(c, s, sysid, h, r, k, shell, extra, Phi, psi, u_acc)) {
                s->accepted++;
                c->obs.accepted_total++;
                break;
            }
            if (++r >= c->p.retry_cap) { c->obs.pw_caps++; break; }
            /* recycling (App. D): keep |k|; periodic permutes and sign-flips l, infinite redraws
             * the direction; Phi and e-hat are redrawn either way */
            wo_stream_init(&st, c->p.seed, sysid, c->sweep, TAG_PW, 0, h, r, 0);
            if (per) {
                int pi = (int)wo_next_index(&st, 6);
                int nl[3] = {l[PERM[pi][0]], l[PERM[pi][1]], l[PERM[pi][2]]};
                for (int a = 0; a < 3; ++a) l[a] = wo_next_co(&st) < 0.5 ? -nl[a] : nl[a];
            } else {
                draw_direction(&st, kh);
            }
        }
    }
}

/* ------------------------------------------------------------------- sweep -------- */
static void sweep_system(wo_ctx* c, int sysid) {
    wo_system* s = &c->sys[sysid];
    for (int level = 0; c->p.wavelets && level < s->n_levels; ++level) {
        grid_t g;
        make_grid(c, s, sysid, level, &g);
        int64_t ncell = g.n[0] * g.n[1] * g.n[2];
        for (int colour = 0; colour < 8; ++colour) {
            for (int64_t cell = 0; cell < ncell; ++cell) {
                int64_t ic[3] = {cell % g.n[0], (cell / g.n[0]) % g.n[1], cell / (g.n[0] * g.n[1])};
                if (cell_colour(&g, ic) != colour) continue;
                process_cell(c, s, sysid, level, &g, cell, ic);
            }
        }
    }
    if (c->p.plane_waves) plane_waves(c, s, sysid);
}

int wo_sweep(void* vctx, int64_t n_sweeps) {
    wo_ctx* c = (wo_ctx*)vctx;
    for (int64_t k = 0; k < n_sweeps; ++k) {
        for (int sysid = 0; sysid < c->nsys; ++sysid) sweep_system(c, sysid);
        c->sweep++;
        c->obs.sweeps++;
    }
    return 0;
}

/* ------------------------------------------------------------------ setup --------- */
int wo_init(void** out, const wo_params* p, int32_t n_systems, const int64_t* sys_bead_offset,
            const double* sys_box_L, const double* sys_lambda_max, int64_t n_chains,
            const int64_t* chain_offset, const double* pos_xyz, int64_t trace_capacity) {
    *out = NULL;
    wo_ctx* c = (wo_ctx*)calloc(1, sizeof(wo_ctx));
    if (!c) return -1;
    c->p = *p;
    c->nsys = n_systems;
    c->N = sys_bead_offset[n_systems];
    int64_t N = c->N;
    c->x = (double*)malloc(sizeof(double) * N);
    c->y = (double*)malloc(sizeof(double) * N);
    c->z = (double*)malloc(sizeof(double) * N);
    c->nx = (double*)malloc(sizeof(double) * N);
    c->ny = (double*)malloc(sizeof(double) * N);
    c->nz = (double*)malloc(sizeof(double) * N);
    c->S = (int64_t*)malloc(sizeof(int64_t) * N);
    c->H = (int64_t*)malloc(sizeof(int64_t) * N);
    c->M = (int64_t*)malloc(sizeof(int64_t) * N);
    c->mark = (int64_t*)calloc(N, sizeof(int64_t));
    c->seen = (int64_t*)calloc(N, sizeof(int64_t));
    c->cnext = (int64_t*)malloc(sizeof(int64_t) * N);
    c->cprev = (int64_t*)malloc(sizeof(int64_t) * N);
    c->ccell = (int64_t*)malloc(sizeof(int64_t) * N);
    c->bond_next = (uint8_t*)calloc(N > 0 ? N : 1, 1);
    c->n_chains = n_chains;
    c->chain_off = (int64_t*)malloc(sizeof(int64_t) * (n_chains + 1));
    memcpy(c->chain_off, chain_offset, sizeof(int64_t) * (n_chains + 1));
    for (int64_t i = 0; i < N; ++i) {
        c->x[i] = pos_xyz[3 * i];
        c->y[i] = pos_xyz[3 * i + 1];
        c->z[i] = pos_xyz[3 * i + 2];
    }
    for (int64_t ch = 0; ch < n_chains; ++ch)
        for (int64_t i = chain_offset[ch]; i + 1 < chain_offset[ch + 1]; ++i) c->bond_next[i] = 1;
    c->trace_cap = trace_capacity;
    c->trace = trace_capacity > 0 ? (wo_trace_rec*)malloc(sizeof(wo_trace_rec) * trace_capacity) : NULL;
    c->rc2 = pow(2.0, 1.0 / 3.0) * p->sigma * p->sigma;
    double rc = p->wca ? pow(2.0, 1.0 / 6.0) * p->sigma : 0.0;
    if (p->bond_type == WO_BOND_FENE) c->r_int = p->R0 > rc ? p->R0 : rc;
    else if (p->bond_type == WO_BOND_HARMONIC) c->r_int = p->r_int_harmonic > rc ? p->r_int_harmonic : rc;
    else c->r_int = rc;
    c->sys = (wo_system*)calloc(n_systems, sizeof(wo_system));
    *out = c;
    if (!(p->band_ratio > 1.0 && p->band_ratio <= 2.0)) { strcpy(c->err, "band_ratio must lie in (1, 2]"); return -2; }
    if (!(p->lambda_min > 0.0)) { strcpy(c->err, "lambda_min must be positive"); return -2; }
    if (p->accept_rule < 0 || p->accept_rule > 1 || p->wavelet_map < 0 || p->wavelet_map > 1 ||
        p->centring < 0 || p->centring > 1) { strcpy(c->err, "bad variant selector"); return -2; }
    if (p->centring == WO_CENTRE_UNIFORM && !p->periodic) { strcpy(c->err, "uniform centring needs a periodic box"); return -2; }
    for (int si = 0; si < n_systems; ++si) {
        wo_system* s = &c->sys[si];
        s->b0 = sys_bead_offset[si];
        s->b1 = sys_bead_offset[si + 1];
        s->N = s->b1 - s->b0;
        s->L = sys_box_L ? sys_box_L[si] : p->box_L;
        s->lmax = sys_lambda_max ? sys_lambda_max[si] : p->lambda_max;
        if (!(s->lmax > p->lambda_min)) { strcpy(c->err, "lambda_max must exceed lambda_min"); return -2; }
        if (p->periodic && s->lmax > 0.5 * s->L) { strcpy(c->err, "lambda_max must not exceed L/2"); return -2; }
        /* systems with the same L/lambda_max share their plane-wave tables */
        /* periodic tables depend on L/lambda_max only; the infinite-system table on nothing */
        const wo_system* donor = NULL;
        for (int sj = 0; sj < si && p->plane_waves; ++sj)
            if (!p->periodic || c->sys[sj].L / c->sys[sj].lmax == s->L / s->lmax) { donor = &c->sys[sj]; break; }
        int rc_ = wo_build_system_tables(c, s, donor);
        if (rc_) return rc_;
        /* linked cells: side >= r_cut + 2 x the largest plane-wave amplitude (k = 2 pi / L) */
        s->nc = 0;
        s->head = NULL;
        if (p->periodic && p->wca) {
            double AFmax = p->plane_waves ? 2.0 * p->A0 / ((2.0 * WO_PI / s->L) * sqrt(5.0 * (double)s->N)) : 0.0;
            double side = sqrt(c->rc2) + 2.0 * AFmax + 1e-6;
            int nc = (int)floor(s->L / side);
            if (nc > 200) nc = 200;
            if (nc >= 3) {
                s->nc = nc;
                s->cg = s->L / nc;
                s->invcg = 1.0 / s->cg;
                s->head = (int64_t*)malloc(sizeof(int64_t) * (size_t)nc * nc * nc);
                cl_build(c, s);
            }
        }
        /* initial state must have finite energy */
        for (int64_t j = s->b0; j + 1 < s->b1; ++j) {
            if (!c->bond_next[j]) continue;
            double r2 = pair_r2(c, s, c->x[j], c->y[j], c->z[j], c->x[j + 1], c->y[j + 1], c->z[j + 1]);
            if (!isfinite(u_bond(c, r2))) { strcpy(c->err, "initial bond overstretched"); return -3; }
        }
    }
    return 0;
}

int wo_positions(void* vctx, double* out) {
    wo_ctx* c = (wo_ctx*)vctx;
    for (int64_t i = 0; i < c->N; ++i) {
        out[3 * i] = c->x[i];
        out[3 * i + 1] = c->y[i];
        out[3 * i + 2] = c->z[i];
    }
    return 0;
}

int wo_set_positions(void* vctx, const double* xyz) {
    wo_ctx* c = (wo_ctx*)vctx;
    for (int64_t i = 0; i < c->N; ++i) {
        c->x[i] = xyz[3 * i];
        c->y[i] = xyz[3 * i + 1];
        c->z[i] = xyz[3 * i + 2];
    }
    for (int si = 0; si < c->nsys; ++si) cl_build(c, &c->sys[si]);
    return 0;
}

int wo_set_sweep(void* vctx, int64_t sweep) {
    ((wo_ctx*)vctx)->sweep = sweep;
    return 0;
}

int wo_observables(void* vctx, wo_obs* out) {
    *out = ((wo_ctx*)vctx)->obs;
    return 0;
}

int wo_system_tau(void* vctx, double* out) {
    wo_ctx* c = (wo_ctx*)vctx;
    for (int i = 0; i < c->nsys; ++i) out[i] = c->sys[i].info.dt * (double)c->sys[i].accepted;
    return 0;
}

/* Eq. "Radius of gyration": <Rg^2> = (1/(2 Nb^2)) sum_i sum_j r_ij^2, unwrapped positions */
int wo_chain_rg2(void* vctx, double* out) {
    wo_ctx* c = (wo_ctx*)vctx;
    for (int64_t ch = 0; ch < c->n_chains; ++ch) {
        int64_t a = c->chain_off[ch], b = c->chain_off[ch + 1];
        double acc = 0.0;
        for (int64_t i = a; i < b; ++i)
            for (int64_t j = a; j < b; ++j) {
                double dx = c->x[i] - c->x[j], dy = c->y[i] - c->y[j], dz = c->z[i] - c->z[j];
                acc += (dx * dx + dy * dy) + dz * dz;
            }
        double nb = (double)(b - a);
        out[ch] = acc / (2.0 * nb * nb);
    }
    return 0;
}

int wo_chain_com(void* vctx, double* out) {
    wo_ctx* c = (wo_ctx*)vctx;
    for (int64_t ch = 0; ch < c->n_chains; ++ch) {
        int64_t a = c->chain_off[ch], b = c->chain_off[ch + 1];
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int64_t i = a; i < b; ++i) {
            sx += c->x[i];
            sy += c->y[i];
            sz += c->z[i];
        }
        double nb = (double)(b - a);
        out[3 * ch] = sx / nb;
        out[3 * ch + 1] = sy / nb;
        out[3 * ch + 2] = sz / nb;
    }
    return 0;
}

int wo_inf_table(void* vctx, int32_t system, double* out, int32_t max) {
    wo_system* s = &((wo_ctx*)vctx)->sys[system];
    if (!s->inf_s) return -1;
    int n = s->n_inf + 1 < max ? s->n_inf + 1 : max;
    memcpy(out, s->inf_s, sizeof(double) * n);
    return s->n_inf + 1;
}

double wo_inf_k_of_v(void* vctx, int32_t system, double v) {
    wo_system* s = &((wo_ctx*)vctx)->sys[system];
    return s->inf_s ? inf_x_of_v(s, v) : NAN;
}

int64_t wo_trace(void* vctx, wo_trace_rec* out, int64_t max) {
    wo_ctx* c = (wo_ctx*)vctx;
    int64_t n = c->trace_n < max ? c->trace_n : max;
    memcpy(out, c->trace, sizeof(wo_trace_rec) * n);
    c->trace_n = 0;
    return n;
}

int wo_get_level_info(void* vctx, int32_t system, wo_level_info* out, int32_t max) {
    wo_ctx* c = (wo_ctx*)vctx;
    wo_system* s = &c->sys[system];
    int n = s->n_levels < max ? s->n_levels : max;
    memcpy(out, s->lev, sizeof(wo_level_info) * n);
    return s->n_levels;
}

int wo_get_system_info(void* vctx, int32_t system, wo_system_info* out) {
    *out = ((wo_ctx*)vctx)->sys[system].info;
    return 0;
}

int wo_cell_ids(void* vctx, int32_t system, int64_t sweep, int32_t level, int32_t* out) {
    wo_ctx* c = (wo_ctx*)vctx;
    wo_system* s = &c->sys[system];
    int64_t keep = c->sweep;
    c->sweep = sweep;
    grid_t g;
    make_grid(c, s, system, level, &g);
    c->sweep = keep;
    for (int64_t j = s->b0; j < s->b1; ++j) out[j - s->b0] = (int32_t)cell_of_point(&g, c->x[j], c->y[j], c->z[j]);
    return 0;
}

int wo_cube_weights(void* vctx, int32_t system, double* out) {
    wo_ctx* c = (wo_ctx*)vctx;
    wo_system* s = &c->sys[system];
    if (!s->cube_w) return -1;
    memcpy(out, s->cube_w, sizeof(double) * s->info.n_modes);
    return s->info.n_modes;
}

int wo_shell_table(void* vctx, int32_t system, double* out, int32_t max) {
    wo_ctx* c = (wo_ctx*)vctx;
    wo_system* s = &c->sys[system];
    if (!s->shell_s) return -1;
    int n = s->n_shell + 1 < max ? s->n_shell + 1 : max;
    memcpy(out, s->shell_s, sizeof(double) * n);
    return s->n_shell + 1;
}

const char* wo_last_error(void* vctx) { return vctx ? ((wo_ctx*)vctx)->err : "no context"; }

void wo_free(void* vctx) {
    wo_ctx* c = (wo_ctx*)vctx;
    if (!c) return;
    for (int i = 0; i < c->nsys; ++i) {
        wo_free_system_tables(&c->sys[i]);
        free(c->sys[i].head);
    }
    free(c->seen); free(c->cnext); free(c->cprev); free(c->ccell);
    free(c->sys);
    free(c->x); free(c->y); free(c->z);
    free(c->nx); free(c->ny); free(c->nz);
    free(c->S); free(c->H); free(c->M); free(c->mark);
    free(c->bond_next); free(c->chain_off); free(c->trace);
    free(c);
}
