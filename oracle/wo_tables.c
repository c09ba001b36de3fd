/*
 * Oracle: random numbers, the tapered-wavelet transforms and the per-system schedule
 * constants (test infrastructure only).
 *
 * Pinned in tests/test_oracle_*.py against the Philox known-answer vectors, the closed
 * forms M3, M4, M6 and lambda_a, scipy quadrature of I(x), P(k=0), R -> 1 and the
 * finite-box self-mobility 1 - 2.837 a/L.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "wo_internal.h"

/* ------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its definition:
 * each round multiplies counter words 0 and 2 by fixed odd constants, swaps the
 * high/low halves into a new counter mixed with the other two words and the key,
 * and the key is bumped by two Weyl constants between rounds.
 * ---------------------------------------------------------------------------------- */
void wo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter layout of a stream, identical in the HIP library:
 *   c0 = (r << 24) | (j << 12) | block,  c1 = (system << 20) | t,
 *   c2 = (tag << 24) | cell,             c3 = sweep,   key = seed (lo, hi). */
void wo_stream_init(wo_stream* s, uint64_t seed, int32_t system, int64_t sweep, int32_t tag,
                    int64_t cell, int64_t t, int32_t r, int32_t j) {
    s->ctr[0] = ((uint32_t)(r & 0xFF) << 24) | ((uint32_t)(j & 0xFFF) << 12);
    s->ctr[1] = ((uint32_t)(system & 0xFFF) << 20) | (uint32_t)(t & 0xFFFFF);
    s->ctr[2] = ((uint32_t)(tag & 0xFF) << 24) | (uint32_t)(cell & 0xFFFFFF);
    s->ctr[3] = (uint32_t)sweep;
    s->key[0] = (uint32_t)seed;
    s->key[1] = (uint32_t)(seed >> 32);
    s->next = 0;
    s->cached = -1;
}

uint64_t wo_next_bits(wo_stream* s) {
    uint32_t i = s->next++;
    int64_t blk = (int64_t)((i >> 1) & 0xFFFu);
    if (blk != s->cached) {
        uint32_t c[4] = {s->ctr[0] | (uint32_t)blk, s->ctr[1], s->ctr[2], s->ctr[3]};
        wo_philox4x32_10(c, s->key, s->w);
        s->cached = blk;
    }
    uint32_t hi = s->w[2 * (i & 1)], lo = s->w[2 * (i & 1) + 1];
    return ((uint64_t)hi << 21) | ((uint64_t)lo >> 11);
}

double wo_next_co(wo_stream* s) { return (double)wo_next_bits(s) * 0x1.0p-53; }
double wo_next_oc(wo_stream* s) { return ((double)wo_next_bits(s) + 1.0) * 0x1.0p-53; }
int64_t wo_next_index(wo_stream* s, int64_t n) {
    unsigned __int128 prod = (unsigned __int128)wo_next_bits(s) * (unsigned __int128)(uint64_t)n;
    return (int64_t)(prod >> 53);
}

void wo_stream_doubles(uint64_t seed, int32_t system, int64_t sweep, int32_t tag, int64_t cell,
                       int64_t t, int32_t r, int32_t j, int32_t n, double* out_co, double* out_oc) {
    wo_stream s;
    wo_stream_init(&s, seed, system, sweep, tag, cell, t, r, j);
    for (int32_t i = 0; i < n; ++i) {
        uint64_t m = wo_next_bits(&s);
        if (out_co) out_co[i] = (double)m * 0x1.0p-53;
        if (out_oc) out_oc[i] = ((double)m + 1.0) * 0x1.0p-53;
    }
}

/* ------------------------------------------------------------------------------------
 * lambda from its PDF ~ lambda^-4 on one band [lo, hi) (Eq. "PDF for lambda" and the
 * inverse transform of App. D with the band edges in place of lambda_min, lambda_max):
 *   lambda = lo * (1 + u [(lo/hi)^3 - 1])^(-1/3).
 * The cube root decides the centre b and hence its cell, so it is computed without libm:
 * Newton's iteration y <- y (4 - x y^3) / 3 for y = x^(-1/3), x in [1/8, 1], from the
 * straight line through (1/8, 2) and (1, 1), a fixed 8 steps.
 * ---------------------------------------------------------------------------------- */
double wo_inv_cbrt(double x) {
    double y = 2.0 - (x - 0.125) * (8.0 / 7.0);
    for (int it = 0; it < 8; ++it) {
        double y3 = y * y * y;
        y = y * (4.0 - x * y3) / 3.0;
    }
    return y;
}

double wo_draw_lambda(double u, double lo, double hi) {
    double cr = lo / hi;
    double c = cr * cr * cr;
    double x = 1.0 + u * (c - 1.0);
    return lo * wo_inv_cbrt(x);
}

/* ------------------------------------------------------------------------------------
 * Tapered wavelet (Eqs. "Tapered wavelet", "Scalar wavelet position/Fourier"):
 *   w(x, p) = (1 - |x|) p x x for |x| <= 1, 0 outside;
 *   phi~(q) = 4 pi q^-6 (5 q sin q - (q^2 - 8) cos q - 8).
 * For q < 3 phi~ is summed from its Taylor series, the radial transform
 * 4 pi int_0^1 r^2 phi(r) sin(qr)/(qr) dr term by term, which avoids the cancellation
 * of the closed form at small q.
 * ---------------------------------------------------------------------------------- */
void wo_wavelet(const double x[3], const double p[3], double out[3]) {
    double rr = sqrt((x[0] * x[0] + x[1] * x[1]) + x[2] * x[2]);
    double f = rr < 1.0 ? (1.0 - rr) : 0.0;
    out[0] = f * (p[1] * x[2] - p[2] * x[1]);
    out[1] = f * (p[2] * x[0] - p[0] * x[2]);
    out[2] = f * (p[0] * x[1] - p[1] * x[0]);
}

double wo_phit(double q) {
    if (q < 3.0) {
        double q2 = q * q, term = 1.0, acc = 0.0;
        for (int n = 0; n < 30; ++n) {
            /* term = (-1)^n q^(2n) / (2n+1)! */
            double mom = 1.0 / (2.0 * (2 * n + 5)) - 1.0 / (3.0 * (2 * n + 6)) - 1.0 / (6.0 * (2 * n + 3));
            acc += mom * term;
            term *= -q2 / ((2.0 * n + 2.0) * (2.0 * n + 3.0));
        }
        return 4.0 * WO_PI * acc;
    }
    double q2 = q * q, q6 = q2 * q2 * q2;
    return 4.0 * WO_PI * (5.0 * q * sin(q) - (q2 - 8.0) * cos(q) - 8.0) / q6;
}

/* moments M_m = int_0^inf k^m phi~(k)^2 dk (Eq. "phi moment"); closed forms of the
 * tapered wavelet, re-derived by quadrature in the tests */
double wo_M(int m) {
    if (m == 3) return 2.0 * WO_PI * WO_PI / 105.0 * (9.0 - 8.0 * log(2.0));
    if (m == 4) return 8.0 * WO_PI * WO_PI * WO_PI / 105.0;
    if (m == 6) return 8.0 * WO_PI * WO_PI * WO_PI / 5.0;
    return NAN;
}

/* ------------------------------------------------------------------------------------
 * I(x) = int_x^inf q^3 phi~(q)^2 dq (Eqs. "Oseen_w FT", "Prob of k_l") and
 * J6(x) = int_x^inf q^6 phi~(q)^2 dq, by 16-point Gauss-Legendre on panels of width
 * 1/4 up to Q = 4096 plus the asymptotic tails
 *   I: 2 pi^2 Q^-4,   J6: 8 pi^2/Q - 4 pi^2 sin(2Q)/Q^2 + (24 - 36 cos 2Q) pi^2/Q^3.
 * ---------------------------------------------------------------------------------- */
#define WO_QP 0.25
#define WO_QMAX 4096.0
#define WO_NPAN 16384
static double gl_x[16], gl_w[16];
static double* suffix_I = NULL;   /* int_{i*QP}^{QMAX} */
static double* suffix_J = NULL;

static void gauss_legendre_16(void) {
    const int n = 16;
    for (int i = 0; i < n; ++i) {
        double z = cos(WO_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int k = 1; k <= n; ++k) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * k - 1.0) * z * p2 - (k - 1.0) * p3) / k;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double dz = p1 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        gl_x[i] = z;
        gl_w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

static void panel(double a, double b, double* vi, double* vj) {
    double mid = 0.5 * (a + b), half = 0.5 * (b - a), si = 0.0, sj = 0.0;
    for (int i = 0; i < 16; ++i) {
        double q = mid + half * gl_x[i];
        double f = wo_phit(q);
        double q3 = q * q * q;
        si += gl_w[i] * q3 * f * f;
        sj += gl_w[i] * q3 * q3 * f * f;
    }
    *vi = si * half;
    *vj = sj * half;
}

static void quad_tables(void) {
    if (suffix_I) return;
    gauss_legendre_16();
    double* sI = (double*)malloc(sizeof(double) * (WO_NPAN + 1));
    double* sJ = (double*)malloc(sizeof(double) * (WO_NPAN + 1));
    sI[WO_NPAN] = 0.0;
    sJ[WO_NPAN] = 0.0;
    for (int i = WO_NPAN - 1; i >= 0; --i) {
        double vi, vj;
        panel(i * WO_QP, (i + 1) * WO_QP, &vi, &vj);
        sI[i] = sI[i + 1] + vi;
        sJ[i] = sJ[i + 1] + vj;
    }
    suffix_J = sJ;
    suffix_I = sI;
}

static double tail_I(double Q) { return 2.0 * WO_PI * WO_PI / (Q * Q * Q * Q); }
static double tail_J(double Q) {
    double pi2 = WO_PI * WO_PI;
    return 8.0 * pi2 / Q - 4.0 * pi2 * sin(2.0 * Q) / (Q * Q) +
           (24.0 - 36.0 * cos(2.0 * Q)) * pi2 / (Q * Q * Q);
}

double wo_I(double x) {
    quad_tables();
    if (x >= WO_QMAX) return tail_I(x);
    int i = (int)floor(x / WO_QP);
    double vi = 0.0, vj = 0.0, top = (i + 1) * WO_QP;
    if (top > x) panel(x, top, &vi, &vj);
    return vi + suffix_I[i + 1] + tail_I(WO_QMAX);
}

double wo_J6(double x) {
    quad_tables();
    if (x >= WO_QMAX) return tail_J(x);
    int i = (int)floor(x / WO_QP);
    double vi = 0.0, vj = 0.0, top = (i + 1) * WO_QP;
    if (top > x) panel(x, top, &vi, &vj);
    return vj + suffix_J[i + 1] + tail_J(WO_QMAX);
}

/* G(x) = int_x^inf t^2 I(t) dt = (J6(x) - x^3 I(x)) / 3 (integration by parts) */
double wo_G(double x) {
    quad_tables();
    double I, J;
    if (x >= WO_QMAX) {
        I = tail_I(x);
        J = tail_J(x);
    } else {
        int i = (int)floor(x / WO_QP);
        double vi = 0.0, vj = 0.0, top = (i + 1) * WO_QP;
        if (top > x) panel(x, top, &vi, &vj);
        I = vi + suffix_I[i + 1] + tail_I(WO_QMAX);
        J = vj + suffix_J[i + 1] + tail_J(WO_QMAX);
    }
    return (J - x * x * x * I) / 3.0;
}

double wo_u_fene(double r2, double k, double R0) {
    double R02 = R0 * R0;
    if (r2 >= R02) return INFINITY;
    return -0.5 * k * R02 * log(1.0 - r2 / R02);
}

double wo_u_wca(double r2, double sigma, double eps) {
    double rc2 = pow(2.0, 1.0 / 3.0) * sigma * sigma;
    if (r2 >= rc2) return 0.0;
    if (r2 <= 0.0) return INFINITY;
    double s2 = sigma * sigma / r2;
    double s6 = s2 * s2 * s2;
    return 4.0 * eps * (s6 * s6 - s6 + 0.25);
}

/* ------------------------------------------------------------------------------------
 * Per-system schedule constants.
 *  levels: bands [lo, hi) with lo_0 = lambda_min, hi = min(lo*band_ratio, lambda_max);
 *          p_l = (lo^-3 - hi^-3)/(lambda_min^-3 - lambda_max^-3) (Eq. "PDF for lambda");
 *          T_l = N (1 - P_F) p_l expected chain starts per sweep;
 *          periodic cell count: the largest even n with L/n >= (2 hi + r_int)(1+1e-9),
 *          else 1.
 *  P_F:    Eq. "P(Fourier)" with R = (L/lmax)^3 M6 N_k / (6 pi^2) and N_k = 1/W_tot,
 *          W_tot = sum over the cube of I(|k_l| lmax) + quasi-continuous shell outside the
 *          cube (continuum integral beyond k_s = (2pi/L)(N_layers + 1/2) minus the cube's
 *          corner modes beyond k_s).
 *          Infinite system: P_F = (lambda_min/lambda_max)^3 (Eq. "P(Fourier) infinite").
 *  dt:     Eq. "dt w+F" with plane waves; Eq. "Time step per wavelet" without.
 * ---------------------------------------------------------------------------------- */
int wo_build_system_tables(wo_ctx* c, wo_system* s, const wo_system* donor) {
    const wo_params* p = &c->p;
    double lmin = p->lambda_min, lmax = s->lmax;
    double N = (double)s->N;
    wo_system_info* info = &s->info;
    memset(info, 0, sizeof(*info));
    double M3 = wo_M(3), M4 = wo_M(4), M6 = wo_M(6);
    double lam_a = 2.0 / WO_PI * M4 / M3;
    double twopi3 = 8.0 * WO_PI * WO_PI * WO_PI;

    /* plane-wave tables */
    double PF = 0.0;
    s->cube_w = s->cube_cdf = s->shell_s = NULL;
    if (p->periodic && p->plane_waves && donor) {
        /* the plane-wave tables depend on L/lambda_max only: copy them */
        int64_t nm = donor->info.n_modes;
        s->cube_w = (double*)malloc(sizeof(double) * nm);
        s->cube_cdf = (double*)malloc(sizeof(double) * nm);
        s->shell_s = (double*)malloc(sizeof(double) * (donor->n_shell + 1));
        memcpy(s->cube_w, donor->cube_w, sizeof(double) * nm);
        memcpy(s->cube_cdf, donor->cube_cdf, sizeof(double) * nm);
        memcpy(s->shell_s, donor->shell_s, sizeof(double) * (donor->n_shell + 1));
        s->n_shell = donor->n_shell;
        s->x_s = donor->x_s;
        *info = donor->info;
        double rat = lmax / lmin;
        PF = 1.0 / (1.0 + info->R * (rat * rat * rat - 1.0));
    } else if (p->periodic && p->plane_waves) {
        int NL = p->n_layers, D = 2 * NL + 1;
        int64_t nm = (int64_t)D * D * D;
        double L = s->L, ks = 2.0 * WO_PI / L;
        s->cube_w = (double*)malloc(sizeof(double) * nm);
        s->cube_cdf = (double*)malloc(sizeof(double) * nm);
        double Wc = 0.0, Wcorner = 0.0, edge2 = (NL + 0.5) * (NL + 0.5);
        /* I depends on |l|^2 only: evaluate once per value */
        int maxl2 = 3 * NL * NL;
        double* Il2 = (double*)malloc(sizeof(double) * (maxl2 + 1));
        for (int v = 0; v <= maxl2; ++v) Il2[v] = wo_I(ks * sqrt((double)v) * lmax);
        int64_t i = 0;
        for (int lx = -NL; lx <= NL; ++lx)
            for (int ly = -NL; ly <= NL; ++ly)
                for (int lz = -NL; lz <= NL; ++lz, ++i) {
                    int l2 = lx * lx + ly * ly + lz * lz;
                    double w = Il2[l2];
                    s->cube_w[i] = w;
                    Wc += w;
                    s->cube_cdf[i] = Wc;
                    if ((double)l2 > edge2) Wcorner += w;
                }
        free(Il2);
        double xs = ks * (NL + 0.5) * lmax;
        double Lk = L / (2.0 * WO_PI);
        double Wcont = Lk * Lk * Lk * (4.0 * WO_PI / (lmax * lmax * lmax)) * wo_G(xs);
        double Wtot = Wc + Wcont - Wcorner;
        double Nk = 1.0 / Wtot;
        double R = (L / lmax) * (L / lmax) * (L / lmax) * M6 * Nk / (6.0 * WO_PI * WO_PI);
        double rat = lmax / lmin;
        PF = 1.0 / (1.0 + R * (rat * rat * rat - 1.0));
        info->R = R;
        info->N_k = Nk;
        info->W_cube = Wc;
        info->W_cont = Wcont;
        info->W_corner = Wcorner;
        info->P_cube = Wc / Wtot;
        info->P_k0 = wo_I(0.0) * Nk;
        info->n_modes = (int32_t)nm;
        s->x_s = xs;
        /* shell: s = x_s/x tabulated at u_i = i/M, where u = 1 - G(x)/G(x_s) */
        int M = 4096;
        s->n_shell = M;
        s->shell_s = (double*)malloc(sizeof(double) * (M + 1));
        double G0 = wo_G(xs);
        s->shell_s[0] = 1.0;
        s->shell_s[M] = 0.0;
        for (int k = 1; k < M; ++k) {
            double target = (1.0 - (double)k / M) * G0;
            double a = 0.0, b = s->shell_s[k - 1];
            for (int it = 0; it < 60; ++it) {
                double m = 0.5 * (a + b);
                if (m <= 0.0 || wo_G(xs / m) < target) a = m; else b = m;
            }
            s->shell_s[k] = 0.5 * (a + b);
        }
    }
    s->inf_s = NULL;
    s->n_inf = 0;
    if (!p->periodic && p->plane_waves && donor) {
        double q = lmin / lmax;
        PF = q * q * q;
        s->n_inf = donor->n_inf;
        s->inf_s = (double*)malloc(sizeof(double) * (s->n_inf + 1));
        memcpy(s->inf_s, donor->inf_s, sizeof(double) * (s->n_inf + 1));
        info->N_k = 3.0 * lmax * lmax * lmax / M6;
        info->R = 1.0;
    } else if (!p->periodic && p->plane_waves) {
        /* Infinite system (Sec. V "Distributions of wavevectors"): P(k) = N_k k^2 I(k lmax) with
         * N_k = 3 lmax^3 / M6 (Eq. "k normalisation infinite"), so x = k lmax has the tail
         * probability v(x) = G(x) / G(0), G(0) = M6 / 3. The inverse (App. D: a table of
         * pre-calculated values, interpolated) is kept as s = x v at t = i/M with v = 1 - t^3:
         * s is smooth in t at both ends (x grows like t from 0, and x v -> 2 pi^2 / G(0) as
         * v -> 0 because I(x) ~ 2 pi^2 x^-4). A plane wave is made with the probability of a
         * wavelet above lmax, P_F = (lmin/lmax)^3 (Eq. "P(Fourier) infinite"). */
        double q = lmin / lmax;
        PF = q * q * q;
        int M = 4096;
        s->n_inf = M;
        s->inf_s = (double*)malloc(sizeof(double) * (M + 1));
        double G0 = wo_G(0.0), xprev = 0.0;
        s->inf_s[0] = 0.0;
        for (int i = 1; i < M; ++i) {
            double t = (double)i / M, v = 1.0 - t * t * t, target = v * G0;
            double a = xprev, b = xprev + 1.0;
            while (wo_G(b) > target) b *= 2.0;
            for (int it = 0; it < 80; ++it) {
                double m = 0.5 * (a + b);
                if (wo_G(m) > target) a = m; else b = m;
            }
            xprev = 0.5 * (a + b);
            s->inf_s[i] = xprev * v;
        }
        s->inf_s[M] = 2.0 * WO_PI * WO_PI / G0;
        info->N_k = 3.0 * lmax * lmax * lmax / M6;
        info->R = 1.0;
    }
    info->P_F = PF;

    /* time step per accepted move */
    double dt = 6.0 * p->A0 * p->A0 * M4 * lam_a * lam_a / (twopi3 * N);
    if (!p->plane_waves) {
        double q = lmin / lmax;
        dt *= (1.0 - q) / (1.0 - q * q * q);
    }
    info->dt = dt;

    /* levels */
    double norm = 1.0 / (lmin * lmin * lmin) - 1.0 / (lmax * lmax * lmax);
    double lo = lmin;
    int nl = 0;
    while (nl < WO_MAX_LEVELS) {
        double hi = lo * p->band_ratio;
        int last = 0;
        if (hi > lmax || lmax - hi < 1e-9 * lmax) { hi = lmax; last = 1; }
        wo_level_info* L = &s->lev[nl];
        memset(L, 0, sizeof(*L));
        L->lo = lo;
        L->hi = hi;
        L->p = (1.0 / (lo * lo * lo) - 1.0 / (hi * hi * hi)) / norm;
        L->T = N * (1.0 - PF) * L->p;
        L->r_int = c->r_int;
        if (p->periodic) {
            int n = (int)floor(s->L / ((2.0 * hi + c->r_int) * (1.0 + 1e-9)));
            if (n % 2) n -= 1;
            if (n < 2) n = 1;
            L->ncell = n;
            L->h = s->L / n;
        } else {
            L->ncell = 0;
            L->h = (2.0 * hi + c->r_int) * (1.0 + 1e-9);
        }
        ++nl;
        if (last) break;
        lo = hi;
    }
    if (nl == WO_MAX_LEVELS && s->lev[nl - 1].hi < lmax) {
        strcpy(c->err, "too many levels: raise band_ratio");
        return -1;
    }
    s->n_levels = nl;
    info->n_levels = nl;
    return 0;
}

void wo_free_system_tables(wo_system* s) {
    free(s->cube_w);
    free(s->cube_cdf);
    free(s->shell_s);
    free(s->inf_s);
    s->cube_w = s->cube_cdf = s->shell_s = s->inf_s = NULL;
}
