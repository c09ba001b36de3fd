// Device side of libwmc: the Wavelet Monte Carlo dynamics sweep on gfx950.
//
// One sweep (Dyer & Ball, arXiv:1611.09160, Sec. IV-V, App. D), per system:
//   for each wavelet level band (ascending lambda):
//     rebuild the neighbour grid (counting sort of beads into cells of side >= r_cut + skin);
//     for colour 0..7: one workgroup per cell of that colour (k_phase). Cells of one colour are
//     at least 2 lambda_hi + r_int apart, so their moves touch disjoint beads and halos and run
//     concurrently with the same result as any serial order.
//   plane-wave chains (k_pw), one workgroup per system.
// Beads are SoA FP64 in HBM; every workgroup reads and writes them directly (write-through),
// keeping its cell's reach list, member list and member trial positions in LDS.
// All schedule-deciding arithmetic (cells, reach lists, anchors, lambda, centres, member
// tests) uses only IEEE add/mul/div/sqrt/floor/rint with contraction off.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>
#include <algorithm>
#include <mutex>
#include <type_traits>
#include "wmc_internal.h"

namespace wmc {

// ------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 multiplies mixing the
// four counter words with the key; the key is bumped by two Weyl constants between rounds.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t lo0 = 0xD2511F53u * c[0];
        uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
        uint32_t lo1 = 0xCD9E8D57u * c[2];
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// A stream is the sequence of doubles of one counter prefix:
//   c0 = (r << 24) | (j << 12) | block, c1 = (system << 20) | t, c2 = (tag << 24) | cell,
//   c3 = sweep; double i uses words 2(i&1), 2(i&1)+1 of block i>>1 (53 bits).
struct Stream {
    uint32_t c0, c1, c2, c3, k0, k1;
    uint32_t next;
    int32_t cached;
    uint32_t w[4];
    __device__ void init(const DevParams& P, int sys, int64_t sweep, int tag, int64_t cell, int64_t t, int r, int j) {
        c0 = ((uint32_t)(r & 0xFF) << 24) | ((uint32_t)(j & 0xFFF) << 12);
        c1 = ((uint32_t)(sys & 0xFFF) << 20) | (uint32_t)(t & 0xFFFFF);
        c2 = ((uint32_t)(tag & 0xFF) << 24) | (uint32_t)(cell & 0xFFFFFF);
        c3 = (uint32_t)sweep;
        k0 = P.seed_lo;
        k1 = P.seed_hi;
        next = 0;
        cached = -1;
    }
    __device__ uint64_t bits() {
        uint32_t i = next++;
        int32_t blk = (int32_t)((i >> 1) & 0xFFFu);
        if (blk != cached) {
            w[0] = c0 | (uint32_t)blk;
            w[1] = c1;
            w[2] = c2;
            w[3] = c3;
            philox10(w, k0, k1);
            cached = blk;
        }
        uint32_t hi = (i & 1) ? w[2] : w[0];
        uint32_t lo = (i & 1) ? w[3] : w[1];
        return ((uint64_t)hi << 21) | ((uint64_t)lo >> 11);
    }
    __device__ double co() { return (double)bits() * 0x1.0p-53; }
    __device__ double oc() { return ((double)bits() + 1.0) * 0x1.0p-53; }
    __device__ int64_t index(int64_t n) { return (int64_t)__umul64hi(bits() << 11, (uint64_t)n); }
};

// x^(-1/3) on [1/8, 1] by a fixed 8 Newton steps y <- y (4 - x y^3)/3 from the line through
// (1/8, 2) and (1, 1); no libm, so lambda (and the centre's cell) is bit-reproducible.
__device__ __forceinline__ double inv_cbrt(double x) {
    double y = 2.0 - (x - 0.125) * (8.0 / 7.0);
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        double y3 = y * y * y;
        y = y * (4.0 - x * y3) / 3.0;
    }
    return y;
}

// lambda in [lo, hi) with PDF ~ lambda^-4 (inverse transform of App. D with band edges)
__device__ __forceinline__ double draw_lambda(double u, double lo, double hi) {
    double cr = lo / hi;
    double c = cr * cr * cr;
    double x = 1.0 + u * (c - 1.0);
    return lo * inv_cbrt(x);
}

__device__ __forceinline__ void ball(Stream& s, double& vx, double& vy, double& vz) {
    double ss;
    do {
        vx = 2.0 * s.co() - 1.0;
        vy = 2.0 * s.co() - 1.0;
        vz = 2.0 * s.co() - 1.0;
        ss = (vx * vx + vy * vy) + vz * vz;
    } while (ss > 1.0);
}

__device__ __forceinline__ void direction(Stream& s, double& px, double& py, double& pz) {
    double vx, vy, vz, ss;
    do {
        vx = 2.0 * s.co() - 1.0;
        vy = 2.0 * s.co() - 1.0;
        vz = 2.0 * s.co() - 1.0;
        ss = (vx * vx + vy * vy) + vz * vz;
    } while (ss > 1.0 || ss == 0.0);
    double nrm = sqrt(ss);
    px = vx / nrm;
    py = vy / nrm;
    pz = vz / nrm;
}

// ------------------------------------------------------------------------------ energies
// FENE (Eq. "FENE potential"), harmonic (zero rest length), WCA (Eq. "WCA potential")
__device__ __forceinline__ double u_bond(const DevParams& P, double r2) {
    if (P.bond_type == WMC_BOND_FENE) {
        if (r2 >= P.R02) return INFINITY;
        return -0.5 * P.k_bond * P.R02 * log(1.0 - r2 / P.R02);
    }
    if (P.bond_type == WMC_BOND_HARMONIC) return 0.5 * P.k_bond * r2;
    return 0.0;
}
// U_bond(r2n) - U_bond(r2o) of one bond; for FENE one logarithm of the ratio of the two
// (R0^2 - r^2) factors instead of two logarithms (equal up to rounding)
__device__ __forceinline__ double u_bond_delta(const DevParams& P, double r2n, double r2o) {
    if (P.bond_type == WMC_BOND_FENE) {
        if (r2n >= P.R02 || r2o >= P.R02) return u_bond(P, r2n) - u_bond(P, r2o);
        return -0.5 * P.k_bond * P.R02 * log((P.R02 - r2n) / (P.R02 - r2o));
    }
    if (P.bond_type == WMC_BOND_HARMONIC) return 0.5 * P.k_bond * (r2n - r2o);
    return 0.0;
}
__device__ __forceinline__ double u_pair(const DevParams& P, double r2) {
    if (r2 >= P.rc2) return 0.0;
    if (r2 <= 0.0) return INFINITY;
    double s2 = P.sigma2 / r2;
    double s6 = s2 * s2 * s2;
    return 4.0 * P.eps * (s6 * s6 - s6 + 0.25);
}

// Acceptance threshold on dU for a uniform u in (0, 1]: Metropolis (Eq. "Metropolis test") accepts
// iff dU <= -kT ln u, probability min(1, e^(-dU/kT)); Glauber iff dU <= kT ln((1 - u)/u), probability
// 1/(1 + e^(dU/kT)) (1 - u is exact for u = m 2^-53)
// VAR = false compiles the paper's defaults only (no register cost for the variants)
template <bool VAR>
__device__ __forceinline__ double accept_threshold(const DevParams& P, double u) {
    if (VAR && P.accept_rule == WMC_ACCEPT_GLAUBER) return P.kT * (log(1.0 - u) - log(u));
    return -P.kT * log(u);
}

// FP32 terms from an FP32 r2 (FP32 tile, mixed precision) with their sensitivity: sens bounds |r2 dU/dr2| and |U| of the term (for
// WCA 6 s^12 + 3 s^6 >= |s^12 - s^6 + 1/4| inside the cut-off; for FENE r2/(R0^2 - r2) R0^2/2 >=
// -ln(1 - r2/R0^2) R0^2/2 times x ln x/(x - 1) <= 1), so that one margin covers both the error
// of r2 and the rounding of the term.
__device__ __forceinline__ float u_bond_f32(const DevParams& P, float r2, float& sens) {
    if (P.bond_type == WMC_BOND_FENE) {
        const float R02 = (float)P.R02, x = 1.0f - r2 / R02;
        if (!(x > 0.0f)) {
            sens = INFINITY;
            return INFINITY;
        }
        sens = 0.5f * (float)P.k_bond * r2 / x;
        return -0.5f * (float)P.k_bond * R02 * logf(x);
    }
    if (P.bond_type == WMC_BOND_HARMONIC) {
        sens = 0.5f * (float)P.k_bond * r2;
        return sens;
    }
    sens = 0.0f;
    return 0.0f;
}
__device__ __forceinline__ float u_pair_f32(const DevParams& P, float r2, float rc2f, float& sens) {
    if (r2 >= rc2f) {
        sens = 0.0f;
        return 0.0f;
    }
    if (r2 <= 0.0f) {
        sens = INFINITY;
        return INFINITY;
    }
    // the hardware reciprocal (1 ulp): its error is one more rounding within the margin's S1 share
    const float s2 = (float)P.sigma2 * __builtin_amdgcn_rcpf(r2), s6 = s2 * s2 * s2, e4 = 4.0f * (float)P.eps;
    sens = e4 * (6.0f * s6 * s6 + 3.0f * s6);
    return e4 * (s6 * s6 - s6 + 0.25f);
}

// ------------------------------------------------------------------------------ geometry
struct Grid {
    double o[3];
    double h, invh, half, L, invL;
    int64_t n[3];
    int64_t k0[3];  // infinite system: lattice index of local cell 0 along each axis
    int periodic;
};

// Colour parity of local cell 0: cells are coloured by the parity of their lattice index, which in an
// infinite system starts at k0 (a periodic grid starts at 0)
__device__ __forceinline__ int grid_parity(const Grid& g) {
    return (int)((g.k0[0] & 1) | ((g.k0[1] & 1) << 1) | ((g.k0[2] & 1) << 2));
}

// Stream key of a cell: its index in a periodic grid, or its lattice index modulo 256 per axis in an
// infinite system, so that neither the colours nor the random streams depend on the positions
__device__ __forceinline__ int64_t cell_key(const Grid& g, const int64_t ic[3]) {
    if (g.periodic) return ic[0] + g.n[0] * (ic[1] + g.n[1] * ic[2]);
    return ((g.k0[0] + ic[0]) & 255) | (((g.k0[1] + ic[1]) & 255) << 8) | (((g.k0[2] + ic[2]) & 255) << 16);
}

__device__ __forceinline__ double minimg(const Grid& g, double d) {
    return g.periodic ? d - g.L * rint(d * g.invL) : d;
}

__device__ int64_t cell_of_point(const Grid& g, double bx, double by, double bz) {
    double b[3] = {bx, by, bz};
    int64_t ic[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double v = b[a];
        if (g.periodic) v = v - g.L * floor(v * g.invL);
        int64_t i = (int64_t)floor((v - g.o[a]) * g.invh);
        if (g.periodic) {
            i %= g.n[a];
            if (i < 0) i += g.n[a];
        } else if (i < 0 || i >= g.n[a]) {
            return -1;
        }
        ic[a] = i;
    }
    return ic[0] + g.n[0] * (ic[1] + g.n[1] * ic[2]);
}

__device__ __forceinline__ double dist2_cell(const Grid& g, const int64_t ic[3], double x, double y, double z) {
    double v[3] = {x, y, z}, acc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double cen = g.o[a] + ((double)ic[a] + 0.5) * g.h;
        double d = minimg(g, v[a] - cen);
        double e = fabs(d) - g.half;
        if (e < 0.0) e = 0.0;
        acc[a] = e * e;
    }
    return (acc[0] + acc[1]) + acc[2];
}

__device__ __forceinline__ void make_grid(const DevParams& P, const DevPtrs& D, const SysDesc& s, const LevelDesc& lv, int sys,
                          int level, int64_t sweep, Grid& g) {
    g.h = lv.h;
    g.invh = 1.0 / lv.h;
    g.half = 0.5 * lv.h;
    g.periodic = P.periodic;
    if (P.periodic) {
        Stream st;
        st.init(P, sys, sweep, TAG_SHIFT + level, 0, 0, 0, 0);
        g.L = s.L;
        g.invL = 1.0 / s.L;
        for (int a = 0; a < 3; ++a) {
            g.o[a] = lv.h * st.co();
            g.n[a] = lv.n;
            g.k0[a] = 0;
        }
    } else {
        g.L = 0.0;
        g.invL = 0.0;
        for (int a = 0; a < 3; ++a) {
            g.o[a] = D.igrid[a];
            g.n[a] = (int64_t)D.igrid[3 + a];
            g.k0[a] = (int64_t)D.igrid[6 + a];
        }
    }
}

__device__ __forceinline__ double pair_r2(const DevParams& P, double invL, double L, double ax, double ay, double az,
                                          double bx, double by, double bz) {
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    if (P.periodic) {
        dx = dx - L * rint(dx * invL);
        dy = dy - L * rint(dy * invL);
        dz = dz - L * rint(dz * invL);
    }
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ double wrap01(double v, double L, double invL) {
    double w = v - L * floor(v * invL);
    return w >= L ? 0.0 : w;
}

// range of neighbour-grid cells covering [lo, hi] on one axis (wrapped); count >= nf -> all
__device__ __forceinline__ void fine_range(double lo, double hi, double invg, int nf, int& f0, int& cnt) {
    int a = (int)floor(lo * invg), b = (int)floor(hi * invg);
    cnt = b - a + 1;
    if (cnt >= nf) {
        f0 = 0;
        cnt = nf;
    } else {
        f0 = ((a % nf) + nf) % nf;
    }
}

// the wavelet of the current test: centre, polarisation, radius and amplitude
struct WaveDesc {
    double b[3], p[3], lam, A;
    int rot;  // WMC_MAP_ROTATION: the exact-rotation map
};

// Displacement of a bead at (x, y, z) by the wavelet, x_r = minimg(r - b)/lambda:
//  linear map (Eqs. "Oseen as <ww>", "Tapered wavelet"): A w(x_r, p) = A (1 - |x_r|) p x x_r;
//  rotation map: lambda x_r turned about p by the angle a = (A/lambda)(1 - |x_r|), by Rodrigues'
//  formula lambda [sin a (p x x_r) + (1 - cos a)(p (p.x_r) - x_r)] with 1 - cos a = 2 sin^2(a/2).
__device__ __forceinline__ void wavelet_disp(const Grid& g, const WaveDesc& wv, double x, double y, double z,
                                             double& w0, double& w1, double& w2) {
    const double xr0 = minimg(g, x - wv.b[0]) / wv.lam;
    const double xr1 = minimg(g, y - wv.b[1]) / wv.lam;
    const double xr2 = minimg(g, z - wv.b[2]) / wv.lam;
    const double rr = sqrt((xr0 * xr0 + xr1 * xr1) + xr2 * xr2);
    if (wv.rot) {
        const double a = rr < 1.0 ? (wv.A / wv.lam) * (1.0 - rr) : 0.0;
        const double sa = sin(a), hs = sin(0.5 * a), omc = 2.0 * hs * hs;
        const double pd = (wv.p[0] * xr0 + wv.p[1] * xr1) + wv.p[2] * xr2;
        w0 = wv.lam * (sa * (wv.p[1] * xr2 - wv.p[2] * xr1) + omc * (wv.p[0] * pd - xr0));
        w1 = wv.lam * (sa * (wv.p[2] * xr0 - wv.p[0] * xr2) + omc * (wv.p[1] * pd - xr1));
        w2 = wv.lam * (sa * (wv.p[0] * xr1 - wv.p[1] * xr0) + omc * (wv.p[2] * pd - xr2));
        return;
    }
    const double f = rr < 1.0 ? wv.A * (1.0 - rr) : 0.0;
    w0 = f * (wv.p[1] * xr2 - wv.p[2] * xr1);
    w1 = f * (wv.p[2] * xr0 - wv.p[0] * xr2);
    w2 = f * (wv.p[0] * xr1 - wv.p[1] * xr0);
}

// Amplitude of a wavelet of radius lam holding n beads (Eq. "Wavelet amplitude"); uniform centres
// use the mean count <n> = (4 pi/3) lam^3 N/L^3 of the homogeneous box instead of n
template <bool VAR>
__device__ __forceinline__ double wavelet_amp(const DevParams& P, const SysDesc& s, double lam, int n) {
    if (VAR && P.centring == WMC_CENTRE_UNIFORM)
        return P.A0 * lam / sqrt((4.0 * kPi / 3.0) * lam * lam * lam * (double)s.N / (s.L * s.L * s.L));
    return P.A0 * lam / sqrt((double)n);
}

// Trial centre of a wavelet from stream st: anchored, b = r_a + lam V with a uniform in the reach list
// (its slot or bead via pick) and V uniform in the unit ball (Eq. "PDF for b", App. D); uniform, b
// uniform in the cell. Returns whether b lies in the cell; a = -1 for uniform centres.
template <bool VAR, class Pick, class Pos>
__device__ __forceinline__ bool draw_trial_centre(const DevParams& P, Stream& st, const Grid& g, const int64_t ic[3],
                                                  int64_t cell, double lam, int nS, Pick pick, Pos pos, int32_t& a,
                                                  double& bx, double& by, double& bz) {
    if (VAR && P.centring == WMC_CENTRE_UNIFORM) {
        a = -1;
        bx = g.o[0] + ((double)ic[0] + st.co()) * g.h;
        by = g.o[1] + ((double)ic[1] + st.co()) * g.h;
        bz = g.o[2] + ((double)ic[2] + st.co()) * g.h;
    } else {
        a = pick(st.index(nS));
        double vx, vy, vz;
        ball(st, vx, vy, vz);
        double ax, ay, az;
        pos(a, ax, ay, az);
        bx = ax + lam * vx;
        by = ay + lam * vy;
        bz = az + lam * vz;
    }
    return cell_of_point(g, bx, by, bz) == cell;
}

// ------------------------------------------------------------------- workgroup helpers
template <int W>
__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < W / 64; ++i) t += red[i];
    return t;
}
// three sums in one exchange (red holds 3 W/64 entries)
template <int W>
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* red) {
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
        c += __shfl_xor(c, o);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red[3 * wv] = a;
        red[3 * wv + 1] = b;
        red[3 * wv + 2] = c;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0, tc = 0.0;
    for (int i = 0; i < W / 64; ++i) {
        ta += red[3 * i];
        tb += red[3 * i + 1];
        tc += red[3 * i + 2];
    }
    a = ta;
    b = tb;
    c = tc;
}
template <int W>
__device__ __forceinline__ double block_max(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double t = red[0];
    for (int i = 1; i < W / 64; ++i) t = fmax(t, red[i]);
    return t;
}
template <int W>
__device__ __forceinline__ int block_min_int(int v, int* redi) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) redi[wv] = v;
    __syncthreads();
    int t = redi[0];
    for (int i = 1; i < W / 64; ++i) t = min(t, redi[i]);
    return t;
}
// exclusive prefix of a flag over the workgroup in thread order; returns the total
template <int W>
__device__ __forceinline__ int block_scan_flag(bool f, int& before, int* redi) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint64_t m = __ballot(f);
    int in_wave = __popcll(m & ((1ull << lane) - 1ull));
    __syncthreads();
    if (lane == 0) redi[wv] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < W / 64; ++i) {
        if (i < wv) off += redi[i];
        tot += redi[i];
    }
    before = off + in_wave;
    return tot;
}

constexpr int SCAN_CH = 8;  // consecutive list entries per thread in the chunked scans

// exclusive prefix of a non-negative count over the workgroup in thread order; returns the total
template <int W>
__device__ __forceinline__ int block_scan_count(int v, int& before, int* redi) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) redi[wv] = x;
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < W / 64; ++i) {
        if (i < wv) off += redi[i];
        tot += redi[i];
    }
    before = off + x - v;
    return tot;
}

__device__ __forceinline__ void atomic_max_double(unsigned long long* p, double v) {
    // non-negative doubles order like their bit patterns
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

__device__ void trace_push(const DevPtrs& D, int kind, int sys, int64_t sweep, int level, int64_t cell, int64_t trial,
                           int retry, int64_t n, int acc, int extra, double dU, double thr) {
    if (!D.trace) return;
    unsigned long long i = atomicAdd(D.trace_n, 1ull);
    if ((int64_t)i >= D.trace_cap) return;
    wmc_trace_rec r;
    r.kind = kind;
    r.system = sys;
    r.sweep = (int32_t)sweep;
    r.level = level;
    r.cell = (int32_t)cell;
    r.trial = (int32_t)trial;
    r.retry = retry;
    r.n = (int32_t)n;
    r.accepted = acc;
    r.extra = extra;
    r.dU = dU;
    r.thr = thr;
    D.trace[i] = r;
}

// ------------------------------------------------------------------ neighbour grid build
__global__ void k_fine_count(DevPtrs D, int64_t N) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const SysDesc& s = D.sys[D.sys_id[i]];
    double x = D.x[i], y = D.y[i], z = D.z[i];
    D.xb[i] = x;
    D.yb[i] = y;
    D.zb[i] = z;
    int nf = s.nf;
    int cx = min(nf - 1, (int)floor(wrap01(x, s.L, s.invL) * s.invg));
    int cy = min(nf - 1, (int)floor(wrap01(y, s.L, s.invL) * s.invg));
    int cz = min(nf - 1, (int)floor(wrap01(z, s.L, s.invL) * s.invg));
    int32_t fc = (int32_t)(s.fine_off + cx + (int64_t)nf * (cy + (int64_t)nf * cz));
    D.fcell[i] = fc;
    atomicAdd(&D.fcount[fc], 1);
}

// exclusive scan of the neighbour-grid counts in chunks of 4096 cells: per-chunk sums, then
// each workgroup adds the sums of the chunks before it and scans its own chunk
constexpr int SCAN_CHUNK = 4096;

__global__ __launch_bounds__(1024) void k_scan_sums(DevPtrs D) {
    __shared__ int red[16];
    const int64_t a = (int64_t)blockIdx.x * SCAN_CHUNK;
    int acc = 0;
    for (int k = threadIdx.x; k < SCAN_CHUNK; k += 1024) {
        int64_t i = a + k;
        if (i < D.total_fine) acc += D.fcount[i];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < 16; ++w) t += red[w];
        D.fblock[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_scan_apply(DevPtrs D, int nsys, int nchunks) {
    __shared__ int part[1024];
    __shared__ int base;
    const int tid = threadIdx.x;
    if (tid == 0) {
        int b = 0;
        for (int c = 0; c < (int)blockIdx.x; ++c) b += D.fblock[c];
        base = b;
    }
    // each thread owns 4 consecutive cells of the chunk
    const int64_t a = (int64_t)blockIdx.x * SCAN_CHUNK + 4 * tid;
    int v[4], sum = 0;
    for (int q = 0; q < 4; ++q) {
        v[q] = (a + q < D.total_fine) ? D.fcount[a + q] : 0;
        sum += v[q];
    }
    part[tid] = sum;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 per-thread sums
    for (int o = 1; o < 1024; o <<= 1) {
        int t = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += t;
        __syncthreads();
    }
    int run = base + part[tid] - sum;
    for (int q = 0; q < 4; ++q) {
        if (a + q < D.total_fine) {
            D.fstart[a + q] = run;
            D.fcount[a + q] = 0;
        }
        run += v[q];
    }
    if ((int)blockIdx.x == nchunks - 1 && tid == 1023) D.fstart[D.total_fine] = base + part[1023];
    if (blockIdx.x == 0) {
        for (int s = tid; s < nsys; s += 1024) D.drift[s] = 0ull;
        for (int s = tid; s < 8 * nsys; s += 1024) D.drift_col[s] = 0ull;
        if (tid == 0) atomicAdd(&D.cnt[CNT_REBUILD], 1ull);
    }
}

__global__ void k_fine_scatter(DevPtrs D, int64_t N) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int32_t fc = D.fcell[i];
    int pos = D.fstart[fc] + atomicAdd(&D.fcount[fc], 1);
    D.fidx[pos] = (int32_t)i;
}

// order each cell's beads by index (deterministic candidate order) and clear the cursor
__global__ void k_fine_sort(DevPtrs D) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= D.total_fine) return;
    int a = D.fstart[c], b = D.fstart[c + 1];
    for (int i = a + 1; i < b; ++i) {
        int32_t v = D.fidx[i];
        int j = i - 1;
        while (j >= a && D.fidx[j] > v) {
            D.fidx[j + 1] = D.fidx[j];
            --j;
        }
        D.fidx[j + 1] = v;
    }
    D.fcount[c] = 0;
}

void launch_fine_build(const DevParams& P, const DevPtrs& D, int64_t N, hipStream_t st) {
    if (N == 0) return;
    int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL(k_fine_count, dim3(nb), dim3(256), 0, st, D, N);
    int nchunks = (int)((D.total_fine + SCAN_CHUNK - 1) / SCAN_CHUNK);
    hipLaunchKernelGGL(k_scan_sums, dim3(nchunks), dim3(1024), 0, st, D);
    hipLaunchKernelGGL(k_scan_apply, dim3(nchunks), dim3(1024), 0, st, D, P.nsys, nchunks);
    hipLaunchKernelGGL(k_fine_scatter, dim3(nb), dim3(256), 0, st, D, N);
    int nc = (int)((D.total_fine + 255) / 256);
    hipLaunchKernelGGL(k_fine_sort, dim3(nc), dim3(256), 0, st, D);
}

// ------------------------------------------------------- infinite-system level grid
__global__ __launch_bounds__(1024) void k_bbox(DevParams P, DevPtrs D, int level, int64_t sweep) {
    __shared__ double red[16];
    const SysDesc& s = D.sys[0];
    const LevelDesc& lv = D.lev[s.lvl_off + level];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = s.b0 + threadIdx.x; i < s.b1; i += 1024) {
        double v[3] = {D.x[i], D.y[i], D.z[i]};
        for (int a = 0; a < 3; ++a) {
            mn[a] = fmin(mn[a], v[a]);
            mx[a] = fmax(mx[a], v[a]);
        }
    }
    double gmn[3], gmx[3];
    for (int a = 0; a < 3; ++a) {
        gmn[a] = -block_max<1024>(-mn[a], red);
        gmx[a] = block_max<1024>(mx[a], red);
    }
    if (threadIdx.x == 0) {
        // the cells of the fixed lattice h (k + u), k integer, that cover the bounding box grown
        // by lambda_hi: the lattice, the colour of a cell (parity of k) and its stream key do not
        // depend on the positions
        Stream st;
        st.init(P, 0, sweep, TAG_SHIFT + level, 0, 0, 0, 0);
        double invh = 1.0 / lv.h;
        for (int a = 0; a < 3; ++a) {
            const double u = st.co();
            const int64_t kmin = (int64_t)floor((gmn[a] - lv.hi) * invh - u);
            const int64_t kmax = (int64_t)floor((gmx[a] + lv.hi) * invh - u);
            D.igrid[a] = ((double)kmin + u) * lv.h;
            D.igrid[3 + a] = (double)(kmax - kmin + 1);
            D.igrid[6 + a] = (double)kmin;
        }
    }
}

void launch_bbox(const DevParams& P, const DevPtrs& D, int level, int64_t sweep, hipStream_t st) {
    hipLaunchKernelGGL(k_bbox, dim3(1), dim3(1024), 0, st, P, D, level, sweep);
}

// Grid-wide barrier of a cooperative launch (every workgroup co-resident). Each wave first
// waits for its own stores to complete, so after the workgroup barrier all of the
// workgroup's writes sit in this XCD's L2; one thread then publishes them at agent scope
// (L2 write-back, the release of the arrival count), waits for the generation to advance and
// acquires (L1 and stale L2 lines dropped) for the whole workgroup, which shares its CU's L1.
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned nblocks, unsigned& gen) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's global stores are complete
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned g = gen;
        unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (arrived == nblocks) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[1], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // spin on relaxed loads (an acquiring load would invalidate the L2 on every poll), then
            // acquire once
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) __builtin_amdgcn_s_sleep(2);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
    gen = gen + 1u;
    __syncthreads();
}

// barrier over the nblocks workgroups of one cooperative group (a plain workgroup barrier when
// the group is a single workgroup)
__device__ __forceinline__ void group_barrier(unsigned* bar, unsigned nblocks, unsigned& gen) {
    if (nblocks > 1) {
        grid_barrier(bar, nblocks, gen);
    } else {
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __syncthreads();
    }
}

// group_barrier in two halves, so that a workgroup can work between its arrival and its wait: the
// arrival publishes what the workgroup wrote before it; the work in between must not write what
// another workgroup of the group reads after the barrier. `released` tells thread 0 that its own
// arrival was the last one.
__device__ __forceinline__ void group_arrive(unsigned* bar, unsigned nblocks, unsigned gen, bool& released) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    released = true;
    if (nblocks > 1 && threadIdx.x == 0) {
        const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        released = arrived == nblocks;
        if (released) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[1], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}
__device__ __forceinline__ void group_wait(unsigned* bar, unsigned nblocks, unsigned& gen, bool released) {
    if (nblocks > 1) {
        if (threadIdx.x == 0 && !released) {
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) __builtin_amdgcn_s_sleep(2);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        gen = gen + 1u;
    }
    __syncthreads();
}

// --------------------------------------------------------------------- cell phase
// One workgroup processes one cell of the current colour:
//  1. reach list S_c = beads within lambda_hi of the cell, ascending index (from the
//     neighbour grid and an LDS bitonic sort, or a bead-order scan for large cells);
//  2. K_c = stochastic rounding of T_l |S_c| / N trials;
//  3. trials are evaluated W at a time in parallel (each trial has its own stream and only
//     reads positions), the first hit starts a recycling chain run by the whole workgroup:
//     direction, members (ballot compaction), displacement, dU over bonds and WCA pairs
//     (neighbour grid), reduction, Metropolis test, write-through on accept; after a
//     rejection W centre redraws are tried in parallel and the first hit continues.
template <int W, int CAPS, int CAPM>
struct PhaseShared {
    int32_t S[CAPS];
    int32_t M[CAPM];
    double MX[CAPM], MY[CAPM], MZ[CAPM];
    double red[W / 64 > 0 ? W / 64 : 1];
    int redi[W / 64 > 0 ? W / 64 : 1];
    int count;
    double pub_b[3];
    double pub_lam;
    int32_t pub_a;
    uint32_t pub_next;
};

// grid coordinates of the local-th cell of a colour (in an infinite system the colour is the parity of
// the lattice index k0 + ic, so local parities are the colour's bits flipped by those of k0)
__device__ __forceinline__ void cell_coords(const DevParams& P, const LevelDesc& lv, const Grid& g, int colour,
                                            int64_t local, int64_t ic[3]) {
    if (P.periodic) {
        int64_t m = lv.n >= 2 ? lv.n / 2 : 1;
        ic[0] = 2 * (local % m) + (lv.n >= 2 ? (colour & 1) : 0);
        ic[1] = 2 * ((local / m) % m) + (lv.n >= 2 ? ((colour >> 1) & 1) : 0);
        ic[2] = 2 * (local / (m * m)) + (lv.n >= 2 ? ((colour >> 2) & 1) : 0);
    } else {
        const int lc = colour ^ grid_parity(g);
        int64_t mx = (g.n[0] - (lc & 1) + 1) / 2, my = (g.n[1] - ((lc >> 1) & 1) + 1) / 2;
        ic[0] = 2 * (local % mx) + (lc & 1);
        ic[1] = 2 * ((local / mx) % my) + ((lc >> 1) & 1);
        ic[2] = 2 * (local / (mx * my)) + ((lc >> 2) & 1);
    }
}

// energy change of the current test, global-memory form: bonds and WCA pairs with >= 1
// member, each once. Members Ml[0..n) with trial positions MXl/MYl/MZl (LDS or global) and
// D.tag set. WCA partners come from the neighbour grid: every bead whose grid-build position
// lies within R (per axis) of a member's current position, R covering the cut-off, both
// displacements and the drift since the build. One work item is a (member, y-z row of grid
// cells) pair; its x range is one or two contiguous runs of the grid's bead list.
// Work items are dealt to threads t0, t0 + stride, ... (one workgroup, or a whole grid).
__device__ void glob_dU(const DevParams& P, const DevPtrs& D, const SysDesc& s, const int32_t* Ml, const double* MXl,
                        const double* MYl, const double* MZl, int n, double R, int t0, int stride,
                        double& acc, unsigned long long& viol, bool pairs = true) {
    const double L = s.L, invL = s.invL;
    auto term = [&](int32_t j, double jx, double jy, double jz, double kx, double ky, double kz, int32_t m) {
        if (m == j) return;
        const int km = D.tag[m];
        if (km >= 0 && m < j) return;
        const double mx = D.x[m], my = D.y[m], mz = D.z[m];
        const double nx = km >= 0 ? MXl[km] : mx, ny = km >= 0 ? MYl[km] : my, nz = km >= 0 ? MZl[km] : mz;
        const double r2o = pair_r2(P, invL, L, jx, jy, jz, mx, my, mz);
        const double r2n = pair_r2(P, invL, L, kx, ky, kz, nx, ny, nz);
        if (r2o < P.rc2 || r2n < P.rc2) acc += u_pair(P, r2n) - u_pair(P, r2o);
    };
    if (P.bond_type != WMC_BOND_NONE) {
        for (int k = t0; k < n; k += stride) {
            const int32_t j = Ml[k];
            const double jx = D.x[j], jy = D.y[j], jz = D.z[j];
            const double kx = MXl[k], ky = MYl[k], kz = MZl[k];
            int32_t part[2] = {-1, -1};
            if (j + 1 < s.b1 && D.bond_next[j]) part[0] = j + 1;
            if (j > s.b0 && D.bond_next[j - 1]) part[1] = j - 1;
            for (int e = 0; e < 2; ++e) {
                const int32_t m = part[e];
                if (m < 0) continue;
                const int km = D.tag[m];
                if (km >= 0 && m < j) continue;
                const double mx = D.x[m], my = D.y[m], mz = D.z[m];
                const double nx = km >= 0 ? MXl[km] : mx, ny = km >= 0 ? MYl[km] : my, nz = km >= 0 ? MZl[km] : mz;
                const double r2o = pair_r2(P, invL, L, jx, jy, jz, mx, my, mz);
                const double r2n = pair_r2(P, invL, L, kx, ky, kz, nx, ny, nz);
                if (r2o > P.r_int * P.r_int) ++viol;
                acc += u_bond_delta(P, r2n, r2o);
            }
        }
    }
    if (!P.wca || !pairs) return;
    if (P.periodic) {
        const int nf = s.nf;
        const int NR = min(nf, (int)floor(2.0 * R * s.invg) + 2);
        const int per = NR * NR;
        for (int it = t0; it < n * per; it += stride) {
            const int k = it / per, q = it - k * per;
            const int qy = q % NR, qz = q / NR;
            const int32_t j = Ml[k];
            const double jx = D.x[j], jy = D.y[j], jz = D.z[j];
            int f0y, cny, f0z, cnz;
            const double cy = wrap01(jy, L, invL), cz = wrap01(jz, L, invL);
            fine_range(cy - R, cy + R, s.invg, nf, f0y, cny);
            fine_range(cz - R, cz + R, s.invg, nf, f0z, cnz);
            if (qy >= cny || qz >= cnz) continue;
            int f0x, cnx;
            const double cx = wrap01(jx, L, invL);
            fine_range(cx - R, cx + R, s.invg, nf, f0x, cnx);
            const int fy = (f0y + qy) % nf, fz = (f0z + qz) % nf;
            const int64_t row = s.fine_off + (int64_t)nf * (fy + (int64_t)nf * fz);
            const double kx = MXl[k], ky = MYl[k], kz = MZl[k];
            const int xa = f0x, xe = min(f0x + cnx, nf);
            // the row's beads two at a time, so that the loads of the second overlap the first
            auto run = [&](int q2, int q3) {
                for (; q2 + 1 < q3; q2 += 2) {
                    const int32_t m0 = D.fidx[q2], m1 = D.fidx[q2 + 1];
                    term(j, jx, jy, jz, kx, ky, kz, m0);
                    term(j, jx, jy, jz, kx, ky, kz, m1);
                }
                if (q2 < q3) term(j, jx, jy, jz, kx, ky, kz, D.fidx[q2]);
            };
            run(D.fstart[row + xa], D.fstart[row + xe]);
            if (f0x + cnx > nf) run(D.fstart[row], D.fstart[row + (f0x + cnx - nf)]);
        }
    } else {
        // infinite system (at most 8192 beads): items are (member, 64-bead block)
        const int64_t nb = s.b1 - s.b0;
        const int nblk = (int)((nb + 63) / 64);
        for (int it = t0; it < n * nblk; it += stride) {
            const int k = it / nblk, c = it - k * nblk;
            const int32_t j = Ml[k];
            const double jx = D.x[j], jy = D.y[j], jz = D.z[j];
            const double kx = MXl[k], ky = MYl[k], kz = MZl[k];
            const int64_t m0 = s.b0 + 64 * (int64_t)c, m1 = min(s.b1, m0 + 64);
            for (int64_t m = m0; m < m1; ++m) term(j, jx, jy, jz, kx, ky, kz, (int32_t)m);
        }
    }
}

// Dg bounds the drift, since the neighbour grid was built, of every bead this cell can meet; the
// largest drift of the beads the cell moves is returned in dl_out.
template <int W, int CAPS, int CAPM, bool VAR>
__device__ __forceinline__ void process_cell(const DevParams& P, const DevPtrs& D,
                                                       PhaseShared<W, CAPS, CAPM>& sh, int sys,
                             int level, int colour, int64_t local, int64_t sweep, const Grid& g,
                             const double Dg, double& dl_out) {
    const SysDesc& s = D.sys[sys];
    const LevelDesc& lv = D.lev[s.lvl_off + level];
    const int tid = threadIdx.x;
    // cell coordinates of the local-th cell of this colour
    int64_t ic[3];
    cell_coords(P, lv, g, colour, local, ic);
    const int64_t cell = ic[0] + g.n[0] * (ic[1] + g.n[1] * ic[2]);
    const int64_t key = cell_key(g, ic);
    const double hi2 = lv.hi * lv.hi;
    dl_out = 0.0;
    const bool glob = lv.use_global != 0;
    int32_t* Sg = D.slot_S + (lv.slot_base + local) * D.slot_len;
    int32_t* Mg = D.slot_M + (lv.slot_base + local) * D.slot_len;
    double* MXg = D.slot_MX + (lv.slot_base + local) * 3 * D.slot_len;

    // ---- 1. reach list
    int nS = 0;
    bool overflow = false;
    if (lv.identity) {
        nS = s.N;
    } else if (glob || !P.periodic) {
        // bead-order scan of the system, compacted in order
        // each thread tests SCAN_CH consecutive beads (independent loads in flight), then one
        // workgroup scan places its hits in bead order
        int32_t* dst = glob ? Sg : sh.S;
        int base = 0;
        for (int64_t c0 = s.b0; c0 < s.b1; c0 += (int64_t)W * SCAN_CH) {
            const int64_t j0 = c0 + (int64_t)tid * SCAN_CH;
            uint32_t mask = 0;
#pragma unroll
            for (int u = 0; u < SCAN_CH; ++u) {
                const int64_t j = j0 + u;
                if (j < s.b1 && dist2_cell(g, ic, D.x[j], D.y[j], D.z[j]) <= hi2) mask |= 1u << u;
            }
            int before;
            const int tot = block_scan_count<W>(__popc(mask), before, sh.redi);
            int idx = base + before;
            for (int u = 0; u < SCAN_CH; ++u) {
                if ((mask >> u) & 1u) {
                    if (glob || idx < CAPS) dst[idx] = (int32_t)(j0 + u);
                    ++idx;
                }
            }
            base += tot;
        }
        nS = base;
        if (!glob && nS > CAPS) overflow = true;
    } else {
        // neighbour-grid gather into LDS, then bitonic sort by bead index
        if (tid == 0) sh.count = 0;
        __syncthreads();
        double R = lv.hi + Dg + 1e-9 * s.L;
        int f0[3], cn[3];
        for (int a = 0; a < 3; ++a) {
            double lo = g.o[a] + (double)ic[a] * g.h - R;
            fine_range(lo, lo + g.h + 2.0 * R, s.invg, s.nf, f0[a], cn[a]);
        }
        const int total = cn[0] * cn[1] * cn[2];
        for (int q = tid; q < total; q += W) {
            int qx = q % cn[0], qy = (q / cn[0]) % cn[1], qz = q / (cn[0] * cn[1]);
            int fx = (f0[0] + qx) % s.nf, fy = (f0[1] + qy) % s.nf, fz = (f0[2] + qz) % s.nf;
            int64_t fc = s.fine_off + fx + (int64_t)s.nf * (fy + (int64_t)s.nf * fz);
            for (int k = D.fstart[fc]; k < D.fstart[fc + 1]; ++k) {
                int32_t j = D.fidx[k];
                if (dist2_cell(g, ic, D.x[j], D.y[j], D.z[j]) <= hi2) {
                    int idx = atomicAdd(&sh.count, 1);
                    if (idx < CAPS) sh.S[idx] = j;
                }
            }
        }
        __syncthreads();
        nS = sh.count;
        if (nS > CAPS) {
            overflow = true;
        } else if (nS > 1) {
            int np2 = 1;
            while (np2 < nS) np2 <<= 1;
            for (int i = nS + tid; i < np2; i += W) sh.S[i] = 0x7FFFFFFF;
            __syncthreads();
            for (int k = 2; k <= np2; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int i = tid; i < np2; i += W) {
                        int l = i ^ j;
                        if (l > i) {
                            int32_t a = sh.S[i], b = sh.S[l];
                            bool up = (i & k) == 0;
                            if ((a > b) == up) {
                                sh.S[i] = b;
                                sh.S[l] = a;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
        }
    }
    __syncthreads();
    if (overflow) {
        if (tid == 0) atomicAdd(&D.cnt[CNT_OVERFLOW], 1ull);
        return;
    }
    const int32_t* S = lv.identity ? nullptr : (glob ? Sg : sh.S);
    auto Sat = [&](int64_t i) -> int32_t { return S ? S[i] : (int32_t)(s.b0 + i); };

    // ---- 2. number of trials: T_l |S_c| / N (anchored centres) or T_l / n^3 (uniform centres)
    const bool uni = VAR && P.centring == WMC_CENTRE_UNIFORM;
    double mu = uni ? lv.T / ((double)g.n[0] * (double)g.n[1] * (double)g.n[2]) : (lv.T * (double)nS) / (double)s.N;
    int64_t K = (int64_t)floor(mu);
    {
        Stream ms;
        ms.init(P, sys, sweep, TAG_META + level, key, 0, 0, 0);
        if (ms.co() < mu - (double)K) K += 1;
    }
    if (K > 0xFFFFF) {
        K = 0xFFFFF;
        if (tid == 0) atomicAdd(&D.cnt[CNT_VIOL], 1ull);
    }
    unsigned long long c_hits = 0, c_att = 0, c_acc = 0, c_caps = 0, c_redraw = 0, c_beads = 0, c_viol = 0;
    double d_local = 0.0;  // max drift of beads moved in this phase

    const double L = s.L, invL = s.invL;
    const double lam_hi = lv.hi;

    auto pos_of = [&](int32_t j, double& px, double& py, double& pz) {
        px = D.x[j];
        py = D.y[j];
        pz = D.z[j];
    };
    bool stop = false;  // a member list overflowed: the cell's remaining moves are skipped

    // ---- 3. trials and chains
    for (int64_t t0 = 0; t0 < K;) {
        int64_t t = t0 + tid;
        bool hit = false;
        double lam = 0.0, bx = 0.0, by = 0.0, bz = 0.0;
        int32_t a = 0;
        Stream st;
        if (t < K && (nS > 0 || uni)) {
            st.init(P, sys, sweep, level, key, t, 0, 0);
            lam = draw_lambda(st.co(), lv.lo, lam_hi);
            hit = draw_trial_centre<VAR>(P, st, g, ic, cell, lam, nS, Sat, pos_of, a, bx, by, bz);
        }
        int first = block_min_int<W>(hit ? (int)(t - t0) : 0x7FFFFFFF, sh.redi);
        if (first == 0x7FFFFFFF) {
            t0 += W;
            continue;
        }
        if (tid == first) {
            sh.pub_lam = lam;
            sh.pub_a = a;
            sh.pub_b[0] = bx;
            sh.pub_b[1] = by;
            sh.pub_b[2] = bz;
            sh.pub_next = st.next;
        }
        __syncthreads();
        const int64_t tc = t0 + first;
        lam = sh.pub_lam;
        a = sh.pub_a;
        double b[3] = {sh.pub_b[0], sh.pub_b[1], sh.pub_b[2]};
        uint32_t nxt = sh.pub_next;
        int jtry = 0;
        ++c_hits;
        const double lam2 = lam * lam;
        for (int r = 0;;) {
            // direction and acceptance draw continue the stream of (tc, r, jtry)
            Stream cs;
            cs.init(P, sys, sweep, level, key, tc, r, jtry);
            cs.next = nxt;
            double px, py, pz;
            direction(cs, px, py, pz);
            const double u_acc = cs.oc();
            __syncthreads();
            // members: reach-list beads within lambda of b, plus the anchor, in list order; kept
            // in LDS when they fit, and also in the cell's global slot on global-list levels
            int n = 0;
            for (int c0 = 0; c0 < nS; c0 += W * SCAN_CH) {
                const int i0 = c0 + tid * SCAN_CH;
                uint32_t mask = 0;
#pragma unroll
                for (int u = 0; u < SCAN_CH; ++u) {
                    const int i = i0 + u;
                    if (i < nS) {
                        const int32_t j = Sat(i);
                        double dx = minimg(g, D.x[j] - b[0]), dy = minimg(g, D.y[j] - b[1]),
                               dz = minimg(g, D.z[j] - b[2]);
                        double d2 = (dx * dx + dy * dy) + dz * dz;
                        if (d2 <= lam2 || j == a) mask |= 1u << u;
                    }
                }
                int before;
                const int tot = block_scan_count<W>(__popc(mask), before, sh.redi);
                int idx = n + before;
                for (int u = 0; u < SCAN_CH; ++u) {
                    if ((mask >> u) & 1u) {
                        const int32_t j = Sat(i0 + u);
                        if (idx < CAPM) sh.M[idx] = j;
                        if (glob) Mg[idx] = j;
                        ++idx;
                    }
                }
                n += tot;
            }
            // members written by lanes of other waves must land before any lane reads them
            __syncthreads();
            const bool inL = n <= CAPM;
            if (!inL && !glob) {
                // nothing of this test has moved yet: count it and end the cell here, publishing
                // the drift and counters of the moves made so far
                if (tid == 0) atomicAdd(&D.cnt[CNT_OVERFLOW], 1ull);
                stop = true;
                break;
            }
            const int32_t* Ml = inL ? sh.M : Mg;
            double *MXl = inL ? sh.MX : MXg, *MYl = inL ? sh.MY : MXg + D.slot_len,
                   *MZl = inL ? sh.MZ : MXg + 2 * D.slot_len;
            WaveDesc wv;
            wv.b[0] = b[0];
            wv.b[1] = b[1];
            wv.b[2] = b[2];
            wv.p[0] = px;
            wv.p[1] = py;
            wv.p[2] = pz;
            wv.lam = lam;
            wv.A = wavelet_amp<VAR>(P, s, lam, n);
            wv.rot = VAR && P.wavelet_map == WMC_MAP_ROTATION;
            double dmax_l = 0.0;
            for (int k = tid; k < n; k += W) {
                int32_t j = Ml[k];
                double w0, w1, w2;
                wavelet_disp(g, wv, D.x[j], D.y[j], D.z[j], w0, w1, w2);
                MXl[k] = D.x[j] + w0;
                MYl[k] = D.y[j] + w1;
                MZl[k] = D.z[j] + w2;
                D.tag[j] = k;
                dmax_l = fmax(dmax_l, sqrt((w0 * w0 + w1 * w1) + w2 * w2));
            }
            const double dmax = block_max<W>(dmax_l, sh.red);  // includes a barrier: tags visible
            const double Rq = P.rc + 2.0 * dmax + fmax(Dg, d_local) + 1e-9 * L;
            double dU;
            const double thr = accept_threshold<VAR>(P, u_acc);
            {
                double acc = 0.0;
                glob_dU(P, D, s, Ml, MXl, MYl, MZl, n, Rq, tid, W, acc, c_viol);
                dU = block_sum<W>(acc, sh.red);
            }
            const bool accept = dU <= thr;
            if (tid == 0) trace_push(D, 0, sys, sweep, level, key, tc, r, n, accept ? 1 : 0, a, dU, thr);
            ++c_att;
            c_beads += n;
            for (int k = tid; k < n; k += W) {
                int32_t j = Ml[k];
                if (accept) {
                    double nx = MXl[k], ny = MYl[k], nz = MZl[k];
                    D.x[j] = nx;
                    D.y[j] = ny;
                    D.z[j] = nz;
                    double dd = fmax(fabs(nx - D.xb[j]), fmax(fabs(ny - D.yb[j]), fabs(nz - D.zb[j])));
                    d_local = fmax(d_local, dd);
                }
                D.tag[j] = -1;
            }
            d_local = block_max<W>(d_local, sh.red);  // barrier: writes visible
            if (accept) {
                ++c_acc;
                if (tid == 0) atomicAdd(&D.cnt[CNT_ACC_BEADS], (unsigned long long)n);
                break;
            }
            if (++r >= P.retry_cap) {
                ++c_caps;
                break;
            }
            // recycle lambda: redraw anchor and centre until the centre is in the cell
            int found = -1;
            for (int j0 = 0; j0 < 4096 && found < 0; j0 += W) {
                int jj = j0 + tid;
                bool h2 = false;
                double ex = 0, ey = 0, ez = 0;
                int32_t a2 = 0;
                Stream rs;
                if (jj < 4096) {
                    rs.init(P, sys, sweep, level, key, tc, r, jj);
                    h2 = draw_trial_centre<VAR>(P, rs, g, ic, cell, lam, nS, Sat, pos_of, a2, ex, ey, ez);
                }
                int fj = block_min_int<W>(h2 ? jj : 0x7FFFFFFF, sh.redi);
                if (fj != 0x7FFFFFFF) {
                    if (jj == fj) {
                        sh.pub_a = a2;
                        sh.pub_b[0] = ex;
                        sh.pub_b[1] = ey;
                        sh.pub_b[2] = ez;
                        sh.pub_next = rs.next;
                    }
                    found = fj;
                }
            }
            __syncthreads();
            if (found < 0) {
                c_redraw += 4096;
                ++c_caps;
                break;
            }
            c_redraw += (unsigned long long)found;
            a = sh.pub_a;
            b[0] = sh.pub_b[0];
            b[1] = sh.pub_b[1];
            b[2] = sh.pub_b[2];
            nxt = sh.pub_next;
            jtry = found;
            __syncthreads();
        }
        if (stop) break;
        t0 = tc + 1;
    }
    __syncthreads();
    // ---- counters
    unsigned long long viol_all = (unsigned long long)block_sum<W>((double)c_viol, sh.red);
    if (tid == 0) {
        unsigned long long* C = D.cnt + CNT_LEVEL + level * 8;
        atomicAdd(&C[0], (unsigned long long)K);
        atomicAdd(&C[1], c_hits);
        atomicAdd(&C[2], c_att);
        atomicAdd(&C[3], c_acc);
        atomicAdd(&C[4], c_caps);
        atomicAdd(&C[5], c_redraw);
        atomicAdd(&C[6], c_beads);
        if (viol_all) atomicAdd(&D.cnt[CNT_VIOL], viol_all);
        if (c_acc) {
            atomicAdd(&D.cnt[CNT_ACCEPTED], c_acc);
            atomicAdd(&D.sys_acc[sys], c_acc);
        }
        if (d_local > 0.0) atomic_max_double(&D.drift[sys], d_local);
        trace_push(D, 1, sys, sweep, level, key, K, nS, 0, (int)c_hits, 0, 0.0, 0.0);
    }
    dl_out = d_local;
    __syncthreads();
}

// ------------------------------------------------------------- cell phase, LDS tile
// The cell's interaction halo -- every bead within lambda_hi + r_int of the cell -- is staged
// in LDS once per phase, sorted by bead index, with FP64 positions and its bond flags. Beads of
// the halo move only through this cell's own moves during the phase, and every bead within the
// pair cut-off or the bond length of a member lies in it, so trials, member tests,
// displacements and dU run from LDS; accepted moves are also written through to HBM.
constexpr int32_t ID_MASK = 0x3FFFFFFF;
constexpr int32_t ID_NEXT = 0x40000000;  // bonded to bead id + 1
constexpr uint32_t ID_PREV = 0x80000000u;  // bonded to bead id - 1

// One-barrier reductions (LDS tiles): reduction k of a kind uses half k % 2 of its exchange area (the
// toggles are block-uniform), so a half is written again only after a later reduction's barrier,
// which every thread passes after its reads of the earlier result. Same results as the block_*
// helpers, one barrier instead of two.
template <int W>
struct Exch {
    static constexpr int NW = W / 64 > 0 ? W / 64 : 1;
    double d[2 * NW];
    double d3[2 * 3 * NW];
    int i[2 * NW];
};
struct ExchPh {
    int d = 0, d3 = 0, i = 0;
};
template <int W>
__device__ __forceinline__ double xsum(double v, Exch<W>& x, ExchPh& p) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double* r = x.d + p.d * Exch<W>::NW;
    p.d ^= 1;
    if (lane == 0) r[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < W / 64; ++i) t += r[i];
    return t;
}
template <int W>
__device__ __forceinline__ double xmax(double v, Exch<W>& x, ExchPh& p) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double* r = x.d + p.d * Exch<W>::NW;
    p.d ^= 1;
    if (lane == 0) r[wv] = v;
    __syncthreads();
    double t = r[0];
    for (int i = 1; i < W / 64; ++i) t = fmax(t, r[i]);
    return t;
}
template <int W>
__device__ __forceinline__ void xsum3(double& a, double& b, double& c, Exch<W>& x, ExchPh& p) {
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
        c += __shfl_xor(c, o);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double* r = x.d3 + p.d3 * 3 * Exch<W>::NW;
    p.d3 ^= 1;
    if (lane == 0) {
        r[3 * wv] = a;
        r[3 * wv + 1] = b;
        r[3 * wv + 2] = c;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0, tc = 0.0;
    for (int i = 0; i < W / 64; ++i) {
        ta += r[3 * i];
        tb += r[3 * i + 1];
        tc += r[3 * i + 2];
    }
    a = ta;
    b = tb;
    c = tc;
}
template <int W>
__device__ __forceinline__ int xmin_int(int v, Exch<W>& x, ExchPh& p) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int* r = x.i + p.i * Exch<W>::NW;
    p.i ^= 1;
    if (lane == 0) r[wv] = v;
    __syncthreads();
    int t = r[0];
    for (int i = 1; i < W / 64; ++i) t = min(t, r[i]);
    return t;
}
template <int W>
__device__ __forceinline__ int xscan_flag(bool f, int& before, Exch<W>& x, ExchPh& p) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t m = __ballot(f);
    const int in_wave = __popcll(m & ((1ull << lane) - 1ull));
    int* r = x.i + p.i * Exch<W>::NW;
    p.i ^= 1;
    if (lane == 0) r[wv] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < W / 64; ++i) {
        if (i < wv) off += r[i];
        tot += r[i];
    }
    before = off + in_wave;
    return tot;
}
template <int W>
__device__ __forceinline__ int xscan_count(int v, int& before, Exch<W>& x, ExchPh& p) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int y = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int z = __shfl_up(y, o);
        if (lane >= o) y += z;
    }
    int* r = x.i + p.i * Exch<W>::NW;
    p.i ^= 1;
    if (lane == 63) r[wv] = y;
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < W / 64; ++i) {
        if (i < wv) off += r[i];
        tot += r[i];
    }
    before = off + y - v;
    return tot;
}

// T = double: absolute FP64 positions (FP64 contexts). T = float (mixed precision): FP32 offsets from
// the tile's centre, minimg(r - c) rounded once; the FP64 positions stay in HBM.
template <int W, int CAPH, int CAPM, int NCD, class T = double>
struct TileShared {
    T x[CAPH], y[CAPH], z[CAPH];
    int32_t id[CAPH];
    int16_t kc[CAPH];           // tile cell list: slots by tile cell, ascending within a cell
    // member index of a moved slot (-1: not moved); with no trial positions kept (CAPM == 0)
    // only whether it moved is needed, one bit per slot
    int16_t tag[CAPM > 0 ? CAPH : 1];
    uint32_t tagb[CAPM > 0 ? 1 : (CAPH + 31) / 32];
    int16_t S[CAPH];
    // first kc position of each tile cell (entry NC: the total); an even count of 4-byte aligned
    // entries, so that the index build can update them as packed pairs
    alignas(4) int16_t cst[(NCD * NCD * NCD + 2) & ~1];
    int16_t M[CAPH];                   // member slots of the current test
    // trial positions (T = float: FP32 displacements) of the first CAPM members (later ones are
    // recomputed when needed)
    T MX[CAPM > 0 ? CAPM : 1], MY[CAPM > 0 ? CAPM : 1], MZ[CAPM > 0 ? CAPM : 1];
    double red[W / 64 > 0 ? W / 64 : 1];
    int redi[W / 64 > 0 ? W / 64 : 1];
    Exch<W> xc;  // exchange area of the one-barrier reductions
    int count;
    double pub_b[3];  // the centre; on an FP32 tile with anchored centres the ball vector V
    float pub_bf[3];  // FP32 tile: the centre's offset from the tile centre
    double pub_lam;
    int32_t pub_a;
    uint32_t pub_next;
    int spec_found;  // first hit of the speculative redraw chunk, -1 if none
};

template <int W, int CAPS, int CAPM, int CAPH, int CAPMT, int NCD, class T = double>
union PhaseLDS {
    PhaseShared<W, CAPS, CAPM> g;
    TileShared<W, CAPH, CAPMT, NCD, T> t;
};

template <int W, int CAPH, int CAPM, int NCD, class T>
__device__ __forceinline__ int tile_tag(const TileShared<W, CAPH, CAPM, NCD, T>& sh, int sl) {
    if (CAPM > 0) return sh.tag[sl];
    return ((sh.tagb[sl >> 5] >> (sl & 31)) & 1u) ? 0 : -1;
}
template <int W, int CAPH, int CAPM, int NCD, class T>
__device__ __forceinline__ void tile_tag_set(TileShared<W, CAPH, CAPM, NCD, T>& sh, int sl, int k) {
    if (CAPM > 0)
        sh.tag[sl] = (int16_t)k;
    else
        atomicOr(&sh.tagb[sl >> 5], 1u << (sl & 31));
}
template <int W, int CAPH, int CAPM, int NCD, class T>
__device__ __forceinline__ void tile_tag_clear(TileShared<W, CAPH, CAPM, NCD, T>& sh, int sl) {
    if (CAPM > 0)
        sh.tag[sl] = -1;
    else
        atomicAnd(&sh.tagb[sl >> 5], ~(1u << (sl & 31)));
}

// Geometry of a tile's cell list: a cube of side 2 He centred on the cell, nc^3 cells of side f.
// A bead's tile coordinate is its minimum-image offset from the centre plus He.
struct TileGeo {
    double c[3];
    double He, f, invf;
    int nc;
};

__device__ __forceinline__ int tile_clamp(const TileGeo& tg, double u) {
    double q = floor(u * tg.invf);
    q = fmin(fmax(q, 0.0), (double)(tg.nc - 1));
    return (int)q;
}

__device__ __forceinline__ double tile_u(const Grid& g, const TileGeo& tg, double v, int a) {
    return minimg(g, v - tg.c[a]) + tg.He;
}
// tile coordinate of a stored position: absolute FP64, or an FP32 offset from the centre
__device__ __forceinline__ double tile_u(const Grid&, const TileGeo& tg, float v, int) { return (double)v + tg.He; }

// trial position of member k (tile slot sl)
template <int W, int CAPH, int CAPM, int NCD>
__device__ __forceinline__ void member_new(const TileShared<W, CAPH, CAPM, NCD>& sh, const Grid& g,
                                           const WaveDesc& wv, int k, int sl, double& nx, double& ny, double& nz) {
    if (CAPM > 0 && k < CAPM) {
        nx = sh.MX[k];
        ny = sh.MY[k];
        nz = sh.MZ[k];
    } else {
        double w0, w1, w2;
        wavelet_disp(g, wv, sh.x[sl], sh.y[sl], sh.z[sl], w0, w1, w2);
        nx = sh.x[sl] + w0;
        ny = sh.y[sl] + w1;
        nz = sh.z[sl] + w2;
    }
}

// The wavelet of the current test on an FP32 tile: centre as an FP32 offset from the tile centre,
// FP32 polarisation, radius and amplitude.
struct WaveDesc32 {
    float b[3], p[3], lam, invlam, A;
    int rot;
};

// FP32 displacement of the bead at tile offset (x, y, z): the two maps of wavelet_disp, with
// x_r = (r - b)/lambda from offsets (no minimum image: a tile is shorter than half the box)
__device__ __forceinline__ void wavelet_disp32(const WaveDesc32& wv, float x, float y, float z, float& w0, float& w1,
                                               float& w2) {
    const float xr0 = (x - wv.b[0]) * wv.invlam, xr1 = (y - wv.b[1]) * wv.invlam, xr2 = (z - wv.b[2]) * wv.invlam;
    const float rr = sqrtf((xr0 * xr0 + xr1 * xr1) + xr2 * xr2);
    if (wv.rot) {
        const float a = rr < 1.0f ? (wv.A * wv.invlam) * (1.0f - rr) : 0.0f;
        const float sa = sinf(a), hs = sinf(0.5f * a), omc = 2.0f * hs * hs;
        const float pd = (wv.p[0] * xr0 + wv.p[1] * xr1) + wv.p[2] * xr2;
        w0 = wv.lam * (sa * (wv.p[1] * xr2 - wv.p[2] * xr1) + omc * (wv.p[0] * pd - xr0));
        w1 = wv.lam * (sa * (wv.p[2] * xr0 - wv.p[0] * xr2) + omc * (wv.p[1] * pd - xr1));
        w2 = wv.lam * (sa * (wv.p[0] * xr1 - wv.p[1] * xr0) + omc * (wv.p[2] * pd - xr2));
        return;
    }
    const float f = rr < 1.0f ? wv.A * (1.0f - rr) : 0.0f;
    w0 = f * (wv.p[1] * xr2 - wv.p[2] * xr1);
    w1 = f * (wv.p[2] * xr0 - wv.p[0] * xr2);
    w2 = f * (wv.p[0] * xr1 - wv.p[1] * xr0);
}

// FP32 displacement of member k (tile slot sl): kept in MX/MY/MZ for the first CAPM members
template <int W, int CAPH, int CAPM, int NCD>
__device__ __forceinline__ void member_w32(const TileShared<W, CAPH, CAPM, NCD, float>& sh, const WaveDesc32& wv, int k,
                                           int sl, float& w0, float& w1, float& w2) {
    if (CAPM > 0 && k < CAPM) {
        w0 = sh.MX[k];
        w1 = sh.MY[k];
        w2 = sh.MZ[k];
    } else {
        wavelet_disp32(wv, sh.x[sl], sh.y[sl], sh.z[sl], w0, w1, w2);
    }
}

// FP32 squared distance of two tile offsets; wrap applies the minimum image (needed only once a
// tile with its drift spans more than the box minus the cut-off)
__device__ __forceinline__ float r2_f32(float dx, float dy, float dz, bool wrap, float Lf, float invLf) {
    if (wrap) {
        dx -= Lf * rintf(dx * invLf);
        dy -= Lf * rintf(dy * invLf);
        dz -= Lf * rintf(dz * invLf);
    }
    return (dx * dx + dy * dy) + dz * dz;
}

// exchanges at distance J inside one thread's 8 consecutive entries v[0..8) (first index i0),
// for the merge of blocks of size k
template <int J>
__device__ __forceinline__ void bitonic_regs(int32_t (&v)[8], int i0, int k) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int f = e ^ J;
        if (f > e) {
            const bool up = ((i0 + e) & k) == 0;
            const int32_t lo = v[e], hi = v[f];
            if ((lo > hi) == up) {
                v[e] = hi;
                v[f] = lo;
            }
        }
    }
}

// Bitonic sort of a[0..np2) in LDS (np2 a power of two). Each thread holds 8 consecutive entries
// in registers for every exchange at distance < 8; exchanges at distance >= 8 go through LDS,
// one pair per iteration.
template <int W>
__device__ void bitonic_sort(int32_t* a, int np2) {
    const int tid = threadIdx.x;
    if (np2 < 8 || np2 > 8 * W) {
        for (int k = 2; k <= np2; k <<= 1) {
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                for (int i = tid; i < np2; i += W) {
                    int l = i ^ jj;
                    if (l > i) {
                        int32_t va = a[i], vb = a[l];
                        bool up = (i & k) == 0;
                        if ((va > vb) == up) {
                            a[i] = vb;
                            a[l] = va;
                        }
                    }
                }
                __syncthreads();
            }
        }
        return;
    }
    const int nchunk = np2 >> 3;
    int32_t v[8];
    // blocks of 2, 4 and 8: within each thread's chunk
    if (tid < nchunk) {
        const int i0 = tid << 3;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = a[i0 + e];
        bitonic_regs<1>(v, i0, 2);
        bitonic_regs<2>(v, i0, 4);
        bitonic_regs<1>(v, i0, 4);
        bitonic_regs<4>(v, i0, 8);
        bitonic_regs<2>(v, i0, 8);
        bitonic_regs<1>(v, i0, 8);
#pragma unroll
        for (int e = 0; e < 8; ++e) a[i0 + e] = v[e];
    }
    __syncthreads();
    for (int k = 16; k <= np2; k <<= 1) {
        for (int jj = k >> 1; jj >= 8; jj >>= 1) {
            for (int q = tid; q < (np2 >> 1); q += W) {
                const int i = ((q / jj) * (jj << 1)) + (q % jj), l = i + jj;
                const int32_t va = a[i], vb = a[l];
                const bool up = (i & k) == 0;
                if ((va > vb) == up) {
                    a[i] = vb;
                    a[l] = va;
                }
            }
            __syncthreads();
        }
        if (tid < nchunk) {
            const int i0 = tid << 3;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = a[i0 + e];
            bitonic_regs<4>(v, i0, k);
            bitonic_regs<2>(v, i0, k);
            bitonic_regs<1>(v, i0, k);
#pragma unroll
            for (int e = 0; e < 8; ++e) a[i0 + e] = v[e];
        }
        __syncthreads();
    }
}

// tile cell of slot i
template <int W, int CAPH, int CAPM, int NCD, class T>
__device__ __forceinline__ int tile_key(const TileShared<W, CAPH, CAPM, NCD, T>& sh, int i, const Grid& g,
                                        const TileGeo& tg) {
    const int cx = tile_clamp(tg, tile_u(g, tg, sh.x[i], 0));
    const int cy = tile_clamp(tg, tile_u(g, tg, sh.y[i], 1));
    const int cz = tile_clamp(tg, tile_u(g, tg, sh.z[i], 2));
    return cx + tg.nc * (cy + tg.nc * cz);
}

// (re)build the tile cell list from the current tile positions, by counting sort: per-cell
// counts (two 16-bit counters per LDS word), their inclusive prefix (each cell's end), a
// scatter that takes positions down from each end (leaving each cell's start), and an
// insertion sort of every cell's few entries by slot. The result is the list sorted by
// (cell, slot), whatever order the atomics took.
template <int W, int CAPH, int CAPM, int NCD, class T>
__device__ void tile_index(TileShared<W, CAPH, CAPM, NCD, T>& sh, int nH, const Grid& g, const TileGeo& tg) {
    const int tid = threadIdx.x;
    const int NC = tg.nc * tg.nc * tg.nc;
    uint32_t* cw = reinterpret_cast<uint32_t*>(sh.cst);
    for (int w = tid; w < (NC + 2) / 2; w += W) cw[w] = 0u;
    __syncthreads();
    for (int i = tid; i < nH; i += W) {
        const int c = tile_key(sh, i, g, tg);
        atomicAdd(&cw[c >> 1], 1u << ((c & 1) << 4));
    }
    __syncthreads();
    // inclusive prefix over entries 0..NC, a contiguous chunk per thread
    const int per = (NC + 1 + W - 1) / W;
    const int c0 = min(NC + 1, tid * per), c1 = min(NC + 1, c0 + per);
    int run = 0;
    for (int c = c0; c < c1; ++c) run += sh.cst[c];
    int before;
    block_scan_count<W>(run, before, sh.redi);
    for (int c = c0; c < c1; ++c) {
        before += sh.cst[c];
        sh.cst[c] = (int16_t)before;
    }
    __syncthreads();
    for (int i = tid; i < nH; i += W) {
        const int c = tile_key(sh, i, g, tg);
        const int sh16 = (c & 1) << 4;
        const uint32_t old = atomicSub(&cw[c >> 1], 1u << sh16);
        const int pos = (int)((old >> sh16) & 0xFFFFu) - 1;
        sh.kc[pos] = (int16_t)i;
    }
    __syncthreads();
    for (int c = tid; c < NC; c += W) {
        const int b = sh.cst[c], e = sh.cst[c + 1];
        for (int p = b + 1; p < e; ++p) {
            const int16_t v = sh.kc[p];
            int q = p - 1;
            while (q >= b && sh.kc[q] > v) {
                sh.kc[q + 1] = sh.kc[q];
                --q;
            }
            sh.kc[q + 1] = v;
        }
    }
    __syncthreads();
}

// slot of bead j in the sorted tile, or -1
template <int W, int CAPH, int CAPM, int NCD, class T>
__device__ __forceinline__ int tile_find(const TileShared<W, CAPH, CAPM, NCD, T>& sh, int nH, int32_t j) {
    int lo = 0, hi = nH - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int32_t v = sh.id[mid] & ID_MASK;
        if (v == j) return mid;
        if (v < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// energy change of the current test over the tile: bonds and WCA pairs with >= 1 member, each
// once; members are tile slots sh.M[0..n) with tags set (trial positions via member_new).
// WCA partners come from the tile cell list: every bead within R (tile coordinates, per
// axis) of a member's current position, R covering the cut-off, both displacements and the
// drift since the list was built. One work item is a (member, y-z row of cells) pair whose
// x range is contiguous in the list.
// FP64 terms. On an FP32 tile (T = float, WV = WaveDesc32) this is the FP64 recheck: the same bonds and pairs
// (found from the FP32 tile), evaluated from the FP64 positions in HBM plus the FP32 displacements
// that an accept would apply.
// A wave with slack in the energy layout below, or -1: in the split layout the last pair wave when
// the pair items leave it idle (the bond wave is nearly as busy as the pair waves); otherwise the
// last wave when its lanes take fewer rounds of pair items than the first lanes.
template <int W>
__device__ __forceinline__ int tile_light_wave(bool split, int items, int G) {
    const int slots = items * G;
    if (split) return slots <= W - 128 ? W / 64 - 2 : -1;
    const int first = (slots + W - 1) / W, last = slots > W - 1 ? (slots - W) / W + 1 : 0;
    return last < first ? W / 64 - 1 : -1;
}

// returns a wave with slack (tile_light_wave)
template <int W, int CAPH, int CAPM, int NCD, class T = double, class WV = WaveDesc>
__device__ int tile_dU(const DevParams& P, const DevPtrs& D, const SysDesc& s,
                        const TileShared<W, CAPH, CAPM, NCD, T>& sh, const Grid& g, const TileGeo& tg,
                        const WV& wv, double R,
                        int nH, int n, double& acc, unsigned long long& viol, float rc2g = 0.0f,
                        double Rp2 = INFINITY) {
    constexpr bool F32 = std::is_same<T, float>::value;
    auto cur = [&](int sl, double& x, double& y, double& z) {
        if constexpr (F32) {
            const int32_t j = sh.id[sl] & ID_MASK;
            x = D.x[j];
            y = D.y[j];
            z = D.z[j];
        } else {
            x = sh.x[sl];
            y = sh.y[sl];
            z = sh.z[sl];
        }
    };
    auto trial = [&](int k, int sl, double& x, double& y, double& z) {
        if constexpr (F32) {
            cur(sl, x, y, z);
            float w0, w1, w2;
            member_w32(sh, wv, k, sl, w0, w1, w2);
            x += (double)w0;
            y += (double)w1;
            z += (double)w2;
        } else {
            member_new(sh, g, wv, k, sl, x, y, z);
        }
    };
    const int tid = threadIdx.x;
    const double L = s.L, invL = s.invL;
    const int NR = min(tg.nc, (int)floor(2.0 * R * tg.invf) + 2);
    const int per = NR * NR;
    const int items = n * per;
    // in a 256-thread tile, bonds on the last wave and pair items on the others when the items
    // fit there: the two chains of dependent loads then run on different SIMDs at once (in the
    // 512-thread tile the pair items need every lane)
    const bool split = W == 256 && P.bond_type != WMC_BOND_NONE && P.wca && items <= W - 64;
    const int b0 = split ? tid - (W - 64) : tid, bstride = split ? 64 : W;
    const int p0 = split ? (tid < W - 64 ? tid : 0x3FFFFFFF) : tid, pstride = split ? W - 64 : W;
    // lanes per pair item: when the items leave lanes idle, G lanes share an item's row of beads
    // (each takes every G-th), so a lane walks fewer pairs in sequence
    int G = 1;
    while (G < 8 && items * 2 * G <= pstride) G <<= 1;
    if (P.bond_type != WMC_BOND_NONE) {
        for (int k = b0 < 0 ? n : b0; k < n; k += bstride) {
            const int sl = sh.M[k];
            const int32_t raw = sh.id[sl];
            const int32_t j = raw & ID_MASK;
            double jx, jy, jz, kx, ky, kz;
            cur(sl, jx, jy, jz);
            trial(k, sl, kx, ky, kz);
            for (int e = 0; e < 2; ++e) {
                bool bonded = e == 0 ? (raw & ID_NEXT) != 0 : ((uint32_t)raw & ID_PREV) != 0;
                if (!bonded) continue;
                const int32_t m = e == 0 ? j + 1 : j - 1;
                int ps = e == 0 ? sl + 1 : sl - 1;
                if (ps < 0 || ps >= nH || (sh.id[ps] & ID_MASK) != m) ps = tile_find(sh, nH, m);
                double mx, my, mz, nx, ny, nz;
                if (ps >= 0) {
                    const int tm = tile_tag(sh, ps);
                    if (tm >= 0 && ps < sl) continue;
                    cur(ps, mx, my, mz);
                    nx = mx;
                    ny = my;
                    nz = mz;
                    if (tm >= 0) trial(tm, ps, nx, ny, nz);
                } else {
                    // partner beyond the halo: only a bond longer than r_int can do this
                    mx = nx = D.x[m];
                    my = ny = D.y[m];
                    mz = nz = D.z[m];
                }
                double r2o = pair_r2(P, invL, L, jx, jy, jz, mx, my, mz);
                double r2n = pair_r2(P, invL, L, kx, ky, kz, nx, ny, nz);
                if (r2o > P.r_int * P.r_int) ++viol;
                acc += u_bond_delta(P, r2n, r2o);
            }
        }
    }
    if (P.wca) {
        for (int ig = p0; ig < items * G; ig += pstride) {
            const int it = ig / G, sub = ig - it * G;
            const int k = it / per, q = it - k * per;
            const int qy = q % NR, qz = q / NR;
            const int sl = sh.M[k];
            double jx, jy, jz;
            cur(sl, jx, jy, jz);
            const double uy = tile_u(g, tg, sh.y[sl], 1), uz = tile_u(g, tg, sh.z[sl], 2);
            const int cy = tile_clamp(tg, uy - R) + qy, cz = tile_clamp(tg, uz - R) + qz;
            if (cy > tile_clamp(tg, uy + R) || cz > tile_clamp(tg, uz + R)) continue;
            const double ux = tile_u(g, tg, sh.x[sl], 0);
            const int row = tg.nc * (cy + tg.nc * cz);
            const int p0 = sh.cst[row + tile_clamp(tg, ux - R)], p1 = sh.cst[row + tile_clamp(tg, ux + R) + 1];
            double kx, ky, kz;
            trial(k, sl, kx, ky, kz);
            float mw0 = 0.0f, mw1 = 0.0f, mw2 = 0.0f;
            if constexpr (F32) member_w32(sh, wv, k, sl, mw0, mw1, mw2);
            for (int pp = p0 + sub; pp < p1; pp += G) {
                const int m = sh.kc[pp];
                if (m == sl) continue;
                const int tm = tile_tag(sh, m);
                if (tm >= 0 && m < sl) continue;
                if constexpr (F32) {
                    // FP32 tile: only pairs that FP32 places within the widened cut-off can be within
                    // the cut-off in FP64 (rc2g exceeds the FP32 error of r2), so only those are read
                    // from HBM
                    // (a pair whose offsets differ by half the box or more is always read)
                    float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
                    if (tm >= 0) member_w32(sh, wv, tm, m, v0, v1, v2);
                    const float ex = sh.x[sl] - sh.x[m], ey = sh.y[sl] - sh.y[m], ez = sh.z[sl] - sh.z[m];
                    const float ro = (ex * ex + ey * ey) + ez * ez;
                    const float fx = ex + (mw0 - v0), fy = ey + (mw1 - v1), fz = ez + (mw2 - v2);
                    const float rn = (fx * fx + fy * fy) + fz * fz;
                    if (fminf(ro, rn) >= rc2g &&
                        (!g.periodic || 2.0f * (fabsf(ex) + fabsf(ey) + fabsf(ez)) < (float)L))
                        continue;
                }
                double mx, my, mz;
                cur(m, mx, my, mz);
                double r2o = pair_r2(P, invL, L, jx, jy, jz, mx, my, mz);
                // a pair further apart than r_cut + 2 dmax stays beyond the cut-off after the move
                if (r2o > Rp2) continue;
                double nx = mx, ny = my, nz = mz;
                if (tm >= 0) trial(tm, m, nx, ny, nz);
                double r2n = pair_r2(P, invL, L, kx, ky, kz, nx, ny, nz);
                if (r2o < P.rc2 || r2n < P.rc2) acc += u_pair(P, r2n) - u_pair(P, r2o);
            }
        }
    }
    return tile_light_wave<W>(split, items, G);
}

// Energy change of the current test on an FP32 tile: the bonds and pairs of tile_dU, with FP32
// distances between tile offsets and FP32 terms; each term's difference is summed in FP64 (acc).
// s1 and s2 sum every counted term's sensitivity and sensitivity / r for the recheck margin; a
// pair that FP32 places just outside the cut-off (r2 < rc2g) adds the sensitivity at the cut-off.
template <int W, int CAPH, int CAPM, int NCD>
__device__ int tile_dU32(const DevParams& P, const DevPtrs& D, const TileShared<W, CAPH, CAPM, NCD, float>& sh,
                          const Grid& g, const TileGeo& tg, const WaveDesc32& wv, double R, int nH, int n, bool wrap,
                          float Lf, float invLf, float rc2f, float rc2g, float Rp2f, double& acc, float& s1,
                          float& s2, unsigned long long& viol) {
    // the margin sums need only a few correct digits: hardware reciprocal square root (1 ulp)
    auto rsq = [](float v) { return __builtin_amdgcn_rsqf(v); };
    const int tid = threadIdx.x;
    const float rint2 = (float)(P.r_int * P.r_int);
    const int NR = min(tg.nc, (int)floor(2.0 * R * tg.invf) + 2);
    const int per = NR * NR;
    const int items = n * per;
    const bool split = W == 256 && P.bond_type != WMC_BOND_NONE && P.wca && items <= W - 64;
    const int b0 = split ? tid - (W - 64) : tid, bstride = split ? 64 : W;
    const int p0 = split ? (tid < W - 64 ? tid : 0x3FFFFFFF) : tid, pstride = split ? W - 64 : W;
    // lanes per pair item: when the items leave lanes idle, G lanes share an item's row of beads
    // (each takes every G-th), so a lane walks fewer pairs in sequence
    int G = 1;
    while (G < 8 && items * 2 * G <= pstride) G <<= 1;
    if (P.bond_type != WMC_BOND_NONE) {
        for (int k = b0 < 0 ? n : b0; k < n; k += bstride) {
            const int sl = sh.M[k];
            const int32_t raw = sh.id[sl];
            const int32_t j = raw & ID_MASK;
            const float jx = sh.x[sl], jy = sh.y[sl], jz = sh.z[sl];
            float w0, w1, w2;
            member_w32(sh, wv, k, sl, w0, w1, w2);
            const float kx = jx + w0, ky = jy + w1, kz = jz + w2;
            for (int e = 0; e < 2; ++e) {
                bool bonded = e == 0 ? (raw & ID_NEXT) != 0 : ((uint32_t)raw & ID_PREV) != 0;
                if (!bonded) continue;
                const int32_t m = e == 0 ? j + 1 : j - 1;
                int ps = e == 0 ? sl + 1 : sl - 1;
                if (ps < 0 || ps >= nH || (sh.id[ps] & ID_MASK) != m) ps = tile_find(sh, nH, m);
                float mx, my, mz, nx, ny, nz;
                if (ps >= 0) {
                    const int tm = tile_tag(sh, ps);
                    if (tm >= 0 && ps < sl) continue;
                    mx = nx = sh.x[ps];
                    my = ny = sh.y[ps];
                    mz = nz = sh.z[ps];
                    if (tm >= 0) {
                        float v0, v1, v2;
                        member_w32(sh, wv, tm, ps, v0, v1, v2);
                        nx += v0;
                        ny += v1;
                        nz += v2;
                    }
                } else {
                    // partner beyond the halo: only a bond longer than r_int can do this
                    mx = nx = (float)minimg(g, D.x[m] - tg.c[0]);
                    my = ny = (float)minimg(g, D.y[m] - tg.c[1]);
                    mz = nz = (float)minimg(g, D.z[m] - tg.c[2]);
                }
                const float r2o = r2_f32(jx - mx, jy - my, jz - mz, wrap, Lf, invLf);
                const float r2n = r2_f32(kx - nx, ky - ny, kz - nz, wrap, Lf, invLf);
                if (r2o > rint2) ++viol;
                float sn, so;
                acc += (double)(u_bond_f32(P, r2n, sn) - u_bond_f32(P, r2o, so));
                s1 += sn + so;
                s2 += sn * rsq(r2n) + so * rsq(r2o);
            }
        }
    }
    if (P.wca) {
        const float sc = 12.0f * (float)P.eps;  // sensitivity at the cut-off, 4 eps (6/4 + 3/2)
        for (int ig = p0; ig < items * G; ig += pstride) {
            const int it = ig / G, sub = ig - it * G;
            const int k = it / per, q = it - k * per;
            const int qy = q % NR, qz = q / NR;
            const int sl = sh.M[k];
            const float jx = sh.x[sl], jy = sh.y[sl], jz = sh.z[sl];
            const double uy = tile_u(g, tg, jy, 1), uz = tile_u(g, tg, jz, 2);
            const int cy = tile_clamp(tg, uy - R) + qy, cz = tile_clamp(tg, uz - R) + qz;
            if (cy > tile_clamp(tg, uy + R) || cz > tile_clamp(tg, uz + R)) continue;
            const double ux = tile_u(g, tg, jx, 0);
            const int row = tg.nc * (cy + tg.nc * cz);
            const int q0 = sh.cst[row + tile_clamp(tg, ux - R)], q1 = sh.cst[row + tile_clamp(tg, ux + R) + 1];
            float w0, w1, w2;
            member_w32(sh, wv, k, sl, w0, w1, w2);
            const float kx = jx + w0, ky = jy + w1, kz = jz + w2;
            for (int pp = q0 + sub; pp < q1; pp += G) {
                const int m = sh.kc[pp];
                if (m == sl) continue;
                const int tm = tile_tag(sh, m);
                if (tm >= 0 && m < sl) continue;
                const float mx = sh.x[m], my = sh.y[m], mz = sh.z[m];
                const float r2o = r2_f32(jx - mx, jy - my, jz - mz, wrap, Lf, invLf);
                // beyond r_cut + 2 dmax (widened past rc2g's widening and the FP32 error) a pair's new
                // FP32 distance also lies beyond rc2g: it adds nothing, margin sums included
                if (r2o > Rp2f) continue;
                float nx = mx, ny = my, nz = mz;
                if (tm >= 0) {
                    float v0, v1, v2;
                    member_w32(sh, wv, tm, m, v0, v1, v2);
                    nx += v0;
                    ny += v1;
                    nz += v2;
                }
                const float r2n = r2_f32(kx - nx, ky - ny, kz - nz, wrap, Lf, invLf);
                const float m2 = fminf(r2o, r2n);
                if (m2 < rc2f) {
                    float sn, so;
                    acc += (double)(u_pair_f32(P, r2n, rc2f, sn) - u_pair_f32(P, r2o, rc2f, so));
                    s1 += sn + so;
                    s2 += sn * rsq(r2n) + so * rsq(r2o);
                } else if (m2 < rc2g) {
                    s1 += sc;
                    s2 += sc * rsq(m2);
                }
            }
        }
    }
    return tile_light_wave<W>(split, items, G);
}

// returns false (before any move) when the halo does not fit; the caller then uses the
// global path for this cell. Dg bounds the drift, since the neighbour grid was built, of every bead
// the cell can meet; the largest drift of the beads the cell moves is returned in dl_out.
template <int W, int CAPH, int CAPM, int NCD, bool VAR, class T>
__device__ __forceinline__ bool process_cell_tile(const DevParams& P, const DevPtrs& D, TileShared<W, CAPH, CAPM, NCD, T>& sh, int sys,
                                  int level, int colour, int64_t local, int64_t sweep, const Grid& g,
                                  const double Dg, double& dl_out) {
    const SysDesc& s = D.sys[sys];
    const LevelDesc& lv = D.lev[s.lvl_off + level];
    const int tid = threadIdx.x;
    int64_t ic[3];
    cell_coords(P, lv, g, colour, local, ic);
    const int64_t cell = ic[0] + g.n[0] * (ic[1] + g.n[1] * ic[2]);
    const int64_t key = cell_key(g, ic);
    const double hi2 = lv.hi * lv.hi;
    const double rh = lv.hi + lv.r_int, rh2 = rh * rh;
    const double L = s.L, invL = s.invL;
    dl_out = 0.0;
    ExchPh xp;  // toggles of the one-barrier reductions
    // FP32 tile (mixed precision): offsets from the tile centre, the FP64 positions in HBM
    constexpr bool F32 = std::is_same<T, float>::value;

    // tile cell list geometry; relative tile coordinates identify pairs only while the tile
    // (plus a cut-off and a margin for moves) is shorter than the box
    TileGeo tg;
    for (int a = 0; a < 3; ++a) tg.c[a] = g.o[a] + ((double)ic[a] + 0.5) * g.h;
    tg.He = 0.5 * g.h + rh + Dg + 1e-9 * L;
    if (2.0 * tg.He + P.rc + 2.0 >= L) return false;
    tg.nc = max(1, min(NCD, (int)floor(2.0 * tg.He / (fmax(P.rc, 0.5) + 0.5))));
    tg.f = 2.0 * tg.He / (double)tg.nc;
    tg.invf = 1.0 / tg.f;

    // ---- 1. halo gather from the neighbour grid
    if (tid == 0) sh.count = 0;
    __syncthreads();
    {
        double R = rh + Dg + 1e-9 * L;
        int f0[3], cn[3];
        for (int a = 0; a < 3; ++a) {
            double lo = g.o[a] + (double)ic[a] * g.h - R;
            fine_range(lo, lo + g.h + 2.0 * R, s.invg, s.nf, f0[a], cn[a]);
        }
        // each (y, z) row of the box is one run of consecutive fine cells in x, so its beads are
        // one contiguous range of the sorted index (two where the box wraps in x): the ranges and
        // their prefix go into the position arrays (free until the sort below), then every
        // thread takes beads t, t + W, ... of the concatenation
        const bool wrapx = f0[0] + cn[0] > s.nf;
        const int nseg = cn[1] * cn[2] * (wrapx ? 2 : 1);
        int32_t* segB = reinterpret_cast<int32_t*>(sh.x);  // first index entry of each range
        int32_t* segP = reinterpret_cast<int32_t*>(sh.y);  // exclusive prefix of the range lengths
        if (nseg + 1 <= (int)(sizeof(T) / 4) * CAPH) {
            for (int q = tid; q < nseg; q += W) {
                const int r = wrapx ? (q >> 1) : q, part = wrapx ? (q & 1) : 0;
                const int fy = (f0[1] + r % cn[1]) % s.nf, fz = (f0[2] + r / cn[1]) % s.nf;
                const int64_t rowb = s.fine_off + (int64_t)s.nf * (fy + (int64_t)s.nf * fz);
                const int xa = part ? 0 : f0[0];
                const int xb = wrapx ? (part ? f0[0] + cn[0] - 1 - s.nf : s.nf - 1) : f0[0] + cn[0] - 1;
                const int a = D.fstart[rowb + xa];
                segB[q] = a;
                segP[q] = D.fstart[rowb + xb + 1] - a;
            }
            __syncthreads();
            const int per = (nseg + W - 1) / W;
            const int c0 = min(nseg, tid * per), c1 = min(nseg, c0 + per);
            int run = 0;
            for (int c = c0; c < c1; ++c) run += segP[c];
            int before;
            const int total = xscan_count<W>(run, before, sh.xc, xp);
            for (int c = c0; c < c1; ++c) {
                const int v = segP[c];
                segP[c] = before;
                before += v;
            }
            if (tid == 0) segP[nseg] = total;
            __syncthreads();
            for (int t = tid; t < total; t += W) {
                // the last range starting at or before t (it holds t: the next one starts after it)
                int lo = 0, hi = nseg - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (segP[mid] <= t) lo = mid; else hi = mid - 1;
                }
                const int32_t j = D.fidx[segB[lo] + (t - segP[lo])];
                if (dist2_cell(g, ic, D.x[j], D.y[j], D.z[j]) <= rh2) {
                    int idx = atomicAdd(&sh.count, 1);
                    if (idx < CAPH) sh.id[idx] = j;
                }
            }
        } else {
            const int total = cn[0] * cn[1] * cn[2];
            for (int q = tid; q < total; q += W) {
                int qx = q % cn[0], qy = (q / cn[0]) % cn[1], qz = q / (cn[0] * cn[1]);
                int fx = (f0[0] + qx) % s.nf, fy = (f0[1] + qy) % s.nf, fz = (f0[2] + qz) % s.nf;
                int64_t fc = s.fine_off + fx + (int64_t)s.nf * (fy + (int64_t)s.nf * fz);
                for (int k = D.fstart[fc]; k < D.fstart[fc + 1]; ++k) {
                    int32_t j = D.fidx[k];
                    if (dist2_cell(g, ic, D.x[j], D.y[j], D.z[j]) <= rh2) {
                        int idx = atomicAdd(&sh.count, 1);
                        if (idx < CAPH) sh.id[idx] = j;
                    }
                }
            }
        }
    }
    __syncthreads();
    const int nH = sh.count;
    if (nH > CAPH) return false;
    // ---- 2. sort by bead index (bitonic), then positions, bond flags and the reach list
    {
        int np2 = 1;
        while (np2 < nH) np2 <<= 1;
        for (int i = nH + tid; i < np2; i += W) sh.id[i] = 0x7FFFFFFF;
        __syncthreads();
        bitonic_sort<W>(sh.id, np2);
    }
    if (CAPM == 0)
        for (int w = tid; w < (nH + 31) / 32; w += W) sh.tagb[w] = 0u;
    int nS = 0;
    for (int c0 = 0; c0 < nH; c0 += W) {
        int i = c0 + tid;
        bool f = false;
        if (i < nH) {
            int32_t j = sh.id[i];
            double x = D.x[j], y = D.y[j], z = D.z[j];
            if constexpr (F32) {
                sh.x[i] = (float)minimg(g, x - tg.c[0]);
                sh.y[i] = (float)minimg(g, y - tg.c[1]);
                sh.z[i] = (float)minimg(g, z - tg.c[2]);
            } else {
                sh.x[i] = x;
                sh.y[i] = y;
                sh.z[i] = z;
            }
            if (CAPM > 0) sh.tag[i] = -1;
            int32_t fl = j;
            if (j + 1 < s.b1 && D.bond_next[j]) fl |= ID_NEXT;
            if (j > s.b0 && D.bond_next[j - 1]) fl = (int32_t)((uint32_t)fl | ID_PREV);
            sh.id[i] = fl;
            f = dist2_cell(g, ic, x, y, z) <= hi2;
        }
        int before;
        int tot = xscan_flag<W>(f, before, sh.xc, xp);
        if (f) sh.S[nS + before] = (int16_t)i;
        nS += tot;
    }
    __syncthreads();
    tile_index<W, CAPH, CAPM, NCD>(sh, nH, g, tg);
    double E = 0.0;     // bound on any tile bead's displacement since the cell list was built
    double Etot = 0.0;  // ... since the tile was loaded (bounds the FP32 offsets with He)

    // ---- 3. trials and chains (as the global path, on LDS)
    const bool uni = VAR && P.centring == WMC_CENTRE_UNIFORM;
    double mu = uni ? lv.T / ((double)g.n[0] * (double)g.n[1] * (double)g.n[2]) : (lv.T * (double)nS) / (double)s.N;
    int64_t K = (int64_t)floor(mu);
    {
        Stream ms;
        ms.init(P, sys, sweep, TAG_META + level, key, 0, 0, 0);
        if (ms.co() < mu - (double)K) K += 1;
    }
    if (K > 0xFFFFF) {
        K = 0xFFFFF;
        if (tid == 0) atomicAdd(&D.cnt[CNT_VIOL], 1ull);
    }
    unsigned long long c_hits = 0, c_att = 0, c_acc = 0, c_caps = 0, c_redraw = 0, c_beads = 0, c_viol = 0;
    unsigned long long c_mre = 0;  // FP32 support tests rechecked in FP64
    double d_local = 0.0;
    // trials are drawn W at a time (one per lane); the draws (lambda, anchor, ball vector, stream
    // position) do not depend on positions, so a lane keeps its trial across the chains of earlier
    // hits and only its hit test, which reads the anchor's current position, is repeated (a uniform
    // centre is drawn whole and kept in the ball vector's place)
    auto slot_of = [&](int64_t i) -> int32_t { return (int32_t)sh.S[i]; };
    // FP64 position of a tile slot (centres decide cells, so they are drawn in FP64: from LDS, or
    // from HBM for an FP32 tile)
    auto slot_pos = [&](int32_t sl, double& px, double& py, double& pz) {
        if constexpr (F32) {
            const int32_t j = sh.id[sl] & ID_MASK;
            px = D.x[j];
            py = D.y[j];
            pz = D.z[j];
        } else {
            px = sh.x[sl];
            py = sh.y[sl];
            pz = sh.z[sl];
        }
    };
    // FP32 tile, anchored centre b = r_a + lam V: its offset f from the tile centre (= the cell's
    // centre) is o_a + lam V in FP32, within eps (2 He' + lam) of the exact offset; the cell test
    // |f| < h/2 per axis is exact unless f lies within 16 times that of a face, where the FP64 test
    // runs on the anchor's position from HBM
    const float hh = (float)g.half;
    auto hit_f32 = [&](int a, double lm, double vx, double vy, double vz, float& f0, float& f1, float& f2) -> bool {
        f0 = sh.x[a] + (float)(lm * vx);
        f1 = sh.y[a] + (float)(lm * vy);
        f2 = sh.z[a] + (float)(lm * vz);
        const float m = fmaxf(fabsf(f0), fmaxf(fabsf(f1), fabsf(f2)));
        const float tb = (float)(0x1p-20 * (tg.He + Etot + lm));
        if (m < hh - tb) return true;
        if (m > hh + tb) return false;
        double ax, ay, az;
        slot_pos(a, ax, ay, az);
        return cell_of_point(g, ax + lm * vx, ay + lm * vy, az + lm * vz) == cell;
    };
    // one try of a recycling redraw (retry rn of trial tc, try jj): anchor and ball vector, or a
    // uniform centre, and whether the centre lies in the cell
    auto redraw_try = [&](int64_t tc, int rn, int jj, double lam, Stream& rs, int& a2, double& ex, double& ey,
                          double& ez, float& g0, float& g1, float& g2) -> bool {
        rs.init(P, sys, sweep, level, key, tc, rn, jj);
        if (F32 && !uni) {
            // the draws of draw_trial_centre (anchor, then ball vector), FP32 cell test
            a2 = slot_of(rs.index(nS));
            ball(rs, ex, ey, ez);
            return hit_f32(a2, lam, ex, ey, ez, g0, g1, g2);
        }
        const bool h = draw_trial_centre<VAR>(P, rs, g, ic, cell, lam, nS, slot_of, slot_pos, a2, ex, ey, ez);
        if (F32) {
            g0 = (float)minimg(g, ex - tg.c[0]);
            g1 = (float)minimg(g, ey - tg.c[1]);
            g2 = (float)minimg(g, ez - tg.c[2]);
        }
        return h;
    };
    // The first 16 tries of the redraw that follows a rejection, taken speculatively while the test
    // is evaluated: a rejected test moves nothing, so they see the positions the redraw would see.
    // A wave with slack in the energy sum takes them after its own work (with none, the redraw runs
    // as usual); the first hit goes to pub_* (read again only after a redraw; an accepted test ends
    // the chain, whose successor publishes its own centre) and its try index, or -1, to spec_found,
    // both read after the reduction barrier of the energy sum. Wider tiles only.
    constexpr bool SPEC = W >= 256;
    auto spec_redraw = [&](int64_t tc, int rn, double lam, int wave) {
        if ((tid >> 6) != wave) return;
        const int lane = tid & 63;
        bool h2 = false;
        double ex = 0, ey = 0, ez = 0;
        float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
        int a2 = 0;
        Stream rs;
        if (lane < 16) h2 = redraw_try(tc, rn, lane, lam, rs, a2, ex, ey, ez, g0, g1, g2);
        const uint64_t hits = __ballot(h2);
        const int fj = hits ? __builtin_ctzll(hits) : -1;
        if (lane == fj) {
            sh.pub_a = a2;
            sh.pub_b[0] = ex;
            sh.pub_b[1] = ey;
            sh.pub_b[2] = ez;
            sh.pub_bf[0] = g0;
            sh.pub_bf[1] = g1;
            sh.pub_bf[2] = g2;
            sh.pub_next = rs.next;
        }
        if (lane == 0) sh.spec_found = fj;
    };
    for (int64_t t0 = 0; t0 < K; t0 += W) {
        const int64_t t = t0 + tid;
        const bool drawn = t < K && (nS > 0 || uni);
        double lam_t = 0.0, vx_t = 0.0, vy_t = 0.0, vz_t = 0.0;
        int as_t = 0;
        uint32_t next_t = 0;
        if (drawn) {
            Stream st;
            st.init(P, sys, sweep, level, key, t, 0, 0);
            lam_t = draw_lambda(st.co(), lv.lo, lv.hi);
            if (uni) {
                as_t = -1;
                vx_t = g.o[0] + ((double)ic[0] + st.co()) * g.h;
                vy_t = g.o[1] + ((double)ic[1] + st.co()) * g.h;
                vz_t = g.o[2] + ((double)ic[2] + st.co()) * g.h;
            } else {
                as_t = sh.S[st.index(nS)];
                ball(st, vx_t, vy_t, vz_t);
            }
            next_t = st.next;
        }
      for (int from = 0;;) {
        bool hit = false;
        double bx = 0.0, by = 0.0, bz = 0.0;
        float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
        if (drawn && tid >= from) {
            if (uni) {
                bx = vx_t;
                by = vy_t;
                bz = vz_t;
                hit = cell_of_point(g, bx, by, bz) == cell;
                if (F32) {
                    f0 = (float)minimg(g, bx - tg.c[0]);
                    f1 = (float)minimg(g, by - tg.c[1]);
                    f2 = (float)minimg(g, bz - tg.c[2]);
                }
            } else if (F32) {
                bx = vx_t;
                by = vy_t;
                bz = vz_t;
                hit = hit_f32(as_t, lam_t, vx_t, vy_t, vz_t, f0, f1, f2);
            } else {
                double ax, ay, az;
                slot_pos(as_t, ax, ay, az);
                bx = ax + lam_t * vx_t;
                by = ay + lam_t * vy_t;
                bz = az + lam_t * vz_t;
                hit = cell_of_point(g, bx, by, bz) == cell;
            }
        }
        int first = xmin_int<W>(hit ? tid : 0x7FFFFFFF, sh.xc, xp);
        if (first == 0x7FFFFFFF) break;
        if (tid == first) {
            sh.pub_lam = lam_t;
            sh.pub_a = as_t;
            sh.pub_b[0] = bx;
            sh.pub_b[1] = by;
            sh.pub_b[2] = bz;
            sh.pub_bf[0] = f0;
            sh.pub_bf[1] = f1;
            sh.pub_bf[2] = f2;
            sh.pub_next = next_t;
        }
        __syncthreads();
        const int64_t tc = t0 + first;
        double lam = sh.pub_lam;
        int as = sh.pub_a;
        // the chain's centre: kept in registers on an FP64 tile; an FP32 tile reads it from LDS
        // where needed (pub_b, pub_bf hold it until the chain's next redraw)
        double b[3] = {0.0, 0.0, 0.0};
        if constexpr (!F32) {
            b[0] = sh.pub_b[0];
            b[1] = sh.pub_b[1];
            b[2] = sh.pub_b[2];
        }
        uint32_t nxt = sh.pub_next;
        int jtry = 0;
        ++c_hits;
        const double lam2 = lam * lam;
        for (int r = 0;;) {
            Stream cs;
            cs.init(P, sys, sweep, level, key, tc, r, jtry);
            cs.next = nxt;
            double px, py, pz;
            direction(cs, px, py, pz);
            const double u_acc = cs.oc();
            // support test: FP64, or (FP32 tile) FP32 offsets with an FP64 recheck from HBM of every
            // bead within the FP32 error bound of the sphere: the offsets carry at most eps He', the
            // difference and sum their own rounding, so |d2_32 - d2| <= eps (7 lam He' + 6.5 lam^2)
            // near |d| = lam (eps = 2^-24, He' = tile half-width plus drift); tolm is 16 times that
            float bf0 = 0.0f, bf1 = 0.0f, bf2 = 0.0f, lam2f = 0.0f, tolm = 0.0f;
            if constexpr (F32) {
                bf0 = sh.pub_bf[0];
                bf1 = sh.pub_bf[1];
                bf2 = sh.pub_bf[2];
                lam2f = (float)lam2;
                tolm = (float)(0x1p-20 * (lam * (tg.He + Etot) + 2.0 * lam2));
            }
            auto in_ball = [&](int sl) -> bool {
                if constexpr (F32) {
                    if (sl == as) return true;
                    const float dx = sh.x[sl] - bf0, dy = sh.y[sl] - bf1, dz = sh.z[sl] - bf2;
                    const float d2 = (dx * dx + dy * dy) + dz * dz;
                    if (fabsf(d2 - lam2f) > tolm) return d2 <= lam2f;
                    ++c_mre;
                    // the FP64 centre (pub_b holds V for an anchored centre)
                    double cb[3] = {sh.pub_b[0], sh.pub_b[1], sh.pub_b[2]};
                    if (!uni) {
                        double ax, ay, az;
                        slot_pos(as, ax, ay, az);
                        cb[0] = ax + lam * cb[0];
                        cb[1] = ay + lam * cb[1];
                        cb[2] = az + lam * cb[2];
                    }
                    const int32_t j = sh.id[sl] & ID_MASK;
                    const double ex = minimg(g, D.x[j] - cb[0]), ey = minimg(g, D.y[j] - cb[1]),
                                 ez = minimg(g, D.z[j] - cb[2]);
                    return ((ex * ex + ey * ey) + ez * ez) <= lam2;
                } else {
                    const double dx = minimg(g, sh.x[sl] - b[0]), dy = minimg(g, sh.y[sl] - b[1]),
                                 dz = minimg(g, sh.z[sl] - b[2]);
                    return ((dx * dx + dy * dy) + dz * dz) <= lam2 || sl == as;
                }
            };
            // (no barrier here: whatever a test reads from LDS before its member scan, the centre in
            // pub_* included, was written before a barrier)
            int n = 0;
            int own_k = -1, own_sl = 0;  // a one-round scan's member of this thread
            if (W >= 256 && nS > W && nS <= 32 * W) {
                // q consecutive reach entries per thread, one workgroup scan (member order kept);
                // a one-wave tile keeps the round-by-round scan, which measured faster there
                const int q = (nS + W - 1) / W, i0 = tid * q;
                uint32_t mask = 0;
                for (int u = 0; u < q; ++u) {
                    const int i = i0 + u;
                    if (i < nS && in_ball(sh.S[i])) mask |= 1u << u;
                }
                int before;
                n = xscan_count<W>(__popc(mask), before, sh.xc, xp);
                for (int u = 0; u < q; ++u)
                    if ((mask >> u) & 1u) sh.M[before++] = sh.S[i0 + u];
            } else if (nS <= W) {
                // one round: a thread holds at most one member and displaces it itself below, so the
                // member list needs no barrier before the displacements
                bool f = false;
                int sl = 0;
                if (tid < nS) {
                    sl = sh.S[tid];
                    f = in_ball(sl);
                }
                int before;
                n = xscan_flag<W>(f, before, sh.xc, xp);
                if (f) {
                    sh.M[before] = (int16_t)sl;
                    own_k = before;
                    own_sl = sl;
                }
            } else {
                for (int c0 = 0; c0 < nS; c0 += W) {
                    int i = c0 + tid;
                    bool f = false;
                    int sl = 0;
                    if (i < nS) {
                        sl = sh.S[i];
                        f = in_ball(sl);
                    }
                    int before;
                    int tot = xscan_flag<W>(f, before, sh.xc, xp);
                    if (f) sh.M[n + before] = (int16_t)sl;
                    n += tot;
                }
            }
            if (nS > W) __syncthreads();
            WaveDesc wv;
            wv.b[0] = b[0];
            wv.b[1] = b[1];
            wv.b[2] = b[2];
            wv.p[0] = px;
            wv.p[1] = py;
            wv.p[2] = pz;
            wv.lam = lam;
            wv.A = wavelet_amp<VAR>(P, s, lam, n);
            wv.rot = VAR && P.wavelet_map == WMC_MAP_ROTATION;
            WaveDesc32 wv32;
            double dmax_l = 0.0;
            if constexpr (F32) {
                wv32.b[0] = bf0;
                wv32.b[1] = bf1;
                wv32.b[2] = bf2;
                wv32.p[0] = (float)px;
                wv32.p[1] = (float)py;
                wv32.p[2] = (float)pz;
                wv32.lam = (float)lam;
                wv32.invlam = (float)(1.0 / lam);
                wv32.A = (float)wv.A;
                wv32.rot = wv.rot;
                for (int k = nS <= W ? own_k : tid; k >= 0 && k < n; k += nS <= W ? n : W) {
                    const int sl = nS <= W ? own_sl : sh.M[k];
                    float w0, w1, w2;
                    wavelet_disp32(wv32, sh.x[sl], sh.y[sl], sh.z[sl], w0, w1, w2);
                    if (CAPM > 0 && k < CAPM) {
                        sh.MX[k] = w0;
                        sh.MY[k] = w1;
                        sh.MZ[k] = w2;
                    }
                    tile_tag_set(sh, sl, k);
                    dmax_l = fmax(dmax_l, (double)sqrtf((w0 * w0 + w1 * w1) + w2 * w2));
                }
            } else {
                for (int k = nS <= W ? own_k : tid; k >= 0 && k < n; k += nS <= W ? n : W) {
                    const int sl = nS <= W ? own_sl : sh.M[k];
                    double w0, w1, w2;
                    wavelet_disp(g, wv, sh.x[sl], sh.y[sl], sh.z[sl], w0, w1, w2);
                    if (CAPM > 0 && k < CAPM) {
                        sh.MX[k] = sh.x[sl] + w0;
                        sh.MY[k] = sh.y[sl] + w1;
                        sh.MZ[k] = sh.z[sl] + w2;
                    }
                    tile_tag_set(sh, sl, k);
                    dmax_l = fmax(dmax_l, sqrt((w0 * w0 + w1 * w1) + w2 * w2));
                }
            }
            // barrier: trial positions and tags visible (an FP32 length is raised by 2^-20, more
            // than its rounding)
            const double dmax = xmax<W>(dmax_l, sh.xc, xp) * (F32 ? 1.0 + 0x1p-20 : 1.0);
            const double Rq = P.rc + 2.0 * dmax + E + 1e-9 * L;
            double acc = 0.0;
            const double thr = accept_threshold<VAR>(P, u_acc);
            double dU;
            bool spec_taken = false;  // the first redraw tries were taken during the energy sum
            if constexpr (F32) {
                // error of the FP32 sum (eps = 2^-24; every offset magnitude <= Hq). Worst case: an
                // offset carries <= eps Hq, the centre's <= 3 eps Hq, so x_r is off by <= 5 eps Hq/lambda
                // per axis and a displacement (A <= A0 lambda) by <= 19 A0 eps Hq; a trial coordinate
                // by <= eps Hq (2.5 + 19 A0), a distance component by twice that, r2 by <= 2 eps r2
                // (Hq (8.7 + 66 A0)/r + 1.5), and a term by <= 2 eps sens (Hq (8.7 + 66 A0)/r + 6)
                // with its own FP32 evaluation. rc2g widens the cut-off by 8 times that r2 bound, so
                // no pair within the FP64 cut-off is missed. The margin itself,
                // 2^-23 (16 S1 + 8 Hq S2) with S1 = sum of sens and S2 = sum of sens/r, is smaller
                // than the worst case (which has all roundings aligned, and ignores that a pair's
                // offset roundings enter its old and new distance alike): its sufficiency is what the
                // mixed_verify mode measures (every |dU32 - dU64| against it).
                const double Hq = tg.He + Etot + dmax;
                const bool wrap = g.periodic && 2.0 * Hq + P.rc >= L;
                const double Hm = wrap ? fmax(Hq, L) : Hq;
                const double K2 = 9.0 + 66.0 * P.A0;
                const float rc2g = (float)(P.rc2 * (1.0 + 0x1p-20 * (K2 * Hm / fmax(P.rc, 1e-3) + 2.0)));
                float s1 = 0.0f, s2 = 0.0f;
                const double rp = P.rc + 2.0 * dmax;
                const float Rp2f = (float)(rp * rp * ((double)rc2g / P.rc2) * (1.0 + 0x1p-9));
                const int light = tile_dU32<W, CAPH, CAPM, NCD>(P, D, sh, g, tg, wv32, Rq, nH, n, wrap, (float)L,
                                                                (float)invL, (float)P.rc2, rc2g, Rp2f, acc, s1, s2, c_viol);
                spec_taken = SPEC && r + 1 < P.retry_cap && light >= 0;
                if (spec_taken) spec_redraw(tc, r + 1, lam, light);
                double S1 = (double)s1, S2 = (double)s2;
                dU = acc;
                xsum3<W>(dU, S1, S2, sh.xc, xp);
                const double m = 0x1.0p-23 * (16.0 * S1 + 8.0 * Hm * S2) + 1e-12;
                const bool near = !(isfinite(dU) && fabs(dU - thr) > m);
                if (near || P.mixed_verify) {
                    double a64 = 0.0;
                    unsigned long long v64 = 0;
                    tile_dU<W, CAPH, CAPM, NCD, float, WaveDesc32>(P, D, s, sh, g, tg, wv32, Rq, nH, n, a64, v64,
                                                                    rc2g, rp * rp * (1.0 + 1e-12));
                    const double d64 = xsum<W>(a64, sh.xc, xp);
                    if (tid == 0) {
                        if (near) atomicAdd(&D.cnt[CNT_RECHECK], 1ull);
                        if (P.mixed_verify) {
                            atomicAdd(&D.cnt[CNT_MARGIN_CHECK], 1ull);
                            bool fail = !near && !isfinite(d64);
                            if (isfinite(dU) && isfinite(d64)) {
                                const double ratio = fabs(dU - d64) / m;
                                fail = fail || ratio > 1.0;
                                if (ratio == ratio)
                                    atomicMax(&D.cnt[CNT_MARGIN_RATIO],
                                              (unsigned long long)__float_as_uint((float)ratio));
                            }
                            if (fail) atomicAdd(&D.cnt[CNT_MARGIN_FAIL], 1ull);
                        }
                    }
                    if (near) dU = d64;
                }
            } else {
                const double rp = (P.rc + 2.0 * dmax) * (1.0 + 1e-12);
                const int light = tile_dU<W, CAPH, CAPM, NCD>(P, D, s, sh, g, tg, wv, Rq, nH, n, acc, c_viol, 0.0f, rp * rp);
                spec_taken = SPEC && r + 1 < P.retry_cap && light >= 0;
                if (spec_taken) spec_redraw(tc, r + 1, lam, light);
                dU = xsum<W>(acc, sh.xc, xp);
            }
            const bool accept = dU <= thr;
            if (tid == 0)
                trace_push(D, 0, sys, sweep, level, key, tc, r, n, accept ? 1 : 0, as >= 0 ? (sh.id[as] & ID_MASK) : -1,
                           dU, thr);
            ++c_att;
            c_beads += n;
            for (int k = tid; k < n; k += W) {
                const int sl = sh.M[k];
                if (accept) {
                    const int32_t j = sh.id[sl] & ID_MASK;
                    double nx, ny, nz;
                    if constexpr (F32) {
                        // FP64 position plus the FP32 displacement; the tile keeps its rounded offset
                        float w0, w1, w2;
                        member_w32(sh, wv32, k, sl, w0, w1, w2);
                        nx = D.x[j] + (double)w0;
                        ny = D.y[j] + (double)w1;
                        nz = D.z[j] + (double)w2;
                        sh.x[sl] = (float)minimg(g, nx - tg.c[0]);
                        sh.y[sl] = (float)minimg(g, ny - tg.c[1]);
                        sh.z[sl] = (float)minimg(g, nz - tg.c[2]);
                    } else {
                        member_new(sh, g, wv, k, sl, nx, ny, nz);
                        sh.x[sl] = nx;
                        sh.y[sl] = ny;
                        sh.z[sl] = nz;
                    }
                    D.x[j] = nx;
                    D.y[j] = ny;
                    D.z[j] = nz;
                    double dd = fmax(fabs(nx - D.xb[j]), fmax(fabs(ny - D.yb[j]), fabs(nz - D.zb[j])));
                    d_local = fmax(d_local, dd);
                }
                tile_tag_clear(sh, sl);
            }
            // a rejection changes no position: the next writes of the tags and member lists follow
            // the next test's member scan, which is a barrier
            if (accept) {
                __syncthreads();
                ++c_acc;
                if (tid == 0) atomicAdd(&D.cnt[CNT_ACC_BEADS], (unsigned long long)n);
                E += dmax;
                Etot += dmax;
                if (E > 0.5 * tg.f) {
                    tile_index<W, CAPH, CAPM, NCD>(sh, nH, g, tg);
                    E = 0.0;
                }
                break;
            }
            if (++r >= P.retry_cap) {
                ++c_caps;
                break;
            }
            // redraws in chunks: 16 tries first (the ball's rejection loop runs as long as its
            // slowest lane, so a narrow first chunk is cheaper; wider tiles took it during the
            // test), then W at a time
            int found = -1, j_first = 0;
            if (spec_taken) {
                found = sh.spec_found;
                j_first = 16;
            }
            if (found < 0) {
                for (int j0 = j_first, len = j0 == 0 && W > 16 ? 16 : W; j0 < 4096 && found < 0; j0 += len, len = W) {
                    int jj = j0 + tid;
                    bool h2 = false;
                    double ex = 0, ey = 0, ez = 0;
                    float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
                    int a2 = 0;
                    Stream rs;
                    if (tid < len && jj < 4096) h2 = redraw_try(tc, r, jj, lam, rs, a2, ex, ey, ez, g0, g1, g2);
                    int fj = xmin_int<W>(h2 ? jj : 0x7FFFFFFF, sh.xc, xp);
                    if (fj != 0x7FFFFFFF) {
                        if (jj == fj) {
                            sh.pub_a = a2;
                            sh.pub_b[0] = ex;
                            sh.pub_b[1] = ey;
                            sh.pub_b[2] = ez;
                            sh.pub_bf[0] = g0;
                            sh.pub_bf[1] = g1;
                            sh.pub_bf[2] = g2;
                            sh.pub_next = rs.next;
                        }
                        found = fj;
                    }
                }
                __syncthreads();  // the finder's pub_* visible
            }
            if (found < 0) {
                c_redraw += 4096;
                ++c_caps;
                break;
            }
            c_redraw += (unsigned long long)found;
            // pub_* are written again only after the next test's member scan (a barrier)
            as = sh.pub_a;
            if constexpr (!F32) {
                b[0] = sh.pub_b[0];
                b[1] = sh.pub_b[1];
                b[2] = sh.pub_b[2];
            }
            nxt = sh.pub_next;
            jtry = found;
        }
        from = first + 1;
      }
    }
    d_local = block_max<W>(d_local, sh.red);
    unsigned long long viol_all = (unsigned long long)block_sum<W>((double)c_viol, sh.red);
    if constexpr (F32) {
        const unsigned long long mre = (unsigned long long)block_sum<W>((double)c_mre, sh.red);
        if (tid == 0 && mre) atomicAdd(&D.cnt[CNT_MEMBER_RECHECK], mre);
    }
    if (tid == 0) {
        unsigned long long* C = D.cnt + CNT_LEVEL + level * 8;
        atomicAdd(&C[0], (unsigned long long)K);
        atomicAdd(&C[1], c_hits);
        atomicAdd(&C[2], c_att);
        atomicAdd(&C[3], c_acc);
        atomicAdd(&C[4], c_caps);
        atomicAdd(&C[5], c_redraw);
        atomicAdd(&C[6], c_beads);
        if (viol_all) atomicAdd(&D.cnt[CNT_VIOL], viol_all);
        if (c_acc) {
            atomicAdd(&D.cnt[CNT_ACCEPTED], c_acc);
            atomicAdd(&D.sys_acc[sys], c_acc);
        }
        if (d_local > 0.0) atomic_max_double(&D.drift[sys], d_local);
        trace_push(D, 1, sys, sweep, level, key, K, nS, 0, (int)c_hits, 0, 0.0, 0.0);
    }
    dl_out = d_local;
    __syncthreads();
    return true;
}

template <int W, int CAPS, int CAPM, int CAPH, int CAPMT, int NCD, bool MIXED, bool VAR>
__global__ __launch_bounds__(W) void k_phase(DevParams P, DevPtrs D, int level, int colour, int64_t sweep,
                                             const int32_t* bmap, int nblocks) {
    __shared__ PhaseLDS<W, CAPS, CAPM, CAPH, CAPMT, NCD, typename std::conditional<MIXED, float, double>::type> sh;
    if (P.periodic) {
        const int sys = bmap[2 * blockIdx.x], local = bmap[2 * blockIdx.x + 1];
        const SysDesc& s = D.sys[sys];
        const LevelDesc& lv = D.lev[s.lvl_off + level];
        Grid g;
        make_grid(P, D, s, lv, sys, level, sweep, g);
        // the drift bound is what the earlier colours of this level published (all complete: one
        // launch per colour); cells of this colour publish into their own colour's slot, so no
        // cell reads a value that a cell of its own launch may still raise
        double Dg = 0.0;
        for (int c = 0; c < colour; ++c) Dg = fmax(Dg, __longlong_as_double((long long)D.drift_col[8 * sys + c]));
        double dl = 0.0;
        if (lv.use_global || !process_cell_tile<W, CAPH, CAPMT, NCD, VAR>(P, D, sh.t, sys, level, colour, local, sweep, g,
                                                                            Dg, dl)) {
            __syncthreads();
            // global-list cells compute in FP64 in both precisions (their time is not arithmetic: FP32
            // terms with the recheck margin measured slower there)
            process_cell<W, CAPS, CAPM, VAR>(P, D, sh.g, sys, level, colour, local, sweep, g, Dg, dl);
        }
        if (threadIdx.x == 0 && dl > 0.0) atomic_max_double(&D.drift_col[8 * sys + colour], dl);
    } else {
        // infinite system: reach lists and pair searches scan every bead, no drift bound is used
        const SysDesc& s = D.sys[0];
        const LevelDesc& lv = D.lev[s.lvl_off + level];
        Grid g;
        make_grid(P, D, s, lv, 0, level, sweep, g);
        const int lc = colour ^ grid_parity(g);
        int64_t mx = (g.n[0] - (lc & 1) + 1) / 2, my = (g.n[1] - ((lc >> 1) & 1) + 1) / 2,
                mz = (g.n[2] - ((lc >> 2) & 1) + 1) / 2;
        int64_t cells = mx * my * mz;
        double dl = 0.0;
        for (int64_t local = blockIdx.x; local < cells; local += gridDim.x)
            process_cell<W, CAPS, CAPM, VAR>(P, D, sh.g, 0, level, colour, local, sweep, g, 0.0, dl);
    }
}

template <bool M, bool V>
static void launch_phase_t(int variant, const DevParams& P, const DevPtrs& D, int level, int colour, int64_t sweep,
                  const int32_t* bmap, int nblocks, hipStream_t st) {
    if (nblocks <= 0) return;
    if (variant == V64)
        hipLaunchKernelGGL((k_phase<64, 1024, 256, 512, 32, 8, M, V>), dim3(nblocks), dim3(64), 0, st, P, D, level, colour,
                           sweep, bmap, nblocks);
    else if (variant == V256)
        hipLaunchKernelGGL((k_phase<256, 4096, 1024, 1024, 512, 12, M, V>), dim3(nblocks), dim3(256), 0, st, P, D, level,
                           colour, sweep, bmap, nblocks);
    else
        hipLaunchKernelGGL((k_phase<512, 8192, 4096, 4096, 128, 18, M, V>), dim3(nblocks), dim3(512), 0, st, P, D, level,
                           colour, sweep, bmap, nblocks);
}

// whether a context uses any of the variants (Glauber, rotation map, uniform centres)
static bool uses_variants(const DevParams& P) {
    return P.accept_rule != WMC_ACCEPT_METROPOLIS || P.wavelet_map != WMC_MAP_LINEAR || P.centring != WMC_CENTRE_ANCHOR;
}

// one kernel per precision and variant set: the FP32 tiles with their rechecks, and the variants,
// cost registers the FP64 path of the paper's method does not need
void launch_phase(int variant, const DevParams& P, const DevPtrs& D, int level, int colour, int64_t sweep,
                  const int32_t* bmap, int nblocks, hipStream_t st) {
    const bool v = uses_variants(P);
    if (P.precision == WMC_MIXED) {
        if (v) launch_phase_t<true, true>(variant, P, D, level, colour, sweep, bmap, nblocks, st);
        else launch_phase_t<true, false>(variant, P, D, level, colour, sweep, bmap, nblocks, st);
    } else {
        if (v) launch_phase_t<false, true>(variant, P, D, level, colour, sweep, bmap, nblocks, st);
        else launch_phase_t<false, false>(variant, P, D, level, colour, sweep, bmap, nblocks, st);
    }
}

// ------------------------------------------- level pass in dependency order (LDS tiles)
// The colour phases of a level ask only that adjacent cells run in colour order: same-colour
// cells are independent and cells further apart than one cell never interact. So one launch
// runs every LDS-tile cell of the level: cells are handed out in colour order through an
// atomic counter, and a cell first waits until each adjacent cell of a lower colour has
// published this pass's epoch. A workgroup waits only on cells handed out before its own,
// whose workgroups are already running, so the pass cannot deadlock; the wait is still bounded
// (counted in CNT_FLOWWAIT when the bound is hit). Same result as eight colour phases.
constexpr unsigned FLOW_SPIN_LIMIT = 1u << 24;

template <int W, int CAPS, int CAPM, int CAPH, int CAPMT, int NCD, bool MIXED, bool VAR>
__global__ __launch_bounds__(W, W == 64 ? 2 : 1) void k_level_flow(DevParams P, DevPtrs D, int level, int64_t sweep,
                                                     const int32_t* items, FlowArgs fa) {
    __shared__ PhaseLDS<W, CAPS, CAPM, CAPH, CAPMT, NCD, typename std::conditional<MIXED, float, double>::type> sh;
    __shared__ int s_idx;
    __shared__ int s_timeout;
    __shared__ double s_dg[27];
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_idx = (int)(atomicAdd(&D.flow_ctr[level], 1ull) - fa.qbase);
        s_timeout = 0;
    }
    if (tid < 27) s_dg[tid] = 0.0;
    __syncthreads();
    const int idx = s_idx;
    if (idx < 0 || idx >= fa.nitems) return;
    int colour = 0;
    while (colour < 7 && idx >= fa.colour_end[colour]) ++colour;
    const int sys = items[2 * idx], local = items[2 * idx + 1];
    const SysDesc& s = D.sys[sys];
    const LevelDesc& lv = D.lev[s.lvl_off + level];
    Grid g;
    make_grid(P, D, s, lv, sys, level, sweep, g);
    int64_t ic[3];
    cell_coords(P, lv, g, colour, local, ic);
    const int n = lv.n;
    // adjacent cells of lower colours (n >= 4: the 26 neighbours are distinct)
    if (tid < 27 && tid != 13) {
        const int dx = tid % 3 - 1, dy = (tid / 3) % 3 - 1, dz = tid / 9 - 1;
        const int jx = (int)((ic[0] + dx + n) % n), jy = (int)((ic[1] + dy + n) % n), jz = (int)((ic[2] + dz + n) % n);
        const int cn = (jx & 1) | ((jy & 1) << 1) | ((jz & 1) << 2);
        if (cn < colour) {
            const int64_t fi = lv.flag_base + jx + (int64_t)n * (jy + (int64_t)n * jz);
            const int32_t* f = D.cell_done + fi;
            unsigned spins = 0;
            while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != fa.epoch) {
                if (++spins >= FLOW_SPIN_LIMIT) {
                    s_timeout = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_dg[tid] = D.cell_drift[fi];
        }
    }
    __syncthreads();
    // Drift bound of this cell: the beads it can meet were moved, since this level's grid build,
    // only by itself and by the adjacent cells of lower colours it has just waited for (a bead moved
    // by a cell further away stays more than lambda_hi + r_int from this one), so the largest drift
    // those cells published bounds them, independent of the timing of any other cell.
    double Dg = 0.0;
    for (int k = 0; k < 27; ++k) Dg = fmax(Dg, s_dg[k]);
    double dl = 0.0;
    if (s_timeout) {
        // a neighbour never published: running now could race with it, so the cell is skipped and
        // the sweep reported invalid (wmc_observables returns WMC_ESCHEDULE)
        if (tid == 0) atomicAdd(&D.cnt[CNT_FLOWWAIT], 1ull);
    } else if (!process_cell_tile<W, CAPH, CAPMT, NCD, VAR>(P, D, sh.t, sys, level, colour, local, sweep, g, Dg, dl)) {
        // the halo does not fit the tile: the global-list path, inline (a call would cost a stack
        // frame and the registers saved around it, for every cell)
        __syncthreads();
        if (tid == 0) atomicAdd(&D.cnt[CNT_FALLBACK], 1ull);
        process_cell<W, CAPS, CAPM, VAR>(P, D, sh.g, sys, level, colour, local, sweep, g, Dg, dl);
    }
    // publish: every wave's stores complete, then this cell's drift and one release of the epoch
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (tid == 0) {
        const int64_t fi = lv.flag_base + ic[0] + (int64_t)n * (ic[1] + (int64_t)n * ic[2]);
        D.cell_drift[fi] = dl;
        __hip_atomic_store(D.cell_done + fi, fa.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <bool M, bool V>
static void launch_level_flow_t(int variant, const DevParams& P, const DevPtrs& D, int level, int64_t sweep,
                       const int32_t* items, const FlowArgs& fa, int width64, hipStream_t st) {
    if (fa.nitems <= 0) return;
    // the smallest tile: a few thousand cells (one large system) finish sooner with four waves
    // per cell, since the pass is its longest chain of cells; many more cells (a batch) fill the
    // GPU better with one wave per cell (width64 overrides the rule)
    if (variant == V64 && (width64 == 256 || (width64 == 0 && fa.nitems <= 4096)))
        hipLaunchKernelGGL((k_level_flow<256, 1024, 256, 512, 32, 8, M, V>), dim3(fa.nitems), dim3(256), 0, st, P, D,
                           level, sweep, items, fa);
    else if (variant == V64)
        hipLaunchKernelGGL((k_level_flow<64, 1024, 256, 512, 32, 8, M, V>), dim3(fa.nitems), dim3(64), 0, st, P, D, level,
                           sweep, items, fa);
    else if (variant == V256)
        hipLaunchKernelGGL((k_level_flow<256, 4096, 1024, 1024, 512, 12, M, V>), dim3(fa.nitems), dim3(256), 0, st, P, D,
                           level, sweep, items, fa);
    else
        hipLaunchKernelGGL((k_level_flow<512, 8192, 4096, 4096, 128, 18, M, V>), dim3(fa.nitems), dim3(512), 0, st, P, D,
                           level, sweep, items, fa);
}

void launch_level_flow(int variant, const DevParams& P, const DevPtrs& D, int level, int64_t sweep,
                       const int32_t* items, const FlowArgs& fa, int width64, hipStream_t st) {
    const bool v = uses_variants(P);
    if (P.precision == WMC_MIXED) {
        if (v) launch_level_flow_t<true, true>(variant, P, D, level, sweep, items, fa, width64, st);
        else launch_level_flow_t<true, false>(variant, P, D, level, sweep, items, fa, width64, st);
    } else {
        if (v) launch_level_flow_t<false, true>(variant, P, D, level, sweep, items, fa, width64, st);
        else launch_level_flow_t<false, false>(variant, P, D, level, sweep, items, fa, width64, st);
    }
}

// ------------------------------------------------- cell phase of a large level, grid-wide
// A level with one or two cells per axis has few cells per colour (one per system), so a
// cooperative launch gives each such cell a group of workgroups (CoopGroup, sized by the
// system's bead count; the groups of one launch are the cells of one colour). Within a group,
// every workgroup repeats the cheap scalar steps (trial draws and hit tests, directions,
// recycling redraws) on the same data and so takes the same path; the list work is split:
//  - reach list: workgroup w scans a contiguous slice of the system's beads; the slices are
//    concatenated in order (grid barrier, prefix of the per-workgroup counts);
//  - members of a test: workgroup w scans a contiguous slice of the reach list; the member
//    list is the ordered concatenation (barrier 1); each workgroup displaces its own members
//    and publishes its largest displacement (barrier 2);
//  - dU: (member, grid row) items over every thread of the grid, per-workgroup partial sums
//    (barrier 3), summed in workgroup order by everyone, so every workgroup takes the same
//    decision; an accepted move is written back by the owning workgroups (barrier 4).
constexpr int CW = 256;     // threads per workgroup
constexpr int CAPL = COOP_LIST_CAP;  // list entries one workgroup keeps in LDS
constexpr int CMAXG = 256;  // at most this many workgroups per group (one count per thread)

constexpr int CPB = 512;  // (member, row) items per batch of the balanced pair search

struct CoopShared {
    int32_t L[CAPL];
    // balanced pair search: per item the member's current and trial position, its bead, the start
    // of its row's first and second (wrapped) run of the sorted index and the first run's length,
    // and the exclusive prefix of the items' candidate counts
    double ip[6][CPB];
    int32_t ij[CPB], is0[CPB], il0[CPB], is1[CPB];
    int32_t pre[CPB + 1];
    double red[CW / 64];
    int redi[CW / 64];
    double pub_b[3];
    double pub_lam;
    int32_t pub_a;
    uint32_t pub_next;
    int pub_off;
    int spec_found;  // first hit of the speculative redraw tries, -1 if none
};

// exclusive prefix (at the workgroup of rank wg in its group) and total of the group's
// per-workgroup counts published before a group barrier
__device__ __forceinline__ void coop_prefix(const int32_t* cnt, int G, int wg, CoopShared& sh, int& off, int& tot) {
    const int v = (int)threadIdx.x < G ? cnt[threadIdx.x] : 0;
    int before;
    tot = block_scan_count<CW>(v, before, sh.redi);
    if ((int)threadIdx.x == wg) sh.pub_off = before;
    __syncthreads();
    off = sh.pub_off;
    __syncthreads();
}
__device__ __forceinline__ double coop_sum(const double* part, int G, CoopShared& sh) {
    return block_sum<CW>((int)threadIdx.x < G ? part[threadIdx.x] : 0.0, sh.red);
}
__device__ __forceinline__ double coop_max(const double* part, int G, CoopShared& sh) {
    return block_max<CW>((int)threadIdx.x < G ? part[threadIdx.x] : 0.0, sh.red);
}

// Pair energy changes of a cell group's test, balanced over the lanes of each workgroup. The
// (member, grid row) items of the pair search are split into equal contiguous blocks per workgroup.
// A batch of items is first resolved into its row runs of the sorted neighbour index (member data
// and run bounds in LDS); a workgroup scan of the runs' lengths then gives every thread an equal,
// contiguous share of the batch's candidate partners (found by one binary search, then walked), so
// a long row no longer holds up its lane while the others idle. Same terms as glob_dU's pair part;
// only the order of the sum differs.
__device__ void coop_pairs(const DevParams& P, const DevPtrs& D, const SysDesc& s, const int32_t* Ml,
                           const double* MXl, const double* MYl, const double* MZl, int n, double R, int wg,
                           int G, CoopShared& sh, double& acc) {
    const int tid = threadIdx.x;
    const double L = s.L, invL = s.invL;
    const int nf = s.nf;
    const int NR = min(nf, (int)floor(2.0 * R * s.invg) + 2);
    const int per = NR * NR;
    const int total = n * per;
    const int Q = (total + G - 1) / G;
    const int i0 = min(total, wg * Q), i1 = min(total, i0 + Q);
    for (int b0 = i0; b0 < i1; b0 += CPB) {
        const int nb = min(CPB, i1 - b0);
        // 1. items: member data and row runs
        for (int i = tid; i < nb; i += CW) {
            const int it = b0 + i;
            const int k = it / per, q = it - k * per;
            const int qy = q % NR, qz = q / NR;
            const int32_t j = Ml[k];
            const double jx = D.x[j], jy = D.y[j], jz = D.z[j];
            int f0y, cny, f0z, cnz;
            fine_range(wrap01(jy, L, invL) - R, wrap01(jy, L, invL) + R, s.invg, nf, f0y, cny);
            fine_range(wrap01(jz, L, invL) - R, wrap01(jz, L, invL) + R, s.invg, nf, f0z, cnz);
            int cnt = 0;
            if (qy < cny && qz < cnz) {
                int f0x, cnx;
                const double cx = wrap01(jx, L, invL);
                fine_range(cx - R, cx + R, s.invg, nf, f0x, cnx);
                const int fy = (f0y + qy) % nf, fz = (f0z + qz) % nf;
                const int64_t row = s.fine_off + (int64_t)nf * (fy + (int64_t)nf * fz);
                const int xe = min(f0x + cnx, nf);
                const int s0 = D.fstart[row + f0x], l0 = D.fstart[row + xe] - s0;
                int s1 = 0, l1 = 0;
                if (f0x + cnx > nf) {
                    s1 = D.fstart[row];
                    l1 = D.fstart[row + (f0x + cnx - nf)] - s1;
                }
                cnt = l0 + l1;
                sh.ip[0][i] = jx;
                sh.ip[1][i] = jy;
                sh.ip[2][i] = jz;
                sh.ip[3][i] = MXl[k];
                sh.ip[4][i] = MYl[k];
                sh.ip[5][i] = MZl[k];
                sh.ij[i] = j;
                sh.is0[i] = s0;
                sh.il0[i] = l0;
                sh.is1[i] = s1;
            }
            sh.pre[i] = cnt;
        }
        __syncthreads();
        // 2. exclusive prefix of the candidate counts (each thread sums CPB / CW consecutive items)
        {
            constexpr int PT = CPB / CW;
            int v[PT], run = 0;
            for (int u = 0; u < PT; ++u) {
                const int i = tid * PT + u;
                v[u] = i < nb ? sh.pre[i] : 0;
                run += v[u];
            }
            int before;
            const int tot = block_scan_count<CW>(run, before, sh.redi);
            for (int u = 0; u < PT; ++u) {
                const int i = tid * PT + u;
                if (i < nb) sh.pre[i] = before;
                before += v[u];
            }
            if (tid == 0) sh.pre[nb] = tot;
        }
        __syncthreads();
        // 3. an equal contiguous share of the candidates per thread
        const int C = sh.pre[nb];
        const int ch = (C + CW - 1) / CW;
        int c = tid * ch;
        const int cend = min(C, c + ch);
        if (c < cend) {
            int lo = 0, hi = nb - 1;  // the last item whose prefix is <= c
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (sh.pre[mid] <= c) lo = mid; else hi = mid - 1;
            }
            int i = lo;
            for (; c < cend; ++c) {
                while (sh.pre[i + 1] <= c) ++i;
                const int o = c - sh.pre[i];
                const int l0 = sh.il0[i];
                const int32_t m = D.fidx[o < l0 ? sh.is0[i] + o : sh.is1[i] + (o - l0)];
                const int32_t j = sh.ij[i];
                if (m == j) continue;
                const int km = D.tag[m];
                if (km >= 0 && m < j) continue;
                const double mx = D.x[m], my = D.y[m], mz = D.z[m];
                const double nx = km >= 0 ? MXl[km] : mx, ny = km >= 0 ? MYl[km] : my, nz = km >= 0 ? MZl[km] : mz;
                const double r2o = pair_r2(P, invL, L, sh.ip[0][i], sh.ip[1][i], sh.ip[2][i], mx, my, mz);
                const double r2n = pair_r2(P, invL, L, sh.ip[3][i], sh.ip[4][i], sh.ip[5][i], nx, ny, nz);
                if (r2o < P.rc2 || r2n < P.rc2) acc += u_pair(P, r2n) - u_pair(P, r2o);
            }
        }
        __syncthreads();  // the next batch rewrites the arrays
    }
}

// one cell of colour `colour` for the group `grp` (index gi); gen is the group's barrier
// generation and Dg its system's drift bound, both carried from colour to colour
template <bool VAR>
__device__ void coop_cell(const DevParams& P, const DevPtrs& D, int level, int colour, int64_t sweep,
                          const CoopGroup grp, int gi, int rank, CoopShared& sh, unsigned& gen, double& Dg) {
    const int sys = grp.sys;
    const SysDesc& s = D.sys[sys];
    const LevelDesc& lv = D.lev[s.lvl_off + level];
    const int tid = threadIdx.x, wg = rank, G = grp.size;
    const int gt = wg * CW + tid, gstride = G * CW;
    unsigned* bar = D.gbar + 2 * (1 + gi);
    Grid g;
    make_grid(P, D, s, lv, sys, level, sweep, g);
    int64_t ic[3];
    cell_coords(P, lv, g, colour, grp.local, ic);
    const int64_t cell = ic[0] + g.n[0] * (ic[1] + g.n[1] * ic[2]);
    const int64_t key = cell_key(g, ic);
    const double hi2 = lv.hi * lv.hi;
    const double L = s.L;
    int32_t* Sg = D.slot_S + (lv.slot_base + grp.local) * D.slot_len;
    int32_t* Mg = D.slot_M + (lv.slot_base + grp.local) * D.slot_len;
    double* MXg = D.slot_MX + (lv.slot_base + grp.local) * 3 * D.slot_len;
    double* MYg = MXg + D.slot_len;
    double* MZg = MXg + 2 * D.slot_len;
    // this group's per-workgroup slots
    int32_t* ccnt = D.coop_i + grp.first;
    double* c_dmax = D.coop_d + grp.first;
    double* c_acc = D.coop_d + COOP_SLOTS + grp.first;
    double* c_dl = D.coop_d + 4 * COOP_SLOTS + grp.first;

    // ---- 1. reach list, bead order
    int nS;
    if (lv.identity) {
        nS = s.N;
    } else {
        const int64_t q = ((int64_t)s.N + G - 1) / G;
        const int64_t lo = s.b0 + (int64_t)wg * q, hi = min(s.b1, lo + q);
        int cnt = 0;
        for (int64_t c0 = lo; c0 < hi; c0 += CW) {
            const int64_t j = c0 + tid;
            const bool f = j < hi && dist2_cell(g, ic, D.x[j], D.y[j], D.z[j]) <= hi2;
            int before;
            const int tot = block_scan_flag<CW>(f, before, sh.redi);
            if (f) sh.L[cnt + before] = (int32_t)j;
            cnt += tot;
        }
        if (tid == 0) ccnt[wg] = cnt;
        group_barrier(bar, G, gen);
        int off;
        coop_prefix(ccnt, G, wg, sh, off, nS);
        for (int i = tid; i < cnt; i += CW) Sg[off + i] = sh.L[i];
        group_barrier(bar, G, gen);
    }
    auto Sat = [&](int64_t i) -> int32_t { return lv.identity ? (int32_t)(s.b0 + i) : Sg[i]; };

    // ---- 2. number of trials (every workgroup draws the same)
    const bool uni = VAR && P.centring == WMC_CENTRE_UNIFORM;
    double mu = uni ? lv.T / ((double)g.n[0] * (double)g.n[1] * (double)g.n[2]) : (lv.T * (double)nS) / (double)s.N;
    int64_t K = (int64_t)floor(mu);
    {
        Stream ms;
        ms.init(P, sys, sweep, TAG_META + level, key, 0, 0, 0);
        if (ms.co() < mu - (double)K) K += 1;
    }
    if (K > 0xFFFFF) K = 0xFFFFF;
    unsigned long long c_hits = 0, c_att = 0, c_acc_n = 0, c_caps = 0, c_redraw = 0, c_beads = 0, c_viol = 0;
    double dloc = 0.0;  // largest drift of beads moved in this phase (same in every workgroup)
    const int qS = (nS + G - 1) / G;
    const int slo = wg * qS, shi = min(nS, slo + qS);

    auto pos_of = [&](int32_t j, double& px, double& py, double& pz) {
        px = D.x[j];
        py = D.y[j];
        pz = D.z[j];
    };

    // ---- 3. trials and chains
    for (int64_t t0 = 0; t0 < K;) {
        const int64_t t = t0 + tid;
        bool hit = false;
        double lam = 0.0, bx = 0.0, by = 0.0, bz = 0.0;
        int32_t a = 0;
        Stream st;
        if (t < K && (nS > 0 || uni)) {
            st.init(P, sys, sweep, level, key, t, 0, 0);
            lam = draw_lambda(st.co(), lv.lo, lv.hi);
            hit = draw_trial_centre<VAR>(P, st, g, ic, cell, lam, nS, Sat, pos_of, a, bx, by, bz);
        }
        const int first = block_min_int<CW>(hit ? (int)(t - t0) : 0x7FFFFFFF, sh.redi);
        if (first == 0x7FFFFFFF) {
            t0 += CW;
            continue;
        }
        if (tid == first) {
            sh.pub_lam = lam;
            sh.pub_a = a;
            sh.pub_b[0] = bx;
            sh.pub_b[1] = by;
            sh.pub_b[2] = bz;
            sh.pub_next = st.next;
        }
        __syncthreads();
        const int64_t tc = t0 + first;
        lam = sh.pub_lam;
        a = sh.pub_a;
        double b[3] = {sh.pub_b[0], sh.pub_b[1], sh.pub_b[2]};
        uint32_t nxt = sh.pub_next;
        int jtry = 0;
        ++c_hits;
        const double lam2 = lam * lam;
        for (int r = 0;;) {
            Stream cs;
            cs.init(P, sys, sweep, level, key, tc, r, jtry);
            cs.next = nxt;
            double px, py, pz;
            direction(cs, px, py, pz);
            const double u_acc = cs.oc();
            __syncthreads();
            // members in this workgroup's slice of the reach list: thread t tests entries t, t + CW,
            // ... (coalesced loads), one scan orders them thread by thread (any order of the
            // members gives the same displacements; only the rounding of the sums follows it)
            int cnt;
            {
                uint32_t mask = 0;
                for (int u = 0, i = slo + tid; i < shi; ++u, i += CW) {
                    const int32_t j = Sat(i);
                    const double dx = minimg(g, D.x[j] - b[0]), dy = minimg(g, D.y[j] - b[1]),
                                 dz = minimg(g, D.z[j] - b[2]);
                    if (((dx * dx + dy * dy) + dz * dz) <= lam2 || j == a) mask |= 1u << u;
                }
                int before;
                cnt = block_scan_count<CW>(__popc(mask), before, sh.redi);
                for (int u = 0, i = slo + tid; i < shi; ++u, i += CW)
                    if ((mask >> u) & 1u) sh.L[before++] = Sat(i);
            }
            if (tid == 0) ccnt[wg] = cnt;
            // Speculation: the first 16 tries of the redraw a rejection would need, on the first 16
            // lanes (the ball's rejection loop lasts as long as its slowest lane). A rejected test
            // moves nothing, so they see the positions that redraw would see; after an acceptance
            // they are dropped. Their draws are taken while the group arrives at barrier 2, their
            // centres and cell tests at barrier 3; the hit goes to pub_* (read again only after a
            // redraw; every workgroup finds the same) and its try index, or -1, to spec_found.
            const bool spec_on = r + 1 < P.retry_cap;
            group_barrier(bar, G, gen);  // 1: member counts
            int off, n;
            coop_prefix(ccnt, G, wg, sh, off, n);
            WaveDesc wv;
            wv.b[0] = b[0];
            wv.b[1] = b[1];
            wv.b[2] = b[2];
            wv.p[0] = px;
            wv.p[1] = py;
            wv.p[2] = pz;
            wv.lam = lam;
            wv.A = wavelet_amp<VAR>(P, s, lam, n);
            wv.rot = VAR && P.wavelet_map == WMC_MAP_ROTATION;
            double dmax_l = 0.0;
            for (int i = tid; i < cnt; i += CW) {
                const int k = off + i;
                const int32_t j = sh.L[i];
                const double xj = D.x[j], yj = D.y[j], zj = D.z[j];
                double w0, w1, w2;
                wavelet_disp(g, wv, xj, yj, zj, w0, w1, w2);
                Mg[k] = j;
                MXg[k] = xj + w0;
                MYg[k] = yj + w1;
                MZg[k] = zj + w2;
                D.tag[j] = k;
                dmax_l = fmax(dmax_l, sqrt((w0 * w0 + w1 * w1) + w2 * w2));
            }
            {
                const double m = block_max<CW>(dmax_l, sh.red);
                if (tid == 0) c_dmax[wg] = m;
            }
            int32_t sp_a = 0;
            double sp_v0 = 0.0, sp_v1 = 0.0, sp_v2 = 0.0;
            uint32_t sp_next = 0;
            {
                bool rel;
                group_arrive(bar, G, gen, rel);  // 2: members, trial positions, tags
                if (spec_on && tid < 16) {
                    // the draws of draw_trial_centre for try tid of retry r + 1
                    Stream rs;
                    rs.init(P, sys, sweep, level, key, tc, r + 1, tid);
                    if (VAR && P.centring == WMC_CENTRE_UNIFORM) {
                        sp_a = -1;
                        sp_v0 = g.o[0] + ((double)ic[0] + rs.co()) * g.h;
                        sp_v1 = g.o[1] + ((double)ic[1] + rs.co()) * g.h;
                        sp_v2 = g.o[2] + ((double)ic[2] + rs.co()) * g.h;
                    } else {
                        sp_a = Sat(rs.index(nS));
                        ball(rs, sp_v0, sp_v1, sp_v2);
                    }
                    sp_next = rs.next;
                }
                group_wait(bar, G, gen, rel);
            }
            const double dmax = coop_max(c_dmax, G, sh);
            const double Rq = P.rc + 2.0 * dmax + fmax(Dg, dloc) + 1e-9 * L;
            const double thr = accept_threshold<VAR>(P, u_acc);
            double dU;
            {
                double acc = 0.0;
                glob_dU(P, D, s, Mg, MXg, MYg, MZg, n, Rq, gt, gstride, acc, c_viol, false);  // bonds
                if (P.wca) coop_pairs(P, D, s, Mg, MXg, MYg, MZg, n, Rq, wg, G, sh, acc);
                const double pa = block_sum<CW>(acc, sh.red);
                if (tid == 0) c_acc[wg] = pa;
                bool rel;
                group_arrive(bar, G, gen, rel);  // 3: partial sums
                if (spec_on && tid < 64) {
                    // (positions are unchanged unless the test is accepted, which drops this)
                    bool h2 = false;
                    double ex = sp_v0, ey = sp_v1, ez = sp_v2;
                    if (tid < 16) {
                        if (sp_a >= 0) {
                            double ax, ay, az;
                            pos_of(sp_a, ax, ay, az);
                            ex = ax + lam * sp_v0;
                            ey = ay + lam * sp_v1;
                            ez = az + lam * sp_v2;
                        }
                        h2 = cell_of_point(g, ex, ey, ez) == cell;
                    }
                    const uint64_t hits = __ballot(h2);
                    const int fj = hits ? __builtin_ctzll(hits) : -1;
                    if (tid == fj) {
                        sh.pub_a = sp_a;
                        sh.pub_b[0] = ex;
                        sh.pub_b[1] = ey;
                        sh.pub_b[2] = ez;
                        sh.pub_next = sp_next;
                    }
                    if (tid == 0) sh.spec_found = fj;
                }
                group_wait(bar, G, gen, rel);
                dU = coop_sum(c_acc, G, sh);
            }
            // first 16 tries of the redraw a rejection would need (-1: no hit, -2: not taken)
            const int spec = spec_on ? sh.spec_found : -2;
            const bool accept = dU <= thr;
            if (wg == 0 && tid == 0) trace_push(D, 0, sys, sweep, level, key, tc, r, n, accept ? 1 : 0, a, dU, thr);
            ++c_att;
            c_beads += n;
            double dl = 0.0;
            for (int i = tid; i < cnt; i += CW) {
                const int k = off + i;
                const int32_t j = sh.L[i];
                if (accept) {
                    const double nx = MXg[k], ny = MYg[k], nz = MZg[k];
                    D.x[j] = nx;
                    D.y[j] = ny;
                    D.z[j] = nz;
                    dl = fmax(dl, fmax(fabs(nx - D.xb[j]), fmax(fabs(ny - D.yb[j]), fabs(nz - D.zb[j]))));
                }
                D.tag[j] = -1;
            }
            if (accept) {
                const double m = block_max<CW>(dl, sh.red);
                if (tid == 0) c_dl[wg] = m;
                group_barrier(bar, G, gen);  // 4: accepted positions
                dloc = fmax(dloc, coop_max(c_dl, G, sh));
                ++c_acc_n;
                if (wg == 0 && tid == 0) atomicAdd(&D.cnt[CNT_ACC_BEADS], (unsigned long long)n);
                break;
            }
            __syncthreads();
            if (++r >= P.retry_cap) {
                ++c_caps;
                break;
            }
            // recycle lambda: redraw anchor and centre until the centre is in the cell (the first
            // 16 tries were taken at barriers 2 and 3)
            int found = spec >= 0 ? spec : -1;
            for (int j0 = spec == -2 ? 0 : 16; j0 < 4096 && found < 0; j0 += CW) {
                const int jj = j0 + tid;
                bool h2 = false;
                double ex = 0, ey = 0, ez = 0;
                int32_t a2 = 0;
                Stream rs;
                if (jj < 4096) {
                    rs.init(P, sys, sweep, level, key, tc, r, jj);
                    h2 = draw_trial_centre<VAR>(P, rs, g, ic, cell, lam, nS, Sat, pos_of, a2, ex, ey, ez);
                }
                const int fj = block_min_int<CW>(h2 ? jj : 0x7FFFFFFF, sh.redi);
                if (fj != 0x7FFFFFFF) {
                    if (jj == fj) {
                        sh.pub_a = a2;
                        sh.pub_b[0] = ex;
                        sh.pub_b[1] = ey;
                        sh.pub_b[2] = ez;
                        sh.pub_next = rs.next;
                    }
                    found = fj;
                }
            }
            __syncthreads();
            if (found < 0) {
                c_redraw += 4096;
                ++c_caps;
                break;
            }
            c_redraw += (unsigned long long)found;
            a = sh.pub_a;
            b[0] = sh.pub_b[0];
            b[1] = sh.pub_b[1];
            b[2] = sh.pub_b[2];
            nxt = sh.pub_next;
            jtry = found;
            __syncthreads();
        }
        t0 = tc + 1;
    }
    // ---- counters (every workgroup holds the same values; workgroup 0 reports them). The
    // largest-displacement slots are free here: their last reads precede the last barrier 3.
    const double viol_all = block_sum<CW>((double)c_viol, sh.red);
    if (tid == 0) c_dmax[wg] = viol_all;
    group_barrier(bar, G, gen);
    const unsigned long long viol_tot = (unsigned long long)coop_sum(c_dmax, G, sh);
    if (wg == 0 && tid == 0) {
        unsigned long long* C = D.cnt + CNT_LEVEL + level * 8;
        atomicAdd(&C[0], (unsigned long long)K);
        atomicAdd(&C[1], c_hits);
        atomicAdd(&C[2], c_att);
        atomicAdd(&C[3], c_acc_n);
        atomicAdd(&C[4], c_caps);
        atomicAdd(&C[5], c_redraw);
        atomicAdd(&C[6], c_beads);
        if (viol_tot) atomicAdd(&D.cnt[CNT_VIOL], viol_tot);
        if (c_acc_n) {
            atomicAdd(&D.cnt[CNT_ACCEPTED], c_acc_n);
            atomicAdd(&D.sys_acc[sys], c_acc_n);
        }
        if (dloc > 0.0) atomic_max_double(&D.drift[sys], dloc);
        trace_push(D, 1, sys, sweep, level, key, K, nS, 0, (int)c_hits, 0, 0.0, 0.0);
    }
    // the next colour's bound: what the drift slot holds once this cell has published
    Dg = fmax(Dg, dloc);
}

template <bool VAR>
__global__ __launch_bounds__(CW) void k_cell_coop(DevParams P, DevPtrs D, int level, CoopColours cc, int64_t sweep,
                                                  const CoopGroup* groups, const int32_t* wg_group) {
    __shared__ CoopShared sh;
    const int e = wg_group[blockIdx.x];
    if (e < 0) return;  // a launch slot no group uses
    const int gi = e & 0xFFFF, rank = e >> 16;
    const int sys = groups[gi].sys;
    unsigned gen = __hip_atomic_load(&D.gbar[2 * (1 + gi) + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double Dg = __longlong_as_double((long long)D.drift[sys]);
    for (int i = 0; i < cc.n; ++i) {
        const CoopGroup* gt = (const CoopGroup*)((const int32_t*)groups + cc.goff[i]);
        coop_cell<VAR>(P, D, level, cc.col[i], sweep, gt[gi], gi, rank, sh, gen, Dg);
    }
}

int cell_coop_blocks() {
    static int nb = -1;
    if (nb < 0) {
        int dev = 0, per_cu = 0;
        hipDeviceProp_t prop;
        // the smaller occupancy of the two instances (variants), so any launch is co-resident
        int per_v = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cell_coop<false>, CW, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_v, k_cell_coop<true>, CW, 0) != hipSuccess ||
            std::min(per_cu, per_v) < 1)
            nb = 0;
        else
            nb = std::min(std::min(per_cu, per_v) * prop.multiProcessorCount, COOP_SLOTS);
    }
    return nb;
}

bool launch_cell_coop(const DevParams& P, const DevPtrs& D, int level, const CoopColours& cc, int64_t sweep,
                      const CoopGroup* groups, const int32_t* wg_group, int nwg, hipStream_t st) {
    if (nwg <= 0 || nwg > cell_coop_blocks() || cc.n < 1 || cc.n > 8) return false;
    DevParams Pc = P;
    DevPtrs Dc = D;
    int lv = level;
    CoopColours ccc = cc;
    int64_t sw = sweep;
    const CoopGroup* gp = groups;
    const int32_t* wp = wg_group;
    void* args[] = {&Pc, &Dc, &lv, &ccc, &sw, &gp, &wp};
    const bool v = uses_variants(P);
    // cell groups compute in FP64 in both precisions, as the global-list cells
    const void* k = v ? (const void*)k_cell_coop<true> : (const void*)k_cell_coop<false>;
    return hipLaunchCooperativeKernel(k, dim3(nwg), dim3(CW), args, 0, st) == hipSuccess;
}

// ------------------------------------------------------------------- plane waves
// One workgroup per system runs its H_F chains (App. D "Generating a plane wave"): k from
// the cube by inverse CDF or from the quasi-continuous shell, Phi and e-hat, displacement
// A_F cos(k.r + Phi) e-hat on every bead, dU over every bond and WCA pair (neighbour
// grid), Metropolis test, k permuted and sign-flipped after a rejection.
__device__ void sample_k(const DevParams& P, const SysDesc& s, const DevPtrs& D, Stream& st, int l[3]) {
    const int NL = P.n_layers, Dm = 2 * NL + 1;
    if (st.co() < s.P_cube) {
        const double* cdf = D.cube_cdf + s.cube_off;
        double target = st.co() * s.W_cube;
        int lo = 0, hi = s.n_modes - 1;
        while (lo < hi) {
            int mid = (lo + hi) / 2;
            if (cdf[mid] > target) hi = mid; else lo = mid + 1;
        }
        l[0] = lo / (Dm * Dm) - NL;
        l[1] = (lo / Dm) % Dm - NL;
        l[2] = lo % Dm - NL;
        return;
    }
    const double* sh = D.shell_s + s.shell_off;
    for (int tries = 0;; ++tries) {
        if (tries >= 100000) {  // never reached with valid tables; keeps the loop bounded
            l[0] = NL + 1;
            l[1] = 0;
            l[2] = 0;
            return;
        }
        double us = st.co() * s.n_shell;
        int i = (int)floor(us);
        double fr = us - (double)i;
        double sv = sh[i] + fr * (sh[i + 1] - sh[i]);
        double vx, vy, vz;
        direction(st, vx, vy, vz);
        if (!(sv > 1e-12)) continue;
        double kmag = (s.x_s / sv) / s.lmax;
        double v[3] = {vx, vy, vz};
        bool ok = true, inside = true;
        for (int a = 0; a < 3; ++a) {
            double la = rint(kmag * v[a] * s.invks);
            if (fabs(la) > 1048576.0) ok = false;
            l[a] = ok ? (int)la : 0;
            if (abs(l[a]) > NL) inside = false;
        }
        if (ok && !inside) return;
    }
}

// Infinite system (App. D "Choosing k for an infinite system"): x = |k| lambda_max from its tail
// probability v in (0, 1], interpolated in the table s = x v at t = i/M, v = 1 - t^3
__device__ __forceinline__ double inf_x_of_v(const SysDesc& s, const DevPtrs& D, double v) {
    const double* tab = D.shell_s + s.shell_off;
    const double t = cbrt(1.0 - v), u = t * (double)s.n_shell;
    int i = (int)floor(u);
    if (i >= s.n_shell) i = s.n_shell - 1;
    const double fr = u - (double)i;
    return (tab[i] + fr * (tab[i + 1] - tab[i])) / v;
}

// |k| shell of a plane wave for the acceptance counters: floor(|l|) (periodic) or floor(x)
__device__ __forceinline__ int k_shell_periodic(const int l[3]) {
    const double lm = sqrt(((double)l[0] * (double)l[0] + (double)l[1] * (double)l[1]) + (double)l[2] * (double)l[2]);
    return lm < (double)(WMC_K_SHELLS - 1) ? (int)lm : WMC_K_SHELLS - 1;
}

__global__ __launch_bounds__(1024) void k_pw(DevParams P, DevPtrs D, int64_t sweep) {
    __shared__ double red[16];
    const int sys = blockIdx.x;
    const SysDesc& s = D.sys[sys];
    const int tid = threadIdx.x;
    const double L = s.L, invL = s.invL;
    Stream cs;
    cs.init(P, sys, sweep, TAG_PWCOUNT, 0, 0, 0, 0);
    double mu = (double)s.N * s.PF;
    int64_t HF = (int64_t)floor(mu);
    if (cs.co() < mu - (double)HF) HF += 1;
    double Dg = __longlong_as_double((long long)D.drift[sys]);
    unsigned long long c_att = 0, c_acc = 0, c_k0 = 0, c_caps = 0, c_beads = 0;
    const int64_t NN = (int64_t)(D.sys[P.nsys - 1].b1);
    double* NX = D.pw_new;
    double* NY = D.pw_new + NN;
    double* NZ = D.pw_new + 2 * NN;
    for (int64_t h = 0; h < HF; ++h) {
        Stream st;
        st.init(P, sys, sweep, TAG_PW, 0, h, 0, 0);
        // periodic: a lattice mode l; infinite: x = |k| lambda_max and an isotropic direction
        int l[3] = {0, 0, 0};
        double xk = 0.0, khat[3] = {0.0, 0.0, 0.0};
        if (P.periodic) {
            sample_k(P, s, D, st, l);
        } else {
            xk = inf_x_of_v(s, D, st.oc());
            direction(st, khat[0], khat[1], khat[2]);
        }
        for (int r = 0;;) {
            const double Phi = 2.0 * kPi * st.co();
            const double psi = 2.0 * kPi * st.co();
            const double u_acc = st.oc();
            const double thr = accept_threshold<true>(P, u_acc);
            const bool zero = P.periodic ? (l[0] == 0 && l[1] == 0 && l[2] == 0) : xk == 0.0;
            if (zero) {
                // k = 0: no displacement, deemed accepted (Sec. V "Choosing plane wave amplitude")
                ++c_k0;
                ++c_acc;
                if (tid == 0)
                    trace_push(D, 2, sys, sweep, -1, h, 0, r, 0, 1,
                               P.periodic ? (int)((512u << 20) | (512u << 10) | 512u) : 0, 0.0, thr);
                break;
            }
            double k[3];
            int shell, extra;
            if (P.periodic) {
                for (int q = 0; q < 3; ++q) k[q] = s.ks * (double)l[q];
                shell = k_shell_periodic(l);
                extra = (int)((((uint32_t)(l[0] + 512) & 0x3FFu) << 20) | (((uint32_t)(l[1] + 512) & 0x3FFu) << 10) |
                              ((uint32_t)(l[2] + 512) & 0x3FFu));
            } else {
                const double km = xk / s.lmax;
                for (int q = 0; q < 3; ++q) k[q] = km * khat[q];
                shell = xk < (double)(WMC_K_SHELLS - 1) ? (int)xk : WMC_K_SHELLS - 1;
                extra = shell;
            }
            double kmag = sqrt((k[0] * k[0] + k[1] * k[1]) + k[2] * k[2]);
            double kh[3] = {k[0] / kmag, k[1] / kmag, k[2] / kmag};
            int ax = 0;
            for (int q = 1; q < 3; ++q)
                if (fabs(kh[q]) < fabs(kh[ax])) ax = q;
            double ref[3] = {0.0, 0.0, 0.0};
            ref[ax] = 1.0;
            double e1[3] = {kh[1] * ref[2] - kh[2] * ref[1], kh[2] * ref[0] - kh[0] * ref[2],
                            kh[0] * ref[1] - kh[1] * ref[0]};
            double n1 = sqrt((e1[0] * e1[0] + e1[1] * e1[1]) + e1[2] * e1[2]);
            for (int q = 0; q < 3; ++q) e1[q] = e1[q] / n1;
            double e2[3] = {kh[1] * e1[2] - kh[2] * e1[1], kh[2] * e1[0] - kh[0] * e1[2],
                            kh[0] * e1[1] - kh[1] * e1[0]};
            double cp = cos(psi), sp = sin(psi);
            double e[3] = {cp * e1[0] + sp * e2[0], cp * e1[1] + sp * e2[1], cp * e1[2] + sp * e2[2]};
            const double AF = 2.0 * P.A0 / (kmag * sqrt(5.0 * (double)s.N));
            for (int64_t j = s.b0 + tid; j < s.b1; j += 1024) {
                double ph = ((k[0] * D.x[j] + k[1] * D.y[j]) + k[2] * D.z[j]) + Phi;
                double f = AF * cos(ph);
                NX[j] = D.x[j] + f * e[0];
                NY[j] = D.y[j] + f * e[1];
                NZ[j] = D.z[j] + f * e[2];
            }
            __syncthreads();
            double acc = 0.0;
            const double R = P.rc + 2.0 * AF + Dg + 1e-9 * L;
            for (int64_t j = s.b0 + tid; j < s.b1; j += 1024) {
                double jx = D.x[j], jy = D.y[j], jz = D.z[j];
                if (P.bond_type != WMC_BOND_NONE && j + 1 < s.b1 && D.bond_next[j]) {
                    double r2o = pair_r2(P, invL, L, jx, jy, jz, D.x[j + 1], D.y[j + 1], D.z[j + 1]);
                    double r2n = pair_r2(P, invL, L, NX[j], NY[j], NZ[j], NX[j + 1], NY[j + 1], NZ[j + 1]);
                    acc += u_bond_delta(P, r2n, r2o);
                }
                if (P.wca && !P.periodic) {
                    // infinite system (at most 8192 beads): every later bead
                    for (int64_t m = j + 1; m < s.b1; ++m) {
                        double r2o = pair_r2(P, invL, L, jx, jy, jz, D.x[m], D.y[m], D.z[m]);
                        double r2n = pair_r2(P, invL, L, NX[j], NY[j], NZ[j], NX[m], NY[m], NZ[m]);
                        if (r2o < P.rc2 || r2n < P.rc2) acc += u_pair(P, r2n) - u_pair(P, r2o);
                    }
                } else if (P.wca) {
                    double cx = wrap01(jx, L, invL), cy = wrap01(jy, L, invL), cz = wrap01(jz, L, invL);
                    int f0[3], cn[3];
                    fine_range(cx - R, cx + R, s.invg, s.nf, f0[0], cn[0]);
                    fine_range(cy - R, cy + R, s.invg, s.nf, f0[1], cn[1]);
                    fine_range(cz - R, cz + R, s.invg, s.nf, f0[2], cn[2]);
                    for (int qz = 0; qz < cn[2]; ++qz)
                        for (int qy = 0; qy < cn[1]; ++qy) {
                            // the row's cells f0[0] .. f0[0] + cn[0] - 1 (mod nf) are one range of
                            // the sorted index, two where they wrap, visited in the same order
                            const int fy = (f0[1] + qy) % s.nf, fz = (f0[2] + qz) % s.nf;
                            const int64_t rowb = s.fine_off + (int64_t)s.nf * (fy + (int64_t)s.nf * fz);
                            const int xe = f0[0] + cn[0];
                            int q = D.fstart[rowb + f0[0]], qend = D.fstart[rowb + min(xe, s.nf)];
                            for (int part = 0; part < 2; ++part) {
                                for (; q < qend; ++q) {
                                    int32_t m = D.fidx[q];
                                    if (m <= j) continue;
                                    double r2o = pair_r2(P, invL, L, jx, jy, jz, D.x[m], D.y[m], D.z[m]);
                                    double r2n = pair_r2(P, invL, L, NX[j], NY[j], NZ[j], NX[m], NY[m], NZ[m]);
                                    if (r2o < P.rc2 || r2n < P.rc2) acc += u_pair(P, r2n) - u_pair(P, r2o);
                                }
                                if (xe <= s.nf) break;
                                q = D.fstart[rowb];
                                qend = D.fstart[rowb + (xe - s.nf)];
                            }
                        }
                }
            }
            const double dU = block_sum<1024>(acc, red);
            const bool accept = dU <= thr;
            ++c_att;
            c_beads += s.N;
            if (tid == 0) {
                trace_push(D, 2, sys, sweep, -1, h, 0, r, s.N, accept ? 1 : 0, extra, dU, thr);
                atomicAdd(&D.cnt[CNT_SHELL + 2 * shell], 1ull);
                if (accept) atomicAdd(&D.cnt[CNT_SHELL + 2 * shell + 1], 1ull);
            }
            if (accept) {
                for (int64_t j = s.b0 + tid; j < s.b1; j += 1024) {
                    D.x[j] = NX[j];
                    D.y[j] = NY[j];
                    D.z[j] = NZ[j];
                }
                Dg += AF;
                ++c_acc;
                if (tid == 0) atomicAdd(&D.cnt[CNT_ACC_BEADS], (unsigned long long)s.N);
                __syncthreads();
                break;
            }
            __syncthreads();
            if (++r >= P.retry_cap) {
                ++c_caps;
                break;
            }
            // recycling (App. D): |k| kept; periodic permutes and sign-flips l, infinite redraws k-hat
            st.init(P, sys, sweep, TAG_PW, 0, h, r, 0);
            if (P.periodic) {
                int pi = (int)st.index(6);
                static const int PERM[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
                int nl[3] = {l[PERM[pi][0]], l[PERM[pi][1]], l[PERM[pi][2]]};
                for (int q = 0; q < 3; ++q) l[q] = st.co() < 0.5 ? -nl[q] : nl[q];
            } else {
                direction(st, khat[0], khat[1], khat[2]);
            }
        }
    }
    if (tid == 0) {
        unsigned long long* C = D.cnt + CNT_PW;
        atomicAdd(&C[0], (unsigned long long)HF);
        atomicAdd(&C[1], c_att);
        atomicAdd(&C[2], c_acc);
        atomicAdd(&C[3], c_k0);
        atomicAdd(&C[4], c_caps);
        atomicAdd(&C[5], c_beads);
        if (c_acc) {
            atomicAdd(&D.cnt[CNT_ACCEPTED], c_acc);
            atomicAdd(&D.sys_acc[sys], c_acc);
        }
        atomic_max_double(&D.drift[sys], Dg);
    }
}


// Plane waves on groups of workgroups (cooperative launch: all co-resident), one group per
// system, sized by its bead count. A group's beads are strided over its workgroups; each test
// takes two group barriers (trial positions written; per-workgroup dU partial sums written) and
// a third after an accepted move. Every workgroup sums the partial sums in the same order, so
// all take the same decision.
__global__ __launch_bounds__(256) void k_pw_coop(DevParams P, DevPtrs D, int64_t sweep, const CoopGroup* groups,
                                                 const int32_t* wg_group) {
    __shared__ double red[4];
    const int e = wg_group[blockIdx.x];
    if (e < 0) return;  // a launch slot no group uses
    const int gi = e & 0xFFFF;
    const CoopGroup grp = groups[gi];
    const int sys = grp.sys;
    const SysDesc& s = D.sys[sys];
    const int tid = threadIdx.x;
    const unsigned G = grp.size;
    const int rank = e >> 16;
    const int64_t stride = (int64_t)G * 256;
    const int64_t g0 = s.b0 + (int64_t)rank * 256 + tid;
    const double L = s.L, invL = s.invL;
    unsigned* bar = D.gbar + 2 * (1 + gi);
    unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    Stream cs;
    cs.init(P, sys, sweep, TAG_PWCOUNT, 0, 0, 0, 0);
    double mu = (double)s.N * s.PF;
    int64_t HF = (int64_t)floor(mu);
    if (cs.co() < mu - (double)HF) HF += 1;
    double Dg = __longlong_as_double((long long)D.drift[sys]);
    unsigned long long c_att = 0, c_acc = 0, c_k0 = 0, c_caps = 0, c_beads = 0;
    const int64_t NN = (int64_t)(D.sys[P.nsys - 1].b1);
    double* NX = D.pw_new;
    double* NY = D.pw_new + NN;
    double* NZ = D.pw_new + 2 * NN;
    int parity = 0;
    for (int64_t h = 0; h < HF; ++h) {
        Stream st;
        st.init(P, sys, sweep, TAG_PW, 0, h, 0, 0);
        int l[3];
        sample_k(P, s, D, st, l);
        for (int r = 0;;) {
            const double Phi = 2.0 * kPi * st.co();
            const double psi = 2.0 * kPi * st.co();
            const double u_acc = st.oc();
            const double thr = accept_threshold<true>(P, u_acc);
            if (l[0] == 0 && l[1] == 0 && l[2] == 0) {
                ++c_k0;
                ++c_acc;
                if (rank == 0 && tid == 0)
                    trace_push(D, 2, sys, sweep, -1, h, 0, r, 0, 1, (int)((512u << 20) | (512u << 10) | 512u), 0.0,
                               thr);
                break;
            }
            double k[3] = {s.ks * (double)l[0], s.ks * (double)l[1], s.ks * (double)l[2]};
            double kmag = sqrt((k[0] * k[0] + k[1] * k[1]) + k[2] * k[2]);
            double kh[3] = {k[0] / kmag, k[1] / kmag, k[2] / kmag};
            int ax = 0;
            for (int q = 1; q < 3; ++q)
                if (fabs(kh[q]) < fabs(kh[ax])) ax = q;
            double ref[3] = {0.0, 0.0, 0.0};
            ref[ax] = 1.0;
            double e1[3] = {kh[1] * ref[2] - kh[2] * ref[1], kh[2] * ref[0] - kh[0] * ref[2],
                            kh[0] * ref[1] - kh[1] * ref[0]};
            double n1 = sqrt((e1[0] * e1[0] + e1[1] * e1[1]) + e1[2] * e1[2]);
            for (int q = 0; q < 3; ++q) e1[q] = e1[q] / n1;
            double e2[3] = {kh[1] * e1[2] - kh[2] * e1[1], kh[2] * e1[0] - kh[0] * e1[2],
                            kh[0] * e1[1] - kh[1] * e1[0]};
            double cp = cos(psi), sp = sin(psi);
            double e[3] = {cp * e1[0] + sp * e2[0], cp * e1[1] + sp * e2[1], cp * e1[2] + sp * e2[2]};
            const double AF = 2.0 * P.A0 / (kmag * sqrt(5.0 * (double)s.N));
            for (int64_t j = g0; j < s.b1; j += stride) {
                double ph = ((k[0] * D.x[j] + k[1] * D.y[j]) + k[2] * D.z[j]) + Phi;
                double f = AF * cos(ph);
                NX[j] = D.x[j] + f * e[0];
                NY[j] = D.y[j] + f * e[1];
                NZ[j] = D.z[j] + f * e[2];
            }
            group_barrier(bar, G, gen);
            double acc = 0.0;
            const double R = P.rc + 2.0 * AF + Dg + 1e-9 * L;
            for (int64_t j = g0; j < s.b1; j += stride) {
                double jx = D.x[j], jy = D.y[j], jz = D.z[j];
                if (P.bond_type != WMC_BOND_NONE && j + 1 < s.b1 && D.bond_next[j]) {
                    double r2o = pair_r2(P, invL, L, jx, jy, jz, D.x[j + 1], D.y[j + 1], D.z[j + 1]);
                    double r2n = pair_r2(P, invL, L, NX[j], NY[j], NZ[j], NX[j + 1], NY[j + 1], NZ[j + 1]);
                    acc += u_bond_delta(P, r2n, r2o);
                }
                if (P.wca) {
                    double cx = wrap01(jx, L, invL), cy = wrap01(jy, L, invL), cz = wrap01(jz, L, invL);
                    int f0[3], cn[3];
                    fine_range(cx - R, cx + R, s.invg, s.nf, f0[0], cn[0]);
                    fine_range(cy - R, cy + R, s.invg, s.nf, f0[1], cn[1]);
                    fine_range(cz - R, cz + R, s.invg, s.nf, f0[2], cn[2]);
                    for (int qz = 0; qz < cn[2]; ++qz)
                        for (int qy = 0; qy < cn[1]; ++qy) {
                            // the row's cells f0[0] .. f0[0] + cn[0] - 1 (mod nf) are one range of
                            // the sorted index, two where they wrap, visited in the same order
                            const int fy = (f0[1] + qy) % s.nf, fz = (f0[2] + qz) % s.nf;
                            const int64_t rowb = s.fine_off + (int64_t)s.nf * (fy + (int64_t)s.nf * fz);
                            const int xe = f0[0] + cn[0];
                            int q = D.fstart[rowb + f0[0]], qend = D.fstart[rowb + min(xe, s.nf)];
                            for (int part = 0; part < 2; ++part) {
                                for (; q < qend; ++q) {
                                    int32_t m = D.fidx[q];
                                    if (m <= j) continue;
                                    double r2o = pair_r2(P, invL, L, jx, jy, jz, D.x[m], D.y[m], D.z[m]);
                                    double r2n = pair_r2(P, invL, L, NX[j], NY[j], NZ[j], NX[m], NY[m], NZ[m]);
                                    if (r2o < P.rc2 || r2n < P.rc2) acc += u_pair(P, r2n) - u_pair(P, r2o);
                                }
                                if (xe <= s.nf) break;
                                q = D.fstart[rowb];
                                qend = D.fstart[rowb + (xe - s.nf)];
                            }
                        }
                }
            }
            double part = block_sum<256>(acc, red);
            double* partials = D.coop_d + (parity ? COOP_SLOTS : 0) + grp.first;
            if (tid == 0) partials[rank] = part;
            group_barrier(bar, G, gen);
            double dU = 0.0;
            for (unsigned b = 0; b < G; ++b) dU += partials[b];
            parity ^= 1;
            const bool accept = dU <= thr;
            ++c_att;
            c_beads += s.N;
            if (rank == 0 && tid == 0) {
                int extra = (int)((((uint32_t)(l[0] + 512) & 0x3FFu) << 20) | (((uint32_t)(l[1] + 512) & 0x3FFu) << 10) |
                                  ((uint32_t)(l[2] + 512) & 0x3FFu));
                trace_push(D, 2, sys, sweep, -1, h, 0, r, s.N, accept ? 1 : 0, extra, dU, thr);
                const int shell = k_shell_periodic(l);
                atomicAdd(&D.cnt[CNT_SHELL + 2 * shell], 1ull);
                if (accept) atomicAdd(&D.cnt[CNT_SHELL + 2 * shell + 1], 1ull);
            }
            if (accept) {
                for (int64_t j = g0; j < s.b1; j += stride) {
                    D.x[j] = NX[j];
                    D.y[j] = NY[j];
                    D.z[j] = NZ[j];
                }
                Dg += AF;
                ++c_acc;
                if (rank == 0 && tid == 0) atomicAdd(&D.cnt[CNT_ACC_BEADS], (unsigned long long)s.N);
                group_barrier(bar, G, gen);
                break;
            }
            if (++r >= P.retry_cap) {
                ++c_caps;
                break;
            }
            st.init(P, sys, sweep, TAG_PW, 0, h, r, 0);
            int pi = (int)st.index(6);
            static const int PERM[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
            int nl[3] = {l[PERM[pi][0]], l[PERM[pi][1]], l[PERM[pi][2]]};
            for (int q = 0; q < 3; ++q) l[q] = st.co() < 0.5 ? -nl[q] : nl[q];
        }
    }
    if (rank == 0 && tid == 0) {
        unsigned long long* C = D.cnt + CNT_PW;
        atomicAdd(&C[0], (unsigned long long)HF);
        atomicAdd(&C[1], c_att);
        atomicAdd(&C[2], c_acc);
        atomicAdd(&C[3], c_k0);
        atomicAdd(&C[4], c_caps);
        atomicAdd(&C[5], c_beads);
        if (c_acc) {
            atomicAdd(&D.cnt[CNT_ACCEPTED], c_acc);
            atomicAdd(&D.sys_acc[sys], c_acc);
        }
        atomic_max_double(&D.drift[sys], Dg);
    }
}

int pw_coop_blocks() {
    static int nb = -1;
    if (nb < 0) {
        int dev = 0, per_cu = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pw_coop, 256, 0) != hipSuccess || per_cu < 1)
            nb = 0;
        else
            nb = std::min(per_cu * prop.multiProcessorCount, COOP_SLOTS);
    }
    return nb;
}

bool launch_pw_coop(const DevParams& P, const DevPtrs& D, int64_t sweep, const CoopGroup* groups,
                    const int32_t* wg_group, int nwg, hipStream_t st) {
    if (nwg <= 0 || nwg > pw_coop_blocks()) return false;
    DevParams Pc = P;
    DevPtrs Dc = D;
    int64_t sw = sweep;
    const CoopGroup* gp = groups;
    const int32_t* wp = wg_group;
    void* args[] = {&Pc, &Dc, &sw, &gp, &wp};
    return hipLaunchCooperativeKernel((const void*)k_pw_coop, dim3(nwg), dim3(256), args, 0, st) == hipSuccess;
}

void launch_pw(const DevParams& P, const DevPtrs& D, int64_t sweep, int nsys, hipStream_t st) {
    hipLaunchKernelGGL(k_pw, dim3(nsys), dim3(1024), 0, st, P, D, sweep);
}

// ------------------------------------------------------------------- observables
// Eq. "Radius of gyration": (1/(2 Nb^2)) sum_ij r_ij^2 = (1/Nb) sum_i |r_i - r_cm|^2
__global__ void k_rg2(DevPtrs D, const int64_t* chain_off, int64_t n_chains, double* out) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chains) return;
    int64_t a = chain_off[c], b = chain_off[c + 1];
    double nb = (double)(b - a), cx = 0, cy = 0, cz = 0;
    for (int64_t i = a; i < b; ++i) {
        cx += D.x[i];
        cy += D.y[i];
        cz += D.z[i];
    }
    cx /= nb;
    cy /= nb;
    cz /= nb;
    double acc = 0.0;
    for (int64_t i = a; i < b; ++i) {
        double dx = D.x[i] - cx, dy = D.y[i] - cy, dz = D.z[i] - cz;
        acc += (dx * dx + dy * dy) + dz * dz;
    }
    out[c] = acc / nb;
}

void launch_rg2(const DevPtrs& D, const int64_t* chain_off, int64_t n_chains, double* out, hipStream_t st) {
    if (n_chains <= 0) return;
    hipLaunchKernelGGL(k_rg2, dim3((unsigned)((n_chains + 255) / 256)), dim3(256), 0, st, D, chain_off, n_chains,
                       out);
}

// ------------------------------------------------------------ library-held arena
// Device memory of the contexts made by wmc_init_static, for callers that cannot allocate device
// memory (code under graph capture, serving loops that forbid allocation). One array per device,
// held until the process ends. In host code `scratch` names a host-side stand-in, not a device
// address: only the pointer hipGetSymbolAddress returns (kept per device) is ever passed on.
static __device__ __align__(256) unsigned char scratch[WMC_STATIC_ARENA_BYTES];

void* static_arena(int device, hipError_t* err) {
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {nullptr};
    *err = hipSuccess;
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        ptr[device] = p;
    }
    return ptr[device];
}

// centre of mass of every chain (Sec. VI.B); mode 0 writes it to out [3 n], mode 1 to D.com_ref, mode
// 2 writes |com - com_ref|^2 to out [n]
__global__ void k_com(DevPtrs D, const int64_t* chain_off, int64_t n_chains, int mode, double* out) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chains) return;
    int64_t a = chain_off[c], b = chain_off[c + 1];
    double cx = 0.0, cy = 0.0, cz = 0.0;
    for (int64_t i = a; i < b; ++i) {
        cx += D.x[i];
        cy += D.y[i];
        cz += D.z[i];
    }
    const double nb = (double)(b - a);
    cx /= nb;
    cy /= nb;
    cz /= nb;
    if (mode == 2) {
        const double dx = cx - D.com_ref[3 * c], dy = cy - D.com_ref[3 * c + 1], dz = cz - D.com_ref[3 * c + 2];
        out[c] = (dx * dx + dy * dy) + dz * dz;
        return;
    }
    double* o = mode == 1 ? D.com_ref : out;
    o[3 * c] = cx;
    o[3 * c + 1] = cy;
    o[3 * c + 2] = cz;
}

void launch_com(const DevPtrs& D, const int64_t* chain_off, int64_t n_chains, int mode, double* out, hipStream_t st) {
    if (n_chains <= 0) return;
    hipLaunchKernelGGL(k_com, dim3((unsigned)((n_chains + 255) / 256)), dim3(256), 0, st, D, chain_off, n_chains, mode,
                       out);
}

// ------------------------------------------------------------------- debug kernels
__global__ void k_cell_ids(DevParams P, DevPtrs D, int sys, int level, int64_t sweep, int32_t* out) {
    const SysDesc& s = D.sys[sys];
    const LevelDesc& lv = D.lev[s.lvl_off + level];
    Grid g;
    make_grid(P, D, s, lv, sys, level, sweep, g);
    int64_t i = s.b0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.b1) return;
    out[i - s.b0] = (int32_t)cell_of_point(g, D.x[i], D.y[i], D.z[i]);
}

void launch_cell_ids(const DevParams& P, const DevPtrs& D, int sys, int level, int64_t sweep, int64_t n, int32_t* out,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_cell_ids, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, D, sys, level, sweep, out);
}

__global__ void k_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1, int64_t n,
                         uint32_t* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[4] = {c0 + (uint32_t)i, c1, c2, c3};
    philox10(c, k0, k1);
    for (int q = 0; q < 4; ++q) out[4 * i + q] = c[q];
}

void launch_philox(const uint32_t* ctr, const uint32_t* key, int64_t n, uint32_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ctr[0], ctr[1], ctr[2], ctr[3],
                       key[0], key[1], n, out);
}

}  // namespace wmc
