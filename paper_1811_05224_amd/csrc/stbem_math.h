// Element-pair mathematics of the space-time Galerkin BEM for the 2D heat
// equation (arXiv:1811.05224, Sec. 1 eq.(4) and Sec. 2 Thm 1), written once
// for the gfx950 kernels.  Every function is __host__ __device__ so the same
// arithmetic can be exercised from a host build of this header.
//
// Time integrals.  With k(r,s) = exp(-alpha r^2/(4s)) / (4 pi s) (that is
// U*/alpha) and a = alpha r^2/4, the double integral over time elements
// tau_k x tau_m of a causal kernel is the four-point difference of its second
// time antiderivative F:
//   F_V(d) = [(d+a) E1(a/d) - d e^{-a/d}]/(4 pi)          single layer
//   F_K(d) =  d e^{-a/d} - a E1(a/d)    (x (x-y).n_y/(2 pi r^2))  double layer
//   F_D(d) =  E1(a/d)/(4 pi)    first antiderivative, paired with d/dt of k
// Touching time elements (lag d = k - m in {0,1}) use these closed forms.
// Separated elements use the exact series obtained by expanding the kernel
// about the distance dc of the element centres: with z = a/dc and the even
// moments mu_2n of the trapezoid weight (box convolved with box),
//   V : e^{-z}/(4 pi dc)  sum_n L_2n(z)           mu_2n/dc^2n
//   K : (a/dc^2) e^{-z}   sum_n L^(1)_2n(z)       mu_2n/dc^2n
//   D : -e^{-z}/(4 pi dc^2) sum_n (2n+1) L_2n+1(z) mu_2n/dc^2n
// (Laguerre generating function e^{-z/(1+u)}/(1+u)^{b+1} = e^{-z} sum L^(b)_n(z)(-u)^n).
// It has no cancellation, unlike the four-point difference of large values.
//
// Spatial integrals.  Pieces are straight (segments, or half-segments for the
// dual mesh).  Separated pieces use a tensor Gauss-Legendre rule; pieces that
// coincide or share a vertex, on touching time elements, have a log (or,
// for K, 1/r) singularity.  There the kernel is split exactly as
// A(r) + B(r) ln r with A smooth and B a polynomial in r^2, the Duffy /
// difference-variable substitution makes ln r = ln u + ln(smooth), and the
// ln u part is integrated with a Gauss rule for the weight -ln u.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "e1_poly_table.h"
#include "exp2_table.h"

#define SDEV __host__ __device__ __forceinline__

namespace stbem {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEuler = 0.57721566490153286061;
constexpr double kInv4Pi = 0.079577471545947667884;   // 1/(4 pi)
constexpr double kInv2Pi = 0.15915494309189533577;    // 1/(2 pi)

constexpr int kMaxGL = 16;       // largest Gauss-Legendre order in the tables
constexpr int kMaxLog = 8;       // largest order of the -ln u rule
constexpr int kMaxTerms = 40;    // series terms for separated time elements
// Truncation of that series: terms n = 0..N are kept, N the first n >= 1 with
// p^(2n+2) < kSeriesTol (p = sum of the half-lengths / centre lag).  As
// |e^{-z} L^(b)_m(z)| <= C(m+b, m) e^{-z/2} and c_n <= 2 c_0 p^(2n) /
// ((2n+1)(2n+2)) (equal steps), each omitted term of the b = 0, 1, 2 sums is
// at most c_0 p^(2n) e^{-z/2}; the whole tail stays below 1.7 kSeriesTol of
// the leading coefficient (p <= 0.62), under the FP64 rounding of the sums.
constexpr double kSeriesTol = 1e-17;

// Quadrature tables on [0,1]: gl_x[n][i], gl_w[n][i] for n = 1..kMaxGL,
// and the n-point rule for int_0^1 f(u) (-ln u) du.
struct Tables {
    double gl_x[kMaxGL + 1][kMaxGL];
    double gl_w[kMaxGL + 1][kMaxGL];
    double lg_x[kMaxLog + 1][kMaxLog];
    double lg_w[kMaxLog + 1][kMaxLog];
    double ex2[64];                       // 2^(-j/64), j = 0..63 (exp_neg)
};

// e^{-z} for z >= 0 by the table-driven method of Tang (1989): with
// z = (64 m + j) ln2/64 + r, |r| <= ln2/128, e^{-z} = 2^{-m} 2^{-j/64} e^{-r},
// e^{-r} from its degree-5 Taylor polynomial (remainder < 4e-17).  ln2/64 is
// split in a 36-bit head and a tail so that k ln2/64 is subtracted exactly.
// Arguments beyond 2^24 ln2/64 (where e^{-z} is 0 in double) are clamped
// before the integer conversion; the scaling by 2^{-m} then underflows to 0.
constexpr double kLn2o64Hi = 0x1.62e42fefa0000p-7;
constexpr double kLn2o64Lo = 2.572804622327669e-14;
constexpr double k64oLn2 = 92.33248261689366;
SDEV double exp_neg(double z, const double* ex2)
{
    const double k = fmin(rint(z * k64oLn2), 16777216.0);
    double r = fma(-k, kLn2o64Hi, z);
    r = fma(-k, kLn2o64Lo, r);
    const double p = fma(fma(fma(fma(fma(-1.0 / 120.0, r, 1.0 / 24.0), r, -1.0 / 6.0), r, 0.5), r, -1.0), r, 1.0);
    const int ki = (int)k;
    return ldexp(ex2[ki & 63] * p, -(ki >> 6));
}

// Geometry of Gamma_h (closed CCW polygon) and the time grid.
struct Geom {
    int ng, nt;
    double alpha;
    const double *vx, *vy;          // polygon vertices
    const double *ex, *ey, *len;    // unit tangent and length of segment i = [v_i, v_{i+1}]
    const double* t;                // nt + 1 time nodes
    int toep;                       // 1: block (k, m) stored at its lag k - m (uniform steps)
};

// storage slot of block (k, m) with packed index b
SDEV long long block_slot(const Geom& g, long long b, int k, int m) { return g.toep ? (long long)(k - m) : b; }

// Quadrature orders chosen by the host per problem.
constexpr int kNearClasses = 6;

struct Orders {
    int q_sing;          // Gauss-Legendre order of the singular rules (smooth parts)
    int q_log;           // order of the -ln u rule
    int q_near[kNearClasses];         // regular rule on touching time elements by distance class
    double eta_cut[kNearClasses - 1]; // distance/length thresholds between the classes
    double eta_raw;      // D_h: pieces farther apart use the raw-kernel form
    double q_tol;        // touching elements: bound on the Gauss remainder of the e^{-z} factor
    double z_floor;      // entries below e^{-z_floor} of the block maximum need absolute accuracy only
};

// ------------------------------------------------------------------ E1
// Ein(z) = sum_{n>=1} (-1)^{n+1} z^n/(n n!), entire; used for 0 <= z <= 2,
// where 24 terms leave a tail below 1e-18 of the sum: z (c_1 + c_2 z + ...),
// c_n = (-1)^{n+1}/(n n!).
struct EinCoef { double c[24]; };
constexpr EinCoef ein_coef()
{
    EinCoef e{};
    double f = 1.0;
    for (int n = 1; n <= 24; ++n) {
        f *= n;
        e.c[n - 1] = ((n & 1) ? 1.0 : -1.0) / (n * f);
    }
    return e;
}
constexpr EinCoef kEin = ein_coef();

// The terms from c_5 on are evaluated in chunks of four coefficients,
// c0 + c1 z + (c2 + c3 z) z^2 each, joined by Horner in z^4, and the first
// four by Horner on top of them: a dependent chain of about 12 operations
// instead of 24, with the rounding of Horner's last steps.
SDEV double ein(double z)
{
    const double z2 = z * z, z4 = z2 * z2;
    const double* c = kEin.c;
    double p = 0.0;
#pragma unroll
    for (int k = 5; k >= 1; --k)
        p = fma(p, z4, fma(fma(c[4 * k + 3], z, c[4 * k + 2]), z2, fma(c[4 * k + 1], z, c[4 * k])));
    p = fma(fma(fma(fma(p, z, c[3]), z, c[2]), z, c[1]), z, c[0]);
    return p * z;
}

// E1(z) for z > 0 (and, with EX, ex = e^{-z}): -gamma - ln z + Ein(z) for
// z <= 2; on [2, 64) e^{-z} times a polynomial for e^z E1(z) per
// half-octave (fitted with mpmath, relative error < 2.1e-16, in the local
// variable); beyond, the continued fraction
// e^{-z}/(z+1 - 1^2/(z+3 - 2^2/(z+5 - ...))) evaluated from the tail.  The
// exponential is shared with the caller.
static_assert(kE1PolyN == 19, "e1t evaluates 4 chunks of 4 and one of 3 coefficients");
template <bool EX>
SDEV double e1t(double z, double& ex)
{
    if (z <= 2.0) {
        if (EX) ex = exp(-z);
        return -kEuler - log(z) + ein(z);
    }
    if (z > 740.0) { ex = 0.0; return 0.0; }
    ex = exp(-z);
    if (z < 64.0) {
        // octave [lo, 2 lo), lo = 2^(o+1), halves [lo, 1.5 lo) and [1.5 lo, 2 lo)
        const int o = z < 4.0 ? 0 : z < 8.0 ? 1 : z < 16.0 ? 2 : z < 32.0 ? 3 : 4;
        const double lo = (double)(2 << o);
        const int hh = z >= 1.5 * lo ? 1 : 0;
        const double x = (z - lo * (1.0 + 0.5 * hh)) * (4.0 / lo) - 1.0;   // z - a exact
        const double* co = kE1Poly[2 * o + hh];
        // fixed length (shorter rows are zero-padded), unrolled so that the
        // coefficient loads of the lane's interval issue ahead of the sum;
        // from co[4] on chunks of four joined by Horner in x^4, the first
        // four by Horner on top (as in ein)
        const double x2 = x * x, x4 = x2 * x2;
        double p = fma(co[18], x2, fma(co[17], x, co[16]));
#pragma unroll
        for (int k = 3; k >= 1; --k)
            p = fma(p, x4, fma(fma(co[4 * k + 3], x, co[4 * k + 2]), x2, fma(co[4 * k + 1], x, co[4 * k])));
        p = fma(fma(fma(fma(p, x, co[3]), x, co[2]), x, co[1]), x, co[0]);
        return ex * p;
    }
    // the fraction's tail n^2/(z + 2n + 1 - ...) for n = 6 .. 1 carried as
    // a ratio nu/de (all terms positive), so that one division remains
    double nu = 36.0, de = z + 13.0;
#pragma unroll
    for (int n = 5; n >= 1; --n) {
        const double d2 = fma(z + (2.0 * n + 1.0), de, -nu);
        nu = (double)(n * n) * de;
        de = d2;
    }
    return ex * de / fma(z + 1.0, de, -nu);
}

SDEV double e1x(double z, double& ex) { return e1t<true>(z, ex); }

// E1 for callers whose arguments are nearly always > 2: the branch z <= 2
// (its 24 series constants) is kept out of line, so that it holds no
// registers in the caller's loops.
template <bool EX>
__host__ __device__ __attribute__((noinline)) double e1_small(double z, double& ex)
{
    if (EX) ex = exp(-z);
    return -kEuler - log(z) + ein(z);
}
template <bool EX>
SDEV double e1t_large(double z, double& ex)
{
    if (z <= 2.0) return e1_small<EX>(z, ex);
    return e1t<EX>(z, ex);
}
SDEV double e1(double z)
{
    double ex;
    return e1t<false>(z, ex);
}

// E1(a/d) + 2 ln r written without ln a when a/d is small:
//   E1(a/d) = -gamma - ln(alpha/4) + ln d - 2 ln r + Ein(a/d)
// so ez(...) - 2 ln r = E1.  For large a/d it is E1 + 2 ln r directly.
SDEV double ez_part(double z, double c0, double lnd, double lnr, double& ex)
{
    if (z <= 2.0) { ex = exp(-z); return c0 + lnd + ein(z); }
    return e1x(z, ex) + 2.0 * lnr;
}

// ------------------------------------------------------------ time blocks
enum Op { OP_V = 0, OP_K = 1, OP_D = 2, OP_DV = 4, OP_DK = 5 };

struct TimeBlock {
    int d;                // 0, 1 (touching elements) or 2 (separated elements)
    int ser;              // 1: separated elements evaluated by the series
    int nterm;            // series terms
    double del[4];        // positive lags of the closed form: d=0 {h_k};
    double sgn[4];        //   d=1 {h_k + h_m, h_k, h_m}; d>=2 all four
    double lnd[4];
    double idel[4];       // 1 / del
    int ndel;
    double dc, inv_dc;    // centre distance (separated)
    double w2;            // alpha / (4 smallest lag): z = w2 r^2 bounds a / delta
    // Series step n (n >= 1 advances P_{2n-1} -> P_{2n} -> P_{2n+1}; n = 0
    // holds the coefficients of P_0 = L_0, P_1 = L_1), with the rescaled
    // Laguerre polynomials P_j = L_j / gam_j, P_{j+1} = (a_j - b_j z) P_j - P_{j-1}:
    //   st[n][0..1] = a, b for j = 2n - 1         st[n][3..4] = a, b for j = 2n
    //   st[n][6..7] = kc_{2n}, kc_{2n+1}          st[n][8..9] = hc_{2n}, hc_{2n+1}
    //   st[n][10]   = (2n + 1) c_n                st[n][11]   = c_n
    // (st[n][2], st[n][5] unused), where c_n = mu_2n / dc^2n, kc and hc are the
    // coefficients of L_m in sum_n c_n L^(1)_2n and sum_n c_n L^(2)_2n (tail
    // sums of c), and the entries 6..11 carry the factor gam_m of their L_m
    // (see time_block).
    alignas(16) double st[kMaxTerms][12];
};

// Build the time block (k, m), k >= m, from the node array.
SDEV void time_block(const Geom& g, int k, int m, TimeBlock& tb)
{
    double hk = g.t[k + 1] - g.t[k], hm = g.t[m + 1] - g.t[m];
    tb.d = (k - m >= 2) ? 2 : (k - m);
    tb.nterm = 0;
    tb.ser = 0;
    {
        double lag = (k == m) ? hk : (k == m + 1 ? (hk < hm ? hk : hm) : g.t[k] - g.t[m + 1]);
        tb.w2 = 0.25 * g.alpha / lag;
    }
    if (tb.d == 0) {
        tb.ndel = 1; tb.del[0] = hk; tb.sgn[0] = 1.0;
    } else if (tb.d == 1) {
        tb.ndel = 3;
        tb.del[0] = hk + hm; tb.sgn[0] = 1.0;
        tb.del[1] = hk;      tb.sgn[1] = -1.0;
        tb.del[2] = hm;      tb.sgn[2] = -1.0;
        if (hk == hm) { tb.ndel = 2; tb.sgn[1] = -2.0; }   // equal steps: one term
    } else {
        tb.ndel = 0;
        double A = 0.5 * hk, B = 0.5 * hm;
        double dc = 0.5 * (g.t[k] + g.t[k + 1]) - 0.5 * (g.t[m] + g.t[m + 1]);
        tb.dc = dc; tb.inv_dc = 1.0 / dc;
        double p = (A + B) / dc, q = (A - B) / dc;
        if (p > 0.62) {
            // series converges too slowly (a short gap between long elements):
            // four-point closed form
            tb.ndel = 4;
            tb.del[0] = g.t[k + 1] - g.t[m];     tb.sgn[0] = 1.0;
            tb.del[1] = g.t[k + 1] - g.t[m + 1]; tb.sgn[1] = -1.0;
            tb.del[2] = g.t[k] - g.t[m];         tb.sgn[2] = -1.0;
            tb.del[3] = g.t[k] - g.t[m + 1];     tb.sgn[3] = 1.0;
            for (int s = 0; s < 4; ++s) { tb.lnd[s] = log(tb.del[s]); tb.idel[s] = 1.0 / tb.del[s]; }
            return;
        }
        tb.ser = 1;
        // mu_2n/dc^2n = 2 dc^2 [p^{2n+2} - q^{2n+2}] / ((2n+1)(2n+2))
        double p2 = p * p, q2 = q * q, pp = p2, qq = q2;
        int n = 0;
        for (; n < kMaxTerms; ++n) {
            tb.st[n][11] = 2.0 * dc * dc * (pp - qq) / ((2.0 * n + 1.0) * (2.0 * n + 2.0));
            if (n > 0 && pp < kSeriesTol) { ++n; break; }
            pp *= p2; qq *= q2;
        }
        tb.nterm = n;
        // L^(1)_2n = sum_{m <= 2n} L_m, so sum_n c_n L^(1)_2n = sum_m kc_m L_m with
        // kc_m = sum_{2n >= m} c_n; likewise sum_n c_n L^(2)_2n = sum_m hc_m L_m,
        // hc_m = sum_{2n >= m} (2n - m + 1) c_n, i.e. hc_m = hc_{m+1} + kc_m.  All
        // terms are positive (p > |q|), so these tail sums do not cancel.
        double kc = 0.0, hc = 0.0;
        for (int e = n - 1; e >= 0; --e) {
            const double cn = tb.st[e][11];
            tb.st[e][7] = e + 1 < n ? kc : 0.0;     // kc_{2e+1}: n' >= e + 1
            hc += tb.st[e][7];
            tb.st[e][9] = e + 1 < n ? hc : 0.0;
            kc += cn;                               // kc_{2e}: n' >= e
            tb.st[e][6] = kc;
            hc += kc;
            tb.st[e][8] = hc;
            tb.st[e][10] = (2.0 * e + 1.0) * cn;
        }
        // Rescaled recurrence (one operation fewer per step): P_j = L_j / gam_j
        // with gam_0 = gam_1 = 1 and gam_{j+1} = C_j gam_{j-1}, C_j = j/(j+1), so
        // that P_{j+1} = (a_j - b_j z) P_j - P_{j-1} with
        // a_j = (2j+1)/(j+1) gam_j/gam_{j+1}, b_j = 1/(j+1) gam_j/gam_{j+1}; the
        // coefficients of the sums take the factor gam_m of their L_m.
        double gjm1 = 1.0, gj = 1.0;                // gam_{j-1}, gam_j at j = 1
        for (int e = 1; e < n; ++e) {
            for (int h = 0; h < 2; ++h) {
                const int j = 2 * e - 1 + h;            // step L_{j-1}, L_j -> L_{j+1}
                const double b = 1.0 / (j + 1.0), gjp1 = j * b * gjm1;
                tb.st[e][3 * h] = (2.0 * j + 1.0) * b * gj / gjp1;
                tb.st[e][3 * h + 1] = b * gj / gjp1;
                tb.st[e][3 * h + 2] = 0.0;
                gjm1 = gj; gj = gjp1;
            }
            // gjm1 = gam_{2e}, gj = gam_{2e+1}
            tb.st[e][6] *= gjm1; tb.st[e][8] *= gjm1; tb.st[e][11] *= gjm1;
            tb.st[e][7] *= gj;   tb.st[e][9] *= gj;   tb.st[e][10] *= gj;
        }
        for (int c = 0; c < 6; ++c) tb.st[0][c] = 0.0;  // term 0 holds L_0 = 1, L_1 = 1 - z
    }
    for (int s = 0; s < tb.ndel; ++s) { tb.lnd[s] = log(tb.del[s]); tb.idel[s] = 1.0 / tb.del[s]; }
}

// Separated time elements: the series at z = a/dc.
//   v  = Delta F_V,  k = Delta F_K,  dd = Delta F_D,
//   va = d/da Delta F_V = -e^{-z}/(4 pi dc^2) sum c_n L^(1)_2n(z)
//   vaa= d2/da2 Delta F_V =  e^{-z}/(4 pi dc^3) sum c_n L^(2)_2n(z)
// (d/dz [e^{-z} L^(b)_n] = -e^{-z} L^(b+1)_n, L^(b+1)_n = sum_{j<=n} L^(b)_j).
struct SeriesVals { double v, k, dd, va, vaa; };

template <bool NEED_V, bool NEED_K, bool NEED_D, bool NEED_H = false>
SDEV SeriesVals series(const TimeBlock& tb, double a)
{
    double z = a * tb.inv_dc, ez = exp(-z);
    double l0 = 1.0, l1 = 1.0 - z;          // L_0, L_1
    const double* s0 = tb.st[0];
    double sv = s0[11], sk = s0[6] + s0[7] * l1, sd = s0[10] * l1, s2 = s0[8] + s0[9] * l1;
    for (int n = 1; n < tb.nterm; ++n) {
        const double* st = tb.st[n];        // advance to L_{2n}, L_{2n+1}
        const double l2 = fma(fma(-st[1], z, st[0]), l1, -l0);
        const double l3 = fma(fma(-st[4], z, st[3]), l2, -l1);
        if (NEED_V) sv = fma(st[11], l2, sv);
        if (NEED_K || NEED_H) sk = fma(st[7], l3, fma(st[6], l2, sk));
        if (NEED_D) sd = fma(st[10], l3, sd);
        if (NEED_H) s2 = fma(st[9], l3, fma(st[8], l2, s2));
        l0 = l2; l1 = l3;
    }
    SeriesVals r;
    double i1 = tb.inv_dc, i2 = i1 * i1;
    r.v = NEED_V ? ez * i1 * kInv4Pi * sv : 0.0;
    r.k = NEED_K ? a * i2 * ez * sk : 0.0;
    r.dd = NEED_D ? -ez * i2 * kInv4Pi * sd : 0.0;
    r.va = NEED_H ? -ez * i2 * kInv4Pi * sk : 0.0;
    r.vaa = NEED_H ? ez * i2 * i1 * kInv4Pi * s2 : 0.0;
    return r;
}

// Touching time elements, regular point: closed forms per lag.
struct TouchVals { double v, k, dd, dv, e; };  // Delta F_V, F_K, F_D, dF_V/dalpha, Delta E1

template <bool NEED_V, bool NEED_K, bool NEED_D, bool NEED_DV, bool NEED_E>
SDEV TouchVals touch(const TimeBlock& tb, double a, double alpha)
{
    TouchVals r = {0, 0, 0, 0, 0};
    for (int s = 0; s < tb.ndel; ++s) {
        double d = tb.del[s], z = a * tb.idel[s], x;
        double E = e1x(z, x), sg = tb.sgn[s];
        if (NEED_V) r.v += sg * ((d + a) * E - d * x);
        if (NEED_K) r.k += sg * (d * x - a * E);
        if (NEED_D || NEED_E) r.e += sg * E;
        if (NEED_DV) r.dv += sg * (a * E - d * x);
    }
    r.v *= kInv4Pi;
    r.dd = r.e * kInv4Pi;
    r.dv *= kInv4Pi / alpha;
    return r;
}

// Touching time elements: D-type values with the a-derivatives of Delta F_V,
//   d/da F_V = (E1(a/d) - d e^{-a/d}/a)/(4 pi),  d2/da2 F_V = d e^{-a/d}/(4 pi a^2).
struct TouchH { double dd, va, vaa, v; };
template <bool WV = false>      // WV: also Delta F_V from the same E1 values
SDEV TouchH touch_h(const TimeBlock& tb, double a)
{
    TouchH r = {0, 0, 0, 0};
    double ia = 1.0 / a;
    for (int s = 0; s < tb.ndel; ++s) {
        double d = tb.del[s], z = a * tb.idel[s], sg = tb.sgn[s];
        double ez, E = e1x(z, ez), x = d * ez * ia;
        r.dd += sg * E;
        r.va += sg * (E - x);
        r.vaa += sg * x * ia;
        if (WV) r.v += sg * ((d + a) * E - d * ez);
    }
    r.dd *= kInv4Pi; r.va *= kInv4Pi; r.vaa *= kInv4Pi;
    if (WV) r.v *= kInv4Pi;
    return r;
}

// Touching time elements, split form value = A + B ln r (B exact).
struct Split { double a, b; };
struct SplitVals { Split v, k, dd, dv, e; };

template <bool NEED_V, bool NEED_K, bool NEED_D, bool NEED_DV, bool NEED_E>
SDEV SplitVals touch_split(const TimeBlock& tb, double a, double lnr, double alpha)
{
    const double c0 = -kEuler - log(0.25 * alpha);
    SplitVals r = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
    double ssum = 0.0;                          // sum of signs: 1 (d=0) or -1 (d=1)
    for (int s = 0; s < tb.ndel; ++s) {
        double d = tb.del[s], z = a * tb.idel[s], sg = tb.sgn[s];
        double x, Ez = ez_part(z, c0, tb.lnd[s], lnr, x);
        ssum += sg;
        if (NEED_V) r.v.a += sg * ((d + a) * Ez - d * x);
        if (NEED_K) r.k.a += sg * (d * x - a * Ez);
        if (NEED_D || NEED_E) r.e.a += sg * Ez;
        if (NEED_DV) r.dv.a += sg * (a * Ez - d * x);
    }
    // ln r coefficients: sum_s sg * (-2)(d_s + a) etc., with the exact
    // identity sum_s sg d_s = h_k (d=0) or 0 (d=1)
    double sd = (tb.d == 0) ? tb.del[0] : 0.0;
    r.v.b = -2.0 * (sd + a * ssum) * kInv4Pi;
    r.v.a *= kInv4Pi;
    r.k.b = 2.0 * a * ssum;
    r.e.b = -2.0 * ssum;
    r.dd.a = r.e.a * kInv4Pi; r.dd.b = r.e.b * kInv4Pi;
    r.dv.b = -2.0 * a * ssum * kInv4Pi / alpha;
    r.dv.a *= kInv4Pi / alpha;
    return r;
}

// ------------------------------------------------------------------ pieces
struct Piece { double ax, ay, ex, ey, len, nx, ny; int id, np; };

SDEV Piece seg_piece(const Geom& g, int i)
{
    Piece p;
    p.ax = g.vx[i]; p.ay = g.vy[i]; p.ex = g.ex[i]; p.ey = g.ey[i]; p.len = g.len[i];
    p.nx = p.ey; p.ny = -p.ex; p.id = i; p.np = g.ng;
    return p;
}

SDEV Piece half_piece(const Geom& g, int h)
{
    int i = h >> 1;
    Piece p = seg_piece(g, i);
    p.len = 0.5 * g.len[i];
    if (h & 1) { p.ax += p.len * p.ex; p.ay += p.len * p.ey; }
    p.id = h; p.np = 2 * g.ng;
    return p;
}

// 0 separated, 1 coincident, 2 P ends where Q starts, 3 Q ends where P starts
SDEV int relation(const Piece& P, const Piece& Q)
{
    if (P.id == Q.id) return 1;
    int nxt = P.id + 1 == P.np ? 0 : P.id + 1;
    if (nxt == Q.id) return 2;
    int nq = Q.id + 1 == Q.np ? 0 : Q.id + 1;
    if (nq == P.id) return 3;
    return 0;
}

SDEV double pt_seg_d2(double px, double py, const Piece& S)
{
    double t = (px - S.ax) * S.ex + (py - S.ay) * S.ey;
    t = t < 0.0 ? 0.0 : (t > S.len ? S.len : t);
    double dx = S.ax + t * S.ex - px, dy = S.ay + t * S.ey - py;
    return dx * dx + dy * dy;
}

// distance between two non-intersecting pieces, over the larger length
SDEV double sep_ratio(const Piece& P, const Piece& Q)
{
    double d2 = pt_seg_d2(P.ax, P.ay, Q);
    double t;
    t = pt_seg_d2(P.ax + P.len * P.ex, P.ay + P.len * P.ey, Q); d2 = t < d2 ? t : d2;
    t = pt_seg_d2(Q.ax, Q.ay, P); d2 = t < d2 ? t : d2;
    t = pt_seg_d2(Q.ax + Q.len * Q.ex, Q.ay + Q.len * Q.ey, P); d2 = t < d2 ? t : d2;
    double L = P.len > Q.len ? P.len : Q.len;
    return sqrt(d2) / L;
}

// ------------------------------------------------------- piece-pair rules
// The kernel functor KF accumulates shape-weighted kernel values:
//   KF::val(w, sP, sQ, dx, dy, r2)             w * kernel at (x,y), x-y = (dx,dy)
//   KF::split(wa, wb, sP, sQ, dx, dy, r2, lnr) wa * A + wb * B of the split form
// sP, sQ are arclengths from the piece starts.

template <class KF>
SDEV void rule_regular(const Tables& T, const Piece& P, const Piece& Q, int q, KF& kf)
{
    for (int a = 0; a < q; ++a) {
        double sP = P.len * T.gl_x[q][a], wP = P.len * T.gl_w[q][a];
        double xx = P.ax + sP * P.ex, xy = P.ay + sP * P.ey;
        for (int b = 0; b < q; ++b) {
            double sQ = Q.len * T.gl_x[q][b];
            double dx = xx - (Q.ax + sQ * Q.ex), dy = xy - (Q.ay + sQ * Q.ey);
            kf.val(wP * Q.len * T.gl_w[q][b], sP, sQ, dx, dy, dx * dx + dy * dy);
        }
    }
}

// coincident pieces: eps = |s - s'| = L v; s ranges over [0, L - eps]
template <class KF>
SDEV void rule_coincident(const Tables& T, const Piece& P, int qv, int ql, KF& kf)
{
    const double L = P.len, lnL = log(L);
    const int qs = 2;    // exact for the (at most bilinear) shape products
    for (int pass = 0; pass < 2; ++pass) {
        int n = pass ? ql : qv;
        for (int a = 0; a < n; ++a) {
            double v = pass ? T.lg_x[ql][a] : T.gl_x[qv][a];
            double wv = pass ? T.lg_w[ql][a] : T.gl_w[qv][a];
            double eps = L * v, r2 = eps * eps, lnr = lnL + log(v);
            double span = L - eps;
            for (int b = 0; b < qs; ++b) {
                double s = span * T.gl_x[qs][b];
                double w = L * wv * span * T.gl_w[qs][b];
                double wa = pass ? 0.0 : w, wb = pass ? -w : w * lnL;
                kf.split(wa, wb, s + eps, s, eps * P.ex, eps * P.ey, r2, lnr);
                kf.split(wa, wb, s, s + eps, -eps * P.ex, -eps * P.ey, r2, lnr);
            }
        }
    }
}

// pieces sharing a vertex V: x = V + sp e1, y = V + sq e2 with sp, sq the
// distances from V; Duffy triangles sq <= sp (A) and sp <= sq (B)
template <class KF>
SDEV void rule_vertex(const Tables& T, const Piece& P, const Piece& Q, int rel, int qg, int ql, KF& kf)
{
    const int pend = (rel == 2), qend = (rel == 3);
    const double e1x = pend ? -P.ex : P.ex, e1y = pend ? -P.ey : P.ey;
    const double e2x = qend ? -Q.ex : Q.ex, e2y = qend ? -Q.ey : Q.ey;
    const double LP = P.len, LQ = Q.len;
    for (int tri = 0; tri < 2; ++tri) {
        for (int c = 0; c < qg; ++c) {
            double w = T.gl_x[qg][c], ww = T.gl_w[qg][c];
            // x - y = u * (fx, fy)
            double fx, fy;
            if (tri == 0) { fx = LP * e1x - w * LQ * e2x; fy = LP * e1y - w * LQ * e2y; }
            else          { fx = w * LP * e1x - LQ * e2x; fy = w * LP * e1y - LQ * e2y; }
            double rho2 = fx * fx + fy * fy, lnrho = 0.5 * log(rho2);
            for (int pass = 0; pass < 2; ++pass) {
                int n = pass ? ql : qg;
                for (int a = 0; a < n; ++a) {
                    double u = pass ? T.lg_x[ql][a] : T.gl_x[qg][a];
                    double wu = pass ? T.lg_w[ql][a] : T.gl_w[qg][a];
                    double sp, sq;
                    if (tri == 0) { sp = LP * u; sq = LQ * u * w; }
                    else          { sq = LQ * u; sp = LP * u * w; }
                    double jac = LP * LQ * u * ww * wu;
                    double wa = pass ? 0.0 : jac, wb = pass ? -jac : jac * lnrho;
                    double sP = pend ? LP - sp : sp, sQ = qend ? LQ - sq : sq;
                    kf.split(wa, wb, sP, sQ, u * fx, u * fy, u * u * rho2, log(u) + lnrho);
                }
            }
        }
    }
}

// Order of the regular rule on a pair of pieces of touching time elements.
// Two things limit it: the distance to the r = 0 singularity (classes of
// eta = distance / length), and the factor e^{-z}, z = w2 r^2, which changes
// along one piece by at most dz = w2 L (2 r_lo + L) (L the longer length,
// r_lo the distance of the pieces).  For the second, the q-point Gauss
// remainder of e^{-dz s} on [0, 1] relative to its integral is at most
// c_q dz^{2q} e^{dz}, c_q = (q!)^4 / ((2q+1) ((2q)!)^3); pairs whose factor
// is below e^{-z_floor} (of the block maximum, attained at r = 0) need that
// bound only relative to e^{-z_floor}.
SDEV int q_slope(double zlo, double dz, double q_tol, double z_floor)
{
    const double lim = q_tol * exp(-dz) * (zlo > z_floor ? exp(zlo - z_floor) : 1.0);
    const double dz2 = dz * dz;
    double c = 1.0 / 24.0, pw = dz2;   // c_1, dz^2
    int q = 1;
    while (q < kMaxGL && c * pw > lim) {
        const double a = 2.0 * q + 1.0;
        c *= (double)(q + 1) * (q + 1) * (q + 1) * (q + 1) * a / ((a + 2.0) * (a * (a + 1.0)) * (a * (a + 1.0)) * (a * (a + 1.0)));
        pw *= dz2;
        ++q;
    }
    return q;
}

SDEV int q_touch(const Orders& O, const TimeBlock& tb, const Piece& P, const Piece& Q, double eta, int qinc)
{
    int qe = O.q_near[kNearClasses - 1];
    for (int c = kNearClasses - 2; c >= 0; --c)
        if (eta < O.eta_cut[c]) qe = O.q_near[c];
    const double L = P.len > Q.len ? P.len : Q.len, rlo = eta * L;
    const double zlo = tb.w2 * rlo * rlo, dz = tb.w2 * L * (2.0 * rlo + L);
    int q = q_slope(zlo, dz, O.q_tol, O.z_floor) + qinc;
    q = q < 3 ? 3 : q;
    q = q > qe ? q : qe;
    return q > kMaxGL ? kMaxGL : q;
}

template <class KF>
SDEV void pair_integral(const Tables& T, const Orders& O, const TimeBlock& tb, int q_far, int qinc,
                        const Piece& P, const Piece& Q, KF& kf)
{
    if (tb.d >= 2) { rule_regular(T, P, Q, q_far, kf); return; }
    int rel = relation(P, Q);
    if (rel == 1) { rule_coincident(T, P, O.q_sing, O.q_log, kf); return; }
    if (rel >= 2) { rule_vertex(T, P, Q, rel, O.q_sing, O.q_log, kf); return; }
    rule_regular(T, P, Q, q_touch(O, tb, P, Q, sep_ratio(P, Q), qinc), kf);
}

// ---------------------------------------------------------- kernel functors
// Compensated sum: s + c carries the running sum to about twice the working
// precision (error-free transformation of each addition, Knuth's TwoSum; no
// products, so contraction into FMA cannot change it).
struct CSum {
    double s, c;
    SDEV void add(double x)
    {
        const double t = s + x, bp = t - s;
        c += (s - (t - bp)) + (x - bp);
        s = t;
    }
    SDEV double value() const { return s + c; }
};

// V_h (and dV_h/dalpha): constant shapes, the kernel depends on r only.
template <bool DERIV>
struct KernV {
    const TimeBlock& tb; double alpha; double acc;
    SDEV KernV(const TimeBlock& t, double al) : tb(t), alpha(al), acc(0.0) {}
    SDEV void val(double w, double, double, double, double, double r2)
    {
        double a = 0.25 * alpha * r2;
        if (tb.ser) {
            if (DERIV) acc -= w * series<false, true, false>(tb, a).k * kInv4Pi / alpha;
            else acc += w * series<true, false, false>(tb, a).v;
        } else {
            if (DERIV) acc += w * touch<false, false, false, true, false>(tb, a, alpha).dv;
            else acc += w * touch<true, false, false, false, false>(tb, a, alpha).v;
        }
    }
    SDEV void split(double wa, double wb, double, double, double, double, double r2, double lnr)
    {
        double a = 0.25 * alpha * r2;
        SplitVals s = touch_split<!DERIV, false, false, DERIV, false>(tb, a, lnr, alpha);
        Split x = DERIV ? s.dv : s.v;
        acc += wa * x.a + wb * x.b;
    }
};

// K_h (and dK_h/dalpha): trial shapes (1 - sQ/L, sQ/L) on the trial piece,
// geometric factor (x-y).n_Q / (2 pi r^2) (resp. -(x-y).n_Q/(8 pi)).
template <bool DERIV>
struct KernK {
    const TimeBlock& tb; double alpha; double nqx, nqy, invLQ; double acc0, acc1;
    SDEV KernK(const TimeBlock& t, double al, const Piece& Q)
        : tb(t), alpha(al), nqx(Q.nx), nqy(Q.ny), invLQ(1.0 / Q.len), acc0(0.0), acc1(0.0) {}
    SDEV void add(double v, double sQ)
    {
        double l1 = sQ * invLQ;
        acc0 += v * (1.0 - l1); acc1 += v * l1;
    }
    SDEV void val(double w, double, double sQ, double dx, double dy, double r2)
    {
        double dn = dx * nqx + dy * nqy;
        if (dn == 0.0) return;
        double a = 0.25 * alpha * r2, v;
        if (!DERIV) {
            double fk = tb.ser ? series<false, true, false>(tb, a).k
                                  : touch<false, true, false, false, false>(tb, a, alpha).k;
            v = dn / r2 * kInv2Pi * fk;
        } else {
            double e = tb.ser ? 4.0 * kPi * series<false, false, true>(tb, a).dd
                                 : touch<false, false, false, false, true>(tb, a, alpha).e;
            v = -dn * 0.125 * (1.0 / kPi) * e;
        }
        add(w * v, sQ);
    }
    SDEV void split(double wa, double wb, double, double sQ, double dx, double dy, double r2, double lnr)
    {
        double dn = dx * nqx + dy * nqy;
        if (dn == 0.0) return;
        double a = 0.25 * alpha * r2;
        if (!DERIV) {
            SplitVals s = touch_split<false, true, false, false, false>(tb, a, lnr, alpha);
            add((wa * s.k.a + wb * s.k.b) * dn / r2 * kInv2Pi, sQ);
        } else {
            SplitVals s = touch_split<false, false, false, false, true>(tb, a, lnr, alpha);
            add(-(wa * s.e.a + wb * s.e.b) * dn * 0.125 * (1.0 / kPi), sQ);
        }
    }
};

// D_h on one pair of half-segment pieces: curl part psi'_P psi'_Q Delta F_V
// plus alpha (n_P.n_Q) psi_P(x) psi_Q(y) Delta F_D, psi linear on each piece.
struct KernD {
    const TimeBlock& tb; double alpha;
    double cc;                 // psi'_P psi'_Q
    double cn;                 // alpha n_P . n_Q
    double p0, dp, q0, dq;     // psi_P(sP) = p0 + dp sP, psi_Q(sQ) = q0 + dq sQ
    CSum acc;                  // compensated: see DMomBP
    SDEV KernD(const TimeBlock& t, double al) : tb(t), alpha(al), acc{0.0, 0.0} {}
    int raw;                         // use the raw-kernel form (smooth kernel)
    double tt, txx, txy, tyx, tyy;   // t_P.t_Q and the tangents
    SDEV void val(double w, double sP, double sQ, double dx, double dy, double r2)
    {
        double a = 0.25 * alpha * r2;
        double sh = (p0 + dp * sP) * (q0 + dq * sQ);
        if (raw) {
            // smooth kernel (separated time elements, or pieces far apart): the
            // curl term is integrated back by parts,
            //   int k psi'_P psi'_Q = -int t_P^T Hess(k) t_Q psi_P psi_Q,
            // Hess of F(alpha |z|^2/4) = F'' (alpha/2)^2 z z^T + F' (alpha/2) I,
            // which avoids the cancellation of the second difference
            double dd, va, vaa;
            if (tb.ser) { SeriesVals s = series<false, false, true, true>(tb, a); dd = s.dd; va = s.va; vaa = s.vaa; }
            else { TouchH s = touch_h(tb, a); dd = s.dd; va = s.va; vaa = s.vaa; }
            double zt = (dx * txx + dy * txy) * (dx * tyx + dy * tyy);
            double h = 0.25 * alpha * alpha * vaa * zt + 0.5 * alpha * va * tt;
            acc.add(w * sh * (cn * dd - h));
        } else {
            TouchVals s = touch<true, false, true, false, false>(tb, a, alpha);
            acc.add(w * cc * s.v);
            acc.add(w * cn * sh * s.dd);
        }
    }
    SDEV void split(double wa, double wb, double sP, double sQ, double, double, double r2, double lnr)
    {
        double a = 0.25 * alpha * r2;
        SplitVals s = touch_split<true, false, true, false, false>(tb, a, lnr, alpha);
        double sh = cn * (p0 + dp * sP) * (q0 + dq * sQ);
        acc.add(wa * cc * s.v.a + wb * cc * s.v.b);
        acc.add(wa * sh * s.dd.a + wb * sh * s.dd.b);
    }
};


// Moments of one pair of half-segment pieces on touching time elements, for
// D_h entries assembled from shared piece-pair moments.  x^, y^ in [0, 1] are
// the arclength coordinates on P and Q divided by the lengths; a dual hat is
// a0 (1 - x^) + a1 x^ on each piece of its support.
// By-parts form: m[0] = int int Delta F_V; m[1..4] = alpha n_P.n_Q times the
// moments of Delta F_D against (1-x^)(1-y^), (1-x^) y^, x^ (1-y^), x^ y^.
// For neighbouring dual functions the curl and the normal part of an entry
// nearly cancel (by up to ~5e3 on coarse meshes), so the quadrature sums are
// compensated: plain sums leave their rounding, amplified by that factor, at
// a few 1e-13 of the entry.
struct DMomBP {
    const TimeBlock& tb; double alpha, iLP, iLQ; CSum m[5];
    SDEV DMomBP(const TimeBlock& t, double al, const Piece& P, const Piece& Q)
        : tb(t), alpha(al), iLP(1.0 / P.len), iLQ(1.0 / Q.len), m{{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}} {}
    SDEV void add(double v, double d, double sP, double sQ)
    {
        const double x = sP * iLP, y = sQ * iLQ;
        m[0].add(v);
        m[1].add(d * (1.0 - x) * (1.0 - y)); m[2].add(d * (1.0 - x) * y);
        m[3].add(d * x * (1.0 - y));         m[4].add(d * x * y);
    }
    SDEV void val(double w, double sP, double sQ, double, double, double r2)
    {
        TouchVals s = touch<true, false, true, false, false>(tb, 0.25 * alpha * r2, alpha);
        add(w * s.v, w * s.dd, sP, sQ);
    }
    SDEV void split(double wa, double wb, double sP, double sQ, double, double, double r2, double lnr)
    {
        SplitVals s = touch_split<true, false, true, false, false>(tb, 0.25 * alpha * r2, lnr, alpha);
        add(wa * s.v.a + wb * s.v.b, wa * s.dd.a + wb * s.dd.b, sP, sQ);
    }
};

// Raw-kernel form (pieces apart): moments of alpha n_P.n_Q Delta F_D minus the
// tangential Hessian term t_P^T Hess t_Q of Delta F_V, against the same four
// bilinear shapes.  Only the regular rule is used with it.  WV: m[4] also
// takes int int Delta F_V (V_h's kernel) at the same nodes.
template <bool WV = false>
struct DMomRaw {
    const TimeBlock& tb; double alpha, cn, tt, txx, txy, tyx, tyy, iLP, iLQ; double m[5];
    SDEV DMomRaw(const TimeBlock& t, double al, const Piece& P, const Piece& Q)
        : tb(t), alpha(al), cn(al * (P.nx * Q.nx + P.ny * Q.ny)), tt(P.ex * Q.ex + P.ey * Q.ey),
          txx(P.ex), txy(P.ey), tyx(Q.ex), tyy(Q.ey), iLP(1.0 / P.len), iLQ(1.0 / Q.len), m{0.0, 0.0, 0.0, 0.0, 0.0} {}
    SDEV void val(double w, double sP, double sQ, double dx, double dy, double r2)
    {
        TouchH s = touch_h<WV>(tb, 0.25 * alpha * r2);
        if (WV) m[4] += w * s.v;
        const double zt = (dx * txx + dy * txy) * (dx * tyx + dy * tyy);
        const double h = 0.25 * alpha * alpha * s.vaa * zt + 0.5 * alpha * s.va * tt;
        const double k = w * (cn * s.dd - h);
        const double x = sP * iLP, y = sQ * iLQ;
        m[0] += k * (1.0 - x) * (1.0 - y); m[1] += k * (1.0 - x) * y;
        m[2] += k * x * (1.0 - y);         m[3] += k * x * y;
    }
};

// Moment sets of one piece pair (touching elements), cn folded in.
SDEV void d_pair_bp(const Tables& T, const Orders& O, const TimeBlock& tb, double alpha,
                    const Piece& P, const Piece& Q, double* m)
{
    DMomBP f(tb, alpha, P, Q);
    pair_integral(T, O, tb, 0, 0, P, Q, f);
    const double cn = alpha * (P.nx * Q.nx + P.ny * Q.ny);
    m[0] = f.m[0].value();
    for (int c = 1; c < 5; ++c) m[c] = cn * f.m[c].value();
}

template <bool WV = false>
SDEV void d_pair_raw(const Tables& T, const Orders& O, const TimeBlock& tb, double alpha,
                     const Piece& P, const Piece& Q, double* m, double* vm = nullptr)
{
    DMomRaw<WV> f(tb, alpha, P, Q);
    rule_regular(T, P, Q, q_touch(O, tb, P, Q, sep_ratio(P, Q), 0), f);
    for (int c = 0; c < 4; ++c) m[c] = f.m[c];
    if (WV) *vm = f.m[4];
}

// separation of the supports of two dual hats (pieces P[0..3], Q[0..3]):
// the smallest eta over the 16 pairs, 0 for pairs that touch
SDEV double d_support_eta(const Piece* P, const Piece* Q)
{
    double eta = 1e300;
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) {
            double e = relation(P[u], Q[v]) ? 0.0 : sep_ratio(P[u], Q[v]);
            eta = e < eta ? e : eta;
        }
    return eta;
}

// ------------------------------------------------------- quadrature orders
// Order of the tensor rule for a smooth kernel that varies on the length
// scale sqrt(4 delta_min / alpha) (delta_min: smallest time lag of the
// block), over pieces of length at most lmax.
SDEV int q_time(double lmax, double delta_min, double alpha)
{
    double rt = lmax * sqrt(alpha / (4.0 * delta_min));
    if (rt <= 0.03) return 3;
    if (rt <= 0.15) return 4;
    if (rt <= 0.3) return 5;
    if (rt <= 0.6) return 6;
    if (rt <= 1.2) return 8;
    if (rt <= 2.4) return 10;
    if (rt <= 4.0) return 12;
    return kMaxGL;
}

// Order of the regular rule for operator op on block (k, m): the alpha-
// derivative kernels vanish like r^2 at coincidence and K carries the factor
// (x-y).n/r^2, both need more points than V and D for the same accuracy.
SDEV int q_inc(int op) { return op == OP_K ? 1 : (op == OP_DV || op == OP_DK) ? 2 : 0; }

SDEV int q_block(int op, double lmax, double delta_min, double alpha)
{
    int q = q_time(lmax, delta_min, alpha) + q_inc(op);
    return q > kMaxGL ? kMaxGL : q;
}

// smallest positive lag of the time block (k, m)
SDEV double block_min_lag(const double* t, int k, int m)
{
    if (k == m) return t[k + 1] - t[k];
    if (k == m + 1) { double a = t[k + 1] - t[k], b = t[m + 1] - t[m]; return a < b ? a : b; }
    return t[k] - t[m + 1];
}


// ---------------------------------------------------------------- entries
// psi_i: pieces 2i-1, 2i (rising, slope 1/Lt0) and 2i+1, 2i+2 (falling).
struct DualSupport { int piece[4]; double v0[4], slope[4]; };

SDEV DualSupport dual_support(const Geom& g, int i)
{
    int ng = g.ng, im = i == 0 ? ng - 1 : i - 1, ip = i + 1 == ng ? 0 : i + 1;
    double Lm = g.len[im], Li = g.len[i], Lp = g.len[ip];
    double Lt0 = 0.5 * (Lm + Li), Lt1 = 0.5 * (Li + Lp);
    DualSupport s;
    s.piece[0] = 2 * im + 1; s.v0[0] = 0.0;                  s.slope[0] = 1.0 / Lt0;
    s.piece[1] = 2 * i;      s.v0[1] = 0.5 * Lm / Lt0;       s.slope[1] = 1.0 / Lt0;
    s.piece[2] = 2 * i + 1;  s.v0[2] = 1.0;                  s.slope[2] = -1.0 / Lt1;
    s.piece[3] = 2 * ip;     s.v0[3] = 1.0 - 0.5 * Li / Lt1; s.slope[3] = -1.0 / Lt1;
    return s;
}

template <int OP>
SDEV double entry(const Tables& T, const Orders& O, const Geom& g, const TimeBlock& tb, int q_far,
                  int i, int j)
{
    if (OP == OP_V || OP == OP_DV) {
        Piece P = seg_piece(g, i), Q = seg_piece(g, j);
        KernV<OP == OP_DV> kf(tb, g.alpha);
        pair_integral(T, O, tb, q_far, q_inc(OP), P, Q, kf);
        return kf.acc;
    } else if (OP == OP_K || OP == OP_DK) {
        // hat_j: rising on segment j-1 (shape sQ/L), falling on segment j
        int jm = j == 0 ? g.ng - 1 : j - 1;
        Piece P = seg_piece(g, i), Q1 = seg_piece(g, jm), Q2 = seg_piece(g, j);
        KernK<OP == OP_DK> k1(tb, g.alpha, Q1), k2(tb, g.alpha, Q2);
        if (relation(P, Q1) != 1) pair_integral(T, O, tb, q_far, q_inc(OP), P, Q1, k1);   // coincident: (x-y).n = 0
        if (relation(P, Q2) != 1) pair_integral(T, O, tb, q_far, q_inc(OP), P, Q2, k2);
        return k1.acc1 + k2.acc0;
    } else {
        DualSupport si = dual_support(g, i), sj = dual_support(g, j);
        // the raw-kernel form needs a smooth kernel on the whole supports
        // (boundary terms of the integration by parts cancel only in the sum)
        int raw = tb.ser;
        if (!raw) {
            double eta = 1e300;
            for (int u = 0; u < 4 && eta > 0.0; ++u) {
                Piece P = half_piece(g, si.piece[u]);
                for (int v = 0; v < 4; ++v) {
                    Piece Q = half_piece(g, sj.piece[v]);
                    double e = relation(P, Q) ? 0.0 : sep_ratio(P, Q);
                    eta = e < eta ? e : eta;
                }
            }
            raw = eta > O.eta_raw;
        }
        CSum acc = {0.0, 0.0};
        for (int u = 0; u < 4; ++u) {
            Piece P = half_piece(g, si.piece[u]);
            for (int v = 0; v < 4; ++v) {
                Piece Q = half_piece(g, sj.piece[v]);
                KernD kf(tb, g.alpha);
                kf.cc = si.slope[u] * sj.slope[v];
                kf.cn = g.alpha * (P.nx * Q.nx + P.ny * Q.ny);
                kf.p0 = si.v0[u]; kf.dp = si.slope[u];
                kf.q0 = sj.v0[v]; kf.dq = sj.slope[v];
                kf.txx = P.ex; kf.txy = P.ey; kf.tyx = Q.ex; kf.tyy = Q.ey;
                kf.tt = P.ex * Q.ex + P.ey * Q.ey;
                kf.raw = raw;
                pair_integral(T, O, tb, q_far, q_inc(OP), P, Q, kf);
                acc.add(kf.acc.s);
                acc.add(kf.acc.c);
            }
        }
        return acc.value();
    }
}

}  // namespace stbem
