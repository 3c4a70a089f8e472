// Initial potential M_h^0 of eq.(4) (arXiv:1811.05224, Sec. 1):
//   M0[(k,i), j] = int_{gamma_i} int_Omega phi_j(y) G_k(|x - y|) dy ds_x,
//   G_k(r) = int_{tau_k} U*(r, t) dt = alpha/(4 pi) [E1(a/t_{k+1}) - E1(a/t_k)],
// a = alpha r^2 / 4, E1(a/0) = 0.  phi_j is the P1 hat of vertex j of Omega_h.
// The alpha-derivative is (1/(4 pi)) [E1 - E1 - e^{-a/t_{k+1}} + e^{-a/t_k}].
//
// For k >= 1, G_k is smooth (its ln r parts cancel): tensor Gauss on the
// segment times a collapsed Gauss rule on the triangle.  For k = 0 it has the
// singularity -(alpha/2pi) ln r; near the segment the kernel is split as
// S(r^2) - (alpha/2pi) ln r (S smooth), the S part uses the tensor rule and
// the ln part uses the closed-form logarithmic potential of a linear density
// on the triangle, integrated along the segment by a tanh-sinh rule on the
// pieces between the projections of the triangle vertices.
#pragma once
#include "stbem_math.h"

namespace stbem {

constexpr int kMaxDE = 64;

struct M0Tables {
    int nde;
    double de_x[kMaxDE], de_w[kMaxDE];     // tanh-sinh on [0,1]
};

struct Mesh2 {
    int nv, ntri;
    const double *ox, *oy;                 // Omega vertices
    const int* tri;                        // 3 * ntri, CCW
    const int *v2t_ptr, *v2t;              // vertex -> triangles
};

// For k >= 1, with z = a/t, E1(a/t_{k+1}) - E1(a/t_k) = ln(t_{k+1}/t_k)
// + Ein(a/t_{k+1}) - Ein(a/t_k) is a power series in a; when a/t_k stays
// <= 4 (a <= amax[k]) it is evaluated from precomputed coefficients
// (row-wise table, Horner); farther pairs use E1 directly.  DERIV adds -(e^{-a/t_{k+1}} - e^{-a/t_k}).
constexpr int kPolyMax = 40;
// Per time element k >= 1: coefficients of the series in a (c[k][0] = cd[k][0]
// = ln(t_{k+1}/t_k)), their count, the range a <= amax[k]; it[k] = 1/t_k.
// ce, cde: the same polynomials economised on [0, amax[k]] (Chebyshev
// truncation, written in powers of y = a es[k] - 1, es[k] = 2/amax[k]),
// evaluated per pair; c, cd stay for the moment form of the late rows.
constexpr int kEconMax = 24;
struct M0Poly {
    const double* c; const double* cd; const int* n; const double* amax; const double* it;   // [nt][kPolyMax], [nt], [nt], [nt+1]
    const double* ce; const double* cde; const double* es;                                  // [nt][kEconMax], [nt]
};

// G_k (or its alpha-derivative) at r^2
template <bool DERIV>
SDEV double m0_kernel(const Geom& g, const M0Poly& PP, int k, double r2)
{
    double a = 0.25 * g.alpha * r2;
    double z1 = a * PP.it[k + 1];
    double x1, x0;
    if (k == 0) {
        double E = e1t<DERIV>(z1, x1);
        return DERIV ? (E - x1) * kInv4Pi : g.alpha * kInv4Pi * E;
    }
    double z0 = a * PP.it[k], dE;
    if (z0 <= 2.0) {
        dE = PP.c[(long long)k * kPolyMax] + ein(z1) - ein(z0);    // ln(t1/t0): no ln a cancellation
        if (DERIV) { x1 = exp(-z1); x0 = exp(-z0); }
    } else {
        dE = e1t<DERIV>(z1, x1) - e1t<DERIV>(z0, x0);
    }
    if (DERIV) return (dE - x1 + x0) * kInv4Pi;
    return g.alpha * kInv4Pi * dE;
}

// smooth part S of G_0 = S - B ln r with B = alpha/(2 pi) (resp. 1/(2 pi))
template <bool DERIV>
SDEV double m0_smooth0(const Geom& g, double r2, double lnr)
{
    double a = 0.25 * g.alpha * r2, t1 = g.t[1], z = a / t1;
    double Ez, ex = 0.0;   // Ez = E1(z) + 2 ln r
    if (z <= 2.0) {
        Ez = -kEuler - log(0.25 * g.alpha / t1) + ein(z);
        if (DERIV) ex = exp(-z);
    } else {
        Ez = e1t<DERIV>(z, ex) + 2.0 * lnr;
    }
    return DERIV ? (Ez - ex) * kInv4Pi : g.alpha * kInv4Pi * Ez;
}

struct Tri { double ax, ay, bx, by, cx, cy; };   // vertices only (distance tests)

// u ln(u^2 + d^2) - 2u + 2 d atan(u/d), and (1/2)[(u^2+d^2) ln(u^2+d^2) - u^2]
SDEV double logU(double u, double d)
{
    double q = u * u + d * d;
    double l = q > 0.0 ? u * log(q) : 0.0;
    return l - 2.0 * u + (d > 0.0 ? 2.0 * d * atan(u / d) : 0.0);
}
SDEV double logW(double u, double d)
{
    double q = u * u + d * d;
    return 0.5 * ((q > 0.0 ? q * log(q) : 0.0) - u * u);
}

SDEV double seg_tri_dist(const Piece& S, const Tri& tr)
{
    // distance between the segment and the triangle's vertices/edges
    const double vx[3] = {tr.ax, tr.bx, tr.cx}, vy[3] = {tr.ay, tr.by, tr.cy};
    double d2 = 1e300;
    for (int e = 0; e < 3; ++e) {
        d2 = fmin(d2, pt_seg_d2(vx[e], vy[e], S));
        int f = e == 2 ? 0 : e + 1;
        Piece Ed;
        Ed.ax = vx[e]; Ed.ay = vy[e];
        double ex = vx[f] - vx[e], ey = vy[f] - vy[e], L = sqrt(ex * ex + ey * ey);
        Ed.ex = ex / L; Ed.ey = ey / L; Ed.len = L;
        d2 = fmin(d2, pt_seg_d2(S.ax, S.ay, Ed));
        d2 = fmin(d2, pt_seg_d2(S.ax + S.len * S.ex, S.ay + S.len * S.ey, Ed));
    }
    return sqrt(d2);
}

struct M0Orders { int qs_near, qt_near; double near_ratio, omax, q_tol, z_floor; };

// The economised row polynomial at y: Horner in y^8 over chunks of eight
// coefficients, each chunk summed against the powers y^0 .. y^7 with the
// coefficient as a factor of one FMA, so that the coefficients (the same for
// all lanes) are used straight from their scalar loads.  Padding zeros at
// the top leave the value unchanged.
static_assert(kEconMax % 8 == 0, "economised rows come in chunks of eight");
SDEV double m0_econ(const double* p, double y)
{
    const double y2 = y * y, y3 = y2 * y, y4 = y2 * y2, y5 = y4 * y, y6 = y4 * y2, y7 = y4 * y3, y8 = y4 * y4;
    double s = 0.0;
#pragma unroll
    for (int k = kEconMax / 8 - 1; k >= 0; --k) {
        const double* c = p + 8 * k;
        double t = c[7] * y7;
        t = fma(c[6], y6, t); t = fma(c[5], y5, t); t = fma(c[4], y4, t);
        t = fma(c[3], y3, t); t = fma(c[2], y2, t); t = fma(c[1], y, t);
        s = fma(s, y8, t + c[0]);
    }
    return s;
}

// ------------------------------------------------ per-triangle moments
// All three barycentric hats of a triangle from one set of kernel values.
struct Tri3 {
    double ax, ay, bx, by, cx, cy;
    double g0[3], gx[3], gy[3];      // hat of local vertex v: g0 + gx x + gy y
};

SDEV Tri3 load_tri3(const Mesh2& m, int t)
{
    Tri3 T;
    int v0 = m.tri[3 * t], v1 = m.tri[3 * t + 1], v2 = m.tri[3 * t + 2];
    T.ax = m.ox[v0]; T.ay = m.oy[v0]; T.bx = m.ox[v1]; T.by = m.oy[v1]; T.cx = m.ox[v2]; T.cy = m.oy[v2];
    const double vx[3] = {T.ax, T.bx, T.cx}, vy[3] = {T.ay, T.by, T.cy};
    double det = (T.bx - T.ax) * (T.cy - T.ay) - (T.by - T.ay) * (T.cx - T.ax);
    for (int v = 0; v < 3; ++v) {
        double px = vx[(v + 1) % 3], py = vy[(v + 1) % 3], qx = vx[(v + 2) % 3], qy = vy[(v + 2) % 3];
        T.gx[v] = -(qy - py) / det;
        T.gy[v] = (qx - px) / det;
        T.g0[v] = ((qx - px) * (-py) - (qy - py) * (-px)) / det;
    }
    return T;
}

// qs Gauss points on the segment x qt x qt collapsed Gauss on the triangle;
// in collapsed coordinates y = A + u (B - A) + v (C - A) the hats are
// (1 - u - v, u, v)
template <class F>
SDEV void m0_regular3(const Tables& T, const Piece& S, const Tri3& tr, int qs, int qt, F f, double* out)
{
    double e1x = tr.bx - tr.ax, e1y = tr.by - tr.ay, e2x = tr.cx - tr.ax, e2y = tr.cy - tr.ay;
    double area2 = fabs(e1x * e2y - e1y * e2x);
    double o0 = 0.0, o1 = 0.0, o2 = 0.0;
    for (int a = 0; a < qt; ++a) {
        double u = T.gl_x[qt][a], wu = T.gl_w[qt][a] * (1.0 - u);
        for (int b = 0; b < qt; ++b) {
            double v = T.gl_x[qt][b] * (1.0 - u), w = wu * T.gl_w[qt][b] * area2;
            double yx = tr.ax + u * e1x + v * e2x, yy = tr.ay + u * e1y + v * e2y;
            double inner = 0.0;
            for (int c = 0; c < qs; ++c) {
                double s = S.len * T.gl_x[qs][c];
                double dx = S.ax + s * S.ex - yx, dy = S.ay + s * S.ey - yy;
                inner += T.gl_w[qs][c] * f(dx * dx + dy * dy);
            }
            inner *= w;
            o0 += (1.0 - u - v) * inner; o1 += u * inner; o2 += v * inner;
        }
    }
    out[0] = o0 * S.len; out[1] = o1 * S.len; out[2] = o2 * S.len;
}

// int_omega hat_v(y) ln|x - y| dy, v = 0, 1, 2, in closed form
SDEV void log_potential3(const Tri3& tr, double x, double y, double* out)
{
    const double vx[3] = {tr.ax, tr.bx, tr.cx}, vy[3] = {tr.ay, tr.by, tr.cy};
    double phx[3];
    for (int v = 0; v < 3; ++v) { phx[v] = tr.g0[v] + tr.gx[v] * x + tr.gy[v] * y; out[v] = 0.0; }
    for (int e = 0; e < 3; ++e) {
        int f = e == 2 ? 0 : e + 1;
        double Px = vx[e] - x, Py = vy[e] - y, Ex = vx[f] - vx[e], Ey = vy[f] - vy[e];
        double J = Px * Ey - Py * Ex;
        double E2 = Ex * Ex + Ey * Ey;
        if (fabs(J) <= 1e-14 * E2) continue;
        double tau0 = -(Px * Ex + Py * Ey) / E2;
        double del = fabs(J) / E2;
        double dU = logU(1.0 - tau0, del) - logU(-tau0, del);
        double dW = logW(1.0 - tau0, del) - logW(-tau0, del);
        double lE = log(E2);
        double I0 = 0.5 * lE + 0.5 * dU;
        double I1 = 0.25 * lE + 0.5 * (dW + tau0 * dU);
        for (int v = 0; v < 3; ++v) {
            double g0 = tr.gx[v] * Px + tr.gy[v] * Py, g1 = tr.gx[v] * Ex + tr.gy[v] * Ey;
            out[v] += J * (-0.25 * phx[v] - (g0 + 0.5 * g1) / 9.0 + (0.5 * phx[v] + g0 / 3.0) * I0 + g1 * I1 / 3.0);
        }
    }
}

SDEV void seg_log_potential3(const M0Tables& D, const Piece& S, const Tri3& tr, double* out)
{
    double cuts[5];
    int nc = 0;
    cuts[nc++] = 0.0;
    const double vx[3] = {tr.ax, tr.bx, tr.cx}, vy[3] = {tr.ay, tr.by, tr.cy};
    for (int v = 0; v < 3; ++v) {
        double s = (vx[v] - S.ax) * S.ex + (vy[v] - S.ay) * S.ey;
        if (s > 1e-12 * S.len && s < S.len * (1.0 - 1e-12)) cuts[nc++] = s;
    }
    cuts[nc++] = S.len;
    for (int a = 1; a < nc; ++a)
        for (int b = a; b > 0 && cuts[b] < cuts[b - 1]; --b) { double t = cuts[b]; cuts[b] = cuts[b - 1]; cuts[b - 1] = t; }
    out[0] = out[1] = out[2] = 0.0;
    for (int p = 0; p + 1 < nc; ++p) {
        double s0 = cuts[p], h = cuts[p + 1] - cuts[p];
        if (h <= 0.0) continue;
        double part[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < D.nde; ++q) {
            double s = s0 + h * D.de_x[q], lp[3];
            log_potential3(tr, S.ax + s * S.ex, S.ay + s * S.ey, lp);
            for (int v = 0; v < 3; ++v) part[v] += D.de_w[q] * lp[v];
        }
        for (int v = 0; v < 3; ++v) out[v] += h * part[v];
    }
}

// the three moments int_{gamma_i} int_omega hat_v G_k ds dy of triangle t;
// FIRST: rows of the first time element (k = 0, singular kernel), else k >= 1
// Rows k0 .. k0+nr-1 (k0 >= 1, nr <= kM0Group) of one segment against one
// triangle with one rule (qs on the segment, qs x qs collapsed on the
// triangle), the rows evaluated together at every node: consecutive rows
// share their time boundary t_k, so each E1 (or Ein) value at a node is
// computed once instead of twice; rows inside their power-series range take
// the series.  Row r's three moments go to out[3r .. 3r+2].  Every row gets
// the same operations, in the same order, as with the per-row kernel.
constexpr int kM0Group = 2;     // of 2, 3, 4 and 8 rows, 2 was fastest (no VGPR spills)

// Ein out of line for the rows' rare small-argument branch (see e1t_large)
__host__ __device__ __attribute__((noinline)) inline double ein_cold(double z) { return ein(z); }

template <bool DERIV>
SDEV void m0_row_values(const Geom& g, const M0Poly& PP, int k0, int nr, double r2, double* val)
{
    const double a = 0.25 * g.alpha * r2, sc = (DERIV ? 1.0 : g.alpha) * kInv4Pi;
    double Eprev = 0.0, einprev = 0.0, xprev = 0.0;
    int have = 0;                              // 1: E1 at t_k known, 2: Ein at t_k known
#pragma unroll
    for (int r = 0; r < kM0Group; ++r) {
        if (r >= nr) continue;
        const int k = k0 + r;
        if (PP.n[k] > 0 && a <= PP.amax[k]) {
            val[r] = sc * m0_econ((DERIV ? PP.cde : PP.ce) + (long long)k * kEconMax, fma(a, PP.es[k], -1.0));
            have = 0;
            continue;
        }
        const double z1 = a * PP.it[k + 1], z0 = a * PP.it[k];
        double dE, x1 = 0.0, x0 = 0.0;
        if (z0 <= 2.0) {
            const double e0 = have == 2 ? einprev : ein_cold(z0);
            const double e1v = ein_cold(z1);
            dE = PP.c[(long long)k * kPolyMax] + e1v - e0;    // ln(t1/t0): no ln a cancellation
            if (DERIV) { x1 = exp(-z1); x0 = have == 2 ? xprev : exp(-z0); }
            einprev = e1v; xprev = x1; have = 2;
        } else {
            double E0;
            if (have == 1) { E0 = Eprev; x0 = xprev; }
            else E0 = e1t_large<DERIV>(z0, x0);
            const double E1v = e1t_large<DERIV>(z1, x1);
            dE = E1v - E0;
            Eprev = E1v; xprev = x1; have = 1;
        }
        val[r] = DERIV ? (dE - x1 + x0) * kInv4Pi : g.alpha * kInv4Pi * dE;
    }
}

template <bool DERIV>
SDEV void m0_rows_moments(const Tables& T, const Geom& g, const M0Poly& PP, const Piece& S, const Tri3& tr,
                          int k0, int nr, int qs, double* out)
{
    const double e1x = tr.bx - tr.ax, e1y = tr.by - tr.ay, e2x = tr.cx - tr.ax, e2y = tr.cy - tr.ay;
    const double area2 = fabs(e1x * e2y - e1y * e2x);
    double o[kM0Group][3];
#pragma unroll
    for (int r = 0; r < kM0Group; ++r) o[r][0] = o[r][1] = o[r][2] = 0.0;
    for (int a = 0; a < qs; ++a) {
        const double u = T.gl_x[qs][a], wu = T.gl_w[qs][a] * (1.0 - u);
        for (int b = 0; b < qs; ++b) {
            const double v = T.gl_x[qs][b] * (1.0 - u), w = wu * T.gl_w[qs][b] * area2;
            const double yx = tr.ax + u * e1x + v * e2x, yy = tr.ay + u * e1y + v * e2y;
            double inner[kM0Group];
#pragma unroll
            for (int r = 0; r < kM0Group; ++r) inner[r] = 0.0;
            for (int c = 0; c < qs; ++c) {
                const double s = S.len * T.gl_x[qs][c];
                const double dx = S.ax + s * S.ex - yx, dy = S.ay + s * S.ey - yy;
                double val[kM0Group];
                m0_row_values<DERIV>(g, PP, k0, nr, dx * dx + dy * dy, val);
#pragma unroll
                for (int r = 0; r < kM0Group; ++r)
                    if (r < nr) inner[r] += T.gl_w[qs][c] * val[r];
            }
#pragma unroll
            for (int r = 0; r < kM0Group; ++r) {
                if (r >= nr) continue;
                const double in = inner[r] * w;
                o[r][0] += (1.0 - u - v) * in; o[r][1] += u * in; o[r][2] += v * in;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kM0Group; ++r) {
        if (r >= nr) continue;
        out[3 * r] = o[r][0] * S.len; out[3 * r + 1] = o[r][1] * S.len; out[3 * r + 2] = o[r][2] * S.len;
    }
}

// First time element: the Gauss order of the regular rule for segment S and
// triangle tr (0: the pair is near, eta < near_ratio, and takes the rule with
// the logarithm split off).  The ln r singularity sits at distance eta * size;
// the factor e^{-z}, z = alpha r^2 / (4 t_1), changes by dz along the elements.
SDEV int m0_first_order(const M0Orders& MO, const Geom& g, const Piece& S, const Tri3& tr, int qs)
{
    Tri tt;
    tt.ax = tr.ax; tt.ay = tr.ay; tt.bx = tr.bx; tt.by = tr.by; tt.cx = tr.cx; tt.cy = tr.cy;
    const double dx1 = tr.bx - tr.ax, dy1 = tr.by - tr.ay, dx2 = tr.cx - tr.ax, dy2 = tr.cy - tr.ay;
    const double diam = sqrt(fmax(fmax(dx1 * dx1 + dy1 * dy1, dx2 * dx2 + dy2 * dy2),
                                  (dx2 - dx1) * (dx2 - dx1) + (dy2 - dy1) * (dy2 - dy1)));
    const double size = fmax(diam, S.len);
    const double eta = seg_tri_dist(S, tt) / size;
    if (eta < MO.near_ratio) return 0;
    const int qn = eta < 1.0 ? kMaxGL : eta < 2.0 ? 12 : eta < 4.0 ? 8 : eta < 8.0 ? 6 : eta < 16.0 ? 5 : 4;
    const double w2 = 0.25 * g.alpha / g.t[1], rlo = eta * size;
    const int qz = q_slope(w2 * rlo * rlo, w2 * size * (2.0 * rlo + size), MO.q_tol, MO.z_floor);
    int q0 = qn > qz ? qn : qz;
    return q0 > qs ? q0 : qs;
}

// PART (first time element only): 0 every pair, 1 the pairs with the
// regular rule, 2 the near pairs; a launch for one kind leaves the other
// kind's code out, which keeps the registers of the regular kind low
template <bool DERIV, bool FIRST, int PART = 0>
SDEV void m0_tri_moments(const Tables& T, const M0Tables& D, const M0Orders& MO, const Geom& g,
                         const Mesh2& m, const M0Poly& PP, int k, int i, int t, int qs, double* out)
{
    Piece S = seg_piece(g, i);
    Tri3 tr = load_tri3(m, t);
    if (FIRST) {
        const int q0 = m0_first_order(MO, g, S, tr, qs);
        if (q0 == 0 && PART != 1) {
            double sm[3], lg[3];
            m0_regular3(T, S, tr, MO.qs_near, MO.qt_near, [&](double r2) { return m0_smooth0<DERIV>(g, r2, 0.5 * log(r2)); }, sm);
            seg_log_potential3(D, S, tr, lg);
            double B = DERIV ? kInv2Pi : g.alpha * kInv2Pi;
            for (int v = 0; v < 3; ++v) out[v] = sm[v] - B * lg[v];
            return;
        }
        if (PART != 2 && q0 > 0) m0_regular3(T, S, tr, q0, q0, [&](double r2) { return m0_kernel<DERIV>(g, PP, 0, r2); }, out);
        return;
    }
    const int n = PP.n[k];
    if (n > 0) {
        const double* c = (DERIV ? PP.cde : PP.ce) + (long long)k * kEconMax;
        const double amax = PP.amax[k], es = PP.es[k], q4 = 0.25 * g.alpha, sc = (DERIV ? 1.0 : g.alpha) * kInv4Pi;
        m0_regular3(T, S, tr, qs, qs, [&](double r2) {
            double a = q4 * r2;
            return a <= amax ? sc * m0_econ(c, fma(a, es, -1.0)) : m0_kernel<DERIV>(g, PP, k, r2);
        }, out);
        return;
    }
    m0_regular3(T, S, tr, qs, qs, [&](double r2) { return m0_kernel<DERIV>(g, PP, k, r2); }, out);
}

// ------------------------------------------------ representation formula
// Potentials of eq. (2) at a point (x, t) of Q.  In the lag s = t - tau,
// s in [s_lo, s_hi] for a time element, with a = alpha r^2 / 4:
//   single layer  int k ds    = [E1(a/s_hi) - E1(a/s_lo)] / (4 pi)
//   double layer  int d_ny k ds = (x-y).n_y / (2 pi r^2) [e^{-a/s_hi} - e^{-a/s_lo}]
// (E1(a/0) = 0, e^{-a/0} = 0).  The differences are formed without
// cancellation: ln(s_hi/s_lo) + Ein(a/s_hi) - Ein(a/s_lo) while a/s_lo <= 2,
// and e^{-a/s_hi} (-expm1(-a (1/s_lo - 1/s_hi))) for the exponentials.
struct PotSeg { double sl, d0, d1; };   // single layer; double layer against the two hats

SDEV void pot_kernels(double alpha, double r2, double dn, double slo, double shi, double& sl, double& dl)
{
    const double a = 0.25 * alpha * r2, zh = a / shi;
    double eh;
    if (slo <= 0.0) {
        sl = e1x(zh, eh) * kInv4Pi;
        dl = dn / (2.0 * kPi * r2) * eh;
        return;
    }
    const double zl = a / slo;
    if (zl <= 2.0) sl = (log(shi / slo) + ein(zh) - ein(zl)) * kInv4Pi;
    else {
        double el;
        sl = (e1x(zh, eh) - e1x(zl, el)) * kInv4Pi;
    }
    eh = exp(-zh);
    dl = dn / (2.0 * kPi * r2) * eh * (-expm1(-a * (1.0 / slo - 1.0 / shi)));
}

// Integrals over segment j for a point at distance d > 0 from it: the
// segment is cut at the foot of the point into pieces whose lengths double
// away from it (distance / length >= 1/2 on every piece), each with a Gauss
// rule of the order the distance class and the slope of e^{-z} ask for.
SDEV PotSeg pot_segment(const Tables& T, const Orders& O, const Geom& g, int j, double x, double y,
                        double slo, double shi)
{
    PotSeg r = {0.0, 0.0, 0.0};
    const double ax = g.vx[j], ay = g.vy[j], ex = g.ex[j], ey = g.ey[j], L = g.len[j];
    // the point in the segment's frame: x - a = pt e + pn n (n = (ey, -ex));
    // at a node y = a + s e, x - y = (pt - s) e + pn n with pt - s formed
    // from the offset to the foot, so r^2 and (x - y).n keep their relative
    // accuracy however close the point is to the segment
    const double px = x - ax, py = y - ay;
    const double pt = px * ex + py * ey, pn = px * ey - py * ex;
    const double sf = pt < 0.0 ? 0.0 : (pt > L ? L : pt);
    const double dt0 = pt - sf;                          // 0 when the foot is inside
    const double d = sqrt(dt0 * dt0 + pn * pn);
    const double w2 = 0.25 * g.alpha / (slo > 0.0 ? slo : shi);
    for (int side = 0; side < 2; ++side) {
        const double span = side ? L - sf : sf;          // from the foot towards one end
        double s0 = 0.0, len = d > 1e-12 * L ? d : 1e-12 * L;
        for (int piece = 0; piece < 64 && s0 < span; ++piece) {
            double s1 = s0 + len;
            s1 = s1 > span ? span : s1;
            const double h = s1 - s0;
            // distance of the piece from the point, and its class
            const double dist = sqrt(d * d + s0 * s0), eta = dist / h;
            int q = O.q_near[kNearClasses - 1];
            for (int c = kNearClasses - 2; c >= 0; --c)
                if (eta < O.eta_cut[c]) q = O.q_near[c];
            int qz = q_slope(w2 * dist * dist, w2 * h * (2.0 * dist + h), O.q_tol, O.z_floor);
            q = q > qz ? q : qz;
            q = q > kMaxGL ? kMaxGL : q;
            for (int a = 0; a < q; ++a) {
                const double u = s0 + h * T.gl_x[q][a], wq = h * T.gl_w[q][a];
                const double s = side ? sf + u : sf - u;     // arclength on the segment
                const double dt = side ? dt0 - u : dt0 + u;   // (x - y).e
                const double r2 = dt * dt + pn * pn;
                double sl, dl;
                pot_kernels(g.alpha, r2, pn, slo, shi, sl, dl);
                const double l1 = s / L;
                r.sl += wq * sl;
                r.d0 += wq * dl * (1.0 - l1);
                r.d1 += wq * dl * l1;
            }
            s0 = s1;
            len *= 2.0;
        }
    }
    return r;
}

// Gauss-Legendre order for e^{-beta |x - y|^2} on a piece of size h at
// distance >= dlo: the 2q-th derivative of a Gaussian of width beta^{-1/2}
// grows like (2q)!/q! beta^q, so the remainder of the q-point rule is about
// c_q (2q)!/q! (beta h^2)^q e^{dz} (c_q the Gauss remainder constant on
// [0, 1]); the slope bound of q_slope covers pieces far on the tail.
SDEV int q_gauss(double bh2, double zlo, double dz, double q_tol, double z_floor)
{
    const double lim = q_tol * exp(-dz) * (zlo > z_floor ? exp(zlo - z_floor) : 1.0);
    double c = 1.0 / 24.0, gf = 2.0, pw = bh2;   // c_1, 2!/1!, (beta h^2)^1
    int q = 1;
    while (q < kMaxGL && c * gf * pw > lim) {
        const double a = 2.0 * q + 1.0;
        c *= (double)(q + 1) * (q + 1) * (q + 1) * (q + 1) * a / ((a + 2.0) * (a * (a + 1.0)) * (a * (a + 1.0)) * (a * (a + 1.0)));
        gf *= 2.0 * a;
        pw *= bh2;
        ++q;
    }
    const int qs = q_slope(zlo, dz, q_tol, z_floor);
    return q > qs ? q : qs;
}

// int_t U*(x - y, t) phi_v(y) dy for the three hats of triangle t: U* is a
// Gaussian of width sqrt(4t/alpha); the triangle is refined regularly into
// n^2 congruent triangles (n a power of two, at most 32) so that the change
// of e^{-z} across one of them stays moderate, and each gets the collapsed
// Gauss rule of the order the slope bound asks for (one more for the
// collapsed direction).  Triangles whose distance makes the Gaussian below
// e^{-60} of its peak contribute nothing.
SDEV void pot_triangle(const Tables& T, const Orders& O, const Geom& g, const Mesh2& m, int tri, double x, double y,
                       double t, double* mom)
{
    mom[0] = mom[1] = mom[2] = 0.0;
    const Tri3 tr = load_tri3(m, tri);
    const double P[3][2] = {{tr.ax, tr.ay}, {tr.bx, tr.by}, {tr.cx, tr.cy}};
    // distance from the point to the triangle (0 inside)
    double d2 = 1e300, diam2 = 0.0;
    int sgn = 0;
    for (int e = 0; e < 3; ++e) {
        const double* A = P[e];
        const double* B = P[e == 2 ? 0 : e + 1];
        const double ex = B[0] - A[0], ey = B[1] - A[1], l2 = ex * ex + ey * ey;
        double u = ((x - A[0]) * ex + (y - A[1]) * ey) / l2;
        u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
        const double dx = x - A[0] - u * ex, dy = y - A[1] - u * ey;
        d2 = fmin(d2, dx * dx + dy * dy);
        diam2 = fmax(diam2, l2);
        sgn += (ex * (y - A[1]) - ey * (x - A[0])) >= 0.0 ? 1 : -1;
    }
    if (sgn == 3 || sgn == -3) d2 = 0.0;
    const double w2 = 0.25 * g.alpha / t, size = sqrt(diam2), d = sqrt(d2);
    if (w2 * d2 > 60.0) return;
    int n = 1;
    while (n < 32 && w2 * (size / n) * (2.0 * d + size / n) > 2.0) n *= 2;
    const double c0 = g.alpha / (4.0 * kPi * t);
    const double ux = (tr.bx - tr.ax) / n, uy = (tr.by - tr.ay) / n, vx = (tr.cx - tr.ax) / n, vy = (tr.cy - tr.ay) / n;
    const double area2 = fabs(ux * vy - uy * vx);
    for (int i = 0; i < n; ++i)
        for (int j = 0; i + j < n; ++j)
            for (int down = 0; down < 2; ++down) {
                if (down && i + j > n - 2) continue;
                // corners of the sub-triangle
                double A0 = tr.ax + i * ux + j * vx, A1 = tr.ay + i * uy + j * vy;
                double B0, B1, C0, C1;
                if (!down) { B0 = A0 + ux; B1 = A1 + uy; C0 = A0 + vx; C1 = A1 + vy; }
                else { B0 = A0 + ux + vx; B1 = A1 + uy + vy; C0 = A0 + vx; C1 = A1 + vy; A0 += ux; A1 += uy; }
                const double cxm = (A0 + B0 + C0) / 3.0 - x, cym = (A1 + B1 + C1) / 3.0 - y;
                const double hs = size / n, dc = fmax(0.0, sqrt(cxm * cxm + cym * cym) - hs);
                if (w2 * dc * dc > 60.0) continue;
                int q = q_gauss(w2 * hs * hs, w2 * dc * dc, w2 * hs * (2.0 * dc + hs), O.q_tol, O.z_floor) + 1;
                q = q < 3 ? 3 : (q > kMaxGL ? kMaxGL : q);
                const double e1x_ = B0 - A0, e1y_ = B1 - A1, e2x = C0 - B0, e2y = C1 - B1;
                for (int a = 0; a < q; ++a) {
                    const double u = T.gl_x[q][a], wu = T.gl_w[q][a] * u * area2;
                    for (int b = 0; b < q; ++b) {
                        const double v = T.gl_x[q][b], w = wu * T.gl_w[q][b];
                        const double yx = A0 + u * e1x_ + u * v * e2x, yy = A1 + u * e1y_ + u * v * e2y;
                        const double dx = x - yx, dy = y - yy;
                        const double k = w * c0 * exp(-w2 * (dx * dx + dy * dy));
                        for (int c = 0; c < 3; ++c) mom[c] += k * (tr.g0[c] + tr.gx[c] * yx + tr.gy[c] * yy);
                    }
                }
            }
}

}  // namespace stbem
