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

// G_k (or its alpha-derivative) at r^2
template <bool DERIV>
SDEV double m0_kernel(const Geom& g, int k, double r2)
{
    double a = 0.25 * g.alpha * r2;
    double t1 = g.t[k + 1], t0 = g.t[k];
    double z1 = a / t1;
    double x1, x0;
    if (k == 0) {
        double E = e1t<DERIV>(z1, x1);
        return DERIV ? (E - x1) * kInv4Pi : g.alpha * kInv4Pi * E;
    }
    double z0 = a / t0, dE;
    if (z0 <= 2.0) {
        dE = log(t1 / t0) + ein(z1) - ein(z0);    // no ln a cancellation
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

// For k >= 1, with z = a/t, E1(a/t_{k+1}) - E1(a/t_k) = ln(t_{k+1}/t_k)
// + Ein(a/t_{k+1}) - Ein(a/t_k) is a power series in a; when a/t_k stays
// <= 4 (a <= amax[k]) it is evaluated from precomputed coefficients
// (row-wise table, Horner); farther pairs use E1 directly.  DERIV adds -(e^{-a/t_{k+1}} - e^{-a/t_k}).
constexpr int kPolyMax = 40;
struct M0Poly { const double* c; const double* cd; const int* n; const double* amax; };   // [nt][kPolyMax], [nt], [nt]

// Horner over the full zero-padded coefficient row (leading zeros leave it
// unchanged), unrolled so that the coefficient loads are issued ahead
SDEV double m0_poly(const double* c, int, double a)
{
    double p = c[kPolyMax - 1];
#pragma unroll
    for (int q = kPolyMax - 2; q >= 0; --q) p = p * a + c[q];
    return p;
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
template <bool DERIV, bool FIRST>
SDEV void m0_tri_moments(const Tables& T, const M0Tables& D, const M0Orders& MO, const Geom& g,
                         const Mesh2& m, const M0Poly& PP, int k, int i, int t, int qs, double* out)
{
    Piece S = seg_piece(g, i);
    Tri3 tr = load_tri3(m, t);
    if (FIRST) {
        Tri tt;
        tt.ax = tr.ax; tt.ay = tr.ay; tt.bx = tr.bx; tt.by = tr.by; tt.cx = tr.cx; tt.cy = tr.cy;
        double dx1 = tr.bx - tr.ax, dy1 = tr.by - tr.ay, dx2 = tr.cx - tr.ax, dy2 = tr.cy - tr.ay;
        double diam = sqrt(fmax(fmax(dx1 * dx1 + dy1 * dy1, dx2 * dx2 + dy2 * dy2),
                                (dx2 - dx1) * (dx2 - dx1) + (dy2 - dy1) * (dy2 - dy1)));
        double size = fmax(diam, S.len);
        double eta = seg_tri_dist(S, tt) / size;
        if (eta < MO.near_ratio) {
            double sm[3], lg[3];
            m0_regular3(T, S, tr, MO.qs_near, MO.qt_near, [&](double r2) { return m0_smooth0<DERIV>(g, r2, 0.5 * log(r2)); }, sm);
            seg_log_potential3(D, S, tr, lg);
            double B = DERIV ? kInv2Pi : g.alpha * kInv2Pi;
            for (int v = 0; v < 3; ++v) out[v] = sm[v] - B * lg[v];
            return;
        }
        // ln r singularity at distance eta * size; the factor e^{-z},
        // z = alpha r^2 / (4 t_1), changes by dz along the elements
        int qn = eta < 1.0 ? kMaxGL : eta < 2.0 ? 12 : eta < 4.0 ? 8 : eta < 8.0 ? 6 : eta < 16.0 ? 5 : 4;
        const double w2 = 0.25 * g.alpha / g.t[1], rlo = eta * size;
        const int qz = q_slope(w2 * rlo * rlo, w2 * size * (2.0 * rlo + size), MO.q_tol, MO.z_floor);
        int q0 = qn > qz ? qn : qz;
        q0 = q0 > qs ? q0 : qs;
        m0_regular3(T, S, tr, q0, q0, [&](double r2) { return m0_kernel<DERIV>(g, 0, r2); }, out);
        return;
    }
    const int n = PP.n[k];
    if (n > 0) {
        const double* c = (DERIV ? PP.cd : PP.c) + (long long)k * kPolyMax;
        const double amax = PP.amax[k], q4 = 0.25 * g.alpha, sc = (DERIV ? 1.0 : g.alpha) * kInv4Pi;
        m0_regular3(T, S, tr, qs, qs, [&](double r2) {
            double a = q4 * r2;
            return a <= amax ? sc * m0_poly(c, n, a) : m0_kernel<DERIV>(g, k, r2);
        }, out);
        return;
    }
    m0_regular3(T, S, tr, qs, qs, [&](double r2) { return m0_kernel<DERIV>(g, k, r2); }, out);
}

}  // namespace stbem
