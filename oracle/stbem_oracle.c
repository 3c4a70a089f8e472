/*
 * CPU oracle for the space-time Galerkin boundary element method of the
 * 2D heat equation (Dohr, Merta, Of, Steinbach, Zapletal, arXiv:1811.05224).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library and never calls it.
 *
 * What it computes (all in x87 long double, slowly and plainly):
 *   U*(z,s) = alpha/(4 pi s) exp(-alpha|z|^2/(4s))            (Sec. 1)
 *   V_h, K_h, M_h^0 of eq.(4)                                   (Sec. 1)
 *   D_h on the dual mesh: integration-by-parts form on touching time
 *   elements, the raw kernel -d_nx d_ny k (its definition, D = -d_n W)
 *   on separated ones, where it is smooth                      (Sec. 2, Thm 1)
 *   and the alpha-derivatives of V_h, K_h, M_h^0.
 *
 * Time integrals are exact: for a kernel kappa(t - tau) that vanishes for
 * t <= tau, int_{tau_k} int_{tau_m} kappa = F(t_{k+1}-t_m) - F(t_{k+1}-t_{m+1})
 *   - F(t_k - t_m) + F(t_k - t_{m+1}) with F the second antiderivative
 * (F = 0 for arguments <= 0; that is causality).  This closed form is used
 * for touching elements (k - m <= 1); for separated elements the same double
 * integral is taken directly, as a Gauss rule in the lag t - tau against the
 * trapezoid weight, which avoids the cancellation of the four-point
 * difference.  With a = alpha r^2 / 4:
 *   F_V(d) = [(d + a) E1(a/d) - d e^{-a/d}] / (4 pi)     single layer
 *   F_K(d) =  d e^{-a/d} - a E1(a/d)   (times (x-y).n_y / (2 pi r^2))
 *   F_D(d) =  E1(a/d) / (4 pi)         first antiderivative, used with the
 *                                      time derivative of the kernel (D_h)
 * Spatial integrals use adaptive tensor Gauss-Legendre with directional
 * error estimates; a vertex shared by two pieces is removed by a Duffy
 * split, a coincident pair by the difference variable eps = |s - s'|, and
 * both singular coordinates are mapped by u = exp(-sigma) so that the log
 * and 1/r behaviour turns into exponential decay.  No singular splitting,
 * no series, no fixed rule: plain definitions integrated to ~1e-16.
 *
 * Pins (CPU tests; none compares the oracle with itself):
 *   E1 and the time primitives: mpmath tables and quadrature of the raw
 *     kernels (V, K, D, dV/dalpha and the E1 kernel of dK/dalpha; M_h^0's);
 *   V_h, K_h, D_h entries: brute-force integration of the raw fundamental
 *     solution on coincident, vertex-sharing and separated pairs of touching
 *     and separated time elements (D_h in the by-parts form, and against
 *     the raw hypersingular kernel where the supports are disjoint);
 *   M_h^0 rows of the first steps: brute force near the boundary;
 *   dV, dK, dM_0: central differences in alpha of V_h, K_h, M_h^0;
 *   together: affine exactness of eq.(4), the constant identity, symmetry
 *     and positivity of V_h and D_h, causality, Toeplitz invariance, the
 *     scaling laws, the lumped mass by quadrature, convergence of the flux.
 *
 * Conventions: segment i joins polygon vertex i to vertex i+1 (cyclic),
 * outward normal n = (e_y, -e_x) for a CCW polygon; time element m is
 * (t_m, t_{m+1}]; DOF l = m * N_Gamma + i.
 * Dual mesh (used for D_h): node i is the midpoint of segment i; dual
 * function psi_i is the continuous piecewise-linear hat on the two dual
 * elements [mid_{i-1}, x_i, mid_i] and [mid_i, x_{i+1}, mid_{i+1}], linear
 * in arclength on each (so it bends at polygon corners).  It is handled on
 * half-segment pieces: piece 2i = [x_i, mid_i], piece 2i+1 = [mid_i, x_{i+1}].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef long double R;
#define PI_L 3.141592653589793238462643383279502884L
#define EULER_L 0.577215664901532860606512090082402431L

/* ------------------------------------------------------------------ E1 */
/* Exponential integral E1(z) = int_z^inf e^{-t}/t dt, z > 0.
 * z <= 2: E1 = -gamma - ln z + sum_{n>=1} (-1)^{n+1} z^n / (n n!)
 * z >  2: continued fraction E1 = e^{-z} / (z+1 - 1/(z+3 - 4/(z+5 - ...))),
 *         evaluated forward with the modified Lentz method.               */
static R e1l(R z)
{
    if (!(z > 0)) return INFINITY;
    if (z > 11300.0L) return 0.0L;
    if (z <= 2.0L) {
        R term = z, sum = z;            /* term_n = (-1)^{n+1} z^n / n! */
        for (int n = 2; n < 200; ++n) {
            term *= -z / n;
            R add = term / n;
            sum += add;
            if (fabsl(add) < 1e-24L * fabsl(sum)) break;
        }
        return -EULER_L - logl(z) + sum;
    }
    const R tiny = 1e-4000L;
    R b = z + 1.0L;
    R f = b, C = b, D = 0.0L;
    for (int n = 1; n < 100000; ++n) {
        R an = -(R)n * (R)n;
        b += 2.0L;
        D = b + an * D; if (D == 0) D = tiny; D = 1.0L / D;
        C = b + an / C; if (C == 0) C = tiny;
        R del = C * D;
        f *= del;
        if (fabsl(del - 1.0L) < 1e-22L) break;
    }
    return expl(-z) / f;
}

/* --------------------------------------------------- time primitives */
static R FV(R a, R d) { if (!(d > 0)) return 0; R z = a / d; return ((d + a) * e1l(z) - d * expl(-z)) / (4 * PI_L); }
static R FK(R a, R d) { if (!(d > 0)) return 0; R z = a / d; return d * expl(-z) - a * e1l(z); }
static R FD(R a, R d) { if (!(d > 0)) return 0; return e1l(a / d) / (4 * PI_L); }
/* d/d alpha of F_V at fixed r (a = alpha r^2/4): (a E1 - d e^{-a/d})/(4 pi alpha) -- the 1/alpha is applied by the caller */
static R FdV(R a, R d) { if (!(d > 0)) return 0; R z = a / d; return (a * e1l(z) - d * expl(-z)) / (4 * PI_L); }
/* E1(a/d) itself; d/dalpha of F_K is -(r^2/4) E1(a/d) */
static R FE(R a, R d) { if (!(d > 0)) return 0; return e1l(a / d); }

typedef struct { R tk0, tk1, tm0, tm1; int d; } TB;    /* tau_k = (tk0,tk1], tau_m = (tm0,tm1] */

static R delta4(R (*F)(R, R), R a, const TB* b)
{
    return F(a, b->tk1 - b->tm0) - F(a, b->tk1 - b->tm1) - F(a, b->tk0 - b->tm0) + F(a, b->tk0 - b->tm1);
}

/* Separated time elements (tau_k after tau_m with a gap): the double time
 * integral itself, int_{tau_k} int_{tau_m} kappa(t - tau) = int w(s) kappa(s) ds,
 * w(s) = |tau_k intersected with (tau_m + s)| (a trapezoid), by Gauss-Legendre on
 * the three linear pieces of w.  kappa is smooth there (s >= gap > 0), and
 * unlike the four-point difference of antiderivatives nothing cancels.
 * kind: 0 k, 1 a e^{-a/s}/s^2 (F_K''), 2 d/ds k, 3 d/dalpha k (times alpha),
 *       4 (e^{-a/s}/s)' = E1(a/s)'' */
static R kappa(int kind, R a, R s)
{
    R x = expl(-a / s);
    switch (kind) {
    case 0: return x / (4 * PI_L * s);
    case 1: return a * x / (s * s);
    case 2: return x * (a - s) / (4 * PI_L * s * s * s);
    case 3: return -(a / s) * x / (4 * PI_L * s);
    case 4: return x * (a - s) / (s * s * s);
    }
    return NAN;
}

/* raw hypersingular kernel -d_nx d_ny k (Sec. 2: D = -d_n W):
 * k(s) [ (alpha^2/(4 s^2)) (z.n_x)(z.n_y) - (alpha/(2 s)) n_x.n_y ] */
static R kappa_raw(R alpha, R a, R s, R zx, R zy, R nn)
{
    R k = expl(-a / s) / (4 * PI_L * s);
    return k * (alpha * alpha / (4 * s * s) * zx * zy - alpha / (2 * s) * nn);
}

#define TQ_N 20
static R gl_x[33][32], gl_w[33][32];
static R tquad(int kind, R a, const TB* b)
{
    R br[4] = {b->tk0 - b->tm1, b->tk0 - b->tm0, b->tk1 - b->tm1, b->tk1 - b->tm0};
    for (int i = 1; i < 4; ++i)
        for (int j = i; j > 0 && br[j] < br[j - 1]; --j) { R t = br[j]; br[j] = br[j - 1]; br[j - 1] = t; }
    R sum = 0;
    for (int p = 0; p < 3; ++p) {
        R lo = br[p], hi = br[p + 1];
        if (!(hi > lo)) continue;
        for (int q = 0; q < TQ_N; ++q) {
            R s = lo + (hi - lo) * gl_x[TQ_N][q];
            R w = fminl(b->tk1, b->tm1 + s) - fmaxl(b->tk0, b->tm0 + s);
            if (w > 0) sum += (hi - lo) * gl_w[TQ_N][q] * w * kappa(kind, a, s);
        }
    }
    return sum;
}

static R tquad_raw(R alpha, R a, R zx, R zy, R nn, const TB* b)
{
    R br[4] = {b->tk0 - b->tm1, b->tk0 - b->tm0, b->tk1 - b->tm1, b->tk1 - b->tm0};
    for (int i = 1; i < 4; ++i)
        for (int j = i; j > 0 && br[j] < br[j - 1]; --j) { R t = br[j]; br[j] = br[j - 1]; br[j - 1] = t; }
    R sum = 0;
    for (int p = 0; p < 3; ++p) {
        R lo = br[p], hi = br[p + 1];
        if (!(hi > lo)) continue;
        for (int q = 0; q < TQ_N; ++q) {
            R s = lo + (hi - lo) * gl_x[TQ_N][q];
            R w = fminl(b->tk1, b->tm1 + s) - fmaxl(b->tk0, b->tm0 + s);
            if (w > 0) sum += (hi - lo) * gl_w[TQ_N][q] * w * kappa_raw(alpha, a, s, zx, zy, nn);
        }
    }
    return sum;
}

/* ------------------------------------------------ Gauss-Legendre nodes */
#define GL_MAX 32     /* gl_x, gl_w: [GL_MAX + 1][GL_MAX] nodes/weights on [0,1] */

__attribute__((constructor)) static void gl_init(void)
{
    for (int n = 1; n <= GL_MAX; ++n) {
        for (int i = 0; i < n; ++i) {
            R x = cosl(PI_L * (i + 0.75L) / (n + 0.5L));
            R dp = 0;
            for (int it = 0; it < 100; ++it) {
                R p0 = 1, p1 = x;
                for (int k = 2; k <= n; ++k) { R p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k; p0 = p1; p1 = p2; }
                if (n == 1) { p1 = x; p0 = 1; }
                dp = n * (x * p1 - p0) / (x * x - 1);
                R dx = p1 / dp;
                x -= dx;
                if (fabsl(dx) < 1e-21L) break;
            }
            {   R p0 = 1, p1 = x;
                for (int k = 2; k <= n; ++k) { R p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k; p0 = p1; p1 = p2; }
                dp = n * (x * p1 - p0) / (x * x - 1); }
            gl_x[n][i] = 0.5L * (1 - x);
            gl_w[n][i] = 1.0L / ((1 - x * x) * dp * dp);          /* = w_[-1,1] / 2 */
        }
    }
}

/* ---------------------------------------------- adaptive integrators */
#define NCMAX 8
typedef void (*fn2)(void* ctx, R u, R v, R* out);
typedef void (*fn1)(void* ctx, R u, R* out);

static void rule2(fn2 f, void* c, int nc, R u0, R u1, R v0, R v1, int nu, int nv, R* out, R* aout)
{
    R du = u1 - u0, dv = v1 - v0, val[NCMAX];
    for (int q = 0; q < nc; ++q) { out[q] = 0; if (aout) aout[q] = 0; }
    for (int i = 0; i < nu; ++i)
        for (int j = 0; j < nv; ++j) {
            R w = gl_w[nu][i] * gl_w[nv][j] * du * dv;
            f(c, u0 + du * gl_x[nu][i], v0 + dv * gl_x[nv][j], val);
            for (int q = 0; q < nc; ++q) { out[q] += w * val[q]; if (aout) aout[q] += fabsl(w * val[q]); }
        }
}

#define NLO 10
#define NHI 14
/* Globally adaptive cubature on a box: every box carries the NHI x NHI
 * result and two directional error estimates (lower order in u, lower order
 * in v); the box with the largest estimate is halved along its worse
 * direction until the summed estimate is below tol or maxbox is reached. */
typedef struct { R u0, u1, v0, v1, eu, ev; R val[NCMAX]; } Box2;

static void box2_eval(fn2 f, void* c, int nc, Box2* b)
{
    R lh[NCMAX], hl[NCMAX];
    rule2(f, c, nc, b->u0, b->u1, b->v0, b->v1, NHI, NHI, b->val, 0);
    rule2(f, c, nc, b->u0, b->u1, b->v0, b->v1, NLO, NHI, lh, 0);
    rule2(f, c, nc, b->u0, b->u1, b->v0, b->v1, NHI, NLO, hl, 0);
    b->eu = b->ev = 0;
    for (int q = 0; q < nc; ++q) {
        R a = fabsl(b->val[q] - lh[q]), d = fabsl(b->val[q] - hl[q]);
        if (a > b->eu) b->eu = a;
        if (d > b->ev) b->ev = d;
    }
}

#define MAXBOX2 600
static void gadapt2(fn2 f, void* c, int nc, R u0, R u1, R v0, R v1, R tol, R* out)
{
    Box2* bx = (Box2*)malloc(sizeof(Box2) * MAXBOX2);
    int n = 1;
    bx[0].u0 = u0; bx[0].u1 = u1; bx[0].v0 = v0; bx[0].v1 = v1;
    box2_eval(f, c, nc, &bx[0]);
    for (;;) {
        R tot = 0, worst = -1; int w = 0;
        for (int i = 0; i < n; ++i) {
            R e = bx[i].eu + bx[i].ev;
            tot += e;
            if (e > worst) { worst = e; w = i; }
        }
        if (tot <= tol || n >= MAXBOX2) break;
        Box2 a = bx[w], b = bx[w];
        if (bx[w].eu >= bx[w].ev) { R m = 0.5L * (a.u0 + a.u1); a.u1 = m; b.u0 = m; }
        else                      { R m = 0.5L * (a.v0 + a.v1); a.v1 = m; b.v0 = m; }
        box2_eval(f, c, nc, &a);
        box2_eval(f, c, nc, &b);
        bx[w] = a; bx[n++] = b;
    }
    for (int q = 0; q < nc; ++q) out[q] = 0;
    for (int i = 0; i < n; ++i) for (int q = 0; q < nc; ++q) out[q] += bx[i].val[q];
    free(bx);
}

/* integrate f over a box to an absolute accuracy ~rtol * int |f| */
static void integrate2(fn2 f, void* c, int nc, R u0, R u1, R v0, R v1, R rtol, R* out)
{
    R est[NCMAX], aest[NCMAX];
    R amax = 0;
    for (int q = 0; q < nc; ++q) aest[q] = 0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            R tmp[NCMAX];
            rule2(f, c, nc, u0 + (u1 - u0) * a / 2, u0 + (u1 - u0) * (a + 1) / 2,
                  v0 + (v1 - v0) * b / 2, v0 + (v1 - v0) * (b + 1) / 2, 8, 8, est, tmp);
            for (int q = 0; q < nc; ++q) aest[q] += tmp[q];
        }
    for (int q = 0; q < nc; ++q) if (aest[q] > amax) amax = aest[q];
    for (int q = 0; q < nc; ++q) out[q] = 0;
    if (amax == 0) return;
    gadapt2(f, c, nc, u0, u1, v0, v1, rtol * amax, out);
}

/* globally adaptive Gauss-Legendre (12 vs 18 points) on [a,b] */
typedef struct { R a, b, e; R val[NCMAX]; } Box1;

static void box1_eval(fn1 f, void* c, int nc, Box1* bx)
{
    R lo[NCMAX], val[NCMAX];
    for (int q = 0; q < nc; ++q) lo[q] = bx->val[q] = 0;
    R d = bx->b - bx->a;
    for (int i = 0; i < 12; ++i) { f(c, bx->a + d * gl_x[12][i], val); for (int q = 0; q < nc; ++q) lo[q] += d * gl_w[12][i] * val[q]; }
    for (int i = 0; i < 18; ++i) { f(c, bx->a + d * gl_x[18][i], val); for (int q = 0; q < nc; ++q) bx->val[q] += d * gl_w[18][i] * val[q]; }
    bx->e = 0;
    for (int q = 0; q < nc; ++q) { R t = fabsl(bx->val[q] - lo[q]); if (t > bx->e) bx->e = t; }
}

#define MAXBOX1 200
static void gadapt1(fn1 f, void* c, int nc, R a, R b, R tol, R* acc)
{
    Box1 bx[MAXBOX1];
    int n = 1;
    bx[0].a = a; bx[0].b = b;
    box1_eval(f, c, nc, &bx[0]);
    for (;;) {
        R tot = 0, worst = -1; int w = 0;
        for (int i = 0; i < n; ++i) { tot += bx[i].e; if (bx[i].e > worst) { worst = bx[i].e; w = i; } }
        if (tot <= tol || n >= MAXBOX1) break;
        Box1 l = bx[w], r = bx[w];
        R m = 0.5L * (l.a + l.b); l.b = m; r.a = m;
        box1_eval(f, c, nc, &l); box1_eval(f, c, nc, &r);
        bx[w] = l; bx[n++] = r;
    }
    for (int i = 0; i < n; ++i) for (int q = 0; q < nc; ++q) acc[q] += bx[i].val[q];
}

/* --------------------------------------------------------- problem */
typedef struct {
    int ng, nt, nv, ntri;
    R alpha;
    R* t;                                   /* nt + 1 */
    R *px, *py;                             /* polygon vertices */
    R *ex, *ey, *L, *nx, *ny;               /* segment unit tangent, length, normal */
    R *ox, *oy;                             /* Omega vertices */
    int* tri;                               /* 3 * ntri */
    int *v2t_ptr, *v2t;                     /* vertex -> triangles */
} Prob;

typedef struct { R ax, ay, ex, ey, L, nx, ny; int id, np; } Piece;

static Prob* prob_new(double alpha, int nt, const double* t, int ng, const double* bxy,
                      int nv, const double* vxy, int ntri, const int* tri)
{
    Prob* p = (Prob*)calloc(1, sizeof(Prob));
    p->ng = ng; p->nt = nt; p->nv = nv; p->ntri = ntri; p->alpha = alpha;
    p->t = (R*)malloc(sizeof(R) * (nt + 1));
    for (int i = 0; i <= nt; ++i) p->t[i] = t[i];
    R* buf = (R*)malloc(sizeof(R) * 7 * ng);
    p->px = buf; p->py = buf + ng; p->ex = buf + 2 * ng; p->ey = buf + 3 * ng;
    p->L = buf + 4 * ng; p->nx = buf + 5 * ng; p->ny = buf + 6 * ng;
    for (int i = 0; i < ng; ++i) { p->px[i] = bxy[2 * i]; p->py[i] = bxy[2 * i + 1]; }
    for (int i = 0; i < ng; ++i) {
        int j = (i + 1) % ng;
        R dx = p->px[j] - p->px[i], dy = p->py[j] - p->py[i];
        R L = sqrtl(dx * dx + dy * dy);
        p->L[i] = L; p->ex[i] = dx / L; p->ey[i] = dy / L;
        p->nx[i] = p->ey[i]; p->ny[i] = -p->ex[i];
    }
    p->ox = (R*)malloc(sizeof(R) * (nv > 0 ? nv : 1));
    p->oy = (R*)malloc(sizeof(R) * (nv > 0 ? nv : 1));
    for (int i = 0; i < nv; ++i) { p->ox[i] = vxy[2 * i]; p->oy[i] = vxy[2 * i + 1]; }
    p->tri = (int*)malloc(sizeof(int) * 3 * (ntri > 0 ? ntri : 1));
    memcpy(p->tri, tri, sizeof(int) * 3 * ntri);
    p->v2t_ptr = (int*)calloc(nv + 1, sizeof(int));
    p->v2t = (int*)malloc(sizeof(int) * 3 * (ntri > 0 ? ntri : 1));
    for (int e = 0; e < 3 * ntri; ++e) p->v2t_ptr[tri[e] + 1]++;
    for (int v = 0; v < nv; ++v) p->v2t_ptr[v + 1] += p->v2t_ptr[v];
    int* fill = (int*)calloc(nv + 1, sizeof(int));
    for (int e = 0; e < 3 * ntri; ++e) { int v = tri[e]; p->v2t[p->v2t_ptr[v] + fill[v]++] = e / 3; }
    free(fill);
    return p;
}

static void prob_free(Prob* p)
{
    if (!p) return;
    free(p->t); free(p->px); free(p->ox); free(p->oy); free(p->tri); free(p->v2t_ptr); free(p->v2t); free(p);
}

static Piece seg_piece(const Prob* p, int i)
{
    Piece q = { p->px[i], p->py[i], p->ex[i], p->ey[i], p->L[i], p->nx[i], p->ny[i], i, p->ng };
    return q;
}

static Piece half_piece(const Prob* p, int h)
{
    int i = h / 2;
    Piece q = seg_piece(p, i);
    q.L = 0.5L * p->L[i];
    if (h & 1) { q.ax = p->px[i] + q.L * p->ex[i]; q.ay = p->py[i] + q.L * p->ey[i]; }
    q.id = h; q.np = 2 * p->ng;
    return q;
}

static TB time_block(const Prob* p, int k, int m)
{
    TB b = { p->t[k], p->t[k + 1], p->t[m], p->t[m + 1], k - m };
    return b;
}

/* ------------------------------------------------ piece-pair kernels */
enum { OP_V = 0, OP_K = 1, OP_D = 2, OP_M0 = 3, OP_DV = 4, OP_DK = 5, OP_DM0 = 6 };

typedef struct {
    const Prob* pr; TB tb; int op;
    const Piece *P, *Q;
} KC;

/* value of the integrand at x = P(sP), y = Q(sQ), with x - y = (dx,dy) */
static void kern(const KC* c, R sP, R sQ, R dx, R dy, R* out)
{
    R r2 = dx * dx + dy * dy;
    R a = c->pr->alpha * r2 / 4;
    int sep = c->tb.d >= 2;      /* separated time elements: integrate in time */
    switch (c->op) {
    case OP_V:
        out[0] = sep ? tquad(0, a, &c->tb) : delta4(FV, a, &c->tb);
        break;
    case OP_DV:
        out[0] = (sep ? tquad(3, a, &c->tb) : delta4(FdV, a, &c->tb)) / c->pr->alpha;
        break;
    case OP_K: {
        R g = (dx * c->Q->nx + dy * c->Q->ny) / (2 * PI_L * r2) * (sep ? tquad(1, a, &c->tb) : delta4(FK, a, &c->tb));
        R l1 = sQ / c->Q->L;
        out[0] = g * (1 - l1); out[1] = g * l1;
        break; }
    case OP_DK: {
        R g = -(dx * c->Q->nx + dy * c->Q->ny) / (8 * PI_L) * (sep ? tquad(4, a, &c->tb) : delta4(FE, a, &c->tb));
        R l1 = sQ / c->Q->L;
        out[0] = g * (1 - l1); out[1] = g * l1;
        break; }
    case OP_D: {
        R p1 = sP / c->P->L, q1 = sQ / c->Q->L;
        if (sep) {
            /* separated time elements: the kernel is smooth, D is taken from
             * its definition, the raw kernel; out[0] (curl part) unused and
             * out[1..4] already carry alpha n.n */
            R zx = dx * c->P->nx + dy * c->P->ny, zy = dx * c->Q->nx + dy * c->Q->ny;
            R nn = c->P->nx * c->Q->nx + c->P->ny * c->Q->ny;
            R raw = tquad_raw(c->pr->alpha, a, zx, zy, nn, &c->tb);
            out[0] = 0;
            out[1] = raw * (1 - p1) * (1 - q1); out[2] = raw * (1 - p1) * q1;
            out[3] = raw * p1 * (1 - q1);       out[4] = raw * p1 * q1;
            break;
        }
        R fv = delta4(FV, a, &c->tb), fd = delta4(FD, a, &c->tb);
        out[0] = fv;
        out[1] = fd * (1 - p1) * (1 - q1); out[2] = fd * (1 - p1) * q1;
        out[3] = fd * p1 * (1 - q1);       out[4] = fd * p1 * q1;
        break; }
    }
}

static int kern_nc(int op) { return op == OP_D ? 5 : (op == OP_K || op == OP_DK) ? 2 : 1; }

/* separated (or smooth) pair: plain tensor domain */
static void f_sep(void* vc, R sP, R sQ, R* out)
{
    const KC* c = (const KC*)vc;
    R dx = (c->P->ax + sP * c->P->ex) - (c->Q->ax + sQ * c->Q->ex);
    R dy = (c->P->ay + sP * c->P->ey) - (c->Q->ay + sQ * c->Q->ey);
    kern(c, sP, sQ, dx, dy, out);
}

/* coincident pair: difference variable eps = |s - s'| and s = (L - eps) t.
 * Touching time elements (d <= 1, log singular at eps = 0): eps = L exp(-sig).
 * Separated time elements (smooth kernel): eps = L sig, sig in [0,1]. */
#define SIGMAX 46.0L
static void f_coinc(void* vc, R sig, R t, R* out)
{
    const KC* c = (const KC*)vc;
    int nc = kern_nc(c->op);
    R L = c->P->L, eps, w;
    if (c->tb.d <= 1) { eps = L * expl(-sig); w = eps; }
    else              { eps = L * sig;        w = L; }
    R s = (L - eps) * t;
    w *= (L - eps);
    R v1[NCMAX], v2[NCMAX];
    kern(c, s + eps, s, eps * c->P->ex, eps * c->P->ey, v1);
    kern(c, s, s + eps, -eps * c->P->ex, -eps * c->P->ey, v2);
    for (int q = 0; q < nc; ++q) out[q] = w * (v1[q] + v2[q]);
}

/* pieces sharing a vertex V: x = V + sp*e1, y = V + sq*e2 (sp, sq distances from V) */
typedef struct { const KC* c; int pend, qend; R e1x, e1y, e2x, e2y; int tri; } VC;

static void f_vert(void* vv, R tau, R w, R* out)
{
    const VC* v = (const VC*)vv;
    const KC* c = v->c;
    int nc = kern_nc(c->op);
    R u = expl(-tau), LP = c->P->L, LQ = c->Q->L;
    R sp, sq;
    if (v->tri == 0) { sp = LP * u; sq = LQ * u * w; }
    else             { sq = LQ * u; sp = LP * u * w; }
    R dx = sp * v->e1x - sq * v->e2x, dy = sp * v->e1y - sq * v->e2y;
    R sP = v->pend ? LP - sp : sp, sQ = v->qend ? LQ - sq : sq;
    R val[NCMAX];
    kern(c, sP, sQ, dx, dy, val);
    R jac = LP * LQ * u * u;
    for (int q = 0; q < nc; ++q) out[q] = jac * val[q];
}

#define RTOL 1e-16L

static void pair_integral(const KC* c, R* out)
{
    int nc = kern_nc(c->op);
    const Piece *P = c->P, *Q = c->Q;
    int np = P->np;
    int rel = 0, pend = 0, qend = 0;
    if (P->id == Q->id) rel = 1;
    else if ((P->id + 1) % np == Q->id) { rel = 2; pend = 1; qend = 0; }
    else if ((Q->id + 1) % np == P->id) { rel = 2; pend = 0; qend = 1; }
    for (int q = 0; q < nc; ++q) out[q] = 0;
    if (rel == 1) {
        integrate2(f_coinc, (void*)c, nc, 0, c->tb.d <= 1 ? SIGMAX : 1.0L, 0, 1, RTOL, out);
    } else if (rel == 2 && c->tb.d <= 1) {
        VC v; v.c = c; v.pend = pend; v.qend = qend;
        v.e1x = pend ? -P->ex : P->ex; v.e1y = pend ? -P->ey : P->ey;
        v.e2x = qend ? -Q->ex : Q->ex; v.e2y = qend ? -Q->ey : Q->ey;
        R o1[NCMAX], o2[NCMAX];
        v.tri = 0; integrate2(f_vert, &v, nc, 0, SIGMAX, 0, 1, RTOL, o1);
        v.tri = 1; integrate2(f_vert, &v, nc, 0, SIGMAX, 0, 1, RTOL, o2);
        for (int q = 0; q < nc; ++q) out[q] = o1[q] + o2[q];
    } else {
        integrate2(f_sep, (void*)c, nc, 0, P->L, 0, Q->L, RTOL, out);
    }
}

/* ----------------------------------------------------- matrix entries */
/* dual function psi_i on half-segment pieces: returns the 4 pieces and the
 * values of psi_i at each piece's start/end and its arclength derivative */
static void dual_support(const Prob* p, int i, int* pc, R* v0, R* v1, R* dpsi)
{
    int ng = p->ng;
    int im = (i - 1 + ng) % ng, ip = (i + 1) % ng;
    R Lm = p->L[im], Li = p->L[i], Lp = p->L[ip];
    R Lt0 = 0.5L * (Lm + Li), Lt1 = 0.5L * (Li + Lp);       /* dual element lengths */
    pc[0] = 2 * im + 1; v0[0] = 0;                 v1[0] = 0.5L * Lm / Lt0; dpsi[0] = 1 / Lt0;
    pc[1] = 2 * i;      v0[1] = 0.5L * Lm / Lt0;   v1[1] = 1;               dpsi[1] = 1 / Lt0;
    pc[2] = 2 * i + 1;  v0[2] = 1;                 v1[2] = 1 - 0.5L * Li / Lt1; dpsi[2] = -1 / Lt1;
    pc[3] = 2 * ip;     v0[3] = 1 - 0.5L * Li / Lt1; v1[3] = 0;             dpsi[3] = -1 / Lt1;
}

static R entry(const Prob* p, int op, int k, int m, int i, int j)
{
    if (k < m) return 0;                     /* causality */
    KC c; c.pr = p; c.tb = time_block(p, k, m); c.op = op;
    R out[NCMAX];
    if (op == OP_V || op == OP_DV) {
        Piece P = seg_piece(p, i), Q = seg_piece(p, j);
        c.P = &P; c.Q = &Q;
        pair_integral(&c, out);
        return out[0];
    }
    if (op == OP_K || op == OP_DK) {
        /* hat_j lives on segment j-1 (rising, shape s/L) and segment j (falling) */
        int jm = (j - 1 + p->ng) % p->ng;
        Piece P = seg_piece(p, i), Q1 = seg_piece(p, jm), Q2 = seg_piece(p, j);
        R acc = 0;
        c.P = &P; c.Q = &Q1; pair_integral(&c, out); acc += out[1];
        c.Q = &Q2;            pair_integral(&c, out); acc += out[0];
        return acc;
    }
    if (op == OP_D) {
        int pi[4], pj[4]; R a0[4], a1[4], da[4], b0[4], b1[4], db[4];
        dual_support(p, i, pi, a0, a1, da);
        dual_support(p, j, pj, b0, b1, db);
        R acc = 0;
        for (int u = 0; u < 4; ++u)
            for (int v = 0; v < 4; ++v) {
                Piece P = half_piece(p, pi[u]), Q = half_piece(p, pj[v]);
                c.P = &P; c.Q = &Q;
                pair_integral(&c, out);
                R nn = c.tb.d >= 2 ? 1.0L / p->alpha : P.nx * Q.nx + P.ny * Q.ny;   /* raw form carries alpha n.n */
                acc += da[u] * db[v] * out[0]
                     + p->alpha * nn * (a0[u] * b0[v] * out[1] + a0[u] * b1[v] * out[2]
                                      + a1[u] * b0[v] * out[3] + a1[u] * b1[v] * out[4]);
            }
        return acc;
    }
    return NAN;
}

/* ------------------------------------------------------- M_h^0 rows */
typedef struct {
    const Prob* pr; int k, deriv;
    R x0, y0, ex, ey;                 /* test segment */
    R ax, ay, bx, by, cx, cy;         /* current (sub)triangle */
    R T[3][3];                        /* barycentric coefficients of the original triangle: phi_v = T[v][0] + T[v][1] x + T[v][2] y */
    R px, py, qx, qy;                 /* polar: apex x, edge start p, edge vector q */
    R s;
} MC;

/* M0 time kernel: int_{tau_k} U*(r, t) dt, or its alpha-derivative */
static R m0_time(const Prob* p, int k, R r2, int deriv)
{
    R a = p->alpha * r2 / 4;
    R t1 = p->t[k + 1], t0 = p->t[k];
    R z1 = a / t1, z0 = (t0 > 0) ? a / t0 : INFINITY;
    R E1 = e1l(z1), E0 = (t0 > 0) ? e1l(z0) : 0;
    if (!deriv) return p->alpha / (4 * PI_L) * (E1 - E0);
    R x1 = expl(-z1), x0 = (t0 > 0) ? expl(-z0) : 0;
    return (E1 - E0 - x1 + x0) / (4 * PI_L);
}

/* smooth case: tensor rule, segment [s0,s1] x collapsed-Gauss triangle */
static void m0_rule(const MC* c, R s0, R s1, const R* A, const R* B, const R* C, int n, R* out)
{
    out[0] = out[1] = out[2] = 0;
    R e1x = B[0] - A[0], e1y = B[1] - A[1], e2x = C[0] - A[0], e2y = C[1] - A[1];
    R area2 = fabsl(e1x * e2y - e1y * e2x);
    for (int is = 0; is < n; ++is) {
        R s = s0 + (s1 - s0) * gl_x[n][is], ws = (s1 - s0) * gl_w[n][is];
        R x = c->x0 + s * c->ex, y = c->y0 + s * c->ey;
        for (int iu = 0; iu < n; ++iu)
            for (int iv = 0; iv < n; ++iv) {
                R u = gl_x[n][iu], v = gl_x[n][iv] * (1 - u);
                R w = ws * gl_w[n][iu] * gl_w[n][iv] * (1 - u) * area2;
                R yx = A[0] + u * e1x + v * e2x, yy = A[1] + u * e1y + v * e2y;
                R dx = x - yx, dy = y - yy;
                R g = w * m0_time(c->pr, c->k, dx * dx + dy * dy, c->deriv);
                for (int q = 0; q < 3; ++q) out[q] += g * (c->T[q][0] + c->T[q][1] * yx + c->T[q][2] * yy);
            }
    }
}

static void m0_adapt(const MC* c, R s0, R s1, const R* A, const R* B, const R* C, R tol, int depth, R* acc)
{
    R lo[3], hi[3];
    m0_rule(c, s0, s1, A, B, C, 8, lo);
    m0_rule(c, s0, s1, A, B, C, 12, hi);
    R e = 0;
    for (int q = 0; q < 3; ++q) { R t = fabsl(hi[q] - lo[q]); if (t > e) e = t; }
    if (e <= tol || depth >= 3) { for (int q = 0; q < 3; ++q) acc[q] += hi[q]; return; }
    R sm = 0.5L * (s0 + s1);
    R AB[2] = {0.5L * (A[0] + B[0]), 0.5L * (A[1] + B[1])};
    R BC[2] = {0.5L * (B[0] + C[0]), 0.5L * (B[1] + C[1])};
    R CA[2] = {0.5L * (C[0] + A[0]), 0.5L * (C[1] + A[1])};
    const R* sub[4][3] = {{A, AB, CA}, {AB, B, BC}, {CA, BC, C}, {AB, BC, CA}};
    for (int h = 0; h < 2; ++h)
        for (int t = 0; t < 4; ++t)
            m0_adapt(c, h ? sm : s0, h ? s1 : sm, sub[t][0], sub[t][1], sub[t][2], tol / 8, depth + 1, acc);
}

/* singular case (first time step, triangle touching the segment):
 * polar coordinates about x: y = x + lam (p + tau q - x), lam = exp(-sig) */
static void f_polar(void* vc, R tau, R sig, R* out)
{
    const MC* c = (const MC*)vc;
    R lam = expl(-sig);
    R ex = c->px + tau * c->qx - c->ax, ey = c->py + tau * c->qy - c->ay;   /* ax,ay hold the apex here */
    R yx = c->ax + lam * ex, yy = c->ay + lam * ey;
    R J = (c->px - c->ax) * c->qy - (c->py - c->ay) * c->qx;               /* signed 2*area of (x, p, p+q) */
    R r2 = lam * lam * (ex * ex + ey * ey);
    R g = J * lam * lam * m0_time(c->pr, c->k, r2, c->deriv);
    for (int q = 0; q < 3; ++q) out[q] = g * (c->T[q][0] + c->T[q][1] * yx + c->T[q][2] * yy);
}

typedef struct { MC* c; const R* V[3]; R s0, s1; } PS;

/* the segment coordinate s = s0 + (s1 - s0) psi(t), psi(t) = t^3 (10 - 15 t + 6 t^2):
 * psi' vanishes to second order at both ends, which flattens the weak
 * singularities of the inner integral where x passes a triangle vertex */
static void f_polar_s(void* vp, R tt, R* out)
{
    PS* ps = (PS*)vp;
    MC c = *ps->c;
    R psi = tt * tt * tt * (10 - 15 * tt + 6 * tt * tt), dpsi = 30 * tt * tt * (1 - tt) * (1 - tt);
    R jac = (ps->s1 - ps->s0) * dpsi;
    R s = ps->s0 + (ps->s1 - ps->s0) * psi;
    R x = c.x0 + s * c.ex, y = c.y0 + s * c.ey;
    out[0] = out[1] = out[2] = 0;
    for (int e = 0; e < 3; ++e) {
        const R* P0 = ps->V[e]; const R* P1 = ps->V[(e + 1) % 3];
        c.ax = x; c.ay = y;
        c.px = P0[0]; c.py = P0[1]; c.qx = P1[0] - P0[0]; c.qy = P1[1] - P0[1];
        R J = (c.px - x) * c.qy - (c.py - y) * c.qx;
        R scale = sqrtl(c.qx * c.qx + c.qy * c.qy);
        if (fabsl(J) <= 1e-15L * scale * scale) continue;              /* x on this edge's line */
        R o[3];
        integrate2(f_polar, &c, 3, 0, 1, 0, 40, RTOL, o);
        for (int q = 0; q < 3; ++q) out[q] += jac * o[q];
    }
}

static R seg_pt_dist2(R ax, R ay, R bx, R by, R px, R py)
{
    R dx = bx - ax, dy = by - ay, L2 = dx * dx + dy * dy;
    R t = L2 > 0 ? ((px - ax) * dx + (py - ay) * dy) / L2 : 0;
    if (t < 0) t = 0; if (t > 1) t = 1;
    R qx = ax + t * dx - px, qy = ay + t * dy - py;
    return qx * qx + qy * qy;
}

static int seg_cross(R ax, R ay, R bx, R by, R cx, R cy, R dx, R dy)
{
    R d1 = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
    R d2 = (bx - ax) * (dy - ay) - (by - ay) * (dx - ax);
    R d3 = (dx - cx) * (ay - cy) - (dy - cy) * (ax - cx);
    R d4 = (dx - cx) * (by - cy) - (dy - cy) * (bx - cx);
    return ((d1 > 0 && d2 < 0) || (d1 < 0 && d2 > 0)) && ((d3 > 0 && d4 < 0) || (d3 < 0 && d4 > 0));
}

/* squared distance between segment [a,b] and the closed triangle V */
static R seg_tri_dist2(R ax, R ay, R bx, R by, const R* V[3])
{
    R best = INFINITY;
    for (int e = 0; e < 3; ++e) {
        const R* P = V[e]; const R* Q = V[(e + 1) % 3];
        if (seg_cross(ax, ay, bx, by, P[0], P[1], Q[0], Q[1])) return 0;
        R d;
        d = seg_pt_dist2(P[0], P[1], Q[0], Q[1], ax, ay); if (d < best) best = d;
        d = seg_pt_dist2(P[0], P[1], Q[0], Q[1], bx, by); if (d < best) best = d;
        d = seg_pt_dist2(ax, ay, bx, by, P[0], P[1]);     if (d < best) best = d;
    }
    /* segment start inside the triangle */
    R s0 = (V[1][0] - V[0][0]) * (ay - V[0][1]) - (V[1][1] - V[0][1]) * (ax - V[0][0]);
    R s1 = (V[2][0] - V[1][0]) * (ay - V[1][1]) - (V[2][1] - V[1][1]) * (ax - V[1][0]);
    R s2 = (V[0][0] - V[2][0]) * (ay - V[2][1]) - (V[0][1] - V[2][1]) * (ax - V[2][0]);
    if ((s0 >= 0 && s1 >= 0 && s2 >= 0) || (s0 <= 0 && s1 <= 0 && s2 <= 0)) return 0;
    return best;
}

/* the 3 moments int_{gamma_i} int_omega phi_v(y) G_k(|x-y|) dy ds_x, v = 0,1,2 */
static void m0_triangle(const Prob* p, int k, int i, int t, int deriv, R* out)
{
    MC c; memset(&c, 0, sizeof c);
    c.pr = p; c.k = k; c.deriv = deriv;
    c.x0 = p->px[i]; c.y0 = p->py[i]; c.ex = p->ex[i]; c.ey = p->ey[i];
    R Vv[3][2];
    for (int v = 0; v < 3; ++v) { Vv[v][0] = p->ox[p->tri[3 * t + v]]; Vv[v][1] = p->oy[p->tri[3 * t + v]]; }
    const R* V[3] = {Vv[0], Vv[1], Vv[2]};
    R det = (Vv[1][0] - Vv[0][0]) * (Vv[2][1] - Vv[0][1]) - (Vv[1][1] - Vv[0][1]) * (Vv[2][0] - Vv[0][0]);
    for (int v = 0; v < 3; ++v) {
        const R* B = Vv[(v + 1) % 3]; const R* C = Vv[(v + 2) % 3];
        /* phi_v(y) = cross(C - B, y - B) / det */
        c.T[v][0] = ((C[0] - B[0]) * (-B[1]) - (C[1] - B[1]) * (-B[0])) / det;
        c.T[v][1] = (-(C[1] - B[1])) / det;
        c.T[v][2] = (C[0] - B[0]) / det;
    }
    R L = p->L[i];
    R bx = c.x0 + L * c.ex, by = c.y0 + L * c.ey;
    R d2 = seg_tri_dist2(c.x0, c.y0, bx, by, V);
    out[0] = out[1] = out[2] = 0;
    if (k == 0 && d2 <= 1e-26L * L * L) {
        /* split the segment at the projections of the triangle vertices */
        R cuts[5]; int nc = 0;
        cuts[nc++] = 0;
        for (int v = 0; v < 3; ++v) {
            R s = (Vv[v][0] - c.x0) * c.ex + (Vv[v][1] - c.y0) * c.ey;
            if (s > 1e-12L * L && s < L * (1 - 1e-12L)) cuts[nc++] = s;
        }
        cuts[nc++] = L;
        for (int a = 1; a < nc; ++a)             /* sort */
            for (int b = a; b > 0 && cuts[b] < cuts[b - 1]; --b) { R tmp = cuts[b]; cuts[b] = cuts[b - 1]; cuts[b - 1] = tmp; }
        PS ps; ps.c = &c; ps.V[0] = Vv[0]; ps.V[1] = Vv[1]; ps.V[2] = Vv[2];
        /* magnitude for the tolerance */
        R mag = 0, tmp[3];
        for (int a = 0; a + 1 < nc; ++a) {
            if (cuts[a + 1] - cuts[a] <= 0) continue;
            ps.s0 = cuts[a]; ps.s1 = cuts[a + 1];
            tmp[0] = tmp[1] = tmp[2] = 0;
            f_polar_s(&ps, 0.5L, tmp);
            mag += fabsl(tmp[0]) + fabsl(tmp[1]) + fabsl(tmp[2]);
        }
        for (int a = 0; a + 1 < nc; ++a) {
            if (cuts[a + 1] - cuts[a] <= 0) continue;
            ps.s0 = cuts[a]; ps.s1 = cuts[a + 1];
            gadapt1(f_polar_s, &ps, 3, 0, 1, 1e-16L * mag + 1e-300L, out);
        }
    } else {
        R est[3];
        m0_rule(&c, 0, L, V[0], V[1], V[2], 8, est);
        R mag = fabsl(est[0]) + fabsl(est[1]) + fabsl(est[2]);
        m0_adapt(&c, 0, L, V[0], V[1], V[2], 1e-16L * mag + 1e-300L, 0, out);
    }
}

/* ------------------------------------------- representation formula
 * u(x,t) = (M~0 u0)(x,t) + (V~ w)(x,t) - (W g)(x,t)     (Sec. 1, eq. (2))
 * with the potentials of the discrete data, at points (x, t) of Q:
 *   V~ w = sum_{m,j} w_mj int_{gamma_j} int_{tau_m, tau < t} k(x-y, t-tau)
 *   W g  = sum_{m,n} g_mn int hat_n(y) int_{tau_m, tau < t} d_ny k(x-y, t-tau)
 *   M~0 u0 = int_Omega U*(x-y, t) u0_h(y) dy
 * k = U^* / alpha.  In the lag s = t - tau (s from s_lo = max(t - t_{m+1}, 0)
 * to s_hi = t - t_m), with a = alpha r^2/4, the time integrals are the
 * definitions integrated once in closed form:
 *   int k ds = [E1(a/s_hi) - E1(a/s_lo)] / (4 pi)          (E1(a/0) = 0)
 *   int d_ny k ds = (x-y).n_y / (2 pi r^2) [e^{-a/s_hi} - e^{-a/s_lo}]
 * The space integrals are globally adaptive (segment split at the foot of
 * x, triangle in collapsed coordinates).                                  */
typedef struct { const Prob* pr; R x, y, slo, shi; int j; } PC;

static void f_pot_seg(void* vc, R s, R* out)
{
    const PC* c = (const PC*)vc;
    const Prob* p = c->pr;
    R yx = p->px[c->j] + s * p->ex[c->j], yy = p->py[c->j] + s * p->ey[c->j];
    R dx = c->x - yx, dy = c->y - yy, r2 = dx * dx + dy * dy;
    R a = p->alpha * r2 / 4;
    R sl = (e1l(a / c->shi) - (c->slo > 0 ? e1l(a / c->slo) : 0)) / (4 * PI_L);
    R dn = dx * p->nx[c->j] + dy * p->ny[c->j];
    R dl = dn / (2 * PI_L * r2) * (expl(-a / c->shi) - (c->slo > 0 ? expl(-a / c->slo) : 0));
    R l1 = s / p->L[c->j];
    out[0] = sl;                 /* single layer density 1 */
    out[1] = dl * (1 - l1);      /* double layer, hat of vertex j */
    out[2] = dl * l1;            /* double layer, hat of vertex j + 1 */
}

typedef struct { const Prob* pr; R x, y, t; R A[2], B[2], C[2], area2; R T[3][3]; } PT;

/* collapsed map of the triangle: y = A + u (B - A) + u v (C - B), dy = u area2 du dv */
static void f_pot_tri(void* vc, R u, R v, R* out)
{
    const PT* c = (const PT*)vc;
    R yx = c->A[0] + u * (c->B[0] - c->A[0]) + u * v * (c->C[0] - c->B[0]);
    R yy = c->A[1] + u * (c->B[1] - c->A[1]) + u * v * (c->C[1] - c->B[1]);
    R dx = c->x - yx, dy = c->y - yy;
    R al = c->pr->alpha;
    R U = al / (4 * PI_L * c->t) * expl(-al * (dx * dx + dy * dy) / (4 * c->t)) * u * c->area2;
    for (int q = 0; q < 3; ++q) out[q] = U * (c->T[q][0] + c->T[q][1] * yx + c->T[q][2] * yy);
}

/* out[0] = M~0 u0, out[1] = V~ w, out[2] = W g at (x, y, t) */
static void potential(const Prob* p, R x, R y, R t, const double* w, const double* g, const double* u0, R* out)
{
    out[0] = out[1] = out[2] = 0;
    for (int m = 0; m < p->nt && p->t[m] < t; ++m) {
        PC c; c.pr = p; c.x = x; c.y = y;
        c.shi = t - p->t[m];
        c.slo = t - p->t[m + 1] > 0 ? t - p->t[m + 1] : 0;
        for (int j = 0; j < p->ng; ++j) {
            c.j = j;
            R L = p->L[j];
            R sf = (x - p->px[j]) * p->ex[j] + (y - p->py[j]) * p->ey[j];   /* foot of x */
            R cuts[3] = {0, sf, L}; int nc = 3;
            if (!(sf > 1e-12L * L && sf < L * (1 - 1e-12L))) { cuts[1] = L; nc = 2; }
            R est[3] = {0, 0, 0}, mid[3];
            for (int a = 0; a + 1 < nc; ++a) {
                f_pot_seg(&c, 0.5L * (cuts[a] + cuts[a + 1]), mid);
                for (int q = 0; q < 3; ++q) est[q] += fabsl(mid[q]) * (cuts[a + 1] - cuts[a]);
            }
            R mag = est[0] + est[1] + est[2];
            R acc[3] = {0, 0, 0};
            for (int a = 0; a + 1 < nc; ++a) gadapt1(f_pot_seg, &c, 3, cuts[a], cuts[a + 1], 1e-18L * mag + 1e-300L, acc);
            int jn = j + 1 == p->ng ? 0 : j + 1;
            out[1] += (R)w[m * p->ng + j] * acc[0];
            out[2] += (R)g[m * p->ng + j] * acc[1] + (R)g[m * p->ng + jn] * acc[2];
        }
    }
    if (!u0) return;
    for (int tt = 0; tt < p->ntri; ++tt) {
        PT c; c.pr = p; c.x = x; c.y = y; c.t = t;
        R Vv[3][2];
        for (int v = 0; v < 3; ++v) { Vv[v][0] = p->ox[p->tri[3 * tt + v]]; Vv[v][1] = p->oy[p->tri[3 * tt + v]]; }
        R det = (Vv[1][0] - Vv[0][0]) * (Vv[2][1] - Vv[0][1]) - (Vv[1][1] - Vv[0][1]) * (Vv[2][0] - Vv[0][0]);
        for (int v = 0; v < 3; ++v) {
            const R* B = Vv[(v + 1) % 3]; const R* C = Vv[(v + 2) % 3];
            c.T[v][0] = ((C[0] - B[0]) * (-B[1]) - (C[1] - B[1]) * (-B[0])) / det;
            c.T[v][1] = (-(C[1] - B[1])) / det;
            c.T[v][2] = (C[0] - B[0]) / det;
        }
        /* the vertex nearest to x is the collapsed corner A, so that a peak
         * of the Gaussian near a vertex sits where the rule is dense */
        int a0 = 0; R best = INFINITY;
        for (int v = 0; v < 3; ++v) { R d2 = (Vv[v][0] - x) * (Vv[v][0] - x) + (Vv[v][1] - y) * (Vv[v][1] - y); if (d2 < best) { best = d2; a0 = v; } }
        for (int q = 0; q < 2; ++q) { c.A[q] = Vv[a0][q]; c.B[q] = Vv[(a0 + 1) % 3][q]; c.C[q] = Vv[(a0 + 2) % 3][q]; }
        c.area2 = fabsl(det);
        R mom[3] = {0, 0, 0};
        integrate2(f_pot_tri, &c, 3, 0, 1, 0, 1, 1e-17L, mom);
        for (int v = 0; v < 3; ++v) out[0] += (R)u0[p->tri[3 * tt + v]] * mom[v];
    }
}

/* ------------------------------------------------------------ C ABI */
typedef struct { Prob* p; } or_problem;

or_problem* or_create(double alpha, int nt, const double* t, int ng, const double* bnd_xy,
                      int nv, const double* vtx_xy, int ntri, const int* tri)
{
    if (ng < 3 || nt < 1 || !(alpha > 0)) return 0;
    or_problem* h = (or_problem*)malloc(sizeof(or_problem));
    h->p = prob_new(alpha, nt, t, ng, bnd_xy, nv, vtx_xy, ntri, tri);
    return h;
}

void or_destroy(or_problem* h) { if (h) { prob_free(h->p); free(h); } }

/* entries of V, K, D, dV/dalpha, dK/dalpha: idx holds n quadruples (k, m, i, j) */
int or_entries(const or_problem* h, int op, long n, const int* idx, double* out, int nthreads)
{
    if (!h || !(op == OP_V || op == OP_K || op == OP_D || op == OP_DV || op == OP_DK)) return -1;
    const Prob* p = h->p;
    for (long e = 0; e < n; ++e) {
        const int* q = idx + 4 * e;
        if (q[0] < 0 || q[0] >= p->nt || q[1] < 0 || q[1] >= p->nt || q[2] < 0 || q[2] >= p->ng || q[3] < 0 || q[3] >= p->ng) return -2;
    }
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (long e = 0; e < n; ++e) {
        const int* q = idx + 4 * e;
        out[e] = (double)entry(p, op, q[0], q[1], q[2], q[3]);
    }
    return 0;
}

/* full rows of M_h^0 (or its alpha-derivative): rows holds n pairs (k, i);
 * out is n x nv, row-major */
int or_m0_rows(const or_problem* h, int deriv, long n, const int* rows, double* out, int nthreads)
{
    if (!h) return -1;
    const Prob* p = h->p;
    for (long e = 0; e < n; ++e)
        if (rows[2 * e] < 0 || rows[2 * e] >= p->nt || rows[2 * e + 1] < 0 || rows[2 * e + 1] >= p->ng) return -2;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    long ntask = n * (long)p->ntri;
    R* mom = (R*)malloc(sizeof(R) * 3 * (ntask > 0 ? ntask : 1));
#pragma omp parallel for schedule(dynamic, 1)
    for (long task = 0; task < ntask; ++task) {
        long e = task / p->ntri; int t = (int)(task % p->ntri);
        m0_triangle(p, rows[2 * e], rows[2 * e + 1], t, deriv, mom + 3 * task);
    }
    for (long e = 0; e < n; ++e) {
        R* acc = (R*)calloc(p->nv, sizeof(R));
        for (int t = 0; t < p->ntri; ++t)
            for (int v = 0; v < 3; ++v) acc[p->tri[3 * t + v]] += mom[3 * (e * p->ntri + t) + v];
        for (int v = 0; v < p->nv; ++v) out[e * p->nv + v] = (double)acc[v];
        free(acc);
    }
    free(mom);
    return 0;
}

/* the potentials of eq. (2) at n points (x, y, t), 0 < t: out is n x 3
 * (M~0 u0, V~ w, W g), so u = out0 + out1 - out2; u0 may be NULL */
int or_potential(const or_problem* h, long n, const double* pts, const double* w, const double* g,
                 const double* u0, double* out, int nthreads)
{
    if (!h || !w || !g) return -1;
    const Prob* p = h->p;
    for (long e = 0; e < n; ++e) if (!(pts[3 * e + 2] > 0)) return -2;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (long e = 0; e < n; ++e) {
        R r[3];
        potential(p, pts[3 * e], pts[3 * e + 1], pts[3 * e + 2], w, g, u0, r);
        for (int q = 0; q < 3; ++q) out[3 * e + q] = (double)r[q];
    }
    return 0;
}

/* pins of the scalar building blocks */
double or_e1(double z) { return (double)e1l(z); }
long double or_e1l(long double z) { return e1l(z); }

/* the exact time integral int_{tau_k} int_{tau_m} kappa(t - tau) for the
 * kernels: which = 0 V (F_V), 1 K (F_K), 2 D (F_D), 3 dV (F_dV/alpha), 4 E1 */
double or_time_integral(const or_problem* h, int which, double r, int k, int m)
{
    const Prob* p = h->p;
    TB b = time_block(p, k, m);
    R a = p->alpha * (R)r * (R)r / 4;
    int sep = b.d >= 2;
    switch (which) {
    case 0: return (double)(sep ? tquad(0, a, &b) : delta4(FV, a, &b));
    case 1: return (double)(sep ? tquad(1, a, &b) : delta4(FK, a, &b));
    case 2: return (double)(sep ? tquad(2, a, &b) : delta4(FD, a, &b));
    case 3: return (double)((sep ? tquad(3, a, &b) : delta4(FdV, a, &b)) / p->alpha);
    case 4: return (double)(sep ? tquad(4, a, &b) : delta4(FE, a, &b));
    }
    return NAN;
}

double or_m0_time(const or_problem* h, double r, int k, int deriv)
{
    return (double)m0_time(h->p, k, (R)r * (R)r, deriv);
}
