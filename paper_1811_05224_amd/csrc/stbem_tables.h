// Host-side construction of the quadrature tables used by the kernels.
#pragma once
#include <math.h>
#include "stbem_math.h"
#include "loggauss_table.h"

namespace stbem {

// Gauss-Legendre rules on [0,1], n = 1..kMaxGL: Newton iteration on P_n in
// long double from the asymptotic initial guess.
inline void build_tables(Tables& T)
{
    for (int n = 0; n <= kMaxGL; ++n)
        for (int i = 0; i < kMaxGL; ++i) T.gl_x[n][i] = T.gl_w[n][i] = 0.0;
    for (int n = 1; n <= kMaxGL; ++n) {
        for (int i = 0; i < n; ++i) {
            long double x = cosl(3.14159265358979323846264L * (i + 0.75L) / (n + 0.5L)), dp = 1;
            for (int it = 0; it < 60; ++it) {
                long double p0 = 1, p1 = x;
                for (int k = 2; k <= n; ++k) { long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k; p0 = p1; p1 = p2; }
                dp = n * (x * p1 - p0) / (x * x - 1);
                long double dx = p1 / dp;
                x -= dx;
                if (fabsl(dx) < 1e-20L) break;
            }
            long double p0 = 1, p1 = x;
            for (int k = 2; k <= n; ++k) { long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k; p0 = p1; p1 = p2; }
            dp = n * (x * p1 - p0) / (x * x - 1);
            T.gl_x[n][n - 1 - i] = (double)(0.5L * (1 + x));
            T.gl_w[n][n - 1 - i] = (double)(1.0L / ((1 - x * x) * dp * dp));
        }
    }
    for (int n = 0; n <= kMaxLog; ++n)
        for (int i = 0; i < kMaxLog; ++i) { T.lg_x[n][i] = kLogGaussX[n][i]; T.lg_w[n][i] = kLogGaussW[n][i]; }
    for (int j = 0; j < 64; ++j) T.ex2[j] = kEx2[j];
}

}  // namespace stbem

namespace stbem {

inline Orders default_orders()
{
    Orders o;
    o.q_sing = 12;
    o.q_log = 6;
    const int q[kNearClasses] = {12, 10, 8, 6, 5, 4};
    const double cut[kNearClasses - 1] = {1.5, 3.0, 6.0, 12.0, 24.0};
    for (int c = 0; c < kNearClasses; ++c) o.q_near[c] = q[c];
    for (int c = 0; c + 1 < kNearClasses; ++c) o.eta_cut[c] = cut[c];
    o.eta_raw = 4.0;
    o.q_tol = 1e-15;
    o.z_floor = 18.42;    // ln 1e8
    return o;
}

}  // namespace stbem
