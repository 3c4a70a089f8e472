// Host build of the kernels' special functions (stbem_math.h is written
// __host__ __device__ so that its arithmetic can be exercised on the CPU).
// Default mode: reads z values from stdin, writes z, E1(z), e^{-z} (from E1's
// path), Ein(z) and exp_neg(z) with 17 significant digits.
// "series" mode: reads lines t0 t1 t2 t3 a (time elements [t0, t1] and
// [t2, t3], separated) and writes the series values of the block
// (Delta F_V, Delta F_K, Delta F_D, d/da and d2/da2 of Delta F_V) and the
// number of terms, or nan when the block is not a series block.
// "touch" mode: reads lines d t0 t1 t2 a (d = 0: the element [t0, t1] with
// itself; d = 1: [t1, t2] after [t0, t1]) and writes the closed forms of
// the touching block (Delta F_V, Delta F_K, Delta F_D, d/dalpha Delta F_V at
// alpha = 1, the four-point sum of E1).
#include "stbem_tables.h"
#include <cmath>
#include <cstdio>
#include <cstring>

int main(int argc, char** argv)
{
    if (argc > 1 && std::strcmp(argv[1], "series") == 0) {
        double t[4], a;
        while (std::scanf("%lf %lf %lf %lf %lf", &t[0], &t[1], &t[2], &t[3], &a) == 5) {
            stbem::Geom g = {};
            g.nt = 3; g.alpha = 1.0; g.t = t;
            static stbem::TimeBlock tb;
            stbem::time_block(g, 2, 0, tb);
            if (!tb.ser) { std::printf("nan nan nan nan nan 0\n"); continue; }
            const stbem::SeriesVals r = stbem::series<true, true, true, true>(tb, a);
            std::printf("%.17e %.17e %.17e %.17e %.17e %d\n", r.v, r.k, r.dd, r.va, r.vaa, tb.nterm);
        }
        return 0;
    }
    if (argc > 1 && std::strcmp(argv[1], "touch") == 0) {
        int d;
        double t[3], a;
        while (std::scanf("%d %lf %lf %lf %lf", &d, &t[0], &t[1], &t[2], &a) == 5) {
            stbem::Geom g = {};
            g.nt = 2; g.alpha = 1.0; g.t = t;
            static stbem::TimeBlock tb;
            stbem::time_block(g, d, 0, tb);
            const stbem::TouchVals r = stbem::touch<true, true, true, true, true>(tb, a, 1.0);
            std::printf("%.17e %.17e %.17e %.17e %.17e\n", r.v, r.k, r.dd, r.dv, r.e);
        }
        return 0;
    }
    static stbem::Tables T;
    stbem::build_tables(T);
    double z;
    while (std::scanf("%lf", &z) == 1) {
        double ex;
        const double e = stbem::e1t<true>(z, ex);
        std::printf("%.17e %.17e %.17e %.17e %.17e\n", z, e, ex, stbem::ein(z), stbem::exp_neg(z, T.ex2));
    }
    return 0;
}
