// Host build of the kernels' special functions (stbem_math.h is written
// __host__ __device__ so that its arithmetic can be exercised on the CPU):
// reads z values from stdin, writes z, E1(z), e^{-z} (from E1's path),
// Ein(z) and exp_neg(z) with 17 significant digits.
#include "stbem_tables.h"
#include <cstdio>

int main()
{
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
