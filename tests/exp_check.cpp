// CPU check of the kernels' FP64 exponential exp_cw (hrlb_math.h, the same source the kernels
// compile): its error in units in the last place against the long-double exponential, on seeded
// samples over [-700, 700], near zero and around the half-ulp boundaries of the reduction
// (x = (k + 1/2) ln 2), plus the exact and limiting values.  Exit status 0 when every error is
// within 1 ulp and the special values hold.
#include <cmath>
#include <cstdio>
#include <random>

#include "hrlb_math.h"

static int fails = 0;
static double worst = 0.0, worst_x = 0.0;

static void ulp_check(double x)
{
    const long double ref = expl((long double)x);
    const double r = (double)ref;
    const double u = std::nextafter(r, INFINITY) - r;
    const double y = hrlb::exp_cw(x);
    const double e = (double)(fabsl((long double)y - ref) / (long double)u);
    if (!(e <= worst)) {
        worst = e;
        worst_x = x;
    }
}

int main()
{
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> wide(-700.0, 700.0), unit(-1.0, 1.0), tiny(-1e-6, 1e-6);
    for (int i = 0; i < 1000000; ++i) ulp_check(wide(g));
    for (int i = 0; i < 500000; ++i) ulp_check(unit(g));
    for (int i = 0; i < 100000; ++i) ulp_check(tiny(g));
    const double ln2 = 0.6931471805599453;
    for (int k = -1000; k <= 1000; ++k)
        for (int d = -4; d <= 4; ++d) {
            const double x = (k + 0.5) * ln2;
            double y = x;
            for (int s = 0; s < (d < 0 ? -d : d); ++s) y = std::nextafter(y, d < 0 ? -INFINITY : INFINITY);
            if (std::fabs(y) < 700.0) ulp_check(y);
        }
    std::printf("worst error %.3f ulp at x = %.17g\n", worst, worst_x);
    if (!(worst <= 1.0)) ++fails;
    // exact and limiting values
    if (hrlb::exp_cw(0.0) != 1.0) { std::printf("exp(0) != 1\n"); ++fails; }
    if (!std::isinf(hrlb::exp_cw(710.0))) { std::printf("exp(710) is not inf\n"); ++fails; }
    if (hrlb::exp_cw(-746.0) != 0.0) { std::printf("exp(-746) != 0\n"); ++fails; }
    if (!std::isnan(hrlb::exp_cw(NAN))) { std::printf("exp(nan) is not nan\n"); ++fails; }
    return fails ? 1 : 0;
}
