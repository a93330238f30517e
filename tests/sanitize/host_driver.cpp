// Driver of the CPU-only sanitizer build of the host runtime: the library's
// Fourier CFL analysis over every option, and crkfr_create's refusals of
// bad configurations (no device call is made on those paths).
#include <cmath>
#include <cstdio>
#include <cstring>

#include "../../include/crkfr.h"

int main()
{
    int fails = 0;
    // a subset of the options (each analysis is a bisection over 4096 wave
    // numbers, slow under the sanitizers): every N, and each option once
    const int opts[][4] = {{0, 1, 0, 0}, {0, 0, 0, 0}, {2, 1, 1, 0}, {3, 1, 2, 1}, {1, 1, 0, 0}};
    for (int N = 1; N <= 4; ++N)
        for (const auto& o : opts) {
            const int stages = o[0], system = o[1], diss = o[2], points = o[3];
            const double c = crkfr_fourier_cfl(N, stages, system, diss, points, 1e-10);
            const bool bad_args = stages == 1;
            if (bad_args ? c != -1.0 : !(c > 0.0 && c < 2.0)) {
                std::printf("cfl N=%d stages=%d system=%d diss=%d points=%d -> %g\n", N, stages, system, diss,
                            points, c);
                ++fails;
            }
        }
    if (crkfr_fourier_cfl(0, 0, 1, 0, 0, 1e-10) != -1.0 || crkfr_fourier_cfl(5, 0, 1, 0, 0, 1e-10) != -1.0) ++fails;
    crkfr_solver* s = nullptr;
    if (crkfr_create(nullptr, nullptr, &s) != CRKFR_EINVAL) ++fails;
    crkfr_config base;
    std::memset(&base, 0, sizeof(base));
    base.equation = CRKFR_EULER2D;
    base.N = 3;
    base.nx = 8;
    base.ny = 8;
    base.x1 = 1.0;
    base.y1 = 1.0;
    base.gamma = 1.4;
    struct Case { const char* what; void (*edit)(crkfr_config&); } cases[] = {
        {"N = 0", [](crkfr_config& c) { c.N = 0; }},
        {"N = 5", [](crkfr_config& c) { c.N = 5; }},
        {"equation", [](crkfr_config& c) { c.equation = 9; }},
        {"nx = 0", [](crkfr_config& c) { c.nx = 0; }},
        {"1D ny", [](crkfr_config& c) { c.equation = CRKFR_EULER1D; c.ny = 3; }},
        {"dtype", [](crkfr_config& c) { c.dtype = 7; }},
        {"points", [](crkfr_config& c) { c.points = 4; }},
        {"bc kind", [](crkfr_config& c) { c.bc[2] = 9; }},
        {"periodic pair", [](crkfr_config& c) { c.bc[0] = CRKFR_BC_OUTFLOW; }},
        {"wall on advection", [](crkfr_config& c) { c.equation = CRKFR_LINADV1D; c.ny = 1; c.bc[0] = c.bc[1] = CRKFR_BC_REFLECT; }},
        {"domain", [](crkfr_config& c) { c.x1 = c.x0; }},
        {"2^31 nodes", [](crkfr_config& c) { c.nx = 11586; c.ny = 11586; }},
    };
    for (const Case& k : cases) {
        crkfr_config c = base;
        k.edit(c);
        s = nullptr;
        const int rc = crkfr_create(&c, nullptr, &s);
        if (rc != CRKFR_EINVAL || s != nullptr || std::strlen(crkfr_last_error()) == 0) {
            std::printf("create(%s) -> %d\n", k.what, rc);
            ++fails;
        }
    }
    crkfr_destroy(nullptr);
    std::printf("sanitized host runtime checks done, %d failures\n", fails);
    return fails ? 1 : 0;
}
