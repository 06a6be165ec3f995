// Initial density fields (Sec. 4.3, density initialization): the triply
// periodic minimal-surface families P, D, G (gyroid) and IWP, written from
// their standard trigonometric level-set approximations, and the centre ball
// (a solid cube with a spherical void at its centre).  Host code: it runs once
// before the design loop.
//
// Element e = (i,j,k) is evaluated at its centre, X = 2 pi (i + 1/2) / n (and
// Y, Z likewise).  The elements with the smallest level-set values are solid
// (density 1), exactly round(vf n^3) of them (ties broken by the flat index),
// the rest void (density 0; a context clamps it to rho_min on entry).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "opentm_amd.h"

namespace {

double level(int kind, double X, double Y, double Z, double cx, double cy, double cz) {
    switch (kind) {
        case OTM_INIT_P: return std::cos(X) + std::cos(Y) + std::cos(Z);
        case OTM_INIT_D:
            return std::cos(X) * std::cos(Y) * std::cos(Z) - std::sin(X) * std::sin(Y) * std::sin(Z);
        case OTM_INIT_G: return std::sin(X) * std::cos(Y) + std::sin(Y) * std::cos(Z) + std::sin(Z) * std::cos(X);
        case OTM_INIT_IWP:
            return 2.0 * (std::cos(X) * std::cos(Y) + std::cos(Y) * std::cos(Z) + std::cos(Z) * std::cos(X)) -
                   (std::cos(2.0 * X) + std::cos(2.0 * Y) + std::cos(2.0 * Z));
        default:  // centre ball: the farthest elements from the centre are solid
            return -std::sqrt(cx * cx + cy * cy + cz * cz);
    }
}

}  // namespace

extern "C" int otm_init_density(int32_t n, int32_t kind, double vf, double* rho_out) {
    if (!rho_out || n < 4 || n > 1024 || !(vf > 0.0 && vf <= 1.0)) return OTM_EINVAL;
    if (kind < OTM_INIT_P || kind > OTM_INIT_BALL) return OTM_EINVAL;
    const int64_t nn = (int64_t)n * n * n;
    std::vector<double> phi((size_t)nn);
    const double two_pi = 2.0 * std::acos(-1.0);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const double X = two_pi * (i + 0.5) / n, Y = two_pi * (j + 0.5) / n, Z = two_pi * (k + 0.5) / n;
                const double cx = (i + 0.5) - 0.5 * n, cy = (j + 0.5) - 0.5 * n, cz = (k + 0.5) - 0.5 * n;
                phi[(size_t)(i + (int64_t)n * (j + (int64_t)n * k))] = level(kind, X, Y, Z, cx, cy, cz);
            }
    const int64_t solid = std::llround(vf * (double)nn);
    std::vector<int64_t> order((size_t)nn);
    std::iota(order.begin(), order.end(), (int64_t)0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return phi[(size_t)a] < phi[(size_t)b]; });
    for (int64_t e = 0; e < nn; ++e) rho_out[e] = 0.0;
    for (int64_t r = 0; r < solid; ++r) rho_out[order[(size_t)r]] = 1.0;
    return OTM_OK;
}
