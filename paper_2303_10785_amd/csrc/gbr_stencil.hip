// Explicit wide-stencil form of the IG4 gradients of MIG4 (Eq. IG4_grads,
// read as differences, alpha = 5/14) and of the metric derivative and
// interface interpolation built on them (Sec. 7, Eq. FP-interp, FP-interp2).
//
// On the infinite line the left-hand side alpha E^-1 + 1 + alpha E has the
// inverse c_m = r^|m| / sqrt(1 - 4 alpha^2), r = (sqrt(1 - 4 alpha^2) - 1) /
// (2 alpha) ~ -0.420 (from the symbol 1 + 2 alpha cos t). The gradient is
// therefore the antisymmetric stencil f'_i = sum_j w_j (f_{i+j} - f_{i-j})
// with w_j = a (c_{j-1} - c_{j+1}) + b (c_{j-2} - c_{j+2}); |w_j| falls below
// 1e-18 by j = 48, so the truncated stencil equals the implicit scheme to
// FP64 rounding. On a periodic line it gives the cyclic solution, and on a
// line extended with a period shift (coordinates, coordinate products) the
// bounded infinite-line solution, with no separate treatment of the wrap.
#include <cmath>
#include <cstdlib>
#include <vector>

#include "gbr_internal.hpp"

namespace gbr {

const Ig4Stencil &ig4_stencil()
{
    static const Ig4Stencil s = [] {
        Ig4Stencil t{};
        const double al = 5.0 / 14.0;
        const double a = 2.0 * (2.0 + al) / 6.0, b = (4.0 * al - 1.0) / 12.0;
        const double q = std::sqrt(1.0 - 4.0 * al * al);
        const double r = (q - 1.0) / (2.0 * al);
        auto c = [&](int m) { return std::pow(r, std::abs(m)) / q; };
        for (int j = 1; j <= kIg4Half; ++j) t.w[j] = a * (c(j - 1) - c(j + 1)) + b * (c(j - 2) - c(j + 2));
        return t;
    }();
    return s;
}

const Ig4Rec &ig4_rec()
{
    static const Ig4Rec r = [] {
        Ig4Rec t{};
        const double al = 5.0 / 14.0;
        const double s = std::sqrt(1.0 - 4.0 * al * al);
        t.q = (1.0 - s) / (2.0 * al);
        t.K = 1.0 / s;
        t.a = 2.0 * (2.0 + al) / 6.0;
        t.b = (4.0 * al - 1.0) / 12.0;
        t.pw[0] = 1.0;
        for (int j = 1; j < 20; ++j) t.pw[j] = t.pw[j - 1] * (-t.q);
        return t;
    }();
    return r;
}

const Ig4MetricStencil &ig4_metric_stencil()
{
    static const Ig4MetricStencil s = [] {
        const Ig4Stencil &g = ig4_stencil();
        const int H = kIg4Half, R = H + 4;
        std::vector<double> I(2 * R + 1, 0.0);
        // coefficient arrays over offsets -R .. R relative to cell i
        auto add_delta = [&](int o, double sc) { I[R + o] += sc; };
        auto add_grad = [&](int k, double sc) {  // sc * f'_k
            for (int j = 1; j <= H; ++j) {
                I[R + k + j] += sc * g.w[j];
                I[R + k - j] -= sc * g.w[j];
            }
        };
        // I_{i+1/2} = 1/2 [(f_i + f'_i / 2 + f''_i / 12) + (f_{i+1} - f'_{i+1} / 2 + f''_{i+1} / 12)],
        // f''_k = 2 (f_{k+1} - 2 f_k + f_{k-1}) - (f'_{k+1} - f'_{k-1}) / 2
        add_delta(0, 0.5);
        add_delta(1, 0.5);
        add_grad(0, 0.25);
        add_grad(1, -0.25);
        for (int k = 0; k <= 1; ++k) {
            const double h = 0.5 / 12.0;
            add_delta(k + 1, 2.0 * h);
            add_delta(k, -4.0 * h);
            add_delta(k - 1, 2.0 * h);
            add_grad(k + 1, -0.5 * h);
            add_grad(k - 1, 0.5 * h);
        }
        Ig4MetricStencil t{};
        for (int m = -(H + 1); m <= H + 2; ++m) t.e[m + H + 1] = I[R + m];
        // D f_i = I_{i+1/2} - I_{i-1/2}: coefficient e_o - e_{o+1} at offset o,
        // antisymmetric about i
        for (int j = 1; j <= kIg4DHalf; ++j) {
            const double ej = (j <= H + 2) ? I[R + j] : 0.0;
            const double ej1 = (j + 1 <= H + 2) ? I[R + j + 1] : 0.0;
            t.d[j] = ej - ej1;
        }
        return t;
    }();
    return s;
}

}  // namespace gbr
