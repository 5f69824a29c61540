// Host post-processing of the stepper's results: Richardson extrapolation
// of second-order waveforms over three resolutions and the error estimate
// from two extrapolants (Section 2.3, item 3; Section 5.1, footnote).
#include <cmath>

#include "tk_internal.h"

extern "C" tk_status tk_richardson(const double *w1, const double *w2, const double *w3, long n, int order,
                                   double *extrap, double *err)
{
    if (!w1 || !w2 || !w3 || n < 0 || order < 1 || order > 16) return TK_E_INVALID;
    const double q = std::ldexp(1.0, order);
    const double inv = 1.0 / (q - 1.0);
    tk_status st = TK_OK;
    for (long k = 0; k < n; ++k) {
        const double *a = w1 + 2 * k, *b = w2 + 2 * k, *c = w3 + 2 * k;
        if (!std::isfinite(a[0]) || !std::isfinite(a[1]) || !std::isfinite(b[0]) || !std::isfinite(b[1]) ||
            !std::isfinite(c[0]) || !std::isfinite(c[1]))
            st = TK_E_NONFINITE;
        // the two extrapolants: from the coarse pair and from the fine pair
        const double r12re = (q * b[0] - a[0]) * inv, r12im = (q * b[1] - a[1]) * inv;
        const double r23re = (q * c[0] - b[0]) * inv, r23im = (q * c[1] - b[1]) * inv;
        if (extrap) {
            extrap[2 * k] = r23re;
            extrap[2 * k + 1] = r23im;
        }
        if (err) {
            const double d = std::hypot(r23re - r12re, r23im - r12im);
            const double m = std::hypot(r23re, r23im);
            err[k] = m > 0.0 ? d / m : d;
        }
    }
    return st;
}
