"""Richardson extrapolation of second-order results, written out plainly.

TEST INFRASTRUCTURE (see oracle/__init__.py): only tests/ and bench.py's
CPU legs use it; the product path never imports it.

Section 2.3, item 3: the code's second-order numerical solutions are
Richardson-extrapolated to lower the discretisation error.  Section 5.1,
footnote: the error estimate is the relative difference between the
waveform's Richardson extrapolant computed two different ways.

Readings (stated in the design notes): three results at spacings h, h/2,
h/4 (grid spacings and time step scaled together); the leading error of the
scheme is of order p = 2, so a result u(h) = u* + C h^p + ... gives the
extrapolant (2^p u(h/2) - u(h)) / (2^p - 1); the "two different ways" are
the extrapolants of the coarse pair (h, h/2) and of the fine pair (h/2, h/4),
the second being the extrapolated result.
"""
import numpy as np


def extrapolant(coarse, fine, order=2):
    """Eliminate the C h^order term between results at h (coarse) and h/2
    (fine): solve u(h) = u* + C h^p, u(h/2) = u* + C (h/2)^p for u*."""
    coarse = np.asarray(coarse, np.complex128)
    fine = np.asarray(fine, np.complex128)
    ratio = 2.0 ** order  # u(h) - u* = ratio * (u(h/2) - u*)
    return (ratio * fine - coarse) / (ratio - 1.0)


def richardson(w1, w2, w3, order=2):
    """Extrapolated result from the fine pair, and the relative difference
    between the two extrapolants (the error estimate)."""
    r_coarse_pair = extrapolant(w1, w2, order)
    r_fine_pair = extrapolant(w2, w3, order)
    diff = np.abs(r_fine_pair - r_coarse_pair)
    mag = np.abs(r_fine_pair)
    err = np.where(mag > 0, diff / np.where(mag > 0, mag, 1.0), diff)
    return r_fine_pair, err
