"""CPU oracle of the instrument pipeline of Sect. 2.8.4 (absorption table,
ARF x RMF fine response, down-sampling matrix DS, combined response) and of
the Poisson likelihood with a background term (Sect. 6).

TEST INFRASTRUCTURE.  Only the test-suite may use this module; it shares no
code with the library.

Readings:
* Interp(x; xp, fp) is piecewise-linear interpolation through the nodes,
  constant beyond the first and last node (so the hat functions of the
  model energy grid sum to one everywhere);
* DS[i, e] is the integral of hat function i (1 at model energy i, 0 at
  the other model energies) over the fine bin [E_lo[e], E_hi[e]], computed
  exactly by splitting the bin at the model energies;
* the absorption table gives the transmission at a reference column
  N_H_ref; at column N_H it is the table value to the power N_H / N_H_ref,
  the same as exp(-N_H sigma) with sigma = -ln(transmission) / N_H_ref;
* the combined response without absorption is
  RSP[i, c] = sum_e DS[i, e] A[e] R[e, c] (cm^2 keV when the flux is per
  keV); absorption stays a separate factor exp(-N_H sigma_i) so that N_H
  remains a parameter;
* background: expected counts per (phase, channel) bin are the model counts
  plus given background counts b[k, c]; logL = sum d ln(m + b) - (m + b)
  - ln d!.
"""
from __future__ import annotations

import numpy as np
from scipy.special import gammaln


def interp(x, xp, fp):
    """Linear interpolation, constant beyond the end nodes."""
    return np.interp(x, xp, fp)


def hat_integral(e_model, i, a, b):
    """Integral over [a, b] of the piecewise-linear function that is 1 at
    e_model[i] and 0 at the other nodes (constant beyond the ends)."""
    xp = np.asarray(e_model, dtype=np.float64)
    fp = np.zeros(xp.size)
    fp[i] = 1.0
    cuts = np.concatenate([[a], xp[(xp > a) & (xp < b)], [b]])
    vals = interp(cuts, xp, fp)
    # the function is linear between consecutive cuts: trapezoids are exact
    return float(np.sum(0.5 * (vals[1:] + vals[:-1]) * np.diff(cuts)))


def ds_matrix(e_model, e_lo, e_hi):
    n, m = len(e_model), len(e_lo)
    ds = np.zeros((n, m))
    for i in range(n):
        for e in range(m):
            ds[i, e] = hat_integral(e_model, i, e_lo[e], e_hi[e])
    return ds


def response(e_model, e_lo, e_hi, area, matrix):
    """RSP[i, c] = sum_e DS[i, e] A[e] R[e, c]."""
    ds = ds_matrix(e_model, e_lo, e_hi)
    rf = np.asarray(area, dtype=np.float64)[:, None] * np.asarray(matrix, dtype=np.float64)
    return ds @ rf


def sigma_from_table(e_tab, att_tab, nh_ref, e_model):
    """Cross-section per H atom at the model energies from a transmission
    table at column nh_ref [cm^-2]."""
    return -np.log(interp(e_model, e_tab, att_tab)) / nh_ref


def loglike_with_background(counts, background, data):
    m = np.asarray(counts, dtype=np.float64) + np.asarray(background, dtype=np.float64)
    d = np.asarray(data, dtype=np.float64)
    if np.any((m <= 0) & (d > 0)):
        return -np.inf
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(d > 0, d * np.log(np.where(m > 0, m, 1.0)), 0.0)
    return float(np.sum(t - m - gammaln(d + 1.0)))
