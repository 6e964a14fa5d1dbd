"""Synthetic transport coefficients for the fluid model (paper section 2.3).

The paper builds its lookup table from BOLSIG+ output for nitrogen at 1 bar;
those data are not available here, so the table is filled from smooth closed
forms of plausible magnitude instead: a mobility of 0.03-0.05 m^2/(V s), a
diffusion coefficient of 0.1-0.15 m^2/s, and Townsend's form
alpha = A p exp(-B p / E) for the ionisation coefficient with the textbook
constants for nitrogen (A = 12 /(cm Torr), B = 342 V/(cm Torr)) at 760 Torr.
The table layout is the paper's: entries at regularly spaced field strengths
up to emax (35 MV/m, 1000 entries by default), columns (mu, D, alpha)."""
import numpy as np

EMAX = 35e6


def synthetic_n2_table(ntab=1000, emax=EMAX):
    """[ntab][3] = (mu, D, alpha) at E = k * emax / (ntab - 1)."""
    E = np.linspace(0.0, emax, ntab)
    mu = 0.03 + 0.02 * np.exp(-E / 1e7)
    dif = 0.1 + 0.05 * E / emax
    with np.errstate(divide="ignore"):
        alpha = np.where(E > 0, 12.0 * 760.0 * 100.0 * np.exp(-342.0 * 760.0 * 100.0 / np.maximum(E, 1e-300)), 0.0)
    return np.stack([mu, dif, alpha], axis=1)


def constant_table(mu, dif, alpha, ntab=2, emax=EMAX):
    """A table with the same (mu, D, alpha) at every entry."""
    return np.tile(np.array([[mu, dif, alpha]], dtype=np.float64), (ntab, 1))
