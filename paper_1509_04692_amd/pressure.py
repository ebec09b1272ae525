"""Pressure of hard particles in NVT from the contact value of the pair
distribution (Sec. 4, Table 1): sample the number of pairs in thin shells
just outside contact with ``System.pair_histogram``, normalise by the
ideal-gas count of each shell, fit the shell values and extrapolate to
contact.  For hard disks of diameter sigma the virial theorem gives

    beta P / rho = 1 + (pi / 2) rho sigma^2 g(sigma+),   P* = beta P sigma^2,

and for hard spheres beta P / rho = 1 + (2 pi / 3) rho sigma^3 g(sigma+).

For particles with shape the paper uses volume perturbations (Sec. 4): shrink
the box (every separation) by a factor 1 - s; C(s), the number of pairs that
then overlap, grows linearly at small s, and since the volume shrinks by
about dim * s * V, beta P / rho = 1 + C'(0) / (dim N).  The counts come from
``System.scale_counts``; C'(0) is the intercept of a polynomial fit of
C(s) / s.  This is host-side arithmetic on the sampled counts; the counts
come from the library's kernels.
"""
import math

import numpy as np


def shell_measure(edges2, dim):
    """Area (2D) or volume (3D) of each shell between consecutive radii."""
    e = np.asarray(edges2, dtype=np.float64)
    if dim == 2:
        return math.pi * np.diff(e)
    r = np.sqrt(e)
    return 4.0 * math.pi / 3.0 * np.diff(r ** 3)


def shell_g(edges2, mean_counts, N, L, dim=2):
    """g(r) averaged over each shell: mean pair count / ideal-gas pair count."""
    ideal = 0.5 * N * (N - 1) * shell_measure(edges2, dim) / float(L) ** dim
    return np.asarray(mean_counts, dtype=np.float64) / ideal


def contact_value(edges2, mean_counts, N, L, sigma, dim=2, degree=2, n_samples=None):
    """Extrapolate the shell averages of g to r = sigma by a least-squares
    polynomial in r through the shell midpoints (weights from Poisson
    counting errors when n_samples is given).  Returns (g_contact, r_mid, g)."""
    e = np.asarray(edges2, dtype=np.float64)
    r = np.sqrt(e)
    r_mid = 0.5 * (r[:-1] + r[1:])
    g = shell_g(e, mean_counts, N, L, dim)
    w = None
    if n_samples:
        counts = np.maximum(np.asarray(mean_counts, dtype=np.float64) * n_samples, 1.0)
        w = np.sqrt(counts) / g  # 1 / relative error of each shell value
    coef = np.polynomial.polynomial.polyfit(r_mid - sigma, g, degree, w=w)
    return float(coef[0]), r_mid, g


def disk_pressure(N, L, sigma, g_contact):
    """Reduced pressure P* = beta P sigma^2 of N hard disks in an L x L box."""
    rho_s2 = N * sigma * sigma / (L * L)
    return rho_s2 * (1.0 + 0.5 * math.pi * rho_s2 * g_contact)


def sphere_pressure(N, L, sigma, g_contact):
    """beta P sigma^3 of N hard spheres in an L^3 box."""
    rho_s3 = N * sigma ** 3 / L ** 3
    return rho_s3 * (1.0 + 2.0 * math.pi / 3.0 * rho_s3 * g_contact)


def scale_slope(scales, mean_counts, degree=2, n_samples=None):
    """C'(0) from mean overlap counts C(s) at scale factors s > 0: intercept
    of a least-squares polynomial in s through C(s) / s (weights from
    Poisson counting errors when n_samples is given)."""
    s = np.asarray(scales, dtype=np.float64)
    c = np.asarray(mean_counts, dtype=np.float64)
    if np.any(s <= 0.0):
        raise ValueError("scale factors must be positive")
    w = None
    if n_samples:
        w = s * np.sqrt(np.maximum(c * n_samples, 1.0)) / np.maximum(c, 1e-300)
    coef = np.polynomial.polynomial.polyfit(s, c / s, degree, w=w)
    return float(coef[0])


def scale_pressure(N, dim, scales, mean_counts, degree=2, n_samples=None):
    """beta P / rho of N hard particles from volume-perturbation counts."""
    return 1.0 + scale_slope(scales, mean_counts, degree, n_samples) / (dim * N)
