"""Stable Neo-Hookean hyperelasticity (oracle, float64).

The paper uses the stable Neo-Hookean model of Smith et al. 2018 for every
solid (Sec. 7, caption of Table 1) but prints no formula.  Reading taken:

    Psi(F) = mu/2 (|F|_F^2 - 3) - mu (J - 1) + lam/2 (J - 1)^2,   J = det F

with mu = mu_L and lam = lam_L + mu_L from Young's modulus E and Poisson
ratio nu, so that linearising at F = I gives exactly linear elasticity with
(E, nu):  dP = mu_L (dF + dF^T) + lam_L tr(dF) I.

    P(F)      = mu F + (lam (J - 1) - mu) cof F
    dP[dF]    = mu dF + lam (cof F : dF) cof F + (lam (J - 1) - mu) dcof[dF]

where cof F = J F^-T has columns (f1 x f2, f2 x f0, f0 x f1) for the columns
f0, f1, f2 of F.  All functions broadcast over leading axes.
"""
import numpy as np


def lame(E, nu):
    """(mu, lam) of the energy above from (E, nu)."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    mu_l = E / (2.0 * (1.0 + nu))
    lam_l = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu_l, lam_l + mu_l


def cof(F):
    """Cofactor matrix: columns are cross products of the other two columns."""
    f0, f1, f2 = F[..., :, 0], F[..., :, 1], F[..., :, 2]
    return np.stack([np.cross(f1, f2), np.cross(f2, f0), np.cross(f0, f1)], axis=-1)


def dcof(F, dF):
    """Directional derivative of cof at F along dF."""
    f0, f1, f2 = F[..., :, 0], F[..., :, 1], F[..., :, 2]
    d0, d1, d2 = dF[..., :, 0], dF[..., :, 1], dF[..., :, 2]
    return np.stack([np.cross(d1, f2) + np.cross(f1, d2),
                     np.cross(d2, f0) + np.cross(f2, d0),
                     np.cross(d0, f1) + np.cross(f0, d1)], axis=-1)


def _b(a, F):
    """Broadcast per-element scalars against trailing 3x3 matrix axes."""
    return np.asarray(a, dtype=np.float64)[..., None, None]


def psi(F, mu, lam):
    J = np.linalg.det(F)
    I2 = np.einsum("...ij,...ij->...", F, F)
    return 0.5 * mu * (I2 - 3.0) - mu * (J - 1.0) + 0.5 * lam * (J - 1.0) ** 2


def stress(F, mu, lam):
    """First Piola-Kirchhoff stress P = dPsi/dF."""
    J = np.linalg.det(F)
    return _b(mu, F) * F + _b(lam * (J - 1.0) - mu, F) * cof(F)


def dstress(F, dF, mu, lam):
    """dP[dF], the second derivative of Psi applied to dF."""
    J = np.linalg.det(F)
    C = cof(F)
    CdF = np.einsum("...ij,...ij->...", C, dF)
    return (_b(mu, F) * dF + _b(lam * CdF, F) * C + _b(lam * (J - 1.0) - mu, F) * dcof(F, dF))
