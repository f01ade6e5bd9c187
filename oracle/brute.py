"""Numpy brute-force twin of the oracle for tiny maps (test infrastructure only).

It scans every pixel of the map and follows the paper's main-text vector
definitions instead of Appendix A:
  - sky basis p, theta_hat, phi_hat (Sec. 2, equations p_sky_basis and
    tangent_sky_basis) and the antenna basis rotated by psi0
    (equation antenna_base_vectors);
  - antenna coordinates from k = sin(rho) cos(sigma) theta'_0 +
    sin(rho) sin(sigma) phi'_0 + cos(rho) p_0, i.e. x' = k.theta'_0,
    y' = k.phi'_0, z' = k.p_0, rho = atan2(|(x', y')|, z'), sigma = atan2(y', x');
  - co-polarisation by Ludwig's third definition (Appendix A):
    e_co = cos(sigma - zeta) rho_hat - sin(sigma - zeta) sigma_hat, with
    rho_hat = cos(rho) cos(sigma) theta'_0 + cos(rho) sin(sigma) phi'_0 - sin(rho) p_0
    (the printed rho_hat carries sin(rho) sin(sigma) on phi'_0, which is not a
    unit vector; the cos(rho) form is the derivative of k along rho);
  - chi = signed angle from the pixel's theta_hat to e_co, measured toward
    its phi_hat (Sec. 2, equation psi, taken with its sign);
  - d = N sum_k D(chi) Lambda(chi) B_k Lambda(-chi) S_k with 4x4 matrices.
Pixel centres are an input (the caller supplies them).
"""
from __future__ import annotations

import numpy as np


def sky_basis(theta, phi):
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    p = np.stack([st * cp, st * sp, ct], -1)
    th = np.stack([ct * cp, ct * sp, -st], -1)
    ph = np.stack([-sp, cp, np.zeros_like(np.asarray(theta, dtype=float))], -1)
    return p, th, ph


def antenna_coords(theta0, phi0, psi0, theta, phi):
    """(rho, sigma, x', y', z') of directions (theta, phi) for pointing (theta0, phi0, psi0)."""
    p0, t0, f0 = sky_basis(theta0, phi0)
    tp = np.cos(psi0) * t0 + np.sin(psi0) * f0
    fp = -np.sin(psi0) * t0 + np.cos(psi0) * f0
    n, _, _ = sky_basis(theta, phi)
    x, y, z = n @ tp, n @ fp, n @ p0
    return np.arctan2(np.hypot(x, y), z), np.arctan2(y, x), x, y, z


def chi_ludwig3(theta0, phi0, psi0, zeta, theta, phi):
    """chi from the Ludwig-3 co-polar vector (with the unit-norm rho_hat)."""
    p0, t0, f0 = sky_basis(theta0, phi0)
    tp = np.cos(psi0) * t0 + np.sin(psi0) * f0
    fp = -np.sin(psi0) * t0 + np.cos(psi0) * f0
    rho, sig, _, _, _ = antenna_coords(theta0, phi0, psi0, theta, phi)
    cr, sr, cs, ss = np.cos(rho), np.sin(rho), np.cos(sig), np.sin(sig)
    rho_hat = (cr * cs)[..., None] * tp + (cr * ss)[..., None] * fp - sr[..., None] * p0
    sig_hat = -ss[..., None] * tp + cs[..., None] * fp
    a = sig - zeta
    e = np.cos(a)[..., None] * rho_hat - np.sin(a)[..., None] * sig_hat
    _, th, ph = sky_basis(theta, phi)
    return np.arctan2(np.sum(e * ph, -1), np.sum(e * th, -1))


def bilinear(grid, T, u, v):
    """grid (n, n, ...) over [-T, T]^2, row-major [iv][iu]; zero outside."""
    n = grid.shape[0]
    h = 2.0 * T / (n - 1)
    tu, tv = (u + T) / h, (v + T) / h
    inside = (tu >= 0) & (tu <= n - 1) & (tv >= 0) & (tv <= n - 1)
    iu = np.clip(np.floor(tu).astype(np.int64), 0, n - 2)
    iv = np.clip(np.floor(tv).astype(np.int64), 0, n - 2)
    fu, fv = tu - iu, tv - iv
    extra = (1,) * (grid.ndim - 2)
    fu_, fv_ = fu.reshape(fu.shape + extra), fv.reshape(fv.shape + extra)
    out = ((1 - fu_) * (1 - fv_) * grid[iv, iu] + fu_ * (1 - fv_) * grid[iv, iu + 1]
           + (1 - fu_) * fv_ * grid[iv + 1, iu] + fu_ * fv_ * grid[iv + 1, iu + 1])
    out[~inside] = 0.0
    return out


def lambda_mat(x):
    c, s = np.cos(2 * x), np.sin(2 * x)
    L = np.zeros(np.shape(x) + (4, 4))
    L[..., 0, 0] = 1
    L[..., 1, 1] = c
    L[..., 1, 2] = -s
    L[..., 2, 1] = s
    L[..., 2, 2] = c
    L[..., 3, 3] = 1
    return L


def tod(pix_theta, pix_phi, I, Q, U, beamsor, T, zeta, eps, s, rho_min, rho_max, norm_mode, norm_scale,
        theta, phi, psi, out_mode=0):
    """Brute-force TOD (out_mode 0) or Stokes pickup of B_TT (out_mode 1)."""
    S = np.stack([I, Q, U, np.zeros_like(I)], -1)
    res = []
    for t0, f0, s0 in zip(np.atleast_1d(theta), np.atleast_1d(phi), np.atleast_1d(psi)):
        rho, sig, x, y, z = antenna_coords(t0, f0, s0, pix_theta, pix_phi)
        sel = z >= np.cos(rho_max)
        if rho_min > 0:
            sel &= z < np.cos(rho_min)
        idx = np.nonzero(sel)[0]
        chi = chi_ludwig3(t0, f0, s0, zeta, pix_theta[idx], pix_phi[idx])
        M = bilinear(beamsor, T, x[idx] / z[idx], y[idx] / z[idx])
        rs = np.einsum("kab,kb->ka", lambda_mat(-chi), S[idx])
        nsum = M[:, 0, 0].sum()
        N = norm_scale / nsum if norm_mode == 1 else norm_scale
        if out_mode == 1:
            res.append(N * (M[:, 0, 0][:, None] * rs[:, :3]).sum(0))
            continue
        ls = np.einsum("kab,kb->ka", lambda_mat(chi), np.einsum("kab,kb->ka", M, rs))
        D = 0.5 * s * np.stack([np.full_like(chi, 1 + eps), (1 - eps) * np.cos(2 * chi),
                                (1 - eps) * np.sin(2 * chi), np.zeros_like(chi)], -1)
        res.append(N * np.sum(D * ls))
    return np.array(res)
