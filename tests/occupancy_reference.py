"""Independent NumPy statement of the occupancy-weighted mean-field EAM (test helper).

Written for the tests from the paper, separately from the C oracle, to pin it:
App. B.2.1, Eqs. (EAM-Substitutional-ave) and (EAM-density-substitutional-ave),
with the Taylor embedding of App. B.2, Eq. (F_taylor_mxe), inside the free
energy of Sec. 2.1, Eq. (Grand-Canonical-Free-Energy).

Representation (deliberately unlike the oracle's site-type form): every site
carries a probability vector X[i, k] over the species k in (A, B, S), the molar
fractions x_ik of the paper; the vacancy / empty state is the missing mass
1 - sum_k X[i, k]. The energy is written over species pairs:
    E_pair = 1/2 sum_i sum_j sum_kl X_ik X_jl a_kl <g_phi^{c(k,l)}>_ij
    rho_i^(k) = sum_j sum_l X_jl b_l <g_f^{c(k,l)}>_ij       (density felt by k at i)
    E_emb = sum_i sum_k X_ik c_k [F(rho0) + F'(rho0)(rho_bar - rho0)],  F = -sqrt
with the radial-shape class c(k, l) = 1 when exactly one of k, l is the
interstitial solute S, 0 when neither is, and no interaction when both are.
E_vib = -3 kT sum_i w_i ln sigma_i with w_i = sum_k X_ik (the probability that
the site holds an atom), E_mix = kT sum_mobile [x ln x + (1 - x) ln(1 - x)].

Phase averages: the pair's relative coordinate is Gaussian with per-axis width
s = sqrt(sigma_i^2 + sigma_j^2); its average is taken with an n-point-per-axis
probabilists' Gauss-Hermite product rule from numpy (n = 3 is the rule the
method uses, larger n approximates the integral itself).

Every function accepts complex positions, widths and fractions, so derivatives
come from the complex step Im F(y + i h) / h (exact to rounding for these
analytic expressions; branch decisions use real parts).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.hermite_e import hermegauss

KB = 8.617333262e-5  # eV/K
HOST_VAC, ALLOY, INTERSTITIAL, HOST_FIXED = 0, 1, 2, 3
SA, SB, SS = 0, 1, 2


def species_fractions(types, x):
    """x_ik per site: the site type fixes which species its fraction x refers to."""
    n = len(types)
    X = np.zeros((n, 3), dtype=np.result_type(x, float))
    t = np.asarray(types)
    X[t == HOST_VAC, SA] = x[t == HOST_VAC]
    X[t == ALLOY, SA] = 1.0 - x[t == ALLOY]
    X[t == ALLOY, SB] = x[t == ALLOY]
    X[t == INTERSTITIAL, SS] = x[t == INTERSTITIAL]
    X[t == HOST_FIXED, SA] = 1.0
    return X


def shape_class(k, l):
    """Radial-shape class of a species pair: 0 host-host, 1 host-solute, None solute-solute."""
    s = (k == SS) + (l == SS)
    return None if s == 2 else s


def _shape(eam, r, cls, which):
    """g(r) = exp(-a (r / r_e - 1)) times the cosine taper; r may be complex."""
    re = eam["r_e"][cls]
    a = eam["alpha"][cls] if which == "phi" else eam["gamma"][cls]
    rs, rc = eam["r_s"], eam["r_c"]
    rr = np.real(r)
    S = np.where(rr <= rs, 1.0, 0.5 * (1.0 + np.cos(np.pi * (r - rs) / (rc - rs))))
    g = np.exp(-a * (r / re - 1.0)) * S
    return np.where(rr >= rc, 0.0, g)


def product_rule(n):
    """Nodes (m, 3) and weights (m,) of the n^3-point rule for a standard 3-D normal."""
    z, w = hermegauss(n)
    w = w / w.sum()
    Z = np.stack(np.meshgrid(z, z, z, indexing="ij"), -1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", w, w, w).ravel()
    return Z, W


def separations(q, box, periodic):
    """rbar_ij = q_j - q_i under the minimum image, shape (n, n, 3)."""
    d = q[None, :, :] - q[:, None, :]
    for a in range(3):
        if periodic[a]:
            d[..., a] -= box[a] * np.round(np.real(d[..., a]) / box[a])
    return d


def pair_tables(eam, q, sigma, box, periodic, n_rule=3, rows=None):
    """Per class c: <g_phi^c>, <g_f^c> and g_f^c(|rbar|) for the pairs (i, j), i != j.

    rows: optional list of site indices; then only those rows are computed
    (shape (len(rows), n)). Returns dict c -> (phi, f, f0)."""
    Z, W = product_rule(n_rule)
    d = separations(q, box, periodic)
    idx = np.arange(q.shape[0]) if rows is None else np.asarray(rows)
    d = d[idx]
    s = np.sqrt(sigma[idx][:, None] ** 2 + sigma[None, :] ** 2)
    self_mask = idx[:, None] == np.arange(q.shape[0])[None, :]
    out = {}
    r0 = np.sqrt((d ** 2).sum(-1) + self_mask)  # the diagonal is masked below
    dt = np.result_type(d, s, float)
    blk = max(1, (1 << 21) // max(1, d.shape[0] * d.shape[1]))  # nodes per vectorised block
    for c in (0, 1):
        phi = np.zeros(d.shape[:2], dtype=dt)
        f = np.zeros(d.shape[:2], dtype=dt)
        for b0 in range(0, len(W), blk):
            z, w = Z[b0:b0 + blk], W[b0:b0 + blk]
            dk = d[:, :, None, :] + s[:, :, None, None] * z[None, None, :, :]
            rk = np.sqrt((dk ** 2).sum(-1) + self_mask[:, :, None])
            phi = phi + _shape(eam, rk, c, "phi") @ w
            f = f + _shape(eam, rk, c, "f") @ w
        f0 = _shape(eam, r0, c, "f")
        out[c] = tuple(np.where(self_mask, 0.0, v) for v in (phi, f, f0))
    return out


def functional(eam, sys_, x=None, tables=None, q=None, sigma=None, n_rule=3):
    """Free energy and per-site pieces of a system. Returns a dict:
    F, e_site, rho_bar, rho0 (density felt by the site's host species; for an
    interstitial site, by the solute), E_pair, E_emb, E_vib, E_mix."""
    q = sys_.q if q is None else q
    sigma = sys_.sigma if sigma is None else sigma
    x = sys_.x if x is None else x
    T = sys_.T
    kT = KB * T
    if tables is None:
        tables = pair_tables(eam, q, sigma, sys_.box, sys_.periodic, n_rule)
    X = species_fractions(sys_.type, x)
    a = np.asarray(eam["pair_a"], dtype=float)
    b = np.asarray(eam["emit_b"], dtype=float)
    c = np.asarray(eam["embed_c"], dtype=float)
    n = X.shape[0]
    dt = np.result_type(X, tables[0][0])
    pair_site = np.zeros(n, dtype=dt)
    for k in range(3):
        for l in range(3):
            cl = shape_class(k, l)
            if cl is None or a[k, l] == 0.0:
                continue
            pair_site = pair_site + 0.5 * X[:, k] * (a[k, l] * tables[cl][0] @ X[:, l])
    # density felt by species k at each site
    rho_bar = np.zeros((n, 3), dtype=dt)
    rho0 = np.zeros((n, 3), dtype=dt)
    for k in range(3):
        for l in range(3):
            cl = shape_class(k, l)
            if cl is None:
                continue
            rho_bar[:, k] = rho_bar[:, k] + tables[cl][1] @ (b[l] * X[:, l])
            rho0[:, k] = rho0[:, k] + tables[cl][2] @ (b[l] * X[:, l])
    emb_site = np.zeros(n, dtype=dt)
    for k in range(3):
        if c[k] == 0.0:
            continue
        use = np.abs(X[:, k]) > 0
        if not np.any(use):
            continue
        r0 = np.where(use, rho0[:, k], 1.0)
        rb = np.where(use, rho_bar[:, k], 1.0)
        assert np.all(np.real(r0) > 0), "no density at an embedded site"
        G = -np.sqrt(r0) - 0.5 / np.sqrt(r0) * (rb - r0)
        emb_site = emb_site + np.where(use, X[:, k] * c[k] * G, 0.0)
    w = X.sum(1)
    vib_site = -3.0 * kT * w * np.log(sigma)
    mobile = np.asarray(sys_.type) != HOST_FIXED
    mix_site = np.zeros(n, dtype=dt)
    xm = x[mobile]
    t1 = np.where(np.real(xm) > 0, xm * np.log(np.where(np.real(xm) > 0, xm, 1.0)), 0.0)
    t0 = np.where(np.real(xm) < 1, (1 - xm) * np.log(np.where(np.real(xm) < 1, 1 - xm, 1.0)), 0.0)
    mix_site[mobile] = kT * (t1 + t0)
    e_site = pair_site + emb_site + vib_site + mix_site
    # the density reported per site: its host species' (A) for host sites, S for interstitials
    kk = np.where(np.asarray(sys_.type) == INTERSTITIAL, SS, SA)
    return dict(F=e_site.sum(), e_site=e_site, rho_bar=rho_bar[np.arange(n), kk],
                rho0=rho0[np.arange(n), kk], E_pair=pair_site.sum(), E_emb=emb_site.sum(),
                E_vib=vib_site.sum(), E_mix=mix_site.sum(), pair_site=pair_site,
                emb_site=emb_site)


def chemical_potentials(eam, sys_, h=1e-30, n_rule=3):
    """mu_i = d(F - E_mix)/dx_i by the complex step (0 on fixed host sites)."""
    tables = pair_tables(eam, sys_.q, sys_.sigma, sys_.box, sys_.periodic, n_rule)
    mu = np.zeros(sys_.n)
    for i in range(sys_.n):
        if sys_.type[i] == HOST_FIXED:
            continue
        x = sys_.x.astype(complex)
        x[i] += 1j * h
        r = functional(eam, sys_, x=x, tables=tables)
        mu[i] = np.imag(r["F"] - r["E_mix"]) / h
    return mu


def gradient(eam, sys_, sites, h=1e-30, n_rule=3):
    """dF/d(q_x, q_y, q_z, sigma) at the given sites by the complex step, shape (len, 4)."""
    base = pair_tables(eam, sys_.q, sys_.sigma, sys_.box, sys_.periodic, n_rule)
    out = np.zeros((len(sites), 4))
    for m, i in enumerate(sites):
        for a in range(4):
            q = sys_.q.astype(complex)
            sg = sys_.sigma.astype(complex)
            if a < 3:
                q[i, a] += 1j * h
            else:
                sg[i] += 1j * h
            row = pair_tables(eam, q, sg, sys_.box, sys_.periodic, n_rule, rows=[i])
            tab = {}
            for c in (0, 1):
                parts = []
                for v_base, v_row in zip(base[c], row[c]):
                    v = v_base.astype(complex)
                    v[i, :] = v_row[0]
                    v[:, i] = v_row[0]  # pair functions are symmetric in (i, j)
                    parts.append(v)
                tab[c] = tuple(parts)
            r = functional(eam, sys_, q=q, sigma=sg, tables=tab)
            out[m, a] = np.imag(r["F"]) / h
    return out
