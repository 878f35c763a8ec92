"""Analytic data and expected time derivatives for the oracle pins.

Everything here is derived from the ADM (3+1) equations of a vacuum
spacetime and from the Z4 constraint-damping system, NOT from the conformal
(W, gt, At, Gt) right-hand side that the oracle implements.  Derivatives of the
analytic fields are exact to rounding (forward-mode autodiff in float64 on
the CPU), so the only difference from the oracle's discrete operator is the
finite-difference truncation error, which must shrink as h^4.

Relations used (Z = Theta = 0 in the data, beta = 0 unless stated):
    d_t gamma_ij = -2 alpha K_ij
    d_t K_ij     = -D_i D_j alpha + alpha (R_ij - 2 K_ik K^k_j + K K_ij)
    d_t Theta    = alpha H / 2,        H = R + K^2 - K_ij K^ij      (Z4)
    d_t Z_i      = alpha M_i,          M_i = D_j K^j_i - d_i K       (Z4)
    Khat = K - 2 Theta,  Gt^i = -d_j gt^ij + 2 gt^ij Z_j             (Z4c variables)
and the conformal variables of paper Sec. 2.1.1:
    W = det(gamma)^-1/6, gt = W^2 gamma, At = W^2 (K_ij - gamma_ij K / 3).
"""
from __future__ import annotations

import numpy as np
import torch
from torch.func import jacfwd, vmap

DT = torch.float64
SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def _det3(m):
    """Determinant by cofactor expansion (plain tensor ops, safe under vmap+jacfwd)."""
    return (m[0, 0] * (m[1, 1] * m[2, 2] - m[1, 2] * m[2, 1])
            - m[0, 1] * (m[1, 0] * m[2, 2] - m[1, 2] * m[2, 0])
            + m[0, 2] * (m[1, 0] * m[2, 1] - m[1, 1] * m[2, 0]))


def _inv3(m):
    """Inverse by the adjugate (plain tensor ops, safe under vmap+jacfwd)."""
    c = torch.stack([
        torch.stack([m[1, 1] * m[2, 2] - m[1, 2] * m[2, 1], m[0, 2] * m[2, 1] - m[0, 1] * m[2, 2],
                     m[0, 1] * m[1, 2] - m[0, 2] * m[1, 1]]),
        torch.stack([m[1, 2] * m[2, 0] - m[1, 0] * m[2, 2], m[0, 0] * m[2, 2] - m[0, 2] * m[2, 0],
                     m[0, 2] * m[1, 0] - m[0, 0] * m[1, 2]]),
        torch.stack([m[1, 0] * m[2, 1] - m[1, 1] * m[2, 0], m[0, 1] * m[2, 0] - m[0, 0] * m[2, 1],
                     m[0, 0] * m[1, 1] - m[0, 1] * m[1, 0]]),
    ])
    return c / _det3(m)


def _sym6(m):
    return torch.stack([m[a, b] for a, b in SYM])


def _christoffel(gam_fn):
    dgam = jacfwd(gam_fn)  # [a, b, c] = d_c gamma_ab

    def chris(x):
        g = gam_fn(x)
        gi = _inv3(g)
        dg = dgam(x)
        low = 0.5 * (dg.permute(0, 2, 1) + dg - dg.permute(2, 0, 1))  # Gamma_kij
        return torch.einsum("kl,lij->kij", gi, low)

    return chris


def conformal_state_fn(prim):
    """prim(x) -> (gamma, K_ij, alpha, beta^i, B^i) ; returns x -> 25-vector."""

    def gt_inv(x):
        g = prim(x)[0]
        W = _det3(g) ** (-1.0 / 6.0)
        return _inv3(W * W * g)

    dgt_inv = jacfwd(gt_inv)  # [i, j, m] = d_m gt^ij

    def state(x):
        g, K, a, b, B = prim(x)
        gi = _inv3(g)
        W = _det3(g) ** (-1.0 / 6.0)
        trK = torch.einsum("ij,ij->", gi, K)
        gt = W * W * g
        At = W * W * (K - g * trK / 3.0)
        Gt = -torch.einsum("ijj->i", dgt_inv(x))
        z = torch.zeros(1, dtype=DT)
        return torch.cat([W.reshape(1), _sym6(gt), trK.reshape(1), _sym6(At), Gt, z, a.reshape(1), b, B])

    return state


def adm_expected_fn(prim):
    """x -> 25-vector of d_t of every field for beta = 0, Theta = Z = 0 data
    (rows 19-24, the shift and B, are returned as 0 and not used)."""
    gam = lambda x: prim(x)[0]
    Kf = lambda x: prim(x)[1]
    alf = lambda x: prim(x)[2]
    chris = _christoffel(gam)
    dchris = jacfwd(chris)  # [k, i, j, m] = d_m Gamma^k_ij
    hess_a = jacfwd(jacfwd(alf))
    grad_a = jacfwd(alf)

    def Kmix(x):
        return _inv3(gam(x)) @ Kf(x)  # K^k_j

    dKmix = jacfwd(Kmix)  # [k, j, m]

    def pieces(x):
        g, K, a = gam(x), Kf(x), alf(x)
        gi = _inv3(g)
        G = chris(x)
        dG = dchris(x)
        Ric = (torch.einsum("kijk->ij", dG) - torch.einsum("kikj->ij", dG)
               + torch.einsum("kkl,lij->ij", G, G) - torch.einsum("kjl,lik->ij", G, G))
        DDa = hess_a(x) - torch.einsum("kij,k->ij", G, grad_a(x))
        Km = gi @ K
        trK = torch.trace(Km)
        dtg = -2.0 * a * K
        dtK = -DDa + a * (Ric - 2.0 * K @ Km + trK * K)
        W = _det3(g) ** (-1.0 / 6.0)
        dtW = W * a * trK / 3.0
        dtgt = W * W * dtg + 2.0 * W * dtW * g
        return g, K, a, gi, Ric, Km, trK, dtg, dtK, W, dtW, dtgt

    def dtgt_inv(x):
        g, K, a, gi, Ric, Km, trK, dtg, dtK, W, dtW, dtgt = pieces(x)
        gti = gi / (W * W)
        return -gti @ dtgt @ gti

    d_dtgt_inv = jacfwd(dtgt_inv)  # [i, j, m]

    def expected(x):
        g, K, a, gi, Ric, Km, trK, dtg, dtK, W, dtW, dtgt = pieces(x)
        G = chris(x)
        dKm = dKmix(x)
        divK = torch.einsum("kjk->j", dKm) + torch.einsum("kkl,lj->j", G, Km) - torch.einsum("lkj,kl->j", G, Km)
        dtrK = torch.einsum("kkj->j", dKm)
        M = divK - dtrK
        R = torch.einsum("ij,ij->", gi, Ric)
        KK = torch.trace(Km @ Km)
        H = R + trK * trK - KK
        dt_trK = -torch.trace(gi @ dtg @ gi @ K) + torch.einsum("ij,ij->", gi, dtK)
        dtTh = 0.5 * a * H
        dtKh = dt_trK - 2.0 * dtTh
        dtAt = 2.0 * W * dtW * (K - g * trK / 3.0) + W * W * (dtK - dtg * trK / 3.0 - g * dt_trK / 3.0)
        gti = gi / (W * W)
        dtGt = -torch.einsum("ijj->i", d_dtgt_inv(x)) + 2.0 * a * gti @ M
        dta = -2.0 * a * trK
        z3 = torch.zeros(3, dtype=DT)
        return torch.cat([dtW.reshape(1), _sym6(dtgt), dtKh.reshape(1), _sym6(dtAt), dtGt, dtTh.reshape(1),
                          dta.reshape(1), z3, z3])

    return expected


def adm_constraints_fn(prim):
    """x -> [H, M^x, M^y, M^z] of the ADM data: H = R + K^2 - K_ij K^ij,
    M^i = gamma^ij (D_k K^k_j - d_j K) (vacuum, paper Sec. 2.3)."""
    gam = lambda x: prim(x)[0]
    Kf = lambda x: prim(x)[1]
    chris = _christoffel(gam)
    dchris = jacfwd(chris)

    def Kmix(x):
        return _inv3(gam(x)) @ Kf(x)

    dKmix = jacfwd(Kmix)

    def cons(x):
        g, K = gam(x), Kf(x)
        gi = _inv3(g)
        G = chris(x)
        dG = dchris(x)
        Ric = (torch.einsum("kijk->ij", dG) - torch.einsum("kikj->ij", dG)
               + torch.einsum("kkl,lij->ij", G, G) - torch.einsum("kjl,lik->ij", G, G))
        Km = gi @ K
        trK = torch.trace(Km)
        H = torch.einsum("ij,ij->", gi, Ric) + trK * trK - torch.trace(Km @ Km)
        dKm = dKmix(x)
        divK = torch.einsum("kjk->j", dKm) + torch.einsum("kkl,lj->j", G, Km) - torch.einsum("lkj,kl->j", G, Km)
        M = gi @ (divK - torch.einsum("kkj->j", dKm))
        return torch.cat([H.reshape(1), M, torch.zeros(21, dtype=DT)])

    return cons


def evaluate(fn, grid, only_active=False) -> np.ndarray:
    """Evaluate x -> 25-vector on the stored (or active) points of a grid;
    returns (25, Nz, Ny, Nx) (zeros off the active set if only_active)."""
    X, Y, Z = grid.coords()
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    mask = grid.active_mask().ravel() if only_active else np.ones(len(pts), bool)
    out = np.zeros((len(pts), 25))
    sel = np.nonzero(mask)[0]
    xs = torch.tensor(pts[sel], dtype=DT)
    vals = []
    for c in range(0, len(xs), 4096):
        vals.append(vmap(fn)(xs[c:c + 4096]).detach().numpy())
    out[sel] = np.concatenate(vals)
    return np.ascontiguousarray(out.T.reshape((25,) + X.shape))


# ---------------------------------------------------------------------------
# Analytic spacetimes
# ---------------------------------------------------------------------------

def generic_prim(eps=0.1):
    """A smooth, non-symmetric, time-dependent (non-stationary) vacuum-style
    data set: gamma = delta + eps h(x), K_ij = eps k(x), alpha = 1 + eps a(x),
    beta = B = 0.  It does not satisfy the constraints, which is the point:
    the Z4c right-hand side is compared with the ADM+Z4 evolution of the same
    data, including the constraint-addition terms."""

    def prim(x):
        X, Y, Z = x[0], x[1], x[2]
        s, c = torch.sin, torch.cos
        h = torch.stack([
            torch.stack([s(X + 2 * Y) , 0.3 * c(Y - Z), 0.2 * s(X * Z)]),
            torch.stack([0.3 * c(Y - Z), c(2 * X - Z), 0.25 * s(Y + Z)]),
            torch.stack([0.2 * s(X * Z), 0.25 * s(Y + Z), s(X) * c(Y) + 0.5 * c(Z)]),
        ])
        k = torch.stack([
            torch.stack([c(X - Y), 0.4 * s(Z + X), 0.3 * c(Y)]),
            torch.stack([0.4 * s(Z + X), s(2 * Y) * c(Z), -0.2 * c(X + Z)]),
            torch.stack([0.3 * c(Y), -0.2 * c(X + Z), s(X + Y - Z)]),
        ])
        g = torch.eye(3, dtype=DT) + eps * h
        K = eps * k
        a = 1.0 + eps * s(X + 0.5 * Y) * c(Z - Y)
        z3 = torch.zeros(3, dtype=DT)
        return g, K, a, z3, z3

    return prim


def kerr_schild_prim(M=1.0, B_amp=0.1):
    """Schwarzschild in Kerr-Schild coordinates (stationary, with shift):
    gamma = delta + 2H l l, H = M/r, alpha = (1+2H)^-1/2,
    beta^i = 2H l^i / (1+2H), K_ij = (D_i beta_j + D_j beta_i) / (2 alpha).
    B^i is an arbitrary smooth field (it only enters the gauge rows)."""

    def base(x):
        r = torch.sqrt(torch.sum(x * x))
        H = M / r
        l = x / r
        g = torch.eye(3, dtype=DT) + 2.0 * H * torch.outer(l, l)
        a = (1.0 + 2.0 * H) ** -0.5
        b_low = 2.0 * H * l
        return g, a, b_low

    gam = lambda x: base(x)[0]
    blow = lambda x: base(x)[2]
    chris = _christoffel(gam)
    dblow = jacfwd(blow)  # [j, i] = d_i beta_j

    def prim(x):
        g, a, bl = base(x)
        r = torch.sqrt(torch.sum(x * x))
        G = chris(x)
        Db = dblow(x).T - torch.einsum("kij,k->ij", G, bl)  # [i, j] = D_i beta_j
        K = (Db + Db.T) / (2.0 * a)
        bu = _inv3(g) @ bl
        B = B_amp * x / r / (1.0 + r)
        return g, K, a, bu, B

    return prim


def kerr_schild_gauge_expected_fn(prim, eta=0.36, shift_coeff=0.75):
    """Closed forms of the gauge rows on stationary data with shift
    (paper Sec. 2.1.1 gauge equations; Theta = 0 so K = Khat):
        d_t alpha  = beta.d alpha - 2 alpha Khat
        d_t beta^i = beta.d beta^i + 0.75 B^i
        d_t B^i    = beta.d B^i + [(d_t - beta.d) Gt^i] - eta B^i,
    and stationarity (d_t Gt = 0) gives (d_t - beta.d) Gt^i = -beta.d Gt^i."""
    state = conformal_state_fn(prim)
    dstate = jacfwd(state)  # [f, m]

    def expected(x):
        s = state(x)
        ds = dstate(x)
        bu = s[19:22]
        adv = ds @ bu
        dta = adv[18] - 2.0 * s[18] * s[7]
        dtb = adv[19:22] + shift_coeff * s[22:25]
        dtB = adv[22:25] - adv[14:17] - eta * s[22:25]
        return torch.cat([torch.zeros(18, dtype=DT), dta.reshape(1), dtb, dtB])

    return expected


def brill_lindquist_prim(masses=(0.5, 0.5), centres=((5.0, 0.0, 0.0), (-5.0, 0.0, 0.0))):
    """gamma = psi^4 delta, K = 0, alpha = psi^-2, beta = B = 0."""
    cs = [torch.tensor(c, dtype=DT) for c in centres]

    def prim(x):
        psi = 1.0 + sum(m / (2.0 * torch.sqrt(torch.sum((x - c) ** 2))) for m, c in zip(masses, cs))
        g = psi ** 4 * torch.eye(3, dtype=DT)
        z3 = torch.zeros(3, dtype=DT)
        return g, torch.zeros(3, 3, dtype=DT), psi ** -2.0, z3, z3

    return prim


# ---------------------------------------------------------------------------
# Shift terms of the Gt equation with Z != 0
# ---------------------------------------------------------------------------

def shifted_z_prim(eps=0.1, beps=0.2):
    """generic_prim's metric, curvature and lapse with a smooth non-zero
    shift beta^i(x) (B = 0)."""
    base = generic_prim(eps)

    def prim(x):
        g, K, a, _, B = base(x)
        X, Y, Z = x[0], x[1], x[2]
        s, c = torch.sin, torch.cos
        b = beps * torch.stack([s(Y + 0.5 * Z) + 0.3, c(X - Z) * 0.7, s(X + Y) * c(Z)])
        return g, K, a, b, B

    return prim


def zt_field(zeps=0.05):
    """A smooth vector field Zt^i(x) standing for (Gt^i - Gt_d^i)/2 (a
    constraint violation carried by the evolved Gt)."""

    def zt(x):
        X, Y, Z = x[0], x[1], x[2]
        s, c = torch.sin, torch.cos
        return zeps * torch.stack([c(2 * X + Y), s(Y - Z) + 0.5, c(X) * s(2 * Z)])

    return zt


def conformal_state_with_z_fn(prim, zt):
    """conformal_state_fn(prim) with Gt^i = Gt_d^i + 2 Zt^i (Gt_d = -d_j gt^ij)."""
    st = conformal_state_fn(prim)

    def state(x):
        u = st(x)
        return torch.cat([u[:14], u[14:17] + 2.0 * zt(x), u[17:]])

    return state


def gt_shift_part_fn(prim, zt, kappa3):
    """x -> 25-vector holding, in rows 14-16, the part of d_t Gt^i that
    depends on the shift, from geometric objects differentiated exactly:
      -d_j (L_beta gt^ij)  +  2 (beta^k d_k Zt^i + kappa3 (Zt^i d_k beta^k 2/3 - Zt^k d_k beta^i)).
    L_beta gt_ij = beta^k d_k gt_ij + gt_ik d_j beta^k + gt_jk d_i beta^k - (2/3) gt_ij d_k beta^k is
    the Lie derivative of the weight -2/3 density gt_ij; with det gt = 1,
    Gt_d^i = -d_j gt^ij, so the first term is the shift part of d_t Gt_d.
    For kappa3 = 1 the second is twice the Lie derivative of the weight 2/3
    vector density Zt^i (the transport of the constraint violation by the
    shift); for kappa3 = 0 only its advection."""
    def gt_low(x):
        g = prim(x)[0]
        W = _det3(g) ** (-1.0 / 6.0)
        return W * W * g

    dgt = jacfwd(gt_low)  # [i, j, k] = d_k gt_ij
    beta = lambda x: prim(x)[3]
    dbeta = jacfwd(beta)  # [i, k] = d_k beta^i
    dzt = jacfwd(zt)

    def lie_gt_inv(x):
        gt = gt_low(x)
        gti = _inv3(gt)
        b = beta(x)
        db = dbeta(x)
        div = torch.trace(db)
        lie = (torch.einsum("k,ijk->ij", b, dgt(x)) + gt @ db + (gt @ db).T - (2.0 / 3.0) * gt * div)
        return -gti @ lie @ gti  # L_beta of gt^ij

    d_lie = jacfwd(lie_gt_inv)  # [i, j, m]

    def expected(x):
        b = beta(x)
        db = dbeta(x)
        z = zt(x)
        dz = dzt(x)  # [i, k] = d_k Zt^i
        part = -torch.einsum("ijj->i", d_lie(x)) + 2.0 * (dz @ b + kappa3 * ((2.0 / 3.0) * z * torch.trace(db)
                                                                              - db @ z))
        out = torch.zeros(25, dtype=DT)
        return torch.cat([out[:14], part, out[17:]])

    return expected
