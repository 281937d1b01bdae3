"""FP64 reverse sweep through the unrolled SF iterations (oracle adjoint).

TEST INFRASTRUCTURE ONLY (see oracle/sf.py).  The paper differentiates the L
unrolled applications of the fixed-point operator T (Sec. "Fixed-Point
Representation"; the warm-start loss eq. NN_loss; "Differentiability" in the
Appendix).  This module writes that reverse pass out by hand, step by step
through the same literal quantities the forward oracle computes: the alpha step
(atan2), the d step (clip at 1), e, the s step, r_1, r_2, the lambda step and
the KKT solve.

Differentiated outputs and their cotangents:
  xi_bar^L, lambda^L                  g_xi_bar, g_lam
  ||r_1(xi_bar^L)||, ||r_2(xi_bar^L)|| g_res1, g_res2 (norm gradients are 0 at 0)
  sum_l L_FP^l, L_FP^l = ||z^{l+1} - z^l||^2 (R5)     weight fp_weight
Inputs receiving gradients: the flow sample xi, xi_bar^0, lambda^0.

Non-smooth points follow the forward tie conventions (R12): d = 1 exactly and
x exactly on a box bound are inactive, atan2(0, 0) has zero derivative.

3D (dim=3, reading Q1): the chain runs through the alpha step (atan2 of the
horizontal components), the beta step (atan2 of the scaled horizontal and
vertical components), the spheroid direction u(alpha, beta) and the clipped
least-squares d step, in that order; everything after e is the planar chain
with three axis blocks.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .sf import SFOracle, split_axes


def _e_vjp(dx, dy, size, g_ex, g_ey):
    """Cotangent of (dx, dy) given that of e = size*d*(cos alpha, sin alpha),
    alpha = atan2(dy, dx), d = max(1, (dx cos alpha + dy sin alpha)/size)."""
    rr = dx * dx + dy * dy
    safe = np.where(rr > 0.0, rr, 1.0)
    da_dx = np.where(rr > 0.0, -dy / safe, 0.0)
    da_dy = np.where(rr > 0.0, dx / safe, 0.0)
    alpha = np.arctan2(dy, dx)
    ca, sa = np.cos(alpha), np.sin(alpha)
    d_unc = (dx * ca + dy * sa) / size
    d = np.maximum(1.0, d_unc)
    # d_unc depends on dx, dy directly and through alpha
    tang = (-dx * sa + dy * ca) / size
    dd_dx = ca / size + tang * da_dx
    dd_dy = sa / size + tang * da_dy
    pass_d = d_unc >= 1.0                       # tie -> the unclipped branch
    dd_dx = np.where(pass_d, dd_dx, 0.0)
    dd_dy = np.where(pass_d, dd_dy, 0.0)
    # e_x = size d cos a, e_y = size d sin a
    g_d = size * (g_ex * ca + g_ey * sa)
    g_a = size * d * (-g_ex * sa + g_ey * ca)
    g_dx = g_d * dd_dx + g_a * da_dx
    g_dy = g_d * dd_dy + g_a * da_dy
    return g_dx, g_dy


def _e3_vjp(dx, dy, dz, a, b, g_ex, g_ey, g_ez):
    """Cotangent of Delta = (dx, dy, dz) given that of e - centre = d u(alpha,
    beta), u = (a cos(alpha) sin(beta), a sin(alpha) sin(beta), b cos(beta)),
    with alpha = atan2(dy, dx), beta = atan2(rho_xy / a, dz / b), rho_xy =
    dx cos(alpha) + dy sin(alpha), and d = max(1, <Delta, u> / <u, u>)."""
    rr = dx * dx + dy * dy
    safe = np.where(rr > 0.0, rr, 1.0)
    alpha = np.arctan2(dy, dx)
    ca, sa = np.cos(alpha), np.sin(alpha)
    rho_xy = dx * ca + dy * sa
    Y, X = rho_xy / a, dz / b
    beta = np.arctan2(Y, X)
    cb, sb = np.cos(beta), np.sin(beta)
    ux, uy, uz = a * ca * sb, a * sa * sb, b * cb
    num = dx * ux + dy * uy + dz * uz
    den = ux * ux + uy * uy + uz * uz
    d_unc = num / den
    d = np.maximum(1.0, d_unc)
    # e = d u
    g_d = g_ex * ux + g_ey * uy + g_ez * uz
    g_ux, g_uy, g_uz = d * g_ex, d * g_ey, d * g_ez
    # d = max(1, num / den); the tie d_unc = 1 takes the unclipped branch
    pass_d = d_unc >= 1.0
    g_num = np.where(pass_d, g_d / den, 0.0)
    g_den = np.where(pass_d, -g_d * num / (den * den), 0.0)
    g_dx, g_dy, g_dz = g_num * ux, g_num * uy, g_num * uz
    g_ux = g_ux + g_num * dx + 2.0 * g_den * ux
    g_uy = g_uy + g_num * dy + 2.0 * g_den * uy
    g_uz = g_uz + g_num * dz + 2.0 * g_den * uz
    # u(alpha, beta)
    g_alpha = a * sb * (-g_ux * sa + g_uy * ca)
    g_beta = a * cb * (g_ux * ca + g_uy * sa) - b * sb * g_uz
    # beta = atan2(Y, X), zero derivative at (0, 0)
    r2 = X * X + Y * Y
    safe2 = np.where(r2 > 0.0, r2, 1.0)
    g_Y = np.where(r2 > 0.0, g_beta * X / safe2, 0.0)
    g_X = np.where(r2 > 0.0, -g_beta * Y / safe2, 0.0)
    g_dz = g_dz + g_X / b
    g_rho = g_Y / a
    # rho_xy = dx cos(alpha) + dy sin(alpha)
    g_dx = g_dx + g_rho * ca
    g_dy = g_dy + g_rho * sa
    g_alpha = g_alpha + g_rho * (-dx * sa + dy * ca)
    # alpha = atan2(dy, dx), zero derivative at (0, 0)
    g_dx = g_dx + np.where(rr > 0.0, -dy / safe, 0.0) * g_alpha
    g_dy = g_dy + np.where(rr > 0.0, dx / safe, 0.0) * g_alpha
    return g_dx, g_dy, g_dz


@dataclass
class SFGrad:
    g_xi: np.ndarray
    g_xi0: np.ndarray
    g_lam0: np.ndarray


class SFAdjoint:
    def __init__(self, orc: SFOracle):
        self.o = orc

    def _geometry(self, q):
        """Split F xi_bar into pair differences and obstacle offsets per axis."""
        o = self.o
        R = o.ops.n_pair_rows + o.ops.n_obs_rows
        comp = split_axes(q, R, o.dim)
        Pr = o.ops.n_pair_rows
        pair = [comp[ax][:Pr] for ax in range(o.dim)]
        obs = [comp[ax][Pr:] - o.obs_cen[ax] for ax in range(o.dim)]
        return pair, obs

    def _eT(self, q, g_e):
        """J_E(q)^T g_e for e(q) stacked like F's rows."""
        o = self.o
        R = o.ops.n_pair_rows + o.ops.n_obs_rows
        Pr = o.ops.n_pair_rows
        pair, obs = self._geometry(q)
        g = split_axes(g_e, R, o.dim)
        out = [np.zeros(R) for _ in range(o.dim)]
        if o.dim == 2:
            res_p = _e_vjp(*pair, o.a, *(gq[:Pr] for gq in g))
            res_o = _e_vjp(*obs, o.obs_ao, *(gq[Pr:] for gq in g)) if o.ops.M > 0 else None
        else:
            res_p = _e3_vjp(*pair, o.a, o.robot_b, *(gq[:Pr] for gq in g))
            res_o = _e3_vjp(*obs, o.obs_ao[0], o.obs_ao[1], *(gq[Pr:] for gq in g)) \
                if o.ops.M > 0 else None
        for ax in range(o.dim):
            out[ax][:Pr] = res_p[ax]
            if res_o is not None:
                out[ax][Pr:] = res_o[ax]
        return np.concatenate(out)

    def gradient(self, xi, xi0, lam0, n_iters, g_xi_bar, g_lam, g_res1=0.0,
                 g_res2=0.0, fp_weight=0.0) -> SFGrad:
        o = self.o
        F, G, rho, h = o.ops.F, o.ops.G, o.rho, o.h
        xi = o.flat(xi)
        res = o.solve(xi, xi0, lam0, n_iters, keep_iterates=True)
        its = res.iterates
        g_xib = o.flat(g_xi_bar).copy()
        g_l = o.flat(g_lam).copy()
        g_xi = np.zeros_like(xi)
        # residual outputs of xi_bar^L
        xL = its[-1][0]
        r1, r2, e, s, _ = o.residual_terms(xL)
        n1, n2 = np.linalg.norm(r1), np.linalg.norm(r2)
        if g_res1 != 0.0 and n1 > 0.0:
            g_r1 = g_res1 * r1 / n1
            g_q = g_r1 - self._eT(F @ xL, g_r1)
            g_xib += F.T @ g_q
        if g_res2 != 0.0 and n2 > 0.0:
            g_r2 = g_res2 * r2 / n2
            gx = G @ xL
            g_xib += G.T @ (g_r2 * np.where(h - gx > 0.0, 0.0, 1.0))
        Sz = o.Sz
        for l in range(n_iters - 1, -1, -1):
            xib, lam = its[l]
            xib1, lam1 = its[l + 1]
            g_xib_prev_fp = np.zeros_like(xib)
            g_lam_prev_fp = np.zeros_like(lam)
            if fp_weight != 0.0:
                dxi, dla = xib1 - xib, lam1 - lam
                g_xib = g_xib + 2.0 * fp_weight * dxi
                g_l = g_l + 2.0 * fp_weight * dla
                g_xib_prev_fp = -2.0 * fp_weight * dxi
                g_lam_prev_fp = -2.0 * fp_weight * dla
            # xi_bar^{l+1} = top block of K^{-1} [eta; b]
            sol = sla.lu_solve(o.K_lu, np.concatenate([g_xib, np.zeros(o.K.shape[0] - Sz)]),
                               trans=1)
            g_eta = sol[:Sz]
            # eta = rho F^T e + lambda^{l+1} + xi + rho G^T (h - s)
            g_lam1 = g_l + g_eta
            if o.objective == "projection":
                g_xi += g_eta                         # the sample enters eta only there
            g_e = rho * (F @ g_eta)
            g_s = -rho * (G @ g_eta) if o.include_G else np.zeros(G.shape[0])
            # lambda^{l+1} = lambda^l - rho F^T r_1 - rho G^T r_2
            g_lam_l = g_lam1.copy()
            g_r1 = -rho * (F @ g_lam1)
            g_r2 = -rho * (G @ g_lam1)
            # recompute the step's intermediates at xi_bar^l
            q = F @ xib
            gx = G @ xib
            # r_2 = G xi_bar - h + s
            g_gx = g_r2.copy()
            g_s = g_s + g_r2
            # r_1 = F xi_bar - e
            g_q = g_r1.copy()
            g_e = g_e - g_r1
            # s = max(0, h - G xi_bar)
            g_gx -= g_s * (h - gx > 0.0)
            # e = e(alpha(q), d(q))
            g_q += self._eT(q, g_e)
            g_xib = F.T @ g_q + G.T @ g_gx + g_xib_prev_fp
            g_l = g_lam_l + g_lam_prev_fp
        return SFGrad(o.shaped(g_xi), o.shaped(g_xib), o.shaped(g_l))


def loss_value(orc: SFOracle, xi, xi0, lam0, n_iters, w_xi, w_lam, w_res1=0.0,
               w_res2=0.0, fp_weight=0.0) -> float:
    """<w_xi, xi_bar^L> + <w_lam, lambda^L> + w_res1 ||r1|| + w_res2 ||r2||
    + fp_weight * sum_l L_FP^l: a scalar whose gradient is gradient()'s output
    for cotangents (w_xi, w_lam, w_res1, w_res2)."""
    res = orc.solve(xi, xi0, lam0, n_iters, keep_iterates=fp_weight != 0.0)
    val = float(np.sum(orc.flat(w_xi) * orc.flat(res.xi_bar))
                + np.sum(orc.flat(w_lam) * orc.flat(res.lam))
                + w_res1 * res.res_r1 + w_res2 * res.res_r2)
    if fp_weight != 0.0:
        fp = 0.0
        for (a0, l0), (a1, l1) in zip(res.iterates[:-1], res.iterates[1:]):
            fp += np.sum((a1 - a0) ** 2) + np.sum((l1 - l0) ** 2)
        val += fp_weight * fp
    return val
