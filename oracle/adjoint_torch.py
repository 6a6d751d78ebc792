"""FP64 gradient reference for the IDIC step -- TEST INFRASTRUCTURE ONLY.

A plain PyTorch (CPU, float64) restatement of the step the C oracle takes
(``tfsph_oracle.c``), written with whole-array operations so that autograd
can differentiate the dust-density misfit

    L = (1 / N_d) sum_j (rho_d,j(T) - target_j)^2,   rho_d,j = sum_k m_k W(|x_j - x_k|, h)

with respect to log t_stop and the initial velocities of both phases.  The
cell of every particle and the neighbour pairs within 2h are taken from the
detached positions of each step and held fixed (they are piecewise constant
in the inputs, so they carry no derivative).

Step (Section 2.3, eqs. 17-21; same readings as the C oracle):
  rho_a = sum_b m_b W(r_ab)                    summation density, gas only
  A_a   = -sum_b m_b (P_a + P_b) grad_a W_ab    P = c_s^2 / rho  (isothermal)
  v~ = v + tau (A + g),  u~ = u + tau g
  per cell: eps = M_d / M_g, beta = tau / t_stop, alpha = eps beta
            (drag coefficient K held constant: alpha = tau K V / M_g, beta = tau K V / M_d
            for the cell volume V, and the scalar parameter is log(1/K); Epstein law
            t*_stop = T_E / rho*_g: alpha = tau M_d / (V T_E), beta = tau M_g / (V T_E), the
            scalar parameter being log T_E),
            V* = ((1+beta) V~ + alpha U~) / D,  U* = (beta V~ + (1+alpha) U~) / D,  D = 1 + alpha + beta
  v = (v~ + alpha U*) / (1 + alpha),  u = (u~ + beta V*) / (1 + beta)   (alpha = beta = 0 in one-phase cells)
  x += tau v
Only the isothermal EOS without artificial viscosity is covered.
"""
from __future__ import annotations

import math

import numpy as np
import torch

_SIGMA = {1: 2.0 / 3.0, 2: 10.0 / (7.0 * math.pi), 3: 1.0 / math.pi}


def _f(q):
    t = 2.0 - q
    return torch.where(q < 1.0, 1.0 - 1.5 * q * q + 0.75 * q ** 3, torch.where(q < 2.0, 0.25 * t ** 3, 0.0 * q))


def _df(q):
    t = 2.0 - q
    return torch.where(q < 1.0, -3.0 * q + 2.25 * q * q, torch.where(q < 2.0, -0.75 * t * t, 0.0 * q))


def _box(p):
    lo = np.array(p.lo[:p.dim], dtype=np.float64)
    L = np.array([p.hi[k] - p.lo[k] for k in range(p.dim)], dtype=np.float64)
    return lo, L


def _cells(p, x):
    """Linear cell index of detached positions x (n, d): floor((x - lo) / Delta), periodic."""
    lo, L = _box(p)
    D = L / np.array(p.n_cells[:p.dim])
    c = np.floor((x - lo) / D).astype(np.int64)
    c = np.mod(c, np.array(p.n_cells[:p.dim]))
    lin = c[:, 0].copy()
    if p.dim > 1:
        lin += p.n_cells[0] * c[:, 1]
    if p.dim > 2:
        lin += p.n_cells[0] * p.n_cells[1] * c[:, 2]
    return lin


def _pairs(p, x, include_self):
    """Index pairs (i, j) with |x_i - x_j| < 2h under the minimum image, and the image shift."""
    _, L = _box(p)
    d = x[:, None, :] - x[None, :, :]
    img = L * np.round(d / L)
    r = np.sqrt(np.sum((d - img) ** 2, axis=2))
    mask = r < 2.0 * p.h
    if not include_self:
        np.fill_diagonal(mask, False)
    i, j = np.nonzero(mask)
    return i, j, img[i, j]


def forward_loss(p, xg0, xd0, mg, md, v0g, v0d, log_tstop, target, steps):
    """Loss after ``steps`` IDIC steps.

    xg0, xd0: absolute FP64 positions (n, dim), numpy; mg, md: masses (numpy);
    v0g, v0d: torch (n, dim) float64 tensors (may require grad); log_tstop: 0-d
    tensor, log t_stop, or log(1/K) when p.K > 0 (K held constant); target: numpy
    (n_dust,) in the same order as xd0.
    Returns (loss, final gas velocity, final dust velocity, final positions).
    """
    dim = p.dim
    sig = _SIGMA[dim]
    h, tau = float(p.h), float(p.dt)
    g = torch.tensor(p.g[:dim], dtype=torch.float64)
    mg_t = torch.as_tensor(mg, dtype=torch.float64)
    md_t = torch.as_tensor(md, dtype=torch.float64)
    ncell = int(np.prod(p.n_cells[:dim]))
    xg = torch.as_tensor(xg0, dtype=torch.float64)
    xd = torch.as_tensor(xd0, dtype=torch.float64)
    v, u = v0g, v0d
    ts = torch.exp(log_tstop)
    kmode = float(getattr(p, "K", 0.0)) > 0.0
    epstein = float(getattr(p, "t_stop_epstein", 0.0)) > 0.0
    vol = float(np.prod([(p.hi[k] - p.lo[k]) / p.n_cells[k] for k in range(dim)]))
    beta = tau / ts
    tkv = tau * vol / ts            # tau K V with K = 1 / exp(log_tstop)
    for _ in range(steps):
        xgn, xdn = xg.detach().numpy(), xd.detach().numpy()
        cg = torch.as_tensor(_cells(p, xgn))
        cd = torch.as_tensor(_cells(p, xdn))
        # gas summation density: self term m_a W(0) plus distinct pairs within 2h
        i, j, img = _pairs(p, xgn, include_self=False)
        it, jt = torch.as_tensor(i), torch.as_tensor(j)
        rv = xg[it] - xg[jt] - torch.as_tensor(img)
        rr = torch.sqrt(torch.sum(rv * rv, dim=1))
        rho = (mg_t + torch.zeros(xg.shape[0], dtype=torch.float64).index_add(0, it, mg_t[jt] * _f(rr / h))) \
            * (sig / h ** dim)
        P = p.c_s ** 2 / rho
        # pressure acceleration over the same distinct pairs
        coef = mg_t[jt] * (P[it] + P[jt]) * _df(rr / h) * (sig / h ** (dim + 1)) / rr
        A = -torch.zeros_like(xg).index_add(0, it, coef[:, None] * rv)
        vt = v + tau * (A + g)
        ut = u + tau * g
        # cell sums and the implicit solve
        Mg = torch.zeros(ncell, dtype=torch.float64).index_add(0, cg, mg_t)
        Md = torch.zeros(ncell, dtype=torch.float64).index_add(0, cd, md_t)
        Pg = torch.zeros((ncell, dim), dtype=torch.float64).index_add(0, cg, mg_t[:, None] * vt)
        Pd = torch.zeros((ncell, dim), dtype=torch.float64).index_add(0, cd, md_t[:, None] * ut)
        both = (Mg > 0) & (Md > 0)
        Mg_s = torch.where(both, Mg, torch.ones_like(Mg))
        Md_s = torch.where(both, Md, torch.ones_like(Md))
        if kmode:
            al = torch.where(both, tkv / Mg_s, torch.zeros_like(Mg_s))
            be = torch.where(both, tkv / Md_s, torch.zeros_like(Md_s))
        elif epstein:      # t*_stop = T_E / rho*_g with T_E = exp(log_tstop)
            al = torch.where(both, tau * (Md_s / vol) / ts, torch.zeros_like(Md_s))
            be = torch.where(both, tau * (Mg_s / vol) / ts, torch.zeros_like(Mg_s))
        else:
            eps = Md_s / Mg_s
            al = torch.where(both, eps * beta, torch.zeros_like(eps))
            be = torch.where(both, beta * torch.ones_like(eps), torch.zeros_like(eps))
        Dd = 1.0 + al + be
        Vt, Ut = Pg / Mg_s[:, None], Pd / Md_s[:, None]
        Vs = ((1.0 + be)[:, None] * Vt + al[:, None] * Ut) / Dd[:, None]
        Us = (be[:, None] * Vt + (1.0 + al)[:, None] * Ut) / Dd[:, None]
        v = (vt + al[cg][:, None] * Us[cg]) / (1.0 + al[cg])[:, None]
        u = (ut + be[cd][:, None] * Vs[cd]) / (1.0 + be[cd])[:, None]
        xg = xg + tau * v
        xd = xd + tau * u
    # dust density misfit at the final positions
    xdn = xd.detach().numpy()
    i, j, img = _pairs(p, xdn, include_self=False)
    it, jt = torch.as_tensor(i), torch.as_tensor(j)
    rv = xd[it] - xd[jt] - torch.as_tensor(img)
    rr = torch.sqrt(torch.sum(rv * rv, dim=1))
    rho_d = (md_t + torch.zeros(xd.shape[0], dtype=torch.float64).index_add(0, it, md_t[jt] * _f(rr / h))) \
        * (sig / h ** dim)
    loss = torch.mean((rho_d - torch.as_tensor(target)) ** 2)
    return loss, v, u, (xg, xd), rho_d


def gradients(p, xg0, xd0, mg, md, v0g, v0d, t_stop, target, steps):
    """(loss, dL/dlog t_stop, dL/dv0 (n_g, d), dL/du0 (n_d, d)) by autograd, all FP64 numpy.
    With p.K > 0, ``t_stop`` is 1/K and the scalar derivative is dL/dlog(1/K)."""
    vg = torch.tensor(v0g, dtype=torch.float64, requires_grad=True)
    vd = torch.tensor(v0d, dtype=torch.float64, requires_grad=True)
    s = torch.tensor(math.log(t_stop), dtype=torch.float64, requires_grad=True)
    loss, *_ = forward_loss(p, xg0, xd0, mg, md, vg, vd, s, target, steps)
    loss.backward()
    return float(loss), float(s.grad), vg.grad.numpy().copy(), vd.grad.numpy().copy()
