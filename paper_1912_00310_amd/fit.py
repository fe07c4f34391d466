"""Fitting coarse-grained cell parameters to target loops with the adjoint.

The modified Grinstein-Koch rule (Eqs. 8-13) prescribes K(b), A(b) and the
field and magnetisation scales of a coarse level; the paper finds its loops
invariant with b to 10-15 % (Fig. 2c).  With sllg_grad the level's simulated
K, A, alpha and ms_scale can instead be fitted so that its loop area and
coercive field reproduce a target, e.g. the loops of the fine (b = 1) grid.

``fit_level`` runs damped Gauss-Newton steps on the residuals
(S - S*, w (Hc - Hc*)) in the logarithms of the fitted parameters; every
step costs one forward sweep of the level and one adjoint sweep, both on the
GPU through the C ABI.
"""
from __future__ import annotations

import math

from .sllg import loop_area_hc

PARAMS = ("K", "A", "alpha", "ms_scale")


def fit_level(material: dict, level: dict, start: dict, target, fit=("K",), hc_weight=0.0,
              steps: int = 6, damping: float = 1e-3, ckpt_every: int = 256, tol: float = 1e-4):
    """Fit the parameters named in ``fit`` (a subset of K, A, alpha,
    ms_scale) of one level so that its ensemble-mean loop has area
    target[0] and, when hc_weight > 0, coercive field target[1] (simulation
    units, Oe).  ``start`` holds all four values (K and A simulated, J/m^3
    and J/m).  Returns (values, history); history lists per step the values,
    S, Hc and the squared residual norm.
    """
    import torch
    vals = {k: float(start[k]) for k in PARAMS}
    hist = []
    for it in range(steps + 1):
        x = {k: torch.tensor(vals[k], dtype=torch.float64, requires_grad=k in fit) for k in PARAMS}
        S, Hc = loop_area_hc(x["K"], x["A"], x["alpha"], x["ms_scale"], material, level, ckpt_every)
        Sv, Hv = float(S.detach()), float(Hc.detach())
        res = [Sv - target[0]]
        outs = [S]
        if hc_weight > 0 and math.isfinite(Hv) and math.isfinite(target[1]):
            res.append(hc_weight * (Hv - target[1]))
            outs.append(Hc)
        err = sum(r * r for r in res)
        hist.append(dict(vals, S=Sv, Hc=Hv, err=err))
        if it == steps or err <= (tol * abs(target[0])) ** 2:
            break
        # Jacobian of the residuals in log-parameters: dr/dlog p = p dr/dp
        rows = []
        for j, o in enumerate(outs):
            g = torch.autograd.grad(o, [x[k] for k in fit], retain_graph=j + 1 < len(outs))
            w = 1.0 if j == 0 else hc_weight
            rows.append([w * float(gi) * vals[k] for gi, k in zip(g, fit)])
        J = torch.tensor(rows, dtype=torch.float64)
        r = torch.tensor(res, dtype=torch.float64)
        JtJ = J.T @ J
        lam = damping * float(torch.trace(JtJ)) / len(fit) + 1e-300
        step = torch.linalg.solve(JtJ + lam * torch.eye(len(fit), dtype=torch.float64), -(J.T @ r))
        for k, dl in zip(fit, step.tolist()):
            vals[k] *= math.exp(max(-0.5, min(0.5, dl)))   # at most a factor e^0.5 per step
    return vals, hist
