"""Sweep-rate / damping scan of the single-macrospin limit against Sharrock's
law (Eq. 14).

Eq. 14 gives the coercive field of an ensemble of uniaxial particles whose
moments must cross an energy barrier KV(1 - H/H_K)^2 within an observation
time tau:  H_c = H_K [1 - sqrt((k_B T/KV) ln(f0 tau/ln 2))].  In a loop
tau scales as 1/SR, and in the high-barrier limit Brown's attempt frequency
f0 is proportional to alpha/(1 + alpha^2) (the damping rate alpha gamma1 of
the LLG equation), i.e. to alpha at small alpha.  Hence:

  * at fixed alpha, (1 - H_c/H_K)^2 falls linearly in ln SR with slope
    k_B T/KV;
  * at fixed SR/alpha, f0 tau is fixed while alpha << 1, so H_c is invariant
    (the argument behind the paper's SR/alpha scaling); for larger alpha
    f0 tau shrinks by 1/(1 + alpha^2) and (1 - H_c/H_K)^2 by
    (k_B T/KV) ln(1 + alpha^2): the invariance breaks and H_c grows.

``scan`` runs each (SR, alpha) pair as its own context on its own stream
(one realization per quad of lanes, all pairs concurrently) and returns the loops'
coercive fields and areas in simulation units with their standard errors;
``sharrock_check`` fits the laws above.  Run

    python -m paper_1912_00310_amd.sharrock [--T 100] [--ratio 2.5] [--n-real 256]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

KB = 1.380649e-23          # J/K
OE_PER_APM = 4.0e-3 * math.pi   # 1 A/m in Oe


def _workloads():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import sllg_workloads as W
    return W


def scan(pairs, T_K=310.0, n_real=256, dt_s=1e-12, streams=4, device="cuda:0", log=None):
    """Loops of the single-cell rod at each (SR in Oe/ns, alpha) pair.
    Returns one dict per pair: Hc, Hc_se, S, S_se (Oe, simulated field), the
    cell's H_K (Oe) and KV/(k_B T), and the steps per loop."""
    import torch

    from .sllg import Sim
    W = _workloads()
    strm = [torch.cuda.Stream(device=device) for _ in range(max(1, streams))]
    sims = []
    t0 = time.time()
    for i, (sr, al) in enumerate(pairs):
        wl = W.macrospin_pair(sr, al, T_K=T_K, n_real=n_real, dt_s=dt_s)
        sim = Sim(wl["material"], wl["levels"], device=device, stream=strm[i % len(strm)])
        sims.append((sr, al, sim))
    # every pair's sweep enqueued before any is waited for: pairs on
    # different streams run concurrently (each occupies a few CUs)
    for sr, al, sim in sims:
        sim.run_sweep()
    out = [None] * len(sims)
    # the shortest sweeps are read first (progress while the long ones run)
    order = sorted(range(len(sims)), key=lambda i: sims[i][0], reverse=True)
    for i in order:
        sr, al, sim = sims[i]
        _, _, st = sim.loop(0, -1)
        p = sim.level_params(0)
        kv = p["K"] * p["a"] ** 3 / (KB * T_K)
        out[i] = dict(SR=sr, alpha=al, T=T_K, Hc=st["Hc_sim"], Hc_se=st["Hc_se"], S=st["S_sim"],
                      S_se=st["S_se"], Mr=st["Mr_sim"], H_K=p["hk"] * OE_PER_APM, KV_kT=kv,
                      n_steps=int(p["n_steps"]), kernel=sim.kernel_name(0))
        if log:
            log(f"SR {sr:g} Oe/ns alpha {al:g}: Hc {st['Hc_sim']:.2f} +- {st['Hc_se']:.2f} Oe, "
                f"S {st['S_sim']:.1f} +- {st['S_se']:.1f} Oe ({int(p['n_steps'])} steps)")
        sim.close()
    if log:
        log(f"{len(pairs)} pairs in {time.time() - t0:.1f} s")
    return out


def _linfit(x, y):
    n = len(x)
    mx, my = sum(x) / n, sum(y) / n
    sxx = sum((a - mx) ** 2 for a in x)
    sxy = sum((a - mx) * (b - my) for a, b in zip(x, y))
    b = sxy / sxx
    return my - b * mx, b


def sharrock_check(at_ratio, at_alpha=None, small_alpha=0.1, h_max=0.95):
    """Fit Eq. 14 to the scans.

    at_ratio: results at fixed SR/alpha.  The intercept A of
    (1 - Hc/H_K)^2 = A - (k_B T/KV) ln(1 + alpha^2) is taken from the points
    with alpha <= small_alpha; the law then predicts Hc at every alpha.
    at_alpha: results at one alpha over several SR; the slope of
    (1 - Hc/H_K)^2 against ln SR, over the points of thermally activated
    switching (Hc/H_K < h_max: nearer H_K the moment follows the sweep
    dynamically and the barrier picture no longer applies), is compared with
    -k_B T/KV.
    """
    rep = {}
    r0 = at_ratio[0]
    kt_kv = 1.0 / r0["KV_kT"]
    small = [r for r in at_ratio if r["alpha"] <= small_alpha and math.isfinite(r["Hc"])]
    if small:
        A = sum((1 - r["Hc"] / r["H_K"]) ** 2 + kt_kv * math.log(1 + r["alpha"] ** 2) for r in small) / len(small)
        pred = []
        for r in at_ratio:
            y = A - kt_kv * math.log(1 + r["alpha"] ** 2)
            hc = r["H_K"] * (1 - math.sqrt(y)) if y > 0 else r["H_K"]
            pred.append(dict(alpha=r["alpha"], SR=r["SR"], Hc=r["Hc"], Hc_se=r["Hc_se"], Hc_eq14=hc))
        rep["fixed_ratio"] = dict(A=A, kT_KV=kt_kv, points=pred)
    if at_alpha:
        pts = [r for r in at_alpha if math.isfinite(r["Hc"]) and r["Hc"] / r["H_K"] < h_max]
        x = [math.log(r["SR"]) for r in pts]
        y = [(1 - r["Hc"] / r["H_K"]) ** 2 for r in pts]
        if len(pts) >= 2:
            a, b = _linfit(x, y)
            rep["fixed_alpha"] = dict(alpha=pts[0]["alpha"], slope=b, minus_kT_KV=-1.0 / pts[0]["KV_kT"],
                                      ratio=b / (-1.0 / pts[0]["KV_kT"]),
                                      points=[dict(SR=r["SR"], Hc=r["Hc"], Hc_se=r["Hc_se"]) for r in pts])
    return rep


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--T", type=float, default=100.0, help="temperature, K")
    ap.add_argument("--ratio", type=float, default=2.5, help="SR/alpha, Oe/ns")
    ap.add_argument("--alphas", default="0.01,0.03,0.1,0.3,1,3,10")
    ap.add_argument("--fixed-alpha", type=float, default=0.1)
    ap.add_argument("--srs", default="0.025,0.075,0.25,0.75,2.5", help="sweep rates at the fixed alpha, Oe/ns")
    ap.add_argument("--n-real", type=int, default=256)
    ap.add_argument("--dt", type=float, default=1e-12)
    a = ap.parse_args()
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
    alphas = [float(x) for x in a.alphas.split(",")]
    srs = [float(x) for x in a.srs.split(",")]
    pairs_r = [(a.ratio * al, al) for al in alphas]
    pairs_a = [(sr, a.fixed_alpha) for sr in srs if (sr, a.fixed_alpha) not in pairs_r]
    res = scan(pairs_r + pairs_a, T_K=a.T, n_real=a.n_real, dt_s=a.dt, log=log)
    at_ratio = res[:len(pairs_r)]
    at_alpha = [r for r in res if r["alpha"] == a.fixed_alpha and r["SR"] in srs]
    print(json.dumps({"T": a.T, "ratio": a.ratio, "dt": a.dt, "n_real": a.n_real, "results": res,
                      "sharrock": sharrock_check(at_ratio, at_alpha)}))


if __name__ == "__main__":
    main()
