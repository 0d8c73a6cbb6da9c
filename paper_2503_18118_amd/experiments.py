"""The paper's numerical experiments (Sec. IV-C Fig. 3, Sec. V-C Fig. 4, Appendix A Fig. 5) on the GPU path.

Both run through the library's capacity sweep (exact Gram, closed forms, FP64
rates, ergodic means and the saturation point); nothing here computes.

* ``fig2``: the power saturation point of Sec. IV-A (Fig. 2): a user's received power reaches the
  fraction t of its limit (eq. (5)) once the centred array covers [y_down, y_up] of eqs. (13)-(16)
  (at y = 0, M >= 4 x t / (lambda sqrt(1 - t^2)), eq. (12)); the exact Gram's diagonal at that M.
* ``fig3``: normalised capacity C(N) / C(N_max) of the Sec. IV scene (100 GHz
  PNUSW ULA, x ~ U[1,10] m, y ~ U[-7.5,7.5] m, t = 0.9) at 0 dB and 200 dB,
  beside the analytic saturation span E[y_up] - E[y_down] of eqs. (15)-(16),
  with the paper's K = 100 users.
* ``fig4``: ergodic sum-rates of the Sec. V scene (x ~ U(1,2) m, K = 10, received
  SNR limit 33 dB for one user at (1.5 m, 0)) for ZF, MMSE, MRC and the capacity
  on the exact Gram, and the modified ZF of eqs. (22)-(23): nominal (ZF formula on
  the closed-form Gram) and as the paper scores it (the closed-form filter
  applied to the true channel).  The closed form is eq. (6) as printed (variant
  PAPER); the uniform closed form (UNIFORM) is run beside it.

* ``fig5``: Appendix A's normalised gap between the Hadamard and Schur-Horn capacity
  bounds, -(1/K) log2 det R (eq. (9)), against K in the Sec. IV scene at N = 65536,
  K = 2 ... 1000 as in the paper (which states neither N nor the drop count).

* ``tracking``: the premise of Sec. V-B (user states from sensing, channels regenerated as users
  move): per frame one user of every drop moves, and the exact Gram is brought up to date by
  recomputing that user's row and column (xlmimo_gram_update_users) instead of the whole Gram.
  Times both and checks that they agree.  Not a figure of the paper.

``python -m paper_2503_18118_amd.experiments [fig2|fig3|fig4|fig5|tracking] [--drops D] [--json PATH]``
prints a table and optionally writes the numbers as JSON.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import snr
from . import xlmimo as X

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))
import workloads as W  # noqa: E402  (seeded input generators)

# 64 ... 131072 antennas.  Below 64 the Sec. V scene's ten users give Grams with condition numbers up
# to 1e12 (N = 32) and 1e17 (N = 16): ZF is then ill-posed even in FP64.
FIG_N = [2 ** e for e in range(6, 18)]
FIG3_N = [2 ** e for e in range(9, 18)]          # 512 ... 131072 (4 K and up, K = 100)
FIG5_K = (2, 4, 8, 16, 32, 64, 128, 256, 512, 1000)


FIG2_USERS = ((1.0, 0.0), (2.0, 0.0), (5.0, 0.0), (10.0, 0.0), (2.0, 3.0), (5.0, -4.0), (10.0, 7.5))


def fig2(ctx, n_drops: int = 0, users=FIG2_USERS, t: float = 0.9) -> dict:
    """Sec. IV-A power saturation (Fig. 2): for each user (x, y) in metres, the array size M at which
    the centred 100 GHz PNUSW ULA covers [y_down, y_up] = [y - x tau, y + x tau], tau = t / sqrt(1 - t^2)
    (eqs. (13)-(16); eq. (12) at y = 0), and the ratio of the exact received power (the Gram's
    diagonal, FP64) at that M to its limit 4 beta0 / (lambda x) (eq. (5)).  Each user is a drop of its
    own with its own M (n_drops is unused)."""
    lam, beta0 = W.LAMBDA_100GHZ, 1.0
    d = lam / 2.0
    tau = t / math.sqrt(1.0 - t * t)
    ms = [int(math.ceil(2.0 * max(abs(y + x * tau), abs(y - x * tau)) / d)) for x, y in users]
    drops = W._pack(ms, [1] * len(users), [[x, y, 0.0] for x, y in users])
    b = X.Batch(drops)
    s = torch.cuda.current_stream()
    e0, e1 = _events()
    e0.record(s)
    g = ctx.gram_exact(W.ula(1, lam, W.AMP_PNUSW), b, X.FP64)
    e1.record(s)
    e1.synchronize()
    power = g.view(torch.complex128).real.cpu().numpy()          # one entry per single-user drop
    ratio = [float(power[i] / (4.0 * beta0 / (lam * x))) for i, (x, _) in enumerate(users)]
    return {"scene": "Sec. IV-A: 100 GHz PNUSW ULA, half-wavelength spacing", "t": t,
            "users": [list(u) for u in users], "saturation_m": ms, "power_ratio": ratio,
            "gpu_ms": e0.elapsed_time(e1)}


def _table_fig2(r):
    lines = [f"Fig. 2 ({r['scene']}; t = {r['t']}): received power at the saturation size M against its limit",
             "| user (x, y) m | M | P / P_lim |", "|---|---|---|"]
    for u, m, q in zip(r["users"], r["saturation_m"], r["power_ratio"]):
        lines.append(f"| ({u[0]:g}, {u[1]:g}) | {m} | {q:.6f} |")
    return "\n".join(lines)


def _timed_sweep(ctx, arr, n_list, batch, form, rho, schemes, t_sat=0.9, eps_sat=0.05):
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    erg, sat, st = ctx.capacity_sweep(arr, n_list, batch, form, rho, schemes, t_sat, eps_sat)
    e1.record(s)
    e1.synchronize()
    return erg.cpu().numpy(), sat.cpu().numpy(), st.cpu().numpy(), e0.elapsed_time(e1)


def fig3(ctx, n_drops: int = 200, n_list=FIG3_N, k: int = 100, snr_db=(0.0, 200.0), t: float = 0.9,
         eps: float = 0.05) -> dict:
    """Normalised capacity of the Sec. IV scene on the exact FP64 Gram (K = 100 users).

    At 200 dB, log2 det(I + rho G) weighs G's smallest eigenvalues by rho ~ 1e20, so the Gram is
    taken in FP64 and N starts at 4 K (N near K leaves G rank-deficient to rounding).
    """
    arr = W.ula(int(n_list[-1]), W.LAMBDA_100GHZ, W.AMP_PNUSW)
    drops = W.rect_drops(W.rng_for(10), n_drops, k, int(n_list[-1]), (1.0, 10.0), (-7.5, 7.5))
    b = X.Batch(drops)
    rho = snr.rho_for_snr(arr, snr_db, 5.5, b.total_users)       # reference user at the mean x
    erg, sat, st, ms = _timed_sweep(ctx, arr, n_list, b, X.FORM_EXACT_FP64, rho, X.CAP, t, eps)
    cap = erg[:, :, 0]
    return {"scene": "Sec. IV: 100 GHz PNUSW ULA, x ~ U[1,10] m, y ~ U[-7.5,7.5] m, t = 0.9",
            "users": k, "drops": n_drops, "n_list": [int(n) for n in n_list], "snr_db": list(snr_db),
            "capacity": cap.tolist(), "normalised_capacity": (cap / cap[-1]).tolist(),
            "e_y_up": float(sat[0]), "e_y_down": float(sat[1]), "analytic_saturation_n": float(sat[2]),
            "empirical_saturation_n": [float(sat[3 + i]) for i in range(len(snr_db))], "eps": eps,
            "flagged_drops": int((st != 0).sum()), "gpu_ms": ms}


def fig4(ctx, n_drops: int = 200, n_list=FIG_N, rx_snr_db: float = 33.0, forms=("PAPER", "UNIFORM"),
         t: float = 0.9, eps: float = 0.05) -> dict:
    """Ergodic sum-rates of the Sec. V scene per scheme.

    ZF, MMSE, MRC and the capacity come from the exact FP64 Gram: at small N the ten users'
    Gram is ill-conditioned and ZF amplifies the FP32 Gram's rounding.  The modified ZF
    (nominal and mismatched) comes from one closed-form sweep per variant, whose true channel for
    the mismatched scheme is the exact FP64 Gram (G~^-1 G amplifies its error by the condition
    number when the filter is accurate).
    """
    arr = W.ula(int(n_list[-1]), W.LAMBDA_100GHZ, W.AMP_PNUSW)
    drops = W.rect_drops(W.rng_for(11), n_drops, 10, int(n_list[-1]), (1.0, 2.0), (-7.5, 7.5))
    b = X.Batch(drops)
    rho = snr.rho_for_snr(arr, [rx_snr_db], 1.5, b.total_users)  # SNR limit of one user at (1.5 m, 0)
    exact_schemes = (("ZF", X.ZF), ("MMSE", X.MMSE), ("MRC", X.MRC), ("CAP", X.CAP))
    cf_schemes = (("MZF", X.MZF), ("MZF_MISM", X.MZF_MISM))
    erg, sat, st, ms = _timed_sweep(ctx, arr, n_list, b, X.FORM_EXACT_FP64, rho,
                                    X.ZF | X.MMSE | X.MRC | X.CAP, t, eps)
    out = {"scene": "Sec. V: 100 GHz PNUSW ULA, x ~ U(1,2) m, y ~ U[-7.5,7.5] m, K = 10, "
                    "received SNR limit 33 dB at (1.5 m, 0)",
           "users": 10, "drops": n_drops, "n_list": [int(n) for n in n_list], "rx_snr_limit_db": rx_snr_db,
           "analytic_saturation_n": float(sat[2]),
           "exact": {"sum_rate": {name: erg[:, 0, i].tolist() for i, (name, _) in enumerate(exact_schemes)},
                     "empirical_saturation_n": {name: float(sat[3 + i]) for i, (name, _) in
                                                enumerate(exact_schemes)},
                     "flagged_drops": int((st != 0).sum()), "gpu_ms": ms},
           "forms": {}}
    for name in forms:
        form = {"PAPER": X.FORM_CF_PAPER, "UNIFORM": X.FORM_CF_UNIFORM}[name]
        erg, sat, st, ms = _timed_sweep(ctx, arr, n_list, b, form, rho, X.MZF | X.MZF_MISM, t, eps)
        out["forms"][name] = {"sum_rate": {sch: erg[:, 0, i].tolist() for i, (sch, _) in enumerate(cf_schemes)},
                              "filter_not_pd_drops": [int(((st[i] & X.ST_FILTER_NOT_PD) != 0).sum())
                                                      for i in range(len(n_list))],
                              "gpu_ms": ms}
    return out


def fig5(ctx, n_drops: int = 100, k_list=FIG5_K, n: int = 65536) -> dict:
    """Appendix A, Fig. 5: the normalised bound gap -E[log2 lambda^R] = -(1/K) log2 det R against K
    in the Sec. IV scene at N = 65536 antennas (beyond the saturation point of every K here)."""
    arr = W.ula(n, W.LAMBDA_100GHZ, W.AMP_PNUSW)
    gaps, ms_k, flagged = [], [], []
    for k in k_list:
        drops = W.rect_drops(W.rng_for(10), n_drops, int(k), n, (1.0, 10.0), (-7.5, 7.5))
        b = X.Batch(drops)
        rho = torch.ones((1, b.total_users), dtype=torch.float64, device="cuda")   # the gap has no SNR
        erg, sat, st, ms = _timed_sweep(ctx, arr, [n], b, X.FORM_EXACT_FP64, rho, X.CORR_GAP)
        gaps.append(float(erg[0, 0, 0]))
        ms_k.append(ms)
        flagged.append(int((st != 0).sum()))
        del b, erg, st
    return {"scene": "Sec. IV: 100 GHz PNUSW ULA, x ~ U[1,10] m, y ~ U[-7.5,7.5] m", "n": n, "drops": n_drops,
            "k_list": [int(k) for k in k_list], "negative_mean_log2_eig_R": gaps, "gpu_ms_by_k": ms_k,
            "flagged_drops_by_k": flagged, "gpu_ms": float(sum(ms_k))}


def _events():
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def tracking(ctx, n_drops: int = 20, k_list=(16, 256, 1000), n: int = 65536, frames: int = 5,
             step_m: float = 0.005, precisions=("FP64", "FP32H")) -> dict:
    """Per frame, the middle user of every drop moves by step_m in y; the Gram is updated by rows
    and, for comparison, recomputed whole; the Cholesky factor of G is updated (rank 2 per moved
    user) and, for comparison, computed anew from the recomputed Gram.  Reports the mean time per
    frame of each, the largest normwise difference between the two Grams and the largest
    difference of log2 det G over all frames."""
    arr = W.ula(n, W.LAMBDA_100GHZ, W.AMP_PNUSW)
    out = {"scene": "Sec. IV: 100 GHz PNUSW ULA, x ~ U[1,10] m, y ~ U[-7.5,7.5] m", "n": n, "drops": n_drops,
           "frames": frames, "step_m": step_m, "k_list": [int(k) for k in k_list], "by_precision": {}}
    s = torch.cuda.current_stream()
    for pname in precisions:
        prec = getattr(X, pname)
        rows = {"full_ms": [], "update_ms": [], "max_normwise_diff": [], "refactor_ms": [], "factor_update_ms": [],
                "max_log2det_diff": []}
        for k in k_list:
            drops = W.rect_drops(W.rng_for(10), n_drops, int(k), n, (1.0, 10.0), (-7.5, 7.5))
            b = X.Batch(drops)
            g = ctx.gram_exact(arr, b, prec)
            full = torch.empty_like(g)
            factor, _, _ = ctx.cholesky(b, g)
            t_full = t_upd = t_refac = t_fupd = 0.0
            worst = worst_ld = 0.0
            moved = (drops.user_off[:-1] + int(k) // 2).astype(np.int64)
            for f in range(frames + 1):        # frame 0 builds the launch plans and is not timed
                b.pos[torch.as_tensor(moved, device=b.pos.device), 1] += step_m
                e0, e1 = _events()
                e0.record(s)
                ctx.gram_update_users(arr, b, moved, g, prec)
                e1.record(s)
                e2, e3 = _events()
                e2.record(s)
                ctx.gram_exact(arr, b, prec, out=full)
                e3.record(s)
                e4, e5 = _events()
                e4.record(s)
                ld_upd, _ = ctx.cholesky_update_users(arr, b, moved, g, factor)
                e5.record(s)
                e6, e7 = _events()
                e6.record(s)
                _, ld_new, _ = ctx.cholesky(b, full)
                e7.record(s)
                e7.synchronize()
                if f:
                    t_upd += e0.elapsed_time(e1)
                    t_full += e2.elapsed_time(e3)
                    t_fupd += e4.elapsed_time(e5)
                    t_refac += e6.elapsed_time(e7)
                worst_ld = max(worst_ld, float((ld_upd - ld_new).abs().max()))
                gu = g.view(torch.complex128)
                gf = full.view(torch.complex128)
                for d in range(n_drops):
                    lo, hi = int(b.gram_off[d]), int(b.gram_off[d + 1])
                    a = gu[lo:hi].view(int(k), int(k))
                    c = gf[lo:hi].view(int(k), int(k))
                    dg = torch.sqrt(torch.diagonal(c).real)
                    worst = max(worst, float(((a - c).abs() / torch.outer(dg, dg)).max()))
            rows["full_ms"].append(t_full / frames)
            rows["update_ms"].append(t_upd / frames)
            rows["max_normwise_diff"].append(worst)
            rows["refactor_ms"].append(t_refac / frames)
            rows["factor_update_ms"].append(t_fupd / frames)
            rows["max_log2det_diff"].append(worst_ld)
            del b, g, full, factor
        out["by_precision"][pname] = rows
    return out


def _table_tracking(r):
    lines = [f"Tracking ({r['scene']}; N = {r['n']}, {r['drops']} drops, one user per drop moves "
             f"{1e3 * r['step_m']:.0f} mm per frame; mean over {r['frames']} frames)",
             "| Gram precision | K | full Gram ms | row update ms | speed-up | max normwise difference "
             "| new factor ms | factor update ms | speed-up | max log2 det difference |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for p, rows in r["by_precision"].items():
        for i, k in enumerate(r["k_list"]):
            fm, um = rows["full_ms"][i], rows["update_ms"][i]
            rf, fu = rows["refactor_ms"][i], rows["factor_update_ms"][i]
            lines.append(f"| {p} | {k} | {fm:.3f} | {um:.3f} | {fm / um:.1f} | {rows['max_normwise_diff'][i]:.1e} "
                         f"| {rf:.3f} | {fu:.3f} | {rf / fu:.1f} | {rows['max_log2det_diff'][i]:.1e} |")
    return "\n".join(lines)


def _table_fig5(r):
    lines = [f"Fig. 5 ({r['scene']}; N = {r['n']}, {r['drops']} drops): -E[log2 lambda^R] against K",
             "| K | " + " | ".join(str(k) for k in r["k_list"]) + " |", "|---|" + "---|" * len(r["k_list"]),
             "| gap | " + " | ".join(f"{v:.5f}" for v in r["negative_mean_log2_eig_R"]) + " |",
             "| GPU ms | " + " | ".join(f"{v:.0f}" for v in r["gpu_ms_by_k"]) + " |"]
    return "\n".join(lines)


def _table_fig3(r):
    lines = [f"Fig. 3 ({r['scene']}; K = {r['users']}, {r['drops']} drops): normalised capacity",
             "| N | " + " | ".join(f"{s:g} dB" for s in r["snr_db"]) + " |",
             "|---|" + "---|" * len(r["snr_db"])]
    for i, n in enumerate(r["n_list"]):
        lines.append(f"| {n} | " + " | ".join(f"{r['normalised_capacity'][i][j]:.4f}"
                                                for j in range(len(r["snr_db"]))) + " |")
    lines.append(f"analytic saturation (eqs. (15)-(16)): N = {r['analytic_saturation_n']:.0f}; "
                 f"empirical (C >= (1 - {r['eps']}) C_max): " +
                 ", ".join(f"{n:.0f}" for n in r["empirical_saturation_n"]))
    return "\n".join(lines)


def _table_fig4(r):
    forms = list(r["forms"])
    cols = list(r["exact"]["sum_rate"]) + [f"{sch} ({f})" for f in forms for sch in r["forms"][f]["sum_rate"]]
    lines = [f"Fig. 4 ({r['scene']}; {r['drops']} drops): ergodic sum-rate [bit/s/Hz]",
             "| N | " + " | ".join(cols) + " |", "|---|" + "---|" * len(cols)]
    for i, n in enumerate(r["n_list"]):
        vals = [r["exact"]["sum_rate"][s][i] for s in r["exact"]["sum_rate"]]
        vals += [r["forms"][f]["sum_rate"][s][i] for f in forms for s in r["forms"][f]["sum_rate"]]
        lines.append(f"| {n} | " + " | ".join(f"{v:.3f}" for v in vals) + " |")
    lines.append(f"analytic saturation (eqs. (15)-(16)): N = {r['analytic_saturation_n']:.0f}; empirical "
                 "(rate >= 0.95 of the last point): " +
                 ", ".join(f"{k} {v:.0f}" for k, v in r["exact"]["empirical_saturation_n"].items()))
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("figure", choices=["fig2", "fig3", "fig4", "fig5", "tracking"])
    ap.add_argument("--drops", type=int, default=1000)
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    ctx = X.Context(0)
    t0 = time.perf_counter()
    run, table = {"fig2": (fig2, _table_fig2), "fig3": (fig3, _table_fig3), "fig4": (fig4, _table_fig4),
                  "fig5": (fig5, _table_fig5),
                  "tracking": (tracking, _table_tracking)}[args.figure]
    r = run(ctx, args.drops)
    r["wall_s"] = time.perf_counter() - t0
    print(table(r))
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(r, fh, indent=1)
    ctx.close()


if __name__ == "__main__":
    main()
