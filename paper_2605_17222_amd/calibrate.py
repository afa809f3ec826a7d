"""Refits the rates of the library's LT cost model (ckks_lt_predict) on the
device it runs on.

For banded TH-BSGS LTs at N = 2^16 over several levels and diagonal counts,
a spread of splits from the autotuner's search space (n1 n2 n3 in [n, 2n))
is timed with HIP events on uniform-residue inputs resident in HBM.  The
predictor is linear in its rates once the per-split features are known:

    t = ntt_limb_s * f_ntt + bconv_product_s * f_bconv + f_bytes / hbm_bytes_per_s + layer_s * f_layers

and the features are read from the library itself, by calling
ckks_lt_predict with one rate set at a time.  The BConv rate is taken from
that kernel's own time (a second pass of each point with every kernel
timed, summed over the points, over the model's conversion products); the
other three rates are fitted to the rest of each LT's time by non-negative
least squares on relative errors.  They are regression coefficients over
features that grow together (limb NTTs, BConv products and hoisting layers
rise with every Decompose and ModDown), so the NTT rate is not the NTT
passes' time per limb, which is reported beside it.  Prints one JSON object:
the rates, the fit's mean and largest relative error, every point, and per
(level, n) the split the fitted model picks against the measured fastest.

    python -m paper_2605_17222_amd.calibrate [--levels 8 16 24] [--diags 16 32 64 128 256]
"""
import argparse
import json
import sys
import time

import numpy as np

_HUGE = 1e300
NTT_KERNELS = ("ntt_fwd_col", "ntt_fwd_row", "ntt_inv_row", "ntt_inv_col")


def features(H, prm, level, split, n_diag):
    """(f_ntt, f_bconv, f_bytes, f_layers) of ckks_lt_predict for one split."""
    def at(rates):
        return H.ckks_lt_predict(prm.log_n, level, prm.alpha, H.CKKS_LT_TH_BSGS, split, n_diag, rates=rates)
    return (at((1.0, 0.0, _HUGE, 0.0)), at((0.0, 1.0, _HUGE, 0.0)), at((0.0, 0.0, 1.0, 0.0)),
            at((0.0, 0.0, _HUGE, 1.0)))


def candidates(n_diag, per_group, H, prm, level):
    """Splits of the autotuner's search space, spread over the current
    model's ranking: its best few, then evenly spaced through the rest."""
    all_splits = []
    for a in range(1, n_diag + 1):
        for b in range(1, 2 * n_diag // a + 1):
            for c in range(1, 2 * n_diag // (a * b) + 1):
                if n_diag <= a * b * c < 2 * n_diag:
                    all_splits.append((a, b, c))
    ranked = sorted(all_splits, key=lambda s: H.ckks_lt_predict(prm.log_n, level, prm.alpha, H.CKKS_LT_TH_BSGS,
                                                                 s, n_diag))
    head = ranked[:per_group // 2]
    rest = ranked[per_group // 2:]
    step = max(1, len(rest) // max(1, per_group - len(head)))
    return head + rest[::step][:per_group - len(head)]


def time_split(torch, H, W, P, prm, level, split, n_diag, steps, warmup, seed):
    n = prm.n
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)

    def residues(mods):
        m = torch.tensor(mods, dtype=torch.int64, device="cuda").view(-1, 1)
        x = torch.empty((len(mods), n), dtype=torch.int64, device="cuda")
        for r0 in range(0, len(mods), 1024):
            r1 = min(len(mods), r0 + 1024)
            torch.randint(0, 2 ** 62, (r1 - r0, n), generator=g, dtype=torch.int64, device="cuda", out=x[r0:r1])
            torch.remainder(x[r0:r1], m[r0:r1], out=x[r0:r1])
        return x

    kmax = prm.alpha + prm.max_level + 1
    beta_max = -(-(prm.max_level + 1) // prm.alpha)
    pq = list(prm.p) + list(prm.q)
    rots = W.th_rotations(*split)
    per_key = pq[:kmax] * (2 * beta_max)
    kall = residues(per_key * len(rots))
    keys = {r: kall[i * len(per_key):(i + 1) * len(per_key)].view(beta_max, 2, kmax, n) for i, r in enumerate(rots)}
    pall = residues(pq[:kmax] * n_diag)
    total = split[0] * split[1] * split[2]
    pts = [pall[t * kmax:(t + 1) * kmax] if t < n_diag else None for t in range(total)]
    qm = [prm.q[j] for j in range(level + 1)]
    c0, c1 = residues(qm), residues(qm)
    out0 = torch.empty((level, n), dtype=torch.int64, device="cuda")
    out1 = torch.empty((level, n), dtype=torch.int64, device="cuda")
    ws_bytes = H.ckks_lt_workspace_size(P, level, split, pts, H.CKKS_LT_TH_BSGS)
    ws = torch.empty(max(1, ws_bytes), dtype=torch.uint8, device="cuda")
    delta = 2.0 ** prm.log_delta
    stream = torch.cuda.current_stream()

    def step():
        H.ckks_lt_eval(P, level, delta, c0, c1, split, pts, delta, keys, H.CKKS_LT_TH_BSGS, out0, out1, ws, ws_bytes,
                       stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / steps * 1e-3
    # the same steps with every kernel timed: the NTT passes' and BConv's own seconds per LT
    H.ckks_profile_enable((1 << len(H.KERNELS)) - 1)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ntt = sum(H.ckks_profile_read(H.KERNELS.index(k))[1] for k in NTT_KERNELS) * 1e-3 / steps
    bconv = H.ckks_profile_read(H.KERNELS.index("bconv"))[1] * 1e-3 / steps
    H.ckks_profile_enable(0)
    return t, ntt, bconv


def nnls(A, b):
    """Non-negative least squares (scipy's active-set solver)."""
    from scipy.optimize import nnls as _nnls
    x, _ = _nnls(A, b)
    return x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--levels", type=int, nargs="+", default=[8, 16, 24])
    ap.add_argument("--diags", type=int, nargs="+", default=[16, 32, 64, 128, 256])
    ap.add_argument("--per-group", type=int, default=8)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=20)
    args = ap.parse_args()
    import torch
    import paper_2605_17222_amd as H
    import workload as W
    if not torch.cuda.is_available():
        sys.exit("calibrate needs a GPU")
    H.lib()
    prm = W.params_n16()
    P = H.ckks_params_create(prm.log_n, prm.q, prm.p, prm.dnum)
    rows, t_meas, t_ntt, t_bconv, groups, where = [], [], [], [], [], []
    t_start = time.time()
    for level in args.levels:
        for n_diag in args.diags:
            grp = []
            for split in candidates(n_diag, args.per_group, H, prm, level):
                t, tn, tb = time_split(torch, H, W, P, prm, level, split, n_diag, args.steps, args.warmup,
                                       seed=level * 1000 + n_diag)
                rows.append(features(H, prm, level, split, n_diag))
                t_meas.append(t)
                t_ntt.append(tn)
                t_bconv.append(tb)
                where.append((level, n_diag, split))
                grp.append((split, len(t_meas) - 1))
                torch.cuda.empty_cache()
            groups.append((level, n_diag, grp))
            print("level %d, %d diagonals: %d splits timed (%.0f s)" % (level, n_diag, len(grp), time.time() - t_start),
                  file=sys.stderr, flush=True)
    A = np.array(rows)
    t = np.array(t_meas)
    ntt_kernel_limb_s = float(np.sum(t_ntt) / np.sum(A[:, 0]))
    bconv_product_s = float(np.sum(t_bconv) / np.sum(A[:, 1]))
    rest = t - bconv_product_s * A[:, 1]
    y = nnls(A[:, [0, 2, 3]] / t[:, None], rest / t)
    x = np.array([y[0], bconv_product_s, y[1], y[2]])
    pred = A @ x
    err = np.abs(pred - t) / t
    rates = {"ntt_limb_s": x[0], "bconv_product_s": x[1],
             "hbm_bytes_per_s": (1.0 / x[2]) if x[2] > 0 else None, "layer_s": x[3]}
    picks = []
    for level, n_diag, grp in groups:
        best = min(grp, key=lambda g: t[g[1]])
        pick = min(grp, key=lambda g: pred[g[1]])
        picks.append({"level": level, "n_diag": n_diag, "best": list(best[0]), "best_s": float(t[best[1]]),
                      "pick": list(pick[0]), "pick_over_best": float(t[pick[1]] / t[best[1]])})
    print(json.dumps({"rates": rates, "ntt_passes_s_per_limb": ntt_kernel_limb_s, "points": len(t),
                      "mean_rel_err": float(err.mean()),
                      "max_rel_err": float(err.max()),
                      "mean_pick_over_best": float(np.mean([p["pick_over_best"] for p in picks])),
                      "max_pick_over_best": float(np.max([p["pick_over_best"] for p in picks])),
                      "groups": picks,
                      "points_detail": [{"level": w[0], "n_diag": w[1], "split": list(w[2]), "s": float(t[i]),
                                         "predicted_s": float(pred[i])} for i, w in enumerate(where)]}))


if __name__ == "__main__":
    main()
