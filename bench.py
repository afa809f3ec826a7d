#!/usr/bin/env python3
"""Benchmark: homomorphic LT evaluations per second on one MI355X.

Workload: one ciphertext at N = 2^16 (2^15 slots), level 24 (q0 of 60 bits,
24 primes of 40 bits), alpha = 9 special primes of 60 bits, dnum = 3, times a
banded matrix with 64 diagonals (offsets 0..63).  A step is one complete
triple-hoisted BSGS LT (split (4,4,4), Algorithm 2) with inputs resident in
HBM; the plain BSGS (8,8) LT on the same data is timed beside it.

Inputs are seeded synthetic residues, uniform in [0, q) per limb: ciphertext,
pre-rotated switching keys and NTT-form plaintext diagonals have exactly the
shapes and value distribution (uniform residues in the NTT domain) of real
ones, and the arithmetic does not depend on their values.  Bit-exactness on
real keys and plaintexts is established by the parity tests, not here.

Printed: one JSON line with LT/s, the roofline of the dominant kernel
(measured with HIP events around its launches, on the launch stream, during
the timed steps), and the CPU oracle timed on this host as a baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CKKS LT evals/s and HBM GB/s at N=2^16, 64 diags; batched vs plain BSGS"
HBM_PEAK_GBS = 8000.0
# rocprofv3 summaries of `bench.py --profile-only --only th` (TH-BSGS (4,4,4)
# at N=2^16, level 24, 64 diagonals), written by
# paper_2605_17222_amd.profiling; their figures are used only while the
# library's sources are the ones that were profiled.
PROFILES = os.path.join(ROOT, "profiles")
PROFILE_TRACE = os.path.join(PROFILES, "kernel_trace_th444_n16_l24_d64.md")
PROFILE_HBM = os.path.join(PROFILES, "hbm_counters_th444_n16_l24_d64.md")
PROFILE_VALU = os.path.join(PROFILES, "valu_counters_th444_n16_l24_d64.md")
PROFILE_LTS = 60  # TH-BSGS LTs in those runs: `--profile-only --only th --steps 10 --warmup 50`
# The kernel (and template instance) behind each timed kernel id in one
# TH-BSGS (4,4,4) step at level 24, as rocprofv3 names it.
# The library's kernels of Algorithm 2's key-switch phases (lines 4-5, 8-14
# fused with the multiply-accumulate, 17-18)
KEYSWITCH_KERNELS = ("keyswitch", "ksmac", "keyswitch_gather")
TH444_KERNEL = {"keyswitch_gather": "ks_gather_kernel<false, 3>", "ksmac": "ksmac_kernel<4, 3, false, false>"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=50,
                    help="untimed steps before each timed single-LT leg (the device's clocks ramp up over the "
                         "first 10-20 steps after an idle gap)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-case", default=None, help=argparse.SUPPRESS)  # one oracle timing, JSON (child process)
    ap.add_argument("--profile-only", action="store_true", help="a few steps, no baseline (for rocprofv3)")
    ap.add_argument("--only", choices=("th", "bsgs", "both"), default="both",
                    help="with --profile-only: which single-LT workload runs (TH-BSGS (4,4,4), plain BSGS (8,8))")
    ap.add_argument("--packed", action="store_true",
                    help="with --profile-only: keys and TH-BSGS plaintexts in the packed layout")
    ap.add_argument("--batch-items", type=int, default=128, help="ragged batch size (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="Poisson serving run length (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--no-chain", action="store_true", help="skip the DFT-like chain")
    ap.add_argument("--no-sweep", action="store_true", help="skip the split sweep (two cost models against time)")
    ap.add_argument("--dense-steps", type=int, default=2,
                    help="timed steps of the dense n = N/2 LT with on-the-fly plaintexts (0: skip)")
    ap.add_argument("--dense-only", action="store_true",
                    help="only the dense on-the-fly LT at N=2^16 (for rocprofv3); prints its JSON")
    return ap.parse_args()


def residue_maker(prm_n, torch, seed):
    """Uniform residues in [0, q) per row, on the device."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)

    def residues(moduli_rows, n=prm_n):
        m = torch.tensor(moduli_rows, dtype=torch.int64, device="cuda").view(-1, 1)
        x = torch.randint(0, 2 ** 62, (len(moduli_rows), n), generator=g, dtype=torch.int64, device="cuda")
        return torch.remainder(x, m, out=x)
    return residues


def device_keys(prm, rots, residues):
    kmax = prm.alpha + prm.max_level + 1
    beta_max = -(-(prm.max_level + 1) // prm.alpha)
    pq = list(prm.p) + list(prm.q)
    return {r: residues(pq[:kmax] * (2 * beta_max)).view(beta_max, 2, kmax, prm.n) for r in rots}


def events_ms(torch, stream, fn, reps):
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), time.perf_counter() - t0


def make_inputs(P, prm, level, split, algo, seed, torch, H, with_pts=True, packed=False):
    """Uniform residues on the device for the ciphertext, keys and plaintexts
    (packed: keys and TH-BSGS plaintexts in the packed resident layout).  The
    keys are views into one allocation, and so are the plaintexts (a resident
    key set and matrix, not hundreds of separate buffers)."""
    import workload as W
    n = prm.n
    pq = list(prm.p) + list(prm.q)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)

    def residues(moduli_rows):
        m = torch.tensor(moduli_rows, dtype=torch.int64, device="cuda").view(-1, 1)
        x = torch.empty((len(moduli_rows), n), dtype=torch.int64, device="cuda")
        for r0 in range(0, len(moduli_rows), 1024):  # bounded temporaries
            r1 = min(len(moduli_rows), r0 + 1024)
            torch.randint(0, 2 ** 62, (r1 - r0, n), generator=g, dtype=torch.int64, device="cuda", out=x[r0:r1])
            torch.remainder(x[r0:r1], m[r0:r1], out=x[r0:r1])
        return x

    qmods = [prm.q[j] for j in range(level + 1)]
    c0, c1 = residues(qmods), residues(qmods)
    kmax = prm.alpha + prm.max_level + 1
    beta_max = -(-(prm.max_level + 1) // prm.alpha)
    if algo == "th":
        rots = W.th_rotations(*split)
        pt_mods = pq[:kmax]
        n_pt = split[0] * split[1] * split[2]
    else:
        rots = W.bsgs_rotations(*split)
        pt_mods = list(prm.q)
        n_pt = split[0] * split[1]
    per_key = pq[:kmax] * (2 * beta_max)
    kall = residues(per_key * len(rots))
    keys = {r: kall[i * len(per_key):(i + 1) * len(per_key)].view(beta_max, 2, kmax, n) for i, r in enumerate(rots)}
    pts = []
    if with_pts:
        pall = residues(pt_mods * n_pt)
        pts = [pall[t * len(pt_mods):(t + 1) * len(pt_mods)] for t in range(n_pt)]
    if packed:
        keys = {r: H.ckks_pack(P, k) for r, k in keys.items()}
        if algo == "th":
            pts = [H.ckks_pack(P, f) for f in pts]
        torch.cuda.synchronize()
    return c0, c1, keys, pts


def step_percentiles(P, prm, level, split, reps, torch, H, warmup=50):
    """Each of `reps` steps bracketed by its own HIP events: p10/p50/p90 ms."""
    c0, c1, keys, pts = make_inputs(P, prm, level, split, "th", 1234, torch, H)
    code = H.CKKS_LT_TH_BSGS
    ws_bytes = H.ckks_lt_workspace_size(P, level, split, pts, code)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out0, out1 = H.empty((level, prm.n)), H.empty((level, prm.n))
    delta = 2.0 ** prm.log_delta
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for _ in range(warmup):
        H.ckks_lt_eval(P, level, delta, c0, c1, split, pts, delta, keys, code, out0, out1, ws, ws_bytes, stream)
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        H.ckks_lt_eval(P, level, delta, c0, c1, split, pts, delta, keys, code, out0, out1, ws, ws_bytes, stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    pick = lambda f: round(ms[min(reps - 1, int(f * reps))], 4)
    del ws, keys, pts
    return {"steps": reps, "p10_ms": pick(0.1), "p50_ms": pick(0.5), "p90_ms": pick(0.9)}


def onfly_leg(P, prm, level, split, n_diag, steps, warmup, torch, H, seed=99, algo="th"):
    """TH-BSGS (or plain BSGS) LT whose diagonals (offsets 0 .. n_diag-1,
    complex uniform [-1, 1] slot vectors resident on the device) the library
    encodes right before each multiply-accumulate; keys and ciphertext uniform
    residues.  One extra step with every kernel timed gives the breakdown."""
    S, n = prm.slots, prm.n
    c0, c1, keys, _ = make_inputs(P, prm, level, split, algo, 4321, torch, H, with_pts=False)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    z = torch.empty((n_diag, S), dtype=torch.complex128, device="cuda")
    zr = torch.view_as_real(z)
    for t0 in range(0, n_diag, 1024):
        zr[t0:t0 + 1024].uniform_(-1.0, 1.0, generator=g)
    slots = [z[t] for t in range(n_diag)]
    code = H.CKKS_LT_TH_BSGS if algo == "th" else H.CKKS_LT_BSGS
    ws_bytes = H.ckks_lt_workspace_size(P, level, split, slots, code, onfly=True)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out0, out1 = H.empty((level, n)), H.empty((level, n))
    delta = 2.0 ** prm.log_delta
    stream = torch.cuda.current_stream()

    def step():
        H.ckks_lt_eval(P, level, delta, c0, c1, split, slots, delta, keys, code, out0, out1, ws, ws_bytes, stream,
                       onfly=True)

    for _ in range(warmup):
        step()
    ms, wall = events_ms(torch, stream, step, steps)
    all_mask = (1 << len(H.KERNELS)) - 1
    H.ckks_profile_enable(all_mask)
    step()
    torch.cuda.synchronize()
    prof = {name: H.ckks_profile_read(k) for k, name in enumerate(H.KERNELS)}
    H.ckks_profile_enable(0)
    K = prm.alpha + level + 1 if algo == "th" else level + 1  # plaintext limbs
    beta_max = -(-(prm.max_level + 1) // prm.alpha)
    kmax = prm.alpha + prm.max_level + 1
    key_bytes = len(keys) * beta_max * 2 * kmax * n * 8
    res = {"algo": algo, "split": list(split), "n_diag": n_diag, "level": level, "keys": len(keys),
           "ms_per_lt": round(ms / steps, 3), "lt_per_s": round(steps / wall, 3),
           "plaintexts_encoded_per_s": round(n_diag * steps / wall, 1),
           "slot_bytes": z.numel() * 16, "key_bytes": key_bytes,
           "resident_plaintext_bytes_avoided": n_diag * K * n * 8, "workspace_bytes": ws_bytes,
           "kernels_ms_per_lt": {k: round(v[1], 3) for k, v in prof.items() if v[0]},
           "recipe": "diagonals complex U[-1,1] on the device (seed %d), keys and ciphertext uniform residues" % seed}
    del ws, z, slots, keys
    torch.cuda.empty_cache()
    return res


def time_lt(P, prm, level, split, algo, steps, warmup, torch, H, profile_mask=0, packed=False):
    c0, c1, keys, pts = make_inputs(P, prm, level, split, algo, 1234, torch, H, packed=packed)
    code = H.CKKS_LT_TH_BSGS if algo == "th" else H.CKKS_LT_BSGS
    ws_bytes = H.ckks_lt_workspace_size(P, level, split, pts, code)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out0 = H.empty((level, prm.n))
    out1 = H.empty((level, prm.n))
    delta = 2.0 ** prm.log_delta
    stream = torch.cuda.current_stream()

    def step():
        H.ckks_lt_eval(P, level, delta, c0, c1, split, pts, delta, keys, code, out0, out1, ws, ws_bytes, stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    H.ckks_profile_enable(profile_mask)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    enqueue_ms = (time.perf_counter() - t0) * 1e3  # host time to enqueue the steps
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_events = ev0.elapsed_time(ev1)
    prof = {}
    if profile_mask:
        for k, name in enumerate(H.KERNELS):
            if profile_mask & (1 << k):
                prof[name] = H.ckks_profile_read(k)
        H.ckks_profile_enable(0)
    return wall, ms_events, prof, ws_bytes, enqueue_ms


# The paper's FPGA latency for its dense LTs (Table VIII, its design, Set-A/B/C): context
# for the same shapes here, not a like-for-like target.
PAPER_FPGA_MS = {"A": 19.44, "B": 726.59, "C": 3113.70}


def paper_sets_leg(steps, torch, H):
    """Dense n = N/2 TH-BSGS LTs at the paper's Set-A/B/C parameters (54-bit
    primes, its splits), top level, diagonals encoded on the fly."""
    import workload as W
    res = {}
    for name in "ABC":
        prm = W.params_paper_set(name)
        split = W.PAPER_SETS[name]["split"]
        P = H.ckks_params_create(prm.log_n, prm.q, prm.p, prm.dnum)
        r = onfly_leg(P, prm, prm.max_level, split, prm.slots, steps, 1, torch, H)
        r["N"] = prm.n
        r["alpha"] = prm.alpha
        r["paper_fpga_ms"] = PAPER_FPGA_MS[name]
        # plain BSGS on the same dense matrix (Q-basis plaintexts, one
        # Decompose per rotation), baby/giant steps as in Table II
        half = (prm.slots.bit_length() - 1) // 2
        bs = (1 << (prm.slots.bit_length() - 1 - half), 1 << half)
        b = onfly_leg(P, prm, prm.max_level, bs, prm.slots, steps, 1, torch, H, algo="bsgs")
        r["plain_bsgs"] = {k: b[k] for k in ("split", "keys", "ms_per_lt", "key_bytes", "kernels_ms_per_lt")}
        res["set_" + name] = r
        del P
        print("set %s done" % name, flush=True, file=sys.stderr)
    return res


def compulsory_bytes(prm, level, split, algo):
    """Keys + plaintexts + ciphertext in and out, uint64 words (each read once)."""
    import workload as W
    n = prm.n
    K = prm.alpha + level + 1
    beta = -(-(level + 1) // prm.alpha)
    if algo == "th":
        nk = len(W.th_rotations(*split))
        pt_limbs = K
        npt = split[0] * split[1] * split[2]
    else:
        nk = len(W.bsgs_rotations(*split))
        pt_limbs = level + 1
        npt = split[0] * split[1]
    words = nk * 2 * beta * K * n + npt * pt_limbs * n + 2 * (level + 1) * n + 2 * level * n
    return words * 8


def host_cpu():
    """Model name, logical CPUs and the CPUs this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count() or 1, "usable_cpus": usable}


def cpu_case(name):
    """One oracle case, timed in this process (the thread count is the
    OpenMP default of the environment): LT evaluation only, keygen,
    encryption and encoding excluded.  Returns a dict (printed as JSON by
    --cpu-case)."""
    import numpy as np
    import oracle as O
    import workload as W
    budget = float(os.environ.get("CKKS_CPU_CASE_SECONDS", "10"))
    if name in ("th444", "bsgs88"):
        w = W.workload_n16(level=24)
    elif name in ("toy_th", "toy_bsgs"):
        w = W.workload_toy()
    elif name == "chain":
        w = None
    else:
        raise ValueError(name)
    if name == "chain":
        prm = W.params_n16()
        o = O.Oracle(prm)
        o.keygen(11)
        delta = 2.0 ** prm.log_delta
        stages = W.dft_chain(3, prm)
        rots = set()
        for st in stages:
            rots |= set(W.th_rotations(*st.split, stride=st.stride, centre=st.centre, slots=prm.slots))
        keys = o.rotkeys(sorted(rots))
        pts = [o.th_plaintexts(st.diags, *st.split, delta, stride=st.stride, centre=st.centre) for st in stages]
        v = W.input_vector(3, prm.slots)
        ct = o.encrypt(24, v, delta, seed=5)

        def run():
            x, lv = ct, 24
            for st, pt in zip(stages, pts):
                x = o.lt_th(lv, x, st.split, pt, keys, stride=st.stride, centre=st.centre)
                lv -= 1
            return x
        what = "4-stage DFT-like chain at N=2^16, level 24 -> 20 (18 keys)"
    else:
        prm = w.params
        o = O.Oracle(prm)
        o.keygen(11)
        delta = 2.0 ** prm.log_delta
        ct = o.encrypt(w.level, w.vector, delta, seed=5)
        if name.endswith("th") or name == "th444":
            keys = o.rotkeys(W.th_rotations(*w.th_split))
            pts = o.th_plaintexts(w.diags, *w.th_split, delta)
            run = lambda: o.lt_th(w.level, ct, w.th_split, pts, keys)  # noqa: E731
            what = "TH-BSGS %s LT, N=2^%d, level %d, %d diagonals" % (w.th_split, prm.log_n, w.level, len(w.diags))
        else:
            keys = o.rotkeys(W.bsgs_rotations(*w.bsgs_split))
            pts = o.bsgs_plaintexts(w.diags, *w.bsgs_split, delta)
            run = lambda: o.lt_bsgs(w.level, ct, w.bsgs_split, pts, keys)  # noqa: E731
            what = "plain BSGS %s LT, N=2^%d, level %d, %d diagonals" % (w.bsgs_split, prm.log_n, w.level,
                                                                         len(w.diags))
    reps, t_total = 0, 0.0
    while reps < 1 or (t_total < budget and reps < 20):
        t0 = time.perf_counter()
        out = run()
        t_total += time.perf_counter() - t0
        reps += 1
    res = {"case": name, "what": what, "reps": reps, "s_per_lt": t_total / reps, "lt_per_s": reps / t_total,
           "threads": int(os.environ.get("OMP_NUM_THREADS", "0")) or None}
    if w is not None:
        lv = w.level
        sc = delta * delta / prm.q[lv]
        res["decrypt_max_err"] = float(np.abs(o.decrypt_slots(out, sc) - W.matvec(w.diags, w.vector)).max())
    return res


def _cpu_subprocess(name, threads, seconds):
    """cpu_case in a child process with OMP_NUM_THREADS = threads (no GPU use)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), CKKS_CPU_CASE_SECONDS=str(seconds))
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-case", name], env=env, capture_output=True,
                       text=True, timeout=600)
    if r.returncode != 0:
        return {"case": name, "threads": threads, "error": (r.stderr or r.stdout)[-400:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    d["threads"] = threads
    return d


def cpu_baseline(prm, level, split, H, specs_batch=None, serving=None):
    """The oracle (plain C++, u128 arithmetic, OpenMP over limbs) timed on this
    host: the benchmark's TH-BSGS (4,4,4) LT on all usable cores (`value`) and
    on one thread, plain BSGS (8,8), the toy configuration and the DFT-like
    chain; the ragged batch and the serving mix are extrapolated from the
    measured (4,4,4) time with the operation-count model (labelled as such)."""
    host = host_cpu()
    allc = host["usable_cpus"]
    th_all = _cpu_subprocess("th444", allc, 8)
    th_one = _cpu_subprocess("th444", 1, 1)
    cases = {"th444_single_thread": th_one,
             "bsgs88_all_cores": _cpu_subprocess("bsgs88", allc, 1),
             "toy_th_all_cores": _cpu_subprocess("toy_th", allc, 2),
             "toy_th_single_thread": _cpu_subprocess("toy_th", 1, 2),
             "chain_all_cores": _cpu_subprocess("chain", allc, 1)}
    res = {"value": th_all.get("lt_per_s"), "unit": "LT/s", "cores": allc, "kind": "oracle",
           "sample": "%s TH-BSGS (4,4,4) LT(s) at N=2^16, level 24, 64 diagonals on %d threads (real keys and "
                     "plaintexts; keygen, encryption and encoding excluded; decrypted max err %s)" % (
                         th_all.get("reps"), allc, "%.1e" % th_all["decrypt_max_err"]
                         if "decrypt_max_err" in th_all else "n/a"),
           "host": host, "th444_all_cores": th_all}
    res.update(cases)
    # extrapolations: oracle seconds scale with the model's modular multiplications
    if "s_per_lt" in th_all:
        base = H.ckks_lt_cost_model(prm.log_n, level, prm.alpha, H.CKKS_LT_TH_BSGS, split)["modmul"]
        t_mm = th_all["s_per_lt"] / base
        if specs_batch:
            mm = sum(H.ckks_lt_cost_model(prm.log_n, lv, prm.alpha, H.CKKS_LT_TH_BSGS, sp)["modmul"]
                     for lv, _, sp in specs_batch)
            res["ragged_batch_extrapolated"] = {"items": len(specs_batch), "s_per_batch": round(mm * t_mm, 2),
                                                "lt_per_s": round(len(specs_batch) / (mm * t_mm), 4),
                                                "note": "extrapolated, not measured: the measured (4,4,4) time per "
                                                        "modular multiplication times each item's model count"}
        if serving:
            mm = sum(H.ckks_lt_cost_model(ln, lv, prm.alpha, H.CKKS_LT_TH_BSGS, (4, 16, 4))["modmul"]
                     for ln, lv in serving) / len(serving)
            res["serving_extrapolated"] = {"mean_s_per_request": round(mm * t_mm, 3),
                                           "max_sustained_req_per_s": round(1.0 / (mm * t_mm), 3),
                                           "note": "extrapolated, not measured: mean model count of the serving "
                                                   "stream's requests (split (4,16,4)) at the measured rate; at "
                                                   "200 req/s offered the oracle would fall behind"}
    return res


def ragged_specs(prm, items, H, seed=77):
    """(level, n_diag, autotuned split) of each item of the ragged batch:
    level ~ U{8..24}, n_diag ~ U{16, 32, 64, 128} (seeded)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64([seed, 5]))
    specs = []
    for _ in range(items):
        level = int(rng.integers(8, 25))
        nd = int(rng.choice([16, 32, 64, 128]))
        sp, _ = H.ckks_lt_autotune(prm.log_n, level, prm.alpha, H.CKKS_LT_TH_BSGS, nd)
        specs.append((level, nd, tuple(sp)))
    return specs


def serving_requests(seconds, rate, seed=2024):
    """The serving stream: (arrival s, ring 0..2 for N = 2^14..2^16, level ~
    U{8..24}, n_diag ~ U{32..256}, ciphertext 0..3) per request (seeded)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64([seed, 6]))
    nreq = int(seconds * rate)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
    reqs = []
    for i in range(nreq):
        g = int(rng.integers(0, 3))
        level = int(rng.integers(8, 25))
        nd = int(rng.integers(32, 257))
        reqs.append((float(arrivals[i]), g, level, nd, int(rng.integers(0, 4))))
    return reqs


SERVING_SPLIT = (4, 16, 4)


def batched_leg(P, prm, items, steps, torch, H, seed=77):
    """Ragged batch: `items` ciphertexts, level ~ U{8..24}, diagonal count ~
    U{16, 32, 64, 128} (banded), each with its own plaintexts and an
    autotuned TH split; keys shared.  A step is one ckks_lt_eval_batch call
    over every item (all of Algorithm 2's lines issued for the whole batch in
    lockstep), timed eagerly and replayed from a HIP graph captured once; if
    the batch's workspace does not fit next to the resident plaintexts, the
    items are split over calls of 32."""
    import workload as W
    residues = residue_maker(prm.n, torch, seed)
    pq = list(prm.p) + list(prm.q)
    specs = ragged_specs(prm, items, H, seed)
    rots = sorted(set().union(*[W.th_rotations(*sp) for _, _, sp in specs]))
    keys = device_keys(prm, rots, residues)
    delta = 2.0 ** prm.log_delta
    batch, pt_bytes = [], 0
    for level, nd, sp in specs:
        K = prm.alpha + level + 1
        qm = [prm.q[j] for j in range(level + 1)]
        pts = [residues(pq[:K]) for _ in range(nd)]  # prefix of the PQ basis: all a level-l LT reads
        pt_bytes += nd * K * prm.n * 8
        batch.append(H.BatchItem(level, delta, residues(qm), residues(qm), sp, pts, delta, keys,
                                 H.empty((level, prm.n)), H.empty((level, prm.n))))
    free, _ = torch.cuda.mem_get_info()
    chunk = items
    wsb = H.ckks_lt_batch_workspace_size(P, batch, H.CKKS_LT_TH_BSGS)
    if wsb > 0.9 * free:
        chunk = 32
    chunks = [batch[i:i + chunk] for i in range(0, len(batch), chunk)]
    wsb = max(H.ckks_lt_batch_workspace_size(P, c, H.CKKS_LT_TH_BSGS) for c in chunks)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def run(st):
        for c in chunks:
            code = H.ckks_lt_eval_batch(P, c, H.CKKS_LT_TH_BSGS, ws, wsb, st)
            assert code == H.CKKS_OK, H.strerror(code)

    run(stream)
    ms, wall = events_ms(torch, stream, lambda: run(stream), steps)
    # the whole step captured once into a HIP graph and replayed
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            run(torch.cuda.current_stream())
    stream.wait_stream(side)
    g.replay()
    ms_g, wall_g = events_ms(torch, stream, g.replay, steps)
    levels = [sp[0] for sp in specs]
    res = {"items": items, "items_per_call": chunk, "steps": steps, "ms_per_batch": round(ms / steps, 3),
           "lt_per_s": round(items * steps / wall, 1), "graph_ms_per_batch": round(ms_g / steps, 3),
           "graph_lt_per_s": round(items * steps / wall_g, 1), "workspace_bytes": wsb,
           "resident_pt_bytes": pt_bytes, "keys": len(rots), "levels": [min(levels), max(levels)],
           "splits": sorted(set("%dx%dx%d" % sp for _, _, sp in specs)),
           "compulsory_bytes": pt_bytes + len(rots) * 2 * 3 * (prm.alpha + prm.max_level + 1) * prm.n * 8 +
           sum(2 * (2 * lv + 1) * prm.n * 8 for lv, _, _ in specs),
           "recipe": "level ~ U{8..24}, n ~ U{16,32,64,128} banded, autotuned TH splits, shared keys, seed %d" % seed}
    res["effective_GB_per_s"] = round(res["compulsory_bytes"] / (ms_g / steps * 1e-3) / 1e9, 1)
    del batch, keys, ws, g
    torch.cuda.empty_cache()
    return res


def same_shape_batch_leg(P, prm, level, split, items, steps, torch, H):
    """`items` copies of the single-LT workload (own ciphertexts and
    plaintexts, shared keys) in one batch."""
    import workload as W
    residues = residue_maker(prm.n, torch, 91)
    pq = list(prm.p) + list(prm.q)
    K = prm.alpha + level + 1
    qm = [prm.q[j] for j in range(level + 1)]
    keys = device_keys(prm, W.th_rotations(*split), residues)
    delta = 2.0 ** prm.log_delta
    nd = split[0] * split[1] * split[2]
    batch = [H.BatchItem(level, delta, residues(qm), residues(qm), split, [residues(pq[:K]) for _ in range(nd)],
                         delta, keys, H.empty((level, prm.n)), H.empty((level, prm.n))) for _ in range(items)]
    wsb = H.ckks_lt_batch_workspace_size(P, batch, H.CKKS_LT_TH_BSGS)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        code = H.ckks_lt_eval_batch(P, batch, H.CKKS_LT_TH_BSGS, ws, wsb, stream)
        assert code == H.CKKS_OK, H.strerror(code)

    step()
    ms, wall = events_ms(torch, stream, step, steps)
    # the same batch captured once into a HIP graph and replayed
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            code = H.ckks_lt_eval_batch(P, batch, H.CKKS_LT_TH_BSGS, ws, wsb, torch.cuda.current_stream())
    assert code == H.CKKS_OK, H.strerror(code)
    stream.wait_stream(side)
    g.replay()
    ms_g, wall_g = events_ms(torch, stream, g.replay, steps)
    del batch, keys, ws, g
    torch.cuda.empty_cache()
    return {"items": items, "ms_per_batch": round(ms / steps, 3), "lt_per_s": round(items * steps / wall, 1),
            "graph_ms_per_batch": round(ms_g / steps, 3), "graph_lt_per_s": round(items * steps / wall_g, 1)}


# TH splits of 64-80 diagonals timed by the sweep: every (n1, n2, n3) with
# n1 n2 n3 = 64 and each factor in {1, 2, 4, 8, 16, 32} that the two models
# rank differently, plus the cube.
SWEEP_SPLITS = ((1, 16, 4), (2, 8, 4), (4, 4, 4), (2, 16, 2), (4, 8, 2), (1, 8, 8), (1, 32, 2), (2, 4, 8),
                (4, 2, 8), (8, 2, 4), (4, 16, 1), (8, 4, 2), (2, 32, 1), (8, 8, 1), (1, 4, 16), (2, 2, 16))


def paper_parallelism(level, K, split):
    """Table III's on-chip parallelism mapped onto this library's schedule:
    all limbs of a polynomial per kernel, up to 8 keys x 8 digit sets per
    key-switch launch, the n3 accumulators of the multiply-accumulate in
    registers."""
    n1, n2, n3 = split
    return dict(m1=1, l1=level + 1, m2=max(1, n1 - 1), l2=K, m3=min(8, max(1, n2 - 1)), m4=min(8, n1), l3=K,
                m5=min(8, n3), l4=K, m6=max(1, n3 - 1), l5=K)


def _ranks(xs):
    order = sorted(range(len(xs)), key=lambda i: xs[i])
    r = [0] * len(xs)
    for pos, i in enumerate(order):
        r[i] = pos
    return r


def _spearman(a, b):
    ra, rb = _ranks(a), _ranks(b)
    n = len(a)
    return 1 - 6 * sum((x - y) ** 2 for x, y in zip(ra, rb)) / (n * (n * n - 1))


def many_diagonals_leg(P, prm, level, steps, warmup, torch, H):
    """LTs with 512 and 1024 diagonals (resident plaintexts): the
    autotuner's TH-BSGS split, its DH-BSGS split (no inner layer, run as
    TH-BSGS (1, n1, n2)), and plain BSGS at its square split.  With this many
    diagonals the inner hoisting layer pays on this device."""
    res = {}
    for n, bsgs in ((512, (32, 16)), (1024, (32, 32))):
        th, th_pred = H.ckks_lt_autotune(prm.log_n, level, prm.alpha, H.CKKS_LT_TH_BSGS, n)
        dh, dh_pred = H.ckks_lt_autotune(prm.log_n, level, prm.alpha, H.CKKS_LT_DH_BSGS, n)
        row = {}
        for name, split, algo in (("th", tuple(th), "th"), ("dh", (1,) + tuple(dh)[:2], "th"),
                                  ("plain_bsgs", bsgs, "bsgs")):
            _, ms, _, _, _ = time_lt(P, prm, level, split, algo, steps, warmup, torch, H)
            row[name] = {"split": list(split), "ms_per_lt": round(ms / steps, 3)}
            torch.cuda.empty_cache()
        row["th_vs_plain_bsgs"] = round(row["plain_bsgs"]["ms_per_lt"] / row["th"]["ms_per_lt"], 3)
        row["th_vs_dh"] = round(row["dh"]["ms_per_lt"] / row["th"]["ms_per_lt"], 3)
        res["n%d" % n] = row
    res["note"] = ("level %d, N=2^%d, uniform-residue inputs; each split timed with all of its n1 n2 n3 "
                   "(TH) or n1 n2 (BSGS) plaintexts present, at least n" % (level, prm.log_n))
    return res


def split_sweep_leg(P, prm, level, steps, warmup, torch, H):
    """Every split of SWEEP_SPLITS timed (events over `steps` LTs after
    `warmup`), priced by the library's predictor (ckks_lt_predict) and by the
    paper's off-chip traffic model (Table III, bytes per LT) turned into time
    by one bandwidth fitted over the sweep (least squares through 0)."""
    K = prm.alpha + level + 1
    rows = []
    for split in SWEEP_SPLITS:
        _, ms, _, _, _ = time_lt(P, prm, level, split, "th", steps, warmup, torch, H)
        tm = H.ckks_th_traffic_model(prm.log_n, level, prm.alpha, split, 64, 64, paper_parallelism(level, K, split))
        rows.append({"split": list(split), "ms": ms / steps,
                     "library_ms": H.ckks_lt_predict(prm.log_n, level, prm.alpha, H.CKKS_LT_TH_BSGS, split, 64) * 1e3,
                     "paper_bytes": tm["total_bytes"]})
        torch.cuda.empty_cache()
    t = [r["ms"] for r in rows]
    b = [r["paper_bytes"] for r in rows]
    ms_per_byte = sum(x * y for x, y in zip(b, t)) / sum(x * x for x in b)
    for r in rows:
        r["paper_ms"] = r["paper_bytes"] * ms_per_byte

    def score(key):
        err = [abs(r[key] - r["ms"]) / r["ms"] for r in rows]
        pick = min(rows, key=lambda r: r[key])
        best = min(t)
        return {"mean_abs_err": round(sum(err) / len(err), 4), "max_abs_err": round(max(err), 4),
                "spearman_vs_measured": round(_spearman([r[key] for r in rows], t), 3),
                "pick": pick["split"], "pick_ms": round(pick["ms"], 4),
                "pick_over_best": round(pick["ms"] / best, 4)}

    best = min(rows, key=lambda r: r["ms"])
    return {"level": level, "n_diag": 64, "steps": steps, "warmup": warmup,
            "measured_best": best["split"], "measured_best_ms": round(best["ms"], 4),
            "library_model": score("library_ms"),
            "paper_table3_model": dict(score("paper_ms"), fitted_GB_per_s=round(1e-6 / ms_per_byte, 1)),
            "splits": [{"split": r["split"], "ms": round(r["ms"], 4), "library_ms": round(r["library_ms"], 4),
                        "paper_bytes": r["paper_bytes"], "paper_ms": round(r["paper_ms"], 4)} for r in rows],
            "note": "library model: 4 rates fitted on MI355X; paper model: Table III's bytes over one fitted bandwidth"}


def chain_leg(P, prm, steps, torch, H):
    """Factored DFT-like chain: 4 sparse LTs (15 diagonals at j 16^s, the
    last stage merged onto 8 offsets), one rescale each, level 24 -> 20."""
    import workload as W
    residues = residue_maker(prm.n, torch, 55)
    pq = list(prm.p) + list(prm.q)
    stages = W.dft_chain(3, prm)
    rots = set()
    for st in stages:
        rots |= set(W.th_rotations(*st.split, stride=st.stride, centre=st.centre, slots=prm.slots))
    keys = device_keys(prm, sorted(rots), residues)
    kmax = prm.alpha + prm.max_level + 1
    delta = 2.0 ** prm.log_delta
    plan = []
    level = 24
    for st in stages:
        n_idx = st.split[0] * st.split[1] * st.split[2]
        S = prm.slots
        present = set((st.stride * (t - st.centre)) % S for t in range(n_idx)) & set(st.diags)
        idx = {(st.stride * (t - st.centre)) % S: t for t in range(n_idx)}
        pts = [None] * n_idx
        for d in present:
            pts[idx[d]] = residues(pq[:kmax])
        out = (H.empty((level, prm.n)), H.empty((level, prm.n)))
        wsb = H.ckks_lt_workspace_size(P, level, st.split, pts, H.CKKS_LT_TH_BSGS, stride=st.stride, centre=st.centre)
        plan.append((level, st, pts, out, wsb))
        level -= 1
    ws = torch.empty(max(p[4] for p in plan), dtype=torch.uint8, device="cuda")
    c0 = residues([prm.q[j] for j in range(25)])
    c1 = residues([prm.q[j] for j in range(25)])
    stream = torch.cuda.current_stream()

    def chain():
        x0, x1, sc = c0, c1, delta
        for level, st, pts, (o0, o1), wsb in plan:
            _, sc = H.ckks_lt_eval(P, level, sc, x0, x1, st.split, pts, delta, keys, H.CKKS_LT_TH_BSGS, o0, o1, ws,
                                   ws.numel(), stream, stride=st.stride, centre=st.centre)
            x0, x1 = o0, o1

    chain()
    ms, wall = events_ms(torch, stream, chain, steps)
    comp = 0
    for level, st, pts, _, _ in plan:
        K = prm.alpha + level + 1
        beta = -(-(level + 1) // prm.alpha)
        nk = len(W.th_rotations(*st.split, stride=st.stride, centre=st.centre, slots=prm.slots))
        npt = sum(1 for f in pts if f is not None)
        comp += (nk * 2 * beta * K + npt * K + 2 * (level + 1) + 2 * level) * prm.n * 8
    del keys, plan, ws
    torch.cuda.empty_cache()
    return {"stages": [{"split": list(st.split), "stride": st.stride, "centre": st.centre, "diagonals": len(st.diags)}
                       for st in stages],
            "keys": len(rots), "ms_per_chain": round(ms / steps, 4), "chains_per_s": round(steps / wall, 2),
            "compulsory_bytes_per_chain": comp, "effective_GB_per_s": round(comp * steps / wall / 1e9, 1)}


def serving_leg(seconds, rate, torch, H, budget_total=200e9, seed=2024, onfly=False):
    """Poisson arrivals (seeded) of single-LT requests: N ~ U{2^14, 2^15,
    2^16}, level ~ U{8..24}, n ~ U{32..256} banded; one resident key set per N
    (split (4,16,4), 21 rotations) and a resident pool of 256 pre-rotated
    plaintexts per N at the top level (prefix-truncated by level and n) --
    or, with onfly, a pool of 256 slot vectors per N that the library encodes
    for each request; requests admitted by the server within an HBM budget of
    budget_total bytes (resident state included)."""
    import workload as W
    split = SERVING_SPLIT
    rings, resident = [], 0
    for log_n in (14, 15, 16):
        prm = W.params_n16(log_n=log_n)
        P = H.ckks_params_create(prm.log_n, prm.q, prm.p, prm.dnum)
        residues = residue_maker(prm.n, torch, seed + log_n)
        pq = list(prm.p) + list(prm.q)
        kmax = prm.alpha + prm.max_level + 1
        keys = device_keys(prm, W.th_rotations(*split), residues)
        if onfly:
            z = torch.empty((256, prm.slots), dtype=torch.complex128, device="cuda")
            torch.view_as_real(z).uniform_(-1.0, 1.0)
            pool = [z[t] for t in range(256)]
            pool_bytes = z.numel() * 16
        else:
            pool = [residues(pq[:kmax]) for _ in range(256)]
            pool_bytes = 256 * kmax * prm.n * 8
        cts = [(residues(list(prm.q)), residues(list(prm.q))) for _ in range(4)]
        resident += sum(k.numel() * 8 for k in keys.values()) + pool_bytes + 4 * 2 * 25 * prm.n * 8
        rings.append((prm, P, keys, pool, cts))
    nreq = int(seconds * rate)
    reqs = []
    out_bytes = 0
    for at, g, level, nd, ci in serving_requests(seconds, rate, seed):
        prm = rings[g][0]
        reqs.append((at, g, level, nd, ci, (H.empty((level, prm.n)), H.empty((level, prm.n)))))
        out_bytes += 2 * level * prm.n * 8
    resident += out_bytes
    free, _ = torch.cuda.mem_get_info()
    arena = int(min(budget_total - resident, free - (8 << 30)))
    torch.cuda.synchronize()

    def run(burst):
        with H.Server(arena, max_batch=8, max_inflight=2) as S:
            rid = [H.ckks_server_add_ring(S, r[1], r[2]) for r in rings]
            t0 = time.perf_counter()
            for at, g, level, nd, ci, (o0, o1) in (reqs[:burst] if burst else reqs):
                if not burst:
                    dt = at - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(dt)
                prm, P, keys, pool, cts = rings[g]
                c0, c1 = cts[ci]
                H.ckks_server_submit(S, rid[g], level, 2.0 ** prm.log_delta, c0, c1, split, pool[:nd],
                                     2.0 ** prm.log_delta, o0, o1, onfly=onfly)
            H.ckks_server_wait_all(S)
            wall = time.perf_counter() - t0
            st = H.ckks_server_stats(S)
        return st, wall

    st, wall = run(0)
    stb, wallb = run(min(nreq, 400))
    res = {"requests": nreq, "rate_req_per_s": rate, "seconds": seconds, "completed": st["completed"],
           "failed": st["failed"], "p50_ms": round(st["p50_s"] * 1e3, 2), "p99_ms": round(st["p99_s"] * 1e3, 2),
           "mean_ms": round(st["mean_s"] * 1e3, 2), "lt_per_s": round(st["completed"] / max(st["span_s"], 1e-9), 1),
           "batches": st["batches"], "max_batch": st["max_batch"], "max_inflight": st["max_inflight"],
           "arena_bytes": arena, "arena_peak_bytes": st["arena_peak"], "resident_bytes": resident,
           "burst": {"requests": min(nreq, 400), "lt_per_s": round(stb["completed"] / max(stb["span_s"], 1e-9), 1),
                     "p50_ms": round(stb["p50_s"] * 1e3, 2), "p99_ms": round(stb["p99_s"] * 1e3, 2)},
           "recipe": "Poisson %.0f req/s, N ~ U{2^14,2^15,2^16}, level ~ U{8..24}, n ~ U{32..256}, split (4,16,4), "
                     "seed %d; max_batch 8, 2 streams; %s" % (rate, seed, "diagonals as resident slot vectors, "
                                                              "encoded on the fly" if onfly else
                                                              "resident plaintext pool")}
    del rings, reqs
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.cpu_case:
        print(json.dumps(cpu_case(args.cpu_case)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2605_17222_amd as H
    import workload as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    H.lib()
    prm = W.params_n16()
    level = 24
    th_split, bs_split = (4, 4, 4), (8, 8)
    P = H.ckks_params_create(prm.log_n, prm.q, prm.p, prm.dnum)
    if args.dense_only:
        r = onfly_leg(P, prm, level, (32, 32, 32), prm.slots, max(1, args.dense_steps), 1, torch, H)
        print(json.dumps({"onfly_dense": r}), flush=True)
        return
    if args.profile_only:
        # calibration for the HBM byte counters: a plain 256 MiB device copy
        src = torch.empty(32 << 20, dtype=torch.int64, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        if args.only in ("th", "both"):
            time_lt(P, prm, level, th_split, "th", max(1, args.steps), args.warmup, torch, H, packed=args.packed)
        if args.only in ("bsgs", "both"):
            time_lt(P, prm, level, bs_split, "bsgs", max(1, args.steps), args.warmup, torch, H, packed=args.packed)
        print("profile run done: %d LTs per algorithm" % (max(1, args.steps) + args.warmup), flush=True)
        return

    all_mask = (1 << len(H.KERNELS)) - 1
    # 1) a short pass with every kernel timed, to find the dominant kernel
    probe_steps = 3
    _, ms_probe, prof, ws_bytes, _ = time_lt(P, prm, level, th_split, "th", probe_steps, args.warmup, torch, H, all_mask)
    dom = max(prof, key=lambda k: prof[k][1])
    dom_id = H.KERNELS.index(dom)
    # 2) the timed region: K steps, HIP events around the dominant kernel only
    wall, ms_ev, prof_dom, _, enq_main = time_lt(P, prm, level, th_split, "th", args.steps, args.warmup, torch, H, 1 << dom_id)
    ms_step = ms_ev / args.steps
    lt_s = args.steps / wall
    # 3) plain BSGS beside it
    bs_steps = max(3, args.steps // 2)
    wall_b, ms_ev_b, _, _, _ = time_lt(P, prm, level, bs_split, "bsgs", bs_steps, args.warmup, torch, H)
    bs_ms = ms_ev_b / bs_steps

    n_l, ms_l, bytes_l = prof_dom[dom]
    avg_s = ms_l / n_l * 1e-3
    K = prm.alpha + level + 1
    # The algorithmic unit of the dominant kernel: for the plaintext
    # multiply-accumulate, the plaintexts it streams (17 MiB per diagonal: K
    # limbs of N words), every present diagonal of the step read once; for
    # the middle key switch fused with it, every operand of lines 8-14 once
    # (the library's own count); for other kernels, each input and output
    # word once (the library's own count)
    if dom == "ptmac":
        unit_bytes = 64 * K * prm.n * 8 / (n_l / args.steps)
        unit = "plaintext bytes per launch (17 MiB per diagonal: %d limbs x %d words x 8 B; 64 diagonals)" % (K, prm.n)
    elif dom == "ksmac":
        unit_bytes = bytes_l / n_l
        unit = ("bytes per launch of Algorithm 2 lines 8-14 fused, each operand once: the 3 middle keys (102 MiB "
                "each), the 4 digit sets (51 MiB each) and their adds (17 MiB each), the 4 unrotated products "
                "(34 MiB each), the 64 plaintexts (17 MiB each) and the 4 accumulator pairs written (34 MiB each)")
    else:
        unit_bytes = bytes_l / n_l
        unit = "algorithmic bytes per launch (each input and output word once)"
    achieved = unit_bytes / avg_s / 1e9
    hbm = None
    try:
        from paper_2605_17222_amd import profiling
        hbm = profiling.current_block(PROFILE_HBM)
        trace_blk = profiling.current_block(PROFILE_TRACE)
        valu_blk = profiling.current_block(PROFILE_VALU)
    except Exception:  # summaries absent or unreadable: no counter figures
        trace_blk = valu_blk = None
    kname = TH444_KERNEL.get(dom)
    traffic = None
    if hbm and kname in hbm["kernels"]:
        traffic = hbm["kernels"][kname]["hbm_bytes"]
    sched = bytes_l / n_l
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE, WRITE_SIZE, copy-calibrated)",
                "traffic_source": os.path.relpath(PROFILE_HBM, ROOT) if traffic else None,
                "traffic_over_unit_bytes": round(traffic / unit_bytes, 3) if traffic else None,
                "algorithmic_unit": unit, "unit_bytes_per_launch": round(unit_bytes),
                "launches_per_step": n_l / args.steps, "avg_launch_us": round(avg_s * 1e6, 2),
                "profiled_avg_launch_us": (trace_blk["kernels"][kname]["avg_us"]
                                           if trace_blk and kname in trace_blk["kernels"] else None),
                "schedule_bytes_per_launch": round(sched),
                "schedule_GB_per_s": round(sched / avg_s / 1e9, 1),
                "schedule_frac": round(sched / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                "schedule_note": ("every operand the launch streams read once: the (a_m, b_m) rotation products, "
                                  "the plaintexts and the accumulators" if dom == "ptmac" else
                                  "the same as the unit: the fused launch materialises nothing" if dom == "ksmac"
                                  else None),
                "share_of_step": round(ms_l / ms_ev, 3)}
    breakdown = {k: {"launches_per_step": v[0] / probe_steps, "ms_per_step": round(v[1] / probe_steps, 4),
                     "GB_per_s": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] else None}
                 for k, v in prof.items() if v[0]}
    # Algorithm 2's key-switch phases together (lines 4-5 in the inner
    # key-switch kernel, 8-14 fused with the multiply-accumulate, 17-18 in
    # the gather kernel): their kernels' algorithmic bytes (each operand
    # once, the library's own count) over their summed kernel time
    ks_names = [k for k in KEYSWITCH_KERNELS if k in prof and prof[k][0]]
    ks_bytes = sum(prof[k][2] for k in ks_names) / probe_steps
    ks_ms = sum(prof[k][1] for k in ks_names) / probe_steps
    keyswitch_phases = {"kernels": ks_names, "bytes_per_step": round(ks_bytes),
                        "ms_per_step": round(ks_ms, 4),
                        "GB_per_s": round(ks_bytes / (ks_ms * 1e-3) / 1e9, 1) if ks_ms else None,
                        "frac_of_hbm_peak": round(ks_bytes / (ks_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if ks_ms else None,
                        "note": "the key-switch kernels of one LT together: algorithmic bytes (each operand once) "
                                "over their summed time, from the pass with every kernel timed"}
    comp = compulsory_bytes(prm, level, th_split, "th")
    whole = {"compulsory_bytes_per_lt": comp, "ms_per_lt": round(ms_step, 4),
             "GB_per_s": round(comp / (ms_step * 1e-3) / 1e9, 1),
             "frac_of_hbm_peak": round(comp / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "hbm_floor_ms": round(comp / (HBM_PEAK_GBS * 1e9) * 1e3, 4),
             "note": "keys + plaintexts + ciphertext in and out, each word once, over the measured step time"}
    # The paper's off-chip traffic model (Table III) for this split, with the
    # reuse this library's kernels get on chip as its parallelism (all limbs
    # of a polynomial per kernel, up to 8 keys x 8 digit sets per key-switch
    # launch, the n3 accumulators of the multiply-accumulate in registers),
    # against the HBM bytes the counters measured per LT and the step time
    par = paper_parallelism(level, K, th_split)
    tm = H.ckks_th_traffic_model(prm.log_n, level, prm.alpha, th_split, 64, 64, par)
    measured = None
    if hbm:
        measured = sum(v["hbm_bytes"] * v["dispatches"] for k, v in hbm["kernels"].items()
                       if not k.startswith("at::")) / PROFILE_LTS
    paper_model = {
        "parallelism": par, "predicted_bytes_per_lt": tm["total_bytes"],
        "predicted_ms_at_hbm_peak": round(tm["total_bytes"] / (HBM_PEAK_GBS * 1e9) * 1e3, 4),
        "measured_hbm_bytes_per_lt": measured,
        "measured_over_predicted_bytes": round(measured / tm["total_bytes"], 3) if measured else None,
        "measured_ms_per_lt": round(ms_step, 4),
        "library_model_predicted_ms": round(H.ckks_lt_predict(prm.log_n, level, prm.alpha, H.CKKS_LT_TH_BSGS,
                                                              th_split, 64) * 1e3, 4),
        "note": "Table III's phases priced for this schedule; its on-chip reuse stands in for the FPGA buffers"}
    # The VALU side, from SQ counters of the same workload (profiles/): per
    # kernel the share of the device's VALU issue slots it used and the share
    # of its waves' lifetimes spent issuing VALU instructions or waiting.
    valu = None
    if valu_blk:
        valu = {"source": os.path.relpath(PROFILE_VALU, ROOT),
                "kernels": {k: {f: v[f] for f in ("valu_issue_frac", "valu_active_per_wave_cycle",
                                                  "wait_per_wave_cycle", "valu_insts_per_wave")}
                            for k, v in valu_blk["kernels"].items()
                            if k.startswith(("ntt_pass", "bconv_kernel", "ks_", "ksmac_kernel", "mac_kernel"))}}
    out = {
        "metric": METRIC, "value": round(lt_s, 2), "unit": "LT/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "single ciphertext TH-BSGS LT, N=2^16, level 24, alpha 9, dnum 3, 64 diagonals, "
                               "split (4,4,4)", "N": prm.n, "level": level, "n_diag": 64, "split": list(th_split)},
        "effective_GB_per_s": round(comp * lt_s / 1e9, 1),
        "compulsory_bytes_per_lt": comp,
        "whole_lt": whole,
        "paper_traffic_model": paper_model,
        "plain_bsgs": {"split": list(bs_split), "ms_per_lt": round(bs_ms, 4), "lt_per_s": round(1e3 / bs_ms, 2),
                       "compulsory_bytes_per_lt": compulsory_bytes(prm, level, bs_split, "bsgs")},
        "th_vs_bsgs_speedup": round(bs_ms / ms_step, 3),
        "workspace_bytes": ws_bytes,
        "roofline": roofline,
        "keyswitch_phases": keyswitch_phases,
        "valu": valu,
        "kernels": breakdown,
        "host_enqueue_ms_per_step": round(enq_main / args.steps, 4),
        "step_ms": step_percentiles(P, prm, level, th_split, 100, torch, H, args.warmup),
    }
    # the split the library's autotuner picks for this workload, timed the same way
    at_split, at_pred = H.ckks_lt_autotune(prm.log_n, level, prm.alpha, H.CKKS_LT_TH_BSGS, 64)
    at_split = tuple(at_split)
    wall_a, ms_a, _, _, enq_a = time_lt(P, prm, level, at_split, "th", args.steps, args.warmup, torch, H)
    out["autotuned_split"] = {"split": list(at_split), "predicted_ms": round(at_pred * 1e3, 4),
                              "ms_per_lt": round(ms_a / args.steps, 4), "lt_per_s": round(args.steps / wall_a, 2),
                              "host_enqueue_ms_per_lt": round(enq_a / args.steps, 4),
                              "compulsory_bytes_per_lt": compulsory_bytes(prm, level, at_split, "th")}
    # the same LTs with keys and TH-BSGS plaintexts resident in the packed
    # layout (limbs of the 40-bit primes in 5 bytes per coefficient): bit-
    # identical results, fewer bytes for the key-switch and MAC kernels
    packed = {}
    for name, split, algo in (("th", th_split, "th"), ("th_autotuned", at_split, "th"), ("plain_bsgs", bs_split, "bsgs")):
        wall_p, ms_p, _, _, _ = time_lt(P, prm, level, split, algo, args.steps, args.warmup, torch, H, packed=True)
        packed[name] = {"split": list(split), "ms_per_lt": round(ms_p / args.steps, 4),
                        "lt_per_s": round(args.steps / wall_p, 2)}
    packed["packed_poly_bytes"] = H.ckks_packed_poly_bytes(P)
    packed["unpacked_poly_bytes"] = (prm.alpha + prm.max_level + 1) * prm.n * 8
    out["packed_resident"] = packed
    print("single-LT legs done", flush=True, file=sys.stderr)
    same = same_shape_batch_leg(P, prm, level, th_split, 32, 5, torch, H)
    same["vs_plain_bsgs"] = round(same["lt_per_s"] / (1e3 / bs_ms), 3)
    out["batched_same_shape"] = same
    if args.batch_items > 0:
        b = batched_leg(P, prm, args.batch_items, 3, torch, H)
        out["batched_ragged"] = b
        print("batched legs done", flush=True, file=sys.stderr)
    if not args.no_sweep:
        out["split_sweep"] = split_sweep_leg(P, prm, level, 10, 20, torch, H)
        print("split sweep done", flush=True, file=sys.stderr)
        out["many_diagonals"] = many_diagonals_leg(P, prm, level, 5, 5, torch, H)
        print("many-diagonals leg done", flush=True, file=sys.stderr)
    if not args.no_chain:
        out["dft_chain"] = chain_leg(P, prm, 10, torch, H)
        print("chain leg done", flush=True, file=sys.stderr)
    # the same workload with its 64 plaintexts encoded on the fly, and the
    # dense n = N/2 LT (every diagonal present) that on-the-fly encoding makes
    # fit on one device, at the largest parameter set's TH split (32, 32, 32)
    out["onfly_banded64"] = onfly_leg(P, prm, level, th_split, 64, args.steps, args.warmup, torch, H)
    print("on-the-fly banded leg done", flush=True, file=sys.stderr)
    if args.dense_steps > 0:
        out["onfly_dense"] = onfly_leg(P, prm, level, (32, 32, 32), prm.slots, args.dense_steps, 1, torch, H)
        print("dense leg done", flush=True, file=sys.stderr)
        out["paper_sets"] = paper_sets_leg(args.dense_steps, torch, H)
        print("paper sets leg done", flush=True, file=sys.stderr)
    if args.serve_seconds > 0:
        out["serving"] = serving_leg(args.serve_seconds, args.serve_rate, torch, H)
        print("serving leg done", flush=True, file=sys.stderr)
        out["serving_onfly"] = serving_leg(args.serve_seconds, args.serve_rate, torch, H, onfly=True)
        print("on-the-fly serving leg done", flush=True, file=sys.stderr)
    if not args.no_cpu_baseline:
        specs_b = ragged_specs(prm, args.batch_items or 128, H)
        serv = [(14 + g, lv) for _, g, lv, _, _ in serving_requests(10.0, 200.0)]
        out["cpu_baseline"] = cpu_baseline(prm, level, th_split, H, specs_b, serv)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
