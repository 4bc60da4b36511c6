#!/usr/bin/env python3
"""Benchmark of the direct-summation hot path on one MI355X.

Default workload (twocomp1m_force): one softened force evaluation of a
two-component Plummer model with N = 2^20 particles (90 % of the mass in an
a = 0.5 core, 10 % in an a = 3 halo, log-uniform masses in [0.1, 10]),
eps = 0.001.  A step is one FP32C force evaluation through the C ABI
(nbody_accel), inputs resident in HBM.  Reported beside it in the same run:
the plain FP64 GPU path and the forward + adjoint (force + VJP) rate, errors
against the FP64 path (all rows) and the CPU oracle (sampled rows), the
roofline of the force kernel and the oracle's own throughput on the host.

Throughput is in ordered pair interactions, N (N - 1) per evaluation; the
fraction of peak uses 20 flops per interaction against the 157.3 TFLOP/s FP32
vector peak of the MI355X.

Other workloads (--workload): plummer64k_fp32c (100 KDK steps, N = 65536),
ensemble512 (512 clusters, 1000 steps in one persistent launch),
grad16k (forward + adjoint of 200 steps, N = 16384), plummer1k_fp64 (10 FP64
steps of N = 1024 with the oracle timed beside it), jerk1m (acceleration + jerk
at N = 2^20 and Hermite steps at N = 65536), hermite6_409600 (the paper's
N = 409600 sixth-order Hermite run: time-to-solution of three steps).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G pair-interactions/s + % FP32 peak, fwd and fwd+adjoint, vs FP64 GPU path"
UNIT = "G pair-interactions/s"
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 vector (packed) peak
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector peak
FLOPS_PER_PAIR = 20          # acceleration-only softened interaction convention
# flops per interaction of the other pair evaluations, counted from their formulas the same way
# (fused multiply-add = 2, inverse square root = 1): the VJP term (d 3, r^2 6, rsqrt 1, r^-2 r^-3
# r^-5 3, u 9, d.u 5, 3 r^-5 d.u 2, g 12, d.w 5, gm 2), acceleration + jerk (d, v 6, r^2 6,
# rsqrt 1, r^-2 r^-3 t 3, alpha 6, a 6, jerk 14) and acceleration + jerk + snap (d, v, acc 9,
# r^2 6, rsqrt 1, r^-2 r^-3 t 3, alpha 6, beta 14, a 6, jerk 14, snap 21)
FLOPS_VJP = 48
FLOPS_JERK = 42
FLOPS_SNAP = 80
# sources of the headline evaluation's kernels (the symmetric FP32C path: staging,
# block-diagonal, half-ring chunks, slot sums and the FP64 rescue); counter figures
# taken on other code are not reported
KERNEL_SOURCES = ("paper_2605_02744_amd/csrc/sym_pairs.hip", "paper_2605_02744_amd/csrc/sym_common.h",
                  "paper_2605_02744_amd/csrc/pair_math.h", "paper_2605_02744_amd/csrc/rescue.hip")


def code_text(src):
    """C++ source without its comments and layout: edits to comments or
    whitespace leave it (and the compiled kernels) unchanged.  The sources hold
    no string literal with comment markers in it."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(" ".join(l.split()) for l in src.splitlines() if l.strip())


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()[:16]


def load_profile(kind, workload):
    """A committed counter summary (profiles/<kind>_<workload>.json) if it was
    taken on the current kernel sources, else None."""
    path = os.path.join(ROOT, "profiles", "%s_%s.json" % (kind, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec


def load_traffic(workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources; else None."""
    rec = load_profile("traffic", workload)
    return rec.get("hbm_bytes_per_launch") if rec else None


def roofline(kernel, flops, ms, peak=FP32_PEAK_TFLOPS, traffic=None, **extra):
    """Roofline entry of a kernel bound by vector-ALU arithmetic: the
    algorithmic flops of one launch (or of the launches that form one
    evaluation) over its duration measured here with HIP events."""
    ach = flops / (ms * 1e-3) / 1e12
    r = {"bound": "alu", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
         "traffic": traffic, "kernel": kernel, "flops_per_launch": flops, "ms_per_launch": round(ms, 5)}
    r.update(extra)
    return r


class GpuEnergy:
    """Reads the energy accumulator of the GPU behind cuda:0 through amdsmi
    (read-only); every method returns None where that is not available."""

    def __init__(self):
        self.h = None
        try:
            import ctypes
            import amdsmi
            hip = ctypes.CDLL("libamdhip64.so")
            buf = ctypes.create_string_buffer(64)
            if hip.hipDeviceGetPCIBusId(buf, 64, 0) != 0:
                return
            bdf = buf.value.decode().lower()
            amdsmi.amdsmi_init(amdsmi.AmdSmiInitFlags.INIT_AMD_GPUS)
            for h in amdsmi.amdsmi_get_processor_handles():
                if str(amdsmi.amdsmi_get_gpu_device_bdf(h)).lower() == bdf:
                    self.h, self.m = h, amdsmi
            if self.h is not None:
                self.joules()
        except Exception:
            self.h = None

    def joules(self):
        if self.h is None:
            return None
        try:
            e = self.m.amdsmi_get_energy_count(self.h)
            return e["energy_accumulator"] * e["counter_resolution"] * 1e-6
        except Exception:
            return None


def idle_power(meter, seconds=2.0):
    """Board power (W) over a quiet window, or None."""
    if meter is None or meter.joules() is None:
        return None
    ja = meter.joules()
    time.sleep(seconds)
    return (meter.joules() - ja) / seconds


def energy_per_call(fn, reps, torch, meter, idle_before=None, settle=2.0, min_busy=4.0):
    """GPU board energy (J) of one call of fn, from the amdsmi energy counter
    over back-to-back calls: `reps` of them, repeated until they have kept the
    GPU busy for at least min_busy seconds.  The counter is refreshed with a
    delay (a read shortly after busy work misses the end of it), so every read
    follows a settling pause of `settle` seconds, and the idle energy of the
    pauses is subtracted: with the idle power measured before the program's
    first GPU work (idle_before) when given, else with that of a one-second
    window just before the calls; the second figure is returned too, since a
    board that has just been busy still draws more.  Returns a dict or None."""
    if meter is None or meter.joules() is None:
        return None
    torch.cuda.synchronize()
    time.sleep(settle)
    ja = meter.joules()
    time.sleep(1.0)
    jb = meter.joules()
    tb = time.perf_counter()
    idle_recent = (jb - ja) / 1.0
    t0 = time.perf_counter()
    calls = 0
    while calls == 0 or time.perf_counter() - t0 < min_busy:
        for _ in range(reps):
            fn()
        calls += reps
        torch.cuda.synchronize()
    reps = calls
    busy = time.perf_counter() - t0
    time.sleep(settle)
    jc = meter.joules()
    window = time.perf_counter() - tb
    idle = idle_before if idle_before is not None else idle_recent
    e_busy = ((jc - jb) - idle * (window - busy)) / reps
    e_recent = ((jc - jb) - idle_recent * (window - busy)) / reps
    return {"joules": e_busy, "busy_s": busy / reps, "idle_w": idle, "idle_w_recent": idle_recent,
            "joules_recent_idle": e_recent, "idle_measured_before_gpu_work": idle_before is not None}


METER = None   # GpuEnergy of cuda:0, where the workload reports energy
IDLE_W = None  # its idle power, measured before any GPU work


def timed(fn, steps, warmup, torch):
    """Runs fn warmup times, then times exactly `steps` calls with HIP events on
    the current stream, bracketed by device synchronisation. Returns (ms/step,
    list of per-call ms, wall ms)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(steps):
        fn()
        evs[k + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    per = [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]
    return sum(per) / steps, per, wall


def rel_err_rows(a, ref):
    num = np.linalg.norm(a - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return num / np.where(den > 0, den, 1.0)


def cpu_baseline_rows(oracle, x, m, eps, budget_s, rng_seed=0):
    """Oracle acceleration rows on a bounded sample of the workload: rows in a
    seeded random order, evaluated in chunks until about budget_s seconds of
    oracle time have been spent."""
    n = m.shape[0]
    order = np.random.default_rng(rng_seed).permutation(n)
    oracle.accel_rows(x, m, order[:8], eps=eps)  # thread pool start-up, untimed
    done, el, refs = 0, 0.0, []
    chunk = 256
    while done < n and el < budget_s:
        rows = order[done:done + chunk]
        t0 = time.perf_counter()
        refs.append(oracle.accel_rows(x, m, rows, eps=eps))
        dt = time.perf_counter() - t0
        el += dt
        done += rows.size
        # aim at chunks of about a tenth of the budget
        chunk = int(max(64, min(8192, rows.size * (0.1 * budget_s) / max(dt, 1e-3))))
    rows = order[:done]
    ref_rows = np.concatenate(refs, axis=1)
    srt = np.argsort(rows)
    return rows[srt], ref_rows[:, srt], el


def bench_force(args, torch, nb):
    import ics
    w = ics.WORKLOADS["twocomp1m_force"]
    n, eps = args.n or w["n"], w["eps"]
    x, _, m = ics.two_component(n, seed=w["seed"])
    dev = torch.device("cuda:0")
    tx = torch.tensor(x, device=dev)
    tm = torch.tensor(m, device=dev)
    a32 = torch.empty_like(tx)
    a64 = torch.empty_like(tx)
    pairs = float(n) * (n - 1)

    tuned = None
    if args.tune:
        tuned = {p: nb.nbody_tune(n, p, args.tune_cache) for p in (args.precision, "fp64")}

    f32 = lambda: nb.nbody_accel(tx, tm, eps=eps, precision=args.precision, out=a32)
    ms, per, wall = timed(f32, args.steps, args.warmup, torch)
    value = pairs / (ms * 1e-3) / 1e9
    c20_tflops = pairs * FLOPS_PER_PAIR / (ms * 1e-3) / 1e12

    res = {"metric": METRIC, "value": round(value, 3), "unit": UNIT, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "twocomp1m_force", "n": n, "eps": eps, "precision": args.precision,
                      "interactions_per_step": pairs, "state": "f64",
                      "flop_convention": "20 flops per ordered interaction"},
           "pct_fp32_peak": round(100 * c20_tflops / FP32_PEAK_TFLOPS, 2),
           "ms_per_step_std": round(float(np.std(per)), 4),
           "wall_ms_timed_region": round(wall, 2)}
    en = energy_per_call(f32, args.steps, torch, METER, IDLE_W)
    if en:
        # GPU board energy of one evaluation (amdsmi energy counter, untimed repeat), for context
        res["gpu_energy"] = {"joules_per_eval": round(en["joules"], 2),
                             "avg_power_w": round(en["joules"] / en["busy_s"], 1),
                             "idle_power_w": round(en["idle_w"], 1),
                             "idle_measured_before_gpu_work": en["idle_measured_before_gpu_work"],
                             "idle_power_w_after_work": round(en["idle_w_recent"], 1),
                             "joules_per_eval_with_idle_after_work": round(en["joules_recent_idle"], 2),
                             "interactions_per_joule": round(pairs / en["joules"], 1)}
    if tuned:
        res["tuned"] = tuned

    if not args.quick:
        # plain FP64 GPU path
        f64 = lambda: nb.nbody_accel(tx, tm, eps=eps, precision="fp64", out=a64)
        ms64, _, _ = timed(f64, max(1, args.steps // 2), 1, torch)
        # forward + adjoint: force then VJP with a fixed cotangent
        wv = torch.tensor(np.random.default_rng(1).standard_normal((3, n)), device=dev)

        def fa():
            nb.nbody_accel(tx, tm, eps=eps, precision=args.precision, out=a32)
            nb.nbody_accel_vjp(tx, tm, wv, eps=eps, precision=args.precision)
        msfa, _, _ = timed(fa, max(1, args.steps // 2), 1, torch)
        res["fp64_path"] = {"value": round(pairs / (ms64 * 1e-3) / 1e9, 3), "unit": UNIT,
                            "ms_per_eval": round(ms64, 4),
                            "pct_fp64_peak": round(100 * pairs * FLOPS_PER_PAIR / (ms64 * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 2),
                            "fp32c_speedup": round(ms64 / ms, 3)}
        res["fwd_adjoint"] = {"value": round(2 * pairs / (msfa * 1e-3) / 1e9, 3), "unit": UNIT,
                              "ms_per_fwd_plus_vjp": round(msfa, 4),
                              "vjp_ms": round(msfa - ms, 4),
                              "note": "force + VJP pair evaluations per second (2 N(N-1) per pass)"}
        # accuracy of this run's result
        nb.nbody_accel(tx, tm, eps=eps, precision="fp64", out=a64)
        nb.nbody_accel(tx, tm, eps=eps, precision=args.precision, out=a32)
        A32, A64 = a32.cpu().numpy(), a64.cpu().numpy()
        e_all = rel_err_rows(A32, A64)
        if args.precision == "fp32c":
            # the same evaluation with the FP64 rescue off: its time and its error, for the
            # rescue's cost and what it buys (the library default keeps it on)
            nb.nbody_set_config(pairs=args.pairs or 0, rescue=2)
            try:
                ms_off, _, _ = timed(f32, max(1, args.steps // 2), 1, torch)
                nb.nbody_accel(tx, tm, eps=eps, precision=args.precision, out=a32)
                e_off = rel_err_rows(a32.cpu().numpy(), A64)
            finally:
                nb.nbody_set_config(pairs=args.pairs or 0)
            res["rescue_off"] = {"ms_per_eval": round(ms_off, 4), "rescue_cost": round(ms / ms_off - 1.0, 4),
                                 "max_rel_vs_fp64gpu": float(e_off.max()),
                                 "rows_over_1e-5": int((e_off > 1e-5).sum()),
                                 "rows_recomputed_in_fp64": int(np.any(A32 != a32.cpu().numpy(), axis=0).sum())}
        res["accuracy"] = {"fp32c_vs_fp64gpu_max_rel": float(e_all.max()),
                           "fp32c_vs_fp64gpu_p99_9": float(np.quantile(e_all, 0.999)),
                           "fp32c_vs_fp64gpu_p99": float(np.quantile(e_all, 0.99)),
                           "fp32c_vs_fp64gpu_median": float(np.median(e_all)),
                           "fp32c_vs_fp64gpu_rows_over_1e-5": int((e_all > 1e-5).sum()),
                           "statistic": "per row |a - a_ref| / |a_ref|, FP64 GPU path over all rows"}

    # roofline of the force evaluation: C20 flops of the N(N-1) ordered interactions
    # / measured duration of one evaluation.  At this size the automatic choice is
    # the symmetric kernel, whose launches (staging, block diagonal, half-ring
    # chunks, slot sums) together form one evaluation: it evaluates each unordered
    # pair once (N(N-1)/2 pair evaluations) and applies it to both particles.
    res["roofline"] = {"bound": "alu", "achieved": round(c20_tflops, 3), "peak": FP32_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(c20_tflops / FP32_PEAK_TFLOPS, 4),
                       "traffic": load_traffic("twocomp1m_force"),
                       "kernel": "sym_accel_kernel<FP32C> (one evaluation: all launches of the symmetric path)",
                       "flops_per_launch": pairs * FLOPS_PER_PAIR, "pair_evaluations": pairs / 2}
    # hardware-counted FP32 work of the same evaluation (SQ_INSTS_VALU_FLOPS_FP32 x 64 lanes from a
    # committed counter run on these sources), over the time measured here
    valu = load_profile("valu", "twocomp1m_force")
    if valu and (args.pairs or 0) != 1 and args.precision == "fp32c" and n == w["n"]:
        cf = valu["fp32_flops_per_eval"]
        res["roofline"]["counted"] = {"fp32_flops_per_interaction": round(cf / pairs, 3),
                                      "achieved": round(cf / (ms * 1e-3) / 1e12, 3),
                                      "frac": round(cf / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4),
                                      "source": "profiles/valu_twocomp1m_force.json"}

    if not args.no_cpu:
        import oracle
        rows, ref_rows, el = cpu_baseline_rows(oracle, x, m, eps, args.cpu_budget)
        rate = len(rows) * (n - 1) / el / 1e9
        cores = oracle.num_threads()
        # the same oracle on one thread, on a smaller sample of the same rows
        oracle.set_num_threads(1)
        try:
            rows1, _, el1 = cpu_baseline_rows(oracle, x, m, eps, max(1.0, args.cpu_budget / 5))
        finally:
            oracle.set_num_threads(cores)
        res["cpu_baseline"] = {"value": round(rate, 4), "unit": UNIT, "cores": cores,
                               "kind": "oracle",
                               "sample": "%d sampled rows x %d j (%.1f s), FP64 Neumaier C oracle" % (len(rows), n - 1, el),
                               "value_1thread": round(len(rows1) * (n - 1) / el1 / 1e9, 4),
                               "sample_1thread": "%d sampled rows x %d j (%.1f s) on one thread" % (len(rows1), n - 1, el1)}
        if "accuracy" in res:
            e32 = rel_err_rows(A32[:, rows], ref_rows)
            e64 = rel_err_rows(A64[:, rows], ref_rows)
            res["accuracy"]["fp32c_vs_oracle_sampled_max_rel"] = float(e32.max())
            res["accuracy"]["fp64gpu_vs_oracle_sampled_max_rel"] = float(e64.max())
            res["accuracy"]["sampled_rows"] = int(len(rows))
            # condition-normalised error |a - a_ref| / (|G| sum_j m_j / s_ij) (the scale of the row's
            # terms) on the rows where FP32C is worst against FP64 and on 256 of the sampled rows
            crow = np.unique(np.concatenate([np.argsort(e_all)[-64:], rows[::max(1, len(rows) // 256)]]))
            cref = oracle.accel_rows(x, m, crow, eps=eps)
            csc = oracle.term_scale_rows(x, m, crow, eps=eps)
            cn = np.linalg.norm(A32[:, crow] - cref, axis=0) / csc
            res["accuracy"]["fp32c_condition_normalised_max"] = float(cn.max())
            res["accuracy"]["fp32c_vs_oracle_worst_rows_max_rel"] = float(rel_err_rows(A32[:, crow], cref).max())
            res["accuracy"]["condition_normalised_rows"] = int(crow.size)
    return res


def bench_kdk64k(args, torch, nb):
    import ics
    w = ics.WORKLOADS["plummer64k_fp32c"]
    n, eps, dt = w["n"], w["eps"], w["dt"]
    x, v, m = ics.plummer(n, seed=w["seed"])
    dev = torch.device("cuda:0")
    tm = torch.tensor(m, device=dev)
    out = {}
    for prec in (args.precision, "fp64"):
        tx, tv = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
        ta = torch.empty_like(tx)
        e0 = nb.nbody_energy(tx, tv, tm, eps=eps).cpu().numpy()
        nb.nbody_step(tx, tv, ta, tm, dt, 0, eps=eps, precision=prec)
        ms, _, wall = timed(lambda: nb.nbody_step(tx, tv, ta, tm, dt, 1, eps=eps, precision=prec, acc_valid=True),
                            args.steps, 0, torch)
        e1 = nb.nbody_energy(tx, tv, tm, eps=eps).cpu().numpy()
        out[prec] = dict(ms=ms, dE=abs((e1[2] - e0[2]) / e0[2]), x=tx.cpu().numpy())
    pairs = float(n) * (n - 1)
    ms = out[args.precision]["ms"]

    # force error of the pair arithmetic at t = 0 and at the final state of its own run (untimed):
    # every row against the FP64 GPU path, sampled rows against the oracle
    def force_error(xs):
        txs = torch.tensor(xs, device=dev)
        a = nb.nbody_accel(txs, tm, eps=eps, precision=args.precision).cpu().numpy()
        a64 = nb.nbody_accel(txs, tm, eps=eps, precision="fp64").cpu().numpy()
        e = rel_err_rows(a, a64)
        r = {"vs_fp64_gpu_max": float(e.max()), "vs_fp64_gpu_p99": float(np.quantile(e, 0.99))}
        if not args.no_cpu:
            import oracle
            rows = np.random.default_rng(11).choice(n, 512, replace=False)
            ref = oracle.accel_rows(xs, m, rows, eps=eps)
            r["vs_oracle_sampled_max"] = float(rel_err_rows(a[:, rows], ref).max())
            r["sampled_rows"] = 512
        return r

    ferr = {"t0": force_error(x), "final": force_error(out[args.precision]["x"])}
    # roofline of the step's dominant launches: one force evaluation at this size and precision (the
    # symmetric path at N = 65536: staging, block diagonal, one half-ring launch, slot sums), timed
    # alone with HIP events on the launch stream; the step adds one kick-drift pass over the state
    txs = torch.tensor(x, device=dev)
    fa = torch.empty_like(txs)
    msf, _, _ = timed(lambda: nb.nbody_accel(txs, tm, eps=eps, precision=args.precision, out=fa), 50, 5, torch)
    roof = roofline("sym_accel_kernel<FP32C> (one evaluation: all launches of the symmetric path)",
                    pairs * FLOPS_PER_PAIR, msf, step_frac=round(pairs * FLOPS_PER_PAIR / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4))
    cpu = None
    if not args.no_cpu:
        import oracle
        oracle.accel_rows(x, m, np.arange(8), eps=eps)  # thread pool start-up, untimed
        t0 = time.perf_counter()
        oracle.kdk(x, v, m, dt, 1, eps=eps)
        el = time.perf_counter() - t0
        cpu = {"value": round(2 * pairs / el / 1e9, 4), "unit": UNIT, "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "one KDK step of the same system: the initial and one further evaluation (%.1f s)" % el}
    return {"metric": METRIC, "value": round(pairs / (ms * 1e-3) / 1e9, 3), "unit": UNIT, "n_gpus": 1,
            "steps": args.steps, "warmup": 0, "ms_per_step": round(ms, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "plummer64k_fp32c", "n": n, "eps": eps, "dt": dt, "precision": args.precision},
            "roofline": roof, "cpu_baseline": cpu,
            "force_error": ferr,
            "pct_fp32_peak": round(100 * pairs * FLOPS_PER_PAIR / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 2),
            "energy_drift": {p: out[p]["dE"] for p in out},
            "fp64_path": {"value": round(pairs / (out["fp64"]["ms"] * 1e-3) / 1e9, 3),
                          "ms_per_step": round(out["fp64"]["ms"], 4)},
            "final_position_maxdiff_vs_fp64": float(np.abs(out[args.precision]["x"] - out["fp64"]["x"]).max())}


def bench_ensemble(args, torch, nb):
    import ics
    w = ics.WORKLOADS["ensemble512"]
    off, epsv, x, v, m = ics.ensemble(w["ncl"], seed=w["seed"], nmin=w["nmin"], nmax=w["nmax"])
    dev = torch.device("cuda:0")
    tm = torch.tensor(m, device=dev)
    sizes = np.diff(off)
    pairs = float((sizes * (sizes - 1)).sum())
    # default: the batched autotuner picks the kernel configuration for this
    # layout (all modes); --bsplit/--split force one instead.  The resident
    # kernel (mode 0, the library default without tuning) is timed beside it.
    tuned = {}
    if args.bsplit is None and not args.split:
        nb.nbody_set_config(rescue=args.rescue)
        tx0, tv0 = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
        for prec in (args.precision, "fp64"):
            tuned[prec] = nb.nbody_tune_batched(off, epsv, tx0, tv0, tm, w["dt"], 50, precision=prec)
        mode = tuned[args.precision]["bsplit"]
    else:
        mode = args.bsplit if args.bsplit is not None else 1
        # bsplit 0 alone would read as "automatic": a pass width forces the resident kernel
        nb.nbody_set_config(bsplit=mode, bpass=args.bpass or (4 if mode == 0 else 0), bitem=args.bitem,
                            rescue=args.rescue)
    res, drift = {}, {}

    def energies(tx, tv):
        # per-cluster total energy E_c (FP64 diagnostics on the GPU), untimed
        out = []
        for c in range(len(sizes)):
            s, e = int(off[c]), int(off[c + 1])
            out.append(nb.nbody_energy(tx[:, s:e].contiguous(), tv[:, s:e].contiguous(), tm[s:e],
                                       eps=float(epsv[c]))[2])
        return torch.stack(out).cpu().numpy()

    for prec in (args.precision, "fp64"):
        tx, tv = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
        ta = torch.empty_like(tx)
        e0 = energies(tx, tv)
        nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, w["dt"], 0, precision=prec)  # plan + a(x)
        steps = args.steps
        # all clusters, all steps: one persistent launch (modes 0-2), or two (mode 3) or three (mode 4)
        # launches per step and one more for the FP32C rescue, captured in a HIP graph and replayed once
        gs = torch.cuda.Stream()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=gs, capture_error_mode="relaxed"):
            nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, w["dt"], steps, precision=prec, acc_valid=True)
        ms, _, _ = timed(graph.replay, 1, 0, torch)
        res[prec] = ms
        rel = np.abs((energies(tx, tv) - e0) / e0)
        drift[prec] = {"max": float(rel.max()), "median": float(np.median(rel))}
    other = {}
    if mode != 0:
        nb.nbody_set_config(bsplit=0, bpass=args.bpass or 4)  # forced, so no tuned choice applies
        tx, tv = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
        ta = torch.empty_like(tx)
        nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, w["dt"], 0, precision=args.precision)
        steps = args.steps
        ms0, _, _ = timed(lambda: nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, w["dt"], steps,
                                                        precision=args.precision, acc_valid=True), 1, 0, torch)
        other = {"resident_kernel_path": {"ms_per_step": round(ms0 / args.steps, 5),
                                          "value": round(pairs * args.steps / (ms0 * 1e-3) / 1e9, 3)}}
    nb.nbody_set_config()
    # the naive alternative: one nbody_step call per cluster (every cluster its own launches), FP64,
    # on contiguous per-cluster copies made beforehand; a few steps, reported per step
    naive_steps = 5
    cl = []
    for c in range(len(sizes)):
        s, e = int(off[c]), int(off[c + 1])
        cl.append((torch.tensor(x[:, s:e], device=dev), torch.tensor(v[:, s:e], device=dev),
                   torch.empty((3, e - s), dtype=torch.float64, device=dev), tm[s:e].contiguous(), float(epsv[c])))
    for cx, cv, ca, cm, ce in cl:
        nb.nbody_step(cx, cv, ca, cm, w["dt"], 0, eps=ce, precision="fp64")

    def naive():
        for cx, cv, ca, cm, ce in cl:
            nb.nbody_step(cx, cv, ca, cm, w["dt"], naive_steps, eps=ce, precision="fp64", acc_valid=True)
    msn, _, _ = timed(naive, 1, 1, torch)
    other["naive_per_cluster_fp64"] = {"ms_per_step": round(msn / naive_steps, 4),
                                       "value": round(pairs * naive_steps / (msn * 1e-3) / 1e9, 3),
                                       "note": "one nbody_step call per cluster, %d steps each" % naive_steps}
    ms = res[args.precision]
    resc = args.precision == "fp32c" and mode in (3, 4) and args.rescue != 2  # the FP32C rescue (default on)
    kname = {0: "ensemble_kernel", 1: "ensemble_kernel (split)", 2: "ens_stream_kernel / ens_wave_kernel",
             3: "ens_waveforce_kernel (one step: publish and force launches%s)" % (", FP64 rescue" if resc else ""),
             4: "esym_force_kernel (one step: publish, force and far-side sum launches%s)"
                % (", FP64 rescue" if resc else "")}[mode]
    # one step of the graph-replayed run: C20 flops of every system's ordered pairs over the step time
    roof = roofline(kname, pairs * FLOPS_PER_PAIR, ms / args.steps)
    cpu = None
    if not args.no_cpu:
        # the oracle's KDK, one step per cluster, clusters in a seeded order until about
        # --cpu-budget seconds have been spent
        import oracle
        order = np.random.default_rng(4).permutation(len(sizes))
        oracle.accel_rows(x[:, :64], m[:64], np.arange(8), eps=float(epsv[0]))  # thread pool start-up
        el, work, ncl = 0.0, 0.0, 0
        for c in order:
            s_, e_ = int(off[c]), int(off[c + 1])
            t0 = time.perf_counter()
            oracle.kdk(x[:, s_:e_], v[:, s_:e_], m[s_:e_], w["dt"], 1, eps=float(epsv[c]))
            el += time.perf_counter() - t0
            work += 2.0 * sizes[c] * (sizes[c] - 1)
            ncl += 1
            if el >= args.cpu_budget:
                break
        cpu = {"value": round(work / el / 1e9, 4), "unit": UNIT, "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "one KDK step (two evaluations) of each of %d clusters in a seeded order (%.1f s)" % (ncl, el)}
    return {"metric": METRIC, "value": round(pairs * args.steps / (ms * 1e-3) / 1e9, 3), "unit": UNIT,
            "n_gpus": 1, "steps": args.steps, "warmup": 0, "ms_per_step": round(ms / args.steps, 5),
            "roofline": roof, "cpu_baseline": cpu,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "ensemble512", "clusters": int(w["ncl"]), "particles": int(off[-1]),
                       "interactions_per_step": pairs, "dt": w["dt"], "precision": args.precision,
                       "fp32c_rescue": resc,
                       "launches": {3: (2 + resc) * args.steps + 1, 4: (3 + resc) * args.steps + 1}.get(mode, 1),
                       "hip_graph": True, "kernel_mode": mode,
                       "autotuned": tuned or None, "bpass": args.bpass, "bitem": args.bitem},
            "pct_fp32_peak": round(100 * pairs * args.steps * FLOPS_PER_PAIR / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 2),
            "energy_drift_per_cluster": drift,
            "fp64_path": {"value": round(pairs * args.steps / (res["fp64"] * 1e-3) / 1e9, 3),
                          "ms_per_step": round(res["fp64"] / args.steps, 5)}, **other}


def bench_grad(args, torch, nb):
    import ics
    w = ics.WORKLOADS["grad16k"]
    n, eps, dt, steps, every = w["n"], w["eps"], w["dt"], w["steps"], w["every"]
    x, v, m = ics.plummer(n, seed=w["seed"])
    xp, vp = ics.perturb(x, v, w["sigma"], seed=w["target_seed"])
    dev = torch.device("cuda:0")
    out = {}
    # warm-up: module load, workspace growth, the first launches and the GPU's clock ramp (a
    # fresh device has been seen to run the first 100 ms several times slower) stay outside
    # the timing: one full forward + backward per precision, twice
    # (the loss's own torch kernels are loaded here too: their first use costs tens of ms)
    # runs: (label, forward precision, sweep precision).  The first is the library's gradient
    # for the requested precision (for FP32C: an FP64 forward and checkpoints, an FP32C reverse
    # sweep, i.e. the FP64 map's gradient), the third the all-FP32C form (the FP32C map's)
    runs = [(args.precision, None, args.precision), ("fp64", "fp64", "fp64"),
            ("all_%s" % args.precision, args.precision, args.precision)]
    wtgt = torch.tensor(xp, device=dev)
    for _ in range(2):
        for _, prec, aprec in runs:
            wx = torch.tensor(x, device=dev, requires_grad=True)
            wv = torch.tensor(v, device=dev, requires_grad=True)
            wm = torch.tensor(m, device=dev, requires_grad=True)
            wT, _ = nb.NBodyTrajectory.apply(wx, wv, wm, dt, steps, every, 1.0, eps, aprec, prec)
            (((wT - wtgt) ** 2).sum() / n).backward()
    torch.cuda.synchronize()
    for label, prec, aprec in runs:
        tgt_x = torch.tensor(xp, device=dev)
        tgt_v = torch.tensor(vp, device=dev)
        tm = torch.tensor(m, device=dev)
        tg = torch.empty_like(tgt_x)
        nb.nbody_step(tgt_x, tgt_v, tg, tm, dt, steps, eps=eps, precision="fp64")
        tx = torch.tensor(x, device=dev, requires_grad=True)
        tv = torch.tensor(v, device=dev, requires_grad=True)
        tmg = torch.tensor(m, device=dev, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xT, _ = nb.NBodyTrajectory.apply(tx, tv, tmg, dt, steps, every, 1.0, eps, aprec, prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = ((xT - tgt_x) ** 2).sum() / n
        torch.cuda.synchronize()
        t1b = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t2 -= t1b - t1  # the loss itself is neither forward nor adjoint
        out[label] = dict(fwd=t1 - t0, bwd=t2 - t1, loss=loss.item(),
                         g={"x": tx.grad.cpu().numpy(), "v": tv.grad.cpu().numpy(), "m": tmg.grad.cpu().numpy()})

    # gradient check (untimed): central differences of the FP64 GPU forward, h = 1e-6, on 64 seeded
    # coordinates (24 position, 24 velocity, 16 mass), error |g - fd| / max(|fd|, 1e-3 max|g|)
    tm = torch.tensor(m, device=dev)
    tg_x, tg_v = torch.tensor(xp, device=dev), torch.tensor(vp, device=dev)
    nb.nbody_step(tg_x, tg_v, torch.empty_like(tg_x), tm, dt, steps, eps=eps, precision="fp64")

    def loss_at(xx, vv, mm):
        px, pv, pm = (torch.tensor(q, device=dev) for q in (xx, vv, mm))
        nb.nbody_step(px, pv, torch.empty_like(px), pm, dt, steps, eps=eps, precision="fp64")
        return float((((px - tg_x) ** 2).sum() / n).item())

    rng = np.random.default_rng(5)
    h = 1e-6
    coords = [("x", int(rng.integers(3)), int(rng.integers(n))) for _ in range(24)]
    coords += [("v", int(rng.integers(3)), int(rng.integers(n))) for _ in range(24)]
    coords += [("m", 0, int(rng.integers(n))) for _ in range(16)]
    worst = {prec: 0.0 for prec in out}
    for kind, c, i in coords:
        xx, vv, mm = x.copy(), v.copy(), m.copy()
        arr = {"x": xx, "v": vv, "m": mm}[kind]
        idx = i if kind == "m" else (c, i)
        arr[idx] += h
        lp = loss_at(xx, vv, mm)
        arr[idx] -= 2 * h
        lq = loss_at(xx, vv, mm)
        fd = (lp - lq) / (2 * h)
        for prec in out:
            g = out[prec]["g"][kind]
            worst[prec] = max(worst[prec], abs(g[idx] - fd) / max(abs(fd), 1e-3 * np.abs(g).max()))
    pairs = float(n) * (n - 1)
    p = out[args.precision]
    # roofline of the gradient's dominant kernel, the VJP of the reverse sweep (vjp_kernel at this size:
    # one launch and its slice sum), timed alone with HIP events in the sweep's configuration; beside it
    # the force kernels of the forward pass (FP64) and of the sweep's recompute (FP32C)
    tx0 = torch.tensor(x, device=dev)
    tw = torch.tensor(np.random.default_rng(3).standard_normal((3, n)), device=dev)
    msv, _, _ = timed(lambda: nb.nbody_accel_vjp(tx0, tm, tw, eps=eps, precision=args.precision), 50, 5, torch)
    fa = torch.empty_like(tx0)
    msa, _, _ = timed(lambda: nb.nbody_accel(tx0, tm, eps=eps, precision=args.precision, out=fa), 50, 5, torch)
    msa64, _, _ = timed(lambda: nb.nbody_accel(tx0, tm, eps=eps, precision="fp64", out=fa), 50, 5, torch)
    vk = "vsym_kernel<%s> (symmetric from 12288 particles: staging, block diagonal, half ring, slot sums; " \
         "48 flops per interaction)" if n >= 12288 and args.precision != "fp64" else "vjp_kernel<%s> (48 flops per interaction)"
    roof = roofline(vk % args.precision.upper(), pairs * FLOPS_VJP, msv,
                    force=roofline("accel_kernel<%s> (with its slice sum and the FP64 rescue)" % args.precision.upper(),
                                   pairs * FLOPS_PER_PAIR, msa),
                    force_fp64=roofline("sym64_kernel (FP64, symmetric from 8192 particles: staging, block "
                                        "diagonal, half ring, slot sum)" if n >= 8192 else "accel_kernel<FP64>",
                                        pairs * FLOPS_PER_PAIR, msa64, peak=FP64_PEAK_TFLOPS))
    cpu = None
    if not args.no_cpu:
        # the oracle's gradient (forward, then the discrete adjoint with two VJPs per step) of a
        # 2-step run of the same system
        import oracle
        cs = 2
        tgt2, _ = oracle.kdk(xp, vp, m, dt, cs, eps=eps)
        t0 = time.perf_counter()
        oracle.loss_grad(x, v, m, tgt2, dt, cs, eps=eps)
        el = time.perf_counter() - t0
        cwork = pairs * (2 * (cs + 1) + 2 * cs)  # two forward passes (loss and adjoint) + 2 VJPs per step
        cpu = {"value": round(cwork / el / 1e9, 4), "unit": UNIT, "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "loss and gradient of a 2-step run of the same system: %d force evaluations and %d "
                         "VJPs (%.1f s)" % (2 * (cs + 1), 2 * cs, el)}
    # forward: steps + 1 evaluations; backward: recompute (steps + nseg) + steps + 1 VJPs
    nseg = -(-steps // every)
    work = pairs * ((steps + 1) + (steps + nseg) + (steps + 1))
    return {"metric": METRIC, "value": round(work / (p["fwd"] + p["bwd"]) / 1e9, 3), "unit": UNIT, "n_gpus": 1,
            "steps": steps, "warmup": 0, "ms_per_step": round(1e3 * (p["fwd"] + p["bwd"]) / steps, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "grad16k", "n": n, "eps": eps, "dt": dt, "every": every, "precision": args.precision},
            "roofline": roof, "cpu_baseline": cpu,
            "fwd_s": p["fwd"], "bwd_s": p["bwd"], "bwd_over_fwd": p["bwd"] / p["fwd"], "loss": p["loss"],
            "gradient_vs_central_differences": {"coords": len(coords), "h": h, "worst_rel": worst[args.precision],
                                                "fp64_worst_rel": worst["fp64"],
                                                "all_%s_worst_rel" % args.precision: worst[runs[2][0]],
                                                "tolerance": 1e-4},
            "forward_precision": "fp64",
            "fp64_path": {"fwd_s": out["fp64"]["fwd"], "bwd_s": out["fp64"]["bwd"], "loss": out["fp64"]["loss"]},
            "all_%s_path" % args.precision: {"forward": args.precision, "adjoint": args.precision,
                                              "fwd_s": out[runs[2][0]]["fwd"], "bwd_s": out[runs[2][0]]["bwd"],
                                              "loss": out[runs[2][0]]["loss"]}}


def bench_kdk1k(args, torch, nb):
    """1024-body Plummer sphere, 10 FP64 KDK steps (dt = 1/128): launch-latency
    bound; reported with the oracle's time for the same run.  ms_per_step is
    the time of one 10-step call."""
    import ics
    import oracle
    w = ics.WORKLOADS["plummer1k_fp64"]
    n, eps, dt, steps = w["n"], w["eps"], w["dt"], w["steps"]
    x, v, m = ics.plummer(n, seed=w["seed"])
    dev = torch.device("cuda:0")
    tm = torch.tensor(m, device=dev)
    # the workload itself, from the initial state, checked against the oracle (untimed)
    tx, tv = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
    ta = torch.empty_like(tx)
    nb.nbody_step(tx, tv, ta, tm, dt, steps, eps=eps, precision="fp64")
    gx, gv = tx.cpu().numpy(), tv.cpu().numpy()
    # timing: 10-step calls continuing the same system (state resident on the GPU), after a
    # few hundred milliseconds of warm-up so that the clocks have ramped up
    sx, sv, sa = tx.clone(), tv.clone(), ta.clone()
    run = lambda: nb.nbody_step(sx, sv, sa, tm, dt, steps, eps=eps, precision="fp64", acc_valid=True)
    ms, _, _ = timed(run, args.steps, max(args.warmup, 1000), torch)
    # the same 10-step call captured once into a HIP graph and replayed (the launches of a short loop
    # cost more than its kernels at this size); one replay is checked bitwise against an eager call
    # from the same state
    gxs, gvs, gas = sx.clone(), sv.clone(), sa.clone()
    gs = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gs, capture_error_mode="relaxed"):
        nb.nbody_step(gxs, gvs, gas, tm, dt, steps, eps=eps, precision="fp64", acc_valid=True)
    s0 = (sx.clone(), sv.clone(), sa.clone())
    for q, q0 in zip((gxs, gvs, gas), s0):
        q.copy_(q0)
    graph.replay()
    ex, ev, ea = (q.clone() for q in s0)
    nb.nbody_step(ex, ev, ea, tm, dt, steps, eps=eps, precision="fp64", acc_valid=True)
    torch.cuda.synchronize()
    replay_same = bool(torch.equal(gxs, ex) and torch.equal(gvs, ev) and torch.equal(gas, ea))
    msg, _, _ = timed(graph.replay, args.steps, 200, torch)
    t0 = time.perf_counter()
    rx, rv = oracle.kdk(x, v, m, dt, steps, eps=eps)
    cpu = time.perf_counter() - t0
    cores = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.kdk(x, v, m, dt, steps, eps=eps)
        cpu1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    pairs = float(n) * (n - 1) * (steps + 1)
    fa = torch.empty_like(tx)
    msf, _, _ = timed(lambda: nb.nbody_accel(tx, tm, eps=eps, precision="fp64", out=fa), 200, 50, torch)
    roof = roofline("accel_kernel<FP64> (launch-latency bound at this size)", float(n) * (n - 1) * FLOPS_PER_PAIR,
                    msf, peak=FP64_PEAK_TFLOPS)
    return {"metric": METRIC, "value": round(pairs / (ms * 1e-3) / 1e9, 3), "unit": UNIT, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "plummer1k_fp64", "n": n, "eps": eps, "dt": dt, "kdk_steps_per_run": steps,
                       "precision": "fp64"},
            "roofline": roof,
            "graph_replay": {"value": round(pairs / (msg * 1e-3) / 1e9, 3), "unit": UNIT,
                             "ms_per_run": round(msg, 4), "bitwise_equal_to_eager": replay_same,
                             "note": "the 10-step call captured into one HIP graph and replayed"},
            "max_abs_dx_vs_oracle": float(np.abs(gx - rx).max()),
            "max_abs_dv_vs_oracle": float(np.abs(gv - rv).max()),
            "cpu_baseline": {"value": round(pairs / cpu / 1e9, 4), "unit": UNIT, "cores": cores,
                             "kind": "oracle", "sample": "the whole 10-step run (%.3f s)" % cpu,
                             "value_1thread": round(pairs / cpu1 / 1e9, 4)}}


def bench_jerk(args, torch, nb):
    """Acceleration + jerk (App. A, Algorithm 3) of an N = 2^20 Plummer sphere
    with velocities, FP32C and FP64, and 20 fourth-order Hermite steps of the
    N = 65536 sphere; each pair evaluation counted once."""
    import ics
    n = args.n or (1 << 20)
    x, v, m = ics.plummer(n, seed=6)
    dev = torch.device("cuda:0")
    tx, tv, tm = (torch.tensor(q, device=dev) for q in (x, v, m))
    pairs = float(n) * (n - 1)
    out = {}
    for prec in (args.precision, "fp64"):
        ms, _, _ = timed(lambda: nb.nbody_accel_jerk(tx, tv, tm, eps=0.001, precision=prec), max(2, args.steps // 3),
                         1, torch)
        out[prec] = ms
    a32, j32 = nb.nbody_accel_jerk(tx, tv, tm, eps=0.001, precision=args.precision)
    a64, j64 = nb.nbody_accel_jerk(tx, tv, tm, eps=0.001, precision="fp64")
    ej = rel_err_rows(j32.cpu().numpy(), j64.cpu().numpy())
    ea = rel_err_rows(a32.cpu().numpy(), a64.cpu().numpy())
    nh = 65536
    xh, vh, mh = ics.plummer(nh, seed=2)
    hx, hv, hm = (torch.tensor(q, device=dev) for q in (xh, vh, mh))
    ha, hj = torch.empty_like(hx), torch.empty_like(hx)
    nb.nbody_step_hermite(hx, hv, ha, hj, hm, 1.0 / 256, 0, eps=0.005, precision=args.precision)
    e0 = nb.nbody_energy(hx, hv, hm, eps=0.005).cpu().numpy()[2]
    hms, _, _ = timed(lambda: nb.nbody_step_hermite(hx, hv, ha, hj, hm, 1.0 / 256, 1, eps=0.005,
                                                     precision=args.precision, acc_valid=True), 20, 0, torch)
    e1 = nb.nbody_energy(hx, hv, hm, eps=0.005).cpu().numpy()[2]
    ms = out[args.precision]
    cpu = None
    if not args.no_cpu:
        # the oracle's acceleration + jerk on rows of the same system in a seeded order, in
        # chunks until about --cpu-budget seconds have been spent
        import oracle
        order = np.random.default_rng(6).permutation(n)
        oracle.accel_jerk_rows(x, v, m, order[:8], eps=0.001)  # thread pool start-up, untimed
        el, done, chunk = 0.0, 0, 256
        while done < n and el < args.cpu_budget:
            rows = order[done:done + chunk]
            t0 = time.perf_counter()
            oracle.accel_jerk_rows(x, v, m, rows, eps=0.001)
            dt = time.perf_counter() - t0
            el += dt
            done += rows.size
            chunk = int(max(64, min(8192, rows.size * (0.1 * args.cpu_budget) / max(dt, 1e-3))))
        cpu = {"value": round(done * (n - 1) / el / 1e9, 4), "unit": UNIT, "cores": oracle.num_threads(),
               "kind": "oracle", "sample": "acceleration and jerk of %d sampled rows x %d j (%.1f s)" % (done, n - 1, el)}
    return {"metric": METRIC, "value": round(pairs / (ms * 1e-3) / 1e9, 3), "unit": UNIT, "n_gpus": 1,
            "cpu_baseline": cpu,
            "steps": max(2, args.steps // 3), "warmup": 1, "ms_per_step": round(ms, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "jerk1m", "n": n, "eps": 0.001, "precision": args.precision},
            "roofline": roofline(("jsym_kernel<%s> (symmetric from 12288 particles: staging, block diagonal, half "
                                  "ring, slot sums; 42 flops per interaction)" if args.precision != "fp64" and args.pairs != 1
                                  else "jerk_kernel<%s> (42 flops per interaction)") % args.precision.upper(),
                                 pairs * FLOPS_JERK, ms),
            "fp64_path": {"value": round(pairs / (out["fp64"] * 1e-3) / 1e9, 3), "ms_per_eval": round(out["fp64"], 4)},
            "accuracy": {"accel_max_rel_vs_fp64": float(ea.max()), "jerk_max_rel_vs_fp64": float(ej.max()),
                         "jerk_p99_rel_vs_fp64": float(np.quantile(ej, 0.99))},
            "hermite64k": {"ms_per_step": round(hms, 4), "energy_drift_20_steps": float(abs((e1 - e0) / e0)),
                           "pairs_per_s_g": round(float(nh) * (nh - 1) / (hms * 1e-3) / 1e9, 3)}}


def bench_hermite6(args, torch, nb):
    """The paper's end-to-end setting: N = 409600 Plummer sphere, three
    sixth-order Hermite steps (start-up evaluations included in the
    time-to-solution), FP32C pairs with FP64 state, and the FP64 path."""
    import ics
    w = ics.WORKLOADS["hermite6_409600"]
    n, eps, dt, steps = args.n or w["n"], w["eps"], w["dt"], w["steps"]
    x, v, m = ics.plummer(n, seed=w["seed"])
    dev = torch.device("cuda:0")
    tm = torch.tensor(m, device=dev)
    pairs = float(n) * (n - 1)
    res = {}
    meter = METER
    for prec in (args.precision, "fp64"):
        # warm-up run (module load, workspace, clock ramp), then the timed run from the initial state
        wx, wv = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
        nb.nbody_step_hermite6(wx, wv, *[torch.empty_like(wx) for _ in range(4)], tm, dt, steps, eps=eps,
                               precision=prec)
        tx, tv = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
        st = [torch.empty_like(tx) for _ in range(4)]
        e0 = nb.nbody_energy(tx, tv, tm, eps=eps).cpu().numpy()[2]
        # time-to-solution: start-up (two evaluations) and `steps` steps
        ms_tts, _, _ = timed(lambda: nb.nbody_step_hermite6(tx, tv, *st, tm, dt, steps, eps=eps, precision=prec),
                             1, 0, torch)
        e1 = nb.nbody_energy(tx, tv, tm, eps=eps).cpu().numpy()[2]
        # per-step time, resuming from the state just reached
        ms_step, _, _ = timed(lambda: nb.nbody_step_hermite6(tx, tv, *st, tm, dt, 1, eps=eps, precision=prec,
                                                              acc_valid=True), args.steps, 0, torch)
        res[prec] = {"time_to_solution_ms": round(ms_tts, 3), "ms_per_step": round(ms_step, 3),
                     "pairs_per_s_g": round(pairs / (ms_step * 1e-3) / 1e9, 3),
                     "energy_error_after_steps": float(abs((e1 - e0) / e0))}
        # energy to solution: the same run repeated from the initial state (untimed)
        def solve():
            sx, sv = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
            nb.nbody_step_hermite6(sx, sv, *[torch.empty_like(sx) for _ in range(4)], tm, dt, steps, eps=eps,
                                   precision=prec)
        en = energy_per_call(solve, max(3, int(3000.0 / ms_tts) + 1), torch, meter, IDLE_W)
        if en:
            res[prec]["gpu_energy_to_solution_j"] = round(en["joules"], 1)
            res[prec]["gpu_edp_j_s"] = round(en["joules"] * ms_tts * 1e-3, 2)
            res[prec]["avg_power_w"] = round(en["joules"] / en["busy_s"], 1)
            res[prec]["idle_power_w"] = round(en["idle_w"], 1)
            res[prec]["gpu_energy_to_solution_j_with_idle_after_work"] = round(en["joules_recent_idle"], 1)
    # roofline of the step's dominant kernel: one acceleration + jerk + snap evaluation (snap_kernel
    # and its slice sum), timed alone with HIP events on the step's input
    accs = torch.tensor(ics.plummer_mean_field(x), device=dev)
    tx0, tv0 = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
    mss, _, _ = timed(lambda: nb.nbody_accel_jerk_snap(tx0, tv0, accs, tm, eps=eps, precision=args.precision),
                      5, 1, torch)
    roof = roofline(("ssym_kernel<%s> (symmetric from 8192 particles: staging, block diagonal, half ring, slot sums; "
                     "80 flops per interaction)" if args.precision != "fp64" and args.pairs != 1
                     else "snap_kernel<%s> (80 flops per interaction)") % args.precision.upper(), pairs * FLOPS_SNAP, mss)
    cpu = None
    if not args.no_cpu:
        import oracle
        rows_all = np.random.default_rng(9).permutation(n)
        acc_h = ics.plummer_mean_field(x)
        oracle.accel_jerk_snap_rows(x, v, acc_h, m, rows_all[:8], eps=eps)  # thread pool start-up
        el, done, chunk = 0.0, 0, 512
        while el < args.cpu_budget and done < n:
            rr = rows_all[done:done + chunk]
            t0 = time.perf_counter()
            oracle.accel_jerk_snap_rows(x, v, acc_h, m, rr, eps=eps)
            el += time.perf_counter() - t0
            done += rr.size
        cpu = {"value": round(done * (n - 1) / el / 1e9, 4), "unit": UNIT, "cores": oracle.num_threads(),
               "kind": "oracle", "sample": "acceleration, jerk and snap of %d sampled rows x %d j (%.1f s)"
                                           % (done, n - 1, el)}
    # per-particle potential (FP64) of the final state: the energy-distribution diagnostic
    ms_phi, _, _ = timed(lambda: nb.nbody_potential(tx, tm, eps=eps), 3, 1, torch)
    res["potential_fp64"] = {"ms": round(ms_phi, 3), "pairs_per_s_g": round(pairs / (ms_phi * 1e-3) / 1e9, 3)}
    r = res[args.precision]
    return {"metric": METRIC, "value": r["pairs_per_s_g"], "unit": UNIT, "n_gpus": 1, "steps": args.steps,
            "warmup": 0, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "hermite6_409600", "n": n, "eps": eps, "dt": dt, "steps_to_solution": steps,
                       "precision": args.precision, "evaluation": "acceleration + jerk + snap per step"},
            "roofline": roof, "cpu_baseline": cpu,
            "paths": res,
            "paper_context": {"time_to_solution_s": {"1 Wormhole n300 chip": 1459.46, "CPU 32 threads": 2875.39},
                              "energy_to_solution_kj": {"1 Wormhole n300 chip": 385.8, "CPU 32 threads": 670.4},
                              "note": "paper's hardware (host CPU and accelerators measured together, energy "
                                      "derived from its EDP column); its time step and initial conditions are "
                                      "not stated; the MI355X figures here are GPU board energy only"}}


def bench_copy(args, torch, nb):
    """A plain device copy of known size, used to calibrate the HBM byte
    counters (FETCH_SIZE / WRITE_SIZE) that price the force kernel's traffic."""
    nbytes = 256 << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    ms, _, _ = timed(lambda: dst.copy_(src), args.steps, args.warmup, torch)
    return {"metric": "copy bandwidth", "value": round(2 * nbytes / (ms * 1e-3) / 1e9, 2), "unit": "GB/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": {"workload": "copy256m", "bytes_read": nbytes, "bytes_written": nbytes}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="twocomp1m_force",
                    choices=["twocomp1m_force", "plummer64k_fp32c", "ensemble512", "grad16k", "copy256m",
                             "plummer1k_fp64", "jerk1m", "hermite6_409600"])
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp32", "fp64"])
    ap.add_argument("--n", type=int, default=None, help="override N of the force workload")
    ap.add_argument("--tune", action="store_true", help="run the autotuner before timing")
    ap.add_argument("--quick", action="store_true", help="force workload: skip FP64, adjoint and accuracy legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work in the CPU baseline")
    ap.add_argument("--split", action="store_true", help="ensemble: split the largest systems over workgroups")
    ap.add_argument("--bsplit", type=int, default=None, choices=[0, 1, 2, 3, 4],
                    help="ensemble kernel: 0 resident systems, 1 resident + split, 2 streamed items, "
                         "3 per-step items of 64, 4 the same with each unordered pair once")
    ap.add_argument("--bpass", type=int, default=0, help="ensemble: i-particles per lane per pass (0 = auto)")
    ap.add_argument("--tune-cache", default=None, help="with --tune: JSON-lines file the tuner appends its choice to")
    ap.add_argument("--bitem", type=int, default=0, help="streamed ensemble: most particles per item (0 = auto)")
    ap.add_argument("--pairs", type=int, default=0, choices=[0, 1, 2],
                    help="force kernel form: 1 ordered, 2 symmetric (each unordered pair once), 0 automatic")
    ap.add_argument("--rescue", type=int, default=0, choices=[0, 1, 2],
                    help="ensemble: the FP32C rescue, 0 automatic (on), 1 on, 2 off")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = {"twocomp1m_force": 10, "plummer64k_fp32c": 100, "ensemble512": 1000, "grad16k": 200,
                      "copy256m": 20, "plummer1k_fp64": 20, "jerk1m": 6, "hermite6_409600": 3}[args.workload]

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    global METER, IDLE_W
    if args.workload in ("twocomp1m_force", "hermite6_409600"):
        # board idle power before this program's first kernel (for the energy figures)
        METER = GpuEnergy()
        IDLE_W = idle_power(METER)
    import paper_2605_02744_amd as nb
    nb.load()
    fn = {"twocomp1m_force": bench_force, "plummer64k_fp32c": bench_kdk64k, "ensemble512": bench_ensemble,
          "grad16k": bench_grad, "copy256m": bench_copy, "plummer1k_fp64": bench_kdk1k,
          "jerk1m": bench_jerk, "hermite6_409600": bench_hermite6}[args.workload]
    if args.pairs:
        nb.nbody_set_config(pairs=args.pairs)
    res = fn(args, torch, nb)
    if args.pairs:
        res.setdefault("config", {})["pairs"] = args.pairs
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
