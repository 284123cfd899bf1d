#!/usr/bin/env python3
"""Benchmark of the SETD pseudo-spectral step on one MI355X.

Workload (the batched configuration the headline metric is quoted on): Model B
(d phi/dt = lap(r phi + u phi^3 - lap phi) + sqrt(2T) div eta, r = -1, u = 1,
T = 0.05) on a 512 x 512 lattice, dx = 1, h = 0.005, SETD2, complex64 state with
FP64-evaluated coefficients, 64 noise realizations advanced together, 2/3
dealiasing, initial phi ~ N(0, 0.05^2) per site.  Inputs are synthetic and
seeded; all fields are resident in HBM before the timed region starts.

One step = one SETD2 transition of every realization: the last-axis pass
(inverse FFT, phi^3, forward FFT) and the axis-0 pass (forward FFT, ETD update
with Philox noise and dealiasing, inverse FFT).

Printed: one JSON line with site-updates/s (a timed segment with no
instrumentation), the roofline record of the dominant kernel (a second timed
segment of the same length, HIP events around every pass on the library's
stream), the plain per-realization FP64 rate of the same model on the same
GPU, the step rates of the KPZ and CGL workloads, a continuous-batching
serving run (p50/p99 job latency, throughput against the same jobs run alone
in FP64, and an audit of 5% of the jobs against solo runs and the oracle), and
the FP64 oracle timed on the host cores over a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_axis0_model_b_512.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_model_b_512.txt")
# VALU issue peak: 256 CUs x 4 SIMDs, a wave64 FP32 instruction (packed FP32
# off) occupies a 16-lane SIMD for 4 cycles, at 2.4 GHz: 614.4e9
# wave-instructions/s (x 64 lanes x 2 flops = 78.6 TFLOP/s, half the packed
# FP32 vector peak of 157.3)
PEAK_VALU_WINST = 256 * 4 / 4 * 2.4e9
KERNEL_SOURCES = ["setd_device.hpp", "setd_kernels.hpp", "setd_launch_impl.hpp", "setd_types.hpp"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2511_22510_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when it is missing or the kernel sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash() or vals.get("kernel") != kernel:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_valu():
    """VALU wave-instructions per launch of each pass kernel from the committed
    rocprofv3 counter summary ({kernel label: count}), empty when it is missing
    or the kernel sources changed since."""
    if not os.path.exists(VALU_FILE):
        return {}
    vals = {}
    for line in open(VALU_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.rsplit("=", 1)   # kernel labels hold "=" themselves
            vals[k.strip()] = v.strip()
    if vals.pop("source_hash", None) != kernel_source_hash():
        return {}
    out = {}
    for k, v in vals.items():
        if k.startswith("valu_insts_per_launch "):
            try:
                out[k.split(" ", 1)[1]] = float(v)
            except ValueError:
                pass
    return out


def time_plan(setd, p, steps, warmup, profile):
    """Time `steps` steps of plan `p` after `warmup` untimed ones, with no
    instrumentation; with `profile`, then time a second segment of `steps`
    steps with HIP events around every pass on the library's stream (per-pass
    durations; the events add a little time per pass, so that segment does not
    give the step rate).  Returns (seconds of the first segment, per-pass
    [total ms, launches] of the second or None, plan info, clean finish,
    seconds of the second segment or None)."""
    import torch
    plan = setd.Plan(p)
    plan.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof, t_prof = None, None
    if profile:
        setd.setd_profile(plan.h, 1, plan.lib)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        plan.step(steps)
        torch.cuda.synchronize()
        t_prof = time.perf_counter() - t2
        prof = setd.setd_profile_read(plan.h, plan.lib)
    out, st = setd.setd_observe(plan.h, setd.OBS_STEP, 4, plan.lib, allow_nonfinite=True)
    ok = (st == setd.SETD_OK) and out[0] == warmup + steps * (2 if profile else 1)
    info = plan.info
    plan.close()
    return t1 - t0, prof, info, ok, t_prof


def serving_run(setd, W, n_jobs, seed, audit=True):
    """A Poisson stream of mixed SETD2 FP32 jobs through the continuous-batching
    server; returns latency percentiles and throughput, the same jobs' rate as
    plain per-job FP64 runs (each job alone, 100 steps), and an audit of the two
    cheapest jobs (5% of 40): the served state against a solo run of the same
    job (bitwise) and against the FP64 oracle (realization 0, all steps)."""
    import numpy as np
    import torch
    trace = W.serving_trace(n_jobs=n_jobs, rate=20.0, seed=seed, steps_range=(1000, 10000))
    srv = setd.Server(arena_bytes=int(64 * 2**30))
    t_start = setd.setd_clock(srv.lib)
    ids = []
    for job in trace:
        while setd.setd_clock(srv.lib) - t_start < job["arrival"]:
            time.sleep(0.0005)
        ids.append((srv.submit(job["problem"], job["steps"]), job))
    srv.drain()
    t_end = setd.setd_clock(srv.lib)
    lat, su = [], 0
    for jid, job in ids:
        times = srv.times(jid)
        lat.append(times[2] - times[0])
        su += W.site_updates(job["problem"], job["steps"])
    out = {"jobs": len(ids), "arrival_rate_per_s": 20.0}
    lat = np.array(lat)
    out.update({
        "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
        "makespan_s": float(t_end - t_start), "site_updates_per_s": float(su / (t_end - t_start)),
    })
    if audit:
        from oracle import oracle as O
        cheap = sorted(ids, key=lambda x: W.site_updates(x[1]["problem"], x[1]["steps"]))[:max(1, n_jobs // 20)]
        rows = []
        for jid, job in cheap:
            p, n = job["problem"], job["steps"]
            served = srv.get(jid, 0)
            solo = setd.Plan(p)
            solo.step(n)
            same = bool(np.array_equal(served, solo.get(0)))
            solo.close()
            o = O.Sim(p, r_first=0, r_count=1)
            o.step(n)
            ref = o.get(0)
            err = float(np.linalg.norm(served - ref) / max(np.linalg.norm(ref), 1e-300))
            rows.append({"job": int(job["id"]), "model": job["model"], "n": list(p["n"]),
                         "realizations": int(p["realizations"]), "steps": int(n),
                         "served_equals_solo": same, "fp32_rel_err_vs_oracle": err})
        out["audit"] = rows
    srv.close()
    torch.cuda.synchronize()
    # plain per-job FP64: every job alone, 100 timed steps after 5 untimed
    su64, t64 = 0, 0.0
    for _, job in ids:
        p = dict(job["problem"], precision=64)
        plan = setd.Plan(p)
        plan.step(5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(100)
        torch.cuda.synchronize()
        t64 += time.perf_counter() - t0
        su64 += W.site_updates(p, 100)
        plan.close()
    out["fp64_per_job_site_updates_per_s"] = su64 / t64
    out["served_fp32_over_fp64_per_job"] = out["site_updates_per_s"] / (su64 / t64)
    return out


LINE_STEPS_PER_LAUNCH = 256


def other_workloads(setd, W, steps):
    """Step rate of the KPZ (1024^2 x 16) and CGL (256^3 x 4) workloads and of
    the 1D lines of the paper's Model A and KPZ figures."""
    res = []
    for name, cfg in (("KPZ 1024x1024, SETD2, FP32, 16 realizations", W.CONFIG_KPZ),
                      ("CGL 256x256x256, SETD2, complex64, 4 realizations", W.CONFIG_CGL)):
        p = W.problem(cfg)
        el, _, info, ok, _ = time_plan(setd, p, steps, 5, profile=False)
        sec = el / steps
        res.append({"workload": name, "site_updates_per_s": float(info.site_updates_per_step) / sec,
                    "ms_per_step": 1e3 * sec, "alg_bytes_per_step": float(info.alg_bytes_per_step),
                    "step_frac": float(info.alg_bytes_per_step / sec / 1e9 / PEAK_HBM_GBS), "ok": bool(ok)})
    return res + line_workloads(setd, W, "ak")


LINES = {"a": ("Model A line N=256 (L=64), SETD1, FP32, 16384 realizations", "LINE_MODEL_A"),
         "k": ("KPZ line N=1024 (L=512), SETD2, FP32, 4096 realizations", "LINE_KPZ")}


def line_workloads(setd, W, which):
    """1D lines: up to 256 steps per launch with the state in registers, so the
    state crosses HBM once per launch and the transforms and noise bound it."""
    res = []
    for key in which:
        name, cfg = LINES[key]
        p = W.problem(getattr(W, cfg))
        k = 8 * LINE_STEPS_PER_LAUNCH
        el, _, info, ok, _ = time_plan(setd, p, k, LINE_STEPS_PER_LAUNCH, profile=False)
        sec = el / k
        res.append({"workload": name, "site_updates_per_s": float(info.site_updates_per_step) / sec,
                    "ms_per_step": 1e3 * sec, "steps_per_launch": LINE_STEPS_PER_LAUNCH,
                    "hbm_bytes_per_launch": float(info.alg_bytes_per_step), "ok": bool(ok)})
    return res


def sde_rate(setd, npaths=1 << 20, nsteps=1000):
    """Scalar SETD-Milstein (Sec. 2) on GBM (lambda 2, mu 1, delta 0, h 2^-10):
    path-steps per second of the batched FP64 kernel, outputs in HBM."""
    import ctypes
    import torch
    lib = setd.load()
    u = torch.empty(npaths, dtype=torch.float64, device="cuda")
    w = torch.empty(npaths, dtype=torch.float64, device="cuda")
    d = setd.setd_sde_desc(setd.SDE_MILSTEIN, 2.0, 0.0, 0.0, 0.0, 1.0, 2.0 ** -10, 1.0, nsteps, npaths, 3)
    stream = torch.cuda.current_stream().cuda_stream
    st = lib.setd_sde_run(ctypes.byref(d), u.data_ptr(), w.data_ptr(), stream)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st |= lib.setd_sde_run(ctypes.byref(d), u.data_ptr(), w.data_ptr(), stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = st == 0 and bool(torch.isfinite(u).all())
    return {"workload": "GBM SETD-Milstein FP64, %d paths x %d steps" % (npaths, nsteps),
            "path_steps_per_s": npaths * nsteps / dt, "seconds": dt, "ok": ok}


def valu_roofline(names, avg_s, dom):
    """The ALU view of each pass: VALU wave-instructions per launch (committed
    counter summary) over the measured launch time, against PEAK_VALU_WINST.
    Transcendental and 64-bit integer multiply instructions take four issue
    slots, so this rate understates how busy the SIMDs are."""
    counts = measured_valu()
    passes = []
    for i, nm in enumerate(names):
        c = counts.get(nm)
        src = nm
        if c is None:
            # the autotuner may pick another variant of the kernel than the
            # counter run did (launch shape only; the counts differ by a few
            # percent): use that variant's count and name it
            same = [k for k in counts if k.split("<")[0] == nm.split("<")[0]]
            if same:
                src = same[0]
                c = counts[src]
        rate = c / avg_s[i] if c else None
        passes.append({"kernel": nm, "valu_insts_per_launch": c, "counted_variant": src if c else None,
                       "achieved": rate, "frac": rate / PEAK_VALU_WINST if rate else None})
    return {"bound": "alu", "unit": "wave-instructions/s", "peak": PEAK_VALU_WINST,
            "achieved": passes[dom]["achieved"], "frac": passes[dom]["frac"], "kernel": names[dom],
            "passes": passes}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the host oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--serving-jobs", type=int, default=40, help="0 skips the serving run")
    ap.add_argument("--no-other", action="store_true", help="skip the KPZ and CGL step rates")
    ap.add_argument("--lines", choices=["a", "k", "ak"], default=None,
                    help="time only the 1D line workloads (a: Model A, k: KPZ) and print them")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 512 MiB device-to-device (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(realizations would shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2511_22510_amd import setd, workloads as W

    torch.cuda.set_device(0)
    if args.lines:
        print(json.dumps({"line_workloads": line_workloads(setd, W, args.lines)}), flush=True)
        return
    if args.copy_calibration:
        src = torch.ones(2**27, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    p = W.problem(W.CONFIG_B)
    elapsed, prof, info, ok, t_prof = time_plan(setd, p, args.steps, args.warmup, profile=True)
    if not ok:
        print("bench: the batched run did not complete cleanly", file=sys.stderr)
        sys.exit(1)
    sites = float(info.site_updates_per_step)
    value = sites * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    rv = int(info.variants[0])
    pass_names = ["k_row_real<float,512,pad=%d,block=%d,pair_groups=%d>" % (3 if rv & 1 else 0, 256 if rv & 2 else 64,
                                                                           1 << ((rv >> 2) & 3)),
                  ("k_axis0r<float,512,tile=%d>" % info.axis_tile[0]) if int(info.variants[1]) >= 4 else
                  "k_axis0<float,512,tile=%d,cols_per_thread=%d>" % (info.axis_tile[0], info.axis_tile[1])]
    tot_ms = prof[:, 0]
    cnt = prof[:, 1]
    dom = int(np.argmax(tot_ms))
    avg_s = tot_ms[dom] / cnt[dom] * 1e-3
    alg = float(info.pass_bytes[dom])
    achieved = alg / avg_s / 1e9
    traffic = measured_traffic(pass_names[dom])
    roofline = {
        "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
        "kernel": pass_names[dom], "avg_launch_us": avg_s * 1e6, "alg_bytes_per_launch": alg,
        "passes": [{"kernel": pass_names[i], "avg_us": float(tot_ms[i] / cnt[i] * 1e3),
                    "alg_bytes": float(info.pass_bytes[i]),
                    "gbs": float(info.pass_bytes[i] / (tot_ms[i] / cnt[i] * 1e-3) / 1e9)}
                   for i in range(len(tot_ms))],
        "timed_with_events_ms_per_step": 1e3 * t_prof / args.steps,
        "valu": valu_roofline(pass_names, tot_ms / cnt * 1e-3, dom),
        "step_alg_bytes": float(info.alg_bytes_per_step),
        "step_frac": float(info.alg_bytes_per_step / (elapsed / args.steps) / 1e9 / PEAK_HBM_GBS),
    }

    line = {
        "metric": "site-updates/s per SETD step, batched FP32 vs plain FP64; p99 job latency",
        "value": value, "unit": "site-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "Model B 512x512, SETD2, complex64 state + FP64 coefficients, "
                               "64 realizations, h=0.005, 2/3 dealiasing",
                   "lattice": [512, 512], "realizations": 64, "scheme": "SETD2", "h": 0.005,
                   "global_batch": 64, "parallelism": "single GPU"},
        "roofline": roofline,
    }

    if not args.no_fp64:
        p64 = W.problem(W.CONFIG_B, precision=64, realizations=1)
        k64 = max(args.steps, 200)
        e64, _, info64, ok64, _ = time_plan(setd, p64, k64, args.warmup, profile=False)
        v64 = float(info64.site_updates_per_step) * k64 / e64
        line["fp64_plain"] = {"workload": "Model B 512x512, SETD2, complex128, 1 realization",
                              "value": v64, "ms_per_step": 1e3 * e64 / k64, "ok": bool(ok64)}
        line["fp32_batched_over_fp64_plain"] = value / v64

    if not args.no_other:
        line["other_workloads"] = other_workloads(setd, W, 50)
        line["sde"] = sde_rate(setd)

    if args.serving_jobs > 0 and hasattr(setd, "Server"):
        line["serving"] = serving_run(setd, W, args.serving_jobs, seed=2024, audit=not args.no_cpu)

    if not args.no_cpu:
        from oracle import oracle as O
        R_cpu, steps_cpu = 8, 300
        o = O.Sim(p, r_first=0, r_count=R_cpu)
        t0 = time.perf_counter()
        o.step(steps_cpu)
        dt = time.perf_counter() - t0
        cores = O.threads()
        line["cpu_baseline"] = {
            "value": 512 * 512 * R_cpu * steps_cpu / dt, "unit": "site-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "Model B 512x512 SETD2 FP64 oracle, %d realizations x %d steps (%.1f s)" % (R_cpu, steps_cpu, dt),
        }

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
