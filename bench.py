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
PROFILES = os.path.join(ROOT, "profiles")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_model_b_512.txt")
# VALU issue peak: 256 CUs x 4 SIMDs, a wave64 FP32 instruction (packed FP32
# off) occupies a 16-lane SIMD for 4 cycles, at 2.4 GHz: 614.4e9
# wave-instructions/s (x 64 lanes x 2 flops = 78.6 TFLOP/s, half the packed
# FP32 vector peak of 157.3)
PEAK_VALU_WINST = 256 * 4 / 4 * 2.4e9
KERNEL_SOURCES = ["setd_device.hpp", "setd_kernels.hpp", "setd_launch_impl.hpp", "setd_types.hpp"]
# kernel variants the autotuner chose for the workloads timed here on MI355X
TUNED_TABLE = os.path.join(ROOT, "paper_2511_22510_amd", "tuned_mi355x.txt")


def spin_up(torch, seconds=1.0):
    """Device work unrelated to the measured plans for about `seconds` (8192^2
    FP32 products and 256 MiB copies: long kernels, so that a profiler's
    trace stays small), so that a timed segment starts at the GPU's steady
    clocks: right after a plan's setup, the first 400 Model B steps were
    measured 8% slower than the next 400."""
    a = torch.full((8192, 8192), 1.0 / 8192, device="cuda")
    c = torch.empty_like(a)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        torch.mm(a, a, out=c)
        for _ in range(4):
            c.copy_(a)
        torch.cuda.synchronize()
    del a, c


def use_tuned_table():
    """Point the library's variant cache at a private copy of the shipped
    table (the library appends what it tunes to the file it is given), so
    that the plans timed here run the kernel variants the committed counter
    profiles measured; classes the table lacks are tuned as usual."""
    if os.environ.get("SETD_TUNE_CACHE") or not os.path.exists(TUNED_TABLE):
        return None
    import tempfile
    fd, path = tempfile.mkstemp(prefix="setd_tune_", suffix=".txt")
    with os.fdopen(fd, "w") as out, open(TUNED_TABLE) as src:
        out.write(src.read())
    os.environ["SETD_TUNE_CACHE"] = path
    return path


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2511_22510_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of `workload` (profiles/traffic_<workload>.txt), or None when it is
    missing, names another kernel, or the kernel sources changed since."""
    path = os.path.join(PROFILES, "traffic_%s.txt" % workload)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
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


def survey_pass_bytes(p):
    """Bytes each kernel launch of one step must move under the pass model of
    the workload definitions (2/3-pruned spectral arrays, real-space fields in
    LDS only): the state and, for SETD2, the previous nonlinear term read and
    written once, and each transform intermediate that LDS cannot hold read
    and written once.  2D real fields: rows (intermediate in/out; KPZ reads a
    second one), then axis 0 (intermediate(s) in and out, state and history in
    and out).  3D: axis-1 inverse, rows, axis-1 forward, axis 0.  All
    realizations of the plan; per step the list sums to the bytes per
    site-update times the sites."""
    d, n = p["ndim"], list(p["n"])
    e = 8 if p.get("precision", 64) == 32 else 16
    R = int(p.get("realizations", 1))
    cplx = bool(p.get("complex_field", 0))
    da = int(p.get("dealias", 1)) == 1

    def kept(i):
        last = i == d - 1
        K = (n[i] - 1) // 3 if da else (n[i] // 2 if (last and not cplx) else n[i] - 1)
        if last and not cplx:
            return K + 1
        return 2 * K + 1 if da else n[i]

    st = 1
    for i in range(d):
        st *= kept(i)
    arrays = 4 if int(p.get("order", 1)) == 2 else 2   # phi (and F_{n-1}) in and out
    kl = kept(d - 1)
    if p.get("nl") == "none":
        return [2.0 * st * e * R]
    if d == 2:
        pre = n[0] * kl
        npre = 2 if p.get("nl") == "kpz" else 1
        return [float((npre + 1) * pre * e * R), float(((1 + npre) * pre + arrays * st) * e * R)]
    small = n[0] * kept(1) * kl
    big = n[0] * n[1] * kl
    return [float((small + big) * e * R), float(2 * big * e * R), float((big + small) * e * R),
            float((2 * small + arrays * st) * e * R)]


def time_plan(setd, p, steps, warmup, profile, prof_steps=None):
    """Time `steps` steps of plan `p` after `warmup` untimed ones, with no
    instrumentation (wall clock, and HIP events on the plan's stream around the
    segment); with `profile`, then time a second segment of `prof_steps` steps
    with HIP events around every pass on the library's stream (per-pass
    durations; each pair of events adds a dispatch gap inside its bracket, so
    that segment does not give the step rate).  Returns a dict: seconds of the
    first segment (wall, events), per-pass [total ms, launches] of the second
    or None, plan info, clean finish, seconds of the second segment or None,
    the plan's workspace bytes."""
    import torch
    plan = setd.Plan(p)
    # the plan's setup and light work before it (launch-bound runs) leave the
    # clocks low: bring them up with unrelated device work first
    spin_up(torch, 0.3)
    plan.step(warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    plan.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof, t_prof = None, None
    ps = prof_steps or steps
    if profile:
        setd.setd_profile(plan.h, 1, plan.lib)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        plan.step(ps)
        torch.cuda.synchronize()
        t_prof = time.perf_counter() - t2
        prof = setd.setd_profile_read(plan.h, plan.lib)
    out, st = setd.setd_observe(plan.h, setd.OBS_STEP, 4, plan.lib, allow_nonfinite=True)
    ok = (st == setd.SETD_OK) and out[0] == warmup + steps + (ps if profile else 0)
    info = plan.info
    nbytes = plan.nbytes
    plan.close()
    return dict(wall=t1 - t0, ev=ev0.elapsed_time(ev1) * 1e-3, prof=prof, info=info, ok=ok, t_prof=t_prof,
                steps=steps, prof_steps=ps, workspace=nbytes)


def pass_roofline(r, p, names, traffic_workload=None):
    """Roofline record of the passes of one timed plan.  Per-pass launch
    durations come from the HIP events around every launch, less the dispatch
    gap those events add inside each bracket: (sum of the bracketed averages -
    the uninstrumented step time) / passes per step, measured in the same run.
    The per-pass segment always runs on one stream; when the plan steps the
    halves of its realizations on two streams, the uninstrumented step
    overlaps them, so no gap is subtracted (the bracketed durations are an
    upper bound).  achieved = the pass model's bytes (survey_pass_bytes) /
    duration; the bytes this build's storage moves (the plan's own pass bytes:
    a dealiased SETD2 plan keeps one carry array instead of phi and F_{n-1})
    are given beside."""
    import numpy as np
    info = r["info"]
    steps_ev = r["ev"] / max(1, r["steps"])
    tot_ms, cnt = r["prof"][:, 0], r["prof"][:, 1]
    ev_avg = tot_ms / cnt * 1e-3
    npass = len(ev_avg)
    two_streams = int(info.streams) == 2
    gap = 0.0 if two_streams else max(0.0, (float(ev_avg.sum()) - steps_ev) / npass)
    avg = ev_avg - gap
    model = survey_pass_bytes(p)
    moved = [float(info.pass_bytes[i]) for i in range(npass)]
    dom = int(np.argmax(avg))
    passes = [{"kernel": names[i], "avg_us": float(avg[i] * 1e6), "avg_us_events": float(ev_avg[i] * 1e6),
               "alg_bytes": model[i], "moved_bytes": moved[i], "gbs": model[i] / avg[i] / 1e9,
               "gbs_moved": moved[i] / avg[i] / 1e9} for i in range(npass)]
    achieved = model[dom] / avg[dom] / 1e9
    traffic = measured_traffic(names[dom], traffic_workload) if traffic_workload else None
    return {
        "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": names[dom],
        "avg_launch_us": float(avg[dom] * 1e6), "avg_launch_us_events": float(ev_avg[dom] * 1e6),
        "event_gap_us": gap * 1e6, "step_streams": 2 if two_streams else 1,
        "alg_bytes_per_launch": model[dom], "moved_bytes_per_launch": moved[dom],
        "frac_moved": moved[dom] / avg[dom] / 1e9 / PEAK_HBM_GBS,
        "passes": passes,
        "step_alg_bytes": float(sum(model)), "step_moved_bytes": float(sum(moved)),
        "step_frac": float(sum(model) / steps_ev / 1e9 / PEAK_HBM_GBS),
        "step_frac_moved": float(sum(moved) / steps_ev / 1e9 / PEAK_HBM_GBS),
    }, dom, avg


def axis0_name(info, N):
    v = int(info.variants[1])
    if v >= 4:
        # register kernel: variants 4 + 2j / 5 + 2j / 12 + j interleave items in groups of 2^j
        j = v - 12 if v >= 12 else (v - 4) // 2
        return "k_axis0r<float,%d,tile=%d,group=%d>" % (N, info.axis_tile[0], 1 << j)
    return "k_axis0<float,%d,tile=%d,cols_per_thread=%d>" % (N, info.axis_tile[0], info.axis_tile[1])


def pass_names_2d(info, N):
    rv = int(info.variants[0])
    return ["k_row_real<float,%d,pad=%d,block=%d,pair_groups=%d>" % (N, 3 if rv & 1 else 0, 256 if rv & 2 else 64,
                                                                     1 << ((rv >> 2) & 3)),
            axis0_name(info, N)]


def pass_names_3d(info, N):
    return ["k_axis1<inverse,%d>" % N, "k_row_cplx<%d>" % N, "k_axis1<forward,%d>" % N, axis0_name(info, N)]


def log(*a):
    print("bench:", *a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- serving
SERVING_MAKERS = ("A", "B", "KPZ", "CGL")


def serving_calibration(setd, W, steps=30):
    """GPU seconds per step of every (model, lattice, realizations) the serving
    trace draws, each timed alone (SETD2 FP32, the trace's physics)."""
    makers = {"A": W.model_a, "B": W.model_b, "KPZ": W.kpz, "CGL": W.cgl}
    costs = {}
    for name, n in W.SERVING_TYPES:
        for R in (1, 4, 16):
            p = makers[name](n, order=2, precision=32, realizations=R, seed=11)
            r = time_plan(setd, p, steps, 3, profile=False)
            costs[(name, tuple(n), R)] = r["ev"] / steps
    return costs


def job_cost(costs, job):
    p = job["problem"]
    return costs[(job["model"], tuple(p["n"]), int(p["realizations"]))] * job["steps"]


def serve_trace(setd, W, trace):
    """Run a trace through the server in real time; per-job latencies.  The
    server keeps every finished job's final state on the host (the audit reads
    them), so its host budget is raised above the trace's total."""
    os.environ["SETD_SERVER_KEEP_BYTES"] = str(32 << 30)
    srv = setd.Server(arena_bytes=int(64 * 2**30))
    t_start = setd.setd_clock(srv.lib)
    ids = []
    for job in trace:
        while setd.setd_clock(srv.lib) - t_start < job["arrival"]:
            time.sleep(0.0005)
        ids.append((srv.submit(job["problem"], job["steps"]), job))
    srv.drain()
    t_end = setd.setd_clock(srv.lib)
    rows = []
    for jid, job in ids:
        t = srv.times(jid)
        st = srv.poll(jid)
        rows.append(dict(job=job, jid=jid, latency=t[2] - t[0], wait=t[1] - t[0], ok=st == (True, setd.SETD_OK)))
    return srv, rows, t_end - t_start


def latency_summary(W, rows, makespan):
    import numpy as np
    lat = np.array([r["latency"] for r in rows])
    su = sum(W.site_updates(r["job"]["problem"], r["job"]["steps"]) for r in rows)
    return {"jobs": len(rows), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "makespan_s": float(makespan),
            "site_updates_per_s": float(su / makespan), "all_ok": all(r["ok"] for r in rows)}


def serving_run(setd, W, n_jobs, seed, audit=True, n_sustained=100):
    """The mixed SETD2 FP32 job stream through the continuous-batching server:
    the fixed trace (Poisson arrivals at 20 jobs/s, which offers several times
    what one GPU can serve, so its latencies include queueing) and the same job
    mix at a sustainable rate chosen from the measured per-type costs so that
    the offered utilisation is 0.7; per-type breakdown; the same jobs as plain
    per-job FP64 runs; and an audit of every 20th job in arrival order: its
    served state equals a solo run (bitwise) and the solo run's first 100
    steps match the FP64 oracle (realization 0)."""
    import numpy as np
    import torch
    costs = serving_calibration(setd, W)
    log("serving: per-type costs measured")
    trace = W.serving_trace(n_jobs=n_jobs, rate=20.0, seed=seed, steps_range=(1000, 10000))
    mean_cost = float(np.mean([job_cost(costs, j) for j in trace]))
    srv, rows, makespan = serve_trace(setd, W, trace)
    log("serving: %d-job trace at 20 jobs/s done in %.1f s" % (n_jobs, makespan))
    out = {"arrival_rate_per_s": 20.0, "offered_utilisation": 20.0 * mean_cost,
           "mean_job_gpu_s_alone": mean_cost}
    out.update(latency_summary(W, rows, makespan))
    by = {}
    for r in rows:
        j = r["job"]
        b = by.setdefault(j["model"], {"jobs": 0, "site_updates": 0, "gpu_s_alone": 0.0, "lat": []})
        b["jobs"] += 1
        b["site_updates"] += W.site_updates(j["problem"], j["steps"])
        b["gpu_s_alone"] += job_cost(costs, j)
        b["lat"].append(r["latency"])
    tot = sum(b["gpu_s_alone"] for b in by.values())
    out["per_type"] = {k: {"jobs": b["jobs"], "site_updates": b["site_updates"],
                           "gpu_s_alone": b["gpu_s_alone"], "share_of_gpu_time": b["gpu_s_alone"] / tot,
                           "p50_latency_s": float(np.percentile(b["lat"], 50)),
                           "p99_latency_s": float(np.percentile(b["lat"], 99))} for k, b in sorted(by.items())}
    if audit:
        from oracle import oracle as O
        arows = []
        for r in rows[::20]:
            job, jid = r["job"], r["jid"]
            p, n = job["problem"], job["steps"]
            solo = setd.Plan(p)
            solo.step(100)
            s100 = solo.get(0)
            solo.step(n - 100)
            R = int(p["realizations"])
            same = all(np.array_equal(srv.get(jid, q), solo.get(q)) for q in sorted({0, R - 1}))
            solo.close()
            o = O.Sim(p, r_first=0, r_count=1)
            o.step(100)
            ref = o.get(0)
            err = float(np.linalg.norm(s100 - ref) / max(np.linalg.norm(ref), 1e-300))
            arows.append({"job": int(job["id"]), "model": job["model"], "n": list(p["n"]), "realizations": R,
                          "steps": int(n), "served_equals_solo": bool(same), "fp32_rel_err_vs_oracle_100_steps": err})
        out["audit"] = arows
        log("serving: audit of %d jobs done" % len(arows))
    srv.close()
    torch.cuda.synchronize()
    # plain per-job FP64: every job alone, 100 timed steps after 5 untimed
    su64, t64 = 0, 0.0
    for r in rows:
        p = dict(r["job"]["problem"], precision=64)
        tp = time_plan(setd, p, 100, 5, profile=False)
        t64 += tp["wall"]
        su64 += W.site_updates(p, 100)
    out["fp64_per_job_site_updates_per_s"] = su64 / t64
    out["served_fp32_over_fp64_per_job"] = out["site_updates_per_s"] / (su64 / t64)
    log("serving: FP64 per-job rate measured")
    if n_sustained > 0:
        lam = 0.7 / mean_cost
        trace2 = W.serving_trace(n_jobs=n_sustained, rate=lam, seed=seed, steps_range=(1000, 10000))
        srv2, rows2, mk2 = serve_trace(setd, W, trace2)
        srv2.close()
        sus = {"arrival_rate_per_s": lam, "offered_utilisation": lam * mean_cost}
        sus.update(latency_summary(W, rows2, mk2))
        out["sustainable"] = sus
        log("serving: sustainable-rate run (%.2f jobs/s) done in %.1f s" % (lam, mk2))
    return out


LINE_STEPS_PER_LAUNCH = 256


def other_workloads(setd, W, steps):
    """Step rate and pass roofline of the KPZ (1024^2 x 16) and CGL (256^3 x 4)
    workloads, and the 1D lines of the paper's Model A and KPZ figures.  Each
    timed segment holds at least about 20 ms of GPU work after its warm-up
    (KPZ: 4 x steps after 20, CGL: steps after 5), so that the clocks have
    settled after the host-side setup of the plan."""
    res = []
    for name, cfg, nm, k, wu in (("KPZ 1024x1024, SETD2, FP32, 16 realizations", W.CONFIG_KPZ, "kpz_1024", 4, 20),
                                 ("CGL 256x256x256, SETD2, complex64, 4 realizations", W.CONFIG_CGL, "cgl_256", 1, 5)):
        p = W.problem(cfg)
        steps_w = k * steps
        r = time_plan(setd, p, steps_w, wu, profile=True)
        info = r["info"]
        N = int(p["n"][0])
        names = pass_names_2d(info, N) if p["ndim"] == 2 else pass_names_3d(info, N)
        if p["nl"] == "kpz":
            names[0] = names[0].replace("k_row_real", "k_row_real<kpz>")
        rl, dom, _ = pass_roofline(r, p, names, traffic_workload=nm)
        sec = r["wall"] / steps_w
        res.append({"workload": name, "steps": steps_w, "site_updates_per_s": float(info.site_updates_per_step) / sec,
                    "ms_per_step": 1e3 * sec, "working_set_bytes": r["workspace"],
                    "alg_bytes_per_step": rl["step_alg_bytes"], "moved_bytes_per_step": rl["step_moved_bytes"],
                    "step_frac": rl["step_alg_bytes"] / sec / 1e9 / PEAK_HBM_GBS,
                    "step_frac_moved": rl["step_moved_bytes"] / sec / 1e9 / PEAK_HBM_GBS,
                    "roofline": rl, "ok": bool(r["ok"])})
        log("%s: %.4f ms/step" % (name, 1e3 * sec))
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
        r = time_plan(setd, p, k, LINE_STEPS_PER_LAUNCH, profile=False)
        info = r["info"]
        sec = r["wall"] / k
        res.append({"workload": name, "site_updates_per_s": float(info.site_updates_per_step) / sec,
                    "ms_per_step": 1e3 * sec, "steps_per_launch": LINE_STEPS_PER_LAUNCH,
                    "hbm_bytes_per_launch": float(info.alg_bytes_per_step), "ok": bool(r["ok"])})
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
    spin_up(torch, 0.3)
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
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the host oracle baseline and the serving audit")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--serving-jobs", type=int, default=200, help="0 skips the serving run")
    ap.add_argument("--sustained-jobs", type=int, default=100,
                    help="jobs of the serving run at the sustainable rate (0 skips it)")
    ap.add_argument("--no-other", action="store_true", help="skip the other workloads")
    ap.add_argument("--lines", choices=["a", "k", "ak"], default=None,
                    help="time only the 1D line workloads (a: Model A, k: KPZ) and print them")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 512 MiB device-to-device (reference kernel for HBM counters)")
    ap.add_argument("--retune", action="store_true",
                    help="tune every plan afresh instead of loading the shipped variant table")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(realizations would shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    tuned = None if args.retune else use_tuned_table()
    import torch
    from paper_2511_22510_amd import setd, workloads as W

    torch.cuda.set_device(0)
    spin_up(torch)
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
    # the per-pass segment is at least 200 steps, so that the event-gap
    # correction (a difference of two timings) is well resolved
    r = time_plan(setd, p, args.steps, args.warmup, profile=True, prof_steps=max(args.steps, 200))
    if not r["ok"]:
        print("bench: the batched run did not complete cleanly", file=sys.stderr)
        sys.exit(1)
    info = r["info"]
    sites = float(info.site_updates_per_step)
    elapsed = r["wall"]
    value = sites * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    names = pass_names_2d(info, 512)
    roofline, dom, avg = pass_roofline(r, p, names, traffic_workload="model_b_512")
    roofline["valu"] = valu_roofline(names, avg, dom)
    log("Model B 512^2 x 64: %.4f ms/step" % ms_per_step)

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
        "working_set_bytes": r["workspace"],
        "kernel_variants": ("shipped table paper_2511_22510_amd/tuned_mi355x.txt" if tuned
                            else "autotuned in this run"),
    }

    # the same model with a working set beyond the 256 MB Infinity Cache
    p256 = W.problem(W.CONFIG_B, realizations=256)
    # (at least 200 steps after 20: a steady-state figure whatever the
    # headline's step count)
    k256 = max(args.steps // 4, 200)
    r2 = time_plan(setd, p256, k256, 20, profile=True, prof_steps=100)
    rl2, _, _ = pass_roofline(r2, p256, pass_names_2d(r2["info"], 512), traffic_workload="model_b_512_r256")
    sec2 = r2["wall"] / k256
    line["beyond_infinity_cache"] = {
        "workload": "Model B 512x512, SETD2, complex64, 256 realizations", "steps": k256,
        "working_set_bytes": r2["workspace"],
        "ms_per_step": 1e3 * sec2, "site_updates_per_s": float(r2["info"].site_updates_per_step) / sec2,
        "roofline": rl2, "ok": bool(r2["ok"])}
    log("Model B 512^2 x 256: %.4f ms/step" % (1e3 * sec2))

    if not args.no_fp64:
        p64 = W.problem(W.CONFIG_B, precision=64, realizations=1)
        k64 = max(args.steps, 200)
        r64 = time_plan(setd, p64, k64, args.warmup, profile=False)
        v64 = float(r64["info"].site_updates_per_step) * k64 / r64["wall"]
        line["fp64_plain"] = {"workload": "Model B 512x512, SETD2, complex128, 1 realization",
                              "value": v64, "ms_per_step": 1e3 * r64["wall"] / k64, "ok": bool(r64["ok"])}
        line["fp32_batched_over_fp64_plain"] = value / v64
        # the first workload as specified: Model A 64^2, plain SETD1, FP64, one
        # realization, all 1000 steps
        pa = W.problem(W.CONFIG_A)
        ra = time_plan(setd, pa, W.CONFIG_A["steps"], args.warmup, profile=False)
        line["config_a"] = {"workload": "Model A 64x64, SETD1, FP64, 1 realization, 1000 steps",
                            "seconds": ra["wall"], "ms_per_step": 1e3 * ra["wall"] / W.CONFIG_A["steps"],
                            "steps_per_s": W.CONFIG_A["steps"] / ra["wall"],
                            "site_updates_per_s": 64 * 64 * W.CONFIG_A["steps"] / ra["wall"], "ok": bool(ra["ok"])}
        log("FP64 plain and Model A 64^2 timed")

    if not args.no_other:
        line["other_workloads"] = other_workloads(setd, W, 50)
        line["sde"] = sde_rate(setd)

    if args.serving_jobs > 0:
        line["serving"] = serving_run(setd, W, args.serving_jobs, seed=2024, audit=not args.no_cpu,
                                      n_sustained=args.sustained_jobs)

    if not args.no_cpu:
        from oracle import oracle as O
        R_cpu, steps_cpu = 24, 100
        o = O.Sim(p, r_first=0, r_count=R_cpu)
        t0 = time.perf_counter()
        o.step(steps_cpu)
        dt = time.perf_counter() - t0
        cores = O.threads()
        line["cpu_baseline"] = {
            "value": 512 * 512 * R_cpu * steps_cpu / dt, "unit": "site-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "Model B 512x512 SETD2 FP64 oracle, realizations 0..%d over the 100-step parity window "
                      "(%.1f s)" % (R_cpu - 1, dt),
        }
        log("CPU oracle timed")

    print(json.dumps(line), flush=True)
    if tuned:
        os.remove(tuned)


if __name__ == "__main__":
    main()
