"""Benchmark of the D3Q95 thermal LBM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline: D3Q95 FP32-shifted, 384^3 periodic grid, omega = 1.8, seeded smooth
random initial fields; K timed update steps (one stream-collide kernel per
step) after W warm-up steps.  Prints ONE JSON line with MLUPS, the roofline
of the dominant kernel (algorithmic bytes 2 Q 4 = 760 B per cell update over
the HIP-event duration of the timed launches, against 8 TB/s HBM; the HBM
bytes per launch measured by rocprofv3 counters on the same kernel source),
the CPU oracle's rate on a bounded sample, the headline step and a plain
copy of the same bytes on a few fresh allocations of its buffers (the step's
speed depends on where in HBM they land; `value` is the first allocation's),
and side measurements: FP64 on
256^3, FP32-shifted vs FP64 error after 200 steps on 256^3, D2Q33 in both
precisions on 8192^2, in-place (AA) streaming on 384^3 and on 768^3 (a grid
whose two-buffer state would not fit in HBM), the two shock tubes with held
end planes, and the forward + adjoint cost on 128^3 x 200 steps with
checkpoints every 20.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D3Q95 MLUPS & HBM GB/s vs roofline (FP32-shifted vs FP64; fwd+adjoint)"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stream_collide_d3q95_fp32s_384c_traffic.json")
# The sources the headline kernel (k_step, D3Q95 FP32-shifted) is built from.
KERNEL_SRCS = [os.path.join(ROOT, "paper_1303_4624_amd", "csrc", f) for f in (
    "lbm_kernels.h", "lbm_kernels_d3q95_f32s.hip", "lbm_internal.h", "lbm_model.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def timed_steps(sim, steps, warmup):
    """Wall and event seconds of `steps` steps after `warmup` untimed ones;
    4 or more warm-up steps (in place 8) also pick the faster block order of
    the forward step on these buffers (Simulation.tune_step, bit-identical
    to plain steps)."""
    import torch
    if warmup >= (4 if sim.streaming == "ab" else 8):
        sim.tune_step(warmup)
    else:
        sim.step(warmup)
    torch.cuda.synchronize()
    stream = sim.stream            # the stream the library launches on
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, ev0.elapsed_time(ev1) / 1e3


def run_headline(extent, omega, steps, warmup):
    import torch
    from paper_1303_4624_amd import Simulation
    from synth_inputs import smooth_ic
    t = time.perf_counter()
    rho, U, th = smooth_ic(extent)
    log(f"[bench] IC {extent} generated in {time.perf_counter() - t:.1f}s")
    sim = Simulation("D3Q95", extent, omega, precision="fp32s", rho0=1.0)
    sim.init_fields(rho, U, th * sim.T0)
    del rho, U, th
    wall, ev = timed_steps(sim, steps, warmup)
    order = sim.block_order
    r, _, _ = sim.moments()
    ok = bool(torch.isfinite(r).all())
    cons = sim.conservation()
    copy_gbs = copy_bandwidth(sim)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return wall, ev, ok, cons, copy_gbs, order


def run_placement(extent, omega, trials, steps=20):
    """The headline step and the streaming copy of the same bytes on `trials`
    successive allocations of the population buffers: each trial frees the
    previous simulation and allocates a new one behind a spacer of 0, 1 or
    2 GiB, so the buffers land on other physical memory.  Returns per trial
    the ms per step, the ms per copy and their ratio."""
    import torch
    from paper_1303_4624_amd import Simulation
    from synth_inputs import smooth_ic
    rho, U, th = smooth_ic(extent)
    out = []
    for t in range(trials):
        spacer = torch.empty((t % 3) << 27, dtype=torch.float64, device="cuda")
        sim = Simulation("D3Q95", extent, omega, precision="fp32s", rho0=1.0)
        sim.init_fields(rho, U, th * sim.T0)
        _, ev = timed_steps(sim, steps, 2)
        gbs = copy_bandwidth(sim)
        step_ms = ev / steps * 1e3
        copy_ms = 2 * sim.pop_bytes / gbs / 1e6
        order = sim.block_order
        sim.close()
        del sim, spacer
        torch.cuda.empty_cache()
        out.append({"step_ms": round(step_ms, 4), "copy_ms": round(copy_ms, 4),
                    "step_over_copy": round(step_ms / copy_ms, 4), "block_order": order})
        log(f"[bench] placement trial {t}: step {step_ms:.3f} ms, copy {copy_ms:.3f} ms")
    return out


def run_fp64_and_error(extent, omega, steps_time, steps_err, model="D3Q95", steps_err_long=0):
    """FP64 and FP32-shifted throughput on `extent`, and the FP32-shifted vs
    FP64 GPU error after `steps_err` (and `steps_err_long`) steps from the
    same initial fields."""
    import torch
    from paper_1303_4624_amd import Simulation
    from synth_inputs import smooth_ic
    rho, U, th = smooth_ic(extent)
    out = {}
    fields = {}
    marks = [m for m in (steps_err, steps_err_long) if m]
    for prec in ("fp64", "fp32s"):
        sim = Simulation(model, extent, omega, precision=prec)
        sim.init_fields(rho, U, th * sim.T0)
        done = 0
        for m in marks:
            sim.step(m - done)
            done = m
            fields[(prec, m)] = [x.clone() for x in sim.moments()]
        T0 = sim.T0
        wall, ev = timed_steps(sim, steps_time, 2)
        out[prec] = {"mlups": sim.N * steps_time / ev / 1e6, "ms_per_step": ev / steps_time * 1e3}
        sim.close()
        del sim
        torch.cuda.empty_cache()

    def err(m):
        r64, u64, t64 = fields[("fp64", m)]
        r32, u32, t32 = fields[("fp32s", m)]
        return {"rho": float((r32 - r64).abs().max() / r64.abs().max()),
                "U": float((u32 - u64).abs().max() / u64.abs().max()),
                "T": float((t32 - t64).abs().max() / T0), "steps": m}

    errs = [err(m) for m in marks]
    del fields
    torch.cuda.empty_cache()
    return out, (errs[0] if len(errs) == 1 else errs)


def run_model(model, extent, precision, steps, omega=1.8):
    """Throughput of another velocity set through the same kernel template
    (the lower-order D3Q19/D3Q15 sets): MLUPS and the fraction of 8 TB/s at
    2 Q b bytes per cell update."""
    import torch
    from paper_1303_4624_amd import Simulation
    from synth_inputs import smooth_ic
    rho, U, th = smooth_ic(extent)
    sim = Simulation(model, extent, omega, precision=precision)
    sim.init_fields(rho, U, th * sim.T0)
    del rho, U, th
    wall, ev = timed_steps(sim, steps, 4)
    N, Q = sim.N, sim.Q
    sim.close()
    del sim
    torch.cuda.empty_cache()
    b = 8 if precision == "fp64" else 4
    mlups = N * steps / ev / 1e6
    return {"grid": list(extent), "steps": steps, "mlups": round(mlups, 2),
            "ms_per_step": round(ev / steps * 1e3, 4), "bytes_per_cell": 2 * Q * b,
            "roofline_frac": round(mlups * 2 * Q * b / 1e3 / HBM_PEAK_GBS, 4)}


def run_aa(extent, steps, tile=None):
    """D3Q95 FP32-shifted with in-place (AA) streaming: one population buffer."""
    import torch
    from paper_1303_4624_amd import Simulation
    from synth_inputs import smooth_ic, tiled_smooth_ic
    rho, U, th = smooth_ic(extent) if tile is None else tiled_smooth_ic(extent, tile)
    sim = Simulation("D3Q95", extent, 1.8, precision="fp32s", streaming="aa")
    sim.init_fields(rho, U, th * sim.T0)
    del rho, U, th
    m0 = sim.conservation()[0]
    wall, ev = timed_steps(sim, steps, 8)
    m1 = sim.conservation()[0]
    N, pb = sim.N, sim.pop_bytes
    sim.close()
    del sim
    torch.cuda.empty_cache()
    mlups = N * steps / ev / 1e6
    return {"grid": list(extent), "steps": steps, "mlups": round(mlups, 2),
            "ms_per_step": round(ev / steps * 1e3, 4),
            "roofline_frac": round(mlups * 760 / 1e3 / HBM_PEAK_GBS, 4),
            "population_GB": round(pb / 1e9, 2), "two_buffer_GB": round(2 * pb / 1e9, 2),
            "mass_rel_change": abs(m1 - m0) / abs(m0),
            "ic": "smooth" if tile is None else f"smooth {tile[0]}^3 tile repeated"}


TUBE_PLATEAUS = {"d3q95_11x11x800_tube": ((300, 480), (540, 700)),
                 "d2q33_11x800_tube": ((340, 390), (470, 580))}


def run_tube(wname, precision, graph_steps=0, streaming="ab"):
    """The shock tube with held end planes: time its whole run (optionally
    replayed in HIP graphs of graph_steps steps, on a side stream; with
    streaming="aa" in place on one buffer)."""
    import torch
    from paper_1303_4624_amd import Simulation
    from synth_inputs import WORKLOADS, tube_states, workload_ic
    w = WORKLOADS[wname]
    D = len(w.extent)
    (lr, lt), (rr, rt) = tube_states(w)
    rho, U, th = workload_ic(w)
    stream = torch.cuda.Stream() if graph_steps else torch.cuda.current_stream()
    with torch.cuda.stream(stream):
        sim = Simulation(w.model, w.extent, w.omega, precision=precision, stream=stream,
                         streaming=streaming)
        sim.init_fields(rho, U, th * sim.T0)
        nh = int(w.extra["hold"])
        sim.set_fixed_planes(nh, nh, (lr,) + (0.0,) * D + (lt * sim.T0,),
                             (rr,) + (0.0,) * D + (rt * sim.T0,))
        if graph_steps:
            sim.set_graph_steps(graph_steps)
            sim.step(graph_steps)              # capture outside the timed region
            sim.init_fields(rho, U, th * sim.T0)
        wall, ev = timed_steps(sim, w.steps, 0)
        N = sim.N
        r, _, T = sim.moments()
        axes = tuple(range(1, D))
        rz = r.mean(dim=axes).cpu().numpy()
        tz = (T.mean(dim=axes) / sim.T0).cpu().numpy()
        sim.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    # plateau means between the rarefaction tail, the contact and the shock
    # at t = 120 (the experiment's comparison quantity)
    (a, b), (c, d) = TUBE_PLATEAUS[wname]
    out = {"steps": w.steps, "ms_per_step": round(ev / w.steps * 1e3, 4),
           "mlups": round(N * w.steps / ev / 1e6, 2),
           "plateaus": {"rho_left": round(float(rz[a:b].mean()), 5),
                        "rho_right": round(float(rz[c:d].mean()), 5),
                        "theta_left": round(float(tz[a:b].mean()), 5),
                        "theta_right": round(float(tz[c:d].mean()), 5)}}
    if graph_steps:
        out["graph_steps"] = graph_steps
    if streaming != "ab":
        out["streaming"] = streaming
    return out


def run_fwd_adjoint(extent, omega, n, k, keep=1, streaming="ab", accuracy=False):
    """Wall time of the checkpointed forward run and of the adjoint, same stream.
    `keep`: trailing segments whose step moments the forward run keeps;
    `streaming`: "aa" runs the forward pass in place on one buffer;
    `accuracy`: also compare dL/domega and one directional derivative in T
    with central differences of the FP64 forward run (outside the timing)."""
    import torch
    from paper_1303_4624_amd import Simulation
    from synth_inputs import fd_direction, smooth_ic, target_theta
    rho, U, th = smooth_ic(extent)
    sim = Simulation("D3Q95", extent, omega, precision="fp32s", streaming=streaming)
    T = th * sim.T0
    sim.init_fields(rho, U, target_theta(extent) * sim.T0)
    # the initial fields are resident in HBM before the timed regions
    T_h = T
    rho, U, T = (torch.as_tensor(x, device="cuda") for x in (rho, U, T))
    sim.step(n)
    tgt = sim.moments()[0].clone()
    # plain forward (no checkpoints), for reference
    sim.init_fields(rho, U, T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(n)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    res = {}
    for rep in range(2):          # second repetition is the timed one
        sim.init_fields(rho, U, T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ck = sim.run_checkpointed(n, k, keep)
        ck_bytes = ck.numel() * 8
        r = sim.moments()[0]
        g = 2.0 * (r - tgt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dT, dw = sim.adjoint(n, k, ck, rho, U, T, g, keep=keep)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res = {"fwd_ms": (t1 - t0) * 1e3, "bwd_ms": (t2 - t1) * 1e3,
               "plain_fwd_ms": t_plain * 1e3}
        del ck
    sim.close()
    torch.cuda.empty_cache()
    if accuracy:
        # L = sum (rho_n - rho*)^2 of the FP64 forward run, central differences
        s64 = Simulation("D3Q95", extent, omega, precision="fp64")

        def loss(T_field, w):
            s64.set_omega(w)
            s64.init_fields(rho, U, T_field)
            s64.step(n)
            return float(((s64.moments()[0] - tgt) ** 2).sum())

        h = 1e-6
        fd_w = (loss(T, omega + h) - loss(T, omega - h)) / (2 * h)
        d = fd_direction(extent, 0) * s64.T0
        fd_t = (loss(T_h + h * d, omega) - loss(T_h - h * d, omega)) / (2 * h)
        s64.close()
        an_t = float((dT.double().cpu() * torch.as_tensor(d)).sum())
        res["domega_rel_err_vs_fp64_fd"] = abs(dw - fd_w) / abs(fd_w)
        res["dT_direction_rel_err_vs_fp64_fd"] = abs(an_t - fd_t) / abs(fd_t)
    del dT
    torch.cuda.empty_cache()
    res["ratio_total_over_fwd"] = (res["fwd_ms"] + res["bwd_ms"]) / res["fwd_ms"]
    res["ratio_total_over_plain_fwd"] = (res["fwd_ms"] + res["bwd_ms"]) / res["plain_fwd_ms"]
    res["grid"] = list(extent)
    if streaming != "ab":
        res["streaming"] = streaming
    res["steps"] = n
    res["checkpoint_every"] = k
    res["kept_segments"] = keep
    res["checkpoint_GB"] = round(ck_bytes / 1e9, 2)
    return res


def copy_bandwidth(sim, reps=10):
    """Read + write rate (GB/s) of the library's plain streaming copy of the
    state into the other population buffer of `sim`: the step's bytes on the
    step's own buffers, without its gather and arithmetic (events on the
    library's stream)."""
    import torch
    sim.stream_copy(1)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.stream_copy(reps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    return 2 * sim.pop_bytes / sec / 1e9


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_baseline(extent=(64, 64, 64), steps=20):
    """The FP64 CPU oracle on a bounded sample of the same kind of workload."""
    import torch
    from oracle import lbm as olbm, velocity_sets as ovs
    from synth_inputs import smooth_ic
    threads = min(16, os.cpu_count() or 1)
    torch.set_num_threads(threads)
    v = ovs.velocity_set("D3Q95")
    rho, U, th = smooth_ic(extent)
    f = olbm.init_populations(v, rho, U, th * v.T0)
    t0 = time.perf_counter()
    f = olbm.run(v, f, 1.8, steps)
    dt = time.perf_counter() - t0
    cells = int(rho.size)
    return {"value": cells * steps / dt / 1e6, "unit": "MLUPS", "cores": torch.get_num_threads(),
            "kind": "oracle", "cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"D3Q95 FP64 {extent[0]}x{extent[1]}x{extent[2]}, {steps} steps, "
                      f"omega 1.8, smooth seeded IC ({dt:.1f} s, torch CPU float64, "
                      f"{torch.get_num_threads()} threads)"}


def cpu_oracle_adjoint_baseline(extent=(32, 32, 32), steps=12):
    """The oracle's gradient (float64 autograd through the forward run) on a
    bounded sample: cell updates of forward + backward per second."""
    import numpy as np
    import torch
    from oracle import lbm as olbm, velocity_sets as ovs
    from synth_inputs import smooth_ic, target_theta
    threads = min(16, os.cpu_count() or 1)
    torch.set_num_threads(threads)
    v = ovs.velocity_set("D3Q95")
    rho, U, th = smooth_ic(extent)
    target = np.asarray(rho) * (1 + 0.001 * target_theta(extent))
    t0 = time.perf_counter()
    olbm.loss_and_grad(v, rho, U, th * v.T0, 1.4, steps, target)
    dt = time.perf_counter() - t0
    cells = int(np.prod(extent))
    return {"value": cells * steps / dt / 1e6, "unit": "MLUPS (forward + adjoint)",
            "cores": torch.get_num_threads(), "kind": "oracle", "cpu": cpu_model(),
            "sample": f"D3Q95 FP64 {extent[0]}^3, {steps} steps, autograd gradient of "
                      f"sum (rho_n - rho*)^2 w.r.t. T_init and omega ({dt:.1f} s)"}


def _read_counters(path):
    """rocprofv3 counter CSV -> list of dicts, one per (dispatch, counter)."""
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _timed_dispatches(rows, name, steps):
    """The last `steps` dispatches of kernel `name` in dispatch order (the
    headline's timed steps come after its warm-up steps); `steps` <= 0: all."""
    sel = sorted((r for r in rows if _instance(r["Kernel_Name"])[0] == name),
                 key=lambda r: int(r["Dispatch_Id"]))
    return sel[-steps:] if steps > 0 else sel


def summarize_profiles(prof_dir: str, grid: int = 384, steps: int = 0) -> str:
    """Text summary of the rocprofv3 runs of the headline command (kernel
    trace, FETCH_SIZE and WRITE_SIZE passes, an L2 pass) under prof_dir: the
    step kernel over the last `steps` launches (the timed region, after the
    warm-up steps), the streaming copy over all of its launches.  Also writes
    the traffic record the bench reads (TRAFFIC_FILE) when the counter passes
    are present.  Needs no GPU."""
    import csv
    N = grid ** 3
    alg = 2 * 95 * 4 * N
    lines = []
    trace = os.path.join(prof_dir, "kt", "kt_kernel_trace.csv")
    avg = {}
    if os.path.exists(trace):
        with open(trace) as fh:
            rows = list(csv.DictReader(fh))
        for name, last in (("k_step", steps), ("k_stream_copy", 0)):
            d = [float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
                 for r in _timed_dispatches(rows, name, last)]
            if d:
                avg[name] = (len(d), sum(d) / len(d), min(d))
        lines.append("kernel trace (rocprofv3 --kernel-trace; k_step: the timed launches):")
        for name in ("k_step", "k_stream_copy"):
            if name in avg:
                calls, a, mn = avg[name]
                lines.append(f"  {name:14s} {calls:3d} launches, average {a / 1e6:.4f} ms "
                             f"(min {mn / 1e6:.4f}) -> {alg / a:.1f} GB/s = {alg / a / 8000:.4f} "
                             f"of 8 TB/s")
        if "k_step" in avg and "k_stream_copy" in avg:
            lines.append(f"  k_step at {avg['k_stream_copy'][1] / avg['k_step'][1]:.4f} of the "
                         "streaming copy of the same bytes on the same buffers")
            lines.append(f"  k_step: {N / (avg['k_step'][1] / 1e9) / 1e6:.1f} MLUPS")
    scales, per = {}, {}
    for ctr, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        path = os.path.join(prof_dir, sub, f"{sub}_counter_collection.csv")
        if not os.path.exists(path):
            continue
        rows = [r for r in _read_counters(path) if r["Counter_Name"] == ctr]
        cal = [float(r["Counter_Value"]) for r in rows
               if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer")
               and int(r["Grid_Size"]) == 131072]
        if not cal:
            continue
        scales[ctr] = (1 << 31) / (cal[0] * 1024)
        for name, last in (("k_step", steps), ("k_stream_copy", 0)):
            v = [float(r["Counter_Value"]) for r in _timed_dispatches(rows, name, last)]
            if v:
                per[(name, ctr)] = (len(v), sum(v) / len(v) * 1024 * scales[ctr])
    if scales:
        lines.append("")
        lines.append("HBM counters, one rocprofv3 --pmc pass per counter, each scaled by what "
                     "it reads for a 2 GiB device copy (__amd_rocclr_copyBuffer) in the same run:")
        for ctr, sc in scales.items():
            lines.append(f"  {ctr} scale {sc:.4f}")
        for name in ("k_step", "k_stream_copy"):
            if (name, "FETCH_SIZE") in per and (name, "WRITE_SIZE") in per:
                n, rd = per[(name, "FETCH_SIZE")]
                _, wr = per[(name, "WRITE_SIZE")]
                lines.append(f"  {name:14s} {n:3d} launches: read {rd / 1e9:.3f} GB, write "
                             f"{wr / 1e9:.3f} GB per launch = {(rd + wr) / alg:.4f} x the "
                             f"algorithmic {alg / 1e9:.3f} GB ({rd / N:.1f} + {wr / N:.1f} B/cell)")
        if ("k_step", "FETCH_SIZE") in per and ("k_step", "WRITE_SIZE") in per:
            rd, wr = per[("k_step", "FETCH_SIZE")][1], per[("k_step", "WRITE_SIZE")][1]
            rec = {"kernel": "k_step<D3Q95, FP32-shifted> (stream + collide)",
                   "grid": [grid] * 3, "kernel_source_sha256_16": kernel_source_hash(),
                   "bytes_per_launch": int(rd + wr), "read_bytes_per_launch": int(rd),
                   "write_bytes_per_launch": int(wr), "algorithmic_bytes_per_launch": alg,
                   "fetch_scale": round(scales["FETCH_SIZE"], 4),
                   "write_scale": round(scales["WRITE_SIZE"], 4),
                   "avg_kernel_ns": avg.get("k_step", (0, 0.0, 0))[1]}
            with open(TRAFFIC_FILE, "w") as fh:
                json.dump(rec, fh, indent=1)
    l2 = os.path.join(prof_dir, "l2", "l2_counter_collection.csv")
    if os.path.exists(l2):
        rows = _read_counters(l2)
        lines.append("")
        lines.append("L2 (TCC) counters per cell update, mean over launches:")
        for name, last in (("k_step", steps), ("k_stream_copy", 0)):
            tot = {}
            cnames = sorted(set(r["Counter_Name"] for r in rows))
            for c in cnames:
                sel = [r for r in rows if r["Counter_Name"] == c]
                for r in _timed_dispatches(sel, name, last):
                    tot.setdefault(c, []).append(float(r["Counter_Value"]))
            if tot:
                txt = ", ".join(f"{c} {sum(v) / len(v) / N:.3f}" for c, v in sorted(tot.items()))
                lines.append(f"  {name:14s} {txt}")
        lines.append("  (TCC_EA0_RDREQ: 128-byte reads from memory; TCC_EA0_WRREQ: 64-byte "
                     "writes; 380 B per cell each way = 2.97 reads, 5.94 writes)")
    return "\n".join(lines)


# Side measurements after the headline (all by default; --only picks some).
_MODEL_QD = {"D2Q33": (33, 2), "D3Q95": (95, 3), "D3Q19": (19, 3), "D3Q15": (15, 3)}
# kernels launched one lane per cell over whole rows padded to 64 lanes
_ROW_KERNELS = ("k_step", "k_step_aa", "k_adjoint")
# kernels launched one lane per cell over ceil(N / 256) blocks of 256
_FLAT_KERNELS = ("k_init", "k_moments", "k_to_ab", "k_from_ab", "k_set_pop", "k_get_pop",
                 "k_lambda_init", "k_dT_init")


def _instance(name: str):
    """(kernel, model, precision, bool template flags) from a full rocprofv3
    kernel name such as 'void lbm::(anonymous namespace)::k_step<lbm::D3Q95,
    lbm::(anonymous namespace)::F32ST, false, false, true>(...)'."""
    import re
    m = re.search(r"(k_\w+)<([^>]*)>", name)
    if not m:
        m2 = re.search(r"(k_\w+)\(", name)
        return (m2.group(1) if m2 else name.split("(")[0]), None, None, ()
    args = [a.strip().replace("lbm::", "").replace("(anonymous namespace)::", "")
            for a in m.group(2).split(",")]
    model = args[0] if args and args[0] in _MODEL_QD else None
    prec = {"F32ST": "F32S", "F64T": "F64"}.get(args[1]) if len(args) > 1 else None
    flags = tuple(int(a == "true") for a in args[2:] if a in ("true", "false"))
    return m.group(1), model, prec, flags


def _alg_bytes_per_cell(kernel, model, prec, flags):
    """Algorithmic HBM bytes per cell of one launch: each value the kernel
    must read or write, once (storage b bytes per population or moment,
    float64 fields and gradients 8 bytes)."""
    if model is None or prec is None:
        return None
    Q, D = _MODEL_QD[model]
    b = 8 if prec == "F64" else 4
    mom = (D + 2) * b
    if kernel == "k_step":                      # STORE_MOM, HOLD, POP
        sm, _, pop = (flags + (0, 0, 1))[:3]
        return Q * b + (Q * b if pop else 0) + (mom if sm else 0)
    if kernel == "k_step_aa":                   # PUSH, HOLD, STORE_MOM
        return 2 * Q * b + (mom if flags[2] else 0)
    if kernel == "k_adjoint":                   # COLLIDE, MARK, HOLD
        return 2 * Q * b + (mom if flags[0] else 0) + (Q * b if flags[1] else 0)
    if kernel in ("k_to_ab", "k_from_ab"):
        return 2 * Q * b
    if kernel in ("k_init", "k_moments"):
        return Q * b + 8 * (D + 2)
    if kernel in ("k_set_pop", "k_get_pop"):
        return Q * b + 8 * Q
    if kernel == "k_conservation":
        return Q * b
    if kernel == "k_lambda_init":
        return 2 * Q * b + 8
    if kernel == "k_dT_init":
        return Q * b + 8 * (D + 2) + 8
    return None


def _lane_cells():
    """Launch lanes -> (cells, workload) for the grids the bench runs."""
    from synth_inputs import WORKLOADS
    shapes = {(384,) * 3: "384^3", (256,) * 3: "256^3", (8192, 8192): "8192^2",
              (768,) * 3: "768^3", (128,) * 3: "128^3"}
    for w in WORKLOADS.values():
        if w.name.endswith("_tube"):
            shapes[tuple(w.extent)] = "x".join(map(str, w.extent))
    out = {}
    for ext, label in shapes.items():
        cells = 1
        for n in ext:
            cells *= n
        rows = cells // ext[0]
        out[("row", rows * (-(-ext[0] // 64) * 64))] = (cells, label)
        out[("flat", -(-cells // 256) * 256)] = (cells, label)
    return out


def _walk_dispatches(rows, grid_of):
    """Yield (row, instance, workload, cells, algorithmic bytes) for the
    library's kernels in dispatch order; a grid-stride launch (the
    conservation sums) and the streaming copy take the workload of the
    launch before them."""
    lanes = _lane_cells()
    cur = (None, None)
    for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
        kernel, model, prec, flags = _instance(r["Kernel_Name"])
        grid = grid_of(r)
        if kernel in _ROW_KERNELS:
            cells, label = lanes.get(("row", grid), (None, None))
        elif kernel in _FLAT_KERNELS:
            cells, label = lanes.get(("flat", grid), (None, None))
        elif kernel in ("k_conservation", "k_stream_copy"):
            cells, label = cur
        else:
            continue
        if cells is None:
            continue
        if kernel in _ROW_KERNELS or kernel in _FLAT_KERNELS:
            cur = (cells, label)
        if kernel == "k_stream_copy":
            inst, alg = kernel, 32 * grid           # one 16-byte vector per lane, each way
        else:
            inst = f"{kernel}<{model},{prec}" + "".join(f",{f}" for f in flags) + ">"
            bpc = _alg_bytes_per_cell(kernel, model, prec, flags)
            alg = bpc * cells if bpc else None
        yield r, inst, label, cells, alg


def summarize_all_kernels(prof_dir: str) -> str:
    """Per-kernel-instance table of a rocprofv3 kernel trace (kt/) and of the
    FETCH_SIZE / WRITE_SIZE passes (fetch/, write/) of a full bench run, all
    taken without kernel-name truncation; needs no GPU."""
    import csv
    with open(os.path.join(prof_dir, "kt", "kt_kernel_trace.csv")) as fh:
        trace = list(csv.DictReader(fh))
    groups, other_ns = {}, 0.0
    lib = set()
    for r, inst, label, cells, alg in _walk_dispatches(
            trace, lambda r: int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])):
        lib.add(r["Dispatch_Id"])
        key = (inst, label, int(r["Workgroup_Size_X"]), int(r["VGPR_Count"]))
        g = groups.setdefault(key, {"ns": [], "alg": alg, "cells": cells})
        g["ns"].append(float(r["End_Timestamp"]) - float(r["Start_Timestamp"]))
    for r in trace:
        if r["Dispatch_Id"] not in lib:
            other_ns += float(r["End_Timestamp"]) - float(r["Start_Timestamp"])

    # counters: mean per (instance, workload) over dispatches, scaled by what
    # the counter reads for the 2 GiB device copy of the same pass
    ctr, scales = {}, {}
    for c, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        path = os.path.join(prof_dir, sub, f"{sub}_counter_collection.csv")
        if not os.path.exists(path):
            continue
        rows = [r for r in _read_counters(path) if r["Counter_Name"] == c]
        cal = [float(r["Counter_Value"]) for r in rows
               if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer")
               and int(r["Grid_Size"]) == 131072]
        if not cal:
            continue
        scales[c] = (1 << 31) / (cal[0] * 1024)
        for r, inst, label, cells, alg in _walk_dispatches(rows, lambda r: int(r["Grid_Size"])):
            ctr.setdefault((inst, label, c), []).append(
                float(r["Counter_Value"]) * 1024 * scales[c] / cells)

    lines = [f"kernel source sha256[:16] = {kernel_source_hash()} (headline kernel sources)"]
    if scales:
        lines.append("counter scales (2 GiB device copy in the same pass): "
                     + ", ".join(f"{c} {s:.4f}" for c, s in scales.items()))
    lines.append("per launch: time from the trace; B/cell = algorithmic bytes per cell "
                 "(each value read or written once), TB/s = algorithmic bytes / average time; "
                 "rd, wr = counter bytes per cell, x = (rd + wr) / algorithmic")
    lines.append("flags: k_step<STORE_MOM,HOLD,POP>, k_step_aa<PUSH,HOLD,STORE_MOM>, "
                 "k_adjoint<COLLIDE,MARK,HOLD>; vgpr is rocprofv3's VGPR_Count (half the "
                 "registers per lane on gfx950); k_stream_copy moves the headline state")
    lines.append("")
    lines.append(f"{'instance':34s} {'grid':>10s} {'wg':>4s} {'vgpr':>4s} {'n':>5s} "
                 f"{'avg us':>10s} {'min us':>10s} {'B/cell':>7s} {'TB/s':>6s} {'of 8':>5s} "
                 f"{'rd':>7s} {'wr':>7s} {'x':>6s}")
    for (inst, label, wg, vgpr), g in groups.items():
        n = len(g["ns"])
        avg = sum(g["ns"]) / n
        alg, cells = g["alg"], g["cells"]
        rd = ctr.get((inst, label, "FETCH_SIZE"))
        wr = ctr.get((inst, label, "WRITE_SIZE"))
        if rd and wr:
            rdv, wrv = sum(rd) / len(rd), sum(wr) / len(wr)
            cnt = f"{rdv:7.1f} {wrv:7.1f} {(rdv + wrv) * cells / alg:6.3f}"
        else:
            cnt = f"{'-':>7s} {'-':>7s} {'-':>6s}"
        lines.append(f"{inst:34s} {label:>10s} {wg:4d} {vgpr:4d} {n:5d} {avg / 1e3:10.2f} "
                     f"{min(g['ns']) / 1e3:10.2f} {alg / cells:7.0f} {alg / avg / 1e3:6.2f} "
                     f"{alg / avg / 8e3:5.2f} {cnt}")
    lines.append("")
    lines.append("other kernels (torch elementwise, reductions, runtime copies and fills, the "
                 f"library's zero fills and partial sums): {other_ns / 1e6:.1f} ms in total")
    return "\n".join(lines)


def summarize_placement(prof_dir: str) -> str:
    """Per-trial table of two rocprofv3 counter passes (lat/, tlb/) over
    `bench.py --placement-trials`: the headline step's time, mean DRAM read
    latency (TCC_EA0_RDREQ_LEVEL / TCC_EA0_RDREQ), address-translation misses
    and the shader clock.  Trials are told apart by their k_init launches;
    needs no GPU."""
    import collections
    out = ["trial  pass  step ms   read latency (cycles)  UTCL1 miss rate  UTCL2 busy  clock GHz"]
    for sub in ("lat", "tlb"):
        path = os.path.join(prof_dir, sub, f"{sub}_counter_collection.csv")
        if not os.path.exists(path):
            continue
        disp = collections.OrderedDict()
        for r in sorted(_read_counters(path), key=lambda r: int(r["Dispatch_Id"])):
            d = disp.setdefault(int(r["Dispatch_Id"]), {
                "name": r["Kernel_Name"], "grid": int(r["Grid_Size"]),
                "ns": float(r["End_Timestamp"]) - float(r["Start_Timestamp"])})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
        trial, acc = -1, collections.OrderedDict()
        for d in disp.values():
            kernel, model, prec, _ = _instance(d["name"])
            if d["grid"] != 384 ** 3 or model != "D3Q95" or prec != "F32S":
                continue
            if kernel == "k_init":
                trial += 1
            elif kernel == "k_step" and trial >= 0:
                acc.setdefault(trial, []).append(d)
        for t, ds in acc.items():
            mean = lambda k: sum(x.get(k, 0.0) for x in ds) / len(ds)
            ms = mean("ns") / 1e6
            lat = (f"{mean('TCC_EA0_RDREQ_LEVEL_sum') / mean('TCC_EA0_RDREQ_sum'):21.0f}"
                   if mean("TCC_EA0_RDREQ_sum") else f"{'-':>21s}")
            if mean("TCP_UTCL1_REQUEST_sum"):
                tlb = (f"{mean('TCP_UTCL1_TRANSLATION_MISS_sum') / mean('TCP_UTCL1_REQUEST_sum'):15.2e}"
                       f"  {mean('GRBM_UTCL2_BUSY') / mean('GRBM_GUI_ACTIVE'):10.4f}"
                       f"  {mean('GRBM_GUI_ACTIVE') / 8 / mean('ns'):9.3f}")
            else:
                tlb = f"{'-':>15s}  {'-':>10s}  {'-':>9s}"
            out.append(f"{t:5d}  {sub:4s}  {ms:7.3f}  {lat}  {tlb}")
    return "\n".join(out)


SECTIONS = ("256c", "d2q33", "lower", "aa", "tubes", "adjoint")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--grid", type=int, default=384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 2 GiB device copy first (reference dispatch for HBM counters)")
    ap.add_argument("--placement-trials", type=int, default=None,
                    help="also time the headline step and the streaming copy on this many "
                         "fresh allocations of the population buffers (default 4, or 0 with "
                         "--no-extras)")
    ap.add_argument("--only", default="",
                    help="comma-separated side measurements to run (default: all of them): "
                         + ",".join(SECTIONS))
    ap.add_argument("--summarize-profiles", metavar="DIR", default="",
                    help="print the summary of rocprofv3 runs of the headline command in DIR "
                         "(kt/, fetch/, write/, l2/) and update the traffic record; no GPU")
    ap.add_argument("--summarize-all-profiles", metavar="DIR", default="",
                    help="print the per-kernel table of rocprofv3 runs of the full bench in DIR "
                         "(kt/ kernel trace, fetch/ and write/ counter passes); no GPU")
    ap.add_argument("--summarize-placement-profiles", metavar="DIR", default="",
                    help="print the per-trial table of rocprofv3 counter passes (lat/, tlb/) "
                         "over --placement-trials runs in DIR; no GPU")
    args = ap.parse_args()
    if args.summarize_placement_profiles:
        print(summarize_placement(args.summarize_placement_profiles))
        return
    if args.summarize_all_profiles:
        print(summarize_all_kernels(args.summarize_all_profiles))
        return
    if args.summarize_profiles:
        print(summarize_profiles(args.summarize_profiles, args.grid, args.steps))
        return
    only = set(x for x in args.only.split(",") if x)
    if only - set(SECTIONS):
        ap.error(f"unknown sections {sorted(only - set(SECTIONS))}")
    want = (lambda name: not only or name in only)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "slab decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1303_4624_amd import _lib
    _lib.library()            # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)

    if args.copy_calibration:
        n = (1 << 31) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
        log("[bench] calibration copy of 2 GiB done")
    extent = (args.grid,) * 3
    omega = 1.8
    Q = 95
    log(f"[bench] headline D3Q95 fp32s {extent}, {args.steps} steps")
    wall, ev, ok, cons, cbw, order = run_headline(extent, omega, args.steps, args.warmup)
    N = args.grid ** 3
    mlups = N * args.steps / ev / 1e6
    per_launch_s = ev / args.steps
    bytes_per_launch = 2 * Q * 4 * N
    achieved = bytes_per_launch / per_launch_s / 1e9
    traffic = measured_traffic() if args.grid == 384 else None
    log(f"[bench] {mlups:.1f} MLUPS, {achieved:.1f} GB/s, wall {wall:.3f}s events {ev:.3f}s")

    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ev / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"D3Q95 FP32-shifted {args.grid}^3 periodic, omega 1.8, "
                               "seeded smooth random rho/U/T fields (wavenumbers <= 8)",
                   "grid": list(extent), "omega": omega, "precision": "fp32s",
                   "cell_updates_per_step": N},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "traffic_unit": "B per launch (rocprofv3 FETCH_SIZE + "
                     "WRITE_SIZE, calibrated on a device copy)",
                     "traffic_over_algorithmic": (round(traffic / bytes_per_launch, 4)
                                                  if traffic else None)},
        "finite": ok,
        "mass_after": cons[0],
        # block order of the forward step kept by the warm-up steps (0:
        # contiguous rows per XCD, 1: z-planes in turn)
        "block_order": order,
    }
    # the same bytes moved by a plain streaming copy on the same buffers
    out["roofline"]["copy_GBs"] = round(cbw, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / cbw, 4)
    if args.placement_trials is None:
        args.placement_trials = 0 if args.no_extras else 4
    if args.placement_trials > 0:
        log(f"[bench] {args.placement_trials} placements of the headline buffers")
        out[f"placement_{args.grid}c"] = run_placement(extent, omega, args.placement_trials)
    if not args.no_extras and want("256c"):
        log("[bench] fp64 vs fp32s on 256^3")
        thr, errs = run_fp64_and_error((256, 256, 256), 1.5, 100, 200, steps_err_long=1000)
        err = errs[0]
        out["fp32s_vs_fp64_256c_1000_steps"] = errs[1]
        out["fp64_256c"] = {k: round(v, 3) for k, v in thr["fp64"].items()}
        out["fp32s_256c"] = {k: round(v, 3) for k, v in thr["fp32s"].items()}
        out["fp64_256c"]["roofline_frac"] = round(
            out["fp64_256c"]["mlups"] * 1520 / 1e3 / HBM_PEAK_GBS, 4)
        out["fp32s_vs_fp64_256c"] = err
    if not args.no_extras and want("d2q33"):
        log("[bench] D2Q33 fp64 vs fp32s on 8192^2")
        thr, err = run_fp64_and_error((8192, 8192), 1.5, 100, 200, model="D2Q33")
        for prec, bpc in (("fp64", 528), ("fp32s", 264)):
            d = {k: round(v, 3) for k, v in thr[prec].items()}
            d["roofline_frac"] = round(d["mlups"] * bpc / 1e3 / HBM_PEAK_GBS, 4)
            out[f"d2q33_{prec}_8192sq"] = d
        out["d2q33_fp32s_vs_fp64_8192sq"] = err
    if not args.no_extras and want("lower"):
        log("[bench] lower-order D3Q19 / D3Q15 on 384^3")
        for model in ("D3Q19", "D3Q15"):
            for prec in ("fp32s", "fp64"):
                out[f"{model.lower()}_{prec}_384c"] = run_model(model, extent, prec, 100)
    if not args.no_extras and want("aa"):
        log("[bench] in-place (AA) streaming, 384^3 and 768^3")
        out["aa_fp32s_384c"] = run_aa((384, 384, 384), 100)
        out["aa_fp32s_768c"] = run_aa((768, 768, 768), 30, tile=(192, 192, 192))
    if not args.no_extras and want("tubes"):
        log("[bench] shock tubes with held end planes")
        for wname in ("d3q95_11x11x800_tube", "d2q33_11x800_tube"):
            for prec in ("fp64", "fp32s"):
                out[f"{wname}_{prec}"] = run_tube(wname, prec)
                out[f"{wname}_{prec}_graph"] = run_tube(wname, prec, graph_steps=40)
            out[f"{wname}_fp32s_aa"] = run_tube(wname, "fp32s", streaming="aa")
    if not args.no_extras and want("adjoint"):
        log("[bench] forward + adjoint on 128^3")
        # 128^3 fits many times over in HBM: keep the moments of every segment
        # (no recomputation); the minimum-memory variant keeps one segment.
        out["fwd_adjoint_128c"] = run_fwd_adjoint((128, 128, 128), 1.4, 200, 20, keep=10,
                                                  accuracy=True)
        out["fwd_adjoint_128c_min_memory"] = run_fwd_adjoint((128, 128, 128), 1.4, 200, 20,
                                                             keep=1)
        out["fwd_adjoint_128c_in_place"] = run_fwd_adjoint((128, 128, 128), 1.4, 200, 20,
                                                           keep=10, streaming="aa")
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_oracle_baseline()
        if not args.no_extras:
            out["cpu_baseline_fwd_adjoint"] = cpu_oracle_adjoint_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
