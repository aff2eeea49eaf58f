"""Benchmark of the D3Q95 thermal LBM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline: D3Q95 FP32-shifted, 384^3 periodic grid, omega = 1.8, seeded smooth
random initial fields; K timed update steps (one stream-collide kernel per
step) after W warm-up steps.  Prints ONE JSON line with MLUPS, the roofline
of the dominant kernel (algorithmic bytes 2 Q 4 = 760 B per cell update over
the HIP-event duration of the timed launches, against 8 TB/s HBM; the HBM
bytes per launch measured by rocprofv3 counters on the same kernel source),
the CPU oracle's rate on a bounded sample, and side measurements: FP64 on
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
    import torch
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
    r, _, _ = sim.moments()
    ok = bool(torch.isfinite(r).all())
    cons = sim.conservation()
    copy_gbs = copy_bandwidth(sim)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return wall, ev, ok, cons, copy_gbs


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
    wall, ev = timed_steps(sim, steps, 4)
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


def summarize_profiles(prof_dir: str, grid: int = 384) -> str:
    """Text summary of the rocprofv3 runs of the headline command (kernel
    stats, FETCH_SIZE and WRITE_SIZE passes, an L2 pass) under prof_dir;
    also writes the traffic record the bench reads (TRAFFIC_FILE) when the
    counter passes are present.  Needs no GPU."""
    import csv
    N = grid ** 3
    alg = 2 * 95 * 4 * N
    lines = []
    stats = os.path.join(prof_dir, "kt", "kt_kernel_stats.csv")
    avg = {}
    if os.path.exists(stats):
        with open(stats) as fh:
            for r in csv.DictReader(fh):
                avg[r["Name"]] = (int(r["Calls"]), float(r["AverageNs"]), float(r["MinNs"]))
        lines.append("kernel statistics (rocprofv3 --kernel-trace --stats):")
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
        for name in ("k_step", "k_stream_copy"):
            v = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"] == name]
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
        rows = [r for r in _read_counters(l2) if r["Kernel_Name"] in ("k_step", "k_stream_copy")]
        lines.append("")
        lines.append("L2 (TCC) counters per cell update, mean over launches:")
        for name in ("k_step", "k_stream_copy"):
            tot = {}
            for r in rows:
                if r["Kernel_Name"] == name:
                    tot.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            if tot:
                txt = ", ".join(f"{c} {sum(v) / len(v) / N:.3f}" for c, v in sorted(tot.items()))
                lines.append(f"  {name:14s} {txt}")
        lines.append("  (TCC_EA0_RDREQ: 128-byte reads from memory; TCC_EA0_WRREQ: 64-byte "
                     "writes; 380 B per cell each way = 2.97 reads, 5.94 writes)")
    return "\n".join(lines)


# Side measurements after the headline (all by default; --only picks some).
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
    ap.add_argument("--only", default="",
                    help="comma-separated side measurements to run (default: all of them): "
                         + ",".join(SECTIONS))
    ap.add_argument("--summarize-profiles", metavar="DIR", default="",
                    help="print the summary of rocprofv3 runs of the headline command in DIR "
                         "(kt/, fetch/, write/, l2/) and update the traffic record; no GPU")
    args = ap.parse_args()
    if args.summarize_profiles:
        print(summarize_profiles(args.summarize_profiles, args.grid))
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
    wall, ev, ok, cons, cbw = run_headline(extent, omega, args.steps, args.warmup)
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
    }
    # the same bytes moved by a plain streaming copy on the same buffers
    out["roofline"]["copy_GBs"] = round(cbw, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / cbw, 4)
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
