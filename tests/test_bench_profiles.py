"""The profile summarizers of bench.py on small synthetic rocprofv3 outputs
(no GPU): kernel-name parsing, algorithmic bytes per instance, grouping of
dispatches by workload, and the counter scaling against the device copy."""
import csv
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

NS = "lbm::(anonymous namespace)::"
N384 = 384 ** 3


def _name(kernel, model, prec, *flags):
    args = [f"lbm::{model}", f"{NS}{prec}"] + [("true" if f else "false") for f in flags]
    return f"void {NS}{kernel}<{', '.join(args)}>({NS}{prec}::S const*, lbm::KParams)"


def test_instance_parsing():
    k, m, p, fl = bench._instance(_name("k_step", "D3Q95", "F32ST", 0, 0, 1))
    assert (k, m, p, fl) == ("k_step", "D3Q95", "F32S", (0, 0, 1))
    k, m, p, fl = bench._instance(_name("k_adjoint", "D2Q33", "F64T", 1, 1, 0))
    assert (k, m, p, fl) == ("k_adjoint", "D2Q33", "F64", (1, 1, 0))
    # k_init carries an int template argument (the storage form), not a flag
    k, m, p, fl = bench._instance(f"void {NS}k_init<lbm::D3Q19, {NS}F32ST, 0>(double const*)")
    assert (k, m, p, fl) == ("k_init", "D3Q19", "F32S", ())
    assert bench._instance("k_stream_copy(float vector[4] const*, long long, int)")[0] == \
        "k_stream_copy"


def test_algorithmic_bytes_per_cell():
    b = bench._alg_bytes_per_cell
    assert b("k_step", "D3Q95", "F32S", (0, 0, 1)) == 760
    assert b("k_step", "D3Q95", "F64", (0, 0, 1)) == 1520
    assert b("k_step", "D3Q95", "F32S", (1, 0, 1)) == 780          # + 5 moments
    assert b("k_step", "D3Q95", "F32S", (1, 0, 0)) == 400          # moments only
    assert b("k_step", "D2Q33", "F32S", (0, 1, 1)) == 264
    assert b("k_step", "D3Q19", "F64", (0, 0, 1)) == 304
    assert b("k_step", "D3Q15", "F32S", (0, 0, 1)) == 120
    assert b("k_step_aa", "D3Q95", "F32S", (1, 0, 0)) == 760
    assert b("k_step_aa", "D3Q95", "F32S", (0, 0, 1)) == 780
    assert b("k_adjoint", "D3Q95", "F32S", (1, 0, 0)) == 780
    assert b("k_adjoint", "D3Q95", "F32S", (1, 1, 0)) == 1160
    assert b("k_adjoint", "D3Q95", "F32S", (0, 1, 0)) == 1140      # transposed streaming + mark
    assert b("k_init", "D3Q95", "F32S", ()) == 420
    assert b("k_moments", "D2Q33", "F64", ()) == 296
    assert b("k_conservation", "D3Q95", "F32S", ()) == 380
    assert b("k_lambda_init", "D3Q95", "F32S", ()) == 768
    assert b("k_dT_init", "D3Q95", "F32S", ()) == 428
    assert b("k_to_ab", "D3Q95", "F32S", ()) == 760
    assert b("k_fill_zero", None, None, ()) is None


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_all_kernels(tmp_path):
    init = f"void {NS}k_init<lbm::D3Q95, {NS}F32ST, 0>(double const*)"
    step = _name("k_step", "D3Q95", "F32ST", 0, 0, 1)
    cons = f"void {NS}k_conservation<lbm::D3Q95, {NS}F32ST, 0>({NS}F32ST::S const*)"
    copy = "k_stream_copy(float vector[4] const*, float vector[4]*, long long, int)"
    copy_lanes = N384 * 95 * 4 // 16
    # dispatch id, name, grid, workgroup, duration in ns
    seq = [(1, "__amd_rocclr_copyBuffer", 131072, 512, 400000),
           (2, init, N384, 256, 4_000_000),
           (3, step, N384, 384, 8_000_000),
           (4, step, N384, 384, 7_000_000),
           (5, cons, 262144, 256, 3_500_000),          # grid-stride: the 384^3 workload's
           (6, copy, copy_lanes, 256, 6_800_000)]
    hdr = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id",
           "Kernel_Name", "Correlation_Id", "Start_Timestamp", "End_Timestamp", "LDS_Block_Size",
           "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Workgroup_Size_X",
           "Workgroup_Size_Y", "Workgroup_Size_Z", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
    t0 = 1_000_000
    rows = []
    for d, n, g, wg, dur in seq:
        rows.append(["KERNEL_DISPATCH", "Agent 1", 1, 0, 1, d, d, n, d, t0, t0 + dur, 0, 0, 64, 0,
                     32, wg, 1, 1, g, 1, 1])
        t0 += dur + 1000
    _write(str(tmp_path / "kt" / "kt_kernel_trace.csv"), hdr, rows)
    chdr = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
            "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
            "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
            "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    # FETCH_SIZE reads half the bytes (KiB), WRITE_SIZE exact; the 2 GiB copy calibrates
    per_cell = {"k_init": (40, 380), "k_step": (383, 380), "k_conservation": (380, 0),
                "k_stream_copy": (380, 380)}
    for ctr, sub, half in (("FETCH_SIZE", "fetch", 2.0), ("WRITE_SIZE", "write", 1.0)):
        crow = []
        for d, n, g, wg, dur in seq:
            if n.startswith("__amd"):
                v = (1 << 31) / 1024 / half
            else:
                key = bench._instance(n)[0]
                v = per_cell[key][0 if ctr == "FETCH_SIZE" else 1] * N384 / 1024 / half
            crow.append([d, d, "Agent 1", 1, 1, 1, g, d, n, wg, 0, 0, 64, 0, 32, ctr, v, 0, dur])
        _write(str(tmp_path / sub / f"{sub}_counter_collection.csv"), chdr, crow)

    txt = bench.summarize_all_kernels(str(tmp_path))
    assert "FETCH_SIZE 2.0000, WRITE_SIZE 1.0000" in txt
    lines = {l.split()[0]: l.split() for l in txt.splitlines() if l.startswith("k_")}
    st = lines["k_step<D3Q95,F32S,0,0,1>"]
    # grid, wg, vgpr, n, avg us, min us, B/cell, TB/s, of 8, rd, wr, x
    assert st[1] == "384^3" and st[4] == "2"
    assert float(st[5]) == 7500.0 and float(st[6]) == 7000.0
    assert st[7] == "760"
    assert abs(float(st[8]) - 760 * N384 / 7.5e-3 / 1e12) < 0.01
    assert (st[10], st[11]) == ("383.0", "380.0")
    assert abs(float(st[12]) - 763 / 760) < 1e-3
    cs = lines["k_conservation<D3Q95,F32S>"]
    assert cs[1] == "384^3" and cs[7] == "380" and cs[10] == "380.0" and cs[11] == "0.0"
    cp = lines["k_stream_copy"]
    assert cp[1] == "384^3" and cp[7] == "760" and cp[12] == "1.000"
    assert "other kernels" in txt


def test_summarize_placement(tmp_path):
    init = f"void {NS}k_init<lbm::D3Q95, {NS}F32ST, 0>(double const*)"
    step = _name("k_step", "D3Q95", "F32ST", 0, 0, 1)
    hdr = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
           "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
           "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
           "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    rows, d = [], 0
    for trial, (ms, lat) in enumerate(((7.8, 2700.0), (7.2, 2600.0))):
        d += 1
        rows.append([d, d, "A", 1, 1, 1, N384, 1, init, 256, 0, 0, 32, 0, 32,
                     "TCC_EA0_RDREQ_sum", 1.0, 0, 4_000_000])
        for _ in range(3):
            d += 1
            for c, v in (("TCC_EA0_RDREQ_sum", 100.0), ("TCC_EA0_RDREQ_LEVEL_sum", 100.0 * lat)):
                rows.append([d, d, "A", 1, 1, 1, N384, 2, step, 384, 0, 0, 64, 0, 32, c, v, 0,
                             int(ms * 1e6)])
    _write(str(tmp_path / "lat" / "lat_counter_collection.csv"), hdr, rows)
    txt = bench.summarize_placement(str(tmp_path)).splitlines()
    assert len(txt) == 3
    t0, t1 = txt[1].split(), txt[2].split()
    assert t0[:4] == ["0", "lat", "7.800", "2700"]
    assert t1[:4] == ["1", "lat", "7.200", "2600"]
