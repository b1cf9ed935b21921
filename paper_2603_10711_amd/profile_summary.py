"""Summarize rocprofv3 CSV output into the short text files kept under profiles/.

    python -m paper_2603_10711_amd.profile_summary stats <kernel_stats.csv> <out.md> --cmd "<command>"
    python -m paper_2603_10711_amd.profile_summary pmc <fetch dir> <write dir> <copy fetch dir> <copy write dir> \
        <workload> <out.json> --cmd "<command>"
    python -m paper_2603_10711_amd.profile_summary pmcplain <fetch dir> <write dir> <copy fetch dir> <copy write dir> \
        <workload> <scp iters> <admm iters> <out.json> --cmd "<command>"
    python -m paper_2603_10711_amd.profile_summary sq <counter dir> <title> <admm iterations per dispatch> <out.md> \
        --cmd "<command>" [--kernel <kernel name prefix, default k_persistent>] [--extra <counter dir> ...]
    python -m paper_2603_10711_amd.profile_summary calibrate
    python -m paper_2603_10711_amd.profile_summary markers <marker-trace dir> <out.md> --cmd "<command>"

``calibrate`` is a plain 1 GiB device-to-device copy (run under rocprofv3 --pmc FETCH_SIZE, then
WRITE_SIZE): a kernel whose HBM traffic is known exactly.  ``pmc`` scales FETCH_SIZE / WRITE_SIZE of
k_persistent by what the same counters read for that copy and records the hash of the kernel
sources the counters were taken with; bench.py reports the traffic only while that hash still
matches.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def stats(csv_path: str, out: str, cmd: str, top: int = 14) -> None:
    rows = list(csv.DictReader(open(csv_path)))
    lines = ["# rocprofv3 kernel statistics", "", f"Command: `{cmd}`", "",
             f"Kernel sources hash: `{kernel_source_hash()}`", "",
             "| kernel | calls | avg (us) | min (us) | max (us) | total (ms) | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"].replace("|", "/")
        if len(name) > 110:
            name = name[:107] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def _counter(dirpath: str, kernel_prefix: str):
    path = glob.glob(os.path.join(dirpath, "*counter_collection.csv"))[0]
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    for k, v in vals.items():
        if k.startswith(kernel_prefix):
            return sum(v) / len(v), k
    raise SystemExit(f"no kernel {kernel_prefix} in {path}")


def pmc(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, workload, out, cmd) -> None:
    copy_bytes = 1 << 30
    cf, _ = _counter(copy_fetch_dir, "__amd_rocclr_copyBuffer")
    cw, _ = _counter(copy_write_dir, "__amd_rocclr_copyBuffer")
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    kf, name = _counter(fetch_dir, "void scp::k_persistent")
    kw, _ = _counter(write_dir, "void scp::k_persistent")
    d = {"kernel": name, "workload": workload, "kernel_hash": kernel_source_hash(), "command": cmd,
         "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw,
         "copy_calibration": {"bytes": copy_bytes, "fetch_kib": cf, "write_kib": cw,
                              "fetch_scale": f_scale, "write_scale": w_scale},
         "hbm_read_bytes_per_launch": kf * 1024.0 * f_scale, "hbm_write_bytes_per_launch": kw * 1024.0 * w_scale}
    d["hbm_bytes_per_launch"] = d["hbm_read_bytes_per_launch"] + d["hbm_write_bytes_per_launch"]
    json.dump(d, open(out, "w"), indent=1)


def pmc_plain(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, workload, scp_iters, admm_iters, out, cmd) -> None:
    """HBM bytes of one plain-form solve: per-dispatch FETCH_SIZE / WRITE_SIZE of every kernel
    (scaled by the copy calibration) times its dispatches in a solve of the full budget: the ADMM
    kernels run scp_iters x admm_iters times, the residual kernel once per SCP iteration, the
    per-SCP-iteration kernels scp_iters times, the reset and metric kernels once."""
    copy_bytes = 1 << 30
    cf, _ = _counter(copy_fetch_dir, "__amd_rocclr_copyBuffer")
    cw, _ = _counter(copy_write_dir, "__amd_rocclr_copyBuffer")
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)

    def per_kernel(dirpath):
        path = glob.glob(os.path.join(dirpath, "*counter_collection.csv"))[0]
        vals = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Kernel_Name"].startswith("void scp::"):
                vals[r["Kernel_Name"].split("<")[0].replace("void scp::", "")].append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in vals.items()}

    kf, kw = per_kernel(fetch_dir), per_kernel(write_dir)
    admm = scp_iters * admm_iters
    count = {"k_step1": admm, "k_step1_lanes4": admm, "k_step234": admm, "k_admm_resident": scp_iters,
             "k_resid": scp_iters, "k_lin": scp_iters, "k_minv_lanes4": scp_iters,
             "k_acc_nodes": scp_iters, "k_acc_traj": scp_iters, "k_acc_apply": scp_iters, "k_check": scp_iters,
             "k_reset": 2, "k_reset_state": 1, "k_met_nodes": 1, "k_met_traj": 1}
    kernels = {}
    total_r = total_w = 0.0
    for k in sorted(set(kf) | set(kw)):
        r = kf.get(k, 0.0) * 1024.0 * f_scale
        w = kw.get(k, 0.0) * 1024.0 * w_scale
        kernels[k] = {"read_bytes_per_dispatch": r, "write_bytes_per_dispatch": w, "dispatches_per_solve": count.get(k, 0)}
        total_r += r * count.get(k, 0)
        total_w += w * count.get(k, 0)
    d = {"workload": workload, "kernel_hash": kernel_source_hash(), "command": cmd,
         "budget": f"{scp_iters} SCP x {admm_iters} ADMM", "kernels": kernels,
         "copy_calibration": {"bytes": copy_bytes, "fetch_kib": cf, "write_kib": cw,
                              "fetch_scale": f_scale, "write_scale": w_scale},
         "hbm_read_bytes_per_solve": total_r, "hbm_write_bytes_per_solve": total_w,
         "hbm_bytes_per_solve": total_r + total_w}
    json.dump(d, open(out, "w"), indent=1)


def _sq_values(dirpath: str, kernel: str) -> dict:
    """Counter value per dispatch (mean over dispatches) of the kernels whose name starts with
    ``void scp::<kernel>``."""
    path = glob.glob(os.path.join(dirpath, "*counter_collection.csv"))[0]
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        if r["Kernel_Name"].startswith("void scp::" + kernel):
            per[r["Counter_Name"]][r["Dispatch_Id"]].append(float(r["Counter_Value"]))
    return {c: sum(sum(v) for v in d.values()) / len(d) for c, d in per.items()}


def sq(dirpath: str, title: str, iters: int, out: str, cmd: str, kernel: str = "k_persistent", extra=()) -> None:
    """SQ counters of one kernel per dispatch and per wave, the VALU issue share, and (from further
    counter passes) the LDS bank-conflict share and the FMA count."""
    val = _sq_values(dirpath, kernel)
    for d in extra:
        for c, v in _sq_values(d, kernel).items():
            val.setdefault(c, v)
    waves = val["SQ_WAVES"]
    lines = [f"# rocprofv3 SQ counters of {kernel}, {title}", "", f"Command: `{cmd}`", "",
             f"Kernel sources hash: `{kernel_source_hash()}`", "", "| counter | per dispatch | per wave |", "|---|---|---|"]
    for c in ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_SALU",
              "SQ_INSTS_LDS", "SQ_INSTS_BRANCH", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_LDS",
              "SQ_ACTIVE_INST_MISC", "SQ_ACTIVE_INST_ANY", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS",
              "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT"):
        if c in val:
            lines.append(f"| {c} | {val[c]:.4g} | {val[c] / waves:.4g} |")
    valu = val["SQ_INSTS_VALU"] / waves
    share = val["SQ_INSTS_VALU"] / val["SQ_WAVE_CYCLES"]
    lines += ["", f"VALU instructions per wave per ADMM iteration ({iters} iterations per dispatch, work outside "
                  f"the ADMM loop amortized): {valu / iters:.0f}.",
              "SQ_WAVE_CYCLES counts quad-cycles; one wave64 FP32 VALU instruction occupies its SIMD for one "
              f"quad-cycle, so the VALU issue share of the wave's life is {share:.3f}."]
    for fma in ("SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_FMA_F64"):
        if fma in val:
            lines.append(f"{fma} per wave per ADMM iteration: {val[fma] / waves / iters:.0f} "
                         f"({val[fma] / val['SQ_INSTS_VALU']:.3f} of the VALU instructions).")
    parts = [("VALU", "SQ_ACTIVE_INST_VALU"), ("scalar ALU", "SQ_ACTIVE_INST_SCA"), ("LDS", "SQ_ACTIVE_INST_LDS"),
             ("branch and other", "SQ_ACTIVE_INST_MISC"), ("waiting", "SQ_WAIT_ANY")]
    if all(c in val for _, c in parts):
        per = [(n, val[c] / waves / iters) for n, c in parts]
        lines.append("Where a wave's quad-cycles go per ADMM iteration (issuing, by instruction kind, then waiting; "
                     f"SQ_WAVE_CYCLES {val['SQ_WAVE_CYCLES'] / waves / iters:.0f}): "
                     + ", ".join(f"{n} {v:.1f}" for n, v in per) + ".")
    if "SQ_LDS_BANK_CONFLICT" in val and val.get("SQ_LDS_IDX_ACTIVE", 0) > 0:
        lines.append(f"LDS bank conflicts: {val['SQ_LDS_BANK_CONFLICT'] / val['SQ_LDS_IDX_ACTIVE']:.4f} of the "
                     "LDS indexed-active cycles (SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE).")
    open(out, "w").write("\n".join(lines) + "\n")


def markers(dirpath: str, out: str, cmd: str) -> None:
    """Host trace ranges (roctx) from a --marker-trace run: per range name, count and durations."""
    path = glob.glob(os.path.join(dirpath, "*marker_api_trace.csv"))[0]
    rows = list(csv.DictReader(open(path)))
    name_col = next(c for c in ("Message", "Function", "Name") if rows and c in rows[0])
    dur = collections.defaultdict(list)
    for r in rows:
        t0, t1 = float(r["Start_Timestamp"]), float(r["End_Timestamp"])
        if t1 > t0:
            dur[r[name_col]].append((t1 - t0) / 1e3)
    lines = ["# rocprofv3 host trace ranges (roctx)", "", f"Command: `{cmd}`", "",
             f"Kernel sources hash: `{kernel_source_hash()}`", "",
             "| range | count | avg (us) | min (us) | max (us) |", "|---|---|---|---|---|"]
    for k, v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{k}` | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | {max(v):.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def calibrate(n_bytes: int = 1 << 30) -> None:
    """A plain device-to-device copy of n_bytes (the counters' calibration kernel)."""
    import torch
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {n_bytes} bytes", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--cmd", required=True)
    p = sub.add_parser("pmc")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "workload", "out"):
        p.add_argument(k)
    p.add_argument("--cmd", required=True)
    pp = sub.add_parser("pmcplain")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "workload"):
        pp.add_argument(k)
    pp.add_argument("scp_iters", type=int)
    pp.add_argument("admm_iters", type=int)
    pp.add_argument("out")
    pp.add_argument("--cmd", required=True)
    q = sub.add_parser("sq")
    for k in ("dir", "title", "iters", "out"):
        q.add_argument(k)
    q.add_argument("--cmd", required=True)
    q.add_argument("--kernel", default="k_persistent")
    q.add_argument("--extra", nargs="*", default=[])
    sub.add_parser("calibrate")
    mk = sub.add_parser("markers")
    mk.add_argument("dir")
    mk.add_argument("out")
    mk.add_argument("--cmd", required=True)
    a = ap.parse_args(argv)
    if a.mode == "calibrate":
        return calibrate()
    if a.mode == "markers":
        return markers(a.dir, a.out, a.cmd)
    if a.mode == "stats":
        stats(a.csv, a.out, a.cmd)
    elif a.mode == "pmcplain":
        pmc_plain(a.fetch, a.write, a.copy_fetch, a.copy_write, a.workload, a.scp_iters, a.admm_iters, a.out, a.cmd)
    elif a.mode == "sq":
        sq(a.dir, a.title, int(a.iters), a.out, a.cmd, a.kernel, a.extra)
    else:
        pmc(a.fetch, a.write, a.copy_fetch, a.copy_write, a.workload, a.out, a.cmd)


if __name__ == "__main__":
    main()
