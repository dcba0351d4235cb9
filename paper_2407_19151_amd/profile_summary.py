"""Turn rocprofv3 CSV output into the short text summaries kept under
profiles/ (and read back by bench.py).  Nothing here runs on the GPU.

    python -m paper_2407_19151_amd.profile_summary trace  <kernel_stats.csv> <cmd>
    python -m paper_2407_19151_amd.profile_summary traffic <fetch_dir> <write_dir>
                                                   <calib_fetch_dir> <calib_write_dir> <cmds...>
    python -m paper_2407_19151_amd.profile_summary valu <pass_a_dir> <pass_b_dir> <cmds...>

Kernels are keyed as bench.py keys them: (mode, <tpc>x<cap>, L<layout>) from
the collide kernel's template arguments (float kinematics: fp32, double:
fp64; the plain order-N forms only).
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KNAME = re.compile(r"collide_kernel<(\d+), (\d+), (float|double), false, (\d), false, false, 0>")


KERNEL_HEADERS = ("mcc_collide.hpp", "mcc_device.hpp", "mcc_kernel_args.hpp", "mcc_variants.hpp")


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def code_text(src: str) -> str:
    """C/C++ source with its comments removed and whitespace collapsed: what
    the compiler sees, so a change to a comment keeps the digest."""
    return " ".join(_COMMENT.sub(" ", src).split())


def source_hash() -> str:
    """sha256 over the code (comments aside) the collide kernels are built
    from: their instantiation units (mcc_collide_*.hip), the headers those
    include and the public header (the digest bench.py checks before it
    reports the counters)."""
    h = hashlib.sha256()
    d = os.path.join(HERE, "csrc")
    files = sorted(f for f in os.listdir(d)
                   if (f.startswith("mcc_collide_") and f.endswith(".hip")) or f in KERNEL_HEADERS)
    paths = [os.path.join(d, f) for f in files]
    paths.append(os.path.join(os.path.dirname(HERE), "include", "mcc.h"))
    for path in paths:
        h.update(os.path.basename(path).encode())
        h.update(code_text(open(path, encoding="utf-8").read()).encode())
    return h.hexdigest()


def kernel_key(name: str):
    m = KNAME.search(name)
    if not m:
        return None
    tpc, cap, kr, lay = m.groups()
    return ("fp32" if kr == "float" else "fp64", "%sx%s" % (tpc, cap), "L" + lay)


def counters(run_dir: str):
    """{kernel key: {counter: average per dispatch}} and the dispatch counts."""
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    disp = collections.defaultdict(set)
    meta = {}
    path = os.path.join(run_dir, "run_counter_collection.csv")
    for r in csv.DictReader(open(path)):
        k = kernel_key(r["Kernel_Name"])
        if k is None:
            continue
        acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
        disp[k].add(r.get("Dispatch_Id", r.get("Correlation_Id", "")))
        meta[k] = {x: r.get(x) for x in ("VGPR_Count", "Accum_VGPR_Count", "SGPR_Count",
                                         "LDS_Block_Size", "Scratch_Size", "Workgroup_Size",
                                         "Grid_Size")}
    avg = {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}
    return avg, {k: len(v) for k, v in disp.items()}, meta


def trace(stats_csv: str, command: str) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0
    out = ["| kernel | calls | average (us) | total (ms) | % |", "|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        t = float(r["TotalDurationNs"])
        if "collide_kernel" not in r["Name"] and t / tot < 1e-3:
            continue
        out.append("| `%s` | %s | %.1f | %.2f | %.2f |" % (
            r["Name"].replace("void mcc::", "").replace("mcc::", ""), r["Calls"],
            float(r["AverageNs"]) / 1e3, t / 1e6, 100.0 * t / tot))
    return "Command (repository root):\n\n    %s\n\n%s\n" % (command, "\n".join(out))


def calibration_kib(run_dir: str, counter: str) -> float:
    """The counter's reading for the copy kernel of a calibration run (the
    largest dispatch)."""
    best = 0.0
    for r in csv.DictReader(open(os.path.join(run_dir, "run_counter_collection.csv"))):
        if r["Counter_Name"] == counter and "copy" in r["Kernel_Name"].lower():
            best = max(best, float(r["Counter_Value"]))
    return best


def traffic(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, commands, copy_kib=1048576.0):
    f, nf, _ = counters(fetch_dir)
    w, _, _ = counters(write_dir)
    cf = calibration_kib(cal_fetch_dir, "FETCH_SIZE")
    cw = calibration_kib(cal_write_dir, "WRITE_SIZE")
    ff, wf = copy_kib / cf, copy_kib / cw
    lines = ["# HBM traffic per launch of the collide kernels, 65,536-cell bench workload, MI355X"]
    lines += ["# command: " + c for c in commands]
    lines += ["# calibration: a %d KiB device-to-device copy reads FETCH_SIZE %.0f KiB and "
              "WRITE_SIZE %.0f KiB" % (copy_kib, cf, cw),
              "# bytes = fetch_kib * 1024 * fetch_factor + write_kib * 1024 * write_factor "
              "(averages over all dispatches)",
              "# bench.py reports these only while source_sha256 matches the code of the collide "
              "kernels",
              "source_sha256 " + source_hash(),
              "fetch_factor %.4f" % ff, "write_factor %.4f" % wf]
    for k in sorted(f):
        if k not in w:
            continue
        fk, wk = f[k]["FETCH_SIZE"], w[k]["WRITE_SIZE"]
        lines.append("kernel %s %s %s fetch_kib %.1f write_kib %.1f dispatches %d bytes %.4g" % (
            k[0], k[1], k[2], fk, wk, nf[k], fk * 1024 * ff + wk * 1024 * wf))
    return "\n".join(lines) + "\n"


# MI355X: 256 CUs x 4 SIMDs; SQ_ACTIVE_INST_VALU counts quad-cycles per SIMD,
# GRBM_GUI_ACTIVE the GPU's busy cycles summed over its 8 XCDs
N_SIMD, N_XCD = 1024, 8


def valu(pass_a, pass_b, commands):
    a, na, meta = counters(pass_a)
    b, _, _ = counters(pass_b)
    lines = ["# VALU work per launch of the collide kernels, 65,536-cell bench workload, MI355X",
             "# (SQ counters summed over the chip, averaged over dispatches)"]
    lines += ["# command: " + c for c in commands]
    lines += ["# valu: SQ_INSTS_VALU (wave instructions); fp64_flops: 64 lanes x (ADD + MUL + "
              "TRANS + 2 FMA) F64 wave instructions (all lanes counted: an upper bound);",
              "# busy: SQ_ACTIVE_INST_VALU x 4 / (GRBM_GUI_ACTIVE / 8 x 1024 SIMDs); lanes: "
              "SQ_THREAD_CYCLES_VALU / (64 x SQ_ACTIVE_INST_VALU); wait: SQ_WAIT_INST_ANY / "
              "SQ_WAVE_CYCLES",
              "source_sha256 " + source_hash()]
    for k in sorted(a):
        c = dict(a[k])
        c.update(b.get(k, {}))
        f64 = 64.0 * (c.get("SQ_INSTS_VALU_ADD_F64", 0.0) + c.get("SQ_INSTS_VALU_MUL_F64", 0.0) +
                      c.get("SQ_INSTS_VALU_TRANS_F64", 0.0) +
                      2.0 * c.get("SQ_INSTS_VALU_FMA_F64", 0.0))
        busy = (c["SQ_ACTIVE_INST_VALU"] * 4.0 / (c["GRBM_GUI_ACTIVE"] / N_XCD * N_SIMD)
                if c.get("GRBM_GUI_ACTIVE") else float("nan"))
        lanes = (c["SQ_THREAD_CYCLES_VALU"] / (64.0 * c["SQ_ACTIVE_INST_VALU"])
                 if c.get("SQ_ACTIVE_INST_VALU") else float("nan"))
        wait = (c["SQ_WAIT_INST_ANY"] / c["SQ_WAVE_CYCLES"] if c.get("SQ_WAVE_CYCLES")
                else float("nan"))
        m = meta[k]
        lines.append("kernel %s %s %s valu %.5g fp64_flops %.5g busy %.3f lanes %.3f wait %.3f "
                     "lds %.5g salu %.5g waves %.0f vgpr %s lds_bytes %s scratch %s" % (
                         k[0], k[1], k[2], c["SQ_INSTS_VALU"], f64, busy, lanes, wait,
                         c.get("SQ_INSTS_LDS", float("nan")), c.get("SQ_INSTS_SALU", float("nan")),
                         c.get("SQ_WAVES", float("nan")), m["VGPR_Count"], m["LDS_Block_Size"],
                         m["Scratch_Size"]))
    return "\n".join(lines) + "\n"


def main(argv):
    what = argv[1]
    if what == "trace":
        sys.stdout.write(trace(argv[2], argv[3]))
    elif what == "traffic":
        sys.stdout.write(traffic(argv[2], argv[3], argv[4], argv[5], argv[6:]))
    elif what == "valu":
        sys.stdout.write(valu(argv[2], argv[3], argv[4:]))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv)
