"""Turn rocprofv3 CSV output into the short markdown summaries kept under
profiles/.

  python -m paper_2604_09233_amd.profile_summary stats <kernel_stats.csv> <title> <command> [note]
      per-kernel durations from `--kernel-trace --stats`
  python -m paper_2604_09233_amd.profile_summary counters <out.md> <precision> <workload> <bench-args> \
      <command-prefix> <copy-bytes> <sq_dir> [<sq_dir> ...] <fetch_dir> <write_dir> <copy_fetch_dir> <copy_write_dir>
      per-dispatch counter averages of the encode kernels from `--pmc` runs
      (each *_dir holds run_counter_collection.csv and run_kernel_trace.csv),
      the HBM traffic per launch from FETCH_SIZE / WRITE_SIZE scaled by what
      the same counters read for a plain copy of <copy-bytes> bytes, and the
      SHA-256 of the encode-kernel sources the counters were taken on (the
      benchmark reports the traffic only while the sources still match);
      the traffic line covers the kernels of <precision> (fp32, bf16, fp16).
"""
import csv
import hashlib
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_TAG = "encode-kernel traffic per launch (bytes):"
# what the encode kernels' machine code depends on: their source file, the
# part of the shared header before the launcher declarations (constants,
# shape and work-list structs, the split-sum helper), and the compiler flags
# they are built with
_HEADER_END = "// ---- launchers (encode_kernels.hip)"


def kernel_source_hash() -> str:
    from . import build

    h = hashlib.sha256()
    with open(os.path.join(HERE, "csrc", "encode_kernels.hip"), "rb") as f:
        h.update(f.read())
    with open(os.path.join(HERE, "csrc", "nfs_internal.h")) as f:
        hdr = f.read()
    h.update(hdr[:hdr.index(_HEADER_END)].encode())
    flags = build.COMMON + build.DEVICE_FLAGS + build.SOURCE_FLAGS.get("encode_kernels.hip", [])
    h.update(" ".join(f for f in flags if not f.startswith("/")).encode())
    return h.hexdigest()


def read_traffic(md_path):
    """{kernel short name: bytes per launch} from a counters summary, or None
    when the summary is missing or was taken on other kernel sources."""
    if not os.path.exists(md_path):
        return None
    out, sha = {}, None
    for line in open(md_path):
        line = line.strip()
        if line.startswith(TRAFFIC_TAG):
            for tok in line[len(TRAFFIC_TAG):].split():
                k, v = tok.split("=")
                if k == "sources_sha256":
                    sha = v
                else:
                    out[k] = float(v)
    if not out or sha != kernel_source_hash():
        return None
    return out


def summarize(path, title, command, note=""):
    rows = list(csv.DictReader(open(path)))
    out = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", f"    {command}", "",
           "Per-kernel statistics from rocprofv3 (`--kernel-trace --stats`), durations in microseconds.", "",
           "| kernel | calls | total us | average us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = _short(r["Name"])
        out.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    if note:
        out += ["", note]
    return "\n".join(out) + "\n"


def _short(name):
    """Kernel name without its parameter list ('(anonymous namespace)::'
    dropped first, so that it is not taken for the parameter list)."""
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0].replace("void ", "").strip()


def _per_dispatch(d, match=None):
    """{kernel: {counter: mean per dispatch}} and {kernel: mean duration ns}."""
    vals = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
        k = _short(r["Kernel_Name"])
        if match and match not in k:
            continue
        vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    dur = defaultdict(list)
    for r in csv.DictReader(open(os.path.join(d, "run_kernel_trace.csv"))):
        k = _short(r["Kernel_Name"])
        if match and match not in k:
            continue
        dur[k].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return ({k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in vals.items()},
            {k: sum(v) / len(v) for k, v in dur.items()})


PREC_ARG = {"fp32": "0", "bf16": "1", "fp16": "2"}


def counters(out_md, precision, workload, bench_args, command, copy_bytes, *dirs):
    sq_dirs, (fetch_dir, write_dir, cfetch_dir, cwrite_dir) = dirs[:-4], dirs[-4:]
    copy_bytes = float(copy_bytes)
    merged, durs = defaultdict(dict), defaultdict(list)
    for d in sq_dirs:
        v, t = _per_dispatch(d, "encode_kernel")
        for k, cs in v.items():
            merged[k].update(cs)
            durs[k].append(t[k])
    fetch, tf = _per_dispatch(fetch_dir, "encode_kernel")
    write, tw = _per_dispatch(write_dir, "encode_kernel")
    cf, _ = _per_dispatch(cfetch_dir)
    cw, _ = _per_dispatch(cwrite_dir)
    # the copy is the largest FETCH/WRITE dispatch of its run
    cfk = max(cf, key=lambda k: cf[k].get("FETCH_SIZE", 0.0))
    cwk = max(cw, key=lambda k: cw[k].get("WRITE_SIZE", 0.0))
    f_fac = copy_bytes / (cf[cfk]["FETCH_SIZE"] * 1024.0)
    w_fac = copy_bytes / (cw[cwk]["WRITE_SIZE"] * 1024.0)
    lines = [f"# Encode-kernel counters: CG solve, {workload}, {precision.upper()} operands", "",
             "encode_kernel<OP, PREC, NQ, NB, MT>: OP 0 = E, 1 = E^H; PREC 0 = fp32, 1 = bf16, 2 = fp16; NQ phase "
             "instructions per tile, NB column blocks, MT held tiles per wave. The run also holds the single "
             "FP32 E that generates the data.", "",
             "Commands (from the repository root, one MI355X), one rocprofv3 run per counter set:", "",
             f"    {command} --pmc <counters> -- python3 bench.py {bench_args}", "",
             "with these counter sets (one run each):", ""]
    for i, d in enumerate(list(sq_dirs) + [fetch_dir, write_dir]):
        names = sorted({r["Counter_Name"] for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv")))})
        lines.append(f"{i + 1}. `{' '.join(names)}`")
    lines += ["",
             "Copy calibration: the same FETCH_SIZE / WRITE_SIZE runs over `torch` copying "
             f"{copy_bytes / 2**20:.0f} MiB (`{cfk}`): FETCH_SIZE reads {cf[cfk]['FETCH_SIZE']:.0f} KiB "
             f"(factor {f_fac:.3f}), WRITE_SIZE {cw[cwk]['WRITE_SIZE']:.0f} KiB (factor {w_fac:.3f}).", ""]
    traffic = {}
    for k in sorted(merged):
        c = merged[k]
        dur = sum(durs[k]) / len(durs[k]) * 1e-9
        op = "E" if "encode_kernel<0" in k else "EH"
        lines += [f"## `{k}` ({op})", "", f"Mean dispatch duration under counter collection: {dur * 1e6:.1f} us.", "",
                  "| counter | per dispatch |", "|---|---|"]
        for name in sorted(c):
            lines.append(f"| {name} | {c[name]:.4g} |")
        lines.append("")
        derived = []
        if "SQ_INSTS_VALU_MFMA_MOPS_F16" in c:
            fl = c["SQ_INSTS_VALU_MFMA_MOPS_F16"] * 512
            derived.append(f"f16 MFMA: {fl:.3g} flop per dispatch, {fl / dur / 1e12:.0f} TFLOP/s = "
                           f"{fl / dur / 2.5e15:.1%} of the 2.5 PFLOP/s dense peak")
        if "SQ_INSTS_VALU_TRANS_F32" in c:
            tr = c["SQ_INSTS_VALU_TRANS_F32"] * 64
            derived.append(f"transcendental: {tr:.3g} lane ops per dispatch, {tr / dur / 1e12:.2f} T/s = "
                           f"{tr / dur / 1.966e13:.1%} of 1.966e13/s (256 CU x 4 SIMD x 8 lanes x 2.4 GHz)")
        if "SQ_INSTS_VALU" in c and "SQ_INSTS_MFMA" in c:
            nv = c["SQ_INSTS_VALU"] - c["SQ_INSTS_MFMA"]
            derived.append(f"VALU (non-MFMA) wave instructions: {nv:.3g} per dispatch, issue rate "
                           f"{nv / dur / 1024 / 2.4e9 * 4:.1%} of one 4-cycle wave64 op per SIMD per clock")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in c:
            derived.append(f"MFMA busy: {c['SQ_VALU_MFMA_BUSY_CYCLES'] / (1024 * dur * 2.4e9):.1%} of SIMD-cycles "
                           "at 2.4 GHz")
        prec_ok = k.split("<")[1].split(",")[1].strip() == PREC_ARG[precision]
        if prec_ok and k in fetch and k in write:
            fb = fetch[k]["FETCH_SIZE"] * 1024.0 * f_fac
            wb = write[k]["WRITE_SIZE"] * 1024.0 * w_fac
            traffic[op] = fb + wb
            derived.append(f"HBM traffic (calibrated): fetch {fb / 1e6:.1f} MB + write {wb / 1e6:.1f} MB = "
                           f"{(fb + wb) / 1e6:.1f} MB per dispatch")
        lines += [f"- {x}" for x in derived] + [""]
    lines += [TRAFFIC_TAG + " " + " ".join(f"{k}={v:.0f}" for k, v in sorted(traffic.items())) +
              f" sources_sha256={kernel_source_hash()}", ""]
    with open(out_md, "w") as f:
        f.write("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(summarize(*sys.argv[2:]), end="")
    elif sys.argv[1] == "counters":
        counters(*sys.argv[2:])
    else:
        print(summarize(*sys.argv[1:]), end="")
