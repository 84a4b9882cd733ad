"""Turn a rocprofv3 `--stats --output-format csv` kernel-statistics file into
a short markdown table (used for the summaries kept under profiles/).

Usage: python -m paper_2604_09233_amd.profile_summary <kernel_stats.csv> <title> <command> [note]
"""
import csv
import sys


def summarize(path, title, command, note=""):
    rows = list(csv.DictReader(open(path)))
    out = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", f"    {command}", "",
           "Per-kernel statistics from rocprofv3 (`--kernel-trace --stats`), durations in microseconds.", "",
           "| kernel | calls | total us | average us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].split("(")[0].replace("void ", "")
        out.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    if note:
        out += ["", note]
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    print(summarize(*sys.argv[1:]), end="")
