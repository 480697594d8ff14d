"""Summaries of rocprofv3 runs of the benchmark, for the profiles/ folder.

    python -m paper_2208_09136_amd.profsum stats DIR
        Markdown table of a `rocprofv3 --kernel-trace --stats` run: calls,
        total and average duration per kernel (from *_kernel_stats.csv).
    python -m paper_2208_09136_amd.profsum counters OUT.json SQ_DIR FETCH_DIR WRITE_DIR [--copy-bytes B]
        Per-dispatch averages of `rocprofv3 --pmc` runs (one directory per
        run, *_counter_collection.csv) for the kernels of the timed step,
        keyed by their role (select_pass1, select_pass2, window_pass1,
        sweep); FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by
        what the same counters read for the plain device copy of B bytes
        the benchmark makes after its steps (--copy-mib).  Writes OUT.json
        (with the digest of the device sources it describes) and prints a
        markdown table.
"""
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def sources_digest():
    """SHA-256 over the device sources (the same digest bench.py checks)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2208_09136_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def short_name(kernel):
    """Kernel name without its return type and parameter list."""
    name = kernel[5:] if kernel.startswith("void ") else kernel
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def role_of(kernel):
    """Role of a kernel in the step, or None."""
    name = short_name(kernel)
    for prefix, role in (("rqa::k_select<1,", "select_pass1"), ("rqa::k_select<2,", "select_pass2"),
                         ("rqa::k_window<1,", "window_pass1"), ("rqa::k_range_sweep<", "sweep")):
        if name.startswith(prefix):
            return role
    return None


def find(dirname, suffix):
    hits = sorted(glob.glob(os.path.join(dirname, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {dirname}")
    return hits


def stats_table(dirname):
    rows = []
    for path in find(dirname, "_kernel_stats.csv"):
        with open(path) as f:
            rows += list(csv.DictReader(f))
    out = ["| kernel | calls | total us | average us | % |", "|---|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def counter_means(dirname):
    """{kernel name: {counter: mean per dispatch}} of one --pmc run; for the
    device copy kernel, which also moves the small per-call descriptors, the
    largest dispatch (the calibration copy)."""
    acc = defaultdict(lambda: defaultdict(list))
    for path in find(dirname, "_counter_collection.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                acc[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: (max(v) if k == COPY_KERNEL else sum(v) / len(v)) for c, v in cs.items()}
            for k, cs in acc.items()}


def counters(out_json, sq_dir, fetch_dir, write_dir, copy_bytes):
    sq, fe, wr = counter_means(sq_dir), counter_means(fetch_dir), counter_means(write_dir)
    copy_kib = float(copy_bytes) / 1024.0
    fetch_factor = copy_kib / fe[COPY_KERNEL]["FETCH_SIZE"] if COPY_KERNEL in fe else None
    write_factor = copy_kib / wr[COPY_KERNEL]["WRITE_SIZE"] if COPY_KERNEL in wr else None
    kernels = {}
    for name, cs in sq.items():
        role = role_of(name)
        if role is None:
            continue
        k = {"kernel": short_name(name), "valu_insts": cs.get("SQ_INSTS_VALU"), "salu_insts": cs.get("SQ_INSTS_SALU"),
             "lds_insts": cs.get("SQ_INSTS_LDS"), "active_inst_valu": cs.get("SQ_ACTIVE_INST_VALU"),
             "wait_inst_lds": cs.get("SQ_WAIT_INST_LDS"), "lds_bank_conflict": cs.get("SQ_LDS_BANK_CONFLICT"),
             "busy_cycles": cs.get("SQ_BUSY_CYCLES"), "gui_active": cs.get("GRBM_GUI_ACTIVE")}
        if name in fe and fetch_factor:
            k["fetch_bytes"] = fe[name]["FETCH_SIZE"] * 1024.0 * fetch_factor
        if name in wr and write_factor:
            k["write_bytes"] = wr[name]["WRITE_SIZE"] * 1024.0 * write_factor
        kernels[role] = k
    doc = {"sources_sha256": sources_digest(),
           "calibration": {"copy_bytes": copy_bytes, "fetch_factor": fetch_factor, "write_factor": write_factor},
           "kernels": kernels}
    with open(out_json, "w") as f:
        json.dump(doc, f, indent=1)
    lines = ["| role | kernel | VALU insts | SALU insts | LDS insts | LDS bank-conflict | LDS wait | "
             "HBM read MB | HBM write MB |", "|---|---|---:|---:|---:|---:|---:|---:|---:|"]
    for role, k in sorted(kernels.items()):
        def g(x, scale=1.0, fmt="{:.3e}"):
            return fmt.format(x * scale) if x is not None else "-"
        lines.append(f"| {role} | `{k['kernel']}` | {g(k['valu_insts'])} | {g(k['salu_insts'])} | "
                     f"{g(k['lds_insts'])} | {g(k['lds_bank_conflict'])} | {g(k['wait_inst_lds'])} | "
                     f"{g(k.get('fetch_bytes'), 1e-6, '{:.1f}')} | {g(k.get('write_bytes'), 1e-6, '{:.1f}')} |")
    print(f"fetch factor {fetch_factor}, write factor {write_factor}")
    print("\n".join(lines))


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(stats_table(argv[1]))
    elif len(argv) >= 5 and argv[0] == "counters":
        copy_bytes = 256 << 20
        if "--copy-bytes" in argv:
            copy_bytes = int(argv[argv.index("--copy-bytes") + 1])
        counters(argv[1], argv[2], argv[3], argv[4], copy_bytes)
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
