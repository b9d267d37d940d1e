"""Summaries of rocprofv3 output for the kernels of this library.

Two kinds of text summary, written under profiles/ and read back by
bench.py:

* kernel statistics from ``rocprofv3 --kernel-trace --stats`` (the
  ``*_kernel_stats.csv`` file): calls, total and average duration per
  kernel;
* HBM traffic from two ``rocprofv3 --pmc`` runs, one with FETCH_SIZE and one
  with WRITE_SIZE (KiB per dispatch).  The counters do not read bytes
  one-to-one on every part, so each is scaled by what it reads for a plain
  device-to-device copy of known size launched in the same process
  (``bench.py --calib-copy-mib``): factor = copy bytes / counter bytes.

* instruction and unit counters (``rocprofv3 --pmc`` with SQ counters, at
  most 8 per run) of chosen kernels: per-dispatch means, per-atom counts and
  utilisations derived with the kernel's average duration from a
  kernel-trace summary and the chip's 256 CUs x 4 SIMDs at 2.4 GHz.

A traffic or counter summary records the SHA-256 of the kernel source it
was measured on; bench.py reports the traffic only while the source is
unchanged.

  python -m paper_2606_06617_amd.profiling stats <kernel_stats.csv> --out F --cmd "..."
  python -m paper_2606_06617_amd.profiling traffic <fetch.csv> <write.csv> --copy-bytes B --out F --cmd "..."
  python -m paper_2606_06617_amd.profiling counters <pmc1.csv> [<pmc2.csv> ...] --stats S --atoms N
         --kernels K1 K2 --out F --cmd "..."

B is what the copy moves in total, read plus written (2 x --calib-copy-mib
MiB, the calib_copy_bytes bench.py prints).
"""
import argparse
import collections
import csv
import hashlib
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCE = os.path.join(ROOT, "paper_2606_06617_amd", "csrc", "kernels.hip")
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def source_hash(path=KERNEL_SOURCE):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def short_name(name):
    """void pswf::k_spread<8, 4>(pswf::Geo, ...) -> k_spread<8,4>"""
    n = name.split("(")[0]
    if n.startswith("void "):
        n = n[5:]
    return n.replace("pswf::", "").replace(" ", "")


def kernel_stats(path):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        out.append({"kernel": short_name(r["Name"]), "calls": int(r["Calls"]),
                    "total_ms": float(r["TotalDurationNs"]) * 1e-6,
                    "avg_us": float(r["AverageNs"]) * 1e-3,
                    "min_us": float(r["MinNs"]) * 1e-3, "max_us": float(r["MaxNs"]) * 1e-3,
                    "pct": float(r["Percentage"])})
    return out


def counter_means(path, counter):
    """Mean counter value per dispatch for every kernel (KiB for *_SIZE)."""
    acc = collections.defaultdict(float)
    disp = collections.defaultdict(set)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = short_name(r["Kernel_Name"])
        acc[k] += float(r["Counter_Value"])
        disp[k].add(r["Dispatch_Id"])
    return {k: acc[k] / len(disp[k]) for k in acc}


def traffic(fetch_csv, write_csv, copy_bytes):
    fetch = counter_means(fetch_csv, "FETCH_SIZE")
    write = counter_means(write_csv, "WRITE_SIZE")
    if COPY_KERNEL not in fetch or COPY_KERNEL not in write:
        raise SystemExit("no %s dispatch in the counter files: run bench.py with --calib-copy-mib" % COPY_KERNEL)
    # the copy reads and writes copy_bytes / 2 each
    ff = (copy_bytes / 2) / (fetch[COPY_KERNEL] * 1024.0)
    fw = (copy_bytes / 2) / (write[COPY_KERNEL] * 1024.0)
    out = {}
    for k in sorted(set(fetch) | set(write)):
        fb = fetch.get(k, 0.0) * 1024.0 * ff
        wb = write.get(k, 0.0) * 1024.0 * fw
        out[k] = {"fetch_kib": fetch.get(k, 0.0), "write_kib": write.get(k, 0.0),
                  "fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb}
    return out, ff, fw


def write_stats(rows, out, cmd):
    with open(out, "w") as f:
        f.write("# rocprofv3 kernel statistics\n# command: %s\n" % cmd)
        f.write("%-34s %6s %11s %11s %11s %11s %6s\n" % ("kernel", "calls", "total_ms", "avg_us", "min_us",
                                                        "max_us", "pct"))
        for r in rows:
            f.write("%-34s %6d %11.3f %11.2f %11.2f %11.2f %6.2f\n" % (r["kernel"][:34], r["calls"], r["total_ms"],
                                                                   r["avg_us"], r["min_us"], r["max_us"], r["pct"]))


def write_traffic(tr, ff, fw, copy_bytes, out, cmd):
    with open(out, "w") as f:
        f.write("# HBM traffic per dispatch from rocprofv3 FETCH_SIZE and WRITE_SIZE (separate runs)\n")
        f.write("# command: %s\n" % cmd)
        f.write("# calibration: %s copying %d bytes; fetch factor %.4f, write factor %.4f\n"
                % (COPY_KERNEL, copy_bytes, ff, fw))
        f.write("source_sha256 %s\n" % source_hash())
        f.write("%-34s %14s %14s %16s %16s %16s\n" % ("kernel", "FETCH_KiB", "WRITE_KiB", "fetch_bytes",
                                                     "write_bytes", "bytes"))
        for k, v in tr.items():
            f.write("%-34s %14.1f %14.1f %16.0f %16.0f %16.0f\n" % (k[:34], v["fetch_kib"], v["write_kib"],
                                                                  v["fetch_bytes"], v["write_bytes"], v["bytes"]))


def read_traffic(path):
    """{kernel: bytes per dispatch} and the recorded source hash, or (None, None)."""
    if not os.path.exists(path):
        return None, None
    sha, rows = None, {}
    for line in open(path):
        if line.startswith("#"):
            continue
        parts = line.split()
        if parts and parts[0] == "source_sha256":
            sha = parts[1]
        elif len(parts) == 6 and parts[0] != "kernel":
            rows[parts[0]] = float(parts[5])
    return rows, sha


CLOCK_HZ = 2.4e9
SIMDS = 256 * 4


def counter_table(paths, kernels):
    """{kernel: {counter: mean per dispatch}} over every counter in the files."""
    acc = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(lambda: collections.defaultdict(set))
    regs = {}
    for path in paths:
        for r in csv.DictReader(open(path)):
            k = short_name(r["Kernel_Name"])
            if k not in kernels:
                continue
            acc[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[k][r["Counter_Name"]].add((path, r["Dispatch_Id"]))
            regs[k] = (r.get("VGPR_Count"), r.get("Accum_VGPR_Count"), r.get("SGPR_Count"), r.get("LDS_Block_Size"))
    return {k: {c: acc[k][c] / len(disp[k][c]) for c in acc[k]} for k in acc}, regs


def derived(cnt, avg_us, atoms):
    """Per-atom instruction counts and unit utilisations of one kernel.

    valu_busy = 4 SQ_ACTIVE_INST_VALU / (SIMDs x cycles of the launch),
    mfma_busy = SQ_VALU_MFMA_BUSY_CYCLES / (SIMDs x cycles),
    lds_bank_conflict = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE,
    with cycles = average duration x 2.4 GHz."""
    cyc = avg_us * 1e-6 * CLOCK_HZ
    out = {}
    for c, label in (("SQ_INSTS_VALU", "valu_per_atom"), ("SQ_INSTS_SALU", "salu_per_atom"),
                     ("SQ_INSTS_LDS", "lds_per_atom"), ("SQ_INSTS_VALU_MFMA_F32", "mfma_f32_per_atom")):
        if c in cnt:
            out[label] = cnt[c] / atoms
    if "SQ_ACTIVE_INST_VALU" in cnt and cyc > 0:
        out["valu_busy"] = 4.0 * cnt["SQ_ACTIVE_INST_VALU"] / (SIMDS * cyc)
    if "SQ_VALU_MFMA_BUSY_CYCLES" in cnt and cyc > 0:
        out["mfma_busy"] = cnt["SQ_VALU_MFMA_BUSY_CYCLES"] / (SIMDS * cyc)
    if "SQ_LDS_BANK_CONFLICT" in cnt and cnt.get("SQ_LDS_IDX_ACTIVE"):
        out["lds_bank_conflict"] = cnt["SQ_LDS_BANK_CONFLICT"] / cnt["SQ_LDS_IDX_ACTIVE"]
    return out


def write_counters(table, regs, stats, atoms, out, cmd):
    avg = {r["kernel"]: r["avg_us"] for r in stats}
    with open(out, "w") as f:
        f.write("# rocprofv3 SQ counters per dispatch (separate --pmc runs of at most 8 counters)\n")
        f.write("# command: %s\n" % cmd)
        f.write("# durations from the kernel-trace summary; utilisations over 256 CUs x 4 SIMDs at 2.4 GHz:\n")
        f.write("#   valu_busy = 4 SQ_ACTIVE_INST_VALU / (SIMDs x cycles), mfma_busy = SQ_VALU_MFMA_BUSY_CYCLES /\n")
        f.write("#   (SIMDs x cycles), lds_bank_conflict = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE; per-atom counts\n")
        f.write("#   are wave instructions per atom of the %d-atom frame\n" % atoms)
        f.write("source_sha256 %s\n" % source_hash())
        for k in sorted(table):
            v, a, sg, lds = regs.get(k, (None,) * 4)
            f.write("\n[%s] avg %.2f us; VGPR %s AGPR %s SGPR %s LDS %s B\n" % (k, avg.get(k, float("nan")), v, a, sg,
                                                                             lds))
            for c in sorted(table[k]):
                f.write("  %-28s %18.1f\n" % (c, table[k][c]))
            for name, val in derived(table[k], avg.get(k, 0.0), atoms).items():
                f.write("  %-28s %18.4f\n" % (name, val))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--out", required=True)
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--copy-bytes", type=int, required=True,
                   help="bytes the calibration copy moves, read plus written (bench.py's calib_copy_bytes: "
                        "2 x --calib-copy-mib MiB)")
    t.add_argument("--out", required=True)
    t.add_argument("--cmd", required=True)
    u = sub.add_parser("counters")
    u.add_argument("csvs", nargs="+")
    u.add_argument("--stats", required=True, help="kernel_stats.csv of a kernel-trace run of the same command")
    u.add_argument("--atoms", type=int, required=True)
    u.add_argument("--kernels", nargs="+", required=True)
    u.add_argument("--out", required=True)
    u.add_argument("--cmd", required=True)
    a = ap.parse_args()
    if a.what == "stats":
        write_stats(kernel_stats(a.csv), a.out, a.cmd)
    elif a.what == "counters":
        table, regs = counter_table(a.csvs, set(a.kernels))
        write_counters(table, regs, kernel_stats(a.stats), a.atoms, a.out, a.cmd)
    else:
        tr, ff, fw = traffic(a.fetch_csv, a.write_csv, a.copy_bytes)
        write_traffic(tr, ff, fw, a.copy_bytes, a.out, a.cmd)


if __name__ == "__main__":
    main()
