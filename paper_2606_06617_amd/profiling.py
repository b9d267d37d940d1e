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

A traffic summary records the SHA-256 of the kernel source it was measured
on; bench.py reports the traffic only while the source is unchanged.

  python -m paper_2606_06617_amd.profiling stats <kernel_stats.csv> --out F --cmd "..."
  python -m paper_2606_06617_amd.profiling traffic <fetch.csv> <write.csv> --copy-bytes B --out F --cmd "..."

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
    a = ap.parse_args()
    if a.what == "stats":
        write_stats(kernel_stats(a.csv), a.out, a.cmd)
    else:
        tr, ff, fw = traffic(a.fetch_csv, a.write_csv, a.copy_bytes)
        write_traffic(tr, ff, fw, a.copy_bytes, a.out, a.cmd)


if __name__ == "__main__":
    main()
