"""Turn rocprofv3 counter CSVs into HBM bytes per launch of a kernel.

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are each scaled by the value the
same counter reads for a plain copy of known size (``calib.py``), then
averaged over the launches of the kernel.  The summary is written as JSON
with a hash of the kernel sources, so that a later change of the kernel
invalidates it.
"""
import argparse
import csv
import glob
import json
import os


def counter_rows(path):
    rows = []
    for f in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def per_dispatch(rows, counter, name_part):
    vals = {}
    for r in rows:
        if r.get("Counter_Name") != counter or name_part not in r.get("Kernel_Name", ""):
            continue
        d = r.get("Dispatch_Id")
        vals[d] = vals.get(d, 0.0) + float(r["Counter_Value"])
    return list(vals.values())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True, help="rocprofv3 output dir of the FETCH_SIZE run")
    ap.add_argument("--write", required=True, help="rocprofv3 output dir of the WRITE_SIZE run")
    ap.add_argument("--calib-fetch", required=True)
    ap.add_argument("--calib-write", required=True)
    ap.add_argument("--calib-bytes", type=float, required=True)
    ap.add_argument("--kernel", required=True, help="substring of the kernel name")
    ap.add_argument("--particles", type=float, required=True, help="particles per launch")
    ap.add_argument("--hash", required=True)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    cf = per_dispatch(counter_rows(a.calib_fetch), "FETCH_SIZE", "")
    cw = per_dispatch(counter_rows(a.calib_write), "WRITE_SIZE", "")
    # The copy kernel is the dispatch with the largest counts.
    f_fac = max(cf) * 1024.0 / a.calib_bytes
    w_fac = max(cw) * 1024.0 / a.calib_bytes
    kf = per_dispatch(counter_rows(a.fetch), "FETCH_SIZE", a.kernel)
    kw = per_dispatch(counter_rows(a.write), "WRITE_SIZE", a.kernel)
    # Skip the first launches (initial unsorted state).
    kf_s = kf[len(kf) // 2:] or kf
    kw_s = kw[len(kw) // 2:] or kw
    fetch = sum(kf_s) / len(kf_s) * 1024.0 / f_fac
    write = sum(kw_s) / len(kw_s) * 1024.0 / w_fac
    out = dict(kernel=a.kernel, kernel_hash=a.hash, fetch_bytes_per_launch=fetch,
               write_bytes_per_launch=write, bytes_per_launch=fetch + write,
               bytes_per_particle=(fetch + write) / a.particles, fetch_factor=f_fac,
               write_factor=w_fac, launches=len(kf_s))
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
