"""HBM traffic and VALU issue of a kernel from rocprofv3 counter runs.

Two programs run under `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` (one counter
per run): the workload, and a device copy of known size that calibrates what each counter
reports per byte on this GPU.  `summarize` turns the four result databases into a
per-launch byte count for one kernel and records it in profiles/<profile>_traffic.json
(<profile>: the summary the counters belong to, --profile), keyed by the library's
timing label, with a hash of the kernel's sources so that a changed kernel is
not credited with old counters.

    python -m paper_1104_3870_amd.profile_traffic copy            # calibration program
    python -m paper_1104_3870_amd.profile_traffic sq --dir DIR --match 'k_dslash_lds<S16, 1, false>' ...
        # mean SQ_WAVES, SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, SQ_BUSY_CYCLES, GRBM_GUI_ACTIVE per
        # dispatch of each matched kernel, and VALU instructions per wave
    python -m paper_1104_3870_amd.profile_traffic summarize --label 'dslash_lds<f16,inv,R32>' \\
        --match 'k_dslash_lds<S16, 1, false>' --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \\
        --sources paper_1104_3870_amd/csrc/dslash_mr.hip --profile NAME
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30
COPY_KERNEL = "copyBuffer"


def copy_program(reps=5):
    import torch

    a = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied %d x %d bytes" % (reps, COPY_BYTES))


def counter_avg(directory, match, counter):
    """Mean counter value per dispatch (FETCH_SIZE, WRITE_SIZE: KB) of kernels whose name
    contains `match`."""
    dbs = glob.glob(os.path.join(directory, "**", "*.db"), recursive=True)
    if not dbs:
        raise FileNotFoundError("no rocprofv3 database under %s" % directory)
    vals = []
    for db in dbs:
        con = sqlite3.connect(db)
        rows = con.execute("select kernel_name, value from counters_collection where counter_name = ?",
                           (counter,)).fetchall()
        vals += [float(v) for k, v in rows if match in k]
        con.close()
    if not vals:
        raise ValueError("no %s samples for kernels matching %r in %s" % (counter, match, directory))
    return sum(vals) / len(vals), len(vals)


def sources_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def summarize(a):
    f_kb, nf = counter_avg(a.fetch, a.match, "FETCH_SIZE")
    w_kb, nw = counter_avg(a.write, a.match, "WRITE_SIZE")
    cf_kb, _ = counter_avg(a.copy_fetch, COPY_KERNEL, "FETCH_SIZE")
    cw_kb, _ = counter_avg(a.copy_write, COPY_KERNEL, "WRITE_SIZE")
    sf = COPY_BYTES / (cf_kb * 1024.0)  # bytes per reported byte
    sw = COPY_BYTES / (cw_kb * 1024.0)
    fetch = f_kb * 1024.0 * sf
    write = w_kb * 1024.0 * sw
    rec = {"kernel_match": a.match, "dispatches": [nf, nw], "fetch_kb": f_kb, "write_kb": w_kb,
           "fetch_scale": sf, "write_scale": sw, "fetch_bytes": fetch, "write_bytes": write,
           "bytes_per_launch": fetch + write, "sources": a.sources, "sources_sha256": sources_sha(a.sources),
           "profile": a.profile}
    path = os.path.join(ROOT, "profiles", os.path.splitext(a.profile)[0] + "_traffic.json")
    allrec = {}
    if os.path.exists(path):
        with open(path) as f:
            allrec = json.load(f)
    allrec[a.label] = rec
    with open(path, "w") as f:
        json.dump(allrec, f, indent=1, sort_keys=True)
    print(json.dumps({a.label: rec}, indent=1))


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE")


def sq(a):
    out = {}
    for m in a.match:
        rec = {}
        for ctr in SQ_COUNTERS:
            try:
                rec[ctr], rec["dispatches"] = counter_avg(a.dir, m, ctr)
            except ValueError:
                rec[ctr] = None
        if rec.get("SQ_WAVES") and rec.get("SQ_INSTS_VALU") is not None:
            rec["valu_insts_per_wave"] = rec["SQ_INSTS_VALU"] / rec["SQ_WAVES"]
        out[m] = rec
    print(json.dumps(out, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("copy")
    s = sub.add_parser("summarize")
    s.add_argument("--label", required=True)
    s.add_argument("--match", required=True)
    for k in ("fetch", "write", "copy-fetch", "copy-write"):
        s.add_argument("--" + k, required=True)
    s.add_argument("--sources", nargs="+", required=True)
    s.add_argument("--profile", required=True)
    q = sub.add_parser("sq")
    q.add_argument("--dir", required=True)
    q.add_argument("--match", nargs="+", required=True)
    a = ap.parse_args()
    if a.cmd == "copy":
        copy_program()
    elif a.cmd == "sq":
        sq(a)
    else:
        summarize(a)
    return 0


if __name__ == "__main__":
    sys.exit(main())
