"""HBM traffic of the dominant search launch, from rocprofv3 counters.

Run mode (under ``rocprofv3 --pmc FETCH_SIZE`` and again under ``--pmc WRITE_SIZE``):
``python3 -m paper_2311_13798_amd.traffic_probe [k]`` runs a plain device copy of known size (1 GiB
read + 1 GiB written, torch elementwise kernel) that calibrates the counters, then the R-MAT s18
workload's k = 9 count (after a k = 4 count that builds the sub-branch arena, as the first count of a
bench step does), whose width-class-3 search launch is the dominant launch of bench.py.

Record mode: ``python3 -m paper_2311_13798_amd.traffic_probe --record FETCH_DIR WRITE_DIR OUT.json
[k]`` reads the two runs' counter CSVs and writes, per launch of the search kernels, FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) and the HBM bytes they stand for, each counter scaled by the bytes the
copy kernel moves over what the same counter reads for it; with the hash of the kernel sources the
numbers belong to (bench.py reports them only while the sources are unchanged).
"""
import csv
import glob
import hashlib
import json
import os
import re
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COPY_BYTES = 1 << 30


def source_sha256() -> str:
    """Hash of the search kernel's sources."""
    h = hashlib.sha256()
    for f in ("search.hip", "arena.h", "device_util.h", "common.h"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def main(k: int = 9):
    import torch

    import paper_2311_13798_amd as ebb
    from graphgen import configs

    torch.cuda.set_device(0)
    n = COPY_BYTES // 4  # float32 elements
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    print("copy done", flush=True)
    g = configs.rmat18()
    G = ebb.Graph.from_csr(g)
    G.count(4)
    print(f"k={k} count={G.count(k)} classes_ms={G.last_timing()}", flush=True)
    G.close()


def _per_dispatch(run_dir: str, counter: str):
    """(kernel name, dispatch id) -> counter value summed over the CSV rows of that dispatch."""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {run_dir}")
    out = {}
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                key = (row["Kernel_Name"], int(row.get("Dispatch_Id", 0)))
                out[key] = out.get(key, 0.0) + float(row["Counter_Value"])
    return out


def write_record(fetch_dir: str, write_dir: str, out_json: str, k: int = 9, command: str = ""):
    fetch = _per_dispatch(fetch_dir, "FETCH_SIZE")
    write = _per_dispatch(write_dir, "WRITE_SIZE")

    def copy_kib(d):
        vals = [v for (name, _), v in d.items() if "elementwise" in name and "MulFunctor" in name]
        if not vals:
            raise ValueError("the copy kernel was not profiled")
        return max(vals)

    ff = COPY_BYTES / (copy_kib(fetch) * 1024.0)
    wf = COPY_BYTES / (copy_kib(write) * 1024.0)
    launches = {}
    for (name, _), fk in sorted(fetch.items(), key=lambda kv: kv[0][1]):
        m = re.search(r"k_search<(\d), false>", name)
        if not m:
            continue
        wk = next((v for (n2, _), v in write.items() if n2 == name), None)
        if wk is None:
            continue
        key = f"ebb::k_search<{m.group(1)}, false>@k={k}"
        launches[key] = {"fetch_KiB": fk, "write_KiB": wk,
                         "hbm_bytes": int(round(fk * 1024.0 * ff + wk * 1024.0 * wf))}
    rec = {"source_sha256": source_sha256(), "command": command,
           "copy_kernel": {"bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES,
                           "fetch_KiB": copy_kib(fetch), "write_KiB": copy_kib(write),
                           "fetch_scale": ff, "write_scale": wf},
           "launches": launches}
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--record":
        kk = int(sys.argv[5]) if len(sys.argv) > 5 else 9
        print(json.dumps(write_record(sys.argv[2], sys.argv[3], sys.argv[4], kk,
                                      " ".join(sys.argv[6:])), indent=1))
    else:
        main(int(sys.argv[1]) if len(sys.argv) > 1 else 9)
