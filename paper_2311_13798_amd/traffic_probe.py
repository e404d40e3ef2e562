"""Workload for the HBM-traffic counters of the dominant search launch (run under rocprofv3 --pmc).

Runs a plain device copy of known size (1 GiB read + 1 GiB written, torch elementwise kernel) that
calibrates FETCH_SIZE / WRITE_SIZE, then the R-MAT s18 workload's k = 9 count (after a k = 4 count
that builds the sub-branch arena, as the first count of a bench step does), whose width-class-3
search launch is the dominant launch of bench.py.
"""
import sys

import torch

import paper_2311_13798_amd as ebb
from graphgen import configs


def main():
    torch.cuda.set_device(0)
    n = 1 << 28  # float32 elements: 1 GiB
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    print("copy done", flush=True)
    k = int(sys.argv[1]) if len(sys.argv) > 1 else 9
    g = configs.rmat18()
    G = ebb.Graph.from_csr(g)
    G.count(4)
    print(f"k={k} count={G.count(k)} classes_ms={G.last_timing()}", flush=True)
    G.close()


if __name__ == "__main__":
    main()
