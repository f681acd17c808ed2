"""Writes the precision table: how often FP32 and float-float counts differ
from FP64 counts, by window width and iteration cap.

Calls only the CPU oracle (oracle/).  FP64 is the defining arithmetic (its
counts are the method's); FP32 and float-float are the two faster
formulations, and the fraction of pixels whose count differs from FP64 is
the accuracy they are judged by.  For every cell (width, cap) of
workloads.PRECISION_WIDTHS x workloads.PRECISION_CAPS the script takes the
cell's 32 windows (workloads.precision_windows: the serving stream's
constants and centres at that width, 640 x 480 grids) and 1024 probed pixels
of each, renders the probed pixels in all three formulations, and records

    pixels        probed pixels in the cell (32 x 1024)
    fp32_diff     probed pixels whose FP32 count differs from FP64
    ff_diff       the same for float-float
    fp32_worst    largest per-window fraction of differing pixels (FP32)
    ff_worst      the same for float-float

    python tests/golden/make_precision_table.py [--workers N]
"""
import argparse
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

OUT = os.path.join(HERE, "precision_table.txt")


def cell(job):
    width, cap = job
    wins = wl.precision_windows(wl.precision_seed(width, cap), width, cap)
    diff = {"fp32": 0, "ff": 0}
    worst = {"fp32": 0.0, "ff": 0.0}
    total = 0
    for w in wins:
        f = w.frame
        ii = np.asarray(w.ii, dtype=np.int32)
        jj = np.asarray(w.jj, dtype=np.int32)
        counts = {dt: oracle.render_pixels(f.c, f.window, f.width, f.height, cap, ii, jj, dt)
                  for dt in ("fp64", "fp32", "ff")}
        for dt in ("fp32", "ff"):
            d = int((counts[dt] != counts["fp64"]).sum())
            diff[dt] += d
            worst[dt] = max(worst[dt], d / ii.size)
        total += ii.size
    return width, cap, total, diff["fp32"], diff["ff"], worst["fp32"], worst["ff"]


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    a = p.parse_args()
    jobs = [(w, c) for w in wl.PRECISION_WIDTHS for c in wl.PRECISION_CAPS]
    with Pool(a.workers) as pool:
        rows = pool.map(cell, jobs)
    with open(OUT, "w") as out:
        out.write("# FP32 and float-float counts against FP64, by window width and cap.\n"
                  "# Windows: workloads.precision_windows (serving-stream constants and\n"
                  "# centres, 640x480 grids, 32 windows x 1024 probed pixels per cell).\n"
                  "# Written by tests/golden/make_precision_table.py (oracle only).\n"
                  "# columns: width cap pixels fp32_diff ff_diff fp32_worst ff_worst\n")
        for r in rows:
            out.write("%g %d %d %d %d %.6f %.6f\n" % r)
            print("width %-6g cap %-5d  fp32 %.4f%%  ff %.4f%%" % (
                r[0], r[1], 100.0 * r[3] / r[2], 100.0 * r[4] / r[2]), flush=True)
    print(OUT)


if __name__ == "__main__":
    main()
