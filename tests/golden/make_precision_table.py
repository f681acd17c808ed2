"""Writes the precision table: how often FP32 and float-float counts differ
from FP64 counts, by window width and iteration cap.

Calls only the CPU oracle (oracle/).  FP64 is the defining arithmetic (its
counts are the method's); FP32 and float-float are the two faster
formulations, and the fraction of pixels whose count differs from FP64 is
the accuracy they are judged by.  For every cell (kind, width, cap) of
{serving, boundary} x workloads.PRECISION_WIDTHS x workloads.PRECISION_CAPS
the script takes the cell's 32 windows (workloads.probe_windows: the serving
stream's constants and centres at that width, or the same constants with
windows centred on the Julia set; 640 x 480 grids) and 1024 probed pixels of
each, renders the probed pixels in all three formulations, and records

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
    kind, width, cap = job
    wins = wl.probe_windows(kind, width, cap)
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
    return kind, width, cap, total, diff["fp32"], diff["ff"], worst["fp32"], worst["ff"]


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    a = p.parse_args()
    jobs = [(k, w, c) for k in ("serving", "boundary") for w in wl.PRECISION_WIDTHS
            for c in wl.PRECISION_CAPS]
    # the most expensive cells (boundary windows, large caps) first
    order = sorted(range(len(jobs)), key=lambda i: (jobs[i][0] != "boundary", -jobs[i][2]))
    with Pool(a.workers) as pool:
        got = dict(zip(order, pool.map(cell, [jobs[i] for i in order])))
    rows = [got[i] for i in range(len(jobs))]
    with open(OUT, "w") as out:
        out.write("# FP32 and float-float counts against FP64, by window width and cap.\n"
                  "# Windows (640x480 grids, 32 windows x 1024 probed pixels per cell):\n"
                  "#   serving   workloads.precision_windows: the serving stream's constants\n"
                  "#             and centres (uniform in [-1.5, 1.5]^2);\n"
                  "#   boundary  workloads.boundary_windows: the same constants, each window\n"
                  "#             centred on a point of the Julia set J(C).\n"
                  "# Written by tests/golden/make_precision_table.py (oracle only).\n"
                  "# columns: kind width cap pixels fp32_diff ff_diff fp32_worst ff_worst\n")
        for r in rows:
            out.write("%s %g %d %d %d %d %.6f %.6f\n" % r)
            print("%-8s width %-6g cap %-5d  fp32 %.4f%%  ff %.4f%%" % (
                r[0], r[1], r[2], 100.0 * r[4] / r[3], 100.0 * r[5] / r[3]), flush=True)
    print(OUT)


if __name__ == "__main__":
    main()
