"""Writes the oracle's count sums of the full-size benchmark workloads.

Calls only the CPU oracle (oracle/): every value in the files it writes is
the oracle's, never the GPU library's.  Frames are rendered in parallel
processes; each is one plain oracle call.  Run from the repository root:

    python tests/golden/make_workload_sums.py

Files:
  parameter_path_fp32_sums.txt   the 256 frames of the parameter path
                                 (1920x1080, cap 100, FP32 formulation)
  general_path_deg3_fp32_sums.txt  the 32 frames of the Z^3 + C path
"""
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as wl  # noqa: E402


def frame_stats(f):
    a = oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, f.mode,
                      getattr(f, "degree", 2))
    return int(a.sum(dtype=np.int64)), int((a == f.max_iter).sum()), int((a == 0).sum())


def write(name, frames, header):
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        stats = pool.map(frame_stats, frames)
    path = os.path.join(HERE, name)
    with open(path, "w") as out:
        out.write(header)
        out.write("# columns: frame count_sum pixels_at_cap pixels_at_zero\n")
        for k, (s, capped, zero) in enumerate(stats):
            out.write("%d %d %d %d\n" % (k, s, capped, zero))
        out.write("# total %d\n" % sum(s for s, _, _ in stats))
    print(path, sum(s for s, _, _ in stats))


if __name__ == "__main__":
    write("parameter_path_fp32_sums.txt", wl.parameter_path(),
          "# Oracle count sums of the parameter path: 256 frames of 1920x1080,\n"
          "# C_k = 0.7885 exp(2 pi i k/256), window Re[-1.78,1.78] x Im[-1,1], cap 100,\n"
          "# FP32 formulation.  Written by tests/golden/make_workload_sums.py (oracle only).\n")
    write("general_path_deg3_fp32_sums.txt", wl.general_path(32, 3),
          "# Oracle count sums of the general-map path Z^3 + C: 32 frames of 1920x1080,\n"
          "# C_k = 0.6 exp(2 pi i k/32), window Re[-1.6,1.6] x Im[-0.9,0.9], cap 100,\n"
          "# FP32 general formulation.  Written by tests/golden/make_workload_sums.py\n"
          "# (oracle only).\n")
