"""Writes the oracle's per-frame image digests of the full-size workloads.

Calls only the CPU oracle (oracle/): every digest in the files it writes is
of an image the oracle rendered, never of one the GPU library rendered.  The
digest of a frame is the SHA-256 of its whole count image as int32
little-endian bytes, row-major, row 0 on top -- the layout the library
writes -- so a GPU image equals the oracle's exactly when the digests agree.

Frames are rendered in parallel worker processes, each frame one plain
single-threaded oracle call, cheapest frames first.  Lines are appended to
<name>.partial as frames finish, so an interrupted run resumes where it
stopped; the final file is written, sorted by frame, once every frame is in.

    python tests/golden/make_workload_digests.py [--workers N] [uneven|paths ...]

Files:
  parameter_path_fp32_digests.txt  256 frames 1920x1080, cap 100, FP32
  general_path_deg3_fp32_digests.txt  32 frames of Z^3 + C, cap 100, FP32
  uneven_batch_fp32_digests.txt    the 503 FP32 frames of the 1024-frame
                                   uneven batch (sides 256..4096, caps
                                   100/500/2000), by their index in the batch

The uneven batch's float-float frames are not digested: the oracle's
float-float arithmetic runs near 6 M pixel-iterations per second on one core,
and those frames hold about 6 x 10^11 pixel-iterations (over a day of CPU).
"""
import argparse
import hashlib
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

COST = {"fp32": 1.0, "fp64": 1.0, "ff": 10.0}


def digest(image: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(image, dtype="<i4").tobytes()).hexdigest()


def frame_digest(job):
    k, f = job
    a = oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, f.mode,
                      getattr(f, "degree", 2))
    return k, digest(a), int(a.sum(dtype=np.int64))


def write(name, frames, header, workers, keys=None):
    """Digests of frames[k] for k in keys (default: all), one line each."""
    keys = list(range(len(frames))) if keys is None else list(keys)
    path = os.path.join(HERE, name)
    part = path + ".partial"
    done = {}
    if os.path.exists(part):
        for line in open(part):
            k, d, s = line.split()
            done[int(k)] = (d, int(s))
    # cheapest first: pixels x cap x dtype cost (an estimate; only the order)
    todo = sorted((k for k in keys if k not in done),
                  key=lambda k: frames[k].pixels * frames[k].max_iter * COST[frames[k].dtype])
    with open(part, "a") as out, Pool(workers) as pool:
        for k, d, s in pool.imap_unordered(frame_digest, [(k, frames[k]) for k in todo]):
            out.write("%d %s %d\n" % (k, d, s))
            out.flush()
            done[k] = (d, s)
            print("%s: %d/%d frames" % (name, len(done), len(keys)), flush=True)
    with open(path, "w") as out:
        out.write(header)
        out.write("# columns: frame sha256(int32 LE row-major image) count_sum\n")
        for k in keys:
            out.write("%d %s %d\n" % (k, done[k][0], done[k][1]))
    os.remove(part)
    print(path)


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    p.add_argument("which", nargs="*", default=["paths", "uneven"])
    a = p.parse_args()
    if "paths" in a.which:
        write("parameter_path_fp32_digests.txt", wl.parameter_path(),
              "# Oracle image digests of the parameter path: 256 frames of 1920x1080,\n"
              "# C_k = 0.7885 exp(2 pi i k/256), window Re[-1.78,1.78] x Im[-1,1], cap 100,\n"
              "# FP32 formulation.  Written by tests/golden/make_workload_digests.py\n"
              "# (oracle only).\n", a.workers)
        write("general_path_deg3_fp32_digests.txt", wl.general_path(32, 3),
              "# Oracle image digests of the general-map path Z^3 + C: 32 frames of\n"
              "# 1920x1080, C_k = 0.6 exp(2 pi i k/32), window Re[-1.6,1.6] x Im[-0.9,0.9],\n"
              "# cap 100, FP32 general formulation.  Written by\n"
              "# tests/golden/make_workload_digests.py (oracle only).\n", a.workers)
    if "uneven" in a.which:
        ub = wl.uneven_batch(0, n=1024)
        write("uneven_batch_fp32_digests.txt", ub,
              "# Oracle image digests of the FP32 frames of the uneven batch: 1024 square\n"
              "# frames, side U{256..4096}, C on the unit disk accepted by the 20-step\n"
              "# Mandelbrot test, cap from {100, 500, 2000}, FP32 or float-float, window\n"
              "# [-1.6,1.6]^2 (workloads.uneven_batch(0, 1024)); first column = the\n"
              "# frame's index in the batch.  Written by\n"
              "# tests/golden/make_workload_digests.py (oracle only).\n", a.workers,
              keys=[k for k, f in enumerate(ub) if f.dtype == "fp32"])


if __name__ == "__main__":
    main()
