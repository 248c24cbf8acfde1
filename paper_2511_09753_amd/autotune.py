"""Command-line front of the tile autotuner (spai_autotune).

    python -m paper_2511_09753_amd.autotune [--workload lognormal|geo-batch] [--grid 96]
                                             [--count 256] [--warm 5] [--reps 2]

Builds the synthetic workload, creates the handle the benchmark would use, runs the
autotuner on it and prints the chosen tiles and their launch times as one JSON line.
"""
import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", choices=["lognormal", "geo-batch"], default="lognormal")
    ap.add_argument("--grid", type=int, default=96, help="lognormal: N of the N^3 grid")
    ap.add_argument("--count", type=int, default=256, help="geo-batch: number of matrices")
    ap.add_argument("--warm", type=int, default=5)
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args(argv)
    from . import spai as S
    from . import workloads as W
    S.load()
    if args.workload == "lognormal":
        A = W.lognormal3d(args.grid, W.seed_for(3))
        h = S.SPAI(A, "lomr", "global", 2.0, True, max_iter=max(args.warm, 30),
                   options=S.Options(precision="mixed"))
        what = f"lognormal {args.grid}^3, LOMR, global cap 2 nnz(A), mixed"
    else:
        mats = W.batch_geometric(args.count, W.seed_for(4))
        h = S.SPAI(None, "mr", "column", 4.0, False, max_iter=max(args.warm, 20),
                   options=S.Options(precision="mixed"), batch=mats)
        what = f"{args.count} geometric graphs, MR, column cap 4, mixed"
    tiles, ms = h.autotune(args.warm, args.reps)
    h.close()
    print(json.dumps({"workload": what, "tiles": tiles, "launch_ms": ms}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
