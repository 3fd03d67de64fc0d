"""Workload driver for rocprofv3 runs (kernel trace, HBM counters).

Runs, in one process: a plain device-to-device copy of a known size (the
calibration for the HBM byte counters), then the 1024 x 1024, NQ = 16 FP64
workload for a few steps (short base-state run, since only the step kernel
is measured; other sizes, one population array and a fixed tile group by
option), or with --batch N the first N instances of the seeded batched
sweep (FP32, NQ = 6) stepped together with a fixed launch shape (one
Q-slice, groups of 4 tiles: the autotuner's usual pick; plain launches, no
graph, so that every dispatch is the measured step).  Usage
under the profiler:
  rocprofv3 --pmc FETCH_SIZE -d <dir> -o run -- python paper_2201_10132_amd/profile_run.py
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--copy-gib", type=float, default=4.0)
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--ny", type=int, default=1024)
    ap.add_argument("--nq", type=int, default=16)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--batch", type=int, default=0, help="instances of the batched sweep")
    ap.add_argument("--qsplit", type=int, default=1, help="Q-slices of the batched step")
    ap.add_argument("--group", type=int, default=4, help="tiles per workgroup of the batched step")
    ap.add_argument("--batch-nq", type=int, default=6, help="Q points per axis of the batched sweep")
    ap.add_argument("--periods", type=int, default=4)
    ap.add_argument("--inplace", type=int, default=0, help="1: one population array")
    ap.add_argument("--spring-shift", type=int, default=0, help="1: the shifted spring term")
    ap.add_argument("--gradients", type=int, default=0, help="1: same-step gradients")
    ap.add_argument("--group-x", type=int, default=0,
                    help="tile group of the single-lattice step (0: the autotuner's choice)")
    ap.add_argument("--group-y", type=int, default=1)
    ap.add_argument("--group-sync", type=int, default=1)
    args = ap.parse_args()
    import torch
    import paper_2201_10132_amd as P

    n = int(args.copy_gib * 2 ** 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)  # calibration dispatch: reads and writes copy_gib GiB
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()
    if args.batch:
        from paper_2201_10132_amd import inputs

        b = P.Batch(inputs.c4_instances(args.batch), precision=1, nq=args.batch_nq, pre_steps=100,
                    autotune=0, qsplit=args.qsplit, group=args.group, graph_steps=0)
        b.init()
        b.step(args.steps)
        print(f"bytes_per_step={b.query('bytes_per_step'):.0f} items={b.query('items'):.0f} "
              f"copy_bytes={8 * n}", flush=True)
        b.close()
        return
    t = P.Tpl(args.nx, args.ny, 60.0, 1.0, 0.7, periods=args.periods, nq=args.nq, pre_steps=100,
              pert_modes=1)
    if args.precision:
        t.set_param("precision", args.precision)
    if args.inplace:
        t.set_param("inplace", 1)
    if args.spring_shift:
        t.set_param("spring_shift", 1)
    if args.gradients:
        t.set_param("gradients", 1)
    if args.group_x:
        t.set_param("autotune", 0)
        t.set_param("group_y", 1)
        t.set_param("group_x", args.group_x)
        t.set_param("group_y", args.group_y)
        t.set_param("group_sync", args.group_sync)
    t.init(seed=0, perturbation=1e-4)
    t.step(args.steps)
    print(f"bytes_per_step={t.query('bytes_per_step'):.0f} copy_bytes={8 * n}", flush=True)
    t.close()


if __name__ == "__main__":
    main()
