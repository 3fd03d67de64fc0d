"""Workload driver for rocprofv3 runs (kernel trace, HBM counters).

Runs, in one process: a plain device-to-device copy of a known size (the
calibration for the HBM byte counters), then the 1024 x 1024, NQ = 16 FP64
workload for a few steps (short base-state run, since only the step kernel
is measured).  Usage under the profiler:
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
    t = P.Tpl(args.nx, args.ny, 60.0, 1.0, 0.7, periods=4, nq=args.nq, pre_steps=100,
              pert_modes=1)
    if args.precision:
        t.set_param("precision", args.precision)
    t.init(seed=0, perturbation=1e-4)
    t.step(args.steps)
    print(f"bytes_per_step={t.query('bytes_per_step'):.0f} copy_bytes={8 * n}", flush=True)
    t.close()


if __name__ == "__main__":
    main()
