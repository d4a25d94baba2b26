"""Small driver for counter runs of one projection kernel (used under rocprofv3).

    python3 profile_run.py --workload low_rank --precision bf16

Generates the workload's rows on the device (seeded, as the benchmark does), creates the
context and hashes the rows `--reps` times.  Prints one line per step."""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["connection_log", "low_rank", "heavy_tail"], default="low_rank")
    ap.add_argument("--precision", default="bf16")
    ap.add_argument("--rows", type=int, default=1_000_000)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--refine", type=int, default=1, help="0 raw signs, 1 FP64 pass (default), 2 count only")
    args = ap.parse_args()
    import torch
    from ace_inputs import c2_points, heavy_tail_points_torch, low_rank_points_torch, projection_matrix
    from paper_1706_06664_amd import ACE
    if args.workload == "connection_log":
        X, _ = c2_points()
        Xd = torch.from_numpy(X).cuda()
        W, K, L = projection_matrix(120, 15, 50, 1706066642), 15, 50
    elif args.workload == "low_rank":
        Xd, _ = low_rank_points_torch(args.rows, 1024, seed=3, device="cuda")
        W, K, L = projection_matrix(1024, 15, 64, 1706066643), 15, 64
    else:
        Xd, _ = heavy_tail_points_torch(args.rows, 4096, seed=4, device="cuda")
        W, K, L = projection_matrix(4096, 16, 100, 1706066644), 16, 100
    ace = ACE(W, K, L, precision=args.precision, refine=args.refine)
    for i in range(args.reps):
        ace.hash(Xd)
        torch.cuda.synchronize()
        print(f"step {i} done: {Xd.shape[0]} rows hashed ({args.workload}, {args.precision})", flush=True)
    ace.close()


if __name__ == "__main__":
    main()
