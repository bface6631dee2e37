"""Train the surrogate networks for T_m (m = 2, 3, 4) on the GPU and save them.

    python -m paper_1606_02054_amd.train_surrogate [--n 10000000] [--epochs 4] [--m 2 3 4]
    python -m paper_1606_02054_amd.train_surrogate --label-only [--n 10000000] [--m 2 3 4]

Training problems: limits U[-6,6], correlations of random SPD matrices, dof
U[2,30]; labels: ln T_m by the lattice (8192 points x 8 shifts, mixed
precision).  Weights go to paper_1606_02054_amd/weights/surrogate_m{m}.npz and a
JSON line per model reports the held-out accuracy.  --label-only draws and
labels the training problems, reports the time of each, and trains nothing.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--m", type=int, nargs="+", default=[2, 3, 4])
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--out", default=None, help="output directory (default: the package's weights/)")
    ap.add_argument("--label-only", action="store_true", help="time the problem draw and the lattice labels only")
    args = ap.parse_args()
    from cfust_inputs import make_design
    from paper_1606_02054_amd import surrogate as S
    design = make_design(8192, 8, seed=args.seed)
    if args.label_only:
        import time
        import torch
        for m in args.m:
            t0 = time.perf_counter()
            b, L, idx, nu = S.draw_training_problems(m, args.n, seed=args.seed + m)
            t1 = time.perf_counter()
            lab = S.label_problems(m, b, L, idx, nu, design)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            print(json.dumps({"m": m, "n": args.n, "draw_s": t1 - t0, "label_s": t2 - t1,
                              "finite": int(torch.isfinite(lab).sum())}), flush=True)
        return
    out_dir = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
    os.makedirs(out_dir, exist_ok=True)
    for m in args.m:
        net, rep = S.train(m, args.n, design, epochs=args.epochs, batch=args.batch, lr=args.lr,
                           seed=args.seed + m, log=lambda s: print(s, flush=True))
        net.save(os.path.join(out_dir, f"surrogate_m{m}.npz"))
        print(json.dumps(dataclasses.asdict(rep)), flush=True)


if __name__ == "__main__":
    main()
