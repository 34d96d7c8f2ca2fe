"""Throughput of the fused kernel against the number of parallel envs, the
measurement the paper reports in its scaling experiment (Section 4.2: env
steps per second as the number of parallel environments grows, one game,
constant action).

    python -m paper_2510_01764_amd.env_sweep [--sizes 1024,4096,...] [--k 64]
        [--workloads mixed,single-const,draw-heavy]

Workloads: the mixed-ROM recipe (16 generated programs, random actions), a
single generated program with one action held throughout, and the draw-heavy
recipe (64 generated programs with 40% DXYN of up to 15 rows near the screen
edges, 20 instructions per frame, random actions).
Each point is graph replays of K steps with observations written every step
into one observation slot (so at small sizes a step's observations can stay
in the on-package cache; the benchmark's K-slot buffer does not allow that).
Times come from HIP events on the engine's stream.
"""
from __future__ import annotations

import argparse


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="1024,4096,16384,65536,262144,1048576")
    ap.add_argument("--k", type=int, default=64)
    ap.add_argument("--replays", type=int, default=6)
    ap.add_argument("--workloads", default="mixed,single-const")
    args = ap.parse_args()
    import torch
    from . import octax as X
    from . import workload as W
    dev = torch.device("cuda")
    K = args.k
    print(f"{'workload':13s} {'envs':>8s} {'ms per launch':>14s} {'M env steps/s':>14s}", flush=True)
    config = {"mixed": "c3", "single-const": "c2", "draw-heavy": "c5"}
    for label in args.workloads.split(","):
        for E in (int(x) for x in args.sizes.split(",")):
            spec = W.make_config(config[label], num_envs=E)
            act_np = spec.actions(0, K)
            if label == "single-const":
                act_np[:] = 0
            act = torch.from_numpy(act_np).to(dev)
            obs = torch.empty((1, E, 4, 64, 32), dtype=torch.uint8, device=dev)
            rew = torch.empty((K, E), dtype=torch.float32, device=dev)
            done = torch.empty((K, E), dtype=torch.uint8, device=dev)
            eng = X.Engine(spec, kernel="fused")
            g = eng.graph(act, obs, rew, done)
            g.launch()
            torch.cuda.synchronize()
            n = args.replays if E <= 65536 else max(2, args.replays // 2)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n):
                g.launch()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / n
            print(f"{label:13s} {E:8d} {ms:14.3f} {E * K / ms / 1e3:14.1f}", flush=True)
            g.close()
            eng.close()
            del obs, rew, done
            torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
