"""Record the autotuner's choices for named workloads on this GPU.

    python -m paper_2406_01939_amd.tune --out FILE [WORKLOAD ...]

Runs pk_autotune (block length, and for the learned policy the run walk's waves per
workgroup) on each workload and writes the results file FILE.  The library reads
autotune_mi355x.json beside libpicard.so when $PICARD_AUTOTUNE_CACHE is not set, so a
file recorded on MI355X and placed there spares later runs the timing (the learned
policy's search runs whole simulations: about a minute on the largest workload).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

DEFAULT = ["mlp_batch16_n500_k1e6_t1e7", "mlp_batch64_n100_k5e4_t2e5", "greedy_batch256_n50_k2e4",
           "greedy_n100_k1e5_t1e6", "greedy_n10_k100_t1e4", "greedy_n30_k1e6_t3e6"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("workloads", nargs="*", default=DEFAULT)
    args = ap.parse_args()
    os.environ["PICARD_AUTOTUNE_CACHE"] = os.path.abspath(args.out)
    import torch
    from paper_2406_01939_amd import api
    from paper_2406_01939_amd.instances import make_instance
    for name in args.workloads:
        inst = make_instance(name)
        policy = "mlp" if inst.params is not None else "greedy"
        prob = api.DeviceProblem.from_instance(inst)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B = api.pk_autotune(prob, policy)
        print(f"{name}: block_len {B} ({time.perf_counter() - t0:.1f} s)", flush=True)
        del prob
        torch.cuda.empty_cache()
    print(json.dumps(json.load(open(args.out)), indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
