"""Benchmark: simulated orders/s of Picard policy simulation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one pk_picard_simulate call on one batch of synthetic orders resident in HBM:
setup (sort, partition, rank table), every Picard pass to convergence, and the final
unpermute.  Prints ONE JSON line with the throughput, the passes to converge, the serial
GPU sweep on the same instance (speed-up), the roofline of the dominant kernel measured
with HIP events on the library's stream, and the CPU oracle's throughput on the host.
For a greedy workload the line also carries a shorter run of the learned policy on its
own workload ("learned": 64 trajectories of 2e5 orders, MFMA roofline of its walk).
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "simulated orders/sec/GPU, Picard vs serial GPU sweep; iterations to converge"
HBM_PEAK_GBS = 8000.0
DEFAULT_WORKLOAD = "greedy_n100_k1e5_t1e6"
LEARNED_WORKLOAD = "mlp_batch64_n100_k5e4_t2e5"
CAPACITY_WORKLOAD = "greedy_cap_n100_k1e5_t1e6"
REVENUE = 200  # per-unit price of the margin reward (revenue - cost) of the gradient legs
FP32_PEAK_TFLOPS = 157.3
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_walk_greedy_n100_k1e5_t1e6_traffic.md")
WALK_SOURCE = os.path.join(ROOT, "paper_2406_01939_amd", "csrc", "walk_greedy.hip")


def _traffic(block_len: int):
    """HBM bytes per walk launch from the committed rocprofv3 counter summary, if the walk
    kernel's source is unchanged since the counters were taken and they were taken at the
    same block length; else None.  The summary carries `key: value` lines, among them
    `source_sha256`, `block_len` and `bytes_per_launch`."""
    try:
        rec = {}
        for line in open(TRAFFIC_FILE):
            k, sep, v = line.partition(":")
            if sep and k.strip() in ("source_sha256", "block_len", "bytes_per_launch"):
                rec[k.strip()] = v.strip().strip("`")
        h = hashlib.sha256(open(WALK_SOURCE, "rb").read()).hexdigest()
        if rec.get("source_sha256") != h or int(rec.get("block_len", -1)) != block_len:
            return None
        return float(rec["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def _progress(msg: str):
    """One line per finished stage, on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_calibration(nbytes: int, reps: int = 3):
    """A plain device-to-device copy of known size (the yardstick for the HBM byte
    counters: FETCH_SIZE and WRITE_SIZE of one copy dispatch against nbytes)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}))


def cpu_baseline(inst, budget_s: float = 8.0):
    """The oracle's serial rollout (single thread) over whole trajectories of the same
    workload, repeated until the time budget is used."""
    from oracle import oracle as O
    O.build(force=False)
    t0 = time.perf_counter()
    orders, reps = 0, 0
    while True:
        for b in range(inst.n_traj):
            O.serial(inst, b)
            orders += inst.horizon(b)
            if time.perf_counter() - t0 > budget_s:
                break
        reps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": orders / dt, "unit": "orders/s", "cores": 1, "kind": "oracle",
            "sample": f"serial oracle rollout, {orders} orders ({reps} pass(es) over the "
                      f"workload's trajectories), {dt:.2f} s, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--warmup-seconds", type=float, default=0.5)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--block-len", type=int, default=0)
    ap.add_argument("--no-serial", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serial-prefix", type=int, default=0, metavar="M",
                    help="time the serial sweep on the first M orders of each trajectory "
                         "(for workloads whose full serial sweep runs for minutes)")
    ap.add_argument("--with-grad", action="store_true",
                    help="learned workloads: also time pk_policy_grad at the final actions")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-policy leg (greedy workloads only)")
    ap.add_argument("--pg-iters", type=int, default=0, metavar="K",
                    help="also run K policy-gradient iterations (Section 4.2) on the learned "
                         "workload with warm-started Picard, cold Picard and serial rollouts")
    ap.add_argument("--partition-sweep", nargs="?", const="greedy", choices=("greedy", "mlp"),
                    help="Section 4.1's partition contrast on the 3e6-order, 1e6-SKU, 30-"
                         "warehouse instance: product and uniform random partitions over 1e4 "
                         "processes and autotuned blocks, demand exponent 0 to -1")
    ap.add_argument("--no-capacity", action="store_true",
                    help="skip the node-capacity leg (Section 3's full state, time blocks)")
    ap.add_argument("--capacity-only", action="store_true",
                    help="only run the node-capacity leg (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter yardstick)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the simulation "
              "is not sharded across GPUs.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return

    import torch
    from paper_2406_01939_amd import api
    from paper_2406_01939_amd.instances import make_instance

    def prefix_problem(prob, m):
        """The same problem restricted to the first m orders of every trajectory (the
        serial rollout of a prefix is the prefix of the serial rollout)."""
        offs = prob.traj_offsets
        idx = np.concatenate([np.arange(offs[b], min(offs[b] + m, offs[b + 1]))
                              for b in range(prob.n_traj)])
        new = np.zeros_like(offs)
        new[1:] = np.cumsum(np.minimum(np.diff(offs), m))
        it = torch.from_numpy(idx).cuda()
        sub = api.DeviceProblem(N=prob.N, K=prob.K, R=prob.R, traj_offsets=new,
                                sku=prob.sku[it].contiguous(), region=prob.region[it].contiguous(),
                                qty=prob.qty[it].contiguous(), init_inv=prob.init_inv,
                                cost=prob.cost, rng_seed=prob.rng_seed, params=prob.params,
                                n_hidden_layers=prob.n_hidden_layers, hidden=prob.hidden)
        return sub, it

    def run(name, steps, warmup, warmup_s, block_len, serial, with_grad=False, serial_prefix=0):
        """Time `steps` simulations of workload `name` (after the warm-up) and, if asked,
        one serial GPU sweep of it; the walk kernel's roofline from the same steps."""
        inst = make_instance(name)
        policy = "mlp" if inst.params is not None else "greedy"
        prob = api.DeviceProblem.from_instance(inst)
        torch.cuda.synchronize()
        _progress(f"{name}: {inst.total_orders} orders on the GPU")
        total = inst.total_orders
        B = block_len if block_len > 0 else api.pk_autotune(prob, policy)
        # warm-up: at least `warmup` steps and `warmup_s` seconds of work (an idle GPU
        # runs at low clocks for a while)
        out = None
        t_w = time.perf_counter()
        k = 0
        while k < warmup or time.perf_counter() - t_w < warmup_s:
            out = api.pk_picard_simulate(prob, policy, block_len=B, out=out)
            torch.cuda.synchronize()
            k += 1
        walk_ms = walk_bytes = walk_flops = 0.0
        walk_launches = 0
        passes = None
        t0 = time.perf_counter()
        for _ in range(steps):
            out = api.pk_picard_simulate(prob, policy, block_len=B, out=out, timing=True)
            st = out["stats"]
            walk_ms += st["walk_ms"]
            walk_bytes += st["walk_bytes"]
            walk_flops += st["walk_flops"]
            walk_launches += st["walk_launches"]
            passes = out["passes"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        _progress(f"{name}: {steps} timed simulations, {dt:.3f} s")
        r = {"value": total * steps / dt, "ms_per_step": 1e3 * dt / steps, "inst": inst,
             "policy": policy, "B": B, "passes": passes, "total": total}
        avg_us = 1e3 * walk_ms / max(walk_launches, 1)
        if policy == "greedy":
            achieved = (walk_bytes / 1e9) / (walk_ms / 1e3) if walk_ms > 0 else 0.0
            r["roofline"] = {"kernel": "k_walk_greedy", "bound": "hbm", "achieved": achieved,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                             "traffic": _traffic(B) if name == DEFAULT_WORKLOAD else None,
                             "bytes_per_launch": walk_bytes / max(walk_launches, 1),
                             "avg_launch_us": avg_us, "launches": walk_launches}
        else:
            achieved = (walk_flops / 1e12) / (walk_ms / 1e3) if walk_ms > 0 else 0.0
            r["roofline"] = {"kernel": "k_walk_mlp", "bound": "mfma", "achieved": achieved,
                             "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                             "flops_per_launch": walk_flops / max(walk_launches, 1),
                             "avg_launch_us": avg_us, "launches": walk_launches}
        if serial:
            sprob, it, stotal = prob, None, total
            if 0 < serial_prefix < int(np.diff(prob.traj_offsets).max()):
                sprob, it = prefix_problem(prob, serial_prefix)
                stotal = sprob.total
            else:
                api.pk_serial_simulate(sprob, policy)  # warm
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ser = api.pk_serial_simulate(sprob, policy)
            torch.cuda.synchronize()
            sdt = time.perf_counter() - t1
            _progress(f"{name}: serial sweep of {stotal} orders {sdt:.3f} s")
            want = out["actions"] if it is None else out["actions"][it]
            r["serial_gpu"] = {"value": stotal / sdt, "unit": "orders/s", "seconds": sdt,
                               "orders": stotal,
                               "identical_actions": bool(torch.equal(ser["actions"], want))}
            if it is not None:
                r["serial_gpu"]["prefix_per_trajectory"] = serial_prefix
            r["speedup_vs_serial_gpu"] = r["value"] / (stotal / sdt)
        if with_grad and policy == "mlp":
            adv = api.pk_reinforce_advantages(prob, out["actions"], out["shipped"],
                                              REVENUE)["advantages"]
            _progress(f"{name}: policy gradient")
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            g = api.pk_policy_grad(prob, out["actions"], adv)
            torch.cuda.synchronize()
            gdt = time.perf_counter() - t2
            _progress(f"{name}: policy gradient {gdt:.3f} s")
            r["policy_grad"] = {"seconds": gdt, "orders_per_s": total / gdt,
                                "objective": g["objective"]}
        return r

    def partition_sweep(M=10_000, betas=(0.0, -0.2, -0.4, -0.6, -0.8, -1.0), reps=3,
                        policy="greedy"):
        """Picard time (best of `reps`, after one warm-up call), passes and speed-up over
        the serial GPU sweep for three partitions of the same instance, per demand
        exponent beta (SKU k drawn with probability proportional to (k+1)^beta)."""
        name = "greedy_n30_k1e6_t3e6"
        rows = []

        def timed(fn):
            best, out = float("inf"), fn()
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = fn()
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            return best, out

        for beta in betas:
            inst = make_instance(name, zipf=-beta)
            if policy == "mlp":  # two hidden layers of 64, seeded (no trained weights)
                from paper_2406_01939_amd.instances import make_params
                inst = dataclasses.replace(inst, params=make_params(inst.R, 6999))
            prob = api.DeviceProblem.from_instance(inst)
            rng = np.random.default_rng(6)
            row = {"beta": beta, "top_sku_orders": int(np.bincount(inst.sku).max())}
            sdt, ser = timed(lambda: api.pk_serial_simulate(prob, policy, want_final=False))
            row["serial_s"] = sdt
            _progress(f"partition sweep beta={beta}: serial sweep {sdt:.3f} s")
            parts = {"product": rng.integers(0, M, inst.K)[inst.sku],
                     "uniform": rng.integers(0, M, inst.total_orders)}
            for label, w in parts.items():
                part = torch.from_numpy(w.astype(np.int32)).cuda()
                dt, out = timed(lambda: api.pk_picard_simulate(prob, policy, partition=part,
                                                               want_final=False))
                _progress(f"partition sweep beta={beta}: {label} {dt:.4f} s")
                row[label] = {"seconds": dt, "passes": int(out["passes"].max()),
                              "speedup_vs_serial_gpu": sdt / dt,
                              "identical_actions": bool(torch.equal(out["actions"],
                                                                    ser["actions"]))}
            # the learned policy takes the library's default block (the autotuner would run
            # a dozen multi-second simulations here)
            B = api.pk_autotune(prob, policy) if policy == "greedy" else 256
            dt, out = timed(lambda: api.pk_picard_simulate(prob, policy, block_len=B,
                                                           want_final=False))
            row["blocks"] = {"block_len": B, "seconds": dt, "passes": int(out["passes"].max()),
                             "speedup_vs_serial_gpu": sdt / dt,
                             "identical_actions": bool(torch.equal(out["actions"],
                                                                   ser["actions"]))}
            _progress(f"partition sweep beta={beta}: serial {sdt:.3f} s; " + "; ".join(
                f"{k} {row[k]['seconds'] * 1e3:.1f} ms ({row[k]['passes']} passes, "
                f"{row[k]['speedup_vs_serial_gpu']:.0f}x)" for k in ("product", "uniform", "blocks")))
            rows.append(row)
            del prob
        return {"workload": name, "policy": policy, "processes": M,
                "timing": f"best of {reps} after a warm-up", "rows": rows}

    def capacity_leg(name=CAPACITY_WORKLOAD, blocks=(32, 48, 64, 96, 128, 255), reps=3,
                     serial=True):
        """Picard with node capacity (time-block processes) against the serial GPU sweep
        with capacity, on the same instance; best of `reps` calls per block length after a
        warm-up call."""
        from paper_2406_01939_amd.instances import workload_capacity
        inst = make_instance(name)
        cap = torch.from_numpy(workload_capacity(name)).cuda()
        prob = api.DeviceProblem.from_instance(inst)
        total = inst.total_orders
        rows = []
        ref = None
        for B in blocks:
            out = api.pk_picard_simulate_capacity(prob, cap, block_len=B)
            best = None
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = api.pk_picard_simulate_capacity(prob, cap, block_len=B)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            if ref is None:
                ref = out["actions"].clone()
            same = bool(torch.equal(out["actions"], ref))
            rows.append({"block_len": B, "seconds": best, "orders_per_s": total / best,
                         "passes": out["passes"], "identical_across_blocks": same})
            _progress(f"capacity {name} B={B}: {1e3 * best:.2f} ms, {out['passes']} passes")
        top = min(rows, key=lambda r: r["seconds"])
        res = {"workload": name, "orders": total, "value": top["orders_per_s"],
               "unit": "orders/s", "block_len": top["block_len"], "passes": top["passes"],
               "ms": 1e3 * top["seconds"], "blocks": rows,
               "capacity_per_node": int(cap[0].item()),
               "nodes_out_of_capacity": None}
        if serial:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ser = api.pk_serial_simulate_capacity(prob, cap)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res["serial_gpu"] = {"value": total / dt, "unit": "orders/s", "seconds": dt,
                                 "identical_actions": bool(torch.equal(ser["actions"], ref))}
            res["speedup_vs_serial_gpu"] = dt / top["seconds"]
            res["nodes_out_of_capacity"] = int((ser["final_cap"] == 0).sum().item())
            _progress(f"capacity serial sweep: {dt:.3f} s")
        return res

    def gamma_ablation(name="greedy_cap_n10_k100_t1e4", B=100,
                       gammas=((0, 1), (1, 2), (1, 1), (2, 1)), reps=3):
        """The appendix's capacity-dependent policy ablation: passes and speed-up over the
        serial GPU sweep per gamma, on the 1e4-order capacity workload."""
        from paper_2406_01939_amd.instances import workload_capacity
        inst = make_instance(name)
        cap = torch.from_numpy(workload_capacity(name)).cuda()
        prob = api.DeviceProblem.from_instance(inst)
        rows = []
        for g in gammas:
            out = api.pk_picard_simulate_capacity(prob, cap, block_len=B, gamma=g)
            best = None
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = api.pk_picard_simulate_capacity(prob, cap, block_len=B, gamma=g)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ser = api.pk_serial_simulate_capacity(prob, cap, gamma=g)
            torch.cuda.synchronize()
            ds = time.perf_counter() - t0
            rows.append({"gamma": g[0] / g[1], "passes": out["passes"], "picard_ms": 1e3 * best,
                         "serial_ms": 1e3 * ds, "speedup_vs_serial_gpu": ds / best,
                         "identical_actions": bool(torch.equal(out["actions"], ser["actions"]))})
            _progress(f"gamma {g[0]}/{g[1]}: {out['passes']} passes, {1e3 * best:.2f} ms")
        return {"workload": name, "block_len": B, "rows": rows}

    if args.capacity_only:
        print(json.dumps({"capacity": capacity_leg(serial=not args.no_serial,
                                                   reps=max(1, args.steps)),
                          "capacity_gamma": gamma_ablation()}))
        return

    def pg_loop(name, iters):
        """End-to-end training (rollout, advantages, gradient, Adam step) for `iters`
        iterations from the same initial parameters, once per rollout mode."""
        from paper_2406_01939_amd.train import PolicyGradient
        inst = make_instance(name)
        prob = api.DeviceProblem.from_instance(inst)
        p0 = prob.params.clone()
        B = api.pk_autotune(prob, "mlp")
        res = {"workload": name, "iterations": iters, "lr": 3e-3, "revenue": REVENUE,
               "block_len": B}
        finals = {}
        for label, mode, warm in (("picard_warm", "picard", True),
                                  ("picard_cold", "picard", False), ("serial", "serial", False)):
            prob.params.copy_(p0)
            pg = PolicyGradient(prob, lr=3e-3, revenue=REVENUE, rollout=mode, warm_start=warm,
                                block_len=B)
            hist = pg.run(iters, callback=lambda h, lab=label: _progress(
                f"pg {lab} it {h.it}: passes {h.passes_max} rollout {h.rollout_ms:.0f} ms "
                f"grad+adam {h.grad_ms:.0f} ms mean return {h.mean_return:.4g}"))
            finals[label] = prob.params.clone()
            res[label] = {"passes": [h.passes_max for h in hist],
                          "rollout_s": sum(h.rollout_ms for h in hist) / 1e3,
                          "total_s": sum(h.rollout_ms + h.grad_ms for h in hist) / 1e3,
                          "mean_return": [h.mean_return for h in hist]}
        res["identical_parameters"] = all(torch.equal(finals["serial"], finals[k])
                                          for k in ("picard_warm", "picard_cold"))
        for k in ("picard_warm", "picard_cold"):
            res[f"rollout_speedup_{k}_vs_serial"] = res["serial"]["rollout_s"] / res[k]["rollout_s"]
            res[f"loop_speedup_{k}_vs_serial"] = res["serial"]["total_s"] / res[k]["total_s"]
        prob.params.copy_(p0)
        return res

    m = run(args.workload, args.steps, args.warmup, args.warmup_seconds, args.block_len,
            not args.no_serial, args.with_grad, args.serial_prefix)
    inst, policy, passes = m["inst"], m["policy"], m["passes"]
    res = {"metric": METRIC, "value": m["value"], "unit": "orders/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int32" if policy == "greedy" else "f32", "data": "synthetic",
           "config": {"workload": args.workload, "policy": policy, "n_warehouses": inst.N,
                      "n_skus": inst.K, "n_regions": inst.R, "n_traj": inst.n_traj,
                      "orders": m["total"], "block_len": m["B"], "parallelism": "1 GPU"},
           "passes_max": int(passes.max()), "passes_mean": float(passes.mean()),
           "roofline": m["roofline"]}
    for k in ("serial_gpu", "speedup_vs_serial_gpu", "policy_grad"):
        if k in m:
            res[k] = m[k]
    if not args.no_learned and policy == "greedy":
        # the learned policy on its own workload (64 trajectories), a shorter run
        lm = run(LEARNED_WORKLOAD, 2, 1, 0.5, 0, True)
        res["learned"] = {"workload": LEARNED_WORKLOAD, "value": lm["value"], "unit": "orders/s",
                          "ms_per_step": lm["ms_per_step"], "orders": lm["total"],
                          "block_len": lm["B"], "passes_max": int(lm["passes"].max()),
                          "passes_mean": float(lm["passes"].mean()), "dtype": "f32",
                          "roofline": lm["roofline"], "serial_gpu": lm["serial_gpu"],
                          "speedup_vs_serial_gpu": lm["speedup_vs_serial_gpu"]}
    if not args.no_capacity and policy == "greedy":
        res["capacity"] = capacity_leg(serial=not args.no_serial)
        res["capacity_gamma"] = gamma_ablation()
    if args.pg_iters > 0:
        res["policy_gradient_loop"] = pg_loop(LEARNED_WORKLOAD, args.pg_iters)
    if args.partition_sweep == "greedy":
        res["partition_sweep"] = partition_sweep()
    elif args.partition_sweep == "mlp":
        res["partition_sweep"] = partition_sweep(policy="mlp", betas=(0.0, -0.4, -0.8, -1.0),
                                                 reps=1)
    if not args.no_cpu and inst.x0 is not None:
        res["cpu_baseline"] = cpu_baseline(inst)
    res["paper_context"] = ("paper (A100 40GB, JAX, 16-bit): 441x Picard speed-up over a "
                            "sequential GPU rollout at 3M orders / 1M products / 30 nodes, "
                            "MLP policy; not this workload")
    print(json.dumps(res))


if __name__ == "__main__":
    main()
