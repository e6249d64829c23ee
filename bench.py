"""Benchmark: simulated orders/s of Picard policy simulation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one pk_picard_simulate call on one batch of synthetic orders resident in HBM:
setup (sort, partition, policy tables), every Picard pass to convergence, and the final
unpermute.  The headline workload is the largest single-GPU configuration: 16
trajectories of 1e7 orders each under the learned MLP softmax policy (N = 500
warehouses, K = 1e6 SKUs, R = 500 regions, quantities 1..4).  The one JSON line carries
its throughput, passes to converge, near-tie count, the serial GPU sweep on the same
instance (a prefix of every trajectory), the roofline of its dominant kernel (the learned
walk, FP32) measured with HIP events on the library's stream, and the CPU oracle's
throughput on the host (one core, and one trajectory per core on all of them).  Two
greedy legs follow, each with its own roofline and CPU baseline: 256 trajectories of
uneven horizon ("batch") and one trajectory of 1e6 orders ("single").  Other legs
(node capacity, the capacity-dependent policy, the policy-gradient loop, the partition
sweep, the gradient) run only when asked for.
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
DEFAULT_WORKLOAD = "mlp_batch16_n500_k1e6_t1e7"
BATCH_WORKLOAD = "greedy_batch256_n50_k2e4"
SINGLE_WORKLOAD = "greedy_n100_k1e5_t1e6"
LEARNED_WORKLOAD = "mlp_batch64_n100_k5e4_t2e5"
CAPACITY_WORKLOAD = "greedy_cap_n100_k1e5_t1e6"
REVENUE = 200  # per-unit price of the margin reward (revenue - cost) of the gradient legs
FP32_PEAK_TFLOPS = 157.3
CSRC = os.path.join(ROOT, "paper_2406_01939_amd", "csrc")
# HBM traffic of the dominant kernel per workload: the committed rocprofv3 counter summary
# and the sources whose text it was measured on
TRAFFIC = {
    SINGLE_WORKLOAD: ("k_walk_greedy_n100_k1e5_t1e6_traffic.md", ("walk_greedy.hip",)),
    BATCH_WORKLOAD: ("k_walk_greedy_batch256_n50_k2e4_traffic.md",
                     ("walk_greedy.hip", "walk_lane.hip")),
    DEFAULT_WORKLOAD: ("k_walk_mlp_batch16_n500_k1e6_t1e7_traffic.md",
                       ("mlp.hip", "mlp_device.h")),
}


def sources_sha256(names) -> str:
    h = hashlib.sha256()
    for n in names:
        h.update(open(os.path.join(CSRC, n), "rb").read())
    return h.hexdigest()


def _traffic(workload: str, block_len: int):
    """HBM bytes per walk launch from the committed rocprofv3 counter summary of this
    workload, if the walk's sources are unchanged since the counters were taken and they
    were taken at the same block length; else None.  The summary carries `key: value`
    lines, among them `source_sha256`, `block_len` and `bytes_per_launch`."""
    if workload not in TRAFFIC:
        return None
    fname, srcs = TRAFFIC[workload]
    try:
        rec = {}
        for line in open(os.path.join(ROOT, "profiles", fname)):
            k, sep, v = line.partition(":")
            if sep and k.strip() in ("source_sha256", "block_len", "bytes_per_launch"):
                rec[k.strip()] = v.strip().strip("`")
        if rec.get("source_sha256") != sources_sha256(srcs) or \
                int(rec.get("block_len", -1)) != block_len:
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


def host_info():
    """The host CPU's model name and the logical CPUs this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": avail, "os_cpu_count": os.cpu_count()}


def _prefix_instance(inst, b: int, m: int):
    """Trajectory b cut to its first m orders, as a one-trajectory instance whose SKUs are
    renumbered to those the prefix orders (their initial inventory rows recomputed from
    the workload's generator when it has no stored inventory).  SKUs never interact, so
    the rollout of the prefix is the same computation."""
    from paper_2406_01939_amd.instances import Instance
    lo = int(inst.traj_offsets[b])
    hi = min(lo + m, int(inst.traj_offsets[b + 1]))
    sku = inst.sku[lo:hi]
    uniq, inv = np.unique(sku, return_inverse=True)
    return Instance(N=inst.N, K=int(uniq.size), R=inst.R,
                    traj_offsets=np.array([0, hi - lo], dtype=np.int64),
                    sku=inv.astype(np.int32), region=inst.region[lo:hi].copy(),
                    qty=inst.qty[lo:hi].copy(), x0=inst.x0_rows(b, uniq)[None].copy(),
                    cost=inst.cost[b:b + 1].copy(), rng_seed=inst.rng_seed, params=inst.params,
                    hidden=inst.hidden, n_hidden_layers=inst.n_hidden_layers, name=inst.name)


def cpu_baseline(inst, budget_s: float = 8.0, threads: int = 1):
    """The oracle's serial rollout on the host, as it stands: whole trajectories of the
    workload (or, for the learned policy, prefixes of them sized so that the sample
    takes about budget_s), one trajectory per thread, repeated until budget_s has passed.
    threads = 1 is the one-core baseline; more threads run different trajectories at once
    (the oracle's C calls release the interpreter lock)."""
    import threading
    from oracle import oracle as O
    O.build(force=False)
    learned = inst.params is not None
    nt = inst.n_traj
    m = None
    if learned:  # size the prefix: time a short one first
        probe = _prefix_instance(inst, 0, 500)
        t0 = time.perf_counter()
        O.serial(probe, 0)
        per = (time.perf_counter() - t0) / probe.total_orders
        m = int(max(500, min(inst.horizon(0), 0.45 * budget_s / max(per, 1e-9))))
    jobs = [_prefix_instance(inst, b, m) if learned else inst.trajectory(b)
            for b in range(min(nt, threads))] if learned else None
    lock = threading.Lock()
    done = {"orders": 0, "runs": 0}
    t0 = time.perf_counter()

    def worker(k):
        i = k
        while time.perf_counter() - t0 < budget_s:
            if learned:
                sub = jobs[k % len(jobs)]
                O.serial(sub, 0)
                n = sub.total_orders
            else:
                b = i % nt
                O.serial(inst, b, greedy=True)
                n = inst.horizon(b)
                i += threads
            with lock:
                done["orders"] += n
                done["runs"] += 1

    ths = [threading.Thread(target=worker, args=(k,)) for k in range(threads)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    dt = time.perf_counter() - t0
    what = (f"prefixes of {m} orders of {min(nt, threads)} trajectories (FP64 learned policy)"
            if learned else "whole trajectories of the workload (greedy policy)")
    return {"value": done["orders"] / dt, "unit": "orders/s", "cores": threads, "kind": "oracle",
            "sample": f"serial oracle rollout, {done['orders']} orders in {done['runs']} "
                      f"rollouts: {what}, {dt:.2f} s, {threads} thread(s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--warmup-seconds", type=float, default=0.0)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--block-len", type=int, default=0)
    ap.add_argument("--no-serial", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="time budget of each CPU-oracle sample")
    ap.add_argument("--serial-prefix", type=int, default=-1, metavar="M",
                    help="time the serial sweep on the first M orders of each trajectory "
                         "(default: 3e5 for workloads whose full serial sweep runs for "
                         "minutes, else the whole workload)")
    ap.add_argument("--legs", default="batch,single,owmr",
                    help="comma-separated greedy legs after the headline: batch (256 "
                         "trajectories of uneven horizon), single (one trajectory of 1e6 "
                         "orders), learned64 (64 trajectories of 2e5 orders, learned), owmr "
                         "(the inventory-control workload); '' for none")
    ap.add_argument("--legs-after-s", type=float, default=470.0,
                    help="skip the remaining legs once the run has taken this long")
    ap.add_argument("--with-grad", action="store_true",
                    help="learned workloads: also time pk_policy_grad at the final actions")
    ap.add_argument("--pg-iters", type=int, default=0, metavar="K",
                    help="also run K policy-gradient iterations (Section 4.2) on the learned "
                         "workload with warm-started Picard, cold Picard and serial rollouts")
    ap.add_argument("--partition-sweep", nargs="?", const="greedy", choices=("greedy", "mlp"),
                    help="Section 4.1's partition contrast on the 3e6-order, 1e6-SKU, 30-"
                         "warehouse instance: product and uniform random partitions over 1e4 "
                         "processes and autotuned blocks, demand exponent 0 to -1")
    ap.add_argument("--capacity", action="store_true",
                    help="also run the node-capacity leg (Section 3's full state, time "
                         "blocks) and the capacity-dependent policy's ablation")
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

    def run(name, steps, warmup, warmup_s, block_len, serial, with_grad=False,
            serial_prefix=-1, cpu=False, cpu_s=8.0):
        """Time `steps` simulations of workload `name` (after `warmup` untimed ones) and,
        if asked, one serial GPU sweep of it (of a prefix of every trajectory when
        serial_prefix > 0) and the CPU oracle; the walk kernel's roofline from the timed
        steps."""
        t_gen = time.perf_counter()
        inst = make_instance(name)
        policy = "mlp" if inst.params is not None else "greedy"
        prob = api.DeviceProblem.from_instance(inst)
        torch.cuda.synchronize()
        _progress(f"{name}: {inst.total_orders} orders on the GPU "
                  f"({time.perf_counter() - t_gen:.1f} s to generate)")
        total = inst.total_orders
        B = block_len if block_len > 0 else api.pk_autotune(prob, policy)
        # warm-up: `warmup` steps, and at least `warmup_s` seconds of work (an idle GPU
        # runs at low clocks for a while)
        out = None
        t_w = time.perf_counter()
        k = 0
        while k < warmup or time.perf_counter() - t_w < warmup_s:
            out = api.pk_picard_simulate(prob, policy, block_len=B, out=out)
            torch.cuda.synchronize()
            k += 1
        acc = dict(walk_ms=0.0, walk_bytes=0, walk_flops=0, walk_launches=0, near_ties=0,
                   orders_walked=0, runs_walked=0, changed_total=0, scan_ms=0.0,
                   scan_bytes=0, scan_launches=0)
        passes = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = api.pk_picard_simulate(prob, policy, block_len=B, out=out, timing=True)
            st = out["stats"]
            for key_ in acc:
                acc[key_] += st.get(key_, 0)
            passes = out["passes"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        _progress(f"{name}: {steps} timed simulations, {dt:.3f} s")
        r = {"value": total * steps / dt, "ms_per_step": 1e3 * dt / steps, "inst": inst,
             "policy": policy, "B": B, "passes": passes, "total": total,
             "walk_waves": out["stats"]["walk_waves"]}
        per = max(steps, 1)
        r["work"] = {"orders_walked_per_step": acc["orders_walked"] / per,
                     "runs_walked_per_step": acc["runs_walked"] / per,
                     "changed_per_step": acc["changed_total"] / per,
                     "walk_ms_per_step": acc["walk_ms"] / per}
        avg_us = 1e3 * acc["walk_ms"] / max(acc["walk_launches"], 1)
        if policy == "greedy":
            achieved = (acc["walk_bytes"] / 1e9) / (acc["walk_ms"] / 1e3) if acc["walk_ms"] > 0 else 0.0
            r["roofline"] = {"kernel": "k_walk_greedy (first pass: k_walk_greedy_lane, then "
                                       "k_walk_greedy on the long runs)",
                             "bound": "hbm", "achieved": achieved,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                             "traffic": _traffic(name, B),
                             "bytes_per_launch": acc["walk_bytes"] / max(acc["walk_launches"], 1),
                             "avg_launch_us": avg_us, "launches": acc["walk_launches"]}
        else:
            achieved = (acc["walk_flops"] / 1e12) / (acc["walk_ms"] / 1e3) if acc["walk_ms"] > 0 else 0.0
            r["roofline"] = {"kernel": "k_walk_mlp", "bound": "mfma", "achieved": achieved,
                             "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": achieved / FP32_PEAK_TFLOPS, "traffic": _traffic(name, B),
                             "flops_per_launch": acc["walk_flops"] / max(acc["walk_launches"], 1),
                             "avg_launch_us": avg_us, "launches": acc["walk_launches"]}
            r["near_ties"] = {"evaluations_per_step": acc["near_ties"] / per,
                              "orders_walked_per_step": acc["orders_walked"] / per,
                              "rule": "top two perturbed scores within 1e-5 relative (FP32, "
                                      "counted by the walk over all passes)"}
        if acc["scan_launches"] > 0:
            sa = (acc["scan_bytes"] / 1e9) / (acc["scan_ms"] / 1e3) if acc["scan_ms"] > 0 else 0.0
            r["roofline_scan"] = {"kernel": "k_scan_entry", "bound": "hbm", "achieved": sa,
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": sa / HBM_PEAK_GBS,
                                  "bytes_per_launch": acc["scan_bytes"] / acc["scan_launches"],
                                  "avg_launch_us": 1e3 * acc["scan_ms"] / acc["scan_launches"],
                                  "launches": acc["scan_launches"]}
        if serial:
            if serial_prefix < 0:  # the learned workloads' serial sweeps run for minutes
                serial_prefix = 300_000 if (policy == "mlp" and total > 20_000_000) else 0
            sprob, it, stotal = prob, None, total
            if 0 < serial_prefix < int(np.diff(prob.traj_offsets).max()):
                sprob, it = prefix_problem(prob, serial_prefix)
                stotal = sprob.total
            else:
                api.pk_serial_simulate(sprob, policy)  # warm
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ser = api.pk_serial_simulate(sprob, policy, want_final=False)
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
            del ser, sprob
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
        del out, prob
        torch.cuda.empty_cache()
        if cpu:
            one = cpu_baseline(inst, cpu_s, 1)
            _progress(f"{name}: CPU oracle, one core: {one['value']:.4g} orders/s")
            r["cpu_baseline"] = one
            if inst.n_traj > 1:
                nth = max(1, min(16, HOST["nproc"], inst.n_traj))
                allc = cpu_baseline(inst, cpu_s, nth)
                _progress(f"{name}: CPU oracle, {nth} cores: {allc['value']:.4g} orders/s")
                r["cpu_baseline_all_cores"] = allc
        return r

    HOST = host_info()

    def owmr_leg(name="owmr_n4000_t3650000", steps=5, cpu_s=5.0):
        """The OWMR inventory workload (the appendix's base case shape): Picard with one
        process per retailer against the serial GPU sweep and the CPU oracle.  Its passes
        are an exclusive scan of the packed cache and a per-retailer walk; the roofline is
        the algorithmic bytes of whole passes (scan: 16 B per order; reset list: 8 B; walk:
        32 B read and 8 B written per order) over the simulation time."""
        from paper_2406_01939_amd import owmr_api as ow
        from paper_2406_01939_amd.instances import make_owmr_instance
        inst = make_owmr_instance(name)
        prob = ow.DeviceOwmr.from_instance(inst)
        out = ow.picard_simulate(prob)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = ow.picard_simulate(prob)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ser = ow.serial_simulate(prob)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ser = ow.serial_simulate(prob)
        torch.cuda.synchronize()
        sdt = time.perf_counter() - t1
        same = bool(torch.equal(ser["q"], out["q"]) and torch.equal(ser["reset"], out["reset"]))
        bytes_sim = out["passes"] * inst.T * (16 + 8 + 40)
        achieved = bytes_sim / dt / 1e9
        res = {"workload": name, "retailers": inst.N, "orders": inst.T, "value": inst.T / dt,
               "unit": "orders/s", "ms_per_step": 1e3 * dt, "steps": steps,
               "passes": out["passes"], "resets_R": ser["R"],
               "bound_2R_plus_2": 2 * ser["R"] + 2, "dtype": "int64",
               "roofline": {"kernel": "whole passes (scan + reset list + retailer walk)",
                            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
               "serial_gpu": {"value": inst.T / sdt, "unit": "orders/s", "seconds": sdt,
                              "identical_actions": same},
               "speedup_vs_serial_gpu": sdt / dt}
        _progress(f"{name}: Picard {1e3 * dt:.2f} ms ({out['passes']} passes, R = {ser['R']}), "
                  f"serial GPU {1e3 * sdt:.1f} ms")
        if cpu_s > 0:
            from oracle import owmr as O
            O.build(force=False)
            n, t2 = 0, time.perf_counter()
            while time.perf_counter() - t2 < cpu_s:
                O.serial(inst)
                n += 1
            cdt = (time.perf_counter() - t2) / n
            res["cpu_baseline"] = {"value": inst.T / cdt, "unit": "orders/s", "cores": 1,
                                   "kind": "oracle", "sample": f"{n} serial oracle rollouts of "
                                   f"the whole workload, {cdt * 1e3:.1f} ms each, one thread"}
            res["speedup_vs_cpu_oracle_one_core"] = cdt / dt
        del prob
        return res

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
        serial GPU sweep per gamma, on the 1e4-order capacity workload, in both readings of
        the shadow price (every node priced relative to the most capacity left; only nodes
        below a fifth of their capacity priced), and the bid-price policy (fixed dual
        prices of stock and capacity, uniform on 0..50 against costs 1..100)."""
        from paper_2406_01939_amd.instances import bid_prices, workload_capacity
        inst = make_instance(name)
        cap0 = workload_capacity(name)
        cap = torch.from_numpy(cap0).cuda()
        prob = api.DeviceProblem.from_instance(inst)
        low = max(1, int(cap0.max()) // 5)
        cases = [dict(gamma=g) for g in gammas]
        cases += [dict(gamma=g + (low,)) for g in gammas if g[0] > 0]
        cases += [dict(bids=bid_prices(inst.K, inst.N, 1))]
        rows = []
        for kw in cases:
            out = api.pk_picard_simulate_capacity(prob, cap, block_len=B, **kw)
            best = None
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = api.pk_picard_simulate_capacity(prob, cap, block_len=B, **kw)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ser = api.pk_serial_simulate_capacity(prob, cap, **kw)
            torch.cuda.synchronize()
            ds = time.perf_counter() - t0
            g = kw.get("gamma")
            if g is None:
                row = {"policy": "bid prices", "price": "fixed, uniform on 0..50"}
            else:
                row = {"policy": "greedy" if g[0] == 0 else "capacity-dependent",
                       "gamma": g[0] / g[1],
                       "price": "below %d of capacity left" % g[2] if len(g) > 2
                                else "relative to the most capacity left"}
            row.update({"passes": out["passes"], "picard_ms": 1e3 * best,
                        "serial_ms": 1e3 * ds, "speedup_vs_serial_gpu": ds / best,
                        "identical_actions": bool(torch.equal(out["actions"], ser["actions"]))})
            rows.append(row)
            _progress(f"capacity policy {kw if g is not None else 'bids'}: {out['passes']} "
                      f"passes, {1e3 * best:.2f} ms")
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

    def leg_summary(m, name):
        """The fields of a secondary leg's object in the result line."""
        out = {"workload": name, "value": m["value"], "unit": "orders/s",
               "ms_per_step": m["ms_per_step"], "orders": m["total"], "block_len": m["B"],
               "passes_max": int(m["passes"].max()), "passes_mean": float(m["passes"].mean()),
               "dtype": "int32" if m["policy"] == "greedy" else "f32",
               "roofline": m["roofline"], "work": m["work"]}
        for k in ("roofline_scan", "near_ties", "serial_gpu", "speedup_vs_serial_gpu",
                  "cpu_baseline", "cpu_baseline_all_cores", "policy_grad"):
            if k in m:
                out[k] = m[k]
        if "cpu_baseline" in m:
            out["speedup_vs_cpu_oracle_one_core"] = m["value"] / m["cpu_baseline"]["value"]
        return out

    cpu = not args.no_cpu
    t_start = time.perf_counter()
    m = run(args.workload, args.steps, args.warmup, args.warmup_seconds, args.block_len,
            not args.no_serial, args.with_grad, args.serial_prefix, cpu, args.cpu_seconds)
    inst, policy, passes = m["inst"], m["policy"], m["passes"]
    res = {"metric": METRIC, "value": m["value"], "unit": "orders/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int32" if policy == "greedy" else "f32", "data": "synthetic",
           "config": {"workload": args.workload, "policy": policy, "n_warehouses": inst.N,
                      "n_skus": inst.K, "n_regions": inst.R, "n_traj": inst.n_traj,
                      "orders": m["total"], "block_len": m["B"], "parallelism": "1 GPU",
                      "walk_waves": m["walk_waves"]},
           "passes_max": int(passes.max()), "passes_mean": float(passes.mean()),
           "roofline": m["roofline"], "host": HOST}
    for k in ("roofline_scan", "near_ties", "work", "serial_gpu", "speedup_vs_serial_gpu",
              "policy_grad", "cpu_baseline", "cpu_baseline_all_cores"):
        if k in m:
            res[k] = m[k]
    if "cpu_baseline" in m:
        res["speedup_vs_cpu_oracle_one_core"] = m["value"] / m["cpu_baseline"]["value"]
    del m, inst
    res["headline_seconds"] = time.perf_counter() - t_start
    legs = {}
    for leg in [x for x in args.legs.split(",") if x]:
        if leg == "owmr":
            if time.perf_counter() - t_start > args.legs_after_s:
                legs[leg] = {"skipped": "time"}
                continue
            legs[leg] = owmr_leg(cpu_s=min(args.cpu_seconds, 5.0) if cpu else 0.0)
            continue
        name = {"batch": BATCH_WORKLOAD, "single": SINGLE_WORKLOAD,
                "learned64": LEARNED_WORKLOAD}[leg]
        if name == args.workload:
            continue
        if time.perf_counter() - t_start > args.legs_after_s:
            legs[leg] = {"workload": name, "skipped": f"the run had taken more than "
                                                      f"{args.legs_after_s:.0f} s"}
            _progress(f"leg {leg} skipped: time")
            continue
        steps = 10 if leg != "learned64" else 2
        lm = run(name, steps, 2 if leg != "learned64" else 1, 0.5, 0, not args.no_serial,
                 cpu=cpu, cpu_s=min(args.cpu_seconds, 5.0))
        legs[leg] = leg_summary(lm, name)
        del lm
    if legs:
        res["legs"] = legs
    if args.capacity:
        res["capacity"] = capacity_leg(serial=not args.no_serial)
        res["capacity_gamma"] = gamma_ablation()
    if args.pg_iters > 0:
        res["policy_gradient_loop"] = pg_loop(LEARNED_WORKLOAD, args.pg_iters)
    if args.partition_sweep == "greedy":
        res["partition_sweep"] = partition_sweep()
    elif args.partition_sweep == "mlp":
        res["partition_sweep"] = partition_sweep(policy="mlp", betas=(0.0, -0.4, -0.8, -1.0),
                                                 reps=1)
    res["paper_context"] = ("paper (A100 40GB, JAX, 16-bit): 441x Picard speed-up over a "
                            "sequential GPU rollout at 3M orders / 1M products / 30 nodes, "
                            "MLP policy; not this workload")
    print(json.dumps(res))

if __name__ == "__main__":
    main()
