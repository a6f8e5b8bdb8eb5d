"""Benchmark of the batched limit-order-book matcher on one MI355X.

Default workload (one "step" = one pass of the matching path over one batch):
4096 books of capacity 100 per side, each fed 100 initial orders and then 10,000
flow messages of the synthetic LOBSTER-like mix; every step resets the books,
processes all 41.4M messages (messages already in HBM) and writes the final
top-10 L2 of every book.  `value` counts the 40.96M flow messages per step (the
initial orders are processed in the timed step too).  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--workload c1|c0] [--no-cpu-baseline]
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2308_13289_amd import lob  # noqa: E402
from paper_2308_13289_amd import workload as W  # noqa: E402

METRIC = "bit-exact LOB messages/sec on 1 MI355X, ragged vs plain batch; step p99 ms"
HBM_PEAK_GBS = 8000.0
LEVELS = 10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


KERNEL_SOURCES = ("paper_2308_13289_amd/csrc/lob_kernels.hip", "paper_2308_13289_amd/csrc/lob_small.hip",
                  "paper_2308_13289_amd/csrc/lob_device.h", "paper_2308_13289_amd/csrc/lob_internal.h",
                  "paper_2308_13289_amd/csrc/lob_lds_engine.h",
                  "paper_2308_13289_amd/build.py")


def _code_only(text):
    """C/C++ source without comments or blank lines (a comment edit does not change
    the kernel a profile was taken on)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            text = f.read()
        h.update((text if p.endswith(".py") else _code_only(text)).encode())
    return h.hexdigest()[:16]


def kernel_name(ctx, w):
    """The matching kernel a plain launch over these books runs (same rule as liblob)."""
    plan = ctx.get_plan()
    if plan.registers and int(w.caps.max()) <= 128:
        return "k_process_small"
    return "k_process<true>" if int(w.caps.max()) > plan.lds_slots else "k_process<false>"


def load_profile(name, khash):
    """The rocprofv3 counter figures of a kernel (profiles/<name>.traffic.json),
    valid only for the kernel source they were taken on; {} otherwise."""
    p = os.path.join(ROOT, "profiles", f"{name}.traffic.json")
    if not os.path.exists(p):
        return {}
    with open(p) as f:
        d = json.load(f)
    return d if d.get("kernel_hash") == khash else {}


def load_traffic(name, khash):
    """HBM bytes per launch measured by rocprofv3 counters."""
    return load_profile(name, khash).get("hbm_bytes_per_launch")


def cpu_baseline(w, n_sample_books, n_single_books=512, gpu_l2=None):
    """The oracle (plain sequential C engine, gcc -O3), as it stands, on a bounded
    sample of the same workload: the books spread over this process's host cores (at
    most 16, the CPU share of one GPU), and a smaller sample on one thread.  gpu_l2:
    the GPU's final L2 of the same books, compared with the oracle's of the timed run
    (after the timing)."""
    from oracle import oracle as O

    def timed(n, threads):
        # rates count flow messages, like the GPU figure; the initial orders are
        # processed too
        n = min(n, w.n_books)
        offs = w.offs[:n + 1]
        t0 = time.perf_counter()
        o = O.run(w.caps[:n], w.msgs[:offs[-1]], offs, l2_mode=O.L2_FINAL, levels=LEVELS, threads=threads)
        return n, int(offs[-1]), int(w.n_flow[:n].sum()), time.perf_counter() - t0, o

    cores = host_cores()
    n, m, f, dt, o = timed(n_sample_books, cores)
    n1, m1, f1, dt1, _ = timed(n_single_books, 1)
    agrees = None
    if gpu_l2 is not None:
        agrees = {"books": n, "final_l2_equal": bool(np.array_equal(gpu_l2[:n], o["l2"]))}
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"value": float(f / dt), "unit": "msgs/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} of {w.n_books} books ({f} flow messages, {m} with the initial orders), "
                      f"final L2, {dt:.2f} s wall on {cores} threads",
            "single_thread": {"value": float(f1 / dt1), "unit": "msgs/s", "cores": 1,
                              "sample": f"first {n1} books ({f1} flow messages, {m1} with the initial orders), "
                                        f"{dt1:.2f} s wall on 1 thread"},
            "host": {"os_cpu_count": os.cpu_count(), "affinity_cpus": affinity,
                     "threads_used": cores, "note": "threads capped at 16, the CPU share of one GPU"},
            "gpu_agrees": agrees}


def bench_uniform(args, w, desc):
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    lens = np.diff(w.offs)
    ctx = lob.Context(w.caps, l2_levels=LEVELS, trade_log_records=w.caps.astype(np.int64) + 2 * lens)
    if args.plan:
        ctx.set_plan(**json.loads(args.plan))
    t0 = time.perf_counter()
    d_msgs = torch.from_numpy(w.msgs).to(dev)
    d_offs = torch.from_numpy(w.offs).to(dev)
    torch.cuda.synchronize()
    h2d_s = time.perf_counter() - t0
    l2 = torch.zeros((w.n_books, 2, LEVELS, 2), dtype=torch.int32, device=dev)

    def step(ev=None):
        ctx.reset(stream=stream)
        if ev:
            ev[0].record(stream)
        ctx.process(d_msgs, d_offs, l2_mode=lob.L2_FINAL, l2_out=l2, stream=stream)
        if ev:
            ev[1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    st = ctx.read_status()
    n_msgs = w.n_msgs                 # every message the launch processes
    n_flow = int(w.n_flow.sum())      # the workload's flow messages (without the initial orders)
    n_trades = int(st["n_trades"].sum())
    live = int(st["n_ask"].sum() + st["n_bid"].sum())
    # algorithmic HBM bytes of one process launch: messages in, trades out, final L2
    # out, book headers in/out, resting orders out (books start empty after reset)
    alg_bytes = n_msgs * 32 + n_trades * 24 + w.n_books * 4 * LEVELS * 4 + w.n_books * 2 * 144 + live * 24
    kavg = float(np.mean(kern_ms)) / 1e3
    achieved = alg_bytes / kavg / 1e9
    khash = kernel_source_hash()
    wl = "c1" if args.workload in ("all", "c1") else args.workload
    traffic = load_traffic(f"{kernel_name(ctx, w)}_{wl}", khash)
    # the bound is instruction issue along each book's serial chain: issue counters
    # of the same kernel beside the HBM fraction, and the waves per SIMD of this launch
    issue = dict(load_profile(f"{kernel_name(ctx, w)}_{wl}", khash).get("issue", {}))
    issue.pop("commands", None)
    issue["waves_per_simd"] = w.n_books / (4 * torch.cuda.get_device_properties(0).multi_processor_count)
    res = {
        "metric": METRIC, "value": n_flow * args.steps / wall, "unit": "msgs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "books": w.n_books, "capacity": int(w.caps.max()),
                   "messages_per_step": n_flow, "initial_orders_per_step": n_msgs - n_flow,
                   "value_counts": "flow messages only; the initial orders of each step are processed too",
                   "trades_per_step": n_trades, "l2": "final top-10",
                   "plan": ctx.get_plan().as_dict()},
        "verified": None,  # filled in from the cpu_baseline leg
        "kernel_ms": {"mean": float(np.mean(kern_ms)), "min": float(np.min(kern_ms)),
                      "max": float(np.max(kern_ms))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes, "kernel": kernel_name(ctx, w),
                     "kernel_hash": khash, "issue": issue},
        "h2d_s": h2d_s,
        "pcie_inclusive_msgs_per_s": n_flow / (h2d_s + wall / args.steps),
        "_l2": l2.cpu().numpy(),  # the final L2, for the cpu_baseline leg; not printed
    }
    ctx.close()
    return res


def bench_ragged(args, n_books=10_000, reps=3):
    """Ragged batch: 10,000 books, capacity in {50,100,500,1000}, flow length
    log-uniform in [1e2, 1e5]; one autotuned lob_process_ragged call against the
    plain kernel run once per capacity bucket (lob_process_messages, each launch
    sized for its bucket's capacity, one launch after the other)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    t0 = time.perf_counter()
    w = W.ragged(n_books=n_books, threads=host_cores())
    log(f"ragged workload: {w.n_msgs} messages generated in {time.perf_counter() - t0:.1f}s")
    lens = np.diff(w.offs)
    ctx = lob.Context(w.caps, l2_levels=LEVELS, trade_log_records=w.caps.astype(np.int64) + 2 * lens)
    d_msgs = torch.from_numpy(w.msgs).to(dev)
    l2 = torch.zeros((n_books, 2, LEVELS, 2), dtype=torch.int32, device=dev)

    def timed(fn):
        ts = []
        for _ in range(reps):
            ctx.reset(stream=stream)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts)), ts

    # plain uniform-batch kernel, one launch per capacity bucket
    buckets = []
    for c in sorted(set(int(x) for x in w.caps)):
        ids = np.nonzero(w.caps == c)[0].astype(np.int32)
        idx = np.concatenate([np.arange(w.offs[i], w.offs[i + 1]) for i in ids])
        offs = np.concatenate([[0], np.cumsum(lens[ids])]).astype(np.int64)
        buckets.append((c, torch.from_numpy(ids).to(dev), d_msgs[torch.from_numpy(idx).to(dev)],
                        torch.from_numpy(offs).to(dev),
                        torch.zeros((len(ids), 2, LEVELS, 2), dtype=torch.int32, device=dev)))

    def plain():
        # each bucket's launch is sized for its own capacity (plan max_capacity): cap
        # 50 and 100 run the register kernel without a tail, cap 500 and 1000 with one
        for c, d_ids, d_bm, d_bo, bl2 in buckets:
            ctx.set_plan(lds_slots=c, books_per_block=4, max_capacity=c)
            ctx.process(d_bm, d_bo, book_ids=d_ids, l2_mode=lob.L2_FINAL, l2_out=bl2, stream=stream)

    plain_ms, plain_all = timed(plain)
    plain_l2 = [bl2.clone() for *_, bl2 in buckets]

    # ablation: the same per-bucket launches with every stream padded by type-0
    # messages to its bucket's longest one, the batching a vmapped engine needs
    # (padding is skipped by the kernel but still read and walked)
    padded, n_padded = [], 0
    for c, d_ids, d_bm, d_bo, bl2 in buckets:
        blens = d_bo[1:] - d_bo[:-1]
        L = int(blens.max())
        n = int(d_ids.shape[0])
        pad = torch.zeros((n * L, 8), dtype=torch.int32, device=dev)
        local = torch.arange(int(d_bo[-1]), device=dev) - torch.repeat_interleave(d_bo[:-1], blens)
        pad[torch.repeat_interleave(torch.arange(n, device=dev) * L, blens) + local] = d_bm
        padded.append((c, d_ids, pad, torch.arange(n + 1, dtype=torch.int64, device=dev) * L, bl2))
        n_padded += n * L
        del local

    def plain_padded():
        for c, d_ids, pad, po, bl2 in padded:
            ctx.set_plan(lds_slots=c, books_per_block=4, max_capacity=c)
            ctx.process(pad, po, book_ids=d_ids, l2_mode=lob.L2_FINAL, l2_out=bl2, stream=stream)

    padded_ms, _ = timed(plain_padded)
    torch.cuda.synchronize()
    padded_same = all(torch.equal(a, b[-1]) for a, b in zip(plain_l2, padded))
    plain_host = [(b[1].cpu().numpy(), p.cpu().numpy()) for b, p in zip(buckets, plain_l2)]
    del padded, plain_l2
    torch.cuda.empty_cache()
    ctx.set_plan(max_capacity=0)
    t1 = time.perf_counter()
    plan, tuned_ms = ctx.autotune_ragged(d_msgs, w.offs, max_trials=args.tune_trials, stream=stream)
    tune_s = time.perf_counter() - t1
    ctx.set_plan(**plan)

    def ragged():
        ctx.process_ragged(d_msgs, w.offs, l2_mode=lob.L2_FINAL, l2_out=l2, stream=stream)

    ragged_ms, ragged_all = timed(ragged)
    # critical path: the longest stream alone
    longest = int(np.argmax(lens))
    one_offs = np.array([w.offs[longest], w.offs[longest + 1]], np.int64)
    one_ms, _ = timed(lambda: ctx.process_ragged(d_msgs, one_offs, book_ids_host=np.array([longest], np.int32),
                                                 stream=stream))
    # the ragged call's final L2 of every book against the per-bucket launches' (the
    # oracle's parity at this size is in the tests)
    ctx.reset(stream=stream)
    ragged()
    torch.cuda.synchronize()
    lr = l2.cpu().numpy()
    ragged_same = all(np.array_equal(lr[ids], p) for ids, p in plain_host)
    res = {"workload": f"{n_books} books, capacity {{50,100,500,1000}} (p .3/.4/.2/.1), flow log-uniform "
                       f"1e2..1e5 (+cap initial orders), final L2",
           "messages": int(w.n_flow.sum()), "initial_orders": w.n_msgs - int(w.n_flow.sum()),
           "max_book_messages": int(lens.max()),
           "ragged_msgs_per_s": int(w.n_flow.sum()) / (ragged_ms / 1e3), "ragged_ms": ragged_ms,
           "plain_per_bucket_msgs_per_s": int(w.n_flow.sum()) / (plain_ms / 1e3), "plain_per_bucket_ms": plain_ms,
           "ragged_over_plain": plain_ms / ragged_ms, "longest_book_alone_ms": one_ms,
           "plain_padded": {"ms": padded_ms, "msgs_per_s": int(w.n_flow.sum()) / (padded_ms / 1e3),
                            "messages_walked": n_padded, "final_l2_equals_plain": padded_same,
                            "note": "type-0 padding to each bucket's longest stream; rate counts real messages"},
           "autotuned_plan": plan, "autotune_s": tune_s, "final_l2_equals_plain": bool(ragged_same)}
    ctx.close()
    return res


def bench_serving(args, n_books=20_000, lams=(50_000, 100_000, 200_000, 500_000), duration_s=0.5):
    """Serving loop: 20,000 books of capacity {50,100,500,1000} resident in HBM;
    replay and step requests (1..1000 messages, log-uniform; steps add up to 4
    agent orders) arrive as a Poisson process; the native server batches them
    continuously under a 1 GiB staging budget.  Latency = host-visible completion
    minus arrival.  (The results' parity with the oracle, replayed in arrival order,
    is checked in the tests.)"""
    from paper_2308_13289_amd import serve as S
    dev = torch.device("cuda:0")
    out = {"workload": f"{n_books} books, capacity {{50,100,500,1000}}, Poisson arrivals for "
                       f"{duration_s}s per rate, 50% replay / 50% step, 1..1000 msgs per request, "
                       f"{args.serve_slots} batch slots of at most {args.serve_max_batch} requests, 1 GiB staging "
                       f"budget", "rates": []}
    # untimed warm-up, a full run at the first rate: the first serving run in a
    # process shows a tail (p99 12-17 ms at 50k req/s against 1 ms on a second run)
    # that a 0.05 s warm-up did not remove
    sw = S.ServingWorkload(n_books, lams[0], duration_s, threads=host_cores())
    ctx = lob.Context(sw.caps, l2_levels=LEVELS, trade_log_records=2 * sw.caps.astype(np.int64) + 2 * 1004)
    ctx.set_plan(lds_slots=128, books_per_block=2)
    srv = S.Server(ctx, n_slots=args.serve_slots, hbm_budget=1 << 30, max_batch=args.serve_max_batch,
                       max_request_msgs=1000, fill_cap=64)
    srv.run(sw.requests(), sw.arrival)
    srv.close()
    ctx.close()
    del sw, ctx, srv
    for lam in lams:
        t0 = time.perf_counter()
        sw = S.ServingWorkload(n_books, lam, duration_s, threads=host_cores())
        caps = sw.caps
        ctx = lob.Context(caps, l2_levels=LEVELS, trade_log_records=2 * caps.astype(np.int64) + 2 * 1004)
        ctx.set_plan(lds_slots=128, books_per_block=2)
        s0, s1 = sw.seed_offsets
        seeds = np.concatenate([sw.w.msgs[a:b] for a, b in zip(s0, s1)])
        soffs = np.concatenate([[0], np.cumsum(s1 - s0)]).astype(np.int64)
        ctx.process(torch.from_numpy(seeds).to(dev), torch.from_numpy(soffs).to(dev))
        torch.cuda.synchronize()
        reqs = sw.requests()
        log(f"serving {lam / 1e3:.0f}k req/s: {sw.n} requests, {int(sw.size.sum())} msgs prepared in "
            f"{time.perf_counter() - t0:.1f}s")
        srv = S.Server(ctx, n_slots=args.serve_slots, hbm_budget=1 << 30, max_batch=args.serve_max_batch,
                       max_request_msgs=1000, fill_cap=64)
        comp = srv.run(reqs, sw.arrival)
        srv.close()
        lat = (comp["complete_ns"] - comp["arrival_ns"]) / 1e6
        kinds = sw.kind[comp["tag"]]
        span_s = (comp["complete_ns"].max() - comp["arrival_ns"].min()) / 1e9
        msgs = int(sw.size.sum() + sw.n_actions.sum())
        ok = bool((comp["status"] == lob.OK).all())
        out["rates"].append({
            "offered_req_per_s": lam, "requests": int(sw.n), "messages": msgs,
            "msgs_per_s": msgs / span_s, "req_per_s": sw.n / span_s,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "step_latency_ms": {"p50": float(np.percentile(lat[kinds == S.STEP], 50)),
                                "p99": float(np.percentile(lat[kinds == S.STEP], 99))},
            "replay_latency_ms": {"p50": float(np.percentile(lat[kinds == S.REPLAY], 50)),
                                  "p99": float(np.percentile(lat[kinds == S.REPLAY], 99))},
            "all_status_ok": ok})
        log(f"  p50 {out['rates'][-1]['latency_ms']['p50']:.3f} ms, p99 {out['rates'][-1]['latency_ms']['p99']:.3f} ms, "
            f"{out['rates'][-1]['msgs_per_s'] / 1e6:.1f} M msgs/s, status ok={ok}")
        ctx.close()
        del sw, reqs, comp
    return out


def bench_step(args, n_books=8192, n_steps=1000, window=100, fills_cap=32):
    """Environment-step form: 8192 books seeded with 50 orders per side, then
    n_steps steps of (100-message data window + up to 4 agent orders) with the L2
    snapshot and agent fills of every step; all windows and actions pre-staged in
    HBM; the n_steps steps captured as one HIP graph."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    t0 = time.perf_counter()
    w = W.step_workload(n_books=n_books, n_steps=n_steps, window=window, threads=host_cores())
    seeds = w.extra["seed_msgs"]
    log(f"step workload: {w.n_msgs} messages generated in {time.perf_counter() - t0:.1f}s")
    ctx = lob.Context(w.caps, l2_levels=LEVELS, trade_log_records=w.caps.astype(np.int64))
    if args.plan:
        ctx.set_plan(**json.loads(args.plan))
    per = seeds + n_steps * window
    d_all = torch.from_numpy(w.msgs).to(dev).view(n_books, per, 8)
    d_seed = d_all[:, :seeds].contiguous().view(-1, 8)
    d_seed_offs = torch.arange(n_books + 1, dtype=torch.int64, device=dev) * seeds
    d_win = d_all[:, seeds:].reshape(n_books, n_steps, window, 8).permute(1, 0, 2, 3).contiguous()
    del d_all
    d_act = torch.from_numpy(w.extra["actions"]).to(dev).permute(1, 0, 2, 3).contiguous()
    n_act = int((w.extra["actions"][:, :, :, 0] != 0).sum())
    del w
    l2 = torch.zeros((n_steps, n_books, 2, LEVELS, 2), dtype=torch.int32, device=dev)
    fills = torch.zeros((n_steps, n_books, fills_cap, 6), dtype=torch.int32, device=dev)
    counts = torch.zeros((n_steps, n_books), dtype=torch.int32, device=dev)

    def seed():
        ctx.reset(stream=stream)
        ctx.process(d_seed, d_seed_offs, stream=stream)

    def one(s, st=stream):
        # st=None: torch's current stream (the capture stream inside torch.cuda.graph)
        ctx.step(d_win[s], l2[s], actions=d_act[s], agent_tid=-1, fills=fills[s], fill_counts=counts[s],
                 stream=st)

    # eager: per-step latency
    seed()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_steps)]
    for s in range(n_steps):
        ev[s][0].record(stream)
        one(s)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])
    eager_out = (l2[-1].clone(), counts.sum().item())
    # graph: all steps captured once, replayed.  With chains > 1 the books are split
    # into that many groups, each stepping through its own chain of launches on its
    # own stream inside the graph (the groups are independent, as the books are): a
    # group's next step starts while the other groups' last waves of this step run.
    seed()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    chains = max(1, args.step_chains)
    bounds = np.linspace(0, n_books, chains + 1).astype(int)
    ids = [torch.arange(bounds[c], bounds[c + 1], dtype=torch.int32, device=dev) for c in range(chains)]
    side = [torch.cuda.Stream(dev) for _ in range(chains - 1)]
    with torch.cuda.graph(g):
        cap = torch.cuda.current_stream(dev)
        fork = torch.cuda.Event()
        fork.record(cap)
        for st in side:
            st.wait_event(fork)
        for s in range(n_steps):
            if chains == 1:
                one(s, None)
                continue
            for c in range(chains):
                lo, hi = int(bounds[c]), int(bounds[c + 1])
                st = cap if c == 0 else side[c - 1]
                ctx.step(d_win[s, lo:hi], l2[s, lo:hi], actions=d_act[s, lo:hi], book_ids=ids[c], agent_tid=-1,
                         fills=fills[s, lo:hi], fill_counts=counts[s, lo:hi], stream=st)
        for st in side:
            join = torch.cuda.Event()
            join.record(st)
            cap.wait_event(join)
    def replays(graph):
        out = []
        for _ in range(max(1, args.graph_reps)):
            seed()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            graph.replay()
            torch.cuda.synchronize()
            out.append(time.perf_counter() - t1)
        return out

    reps = replays(g)
    same = bool(torch.equal(l2[-1], eager_out[0]) and counts.sum().item() == eager_out[1])
    one_chain = None
    if chains > 1:  # the same steps as one chain of launches over all books, for reference
        del g
        g1 = torch.cuda.CUDAGraph()
        seed()
        torch.cuda.synchronize()
        with torch.cuda.graph(g1):
            for s in range(n_steps):
                one(s, None)
        one_chain = n_steps / min(replays(g1))
        same = same and bool(torch.equal(l2[-1], eager_out[0]) and counts.sum().item() == eager_out[1])
        del g1
    total_msgs = n_books * n_steps * window + n_act
    best = min(reps)
    res = {"workload": f"{n_books} books x {n_steps} steps x ({window} data msgs + 0-4 agent orders), "
                       f"capacity 100, L2 + agent fills per step, hipGraph of all steps",
           "graph_chains": chains, "steps_per_s_one_chain": one_chain,
           "steps_per_s": n_steps / best, "msgs_per_s": total_msgs / best,
           "graph_s": best, "graph_replays_s": reps,
           "eager_step_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                             "mean": float(step_ms.mean()), "max": float(step_ms.max())},
           "graph_equals_eager": same, "agent_fills": int(counts.sum().item())}
    ctx.close()
    return res


def bench_exec(args, n_books=8192, n_steps=200, window=100, F=64):
    """Execution-environment steps (Section 5.2; lob_exec_step): 8192 books of
    capacity 100 seeded with 100 orders, each with a buy or sell task of 300-2000
    shares; per step a 100-message data window, the agent's four-level action (a
    random size per level), the matcher with per-message level-1 rows, and the
    observation vector and reward.  Eager steps, timed one by one with HIP events."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    w = W.uniform(n_books, window * n_steps, cap=100, tag=W.TAGS["c3"], threads=host_cores(),
                  name=f"exec{n_books}x{window * n_steps}c100")
    seeds = 100
    per = seeds + window * n_steps
    d_all = torch.from_numpy(w.msgs).to(dev).view(n_books, per, 8)
    ctx = lob.Context(w.caps, l2_levels=LEVELS, trade_log_records=np.full(n_books, 2 * (window + 4) + 8))
    ctx.process(d_all[:, :seeds].contiguous().view(-1, 8),
                torch.arange(n_books + 1, dtype=torch.int64, device=dev) * seeds, stream=stream)
    l2 = ctx.read_l2(stream=stream).cpu().numpy()  # [n][2][L][2]: the seeded books' best prices
    rng = np.random.default_rng(11)
    state = np.zeros(n_books, lob.EXEC_STATE_DTYPE)
    state["task_side"] = np.where(np.arange(n_books) % 2 == 1, 1, -1)
    state["task_qty"] = rng.integers(300, 2000, n_books)
    state["p_init"] = (l2[:, 0, 0, 0].astype(np.int64) + l2[:, 1, 0, 0]) // 2
    start = w.msgs.reshape(n_books, per, 8)[:, seeds, 6:8]
    state["start_s"], state["start_ns"] = start[:, 0], start[:, 1]
    state["end_s"] = start[:, 0] + 1_000_000  # no forced market order within the timed steps
    state["next_oid"] = 1_000_000_000
    d_state = torch.from_numpy(state.view(np.uint8)).to(dev)
    d_win = d_all[:, seeds:].reshape(n_books, n_steps, window, 8).permute(1, 0, 2, 3).contiguous()
    del d_all
    d_act = torch.from_numpy(rng.integers(-20, 60, (n_steps, n_books, 4)).astype(np.int32)).to(dev)
    obs = torch.zeros((n_books, 6 * window + 8), dtype=torch.int32, device=dev)
    reward = torch.zeros(n_books, dtype=torch.float64, device=dev)
    fills = torch.zeros((n_books, F, 6), dtype=torch.int32, device=dev)
    counts = torch.zeros(n_books, dtype=torch.int32, device=dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(n_steps):
        ev[s][0].record(stream)
        ctx.exec_step(d_win[s], d_act[s], d_state, obs, reward, fills, counts, tick=100, passive_ticks=2,
                      agent_tid=-1, lam=0.3, stream=stream)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    st = d_state.cpu().numpy().view(lob.EXEC_STATE_DTYPE)
    res = {"workload": f"{n_books} books x {n_steps} execution steps x ({window} data msgs + the agent's "
                       f"orders), capacity 100, observation + reward per step",
           "steps_per_s": n_steps / wall, "msgs_per_s": n_books * n_steps * window / wall,
           "step_ms": {"p50": float(np.percentile(ms, 50)), "p99": float(np.percentile(ms, 99)),
                       "mean": float(ms.mean())},
           "agent_executed_qty": int(st["exec_qty"].sum()), "tasks_done": int(st["done"].sum()),
           "flags": int(np.bitwise_or.reduce(st["flags"]))}
    ctx.close()
    return res


def _time_plan(w, plan, reps, warmup=1):
    """msgs/s of one plain process launch over workload w with the given plan (books
    reset before every launch), and the launch's final L2 (host array, key "l2")."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    lens = np.diff(w.offs)
    ctx = lob.Context(w.caps, l2_levels=LEVELS, trade_log_records=w.caps.astype(np.int64) + 2 * lens)
    ctx.set_plan(**plan)
    d_msgs = torch.from_numpy(w.msgs).to(dev)
    d_offs = torch.from_numpy(w.offs).to(dev)
    l2 = torch.zeros((w.n_books, 2, LEVELS, 2), dtype=torch.int32, device=dev)
    ms = []
    for k in range(warmup + reps):
        ctx.reset(stream=stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.process(d_msgs, d_offs, l2_mode=lob.L2_FINAL, l2_out=l2, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        if k >= warmup:
            ms.append(a.elapsed_time(b))
    out_l2 = l2.cpu().numpy()
    ctx.close()
    m = float(np.median(ms))
    return {"plan": plan, "kernel_ms": m, "msgs_per_s": w.n_msgs / (m / 1e3), "l2": out_l2}


def _plans_agree(rows):
    """Final L2 of every book equal across the plans (the first is the reference);
    drops the arrays."""
    ref = rows[0].pop("l2")
    for r in rows[1:]:
        r["final_l2_equals_first_plan"] = bool(np.array_equal(r.pop("l2"), ref))
    return rows


def bench_layout(args, reps=3):
    """Sorted sides (this library's layout; registers or LDS) against the paper's
    unsorted fixed-size arrays (a full search of the side per trade and per cancel),
    on the headline workload and on deep books (capacity 1000, half full)."""
    out = {}
    w = W.c1(threads=host_cores())
    out["c1_4096x10100_cap100"] = _plans_agree([_time_plan(w, p, reps) for p in
                                                ({"registers": 1}, {"registers": 0}, {"layout": 1})])
    del w
    w = W.uniform(1024, 5000, cap=1000, tag=21, threads=host_cores(), name="deep1024x5000c1000")
    out["deep_1024x6000_cap1000"] = _plans_agree([_time_plan(w, p, reps) for p in
                                                  ({"registers": 1}, {"registers": 0}, {"layout": 1})])
    return out


def bench_occupancy(args, reps=3):
    """The C1 book shape (capacity 100, 100 initial + 10,000 flow messages) at 1, 2,
    4, 8 and 16 books per SIMD: the serial latency of one book against the
    throughput more waves in flight reach (default plan)."""
    out = []
    for n in (1024, 2048, 4096, 8192, 16384):
        w = W.uniform(n, 10_000, tag=W.TAGS["c1"], threads=host_cores(), name=f"uniform{n}x10000c100")
        r = _time_plan(w, {"registers": 1}, reps)
        out.append({"books": n, "kernel_ms": r["kernel_ms"], "msgs_per_s": r["msgs_per_s"],
                    "ns_per_msg_per_book": r["kernel_ms"] * 1e6 / (w.n_msgs / n)})
        del w
    return {"occupancy": out}


# the paper's own timings (RTX 2080 Ti, JAX; Tables 1-4), quoted as context
PAPER_MS = {
    "single_book": {10: {"add": 0.115, "cancel": 0.081, "match": 0.184},
                    100: {"add": 0.117, "cancel": 0.095, "match": 0.206},
                    1000: {"add": 0.162, "cancel": 0.093, "match": 0.243}},
    "market_qty": {0: 0.132, 10: 0.206, 500: 0.271, 1000: 0.336, 10000: 2.326},
    "thousand_books": {10: {"add": 1.402, "cancel": 1.407, "match": 1.393},
                       100: {"add": 2.649, "cancel": 2.614, "match": 2.612},
                       1000: {"add": 11.75, "cancel": 11.43, "match": 11.47}},
}


def _stats(ms):
    ms = np.asarray(ms)
    return {"mean_ms": float(ms.mean()), "p50_ms": float(np.percentile(ms, 50)),
            "p99_ms": float(np.percentile(ms, 99))}


def bench_micro(args, trials=1000, trials_many=100, n_books=1000):
    """The paper's per-operation timings on this library: a book of capacity N in
    {10, 100, 1000} filled to one third per side, then one message -- add (limit, no
    cross), cancel, match (limit across the spread), or a market order of size Q_a
    (N = 100) -- to one book (single_book, market_qty) or the same message to 1000
    identical books in one call (thousand_books).  Every trial restores the book
    first (reset + write_book, untimed); HIP events bracket the one process call."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {"single_book": {}, "market_qty": {}, "thousand_books": {}, "trials": trials,
           "trials_thousand_books": trials_many, "paper_2080ti_ms": PAPER_MS}
    for N in (10, 100, 1000):
        seeds, _ = W.micro_book(N)
        ctx = lob.Context(np.full(n_books, N, np.int32), l2_levels=LEVELS, trade_log_records=2 * N + 64)
        if args.plan:
            ctx.set_plan(**json.loads(args.plan))
        d_seeds = torch.from_numpy(np.tile(seeds, (n_books, 1))).to(dev)
        d_soffs = torch.arange(n_books + 1, dtype=torch.int64, device=dev) * len(seeds)
        ctx.process(d_seeds, d_soffs, stream=stream)
        dump = ctx.read_book(N, stream=stream)
        one = torch.zeros(1, dtype=torch.int32, device=dev)
        off1 = torch.tensor([0, 1], dtype=torch.int64, device=dev)
        offs_all = torch.arange(n_books + 1, dtype=torch.int64, device=dev)
        cases = [(op, None) for op in W.MICRO_OPS]
        if N == 100:
            cases += [("market", q) for q in (0, 10, 500, 1000, 10000)]
        out["single_book"][N] = {}
        out["thousand_books"][N] = {}
        for op, q in cases:
            msgs = W.micro_messages(N, op, trials, market_qty=q)
            d_msgs = torch.from_numpy(msgs).to(dev)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(trials)]
            for t in range(trials):
                ctx.reset(book_ids=one, stream=stream)
                ctx.write_book(dump[:1], book_ids=one, stream=stream)
                ev[t][0].record(stream)
                ctx.process(d_msgs[t:t + 1], off1, book_ids=one, stream=stream)
                ev[t][1].record(stream)
            torch.cuda.synchronize()
            st = _stats([a.elapsed_time(b) for a, b in ev])
            if op == "market":
                out["market_qty"][q] = st
                continue
            out["single_book"][N][op] = st
            d_many = torch.from_numpy(np.repeat(msgs[:trials_many], n_books, axis=0)).to(dev)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(trials_many)]
            for t in range(trials_many):
                ctx.reset(stream=stream)
                ctx.write_book(dump, stream=stream)
                ev[t][0].record(stream)
                ctx.process(d_many[t * n_books:(t + 1) * n_books], offs_all, stream=stream)
                ev[t][1].record(stream)
            torch.cuda.synchronize()
            st = _stats([a.elapsed_time(b) for a, b in ev])
            st["per_book_us"] = st["mean_ms"] * 1e3 / n_books
            out["thousand_books"][N][op] = st
        out["plan_N%d" % N] = ctx.get_plan().as_dict()
        ctx.close()
    return out


def bench_copy(args, nbytes=1 << 30):
    """Calibration for HBM byte counters: one device-to-device copy of a known size
    (reads nbytes, writes nbytes)."""
    dev = torch.device("cuda:0")
    a = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": "copy calibration", "bytes_read": nbytes, "bytes_written": nbytes, "s": dt,
            "GB_per_s": 2 * nbytes / dt / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="all",
                    choices=["all", "c1", "c0", "c2", "c3", "c4", "copy", "micro", "layout", "occupancy", "exec"])
    ap.add_argument("--tune-trials", type=int, default=19)
    ap.add_argument("--graph-reps", type=int, default=2)
    ap.add_argument("--serve-slots", type=int, default=4, help="serving: batches in flight")
    ap.add_argument("--serve-max-batch", type=int, default=4096, help="serving: requests per batch at most")
    ap.add_argument("--step-chains", type=int, default=2,
                    help="step form: book groups stepping in independent chains inside the graph")
    ap.add_argument("--plan", default=None, help="JSON lob_plan fields")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 "
                                   "(books shard across GPUs with no communication between them)"}))
        sys.exit(2)
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    lob.load()
    if args.workload == "c3":
        print(json.dumps(bench_step(args)), flush=True)
        return
    if args.workload == "c2":
        print(json.dumps(bench_ragged(args)), flush=True)
        return
    if args.workload == "c4":
        print(json.dumps(bench_serving(args)), flush=True)
        return
    if args.workload == "copy":
        print(json.dumps(bench_copy(args)), flush=True)
        return
    if args.workload == "micro":
        print(json.dumps(bench_micro(args)), flush=True)
        return
    if args.workload == "layout":
        print(json.dumps(bench_layout(args)), flush=True)
        return
    if args.workload == "occupancy":
        print(json.dumps(bench_occupancy(args)), flush=True)
        return
    if args.workload == "exec":
        print(json.dumps(bench_exec(args)), flush=True)
        return
    t0 = time.perf_counter()
    if args.workload in ("c1", "all"):
        w = W.c1(threads=host_cores())
        desc = "4096 books, capacity 100/side, 100 initial + 10000 flow messages each (41.4M msgs)"
    else:
        w = W.c0(threads=host_cores())
        desc = "64 books, capacity 100/side, 100 initial + 1000 flow messages each"
    log(f"generated {w.n_msgs} messages in {time.perf_counter() - t0:.1f}s")
    res = bench_uniform(args, w, desc)
    log(f"timed {args.steps} steps: {res['ms_per_step']:.2f} ms/step, {res['value'] / 1e9:.3f} G msgs/s")
    gpu_l2 = res.pop("_l2")
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, w.n_books, gpu_l2=gpu_l2)
        res["verified"] = {"by": "the cpu_baseline leg: the oracle's final L2 of its timed run",
                           **res["cpu_baseline"]["gpu_agrees"]}
        log(f"cpu baseline: {res['cpu_baseline']['value'] / 1e6:.2f} M msgs/s, final L2 of "
            f"{res['verified']['books']} books equal: {res['verified']['final_l2_equal']}")
    del gpu_l2
    del w
    if args.workload == "all":
        res["ragged"] = bench_ragged(args)
        log(f"ragged: {res['ragged']['ragged_msgs_per_s'] / 1e9:.3f} G msgs/s vs plain per bucket "
            f"{res['ragged']['plain_per_bucket_msgs_per_s'] / 1e9:.3f}, padded "
            f"{res['ragged']['plain_padded']['msgs_per_s'] / 1e9:.3f}")
        res["step_form"] = bench_step(args)
        log(f"step form: {res['step_form']['steps_per_s']:.0f} steps/s, "
            f"p99 {res['step_form']['eager_step_ms']['p99']:.3f} ms")
        res["serving"] = bench_serving(args)
        res["exec_env"] = bench_exec(args)
        log(f"execution env: {res['exec_env']['steps_per_s']:.0f} steps/s, "
            f"p99 {res['exec_env']['step_ms']['p99']:.3f} ms")
        res["layout_ablation"] = bench_layout(args, reps=2)
        log("layout ablation (C1 msgs/s): " + ", ".join(
            f"{r['plan']}: {r['msgs_per_s'] / 1e9:.2f} G" for r in res["layout_ablation"]["c1_4096x10100_cap100"]))
        res["paper_tables"] = bench_micro(args, trials=200, trials_many=50)
        log("paper tables: single-book add/cancel/match at N=100: " + ", ".join(
            f"{res['paper_tables']['single_book'][100][op]['mean_ms'] * 1e3:.1f} us" for op in W.MICRO_OPS))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
