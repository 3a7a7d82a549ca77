#!/usr/bin/env python3
"""Benchmark of the QBX hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload star4096] [--mode fwdbwd]

A step is one pass of the whole hot path over one batch of synthetic input that
already sits in HBM: source grid and centers (upsampling), the pair kernels,
evaluation, and (mode fwdbwd) the adjoint for the density and node gradients.
Prints ONE JSON line: interactions/s (centers x sources x operators per second,
forward and forward+backward), the dominant kernel's achieved FP64 rate against
MI355X's vector FP64 peak (its launch durations timed with HIP events on the
launch stream), and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("QBX source-center interactions/s, fwd & fwd+bwd, FP64 @≤1e-11 rel; "
          "% FP64 peak")
SOLVE_METRIC = ("Dirichlet combined-field solve (Section 4.3), GMRES to 1e-14 over QBX products, "
                "FP64: centers x sources of all products per second")
SPLIT_METRIC = ("QBX layer potential with the near/far split of Section 5, FP64 @<=1e-11 rel "
                "to the split oracle: the workload's centers x sources per second")
PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64 (256 CUs x 2.4 GHz x 128 flop/clk)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """sha256 over the HIP sources of libqbx (names and contents)."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1207_4461_amd", "csrc", "*"))):
        if f.endswith((".h", ".hip", ".cpp")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a copy of known
    size), or None when there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc_traffic.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_json:"):
                d = json.loads(line.split(":", 1)[1])
                if d.get("source_sha256") != kernel_source_hash():
                    return None
                return d["bytes_per_launch"]
    return None


def host_cpu() -> dict:
    """The host the oracle runs on: logical CPUs, CPU model, torch's thread count."""
    import torch

    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "threads": torch.get_num_threads()}


def cpu_baseline(args, mode, pb, fwd, step, gpu_vjp):
    """The oracle (as it stands) on the host cores, on bounded samples of the workload:

    - forward: a random sample of targets (both sides) against all sources, sized for
      about a third of --cpu-seconds, and the same on one thread;
    - forward + backward (mode fwdbwd): the oracle's gradient restricted to one
      panel, exact there (that panel's centers against all sources, every other
      center against that panel's sources), compared element by element with the
      GPU adjoint.
    Rates are the sample's centers x sources x operators per second; `value` is the
    rate of the mode the headline measures.  The full step's CPU time is the linear
    extrapolation of that rate to the workload's interactions."""
    import numpy as np
    import torch

    from oracle import qbx_oracle as O
    from paper_1207_4461_amd import flops

    host = host_cpu()
    rng = np.random.default_rng(0)

    def oracle_at(idx):
        if mode == "grad":
            return O.layer_potential_gradient(pb.nodes, pb.density, pb.k, pb.p, pb.r,
                                              pb.oversample, pb.side, pb.kind,
                                              targets=idx)[1].numpy()
        if mode in ("split", "splitbwd"):
            return O.layer_potential_split(pb.nodes, pb.density, pb.k, pb.p, pb.r,
                                           pb.oversample, pb.side, pb.kind, gamma=args.gamma,
                                           targets=idx).numpy()
        return O.layer_potential(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample,
                                 pb.side, pb.kind, targets=idx).numpy()

    # calibrate on 2 targets, then size the forward sample
    t0 = time.perf_counter()
    oracle_at(np.arange(2))
    per = (time.perf_counter() - t0) / 2
    share = args.cpu_seconds / (3.0 if mode == "fwdbwd" else 1.0)
    n = int(min(pb.n_targets, max(2, share / max(per, 1e-6))))
    idx = np.sort(rng.choice(pb.n_targets, size=n, replace=False))
    t0 = time.perf_counter()
    ref = oracle_at(idx)
    tc = time.perf_counter() - t0
    ncent = len(idx) * pb.n_sides
    fwd_inter = flops.interactions(ncent, pb.n_sources, pb.kind)
    fwd_rate = fwd_inter / tc
    if mode == "grad":
        u = step()[1].cpu().numpy()[:, :, idx]
    else:
        u = (step().cpu().numpy()[:, :, idx] if mode in ("split", "splitbwd")
             else fwd().cpu().numpy()[:, :, idx])
    err = float(max(np.abs(u[s, k] - ref[s, k]).max() / np.abs(ref[s, k]).max()
                    for s in range(u.shape[0]) for k in range(u.shape[1])))
    label = {"grad": "normal derivative", "split": "split forward",
             "splitbwd": "split forward"}.get(mode, "forward")
    fwd_sample = (f"{label} at {len(idx)} random targets x {pb.n_sides} sides ({ncent} centers) "
                  f"against all {pb.n_sources} sources, {tc:.1f} s; GPU/oracle max rel err "
                  f"{err:.2e}")
    log(f"cpu oracle {label}: {fwd_rate:.3e} interactions/s over {tc:.1f} s, parity {err:.2e}")

    # the same forward on one thread (one target, both sides)
    threads = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle_at(idx[:1])
        t1 = time.perf_counter() - t0
    finally:
        torch.set_num_threads(threads)
    one_core = flops.interactions(pb.n_sides, pb.n_sources, pb.kind) / t1
    log(f"cpu oracle {label} on 1 thread: {one_core:.3e} interactions/s over {t1:.1f} s")

    inter_step = flops.interactions(pb.n_centers, pb.n_sources, pb.kind)
    cpu = {"value": fwd_rate, "unit": "interactions/s", "cores": threads, "kind": "oracle",
           "sample": fwd_sample, "nproc": host["nproc"], "cpu_model": host["cpu_model"],
           "mode": label, "fwd_value": fwd_rate, "one_thread_fwd_value": one_core}
    if mode == "fwdbwd":
        panel = int(rng.integers(0, pb.n_panels))
        t0 = time.perf_counter()
        rd, rn = O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                       pb.cotangent, panels=[panel])
        tb = time.perf_counter() - t0
        # pairs of the restricted loss: the panel's centers against all sources, every
        # other center against the panel's sources
        qs = 16 * pb.oversample
        pairs = (16 * pb.n_sides * pb.n_sources
                 + (pb.n_targets - 16) * pb.n_sides * qs)
        bwd_inter = pairs * pb.n_kinds
        gd, gn = gpu_vjp()
        gd = gd.cpu().numpy().reshape(pb.n_kinds, -1, 16)[:, panel]
        gn = gn.cpu().numpy()[panel]
        rd = rd.reshape(pb.n_kinds, -1, 16)[:, panel]
        ed = float(np.abs(gd - rd).max() / np.abs(rd).max())
        en = float(np.abs(gn - rn[panel]).max() / np.abs(rn[panel]).max())
        rate = bwd_inter / tb
        log(f"cpu oracle forward+backward: {rate:.3e} interactions/s over {tb:.1f} s, parity "
            f"density {ed:.2e} nodes {en:.2e}")
        cpu.update({
            "value": rate, "mode": "forward+backward",
            "sample": (f"forward+backward: the oracle's gradient restricted to panel {panel} "
                       f"(its {16 * pb.n_sides} centers x all {pb.n_sources} sources, and the "
                       f"other {(pb.n_targets - 16) * pb.n_sides} centers x its {qs} sources), "
                       f"{tb:.1f} s; GPU/oracle max rel err on that panel: density "
                       f"{ed:.2e}, nodes {en:.2e} (at 4096 panels one ulp on every node "
                       f"coordinate moves the D density gradient by about 1.8e-11 and the "
                       f"node gradient by 3.4e-11: the tests' bars follow that). Forward: "
                       f"{fwd_sample}"),
            "bwd_parity": {"panel": panel, "density": ed, "nodes": en}})
    cpu["extrapolation"] = (f"linear in interactions: the full step ({inter_step:.3e} "
                            f"interactions) would take {inter_step / cpu['value']:.0f} s on "
                            f"these {threads} threads, {inter_step / one_core:.0f} s "
                            f"(forward only) on one")
    return cpu


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="star4096",
                    choices=["ellipse32", "star256", "star1024", "random64", "star4096",
                             "paper80"],
                    help="paper80: the size of the paper's own timing (Section 5), for context")
    ap.add_argument("--mode", default=None,
                    choices=["fwd", "fwdbwd", "grad", "split", "splitbwd", "solve"],
                    help="grad: the target derivatives (grad S, grad D, S', D') instead; "
                         "split: the forward with the near/far split (QBX for near panels "
                         "only, each other panel's own 16-point rule applied directly); "
                         "splitbwd: "
                         "that forward and its density adjoint; solve: the "
                         "exterior Dirichlet problem with point-charge data, GMRES to 1e-14 "
                         "(products by the split when --gamma > 0)")
    ap.add_argument("--gamma", type=float, default=6.0,
                    help="split and solve modes: panels within gamma panel radii count as "
                         "near (solve: 0 for plain QBX products)")
    ap.add_argument("--backward", default="fused", choices=["fused", "tape"],
                    help="fwdbwd step: plain forward + fused adjoint (default), or forward "
                         "with tape + source-major adjoint")
    ap.add_argument("--autotune", type=int, default=1,
                    help="time the launch shapes on the workload first (untimed) and use the best")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB: run one plain device-to-device copy of this size first, the "
                         "reference for scaling the HBM byte counters of a --pmc profile")
    ap.add_argument("--restart", type=int, default=300,
                    help="solve mode: Krylov vectors kept between GMRES restarts")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--with-random64", type=int, default=1,
                    help="default run (star4096 fwd+bwd): also time the random64 batch against "
                         "one launch per contour and report it under the key random64")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time of the oracle sample")
    return ap.parse_args()


def tune_fields(mode: str, backward: str) -> int:
    """The launch shapes the timed steps use: the forward's, and the adjoint's
    of the chosen backward."""
    from paper_1207_4461_amd import qbx
    if mode == "fwd":
        return qbx.TUNE_FORWARD
    if mode == "grad":
        return qbx.TUNE_FORWARD | qbx.TUNE_TAPE   # the derivative pass has the tape's shape
    if backward == "fused":
        return qbx.TUNE_FORWARD | qbx.TUNE_FUSED
    return qbx.TUNE_TAPE | qbx.TUNE_ADJOINT


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: only one GPU is measured (the library runs the hot path on a single "
              "MI355X and has no multi-GPU sharding); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import ctypes as C

    import numpy as np
    import torch

    from paper_1207_4461_amd import _lib, flops, inputs as I, qbx

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lib = _lib.load()
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy} MiB read + {args.calibrate_copy} MiB written")
        del src, dst
    if args.workload == "random64":
        return bench_batched(args)
    if args.mode == "solve":
        return bench_solve(args)
    mode = args.mode or "fwdbwd"
    pb = getattr(I, args.workload)()
    dev = torch.device("cuda:0")
    nodes = torch.from_numpy(pb.nodes).to(dev)
    dens = torch.from_numpy(np.ascontiguousarray(pb.density)).to(dev)
    cot = torch.from_numpy(np.ascontiguousarray(pb.cotangent)).to(dev)
    tuning = qbx.get_tuning()
    if args.autotune and mode not in ("split", "splitbwd"):   # the split's shapes are fixed
        t0 = time.perf_counter()
        tuning = qbx.autotune(nodes, dens, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                              passes=1, fields=tune_fields(mode, args.backward))
        log(f"autotune {time.perf_counter() - t0:.1f} s: {tuning}")
    ws = torch.empty(qbx.workspace_bytes(pb.n_panels, pb.p, pb.oversample, pb.side, pb.kind),
                     dtype=torch.uint8, device=dev)
    log(f"workload {args.workload} ({pb.name}): P={pb.n_panels} p={pb.p} k={pb.k} "
        f"centers={pb.n_centers} sources={pb.n_sources} kind={pb.kind} mode={mode}")

    def fwd():
        return qbx.layer_potential(nodes, dens, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                                   workspace=ws)

    tape = torch.empty(qbx.tape_bytes(pb.n_panels, pb.p, pb.side, pb.kind), dtype=torch.uint8,
                       device=dev)

    def step():
        if mode == "fwd":
            return fwd()
        if mode == "grad":
            return qbx.layer_potential_gradient(nodes, dens, pb.k, pb.p, pb.r, pb.oversample,
                                                pb.side, pb.kind, workspace=ws)
        if mode in ("split", "splitbwd"):
            u = qbx.layer_potential_split(nodes, dens, pb.k, pb.p, pb.r, pb.oversample,
                                          pb.side, pb.kind, gamma=args.gamma, workspace=ws)
            if mode == "splitbwd":
                qbx.layer_potential_split_vjp(nodes, dens, cot, pb.k, pb.p, pb.r, pb.oversample,
                                              pb.side, pb.kind, gamma=args.gamma, workspace=ws)
            return u
        if args.backward == "fused":
            # forward, then the adjoint without a tape (one fused pass over the pairs)
            u = fwd()
            qbx.layer_potential_vjp(nodes, dens, cot, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                                    pb.kind, workspace=ws)
            return u
        # forward storing the tape, then the source-major adjoint
        u = qbx.layer_potential(nodes, dens, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                                tape=tape, workspace=ws)
        qbx.layer_potential_vjp(nodes, dens, cot, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                                pb.kind, tape=tape, workspace=ws)
        return u

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # forward alone (for the fwd interactions/s figure)
    nfwd = max(1, args.steps)
    t0 = time.perf_counter()
    for _ in range(nfwd):
        fwd()
    torch.cuda.synchronize()
    fwd_s = (time.perf_counter() - t0) / nfwd

    # timed steps
    lib.qbx_kernel_timer(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    NC = _lib.QBX_TIMER_CLASSES
    ms = (C.c_double * NC)()
    nl = (C.c_int * NC)()
    _lib.check(lib.qbx_kernel_timer_read(ms, nl))
    lib.qbx_kernel_timer(0)
    step_ms = dt / args.steps * 1e3
    inter = flops.interactions(pb.n_centers, pb.n_sources, pb.kind)
    value = inter / (dt / args.steps)

    # per pair-kernel class: algorithmic flops per launch / average launch time
    pairs = pb.n_centers * pb.n_sources
    names = ["forward pair kernel", "adjoint source pass", "batched persistent kernel",
             "forward-with-tape pair kernel", "fused adjoint pair kernel",
             "target-derivative pair kernel", "split near pass", "split far pass",
             "split far-pass adjoint"]
    per_pair = [flops.flops_forward_pair(pb.p, pb.kind), flops.flops_adjoint_pair(pb.p, pb.kind),
                0, flops.flops_tape_pair(pb.p, pb.kind), flops.flops_fused_pair(pb.p, pb.kind),
                flops.flops_grad_pair(pb.p, pb.kind), flops.flops_forward_pair(pb.p, pb.kind),
                flops.flops_far_pair(pb.kind), flops.flops_far_pair(pb.kind)]
    pairs_of = [pairs] * 6 + [0, 0, 0]
    if mode in ("split", "splitbwd"):
        pairs_of[6], pairs_of[7] = flops.split_pairs(pb.nodes, pb.oversample, pb.n_sides,
                                                     args.gamma)
        pairs_of[8] = pairs_of[7]
    kernels = {}
    for c in range(NC):
        if nl[c] == 0 or per_pair[c] == 0:
            continue
        avg = ms[c] / nl[c]
        fl = per_pair[c] * pairs_of[c]
        kernels[names[c]] = {"avg_ms": round(avg, 4), "launches": int(nl[c]), "pairs": pairs_of[c],
                             "flop_per_launch": fl, "tflops": round(fl / (avg * 1e-3) / 1e12, 3)}
    cls = max((c for c in range(NC) if nl[c] and per_pair[c]), key=lambda c: ms[c])
    dom = kernels[names[cls]]
    achieved = dom["tflops"]
    avg_ms = dom["avg_ms"]
    kernel_names = ["k_forward", "k_adjoint_src", "", "k_forward_tape", "k_adjoint_fused",
                    "k_forward_grad", "k_split_near", "k_split_far", "k_split_far_adj"]
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
            "traffic": measured_traffic(kernel_names[cls], args.workload),
            "kernel": names[cls], "kernel_avg_ms": avg_ms, "launches": dom["launches"],
            "flop_per_launch": dom["flop_per_launch"],
            "flop_per_pair": per_pair[cls], "all_pair_kernels": kernels}
    log(f"step {step_ms:.2f} ms, {names[cls]} avg {avg_ms:.3f} ms, {achieved:.2f} TFLOP/s")

    # CPU oracle on a bounded sample of the same workload
    cpu = None
    if args.cpu_baseline:
        cpu = cpu_baseline(args, mode, pb, fwd, step,
                           lambda: qbx.layer_potential_vjp(nodes, dens, cot, pb.k, pb.p, pb.r,
                                                           pb.oversample, pb.side, pb.kind,
                                                           workspace=ws))

    # the batched workload beside the headline (the default run only): random64's
    # persistent launches against one launch per contour, fwd+bwd, each autotuned
    extra = {}
    if args.with_random64 and args.workload == "star4096" and mode == "fwdbwd":
        r = measure_random64(args, "fwdbwd", args.backward, 3, 1, bool(args.autotune))
        extra["random64"] = {
            "workload": "random64: 64 random star contours, 16..512 panels x 16 nodes, "
                        "oversample 4, k~U(5,50), p in {8,12,16}, S or D, exterior, fwd+bwd",
            "interactions_per_s": r["inter"] / r["t_bat"],
            "batched_ms_per_step": round(r["t_bat"] * 1e3, 3),
            "per_contour_ms_per_step": round(r["t_per"] * 1e3, 3),
            "batched_speedup_vs_per_contour": round(r["t_per"] / r["t_bat"], 4),
            "persistent_kernels_ms_per_step": round(r["per_step_ms"], 3),
            "achieved_tflops": round(r["achieved"], 3),
            "frac": round(r["achieved"] / PEAK_FP64_TFLOPS, 4)}
        # the size of the paper's one timing, for context (another machine, another era)
        pc = I.paper80()
        pn = torch.from_numpy(pc.nodes).to(dev)
        pd = torch.from_numpy(np.ascontiguousarray(pc.density)).to(dev)
        pw = torch.empty(qbx.workspace_bytes(pc.n_panels, pc.p, pc.oversample, pc.side, pc.kind),
                         dtype=torch.uint8, device=dev)
        call = lambda: qbx.layer_potential(pn, pd, pc.k, pc.p, pc.r, pc.oversample, pc.side,
                                           pc.kind, workspace=pw)
        call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            call()
        torch.cuda.synchronize()
        t_pc = (time.perf_counter() - t0) / 20
        extra["paper_context"] = {
            "paper": "Section 5: a single-layer apply at p = 5, 7680 sources, 1280 targets, "
                     "0.6 s on 16 cores of a 2.93 GHz Intel Nehalem (about 1.6e7 pairs/s)",
            "this_gpu": f"the same size ({pc.name}: 80 panels, oversample 6, p = 5, S, one side):"
                        f" {t_pc * 1e3:.3f} ms per call, including the source grid and "
                        f"centers ({pc.n_centers * pc.n_sources / t_pc:.3e} pairs/s)"}
        log(f"paper-size forward: {t_pc * 1e3:.3f} ms")

    out = {
        "metric": METRIC if mode not in ("split", "splitbwd") else SPLIT_METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {pb.name}, {pb.n_panels} panels x 16 nodes, "
                               f"oversample {pb.oversample}, k={pb.k}, p={pb.p}, "
                               f"side={'both' if pb.side == 0 else pb.side}, "
                               f"kind={'S+D' if pb.kind == 3 else ('S' if pb.kind == 1 else 'D')}",
                   "mode": mode, "backward": args.backward if mode == "fwdbwd" else None,
                   "gamma": args.gamma if mode in ("split", "splitbwd") else None,
                   "centers": pb.n_centers, "sources": pb.n_sources,
                   "interactions_per_step": inter, "tuning": tuning},
        "fwd_value": inter / fwd_s,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_solve(args):
    """The exterior Dirichlet problem on the workload's curve: data of two point charges
    inside it, GMRES to 1e-14 (qbx_solve_dirichlet), the field checked at three exterior
    points against the exact one.  A step is one whole solve."""
    import ctypes as C

    import numpy as np
    import scipy.special as sps
    import torch

    from paper_1207_4461_amd import _lib, flops, inputs as I, qbx

    lib = _lib.load()
    pb = getattr(I, args.workload)()
    dev = torch.device("cuda:0")
    P, k, p = pb.n_panels, pb.k, pb.p
    charges = [(0.1, 0.2, 1.0), (-0.3, 0.1, 0.5 - 0.2j)]
    obs = np.array([(2.0, 0.5), (-1.5, 1.7), (0.3, -2.2)])

    def field(pts):
        return sum(c * sps.hankel1(0, k * np.hypot(pts[:, 0] - cx, pts[:, 1] - cy))
                   for cx, cy, c in charges)

    nodes = torch.from_numpy(pb.nodes).to(dev)
    f = torch.from_numpy(field(pb.nodes.reshape(-1, 2))).to(dev)
    restart = args.restart
    ws = torch.empty(qbx.solve_workspace_bytes(P, p, pb.oversample, I.EXTERIOR, restart),
                     dtype=torch.uint8, device=dev)
    gamma = args.gamma

    def solve():
        return qbx.solve_dirichlet(nodes, f, k, p, pb.r, pb.oversample, I.EXTERIOR, 1j, gamma,
                                   1e-14, restart, 3000, workspace=ws)

    log(f"solve on {args.workload}: P={P} p={p} k={k} gamma={gamma}")
    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    lib.qbx_kernel_timer(1)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sigma, iters, res = solve()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    NC = _lib.QBX_TIMER_CLASSES
    ms = (C.c_double * NC)()
    nl = (C.c_int * NC)()
    _lib.check(lib.qbx_kernel_timer_read(ms, nl))
    lib.qbx_kernel_timer(0)
    cls = 7 if gamma > 0 else 0
    products = nl[cls] // args.steps
    n_ctr = 2 * pb.n_targets
    inter = flops.interactions(n_ctr, pb.n_sources, 3) * products
    if gamma > 0:
        pairs = flops.split_pairs(pb.nodes, pb.oversample, 2, gamma)[1]
        fl = flops.flops_far_pair(3) * pairs
        kname = "split far pass"
    else:
        fl = flops.flops_forward_pair(p, 3) * n_ctr * pb.n_sources
        kname = "forward pair kernel"
    avg = ms[cls] / nl[cls]
    achieved = fl / (avg * 1e-3) / 1e12
    # the field off the curve: the nodes' own 16-point rule as explicit sources
    t = I.panel_parameters(P).reshape(-1)
    d = pb.curve.deriv(t)
    speed = np.hypot(d[:, 0], d[:, 1])
    _, om = np.polynomial.legendre.leggauss(16)
    w = torch.from_numpy(np.tile(om, P) * (np.pi / P) * speed).to(dev)
    nrm = torch.from_numpy(np.ascontiguousarray(np.stack([d[:, 1], -d[:, 0]], 1) / speed[:, None])).to(dev)
    q = w * sigma
    eps = 1e-3
    out = qbx.apply_explicit(nodes.reshape(-1, 2), nrm, torch.stack([q, q]),
                             torch.from_numpy(obs - np.array([eps, 0.0])).to(dev),
                             torch.full((3,), eps, dtype=torch.float64, device=dev),
                             torch.ones(3, dtype=torch.complex128, device=dev), k, 8, kind=3)
    u = (1j * out[0] - out[1]).cpu().numpy()
    ex = field(obs)
    err = float(np.abs(u - ex).max() / np.abs(ex).max())
    log(f"solve {dt:.3f} s, {iters} Krylov products ({products} in all), residual {res:.2e}, "
        f"field error {err:.2e}; {kname} {avg:.2f} ms, {achieved:.2f} TFLOP/s")
    cpu = None
    if args.cpu_baseline:
        from oracle import qbx_oracle as O

        idx = np.sort(np.random.default_rng(0).choice(pb.n_targets, 8, replace=False))
        sg = sigma.cpu().numpy()
        t0 = time.perf_counter()
        O.layer_potential(pb.nodes, np.stack([sg, sg]), k, p, pb.r, pb.oversample, I.BOTH, 3,
                          targets=idx)
        tc = time.perf_counter() - t0
        cpu = {"value": flops.interactions(2 * len(idx), pb.n_sources, 3) / tc,
               "unit": "interactions/s", "cores": torch.get_num_threads(), "kind": "oracle",
               "sample": f"one S+D product of the oracle (plain QBX, both sides) at {len(idx)} "
                         f"random targets against all {pb.n_sources} sources, {tc:.1f} s"}
    outj = {
        "metric": SOLVE_METRIC, "value": inter / dt, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} curve ({P} panels x 16 nodes, oversample "
                               f"{pb.oversample}, k={k}, p={p}): exterior Dirichlet problem, "
                               "data of 2 point charges inside, alpha = i",
                   "mode": "solve", "gamma": gamma, "restart": restart,
                   "krylov_products": iters, "products": products, "residual": res,
                   "field_rel_error": err},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                     "traffic": None, "kernel": kname, "kernel_avg_ms": round(avg, 4),
                     "launches": int(nl[cls]), "flop_per_launch": fl},
        "cpu_baseline": cpu,
    }
    print(json.dumps(outj), flush=True)


def measure_random64(args, mode: str, backward: str, steps: int, warmup: int, autotune: bool):
    """random64 (64 random contours): the batched persistent launches against one launch
    per contour, each after its own autotuning; returns the measured figures."""
    import ctypes as C

    import numpy as np
    import torch

    from paper_1207_4461_amd import _lib, flops, inputs as I, qbx

    lib = _lib.load()
    pbs = I.random64()
    dev = torch.device("cuda:0")
    B = qbx.Batch(pbs, oversample=4, device=dev)
    cot = B.pack_out([pb.cotangent for pb in pbs])
    inter = sum(flops.interactions(pb.n_centers, pb.n_sources, pb.kind) for pb in pbs)
    log(f"workload random64: {len(pbs)} contours, {sum(pb.n_panels for pb in pbs)} panels, "
        f"{inter:.3e} interactions per pass, mode={mode}")
    fused = backward == "fused"

    def step_batched():
        if mode == "fwd":
            return B.forward()
        u = B.forward(with_tape=not fused)
        B.adjoint(cot, use_tape=not fused)
        return u

    per = []
    for pb in pbs:
        per.append(dict(
            nodes=torch.from_numpy(pb.nodes).to(dev),
            dens=torch.from_numpy(np.ascontiguousarray(pb.density)).to(dev),
            cot=torch.from_numpy(np.ascontiguousarray(pb.cotangent)).to(dev),
            ws=torch.empty(qbx.workspace_bytes(pb.n_panels, pb.p, pb.oversample, pb.side, pb.kind),
                           dtype=torch.uint8, device=dev),
            tape=torch.empty(qbx.tape_bytes(pb.n_panels, pb.p, pb.side, pb.kind),
                             dtype=torch.uint8, device=dev)))

    def step_per_contour():
        for pb, q in zip(pbs, per):
            if mode == "fwd":
                qbx.layer_potential(q["nodes"], q["dens"], pb.k, pb.p, pb.r, pb.oversample,
                                    pb.side, pb.kind, workspace=q["ws"])
            else:
                tp = None if fused else q["tape"]
                qbx.layer_potential(q["nodes"], q["dens"], pb.k, pb.p, pb.r, pb.oversample,
                                    pb.side, pb.kind, tape=tp, workspace=q["ws"])
                qbx.layer_potential_vjp(q["nodes"], q["dens"], q["cot"], pb.k, pb.p, pb.r,
                                        pb.oversample, pb.side, pb.kind, tape=tp,
                                        workspace=q["ws"])

    def timed(fn, n):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    if autotune:
        # the per-contour loop runs with the launch shapes tuned on its largest contour
        big = max(range(len(pbs)), key=lambda i: pbs[i].n_panels)
        q = per[big]
        t0 = time.perf_counter()
        tc = qbx.autotune(q["nodes"], q["dens"], pbs[big].k, pbs[big].p, pbs[big].r,
                          pbs[big].oversample, pbs[big].side, pbs[big].kind, passes=1,
                          fields=tune_fields(mode, backward))
        log(f"per-contour autotune on contour {big} {time.perf_counter() - t0:.1f} s: {tc}")
        for pb, q in zip(pbs, per):   # workspace sizes follow the tuning
            q["ws"] = torch.empty(qbx.workspace_bytes(pb.n_panels, pb.p, pb.oversample, pb.side,
                                                      pb.kind), dtype=torch.uint8, device=dev)
    t_per = timed(step_per_contour, max(1, steps))
    tuning = qbx.get_tuning()
    if autotune:
        t0 = time.perf_counter()
        tuning = B.autotune(passes=1, fields=tune_fields(mode, backward))
        log(f"batched autotune {time.perf_counter() - t0:.1f} s: {tuning}")
    lib.qbx_kernel_timer(1)
    t_bat = timed(step_batched, max(1, steps))
    NC = _lib.QBX_TIMER_CLASSES
    ms = (C.c_double * NC)()
    nl = (C.c_int * NC)()
    _lib.check(lib.qbx_kernel_timer_read(ms, nl))
    lib.qbx_kernel_timer(0)
    # algorithmic flops of the persistent launches of one step
    if mode == "fwd":
        fl = sum(flops.flops_forward_pair(pb.p, pb.kind) * pb.n_centers * pb.n_sources for pb in pbs)
    elif fused:
        fl = sum((flops.flops_forward_pair(pb.p, pb.kind) + flops.flops_fused_pair(pb.p, pb.kind))
                 * pb.n_centers * pb.n_sources for pb in pbs)
    else:
        fl = sum((flops.flops_tape_pair(pb.p, pb.kind) + flops.flops_adjoint_pair(pb.p, pb.kind))
                 * pb.n_centers * pb.n_sources for pb in pbs)
    # one (fwd) or two (fwd+bwd) timed passes per step, each over all the classes' launches
    per_step_ms = ms[2] / max(1, nl[2]) * (1 if mode == "fwd" else 2)
    achieved = fl / (per_step_ms * 1e-3) / 1e12
    log(f"batched {t_bat * 1e3:.2f} ms/step, per-contour {t_per * 1e3:.2f} ms/step, "
        f"persistent kernels {per_step_ms:.2f} ms/step, {achieved:.2f} TFLOP/s")
    return {"inter": inter, "t_bat": t_bat, "t_per": t_per, "tuning": tuning,
            "per_step_ms": per_step_ms, "achieved": achieved, "fused": fused}


def bench_batched(args):
    """64 random contours (random64): one persistent launch per pass vs one launch per contour."""
    mode = args.mode or "fwdbwd"
    r = measure_random64(args, mode, args.backward, args.steps, args.warmup, bool(args.autotune))
    fused, achieved, t_bat, t_per = r["fused"], r["achieved"], r["t_bat"], r["t_per"]
    out = {
        "metric": METRIC, "value": r["inter"] / t_bat, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_bat * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "random64: 64 random star contours, 16..512 panels x 16 nodes, "
                               "oversample 4, k~U(5,50), p in {8,12,16}, S or D, exterior",
                   "mode": mode, "backward": args.backward if mode == "fwdbwd" else None,
                   "interactions_per_step": r["inter"],
                   "tuning": r["tuning"], "per_contour_ms_per_step": t_per * 1e3,
                   "batched_speedup_vs_per_contour": t_per / t_bat},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                     "traffic": None,
                     "kernel": ("batched persistent kernels (forward + fused adjoint)" if fused
                                else "batched persistent kernels (forward-with-tape + adjoint "
                                     "source pass)") if mode != "fwd"
                     else "batched persistent forward",
                     "kernel_ms_per_step": round(r["per_step_ms"], 3)},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
