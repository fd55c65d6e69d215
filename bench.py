#!/usr/bin/env python3
"""Benchmark of the RSM repetitive-task hot path on one MI355X.

Workload (the one the headline metric is quoted on): the two-stage
downscaler-style filter on 30 frames of 1080x1920 FP32 -- an 8-tap
horizontal weighted sum with paving 8, then an 8-tap vertical one -- run
forward and through its adjoint (loss sum(w * out^2)), inputs resident in
HBM.  One step = one training-step call: the fused forward (input ->
output, intermediate kept on chip), dL/dout = 2 w out and the fused adjoint
(input gradient and both stages' weight gradients) in one kernel, then one
small launch that reduces the weight-gradient partial rows.

  value      tiled elems/s: pattern elements gathered by every tiler of the
             step (forward 69.98 M + adjoint 69.98 M per step) / step time
  roofline   the training-step kernel (the step's only large kernel,
             fir_chain_train_pair_kernel<8>): algorithmic bytes per launch
             (read x and the loss weights, write the output and dL/dx) / its
             average duration, measured with HIP events the library records
             immediately around the launch, on its stream, in the timed loop
  cpu_baseline  the CPU oracle (plain C, FP64) on the whole 30-frame step,
             one process per host core over slices of frames; the
             single-thread time is reported beside it

Four copies of the input and of the input gradient (about 1 GB each set)
rotate between steps, so the 256 MiB Infinity Cache does not serve repeated
reads.

Other measurements go under "extra": the same step as separate calls and
through torch.autograd, unfused variants, the overlapping-window adjoint
and training step, the horizontal stage under each placement request, the
polyphase downscaler, the small 64x64 task (per call, planned and
prepared), the 4096^3 matrix products (with their error against FP64),
batched vs plain 2-D filters, the sparse product and the CG solve.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2516.6
FP32_PEAK_TFLOPS = 157.3       # FP32 vector/matrix peak with packed math
FP32_NOPK_TFLOPS = 78.6        # FP32 FMA peak without packed math (what the filters compile to)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of the input (known bytes) for counter scaling")
    return ap.parse_args()


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "fir_chain_train_two_stage_30x1080x1920_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1105_4424_amd", "csrc", "k_window.hip")


def kernel_source_hash():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the training-step kernel from the committed counter
    summary, or None when the summary is missing or was taken on a different
    revision of the kernel source."""
    try:
        fields = {}
        for line in open(TRAFFIC_SUMMARY):
            if ": " in line and line.startswith("- "):
                k, v = line[2:].split(": ", 1)
                fields[k.strip()] = v.strip().strip("`")
        if fields.get("kernel source sha256[:16]") != kernel_source_hash():
            return None
        return float(fields["traffic bytes per launch"])
    except (OSError, KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library runs every kernel on a single MI355X "
              "and has no multi-GPU path (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import rsm_workloads as W
    from paper_1105_4424_amd import _abi, rsm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    F, H, Wd, T = 30, 1080, 1920, 8
    log("generating inputs (30 x 1080 x 1920 FP32)")
    ts = W.two_stage_filter(frames=F, rows=H, cols=Wd, taps=T)
    w = W.loss_weights(ts.v.rep_shape)
    stages = [ts.h, ts.v]
    NCOPY = 4
    xs = [torch.from_numpy(ts.x).to(dev)]
    xs += [xs[0].clone() for _ in range(NCOPY - 1)]
    ch = torch.from_numpy(ts.c_h).to(dev)
    cv = torch.from_numpy(ts.c_v).to(dev)
    w2 = (2.0 * torch.from_numpy(w)).to(dev)
    out = torch.empty(ts.v.rep_shape, device=dev)
    gy = torch.empty_like(out)
    gxs = [torch.empty_like(xs[0]) for _ in range(NCOPY)]
    gch = torch.empty(T, device=dev)
    gcv = torch.empty(T, device=dev)
    chain = rsm.Chain(stages, [ch, cv])

    n_h = int(np.prod(ts.h.rep_shape)) * T
    n_v = int(np.prod(ts.v.rep_shape)) * T
    tiled_per_step = 2 * (n_h + n_v)
    x_bytes = xs[0].numel() * 4
    out_bytes = out.numel() * 4
    train_bytes = x_bytes + out_bytes + out_bytes + x_bytes  # read x, w; write out, dL/dx
    fwd_bytes = x_bytes + out_bytes                  # read x, write out
    adj_bytes = x_bytes + out_bytes + x_bytes        # read x, read dL/dout, write dL/dx
    wd = torch.from_numpy(w).to(dev)

    def step(k, ev=None):
        # one training step: forward, dL/dout = 2 w out and the adjoint of both
        # stages, fused into one pass over x; ev: events the library records
        # immediately around that kernel
        if ev is not None:
            rsm.time_next_kernel(ev[0], ev[1])
        chain.train(xs[k % NCOPY], wd, out, gxs[k % NCOPY], [gch, gcv])

    def step_separate(k, ev=None):
        # the same step as three calls: fused forward, torch's 2 w * out,
        # fused adjoint (events around the forward and the adjoint kernels)
        x = xs[k % NCOPY]
        if ev is not None:
            rsm.time_next_kernel(ev[0], ev[1])
        chain.forward(x, out)
        torch.mul(w2, out, out=gy)
        if ev is not None:
            rsm.time_next_kernel(ev[2], ev[3])
        chain.adjoint(x, gy, gxs[k % NCOPY], [gch, gcv])

    # A pair of timing events around a kernel costs about 14 us of queue time
    # (the stream drains at each timestamp), so the kernels are timed on every
    # SAMPLE-th step of the timed loop (steps 0, SAMPLE, ...), not on all.
    SAMPLE = 4

    def timed(fn, n_ev):
        for k in range(args.warmup):
            fn(k)
        torch.cuda.synchronize()
        evs = {k: [torch.cuda.Event(enable_timing=True) for _ in range(n_ev)]
               for k in range(0, args.steps, SAMPLE)}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            fn(k, evs.get(k))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        us = [float(np.mean([e[2 * i].elapsed_time(e[2 * i + 1]) for e in evs.values()])) * 1e3
              for i in range(n_ev // 2)]
        return ms, us

    log("warmup %d + %d timed steps (fused training step)" % (args.warmup, args.steps))
    ms_per_step, (train_us,) = timed(step, 2)
    value = tiled_per_step / (ms_per_step * 1e-3)
    train_gbs = train_bytes / (train_us * 1e-6) / 1e9
    log("step %.3f ms | fused training step kernel %.1f us %.0f GB/s"
        % (ms_per_step, train_us, train_gbs))
    sep_ms, (fwd_us, adj_us) = timed(step_separate, 4)
    fwd_gbs = fwd_bytes / (fwd_us * 1e-6) / 1e9
    adj_gbs = adj_bytes / (adj_us * 1e-6) / 1e9
    log("separate path: step %.3f ms | fwd %.1f us %.0f GB/s | adjoint %.1f us %.0f GB/s"
        % (sep_ms, fwd_us, fwd_gbs, adj_us, adj_gbs))

    # a device copy of the same size (x into dL/dx, alternating buffers), the
    # practical ceiling for a kernel that reads and writes once
    cev = []
    for k in range(14):
        e = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        e[0].record()
        gxs[k % NCOPY].copy_(xs[k % NCOPY])
        e[1].record()
        if k >= 4:
            cev.append(e)
    torch.cuda.synchronize()
    copy_us = float(np.median([a.elapsed_time(b) for a, b in cev])) * 1e3
    copy_gbs = 2 * x_bytes / (copy_us * 1e-6) / 1e9
    props = torch.cuda.get_device_properties(0)
    log("device copy of %.1f MB: %.1f us %.0f GB/s" % (x_bytes / 1e6, copy_us, copy_gbs))

    result = {
        "metric": "tiled elems/s + HBM GB/s (fwd, adjoint); batched vs plain on 1 MI355X",
        "value": value,
        "unit": "tiled elems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "two-stage 8-tap downscaler filter, training step (forward, "
                               "loss sum(w*out^2), adjoint), 30 frames 1080x1920 FP32",
                   "frames": F, "rows": H, "cols": Wd, "taps": T, "paving": T,
                   "tiled_elems_per_step": tiled_per_step, "hbm_bytes_per_step": train_bytes},
        "roofline": {"bound": "hbm", "achieved": train_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": train_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "fir_chain_train_pair_kernel<8>",
                     "bytes_per_launch": train_bytes,
                     "avg_us": train_us, "timed_launches": len(range(0, args.steps, SAMPLE)),
                     "torch_copy_gbs": copy_gbs,
                     "frac_of_torch_copy": train_gbs / copy_gbs},
        "extra": {"device": {"name": props.name, "arch": getattr(props, "gcnArchName", ""),
                             "compute_units": props.multi_processor_count},
                  "separate_path": {"ms_per_step": sep_ms,
                                    "value": tiled_per_step / (sep_ms * 1e-3)},
                  "forward_fused": {"kernel": "fir_chain_pair_kernel<8>", "avg_us": fwd_us,
                                    "bytes": fwd_bytes, "gbs": fwd_gbs,
                                    "frac": fwd_gbs / HBM_PEAK_GBS},
                  "adjoint_fused": {"kernel": "fir_chain_adjoint_pair_kernel<8>", "avg_us": adj_us,
                                    "bytes": adj_bytes, "gbs": adj_gbs,
                                    "frac": adj_gbs / HBM_PEAK_GBS,
                                    "cache_assisted": True,
                                    "note": "runs right after the forward pass over the same x, "
                                            "part of which the 256 MiB last-level cache still "
                                            "holds: not an HBM-only rate"}},
    }

    if args.copy_calibration:
        # a plain copy of known size: 248.832 MB read + 248.832 MB written per launch
        for _ in range(3):
            gxs[0].copy_(xs[0])
        torch.cuda.synchronize()

    if not args.no_extra:
        result["extra"].update(extras(args, ts, xs, stages, ch, cv, w2, chain))

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(args, W)

    print(json.dumps(result), flush=True)


def time_fn(fn, reps=20, warm=3):
    import numpy as np
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev])) * 1e3


def wall_us(fn, calls=400, warm=20):
    """Wall time per call of back-to-back calls on the host thread (the
    stream drains once at the end)."""
    import time
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / calls * 1e6


def bf16_to_f64(u16):
    """BF16 bit patterns (uint16) widened exactly to FP64."""
    import numpy as np
    return (u16.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def product_errors(got, ref32, refbf, abs32, absbf, rows):
    """Normwise and elementwise error of sampled rows of a product against
    FP64 products of the FP32 inputs and (if given) of the BF16-rounded ones."""
    import numpy as np

    def one(ref, absr):
        d = got - ref
        return {"normwise": float(np.linalg.norm(d) / np.linalg.norm(ref)),
                "max_abs_over_abs_sum": float(np.max(np.abs(d) / absr)),
                "max_rel_large": float(np.max(np.abs(d)[np.abs(ref) > 1e-3 * np.abs(ref).max()]
                                              / np.abs(ref)[np.abs(ref) > 1e-3 * np.abs(ref).max()]))}

    out = {"sample": "%d whole rows of C (rows %d..%d evenly spaced), %d outputs"
                     % (len(rows), rows[0], rows[-1], got.size),
           "fp32_inputs": one(ref32, abs32)}
    if refbf is not None:
        out["bf16_rounded_inputs"] = one(refbf, absbf)
    return out


def extras(args, ts, xs, stages, ch, cv, w2, chain):
    import numpy as np
    import torch

    import rsm_workloads as W
    from paper_1105_4424_amd import _abi, rsm

    dev = xs[0].device
    ex = {}
    # unfused forward (two tap kernels, the intermediate written and re-read)
    mid = torch.empty(ts.h.rep_shape, device=dev)
    out = torch.empty(ts.v.rep_shape, device=dev)
    gy = torch.empty_like(out)
    state = {"k": 0}

    def unfused_fwd():
        k = state["k"] = state["k"] + 1
        chain.forward(xs[k % len(xs)], out, mids=[mid], flags=_abi.NO_FUSE)

    us = time_fn(unfused_fwd)
    b = xs[0].numel() * 4 + 2 * mid.numel() * 4 + out.numel() * 4
    ex["forward_unfused"] = {"avg_us": us, "bytes": b, "gbs": b / us / 1e3, "frac": b / us / 1e3 / HBM_PEAK_GBS}
    torch.mul(w2, out, out=gy)
    gx = torch.empty_like(xs[0])
    gch = torch.empty(8, device=dev)
    gcv = torch.empty(8, device=dev)

    def unfused_adj():
        k = state["k"] = state["k"] + 1
        chain.adjoint(xs[k % len(xs)], gy, gx, [gch, gcv], mids=[mid], flags=_abi.NO_FUSE)

    us = time_fn(unfused_adj)
    b = (out.numel() + 2 * mid.numel() + 2 * xs[0].numel() + mid.numel() * 0) * 4 + mid.numel() * 4
    ex["adjoint_unfused"] = {"avg_us": us, "bytes": b, "gbs": b / us / 1e3, "frac": b / us / 1e3 / HBM_PEAK_GBS}
    log("unfused fwd %.1f us, unfused adjoint %.1f us" % (ex["forward_unfused"]["avg_us"], us))

    # fused forward alone over four input copies (about 1 GB, so the 256 MiB
    # Infinity Cache serves none of its reads and no adjoint's dirty lines
    # are pending), events around the kernel
    xr = list(xs)
    evs = []
    for k in range(24):
        e = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        rsm.time_next_kernel(*e)
        chain.forward(xr[k % len(xr)], out)
        if k >= 4:
            evs.append(e)
    torch.cuda.synchronize()
    us = float(np.median([a.elapsed_time(b) for a, b in evs])) * 1e3
    b = xs[0].numel() * 4 + out.numel() * 4
    ex["forward_fused_standalone"] = {"kernel": "fir_chain_pair_kernel<8>", "avg_us": us, "bytes": b,
                                      "gbs": b / us / 1e3, "frac": b / us / 1e3 / HBM_PEAK_GBS}
    log("fused forward alone %.1f us %.0f GB/s" % (us, b / us / 1e3))
    del xr

    # the same training step as a user of torch writes it: the chain behind
    # torch.autograd.Function (rsm.TiledChain), the loss formed by torch, and
    # loss.backward() running the fused adjoint; wall clock per step, inputs
    # rotated over the copies
    wl = w2 * 0.5
    leaves = [x.detach().clone().requires_grad_(True) for x in xs]
    chl = ch.detach().clone().requires_grad_(True)
    cvl = cv.detach().clone().requires_grad_(True)

    def autograd_step(k):
        xl = leaves[k % len(leaves)]
        xl.grad = None
        chl.grad = None
        cvl.grad = None
        y = rsm.TiledChain.apply(xl, chl, cvl, stages, True)
        loss = (wl * y * y).sum()
        loss.backward()

    for k in range(args.warmup):
        autograd_step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        autograd_step(k)
    torch.cuda.synchronize()
    ag_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    n_tiled = 2 * sum(int(np.prod(st.rep_shape)) * int(np.prod(st.inputs[0].pattern_shape)) for st in stages)
    ex["training_step_autograd"] = {
        "route": "rsm.TiledChain.apply (torch.autograd.Function) + torch loss + loss.backward()",
        "ms_per_step": ag_ms, "value": n_tiled / (ag_ms * 1e-3), "unit": "tiled elems/s",
        "kernels": "fir_chain_pair_kernel<8> (forward), torch elementwise loss and its gradient, "
                   "fir_chain_adjoint_pair_kernel<8> + weight-gradient reduction (backward)"}
    log("autograd route: %.3f ms per step" % ag_ms)
    del leaves

    # adjoint of an overlapping horizontal stage (13 taps every 8 columns,
    # centred origin -6: windows overlap by 5 and wrap at both borders) on the
    # same 30 frames: the input gradient as a per-element gather plus the
    # per-repetition weight-gradient kernel, against the generic atomic
    # scatter-add.  Algorithmic bytes: x and dL/dy read, dL/dx written once.
    F, H, Wd = xs[0].shape
    to = W.h_stage(F, H, Wd, taps=13, pave=8, origin=-6)
    rep_o = (F, H, -(-Wd // 8))
    po = W.Problem(rep_o, [to], W.identity_output(rep_o), W.WSUM)
    co = torch.from_numpy(W.normalised_coeffs(W.rng_for(7), 13)).to(dev)
    gyo = torch.rand(rep_o, device=dev)
    gco = torch.empty(13, device=dev)

    def overlap_adj(flags):
        def run():
            k = state["k"] = state["k"] + 1
            rsm.run_adjoint(po, xs[k % len(xs)], gyo, gx, gco, co, flags=flags)
        return run

    us_g = time_fn(overlap_adj(0))
    us_a = time_fn(overlap_adj(_abi.FORCE_GENERIC), reps=5, warm=1)
    b = 2 * xs[0].numel() * 4 + gyo.numel() * 4
    ex["adjoint_overlapping_13tap_step8"] = {
        "kernels": rsm.plan(po, flags=_abi.PLAN_ADJOINT),
        "avg_us": us_g, "bytes": b, "gbs": b / us_g / 1e3, "frac": b / us_g / 1e3 / HBM_PEAK_GBS,
        "generic_atomic_us": us_a, "speedup_vs_generic": us_a / us_g}
    log("overlapping adjoint: gather %.1f us (%.0f GB/s), generic atomic %.1f us"
        % (us_g, b / us_g / 1e3, us_a))
    del gyo

    # the horizontal stage alone under every port placement the planner
    # honours (the paper's MemoryMapping: one address space per port, in
    # order input, output, weights): taps in registers with uniform weights
    # (the default), the window staged in LDS, one pattern element per lane,
    # everything read in place
    hmid = torch.empty(ts.h.rep_shape, device=dev)
    b_hs = (xs[0].numel() + hmid.numel()) * 4
    ex["placements_horizontal_stage_30x1080x1920"] = {}
    for spaces in (None, ["local", "any", "any"], ["any", "any", "private"], ["global", "any", "any"]):
        name, ports = rsm.plan_placed(ts.h, spaces)

        def run_h(spaces=spaces):
            k = state["k"] = state["k"] + 1
            rsm.run_placed(ts.h, [xs[k % len(xs)]], hmid, spaces, coeffs=ch)

        us = time_fn(run_h, reps=10 if name in ("generic", "pattern_reduce") else 20)
        ex["placements_horizontal_stage_30x1080x1920"][name] = {
            "request": spaces, "ports": ports, "avg_us": us, "bytes": b_hs, "gbs": b_hs / us / 1e3,
            "frac": b_hs / us / 1e3 / HBM_PEAK_GBS}
        log("placement %s (%s): %.1f us %.0f GB/s" % (name, [sp for sp, _ in ports], us, b_hs / us / 1e3))
    del hmid

    # polyphase downscaler (weighted sums writing several outputs per
    # repetition): 30 frames of 1920x1080 -> 720x480; horizontally 3 outputs
    # per 13-tap window every 8 columns, vertically 4 outputs per 14-tap
    # window every 9 rows.  Algorithmic bytes: each stage's input read once
    # and output written once; each adjoint reads x and dL/dy once and
    # writes dL/dx once.
    log("polyphase downscaler 30 x 1080 x 1920 -> 30 x 480 x 720")
    pp = W.polyphase_downscaler()
    pch = torch.from_numpy(pp.c_h).to(dev)
    pcv = torch.from_numpy(pp.c_v).to(dev)
    pmid = torch.empty(pp.h.output.array_shape, device=dev)
    pout = torch.empty(pp.v.output.array_shape, device=dev)
    del pp.x

    def poly_h():
        k = state["k"] = state["k"] + 1
        rsm.run(pp.h, [xs[k % len(xs)]], pmid, coeffs=pch)

    us_h = time_fn(poly_h)
    us_v = time_fn(lambda: rsm.run(pp.v, [pmid], pout, coeffs=pcv))
    pgy = torch.rand(pp.h.output.array_shape, device=dev)
    pgc = torch.empty(pp.c_h.shape, device=dev)

    def poly_h_adj():
        k = state["k"] = state["k"] + 1
        rsm.run_adjoint(pp.h, xs[k % len(xs)], pgy, gx, pgc, pch)

    us_ha = time_fn(poly_h_adj)
    b_h = (xs[0].numel() + pmid.numel()) * 4
    b_v = (pmid.numel() + pout.numel()) * 4
    b_ha = (2 * xs[0].numel() + pmid.numel()) * 4
    ex["polyphase_downscaler_30x1080x1920"] = {
        "horizontal": {"kernel": rsm.plan(pp.h), "avg_us": us_h, "bytes": b_h, "gbs": b_h / us_h / 1e3,
                       "frac": b_h / us_h / 1e3 / HBM_PEAK_GBS},
        "vertical": {"kernel": rsm.plan(pp.v), "avg_us": us_v, "bytes": b_v, "gbs": b_v / us_v / 1e3,
                     "frac": b_v / us_v / 1e3 / HBM_PEAK_GBS,
                     "note": "its 93 MB input was just written by the horizontal stage and is partly "
                             "cache-resident"},
        "horizontal_adjoint": {"kernels": rsm.plan(pp.h, flags=_abi.PLAN_ADJOINT), "avg_us": us_ha,
                               "bytes": b_ha, "gbs": b_ha / us_ha / 1e3,
                               "frac": b_ha / us_ha / 1e3 / HBM_PEAK_GBS}}
    log("polyphase: H %.1f us (%.0f GB/s), V %.1f us, H adjoint %.1f us (%.0f GB/s)"
        % (us_h, b_h / us_h / 1e3, us_v, us_ha, b_ha / us_ha / 1e3))
    del pmid, pout, pgy

    # training step of the overlapping pair (13 taps every 8 columns, then
    # every 8 rows, centred): it runs stage by stage through the workspace
    to = W.two_stage_filter(frames=F, rows=H, cols=Wd, taps=13, pave=8, h_origin=-6, v_origin=-6)
    del to.x
    tw = torch.rand(to.v.rep_shape, device=dev)
    tout = torch.empty(to.v.rep_shape, device=dev)
    tch = torch.from_numpy(to.c_h).to(dev)
    tcv = torch.from_numpy(to.c_v).to(dev)
    tg = [torch.empty(13, device=dev), torch.empty(13, device=dev)]
    tchain = rsm.Chain([to.h, to.v], [tch, tcv])

    def train_overlap():
        k = state["k"] = state["k"] + 1
        tchain.train(xs[k % len(xs)], tw, tout, gx, tg)

    us_t = time_fn(train_overlap, reps=10)
    ex["training_step_overlapping_13tap_step8"] = {
        "route": "stage by stage (windows overlap: not fusable in one pass)", "avg_us": us_t,
        "fused_minimum_bytes": 2 * xs[0].numel() * 4 + 2 * tout.numel() * 4,
        "gbs_on_fused_minimum": (2 * xs[0].numel() * 4 + 2 * tout.numel() * 4) / us_t / 1e3}
    log("overlapping-pair training step %.1f us" % us_t)
    del tw, tout

    # small plain task: 64x64 -> 16x16 sums
    x0, p0 = W.small_sum()
    xd = torch.from_numpy(x0).to(dev)
    o0 = torch.empty((16, 16), device=dev)
    pr0 = rsm.Prepared(p0)
    ex["small_sum_64x64"] = {
        "avg_us": time_fn(lambda: rsm.run(p0, [xd], o0)), "kernel": rsm.plan(p0),
        "call_us": wall_us(lambda: rsm.run(p0, [xd], o0)),
        "prepared_call_us": wall_us(lambda: pr0.run([xd], o0)),
        "note": "avg_us: HIP events around one rsm.run call (host marshalling, the plan kept for "
                "these descriptors, launch, kernel); call_us / prepared_call_us: wall time per call "
                "of 400 back-to-back calls through rsm.run and through rsm.Prepared.run"}
    pr0.close()

    # matrix product on the matrix cores
    M = N = K = 4096
    log("matrix product 4096^3")
    a, bm, ab, bb = W.matmul_inputs(M, N, K)
    pm = W.matmul_tilers(M, N, K)
    da = torch.from_numpy(ab.view(np.int16)).view(torch.bfloat16).to(dev)
    db = torch.from_numpy(bb.view(np.int16)).view(torch.bfloat16).to(dev)
    cm = torch.empty((M, N), device=dev)
    pm.compute = "bf16"
    # the clock settles only after some milliseconds of matrix-core load:
    # about 50 products of warm-up before timing
    us = time_fn(lambda: rsm.run(pm, [da, db], cm), reps=30, warm=50)
    tf = 2.0 * M * N * K / us / 1e6
    ex["matmul_bf16_4096"] = {"avg_us": us, "tflops": tf, "frac": tf / BF16_PEAK_TFLOPS,
                              "kernel": rsm.plan(pm, dtypes=(torch.bfloat16,))}
    # error of the product against FP64 on a sample of whole rows of C
    rows = np.linspace(0, M - 1, 64).astype(np.int64)
    ref32 = a[rows].astype(np.float64) @ bm.astype(np.float64)
    refbf = bf16_to_f64(ab[rows]) @ bf16_to_f64(bb)
    absbf = np.abs(bf16_to_f64(ab[rows])) @ np.abs(bf16_to_f64(bb))
    abs32 = np.abs(a[rows].astype(np.float64)) @ np.abs(bm.astype(np.float64))
    got = cm[torch.from_numpy(rows).to(dev)].double().cpu().numpy()
    ex["matmul_bf16_4096"]["error_vs_fp64"] = product_errors(got, ref32, refbf, abs32, absbf, rows)
    log("bf16 product error: %.3e normwise vs FP64 of the FP32 inputs, %.3e vs FP64 of the BF16 inputs"
        % (ex["matmul_bf16_4096"]["error_vs_fp64"]["fp32_inputs"]["normwise"],
           ex["matmul_bf16_4096"]["error_vs_fp64"]["bf16_rounded_inputs"]["normwise"]))
    pm.compute = "f32"
    fa = torch.from_numpy(a).to(dev)
    fb = torch.from_numpy(bm).to(dev)
    us = time_fn(lambda: rsm.run(pm, [fa, fb], cm), reps=10, warm=8)
    tf = 2.0 * M * N * K / us / 1e6
    ex["matmul_f32_4096"] = {"avg_us": us, "tflops": tf, "frac": tf / FP32_PEAK_TFLOPS,
                             "kernel": rsm.plan(pm)}
    got = cm[torch.from_numpy(rows).to(dev)].double().cpu().numpy()
    ex["matmul_f32_4096"]["error_vs_fp64"] = product_errors(got, ref32, None, abs32, None, rows)
    log("matmul bf16 %.1f TF/s, f32 %.1f TF/s" % (ex["matmul_bf16_4096"]["tflops"], tf))
    del da, db, fa, fb, cm

    # 512 uneven 2-D filters: one persistent graph launch vs 512 plain launches
    log("batched 2-D filters: 512 instances")
    insts = W.filter_batch(512)
    bx = [torch.from_numpy(i.x).to(dev) for i in insts]
    bc = [torch.from_numpy(i.coeffs).to(dev) for i in insts]
    bo = [torch.empty(i.out_shape, device=dev) for i in insts]
    batch = rsm.Batch([i.problem() for i in insts], bx, bo, bc)
    info = batch.info()
    us_b = time_fn(batch.run, reps=20)
    us_p = time_fn(batch.run_plain, reps=10)
    nbytes = sum(4 * (i.H * i.W + i.out_shape[0] * i.out_shape[1]) for i in insts)
    flops = sum(2 * i.out_shape[0] * i.out_shape[1] * i.k * i.k for i in insts)
    ideal_us = sum(max(4e-6 * (i.H * i.W + i.out_shape[0] * i.out_shape[1]) / HBM_PEAK_GBS * 1e3,
                       2e-6 * i.out_shape[0] * i.out_shape[1] * i.k * i.k / FP32_NOPK_TFLOPS)
                   for i in insts)
    ex["batched_2d_filters_512"] = {
        "batched_us": us_b, "plain_us": us_p, "speedup": us_p / us_b, "bytes": nbytes,
        "flops": flops, "gbs": nbytes / us_b / 1e3, "roofline_ideal_us": ideal_us,
        "frac": ideal_us / us_b, "tiles": info["n_tiles"], "grid": info["grid"],
        "tuned_classes": info["tuned_classes"]}
    log("batched %.1f us, plain %.1f us, ideal %.1f us" % (us_b, us_p, ideal_us))
    batch.close()
    del bx, bo

    # sparse matrix-vector product of the case study's size (indirect tilers), FP64
    A = W.stencil27_csr(51)
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col_idx).to(dev)
    va = torch.from_numpy(A.vals).to(dev)
    xv = torch.from_numpy(W.rng_for(6).uniform(-1, 1, A.n)).to(dev)
    yv = torch.empty(A.n, dtype=torch.float64, device=dev)
    us = time_fn(lambda: rsm.run_csr(rp, ci, va, xv, yv), reps=50)
    b = A.nnz * 12 + (A.n + 1) * 4 + A.n * 8 * 2
    ex["spmv_f64_stencil27_51cubed"] = {"avg_us": us, "bytes": b, "gbs": b / us / 1e3,
                                        "frac": b / us / 1e3 / HBM_PEAK_GBS, "n": A.n, "nnz": A.nnz,
                                        "cache_assisted": True,
                                        "note": "the 44 MB working set is re-read by 50 back-to-back "
                                                "products and stays in the 256 MiB last-level cache: "
                                                "a cache-resident rate, not an HBM one"}
    log("spmv %.1f us %.0f GB/s" % (us, b / us / 1e3))

    # the case study's conjugate-gradient loop at its size, FP64, tol 1e-10;
    # GFLOP/s by the flop model of the paper's Table 1: iterations x (2 NNZ + 10 N)
    bv = torch.from_numpy(W.cg_rhs(A.n)).to(dev)
    xc = torch.zeros(A.n, dtype=torch.float64, device=dev)

    def solve():
        xc.zero_()
        return rsm.cg_solve(rp, ci, va, bv, xc, tol=1e-10, check_every=32)

    info = solve()
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        info = solve()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    flops = info["iterations"] * (2 * A.nnz + 10 * A.n)
    ex["cg_f64_stencil27_51cubed"] = {
        "iterations": info["iterations"], "converged": info["converged"], "ms": ms,
        "us_per_iteration": ms * 1e3 / max(info["iterations"], 1), "gflops": flops / ms / 1e6,
        "tol": 1e-10, "n": A.n, "nnz": A.nnz, "cache_assisted": True,
        "note": "the 53 MB working set of matrix and vectors stays in the 256 MiB last-level cache "
                "across iterations",
        "paper_1gpu_context": {"gflops": 1.45, "iterations": 116, "seconds": 0.659,
                               "hardware": "Tesla T10, FEM matrix (Table 1)"}}
    log("cg %d iterations %.2f ms (%.1f us/iter) %.1f GFLOP/s" %
        (info["iterations"], ms, ms * 1e3 / max(info["iterations"], 1), flops / ms / 1e6))
    return ex


def _cpu_slice(frames, seed, q):
    """Worker of the all-core CPU baseline: the oracle's forward of both
    stages and their adjoint on `frames` frames (inputs made before timing)."""
    import rsm_workloads as W
    import oracle
    ts = W.two_stage_filter(frames=frames, seed=seed)
    w = W.loss_weights(ts.v.rep_shape, seed=seed + 1000)
    t0 = time.perf_counter()
    oracle.chain_adjoint([ts.h, ts.v], ts.x, w)
    q.put((t0, time.perf_counter()))


def host_cpu():
    """(threads this process may use, CPU model name)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return n, model


def cpu_baseline(args, W):
    """The oracle (plain C, FP64, unchanged) on the whole 30-frame step --
    forward of both stages and their adjoint -- once on one thread, and once
    as one process per host core, each running the single-thread oracle on
    its slice of the frames (frames are independent repetitions).  The
    all-core figure is the reported value."""
    import multiprocessing as mp

    import oracle

    per_frame_tiled = 2 * (1080 * 240 * 8 + 135 * 240 * 8)
    threads, model = host_cpu()
    # the machine's CPU share for one GPU is 16 threads, whatever the host shows
    procs = max(1, min(16, threads, 30))

    log("cpu baseline: oracle on 30 frames, one thread")
    ts = W.two_stage_filter(frames=30)
    w = W.loss_weights(ts.v.rep_shape)
    t0 = time.perf_counter()
    oracle.chain_adjoint([ts.h, ts.v], ts.x, w)
    t1 = time.perf_counter() - t0
    del ts, w

    log("cpu baseline: oracle on 30 frames, %d processes" % procs)
    ctx = mp.get_context("spawn")   # no fork of a process that holds the GPU
    walls = []
    for rep in range(3):
        q = ctx.Queue()
        share = [30 // procs + (1 if k < 30 % procs else 0) for k in range(procs)]
        ps = [ctx.Process(target=_cpu_slice, args=(share[k], 100 + k, q)) for k in range(procs)]
        for p in ps:
            p.start()
        spans = [q.get() for _ in ps]
        for p in ps:
            p.join()
        walls.append(max(e for _, e in spans) - min(b for b, _ in spans))
    tn = sorted(walls)[1]
    return {"value": 30 * per_frame_tiled / tn, "unit": "tiled elems/s", "cores": procs,
            "kind": "oracle", "seconds": tn,
            "single_thread": {"value": 30 * per_frame_tiled / t1, "seconds": t1, "cores": 1},
            "cpu_model": model, "host_threads": threads,
            "sample": "the whole step: 30 frames of 1080x1920, forward of both stages + adjoint, FP64 C "
                      "oracle; %d processes of the single-thread oracle over frame slices (%s frames each, "
                      "same shapes and distributions, per-slice seeds), median wall time of 3 runs from "
                      "the first slice's start to the last slice's end; the single-thread figure runs "
                      "the 30 frames in one process" % (procs, "/".join(sorted({str(x) for x in share})))}


if __name__ == "__main__":
    main()
