"""Throughput and time to a target error of the VEGAS+ iteration on one MI355X.

Default run (one JSON line): the learned warp against plain VEGAS+ on the
d=16 correlated Gaussian (s = 0.03, rho = 0.9, 1024 intervals, 1e6
evaluations per iteration, FP32 sample path with FP64 accumulators; the warp
is four coupling layers with 2x64 BF16 MLPs).  Each method runs from create,
through the same continuation warm-up, until its combined relative error
estimate reaches 1e-4 or the caps (2000 iterations, 600 s); the line gives
both wall times, both estimates against the closed form, and the warped
iteration's throughput over K timed iterations after the run.  Sub-records
give the other workloads in the same run (d=4 Gaussian product in FP64, the
d=8 three-Gaussian mixture, the d=4 ridge, the batch of 4096 Genz
integrals), each with its dominant kernel against the roofline (timed with
HIP events inside the library on its stream) and the CPU oracle timed on a
bounded sample of the same workload.

--workload NAME runs one workload alone.  Inputs (map, allocation,
parameters) are resident in HBM before timing starts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz -> VALU lane-operations/s
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9


def valu_ops_per_eval(dim: int, family: int, n_terms: int = 0) -> int:
    """Algorithmic VALU issue slots of one sample of the FP32 path: the
    operations the method itself needs, each counted once.  Every VALU
    instruction takes one issue slot, the transcendental exp2 included: it
    runs on its own half-rate unit while the other VALU instructions issue
    (alone, exp2 retires at half rate; in the 1000-term ridge integrand,
    4345 instructions per sample of which 1001 are exp2 retire at 0.9 per
    slot, which two slots per exp2 would put above 1).  The exp2 unit's own
    bound, two slots per exp2, stays below the issue bound for every
    family here.

    Philox4x32-10, per block of 4 axes: 10 rounds x (2 32x32->64 products +
    2 three-input xors) = 40.  Per axis: fixed-point bin (product, two
    shifts/masks, stratum multiply-add, divide-by-constant high product and
    shift, remainder) 7, offset (2 converts, fma, multiply) 4, map (address,
    difference, fma, two Jacobian products) 5, integrand accumulators 3, two
    histogram addresses 2 -> 21.  Integrand finish: GAUSS_DIAG mean and
    spread 5, per Gaussian term 3 + exp2, prefactor 3 + exp2; GAUSS_CORR
    spread, quadratic form 8 + exp2.  Weight, square and FP64 cube
    moments: 8.
    """
    import vegas_inputs as vi
    blocks = (dim + 3) // 4
    if family == vi.GAUSS_DIAG:
        finish = 5 + 4 * n_terms + 4
    elif family == vi.GAUSS_CORR:
        finish = 9
    else:
        finish = 4
    return 40 * blocks + 21 * dim + finish + 8


WORKLOADS = {
    "gauss3_8d": "d=8 mixture of 3 Gaussians s=0.05, 1024 intervals, FP32 sample path + FP64 accumulators",
    "ridge_4d": "d=4 ridge of 1000 Gaussians s=0.01 on the diagonal, 1024 intervals, FP32 + FP64 accumulators",
    "gauss_prod_4d": "d=4 Gaussian product s=0.1, 128 intervals, FP64 throughout",
    "corr_gauss_16d": "d=16 correlated Gaussian rho=0.9 s=0.03, 1024 intervals, FP32 + FP64 accumulators",
    "corr_gauss_16d_mild": "d=16 correlated Gaussian rho=0.3 s=0.2, 64 intervals, FP32 + FP64 accumulators",
    "genz_batch": "4096 Genz product-peak / Gaussian integrals, d in 3..12, budgets log-uniform in 1e4..1e7 "
                  "evals/iteration, 256 intervals, streams schedule (one context per problem over autotuned "
                  "streams), FP32 sample path + FP64 accumulators",
}


FILL_SOURCES = ["fill.hip", "fill_dev.hpp", "batch.hip", "sample.hpp", "common.hpp", "families.hpp", "layout.hpp"]
FLOW_SOURCES = ["flow.hip", "flow_train.hip", "flow.hpp", "flow_dev.hpp", "common.hpp", "fill_dev.hpp", "layout.hpp",
                "../build.py"]                 # its per-file code generation options


def source_hash(files=FILL_SOURCES) -> str:
    """Hash of a kernel's sources: a profiled HBM figure is reported only
    while it still describes the kernel being timed."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2408_09229_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def fill_source_hash() -> str:
    return source_hash(FILL_SOURCES)


def profiled_traffic(workload: str, prefix: str = "k_fill", files=FILL_SOURCES, kernel=None):
    """HBM bytes per launch of a kernel from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary profiles/<prefix>_<workload>.md (scaled by a device
    copy of known size; with kernel given, that kernel's entry of the
    summary's record), or None when there is none or the sources changed
    since it was taken."""
    import re
    path = os.path.join(ROOT, "profiles", f"{prefix}_{workload}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_hash") != source_hash(files):
        return None
    if kernel is not None:
        rec = rec.get("kernels", {}).get(kernel, {})
    return rec.get("traffic_bytes")


def host_info():
    """Cores and CPU model of the host the oracle is timed on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(w, budget_evals: int, iters: int, target_s: float = 15.0):
    """The oracle on the same integrand, dimension and intervals: `iters`
    iterations of at most `budget_evals` evaluations, cut so that the whole
    sample takes about target_s seconds (a one-iteration probe at 2e4
    evaluations sets the rate)."""
    import oracle
    probe = min(budget_evals, 20_000)
    t0 = time.perf_counter()
    oracle.run(w.dim, w.n_g, probe, w.family, w.params, n_iter=1, seed=w.seed, alpha=w.alpha, beta=w.beta)
    per_eval = (time.perf_counter() - t0) / probe
    n = int(min(budget_evals, max(probe, target_s / iters / per_eval)))
    ww = w.with_(n_eval=n, n_iter=iters)
    t0 = time.perf_counter()
    oracle.run(ww.dim, ww.n_g, ww.n_eval, ww.family, ww.params, n_iter=ww.n_iter, seed=ww.seed,
               alpha=ww.alpha, beta=ww.beta)
    dt = time.perf_counter() - t0
    return {"value": n * iters / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} iterations x {n:,} evals of the same integrand, dim and intervals "
                      f"(single-threaded FP64 C oracle, {dt:.1f} s)", **host_info()}


def cpu_baseline_batch(insts, budget_evals: int):
    """The oracle over the first problems of the batch (one iteration each)
    until their budgets add up to about budget_evals."""
    import oracle
    import vegas_inputs as vi
    t0 = time.perf_counter()
    done = 0
    n = 0
    for i, x in enumerate(insts):
        if done >= budget_evals:
            break
        oracle.run(x.dim, vi.BATCH_N_G, x.n_eval, x.family, x.params, n_iter=1, seed=0, inst=i)
        done += x.n_eval
        n += 1
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"one iteration of the first {n} problems of the batch ({done:.2e} evals; "
                      f"single-threaded FP64 C oracle, {dt:.1f} s)", **host_info()}


def cpu_baseline_warp(w, train_stride: int, steps: int, target_s: float = 10.0):
    """The oracle's plain iteration on the same workload (sized to about
    target_s seconds), and its warp on a sample sized the same way: the FP64
    numpy forward pass with BF16 emulation for every sample, plus the loss
    gradient through the inverse chain for the training share of a warped
    iteration (steps / train_stride of the samples).  Evals/s of the plain
    iteration, and of a warped one (the costs per sample added)."""
    import numpy as np
    from oracle import flow as fl
    base = cpu_baseline(w, w.n_eval, 16, target_s=target_s)
    rng = np.random.default_rng(0)
    th = fl.init_params(w.dim, 0)
    probe = 20_000
    t0 = time.perf_counter()
    _, _, zf = fl.forward(th, rng.random((probe, w.dim)), emu=True, return_z=True)
    fl.loss_grad(th, zf, np.full(probe, 1.0 / probe), emu=True)
    n = int(max(probe, min(1_000_000, target_s / ((time.perf_counter() - t0) / probe))))
    y = rng.random((n, w.dim))
    t0 = time.perf_counter()
    _, _, zf = fl.forward(th, y, emu=True, return_z=True)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    fl.loss_grad(th, zf, np.full(n, 1.0 / n), emu=True)
    t_grad = time.perf_counter() - t0
    share = steps / max(train_stride, 1)
    per_flow = (t_fwd + share * t_grad) / n
    per_plain = 1.0 / base["value"]
    base["warp_value"] = 1.0 / (per_flow + per_plain)
    base["sample"] += (f"; warp: forward of {n:,} samples ({t_fwd:.1f} s) and the loss gradient on them "
                       f"({t_grad:.1f} s), FP64 numpy with BF16 emulation; a warped iteration trains "
                       f"{steps} steps on 1/{train_stride} of its samples, so warped evals/s = 1/(plain + "
                       f"forward + {share:g} x gradient seconds per sample)")
    return base


# algorithmic multiply-add flops of the warp, per sample (2 per multiply-add;
# the conditioner MLP is 8 -> 64 -> 64 -> 16)
FLOW_MLP_FLOPS = 2 * (8 * 64 + 64 * 64 + 64 * 16)            # one layer's forward
FLOW_SAMPLE_FLOPS = 4 * FLOW_MLP_FLOPS                       # the sampling pass
# one training step: the inverse pass (4 forwards) and, per layer, the forward
# again plus dO W3, dA2 W2, dA1 W1 and the three weight gradients
FLOW_TRAIN_FLOPS = 4 * FLOW_MLP_FLOPS + 4 * (FLOW_MLP_FLOPS + 2 * 2 * (16 * 64 + 64 * 64 + 64 * 8))


def run_batch(args, insts=None):
    """The batched workload: every step is one iteration of all 4096 problems."""
    import torch
    import numpy as np
    import vegas_inputs as vi
    from paper_2408_09229_amd import VegasBatch, make_config
    from tests import closed_forms as cf
    insts = insts or vi.genz_batch(4096, seed=0)
    torch.cuda.set_device(0)
    cfgs = [make_config(x.dim, vi.BATCH_N_G, x.n_eval, seed=0, instance=i, precision=vi.BATCH_PRECISION,
                        max_iter=args.warmup + args.steps + 1) for i, x in enumerate(insts)]
    cache = args.tune_cache or os.path.join(os.path.expanduser("~"), ".cache", "vegas_mi355x", "tune.txt")
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    b = VegasBatch(cfgs, [(x.family, x.params) for x in insts], tune_cache=cache)
    inf = b.info()
    n_eval = inf.n_eval_total
    print(f"[bench] genz_batch: n={len(insts)} evals/iteration={n_eval:.4e} cubes={inf.n_cubes_total:.3e} "
          f"streams={inf.n_streams} tuned={inf.tuned} ({inf.tune_ms:.2f} ms fill pass) "
          f"ws={inf.workspace_bytes / 2**30:.2f} GiB", file=sys.stderr, flush=True)
    b.adapt(args.warmup)
    torch.cuda.synchronize()
    b.set_timing(True)
    st = b.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    b.integrate(args.steps)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    phases, n_timed = b.get_timing()
    res = b.results()
    # streams schedule: the timed span is the whole iteration of every
    # problem (fills and updates on all streams), so the fill's rate below is
    # a lower bound
    iter_ms = phases[0] / max(n_timed, 1)
    ops = sum(valu_ops_per_eval(x.dim, x.family) * x.n_eval for x in insts)
    ach = ops / (iter_ms / 1e3)
    ex = np.array([cf.genz_ppeak(x.params, x.dim) if x.family == vi.GENZ_PPEAK else cf.genz_gauss(x.params, x.dim)
                   for x in insts])
    z = (res["integral"] - ex) / np.sqrt(res["sigma2"])
    rel = np.abs(res["integral"] / ex - 1.0)
    print(f"[bench] iteration of all problems {iter_ms:.3f} ms; max|z| {np.abs(z).max():.2f}, "
          f"|z|>3 {np.mean(np.abs(z) > 3):.4f}", file=sys.stderr, flush=True)
    out = {
        "metric": "integrand evals/sec (VEGAS+ iteration)",
        "value": n_eval * args.steps / (ms / 1e3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": vi.BATCH_PRECISION,
        "data": "synthetic",
        "config": {"workload": f"genz_batch: {WORKLOADS['genz_batch']}, {n_eval:.3e} evals/iteration",
                   "n_problems": len(insts), "n_eval": n_eval, "n_intervals": vi.BATCH_N_G,
                   "schedule": {"kind": "streams", "n_streams": inf.n_streams, "tuned": inf.tuned},
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": VALU_LANE_OPS_PEAK / 1e12,
                     "unit": "T VALU issue-slots/s", "frac": ach / VALU_LANE_OPS_PEAK,
                     "traffic": profiled_traffic("genz_batch"),
                     "kernel": "k_fill of every problem, timed as the whole iteration", "kernel_ms": iter_ms},
        "result": {"iterations_combined": int(res["n_iter_combined"][0]), "max_abs_z": float(np.abs(z).max()),
                   "frac_abs_z_gt3": float(np.mean(np.abs(z) > 3)), "median_rel_err": float(np.median(rel))},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(insts, int(args.cpu_evals))
    b.close()
    return out


def copy_calibration() -> int:
    """A plain 256 MiB device copy, three times: its FETCH_SIZE / WRITE_SIZE
    counters give the scale factors of the HBM counters."""
    import torch
    src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return src.numel() * 4


def run_single(args, w):
    """One workload: W untimed iterations, then K timed ones."""
    import torch
    import vegas_inputs as vi
    from paper_2408_09229_amd import Vegas, make_config
    torch.cuda.set_device(0)
    cfg = make_config(w.dim, w.n_g, w.n_eval, alpha=w.alpha, beta=w.beta, seed=w.seed, precision=w.precision,
                      max_iter=args.warmup + args.steps + 1)
    v = Vegas(cfg, w.family, w.params)
    print(f"[bench] {w.name}: n_eval={w.n_eval} tiles={v.info.n_tiles} wg={v.info.n_workgroups}",
          file=sys.stderr, flush=True)
    v.adapt(args.warmup)
    torch.cuda.synchronize()
    v.set_timing(True)
    st = v.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    v.integrate(args.steps)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    phases, n_timed = v.get_timing()
    r = v.result()
    ms_step = ms / args.steps
    value = w.n_eval * args.steps / (ms / 1e3)
    fill_ms = phases[0] / max(n_timed, 1)
    from tests import closed_forms
    exact = closed_forms.exact(w)
    n_terms = int(w.params[2]) if w.family == vi.GAUSS_DIAG else 0
    ops = valu_ops_per_eval(w.dim, w.family, n_terms) * w.n_eval
    ach = ops / (fill_ms / 1e3)
    print(f"[bench] integral={r.integral:.12f} +- {math.sqrt(r.sigma2):.3e} chi2/dof={r.chi2_dof:.2f} "
          f"phases ms/it: fill {fill_ms:.3f} fixup+est {phases[1] / n_timed:.3f} alloc "
          f"{phases[2] / n_timed:.3f} map {phases[3] / n_timed:.3f}", file=sys.stderr, flush=True)
    out = {
        "metric": "integrand evals/sec (VEGAS+ iteration)",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.precision,
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {WORKLOADS[w.name]}, {w.n_eval:.0e} evals/iteration",
                   "n_eval": w.n_eval, "dim": w.dim, "n_intervals": w.n_g, "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": VALU_LANE_OPS_PEAK / 1e12,
                     "unit": "T VALU issue-slots/s", "frac": ach / VALU_LANE_OPS_PEAK, "traffic": profiled_traffic(w.name),
                     "kernel": "k_fill", "kernel_ms": fill_ms},
        "result": {"integral": r.integral, "sigma": math.sqrt(r.sigma2), "chi2_dof": r.chi2_dof,
                   "exact": exact, "z": (r.integral - exact) / math.sqrt(r.sigma2) if r.sigma2 > 0 else None},
        "phases_ms_per_step": {"fill": fill_ms, "fixup_estimate": phases[1] / n_timed,
                               "allocation": phases[2] / n_timed, "map": phases[3] / n_timed},
    }
    if w.precision == "f64":
        # FP64 sample path: the issue slots are FP64 instructions, which the
        # chip issues at half the FP32 rate
        out["roofline"]["note"] = "FP64 sample path; the issue count is the FP32 path's"
    if args.copy_calibration:
        out["copy_calibration_bytes"] = copy_calibration()
    if not args.no_cpu_baseline:
        if w.name == "gauss_prod_4d":
            out["cpu_baseline"] = cpu_baseline(w, w.n_eval, w.n_iter)     # the whole run
        else:
            out["cpu_baseline"] = cpu_baseline(w, int(args.cpu_evals), args.cpu_iters)
    v.close()
    return out


def warp_run(args, w, method: str, exact: float):
    """One method on the correlated Gaussian: create, the continuation
    warm-up, then iterations combined by Eq. 8-9 in chunks until the relative
    error estimate reaches the target or the caps.  The wall time counts from
    create.

    Plain VEGAS+: every warm-up iteration refines the map and the
    allocation, as do the combined iterations (Alg. 1).
    Warp: each warm-up step runs one plain iteration, which refines the map
    while the step's width is at least map_hold x the target's, and then
    cont_iters iterations through the warp, which train it (library starting
    weights, KL loss) and reallocate with the map held.  Then the map stays
    held; the warp keeps training, judged by cost against a plain control
    every 16th iteration."""
    import numpy as np
    import torch
    import vegas_inputs as vi
    from paper_2408_09229_amd import Vegas, make_config
    target = args.target
    sharp = w.name == "corr_gauss_16d"
    warm = vi.continuation(w, args.cont_steps) if sharp else [w.params] * w.n_adapt
    per = args.cont_iters if sharp else 1
    s_target = float(w.params[1])
    cap_it, cap_s = args.cap_iters, args.cap_seconds
    n_warm = len(warm) * (per + 1)
    cfg = make_config(w.dim, w.n_g, w.n_eval, precision="f32", seed=w.seed,
                      max_iter=n_warm + cap_it + args.steps + args.warmup + args.chunk + 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v = Vegas(cfg, w.family, warm[0])
    if method == "warp":
        v.attach_flow(None, lr=args.flow_lr, train=True, loss=args.flow_loss, judge=0,
                      steps_per_iter=args.flow_steps, train_stride=args.train_stride, init_seed=w.seed)
    for p in warm:
        v.set_params(p)
        if method == "warp":
            v.enable_flow(False)
            v.set_adapt(float(p[1]) >= args.map_hold * s_target, True)
            v.adapt(1)
            v.set_adapt(False, True)
            v.enable_flow(True)
            v.adapt(per)
        else:
            v.adapt(per + 1)
    if method == "warp":
        v.set_flow_config(lr=args.flow_lr_final, train=True, loss=args.flow_loss, judge="cost",
                          steps_per_iter=args.flow_steps_final, control_period=16, train_stride=args.train_stride)
    n0 = len(v.get_iterations()[0])
    n = 0
    rel = math.inf
    r = None
    while n < cap_it and time.perf_counter() - t0 < cap_s:
        v.integrate(args.chunk)
        n += args.chunk
        r = v.result(allow_nonfinite=True)
        rel = math.sqrt(r.sigma2) / abs(r.integral) if r.integral != 0 else math.inf
        if rel <= target:
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    I_all, s2_all = v.get_iterations()
    Ii, si = I_all[n0:], s2_all[n0:]
    kinds = v.flow_kinds()[n0:] if method == "warp" else np.zeros(len(Ii), np.int32)
    sel = kinds != 2
    sig = math.sqrt(r.sigma2)
    rec = {"iterations": n, "warmup_iterations": n0, "wall_s": wall, "reached": bool(rel <= target),
           "integral": r.integral, "sigma": sig, "rel_err_estimate": rel,
           "true_rel_err": abs(r.integral - exact) / exact, "z": (r.integral - exact) / sig if sig > 0 else None,
           "resolved": bool(sig > 0 and abs(r.integral - exact) < 3.0 * sig),
           "median_rel_var_per_eval": float(np.median(si[sel] / np.maximum(Ii[sel] ** 2, 1e-300) * w.n_eval)),
           "nonfinite_samples": int(r.n_nonfinite)}
    if method == "warp":
        on, kept, rej = v.flow_status()
        rec["judge"] = {"warp_on_at_end": on, "kept": kept, "rejected": rej,
                        "control_iterations": int(np.sum(kinds == 2)), "warped_iterations": int(np.sum(kinds == 1))}
    print(f"[bench] {method}: {json.dumps(rec)}", file=sys.stderr, flush=True)
    return v, rec


def run_warp_compare(args, w):
    """Learned warp against plain VEGAS+ (time to the target error), then the
    warped iteration's throughput over K timed iterations."""
    import torch
    from tests import closed_forms as cf
    exact = cf.exact(w)
    torch.cuda.set_device(0)
    out = {}
    vp, out["plain"] = warp_run(args, w, "plain", exact)
    vp.close()
    v, out["warp"] = warp_run(args, w, "warp", exact)
    # throughput of the warped iteration as the run left it: W more
    # iterations untimed, then K timed between events on the library's stream
    v.set_flow_config(lr=args.flow_lr_final, train=True, loss=args.flow_loss, judge="guard",
                      steps_per_iter=args.flow_steps_final, control_period=16, train_stride=args.train_stride)
    v.integrate(args.warmup)
    torch.cuda.synchronize()
    v.set_timing(True)
    v.set_flow_timing(True)
    st = v.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    v.integrate(args.steps)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kinds = v.flow_kinds()[-args.steps:]
    ft = v.flow_timing()
    v.close()
    # the warp's two MFMA kernels: the sampling pass over every sample (one
    # launch per warped iteration), and the gradient kernel (inverse pass
    # and every layer's backward pass) over 1/stride of them, once per Adam
    # step; the roofline line names the one with the most time per
    # iteration, at its own per-launch duration.  The whole training (one
    # sums launch, then two launches per Adam step) is reported beside them.
    samp_ms, train_ms, grad_ms = ft["sample_ms"], ft["train_ms"], ft["grad_launch_ms"]
    n_train = (w.n_eval + args.train_stride - 1) // args.train_stride
    kernels = {
        "k_flow_sample": (FLOW_SAMPLE_FLOPS * w.n_eval, samp_ms, 1),
        "k_flow_grad": (FLOW_TRAIN_FLOPS * n_train, grad_ms, args.flow_steps_final),
    }
    dom = max(kernels, key=lambda k: (kernels[k][1] or 0.0) * kernels[k][2])
    flops, dom_ms, _ = kernels[dom]
    ach = flops / (dom_ms / 1e3) if dom_ms else None
    phases = {k: {"ms_per_launch": m, "launches_per_iteration": n,
                  "tflops": (f / (m / 1e3) / 1e12) if m else None,
                  "frac": (f / (m / 1e3) / 2.5e15) if m else None} for k, (f, m, n) in kernels.items()}
    tf = FLOW_TRAIN_FLOPS * n_train * args.flow_steps_final
    phases["training (per iteration: k_flow_sumsq once, then k_flow_grad and k_flow_update per Adam step)"] = {"ms": train_ms, "tflops": (tf / (train_ms / 1e3) / 1e12) if train_ms else None,
                                "frac": (tf / (train_ms / 1e3) / 2.5e15) if train_ms else None}
    pl, wp = out["plain"], out["warp"]
    line = {
        "metric": "integrand evals/sec and wall time to 1e-4 rel. error; learned warp vs plain VEGAS+",
        "value": w.n_eval * args.steps / (ms / 1e3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {WORKLOADS[w.name]}, {w.n_eval:.0e} evals/iteration; learned warp "
                               f"4 affine coupling layers in Gaussian coordinates, 2x64 BF16 MLPs",
                   "n_eval": w.n_eval, "dim": w.dim, "n_intervals": w.n_g, "target_rel_err": args.target,
                   "caps": {"iterations": args.cap_iters, "seconds": args.cap_seconds},
                   "warmup": f"continuation over {args.cont_steps} steps (plain: {args.cont_iters + 1} "
                             f"iterations each; warp: 1 plain refining the map while the width is >= "
                             f"{args.map_hold} x the target's, then {args.cont_iters} warped)",
                   "warp": {"lr": args.flow_lr, "adam_steps_per_iteration": args.flow_steps,
                            "lr_final": args.flow_lr_final, "adam_steps_per_iteration_final": args.flow_steps_final,
                            "train_stride": args.train_stride, "loss": args.flow_loss, "control_period": 16,
                            "map_hold": args.map_hold},
                   "parallelism": "single-gpu"},
        "time_to_target_s": {"warp": wp["wall_s"] if wp["reached"] else None,
                             "plain": pl["wall_s"] if pl["reached"] else None},
        "exact": exact,
        "comparison": out,
        "timed_iterations": {"warped": int((kinds == 1).sum()), "control": int((kinds == 2).sum()),
                             "plain": int((kinds == 0).sum())},
        "roofline": {"bound": "mfma", "achieved": ach / 1e12 if ach else None, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": ach / 2.5e15 if ach else None,
                     "traffic": profiled_traffic(w.name, "k_flow", FLOW_SOURCES, kernel=dom), "kernel": dom,
                     "kernel_ms": dom_ms, "flops_per_launch": flops, "phases": phases},
    }
    if args.copy_calibration:
        line["copy_calibration_bytes"] = copy_calibration()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_warp(w, args.train_stride, args.flow_steps_final)
    return line


def subrecords(args):
    """The other workloads in the same run, one record each."""
    import vegas_inputs as vi
    subs = {}
    for name in ("gauss_prod_4d", "gauss3_8d", "ridge_4d"):
        w = getattr(vi, name)()
        a = argparse.Namespace(**vars(args))
        a.steps, a.warmup = (w.n_iter, 0) if name == "gauss_prod_4d" else (args.sub_steps, 2)
        subs[name] = run_single(a, w)
    a = argparse.Namespace(**vars(args))
    a.steps, a.warmup = vi.BATCH_ITER, vi.BATCH_ADAPT
    subs["genz_batch"] = run_batch(a)
    return subs


# --------------------------------------------------------------------------
# the paper's own measurements (--study NAME): one JSON line per point
# --------------------------------------------------------------------------
STUDY_ITERS = 20          # max_it of the paper's configurations (Tab. 2)


def _emit(rec):
    print(json.dumps(rec), flush=True)


def _config_of(w, n_g=None, alpha=None, beta=None, precision=None, max_iter=0):
    from paper_2408_09229_amd import make_config
    return make_config(w.dim, n_g or w.n_g, w.n_eval, alpha=w.alpha if alpha is None else alpha,
                       beta=w.beta if beta is None else beta, seed=w.seed,
                       precision=precision or w.precision, max_iter=max_iter)


def study_phases(args):
    """Tab. 1: where a whole run's time goes, for Roos & Arnold (10-d) and the
    ridge of Tab. 3 (4-d), at 1e7 .. 1e10 integrand evaluations in all, with
    the "def" parameters (1024 intervals, alpha 0.5, beta 0.75, 20
    iterations, none skipped).  Phases: init (create: workspace, uniform map
    and allocation, first offsets), fill, results (tile fix-up and the
    iteration's estimate), allocation (new n_h and the sample offsets, the
    paper's update of evals per cube and its mapping of evaluations to
    cubes), map (rebinning), host (launch gaps and the combination), clear
    (destroy).  GPU phases come from HIP events around each kernel group;
    host phases from the host clock around the calls.  A first untimed run
    of each shape loads the kernels, as the paper leaves out the context
    start-up."""
    import torch
    import vegas_inputs as vi
    from paper_2408_09229_amd import Vegas
    from tests import closed_forms as cf
    torch.cuda.set_device(0)
    totals = [float(x) for x in args.study_totals.split(",")]
    for w0 in (vi.roos_10d(), vi.ridge_tab3()):
        for prec in args.study_precisions.split(","):
            for total in totals:
                w = w0.with_(n_eval=int(total / STUDY_ITERS), precision=prec)
                cfg = _config_of(w)
                for rep in range(2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    v = Vegas(cfg, w.family, w.params, w.lo, w.hi)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    v.set_timing(True)
                    v.integrate(STUDY_ITERS)
                    r = v.result()
                    torch.cuda.synchronize()
                    t2 = time.perf_counter()
                    ph, n = v.get_timing()
                    v.close()
                    torch.cuda.synchronize()
                    t3 = time.perf_counter()
                if n != STUDY_ITERS:
                    raise RuntimeError(f"timed {n} iterations, expected {STUDY_ITERS}")
                ms = {"init": (t1 - t0) * 1e3, "fill": ph[0], "results": ph[1], "allocation": ph[2], "map": ph[3]}
                ms["host"] = max((t2 - t1) * 1e3 - float(ph.sum()), 0.0)
                ms["clear"] = (t3 - t2) * 1e3
                tot = sum(ms.values())
                exact = cf.exact(w)
                _emit({"study": "phases", "integrand": w0.name, "precision": prec, "evals_total": total,
                       "n_eval": w.n_eval, "iterations": STUDY_ITERS, "total_ms": tot,
                       "percent": {k: 100.0 * x / tot for k, x in ms.items()}, "ms": ms,
                       "integral": r.integral, "sigma": math.sqrt(r.sigma2), "exact": exact})


def study_scaling(args):
    """Tab. 6 / the fill-scaling figure: the fill kernel's time per iteration
    (mean, standard error, min, max over the iterations of a run) while one
    parameter moves and the others stay at 8 dimensions, 1024 intervals and
    2e10 evaluations in all (1e9 per iteration over 20 iterations).  The
    integrand is Roos & Arnold (the paper does not name the one it used).
    Dimensions stop at 16, the library's limit (the paper goes to 32).  The
    paper's fourth axis, its thread count, has no counterpart: the fill
    here runs one persistent workgroup per CU over sample tiles whose size
    follows from the budget."""
    import numpy as np
    import torch
    import vegas_inputs as vi
    from paper_2408_09229_amd import Vegas
    torch.cuda.set_device(0)
    base = {"evals_total": 2e10, "dim": 8, "n_g": 1024}
    # the paper's dimension axis ends at 32; the library takes at most 16
    axes = {"evals_total": [2e6, 2e7, 2e8, 2e9, 2e10], "dim": [2, 4, 8, 12, 16],
            "n_g": [16, 64, 256, 1024, 4096]}
    iters = args.study_iters
    for axis, values in axes.items():
        for val in values:
            p = dict(base, **{axis: val})
            w = vi.roos_10d().with_(dim=int(p["dim"]), n_g=int(p["n_g"]), n_eval=int(p["evals_total"] / STUDY_ITERS),
                                    precision=args.study_precisions.split(",")[0])
            w = w.with_(lo=np.zeros(w.dim), hi=np.ones(w.dim))
            v = Vegas(_config_of(w), w.family, w.params, w.lo, w.hi)
            v.set_timing(True)
            v.adapt(1)
            per = []
            prev = v.get_timing()[0][0]
            for _ in range(iters):
                v.adapt(1)
                cur = v.get_timing()[0][0]
                per.append(cur - prev)
                prev = cur
            v.close()
            a = np.array(per)
            _emit({"study": "scaling", "axis": axis, "value": val, "dim": w.dim, "n_g": w.n_g, "n_eval": w.n_eval,
                   "precision": w.precision, "fill_ms_mean": float(a.mean()),
                   "fill_ms_stderr": float(a.std(ddof=1) / math.sqrt(len(a))) if len(a) > 1 else 0.0,
                   "fill_ms_min": float(a.min()), "fill_ms_max": float(a.max()), "iterations": len(a),
                   "evals_per_s": w.n_eval / (a.mean() * 1e-3)})


PARAM_SETS = {"def": {"n_g": 1024, "alpha": 0.5}, "vf": {"n_g": 50, "alpha": 1.5}, "tq": {"n_g": None, "alpha": 0.5}}


def tq_intervals(n_eval: int) -> int:
    """The "tq" set's interval count "computed on n_eval" (Tab. 2), which the
    paper does not spell out: read here as one interval per 1000 evaluations,
    kept within 2 .. 1024."""
    return max(2, min(1024, n_eval // 1000))


def study_accuracy(args):
    """The test-integrand comparison: wall time against relative standard
    error for Tab. 3's integrands #1-7 at their dimensions, under the def,
    vf and tq parameter sets (Tab. 2: 20 iterations, none skipped, beta
    0.75), at several budgets.  Each point is the mean over five runs after
    an untimed one; the summary line per set and budget is the geometric
    mean over the seven integrands, as the paper plots it."""
    import numpy as np
    import torch
    import vegas_inputs as vi
    from paper_2408_09229_amd import Vegas
    from tests import closed_forms as cf
    torch.cuda.set_device(0)
    budgets = [float(x) for x in args.study_budgets.split(",")]
    for set_name in args.study_sets.split(","):
        ps = PARAM_SETS[set_name]
        for total in budgets:
            n_eval = int(total / STUDY_ITERS)
            n_g = ps["n_g"] or tq_intervals(n_eval)
            per = []
            for w0 in vi.tab3_suite():
                w = w0.with_(n_eval=n_eval, n_g=n_g, alpha=ps["alpha"], beta=0.75,
                             precision=args.study_precisions.split(",")[0])
                exact = cf.exact(w)
                walls, rels, zs = [], [], []
                for rep in range(6):
                    w_rep = w.with_(seed=rep)
                    cfg = _config_of(w_rep)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    v = Vegas(cfg, w.family, w.params, w.lo, w.hi)
                    v.integrate(STUDY_ITERS)
                    r = v.result()
                    v.close()
                    torch.cuda.synchronize()
                    if rep == 0:
                        continue
                    walls.append(time.perf_counter() - t0)
                    sig = math.sqrt(r.sigma2)
                    rels.append(sig / abs(r.integral))
                    zs.append((r.integral - exact) / sig if sig > 0 else 0.0)
                rec = {"study": "accuracy", "set": set_name, "integrand": w0.name, "dim": w.dim, "n_g": n_g,
                       "alpha": ps["alpha"], "evals_total": total, "wall_s": float(np.mean(walls)),
                       "rel_std_err": float(np.mean(rels)), "max_abs_z": float(np.max(np.abs(zs)))}
                _emit(rec)
                per.append(rec)
            _emit({"study": "accuracy_geomean", "set": set_name, "evals_total": total, "n_g": n_g,
                   "wall_s": float(np.exp(np.mean(np.log([p["wall_s"] for p in per])))),
                   "rel_std_err": float(np.exp(np.mean(np.log([p["rel_std_err"] for p in per])))),
                   "max_abs_z": float(max(p["max_abs_z"] for p in per))})


def study_beta(args):
    """Adaptive stratification on and off: beta 0.25 against beta 0 with
    alpha 1.5 and 500 intervals, 20 iterations of which the first 5 are not
    combined, wall time against relative standard error at several budgets;
    mean over five runs after an untimed one.  Integrands: the Tab. 3 ridge
    and Gaussian (peaked), Roos & Arnold and the cosine (smooth)."""
    import numpy as np
    import torch
    import vegas_inputs as vi
    from paper_2408_09229_amd import Vegas
    from tests import closed_forms as cf
    torch.cuda.set_device(0)
    budgets = [float(x) for x in args.study_budgets.split(",")]
    suite = {w.name: w for w in vi.tab3_suite()}
    for w0 in (vi.ridge_tab3(), suite["gauss4"], suite["roos10"], suite["cosine10"]):
        for beta in (0.25, 0.0):
            for total in budgets:
                n_eval = int(total / STUDY_ITERS)
                w = w0.with_(n_eval=n_eval, n_g=500, alpha=1.5, beta=beta,
                             precision=args.study_precisions.split(",")[0])
                exact = cf.exact(w)
                walls, rels, errs = [], [], []
                for rep in range(6):
                    cfg = _config_of(w.with_(seed=rep))
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    v = Vegas(cfg, w.family, w.params, w.lo, w.hi)
                    v.adapt(5)
                    v.integrate(STUDY_ITERS - 5)
                    r = v.result()
                    v.close()
                    torch.cuda.synchronize()
                    if rep == 0:
                        continue
                    walls.append(time.perf_counter() - t0)
                    rels.append(math.sqrt(r.sigma2) / abs(r.integral))
                    errs.append(abs(r.integral - exact) / abs(exact))
                _emit({"study": "beta", "integrand": w0.name, "beta": beta, "evals_total": total,
                       "wall_s": float(np.mean(walls)), "rel_std_err": float(np.mean(rels)),
                       "true_rel_err": float(np.mean(errs))})


def study_applications(args):
    """The application integrands (Sec. 4.5-4.6) compiled at run time: the
    Asian call (8 normal variates) and the harmonic-oscillator path integral
    (N = 8 lattice spacings, T = 4, ends at 0; 7 interior points on
    [-5, 5]^7), in FP64 with the "def" parameters (1024 intervals, alpha 0.5,
    beta 0.75, 20 iterations, none skipped); wall time (create to result)
    against relative standard error at several budgets, the mean over five
    runs after an untimed one, and the hipRTC compile time of each source."""
    import numpy as np
    import torch
    from paper_2408_09229_amd import UserIntegrand, Vegas, make_config
    from paper_2408_09229_amd import integrands as itg
    from tests import closed_forms as cf
    torch.cuda.set_device(0)
    budgets = [float(x) for x in args.study_budgets.split(",")]
    lo_f, hi_f = itg.feynman_box(8)
    cases = [("asian_call8", itg.ASIAN_CALL, 8, itg.asian_params(), np.zeros(8), np.ones(8),
              cf.asian_call(itg.asian_params(), 8)),
             ("feynman_ho7", itg.FEYNMAN_HO, 7, itg.feynman_params(0.0, 4.0, 8), lo_f, hi_f,
              cf.feynman_ho(itg.feynman_params(0.0, 4.0, 8), 7))]
    for name, src, dim, params, lo, hi, exact in cases:
        t0 = time.perf_counter()
        fn = UserIntegrand(src, dim, "f64")
        compile_ms = (time.perf_counter() - t0) * 1e3
        for total in budgets:
            n_eval = int(total / STUDY_ITERS)
            walls, rels, errs = [], [], []
            for rep in range(6):
                cfg = make_config(dim, 1024, n_eval, alpha=0.5, beta=0.75, seed=rep, precision="f64")
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                v = Vegas(cfg, 0, params, lo, hi, user=fn)
                v.integrate(STUDY_ITERS)
                r = v.result()
                v.close()
                torch.cuda.synchronize()
                if rep == 0:
                    continue
                walls.append(time.perf_counter() - t0)
                rels.append(math.sqrt(r.sigma2) / abs(r.integral))
                errs.append(abs(r.integral - exact) / abs(exact))
            _emit({"study": "applications", "integrand": name, "dim": dim, "evals_total": total,
                   "compile_ms": compile_ms, "wall_s": float(np.mean(walls)), "rel_std_err": float(np.mean(rels)),
                   "true_rel_err": float(np.mean(errs)), "exact": exact})
        fn.close()


STUDIES = {"phases": study_phases, "scaling": study_scaling, "accuracy": study_accuracy, "beta": study_beta,
           "applications": study_applications}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="headline", choices=["headline"] + sorted(WORKLOADS))
    ap.add_argument("--n-eval", type=float, default=0, help="override evals/iteration (0: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sub", action="store_true", help="headline: skip the other workloads' records")
    ap.add_argument("--sub-steps", type=int, default=20, help="timed iterations of the d=8 and ridge records")
    ap.add_argument("--cpu-evals", type=float, default=1.5e7)
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--issue-rates", action="store_true",
                    help="only measure the issue rates of the VALU instruction kinds the path uses and the "
                         "LDS atomic add rates")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (for scaling HBM counters)")
    ap.add_argument("--tune-cache", default="", help="autotuner cache of the batched workload")
    ap.add_argument("--target", type=float, default=1e-4, help="warp comparison: relative error target")
    ap.add_argument("--cap-iters", type=int, default=2000, help="warp comparison: iteration cap per method")
    ap.add_argument("--cap-seconds", type=float, default=600.0, help="warp comparison: time cap per method")
    ap.add_argument("--chunk", type=int, default=5, help="warp comparison: iterations between error checks")
    ap.add_argument("--cont-steps", type=int, default=30, help="warp comparison: continuation steps")
    ap.add_argument("--cont-iters", type=int, default=2, help="warp comparison: iterations per step")
    ap.add_argument("--flow-lr", type=float, default=2e-3, help="warp comparison: Adam step during the warm-up")
    ap.add_argument("--flow-steps", type=int, default=16, help="warp comparison: Adam steps per warm-up iteration")
    ap.add_argument("--flow-lr-final", type=float, default=1e-3, help="warp comparison: Adam step afterwards")
    ap.add_argument("--flow-steps-final", type=int, default=12,
                    help="warp comparison: Adam steps per combined iteration")
    ap.add_argument("--train-stride", type=int, default=32,
                    help="warp comparison: a training step uses every n-th sample of the iteration")
    ap.add_argument("--flow-loss", default="kl", choices=["variance", "kl"], help="warp comparison: training loss")
    ap.add_argument("--study", default="", choices=[""] + sorted(STUDIES),
                    help="one of the paper's measurements instead of the benchmark (JSON lines)")
    ap.add_argument("--study-totals", default="1e7,1e8,1e9,1e10", help="phases: evaluations in all (20 iterations)")
    ap.add_argument("--study-budgets", default="1e6,1e7,1e8,1e9",
                    help="accuracy / beta: evaluations in all (20 iterations)")
    ap.add_argument("--study-sets", default="def,vf,tq", help="accuracy: parameter sets")
    ap.add_argument("--study-precisions", default="f32,f64", help="sample-path precisions (scaling, accuracy and "
                    "beta take the first)")
    ap.add_argument("--study-iters", type=int, default=10, help="scaling: timed iterations per point")
    ap.add_argument("--seed", type=int, default=-1, help="warp comparison: sampling and warp seed (-1: the workload's)")
    ap.add_argument("--map-hold", type=float, default=2.0,
                    help="warp comparison: the map refines while the warm-up width is >= this x the target's")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the VEGAS+ path here "
              "runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.issue_rates:
        import ctypes
        lib = ctypes.CDLL(os.path.join(ROOT, "paper_2408_09229_amd", "libvegas_issue_rates.so"))
        out = (ctypes.c_double * 8)()
        torch.cuda.set_device(0)
        assert lib.vegas_issue_rates(out, 8, ctypes.c_double(2.4), 1024) == 0
        names = ["fma_f32", "mul+exp2_f32", "mad_u64_u32+xor", "fma_f64", "bitop3", "add_f64+rcp_f64",
                 "exp2_f32", "exp2_f32:fma_f32 1:3 independent"]
        rates = {n: round(v, 3) for n, v in zip(names, out)}
        lds = (ctypes.c_double * 6)()
        assert lib.vegas_lds_atomic_rates(lds, ctypes.c_double(2.4), 256) == 0
        lnames = ["ds_add_u32", "ds_add_f32", "ds_add_f64"]
        rates["lds_atomic_adds_per_cu_cycle"] = {
            "conflict_free": {n: round(lds[i], 2) for i, n in enumerate(lnames)},
            "random_1024": {n: round(lds[3 + i], 2) for i, n in enumerate(lnames)}}
        print(json.dumps(rates))
        return

    if args.study:
        STUDIES[args.study](args)
        return

    import vegas_inputs as vi
    if args.workload == "headline":
        w = vi.corr_gauss_16d()
        if args.seed >= 0:
            w = w.with_(seed=args.seed)
        line = run_warp_compare(args, w)
        if not args.no_sub:
            line["sub_records"] = subrecords(args)
        print(json.dumps(line), flush=True)
        return
    if args.workload == "genz_batch":
        print(json.dumps(run_batch(args)), flush=True)
        return
    w = getattr(vi, args.workload)()
    if args.workload in ("corr_gauss_16d", "corr_gauss_16d_mild"):
        if args.seed >= 0:
            w = w.with_(seed=args.seed)
        print(json.dumps(run_warp_compare(args, w)), flush=True)
        return
    if args.n_eval:
        w = w.with_(n_eval=int(args.n_eval))
    print(json.dumps(run_single(args, w)), flush=True)


if __name__ == "__main__":
    main()
