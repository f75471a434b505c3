"""Benchmark: bins x (NLL + gradient) per second on one MI355X.

Workload: a 1D histogram of 1e7 bins on [0,100] with two Gaussian peaks
(amplitudes 1e3..1e5, means in [10,90], widths 0.5..3) on a cubic
background, Poisson counts; one step is one nll_grad call (NLL and the
10-component reverse-mode gradient over every bin, FP64 accumulation).
Eight distinct histograms (320 MB, more than the 256 MB last-level cache)
are visited in turn so every step reads its counts from HBM.

The K timed steps are replayed from a captured HIP graph (so host launch
overhead stays out of the kernel timing) between HIP events recorded on the
stream the kernels run on.  One JSON line is printed.

The CPU baseline times the FP64 oracle (test infrastructure) on the host on
one full histogram, repeated for ~10 s.

The same line also carries the metric's second half (unless --hot-only):
  fits        4096 uneven histograms fitted by one autotuned, graph-replayed
              fit_batch launch from the plain method's starts; fits/s agreeing
              with the FP64-bin fit within 1e-6, and the oracle's fitter on
              the host as its CPU baseline;
  learned     the learned initialiser trained on --train-fits plain fits, then
              plain vs learned starts on that batch at the same launch shape
              (HIP events, median of 5); a learned fit counts only where its
              NLL is within 1e-6 of the plain fit's;
  single_fit  the 10,000-bin single fit (at most 200 BFGS iterations, to
              EDM < 1e-10), Poisson and Neyman, beside the oracle's fitter.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NBINS = 10_000_000
NCOPIES = 8
HBM_PEAK_GBS = 8000.0
FP64_VEC_PEAK_TFLOPS = 78.6

# Algorithmic FP64 flops per bin of the timed workload (two Gaussians, cubic
# background, Poisson objective, value + 10-component gradient), counting
# +, -, * as one flop and a fused multiply-add as two; the elementary
# functions are counted at the flops of a textbook FP64 evaluation
# (exp: Cody-Waite reduction + degree-11 polynomial = 26; log: reduction +
# degree-8 polynomial in s^2 with s = f/(2+f) = 30 including its division;
# division: reciprocal + two Newton steps + residual correction = 10).
FLOPS_BASIC = 49
FLOPS_EXP, FLOPS_LOG, FLOPS_DIV = 26, 30, 10
FLOPS_PER_BIN = FLOPS_BASIC + 2 * FLOPS_EXP + FLOPS_LOG + FLOPS_DIV
BYTES_PER_BIN = 4  # one u32 count per bin


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "nll_grad_1e7_traffic.json")


# Sources of the timed 1D kernel and of its launch (grid sizing in abi.cpp).
KERNEL_SOURCES = ("device.hpp", "fastmath.hpp", "chunk.hpp", "nll_kernels.hpp", "nll1d_ng2.hip",
                  "finish.hpp", "finish.hip", "abi.cpp")
HOT_KERNEL = {"fp64": "void hf::k_nll_1d<2, 3, 2, true, false>(hf::NllArgs)",
              "fp32bin": "void hf::k_nll_1d<2, 3, 2, true, true>(hf::NllArgs)"}


def kernel_source_hash():
    """Hash of the HIP sources the timed kernel is built from; HBM traffic
    measured with rocprofv3 counters is only reported for the same sources."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2203_06139_amd", "csrc", name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def summarize_traffic(fetch_csv, write_csv, calib_mib, precision, objective, command):
    """Turns two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE, with --copy-calibration) into the traffic summary the bench
    line reports: each counter's mean KiB per dispatch of the timed kernel,
    scaled by true / counted bytes of the calibration copies."""
    import csv

    def read(path, counter):
        kern, copies = [], []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"])
                if r["Kernel_Name"] == HOT_KERNEL[precision]:
                    kern.append(v)
                elif r["Kernel_Name"] == "__amd_rocclr_copyBuffer":
                    copies.append((int(r["Grid_Size"]), v))
        if not kern or not copies:
            raise SystemExit("%s: no %s rows for the kernel or the copies" % (path, counter))
        big = max(g for g, _ in copies)
        cal = [v for g, v in copies if g == big][-4:]
        return sum(kern) / len(kern), sum(cal) / len(cal), len(kern)

    true_kib = calib_mib * 1024.0
    fk, fc, nf = read(fetch_csv, "FETCH_SIZE")
    wk, wc, nw = read(write_csv, "WRITE_SIZE")
    fscale, wscale = true_kib / fc, true_kib / wc
    fetch_b, write_b = fk * 1024.0 * fscale, wk * 1024.0 * wscale
    out = {"kernel": HOT_KERNEL[precision], "source_hash": kernel_source_hash(),
           "commands": [command], "fetch_scale": fscale, "write_scale": wscale,
           "fetch_kib_raw": fk, "write_kib_raw": wk, "dispatches": [nf, nw],
           "per_launch_bytes": {"%s/%s" % (precision, objective): int(round(fetch_b + write_b))},
           "fetch_bytes": int(round(fetch_b)), "write_bytes": int(round(write_b)),
           "note": "FETCH_SIZE/WRITE_SIZE per dispatch x calibration scale"}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def measured_traffic(precision, objective):
    """Bytes per launch (fetch + write) from the committed counter summary,
    or None when the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    key = "%s/%s" % (precision, objective)
    if t.get("source_hash") != kernel_source_hash() or key not in t.get("per_launch_bytes", {}):
        return None
    return t["per_launch_bytes"][key]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(case, obj, seconds=10.0):
    import oracle
    spec = case["spec"]
    m = oracle.Model(spec["kind"], spec["n_gauss"], spec["poly_degree"], spec["t_shift"],
                     spec["t_scale"])
    cores = cpu_cores()
    reps, t0 = 0, time.perf_counter()
    ref = None
    while True:
        ref = oracle.nll_grad(m, obj, case["counts"], case["theta_eval"], case["range"],
                              nthreads=cores)
        reps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return ref, dict(value=reps * NBINS / dt, unit="bins*(NLL+grad)/s", cores=cores,
                     kind="oracle",
                     sample="%d full passes over one 1e7-bin histogram in %.1f s, %d threads"
                     % (reps, dt, cores))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--precision", choices=["fp64", "fp32bin"], default="fp64")
    ap.add_argument("--objective", choices=["poisson", "neyman", "pearson"], default="poisson")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--hot-only", action="store_true",
                    help="default workload: time the 1e7-bin NLL + gradient only, without the "
                         "fits, learned-initialiser and single-fit sections")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--train-fits", type=int, default=1_000_000,
                    help="learned workload: plain fits the initialiser is trained on")
    ap.add_argument("--epochs", type=int, default=8, help="learned workload: training epochs")
    ap.add_argument("--workload", choices=["large1d", "hist2d", "fits", "smallfits", "learned",
                                           "gradient", "fisher", "gradmap", "unbinned", "binavg",
                                           "edges"],
                    default="large1d",
                    help="large1d: the 1e7-bin NLL+gradient (default); hist2d: 2048^2 weighted "
                         "NLL+gradient+weight gradient; fits: 4096 uneven histograms fitted by "
                         "fit_batch; smallfits: 16384 histograms of 128..1024 bins, with and "
                         "without one wave per histogram; learned: plain vs "
                         "learned-initialiser fits of the 4096 batch; "
                         "gradient: fits with the reverse-mode gradient vs central differences "
                         "for 1..4 Gaussians; fisher: the expected Hessian of the 1e7-bin "
                         "workload (and of the 2048^2 one); gradmap: the elementwise Gaussian "
                         "gradient of 2^27 parameter sets; unbinned: the extended unbinned "
                         "NLL + gradient of 1e7 events; binavg: the 1e7-bin NLL + gradient "
                         "with the model averaged over each bin; edges: the same on 1e7 bins "
                         "of varying widths")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic summary from two rocprofv3 --pmc counter CSVs of a "
                         "run with --copy-calibration (no GPU work)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after timing, copy a MIB-sized device buffer 4 times (a plain "
                         "copy of known size to scale HBM counters against)")
    args = ap.parse_args()
    if args.summarize_traffic:
        # the profiled run is this script with the same flags
        cmd = ("python bench.py --steps %d --warmup %d --no-cpu-baseline --copy-calibration %d "
               "--precision %s --objective %s" % (args.steps, args.warmup, args.copy_calibration,
                                                  args.precision, args.objective))
        summarize_traffic(args.summarize_traffic[0], args.summarize_traffic[1],
                          args.copy_calibration, args.precision, args.objective, cmd)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: the histogram objective is not sharded across GPUs "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_2203_06139_amd as hf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.workload == "hist2d":
        return bench_hist2d(args, hf, datagen, np, torch, dev)
    if args.workload == "fits":
        return bench_fits(args, hf, datagen, np, torch, dev)
    if args.workload == "smallfits":
        return bench_smallfits(args, hf, datagen, np, torch, dev)
    if args.workload == "learned":
        return bench_learned(args, hf, datagen, np, torch, dev)
    if args.workload == "gradient":
        return bench_gradient(args, hf, datagen, np, torch, dev)
    if args.workload == "fisher":
        return bench_fisher(args, hf, datagen, np, torch, dev)
    if args.workload == "gradmap":
        return bench_gradmap(args, hf, np, torch, dev)
    if args.workload == "unbinned":
        return bench_unbinned(args, hf, datagen, np, torch, dev)
    if args.workload == "binavg":
        return bench_binavg(args, hf, datagen, np, torch, dev)
    if args.workload == "edges":
        return bench_binavg(args, hf, datagen, np, torch, dev, edges=True)
    obj = {"poisson": hf.POISSON, "neyman": hf.NEYMAN, "pearson": hf.PEARSON}[args.objective]
    prec = hf.FP64 if args.precision == "fp64" else hf.FP32_BIN

    log("generating %d histograms of %d bins" % (NCOPIES, NBINS))
    hists, thetas, cases = [], [], []
    for k in range(NCOPIES):
        c = datagen.large_fit_case(seed=20 + k, nbins=NBINS)
        cases.append(c)
        hists.append(hf.make_hist(c["counts"], c["range"], device=dev))
        thetas.append(torch.as_tensor(c["theta_eval"], dtype=torch.float64, device=dev))
    model = hf.Model.from_spec(cases[0]["spec"])
    P = model.nparams
    nll_out = [torch.empty(1, dtype=torch.float64, device=dev) for _ in range(NCOPIES)]
    grad_out = [torch.empty(P, dtype=torch.float64, device=dev) for _ in range(NCOPIES)]

    def step(k):
        j = k % NCOPIES
        hf.nll_grad(hists[j], model, thetas[j], objective=obj, precision=prec,
                    nll_out=nll_out[j], grad_out=grad_out[j])

    log("warmup %d" % args.warmup)
    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()

    # K steps = full replays of a 32-step graph + one replay of a remainder graph
    steps = args.steps
    per_graph = min(NCOPIES * 4, steps)
    graphs = []  # (graph, replays)
    if not args.no_graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        for count, replays in ((per_graph, steps // per_graph), (steps % per_graph, 1)):
            if count == 0 or replays == 0:
                continue
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(side):
                with torch.cuda.graph(g, stream=side):
                    for k in range(count):
                        step(k)
            graphs.append((g, replays))
        torch.cuda.synchronize()
        for g, _ in graphs:
            g.replay()  # untimed replay
        torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_host = time.perf_counter()
    ev0.record(stream)
    if graphs:
        for g, replays in graphs:
            for _ in range(replays):
                g.replay()
    else:
        for k in range(steps):
            step(k)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / steps
    value = NBINS / (ms_per_step * 1e-3)
    log("timed %d steps: %.3f ms total, %.2f us/step (host %.3f s)"
        % (steps, ms, 1e3 * ms_per_step, t_host))

    # parity of the timed configuration against the oracle on copy 0
    result = dict(
        metric="bins*(NLL+grad)/s",
        value=value,
        unit="bins/s",
        n_gpus=1,
        steps=steps,
        warmup=args.warmup,
        ms_per_step=ms_per_step,
        higher_is_better=True,
        scaling="weak",
        vs_baseline=None,
        dtype="f64" if prec == hf.FP64 else "f32-bin/f64-acc",
        data="synthetic",
        config=dict(workload="1D histogram, 1e7 bins on [0,100], two Gaussians + cubic "
                             "background (10 parameters), %s NLL + reverse-mode gradient, "
                             "%s bins, 8 rotating histograms" % (args.objective, args.precision),
                    nbins=NBINS, params=P, objective=args.objective,
                    precision=args.precision, graph=bool(graphs)),
    )
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 4 x %d MiB device-to-device" % args.copy_calibration)
    flops = FLOPS_PER_BIN * NBINS
    achieved = flops / (ms_per_step * 1e-3) / 1e12
    traffic = measured_traffic(args.precision, args.objective)
    result["roofline"] = dict(bound="alu", achieved=achieved, peak=FP64_VEC_PEAK_TFLOPS,
                              unit="TFLOP/s", frac=achieved / FP64_VEC_PEAK_TFLOPS, traffic=traffic,
                              flops_per_bin=FLOPS_PER_BIN,
                              timed="one call: the main kernel and its finishing kernel",
                              hbm_gbs=BYTES_PER_BIN * NBINS / (ms_per_step * 1e-3) / 1e9,
                              hbm_frac=BYTES_PER_BIN * NBINS / (ms_per_step * 1e-3) / 1e9 /
                              HBM_PEAK_GBS)
    torch.cuda.synchronize()
    j0 = 0
    g_nll = nll_out[j0].item()
    g_grad = grad_out[j0].cpu().numpy()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        ref, cb = cpu_baseline(cases[j0], obj)
        result["cpu_baseline"] = cb
        tol = 1e-10 if prec == hf.FP64 else 1e-5
        err_nll = abs(g_nll - ref.nll) / ref.scales[0]
        err_grad = float(np.max(np.abs(g_grad - ref.grad) / ref.scales[1:]))
        result["parity"] = dict(rel_err_nll=err_nll, rel_err_grad=err_grad, tol=tol,
                                ok=bool(err_nll <= tol and err_grad <= tol))
        result["cpu_baseline"]["host"] = host_cpu()
    if not args.hot_only:
        # the metric's second half: fits/s of the batched fitter, plain vs
        # learned starts, and the single plain fit
        log("fits section")
        fits, batch = fits_section(hf, datagen, np, torch, dev, hf.FP32_BIN, args.steps,
                                   cpu=not args.no_cpu_baseline)
        result["fits"] = fits
        log("learned section")
        result["learned"] = learned_section(hf, np, torch, dev, batch, args.train_fits,
                                            args.epochs)
        log("single-fit section")
        result["single_fit"] = single_fit_section(hf, datagen, np, torch, dev,
                                                  cpu=not args.no_cpu_baseline)
        log("gradient section")
        rows, per_call = gradient_section(hf, datagen, np, torch, dev)
        result["gradient"] = dict(
            metric="fit time, central-difference over reverse-mode gradient, same fits",
            speedup_by_gaussians={str(r["gaussians"]): r["speedup"] for r in rows},
            sweep=rows, per_call=per_call, paper_context=PAPER_CONTEXT)
    print(json.dumps(result), flush=True)


def time_graph(torch, step, steps):
    """Time exactly `steps` calls of step(k) replayed from HIP graphs; returns ms per call."""
    per_graph = min(32, steps)
    graphs = []
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for count, replays in ((per_graph, steps // per_graph), (steps % per_graph, 1)):
        if count == 0 or replays == 0:
            continue
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                for k in range(count):
                    step(k)
        graphs.append((g, replays))
    torch.cuda.synchronize()
    for g, _ in graphs:
        g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for g, replays in graphs:
        for _ in range(replays):
            g.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def bench_hist2d(args, hf, datagen, np, torch, dev):
    """2048^2 weighted Poisson NLL + theta gradient + per-bin weight gradient
    (the backward of the differentiable objective), 12 bytes per bin."""
    c = datagen.hist2d_case()
    h = hf.make_hist(c["counts"], (0.0, 1.0), (0.0, 1.0), weights=c["weights"], device=dev)
    th = torch.as_tensor(c["theta_eval"], dtype=torch.float64, device=dev)
    m = hf.Model(hf.GAUSS2D)
    seed = torch.ones(1, dtype=torch.float64, device=dev)
    nll = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(7, dtype=torch.float64, device=dev)
    gw = torch.empty(c["counts"].shape, dtype=torch.float32, device=dev)
    prec = hf.FP64 if args.precision == "fp64" else hf.FP32_BIN

    def step(k):
        hf.nll_grad(h, m, th, objective=hf.POISSON, precision=prec, seed=seed, nll_out=nll,
                    grad_out=g, grad_w_out=gw)

    for k in range(args.warmup):
        step(k)
    ms = time_graph(torch, step, args.steps)
    nb = c["counts"].size
    print(json.dumps(dict(metric="bins*(NLL+grad+grad_w)/s", value=nb / (ms * 1e-3), unit="bins/s",
                          n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=ms,
                          higher_is_better=True, scaling="weak", vs_baseline=None,
                          dtype="f64" if prec == hf.FP64 else "f32-bin/f64-acc",
                          data="synthetic",
                          config=dict(workload="2D histogram 2048x2048, correlated Gaussian + "
                                               "constant (7 parameters), f32 weights, weighted "
                                               "Poisson NLL + gradient + weight gradient",
                                      nbins=nb, precision=args.precision),
                          hbm_gbs=12 * nb / (ms * 1e-3) / 1e9)), flush=True)


def bench_fisher(args, hf, datagen, np, torch, dev):
    """Expected Hessian F = J^T diag(w c) J of the 1e7-bin two-Gaussian +
    cubic workload (P = 10: 55 upper-triangle FMAs per bin), then of the
    2048^2 2D workload (P = 7: 28 per bin).  The Poisson F does not read the
    counts (c = 1/mu), so these kernels are bound by the FP64 vector units;
    the figure reported is the contraction's algorithmic FP64 rate,
    2 P(P+1)/2 flops per bin, against the 78.6 TFLOP/s FP64 vector peak."""
    obj = {"poisson": hf.POISSON, "neyman": hf.NEYMAN, "pearson": hf.PEARSON}[args.objective]
    c1 = datagen.large_fit_case()
    c2 = datagen.hist2d_case()
    work = [
        ("1D histogram, 1e7 bins on [0,100], two Gaussians + cubic (10 parameters)",
         hf.make_hist(c1["counts"], c1["range"], device=dev), hf.Model.from_spec(c1["spec"]),
         c1["theta_eval"], c1["counts"].size),
        ("2D histogram 2048x2048, correlated Gaussian + constant (7 parameters), f32 weights",
         hf.make_hist(c2["counts"], (0.0, 1.0), (0.0, 1.0), weights=c2["weights"], device=dev),
         hf.Model(hf.GAUSS2D), c2["theta_eval"], c2["counts"].size),
    ]
    for name, h, m, th, nb in work:
        P = m.nparams
        tht = torch.as_tensor(th, dtype=torch.float64, device=dev)
        out = torch.empty((P, P), dtype=torch.float64, device=dev)

        def step(k):
            hf.nll_fisher(h, m, tht, objective=obj, out=out)

        for k in range(args.warmup):
            step(k)
        ms = time_graph(torch, step, args.steps)
        flops = 2.0 * (P * (P + 1) // 2) * nb
        achieved = flops / (ms * 1e-3) / 1e12
        print(json.dumps(dict(
            metric="bins*Fisher/s", value=nb / (ms * 1e-3), unit="bins/s", n_gpus=1,
            steps=args.steps, warmup=args.warmup, ms_per_step=ms, higher_is_better=True,
            scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
            config=dict(workload=name + ", expected Hessian, " + args.objective, nbins=nb,
                        nparams=P),
            roofline=dict(bound="alu", achieved=achieved, peak=78.6, unit="TFLOP/s",
                          frac=achieved / 78.6, traffic=None,
                          note="contraction flops only (2 per upper-triangle entry per bin)"))),
              flush=True)


def bench_gradmap(args, hf, np, torch, dev):
    """Elementwise Gaussian and its gradient over 2^27 independent parameter
    sets.  First the listing's configuration (per-element x and p, one shared
    sigma, outputs dx and dp: 32 bytes per element), then every input per
    element with every output (x, p, sigma and a seed in; g, dx, dp, dsigma
    out: 64 bytes).
    Both stream HBM: the roofline is the 8 TB/s peak."""
    n = 1 << 27
    gen = torch.Generator(device=dev).manual_seed(12)
    p = torch.rand(n, dtype=torch.float64, device=dev, generator=gen) * 6 - 3
    x = p + torch.randn(n, dtype=torch.float64, device=dev, generator=gen) * 2
    s1 = torch.tensor([1.25], dtype=torch.float64, device=dev)
    sn = torch.rand(n, dtype=torch.float64, device=dev, generator=gen) + 0.5
    w = torch.randn(n, dtype=torch.float64, device=dev, generator=gen)
    runs = [
        ("listing: x, p per element, sigma shared; outputs dx, dp", 32,
         lambda k: hf.gauss_grad_map(x, p, s1, want_g=False)),
        ("all per element with a seed; outputs g, dx, dp, dsigma", 64,
         lambda k: hf.gauss_grad_map(x, p, sn, seed=w, want_dsigma=True)),
    ]
    for name, bpe, step in runs:
        for k in range(args.warmup):
            step(k)
        torch.cuda.synchronize()
        # eager launches: the outputs are allocated per call by the binding
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for k in range(args.steps):
            step(k)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        gbs = bpe * n / (ms * 1e-3) / 1e9
        print(json.dumps(dict(
            metric="elements*(g,grad)/s", value=n / (ms * 1e-3), unit="elements/s", n_gpus=1,
            steps=args.steps, warmup=args.warmup, ms_per_step=ms, higher_is_better=True,
            scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
            config=dict(workload="elementwise Gaussian gradient, 2^27 parameter sets, " + name,
                        n=n, bytes_per_element=bpe),
            roofline=dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=gbs / HBM_PEAK_GBS, traffic=None))), flush=True)


# Algorithmic FP64 flops per event of the unbinned workload (two Gaussians,
# cubic, value + 10-component gradient), counted like FLOPS_PER_BIN: per
# Gaussian z, z^2/2, exp, G, G z, G z^2 (6 + exp); cubic t and Horner (8) and
# powers (3); log; reciprocal; the weighted value and 10 gradient FMAs (22).
FLOPS_PER_EVENT = 2 * (6 + FLOPS_EXP) + 11 + FLOPS_LOG + FLOPS_DIV + 22


def bench_unbinned(args, hf, datagen, np, torch, dev):
    """Extended unbinned NLL + gradient of 1e7 events drawn from the 1e7-bin
    workload's intensity (two Gaussians + cubic on [0, 100]): 8 bytes per
    event, bound by the FP64 vector units."""
    c = datagen.unbinned_case()
    x = torch.as_tensor(c["events"], device=dev)
    th = torch.as_tensor(c["theta_eval"], dtype=torch.float64, device=dev)
    m = hf.Model.from_spec(c["spec"])
    nll = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(m.nparams, dtype=torch.float64, device=dev)

    def step(k):
        hf.nll_unbinned(x, 0.0, 100.0, m, th, nll_out=nll, grad_out=g)

    for k in range(args.warmup):
        step(k)
    ms = time_graph(torch, step, args.steps)
    n = x.numel()
    achieved = FLOPS_PER_EVENT * n / (ms * 1e-3) / 1e12
    print(json.dumps(dict(
        metric="events*(NLL+grad)/s", value=n / (ms * 1e-3), unit="events/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=ms, higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload="extended unbinned NLL + gradient, 1e7 events on [0,100], two "
                             "Gaussians + cubic (10 parameters)", n_events=n),
        roofline=dict(bound="alu", achieved=achieved, peak=FP64_VEC_PEAK_TFLOPS, unit="TFLOP/s",
                      frac=achieved / FP64_VEC_PEAK_TFLOPS, traffic=None,
                      flops_per_event=FLOPS_PER_EVENT))), flush=True)


def bench_binavg(args, hf, datagen, np, torch, dev, edges=False):
    """The 1e7-bin two-Gaussian + cubic Poisson NLL + gradient with mu_i the
    model's average over bin i (an erf and an exp per Gaussian per bin edge),
    FP64, on one resident histogram; with edges, the centre model on 1e7 bins
    whose widths vary 100-fold (8 more bytes per bin, one exp per Gaussian
    per bin)."""
    c = datagen.large_fit_case()
    spec = dict(c["spec"], bin_average=0 if edges else 1)
    e = None
    if edges:
        w = np.exp(np.random.default_rng(8).uniform(np.log(0.01), np.log(1.0), c["nbins"]))
        e = np.concatenate([[0.0], np.cumsum(w)])
        e = 100.0 * e / e[-1]
    h = hf.make_hist(c["counts"], c["range"], device=dev, edges=e)
    m = hf.Model.from_spec(spec)
    th = torch.as_tensor(c["theta_eval"], dtype=torch.float64, device=dev)
    nll = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(m.nparams, dtype=torch.float64, device=dev)

    def step(k):
        hf.nll_grad(h, m, th, objective=hf.POISSON, nll_out=nll, grad_out=g)

    for k in range(args.warmup):
        step(k)
    ms = time_graph(torch, step, args.steps)
    nb = c["counts"].size
    print(json.dumps(dict(
        metric="bins*(NLL+grad)/s", value=nb / (ms * 1e-3), unit="bins/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=ms, higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload=("1D histogram, 1e7 bins of varying widths on [0,100], two "
                              "Gaussians + cubic at the bin midpoints" if edges else
                              "1D histogram, 1e7 bins on [0,100], two Gaussians + cubic, model "
                              "averaged over each bin") + ", Poisson NLL + gradient", nbins=nb))),
          flush=True)


def fits_cpu_baseline(c, theta0, np, seconds=10.0):
    """The oracle's fitter (FP64 bins, Fisher start, same starts) over host
    threads, one histogram per thread at a time, on the first histograms of
    the batch until about `seconds` have passed; fits/s over that sample."""
    import oracle
    spec = c["spec"]
    m = oracle.Model(spec["kind"], spec["n_gauss"], spec["poly_degree"], spec["t_shift"],
                     spec["t_scale"])
    cores = cpu_cores()
    off = c["offsets"]
    counts = c["counts"].astype(np.float64)
    done, t0 = 0, time.perf_counter()
    B = len(off) - 1
    while done < B and time.perf_counter() - t0 < seconds:
        n = min(4 * cores, B - done)
        sub = off[done:done + n + 1] - off[done]
        oracle.fit_many(m, oracle.POISSON, counts[off[done]:off[done + n]], sub,
                        c["ranges"][done:done + n], theta0[done:done + n], nthreads=cores,
                        hessian_init=1)
        done += n
    dt = time.perf_counter() - t0
    bins = int(off[done] - off[0])
    return dict(value=done / dt, unit="fits/s", cores=cores, kind="oracle",
                sample="the first %d of the %d histograms (%d bins), %.1f s, %d threads, FP64 "
                       "bins" % (done, B, bins, dt, cores))


def gradient_section(hf, datagen, np, torch, dev):
    """The paper's comparison (sec. 4, Fig. 2b) on this framework: the same
    fits with the gradient from the reverse-mode adjoint sweep and from
    central differences of the objective (2P value sweeps per gradient), as
    the number of parameters grows: K = 1..4 Gaussians on a linear
    background (P = 3K + 2), 512 histograms of 10,000 bins each, FP64 bins,
    one fit_batch launch per mode.  Plus the cost of one gradient of the
    1e7-bin two-Gaussian + cubic histogram: nll_grad against 2P+1 nll_eval.
    Returns (rows per K, per-call costs)."""
    # the library's default launch shape: a shape tuned for another model
    # (its LDS cache) need not fit these models' kernels
    before, before_waves = hf.fit_get_tuning(), hf.fit_get_wave_bins()
    hf.fit_set_tuning(2, 0, 256)
    hf.fit_set_wave_bins(0)
    rows = []
    for K in (1, 2, 3, 4):
        c = datagen.kgauss_batch_case(K)
        counts = torch.from_numpy(c["counts"].view(np.int32)).to(dev)
        off = torch.as_tensor(c["offsets"], device=dev)
        rg = torch.as_tensor(c["ranges"], device=dev)
        t0 = torch.as_tensor(c["theta0"], device=dev)
        m = hf.Model.from_spec(c["spec"])
        row = dict(gaussians=K, params=3 * K + 2, histograms=len(c["offsets"]) - 1)
        ref = None
        for name, mode in (("adjoint", hf.ADJOINT), ("central_diff", hf.FINITE_DIFF)):
            out = hf.fit_batch(counts, off, rg, m, t0, objective=hf.POISSON, precision=hf.FP64,
                               gradient=mode)
            torch.cuda.synchronize()
            ms = time_graph(torch, lambda k: hf.fit_batch(counts, off, rg, m, t0,
                                                          objective=hf.POISSON, precision=hf.FP64,
                                                          gradient=mode, out=out), 3)
            if ref is None:
                ref = (out.nll.clone(), out.status.clone())
            ok = ((out.status == 0) & (ref[1] == 0) & ((out.nll - ref[0]).abs() < 1e-6)).sum().item()
            row[name] = dict(ms=ms, fits_per_s=ok / (ms * 1e-3), agreeing=ok,
                             mean_iters=float(out.iters.float().mean().item()),
                             mean_evals=float(out.nevals.float().mean().item()))
            log("K=%d %s: %.2f ms, %d agreeing, %.1f iterations, %.1f sweeps" % (
                K, name, ms, ok, row[name]["mean_iters"], row[name]["mean_evals"]))
        row["speedup"] = row["central_diff"]["ms"] / row["adjoint"]["ms"]
        rows.append(row)
    hf.fit_set_tuning(*before)
    hf.fit_set_wave_bins(before_waves)
    # one gradient of the 1e7-bin histogram: adjoint sweep vs 2P+1 value sweeps
    case = datagen.large_fit_case(seed=2)
    spec = case["spec"]
    mL = hf.Model.from_spec(spec)
    h = hf.make_hist(case["counts"], case["range"], device=dev)
    th = torch.as_tensor(case["theta_eval"], dtype=torch.float64, device=dev)
    nll = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(mL.nparams, dtype=torch.float64, device=dev)
    for _ in range(4):
        hf.nll_grad(h, mL, th, nll_out=nll, grad_out=g)
        hf.nll_eval(h, mL, th, out=nll)
    t_grad = time_graph(torch, lambda k: hf.nll_grad(h, mL, th, nll_out=nll, grad_out=g), 64)
    t_eval = time_graph(torch, lambda k: hf.nll_eval(h, mL, th, out=nll), 64)
    P = mL.nparams
    per_call = dict(nbins=int(case["counts"].size), params=P, nll_grad_us=t_grad * 1e3,
                    nll_eval_us=t_eval * 1e3, central_diff_gradient_us=(2 * P + 1) * t_eval * 1e3,
                    speedup=(2 * P + 1) * t_eval / t_grad)
    return rows, per_call


# What the paper reports for the same comparison, quoted as context only.
PAPER_CONTEXT = ("paper (sec. 4, Fig. 2): about 10x faster ROOT histogram fits of sums of "
                 "Gaussians with the Clad reverse-mode gradient than with numerical "
                 "derivatives; CPU, hardware not stated")


def bench_gradient(args, hf, datagen, np, torch, dev):
    """The paper's comparison (see gradient_section) as its own bench line."""
    rows, per_call = gradient_section(hf, datagen, np, torch, dev)
    last = rows[-1]
    print(json.dumps(dict(
        metric="fits/s, reverse-mode vs central-difference gradient", value=last["adjoint"]["fits_per_s"],
        unit="fits/s", n_gpus=1, steps=3, warmup=1, ms_per_step=last["adjoint"]["ms"],
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload="512 1D histograms of 10,000 bins, K Gaussians + linear background "
                             "(K = 1..4), Poisson, FP64 bins, Fisher-started BFGS; value: adjoint "
                             "gradient at K = 4"),
        sweep=rows, per_call=per_call, paper_context=PAPER_CONTEXT)), flush=True)


def host_cpu():
    """Host CPU model (from /proc/cpuinfo) and the host's logical CPU count."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(model=model, logical_cpus=os.cpu_count(),
                usable_cpus=len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                else os.cpu_count())


def event_time(torch, fn, trials):
    """Median over `trials` of fn()'s elapsed time between HIP events on the
    current stream (host synchronisations inside fn are part of it); returns
    (median ms, all trials)."""
    out = []
    for _ in range(trials):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return sorted(out)[len(out) // 2], out


def fits_section(hf, datagen, np, torch, dev, prec, steps, cpu=True):
    """4096 histograms (256..65536 bins, Gauss + exponential background) fitted
    from the default starts in one graph-replayed fit_batch launch at the
    autotuned shape; fits/s counts fits whose final NLL agrees with the
    FP64-bin fit from the same start within 1e-6.  Returns (section dict,
    batch data reused by the learned section)."""
    c = datagen.batch_case()
    B = len(c["nbins"])
    counts = torch.from_numpy(c["counts"].view(np.int32)).to(dev)
    off = torch.as_tensor(c["offsets"], device=dev)
    rg = torch.as_tensor(c["ranges"], device=dev)
    m = hf.Model.from_spec(c["spec"])
    # the plain method's own starting points (computed once, outside the timing)
    t0 = hf.default_starts(counts, off, rg, m)
    from paper_2203_06139_amd.autotune import tune_fit
    # tuned on the whole batch: its longest fits decide the wall time, and a
    # random sample can miss them
    best, _ = tune_fit(counts, off, rg, m, t0, precision=prec, sample=B, use_cache=False)
    log("autotuned: %s" % best)
    kw = dict(objective=hf.POISSON, precision=prec, polish_edm=best["polish_edm"])
    ref = hf.fit_batch(counts, off, rg, m, t0, objective=hf.POISSON, precision=hf.FP64)
    out = hf.fit_batch(counts, off, rg, m, t0, **kw)
    torch.cuda.synchronize()
    steps = max(1, min(steps, 5))
    ms = time_graph(torch, lambda k: hf.fit_batch(counts, off, rg, m, t0, out=out, **kw), steps)
    ok = int(((out.status == 0) & (ref.status == 0) & ((out.nll - ref.nll).abs() < 1e-6))
             .sum().item())
    sec = dict(metric="fits/s at |dNLL|<1e-6", value=ok / (ms * 1e-3), unit="fits/s",
               ms_per_batch=ms, steps=steps,
               dtype="f64" if prec == hf.FP64 else "f32-bin/f64-acc",
               config=dict(workload="4096 1D histograms, 256..65536 bins (log-uniform), Gauss + "
                                    "exponential background, Poisson, default starts, one "
                                    "graph-replayed fit_batch launch", histograms=B,
                           total_bins=int(c["offsets"][-1])),
               agreeing=ok, mean_iters=float(out.iters.float().mean().item()),
               mean_evals=float(out.nevals.float().mean().item()),
               max_evals=int(out.nevals.max().item()), tuning=best, cpu_baseline=None)
    if cpu:
        log("cpu baseline (oracle fits)")
        sec["cpu_baseline"] = fits_cpu_baseline(c, t0.cpu().numpy(), np)
    return sec, dict(c=c, counts=counts, off=off, rg=rg, tuning=best)


def learned_section(hf, np, torch, dev, batch, train_fits, epochs, trials=5):
    """The learned initialiser: trained on `train_fits` plain fits of 4096-bin
    histograms (seeds disjoint from the batch), then the 4096-histogram batch
    fitted both ways at the same (tuned) launch shape and polish threshold:
      plain   = default starts + fit_batch,
      learned = 256-bin rebin + network + fit_batch + plain refit of the fits
                that did not reach a physical minimum.
    Each path is timed with HIP events, median of `trials`.  A learned fit
    agrees when both converged and |NLL_learned - NLL_plain| < 1e-6; fits
    that reached a lower or a higher minimum are reported apart and do not
    count."""
    from paper_2203_06139_amd.learned_init import FitSet, LearnedInit, plain_fit, timed
    pol = batch["tuning"]["polish_edm"]
    li = LearnedInit(dev, seed=0, batch=1024)
    kept, t_data = timed(lambda: li.build_training_set(train_fits, seed=10_000, log=log))
    hist, t_train = timed(lambda: li.train(epochs=epochs, lr=1e-3, log=log))
    fs = FitSet(batch["counts"], batch["off"], batch["rg"])
    res = {}
    plain_run = lambda: res.__setitem__("plain", plain_fit(fs, polish_edm=pol)[1])
    learned_run = lambda: res.__setitem__("learned", li.fit(fs, polish_edm=pol))
    plain_run()
    learned_run()  # warm-up of both paths
    ms_plain, tr_plain = event_time(torch, plain_run, trials)
    ms_learned, tr_learned = event_time(torch, learned_run, trials)
    plain = res["plain"]
    learned, nfb = res["learned"]
    both = (plain.status == 0) & (learned.status == 0)
    dn = learned.nll - plain.nll
    n_equal = int((both & (dn.abs() < 1e-6)).sum().item())
    n_lower = int((both & (dn <= -1e-6)).sum().item())
    n_higher = int((both & (dn >= 1e-6)).sum().item())
    n_plain = int((plain.status == 0).sum().item())
    B = int(plain.status.numel())
    return dict(
        metric="fits/s at |dNLL|<1e-6 vs the plain fit", unit="fits/s",
        value=n_equal / (ms_learned * 1e-3),
        plain=dict(fits_per_s=n_plain / (ms_plain * 1e-3), converged=n_plain, ms=ms_plain,
                   trials_ms=tr_plain, mean_iters=float(plain.iters.float().mean().item()),
                   mean_evals=float(plain.nevals.float().mean().item())),
        learned=dict(fits_per_s_agreeing=n_equal / (ms_learned * 1e-3), agreeing=n_equal,
                     lower_minimum=n_lower, higher_minimum=n_higher,
                     not_both_converged=B - int(both.sum().item()), fallbacks=nfb,
                     ms=ms_learned, trials_ms=tr_learned,
                     mean_iters=float(learned.iters.float().mean().item()),
                     mean_evals=float(learned.nevals.float().mean().item())),
        speedup=(n_equal / ms_learned) / max(n_plain / ms_plain, 1e-30),
        tuning=batch["tuning"],
        training=dict(train_fits=train_fits, kept=kept, epochs=epochs,
                      final_loss=hist[-1], data_seconds=t_data, train_seconds=t_train))


def single_fit_section(hf, datagen, np, torch, dev, trials=5, cpu=True):
    """The plain single fit: 10,000 bins on [0,10], Gauss + line (5
    parameters), Poisson counts, started at (8e3, 4.8, 0.6, 45, -1.5); BFGS
    with the Fisher start, at most 200 iterations, stopping at EDM < 1e-10,
    FP64 bins, Poisson NLL and Neyman chi-square; one fit_batch of one
    histogram (one workgroup), HIP events, median of `trials`.  Past
    convergence further iterations would only trade rounding noise, so the
    fit stops there; time per iteration is reported beside the fit time.
    CPU baseline: the oracle's fitter from the same start with the same
    rules, one thread."""
    import oracle
    c = datagen.single_fit_case()
    m = hf.Model.from_spec(c["spec"])
    counts = torch.from_numpy(c["counts"].view(np.int32)).to(dev)
    off = torch.tensor([0, counts.numel()], dtype=torch.int64, device=dev)
    rg = torch.tensor([c["range"]], dtype=torch.float64, device=dev)
    th0 = torch.as_tensor(c["theta0"][None, :], dtype=torch.float64, device=dev)
    spec = c["spec"]
    om = oracle.Model(spec["kind"], spec["n_gauss"], spec["poly_degree"], spec["t_shift"],
                      spec["t_scale"])
    out = {}
    for name, obj in (("poisson", hf.POISSON), ("neyman", hf.NEYMAN)):
        kw = dict(objective=obj, precision=hf.FP64, max_iter=200, edm_tol=1e-10,
                  hessian_init=hf.FISHER)
        r = hf.fit_batch(counts, off, rg, m, th0, **kw)
        ms, tr = event_time(torch, lambda: hf.fit_batch(counts, off, rg, m, th0, out=r, **kw),
                            trials)
        it = int(r.iters[0].item())
        d = dict(ms=ms, trials_ms=tr, iters=it, evals=int(r.nevals[0].item()),
                 us_per_iter=1e3 * ms / max(it, 1), nll=float(r.nll[0].item()),
                 status=int(r.status[0].item()))
        if cpu:
            t = time.perf_counter()
            orf = oracle.fit(om, obj, c["counts"], c["theta0"], c["range"], max_iter=200,
                             edm_tol=1e-10, hessian_init=1)
            dt = time.perf_counter() - t
            d["cpu_baseline"] = dict(ms=1e3 * dt, cores=1, kind="oracle", iters=orf.iters,
                                     evals=orf.nevals, nll=orf.nll, status=orf.status,
                                     sample="one fit, same start and stopping rule, 1 thread")
            d["abs_dnll_vs_oracle"] = abs(d["nll"] - orf.nll)
        out[name] = d
    return dict(config="10,000 bins on [0,10], Gauss + line (5 parameters), BFGS from the "
                       "Fisher start, at most 200 iterations, EDM < 1e-10, FP64 bins, one "
                       "fit_batch of one histogram", **out)


def bench_fits(args, hf, datagen, np, torch, dev):
    prec = hf.FP64 if args.precision == "fp64" else hf.FP32_BIN
    sec, _ = fits_section(hf, datagen, np, torch, dev, prec, args.steps,
                          cpu=not args.no_cpu_baseline)
    cfg = sec.pop("config")
    cpu = sec.pop("cpu_baseline")
    print(json.dumps(dict(metric=sec.pop("metric"), value=sec.pop("value"), unit=sec.pop("unit"),
                          n_gpus=1, steps=sec.pop("steps"), warmup=1,
                          ms_per_step=sec.pop("ms_per_batch"), higher_is_better=True,
                          scaling="weak", vs_baseline=None, dtype=sec.pop("dtype"),
                          data="synthetic", config=dict(cfg, **sec), cpu_baseline=cpu)),
          flush=True)


def bench_smallfits(args, hf, datagen, np, torch, dev):
    """16384 histograms of 128..1024 bins (log-uniform; Gauss + exponential
    background, Poisson) from the default starts, FP32 bins + FP64 polish:
    the autotuned shape (which includes the size below which every wave fits
    a histogram of its own) against the same shape with one workgroup per
    histogram; and the same from starts near the truth, waves below 1024
    bins.  fits/s counts fits within 1e-6 of the FP64-bin fit."""
    from paper_2203_06139_amd.autotune import tune_fit
    c = datagen.batch_case(seed=11, B=16384, lo_bins=128, hi_bins=1024)
    B = len(c["nbins"])
    counts = torch.from_numpy(c["counts"].view(np.int32)).to(dev)
    off = torch.as_tensor(c["offsets"], device=dev)
    rg = torch.as_tensor(c["ranges"], device=dev)
    m = hf.Model.from_spec(c["spec"])
    t0 = hf.default_starts(counts, off, rg, m)
    best, _ = tune_fit(counts, off, rg, m, t0, precision=hf.FP32_BIN, sample=B, use_cache=False)
    log("autotuned: %s" % best)
    kw = dict(objective=hf.POISSON, precision=hf.FP32_BIN, polish_edm=best["polish_edm"])
    steps = max(1, min(args.steps, 20))

    def modes(start, waves):
        ref = hf.fit_batch(counts, off, rg, m, start, objective=hf.POISSON, precision=hf.FP64)
        res = {}
        for name, wb in (("workgroup_per_histogram", 0), ("waves", waves)):
            hf.fit_set_wave_bins(wb)
            out = hf.fit_batch(counts, off, rg, m, start, **kw)
            ms = time_graph(torch, lambda k: hf.fit_batch(counts, off, rg, m, start, out=out, **kw),
                            steps)
            ok = int(((out.status == 0) & (ref.status == 0) & ((out.nll - ref.nll).abs() < 1e-6))
                     .sum().item())
            res[name] = dict(wave_bins=wb, ms=ms, agreeing=ok, fits_per_s=ok / (ms * 1e-3))
        return res

    res = modes(t0, best["wave_bins"])
    # the same histograms from starts near the truth (amplitudes, widths and
    # background 5% off, means 0.3 widths off): no wrong-start runaways, so
    # the bulk of short fits sets the time
    rng = np.random.default_rng(12)
    th = c["theta_true"].copy()
    th[:, 0] *= 1 + 0.05 * rng.standard_normal(B)
    th[:, 1] += 0.3 * th[:, 2] * rng.standard_normal(B)
    th[:, 2] *= 1 + 0.05 * rng.standard_normal(B)
    th[:, 3] += 0.05 * rng.standard_normal(B)
    near = modes(torch.as_tensor(th, device=dev), 1024)
    hf.fit_set_wave_bins(0)
    t = res["waves"]
    print(json.dumps(dict(
        metric="fits/s at |dNLL|<1e-6", value=t["fits_per_s"], unit="fits/s", n_gpus=1,
        steps=steps, warmup=1, ms_per_step=t["ms"], higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32-bin/f64-acc", data="synthetic",
        config=dict(workload="16384 1D histograms, 128..1024 bins (log-uniform), Gauss + "
                             "exponential background, Poisson, default starts, one "
                             "graph-replayed fit_batch launch", histograms=B,
                    total_bins=int(c["offsets"][-1])),
        tuning=best, modes=res,
        speedup=res["workgroup_per_histogram"]["ms"] / t["ms"],
        near_true_starts=dict(modes=near, speedup=near["workgroup_per_histogram"]["ms"] /
                              near["waves"]["ms"]))), flush=True)


def bench_learned(args, hf, datagen, np, torch, dev):
    _, batch = fits_section(hf, datagen, np, torch, dev, hf.FP32_BIN, args.steps, cpu=False)
    sec = learned_section(hf, np, torch, dev, batch, args.train_fits, args.epochs)
    print(json.dumps(dict(
        metric="fits/s at |dNLL|<1e-6: plain vs batched+learned init", value=sec["value"],
        unit="fits/s", n_gpus=1, steps=1, warmup=1, ms_per_step=sec["learned"]["ms"],
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32-bin/f64-acc",
        data="synthetic",
        config=dict(workload="4096 1D histograms, 256..65536 bins, Gauss + exponential "
                             "background, Poisson; plain = default starts + fit_batch, learned "
                             "= 256-bin rebin + BF16-MFMA MLP starts + fit_batch + plain "
                             "fallback", histograms=int(batch["off"].numel() - 1)),
        plain=sec["plain"], learned=sec["learned"], speedup=sec["speedup"],
        tuning=sec["tuning"], training=sec["training"])), flush=True)


if __name__ == "__main__":
    main()
