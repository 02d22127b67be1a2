#!/usr/bin/env python3
"""Benchmark: slices/s of the log-polar R, R# and FBP on one MI355X.

One step = the whole hot path on one batch of 2048 x 2048 slices (2048 angles x 2048 bins):
g = R f, then R# g, then FBP g (ramp + R#).  Inputs are resident in HBM before the timed
region.  Also reported: per-operator slices/s batched (the batch's kernels as one HIP graph
replay, and eagerly) vs plain (batch-1 calls in a loop) with each operator's HBM fraction on
algorithmic bytes and its roofline fraction max(t_HBM, t_VALU, t_LDS) / t, per-kernel durations
from HIP events recorded on the launch stream, the roofline position of the dominant kernel,
the 1024 x 1024 geometry's R, R# and FBP, the batched least-squares reconstruction by autograd,
ragged batches, and the FP64 oracle timed on the host on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "slices/s for R and R# at N=2048 fp32, batched vs plain; % of HBM peak"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published
# Algorithmic FP32 operations per fine log-polar sample of the two interpolation kernels:
# the 4 x 4 tensor-product weights and their sum (4 + 16 products, 16 sums), the eight
# cubic weights (2 x 10), and the four-tap decimation filter or its transpose (8).
ALG_FLOPS_PER_SAMPLE = {"k_lp2cart_adj": 64, "k_cart2lp": 64}
LDS_PEAK_GBS = 128 * 256 * 2.4  # assumed LDS bandwidth: 128 B per clock per CU, 256 CUs, 2.4 GHz


def _partition_constants(m):
    beta = math.pi / m
    sh, ch = math.sin(beta / 2), math.cos(beta / 2)
    return sh / (1 + sh), (ch - sh) / (1 + sh)


def operator_model(g, n_own, samples, batch):
    """Algorithmic work of one R (or R#, its mirror) per slice at the method's minimum sizes, so
    that padding never inflates it: N_rho at its bound (sec. 3 eq. vrho) and K = 2 n_own.

      bytes  4 N^2 (image) + 4 N_theta N_s (sinogram) + 32 M n_own (N_rho/2 + 1) (the half
             spectra written and read between the rho and theta FFT passes, twice) + the kernel
             table 8 (K/2 + 1)(N_rho/2 + 1) once per batch
      flops  prefilter 8 per pixel (the recursive form: two first-order passes per axis);
             60 per fine sample inside D (16-tap bicubic, its weights, the decimation);
             real rho FFTs 2.5 N_rho log2 N_rho per row (M (n_own + 4) rows forward, M n_own
             inverse); complex theta FFTs 5 K log2 K per column, forward and inverse, M (N_rho/2 + 1)
             columns; the multiplier 6 per lattice point; the 4-tap evaluation 18 per sinogram sample
      lds    16 taps x 4 bytes per fine sample
    Returns per-slice (bytes, flops, lds_bytes) and the times they take at the peaks."""
    n, nt, ns, m = g["n"], g["n_theta"], g["n_s"], g["m"]
    a_R, a_r = _partition_constants(m)
    nr = math.ceil(math.log(a_r) / math.log(1.0 - 2.0 * a_R / n))
    K = 2 * n_own
    cols = nr // 2 + 1
    by = 4 * n * n + 4 * nt * ns + 32 * m * n_own * cols + 8 * (K // 2 + 1) * cols / batch
    fl = (8 * n * n + 60 * samples + 2.5 * nr * math.log2(nr) * m * (2 * n_own + 4)
          + 2 * 5 * K * math.log2(K) * m * cols + 6 * m * K * cols + 18 * nt * ns)
    lds = 64 * samples
    return {"alg_bytes_per_slice": round(by), "alg_flops_per_slice": round(fl), "lds_bytes_per_slice": lds,
            "t_hbm_us": by / (HBM_PEAK_GBS * 1e3), "t_valu_us": fl / (FP32_PEAK_TFLOPS * 1e6),
            "t_lds_us": lds / (LDS_PEAK_GBS * 1e3), "n_rho_min": nr, "k_min": K}


def roofline_fractions(model, ms_per_slice):
    """HBM fraction on algorithmic bytes and roofline fraction max(t_HBM, t_VALU, t_LDS) / t."""
    t_us = ms_per_slice * 1e3
    return {"hbm_frac": round(model["t_hbm_us"] / t_us, 4),
            "roofline_frac": round(max(model["t_hbm_us"], model["t_valu_us"], model["t_lds_us"]) / t_us, 4)}


def kernel_bytes(name, g, n_own, batch):
    """Algorithmic HBM bytes of one launch of each kernel (what it must read and write)."""
    n, nt, ns, m, nr, K = g["n"], g["n_theta"], g["n_s"], g["m"], g["n_rho"], g["k_theta"]
    n_sup = n_own + 4
    nc1 = nr // 2 + 1
    img = 4 * n * n
    sino = 4 * nt * ns
    lp_sup = 4 * m * n_sup * nr
    sp_sup = 8 * m * n_sup * nc1
    sp_own = 8 * m * n_own * nc1
    table = 8 * nc1 * (K // 2 + 1)
    per_slice = {
        "k_prefilter": 2 * img,
        "k_cart2lp": img + lp_sup,
        "k_rfft_rows": lp_sup + sp_sup,
        "k_theta_conv": sp_sup + sp_own,
        "k_irfft_eval": sp_own + sino,
        "k_splat_rfft": sino + sp_own,
        "k_irfft_scale": sp_sup + lp_sup,
        "k_lp2cart_adj": lp_sup + img,
        "k_ramp": 2 * sino,
    }
    extra = table if name == "k_theta_conv" else 0
    return per_slice[name] * batch + extra


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_2048x2048_b64.txt")


CSRC = os.path.join(ROOT, "paper_1506_00014_amd", "csrc")
# files every kernel's code or launch configuration depends on besides its own: the plan
# (geometry tables, launch-parameter defaults) and the shared device headers
COMMON_SOURCES = ("plan.hip", "rl_internal.h", "fft_device.h")


def file_digest(name):
    """SHA-256 of one HIP source or device header of the library."""
    with open(os.path.join(CSRC, name), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def kernel_sources(kernel):
    """The sources a kernel's counters depend on: the file that defines it and COMMON_SOURCES.
    Counters taken on other versions of these files are stale; other files do not matter."""
    pat = re.compile(r"__global__[^;{]*?\b" + re.escape(kernel) + r"\s*\(", re.S)
    own = [f for f in sorted(os.listdir(CSRC)) if f.endswith(".hip") and pat.search(open(os.path.join(CSRC, f)).read())]
    return own + [f for f in COMMON_SOURCES if f not in own] if own else []


def measured_traffic(kernel, batch, n):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, each scaled by what the same counter reads for a plain device copy of known size.
    None if the summary is absent, is for another workload, or the sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    kv = {}
    for ln in lines:
        if ln.startswith("    ") or ":" not in ln or ln.startswith("#"):
            continue
        k, v = ln.split(":", 1)
        kv[k.strip()] = v.strip()
    try:
        if int(kv["batch"]) != batch or int(kv["n"]) != n:
            return None
        srcs = kernel_sources(kernel)
        if not srcs or any(kv[f"source_sha256 {f}"] != file_digest(f) for f in srcs):
            return None
        copy_bytes = float(kv["copy_bytes"])
        f_scale = copy_bytes / (1024.0 * float(kv["copy_fetch_kib"]))
        w_scale = copy_bytes / (1024.0 * float(kv["copy_write_kib"]))
        fetch = 1024.0 * float(kv[f"{kernel}_fetch_kib"]) * f_scale
        write = 1024.0 * float(kv[f"{kernel}_write_kib"]) * w_scale
    except (KeyError, ValueError, ZeroDivisionError):
        return None
    return {"bytes": round(fetch + write), "fetch": round(fetch), "write": round(write),
            "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)}


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain device-to-device copy of known size, run under rocprofv3 --pmc to calibrate
    FETCH_SIZE and WRITE_SIZE (bytes the counter reports per byte actually moved)."""
    import torch

    torch.cuda.set_device(0)
    src = torch.rand(nbytes // 4, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def _cpu_sample(g, seed=303, parts=1):
    """One timed sample of the FP64 oracle on `parts` of the M partitions of one slice: the
    prefilter, the partition forwards (with their polar evaluation), the ramp filter and the
    partition transposes.  Returns the component times in seconds."""
    import numpy as np

    from oracle import bspline, radon as oradon
    from oracle.geometry import Geometry
    from paper_1506_00014_amd import inputs

    og = Geometry(g["n"], g["n_theta"], g["n_s"], g["m"], g["n_rho"], g["k_theta"], g["r_dec"]).validate()
    f = inputs.uniform_image(g["n"], seed)
    oradon._H(og)  # plan-time kernel table, not part of the sample
    t0 = time.perf_counter()
    c = bspline.prefilter_2d(f)
    t_q = time.perf_counter() - t0
    gpart = np.zeros((og.n_theta, og.n_s))
    t_fwd = t_adj = 0.0
    for p in range(parts):
        t0 = time.perf_counter()
        clp = oradon._partition_forward(og, c, p, "fft")
        for i, j, tau in oradon.eval_taus(og, p):
            gpart[j] = bspline.eval_periodic_1d(clp[i], tau) / og.a_R
        t_fwd += time.perf_counter() - t0
    t0 = time.perf_counter()
    oradon.ramp_filter(og, gpart[: max(1, og.n_theta // 16)])  # 1/16 of the rows, scaled below
    t_ramp = 16.0 * (time.perf_counter() - t0)
    for p in range(parts):
        t0 = time.perf_counter()
        oradon._partition_adjoint(og, gpart, p, "fft")
        t_adj += time.perf_counter() - t0
    return {"q": t_q, "fwd": t_fwd / parts, "adj": t_adj / parts, "ramp": t_ramp}


def _cpu_sample_worker(args):
    from threadpoolctl import threadpool_limits

    g, seed = args
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        r = _cpu_sample(g, seed)
        r["wall"] = time.perf_counter() - t0
    return r


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, log, reps=3):
    """The FP64 oracle on the host cores, single-threaded (median of `reps` samples) and on all
    cores (one sample per core, run concurrently in worker processes, each single-threaded: the
    slices of a batch are independent).  Per-slice time of one step = R (prefilter + M partition
    forwards) + R# (M partition transposes + prefilter) + FBP (ramp + M transposes + prefilter)."""
    import statistics
    from concurrent.futures import ProcessPoolExecutor

    from threadpoolctl import threadpool_limits

    M = g["m"]

    def per_slice(r):
        return (r["q"] + M * r["fwd"]) + (M * r["adj"] + r["q"]) + (r["ramp"] + M * r["adj"] + r["q"])

    samples = []
    with threadpool_limits(limits=1):
        for k in range(reps):
            t0 = time.perf_counter()
            r = _cpu_sample(g, 303)
            r["wall"] = time.perf_counter() - t0
            samples.append(r)
            log(f"cpu sample {k}: {r}")
    st = statistics.median(per_slice(r) for r in samples)
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    cores = max(1, min(cores, os.cpu_count() or 1, 16))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores) as ex:
        par = list(ex.map(_cpu_sample_worker, [(g, 303 + i) for i in range(cores)]))
    wall = time.perf_counter() - t0
    # all-core throughput: `cores` slices' worth of samples finished in `wall` seconds; scale the
    # sample (one partition each way) to a whole step per slice
    sample_work = statistics.median(r["wall"] for r in par)
    per_slice_par = statistics.median(per_slice(r) for r in par)
    all_core = cores / (per_slice_par * wall / sample_work)
    return {
        "value": round(1.0 / st, 5),
        "unit": "slices/s",
        "cores": 1,
        "kind": "oracle",
        "all_core_value": round(all_core, 5),
        "all_core_cores": cores,
        "nproc": os.cpu_count(),
        "cpu_model": _cpu_model(),
        "sample": (f"one partition forward (with its polar evaluation) and one partition transpose of one "
                   f"{g['n']}x{g['n']} slice ({g['n_theta']}x{g['n_s']} sinogram), the prefilter and the ramp "
                   f"filter (timed on 1/16 of the rows), scaled to one step per slice (3 prefilters + {M} "
                   f"forward + {2 * M} transposed partitions + ramp); numpy FP64; value: median of {reps} "
                   f"single-thread samples ({st:.1f} s per slice); all_core_value: {cores} single-thread "
                   f"samples run concurrently in worker processes ({wall:.1f} s wall); plan-time kernel "
                   f"table excluded"),
    }


def em_detail(plan, f, sino, B, reps, time_op, detail, log):
    """One EM step (R, ratio, R#, update) on the whole batch; the normalisation R# chi_C is
    computed once, outside the timed region."""
    import torch
    from paper_1506_00014_amd import _lib

    em_norm = plan.em_norm()
    f_em = torch.ones_like(f)
    em_ws = torch.empty(plan.workspace_bytes(B, _lib.RL_OP_EM), dtype=torch.uint8, device=f.device)
    t_em = time_op(lambda: plan.em(sino, f_em, 1, norm=em_norm, ws=em_ws), reps)
    detail["per_op"]["EM step"] = {"batched_slices_per_s": round(B / (t_em / 1000.0), 1),
                                   "batched_ms_per_slice": round(t_em / B, 4)}
    log(f"EM step: {detail['per_op']['EM step']}")


def m_sweep_detail(n, time_op, log, batch=16, seed=405):
    """R and R# on `batch` slices of n x n (n angles x n bins) for M = 3, 4, 6, 8 partitions, with
    the FFT lengths at the smallest powers of two meeting their bounds and at the smallest 2^a 3^b
    (rl_geom_default's two policies; M sets N_rho, K and r)."""
    import torch
    from paper_1506_00014_amd import RadonPlan, _lib

    gen = torch.Generator(device="cuda").manual_seed(seed)
    f = torch.rand(batch, n, n, device="cuda", generator=gen)
    out = {}
    for m in (3, 4, 6, 8):
        for smooth in (False, True):
            plan = RadonPlan(n, n, n, m=m, smooth=smooth)
            ws = torch.empty(max(plan.workspace_bytes(batch, op) for op in (_lib.RL_OP_FWD, _lib.RL_OP_ADJ)),
                             dtype=torch.uint8, device="cuda")
            g = plan.forward(f, ws)
            tf = time_op(lambda: plan.forward(f, ws), 3)
            ta = time_op(lambda: plan.adjoint(g, ws), 3)
            geo = plan.geom
            key = f"{m}" + (" 2^a3^b" if smooth else "")
            out[key] = {"n_rho": geo["n_rho"], "k_theta": geo["k_theta"], "r_dec": geo["r_dec"],
                        "R_slices_per_s": round(batch / (tf / 1000.0), 1),
                        "R#_slices_per_s": round(batch / (ta / 1000.0), 1)}
            log(f"M={key}: {out[key]}")
            del plan, ws, g
    return out


def ragged_detail(torch, log, count=256, seed=401):
    """Ragged batch: `count` slices with N drawn from {256, 512, 768, 1024} (N x N sinograms),
    R and R# for the whole set as one replay of a captured graph vs one plain call per slice."""
    import numpy as np

    from paper_1506_00014_amd import RadonPlan, RaggedBatch

    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in rng.choice([256, 512, 768, 1024], size=count)]
    plans = {n: RadonPlan(n, n, n) for n in sorted(set(sizes))}
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    items = [(plans[n], torch.rand(n, n, generator=gen, device=dev), torch.empty(n, n, device=dev)) for n in sizes]
    batch = RaggedBatch(items)
    ws1 = {n: torch.empty(max(p.workspace_bytes(1, op) for op in (0, 1)), dtype=torch.uint8, device=dev)
           for n, p in plans.items()}
    out = {"slices": count, "sizes": {str(n): sizes.count(n) for n in sorted(set(sizes))}}
    for name, run, plain in (("R", batch.forward, lambda p, i, s: p.forward(i, ws1[i.shape[0]])),
                             ("R#", batch.adjoint, lambda p, i, s: p.adjoint(s, ws1[i.shape[0]]))):
        run()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            with torch.cuda.graph(graph, stream=st):
                run()
        torch.cuda.current_stream().wait_stream(st)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        graph.replay()
        ev0.record()
        for _ in range(3):
            graph.replay()
        ev1.record()
        torch.cuda.synchronize()
        t_graph = ev0.elapsed_time(ev1) / 3
        for p, i, s in items:
            plain(p, i, s)
        torch.cuda.synchronize()
        ev0.record()
        for p, i, s in items:
            plain(p, i, s)
        ev1.record()
        torch.cuda.synchronize()
        t_plain = ev0.elapsed_time(ev1)
        out[name] = {"graph_slices_per_s": round(count / (t_graph / 1000.0), 1),
                     "plain_slices_per_s": round(count / (t_plain / 1000.0), 1),
                     "graph_over_plain": round(t_plain / t_graph, 3)}
        log(f"ragged {name}: {out[name]}")
    return out


def graph_time(torch, fn, reps):
    """Mean ms of one replay of a HIP graph capturing fn() (the batch's kernels, enqueued once)."""
    fn()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(graph, stream=st):
            fn()
    torch.cuda.current_stream().wait_stream(st)
    graph.replay()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        graph.replay()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def c2_detail(torch, time_op, log, batch=64, n=1024, seed=201):
    """One 1024 x 1024 geometry (1024 angles x 1024 bins): R, R# and FBP timed separately on a
    batch (one graph replay each) and per slice (plain batch-1 calls)."""
    from paper_1506_00014_amd import RadonPlan, _lib

    plan = RadonPlan(n, n, n)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    f = torch.rand(batch, n, n, device="cuda", generator=gen)
    ws = torch.empty(max(plan.workspace_bytes(batch, op) for op in (0, 1, 2)), dtype=torch.uint8, device="cuda")
    ws1 = torch.empty(max(plan.workspace_bytes(1, op) for op in (0, 1, 2)), dtype=torch.uint8, device="cuda")
    g = plan.forward(f, ws)
    model = operator_model(plan.geom, plan.n_own(), plan.fine_samples(), batch)
    out = {"geometry": plan.geom, "batch": batch}
    for name, fb, f1 in (("R", lambda: plan.forward(f, ws), lambda i: plan.forward(f[i], ws1)),
                         ("R#", lambda: plan.adjoint(g, ws), lambda i: plan.adjoint(g[i], ws1)),
                         ("FBP", lambda: plan.fbp(g, ws), lambda i: plan.fbp(g[i], ws1))):
        tb = graph_time(torch, fb, 5)
        tp = time_op(lambda: [f1(i) for i in range(batch)], 1)
        rec = {"graph_slices_per_s": round(batch / (tb / 1000.0), 1),
               "plain_slices_per_s": round(batch / (tp / 1000.0), 1)}
        if name != "FBP":
            rec.update(roofline_fractions(model, tb / batch))
        out[name] = rec
        log(f"1024^2 {name}: {rec}")
    return out


def c5_detail(torch, log, count=64, n=2048, n_theta=1024, n_s=2048, steps=50, photons=1e4):
    """Batched least-squares reconstruction by autograd: `count` 30-ellipse phantoms of n x n, their
    analytic line integrals at n_theta x n_s as log Poisson data (photons per ray), `steps`
    gradient steps on ||R f - g||^2 from f = 0 with step 1 / (2 ||R^T R||) (20 power steps), and
    the relative error to the phantoms next to FBP's."""
    from paper_1506_00014_amd import RadonPlan, inputs, recon

    plan = RadonPlan(n, n_theta, n_s)
    t0 = time.perf_counter()
    phantoms, data = inputs.noisy_ellipse_stack(count, n, n_theta, n_s, 30, photons, torch.device("cuda", 0))
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    lam = 2.0 * recon.power_iteration(plan, 20, seed=502)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f = recon.least_squares_gd(plan, data, steps, lam, callback=lambda k, l: losses.append(l))
    torch.cuda.synchronize()
    t_gd = time.perf_counter() - t0
    pn = phantoms.norm()
    err = ((f - phantoms).norm() / pn).item()
    err_fbp = ((plan.fbp(data) - phantoms).norm() / pn).item()
    out = {"slices": count, "n": n, "n_theta": n_theta, "n_s": n_s, "photons_per_ray": photons, "steps": steps,
           "lambda": lam, "rel_error_gd": round(err, 4), "rel_error_fbp_ramlak": round(err_fbp, 4),
           "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
           "ms_per_step": round(t_gd * 1000.0 / steps, 3),
           "slice_steps_per_s": round(count * steps / t_gd, 1), "data_generation_s": round(t_data, 2)}
    log(f"reconstruction: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-ragged", action="store_true", help="skip the ragged-batch detail measurement")
    ap.add_argument("--no-m-sweep", action="store_true",
                    help="skip the R / R# rates at M = 3, 4, 6, 8 partitions")
    ap.add_argument("--no-c2", action="store_true", help="skip the 1024^2 R / R# / FBP timings")
    ap.add_argument("--no-c5", action="store_true", help="skip the batched least-squares reconstruction")
    ap.add_argument("--no-em", action="store_true",
                    help="skip the EM step measurement (its normalisation is a batch-1 back-projection)")
    ap.add_argument("--tune", action="append", default=[], metavar="FIELD=VALUE",
                    help="set an execution-only launch parameter of the 2048^2 plan (rl_tune field), e.g. adj_walk=1")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (FETCH_SIZE / WRITE_SIZE calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); slices are independent, so "
              "a multi-GPU run would shard the batch with no communication.", file=sys.stderr)
        sys.exit(2)

    import ctypes

    import torch

    from paper_1506_00014_amd import RadonPlan, _lib

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    n = args.n
    B = args.batch
    plan = RadonPlan(n, n, n)
    if args.tune:
        plan.tuning = {kv.split("=", 1)[0]: int(kv.split("=", 1)[1]) for kv in args.tune}
    g = plan.geom
    n_own = plan.n_own()
    gen = torch.Generator(device=dev)
    gen.manual_seed(303)
    f = torch.rand(B, n, n, generator=gen, device=dev, dtype=torch.float32)
    ws_bytes = max(plan.workspace_bytes(B, op) for op in (0, 1, 2))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    ws1 = torch.empty(max(plan.workspace_bytes(1, op) for op in (0, 1, 2)), dtype=torch.uint8, device=dev)
    lib = _lib.load()

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    log(f"plan {g}, batch {B}, workspace {ws_bytes / 2**30:.2f} GiB, launch parameters {plan.tuning}")

    def step():
        sino = plan.forward(f, ws)
        back = plan.adjoint(sino, ws)
        rec = plan.fbp(sino, ws)
        return sino, back, rec

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    K = args.steps
    _lib.check("rl_profile_start", lib.rl_profile_start(32 * K + 64))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.rl_profile_stop()
    log(f"timed {K} steps")
    ms_per_step = (t1 - t0) * 1000.0 / K
    value = B / (ms_per_step / 1000.0)

    # per-kernel durations (HIP events on the launch stream, over the timed region)
    per_kernel = {}
    name = ctypes.c_char_p()
    ms = ctypes.c_float()
    for i in range(lib.rl_profile_count()):
        _lib.check("rl_profile_record", lib.rl_profile_record(i, ctypes.byref(name), ctypes.byref(ms)))
        e = per_kernel.setdefault(name.value.decode(), [0, 0.0])
        e[0] += 1
        e[1] += ms.value
    kernels = {}
    for kname, (cnt, tot) in per_kernel.items():
        avg = tot / cnt
        by = kernel_bytes(kname, g, n_own, B)
        kernels[kname] = {"launches": cnt, "avg_ms": round(avg, 4), "ms_per_step": round(tot / K, 4),
                          "alg_bytes_per_launch": by, "alg_GBps": round(by / (avg * 1e-3) / 1e9, 1)}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    dk = kernels[dom]
    tr = measured_traffic(dom, B, n)
    if dom in ALG_FLOPS_PER_SAMPLE:
        # an interpolation kernel: bound by arithmetic issue, not by HBM (its bytes are in detail)
        flops = plan.fine_samples() * B * ALG_FLOPS_PER_SAMPLE[dom]
        achieved = flops / (dk["avg_ms"] * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                    "traffic": tr["bytes"] if tr else None, "alg_flops": flops,
                    "alg_bytes": dk["alg_bytes_per_launch"], "hbm_GBps": dk["alg_GBps"]}
    else:
        roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["alg_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(dk["alg_GBps"] / HBM_PEAK_GBS, 4), "traffic": tr["bytes"] if tr else None,
                    "alg_bytes": dk["alg_bytes_per_launch"]}
    if tr:
        roofline["traffic_detail"] = tr

    # per-operator rates, batched vs plain
    def time_op(fn, reps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    sino = plan.forward(f, ws)
    torch.cuda.synchronize()
    reps = max(1, K // 2)
    ops = {
        "R": (lambda: plan.forward(f, ws), lambda i: plan.forward(f[i], ws1)),
        "R#": (lambda: plan.adjoint(sino, ws), lambda i: plan.adjoint(sino[i], ws1)),
        "FBP": (lambda: plan.fbp(sino, ws), lambda i: plan.fbp(sino[i], ws1)),
        "FBP cosine": (lambda: plan.fbp(sino, ws, filter="cosine"), None),
        "FBP shepp-logan": (lambda: plan.fbp(sino, ws, filter="shepp-logan"), None),
        # the paper's fast back-projection (Algorithm 2) and FBP through it
        "R# (Alg. 2)": (lambda: plan.bp_lp(sino, ws), lambda i: plan.bp_lp(sino[i], ws1)),
        "FBP (Alg. 2)": (lambda: plan.fbp_lp(sino, ws), lambda i: plan.fbp_lp(sino[i], ws1)),
    }
    model = operator_model(g, n_own, plan.fine_samples(), B)
    detail = {"per_op": {}, "kernels": kernels, "model": model}
    for op, (batched, single) in ops.items():
        tb = graph_time(torch, batched, reps)
        te = time_op(batched, reps)
        rec = {"batched_slices_per_s": round(B / (tb / 1000.0), 1), "batched_ms_per_slice": round(tb / B, 4),
               "batched_eager_slices_per_s": round(B / (te / 1000.0), 1)}
        if op in ("R", "R#"):
            rec.update(roofline_fractions(model, tb / B))
        if single is not None and not args.no_plain:
            tp = time_op(lambda: [single(i) for i in range(B)], 1)
            rec["plain_slices_per_s"] = round(B / (tp / 1000.0), 1)
            rec["batched_over_plain"] = round(tp / tb, 3)
        detail["per_op"][op] = rec
        log(f"{op}: {rec}")
    # EM reconstruction: one step (R, ratio, R#, update) on the whole batch
    if not args.no_em:
        em_detail(plan, f, sino, B, reps, time_op, detail, log)
    if not args.no_m_sweep:
        detail["m_sweep"] = m_sweep_detail(n, time_op, log)
    if not args.no_c2:
        detail["c2_1024"] = c2_detail(torch, time_op, log)
    if not args.no_c5:
        detail["reconstruction"] = c5_detail(torch, log)
    if not args.no_ragged:
        detail["ragged_batch"] = ragged_detail(torch, log)
    detail["paper_context"] = ("GTX 770, CUDA 7, FP32, M=3, N_theta=1.5N: EM 100 steps on 2048 slices of 2048^2 "
                               "4.2e4 s (0.205 s per slice-step, 4.9 slice-steps/s); "
                               "R# 9.9e-2 s per 2048^2 slice "
                               "(10.1 slices/s); one R + one R# 0.205 s per slice (4.9 slices/s); context only")

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"R, R# and FBP (ramp) on a batch of {B} slices of {n}x{n}, "
                               f"{g['n_theta']} angles x {g['n_s']} bins, f ~ U[0,1]",
                   "n": n, "n_theta": g["n_theta"], "n_s": g["n_s"], "batch": B, "m": g["m"],
                   "n_rho": g["n_rho"], "k_theta": g["k_theta"], "r_dec": g["r_dec"],
                   "launch_parameters": plan.tuning},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(g, log)
    out["detail"] = detail
    print(json.dumps(out))


if __name__ == "__main__":
    main()
