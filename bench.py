"""Benchmark of the randomized Tucker hot path on one MI355X.

One step = one Sub-R-HOSVD of a resident tensor: the all-mode sampled
sketch, the batched CholeskyQR2 + W step, and the core projection (the one
full read of X).  Default workload: the FP32 256^4 tensor of multilinear
rank 32 (decay 0.8, relative noise 1e-4), target ranks 32, p = 10,
s_k = 10 n_k = 2560 sampled fibers per mode.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2|c3-bf16|c3-f16|c3-f32|c1|c4|c5|c6|c7|c8]

c8 is the same step on an FP32 tensor of uneven modes 5x10x12x112x80x270
with ranks (5, 8, 10, 28, 50, 150), p = 10, s_k = min(10 n_k, n_notk): the
last mode's sketch is 160 wide (the wide QR / W-step path).

c5 is Sub-R-RtL-HT on the FP32 18^8 tensor (balanced tree, node ranks 12,
p = 4, w_S = min(20 n, n_notS) sampled columns per node): node sketches,
QR + W per node, transfer tensors and the root contraction.  c6 is the same
on the closed-form tensor 1/||x|| over [1, 15]^8 in FP32 (node ranks 7); c7
the same with the serial tests' rule w_S = min(2^(d-2) n_S, n_notS), which
samples the root's two children densely.
Both also time the format's residual pass (htucker_reconstruct).

c4 is the batching form: 512 FP32 tensors of order 3-5 (n_k in [16, 96],
at most 2^24 entries each, ranks in [4, 16], p = 5), every mode of every
tensor and every tensor's reconstruction residual in one plan run, captured
in a HIP graph and replayed (its `value` counts X twice: core and residual).

Prints one JSON line.  `value` is tensor GB/s streamed per step:
(sum_k s_k n_k + prod n_k) * bytes / step time.  `roofline` is the streaming
pass of the core (its algorithmic bytes prod n_k * bytes per launch over its
HIP-event-timed average duration).  `cpu_baseline` is the FP64 oracle on a
bounded sample of the same workload on this host.
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

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--core", default="U", choices=["U", "Q"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--autotune-cache", default=None,
                    help="c4: JSON file of stored batch schedules keyed by shape class (read, then updated)")
    ap.add_argument("--cpu-slabs", type=int, default=12,
                    help="mode-0 slabs of X the oracle core baseline processes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for scaling the "
                         "FETCH_SIZE / WRITE_SIZE counters of the streaming pass)")
    return ap.parse_args()


# HBM bytes per launch of the streaming pass, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by a plain copy of known size; valid only for the
# kernel source it was taken on
# HBM traffic summaries of the streaming pass over X: the FP32 256^4 pass
# (the BF16-piece form, fused2x6_kernel)
TRAFFIC = {
    "x6": (os.path.join(ROOT, "profiles", "core_stream_x6_256x4_traffic.txt"),
           os.path.join(ROOT, "paper_2603_21379_amd", "csrc", "k_core_x6.hip")),
    # the uneven shape's pass over X: the middle-mode MFMA contraction (112 -> 28)
    "uneven": (os.path.join(ROOT, "profiles", "core_pass_mode_mfma_uneven_5x10x12x112x80x270_traffic.txt"),
               os.path.join(ROOT, "paper_2603_21379_amd", "csrc", "k_mode_f32.hip")),
    # the batched core pass (whole-slab form) of the 512-tensor batch
    "batch": (os.path.join(ROOT, "profiles", "batch_512_f32_order3to5_core_pass_traffic.txt"),
              os.path.join(ROOT, "paper_2603_21379_amd", "csrc", "k_batch.hip")),
    # the H-Tucker root pass at 18^8
    "root": (os.path.join(ROOT, "profiles", "htucker_root_pass_f32_18x8_traffic.txt"),
             os.path.join(ROOT, "paper_2603_21379_amd", "csrc", "k_root.hip")),
}
TRAFFIC_KEY = {"c8_": "uneven", "c4_": "batch", "c5_": "root"}


def measured_traffic(workload_name):
    """HBM bytes per launch from the committed counter summary of the kernel
    form that runs, or None when the summary is missing or the kernel source
    changed since the counters were taken."""
    import hashlib
    key = next((v for k, v in TRAFFIC_KEY.items() if workload_name.startswith(k)), "x6")
    path, src = TRAFFIC[key]
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if kv.get("kernel_source_sha256") != sha or kv.get("workload") != workload_name:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def streaming_ceiling(X, reps=5):
    """Read-only streaming reference over the same buffer in the same session
    (the library's stream_read kernel), in GB/s."""
    import torch
    from paper_2603_21379_amd import binding as B
    parts = torch.empty(B.stream_read_blocks(), dtype=torch.float64, device=X.device)
    B.stream_read(X, parts)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        B.stream_read(X, parts)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return X.numel() * X.element_size() / (ms * 1e-3) / 1e9


def device_draw_ms(ncols, ss, ells, fdt, reps=5):
    """Time of the seeded device-side draw of the same sketch shapes
    (indices and Omega for every mode), in ms."""
    import torch
    from paper_2603_21379_amd import binding as B
    B.draw_sketches(ncols, ss, ells, 1, omega_dtype=fdt)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for r in range(reps):
        B.draw_sketches(ncols, ss, ells, 2 + r, omega_dtype=fdt)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def backward_ms(X, F, G):
    """A7 on the resident tensor: the core VJP (factor gradients for a given
    core adjoint, X recontracted), the reconstruction VJP (X standing in for
    the adjoint of Xhat) and the whole backward of the projection loss
    ||X - R(C(X, F), F)||^2 (gradients of X and of every factor), each timed
    with events after a sizing call.
    FP32/FP64 tensors only (the backward entry points' dtypes)."""
    import torch
    from paper_2603_21379_amd import binding as B
    if X.dtype not in (torch.float32, torch.float64):
        return None
    Fb = [torch.empty_like(f) for f in F]
    Gb = torch.empty_like(G)
    dims = list(X.shape)
    out = {}
    Xb = torch.empty_like(X)
    for name, fn in (("ms_core_vjp", lambda: B.tucker_core_vjp(X, F, G, Fbar=Fb)),
                     ("ms_reconstruct_vjp", lambda: B.tucker_reconstruct_vjp(dims, G, F, X, Gbar=Gb, Fbar=Fb)),
                     ("ms_projection_loss_vjp", lambda: B.tucker_projection_loss_vjp(X, F, G, Xbar=Xb, Fbar=Fb))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(e0.elapsed_time(e1), 3)
    return out


def copy_calibration():
    import torch
    nbytes = 4 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}),
          flush=True)


def workload(name):
    from synthgen import configs
    table = {"c1": (configs.C1, "f64"), "c2": (configs.C2, "f32"),
             "c3-bf16": (configs.C3, "bf16"), "c3-f16": (configs.C3, "f16"),
             "c3-f32": (configs.C3, "f32"), "c8": (configs.C8, "f32")}
    if name not in table:
        raise SystemExit(f"unknown config {name}")
    return table[name]


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not a build)", file=sys.stderr)
        sys.exit(2)
    if args.config == "c4":
        bench_batch(args)
        return
    if args.config in ("c5", "c6", "c7"):
        bench_ht(args)
        return
    import numpy as np
    import torch

    import synthgen
    from paper_2603_21379_amd import binding as B
    from paper_2603_21379_amd import tucker as T

    cfg, dtype = workload(args.config)
    dims, ranks = cfg.dims, cfg.ranks
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
           "f16": torch.float16}[dtype]
    fdt = torch.float64 if dtype == "f64" else torch.float32
    esize = synthgen.itemsize(dtype)
    N = math.prod(dims)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t0 = time.time()
    log(f"generating {cfg.name} ({dtype}, {N * esize / 1e9:.2f} GB) on the host")
    inp = synthgen.tucker_tensor(dims, ranks, cfg.decay, cfg.noise, cfg=cfg.cfg_id, dtype=dtype)
    ells = synthgen.default_ell(dims, ranks, cfg.p)
    ss = synthgen.default_s(dims, cfg.alpha)
    omega_dt = synthgen.factor_dtype(dtype)
    t_sk = time.perf_counter()
    sk = synthgen.mode_sketches(dims, ells, ss, cfg=cfg.cfg_id, omega_dtype=omega_dt)
    ms_host_sketch = (time.perf_counter() - t_sk) * 1e3
    log(f"generated in {time.time() - t0:.1f}s; uploading")
    Xh = inp.X.view(np.int16) if dtype == "bf16" else inp.X
    X = torch.from_numpy(Xh).to(dev)
    if dtype == "bf16":
        X = X.view(torch.bfloat16)
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    skd = T.mode_sketches_to_device(sk, dims, dev, fdt)
    torch.cuda.synchronize()
    ms_upload_sketch = (time.perf_counter() - t_up) * 1e3

    d = len(dims)
    cols = list(ranks) if args.core == "U" else list(ells)
    Z = [torch.empty(n, e, dtype=torch.float64, device=dev) for n, e in zip(dims, ells)]
    Y = [torch.empty(n, s, dtype=tdt, device=dev) for n, s in zip(dims, ss)]
    F = [torch.empty(n, c, dtype=fdt, device=dev) for n, c in zip(dims, cols)]
    G = torch.empty(cols, dtype=fdt, device=dev)
    info = torch.zeros(d, dtype=torch.int32, device=dev)

    # one workspace for the whole step, sized by the library's own queries
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=dev)

    def step(wsb):
        B.tucker_sketch_all_modes(X, skd, Z, Y, ws=wsb)
        B.tucker_qr(Z, Y, r=cols, U=F, info=info, ws=wsb)
        B.tucker_core(X, F, G, ws=wsb)

    # size the workspace: the binding raises when it is smaller than what a
    # call's size query returns, so grow it to the largest of the three calls
    for _ in range(4):
        try:
            step(ws)
            break
        except ValueError as e:
            need = int(str(e).split("required ")[1])
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    log(f"workspace {ws.numel() / 1e9:.3f} GB; warmup {args.warmup}")
    for _ in range(args.warmup):
        step(ws)
    torch.cuda.synchronize()

    B.tk_profile_read(reset=True)
    B.tk_profile_enable(True)
    # events on the stream the library launches on (torch's current stream)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record()
        B.tucker_sketch_all_modes(X, skd, Z, Y, ws=ws)
        ev[i][1].record()
        B.tucker_qr(Z, Y, r=cols, U=F, info=info, ws=ws)
        ev[i][2].record()
        B.tucker_core(X, F, G, ws=ws)
        ev[i][3].record()
    torch.cuda.synchronize()
    t_stop = time.perf_counter()
    B.tk_profile_enable(False)
    core_ms, launches = B.tk_profile_read(reset=True)
    ms_per_step = (t_stop - t_start) * 1e3 / args.steps
    stage = [sum(e[j].elapsed_time(e[j + 1]) for e in ev) / args.steps for j in range(3)]
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step (sketch {stage[0]:.3f}, "
        f"qr+w {stage[1]:.3f}, core {stage[2]:.3f}); streaming pass "
        f"{core_ms / max(launches, 1):.3f} ms x {launches}")

    b_sketch = sum(s * n for s, n in zip(ss, dims)) * esize
    b_core = N * esize
    value = (b_sketch + b_core) / (ms_per_step * 1e-3) / 1e9
    core_avg_ms = core_ms / max(launches, 1)
    achieved = b_core / (core_avg_ms * 1e-3) / 1e9

    sketch_core_gbs = (b_sketch + b_core) / ((stage[0] + stage[2]) * 1e-3) / 1e9
    flops_core = core_flops(dims, cols)
    traffic = measured_traffic(cfg.name)

    # A5 (the residual ||X - G x_k F_k||^2, one fused pass over X), timed
    # separately; its value gives the GPU error
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    T.residual(X, G, F)   # first call sizes its workspace
    torch.cuda.synchronize()
    B.tk_profile_read(reset=True)
    B.tk_profile_enable(True)
    n_resid = 5
    e0.record()
    for _ in range(n_resid):
        r2 = T.residual(X, G, F)
    e1.record()
    torch.cuda.synchronize()
    B.tk_profile_enable(False)
    ms_resid = e0.elapsed_time(e1) / n_resid
    pass_ms, pass_launches = B.tk_profile_read(reset=True)
    ms_resid_pass = pass_ms / max(pass_launches, 1)
    r2h = r2.cpu()
    eps = math.sqrt(float(r2h[0]) / float(r2h[1]))
    info_h = info.cpu().tolist()
    log(f"eps_gpu = {eps:.6e}, info = {info_h}; residual {ms_resid:.3f} ms per call over "
        f"{n_resid} calls, of which the streaming pass {ms_resid_pass:.3f} ms "
        f"({b_core / (ms_resid_pass * 1e-3) / 1e9:.1f} GB/s)")
    ceiling = streaming_ceiling(X)
    log(f"read-only streaming reference over X: {ceiling:.1f} GB/s")
    ms_device_draw = device_draw_ms([N // n for n in dims], ss, ells, fdt)
    back = backward_ms(X, F, G)
    if back:
        log(f"backward (A7): core VJP {back['ms_core_vjp']:.2f} ms, reconstruction VJP "
            f"{back['ms_reconstruct_vjp']:.2f} ms, projection-loss backward "
            f"{back['ms_projection_loss_vjp']:.2f} ms")
    log(f"sketch operands: device draw {ms_device_draw:.3f} ms; host generation "
        f"{ms_host_sketch:.1f} ms + upload {ms_upload_sketch:.2f} ms")

    result = {
        "metric": "tensor GB/s streamed (sketch+core), frac of HBM roofline; rel err vs FP64 oracle",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "bf16": "bf16", "f16": "f16"}[dtype],
        "data": "synthetic",
        "config": {"workload": f"sub-r-hosvd {cfg.name}", "dims": list(dims),
                   "ranks": list(ranks), "p": cfg.p, "s": ss, "core_factor": args.core,
                   "decay": cfg.decay, "noise_rel": cfg.noise},
        "frac_hbm_step": round(value / HBM_PEAK_GBS, 4),
        "sketch_core": {"gbs": round(sketch_core_gbs, 1),
                        "frac_hbm": round(sketch_core_gbs / HBM_PEAK_GBS, 4),
                        "ms_sketch": round(stage[0], 4), "ms_qr_w": round(stage[1], 4),
                        "ms_core": round(stage[2], 4)},
        "core_tflops": round(flops_core / (stage[2] * 1e-3) / 1e12, 2),
        "rel_err_gpu": eps,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "core streaming pass",
                     "avg_ms": round(core_avg_ms, 4),
                     "bytes_per_launch": b_core,
                     "measured_ceiling": round(ceiling, 1),
                     "frac_of_ceiling": round(achieved / ceiling, 4)},
        "sketch_core_frac_of_ceiling": round(sketch_core_gbs / ceiling, 4),
        "ms_resid": round(ms_resid, 4),
        "ms_resid_pass": round(ms_resid_pass, 4),
        "backward": back,
        "sketch_draw": {"ms_device": round(ms_device_draw, 4),
                        "ms_host_generate": round(ms_host_sketch, 2),
                        "ms_upload": round(ms_upload_sketch, 3)},
        "resid_gbs": round(b_core / (ms_resid * 1e-3) / 1e9, 1),
    }
    del Y, Z
    torch.cuda.empty_cache()
    if not args.no_cpu:
        result["cpu_baseline"], Us_or = cpu_baseline(inp, sk, dims, ranks, cols, dtype, args, F)
        result["rel_err_vs_oracle"] = oracle_error(inp, Us_or, dtype, eps)
        log(f"eps_oracle = {result['rel_err_vs_oracle']['eps_oracle']:.6e}, "
            f"|eps_gpu - eps_oracle| / eps_oracle = {result['rel_err_vs_oracle']['rel_diff']:.2e}")
    print(json.dumps(result), flush=True)


def bench_batch(args):
    """Batching form: one step = one run of the batch plan (sketch, QR, W
    step, core of every mode and the reconstruction residual of all 512
    tensors), replayed from a graph."""
    import numpy as np
    import torch

    import synthgen
    from synthgen import configs
    from paper_2603_21379_amd import binding as B
    from paper_2603_21379_amd import tucker as T

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    specs = synthgen.batch_specs(configs.C4_COUNT, cfg=configs.C4_CFG_ID)
    total = sum(math.prod(sp.dims) for sp in specs)
    log(f"generating {len(specs)} tensors ({total * 4 / 1e9:.2f} GB FP32) on the host")
    X, U, G, sketches, ranks = [], [], [], [], []
    b_sketch = 0
    for i, sp in enumerate(specs):
        inp = synthgen.tucker_tensor(sp.dims, sp.ranks, 0.6, 1e-5, cfg=configs.C4_CFG_ID, dtype="f32", run=i)
        sk = synthgen.mode_sketches(sp.dims, sp.ells, sp.ss, cfg=configs.C4_CFG_ID, omega_dtype="f32", run=i)
        X.append(torch.from_numpy(inp.X).to(dev))
        sketches += T.mode_sketches_to_device(sk, sp.dims, dev, torch.float32)
        U += [torch.empty(n, r, dtype=torch.float32, device=dev) for n, r in zip(sp.dims, sp.ranks)]
        G.append(torch.empty(sp.ranks, dtype=torch.float32, device=dev))
        ranks.append(sp.ranks)
        b_sketch += sum(s * n for s, n in zip(sp.ss, sp.dims)) * 4
        del inp
    info = torch.zeros(len(U), dtype=torch.int32, device=dev)
    resid2 = torch.full((2 * len(specs),), float("nan"), dtype=torch.float64, device=dev)
    log(f"generated and uploaded in {time.time() - t0:.1f}s; planning")
    plan = B.BatchPlan(X, ranks, sketches, U, G, info, resid2=resid2)
    report = plan.autotune(cache=args.autotune_cache)
    log("autotune:\n" + report.strip())
    # eager runs with the streaming pass bracketed by the library's events
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    B.tk_profile_read(reset=True)
    B.tk_profile_enable(True)
    for _ in range(args.steps):
        plan.run()
    torch.cuda.synchronize()
    B.tk_profile_enable(False)
    core_ms, launches = B.tk_profile_read(reset=True)
    # one run captured in a graph, replayed for the timed steps
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.run(stream=s)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t_start) * 1e3 / args.steps
    b_core = total * 4
    # X is read by the sketch gathers, the core pass and the residual pass
    value = (b_sketch + 2 * b_core) / (ms_per_step * 1e-3) / 1e9
    core_avg = core_ms / max(launches, 1)
    achieved = b_core / (core_avg * 1e-3) / 1e9
    # error of every tensor from the last replay's own residual pass; a few
    # cross-checked against the single-tensor residual entry point
    r2h = resid2.cpu().numpy()
    errs = [math.sqrt(r2h[2 * i] / r2h[2 * i + 1]) for i in range(len(specs))]
    cross = 0.0
    m = 0
    for i, sp in enumerate(specs):
        d = len(sp.dims)
        if i < 16:
            e1 = T.rel_error(X[i], G[i], U[m:m + d])
            cross = max(cross, abs(errs[i] - e1) / e1)
        m += d
    log(f"timed {args.steps} graph replays: {ms_per_step:.3f} ms/step; streaming pass "
        f"{core_avg:.3f} ms; eps max {max(errs):.3e} median {float(np.median(errs)):.3e} "
        f"(vs single-tensor residual: {cross:.1e} relative); info nonzero {int((info != 0).sum())}")
    # QR / W-step flags of the modes (1, 2: a CholeskyQR pass was shifted; 4: a
    # Cholesky failed even with the shift; 8: the eigensolver ran out of sweeps)
    flags = {}
    for v in info.cpu().tolist():
        if v:
            flags[str(v)] = flags.get(str(v), 0) + 1
    result = {
        "metric": "tensor GB/s streamed (sketch+core+residual), frac of HBM roofline; rel err vs FP64 oracle",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched sub-r-hosvd, {len(specs)} tensors of order 3-5",
                   "entries": total, "p": 5, "decay": 0.6, "noise_rel": 1e-5, "graph": True},
        "frac_hbm_step": round(value / HBM_PEAK_GBS, 4),
        "rel_err_gpu": {"max": max(errs), "median": float(np.median(errs)), "from": "graph replay residual",
                        "vs_single_tensor_path": cross},
        "info_flags": flags,
        "autotune": report.strip().splitlines()[-1],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("c4_batch_512_f32_order3to5"),
                     "kernel": "batched streaming pass", "avg_ms": round(core_avg, 4),
                     "bytes_per_launch": b_core},
    }
    print(json.dumps(result), flush=True)


def bench_ht(args):
    """One step = one htucker_decompose of a resident FP32 tensor (18^8
    hierarchical rank 12, or the closed-form 15^8)."""
    import numpy as np
    import torch

    import synthgen
    from synthgen import configs
    from paper_2603_21379_amd import binding as B
    from paper_2603_21379_amd import tucker as T

    c = {"c5": configs.C5, "c6": configs.C6, "c7": configs.C7}[args.config]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    log(f"generating {c.name} on the host")
    if args.config in ("c6", "c7"):
        Xh = synthgen.inverse_norm_tensor(c.n, c.order, c.dtype)
        tr, dims = synthgen.balanced_tree(c.order), Xh.shape
    else:
        inp = synthgen.ht_tensor(c.n, c.order, c.rank, c.noise, cfg=c.cfg_id, dtype=c.dtype)
        tr, dims, Xh = inp.tree, inp.dims, inp.X
        del inp
    N = math.prod(dims)
    ranks, ells, ws = {}, {}, {}
    for t in range(1, tr.num_nodes):
        nS = math.prod(dims[k] for k in tr.modes(t))
        ells[t] = min(c.rank + c.p, nS, N // nS)
        ranks[t] = min(c.rank, ells[t])
        if c.sample_rule == "nS":
            ws[t] = min(c.w_alpha ** (c.order - 2) * nS, N // nS)
        else:
            ws[t] = min(c.w_alpha * c.n, N // nS)
    dense = [t for t in ws if ws[t] == N // math.prod(dims[k] for k in tr.modes(t))]
    if dense:
        log(f"dense nodes (every column sampled): {dense}")
    sk = synthgen.node_sketches(dims, tr, ells, ws, cfg=c.cfg_id, omega_dtype="f32")
    X = torch.from_numpy(Xh).to(dev)
    del Xh
    pairs = [(sk[t], N // math.prod(dims[k] for k in tr.modes(t))) for t in range(1, tr.num_nodes)]
    dsk = T.upload_sketches(pairs, dev, torch.float32)
    skd = {t: dsk[t - 1] for t in range(1, tr.num_nodes)}
    log(f"generated and uploaded in {time.time() - t0:.1f}s ({N * 4 / 1e9:.1f} GB)")
    res = T.sub_r_rtl_ht(X, tr, ranks, skd)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        T.sub_r_rtl_ht(X, tr, ranks, skd)
    torch.cuda.synchronize()
    B.tk_profile_read(reset=True)
    B.tk_profile_enable(True)
    t_start = time.perf_counter()
    for _ in range(args.steps):
        res = T.sub_r_rtl_ht(X, tr, ranks, skd)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t_start) * 1e3 / args.steps
    B.tk_profile_enable(False)
    root_ms, launches = B.tk_profile_read(reset=True)
    root_avg = root_ms / max(launches, 1)
    # a dense node reads X twice (its sketch and its W step); a sampled one
    # its gathered fibers
    b_sketch = sum(2 * N if t in dense else ws[t] * math.prod(dims[k] for k in tr.modes(t))
                   for t in ws) * 4
    b_root = N * 4
    value = (b_sketch + b_root) / (ms_per_step * 1e-3) / 1e9
    achieved = b_root / (root_avg * 1e-3) / 1e9
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step; root pass {root_avg:.3f} ms; "
        f"info {res.info.cpu().tolist()}")
    # the format's residual: nested bases, then one streaming pass over X
    leaves = {t: res.U[t] for t in res.U if tr.is_leaf(t)}
    T.ht_reconstruct(dims, tr, ranks, leaves, res.B, Xref=X)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(3):
        _, r2 = T.ht_reconstruct(dims, tr, ranks, leaves, res.B, Xref=X)
    e1.record()
    torch.cuda.synchronize()
    ms_resid = e0.elapsed_time(e1) / 3
    r2 = r2.cpu().tolist()
    eps = math.sqrt(r2[0] / r2[1])
    log(f"residual pass {ms_resid:.3f} ms ({N * 4 / ms_resid / 1e6:.1f} GB/s); rel err {eps:.4e}")
    # the format's VJP (gradients of the leaf bases and transfer tensors), X
    # standing in for the adjoint of the full tensor
    T.ht_reconstruct_vjp(dims, tr, ranks, leaves, res.B, X)
    torch.cuda.synchronize()
    e0.record()
    T.ht_reconstruct_vjp(dims, tr, ranks, leaves, res.B, X)
    e1.record()
    torch.cuda.synchronize()
    ms_vjp = e0.elapsed_time(e1)
    log(f"format VJP {ms_vjp:.3f} ms")
    result = {
        "metric": "tensor GB/s streamed (sketch+core), frac of HBM roofline; rel err vs FP64 oracle",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sub-r-rtl-ht {c.name}", "n": c.n, "order": c.order,
                   "node_rank": c.rank, "p": c.p, "w_alpha": c.w_alpha, "noise_rel": c.noise,
                   "sample_rule": c.sample_rule, "dense_nodes": dense},
        "frac_hbm_step": round(value / HBM_PEAK_GBS, 4),
        "rel_error": eps, "ms_resid": round(ms_resid, 4), "ms_format_vjp": round(ms_vjp, 3),
        "resid_gbs": round(N * 4 / ms_resid / 1e6, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(c.name),
                     "kernel": "root contraction pass", "avg_ms": round(root_avg, 4),
                     "bytes_per_launch": b_root},
    }
    print(json.dumps(result), flush=True)


def core_flops(dims, cols):
    """Algorithmic flops of the core projection contracting the last mode
    first: sum over k of 2 * prod(cols[k:]) * prod(dims[:k+1])."""
    d = len(dims)
    total = 0
    for k in range(d - 1, -1, -1):
        total += 2 * math.prod(dims[:k + 1]) * math.prod(cols[k:])
    return total


def cpu_baseline(inp, sk, dims, ranks, cols, dtype, args, F_gpu):
    """The FP64 oracle on a bounded sample: every mode's sketch, QR and W step
    at full size, and the core over the first `cpu_slabs` mode-0 slabs of X.
    Reported as the oracle's own tensor GB/s on that sample."""
    import numpy as np

    import oracle
    import synthgen
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        cores = len(os.sched_getaffinity(0))
    esize = synthgen.itemsize(dtype)
    to64 = (lambda a: synthgen.to_f64(a, dtype))
    t0 = time.perf_counter()
    Us = []
    for k in range(len(dims)):
        Y = oracle.gather_fibers(inp.X, k, sk[k].idx, to64=to64)
        Zk = oracle.range_sketch(Y, sk[k].omega)
        Q = oracle.orth(Zk)
        _, U, _ = oracle.w_step(Q, Y, cols[k])
        Us.append(U)
    t1 = time.perf_counter()
    slabs = min(args.cpu_slabs, dims[0])
    part = oracle.core_streamed(inp.X[:slabs], [Us[0][:slabs]] + Us[1:], to64=to64, slab=1)
    t2 = time.perf_counter()
    b_sketch = sum(len(s.idx) * n for s, n in zip(sk, dims)) * esize
    b_core = slabs * math.prod(dims[1:]) * esize
    dist = max(oracle.projector_distance(f.double().cpu().numpy(), u) for f, u in zip(F_gpu, Us))
    del part
    return ({"value": round((b_sketch + b_core) / (t2 - t0) / 1e9, 4), "unit": "GB/s",
             "cores": int(cores), "kind": "oracle",
             "sample": f"full sketch+QR+W of every mode, core over {slabs} of {dims[0]} mode-0 slabs",
             "sketch_s": round(t1 - t0, 3), "core_s": round(t2 - t1, 3),
             "max_projector_dist_gpu_vs_oracle": dist}, Us)


# gate of |eps_gpu - eps_oracle| / eps_oracle per tensor dtype
EPS_TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 3e-3, "f16": 3e-3}


def oracle_error(inp, Us, dtype, eps_gpu):
    """The error half of the metric: the oracle's end-to-end relative error
    (its own factors, the core of the whole tensor contracted last mode first
    over exactly upcast row chunks) beside the GPU's, at the full size.  With
    orthonormal FP64 factors ||X - X_hat||^2 = ||X||^2 - ||G||^2; below a
    relative error of 1e-4 that subtraction cancels, and the explicit
    residual is used instead (only the small FP64 workload is there)."""
    import oracle
    import synthgen
    to64 = (lambda a: synthgen.to_f64(a, dtype))
    t0 = time.perf_counter()
    G_or = oracle.core_chunked(inp.X, Us, to64=to64)
    try:
        eps_or = oracle.rel_error_orthonormal(G_or, oracle.sq_norm(inp.X, to64=to64))
        how = "||X||^2 - ||G||^2 (orthonormal FP64 factors)"
    except ValueError:
        eps_or = oracle.rel_error(inp.X, G_or, Us, to64=to64, slab=1)
        how = "explicit residual"
    rel = abs(eps_gpu - eps_or) / eps_or
    return {"eps_gpu": eps_gpu, "eps_oracle": eps_or, "rel_diff": rel,
            "tol": EPS_TOL[dtype], "within_tol": bool(rel <= EPS_TOL[dtype]),
            "oracle_error_form": how, "oracle_s": round(time.perf_counter() - t0, 2)}


if __name__ == "__main__":
    main()
