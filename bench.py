#!/usr/bin/env python3
"""Benchmark of the fast quaternion T-product on one MI355X.

One step = one whole T-product C = A * B on inputs already resident in HBM:
forward tube FFT of A and B, coupled facewise products, inverse tube FFT
(the three stages of qt_tprod, issued through the C-ABI one stage at a time
so that HIP events on the launch stream time each kernel).

Default workload: A, B of 1024 x 1024 x 32, components i.i.d. N(0, 1)
(seeds 3000/3001), FP32 path and bf16 hi+lo split path.  `value` is the
whole-step TFLOP/s-equivalent of the headline precision, with the
algorithmic count F = 32 m n s p (facewise products; the count of the proof
of Theorem 5.2 with additions) + 10 p log2(p) (mn + ns + ms) (two complex
length-p FFTs per quaternion tube, 5 N log2 N each).

Prints progress to stderr and ONE JSON line to stdout.
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

PEAK_TFLOPS = {"fp32": 157.3, "split_bf16": 2516.6, "split_fp16": 2516.6, "fp64": 78.6}
PEAK_HBM_GBPS = 8000.0

WORKLOADS = {
    "c1": dict(cfg=1, desc="A, B 8x8x8 quaternion, components N(0,1) (seeds 1000/1001)"),
    "c2": dict(cfg=2, desc="A, B 256x256x64 quaternion, components U[0,1) (seeds 2000/2001)"),
    "c3": dict(cfg=3, desc="A, B 1024x1024x32 quaternion, components N(0,1) (seeds 3000/3001)"),
    "c5": dict(cfg=5, desc="A 512x64x100, B 64x512x100 quaternion, components N(0,1) "
                           "(seeds 5000/5001)"),
    "c4": dict(cfg=4, desc="512 independent T-products, m,n,s ~ U{16..256}, p ~ U{8,12,16,30,32,45,64}, "
                           "N(0,1) (sizes seed 4000, problem i seed 4100000+i)"),
    "matvec": dict(cfg=6, desc="block-circulant quaternion mat-vec: A 2048x2048x16, B 2048x1x16 quaternion, "
                                "N(0,1) (seeds 6000/6001), coupled product on resident Fourier operands"),
    "complex": dict(cfg=3, desc="complex A, B 1024x1024x32 (planes Re, Im of the quaternion N(0,1) inputs, "
                                "seeds 3000/3001): one uncoupled complex product per frequency"),
    "real": dict(cfg=3, desc="real A, B 1024x1024x32 (plane 0 of the quaternion N(0,1) inputs, seeds 3000/3001): "
                          "Hermitian half spectrum, 17 complex products"),
    "chain": dict(cfg=3, desc="chain (A * B) * C, A, B, C 1024x1024x32 quaternion, N(0,1) "
                              "(seeds 3000/3001/3002), kept in the Fourier domain between the products"),
    "tsvd": dict(cfg=2, desc="quaternion t-SVD A = U * S * V^H of A 256x256x64, components U[0,1) "
                             "(seed 2000, the colour-video-like tensor)"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    """Host CPU model name (Linux), or the platform string."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def flops(m, n, s, p):
    f_gemm = 32.0 * m * n * s * p
    f_fft = 10.0 * p * math.log2(p) * (m * n + n * s + m * s) if p > 1 else 0.0
    return f_gemm, f_fft


COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "facewise_split_bf16_c3_hbm_counters.md")
KERNEL_SOURCES = ("facewise_impl.h", "facewise.hip", "qt_internal.h")


def measured_traffic(workload, precision):
    """Memory-side bytes per launch of the split product, from the committed
    FETCH_SIZE / WRITE_SIZE summary (calibrated against a plain copy); None
    when that summary does not cover this workload and precision or the
    kernel sources have changed since the counters were taken."""
    if workload != "c3" or precision != "split_bf16" or not os.path.exists(COUNTER_SUMMARY):
        return None
    fp = kernel_fingerprint()
    with open(COUNTER_SUMMARY) as fh:
        for line in fh:
            if line.startswith("traffic_bytes_per_launch:"):
                tok = line.split()
                if tok[3] == fp:
                    return float(tok[1])
    return None


def kernel_fingerprint():
    """SHA-1 of the product kernel's sources with comments and whitespace
    removed, so that only code changes invalidate a counter measurement."""
    import hashlib
    import re
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2212_14318_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--precisions", default="split_bf16,fp32",
                    help="comma list; the first is the headline `value`")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--backward", action="store_true",
                    help="c5: time forward + hand-written backward instead of the forward alone")
    ap.add_argument("--p", type=int, default=0,
                    help="c1 / c2 / c3: draw the inputs with this many faces instead (same shapes, seeds and "
                         "distribution), e.g. a prime p for the Bluestein transforms")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the short batch / backward / t-SVD runs")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this size first (HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only; the T-product runs on a single "
              "MI355X and --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2212_14318_amd import _native as nat
    from paper_2212_14318_amd import ops

    if not torch.cuda.is_available():
        print("bench.py: no ROCm GPU visible", file=sys.stderr)
        sys.exit(3)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream

    wl = WORKLOADS[args.workload]
    cfg = wl["cfg"]
    if args.workload == "c4":
        return _emit(bench_batched(args, wl, dev, stream))
    if args.workload == "c5" and args.backward:
        return _emit(bench_backward(args, wl, dev, stream))
    if args.workload == "tsvd":
        return _emit(bench_tsvd(args, wl, dev, stream))
    if args.workload == "chain":
        return bench_chain(args, wl, dev, stream)
    if args.workload == "matvec":
        return bench_matvec(args, wl, dev, stream)
    if args.workload in ("complex", "real"):
        return bench_complex(args, wl, dev, stream, real=args.workload == "real")
    t0 = time.time()
    if args.p:
        if cfg not in (1, 2, 3):
            print("bench.py: --p applies to the c1, c2 and c3 workloads", file=sys.stderr)
            sys.exit(2)
        c = synth.CONFIGS[cfg]
        A64 = synth.quat_tensor(c["m"], c["n"], args.p, 1000 * cfg, c["dist"])
        B64 = synth.quat_tensor(c["n"], c["s"], args.p, 1000 * cfg + 1, c["dist"])
        wl = dict(wl, desc=wl["desc"].replace(f"x{c['p']} ", f"x{args.p} ").replace(
            f"x{c['p']} quaternion", f"x{args.p} quaternion") + f" (p = {args.p})")
    else:
        inputs = synth.config_inputs(cfg)
        A64, B64 = inputs[0], inputs[1]
    _, p, m, n = A64.shape
    s = B64.shape[3]
    log(f"[bench] inputs {args.workload} m={m} n={n} s={s} p={p} drawn in {time.time() - t0:.1f}s")
    lda, ldb = nat.qt_fourier_ld(n), nat.qt_fourier_ld(s)

    def make_buffers(dt):
        """Inputs in the dtype of a precision (FP64 for fp64, else FP32), their
        Fourier buffers, and input/output sets rotated from step to step so
        that the spatial tensors of a small workload are not still in the
        256 MB Infinity Cache from the previous step (at least 768 MiB of A, B,
        C across the sets, at most 16 sets)."""
        A = torch.from_numpy(A64).to(dev, dt)
        B = torch.from_numpy(B64).to(dev, dt)
        C = torch.empty((4, p, m, s), dtype=dt, device=dev)
        set_bytes = (A.numel() + B.numel() + C.numel()) * A.element_size()
        nsets = min(16, max(1, -(-(768 << 20) // set_bytes)))
        return dict(
            bufs=[(A, B, C)] + [(A.clone(), B.clone(), torch.empty_like(C)) for _ in range(nsets - 1)],
            nsets=nsets,
            Ah=torch.empty((4, p, m, lda), dtype=dt, device=dev),
            Bh=torch.empty((4, p, n, ldb), dtype=dt, device=dev),
            Ch=torch.empty((4, p, m, ldb), dtype=dt, device=dev))

    cur = make_buffers(torch.float32)
    f_gemm, f_fft = flops(m, n, s, p)
    F = f_gemm + f_fft
    fft_fwd_bytes = 32.0 * p * (m * n + n * s)       # read + write 16 B per quaternion
    fft_inv_bytes = 32.0 * p * (m * s)

    if args.copy_calib_mib:
        nb = args.copy_calib_mib << 20
        src = torch.empty(nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {nb} bytes read + {nb} bytes written")
        del src, dst

    def stage_calls(prec_id, ev, k=0):
        # forward transforms in the operand format of the precision (split-bf16:
        # hi/lo words), product, inverse transform of the FP32 product
        A, B, C = cur["bufs"][k % cur["nsets"]]
        Ah, Bh, Ch = cur["Ah"], cur["Bh"], cur["Ch"]
        st = nat.qt_tube_fft(m, n, p, A.data_ptr(), n, Ah.data_ptr(), lda, 0, prec_id, sh)
        nat.check(st, "qt_tube_fft(A)")
        st = nat.qt_tube_fft(n, s, p, B.data_ptr(), s, Bh.data_ptr(), ldb, 0, prec_id, sh)
        nat.check(st, "qt_tube_fft(B)")
        ev[0].record(stream)
        st = nat.qt_fourier_tprod(m, n, s, p, Ah.data_ptr(), lda, Bh.data_ptr(), ldb,
                                  Ch.data_ptr(), ldb, prec_id, sh)
        nat.check(st, "qt_fourier_tprod")
        ev[1].record(stream)
        inv_id = nat.QT_FP64 if prec_id == nat.QT_FP64 else nat.QT_FP32
        st = nat.qt_tube_fft(m, s, p, Ch.data_ptr(), ldb, C.data_ptr(), s, 1, inv_id, sh)
        nat.check(st, "qt_tube_fft(C^, inverse)")

    results = {}
    precs = [x for x in args.precisions.split(",") if x]
    for prec in precs:
        prec_id = nat.PRECISIONS[prec]
        dt = torch.float64 if prec == "fp64" else torch.float32
        if cur["Ah"].dtype != dt:
            cur = None
            torch.cuda.empty_cache()
            cur = make_buffers(dt)
        bufs, nsets = cur["bufs"], cur["nsets"]
        A, B, C = bufs[0]
        # check the staged path against the single entry point once (untimed)
        ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        try:
            C_ref = ops.tprod(A, B, precision=prec)
        except nat.QtError as e:
            log(f"[bench] precision {prec} not available: {e}")
            continue
        try:
            stage_calls(prec_id, ev0)
        except nat.QtError as e:
            # split fp16 needs per-call scales and has no staged entry points: time
            # whole qt_tprod calls (no per-kernel split for this precision)
            log(f"[bench] {prec}: staged path not available ({e}); timing whole qt_tprod calls")
            del C_ref
            for k in range(args.warmup):
                Ak, Bk, Ck = bufs[k % nsets]
                ops.tprod(Ak, Bk, precision=prec, out=Ck)
            torch.cuda.synchronize()
            t_start = time.perf_counter()
            for k in range(args.steps):
                Ak, Bk, Ck = bufs[k % nsets]
                ops.tprod(Ak, Bk, precision=prec, out=Ck)
            torch.cuda.synchronize()
            ms_step = (time.perf_counter() - t_start) * 1e3 / args.steps
            results[prec] = dict(ms_per_step=ms_step, tflops_equiv=F / (ms_step * 1e-3) / 1e12,
                                 C=bufs[(args.steps - 1) % nsets][2].cpu().numpy())
            log(f"[bench] {prec}: {ms_step:.3f} ms/step  {results[prec]['tflops_equiv']:.1f} TFLOP/s-equiv"
                f"  (whole qt_tprod)")
            continue
        torch.cuda.synchronize()
        same = bool(torch.equal(C, C_ref))
        del C_ref
        for k in range(args.warmup):
            stage_calls(prec_id, ev0, k)
        torch.cuda.synchronize()
        marks = []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(args.steps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record(stream)
            stage_calls(prec_id, (e[1], e[2]), k)
            e[3].record(stream)
            marks.append(e)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        fwd = [mk[0].elapsed_time(mk[1]) for mk in marks]
        gem = [mk[1].elapsed_time(mk[2]) for mk in marks]
        inv = [mk[2].elapsed_time(mk[3]) for mk in marks]
        ms_step = wall * 1e3 / args.steps
        t_gemm = sum(gem) / len(gem)
        t_fwd = sum(fwd) / len(fwd)
        t_inv = sum(inv) / len(inv)
        # sampled error against the FP64 oracle is computed after all GPU timing
        results[prec] = dict(
            ms_per_step=ms_step, tflops_equiv=F / (ms_step * 1e-3) / 1e12,
            gemm_ms=t_gemm, fft_fwd_ms=t_fwd, fft_inv_ms=t_inv,
            gemm_tflops=f_gemm / (t_gemm * 1e-3) / 1e12,
            fft_fwd_gbps=fft_fwd_bytes / (t_fwd * 1e-3) / 1e9,
            fft_inv_gbps=fft_inv_bytes / (t_inv * 1e-3) / 1e9,
            staged_equals_qt_tprod=same,
            C=bufs[(args.steps - 1) % nsets][2].cpu().numpy(),
        )
        log(f"[bench] {prec}: {ms_step:.3f} ms/step  {results[prec]['tflops_equiv']:.1f} TFLOP/s-equiv"
            f"  gemm {t_gemm:.3f} ms ({results[prec]['gemm_tflops']:.1f} TF)"
            f"  fft {t_fwd:.3f}+{t_inv:.3f} ms  staged==qt_tprod: {same}")

    if not results:
        print("bench.py: no precision could run", file=sys.stderr)
        sys.exit(4)

    # ---- accuracy: sampled relative Frobenius error vs the FP64 oracle ----
    import oracle
    rng = np.random.Generator(np.random.PCG64(31337))
    per_face = 12
    kk = np.repeat(np.arange(p), per_face)
    ii = rng.integers(0, m, kk.size)
    jj = rng.integers(0, s, kk.size)
    ref = oracle.tprod_entries(A64, B64, kk, ii, jj)
    for prec, r in results.items():
        got = r.pop("C")[:, kk, ii, jj].astype(np.float64)
        r["rel_err"] = float(np.sqrt(np.sum((got - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)))
        log(f"[bench] {prec}: sampled rel. Frobenius error vs FP64 oracle = {r['rel_err']:.3e}")

    # ---- CPU baseline: the oracle itself on a bounded sample of the job ----
    cpu = cpu_fft = None
    if not args.no_cpu_baseline:
        import threadpoolctl
        np.ones((8, 8)) @ np.ones((8, 8))
        threads = max([d.get("num_threads", 1) for d in threadpoolctl.threadpool_info()] or [1])
        faces_done = 0
        t0 = time.perf_counter()
        while faces_done < p and time.perf_counter() - t0 < args.cpu_seconds:
            oracle.tprod_faces(A64, B64, [faces_done])
            faces_done += 1
        t_cpu = time.perf_counter() - t0
        frac = faces_done / p
        cpu = {"value": F * frac / t_cpu / 1e12, "unit": "TFLOP/s-equiv", "cores": int(threads),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{faces_done} of {p} output faces of the same workload (FP64 "
                         f"definition, block-row form), {t_cpu:.1f} s; value = F x {faces_done}/{p} / time"}
        log(f"[bench] oracle CPU baseline: {cpu['value']:.4g} TFLOP/s-equiv on {threads} threads "
            f"({faces_done} faces in {t_cpu:.1f}s)")
        # the paper's FFT-based Algorithm 5.1 on the host, whole workload, in FP64
        # (complex128) and FP32 (complex64)
        cpu_fft = {}
        for label, cdt in (("fp64", np.complex128), ("fp32", np.complex64)):
            t0 = time.perf_counter()
            Cf = oracle.tprod_fft(A64, B64, dtype=cdt)
            t_fft = time.perf_counter() - t0
            err_fft = float(np.sqrt(np.sum((Cf[:, kk, ii, jj] - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)))
            del Cf
            cpu_fft[label] = {"value": F / t_fft / 1e12, "unit": "TFLOP/s-equiv", "cores": int(threads),
                              "kind": "oracle_fft", "cpu_model": cpu_model(),
                              "sample": f"whole workload by Algorithm 5.1 (numpy FFT + {np.dtype(cdt).name} "
                                        f"products), {t_fft:.1f} s, sampled rel. error vs the definition "
                                        f"{err_fft:.1e}"}
            log(f"[bench] CPU FFT-based (Algorithm 5.1, {label}): {cpu_fft[label]['value']:.4g} "
                f"TFLOP/s-equiv on {threads} threads ({t_fft:.1f}s, rel err {err_fft:.1e})")

    head = precs[0] if precs[0] in results else next(iter(results))
    r = results[head]
    peak = PEAK_TFLOPS[head]
    staged = "gemm_tflops" in r
    roof = None if not staged else {"bound": "mfma", "achieved": round(r["gemm_tflops"], 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(r["gemm_tflops"] / peak, 4),
            "traffic": measured_traffic(args.workload, head),
            "kernel": "facewise coupled product (qt_fourier_tprod)",
            "algorithmic_flops_per_launch": f_gemm,
            "algorithmic_bytes_per_launch": 16.0 * p * (m * n + n * s + m * s)}
    if staged and head.startswith("split"):
        roof["issued_frac"] = round(3 * r["gemm_tflops"] / peak, 4)
    dtype = {"fp32": "f32", "split_bf16": "bf16x3-split/f32-acc", "split_fp16": "fp16x3-split/f32-acc",
             "fp64": "f64"}[head]
    out = {
        "metric": "T-product TFLOP/s-equiv & % roofline, split-BF16 vs FP32 at stated rel. error",
        "value": round(r["tflops_equiv"], 3),
        "unit": "TFLOP/s-equiv",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": wl["desc"], "m": m, "n": n, "s": s, "p": p, "precision": head,
                   "input_sets": nsets,
                   "flops_per_step": F},
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_fft_baseline": cpu_fft,
        "per_precision": {k: {kk2: (float(f"{v:.5g}") if isinstance(v, float) else v)
                              for kk2, v in d.items()} for k, d in results.items()},
        "fft_roofline": None if not staged else {
            "bound": "hbm", "fwd_achieved": round(r["fft_fwd_gbps"], 1),
            "inv_achieved": round(r["fft_inv_gbps"], 1), "peak": PEAK_HBM_GBPS,
            "unit": "GB/s", "fwd_frac": round(r["fft_fwd_gbps"] / PEAK_HBM_GBPS, 4),
            "inv_frac": round(r["fft_inv_gbps"] / PEAK_HBM_GBPS, 4)},
    }
    if "fp32" in results and head != "fp32":
        out["speedup_vs_fp32"] = round(results["fp32"]["ms_per_step"] / r["ms_per_step"], 3)
    if "fp32" in results and "gemm_tflops" in results["fp32"]:
        # the FP32 tiles form each complex product with three real products, so
        # the MFMA pipe issues 24 m n s p flops for the 32 m n s p counted
        r32 = results["fp32"]["gemm_tflops"]
        out["fp32_roofline"] = {"bound": "mfma", "achieved": round(r32, 3), "peak": PEAK_TFLOPS["fp32"],
                                "unit": "TFLOP/s", "frac": round(r32 / PEAK_TFLOPS["fp32"], 4),
                                "issued_frac": round(0.75 * r32 / PEAK_TFLOPS["fp32"], 4),
                                "issued_flops_per_launch": 24.0 * m * n * s * p,
                                "note": "frac counts 32 m n s p algorithmic flops; three real products per "
                                        "complex product issue 0.75 of that on the MFMA pipe"}
    if not args.no_extras:
        out["extra_workloads"] = extra_workloads(args, dev, stream)
    print(json.dumps(out), flush=True)


def extra_workloads(args, dev, stream):
    """Shorter runs of the batch, differentiation and t-SVD workloads, so that
    one bench line carries their times too."""
    import copy
    sub = copy.copy(args)
    sub.steps, sub.warmup = 20, 5
    extras = {}
    for name, fn in (("c4", bench_batched), ("c5_fwd_bwd", bench_backward), ("tsvd", bench_tsvd)):
        wl = WORKLOADS["c5" if name == "c5_fwd_bwd" else name]
        sub.precisions = "fp32" if name == "tsvd" else args.precisions
        sub.no_cpu_baseline = True
        try:
            res = fn(sub, wl, dev, stream)
        except Exception as e:      # report, never hide the headline
            log(f"[bench] extra workload {name} failed: {e}")
            extras[name] = {"error": str(e)}
            continue
        extras[name] = {"workload": res["config"]["workload"], "steps": sub.steps,
                        "per_precision": res["per_precision"], "roofline": res.get("roofline")}
    return extras


def _emit(out):
    print(json.dumps(out), flush=True)


def bench_batched(args, wl, dev, stream):
    """Batched workload: replays of one captured plan (one hipGraphLaunch per
    step) over 512 problems; value = sum of per-problem F / time per replay."""
    import numpy as np
    import torch

    import synth
    from paper_2212_14318_amd import BatchedPlan, autotune

    sizes = synth.batch_problem_sizes()
    As, Bs = [], []
    F = 0.0
    for i, (m, n, s, p) in enumerate(sizes):
        A, B = synth.batch_problem_inputs(i, int(m), int(n), int(s), int(p))
        As.append(torch.from_numpy(A).to(dev, torch.float32))
        Bs.append(torch.from_numpy(B).to(dev, torch.float32))
        fg, ff = flops(int(m), int(n), int(s), int(p))
        F += fg + ff
    log(f"[bench] c4: {len(sizes)} problems resident, F = {F:.4e}")
    res = {}
    precs = [x for x in args.precisions.split(",") if x]
    for prec in precs:
        autotune(prec)
        plan = BatchedPlan(As, Bs, prec)
        for _ in range(args.warmup):
            plan.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.launch()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        res[prec] = {"ms_per_step": ms, "tflops_equiv": F / (ms * 1e-3) / 1e12}
        plan.close()
        log(f"[bench] c4 {prec}: {ms:.3f} ms per replay, {res[prec]['tflops_equiv']:.1f} TFLOP/s-equiv")
    head = precs[0]
    return {"metric": "T-product TFLOP/s-equiv & % roofline, split-BF16 vs FP32 at stated rel. error",
            "value": round(res[head]["tflops_equiv"], 3), "unit": "TFLOP/s-equiv", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res[head]["ms_per_step"], 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16x3-split/f32-acc" if head == "split_bf16" else "f32", "data": "synthetic",
            "config": {"workload": wl["desc"], "precision": head, "flops_per_step": F},
            "per_precision": res, "roofline": None, "cpu_baseline": None}


def bench_backward(args, wl, dev, stream):
    """Differentiation workload: one step = forward C = A * B, G = C - T, and
    the hand-written backward dA = G * B^H, dB = A^H * G."""
    import torch

    import synth
    from paper_2212_14318_amd import tprod, tprod_backward

    A64, B64, T64 = synth.config_inputs(5)
    _, p, m, n = A64.shape
    s = B64.shape[3]
    A = torch.from_numpy(A64).to(dev, torch.float32)
    B = torch.from_numpy(B64).to(dev, torch.float32)
    T = torch.from_numpy(T64).to(dev, torch.float32)
    fg, ff = flops(m, n, s, p)
    F = (fg + ff) + 2 * fg + ff + 10.0 * p * math.log2(p) * (m * n + n * s)
    res = {}
    precs = [x for x in args.precisions.split(",") if x]
    for prec in precs:
        def step():
            C = tprod(A, B, prec)
            G = C.sub_(T)
            return tprod_backward(A, B, G, prec)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        res[prec] = {"ms_per_step": ms, "tflops_equiv": F / (ms * 1e-3) / 1e12}
        log(f"[bench] c5 fwd+bwd {prec}: {ms:.3f} ms/step, {res[prec]['tflops_equiv']:.1f} TFLOP/s-equiv")
    head = precs[0]
    return {"metric": "T-product TFLOP/s-equiv & % roofline, split-BF16 vs FP32 at stated rel. error",
            "value": round(res[head]["tflops_equiv"], 3), "unit": "TFLOP/s-equiv", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res[head]["ms_per_step"], 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16x3-split/f32-acc" if head == "split_bf16" else "f32", "data": "synthetic",
            "config": {"workload": wl["desc"] + " + backward", "precision": head, "flops_per_step": F},
            "per_precision": res, "roofline": None, "cpu_baseline": None}


def svd_flops(rows, cols):
    """Operation count of a complex SVD with both singular-vector sets, rows
    >= cols: the real count 4 r^2 c + 8 r c^2 + 9 c^3 (Golub and Van Loan's
    R-SVD) times 4 real operations per complex one."""
    return 4.0 * (4.0 * rows * rows * cols + 8.0 * rows * cols * cols + 9.0 * cols ** 3)


def tsvd_flops(m, n, p):
    """Algorithmic work of the t-SVD's Fourier-domain stage: one complex SVD of the
    2 max(m,n) x 2 min(m,n) matrix chi_f(A) per pair {f, -f} with f != -f, and
    half of that for each self-paired frequency (a quaternion SVD of half the
    size: an eighth of the elements at four times the operations each)."""
    r, c = max(m, n), min(m, n)
    selfp = 1 if p % 2 else 2
    pairs = p // 2 + 1 - selfp
    return (pairs + 0.5 * selfp) * svd_flops(2 * r, 2 * c)


def bench_tsvd(args, wl, dev, stream):
    """t-SVD workload: one step = qt_tsvd (tube FFT, Jacobi sweeps per
    frequency pair, S^ fill, inverse FFTs of U^, V^, S^).  The Fourier-domain
    stage (preparation, block-sweep rounds, finish) is timed on its own through
    qt_fourier_tsvd on the transformed input; its roofline is the FP32 vector
    ALU (the Jacobi sweeps are column updates in VALU on columns staged in
    LDS), reported against the SVD operation count."""
    import numpy as np
    import torch

    import oracle
    import synth
    from oracle import tsvd as ots
    from paper_2212_14318_amd import _native as nat

    A64 = synth.config_inputs(2)[0]
    _, p, m, n = A64.shape
    F = tsvd_flops(m, n, p)
    res = {}
    precs = [x for x in args.precisions.split(",") if x]
    if precs and precs[0].startswith("split"):
        precs = ["fp32"]
    sh = stream.cuda_stream
    ref_sig = None
    for prec in precs:
        P = nat.PRECISIONS[prec]
        dt = torch.float64 if prec == "fp64" else torch.float32
        A = torch.from_numpy(A64).to(dev, dt)
        k = min(m, n)
        U = torch.empty((4, p, m, m), dtype=dt, device=dev)
        S = torch.empty((4, p, m, n), dtype=dt, device=dev)
        V = torch.empty((4, p, n, n), dtype=dt, device=dev)
        sig = torch.empty((p, k), dtype=dt, device=dev)
        need = nat.qt_tsvd_workspace_size(m, n, p, P)
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        lda, ldu = nat.qt_fourier_ld(n), nat.qt_fourier_ld(m)
        Ah = torch.empty((4, p, m, lda), dtype=dt, device=dev)
        Uh = torch.empty((4, p, m, ldu), dtype=dt, device=dev)
        Vh = torch.empty((4, p, n, lda), dtype=dt, device=dev)
        sig2 = torch.empty_like(sig)
        pneed = nat.qt_fourier_tsvd_workspace_size(m, n, p, P)
        pws = torch.empty(pneed, dtype=torch.uint8, device=dev)

        def whole():
            nat.check(nat.qt_tsvd(m, n, p, A.data_ptr(), U.data_ptr(), S.data_ptr(), V.data_ptr(), sig.data_ptr(),
                                  P, ws.data_ptr(), need, sh), "qt_tsvd")

        def pairs():
            nat.check(nat.qt_fourier_tsvd(m, n, p, Ah.data_ptr(), lda, Uh.data_ptr(), ldu, Vh.data_ptr(), lda,
                                          sig2.data_ptr(), P, pws.data_ptr(), pneed, sh), "qt_fourier_tsvd")

        nat.check(nat.qt_tube_fft(m, n, p, A.data_ptr(), n, Ah.data_ptr(), lda, 0, P, sh), "qt_tube_fft")
        steps, warm = max(1, min(args.steps, 10)), max(1, min(args.warmup, 2))
        times = {}
        for name, fn in (("whole", whole), ("pairs", pairs)):
            for _ in range(warm):
                fn()
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(stream)
            for _ in range(steps):
                fn()
            ev[1].record(stream)
            torch.cuda.synchronize()
            times[name] = ev[0].elapsed_time(ev[1]) / steps
        if ref_sig is None:
            ref_sig = ots.tsvd(A64)[3]
        got = sig.double().cpu().numpy()
        err = float(np.abs(got - ref_sig).max() / ref_sig.max())
        same = bool(torch.equal(sig, sig2))
        res[prec] = {"ms_per_step": times["whole"], "pair_kernel_ms": times["pairs"],
                     "pair_kernel_tflops": F / (times["pairs"] * 1e-3) / 1e12,
                     "sigma_max_rel_err": err, "stage_equals_qt_tsvd": same, "steps": steps}
        log(f"[bench] tsvd {prec}: {times['whole']:.3f} ms per qt_tsvd, Fourier-domain stage {times['pairs']:.3f} ms "
            f"({res[prec]['pair_kernel_tflops']:.3f} TFLOP/s of SVD work), sigma err {err:.2e}")
    head = precs[0]
    r = res[head]
    cpu = None
    if not getattr(args, "no_cpu_baseline", False):
        import threadpoolctl
        threads = max([d.get("num_threads", 1) for d in threadpoolctl.threadpool_info()] or [1])
        t0 = time.perf_counter()
        ots.tsvd(A64)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": F / t_cpu / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"the whole workload by the oracle's t-SVD (numpy complex128 SVD per frequency pair), "
                         f"{t_cpu:.1f} s"}
    peak = PEAK_TFLOPS["fp32"] if head == "fp32" else PEAK_TFLOPS["fp64"]
    return {"metric": "T-product TFLOP/s-equiv & % roofline, split-BF16 vs FP32 at stated rel. error",
            "value": round(F / (r["ms_per_step"] * 1e-3) / 1e12, 4), "unit": "TFLOP/s", "n_gpus": 1,
            "steps": r["steps"], "warmup": 2, "ms_per_step": round(r["ms_per_step"], 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if head == "fp32" else "f64", "data": "synthetic",
            "config": {"workload": wl["desc"], "precision": head, "svd_flops_per_step": F},
            "roofline": {"bound": "alu", "achieved": round(r["pair_kernel_tflops"], 4), "peak": peak,
                         "unit": "TFLOP/s", "frac": round(r["pair_kernel_tflops"] / peak, 5), "traffic": None,
                         "kernel": "t-SVD Fourier-domain stage (qt_fourier_tsvd: prep, block-sweep rounds, finish)"},
            "per_precision": res, "cpu_baseline": cpu}


def bench_chain(args, wl, dev, stream):
    """Fourier-domain-resident chain D = (A * B) * C: three forward transforms,
    two coupled products (split-bf16: the FP32 intermediate is turned into
    operand words in place) and one inverse transform, against two qt_tprod
    calls.  value = F(A * B) + F((A * B) * C) over the resident chain's time."""
    import torch

    import synth
    from paper_2212_14318_amd import _native as nat
    from paper_2212_14318_amd import fourier_tprod, split_words, tprod, tube_fft

    A64, B64 = synth.config_inputs(3)[:2]
    _, p, m, n = A64.shape
    C64 = synth.quat_tensor(n, n, p, seed=3002)
    A, B, C = (torch.from_numpy(x).to(dev, torch.float32) for x in (A64, B64, C64))
    ld = nat.qt_fourier_ld(n)
    Ah, Bh, Ch = (torch.empty((4, p, n, ld), device=dev) for _ in range(3))
    D = torch.empty((4, p, n, n), device=dev)
    fg, ff = flops(n, n, n, p)
    F = 2 * (fg + ff)
    res = {}
    precs = [x for x in args.precisions.split(",") if x]
    for prec in precs:
        def resident():
            tube_fft(A, precision=prec, out=Ah)
            tube_fft(B, precision=prec, out=Bh)
            tube_fft(C, precision=prec, out=Ch)
            Xh = fourier_tprod(Ah, Bh, n, n, precision=prec)
            if prec == "split_bf16":
                split_words(Xh, cols=n)
            Dh = fourier_tprod(Xh, Ch, n, n, precision=prec, out=Ah)
            tube_fft(Dh, inverse=True, cols=n, out=D)

        def two_calls():
            tprod(tprod(A, B, prec), C, prec, out=D)

        times = {}
        for name, fn in (("resident", resident), ("two_calls", two_calls)):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            times[name] = (time.perf_counter() - t0) * 1e3 / args.steps
        res[prec] = {"ms_per_step": times["resident"], "two_calls_ms": times["two_calls"],
                     "tflops_equiv": F / (times["resident"] * 1e-3) / 1e12}
        log(f"[bench] chain {prec}: resident {times['resident']:.3f} ms, two qt_tprod calls "
            f"{times['two_calls']:.3f} ms, {res[prec]['tflops_equiv']:.1f} TFLOP/s-equiv")
    head = precs[0]
    _emit({"metric": "T-product TFLOP/s-equiv & % roofline, split-BF16 vs FP32 at stated rel. error",
           "value": round(res[head]["tflops_equiv"], 3), "unit": "TFLOP/s-equiv", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res[head]["ms_per_step"], 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16x3-split/f32-acc" if head == "split_bf16" else "f32", "data": "synthetic",
           "config": {"workload": wl["desc"], "precision": head, "flops_per_step": F},
           "per_precision": res, "roofline": None, "cpu_baseline": None})


def bench_complex(args, wl, dev, stream, real=False):
    """Complex T-product (second Cayley-Dickson half zero): two-plane tube
    FFTs and 8 m n s p flops of uncoupled complex products.  Real T-product
    (one plane): Hermitian half spectrum, 8 m n s (p/2 + 1) flops.  Timed
    against the quaternion path on the same tensors embedded with zero
    planes; sampled entries are checked against the oracle's definition."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_2212_14318_amd import _native as nat
    from paper_2212_14318_amd import tprod, tprod_complex, tprod_real

    planes = 1 if real else 2
    A64, B64 = (x[:planes].copy() for x in synth.config_inputs(3)[:2])
    _, p, m, n = A64.shape
    s = B64.shape[3]
    A, B = (torch.from_numpy(x).to(dev, torch.float32) for x in (A64, B64))
    Aq, Bq = (torch.cat([x, torch.zeros((4 - planes,) + x.shape[1:], device=dev)]) for x in (A, B))
    C = torch.empty((planes, p, m, s), device=dev)
    Cq = torch.empty((4, p, m, s), device=dev)
    F = 8.0 * m * n * s * ((p // 2 + 1) if real else p)
    rng = np.random.Generator(np.random.PCG64(7))
    kk, ii, jj = rng.integers(0, p, 64), rng.integers(0, m, 64), rng.integers(0, s, 64)
    Aq64, Bq64 = (np.concatenate([x, np.zeros((4 - planes,) + x.shape[1:])]) for x in (A64, B64))
    ref = oracle.tprod_entries(Aq64, Bq64, kk, ii, jj)[:planes]
    res = {}
    precs = [x for x in args.precisions.split(",") if x]
    for prec in precs:
        wsz = (nat.qt_real_workspace_size if real else nat.qt_complex_workspace_size)(m, n, s, p,
                                                                                     nat.PRECISIONS[prec])
        ws = torch.empty(wsz, dtype=torch.uint8, device=dev)
        if real:
            run = lambda: tprod_real(A[0], B[0], prec, out=C[0], ws=ws)
        else:
            run = lambda: tprod_complex(A, B, prec, out=C, ws=ws)
        times = {}
        for name, fn in (("complex", run), ("quaternion", lambda: tprod(Aq, Bq, prec, out=Cq))):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            times[name] = (time.perf_counter() - t0) * 1e3 / args.steps
        got = C.double().cpu().numpy()[:, kk, ii, jj]
        err = float(np.sqrt(np.sum((got - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)))
        res[prec] = {"ms_per_step": times["complex"], "quaternion_path_ms": times["quaternion"],
                     "tflops": F / (times["complex"] * 1e-3) / 1e12, "sampled_rel_err": err}
        log(f"[bench] {'real' if real else 'complex'} {prec}: {times['complex']:.3f} ms "
            f"({res[prec]['tflops']:.1f} TFLOP/s), quaternion path on zero planes {times['quaternion']:.3f} ms, "
            f"sampled rel err {err:.2e}")
    head = precs[0]
    _emit({"metric": "T-product TFLOP/s-equiv & % roofline, split-BF16 vs FP32 at stated rel. error",
           "value": round(res[head]["tflops"], 3), "unit": "TFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res[head]["ms_per_step"], 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16x3-split/f32-acc" if head == "split_bf16" else "f32", "data": "synthetic",
           "config": {"workload": wl["desc"], "precision": head, "flops_per_step": F},
           "per_precision": res, "roofline": None, "cpu_baseline": None})


def bench_matvec(args, wl, dev, stream):
    """Narrow coupled product (s = 1): A^ is read once from HBM, so the
    roofline is HBM bandwidth over 16 m n p bytes (plus the small B^, C^).
    The 64-column MFMA tile path at s = 5 is timed beside it."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_2212_14318_amd import _native as nat
    from paper_2212_14318_amd import fourier_tprod, tube_fft

    m = n = 2048
    p = 16
    A64 = synth.quat_tensor(m, n, p, seed=6000)
    A = torch.from_numpy(A64).to(dev, torch.float32)
    res = {}
    precs = [x for x in args.precisions.split(",") if x]
    for s_cols in (1, 5):
        B64 = synth.quat_tensor(n, s_cols, p, seed=6001)
        B = torch.from_numpy(B64).to(dev, torch.float32)
        for prec in precs:
            Ah = tube_fft(A, precision=prec, out=torch.empty((4, p, m, nat.qt_fourier_ld(n)), device=dev))
            Bh = tube_fft(B, precision=prec, out=torch.empty((4, p, n, nat.qt_fourier_ld(s_cols)), device=dev))
            Ch = torch.empty((4, p, m, nat.qt_fourier_ld(s_cols)), device=dev)
            for _ in range(args.warmup):
                fourier_tprod(Ah, Bh, n, s_cols, precision=prec, out=Ch)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(stream)
            for _ in range(args.steps):
                fourier_tprod(Ah, Bh, n, s_cols, precision=prec, out=Ch)
            ev[1].record(stream)
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / args.steps
            nbytes = 16.0 * p * (m * n + 2 * n * s_cols + m * s_cols)
            res[f"{prec}_s{s_cols}"] = {"ms": ms, "gbps": nbytes / (ms * 1e-3) / 1e9,
                                        "tflops_equiv": 32.0 * m * n * s_cols * p / (ms * 1e-3) / 1e12}
            if s_cols == 1:
                C = torch.empty((4, p, m, 1), device=dev)
                tube_fft(Ch, inverse=True, cols=1, out=C)
                kk = np.arange(p)
                ii = np.random.Generator(np.random.PCG64(7)).integers(0, m, p)
                ref = oracle.tprod_entries(A64, B64, kk, ii, np.zeros(p, dtype=np.int64))
                got = C.cpu().numpy()[:, kk, ii, 0].astype(np.float64)
                res[f"{prec}_s1"]["rel_err"] = float(np.sqrt(((got - ref) ** 2).sum() / (ref ** 2).sum()))
            log(f"[bench] matvec {prec} s={s_cols}: {ms:.3f} ms, {res[f'{prec}_s{s_cols}']['gbps']:.0f} GB/s "
                f"of A^ + B^ + C^" + (f", rel err {res[f'{prec}_s1']['rel_err']:.2e}" if s_cols == 1 else ""))
            del Ah, Bh, Ch
    head = precs[0]
    r = res[f"{head}_s1"]
    _emit({"metric": "T-product TFLOP/s-equiv & % roofline, split-BF16 vs FP32 at stated rel. error",
           "value": round(r["tflops_equiv"], 4), "unit": "TFLOP/s-equiv", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms"], 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl["desc"], "precision": head},
           "roofline": {"bound": "hbm", "achieved": round(r["gbps"], 1), "peak": PEAK_HBM_GBPS,
                        "unit": "GB/s", "frac": round(r["gbps"] / PEAK_HBM_GBPS, 4), "traffic": None},
           "per_precision": res, "cpu_baseline": None})


if __name__ == "__main__":
    main()
