"""Throughput benchmark of the MW transforms on one MI355X.

Workload (default): L = 512, spin 2, one complex map, f_lm = (N(0,1) + i N(0,1))/(l+1)
for l >= 2 (seed 1002).  One step = one inverse (f_lm -> map) plus one forward
(map -> f_lm) on data resident in HBM.  Prints ONE JSON line.
"""
import argparse
import gc
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6e12   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz

# HBM traffic of the contraction kernels per launch at L=512 s=2, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) scaled by the same counters
# read for a plain copy of known size (profiles/traffic_roundtrip_L512_s2.md).
# Valid only while the kernel and plan sources are unchanged: keyed by their SHA-256.
TRAFFIC = {
    ("contract_inverse", 512, 2): {"bytes": 37805630, "source_sha256": "d19b76c4cae29154cb8c1342d4d175a4709746dbd6ea603e9d52b09c7452be47"},
    ("contract_forward", 512, 2): {"bytes": 29427290, "source_sha256": "d19b76c4cae29154cb8c1342d4d175a4709746dbd6ea603e9d52b09c7452be47"},
}
KERNEL_SOURCES = ("paper_1110_6298_amd/csrc/mw_contract.hip", "paper_1110_6298_amd/csrc/mw_plan.cpp")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


PEAK_FP32_MFMA = 157.3e12   # dense FP32 matrix-core peak


def contraction_term_flops(L, s, real=False):
    """The contraction part of contraction_flops: 4 flop per folded term."""
    return 4.0 * sum(((l + 1) if real else (2 * l + 1)) * (l + 1) for l in range(abs(s), L))


def contraction_flops(L, s, real=False):
    """Algorithmic flops of one contraction launch: 4 per folded term (l, m, m'>=0)
    (complex H times the real product Delta*Delta), plus 5 per Wigner
    eighth-wedge element 0 <= m <= m' <= l generated (one three-term step).  A
    real scalar map needs the orders m >= 0 only."""
    terms = sum(((l + 1) if real else (2 * l + 1)) * (l + 1) for l in range(abs(s), L))
    wedge = sum((l + 1) * (l + 2) // 2 for l in range(L))
    return 4.0 * terms + 5.0 * wedge


def progress(msg):
    """One progress line on stderr (the JSON result alone goes to stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def oracle_configs(oracle, mwsynth):
    """The oracle on the host cores for the workloads other than the L=512 map:
    whole round trips of the L=64 map for at least 5 s; for the 256-map batch one
    round trip per (L, spin) class, scaled by the class counts; one round trip of
    the L=2048 real map (inverse and forward timed apart); for the 32-map
    gradient 2 A^H (A x - y), one map's forward and forward adjoint, times 32."""
    out = {}
    w = mwsynth.workload_scalar_l64()
    t, n = time.perf_counter(), 0
    while time.perf_counter() - t < 5.0:
        oracle.forward(oracle.inverse(w["flm"], w["L"], w["s"]), w["L"], w["s"])
        n += 1
    dt = time.perf_counter() - t
    out["scalar_l64"] = {"value": n / dt, "unit": "round trips/s", "sample": "%d round trips, %.1f s" % (n, dt)}
    progress("oracle: L=64 done")
    maps = mwsynth.workload_batch_mixed()
    cls = {}
    for m in maps:
        cls.setdefault((m["L"], m["s"]), []).append(m)
    total = 0.0
    for (L, s), ms in sorted(cls.items()):
        t = time.perf_counter()
        oracle.forward(oracle.inverse(ms[0]["flm"], L, s), L, s)
        dt = time.perf_counter() - t
        total += dt * len(ms)
        progress("oracle: batch class L=%d s=%d, %.2f s x %d maps" % (L, s, dt, len(ms)))
    out["batch256"] = {"value": len(maps) / total, "unit": "map round trips/s",
                       "sample": "one round trip per (L, spin) class (%d classes), scaled by the class counts: "
                                 "%.0f s for the batch" % (len(cls), total)}
    w = mwsynth.workload_real_l2048()
    t = time.perf_counter()
    x = oracle.inverse(w["flm"], w["L"], w["s"])
    ti = time.perf_counter() - t
    progress("oracle: L=2048 inverse %.1f s" % ti)
    t = time.perf_counter()
    oracle.forward(x, w["L"], w["s"])
    tf = time.perf_counter() - t
    progress("oracle: L=2048 forward %.1f s" % tf)
    out["real_l2048"] = {"value": 1.0 / (ti + tf), "unit": "round trips/s",
                         "sample": "1 round trip: inverse %.1f s, forward %.1f s" % (ti, tf)}
    w = mwsynth.workload_grad_l256()
    L, s = w["L"], w["s"]
    t = time.perf_counter()
    r = oracle.forward(w["x"][0], L, s) - w["y"]
    oracle.forward_adjoint(2.0 * r, L, s)
    dt = time.perf_counter() - t
    out["grad_l256"] = {"value": 1.0 / (dt * w["x"].shape[0]), "unit": "gradients/s (all 32 maps)",
                        "sample": "one map's forward and forward adjoint, %.2f s, times %d" % (dt, w["x"].shape[0])}
    progress("oracle: gradient done")
    for v in out.values():
        v.update({"cores": oracle.max_threads(), "kind": "oracle"})
    return out


def rel(a, b):
    import numpy as np
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_per_degree(got, ref, L):
    """Per-degree relative error of coefficient vectors: the largest over l of
    max_m |got - ref| / max_m |ref| (degrees whose reference is zero skipped)."""
    import numpy as np
    worst = 0.0
    for l in range(L):
        sl = slice(l * l, (l + 1) * (l + 1))
        den = float(np.abs(ref[sl]).max())
        if den > 0:
            worst = max(worst, float(np.abs(got[sl] - ref[sl]).max()) / den)
    return worst


def time_steps(torch, step, steps, warmup):
    """ms per step of `step` (enqueued on the current stream), timed with events
    around `steps` calls after `warmup` untimed ones.  Python's cyclic garbage
    collector is run before and paused during the timed calls: a collection
    pass over the interpreter's heap stalls the host for tens of ms, and with it
    the GPU, which would otherwise be charged to the transforms."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    try:
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(steps):
            step()
        t1.record()
        torch.cuda.synchronize()
    finally:
        gc.enable()
    return t0.elapsed_time(t1) / steps


def kernel_profile(mw, step, steps):
    """Average duration (ms) of each stage from libmw's own HIP events, recorded
    on the launch stream around every launch."""
    mw.profile_enable(True)
    for _ in range(steps):
        step()
    prof = mw.profile_read()
    mw.profile_enable(False)
    return {k: v[0] / v[1] for k, v in prof.items()}


def batched_workload(torch, mw, dev, steps, warmup, precision, graph=False):
    """The 256-map batch: L uniform on {128, 256, 512}, spin on {0, 2}, half of the
    maps drawn with real-map coefficient symmetry (only the s = 0 ones run the
    real path).  One step = one batched inverse + one batched forward call."""
    import mwsynth
    maps = mwsynth.workload_batch_mixed()
    Ls = [m["L"] for m in maps]
    ss = [m["s"] for m in maps]
    rs = [1 if (m["real"] and m["s"] == 0) else 0 for m in maps]
    flm = [torch.from_numpy(m["flm"]).to(dev) for m in maps]
    grids = [torch.empty((L, 2 * L - 1), dtype=torch.float64 if r else torch.complex128, device=dev)
             for L, r in zip(Ls, rs)]
    back = [torch.empty(L * L, dtype=torch.complex128, device=dev) for L in Ls]
    mw.prepare(Ls, ss, rs, precision=precision)

    def step():
        mw.inverse_batch(flm, Ls, ss, rs, precision=precision, outs=grids)
        mw.forward_batch(grids, Ls, ss, rs, precision=precision, outs=back)

    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        ms = time_steps(torch, g.replay, steps, warmup)
    else:
        ms = time_steps(torch, step, steps, warmup)
    err = 0.0
    for b in range(len(maps)):
        ref = maps[b]["flm"]
        got = back[b].cpu().numpy()
        err = max(err, rel(got, ref))
    # one step with libmw's per-launch events: the summed time of each stage and
    # the contraction roofline over the whole batch (algorithmic flops of every
    # map's two contractions over the two contraction stages' summed time)
    roof = None
    if not graph:
        torch.cuda.synchronize()
        mw.profile_enable(True)
        step()
        prof = mw.profile_read()
        mw.profile_enable(False)
        t_c = sum(prof[k][0] for k in ("contract_forward", "contract_inverse") if k in prof) * 1e-3
        fl = sum(contraction_flops(L, sp, real=bool(r)) for L, sp, r in zip(Ls, ss, rs)) * 2
        terms = sum(contraction_term_flops(L, sp, real=bool(r)) for L, sp, r in zip(Ls, ss, rs)) * 2
        roof = {"stages_ms": {k: v[0] for k, v in prof.items()},
                "contraction": {"bound": "alu", "achieved": fl / t_c / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                                "unit": "TFLOP/s", "frac": fl / t_c / PEAK_FP64_VALU}}
        if precision != mw.FP64:
            roof["contraction"]["mfma"] = {"achieved": terms / t_c / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                                           "unit": "TFLOP/s", "frac": terms / t_c / PEAK_FP32_MFMA}
    return ms, len(maps), err, roof


def large_workload(torch, mw, dev, steps, warmup):
    """L = 2048, s = 0, one real map with C_l = (l+1)^-2 (seed 1004): round trips
    in FP64 and FP32C, per-kernel durations and the contraction roofline."""
    import mwsynth
    w = mwsynth.workload_real_l2048()
    L, flm_h = w["L"], w["flm"]
    flm = torch.from_numpy(flm_h).to(dev)
    out = {}
    for name, prec in (("fp64", mw.FP64), ("fp32c", mw.FP32C)):
        x = torch.empty((L, 2 * L - 1), dtype=torch.float64, device=dev)
        back = torch.empty(L * L, dtype=torch.complex128, device=dev)
        mw.prepare([L], [0], [1], precision=prec)

        def step():
            mw.inverse(flm, L, 0, reality=1, precision=prec, out=x)
            mw.forward(x, L, 0, reality=1, precision=prec, out=back)

        ms = time_steps(torch, step, steps, warmup)
        pk = kernel_profile(mw, step, steps)
        back_h = back.cpu().numpy()
        err = rel(back_h, flm_h)
        err_deg = rel_per_degree(back_h, flm_h, L)
        flops = contraction_flops(L, 0, real=True)
        dom = "contract_forward" if pk.get("contract_forward", 0) >= pk.get("contract_inverse", 0) \
            else "contract_inverse"
        ach = flops / (pk[dom] * 1e-3)
        out[name] = {"round_trips_per_s": 1e3 / ms, "ms_per_step": ms, "round_trip_rel_err": err,
                     "round_trip_rel_err_per_degree": err_deg,
                     "kernels": {k: {"avg_us": 1e3 * v} for k, v in pk.items()}}
        if prec == mw.FP64:
            out[name]["roofline"] = {"kernel": dom, "bound": "alu", "achieved": ach / 1e12,
                                     "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                                     "frac": ach / PEAK_FP64_VALU, "flops_per_launch": flops}
    out["workload"] = "L=2048, s=0, one real map, C_l=(l+1)^-2, seed 1004; one step = inverse + forward"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--L", type=int, default=512)
    ap.add_argument("--spin", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-map batched workload")
    ap.add_argument("--no-large", action="store_true", help="skip the L=2048 real-map workload")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum CPU time of the oracle baseline sample (whole round trips)")
    ap.add_argument("--cpu-1core", action="store_true",
                    help="also time one oracle round trip on one host core (about 100 s at L=512)")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="also time the oracle on the host cores for the other workloads (L=64 map, "
                         "256-map batch, L=2048 real map, 32-map gradient; several minutes)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the timed work, negate a float64 buffer of this many MiB once "
                         "(a plain read+write kernel of known size, for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(maps are independent, so a batch would shard by map with no exchange)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import mwsynth
    import paper_1110_6298_amd as mw

    L, s = args.L, args.spin
    w = mwsynth.workload_spin2_l512(L) if s == 2 else dict(L=L, s=s, flm=mwsynth.flm_gaussian(L, s, 1002, 1.0))
    flm_h = w["flm"]
    dev = torch.device("cuda", 0)
    flm = torch.from_numpy(flm_h).to(dev)
    xmap = {p: torch.empty((L, 2 * L - 1), dtype=torch.complex128, device=dev) for p in (mw.FP64, mw.FP32C)}
    back = {p: torch.empty(L * L, dtype=torch.complex128, device=dev) for p in (mw.FP64, mw.FP32C)}
    mw.prepare([L], [s])
    mw.prepare([L], [s], precision=mw.FP32C)

    def stepper(prec):
        def step():
            mw.inverse(flm, L, s, precision=prec, out=xmap[prec])
            mw.forward(xmap[prec], L, s, precision=prec, out=back[prec])
        return step

    progress("L=%d s=%d FP64 round trips" % (L, s))
    wall0 = time.perf_counter()
    ms_step = time_steps(torch, stepper(mw.FP64), args.steps, args.warmup)
    wall = time.perf_counter() - wall0
    per_kernel = kernel_profile(mw, stepper(mw.FP64), args.steps)
    progress("L=%d s=%d FP32C round trips" % (L, s))
    ms_mixed = time_steps(torch, stepper(mw.FP32C), args.steps, args.warmup)
    per_kernel_mixed = kernel_profile(mw, stepper(mw.FP32C), args.steps)

    dom = max(per_kernel, key=lambda k: per_kernel[k])
    flops = contraction_flops(L, s)
    kernels = {k: {"avg_us": 1e3 * v} for k, v in per_kernel.items()}
    for k in ("contract_forward", "contract_inverse"):
        if k in per_kernel:
            kernels[k]["tflops"] = flops / (per_kernel[k] * 1e-3) / 1e12
    dom_c = "contract_forward" if per_kernel.get("contract_forward", 0) >= per_kernel.get("contract_inverse", 0) \
        else "contract_inverse"
    achieved = flops / (per_kernel[dom_c] * 1e-3)

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    x_h = xmap[mw.FP64].cpu().numpy()
    back_h = back[mw.FP64].cpu().numpy()
    x32_h = xmap[mw.FP32C].cpu().numpy()
    back32_h = back[mw.FP32C].cpu().numpy()
    result = {
        "metric": "MW fwd+inv transforms/sec at L=512 s=2 (FP64 vs mixed) at stated max rel error",
        "value": 1e3 / ms_step,
        "unit": "round trips/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "MW spin-%d round trip (inverse + forward), L=%d, one complex map, "
                               "f_lm ~ (N+iN)/(l+1), seed 1002" % (s, L), "L": L, "spin": s,
                   "precision": "fp64", "maps_per_step": 1},
        "round_trip_rel_err": rel(back_h, flm_h),
        "round_trip_rel_err_per_degree": rel_per_degree(back_h, flm_h, L),
        "wall_ms_per_step": 1e3 * wall / args.steps,
        "kernels": kernels,
        "dominant_kernel": dom,
        "roofline": {"kernel": dom_c, "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": None,
                     "flops_per_launch": flops},
        "mixed": {"precision": "fp32c", "dtype": "f32 contraction (MFMA), f64 recursion and Fourier stages",
                  "value": 1e3 / ms_mixed, "unit": "round trips/s", "ms_per_step": ms_mixed,
                  "stated_max_rel_err": 1e-6,
                  "rel_err_vs_fp64": {"inverse_map": rel(x32_h, x_h), "forward_coeffs": rel(back32_h, back_h)},
                  "round_trip_rel_err": rel(back32_h, flm_h),
                  "round_trip_rel_err_per_degree": rel_per_degree(back32_h, flm_h, L),
                  "kernels": {k: {"avg_us": 1e3 * v} for k, v in per_kernel_mixed.items()}},
    }
    # mixed path: the chains stay FP64 (VALU-bound), the contraction's products
    # run on the FP32 matrix cores; both rates for the dominant mixed kernel
    dom_m = "contract_forward" if per_kernel_mixed.get("contract_forward", 0) >= \
        per_kernel_mixed.get("contract_inverse", 0) else "contract_inverse"
    t_m = per_kernel_mixed[dom_m] * 1e-3
    result["mixed"]["roofline"] = {
        "kernel": dom_m, "bound": "alu", "achieved": flops / t_m / 1e12, "peak": PEAK_FP64_VALU / 1e12,
        "unit": "TFLOP/s", "frac": flops / t_m / PEAK_FP64_VALU, "flops_per_launch": flops,
        "mfma": {"achieved": contraction_term_flops(L, s) / t_m / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                 "unit": "TFLOP/s", "frac": contraction_term_flops(L, s) / t_m / PEAK_FP32_MFMA}}
    tr = TRAFFIC.get((dom_c, L, s))
    if tr is not None and tr["source_sha256"] == kernel_source_hash():
        result["roofline"]["traffic"] = tr["bytes"]

    if not args.no_batch:
        batched = {}
        for name, prec, graph in (("fp64", mw.FP64, False), ("fp32c", mw.FP32C, False),
                                  ("fp64_graph", mw.FP64, True), ("fp32c_graph", mw.FP32C, True)):
            progress("256-map batch, %s" % name)
            ms_b, nmaps, err_b, roof = batched_workload(torch, mw, dev, args.batch_steps, 2, prec, graph)
            batched[name] = {"maps_round_trips_per_s": nmaps * 1e3 / ms_b, "ms_per_step": ms_b,
                             "round_trip_rel_err": err_b}
            if roof is not None:
                batched[name]["profile"] = roof
        batched["workload"] = ("256 maps, L uniform on {128,256,512}, spin uniform on {0,2}, 128 with real-map "
                               "coefficient symmetry (s=0 ones on the real path), f_lm ~ N(0,1)/(l+1), seed 1003; "
                               "one step = batched inverse + batched forward")
        result["batched"] = batched

    if not args.no_large:
        progress("L=2048 real map")
        result["large_l2048"] = large_workload(torch, mw, dev, 5, 1)

    if not args.no_cpu_baseline:
        import oracle
        progress("oracle baseline on the host cores")
        oracle.build(force=False)
        t = time.perf_counter()
        count = 0
        while True:
            xo = oracle.inverse(flm_h, L, s)
            fo = oracle.forward(xo, L, s)
            count += 1
            dt = time.perf_counter() - t
            if dt >= args.cpu_seconds:
                break
        result["cpu_baseline"] = {"value": count / dt, "unit": "round trips/s", "cores": oracle.max_threads(),
                                  "kind": "oracle",
                                  "sample": "%d full round trips (inverse + forward) of the same L=%d s=%d map, "
                                            "%.1f s" % (count, L, s, dt)}
        if args.cpu_1core:
            progress("oracle baseline on one host core")
            oracle.set_threads(1)
            t = time.perf_counter()
            oracle.forward(oracle.inverse(flm_h, L, s), L, s)
            dt1 = time.perf_counter() - t
            oracle.set_threads(result["cpu_baseline"]["cores"])
            result["cpu_baseline_1core"] = {"value": 1.0 / dt1, "unit": "round trips/s", "cores": 1,
                                            "kind": "oracle", "sample": "1 round trip, %.1f s" % dt1}
        if args.cpu_configs:
            result["cpu_baseline_configs"] = oracle_configs(oracle, mwsynth)
        result["max_rel_err_vs_oracle"] = {"inverse_map": rel(x_h, xo), "forward_coeffs": rel(back_h, fo),
                                           "forward_coeffs_per_degree": rel_per_degree(back_h, fo, L)}
        result["mixed"]["max_rel_err_vs_oracle"] = {"inverse_map": rel(x32_h, xo),
                                                    "forward_coeffs": rel(back32_h, fo),
                                                    "forward_coeffs_per_degree": rel_per_degree(back32_h, fo, L)}
    print(json.dumps(result))


if __name__ == "__main__":
    main()
