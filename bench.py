#!/usr/bin/env python3
"""Benchmark of the batched negacyclic NTT on one MI355X.

Workload (the headline configuration): N = 2^16, L = 45 primes in [2^59, 2^60) drawn
from seed 2, one ciphertext = 2 polynomials of uniform residues; one step is the
forward NTT of the whole ciphertext followed by its inverse, i.e. 180 limb-NTTs.

Inputs are resident in HBM before timing starts.  The step rotates through copies of
the ciphertext totalling more than the 256 MB Infinity Cache, so every step reads its
input from HBM.  Forward then inverse returns each buffer to its original content, so
the copies stay valid for the whole run.  Steps are independent and are issued round-robin
over --streams streams (2 by default; copy j always on stream j mod S), so that one step's
kernels fill the tail of the other stream's; the same steps on one stream are reported
beside them.

Printed (stdout, one JSON line): limb-NTTs/s over the timed steps, the roofline of the
dominant kernel (algorithmic bytes of one launch / its average duration from HIP events
on the launch stream), the same kernel's VALU issue utilization (executed instructions from
the committed counters), per-step p50/p99, the plain one-call-per-polynomial rate, and the
CPU oracle timed on this host.  Everything else goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NTTs/s + % HBM roofline at N=2^16×45 limbs; batched vs plain, p99 latency"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
# VALU issue rate: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 32-bit integer instruction per
# 4 cycles on a 16-lane SIMD
VALU_ISSUE_PEAK_GINST = 256 * 4 * 2.4 / 4
WORKLOAD = dict(N=1 << 16, L=45, P=2, bits=60, seed=2)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the kernels' device-code sources (the tuner's cache key uses the same one)."""
    from paper_2012_01968_amd import autotune
    return autotune.source_hash()


def ramp(step, ms: float) -> None:
    """Run step(i) until at least `ms` of wall time has passed (GPU clock ramp-up)."""
    import torch
    t0 = time.perf_counter()
    i = 0
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(8):
            step(i)
            i += 1
        torch.cuda.synchronize()


def variant_key(info: dict, ots: int) -> str:
    """Name of a plan configuration, as used by the traffic summary."""
    path = "fused" if info["kernel_path"] == 2 else "split"
    tiles = "".join(f"-{k}={info[k]}" for k in ("r1", "wg_size", "col_width") if info.get(k))
    return f"{'ot%d' % ots if ots else 'table'}-{path}-n1={info['log2_n1']}{tiles}"


def tune_shape(N: int, primes, polys: int) -> dict:
    """The tuner's choice for one shape (measured now unless cached for this build)."""
    from paper_2012_01968_amd import autotune
    cached = autotune.lookup(N, primes, polys) is not None
    t0 = time.perf_counter()
    e = autotune.tune(N, primes, polys)
    log(f"tuned N={N} L={len(primes)} P={polys}: {e['opts']} {e['us']:.1f} us "
        f"({len(e['tried'])} candidates, {'cached' if cached else f'{time.perf_counter() - t0:.1f} s'})")
    return {"opts": e["opts"], "us": e["us"], "candidates": len(e["tried"]), "cached": cached,
            "seconds": round(time.perf_counter() - t0, 2)}


def read_traffic(kernel: str, src_hash: str, path: str | None = None, field: str = "bytes_per_launch"):
    """A per-launch counter figure (HBM bytes, or VALU instructions with
    field="valu_insts_per_launch") from the committed counter summary, if it matches this
    source."""
    path = path or os.path.join(ROOT, "profiles", "traffic_counters.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#") or ":" not in line:
            continue
        k, _, v = line.rpartition(":")   # keys may hold ':' themselves
        rec[k.strip()] = v.strip()
    if rec.get("source_hash") != src_hash:
        return None
    key = f"{field}[{kernel}]"
    return float(rec[key]) if key in rec else None


def twiddle_bytes(pass_kind: str, N: int, L: int, log2_n1: int, ots: int, b: int = 10) -> int:
    """Algorithmic twiddle bytes of one launch (16 B per entry: value and Shoup companion)."""
    N1 = 1 << log2_n1
    if pass_kind == "col":
        return 16 * L * N1
    if pass_kind == "fused":
        return twiddle_bytes("col", N, L, log2_n1, ots, b) + twiddle_bytes("row", N, L, log2_n1, ots, b)
    if log2_n1 == 0:
        N1 = 1
    table = N // (1 << ots) - N1
    ot = ((1 << b) + N // (1 << b)) if ots else 0
    return 16 * L * (table + ot)


def data_bytes(pass_kind: str, N: int, L: int, P: int) -> int:
    """Algorithmic data bytes of one launch: every pass reads and writes each residue once."""
    return (2 if pass_kind == "fused" else 1) * 16 * P * L * N


VARIANTS = {   # name -> plan options (twiddle source x kernel path)
    "table-split": dict(kernel_path=1),
    "ot-split": dict(kernel_path=1, twiddle_mode=2, ot_stages=2),
    "table-fused": dict(kernel_path=2),
    "ot-fused": dict(kernel_path=2, twiddle_mode=2, ot_stages=2),
}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--ramp-ms", type=float, default=50.0,
                    help="before the warmup steps, run steps for at least this long: the GPU's clocks rise "
                         "over tens of milliseconds, and a cold start would be timed otherwise")
    ap.add_argument("--variant", choices=["auto", "tuned"] + list(VARIANTS), default="auto",
                    help="auto measures every named variant (table / OT twiddles x split / fused launch) and the "
                         "tuner's choice, and reports the fastest")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the plan tuner: named variants only, default plans in the other sections")
    ap.add_argument("--log2-n1", type=int, default=0)
    ap.add_argument("--streams", type=int, default=2,
                    help="streams the timed steps are issued on, round-robin (1 = every step on one stream); "
                         "steps are independent, so steps on different streams overlap on the GPU")
    ap.add_argument("--rotate-gib", type=float, default=1.25, help="total size of the rotating input copies")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of the Poisson request stream of the serving section (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="request arrival rate (1/s)")
    ap.add_argument("--serve-high-rate", type=float, default=12000.0,
                    help="arrival rate of a second, 5-second stream above the per-request path's capacity (0 skips)")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch section")
    ap.add_argument("--no-polymul", action="store_true", help="skip the large-parameter product section")
    ap.add_argument("--no-ablation", action="store_true", help="skip the Table II ablation-ladder section")
    ap.add_argument("--no-word32", action="store_true", help="skip the 32-bit word section")
    ap.add_argument("--no-crt", action="store_true", help="skip the RNS <-> integer conversion section")
    ap.add_argument("--profile-polymul", action="store_true",
                    help="counter-collection driver for the product workload: --steps products with one "
                         "twiddle mode (--variant, --log2-n1), then one plain device copy of an operand")
    ap.add_argument("--profile-run", action="store_true",
                    help="counter-collection driver: --steps steps of one twiddle mode (no timing, no JSON), "
                         "then one plain device copy of a ciphertext for the counters' byte calibration")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        log("bench.py measures one GPU: the transform shards by RNS limb with no exchange, and this "
            "build runs on a single MI355X, so --gpus above 1 is not supported.")
        return 2

    import torch
    import synth
    import paper_2012_01968_amd as ntt

    N, L, P = WORKLOAD["N"], WORKLOAD["L"], WORKLOAD["P"]
    primes = synth.gen_primes(WORKLOAD["seed"], N, WORKLOAD["bits"], L)
    host = synth.residue_batch(WORKLOAD["seed"], primes, N, P)
    ct_bytes = host.nbytes
    R = max(2, int(np.ceil(args.rotate_gib * 2**30 / ct_bytes)))
    n_streams = max(1, args.streams)
    R = -(-R // n_streams) * n_streams    # a multiple of the stream count: copy j stays on one stream
    streams = [torch.cuda.Stream() for _ in range(n_streams)] if n_streams > 1 else []
    dev0 = torch.from_numpy(host.view(np.int64)).to("cuda")
    bufs = torch.empty((R,) + tuple(dev0.shape), dtype=torch.int64, device="cuda")
    bufs[:] = dev0
    torch.cuda.synchronize()
    log(f"workload N={N} L={L} P={P}: {ct_bytes/1e6:.1f} MB per ciphertext, {R} rotating copies "
        f"({R*ct_bytes/2**30:.2f} GiB)")

    if args.profile_polymul:
        return polymul_profile_run(args)
    if args.profile_run:
        mode = "ot-fused" if args.variant == "auto" else args.variant
        if mode == "tuned":
            # the tuner's cached plan for this shape, as the timed run would take it (no tuning here)
            from paper_2012_01968_amd import autotune
            entry = autotune.lookup(N, primes, P)
            if entry is None:
                log("profile run: no cached tuned plan for this shape and kernel build")
                return 1
            plan = ntt.ntt_plan_create(N, primes, **entry["opts"])
        else:
            plan = ntt.ntt_plan_create(N, primes, log2_n1=args.log2_n1, **VARIANTS[mode])
        for i in range(args.steps):
            ntt.ntt_forward(plan, bufs[i % R])
            ntt.ntt_inverse(plan, bufs[i % R])
        torch.cuda.synchronize()
        bufs[R - 1].copy_(bufs[1])        # calibration: one plain copy of ct_bytes read + ct_bytes written
        torch.cuda.synchronize()
        plan.destroy()
        log(f"profile run: {args.steps} steps ({mode}) + one {ct_bytes}-byte device copy")
        return 0

    # plan creation (prime checks, roots, twiddle, Shoup and OT tables, allocation and upload;
    # no kernel launch): host time per plan, median of 3 after one untimed creation
    plan_ms = {}
    for mode in ("table-split", "ot-split"):
        ntt.ntt_plan_create(N, primes, log2_n1=args.log2_n1, **VARIANTS[mode]).destroy()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            pl = ntt.ntt_plan_create(N, primes, log2_n1=args.log2_n1, **VARIANTS[mode])
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
            pl.destroy()
        plan_ms[mode] = round(float(np.median(ts)), 2)
    log("plan creation (ms): " + ", ".join(f"{k}={v}" for k, v in plan_ms.items()))

    variants = dict(VARIANTS)
    tuned = None
    if args.variant in ("auto", "tuned") and not args.no_tune:
        tuned = tune_shape(N, primes, P)
        variants["tuned"] = tuned["opts"]
    modes = list(variants) if args.variant == "auto" else [args.variant]
    results = {}
    for mode in modes:
        opts = dict(variants[mode])
        opts.setdefault("log2_n1", args.log2_n1)
        plan = ntt.ntt_plan_create(N, primes, **opts)
        info = ntt.ntt_plan_get_info(plan)
        npass = ntt.ntt_plan_num_passes(plan)
        fused = info["kernel_path"] == ntt.PATH_FUSED

        def timed_steps(S: int):
            """Time args.steps steps issued round-robin over S streams (step i on stream i mod S,
            so copy j is always on stream j mod S); returns (ms per step, wall s, per-step ms)."""
            sts = streams[:S] if S > 1 else [torch.cuda.current_stream()]

            def step(i):
                b = bufs[i % R]
                ntt.ntt_forward(plan, b, None, sts[i % S])
                ntt.ntt_inverse(plan, b, None, sts[i % S])

            ramp(step, args.ramp_ms)
            for i in range(args.warmup):
                step(i)
            torch.cuda.synchronize()
            # the timed steps: events only around the whole run (an event between steps makes the
            # queue drain before the next kernel starts, which would be timed as well); with several
            # streams they wait for the start event and the end event waits for all of them
            main_st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(main_st)
            if S > 1:
                for st in sts:
                    st.wait_event(e0)
            for i in range(args.steps):
                step(args.warmup + i)
            if S > 1:
                for st in sts:
                    done = torch.cuda.Event()
                    done.record(st)
                    main_st.wait_event(done)
            e1.record(main_st)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ms = e0.elapsed_time(e1) / args.steps
            # per-step latency: a second pass with events around every step on its own stream (the
            # start event completes when the stream reaches the step, so this is the step's time
            # from its start to its end, sharing the GPU with the other streams' steps)
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)]
            for i in range(args.steps):
                evs[i][0].record(sts[i % S])
                step(i)
                evs[i][1].record(sts[i % S])
            torch.cuda.synchronize()
            per = np.array([a.elapsed_time(b) for a, b in evs])
            return ms, wall, per

        ms, wall, per = timed_steps(n_streams)
        ms_s, ms1, per1, used = ms, ms, per, n_streams
        if n_streams > 1:
            ms1, _, per1 = timed_steps(1)
            if ms1 < ms:   # report the faster schedule (the streams' gain is measured, not assumed)
                ms, per, used = ms1, per1, 1

        # per-kernel durations: each kernel launched back to back over K distinct rotating copies,
        # with events only around each run of K launches (an event between two kernels drains the
        # queue, and the drain would be charged to the kernel).  Every copy still goes through the
        # forward passes and then the inverse passes in order, so it ends as it started.
        if fused:
            names = ["fwd_fused", "inv_fused"]
        else:
            names = (["fwd_col", "fwd_row"] if npass == 2 else ["fwd_row"]) + \
                    (["inv_row", "inv_col"] if npass == 2 else ["inv_row"])
        K = min(R, args.steps)
        reps = max(1, args.steps // K)
        runs = []
        for _ in range(reps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * npass + 1)]
            ev[0].record()
            for p in range(npass):
                for i in range(K):
                    ntt.ntt_forward_pass(plan, bufs[i], p)
                ev[1 + p].record()
            for p in range(npass):
                for i in range(K):
                    ntt.ntt_inverse_pass(plan, bufs[i], p)
                ev[1 + npass + p].record()
            runs.append(ev)
        torch.cuda.synchronize()
        kms = {n: float(np.mean([ev[j].elapsed_time(ev[j + 1]) / K for ev in runs]))
               for j, n in enumerate(names)}

        # plain path: one call per polynomial
        for i in range(3):
            for p in range(P):
                ntt.ntt_forward(plan, bufs[i % R][p])
                ntt.ntt_inverse(plan, bufs[i % R][p])
        torch.cuda.synchronize()
        pe0, pe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        pe0.record()
        for i in range(args.steps):
            b = bufs[i % R]
            for p in range(P):
                ntt.ntt_forward(plan, b[p])
            for p in range(P):
                ntt.ntt_inverse(plan, b[p])
        pe1.record()
        torch.cuda.synchronize()
        plain_ms = pe0.elapsed_time(pe1) / args.steps

        ok = bool(torch.equal(bufs[0], dev0) and torch.equal(bufs[R - 1], dev0))
        results[mode] = dict(plan=plan, info=info, npass=npass, ms=ms, ms1=ms1, per=per, per1=per1, used=used,
                             wall=wall, kms=kms,
                             plain_ms=plain_ms, roundtrip_ok=ok)
        log(f"[{mode}] {ms_s*1e3:.1f} us/step over {n_streams} streams, {ms1*1e3:.1f} on one  "
            f"({180/ms*1e3/1e6:.3f} M NTTs/s)  kernels(us): "
            + ", ".join(f"{k}={v*1e3:.1f}" for k, v in kms.items())
            + f"  plain {plain_ms*1e3:.1f} us/step  roundtrip_ok={ok}")

    best = min(results, key=lambda m: results[m]["ms"])
    r = results[best]
    info = r["info"]
    ots = info["ot_stages"] if info["twiddle_mode"] == ntt.TWIDDLE_OT else 0
    n_limb_ntts = 2 * P * L
    value = n_limb_ntts / (r["ms"] * 1e-3)

    # roofline of the dominant kernel
    dom = max(r["kms"], key=r["kms"].get)
    kind = dom.split("_")[1]
    alg_bytes = data_bytes(kind, N, L, P) + twiddle_bytes(kind, N, L, info["log2_n1"], ots)
    achieved = alg_bytes / (r["kms"][dom] * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    traffic = read_traffic(f"{variant_key(info, ots)}:{dom}", src_hash)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "kernel_us": round(r["kms"][dom] * 1e3, 2), "alg_bytes_per_launch": alg_bytes}
    # the same kernel against the VALU issue rate: executed instructions from the counters
    valu = read_traffic(f"{variant_key(info, ots)}:{dom}", src_hash, field="valu_insts_per_launch")
    valu_issue = None
    if valu is not None:
        ginst = valu / (r["kms"][dom] * 1e-3) / 1e9
        valu_issue = {"kernel": dom, "insts_per_launch": int(valu), "achieved_ginst_s": round(ginst, 1),
                      "peak_ginst_s": VALU_ISSUE_PEAK_GINST, "frac": round(ginst / VALU_ISSUE_PEAK_GINST, 4)}
    step_bytes = 2 * sum(16 * P * L * N + twiddle_bytes(k, N, L, info["log2_n1"], ots)
                         for k in (["col", "row"] if info["log2_n1"] else ["row"]))
    step_frac = step_bytes / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS

    # warm figure, labelled apart: every step on the same copy on one stream, so its 47 MB stay
    # in the 256 MB Infinity Cache between steps (the headline rotates through copies instead)
    wplan = r["plan"]
    for _ in range(args.warmup):
        ntt.ntt_forward(wplan, bufs[0])
        ntt.ntt_inverse(wplan, bufs[0])
    torch.cuda.synchronize()
    w0, w1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0.record()
    for _ in range(args.steps):
        ntt.ntt_forward(wplan, bufs[0])
        ntt.ntt_inverse(wplan, bufs[0])
    w1.record()
    torch.cuda.synchronize()
    warm_ms = w0.elapsed_time(w1) / args.steps
    log(f"[warm, one copy, one stream] {warm_ms * 1e3:.1f} us/step")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(host, primes, N, r["plan"], bufs, dev0, n_limb_ntts)
    # the same kernel against what a plain device copy reaches on this GPU (the copies overwrite
    # the rotating buffers, which are not used after this)
    copies = copy_bandwidth(torch, bufs)
    # the yardstick is a copy at the passes' own granularity: one ciphertext per launch
    copy_gbs = max(copies["library"], copies["torch"])
    roofline["copy_gbs"] = round(copy_gbs, 1)
    roofline["copy_gbs_by_kernel"] = {k: round(v, 1) for k, v in copies.items()}
    roofline["frac_of_copy"] = round(achieved / copy_gbs, 4)
    log(f"device copy: {copy_gbs:.0f} GB/s (" + ", ".join(f"{k} {v:.0f}" for k, v in copies.items())
        + f"); dominant kernel at {achieved / copy_gbs:.3f} of the faster per-ciphertext copy")
    for m in results:
        results[m]["plan"].destroy()
    del bufs
    torch.cuda.empty_cache()
    polymul = None if args.no_polymul else polymul_bench(args)
    ablation = None if args.no_ablation else ablation_bench(args)
    word32 = None if args.no_word32 else word32_bench(args, r["ms1"])   # both on one stream
    crt = None if args.no_crt else crt_bench(args)
    uneven = None if args.no_uneven else uneven_batch_bench(args)
    serving = serve_bench(args) if args.serve_seconds > 0 else None

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "limb-NTTs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "one ciphertext, N=2^16, L=45 primes in [2^59,2^60) (seed 2), 2 polys, "
                               "forward NTT then inverse NTT (180 limb-NTTs per step); independent steps over "
                               "rotating copies, issued round-robin on `streams` streams",
                   "N": N, "L": L, "polys": P, "variant": best, "plan": variant_key(info, ots),
                   "ot_stages": ots, "log2_n1": info["log2_n1"], "rotating_copies": R,
                   "streams": r["used"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_hbm_frac": round(step_frac, 4),
        "valu_issue": valu_issue,
        "p50_ms": round(float(np.percentile(r["per"], 50)), 5),
        "p99_ms": round(float(np.percentile(r["per"], 99)), 5),
        "plain_value": round(n_limb_ntts / (r["plain_ms"] * 1e-3), 1),
        "single_stream_value": round(n_limb_ntts / (r["ms1"] * 1e-3), 1),
        "single_stream_ms_per_step": round(r["ms1"], 5),
        "single_stream_p50_ms": round(float(np.percentile(r["per1"], 50)), 5),
        "single_stream_p99_ms": round(float(np.percentile(r["per1"], 99)), 5),
        "warm_same_buffer_ms_per_step": round(warm_ms, 5),
        "kernel_us": {k: round(v * 1e3, 2) for k, v in r["kms"].items()},
        "modes_us_per_step": {m: round(results[m]["ms"] * 1e3, 2) for m in results},
        "modes_us_per_step_one_stream": {m: round(results[m]["ms1"] * 1e3, 2) for m in results},
        "roundtrip_ok": r["roundtrip_ok"],
        "autotune": tuned,
        "plan_create_ms": plan_ms,
        "polymul": polymul,
        "ablation": ablation,
        "word32": word32,
        "crt": crt,
        "uneven_batch": uneven,
        "serving": serving,
        "source_hash": src_hash,
    }
    print(json.dumps(out), flush=True)
    return 0


POLYMUL = dict(logN=17, L=60, polys=2, bits=60, seed=3)


def polymul_profile_run(args) -> int:
    """Counter driver for the product workload: `args.steps` products c = a * b with one named
    plan, then one plain device copy of an operand (its bytes calibrate the counters)."""
    import torch
    import synth
    import paper_2012_01968_amd as ntt

    cfg = POLYMUL
    N, L, P = 1 << cfg["logN"], cfg["L"], cfg["polys"]
    primes = synth.gen_primes(cfg["seed"], N, cfg["bits"], L)
    host = synth.residue_batch(cfg["seed"], primes, N, 2 * P)
    da = torch.from_numpy(np.ascontiguousarray(host[:P]).view(np.int64)).to("cuda")
    db = torch.from_numpy(np.ascontiguousarray(host[P:]).view(np.int64)).to("cuda")
    dc = torch.empty_like(da)
    mode = "table-split" if args.variant in ("auto", "tuned") else args.variant
    plan = ntt.ntt_plan_create(N, primes, log2_n1=args.log2_n1, **VARIANTS[mode])
    for _ in range(args.steps):
        ntt.ntt_polymul_negacyclic(plan, da, db, dc)
    torch.cuda.synchronize()
    dc.copy_(da)                     # calibration: one plain copy of P*L*N*8 bytes each way
    torch.cuda.synchronize()
    plan.destroy()
    log(f"profile run: {args.steps} products ({mode}, log2_n1={args.log2_n1}) + one {da.numel() * 8}-byte copy")
    return 0


def polymul_bench(args):
    """Negacyclic products at N = 2^17, L = 60: c = a * b for 2-polynomial operands a and b
    (a ciphertext pair: forward NTT of a and of b, element-wise product, inverse NTT), with
    table and OT twiddles.  Reports time per product on one stream and for independent
    products issued over --streams streams, the twiddle bytes each plan reads per product, and
    checks every product against the oracle."""
    import torch
    import oracle
    import synth
    import paper_2012_01968_amd as ntt

    cfg = POLYMUL
    N, L, P = 1 << cfg["logN"], cfg["L"], cfg["polys"]
    primes = synth.gen_primes(cfg["seed"], N, cfg["bits"], L)
    host = synth.residue_batch(cfg["seed"], primes, N, 2 * P)
    da = torch.from_numpy(np.ascontiguousarray(host[:P]).view(np.int64)).to("cuda")
    db = torch.from_numpy(np.ascontiguousarray(host[P:]).view(np.int64)).to("cuda")
    dc = torch.empty_like(da)
    limb_ntts = 3 * P * L                     # NTT(a), NTT(b), inverse of the product
    out = {"workload": f"c = a * b mod (X^N + 1, q_l), N=2^{cfg['logN']}, L={L} primes in [2^59,2^60) "
                       f"(seed {cfg['seed']}), a and b of {P} polys each ({limb_ntts} limb-NTTs per product)"}
    modes = {"table": dict(kernel_path=1), "ot": dict(kernel_path=1, twiddle_mode=2, ot_stages=2)}
    if not args.no_tune:
        modes["tuned"] = tune_shape(N, primes, P)["opts"]
    steps = max(5, min(args.steps, 50))
    S = max(1, args.streams)
    want = None
    for name, opts in modes.items():
        plan = ntt.ntt_plan_create(N, primes, **opts)
        info = ntt.ntt_plan_get_info(plan)
        ots = info["ot_stages"] if info["twiddle_mode"] == ntt.TWIDDLE_OT else 0
        step = lambda i: ntt.ntt_polymul_negacyclic(plan, da, db, dc)
        ramp(step, args.ramp_ms)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(steps):
            step(i)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        if want is None:
            want = oracle.polymul(host[:P], host[P:], primes, oracle.roots(primes, N),
                                  max(1, min(16, os.cpu_count() or 1)))
        ok = bool(np.array_equal(dc.cpu().numpy().view(np.uint64), want))
        # independent products round-robin over streams (product i on stream i mod S, into its
        # own output; a and b are only read), as the headline's steps
        ms_s = None
        if S > 1:
            cs = [torch.empty_like(da) for _ in range(S)]
            sts = [torch.cuda.Stream() for _ in range(S)]
            step_s = lambda i: ntt.ntt_polymul_negacyclic(plan, da, db, cs[i % S], None, sts[i % S])
            ramp(step_s, args.ramp_ms)
            torch.cuda.synchronize()
            main_st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(main_st)
            for st in sts:
                st.wait_event(e0)
            for i in range(steps):
                step_s(i)
            for st in sts:
                done = torch.cuda.Event()
                done.record(st)
                main_st.wait_event(done)
            e1.record(main_st)
            torch.cuda.synchronize()
            ms_s = e0.elapsed_time(e1) / steps
            ok = ok and all(bool(np.array_equal(c.cpu().numpy().view(np.uint64), want)) for c in cs)
            del cs
        # twiddle bytes read per product: forward column and row passes of a and of b, the
        # fused rows (forward and inverse row twiddles) and the inverse column pass
        n1 = info["log2_n1"]
        col = twiddle_bytes("col", N, L, n1, ots) if n1 else 0
        row = twiddle_bytes("row", N, L, n1, ots)
        tw = 3 * col + 3 * row if n1 else 3 * row
        out[name] = {"plan": variant_key(info, ots), "ms_per_product": round(ms, 4),
                     "limb_ntts_per_s": round(limb_ntts / (ms * 1e-3), 1),
                     "twiddle_mb_per_product": round(tw / 1e6, 2), "matches_oracle": ok}
        if ms_s is not None:
            out[name].update({"streams": S, "ms_per_product_streams": round(ms_s, 4),
                              "limb_ntts_per_s_streams": round(limb_ntts / (ms_s * 1e-3), 1)})
        log(f"[polymul {name}] {ms:.3f} ms/product  {limb_ntts / ms / 1e3:.3f} M limb-NTTs/s  "
            + (f"({ms_s:.3f} ms over {S} streams)  " if ms_s is not None else "")
            + f"twiddles {tw / 1e6:.1f} MB/product  oracle={'ok' if ok else 'MISMATCH'}")
        plan.destroy()
    del da, db, dc
    torch.cuda.empty_cache()
    return out


UNEVEN = dict(polys=256, logNs=(13, 14, 15, 16, 17), weights=(0.1, 0.2, 0.3, 0.3, 0.1), L=(4, 60), bits=60,
              seed=4)


def uneven_batch_bench(args):
    """256 independent polynomials of uneven N and limb count, forward then inverse NTT
    each, as one batch: one plain call sequence per polynomial, grouped launches, the grouped
    launches replayed from a captured hipGraph (sequential or branched), and steps replayed
    over --streams streams from batches of their own copies."""
    import torch
    import synth
    import paper_2012_01968_amd as ntt

    cfg = UNEVEN
    Lmax = cfg["L"][1]
    chain, logNs, Ls = uneven_jobs(cfg)
    plans, plan_names = {}, {}
    for k in cfg["logNs"]:
        k = int(k)
        # the batch holds this many limb-vectors of size 2^k: tune for that many full polynomials
        polys_k = max(1, -(-int(Ls[logNs == k].sum()) // Lmax))
        opts = {} if args.no_tune else tune_shape(1 << k, chain, polys_k)["opts"]
        plans[k] = ntt.ntt_plan_create(1 << k, chain, **opts)
        info = ntt.ntt_plan_get_info(plans[k])
        plan_names[k] = variant_key(info, info["ot_stages"] if info["twiddle_mode"] == ntt.TWIDDLE_OT else 0)
    src = {k: torch.from_numpy(synth.residue_batch(cfg["seed"] + k, chain, 1 << k, 1).view(np.int64)).to("cuda")
           .view(Lmax, 1 << k) for k in plans}
    jobs, bufs = [], []
    for i, (k, L) in enumerate(zip(logNs.tolist(), Ls.tolist())):
        b = src[k][:L].clone()
        bufs.append(b)
        jobs.append((plans[k], b, 1, L if L < Lmax else 0, ntt.OP_FORWARD_INVERSE))
    limb_ntts = 2 * int(Ls.sum())
    data_gib = sum(b.numel() for b in bufs) * 8 / 2**30
    batch = ntt.ntt_batch_create(jobs)
    out = {"workload": f"{cfg['polys']} polys, N from 2^13..2^17 (weights {list(cfg['weights'])}), "
                       f"L uniform in [{cfg['L'][0]}, {cfg['L'][1]}], forward+inverse each (seed {cfg['seed']})",
           "limb_ntts_per_step": limb_ntts, "data_gib": round(data_gib, 3),
           "polys_by_logN": {int(k): int((logNs == k).sum()) for k in cfg["logNs"]},
           "plans": plan_names}
    steps = max(5, min(args.steps, 40))
    for name, mode in (("plain", ntt.BATCH_PLAIN), ("grouped", ntt.BATCH_GROUPED), ("graph", ntt.BATCH_GRAPH),
                       ("graph_branched", ntt.BATCH_GRAPH_BRANCHED)):
        ramp(lambda i: ntt.ntt_batch_run(batch, mode), args.ramp_ms)
        for _ in range(3):
            ntt.ntt_batch_run(batch, mode)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(steps):
            ntt.ntt_batch_run(batch, mode)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        evs[0].record()
        for i in range(steps):
            ntt.ntt_batch_run(batch, mode)
            evs[i + 1].record()
        torch.cuda.synchronize()
        per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
        out[name] = {"ms_per_step": round(ms, 4), "limb_ntts_per_s": round(limb_ntts / (ms * 1e-3), 1),
                     "p50_ms": round(float(np.percentile(per, 50)), 4),
                     "p99_ms": round(float(np.percentile(per, 99)), 4)}
        log(f"[uneven {name}] {ms:.3f} ms/step  {limb_ntts / ms / 1e3:.3f} M limb-NTTs/s")
    # independent steps over two streams, as the headline's: a second batch of the same jobs on
    # copies of their own, and step i replays batch i mod 2's graph on stream i mod 2
    S = max(1, args.streams)
    if S > 1:
        extra = []
        for _ in range(S - 1):
            bufs_s = [b.clone() for b in bufs]
            extra.append((bufs_s, ntt.ntt_batch_create(
                [(j[0], b, j[2], j[3], j[4]) for j, b in zip(jobs, bufs_s)])))
        batches = [batch] + [bt for _, bt in extra]
        sts = [torch.cuda.Stream() for _ in range(S)]
        step_s = lambda i: ntt.ntt_batch_run(batches[i % S], ntt.BATCH_GRAPH, sts[i % S])
        ramp(step_s, args.ramp_ms)
        torch.cuda.synchronize()
        main_st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(main_st)
        for st in sts:
            st.wait_event(e0)
        for i in range(steps):
            step_s(i)
        for st in sts:
            done = torch.cuda.Event()
            done.record(st)
            main_st.wait_event(done)
        e1.record(main_st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out["graph_streams"] = {"streams": S, "ms_per_step": round(ms, 4),
                                "limb_ntts_per_s": round(limb_ntts / (ms * 1e-3), 1)}
        log(f"[uneven graph over {S} streams] {ms:.3f} ms/step  {limb_ntts / ms / 1e3:.3f} M limb-NTTs/s")
        for bufs_s, bt in extra:
            bufs = bufs + bufs_s
            bt.destroy()
    ok = all(torch.equal(b, src[k][:L]) for b, k, L in
             zip(bufs, logNs.tolist() * (len(bufs) // len(logNs)), Ls.tolist() * (len(bufs) // len(Ls))))
    out["roundtrip_ok"] = bool(ok)
    out["matches_oracle"] = uneven_forward_matches_oracle(plans, src, chain, logNs, Ls, Lmax)
    log(f"[uneven] forward of all {cfg['polys']} polys (grouped and both graph runs) "
        f"{'matches' if out['matches_oracle'] else 'DIFFERS FROM'} the oracle")
    out["graph_vs_plain"] = round(out["plain"]["ms_per_step"] / out["graph"]["ms_per_step"], 3)
    out["branched_vs_plain"] = round(out["plain"]["ms_per_step"] / out["graph_branched"]["ms_per_step"], 3)
    batch.destroy()
    for p in plans.values():
        p.destroy()
    return out


def uneven_jobs(cfg=None):
    """The uneven workload: the prime chain, each polynomial's log2 N and limb count."""
    import synth
    cfg = cfg or UNEVEN
    chain = synth.gen_primes(cfg["seed"], 1 << max(cfg["logNs"]), cfg["bits"], cfg["L"][1])
    rng = np.random.default_rng(cfg["seed"])
    logNs = rng.choice(cfg["logNs"], size=cfg["polys"], p=cfg["weights"])
    Ls = rng.integers(cfg["L"][0], cfg["L"][1] + 1, size=cfg["polys"])
    return chain, logNs, Ls


def uneven_forward_matches_oracle(plans, src, chain, logNs, Ls, Lmax) -> bool:
    """Forward NTT of every polynomial of the uneven batch (one batch of forward jobs, run
    grouped and replayed from its sequential and its branched graph) against the oracle.  Each polynomial is the first L
    limbs of its size's source polynomial, so the expected output is the first L limbs of the
    oracle's forward transform of that source."""
    import torch
    import oracle
    import paper_2012_01968_amd as ntt

    want = {k: oracle.forward(src[k].cpu().numpy().view(np.uint64), chain, oracle.roots(chain, 1 << k),
                              max(1, min(16, os.cpu_count() or 1))) for k in plans}
    ok = True
    for mode in (ntt.BATCH_GROUPED, ntt.BATCH_GRAPH, ntt.BATCH_GRAPH_BRANCHED):
        bufs, jobs = [], []
        for k, L in zip(logNs.tolist(), Ls.tolist()):
            b = src[k][:L].clone()
            bufs.append(b)
            jobs.append((plans[k], b, 1, L if L < Lmax else 0, ntt.OP_FORWARD))
        batch = ntt.ntt_batch_create(jobs)
        ntt.ntt_batch_run(batch, mode)
        torch.cuda.synchronize()
        for b, k, L in zip(bufs, logNs.tolist(), Ls.tolist()):
            ok &= bool(np.array_equal(b.cpu().numpy().view(np.uint64), want[k][:L]))
        batch.destroy()
        del bufs
    return ok


ABLATION = dict(logNs=(14, 15, 16, 17), L=21, bits=60, seed=6)
# Table II (Titan V, microseconds for the 21-limb forward NTT), context only
PAPER_TABLE2_US = {14: {"radix2": 166, "smem": 48.6, "smem_ot": 44.1}, 15: {"radix2": 340, "smem": 92.0, "smem_ot": 84.2},
                   16: {"radix2": 693, "smem": 171.8, "smem_ot": 156.3},
                   17: {"radix2": 1427, "smem": 329.0, "smem_ot": 304.2}}


def ablation_bench(args):
    """The paper's ablation ladder (Table II) on this GPU: forward NTT of one polynomial of 21
    limbs (60-bit primes, seed 6) at N = 2^14 .. 2^17 by the radix-2 path (one launch per
    stage), the register-only path at radix 4 .. 32, and the two-pass path with table
    twiddles and with OT on the last two stages (base 2^10).  Inputs rotate through copies
    larger than the Infinity Cache; each plan's first forward is checked against the oracle."""
    import torch
    import oracle
    import synth
    import paper_2012_01968_amd as ntt

    cfg = ABLATION
    L = cfg["L"]
    variants = {"radix2": dict(kernel_path=ntt.PATH_RADIX2)}
    for k in (2, 3, 4, 5):
        variants[f"register_radix{1 << k}"] = dict(kernel_path=ntt.PATH_REGISTER, log2_radix=k)
    variants["two_pass_table"] = dict(kernel_path=ntt.PATH_SPLIT)
    variants["two_pass_ot"] = dict(kernel_path=ntt.PATH_SPLIT, twiddle_mode=ntt.TWIDDLE_OT, ot_stages=2,
                                   ot_log2_base=10)
    out = {"workload": f"forward NTT of 1 poly x {L} limbs (60-bit primes, seed {cfg['seed']}), N = 2^14..2^17; "
                       "Table II's ladder", "paper_titan_v_us": PAPER_TABLE2_US}
    steps = max(5, min(args.steps, 40))
    for logN in cfg["logNs"]:
        N = 1 << logN
        primes = synth.gen_primes(cfg["seed"], N, cfg["bits"], L)
        host = synth.residue_batch(cfg["seed"], primes, N, 1)
        want = oracle.forward(host, primes, oracle.roots(primes, N), max(1, min(16, os.cpu_count() or 1)))
        x = torch.from_numpy(host.view(np.int64)).to("cuda")
        R = max(2, int(np.ceil(512 * 2**20 / (x.numel() * 8))))
        bufs = x.unsqueeze(0).repeat(R, 1, 1, 1)
        row = {}
        ok = True
        for name, opts in variants.items():
            plan = ntt.ntt_plan_create(N, primes, **opts)
            d = x.clone()
            ntt.ntt_forward(plan, d)
            torch.cuda.synchronize()
            ok &= bool(np.array_equal(d.cpu().numpy().view(np.uint64), want))
            ramp(lambda i: ntt.ntt_forward(plan, bufs[i % R]), args.ramp_ms)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(steps):
                ntt.ntt_forward(plan, bufs[i % R])
            e1.record()
            torch.cuda.synchronize()
            row[name + "_us"] = round(e0.elapsed_time(e1) * 1e3 / steps, 2)
            plan.destroy()
        reg = {k: row[f"register_radix{1 << k}_us"] for k in (2, 3, 4, 5)}
        best_k = min(reg, key=reg.get)
        row["best_register_radix"] = 1 << best_k
        row["speedup_two_pass_ot_vs_radix2"] = round(row["radix2_us"] / row["two_pass_ot_us"], 3)
        row["speedup_two_pass_table_vs_radix2"] = round(row["radix2_us"] / row["two_pass_table_us"], 3)
        row["speedup_best_register_vs_radix2"] = round(row["radix2_us"] / reg[best_k], 3)
        row["ot_gain"] = round(row["two_pass_table_us"] / row["two_pass_ot_us"] - 1, 4)
        row["limb_ntts_per_s_two_pass_best"] = round(
            L / (min(row["two_pass_table_us"], row["two_pass_ot_us"]) * 1e-6), 1)
        row["matches_oracle"] = ok
        out[str(logN)] = row
        log(f"[ablation 2^{logN} x {L}] " + ", ".join(f"{k}={v}" for k, v in row.items()))
        del bufs, x
        torch.cuda.empty_cache()
    return out


WORD32 = dict(N=1 << 16, L=90, P=2, bits=30, seed=7)


def word32_bench(args, headline_ms):
    """The 32-bit word path at the headline's modulus budget: one ciphertext of 2 polys at
    N = 2^16 over 90 primes below 2^30 (about the 45 x 60 bits of the 64-bit workload),
    forward then inverse per step (360 limb-NTTs), over rotating copies larger than the
    Infinity Cache; checked against the oracle."""
    import torch
    import oracle
    import synth
    import paper_2012_01968_amd as ntt

    cfg = WORD32
    N, L, P = cfg["N"], cfg["L"], cfg["P"]
    primes = synth.gen_primes(cfg["seed"], N, cfg["bits"], L)
    host = synth.residue_batch(cfg["seed"], primes, N, P)
    x = torch.from_numpy(host.astype(np.int32)).to("cuda")
    R = max(2, int(np.ceil(args.rotate_gib * 2**30 / (x.numel() * 4))))
    bufs = x.unsqueeze(0).repeat(R, 1, 1, 1)
    plan = ntt.ntt_plan_create(N, primes, word_bits=32)
    d = x.clone()
    ntt.ntt_forward_u32(plan, d)
    torch.cuda.synchronize()
    want = oracle.forward(host, primes, oracle.roots(primes, N), max(1, min(16, os.cpu_count() or 1)))
    ok = bool(np.array_equal(d.cpu().numpy().astype(np.uint64), want))

    def step(i):
        ntt.ntt_forward_u32(plan, bufs[i % R])
        ntt.ntt_inverse_u32(plan, bufs[i % R])

    ramp(step, args.ramp_ms)
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        step(i)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    ok &= bool(torch.equal(bufs[0], x))
    info = ntt.ntt_plan_get_info(plan)
    plan.destroy()
    limb_ntts = 2 * P * L
    # two passes per direction, 4 B read + 4 B written per coefficient and pass, 8 B per twiddle
    n1 = 1 << info["log2_n1"] if info["log2_n1"] else 1
    step_bytes = 2 * (2 * 8 * P * L * N + 8 * L * N) if info["log2_n1"] else 2 * (8 * P * L * N + 8 * L * N)
    del bufs
    torch.cuda.empty_cache()
    out = {"workload": f"one ciphertext, N=2^16, L={L} primes in [2^29,2^30) (seed {cfg['seed']}), {P} polys, "
                       "forward+inverse", "log2_n1": info["log2_n1"], "n1": n1,
           "ms_per_step": round(ms, 5), "limb_ntts_per_s": round(limb_ntts / (ms * 1e-3), 1),
           "modulus_bits": sum(q.bit_length() for q in primes),
           "step_hbm_frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "speedup_vs_64bit_headline": round(headline_ms / ms, 3) if headline_ms else None,
           "matches_oracle": ok}
    log(f"[word32] {ms * 1e3:.1f} us/step ({limb_ntts / ms / 1e3:.3f} M limb-NTTs/s), "
        f"{headline_ms / ms if headline_ms else float('nan'):.2f}x the 64-bit step, oracle={'ok' if ok else 'MISMATCH'}")
    return out


def crt_bench(args):
    """RNS <-> integer conversions at the headline shape (N = 2^16, 45 primes of 60 bits,
    2 polys): integers below Q to residues and back, time per call, with the first 256
    coefficients of each polynomial checked against the oracle."""
    import torch
    import oracle
    import synth
    import paper_2012_01968_amd as ntt

    N, L, P = WORKLOAD["N"], WORKLOAD["L"], WORKLOAD["P"]
    primes = synth.gen_primes(WORKLOAD["seed"], N, WORKLOAD["bits"], L)
    Q = 1
    for q in primes:
        Q *= q
    plan = ntt.ntt_plan_create(N, primes)
    W = ntt.ntt_crt_words(plan)
    words = np.stack([synth.uniform_wide(13, p, Q, N) for p in range(P)])
    dw = torch.from_numpy(words.view(np.int64)).to("cuda")
    res = torch.empty((P, L, N), dtype=torch.int64, device="cuda")
    back = torch.empty_like(dw)
    out = {"workload": f"{P} polys, N=2^16, integers below Q = product of {L} primes of 60 bits ({W} words)"}
    for name, fn in (("decompose", lambda: ntt.ntt_rns_decompose(plan, dw, W, res)),
                     ("reconstruct", lambda: ntt.ntt_crt_reconstruct(plan, res, back))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_us"] = round(e0.elapsed_time(e1) * 1e3 / 10, 2)
    k = 256
    got_res = res.cpu().numpy().view(np.uint64)[:, :, :k]
    ok = bool(np.array_equal(got_res, oracle.rns_decompose_words(words[:, :, :k], primes)))
    ok &= bool(np.array_equal(back.cpu().numpy().view(np.uint64), words))
    out["matches_oracle"] = ok
    plan.destroy()
    log(f"[crt] decompose {out['decompose_us']} us, reconstruct {out['reconstruct_us']} us, oracle={'ok' if ok else 'MISMATCH'}")
    return out


SERVE = dict(logNs=(14, 15, 16), L=(8, 45), polys=2, bits=60, seed=5, lanes=3, capacity_gib=8.0)


def serve_bench(args):
    """Poisson request stream: each request is one ciphertext (2 polys) that needs the
    forward NTT, a product with a resident NTT-domain key and the inverse NTT.  The
    continuous-batching loop and the one-launch-per-request path serve the same stream;
    a saturated run (every request waiting at t=0) gives each one's peak rate."""
    import torch
    import synth
    import paper_2012_01968_amd as ntt
    from paper_2012_01968_amd.serve import GpuExecutor, Request, Server

    cfg = SERVE
    Lmax = cfg["L"][1]
    chain = synth.gen_primes(cfg["seed"], 1 << max(cfg["logNs"]), cfg["bits"], Lmax)
    plans, keys, src = {}, {}, {}
    for k in cfg["logNs"]:
        N = 1 << k
        plans[N] = ntt.ntt_plan_create(N, chain, **({} if args.no_tune else tune_shape(N, chain, cfg["polys"])["opts"]))
        key = torch.from_numpy(synth.residue_batch(cfg["seed"] * 100 + k, chain, N, 1).view(np.int64)).to("cuda")
        ntt.ntt_forward(plans[N], key)
        keys[N] = key.view(Lmax, N)
        src[N] = torch.from_numpy(synth.residue_batch(cfg["seed"] + k, chain, N, cfg["polys"]).view(np.int64)) \
            .to("cuda").view(cfg["polys"], Lmax, N)
    torch.cuda.synchronize()

    def requests(n, rate, seed):
        rng = np.random.default_rng(seed)
        t = np.cumsum(rng.exponential(1.0 / rate, n)) if rate > 0 else np.zeros(n)
        ks = rng.choice(cfg["logNs"], size=n)
        Ls = rng.integers(cfg["L"][0], cfg["L"][1] + 1, size=n)
        return [Request(i, 1 << int(k), int(L), float(t[i]), polys=cfg["polys"], payload=src[1 << int(k)][:, :int(L)])
                for i, (k, L) in enumerate(zip(ks.tolist(), Ls.tolist()))]

    cap = int(cfg["capacity_gib"] * 2**30)
    n = int(round(args.serve_rate * args.serve_seconds))
    out = {"workload": f"Poisson arrivals at {args.serve_rate:g}/s for {args.serve_seconds:g} s ({n} requests, "
                       f"seed {cfg['seed']}); request = 2 polys, N in {{2^14, 2^15, 2^16}}, L uniform in "
                       f"[{cfg['L'][0]}, {cfg['L'][1]}]; forward NTT, product with resident key, inverse NTT",
           "arena_gib": cfg["capacity_gib"], "lanes": cfg["lanes"]}
    for policy, mode, lanes in (("continuous", ntt.BATCH_GROUPED, cfg["lanes"]), ("per_request", ntt.BATCH_PLAIN, 1)):
        ex = GpuExecutor(plans, keys, cap, lanes=lanes, mode=mode)
        Server(ex, cap, policy=policy).run(requests(64, 0, 99))             # warm-up
        st = Server(ex, cap, policy=policy).run(requests(n, args.serve_rate, cfg["seed"]))
        hi = None
        if args.serve_high_rate > 0:
            hi = Server(ex, cap, policy=policy).run(requests(int(5 * args.serve_high_rate), args.serve_high_rate,
                                                            cfg["seed"] + 2))
        sat = Server(ex, cap, policy=policy).run(requests(2000, 0, cfg["seed"] + 1))
        ex.close()
        out[policy] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.as_dict().items()}
        if hi is not None:
            out[policy + "_high_load"] = {"rate": args.serve_high_rate, "requests": hi.completed,
                                          "throughput_rps": round(hi.throughput_rps, 1), "p50_ms": round(hi.p50_ms, 3),
                                          "p99_ms": round(hi.p99_ms, 3), "mean_batch": round(hi.mean_batch, 2),
                                          "peak_gib": round(hi.peak_bytes / 2**30, 3)}
            log(f"[serve {policy} @ {args.serve_high_rate:g}/s] p50 {hi.p50_ms:.3f} ms p99 {hi.p99_ms:.3f} ms, "
                f"{hi.throughput_rps:.0f} req/s, mean batch {hi.mean_batch:.2f}")
        out[policy + "_saturated"] = {"requests": 2000, "throughput_rps": round(sat.throughput_rps, 1),
                                      "p50_ms": round(sat.p50_ms, 3), "p99_ms": round(sat.p99_ms, 3),
                                      "mean_batch": round(sat.mean_batch, 2), "peak_gib": round(sat.peak_bytes / 2**30, 3)}
        log(f"[serve {policy}] {st.completed} done, p50 {st.p50_ms:.3f} ms p99 {st.p99_ms:.3f} ms, "
            f"{st.throughput_rps:.0f} req/s, mean batch {st.mean_batch:.2f}; saturated {sat.throughput_rps:.0f} req/s "
            f"(p99 {sat.p99_ms:.1f} ms, mean batch {sat.mean_batch:.1f})")
        del ex
        torch.cuda.empty_cache()
    for p in plans.values():
        p.destroy()
    c, pr = out["continuous"], out["per_request"]
    out["p99_ratio_plain_over_continuous"] = round(pr["p99_ms"] / c["p99_ms"], 3)
    if "continuous_high_load" in out:
        out["high_load_p99_ratio_plain_over_continuous"] = round(
            out["per_request_high_load"]["p99_ms"] / out["continuous_high_load"]["p99_ms"], 3)
    out["saturated_speedup"] = round(out["continuous_saturated"]["throughput_rps"]
                                     / out["per_request_saturated"]["throughput_rps"], 3)
    return out


def host_cpu_facts() -> dict:
    """What the CPU baseline ran on: logical CPUs, CPUs this process may use, and the model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": model}


def cpu_baseline(host, primes, N, plan, bufs, dev0, n_limb_ntts, seconds: float = 6.0):
    """The CPU oracle (plain C, __int128 %) on this host, in two legs: one thread, and one
    thread per CPU this process may use (at most 16, the host's CPU share per GPU).  Each leg
    repeats forward + inverse of the same ciphertext until about `seconds` of wall time.
    Also checks the GPU forward output of that ciphertext against the oracle's."""
    import torch
    import oracle
    import paper_2012_01968_amd as ntt

    facts = host_cpu_facts()
    psis = oracle.roots(primes, N)

    def leg(threads):
        reps = 0
        t0 = time.perf_counter()
        while True:
            f = oracle.forward(host, primes, psis, threads)
            back = oracle.inverse(f, primes, psis, threads)
            reps += 1
            if time.perf_counter() - t0 > seconds:
                break
        wall = time.perf_counter() - t0
        return reps, wall, f, back

    r1, w1, _, _ = leg(1)
    threads = max(1, min(16, facts["affinity_cpus"]))
    reps, wall, f, back = leg(threads)
    d = dev0.clone()
    ntt.ntt_forward(plan, d)
    torch.cuda.synchronize()
    parity = bool(np.array_equal(d.cpu().numpy().view(np.uint64), f) and np.array_equal(back, host))
    log(f"cpu oracle: 1 thread {r1} step(s) in {w1:.2f} s; {threads} threads {reps} step(s) in {wall:.2f} s "
        f"({facts['cpu_model']}, nproc {facts['nproc']}, affinity {facts['affinity_cpus']}); "
        f"GPU forward parity={parity}")
    return {"value": round(n_limb_ntts * reps / wall, 1), "unit": "limb-NTTs/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} full step(s) on {threads} threads: forward+inverse of the 2x45x2^16 ciphertext "
                      f"(radix-2, __int128 %), threads over limb-vectors",
            "one_core": {"value": round(n_limb_ntts * r1 / w1, 1), "cores": 1,
                         "sample": f"{r1} full step(s) on 1 thread"},
            **facts,
            "gpu_forward_matches": parity}


def copy_bandwidth(torch, bufs) -> dict:
    """Device-to-device copy rates (GB/s, bytes read + written) over the rotating copies: copy
    i reads ciphertext i of the first half and writes ciphertext i of the second half, back to
    back between two events, once with the library's one-pass copy kernel (one 16-byte vector
    per lane; `library`) and once with torch's copy (`torch`).  Every read hits a buffer last
    touched more than the Infinity Cache's size ago, so the rates are HBM's.  Best of three.
    `library_one_launch` moves the same bytes in a single launch (all H ciphertexts at once): the
    difference is what the start and end of each ciphertext-sized launch cost."""
    import paper_2012_01968_amd as ntt
    R = bufs.shape[0]
    H = R // 2
    nbytes = bufs[0].numel() * 8
    out = {}
    for name, copy in (("library", lambda d, s: ntt.ntt_device_copy(d, s)), ("torch", lambda d, s: d.copy_(s))):
        copy(bufs[H], bufs[0])
        torch.cuda.synchronize()
        best = None
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(H):
                copy(bufs[H + i], bufs[i])
            e1.record()
            torch.cuda.synchronize()
            gbs = 2 * nbytes * H / (e0.elapsed_time(e1) * 1e-3) / 1e9
            best = gbs if best is None else max(best, gbs)
        out[name] = best
    # the same bytes in one launch: the library's copy of the whole first half into the second
    one = lambda: ntt.ntt_device_copy(bufs[H:2 * H], bufs[:H])
    one()
    torch.cuda.synchronize()
    best = None
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        one()
        e1.record()
        torch.cuda.synchronize()
        gbs = 2 * nbytes * H / (e0.elapsed_time(e1) * 1e-3) / 1e9
        best = gbs if best is None else max(best, gbs)
    out["library_one_launch"] = best
    return out


if __name__ == "__main__":
    sys.exit(main())
