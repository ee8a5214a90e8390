#!/usr/bin/env python3
"""Benchmark: 2^19-bit multiplications per second on one MI355X.

One step = one batched MFMA-split multiplication of 256 independent pairs of
2^19-bit integers (16384 u32 limbs each, uniform random limbs from seed 1002)
into their full 2^20-bit products: digit split, int8 MFMA Toeplitz
contraction with int32 accumulation, 64-bit recombination and the carry
scan, all in one kernel launch with the operands already resident in HBM.
The plain u64 schoolbook kernel is timed beside it on the same inputs and
both outputs are compared byte for byte.

Output: one JSON line (see the fields below).  ``--gpus N`` with N > 1 exits:
this benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2^19-bit muls/s on 1 GPU, MFMA-split vs plain u64 kernel, bit-exact"
# one v_mad_u64_u32 (32x32-bit product added to 64 bits) per lane per cycle:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (the register-only probe of
# --mode mfma-peak reaches 34.8 of it at about 2.1 GHz)
MAD_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
INT8_PEAK_TOPS = 5000.0      # MI355X dense int8 MFMA, TOP/s (2 ops per MAC)
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--batch", type=int, default=256)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="target CPU work (core-seconds) of the oracle sample")
    p.add_argument("--mode", default="bench",
                   choices=["bench", "copy", "mfma-peak", "ragged", "divmod", "addsub", "poly",
                            "configs", "cpu-oracle"],
                   help="copy: a plain copy kernel of known size (counter calibration); "
                        "mfma-peak: register-only int8 MFMA rate probe; ragged / divmod: the "
                        "4096-product ragged batch and the 512-division batch (extra lines)")
    p.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "mfma_mul_2e19_traffic.json"),
                   help="HBM traffic per launch from rocprofv3 counters, if measured")
    return p.parse_args()


def time_launches(fn, steps, warmup, torch, per_launch=None):
    """Run fn (one kernel launch on torch's current stream) warmup + steps
    times; returns (total_ms over the timed steps, mean per-launch ms from
    per-launch event pairs).  per_launch (a list), if given, receives every
    launch's ms."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for e0, e1 in ev:
        e0.record()
        fn()
        e1.record()
    t_end.record()
    torch.cuda.synchronize()
    total = t_start.elapsed_time(t_end)
    per = [e0.elapsed_time(e1) for e0, e1 in ev]
    if per_launch is not None:
        per_launch.extend(per)
    return total, float(np.mean(per))


def cpu_baseline(a_np, b_np, gpu_out, target_s):
    """The oracle (plain C schoolbook on u64 digits, as it stands) on a
    bounded sample of the same pairs, one pair per host thread; also checks
    the GPU products of the sampled pairs byte for byte."""
    import concurrent.futures as cf
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    first = oracle.mul1(a_np[0], b_np[0])
    one = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 64))
    n = int(max(cores, min(a_np.shape[0], target_s / max(one, 1e-3))))
    n = min(n, a_np.shape[0])
    idx = list(range(1, n))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        outs = list(ex.map(lambda i: oracle.mul1(a_np[i], b_np[i]), idx))
    wall = time.perf_counter() - t0
    exact = bool(np.array_equal(first, gpu_out[0]) and
                 all(np.array_equal(o, gpu_out[i]) for o, i in zip(outs, idx)))
    return {
        "value": round(len(idx) / wall, 3),
        "unit": "muls/s",
        "cores": cores,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": f"{len(idx)} of the {a_np.shape[0]} pairs (2^19 x 2^19 bits), one pair per thread, "
                  f"{cores} threads",
    }, exact, n


def cpu_model():
    """The host CPU's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the batched big-integer path has no "
              "multi-GPU step (instances are independent; see the sharding notes)", file=sys.stderr)
        sys.exit(2)

    if args.mode == "cpu-oracle":
        from paper_2607_28897_amd import inputs
        return cpu_oracle_mode(inputs, args)

    import torch
    import paper_2607_28897_amd as bi
    from paper_2607_28897_amd import inputs

    if args.mode == "copy":
        return copy_mode(torch)
    if args.mode == "mfma-peak":
        return peak_mode(torch, bi)
    if args.mode == "ragged":
        return ragged_mode(torch, bi, inputs, args)
    if args.mode == "divmod":
        return divmod_mode(torch, bi, inputs, args)
    if args.mode == "addsub":
        return addsub_mode(torch, bi, inputs, args)
    if args.mode == "poly":
        return poly_mode(torch, bi, args)
    if args.mode == "configs":
        return configs_mode(torch, bi, inputs, args)

    cfg = inputs.pairs_2e19(args.batch)
    a_np, b_np, n = cfg["a"], cfg["b"], cfg["n"]
    a = torch.from_numpy(a_np.view(np.int32)).cuda()
    b = torch.from_numpy(b_np.view(np.int32)).cuda()
    batch = a.shape[0]
    out_m = torch.empty((batch, 2 * n), dtype=torch.int32, device="cuda")
    L = bi.lib()
    import ctypes
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    pa, pb = ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr())

    def mul_call(out, algo):
        po = ctypes.c_void_p(out.data_ptr())

        def run():
            rc = L.bigint_mul(po, pa, n, pb, n, batch, algo, stream)
            if rc:
                raise bi.BigIntError(rc, "bigint_mul")
        return run

    torch.cuda.synchronize()
    # The plain u64 kernel first (it also brings the clocks up from idle),
    # then the MFMA-split headline, each after its own warm-up launches.
    out_p = torch.empty_like(out_m)
    p_steps = max(10, args.steps // 2)
    p_total, _ = time_launches(mul_call(out_p, bi.MUL_PLAIN), p_steps, max(1, args.warmup // 5), torch)
    print(f"# plain: {p_total / p_steps:.4f} ms/step", file=sys.stderr, flush=True)
    per = []
    total_ms, kernel_ms = time_launches(mul_call(out_m, bi.MUL_MFMA), args.steps, args.warmup, torch, per)
    print(f"# mfma: {total_ms / args.steps:.4f} ms/step", file=sys.stderr, flush=True)
    same = bool(torch.equal(out_m, out_p))
    del out_p

    ms = total_ms / args.steps
    value = batch / (ms * 1e-3)
    P, waves, dbits = bi.mfma_config(n, n)
    # executed work of one launch: the digit products of the tuned digit width
    # (offset 8-bit digits: Na = 4 n), 2 int8 ops each
    Nx = (32 * n + 6) // 7 if dbits == 7 else 4 * n
    ops = 2.0 * batch * Nx * Nx
    achieved = ops / (kernel_ms * 1e-3) / 1e12      # TOP/s
    N7 = (32 * n + 6) // 7
    seven = 2.0 * batch * N7 * N7 / (kernel_ms * 1e-3) / 1e12
    traffic = stored_traffic(args.traffic_json, kernel_sha())

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "muls/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "source_sha": source_sha(),
        "config": {
            "workload": f"{batch} pairs of 2^19-bit integers ({n} u32 limbs), uniform random limbs "
                        f"(seed 1002), full 2^20-bit products, MFMA-split multiply",
            "batch": batch,
            "operand_bits": 32 * n,
            "digit_bits": dbits,
            "digits_per_operand": Nx,
            "strips_per_band": P,
            "waves": waves,
        },
        "roofline": {
            "bound": "mfma",
            "achieved": round(achieved, 1),
            "peak": INT8_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": round(achieved / INT8_PEAK_TOPS, 4),
            "traffic": traffic,
            "kernel_ms": round(kernel_ms, 4),
            "kernel_ms_median": round(float(np.median(per)), 4),
            "kernel_ms_min": round(float(np.min(per)), 4),
            "algorithmic_unit": f"2 x {Nx:,}^2 int8 ops ({dbits}-bit digit products) per 2^19-bit product, "
                                f"{ops:.4g} per launch",
            "seven_bit_equivalent_TOPs": round(seven, 1),
            "seven_bit_equivalent_unit": f"2 x {N7:,}^2 int8 ops (7-bit digit products) per 2^19-bit product",
        },
        "plain": {
            "value": round(batch / (p_total / p_steps * 1e-3), 1),
            "unit": "muls/s",
            "ms_per_step": round(p_total / p_steps, 4),
            "steps": p_steps,
            "roofline": {
                "bound": "alu",
                "achieved": round(batch * n * n / (p_total / p_steps * 1e-3) / 1e12, 2),
                "peak": round(MAD_PEAK_TOPS, 1),
                "unit": "10^12 v_mad_u64_u32/s",
                "frac": round(batch * n * n / (p_total / p_steps * 1e-3) / 1e12 / MAD_PEAK_TOPS, 4),
                "algorithmic_unit": "n^2 = 16384^2 32x32-bit products (4 per 64x64-bit digit product) per 2^19-bit product",
            },
        },
        "mfma_equals_plain": same,
    }
    line["mfma_7bit"] = seven_bit_leg(torch, bi, mul_call, out_m, batch, n, args)
    line["karatsuba"] = karatsuba_leg(torch, bi, mul_call, out_m, batch, args)
    line["small_batches"] = small_batch_leg(torch, bi, a, b, out_m, n, args)
    line["ragged_4096"] = ragged_leg(torch, bi, inputs, args)
    line["divmod_512"] = divmod_leg(torch, bi, inputs, args)
    if not args.no_cpu:
        cpu, exact, _ = cpu_baseline(a_np, b_np, out_m.cpu().numpy().view(np.uint32), args.cpu_seconds)
        line["cpu_baseline"] = cpu
        line["bit_exact_sample"] = exact
    print(json.dumps(line), flush=True)


def mfma_roofline(int8_ops, ms, unit):
    a = int8_ops / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": round(a, 1), "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
            "frac": round(a / INT8_PEAK_TOPS, 4), "traffic": None, "algorithmic_unit": unit}


def seven_bit_leg(torch, bi, mul_call, ref, batch, n, args):
    """The 2^19-bit batch with the digit width forced to 7 bits (the
    configuration's tile as written), same inputs, same bytes."""
    out = torch.empty_like(ref)
    steps = max(5, args.steps // 2)
    bi.set_mfma_config(0, 0, 7)
    try:
        total, kern = time_launches(mul_call(out, bi.MUL_MFMA), steps, max(2, args.warmup // 2), torch)
    finally:
        bi.set_mfma_config(0, 0, 0)
    print(f"# mfma 7-bit: {total / steps:.4f} ms/step", file=sys.stderr, flush=True)
    N7 = (32 * n + 6) // 7
    ms = total / steps
    return {"value": round(batch / (ms * 1e-3), 1), "unit": "muls/s", "ms_per_step": round(ms, 4),
            "steps": steps, "digit_bits": 7,
            "roofline": mfma_roofline(2.0 * batch * N7 * N7, kern,
                                      f"2 x {N7:,}^2 int8 ops (7-bit digit products) per product"),
            "equals_8bit": bool(torch.equal(out, ref))}


def karatsuba_leg(torch, bi, mul_call, ref, batch, args):
    """One Karatsuba level (three 2^18-bit half products per pair) over the
    same MFMA-split multiply, same inputs."""
    out = torch.empty_like(ref)
    steps = max(5, args.steps // 2)
    total, _ = time_launches(mul_call(out, bi.MUL_KARATSUBA), steps, 2, torch)
    print(f"# karatsuba: {total / steps:.4f} ms/step", file=sys.stderr, flush=True)
    ms = total / steps
    return {"value": round(batch / (ms * 1e-3), 1), "unit": "muls/s", "ms_per_step": round(ms, 4),
            "steps": steps,
            "what": "one Karatsuba level (three 2^18-bit products per pair) over the same MFMA-split multiply",
            "equals_mfma": bool(torch.equal(out, ref))}


def small_batch_leg(torch, bi, a, b, ref, n, args):
    """The first 1 and 16 pairs of the same 2^19-bit batch alone: each
    product's bands split over several work-groups (k_mul_mfma_part, then
    k_mul_mfma_close); both equal the batch's products.  (One work-group per
    product takes about 0.52 ms for either, the headline kernel's time.)"""
    out = []
    steps = max(10, args.steps // 2)
    for k in (x for x in (1, 16) if x <= a.shape[0]):
        ta, tb = a[:k].contiguous(), b[:k].contiguous()
        p = bi.mul(ta, tb, bi.MUL_MFMA)
        total, _ = time_launches(lambda: bi.mul(ta, tb, bi.MUL_MFMA), steps, 2, torch)
        ms = total / steps
        out.append({"products": k, "parts_per_product": bi.mfma_split_parts(n, n, k), "ms": round(ms, 4),
                    "equal": bool(torch.equal(p, ref[:k]))})
        print(f"# {k} products alone: {ms:.4f} ms (split)", file=sys.stderr, flush=True)
    return out


def ragged_leg(torch, bi, inputs, args):
    """The ragged configuration: 4096 products, operand bits log-uniform in
    [2^15, 2^19] (seed 1003), one call = the plan's segment launches replayed
    from its hipGraph.  Roofline on the digit products the tuned digit widths
    execute."""
    c = inputs.ragged_mul_2e15_2e19()
    lens = c["lens"]
    ta = torch.from_numpy(c["a"].view(np.int32)).cuda()
    tb = torch.from_numpy(c["b"].view(np.int32)).cuda()
    tao, tbo = torch.from_numpy(c["a_off"]).cuda(), torch.from_numpy(c["b_off"]).cuda()
    plan = bi.MulPlan(lens, lens)
    out, oo = plan(ta, tao, tb, tbo)
    steps = max(5, args.steps // 2)
    total, _ = time_launches(lambda: plan(ta, tao, tb, tbo, out=out, out_off=oo), steps, args.warmup, torch)
    ms = total / steps
    print(f"# ragged 4096: {ms:.4f} ms/call", file=sys.stderr, flush=True)
    macs = 0.0
    for n_ in np.unique(lens):
        dbits = bi.mfma_config(int(n_), int(n_))[2]
        N = (32 * int(n_) + 6) // 7 if dbits == 7 else 4 * int(n_)
        macs += float(N) * N * int((lens == n_).sum())
    info = plan.info()
    # each segment's launch alone (direct, same buffers): its time, its
    # executed int8 ops against the peak, and the plan's modelled busy
    # fraction of its resident work-groups
    segs = []
    for k, sg in enumerate(plan.segments()):
        t, _ = time_launches(lambda: plan.run_segment(k, ta, tao, tb, tbo, out, oo), steps, args.warmup,
                             torch)
        sms = t / steps
        segs.append({"instances": sg["instances"], "parts_per_instance": sg["parts"],
                     "digit_bits": sg["digit_bits"],
                     "strips_per_band": sg["strips_per_band"], "waves": sg["waves"],
                     "resident_work_groups": sg["slots"], "ms": round(sms, 4),
                     "frac": round(2.0 * sg["digit_products"] / (sms * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4),
                     "modelled_busy": round(sg["modelled_busy"], 3)})
    plan.close()
    return {"workload": "4096 products, operand bits log-uniform in [2^15, 2^19] (seed 1003)",
            "value": round(4096 / (ms * 1e-3), 1), "unit": "muls/s", "ms_per_call": round(ms, 4),
            "steps": steps, "launches_per_call": info["launches_per_call"],
            "graph_replays": info["graph_replays"],
            "roofline": mfma_roofline(2.0 * macs, ms, f"sum over pairs of 2 x (digits)^2 int8 ops at the "
                                                    f"tuned digit width, {2.0 * macs:.4g} per call"),
            "segments": segs}


def divmod_leg(torch, bi, inputs, args):
    """The division configuration: 512 divisions, dividend bits log-uniform in
    [2^16, 2^18], divisor half the limbs (seed 1004), one call = the plan's
    launches replayed from its hipGraph.  Roofline on the int8 MACs the
    division's MFMA products issue (counted per division by the diagnostic
    entry point, outside the timed region); Div/Mul against one product of
    every dividend with itself."""
    c = inputs.ragged_div_2e16_2e18()
    nu, nv = c["nu"], c["nv"]
    tu = torch.from_numpy(c["u"].view(np.int32)).cuda()
    tv = torch.from_numpy(c["v"].view(np.int32)).cuda()
    tuo, tvo = torch.from_numpy(c["u_off"]).cuda(), torch.from_numpy(c["v_off"]).cuda()
    plan = bi.DivPlan(nu, nv)
    steps = max(5, args.steps // 2)
    total, _ = time_launches(lambda: plan(tu, tuo, tv, tvo), steps, args.warmup, torch)
    ms = total / steps
    print(f"# divmod 512: {ms:.4f} ms/call", file=sys.stderr, flush=True)
    mplan = bi.MulPlan(nu, nu)
    out, oo = mplan(tu, tuo, tu, tuo)
    mtotal, _ = time_launches(lambda: mplan(tu, tuo, tu, tuo, out=out, out_off=oo), steps, args.warmup, torch)
    mms = mtotal / steps
    _, _, st, cnt = plan.counters(tu, tuo, tv, tvo)
    cnt = cnt.cpu().numpy()
    macs = float(cnt[:, 3].sum())

    def hist(col):
        vals, counts = np.unique(cnt[:, col], return_counts=True)
        return {str(int(v)): int(k) for v, k in zip(vals, counts)}

    info = plan.info()
    plan.close()
    mplan.close()
    return {"workload": "512 divisions, dividend bits log-uniform in [2^16, 2^18], divisor half the limbs "
                        "(seed 1004)",
            "value": round(512 / (ms * 1e-3), 1), "unit": "divs/s", "ms_per_call": round(ms, 4),
            "steps": steps, "launches_per_call": info["launches_per_call"],
            "graph_replays": info["graph_replays"],
            "all_status_ok": bool((st == 0).all().item()),
            "same_size_products_ms": round(mms, 4), "div_over_mul": round(ms / mms, 3),
            "roofline": mfma_roofline(2.0 * macs, ms, f"2 int8 ops per digit product the division's MFMA "
                                                    f"products compute, {2.0 * macs:.4g} per call"),
            "newton_steps_histogram": hist(0), "negative_branch_steps_histogram": hist(1),
            "quotient_corrections_histogram": hist(2),
            "critical_path": critical_path(cnt[:, 3], ms)}


def critical_path(div_macs, ms):
    """The call's time is the latency of its largest division, which runs on
    one work-group (one CU): that division's MFMA multiply-accumulates at one
    CU's share of the int8 peak, against the call time."""
    top = float(np.max(div_macs))
    cu_macs_per_s = INT8_PEAK_TOPS * 1e12 / 2 / 256
    us = top / cu_macs_per_s * 1e6
    return {"largest_division_macs": top, "at_one_cu_peak_us": round(us, 1),
            "frac_of_call": round(us / (ms * 1e3), 3),
            "what": "one division per work-group: the batch cannot finish before its largest division, "
                    "whose products run on one CU"}


def copy_mode(torch):
    """y = -x over 256 MiB of int32: 256 MiB read + 256 MiB written per launch,
    the reference for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    n = 64 * 1024 * 1024
    x = torch.arange(n, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                      "launches": 3}))


def peak_mode(torch, bi):
    """Achievable int8 MFMA rate with no memory traffic (v_mfma_i32_16x16x64_i8,
    8 independent accumulators per wave, 64 per loop round), for 4..32 waves
    per CU, with constant operands and with operands whose bits change every
    round (as random digits do), and the same with v_mfma_i32_32x32x32_i8
    (4 accumulators, 32 per round, the same work); then the rate of the plain kernel's
    v_mad_u64_u32 (8 independent chains per lane), in 10^12 operations/s."""
    import ctypes
    L = bi.lib()
    out = torch.empty(8192 * 256, dtype=torch.int32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    res = {}
    for toggle in (0, 1, 3):
        for per_cu in (1, 2, 4, 8):
            blocks, iters = ncu * per_cu, 1000
            L.bigint_diag_mfma_rate(ctypes.c_void_p(out.data_ptr()), blocks, 20, toggle, s)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rc = L.bigint_diag_mfma_rate(ctypes.c_void_p(out.data_ptr()), blocks, iters, toggle, s)
            e1.record()
            torch.cuda.synchronize()
            if rc:
                raise bi.BigIntError(rc, "bigint_diag_mfma_rate")
            ms = e0.elapsed_time(e1)
            macs = blocks * 4 * iters * 64 * 16384
            key = ("toggling" if toggle & 1 else "constant") + ("_32x32x32" if toggle & 2 else "") + \
                f"_{4 * per_cu}_waves_per_cu_TOPs"
            res[key] = round(2 * macs / ms / 1e9, 1)
    # the plain kernel's inner operation: 32x32-bit products added to 64 bits
    out64 = torch.empty(8192 * 256, dtype=torch.int64, device="cuda")
    for per_cu in (1, 2, 4, 8):
        blocks, iters = ncu * per_cu, 1000
        L.bigint_diag_mad_rate(ctypes.c_void_p(out64.data_ptr()), blocks, 20, s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rc = L.bigint_diag_mad_rate(ctypes.c_void_p(out64.data_ptr()), blocks, iters, s)
        e1.record()
        torch.cuda.synchronize()
        if rc:
            raise bi.BigIntError(rc, "bigint_diag_mad_rate")
        ms = e0.elapsed_time(e1)
        res[f"mad_u64_u32_{4 * per_cu}_waves_per_cu_Tops"] = round(blocks * 256 * iters * 64 / ms / 1e9, 2)
    print(json.dumps({"mode": "mfma-peak", "cus": ncu, **res}))


def ragged_mode(torch, bi, inputs, args):
    """4096 products, bit lengths log-uniform in [2^15, 2^19] (seed 1003), the
    plan's segment launches replayed from a hipGraph and launched directly,
    the plain kernel beside them, and every segment timed alone."""
    c = inputs.ragged_mul_2e15_2e19()
    lens = c["lens"]
    ta = torch.from_numpy(c["a"].view(np.int32)).cuda()
    tb = torch.from_numpy(c["b"].view(np.int32)).cuda()
    tao, tbo = torch.from_numpy(c["a_off"]).cuda(), torch.from_numpy(c["b_off"]).cuda()
    # algorithmic work: 7-bit digit products of every pair (2 int8 ops each)
    Nd = (32 * lens.astype(np.float64) + 6) // 7
    ops = 2.0 * float((Nd * Nd).sum())
    res = {"mode": "ragged", "workload": "4096 products, operand bits log-uniform in [2^15, 2^19]",
           "int8_ops_per_launch_7bit_digits": ops}
    # tuned tile configuration per octave of operand bits, with its share of the work
    bins = []
    for lo in (15, 16, 17, 18):
        sel = (32 * lens > 2**lo) & (32 * lens <= 2**(lo + 1)) if lo > 15 else (32 * lens <= 2**16)
        n_hi = int(lens[sel].max())
        P, waves, dbits = bi.mfma_config(n_hi, n_hi)
        bins.append({"bits": f"2^{lo}-2^{lo + 1}", "instances": int(sel.sum()),
                     "work_share": round(float((Nd[sel] ** 2).sum() / (Nd ** 2).sum()), 3),
                     "config_at_largest": {"strips_per_band": P, "waves": waves, "digit_bits": dbits}})
    res["bins"] = bins
    for flags, name in ((0, "mfma_graph"), (2, "mfma_direct"), (1, "plain")):
        plan = bi.MulPlan(lens, lens, flags)
        out, oo = plan(ta, tao, tb, tbo)
        steps = max(2, args.steps // (10 if flags == 1 else 2))
        total, per = time_launches(lambda: plan(ta, tao, tb, tbo, out=out, out_off=oo), steps,
                                   args.warmup, torch)
        ms = total / steps
        res[name] = {"ms": round(ms, 4), "muls_per_s": round(4096 / ms * 1e3, 1),
                     "TOPs_7bit_digit_equivalent": round(ops / ms / 1e9, 1)}
        if flags == 0:
            ref = out.clone()
        else:
            res[name]["equals_mfma_graph"] = bool(torch.equal(out, ref))
        plan.close()
    res["segments"] = ragged_leg(torch, bi, inputs, args)["segments"]
    print(json.dumps(res))


def divmod_mode(torch, bi, inputs, args):
    """512 divisions (dividend log-uniform in [2^16, 2^18] bits, divisor half
    as many limbs), and the same-size products for the Div/Mul ratio; then
    uniform batches of 2^13..2^18-bit dividends."""
    c = inputs.ragged_div_2e16_2e18()
    nu, nv = c["nu"], c["nv"]
    tu = torch.from_numpy(c["u"].view(np.int32)).cuda()
    tv = torch.from_numpy(c["v"].view(np.int32)).cuda()
    tuo, tvo = torch.from_numpy(c["u_off"]).cuda(), torch.from_numpy(c["v_off"]).cuda()
    plan = bi.DivPlan(nu, nv)
    steps = max(3, args.steps // 5)
    total, _ = time_launches(lambda: plan(tu, tuo, tv, tvo), steps, args.warmup, torch)
    ms = total / steps
    # one full product of each dividend with itself, the Div/Mul reference
    mplan = bi.MulPlan(nu, nu)
    out, oo = mplan(tu, tuo, tu, tuo)
    mtotal, _ = time_launches(lambda: mplan(tu, tuo, tu, tuo, out=out, out_off=oo), steps,
                              args.warmup, torch)
    mms = mtotal / steps
    # per-division counters of the procedure (outside the timed region)
    _, _, st, cnt = plan.counters(tu, tuo, tv, tvo)
    cnt = cnt.cpu().numpy()

    def hist(col):
        vals, counts = np.unique(cnt[:, col], return_counts=True)
        return {str(int(v)): int(c) for v, c in zip(vals, counts)}

    # uniform batches on the paper's dataset shapes (NumBits x NumInsts = 2^32),
    # dividend NumBits, divisor half of it; Div/Mul against the product mod B^n
    # of two dividend-sized operands
    g = torch.Generator(device="cuda")
    g.manual_seed(1007)
    rows = []
    for bits in (2**13, 2**14, 2**15, 2**16, 2**17, 2**18, 2**19):
        n, insts = bits // 32, 2**32 // bits
        u = _rand_dev(torch, g, insts, n)
        v = _rand_dev(torch, g, insts, n // 2)
        v[:, -1] |= 1
        t_div, _ = time_launches(lambda: bi.divmod(u, v), 3, 1, torch)
        t_mul, _ = time_launches(lambda: bi.mullo(u, u), 3, 1, torch)
        rows.append({"num_bits": bits, "num_insts": insts, "divmod_ms": round(t_div / 3, 3),
                     "mul_ms": round(t_mul / 3, 3), "div_over_mul": round(t_div / t_mul, 2)})
        del u, v
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "divmod", "workload": "512 divisions, dividend bits log-uniform in "
                      "[2^16, 2^18], divisor half the limbs", "ms": round(ms, 4),
                      "divs_per_s": round(512 / ms * 1e3, 1),
                      "same_size_products_ms": round(mms, 4), "div_over_mul": round(ms / mms, 3),
                      "all_status_ok": bool((st == 0).all().item()),
                      "newton_steps_histogram": hist(0),
                      "negative_branch_steps_histogram": hist(1),
                      "quotient_corrections_histogram": hist(2), "uniform_rows": rows}))
    plan.close()
    mplan.close()


def _rand_dev(torch, g, rows, n):
    """rows x n random u32 limbs generated on the device (too large for host copies)."""
    x = torch.randint(-2**31, 2**31, (rows, n), dtype=torch.int32, device="cuda", generator=g)
    return x


def addsub_mode(torch, bi, inputs, args):
    """1-Add, 1-Sub and 6-Add in GB/s on the paper's addition datasets
    (NumBits 2^12..2^18, NumBits x NumInsts = 2^32, Table tab-add; bytes = 3 NumInsts NumBits / 8,
    each input and the result once), and on the 2^17-bit configuration
    (1024 pairs, half carry-adversarial; 48 MiB, which fits the 256 MB
    Infinity Cache: hot = back-to-back launches, cold = each launch after
    512 MiB of other writes)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(1005)
    res = {"mode": "addsub", "unit": "GB/s", "rows": []}
    steps = max(3, args.steps // 5)
    for bits in (2**12, 2**13, 2**14, 2**15, 2**16, 2**17, 2**18):
        n, insts = bits // 32, 2**32 // bits
        a = _rand_dev(torch, g, insts, n)
        b = _rand_dev(torch, g, insts, n)
        out = torch.empty_like(a)
        byts = 3 * insts * bits / 8
        row = {"num_bits": bits, "num_insts": insts}
        for name, fn in (("add", lambda: bi.add(a, b, out=out)), ("sub", lambda: bi.sub(a, b, out=out)),
                         ("add6", lambda: bi.add6(a, b, out=out))):
            total, _ = time_launches(fn, steps, args.warmup, torch)
            row[name] = round(byts / (total / steps * 1e-3) / 1e9, 1)
        res["rows"].append(row)
        del a, b, out
        torch.cuda.empty_cache()
    c = inputs.pairs_2e17_mixed()
    a = torch.from_numpy(c["a"].view(np.int32)).cuda()
    b = torch.from_numpy(c["b"].view(np.int32)).cuda()
    out = torch.empty_like(a)
    byts = 3 * a.numel() * 4
    cfg = {"workload": "1024 pairs of 2^17-bit integers, half carry-adversarial"}
    for name, fn in (("add", lambda: bi.add(a, b, out=out)), ("sub", lambda: bi.sub(a, b, out=out)),
                     ("add6", lambda: bi.add6(a, b, out=out))):
        total, _ = time_launches(fn, steps * 5, args.warmup, torch)
        cfg[name] = round(byts / (total / (steps * 5) * 1e-3) / 1e9, 1)
    # cold: 512 MiB written before every launch (twice the 256 MB Infinity
    # Cache), each launch timed alone with events
    flush = torch.empty(2**27, dtype=torch.int32, device="cuda")
    for name, fn in (("add", lambda: bi.add(a, b, out=out)), ("sub", lambda: bi.sub(a, b, out=out))):
        fn()
        t = 0.0
        for i in range(steps * 5):
            flush.fill_(i)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t += e0.elapsed_time(e1)
        cfg[name + "_cold"] = round(byts / (t / (steps * 5) * 1e-3) / 1e9, 1)
    del flush
    res["pairs_2e17_mixed"] = cfg
    print(json.dumps(res))


def poly_mode(torch, bi, args):
    """Poly = (a a + b)(b b + b) + a b against one product, both mod B^n (the
    paper's fixed precision, Table tab-mul), on its datasets NumBits 2^12..2^19,
    NumBits x NumInsts = 2^32."""
    g = torch.Generator(device="cuda")
    g.manual_seed(1006)
    res = {"mode": "poly", "unit": "ms", "rows": []}
    for bits in (2**12, 2**13, 2**14, 2**15, 2**16, 2**17, 2**18, 2**19):
        n, insts = bits // 32, 2**32 // bits
        a = _rand_dev(torch, g, insts, n)
        b = _rand_dev(torch, g, insts, n)
        steps = 3
        t_mul, _ = time_launches(lambda: bi.mullo(a, b), steps, 1, torch)
        t_poly, _ = time_launches(lambda: bi.poly(a, b), steps, 1, torch)
        res["rows"].append({"num_bits": bits, "num_insts": insts,
                            "mul_ms": round(t_mul / steps, 3), "poly_ms": round(t_poly / steps, 3),
                            "poly_over_mul": round(t_poly / t_mul, 3)})
        del a, b
        torch.cuda.empty_cache()
    print(json.dumps(res))


def configs_mode(torch, bi, inputs, args):
    """The two smaller uniform configurations, every operation on them:
    64 pairs of 2^15-bit and 1024 pairs of 2^17-bit integers (half of the
    latter carry-adversarial).  add / sub (sub on the ordered pairs, a >= b)
    in GB/s against HBM; full products with the MFMA-split and the plain
    kernel, compared with each other, against their rooflines."""
    import ctypes
    L = bi.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {"mode": "configs", "rows": []}
    for name, c in (("64 pairs of 2^15-bit integers, uniform", inputs.pairs_2e15()),
                    ("1024 pairs of 2^17-bit integers, half carry-adversarial", inputs.pairs_2e17_mixed())):
        n = c["n"]
        dev = {k: torch.from_numpy(c[k].view(np.int32)).cuda() for k in ("a", "b", "sub_a", "sub_b")}
        batch = dev["a"].shape[0]
        s_out = torch.empty_like(dev["a"])
        carry = torch.empty(batch, dtype=torch.int32, device="cuda")
        out_m = torch.empty((batch, 2 * n), dtype=torch.int32, device="cuda")
        out_p = torch.empty_like(out_m)
        P = {k: ctypes.c_void_p(v.data_ptr()) for k, v in dev.items()}
        po, pc = ctypes.c_void_p(s_out.data_ptr()), ctypes.c_void_p(carry.data_ptr())

        def call(rc, what):
            if rc:
                raise bi.BigIntError(rc, what)

        runs = {
            "add": lambda: call(L.bigint_add(po, pc, P["a"], P["b"], n, batch, stream), "bigint_add"),
            "sub": lambda: call(L.bigint_sub(po, pc, P["sub_a"], P["sub_b"], n, batch, stream), "bigint_sub"),
            "mul_mfma": lambda: call(L.bigint_mul(ctypes.c_void_p(out_m.data_ptr()), P["a"], n, P["b"], n,
                                                  batch, bi.MUL_MFMA, stream), "bigint_mul"),
            "mul_plain": lambda: call(L.bigint_mul(ctypes.c_void_p(out_p.data_ptr()), P["a"], n, P["b"], n,
                                                   batch, bi.MUL_PLAIN, stream), "bigint_mul"),
        }
        row = {"workload": name, "batch": batch, "limbs": n}
        for k, fn in runs.items():
            steps = max(5, args.steps // 2) if k != "mul_plain" else 5
            _, per = time_launches(fn, steps, max(2, args.warmup // 4), torch)
            row[k + "_ms"] = round(per, 4)
        byts = 3 * batch * n * 4 + 4 * batch
        row["add_GBps"] = round(byts / (row["add_ms"] * 1e-3) / 1e9, 1)
        row["sub_GBps"] = round(byts / (row["sub_ms"] * 1e-3) / 1e9, 1)
        row["add_frac_hbm"] = round(row["add_GBps"] / HBM_PEAK_GBS, 3)
        Na = (32 * n + 6) // 7
        mf = 2.0 * batch * Na * Na / (row["mul_mfma_ms"] * 1e-3) / 1e12
        row["mul_mfma_TOPs_7bit"] = round(mf, 1)
        row["mul_mfma_frac"] = round(mf / INT8_PEAK_TOPS, 3)
        pl = batch * n * n / (row["mul_plain_ms"] * 1e-3) / 1e12
        row["mul_plain_mads_e12"] = round(pl, 2)
        row["mul_plain_frac_alu"] = round(pl / MAD_PEAK_TOPS, 3)
        row["mfma_products_per_s"] = round(batch / (row["mul_mfma_ms"] * 1e-3), 1)
        row["plain_products_per_s"] = round(batch / (row["mul_plain_ms"] * 1e-3), 1)
        row["mfma_equals_plain"] = bool(torch.equal(out_m, out_p))
        res["rows"].append(row)
        del dev, s_out, carry, out_m, out_p
        torch.cuda.empty_cache()
    print(json.dumps(res))


def cpu_oracle_mode(inputs, args):
    """The CPU baseline leg for every operation of every configuration: the
    oracle as it stands (plain C behind its Python binding, no GPU), on all
    host cores (every thread takes every cores-th instance) and on one core, each over a bounded sample of the configuration's
    instances (about --cpu-seconds / 10 of work per line)."""
    import concurrent.futures as cf
    import oracle
    oracle.build()
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 64))
    budget = max(0.5, args.cpu_seconds / 10)

    def rows(flat, off):
        return [flat[off[i]:off[i + 1]] for i in range(len(off) - 1)]

    c1, c2, c3 = inputs.pairs_2e15(), inputs.pairs_2e17_mixed(), inputs.pairs_2e19()
    c4, c5 = inputs.ragged_mul_2e15_2e19(), inputs.ragged_div_2e16_2e18()
    work = []
    for name, c in (("64 x 2^15 bits", c1), ("1024 x 2^17 bits", c2), ("256 x 2^19 bits", c3)):
        a, b, sa, sb = c["a"], c["b"], c.get("sub_a", c["a"]), c.get("sub_b", c["b"])
        work.append((name, "add", "adds/s", [lambda i, a=a, b=b: oracle.add1(a[i], b[i])], len(a)))
        work.append((name, "sub", "subs/s", [lambda i, a=sa, b=sb: oracle.sub1(a[i], b[i])], len(a)))
        work.append((name, "mul", "muls/s", [lambda i, a=a, b=b: oracle.mul1(a[i], b[i])], len(a)))
    ra, rb = rows(c4["a"], c4["a_off"]), rows(c4["b"], c4["b_off"])
    work.append(("4096 ragged, 2^15..2^19 bits", "mul", "muls/s",
                 [lambda i: oracle.mul1(ra[i], rb[i])], len(ra)))
    ru, rv = rows(c5["u"], c5["u_off"]), rows(c5["v"], c5["v_off"])
    work.append(("512 ragged divisions, 2^16..2^18 bits", "divmod", "divs/s",
                 [lambda i: oracle.divmod1(ru[i], rv[i])], len(ru)))
    out = []
    for name, op, unit, (fn,), batch in work:
        # one core: instances in order until the budget is spent
        t0 = time.perf_counter()
        k = 0
        while k < batch and (k == 0 or time.perf_counter() - t0 < budget):
            fn(k)
            k += 1
        one = (time.perf_counter() - t0) / k
        # all cores: a sample sized to about the same wall time
        m = int(min(batch, max(cores, cores * budget / max(one, 1e-7))))
        with cf.ThreadPoolExecutor(max_workers=cores) as ex:
            list(ex.map(lambda _: None, range(cores)))     # threads started before the clock
            t0 = time.perf_counter()
            futs = [ex.submit(lambda lo: [fn(i) for i in range(lo, m, cores)], w) for w in range(cores)]
            for f in futs:
                f.result()
            wall = time.perf_counter() - t0
        out.append({"workload": name, "op": op, "unit": unit, "cores": cores,
                    "value": round(m / wall, 2), "one_core": round(1.0 / one, 2),
                    "sample": f"{m} of {batch} (all cores), {k} (one core)"})
        print(json.dumps(out[-1]), flush=True)
    return out


def stored_traffic(path, sha):
    """HBM bytes per launch from counters stored at `path`, or None when there
    are none or they were taken on other kernel sources than those hashing to
    `sha`."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    return t.get("bytes_per_launch") if t.get("kernel_sha") == sha else None


def kernel_sha():
    """Hash of the sources of the uniform MFMA multiply kernel k_mul_mfma (its
    device headers, and its definition and launchers in kernels.hip up to the
    split-product code that follows them), to know whether counters taken
    earlier still describe the current kernel."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2607_28897_amd", "csrc")
    for f in ("common.hpp", "dev_addsub.hpp", "dev_mul_mfma.hpp"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(d, "kernels.hip"), "r") as fh:
        src = fh.read()
    i = src.index("__global__ __launch_bounds__(512) void k_mul_mfma(")
    j = src.index("// ---- fewer products than CUs", i)
    h.update(src[i:j].encode())
    return h.hexdigest()[:16]


def source_sha():
    """Hash of every library source and of the C-ABI header: names the build a
    bench line was measured on (the GPU-side copy of the tree has no git)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2607_28897_amd", "csrc")
    for f in sorted(os.listdir(d)) + [os.path.join("..", "..", "include", "bigint_rocm.h")]:
        path = os.path.join(d, f)
        if os.path.isfile(path):
            h.update(f.encode())
            with open(path, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
