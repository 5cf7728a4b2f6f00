"""Benchmark: gate-amplitude updates/s of the plain gate path on the
plain-path-at-scale workload (QFT of a seeded random basis state followed by
a seeded random depth-20 circuit, on a 30-qubit complex128 state and on a
32-qubit complex64 state), with the dominant kernel's HBM roofline and the
FP64 CPU oracle timed beside it.

One step = for each of the two registers: set the basis state, run the QFT,
run the random circuit (tile-pass schedule), compute all probabilities with
their FP64 total, and <Z_0>.  Inputs are generated before the timed region;
states live in HBM throughout.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--sizes 30:c128,32:c64]
"""

from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# Vector-ALU peak for FP64 and for FP32 without packed-FP32 instructions (all
# HIP code here is built with them disabled): 256 CUs x 4 SIMDs x 16 lanes x
# 2 flop (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.txt")


def sources_digest() -> str:
    """SHA-1 over the HIP sources: counter figures taken on other sources are stale."""
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_1805_00988_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key: str):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
    (scaled by the copy-kernel factors) for kernel@register, if the counters
    were taken on the current sources; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    digest = sources_digest()
    with open(TRAFFIC_FILE) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 5 and not line.startswith("#") and parts[0] == kernel_key:
                if parts[4] != digest:
                    return None
                return float(parts[1]) + float(parts[2])
    return None


def roofline_of(key: str, cnt: int, ms: float, by: float, fl: float) -> dict:
    """Roofline of one kernel from its launches: the binding roof is the one
    of the kernel's arithmetic intensity (algorithmic flops per algorithmic
    byte) against the vector-ALU ridge; both views are reported."""
    sec = ms * 1e-3 / cnt
    gbs = (by / cnt) / sec / 1e9
    tfl = (fl / cnt) / sec / 1e12
    ridge = ALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    ai = fl / by if by > 0 else 0.0
    hbm = {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    alu = {"achieved": round(tfl, 2), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": round(tfl / ALU_PEAK_TFLOPS, 4)}
    bound = "alu" if ai > ridge else "hbm"
    tr = measured_traffic(key)
    out = {"bound": bound, **(alu if bound == "alu" else hbm), "traffic": tr,
           "kernel": key, "launches": cnt, "avg_launch_ms": round(ms / cnt, 4),
           "algorithmic_bytes_per_launch": by / cnt, "algorithmic_flops_per_launch": fl / cnt,
           "flop_per_byte": round(ai, 3), "ridge_flop_per_byte": round(ridge, 3),
           "hbm_view": hbm, "alu_view": alu}
    return out


def parse_sizes(spec: str):
    out = []
    for item in spec.split(","):
        n, dt = item.split(":")
        out.append((int(n), dt))
    return out


def updates(circ) -> int:
    return circ.updates()


def read_stats(lib, handle):
    from paper_1805_00988_amd import _lib
    cap = 16
    arr = (_lib.sv_kernel_stat * cap)()
    n = ctypes.c_int()
    _lib.check(lib.sv_timing_read(handle, arr, cap, ctypes.byref(n)))
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms), float(arr[i].bytes),
                                   float(arr[i].flops))
            for i in range(n.value)}


def cpu_baseline(n: int, circ, budget_s: float, budget_1t_s: float):
    """FP64 oracle on the host: the first gates of the random circuit of the
    n-qubit register, run until the time budget is spent, on all host
    threads (the reported value) and again on one thread."""
    import oracle as O

    def leg(budget):
        psi = O.basis_state(n, 0)
        done_updates = 0
        g_done = 0
        t0 = time.perf_counter()
        for g in circ.gates:
            O.run_gates(n, [g], psi)
            done_updates += (1 << n) >> len(g.controls)
            g_done += 1
            if time.perf_counter() - t0 >= budget:
                break
        return done_updates / (time.perf_counter() - t0), g_done, time.perf_counter() - t0

    threads = O.num_threads()
    v_all, g_all, dt_all = leg(budget_s)
    O.set_num_threads(1)
    try:
        v_one, g_one, dt_one = leg(budget_1t_s)
    finally:
        O.set_num_threads(0)
    return {"value": v_all, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {g_all} gates of the depth-20 random circuit on the {n}-qubit "
                      f"state in FP64 complex ({dt_all:.1f} s, {threads} threads)",
            "one_thread": {"value": v_one, "unit": "updates/s", "cores": 1,
                           "sample": f"first {g_one} gates of the same circuit ({dt_one:.1f} s)"}}


def target_bucket(lo: int) -> str:
    """Bucket of a launch's lowest stride qubit (the target of a one-qubit
    gate, the lowest qubit of a phase gate's subspace mask)."""
    for a, b in ((0, 0), (1, 6), (7, 12), (13, 19), (20, 25), (26, 63)):
        if a <= lo <= b:
            return f"q{a}" if a == b else f"q{a}-{b}"
    return "q?"


def per_gate_breakdown(regs, lib, sv, _lib):
    """Alg. 1 as the paper runs it, one launch per gate (sv_run in per-gate
    mode, one gate per call) over the headline circuits of every register,
    untimed: each launch's kernel time from the library's HIP events,
    grouped by kernel and by the gate's lowest stride qubit.  GB/s counts the
    launch's algorithmic bytes (2 s N / 2^controls; phase gates touch only
    their subspace)."""
    out = {}
    for r in regs:
        h = r["state"].handle
        _lib.check(lib.sv_set_basis(h, r["qft"].basis))
        _lib.check(lib.sv_timing(h, 1))
        agg = {}
        for key, c in (("ops_qft", r["qft"]), ("ops_rnd", r["rnd"])):
            ops = r[key]
            for i, g in enumerate(c.gates):
                _lib.check(lib.sv_run(h, sv._opptr(ops[i:i + 1]), 1, None, 0, sv.SV_RUN_PER_GATE))
                per = read_stats(lib, h)
                phase = g.name in ("Z", "S", "T", "U1")
                lo = min((*g.targets, *g.controls)) if phase else min(g.targets)
                for kname, (cnt, ms, by, _fl) in per.items():
                    a = agg.setdefault(kname, {}).setdefault(target_bucket(lo), [0, 0.0, 0.0])
                    a[0] += cnt
                    a[1] += ms
                    a[2] += by
        _lib.check(lib.sv_timing(h, 0))
        reg = {}
        for kname, buckets in agg.items():
            tot = [sum(v[i] for v in buckets.values()) for i in range(3)]
            reg[kname] = {"all": {"launches": tot[0], "avg_ms": round(tot[1] / tot[0], 4),
                                  "GBps": round(tot[2] / (tot[1] * 1e-3) / 1e9, 1)},
                          **{b: {"launches": v[0], "avg_ms": round(v[1] / v[0], 4),
                                 "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1)}
                             for b, v in sorted(buckets.items())}}
        out[f"{r['n']}q_{r['dtype']}"] = reg
    return out


PREC_NAMES = {0: "native", 1: "fp32", 2: "bf16x3"}


def bench_fused(args, regs, lib, sv, _lib, torch):
    """The same workload through the fused path, with the fused path's
    autotuner (sv_fused_tune) choosing, per register and circuit, between
    plain tile passes and fused passes of at most 4 or 5 qubits in each
    allowed arithmetic (complex64: FP32 and split-BF16 matrix cores;
    complex128: FP64).  Fidelity is taken against the plain path's final
    state of the same register."""
    plain_final = {}
    for r in regs:  # reference: plain final state of this step's input
        plain_final[r["n"]] = r["state"].amps.clone()
    nb = ctypes.c_int()
    norm = ctypes.c_double()
    kk, pp, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    choice = {}
    for r in regs:  # tune each circuit from the state it starts from
        h = r["state"].handle
        _lib.check(lib.sv_set_basis(h, r["qft"].basis))
        for key, c in (("ops_qft", r["qft"]), ("ops_rnd", r["rnd"])):
            _lib.check(lib.sv_fused_tune(h, sv._opptr(r[key]), len(c.gates), None, 0, args.fuse_k, 0b111, 1,
                                         ctypes.byref(kk), ctypes.byref(pp), ctypes.byref(ms)))
            choice[(r["n"], key)] = (kk.value, pp.value)
            _lib.check(lib.sv_run(h, sv._opptr(r[key]), len(c.gates), None, 0, sv.SV_RUN_TILED))

    def fstep():
        for r in regs:
            h = r["state"].handle
            _lib.check(lib.sv_set_basis(h, r["qft"].basis))
            blocks = 0
            for key, c in (("ops_qft", r["qft"]), ("ops_rnd", r["rnd"])):
                k, prec = choice[(r["n"], key)]
                if k == 0:
                    _lib.check(lib.sv_run(h, sv._opptr(r[key]), len(c.gates), None, 0, sv.SV_RUN_TILED))
                else:
                    _lib.check(lib.sv_run_fused(h, sv._opptr(r[key]), len(c.gates), None, 0, k, prec,
                                                ctypes.byref(nb)))
                    blocks += nb.value
            _lib.check(lib.sv_probabilities(h, ctypes.c_void_p(r["probs"].data_ptr()), ctypes.byref(norm)))
            r["fused_blocks"], r["fused_norm"] = blocks, norm.value

    fstep()
    for r in regs:
        _lib.check(lib.sv_timing(r["state"].handle, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        fstep()
        print(f"# fused step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"workload": "the same QFT + random circuit through the fused path, configuration per circuit "
                       "chosen by the autotuner (sv_fused_tune)",
           "k_max": args.fuse_k, "ms_per_step": dt / args.steps * 1e3, "registers": {}}
    total = 0
    for r in regs:
        per = read_stats(lib, r["state"].handle)
        _lib.check(lib.sv_timing(r["state"].handle, 0))
        a = r["state"].amps
        b = plain_final[r["n"]]
        ov, na, nb2 = 0j, 0.0, 0.0
        for c0 in range(0, a.numel(), 1 << 28):  # BLAS dot takes < 2^31 elements
            ac, bc = a[c0:c0 + (1 << 28)], b[c0:c0 + (1 << 28)]
            ov += complex(torch.vdot(bc, ac).item())
            na += float(torch.vdot(ac, ac).real.item())
            nb2 += float(torch.vdot(bc, bc).real.item())
        fid = abs(ov) ** 2 / (na * nb2)
        total += r["updates"]
        fk = per.get("fused_block", (0, 0.0, 0.0, 0.0))
        out["registers"][f"{r['n']}q_{r['dtype']}"] = {
            "choice": {name: ("plain" if choice[(r["n"], key)][0] == 0 else
                              f"k{choice[(r['n'], key)][0]}_{PREC_NAMES[choice[(r['n'], key)][1]]}")
                       for name, key in (("qft", "ops_qft"), ("random", "ops_rnd"))},
            "blocks_per_step": r["fused_blocks"], "norm": r["fused_norm"],
            "fidelity_vs_plain": fid,
            "fused_pass_launches": fk[0] // args.steps,
            "fused_pass_ms_per_step": round(fk[1] / args.steps, 3),
            "fused_pass_GBps": round(fk[2] / (fk[1] * 1e-3) / 1e9, 1) if fk[1] > 0 else None}
        del b
    out["value"] = total * args.steps / dt
    out["unit"] = "updates/s"
    return out


def compare_states(a, ref, torch):
    """Fidelity |<ref|a>|^2 / (|ref|^2 |a|^2) and max |a - ref| over chunks
    (a may be complex64; every chunk is promoted to complex128)."""
    ov, na, nr, mx = 0j, 0.0, 0.0, 0.0
    for c0 in range(0, a.numel(), 1 << 26):
        x = a[c0:c0 + (1 << 26)].to(torch.complex128)
        y = ref[c0:c0 + (1 << 26)]
        ov += complex(torch.vdot(y, x).item())
        na += float(torch.vdot(x, x).real.item())
        nr += float(torch.vdot(y, y).real.item())
        mx = max(mx, float((x - y).abs().max().item()))
        del x
    return abs(ov) ** 2 / (na * nr), mx


def bench_fusion(n, seed, steps, warmup, torch):
    """Fusion workload: n-qubit seeded random circuit of depth 40 (a random
    one-qubit gate per qubit and n/2 CZ on random pairs per layer), complex64,
    run plain (tile passes, one gate at a time) and fused (each tile pass's
    gates fused into blocks of at most k = 4 or 5 qubits on the matrix cores,
    FP32 or split-BF16).  Every variant's final state is compared with the
    complex128 plain path on the same circuit."""
    import circuits as C
    import paper_1805_00988_amd as sv
    from paper_1805_00988_amd import _lib

    lib = _lib.load()
    circ = C.config2(n=n, seed=seed, depth=40)
    ops = sv.ops_from_gates(circ.gates)
    ref = sv.State(n, "c128")
    _lib.check(lib.sv_set_basis(ref.handle, 0))
    _lib.check(lib.sv_run(ref.handle, sv._opptr(ops), len(circ), None, 0, sv.SV_RUN_TILED))
    torch.cuda.synchronize()
    st = sv.State(n, "c64")
    nb = ctypes.c_int()
    variants = [("plain", 0, 0), ("fused_k4_fp32", 4, sv.SV_PREC_FP32),
                ("fused_k4_bf16x3", 4, sv.SV_PREC_SPLIT_BF16), ("fused_k5_fp32", 5, sv.SV_PREC_FP32),
                ("fused_k5_bf16x3", 5, sv.SV_PREC_SPLIT_BF16)]
    res = {}
    for label, k, prec in variants:
        def step():
            _lib.check(lib.sv_set_basis(st.handle, 0))
            if k == 0:
                _lib.check(lib.sv_run(st.handle, sv._opptr(ops), len(circ), None, 0, sv.SV_RUN_TILED))
            else:
                _lib.check(lib.sv_run_fused(st.handle, sv._opptr(ops), len(circ), None, 0, k, prec,
                                            ctypes.byref(nb)))
        for _ in range(warmup):
            step()
        _lib.check(lib.sv_timing(st.handle, 1))
        dt = timed(step, steps, torch)
        per = read_stats(lib, st.handle)
        _lib.check(lib.sv_timing(st.handle, 0))
        fid, mx = compare_states(st.amps, ref.amps, torch)
        kern = "fused_block" if k else "tile_pass"
        kc, kms, kby, kfl = per.get(kern, (1, 0.0, 0.0, 0.0))
        res[label] = {"updates_per_s": circ.updates() * steps / dt, "ms_per_step": dt / steps * 1e3,
                      "blocks": nb.value if k else None, "pass_launches": kc // steps,
                      "pass_avg_ms": round(kms / kc, 3) if kc else None,
                      "pass_GBps": round(kby / (kms * 1e-3) / 1e9, 1) if kms > 0 else None,
                      "infidelity_vs_c128": 1.0 - fid, "max_abs_err_vs_c128": mx}
    _lib.check(lib.sv_set_basis(st.handle, 0))
    kk, pp, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _lib.check(lib.sv_fused_tune(st.handle, sv._opptr(ops), len(circ), None, 0, 5, 0b111, 1, ctypes.byref(kk),
                                 ctypes.byref(pp), ctypes.byref(ms)))
    tuned = {"choice": "plain" if kk.value == 0 else f"k{kk.value}_{PREC_NAMES[pp.value]}",
             "tuner_ms": round(ms.value, 3)}
    del st, ref
    fused = {k: v for k, v in res.items() if k != "plain"}
    best = max(fused, key=lambda k: fused[k]["updates_per_s"])
    return {"workload": f"{n}-qubit random circuit, depth 40 (1q layer + {n // 2} CZ), complex64, seed {seed}",
            "gates": len(circ), "updates_per_step": circ.updates(), "variants": res, "best_fused": best,
            "speedup_best_fused_vs_plain": res[best]["updates_per_s"] / res["plain"]["updates_per_s"],
            "autotuner": tuned}


def timed(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fn()
        print(f"# step {i + 1}/{steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def qft_sweep(args, torch, sv):
    """The paper's benchmarking procedure (Sec. 3): for every sample, the QFT
    for every qubit count 1..N in a seeded random order, each timed from
    register creation to the end of its work, through the register interface
    (cu1 and h queued, then one tiled run).  Reports the median time per
    qubit count and the sweep's gate-amplitude updates/s."""
    nmax = args.sweep_max
    rng = np.random.default_rng(args.seed)
    times = {n: [] for n in range(1, nmax + 1)}

    def one(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reg = sv.State(n, "c64")
        for j in range(n):
            for k in range(j):
                reg.cu1(j, k, math.pi / float(2 ** (j - k)))
            reg.h(j)
        reg.sync()
        dt = time.perf_counter() - t0
        reg.close()
        return dt

    for _ in range(max(1, args.warmup)):
        for n in rng.permutation(np.arange(1, nmax + 1)):
            one(int(n))
    for _ in range(args.steps):
        for n in rng.permutation(np.arange(1, nmax + 1)):
            times[int(n)].append(one(int(n)))
    med = {n: float(np.median(v)) for n, v in times.items()}
    updates = sum((1 << n) * (n + n * (n - 1) // 4) for n in range(1, nmax + 1))
    total = sum(med.values())
    return {"value": updates / total, "dtype": "f32",
            "config": {"workload": f"QFT on 1..{nmax} qubits in random order per sample (the paper's "
                                   "benchmarking procedure), complex64, register interface, "
                                   f"{args.steps} samples"},
            "ms_per_step": total * 1e3,
            "median_s_per_qubit_count": {str(n): med[n] for n in sorted(med)}}


def other_workload(args):
    """Fusion (30 qubits, depth 40, complex64, fused at k = 4 and 5), batch
    (4096 ladder-ansatz circuits of 10..20 qubits, one graph launch) or
    adjoint (24-qubit ansatz, 576 parameters, loss and full gradient)."""
    import torch

    import circuits as C
    import paper_1805_00988_amd as sv
    from paper_1805_00988_amd import _lib

    lib = _lib.load()
    torch.cuda.set_device(0)
    out = {"metric": "gate-amplitude updates/s", "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "data": "synthetic", "vs_baseline": None}
    if args.workload == "fusion":
        f = bench_fusion(30, args.seed, args.steps, args.warmup, torch)
        best = f["variants"][f["best_fused"]]
        out.update({"value": best["updates_per_s"], "dtype": "f32",
                    "config": {"workload": f["workload"], "variant": f["best_fused"]},
                    "ms_per_step": best["ms_per_step"], "fusion": f})
    elif args.workload == "batch":
        circs = [c.bound() for c in C.config3(seed=args.seed)]
        b = sv.Batch(circs, "c64", z_mask=1)
        for _ in range(max(1, args.warmup)):
            b.run()
        dt = timed(lambda: b.run(), args.steps, torch)
        ups = sum(c.updates() for c in circs)
        if args.no_tune:  # profile one configuration alone
            if args.batch_config:
                m, w, g, f = (int(x) for x in args.batch_config.split(","))
                b.config(m, w, g, f)
                b.run()
                dt = timed(lambda: b.run(), args.steps, torch)
            print(json.dumps({"batch_ms_per_step": dt / args.steps * 1e3,
                              "config": args.batch_config or "default"}), flush=True)
            return None
        tuned = b.tune(reps=2)
        dt2 = timed(lambda: b.run(), args.steps, torch)
        z_batch = b.results()
        # the same circuits through the plain path: one register per width,
        # sv_run (tile passes) and sv_expectation per circuit
        regs = {w: sv.State(w, "c64") for w in sorted({c.n for c in circs})}
        ops = [sv.ops_from_gates(c.gates) for c in circs]
        for o in ops:
            o["param_index"] = -1  # bound circuits carry their angles in theta
        zm = np.array([1], np.uint64)
        zc = np.array([1.0], np.float64)
        ez = ctypes.c_double()
        z_plain = np.zeros(len(circs))

        def plain_all():
            for i, c in enumerate(circs):
                h = regs[c.n].handle
                _lib.check(lib.sv_set_basis(h, 0))
                _lib.check(lib.sv_run(h, sv._opptr(ops[i]), len(c.gates), None, 0, sv.SV_RUN_TILED))
                _lib.check(lib.sv_expectation(h, 1, zm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                              zc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(ez)))
                z_plain[i] = ez.value
        plain_all()
        dtp = timed(plain_all, args.steps, torch)
        # tail: each width's first circuit alone in a batch of one (one
        # workgroup walks it), with the tuned tile size and sweep width
        tail = {}
        for w in sorted({c.n for c in circs}):
            one = sv.Batch([next(c for c in circs if c.n == w)], "c64", z_mask=1)
            _lib.check(lib.sv_batch_tune(one.handle, 1, None, None, None, None, None))
            one.run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                one.run()
            torch.cuda.synchronize()
            tail[str(w)] = round((time.perf_counter() - t0) / 3 * 1e3, 3)
            one.close()
        out.update({"value": ups * args.steps / dt2, "dtype": "f32",
                    "config": {"workload": "4096 ladder-ansatz circuits, widths 10..20, 8 layers, complex64, "
                                           "one graph launch, <Z_0> per circuit"},
                    "ms_per_step": dt2 / args.steps * 1e3,
                    "ms_per_step_default": dt / args.steps * 1e3, "ms_per_step_tuned": dt2 / args.steps * 1e3,
                    "tuned": tuned,
                    "plain": {"ms_per_step": dtp / args.steps * 1e3, "updates_per_s": ups * args.steps / dtp,
                              "how": "per circuit: sv_set_basis, sv_run (tile passes), sv_expectation",
                              "max_abs_diff_z0_vs_batch": float(np.max(np.abs(z_plain - z_batch)))},
                    "speedup_vs_plain": dtp / dt2,
                    "one_circuit_alone_ms_by_width": tail})
    elif args.workload == "qft_sweep":
        out.update(qft_sweep(args, torch, sv))
    else:
        from paper_1805_00988_amd.autograd import ExpectationCircuit
        circ, masks, coeffs = C.config4(seed=args.seed)
        ec = ExpectationCircuit(circ.n, circ.gates, masks, coeffs, "c128")
        for _ in range(max(1, args.warmup)):
            ec.loss_and_grad(circ.params)
        dt = timed(lambda: ec.loss_and_grad(circ.params), args.steps, torch)
        out.update({"value": circ.updates() * args.steps / dt, "dtype": "f64",
                    "config": {"workload": "24-qubit ansatz, 12 layers RY/RZ + CNOT ring, complex128, "
                                           "loss + 576-parameter adjoint gradient (forward included)"},
                    "ms_per_step": dt / args.steps * 1e3})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sizes", default="30:c128,32:c64")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="tiled", choices=["tiled", "per_gate"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-seconds-1t", type=float, default=8.0,
                    help="time budget of the one-thread oracle leg")
    ap.add_argument("--no-seeds", action="store_true", help="skip the seed 1 and 2 runs")
    ap.add_argument("--no-per-gate", action="store_true",
                    help="skip the one-launch-per-gate breakdown by kernel and target")
    ap.add_argument("--cpu-qubits", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fused", action="store_true")
    ap.add_argument("--fuse-k", type=int, default=5, help="widest fused block the autotuner may choose")
    ap.add_argument("--workload", default="plain-at-scale",
                    choices=["plain-at-scale", "fusion", "batch", "adjoint", "qft_sweep"],
                    help="plain-at-scale (default headline line); the others time the "
                         "fusion, batched, adjoint and QFT-sweep workloads on their own")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch workload: time the default launch configuration only (no tuner, no "
                         "per-circuit comparison)")
    ap.add_argument("--batch-config", default="",
                    help="with --no-tune: tile qubits, sweep width, grid, fusion width (e.g. 13,4,512,1)")
    ap.add_argument("--sweep-max", type=int, default=24,
                    help="largest qubit count of the QFT sweep workload")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding of the "
                          "state vector is a design note, not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload != "plain-at-scale":
        res = other_workload(args)
        if res is not None:
            print(json.dumps(res), flush=True)
        return

    import torch

    import circuits as C
    import paper_1805_00988_amd as sv
    from paper_1805_00988_amd import _lib

    lib = _lib.load()
    torch.cuda.set_device(0)
    mode = sv.SV_RUN_TILED if args.mode == "tiled" else sv.SV_RUN_PER_GATE

    regs = []
    for n, dt in parse_sizes(args.sizes):
        qft, rnd = C.config1(n, args.seed)
        st = sv.State(n, dt)
        probs = torch.empty(1 << n, dtype=torch.float32 if dt == "c64" else torch.float64,
                            device="cuda")
        regs.append({
            "n": n, "dtype": dt, "state": st, "probs": probs, "qft": qft, "rnd": rnd,
            "ops_qft": sv.ops_from_gates(qft.gates), "ops_rnd": sv.ops_from_gates(rnd.gates),
            "updates": updates(qft) + updates(rnd),
            "plain_bytes": 2 * (8 if dt == "c64" else 16) * (updates(qft) + updates(rnd)),
        })

    zmask = np.array([1], np.uint64)
    zcoef = np.array([1.0], np.float64)
    norm = ctypes.c_double()
    ez = ctypes.c_double()

    def step():
        for r in regs:
            h = r["state"].handle
            _lib.check(lib.sv_set_basis(h, r["qft"].basis))
            _lib.check(lib.sv_run(h, sv._opptr(r["ops_qft"]), len(r["qft"].gates), None, 0, mode))
            _lib.check(lib.sv_run(h, sv._opptr(r["ops_rnd"]), len(r["rnd"].gates), None, 0, mode))
            _lib.check(lib.sv_probabilities(h, ctypes.c_void_p(r["probs"].data_ptr()),
                                            ctypes.byref(norm)))
            _lib.check(lib.sv_expectation(h, 1, zmask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                          zcoef.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          ctypes.byref(ez)))
            r["norm"], r["z0"] = norm.value, ez.value

    for i in range(args.warmup):
        step()
        print(f"# warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    for r in regs:
        _lib.check(lib.sv_timing(r["state"].handle, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        print(f"# timed step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    stats = {}
    for r in regs:
        per = read_stats(lib, r["state"].handle)
        _lib.check(lib.sv_timing(r["state"].handle, 0))
        r["kernels"] = per
        for name, v in per.items():
            stats[f"{name}@{r['n']}q_{r['dtype']}"] = v

    elapsed = t1 - t0
    total_updates = sum(r["updates"] for r in regs) * args.steps
    total_plain_bytes = sum(r["plain_bytes"] for r in regs) * args.steps
    value = total_updates / elapsed

    dom_key = max(stats, key=lambda k: stats[k][1])
    roofline = roofline_of(dom_key, *stats[dom_key])

    breakdown = {}
    for r in regs:
        kern_ms = sum(v[1] for v in r["kernels"].values())
        breakdown[f"{r['n']}q_{r['dtype']}"] = {
            "gates": len(r["qft"].gates) + len(r["rnd"].gates),
            "updates_per_step": r["updates"],
            "kernel_ms_per_step": round(kern_ms / args.steps, 3),
            "kernels": {k: {"launches": v[0] // args.steps, "ms_per_step": round(v[1] / args.steps, 3),
                            "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None,
                            "TFLOPs": round(v[3] / (v[1] * 1e-3) / 1e12, 2) if v[1] > 0 else None}
                        for k, v in r["kernels"].items()},
            "norm": r["norm"], "z0": r["z0"],
        }

    # the same step at the other seeds of the workload (short runs)
    seeds = {str(args.seed): value}
    if not args.no_seeds:
        for sd in (1, 2):
            if sd == args.seed:
                continue
            alt = []
            for r in regs:
                q2, r2 = C.config1(r["n"], sd)
                alt.append((r, q2, r2, sv.ops_from_gates(q2.gates), sv.ops_from_gates(r2.gates)))

            def step_seed():
                for r, q2, r2, oq, orr in alt:
                    h = r["state"].handle
                    _lib.check(lib.sv_set_basis(h, q2.basis))
                    _lib.check(lib.sv_run(h, sv._opptr(oq), len(q2.gates), None, 0, mode))
                    _lib.check(lib.sv_run(h, sv._opptr(orr), len(r2.gates), None, 0, mode))
                    _lib.check(lib.sv_probabilities(h, ctypes.c_void_p(r["probs"].data_ptr()),
                                                    ctypes.byref(norm)))
                    _lib.check(lib.sv_expectation(h, 1, zmask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                                  zcoef.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                  ctypes.byref(ez)))
            step_seed()
            ns = max(1, min(3, args.steps))
            dts = timed(step_seed, ns, torch)
            ups = sum(updates(q2) + updates(r2) for _r, q2, r2, _a, _b in alt)
            seeds[str(sd)] = ups * ns / dts

    per_gate = None
    if not args.no_per_gate and mode == sv.SV_RUN_TILED:
        per_gate = per_gate_breakdown(regs, lib, sv, _lib)

    fused = None
    if not args.no_fused:
        same = bench_fused(args, regs, lib, sv, _lib, torch)
        for r in regs:  # free the registers before the fusion workload's states
            r["state"] = None
            r["probs"] = None
        torch.cuda.empty_cache()
        fused = {"fusion_workload": bench_fusion(30, args.seed, args.steps, 1, torch), "same_workload": same}

    cpu = None
    if not args.no_cpu:
        n_cpu = args.cpu_qubits
        rnd = C.random_circuit(n_cpu, 20, args.seed + 1000, "X", n_cpu // 2)
        cpu = cpu_baseline(n_cpu, rnd, args.cpu_seconds, args.cpu_seconds_1t)

    dts = sorted({r["dtype"] for r in regs})
    out = {
        "metric": "gate-amplitude updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "+".join({"c64": "f32", "c128": "f64"}[d] for d in dts),
        "data": "synthetic",
        "config": {"workload": "QFT on a seeded random basis state + seeded random depth-20 "
                               "circuit (one random 1q gate per qubit, n//2 CNOTs per layer)",
                   "registers": [f"{r['n']}q {r['dtype']}" for r in regs],
                   "mode": args.mode, "seed": args.seed},
        "hbm_roofline_frac_effective": round(total_plain_bytes / elapsed / (HBM_PEAK_GBS * 1e9), 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "seeds": seeds,
        "per_gate": per_gate,
        "fused": fused,
        "breakdown": breakdown,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
