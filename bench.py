#!/usr/bin/env python3
"""Benchmark of the principal-minor library on one MI355X.

Headline workload: all 65,536 principal minors of each of 8192 synthetic propagator
matrices of order n = 16 (2D square-lattice G0 with L=32, t=1, mu=-0.5, beta=5; vertices
uniform on sites and imaginary time; one matrix in 64 made near-singular), fp64 path.
One step = one apm_all_minors launch over the whole batch, inputs resident in HBM.

Printed on stdout: ONE JSON line (metric, value = matrices/s, roofline of the minors
kernel, the CPU oracle baseline, the fp32-scaled variant and the other workloads in
"extra").  Everything else goes to stderr.

Second part of the metric ("mc"): Monte Carlo over vertex configurations weighted by
|c[V]| (8192 walkers, n = 10, 16 x 16 lattice, mu = 0, beta = 4), effective samples per
second of sign(c) and log|c| with the learned proposal (trained online for
--mc-train-steps steps, then frozen) against the uniform proposal (same number of
burn-in steps), over --mc-steps measured steps each.

Flags: --steps K --warmup W (timed / untimed steps), --gpus N (only N = 1 is supported),
--no-cpu (skip the oracle baseline leg), --no-extra (skip the secondary workloads),
--no-mc, --mc-train-steps, --mc-steps, --copy-calibration (run only a plain 1 GiB device
copy; used to calibrate the HBM traffic counters).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "matrices/s all-principal-minors at n=16 (FP64 vs FP32-scaled); MC ESS/s"
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ["paper_2104_07638_amd/csrc/fpm_impl.h", "paper_2104_07638_amd/csrc/apm_device.h",
                  "paper_2104_07638_amd/csrc/fpm_r64.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fpm_r64_n16_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def ensure_built():
    if not os.path.exists(os.path.join(ROOT, "paper_2104_07638_amd", "libapm.so")):
        import __graft_entry__
        __graft_entry__.build()


class Timer:
    """HIP events on the current stream (the stream the library launches on)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = []

    def __enter__(self):
        t = self.torch
        self.e0 = t.cuda.Event(enable_timing=True)
        self.e1 = t.cuda.Event(enable_timing=True)
        self.e0.record()
        return self

    def __exit__(self, *exc):
        self.e1.record()
        self.pairs.append((self.e0, self.e1))

    def times_ms(self):
        self.torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in self.pairs]

    def avg_ms(self):
        v = self.times_ms()
        return sum(v) / len(v)


def settle(torch, fn, seconds=0.2):
    """Run fn back to back for a fixed wall time before any timing: the GPU raises its clocks
    over the first tens of milliseconds of load, and a launch measured before that runs up
    to 20% slower than in steady state."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


def time_fn(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    t = Timer(torch)
    for _ in range(reps):
        with t:
            fn()
    return t.avg_ms()


def copy_calibration():
    import torch
    n = (1 << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    log(f"copied 3 x {n * 8} bytes")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-mc", action="store_true")
    ap.add_argument("--mc-train-steps", type=int, default=60000)
    ap.add_argument("--mc-steps", type=int, default=5000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (matrices are independent; the batch would be "
              "sharded with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    ensure_built()
    import numpy as np
    import torch

    import paper_2104_07638_amd as apm
    import workloads as W

    torch.cuda.set_device(0)
    n, B = 16, 8192
    lat = W.Lattice(32, 1.0, -0.5, 5.0)
    log("generating inputs ...")
    A = W.lattice_batch(B, n, lat, seed=W.BASE_SEED)
    A, stress_log = W.inject_stress(A, every=64)
    dA = torch.from_numpy(A).cuda()
    out = torch.empty((B, 1 << n), dtype=torch.float64, device="cuda")
    info = torch.empty(B, dtype=torch.int32, device="cuda")

    def step():
        apm.all_minors(dA, "r64", out=out, info=info)

    settle(torch, step)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kt = Timer(torch)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        with kt:
            step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms = kt.avg_ms()
    per_launch = sorted(kt.times_ms())
    value = B * args.steps / elapsed
    ms_per_step = elapsed * 1e3 / args.steps
    infos = info.cpu().numpy()
    log(f"r64 n={n} B={B}: {ms_per_step:.3f} ms/step, kernel {kern_ms:.3f} ms, {value / 1e6:.2f} M matrices/s; "
        f"shifted pivots: {int((infos > 0).sum())} matrices (max {int(infos.max())}, total {int(infos[infos > 0].sum())}), errors: {int((infos < 0).sum())}")

    bytes_per_matrix = 8 * n * n + 8 * (1 << n) + 4
    achieved = bytes_per_matrix * B / (kern_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_hash") == kernel_hash():
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                "kernel": f"fpm_uniform_kernel<FR64,{n},5>", "bytes_per_launch": bytes_per_matrix * B,
                "kernel_ms": round(kern_ms, 4), "kernel_ms_median": round(per_launch[len(per_launch) // 2], 4),
                "kernel_ms_min": round(per_launch[0], 4)}

    peaks = measured_peaks(torch, apm)
    # the faster of the two device copies (read + write bytes per second) as the measured ceiling
    mp = max(peaks["copy_GBs"], peaks["torch_copy_GBs"])
    roofline["measured_peak"] = mp
    roofline["measured_peak_kind"] = "device copy, read + write bytes (faster of the library probe and torch copy_)"
    roofline["frac_measured_peak"] = round(achieved / mp, 4)

    # ---- fp32-scaled variant on the same batch (mantissa + int16 exponent output)
    out32 = torch.empty((B, 1 << n), dtype=torch.float32, device="cuda")
    ex32 = torch.empty((B, 1 << n), dtype=torch.int16, device="cuda")
    ms32 = time_fn(torch, lambda: apm.all_minors(dA, "r32s", out=out32, exp=ex32, info=info), args.steps)
    fp32s = {"value": round(B / (ms32 * 1e-3), 1), "unit": "matrices/s", "ms_per_step": round(ms32, 4),
             "ratio_vs_fp64": round(kern_ms / ms32, 3),
             "achieved_GBs": round((8 * n * n + 6 * (1 << n) + 4) * B / (ms32 * 1e-3) / 1e9, 1)}
    log(f"r32s: {ms32:.3f} ms, {fp32s['value'] / 1e6:.2f} M matrices/s")

    # CDet connected sums of the same batch (a = det^2, rooted at vertex 0)
    cs_out = torch.empty_like(out)
    ms_cs = time_fn(torch, lambda: apm.connected_sums(out, out=cs_out), max(2, args.steps // 10))
    csum = {"ms": round(ms_cs, 3), "matrices_per_s": round(B / (ms_cs * 1e-3), 1),
            "TFLOPs": round(2 * B * 3 ** (n - 1) / (ms_cs * 1e-3) / 1e12, 2),
            "frac_fp64_peak": round(2 * B * 3 ** (n - 1) / (ms_cs * 1e-3) / 78.6e12, 4),
            "frac_measured_fp64_peak": round(2 * B * 3 ** (n - 1) / (ms_cs * 1e-3) / 1e12 / peaks["fma64_TFLOPs"], 4)}
    log(f"connected sums n={n}: {csum}")
    del cs_out

    # ---- the same workload with the diagonal set to zero (every left-spine pivot vanishes)
    Az = W.zero_diagonal(W.lattice_batch(B, n, lat, seed=W.BASE_SEED))
    dAz = torch.from_numpy(Az).cuda()
    outz = torch.empty_like(out)
    infoz = torch.empty_like(info)
    msz = time_fn(torch, lambda: apm.all_minors(dAz, "r64", out=outz, info=infoz), args.steps)
    iz = infoz.cpu().numpy()
    zero_diag = {"workload": "the headline batch with zero diagonal (no injections)", "r64_ms": round(msz, 4),
                 "r64_matrices_per_s": round(B / (msz * 1e-3), 1), "shifts_total": int(iz[iz > 0].sum()),
                 "shifts_max": int(iz.max()), "errors": int((iz < 0).sum())}
    log(f"zero diagonal r64: {zero_diag}")
    del dAz

    extra = {"csum_n16_8192": csum, "zero_diagonal_n16_8192": zero_diag, "measured_peaks": peaks}
    if not args.no_extra:
        extra.update(run_extra(torch, apm, W, np, args.steps))

    mc = None
    if not args.no_mc:
        mc = run_mc(torch, apm, W, np, args.mc_train_steps, args.mc_steps)

    cpu = None
    accuracy = None
    if not args.no_cpu:
        cpu, accuracy = cpu_leg(np, A, stress_log, out, out32, ex32, apm, Az, outz)

    res = {"metric": METRIC, "value": round(value, 1), "unit": "matrices/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "all principal minors, 8192 2D-lattice propagator matrices of order 16 "
                                  "(L=32, t=1, mu=-0.5, beta=5), 1 in 64 near-singular",
                      "n": n, "batch": B, "output": "fp64, 2^16 minors per matrix"},
           "roofline": roofline, "cpu_baseline": cpu, "fp32s": fp32s, "accuracy": accuracy, "mc": mc,
           "extra": extra}
    print(json.dumps(res), flush=True)


def measured_peaks(torch, apm):
    """Measured ceilings beside the datasheet ones: a 2 GiB device copy by the library's copy
    probe (16-byte accesses, best of three grid sizes; read + write bytes per second; torch's
    copy beside it) and the library's fp64 FMA-loop probe (8 independent chains per thread,
    4096 workgroups of 256 threads)."""
    nb = (2 << 30) // 8
    x = torch.ones(nb, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    ms_t = time_fn(torch, lambda: y.copy_(x), 5)
    best = None
    for blocks in (2048, 4096, 8192):
        msb = time_fn(torch, lambda: apm.probe_copy(y, x, blocks), 5)
        best = msb if best is None else min(best, msb)
    copy_gbs = 2 * nb * 8 / (best * 1e-3) / 1e9
    torch_gbs = 2 * nb * 8 / (ms_t * 1e-3) / 1e9
    del x, y
    fmas = [0]

    def fma():
        fmas[0] = apm.probe_fma64(4096, 4096)[1]

    msf = time_fn(torch, fma, 5)
    tf = 2 * fmas[0] / (msf * 1e-3) / 1e12
    res = {"copy_GBs": round(copy_gbs, 1), "copy_frac_datasheet": round(copy_gbs / PEAK_HBM_GBS, 4),
           "torch_copy_GBs": round(torch_gbs, 1),
           "fma64_TFLOPs": round(tf, 2), "fma64_frac_datasheet": round(tf / 78.6, 4)}
    log(f"measured peaks: {res}")
    return res


def run_extra(torch, apm, W, np, steps):
    """Secondary workloads: each timed with HIP events on the current stream."""
    ex = {}
    # 1024 real 8 x 8 lattice matrices (L=16, mu=0, beta=4): launch-latency bound
    A1 = torch.from_numpy(W.lattice_batch(1024, 8, W.Lattice(16, 1.0, 0.0, 4.0))).cuda()
    o1 = torch.empty((1024, 256), dtype=torch.float64, device="cuda")
    ms = time_fn(torch, lambda: apm.all_minors(A1, "r64", out=o1), steps)
    ex["lattice_n8_1024_r64"] = {"us_per_launch": round(ms * 1e3, 2), "matrices_per_s": round(1024 / (ms * 1e-3), 1)}
    # 4096 complex n = 14 Keldysh matrices, complex128 and complex64-scaled
    K = torch.from_numpy(W.keldysh_batch(4096, 14)).cuda()
    oc = torch.empty((4096, 1 << 14), dtype=torch.complex128, device="cuda")
    ms = time_fn(torch, lambda: apm.all_minors(K, "c128", out=oc), steps)
    ex["keldysh_n14_4096_c128"] = {"ms": round(ms, 4), "matrices_per_s": round(4096 / (ms * 1e-3), 1),
                                   "GBs": round((16 * 196 + 16 * (1 << 14)) * 4096 / (ms * 1e-3) / 1e9, 1)}
    del oc
    oc = torch.empty((4096, 1 << 14), dtype=torch.complex64, device="cuda")
    ec = torch.empty((4096, 1 << 14), dtype=torch.int16, device="cuda")
    ms = time_fn(torch, lambda: apm.all_minors(K, "c64s", out=oc, exp=ec), steps)
    ex["keldysh_n14_4096_c64s"] = {"ms": round(ms, 4), "matrices_per_s": round(4096 / (ms * 1e-3), 1),
                                   "GBs": round((16 * 196 + 10 * (1 << 14)) * 4096 / (ms * 1e-3) / 1e9, 1)}
    del oc, ec
    # mixed orders: 8192 lattice matrices with n uniform in {10..16} (L=32, beta=5, mu=-0.5):
    # all minors in one persistent launch, then the rooted CDet connected sums (a = det^2)
    mats, ns = W.lattice_ragged(8192, 10, 16, W.Lattice(32, 1.0, -0.5, 5.0), seed=W.BASE_SEED + 1)
    flat = torch.from_numpy(np.concatenate([m.ravel() for m in mats])).cuda()
    n_t = torch.from_numpy(ns).cuda()
    sizes = np.left_shift(1, ns.astype(np.int64))
    ooff = torch.from_numpy(np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)).cuda()
    tot = int(sizes.sum())
    mm = torch.empty(tot, dtype=torch.float64, device="cuda")
    cc = torch.empty_like(mm)
    ms_m = time_fn(torch, lambda: apm.all_minors_ragged(flat, n_t, 16, "r64", out=mm, out_off=ooff), steps)
    bd = apm.make_batch(8192, 0, n_t, 16, ooff, ooff)

    def csum():
        rc = apm.apm_connected_sums(apm._ptr(mm), None, bd, apm._ptr(cc), apm.APM_CS_ROOTED, apm._stream(None))
        assert rc == 0

    ms_c = time_fn(torch, csum, max(2, steps // 4))

    # the whole pipeline (queue preparation, persistent minors launch, connected sums) as
    # one CDet plan: recorded once into a HIP graph by the library, one launch per step
    # (matrices packed in `flat`, minors and sums at the offsets `ooff`)
    plan = apm.plan_cdet(flat, mm, cc, n=n_t, n_max=16, out_off=ooff)
    ms_g = time_fn(torch, plan.launch, max(2, steps // 4))
    plan.close()
    fma = float(np.sum(3.0 ** (ns.astype(np.float64) - 1)))
    ex["mixed_n10_16_8192_cdet"] = {
        "minors_ms": round(ms_m, 4), "minors_GBs": round((8 * float(np.sum(ns.astype(np.float64) ** 2)) + 8 * tot)
                                                          / (ms_m * 1e-3) / 1e9, 1),
        "csum_ms": round(ms_c, 4), "csum_fma": fma, "csum_TFLOPs": round(2 * fma / (ms_c * 1e-3) / 1e12, 2),
        "csum_frac_fp64_peak": round(2 * fma / (ms_c * 1e-3) / 78.6e12, 4),
        "plan_ms": round(ms_g, 4), "matrices_per_s": round(8192 / (ms_g * 1e-3), 1)}
    del mm, cc, flat
    # permanent principal minors: 2048 real n = 12, entries N(0,1)/sqrt(12)
    P = torch.from_numpy(W.gauss_batch(2048, 12)).cuda()
    po = torch.empty((2048, 1 << 12), dtype=torch.float64, device="cuda")
    ms = time_fn(torch, lambda: apm.all_perm_minors(P, out=po), steps)
    ex["perm_n12_2048"] = {"ms": round(ms, 4), "matrices_per_s": round(2048 / (ms * 1e-3), 1),
                           "products_per_s": round(2048 * 3 ** 12 / (ms * 1e-3), 1)}
    # leading principal minors of the headline lattice batch (8192 x n = 16)
    LA = torch.from_numpy(W.lattice_batch(8192, 16, W.Lattice(32, 1.0, -0.5, 5.0), seed=W.BASE_SEED + 2)).cuda()
    lo = torch.empty((8192, 16), dtype=torch.float64, device="cuda")
    li = torch.empty(8192, dtype=torch.int32, device="cuda")
    ms = time_fn(torch, lambda: apm.leading_minors(LA, out=lo, info=li), steps)
    ex["leading_n16_8192_r64"] = {"ms": round(ms, 4), "matrices_per_s": round(8192 / (ms * 1e-3), 1),
                                  "GBs": round((LA.numel() + lo.numel()) * 8 / (ms * 1e-3) / 1e9, 1)}
    del LA, lo, li
    # XOR minors (Keldysh-index determinants): 4096 Keldysh block matrices of 14 blocks
    # (28 x 28 complex128), every branch assignment and the trailing-block side products
    K2 = torch.from_numpy(W.keldysh_block(4096, 14, seed=W.BASE_SEED + 4)).cuda()
    xo = torch.empty((4096, (2 << 14) - 2), dtype=torch.complex128, device="cuda")
    xi = torch.empty(4096, dtype=torch.int32, device="cuda")
    ms = time_fn(torch, lambda: apm.xor_minors(K2, out=xo, info=xi), steps)
    by = K2.numel() * 16 + xo.numel() * 16
    ex["xor_keldysh_n14_4096_c128"] = {"ms": round(ms, 4), "matrices_per_s": round(4096 / (ms * 1e-3), 1),
                                       "GBs": round(by / (ms * 1e-3) / 1e9, 1),
                                       "frac_hbm_peak": round(by / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    # fp64: seeded real block matrices, N(0, 1) entries plus 3 on the diagonal (the real parts
    # of the Keldysh matrices have a zero diagonal: their first pivot vanishes)
    rng = np.random.default_rng(W.BASE_SEED + 6)
    K2r = torch.from_numpy(rng.standard_normal((4096, 28, 28)) + 3.0 * np.eye(28)).cuda()
    xr = torch.empty((4096, (2 << 14) - 2), dtype=torch.float64, device="cuda")
    ms = time_fn(torch, lambda: apm.xor_minors(K2r, out=xr, info=xi), steps)
    if int((xi != 0).sum()) != 0:
        log(f"xor r64 leg: {int((xi != 0).sum())} matrices with info != 0")
    by = K2r.numel() * 8 + xr.numel() * 8
    ex["xor_n14_4096_r64"] = {"ms": round(ms, 4), "matrices_per_s": round(4096 / (ms * 1e-3), 1),
                              "GBs": round(by / (ms * 1e-3) / 1e9, 1)}
    # XNOR minors (whole-block subsets, Sec. III) of the same complex batch
    xn = torch.empty((4096, 1 << 14), dtype=torch.complex128, device="cuda")
    ms = time_fn(torch, lambda: apm.xnor_minors(K2, out=xn, info=xi), steps)
    by = K2.numel() * 16 + xn.numel() * 16
    ex["xnor_keldysh_n14_4096_c128"] = {"ms": round(ms, 4), "matrices_per_s": round(4096 / (ms * 1e-3), 1),
                                        "GBs": round(by / (ms * 1e-3) / 1e9, 1)}
    del K2, xo, K2r, xr, xn
    # NAND minors (at most one row per block, 3^n): 1024 Keldysh block matrices of 10 blocks
    K3 = torch.from_numpy(W.keldysh_block(1024, 10, seed=W.BASE_SEED + 5)).cuda()
    na = torch.empty((1024, 3 ** 10), dtype=torch.complex128, device="cuda")
    ni = torch.empty(1024, dtype=torch.int32, device="cuda")
    ms = time_fn(torch, lambda: apm.nand_minors(K3, out=na, info=ni), steps)
    by = K3.numel() * 16 + na.numel() * 16
    nic = ni.cpu()
    ex["nand_keldysh_n10_1024_c128"] = {"ms": round(ms, 4), "matrices_per_s": round(1024 / (ms * 1e-3), 1),
                                        "GBs": round(by / (ms * 1e-3) / 1e9, 1),
                                        "matrices_shifted": int((nic > 0).sum()),
                                        "shifts_total": int(nic[nic > 0].sum()), "errors": int((nic < 0).sum())}
    del K3, na, ni
    for k, v in ex.items():
        log(f"{k}: {v}")
    return ex


def tau_int(np, x, c=5.0):
    """Integrated autocorrelation time of the (steps, walkers) series x: the walker-averaged
    autocorrelation function summed with Sokal's automatic window (smallest M >= c tau)."""
    x = x - x.mean(axis=0, keepdims=True)
    N = x.shape[0]
    f = np.fft.rfft(x, n=2 * N, axis=0)
    acf = np.fft.irfft(f * np.conj(f), axis=0)[:N].mean(axis=1)
    if acf[0] <= 0:
        return float("nan")
    rho = acf / acf[0]
    tau = 1.0
    for M in range(1, N):
        tau += 2.0 * rho[M]
        if M >= c * tau:
            break
    return float(tau)


def run_mc(torch, apm, W, np, n_train, n_meas, walkers=8192, n_series=1024):
    """ESS/s of the learned proposal against the uniform one on the same target."""
    model = W.McModel(n=10, L=16, t=1.0, mu=0.0, beta=4.0, n_tau=128, n_bin=16, eps=0.1, resolve=1e-10)
    g0 = torch.from_numpy(W.mc_g0_table(model)).cuda()
    m = apm.mc_model(model.n, model.L, model.n_tau, model.n_bin, model.eps, g0, model.resolve)
    out = {"workload": f"{walkers} walkers, n={model.n}, L={model.L}, t=1, mu=0, beta=4, {model.n_tau} time points, "
                       f"weight |c[V]| (a = det^2, rooted recursion) resolved above 1e-10 of its rounding scale",
           "train_steps": n_train, "measured_steps": n_meas}
    for kind in ("uniform", "learned"):
        learned = kind == "learned"
        chain = apm.McChain(W.mc_cluster_states(walkers, model, seed=W.BASE_SEED))
        net = apm.Mlp(model.d_in, model.d_out, W.mlp_init(model.d_in, model.d_out)) if learned else None
        work = apm.mc_work(m, walkers, learned)
        apm.mc_evaluate(m, chain, work)
        rec = apm.McRecord(walkers)
        t0 = time.perf_counter()
        for i in range(n_train):
            apm.mc_step(m, chain, work, seed=2021, step=i, net=net,
                        train=dict(lr=1e-3, t=i + 1) if learned else None, record=rec)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        loss = rec.loss.item() if learned else None
        hs = torch.empty((n_meas, walkers), dtype=torch.int8, device="cuda")
        hl = torch.empty((n_meas, walkers), dtype=torch.float32, device="cuda")
        ha = torch.empty((n_meas, walkers), dtype=torch.uint8, device="cuda")
        recs = []
        for i in range(n_meas):
            r = rec._c(hl[i], hs[i])
            r.accepted = ha[i].data_ptr()
            recs.append(r)
        tm = Timer(torch)
        with tm:
            for i in range(n_meas):
                apm.mc_step(m, chain, work, seed=2021, step=n_train + i, net=net, record=recs[i])
        ms = tm.avg_ms()
        sg = hs[:, :n_series].cpu().numpy().astype(np.float64)
        lw = hl[:, :n_series].cpu().numpy().astype(np.float64)
        ts, tl = tau_int(np, sg), tau_int(np, lw)
        sec = ms * 1e-3
        out[kind] = {"ms_per_step": round(ms / n_meas, 4), "acceptance": round(float(ha.float().mean().item()), 4),
                     "mean_sign": round(float(hs.float().mean().item()), 5),
                     "mean_log_c": round(float(hl.mean().item()), 3),
                     "tau_int_sign": round(ts, 2), "tau_int_log_c": round(tl, 2),
                     "ess_per_s_sign": round(walkers * n_meas / ts / sec, 1),
                     "ess_per_s_log_c": round(walkers * n_meas / tl / sec, 1),
                     "burn_in_s": round(t_train, 2)}
        if learned:
            out[kind]["final_train_loss"] = round(loss, 3)
        log(f"mc {kind}: {out[kind]}")
        del hs, hl, ha, work
    # resolution cutoff: the share of proposals given weight 0 (|c[V]| below kappa times the
    # recursion's rounding scale, or c[V] = 0), counted over untimed steps of the uniform chain
    # at equilibrium, and the equilibrium mean of log|c| with kappa = 1e-10 against 1e-12
    out["cutoff"] = mc_cutoff_check(torch, apm, W, np, model, walkers, n_train, min(n_meas, 2000))
    u, l = out["uniform"], out["learned"]
    out["gain_ess_per_s_sign"] = round(l["ess_per_s_sign"] / u["ess_per_s_sign"], 3)
    out["gain_ess_per_s_log_c"] = round(l["ess_per_s_log_c"] / u["ess_per_s_log_c"], 3)
    out["note"] = ("equal-error comparison: the wall time to reach a given standard error of the mean scales as "
                   "1 / (ESS/s), so the gain is the ratio of the learned to the uniform ESS/s")
    return out


def mc_cutoff_check(torch, apm, W, np, model, walkers, n_burn, n_meas):
    """Uniform-proposal chains at resolution cutoffs kappa = 1e-10 (the benchmark's) and
    1e-12: the share of proposals with weight 0, and the mean of log|c| over the measured
    steps with its standard error (integrated autocorrelation time of the walker means)."""
    res = {}
    for kappa in (1e-10, 1e-12):
        mdl = W.McModel(n=model.n, L=model.L, t=model.t, mu=model.mu, beta=model.beta, n_tau=model.n_tau,
                        n_bin=model.n_bin, eps=model.eps, resolve=kappa)
        g0 = torch.from_numpy(W.mc_g0_table(mdl)).cuda()
        m = apm.mc_model(mdl.n, mdl.L, mdl.n_tau, mdl.n_bin, mdl.eps, g0, mdl.resolve)
        chain = apm.McChain(W.mc_cluster_states(walkers, mdl, seed=W.BASE_SEED))
        work = apm.mc_work(m, walkers, False)
        apm.mc_evaluate(m, chain, work)
        rec = apm.McRecord(walkers)
        for i in range(n_burn):
            apm.mc_step(m, chain, work, seed=2021, step=i, record=rec)
        zero = torch.zeros((), dtype=torch.int64, device="cuda")
        hl = torch.empty((n_meas, walkers), dtype=torch.float32, device="cuda")
        for i in range(n_meas):
            apm.mc_step(m, chain, work, seed=2021, step=n_burn + i, record=rec)
            zero += torch.isinf(rec.logc_prop).sum()
            hl[i] = rec.obs_logw
        torch.cuda.synchronize()
        x = hl.cpu().numpy().astype(np.float64)
        tau = tau_int(np, x)
        mean = float(x.mean())
        se = float(np.sqrt(x.var() * tau / x.size))
        res[f"kappa_{kappa:g}"] = {"zero_weight_share": round(int(zero.item()) / (walkers * n_meas), 5),
                                   "mean_log_c": round(mean, 4), "stderr_log_c": round(se, 4),
                                   "tau_int_log_c": round(tau, 1)}
        del work, hl
    a, b = res["kappa_1e-10"], res["kappa_1e-12"]
    res["mean_log_c_difference_in_stderr"] = round(abs(a["mean_log_c"] - b["mean_log_c"]) /
                                                   np.hypot(a["stderr_log_c"], b["stderr_log_c"]), 2)
    log(f"mc cutoff: {res}")
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(np, A, stress_log, out, out32, ex32, apm, Az, outz):
    """The CPU oracle (LU per subset, fp64, all host threads) timed on a bounded sample of
    the same batch; then the per-result error of the GPU paths against the oracle on all
    128 near-singular matrices, 64 sampled others and 32 zero-diagonal matrices."""
    import oracle
    from oracle import metrics
    oracle._load()
    stressed = [b for b, _, _ in stress_log]
    t0 = time.perf_counter()
    count = 0
    chunk = 64
    while time.perf_counter() - t0 < 10.0:
        idx = list(range(count % A.shape[0], min(count % A.shape[0] + chunk, A.shape[0])))
        oracle.minors(A[idx])
        count += len(idx)
    el = time.perf_counter() - t0
    cores = oracle.max_threads()
    cpu = {"value": round(count / el, 2), "unit": "matrices/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
           "sample": f"{count} matrices of the 8192-matrix order-16 batch, LU with partial pivoting per subset, "
                     f"fp64, OpenMP over matrices on {cores} threads, {el:.1f} s"}
    log(f"cpu oracle: {cpu}")

    rng = np.random.default_rng(2024)
    others = sorted(set(rng.choice(A.shape[0], 72, replace=False).tolist()) - set(stressed))[:64]
    acc = {"metric": "|x - ref| / max(|ref|, Hadamard bound of A[S]) over every minor, against LU per subset"}
    for name, group in (("stressed_128", stressed), ("sampled_64", others)):
        ref = oracle.minors(A[group])
        x64 = out[group].cpu().numpy()
        x32 = apm.decode_scaled(out32[group], ex32[group]).cpu().numpy()
        e64 = e32 = r32 = 0.0
        for k, b in enumerate(group):
            H = metrics.hadamard_bounds(A[b])
            e64 = max(e64, float(metrics.mixed_err(x64[k], ref[k], H).max()))
            e32 = max(e32, float(metrics.mixed_err(x32[k], ref[k], H).max()))
            nz = np.abs(ref[k]) > 1e-3 * H
            r32 = max(r32, float(np.max(np.abs(x32[k][nz] - ref[k][nz]) / np.abs(ref[k][nz]))))
        acc[name] = {"matrices": len(group), "r64_max_mixed_err": e64, "r32s_max_mixed_err": e32,
                     "r32s_max_rel_err_minors_above_1e-3_of_H": r32}
    zsel = sorted(rng.choice(Az.shape[0], 32, replace=False).tolist())
    ref = oracle.minors(Az[zsel])
    xz = outz[zsel].cpu().numpy()
    ez = max(float(metrics.mixed_err(xz[k], ref[k], metrics.hadamard_bounds(Az[b])).max())
             for k, b in enumerate(zsel))
    acc["zero_diagonal_32"] = {"matrices": 32, "r64_max_mixed_err": ez}
    acc["r64_max_mixed_err"] = max(acc["stressed_128"]["r64_max_mixed_err"], acc["sampled_64"]["r64_max_mixed_err"],
                                   ez)
    acc["r32s_max_mixed_err"] = max(acc["stressed_128"]["r32s_max_mixed_err"],
                                    acc["sampled_64"]["r32s_max_mixed_err"])
    log(f"accuracy: {acc}")
    return cpu, acc


if __name__ == "__main__":
    main()
