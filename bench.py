"""Throughput benchmark of the partitioned LMMSE estimator on one MI355X.

Workload (default): the paper-sized uplink, M=128 antennas, K=12 users,
N=1200 used subcarriers of a 2048-point FFT, 12 code-spread pilot symbols per
slot, a batch of 64 slots (98,304 LS columns, 117,964,800 channel
coefficients per step), overlapping windows of 150 keeping the central 100,
the fixed design of eq. 16 with a uniform profile over the 144-sample cyclic
prefix (L = 144), channels drawn with an exponential profile (tau_rms = 4
samples, 72 taps), SNR 10 dB.
A step is one call of lmmse_estimate: LS despreading of the pilot symbols and
block filtering of every column (one fused launch), with the plan's FP64
filters.  Inputs are resident in HBM before timing.

Prints one JSON line (rank 0, N=1 only).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "fp32_mfma_TFs": 157.3, "bf16_mfma_TFs": 2516.6,
        "fp16_mfma_TFs": 2516.6, "fp64_TFs": 78.6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--wn", type=int, default=150)
    ap.add_argument("--b", type=int, default=100)
    ap.add_argument("--rsource", default="uniform", choices=["exp", "uniform", "sample"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the split-precision, sample-covariance and fwd+bwd lines")
    ap.add_argument("--fwdbwd-only", action="store_true",
                    help="only time the fwd+bwd training step (16 slots) and print its line")
    ap.add_argument("--large-only", action="store_true",
                    help="only run the large sample-covariance workload (M=256, K=24, N=3300)")
    ap.add_argument("--detect-only", action="store_true",
                    help="only run the MMSE detection line")
    ap.add_argument("--fit-only", action="store_true",
                    help="only run the 200-step design fit of the differentiation workload")
    ap.add_argument("--comb-only", action="store_true",
                    help="only run the comb-pilot 3W / 12W lines")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    return ap.parse_args()


# the files holding each filtering kernel's device code
KERNEL_SOURCES = {
    "fp32": ("apply_f32.hip", "chunk_io.h", "dft.h"),
    "split": ("apply_split.hip", "chunk_io.h", "dft.h", "split.h"),
}


def src_digest(family: str) -> str:
    """Hash of the sources of a filtering kernel (to match stored counters)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(ROOT, "paper_1802_05427_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str, family: str, coeffs: int):
    """HBM bytes per launch from committed rocprofv3 counters (FETCH_SIZE and
    WRITE_SIZE, each scaled by what the counter reads for a plain device copy
    of known size), if they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    e = rec.get(kernel)
    if not e or e.get("src_digest") != src_digest(family) or e.get("coeffs") != coeffs:
        return None
    return e.get("hbm_bytes_per_launch")


def time_calls(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    per = sorted(a.elapsed_time(b) for a, b in evs)
    return per[len(per) // 2]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def log(msg, quiet=False):
    if not quiet:
        print(msg, file=sys.stderr, flush=True)


def fwd_bwd(M, K, N, N_fft, B, Wn, taps, sigma2, pil, dev, stream, steps, warmup):
    """One fwd+bwd training step of the fixed design on 16 slots with tau ~ U[2, 24]:
    design, despread, filter, loss gradient, backward to h_ls / tau / sigma2 (the
    two parameter gradients left on the device, lmmse_backward_dev, as a training
    loop that keeps them on the GPU does; the host-returning call would wait for
    each step to finish).  The despreading runs on a second stream beside the
    FP64 design, which it does not need."""
    import torch

    from paper_1802_05427_amd import Plan
    from synth.torch_slots import draw_batch
    S2 = 16
    g = torch.Generator(device=dev)
    g.manual_seed(180205427)
    y3, H3, _ = draw_batch(g, S2, M, K, N, N_fft, taps, 2.0, 24.0, sigma2, pil)
    # MSE gradient 2 (o - H) / n = c o + (-c H): the scaled target is a
    # constant of the batch, so the gradient is one elementwise pass per step
    c = 2.0 / H3.numel()
    negcH = H3 * (-c)
    with Plan(M=M, K=K, N=N, N_fft=N_fft, B=B, Wn=Wn, rsource="exp", taps=taps, tau_rms=8.0,
              sigma2=1e-4, max_slots=S2) as pl:
        par = torch.empty(2, dtype=torch.float64, device=dev)
        side = torch.cuda.Stream(device=dev)   # default priority

        def step():
            # the despreading runs beside the FP64 design (neither reads what
            # the other writes); the filter waits for both
            cur = torch.cuda.current_stream()
            side.wait_stream(cur)
            with torch.cuda.stream(side):
                h = pl.despread(y3, pil)
            pl.set_design(8.0, 1e-4)
            cur.wait_stream(side)
            h.record_stream(cur)
            o = pl.apply(h)
            gr = torch.add(negcH, o, alpha=c)
            return pl.backward(h, gr, want_params=True, params_out=par)
        t_ms = time_calls(step, steps, warmup, stream)
    return {"per_s": round(1e3 / t_ms, 1), "ms": round(t_ms, 4), "slots": S2,
            "coeffs": S2 * M * K * N,
            "workload": "16 slots, overlapping 150/100, exponential design (tau, sigma2), "
                        "tau_rms ~ U[2, 24] per (slot, user), SNR 10 dB; parameter gradients "
                        "kept on the device, despreading beside the design on a second stream"}


def timed_estimate(y, pil, sigma2, dev, stream, B, Wn, rsource, precision="fp32", flops=None,
                   ceiling=None, steps=10, warmup=2):
    """lmmse_estimate on the headline batch with another block plan or source:
    median event time, coefficients/s and, for FP32 products, the achieved
    FP32 matrix-core rate at `flops` per coefficient."""
    import torch

    from paper_1802_05427_amd import Plan
    S, M, K, N = (int(v) for v in y.shape)
    coeffs = S * M * K * N
    with Plan(M=M, K=K, N=N, N_fft=2048, B=B, Wn=Wn, rsource=rsource, taps=72, tau_rms=4.0, L=144.0,
              sigma2=sigma2, max_slots=S, precision=precision) as pl:
        out = torch.empty_like(y)
        t_ms = time_calls(lambda: pl.estimate(y, pil, sigma2, out=out), steps, warmup, stream)
    r = {"B": B, "Wn": Wn, "rsource": rsource, "precision": precision, "ms": round(t_ms, 4),
         "value": round(coeffs / (t_ms * 1e-3), 1)}
    if flops:
        r["tflops"] = round(flops * coeffs / (t_ms * 1e-3) / 1e12, 2)
        r["mfma_fp32_frac"] = round(r["tflops"] / PEAK["fp32_mfma_TFs"], 4)
        r["flop_per_coef"] = flops
    if ceiling:
        r["ceiling_coeff_per_s"] = round(ceiling, 1)
    if precision != "fp32":
        r["hbm_frac"] = round(16.0 * coeffs / (t_ms * 1e-3) / 1e9 / PEAK["hbm_GBs"], 4)
    return r


def gap_per_snr(M, K, N, N_fft, B, Wn, taps, tau, rsource, dev):
    """NMSE gap and discrepancy against the FP64 oracle per SNR point (0, 10,
    20 dB) for FP32, BF16x3 and FP16x3, one seeded slot each."""
    import torch

    import oracle as O
    from paper_1802_05427_amd import Plan
    from synth import make_slot_batch
    okw = dict(N_fft=N_fft, tau=tau, taps=taps, L=144.0)
    res = {}
    for snr in (0.0, 10.0, 20.0):
        sb = make_slot_batch(M=M, K=K, N=N, N_fft=N_fft, taps=taps, tau=tau, snr_db=snr, slots=1,
                             config_id=2, first_slot=100 + int(snr))
        ref = O.estimate(sb.y, sb.pilots, sb.sigma2, B, Wn, rsource, **okw)
        y1 = torch.from_numpy(sb.y).to(dev)
        p1 = torch.from_numpy(sb.pilots).to(dev)
        for prec in ("fp32", "bf16x3", "fp16x3"):
            with Plan(M=M, K=K, N=N, N_fft=N_fft, B=B, Wn=Wn, rsource=rsource, taps=taps, tau_rms=tau,
                      L=144.0, sigma2=sb.sigma2, max_slots=1, precision=prec) as pl:
                o = pl.estimate(y1, p1, sb.sigma2).cpu().numpy()
            res.setdefault(prec, {})[f"{snr:g}dB"] = {
                "nmse_gap_db": abs(O.nmse_db(o, sb.H) - O.nmse_db(ref, sb.H)),
                "discrepancy_db": round(O.discrepancy_db(o, ref), 1),
                "nmse_db": round(O.nmse_db(ref, sb.H), 3)}
    return res


def fit_line(M, K, N, N_fft, B, Wn, taps, sigma2, pil, dev, steps=200):
    """The design fit of the differentiation workload: 200 Adam steps (lr 0.05)
    on (log tau_rms, log sigma2) from tau 8, sigma2 1e-4, each on a fresh
    16-slot batch with tau_rms ~ U[2, 24] per (slot, user) drawn on the GPU
    (generation, despreading, estimate, loss, backward, Adam update); the
    endpoint beside the stored FP64 optimum of the expected error."""
    import torch

    from paper_1802_05427_amd import Plan
    from paper_1802_05427_amd.fit import fit_design
    from synth.torch_slots import draw_batch
    S2 = 16
    with Plan(M=M, K=K, N=N, N_fft=N_fft, B=B, Wn=Wn, rsource="exp", taps=taps, tau_rms=8.0,
              sigma2=1e-4, max_slots=S2) as pl:
        def fn(step):
            g = torch.Generator(device=dev)
            g.manual_seed(180205427 + 7919 * step)
            y, H, _ = draw_batch(g, S2, M, K, N, N_fft, taps, 2.0, 24.0, sigma2, pil)
            return pl.despread(y, pil), H

        fit_design(pl, fn, steps=3, lr=0.05)   # warm-up (kernels, allocator)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = fit_design(pl, fn, steps=steps, lr=0.05, tau0=8.0, sigma2_0=1e-4)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    tail = st.history[-20:]
    tau_f = math.exp(sum(math.log(h[1]) for h in tail) / len(tail))
    sig_f = math.exp(sum(math.log(h[2]) for h in tail) / len(tail))
    res = {"workload": "design fit: 16 slots per step, overlapping 150/100, exponential design, "
                       "tau_rms ~ U[2, 24] per (slot, user), SNR 10 dB, Adam lr 0.05 from tau 8, "
                       "sigma2 1e-4", "steps": steps, "seconds": round(wall, 3),
           "steps_per_s": round(steps / wall, 1), "tau_final": round(tau_f, 4),
           "sigma2_final": round(sig_f, 5),
           "loss_last10": sum(h[0] for h in st.history[-10:]) / 10,
           "loss_first10": sum(h[0] for h in st.history[:10]) / 10}
    try:
        with open(os.path.join(ROOT, "tests", "golden", "fit_optimum_diff_workload.json")) as f:
            opt = json.load(f)
        res["fp64_optimum"] = {"tau": round(opt["tau"], 4), "sigma2": round(opt["sigma2"], 5),
                               "expected_mse": opt["mse"]}
    except OSError:
        pass
    return res


def large_sample(dev, stream, precision="fp16x3", slots=32, steps=3, warmup=1):
    """The large uplink with per-window sample covariance: M=256, K=24, N=3300
    of a 4096-point FFT, overlapping B=132 in windows of 198, 32 slots, tau_rms
    32 (144 taps), SNR 15 dB; FP64 design per (slot, user, window), split
    filter.  Forward (estimate from the pilot symbols) and one fwd+bwd step
    (estimate from the LS values keeping each window's FP64 design, MSE
    gradient, backward to h_ls and sigma2 from the kept design).
    Accuracy: one seeded slot against the FP64 oracle on users 0 and 1."""
    import numpy as np
    import torch

    import oracle as O
    from paper_1802_05427_amd import Plan
    from synth import make_pilots, make_slot_batch
    from synth.torch_slots import draw_batch
    M, K, N, Nf, B, Wn, taps, tau = 256, 24, 3300, 4096, 132, 198, 144, 32.0
    sigma2 = 10.0 ** -1.5
    pil = torch.from_numpy(make_pilots(K, N)).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(180205427 + 4)
    ys, Hs = [], []
    for s0 in range(0, slots, 4):
        y, H, _ = draw_batch(g, min(4, slots - s0), M, K, N, Nf, taps, tau, tau, sigma2, pil)
        ys.append(y)
        Hs.append(H)
    y = torch.cat(ys)
    H = torch.cat(Hs)
    del ys, Hs
    coeffs = slots * M * K * N
    nmat = slots * K * (N // B)
    res = {"workload": f"large uplink M={M} K={K} N={N} N_fft={Nf}, {slots} slots, overlapping "
                       f"B={B} Wn={Wn}, sample covariance per (slot, user, window), {precision} filter",
           "slots": slots, "coeffs": coeffs}
    with Plan(M=M, K=K, N=N, N_fft=Nf, B=B, Wn=Wn, rsource="sample", sigma2=sigma2, max_slots=slots,
              precision=precision) as pl:
        out = torch.empty_like(y)
        t_ms = time_calls(lambda: pl.estimate(y, pil, sigma2, out=out), steps, warmup, stream)
        res["forward_ms"] = round(t_ms, 3)
        res["value"] = round(coeffs / (t_ms * 1e-3), 1)
        # FP64 design work per window, Hermitian-aware counts: covariance
        # Wn(Wn+1)/2 M complex MACs, sweep Wn^3 / 2 complex MACs
        fl = 8.0 * (Wn * (Wn + 1) / 2 * M + Wn ** 3 / 2) * nmat
        res["design_fp64_TFs_at_forward_time"] = round(fl / (t_ms * 1e-3) / 1e12, 2)
        res["nmse_db"] = round(10 * float(np.log10(((out - H).abs().pow(2).sum()
                                                    / H.abs().pow(2).sum()).item())), 3)
        h = pl.despread(y, pil)
        scale = 2.0 / out.numel()
        negcH = H * (-scale)   # MSE gradient = scale o + (-scale H), one pass per step

        par = torch.empty(2, dtype=torch.float64, device=dev)
        # the forward keeps each window's FP64 design for the backward
        # (lmmse_estimate_ls_keep / lmmse_backward_kept), about 20 GB here
        kst = torch.empty(pl.design_state_bytes(slots), dtype=torch.uint8, device=dev)

        def step():
            o = pl.estimate_ls(h, sigma2, keep=kst)
            gr = torch.add(negcH, o, alpha=scale)
            return pl.backward(h, gr, want_params=True, params_out=par, kept=kst)
        t_fb = time_calls(step, max(1, steps - 1), warmup, stream)
        res["fwd_bwd_ms"] = round(t_fb, 3)
        res["fwd_bwd_per_s"] = round(1e3 / t_fb, 3)
        del out, h, negcH, kst
    del y, H
    torch.cuda.empty_cache()
    # accuracy on one seeded host slot (users 0 and 1 against the oracle)
    sb = make_slot_batch(M=M, K=K, N=N, N_fft=Nf, taps=taps, tau=tau, snr_db=15.0, slots=1, config_id=4)
    with Plan(M=M, K=K, N=N, N_fft=Nf, B=B, Wn=Wn, rsource="sample", sigma2=sb.sigma2, max_slots=1,
              precision=precision) as pl:
        o1 = pl.estimate(torch.from_numpy(sb.y).to(dev), torch.from_numpy(sb.pilots).to(dev),
                         sb.sigma2).cpu().numpy()
    X = O.despread(sb.y, sb.pilots)
    lam = sb.sigma2 / K
    starts, offs = O.window_starts(N, B, Wn)
    users = [0, 1]
    ref = np.zeros((1, M, len(users), N), complex)
    for ui, k in enumerate(users):
        for b, (st, off) in enumerate(zip(starts, offs)):
            Xw = X[0, :, k, st:st + Wn]
            R = O.sample_covariance(Xw)
            W = O.lmmse._filter(R[off:off + B], R, lam)
            ref[0, :, ui, b * B:(b + 1) * B] = Xw @ W.T
    got = o1[:, :, users]
    tru = sb.H[:, :, users]
    res["nmse_gap_db"] = abs(O.nmse_db(got, tru) - O.nmse_db(ref, tru))
    res["discrepancy_db"] = round(O.discrepancy_db(got, ref), 1)
    res["accuracy_sample"] = "slot 0, users 0-1 (50 windows) vs the FP64 oracle"
    return res


def comb_lines(dev, stream, steps=20, warmup=3):
    """The paper's comb-pilot estimators (Sec. IV-B): one pilot symbol with
    comb spacing 12, 4 active UEs, the paper-sized band (N=1200 of 2048),
    128 antennas, 64 slots, the 6-tap profile of the paper's simulation setup
    (delays 0..5, -2/-8/-10/-12/-15/-18 dB) at SNR 20 dB, design from eq. 16
    with L = 8.  HBM-bound: 8 B written per output coefficient plus the comb
    tones read (8/12 B per output)."""
    import numpy as np
    import torch

    import oracle as O
    from paper_1802_05427_amd import CombPlan
    from synth import make_comb_batch
    M, K, N, Nf, S, slots, uniq = 128, 4, 1200, 2048, 12, 64, 4
    cb = make_comb_batch(M=M, K=K, N=N, N_fft=Nf, powers_db=[-2, -8, -10, -12, -15, -18],
                         snr_db=20.0, slots=uniq, comb=S)
    y = torch.from_numpy(cb.y).to(dev).repeat(slots // uniq, 1, 1).contiguous()
    pil = torch.from_numpy(cb.pilots).to(dev)
    coeffs = slots * M * K * N
    res = {}
    rd = lambda d: O.r_uniform(d, 8.0, Nf)
    for kind in ("3w", "12w"):
        with CombPlan(M=M, K=K, N=N, N_fft=Nf, comb=S, kind=kind, rsource="uniform", L=8.0,
                      sigma2=cb.sigma2, max_slots=slots) as pl:
            out = torch.empty((slots, M, K, N), dtype=torch.complex64, device=dev)
            t_ms = time_calls(lambda: pl.estimate(y, pil, out=out), steps, warmup, stream)
            o1 = out[:1].cpu().numpy()
        ref = O.comb_estimate(cb.y[:1], cb.pilots, cb.sigma2, S, range(K), kind, rd)
        gbs = coeffs * (8.0 + 8.0 / S) / (t_ms * 1e-3) / 1e9
        res[kind] = {"value": round(coeffs / (t_ms * 1e-3), 1), "ms": round(t_ms, 4),
                     "hbm_GBs": round(gbs, 1), "hbm_frac": round(gbs / PEAK["hbm_GBs"], 4),
                     "nmse_db": round(O.nmse_db(o1, cb.H[:1]), 3),
                     "nmse_gap_db": abs(O.nmse_db(o1, cb.H[:1]) - O.nmse_db(ref, cb.H[:1])),
                     "discrepancy_db": round(O.discrepancy_db(o1, ref), 1)}
    for kind, ref_fn in (("ls_hold", lambda: O.comb_ls_hold(cb.y[:1], cb.pilots, S, range(K))),
                         ("ls_linear3", lambda: O.comb_ls_linear(cb.y[:1], cb.pilots, S, range(K), fold=3)),
                         ("ls_quadratic", lambda: O.comb_ls_quadratic(cb.y[:1], cb.pilots, S, range(K))),
                         ("ls_spline", lambda: O.comb_ls_spline(cb.y[:1], cb.pilots, S, range(K)))):
        with CombPlan(M=M, K=K, N=N, N_fft=Nf, comb=S, kind=kind, rsource="uniform", L=8.0,
                      sigma2=cb.sigma2, max_slots=slots) as pl:
            out = torch.empty((slots, M, K, N), dtype=torch.complex64, device=dev)
            t_ms = time_calls(lambda: pl.estimate(y, pil, out=out), steps, warmup, stream)
            o1 = out[:1].cpu().numpy()
        ref = ref_fn()
        res[kind] = {"ms": round(t_ms, 4), "nmse_db": round(O.nmse_db(o1, cb.H[:1]), 3),
                     "discrepancy_db": round(O.discrepancy_db(o1, ref), 1)}
    res["workload"] = (f"comb pilots (spacing {S}), M={M}, {K} active UEs, N={N} of {Nf}, {slots} slots, "
                       "6-tap profile, SNR 20 dB, eq. 16 design with L=8")
    return res


def detect_line(dev, stream, steps=20, warmup=3):
    """MMSE detection (eq. 22) downstream of the estimator on the paper-sized
    system: 64 slots, 128 antennas, 12 users, N=1200, 12 QPSK data symbols
    per slot, SNR 10 dB.  HBM-bound: H (M K), Y (M T) read and X (T K)
    written per subcarrier, 8 B each."""
    import numpy as np
    import torch

    import oracle as O
    from paper_1802_05427_amd import mmse_detect
    from synth import make_pilots
    from synth.torch_slots import draw_batch
    M, K, N, Nf, T, S = 128, 12, 1200, 2048, 12, 64
    sigma2 = 0.1
    pil = torch.from_numpy(make_pilots(K, N)).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(180205427 + 8)
    Hs = []
    for s0 in range(0, S, 16):
        Hs.append(draw_batch(g, 16, M, K, N, Nf, 72, 4.0, 4.0, 0.0, pil)[1])
    H = torch.cat(Hs).contiguous()
    del Hs
    bits = torch.randint(0, 2, (S, T, K, N, 2), generator=g, device=dev).float()
    X = torch.complex(1 - 2 * bits[..., 0], 1 - 2 * bits[..., 1]) / np.sqrt(2.0)
    Y = torch.zeros((S, M, T, N), dtype=torch.complex64, device=dev)
    for k in range(K):   # Y[s, m, t, n] = sum_k H[s, m, k, n] X[s, t, k, n]
        Y += H[:, :, k, None, :] * X[:, None, :, k, :]
    Y += torch.complex(torch.randn(Y.shape, generator=g, device=dev),
                       torch.randn(Y.shape, generator=g, device=dev)) * float(np.sqrt(sigma2 / 2))
    out = torch.empty((S, T, K, N), dtype=torch.complex64, device=dev)
    t_ms = time_calls(lambda: mmse_detect(H, Y, sigma2, out=out), steps, warmup, stream)
    ref = O.mmse_detect(H[:1].cpu().numpy().astype(np.complex128), Y[:1].cpu().numpy().astype(np.complex128),
                        sigma2)
    got = out[:1].cpu().numpy()
    byts = S * N * 8.0 * (M * K + M * T + T * K)
    gbs = byts / (t_ms * 1e-3) / 1e9
    ser = float(np.mean(np.abs(O.qpsk_decide(got) - X[:1].cpu().numpy()) > 1e-3))
    return {"workload": f"MMSE detection, {S} slots, M={M}, K={K}, N={N}, {T} data symbols, SNR 10 dB",
            "ms": round(t_ms, 4), "subcarriers_per_s": round(S * N / (t_ms * 1e-3), 1),
            "hbm_GBs": round(gbs, 1), "hbm_frac": round(gbs / PEAK["hbm_GBs"], 4),
            "rel_err_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "symbol_error_rate": ser}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the estimator shards over slots with no "
              "communication, and the multi-GPU form is not implemented",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1802_05427_amd import Plan
    from synth import make_slot_batch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        n = 1 << 27   # 128 Mi float32 = 512 MiB read + 512 MiB written per copy
        a = torch.ones(n, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n, "launches": 5}), flush=True)
        return
    if args.detect_only:
        print(json.dumps({"metric": "MMSE detection", "detail": detect_line(dev, torch.cuda.current_stream())}),
              flush=True)
        return
    if args.comb_only:
        r = comb_lines(dev, torch.cuda.current_stream())
        print(json.dumps({"metric": "channel coeffs estimated/s, comb-pilot 3W / 12W", "detail": r}),
              flush=True)
        return
    if args.large_only:
        r = large_sample(dev, torch.cuda.current_stream(), steps=max(2, min(args.steps, 5)),
                         warmup=1)
        print(json.dumps({"metric": "channel coeffs estimated/s (M*K*N), large sample-covariance",
                          "value": r["value"], "unit": "coeff/s", "n_gpus": 1, "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "fp16x3",
                          "data": "synthetic", "config": {"workload": r["workload"]}, "detail": r}),
              flush=True)
        return
    M, K, N, N_fft, taps, tau, snr = 128, 12, 1200, 2048, 72, 4.0, 10.0
    B, Wn, S = args.b, args.wn, args.slots
    if args.fit_only:
        from synth import make_pilots
        pil = torch.from_numpy(make_pilots(K, N)).to(dev)
        r = fit_line(M, K, N, N_fft, B, Wn, taps, 0.1, pil, dev)
        print(json.dumps({"metric": "design fit", "detail": r}), flush=True)
        return
    if args.fwdbwd_only:
        from synth import make_pilots
        pil = torch.from_numpy(make_pilots(K, N)).to(dev)
        r = fwd_bwd(M, K, N, N_fft, B, Wn, taps, 0.1, pil, dev, torch.cuda.current_stream(),
                    args.steps, args.warmup)
        print(json.dumps({"metric": "fwd+bwd steps/s", "value": r["per_s"], "unit": "steps/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": r["ms"], "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": r["workload"], "slots": r["slots"]}}), flush=True)
        return
    uniq = min(S, 8)
    t0 = time.time()
    sb = make_slot_batch(M=M, K=K, N=N, N_fft=N_fft, taps=taps, tau=tau, snr_db=snr, slots=uniq,
                         config_id=2)
    log(f"generated {uniq} slots in {time.time() - t0:.1f}s", args.quiet)
    y_u = torch.from_numpy(sb.y).to(dev)
    reps = (S + uniq - 1) // uniq
    y = y_u.repeat(reps, 1, 1, 1)[:S].contiguous()
    pil = torch.from_numpy(sb.pilots).to(dev)
    sigma2 = sb.sigma2
    coeffs = S * M * K * N

    plan = Plan(M=M, K=K, N=N, N_fft=N_fft, B=B, Wn=Wn, rsource=args.rsource, taps=taps, tau_rms=tau,
                L=144.0, sigma2=sigma2, max_slots=S, precision=args.precision)
    fixed = args.rsource != "sample"
    okw = dict(N_fft=N_fft, tau=tau, taps=taps, L=144.0)
    out = torch.empty_like(y)
    stream = torch.cuda.current_stream()

    # fixed-design filter construction (FP64), timed separately
    design_ms = None
    if fixed:
        for _ in range(3):
            plan.set_design(tau, sigma2)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            plan.set_design(tau, sigma2)
        e1.record(stream)
        torch.cuda.synchronize()
        design_ms = round(e0.elapsed_time(e1) / 10, 4)

    for _ in range(args.warmup):
        plan.estimate(y, pil, sigma2, out=out)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        plan.estimate(y, pil, sigma2, out=out)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    per = [a.elapsed_time(b) for a, b in evs]
    ms = float(np.mean(per))
    ms_med = float(np.median(per))
    value = coeffs / (wall / args.steps)
    log(f"estimate: mean {ms:.4f} ms, median {ms_med:.4f} ms, wall/step {1e3 * wall / args.steps:.4f} ms",
        args.quiet)

    # accuracy on the unique slots vs the FP64 oracle
    import oracle as O
    out_u = out[:uniq].cpu().numpy()
    ref = O.estimate(sb.y[:1], sb.pilots, sigma2, B, Wn, args.rsource, **okw)
    gap = abs(O.nmse_db(out_u[:1], sb.H[:1]) - O.nmse_db(ref, sb.H[:1]))
    disc = O.discrepancy_db(out_u[:1], ref)
    nmse_gpu = O.nmse_db(out_u, sb.H)

    # roofline of the one kernel a step launches, from the mean event time:
    # the complex B x Wn filter per block is 8*B*Wn flops per column per block
    # (8*Wn per coefficient), the fused despreading a K-point DFT (8K) and the
    # conj-pilot multiply (6) per coefficient
    flops_per_coef = 8.0 * Wn + 8.0 * K + 6.0
    kernel_flops = flops_per_coef * coeffs
    achieved = kernel_flops / (ms * 1e-3) / 1e12
    peak = {"fp32": PEAK["fp32_mfma_TFs"], "bf16x3": PEAK["bf16_mfma_TFs"] / 3,
            "fp16x3": PEAK["fp16_mfma_TFs"] / 3}[args.precision]
    bytes_per_coef = 16.0
    gbs = bytes_per_coef * coeffs / (ms * 1e-3) / 1e9
    family = "fp32" if args.precision == "fp32" else "split"
    kname = ("apply_f32_kernel<13, 12>" if args.precision == "fp32"
             else f"apply_split_kernel<13, 12, {args.precision}>")
    traffic = (stored_traffic(kname, family, coeffs)
               if (args.rsource in ("exp", "uniform") and B == 100 and Wn == 150) else None)
    if args.precision == "fp32":
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                "frac": round(gbs / PEAK["hbm_GBs"], 4), "traffic": traffic}

    extras = {}
    if not args.no_extras and args.rsource in ("exp", "uniform") and args.precision == "fp32":
        # split precision on the same workload
        for prec in ("bf16x3", "fp16x3"):
            with Plan(M=M, K=K, N=N, N_fft=N_fft, B=B, Wn=Wn, rsource=args.rsource, taps=taps,
                      tau_rms=tau, L=144.0, sigma2=sigma2, max_slots=S, precision=prec) as pl:
                o2 = torch.empty_like(y)
                t_ms = time_calls(lambda: pl.estimate(y, pil, sigma2, out=o2), max(5, args.steps // 2), 2, stream)
                o2u = o2[:1].cpu().numpy()
                extras[prec] = {
                    "value": round(coeffs / (t_ms * 1e-3), 1), "ms": round(t_ms, 4),
                    "speedup_vs_fp32": round(ms_med / t_ms, 3),
                    "hbm_GBs": round(16.0 * coeffs / (t_ms * 1e-3) / 1e9, 1),
                    "hbm_frac": round(16.0 * coeffs / (t_ms * 1e-3) / 1e9 / PEAK["hbm_GBs"], 4),
                    "nmse_gap_db": abs(O.nmse_db(o2u, sb.H[:1]) - O.nmse_db(ref, sb.H[:1])),
                    "discrepancy_db": round(O.discrepancy_db(o2u, ref), 1)}
        # sample covariance (per-window FP64 design + FP32 filter), 16 slots
        S2 = 16
        y16 = y[:S2].contiguous()
        with Plan(M=M, K=K, N=N, N_fft=N_fft, B=B, Wn=Wn, rsource="sample", sigma2=sigma2,
                  max_slots=S2) as pl:
            o3 = torch.empty_like(y16)
            t_ms = time_calls(lambda: pl.estimate(y16, pil, sigma2, out=o3), 3, 1, stream)
            o3u = o3[:1].cpu().numpy()
        ref_s = O.estimate(sb.y[:1], sb.pilots, sigma2, B, Wn, "sample")
        extras["sample_cov"] = {
            "value": round(S2 * M * K * N / (t_ms * 1e-3), 1), "ms": round(t_ms, 4), "slots": S2,
            "nmse_gap_db": abs(O.nmse_db(o3u, sb.H[:1]) - O.nmse_db(ref_s, sb.H[:1])),
            "discrepancy_db": round(O.discrepancy_db(o3u, ref_s), 1)}
        extras["gap_per_snr"] = gap_per_snr(M, K, N, N_fft, B, Wn, taps, tau, args.rsource, dev)
        extras["non_overlap"] = timed_estimate(y, pil, sigma2, dev, stream, B=100, Wn=100,
                                               rsource=args.rsource, flops=8.0 * 100 + 8.0 * K + 6.0,
                                               ceiling=PEAK["fp32_mfma_TFs"] * 1e12 / (8.0 * 100 + 8.0 * K + 6.0))
        extras["full_band"] = {
            "fixed_fp32": timed_estimate(y, pil, sigma2, dev, stream, B=N, Wn=N, rsource=args.rsource,
                                         flops=8.0 * N + 8.0 * K + 6.0,
                                         ceiling=PEAK["fp32_mfma_TFs"] * 1e12 / (8.0 * N + 8.0 * K + 6.0)),
            "fixed_bf16x3": timed_estimate(y, pil, sigma2, dev, stream, B=N, Wn=N, rsource=args.rsource,
                                           precision="bf16x3"),
            "sample_fp32": timed_estimate(y, pil, sigma2, dev, stream, B=N, Wn=N, rsource="sample"),
        }
        extras["fwd_bwd"] = fwd_bwd(M, K, N, N_fft, B, Wn, taps, sigma2, pil, dev, stream, 5, 2)
        extras["fit"] = fit_line(M, K, N, N_fft, B, Wn, taps, sigma2, pil, dev)
        del y, out
        torch.cuda.empty_cache()
        extras["large_sample"] = large_sample(dev, stream)
        extras["comb"] = comb_lines(dev, stream)
        extras["detect"] = detect_line(dev, stream)

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu_threads = len(os.sched_getaffinity(0))
        except AttributeError:
            cpu_threads = os.cpu_count() or 1
        # whole slots, cycling over the distinct ones, until about cpu_seconds of work
        n_done, t_cpu = 0, 0.0
        while t_cpu < args.cpu_seconds:
            i = n_done % uniq
            t1 = time.perf_counter()
            O.estimate(sb.y[i:i + 1], sb.pilots, sigma2, B, Wn, args.rsource, **okw)
            t_cpu += time.perf_counter() - t1
            n_done += 1
        # the same on one thread (BLAS limited to one thread)
        from threadpoolctl import threadpool_limits
        n1, t1c = 0, 0.0
        with threadpool_limits(limits=1):
            while t1c < args.cpu_seconds:
                i = n1 % uniq
                t1 = time.perf_counter()
                O.estimate(sb.y[i:i + 1], sb.pilots, sigma2, B, Wn, args.rsource, **okw)
                t1c += time.perf_counter() - t1
                n1 += 1
        cpu = {"value": round(n_done * M * K * N / t_cpu, 1), "unit": "coeff/s", "cores": cpu_threads,
               "kind": "oracle",
               "sample": f"{n_done} slot(s) of the same workload, FP64 NumPy oracle "
                         f"(despread, design, filter), {t_cpu:.1f}s",
               "value_1thread": round(n1 * M * K * N / t1c, 1),
               "sample_1thread": f"{n1} slot(s), BLAS limited to one thread, {t1c:.1f}s",
               "cpu_model": cpu_model()}

    rec = {
        "metric": "channel coeffs estimated/s (M*K*N) at stated NMSE gap vs FP64",
        "value": round(value, 1),
        "unit": "coeff/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else args.precision,
        "data": f"synthetic: {uniq} seeded slots (exponential PDP tau 4, 72 taps, SNR 10 dB) tiled to {S}",
        "config": {"workload": f"paper-sized uplink M={M} K={K} N={N} N_fft={N_fft}, {S} slots, "
                               f"{'overlapping' if Wn > B else 'non-overlapping'} B={B} Wn={Wn}, "
                               + {"uniform": "fixed design with a uniform profile over the "
                                             "144-sample cyclic prefix (L=144)",
                                  "exp": "fixed design with the matched exponential profile (tau 4)",
                                  "sample": "sample covariance per (slot, user, window)"}[args.rsource]
                               + f", {args.precision}",
                   "slots": S, "coeffs_per_step": coeffs, "B": B, "Wn": Wn,
                   "precision": args.precision, "rsource": args.rsource},
        "nmse_gap_db": gap,
        "discrepancy_db": round(disc, 1),
        "nmse_db": round(nmse_gpu, 3),
        "kernel_ms_mean": round(ms, 5),
        "kernel_ms_median": round(ms_med, 5),
        "design_ms": design_ms,
        "roofline": roof,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    plan.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
