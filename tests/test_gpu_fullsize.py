"""GPU parity at the benchmarked sizes, in the launch configurations the
bench times, on sampled outputs the FP64 oracle computes column by column:

  * the fused despread + block filter on 64 paper-sized slots (M=128, K=12,
    N=1200 of 2048, overlapping 150/100, exponential design), FP32 and
    BF16x3, every user and block of sampled (slot, antenna) columns;
  * the comb-pilot 3W / 12W estimators on 64 slots of 128 antennas and 4
    UEs, sampled (slot, antenna) columns;
  * MMSE detection on 64 slots of 128 antennas, 12 users and 12 data
    symbols, sampled (slot, subcarrier) problems;
  * the large sample-covariance workload on 32 slots, sampled windows;
  * the fixed-design forward and backward of the timed training step on
    16 slots, whole batch.

The slots are distinct (drawn on the GPU from one seeded generator)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1802_05427_amd import CombPlan, Plan, mmse_detect
from synth import make_comb_batch, make_pilots
from synth.torch_slots import draw_batch

pytestmark = pytest.mark.gpu

M, K, N, NF, B, WN, TAPS, TAU, S = 128, 12, 1200, 2048, 100, 150, 72, 4.0, 64
SAMPLES = [(0, 0), (0, 127), (17, 55), (38, 3), (63, 0), (63, 127)]   # (slot, antenna)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def batch(dev):
    pil = torch.from_numpy(make_pilots(K, N)).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(180205427 + 64)
    sigma2 = 0.1   # SNR 10 dB
    ys = [draw_batch(g, 16, M, K, N, NF, TAPS, TAU, TAU, sigma2, pil)[0] for _ in range(S // 16)]
    return torch.cat(ys).contiguous(), pil, sigma2


@pytest.mark.parametrize("precision,limit_db", [("fp32", -120.0), ("bf16x3", -110.0)])
def test_headline_batch_sampled_columns(dev, batch, precision, limit_db):
    y, pil, sigma2 = batch
    print(f"full-size estimate {precision}: {S} slots", flush=True)
    with Plan(M=M, K=K, N=N, N_fft=NF, B=B, Wn=WN, rsource="exp", taps=TAPS, tau_rms=TAU,
              sigma2=sigma2, max_slots=S, precision=precision) as plan:
        out = torch.empty_like(y)
        plan.estimate(y, pil, sigma2, out=out)
        torch.cuda.synchronize()
    pil_h = pil.cpu().numpy()
    for s, m in SAMPLES:
        ys = y[s:s + 1, m:m + 1].cpu().numpy().astype(np.complex128)
        ref = O.estimate(ys, pil_h, sigma2, B, WN, "exp", N_fft=NF, tau=TAU, taps=TAPS)
        got = out[s:s + 1, m:m + 1].cpu().numpy()
        disc = O.discrepancy_db(got, ref)
        print(f"  slot {s} antenna {m}: discrepancy {disc:.1f} dB", flush=True)
        assert disc < limit_db, (s, m, disc)


@pytest.mark.parametrize("kind", ["3w", "12w"])
def test_comb_batch_sampled_columns(dev, kind):
    Kc, Sc = 4, 12
    cb = make_comb_batch(M=M, K=Kc, N=N, N_fft=NF, powers_db=[-2, -8, -10, -12, -15, -18],
                         snr_db=20.0, slots=S, comb=Sc)
    y = torch.from_numpy(cb.y).to(dev)
    pil = torch.from_numpy(cb.pilots).to(dev)
    print(f"full-size comb {kind}: {S} slots", flush=True)
    with CombPlan(M=M, K=Kc, N=N, N_fft=NF, comb=Sc, kind=kind, rsource="uniform", L=8.0,
                  sigma2=cb.sigma2, max_slots=S) as pl:
        out = pl.estimate(y, pil)
        torch.cuda.synchronize()
    rd = lambda d: O.r_uniform(d, 8.0, NF)
    for s, m in SAMPLES:
        ref = O.comb_estimate(cb.y[s:s + 1, m:m + 1], cb.pilots, cb.sigma2, Sc, range(Kc), kind, rd)
        disc = O.discrepancy_db(out[s:s + 1, m:m + 1].cpu().numpy(), ref)
        print(f"  slot {s} antenna {m}: discrepancy {disc:.1f} dB", flush=True)
        assert disc < -120.0, (s, m, disc)


def test_detection_batch_sampled_subcarriers(dev):
    T, sigma2 = 12, 0.1
    pil = torch.from_numpy(make_pilots(K, N)).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(180205427 + 65)
    H = torch.cat([draw_batch(g, 16, M, K, N, NF, TAPS, TAU, TAU, 0.0, pil)[1]
                   for _ in range(S // 16)]).contiguous()
    bits = torch.randint(0, 2, (S, T, K, N, 2), generator=g, device=dev).float()
    X = torch.complex(1 - 2 * bits[..., 0], 1 - 2 * bits[..., 1]) / np.sqrt(2.0)
    Y = torch.zeros((S, M, T, N), dtype=torch.complex64, device=dev)
    for k in range(K):
        Y += H[:, :, k, None, :] * X[:, None, :, k, :]
    Y += torch.complex(torch.randn(Y.shape, generator=g, device=dev),
                       torch.randn(Y.shape, generator=g, device=dev)) * float(np.sqrt(sigma2 / 2))
    print(f"full-size detection: {S} slots", flush=True)
    out = mmse_detect(H, Y, sigma2)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    picks = [(0, 0), (63, N - 1)] + [(int(rng.integers(S)), int(rng.integers(N))) for _ in range(10)]
    for s, n in picks:
        h = H[s:s + 1, :, :, n:n + 1].cpu().numpy().astype(np.complex128)
        yy = Y[s:s + 1, :, :, n:n + 1].cpu().numpy().astype(np.complex128)
        ref = O.mmse_detect(h, yy, sigma2)[0, :, :, 0]
        got = out[s, :, :, n].cpu().numpy()
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert rel < 1e-5, (s, n, rel)
    print(f"  {len(picks)} subcarrier problems within 1e-5", flush=True)


def test_large_sample_batch_sampled_windows(dev):
    """The large workload (M=256, K=24, N=3300 of 4096, windows of 198 around
    blocks of 132, per-window sample covariance, FP16x3 filter) on 32 slots:
    sampled (slot, user, block) windows, the oracle's covariance, filter and
    product for all 256 antennas of each."""
    Ml, Kl, Nl, Nfl, Bl, Wl, Sl = 256, 24, 3300, 4096, 132, 198, 32
    sigma2 = 10.0 ** -1.5
    pil = torch.from_numpy(make_pilots(Kl, Nl)).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(180205427 + 66)
    y = torch.cat([draw_batch(g, 4, Ml, Kl, Nl, Nfl, 144, 32.0, 32.0, sigma2, pil)[0]
                   for _ in range(Sl // 4)]).contiguous()
    print(f"full-size large sample-covariance estimate: {Sl} slots", flush=True)
    with Plan(M=Ml, K=Kl, N=Nl, N_fft=Nfl, B=Bl, Wn=Wl, rsource="sample", sigma2=sigma2,
              max_slots=Sl, precision="fp16x3") as pl:
        out = pl.estimate(y, pil, sigma2)
        torch.cuda.synchronize()
    starts, offs = O.window_starts(Nl, Bl, Wl)
    nb, lam = Nl // Bl, sigma2 / Kl
    pil_h = pil.cpu().numpy()
    for s, k, b in [(0, 0, 0), (31, 23, nb - 1), (13, 7, 12), (22, 16, 1)]:
        X = O.despread(y[s:s + 1].cpu().numpy().astype(np.complex128), pil_h)[0, :, k, :]
        Xw = X[:, starts[b]:starts[b] + Wl]
        R = O.sample_covariance(Xw)
        W = O.lmmse._filter(R[offs[b]:offs[b] + Bl], R, lam)
        disc = O.discrepancy_db(out[s, :, k, b * Bl:(b + 1) * Bl].cpu().numpy(), Xw @ W.T)
        print(f"  slot {s} user {k} block {b}: discrepancy {disc:.1f} dB", flush=True)
        # FP32 covariance on the matrix cores, FP64 design, FP16x3 filter
        assert disc < -85.0, (s, k, b, disc)


def test_fixed_fwd_bwd_batch(dev):
    """The timed training step (fixed exponential design at tau 8 and sigma2
    1e-4, 16 paper-sized slots with tau ~ U[2, 24] at 10 dB): the forward
    and the backward to h_ls, tau and sigma2, against the oracle's on the
    whole batch.  The same complex64 LS values (the oracle's despreading)
    feed both sides, and the loss gradient is the oracle's."""
    S2, dtau, dsig = 16, 8.0, 1e-4
    pil = torch.from_numpy(make_pilots(K, N)).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(180205427)
    y, H, _ = draw_batch(g, S2, M, K, N, NF, TAPS, 2.0, 24.0, 0.1, pil)
    X32 = O.despread(y.cpu().numpy().astype(np.complex128), pil.cpu().numpy()).astype(np.complex64)
    X = X32.astype(np.complex128)
    n = np.arange(N)
    R = O.toeplitz_from_r(lambda d: O.r_exponential(d, dtau, TAPS, NF), n, n)
    Ws, st = O.block_filters(R, B, WN, dsig / K)
    ref = O.apply_filters(Ws, st, B, X)
    _, G = O.mse_loss_and_grad(ref, H.cpu().numpy())
    G32 = G.astype(np.complex64)
    print(f"full-size fixed fwd+bwd: {S2} slots", flush=True)
    with Plan(M=M, K=K, N=N, N_fft=NF, B=B, Wn=WN, rsource="exp", taps=TAPS, tau_rms=dtau,
              sigma2=dsig, max_slots=S2) as pl:
        h = torch.from_numpy(X32).to(dev)
        o = pl.apply(h)
        d_hls, d_tau, d_sig = pl.backward(h, torch.from_numpy(G32).to(dev))
        torch.cuda.synchronize()
        o, d_hls = o.cpu().numpy(), d_hls.cpu().numpy()
    dX_o, gtau_o, gsig_o = O.grad_fixed_design(X, G32.astype(np.complex128), B, WN, dtau, TAPS, NF,
                                               dsig, K)
    disc = O.discrepancy_db(o, ref)
    ex = np.linalg.norm(d_hls - dX_o) / np.linalg.norm(dX_o)
    print(f"  forward {disc:.1f} dB  dX rel {ex:.2e}  dtau gpu {d_tau:.6e} oracle {gtau_o:.6e}"
          f"  dsig gpu {d_sig:.6e} oracle {gsig_o:.6e}", flush=True)
    assert disc < -120.0
    assert ex < 1e-5
    assert abs(d_tau - gtau_o) <= 1e-4 * abs(gtau_o)
    assert abs(d_sig - gsig_o) <= 1e-4 * abs(gsig_o)
