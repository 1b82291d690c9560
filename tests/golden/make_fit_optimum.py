"""Writes fit_optimum_diff_workload.json: the FP64 oracle's optimum of the
fixed exponential design for the differentiation workload (M=128 does not
enter: the expected error is per coefficient), computed only with oracle/.

Workload: N=1200 used subcarriers of a 2048-point FFT, K=12 pilot symbols,
overlapping windows of 150 keeping the central 100, 72 taps, SNR 10 dB
(sigma2 = 0.1), tau_rms ~ U[2, 24] per (slot, user).

Run from the repository root: python tests/golden/make_fit_optimum.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.fit_optimum import fit_optimum  # noqa: E402

CONFIG = dict(N=1200, B=100, Wn=150, K=12, taps=72, N_fft=2048, sigma2=0.1, tau_lo=2.0, tau_hi=24.0)


def main():
    c = CONFIG
    tau, sig, mse, _ = fit_optimum(c["N"], c["B"], c["Wn"], c["K"], c["taps"], c["N_fft"],
                                   c["sigma2"], c["tau_lo"], c["tau_hi"])
    out = dict(config=c, tau=tau, sigma2=sig, mse=mse,
               note="minimiser of the expected per-coefficient error over the design "
                    "(tau_rms, sigma2) at the spread-averaged correlation; oracle/fit_optimum.py")
    with open(os.path.join(HERE, "fit_optimum_diff_workload.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
