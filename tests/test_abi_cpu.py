"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the header declares, validates descriptors, and its block plan
matches the oracle's clamp rule."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1802_05427_amd import _lib
from paper_1802_05427_amd.api import block_plan, make_desc, workspace_size

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "lmmse.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lmmse_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(lib):
    names = _header_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.PROTOTYPES, n


def test_status_strings(lib):
    for s in range(9):
        assert _lib.status_string(s)
    assert _lib.status_string(99) == "unknown status"
    assert lib.lmmse_version() >= 10000


def _d(**kw):
    base = dict(M=128, K=12, N=1200, N_fft=2048, B=100, Wn=150, rsource="exp", taps=72,
                tau_rms=4.0, sigma2=0.1, max_slots=64)
    base.update(kw)
    return make_desc(**base)


@pytest.mark.parametrize("kw", [
    {}, dict(Wn=100), dict(B=1200, Wn=1200), dict(rsource="uniform", L=144.0),
    dict(rsource="sample"), dict(rsource="user"), dict(precision="bf16x3"),
    dict(precision="fp16x3"),
    dict(M=8, K=2, N=72, N_fft=128, B=12, Wn=12, taps=8, tau_rms=2.0),
    dict(M=256, K=24, N=3300, N_fft=4096, B=132, Wn=198, taps=144, tau_rms=32.0, max_slots=32),
    # full band of the paper-sized system: fixed, sample (push-through), caller R
    dict(B=1200, Wn=1200, rsource="uniform", L=144.0), dict(rsource="sample", B=1200, Wn=1200),
    dict(rsource="sample", B=300, Wn=300), dict(rsource="sample", B=100, Wn=300),
    dict(rsource="user_r"), dict(rsource="user_r", B=1200, Wn=1200),
    dict(rsource="user_r", precision="bf16x3"),
    # largest batch of the paper-sized system: 2330 * 128 * 12 * 1200 < 2^32 coefficients
    dict(max_slots=2330),
])
def test_validate_accepts_workloads(lib, kw):
    d = _d(**kw)
    assert lib.lmmse_plan_validate(ctypes.byref(d)) == _lib.OK


@pytest.mark.parametrize("kw,code", [
    (dict(M=0), _lib.INVALID_ARG), (dict(K=0), _lib.INVALID_ARG), (dict(N_fft=100), _lib.INVALID_ARG),
    (dict(max_slots=0), _lib.INVALID_ARG), (dict(rsource=9), _lib.INVALID_ARG),
    (dict(precision=7), _lib.INVALID_ARG), (dict(tau_rms=0.0), _lib.INVALID_ARG),
    (dict(taps=0), _lib.INVALID_ARG), (dict(sigma2=0.0), _lib.INVALID_ARG),
    (dict(sigma2=float("nan")), _lib.INVALID_ARG),
    (dict(rsource="uniform", L=-1.0), _lib.INVALID_ARG),
    (dict(B=7), _lib.UNSUPPORTED), (dict(Wn=151), _lib.UNSUPPORTED), (dict(Wn=80), _lib.UNSUPPORTED),
    (dict(Wn=1300), _lib.UNSUPPORTED), (dict(K=65), _lib.UNSUPPORTED),
    # push-through windows: FP32 only, M <= 256
    (dict(rsource="sample", B=300, Wn=300, precision="bf16x3"), _lib.UNSUPPORTED),
    (dict(rsource="sample", B=1200, Wn=1200, precision="fp16x3"), _lib.UNSUPPORTED),
    (dict(rsource="sample", B=1200, Wn=1200, M=300), _lib.UNSUPPORTED),
    (dict(rsource=5), _lib.INVALID_ARG), (dict(rsource="user_r", sigma2=0.0), _lib.INVALID_ARG),
    # one work-item per coefficient: a batch of 2^32 coefficients or more is refused
    (dict(max_slots=2331), _lib.UNSUPPORTED),
])
def test_validate_rejects(lib, kw, code):
    d = _d(**kw)
    assert lib.lmmse_plan_validate(ctypes.byref(d)) == code
    # plan creation refuses the same descriptors before touching a device
    h = ctypes.c_void_p()
    assert lib.lmmse_plan_create(ctypes.byref(d), ctypes.byref(h)) == code
    assert not h.value


def test_null_arguments(lib):
    assert lib.lmmse_plan_validate(None) == _lib.INVALID_ARG
    assert lib.lmmse_plan_create(None, None) == _lib.INVALID_ARG
    assert lib.lmmse_plan_destroy(None) == _lib.INVALID_ARG
    assert lib.lmmse_estimate(None, 1, None, None, 0.1, None, None, 0, None) == _lib.INVALID_ARG
    assert lib.lmmse_backward(None, 1, None, None, None, None, None, None, 0, None) == _lib.INVALID_ARG
    assert lib.lmmse_backward_dev(None, 1, None, None, None, None, None, 0, None) == _lib.INVALID_ARG
    assert lib.lmmse_design_state_size(None, 1, None) == _lib.INVALID_ARG
    assert lib.lmmse_estimate_ls_keep(None, 1, None, 0.1, None, None, 0, None, 0, None) == _lib.INVALID_ARG
    assert lib.lmmse_backward_kept(None, 1, None, None, None, None, None, 0, None, 0, None) == _lib.INVALID_ARG
    assert lib.lmmse_sync_status(None, None, None) == _lib.INVALID_ARG


def test_block_plan_matches_oracle():
    rng = np.random.default_rng(7)
    cases = [(1200, 100, 150), (1200, 100, 100), (3300, 132, 198), (72, 12, 12), (72, 72, 72),
             (1200, 1200, 1200), (72, 12, 24)]
    for _ in range(100):
        B = int(rng.integers(1, 30))
        nb = int(rng.integers(1, 20))
        N = B * nb
        Wn = B + 2 * int(rng.integers(0, (N - B) // 2 + 1))
        cases.append((N, B, Wn))
    for N, B, Wn in cases:
        s, o, c, nc = block_plan(N, B, Wn)
        so, oo = O.window_starts(N, B, Wn)
        assert s == so and o == oo
        assert nc == len(set(oo))
        if Wn - B <= 2 * B:
            assert nc <= 3
        firsts = {}
        for b, off in enumerate(o):
            firsts.setdefault(off, len(firsts))
            assert c[b] == firsts[off]


def test_block_plan_rejects_bad_shapes():
    with pytest.raises(_lib.LmmseError):
        block_plan(100, 7, 7)
    with pytest.raises(_lib.LmmseError):
        block_plan(100, 10, 15)


def test_workspace_sizes():
    # K = 12 is despread inside the filtering launch: no workspace for the forward
    assert workspace_size(_d(), 64) >= 0
    d3 = _d(K=3)
    assert workspace_size(d3, 4) >= 4 * 128 * 3 * 1200 * 8
    with pytest.raises(_lib.LmmseError):
        workspace_size(_d(), 65)


@pytest.mark.parametrize("rsource", ["exp", "uniform", "sample", "user"])
@pytest.mark.parametrize("kw", [dict(), dict(K=3), dict(B=132, Wn=198, N=3300, N_fft=4096, K=24, M=2)])
def test_workspace_size_of_an_empty_batch(rsource, kw):
    """Zero slots (and every smaller batch) must size without faulting."""
    d = _d(rsource=rsource, **kw)
    assert workspace_size(d, 0) >= 0
    for s in (1, 2, 3):
        assert workspace_size(d, s) >= 0


def test_plan_create_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    d = _d()
    h = ctypes.c_void_p()
    assert lib.lmmse_plan_create(ctypes.byref(d), ctypes.byref(h)) == _lib.NO_DEVICE
    assert not h.value


def test_sample_window_limits():
    """The sample design holds windows up to 256 (registers up to 160, then the
    workspace-resident sweep); wider windows take the push-through form, whose
    work area is M x M per window (refused above 256 antennas or in split
    precision)."""
    d = _d(rsource="sample", N=3300, N_fft=4096, B=132, Wn=198, K=24, M=256, max_slots=32)
    need = workspace_size(d, 32)
    # at least H_LS, the FP32 filters and one slot of FP64 window matrices
    nmat1 = 24 * 25
    assert need >= 32 * 256 * 24 * 3300 * 8 + 32 * nmat1 * 132 * 198 * 8 + nmat1 * 198 * 198 * 16
    # the design works through the slots in chunks of at most about 2 GiB
    assert need < 32 * 256 * 24 * 3300 * 8 + 32 * nmat1 * 132 * 198 * 8 + (3 << 30) \
        + 32 * nmat1 * 8 + (1 << 20)
    with pytest.raises(_lib.LmmseError):
        workspace_size(_d(rsource="sample", N=1040, B=130, Wn=260, precision="bf16x3"), 1)
    # full band of 64 paper-sized slots: H_LS plus the M x M FP64 matrices of
    # every (slot, user), no Wn x Wn matrix and no panel scratch (a 128 x 128
    # system is inverted whole by one workgroup)
    fb = workspace_size(_d(rsource="sample", B=1200, Wn=1200), 64)
    nmat = 64 * 12
    assert fb == 64 * 128 * 12 * 1200 * 8 + nmat * 128 * 128 * 16


@pytest.mark.parametrize("kw,code", [
    (dict(), _lib.OK), (dict(kind="3w"), _lib.OK), (dict(rsource="exp", tau_rms=2.0, taps=6), _lib.OK),
    (dict(K=0), _lib.INVALID_ARG), (dict(kind=7), _lib.INVALID_ARG), (dict(sigma2=0.0), _lib.INVALID_ARG),
    (dict(rsource="sample"), _lib.INVALID_ARG), (dict(L=-1.0), _lib.INVALID_ARG),
    (dict(K=13), _lib.UNSUPPORTED), (dict(N=1210), _lib.UNSUPPORTED),
    (dict(comb=8, N=1200, kind="3w"), _lib.UNSUPPORTED), (dict(comb=18, N=1206 * 3, N_fft=4096), _lib.UNSUPPORTED),
    (dict(N=120), _lib.UNSUPPORTED), (dict(N=2400, N_fft=2048), _lib.UNSUPPORTED),
    (dict(kind="ls_linear", N=24), _lib.OK), (dict(kind="ls_quadratic", N=24), _lib.UNSUPPORTED),
    (dict(kind="ls_spline", N=36), _lib.OK), (dict(kind="ls_spline", N=24), _lib.UNSUPPORTED),
    (dict(kind="ls_spline", N=24576, N_fft=32768), _lib.OK),
    (dict(kind="ls_spline", N=24588, N_fft=32768), _lib.UNSUPPORTED),
    (dict(kind="ls_quadratic", N=24588, N_fft=32768), _lib.OK),
])
def test_comb_validate(kw, code):
    from paper_1802_05427_amd import comb_validate
    base = dict(M=16, K=4, N=1200, N_fft=2048, comb=12, kind="12w", rsource="uniform", L=8.0,
                sigma2=0.01, max_slots=4)
    base.update(kw)
    assert comb_validate(**base) == code
