"""Per-block parity checks shared by the GPU tests (no estimator arithmetic).

A whole-array discrepancy can hide an error confined to a few blocks, such as
the band-edge blocks whose windows are shifted inside the band (their own
filter classes).  These helpers compare every output block separately."""
import numpy as np


def block_discrepancies_db(out, ref, B: int):
    """10 log10(||out_b - ref_b||^2 / ||ref_b||^2) for every block b of B
    consecutive output subcarriers (last axis), over all other axes."""
    out = np.asarray(out, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    N = ref.shape[-1]
    res = []
    for b in range(N // B):
        o = out[..., b * B:(b + 1) * B]
        r = ref[..., b * B:(b + 1) * B]
        res.append(10.0 * np.log10(np.sum(np.abs(o - r) ** 2) / np.sum(np.abs(r) ** 2)))
    return res


def assert_blocks(out, ref, B: int, limit_db: float):
    """Every block, the first and the last (band-edge classes) named
    explicitly, below limit_db."""
    d = block_discrepancies_db(out, ref, B)
    assert d[0] < limit_db, ("first block", d[0])
    assert d[-1] < limit_db, ("last block", d[-1])
    worst = int(np.argmax(d))
    assert d[worst] < limit_db, ("block", worst, d[worst])
    return max(d)
