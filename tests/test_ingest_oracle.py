"""Pins of the ingest reference (CPU): the layout mapping on a cube whose
values encode their own (line, band, sample) indices, and the censoring
rules."""
import numpy as np

from oracle.ingest import repack_bil


def test_layout_mapping_by_index_encoding():
    N, B, S = 5, 4, 3
    bil = np.zeros((N, B, S), dtype=np.float32)
    for l in range(N):
        for b in range(B):
            for s in range(S):
                bil[l, b, s] = 100 * l + 10 * b + s
    rad, valid = repack_bil(bil)
    assert rad.shape == (S, N, B) and rad.flags["C_CONTIGUOUS"]
    flat = rad.reshape(-1)
    # pixel (column c, line l) is the run flat[(c N + l) B : (c N + l + 1) B]
    for c in range(S):
        for l in range(N):
            expect = [100 * l + 10 * b + c for b in range(B)]
            assert list(flat[(c * N + l) * B:(c * N + l + 1) * B]) == expect
    assert valid.shape == (S, N) and valid.all()


def test_censoring_rules():
    bil = np.ones((2, 3, 2), dtype=np.float32)
    bil[0, 1, 0] = np.nan        # line 0, sample 0: a NaN band
    bil[1, 2, 1] = -9999.0       # line 1, sample 1: the no-data value
    bil[1, 0, 0] = np.inf        # line 1, sample 0: an infinite band
    _, v = repack_bil(bil)
    assert v.tolist() == [[0, 0], [1, 1]]
    _, v = repack_bil(bil, nodata=-9999.0)
    assert v.tolist() == [[0, 0], [1, 0]]
