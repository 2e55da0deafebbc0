"""Reference of the ingest repack (band-interleaved-by-line to the retrieval's
column-contiguous layout) - TEST INFRASTRUCTURE ONLY: only the tests and the
benchmark may use it.

A BIL cube holds, for each line, each band's row of samples: bil[l, b, s].
The retrieval reads radiance[s, l, b] (each detector column contiguous).
Censored values (non-finite, or equal to the no-data value) make the pixel
invalid; invalid pixels are skipped by the statistics (Sec. III-A).
"""
from __future__ import annotations

import numpy as np


def repack_bil(bil, nodata=None):
    """(radiance [S, N, B] float32, valid [S, N] uint8) of bil [N, B, S]."""
    bil = np.asarray(bil, dtype=np.float32)
    rad = np.ascontiguousarray(np.transpose(bil, (2, 0, 1)))
    bad = ~np.isfinite(rad)
    if nodata is not None:
        bad |= rad == np.float32(nodata)
    valid = (~bad.any(axis=2)).astype(np.uint8)
    return rad, valid
