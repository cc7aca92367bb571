"""The oracle's own construction of the dyadic parts data (test infrastructure
only): rows of X = max(0, fl32(W0 H0 + fl32(0.01 z))) in FP32 on the host, with
W0, H0 from datagen.dyadic_parts_factors and z from this package's Philox
(stream 2, key = the workload seed, element (i, j) at flat index i n + j).  W0 H0
is exact in FP32 for these factors, so these are the numbers the device forms
from the same recipe."""
import concurrent.futures

import numpy as np

import datagen

from . import philox


def dyadic_parts_rows(name, row0=0, rows=None, panel=4096, threads=8, out=None):
    """Rows row0 .. row0 + rows - 1 of the workload's X (FP32)."""
    c = datagen.CONFIGS[name]
    m, n = c["m"], c["n"]
    rows = m - row0 if rows is None else rows
    seed = datagen.cfg_seed(name)
    W0, H0 = datagen.dyadic_parts_factors(m, n, c["r_true"], seed)
    X = np.empty((rows, n), dtype=np.float32) if out is None else out

    def fill(i):
        cnt = min(panel, rows - i)
        z = philox.normal(cnt, n, datagen.DYADIC_NOISE_STREAM, seed, row0=row0 + i).astype(np.float32)
        z *= datagen.DYADIC_NOISE
        z += W0[row0 + i:row0 + i + cnt] @ H0
        np.maximum(z, np.float32(0.0), out=z)
        X[i:i + cnt] = z

    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        list(ex.map(fill, range(0, rows, panel)))
    return X
