"""Grid statistics in the format of the paper's Table 1 ("Uniform grid attributes").

Given a finished grid, the table's columns are

* cells                  = rx * ry * rz
* % empty cells          = 100 * (cells - nonEmpty) / cells
* avg # items / n-empt   = NO / nonEmpty
* max # cells / item     = max over objects of its cell count
* avg # cells / item     = NO / #objects
* memory                 = 4 * (cells + NO) bytes (one 32-bit offset per cell in
                           G, one 32-bit object id per pair in O), printed in MiB.

These are plain host-side reductions used for reporting; they are not part of
the build.
"""
from __future__ import annotations

import numpy as np


def table1(res, ntris: int, npairs: int, nonempty: int, max_cells_per_item: int) -> dict:
    cells = int(np.prod(np.asarray(res, np.int64)))
    return {
        "triangles": int(ntris),
        "dimensions": "x".join(str(int(r)) for r in res),
        "cells": cells,
        "pct_empty": 100.0 * (cells - nonempty) / cells if cells else 0.0,
        "avg_items_per_nonempty": (npairs / nonempty) if nonempty else 0.0,
        "max_cells_per_item": int(max_cells_per_item),
        "avg_cells_per_item": (npairs / ntris) if ntris else 0.0,
        "memory_MiB": 4.0 * (cells + npairs) / 2.0 ** 20,
    }


def table1_from_ranges(res, ntris: int, ranges: np.ndarray, counts: np.ndarray) -> dict:
    """Table 1 row from the per-cell [begin, end) table and the per-object counts."""
    r = np.asarray(ranges).reshape(-1, 2).astype(np.int64)
    nonempty = int(np.count_nonzero(r[:, 1] > r[:, 0]))
    npairs = int(r[-1, 1]) if r.shape[0] else 0
    maxc = int(np.asarray(counts).max()) if len(counts) else 0
    return table1(res, ntris, npairs, nonempty, maxc)
